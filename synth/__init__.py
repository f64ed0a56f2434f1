"""Seeded synthetic inputs shaped like the workloads of the paper's Section 5
(synthetic low-rank matrices, simulation snapshots, a colour image), for both
the oracle tests and the GPU path.

This module only builds test matrices.  It holds none of the method's
arithmetic (no sketch, rangefinder or solve); building a low-rank quaternion
matrix from its factors needs a Hamilton product, which is written here a
third time, independently of the oracle and of the HIP kernels.

Everything is drawn from a ``torch.Generator`` seeded with the data key
(1000 + workload number by default) on the requested device, so that large
inputs can be generated directly in HBM.  A CPU and a GPU generator give
different values for the same seed: parity tests generate on the CPU and
copy.  A quaternion matrix is a tensor of shape (4, m, n) (planes w, x, y, z),
or (3, m, n) for a pure quaternion (planes x, y, z; w = 0).
"""
from __future__ import annotations

import math

import torch


def _gen(seed, device):
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def qgauss(shape_mn, gen, device, dtype=torch.float64, std=1.0):
    m, n = shape_mn
    return torch.randn((4, m, n), generator=gen, device=device, dtype=dtype) * std


def qprod(a, b):
    """Hamilton product of (4, m, p) and (4, p, n) tensors (planes w, x, y, z)."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return torch.stack([
        aw @ bw - ax @ bx - ay @ by - az @ bz,
        aw @ bx + ax @ bw + ay @ bz - az @ by,
        aw @ by - ax @ bz + ay @ bw + az @ bx,
        aw @ bz + ax @ by - ay @ bx + az @ bw,
    ])


def lowrank_plus_noise(m, n, sigma, noise_rel, seed, device="cpu", dtype=torch.float64,
                       factor_std=0.5):
    """A = G1 diag(sigma) G2 + E with G1 (m x r), G2 (r x n) quaternion Gaussian
    with component std ``factor_std`` (N(0, 1/4) by default), and E quaternion
    Gaussian scaled to ||E||_F = noise_rel * ||G1 diag(sigma) G2||_F."""
    gen = _gen(seed, device)
    sigma = torch.as_tensor(sigma, dtype=torch.float64)
    r = sigma.numel()
    g1 = qgauss((m, r), gen, device, torch.float64, factor_std)
    g2 = qgauss((r, n), gen, device, torch.float64, factor_std)
    a0 = qprod(g1 * sigma.to(device)[None, None, :], g2)
    if noise_rel > 0:
        e = torch.randn((4, m, n), generator=gen, device=device, dtype=torch.float64)
        e *= noise_rel * torch.linalg.vector_norm(a0) / torch.linalg.vector_norm(e)
        a0 += e
    return a0.to(dtype)


def config1(device="cpu"):
    """1000 x 800 = G1 D G2 + E, D = diag(0.8^i), i = 0..19, ||E|| = 1e-6 ||G1 D G2||."""
    sig = 0.8 ** torch.arange(20, dtype=torch.float64)
    return lowrank_plus_noise(1000, 800, sig, 1e-6, 1001, device=device)


def config2(device="cpu", m=20000, n=15000, dtype=torch.float32):
    """m x n rank-50 matrix, sigma_i = i^-2 (i = 1..50), noise 1e-4 relative."""
    sig = torch.arange(1, 51, dtype=torch.float64) ** -2.0
    return lowrank_plus_noise(m, n, sig, 1e-4, 1002, device=device, dtype=dtype)


def image_planes(m, n, seed=1003, device="cpu", modes=64, fmax=32, noise=0.02,
                 dtype=torch.bfloat16):
    """Pure quaternion 'colour image' (3, m, n): each of the i, j, k planes is a
    sum of ``modes`` 2-D cosines cos(2 pi (fx x / m + fy y / n) + phi) with
    integer (fx, fy) in [-fmax, fmax]^2 \\ {0}, amplitude 1 / ||f|| and phase
    U[0, 2 pi); mapped affinely onto [0.02, 0.98]; plus U(-noise, noise)."""
    gen = _gen(seed, device)
    x = torch.arange(m, device=device, dtype=torch.float64)[:, None] / m
    y = torch.arange(n, device=device, dtype=torch.float64)[:, None] / n
    planes = []
    for _ in range(3):
        f = torch.randint(-fmax, fmax + 1, (modes, 2), generator=gen, device=device)
        zero = (f[:, 0] == 0) & (f[:, 1] == 0)
        f[zero, 0] = 1
        amp = 1.0 / torch.linalg.vector_norm(f.double(), dim=1)
        phi = torch.rand(modes, generator=gen, device=device, dtype=torch.float64) * 2 * math.pi
        al = 2 * math.pi * x * f[:, 0].double()[None, :] + phi[None, :]     # m x modes
        be = 2 * math.pi * y * f[:, 1].double()[None, :]                    # n x modes
        # cos(al + be) = cos al cos be - sin al sin be: an (m x 2M)(2M x n) product
        left = torch.cat([torch.cos(al) * amp, -torch.sin(al) * amp], dim=1)
        right = torch.cat([torch.cos(be), torch.sin(be)], dim=1).T
        p = (left.float() @ right.float())
        lo, hi = p.min(), p.max()
        p = 0.02 + 0.96 * (p - lo) / (hi - lo)
        p += (torch.rand(p.shape, generator=gen, device=device, dtype=torch.float32) * 2 - 1) * noise
        planes.append(p.to(dtype))
        del p, left, right, al, be
    return torch.stack(planes)


def flow_snapshots(grid=128, steps=300, modes=40, seed=1005, device="cpu", noise_rel=1e-3,
                   kmax=8, dtype=torch.float32):
    """Pure quaternion snapshot matrix (3, grid^3, steps) of a divergence-free
    velocity field: u(x, t) = sum_c a_c sin(w_c t + psi_c) p_c cos(kappa_c . x + theta_c),
    integer wave vectors ||kappa_c|| <= kmax, unit p_c orthogonal to kappa_c,
    w_c in [0.01, 0.1]; plus Gaussian noise of relative size ``noise_rel``.
    Grid points are ordered x + grid (y + grid z)."""
    gen = _gen(seed, device)
    ks = []
    while len(ks) < modes:
        kv = torch.randint(-kmax, kmax + 1, (3,), generator=gen, device=device).cpu()
        nrm = float(torch.linalg.vector_norm(kv.double()))
        if 0 < nrm <= kmax:
            ks.append(kv.double())
    kap = torch.stack(ks).to(device)                                   # modes x 3
    r = torch.randn((modes, 3), generator=gen, device=device, dtype=torch.float64)
    p = torch.linalg.cross(kap, r)
    p = p / torch.linalg.vector_norm(p, dim=1, keepdim=True)            # p . kappa = 0
    amp = 0.5 + torch.rand(modes, generator=gen, device=device, dtype=torch.float64)
    om = 0.01 + 0.09 * torch.rand(modes, generator=gen, device=device, dtype=torch.float64)
    ps = 2 * math.pi * torch.rand(modes, generator=gen, device=device, dtype=torch.float64)
    th = 2 * math.pi * torch.rand(modes, generator=gen, device=device, dtype=torch.float64)
    g = torch.arange(grid, device=device, dtype=torch.float64) * (2 * math.pi / grid)
    zz, yy, xx = torch.meshgrid(g, g, g, indexing="ij")
    pts = torch.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], dim=1)   # m x 3
    t = torch.arange(steps, device=device, dtype=torch.float64)
    temporal = amp[:, None] * torch.sin(om[:, None] * t[None, :] + ps[:, None])   # modes x n
    out = []
    for comp in range(3):
        spatial = torch.cos(pts @ kap.T + th[None, :]) * p[:, comp][None, :]       # m x modes
        out.append((spatial.float() @ temporal.float()))
    a = torch.stack(out)
    if noise_rel > 0:
        e = torch.randn(a.shape, generator=gen, device=device, dtype=torch.float32)
        e *= noise_rel * torch.linalg.vector_norm(a) / torch.linalg.vector_norm(e)
        a += e
    return a.to(dtype)


def batch_specs(count=64, seed=1004):
    """Shapes of the batched workload: m log-uniform in [512, 8192], n in
    [256, 4096], rank r in {8..64}, geometric decay rho in [0.7, 0.95],
    k = 2r and l = min(2k + 1, m, n)."""
    gen = _gen(seed, "cpu")
    specs = []
    for _ in range(count):
        u = torch.rand(5, generator=gen, dtype=torch.float64)
        m = int(round(math.exp(math.log(512) + u[0].item() * (math.log(8192) - math.log(512)))))
        n = int(round(math.exp(math.log(256) + u[1].item() * (math.log(4096) - math.log(256)))))
        r = 8 + int(u[2].item() * 57)
        rho = 0.7 + 0.25 * u[3].item()
        k = 2 * r
        l = min(2 * k + 1, m, n)
        k = min(k, l)
        specs.append(dict(m=m, n=n, r=r, rho=rho, k=k, l=l))
    return specs


def batch_matrix(spec, index, device="cpu", dtype=torch.float32):
    sig = spec["rho"] ** torch.arange(spec["r"], dtype=torch.float64)
    return lowrank_plus_noise(spec["m"], spec["n"], sig, 1e-4, 20000 + index, device=device,
                              dtype=dtype)


def pure_to_full(a3):
    """(3, m, n) pure quaternion -> (4, m, n) with a zero real plane."""
    z = torch.zeros_like(a3[0])
    return torch.stack([z, a3[0], a3[1], a3[2]])
