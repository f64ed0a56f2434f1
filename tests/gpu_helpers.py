"""Helpers shared by the GPU parity tests: move oracle-side NumPy inputs to
the device in the library's layout and back."""
import numpy as np
import torch

import paper_2404_14783_amd as qs

TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def to_device(a_np, dtype, pure=False):
    """(4, m, n) NumPy -> (4 or 3, m, n) device tensor with column-major planes."""
    t = torch.from_numpy(np.ascontiguousarray(a_np[1:] if pure else a_np))
    t = t.to(TORCH[dtype])
    return qs.to_colmajor(t.cuda())


def input_values(a_np, dtype):
    """The values the device sees for a given input dtype (exact widening)."""
    t = torch.from_numpy(np.ascontiguousarray(a_np)).to(TORCH[dtype])
    return t.double().numpy()


def to_numpy(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    n = np.linalg.norm(np.asarray(b).ravel())
    return d / n if n > 0 else d


def run_sketch(a_np, m, n, k, l, block, dtype="f64", sketch="f64", emb="gaussian", seed=0,
               terms=1, pure=False, order=None):
    sk = qs.Sketcher(m, n, k, l, seed=seed, embedding=emb, input_dtype=dtype, sketch_dtype=sketch,
                     split_terms=terms, pure=pure, max_block_cols=block)
    dev = to_device(a_np, dtype, pure=pure)
    starts = list(range(0, n, block))
    if order is not None:
        starts = [starts[i] for i in order]
    for c0 in starts:
        sk.update(c0, dev[:, :, c0:c0 + block])
    torch.cuda.synchronize()
    return sk, dev


# ---------------------------------------------------------------------------
# Element-wise sketch parity.
#
# Every entry of Y = A Omega (plane p, entry (i, j)) is a signed sum over the
# contraction index t and the input planes q of A_q[i, t] * Omega_r[t, j]
# (Appendix B.1's real form of the Hamilton product), so the sum of the
# absolute values of its terms is at most
#     B[i, j] = sum_t (sum_q |A_q[i, t]|) * max_r |Omega_r[t, j]|,
# and likewise for W = Psi A with B = (max_r |Psi_r|) (sum_q |A_q|).  A sum of
# K such terms evaluated in floating point with unit roundoff u is within
# about sqrt(K) u B of the exact value (probabilistic rounding-error bound;
# the worst case is K u B).  The device must stay within C_ACC sqrt(K) u B
# of the oracle's FP64 value entry by entry; the measured margin (the largest
# |dev - ref| / (sqrt(K) u B)) is printed.

U32 = 2.0 ** -24
U64 = 2.0 ** -53
C_ACC = 8.0


def plane_abs_sum(a):
    """sum_q |A_q| of a (P, r, c) array of planes."""
    return np.sum(np.abs(np.asarray(a, dtype=np.float64)), axis=0)


def plane_abs_max(a):
    """max_r |A_r| of a (P, r, c) array of planes."""
    return np.max(np.abs(np.asarray(a, dtype=np.float64)), axis=0)


def y_bound(a_ops, om):
    """B for rows of Y = A Omega: (sum_q |A_q|) (max_r |Omega_r|)."""
    return plane_abs_sum(a_ops) @ plane_abs_max(om)


def w_bound(ps, a_ops):
    """B for W = Psi A: (max_r |Psi_r|) (sum_q |A_q|)."""
    return plane_abs_max(ps) @ plane_abs_sum(a_ops)


def elementwise_margin(dev, ref, bound, K, u=U32, op_rel=0.0):
    """max over entries of |dev - ref| / ((sqrt(K) u + op_rel) B): the
    accumulation error in units of the probabilistic bound.  op_rel is an
    extra relative error per operand value (zero when the device multiplies
    exactly the oracle's operands)."""
    dev = np.asarray(dev, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = (np.sqrt(K) * u + op_rel) * np.broadcast_to(bound, ref.shape)
    diff = np.abs(dev - ref)
    if not np.all(np.isfinite(dev)):
        return np.inf
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(scale > 0, diff / np.where(scale > 0, scale, 1.0), np.where(diff > 0, np.inf, 0.0))
    return float(r.max()) if r.size else 0.0


def assert_elementwise(dev, ref, bound, K, label, u=U32, op_rel=0.0, c=C_ACC):
    """Every entry within c (sqrt(K) u + op_rel) B of the oracle's value."""
    mg = elementwise_margin(dev, ref, bound, K, u=u, op_rel=op_rel)
    print(f"{label}: element-wise margin {mg:.3g} (limit {c:g}; K = {K})", flush=True)
    assert mg <= c, (label, mg)
    return mg


def sketch_bounds(a_ops, om, ps):
    """(B_Y, B_W) of whole sketches for operand values a_ops (P, m, n), Omega
    (4, n, k) and Psi (4, l, m)."""
    return y_bound(a_ops, om), w_bound(ps, a_ops)


def operand_rel(cfg):
    """Relative error per data value of the device's operands against the
    oracle's (``data_operand``): zero except for the fp8 format with the
    residual, whose residual the device carries as two bf16 terms, i.e. to
    2^-17 of itself (and the residual is at most the value).  The e4m3-term
    format ('fp8x') multiplies exactly the oracle's terms."""
    if cfg.dtype == "fp8" and cfg.fp8_residual:
        return 2.0 ** -17
    return 0.0


def check_sketches(y, w, ref, a, label, block_cols=None):
    """Y and W of a device context against the oracle sketch ``ref`` of the
    same data ``a`` (P, m, n), entry by entry (see the bound above).  The data
    operand is formed per update block as the oracle does."""
    from oracle.sketch import data_operand
    cfg = ref.cfg
    a = np.asarray(a, dtype=np.float64)
    if a.shape[0] == 3:
        a = np.concatenate([np.zeros_like(a[:1]), a], axis=0)
    bc = block_cols or cfg.n
    a_ops = np.concatenate([data_operand(a[:, :, c0:c0 + bc], cfg) for c0 in range(0, cfg.n, bc)],
                           axis=2)
    by, bw = sketch_bounds(a_ops, ref.omega_rows(0, cfg.n), ref.psi())
    u = U64 if cfg.dtype == "f64" else U32
    terms = cfg.terms if cfg.dtype in ("bf16", "fp8x") else (3 if cfg.dtype == "fp8" else 1)
    orel = operand_rel(cfg)
    my = assert_elementwise(y, ref.Y, by, 4 * cfg.n * terms, label + " Y", u=u, op_rel=orel)
    mw = None
    if w is not None:
        mw = assert_elementwise(w, ref.W, bw, 4 * cfg.m * terms, label + " W", u=u, op_rel=orel)
    return my, mw


class BoundTracker:
    """The element-wise bounds B of a streamed sketch, updated alongside an
    oracle ``Sketch`` (same updates, same operand formation): for
    A <- theta A + eta H on columns J, B_Y <- |theta| B_Y + |eta| B(H Omega_J)
    and B_W <- |theta| B_W, B_W[:, J] += |eta| B(Psi H).  The scalings by
    theta and eta add one rounding each, counted in K."""

    def __init__(self, ref):
        self.ref = ref
        c = ref.cfg
        self.by = np.zeros((c.m, c.k))
        self.bw = np.zeros((c.l, c.n))
        self.terms = c.terms if c.dtype in ("bf16", "fp8x") else (3 if c.dtype == "fp8" else 1)
        self.ky = 0
        self.kw = 0

    def update(self, col0, block, theta=1.0, eta=1.0):
        from oracle.sketch import data_operand
        block = np.asarray(block, dtype=np.float64)
        if block.shape[0] == 3:
            block = np.concatenate([np.zeros_like(block[:1]), block], axis=0)
        nc = block.shape[2]
        self.by *= abs(theta)
        self.bw *= abs(theta)
        if theta != 1.0:
            self.ky += 2
            self.kw += 2
        if eta != 0.0:
            ops = data_operand(block, self.ref.cfg)
            self.by += abs(eta) * y_bound(ops, self.ref.omega_rows(col0, nc))
            self.bw[:, col0:col0 + nc] += abs(eta) * w_bound(self.ref.psi(), ops)
            self.ky += 4 * nc * self.terms + 1
            self.kw += 4 * self.ref.cfg.m * self.terms + 1

    def scale(self, theta):
        self.by *= abs(theta)
        self.bw *= abs(theta)
        self.ky += 1
        self.kw += 1

    def check(self, y, w, label, u=None):
        c = self.ref.cfg
        if u is None:
            u = U64 if c.dtype == "f64" else U32
        orel = operand_rel(c)
        assert_elementwise(y, self.ref.Y, self.by, self.ky, label + " Y", u=u, op_rel=orel)
        if w is not None:
            assert_elementwise(w, self.ref.W, self.bw, self.kw, label + " W", u=u, op_rel=orel)


# ---------------------------------------------------------------------------
# Sensitivity of the oracle's QB-stage diagnostics to rounding-level input
# perturbations (the scale of agreement that can be asked of quantities that
# depend on the non-unique H).

def oracle_sensitivity(ref, kind, rel_pert=1e-15, draws=4, with_range=True):
    """Relative change of the oracle's kappa / eps when Y is perturbed by a
    random relative 1e-15, the largest over a few draws (a single draw
    varies by several times): the scale below which GPU and oracle cannot be
    expected to agree (these diagnostics depend on the non-unique H).  The
    fourth value, the change of the projector onto range(H), forms m x m
    matrices and is skipped (0) when with_range is False."""
    out = [_sensitivity_draw(ref, kind, rel_pert, sd, with_range) for sd in range(draws)]
    return tuple(max(o[i] for o in out) for i in range(4))


def _sensitivity_draw(ref, kind, rel_pert, seed, with_range=True):
    from oracle import quaternion as qt
    from oracle.rangefinders import pseudo_qr, pseudo_svd
    rng = np.random.default_rng(seed)
    y2 = ref.Y * (1.0 + rel_pert * rng.standard_normal(ref.Y.shape))
    proj = (lambda z: qt.hamilton(z, qt.pinv(z))) if with_range else (lambda z: np.zeros((4, 1, 1)))
    if kind == "pseudo_qr":
        ha, a = pseudo_qr(ref.Y, seed=ref.cfg.seed)
        hb, b = pseudo_qr(y2, seed=ref.cfg.seed)
        ek = abs(a["kappa"] - b["kappa"]) / a["kappa"]
        ee = max(abs(x - y) / x for x, y in zip(a["eps"], b["eps"]))
        e0 = abs(a["kappa0"] - b["kappa0"]) / a["kappa0"]
        return ek, ee, e0, qt.fro(proj(ha) - proj(hb))
    ha, a = pseudo_svd(ref.Y, seed=ref.cfg.seed)
    hb, b = pseudo_svd(y2, seed=ref.cfg.seed)
    return abs(a["kappa"] - b["kappa"]) / a["kappa"], 0.0, 0.0, qt.fro(proj(ha) - proj(hb))


def error_sensitivity(a, ref, kind, rel_pert=1e-15, seed=1):
    """Relative change of the oracle's approximation error when Y is
    perturbed by a random relative 1e-15 (the error depends on H through
    X = (Psi H)^dagger W, which the ill-conditioned pseudo-QR factor
    amplifies)."""
    import copy
    from oracle import onepass
    rng = np.random.default_rng(seed)
    h0, x0, _ = onepass.qb_stage(ref, kind)
    e0 = onepass.rel_error(a, h0, x0)
    r2 = copy.copy(ref)
    r2.Y = ref.Y * (1.0 + rel_pert * rng.standard_normal(ref.Y.shape))
    h2, x2, _ = onepass.qb_stage(r2, kind)
    return abs(onepass.rel_error(a, h2, x2) - e0) / e0


# ---------------------------------------------------------------------------
# HX, the unique product of the QB stage (Lemma 4.2), on sampled rows and
# columns.

def qnorm_rows(h):
    """||h[i, :]||_2 of a quaternion matrix (4, r, c)."""
    return np.sqrt(np.sum(h * h, axis=(0, 2)))


def qnorm_cols(x):
    return np.sqrt(np.sum(x * x, axis=(0, 1)))


def hx_margin(q, x, h_o, x_o, rows, cols):
    """Largest |(QX - H_o X_o)_ij| / (||H_o[i,:]|| ||X_o[:,j]||) over the
    sampled rows (all columns) and sampled columns (all rows)."""
    from oracle import quaternion as qt
    out = 0.0
    d = qt.hamilton(q[:, rows, :], x) - qt.hamilton(h_o[:, rows, :], x_o)
    s = qnorm_rows(h_o[:, rows, :])[:, None] * qnorm_cols(x_o)[None, :]
    out = max(out, float(np.max(np.abs(d) / s[None])))
    d = qt.hamilton(q, x[:, :, cols]) - qt.hamilton(h_o, x_o[:, :, cols])
    s = qnorm_rows(h_o)[:, None] * qnorm_cols(x_o[:, :, cols])[None, :]
    out = max(out, float(np.max(np.abs(d) / s[None])))
    return out


def sample(n, fixed, count, seed):
    rng = np.random.default_rng(seed)
    idx = np.concatenate([np.asarray([f for f in fixed if 0 <= f < n]), rng.integers(0, n, count)])
    return np.unique(idx)
