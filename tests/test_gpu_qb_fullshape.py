"""Oracle parity at the full workloads' shapes, through the C ABI:

* the 20000 x 15000 FP32 matrix (rank 50, sigma_i = i^-2, 1e-4 noise),
  Gaussian test matrices, k = 100, l = 201, column blocks of 2048, in the
  FP64 path and in the benchmark's BF16 two-term path;
* the 31365 x 27125 pure-quaternion BF16 image, quaternion Rademacher test
  matrices, k = 200, l = 401, BF16 operands.

The oracle streams the same matrix block by block (Section 4.1, linear
updates) into its FP64 sketch with the device's operand values, so every
entry of Y and W is compared (``gpu_helpers``: within 8 sqrt(K) u B of the
oracle's value, B the sum of the absolute values of the entry's K terms).

The QB stage (Alg. 4: rangefinder, Psi H, core solve by Alg. 2) is compared
on identical inputs: the device context is loaded with the oracle's sketches
(FP32-rounded where the context keeps FP32 sketches, and the oracle then
works on those same rounded values), and keeps the test matrix Psi it staged
during its own updates.  H and X are not unique, HX is (Lemma 4.2): sampled
rows and columns of HX are compared entry by entry against
||H_o[i, :]|| ||X_o[:, j]|| (a bound on |(HX)_ij|), and kappa and the eps of
the corrections against the oracle's own change under a relative 1e-15
perturbation of Y.
"""
import sys

import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle import onepass
from oracle.sketch import Sketch, SketchConfig
from tests.gpu_helpers import U64, BoundTracker, hx_margin, oracle_sensitivity, sample, to_numpy

pytestmark = pytest.mark.gpu

# HX from identical inputs: FP64 arithmetic on both sides, different
# factorisation routes (CholeskyQR2 against Householder, the eigensolver of
# R R^* against the SVD of chi_Y), so agreement is to a modest multiple of
# the conditioning of the rangefinder and core solve times 2^-53
HX_TOL = 1e-9


def rounded_copy(ref, to_f32):
    """The oracle sketch with Y and W as the context stores them."""
    import copy
    r = copy.copy(ref)
    if to_f32:
        r.Y = ref.Y.astype(np.float32).astype(np.float64)
        r.W = ref.W.astype(np.float32).astype(np.float64)
    return r


def qb_compare(sk, ref, kind, rows, cols, label):
    """Run the device QB stage on the sketches loaded into ``sk`` and the
    oracle's on ``ref``; compare HX, kappa and eps."""
    q, x, rep = sk.finalize(kind)
    qn, xn = to_numpy(q), to_numpy(x)
    del q, x
    h_o, x_o, info = onepass.qb_stage(ref, kind)
    mg = hx_margin(qn, xn, h_o, x_o, rows, cols)
    sk_, se_, s0_, _ = oracle_sensitivity(ref, kind, draws=2, with_range=False)
    d_k = abs(rep["kappa"] - info["kappa"]) / info["kappa"]
    msg = (f"{label} {kind}: HX margin {mg:.2e} (limit {HX_TOL:g}); kappa {rep['kappa']:.6f} "
           f"(oracle {info['kappa']:.6f}, diff {d_k:.1e}, sensitivity {sk_:.1e})")
    if kind == "pseudo_qr":
        d_e = max(abs(u - v) / v for u, v in zip(rep["eps"], info["eps"]))
        msg += f"; eps diff {d_e:.1e} (sensitivity {se_:.1e})"
    print(msg, flush=True)
    assert mg < HX_TOL, (label, kind, mg)
    assert d_k <= max(1e-9, 100 * sk_), (label, kind, d_k, sk_)
    if kind == "pseudo_qr":
        assert rep["kappa"] < 10 and len(rep["eps"]) == 3
        assert d_e <= max(1e-9, 100 * se_), (label, d_e, se_)
    else:
        assert rep["orth_defect"] < 1e-10
        assert abs(rep["kappa"] - 1.0) < 1e-8
    return qn, xn, h_o, x_o


# ----------------------------------------------------------- 20000 x 15000

M, N, K, L, BLOCK = 20000, 15000, 100, 201, 2048
C2_ROWS = sample(M, [0, 1, 15, 16, 63, 64, 19967, 19968, M - 1], 12, 41)
C2_COLS = sample(N, [0, 1, 63, 64, 2047, 2048, 14335, 14336, N - 1], 12, 42)
C2_PATHS = {"f64": dict(sketch_dtype="f64", split_terms=1),
            "bf16x2": dict(sketch_dtype="bf16", split_terms=2)}


@pytest.fixture(scope="module")
def c2():
    """The matrix on the device and the oracle's FP64 sketches of it, with
    the unrounded test matrices (the FP64 path) and with the bf16-rounded ones
    (the QB stage of the BF16 path takes sketches made with those)."""
    a = qs.to_colmajor(synth.config2(device="cuda", m=M, n=N))
    torch.cuda.synchronize()
    refs = {"f64": Sketch(SketchConfig(M, N, K, L, seed=0, dtype="f64")),
            "bf16x2": Sketch(SketchConfig(M, N, K, L, seed=0, dtype="f64", embedding_dtype="bf16"))}
    bt = BoundTracker(refs["f64"])
    for c0 in range(0, N, BLOCK):
        blk = a[:, :, c0:c0 + BLOCK].double().cpu().numpy()
        for p in refs:
            refs[p].update(c0, blk)
        bt.update(c0, blk)
        del blk
        print(f"c2 oracle: columns {c0} .. {min(N, c0 + BLOCK)} done", file=sys.stderr, flush=True)
    yield a, refs, bt
    del a
    torch.cuda.empty_cache()


def c2_context(a, path):
    sk = qs.Sketcher(M, N, K, L, seed=0, embedding="gaussian", input_dtype="f32",
                     max_block_cols=BLOCK, **C2_PATHS[path])
    for c0 in range(0, N, BLOCK):
        sk.update(c0, a[:, :, c0:c0 + BLOCK])
    torch.cuda.synchronize()
    return sk


@pytest.mark.timeout(600)
def test_c2_sketches_every_entry(c2):
    """Every entry of the FP64 path's sketches (the BF16 path's are compared
    on sampled rows and columns in test_gpu_fullsize.py)."""
    a, refs, bt = c2
    sk = c2_context(a, "f64")
    y, w = (to_numpy(t) for t in sk.sketches())
    sk.close()
    bt.check(y, w, "20000x15000 f64", u=U64)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("path", ["f64", "bf16x2"])
def test_c2_qb_stage_vs_oracle(c2, path):
    """The device QB stage on the oracle's sketches (rounded to FP32 for the
    BF16 context, whose sketches are FP32), with the Psi the context staged
    during its updates; then, for the FP64 path, the relative errors of the
    device's own end-to-end result against the oracle's."""
    a, refs, _ = c2
    sk = c2_context(a, path)
    own = {}
    if path == "f64":
        # the FP64 device sketch is the oracle's to rounding: compare the
        # end-to-end errors too
        for kind in ("pseudo_qr", "pseudo_svd"):
            q, x, _ = sk.finalize(kind)
            own[kind] = sk.rel_error(a, q, x)
            del q, x
    ref = rounded_copy(refs[path], to_f32=path != "f64")
    yd = qs.to_colmajor(torch.from_numpy(ref.Y).cuda())
    wd = qs.to_colmajor(torch.from_numpy(ref.W).cuda())
    sk.set_sketches(yd, wd, N)
    del yd, wd
    for kind in ("pseudo_qr", "pseudo_svd"):
        qn, xn, h_o, x_o = qb_compare(sk, ref, kind, C2_ROWS, C2_COLS, f"20000x15000 {path}")
        if path == "f64":
            e_o = onepass.rel_error(_host_planes(a), h_o, x_o)
            d = abs(own[kind] - e_o) / e_o
            print(f"  end-to-end error {own[kind]:.9e} (oracle {e_o:.9e}, rel. diff {d:.1e})", flush=True)
            assert d < 1e-6
    sk.close()


_HOST = {}


def _host_planes(a):
    """FP64 host copy of a device matrix (cached: the error pass reads it
    once per rangefinder)."""
    key = a.data_ptr()
    if key not in _HOST:
        _HOST.clear()
        _HOST[key] = a.double().cpu().numpy()
    return _HOST[key]


# ------------------------------------------------------------------- image

IM, IN, IK, IL, IBLOCK = 31365, 27125, 200, 401, 2048
IM_ROWS = sample(IM, [0, 1, 127, 128, IM - 37, IM - 1], 10, 43)
IM_COLS = sample(IN, [0, 1, 2047, 2048, 26623, 26624, IN - 1], 10, 44)


@pytest.mark.timeout(900)
def test_image_sketches_and_qb_stage_vs_oracle():
    """Every entry of both sketches, then the QB stage on the oracle's
    sketches with both rangefinders, at k = 200, l = 401."""
    a = qs.to_colmajor(synth.image_planes(IM, IN, device="cuda", dtype=torch.bfloat16))
    torch.cuda.synchronize()
    sk = qs.Sketcher(IM, IN, IK, IL, seed=0, embedding="rademacher", input_dtype="bf16",
                     sketch_dtype="bf16", pure=True, split_terms=1, max_block_cols=IBLOCK)
    for c0 in range(0, IN, IBLOCK):
        sk.update(c0, a[:, :, c0:c0 + IBLOCK])
    # the data are bf16 values and the test matrices +-1, exact in every
    # format: the oracle's FP64 sketch has the device's operand values
    ref = Sketch(SketchConfig(IM, IN, IK, IL, seed=0, embedding="rademacher", dtype="f64"))
    bt = BoundTracker(ref)
    for c0 in range(0, IN, IBLOCK):
        blk = a[:, :, c0:c0 + IBLOCK].double().cpu().numpy()
        blk = np.concatenate([np.zeros_like(blk[:1]), blk], axis=0)
        ref.update(c0, blk)
        bt.update(c0, blk)
        del blk
        print(f"image oracle: columns {c0} .. {min(IN, c0 + IBLOCK)} done", file=sys.stderr, flush=True)
    del a
    torch.cuda.empty_cache()
    y, w = (to_numpy(t) for t in sk.sketches())
    bt.check(y, w, "image", u=2.0 ** -24)
    del y, w
    ref32 = rounded_copy(ref, to_f32=True)
    yd = qs.to_colmajor(torch.from_numpy(ref32.Y).cuda())
    wd = qs.to_colmajor(torch.from_numpy(ref32.W).cuda())
    sk.set_sketches(yd, wd, IN)
    del yd, wd
    for kind in ("pseudo_qr", "pseudo_svd"):
        qb_compare(sk, ref32, kind, IM_ROWS, IM_COLS, "image")
    sk.close()
