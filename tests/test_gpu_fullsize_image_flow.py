"""Parity at the other two full-size workloads, in the launch configuration
the library uses for them:

* image: a pure quaternion 31365 x 27125 "colour image" (i, j, k planes,
  real part 0) stored in BF16, BF16 operands, quaternion Rademacher test
  matrices, k = 200, l = 401, column blocks of 2048;
* flow: a pure quaternion 2,097,152 x 300 snapshot matrix (three velocity
  components on a 128^3 grid) in FP32, streamed as 30 linear updates of 10
  columns, e4m3 operands with per-tile scales plus the residual correction
  terms, Gaussian test matrices, k = 60, l = 121.

The oracle checks sampled outputs one by one from the same operand values
(Section 4.1): rows of Y = A Omega, and columns (image) or rows (flow) of
W = Psi A; a row of W needs one row of Psi and all of A, which the test
streams through in chunks.  The QB stage is checked through properties that
hold at any size (Alg. 3 orthonormality, Prop. 3.4's kappa after three
corrections, Lemma 4.2's independence of HX from the rangefinder).

Tolerances: the operands are the oracle's values exactly (BF16 data and +-1
test entries; e4m3 test matrices times data whose e4m3 residual is carried
to 2^-16 of itself, i.e. to 2^-20 of the value), so what remains is the
FP32 accumulation over K terms per output.  With unit roundoff u = 2^-24
the usual probabilistic bound for a sum of K random-sign terms is of order
sqrt(K) u relative; the tests allow 4 sqrt(K) u, and at least 1e-5.
"""
import math

import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle import embeddings, lowprec, quaternion as qt
from tests.gpu_helpers import assert_elementwise, plane_abs_max, plane_abs_sum, w_bound, y_bound, to_numpy

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def accum_tol(terms):
    return max(1e-5, 4.0 * math.sqrt(terms) * U32)


def full_planes(a3):
    """(3, ...) pure quaternion planes -> (4, ...) with a zero real plane."""
    return np.concatenate([np.zeros_like(a3[:1]), a3], axis=0)


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def stream(sk, a, n, block):
    for c0 in range(0, n, block):
        sk.update(c0, a[:, :, c0:c0 + block])
    torch.cuda.synchronize()


def qb_checks(sk, a, label):
    """Run both rangefinders; return the two relative errors."""
    errs = {}
    for kind in ("pseudo_qr", "pseudo_svd"):
        q, x, rep = sk.finalize(kind)
        errs[kind] = sk.rel_error(a, q, x)
        if kind == "pseudo_svd":
            assert rep["orth_defect"] < 1e-10, (label, rep)
            assert abs(rep["kappa"] - 1.0) < 1e-8, (label, rep)
        else:
            assert rep["kappa"] < 10.0 and rep["kappa"] <= rep["kappa_initial"], (label, rep)
        del q, x
    print(label, "errors", errs, flush=True)
    assert abs(errs["pseudo_qr"] - errs["pseudo_svd"]) <= 1e-8 * errs["pseudo_qr"]
    return errs


# ---------------------------------------------------------------- image

IM, IN, IK, IL, IBLOCK = 31365, 27125, 200, 401, 2048


@pytest.fixture(scope="module")
def image_dev():
    a = qs.to_colmajor(synth.image_planes(IM, IN, device="cuda", dtype=torch.bfloat16))
    torch.cuda.synchronize()
    yield a
    del a
    torch.cuda.empty_cache()


def test_image_sampled_sketches(image_dev):
    sk = qs.Sketcher(IM, IN, IK, IL, seed=0, embedding="rademacher", input_dtype="bf16",
                     sketch_dtype="bf16", pure=True, split_terms=1, max_block_cols=IBLOCK)
    stream(sk, image_dev, IN, IBLOCK)
    y, w = sk.sketches()
    rng = np.random.default_rng(31)
    rows = np.unique(np.concatenate([[0, 1, 127, 128, 2047, 2048, IM - 37, IM - 1],
                                     rng.integers(0, IM, 8)]))
    cols = np.unique(np.concatenate([[0, 1, 2047, 2048, 26623, 26624, IN - 1],
                                     rng.integers(0, IN, 8)]))
    y_dev = to_numpy(y[:, rows, :])
    w_dev = to_numpy(w[:, :, cols])
    sk.close()
    del y, w
    a_rows = full_planes(image_dev[:, rows, :].double().cpu().numpy())
    om = embeddings.omega("rademacher", np.arange(IN), IK, 0, "bf16")
    y_ref = qt.hamilton(a_rows, om)
    by = y_bound(a_rows, om)
    del om
    a_cols = full_planes(image_dev[:, :, cols].double().cpu().numpy())
    ps = embeddings.psi("rademacher", IL, np.arange(IM), 0, "bf16")
    w_ref = qt.hamilton(ps, a_cols)
    bw = w_bound(ps, a_cols)
    ey, ew = rel(y_dev, y_ref), rel(w_dev, w_ref)
    print(f"image: sampled rel. diff Y {ey:.2e}, W {ew:.2e}", flush=True)
    assert_elementwise(y_dev, y_ref, by, 3 * IN, "image Y rows")
    assert_elementwise(w_dev, w_ref, bw, 3 * IM, "image W cols")
    assert ey < accum_tol(3 * IN) and ew < accum_tol(3 * IM)


def test_image_qb_stage(image_dev):
    errs = {}
    for sketch in ("f64", "bf16"):
        sk = qs.Sketcher(IM, IN, IK, IL, seed=0, embedding="rademacher", input_dtype="bf16",
                         sketch_dtype=sketch, pure=True, split_terms=1, max_block_cols=IBLOCK)
        stream(sk, image_dev, IN, IBLOCK)
        errs[sketch] = qb_checks(sk, image_dev, "image " + sketch)
        sk.close()
    # same test matrices and exact operands: the BF16 path reaches the FP64
    # path's error within 1e-3 relative
    for kind in ("pseudo_qr", "pseudo_svd"):
        assert abs(errs["bf16"][kind] - errs["f64"][kind]) <= 1e-3 * errs["f64"][kind]


# ----------------------------------------------------------------- flow

FGRID, FN, FK, FL, FBLOCK = 128, 300, 60, 121, 10
FM = FGRID ** 3


@pytest.fixture(scope="module")
def flow_dev():
    a = qs.to_colmajor(synth.flow_snapshots(FGRID, FN, device="cuda"))
    torch.cuda.synchronize()
    yield a
    del a
    torch.cuda.empty_cache()


def test_flow_sampled_sketches(flow_dev):
    sk = qs.Sketcher(FM, FN, FK, FL, seed=0, embedding="gaussian", input_dtype="f32",
                     sketch_dtype="fp8", pure=True, split_terms=2, max_block_cols=FBLOCK)
    stream(sk, flow_dev, FN, FBLOCK)
    y, w = sk.sketches()
    rng = np.random.default_rng(32)
    rows = np.unique(np.concatenate([[0, 1, 31, 32, 1023, 1024, FM - 33, FM - 1],
                                     rng.integers(0, FM, 8)]))
    wrows = np.array([0, 1, 63, 64, FL - 1])
    y_dev = to_numpy(y[:, rows, :])
    w_dev = to_numpy(w[:, wrows, :])
    sk.close()
    del y, w
    # rows of Y: A[rows, :] Omega, with e4m3 test matrices
    a_rows = full_planes(flow_dev[:, rows, :].double().cpu().numpy())
    om = embeddings.omega("gaussian", np.arange(FN), FK, 0, "fp8")
    y_ref = qt.hamilton(a_rows, om)
    by = y_bound(a_rows, om)
    # rows of W: Psi[wrows, :] A, accumulated over chunks of rows of A
    w_ref = np.zeros((4, len(wrows), FN))
    bw = np.zeros((len(wrows), FN))
    chunk = 1 << 18
    for r0 in range(0, FM, chunk):
        r = np.arange(r0, min(FM, r0 + chunk), dtype=np.uint64)
        ps = lowprec.round_dtype(embeddings.entries("gaussian", r[None, :],
                                                    wrows.astype(np.uint64)[:, None],
                                                    embeddings.STREAM_PSI, 0), "fp8")
        a_chunk = full_planes(flow_dev[:, r0:r0 + len(r), :].double().cpu().numpy())
        w_ref += qt.hamilton(ps, a_chunk)
        bw += plane_abs_max(ps) @ plane_abs_sum(a_chunk)
        del ps, a_chunk
    ey, ew = rel(y_dev, y_ref), rel(w_dev, w_ref)
    print(f"flow: sampled rel. diff Y {ey:.2e}, W {ew:.2e}", flush=True)
    # e4m3 data plus the residual carried as two bf16 terms: 2^-17 per operand
    assert_elementwise(y_dev, y_ref, by, 3 * 3 * FN, "flow Y rows", op_rel=2.0 ** -17)
    assert_elementwise(w_dev, w_ref, bw, 3 * 3 * FM, "flow W rows", op_rel=2.0 ** -17)
    assert ey < accum_tol(3 * FN) and ew < accum_tol(3 * FM)


def test_flow_qb_stage(flow_dev):
    sk = qs.Sketcher(FM, FN, FK, FL, seed=0, embedding="gaussian", input_dtype="f32",
                     sketch_dtype="fp8", pure=True, split_terms=2, max_block_cols=FBLOCK)
    stream(sk, flow_dev, FN, FBLOCK)
    e8 = qb_checks(sk, flow_dev, "flow fp8")
    sk.close()
    sk = qs.Sketcher(FM, FN, FK, FL, seed=0, embedding="gaussian", input_dtype="f32",
                     sketch_dtype="f64", pure=True, max_block_cols=FBLOCK)
    stream(sk, flow_dev, FN, FBLOCK)
    e64 = qb_checks(sk, flow_dev, "flow f64")
    sk.close()
    # the e4m3 test matrices are another draw than the FP64 ones, so the two
    # errors need not agree to rounding; the accuracy target of the low
    # precision path is the FP64 plain method's error within 1e-3 relative
    for kind in e8:
        assert abs(e8[kind] - e64[kind]) <= 1e-3 * e64[kind], (e8, e64)
