"""Parity at the benchmark's full size: A in Q^{20000 x 15000} (four FP32
planes, rank 50 with sigma_i = i^-2 plus 1e-4 noise), Gaussian test
matrices, k = 100, l = 201, column blocks of 2048, in the launch
configuration that bench.py times.

The oracle cannot sketch the whole matrix in seconds, so it computes sampled
entries one row or column at a time: rows of Y = A Omega and columns of
W = Psi A at tile boundaries, ragged tails and random positions, from the
same operand values (Section 4.1).  The QB stage is checked through
properties that hold at any size: pseudo-SVD returns an orthonormal basis
(Alg. 3), pseudo-QR's kappa is small after three corrections (Prop. 3.4),
both rangefinders give the same error (Lemma 4.2: HX does not depend on the
rangefinder), and the low-precision sketches reach the FP64 error within
1e-3 relative.
"""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle import embeddings, lowprec, quaternion as qt
from tests.gpu_helpers import assert_elementwise, w_bound, y_bound, to_numpy

pytestmark = pytest.mark.gpu

M, N, K, L, BLOCK = 20000, 15000, 100, 201, 2048
SEED = 0


@pytest.fixture(scope="module")
def a_dev():
    a = qs.to_colmajor(synth.config2(device="cuda", m=M, n=N))
    torch.cuda.synchronize()
    yield a
    del a
    torch.cuda.empty_cache()


def run_updates(a, sketch, terms=1):
    sk = qs.Sketcher(M, N, K, L, seed=SEED, embedding="gaussian", input_dtype="f32",
                     sketch_dtype=sketch, split_terms=terms, max_block_cols=BLOCK)
    for c0 in range(0, N, BLOCK):
        sk.update(c0, a[:, :, c0:c0 + BLOCK])
    torch.cuda.synchronize()
    return sk


def operand(vals, sketch, terms):
    """The values the sketch multiplies (FP32 data as is, bf16 split summed)."""
    if sketch == "bf16":
        return sum(lowprec.split_bf16(vals, terms))
    return vals


def sample_rows():
    rng = np.random.default_rng(7)
    fixed = [0, 1, 15, 16, 63, 64, 127, 128, 1279, 1280, 19967, 19968, M - 2, M - 1]
    return np.unique(np.concatenate([fixed, rng.integers(0, M, 10)]))


def sample_cols():
    rng = np.random.default_rng(8)
    fixed = [0, 1, 63, 64, 2047, 2048, 2049, 4095, 4096, 14335, 14336, N - 2, N - 1]
    return np.unique(np.concatenate([fixed, rng.integers(0, N, 10)]))


@pytest.mark.parametrize("sketch,terms", [("f32", 1), ("bf16", 3), ("bf16", 2)])
def test_fullsize_sampled_sketches(a_dev, sketch, terms):
    sk = run_updates(a_dev, sketch, terms)
    y, w = sk.sketches()
    rows, cols = sample_rows(), sample_cols()
    y_dev = to_numpy(y[:, rows, :])
    w_dev = to_numpy(w[:, :, cols])
    sk.close()
    del y, w
    rnd = "f32" if sketch == "f32" else "bf16"
    # rows of Y: A[rows, :] Omega over all n columns
    a_rows = operand(a_dev[:, rows, :].double().cpu().numpy(), sketch, terms)
    om = embeddings.omega("gaussian", np.arange(N), K, SEED, rnd)
    y_ref = qt.hamilton(a_rows, om)
    # columns of W: Psi A[:, cols] over all m rows
    a_cols = operand(a_dev[:, :, cols].double().cpu().numpy(), sketch, terms)
    ps = embeddings.psi("gaussian", L, np.arange(M), SEED, rnd)
    w_ref = qt.hamilton(ps, a_cols)
    ey = np.linalg.norm(y_dev - y_ref) / np.linalg.norm(y_ref)
    ew = np.linalg.norm(w_dev - w_ref) / np.linalg.norm(w_ref)
    print(f"{sketch} x{terms}: sampled rel. diff Y {ey:.2e}, W {ew:.2e}", flush=True)
    # entry by entry: within 8 sqrt(K) u B of the oracle (B = sum of |terms|)
    assert_elementwise(y_dev, y_ref, y_bound(a_rows, om), 4 * N * terms, f"full-size {sketch} x{terms} Y rows")
    assert_elementwise(w_dev, w_ref, w_bound(ps, a_cols), 4 * M * terms, f"full-size {sketch} x{terms} W cols")
    assert ey < 1e-5 and ew < 1e-5


def test_fullsize_qb_properties(a_dev):
    errs = {}
    for sketch, terms in (("f64", 1), ("bf16", 3)):
        sk = run_updates(a_dev, sketch, terms)
        for kind in ("pseudo_qr", "pseudo_svd"):
            q, x, rep = sk.finalize(kind)
            errs[(sketch, kind)] = sk.rel_error(a_dev, q, x)
            if kind == "pseudo_svd":
                assert rep["orth_defect"] < 1e-10
                assert abs(rep["kappa"] - 1.0) < 1e-8
            else:
                assert rep["kappa"] < 10.0 and rep["kappa"] <= rep["kappa_initial"]
            del q, x
        sk.close()
    print("full-size errors", errs, flush=True)
    for sketch in ("f64", "bf16"):
        e_qr, e_svd = errs[(sketch, "pseudo_qr")], errs[(sketch, "pseudo_svd")]
        assert abs(e_qr - e_svd) <= 1e-8 * e_qr
    for kind in ("pseudo_qr", "pseudo_svd"):
        ref = errs[("f64", kind)]
        assert abs(errs[("bf16", kind)] - ref) <= 1e-3 * ref
