"""GPU parity of the HIP path with the oracle, through the C ABI.

Tolerances:
  * sketches, entry by entry: every entry of Y and W is a sum of K signed
    products (K = 4n for Y, 4m for W, times the number of bf16 terms); the
    device's value must lie within 8 sqrt(K) u B of the oracle's, with B the
    sum of the absolute values of the terms and u the unit roundoff of the
    accumulation (2^-53 for FP64, 2^-24 for FP32; ``gpu_helpers``).  The BF16
    operands are exact (the oracle forms the same bf16 values), so what
    remains is the accumulation order;
  * test-matrix values: bit-exact for Rademacher and for BF16 rounding of the
    Gaussian, 1e-14 relative or absolute for FP64, 2e-6 (a few FP32 ulp) for
    FP32.
The QB-stage outputs H and X are not unique (Lemma 4.2, phases and pair
representatives), so the product HX, kappa(H), the error ||A - HX|| and the
orthonormality of pseudo-SVD are compared instead.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import embeddings, onepass, quaternion as qt
from oracle.sketch import SketchConfig, sketch_matrix
from tests.gpu_helpers import (check_sketches, error_sensitivity, input_values, oracle_sensitivity, rel,
                               run_sketch, to_numpy)

pytestmark = pytest.mark.gpu


def identity_q(n):
    a = np.zeros((4, n, n))
    a[0] = np.eye(n)
    return a


@pytest.mark.parametrize("sketch,emb", [("f64", "gaussian"), ("f64", "rademacher"),
                                        ("f32", "gaussian"), ("bf16", "gaussian"),
                                        ("bf16", "rademacher")])
def test_test_matrix_values(sketch, emb):
    """With A = I the sketches are the test matrices themselves:
    Y = Omega[0:n, :] and W = Psi[:, 0:m]."""
    n, k, l = 320, 16, 37
    a = identity_q(n)
    dt = "f64" if sketch == "f64" else "f32"
    sk, _ = run_sketch(a, n, n, k, l, 64, dtype=dt, sketch=sketch, emb=emb, seed=12345)
    y, w = (to_numpy(t) for t in sk.sketches())
    rnd = {"f64": "f64", "f32": "f32", "bf16": "bf16"}[sketch]
    om = embeddings.omega(emb, np.arange(n), k, 12345, rnd)
    ps = embeddings.psi(emb, l, np.arange(n), 12345, rnd)
    if sketch == "bf16" or emb == "rademacher":
        np.testing.assert_array_equal(y, om)
        np.testing.assert_array_equal(w, ps)
    elif sketch == "f64":
        # the oracle rounds 2 pi u before its cosine, the device evaluates
        # cos(pi * 2u): both are within a few ulp of |theta| in absolute terms
        np.testing.assert_allclose(y, om, rtol=1e-14, atol=1e-14)
        np.testing.assert_allclose(w, ps, rtol=1e-14, atol=1e-14)
    else:
        assert np.max(np.abs(y - om) / np.maximum(np.abs(om), 1e-30)) < 2e-6
        assert np.max(np.abs(w - ps) / np.maximum(np.abs(ps), 1e-30)) < 2e-6


CASES = [
    # sketch dtype, input dtype, embedding, terms, tolerance
    ("f64", "f64", "gaussian", 1, 1e-12),
    ("f64", "f64", "rademacher", 1, 1e-12),
    ("f32", "f32", "gaussian", 1, 1e-5),
    ("f32", "f32", "rademacher", 1, 1e-5),
    ("bf16", "f32", "gaussian", 1, 1e-5),
    ("bf16", "f32", "gaussian", 2, 1e-5),
    ("bf16", "f32", "gaussian", 3, 1e-5),
    ("bf16", "bf16", "rademacher", 1, 1e-5),
]


@pytest.mark.parametrize("sketch,dtype,emb,terms,tol", CASES)
def test_sketch_parity_ragged(sketch, dtype, emb, terms, tol):
    """Y and W against the oracle on a ragged shape (several tiles plus tails)
    streamed in uneven blocks."""
    m, n, k, l, block = 333, 257, 12, 25, 50
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(10)), 1e-3, 77).numpy()
    a = input_values(a, dtype)
    sk, _ = run_sketch(a, m, n, k, l, block, dtype=dtype, sketch=sketch, emb=emb, seed=5,
                       terms=terms)
    y, w = (to_numpy(t) for t in sk.sketches())
    cfg = SketchConfig(m, n, k, l, seed=5, embedding=emb, dtype=sketch, terms=terms)
    ref = sketch_matrix(a, cfg, block_cols=block)
    check_sketches(y, w, ref, a, f"ragged {sketch}/{dtype}/{emb}/x{terms}", block_cols=block)
    assert rel(y, ref.Y) < tol
    assert rel(w, ref.W) < tol


MFMA_CASES = [
    ("f32", "f32", "gaussian", 1, False),
    ("bf16", "f32", "gaussian", 3, False),
    ("bf16", "f32", "rademacher", 2, True),
    ("bf16", "bf16", "rademacher", 1, True),
]


@pytest.mark.parametrize("sketch,dtype,emb,terms,pure", MFMA_CASES)
def test_matrix_core_sketch_multitile(sketch, dtype, emb, terms, pure):
    """Shapes that exercise the matrix-core kernels' tiling: 7 column tiles
    of Y, two row groups of W, several row chunks of A (split K) and ragged
    edges everywhere.  FP32 accumulation bound 1e-5."""
    m, n, k, l, block = 1500, 300, 100, 201, 130
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.85 ** np.arange(30)), 1e-3, 88).numpy()
    if pure:
        a[0] = 0.0
    a = input_values(a, dtype)
    sk, _ = run_sketch(a, m, n, k, l, block, dtype=dtype, sketch=sketch, emb=emb, seed=21,
                       terms=terms, pure=pure)
    y, w = (to_numpy(t) for t in sk.sketches())
    cfg = SketchConfig(m, n, k, l, seed=21, embedding=emb, dtype=sketch, terms=terms)
    ref = sketch_matrix(a, cfg, block_cols=block)
    check_sketches(y, w, ref, a, f"multitile {sketch}/{dtype}/{emb}/x{terms}", block_cols=block)


def test_streaming_order_and_pure_input():
    m, n, k, l, block = 200, 160, 8, 17, 32
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.7 ** np.arange(6)), 1e-3, 78).numpy()
    a[0] = 0.0                                      # pure quaternion
    s1, _ = run_sketch(a, m, n, k, l, block, seed=3)
    s2, _ = run_sketch(a, m, n, k, l, block, seed=3, order=[4, 1, 3, 0, 2], pure=True)
    y1, w1 = (to_numpy(t) for t in s1.sketches())
    y2, w2 = (to_numpy(t) for t in s2.sketches())
    assert rel(y2, y1) < 1e-13 and rel(w2, w1) < 1e-13


@pytest.fixture(scope="module")
def config1():
    a = synth.config1().numpy()
    cfg = SketchConfig(1000, 800, 40, 81, seed=0)
    ref = sketch_matrix(a, cfg, block_cols=256)
    sk, dev = run_sketch(a, 1000, 800, 40, 81, 256, seed=0)
    return a, ref, sk, dev


def test_config1_sketches(config1):
    a, ref, sk, _ = config1
    y, w = (to_numpy(t) for t in sk.sketches())
    check_sketches(y, w, ref, a, "config 1 f64", block_cols=256)


@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_config1_qb_stage(config1, kind):
    a, ref, sk, dev = config1
    q, x, rep = sk.finalize(kind)
    qn, xn = to_numpy(q), to_numpy(x)
    h_o, x_o, info = onepass.qb_stage(ref, kind)
    hx = qt.hamilton(qn, xn)
    hx_o = qt.hamilton(h_o, x_o)
    d_hx = rel(hx, hx_o)
    e_gpu = sk.rel_error(dev, q, x)
    e_o = onepass.rel_error(a, h_o, x_o)
    # the oracle's own change under a rounding-level perturbation of its
    # input: the scale of agreement that can be asked of kappa, eps and the
    # error, which depend on the non-unique H
    es = error_sensitivity(a, ref, kind)
    sk_, se_, s0_, sr_ = oracle_sensitivity(ref, kind)
    kap = rep["kappa"]
    d_e = abs(e_gpu - e_o) / e_o
    d_k = abs(kap - info["kappa"]) / info["kappa"]
    print(f"config 1 {kind}: |HX - HX_o|/|HX_o| {d_hx:.2e}; error diff {d_e:.2e} "
          f"(oracle sensitivity {es:.2e}, ratio {d_e / max(es, 1e-300):.3g}); kappa diff {d_k:.2e} "
          f"(sensitivity {sk_:.2e}, ratio {d_k / max(sk_, 1e-300):.3g})", flush=True)
    if kind == "pseudo_qr":
        d_eps = max(abs(u - v) / v for u, v in zip(rep["eps"], info["eps"]))
        d_k0 = abs(rep["kappa_initial"] - info["kappa0"]) / info["kappa0"]
        print(f"  eps diff {d_eps:.2e} (sensitivity {se_:.2e}, ratio {d_eps / max(se_, 1e-300):.3g}); "
              f"kappa0 diff {d_k0:.2e} (sensitivity {s0_:.2e})", flush=True)
    assert d_hx < 1e-9                                 # HX is unique (Lemma 4.2)
    assert d_e <= max(1e-6, 100 * es)
    np.testing.assert_allclose(e_gpu, onepass.rel_error(a, qn, xn), rtol=1e-9)
    # same range as the oracle's factor, up to the oracle's own sensitivity
    # (the paper notes pseudo-QR's weaker range precision, Section 3.3)
    proj = lambda z: qt.hamilton(z, qt.pinv(z))
    assert qt.fro(proj(qn) - proj(h_o)) < max(1e-8, 10 * sr_)
    np.testing.assert_allclose(kap, info["kappa"], rtol=max(1e-9, 100 * sk_))
    if kind == "pseudo_qr":
        assert kap < 10 and len(rep["eps"]) == 3
        np.testing.assert_allclose(rep["eps"], info["eps"], rtol=max(1e-9, 100 * se_))
        # the device estimates kappa(H0) from the Gram of H0, whose relative
        # accuracy for the smallest singular value is ~ kappa0^2 u
        k0 = info["kappa0"]
        np.testing.assert_allclose(rep["kappa_initial"], k0, rtol=max(1e-6, 100 * s0_, 10 * k0 * k0 * 2.0 ** -53))
    else:
        assert rep["orth_defect"] < 1e-10
        np.testing.assert_allclose(qt.hamilton(qt.conj_t(qn), qn), qt.eye(40), atol=1e-10)
        # Thm 3.1: the columns are left singular vectors of Y, so Q^* Y Y^* Q is
        # diagonal, holding sigma_i^2 in descending order
        y = to_numpy(sk.sketches()[0])
        g = qt.hamilton(qt.hamilton(qt.conj_t(qn), y), qt.hamilton(qt.conj_t(y), qn))
        sig2 = qt.singular_values(ref.Y) ** 2
        dg = g[0].diagonal()
        top = sig2 > 1e-6 * sig2[0]                    # well-resolved singular values
        np.testing.assert_allclose(dg[top], sig2[top], rtol=1e-9)
        off = g.copy()
        off[0] -= np.diag(dg)
        assert np.abs(off).max() < 1e-10 * sig2[0]


@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_exact_low_rank_recovery(kind):
    """Exact rank r <= k with no noise is recovered to rounding (Z15 for the
    rank-deficient pseudo-QR factor)."""
    m, n, k, l = 300, 240, 8, 17
    a = synth.lowrank_plus_noise(m, n, torch.tensor([1.0, 0.5, 0.3, 0.2]), 0.0, 79).numpy()
    sk, dev = run_sketch(a, m, n, k, l, 60, seed=9)
    q, x, rep = sk.finalize(kind)
    assert sk.rel_error(dev, q, x) < 1e-8


@pytest.mark.parametrize("emb,rnd", [("gaussian", "bf16"), ("gaussian", "fp8"), ("rademacher", "bf16")])
def test_fp64_sketch_with_rounded_test_matrices(emb, rnd):
    """An FP64 context with embedding_round takes the test matrices of a
    low-precision sketch (the reference of the equal-error comparison): with
    A = I its sketches are exactly those rounded values; on data, Y, W and
    the QB stage (which regenerates Psi for Psi Q) match the oracle's FP64
    sketch with the same rounded test matrices."""
    import paper_2404_14783_amd as qs
    n, k, l = 320, 16, 37
    dev = qs.to_colmajor(torch.from_numpy(identity_q(n)).cuda())
    sk = qs.Sketcher(n, n, k, l, seed=12345, embedding=emb, max_block_cols=64, embedding_round=rnd)
    for c0 in range(0, n, 64):
        sk.update(c0, dev[:, :, c0:c0 + 64])
    y, w = (to_numpy(t) for t in sk.sketches())
    sk.close()
    np.testing.assert_array_equal(y, embeddings.omega(emb, np.arange(n), k, 12345, rnd))
    np.testing.assert_array_equal(w, embeddings.psi(emb, l, np.arange(n), 12345, rnd))
    m, n, k, l, block = 333, 257, 12, 25, 50
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(10)), 1e-4, 77).numpy()
    cfg = SketchConfig(m, n, k, l, seed=5, embedding=emb, dtype="f64", embedding_dtype=rnd)
    ref = sketch_matrix(a, cfg, block_cols=block)
    sk = qs.Sketcher(m, n, k, l, seed=5, embedding=emb, max_block_cols=block, embedding_round=rnd)
    dev = qs.to_colmajor(torch.from_numpy(a).cuda())
    for c0 in range(0, n, block):
        sk.update(c0, dev[:, :, c0:c0 + block])
    y, w = (to_numpy(t) for t in sk.sketches())
    check_sketches(y, w, ref, a, f"f64 with {rnd} test matrices ({emb})", block_cols=block)
    for kind in ("pseudo_qr", "pseudo_svd"):
        q, x, _ = sk.finalize(kind)
        h_o, x_o, _ = onepass.qb_stage(ref, kind)
        d = rel(qt.hamilton(to_numpy(q), to_numpy(x)), qt.hamilton(h_o, x_o))
        print(f"  {kind}: |HX - HX_o| / |HX_o| = {d:.2e}", flush=True)
        assert d < 1e-9
    sk.close()


@pytest.mark.parametrize("dtype,terms,pure,block", [("bf16", 1, True, 50), ("f32", 2, False, 70)])
def test_rademacher_generated_in_kernel_matches_staged(monkeypatch, dtype, terms, pure, block):
    """Rademacher test matrices with bf16 operands are generated inside the
    product kernels (never written to device memory); the staged form
    (QSK_STAGE_RADEMACHER=1 at context creation) feeds the same operand
    values in the same order, so both give the same sketches bit for bit,
    on blocks whose first column is not a multiple of 32 (the Omega tile of
    a step then straddles two Philox calls).  The QB stage on the two gives
    the same HX to FP64 rounding."""
    m, n, k, l = 1300, 333, 40, 81
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.85 ** np.arange(20)), 1e-3, 91).numpy()
    if pure:
        a[0] = 0.0
    a = input_values(a, dtype)
    out = []
    for staged in ("1", "0"):
        monkeypatch.setenv("QSK_STAGE_RADEMACHER", staged)
        sk, _ = run_sketch(a, m, n, k, l, block, dtype=dtype, sketch="bf16", emb="rademacher", seed=17,
                           terms=terms, pure=pure)
        out.append([to_numpy(t) for t in sk.sketches()])
        q, x, _ = sk.finalize("pseudo_qr")
        out[-1].append(qt.hamilton(to_numpy(q), to_numpy(x)))
        sk.close()
    np.testing.assert_array_equal(out[0][0], out[1][0])          # Y
    np.testing.assert_array_equal(out[0][1], out[1][1])          # W
    # the QB stage reads Psi from the staging buffer or regenerates it: the
    # same values, FP64 sums in another order
    assert rel(out[1][2], out[0][2]) < 1e-9
    ref = sketch_matrix(a, SketchConfig(m, n, k, l, seed=17, embedding="rademacher", dtype="bf16", terms=terms),
                        block_cols=block)
    check_sketches(out[1][0], out[1][1], ref, a, f"generated rademacher {dtype} x{terms}", block_cols=block)
