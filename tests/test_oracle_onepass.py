"""Pins of the oracle's sketching and one-pass pipeline against Section 4:
the definition of the sketches through an independent route (the real
representation), streaming linearity, rangefinder independence of HX
(Lemma 4.2), the QB error identity (Thm 4.1), exact recovery, the RQSVD
special case, the truncation bound (Thm 4.2) and the Gaussian expectation
bound (Thm 4.3).  CPU only."""
import numpy as np
import pytest
import torch

import synth
from oracle import embeddings, onepass, quaternion as qt
from oracle.sketch import Sketch, SketchConfig, sketch_matrix

h = qt.hamilton


def small_lowrank(m, n, r, noise, seed, decay=0.7):
    sig = decay ** np.arange(r)
    return synth.lowrank_plus_noise(m, n, torch.tensor(sig), noise, seed).numpy()


def test_sketch_definition_via_real_representation():
    a = small_lowrank(40, 30, 5, 1e-3, 1)
    cfg = SketchConfig(40, 30, 6, 13, seed=3)
    sk = sketch_matrix(a, cfg, block_cols=7)
    om = embeddings.omega("gaussian", np.arange(30), 6, 3)
    ps = embeddings.psi("gaussian", 13, np.arange(40), 3)
    # Y_r = Upsilon_A Omega_r and W_r = Upsilon_Psi A_r (Appendix B.1)
    np.testing.assert_allclose(qt.compact_real(sk.Y), qt.upsilon(a) @ qt.compact_real(om), atol=1e-11)
    np.testing.assert_allclose(qt.compact_real(sk.W), qt.upsilon(ps) @ qt.compact_real(a), atol=1e-11)


def test_streaming_equals_one_shot_and_linear_updates():
    a = small_lowrank(40, 30, 5, 1e-3, 2)
    cfg = SketchConfig(40, 30, 6, 13, seed=4, embedding="rademacher")
    one = sketch_matrix(a, cfg)
    blk = sketch_matrix(a, cfg, block_cols=4)
    np.testing.assert_allclose(blk.Y, one.Y, atol=1e-12)
    np.testing.assert_allclose(blk.W, one.W, atol=1e-12)
    # A built from two overlapping additive updates gives the same sketches
    s = Sketch(cfg)
    half = 0.5 * a
    s.update(0, half[:, :, :20])
    s.update(10, half[:, :, 10:])
    s.update(0, half[:, :, :10])
    s.update(20, half[:, :, 20:])
    np.testing.assert_allclose(s.Y, one.Y, atol=1e-12)
    np.testing.assert_allclose(s.W, one.W, atol=1e-12)


def test_general_linear_update_reaches_sketch_of_final_matrix():
    """A <- theta A + eta H over a sequence of column blocks (Section 5.3's
    linear updates, theta = 0 included): the streamed sketches equal
    Y = A Omega and W = Psi A of the final matrix, formed here from A through
    the real representation (Appendix B.1)."""
    m, n, k, l = 40, 30, 6, 13
    cfg = SketchConfig(m, n, k, l, seed=5)
    rng = np.random.default_rng(9)
    s = Sketch(cfg)
    a = np.zeros((4, m, n))
    steps = [(1.0, 1.0, 0, 12), (0.5, 2.0, 8, 22), (-1.5, 0.25, 0, 30), (0.0, 0.75, 3, 9),
             (2.0, -3.0, 25, 5), (1.0, 0.0, 0, 4), (0.25, 1.0, 10, 20)]
    for theta, eta, c0, nc in steps:
        hblk = rng.standard_normal((4, m, nc))
        s.update(c0, hblk, theta=theta, eta=eta)
        a = theta * a
        a[:, :, c0:c0 + nc] += eta * hblk
    om = embeddings.omega("gaussian", np.arange(n), k, 5)
    ps = embeddings.psi("gaussian", l, np.arange(m), 5)
    np.testing.assert_allclose(qt.compact_real(s.Y), qt.upsilon(a) @ qt.compact_real(om), atol=1e-11)
    np.testing.assert_allclose(qt.compact_real(s.W), qt.upsilon(ps) @ qt.compact_real(a), atol=1e-11)
    assert s.columns_seen == sum(st[3] for st in steps)


def test_row_and_column_block_updates_reach_the_one_shot_sketch():
    """Sub-block updates over a ragged 2-D partition of A (rows and columns)
    give the sketches of the whole matrix (linearity, Section 5.3)."""
    from oracle.sketch import update_block
    a = small_lowrank(37, 29, 4, 1e-3, 14)
    cfg = SketchConfig(37, 29, 5, 11, seed=8)
    one = sketch_matrix(a, cfg)
    s = Sketch(cfg)
    for r0, r1 in ((0, 10), (10, 11), (11, 37)):
        for c0, c1 in ((0, 13), (13, 29)):
            update_block(s, r0, c0, a[:, r0:r1, c0:c1])
    np.testing.assert_allclose(s.Y, one.Y, atol=1e-12)
    np.testing.assert_allclose(s.W, one.W, atol=1e-12)


def test_update_with_negated_eta_undoes_it():
    cfg = SketchConfig(30, 20, 4, 9, seed=6, embedding="rademacher")
    s = Sketch(cfg)
    base = small_lowrank(30, 20, 3, 1e-3, 3)
    s.update(0, base)
    y0, w0 = s.Y.copy(), s.W.copy()
    hblk = np.random.default_rng(4).standard_normal((4, 30, 7))
    s.update(5, hblk, eta=0.3)
    assert np.linalg.norm(s.W - w0) > 1e-3
    s.update(5, hblk, eta=-0.3)
    np.testing.assert_allclose(s.Y, y0, atol=1e-12)
    np.testing.assert_allclose(s.W, w0, atol=1e-12)


def test_hx_independent_of_rangefinder_lemma42():
    a = small_lowrank(60, 50, 6, 1e-2, 5)
    sk = sketch_matrix(a, SketchConfig(60, 50, 8, 17, seed=1))
    h1, x1, _ = onepass.qb_stage(sk, "pseudo_qr")
    h2, x2, _ = onepass.qb_stage(sk, "pseudo_svd")
    np.testing.assert_allclose(h(h1, x1), h(h2, x2), atol=1e-11)
    # ... and equals Q (Psi Q)^dagger Psi A with Q any orthonormal basis of R(Y)
    q, _, _ = qt.qsvd_bruteforce(sk.Y)
    psi = sk.psi()
    hx = h(q, h(qt.pinv(h(psi, q)), h(psi, a)))
    np.testing.assert_allclose(h(h1, x1), hx, atol=1e-10)


def test_qb_error_identity_thm41():
    m, n, k, l = 30, 24, 5, 11
    a = small_lowrank(m, n, 8, 1e-2, 6, decay=0.6)
    sk = sketch_matrix(a, SketchConfig(m, n, k, l, seed=2))
    hq, x, _ = onepass.qb_stage(sk, "pseudo_svd")
    q = hq                                               # orthonormal
    # orthonormal complement Q_perp by quaternion Gram-Schmidt (right scalars)
    rng = np.random.default_rng(0)
    basis = [q[:, :, j:j + 1] for j in range(k)]
    while len(basis) < m:
        v = rng.standard_normal((4, m, 1))
        for _ in range(2):
            for b in basis:
                v = v - h(b, h(qt.conj_t(b), v))
        basis.append(v / qt.fro(v))
    qperp = np.concatenate(basis[k:], axis=2)
    np.testing.assert_allclose(h(qt.conj_t(qperp), qperp), qt.eye(m - k), atol=1e-10)
    psi = sk.psi()
    psi1, psi2 = h(psi, qperp), h(psi, q)
    lhs = qt.fro(a - h(hq, x)) ** 2
    rhs = qt.fro(a - h(q, h(qt.conj_t(q), a))) ** 2 + \
        qt.fro(h(qt.pinv(psi2), h(psi1, h(qt.conj_t(qperp), a)))) ** 2
    np.testing.assert_allclose(lhs, rhs, rtol=1e-9)


@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_exact_recovery_rank_le_k(kind):
    a = small_lowrank(50, 40, 4, 0.0, 7)
    sk = sketch_matrix(a, SketchConfig(50, 40, 4, 9, seed=5))
    hq, x, _ = onepass.qb_stage(sk, kind)
    assert onepass.rel_error(a, hq, x) < 1e-10


def test_rqsvd_special_case():
    """With Psi = I and orthonormal H, X = H^dagger A (Section 4.1)."""
    a = small_lowrank(20, 16, 3, 1e-3, 8)
    y = h(a, embeddings.omega("gaussian", np.arange(16), 4, 0))
    hq, _ = onepass.rangefinder(y, "pseudo_svd")
    from oracle.solve import qsolve
    x = qsolve(hq, a)                           # (I H) \ (I A)
    np.testing.assert_allclose(x, h(qt.conj_t(hq), a), atol=1e-12)
    np.testing.assert_allclose(onepass.project(hq, a), x, atol=1e-12)


def test_two_pass_projection_is_optimal_in_the_range():
    """H H^* A is the best approximation of A within range(H) (H orthonormal),
    so the two-pass error is at most the one-pass error with the same H."""
    a = small_lowrank(60, 45, 6, 1e-2, 12)
    cfg = SketchConfig(60, 45, 8, 17, seed=13)
    sk = sketch_matrix(a, cfg, block_cols=10)
    hq, x1, _ = onepass.qb_stage(sk, "pseudo_svd")
    x2 = onepass.project(hq, a)
    e1, e2 = onepass.rel_error(a, hq, x1), onepass.rel_error(a, hq, x2)
    assert e2 <= e1 * (1 + 1e-12) and e2 < e1
    # the residual of the projection is orthogonal to range(H)
    res = a - h(hq, x2)
    assert np.abs(h(qt.conj_t(hq), res)).max() < 1e-12 * np.abs(a).max()


def test_truncation_bound_thm42():
    a = small_lowrank(60, 50, 10, 1e-2, 9, decay=0.75)
    sk = sketch_matrix(a, SketchConfig(60, 50, 10, 21, seed=3))
    for kind in ("pseudo_qr", "pseudo_svd"):
        hq, x, info = onepass.qb_stage(sk, kind)
        r = 5
        hu, s, v = onepass.truncate(hq, x, r)
        trunc = h(hu * s[None, None, :], qt.conj_t(v))
        lhs = qt.fro(trunc - h(hq, x))
        sig = qt.singular_values(a)
        tail = np.sqrt(np.sum(sig[r:] ** 2))
        rhs = info["kappa"] * (qt.fro(a - h(hq, x)) + tail)
        assert lhs <= rhs


def test_expected_qb_error_thm43():
    """E||HX - A||_F^2 <= (2l+1)/(2(l-s)+1) (2s+1)/(2(s-r)+1) ||Sigma_2||_F^2."""
    m, n, r, s_, l = 40, 30, 3, 5, 11
    a = small_lowrank(m, n, 12, 0.0, 10, decay=0.5)
    sig = qt.singular_values(a)
    tail2 = np.sum(sig[r:] ** 2)
    errs = []
    for seed in range(24):
        sk = sketch_matrix(a, SketchConfig(m, n, s_, l, seed=100 + seed))
        hq, x, _ = onepass.qb_stage(sk, "pseudo_qr")
        errs.append(qt.fro(a - h(hq, x)) ** 2)
    bound = (2 * l + 1) / (2 * (l - s_) + 1) * (2 * s_ + 1) / (2 * (s_ - r) + 1) * tail2
    assert np.mean(errs) <= bound
    assert min(errs) >= np.sum(sig[s_:] ** 2) * (1 - 1e-9)   # rank s: no better than optimal


def test_config1_error_level():
    """Config 1: k = 40 >= r = 20, noise 1e-6: the QB error is within the
    Thm 4.3 factor (~1.97 in expectation) of the optimal rank-20 error."""
    a = synth.config1().numpy()
    sk = sketch_matrix(a, SketchConfig(1000, 800, 40, 81, seed=0), block_cols=256)
    opt = onepass.optimal_error(a, 20)
    for kind in ("pseudo_qr", "pseudo_svd"):
        hq, x, info = onepass.qb_stage(sk, kind)
        e = onepass.rel_error(a, hq, x)
        assert e < 2.5 * opt
        assert info["kappa"] < 10
