"""Pins of the oracle's rangefinders and solver against what Section 3 of the
paper proves: range equality (Prop. 3.1), the singular-value structure of the
raw pseudo-QR factor (Prop. 3.2), the exact action of one correction step on
the singular values and the condition-number reduction (Prop. 3.3, Cor. 3.1,
Prop. 3.4), the orthonormality of pseudo-SVD (Thm 3.1 and the bad-part
repair), and textbook properties of Alg. 2.  CPU only."""
import numpy as np
import pytest

from oracle import quaternion as qt
from oracle.rangefinders import classify_pairs, pseudo_qr, pseudo_svd
from oracle.solve import qsolve

h = qt.hamilton


def orthonormal_q(m, k, seed):
    rng = np.random.default_rng(seed)
    u, _, _ = qt.qsvd_bruteforce(rng.standard_normal((4, m, k)))
    return u


def sketch_with_condition(m, k, cond, seed, with_basis=False):
    """Y = U diag(logspace(0, -log10 cond)) V* with quaternion-orthonormal U, V."""
    u = orthonormal_q(m, k, seed)
    v = orthonormal_q(k, k, seed + 1)
    s = np.logspace(0, -np.log10(cond), k)
    y = h(u * s[None, None, :], qt.conj_t(v))
    return (y, u) if with_basis else y


def projector(a):
    return h(a, qt.pinv(a))


def test_pseudo_qr_raw_factor_structure():
    y = np.random.default_rng(0).standard_normal((4, 60, 12))
    hq, info = pseudo_qr(y, n_correction=0)
    # compact representation orthonormal (eq. Y_equals_HcR)
    hc = qt.compact(hq)
    np.testing.assert_allclose(hc.conj().T @ hc, np.eye(12), atol=1e-13)
    # Y = H R with R complex upper triangular, real positive diagonal
    r = info["R"]
    assert np.all(np.abs(np.tril(r, -1)) < 1e-14) and np.all(np.diag(r).real > 0)
    rq = qt.from_pair(r, np.zeros_like(r))
    np.testing.assert_allclose(h(hq, rq), y, atol=1e-12)
    # Prop. 3.1: same range
    assert qt.fro(projector(hq) - projector(y)) < 1e-11
    # Prop. 3.2: singular values sqrt(1 +- mu_i), sigma_max <= sqrt(2):
    # the eigenvalues of [[I, T], [T*, I]] pair up as 1 + mu and 1 - mu.
    s = qt.singular_values(hq)
    assert s[0] <= np.sqrt(2) + 1e-12
    np.testing.assert_allclose(s ** 2 + s[::-1] ** 2, 2.0, atol=1e-12)


def test_one_correction_maps_singular_values():
    """H_new = (1 - eps) H + eps (H^dagger)^* maps each singular value
    sigma -> (1 - eps) sigma + eps / sigma with the same singular vectors."""
    y = sketch_with_condition(50, 10, 1e4, 3)
    h0, _ = pseudo_qr(y, n_correction=0)
    h1, info = pseudo_qr(y, n_correction=1)
    eps = info["eps"][0]
    s0 = qt.singular_values(h0)
    want = np.sort((1 - eps) * s0 + eps / s0)[::-1]
    np.testing.assert_allclose(qt.singular_values(h1), want, rtol=1e-8)
    # eps approximates sigma_min(H0) from above within Prop. 3.3's delta range
    assert s0[-1] * (1 - 1e-9) <= eps <= s0[-1] * np.sqrt(7) / 2
    # range preserved
    assert qt.fro(projector(h1) - projector(y)) < 1e-8


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6, 1e7])
def test_three_corrections_reach_kappa_below_10(cond):
    """Prop. 3.4: kappa(H0) < 1e8 gives kappa < 10 after three steps."""
    y = sketch_with_condition(80, 16, cond, 5)
    hq, info = pseudo_qr(y, n_correction=3)
    assert info["kappa0"] < 1e8
    assert info["kappa"] < 10
    assert len(info["eps"]) == 3
    assert qt.fro(projector(hq) - projector(y)) < 1e-6 * max(1.0, cond / 1e4)


def test_correction_reduces_kappa_to_square_root():
    """Prop. 3.3: with eps in [sigma_s, delta sigma_s] and kappa large,
    kappa(H_new) < sqrt(kappa(H))."""
    y = sketch_with_condition(80, 16, 1e6, 9)
    h0, info0 = pseudo_qr(y, n_correction=0)
    h1, info1 = pseudo_qr(y, n_correction=1)
    assert info1["kappa"] < np.sqrt(info0["kappa0"])


@pytest.mark.parametrize("cond", [1e2, 1e6, 1e10, 1e14, 1e20])
def test_pseudo_svd_orthonormal_and_same_range(cond):
    """Orthonormal H with R(H) = R(Y).  With LAPACK's SVD of chi_Y (the paper's
    route) orthogonality degrades roughly like u kappa(Y) up to kappa ~ 1e13,
    where the pair rule starts sending the tiny pairs through the repair."""
    y, u = sketch_with_condition(60, 12, cond, 11, with_basis=True)
    hs, info = pseudo_svd(y, seed=0)
    tol = min(1e-14 * cond, 1e-4) if cond > 1e2 else 1e-13
    np.testing.assert_allclose(h(qt.conj_t(hs), hs), qt.eye(12), atol=tol)
    if cond <= 1e10:
        assert qt.fro(h(hs, qt.conj_t(hs)) - h(u, qt.conj_t(u))) < 1e-14 * cond
        assert info["t_bad"] == 0
    if cond >= 1e14:
        assert info["t_bad"] >= 1


def test_pseudo_svd_singular_vectors_when_distinct():
    """Thm 3.1: with distinct singular values H Sigma V* is a compact QSVD, so
    H* Y Y* H = Sigma^2 is diagonal."""
    y = sketch_with_condition(40, 8, 1e3, 21)
    hs, info = pseudo_svd(y)
    g = h(h(qt.conj_t(hs), y), h(qt.conj_t(y), hs))
    np.testing.assert_allclose(g[0], np.diag(info["sigma"] ** 2), atol=1e-12)
    np.testing.assert_allclose(g[1:], 0, atol=1e-12)


def test_pseudo_svd_identity_counterexample_and_repeated_values():
    """Y = I_2 (the paper's counterexample, Section 3.2) and a Y with a
    repeated singular value: all pairs are bad and the second-SVD repair must
    still give an orthonormal H with the range of Y."""
    y = qt.eye(2)
    hs, info = pseudo_svd(y)
    assert info["t_bad"] == 2
    np.testing.assert_allclose(h(qt.conj_t(hs), hs), qt.eye(2), atol=1e-12)
    u = orthonormal_q(30, 6, 4)
    v = orthonormal_q(6, 6, 5)
    s = np.array([1.0, 0.5, 0.5, 0.25, 0.1, 0.05])
    y = h(u * s[None, None, :], qt.conj_t(v))
    hs, info = pseudo_svd(y)
    assert info["t_bad"] == 2                     # the double value 0.5
    np.testing.assert_allclose(h(qt.conj_t(hs), hs), qt.eye(6), atol=1e-12)
    assert qt.fro(projector(hs) - projector(y)) < 1e-10


@pytest.mark.parametrize("case", ["identity", "repeated", "tiny"])
def test_pseudo_svd_gram_schmidt_branch(case):
    """Alg. 3's Gram-Schmidt branch for the bad part: orthonormal H with the
    range of Y (Thm 3.1 needs the repair for Y = I_2, repeated values and
    values below the pair rule's threshold), the same t as the SVD branch,
    and the same good columns."""
    if case == "identity":
        y = qt.eye(2)
    else:
        u = orthonormal_q(30, 6, 4)
        v = orthonormal_q(6, 6, 5)
        s = (np.array([1.0, 0.5, 0.5, 0.25, 0.1, 0.05]) if case == "repeated"
             else np.array([1.0, 0.5, 0.25, 0.1, 1e-15, 1e-16]))
        y = h(u * s[None, None, :], qt.conj_t(v))
    hs, info = pseudo_svd(y, branch="gs")
    hv, info_v = pseudo_svd(y, branch="svd")
    assert info["t_bad"] == info_v["t_bad"] >= 1
    k = y.shape[2]
    np.testing.assert_allclose(h(qt.conj_t(hs), hs), qt.eye(k), atol=1e-12)
    if case != "tiny":
        # the bad part spans a determined subspace: both branches find it
        assert qt.fro(projector(hs) - projector(y)) < 1e-10
        assert qt.fro(projector(hs) - projector(hv)) < 1e-10
    ng = k - info["t_bad"]
    np.testing.assert_array_equal(hs[:, :, :ng], hv[:, :, :ng])


def test_pair_classification_rule():
    s = np.array([3.0, 3.0, 2.0, 2.0, 2.0, 2.0, 1e-15, 1e-15])
    np.testing.assert_array_equal(classify_pairs(s, 4), [True, False, False, False])


def test_qsolve_square_and_least_squares():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((4, 5, 5))
    b = rng.standard_normal((4, 5, 3))
    x = qsolve(a, b)
    np.testing.assert_allclose(h(a, x), b, atol=1e-11)
    # overdetermined: normal equations A*(A X - B) = 0 and X = A^dagger B
    a = rng.standard_normal((4, 9, 4))
    b = rng.standard_normal((4, 9, 2))
    x = qsolve(a, b)
    np.testing.assert_allclose(h(qt.conj_t(a), h(a, x) - b), 0, atol=1e-11)
    np.testing.assert_allclose(x, h(qt.pinv(a), b), atol=1e-11)
