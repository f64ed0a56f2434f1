"""Pins of the oracle's quaternion algebra against what Section 2 and
Appendix B.1 of the paper fix (identities, homomorphisms, norm relations) and
against brute force.  CPU only."""
import numpy as np
import pytest

from oracle import quaternion as qt

RNG = np.random.default_rng(7)


def rq(m, n):
    return RNG.standard_normal((4, m, n))


def loop_product(a, b):
    """Brute-force matrix product with the scalar unit table."""
    m, p, n = a.shape[1], a.shape[2], b.shape[2]
    c = np.zeros((4, m, n))
    for i in range(m):
        for j in range(n):
            acc = [0.0] * 4
            for t in range(p):
                s = qt.hamilton_scalar(a[:, i, t], b[:, t, j])
                acc = [x + y for x, y in zip(acc, s)]
            c[:, i, j] = acc
    return c


def test_unit_rules():
    one, i, j, k = np.eye(4)
    m = qt.hamilton_scalar
    minus_one = [-1.0, 0, 0, 0]
    assert m(i, i) == minus_one and m(j, j) == minus_one and m(k, k) == minus_one
    assert m(m(i, j), k) == minus_one                     # ijk = -1
    assert m(i, j) == list(k) and m(j, i) == list(-k)     # noncommutative
    assert m(j, k) == list(i) and m(k, i) == list(j)


def test_hamilton_matches_loop_and_representations():
    a, b = rq(5, 4), rq(4, 3)
    c = qt.hamilton(a, b)
    np.testing.assert_allclose(c, loop_product(a, b), rtol=0, atol=1e-13)
    # chi is multiplicative (Prop. 2.1) and Upsilon too (Appendix B.1)
    np.testing.assert_allclose(qt.chi(c), qt.chi(a) @ qt.chi(b), atol=1e-13)
    np.testing.assert_allclose(qt.upsilon(c), qt.upsilon(a) @ qt.upsilon(b), atol=1e-13)
    assert not np.allclose(qt.hamilton(a[:, :3, :3], b[:, :3, :3]),
                           qt.hamilton(b[:, :3, :3], a[:, :3, :3]))


def test_conjugate_transpose_rules():
    p, q = rq(4, 3), rq(4, 2)
    # P* Q = (Q* P)* (Section 2)
    np.testing.assert_allclose(qt.hamilton(qt.conj_t(p), q), qt.conj_t(qt.hamilton(qt.conj_t(q), p)),
                               atol=1e-13)
    np.testing.assert_allclose(qt.chi(qt.conj_t(p)), qt.chi(p).conj().T, atol=0)
    # conj(P* Q) differs from conj(P*) conj(Q) in general
    lhs = qt.conj(qt.hamilton(qt.conj_t(p), q))
    rhs = qt.hamilton(qt.conj(qt.conj_t(p)), qt.conj(q))
    assert not np.allclose(lhs, rhs)


def test_compact_and_j_adjoint():
    q = rq(6, 4)
    qc = qt.compact(q)
    J = qt.symplectic(6)
    # chi_Q = [Q_c, J conj(Q_c)] (Lemma 2.1); J* = J^-1 = -J
    np.testing.assert_allclose(qt.chi(q), np.hstack([qc, J @ np.conj(qc)]), atol=0)
    np.testing.assert_allclose(J.conj().T, -J)
    np.testing.assert_allclose(J.conj().T @ qt.chi(q) @ qt.symplectic(4), np.conj(qt.chi(q)), atol=1e-14)
    v = qc[:, 0]
    assert abs(np.vdot(v, J @ np.conj(v))) < 1e-13
    np.testing.assert_array_equal(qt.from_compact(qc), q)


def test_norm_identities():
    q = rq(5, 7)
    f = qt.fro(q)
    np.testing.assert_allclose(f, np.linalg.norm(qt.upsilon(q)) / 2, rtol=1e-14)
    np.testing.assert_allclose(f, np.linalg.norm(qt.compact_real(q)), rtol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(qt.chi(q)), np.sqrt(2) * f, rtol=1e-14)
    # ||A B||_F = ||Upsilon_A B_r||_F (Appendix B.1)
    a, b = rq(3, 5), rq(5, 2)
    np.testing.assert_allclose(qt.fro(qt.hamilton(a, b)),
                               np.linalg.norm(qt.upsilon(a) @ qt.compact_real(b)), rtol=1e-13)


def test_chi_duplicates_singular_values_and_qsvd():
    a = rq(6, 4)
    s = np.linalg.svd(qt.chi(a), compute_uv=False)
    np.testing.assert_allclose(s[0::2], s[1::2], rtol=1e-12)           # Prop. 2.2
    u, sig, v = qt.qsvd_bruteforce(a)
    recon = qt.hamilton(u * sig[None, None, :], qt.conj_t(v))
    np.testing.assert_allclose(recon, a, atol=1e-12)                    # A = U Sigma V*
    np.testing.assert_allclose(qt.hamilton(qt.conj_t(u), u), qt.eye(4), atol=1e-12)
    # Real data: the quaternion singular values are the real SVD's
    r = np.zeros((4, 5, 3))
    r[0] = RNG.standard_normal((5, 3))
    np.testing.assert_allclose(qt.singular_values(r), np.linalg.svd(r[0], compute_uv=False),
                               rtol=1e-12)


def test_pinv_penrose_equations():
    a = rq(6, 3)
    x = qt.pinv(a)
    h = qt.hamilton
    np.testing.assert_allclose(h(h(a, x), a), a, atol=1e-12)
    np.testing.assert_allclose(h(h(x, a), x), x, atol=1e-12)
    ax = h(a, x)
    xa = h(x, a)
    np.testing.assert_allclose(qt.conj_t(ax), ax, atol=1e-12)
    np.testing.assert_allclose(qt.conj_t(xa), xa, atol=1e-12)


def test_planted_sign_error_is_caught(monkeypatch):
    """A plausible mistake in the Hamilton product (one flipped sign) must
    break the chi homomorphism pin."""
    good = qt.hamilton

    def bad(a, b):
        c = good(a, b)
        aw, ax, ay, az = a
        bw, bx, by, bz = b
        c[3] = aw @ bz + ax @ by + ay @ bx + az @ bw        # sign error on ay bx
        return c
    monkeypatch.setattr(qt, "hamilton", bad)
    a, b = rq(3, 3), rq(3, 2)
    assert not np.allclose(qt.chi(qt.hamilton(a, b)), qt.chi(a) @ qt.chi(b), atol=1e-10)
