"""Quaternion matrices as four real planes, and their representations.

A quaternion matrix Q = Q_w + Q_x i + Q_y j + Q_z k (Section 2) is held as a
float64 array of shape (4, m, n) with planes (w, x, y, z).

Paper passages written out here:
  * Hamilton product rules i^2 = j^2 = k^2 = ijk = -1 (Section 2);
  * conjugate transpose Q* and ||Q||_F over the four planes (Section 2);
  * Q = Q0 + Q1 j with Q0 = Q_w + Q_x i, Q1 = Q_y + Q_z i, the full complex
    representation chi_Q = [[Q0, Q1], [-conj Q1, conj Q0]] (Section 2.2,
    Prop. 2.1) and the compact representation Q_c = [Q0; -conj Q1]
    (Section 2.2, Lemma 2.1);
  * the inverse map of Alg. 2: X = Z(1:n) - conj(Z(n+1:2n)) j;
  * the real representation Upsilon_Q (Appendix B.1);
  * the QSVD through chi: chi's singular values are those of Q, each twice
    (Thm 2.1, Prop. 2.2).
"""
from __future__ import annotations

import numpy as np


def zeros(m, n):
    return np.zeros((4, m, n), dtype=np.float64)


def eye(n):
    q = zeros(n, n)
    q[0] = np.eye(n)
    return q


def as_planes(a):
    a = np.asarray(a, dtype=np.float64)
    if a.ndim != 3 or a.shape[0] != 4:
        raise ValueError("quaternion matrix must have shape (4, m, n)")
    return a


def hamilton(a, b):
    """Quaternion matrix product C = A B from the multiplication rules of
    Section 2 (ij = k = -ji, jk = i = -kj, ki = j = -ik, i^2=j^2=k^2=-1).

    Written as the sixteen real products of the components, one plane pair
    at a time; no representation is used, so this is the first of three
    independent routes the tests compare.
    """
    aw, ax, ay, az = as_planes(a)
    bw, bx, by, bz = as_planes(b)
    cw = aw @ bw - ax @ bx - ay @ by - az @ bz
    cx = aw @ bx + ax @ bw + ay @ bz - az @ by
    cy = aw @ by - ax @ bz + ay @ bw + az @ bx
    cz = aw @ bz + ax @ by - ay @ bx + az @ bw
    return np.stack([cw, cx, cy, cz])


def hamilton_scalar(p, q):
    """Product of two single quaternions given as length-4 sequences, by
    expanding (p_w + p_x i + p_y j + p_z k)(q_w + ...) term by term with an
    explicit unit-multiplication table.  Used only to pin ``hamilton``."""
    # unit products e_a e_b = sign * e_c, units ordered (1, i, j, k)
    table = {
        (0, 0): (1, 0), (0, 1): (1, 1), (0, 2): (1, 2), (0, 3): (1, 3),
        (1, 0): (1, 1), (1, 1): (-1, 0), (1, 2): (1, 3), (1, 3): (-1, 2),
        (2, 0): (1, 2), (2, 1): (-1, 3), (2, 2): (-1, 0), (2, 3): (1, 1),
        (3, 0): (1, 3), (3, 1): (1, 2), (3, 2): (-1, 1), (3, 3): (-1, 0),
    }
    out = [0.0, 0.0, 0.0, 0.0]
    for a in range(4):
        for b in range(4):
            s, c = table[(a, b)]
            out[c] += s * p[a] * q[b]
    return out


def conj(a):
    """Entry-wise conjugate  conj(Q) = Q_w - Q_x i - Q_y j - Q_z k."""
    a = as_planes(a)
    return np.stack([a[0], -a[1], -a[2], -a[3]])


def conj_t(a):
    """Conjugate transpose Q* = Q_w^T - Q_x^T i - Q_y^T j - Q_z^T k."""
    a = as_planes(a)
    return np.stack([a[0].T, -a[1].T, -a[2].T, -a[3].T])


def fro(a):
    """||Q||_F = (sum over the four planes of ||Q_p||_F^2)^(1/2)."""
    a = as_planes(a)
    return float(np.sqrt(np.sum(a * a)))


def complex_pair(a):
    """Q = Q0 + Q1 j with Q0 = Q_w + Q_x i and Q1 = Q_y + Q_z i."""
    a = as_planes(a)
    return a[0] + 1j * a[1], a[2] + 1j * a[3]


def from_pair(q0, q1):
    return np.stack([q0.real, q0.imag, q1.real, q1.imag]).astype(np.float64)


def chi(a):
    """Full complex representation chi_Q in C^{2m x 2n} (Section 2.2)."""
    q0, q1 = complex_pair(a)
    return np.block([[q0, q1], [-np.conj(q1), np.conj(q0)]])


def compact(a):
    """Compact complex representation Q_c = [Q0; -conj(Q1)] in C^{2m x n}."""
    q0, q1 = complex_pair(a)
    return np.vstack([q0, -np.conj(q1)])


def from_compact(z):
    """Inverse of ``compact`` as in Alg. 2, step 3:
    X = Z(1:n, :) - conj(Z(n+1:2n, :)) j, i.e. X0 = Z_top, X1 = -conj(Z_bot).
    """
    z = np.asarray(z)
    if z.shape[0] % 2:
        raise ValueError("compact representation needs an even row count")
    n = z.shape[0] // 2
    return from_pair(z[:n], -np.conj(z[n:]))


def symplectic(m):
    """J = [[0, -I_m], [I_m, 0]] (Section 2.2)."""
    j = np.zeros((2 * m, 2 * m), dtype=np.complex128)
    j[:m, m:] = -np.eye(m)
    j[m:, :m] = np.eye(m)
    return j


def upsilon(a):
    """Real representation Upsilon_Q in R^{4m x 4n} (Appendix B.1)."""
    w, x, y, z = as_planes(a)
    return np.block([
        [w, -x, -y, -z],
        [x, w, -z, y],
        [y, z, w, -x],
        [z, -y, x, w],
    ])


def compact_real(a):
    """Q_r = [Q_w; Q_x; Q_y; Q_z], the first block column of Upsilon_Q."""
    a = as_planes(a)
    return np.vstack([a[0], a[1], a[2], a[3]])


def from_compact_real(r):
    r = np.asarray(r, dtype=np.float64)
    m = r.shape[0] // 4
    return np.stack([r[:m], r[m:2 * m], r[2 * m:3 * m], r[3 * m:]])


def singular_values(a):
    """Singular values of a quaternion matrix: the SVD of chi_Q returns each
    of them twice (Prop. 2.2); keep one of each adjacent pair."""
    s = np.linalg.svd(chi(a), compute_uv=False)
    return s[0::2].copy()


def qsvd_bruteforce(a):
    """Compact QSVD A = U Sigma V* through chi (Thm 2.1, Prop. 2.2), for
    tiny test inputs whose singular values are distinct.

    Takes one left/right singular vector per duplicated pair of chi_A's SVD
    (columns 1, 3, 5, ... in 1-based numbering) and maps it back with the
    compact-representation inverse.  Returns (U, sigma, V) with U, V
    quaternion and sigma real, descending.
    """
    u, s, vh = np.linalg.svd(chi(a), full_matrices=False)
    v = vh.conj().T
    r = min(a.shape[1], a.shape[2])
    uq = from_compact(u[:, 0:2 * r:2])
    vq = from_compact(v[:, 0:2 * r:2])
    return uq, s[0:2 * r:2].copy(), vq


def pinv(a):
    """Quaternion Moore-Penrose inverse through chi_{A^dagger} = (chi_A)^dagger
    (Lemma 2.2): the compact representation of A^dagger is the first block
    column of pinv(chi_A)."""
    a = as_planes(a)
    n = a.shape[2]
    p = np.linalg.pinv(chi(a))
    return from_pair(p[:n, :a.shape[1]], p[:n, a.shape[1]:])


def random_gaussian(rng, m, n, scale=1.0):
    """Quaternion standard Gaussian matrix (Def. 4.1) from a NumPy generator;
    used by oracle self-tests only (the sketches draw from Philox)."""
    return scale * rng.standard_normal((4, m, n))
