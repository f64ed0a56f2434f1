"""One-pass pipeline (Section 4.1): QB stage (Alg. 4), truncation stage
(Alg. 5) and the relative error of Section 5.

QB stage: H <- F(Y) with F a range-preserving rangefinder; X <- (Psi H) \\ W
by Alg. 2 (eq. reconstructionOfTwoSketch).  Only Y, W and Psi are used: A is
never read (Section 4.1).
Truncation: QSVD of X, keep r terms, H <- H U_r.
"""
from __future__ import annotations

import numpy as np

from . import quaternion as qt
from .rangefinders import pseudo_qr, pseudo_svd
from .solve import qsolve


def rangefinder(y, kind, seed=0, n_correction=3, n_power=3):
    if kind == "pseudo_qr":
        return pseudo_qr(y, n_correction=n_correction, n_power=n_power, seed=seed)
    if kind == "pseudo_svd":
        return pseudo_svd(y, seed=seed)
    if kind == "pseudo_svd_gs":
        return pseudo_svd(y, seed=seed, branch="gs")
    raise ValueError(kind)


def qb_stage(sk, kind, n_correction=3, n_power=3):
    """Alg. 4 on a ``sketch.Sketch``: returns (H, X, info)."""
    h, info = rangefinder(sk.Y, kind, seed=sk.cfg.seed, n_correction=n_correction,
                          n_power=n_power)
    p = qt.hamilton(sk.psi(), h)          # Psi H, with the Psi values that formed W
    x = qsolve(p, sk.W)                    # overdetermined: least squares (Alg. 2)
    return h, x, info


def project(h, a):
    """The second pass of the two-pass variant, randomized QSVD (Section 4.1:
    the one-pass algorithm with Psi = I and orthonormal H): X = H^* A, which
    is H^dagger A for orthonormal H."""
    return qt.hamilton(qt.conj_t(h), qt.as_planes(a))


def truncate(h, x, r):
    """Alg. 5: (U, Sigma, V) = QSVD(X); keep r; H <- H U_r.  The QSVD is taken
    through chi (Prop. 2.2); the paper's own QSVD routine is unpublished."""
    u, s, v = qt.qsvd_bruteforce(x)
    return qt.hamilton(h, u[:, :, :r]), s[:r].copy(), v[:, :, :r]


def rel_error(a, h, x, block_cols=4096):
    """||A - H X||_F / ||A||_F (Section 5.1), streamed over column blocks."""
    a = qt.as_planes(a)
    num = 0.0
    den = 0.0
    for c0 in range(0, a.shape[2], block_cols):
        blk = a[:, :, c0:c0 + block_cols]
        d = blk - qt.hamilton(h, x[:, :, c0:c0 + block_cols])
        num += float(np.sum(d * d))
        den += float(np.sum(blk * blk))
    return float(np.sqrt(num / den))


def rel_error_truncated(a, h, s, v):
    """||A - H Sigma V*||_F / ||A||_F."""
    hs = h * s[None, None, :]
    return rel_error(a, hs, qt.conj_t(v))


def optimal_error(a, r):
    """Optimal rank-r relative error sqrt(sum_{i>r} sigma_i^2) / ||A||_F from
    the singular values of chi_A (Thm 2.1, Prop. 2.2)."""
    s = qt.singular_values(a)
    return float(np.sqrt(np.sum(s[r:] ** 2) / np.sum(s ** 2)))
