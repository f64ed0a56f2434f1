"""Random quaternion test matrices Omega (n x s) and Psi (l x m) (Section 4.1),
drawn from Philox4x32-10 so that any entry can be regenerated from its
indices.

Distributions:
  * quaternion standard Gaussian: all four components i.i.d. N(0, 1)
    (Def. 4.1);
  * quaternion Rademacher: all four components i.i.d. +-1 with probability
    1/2, a centred, unit-variance sub-Gaussian matrix (Def. 4.2, which names
    Rademacher among the common sub-Gaussian variables).

Counter layout (the paper's MATLAB code draws with an unnamed generator; this
is the layout both sides of this project implement).  An entry is addressed
by its contraction index t (a row of Omega = a column of A; a column of Psi =
a row of A) and its other index o (a column of Omega, a row of Psi), and a
stream id: 0 = Omega, 1 = Psi, 2 = power-iteration start vectors,
3 = the diag(f) factors of pseudo-SVD.  Key = (seed mod 2^32, seed >> 32).

  Gaussian entry:   counter (t, o, stream, 0) -> words x0..x3;
                    u_i = (x_i + 1/2) 2^-32 in (0, 1);
                    w = sqrt(-2 ln u0) cos(2 pi u1), x = sqrt(-2 ln u0) sin(2 pi u1),
                    y = sqrt(-2 ln u2) cos(2 pi u3), z = sqrt(-2 ln u2) sin(2 pi u3)
                    (Box and Muller, 1958), evaluated in FP64.
  Rademacher entry: counter (t >> 5, o, stream, 1) -> 128 bits; with
                    b = t & 31, word x_(b >> 3) supplies bits 4(b & 7) .. +3,
                    one per component (w, x, y, z); bit 0 -> +1, bit 1 -> -1.
                    One Philox call thus serves 32 consecutive t.

For a low-precision sketch the drawn values are rounded once, from the FP64
value, to the operand format (``lowprec.round_dtype``).  A rounded Gaussian
is still an entry-independent sub-Gaussian test matrix in the sense of
Def. 4.2; the core solve must use exactly these rounded values of Psi.
"""
from __future__ import annotations

import numpy as np

from . import lowprec
from .philox import philox4x32, seed_key

STREAM_OMEGA = 0
STREAM_PSI = 1
STREAM_POWER = 2
STREAM_DIAGF = 3

_TWO_M32 = 2.0 ** -32


def _uniform(words):
    return (words.astype(np.float64) + 0.5) * _TWO_M32


def gaussian_entries(t, o, stream, seed):
    """Quaternion Gaussian entries at index arrays (t, o); returns (4, *shape)."""
    k0, k1 = seed_key(seed)
    t, o = np.broadcast_arrays(np.asarray(t, np.uint64), np.asarray(o, np.uint64))
    x0, x1, x2, x3 = philox4x32(t, o, np.uint64(stream), np.uint64(0), k0, k1)
    u0, u1, u2, u3 = _uniform(x0), _uniform(x1), _uniform(x2), _uniform(x3)
    ra = np.sqrt(-2.0 * np.log(u0))
    rb = np.sqrt(-2.0 * np.log(u2))
    return np.stack([ra * np.cos(2.0 * np.pi * u1), ra * np.sin(2.0 * np.pi * u1),
                     rb * np.cos(2.0 * np.pi * u3), rb * np.sin(2.0 * np.pi * u3)])


def rademacher_entries(t, o, stream, seed):
    """Quaternion Rademacher entries at index arrays (t, o); returns (4, *shape)."""
    k0, k1 = seed_key(seed)
    t, o = np.broadcast_arrays(np.asarray(t, np.uint64), np.asarray(o, np.uint64))
    x = philox4x32(t >> np.uint64(5), o, np.uint64(stream), np.uint64(1), k0, k1)
    b = t & np.uint64(31)
    word = b >> np.uint64(3)
    sel = np.where(word == 0, x[0], np.where(word == 1, x[1], np.where(word == 2, x[2], x[3])))
    shift = np.uint64(4) * (b & np.uint64(7))
    nib = (sel >> shift) & np.uint64(0xF)
    comps = [((nib >> np.uint64(p)) & np.uint64(1)).astype(np.float64) for p in range(4)]
    return np.stack([1.0 - 2.0 * c for c in comps])


def entries(kind, t, o, stream, seed):
    if kind == "gaussian":
        return gaussian_entries(t, o, stream, seed)
    if kind == "rademacher":
        return rademacher_entries(t, o, stream, seed)
    raise ValueError(kind)


def omega(kind, rows, k, seed, dtype="f64"):
    """Rows ``rows`` (an index array into 0..n-1) of Omega in Q^{n x k},
    rounded to ``dtype``.  Returns shape (4, len(rows), k)."""
    rows = np.asarray(rows, dtype=np.uint64)
    t = rows[:, None]
    o = np.arange(k, dtype=np.uint64)[None, :]
    return lowprec.round_dtype(entries(kind, t, o, STREAM_OMEGA, seed), dtype)


def psi(kind, l, cols, seed, dtype="f64"):
    """Columns ``cols`` (an index array into 0..m-1) of Psi in Q^{l x m},
    rounded to ``dtype``.  Returns shape (4, l, len(cols))."""
    cols = np.asarray(cols, dtype=np.uint64)
    t = cols[None, :]
    o = np.arange(l, dtype=np.uint64)[:, None]
    return lowprec.round_dtype(entries(kind, t, o, STREAM_PSI, seed), dtype)


def power_start(k, step, seed):
    """Start vector (k x 1 quaternion Gaussian) of the power iteration used to
    estimate epsilon in correction step ``step``."""
    t = np.arange(k, dtype=np.uint64)[:, None]
    return gaussian_entries(t, np.uint64(step), STREAM_POWER, seed)


def diag_f(count, seed):
    """f_j = 1 + u_j with u_j ~ Uniform(0, 1), j = 0..count-1 (the diag(f)
    factors of pseudo-SVD's bad-part repair, eq. sudoSVD_Hbdiagf)."""
    k0, k1 = seed_key(seed)
    j = np.arange(count, dtype=np.uint64)
    x0, _, _, _ = philox4x32(j, np.uint64(0), np.uint64(STREAM_DIAGF), np.uint64(0), k0, k1)
    return 1.0 + _uniform(x0)
