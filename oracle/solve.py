"""Quaternion linear-equation solver through the complex representation
(Alg. 2, Section 3.1).

For A in Q^{n1 x n2} and B in Q^{n1 x l}: build chi_A (2 n1 x 2 n2) and
B_c (2 n1 x l), solve chi_A Z = B_c, and return X = Z(1:n2) - conj(Z(n2+1:2n2)) j.
The paper's argument (Section 3.1) shows that Z is then the compact
representation of a solution of A X = B, because chi_A J conj(Z) =
J conj(chi_A Z) (Lemma 2.1).

"Solve" is MATLAB's backslash in the paper: LU for a square system, least
squares for an overdetermined one.  Where the paper is silent on rank
deficiency (Alg. 2 types X as complex and never discusses it), the oracle takes
the minimum-norm least-squares solution, which through Lemma 2.2 is
X = A^dagger B.
"""
from __future__ import annotations

import numpy as np

from . import quaternion as qt


def qsolve(a, b):
    """Alg. 2: X with A X = B (square, nonsingular) or X = argmin ||A X - B||_F
    of minimum norm (rectangular or singular)."""
    a = qt.as_planes(a)
    b = qt.as_planes(b)
    ca = qt.chi(a)
    bc = qt.compact(b)
    square = a.shape[1] == a.shape[2]
    z = None
    if square:
        try:
            z = np.linalg.solve(ca, bc)
        except np.linalg.LinAlgError:
            z = None
    if z is None:
        z, *_ = np.linalg.lstsq(ca, bc, rcond=None)
    return qt.from_compact(z)
