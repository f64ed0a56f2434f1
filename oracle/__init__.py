"""Plain, slow CPU FP64 oracle of the one-pass randomized quaternion low-rank
approximation (Chang & Yang, arXiv 2404.14783).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path; the only common dependency is the seeded input generator in ``synth``,
which holds none of the method's arithmetic.

Every function cites the passage of the paper it writes out.  The oracle
follows the paper's steps in the paper's order, using NumPy/LAPACK complex
routines for the steps the paper delegates to "mature libraries" (thin QR,
SVD, the backslash solve), exactly as the paper does (Section 3, opening).

Modules
-------
quaternion   planes, Hamilton product, conjugate transpose, chi / compact /
             real representations, brute-force QSVD via chi (Section 2,
             Appendix B.1)
philox       Philox4x32-10 counter-based generator (Salmon et al., SC'11)
embeddings   quaternion Gaussian (Def. 4.1) and Rademacher (Def. 4.2) test
             matrices drawn from Philox, and their rounding to sketch dtypes
lowprec      exact emulation of the low-precision operand formats (bf16,
             fp8 e4m3 with power-of-two block scales) and the residual split
sketch       Y = A Omega, W = Psi A with column-block linear updates
             (Section 4.1)
rangefinders pseudo-QR with correction steps (Alg. 1, eq. CondNumReductionIter)
             and pseudo-SVD with the good/bad pair repair (Alg. 3)
solve        quaternion linear-equation solver through chi (Alg. 2)
onepass      QB stage (Alg. 4), truncation stage (Alg. 5), relative error

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py``; none is "parity unpinned" except the
sub-Gaussian bound constants of Thm 4.5, which the paper leaves unspecified
and which the oracle does not implement.
"""
