"""The paper's two practical quaternion rangefinders (Section 3).

pseudo_qr   Alg. 1: thin complex QR of the compact representation Y_c, the
            map H0 = U(1:m), H1 = -conj U(m+1:2m) (eq. relation_Q_H), then the
            range-preserving correction step
                H <- (1 - eps) H + eps (H^dagger)^*      (eq. CondNumReductionIter)
            a fixed number of times, with H^dagger from Alg. 2 applied to
            chi_{H*H} Z = (H*)_c, and eps from power iterates approximating
            sigma_1(H^dagger) = 1 / sigma_s(H) (Prop. 3.3 and the text after it).
pseudo_svd  Alg. 3: thin complex SVD of chi_Y (eq. USVOfchiY), one left vector
            per duplicated pair for the good part (eq. ComplexUSVToQuaternion),
            and the bad part repaired by H_b diag(f) (eq. sudoSVD_Hbdiagf) and a
            second SVD (eq. sudoSVD_svd_chi_Hb).

Readings where the paper is silent (each listed in the design notes):
  * QR phase: diag(R) is made real and positive, which makes H unique.
  * Correction count: exactly ``n_correction`` steps (default 3, "often 3"),
    no early exit.
  * eps: ``n_power`` (default 3) normalised power steps on chi_{H*H}^{-1} from a
    Philox start vector (stream 2, one per step), then eps = rho^{-1/2} with
    rho the Rayleigh quotient v* chi_{H*H}^{-1} v.
  * Rank deficiency: if lambda_min(chi_{H*H}) <= RANK_TOL * lambda_max, H*H is
    not invertible; the corrections are skipped and the flag is raised.
  * Pair rule of pseudo-SVD: pair i (columns 2i, 2i+1 of the SVD, 0-based) is
    good iff sigma_{2i+1} > TAU_S sigma_0, |sigma_2i - sigma_{2i+1}| <=
    tau_p sigma_0 and both neighbouring pairs are more than tau_p sigma_0 away;
    tau_p = 64 * 2s * u (u = 2^-53).  The bad part always takes the
    second-SVD route.
  * diag(f): f_j = 1 + u_j, u_j from Philox stream 3.
  * Second SVD: one column per pair among the leading 2t columns.
"""
from __future__ import annotations

import numpy as np

from . import embeddings, quaternion as qt
from .solve import qsolve

RANK_TOL = 1e-13
TAU_S = 1e-13
U64 = 2.0 ** -53


def _phase_normalise(u, r):
    d = np.diag(r)
    ad = np.abs(d)
    ph = np.where(ad > 0, d / np.where(ad > 0, ad, 1.0), 1.0)
    return u * ph[None, :], (np.conj(ph)[:, None] * r)


def rank_deficient_gram(g):
    """True when the quaternion Gram H*H is numerically singular."""
    ev = np.linalg.eigvalsh(qt.chi(g))
    return ev[0] <= RANK_TOL * max(ev[-1], 0.0)


def condition_number(h):
    """kappa(H) = sigma_max / sigma_min (Section 3.1, after Remark 3.1)."""
    s = qt.singular_values(h)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")


def epsilon_power(g, step, seed, n_power):
    """eps ~ sigma_s(H) from n_power power iterates on (H*H)^{-1}, in the
    complex representation: v <- chi_G^{-1} v / ||.||; rho = v* chi_G^{-1} v."""
    k = g.shape[1]
    cg = qt.chi(g)
    v = qt.compact(embeddings.power_start(k, step, seed))[:, 0]
    v = v / np.linalg.norm(v)
    for _ in range(n_power):
        v = np.linalg.solve(cg, v)
        v = v / np.linalg.norm(v)
    rho = float(np.real(np.vdot(v, np.linalg.solve(cg, v))))
    return rho ** -0.5


def pseudo_qr(y, n_correction=3, n_power=3, seed=0):
    """Alg. 1.  Returns (H, info) with info = {eps: [...], kappa0, kappa,
    rank_deficient}."""
    y = qt.as_planes(y)
    yc = qt.compact(y)                                  # step 1
    u, r = np.linalg.qr(yc, mode="reduced")             # step 2
    u, r = _phase_normalise(u, r)
    h = qt.from_compact(u)                              # step 3: H0 = U_top, H1 = -conj U_bot
    info = {"eps": [], "kappa0": condition_number(h), "rank_deficient": False, "R": r}
    for step in range(n_correction):                    # step 4
        g = qt.hamilton(qt.conj_t(h), h)
        if rank_deficient_gram(g):
            info["rank_deficient"] = True
            break
        h_dag = qsolve(g, qt.conj_t(h))                 # chi_{H*H} Z = (H*)_c  -> H^dagger
        eps = epsilon_power(g, step, seed, n_power)
        h = (1.0 - eps) * h + eps * qt.conj_t(h_dag)
        info["eps"].append(eps)
    info["kappa"] = condition_number(h)
    return h, info


def classify_pairs(s, k):
    """Good/bad split of the 2k singular values of chi_Y (Alg. 3, step 1)."""
    sig0 = s[0]
    tau_p = 64.0 * 2 * k * U64
    good = []
    for i in range(k):
        a, b = s[2 * i], s[2 * i + 1]
        ok = b > TAU_S * sig0 and abs(a - b) <= tau_p * sig0
        if ok and i > 0:
            ok = (s[2 * i - 1] - a) > tau_p * sig0
        if ok and i < k - 1:
            ok = (b - s[2 * i + 2]) > tau_p * sig0
        good.append(bool(ok))
    return np.array(good, dtype=bool)


# Gram-Schmidt branch of Alg. 3: a candidate column of U_b counts as
# linearly independent of the columns taken so far (and their J-partners)
# when its residual after two projections keeps more than GS_TOL of its norm.
GS_TOL = 1e-8


def _j_conj(x):
    """J conj(x) for a 2m-vector x (the J-partner of a compact column)."""
    m = x.shape[0] // 2
    return np.concatenate([-np.conj(x[m:]), np.conj(x[:m])])


def pseudo_svd(y, seed=0, branch="svd"):
    """Alg. 3.  Returns (H, info) with info = {t_bad, sigma, kappa}.
    branch: 'svd' repairs the bad part through H_b diag(f) and a second SVD;
    'gs' takes the Gram-Schmidt branch: the columns of U_b in turn, each
    orthogonalised against the columns already taken and their J-partners,
    kept when linearly independent, until t are taken."""
    y = qt.as_planes(y)
    k = y.shape[2]
    u, s, _ = np.linalg.svd(qt.chi(y), full_matrices=False)     # step 1
    good = classify_pairs(s, k)
    gi = np.nonzero(good)[0]
    bi = np.nonzero(~good)[0]
    cols = [qt.from_compact(u[:, 2 * gi])]                        # step 2: H_g
    t = len(bi)
    if t:
        ub = u[:, np.concatenate([2 * bi, 2 * bi + 1])]            # U_b, 2m x 2t
        if branch == "svd":
            hb = qt.from_compact(ub)                               # (H_b)_c = U_b
            hb = hb * embeddings.diag_f(2 * t, seed)[None, None, :]  # H_b diag(f)
            uh, _, _ = np.linalg.svd(qt.chi(hb), full_matrices=False)  # SVD of chi_{H_b}
            cols.append(qt.from_compact(uh[:, 0:2 * t:2]))         # H_b~ from U_h1
        elif branch == "gs":
            basis = np.zeros((ub.shape[0], 0), dtype=np.complex128)
            taken = []
            for c in range(ub.shape[1]):                           # U_b's columns in turn
                x = ub[:, c].copy()
                nx0 = np.linalg.norm(x)
                for _ in range(2):
                    x = x - basis @ (basis.conj().T @ x)
                nx = np.linalg.norm(x)
                if nx > GS_TOL * nx0:
                    x = x / nx
                    taken.append(x)
                    basis = np.column_stack([basis, x, _j_conj(x)])
                if len(taken) == t:
                    break
            cols.append(qt.from_compact(np.stack(taken, axis=1)))
        else:
            raise ValueError(branch)
    h = np.concatenate(cols, axis=2)                               # H = [H_g, H_b~]
    info = {"t_bad": int(t), "sigma": s[0::2].copy(), "kappa": condition_number(h)}
    return h, info
