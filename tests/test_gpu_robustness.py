"""Rangefinder robustness over the condition number of the sketch (Section
3.3's comparison: Y of 1000 x 200 with kappa(Y) from 1e6 to 1e22), FP64 on
the GPU: the sketch is loaded with qsketch_set_sketches and each rangefinder
runs alone (qsketch_finalize with X = NULL).

Y = U diag(sigma) V^* with U, V orthonormal (the oracle's pseudo-SVD of
seeded Gaussian matrices) and sigma_i = kappa^(-i/(k-1)).  Checked against
what the paper and the mathematics fix, for the device and the oracle alike:
  * pseudo-SVD returns orthonormal columns for every kappa (Section 3.3);
  * pseudo-SVD contains the numerically determined part of range(Y): the
    leading singular directions with sigma_i >= 1e-6 sigma_1 are captured
    to 1e-8 (||U_lead - H H^dagger U_lead||_F);
  * pseudo-QR, in the regime the paper gives it (kappa(Y) below 1e8; with
    this construction the raw factor's Gram stays numerically nonsingular
    up to about kappa(Y) = 1e7), reaches kappa(H) < 10 after three
    corrections (Prop. 3.4) and captures the leading directions to 1e-4 in
    the oracle; the device, whose first factor is a CholeskyQR2, must do no
    worse than 10x the oracle (or 1e-8);
  * outside that regime pseudo-QR's output is only required to be finite;
  * the number of repaired pseudo-SVD pairs matches the oracle's within one
    (a singular value on the pair rule's threshold may fall either way);
  * the same holds with the bad part repaired by Alg. 3's Gram-Schmidt
    branch (pseudo_svd_gs), and where the bad part spans a determined
    subspace (a repeated singular value) both branches return its range.
"""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
from oracle import quaternion as qt
from oracle.rangefinders import condition_number, pseudo_qr, pseudo_svd
from tests.gpu_helpers import to_device, to_numpy

pytestmark = pytest.mark.gpu

M, K = 1000, 200


@pytest.fixture(scope="module")
def factors():
    rng = np.random.default_rng(2024)
    u, _ = pseudo_svd(qt.random_gaussian(rng, M, K))
    v, _ = pseudo_svd(qt.random_gaussian(rng, K, K))
    return u, v


def capture_error(h, u_lead):
    """||U_lead - H H^dagger U_lead||_F (H of full column rank)."""
    c = qt.hamilton(qt.pinv(h), u_lead)
    return float(np.linalg.norm((u_lead - qt.hamilton(h, c)).ravel()))


@pytest.mark.parametrize("kappa", [1e6, 1e7, 1e8, 1e10, 1e14, 1e18, 1e22])
def test_rangefinders_over_kappa(factors, kappa):
    u, v = factors
    sig = kappa ** (-np.arange(K) / (K - 1))
    y = qt.hamilton(u * sig[None, None, :], qt.conj_t(v))
    lead = int(np.sum(sig >= 1e-6))
    u_lead = u[:, :, :lead]
    sk = qs.Sketcher(M, K, K, K)
    sk.set_sketches(to_device(y, "f64"), None, K)
    print(f"kappa(Y) = {kappa:.0e}", flush=True)
    for kind in ("pseudo_svd", "pseudo_svd_gs", "pseudo_qr"):
        q, x, rep = sk.finalize(kind, solve=False)
        assert x is None
        h = to_numpy(q)
        assert np.isfinite(h).all()
        if kind.startswith("pseudo_svd"):
            h_ref, info = pseudo_svd(y, branch="gs" if kind.endswith("gs") else "svd")
            e_dev, e_ref = capture_error(h, u_lead), capture_error(h_ref, u_lead)
            print(f"  {kind}: orth {rep['orth_defect']:.1e}, t_bad {rep['t_bad']} "
                  f"(oracle {info['t_bad']}), capture {e_dev:.1e} (oracle {e_ref:.1e})", flush=True)
            assert rep["orth_defect"] < 1e-10
            assert rep["t_bad"] == info["t_bad"]
            assert e_dev < 1e-8 and e_ref < 1e-8
        else:
            h_ref, info = pseudo_qr(y)
            kap_ref = condition_number(h_ref)
            print(f"  pseudo-QR: kappa {rep['kappa']:.3f} (oracle {kap_ref:.3f}), flags {rep['flags']}",
                  flush=True)
            if kappa <= 1e7:
                e_dev, e_ref = capture_error(h, u_lead), capture_error(h_ref, u_lead)
                print(f"    capture {e_dev:.1e} (oracle {e_ref:.1e})", flush=True)
                assert rep["kappa"] < 10.0 and kap_ref < 10.0
                assert e_ref < 1e-4 and e_dev <= max(10.0 * e_ref, 1e-8)
    sk.close()


def projector(h):
    return qt.hamilton(h, qt.pinv(h))


@pytest.mark.parametrize("kind", ["pseudo_svd", "pseudo_svd_gs"])
def test_repeated_singular_value_repair(factors, kind):
    """A repeated singular value makes its pairs bad (the pair rule needs a
    gap); the repaired H must still span range(Y) exactly, like the oracle's
    branch of the same name."""
    u, v = factors
    sig = 0.98 ** np.arange(K)                # kappa(Y) ~ 60: range determined to rounding
    sig[10:14] = sig[10]                      # a fourfold value
    y = qt.hamilton(u * sig[None, None, :], qt.conj_t(v))
    sk = qs.Sketcher(M, K, K, K)
    sk.set_sketches(to_device(y, "f64"), None, K)
    q, _, rep = sk.finalize(kind, solve=False)
    h = to_numpy(q)
    h_ref, info = pseudo_svd(y, branch="gs" if kind.endswith("gs") else "svd")
    print(f"{kind}: t_bad {rep['t_bad']} (oracle {info['t_bad']}), orth {rep['orth_defect']:.1e}", flush=True)
    assert rep["t_bad"] == info["t_bad"] >= 4
    assert rep["orth_defect"] < 1e-10
    # full rank k = 200 in a 1000-dim space: compare ranges through the
    # projectors onto range(Y) = range(U)
    pu = qt.hamilton(u, qt.conj_t(u))
    e_dev, e_ref = qt.fro(projector(h) - pu), qt.fro(projector(h_ref) - pu)
    print(f"  range: ||P_H - P_Y||_F {e_dev:.1e} (oracle {e_ref:.1e})", flush=True)
    assert e_dev < 1e-10 and e_ref < 1e-10
    sk.close()
