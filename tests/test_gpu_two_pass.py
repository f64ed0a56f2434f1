"""The two-pass variant, randomized QSVD (Section 4.1: the one-pass algorithm
with Psi = I and an orthonormal H gives X = H^dagger A = H^* A): a y_only
context streams Y alone, the rangefinder runs without a core solve, and
qsketch_project forms X = Q^* A in a second pass over A.

Tolerances: the projection multiplies the given FP64 Q with the exact input
values in FP64 on the matrix cores, so it matches the oracle's FP64 product
to 1e-12 relative; the end-to-end error matches the oracle's two-pass error
to the equal-error criterion 1e-3 relative (BF16 sketch operands, FP32 Y).
"""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle import onepass, quaternion as qt
from oracle.sketch import SketchConfig, sketch_matrix
from tests.gpu_helpers import input_values, rel, to_device, to_numpy

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,pure,m", [("f64", False, 333), ("f32", False, 333), ("bf16", False, 333),
                                          ("f32", True, 333), ("bf16", True, 333),
                                          ("f64", False, 3001), ("bf16", True, 3001)])
def test_project_parity(dtype, pure, m):
    """X[:, J] = Q^* A_J for a seeded Q (not from the device) over uneven
    blocks with ragged tails (m, k and every block width off the 16 grid);
    m = 3001 splits the contraction over row chunks."""
    n, k, l = 257, 21, 43
    print(f"project: {dtype} pure={pure} m={m}", flush=True)
    rng = np.random.default_rng(41)
    q = rng.standard_normal((4, m, k))
    a = input_values(rng.standard_normal((4, m, n)), dtype)
    if pure:
        a[0] = 0.0
    sk = qs.Sketcher(m, n, k, l, input_dtype=dtype, sketch_dtype="f64" if dtype == "f64" else "f32",
                     pure=pure, max_block_cols=100)
    dev = to_device(a, dtype, pure=pure)
    qd = to_device(q, "f64")
    x = None
    for c0, nc in ((0, 100), (100, 37), (137, 1), (138, 100), (238, 19)):
        x = sk.project(c0, dev[:, :, c0:c0 + nc], qd, x)
    torch.cuda.synchronize()
    ref = onepass.project(q, a)
    e = rel(to_numpy(x), ref)
    print(f"  rel. diff X {e:.2e}", flush=True)
    assert e < 1e-12
    sk.close()


def test_two_pass_end_to_end():
    m, n, k, l, block = 1200, 700, 24, 49, 128
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(16)), 1e-4, 51).numpy()
    a = input_values(a, "f32")
    dev = to_device(a, "f32")
    kw = dict(seed=3, input_dtype="f32", sketch_dtype="bf16", split_terms=2, max_block_cols=block)
    two = qs.Sketcher(m, n, k, l, y_only=True, **kw)
    one = qs.Sketcher(m, n, k, l, **kw)
    for c0 in range(0, n, block):
        two.update(c0, dev[:, :, c0:c0 + block])
        one.update(c0, dev[:, :, c0:c0 + block])
    y2, w2 = two.sketches()
    y1, _ = one.sketches()
    assert w2 is None
    np.testing.assert_array_equal(to_numpy(y2), to_numpy(y1))   # the same Y kernel launches
    with pytest.raises(qs.QSketchError):
        two.finalize("pseudo_svd", solve=True)                    # no W to solve against
    q, x, rep = two.finalize("pseudo_svd")
    assert x is None and rep["orth_defect"] < 1e-10
    xp = None
    for c0 in range(0, n, block):
        xp = two.project(c0, dev[:, :, c0:c0 + block], q, xp)
    e_two = two.rel_error(dev, q, xp)
    q1, x1, _ = one.finalize("pseudo_svd")
    e_one = one.rel_error(dev, q1, x1)
    # oracle: the same BF16 operand values, FP64 arithmetic
    cfg = SketchConfig(m, n, k, l, seed=3, dtype="bf16", terms=2)
    sk = sketch_matrix(a, cfg, block_cols=block)
    hq, _ = onepass.rangefinder(sk.Y, "pseudo_svd", seed=3)
    e_ref = onepass.rel_error(a, hq, onepass.project(hq, a))
    print(f"two-pass error {e_two:.6e} (oracle {e_ref:.6e}), one-pass {e_one:.6e}", flush=True)
    assert abs(e_two - e_ref) <= 1e-3 * e_ref
    assert e_two <= e_one * (1 + 1e-9)
    two.close()
    one.close()
