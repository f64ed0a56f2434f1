"""Error behaviour through the C ABI: a sketch from which no Q can be formed
(all zero, or holding a non-finite value) makes qsketch_finalize return
QSK_E_NUMERIC without poisoning the context, and the bounded loops of the QB
stage (bisection, Jacobi sweeps, inverse iteration) end on such input."""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from tests.gpu_helpers import input_values, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_zero_and_nonfinite_sketch(kind):
    m, n, k, l = 300, 200, 12, 25
    sk = qs.Sketcher(m, n, k, l, seed=4, input_dtype="f32", sketch_dtype="bf16", split_terms=2,
                     max_block_cols=100)
    print(f"errors: {kind}, zero sketch", flush=True)
    with pytest.raises(qs.QSketchError) as ei:
        sk.finalize(kind)                                   # nothing streamed yet: Y = 0
    assert ei.value.status == qs.QSK_E_NUMERIC
    y, w = sk.sketches()
    y[1, 5, 3] = float("nan")
    sk.set_sketches(y, w, 0)
    print(f"errors: {kind}, non-finite sketch", flush=True)
    with pytest.raises(qs.QSketchError) as ei:
        sk.finalize(kind)
    assert ei.value.status == qs.QSK_E_NUMERIC
    # the context still works
    sk.reset()
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.7 ** np.arange(6)), 1e-3, 6).numpy()
    dev = to_device(input_values(a, "f32"), "f32")
    for c0 in range(0, n, 100):
        sk.update(c0, dev[:, :, c0:c0 + 100])
    q, x, rep = sk.finalize(kind)
    assert torch.isfinite(q).all() and torch.isfinite(x).all()
    assert sk.rel_error(dev, q, x) < 1e-2
    sk.close()
