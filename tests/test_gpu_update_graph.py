"""qsketch_update_many: a stream of linear updates A += H (Section 4,
opening; Section 5.3) captured once into a HIP graph and replayed.  Every
replay must give the sketches of the same updates issued one by one, bit for
bit (the graph holds the same kernels with the same arguments), with eager
work of the context between the replays (reset, sketch copies, a finalize),
after the blocks' contents change in place, and after new block tensors
force a new capture; also with update coalescing, where the capture records
the pending-column state the replays continue from.
"""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle.sketch import Sketch, SketchConfig
from tests.gpu_helpers import BoundTracker, input_values, to_device, to_numpy

pytestmark = pytest.mark.gpu


def blocks_of(dev, n, block):
    return [dev[:, :, c0:c0 + block] for c0 in range(0, n, block)], list(range(0, n, block))


@pytest.mark.parametrize("sketch,terms,pure,coalesce", [("bf16", 2, False, 0), ("fp8", 2, True, 0),
                                                        ("bf16", 2, False, 64), ("f32", 1, False, 0),
                                                        ("fp8x", 3, True, 0), ("fp8x", 3, False, 128)])
def test_update_graph_replays_match_single_updates(sketch, terms, pure, coalesce):
    m, n, k, l, block = 3000, 300, 24, 49, 10
    print(f"update graph: {sketch} x{terms} pure={pure} coalesce={coalesce}", flush=True)
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(12)), 1e-3, 701).numpy()
    if pure:
        a[0] = 0.0
    a = input_values(a, "f32")
    dev = to_device(a, "f32", pure=pure)
    kw = dict(seed=5, input_dtype="f32", sketch_dtype=sketch, split_terms=terms, pure=pure,
              max_block_cols=block, coalesce_cols=coalesce)
    one = qs.Sketcher(m, n, k, l, **kw)
    gr = qs.Sketcher(m, n, k, l, **kw)
    blocks, cols = blocks_of(dev, n, block)

    def eager():
        one.reset()
        for c0, b in zip(cols, blocks):
            one.update(c0, b)
        return [to_numpy(t) for t in one.sketches()]

    for rep in range(3):
        if rep == 2:
            dev.mul_(-0.5)                     # new contents, same addresses: a replay
        ref = eager()
        gr.reset()
        gr.update_many(cols, blocks)
        assert gr.columns_seen == n
        got = [to_numpy(t) for t in gr.sketches()]
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
        gr.finalize("pseudo_qr")                # eager work between the replays

    # other tensors (a copy): captured again
    dev2 = dev.clone()
    blocks2, _ = blocks_of(dev2, n, block)
    gr.reset()
    gr.update_many(cols, blocks2)
    np.testing.assert_array_equal(to_numpy(gr.sketches()[0]), eager()[0])
    # and the oracle agrees with the graph's sketches (the data of the last pass)
    ah = dev.double().cpu().numpy()
    if pure:
        ah = np.concatenate([np.zeros_like(ah[:1]), ah], axis=0)
    cfg = (SketchConfig(m, n, k, l, seed=5, dtype="fp8", fp8_block=32, fp8_residual=True) if sketch == "fp8"
           else SketchConfig(m, n, k, l, seed=5, dtype=sketch, terms=terms))
    ref = Sketch(cfg)
    bt = BoundTracker(ref)
    eff = (coalesce // block) * block if coalesce else block
    for c0 in range(0, n, eff):
        ref.update(c0, ah[:, :, c0:c0 + eff])
        bt.update(c0, ah[:, :, c0:c0 + eff])
    y, w = (to_numpy(t) for t in gr.sketches())
    bt.check(y, w, f"update graph {sketch}")
    one.close()
    gr.close()


def test_update_many_rejects_bad_block_before_running():
    m, n, k, l = 500, 100, 8, 17
    a = input_values(synth.lowrank_plus_noise(m, n, torch.tensor([1.0, 0.5]), 1e-3, 702).numpy(), "f32")
    dev = to_device(a, "f32")
    sk = qs.Sketcher(m, n, k, l, input_dtype="f32", sketch_dtype="bf16", split_terms=2, max_block_cols=20)
    with pytest.raises(qs.QSketchError) as ei:
        sk.update_many([0, 95], [dev[:, :, 0:20], dev[:, :, 80:100]])     # second block past n
    assert ei.value.status == qs.QSK_E_ARG
    y, w = sk.sketches()
    assert float(y.abs().max()) == 0.0 and float(w.abs().max()) == 0.0
    sk.close()
