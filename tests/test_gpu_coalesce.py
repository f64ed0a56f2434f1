"""Coalescing of thin updates (qsk_config.coalesce_cols): a context gathers
consecutive narrow column blocks and runs the sketch products on the
gathered block.  The sketches are linear in A (Section 4, opening; Section
5.3), so the result equals the oracle's sketch streamed in the gathered
blocks, entry by entry within the accumulation bound (``gpu_helpers``); in
the FP8 format the per-tile scales are those of the gathered block, which
the oracle reproduces by streaming the same gathered blocks.  Calls that
need the sketches (finalize, sketches, a general update, a non-contiguous
block) run the pending columns first; reset and set_sketches drop them.
"""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle import onepass, quaternion as qt
from oracle.sketch import Sketch, SketchConfig
from tests.gpu_helpers import BoundTracker, input_values, rel, to_device, to_numpy

pytestmark = pytest.mark.gpu


def oracle_cfg(m, n, k, l, seed, sketch, terms):
    if sketch == "fp8":
        return SketchConfig(m, n, k, l, seed=seed, dtype="fp8", fp8_block=32, fp8_residual=terms == 2)
    return SketchConfig(m, n, k, l, seed=seed, dtype=sketch, terms=terms)


@pytest.mark.parametrize("sketch,terms,pure", [("bf16", 2, False), ("fp8", 2, True), ("f32", 1, False),
                                               ("fp8x", 3, True), ("fp8x", 2, False)])
def test_coalesced_stream_matches_oracle(sketch, terms, pure):
    """300 columns arriving in blocks of 10 with coalesce_cols = 64: the
    context gathers 6 blocks (60 columns) per product; the oracle streams
    the same 60-column blocks."""
    m, n, k, l, block, gather = 1500, 300, 24, 49, 10, 64
    print(f"coalesced stream: {sketch} x{terms} pure={pure}", flush=True)
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(12)), 1e-3, 601).numpy()
    if pure:
        a[0] = 0.0
    a = input_values(a, "f32")
    dev = to_device(a, "f32", pure=pure)
    sk = qs.Sketcher(m, n, k, l, seed=3, input_dtype="f32", sketch_dtype=sketch, split_terms=terms,
                     pure=pure, max_block_cols=block, coalesce_cols=gather)
    for c0 in range(0, n, block):
        sk.update(c0, dev[:, :, c0:c0 + block])
    ref = Sketch(oracle_cfg(m, n, k, l, 3, sketch, terms))
    bt = BoundTracker(ref)
    eff = (gather // block) * block                   # 60 columns per gathered block
    for c0 in range(0, n, eff):
        ref.update(c0, a[:, :, c0:c0 + eff])
        bt.update(c0, a[:, :, c0:c0 + eff])
    y, w = (to_numpy(t) for t in sk.sketches())
    bt.check(y, w, f"coalesced {sketch} x{terms}")
    assert sk.columns_seen == n
    for kind in ("pseudo_qr", "pseudo_svd"):
        q, x, _ = sk.finalize(kind)
        h_o, x_o, _ = onepass.qb_stage(ref, kind)
        d = rel(qt.hamilton(to_numpy(q), to_numpy(x)), qt.hamilton(h_o, x_o))
        print(f"  {kind}: |HX - HX_o| / |HX_o| = {d:.2e}", flush=True)
        assert d < 1e-4
    sk.close()


def test_coalescing_flushes_and_drops():
    """A non-contiguous block, a general update and a finalize in the middle
    of a stream run the pending columns first (the sketches then equal an
    uncoalesced context's up to FP32 rounding order); reset drops them."""
    m, n, k, l = 800, 200, 12, 25
    a = input_values(synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(8)), 1e-3, 602).numpy(), "f32")
    dev = to_device(a, "f32")
    kw = dict(seed=4, input_dtype="f32", sketch_dtype="bf16", split_terms=2, max_block_cols=40)
    co = qs.Sketcher(m, n, k, l, coalesce_cols=100, **kw)
    pl = qs.Sketcher(m, n, k, l, **kw)
    steps = [(0, 10), (10, 10), (20, 20), (100, 10), (110, 30), ("lin", None), (40, 10), ("fin", None),
             (50, 40), (90, 10), (140, 40), (180, 20)]
    for c0, nc in steps:
        if c0 == "lin":
            h = dev[:, :, 150:160]
            co.update(150, h, theta=0.5, eta=2.0)
            pl.update(150, h, theta=0.5, eta=2.0)
        elif c0 == "fin":
            q1, x1, _ = co.finalize("pseudo_svd")
            q2, x2, _ = pl.finalize("pseudo_svd")
            hx1 = qt.hamilton(to_numpy(q1), to_numpy(x1))
            hx2 = qt.hamilton(to_numpy(q2), to_numpy(x2))
            assert rel(hx1, hx2) < 1e-5
        else:
            co.update(c0, dev[:, :, c0:c0 + nc])
            pl.update(c0, dev[:, :, c0:c0 + nc])
    y1, w1 = (to_numpy(t) for t in co.sketches())
    y2, w2 = (to_numpy(t) for t in pl.sketches())
    assert rel(y1, y2) < 1e-6 and rel(w1, w2) < 1e-6
    # pending columns are dropped by reset
    co.update(0, dev[:, :, 0:10])
    co.reset()
    y3, w3 = (to_numpy(t) for t in co.sketches())
    assert float(np.abs(y3).max()) == 0.0 and float(np.abs(w3).max()) == 0.0
    co.close()
    pl.close()
