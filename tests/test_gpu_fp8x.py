"""The FP8X operand format on the fp8 matrix cores: the data as T e4m3
terms with the power-of-two 32 x 32 tile scales (term t at scale 16^-t
times the tile scale), test matrices rounded to e4m3, the products on the
scaled e4m3 x e4m3 instruction with FP32 accumulation.  The device
multiplies exactly the oracle's operand values (``lowprec.quantize_e4m3_terms``),
so Y and W must match the oracle's sketch entry by entry within the FP32
accumulation bound (``gpu_helpers``), for ragged shapes (rows not a multiple
of the 128-row step, column blocks not a multiple of 16 or 128), several
tiles and row groups, pure and full quaternions, bf16 and FP32 input, one to
four terms, Gaussian and Rademacher test matrices; and the QB stage on the
result must match the oracle's (Alg. 4; HX is unique, Lemma 4.2).
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


def run_case(m, n, k, l, block, terms, pure, emb, in_dt, seed, data_seed, qb=False):
    print(f"fp8x: {m}x{n} k={k} l={l} block={block} T={terms} pure={pure} {emb} {in_dt}", flush=True)
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.7 ** np.arange(10)), 1e-3, data_seed).numpy()
    a[:, : m // 3, : n // 4] *= 1e-3                    # tiles of very different scales
    if pure:
        a[0] = 0.0
    a = input_values(a, in_dt)
    dev = to_device(a, in_dt, pure=pure)
    sk = qs.Sketcher(m, n, k, l, seed=seed, embedding=emb, input_dtype=in_dt, sketch_dtype="fp8x",
                     split_terms=terms, pure=pure, max_block_cols=block)
    ref = Sketch(SketchConfig(m, n, k, l, seed=seed, embedding=emb, dtype="fp8x", terms=terms, fp8_block=32))
    bt = BoundTracker(ref)
    for c0 in range(0, n, block):
        sk.update(c0, dev[:, :, c0:c0 + block])
        ref.update(c0, a[:, :, c0:c0 + block])
        bt.update(c0, a[:, :, c0:c0 + block])
    y, w = (to_numpy(t) for t in sk.sketches())
    bt.check(y, w, f"fp8x T={terms} {emb} pure={pure} {in_dt}")
    if qb:
        for kind in ("pseudo_qr", "pseudo_svd"):
            q, x, _ = sk.finalize(kind)
            h_o, x_o, _ = onepass.qb_stage(ref, kind)
            d = rel(qt.hamilton(to_numpy(q), to_numpy(x)), qt.hamilton(h_o, x_o))
            print(f"  {kind}: |HX - HX_o| / |HX_o| = {d:.2e}", flush=True)
            assert d < 1e-4
    sk.close()


@pytest.mark.parametrize("terms", [1, 2, 3, 4])
def test_fp8x_ragged(terms):
    run_case(300, 200, 24, 49, 70, terms, pure=False, emb="gaussian", in_dt="f32", seed=3, data_seed=801)


@pytest.mark.parametrize("pure,emb,in_dt", [(True, "gaussian", "f32"), (True, "rademacher", "bf16"),
                                            (False, "rademacher", "f32")])
def test_fp8x_formats(pure, emb, in_dt):
    run_case(411, 150, 20, 41, 150, 3, pure=pure, emb=emb, in_dt=in_dt, seed=4, data_seed=802)


def test_fp8x_multitile_and_qb_stage():
    """Several 128-row steps and split-K chunks, two row groups of W tiles
    (l = 201), seven column tiles of Y (k = 100), blocks of 150 columns (two
    128-column steps of Y, the second ragged), and the QB stage."""
    run_case(1500, 300, 100, 201, 150, 3, pure=True, emb="gaussian", in_dt="f32", seed=5, data_seed=803,
             qb=True)


def test_fp8x_rejected_where_unsupported():
    with pytest.raises(qs.QSketchError):
        qs.Sketcher(100, 80, 10, 21, input_dtype="f32", sketch_dtype="fp8x", split_terms=5)
    with pytest.raises(qs.QSketchError):
        qs.Batch([(200, 100, 10, 21, 0)], input_dtype="f32", sketch_dtype="fp8x", split_terms=2)
