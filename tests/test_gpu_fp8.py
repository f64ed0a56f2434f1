"""The fp8 operand format (sketch_dtype fp8): data quantised to e4m3 with a
power-of-two scale per 32 x 32 tile of each plane of the update block, with
(split_terms 2) or without (split_terms 1) the exact FP32 residual as a
correction term; test matrices rounded to e4m3.  The oracle forms the same
operand values (oracle.lowprec) and multiplies in FP64.

Tolerances, entry by entry (``gpu_helpers.check_sketches``): without the
residual the device multiplies exactly the oracle's operand values, so what
remains is the FP32 accumulation error, within 8 sqrt(K) u B per entry (B the
sum of the absolute values of the entry's K terms); with it the residual is
carried as two bf16 terms, i.e. to 2^-17 of the residual, itself at most the
value, which adds 2^-17 B to the bound.
"""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle import onepass, quaternion as qt
from oracle.sketch import SketchConfig, sketch_matrix
from tests.gpu_helpers import check_sketches, input_values, rel, run_sketch, to_numpy

pytestmark = pytest.mark.gpu


def oracle(a, m, n, k, l, block, seed, emb, terms):
    cfg = SketchConfig(m, n, k, l, seed=seed, embedding=emb, dtype="fp8", fp8_block=32,
                       fp8_residual=terms == 2)
    return sketch_matrix(a, cfg, block_cols=block)


@pytest.mark.parametrize("dtype,emb,terms", [("f32", "gaussian", 2), ("f32", "gaussian", 1),
                                             ("f32", "rademacher", 2), ("bf16", "rademacher", 1),
                                             ("bf16", "gaussian", 2)])
def test_fp8_sketch_parity_ragged(dtype, emb, terms):
    """Several tiles plus ragged tails, streamed in uneven blocks (50 columns:
    the tile grid restarts at every block)."""
    m, n, k, l, block = 333, 257, 12, 25, 50
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(10)), 1e-3, 77).numpy()
    a = input_values(a, dtype)
    sk, _ = run_sketch(a, m, n, k, l, block, dtype=dtype, sketch="fp8", emb=emb, seed=5, terms=terms)
    y, w = (to_numpy(t) for t in sk.sketches())
    ref = oracle(a, m, n, k, l, block, 5, emb, terms)
    check_sketches(y, w, ref, a, f"fp8 ragged {dtype}/{emb}/x{terms}", block_cols=block)
    assert rel(y, ref.Y) < 1e-5, rel(y, ref.Y)
    assert rel(w, ref.W) < 1e-5, rel(w, ref.W)


@pytest.mark.parametrize("terms,pure", [(2, False), (1, True), (2, True)])
def test_fp8_sketch_parity_multitile(terms, pure):
    """Matrix-core tiling (7 column tiles of Y, 13 row tiles of W, split K)
    with tiles of very different magnitude: a zero tile, a tile holding one
    outlier 1e6 times its neighbours (which then quantise to subnormals or
    zero and live in the residual), and tiny values near the bottom of the
    FP32 range."""
    m, n, k, l, block = 1500, 300, 100, 201, 130
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.85 ** np.arange(30)), 1e-3, 88).numpy()
    a[:, 64:96, 32:64] = 0.0                         # an all-zero tile (scale 1)
    a[1, 100, 70] = 1e6 * np.abs(a).max()            # outlier in tile (3, 2) of block 0
    a[2, 1400:1432, 200:232] *= 1e-30                # tiny values
    if pure:
        a[0] = 0.0
    a = input_values(a, "f32")
    sk, _ = run_sketch(a, m, n, k, l, block, dtype="f32", sketch="fp8", emb="gaussian", seed=21,
                       terms=terms, pure=pure)
    y, w = (to_numpy(t) for t in sk.sketches())
    ref = oracle(a, m, n, k, l, block, 21, "gaussian", terms)
    check_sketches(y, w, ref, a, f"fp8 multitile x{terms} pure={pure}", block_cols=block)


@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_fp8_one_pass_error(kind):
    """Rank 20 plus 1e-4 noise (FP32 values).  The e4m3 test matrices are a
    different draw from the Gaussian ones (rounding to 4 significant bits),
    so the FP64 reference is the oracle's one-pass approximation with the
    same e4m3 test matrices and exact data: with the residual term the
    device reaches its error within 1e-3 relative; without it the error is
    larger, and the QB stage on that sketch gives the oracle's HX for the
    oracle's sketch of the fp8-quantised data (HX is unique, Lemma 4.2)."""
    m, n, k, l, block = 1000, 800, 40, 81, 256
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.8 ** np.arange(20)), 1e-4, 99).numpy()
    a = input_values(a, "f32")
    ref2 = oracle(a, m, n, k, l, block, 0, "gaussian", 2)          # exact data, e4m3 test matrices
    h2, x2, _ = onepass.qb_stage(ref2, kind)
    e_ref = onepass.rel_error(a, h2, x2)
    e = {}
    for terms in (2, 1):
        sk, dev = run_sketch(a, m, n, k, l, block, dtype="f32", sketch="fp8", seed=0, terms=terms)
        q, x, rep = sk.finalize(kind)
        e[terms] = sk.rel_error(dev, q, x)
        if terms == 1:
            ref = oracle(a, m, n, k, l, block, 0, "gaussian", 1)
            h_o, x_o, _ = onepass.qb_stage(ref, kind)
            hx = qt.hamilton(to_numpy(q), to_numpy(x))
            assert rel(hx, qt.hamilton(h_o, x_o)) < 1e-4
        sk.close()
    assert abs(e[2] - e_ref) <= 1e-3 * e_ref, (e, e_ref)
    assert e[1] > 10 * e_ref
