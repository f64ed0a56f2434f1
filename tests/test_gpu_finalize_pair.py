"""qsketch_finalize_pair: two QB stages (Alg. 4) of one sketch run side by
side on two streams of the context.  Each stage must give exactly what
qsketch_finalize gives for it alone, bit for bit (the same kernels read the
same inputs; only their interleaving on the device differs): Q, X and the
report, for both rangefinders (Alg. 1, Alg. 3 and its Gram-Schmidt branch),
every operand format, pure input, with and without the core solve, with the
Gram of Y computed by the pair itself or cached by an earlier finalize, and
where a Cholesky breakdown of the Gram sends a stage to the careful path.
"""
import numpy as np
import pytest
import torch

import paper_2404_14783_amd as qs
import synth
from oracle import quaternion as qt
from oracle.rangefinders import pseudo_svd
from tests.gpu_helpers import input_values, to_device, to_numpy

pytestmark = pytest.mark.gpu


def assert_same(pair, seq, what):
    for (qp, xp, rp), (qs_, xs, rs), kind in zip(pair, seq, ("a", "b")):
        assert torch.equal(qp, qs_), f"{what}: Q of stage {kind} differs"
        if xs is None:
            assert xp is None
        else:
            assert torch.equal(xp, xs), f"{what}: X of stage {kind} differs"
        assert rp == rs, f"{what}: report of stage {kind} differs: {rp} vs {rs}"


def run_both(sk, kinds, solve=None):
    seq = [sk.finalize(kd, solve=solve) for kd in kinds]
    pair = sk.finalize_pair(kinds, solve=solve)
    return pair, seq


@pytest.mark.parametrize("sketch,emb,pure", [("f64", "gaussian", False), ("bf16", "rademacher", False),
                                             ("f32", "gaussian", True), ("fp8x", "gaussian", False)])
def test_pair_matches_sequential(sketch, emb, pure):
    m, n, k, l, block = 2500, 700, 32, 65, 256
    print(f"finalize pair: {sketch} {emb} pure={pure}", flush=True)
    a = synth.lowrank_plus_noise(m, n, torch.tensor(0.7 ** np.arange(20)), 1e-3, 91).numpy()
    if pure:
        a[0] = 0.0
    a = input_values(a, "f32")
    dev = to_device(a, "f32", pure=pure)
    terms = {"bf16": 2, "fp8x": 3}.get(sketch, 1)
    sk = qs.Sketcher(m, n, k, l, seed=3, embedding=emb, input_dtype="f32", sketch_dtype=sketch,
                     split_terms=terms, pure=pure, max_block_cols=block)
    for c0 in range(0, n, block):
        sk.update(c0, dev[:, :, c0:c0 + block])
    kinds = ("pseudo_qr", "pseudo_svd")
    # the pair first: it forms the Gram of Y itself
    pair = sk.finalize_pair(kinds)
    seq = [sk.finalize(kd) for kd in kinds]
    assert_same(pair, seq, "fresh Gram")
    assert pair[0][2]["columns_seen"] == n
    # a further update (the cached Gram is dropped), the sequential calls first
    sk.update(0, dev[:, :, :block])
    pair, seq = run_both(sk, kinds)
    assert_same(pair, seq, "after an update")
    # swapped order, the Gram-Schmidt repair, rangefinders only
    pair, seq = run_both(sk, ("pseudo_svd_gs", "pseudo_qr"))
    assert_same(pair, seq, "svd_gs + qr")
    pair, seq = run_both(sk, kinds, solve=False)
    assert_same(pair, seq, "rangefinders only")
    # caller-provided outputs are written in place
    outs = [(torch.zeros_like(pair[0][0]), None), (torch.zeros_like(pair[1][0]), None)]
    got = sk.finalize_pair(kinds, outputs=outs, solve=False)
    assert got[0][0].data_ptr() == outs[0][0].data_ptr()
    assert_same(got, seq, "given outputs")
    sk.close()


def test_pair_careful_path():
    """Sketches whose Grams break a Cholesky factorisation (kappa(Y) = 1e14
    and 1e22, loaded with qsketch_set_sketches): the pair's optimistic runs
    fail and each stage is run again the careful way (pseudo-QR stops its
    corrections at a singular Gram; at 1e22 the first Gram needs the shifted
    CholeskyQR)."""
    m, k = 600, 40
    rng = np.random.default_rng(77)
    u, _ = pseudo_svd(qt.random_gaussian(rng, m, k))
    v, _ = pseudo_svd(qt.random_gaussian(rng, k, k))
    sk = qs.Sketcher(m, k, k, k, y_only=True)
    for kappa in (1e14, 1e22):
        sig = kappa ** (-np.arange(k) / (k - 1))
        y = qt.hamilton(u * sig[None, None, :], qt.conj_t(v))
        sk.set_sketches(to_device(y, "f64"), None, k)
        kinds = ("pseudo_qr", "pseudo_svd")
        pair, seq = run_both(sk, kinds, solve=False)
        print(f"kappa(Y) = {kappa:.0e}: flags {seq[0][2]['flags']} / {seq[1][2]['flags']}", flush=True)
        assert seq[0][2]["flags"], seq[0][2]          # the careful path ran
        assert_same(pair, seq, f"careful path, kappa {kappa:.0e}")
        assert all(np.isfinite(to_numpy(q)).all() for q, _, _ in pair)
    sk.close()


def test_pair_rejects_shared_outputs():
    m, n, k, l = 300, 200, 8, 17
    sk = qs.Sketcher(m, n, k, l)
    a = to_device(input_values(synth.lowrank_plus_noise(m, n, torch.ones(4), 1e-2, 5).numpy(), "f64"), "f64")
    sk.update(0, a)
    q = torch.empty(4, k, m, dtype=torch.float64, device=sk.device).transpose(1, 2)
    with pytest.raises(qs.QSketchError):
        sk.finalize_pair(outputs=[(q, None), (q, None)], solve=False)
    # the context stays usable
    pair, seq = run_both(sk, ("pseudo_qr", "pseudo_svd"))
    assert_same(pair, seq, "after a rejected call")
    sk.close()


def test_pair_one_stage_without_solve():
    """Xb = NULL: the second stage runs its rangefinder only, the first
    solves; each matches its own qsketch_finalize call."""
    import ctypes
    m, n, k, l = 1500, 400, 16, 33
    sk = qs.Sketcher(m, n, k, l, seed=9, input_dtype="f32", sketch_dtype="bf16", split_terms=2)
    a = input_values(synth.lowrank_plus_noise(m, n, torch.tensor(0.6 ** np.arange(10)), 1e-3, 17).numpy(), "f32")
    sk.update(0, to_device(a, "f32"))
    qa, xa, ra = sk.finalize("pseudo_svd")
    qb, _, rb = sk.finalize("pseudo_qr", solve=False)
    outs = [sk._qb_outputs(None, None, True), sk._qb_outputs(None, None, False)]
    reps = [qs.QskReport(), qs.QskReport()]
    st = sk._lib.qsketch_finalize_pair(
        sk._ctx, qs.RANGEFINDERS["pseudo_svd"], outs[0][2], outs[0][3], outs[0][4], outs[0][5],
        ctypes.byref(reps[0]), qs.RANGEFINDERS["pseudo_qr"], outs[1][2], outs[1][3], outs[1][4], outs[1][5],
        ctypes.byref(reps[1]))
    assert st == 0, sk._lib.qsketch_last_error(sk._ctx)
    assert outs[1][1] is None
    assert torch.equal(outs[0][0], qa) and torch.equal(outs[0][1], xa)
    assert torch.equal(outs[1][0], qb)
    assert reps[0].as_dict() == ra and reps[1].as_dict() == rb
    sk.close()
