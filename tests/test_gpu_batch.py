"""The batched path (qsketch_batch_*): independent problems of different
shapes, sketched and finalised together through grouped launches, give
problem by problem the oracle's one-pass result on the same operands
(Alg. 4; HX is unique, Lemma 4.2) and the result of a single-problem
context.  One batch includes an exactly low-rank problem, which takes the
rank-deficient branches (shifted CholeskyQR, skipped corrections, minimum-norm
core solve) while its neighbours do not.
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

SHAPES = [  # m, n, k, l, seed
    (333, 257, 12, 25, 11),
    (700, 300, 20, 41, 12),
    (512, 640, 16, 33, 13),
    (1200, 250, 40, 81, 14),
    (257, 511, 8, 17, 15),
]


def inputs(shapes, dtype, exact_rank=None):
    mats = []
    for i, (m, n, k, l, seed) in enumerate(shapes):
        if exact_rank is not None and i == 0:
            sig, noise = torch.tensor([1.0, 0.5, 0.3, 0.2][:exact_rank]), 0.0
        else:
            sig, noise = torch.tensor(0.8 ** np.arange(max(2, k // 2))), 1e-3
        a = synth.lowrank_plus_noise(m, n, sig, noise, 300 + i).numpy()
        mats.append(input_values(a, dtype))
    return mats


@pytest.mark.parametrize("sketch,terms", [("bf16", 2), ("f32", 1)])
@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_batch_matches_oracle_and_single(sketch, terms, kind):
    mats = inputs(SHAPES, "f32")
    devs = [to_device(a, "f32") for a in mats]
    b = qs.Batch(SHAPES, input_dtype="f32", sketch_dtype=sketch, split_terms=terms)
    qb, xb, reps = b.run(devs, kind)
    errs = b.rel_error(devs, qb, xb)
    for i, (m, n, k, l, seed) in enumerate(SHAPES):
        a = mats[i]
        # oracle on the same operands (bf16 split / fp32 values, rounded test matrices)
        cfg = SketchConfig(m, n, k, l, seed=seed, dtype=sketch, terms=terms)
        ref = sketch_matrix(a, cfg)
        h_o, x_o, info = onepass.qb_stage(ref, kind)
        hx_o = qt.hamilton(h_o, x_o)
        hx_b = qt.hamilton(to_numpy(qb[i]), to_numpy(xb[i]))
        e_o = onepass.rel_error(a, h_o, x_o)
        assert rel(hx_b, hx_o) < 1e-4, (i, rel(hx_b, hx_o))
        assert abs(errs[i] - e_o) <= 1e-4 * e_o, (i, errs[i], e_o)
        # a single-problem context on the same data
        sk = qs.Sketcher(m, n, k, l, seed=seed, input_dtype="f32", sketch_dtype=sketch,
                         split_terms=terms, max_block_cols=n)
        sk.update(0, devs[i])
        q1, x1, rep1 = sk.finalize(kind)
        hx_1 = qt.hamilton(to_numpy(q1), to_numpy(x1))
        assert rel(hx_b, hx_1) < 1e-5, (i, rel(hx_b, hx_1))
        np.testing.assert_allclose(reps[i]["kappa"], rep1["kappa"], rtol=1e-4)
        if kind == "pseudo_qr":
            assert reps[i]["kappa"] < 10 and len(reps[i]["eps"]) == 3
        else:
            assert reps[i]["orth_defect"] < 1e-10
        sk.close()
    b.close()


@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_batch_with_exact_low_rank_problem(kind):
    shapes = [(300, 240, 8, 17, 9)] + SHAPES[:3]
    mats = inputs(shapes, "f32", exact_rank=4)
    devs = [to_device(a, "f32") for a in mats]
    b = qs.Batch(shapes, input_dtype="f32", sketch_dtype="f32")
    qb, xb, reps = b.run(devs, kind)
    errs = b.rel_error(devs, qb, xb)
    assert errs[0] < 1e-5, errs[0]
    for i in range(1, len(shapes)):
        m, n, k, l, seed = shapes[i]
        cfg = SketchConfig(m, n, k, l, seed=seed, dtype="f32")
        h_o, x_o, _ = onepass.qb_stage(sketch_matrix(mats[i], cfg), kind)
        e_o = onepass.rel_error(mats[i], h_o, x_o)
        assert abs(errs[i] - e_o) <= 1e-4 * e_o, (i, errs[i], e_o)
    b.close()


def test_batch_rerun_is_repeatable():
    """A second run on the same batch context (and its argument tables)
    reproduces the first bit for bit."""
    mats = inputs(SHAPES[:3], "f32")
    devs = [to_device(a, "f32") for a in mats]
    b = qs.Batch(SHAPES[:3], input_dtype="f32", sketch_dtype="bf16", split_terms=2)
    q1, x1, _ = b.run(devs, "pseudo_svd")
    q2, x2, _ = b.run(devs, "pseudo_svd")
    for i in range(3):
        assert torch.equal(q1[i], q2[i]) and torch.equal(x1[i], x2[i])
    b.close()


@pytest.mark.parametrize("kind", ["pseudo_qr", "pseudo_svd"])
def test_batch_graph_replays_match_careful_run(kind):
    """The optimistic run, issued as stream-ordered launches and as a
    captured graph, gives the careful run's outputs bit for bit.  The graph
    is replayed several times with other work in between (a careful run of
    the other rangefinder, an error pass), and recaptured when the output
    buffers change; every replay is checked."""
    other = "pseudo_svd" if kind == "pseudo_qr" else "pseudo_qr"
    mats = inputs(SHAPES, "f32")
    devs = [to_device(a, "f32") for a in mats]
    b = qs.Batch(SHAPES, input_dtype="f32", sketch_dtype="bf16", split_terms=2)
    b.set_exec("careful")
    q0, x0, r0 = b.run(devs, kind)
    b.set_exec("stream")
    q1, x1, r1 = b.run(devs, kind)
    for i in range(len(SHAPES)):
        assert torch.equal(q0[i], q1[i]) and torch.equal(x0[i], x1[i]), i
        assert r0[i]["kappa"] == r1[i]["kappa"] and r0[i]["passes"] == r1[i]["passes"], i
    outs = b.outputs()
    for rep in range(4):
        b.set_exec("graph")
        if rep == 2:
            outs = b.outputs()                     # new pointers: a new capture
        q2, x2, r2 = b.run(devs, kind, outputs=outs)
        torch.cuda.synchronize()
        for i in range(len(SHAPES)):
            assert torch.equal(q0[i], q2[i]) and torch.equal(x0[i], x2[i]), (rep, i)
            assert r0[i]["kappa"] == r2[i]["kappa"], (rep, i)
        # other work between the replays
        b.set_exec("careful")
        b.run(devs, other)
        b.rel_error(devs, q2, x2)
    b.close()


@pytest.mark.parametrize("sketch,terms", [("bf16", 2), ("f32", 1)])
def test_batch_autotune(sketch, terms):
    """The autotuner picks one of the candidate tile shapes (13 row tiles of
    W only with bf16 operands), runs after it give the same approximation,
    and a second batch with the same shapes takes the remembered choice
    without timing."""
    mats = inputs(SHAPES, "f32")
    devs = [to_device(a, "f32") for a in mats]
    b = qs.Batch(SHAPES, input_dtype="f32", sketch_dtype=sketch, split_terms=terms)
    q0, x0, _ = b.run(devs, "pseudo_qr")
    nmt, nj, wb = b.autotune(devs, reps=2)
    assert nmt in ((4, 7, 8, 13) if sketch == "bf16" else (4, 7)) and nj in (4, 7)
    assert wb in (512, 2048, 8192)
    q1, x1, _ = b.run(devs, "pseudo_qr")
    for i in range(len(SHAPES)):
        hx0 = qt.hamilton(to_numpy(q0[i]), to_numpy(x0[i]))
        hx1 = qt.hamilton(to_numpy(q1[i]), to_numpy(x1[i]))
        assert rel(hx1, hx0) < 1e-12, (i, rel(hx1, hx0))
    b2 = qs.Batch(SHAPES, input_dtype="f32", sketch_dtype=sketch, split_terms=terms)
    assert b2.autotune(devs, reps=0) == (nmt, nj, wb)
    b2.close()
    b.close()


_CACHE_CHILD = r"""
import sys, torch
sys.path.insert(0, sys.argv[1])
import paper_2404_14783_amd as qs
shapes = [(300, 200, 12, 25, 0), (257, 130, 8, 17, 1)]
devs = [qs.to_colmajor(torch.randn(4, m, n, device="cuda")) for (m, n, k, l, s) in shapes]
b = qs.Batch(shapes, input_dtype="f32", sketch_dtype="bf16", split_terms=2)
print("TILES", *b.autotune(devs, reps=int(sys.argv[2])))
b.close()
"""


def test_batch_tune_cache_file(tmp_path):
    """QSK_TUNE_CACHE: a process that tunes appends its choice to the file;
    a new process takes an entry of the file without timing (reps = 0), also
    one that no timing would produce, and ignores lines that do not parse."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, QSK_TUNE_CACHE=str(cache))

    def child(reps):
        r = subprocess.run([sys.executable, "-c", _CACHE_CHILD, root, str(reps)], env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        line = [x for x in r.stdout.splitlines() if x.startswith("TILES")][-1]
        return tuple(int(v) for v in line.split()[1:])

    first = child(2)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    fields = lines[0].split()
    assert len(fields) == 6 and tuple(int(v) for v in fields[3:]) == first
    # the same key with another choice, after a malformed line: taken as is
    other = (13, 7, 8192) if first != (13, 7, 8192) else (4, 4, 512)
    cache.write_text("not an entry\n" + " ".join(fields[:3] + [str(v) for v in other]) + "\n")
    assert child(0) == other
    assert len(cache.read_text().splitlines()) == 2          # nothing appended


# HX of the batch workload against the oracle: the device sketches differ
# from the oracle's (same operands) by FP32 accumulation only
BATCH_HX_TOL = 1e-4


@pytest.mark.timeout(900)
def test_batch64_workload_every_problem_vs_oracle():
    """The 64-problem workload of the benchmark (log-uniform m in [512, 8192]
    and n in [256, 4096], rank 8..64 with geometric decay, k = 2r,
    l = 2k + 1, FP32 data, BF16 two-term operands, autotuned tiles), every
    problem against the oracle's one-pass result on the same operands
    (Alg. 4): the relative error within 1e-3 of the oracle's (the equal-error
    criterion) and sampled rows and columns of HX entry by entry (HX is
    unique, Lemma 4.2)."""
    from tests.gpu_helpers import hx_margin, sample
    specs = synth.batch_specs(64)
    shapes = [(sp["m"], sp["n"], sp["k"], sp["l"], i) for i, sp in enumerate(specs)]
    mats = [qs.to_colmajor(synth.batch_matrix(sp, i, device="cuda")) for i, sp in enumerate(specs)]
    b = qs.Batch(shapes, input_dtype="f32", sketch_dtype="bf16", split_terms=2)
    b.autotune(mats, reps=1)
    dev = {}
    for kind in ("pseudo_qr", "pseudo_svd"):
        qb, xb, reps = b.run(mats, kind)
        errs = b.rel_error(mats, qb, xb)
        dev[kind] = ([to_numpy(t) for t in qb], [to_numpy(t) for t in xb], reps, errs)
        del qb, xb
    b.close()
    worst_e, worst_hx = 0.0, 0.0
    for i, (m, n, k, l, seed) in enumerate(shapes):
        a = mats[i].double().cpu().numpy()
        ref = sketch_matrix(a, SketchConfig(m, n, k, l, seed=seed, dtype="bf16", terms=2))
        rows = sample(m, [0, m - 1], 6, 100 + i)
        cols = sample(n, [0, n - 1], 6, 200 + i)
        for kind in ("pseudo_qr", "pseudo_svd"):
            q, x, reps, errs = dev[kind]
            h_o, x_o, _ = onepass.qb_stage(ref, kind)
            e_o = onepass.rel_error(a, h_o, x_o)
            de = abs(errs[i] - e_o) / e_o
            mg = hx_margin(q[i], x[i], h_o, x_o, rows, cols)
            worst_e, worst_hx = max(worst_e, de), max(worst_hx, mg)
            assert de <= 1e-3, (i, kind, errs[i], e_o)
            assert mg < BATCH_HX_TOL, (i, kind, mg)
            if kind == "pseudo_qr":
                assert reps[i]["kappa"] < 10 and len(reps[i]["eps"]) == 3, (i, reps[i])
            else:
                assert reps[i]["orth_defect"] < 1e-10, (i, reps[i])
        del a, ref
    print(f"batch64: worst relative error difference {worst_e:.2e} (limit 1e-3), "
          f"worst HX margin {worst_hx:.2e} (limit {BATCH_HX_TOL:g})", flush=True)
