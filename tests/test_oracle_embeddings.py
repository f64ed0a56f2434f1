"""Pins of the oracle's random test matrices and low-precision formats:
Philox4x32-10 against published known-answer vectors, the Gaussian and
Rademacher distributions against Def. 4.1 / Def. 4.2 and the moments of
Lemma 4.5, and the operand rounding against PyTorch's own casts.  CPU only."""
import os

import numpy as np
import pytest
import torch

from oracle import embeddings, lowprec, quaternion as qt
from oracle.philox import philox4x32

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32(v[0], v[1], v[2], v[3], v[4], v[5])
        assert [int(o) for o in out] == v[6:10]


def test_philox_vectorised_matches_scalar():
    t = np.arange(50, dtype=np.uint64)
    vec = philox4x32(t, 7, 1, 0, 123, 456)
    for i in (0, 17, 49):
        sc = philox4x32(i, 7, 1, 0, 123, 456)
        assert [int(a[i]) for a in vec] == [int(s) for s in sc]


def test_gaussian_components_standard_normal():
    # Def. 4.1: all four components i.i.d. N(0, 1)
    g = embeddings.gaussian_entries(np.arange(200000)[:, None], np.arange(1)[None, :], 0, 11)
    x = g.reshape(4, -1)
    assert np.all(np.abs(x.mean(axis=1)) < 0.01)
    assert np.all(np.abs(x.var(axis=1) - 1) < 0.015)
    c = np.corrcoef(x)
    assert np.max(np.abs(c - np.eye(4))) < 0.01
    # Kolmogorov-Smirnov distance to the normal CDF
    from scipy.stats import kstest
    for p in range(4):
        assert kstest(x[p], "norm").statistic < 0.006


def test_gaussian_frobenius_moments_lemma45():
    """E||G||_F^2 = 4mn and E||G^dagger||_F^2 = m / (4(n-m)+2) for m <= n
    (Lemma 4.5), by Monte Carlo over independent Philox streams."""
    m, n, trials = 10, 20, 2000
    fro2, pinv2 = [], []
    for s in range(trials):
        g = embeddings.gaussian_entries(np.arange(m)[:, None], np.arange(n)[None, :], 0, 5000 + s)
        fro2.append(qt.fro(g) ** 2)
        sv = qt.singular_values(g)
        pinv2.append(np.sum(sv ** -2.0))
    assert abs(np.mean(fro2) / (4 * m * n) - 1) < 0.01
    want = m / (4 * (n - m) + 2)
    assert abs(np.mean(pinv2) / want - 1) < 0.04


def test_sgt_moment_lemma45():
    """E||S G T||_F^2 = 4 ||S||_F^2 ||T||_F^2 for Gaussian G (Lemma 4.5)."""
    rng = np.random.default_rng(3)
    s_, t_ = rng.standard_normal((4, 3, 6)), rng.standard_normal((4, 5, 2))
    vals = []
    for s in range(3000):
        g = embeddings.gaussian_entries(np.arange(6)[:, None], np.arange(5)[None, :], 0, 9000 + s)
        vals.append(qt.fro(qt.hamilton(qt.hamilton(s_, g), t_)) ** 2)
    want = 4 * qt.fro(s_) ** 2 * qt.fro(t_) ** 2
    assert abs(np.mean(vals) / want - 1) < 0.05


def test_rademacher_exact_and_balanced():
    r = embeddings.rademacher_entries(np.arange(4096)[:, None], np.arange(8)[None, :], 1, 3)
    assert set(np.unique(r)) == {-1.0, 1.0}
    assert abs(r.mean()) < 0.02
    x = r.reshape(4, -1)
    assert np.max(np.abs(np.corrcoef(x) - np.eye(4))) < 0.03
    # 32 consecutive t share one Philox call, but neighbouring entries differ
    assert not np.all(r[:, 0:32, 0] == r[:, 32:64, 0])


def test_rounding_matches_torch_casts():
    rng = np.random.default_rng(0)
    x32 = rng.standard_normal(100000).astype(np.float32)
    t = torch.from_numpy(x32)
    np.testing.assert_array_equal(lowprec.round_bf16(x32.astype(np.float64)),
                                  t.to(torch.bfloat16).double().numpy())
    x8 = (rng.standard_normal(100000) * 30).astype(np.float32)
    x8 = np.clip(x8, -440, 440)
    np.testing.assert_array_equal(lowprec.round_e4m3(x8.astype(np.float64)),
                                  torch.from_numpy(x8).to(torch.float8_e4m3fn).double().numpy())
    # subnormals of e4m3
    small = np.array([2.0 ** -9, 3 * 2.0 ** -10, 2.0 ** -11, -5 * 2.0 ** -10], dtype=np.float32)
    np.testing.assert_array_equal(lowprec.round_e4m3(small.astype(np.float64)),
                                  torch.from_numpy(small).to(torch.float8_e4m3fn).double().numpy())


def test_bf16_split_terms():
    rng = np.random.default_rng(1)
    a = rng.standard_normal(50000).astype(np.float32).astype(np.float64)
    t1 = lowprec.split_bf16(a, 1)
    t3 = lowprec.split_bf16(a, 3)
    for t in t3:
        np.testing.assert_array_equal(t, lowprec.round_bf16(t))     # each term is bf16
    e1 = np.max(np.abs(a - t1[0]) / np.abs(a))
    e3 = np.max(np.abs(a - sum(t3)) / np.abs(a))
    assert e1 <= 2.0 ** -8 and e3 <= 2.0 ** -24


def test_fp8_block_quantisation():
    rng = np.random.default_rng(2)
    a = (rng.standard_normal((70, 45)) * np.exp(rng.standard_normal((70, 45)))).astype(np.float32)
    a = a.astype(np.float64)
    deq, sc = lowprec.quantize_e4m3_blocks(a, 32, 32)
    assert sc.shape == (3, 2)
    assert np.all(np.log2(sc) == np.round(np.log2(sc)))            # powers of two
    # per block: |a|/scale <= 448, relative error <= 2^-4 for normal range values
    for bi in range(3):
        for bj in range(2):
            blk = a[bi * 32:(bi + 1) * 32, bj * 32:(bj + 1) * 32]
            assert np.max(np.abs(blk)) / sc[bi, bj] <= 448
    # and the smallest such power of two: half the scale would overflow 448
    for bi in range(3):
        for bj in range(2):
            amax = np.max(np.abs(a[bi * 32:(bi + 1) * 32, bj * 32:(bj + 1) * 32]))
            assert amax / (sc[bi, bj] / 2) > 448
    # edge values: exact 448 * 2^e keeps scale 2^e, one ulp above doubles it,
    # an all-zero block has scale 1
    for e in (-20, -1, 0, 3, 40):
        v = 448.0 * 2.0 ** e
        assert lowprec.pow2_scale(np.array(v)) == 2.0 ** e
        assert lowprec.pow2_scale(np.array(np.nextafter(np.float32(v), np.float32(np.inf)), dtype=np.float64)) == 2.0 ** (e + 1)
    assert lowprec.pow2_scale(np.array(0.0)) == 1.0
    res = a - deq
    np.testing.assert_array_equal(res.astype(np.float32).astype(np.float64), res)  # exact in FP32
    big = np.abs(a) > 1e-2 * np.max(np.abs(a))
    assert np.max(np.abs(res[big] / a[big])) <= 2.0 ** -4 + 1e-12


def test_planted_box_muller_error_is_caught(monkeypatch):
    """Dropping the factor 2 in -2 ln u would give variance 1/2: the moment
    pin must catch it."""
    orig = np.log

    def half_log(x):
        return 0.5 * orig(x)
    monkeypatch.setattr(embeddings.np, "log", half_log)
    g = embeddings.gaussian_entries(np.arange(20000)[:, None], np.arange(1)[None, :], 0, 11)
    assert np.abs(g.reshape(4, -1).var(axis=1) - 1).max() > 0.2


def test_diag_f_distribution():
    """The bad-part scaling of pseudo-SVD draws f_j from Uniform(0, 1) + 1
    (eq. sudoSVD_Hbdiagf): every value lies in (1, 2), the sample mean and
    variance match 3/2 and 1/12, the values are distinct (the point of the
    scaling is to avoid repeated singular values), and the sequence comes
    from its own Philox stream (a different seed gives different values)."""
    n = 200000
    f = embeddings.diag_f(n, 5)
    assert f.shape == (n,)
    assert np.all(f > 1.0) and np.all(f < 2.0)
    sd = np.sqrt(1.0 / 12.0 / n)
    assert abs(f.mean() - 1.5) < 6 * sd
    # variance of a uniform: 1/12; its sampling sd is sqrt(1/180 / n)
    assert abs(f.var() - 1.0 / 12.0) < 6 * np.sqrt(1.0 / 180.0 / n)
    # distinct over the sizes a repair uses (2t <= 2k columns)
    assert np.unique(f[:4096]).size == 4096
    # the empirical distribution of f - 1 is uniform on (0, 1): Kolmogorov
    # distance below 1.95 / sqrt(n) (the 0.1% point)
    u = np.sort(f - 1.0)
    ks = np.max(np.maximum(np.arange(1, n + 1) / n - u, u - np.arange(n) / n))
    assert ks < 1.95 / np.sqrt(n)
    assert not np.array_equal(embeddings.diag_f(64, 5), embeddings.diag_f(64, 6))
    np.testing.assert_array_equal(embeddings.diag_f(64, 5), f[:64])


def _e4m3_terms_torch(a, s, terms):
    """Independent scalar reference of the multi-term e4m3 split: PyTorch's
    float8_e4m3fn cast (RNE) one element at a time, float64 arithmetic."""
    out = np.zeros((terms,) + a.shape)
    for idx in np.ndindex(a.shape):
        r = float(a[idx])
        for t in range(terms):
            st = float(s[idx]) / 16.0 ** t
            q = float(torch.tensor(r / st, dtype=torch.float64).to(torch.float8_e4m3fn).double())
            out[(t,) + idx] = q * st
            r -= q * st
    return out


def test_e4m3_term_split():
    """Multi-term e4m3 block quantisation: term 0 is the plain block
    quantisation; every term is an e4m3 value times scale 16^-t (a PyTorch
    float8_e4m3fn round trip leaves it unchanged); the terms agree with an
    element-by-element reference built on PyTorch's cast; what is left after
    T terms is at most 16 s 16^(1-T) per element; data that are e4m3 values
    times the tile scale are exact in one term."""
    rng = np.random.default_rng(5)
    a = (rng.standard_normal((70, 45)) * np.exp(rng.uniform(-6, 3, (70, 45)))).astype(np.float32).astype(np.float64)
    a[:32, :32] *= 1e-3                               # tiles of very different scales
    a[40:, 32:] = 0.0                                 # an all-zero tile
    deq1, sc1 = lowprec.quantize_e4m3_blocks(a, 32, 32)
    for terms in (1, 2, 3, 4):
        parts, sc = lowprec.quantize_e4m3_terms(a, 32, 32, terms)
        np.testing.assert_array_equal(sc, sc1)
        np.testing.assert_array_equal(parts[0], deq1)
        s_full = np.repeat(np.repeat(sc, 32, axis=0), 32, axis=1)[:70, :45]
        for t, d in enumerate(parts):
            q = d / (s_full / 16.0 ** t)
            rt = torch.from_numpy(q.astype(np.float32)).to(torch.float8_e4m3fn).double().numpy()
            np.testing.assert_array_equal(rt, q)
            assert np.abs(q).max() <= (448.0 if t == 0 else 256.0)
        left = a - sum(parts)
        assert np.all(np.abs(left) <= 16.0 * s_full * 16.0 ** (1 - terms))
        if terms == 4:
            # four terms carry about as many bits as two bf16 terms near the tile maximum
            rel = np.abs(left).max() / np.abs(a).max()
            assert rel < 2.0 ** -16
    sub = a[32:64, :32]
    ref = _e4m3_terms_torch(sub, np.full(sub.shape, lowprec.pow2_scale(np.abs(sub).max())), 3)
    parts, _ = lowprec.quantize_e4m3_terms(sub, 32, 32, 3)
    np.testing.assert_array_equal(np.stack(parts), ref)
    # exact data in one term
    s = 2.0 ** -5
    vals = lowprec.round_e4m3(rng.uniform(-448, 448, (32, 32))) * s
    vals[0, 0] = 448 * s                              # fixes the tile scale at s
    parts, sc = lowprec.quantize_e4m3_terms(vals, 32, 32, 1)
    assert sc[0, 0] == s
    np.testing.assert_array_equal(parts[0], vals)
