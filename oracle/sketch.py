"""The two sketches Y = A Omega (m x s) and W = Psi A (l x n) (Section 4.1,
eq. Y=AOmegaW=PsiA), formed by linear updates over column blocks of A
(Section 4, opening, and Section 5.3: the sketches are updated as data
arrive, without revisiting A).

For an update that adds H to the columns J of A (A[:, J] += H):
    Y      += H Omega[J, :]
    W[:, J] += Psi H
Both are plain Hamilton products (``quaternion.hamilton``) in FP64.

General linear update A <- theta A + eta H (Section 5.3 streams its image
through linear updates of the sketches in the manner of Tropp et al.; the
sketches are linear in A, so the update carries over to them):
    Y <- theta Y + eta H Omega[J, :],   W <- theta W,   W[:, J] += eta Psi H.
theta = 0 stores exact zeros.

Low-precision emulation: when the sketch runs on low-precision operands, the
oracle forms the exact operand values the device uses (``lowprec``) and then
computes the same products in FP64, so that any difference from the device
is the device's accumulation error alone.
"""
from __future__ import annotations

import numpy as np

from . import embeddings, lowprec, quaternion as qt


class SketchConfig:
    """m, n: A in Q^{m x n}; k, l: sketch sizes (paper s, l), r <= s <= l
    (Section 4.1); embedding 'gaussian' or 'rademacher'; dtype of the sketch
    operands 'f64' | 'f32' | 'bf16' | 'fp8' | 'fp8x'; terms: number of bf16
    terms of the residual split of the data (bf16), or of e4m3 terms of the
    block quantisation ('fp8x': q_t with scales 16^-t times the tile scale,
    the residual carried on in e4m3); fp8_block: tile edge of the
    power-of-two fp8 scales; fp8_residual: add the exact FP32 residual of
    the fp8 quantisation as a second term; embedding_dtype: the format of the
    test-matrix values when it differs from the operand dtype (an FP64 sketch
    with the rounded test matrices of a low-precision one: a rounded Gaussian
    matrix is still an entry-independent sub-Gaussian test matrix, Def. 4.2)."""

    def __init__(self, m, n, k, l, seed=0, embedding="gaussian", dtype="f64",
                 terms=1, fp8_block=32, fp8_residual=True, embedding_dtype=None):
        if not (1 <= k <= l <= min(m, n)):
            raise ValueError("need 1 <= k <= l <= min(m, n)")
        self.m, self.n, self.k, self.l = int(m), int(n), int(k), int(l)
        self.seed = int(seed)
        self.embedding = embedding
        self.dtype = dtype
        self.terms = int(terms)
        self.fp8_block = int(fp8_block)
        self.fp8_residual = bool(fp8_residual)
        self.embedding_dtype = embedding_dtype or dtype


def data_operand(block, cfg):
    """The value of a block of A that the sketch multiplies, per the operand
    format: FP64/FP32 data as given; bf16: sum of the split terms; fp8: the
    dequantised block (plus the exact residual when enabled); fp8x: the sum
    of the e4m3 terms."""
    block = qt.as_planes(block)
    if cfg.dtype in ("f64", "f32"):
        return block
    if cfg.dtype == "bf16":
        return sum(lowprec.split_bf16(block, cfg.terms))
    if cfg.dtype == "fp8":
        out = np.empty_like(block)
        for p in range(4):
            deq, _ = lowprec.quantize_e4m3_blocks(block[p], cfg.fp8_block, cfg.fp8_block)
            out[p] = deq + (block[p] - deq if cfg.fp8_residual else 0.0)
        return out
    if cfg.dtype == "fp8x":
        out = np.empty_like(block)
        for p in range(4):
            terms, _ = lowprec.quantize_e4m3_terms(block[p], cfg.fp8_block, cfg.fp8_block, cfg.terms)
            out[p] = sum(terms)
        return out
    raise ValueError(cfg.dtype)


class Sketch:
    """Streaming state (Y, W) of the one-pass algorithm."""

    def __init__(self, cfg: SketchConfig):
        self.cfg = cfg
        self.Y = qt.zeros(cfg.m, cfg.k)
        self.W = qt.zeros(cfg.l, cfg.n)
        self.columns_seen = 0
        self._psi = None

    def psi(self):
        """Psi (l x m) as the sketch uses it (rounded to the operand dtype)."""
        if self._psi is None:
            c = self.cfg
            self._psi = embeddings.psi(c.embedding, c.l, np.arange(c.m), c.seed, c.embedding_dtype)
        return self._psi

    def omega_rows(self, col0, ncols):
        c = self.cfg
        return embeddings.omega(c.embedding, np.arange(col0, col0 + ncols), c.k, c.seed, c.embedding_dtype)

    def scale(self, theta):
        """A <- theta A, so Y <- theta Y and W <- theta W."""
        if theta == 0.0:
            self.Y[...] = 0.0
            self.W[...] = 0.0
        else:
            self.Y *= theta
            self.W *= theta

    def update(self, col0, block, theta=1.0, eta=1.0):
        """A <- theta A + eta H with H = block on the columns J = col0 ..
        col0 + ncols - 1 (defaults: A[:, J] += block), so
        Y <- theta Y + eta block Omega[J, :] and W <- theta W,
        W[:, J] += eta Psi block."""
        block = qt.as_planes(block)
        c = self.cfg
        ncols = block.shape[2]
        if block.shape[1] != c.m or col0 < 0 or col0 + ncols > c.n:
            raise ValueError("block out of range")
        if theta != 1.0:
            self.scale(theta)
        if eta != 0.0:
            a = data_operand(block, c)
            self.Y += eta * qt.hamilton(a, self.omega_rows(col0, ncols))
            self.W[:, :, col0:col0 + ncols] += eta * qt.hamilton(self.psi(), a)
        self.columns_seen += ncols


def update_block(sk, row0, col0, block):
    """A[row0 : row0 + nrows, col0 : col0 + ncols] += block: the column-block
    update of the full-height block that is zero outside those rows (the
    sketches are linear in A; the operand formats see that full block)."""
    block = qt.as_planes(block)
    full = np.zeros((4, sk.cfg.m, block.shape[2]))
    full[:, row0:row0 + block.shape[1], :] = block
    sk.update(col0, full)


def sketch_matrix(a, cfg, block_cols=None):
    """Sketch a whole matrix by streaming it in column blocks."""
    a = qt.as_planes(a)
    s = Sketch(cfg)
    bc = block_cols or a.shape[2]
    for c0 in range(0, a.shape[2], bc):
        s.update(c0, a[:, :, c0:c0 + bc])
    return s
