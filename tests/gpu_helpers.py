"""Helpers shared by the GPU parity tests: move oracle-side NumPy inputs to
the device in the library's layout and back."""
import numpy as np
import torch

import paper_2404_14783_amd as qs

TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def to_device(a_np, dtype, pure=False):
    """(4, m, n) NumPy -> (4 or 3, m, n) device tensor with column-major planes."""
    t = torch.from_numpy(np.ascontiguousarray(a_np[1:] if pure else a_np))
    t = t.to(TORCH[dtype])
    return qs.to_colmajor(t.cuda())


def input_values(a_np, dtype):
    """The values the device sees for a given input dtype (exact widening)."""
    t = torch.from_numpy(np.ascontiguousarray(a_np)).to(TORCH[dtype])
    return t.double().numpy()


def to_numpy(t):
    return t.detach().double().cpu().numpy()


def rel(a, b):
    d = np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel())
    n = np.linalg.norm(np.asarray(b).ravel())
    return d / n if n > 0 else d


def run_sketch(a_np, m, n, k, l, block, dtype="f64", sketch="f64", emb="gaussian", seed=0,
               terms=1, pure=False, order=None):
    sk = qs.Sketcher(m, n, k, l, seed=seed, embedding=emb, input_dtype=dtype, sketch_dtype=sketch,
                     split_terms=terms, pure=pure, max_block_cols=block)
    dev = to_device(a_np, dtype, pure=pure)
    starts = list(range(0, n, block))
    if order is not None:
        starts = [starts[i] for i in order]
    for c0 in starts:
        sk.update(c0, dev[:, :, c0:c0 + block])
    torch.cuda.synchronize()
    return sk, dev
