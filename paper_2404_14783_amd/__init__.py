"""Python binding of the qsketch C ABI (include/qsketch.h).

Argument marshalling only: every step of the sketch and of the QB stage runs in
the HIP kernels of ``libqsketch.so``; PyTorch supplies device memory and the
stream.  The library must have been built (``paper_2404_14783_amd.build``);
importing this module fails loudly if it is missing.

Quaternion matrices are torch tensors of shape (4, rows, cols) (planes w, x,
y, z), or (3, rows, cols) for a pure quaternion (planes x, y, z), whose planes
are column-major: ``t.stride(1) == 1``.  ``qempty`` and ``to_colmajor`` make
such tensors.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsketch.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "qsketch.h")

QSK_OK, QSK_E_ARG, QSK_E_STATE, QSK_E_NOMEM, QSK_E_HIP, QSK_E_NUMERIC, QSK_E_UNSUPPORTED = range(7)
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3, "fp8x": 4}
EMBEDDINGS = {"gaussian": 0, "rademacher": 1}
RANGEFINDERS = {"pseudo_qr": 0, "pseudo_svd": 1, "pseudo_svd_gs": 2}
FLAG_NAMES = {1: "chol_fallback", 2: "rank_deficient", 4: "nonfinite", 8: "bad_pairs"}
TORCH_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


class QskConfig(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64),
        ("k", ctypes.c_int32), ("l", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("embedding", ctypes.c_int32), ("input_dtype", ctypes.c_int32),
        ("sketch_dtype", ctypes.c_int32), ("pure", ctypes.c_int32),
        ("split_terms", ctypes.c_int32), ("n_correction", ctypes.c_int32),
        ("n_power", ctypes.c_int32), ("max_block_cols", ctypes.c_int64),
        ("y_only", ctypes.c_int32), ("embedding_round", ctypes.c_int32),
        ("coalesce_cols", ctypes.c_int32),
    ]


class QskReport(ctypes.Structure):
    _fields_ = [
        ("kappa", ctypes.c_double), ("kappa_initial", ctypes.c_double),
        ("eps", ctypes.c_double * 8), ("n_eps", ctypes.c_int32),
        ("t_bad", ctypes.c_int32), ("flags", ctypes.c_int32), ("passes", ctypes.c_int32),
        ("columns_seen", ctypes.c_int64), ("orth_defect", ctypes.c_double),
    ]

    def as_dict(self):
        return {
            "kappa": self.kappa, "kappa_initial": self.kappa_initial,
            "eps": [self.eps[i] for i in range(self.n_eps)], "t_bad": self.t_bad,
            "flags": [v for b, v in FLAG_NAMES.items() if self.flags & b],
            "passes": self.passes, "columns_seen": self.columns_seen,
            "orth_defect": self.orth_defect,
        }


_P4 = ctypes.c_void_p * 4
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"qsketch: {LIB_PATH} is not built; run `python -m paper_2404_14783_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.qsketch_config_default.argtypes = [ctypes.POINTER(QskConfig)]
    lib.qsketch_config_default.restype = None
    lib.qsketch_init.argtypes = [ctypes.POINTER(QskConfig), vp, ctypes.POINTER(vp)]
    lib.qsketch_init.restype = i32
    lib.qsketch_update.argtypes = [vp, i64, i64, _P4, i64]
    lib.qsketch_update.restype = i32
    lib.qsketch_update_many.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                        ctypes.POINTER(vp), ctypes.POINTER(i64)]
    lib.qsketch_update_many.restype = i32
    lib.qsketch_update_linear.argtypes = [vp, ctypes.c_double, ctypes.c_double, i64, i64, _P4, i64]
    lib.qsketch_update_linear.restype = i32
    lib.qsketch_update_block.argtypes = [vp, i64, i64, i64, i64, _P4, i64]
    lib.qsketch_update_block.restype = i32
    lib.qsketch_scale.argtypes = [vp, ctypes.c_double]
    lib.qsketch_scale.restype = i32
    lib.qsketch_set_sketches.argtypes = [vp, vp, i64, vp, i64, i64]
    lib.qsketch_set_sketches.restype = i32
    lib.qsketch_finalize.argtypes = [vp, i32, _P4, i64, vp, i64, ctypes.POINTER(QskReport)]
    lib.qsketch_truncate.argtypes = [vp, _P4, i64, _P4, i64, i32, _P4, i64, vp, _P4, i64]
    lib.qsketch_truncate.restype = i32
    lib.qsketch_project.argtypes = [vp, _P4, i64, i64, i64, _P4, i64, _P4, i64]
    lib.qsketch_project.restype = i32
    lib.qsketch_project_noalloc.argtypes = [vp, _P4, i64, i64, i64, _P4, i64, _P4, i64]
    lib.qsketch_project_noalloc.restype = i32
    lib.qsketch_finalize.restype = i32
    lib.qsketch_finalize_pair.argtypes = [vp, i32, _P4, i64, vp, i64, ctypes.POINTER(QskReport),
                                          i32, _P4, i64, vp, i64, ctypes.POINTER(QskReport)]
    lib.qsketch_finalize_pair.restype = i32
    lib.qsketch_sketches.argtypes = [vp, _P4, i64, vp, i64]
    lib.qsketch_sketches.restype = i32
    lib.qsketch_reset.argtypes = [vp]
    lib.qsketch_reset.restype = i32
    lib.qsketch_rel_error.argtypes = [vp, _P4, i64, _P4, i64, _P4, i64, ctypes.POINTER(ctypes.c_double)]
    lib.qsketch_rel_error.restype = i32
    lib.qsketch_set_timing.argtypes = [vp, i32]
    lib.qsketch_set_timing.restype = i32
    lib.qsketch_get_timing.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.qsketch_get_timing.restype = i32
    lib.qsketch_stream.argtypes = [vp]
    lib.qsketch_stream.restype = vp
    lib.qsketch_destroy.argtypes = [vp]
    lib.qsketch_destroy.restype = None
    lib.qsketch_strerror.argtypes = [i32]
    lib.qsketch_strerror.restype = ctypes.c_char_p
    lib.qsketch_last_error.argtypes = [vp]
    lib.qsketch_last_error.restype = ctypes.c_char_p
    pp, pi64 = ctypes.POINTER(vp), ctypes.POINTER(i64)
    lib.qsketch_batch_init.argtypes = [i32, ctypes.POINTER(QskConfig), vp, ctypes.POINTER(vp)]
    lib.qsketch_batch_init.restype = i32
    lib.qsketch_batch_run.argtypes = [vp, i32, pp, pi64, pp, pi64, pp, pi64, ctypes.POINTER(QskReport)]
    lib.qsketch_batch_run.restype = i32
    lib.qsketch_batch_rel_error.argtypes = [vp, pp, pi64, pp, pi64, pp, pi64, ctypes.POINTER(ctypes.c_double)]
    lib.qsketch_batch_rel_error.restype = i32
    lib.qsketch_batch_autotune.argtypes = [vp, pp, pi64, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                           ctypes.POINTER(i32)]
    lib.qsketch_batch_autotune.restype = i32
    lib.qsketch_batch_set_exec.argtypes = [vp, i32]
    lib.qsketch_batch_set_exec.restype = i32
    lib.qsketch_batch_destroy.argtypes = [vp]
    lib.qsketch_batch_destroy.restype = None
    lib.qsketch_batch_last_error.argtypes = [vp]
    lib.qsketch_batch_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def header_functions():
    """Names of the functions declared in include/qsketch.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(qsketch_[a-z_]+)\s*\(", text)))


class QSketchError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"qsketch status {status}: {msg}")
        self.status = status


def qempty(planes, rows, cols, dtype, device):
    """Tensor (planes, rows, cols) with column-major planes."""
    return torch.empty((planes, cols, rows), dtype=dtype, device=device).transpose(1, 2)


def qzeros(planes, rows, cols, dtype, device):
    return torch.zeros((planes, cols, rows), dtype=dtype, device=device).transpose(1, 2)


def to_colmajor(t):
    """Copy of a (P, rows, cols) tensor with column-major planes (no copy if it has them)."""
    if t.stride(1) == 1 and t.stride(2) >= t.shape[1]:
        return t
    return t.transpose(1, 2).contiguous().transpose(1, 2)


def _plane_ptrs(t, pure):
    if t.dim() != 3 or t.stride(1) != 1:
        raise ValueError("quaternion tensor must be (P, rows, cols) with column-major planes")
    ld = t.stride(2) if t.shape[2] > 1 else max(t.shape[1], 1)
    if pure:
        if t.shape[0] != 3:
            raise ValueError("pure quaternion input must have 3 planes (x, y, z)")
        ptrs = [None] + [t[p].data_ptr() for p in range(3)]
    else:
        if t.shape[0] != 4:
            raise ValueError("quaternion input must have 4 planes (w, x, y, z)")
        ptrs = [t[p].data_ptr() for p in range(4)]
    return _P4(*ptrs), ld


class Sketcher:
    """One-pass sketch state (Y, W) of A in Q^{m x n}, on the current CUDA
    (HIP) device and stream."""

    def __init__(self, m, n, k, l, seed=0, embedding="gaussian", input_dtype="f64",
                 sketch_dtype="f64", pure=False, split_terms=1, n_correction=3, n_power=3,
                 max_block_cols=0, y_only=False, embedding_round="f64", coalesce_cols=0, stream=None):
        lib = _load()
        cfg = QskConfig()
        lib.qsketch_config_default(ctypes.byref(cfg))
        cfg.m, cfg.n, cfg.k, cfg.l = int(m), int(n), int(k), int(l)
        cfg.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
        cfg.embedding = EMBEDDINGS[embedding]
        cfg.input_dtype = DTYPES[input_dtype]
        cfg.sketch_dtype = DTYPES[sketch_dtype]
        cfg.pure = 1 if pure else 0
        cfg.split_terms = int(split_terms)
        cfg.n_correction = int(n_correction)
        cfg.n_power = int(n_power)
        cfg.max_block_cols = int(max_block_cols)
        cfg.y_only = 1 if y_only else 0
        cfg.embedding_round = DTYPES[embedding_round]
        cfg.coalesce_cols = int(coalesce_cols)
        self.y_only = bool(y_only)
        self.m, self.n, self.k, self.l = cfg.m, cfg.n, cfg.k, cfg.l
        self.pure = bool(pure)
        self.input_dtype = input_dtype
        self.sketch_dtype = sketch_dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._config = dict(m=self.m, n=self.n, k=self.k, l=self.l, seed=int(seed), embedding=embedding,
                            input_dtype=input_dtype, sketch_dtype=sketch_dtype, pure=self.pure,
                            split_terms=int(split_terms), n_correction=int(n_correction),
                            n_power=int(n_power), max_block_cols=int(max_block_cols),
                            y_only=bool(y_only), embedding_round=embedding_round,
                            coalesce_cols=int(coalesce_cols))
        self.columns_seen = 0
        self._ctx = ctypes.c_void_p()
        st = lib.qsketch_init(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                              ctypes.byref(self._ctx))
        if st != QSK_OK:
            raise QSketchError(st, lib.qsketch_strerror(st).decode())
        self._lib = lib

    def _check(self, st):
        if st != QSK_OK:
            msg = self._lib.qsketch_last_error(self._ctx).decode() or self._lib.qsketch_strerror(st).decode()
            raise QSketchError(st, msg)

    def update(self, col0, block, theta=1.0, eta=1.0):
        """A <- theta A + eta H with H = block on columns col0 : col0 + ncols
        (planes column-major, input dtype); the defaults give A[:, J] += block."""
        if block.dtype != TORCH_DTYPE[self.input_dtype]:
            raise TypeError(f"block dtype {block.dtype} != input dtype {self.input_dtype}")
        ptrs, ld = _plane_ptrs(block, self.pure)
        if theta == 1.0 and eta == 1.0:
            self._check(self._lib.qsketch_update(self._ctx, int(col0), int(block.shape[2]), ptrs, ld))
        else:
            self._check(self._lib.qsketch_update_linear(self._ctx, float(theta), float(eta), int(col0),
                                                        int(block.shape[2]), ptrs, ld))
        self.columns_seen += int(block.shape[2])

    def update_many(self, col0s, blocks):
        """The updates A[:, c0 : c0 + ncols] += block for the pairs of col0s
        and blocks, in order, as one HIP graph (captured on the first call
        with these arguments, replayed on later calls with the same tensors)."""
        n = len(blocks)
        if n != len(col0s) or n < 1:
            raise ValueError("one column offset per block")
        c0 = (ctypes.c_int64 * n)(*[int(c) for c in col0s])
        nc = (ctypes.c_int64 * n)()
        lds = (ctypes.c_int64 * n)()
        ptrs = (ctypes.c_void_p * (4 * n))()
        for i, b in enumerate(blocks):
            if b.dtype != TORCH_DTYPE[self.input_dtype]:
                raise TypeError(f"block dtype {b.dtype} != input dtype {self.input_dtype}")
            p4, ld = _plane_ptrs(b, self.pure)
            for q in range(4):
                ptrs[4 * i + q] = p4[q]
            nc[i] = int(b.shape[2])
            lds[i] = ld
        self._check(self._lib.qsketch_update_many(self._ctx, n, c0, nc, ptrs, lds))
        self.columns_seen += sum(int(b.shape[2]) for b in blocks)

    def update_block(self, row0, col0, block):
        """A[row0 : row0 + nrows, col0 : col0 + ncols] += block."""
        if block.dtype != TORCH_DTYPE[self.input_dtype]:
            raise TypeError(f"block dtype {block.dtype} != input dtype {self.input_dtype}")
        ptrs, ld = _plane_ptrs(block, self.pure)
        self._check(self._lib.qsketch_update_block(self._ctx, int(row0), int(block.shape[1]), int(col0),
                                                   int(block.shape[2]), ptrs, ld))
        self.columns_seen += int(block.shape[2])

    def scale(self, theta):
        """A <- theta A."""
        self._check(self._lib.qsketch_scale(self._ctx, float(theta)))

    def set_sketches(self, y=None, w=None, columns_seen=0):
        """Load Y (4, m, k) and/or W (4, l, n) FP64 device planes."""
        def ptrs(t, rows):
            if t is None:
                return None, rows
            if t.dtype != torch.float64 or tuple(t.shape[1:]) != (rows, t.shape[2]):
                raise ValueError("sketch planes must be FP64 (4, rows, cols)")
            p, ld = _plane_ptrs(t, False)
            return ctypes.cast(p, ctypes.c_void_p), ld
        if w is not None and tuple(w.shape) != (4, self.l, self.n):
            raise ValueError("W must be (4, l, n)")
        if y is not None and tuple(y.shape) != (4, self.m, self.k):
            raise ValueError("Y must be (4, m, k)")
        yp, ldy = ptrs(y, self.m)
        wp, ldw = ptrs(w, self.l)
        self._check(self._lib.qsketch_set_sketches(self._ctx, yp, ldy, wp, ldw, int(columns_seen)))
        self.stream.synchronize()
        self.columns_seen = int(columns_seen)

    def config(self):
        """The configuration a restored context must be created with."""
        return dict(self._config)

    def checkpoint(self):
        """Host copy of the sketch state: {'config', 'Y', 'W', 'columns_seen'}
        (Y, W as FP64 CPU tensors)."""
        y, w = self.sketches()
        return {"config": self.config(), "Y": y.cpu(), "W": None if w is None else w.cpu(),
                "columns_seen": self.columns_seen}

    @classmethod
    def restore(cls, state, stream=None):
        """A new context with the checkpoint's configuration and sketches."""
        sk = cls(**state["config"], stream=stream)
        y = to_colmajor(state["Y"].to(sk.device))
        w = None if state["W"] is None else to_colmajor(state["W"].to(sk.device))
        sk.set_sketches(y, w, state["columns_seen"])
        return sk

    def finalize(self, rangefinder="pseudo_qr", q=None, x=None, solve=None):
        """QB stage: returns (Q, X, report) with Q (4, m, k) and X (4, k, n)
        FP64; solve=False (the default in a y_only context) runs the
        rangefinder only and returns X = None."""
        if solve is None:
            solve = not self.y_only
        if q is None:
            q = qempty(4, self.m, self.k, torch.float64, self.device)
        qp, ldq = _plane_ptrs(q, False)
        xarg, ldx = None, self.k
        if solve:
            if x is None:
                x = qempty(4, self.k, self.n, torch.float64, self.device)
            xp, ldx = _plane_ptrs(x, False)
            xarg = ctypes.cast(xp, ctypes.c_void_p)
        else:
            x = None
        rep = QskReport()
        self._check(self._lib.qsketch_finalize(self._ctx, RANGEFINDERS[rangefinder], qp, ldq, xarg, ldx,
                                               ctypes.byref(rep)))
        return q, x, rep.as_dict()

    def _qb_outputs(self, q, x, solve):
        if q is None:
            q = qempty(4, self.m, self.k, torch.float64, self.device)
        qp, ldq = _plane_ptrs(q, False)
        xarg, ldx = None, self.k
        if solve:
            if x is None:
                x = qempty(4, self.k, self.n, torch.float64, self.device)
            xp, ldx = _plane_ptrs(x, False)
            xarg = ctypes.cast(xp, ctypes.c_void_p)
        else:
            x = None
        return q, x, qp, ldq, xarg, ldx

    def finalize_pair(self, rangefinders=("pseudo_qr", "pseudo_svd"), outputs=None, solve=None):
        """Two QB stages side by side on the device (qsketch_finalize_pair):
        the results of finalize(rangefinders[0]) and finalize(rangefinders[1]),
        as a list of two (Q, X, report); outputs: optional [(q, x), (q, x)]."""
        if solve is None:
            solve = not self.y_only
        outputs = outputs or [(None, None), (None, None)]
        a = self._qb_outputs(*outputs[0], solve)
        b = self._qb_outputs(*outputs[1], solve)
        ra, rb = QskReport(), QskReport()
        self._check(self._lib.qsketch_finalize_pair(
            self._ctx, RANGEFINDERS[rangefinders[0]], a[2], a[3], a[4], a[5], ctypes.byref(ra),
            RANGEFINDERS[rangefinders[1]], b[2], b[3], b[4], b[5], ctypes.byref(rb)))
        return [(a[0], a[1], ra.as_dict()), (b[0], b[1], rb.as_dict())]

    def truncate(self, q, x, r):
        """Truncation stage: (Q U_r (4, m, r), sigma (r,), V_r (4, n, r)) with
        Q X ~= (Q U_r) diag(sigma) V_r^*."""
        hu = qempty(4, self.m, r, torch.float64, self.device)
        v = qempty(4, self.n, r, torch.float64, self.device)
        sig = torch.empty(r, dtype=torch.float64, device=self.device)
        qp, ldq = _plane_ptrs(q, False)
        xp, ldx = _plane_ptrs(x, False)
        hp, ldh = _plane_ptrs(hu, False)
        vp_, ldv = _plane_ptrs(v, False)
        self._check(self._lib.qsketch_truncate(self._ctx, qp, ldq, xp, ldx, int(r), hp, ldh,
                                               ctypes.c_void_p(sig.data_ptr()), vp_, ldv))
        return hu, sig, v

    def project(self, col0, block, q, x=None, noalloc=False):
        """Second pass of the two-pass variant: X[:, J] = Q^* block for the
        columns J = col0 .. col0 + ncols - 1; X (4, k, n) FP64 is created
        (zeros) when not given.  Returns X.  noalloc=True calls
        qsketch_project_noalloc (no device allocation in the library)."""
        if block.dtype != TORCH_DTYPE[self.input_dtype]:
            raise TypeError(f"block dtype {block.dtype} != input dtype {self.input_dtype}")
        if x is None:
            x = qzeros(4, self.k, self.n, torch.float64, self.device)
        bp, ld = _plane_ptrs(block, self.pure)
        qp, ldq = _plane_ptrs(q, False)
        xp, ldx = _plane_ptrs(x, False)
        fn = self._lib.qsketch_project_noalloc if noalloc else self._lib.qsketch_project
        self._check(fn(self._ctx, qp, ldq, int(col0), int(block.shape[2]), bp, ld, xp, ldx))
        return x

    def sketches(self):
        """(Y, W) as FP64 (4, m, k) and (4, l, n); W is None in a y_only context."""
        y = qempty(4, self.m, self.k, torch.float64, self.device)
        yp, ldy = _plane_ptrs(y, False)
        w, wp, ldw = None, None, self.l
        if not self.y_only:
            w = qempty(4, self.l, self.n, torch.float64, self.device)
            wp, ldw = _plane_ptrs(w, False)
            wp = ctypes.cast(wp, ctypes.c_void_p)
        self._check(self._lib.qsketch_sketches(self._ctx, yp, ldy, wp, ldw))
        return y, w

    def reset(self):
        self._check(self._lib.qsketch_reset(self._ctx))
        self.columns_seen = 0

    def rel_error(self, a, q, x):
        ap, lda = _plane_ptrs(a, self.pure)
        qp, ldq = _plane_ptrs(q, False)
        xp, ldx = _plane_ptrs(x, False)
        out = ctypes.c_double()
        self._check(self._lib.qsketch_rel_error(self._ctx, ap, lda, qp, ldq, xp, ldx, ctypes.byref(out)))
        return out.value

    def set_timing(self, enable=True):
        self._check(self._lib.qsketch_set_timing(self._ctx, 1 if enable else 0))

    def timing(self):
        """{kernel: (total_ms, launches)} for stage / y / w / w_reduce."""
        out = {}
        for i, name in enumerate(("stage", "y", "w", "w_reduce")):
            ms = ctypes.c_double()
            n = ctypes.c_int64()
            self._check(self._lib.qsketch_get_timing(self._ctx, i, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (ms.value, n.value)
        return out

    def close(self):
        if self._ctx:
            self._lib.qsketch_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _config(m, n, k, l, seed=0, embedding="gaussian", input_dtype="f32", sketch_dtype="bf16",
            pure=False, split_terms=1, n_correction=3, n_power=3, max_block_cols=0):
    lib = _load()
    cfg = QskConfig()
    lib.qsketch_config_default(ctypes.byref(cfg))
    cfg.m, cfg.n, cfg.k, cfg.l = int(m), int(n), int(k), int(l)
    cfg.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    cfg.embedding = EMBEDDINGS[embedding]
    cfg.input_dtype = DTYPES[input_dtype]
    cfg.sketch_dtype = DTYPES[sketch_dtype]
    cfg.pure = 1 if pure else 0
    cfg.split_terms = int(split_terms)
    cfg.n_correction = int(n_correction)
    cfg.n_power = int(n_power)
    cfg.max_block_cols = int(max_block_cols)
    return cfg


class Batch:
    """Independent problems run together (qsketch_batch_*): ``shapes`` is a list
    of (m, n, k, l, seed); the remaining settings are common."""

    def __init__(self, shapes, embedding="gaussian", input_dtype="f32", sketch_dtype="bf16",
                 pure=False, split_terms=1, n_correction=3, n_power=3, stream=None):
        lib = _load()
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        cfgs = (QskConfig * len(self.shapes))()
        for i, (m, n, k, l, seed) in enumerate(self.shapes):
            cfgs[i] = _config(m, n, k, l, seed, embedding, input_dtype, sketch_dtype, pure,
                              split_terms, n_correction, n_power)
        self.count = len(self.shapes)
        self.pure = bool(pure)
        self.input_dtype = input_dtype
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._b = ctypes.c_void_p()
        st = lib.qsketch_batch_init(self.count, cfgs, ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(self._b))
        if st != QSK_OK:
            raise QSketchError(st, lib.qsketch_strerror(st).decode())
        self._lib = lib

    def _check(self, st):
        if st != QSK_OK:
            msg = self._lib.qsketch_batch_last_error(self._b).decode() or self._lib.qsketch_strerror(st).decode()
            raise QSketchError(st, msg)

    def _ptr_tables(self, mats):
        n = self.count
        ptrs = (ctypes.c_void_p * (4 * n))()
        lds = (ctypes.c_int64 * n)()
        for i, t in enumerate(mats):
            p4, ld = _plane_ptrs(t, self.pure and t.shape[0] == 3)
            for q in range(4):
                ptrs[4 * i + q] = p4[q]
            lds[i] = ld
        return ptrs, lds

    def outputs(self):
        qs_ = [qempty(4, m, k, torch.float64, self.device) for (m, n, k, l, s) in self.shapes]
        xs_ = [qempty(4, k, n, torch.float64, self.device) for (m, n, k, l, s) in self.shapes]
        return qs_, xs_

    def run(self, mats, rangefinder="pseudo_qr", outputs=None):
        """One-pass approximation of every matrix in ``mats`` (list of (4 or 3,
        m, n) column-major device tensors); returns (Qs, Xs, reports)."""
        if len(mats) != self.count:
            raise ValueError("one matrix per problem")
        for t in mats:
            if t.dtype != TORCH_DTYPE[self.input_dtype]:
                raise TypeError(f"dtype {t.dtype} != input dtype {self.input_dtype}")
        qs_, xs_ = outputs if outputs is not None else self.outputs()
        ap, ald = self._ptr_tables(mats)
        qp, qld = self._ptr_tables(qs_)
        xp, xld = self._ptr_tables(xs_)
        reps = (QskReport * self.count)()
        self._check(self._lib.qsketch_batch_run(self._b, RANGEFINDERS[rangefinder], ap, ald, qp, qld,
                                                xp, xld, reps))
        return qs_, xs_, [r.as_dict() for r in reps]

    def autotune(self, mats, reps=3):
        """Time the candidate launch shapes of the grouped sketch launches on
        ``mats`` and keep the fastest (remembered per process, and in the
        file QSK_TUNE_CACHE names); returns (W row tiles, Y column tiles,
        W blocks of the row splits)."""
        ap, ald = self._ptr_tables(mats)
        nmt, nj, wb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self._lib.qsketch_batch_autotune(self._b, ap, ald, reps, ctypes.byref(nmt),
                                                     ctypes.byref(nj), ctypes.byref(wb)))
        return nmt.value, nj.value, wb.value

    EXEC_MODES = {"careful": 0, "stream": 1, "graph": 2}

    def set_exec(self, mode):
        """Execution of run(): 'careful', 'stream' (optimistic launches) or
        'graph' (optimistic, captured once and replayed; the default)."""
        self._check(self._lib.qsketch_batch_set_exec(self._b, self.EXEC_MODES[mode]))

    def rel_error(self, mats, qs_, xs_):
        ap, ald = self._ptr_tables(mats)
        qp, qld = self._ptr_tables(qs_)
        xp, xld = self._ptr_tables(xs_)
        out = (ctypes.c_double * self.count)()
        self._check(self._lib.qsketch_batch_rel_error(self._b, ap, ald, qp, qld, xp, xld, out))
        return list(out)

    def close(self):
        if self._b:
            self._lib.qsketch_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def config_status(**kw):
    """Run qsketch_init's validation on a configuration without a device:
    returns the status for configurations rejected before any HIP call."""
    lib = _load()
    cfg = QskConfig()
    lib.qsketch_config_default(ctypes.byref(cfg))
    for k, v in kw.items():
        setattr(cfg, k, v)
    ctx = ctypes.c_void_p()
    st = lib.qsketch_init(ctypes.byref(cfg), None, ctypes.byref(ctx))
    if st == QSK_OK:
        lib.qsketch_destroy(ctx)
    return st
