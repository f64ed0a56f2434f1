"""The C-ABI library loads and exports every entry point include/qsketch.h
declares; argument validation that happens before any device call works on
the CPU.  No compute calls (there is no GPU here)."""
import ctypes
import os

import pytest

import paper_2404_14783_amd as qs


def test_library_exports_every_header_symbol():
    lib = qs._load()
    names = qs.header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), f"{name} declared in qsketch.h but not exported"


def test_config_default_and_strerror():
    lib = qs._load()
    cfg = qs.QskConfig()
    lib.qsketch_config_default(ctypes.byref(cfg))
    assert cfg.n_correction == 3 and cfg.n_power == 3 and cfg.split_terms == 1
    assert lib.qsketch_strerror(qs.QSK_E_ARG) == b"invalid argument"
    assert lib.qsketch_last_error(None) == b"null context"
    lib.qsketch_destroy(None)            # no-op


@pytest.mark.parametrize("bad", [
    dict(m=100, n=80, k=10, l=9),           # l < k
    dict(m=100, n=80, k=0, l=9),            # k < 1
    dict(m=100, n=80, k=10, l=81),          # l > n
    dict(m=100, n=80, k=300, l=300),        # k above the supported maximum
    dict(m=0, n=80, k=1, l=1),
    dict(m=100, n=80, k=10, l=21, n_correction=9),
    dict(m=100, n=80, k=10, l=21, sketch_dtype=2, split_terms=4),
    dict(m=100, n=80, k=10, l=21, input_dtype=1, sketch_dtype=4, split_terms=5),   # e4m3 terms: 1..4
    dict(m=100, n=80, k=10, l=21, input_dtype=1, sketch_dtype=4, split_terms=0),
    dict(m=100, n=80, k=10, l=21, input_dtype=1, sketch_dtype=5),
    dict(m=100, n=80, k=10, l=21, embedding=5),
    dict(m=100, n=80, k=10, l=21, y_only=2),
    dict(m=100, n=80, k=10, l=21, embedding_round=4),
    dict(m=100, n=80, k=10, l=21, input_dtype=1, sketch_dtype=2, embedding_round=2),  # only FP64 sketches
    dict(m=100, n=80, k=10, l=21, coalesce_cols=81),
    dict(m=100, n=80, k=10, l=21, coalesce_cols=-1),
])
def test_invalid_configs_rejected_before_device_use(bad):
    assert qs.config_status(**bad) == qs.QSK_E_ARG


def test_unsupported_combinations():
    # FP64 data with a low-precision sketch is not accepted
    assert qs.config_status(m=100, n=80, k=10, l=21, input_dtype=0, sketch_dtype=2) == qs.QSK_E_UNSUPPORTED
    assert qs.config_status(m=100, n=80, k=10, l=21, input_dtype=0, sketch_dtype=4, split_terms=3) == \
        qs.QSK_E_UNSUPPORTED


def test_struct_layouts_match_header():
    # field order/size of the ctypes mirrors (int64 m,n; int32 k,l; uint64 seed; 7 int32;
    # padding; int64 max_block_cols; int32 y_only; int32 embedding_round; int32
    # coalesce_cols; tail padding)
    assert ctypes.sizeof(qs.QskConfig) == 8 + 8 + 4 + 4 + 8 + 7 * 4 + 4 + 8 + 4 + 4 + 4 + 4
    assert qs.QskConfig.max_block_cols.offset == 64 and qs.QskConfig.y_only.offset == 72
    assert qs.QskConfig.embedding_round.offset == 76 and qs.QskConfig.coalesce_cols.offset == 80
    assert ctypes.sizeof(qs.QskReport) == 8 + 8 + 64 + 4 * 4 + 8 + 8
