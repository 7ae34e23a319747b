"""The C-ABI library without a GPU: it loads, exports every symbol that
include/sw.h declares, builds the same cutoff tables as the oracle, and
rejects invalid parameters before any device work."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(sw_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def swlib():
    from paper_1202_0635_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libswmc.so is not built (run __graft_entry__.build())")
    return _lib


def test_every_declared_symbol_is_exported(swlib):
    lib = ctypes.CDLL(swlib.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    # and the binding declares a signature for each of them
    assert set(names) <= set(swlib.SIGNATURES)


def _lattice(swlib, L, q, model, T, J=1.0, seed=0, reserved=0):
    return swlib.SwLattice(L, q, model, reserved, T, J, seed)


@pytest.mark.parametrize("model,q", [(0, 2), (0, 3), (0, 4), (0, 7), (0, 32), (1, 2), (1, 3), (1, 4),
                                     (1, 5), (1, 6), (1, 12), (1, 32)])
@pytest.mark.parametrize("T", [0.05, 0.9, 1.1345926571065, 3.0])
def test_cutoff_table_equals_oracle(swlib, orc, model, q, T):
    J = 1.0 if q != 3 else 0.7
    p = _lattice(swlib, 16, q, model, T, J)
    n = q * q if model == 0 else q ** 3
    out = np.zeros(n, dtype=np.uint32)
    st = swlib.lib().sw_cutoff_table(ctypes.byref(p), out.ctypes.data_as(ctypes.c_void_p), n)
    assert st == 0
    assert np.array_equal(out, orc.cutoffs(model, q, T, J))


def test_state_bytes_and_invalid_parameters(swlib):
    lib = swlib.lib()
    good = _lattice(swlib, 4096, 2, 0, 1.0)
    n = lib.sw_state_bytes(ctypes.byref(good))
    assert n >= 4096 * 4096 * (1 + 4 + 4) and n % 256 == 0
    bad = [
        _lattice(swlib, 1, 2, 0, 1.0), _lattice(swlib, 65536, 2, 0, 1.0), _lattice(swlib, 16, 1, 0, 1.0),
        _lattice(swlib, 16, 33, 0, 1.0), _lattice(swlib, 16, 2, 2, 1.0), _lattice(swlib, 16, 2, 0, 0.0),
        _lattice(swlib, 16, 2, 0, -1.0), _lattice(swlib, 16, 2, 0, math.inf), _lattice(swlib, 16, 2, 0, 1.0, J=0.0),
        _lattice(swlib, 16, 2, 0, 1.0, reserved=1),
    ]
    for p in bad:
        assert lib.sw_state_bytes(ctypes.byref(p)) == 0
        ctx = ctypes.c_void_p()
        assert lib.sw_init(ctypes.byref(p), None, 0, None, ctypes.byref(ctx)) == swlib.SW_EINVAL
        assert not ctx.value
        assert lib.sw_last_error()  # a reason is given
    # a caller buffer that is unaligned or too small is rejected before device work
    ctx = ctypes.c_void_p()
    assert lib.sw_init(ctypes.byref(good), ctypes.c_void_p(0x1001), n, None, ctypes.byref(ctx)) == swlib.SW_EINVAL
    assert lib.sw_init(ctypes.byref(good), ctypes.c_void_p(0x1000), n - 256, None, ctypes.byref(ctx)) == swlib.SW_ENOMEM
    # wrong table size
    out = np.zeros(3, dtype=np.uint32)
    assert lib.sw_cutoff_table(ctypes.byref(good), out.ctypes.data_as(ctypes.c_void_p), 3) == swlib.SW_EINVAL


def test_null_context_calls_fail_cleanly(swlib):
    lib = swlib.lib()
    assert lib.sw_sweep(None, 1, 0) == swlib.SW_EINVAL
    assert lib.sw_measure(None, None) == swlib.SW_EINVAL
    assert lib.sw_read_spins(None, None, 0) == swlib.SW_EINVAL
    lib.sw_free(None)
    for st in (0, -1, -2, -3, -4, -5, -6, 7):
        assert lib.sw_strerror(st)


def test_static_entry_rejects_before_device_work(swlib):
    """sw_sweep_static checks its arguments before any HIP call (no GPU here)."""
    lib = swlib.lib()
    dummy = ctypes.c_void_p(0x1000)
    big = _lattice(swlib, 1025, 2, 0, 1.0)
    assert lib.sw_sweep_static(ctypes.byref(big), dummy, 0, 1, dummy, None, None, None) == swlib.SW_EINVAL
    assert b"1024" in lib.sw_last_error()
    ok = _lattice(swlib, 64, 2, 0, 1.0)
    assert lib.sw_sweep_static(ctypes.byref(ok), None, 0, 1, dummy, None, None, None) == swlib.SW_EINVAL
    assert lib.sw_sweep_static(ctypes.byref(ok), dummy, 0, -1, dummy, None, None, None) == swlib.SW_EINVAL
    assert lib.sw_sweep_static(ctypes.byref(ok), dummy, 0, 0, dummy, dummy, None, None) == swlib.SW_EINVAL
    bad = _lattice(swlib, 64, 1, 0, 1.0)
    assert lib.sw_sweep_static(ctypes.byref(bad), dummy, 0, 1, dummy, None, None, None) == swlib.SW_EINVAL
    assert lib.sw_sweep_static(ctypes.byref(ok), ctypes.c_void_p(0x1001), 0, 1, dummy, None, None, None) == swlib.SW_EINVAL


def test_side_limits(swlib):
    """Single lattices take L up to 65535 (two-level labels); batches and the
    static entry point keep one-level label words and stop at 46340."""
    lib = swlib.lib()
    wide = _lattice(swlib, 65535, 2, 0, 1.0)
    assert lib.sw_state_bytes(ctypes.byref(wide)) > 65535 * 65535 * 4
    over = _lattice(swlib, 46341, 2, 0, 1.0)
    assert lib.sw_state_bytes(ctypes.byref(over)) > 0
    assert lib.sw_batch_bytes(ctypes.byref(over), 1) == 0
    dummy = ctypes.c_void_p(0x1000)
    assert lib.sw_sweep_static(ctypes.byref(over), dummy, 0, 1, dummy, None, None, None) == swlib.SW_EINVAL
