"""The C-ABI library loads without a GPU and exports every function that
include/bcmg.h declares; calls that touch no device work on the CPU."""
import ctypes as C

import pytest

from paper_2207_14208_amd import _native as N


def test_every_declared_symbol_is_exported():
    names = N.header_functions()
    assert len(names) >= 30
    L = N.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(N.PROTOTYPES), set(names) ^ set(N.PROTOTYPES)


def test_host_only_calls():
    L = N.lib()
    assert L.bcmg_version() >= 100
    o = N.default_options()
    assert (o.nu1, o.nu2, o.coarsest_N, o.ext_iters, o.precision) == (2, 1, 4, 4, N.FP64)
    assert (o.layout, o.cycle, o.smoother, o.check_interval) == (N.LAYOUT_SPLIT, N.CYCLE_V, N.SMOOTH_RB, 1)
    b = C.c_int64()
    N.check(L.bcmg_estimate_bytes(3, 256, N.FP64, C.byref(b)))
    assert b.value > 257 ** 3 * 33
    # argument validation happens on the host before any device call
    h = C.c_void_p()
    for dim, n, kw in [(4, 64, {}), (2, 63, {}), (2, 4, {}), (3, 2048, {}), (2, 64, {"ext_iters": 0}),
                       (2, 64, {"coarsest_N": 2}), (2, 64, {"max_cycles": 0}), (2, 64, {"precision": 7}),
                       (2, 64, {"layout": 2}), (2, 64, {"cycle": 2}), (2, 64, {"smoother": 2}),
                       (2, 64, {"check_interval": 0}), (2, 64, {"check_interval": 17})]:
        o = N.default_options(**kw)
        st = L.bcmg_setup(dim, n, C.c_void_p(16), C.byref(o), None, C.byref(h))
        assert st == N.ERR_INVALID, (dim, n, kw)
        assert L.bcmg_last_error().decode()
    st = L.bcmg_setup(2, 64, None, None, None, C.byref(h))
    assert st == N.ERR_INVALID


def test_unknown_option_rejected():
    with pytest.raises(TypeError):
        N.default_options(bogus=1)


def test_set_allocator_arguments():
    """bcmg_set_allocator takes both callbacks or neither (host-only call)."""
    L = N.lib()
    cb_a = N.ALLOC_FN(lambda n, s, c: None)
    cb_f = N.FREE_FN(lambda p, n, s, c: None)
    a = C.cast(cb_a, C.c_void_p)
    f = C.cast(cb_f, C.c_void_p)
    assert L.bcmg_set_allocator(a, None, None) == N.ERR_INVALID
    assert L.bcmg_set_allocator(None, f, None) == N.ERR_INVALID
    assert L.bcmg_set_allocator(a, f, None) == N.OK
    assert L.bcmg_set_allocator(None, None, None) == N.OK
