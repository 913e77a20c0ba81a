"""The C-ABI library loads, exports every symbol include/rewl.h declares, and
validates arguments on the host (no GPU needed for any of this)."""
import ctypes as C
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rewl.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(rewl_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


def _lib():
    import paper_1508_02748_amd as R
    if not os.path.exists(R.LIB_PATH):
        pytest.skip("librewl.so not built")
    return R, R.lib()


def test_every_declared_symbol_is_exported():
    R, L = _lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


def test_plan_validation_and_windows_on_host():
    R, L = _lib()
    from oracle.rewl import window

    def create(**kw):
        p = R.Problem(**kw)
        h = C.c_void_p()
        arr = (R._Problem * 1)(p._c())
        return L.rewl_plan_create(arr, 1, None, C.byref(h)), h

    for bad in (dict(L=5), dict(L=2), dict(L=66), dict(L=16, n_windows=0), dict(L=16, overlap=(4, 4)),
                dict(L=16, walkers_per_window=0), dict(L=16, walkers_per_window=257), dict(L=16, k_final=41),
                dict(L=16, flat=(6, 5)), dict(L=16, interval=0), dict(L=16, interval=2 ** 30 + 1), dict(L=16, init=2),
                dict(L=16, overlap=(-1, 4)), dict(L=16, flat=(1, 0)), dict(L=16, stage_sync=2)):
        st, h = create(**bad)
        assert st == R.REWL_EINVAL, bad
        assert L.rewl_last_error()
    st, h = create(L=16, n_windows=8, walkers_per_window=4)
    assert st == R.REWL_OK
    try:
        for w in range(8):
            lo, hi = C.c_int32(), C.c_int32()
            assert L.rewl_window_bounds(h, 0, w, C.byref(lo), C.byref(hi)) == 0
            assert (lo.value, hi.value) == window(256, 8, 3, 4, w)
        sizes = (C.c_size_t * 3)()
        assert L.rewl_plan_buffer_sizes(h, sizes) == 0
        # ln g (8 bytes per bin) and stage base (4 bytes) tables in 4x4 tiles of (e, m), 4 walkers per window
        tiles = sum(-(-(window(256, 8, 3, 4, w)[1] - window(256, 8, 3, 4, w)[0] + 1) // 4) * -(-257 // 4)
                    for w in range(8))
        bins = tiles * 16 * 4
        assert sizes[0] >= bins * 12 and sizes[0] < bins * 12 + 256
        # calls needing device buffers fail cleanly before bind
        assert L.rewl_init(h) == R.REWL_ESTATE
        assert L.rewl_run(h, 1) == R.REWL_ESTATE
    finally:
        L.rewl_plan_destroy(h)


def test_audit_shift_and_fixed_tuning_fields_on_host():
    """audit_shift is 0 (2^30) or 1..30, the interval must fit in one audit period, and neither the
    audit shift nor the table layout of a plan can change after it is created."""
    R, L = _lib()

    def create(tn, interval=64):
        arr = (R._Problem * 1)(R.Problem(L=8, interval=interval)._c())
        h = C.c_void_p()
        return L.rewl_plan_create(arr, 1, C.byref(tn._c()), C.byref(h)), h

    for a, X, ok in ((0, 2 ** 30, True), (30, 2 ** 30, True), (6, 64, True), (6, 65, False), (31, 64, False),
                     (-1, 64, False)):
        st, h = create(R.Tuning(audit_shift=a), X)
        assert (st == R.REWL_OK) == ok, (a, X)
        if st == R.REWL_OK:
            L.rewl_plan_destroy(h)
    st, h = create(R.Tuning(audit_shift=6, table_layout=R.LAYOUT_BAND))
    assert st == R.REWL_OK
    try:
        assert L.rewl_set_tuning(h, C.byref(R.Tuning(audit_shift=6, table_layout=R.LAYOUT_BAND,
                                                      walkers_per_wg=128)._c())) == R.REWL_OK
        assert L.rewl_set_tuning(h, C.byref(R.Tuning(audit_shift=7, table_layout=R.LAYOUT_BAND)._c())) == R.REWL_EINVAL
        assert L.rewl_set_tuning(h, C.byref(R.Tuning(audit_shift=6)._c())) == R.REWL_EINVAL
    finally:
        L.rewl_plan_destroy(h)


def test_packed_layouts_on_host():
    """Packed layouts keep one 8-byte word per bin (against 12 bytes) and need k_final <= 24, an
    interval of at most 2^24 trials and audit_shift <= 24; the band bit applies as in the unpacked
    layouts."""
    R, L = _lib()

    def create(layout, audit_shift=0, **kw):
        q = dict(L=16, n_windows=8, walkers_per_window=4, k_final=20, interval=10_000)
        q.update(kw)
        arr = (R._Problem * 1)(R.Problem(**q)._c())
        h = C.c_void_p()
        tn = R.Tuning(table_layout=layout, audit_shift=audit_shift)
        return L.rewl_plan_create(arr, 1, C.byref(tn._c()), C.byref(h)), h

    def tables(layout):
        st, h = create(layout)
        assert st == R.REWL_OK
        sizes = (C.c_size_t * 3)()
        assert L.rewl_plan_buffer_sizes(h, sizes) == 0
        L.rewl_plan_destroy(h)
        return sizes[0]

    for plain, packed in ((R.LAYOUT_DENSE, R.LAYOUT_DENSE_PACKED), (R.LAYOUT_BAND, R.LAYOUT_BAND_PACKED)):
        a, b = tables(plain), tables(packed)
        assert abs(b * 12 - a * 8) <= 256 * 12, (plain, a, b)
    for layout in (R.LAYOUT_DENSE_PACKED, R.LAYOUT_BAND_PACKED):
        for kw, ok in ((dict(k_final=24), True), (dict(k_final=25), False), (dict(interval=2 ** 24), True),
                       (dict(interval=2 ** 24 + 1), False)):
            st, h = create(layout, **kw)
            assert (st == R.REWL_OK) == ok, (layout, kw)
            if st == R.REWL_OK:
                L.rewl_plan_destroy(h)
        for a, ok in ((24, True), (25, False)):
            st, h = create(layout, audit_shift=a, interval=64)
            assert (st == R.REWL_OK) == ok, (layout, a)
            if st == R.REWL_OK:
                L.rewl_plan_destroy(h)
    st, h = create(4)
    assert st == R.REWL_EINVAL
    st, h = create(R.LAYOUT_BAND_PACKED, split=R.SPLIT_BOTH, m_windows=2, m_overlap=(1, 2))
    assert st == R.REWL_EINVAL


def test_mixed_interval_rejected():
    R, L = _lib()
    arr = (R._Problem * 2)(R.Problem(L=8, interval=100)._c(), R.Problem(L=8, interval=200)._c())
    h = C.c_void_p()
    assert L.rewl_plan_create(arr, 2, None, C.byref(h)) == R.REWL_EINVAL


def test_grid_reweighting_validation_on_host():
    R, L = _lib()
    nb = C.c_size_t()
    assert L.rewl_lnz_grid_workspace_size(1025, 1024, 256, C.byref(nb)) == 0
    assert nb.value == (4 * 1024 * 1025 + 2 * 1024 * 256) * 8
    assert L.rewl_lnz_grid_workspace_size(0, 4, 4, C.byref(nb)) == R.REWL_EINVAL
    fake = C.c_void_p(256)   # never dereferenced: every call below fails validation first
    # geometry outside the lattice, negative sizes, a workspace that is too small, no outputs
    assert L.rewl_lnz_grid_forward(fake, 16, 0, 18, 0, 17, fake, 4, fake, 4, fake, 1 << 20, fake, None) \
        == R.REWL_EINVAL
    assert L.rewl_lnz_grid_forward(fake, 16, 0, 17, 0, 17, fake, -1, fake, 4, fake, 1 << 20, fake, None) \
        == R.REWL_EINVAL
    assert L.rewl_lnz_grid_forward(fake, 16, 0, 17, 0, 17, fake, 4, fake, 4, fake, 8, fake, None) \
        == R.REWL_EINVAL
    assert L.rewl_lnz_grid_backward(fake, 16, 0, 17, 0, 17, fake, 4, fake, 4, fake, None, fake, 1 << 20,
                                    None, None, None, None, None) == R.REWL_EINVAL
    assert L.rewl_lnz_grid_backward(fake, 16, 0, 17, 0, 17, fake, 4, fake, 4, fake, None, fake, 1 << 20,
                                    fake, None, None, None, None) == R.REWL_EINVAL
    assert L.rewl_last_error()


def test_plan_create_fuzz_against_the_window_formula():
    # random problems, valid and not: the host never crashes, rejects exactly the
    # invalid ones, and its windows and table sizes follow the window formula
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies
    R, L = _lib()
    from oracle.rewl import window
    seen = {"ok": 0, "bad": 0}

    @hyp.settings(max_examples=300, deadline=None, derandomize=True)
    @hyp.given(Ls=st.integers(0, 70), nw=st.integers(-1, 80), on=st.integers(-1, 5), od=st.integers(0, 5),
               W=st.integers(0, 260), K=st.integers(-1, 42))
    def check(Ls, nw, on, od, W, K):
        p = R.Problem(L=Ls, n_windows=nw, overlap=(on, od), walkers_per_window=W, k_final=K)
        h = C.c_void_p()
        arr = (R._Problem * 1)(p._c())
        status = L.rewl_plan_create(arr, 1, None, C.byref(h))
        valid = (4 <= Ls <= 64 and Ls % 2 == 0 and nw >= 1 and 1 <= od and 0 <= on < od and 1 <= W <= 256
                 and 0 <= K <= 40)
        N = Ls * Ls
        if valid:
            wins = [window(N, nw, on, od, w) for w in range(nw)]
            valid = all(lo <= hi for lo, hi in wins)
        if not valid:
            assert status == R.REWL_EINVAL and L.rewl_last_error()
            seen["bad"] += 1
            return
        assert status == R.REWL_OK
        seen["ok"] += 1
        try:
            total = 0
            for w, (lo, hi) in enumerate(wins):
                a, b = C.c_int32(), C.c_int32()
                assert L.rewl_window_bounds(h, 0, w, C.byref(a), C.byref(b)) == 0
                assert (a.value, b.value) == (lo, hi)
                total += -(-(hi - lo + 1) // 4) * -(-(N + 1) // 4) * 16 * W
            sizes = (C.c_size_t * 3)()
            assert L.rewl_plan_buffer_sizes(h, sizes) == 0
            assert total * 12 <= sizes[0] < total * 12 + 256
            assert sizes[1] >= nw * W * Ls * ((Ls + 31) // 32) * 4
        finally:
            L.rewl_plan_destroy(h)

    check()
    assert seen["ok"] >= 20 and seen["bad"] >= 20, seen


def test_split_validation_on_host():
    R, L = _lib()
    h = C.c_void_p()
    for bad in (dict(L=8, split=2), dict(L=8, split=-1)):
        arr = (R._Problem * 1)(R.Problem(**bad)._c())
        assert L.rewl_plan_create(arr, 1, None, C.byref(h)) == R.REWL_EINVAL
    arr = (R._Problem * 2)(R.Problem(L=8)._c(), R.Problem(L=8, split=R.SPLIT_MAGNETIZATION)._c())
    assert L.rewl_plan_create(arr, 2, None, C.byref(h)) == R.REWL_EINVAL
    c = R.Problem(L=8)._c()
    c.reserved = 1
    assert L.rewl_plan_create((R._Problem * 1)(c), 1, None, C.byref(h)) == R.REWL_EINVAL
    # magnetization windows: all 65 energy rows by the window's m columns, in 4 x 4 tiles
    arr = (R._Problem * 1)(R.Problem(L=8, n_windows=3, overlap=(1, 2), walkers_per_window=2,
                                     split=R.SPLIT_MAGNETIZATION)._c())
    assert L.rewl_plan_create(arr, 1, None, C.byref(h)) == R.REWL_OK
    try:
        from oracle.rewl import window
        sizes = (C.c_size_t * 3)()
        assert L.rewl_plan_buffer_sizes(h, sizes) == 0
        bins = sum(-(-65 // 4) * -(-(window(64, 3, 1, 2, w)[1] - window(64, 3, 1, 2, w)[0] + 1) // 4) * 16 * 2
                   for w in range(3))
        assert bins * 12 <= sizes[0] < bins * 12 + 256
    finally:
        L.rewl_plan_destroy(h)
