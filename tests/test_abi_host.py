"""Host-side checks of libks: it loads, exports every symbol of include/ks.h, and
its planner (argument checks, level schedule, workspace layout) behaves, all
without a GPU (no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_2502_11686_amd import ks

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "ks.h")).read()
    return sorted(set(re.findall(r"\b(ks_[a-z_0-9]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    L = ks.lib()
    decl = header_symbols()
    assert decl, "no declarations found"
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(ks.SYMBOLS) == decl


def test_status_strings():
    L = ks.lib()
    for st in range(-8, 1):
        assert L.ks_status_string(st)


@pytest.mark.parametrize("k,n,m", [(0, 2, 2), (1000, 4, 2), (100000, 6, 3), (77, 3, 6)])
def test_layout_matches_level_schedule(k, n, m):
    """Level l has floor((k+1)/2^l) columns, ceil(N_l/2) R records; every column
    is eliminated exactly once at level ctz(i+1)."""
    plan = ks.Plan.__new__(ks.Plan)  # host-only: create a plan on a fake aligned address
    d = ks.make_desc(k, n, m, True, True)
    nbytes = ks.workspace_bytes(k, n, m, True, True)
    assert nbytes > 0 and nbytes % 256 == 0
    h = ctypes.c_void_p()
    st = ks.lib().ks_create(ctypes.byref(d), ctypes.c_void_p(1 << 20), nbytes, None, ctypes.byref(h))
    assert st == ks.KS_OK
    lay = ks.Layout()
    assert ks.lib().ks_plan_layout(h, ctypes.byref(lay)) == ks.KS_OK
    ks.lib().ks_destroy(h)
    N, l, rec = k + 1, 0, 0
    while True:
        assert lay.level_columns[l] == N
        assert lay.level_rec_offset[l] == rec
        rec += (N + 1) // 2
        if N == 1:
            break
        N //= 2
        l += 1
    assert lay.levels == l + 1 == (k + 1).bit_length()
    assert rec == k + 1
    assert lay.rrow_stride == n * (3 * n + 1)
    # brute force: elimination level of each column is ctz(i+1)
    lv = [((i + 1) & -(i + 1)).bit_length() - 1 for i in range(min(k + 1, 5000))]
    for i, li in enumerate(lv):
        j = (i + 1) // (1 << li) - 1
        assert j % 2 == 0 and j < lay.level_columns[li]


def test_argument_errors():
    L = ks.lib()
    h = ctypes.c_void_p()
    bad = [ks.make_desc(-1, 2, 1, True, True), ks.make_desc(10, 0, 1, True, True),
           ks.make_desc(10, 2, -1, True, True), ks.make_desc(10, 7, 3, True, True)]
    for d in bad:
        assert L.ks_workspace_bytes(ctypes.byref(d)) == 0
        assert L.ks_create(ctypes.byref(d), ctypes.c_void_p(1 << 20), 1 << 30, None, ctypes.byref(h)) == ks.KS_E_ARG
    d = ks.make_desc(10, 2, 1, True, True)
    nb = ks.workspace_bytes(10, 2, 1, True, True)
    assert L.ks_create(ctypes.byref(d), None, nb, None, ctypes.byref(h)) == ks.KS_E_WORKSPACE
    assert L.ks_create(ctypes.byref(d), ctypes.c_void_p((1 << 20) + 8), nb, None, ctypes.byref(h)) == ks.KS_E_WORKSPACE
    assert L.ks_create(ctypes.byref(d), ctypes.c_void_p(1 << 20), nb - 256, None, ctypes.byref(h)) == ks.KS_E_WORKSPACE
    assert L.ks_covariances(None, None) == ks.KS_E_ARG
    assert L.ks_destroy(None) == ks.KS_E_ARG


def _fake_io(with_cov=True):
    # distinct non-null addresses; submit is host-only and never dereferences them
    return ks.Io(*[ctypes.c_void_p(0x10000 * (i + 1)) for i in range(8)],
                 ctypes.c_void_p(0x100000) if with_cov else None)


def test_engine_admission_is_exact_footprint_first_fit():
    """Admission by device footprint: each request holds exactly its single-plan
    workspace (rounded to 256 B); requests that do not fit now are refused with
    KS_E_BUSY, ones that can never fit with KS_E_WORKSPACE; submit launches
    nothing (host-only)."""
    L = ks.lib()
    ws = 64 << 20
    h = ctypes.c_void_p()
    assert L.ks_engine_create(ctypes.c_void_p(1 << 30), ws, None, ctypes.byref(h)) == ks.KS_OK
    st = ks.EngineStats()
    assert L.ks_engine_query(h, ctypes.byref(st)) == ks.KS_OK
    region = st.region_bytes
    assert st.free_bytes == region == st.largest_free and region <= ws - ws // 16
    shape = (20000, 6, 3, False, False, False)
    fp = ks.Engine.footprint(shape)
    assert fp == (ks.workspace_bytes(*shape) + 255) // 256 * 256
    d = ks.make_desc(*shape)
    io = _fake_io()
    tickets = []
    while True:
        t = ctypes.c_uint64()
        r = L.ks_engine_submit(h, ctypes.byref(d), ctypes.byref(io), 1, ctypes.byref(t))
        if r == ks.KS_E_BUSY:
            break
        assert r == ks.KS_OK
        tickets.append(t.value)
    assert len(tickets) == region // fp
    assert tickets == list(range(1, len(tickets) + 1))
    assert L.ks_engine_query(h, ctypes.byref(st)) == ks.KS_OK
    assert st.inflight == len(tickets) and st.free_bytes == region - len(tickets) * fp
    # a smaller request still fits in what is left
    small = (100, 6, 3, False, False, False)
    if region - len(tickets) * fp >= ks.Engine.footprint(small):
        t = ctypes.c_uint64()
        ds = ks.make_desc(*small)
        assert L.ks_engine_submit(h, ctypes.byref(ds), ctypes.byref(io), 1, ctypes.byref(t)) == ks.KS_OK
    # never fits
    big = ks.make_desc(10_000_000, 6, 3, False, False)
    t = ctypes.c_uint64()
    assert L.ks_engine_submit(h, ctypes.byref(big), ctypes.byref(io), 1, ctypes.byref(t)) == ks.KS_E_WORKSPACE
    # argument errors
    bad = ks.make_desc(100, 7, 3, False, False)
    assert L.ks_engine_submit(h, ctypes.byref(bad), ctypes.byref(io), 1, ctypes.byref(t)) == ks.KS_E_ARG
    nocov = _fake_io(with_cov=False)
    assert L.ks_engine_submit(h, ctypes.byref(d), ctypes.byref(nocov), 1, ctypes.byref(t)) == ks.KS_E_ARG
    cnt = ctypes.c_int32()
    assert L.ks_engine_retired(h, 0, None, None, ctypes.byref(cnt)) == ks.KS_OK and cnt.value == 0
    res = ctypes.c_int()
    assert L.ks_engine_poll(h, tickets[0], ctypes.byref(res)) == ks.KS_E_BUSY
    assert L.ks_engine_poll(h, 10**9, ctypes.byref(res)) == ks.KS_E_ARG
    assert L.ks_engine_destroy(h) == ks.KS_OK


def test_engine_create_errors():
    L = ks.lib()
    h = ctypes.c_void_p()
    assert L.ks_engine_create(None, 64 << 20, None, ctypes.byref(h)) == ks.KS_E_WORKSPACE
    assert L.ks_engine_create(ctypes.c_void_p((1 << 30) + 8), 64 << 20, None, ctypes.byref(h)) == ks.KS_E_WORKSPACE
    assert L.ks_engine_create(ctypes.c_void_p(1 << 30), 1000, None, ctypes.byref(h)) == ks.KS_E_WORKSPACE
    assert L.ks_engine_create(ctypes.c_void_p(1 << 30), 64 << 20, None, None) == ks.KS_E_ARG


def _fake_plan(k, n, m, fp32=False):
    d = ks.make_desc(k, n, m, True, True, fp32)
    h = ctypes.c_void_p()
    nbytes = ks.workspace_bytes(k, n, m, True, True, fp32)
    assert ks.lib().ks_create(ctypes.byref(d), ctypes.c_void_p(1 << 20), nbytes, None, ctypes.byref(h)) == ks.KS_OK
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert ks.lib().ks_plan_schedule(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == ks.KS_OK
    ks.lib().ks_destroy(h)
    return a.value, b.value, c.value


def test_tuning_table_drives_the_schedule(monkeypatch):
    """The tuning entry of (n, form) decides which top levels run in the tail
    kernels and which levels run in FP32; the environment overrides it."""
    monkeypatch.delenv("KS_TAIL_PASSES", raising=False)
    monkeypatch.delenv("KS_FP32_SWITCH", raising=False)
    saved = ks.get_tuning(5, False), ks.get_tuning(5, True)
    try:
        k, n = 100000, 5  # a class with the wavefront-family backward tail
        L = (k + 1).bit_length() - 1
        ks.set_tuning(n, False, **dict(ks.TUNING_DEFAULTS, fwd_tail_passes=0, bwd_tail_passes=0))
        assert ks.get_tuning(n, False) == dict(ks.TUNING_DEFAULTS, fwd_tail_passes=0, bwd_tail_passes=0)
        assert _fake_plan(k, n, 3) == (0, L, L + 1)          # base level only, no backward tail
        ks.set_tuning(n, False, fwd_tail_passes=10**6, bwd_tail_passes=10**6)
        assert _fake_plan(k, n, 3) == (0, 0, 0)              # everything in the tails
        ks.set_tuning(n, True, **dict(ks.TUNING_DEFAULTS, fp32_switch_columns=4096))
        fp32_levels = sum(1 for l in range(L) if (k + 1) >> l > 4096)
        lev, l0, l1 = _fake_plan(k, n, 3, fp32=True)
        assert lev == fp32_levels and l0 > lev and l1 >= lev
        monkeypatch.setenv("KS_TAIL_PASSES", "0")
        assert _fake_plan(k, n, 3)[1:] == (L, L + 1)
        with pytest.raises(ks.KsError):
            ks.set_tuning(0, False, fwd_tail_passes=1)
        with pytest.raises(ks.KsError):
            ks.set_tuning(5, False, fwd_tail_passes=-1)
    finally:
        monkeypatch.delenv("KS_TAIL_PASSES", raising=False)
        for fp32, e in zip((False, True), saved):
            ks.set_tuning(5, fp32, **e)


def test_level_groups_tuning_round_trip(monkeypatch):
    """Level-group choices are stored per (n, form), validated, and the
    environment overrides them."""
    for v in ("KS_FWD_GROUP", "KS_FWD_GROUP_FROM", "KS_BWD_GROUP", "KS_BWD_GROUP_FROM"):
        monkeypatch.delenv(v, raising=False)
    saved = ks.get_tuning(6, False)
    try:
        ks.set_tuning(6, False, fwd_group=4, fwd_group_from=1, bwd_group=3, bwd_group_from=2)
        t = ks.get_tuning(6, False)
        assert (t["fwd_group"], t["fwd_group_from"], t["bwd_group"], t["bwd_group_from"]) == (4, 1, 3, 2)
        monkeypatch.setenv("KS_FWD_GROUP", "2")
        assert ks.get_tuning(6, False)["fwd_group"] == 2
        for bad in (dict(fwd_group=0), dict(fwd_group=9), dict(bwd_group=0), dict(bwd_group_from=-1)):
            with pytest.raises(ks.KsError):
                ks.set_tuning(6, False, **bad)
    finally:
        monkeypatch.delenv("KS_FWD_GROUP", raising=False)
        ks.set_tuning(6, False, **saved)


def test_static_entry_rejects_oversized_and_invalid_problems():
    """ks_smooth_cov_static refuses, before any HIP call, a problem whose
    working data exceed its static array (KS_E_WORKSPACE) and an invalid
    description or missing output (KS_E_ARG); the pointers are never used."""
    L = ks.lib()
    fake = ctypes.c_void_p(1 << 20)
    k = 200000  # n = 6: about 0.5 GB of working data
    assert ks.workspace_bytes(k, 6, 3, False, False) > ks.STATIC_SCRATCH_BYTES
    d = ks.make_desc(k, 6, 3, False, False)
    assert L.ks_smooth_cov_static(ctypes.byref(d), *([fake] * 9), None) == ks.KS_E_WORKSPACE
    small = ks.make_desc(1000, 6, 3, False, False)
    assert ks.workspace_bytes(1000, 6, 3, False, False) <= ks.STATIC_SCRATCH_BYTES
    assert L.ks_smooth_cov_static(ctypes.byref(small), *([fake] * 7), None, fake, None) == ks.KS_E_ARG
    bad = ks.make_desc(1000, 7, 3, False, False)  # no kernels for n = 7
    assert L.ks_smooth_cov_static(ctypes.byref(bad), *([fake] * 9), None) == ks.KS_E_ARG
    assert L.ks_smooth_cov_static(None, *([fake] * 9), None) == ks.KS_E_ARG


def test_matrix_core_levels_stay_out_of_the_forward_tail(monkeypatch):
    """Forward variant 1 of n = 48 with diagonal covariances: however many
    tail passes are allowed, the levels that run the matrix-core forward
    (level 0 and the levels of at least 512 units) keep launches of their own,
    since the tail has the arithmetic of the narrow-level kernels."""
    monkeypatch.setenv("KS_FWD_VARIANT", "1")
    monkeypatch.setenv("KS_TAIL_PASSES", "1000000")
    k = 20000
    first_narrow = next(l for l in range(1, 20) if ((k + 1) >> l) // 2 < 512)
    assert _fake_plan(k, 48, 24)[1] == first_narrow
    assert _fake_plan(300, 48, 24)[1] == 1  # every level >= 1 narrow: only level 0 stays out
    monkeypatch.setenv("KS_FWD_VARIANT", "0")
    assert _fake_plan(k, 48, 24)[1] == 0  # the default family: everything may go to the tail
