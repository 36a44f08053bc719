"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/spiir.h declares, validates descriptors and plans
banks (lane packing, pieces, footprint) without touching a device."""
import ctypes as C
import subprocess

import numpy as np
import pytest

from paper_1702_02256_amd import spiir as S
from paper_1702_02256_amd import workloads as W


def _have_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_library_exports_every_declared_symbol():
    lib = S.load_library()
    declared = S.header_symbols()
    assert "spiir_create" in declared and "spiir_process_block" in declared
    for name in declared:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(declared) <= exported
    # every exported spiir_ symbol is declared (no undocumented entry points)
    assert {e for e in exported if e.startswith("spiir_")} <= set(declared)


def test_strerror():
    assert S.spiir_strerror(0) == "ok"
    assert "invalid" in S.spiir_strerror(S.SPIIR_EINVAL)
    assert "non-finite" in S.spiir_strerror(S.SPIIR_ENONFINITE)
    assert S.spiir_strerror(12345) == "unknown status"


def _small_multirate(T=3, H=3, seed=5):
    nf = np.random.default_rng(seed).integers(1, 40, size=(T, H)).astype(np.int32)
    return W.random_bank(seed, nf, 1024, W.multirate_dmax(1024, H))


def test_plan_single_template_padding():
    wl = W.config1()
    p = S.spiir_plan(wl.bank, 4096, filters_per_lane=4, waves_per_group=4)
    assert p["total_filters"] == 128
    assert p["n_groups"] == 1 and p["n_pieces"] == 1
    assert p["filter_slots"] == 4 * 256
    assert p["carry_chunk"] == 32 and p["lanes_per_group"] == 256


def test_plan_packs_segments_end_to_end():
    wl = W.config2(n_templates=8, n_blocks=1)
    p = S.spiir_plan(wl.bank, 2048, filters_per_lane=4, waves_per_group=4)
    # 512 filters / 4 per lane = 128 lanes: two templates per 256-lane group
    assert p["n_groups"] == 4 and p["n_pieces"] == 8
    p8 = S.spiir_plan(wl.bank, 2048, filters_per_lane=8, waves_per_group=1)
    assert p8["n_groups"] == 8 and p8["filter_slots"] == 8 * 512


def test_plan_splits_segments_across_groups():
    nf = np.array([[3000], [10]], np.int32)
    tb = W.random_bank(3, nf, 4096, [100])
    p = S.spiir_plan(tb, 4096, filters_per_lane=4, waves_per_group=4)
    # 750 + 3 lanes over 256-lane groups -> 3 groups; template 0 is split in 3
    assert p["n_groups"] == 3
    assert p["n_pieces"] == 4
    assert p["filter_slots"] >= 3010


def test_plan_waste_is_bounded():
    wl = W.config3(n_templates=64, n_blocks=1)
    p = S.spiir_plan(wl.bank, 4096, filters_per_lane=4, waves_per_group=4)
    segs = int((wl.bank.n_filters > 0).sum())
    # per segment at most F-1 padding slots plus one padding lane (segments span
    # an even number of lanes), plus one partial group per band
    assert p["filter_slots"] - p["total_filters"] <= segs * 7 + 7 * 4 * 256
    assert p["n_pieces"] >= segs


def test_footprint_matches_plan_and_scales():
    a = _small_multirate(T=4)
    b = _small_multirate(T=40)
    fa, fb = S.spiir_footprint(a, 1024), S.spiir_footprint(b, 1024)
    assert fa == S.spiir_plan(a, 1024)["footprint"]
    assert fb > fa > 0


@pytest.mark.parametrize("field,value", [
    ("n_bands", 0), ("n_bands", 13), ("max_block", 0), ("max_block", 1023 + 2),
    ("precision", 7), ("carry_chunk", 48), ("carry_chunk", 8), ("filters_per_lane", 3), ("window_copies", 3),
    ("waves_per_group", 17), ("base_rate_hz", 0), ("n_templates", 0), ("device", -1),
    ("time_chunks", 3), ("time_chunks", 128), ("time_chunks", -2),
])
def test_descriptor_validation(field, value):
    tb = _small_multirate()
    h = S._DescHolder(tb, 1024)
    setattr(h.desc, field, value)
    lib = S.load_library()
    out = C.c_size_t()
    assert lib.spiir_footprint(C.byref(h.desc), C.byref(out)) == S.SPIIR_EINVAL
    bank = C.c_void_p(123)
    assert lib.spiir_create(C.byref(h.desc), None, C.byref(bank)) == S.SPIIR_EINVAL
    assert bank.value is None


@pytest.mark.parametrize("bad", ["nan_a1", "neg_delay", "big_delay", "no_taps", "neg_count"])
def test_table_validation(bad):
    tb = _small_multirate()
    if bad == "nan_a1":
        tb.a1 = tb.a1.copy()
        tb.a1[5] = np.nan
    elif bad == "neg_delay":
        tb.delay = tb.delay.copy()
        tb.delay[2] = -1
    elif bad == "big_delay":
        tb.delay = tb.delay.copy()
        tb.delay[2] = 16384
    elif bad == "neg_count":
        tb.n_filters = tb.n_filters.copy()
        tb.n_filters[0, 0] = -1
    h = S._DescHolder(tb, 1024)
    if bad == "no_taps":
        h.desc.n_taps_up = 0
    out = C.c_size_t()
    assert S.load_library().spiir_footprint(C.byref(h.desc), C.byref(out)) == S.SPIIR_EINVAL


def test_process_calls_reject_null_bank():
    lib = S.load_library()
    assert lib.spiir_process_block(None, None, 16, None, 16, None) == S.SPIIR_EINVAL
    assert lib.spiir_process_batch(0, None, None) == S.SPIIR_EINVAL
    assert lib.spiir_destroy(None) == S.SPIIR_OK
    assert lib.spiir_reset(None) == S.SPIIR_EINVAL
    assert lib.spiir_status(None, None) == S.SPIIR_EINVAL
    g = C.c_void_p(123)
    assert lib.spiir_graph_create(0, None, C.byref(g)) == S.SPIIR_EINVAL
    assert g.value is None
    assert lib.spiir_graph_launch(None, None) == S.SPIIR_EINVAL
    assert lib.spiir_graph_destroy(None) == S.SPIIR_OK
    assert lib.spiir_process_peaks(None, None, 16, None, 16, None, 0.0, None) == S.SPIIR_EINVAL
    assert lib.spiir_process_batch_peaks(0, None, None, 0.0, None) == S.SPIIR_EINVAL
    info = S.PlanInfo()
    assert lib.spiir_bank_plan(None, C.byref(info)) == S.SPIIR_EINVAL


@pytest.mark.skipif(_have_gpu(), reason="checks the no-device error path")
def test_create_without_device_reports_device_error():
    tb = _small_multirate()
    h = S._DescHolder(tb, 1024)
    bank = C.c_void_p()
    rc = S.load_library().spiir_create(C.byref(h.desc), None, C.byref(bank))
    assert rc == S.SPIIR_EDEVICE and bank.value is None


def test_plan_time_chunks():
    wl = W.config1()
    p1 = S.spiir_plan(wl.bank, 4096)
    p32 = S.spiir_plan(wl.bank, 4096, time_chunks=32)
    assert p1["time_chunks"] == 1 and p32["time_chunks"] == 32
    # chunk states and the a1^length table are allocated only for a split bank
    assert p32["footprint"] > p1["footprint"]
    assert S.spiir_plan(wl.bank, 4096, time_chunks=1)["footprint"] == p1["footprint"]


def test_automatic_time_split_follows_the_bank_size():
    # the split pays while the longest workgroup's samples, cut in P, are no
    # fewer than the bank's work per workgroup slot of the device
    auto = S.TIME_CHUNKS_AUTO
    assert S.spiir_plan(W.config1().bank, 4096, time_chunks=auto)["time_chunks"] == 64
    sizes = {64: 16, 256: 4, 1024: 1}  # single-rate templates of 512 filters -> P
    for T, P in sizes.items():
        bank = W.config2(n_templates=T, n_blocks=1).bank
        p = S.spiir_plan(bank, 2048, time_chunks=auto)
        assert p["time_chunks"] == P, (T, p["time_chunks"])
        assert p == S.spiir_plan(bank, 2048, time_chunks=P)
    # an explicit shape is kept and split; a bank without filters is not split
    p = S.spiir_plan(W.config2(n_templates=64, n_blocks=1).bank, 2048, time_chunks=auto,
                     filters_per_lane=2, waves_per_group=2)
    assert (p["filters_per_lane"], p["lanes_per_group"]) == (2, 128) and p["time_chunks"] > 1
    empty = W.random_bank(5, np.zeros((2, 3), np.int32), 1024, W.multirate_dmax(1024, 3))
    assert S.spiir_plan(empty, 1024, time_chunks=auto)["time_chunks"] == 1


def test_default_shape_follows_the_bank_size():
    # a full multi-rate bank: the large workgroups (4 filters per lane, 8
    # waves) with either sum
    big = W.config3(n_blocks=1).bank
    for prec in ("fp32", "fp32_compensated"):
        p = S.spiir_plan(big, 4096, precision=prec)
        assert (p["filters_per_lane"], p["lanes_per_group"]) == (4, 512), prec
    # every filter slot is a filter or padding: F = 6 packs segments in lanes of 6
    six = S.spiir_plan(big, 4096, precision="fp32_compensated", filters_per_lane=6)
    assert six["lanes_per_group"] == 256
    assert six["filter_slots"] % 6 == 0 and six["filter_slots"] >= six["total_filters"]
    # a multi-rate bank with few rounds of them takes 4-wave groups; a
    # single-rate bank only when it does not fill the device
    small = W.config3(n_templates=1024, n_blocks=1).bank
    single = W.config2(n_blocks=1).bank
    for prec in ("fp32", "fp32_compensated"):
        p = S.spiir_plan(small, 4096, precision=prec)
        assert (p["filters_per_lane"], p["lanes_per_group"]) == (4, 256), prec
        p = S.spiir_plan(single, 2048, precision=prec)
        assert (p["filters_per_lane"], p["lanes_per_group"]) == (4, 512), prec
        p = S.spiir_plan(W.config2(n_templates=256, n_blocks=1).bank, 2048, precision=prec)
        assert (p["filters_per_lane"], p["lanes_per_group"]) == (4, 256), prec
    # an explicit F keeps its own default width; explicit shapes are kept
    bank = W.config3(n_templates=8, n_blocks=1).bank
    assert S.spiir_plan(bank, 4096, filters_per_lane=8)["lanes_per_group"] == 256
    assert S.spiir_plan(bank, 4096, filters_per_lane=4)["lanes_per_group"] == 512
    assert S.spiir_plan(bank, 4096, precision="fp32_compensated", filters_per_lane=4,
                        waves_per_group=8)["lanes_per_group"] == 512


def test_window_copies_follow_occupancy():
    # delays up to 4095 samples: two window copies leave one 8-wave group per
    # compute unit, one copy two; a bank of 4096 such templates has enough
    # groups to use them, so the library keeps one copy ...
    b2 = W.config2(n_templates=4096, n_blocks=1).bank
    p2 = S.spiir_plan(b2, 2048)
    assert p2["window_copies"] == 1
    assert S.spiir_plan(b2, 2048, window_copies=2)["lds_bytes"] > p2["lds_bytes"]
    # ... while 1024 of them make only one group per compute unit either way
    assert S.spiir_plan(W.config2(n_templates=1024, n_blocks=1).bank, 2048)["window_copies"] == 2
    # the multi-rate bank keeps the two-copy window (3 or more waves per SIMD)
    b3 = W.config3(n_templates=8, n_blocks=1).bank
    assert S.spiir_plan(b3, 4096)["window_copies"] == 2
    assert S.spiir_plan(b3, 4096, precision="fp32_compensated")["window_copies"] == 2
    assert S.spiir_plan(b3, 4096, window_copies=1)["window_copies"] == 1


def test_long_delays_fall_back_to_a_smaller_launch_shape():
    # a two-copy delay window of 16383 samples does not fit the LDS next to
    # 8-wave reduction buffers; 8-wave groups keep one copy, and with two
    # copies asked for the shape steps down instead of refusing the bank
    tb = W.random_bank(21, np.array([[64], [64]], np.int32), 4096, [16383])
    tb.delay = tb.delay.copy()
    tb.delay[0] = 16383
    assert S.spiir_plan(tb, 4096)["lds_bytes"] <= 160 * 1024
    p = S.spiir_plan(tb, 4096, filters_per_lane=4)
    assert p["window_copies"] == 1 and p["lanes_per_group"] == 512 and p["lds_bytes"] <= 160 * 1024
    p2 = S.spiir_plan(tb, 4096, filters_per_lane=4, window_copies=2)
    assert p2["lanes_per_group"] < 512 and p2["lds_bytes"] <= 160 * 1024
    with pytest.raises(S.SpiirError):  # an explicit shape is not changed
        S.spiir_plan(tb, 4096, waves_per_group=8, window_copies=2)
    # ordinary delays keep the 8-wave default
    assert S.spiir_plan(W.config3(n_templates=8, n_blocks=1).bank, 4096, filters_per_lane=4)["lanes_per_group"] == 512


def test_caller_workspace_leaves_the_workspace_out_of_the_footprint():
    tb = _small_multirate(T=4, H=3)
    own = S.spiir_plan(tb, 4096)
    cal = S.spiir_plan(tb, 4096, workspace=S.WORKSPACE_CALLER)
    assert own["workspace"] == S.WORKSPACE_OWN and cal["workspace"] == S.WORKSPACE_CALLER
    assert own["workspace_bytes"] == cal["workspace_bytes"] > 0
    assert own["workspace_bytes"] % 256 == 0
    # the workspace is the one difference between the two footprints
    assert 0 <= own["workspace_bytes"] - (own["footprint"] - cal["footprint"]) < 256
    with pytest.raises(S.SpiirError) as ei:
        S.spiir_plan(tb, 4096, workspace=2)
    assert ei.value.code == S.SPIIR_EINVAL


def test_clone_rejects_null():
    lib = S.load_library()
    out = C.c_void_p(123)
    assert lib.spiir_clone(None, None, C.byref(out)) == S.SPIIR_EINVAL
    assert out.value is None
    assert lib.spiir_clone(None, None, None) == S.SPIIR_EINVAL


def test_matrix_core_engine_descriptor_rules():
    wl = W.config2(n_templates=3, n_blocks=1)
    p = S.spiir_plan(wl.bank, 2048, engine=S.ENGINE_MFMA)
    assert p["engine"] == S.ENGINE_MFMA
    # one template per 256-slot workgroup: 512 filters -> 2 workgroups each
    assert p["n_groups"] == 6 and p["n_pieces"] == 6 and p["filter_slots"] == 6 * 256
    for kw in ({"precision": "fp32_compensated"}, {"time_chunks": 4}):
        with pytest.raises(S.SpiirError) as ei:
            S.spiir_plan(wl.bank, 2048, engine=S.ENGINE_MFMA, **kw)
        assert ei.value.code == S.SPIIR_EINVAL
    with pytest.raises(S.SpiirError):
        S.spiir_plan(wl.bank, 2000, engine=S.ENGINE_MFMA)       # max_block % 128
    with pytest.raises(S.SpiirError):
        S.spiir_plan(_small_multirate(), 1024, engine=S.ENGINE_MFMA)  # more than one band
    with pytest.raises(S.SpiirError):
        S.spiir_plan(wl.bank, 2048, engine=2)
