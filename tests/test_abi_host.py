"""Host-side tests of the C ABI: the built library loads, exports every declared
entry point, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2307_16550_amd import gridhop as gh
from paper_2307_16550_amd import scene as sc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in ("gridhop.h", "gridhop_test.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(gh_[a-z_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gh.LIB_PATH):
        pytest.fail("libgridhop.so is not built (python -m paper_2307_16550_amd.build)")
    return gh.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert set(names) == set(gh.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version(lib):
    assert lib.gh_abi_version() == 4


def radar(**kw):
    s = sc.make_scene(1, 0)
    r = gh.Radar.from_scene(s)
    for k, v in kw.items():
        setattr(r.c_struct, k, v)
    return r


GRID = gh.make_grid((5, -10, -10, -10), (25, 10, 10, 10), (32, 32, 8, 8))
FAKE = ctypes.c_void_p(0x1000)     # never dereferenced: validation fails first


@pytest.mark.parametrize("field,value", [
    ("n_samples", 48), ("n_samples", 4), ("n_chirps", 2048), ("pad_range", 3), ("pad_doppler", 16),
    ("n_rx", 0), ("n_rx", 17), ("centered", 2), ("f0_hz", -1.0), ("bandwidth_hz", float("nan")),
    ("c_mps", 0.0), ("t_chirp_s", float("inf")),
])
def test_invalid_radar_rejected(lib, field, value):
    r = radar(**{field: value})
    rc = lib.gh_rd_maps(ctypes.byref(r.c_struct), FAKE, ctypes.c_void_p(0x100000000), 0, None)
    assert rc == gh.GH_EINVAL
    assert gh.last_error()


def test_null_and_overlap_rejected(lib):
    r = radar()
    assert lib.gh_rd_maps(None, FAKE, FAKE, 0, None) == gh.GH_EINVAL
    assert lib.gh_rd_maps(ctypes.byref(r.c_struct), None, FAKE, 0, None) == gh.GH_EINVAL
    assert lib.gh_rd_maps(ctypes.byref(r.c_struct), FAKE, FAKE, 0, None) == gh.GH_EINVAL
    assert "overlap" in gh.last_error()
    r.c_struct.rx = None
    assert lib.gh_rd_maps(ctypes.byref(r.c_struct), FAKE, ctypes.c_void_p(0x100000000), 0, None) == gh.GH_EINVAL


@pytest.mark.parametrize("lo,hi,n", [
    ((5, -10, -10, -10), (25, 10, 10, 10), (0, 32, 8, 8)),
    ((25, -10, -10, -10), (5, 10, 10, 10), (32, 32, 8, 8)),
    ((5, -10, -10, -10), (25, 10, 10, 10), (32, 32, 128, 64)),     # slab above 4096
    ((5, -10, -10, float("nan")), (25, 10, 10, 10), (32, 32, 8, 8)),
])
def test_invalid_grid_rejected(lib, lo, hi, n):
    r = radar()
    g = gh.make_grid(lo, hi, n)
    rc = lib.gh_decision(ctypes.byref(r.c_struct), ctypes.byref(g), FAKE, 0, 0, None, FAKE, None, None)
    assert rc in (gh.GH_EINVAL, gh.GH_EUNSUPPORTED)


def test_decision_argument_checks(lib):
    r = radar()
    assert lib.gh_decision(ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, 0, 7, None, FAKE, None, None) == gh.GH_EINVAL
    assert lib.gh_decision(ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, 0, 0, None, None, None, None) == gh.GH_EINVAL


def test_workspace_queries_and_shortfall(lib):
    r = radar()
    need = lib.gh_direct_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 0)
    assert need >= 3 * 32 * 32 * 32 * 8
    rc = lib.gh_direct_decision(ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, 0, FAKE, need - 1, None, FAKE,
                                None, None)
    assert rc == gh.GH_EWORKSPACE
    assert lib.gh_direct_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 9) == 0
    nb = lib.gh_bomp_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 0, 0)
    assert nb >= 32 * 32 * 16


def test_bomp_and_refine_argument_checks(lib):
    r = radar()
    ws = lib.gh_bomp_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 0, 0)
    args = [ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, ctypes.c_void_p(0x200000000), FAKE, 0, 0, 0, FAKE]
    assert lib.gh_bomp_step(*args, 3, 3, FAKE, None, FAKE, ws, None) == gh.GH_EINVAL      # n_support == max
    assert lib.gh_bomp_step(*args, 0, 33, FAKE, None, FAKE, ws, None) == gh.GH_EINVAL     # max above limit
    assert lib.gh_bomp_step(*args, 0, 3, FAKE, None, FAKE, ws - 1, None) == gh.GH_EWORKSPACE
    rws = lib.gh_refine_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 3)
    assert rws >= 2 * 3 * 3 * 12 * 8
    assert lib.gh_refine_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 0) == 0
    rargs = [ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, FAKE]
    assert lib.gh_refine(*rargs, 1, 0, FAKE, rws, FAKE, None, None) == gh.GH_EINVAL           # max_iter 0
    assert lib.gh_refine(*rargs, 3, 20, FAKE, rws - 1, FAKE, None, None) == gh.GH_EWORKSPACE
    assert lib.gh_refine(*rargs, 3, 20, None, rws, FAKE, None, None) == gh.GH_EINVAL
    assert lib.gh_refine(*rargs, 3, 20, FAKE, rws, FAKE, ctypes.c_void_p(0x1004), None) == gh.GH_EINVAL  # status misaligned
    assert lib.gh_refine(*rargs, 0, 20, None, 0, FAKE, None, None) == gh.GH_OK


def test_refine_noalloc_argument_checks(lib):
    """The no-allocation refinement rejects more cells than its static scratch
    serves, and the arguments gh_refine rejects, before touching a device."""
    r = radar()
    rargs = [ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, FAKE]
    assert lib.gh_refine_noalloc(*rargs, gh.REFINE_NOALLOC_MAX_CELLS + 1, 20, FAKE, None, None) == gh.GH_EUNSUPPORTED
    assert "at most 1024 cells" in gh.last_error()
    assert lib.gh_refine_noalloc(*rargs, -1, 20, FAKE, None, None) == gh.GH_EINVAL
    assert lib.gh_refine_noalloc(*rargs, 3, 0, FAKE, None, None) == gh.GH_EINVAL                # max_iter 0
    assert lib.gh_refine_noalloc(*rargs, 3, 101, FAKE, None, None) == gh.GH_EINVAL
    assert lib.gh_refine_noalloc(*rargs, 3, 20, None, None, None) == gh.GH_EINVAL               # theta NULL
    assert lib.gh_refine_noalloc(*rargs, 3, 20, FAKE, ctypes.c_void_p(0x1004), None) == gh.GH_EINVAL
    assert lib.gh_refine_noalloc(ctypes.byref(r.c_struct), ctypes.byref(GRID), None, FAKE, 3, 20, FAKE, None,
                                 None) == gh.GH_EINVAL
    assert lib.gh_refine_noalloc(*rargs, 0, 20, FAKE, None, None) == gh.GH_OK


def test_header_limits_of_refine_noalloc():
    text = open(os.path.join(ROOT, "include", "gridhop.h")).read()
    assert re.search(r"#define GH_REFINE_NOALLOC_MAX_CELLS (\d+)", text).group(1) == str(gh.REFINE_NOALLOC_MAX_CELLS)
    assert "#define GH_REFINE_NOALLOC_SCRATCH_BYTES (4u << 20)" in text


def test_bomp_seed_argument_checks(lib):
    r = radar()
    ws = lib.gh_bomp_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 0, 0)
    args = [ctypes.byref(r.c_struct), ctypes.byref(GRID)]
    assert lib.gh_bomp_seed(*args, 0, FAKE, FAKE, 3, None, FAKE, ws - 1, None) == gh.GH_EWORKSPACE
    assert lib.gh_bomp_seed(*args, 0, None, FAKE, 3, None, FAKE, ws, None) == gh.GH_EINVAL        # no block maxima
    assert lib.gh_bomp_seed(*args, 0, FAKE, FAKE, 33, None, FAKE, ws, None) == gh.GH_EINVAL       # max_support
    assert lib.gh_bomp_seed(*args, 5, FAKE, FAKE, 3, None, FAKE, ws, None) == gh.GH_EINVAL        # interp
    assert lib.gh_bomp_seed(*args, 0, FAKE, ctypes.c_void_p(0x1004), 3, None, FAKE, ws, None) == gh.GH_EINVAL


def test_bomp_select_and_fit_argument_checks(lib):
    r = radar()
    ws = lib.gh_bomp_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 0, 0)
    sargs = [ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, None, FAKE, 0, 0, 0, FAKE]
    assert lib.gh_bomp_select(*sargs, 1, 3, None, FAKE, ws, None) == gh.GH_EINVAL        # residual needed past 0
    assert lib.gh_bomp_select(*sargs, 3, 3, None, FAKE, ws, None) == gh.GH_EINVAL        # n_support == max
    assert lib.gh_bomp_select(*sargs, 0, 3, None, FAKE, ws - 1, None) == gh.GH_EWORKSPACE  # y alone at 0
    fargs = [ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, FAKE, FAKE]
    assert lib.gh_bomp_fit(*fargs, 0, 3, FAKE, FAKE, ws, None) == gh.GH_EINVAL           # nothing selected
    assert lib.gh_bomp_fit(*fargs, 4, 3, FAKE, FAKE, ws, None) == gh.GH_EINVAL           # above max_support
    assert lib.gh_bomp_fit(*fargs, 1, 3, None, FAKE, ws, None) == gh.GH_EINVAL           # alpha NULL
    assert lib.gh_bomp_fit(*fargs, 1, 3, FAKE, FAKE, 256, None) == gh.GH_EWORKSPACE


def test_error_message_cleared_after_success(lib):
    r = radar()
    lib.gh_rd_maps(None, FAKE, FAKE, 0, None)
    assert gh.last_error()
    assert lib.gh_refine(ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, FAKE, 0, 20, None, 0, FAKE, None,
                         None) == gh.GH_OK
    assert gh.last_error() == ""


def test_misaligned_pointers_rejected(lib):
    r = radar()
    odd = ctypes.c_void_p(0x1008)      # 8-byte aligned only
    far = ctypes.c_void_p(0x100000000)
    assert lib.gh_rd_maps(ctypes.byref(r.c_struct), odd, far, 0, None) == gh.GH_EINVAL
    assert "aligned" in gh.last_error()
    assert lib.gh_decision(ctypes.byref(r.c_struct), ctypes.byref(GRID), odd, 0, 0, None, FAKE, None, None) == gh.GH_EINVAL
    need = lib.gh_direct_workspace_bytes(ctypes.byref(r.c_struct), ctypes.byref(GRID), 1)
    assert lib.gh_direct_decision(ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, 1, odd, need, None, FAKE,
                                  None, None) == gh.GH_EINVAL
    assert lib.gh_refine(ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, odd, 1, 20, FAKE, 1 << 20, FAKE,
                         None, None) == gh.GH_EINVAL


def test_map_storage_checks(lib):
    r = radar()
    far = ctypes.c_void_p(0x100000000)
    assert lib.gh_rd_maps(ctypes.byref(r.c_struct), FAKE, far, 3, None) == gh.GH_EINVAL
    assert lib.gh_decision(ctypes.byref(r.c_struct), ctypes.byref(GRID), FAKE, -1, 0, None, FAKE, None, None) == gh.GH_EINVAL
    r1 = radar(pad_doppler=1)
    for dt in (gh.MAP_F16, gh.MAP_BF16):
        assert lib.gh_rd_maps(ctypes.byref(r1.c_struct), FAKE, far, dt, None) == gh.GH_EUNSUPPORTED
        assert "pad_doppler" in gh.last_error()
        assert lib.gh_decision(ctypes.byref(r1.c_struct), ctypes.byref(GRID), FAKE, dt, 0, None, FAKE, None,
                               None) == gh.GH_EUNSUPPORTED



def test_point_decision_argument_checks(lib):
    r = radar()
    far = ctypes.c_void_p(0x100000000)
    need = lib.gh_direct_points_workspace_bytes(ctypes.byref(r.c_struct), 16)
    assert need >= 16 * 3 * (32 // 8) * 6 * 8
    assert lib.gh_direct_points_workspace_bytes(ctypes.byref(r.c_struct), 0) == 0
    assert lib.gh_direct_points_workspace_bytes(ctypes.byref(r.c_struct), 70000) == 0
    args = [ctypes.byref(r.c_struct), FAKE, far]
    assert lib.gh_direct_points(*args, 16, FAKE, None, None, FAKE, need - 1, None) == gh.GH_EWORKSPACE
    assert lib.gh_direct_points(*args, -1, FAKE, None, None, FAKE, need, None) == gh.GH_EINVAL
    assert lib.gh_direct_points(*args, 16, None, None, None, FAKE, need, None) == gh.GH_EINVAL
    assert lib.gh_direct_points(*args, 0, FAKE, None, None, None, 0, None) == gh.GH_OK
    margs = [ctypes.byref(r.c_struct), FAKE, 0]
    assert lib.gh_gh_points(*margs, 2, far, 4, FAKE, None, None, None) == gh.GH_EINVAL          # interp
    assert lib.gh_gh_points(ctypes.byref(r.c_struct), FAKE, 5, 0, far, 4, FAKE, None, None, None) == gh.GH_EINVAL
    assert lib.gh_gh_points(*margs, 0, far, 70000, FAKE, None, None, None) == gh.GH_EINVAL
    assert lib.gh_gh_points(*margs, 0, far, 0, FAKE, None, None, None) == gh.GH_OK
    assert lib.gh_gh_points(*margs, 0, ctypes.c_void_p(0x100000008), 4, FAKE, None, None, None) == gh.GH_EINVAL


def batch_frames(specs):
    """gh_frame array from (k, ms, mc, pad_d, grid n) tuples; device pointers are fake."""
    keep, frames = [], (gh.GhFrame * len(specs))()
    for f, (k, ms, mc, pad_d, n) in enumerate(specs):
        s = sc.make_scene(1, 0, k=k, ms=ms, mc=mc, n=n)
        r = gh.Radar(s.f0, s.bw, s.tc, ms, mc, s.tx, s.rx, 4, pad_d, 1)
        keep.append(r)
        frames[f] = gh.GhFrame(r.c_struct, gh.grid_of(s.grid), FAKE, None, FAKE)
    return frames, keep


def test_batch_struct_layout():
    # gh_frame: gh_radar (4 doubles, 6 int32, tx[2], rx pointer = 80 bytes), gh_grid (80), 3 pointers
    assert ctypes.sizeof(gh.GhFrame) == 184 and gh.GhFrame.d_y.offset == 160
    # gh_batch_info: 16 int32, then two int64
    assert ctypes.sizeof(gh.GhBatchInfo) == 80 and gh.GhBatchInfo.points.offset == 64


def test_batch_tune_tiles_argument_checks(lib):
    assert lib.gh_batch_tune_tiles(None, 0, 0, 1, None) == gh.GH_EINVAL
    assert "batch is NULL" in gh.last_error()


def test_batch_argument_checks(lib):
    frames, keep = batch_frames([(3, 64, 32, 4, (8, 8, 4, 4)), (4, 128, 64, 2, (16, 12, 3, 24))])
    need = lib.gh_batch_workspace_bytes(frames, 2)
    maps = 3 * 256 * 128 * 8 + 4 * 512 * 128 * 8
    assert maps < need <= maps + 2 * 1024 + 3 * 256 + 2 * 4096
    assert lib.gh_batch_workspace_bytes(frames, 0) == 0
    out = ctypes.c_void_p()
    big = 1 << 40
    assert lib.gh_batch_create(frames, 2, 0, FAKE, big, None, None) == gh.GH_EINVAL
    assert lib.gh_batch_create(frames, 0, 0, FAKE, big, ctypes.byref(out), None) == gh.GH_EINVAL
    assert lib.gh_batch_create(frames, 2, 2, FAKE, big, ctypes.byref(out), None) == gh.GH_EINVAL
    assert lib.gh_batch_create(frames, 2, 0, None, big, ctypes.byref(out), None) == gh.GH_EINVAL
    assert lib.gh_batch_create(frames, 2, 0, FAKE, need - 1, ctypes.byref(out), None) == gh.GH_EWORKSPACE
    assert out.value is None
    # invalid frame radar: named by its index
    bad, keep2 = batch_frames([(3, 64, 32, 4, (8, 8, 4, 4)), (3, 64, 32, 4, (8, 8, 4, 4))])
    bad[1].radar.n_samples = 48
    assert lib.gh_batch_workspace_bytes(bad, 2) == 0
    assert "frame 1" in gh.last_error() and "n_samples" in gh.last_error()
    # shapes outside the batch sweep
    for spec in [(3, 64, 8, 1, (8, 8, 4, 4)),        # N_d = 8 < 16
                 (3, 64, 32, 4, (8, 8, 2, 65)),       # Nvy > 64
                 (3, 64, 32, 4, (8, 8, 33, 64)),      # 33 vx points per lane
                 (3, 64, 32, 4, (8, 8, 65, 32))]:     # 33 vx points per lane
        fr, keep3 = batch_frames([spec])
        assert lib.gh_batch_create(fr, 1, 0, FAKE, big, ctypes.byref(out), None) == gh.GH_EUNSUPPORTED, spec
    # NULL and misaligned frame pointers
    frames[1].d_block = None
    assert lib.gh_batch_create(frames, 2, 0, FAKE, big, ctypes.byref(out), None) == gh.GH_EINVAL
    frames[1].d_block = FAKE.value
    frames[0].d_y = 0x1008
    assert lib.gh_batch_create(frames, 2, 0, FAKE, big, ctypes.byref(out), None) == gh.GH_EINVAL
    # NULL batch objects
    info = gh.GhBatchInfo()
    assert lib.gh_batch_run(None, None, None) == gh.GH_EINVAL
    assert lib.gh_batch_tune(None, 0, 0, 0, 0) == gh.GH_EINVAL
    assert lib.gh_batch_get_info(None, ctypes.byref(info)) == gh.GH_EINVAL
    assert lib.gh_batch_frame_maps(None, 0, ctypes.byref(out)) == gh.GH_EINVAL
    lib.gh_batch_destroy(None)


def test_factored_argument_checks(lib):
    r = radar()
    far = ctypes.c_void_p(0x100000000)
    rs = ctypes.byref(r.c_struct)
    assert lib.gh_range_spectra(rs, None, far, None) == gh.GH_EINVAL
    assert lib.gh_range_spectra(rs, FAKE, ctypes.c_void_p(0x1008), None) == gh.GH_EINVAL    # misaligned
    assert lib.gh_range_spectra(rs, FAKE, FAKE, None) == gh.GH_EINVAL                       # overlap
    g = ctypes.byref(GRID)
    nd = lib.gh_factored_workspace_bytes(rs, g, gh.FACTOR_DIRECT)
    ng = lib.gh_factored_workspace_bytes(rs, g, gh.FACTOR_GH)
    # direct: the range zoom G (K x Nloc x Mc complex64) plus the peak buffers
    assert nd - ng == 3 * 32 * 32 * 32 * 8 and ng >= 32 * 32 * 16
    assert lib.gh_factored_workspace_bytes(rs, g, 2) == 0
    args = [rs, g]
    assert lib.gh_factored_decision(*args, 2, 0, 0, FAKE, FAKE, nd, None, None, FAKE, None) == gh.GH_EINVAL
    assert lib.gh_factored_decision(*args, gh.FACTOR_GH, 3, 0, FAKE, FAKE, ng, None, None, FAKE, None) == gh.GH_EINVAL
    assert lib.gh_factored_decision(*args, gh.FACTOR_DIRECT, 0, 2, FAKE, FAKE, nd, None, None, FAKE, None) == gh.GH_EINVAL
    assert lib.gh_factored_decision(*args, gh.FACTOR_GH, gh.POLAR, 0, FAKE, FAKE, ng - 1, None, None, FAKE,
                                    None) == gh.GH_EWORKSPACE
    assert lib.gh_factored_decision(*args, gh.FACTOR_GH, gh.POLAR, 0, FAKE, FAKE, ng, None, None, None,
                                    None) == gh.GH_EINVAL
    # the polar rule is for the factorised decision only
    assert lib.gh_decision(rs, g, FAKE, 0, gh.POLAR, None, FAKE, None, None) == gh.GH_EINVAL


def test_batch_lds_limits(lib):
    """A wave's LDS slice (768 B of coordinate records + 16 or 32 B per Doppler bin) must fit 64 KB."""
    out = ctypes.c_void_p()
    big = 1 << 40
    fr, keep = batch_frames([(3, 64, 1024, 4, (4, 4, 4, 4))])          # N_d = 4096
    assert lib.gh_batch_create(fr, 1, gh.BILINEAR, FAKE, big, ctypes.byref(out), None) == gh.GH_EUNSUPPORTED
    fr, keep = batch_frames([(3, 64, 512, 4, (4, 4, 4, 4))])           # N_d = 2048
    assert lib.gh_batch_create(fr, 1, gh.BICUBIC, FAKE, big, ctypes.byref(out), None) == gh.GH_EUNSUPPORTED
    assert "LDS" in gh.last_error()


def test_missing_library_fails_loudly(monkeypatch):
    """No fallback: without the built library every entry point raises instead of computing elsewhere."""
    monkeypatch.setattr(gh, "_lib", None)
    monkeypatch.setattr(gh, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libgridhop.so"))
    with pytest.raises(ImportError):
        gh.load()
    with pytest.raises(ImportError):
        gh.last_error()


def test_test_switches(lib):
    """gh_test_set_knob: per-thread overrides with range checks, the previous value returned."""
    assert lib.gh_test_set_knob(99, 1) == gh.GH_EINVAL
    assert lib.gh_test_set_knob(gh.GH_KNOB_BOMP_MAPS_FFT, 2) == gh.GH_EINVAL
    assert lib.gh_test_set_knob(gh.GH_KNOB_REFINE_ROWS, 24) == gh.GH_EINVAL       # not a power of two
    assert lib.gh_test_set_knob(gh.GH_KNOB_SWEEP_LDS_KIB, 4) == gh.GH_EINVAL      # below 8 KiB
    assert lib.gh_test_set_knob(gh.GH_KNOB_REFINE_ROWS, 16) == 0
    assert lib.gh_test_set_knob(gh.GH_KNOB_REFINE_ROWS, 0) == 16
    with gh.knob(gh.GH_KNOB_REFINE_SPIN_LIMIT, 5):
        assert lib.gh_test_set_knob(gh.GH_KNOB_REFINE_SPIN_LIMIT, 5) == 5
    assert lib.gh_test_set_knob(gh.GH_KNOB_REFINE_SPIN_LIMIT, 0) == 0
    import threading
    seen = []
    with gh.knob(gh.GH_KNOB_SWEEP_GENERIC, 1):
        th = threading.Thread(target=lambda: seen.append(lib.gh_test_set_knob(gh.GH_KNOB_SWEEP_GENERIC, 0)))
        th.start()
        th.join()
    assert seen == [0]      # another thread's switches are its own


def test_library_reads_no_environment():
    """No product source reads the environment: behaviour depends on arguments only."""
    for root, _, files in os.walk(os.path.join(ROOT, "paper_2307_16550_amd", "csrc")):
        for f in files:
            text = open(os.path.join(root, f)).read()
            assert "getenv" not in text, f
