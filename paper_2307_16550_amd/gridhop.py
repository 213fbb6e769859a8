"""Python binding of the gfx950 grid-hopping C ABI (include/gridhop.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  The library must have been built (python -m
paper_2307_16550_amd.build); loading fails loudly otherwise, and there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # imported first: the library binds to the HIP runtime torch has loaded

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgridhop.so")

GH_OK, GH_EINVAL, GH_EUNSUPPORTED, GH_EHIP, GH_EWORKSPACE = 0, -1, -2, -3, -4
BILINEAR, BICUBIC, POLAR = 0, 1, 2
FACTOR_DIRECT, FACTOR_GH = 0, 1
GEMM_F32, GEMM_BF16 = 0, 1
MAP_C64, MAP_F16, MAP_BF16 = 0, 1, 2
MAX_SUPPORT = 32

EXPORTS = ("gh_abi_version", "gh_last_error", "gh_rd_maps", "gh_decision", "gh_argmax", "gh_direct_workspace_bytes",
           "gh_direct_decision", "gh_bomp_workspace_bytes", "gh_bomp_step", "gh_bomp_select", "gh_bomp_seed", "gh_bomp_fit",
           "gh_refine_workspace_bytes",
           "gh_refine", "gh_refine_noalloc", "gh_direct_points_workspace_bytes", "gh_direct_points", "gh_gh_points",
           "gh_range_spectra", "gh_factored_workspace_bytes", "gh_factored_decision",
           "gh_batch_workspace_bytes", "gh_batch_create", "gh_batch_tune", "gh_batch_tune_tiles", "gh_batch_get_info",
           "gh_batch_run",
           "gh_batch_frame_maps", "gh_batch_destroy", "gh_test_set_knob")


class GhRadar(ctypes.Structure):
    _fields_ = [("f0_hz", ctypes.c_double), ("bandwidth_hz", ctypes.c_double), ("t_chirp_s", ctypes.c_double),
                ("c_mps", ctypes.c_double), ("n_samples", ctypes.c_int32), ("n_chirps", ctypes.c_int32),
                ("pad_range", ctypes.c_int32), ("pad_doppler", ctypes.c_int32), ("n_rx", ctypes.c_int32),
                ("centered", ctypes.c_int32), ("tx", ctypes.c_double * 2), ("rx", ctypes.POINTER(ctypes.c_double))]


class GhGrid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4), ("n", ctypes.c_int32 * 4)]


class GhPeak(ctypes.Structure):
    _fields_ = [("value", ctypes.c_float), ("reserved", ctypes.c_int32), ("index", ctypes.c_int64)]


class GhFrame(ctypes.Structure):
    _fields_ = [("radar", GhRadar), ("grid", GhGrid), ("d_y", ctypes.c_void_p), ("d_decision", ctypes.c_void_p),
                ("d_block", ctypes.c_void_p)]


class GhBatchInfo(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("interp", ctypes.c_int32), ("units", ctypes.c_int32 * 3),
                ("workgroups", ctypes.c_int32 * 3), ("max_workgroups", ctypes.c_int32 * 3),
                ("sweep_waves", ctypes.c_int32), ("column_height", ctypes.c_int32),
                ("sweep_locations", ctypes.c_int32), ("range_chirps", ctypes.c_int32), ("doppler_rows", ctypes.c_int32),
                ("points", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64)]


class GridHopError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gridhop status {code}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libgridhop.so (built in-tree) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_16550_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64p = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    rp, gp_, pp = ctypes.POINTER(GhRadar), ctypes.POINTER(GhGrid), ctypes.c_void_p
    lib.gh_abi_version.restype = ctypes.c_int
    lib.gh_last_error.restype = ctypes.c_char_p
    lib.gh_rd_maps.argtypes = [rp, vp, vp, i32, vp]
    lib.gh_decision.argtypes = [rp, gp_, vp, i32, i32, vp, pp, pp, vp]
    lib.gh_argmax.argtypes = [pp, ctypes.c_int64, pp, vp]
    lib.gh_direct_workspace_bytes.argtypes = [rp, gp_, i32]
    lib.gh_direct_workspace_bytes.restype = sz
    lib.gh_direct_decision.argtypes = [rp, gp_, vp, i32, vp, sz, vp, pp, pp, vp]
    lib.gh_bomp_workspace_bytes.argtypes = [rp, gp_, i32, i32]
    lib.gh_bomp_workspace_bytes.restype = sz
    lib.gh_bomp_step.argtypes = [rp, gp_, vp, vp, vp, i32, i32, i32, vp, i32, i32, vp, pp, vp, sz, vp]
    lib.gh_bomp_select.argtypes = [rp, gp_, vp, vp, vp, i32, i32, i32, vp, i32, i32, pp, vp, sz, vp]
    lib.gh_bomp_fit.argtypes = [rp, gp_, vp, vp, vp, i32, i32, vp, vp, sz, vp]
    lib.gh_bomp_seed.argtypes = [rp, gp_, i32, pp, vp, i32, pp, vp, sz, vp]
    lib.gh_refine_workspace_bytes.argtypes = [rp, gp_, i32]
    lib.gh_refine_workspace_bytes.restype = sz
    lib.gh_refine.argtypes = [rp, gp_, vp, vp, i32, i32, vp, sz, vp, vp, vp]
    lib.gh_refine_noalloc.argtypes = [rp, gp_, vp, vp, i32, i32, vp, vp, vp]
    lib.gh_test_set_knob.argtypes = [i32, i32]
    lib.gh_test_set_knob.restype = ctypes.c_int
    lib.gh_direct_points_workspace_bytes.argtypes = [rp, i32]
    lib.gh_direct_points_workspace_bytes.restype = sz
    lib.gh_direct_points.argtypes = [rp, vp, vp, i32, vp, vp, vp, vp, sz, vp]
    lib.gh_gh_points.argtypes = [rp, vp, i32, i32, vp, i32, vp, vp, vp, vp]
    lib.gh_range_spectra.argtypes = [rp, vp, vp, vp]
    lib.gh_factored_workspace_bytes.argtypes = [rp, gp_, i32]
    lib.gh_factored_workspace_bytes.restype = sz
    lib.gh_factored_decision.argtypes = [rp, gp_, i32, i32, i32, vp, vp, sz, vp, vp, pp, vp]
    fp = ctypes.POINTER(GhFrame)
    lib.gh_batch_workspace_bytes.argtypes = [fp, i32]
    lib.gh_batch_workspace_bytes.restype = sz
    lib.gh_batch_create.argtypes = [fp, i32, i32, vp, sz, ctypes.POINTER(ctypes.c_void_p), vp]
    lib.gh_batch_tune.argtypes = [vp, i32, i32, i32, i32]
    lib.gh_batch_tune_tiles.argtypes = [vp, i32, i32, i32, vp]
    lib.gh_batch_get_info.argtypes = [vp, ctypes.POINTER(GhBatchInfo)]
    lib.gh_batch_run.argtypes = [vp, pp, vp]
    lib.gh_batch_frame_maps.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_void_p)]
    lib.gh_batch_destroy.argtypes = [vp]
    lib.gh_batch_destroy.restype = None
    for name in ("gh_rd_maps", "gh_decision", "gh_argmax", "gh_direct_decision", "gh_bomp_step", "gh_bomp_select",
                 "gh_bomp_seed", "gh_bomp_fit", "gh_refine", "gh_refine_noalloc",
                 "gh_direct_points", "gh_gh_points", "gh_range_spectra", "gh_factored_decision", "gh_batch_create", "gh_batch_tune", "gh_batch_tune_tiles", "gh_batch_get_info",
                 "gh_batch_run", "gh_batch_frame_maps"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def last_error() -> str:
    return load().gh_last_error().decode()


def _check(rc):
    if rc != GH_OK:
        raise GridHopError(rc, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Radar:
    """gh_radar with its receiver array kept alive."""

    def __init__(self, f0, bw, tc, ms, mc, tx, rx, pad_r=4, pad_d=4, centered=1, c=299_792_458.0):
        self.rx = np.ascontiguousarray(np.asarray(rx, np.float64).reshape(-1, 2))
        self.k = self.rx.shape[0]
        self.ms, self.mc, self.pad_r, self.pad_d = int(ms), int(mc), int(pad_r), int(pad_d)
        self.c_struct = GhRadar(float(f0), float(bw), float(tc), float(c), self.ms, self.mc, self.pad_r, self.pad_d,
                                self.k, int(centered), (ctypes.c_double * 2)(*[float(v) for v in tx]),
                                self.rx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))

    def with_rx(self, rx) -> "Radar":
        """The same radar with other receiver positions (K x 2, metres)."""
        c = self.c_struct
        return Radar(c.f0_hz, c.bandwidth_hz, c.t_chirp_s, self.ms, self.mc, (c.tx[0], c.tx[1]), rx, self.pad_r,
                     self.pad_d, c.centered, c.c_mps)

    @property
    def nr(self):
        return self.pad_r * self.ms

    @property
    def nd(self):
        return self.pad_d * self.mc

    @classmethod
    def from_scene(cls, s):
        return cls(s.f0, s.bw, s.tc, s.ms, s.mc, s.tx, s.rx, s.pad, s.pad, s.centered, s.c)


def make_grid(lo, hi, n) -> GhGrid:
    return GhGrid((ctypes.c_double * 4)(*map(float, lo)), (ctypes.c_double * 4)(*map(float, hi)),
                  (ctypes.c_int32 * 4)(*map(int, n)))


def grid_of(g) -> GhGrid:
    return make_grid(g.lo, g.hi, g.n)


def peaks_tensor(n, device):
    """Device buffer for n gh_peak records (16 bytes each)."""
    return torch.empty((n, 2), dtype=torch.int64, device=device)


def decode_peaks(t: torch.Tensor):
    """(values float32, indices int64) from a gh_peak buffer."""
    raw = t.detach().cpu().contiguous().numpy()
    vals = raw.view(np.float32).reshape(-1, 4)[:, 0].copy()
    return vals, raw[:, 1].copy()


def _c64(t):
    if t.dtype != torch.complex64 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("expected a contiguous complex64 CUDA tensor")
    return t


_MAP_TORCH = {MAP_C64: torch.complex64, MAP_F16: torch.float16, MAP_BF16: torch.bfloat16}


def map_dtype_of(maps: torch.Tensor) -> int:
    """Storage code of a map tensor: complex64 [K, N_r, N_d], or float16 / bfloat16
    [K, N_r, N_d, 2] holding Z / (Ms * Mc)."""
    for code, dt in _MAP_TORCH.items():
        if maps.dtype == dt:
            if code != MAP_C64 and (maps.dim() != 4 or maps.shape[-1] != 2):
                raise ValueError("16-bit maps must have shape [K, N_r, N_d, 2]")
            if not maps.is_contiguous():
                raise ValueError("maps must be contiguous")
            return code
    raise ValueError(f"unsupported map dtype {maps.dtype}")


def rd_maps(radar: Radar, y: torch.Tensor, maps: torch.Tensor | None = None, map_dtype=MAP_C64,
            stream=None) -> torch.Tensor:
    lib = load()
    _c64(y)
    if maps is None:
        shape = (radar.k, radar.nr, radar.nd) if map_dtype == MAP_C64 else (radar.k, radar.nr, radar.nd, 2)
        maps = torch.empty(shape, dtype=_MAP_TORCH[map_dtype], device=y.device)
    code = map_dtype_of(maps)
    _check(lib.gh_rd_maps(ctypes.byref(radar.c_struct), _ptr(y), _ptr(maps), code, _stream(stream)))
    return maps


def decision(radar: Radar, grid: GhGrid, maps, interp=BILINEAR, dec=None, block=None, argmax=None,
             write_volume=True, want_argmax=True, stream=None):
    lib = load()
    code = map_dtype_of(maps)
    nloc = grid.n[0] * grid.n[1]
    if dec is None and write_volume:
        dec = torch.empty(tuple(grid.n), dtype=torch.float32, device=maps.device)
    if block is None:
        block = peaks_tensor(nloc, maps.device)
    if argmax is None and want_argmax:
        argmax = peaks_tensor(1, maps.device)
    _check(lib.gh_decision(ctypes.byref(radar.c_struct), ctypes.byref(grid), _ptr(maps), code, int(interp),
                           _ptr(dec), _ptr(block), _ptr(argmax), _stream(stream)))
    return dec, block, argmax


def argmax(block: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """Global maximum of a gh_peak buffer (value, index; ties to the lowest index)."""
    lib = load()
    if out is None:
        out = peaks_tensor(1, block.device)
    _check(lib.gh_argmax(_ptr(block), block.shape[0], _ptr(out), _stream(stream)))
    return out


def direct_workspace_bytes(radar: Radar, grid: GhGrid, gemm=GEMM_F32) -> int:
    n = load().gh_direct_workspace_bytes(ctypes.byref(radar.c_struct), ctypes.byref(grid), int(gemm))
    if n == 0:
        raise GridHopError(GH_EINVAL, last_error())
    return n


def direct_decision(radar: Radar, grid: GhGrid, y, gemm=GEMM_F32, ws=None, dec=None, block=None, argmax=None,
                    write_volume=True, want_argmax=True, stream=None):
    lib = load()
    _c64(y)
    nloc = grid.n[0] * grid.n[1]
    if ws is None:
        ws = torch.empty(direct_workspace_bytes(radar, grid, gemm), dtype=torch.uint8, device=y.device)
    if dec is None and write_volume:
        dec = torch.empty(tuple(grid.n), dtype=torch.float32, device=y.device)
    if block is None:
        block = peaks_tensor(nloc, y.device)
    if argmax is None and want_argmax:
        argmax = peaks_tensor(1, y.device)
    _check(lib.gh_direct_decision(ctypes.byref(radar.c_struct), ctypes.byref(grid), _ptr(y), int(gemm), _ptr(ws),
                                  ws.numel(), _ptr(dec), _ptr(block), _ptr(argmax), _stream(stream)))
    return dec, block, argmax


def bomp_workspace_bytes(radar: Radar, grid: GhGrid, use_direct=False, gemm=GEMM_F32) -> int:
    n = load().gh_bomp_workspace_bytes(ctypes.byref(radar.c_struct), ctypes.byref(grid), int(use_direct), int(gemm))
    if n == 0:
        raise GridHopError(GH_EINVAL, last_error())
    return n


class BompState:
    """Device buffers of a Block-OMP run (residual, maps, support, alpha, workspace)."""

    def __init__(self, radar: Radar, grid: GhGrid, y: torch.Tensor, max_support=3, use_direct=False,
                 interp=BILINEAR, gemm=GEMM_F32):
        self.radar, self.grid, self.y = radar, grid, _c64(y)
        self.use_direct, self.interp, self.gemm = int(use_direct), int(interp), int(gemm)
        self.max_support = int(max_support)
        dev = y.device
        self.resid = y.clone()
        self.maps = None if use_direct else torch.empty((radar.k, radar.nr, radar.nd), dtype=torch.complex64,
                                                        device=dev)
        self.support = torch.full((self.max_support,), -1, dtype=torch.int64, device=dev)
        self.alpha = torch.zeros((self.max_support, radar.k), dtype=torch.complex64, device=dev)
        self.selected = peaks_tensor(1, dev)
        self.ws = torch.empty(bomp_workspace_bytes(radar, grid, use_direct, gemm), dtype=torch.uint8, device=dev)
        self.n = 0
        self._selected_pending = False

    def reset(self):
        """Start over: the next step selects on y itself (the residual is not read then)."""
        self.n = 0
        self._selected_pending = False

    def step(self, stream=None):
        if self._selected_pending:
            raise RuntimeError("select() was called without fit()")
        lib = load()
        _check(lib.gh_bomp_step(ctypes.byref(self.radar.c_struct), ctypes.byref(self.grid), _ptr(self.y),
                                _ptr(self.resid), _ptr(self.maps), self.use_direct, self.interp, self.gemm,
                                _ptr(self.support), self.n, self.max_support, _ptr(self.alpha), _ptr(self.selected),
                                _ptr(self.ws), self.ws.numel(), _stream(stream)))
        self.n += 1

    def select(self, stream=None):
        """First half of step(): the decision on the residual and the new selection
        (support[n]); fit() completes the iteration."""
        if self._selected_pending:
            raise RuntimeError("select() called twice without fit()")
        lib = load()
        _check(lib.gh_bomp_select(ctypes.byref(self.radar.c_struct), ctypes.byref(self.grid), _ptr(self.y),
                                  _ptr(self.resid), _ptr(self.maps), self.use_direct, self.interp, self.gemm,
                                  _ptr(self.support), self.n, self.max_support, _ptr(self.selected),
                                  _ptr(self.ws), self.ws.numel(), _stream(stream)))
        self._selected_pending = True

    def seed(self, block, selected=None, stream=None):
        """The first selection from a grid-hopping decision already made on the frame
        (gh_bomp_seed): self.maps must hold rd_maps of y and `block` that decision's
        per-location maxima over the same grid with the same interp.  The selected
        maximum (the decision's argmax) goes to `selected` (gh_peak [1]) when given,
        else to self.selected.  fit() completes the iteration."""
        if self.use_direct:
            raise ValueError("seed() applies to grid-hopping runs")
        if self._selected_pending:
            raise RuntimeError("seed() called twice without fit()")
        lib = load()
        out = self.selected if selected is None else selected
        _check(lib.gh_bomp_seed(ctypes.byref(self.radar.c_struct), ctypes.byref(self.grid), self.interp,
                                _ptr(block), _ptr(self.support), self.max_support, _ptr(out),
                                _ptr(self.ws), self.ws.numel(), _stream(stream)))
        self.n = 0
        self._selected_pending = True

    def fit(self, stream=None):
        """Second half of step(): least squares over the n + 1 selected cells and the residual."""
        if not self._selected_pending:
            raise RuntimeError("fit() needs a select() first")
        lib = load()
        _check(lib.gh_bomp_fit(ctypes.byref(self.radar.c_struct), ctypes.byref(self.grid), _ptr(self.y),
                               _ptr(self.resid), _ptr(self.support), self.n + 1, self.max_support, _ptr(self.alpha),
                               _ptr(self.ws), self.ws.numel(), _stream(stream)))
        self._selected_pending = False
        self.n += 1


def refine_workspace_bytes(radar: Radar, grid: GhGrid, n_cells: int) -> int:
    n = load().gh_refine_workspace_bytes(ctypes.byref(radar.c_struct), ctypes.byref(grid), int(n_cells))
    if n == 0:
        raise GridHopError(GH_EINVAL, last_error())
    return n


def refine(radar: Radar, grid: GhGrid, y, cells: torch.Tensor, max_iter=20, theta=None, ws=None, status=None,
           stream=None):
    """Refined (x, y, vx, vy) [n, 4] from each starting cell; `status` (int32 [1], optional)
    receives the number of cells left NaN by an expired cluster barrier."""
    lib = load()
    _c64(y)
    if cells.dtype != torch.int64 or not cells.is_cuda:
        raise ValueError("cells must be an int64 CUDA tensor")
    if theta is None:
        theta = torch.empty((cells.numel(), 4), dtype=torch.float64, device=y.device)
    if ws is None and cells.numel() > 0:
        ws = torch.empty(refine_workspace_bytes(radar, grid, cells.numel()), dtype=torch.uint8, device=y.device)
    nws = 0 if ws is None else ws.numel()
    if status is not None and (status.dtype != torch.int32 or not status.is_cuda or status.numel() < 1):
        raise ValueError("status must be an int32 CUDA tensor with at least one element")
    _check(lib.gh_refine(ctypes.byref(radar.c_struct), ctypes.byref(grid), _ptr(y), _ptr(cells), cells.numel(),
                         int(max_iter), _ptr(ws), nws, _ptr(theta), _ptr(status), _stream(stream)))
    return theta


REFINE_NOALLOC_MAX_CELLS = 1024


def refine_noalloc(radar: Radar, grid: GhGrid, y, cells: torch.Tensor, max_iter=20, theta=None, status=None,
                   stream=None):
    """gh_refine_noalloc: as refine(), with the library's static scratch (no workspace)."""
    lib = load()
    _c64(y)
    if cells.dtype != torch.int64 or not cells.is_cuda:
        raise ValueError("cells must be an int64 CUDA tensor")
    if theta is None:
        theta = torch.empty((cells.numel(), 4), dtype=torch.float64, device=y.device)
    if status is not None and (status.dtype != torch.int32 or not status.is_cuda or status.numel() < 1):
        raise ValueError("status must be an int32 CUDA tensor with at least one element")
    _check(lib.gh_refine_noalloc(ctypes.byref(radar.c_struct), ctypes.byref(grid), _ptr(y), _ptr(cells),
                                 cells.numel(), int(max_iter), _ptr(theta), _ptr(status), _stream(stream)))
    return theta


GH_KNOB_SWEEP_GENERIC, GH_KNOB_SWEEP_LDS_KIB, GH_KNOB_BOMP_MAPS_FFT = 1, 2, 3
GH_KNOB_REFINE_SINGLE, GH_KNOB_REFINE_ROWS, GH_KNOB_REFINE_SPIN_LIMIT = 4, 5, 6


class knob:
    """Context manager of a test switch (include/gridhop_test.h) for the calling thread:
    `with knob(GH_KNOB_BOMP_MAPS_FFT, 1): ...` restores the previous value on exit."""

    def __init__(self, which: int, value: int):
        self.which, self.value, self.prev = int(which), int(value), None

    def __enter__(self):
        rc = load().gh_test_set_knob(self.which, self.value)
        if rc < 0:
            raise GridHopError(rc, last_error())
        self.prev = rc
        return self

    def __exit__(self, *exc):
        load().gh_test_set_knob(self.which, self.prev)
        return False


def _points_outputs(theta, k, want_grad, want_grad_rx):
    if theta.dtype != torch.float64 or not theta.is_cuda or theta.dim() != 2 or theta.shape[1] != 4:
        raise ValueError("theta must be a float64 CUDA tensor of shape [n, 4]")
    theta = theta.contiguous()
    n = theta.shape[0]
    value = torch.empty(n, dtype=torch.float64, device=theta.device)
    grad = torch.empty((n, 4), dtype=torch.float64, device=theta.device) if want_grad else None
    grad_rx = torch.empty((n, k, 2), dtype=torch.float64, device=theta.device) if want_grad_rx else None
    return theta, value, grad, grad_rx


def direct_points(radar: Radar, y, theta: torch.Tensor, want_grad=True, want_grad_rx=False, ws=None, stream=None):
    """Direct decision at continuous points theta [n, 4] (x, y, vx, vy): (value [n], grad [n, 4] or None,
    grad_rx [n, K, 2] or None)."""
    lib = load()
    _c64(y)
    theta, value, grad, grad_rx = _points_outputs(theta, radar.k, want_grad, want_grad_rx)
    n = theta.shape[0]
    if n == 0:
        return value, grad, grad_rx
    if ws is None:
        nb = lib.gh_direct_points_workspace_bytes(ctypes.byref(radar.c_struct), n)
        if nb == 0:
            raise GridHopError(GH_EINVAL, last_error())
        ws = torch.empty(nb, dtype=torch.uint8, device=theta.device)
    _check(lib.gh_direct_points(ctypes.byref(radar.c_struct), _ptr(y), _ptr(theta), n, _ptr(value), _ptr(grad),
                                _ptr(grad_rx), _ptr(ws), ws.numel(), _stream(stream)))
    return value, grad, grad_rx


def gh_points(radar: Radar, maps, theta: torch.Tensor, interp=BILINEAR, want_grad=True, want_grad_rx=False,
              stream=None):
    """Grid-hopping decision at continuous points theta [n, 4]: (value, grad or None, grad_rx or None)."""
    lib = load()
    code = map_dtype_of(maps)
    theta, value, grad, grad_rx = _points_outputs(theta, radar.k, want_grad, want_grad_rx)
    n = theta.shape[0]
    if n == 0:
        return value, grad, grad_rx
    _check(lib.gh_gh_points(ctypes.byref(radar.c_struct), _ptr(maps), code, int(interp), _ptr(theta), n,
                            _ptr(value), _ptr(grad), _ptr(grad_rx), _stream(stream)))
    return value, grad, grad_rx



def range_spectra(radar: Radar, y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Per-chirp zero-padded range spectra, complex64 [K, N_r, Mc]."""
    lib = load()
    _c64(y)
    if out is None:
        out = torch.empty((radar.k, radar.nr, radar.mc), dtype=torch.complex64, device=y.device)
    _check(lib.gh_range_spectra(ctypes.byref(radar.c_struct), _ptr(y), _ptr(_c64(out)), _stream(stream)))
    return out


def factored_workspace_bytes(radar: Radar, grid: GhGrid, method: int) -> int:
    n = load().gh_factored_workspace_bytes(ctypes.byref(radar.c_struct), ctypes.byref(grid), int(method))
    if n == 0:
        raise GridHopError(GH_EINVAL, last_error())
    return n


def factored_decision(radar: Radar, grid: GhGrid, method: int, inp: torch.Tensor, range_interp=POLAR,
                      gemm=GEMM_F32, ws=None, loc=None, vel=None, result=None, write_loc=True, write_vel=True,
                      stream=None):
    """Eqs. (5)-(6): (E [Nx, Ny] or None, V [Nvx, Nvy] or None, result gh_peak [2]: (E(x^), location),
    (V(v^), 4D index)).  inp: the frames (FACTOR_DIRECT) or range_spectra (FACTOR_GH)."""
    lib = load()
    _c64(inp)
    dev = inp.device
    if ws is None:
        ws = torch.empty(factored_workspace_bytes(radar, grid, method), dtype=torch.uint8, device=dev)
    if loc is None and write_loc:
        loc = torch.empty((grid.n[0], grid.n[1]), dtype=torch.float32, device=dev)
    if vel is None and write_vel:
        vel = torch.empty((grid.n[2], grid.n[3]), dtype=torch.float32, device=dev)
    if result is None:
        result = peaks_tensor(2, dev)
    _check(lib.gh_factored_decision(ctypes.byref(radar.c_struct), ctypes.byref(grid), int(method), int(range_interp),
                                    int(gemm), _ptr(inp), _ptr(ws), ws.numel(), _ptr(loc), _ptr(vel), _ptr(result),
                                    _stream(stream)))
    return loc, vel, result


class Batch:
    """Frames of different shapes decided together (gh_batch_*): maps, grid-hopping
    decisions (block maxima, optional volumes) and per-frame argmax, each step one
    persistent launch over all frames.  Owns the workspace, the output buffers and
    the C object; the frame tensors `ys` must stay allocated (they are kept here)."""

    def __init__(self, radars, grids, ys, interp=BILINEAR, write_volume=False, stream=None):
        lib = load()
        if not (len(radars) == len(grids) == len(ys)) or len(ys) == 0:
            raise ValueError("radars, grids and ys must be non-empty and of equal length")
        self.radars, self.grids = list(radars), list(grids)
        self.ys = [_c64(y) for y in ys]
        dev = self.ys[0].device
        self.nf = len(ys)
        self.interp = int(interp)
        self.blocks = [peaks_tensor(g.n[0] * g.n[1], dev) for g in self.grids]
        self.decs = [torch.empty(tuple(g.n), dtype=torch.float32, device=dev) if write_volume else None
                     for g in self.grids]
        frames = (GhFrame * self.nf)()
        for f in range(self.nf):
            frames[f] = GhFrame(self.radars[f].c_struct, self.grids[f], _ptr(self.ys[f]), _ptr(self.decs[f]),
                                _ptr(self.blocks[f]))
        nb = lib.gh_batch_workspace_bytes(frames, self.nf)
        if nb == 0:
            raise GridHopError(GH_EINVAL, last_error())
        self.ws = torch.empty(nb, dtype=torch.uint8, device=dev)
        self.argmax = peaks_tensor(self.nf, dev)
        h = ctypes.c_void_p()
        _check(lib.gh_batch_create(frames, self.nf, self.interp, _ptr(self.ws), nb, ctypes.byref(h),
                                   _stream(stream)))
        self._h = h

    @classmethod
    def from_scenes(cls, scenes, interp=BILINEAR, write_volume=False, device="cuda:0"):
        radars = [Radar.from_scene(s) for s in scenes]
        grids = [grid_of(s.grid) for s in scenes]
        ys = [torch.from_numpy(s.y).to(device) for s in scenes]
        return cls(radars, grids, ys, interp, write_volume)

    def info(self) -> dict:
        inf = GhBatchInfo()
        _check(load().gh_batch_get_info(self._h, ctypes.byref(inf)))
        return dict(n_frames=inf.n_frames, interp=inf.interp, units=list(inf.units),
                    workgroups=list(inf.workgroups), max_workgroups=list(inf.max_workgroups),
                    sweep_waves=inf.sweep_waves, column_height=inf.column_height,
                    sweep_locations=inf.sweep_locations, range_chirps=inf.range_chirps,
                    doppler_rows=inf.doppler_rows, points=inf.points,
                    workspace_bytes=inf.workspace_bytes)

    def tune(self, range_wg=0, doppler_wg=0, sweep_wg=0, sweep_waves=0):
        _check(load().gh_batch_tune(self._h, int(range_wg), int(doppler_wg), int(sweep_wg), int(sweep_waves)))

    def tune_tiles(self, range_chirps=0, doppler_rows=0, sweep_locations=0, stream=None):
        """Map-pass tiles (0: each frame's planner) and locations per sweep unit (0 keeps);
        re-plans the work units and resets the map passes' workgroup counts."""
        _check(load().gh_batch_tune_tiles(self._h, int(range_chirps), int(doppler_rows), int(sweep_locations),
                                          _stream(stream)))

    def run(self, want_argmax=True, stream=None) -> torch.Tensor:
        _check(load().gh_batch_run(self._h, _ptr(self.argmax) if want_argmax else None, _stream(stream)))
        return self.argmax

    def maps(self, f: int) -> torch.Tensor:
        """Frame f's complex64 maps [K, N_r, N_d] (a view of the workspace)."""
        p = ctypes.c_void_p()
        _check(load().gh_batch_frame_maps(self._h, int(f), ctypes.byref(p)))
        r = self.radars[f]
        off = p.value - self.ws.data_ptr()
        n = r.k * r.nr * r.nd * 8
        return self.ws[off:off + n].view(torch.complex64).view(r.k, r.nr, r.nd)

    def capture(self, want_argmax=True) -> "torch.cuda.CUDAGraph":
        """A HIP graph of one run (kernel launches only), after one eager warm-up run."""
        self.run(want_argmax)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(want_argmax)
        return g

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().gh_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(batch: Batch, reps=3, factors=(0.25, 0.5, 1.0, 2.0), range_chirps=(0, 4, 8, 16),
             doppler_rows=(0, 1, 2, 4, 8), sweep_locations=(1, 2, 4)) -> dict:
    """Coordinate search of the batch's launch shapes: the tiles first (locations
    per sweep unit, then range chirps and Doppler rows per map workgroup, 0 being
    each frame's planner), then sweep waves per workgroup and sweep workgroups
    (as factors of the resident maximum), then the range and Doppler workgroups,
    each setting timed over `reps` runs with HIP events on the current stream.
    Leaves the fastest setting applied; returns it with every trial
    ({"best": {...}, "ms": float, "trials": [...]})."""
    def timed():
        batch.run()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        for _ in range(reps):
            batch.run()
        end.record()
        end.synchronize()
        return start.elapsed_time(end) / reps

    trials = []
    # tiles: each change re-plans the work units and resets the map workgroups to the maximum
    tiles = dict(range_chirps=batch.info()["range_chirps"], doppler_rows=batch.info()["doppler_rows"],
                 sweep_locations=batch.info()["sweep_locations"])
    tiles_ms = None

    def try_tiles(**kw):
        nonlocal tiles, tiles_ms
        cand = dict(tiles, **kw)
        try:
            batch.tune_tiles(cand["range_chirps"], cand["doppler_rows"], cand["sweep_locations"])
        except GridHopError:
            return
        ms = timed()
        trials.append(dict(cand, ms=ms))
        if tiles_ms is None or ms < tiles_ms:
            tiles, tiles_ms = cand, ms

    try_tiles()
    for v in sweep_locations:
        try_tiles(sweep_locations=v)
    for v in range_chirps:
        try_tiles(range_chirps=v)
    for v in doppler_rows:
        try_tiles(doppler_rows=v)
    batch.tune_tiles(tiles["range_chirps"], tiles["doppler_rows"], tiles["sweep_locations"])

    inf = batch.info()
    best = dict(range_wg=inf["workgroups"][0], doppler_wg=inf["workgroups"][1], sweep_wg=inf["workgroups"][2],
                sweep_waves=inf["sweep_waves"])
    best_ms = timed()
    trials.append(dict(best, ms=best_ms))

    def consider(**kw):
        nonlocal best, best_ms
        cand = dict(best, **kw)
        try:
            batch.tune(cand["range_wg"], cand["doppler_wg"], cand["sweep_wg"], cand["sweep_waves"])
        except GridHopError:
            return
        ms = timed()
        trials.append(dict(cand, ms=ms))
        if ms < best_ms:
            best, best_ms = cand, ms

    for waves in (1, 2, 4):
        try:
            batch.tune(sweep_waves=waves)
        except GridHopError:
            continue
        m = batch.info()["max_workgroups"][2]
        for fct in factors:
            consider(sweep_waves=waves, sweep_wg=max(1, int(m * fct)))
    for w, key in ((0, "range_wg"), (1, "doppler_wg")):
        m = batch.info()["max_workgroups"][w]
        for fct in factors:
            consider(**{key: max(1, int(m * fct))})
    batch.tune(best["range_wg"], best["doppler_wg"], best["sweep_wg"], best["sweep_waves"])
    return dict(best=dict(best, **tiles), ms=best_ms, trials=trials)
