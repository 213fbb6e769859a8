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
BILINEAR, BICUBIC = 0, 1
GEMM_F32, GEMM_BF16 = 0, 1
MAP_C64, MAP_F16, MAP_BF16 = 0, 1, 2
MAX_SUPPORT = 32

EXPORTS = ("gh_abi_version", "gh_last_error", "gh_rd_maps", "gh_decision", "gh_argmax", "gh_direct_workspace_bytes",
           "gh_direct_decision", "gh_bomp_workspace_bytes", "gh_bomp_step", "gh_refine_workspace_bytes",
           "gh_refine", "gh_direct_points_workspace_bytes", "gh_direct_points", "gh_gh_points")


class GhRadar(ctypes.Structure):
    _fields_ = [("f0_hz", ctypes.c_double), ("bandwidth_hz", ctypes.c_double), ("t_chirp_s", ctypes.c_double),
                ("c_mps", ctypes.c_double), ("n_samples", ctypes.c_int32), ("n_chirps", ctypes.c_int32),
                ("pad_range", ctypes.c_int32), ("pad_doppler", ctypes.c_int32), ("n_rx", ctypes.c_int32),
                ("centered", ctypes.c_int32), ("tx", ctypes.c_double * 2), ("rx", ctypes.POINTER(ctypes.c_double))]


class GhGrid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 4), ("hi", ctypes.c_double * 4), ("n", ctypes.c_int32 * 4)]


class GhPeak(ctypes.Structure):
    _fields_ = [("value", ctypes.c_float), ("reserved", ctypes.c_int32), ("index", ctypes.c_int64)]


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
    lib.gh_refine_workspace_bytes.argtypes = [rp, gp_, i32]
    lib.gh_refine_workspace_bytes.restype = sz
    lib.gh_refine.argtypes = [rp, gp_, vp, vp, i32, i32, vp, sz, vp, vp]
    lib.gh_direct_points_workspace_bytes.argtypes = [rp, i32]
    lib.gh_direct_points_workspace_bytes.restype = sz
    lib.gh_direct_points.argtypes = [rp, vp, vp, i32, vp, vp, vp, vp, sz, vp]
    lib.gh_gh_points.argtypes = [rp, vp, i32, i32, vp, i32, vp, vp, vp, vp]
    for name in ("gh_rd_maps", "gh_decision", "gh_argmax", "gh_direct_decision", "gh_bomp_step", "gh_refine",
                 "gh_direct_points", "gh_gh_points"):
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

    def reset(self):
        self.resid.copy_(self.y)
        self.n = 0

    def step(self, stream=None):
        lib = load()
        _check(lib.gh_bomp_step(ctypes.byref(self.radar.c_struct), ctypes.byref(self.grid), _ptr(self.y),
                                _ptr(self.resid), _ptr(self.maps), self.use_direct, self.interp, self.gemm,
                                _ptr(self.support), self.n, self.max_support, _ptr(self.alpha), _ptr(self.selected),
                                _ptr(self.ws), self.ws.numel(), _stream(stream)))
        self.n += 1


def refine_workspace_bytes(radar: Radar, grid: GhGrid, n_cells: int) -> int:
    n = load().gh_refine_workspace_bytes(ctypes.byref(radar.c_struct), ctypes.byref(grid), int(n_cells))
    if n == 0:
        raise GridHopError(GH_EINVAL, last_error())
    return n


def refine(radar: Radar, grid: GhGrid, y, cells: torch.Tensor, max_iter=20, theta=None, ws=None, stream=None):
    lib = load()
    _c64(y)
    if cells.dtype != torch.int64 or not cells.is_cuda:
        raise ValueError("cells must be an int64 CUDA tensor")
    if theta is None:
        theta = torch.empty((cells.numel(), 4), dtype=torch.float64, device=y.device)
    if ws is None and cells.numel() > 0:
        ws = torch.empty(refine_workspace_bytes(radar, grid, cells.numel()), dtype=torch.uint8, device=y.device)
    nws = 0 if ws is None else ws.numel()
    _check(lib.gh_refine(ctypes.byref(radar.c_struct), ctypes.byref(grid), _ptr(y), _ptr(cells), cells.numel(),
                         int(max_iter), _ptr(ws), nws, _ptr(theta), _stream(stream)))
    return theta


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

