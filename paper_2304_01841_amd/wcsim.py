"""Thin ctypes binding of libwcsim (C ABI in include/wcsim.h).

Argument marshalling only: torch tensors supply device memory and streams,
every step of the simulation runs in the HIP library.  Importing this module
loads ``libwcsim.so`` from the package directory and raises ImportError when it
is missing (there is no fallback path).

Names follow the C ABI: :class:`Plane` wraps ``wcsim_plane_create`` and
friends, :func:`rasterize`, :func:`scatter_add`, :func:`convolve` and
:func:`simulate_event` wrap the DepoTransform steps (arXiv:2304.01841, Sec. 2).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwcsim.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libwcsim.so is not built (run paper_2304_01841_amd/build.py): " + LIB_PATH)
_lib = ctypes.CDLL(LIB_PATH)

OK, E_INVALID, E_NOMEM, E_DEVICE, E_STATE = 0, -1, -2, -3, -4
MEM_HOST, MEM_DEVICE = 0, 1
OUT_WIRE, OUT_PITCH = 0, 1


class WcsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("wcsim status %d: %s" % (status, msg))
        self.status = status


class Depo(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double),
                ("t", ctypes.c_double), ("q", ctypes.c_double)]


class Physics(ctypes.Structure):
    _fields_ = [("drift_speed", ctypes.c_double), ("DL", ctypes.c_double),
                ("DT", ctypes.c_double), ("nsigma", ctypes.c_double),
                ("fluctuate", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("lifetime", ctypes.c_double),
                ("drift_accel", ctypes.c_double)]


class PlaneDesc(ctypes.Structure):
    _fields_ = [("plane_id", ctypes.c_int32), ("nwires", ctypes.c_int32),
                ("nimpact", ctypes.c_int32), ("nticks", ctypes.c_int32),
                ("pitch", ctypes.c_double), ("tick", ctypes.c_double), ("t0", ctypes.c_double),
                ("plane_x", ctypes.c_double), ("dir_y", ctypes.c_double),
                ("dir_z", ctypes.c_double), ("pitch_origin", ctypes.c_double),
                ("resp_npitch", ctypes.c_int32), ("resp_nticks", ctypes.c_int32),
                ("resp_origin", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("response", ctypes.POINTER(ctypes.c_float)),
                ("elec_nticks", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("elec_response", ctypes.POINTER(ctypes.c_float))]


class Schedule(ctypes.Structure):
    _fields_ = [("fft_ticks", ctypes.c_int32), ("fft_pitch", ctypes.c_int32),
                ("freq_chunk", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("wire_mode", ctypes.c_int32), ("deterministic", ctypes.c_int32)]


class PlaneInfo(ctypes.Structure):
    _fields_ = [("npitch", ctypes.c_int64), ("nticks", ctypes.c_int64),
                ("nwires", ctypes.c_int64), ("nimpact", ctypes.c_int64),
                ("fft_ticks", ctypes.c_int32), ("fft_pitch", ctypes.c_int32),
                ("freq_chunk", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("nchunks", ctypes.c_int32), ("pitch_blocks", ctypes.c_int32),
                ("tile_pitch", ctypes.c_int32), ("tile_ticks", ctypes.c_int32),
                ("ntiles", ctypes.c_int64), ("spectrum_bytes", ctypes.c_int64),
                ("pitch_cols", ctypes.c_int32), ("wire_fold", ctypes.c_int32),
                ("wire_polyphase", ctypes.c_int32), ("wire_blocks", ctypes.c_int32),
                ("deterministic", ctypes.c_int32)]


_P = ctypes.c_void_p
_i64, _u64, _i32, _sz = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t
_st = ctypes.c_int

# name -> (restype, argtypes)
_SIGS = {
    "wcsim_version": (_i32, []),
    "wcsim_last_error": (ctypes.c_char_p, []),
    "wcsim_plane_create": (_st, [_P, _P, _P, _P]),
    "wcsim_plane_create_with_schedule": (_st, [_P, _P, _P, _P, _P]),
    "wcsim_plane_create_sharing": (_st, [_P, _P, _P, _P, _P]),
    "wcsim_plane_destroy": (None, [_P]),
    "wcsim_plane_get_info": (_st, [_P, _P]),
    "wcsim_rasterize": (_st, [_P, _P, _i64, _i32, _u64, _P, _P]),
    "wcsim_patches_count": (_st, [_P, _P, _P]),
    "wcsim_patches_device": (_st, [_P, _P, _P, _P]),
    "wcsim_patches_copy_to_host": (_st, [_P, _P, _P, _P]),
    "wcsim_patches_destroy": (None, [_P]),
    "wcsim_scatter_add": (_st, [_P, _P, _P, _i32, _P]),
    "wcsim_convolve_workspace_bytes": (_sz, [_P, _i32]),
    "wcsim_convolve": (_st, [_P, _P, _P, _i32, _P, _P]),
    "wcsim_simulate_workspace_bytes": (_sz, [_P, _i64, _i32]),
    "wcsim_simulate_event": (_st, [_P, _P, _i64, _i32, _u64, _P, _i32, _i32, _P, _P]),
    "wcsim_simulate_event_profiled": (_st, [_P, _P, _i64, _i32, _u64, _P, _i32, _i32, _P, _P,
                                            _P]),
    "wcsim_simulate_event_noalloc": (_st, [_P, _P, _i64, _u64, _P, _i32, _P]),
    "wcsim_tune_schedules": (_st, [_P, _P, _P, _i32, _P, _i64, _i32, _i32, _P, _P]),
    "wcsim_workspace_grid": (_P, [_P, _P, _i64]),
    "wcsim_workspace_grid_complete": (_st, [_P, _P, _i64, _P]),
    "wcsim_workspace_invalid_count": (_st, [_P, _P, _P]),
    "wcsim_batch_workspace_bytes": (_sz, [_P, _P, _i32, _i32]),
    "wcsim_simulate_batch": (_st, [_P, _P, _P, _P, _i32, _P, _i32, _P, _P]),
    "wcsim_batch_chunk_count": (_i32, [_P, _P, _i32, _i32]),
    "wcsim_simulate_batch_profiled": (_st, [_P, _P, _P, _P, _i32, _P, _i32, _P, _P, _P, _i32]),
    "wcsim_batch_create": (_st, [_P, _P, _i32, _i32, _P, _P]),
    "wcsim_batch_run": (_st, [_P, _P, _P, _P, _P, _P]),
    "wcsim_batch_destroy": (None, [_P]),
    "wcsim_philox4x32_10": (_st, [_P, _P, _i64, _P, _P]),
    "wcsim_digitize": (_st, [_P, _i64, _i64, ctypes.c_float, ctypes.c_float, ctypes.c_float, _i32,
                             _u64, _u64, _P, _P]),
    "wcsim_digitize_coloured": (_st, [_P, _i64, _i64, ctypes.c_float, ctypes.c_float,
                                      ctypes.c_float, _P, _i32, _i32, _u64, _u64, _P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(status: int):
    if status != OK:
        raise WcsimError(status, _lib.wcsim_last_error().decode(errors="replace"))


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev_ptr(t: torch.Tensor, dtype=None, what="tensor") -> int:
    if not t.is_cuda:
        raise ValueError(what + " must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s" % (what, dtype))
    if not t.is_contiguous():
        raise ValueError(what + " must be contiguous")
    return t.data_ptr()


def version() -> int:
    return _lib.wcsim_version()


def physics_struct(phys: dict) -> Physics:
    return Physics(float(phys["drift_speed"]), float(phys["DL"]), float(phys["DT"]),
                   float(phys["nsigma"]), int(phys["fluctuate"]), 0,
                   int(phys["seed"]) & (2**64 - 1), float(phys.get("lifetime", 0.0)),
                   float(phys.get("drift_accel", 0.0)))


def plane_desc_struct(plane: dict, resp: np.ndarray, r0: int) -> PlaneDesc:
    """wcsim_plane_desc of a plane dict and a contiguous float32 response (the
    caller keeps `resp` alive while the struct is in use).  An optional
    plane["elec_response"] (1-D) is the electronics response; the struct keeps
    its float32 copy alive."""
    Rp, Rt = resp.shape
    elec = plane.get("elec_response")
    e32 = None if elec is None else np.ascontiguousarray(elec, dtype=np.float32).reshape(-1)
    d = PlaneDesc(int(plane["plane_id"]), int(plane["nwires"]), int(plane["nimpact"]),
                  int(plane["nticks"]), float(plane["pitch"]), float(plane["tick"]),
                  float(plane["t0"]), float(plane["plane_x"]), float(plane["dir_y"]),
                  float(plane["dir_z"]), float(plane["pitch_origin"]), Rp, Rt, int(r0), 0,
                  resp.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                  0 if e32 is None else int(e32.size), 0,
                  None if e32 is None else e32.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    d._keep = e32
    return d


def schedule_struct(schedule: dict | None) -> Schedule:
    schedule = schedule or {}
    return Schedule(int(schedule.get("fft_ticks", 0)), int(schedule.get("fft_pitch", 0)),
                    int(schedule.get("freq_chunk", 0)), int(schedule.get("tile", 0)),
                    int(schedule.get("wire_mode", 0)), int(schedule.get("deterministic", 0)))


class Plane:
    """A plane with its resident response spectrum (wcsim_plane)."""

    def __init__(self, plane: dict, phys: dict, response: np.ndarray, r0: int | None = None,
                 schedule: dict | None = None, stream=None, share: "Plane | None" = None):
        resp = np.ascontiguousarray(response, dtype=np.float32)
        Rp, Rt = resp.shape
        if r0 is None:
            r0 = Rp // 2
        self._resp = resp
        d = plane_desc_struct(plane, resp, r0)
        ph = physics_struct(phys)
        h = ctypes.c_void_p()
        if share is not None:
            st = _lib.wcsim_plane_create_sharing(ctypes.byref(d), ctypes.byref(ph), share.handle,
                                                 _stream(stream), ctypes.byref(h))
        elif schedule:
            sc = schedule_struct(schedule)
            st = _lib.wcsim_plane_create_with_schedule(ctypes.byref(d), ctypes.byref(ph),
                                                       ctypes.byref(sc), _stream(stream),
                                                       ctypes.byref(h))
        else:
            st = _lib.wcsim_plane_create(ctypes.byref(d), ctypes.byref(ph), _stream(stream),
                                         ctypes.byref(h))
        _check(st)
        self.handle = h
        self.plane = dict(plane)
        self.phys = dict(phys)
        self.r0 = int(r0)
        info = PlaneInfo()
        _check(_lib.wcsim_plane_get_info(self.handle, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in PlaneInfo._fields_}

    @property
    def npitch(self) -> int:
        return self.info["npitch"]

    @property
    def nticks(self) -> int:
        return self.info["nticks"]

    @property
    def nwires(self) -> int:
        return self.info["nwires"]

    def out_rows(self, kind: int) -> int:
        return self.nwires if kind == OUT_WIRE else self.npitch

    def destroy(self):
        if self.handle:
            _lib.wcsim_plane_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _depo_arg(depos):
    """(pointer, n, mem kind, keepalive) of a depo array ([n, 5] float64)."""
    if isinstance(depos, torch.Tensor):
        if depos.dtype != torch.float64 or depos.dim() != 2 or depos.shape[1] != 5:
            raise ValueError("depos must be a [n, 5] float64 tensor")
        if depos.is_cuda:
            return _dev_ptr(depos, what="depos"), depos.shape[0], MEM_DEVICE, depos
        depos = depos.numpy()
    a = np.ascontiguousarray(depos, dtype=np.float64)
    if a.ndim != 2 or a.shape[1] != 5:
        raise ValueError("depos must be [n, 5]")
    return a.ctypes.data, a.shape[0], MEM_HOST, a


class Patches:
    """Patch set returned by :func:`rasterize` (wcsim_patches)."""

    def __init__(self, handle):
        self.handle = handle
        n, nv = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.wcsim_patches_count(handle, ctypes.byref(n), ctypes.byref(nv)))
        self.ndepos, self.nvalues = n.value, nv.value

    def to_host(self, values: bool = True):
        """(meta [n][4] int32, offsets [n + 1] int64, values float32 or None)."""
        meta = np.zeros((self.ndepos, 4), np.int32)
        offs = np.zeros(self.ndepos + 1, np.int64)
        vals = np.zeros(max(self.nvalues, 1), np.float32) if values else None
        _check(_lib.wcsim_patches_copy_to_host(self.handle, meta.ctypes.data, offs.ctypes.data,
                                               vals.ctypes.data if values else None))
        return meta, offs, (vals[:self.nvalues] if values else None)

    def destroy(self):
        if self.handle:
            _lib.wcsim_patches_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def rasterize(plane: Plane, depos, event_id: int = 0, stream=None) -> Patches:
    ptr, n, mem, _keep = _depo_arg(depos)
    h = ctypes.c_void_p()
    _check(_lib.wcsim_rasterize(plane.handle, ptr, n, mem, int(event_id) & (2**64 - 1),
                                _stream(stream), ctypes.byref(h)))
    return Patches(h)


def scatter_add(plane: Plane, patches: Patches, grid: torch.Tensor, zero_first: bool = True,
                stream=None):
    if tuple(grid.shape) != (plane.npitch, plane.nticks):
        raise ValueError("grid must be [npitch, nticks]")
    _check(_lib.wcsim_scatter_add(plane.handle, patches.handle,
                                  _dev_ptr(grid, torch.float32, "grid"), int(bool(zero_first)),
                                  _stream(stream)))


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def convolve_workspace(plane: Plane, kind: int = OUT_WIRE, device="cuda") -> torch.Tensor:
    return _workspace(_lib.wcsim_convolve_workspace_bytes(plane.handle, kind), device)


def convolve(plane: Plane, grid: torch.Tensor, out: torch.Tensor | None = None,
             kind: int = OUT_WIRE, workspace: torch.Tensor | None = None, stream=None):
    if tuple(grid.shape) != (plane.npitch, plane.nticks):
        raise ValueError("grid must be [npitch, nticks]")
    if out is None:
        out = torch.empty((plane.out_rows(kind), plane.nticks), dtype=torch.float32,
                          device=grid.device)
    if tuple(out.shape) != (plane.out_rows(kind), plane.nticks):
        raise ValueError("out has the wrong shape")
    if workspace is None:
        workspace = convolve_workspace(plane, kind, grid.device)
    _check(_lib.wcsim_convolve(plane.handle, _dev_ptr(grid, torch.float32, "grid"),
                               _dev_ptr(out, torch.float32, "out"), kind,
                               _dev_ptr(workspace, what="workspace"), _stream(stream)))
    return out


def simulate_workspace(plane: Plane, n: int, kind: int = OUT_WIRE, device="cuda") -> torch.Tensor:
    return _workspace(_lib.wcsim_simulate_workspace_bytes(plane.handle, int(n), kind), device)


def workspace_grid(plane: Plane, workspace: torch.Tensor, n: int, complete: bool = True,
                   stream=None) -> torch.Tensor:
    """View of the plane grid left in a simulate workspace by the last event of
    n depos; with `complete` the blocks no depo window reached are zeroed
    first (wcsim_workspace_grid_complete), otherwise they hold stale values."""
    if complete:
        _check(_lib.wcsim_workspace_grid_complete(plane.handle, workspace.data_ptr(), int(n),
                                                  _stream(stream)))
    off = _lib.wcsim_workspace_grid(plane.handle, workspace.data_ptr(), int(n)) - \
        workspace.data_ptr()
    nb = plane.npitch * plane.nticks * 4
    return workspace[off:off + nb].view(torch.float32).view(plane.npitch, plane.nticks)


def workspace_invalid_count(workspace: torch.Tensor, stream=None) -> int:
    c = ctypes.c_int64()
    _check(_lib.wcsim_workspace_invalid_count(workspace.data_ptr(), _stream(stream),
                                              ctypes.byref(c)))
    return c.value


def simulate_event(plane: Plane, depos, event_id: int = 0, out=None, kind: int = OUT_WIRE,
                   workspace: torch.Tensor | None = None, stream=None, device="cuda"):
    """Whole DepoTransform for one event.  `out` may be a CUDA tensor (device
    output), a numpy array (host output) or None (a new CUDA tensor)."""
    ptr, n, mem, _keep = _depo_arg(depos)
    rows = plane.out_rows(kind)
    if out is None:
        out = torch.empty((rows, plane.nticks), dtype=torch.float32, device=device)
    if isinstance(out, torch.Tensor):
        out_ptr, out_mem = _dev_ptr(out, torch.float32, "out"), MEM_DEVICE
    else:
        if out.dtype != np.float32 or not out.flags.c_contiguous:
            raise ValueError("host out must be C-contiguous float32")
        out_ptr, out_mem = out.ctypes.data, MEM_HOST
    if tuple(out.shape) != (rows, plane.nticks):
        raise ValueError("out has the wrong shape")
    if workspace is None:
        workspace = simulate_workspace(plane, n, kind, device)
    need = _lib.wcsim_simulate_workspace_bytes(plane.handle, n, kind)
    if workspace.numel() < need:
        raise ValueError("workspace too small: %d < %d bytes" % (workspace.numel(), need))
    _check(_lib.wcsim_simulate_event(plane.handle, ptr, n, mem, int(event_id) & (2**64 - 1),
                                     out_ptr, kind, out_mem, _dev_ptr(workspace, what="workspace"),
                                     _stream(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def simulate_event_noalloc(plane: Plane, depos: torch.Tensor, event_id: int, out: torch.Tensor,
                           kind: int = OUT_WIRE, stream=None) -> torch.Tensor:
    """wcsim_simulate_event_noalloc: device depos and output, the library's
    fixed device workspace (no allocation in the call)."""
    ptr, n, mem, _keep = _depo_arg(depos)
    if mem != MEM_DEVICE:
        raise ValueError("depos must be a CUDA tensor")
    if tuple(out.shape) != (plane.out_rows(kind), plane.nticks):
        raise ValueError("out has the wrong shape")
    _check(_lib.wcsim_simulate_event_noalloc(plane.handle, ptr, n, int(event_id) & (2**64 - 1),
                                             _dev_ptr(out, torch.float32, "out"), kind,
                                             _stream(stream)))
    return out


NUM_STAGE_EVENTS = 8
STAGE_NAMES = ("clear_grid", "bin_depos", "raster_tiles", "raster_large", "fft_ticks",
               "conv_pitch", "ifft_ticks")


def simulate_event_profiled(plane: Plane, depos: torch.Tensor, event_id: int, out: torch.Tensor,
                            kind: int, workspace: torch.Tensor, events, stream=None):
    """simulate_event (device output) recording the stage events (raw
    hipEvent_t handles, NUM_STAGE_EVENTS of them) on `stream`."""
    ptr, n, mem, _keep = _depo_arg(depos)
    arr = (ctypes.c_void_p * NUM_STAGE_EVENTS)(*events)
    _check(_lib.wcsim_simulate_event_profiled(plane.handle, ptr, n, mem,
                                              int(event_id) & (2**64 - 1),
                                              _dev_ptr(out, torch.float32, "out"), kind,
                                              MEM_DEVICE, _dev_ptr(workspace, what="workspace"),
                                              _stream(stream), arr))
    return out


class HipEvents:
    """Raw HIP events from the HIP runtime (timing enabled)."""

    def __init__(self, count: int):
        self._hip = ctypes.CDLL("libamdhip64.so")
        self._hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self._hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                                  ctypes.c_void_p]
        self._hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.handles = []
        for _ in range(count):
            h = ctypes.c_void_p()
            if self._hip.hipEventCreate(ctypes.byref(h)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.handles.append(h.value)

    def elapsed_ms(self, a: int, b: int) -> float:
        ms = ctypes.c_float()
        if self._hip.hipEventElapsedTime(ctypes.byref(ms), self.handles[a], self.handles[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def destroy(self):
        for h in self.handles:
            self._hip.hipEventDestroy(h)
        self.handles = []


def batch_workspace(planes, ns, kind: int = OUT_WIRE, device="cuda") -> torch.Tensor:
    arr_p = (ctypes.c_void_p * len(planes))(*[p.handle.value for p in planes])
    arr_n = (ctypes.c_int64 * len(ns))(*[int(v) for v in ns])
    return _workspace(_lib.wcsim_batch_workspace_bytes(arr_p, arr_n, len(planes), kind), device)


def simulate_batch(planes, depos_list, event_ids, outs, kind: int = OUT_WIRE,
                   workspace: torch.Tensor | None = None, stream=None):
    ne = len(planes)
    for d in depos_list:
        _dev_ptr(d, torch.float64, "depos")
    arr_p = (ctypes.c_void_p * ne)(*[p.handle.value for p in planes])
    arr_d = (ctypes.c_void_p * ne)(*[d.data_ptr() for d in depos_list])
    arr_n = (ctypes.c_int64 * ne)(*[d.shape[0] for d in depos_list])
    arr_e = (ctypes.c_uint64 * ne)(*[int(e) & (2**64 - 1) for e in event_ids])
    arr_o = (ctypes.c_void_p * ne)(*[_dev_ptr(o, torch.float32, "out") for o in outs])
    if workspace is None:
        workspace = batch_workspace(planes, [d.shape[0] for d in depos_list], kind,
                                    depos_list[0].device)
    _check(_lib.wcsim_simulate_batch(arr_p, arr_d, arr_n, arr_e, ne, arr_o, kind,
                                     _dev_ptr(workspace, what="workspace"), _stream(stream)))
    return outs


BATCH_STAGE_EVENTS = 9
BATCH_STAGE_NAMES = ("bin_depos", "raster_tiles", "raster_large", None, "fft_ticks", "conv_pitch",
                     "ifft_ticks")


def batch_chunk_count(planes, ns, kind: int = OUT_WIRE) -> int:
    arr_p = (ctypes.c_void_p * len(planes))(*[p.handle.value for p in planes])
    arr_n = (ctypes.c_int64 * len(ns))(*[int(v) for v in ns])
    return int(_lib.wcsim_batch_chunk_count(arr_p, arr_n, len(planes), kind))


def simulate_batch_profiled(planes, depos_list, event_ids, outs, events, kind: int = OUT_WIRE,
                            workspace: torch.Tensor | None = None, stream=None):
    """simulate_batch recording BATCH_STAGE_EVENTS raw hipEvent_t handles per
    chunk (see wcsim_simulate_batch_profiled)."""
    ne = len(planes)
    for d in depos_list:
        _dev_ptr(d, torch.float64, "depos")
    arr_p = (ctypes.c_void_p * ne)(*[p.handle.value for p in planes])
    arr_d = (ctypes.c_void_p * ne)(*[d.data_ptr() for d in depos_list])
    arr_n = (ctypes.c_int64 * ne)(*[d.shape[0] for d in depos_list])
    arr_e = (ctypes.c_uint64 * ne)(*[int(e) & (2**64 - 1) for e in event_ids])
    arr_o = (ctypes.c_void_p * ne)(*[_dev_ptr(o, torch.float32, "out") for o in outs])
    arr_v = (ctypes.c_void_p * len(events))(*events)
    if workspace is None:
        workspace = batch_workspace(planes, [d.shape[0] for d in depos_list], kind,
                                    depos_list[0].device)
    _check(_lib.wcsim_simulate_batch_profiled(arr_p, arr_d, arr_n, arr_e, ne, arr_o, kind,
                                              _dev_ptr(workspace, what="workspace"),
                                              _stream(stream), arr_v, len(events)))
    return outs


class Batch:
    """hipGraph-captured batch (wcsim_batch_create / wcsim_batch_run): events
    on `planes` with up to `capacity[e]` depos each."""

    def __init__(self, planes, capacity, kind: int = OUT_WIRE, device="cuda"):
        self.planes = list(planes)
        self.kind = kind
        ne = len(self.planes)
        arr_p = (ctypes.c_void_p * ne)(*[p.handle.value for p in self.planes])
        arr_c = (ctypes.c_int64 * ne)(*[int(c) for c in capacity])
        nbytes = _lib.wcsim_batch_workspace_bytes(arr_p, arr_c, ne, kind)
        self.workspace = _workspace(nbytes, device)
        h = ctypes.c_void_p()
        _check(_lib.wcsim_batch_create(arr_p, arr_c, ne, kind,
                                       _dev_ptr(self.workspace, what="workspace"),
                                       ctypes.byref(h)))
        self.handle = h

    def run(self, depos_list, event_ids, outs, stream=None):
        ne = len(self.planes)
        for d in depos_list:
            _dev_ptr(d, torch.float64, "depos")
        arr_d = (ctypes.c_void_p * ne)(*[d.data_ptr() for d in depos_list])
        arr_n = (ctypes.c_int64 * ne)(*[d.shape[0] for d in depos_list])
        arr_e = (ctypes.c_uint64 * ne)(*[int(e) & (2**64 - 1) for e in event_ids])
        arr_o = (ctypes.c_void_p * ne)(*[_dev_ptr(o, torch.float32, "out") for o in outs])
        _check(_lib.wcsim_batch_run(self.handle, arr_d, arr_n, arr_e, arr_o, _stream(stream)))
        return outs

    def destroy(self):
        if self.handle:
            _lib.wcsim_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def digitize(wave: torch.Tensor, gain: float, pedestal: float, sigma: float = 0.0, bits: int = 12,
             seed: int = 0, event_id: int = 0, out: torch.Tensor | None = None,
             stream=None, fir: torch.Tensor | None = None) -> torch.Tensor:
    """ADC codes of a [nrows, ncols] float32 device waveform (wcsim_digitize,
    or wcsim_digitize_coloured with `fir`, a float32 device tensor of noise
    filter taps): uint16 codes returned as an int16 tensor of the same bit
    patterns."""
    if wave.dim() != 2:
        raise ValueError("wave must be [nrows, ncols]")
    nrows, ncols = wave.shape
    if out is None:
        out = torch.empty((nrows, ncols), dtype=torch.int16, device=wave.device)
    elif tuple(out.shape) != (nrows, ncols):
        raise ValueError("out must be [nrows, ncols]")
    common = (float(gain), float(pedestal), float(sigma))
    tail = (int(seed) & (2**64 - 1), int(event_id) & (2**64 - 1),
            _dev_ptr(out, torch.int16, "out"), _stream(stream))
    if fir is None:
        _check(_lib.wcsim_digitize(_dev_ptr(wave, torch.float32, "wave"), nrows, ncols, *common,
                                   int(bits), *tail))
    else:
        _check(_lib.wcsim_digitize_coloured(_dev_ptr(wave, torch.float32, "wave"), nrows, ncols,
                                            *common, _dev_ptr(fir, torch.float32, "fir"),
                                            int(fir.numel()), int(bits), *tail))
    return out


def philox4x32_10(ctr: torch.Tensor, key: torch.Tensor, stream=None) -> torch.Tensor:
    """GPU Philox4x32-10 of n counters ([n, 4] int32 bit patterns) and keys
    ([n, 2]); returns [n, 4] int32 bit patterns."""
    n = ctr.shape[0]
    out = torch.empty_like(ctr)
    _check(_lib.wcsim_philox4x32_10(_dev_ptr(ctr, torch.int32, "ctr"),
                                    _dev_ptr(key, torch.int32, "key"), n,
                                    _dev_ptr(out, torch.int32, "out"), _stream(stream)))
    return out


def tune_schedules(plane: dict, phys: dict, response: np.ndarray, depos: torch.Tensor,
                   candidates: list, r0: int | None = None, kind: int = OUT_WIRE, reps: int = 5,
                   stream=None) -> list:
    """Median ms per event of wcsim_simulate_event under each candidate
    schedule (dicts with fft_ticks, fft_pitch, freq_chunk, tile; 0 or absent =
    default), -1.0 for a candidate that is invalid for this plane."""
    resp = np.ascontiguousarray(response, dtype=np.float32)
    if r0 is None:
        r0 = resp.shape[0] // 2
    d = plane_desc_struct(plane, resp, r0)
    ph = physics_struct(phys)
    arr = (Schedule * len(candidates))(*[schedule_struct(c) for c in candidates])
    ms = (ctypes.c_float * len(candidates))()
    if depos.dtype != torch.float64 or depos.dim() != 2 or depos.shape[1] != 5:
        raise ValueError("depos must be a [n, 5] float64 tensor")
    n = int(depos.shape[0])
    ptr = _dev_ptr(depos, torch.float64, "depos") if n else None
    _check(_lib.wcsim_tune_schedules(ctypes.byref(d), ctypes.byref(ph), arr, len(candidates), ptr,
                                     n, int(kind), int(reps), _stream(stream), ms))
    return [float(v) for v in ms]
