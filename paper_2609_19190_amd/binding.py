"""Thin ctypes binding of libflashrad.so (include/fr.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  torch tensors are used for device memory and
streams; their data pointers are passed to the C ABI.  There is no CPU
fallback: if the library is missing this module raises on load.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library binds to the HIP runtime torch uses

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflashrad.so")

FR_OK, FR_E_ARG, FR_E_EMPTY_MASK, FR_E_RANGE, FR_E_NOMEM, FR_E_DEVICE, FR_E_CAPACITY = (
    0, -1, -2, -3, -4, -5, -6)
FR_E_TIMEOUT, FR_E_CANCELLED = -7, -8
# admission replay: event kinds and outcomes
FR_ADMIT_SUBMIT, FR_ADMIT_CANCEL, FR_ADMIT_COMPLETE, FR_ADMIT_FAIL_NEXT = 0, 1, 2, 3
FR_ADMITTED, FR_ADMIT_EXPIRED, FR_ADMIT_CANCELLED, FR_ADMIT_ALLOC_FAILED, FR_ADMIT_REJECTED = (
    0, 1, 2, 3, 4)
FR_I16, FR_F32 = 1, 2
FR_FBW, FR_FBN = 1, 2
FR_FIRSTORDER, FR_GLCM, FR_GLRLM, FR_GLSZM, FR_GLDM, FR_NGTDM, FR_ALL = 1, 2, 4, 8, 16, 32, 63

FR_MERGED, FR_AVERAGED = 0, 1

EXPORTED = ("fr_discretise", "fr_map_count", "fr_map_name", "fr_map", "fr_map_ex", "fr_map_status",
            "fr_map_noalloc",
            "fr_map_matrices",
            "fr_scalar", "fr_scalar_last_error",
            "fr_batch_create", "fr_batch_destroy", "fr_batch_prepare", "fr_batch_launch",
            "fr_batch_status", "fr_batch_autotune", "fr_batch_describe", "fr_batch_last_error",
            "fr_server_create", "fr_server_footprint", "fr_server_submit", "fr_server_submit_ex",
            "fr_server_cancel", "fr_server_inject_alloc_failures", "fr_server_poll",
            "fr_server_wait", "fr_server_result", "fr_server_release", "fr_server_stats",
            "fr_server_copy", "fr_server_destroy", "fr_server_last_error", "fr_admission_replay",
            "fr_profile_enable", "fr_profile_read", "fr_last_error", "fr_version",
            "fr_source_hash")


class FrJob(ctypes.Structure):
    """struct fr_job (include/fr.h), field for field."""
    _fields_ = [("volume", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("out_maps", ctypes.c_void_p), ("out_capacity_floats", ctypes.c_int64),
                ("n_mask", ctypes.c_int64), ("spacing_mm", ctypes.c_double * 3),
                ("disc_value", ctypes.c_double), ("disc_lower", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("disc_mode", ctypes.c_int32),
                ("kernel_radius", ctypes.c_int32), ("families", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)]


class FrMapOptions(ctypes.Structure):
    """struct fr_map_options (include/fr.h)."""
    _fields_ = [("glcm_distance", ctypes.c_int32), ("gldm_alpha", ctypes.c_int32),
                ("aggregation", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def map_options(glcm_distance: int = 1, gldm_alpha: int = 0, aggregation: int = FR_MERGED):
    return FrMapOptions(glcm_distance=glcm_distance, gldm_alpha=gldm_alpha, aggregation=aggregation,
                        reserved=0)


class FrServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("slots", ctypes.c_int32),
                ("max_bypass", ctypes.c_int32)]


class FrSubmitOptions(ctypes.Structure):
    _fields_ = [("deadline_ms", ctypes.c_double), ("reserved", ctypes.c_int32 * 2)]


class FrAdmitEvent(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("deadline_ms", ctypes.c_double),
                ("ticket", ctypes.c_int64), ("bytes", ctypes.c_int64),
                ("kind", ctypes.c_int32), ("value", ctypes.c_int32)]


class FrAdmitRecord(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("ticket", ctypes.c_int64), ("offset", ctypes.c_int64),
                ("outcome", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class FrResult(ctypes.Structure):
    _fields_ = [("maps", ctypes.c_void_p), ("n_mask", ctypes.c_int64),
                ("footprint_bytes", ctypes.c_int64), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("done", ctypes.c_int32), ("status", ctypes.c_int32), ("ng", ctypes.c_int32),
                ("count", ctypes.c_int32)]


class FrServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("mapped_voxels", ctypes.c_int64),
                ("arena_bytes", ctypes.c_int64), ("arena_used_bytes", ctypes.c_int64),
                ("arena_peak_bytes", ctypes.c_int64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("slots", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("inflight", ctypes.c_int32)]


class FrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'` "
                              "(no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, I64, D, U = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                             ctypes.c_uint32)
        L.fr_discretise.argtypes = [P, I32, I32, I32, I32, P, I32, D, D, P, P, P, P, P, P]
        L.fr_discretise.restype = I32
        L.fr_map_count.argtypes = [U]
        L.fr_map_count.restype = I32
        L.fr_map_name.argtypes = [U, I32]
        L.fr_map_name.restype = ctypes.c_char_p
        L.fr_map.argtypes = [P, I32, I32, I32, I32, P, P, I32, D, D, I32, U, I64, P, I64, P]
        L.fr_map.restype = I32
        L.fr_map_ex.argtypes = [P, I32, I32, I32, I32, P, P, I32, D, D, I32, U, P, I64, P, I64, P]
        L.fr_map_ex.restype = I32
        L.fr_map_status.argtypes = [P, P]
        L.fr_map_status.restype = I32
        L.fr_map_noalloc.argtypes = [P, I32, I32, I32, I32, P, P, I32, D, D, I32, U, I64, P, I64, P]
        L.fr_map_noalloc.restype = I32
        L.fr_map_matrices.argtypes = [P, I32, I32, I32, I32, P, P, I32, D, D, I32, U, P, I64, P, I64,
                                      I32, P, P, P, P, P, P, P, P, P]
        L.fr_map_matrices.restype = I32
        for name, args in (("fr_batch_create", [P]), ("fr_batch_destroy", [P]),
                           ("fr_batch_prepare", [P, P, I32]), ("fr_batch_launch", [P, P, I32]),
                           ("fr_batch_status", [P, P, P, P]), ("fr_batch_autotune", [P, P]),
                           ("fr_batch_describe", [P, P, P, I32])):
            getattr(L, name).argtypes = args
            getattr(L, name).restype = I32
        L.fr_batch_last_error.restype = ctypes.c_char_p
        for name, args in (("fr_server_create", [P, P]), ("fr_server_footprint", [P, P]),
                           ("fr_server_submit", [P, P, P]), ("fr_server_submit_ex", [P, P, P, P]),
                           ("fr_server_cancel", [P, I64]),
                           ("fr_server_inject_alloc_failures", [P, I32]),
                           ("fr_admission_replay", [I64, I32, I32, P, I32, P, I32, P]),
                           ("fr_server_poll", [P, P, I32, P]),
                           ("fr_server_wait", [P, I64, D]), ("fr_server_result", [P, I64, P]),
                           ("fr_server_release", [P, I64]), ("fr_server_stats", [P, P]),
                           ("fr_server_copy", [P, I64, P, I64, P]),
                           ("fr_server_destroy", [P])):
            getattr(L, name).argtypes = args
            getattr(L, name).restype = I32
        L.fr_server_last_error.restype = ctypes.c_char_p
        L.fr_scalar.argtypes = [P, I32, I32, I32, I32, P, P, I32, D, D, U, P, I32]
        L.fr_scalar.restype = I32
        L.fr_scalar_last_error.restype = ctypes.c_char_p
        L.fr_profile_enable.argtypes = [I32]
        L.fr_profile_enable.restype = I32
        L.fr_profile_read.argtypes = [P, P]
        L.fr_profile_read.restype = I32
        L.fr_last_error.restype = ctypes.c_char_p
        L.fr_version.restype = ctypes.c_char_p
        L.fr_source_hash.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != FR_OK:
        raise FrError(rc, lib().fr_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype(vol: torch.Tensor) -> int:
    if vol.dtype == torch.int16:
        return FR_I16
    if vol.dtype == torch.float32:
        return FR_F32
    raise TypeError(f"volume dtype {vol.dtype}: int16 or float32 expected")


def _dev3(vol: torch.Tensor, mask: torch.Tensor):
    if vol.dim() != 3 or mask.shape != vol.shape:
        raise ValueError("volume and mask must be 3-D tensors of the same shape [nz][ny][nx]")
    if not (vol.is_cuda and mask.is_cuda):
        raise ValueError("volume and mask must be device tensors")
    if mask.dtype != torch.uint8:
        raise TypeError("mask must be uint8")
    if not (vol.is_contiguous() and mask.is_contiguous()):
        raise ValueError("volume and mask must be contiguous")
    nz, ny, nx = vol.shape
    return nx, ny, nz


def fr_discretise(volume: torch.Tensor, mask: torch.Tensor, mode: int, value: float,
                  lower: float = float("nan"), levels: torch.Tensor | None = None, stream=None):
    """Returns (levels uint8 tensor, ng, xmin, xmax, n_mask)."""
    nx, ny, nz = _dev3(volume, mask)
    if levels is None:
        levels = torch.empty_like(mask)
    ng, n = ctypes.c_int32(), ctypes.c_int64()
    xmin, xmax = ctypes.c_double(), ctypes.c_double()
    _check(lib().fr_discretise(volume.data_ptr(), _dtype(volume), nx, ny, nz, mask.data_ptr(),
                               mode, float(value), float(lower), levels.data_ptr(),
                               ctypes.byref(ng), ctypes.byref(xmin), ctypes.byref(xmax),
                               ctypes.byref(n), _stream(stream)))
    return levels, ng.value, xmin.value, xmax.value, n.value


def fr_map_count(families: int) -> int:
    return lib().fr_map_count(families)


def fr_map_name(families: int, k: int) -> str:
    s = lib().fr_map_name(families, k)
    if s is None:
        raise IndexError(k)
    return s.decode()


def fr_map(volume: torch.Tensor, mask: torch.Tensor, spacing, mode: int, value: float,
           lower: float, radius: int, families: int, n_mask: int,
           out: torch.Tensor | None = None, stream=None, options: FrMapOptions | None = None
           ) -> torch.Tensor:
    """Maps [count][n_mask] float32 on the device, enqueued on `stream` without
    waiting (fr_map_ex when options are given).  Data errors found on the
    device are reported by fr_map_check / fr_map_status."""
    nx, ny, nz = _dev3(volume, mask)
    count = fr_map_count(families)
    if out is None:
        out = torch.empty((count, n_mask), dtype=torch.float32, device=volume.device)
    sp = (ctypes.c_double * 3)(*[float(s) for s in spacing])
    if options is None:
        _check(lib().fr_map(volume.data_ptr(), _dtype(volume), nx, ny, nz, mask.data_ptr(), sp, mode,
                            float(value), float(lower), radius, families, n_mask, out.data_ptr(),
                            out.numel(), _stream(stream)))
    else:
        _check(lib().fr_map_ex(volume.data_ptr(), _dtype(volume), nx, ny, nz, mask.data_ptr(), sp,
                               mode, float(value), float(lower), radius, families,
                               ctypes.byref(options), n_mask, out.data_ptr(), out.numel(),
                               _stream(stream)))
    return out


def fr_map_noalloc(volume: torch.Tensor, mask: torch.Tensor, spacing, mode: int, value: float,
                   lower: float, radius: int, families: int, n_mask: int, out: torch.Tensor,
                   stream=None) -> torch.Tensor:
    """fr_map without any device allocation: the caller provides `out`
    ([count][n_mask] float32 on the device); the library's fixed scratch
    array holds everything else."""
    nx, ny, nz = _dev3(volume, mask)
    sp = (ctypes.c_double * 3)(*[float(s) for s in spacing])
    _check(lib().fr_map_noalloc(volume.data_ptr(), _dtype(volume), nx, ny, nz, mask.data_ptr(), sp,
                                mode, float(value), float(lower), radius, families, n_mask,
                                out.data_ptr(), out.numel(), _stream(stream)))
    return out


def fr_map_status(stream=None):
    """(status, Ng) of the last map enqueued on this device (synchronises)."""
    ng = ctypes.c_int32()
    rc = lib().fr_map_status(_stream(stream), ctypes.byref(ng))
    return rc, ng.value


def fr_map_check(stream=None) -> int:
    """Synchronise and raise FrError if the last map failed a device-side data
    check; returns the VOI Ng."""
    rc, ng = fr_map_status(stream)
    _check(rc)
    return ng


def fr_map_matrices(volume: torch.Tensor, mask: torch.Tensor, spacing, mode: int, value: float,
                    lower: float, radius: int, families: int, n_mask: int,
                    sample: torch.Tensor, ng: int, stream=None,
                    options: FrMapOptions | None = None) -> dict:
    """Dense integer matrices (and maps) of the sampled mask voxels."""
    nx, ny, nz = _dev3(volume, mask)
    dev = volume.device
    ns = sample.numel()
    S = 2 * radius + 1
    t = lambda *shape, dt=torch.int32: torch.empty(shape, dtype=dt, device=dev)
    res = dict(glcm=t(ns, ng, ng), glrlm=t(ns, ng, S), glszm=t(ns, ng, S ** 3), gldm=t(ns, ng, 27),
               ngtdm_n=t(ns, ng), ngtdm_S=t(ns, ng, dt=torch.int64), hist=t(ns, ng),
               maps=torch.empty((fr_map_count(families), ns), dtype=torch.float32, device=dev))
    sp = (ctypes.c_double * 3)(*[float(s) for s in spacing])
    sample = sample.to(device=dev, dtype=torch.int64).contiguous()
    _check(lib().fr_map_matrices(volume.data_ptr(), _dtype(volume), nx, ny, nz, mask.data_ptr(),
                                 sp, mode, float(value), float(lower), radius, families,
                                 ctypes.byref(options) if options is not None else None, n_mask,
                                 sample.data_ptr(), ns, ng, res["glcm"].data_ptr(),
                                 res["glrlm"].data_ptr(), res["glszm"].data_ptr(),
                                 res["gldm"].data_ptr(), res["ngtdm_n"].data_ptr(),
                                 res["ngtdm_S"].data_ptr(), res["hist"].data_ptr(),
                                 res["maps"].data_ptr(), _stream(stream)))
    return res


def fr_scalar(volume, mask, spacing, mode: int, value: float, lower: float,
              families: int):
    """Whole-VOI features (FP64, host) of numpy arrays [nz][ny][nx]; returns
    a numpy float64 vector in fr_map_name order."""
    import numpy as np
    vol = np.ascontiguousarray(volume)
    msk = np.ascontiguousarray(mask, dtype=np.uint8)
    if vol.dtype == np.int16:
        dt = FR_I16
    elif vol.dtype == np.float32:
        dt = FR_F32
    else:
        raise TypeError(f"volume dtype {vol.dtype}: int16 or float32 expected")
    if vol.ndim != 3 or msk.shape != vol.shape:
        raise ValueError("volume and mask must be 3-D arrays of the same shape")
    nz, ny, nx = vol.shape
    out = np.empty(max(fr_map_count(families), 1), np.float64)
    sp = (ctypes.c_double * 3)(*[float(s) for s in spacing])
    rc = lib().fr_scalar(vol.ctypes.data, dt, nx, ny, nz, msk.ctypes.data, sp, mode, float(value),
                         float(lower), families, out.ctypes.data, out.size)
    if rc != FR_OK:
        raise FrError(rc, lib().fr_scalar_last_error().decode())
    return out[:fr_map_count(families)]


def _bcheck(rc: int):
    if rc != FR_OK:
        raise FrError(rc, lib().fr_batch_last_error().decode())


def fr_batch_create() -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _bcheck(lib().fr_batch_create(ctypes.byref(h)))
    return h


def fr_batch_destroy(h) -> None:
    _bcheck(lib().fr_batch_destroy(h))


def fr_batch_prepare(h, jobs) -> None:
    """jobs: sequence of FrJob."""
    arr = (FrJob * len(jobs))(*jobs)
    _bcheck(lib().fr_batch_prepare(h, arr, len(jobs)))


def fr_batch_launch(h, stream=None, use_graph: bool = False) -> None:
    _bcheck(lib().fr_batch_launch(h, _stream(stream), 1 if use_graph else 0))


def fr_batch_status(h, n_jobs: int, stream=None):
    """(rc, per-job status list, per-job Ng list); rc < 0 if any job failed."""
    st = (ctypes.c_int32 * n_jobs)()
    ng = (ctypes.c_int32 * n_jobs)()
    rc = lib().fr_batch_status(h, st, ng, _stream(stream))
    if rc not in (FR_OK, FR_E_RANGE):
        _bcheck(rc)
    return rc, list(st), list(ng)


def fr_batch_autotune(h, stream=None) -> None:
    _bcheck(lib().fr_batch_autotune(h, _stream(stream)))


def fr_batch_describe(h):
    """List of per-variant dicts of the prepared plan."""
    nv = ctypes.c_int32()
    _bcheck(lib().fr_batch_describe(h, ctypes.byref(nv), None, 0))
    tab = (ctypes.c_int32 * (8 * max(nv.value, 1)))()
    _bcheck(lib().fr_batch_describe(h, ctypes.byref(nv), tab, len(tab)))
    keys = ("dtype", "radius", "lcap", "jobs", "items", "vpw", "grid", "kernel_lmax")
    return [dict(zip(keys, tab[8 * i:8 * i + 8])) for i in range(nv.value)]


class Batch:
    """A prepared batch of VOIs: fr_batch_* with the job tensors kept alive.

    jobs: sequence of dicts with keys volume, mask (device tensors), spacing,
    mode, value, lower, radius, families, n_mask and optionally out (device
    float32 [count][n_mask]); outputs are allocated when absent.
    """

    def __init__(self, jobs):
        self.h = fr_batch_create()
        self.keep, self.outs, structs = [], [], []
        for j in jobs:
            nx, ny, nz = _dev3(j["volume"], j["mask"])
            count = fr_map_count(j["families"])
            out = j.get("out")
            if out is None:
                out = torch.empty((count, j["n_mask"]), dtype=torch.float32,
                                  device=j["volume"].device)
            self.keep += [j["volume"], j["mask"], out]
            self.outs.append(out)
            structs.append(FrJob(volume=j["volume"].data_ptr(), mask=j["mask"].data_ptr(),
                                 out_maps=out.data_ptr(), out_capacity_floats=out.numel(),
                                 n_mask=j["n_mask"],
                                 spacing_mm=(ctypes.c_double * 3)(*map(float, j["spacing"])),
                                 disc_value=float(j["value"]), disc_lower=float(j["lower"]),
                                 dtype=_dtype(j["volume"]), nx=nx, ny=ny, nz=nz,
                                 disc_mode=j["mode"], kernel_radius=j["radius"],
                                 families=j["families"], reserved=0))
        self.n = len(structs)
        try:
            fr_batch_prepare(self.h, structs)
        except Exception:
            self.close()
            raise

    def launch(self, stream=None, use_graph: bool = False):
        fr_batch_launch(self.h, stream, use_graph)

    def status(self, stream=None):
        return fr_batch_status(self.h, self.n, stream)

    def autotune(self, stream=None):
        fr_batch_autotune(self.h, stream)

    def describe(self):
        return fr_batch_describe(self.h)

    def close(self):
        if self.h is not None:
            torch.cuda.synchronize()
            fr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(rc: int):
    if rc != FR_OK:
        raise FrError(rc, lib().fr_server_last_error().decode())


def make_job(volume: torch.Tensor, mask: torch.Tensor, spacing, mode: int, value: float,
             lower: float, radius: int, families: int, n_mask: int, out=None) -> FrJob:
    """An FrJob for device tensors (out=None: no output buffer, as served jobs)."""
    nx, ny, nz = _dev3(volume, mask)
    return FrJob(volume=volume.data_ptr(), mask=mask.data_ptr(),
                 out_maps=out.data_ptr() if out is not None else None,
                 out_capacity_floats=out.numel() if out is not None else 0, n_mask=n_mask,
                 spacing_mm=(ctypes.c_double * 3)(*map(float, spacing)), disc_value=float(value),
                 disc_lower=float(lower), dtype=_dtype(volume), nx=nx, ny=ny, nz=nz,
                 disc_mode=mode, kernel_radius=radius, families=families, reserved=0)


def fr_server_create(hbm_budget_bytes: int, slots: int = 4, max_bypass: int = 0):
    h = ctypes.c_void_p()
    cfg = FrServerConfig(hbm_budget_bytes=int(hbm_budget_bytes), slots=int(slots),
                         max_bypass=int(max_bypass))
    _scheck(lib().fr_server_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def fr_server_footprint(job: FrJob) -> int:
    b = ctypes.c_int64()
    _scheck(lib().fr_server_footprint(ctypes.byref(job), ctypes.byref(b)))
    return b.value


def fr_server_submit(h, job: FrJob, deadline_ms: float = 0.0) -> int:
    t = ctypes.c_int64()
    if deadline_ms:
        opt = FrSubmitOptions(deadline_ms=float(deadline_ms))
        _scheck(lib().fr_server_submit_ex(h, ctypes.byref(job), ctypes.byref(opt), ctypes.byref(t)))
    else:
        _scheck(lib().fr_server_submit(h, ctypes.byref(job), ctypes.byref(t)))
    return t.value


def fr_server_cancel(h, ticket: int) -> None:
    _scheck(lib().fr_server_cancel(h, ticket))


def fr_server_inject_alloc_failures(h, n: int) -> None:
    _scheck(lib().fr_server_inject_alloc_failures(h, n))


def fr_admission_replay(budget_bytes: int, slots: int, max_bypass: int, events):
    """Replay the admission policy in virtual time (host only, no device).
    events: sequence of dicts with keys t, kind and, by kind, ticket, bytes,
    deadline_ms, value.  Returns the records as (t, ticket, offset, outcome)."""
    ev = (FrAdmitEvent * max(len(events), 1))()
    for i, e in enumerate(events):
        ev[i] = FrAdmitEvent(t=float(e["t"]), deadline_ms=float(e.get("deadline_ms", 0.0)),
                             ticket=int(e.get("ticket", 0)), bytes=int(e.get("bytes", 0)),
                             kind=int(e["kind"]), value=int(e.get("value", 0)))
    cap = 4 * len(events) + 4
    rec = (FrAdmitRecord * cap)()
    n = ctypes.c_int32()
    _scheck(lib().fr_admission_replay(int(budget_bytes), int(slots), int(max_bypass), ev,
                                      len(events), rec, cap, ctypes.byref(n)))
    return [(r.t, r.ticket, r.offset, r.outcome) for r in rec[:n.value]]


def fr_server_poll(h, max_tickets: int = 256):
    buf = (ctypes.c_int64 * max_tickets)()
    n = ctypes.c_int32()
    _scheck(lib().fr_server_poll(h, buf, max_tickets, ctypes.byref(n)))
    return list(buf[:n.value])


def fr_server_wait(h, ticket: int, timeout_ms: float = -1.0) -> None:
    _scheck(lib().fr_server_wait(h, ticket, float(timeout_ms)))


def fr_server_result(h, ticket: int) -> FrResult:
    r = FrResult()
    _scheck(lib().fr_server_result(h, ticket, ctypes.byref(r)))
    return r


def fr_server_release(h, ticket: int) -> None:
    _scheck(lib().fr_server_release(h, ticket))


def fr_server_stats(h) -> dict:
    info = FrServerInfo()
    _scheck(lib().fr_server_stats(h, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in FrServerInfo._fields_}


def fr_server_destroy(h) -> None:
    _scheck(lib().fr_server_destroy(h))


def fr_server_copy(h, ticket: int, dst: torch.Tensor, stream=None) -> None:
    """Copy a finished job's maps into dst (float32, >= count * n_mask
    elements, device or host), asynchronously on `stream`."""
    if dst.dtype != torch.float32 or not dst.is_contiguous():
        raise TypeError("dst must be a contiguous float32 tensor")
    st = _stream(stream) if dst.is_cuda else ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _scheck(lib().fr_server_copy(h, ticket, dst.data_ptr(), dst.numel(), st))


class Server:
    """fr_server_* with the submitted input tensors kept alive until release."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 4, max_bypass: int = 0):
        self.h = fr_server_create(hbm_budget_bytes, slots, max_bypass)
        self.inputs = {}

    def submit(self, volume, mask, spacing, mode, value, lower, radius, families, n_mask,
               deadline_ms: float = 0.0) -> int:
        job = make_job(volume, mask, spacing, mode, value, lower, radius, families, n_mask)
        # the server's streams do not wait for the stream that produced the
        # inputs: finish that work before the job can be admitted
        for t_ in (volume, mask):
            if t_.is_cuda:
                torch.cuda.current_stream(t_.device).synchronize()
        t = fr_server_submit(self.h, job, deadline_ms)
        self.inputs[t] = (volume, mask)
        return t

    def submit_case(self, case, vol, mask, radius=None, value=None, deadline_ms: float = 0.0) -> int:
        return self.submit(vol, mask, case.spacing, case.mode,
                           case.value if value is None else value, case.lower,
                           case.radius if radius is None else radius, case.families, case.n_mask,
                           deadline_ms)

    def cancel(self, ticket: int):
        fr_server_cancel(self.h, ticket)

    def inject_alloc_failures(self, n: int):
        fr_server_inject_alloc_failures(self.h, n)

    def poll(self, max_tickets: int = 256):
        return fr_server_poll(self.h, max_tickets)

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        fr_server_wait(self.h, ticket, timeout_ms)

    def result(self, ticket: int) -> FrResult:
        return fr_server_result(self.h, ticket)

    def maps(self, ticket: int, stream=None) -> torch.Tensor:
        r = self.result(ticket)
        vol = self.inputs.get(ticket, (None,))[0]
        dev = vol.device if vol is not None and vol.is_cuda else torch.device("cuda", torch.cuda.current_device())
        out = torch.empty((r.count, r.n_mask), dtype=torch.float32, device=dev)
        fr_server_copy(self.h, ticket, out, stream)
        return out

    def release(self, ticket: int):
        fr_server_release(self.h, ticket)
        self.inputs.pop(ticket, None)

    def stats(self) -> dict:
        return fr_server_stats(self.h)

    def close(self):
        if self.h is not None:
            fr_server_destroy(self.h)
            self.h = None
            self.inputs.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fr_profile_enable(enable: bool = True):
    _check(lib().fr_profile_enable(1 if enable else 0))


def fr_profile_read():
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().fr_profile_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def fr_version() -> str:
    return lib().fr_version().decode()


def fr_source_hash() -> str:
    return lib().fr_source_hash().decode()
