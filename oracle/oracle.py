"""ctypes front end of the FP64 CPU oracle (fr_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package's smoke
check and by the benchmark's CPU-baseline leg, never by the product path.
It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

I16, F32 = 1, 2
FBW, FBN = 1, 2
FAMILY_SIZES = [("firstorder", 18), ("glcm", 24), ("glrlm", 16), ("glszm", 16),
                ("gldm", 14), ("ngtdm", 5)]


def build() -> str:
    """Compile fr_oracle.c with gcc (FP64, no FP contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
           "-o", LIB + ".tmp", SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        P, I, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint32
        I64 = ctypes.c_int64
        L.or_discretise.argtypes = [P, I, I, I, I, P, I, D, D, P, P, P, P]
        L.or_map.argtypes = [P, I, I, I, I, P, P, I, D, D, I, U, P, I64, P, I]
        L.or_map_ex.argtypes = [P, I, I, I, I, P, P, I, D, D, I, U, P, I64, P, I, P]
        L.or_matrices_ex.argtypes = [P, P, I, I, I, I, I, I, I, I, I, I, I,
                                     P, P, P, P, P, P, P, P, P, P, P]
        L.or_scalar.argtypes = [P, I, I, I, I, P, P, I, D, D, U, P]
        L.or_matrices.argtypes = [P, P, I, I, I, I, I, I, I, I, I, I, I,
                                  P, P, P, P, P, P, P, P, P, P]
        L.or_glcm_features.argtypes = [P, I, D, P, P]
        L.or_runzone_features.argtypes = [P, I, I, D, P]
        L.or_gldm_features.argtypes = [P, I, I, P]
        L.or_ngtdm_features.argtypes = [P, P, I, P]
        L.or_firstorder_features.argtypes = [P, I, P, I, D, P]
        L.or_map_count.argtypes = [U]
        L.or_map_name.argtypes = [U, I, ctypes.c_char_p, I]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dtype_code(vol: np.ndarray) -> int:
    if vol.dtype == np.int16:
        return I16
    if vol.dtype == np.float32:
        return F32
    raise TypeError(f"volume dtype {vol.dtype} not supported (int16 or float32)")


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def discretise(vol, mask, mode, value, lower=float("nan")):
    vol = np.ascontiguousarray(vol)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = vol.shape
    levels = np.zeros(vol.shape, np.uint8)
    ng = ctypes.c_int()
    xmin, xmax = ctypes.c_double(), ctypes.c_double()
    rc = lib().or_discretise(_ptr(vol), _dtype_code(vol), nx, ny, nz, _ptr(mask), mode,
                             float(value), float(lower), _ptr(levels), ctypes.byref(ng),
                             ctypes.byref(xmin), ctypes.byref(xmax))
    _check(rc, "or_discretise")
    return levels, ng.value, xmin.value, xmax.value


def map_count(families: int) -> int:
    return lib().or_map_count(families)


def map_names(families: int):
    buf = ctypes.create_string_buffer(96)
    out = []
    for k in range(map_count(families)):
        _check(lib().or_map_name(families, k, buf, 96), "or_map_name")
        out.append(buf.value.decode())
    return out


def _options(glcm_distance, gldm_alpha, averaged):
    if (glcm_distance, gldm_alpha, averaged) == (1, 0, False):
        return None
    return np.array([glcm_distance, gldm_alpha, 1 if averaged else 0], np.int32)


def spatial_map(case=None, *, vol=None, mask=None, spacing=None, mode=None, value=None,
                lower=float("nan"), radius=None, families=None, sample=None, nthreads=0,
                glcm_distance=1, gldm_alpha=0, averaged=False):
    """FP64 maps [count][n] for the mask voxels in `sample` (compact indices,
    raster order) or for every mask voxel; glcm_distance, gldm_alpha and
    averaged select the extraction variants (defaults: 1, 0, merged)."""
    if case is not None:
        vol, mask, spacing = case.volume, case.mask, case.spacing
        mode, value, lower, radius, families = case.mode, case.value, case.lower, case.radius, case.families
    vol = np.ascontiguousarray(vol)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = vol.shape
    sp = np.asarray(spacing, np.float64)
    if sample is None:
        ns = int(np.count_nonzero(mask))
        sptr = None
    else:
        sample = np.ascontiguousarray(sample, dtype=np.int64)
        ns = sample.size
        sptr = _ptr(sample)
    out = np.empty((map_count(families), ns), np.float64)
    opt = _options(glcm_distance, gldm_alpha, averaged)
    rc = lib().or_map_ex(_ptr(vol), _dtype_code(vol), nx, ny, nz, _ptr(mask), _ptr(sp), mode,
                         float(value), float(lower), radius, families, sptr, ns, _ptr(out),
                         nthreads, None if opt is None else _ptr(opt))
    _check(rc, "or_map")
    return out


def scalar(case=None, *, vol=None, mask=None, spacing=None, mode=None, value=None,
           lower=float("nan"), families=None):
    if case is not None:
        vol, mask, spacing = case.volume, case.mask, case.spacing
        mode, value, lower, families = case.mode, case.value, case.lower, case.families
    vol = np.ascontiguousarray(vol)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = vol.shape
    sp = np.asarray(spacing, np.float64)
    out = np.empty(map_count(families), np.float64)
    rc = lib().or_scalar(_ptr(vol), _dtype_code(vol), nx, ny, nz, _ptr(mask), _ptr(sp), mode,
                         float(value), float(lower), families, _ptr(out))
    _check(rc, "or_scalar")
    return out


def matrices(levels, vol, ng, centre_zyx=None, radius=1, glcm_distance=1, gldm_alpha=0):
    """Integer matrices of one neighbourhood (radius < 0: the whole VOI).
    Returned dense over actual levels 1..ng (row a = level a+1); the GLCM at
    glcm_distance, the GLDM with gldm_alpha."""
    levels = np.ascontiguousarray(levels, dtype=np.uint8)
    vol = np.ascontiguousarray(vol)
    nz, ny, nx = vol.shape
    if radius >= 0:
        S = 2 * radius + 1
        lmax, zmax = S, S ** 3
        cz, cy, cx = centre_zyx
    else:
        lmax = max(nx, ny, nz)
        zmax = int(np.count_nonzero(levels))
        cz = cy = cx = 0
    out = dict(
        glcm=np.zeros((ng, ng), np.int64), glrlm=np.zeros((ng, lmax), np.int64),
        glszm=np.zeros((ng, zmax), np.int64), gldm=np.zeros((ng, 27), np.int64),
        ngtdm_n=np.zeros(ng, np.int64), ngtdm_S=np.zeros(ng, np.int64),
        ngtdm_s=np.zeros(ng, np.float64), hist=np.zeros(ng, np.int64),
        vals=np.zeros(zmax, np.float64))
    K = ctypes.c_int()
    opt = _options(glcm_distance, gldm_alpha, False)
    rc = lib().or_matrices_ex(_ptr(levels), _ptr(vol), _dtype_code(vol), nx, ny, nz, radius,
                              cx, cy, cz, ng, lmax, zmax,
                              _ptr(out["glcm"]), _ptr(out["glrlm"]), _ptr(out["glszm"]),
                              _ptr(out["gldm"]), _ptr(out["ngtdm_n"]), _ptr(out["ngtdm_S"]),
                              _ptr(out["ngtdm_s"]), _ptr(out["hist"]), _ptr(out["vals"]),
                              ctypes.byref(K), None if opt is None else _ptr(opt))
    _check(rc, "or_matrices")
    out["K"] = K.value
    out["vals"] = out["vals"][:K.value]
    return out


def glcm_features(P, ng_norm=None):
    P = np.ascontiguousarray(P, dtype=np.int64)
    ng = P.shape[0]
    f = np.empty(24)
    extra = np.empty(4)
    _check(lib().or_glcm_features(_ptr(P), ng, float(ng if ng_norm is None else ng_norm),
                                  _ptr(f), _ptr(extra)), "or_glcm_features")
    return f, dict(HX=extra[0], HY=extra[1], HXY1=extra[2], HXY2=extra[3])


def runzone_features(M, units):
    M = np.ascontiguousarray(M, dtype=np.int64)
    f = np.empty(16)
    _check(lib().or_runzone_features(_ptr(M), M.shape[0], M.shape[1], float(units), _ptr(f)),
           "or_runzone_features")
    return f


def gldm_features(D):
    D = np.ascontiguousarray(D, dtype=np.int64)
    f = np.empty(14)
    _check(lib().or_gldm_features(_ptr(D), D.shape[0], D.shape[1], _ptr(f)), "or_gldm_features")
    return f


def ngtdm_features(n, s):
    n = np.ascontiguousarray(n, dtype=np.int64)
    s = np.ascontiguousarray(s, dtype=np.float64)
    f = np.empty(5)
    _check(lib().or_ngtdm_features(_ptr(n), _ptr(s), n.size, _ptr(f)), "or_ngtdm_features")
    return f


def firstorder_features(vals, hist, voxel_volume=1.0):
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    hist = np.ascontiguousarray(hist, dtype=np.int64)
    f = np.empty(18)
    _check(lib().or_firstorder_features(_ptr(vals), vals.size, _ptr(hist), hist.size,
                                        float(voxel_volume), _ptr(f)), "or_firstorder_features")
    return f
