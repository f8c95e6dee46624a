"""CPU oracle for full search (FS) and DCDS motion estimation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_0806_0689_amd``) never imports it and shares no code with it.

The arithmetic lives in ``me_oracle.c`` (plain scalar C, single-threaded); this
module only builds it with gcc and marshals numpy arrays through ctypes.
``cnn.py`` holds the fp64 numpy oracle of the learned start proposer and
``quality.py`` that of the quality measures (MAD, MSE, PSNR, distance) and
``mvp.py`` that of the MVP statistics of §II-C.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "me_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CC_FLAGS = ["-O2", "-std=c99", "-shared", "-fPIC"]

VARIANT_DCDS = 0
VARIANT_DCDS_S = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc; returns the shared-object path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CC_FLAGS, "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load_library(path: str):
    """Load an oracle shared object (the default one or a test's mutant build)."""
    L = ctypes.CDLL(path)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i16p = ctypes.POINTER(ctypes.c_int16)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ci = ctypes.c_int
    L.oracle_fs.argtypes = [u8p, u8p, ci, ci, ci, ci, ci, i16p, u32p, u32p]
    L.oracle_fs.restype = ci
    L.oracle_dcds.argtypes = [u8p, u8p, ci, ci, ci, ci, ci, i16p, u8p, ci, i16p, u32p, u32p]
    L.oracle_dcds.restype = ci
    L.oracle_dcds_surface.argtypes = [ci, i64p, u8p, ci, ci, ci, ci, ci, i16p, i64p, u32p, u8p, u32p, ci,
                                      ctypes.POINTER(ci)]
    L.oracle_dcds_surface.restype = ci
    L.oracle_block_sad.argtypes = [u8p, u8p, ci, ci, ci, ci, ci, ci, ci, ci]
    L.oracle_block_sad.restype = ctypes.c_int64
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = load_library(_LIB)
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _frames(cur, ref):
    cur = np.ascontiguousarray(cur, dtype=np.uint8)
    ref = np.ascontiguousarray(ref, dtype=np.uint8)
    if cur.shape != ref.shape or cur.ndim != 2:
        raise ValueError("cur and ref must be 2-D uint8 arrays of one shape")
    return cur, ref


def fullsearch(cur, ref, block=16, range_=7):
    """FS per block: returns (mv int16[Hb,Wb,2], sad uint32[Hb,Wb], nsp uint32[Hb,Wb])."""
    cur, ref = _frames(cur, ref)
    H, W = cur.shape
    hb, wb = H // block, W // block
    mv = np.zeros((hb, wb, 2), np.int16)
    sad = np.zeros((hb, wb), np.uint32)
    nsp = np.zeros((hb, wb), np.uint32)
    rc = lib().oracle_fs(_ptr(cur, ctypes.c_uint8), _ptr(ref, ctypes.c_uint8), W, H, W, block, range_,
                         _ptr(mv, ctypes.c_int16), _ptr(sad, ctypes.c_uint32), _ptr(nsp, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("oracle_fs failed with %d" % rc)
    return mv, sad, nsp


def dcds(cur, ref, block=16, range_=7, start=None, orient=None, variant=VARIANT_DCDS):
    """DCDS per block (optionally from per-block starts); same outputs as fullsearch."""
    cur, ref = _frames(cur, ref)
    H, W = cur.shape
    hb, wb = H // block, W // block
    mv = np.zeros((hb, wb, 2), np.int16)
    sad = np.zeros((hb, wb), np.uint32)
    nsp = np.zeros((hb, wb), np.uint32)
    if start is not None:
        start = np.ascontiguousarray(start, dtype=np.int16).reshape(hb, wb, 2)
        if orient is not None:
            orient = np.ascontiguousarray(orient, dtype=np.uint8).reshape(hb, wb)
    rc = lib().oracle_dcds(_ptr(cur, ctypes.c_uint8), _ptr(ref, ctypes.c_uint8), W, H, W, block, range_,
                           _ptr(start, ctypes.c_int16), _ptr(orient, ctypes.c_uint8), variant,
                           _ptr(mv, ctypes.c_int16), _ptr(sad, ctypes.c_uint32), _ptr(nsp, ctypes.c_uint32))
    if rc != 0:
        raise ValueError("oracle_dcds failed with %d" % rc)
    return mv, sad, nsp


def dcds_surface(cost, valid=None, start=None, orient_v=False, variant=VARIANT_DCDS, want_set=False,
                 want_trace=False):
    """DCDS over one cost surface cost[dy+R, dx+R] (ideal-condition analysis).

    Returns (mv (dx, dy), distortion, nsp[, S as a bool array][, trace]) where
    trace lists |S| after Step 1, after each Step-2/3 diamond and after Step 4.
    """
    cost = np.ascontiguousarray(cost, dtype=np.int64)
    n = cost.shape[0]
    if cost.shape != (n, n) or n % 2 != 1:
        raise ValueError("cost must be square with odd side 2R+1")
    R = n // 2
    if valid is not None:
        valid = np.ascontiguousarray(valid, dtype=np.uint8)
    mv = np.zeros(2, np.int16)
    d = np.zeros(1, np.int64)
    nsp = np.zeros(1, np.uint32)
    s_out = np.zeros((n, n), np.uint8) if want_set else None
    sx, sy = (0, 0) if start is None else (int(start[0]), int(start[1]))
    cap = 4 * n * n + 8
    trace = np.zeros(cap, np.uint32)
    tn = ctypes.c_int(0)
    rc = lib().oracle_dcds_surface(R, _ptr(cost, ctypes.c_int64), _ptr(valid, ctypes.c_uint8), sx, sy,
                                   int(start is not None), int(bool(orient_v)), variant,
                                   _ptr(mv, ctypes.c_int16), _ptr(d, ctypes.c_int64),
                                   _ptr(nsp, ctypes.c_uint32), _ptr(s_out, ctypes.c_uint8),
                                   _ptr(trace, ctypes.c_uint32), cap, ctypes.byref(tn))
    if rc != 0:
        raise ValueError("oracle_dcds_surface failed with %d" % rc)
    out = ((int(mv[0]), int(mv[1])), int(d[0]), int(nsp[0]))
    if want_set:
        out = out + (s_out.astype(bool),)
    if want_trace:
        out = out + ([int(v) for v in trace[:min(tn.value, cap)]],)
    return out


def block_sad(cur, ref, block, x0, y0, dx, dy):
    cur, ref = _frames(cur, ref)
    H, W = cur.shape
    return int(lib().oracle_block_sad(_ptr(cur, ctypes.c_uint8), _ptr(ref, ctypes.c_uint8), W, H, W, block,
                                      x0, y0, dx, dy))
