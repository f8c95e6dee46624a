"""Block-matching motion estimation (FS and DCDS) on AMD MI355X.

Python binding of ``libme.so`` (``include/me.h``).  This module only marshals
arguments: every step of a search runs in the library's HIP kernels.  PyTorch
provides device memory and streams.  There is no CPU fallback: if the library
is not built, every call raises.

Low-level functions carry the C names (``me_search``, ``me_fullsearch``,
``me_dcds``, ``me_dcds_ex``, ``me_dcds_surface``, ``me_frame_quality``, ...)
and take raw pointers and sizes.  The helpers ``search``, ``fullsearch``,
``dcds``, ``frame_quality`` and ``dcds_surface`` take torch tensors.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libme.so")

ME_OK = 0
ME_EINVAL = -1
ME_EUNSUPPORTED = -2
ME_ENOMEM = -3
ME_EDEVICE = -4

ME_ALGO_FS = 0
ME_ALGO_DCDS = 1
ME_ALGO_DCDS_S = 2

# Every symbol include/me.h declares (checked by the ABI tests).
EXPORTS = [
    "me_status_string",
    "me_set_config",
    "me_get_config",
    "me_search",
    "me_fullsearch",
    "me_dcds",
    "me_dcds_ex",
    "me_dcds_surface",
    "me_frame_quality",
    "me_mvp_stats",
    "me_mvp_tables_size",
    "me_mvp_tables",
    "me_batch",
    "me_batch_noalloc",
    "me_autotune",
    "me_autotune_save",
    "me_autotune_load",
    "me_shutdown",
    "me_proposer_num_params",
    "me_proposer_create",
    "me_proposer_destroy",
    "me_proposer_init",
    "me_proposer_set_weights",
    "me_proposer_get_weights",
    "me_proposer_get_grads",
    "me_proposer_get_state",
    "me_proposer_set_state",
    "me_proposer_forward",
    "me_proposer_backward",
    "me_proposer_train_step",
    "me_proposer_infer",
    "me_dcds_learned",
]

MAX_JOBS = 4096


class MeConfig(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
                ("tiles_per_grab", ctypes.c_int32)]


class MeJob(ctypes.Structure):
    _fields_ = [
        ("cur", ctypes.c_void_p), ("ref", ctypes.c_void_p),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("pitch", ctypes.c_int32), ("n_pairs", ctypes.c_int32),
        ("pair_stride", ctypes.c_int64),
        ("mv", ctypes.c_void_p), ("sad", ctypes.c_void_p), ("nsp", ctypes.c_void_p),
        ("start", ctypes.c_void_p), ("orient", ctypes.c_void_p),
        ("sse", ctypes.c_void_p),
    ]


# me_quality, one record per frame pair (include/me.h).
QUALITY_FIELDS = [("sad", "<u8"), ("sse", "<u8"), ("blocks", "<u4"), ("equal", "<u4"), ("dist", "<f8"),
                  ("mad", "<f8"), ("mse", "<f8"), ("psnr", "<f8")]
QUALITY_BYTES = 56


class MEError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, status_string(status), status))


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libme.so is not built (run __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.me_status_string.argtypes = [ctypes.c_int]
        L.me_status_string.restype = ctypes.c_char_p
        frame = [vp, vp, i32, i32, i32, i64, i32, i32, i32]
        L.me_fullsearch.argtypes = frame + [vp, vp, vp, vp]
        L.me_fullsearch.restype = ctypes.c_int
        L.me_dcds.argtypes = frame + [vp, vp, vp, vp]
        L.me_dcds.restype = ctypes.c_int
        L.me_dcds_ex.argtypes = frame + [i32, vp, vp, vp, vp, vp, vp]
        L.me_dcds_ex.restype = ctypes.c_int
        L.me_search.argtypes = frame + [i32, vp, vp, vp, vp, vp, vp, vp]
        L.me_search.restype = ctypes.c_int
        L.me_frame_quality.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, vp, vp]
        L.me_frame_quality.restype = ctypes.c_int
        L.me_mvp_stats.argtypes = frame + [vp, vp, vp, vp]
        L.me_mvp_stats.restype = ctypes.c_int
        L.me_mvp_tables_size.argtypes = [i32]
        L.me_mvp_tables_size.restype = i32
        L.me_mvp_tables.argtypes = [vp, vp, vp, i32, vp, vp]
        L.me_mvp_tables.restype = ctypes.c_int
        L.me_dcds_surface.argtypes = [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]
        L.me_dcds_surface.restype = ctypes.c_int
        L.me_set_config.argtypes = [i32, i32, ctypes.POINTER(MeConfig)]
        L.me_set_config.restype = ctypes.c_int
        L.me_get_config.argtypes = [i32, i32, ctypes.POINTER(MeConfig)]
        L.me_get_config.restype = ctypes.c_int
        L.me_batch.argtypes = [ctypes.POINTER(MeJob), i32, i32, i32, i32, vp]
        L.me_batch.restype = ctypes.c_int
        L.me_batch_noalloc.argtypes = [ctypes.POINTER(MeJob), i32, i32, i32, i32, vp]
        L.me_batch_noalloc.restype = ctypes.c_int
        L.me_autotune.argtypes = [ctypes.POINTER(MeJob), i32, i32, i32, i32, i32, ctypes.POINTER(MeConfig),
                                  ctypes.POINTER(ctypes.c_float), vp]
        L.me_autotune.restype = ctypes.c_int
        L.me_autotune_save.argtypes = [ctypes.c_char_p]
        L.me_autotune_save.restype = ctypes.c_int
        L.me_autotune_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.me_autotune_load.restype = ctypes.c_int
        L.me_shutdown.argtypes = []
        L.me_shutdown.restype = ctypes.c_int
        fp = ctypes.POINTER(ctypes.c_float)
        L.me_proposer_num_params.argtypes = []
        L.me_proposer_num_params.restype = i32
        L.me_proposer_create.argtypes = [ctypes.POINTER(vp)]
        L.me_proposer_create.restype = ctypes.c_int
        L.me_proposer_destroy.argtypes = [vp]
        L.me_proposer_destroy.restype = ctypes.c_int
        L.me_proposer_init.argtypes = [vp, ctypes.c_uint64]
        L.me_proposer_init.restype = ctypes.c_int
        for name in ("me_proposer_set_weights", "me_proposer_get_weights", "me_proposer_get_grads"):
            getattr(L, name).argtypes = [vp, fp, i32]
            getattr(L, name).restype = ctypes.c_int
        L.me_proposer_get_state.argtypes = [vp, fp, fp, ctypes.POINTER(i64), i32]
        L.me_proposer_get_state.restype = ctypes.c_int
        L.me_proposer_set_state.argtypes = [vp, fp, fp, i64, i32]
        L.me_proposer_set_state.restype = ctypes.c_int
        L.me_proposer_forward.argtypes = [vp] + frame[:7] + [vp, vp]
        L.me_proposer_forward.restype = ctypes.c_int
        L.me_proposer_backward.argtypes = [vp, vp, vp]
        L.me_proposer_backward.restype = ctypes.c_int
        L.me_proposer_train_step.argtypes = [vp] + frame[:7] + [vp, ctypes.c_float, vp, vp]
        L.me_proposer_train_step.restype = ctypes.c_int
        L.me_proposer_infer.argtypes = [vp] + frame[:7] + [i32, vp, vp, vp]
        L.me_proposer_infer.restype = ctypes.c_int
        L.me_dcds_learned.argtypes = [vp] + frame[:7] + [i32, i32, vp, vp, vp, vp]
        L.me_dcds_learned.restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().me_status_string(int(status)).decode()


# ----------------------------------------------------------------------------
# Raw C entry points (pointers as ints, sizes as ints, stream handle as int).
# ----------------------------------------------------------------------------
def me_fullsearch(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, mv, sad, nsp, stream=0):
    return lib().me_fullsearch(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, mv, sad, nsp,
                               stream)


def me_dcds(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, mv, sad, nsp, stream=0):
    return lib().me_dcds(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, mv, sad, nsp, stream)


def me_dcds_ex(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, algo, start, orient, mv, sad,
               nsp, stream=0):
    return lib().me_dcds_ex(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, algo, start,
                            orient, mv, sad, nsp, stream)


def me_search(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, algo, start, orient, mv, sad, nsp,
              sse, stream=0):
    return lib().me_search(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, algo, start, orient,
                           mv, sad, nsp, sse, stream)


def me_frame_quality(mv, sad, sse, mv_true, width, height, n_pairs, block, out, stream=0):
    return lib().me_frame_quality(mv, sad, sse, mv_true, width, height, n_pairs, block, out, stream)


def me_mvp_stats(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, hist, d1, d2, stream=0):
    return lib().me_mvp_stats(cur, ref, width, height, pitch, pair_stride, n_pairs, block, range_, hist, d1, d2,
                              stream)


def me_mvp_tables_size(range_):
    return lib().me_mvp_tables_size(range_)


def me_mvp_tables(hist, d1, d2, range_, out, stream=0):
    return lib().me_mvp_tables(hist, d1, d2, range_, out, stream)


def me_dcds_surface(cost, valid, n, range_, algo, start, orient, mv, cost_out, nsp, stream=0):
    return lib().me_dcds_surface(cost, valid, n, range_, algo, start, orient, mv, cost_out, nsp, stream)


def me_set_config(block, range_, cfg):
    """cfg: (rows_per_lane, waves_per_group[, tiles_per_grab]) or None for the
    default; a missing or 0 tiles_per_grab means the default grab."""
    p = None if cfg is None else ctypes.byref(MeConfig(int(cfg[0]), int(cfg[1]),
                                                       int(cfg[2]) if len(cfg) > 2 else 0))
    return lib().me_set_config(block, range_, p)


def me_get_config(block, range_):
    """(rows_per_lane, waves_per_group, tiles_per_grab) in force."""
    c = MeConfig()
    rc = lib().me_get_config(block, range_, ctypes.byref(c))
    _check(rc, "me_get_config")
    return c.rows_per_lane, c.waves_per_group, c.tiles_per_grab


def me_batch(jobs, n_jobs, algo, block, range_, stream=0):
    """jobs: a ctypes array of MeJob (or None)."""
    return lib().me_batch(jobs, n_jobs, algo, block, range_, stream)


def me_batch_noalloc(jobs, n_jobs, algo, block, range_, stream=0):
    """jobs: a ctypes array of MeJob (or None).  Allocates nothing in the library."""
    return lib().me_batch_noalloc(jobs, n_jobs, algo, block, range_, stream)


def me_autotune(jobs, n_jobs, algo, block, range_, reps, stream=0):
    """Returns (status, (rows_per_lane, waves_per_group, tiles_per_grab), ms)."""
    best = MeConfig()
    ms = ctypes.c_float(0.0)
    rc = lib().me_autotune(jobs, n_jobs, algo, block, range_, reps, ctypes.byref(best), ctypes.byref(ms), stream)
    return rc, (best.rows_per_lane, best.waves_per_group, best.tiles_per_grab), ms.value


def me_autotune_save(path):
    return lib().me_autotune_save(os.fsencode(path))


def me_autotune_load(path):
    """Returns (status, applied, rejected)."""
    a, r = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = lib().me_autotune_load(os.fsencode(path), ctypes.byref(a), ctypes.byref(r))
    return rc, a.value, r.value


def me_shutdown():
    return lib().me_shutdown()


def set_config(block, range_, cfg):
    _check(me_set_config(block, range_, cfg), "me_set_config")


# ----------------------------------------------------------------------------
# Tensor helpers.
# ----------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _frames(cur, ref):
    """Accepts [H, W] or [P, H, W] uint8 CUDA tensors with unit column stride."""
    torch = _torch()
    if cur.dtype != torch.uint8 or ref.dtype != torch.uint8:
        raise TypeError("frames must be uint8")
    if not cur.is_cuda or not ref.is_cuda:
        raise TypeError("frames must be on the GPU")
    if cur.shape != ref.shape or cur.dim() not in (2, 3):
        raise ValueError("cur and ref must both be [H, W] or [P, H, W]")
    if cur.stride() != ref.stride() or cur.stride(-1) != 1:
        raise ValueError("cur and ref must share strides, with unit column stride")
    if cur.dim() == 2:
        P, (H, W) = 1, cur.shape
        stride = H * cur.stride(0)
    else:
        P, H, W = cur.shape
        stride = cur.stride(0)
    return P, H, W, cur.stride(-2), stride


def _arg(t, n, dtype, device, name):
    """A caller tensor that a kernel reads or writes by block index: it must
    live on the frames' device with the given dtype, be contiguous and hold
    exactly n elements, or the kernel would run past it."""
    if t is None:
        return None
    if t.device != device or t.dtype != dtype or not t.is_contiguous() or t.numel() != n:
        raise ValueError("%s must be a contiguous %s tensor of %d elements on %s (got %s, %d elements, %s%s)" % (
            name, dtype, n, device, t.dtype, t.numel(), t.device, "" if t.is_contiguous() else ", not contiguous"))
    return t


def _block_args(P, hb, wb, device, start=None, orient=None):
    torch = _torch()
    n = P * hb * wb
    return (_arg(start, 2 * n, torch.int16, device, "start"), _arg(orient, n, torch.uint8, device, "orient"))


def _outputs(P, hb, wb, device, out):
    torch = _torch()
    if out is not None:
        mv, sad, nsp = out
        n = P * hb * wb
        return (_arg(mv, 2 * n, torch.int16, device, "mv"), _arg(sad, n, torch.int32, device, "sad"),
                _arg(nsp, n, torch.int32, device, "nsp"))
    mv = torch.empty((P, hb, wb, 2), dtype=torch.int16, device=device)
    sad = torch.empty((P, hb, wb), dtype=torch.int32, device=device)
    nsp = torch.empty((P, hb, wb), dtype=torch.int32, device=device)
    return mv, sad, nsp


def _check(rc, where):
    if rc != ME_OK:
        raise MEError(rc, where)


def sequence_pairs(seq):
    """Views (cur, ref) = (frames 1.., frames ..-1) of a [T, H, W] sequence."""
    return seq[1:], seq[:-1]


def fullsearch(cur, ref, block=16, range_=7, out=None, stream=None):
    """FS on one pair ([H, W]) or P pairs ([P, H, W]); returns (mv, sad, nsp) as
    [P, H/B, W/B, 2] int16 and [P, H/B, W/B] int32 tensors."""
    P, H, W, pitch, stride = _frames(cur, ref)
    mv, sad, nsp = _outputs(P, H // block, W // block, cur.device, out)
    rc = me_fullsearch(cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P, block, range_, mv.data_ptr(),
                       sad.data_ptr(), nsp.data_ptr(), _stream(stream))
    _check(rc, "me_fullsearch")
    return mv, sad, nsp


def dcds(cur, ref, block=16, range_=7, algo=ME_ALGO_DCDS, start=None, orient=None, out=None, stream=None):
    """DCDS (or DCDS^S with algo=ME_ALGO_DCDS_S), optionally from per-block start
    vectors (int16 [P, H/B, W/B, 2]) and first-cross orientations (uint8)."""
    P, H, W, pitch, stride = _frames(cur, ref)
    mv, sad, nsp = _outputs(P, H // block, W // block, cur.device, out)
    start, orient = _block_args(P, H // block, W // block, cur.device, start, orient)
    sp = start.data_ptr() if start is not None else None
    op = orient.data_ptr() if orient is not None else None
    rc = me_dcds_ex(cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P, block, range_, algo, sp, op,
                    mv.data_ptr(), sad.data_ptr(), nsp.data_ptr(), _stream(stream))
    _check(rc, "me_dcds_ex")
    return mv, sad, nsp


def search(cur, ref, block=16, range_=7, algo=ME_ALGO_DCDS, start=None, orient=None, sse=False, out=None,
           stream=None):
    """Any search (algo ME_ALGO_FS, ME_ALGO_DCDS or ME_ALGO_DCDS_S); returns
    (mv, sad, nsp) and, with sse=True, the per-block squared error of the
    motion-compensated block as a fourth int32 [P, H/B, W/B] tensor."""
    torch = _torch()
    P, H, W, pitch, stride = _frames(cur, ref)
    mv, sad, nsp = _outputs(P, H // block, W // block, cur.device, out[:3] if out is not None else None)
    start, orient = _block_args(P, H // block, W // block, cur.device, start, orient)
    e = None
    if sse:
        e = out[3] if out is not None and len(out) > 3 else torch.empty_like(sad)
        e = _arg(e, sad.numel(), torch.int32, cur.device, "sse")
    sp = start.data_ptr() if start is not None else None
    op = orient.data_ptr() if orient is not None else None
    rc = me_search(cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P, block, range_, algo, sp, op,
                   mv.data_ptr(), sad.data_ptr(), nsp.data_ptr(), e.data_ptr() if e is not None else None,
                   _stream(stream))
    _check(rc, "me_search")
    return (mv, sad, nsp, e) if sse else (mv, sad, nsp)


def frame_quality(mv, sad, sse, mv_true=None, block=16, stream=None):
    """Per-pair quality records (MAD, MSE, PSNR of the compensated frame;
    distance from and agreement with mv_true) of one search's outputs
    ([P, H/B, W/B, ...] tensors).  Returns a host numpy structured array with
    the fields of me_quality (QUALITY_FIELDS)."""
    import numpy as np
    torch = _torch()
    if mv.dim() == 3:
        mv, sad, sse = mv[None], sad[None], sse[None]
        mv_true = mv_true[None] if mv_true is not None else None
    P, hb, wb = mv.shape[:3]
    n = P * hb * wb
    if not mv.is_cuda:
        raise ValueError("quality inputs must be GPU tensors")
    _arg(mv, 2 * n, torch.int16, mv.device, "mv")
    _arg(sad, n, torch.int32, mv.device, "sad")
    _arg(sse, n, torch.int32, mv.device, "sse")
    _arg(mv_true, 2 * n, torch.int16, mv.device, "mv_true")
    out = torch.empty(max(1, P) * QUALITY_BYTES, dtype=torch.uint8, device=mv.device)
    rc = me_frame_quality(mv.data_ptr(), sad.data_ptr(), sse.data_ptr(),
                          mv_true.data_ptr() if mv_true is not None else None, wb * block, hb * block, P, block,
                          out.data_ptr(), _stream(stream))
    _check(rc, "me_frame_quality")
    return out[:P * QUALITY_BYTES].cpu().numpy().view(np.dtype(QUALITY_FIELDS))


def _mvp_counts(counts, range_, device):
    torch = _torch()
    hist, d1, d2 = counts
    n = 2 * range_ + 1
    return (_arg(hist, n * n, torch.int32, device, "hist"), _arg(d1, 9 * n * n, torch.int32, device, "d1"),
            _arg(d2, 25 * n * n, torch.int32, device, "d2"))


def mvp_stats(cur, ref, block=16, range_=7, counts=None, stream=None):
    """Adds the blocks of these pairs to the MVP counters (hist [n*n], d1
    [9, n*n], d2 [n*n, 25] int32 tensors, n = 2 range + 1; zeroed here unless
    given) and returns them."""
    torch = _torch()
    P, H, W, pitch, stride = _frames(cur, ref)
    n = 2 * range_ + 1
    if counts is None:
        counts = (torch.zeros(n * n, dtype=torch.int32, device=cur.device),
                  torch.zeros((9, n * n), dtype=torch.int32, device=cur.device),
                  torch.zeros((n * n, 25), dtype=torch.int32, device=cur.device))
    hist, d1, d2 = _mvp_counts(counts, range_, cur.device)
    rc = me_mvp_stats(cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P, block, range_, hist.data_ptr(),
                      d1.data_ptr(), d2.data_ptr(), _stream(stream))
    _check(rc, "me_mvp_stats")
    return counts


def mvp_tables(counts, range_, stream=None):
    """The tables of §II-C from mvp_stats counters, as host numpy arrays:
    quarter [R+1, R+1], ax, ay, bx, by [2R+1], regions [5], eta [5],
    d1 [9, 2R+1, 2R+1], d2 [2R+1, 2R+1, 5, 5], t1, t2 [5, 5]."""
    torch = _torch()
    size = me_mvp_tables_size(range_)
    if size < 0:
        raise MEError(size, "me_mvp_tables_size")
    hist, d1, d2 = _mvp_counts(counts, range_, counts[0].device)
    out = torch.empty(size, dtype=torch.float64, device=hist.device)
    _check(me_mvp_tables(hist.data_ptr(), d1.data_ptr(), d2.data_ptr(), range_, out.data_ptr(), _stream(stream)),
           "me_mvp_tables")
    v = out.cpu().numpy()
    R, n = range_, 2 * range_ + 1
    parts, at = {}, 0
    for name, shape in (("quarter", (R + 1, R + 1)), ("ax", (n,)), ("ay", (n,)), ("bx", (n,)), ("by", (n,)),
                        ("regions", (5,)), ("eta", (5,)), ("d1", (9, n, n)), ("d2", (n, n, 5, 5)),
                        ("t1", (5, 5)), ("t2", (5, 5))):
        k = 1
        for s_ in shape:
            k *= s_
        parts[name] = v[at:at + k].reshape(shape)
        at += k
    assert at == size
    return parts


def make_jobs(pairs, block, starts=None, orients=None, outs=None, sses=None):
    """Job table for me_batch from a list of (cur, ref) tensor pairs ([H, W] or
    [P, H, W]); allocates outputs unless given.  sses: optional per-job int32
    tensors for the compensated-block squared error.  Returns (ctypes array,
    outputs)."""
    jobs = (MeJob * max(1, len(pairs)))()
    outputs = []
    for i, (cur, ref) in enumerate(pairs):
        P, H, W, pitch, stride = _frames(cur, ref)
        o = _outputs(P, H // block, W // block, cur.device, outs[i] if outs is not None else None)
        mv, sad, nsp = o
        st, orr = _block_args(P, H // block, W // block, cur.device, starts[i] if starts is not None else None,
                              orients[i] if orients is not None else None)
        e = _arg(sses[i], sad.numel(), sad.dtype, cur.device, "sse") if sses is not None else None
        jobs[i] = MeJob(cur.data_ptr(), ref.data_ptr(), W, H, pitch, P, stride, mv.data_ptr(), sad.data_ptr(),
                        nsp.data_ptr(), st.data_ptr() if st is not None else None,
                        orr.data_ptr() if orr is not None else None, e.data_ptr() if e is not None else None)
        outputs.append(o)
    return jobs, outputs


def batch(pairs, block=16, range_=15, algo=ME_ALGO_DCDS, starts=None, orients=None, outs=None, sses=None,
          stream=None):
    """One persistent launch over many sequences; returns one (mv, sad, nsp) per job."""
    jobs, outputs = make_jobs(pairs, block, starts, orients, outs, sses)
    _check(me_batch(jobs, len(pairs), algo, block, range_, _stream(stream)), "me_batch")
    return outputs


def batch_noalloc(pairs, block=16, range_=15, algo=ME_ALGO_DCDS, starts=None, orients=None, outs=None, sses=None,
                  stream=None):
    """me_batch_noalloc over (cur, ref) pairs; outputs as batch() (allocated
    here by torch unless given in outs)."""
    jobs, outputs = make_jobs(pairs, block, starts, orients, outs, sses)
    _check(me_batch_noalloc(jobs, len(pairs), algo, block, range_, _stream(stream)), "me_batch_noalloc")
    return outputs


def autotune(pairs, block=16, range_=15, algo=ME_ALGO_DCDS, reps=5, stream=None):
    """Times every DCDS configuration on this batch and keeps the fastest."""
    jobs, outputs = make_jobs(pairs, block)
    rc, cfg, ms = me_autotune(jobs, len(pairs), algo, block, range_, reps, _stream(stream))
    _check(rc, "me_autotune")
    return cfg, ms


class Proposer:
    """Learned start proposer (bf16 CNN) living on the current GPU."""

    def __init__(self, seed=None):
        h = ctypes.c_void_p()
        _check(lib().me_proposer_create(ctypes.byref(h)), "me_proposer_create")
        self.h = h
        self.n = lib().me_proposer_num_params()
        if seed is not None:
            _check(lib().me_proposer_init(self.h, seed), "me_proposer_init")

    def close(self):
        if self.h:
            lib().me_proposer_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fp(self, a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def set_weights(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib().me_proposer_set_weights(self.h, self._fp(w), len(w)), "me_proposer_set_weights")

    def get_weights(self):
        import numpy as np
        w = np.zeros(self.n, np.float32)
        _check(lib().me_proposer_get_weights(self.h, self._fp(w), self.n), "me_proposer_get_weights")
        return w

    def get_grads(self):
        import numpy as np
        g = np.zeros(self.n, np.float32)
        _check(lib().me_proposer_get_grads(self.h, self._fp(g), self.n), "me_proposer_get_grads")
        return g

    def get_state(self):
        import numpy as np
        m = np.zeros(self.n, np.float32)
        v = np.zeros(self.n, np.float32)
        step = ctypes.c_int64(0)
        _check(lib().me_proposer_get_state(self.h, self._fp(m), self._fp(v), ctypes.byref(step), self.n),
               "me_proposer_get_state")
        return m, v, step.value

    def set_state(self, m, v, step):
        import numpy as np
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        _check(lib().me_proposer_set_state(self.h, self._fp(m), self._fp(v), int(step), self.n),
               "me_proposer_set_state")

    def forward(self, cur, ref, stream=None):
        torch = _torch()
        P, H, W, pitch, stride = _frames(cur, ref)
        head = torch.empty((P, H // 16, W // 16, 3), dtype=torch.float32, device=cur.device)
        rc = lib().me_proposer_forward(self.h, cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P,
                                       head.data_ptr(), _stream(stream))
        _check(rc, "me_proposer_forward")
        self._last = (head.numel(), cur.device)
        return head

    def backward(self, dhead, stream=None):
        """Gradients for a head gradient shaped as the last forward's head."""
        torch = _torch()
        last = getattr(self, "_last", None)
        if last is None:
            raise MEError(ME_EINVAL, "me_proposer_backward (no forward yet)")
        dhead = _arg(dhead.contiguous(), last[0], torch.float32, last[1], "dhead")
        _check(lib().me_proposer_backward(self.h, dhead.data_ptr(), _stream(stream)), "me_proposer_backward")

    def train_step(self, cur, ref, target, lr, stream=None):
        """One Adam step; returns the (device) loss tensor before the step."""
        torch = _torch()
        P, H, W, pitch, stride = _frames(cur, ref)
        loss = torch.empty((1,), dtype=torch.float32, device=cur.device)
        target = _arg(target.contiguous(), P * (H // 16) * (W // 16) * 2, torch.int16, cur.device, "target")
        rc = lib().me_proposer_train_step(self.h, cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P,
                                          target.data_ptr(), float(lr), loss.data_ptr(), _stream(stream))
        _check(rc, "me_proposer_train_step")
        self._last = (P * (H // 16) * (W // 16) * 3, cur.device)
        return loss

    def infer(self, cur, ref, range_, stream=None):
        torch = _torch()
        P, H, W, pitch, stride = _frames(cur, ref)
        start = torch.empty((P, H // 16, W // 16, 2), dtype=torch.int16, device=cur.device)
        orient = torch.empty((P, H // 16, W // 16), dtype=torch.uint8, device=cur.device)
        rc = lib().me_proposer_infer(self.h, cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P, range_,
                                     start.data_ptr(), orient.data_ptr(), _stream(stream))
        _check(rc, "me_proposer_infer")
        return start, orient


def dcds_learned(proposer, cur, ref, range_=31, algo=ME_ALGO_DCDS, out=None, stream=None):
    """DCDS on 16x16 blocks from the proposer's starts (None: plain DCDS)."""
    P, H, W, pitch, stride = _frames(cur, ref)
    mv, sad, nsp = _outputs(P, H // 16, W // 16, cur.device, out)
    h = proposer.h if proposer is not None else None
    rc = lib().me_dcds_learned(h, cur.data_ptr(), ref.data_ptr(), W, H, pitch, stride, P, range_, algo,
                               mv.data_ptr(), sad.data_ptr(), nsp.data_ptr(), _stream(stream))
    _check(rc, "me_dcds_learned")
    return mv, sad, nsp


def dcds_surface(cost, valid=None, algo=ME_ALGO_DCDS, start=None, orient=None, stream=None):
    """DCDS over int32 cost surfaces [n, 2R+1, 2R+1] (device); returns (mv, cost, nsp)."""
    torch = _torch()
    if cost.dtype != torch.int32 or cost.dim() != 3 or not cost.is_contiguous():
        raise ValueError("cost must be a contiguous int32 [n, 2R+1, 2R+1] tensor")
    n, side, side2 = cost.shape
    if side != side2 or side % 2 != 1:
        raise ValueError("surfaces must be square with odd side")
    valid = _arg(valid, n * side * side, torch.uint8, cost.device, "valid")
    start = _arg(start, 2 * n, torch.int16, cost.device, "start")
    orient = _arg(orient, n, torch.uint8, cost.device, "orient")
    mv = torch.empty((n, 2), dtype=torch.int16, device=cost.device)
    cout = torch.empty((n,), dtype=torch.int32, device=cost.device)
    nsp = torch.empty((n,), dtype=torch.int32, device=cost.device)
    vp = valid.data_ptr() if valid is not None else None
    sp = start.data_ptr() if start is not None else None
    op = orient.data_ptr() if orient is not None else None
    rc = me_dcds_surface(cost.data_ptr(), vp, n, side // 2, algo, sp, op, mv.data_ptr(), cout.data_ptr(),
                         nsp.data_ptr(), _stream(stream))
    _check(rc, "me_dcds_surface")
    return mv, cout, nsp
