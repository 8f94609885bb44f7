"""ctypes binding of libhmfsr's C ABI (``include/hmfsr.h``).

Argument marshalling only: every step of the merge runs in the library's HIP
kernels. Functions keep the C names; they take integer device addresses and a
raw hipStream_t handle, and raise ``HmfsrError`` on any non-OK status. The
library must have been built (``paper_1905_03277_amd.build``); there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmfsr.so")

HMFSR_OK, HMFSR_E_INVALID, HMFSR_E_UNSUPPORTED, HMFSR_E_HIP, HMFSR_E_NOMEM = 0, -1, -2, -3, -4
HMFSR_E_TOO_LARGE, HMFSR_E_DATA = -5, -6
NOALLOC_SCRATCH_BYTES = 64 << 20   # HMFSR_NOALLOC_SCRATCH_BYTES

# Every symbol include/hmfsr.h declares.
EXPORTED = ("hmfsr_merge", "hmfsr_merge_noalloc", "hmfsr_merge_backward", "hmfsr_stream_begin", "hmfsr_stream_add",
            "hmfsr_stream_end", "hmfsr_align", "hmfsr_noise_table", "hmfsr_auto_tuning",
            "hmfsr_merge_maps", "hmfsr_merge_batch", "hmfsr_batch_plan", "hmfsr_autotune",
            "hmfsr_profile_begin", "hmfsr_profile_end", "hmfsr_strerror", "hmfsr_version",
            "hmfsr_release")

STAGE_PRIOR, STAGE_ROBUST, STAGE_MERGE, STAGE_BATCH = 0, 1, 2, 3
STAGE_MERGE_BWD, STAGE_ROBUST_BWD, STAGE_GRAD_REDUCE, STAGE_ALIGN = 4, 5, 6, 7
NUM_STAGES = 8
STAGE_NAMES = {STAGE_PRIOR: "k_prior", STAGE_ROBUST: "k_robust", STAGE_MERGE: "k_merge",
               STAGE_BATCH: "batch_graph", STAGE_MERGE_BWD: "k_merge_bwd",
               STAGE_ROBUST_BWD: "k_robust_bwd", STAGE_GRAD_REDUCE: "k_grad_reduce",
               STAGE_ALIGN: "align"}

# Order of hmfsr_merge_backward's grad_tuning.
GRAD_NAMES = ("k_detail", "k_denoise", "d_th", "d_tr", "k_stretch", "k_shrink", "s", "t", "s_motion")


class hmfsr_desc(ctypes.Structure):
    _fields_ = [("n_frames", ctypes.c_int32), ("height", ctypes.c_int32),
                ("width", ctypes.c_int32), ("ref_frame", ctypes.c_int32),
                ("cfa", ctypes.c_int32), ("black_level", ctypes.c_float),
                ("white_level", ctypes.c_float), ("noise_a", ctypes.c_float),
                ("noise_b", ctypes.c_float), ("tile_size", ctypes.c_int32),
                ("scale", ctypes.c_float), ("out_height", ctypes.c_int32),
                ("out_width", ctypes.c_int32), ("noise_bins", ctypes.c_int32),
                ("noise_table", ctypes.c_void_p)]


class hmfsr_tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in
                ("k_detail", "k_denoise", "d_th", "d_tr", "k_stretch", "k_shrink", "s", "t",
                 "s_motion", "m_th", "hf_ratio")]


class hmfsr_align_params(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("radius_coarse", ctypes.c_int32),
                ("radius_fine", ctypes.c_int32), ("lk_iterations", ctypes.c_int32),
                ("gate", ctypes.c_float)]


ALIGN_DEFAULTS = dict(levels=4, radius_coarse=4, radius_fine=2, lk_iterations=3, gate=4.0)


class hmfsr_stage_times(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double * NUM_STAGES), ("launches", ctypes.c_int64 * NUM_STAGES)]


class hmfsr_batch_info(ctypes.Structure):
    _fields_ = [("robust_items", ctypes.c_int32), ("robust_groups", ctypes.c_int32),
                ("merge_items", ctypes.c_int32 * 8), ("merge_groups", ctypes.c_int32 * 8)]


class HmfsrError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhmfsr.so (once). Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1905_03277_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32 = ctypes.c_void_p, ctypes.c_int32
        pd, pt = ctypes.POINTER(hmfsr_desc), ctypes.POINTER(hmfsr_tuning)
        L.hmfsr_merge.argtypes = [pd, pt, vp, vp, vp, vp, vp]
        L.hmfsr_merge.restype = i32
        L.hmfsr_merge_noalloc.argtypes = [pd, pt, vp, vp, vp, vp, vp]
        L.hmfsr_merge_noalloc.restype = i32
        L.hmfsr_merge_backward.argtypes = [pd, pt, vp, vp, vp, vp, vp, vp, vp]
        L.hmfsr_merge_backward.restype = i32
        L.hmfsr_stream_begin.argtypes = [pd, pt, vp, vp, vp]
        L.hmfsr_stream_begin.restype = i32
        L.hmfsr_stream_add.argtypes = [pd, pt, vp, vp, vp, vp, vp]
        L.hmfsr_stream_add.restype = i32
        L.hmfsr_stream_end.argtypes = [pd, pt, vp, vp, vp]
        L.hmfsr_stream_end.restype = i32
        L.hmfsr_align.argtypes = [pd, ctypes.POINTER(hmfsr_align_params), vp, vp, vp, vp]
        L.hmfsr_align.restype = i32
        L.hmfsr_noise_table.argtypes = [pd, i32, i32, ctypes.c_uint64, vp, vp]
        L.hmfsr_noise_table.restype = i32
        L.hmfsr_auto_tuning.argtypes = [pd, vp, pt, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), vp]
        L.hmfsr_auto_tuning.restype = i32
        L.hmfsr_merge_maps.argtypes = [pd, pt, vp, vp, vp, vp, vp, vp, vp]
        L.hmfsr_merge_maps.restype = i32
        L.hmfsr_merge_batch.argtypes = [i32, pd, pt, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), vp]
        L.hmfsr_merge_batch.restype = i32
        L.hmfsr_batch_plan.argtypes = [ctypes.POINTER(hmfsr_batch_info)]
        L.hmfsr_batch_plan.restype = i32
        L.hmfsr_autotune.argtypes = [pd, pt, vp, vp, vp, vp, ctypes.POINTER(i32)]
        L.hmfsr_autotune.restype = i32
        L.hmfsr_profile_begin.argtypes = []
        L.hmfsr_profile_begin.restype = i32
        L.hmfsr_profile_end.argtypes = [ctypes.POINTER(hmfsr_stage_times)]
        L.hmfsr_profile_end.restype = i32
        L.hmfsr_strerror.argtypes = [i32]
        L.hmfsr_strerror.restype = ctypes.c_char_p
        L.hmfsr_version.argtypes = []
        L.hmfsr_version.restype = i32
        L.hmfsr_release.argtypes = []
        L.hmfsr_release.restype = None
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().hmfsr_strerror(int(status)).decode()


def _check(status: int, what: str):
    if status != HMFSR_OK:
        raise HmfsrError(status, what)


def make_desc(d) -> hmfsr_desc:
    """hmfsr_desc from any object with the same field names. ``noise_table``
    (optional) must be a contiguous float32 device tensor [bins][4]; the bin
    count is taken from its shape."""
    vals = []
    table = getattr(d, "noise_table", None)
    for f, _ in hmfsr_desc._fields_:
        if f == "noise_table":
            if table is None:
                vals.append(None)
            else:
                if not (hasattr(table, "is_cuda") and table.is_cuda and table.is_contiguous()
                        and str(table.dtype) == "torch.float32" and table.dim() == 2
                        and table.shape[1] == 4):
                    raise ValueError("noise_table must be a contiguous float32 device tensor [bins][4]")
                vals.append(table.data_ptr())
        elif f == "noise_bins":
            vals.append(0 if table is None else int(table.shape[0]))
        else:
            vals.append(getattr(d, f))
    return hmfsr_desc(*vals)


def make_tuning(t) -> hmfsr_tuning:
    """hmfsr_tuning from any object with the same field names (hf_ratio may be
    absent: 0, the high-frequency rejection off)."""
    return hmfsr_tuning(*(getattr(t, f, 0.0) if f == "hf_ratio" else getattr(t, f)
                          for f, _ in hmfsr_tuning._fields_))


def hmfsr_merge(desc: hmfsr_desc, tuning: hmfsr_tuning, frames: int, motion: int, out: int,
                saved: int = 0, stream: int = 0) -> None:
    _check(lib().hmfsr_merge(ctypes.byref(desc), ctypes.byref(tuning), frames, motion, out,
                             saved or None, stream or None), "hmfsr_merge")


def hmfsr_merge_noalloc(desc: hmfsr_desc, tuning: hmfsr_tuning, frames: int, motion: int, out: int,
                        saved: int = 0, stream: int = 0) -> None:
    _check(lib().hmfsr_merge_noalloc(ctypes.byref(desc), ctypes.byref(tuning), frames, motion, out,
                                     saved or None, stream or None), "hmfsr_merge_noalloc")


def hmfsr_merge_backward(desc: hmfsr_desc, tuning: hmfsr_tuning, frames: int, motion: int,
                         saved: int, grad_out: int, grad_tuning: int, grad_motion: int,
                         stream: int = 0) -> None:
    _check(lib().hmfsr_merge_backward(ctypes.byref(desc), ctypes.byref(tuning), frames, motion,
                                      saved or None, grad_out, grad_tuning, grad_motion,
                                      stream or None), "hmfsr_merge_backward")


def hmfsr_stream_begin(desc, tuning, base_frame: int, state: int, stream: int = 0) -> None:
    _check(lib().hmfsr_stream_begin(ctypes.byref(desc), ctypes.byref(tuning), base_frame, state,
                                    stream or None), "hmfsr_stream_begin")


def hmfsr_stream_add(desc, tuning, base_frame: int, frame: int, motion: int, state: int,
                     stream: int = 0) -> None:
    _check(lib().hmfsr_stream_add(ctypes.byref(desc), ctypes.byref(tuning), base_frame, frame, motion,
                                  state, stream or None), "hmfsr_stream_add")


def hmfsr_stream_end(desc, tuning, state: int, out: int, stream: int = 0) -> None:
    _check(lib().hmfsr_stream_end(ctypes.byref(desc), ctypes.byref(tuning), state, out, stream or None),
           "hmfsr_stream_end")


def make_align_params(params=None) -> hmfsr_align_params:
    """hmfsr_align_params from a dict (missing keys take the defaults)."""
    p = dict(ALIGN_DEFAULTS)
    p.update(params or {})
    return hmfsr_align_params(*((float if t is ctypes.c_float else int)(p[f]) for f, t in hmfsr_align_params._fields_))


def hmfsr_align(desc, params, frames: int, motion: int, block_match: int = 0, stream: int = 0) -> None:
    """params: hmfsr_align_params or None (the library's defaults)."""
    _check(lib().hmfsr_align(ctypes.byref(desc), ctypes.byref(params) if params is not None else None,
                             frames, motion, block_match or None, stream or None), "hmfsr_align")


def hmfsr_noise_table(desc, bins: int, patches: int, seed: int, table: int, stream: int = 0) -> None:
    _check(lib().hmfsr_noise_table(ctypes.byref(desc), int(bins), int(patches), int(seed), table,
                                   stream or None), "hmfsr_noise_table")


def hmfsr_auto_tuning(desc, frames: int, stream: int = 0):
    """(hmfsr_tuning, tile size, SNR) for the burst's base frame."""
    tun = hmfsr_tuning()
    tile = ctypes.c_int32(0)
    snr = ctypes.c_double(0.0)
    _check(lib().hmfsr_auto_tuning(ctypes.byref(desc), frames, ctypes.byref(tun), ctypes.byref(tile),
                                   ctypes.byref(snr), stream or None), "hmfsr_auto_tuning")
    return tun, tile.value, snr.value


def hmfsr_merge_maps(desc, tuning, frames: int, motion: int, omega: int, robust: int,
                     robust_min: int, s_tile: int, stream: int = 0) -> None:
    _check(lib().hmfsr_merge_maps(ctypes.byref(desc), ctypes.byref(tuning), frames, motion,
                                  omega or None, robust or None, robust_min or None,
                                  s_tile or None, stream or None), "hmfsr_merge_maps")


def hmfsr_merge_batch(descs, tunings, frames, motion, out, stream: int = 0) -> None:
    """descs / tunings: sequences of hmfsr_desc / hmfsr_tuning; frames, motion,
    out: sequences of device addresses."""
    n = len(descs)
    D = (hmfsr_desc * n)(*descs)
    T = (hmfsr_tuning * n)(*tunings)
    F = (ctypes.c_void_p * n)(*frames)
    M = (ctypes.c_void_p * n)(*motion)
    O = (ctypes.c_void_p * n)(*out)
    _check(lib().hmfsr_merge_batch(n, D, T, F, M, O, stream or None), "hmfsr_merge_batch")


def hmfsr_batch_plan() -> dict:
    """Items and workgroups of the persistent launches of the last captured
    batch graph on the current device."""
    info = hmfsr_batch_info()
    _check(lib().hmfsr_batch_plan(ctypes.byref(info)), "hmfsr_batch_plan")
    return {"robust_items": info.robust_items, "robust_groups": info.robust_groups,
            "merge_items": list(info.merge_items), "merge_groups": list(info.merge_groups)}


def hmfsr_autotune(desc, tuning, frames: int, motion: int, out: int, stream: int = 0) -> int:
    """Time every tile shape on this burst; returns the chosen shape's index."""
    chosen = ctypes.c_int32(-1)
    _check(lib().hmfsr_autotune(ctypes.byref(desc), ctypes.byref(tuning), frames, motion, out,
                                stream or None, ctypes.byref(chosen)), "hmfsr_autotune")
    return chosen.value


def hmfsr_profile_begin() -> None:
    _check(lib().hmfsr_profile_begin(), "hmfsr_profile_begin")


def hmfsr_profile_end() -> dict:
    """{stage name: (total ms, launches)} of the launches since hmfsr_profile_begin."""
    t = hmfsr_stage_times()
    _check(lib().hmfsr_profile_end(ctypes.byref(t)), "hmfsr_profile_end")
    return {STAGE_NAMES.get(i, f"stage{i}"): (t.ms_total[i], int(t.launches[i]))
            for i in range(NUM_STAGES) if t.launches[i]}


def hmfsr_version() -> int:
    return int(lib().hmfsr_version())


def hmfsr_release() -> None:
    lib().hmfsr_release()
