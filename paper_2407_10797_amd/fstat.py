"""Python binding of libfstat (include/fstat.h): argument marshalling only.

Every step of the F-statistic runs in the HIP kernels of ``libfstat.so``;
PyTorch supplies device memory and the current HIP stream.  If the library
has not been built this module raises on first use: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfstat.so")

FSTAT_OK = 0
FSTAT_EINVAL = -1
FSTAT_ENOMEM = -2
FSTAT_EDEVICE = -3
FSTAT_EUNSUPPORTED = -4
FSTAT_FP64 = 1
FSTAT_MIXED = 2
FSTAT_DEVICE_PTRS = 1
FSTAT_EVAL_MIXED = 2
FSTAT_PROFILE = 4
FSTAT_EVAL_SURROGATE = 8
FSTAT_AUTOTUNE_FORCE = 16
FSTAT_EVAL_EXACT = 32
FSTAT_AUTOTUNE_MODE = 64

EXPORTS = ("fstat_plan_create", "fstat_plan_set_orbit", "fstat_eval", "fstat_eval_noalloc",
           "fstat_extrinsic",
           "fstat_waveform", "pso_stage",
           "fstat_search", "fstat_search_boxes",
           "fstat_profile_read", "fstat_interp_stats", "fstat_autotune", "fstat_mlp_grad", "fstat_mlp_forward",
           "fstat_surrogate_train", "fstat_surrogate_stats", "fstat_surrogate_params",
           "fstat_plan_destroy",
           "fstat_calibrate", "fstat_last_error")


class fstat_data_desc(ctypes.Structure):
    _fields_ = [("T_obs", ctypes.c_double), ("df", ctypes.c_double),
                ("k_lo", ctypes.c_int64), ("nbins", ctypes.c_int64),
                ("data", ctypes.c_void_p), ("psd", ctypes.c_void_p),
                ("n_channels", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("channels", ctypes.c_void_p)]


CHANNELS = {"X": 0, "Y": 1, "Z": 2, "A": 3, "E": 4, "T": 5}


def channel_code(c) -> int:
    return CHANNELS[c] if isinstance(c, str) else int(c)


class fstat_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("chunk", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("refine_budget", ctypes.c_double)]


class pso_stage_desc(ctypes.Structure):
    _fields_ = [("n_runs", ctypes.c_int32), ("n_part", ctypes.c_int32),
                ("iters", ctypes.c_int32), ("ring_k", ctypes.c_int32),
                ("w_start", ctypes.c_double), ("w_end", ctypes.c_double),
                ("c1", ctypes.c_double), ("c2", ctypes.c_double), ("vmax", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("box", ctypes.c_void_p), ("np", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("use_graph", ctypes.c_int32)]


class pso_result(ctypes.Structure):
    _fields_ = [("best_x", ctypes.c_void_p), ("best_F", ctypes.c_void_p),
                ("trace", ctypes.c_void_p), ("final_x", ctypes.c_void_p)]


class fstat_search_desc(ctypes.Structure):
    _fields_ = [("box", (ctypes.c_double * 2) * 6), ("n_slices", ctypes.c_int32),
                ("runs", ctypes.c_int32 * 3), ("iters", ctypes.c_int32 * 3), ("np", ctypes.c_int32 * 3),
                ("n_part", ctypes.c_int32), ("ring_k", ctypes.c_int32),
                ("w_start", ctypes.c_double), ("w_end", ctypes.c_double), ("c1", ctypes.c_double),
                ("c2", ctypes.c_double), ("vmax", ctypes.c_double),
                ("width2", ctypes.c_double * 2), ("width3", ctypes.c_double * 5),
                ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint32 * 3), ("use_graph", ctypes.c_int32),
                ("max_stage", ctypes.c_int32), ("checkpoint", ctypes.c_char_p)]


class fstat_search_result(ctypes.Structure):
    _fields_ = [("stages_done", ctypes.c_int32), ("stages_resumed", ctypes.c_int32),
                ("stage1_x", ctypes.c_void_p), ("stage1_F", ctypes.c_void_p),
                ("stage2_x", ctypes.c_void_p), ("stage2_F", ctypes.c_void_p),
                ("stage3_x", (ctypes.c_double * 6) * 2), ("stage3_F", ctypes.c_double * 2),
                ("best_x", ctypes.c_double * 6), ("best_F", ctypes.c_double),
                ("amps", ctypes.c_double * 4), ("extrinsic", ctypes.c_double * 4),
                ("stage_ms", ctypes.c_double * 3), ("evals", ctypes.c_int64 * 3)]


class fstat_surrogate_desc(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int64), ("batch", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("lr", ctypes.c_double), ("seed", ctypes.c_uint64), ("loss_trace", ctypes.c_void_p),
                ("val_rmse", ctypes.c_double), ("val_max", ctypes.c_double)]


class FstatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libfstat error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfstat.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
        L.fstat_plan_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(fstat_data_desc),
                                        ctypes.POINTER(fstat_opts), vp]
        L.fstat_plan_create.restype = ctypes.c_int
        L.fstat_eval.argtypes = [vp, vp, i64, vp, i32, vp, vp, vp, i64, u32, vp]
        L.fstat_eval.restype = ctypes.c_int
        L.fstat_eval_noalloc.argtypes = [vp, vp, i64, vp, i32, vp, vp, vp, i64, u32, vp]
        L.fstat_eval_noalloc.restype = ctypes.c_int
        L.fstat_extrinsic.argtypes = [vp, vp, i64, vp, u32, vp]
        L.fstat_plan_set_orbit.argtypes = [vp, ctypes.c_double, ctypes.c_double, i32, vp, u32, vp]
        L.fstat_plan_set_orbit.restype = ctypes.c_int
        L.fstat_extrinsic.restype = ctypes.c_int
        L.fstat_waveform.argtypes = [ctypes.c_double, ctypes.c_double, i64, i64, vp, vp, vp, u32, vp]
        L.fstat_waveform.restype = ctypes.c_int
        L.pso_stage.argtypes = [vp, ctypes.POINTER(pso_stage_desc), ctypes.POINTER(pso_result), vp]
        L.pso_stage.restype = ctypes.c_int
        L.fstat_search.argtypes = [vp, ctypes.POINTER(fstat_search_desc),
                                   ctypes.POINTER(fstat_search_result), vp]
        L.fstat_search.restype = ctypes.c_int
        L.fstat_search_boxes.argtypes = [ctypes.POINTER(fstat_search_desc), i32, vp, i32, vp]
        L.fstat_search_boxes.restype = ctypes.c_int
        L.fstat_profile_read.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                         ctypes.POINTER(i64)]
        L.fstat_profile_read.restype = ctypes.c_int
        L.fstat_mlp_grad.argtypes = [vp, vp, vp, i32, ctypes.POINTER(ctypes.c_double), vp, vp]
        L.fstat_mlp_grad.restype = ctypes.c_int
        L.fstat_interp_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                         ctypes.POINTER(i64), vp, vp]
        L.fstat_interp_stats.restype = ctypes.c_int
        L.fstat_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.fstat_mlp_forward.restype = ctypes.c_int
        L.fstat_surrogate_train.argtypes = [vp, ctypes.POINTER(fstat_surrogate_desc), vp]
        L.fstat_surrogate_train.restype = ctypes.c_int
        L.fstat_surrogate_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, i64]
        L.fstat_surrogate_stats.restype = ctypes.c_int
        L.fstat_surrogate_params.argtypes = [vp, vp, vp, vp]
        L.fstat_surrogate_params.restype = ctypes.c_int
        L.fstat_autotune.argtypes = [vp, vp, i64, i32, vp, i32, u32, ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double), vp]
        L.fstat_autotune.restype = ctypes.c_int
        L.fstat_calibrate.argtypes = [i32, i64, i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), vp]
        L.fstat_calibrate.restype = ctypes.c_int
        L.fstat_plan_destroy.argtypes = [vp]
        L.fstat_plan_destroy.restype = None
        L.fstat_last_error.argtypes = []
        L.fstat_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def fstat_last_error() -> str:
    return lib().fstat_last_error().decode()


def _check(rc: int) -> None:
    if rc != FSTAT_OK:
        raise FstatError(rc, fstat_last_error())


# ---- same-name wrappers of the C entry points --------------------------------

def fstat_plan_create(desc: fstat_data_desc, opts: fstat_opts | None = None, stream=None):
    h = ctypes.c_void_p()
    _check(lib().fstat_plan_create(ctypes.byref(h), ctypes.byref(desc),
                                   ctypes.byref(opts) if opts is not None else None, stream))
    return h


def fstat_eval(plan, params, n, np_ptr, np_uniform, F_hat, F_part, amps, part_stride, flags,
               stream=None):
    _check(lib().fstat_eval(plan, params, int(n), np_ptr, int(np_uniform), F_hat, F_part, amps,
                            int(part_stride), int(flags), stream))


def fstat_eval_noalloc(plan, params, n, np_ptr, np_uniform, F_hat, F_part, amps, part_stride,
                       flags, stream=None):
    _check(lib().fstat_eval_noalloc(plan, params, int(n), np_ptr, int(np_uniform), F_hat, F_part,
                                    amps, int(part_stride), int(flags), stream))


FSTAT_CALIB_FMA64, FSTAT_CALIB_FMA32, FSTAT_CALIB_COPY = 0, 1, 2


def calibrate(kind: int, size: int, reps: int = 10):
    """Measured peak of one resource: (rate, ms per launch); rate in TFLOP/s
    for the FMA kinds, GB/s (read + written) for the copy."""
    rate, ms = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().fstat_calibrate(int(kind), int(size), int(reps), ctypes.byref(rate),
                                 ctypes.byref(ms), _stream()))
    return rate.value, ms.value


def fstat_plan_set_orbit(plan, t0, dt, n_seg, nodes, flags, stream=None):
    _check(lib().fstat_plan_set_orbit(plan, float(t0), float(dt), int(n_seg), nodes, int(flags),
                                      stream))


def fstat_extrinsic(amps, params, n, out, flags, stream=None):
    _check(lib().fstat_extrinsic(amps, params, int(n), out, int(flags), stream))


def fstat_waveform(T_obs, df, k_lo, nbins, params6, amps4, out, flags, stream=None):
    _check(lib().fstat_waveform(float(T_obs), float(df), int(k_lo), int(nbins), params6, amps4,
                                out, int(flags), stream))


def pso_stage(plan, desc: pso_stage_desc, result: pso_result, stream=None):
    _check(lib().pso_stage(plan, ctypes.byref(desc), ctypes.byref(result), stream))


def fstat_search(plan, desc: fstat_search_desc, result: fstat_search_result, stream=None):
    _check(lib().fstat_search(plan, ctypes.byref(desc), ctypes.byref(result), stream))


def fstat_search_boxes(desc: fstat_search_desc, stage, centres, n_centres, boxes_out):
    n = lib().fstat_search_boxes(ctypes.byref(desc), int(stage), centres, int(n_centres), boxes_out)
    if n < 0:
        raise FstatError(n, fstat_last_error())
    return n


YEAR_S = 365.25 * 86400.0

# Sec. III.B: 24 t_c intervals x 24 runs (N_seg 16, 8000 iterations), 24 spaces
# x 8 runs, 2 spaces (theta, pi - theta) x 48 runs (N_seg 1, 15000
# iterations); 128 particles; c1 = c2 = 2, vmax = 0.5 (Sec. III.A).
PAPER_SEARCH = dict(n_slices=24, runs=(24, 8, 48), iters=(8000, 8000, 15000), np=(16, 16, 1),
                    n_part=128, ring_k=1, w=(0.9, 0.4), c1=2.0, c2=2.0, vmax=0.5,
                    width2=(0.01 * YEAR_S, 0.6),
                    width3=(0.004 * YEAR_S, 0.3, 0.4, 0.4, 0.006))


def search_desc(box, seed: int = 1, flags=(0, 0, 0), use_graph: bool = True, max_stage: int = 0,
                checkpoint: str | None = None, **kw) -> fstat_search_desc:
    """Descriptor for fstat_search: PAPER_SEARCH settings overridden by kw."""
    c = dict(PAPER_SEARCH, **kw)
    box = np.asarray(box, dtype=np.float64).reshape(6, 2)
    d = fstat_search_desc()
    for j in range(6):
        d.box[j][0], d.box[j][1] = box[j]
    d.n_slices = int(c["n_slices"])
    for s in range(3):
        d.runs[s], d.iters[s], d.np[s] = int(c["runs"][s]), int(c["iters"][s]), int(c["np"][s])
        d.flags[s] = int(flags[s])
    d.n_part, d.ring_k = int(c["n_part"]), int(c["ring_k"])
    d.w_start, d.w_end = float(c["w"][0]), float(c["w"][1])
    d.c1, d.c2, d.vmax = float(c["c1"]), float(c["c2"]), float(c["vmax"])
    for j in range(2):
        d.width2[j] = float(c["width2"][j])
    for j in range(5):
        d.width3[j] = float(c["width3"][j])
    d.seed = int(seed)
    d.use_graph = int(use_graph)
    d.max_stage = int(max_stage)
    d.checkpoint = checkpoint.encode() if checkpoint else None
    return d


def search_boxes(desc: fstat_search_desc, stage: int, centres=None) -> np.ndarray:
    """Boxes [n, 6, 2] that stage `stage` of fstat_search searches."""
    cen = None if centres is None else np.ascontiguousarray(np.atleast_2d(centres), dtype=np.float64)
    nc = 0 if cen is None else cen.shape[0]
    cap = {1: desc.n_slices, 2: nc, 3: 2}.get(int(stage), 0)
    out = np.zeros((max(cap, 1), 6, 2))
    n = fstat_search_boxes(desc, stage, cen.ctypes.data if cen is not None else None, nc,
                           out.ctypes.data)
    return out[:n]


def fstat_profile_read(plan, reset: bool = True):
    ms, mm, n, bins = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fstat_profile_read(plan, int(reset), ctypes.byref(ms), ctypes.byref(mm),
                                    ctypes.byref(n), ctypes.byref(bins)))
    return ms.value, mm.value, n.value, bins.value


def fstat_mlp_grad(params, x, t):
    """(loss, grad, y) of one device forward/backward pass of the surrogate."""
    params = np.ascontiguousarray(params, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(t, dtype=np.float32)
    B = x.shape[0]
    grad = np.zeros_like(params)
    y = np.zeros(B, dtype=np.float32)
    loss = ctypes.c_double()
    _check(lib().fstat_mlp_grad(params.ctypes.data, x.ctypes.data, t.ctypes.data, int(B),
                                ctypes.byref(loss), grad.ctypes.data, y.ctypes.data))
    return loss.value, grad, y


def fstat_interp_stats(plan, stream=None, bin_mix=False):
    items, rej, ref = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    mix = (ctypes.c_int64 * 14)() if bin_mix else None
    _check(lib().fstat_interp_stats(plan, ctypes.byref(items), ctypes.byref(rej), ctypes.byref(ref),
                                    mix, stream))
    if bin_mix:
        return items.value, rej.value, ref.value, list(mix)
    return items.value, rej.value, ref.value


def fstat_mlp_forward(params, x):
    """y of the fused inference kernel of the surrogate network."""
    params = np.ascontiguousarray(params, dtype=np.float32)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.zeros(x.shape[0], dtype=np.float32)
    _check(lib().fstat_mlp_forward(params.ctypes.data, x.ctypes.data, ctypes.c_int64(x.shape[0]),
                                   y.ctypes.data))
    return y


def fstat_surrogate_train(plan, desc: fstat_surrogate_desc, stream=None):
    _check(lib().fstat_surrogate_train(plan, ctypes.byref(desc), stream))


def fstat_surrogate_stats(plan, n_flags: int = 0):
    used, fb = ctypes.c_int64(), ctypes.c_int64()
    flags = np.zeros(max(n_flags, 0), dtype=np.int32)
    _check(lib().fstat_surrogate_stats(plan, ctypes.byref(used), ctypes.byref(fb),
                                       flags.ctypes.data if n_flags > 0 else None, int(n_flags)))
    if n_flags > 0:
        return used.value, fb.value, flags
    return used.value, fb.value


N_SURROGATE_PARAMS = 198657


def fstat_surrogate_params(plan, params=None, stream=None):
    """Set the surrogate's weights from `params` (float32 [198,657]) or, with
    None, return the plan's trained weights."""
    if params is not None:
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != N_SURROGATE_PARAMS:
            raise ValueError("surrogate weights must have 198,657 values")
        _check(lib().fstat_surrogate_params(plan, p.ctypes.data, None, stream))
        return None
    out = np.zeros(N_SURROGATE_PARAMS, dtype=np.float32)
    _check(lib().fstat_surrogate_params(plan, None, out.ctypes.data, stream))
    return out


def fstat_autotune(plan, params, n, np_uniform, flags, stream=None, np_ptr=None, part_stride=0):
    c, m, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    _check(lib().fstat_autotune(plan, params, int(n), int(np_uniform), np_ptr, int(part_stride),
                                int(flags), ctypes.byref(c), ctypes.byref(m), ctypes.byref(ms),
                                stream))
    return c.value, m.value, ms.value


def fstat_plan_destroy(plan) -> None:
    if plan:
        lib().fstat_plan_destroy(plan)


# ---- torch conveniences (device memory + current stream) ---------------------

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device available")
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A plan over one data set, with inputs kept resident in device memory."""

    def __init__(self, data, psd, T_obs: float, df: float, k_lo: int,
                 precision: int = 0, chunk: int = 0, profile: bool = False,
                 refine_budget: float = 0.0, channels=None):
        """data, psd: [nbins] (one TDI-X channel) or, with `channels` (e.g.
        "AET"), [len(channels), nbins]."""
        torch = _torch()
        dev = torch.device("cuda")
        d = torch.as_tensor(np.ascontiguousarray(data, dtype=np.complex128)
                            if isinstance(data, np.ndarray) else data)
        d = d.to(dev, torch.complex128).contiguous()
        p = torch.as_tensor(psd).to(dev, torch.float64).contiguous()
        nch = 1 if channels is None else len(channels)
        self.channels = None if channels is None else [channel_code(c) for c in channels]
        if p.numel() % nch or d.numel() != p.numel():
            raise ValueError("data and psd must be [channels, nbins]")
        self.nbins = int(p.numel()) // nch
        self.T_obs, self.df, self.k_lo = float(T_obs), float(df), int(k_lo)
        self._chan = (np.ascontiguousarray(self.channels, dtype=np.int32)
                      if self.channels is not None else None)
        desc = fstat_data_desc(self.T_obs, self.df, self.k_lo, self.nbins,
                               d.data_ptr(), p.data_ptr(), nch if channels is not None else 0, 0,
                               self._chan.ctypes.data if self._chan is not None else None)
        opts = fstat_opts(int(precision), FSTAT_DEVICE_PTRS | (FSTAT_PROFILE if profile else 0),
                          int(chunk), 0, float(refine_budget))
        self.handle = fstat_plan_create(desc, opts, _stream())
        torch.cuda.current_stream().synchronize()

    def eval(self, params, np_parts=1, part_stride: int | None = None, mixed: bool = False,
             want_parts: bool = False, surrogate: bool = False, exact: bool = False,
             want_amps: bool = False, noalloc: bool = False):
        """F_hat [n] (and F_part [n, stride], amps [n, stride, 4]) for params
        [n, 6] on the device; noalloc: through fstat_eval_noalloc (the
        library's fixed scratch instead of the plan's workspace)."""
        torch = _torch()
        prm = torch.as_tensor(params).to("cuda", torch.float64).contiguous()
        n = prm.shape[0]
        F = torch.empty(n, device="cuda", dtype=torch.float64)
        if isinstance(np_parts, int):
            npp, npu = None, np_parts
            stride = part_stride or np_parts
            np_t = None
        else:
            np_t = torch.as_tensor(np_parts).to("cuda", torch.int32).contiguous()
            npp, npu = np_t.data_ptr(), 0
            stride = part_stride or int(np_t.max().item())
        Fp = torch.zeros((n, stride), device="cuda", dtype=torch.float64) if want_parts else None
        Am = torch.zeros((n, stride, 4), device="cuda", dtype=torch.float64) if want_amps else None
        flags = (FSTAT_DEVICE_PTRS | (FSTAT_EVAL_MIXED if mixed else 0)
                 | (FSTAT_EVAL_SURROGATE if surrogate else 0) | (FSTAT_EVAL_EXACT if exact else 0))
        (fstat_eval_noalloc if noalloc else fstat_eval)(
            self.handle, prm.data_ptr(), n, npp, npu, F.data_ptr(),
            Fp.data_ptr() if Fp is not None else None,
            Am.data_ptr() if Am is not None else None, stride, flags, _stream())
        out = (F,)
        if want_parts:
            out += (Fp,)
        if want_amps:
            out += (Am,)
        return out if len(out) > 1 else F

    def pso(self, box, np_runs, n_part: int, iters: int, ring_k: int = 1, w=(0.7, 0.7),
            c1: float = 1.5, c2: float = 1.5, vmax: float = 0.5, seed: int = 1,
            mixed: bool = False, use_graph: bool = True, want_trace: bool = True,
            want_final: bool = False, surrogate: bool = False, exact: bool = False):
        """Run pso_stage: box [R, 6, 2] (physical), np_runs [R].  Returns dict
        with best_x [R, 6], best_F [R], trace [iters, R], final_x [R, n_part, 6]."""
        _torch()
        box = np.ascontiguousarray(box, dtype=np.float64).reshape(-1, 6, 2)
        R = box.shape[0]
        npr = np.ascontiguousarray(np.broadcast_to(np.asarray(np_runs, dtype=np.int32), (R,)))
        best_x = np.zeros((R, 6)); best_F = np.zeros(R)
        trace = np.zeros((max(iters, 1), R)) if want_trace else None
        final_x = np.zeros((R, n_part, 6)) if want_final else None
        desc = pso_stage_desc(R, int(n_part), int(iters), int(ring_k), float(w[0]), float(w[1]),
                              float(c1), float(c2), float(vmax), int(seed), box.ctypes.data,
                              npr.ctypes.data,
                              (FSTAT_EVAL_MIXED if mixed else 0) | (FSTAT_EVAL_SURROGATE if surrogate else 0)
                              | (FSTAT_EVAL_EXACT if exact else 0),
                              int(use_graph))
        res = pso_result(best_x.ctypes.data, best_F.ctypes.data,
                         trace.ctypes.data if trace is not None else None,
                         final_x.ctypes.data if final_x is not None else None)
        pso_stage(self.handle, desc, res, _stream())
        out = dict(best_x=best_x, best_F=best_F)
        if trace is not None:
            out["trace"] = trace[:iters]
        if final_x is not None:
            out["final_x"] = final_x
        return out

    def set_orbit(self, t0: float = 0.0, dt: float = 1.0, nodes=None):
        """Numerical orbit: nodes [n_seg, 3, 3, 10] positions [s] at the
        Chebyshev points of each segment (see fstat_plan_set_orbit); None
        returns to the analytic orbit."""
        if nodes is None:
            fstat_plan_set_orbit(self.handle, 0.0, 1.0, 0, None, 0, _stream())
            return
        if tuple(nodes.shape[1:]) != (3, 3, 10) or len(nodes.shape) != 4:
            raise ValueError("nodes must be [n_seg, 3, 3, 10]")
        if hasattr(nodes, "is_cuda") and nodes.is_cuda:       # a device tensor
            import torch
            nd = nodes.to(torch.float64).contiguous()
            fstat_plan_set_orbit(self.handle, t0, dt, nd.shape[0], nd.data_ptr(),
                                 FSTAT_DEVICE_PTRS, _stream())
            return
        nd = np.ascontiguousarray(nodes, dtype=np.float64)
        fstat_plan_set_orbit(self.handle, t0, dt, nd.shape[0], nd.ctypes.data, 0, _stream())

    def search(self, desc: fstat_search_desc) -> dict:
        """Run fstat_search; returns its results as numpy arrays and floats."""
        _torch()
        n = desc.n_slices
        s1x, s1F = np.zeros((n, 6)), np.zeros(n)
        s2x, s2F = np.zeros((n, 6)), np.zeros(n)
        r = fstat_search_result()
        r.stage1_x, r.stage1_F = s1x.ctypes.data, s1F.ctypes.data
        r.stage2_x, r.stage2_F = s2x.ctypes.data, s2F.ctypes.data
        fstat_search(self.handle, desc, r, _stream())
        return dict(stages_done=r.stages_done, stages_resumed=r.stages_resumed,
                    stage1_x=s1x, stage1_F=s1F, stage2_x=s2x, stage2_F=s2F,
                    stage3_x=np.array(r.stage3_x), stage3_F=np.array(r.stage3_F),
                    best_x=np.array(r.best_x), best_F=r.best_F, amps=np.array(r.amps),
                    extrinsic=np.array(r.extrinsic), stage_ms=np.array(r.stage_ms),
                    evals=np.array(r.evals))

    def train_surrogate(self, n_samples: int = 2_000_000, batch: int = 4096, steps: int = 4000,
                        lr: float = 1e-3, seed: int = 5001, want_trace: bool = False):
        """Train the eccentric-phase surrogate on the device; returns a dict with
        held-out rmse/max error (network units) and optionally the loss trace."""
        trace = np.zeros(steps) if want_trace else None
        desc = fstat_surrogate_desc(int(n_samples), int(batch), int(steps), float(lr), int(seed),
                                    trace.ctypes.data if trace is not None else None, 0.0, 0.0)
        fstat_surrogate_train(self.handle, desc, _stream())
        out = dict(val_rmse=desc.val_rmse, val_max=desc.val_max)
        if trace is not None:
            out["loss_trace"] = trace
        return out

    def autotune(self, params, np_parts, mixed: bool = False, force: bool = False,
                 exact: bool = False, mode: bool = False):
        """Pick the work-item size and grid multiplier for this precision (and
        with `mode` whether the exact loop beats the interpolating one) for a
        batch like params [n, 6] with np_parts (int, or [n] per particle);
        returns (chunk, grid multiplier, best ms or -1 if cached)."""
        torch = _torch()
        prm = torch.as_tensor(params).to("cuda", torch.float64).contiguous()
        flags = (FSTAT_DEVICE_PTRS | (FSTAT_EVAL_MIXED if mixed else 0)
                 | (FSTAT_AUTOTUNE_FORCE if force else 0) | (FSTAT_EVAL_EXACT if exact else 0)
                 | (FSTAT_AUTOTUNE_MODE if mode else 0))
        if isinstance(np_parts, int):
            return fstat_autotune(self.handle, prm.data_ptr(), prm.shape[0], int(np_parts), flags,
                                  _stream())
        npt = torch.as_tensor(np_parts).to("cuda", torch.int32).contiguous()
        return fstat_autotune(self.handle, prm.data_ptr(), prm.shape[0], 0, flags, _stream(),
                              npt.data_ptr(), int(npt.max().item()))

    def interp_stats(self, bin_mix: bool = False):
        """(work items, items handed to the exact loop, items refined exactly) of
        the last evaluation, and with bin_mix the bins by kind of per-bin work
        ([0..2] phase and sine per bin at transfer degree 5, 7, 9; [3..5] the
        difference recurrence at degree 5, 7, 9 -- mixed path: [0] degree 4,
        [2] degree 6 with nine phase differences, [3], [5] the same with four;
        [6] exact), then [7 + k] the lanes with bins (runs) of the items of
        kind k < 6 and [13] the items evaluated exactly."""
        return fstat_interp_stats(self.handle, _stream(), bin_mix)

    def surrogate_stats(self, n_flags: int = 0):
        """(particles that used the surrogate, particles that fell back) in the last
        surrogate evaluation, and with n_flags > 0 the per-particle flags of its
        first n_flags particles (1: surrogate used)."""
        return fstat_surrogate_stats(self.handle, n_flags)

    def surrogate_params(self, params=None):
        """The trained surrogate weights (float32 [198,657]), or with `params`
        load them into this plan (marks the surrogate trained)."""
        return fstat_surrogate_params(self.handle, params, _stream())

    def profile_read(self, reset: bool = True):
        """(bin-loop stage ms, its main kernel ms, evaluations, bin-template
        evaluations), totals since the last reset."""
        return fstat_profile_read(self.handle, reset)

    def close(self):
        if getattr(self, "handle", None):
            fstat_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def waveform(T_obs, df, k_lo, nbins, params6, amps4, channel="X"):
    """sum_i a_i A^i of a TDI channel on the grid, computed on the device;
    returns a torch complex128 tensor on the device."""
    torch = _torch()
    p = torch.as_tensor(np.asarray(params6, dtype=np.float64)).cuda()
    a = torch.as_tensor(np.asarray(amps4, dtype=np.float64)).cuda()
    out = torch.empty(int(nbins), device="cuda", dtype=torch.complex128)
    fstat_waveform(T_obs, df, k_lo, nbins, p.data_ptr(), a.data_ptr(), out.data_ptr(),
                   FSTAT_DEVICE_PTRS | (channel_code(channel) << 8), _stream())
    return out


def extrinsic(amps, params=None):
    """(D_L, iota, psi, phi_c) [n, 4] from amplitudes [n, 4] on the device
    (App. B); D_L in metres when params [n, 6] are given, else in 1/a units."""
    torch = _torch()
    a = torch.as_tensor(amps).to("cuda", torch.float64).reshape(-1, 4).contiguous()
    p = None
    if params is not None:
        p = torch.as_tensor(params).to("cuda", torch.float64).reshape(-1, 6).contiguous()
        if p.shape[0] != a.shape[0]:
            raise ValueError("params and amps differ in rows")
    out = torch.empty_like(a)
    fstat_extrinsic(a.data_ptr(), p.data_ptr() if p is not None else None, a.shape[0],
                    out.data_ptr(), FSTAT_DEVICE_PTRS, _stream())
    return out
