"""ctypes view of liblsr.so.  Fails loudly when the HIP library is missing."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblsr.so")

ACCEPTED, REJECTED, DEGENERATE = 1, 2, 3
FP32, BF16_SCREEN = 0, 1

_LIB = None
_CTX = {}


class LsrError(RuntimeError):
    pass


class Params(C.Structure):
    _fields_ = [
        ("r_normal", C.c_float), ("r_feature", C.c_float), ("max_corr", C.c_float), ("tau", C.c_float),
        ("n_trials", C.c_int64), ("gnc_div", C.c_double), ("gnc_every", C.c_int32),
        ("gnc_max_iter", C.c_int32), ("polish_iter", C.c_int32), ("min_inlier_ratio", C.c_float),
        ("min_consistent", C.c_int64), ("normal_check", C.c_int32), ("normal_cos", C.c_float),
        ("precision", C.c_int32), ("seed", C.c_uint64),
    ]


class Result(C.Structure):
    _fields_ = [
        ("T", C.c_double * 16), ("energy", C.c_double), ("mu_final", C.c_double),
        ("inlier_ratio", C.c_double), ("fitness", C.c_double),
        ("n_valid_P", C.c_int64), ("n_valid_Q", C.c_int64), ("n_recip", C.c_int64),
        ("n_consistent", C.c_int64), ("n_inliers", C.c_int64), ("n_fallback_rows", C.c_int64),
        ("n_screen_chunks", C.c_int64), ("n_screen_chunks_swept", C.c_int64),
        ("status", C.c_int32), ("iters", C.c_int32),
    ]


MAX_VARIANTS = 8
PRUNED_SCREEN = 5          # screen variant that skips the partner's chunks by their centroid bounds


class Tune(C.Structure):
    _fields_ = [("screen_shape", C.c_int32), ("consistency_shape", C.c_int32),
                ("n_screen_shapes", C.c_int32), ("n_consistency_shapes", C.c_int32),
                ("screen_ms", C.c_float * MAX_VARIANTS), ("consistency_ms", C.c_float * MAX_VARIANTS),
                ("from_cache", C.c_int32), ("pad", C.c_int32)]


class Trace(C.Structure):
    _fields_ = [("nnQ", C.c_void_p), ("nnP", C.c_void_p), ("mutual", C.c_void_p), ("consistent", C.c_void_p),
                ("desc_P", C.c_void_p), ("desc_Q", C.c_void_p), ("valid_P", C.c_void_p), ("valid_Q", C.c_void_p)]


class RansacResult(C.Structure):
    _fields_ = [("T", C.c_double * 16), ("inlier_ratio", C.c_double), ("fitness", C.c_double),
                ("sum_d2", C.c_double), ("n_hypotheses", C.c_int64), ("n_survivors", C.c_int64),
                ("n_fitted", C.c_int64), ("best", C.c_int64), ("n_inliers", C.c_int64),
                ("n_valid_P", C.c_int64), ("n_valid_Q", C.c_int64), ("status", C.c_int32), ("pad", C.c_int32)]


class RansacTrace(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("hyp", C.c_void_p), ("members", C.c_void_p), ("n_inliers", C.c_void_p),
                ("sum_d2", C.c_void_p), ("T", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("z_min", C.c_double), ("z_max", C.c_double)]


class Edge(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("T", C.c_double * 16)]


class LoopParams(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("tau", C.c_double), ("l_min", C.c_double), ("tol", C.c_double),
                ("eps", C.c_float), ("max_iter", C.c_int32)]


class LoopResult(C.Structure):
    _fields_ = [("l", C.c_double), ("f_loop", C.c_double), ("energy", C.c_double), ("mu", C.c_double),
                ("n_corr", C.c_int64), ("status", C.c_int32), ("iters", C.c_int32)]


class Cloud(C.Structure):
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("nx", C.c_void_p), ("ny", C.c_void_p), ("nz", C.c_void_p), ("n", C.c_int64)]


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LsrError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.lsr_create.argtypes = [C.POINTER(vp), C.c_int, C.c_size_t]
        L.lsr_destroy.argtypes = [vp]
        L.lsr_last_error.argtypes = [vp]
        L.lsr_last_error.restype = C.c_char_p
        L.lsr_default_params.argtypes = [C.POINTER(Params)]
        L.lsr_register_pair.argtypes = [vp, C.POINTER(Cloud), C.POINTER(Cloud), C.POINTER(Params), vp, vp]
        L.lsr_register_batch.argtypes = [vp, C.POINTER(Cloud), C.POINTER(Cloud), vp, vp, i32,
                                         C.POINTER(Params), vp, vp]
        L.lsr_register_batch_trace.argtypes = [vp, C.POINTER(Cloud), C.POINTER(Cloud), vp, vp, i32,
                                               C.POINTER(Params), vp, C.POINTER(Trace), vp]
        L.lsr_align_loss.argtypes = [vp, vp, i64, vp, i64, vp, vp, i32, vp, vp, vp, vp]
        L.lsr_align_loss_backward.argtypes = [vp, vp, i64, vp, i64, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.lsr_stage_normals.argtypes = [vp, C.POINTER(Cloud), C.c_float, vp, vp]
        L.lsr_stage_fpfh.argtypes = [vp, C.POINTER(Cloud), vp, C.c_float, vp, vp, vp]
        L.lsr_voxel_downsample.argtypes = [vp, C.POINTER(Cloud), C.c_float, vp, vp, vp]
        L.lsr_stage_spfh.argtypes = [vp, C.POINTER(Cloud), vp, C.c_float, vp, vp, vp]
        L.lsr_stage_match.argtypes = [vp, vp, vp, i64, vp, vp, i64, i32, vp, vp, vp, vp, vp, vp]
        L.lsr_stage_consistency.argtypes = [vp, C.POINTER(Cloud), C.POINTER(Cloud), vp, vp, i64, C.c_float,
                                            C.c_uint64, vp, vp, vp]
        L.lsr_stage_gnc.argtypes = [vp, vp, vp, i64, C.POINTER(Params), vp, vp, vp]
        L.lsr_stage_gnc_noalloc.argtypes = [vp, vp, vp, i64, C.POINTER(Params), vp, vp, vp]
        L.lsr_stage_verify.argtypes = [vp, C.POINTER(Cloud), vp, C.POINTER(Cloud), vp, vp, C.c_float, i32,
                                       C.c_float, vp, vp]
        L.lsr_ransac_pair.argtypes = [vp, C.POINTER(Cloud), C.POINTER(Cloud), C.POINTER(Params), i64, vp, vp]
        L.lsr_stage_ransac.argtypes = [vp, C.POINTER(Cloud), vp, C.POINTER(Cloud), vp, vp, i64, C.POINTER(Params),
                                       vp, C.POINTER(RansacTrace), vp]
        L.lsr_surfel_correct.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, i32, C.POINTER(Camera), vp, vp, vp, vp,
                                         vp]
        L.lsr_default_loop_params.argtypes = [C.POINTER(LoopParams)]
        L.lsr_edge_info.argtypes = [vp, vp, i32, vp, i32, C.c_float, vp, vp, vp]
        L.lsr_loop_solve.argtypes = [vp, i32, vp, vp, vp, vp, i32, vp, vp, C.POINTER(LoopParams), vp, vp, vp]
        L.lsr_loop_verify.argtypes = [vp, vp, i32, vp, vp, vp, i32, C.POINTER(LoopParams), vp, vp, vp]
        L.lsr_se3_retract.argtypes = [vp, i32, vp, vp, vp, vp]
        L.lsr_se3_retract_grad.argtypes = [vp, i32, vp, vp, vp, vp]
        L.lsr_set_timing.argtypes = [vp, C.c_int]
        L.lsr_autotune.argtypes = [vp, C.POINTER(Cloud), C.POINTER(Cloud), vp, vp, i32, C.POINTER(Params), i32,
                                   C.POINTER(Tune), vp]
        L.lsr_get_tune.argtypes = [vp, C.POINTER(Tune)]
        L.lsr_set_tune_cache.argtypes = [vp, C.c_char_p]
        L.lsr_set_tune.argtypes = [vp, C.POINTER(Tune)]
        L.lsr_get_timing.argtypes = [vp, C.c_int, vp, vp, C.POINTER(C.c_int)]
        for f in ("lsr_set_timing", "lsr_get_timing", "lsr_create", "lsr_register_pair", "lsr_register_batch",
                  "lsr_register_batch_trace", "lsr_align_loss",
                  "lsr_align_loss_backward", "lsr_stage_normals", "lsr_stage_fpfh", "lsr_stage_spfh", "lsr_voxel_downsample", "lsr_stage_match",
                  "lsr_stage_consistency", "lsr_stage_gnc", "lsr_stage_verify", "lsr_autotune", "lsr_get_tune",
                  "lsr_set_tune", "lsr_ransac_pair", "lsr_stage_ransac", "lsr_stage_gnc_noalloc",
                  "lsr_surfel_correct", "lsr_edge_info", "lsr_loop_solve", "lsr_loop_verify", "lsr_se3_retract",
                  "lsr_se3_retract_grad", "lsr_set_tune_cache"):
            getattr(L, f).restype = C.c_int
        _LIB = L
    return _LIB


def default_params(**kw) -> Params:
    p = Params()
    lib().lsr_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


class Context:
    """One lsr_ctx on one device (owns the library's scratch memory)."""

    def __init__(self, device: int = 0, workspace_cap: int = 0):
        h = C.c_void_p()
        rc = lib().lsr_create(C.byref(h), int(device), int(workspace_cap))
        if rc != 0:
            raise LsrError(f"lsr_create({device}) failed with {rc}")
        self.h = h
        self.device = device

    def check(self, rc):
        if rc != 0:
            raise LsrError(f"liblsr error {rc}: {lib().lsr_last_error(self.h).decode()}")

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.lsr_destroy(self.h)
            self.h = None


def get_context(device=None) -> Context:
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _CTX:
        _CTX[dev] = Context(dev)
    return _CTX[dev]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def _cloud(t: torch.Tensor, normals=True) -> Cloud:
    if not (t.is_cuda and t.dtype == torch.float32 and t.dim() == 2 and t.shape[0] in (3, 6)
            and (t.shape[1] <= 1 or t.stride(1) == 1)):
        raise LsrError("a cloud must be a CUDA float32 tensor of shape (6, N) or (3, N) with contiguous rows")
    if normals and t.shape[0] != 6:
        raise LsrError("this call needs input normals: shape (6, N)")
    n = t.shape[1]
    rows = [C.c_void_p(t[k].data_ptr() if n else 0) for k in range(t.shape[0])]
    rows += [C.c_void_p(0)] * (6 - len(rows))
    return Cloud(*rows, n)


RESULT_BYTES = C.sizeof(Result)


def _parse_results(buf: torch.Tensor, n: int):
    raw = buf.cpu().numpy().tobytes()
    out = []
    for k in range(n):
        r = Result.from_buffer_copy(raw[k * RESULT_BYTES:(k + 1) * RESULT_BYTES])
        d = {name: getattr(r, name) for name, _ in Result._fields_ if name != "T"}
        d["T"] = np.array(r.T[:]).reshape(4, 4)
        out.append(d)
    return out


def register_pair(P: torch.Tensor, Q: torch.Tensor, params: Params | None = None, ctx: Context | None = None,
                  out: torch.Tensor | None = None, sync: bool = True, trace: bool = False):
    """Register one pair.  Returns a dict (after a stream sync) or, with
    sync=False, the raw device result buffer.  trace=True runs the pair as a
    batch of one with its per-point trace (lsr_register_batch_trace) and
    returns (result, trace dict of numpy arrays)."""
    if trace:
        res, tr = register_batch(P, Q, [0, P.shape[1]], [0, Q.shape[1]], params, ctx=ctx, trace=True)
        return res[0], {k: v.cpu().numpy() for k, v in tr.items()}
    ctx = ctx or get_context(P.device.index)
    prm = params or default_params()
    cp, cq = _cloud(P), _cloud(Q)
    if out is None:
        out = torch.empty(RESULT_BYTES, dtype=torch.uint8, device=P.device)
    ctx.check(lib().lsr_register_pair(ctx.h, C.byref(cp), C.byref(cq), C.byref(prm), _ptr(out), _stream()))
    return _parse_results(out, 1)[0] if sync else out


def register_batch(P_all: torch.Tensor, Q_all: torch.Tensor, offP, offQ, params: Params | None = None,
                   ctx: Context | None = None, out: torch.Tensor | None = None, sync: bool = True,
                   trace: bool = False):
    """Register len(offP) - 1 pairs: pair b's P is columns offP[b]:offP[b+1] of P_all.
    trace=True (lsr_register_batch_trace) also returns a dict of per-point
    device tensors nnQ, nnP, mutual, consistent, desc_P, desc_Q, valid_P,
    valid_Q in the callers' point order."""
    ctx = ctx or get_context(P_all.device.index)
    prm = params or default_params()
    offP = np.ascontiguousarray(offP, np.int64)
    offQ = np.ascontiguousarray(offQ, np.int64)
    n = len(offP) - 1
    if len(offQ) != n + 1:
        raise LsrError("offP and offQ must have the same length")
    cp, cq = _cloud(P_all), _cloud(Q_all)
    if out is None:
        out = torch.empty(max(n, 1) * RESULT_BYTES, dtype=torch.uint8, device=P_all.device)
    if trace:
        dev = P_all.device
        nP, nQ = P_all.shape[1], Q_all.shape[1]
        tr = {"nnQ": torch.full((nP,), -2, dtype=torch.int32, device=dev),
              "nnP": torch.full((nQ,), -2, dtype=torch.int32, device=dev),
              "mutual": torch.zeros(nP, dtype=torch.uint8, device=dev),
              "consistent": torch.zeros(nP, dtype=torch.uint8, device=dev),
              "desc_P": torch.zeros((nP, 33), dtype=torch.float32, device=dev),
              "desc_Q": torch.zeros((nQ, 33), dtype=torch.float32, device=dev),
              "valid_P": torch.full((nP,), -1, dtype=torch.int32, device=dev),
              "valid_Q": torch.full((nQ,), -1, dtype=torch.int32, device=dev)}
        t = Trace(*[_ptr(tr[k]) for k, _ in Trace._fields_])
        ctx.check(lib().lsr_register_batch_trace(ctx.h, C.byref(cp), C.byref(cq), offP.ctypes.data_as(C.c_void_p),
                                                 offQ.ctypes.data_as(C.c_void_p), n, C.byref(prm), _ptr(out),
                                                 C.byref(t), _stream()))
        return (_parse_results(out, n) if sync else out), tr
    ctx.check(lib().lsr_register_batch(ctx.h, C.byref(cp), C.byref(cq), offP.ctypes.data_as(C.c_void_p),
                                       offQ.ctypes.data_as(C.c_void_p), n, C.byref(prm), _ptr(out), _stream()))
    return _parse_results(out, n) if sync else out


def _tune_dict(t: Tune) -> dict:
    return {"screen_shape": t.screen_shape, "consistency_shape": t.consistency_shape,
            "screen_ms": list(t.screen_ms[:t.n_screen_shapes]),
            "consistency_ms": list(t.consistency_ms[:t.n_consistency_shapes]), "from_cache": bool(t.from_cache)}


def autotune(P_all: torch.Tensor, Q_all: torch.Tensor, offP, offQ, params: Params | None = None, reps: int = 2,
             ctx: Context | None = None, cache: str | None = None) -> dict:
    """Time every launch-shape variant on this batch and keep the fastest (lsr_autotune).
    cache: a JSON tune-cache file (lsr_set_tune_cache) consulted and updated."""
    ctx = ctx or get_context(P_all.device.index)
    if cache is not None:
        ctx.check(lib().lsr_set_tune_cache(ctx.h, cache.encode() if cache else None))
    prm = params or default_params()
    offP = np.ascontiguousarray(offP, np.int64)
    offQ = np.ascontiguousarray(offQ, np.int64)
    n = len(offP) - 1
    if len(offQ) != n + 1:
        raise LsrError("offP and offQ must have the same length")
    cp, cq = _cloud(P_all), _cloud(Q_all)
    t = Tune()
    ctx.check(lib().lsr_autotune(ctx.h, C.byref(cp), C.byref(cq), offP.ctypes.data_as(C.c_void_p),
                                 offQ.ctypes.data_as(C.c_void_p), n, C.byref(prm), reps, C.byref(t), _stream()))
    return _tune_dict(t)


def get_tune(ctx: Context | None = None) -> dict:
    ctx = ctx or get_context()
    t = Tune()
    ctx.check(lib().lsr_get_tune(ctx.h, C.byref(t)))
    return {"screen_shape": t.screen_shape, "consistency_shape": t.consistency_shape,
            "n_screen_shapes": t.n_screen_shapes, "n_consistency_shapes": t.n_consistency_shapes}


def set_tune(screen_shape: int, consistency_shape: int, ctx: Context | None = None):
    ctx = ctx or get_context()
    t = Tune()
    t.screen_shape, t.consistency_shape = screen_shape, consistency_shape
    ctx.check(lib().lsr_set_tune(ctx.h, C.byref(t)))


def voxel_downsample(cloud: torch.Tensor, voxel: float, ctx: Context | None = None):
    """(6, M) float32 CUDA tensor of voxel means (ordered by voxel index)."""
    ctx = ctx or get_context(cloud.device.index)
    n = cloud.shape[1]
    out = torch.empty((6, max(n, 1)), dtype=torch.float32, device=cloud.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=cloud.device)
    c = _cloud(cloud)
    ptrs = (C.c_void_p * 6)(*[out[k].data_ptr() for k in range(6)])
    ctx.check(lib().lsr_voxel_downsample(ctx.h, C.byref(c), C.c_float(voxel), ptrs, _ptr(cnt), _stream()))
    m = int(cnt.cpu()[0])
    if m < 0:
        raise LsrError("voxel downsample: non-finite coordinate or voxel index out of range")
    return out[:, :m]


def surfel_correct(S: torch.Tensor, t0: torch.Tensor, tu: torch.Tensor, T_old, T_new, t_kf, camera: dict,
                   ctx: Context | None = None, sync: bool = True):
    """Dense surface correction of a surfel map (see lsr_surfel_correct).

    S: (6, n) float32 CUDA surfels; t0, tu: (n,) int32 CUDA windows; T_old,
    T_new: (K, 4, 4) float64 keyframe poses and t_kf (K,) int32 time stamps
    (host arrays); camera: fx fy cx cy width height z_min z_max.  Returns
    (kept (6, m) view, new_index (n,), k_obs (n,), n_kept tensor); with sync
    the kept view is trimmed to m, else it has n columns and n_kept is a
    device tensor to read later."""
    ctx = ctx or get_context(S.device.index)
    n = S.shape[1]
    c = _cloud(S)
    To = np.ascontiguousarray(T_old, np.float64).reshape(-1, 16)
    Tn = np.ascontiguousarray(T_new, np.float64).reshape(-1, 16)
    tk = np.ascontiguousarray(t_kf, np.int32)
    out = torch.empty((6, max(n, 1)), dtype=torch.float32, device=S.device)
    new_index = torch.empty(max(n, 1), dtype=torch.int32, device=S.device)
    k_obs = torch.empty(max(n, 1), dtype=torch.int32, device=S.device)
    cnt = torch.zeros(1, dtype=torch.int64, device=S.device)
    src = (C.c_void_p * 6)(c.x, c.y, c.z, c.nx, c.ny, c.nz)
    dst = (C.c_void_p * 6)(*[out[k].data_ptr() for k in range(6)])
    cam = Camera(**camera)
    ctx.check(lib().lsr_surfel_correct(ctx.h, src, _ptr(t0.contiguous()), _ptr(tu.contiguous()), n,
                                       To.ctypes.data_as(C.c_void_p), Tn.ctypes.data_as(C.c_void_p),
                                       tk.ctypes.data_as(C.c_void_p), len(tk), C.byref(cam), dst, _ptr(new_index),
                                       _ptr(k_obs), _ptr(cnt), _stream()))
    if not sync:
        return out, new_index[:n], k_obs[:n], cnt
    m = int(cnt.cpu()[0])
    return out[:, :m], new_index[:n], k_obs[:n], m


def loop_params(**kw) -> LoopParams:
    """lsr_loop_params with the paper's defaults (lambda 1000, tau 0.2 m,
    l_min 0.25, eps 0.05 m); keyword 'lambda' sets lambda_."""
    p = LoopParams()
    lib().lsr_default_loop_params(C.byref(p))
    for k, v in kw.items():
        k = "lambda_" if k == "lambda" else k
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _edge_array(E):
    arr = (Edge * max(len(E), 1))()
    for k, (i, j, T) in enumerate(E):
        arr[k].i, arr[k].j = int(i), int(j)
        arr[k].T[:] = [float(v) for v in np.asarray(T, np.float64).reshape(16)]
    return arr


def _cloud_array(frags):
    arr = (Cloud * len(frags))()
    for k, f in enumerate(frags):
        arr[k] = _cloud(f, normals=False)
    return arr


def _parse_loop(buf: torch.Tensor, n: int):
    raw = buf.cpu().numpy().tobytes()
    sz = C.sizeof(LoopResult)
    out = []
    for k in range(n):
        r = LoopResult.from_buffer_copy(raw[k * sz:(k + 1) * sz])
        out.append({name: getattr(r, name) for name, _ in LoopResult._fields_})
    return out


def edge_info(frags, edges, eps=0.05, ctx=None):
    """Information matrices (m, 6, 6) float64 and correspondence counts (m,)
    int64 (CUDA tensors) of edges (i, j, T) between fragments (CUDA (3|6, n))."""
    ctx = ctx or get_context(frags[0].device.index)
    m = len(edges)
    info = torch.zeros((max(m, 1), 6, 6), dtype=torch.float64, device=frags[0].device)
    cnt = torch.zeros(max(m, 1), dtype=torch.int64, device=frags[0].device)
    ctx.check(lib().lsr_edge_info(ctx.h, _cloud_array(frags), len(frags), _edge_array(edges), m, C.c_float(eps),
                                  _ptr(info), _ptr(cnt), _stream()))
    return info[:m], cnt[:m]


def loop_solve(T_init, odo, info_odo, loops, info_loop, count_loop, params=None, ctx=None, poses=True):
    """Line-process pose graph per loop candidate (see lsr_loop_solve).
    Returns (list of result dicts, optimised poses (C, n, 4, 4) CUDA tensor or None)."""
    ctx = ctx or get_context(info_odo.device.index)
    T_init = np.ascontiguousarray(T_init, np.float64).reshape(-1, 16)
    n, c = T_init.shape[0], len(loops)
    dev = info_odo.device
    res = torch.zeros(max(c, 1) * C.sizeof(LoopResult), dtype=torch.uint8, device=dev)
    T_out = torch.zeros((max(c, 1), n, 4, 4), dtype=torch.float64, device=dev) if poses else None
    ctx.check(lib().lsr_loop_solve(ctx.h, n, T_init.ctypes.data_as(C.c_void_p), _edge_array(odo),
                                   _ptr(info_odo.contiguous()), _edge_array(loops), c,
                                   _ptr(info_loop.contiguous()), _ptr(count_loop.contiguous()),
                                   C.byref(params or loop_params()), _ptr(T_out), _ptr(res), _stream()))
    return _parse_loop(res, c), (T_out[:c] if poses else None)


def loop_verify(frags, T_init, odo, loops, params=None, ctx=None, poses=True, sync=True):
    """Edge information of the chain and its loop candidates, then the pose
    graph per candidate (see lsr_loop_verify)."""
    ctx = ctx or get_context(frags[0].device.index)
    T_init = np.ascontiguousarray(T_init, np.float64).reshape(-1, 16)
    n, c = T_init.shape[0], len(loops)
    dev = frags[0].device
    res = torch.zeros(max(c, 1) * C.sizeof(LoopResult), dtype=torch.uint8, device=dev)
    T_out = torch.zeros((max(c, 1), n, 4, 4), dtype=torch.float64, device=dev) if poses else None
    ctx.check(lib().lsr_loop_verify(ctx.h, _cloud_array(frags), len(frags), T_init.ctypes.data_as(C.c_void_p),
                                    _edge_array(odo), _edge_array(loops), c, C.byref(params or loop_params()),
                                    _ptr(T_out), _ptr(res), _stream()))
    if not sync:
        return res, T_out
    return _parse_loop(res, c), (T_out[:c] if poses else None)


def se3_retract(xi: torch.Tensor, T: torch.Tensor, ctx=None) -> torch.Tensor:
    """[Rod(w) | v] T per pose (xi (n, 6) and T (n, 4, 4) float64 CUDA)."""
    ctx = ctx or get_context(T.device.index)
    xi, T = xi.contiguous(), T.contiguous()
    out = torch.empty_like(T)
    ctx.check(lib().lsr_se3_retract(ctx.h, T.shape[0], _ptr(xi), _ptr(T), _ptr(out), _stream()))
    return out


def se3_retract_grad(xi: torch.Tensor, g_left: torch.Tensor, ctx=None) -> torch.Tensor:
    """dE/dxi of E(Exp(xi) T) from the left-perturbation gradient at Exp(xi) T."""
    ctx = ctx or get_context(xi.device.index)
    xi, g_left = xi.contiguous(), g_left.contiguous()
    out = torch.empty_like(g_left)
    ctx.check(lib().lsr_se3_retract_grad(ctx.h, xi.shape[0], _ptr(xi), _ptr(g_left), _ptr(out), _stream()))
    return out


def _xyz_ptrs(t):
    arr = (C.c_void_p * 3)(*[t[k].data_ptr() for k in range(3)])
    return arr


def align_loss(P_xyz, Q_xyz, corr, coff, T, mu, ctx=None):
    """E[k] for each problem k (see lsr_align_loss).  T: (n,4,4) float64, mu: (n,) float64."""
    ctx = ctx or get_context(P_xyz.device.index)
    coff = np.ascontiguousarray(coff, np.int64)
    n = len(coff) - 1
    E = torch.empty(n, dtype=torch.float64, device=P_xyz.device)
    T = T.contiguous()
    mu = mu.contiguous()
    ctx.check(lib().lsr_align_loss(ctx.h, _xyz_ptrs(P_xyz), P_xyz.shape[1], _xyz_ptrs(Q_xyz), Q_xyz.shape[1],
                                   _ptr(corr),
                                   coff.ctypes.data_as(C.c_void_p), n, _ptr(T), _ptr(mu), _ptr(E), _stream()))
    return E


def align_loss_backward(P_xyz, Q_xyz, corr, coff, T, mu, dE, ctx=None):
    """(dP (3,NP) f32, dQ (3,NQ) f32, dxi (n,6) f64) scaled by dE (n,)."""
    ctx = ctx or get_context(P_xyz.device.index)
    coff = np.ascontiguousarray(coff, np.int64)
    n = len(coff) - 1
    dP = torch.zeros((3, P_xyz.shape[1]), dtype=torch.float32, device=P_xyz.device)
    dQ = torch.zeros((3, Q_xyz.shape[1]), dtype=torch.float32, device=P_xyz.device)
    dxi = torch.empty((n, 6), dtype=torch.float64, device=P_xyz.device)
    ctx.check(lib().lsr_align_loss_backward(ctx.h, _xyz_ptrs(P_xyz), P_xyz.shape[1], _xyz_ptrs(Q_xyz),
                                            Q_xyz.shape[1], _ptr(corr),
                                            coff.ctypes.data_as(C.c_void_p), n, _ptr(T.contiguous()),
                                            _ptr(mu.contiguous()), _ptr(dE.contiguous()), _xyz_ptrs(dP),
                                            _xyz_ptrs(dQ), _ptr(dxi), _stream()))
    return dP, dQ, dxi


def set_timing(enable: bool, ctx: Context | None = None):
    ctx = ctx or get_context()
    ctx.check(lib().lsr_set_timing(ctx.h, int(bool(enable))))


def get_timing(ctx: Context | None = None):
    """[(step name, ms), ...] recorded since the last call (syncs the device)."""
    ctx = ctx or get_context()
    mx = 4096
    names = C.create_string_buffer(32 * mx)
    ms = (C.c_double * mx)()
    n = C.c_int()
    ctx.check(lib().lsr_get_timing(ctx.h, mx, names, ms, C.byref(n)))
    raw = names.raw
    return [(raw[32 * k:32 * k + 32].split(b"\0")[0].decode(), ms[k]) for k in range(n.value)]


# ---- stage entry points --------------------------------------------------------------------

def stage_normals(cloud, r_normal, ctx=None):
    ctx = ctx or get_context(cloud.device.index)
    out = torch.empty((cloud.shape[1], 3), dtype=torch.float64, device=cloud.device)
    c = _cloud(cloud)
    ctx.check(lib().lsr_stage_normals(ctx.h, C.byref(c), C.c_float(r_normal), _ptr(out), _stream()))
    return out


def stage_fpfh(xyz, nrm, r_feature, ctx=None):
    ctx = ctx or get_context(xyz.device.index)
    n = xyz.shape[1]
    F = torch.empty((n, 33), dtype=torch.float32, device=xyz.device)
    v = torch.empty(n, dtype=torch.int32, device=xyz.device)
    c = _cloud(xyz[:3].contiguous() if xyz.shape[0] == 6 else xyz, normals=False)
    ctx.check(lib().lsr_stage_fpfh(ctx.h, C.byref(c), _ptr(nrm.contiguous()), C.c_float(r_feature), _ptr(F),
                                   _ptr(v), _stream()))
    return F, v


def stage_spfh(xyz, nrm, r_feature, ctx=None):
    ctx = ctx or get_context(xyz.device.index)
    n = xyz.shape[1]
    S = torch.empty((n, 33), dtype=torch.float32, device=xyz.device)
    k = torch.empty(n, dtype=torch.int32, device=xyz.device)
    c = _cloud(xyz[:3].contiguous() if xyz.shape[0] == 6 else xyz, normals=False)
    ctx.check(lib().lsr_stage_spfh(ctx.h, C.byref(c), _ptr(nrm.contiguous()), C.c_float(r_feature), _ptr(S),
                                   _ptr(k), _stream()))
    return S, k


def stage_match(F, vF, G, vG, precision=FP32, ctx=None):
    ctx = ctx or get_context(F.device.index)
    nP, nQ = F.shape[0], G.shape[0]
    dev = F.device
    nnQ = torch.empty(nP, dtype=torch.int32, device=dev)
    dQ = torch.empty(nP, dtype=torch.float32, device=dev)
    nnP = torch.empty(nQ, dtype=torch.int32, device=dev)
    dP = torch.empty(nQ, dtype=torch.float32, device=dev)
    fb = torch.zeros(1, dtype=torch.int64, device=dev)
    ctx.check(lib().lsr_stage_match(ctx.h, _ptr(F.contiguous()), _ptr(vF.contiguous()), nP, _ptr(G.contiguous()),
                                    _ptr(vG.contiguous()), nQ, int(precision), _ptr(nnQ), _ptr(dQ), _ptr(nnP),
                                    _ptr(dP), _ptr(fb), _stream()))
    return nnQ, dQ, nnP, dP, fb


def stage_consistency(P, Q, nnQ, mutual, n_trials, tau, seed, ctx=None):
    ctx = ctx or get_context(P.device.index)
    flag = torch.empty(P.shape[1], dtype=torch.uint8, device=P.device)
    passed = torch.zeros(1, dtype=torch.int64, device=P.device)
    cp, cq = _cloud(P, normals=False), _cloud(Q, normals=False)
    ctx.check(lib().lsr_stage_consistency(ctx.h, C.byref(cp), C.byref(cq), _ptr(nnQ.contiguous()),
                                          _ptr(mutual.contiguous()), int(n_trials), C.c_float(tau),
                                          C.c_uint64(seed), _ptr(flag), _ptr(passed), _stream()))
    return flag, passed


def stage_gnc(p, q, params=None, ctx=None):
    """p, q: (m,3) float64 CUDA tensors -> (T (4,4), info {status, iters, mu_final, energy})."""
    ctx = ctx or get_context(p.device.index)
    prm = params or default_params()
    T = torch.empty(16, dtype=torch.float64, device=p.device)
    info = torch.empty(4, dtype=torch.float64, device=p.device)
    ctx.check(lib().lsr_stage_gnc(ctx.h, _ptr(p.contiguous()), _ptr(q.contiguous()), p.shape[0], C.byref(prm),
                                  _ptr(T), _ptr(info), _stream()))
    return T.view(4, 4), info


def stage_gnc_noalloc(p, q, T, info, params=None, ctx=None):
    """lsr_stage_gnc_noalloc into caller-provided T (16 float64) and info (4
    float64) CUDA tensors: p, q (m,3) float64 CUDA tensors."""
    ctx = ctx or get_context(p.device.index)
    prm = params or default_params()
    ctx.check(lib().lsr_stage_gnc_noalloc(ctx.h, _ptr(p), _ptr(q), p.shape[0], C.byref(prm), _ptr(T), _ptr(info),
                                          _stream()))


def stage_verify(P, nrmP, Q, nrmQ, T, delta, normal_check=0, normal_cos=0.8660254, ctx=None):
    ctx = ctx or get_context(P.device.index)
    info = torch.empty(3, dtype=torch.float64, device=P.device)
    cp, cq = _cloud(P, normals=False), _cloud(Q, normals=False)
    ctx.check(lib().lsr_stage_verify(ctx.h, C.byref(cp), _ptr(nrmP), C.byref(cq), _ptr(nrmQ),
                                     _ptr(T.contiguous()), C.c_float(delta), int(normal_check),
                                     C.c_float(normal_cos), _ptr(info), _stream()))
    return info


RANSAC_RESULT_BYTES = C.sizeof(RansacResult)


def _parse_ransac(buf: torch.Tensor) -> dict:
    r = RansacResult.from_buffer_copy(buf.cpu().numpy().tobytes()[:RANSAC_RESULT_BYTES])
    d = {name: getattr(r, name) for name, _ in RansacResult._fields_ if name not in ("T", "pad")}
    d["T"] = np.array(r.T[:]).reshape(4, 4)
    return d


def ransac_pair(P: torch.Tensor, Q: torch.Tensor, params: Params | None = None, n_hyp: int = 0,
                ctx: Context | None = None, out: torch.Tensor | None = None, sync: bool = True):
    """Algorithm 1 on one pair (lsr_ransac_pair): descriptors, the one-way
    descriptor neighbour cache, RANSAC consensus.  Returns a dict (or the raw
    device result when sync=False)."""
    ctx = ctx or get_context(P.device.index)
    prm = params or default_params()
    cp, cq = _cloud(P), _cloud(Q)
    if out is None:
        out = torch.empty(RANSAC_RESULT_BYTES, dtype=torch.uint8, device=P.device)
    ctx.check(lib().lsr_ransac_pair(ctx.h, C.byref(cp), C.byref(cq), C.byref(prm), int(n_hyp), _ptr(out),
                                    _stream()))
    return _parse_ransac(out) if sync else out


def stage_ransac(P, Q, nnQ, params=None, n_hyp=0, nrmP=None, nrmQ=None, trace_capacity=0, ctx=None):
    """RANSAC consensus on injected inputs (lsr_stage_ransac).  P, Q: (3|6, N)
    float32 CUDA tensors; nnQ: int32 CUDA tensor (P's descriptor neighbours in
    Q, -1 none); nrmP/nrmQ: (N,3) float64 CUDA tensors when the normal check is
    on.  Returns (result dict, trace dict of numpy arrays or None)."""
    ctx = ctx or get_context(P.device.index)
    prm = params or default_params()
    cp, cq = _cloud(P, normals=False), _cloud(Q, normals=False)
    out = torch.empty(RANSAC_RESULT_BYTES, dtype=torch.uint8, device=P.device)
    tr = None
    trs = None
    if trace_capacity > 0:
        dev, c = P.device, int(trace_capacity)
        tr = {"hyp": torch.full((c,), -1, dtype=torch.int64, device=dev),
              "members": torch.full((c, 4), -1, dtype=torch.int32, device=dev),
              "n_inliers": torch.full((c,), -3, dtype=torch.int32, device=dev),
              "sum_d2": torch.zeros(c, dtype=torch.float64, device=dev),
              "T": torch.zeros((c, 16), dtype=torch.float64, device=dev)}
        trs = RansacTrace(c, *[_ptr(tr[k]) for k in ("hyp", "members", "n_inliers", "sum_d2", "T")])
    ctx.check(lib().lsr_stage_ransac(ctx.h, C.byref(cp), _ptr(nrmP), C.byref(cq), _ptr(nrmQ),
                                     _ptr(nnQ.contiguous()), int(n_hyp), C.byref(prm), _ptr(out),
                                     C.byref(trs) if trs is not None else None, _stream()))
    res = _parse_ransac(out)
    if tr is not None:
        n = min(res["n_survivors"], trace_capacity)
        tr = {k: v[:n].cpu().numpy() for k, v in tr.items()}
    return res, tr
