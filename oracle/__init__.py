"""Python view of the CPU FP64 oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  It wraps ``liboracle.so`` (plain C, see oracle.c) with numpy
arrays; it shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ACCEPTED, REJECTED, DEGENERATE = 1, 2, 3


class Params(C.Structure):
    _fields_ = [
        ("r_normal", C.c_float), ("r_feature", C.c_float), ("max_corr", C.c_float), ("tau", C.c_float),
        ("n_trials", C.c_int64), ("gnc_div", C.c_double), ("gnc_every", C.c_int32),
        ("gnc_max_iter", C.c_int32), ("polish_iter", C.c_int32), ("min_inlier_ratio", C.c_float),
        ("min_consistent", C.c_int64), ("normal_check", C.c_int32), ("normal_cos", C.c_float),
        ("seed", C.c_uint64),
    ]


class Result(C.Structure):
    _fields_ = [
        ("T", C.c_double * 16), ("energy", C.c_double), ("mu_final", C.c_double),
        ("inlier_ratio", C.c_double), ("fitness", C.c_double),
        ("n_valid_P", C.c_int64), ("n_valid_Q", C.c_int64), ("n_recip", C.c_int64),
        ("n_consistent", C.c_int64), ("n_inliers", C.c_int64),
        ("status", C.c_int32), ("iters", C.c_int32),
    ]


class Camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("width", C.c_int32), ("height", C.c_int32), ("z_min", C.c_double), ("z_max", C.c_double)]


class Edge(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("T", C.c_double * 16)]


class LoopParams(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("tau", C.c_double), ("l_min", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int32)]


class LoopResult(C.Structure):
    _fields_ = [("l", C.c_double), ("f_loop", C.c_double), ("energy", C.c_double), ("mu", C.c_double),
                ("status", C.c_int32), ("iters", C.c_int32)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from .build import build
            build()
        _LIB = C.CDLL(path)
        _LIB.orc_splitmix64.restype = C.c_uint64
        _LIB.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        for f in ("orc_neighbors_grid", "orc_neighbors_brute", "orc_voxel", "orc_consistency"):
            getattr(_LIB, f).restype = C.c_int64
        _LIB.orc_gnc.restype = C.c_int32
        _LIB.orc_rigid_fit.restype = C.c_int32
        _LIB.orc_ransac.restype = C.c_int32
        _LIB.orc_register_pair.restype = C.c_int32
        _LIB.orc_align_loss.restype = C.c_double
        _LIB.orc_surfel_correct.restype = C.c_int64
        _LIB.orc_loop_solve.restype = C.c_int32
    return _LIB


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def default_params(**kw) -> Params:
    p = Params()
    lib().orc_default_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def neighbors(xyz, r, brute=False):
    """CSR radius neighbourhoods (offsets, idx) of an (3, n) float32 cloud."""
    xyz = _f32(xyz)
    n = xyz.shape[1]
    off = np.zeros(n + 1, np.int64)
    f = lib().orc_neighbors_brute if brute else lib().orc_neighbors_grid
    args = [_p(xyz[0]), _p(xyz[1]), _p(xyz[2]), C.c_int64(n), C.c_float(r)]
    cap = 0
    idx = np.zeros(1, np.int64)
    tot = f(*args, _p(off), _p(idx), C.c_int64(cap))
    if tot < 0:
        cap = int(off[-1])
        idx = np.zeros(max(cap, 1), np.int64)
        tot = f(*args, _p(off), _p(idx), C.c_int64(cap))
    return off, idx[:tot]


def voxel(cloud, v):
    c = _f32(cloud)
    n = c.shape[1]
    out = np.zeros((6, max(n, 1)), np.float32)
    m = lib().orc_voxel(*[_p(c[k]) for k in range(6)], C.c_int64(n), C.c_float(v),
                        *[_p(out[k]) for k in range(6)])
    return np.ascontiguousarray(out[:, :m])


def normals(cloud, r_n):
    """(n,3) float64 normals, eigen gap, orientation dot, neighbour count."""
    c = _f32(cloud)
    n = c.shape[1]
    nrm = np.zeros((n, 3)); gap = np.zeros(n); ori = np.zeros(n); cnt = np.zeros(n, np.int32)
    lib().orc_normals(*[_p(c[k]) for k in range(6)], C.c_int64(n), C.c_float(r_n),
                      _p(nrm), _p(gap), _p(ori), _p(cnt))
    return nrm, gap, ori, cnt


def spfh(xyz, nrm, r_f):
    xyz = _f32(xyz); nrm = _f64(nrm)
    n = xyz.shape[1]
    S = np.zeros((n, 33)); k = np.zeros(n, np.int32); kp = np.zeros(n, np.int32); mg = np.zeros(n)
    lib().orc_spfh(_p(xyz[0]), _p(xyz[1]), _p(xyz[2]), _p(nrm), C.c_int64(n), C.c_float(r_f),
                   _p(S), _p(k), _p(kp), _p(mg))
    return S, k, kp, mg


def fpfh(xyz, nrm, r_f):
    """(n,33) FPFH, valid flags, per-point SPFH margin and descriptor margin."""
    xyz = _f32(xyz); nrm = _f64(nrm)
    n = xyz.shape[1]
    F = np.zeros((n, 33)); v = np.zeros(n, np.int32); sm = np.zeros(n); dm = np.zeros(n)
    lib().orc_fpfh(_p(xyz[0]), _p(xyz[1]), _p(xyz[2]), _p(nrm), C.c_int64(n), C.c_float(r_f),
                   _p(F), _p(v), _p(sm), _p(dm))
    return F, v, sm, dm


def match(F, vF, G, vG):
    """Both-direction nearest neighbours with second best (dict of arrays)."""
    F = _f64(F); G = _f64(G)
    vF = np.ascontiguousarray(vF, np.int32); vG = np.ascontiguousarray(vG, np.int32)
    nP, nQ = len(F), len(G)
    o = {k: np.zeros(nP, np.int32) for k in ("nnQ", "nn2Q")}
    o.update({k: np.zeros(nP) for k in ("d1Q", "d2Q")})
    o.update({k: np.zeros(nQ, np.int32) for k in ("nnP", "nn2P")})
    o.update({k: np.zeros(nQ) for k in ("d1P", "d2P")})
    lib().orc_match(_p(F), _p(vF), C.c_int64(nP), _p(G), _p(vG), C.c_int64(nQ),
                    _p(o["nnQ"]), _p(o["d1Q"]), _p(o["nn2Q"]), _p(o["d2Q"]),
                    _p(o["nnP"]), _p(o["d1P"]), _p(o["nn2P"]), _p(o["d2P"]))
    return o


def tie_flags(F, G, m, eps=1e-4):
    F = _f64(F); G = _f64(G)
    tP = np.zeros(len(F), np.uint8); tQ = np.zeros(len(G), np.uint8)
    lib().orc_tie_flags(_p(F), C.c_int64(len(F)), _p(G), C.c_int64(len(G)),
                        _p(m["nnQ"]), _p(m["d1Q"]), _p(m["nn2Q"]), _p(m["d2Q"]),
                        _p(m["nnP"]), _p(m["d1P"]), _p(m["nn2P"]), _p(m["d2P"]),
                        C.c_double(eps), _p(tP), _p(tQ))
    return tP.astype(bool), tQ.astype(bool)


def mutual(nnQ, nnP):
    nnQ = np.asarray(nnQ); nnP = np.asarray(nnP)
    ok = nnQ >= 0
    m = np.zeros(len(nnQ), bool)
    m[ok] = nnP[nnQ[ok]] == np.nonzero(ok)[0]
    return m


def splitmix64(seed, n):
    return int(lib().orc_splitmix64(C.c_uint64(seed), C.c_uint64(n)))


def consistency(P_xyz, Q_xyz, nnQ, mut, n_trials, tau, seed):
    P = _f32(P_xyz); Q = _f32(Q_xyz)
    nnQ = np.ascontiguousarray(nnQ, np.int32)
    mu = np.ascontiguousarray(mut, np.uint8)
    flag = np.zeros(P.shape[1], np.uint8)
    passed = lib().orc_consistency(_p(P[0]), _p(P[1]), _p(P[2]), C.c_int64(P.shape[1]),
                                   _p(Q[0]), _p(Q[1]), _p(Q[2]), _p(nnQ), _p(mu),
                                   C.c_int64(n_trials), C.c_float(tau), C.c_uint64(seed), _p(flag))
    return flag.astype(bool), int(passed)


def default_trials(nP):
    return min(4_000_000, 100 * int(nP))


def gnc(p, q, params=None):
    """p, q: (m,3) float64 correspondences -> (status, T, mu_final, energy, iters)."""
    p = _f64(p); q = _f64(q)
    prm = params or default_params()
    T = np.zeros(16); mu = C.c_double(); E = C.c_double(); it = C.c_int32()
    st = lib().orc_gnc(_p(p), _p(q), C.c_int64(len(p)), C.byref(prm), _p(T),
                       C.byref(mu), C.byref(E), C.byref(it))
    return int(st), T.reshape(4, 4), mu.value, E.value, it.value


def verify(P, nrmP, Q, nrmQ, T, delta, normal_check=0, normal_cos=0.8660254):
    P = _f32(P); Q = _f32(Q)
    nrmP = _f64(nrmP) if nrmP is not None else np.zeros((P.shape[1], 3))
    nrmQ = _f64(nrmQ) if nrmQ is not None else np.zeros((Q.shape[1], 3))
    T = _f64(T).reshape(16)
    ni = C.c_int64(); ratio = C.c_double(); fit = C.c_double()
    lib().orc_verify(_p(P[0]), _p(P[1]), _p(P[2]), _p(nrmP), C.c_int64(P.shape[1]),
                     _p(Q[0]), _p(Q[1]), _p(Q[2]), _p(nrmQ), C.c_int64(Q.shape[1]),
                     _p(T), C.c_float(delta), C.c_int32(normal_check), C.c_float(normal_cos),
                     C.byref(ni), C.byref(ratio), C.byref(fit))
    return ni.value, ratio.value, fit.value


class RansacInfo(C.Structure):
    _fields_ = [("n_survivors", C.c_int64), ("n_fitted", C.c_int64), ("best", C.c_int64), ("second", C.c_int64),
                ("n_inliers", C.c_int64), ("second_inliers", C.c_int64), ("ratio", C.c_double),
                ("fitness", C.c_double), ("sum_d2", C.c_double), ("second_sum_d2", C.c_double)]


def rigid_fit(p, q):
    """Least-squares rigid transform of (m,3) pairs (q ~ R p + t): (ok, T 4x4)."""
    p = _f64(p); q = _f64(q)
    T = np.zeros(16)
    ok = lib().orc_rigid_fit(_p(p), _p(q), C.c_int64(len(p)), _p(T))
    return bool(ok), T.reshape(4, 4)


def ransac_hypotheses(P, Q, nnQ, n_hyp, tau=0.9, seed=0x1801015720):
    """Hypotheses of the RANSAC consensus and their polygon pre-rejection:
    (ok bool[n_hyp], members int64[n_hyp, 4]; rows of survivors only)."""
    P = _f32(P); Q = _f32(Q)
    nnQ = np.ascontiguousarray(nnQ, np.int32)
    ok = np.zeros(n_hyp, np.uint8)
    mem = np.full((n_hyp, 4), -1, np.int64)
    lib().orc_ransac_hypotheses(_p(P[0]), _p(P[1]), _p(P[2]), C.c_int64(P.shape[1]), _p(Q[0]), _p(Q[1]),
                                _p(Q[2]), _p(nnQ), C.c_int64(n_hyp), C.c_float(tau), C.c_uint64(seed),
                                _p(ok), _p(mem))
    return ok.astype(bool), mem


def ransac(P, nrmP, Q, nrmQ, nnQ, n_hyp, tau=0.9, seed=0x1801015720, delta=0.015, normal_check=1,
           normal_cos=0.8660254, min_ratio=0.25):
    """RANSAC consensus (Algorithm 1) on the one-directional cache nnQ:
    (status, T 4x4, info dict)."""
    P = _f32(P); Q = _f32(Q)
    nrmP = _f64(nrmP) if nrmP is not None else np.zeros((P.shape[1], 3))
    nrmQ = _f64(nrmQ) if nrmQ is not None else np.zeros((Q.shape[1], 3))
    nnQ = np.ascontiguousarray(nnQ, np.int32)
    T = np.zeros(16)
    info = RansacInfo()
    st = lib().orc_ransac(_p(P[0]), _p(P[1]), _p(P[2]), _p(nrmP), C.c_int64(P.shape[1]),
                          _p(Q[0]), _p(Q[1]), _p(Q[2]), _p(nrmQ), C.c_int64(Q.shape[1]),
                          _p(nnQ), C.c_int64(n_hyp), C.c_float(tau), C.c_uint64(seed), C.c_float(delta),
                          C.c_int32(normal_check), C.c_float(normal_cos), C.c_float(min_ratio), _p(T),
                          C.byref(info))
    return int(st), T.reshape(4, 4), {k: getattr(info, k) for k, _ in RansacInfo._fields_}


def align_loss(p, q, T, mu, grad=True):
    p = _f64(p); q = _f64(q); T = _f64(T).reshape(16)
    m = len(p)
    dp = np.zeros((m, 3)) if grad else None
    dq = np.zeros((m, 3)) if grad else None
    dxi = np.zeros(6) if grad else None
    E = lib().orc_align_loss(_p(p), _p(q), C.c_int64(m), _p(T), C.c_double(mu), _p(dp), _p(dq), _p(dxi))
    return (E, dp, dq, dxi) if grad else E


def register_pair(P, Q, params=None):
    """Whole pipeline.  Returns (Result, nnQ, consistent flags)."""
    P = _f32(P); Q = _f32(Q)
    prm = params or default_params()
    out = Result()
    nnQ = np.zeros(P.shape[1], np.int32)
    cons = np.zeros(P.shape[1], np.uint8)
    Pp = (C.c_void_p * 6)(*[P[k].ctypes.data for k in range(6)])
    Qp = (C.c_void_p * 6)(*[Q[k].ctypes.data for k in range(6)])
    lib().orc_register_pair(Pp, C.c_int64(P.shape[1]), Qp, C.c_int64(Q.shape[1]), C.byref(prm),
                            C.byref(out), _p(nnQ), _p(cons))
    return out, nnQ, cons.astype(bool)


def result_dict(r: Result) -> dict:
    d = {k: getattr(r, k) for k, _ in Result._fields_ if k != "T"}
    d["T"] = np.array(r.T[:]).reshape(4, 4)
    return d


def surfel_correct(S, t0, tu, T_old, T_new, t_kf, cam):
    """Dense surface correction of Sec. VI, eq. 7 (see surfel.c).

    S: (6, n) float32 surfels (x y z nx ny nz); t0, tu: (n,) int32 window;
    T_old, T_new: (K, 4, 4) camera-to-world poses; t_kf: (K,) int32;
    cam: dict of fx fy cx cy width height z_min z_max.
    Returns (kept (6, m) float32, new_index (n,), k_obs (n,))."""
    S = _f32(S)
    n = S.shape[1]
    t0 = np.ascontiguousarray(t0, np.int32); tu = np.ascontiguousarray(tu, np.int32)
    To = _f64(T_old).reshape(-1, 16); Tn = _f64(T_new).reshape(-1, 16)
    tk = np.ascontiguousarray(t_kf, np.int32)
    out = np.zeros((6, n), np.float32)
    idx = np.zeros(n, np.int32); k = np.zeros(n, np.int32)
    cm = Camera(**cam)
    m = lib().orc_surfel_correct(*[_p(S[r]) for r in range(6)], _p(t0), _p(tu), C.c_int64(n), _p(To), _p(Tn),
                                 _p(tk), C.c_int32(len(tk)), C.byref(cm), *[_p(out[r]) for r in range(6)],
                                 _p(idx), _p(k))
    return out[:, :m].copy(), idx, k


def loop_params(**kw) -> LoopParams:
    """Loop-verification parameters: the paper's lambda = 1000, tau = 0.2 m,
    l < 0.25 rejects (Sec. V); tol 1e-12, at most 100 iterations."""
    p = LoopParams(lambda_=1000.0, tau=0.2, l_min=0.25, tol=1e-12, max_iter=100)
    for k, v in kw.items():
        setattr(p, "lambda_" if k == "lambda" else k, v)
    return p


def _edges(E):
    arr = (Edge * max(len(E), 1))()
    for k, (i, j, T) in enumerate(E):
        arr[k].i, arr[k].j = int(i), int(j)
        arr[k].T[:] = [float(x) for x in np.asarray(T, np.float64).reshape(16)]
    return arr


def edge_info(Pi, Pj, A, eps=0.05):
    """(Lambda (6, 6), |K|) of an edge whose transform A maps fragment i into j."""
    Pi = _f32(Pi); Pj = _f32(Pj)
    L = np.zeros(36); cnt = C.c_int64()
    lib().orc_edge_info(_p(Pi[0]), _p(Pi[1]), _p(Pi[2]), C.c_int64(Pi.shape[1]), _p(Pj[0]), _p(Pj[1]),
                        _p(Pj[2]), C.c_int64(Pj.shape[1]), _p(_f64(A).reshape(16)), C.c_float(eps), _p(L),
                        C.byref(cnt))
    return L.reshape(6, 6), cnt.value


def loop_solve(T_init, odo, L_odo, loop, L_loop, count_loop, params=None):
    """One loop candidate against a chain.  odo: list of (i, j, A) for the
    n - 1 odometry edges, L_odo (n - 1, 6, 6); loop: (i, j, A).  Returns
    (result dict, optimised poses (n, 4, 4))."""
    T_init = _f64(T_init).reshape(-1, 16)
    n = T_init.shape[0]
    prm = params or loop_params()
    out = np.zeros((n, 16))
    res = LoopResult()
    lo = _f64(L_odo).reshape(-1, 36) if n > 1 else np.zeros((1, 36))
    lib().orc_loop_solve(C.c_int32(n), _p(T_init), _edges(odo), _p(lo), _edges([loop]), _p(_f64(L_loop).reshape(36)),
                         C.c_int64(int(count_loop)), C.byref(prm), _p(out), C.byref(res))
    d = {k: getattr(res, k) for k, _ in LoopResult._fields_}
    return d, out.reshape(n, 4, 4)
