"""Shared helpers for the GPU parity tests (inputs, oracle runs, tolerances)."""
import numpy as np
import torch

import synth

# Tolerances (see the parity section of the design notes):
DESC_RTOL = 1e-4          # descriptors: per-point relative L2 error
POSE_TOL = 1e-5           # radians / metres
NORMAL_TOL = 1e-10        # normals, FP64 on both sides, different eigen-solvers
MARGIN = 1e-9             # decisions closer than this (bin units / dot) to a boundary are exempt
# result fields that count the screen's work, not results: they differ between
# precisions and launch-shape variants
WORK_KEYS = ("n_fallback_rows", "n_screen_chunks", "n_screen_chunks_swept")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def pair(config, idx=0, n=None, overlap=None):
    return synth.make_pair(config, idx, n_points=n, overlap=overlap)


def rot_err(A, B):
    R = A[:3, :3].T @ B[:3, :3]
    ang = np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1))
    return float(ang), float(np.linalg.norm(A[:3, 3] - B[:3, 3]))


def desc_exempt(orc, cloud, nrm, gap, ori, r_f):
    """Points whose descriptor depends on a decision within MARGIN of its
    boundary (bins, source choice) or on an ill-conditioned normal."""
    F, v, sm, dm = orc.fpfh(cloud[:3], nrm, r_f)
    bad_n = ((gap >= 0) & (gap < 1e-7)) | (ori < 1e-9)
    off, idx = orc.neighbors(cloud[:3], r_f)
    # a descriptor sees normals within 2 r_f (neighbours of neighbours)
    touch = bad_n.copy()
    for _ in range(2):
        nxt = touch.copy()
        for i in np.nonzero(touch)[0]:
            nxt[idx[off[i]:off[i + 1]]] = True
        touch = nxt
    return F, v, (dm < MARGIN) | touch


def orc_params(orc, prm):
    """The oracle's parameters for a GPU parameter block."""
    return orc.default_params(r_normal=prm.r_normal, r_feature=prm.r_feature, max_corr=prm.max_corr,
                              tau=prm.tau, n_trials=prm.n_trials, gnc_div=prm.gnc_div,
                              gnc_every=prm.gnc_every, gnc_max_iter=prm.gnc_max_iter,
                              polish_iter=prm.polish_iter, min_inlier_ratio=prm.min_inlier_ratio,
                              min_consistent=prm.min_consistent, seed=prm.seed)


def check_chain(orc, P, Q, r, tr, prm, label=""):
    """Stage-by-stage parity of one pair of a full GPU run against the oracle.

    r: the GPU's result; tr: its per-point trace (numpy nnQ, nnP, mutual,
    consistent, desc_P, desc_Q, valid_P, valid_Q of this pair).  Each GPU
    stage is checked on the GPU's own input to that stage, so that a
    legitimate difference upstream (a descriptor decision within MARGIN of a
    bin edge, a near-tie) cannot hide a later mismatch:
      validity flags exact, descriptors within DESC_RTOL of the oracle's
      except the oracle's exempt points; descriptor neighbours equal the
      oracle's matcher run on the GPU's descriptors outside the tie margin
      (both directions); the reciprocal flags follow from the GPU's
      neighbours; the consistency flags equal the oracle's filter run on the
      GPU's correspondences, bit for bit; the pose is within POSE_TOL of the
      oracle's robust solve on the GPU's consistent set; the inlier count of
      the GPU's pose equals the oracle's verification of that pose, and the
      status follows from it.  Returns a summary (the number of
      correspondences that differ from the oracle's own, the tie-exempt
      share, the pose error)."""
    nP, nQ = P.shape[1], Q.shape[1]
    nrmP, gP, oP = orc.normals(P, prm.r_normal)[:3]
    nrmQ, gQ, oQ = orc.normals(Q, prm.r_normal)[:3]
    F, vF, exP = desc_exempt(orc, P, nrmP, gP, oP, prm.r_feature)
    G, vG, exQ = desc_exempt(orc, Q, nrmQ, gQ, oQ, prm.r_feature)
    assert np.array_equal(tr["valid_P"], vF) and np.array_equal(tr["valid_Q"], vG), label
    assert (r["n_valid_P"], r["n_valid_Q"]) == (int(vF.sum()), int(vG.sum())), label
    for Fo, Fg, ex, side in ((F, tr["desc_P"], exP, "P"), (G, tr["desc_Q"], exQ, "Q")):
        err = np.linalg.norm(Fg - Fo, axis=1) / np.maximum(np.linalg.norm(Fo, axis=1), 1e-30)
        bad = np.nonzero((err > DESC_RTOL) & ~ex)[0]
        assert len(bad) == 0, (label, "descriptors", side, bad[:5], err[bad[:5]])
    FG, GG = tr["desc_P"].astype(np.float32), tr["desc_Q"].astype(np.float32)
    mg = orc.match(FG, tr["valid_P"], GG, tr["valid_Q"])
    tP, tQ = orc.tie_flags(FG, GG, mg)
    nnQ, nnP = tr["nnQ"].astype(np.int64), tr["nnP"].astype(np.int64)
    badQ = np.nonzero((nnQ != mg["nnQ"]) & ~tP)[0]
    badP = np.nonzero((nnP != mg["nnP"]) & ~tQ)[0]
    assert len(badQ) == 0 and len(badP) == 0, (label, "neighbours outside the tie margin", badQ[:5], badP[:5])
    m = orc.match(F, vF, G, vG)
    tP, tQ = orc.tie_flags(F, G, m)
    mut = orc.mutual(nnQ, nnP)
    assert np.array_equal(tr["mutual"].astype(bool), mut), label
    assert r["n_recip"] == int(mut.sum()), label
    mut_o = orc.mutual(m["nnQ"], m["nnP"])
    cg = set(zip(np.nonzero(mut)[0].tolist(), nnQ[mut].tolist()))
    co = set(zip(np.nonzero(mut_o)[0].tolist(), m["nnQ"][mut_o].tolist()))
    n_cdiff = len(cg ^ co)
    T_trials = prm.n_trials if prm.n_trials > 0 else orc.default_trials(nP)
    want, _ = orc.consistency(P[:3], Q[:3], nnQ.astype(np.int32), mut, T_trials, prm.tau, prm.seed)
    assert np.array_equal(tr["consistent"].astype(bool), want), (label, "consistency flags")
    K = int(want.sum())
    assert r["n_consistent"] == K, label
    idx = np.nonzero(want)[0]
    p = P[:3, idx].T.astype(np.float64)
    q = Q[:3, nnQ[idx]].T.astype(np.float64)
    st, To, _, _, _ = orc.gnc(p, q, orc_params(orc, prm))
    out = {"n_c_diff": n_cdiff, "tie_exempt_P": float(tP[vF == 1].mean()) if vF.any() else 0.0,
           "K": K, "pose_err": None}
    if st == orc.DEGENERATE:
        assert r["status"] == orc.DEGENERATE, label
        return out
    ang, tr_err = rot_err(r["T"], To)
    assert ang <= POSE_TOL and tr_err <= POSE_TOL, (label, ang, tr_err)
    out["pose_err"] = (ang, tr_err)
    ni, ratio, _ = orc.verify(P, None, Q, None, r["T"], prm.max_corr)
    assert r["n_inliers"] == ni, (label, r["n_inliers"], ni)
    ok = K >= prm.min_consistent and ratio >= np.float64(np.float32(prm.min_inlier_ratio))
    assert r["status"] == (orc.ACCEPTED if ok else orc.REJECTED), (label, r["status"], ratio, K)
    return out


def trace_slice(tr, offP, offQ, b):
    """Pair b's part of a batch trace, as numpy arrays."""
    sP, sQ = slice(int(offP[b]), int(offP[b + 1])), slice(int(offQ[b]), int(offQ[b + 1]))
    return {"nnQ": tr["nnQ"][sP].cpu().numpy(), "nnP": tr["nnP"][sQ].cpu().numpy(),
            "mutual": tr["mutual"][sP].cpu().numpy(), "consistent": tr["consistent"][sP].cpu().numpy(),
            "desc_P": tr["desc_P"][sP].cpu().numpy(), "desc_Q": tr["desc_Q"][sQ].cpu().numpy(),
            "valid_P": tr["valid_P"][sP].cpu().numpy(), "valid_Q": tr["valid_Q"][sQ].cpu().numpy()}
