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
