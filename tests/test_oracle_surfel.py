"""Pins of the oracle's dense surface correction (Sec. VI, eq. 7) against
facts that do not depend on its code: identity and global corrections,
the closed-form average of two corrections, the textbook pinhole projection
(division form) away from the image border, window and removal rules, order
preservation, and covariance under a rigid motion of the whole world."""
import numpy as np
import pytest

import oracle
from synth.surfels import CAMERA, make_surfel_map


def _project_div(T_old, p, cam):
    """Textbook pinhole projection (division form) of world points p (3, n)
    into a camera-to-world pose; returns u, v, depth and the distance of
    (u, v) to the image border in pixels."""
    R, t = T_old[:3, :3], T_old[:3, 3]
    c = R.T @ (p - t[:, None])
    u = cam["fx"] * c[0] / c[2] + cam["cx"]
    v = cam["fy"] * c[1] / c[2] + cam["cy"]
    border = np.minimum.reduce([u, cam["width"] - u, v, cam["height"] - v])
    return u, v, c[2], border


def _rig(T):
    return np.asarray(T, np.float64)


def _random_pose(rng):
    A = rng.normal(size=(3, 3))
    Qm, Rm = np.linalg.qr(A)
    Qm = Qm @ np.diag(np.sign(np.diag(Rm)))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] *= -1
    T = np.eye(4)
    T[:3, :3] = Qm
    T[:3, 3] = rng.normal(size=3)
    return T


@pytest.fixture(scope="module")
def smap():
    return make_surfel_map(20000, 64)


def test_identity_correction_keeps_surfels(smap):
    out, idx, k = oracle.surfel_correct(smap.S, smap.t0, smap.tu, smap.T_old, smap.T_old, smap.t_kf,
                                        smap.camera)
    kept = idx >= 0
    assert kept.sum() == out.shape[1] > 0
    assert np.array_equal(idx[kept], np.arange(out.shape[1]))          # order kept
    assert np.allclose(out[:3], smap.S[:3, kept], atol=2e-6, rtol=0)
    n = smap.S[3:, kept] / np.linalg.norm(smap.S[3:, kept], axis=0)
    assert np.allclose(out[3:], n, atol=1e-7, rtol=0)


def test_global_correction_moves_by_it(smap):
    rng = np.random.default_rng(3)
    G = _random_pose(rng)
    T_new = np.einsum("ij,kjl->kil", G, smap.T_old)
    out, idx, k = oracle.surfel_correct(smap.S, smap.t0, smap.tu, smap.T_old, T_new, smap.t_kf, smap.camera)
    kept = idx >= 0
    p = G[:3, :3] @ smap.S[:3, kept].astype(np.float64) + G[:3, 3:4]
    n = G[:3, :3] @ smap.S[3:, kept].astype(np.float64)
    n /= np.linalg.norm(n, axis=0)
    assert np.allclose(out[:3], p, atol=4e-6, rtol=0)
    assert np.allclose(out[3:], n, atol=1e-6, rtol=0)


def test_observation_count_matches_division_form_projection(smap):
    """k_obs against the textbook projection, for surfels whose projections
    all lie more than 1e-6 px from the image border and 1e-9 m from the depth
    limits in every keyframe of their window."""
    out, idx, k = oracle.surfel_correct(smap.S, smap.t0, smap.tu, smap.T_old, smap.T_new, smap.t_kf,
                                        smap.camera)
    p = smap.S[:3].astype(np.float64)
    want = np.zeros(p.shape[1], np.int64)
    near = np.zeros(p.shape[1], bool)
    for f in range(len(smap.t_kf)):
        win = (smap.t0 < smap.t_kf[f]) & (smap.t_kf[f] < smap.tu)
        u, v, z, border = _project_div(smap.T_old[f], p, CAMERA)
        inz = (z >= CAMERA["z_min"]) & (z <= CAMERA["z_max"])
        vis = inz & (border > 0) & (u >= 0) & (v >= 0)
        want += win & vis
        near |= win & inz & (np.abs(border) < 1e-6)
        near |= win & ((np.abs(z - CAMERA["z_min"]) < 1e-9) | (np.abs(z - CAMERA["z_max"]) < 1e-9))
    assert near.mean() < 0.01
    assert np.array_equal(k[~near], want[~near])
    assert 0.3 < (k > 0).mean() < 0.95          # the recipe both keeps and removes surfels


def test_average_of_two_corrections_closed_form():
    """Two cameras looking at one surfel: the update is the mean of the two
    corrected positions; a third keyframe outside the window is ignored."""
    cam = dict(CAMERA)
    p = np.array([[0.1], [0.05], [2.0]], np.float32)
    S = np.vstack([p, np.array([[0.0], [0.0], [-1.0]], np.float32)])
    T1 = np.eye(4)
    T2 = np.eye(4)
    T2[:3, 3] = [0.2, 0.0, 0.0]
    rng = np.random.default_rng(11)
    G1 = _random_pose(rng) @ np.diag([1.0, 1, 1, 1])
    G1[:3, 3] *= 0.1
    G2 = np.eye(4)
    G2[:3, 3] = [0.0, 0.3, 0.0]
    T_old = np.stack([T1, T2, T1])
    T_new = np.stack([G1 @ T1, G2 @ T2, G2 @ T1])
    t_kf = np.array([10, 20, 30], np.int32)
    out, idx, k = oracle.surfel_correct(S, np.array([5], np.int32), np.array([25], np.int32), T_old, T_new,
                                        t_kf, cam)
    assert k[0] == 2 and idx[0] == 0
    pp = p[:, 0].astype(np.float64)
    want = ((G1[:3, :3] @ pp + G1[:3, 3]) + (G2[:3, :3] @ pp + G2[:3, 3])) / 2
    assert np.allclose(out[:3, 0], want, atol=1e-6, rtol=0)
    n = G1[:3, :3] @ [0, 0, -1.0] + G2[:3, :3] @ [0, 0, -1.0]
    assert np.allclose(out[3:, 0], n / np.linalg.norm(n), atol=1e-6, rtol=0)


def test_window_is_strict_and_empty_windows_remove():
    cam = dict(CAMERA)
    S = np.array([[0.0], [0.0], [2.0], [0.0], [0.0], [-1.0]], np.float32).repeat(4, axis=1)
    T_old = np.stack([np.eye(4)])
    G = np.eye(4)
    G[:3, 3] = [0.0, 0.0, 0.5]
    T_new = np.stack([G])
    t_kf = np.array([10], np.int32)
    t0 = np.array([9, 10, 9, 0], np.int32)
    tu = np.array([11, 11, 10, 5], np.int32)           # inside, t0 == t_kf, tu == t_kf, before
    out, idx, k = oracle.surfel_correct(S, t0, tu, T_old, T_new, t_kf, cam)
    assert k.tolist() == [1, 0, 0, 0]
    assert idx.tolist() == [0, -1, -1, -1]
    assert out.shape[1] == 1 and np.allclose(out[:3, 0], [0, 0, 2.5])


def test_behind_the_camera_and_out_of_range_removed():
    cam = dict(CAMERA)
    S = np.array([[0.0, 0.0, 0.0, 3.0],
                  [0.0, 0.0, 0.0, 0.0],
                  [-2.0, 6.0, 0.05, 2.0],
                  [0, 0, 0, 0], [0, 0, 0, 0], [1, 1, 1, 1]], np.float32)   # behind, beyond z_max, too near, off image
    out, idx, k = oracle.surfel_correct(S, np.zeros(4, np.int32), np.full(4, 20, np.int32),
                                        np.stack([np.eye(4)]), np.stack([np.eye(4)]), np.array([10], np.int32), cam)
    assert k.tolist() == [0, 0, 0, 0] and out.shape[1] == 0


def test_rigid_motion_of_the_world_is_covariant(smap):
    """Moving surfels and every pose (before and after) by one rigid motion W
    moves the corrected surfels by W (observations are camera-relative)."""
    rng = np.random.default_rng(5)
    Wm = _random_pose(rng)
    S2 = np.vstack([Wm[:3, :3] @ smap.S[:3].astype(np.float64) + Wm[:3, 3:4],
                    Wm[:3, :3] @ smap.S[3:].astype(np.float64)]).astype(np.float32)
    To2 = np.einsum("ij,kjl->kil", Wm, smap.T_old)
    Tn2 = np.einsum("ij,kjl->kil", Wm, smap.T_new)
    out1, idx1, k1 = oracle.surfel_correct(smap.S, smap.t0, smap.tu, smap.T_old, smap.T_new, smap.t_kf,
                                           smap.camera)
    out2, idx2, k2 = oracle.surfel_correct(S2, smap.t0, smap.tu, To2, Tn2, smap.t_kf, smap.camera)
    same = (k1 == k2)
    assert same.mean() > 0.999                     # observation decisions move with the world
    both = same & (idx1 >= 0)
    a = out1[:, idx1[both]].astype(np.float64)
    b = out2[:, idx2[both]].astype(np.float64)
    assert np.allclose(Wm[:3, :3] @ a[:3] + Wm[:3, 3:4], b[:3], atol=2e-5, rtol=0)
    assert np.allclose(Wm[:3, :3] @ a[3:], b[3:], atol=2e-6, rtol=0)
