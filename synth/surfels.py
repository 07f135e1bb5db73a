"""Surfel maps and keyframe trajectories (stand-in for the dense model and
camera trajectory of the paper's SLAM system, which are absent here).

Recipe: a room U[4,6] x U[4,6] x U[2.5,3] m whose floor, ceiling and walls
carry n surfels, area-uniform, with unit normals facing into the room.  K
keyframes 10 frames apart on a closed loop through the room (an ellipse at
0.3 of the room's half-widths around its centre, 1.2-1.6 m high), each
looking outward along a yaw that turns with the path plus jitter, pitch
U(-15, 15) deg; pinhole camera 640 x 480, f = 525 px, depth 0.1-5 m.
Poses are camera-to-world (x right, y down, z forward).  The trajectory
before the loop correction (old poses) carries a random-walk drift of about
0.05 deg and 2 mm per keyframe; after it (new poses) the true poses with a
0.01 deg / 1 mm residual.  Each surfel's fusion window follows the loop:
the keyframes pass the surfel's azimuth about the room centre at
f_c = K azimuth / 2 pi, and the window spans f_c -+ U(0.08, 0.16) K keyframes
(first and last update, in frames); surfels near azimuth 0 are seen again
when the loop closes, outside their window.  Surfels are stored in order of
their first update, as a fusion map appends a surfel when it is first seen.

Only seeded sampling and pose composition here, none of the correction's
arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SURFEL_SEED = 1801_01572 * 10 + 6
CAMERA = {"fx": 525.0, "fy": 525.0, "cx": 319.5, "cy": 239.5, "width": 640, "height": 480,
          "z_min": 0.1, "z_max": 5.0}


@dataclass
class SurfelMap:
    S: np.ndarray          # (6, n) float32: x y z nx ny nz
    t0: np.ndarray         # (n,) int32 first update (frame)
    tu: np.ndarray         # (n,) int32 last update (frame)
    T_old: np.ndarray      # (K, 4, 4) float64 keyframe poses before the correction
    T_new: np.ndarray      # (K, 4, 4) after it
    t_kf: np.ndarray       # (K,) int32 keyframe frames, ascending
    camera: dict


def _rot(axis, ang):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def _small(rng, deg, m):
    T = np.eye(4)
    T[:3, :3] = _rot(rng.normal(size=3), np.deg2rad(deg) * abs(rng.normal()))
    T[:3, 3] = rng.normal(scale=m, size=3)
    return T


def _room_surfels(rng, n, W, D, H):
    faces = [  # origin, edge a, edge b, inward normal
        ((0, 0, 0), (W, 0, 0), (0, D, 0), (0, 0, 1)),
        ((0, 0, H), (W, 0, 0), (0, D, 0), (0, 0, -1)),
        ((0, 0, 0), (W, 0, 0), (0, 0, H), (0, 1, 0)),
        ((0, D, 0), (W, 0, 0), (0, 0, H), (0, -1, 0)),
        ((0, 0, 0), (0, D, 0), (0, 0, H), (1, 0, 0)),
        ((W, 0, 0), (0, D, 0), (0, 0, H), (-1, 0, 0)),
    ]
    areas = np.array([np.linalg.norm(np.cross(a, b)) for _, a, b, _ in faces])
    f = rng.choice(len(faces), size=n, p=areas / areas.sum())
    u, v = rng.random(n), rng.random(n)
    S = np.zeros((6, n), np.float64)
    for k, (o, a, b, nrm) in enumerate(faces):
        sel = f == k
        S[:3, sel] = (np.asarray(o, float)[:, None] + np.outer(a, u[sel]) + np.outer(b, v[sel]))
        S[3:, sel] = np.asarray(nrm, float)[:, None]
    return S


def make_surfel_map(n: int, n_kf: int, seed: int = SURFEL_SEED) -> SurfelMap:
    rng = np.random.default_rng(seed)
    W, D, H = rng.uniform(4, 6), rng.uniform(4, 6), rng.uniform(2.5, 3.0)
    S = _room_surfels(rng, n, W, D, H)
    c = np.array([W / 2, D / 2])
    T_true = np.zeros((n_kf, 4, 4))
    for f in range(n_kf):
        a = 2 * np.pi * f / n_kf
        pos = np.array([c[0] + 0.3 * W / 2 * np.cos(a), c[1] + 0.3 * D / 2 * np.sin(a),
                        1.4 + 0.2 * np.sin(3 * a)])
        yaw = a + rng.uniform(-0.6, 0.6)
        pitch = np.deg2rad(rng.uniform(-15, 15))
        fwd = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
        right = np.cross(fwd, [0.0, 0.0, 1.0])
        right /= np.linalg.norm(right)
        down = np.cross(fwd, right)
        T = np.eye(4)
        T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = right, down, fwd, pos
        T_true[f] = T
    drift = np.eye(4)
    T_old = np.zeros_like(T_true)
    T_new = np.zeros_like(T_true)
    for f in range(n_kf):
        drift = drift @ _small(rng, 0.05, 0.002)
        T_old[f] = drift @ T_true[f]
        T_new[f] = _small(rng, 0.01, 0.001) @ T_true[f]
    t_kf = (10 * np.arange(n_kf)).astype(np.int32)
    az = np.mod(np.arctan2(S[1] - c[1], S[0] - c[0]), 2 * np.pi)
    fc = n_kf * az / (2 * np.pi)
    h = rng.uniform(0.08, 0.16, size=n) * n_kf
    t0 = np.maximum(np.round(10 * (fc - h)), -1).astype(np.int32)
    tu = np.round(10 * (fc + h)).astype(np.int32)
    order = np.argsort(t0, kind="stable")
    return SurfelMap(S=np.ascontiguousarray(S[:, order], dtype=np.float32), t0=np.ascontiguousarray(t0[order]),
                     tu=np.ascontiguousarray(tu[order]), T_old=T_old, T_new=T_new, t_kf=t_kf, camera=dict(CAMERA))
