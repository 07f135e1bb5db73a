"""Fragment chains with loop candidates (stand-in for the paper's sequence of
scene fragments and its loop proposals, which are absent here).

Recipe: a room U[4,6] x U[4,6] x U[2.5,3] m (floor, ceiling, walls) plus
6-10 boxes on the floor.  n fragments along a camera path that circles the
room 1.25 times (an ellipse at 0.35 of the half-widths, 1.3-1.6 m high),
each camera looking outward; fragment s holds the surface points within
1.2 m of the point 2 m ahead of its camera, m points area-uniform with
sigma = 3 mm noise, in its own frame (P_s = T_s^-1 world).  Odometry edge s
measures the true motion between fragments s and s + 1 up to a random error
of about 0.3 deg / 5 mm (so the dead-reckoned trajectory drifts); initial
poses chain those measurements from the true first pose.  Loop candidates:
true loops join fragments that look at the same wall on both passes (their
transform is the true one up to 0.5 deg / 1 cm, as a good registration
gives), false loops join two fragments that look at different parts of
the same wall with the transform that slides the first one's view along the
wall onto the second one's and turns it 5-20 deg about the wall normal:
plane-on-plane, so many points still find a neighbour, as after a failed
registration of look-alike surfaces.

Transforms map a fragment's frame into another's: an edge (i, j, A) has
q_j ~ A p_i.  Only seeded sampling and pose composition here, none of the
verification's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

CHAIN_SEED = 1801_01572 * 10 + 7


@dataclass
class Chain:
    frags: list            # n arrays (6, m) float32: x y z nx ny nz, each in its own frame
    T_true: np.ndarray     # (n, 4, 4) fragment -> world
    T_init: np.ndarray     # (n, 4, 4) dead-reckoned from the odometry
    odo: list              # n - 1 edges (s, s + 1, A)
    loops: list            # candidates (i, j, A)
    loop_true: np.ndarray  # (C,) bool


def _rot(axis, ang):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def _pert(rng, deg, m, exact=False):
    T = np.eye(4)
    ang = np.deg2rad(deg) if exact else np.deg2rad(deg) * abs(rng.normal())
    T[:3, :3] = _rot(rng.normal(size=3), ang)
    d = rng.normal(size=3)
    T[:3, 3] = d / np.linalg.norm(d) * m if exact else rng.normal(scale=m, size=3)
    return T


def _inv(T):
    R, t = T[:3, :3], T[:3, 3]
    o = np.eye(4)
    o[:3, :3] = R.T
    o[:3, 3] = -R.T @ t
    return o


def _surface(rng, n, W, D, H, boxes):
    rects = [((0, 0, 0), (W, 0, 0), (0, D, 0), (0, 0, 1)), ((0, 0, H), (W, 0, 0), (0, D, 0), (0, 0, -1)),
             ((0, 0, 0), (W, 0, 0), (0, 0, H), (0, 1, 0)), ((0, D, 0), (W, 0, 0), (0, 0, H), (0, -1, 0)),
             ((0, 0, 0), (0, D, 0), (0, 0, H), (1, 0, 0)), ((W, 0, 0), (0, D, 0), (0, 0, H), (-1, 0, 0))]
    for (x, y, sx, sy, sz) in boxes:       # five outer faces of a box standing on the floor
        o = np.array([x, y, 0.0])
        rects += [(o + (0, 0, sz), (sx, 0, 0), (0, sy, 0), (0, 0, 1)),
                  (o, (sx, 0, 0), (0, 0, sz), (0, -1, 0)), (o + (0, sy, 0), (sx, 0, 0), (0, 0, sz), (0, 1, 0)),
                  (o, (0, sy, 0), (0, 0, sz), (-1, 0, 0)), (o + (sx, 0, 0), (0, sy, 0), (0, 0, sz), (1, 0, 0))]
    areas = np.array([np.linalg.norm(np.cross(a, b)) for _, a, b, _ in rects])
    f = rng.choice(len(rects), size=n, p=areas / areas.sum())
    u, v = rng.random(n), rng.random(n)
    X = np.zeros((6, n))
    for k, (o, a, b, nrm) in enumerate(rects):
        sel = f == k
        X[:3, sel] = np.asarray(o, float)[:, None] + np.outer(a, u[sel]) + np.outer(b, v[sel])
        X[3:, sel] = np.asarray(nrm, float)[:, None]
    return X


def make_chain(n: int = 32, m: int = 20000, n_true: int = 8, n_false: int = 8, seed: int = CHAIN_SEED) -> Chain:
    rng = np.random.default_rng(seed)
    W, D, H = rng.uniform(4, 6), rng.uniform(4, 6), rng.uniform(2.5, 3.0)
    boxes = []
    for _ in range(rng.integers(6, 11)):
        sx, sy, sz = rng.uniform(0.3, 0.9, size=3)
        boxes.append((rng.uniform(0.2, W - sx - 0.2), rng.uniform(0.2, D - sy - 0.2), sx, sy, sz))
    density = 40000.0                                  # candidate samples per m^2
    area = 2 * (W * D + W * H + D * H) + sum(2 * sz * (sx + sy) + sx * sy for (_, _, sx, sy, sz) in boxes)
    world = _surface(rng, int(density * area), W, D, H, boxes)
    c = np.array([W / 2, D / 2])
    ang = 2.5 * np.pi * np.arange(n) / max(n - 1, 1)
    T_true = np.zeros((n, 4, 4))
    looks = np.zeros((n, 3))
    frags = []
    for s in range(n):
        a = ang[s]
        pos = np.array([c[0] + 0.35 * W / 2 * np.cos(a), c[1] + 0.35 * D / 2 * np.sin(a),
                        1.45 + 0.15 * np.sin(2 * a)])
        yaw = a + rng.uniform(-0.2, 0.2)
        pitch = np.deg2rad(rng.uniform(-20, 5))
        fwd = np.array([np.cos(yaw) * np.cos(pitch), np.sin(yaw) * np.cos(pitch), np.sin(pitch)])
        right = np.cross(fwd, [0.0, 0.0, 1.0])
        right /= np.linalg.norm(right)
        T = np.eye(4)
        T[:3, 0], T[:3, 1], T[:3, 2], T[:3, 3] = right, np.cross(fwd, right), fwd, pos
        T_true[s] = T
        look = pos + 2.0 * fwd
        looks[s] = look
        sel = np.nonzero(np.sum((world[:3] - look[:, None]) ** 2, axis=0) <= 1.2 ** 2)[0]
        pick = rng.choice(sel, size=min(m, len(sel)), replace=False)
        X = world[:, pick].copy()
        X[:3] += rng.normal(scale=0.003, size=X[:3].shape)
        Ti = _inv(T)
        P = np.vstack([Ti[:3, :3] @ X[:3] + Ti[:3, 3:4], Ti[:3, :3] @ X[3:]])
        frags.append(P.astype(np.float32))
    odo = []
    T_init = np.zeros_like(T_true)
    T_init[0] = T_true[0]
    for s in range(n - 1):
        A = _pert(rng, 0.3, 0.005) @ _inv(T_true[s + 1]) @ T_true[s]
        odo.append((s, s + 1, A))
        T_init[s + 1] = T_init[s] @ _inv(A)
    # true loops: the second pass over the same wall (angle + 2 pi)
    loops, truth = [], []
    second = [s for s in range(n) if ang[s] >= 2 * np.pi - 1e-9]
    pairs = []
    for j in second:
        i = int(np.argmin(np.abs(ang[: j] - (ang[j] - 2 * np.pi))))
        if j - i > 2:
            pairs.append((i, j))
    for k in range(min(n_true, len(pairs))):
        i, j = pairs[k % len(pairs)]
        loops.append((i, j, _pert(rng, 0.5, 0.01) @ _inv(T_true[j]) @ T_true[i]))
        truth.append(True)
    # the wall each fragment looks at: nearest of x = 0, x = W, y = 0, y = D to its look-at point
    dist = np.stack([looks[:, 0], W - looks[:, 0], looks[:, 1], D - looks[:, 1]], 1)
    wall = np.argmin(dist, 1)
    normals = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0]])
    cand = [(i, j) for i in range(n) for j in range(i + 3, n)
            if wall[i] == wall[j] and (i, j) not in pairs
            and np.linalg.norm(looks[i] - looks[j]) > 0.6 and abs(ang[j] - ang[i]) < 2 * np.pi - 0.8]
    order = rng.permutation(len(cand))
    for k in order[:n_false]:
        i, j = cand[k]
        nw = normals[wall[i]]
        slide = np.eye(4)
        d = looks[j] - looks[i]
        slide[:3, 3] = d - np.dot(d, nw) * nw                  # along the wall
        turn = np.eye(4)
        turn[:3, :3] = _rot(nw, np.deg2rad(rng.uniform(5, 20)) * rng.choice([-1, 1]))
        turn[:3, 3] = looks[j] - turn[:3, :3] @ looks[j]          # about the normal through j's view
        Tw = turn @ slide
        loops.append((i, j, _inv(T_true[j]) @ Tw @ T_true[i]))
        truth.append(False)
    return Chain(frags=frags, T_true=T_true, T_init=T_init, odo=odo, loops=loops, loop_true=np.array(truth))
