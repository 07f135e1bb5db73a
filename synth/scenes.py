"""Scene primitives, surface sampling, cropping and rigid transforms.

Workload recipes (one per configuration index):

0  2 m cube: floor + two walls, two boxes on the floor, one floating sphere.
   Q = 5,000 area-uniform samples of the whole scene; P = 5,000 independent
   area-uniform samples of a half-space crop holding 70% of the surface area.
   Noise sigma = 3 mm.
1  Room U[4,6] x U[4,6] x U[2.5,3] m with 10-20 boxes / cylinders.  Surfaces
   are sampled on a jittered 1 cm lattice (the density a 1 cm voxel grid
   leaves), two independent samplings give the two fragments, each the 50,000
   samples nearest to its own centre, with 50% of P inside Q's crop ball.
   Noise sigma = 5 mm added after cropping.
2  256 pairs of the room recipe, sizes U[5k, 80k] per fragment, overlap
   U[0.3, 0.9], 20% of the pairs disjoint crops of the same room (negatives).
3  3 x 3 rooms with doorways (building scale), two 500,000-point fragments,
   40% overlap, 1 cm lattice, sigma = 5 mm.
4  64 pairs of 20,000-point fragments from the room recipe (50% overlap).
5  Test recipe for recovery checks: a room holding 25 objects of varied
   curvature (spheres, cylinders, boxes), 20,000-point fragments, 50% overlap,
   sigma = 1 mm.  Its local geometry is distinctive enough for descriptor
   matching to find true correspondences.

The rigid transform law is shared: rotation axis uniform on the sphere,
angle U(0, 60 deg), translation U(-0.5, 0.5)^3 m.  P is expressed in its own
frame, so q ~ R_gt p + t_gt for corresponding points.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 1801_01572 * 10

CONFIG_NAMES = {
    0: "cube-scene 5k/5k, 70% crop, sigma 3 mm",
    1: "indoor room 50k/50k, 1 cm lattice, 50% overlap, sigma 5 mm",
    2: "256 ragged room pairs U[5k,80k], overlap U[0.3,0.9], 20% negatives",
    3: "3x3-room building 500k/500k, 40% overlap",
    4: "64 room pairs 20k/20k, 50% overlap",
    5: "geometry-rich room (spheres, cylinders, boxes) 20k/20k, 50% overlap, sigma 1 mm",
}


@dataclass
class Pair:
    P: np.ndarray          # (6, nP) float32 SoA: x y z nx ny nz (P's own frame)
    Q: np.ndarray          # (6, nQ) float32 SoA
    T_gt: np.ndarray       # (4, 4) float64, maps P into Q's frame
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# primitives: each is a dict with a 'kind' and its parameters
# --------------------------------------------------------------------------

def _rect(o, a, b, n):
    return {"kind": "rect", "o": np.asarray(o, float), "a": np.asarray(a, float),
            "b": np.asarray(b, float), "n": np.asarray(n, float)}


def _disk(c, r, n, e1, e2):
    return {"kind": "disk", "c": np.asarray(c, float), "r": float(r), "n": np.asarray(n, float),
            "e1": np.asarray(e1, float), "e2": np.asarray(e2, float)}


def _cyl(c, r, h):
    return {"kind": "cyl", "c": np.asarray(c, float), "r": float(r), "h": float(h)}


def _sphere(c, r):
    return {"kind": "sphere", "c": np.asarray(c, float), "r": float(r)}


def _area(p):
    k = p["kind"]
    if k == "rect":
        return float(np.linalg.norm(p["a"]) * np.linalg.norm(p["b"]))
    if k == "disk":
        return float(np.pi * p["r"] ** 2)
    if k == "cyl":
        return float(2 * np.pi * p["r"] * p["h"])
    return float(4 * np.pi * p["r"] ** 2)


def _box_prims(cx, cy, hx, hy, hz, yaw):
    ex = np.array([np.cos(yaw), np.sin(yaw), 0.0])
    ey = np.array([-np.sin(yaw), np.cos(yaw), 0.0])
    ez = np.array([0.0, 0.0, 1.0])
    c = np.array([cx, cy, 0.0])
    return [
        _rect(c + hx * ex - hy * ey, 2 * hy * ey, hz * ez, ex),
        _rect(c - hx * ex - hy * ey, 2 * hy * ey, hz * ez, -ex),
        _rect(c - hx * ex + hy * ey, 2 * hx * ex, hz * ez, ey),
        _rect(c - hx * ex - hy * ey, 2 * hx * ex, hz * ez, -ey),
        _rect(c - hx * ex - hy * ey + hz * ez, 2 * hx * ex, 2 * hy * ey, ez),
    ]


def _cyl_prims(cx, cy, r, h):
    return [
        _cyl([cx, cy, 0.0], r, h),
        _disk([cx, cy, h], r, [0, 0, 1], [1, 0, 0], [0, 1, 0]),
    ]


def _inside_solids(pts, solids, eps=1e-3):
    """Mask of points strictly inside any solid object (hidden surfaces).
    Each solid is tested only against the points in the x-slab its footprint
    spans (points sorted by x once); the mask is the same as a full test."""
    bad = np.zeros(len(pts), bool)
    order = np.argsort(pts[:, 0], kind="stable")
    xs = pts[order, 0]

    def slab(cx, rad):
        lo, hi = np.searchsorted(xs, cx - rad - 1e-9), np.searchsorted(xs, cx + rad + 1e-9, side="right")
        return order[lo:hi]

    for s in solids:
        if s[0] == "box":
            _, cx, cy, hx, hy, hz, yaw = s
            idx = slab(cx, float(np.hypot(hx, hy)))
            q = pts[idx]
            d = q[:, :2] - np.array([cx, cy])
            lx = d[:, 0] * np.cos(yaw) + d[:, 1] * np.sin(yaw)
            ly = -d[:, 0] * np.sin(yaw) + d[:, 1] * np.cos(yaw)
            bad[idx] |= (np.abs(lx) < hx - eps) & (np.abs(ly) < hy - eps) & (q[:, 2] < hz - eps)
        elif s[0] == "cyl":
            _, cx, cy, r, h = s
            idx = slab(cx, r)
            q = pts[idx]
            rr = np.hypot(q[:, 0] - cx, q[:, 1] - cy)
            bad[idx] |= (rr < r - eps) & (q[:, 2] < h - eps)
        else:  # sphere
            _, c, r = s
            idx = slab(c[0], r)
            bad[idx] |= np.linalg.norm(pts[idx] - c, axis=1) < r - eps
    return bad


# --------------------------------------------------------------------------
# sampling
# --------------------------------------------------------------------------

def _sample_prim_uniform(p, n, rng):
    k = p["kind"]
    if n == 0:
        return np.zeros((0, 3)), np.zeros((0, 3))
    if k == "rect":
        u, v = rng.random(n), rng.random(n)
        x = p["o"] + u[:, None] * p["a"] + v[:, None] * p["b"]
        return x, np.broadcast_to(p["n"], x.shape).copy()
    if k == "disk":
        rr = p["r"] * np.sqrt(rng.random(n))
        th = 2 * np.pi * rng.random(n)
        x = p["c"] + (rr * np.cos(th))[:, None] * p["e1"] + (rr * np.sin(th))[:, None] * p["e2"]
        return x, np.broadcast_to(p["n"], x.shape).copy()
    if k == "cyl":
        th = 2 * np.pi * rng.random(n)
        z = p["h"] * rng.random(n)
        nrm = np.stack([np.cos(th), np.sin(th), np.zeros(n)], 1)
        x = p["c"] + p["r"] * nrm + np.stack([np.zeros(n), np.zeros(n), z], 1)
        return x, nrm
    g = rng.standard_normal((n, 3))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return p["c"] + p["r"] * g, g


def _sample_area(prims, n, rng):
    """n area-weighted uniform samples over all primitives."""
    areas = np.array([_area(p) for p in prims])
    counts = rng.multinomial(n, areas / areas.sum())
    xs, ns = zip(*[_sample_prim_uniform(p, int(c), rng) for p, c in zip(prims, counts)])
    return np.concatenate(xs), np.concatenate(ns)


def _lattice_1d(length, h, rng, jit):
    m = int(np.ceil(length / h)) + 1
    u = (np.arange(m) + rng.random()) * h
    return u[u < length], jit


def _sample_prim_lattice(p, h, rng, jit=0.25):
    """Jittered lattice of spacing h on one primitive (~1 sample per h^2)."""
    k = p["kind"]
    if k == "rect":
        la, lb = np.linalg.norm(p["a"]), np.linalg.norm(p["b"])
        u, _ = _lattice_1d(la, h, rng, jit)
        v, _ = _lattice_1d(lb, h, rng, jit)
        U, V = np.meshgrid(u, v, indexing="ij")
        U = np.clip(U.ravel() + rng.uniform(-jit, jit, U.size) * h, 0, la)
        V = np.clip(V.ravel() + rng.uniform(-jit, jit, V.size) * h, 0, lb)
        x = p["o"] + (U / la)[:, None] * p["a"] + (V / lb)[:, None] * p["b"]
        return x, np.broadcast_to(p["n"], x.shape).copy()
    if k == "disk":
        r = p["r"]
        u, _ = _lattice_1d(2 * r, h, rng, jit)
        U, V = np.meshgrid(u - r, u - r, indexing="ij")
        U = U.ravel() + rng.uniform(-jit, jit, U.size) * h
        V = V.ravel() + rng.uniform(-jit, jit, V.size) * h
        keep = U * U + V * V < r * r
        U, V = U[keep], V[keep]
        x = p["c"] + U[:, None] * p["e1"] + V[:, None] * p["e2"]
        return x, np.broadcast_to(p["n"], x.shape).copy()
    if k == "cyl":
        r, hh = p["r"], p["h"]
        nth = max(3, int(round(2 * np.pi * r / h)))
        th = 2 * np.pi * (np.arange(nth) + rng.random()) / nth
        z, _ = _lattice_1d(hh, h, rng, jit)
        TH, Z = np.meshgrid(th, z, indexing="ij")
        TH = TH.ravel() + rng.uniform(-jit, jit, TH.size) * (2 * np.pi / nth)
        Z = np.clip(Z.ravel() + rng.uniform(-jit, jit, Z.size) * h, 0, hh)
        nrm = np.stack([np.cos(TH), np.sin(TH), np.zeros(TH.size)], 1)
        x = p["c"] + r * nrm + np.stack([np.zeros(Z.size), np.zeros(Z.size), Z], 1)
        return x, nrm
    # sphere: golden-angle spiral with ~ one sample per h^2, randomly rotated
    m = max(8, int(round(4 * np.pi * p["r"] ** 2 / h ** 2)))
    i = np.arange(m) + 0.5
    zc = 1 - 2 * i / m
    rr = np.sqrt(1 - zc * zc)
    ph = np.pi * (3 - np.sqrt(5)) * i
    g = np.stack([rr * np.cos(ph), rr * np.sin(ph), zc], 1)
    g = g @ _rand_rot(rng, np.pi).T
    return p["c"] + p["r"] * g, g


def _sample_lattice(prims, h, rng):
    xs, ns = zip(*[_sample_prim_lattice(p, h, rng) for p in prims])
    return np.concatenate(xs), np.concatenate(ns)


# --------------------------------------------------------------------------
# rigid transforms
# --------------------------------------------------------------------------

def _axis_angle(axis, ang):
    a = axis / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * (K @ K)


def _rand_rot(rng, max_angle):
    axis = rng.standard_normal(3)
    return _axis_angle(axis, rng.uniform(0, max_angle))


def random_rigid(rng, max_angle_deg=60.0, max_trans=0.5):
    """Axis uniform on the sphere, angle U(0, max), translation U(-m, m)^3."""
    T = np.eye(4)
    T[:3, :3] = _rand_rot(rng, np.deg2rad(max_angle_deg))
    T[:3, 3] = rng.uniform(-max_trans, max_trans, 3)
    return T


def _to_soa(x, n):
    return np.ascontiguousarray(np.concatenate([x.T, n.T], 0).astype(np.float32))


def _finish(rng, A_x, A_n, B_x, B_n, sigma, meta):
    """Add noise, shuffle order, express B in its own frame: P = T^-1 B, Q = A."""
    A_x = A_x + rng.normal(0, sigma, A_x.shape)
    B_x = B_x + rng.normal(0, sigma, B_x.shape)
    pa = rng.permutation(len(A_x))
    pb = rng.permutation(len(B_x))
    A_x, A_n, B_x, B_n = A_x[pa], A_n[pa], B_x[pb], B_n[pb]
    T = random_rigid(rng)
    R, t = T[:3, :3], T[:3, 3]
    P_x = (B_x - t) @ R          # row-vector form of R^T (b - t)
    P_n = B_n @ R
    return Pair(P=_to_soa(P_x, P_n), Q=_to_soa(A_x, A_n), T_gt=T, meta=meta)


# --------------------------------------------------------------------------
# scenes
# --------------------------------------------------------------------------

def _cube_scene(rng):
    L = 2.0
    prims = [
        _rect([0, 0, 0], [L, 0, 0], [0, L, 0], [0, 0, 1]),
        _rect([0, 0, 0], [0, L, 0], [0, 0, L], [1, 0, 0]),
        _rect([0, 0, 0], [L, 0, 0], [0, 0, L], [0, 1, 0]),
    ]
    solids = []
    for _ in range(2):
        hx, hy, hz = rng.uniform(0.1, 0.3, 3)
        cx, cy = rng.uniform(0.4, 1.6, 2)
        yaw = rng.uniform(0, np.pi)
        prims += _box_prims(cx, cy, hx, hy, 2 * hz, yaw)
        solids.append(("box", cx, cy, hx, hy, 2 * hz, yaw))
    r = rng.uniform(0.15, 0.35)
    c = np.array([rng.uniform(0.6, 1.4), rng.uniform(0.6, 1.4), rng.uniform(0.9, 1.5)])
    prims.append(_sphere(c, r))
    solids.append(("sphere", c, r))
    return prims, solids


def _room_scene(rng, n_obj=None, size=None):
    Lx, Ly = rng.uniform(4, 6, 2) if size is None else size[:2]
    H = rng.uniform(2.5, 3.0) if size is None else size[2]
    prims = [
        _rect([0, 0, 0], [Lx, 0, 0], [0, Ly, 0], [0, 0, 1]),
        _rect([0, 0, H], [Lx, 0, 0], [0, Ly, 0], [0, 0, -1]),
        _rect([0, 0, 0], [0, Ly, 0], [0, 0, H], [1, 0, 0]),
        _rect([Lx, 0, 0], [0, Ly, 0], [0, 0, H], [-1, 0, 0]),
        _rect([0, 0, 0], [Lx, 0, 0], [0, 0, H], [0, 1, 0]),
        _rect([0, Ly, 0], [Lx, 0, 0], [0, 0, H], [0, -1, 0]),
    ]
    solids = []
    n_obj = int(rng.integers(10, 21)) if n_obj is None else n_obj
    for _ in range(n_obj):
        if rng.random() < 0.6:
            hx, hy = rng.uniform(0.15, 0.6, 2)
            hz = rng.uniform(0.3, 1.5)
            m = max(hx, hy) * 1.5 + 0.05
            cx, cy = rng.uniform(m, Lx - m), rng.uniform(m, Ly - m)
            yaw = rng.uniform(0, np.pi)
            prims += _box_prims(cx, cy, hx, hy, hz, yaw)
            solids.append(("box", cx, cy, hx, hy, hz, yaw))
        else:
            r = rng.uniform(0.1, 0.4)
            hz = rng.uniform(0.4, 1.5)
            cx, cy = rng.uniform(r + 0.05, Lx - r - 0.05), rng.uniform(r + 0.05, Ly - r - 0.05)
            prims += _cyl_prims(cx, cy, r, hz)
            solids.append(("cyl", cx, cy, r, hz))
    return prims, solids, np.array([Lx, Ly, H])


def _rich_room_scene(rng):
    prims, solids, ext = _room_scene(rng, n_obj=0)
    Lx, Ly, H = ext
    for _ in range(25):
        k = rng.random()
        if k < 0.4:
            r = rng.uniform(0.05, 0.3)
            c = np.array([rng.uniform(0.5, Lx - 0.5), rng.uniform(0.5, Ly - 0.5), rng.uniform(0.3, H - 0.5)])
            prims.append(_sphere(c, r))
            solids.append(("sphere", c, r))
        elif k < 0.7:
            r, hz = rng.uniform(0.04, 0.3), rng.uniform(0.3, 1.5)
            cx, cy = rng.uniform(0.5, Lx - 0.5), rng.uniform(0.5, Ly - 0.5)
            prims += _cyl_prims(cx, cy, r, hz)
            solids.append(("cyl", cx, cy, r, hz))
        else:
            hx, hy = rng.uniform(0.1, 0.5, 2)
            hz = rng.uniform(0.2, 1.2)
            cx, cy = rng.uniform(0.6, Lx - 0.6), rng.uniform(0.6, Ly - 0.6)
            yaw = rng.uniform(0, np.pi)
            prims += _box_prims(cx, cy, hx, hy, hz, yaw)
            solids.append(("box", cx, cy, hx, hy, hz, yaw))
    return prims, solids, ext


def _building_scene(rng, nx=3, ny=3, room=5.0, H=3.0, thick=0.1, door=1.0, door_h=2.1):
    """nx x ny rooms; interior walls (two faces, thickness `thick`) with doorways."""
    Lx, Ly = nx * room, ny * room
    prims, solids, _ = _room_scene(rng, n_obj=0, size=(Lx, Ly, H))

    def wall_x(x0, y0, y1, nrm):   # plane x = x0, spanning y in [y0, y1], with a doorway
        yc = 0.5 * (y0 + y1) + rng.uniform(-1, 1)
        a, b = yc - door / 2, yc + door / 2
        out = [_rect([x0, y0, 0], [0, a - y0, 0], [0, 0, H], nrm),
               _rect([x0, b, 0], [0, y1 - b, 0], [0, 0, H], nrm),
               _rect([x0, a, door_h], [0, door, 0], [0, 0, H - door_h], nrm)]
        return out

    def wall_y(y0, x0, x1, nrm):
        xc = 0.5 * (x0 + x1) + rng.uniform(-1, 1)
        a, b = xc - door / 2, xc + door / 2
        return [_rect([x0, y0, 0], [a - x0, 0, 0], [0, 0, H], nrm),
                _rect([b, y0, 0], [x1 - b, 0, 0], [0, 0, H], nrm),
                _rect([a, y0, door_h], [door, 0, 0], [0, 0, H - door_h], nrm)]

    for i in range(1, nx):
        for j in range(ny):
            x = i * room
            prims += wall_x(x - thick / 2, j * room, (j + 1) * room, [-1, 0, 0])
            prims += wall_x(x + thick / 2, j * room, (j + 1) * room, [1, 0, 0])
    for j in range(1, ny):
        for i in range(nx):
            y = j * room
            prims += wall_y(y - thick / 2, i * room, (i + 1) * room, [0, -1, 0])
            prims += wall_y(y + thick / 2, i * room, (i + 1) * room, [0, 1, 0])
    for i in range(nx):
        for j in range(ny):
            for _ in range(int(rng.integers(4, 9))):
                hx, hy = rng.uniform(0.15, 0.5, 2)
                hz = rng.uniform(0.3, 1.5)
                m = max(hx, hy) * 1.5 + 0.15
                cx = rng.uniform(i * room + m, (i + 1) * room - m)
                cy = rng.uniform(j * room + m, (j + 1) * room - m)
                yaw = rng.uniform(0, np.pi)
                prims += _box_prims(cx, cy, hx, hy, hz, yaw)
                solids.append(("box", cx, cy, hx, hy, hz, yaw))
    return prims, solids, np.array([Lx, Ly, H])


def _nearest(x, c, n):
    d2 = ((x - c) ** 2).sum(1)
    n = min(n, len(x))
    return np.argpartition(d2, n - 1)[:n]


def _crop_pair(rng, S1, S2, nA, nB, overlap, extent):
    """A = nA samples of S1 nearest a centre; B = nB samples of S2 nearest a
    shifted centre, the shift chosen so that a fraction `overlap` of B lies in
    A's crop ball (0 gives disjoint crops)."""
    lo = np.array([0.6, 0.6, 0.8])
    hi = np.maximum(extent - lo, lo + 1e-3)
    cA = rng.uniform(lo, hi)
    ia = _nearest(S1[0], cA, nA)
    rhoA = np.sqrt(((S1[0][ia] - cA) ** 2).sum(1).max())
    ang = rng.uniform(0, 2 * np.pi)
    d = np.array([np.cos(ang), np.sin(ang), 0.0])
    sub = rng.random(len(S2[0])) < 0.125
    S2s = S2[0][sub]
    nBs = max(8, nB // 8)

    def ov(s):
        ib = _nearest(S2s, cA + s * d, nBs)
        return float(np.mean(((S2s[ib] - cA) ** 2).sum(1) <= rhoA ** 2))

    s_lo, s_hi = 0.0, max(1.0, 2.5 * rhoA)
    while ov(s_hi) > 0 and s_hi < 4 * np.linalg.norm(extent):
        s_hi *= 1.5
    if overlap <= 0:
        s = s_hi + 0.25
    else:
        for _ in range(14):
            mid = 0.5 * (s_lo + s_hi)
            if ov(mid) > overlap:
                s_lo = mid
            else:
                s_hi = mid
        s = 0.5 * (s_lo + s_hi)
    ib = _nearest(S2[0], cA + s * d, nB)
    ov_true = float(np.mean(((S2[0][ib] - cA) ** 2).sum(1) <= rhoA ** 2))
    return (S1[0][ia], S1[1][ia], S2[0][ib], S2[1][ib], ov_true)


def _rng(config, pair, seed):
    s = BASE_SEED + config if seed is None else int(seed)
    return np.random.default_rng([s, int(pair)])


def _room_pair(rng, nP, nQ, overlap, sigma, meta, h=0.01, scene="room"):
    if scene == "room":
        prims, solids, ext = _room_scene(rng)
    elif scene == "rich":
        prims, solids, ext = _rich_room_scene(rng)
    else:
        prims, solids, ext = _building_scene(rng)
    S = []
    for _ in range(2):
        x, n = _sample_lattice(prims, h, rng)
        keep = ~_inside_solids(x, solids)
        S.append((x[keep], n[keep]))
    A_x, A_n, B_x, B_n, ov = _crop_pair(rng, S[0], S[1], nQ, nP, overlap, ext)
    meta = dict(meta, overlap=ov, n_P=len(B_x), n_Q=len(A_x), room=ext.tolist())
    return _finish(rng, A_x, A_n, B_x, B_n, sigma, meta)


def _c2_plan(seed):
    rng = np.random.default_rng([BASE_SEED + 2 if seed is None else int(seed), 1 << 20])
    neg = set(rng.permutation(256)[: int(round(0.2 * 256))].tolist())
    sizes = rng.integers(5000, 80001, size=(256, 2))
    ovl = rng.uniform(0.3, 0.9, 256)
    return neg, sizes, ovl


def make_pair(config: int, pair: int = 0, seed=None, n_points=None, overlap=None) -> Pair:
    """One seeded fragment pair of the given workload recipe.

    ``n_points`` (int or (nP, nQ)) and ``overlap`` override the recipe's sizes,
    e.g. for small parity cases with the same structure.
    """
    rng = _rng(config, pair, seed)
    if isinstance(n_points, (int, np.integer)):
        n_points = (int(n_points), int(n_points))
    meta = {"config": config, "pair": pair, "negative": False}
    if config == 0:
        nP, nQ = n_points or (5000, 5000)
        prims, solids = _cube_scene(rng)
        ov = 0.7 if overlap is None else overlap
        xa, na = _sample_area(prims, 4 * nQ, rng)
        keep = ~_inside_solids(xa, solids)
        xa, na = xa[keep][:nQ], na[keep][:nQ]
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        xd, nd = _sample_area(prims, 200_000, rng)
        keep = ~_inside_solids(xd, solids)
        thr = np.quantile(xd[keep] @ d, 1 - ov)
        xb, nb = _sample_area(prims, int(8 * nP / max(ov, 0.05)), rng)
        keep = (~_inside_solids(xb, solids)) & (xb @ d >= thr)
        xb, nb = xb[keep][:nP], nb[keep][:nP]
        meta.update(overlap=ov, n_P=len(xb), n_Q=len(xa))
        return _finish(rng, xa, na, xb, nb, 0.003, meta)
    if config in (1, 4):
        nP, nQ = n_points or ((50_000, 50_000) if config == 1 else (20_000, 20_000))
        return _room_pair(rng, nP, nQ, 0.5 if overlap is None else overlap, 0.005, meta)
    if config == 2:
        neg, sizes, ovl = _c2_plan(seed)
        nP, nQ = n_points or (int(sizes[pair % 256, 0]), int(sizes[pair % 256, 1]))
        negative = (pair % 256) in neg
        ov = 0.0 if negative else float(ovl[pair % 256])
        if overlap is not None:
            ov = overlap
        meta["negative"] = negative
        return _room_pair(rng, nP, nQ, ov, 0.005, meta)
    if config == 5:
        nP, nQ = n_points or (20_000, 20_000)
        return _room_pair(rng, nP, nQ, 0.5 if overlap is None else overlap, 0.001, meta, scene="rich")
    if config == 3:
        nP, nQ = n_points or (500_000, 500_000)
        return _room_pair(rng, nP, nQ, 0.4 if overlap is None else overlap, 0.005, meta,
                          scene="building")
    raise ValueError(f"unknown configuration {config}")


def _mk(args):
    return make_pair(*args[:2], **args[2])


def make_batch(config: int, n_pairs: int, seed=None, n_points=None, overlap=None,
               workers=None, first_pair: int = 0):
    """``n_pairs`` pairs of a recipe, generated in a process pool."""
    kw = dict(seed=seed, n_points=n_points, overlap=overlap)
    jobs = [(config, first_pair + k, kw) for k in range(n_pairs)]
    workers = workers or min(16, os.cpu_count() or 1, n_pairs)
    if workers <= 1 or n_pairs <= 1:
        return [_mk(j) for j in jobs]
    with _cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_mk, jobs))
