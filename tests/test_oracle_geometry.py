"""Pins of the CPU oracle's geometric stages against brute force, closed forms
and invariances (radius neighbourhoods of Sec. IV eq. 1; normals; FPFH as
cited by Algorithm 1; voxel downsampling of Algorithm 1's first step)."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _cloud(n, seed, extent=0.2):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, extent, (3, n)).astype(np.float32)


# ---------------------------------------------------------------- neighbourhoods

@pytest.mark.parametrize("seed", [0, 1])
def test_neighbors_grid_equals_brute_force(orc, seed):
    x = _cloud(1500, seed)
    a = orc.neighbors(x, 0.02)
    b = orc.neighbors(x, 0.02, brute=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[0][-1] > 1500            # non-trivial neighbourhoods


def test_neighbors_degenerate_inputs(orc):
    """Duplicates are never neighbours (d > 0); points exactly r apart on the
    cell lattice are (<= is inclusive); a lone point has none."""
    r = 0.25                                   # exactly representable
    g = np.arange(6, dtype=np.float32) * r     # on the grid lattice
    X, Y = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size, np.float32)])
    pts = np.concatenate([pts, pts[:, :5], np.array([[9.0], [9.0], [9.0]], np.float32)], 1)
    a = orc.neighbors(pts, r)
    b = orc.neighbors(pts, r, brute=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    off, idx = a
    assert np.diff(off)[-1] == 0                              # isolated point
    i = 7                                                     # interior lattice point (1,1)
    nb = set(idx[off[i]:off[i + 1]].tolist())
    assert nb == {1, 6, 8, 13, 37}                            # 4-connected at r, plus the copy of 1
    dup = 36                                                  # copy of point 0
    assert 0 not in idx[off[dup]:off[dup + 1]]


# ---------------------------------------------------------------- voxel

def test_voxel_equals_groupby(orc):
    rng = np.random.default_rng(3)
    c = np.concatenate([rng.uniform(-0.3, 0.3, (3, 4000)), rng.normal(0, 1, (3, 4000))]).astype(np.float32)
    c[3:] /= np.linalg.norm(c[3:], axis=0)
    v = np.float32(0.05)
    out = orc.voxel(c, v)
    keys = np.floor(c[:3].astype(np.float64) / np.float64(v)).astype(np.int64)
    uk, inv = np.unique(keys.T, axis=0, return_inverse=True)      # lexicographic (kx, ky, kz)
    inv = inv.ravel()
    assert out.shape[1] == len(uk)
    for k in range(len(uk)):
        m = inv == k
        mean = c[:3, m].astype(np.float64).mean(1)
        assert np.allclose(out[:3, k], mean, rtol=0, atol=1e-7)
        nm = c[3:, m].astype(np.float64).sum(1)
        nm /= np.linalg.norm(nm)
        assert np.allclose(out[3:, k], nm, atol=1e-6)


# ---------------------------------------------------------------- normals

def _plane_cloud(n, seed, z0=0.5):
    rng = np.random.default_rng(seed)
    xy = rng.uniform(0, 0.3, (2, n))
    nin = np.tile(np.array([[0.1], [0.2], [1.0]]), (1, n))
    return np.concatenate([xy, np.full((1, n), z0), nin]).astype(np.float32)


def test_normals_plane_exact(orc):
    c = _plane_cloud(3000, 0)
    nrm, gap, ori, cnt = orc.normals(c, 0.025)
    ok = cnt >= 2
    assert ok.mean() > 0.95
    assert np.abs(nrm[ok] - np.array([0, 0, 1.0])).max() <= 1e-14


def test_normals_fallback_and_orientation(orc):
    c = _plane_cloud(50, 1)
    c[:3] *= 100.0                                   # spread apart: no neighbours
    c[3:, 0] = [0, 0, -2.0]
    nrm, gap, ori, cnt = orc.normals(c, 0.025)
    assert (cnt == 0).all()
    assert np.allclose(nrm[0], [0, 0, -1.0])
    n_in = c[3:, 1].astype(np.float64)
    assert np.allclose(nrm[1], n_in / np.linalg.norm(n_in), atol=1e-15)
    # orientation follows the input normal
    d = _plane_cloud(2000, 2)
    d[5] = -1.0
    nrm, *_ = orc.normals(d, 0.025)
    assert (nrm[:, 2] < 0).all()


def test_normals_equal_library_eigensolver(orc):
    """Jacobi eigenvector equals numpy's symmetric eigensolver on the same
    neighbourhood covariance (special case reducing to a library routine)."""
    rng = np.random.default_rng(5)
    x = rng.normal(0, 1, (3, 600)) * np.array([[0.02], [0.01], [0.003]])
    c = np.concatenate([x, np.tile([[0.0], [0.0], [1.0]], (1, 600))]).astype(np.float32)
    nrm, gap, ori, cnt = orc.normals(c, 0.02)
    off, idx = orc.neighbors(c[:3], 0.02)
    for i in range(0, 600, 37):
        s = np.sort(np.append(idx[off[i]:off[i + 1]], i))
        if len(s) < 3:
            continue
        p = c[:3, s].astype(np.float64).T
        C = np.cov(p.T, bias=True)
        w, V = np.linalg.eigh(C)
        v = V[:, 0] * np.sign(V[2, 0])
        assert np.abs(np.abs(nrm[i] @ v) - 1) < 1e-12


def test_normals_rotation_covariant(orc):
    rng = np.random.default_rng(7)
    n = 3000
    u, v = rng.uniform(-0.2, 0.2, (2, n))
    z = 0.5 * (u ** 2 - 0.7 * v ** 2) + rng.normal(0, 0.001, n)
    x = np.stack([u, v, z])
    nin = np.tile([[0.0], [0.0], [1.0]], (1, n))
    c = np.concatenate([x, nin]).astype(np.float32)
    # exact rotation: a signed axis permutation keeps float32 coordinates exact
    R = np.array([[0, -1, 0], [0, 0, 1], [-1, 0, 0]], float)
    cr = np.concatenate([R @ c[:3].astype(float), R @ c[3:].astype(float)]).astype(np.float32)
    n1, *_ = orc.normals(c, 0.025)
    n2, *_ = orc.normals(cr, 0.025)
    assert np.abs(n1 @ R.T - n2).max() <= 1e-12


def test_normals_sphere_radial(orc):
    rng = np.random.default_rng(9)
    g = rng.normal(size=(3, 8000))
    g /= np.linalg.norm(g, axis=0)
    R = 0.3
    c = np.concatenate([R * g, g]).astype(np.float32)
    nrm, gap, ori, cnt = orc.normals(c, 0.03)
    cosang = np.sum(nrm * g.T, axis=1)
    ang = np.degrees(np.arccos(np.clip(cosang, -1, 1)))
    assert ang.mean() < 1.0 and ang.max() < 6.0


# ---------------------------------------------------------------- SPFH / FPFH

def test_spfh_hand_example(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "spfh_pair_30deg.txt")) if not l.startswith("#")]
    b = np.deg2rad(30.0)
    xyz = np.array([[0, 0.01], [0, 0], [0, 0]], np.float32)
    nrm = np.array([[0, 0, 1.0], [np.sin(b), 0, np.cos(b)]])
    S, k, kp, mg = orc.spfh(xyz, nrm, 0.05)
    for r in rows:
        i = int(r[0])
        want = np.zeros(33)
        want[[int(t) for t in r[1:]]] = 1.0
        assert np.array_equal(S[i], want)
    assert (k == 1).all() and (kp == 1).all()


def _star_4pt():
    xyz = np.array([[0, 1 / 64, 0, -13 / 512], [0, 0, 3 / 128, 0], [0, 0, 0, 0]], np.float32)
    nrm = np.array([[0, 0, 1.0], [0.6, 0, 0.8], [0, 0.8, 0.6], [1.0, 0, 0]])
    return xyz, nrm, 0.027


def test_fpfh_hand_example(orc):
    """Four-point star with unequal distances, unequal neighbour SPFHs and one
    skipped pair (k_A = 3 neighbours, 2 counted pairs): the hand-derived FPFH
    of tests/golden/fpfh_star_4pt.txt."""
    from fractions import Fraction
    rows = [l.split() for l in open(os.path.join(GOLD, "fpfh_star_4pt.txt")) if not l.startswith("#")]
    xyz, nrm, r = _star_4pt()
    want = np.zeros((4, 33))
    for i, c, v in rows:
        want[int(i), int(c)] = float(Fraction(v))
    S, k, kp, _ = orc.spfh(xyz, nrm, r)
    assert list(k) == [3, 1, 1, 1] and list(kp) == [2, 1, 1, 0]
    F, valid, _, _ = orc.fpfh(xyz, nrm, r)
    assert valid.all()
    assert np.abs(F - want).max() <= 1e-14


def test_fpfh_plane_indicator(orc):
    c = _plane_cloud(4000, 11)
    nrm = np.tile([0, 0, 1.0], (4000, 1))
    F, valid, sm, dm = orc.fpfh(c[:3], nrm, 0.05)
    want = np.zeros(33)
    want[[5, 16, 27]] = 1.0
    assert valid.all()
    assert np.array_equal(F, np.tile(want, (4000, 1)))


def test_spfh_sphere_closed_form(orc):
    """On a sphere with exact radial normals every pair has alpha = 0,
    phi = -d/(2R), theta = -2 asin(d/(2R)) for chord d (n_t = u + (d/R) e),
    so the histogram follows from the chord lengths alone."""
    rng = np.random.default_rng(13)
    g = rng.normal(size=(3, 1200))
    g /= np.linalg.norm(g, axis=0)
    Rs = 0.05
    xyz = (Rs * g).astype(np.float32)
    nrm = xyz.astype(np.float64).T / np.linalg.norm(xyz.astype(np.float64), axis=0)[:, None]
    rf = 0.02
    S, k, kp, mg = orc.spfh(xyz, nrm, rf)
    off, idx = orc.neighbors(xyz, rf, brute=True)
    P = xyz.astype(np.float64)
    checked = 0
    for i in range(0, 1200, 7):
        js = idx[off[i]:off[i + 1]]
        if len(js) == 0:
            continue
        d = np.linalg.norm(P[:, js] - P[:, [i]], axis=0)
        phi = -d / (2 * Rs)
        th = -2 * np.arcsin(d / (2 * Rs))
        xp = 11 * (phi + 1) / 2
        xt = 11 * (th + np.pi) / (2 * np.pi)
        if min(np.abs(xp - np.round(xp)).min(), np.abs(xt - np.round(xt)).min()) < 1e-6:
            continue                                   # too close to a bin edge to pin
        want = np.zeros(33)
        want[5] = 1.0
        np.add.at(want, 11 + np.floor(xp).astype(int), 1.0 / len(js))
        np.add.at(want, 22 + np.floor(xt).astype(int), 1.0 / len(js))
        assert np.allclose(S[i], want, atol=1e-12), i
        checked += 1
    assert checked > 100


def _rich_patch(n, seed):
    rng = np.random.default_rng(seed)
    u, v = rng.uniform(-0.15, 0.15, (2, n))
    z = 0.8 * u * v + 0.5 * u ** 2 + 0.03 * np.sin(40 * v) + rng.normal(0, 0.0005, n)
    nin = np.stack([-(0.8 * v + u), -(0.8 * u + 1.2 * np.cos(40 * v)), np.ones(n)])
    return np.concatenate([np.stack([u, v, z]), nin / np.linalg.norm(nin, axis=0)]).astype(np.float32)


def test_fpfh_rigid_invariance(orc):
    c = _rich_patch(4000, 17)
    R = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float)          # exact in float32
    cr = np.concatenate([R @ c[:3].astype(float), R @ c[3:].astype(float)]).astype(np.float32)
    n1, *_ = orc.normals(c, 0.025)
    n2, *_ = orc.normals(cr, 0.025)
    F1, v1, _, m1 = orc.fpfh(c[:3], n1, 0.05)
    F2, v2, _, m2 = orc.fpfh(cr[:3], n2, 0.05)
    safe = (m1 > 1e-9) & (m2 > 1e-9)
    assert safe.mean() > 0.9 and np.array_equal(v1, v2)
    assert np.abs(F1[safe] - F2[safe]).max() < 1e-12
    # a generic motion changes float32 inputs by rounding only
    ang = 0.7
    Rg = np.array([[np.cos(ang), -np.sin(ang), 0], [np.sin(ang), np.cos(ang), 0], [0, 0, 1]]) @ \
        np.array([[1, 0, 0], [0, np.cos(0.4), -np.sin(0.4)], [0, np.sin(0.4), np.cos(0.4)]])
    t = np.array([[0.5], [-0.25], [2.0]])
    cg = np.concatenate([Rg @ c[:3].astype(float) + t, Rg @ c[3:].astype(float)]).astype(np.float32)
    n3, *_ = orc.normals(cg, 0.025)
    F3, v3, _, m3 = orc.fpfh(cg[:3], n3, 0.05)
    same = (np.abs(F1 - F3).max(1) < 1e-3)
    assert same.mean() > 0.9


def test_fpfh_permutation_invariance(orc):
    c = _rich_patch(3000, 19)
    perm = np.random.default_rng(0).permutation(3000)
    n1, *_ = orc.normals(c, 0.025)
    n2, *_ = orc.normals(c[:, perm], 0.025)
    F1, v1, _, m1 = orc.fpfh(c[:3], n1, 0.05)
    F2, v2, _, m2 = orc.fpfh(c[:3, perm], n2, 0.05)
    assert np.abs(n1[perm] - n2).max() < 1e-12
    assert np.abs(F1[perm] - F2).max() < 1e-12 and np.array_equal(v1[perm], v2)


def test_fpfh_invalid_isolated_point(orc):
    c = _plane_cloud(500, 23)
    c[:3, 0] = [5.0, 5.0, 5.0]
    nrm = np.tile([0, 0, 1.0], (500, 1))
    F, valid, _, _ = orc.fpfh(c[:3], nrm, 0.05)
    assert valid[0] == 0 and not F[0].any()
    assert valid[1:].all()
    sums = F[1:].reshape(-1, 3, 11).sum(2)
    assert np.allclose(sums, 1.0, atol=1e-14)
