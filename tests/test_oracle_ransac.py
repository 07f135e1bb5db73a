"""Pins of the oracle's RANSAC consensus (Section IV, Algorithm 1: random
4-point hypotheses from P through the one-directional feature cache,
similar-polygon pre-rejection, rigid fit, inlier ratio and fitness on Q's
grid, the best hypothesis) and of its least-squares rigid fit."""
import numpy as np
import pytest

from test_oracle_match import _drawn_quads


def _rot(rng, ang=None):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    th = rng.uniform(0.1, 3.0) if ang is None else ang
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K


def _kabsch(p, q):
    """Least-squares rigid transform by SVD of the cross-covariance (Kabsch /
    Umeyama without scale), an independent route to the same optimum."""
    pm, qm = p.mean(0), q.mean(0)
    U, _, Vt = np.linalg.svd((p - pm).T @ (q - qm))
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = qm - R @ pm
    return T


def test_rigid_fit_exact_and_least_squares(orc):
    rng = np.random.default_rng(40)
    for k in range(20):
        R = _rot(rng)
        t = rng.uniform(-2, 2, 3)
        p = rng.uniform(-1, 1, (4 if k % 2 else 30, 3))
        ok, T = orc.rigid_fit(p, p @ R.T + t)                  # exact pairs: the transform itself
        assert ok and np.abs(T[:3, :3] - R).max() < 1e-12 and np.abs(T[:3, 3] - t).max() < 1e-12
        q = p @ R.T + t + rng.normal(0, 0.05, p.shape)         # noisy pairs: the SVD optimum
        ok, T = orc.rigid_fit(p, q)
        assert ok and np.abs(T - _kabsch(p, q)).max() < 1e-11
        assert abs(np.linalg.det(T[:3, :3]) - 1) < 1e-12


def test_rigid_fit_degenerate(orc):
    p = np.linspace(0, 1, 4)[:, None] * np.array([[1.0, 2.0, 0.5]])   # collinear: rotation about the line free
    ok, T = orc.rigid_fit(p, p + 0.3)
    assert not ok and np.array_equal(T, np.eye(4))
    ok, _ = orc.rigid_fit(np.zeros((4, 3)), np.ones((4, 3)))
    assert not ok


def _brute_ransac(P, Q, nP_, nQ_, nnQ, n_hyp, tau, seed, delta, normal_check, cth, orc):
    """Every step by hand: reconstructed draws (eligible = has a cached
    neighbour), polygon test, SVD fit, exhaustive nearest neighbours, the
    tie rule."""
    Pd, Qd = P[:3].astype(np.float64), Q[:3].astype(np.float64)
    t2 = float(np.float64(np.float32(tau)) ** 2)
    d2max = float(np.float64(np.float32(delta)) ** 2)
    best = None
    surv = 0
    for t, qd in enumerate(_drawn_quads(orc, P.shape[1], nnQ >= 0, n_hyp, seed)):
        if qd is None:
            continue
        good = True
        for k in range(4):
            a, b = qd[k], qd[(k + 1) % 4]
            ea = np.sum((Pd[:, a] - Pd[:, b]) ** 2)
            eb = np.sum((Qd[:, nnQ[a]] - Qd[:, nnQ[b]]) ** 2)
            if ea == 0 or eb == 0 or ea < t2 * eb or eb < t2 * ea:
                good = False
        if not good:
            continue
        surv += 1
        T = _kabsch(Pd[:, qd].T, Qd[:, nnQ[qd]].T)
        tp = T[:3, :3] @ Pd + T[:3, 3:4]
        d2 = ((tp[:, :, None] - Qd[:, None, :]) ** 2).sum(0)
        if normal_check:
            agree = (nP_ @ T[:3, :3].T) @ nQ_.T >= np.float64(np.float32(cth))
            d2 = np.where(agree, d2, np.inf)
        dmin = d2.min(1)
        inl = dmin <= d2max
        key = (-int(inl.sum()), float(dmin[inl].sum()), t)
        if best is None or key < best[0]:
            best = (key, T)
    return best, surv


@pytest.mark.parametrize("normal_check", [0, 1])
def test_ransac_equals_brute_force(orc, normal_check):
    rng = np.random.default_rng(41 + normal_check)
    n = 160
    P = np.vstack([rng.uniform(0, 0.5, (3, n)), rng.normal(size=(3, n))]).astype(np.float32)
    P[3:] /= np.linalg.norm(P[3:], axis=0)
    R = _rot(rng, 0.7)
    t = np.array([0.1, -0.05, 0.2])
    Q = np.vstack([R @ P[:3] + t[:, None] + rng.normal(0, 0.002, (3, n)), R @ P[3:]]).astype(np.float32)
    nnQ = np.arange(n, dtype=np.int32)
    wrong = rng.random(n) < 0.6
    nnQ[wrong] = rng.integers(0, n, wrong.sum())
    nnQ[rng.random(n) < 0.1] = -1                              # points without a descriptor
    nP_, nQ_ = P[3:].T.astype(np.float64), Q[3:].T.astype(np.float64)
    st, T, info = orc.ransac(P, nP_, Q, nQ_, nnQ, 400, seed=5, delta=0.01, normal_check=normal_check)
    (key, Tb), surv = _brute_ransac(P, Q, nP_, nQ_, nnQ, 400, 0.9, 5, 0.01, normal_check, 0.8660254, orc)
    assert info["n_survivors"] == surv and info["n_fitted"] == surv
    assert info["best"] == key[2] and info["n_inliers"] == -key[0]
    assert abs(info["sum_d2"] - key[1]) <= 1e-12 * max(key[1], 1e-30)
    assert np.abs(T - Tb).max() < 1e-10
    assert info["n_inliers"] > 0.8 * n and np.abs(T[:3, :3] - R).max() < 0.02    # the consensus is the truth
    assert st == orc.ACCEPTED and abs(info["ratio"] - info["n_inliers"] / n) < 1e-15


def test_ransac_survivors_are_the_polygon_test(orc):
    """With every point eligible for both (a cached neighbour and a reciprocal
    one), the hypotheses are the consistency filter's trials: the survivors
    are exactly its passing trials."""
    rng = np.random.default_rng(43)
    n = 300
    P = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    Q = (P * 1.02 + rng.normal(0, 0.02, (3, n))).astype(np.float32)
    nnQ = rng.permutation(n).astype(np.int32)
    nnQ[: n // 2] = np.arange(n // 2)
    _, passed = orc.consistency(P, Q, nnQ, np.ones(n, bool), 5000, 0.9, 77)
    _, _, info = orc.ransac(P, None, Q, None, nnQ, 5000, seed=77, delta=0.02, normal_check=0)
    assert info["n_survivors"] == passed > 0


def test_ransac_no_survivor_is_degenerate(orc):
    rng = np.random.default_rng(44)
    P = rng.uniform(-1, 1, (3, 50)).astype(np.float32)
    st, T, info = orc.ransac(P, None, (2 * P).astype(np.float32), None, np.arange(50, dtype=np.int32), 300,
                             normal_check=0)
    assert st == orc.DEGENERATE and info["best"] == -1 and np.array_equal(T, np.eye(4))
