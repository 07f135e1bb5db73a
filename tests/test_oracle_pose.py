"""Pins of the oracle's robust pose solve (line-process energy of eqs. 2-5
restricted to one fragment pair, graduated non-convexity), verification, the
alignment-energy adjoint, and end-to-end recovery of a known transform."""
import numpy as np
import pytest


def _rigid(rng, ang=0.8, trans=0.5):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    th = rng.uniform(0.1, ang)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    T[:3, 3] = rng.uniform(-trans, trans, 3)
    return T


def _rot_err_deg(A, B):
    R = A[:3, :3].T @ B[:3, :3]
    return np.degrees(np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1)))


def _umeyama(p, q, w=None):
    """Weighted least-squares rigid fit (Horn 1987 / Umeyama 1991) via SVD."""
    w = np.ones(len(p)) if w is None else w
    mp, mq = (w[:, None] * p).sum(0) / w.sum(), (w[:, None] * q).sum(0) / w.sum()
    H = ((p - mp) * w[:, None]).T @ (q - mq)
    U, S, Vt = np.linalg.svd(H)
    D = np.diag([1, 1, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    return R, mq - R @ mp


def test_gnc_exact_correspondences(orc):
    rng = np.random.default_rng(0)
    T = _rigid(rng)
    p = rng.uniform(-1, 1, (500, 3))
    q = p @ T[:3, :3].T + T[:3, 3]
    st, Te, mu, E, it = orc.gnc(p, q)
    assert st == orc.ACCEPTED
    assert np.abs(Te - T).max() <= 1e-12
    R = Te[:3, :3]
    assert abs(np.linalg.det(R) - 1) <= 1e-12 and np.linalg.norm(R.T @ R - np.eye(3)) <= 1e-12


def test_gnc_least_squares_limit_is_umeyama(orc):
    """mu -> infinity makes every weight l -> 1: the fixed point is the
    least-squares rigid fit."""
    rng = np.random.default_rng(1)
    T = _rigid(rng)
    p = rng.uniform(-1, 1, (300, 3))
    q = p @ T[:3, :3].T + T[:3, 3] + rng.normal(0, 0.05, (300, 3))
    prm = orc.default_params(max_corr=1.0e6, polish_iter=64)
    st, Te, mu, E, it = orc.gnc(p, q, prm)
    R, t = _umeyama(p, q)
    assert st == orc.ACCEPTED
    assert np.abs(Te[:3, :3] - R).max() <= 1e-12 and np.abs(Te[:3, 3] - t).max() <= 1e-12


def test_gnc_outliers_and_stationarity(orc):
    rng = np.random.default_rng(2)
    T = _rigid(rng)
    n = 2000
    p = rng.uniform(-1.5, 1.5, (n, 3))
    q = p @ T[:3, :3].T + T[:3, 3] + rng.normal(0, 0.003, (n, 3))
    out = rng.random(n) < 0.5
    q[out] = rng.uniform(-2, 2, (out.sum(), 3))
    prm = orc.default_params(max_corr=0.015)
    st, Te, mu, E, it = orc.gnc(p, q, prm)
    assert st == orc.ACCEPTED
    assert _rot_err_deg(Te, T) < 0.05 and np.linalg.norm(Te[:3, 3] - T[:3, 3]) < 0.003
    E2, dp, dq, dxi = orc.align_loss(p, q, Te, mu)
    assert abs(E2 - E) <= 1e-12 * (1 + E)
    assert np.abs(dxi).max() <= 1e-9 * (1 + E)             # stationary point of E_mu
    # the inlier-weighted least-squares fit agrees with the robust solution
    l = (mu / (mu + np.sum((p @ Te[:3, :3].T + Te[:3, 3] - q) ** 2, 1))) ** 2
    R, t = _umeyama(p, q, l)
    assert np.abs(R - Te[:3, :3]).max() < 1e-10


def test_gnc_energy_monotone_within_fixed_mu(orc):
    """Within the polish phase (fixed mu) the robust energy never increases."""
    rng = np.random.default_rng(3)
    T = _rigid(rng)
    p = rng.uniform(-1, 1, (800, 3))
    q = p @ T[:3, :3].T + T[:3, 3] + rng.normal(0, 0.004, (800, 3))
    q[:300] = rng.uniform(-1.5, 1.5, (300, 3))
    energies = []
    for k in range(1, 8):
        prm = orc.default_params(max_corr=1.0e3, polish_iter=k)     # no annealing: mu fixed
        st, Te, mu, E, it = orc.gnc(p, q, prm)
        energies.append(E)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(energies, energies[1:]))


def test_gnc_degenerate(orc):
    p = np.zeros((2, 3))
    assert orc.gnc(p, p)[0] == orc.DEGENERATE
    s = np.linspace(0, 1, 50)[:, None] * np.array([[1.0, 2.0, 3.0]])     # collinear
    assert orc.gnc(s, s + 0.1)[0] == orc.DEGENERATE


def test_align_loss_gradients(orc):
    rng = np.random.default_rng(4)
    m = 40
    T = _rigid(rng)
    p = rng.uniform(-1, 1, (m, 3))
    q = p @ T[:3, :3].T + T[:3, 3] + rng.normal(0, 0.05, (m, 3))
    q[:10] += rng.normal(0, 0.5, (10, 3))
    mu = 0.02
    E, dp, dq, dxi = orc.align_loss(p, q, T, mu)
    h = 1e-4
    for arr, g in ((p, dp), (q, dq)):
        num = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            a1, a2 = arr.copy(), arr.copy()
            a1[idx] += h; a2[idx] -= h
            args1 = (a1, q) if arr is p else (p, a1)
            args2 = (a2, q) if arr is p else (p, a2)
            num[idx] = (orc.align_loss(*args1, T, mu, grad=False) - orc.align_loss(*args2, T, mu, grad=False)) / (2 * h)
        assert np.abs(num - g).max() <= 1e-6 * (1 + np.abs(g).max())
    for k in range(6):
        xi = np.zeros(6)
        xi[k] = h
        Ts = []
        for s in (1, -1):
            w = s * xi[:3]
            th = np.linalg.norm(w)
            K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
            Rd = np.eye(3) + (np.sin(th) / th if th else 1) * K + ((1 - np.cos(th)) / th ** 2 if th else .5) * K @ K
            D = np.eye(4)
            D[:3, :3] = Rd
            D[:3, 3] = s * xi[3:]
            Ts.append(D @ T)
        num = (orc.align_loss(p, q, Ts[0], mu, grad=False) - orc.align_loss(p, q, Ts[1], mu, grad=False)) / (2 * h)
        assert abs(num - dxi[k]) <= 1e-6 * (1 + np.abs(dxi).max())


def test_align_loss_closed_forms(orc):
    p = np.array([[0.1, 0.2, 0.3]])
    q = np.array([[0.4, -0.2, 0.3]])
    T = np.eye(4)
    mu = 0.5
    s = 0.3 ** 2 + 0.4 ** 2
    E, dp, dq, dxi = orc.align_loss(p, q, T, mu)
    assert abs(E - mu * s / (mu + s)) < 1e-15
    l = (mu / (mu + s)) ** 2
    r = p[0] - q[0]
    assert np.allclose(dp[0], 2 * l * r) and np.allclose(dq[0], -2 * l * r)
    assert np.allclose(dxi[3:], 2 * l * r) and np.allclose(dxi[:3], 2 * l * np.cross(p[0], r))
    # mu -> infinity: the least-squares gradient
    E, dp, dq, dxi = orc.align_loss(p, q, T, 1e12)
    assert np.allclose(dp[0], 2 * r, rtol=1e-9) and abs(E - s) < 1e-9


def test_verify_equals_brute_force(orc):
    rng = np.random.default_rng(6)
    P = rng.uniform(0, 0.3, (3, 1500)).astype(np.float32)
    Q = rng.uniform(0, 0.3, (3, 1800)).astype(np.float32)
    T = _rigid(rng, ang=0.2, trans=0.05)
    delta = 0.015
    ni, ratio, fit = orc.verify(P, None, Q, None, T, delta)
    tp = (T[:3, :3] @ P.astype(np.float64)) + T[:3, 3:4]
    d2 = ((tp[:, :, None] - Q.astype(np.float64)[:, None, :]) ** 2).sum(0).min(1)
    inl = d2 <= np.float64(np.float32(delta)) ** 2
    assert ni == inl.sum() and abs(ratio - inl.mean()) < 1e-15
    assert abs(fit - np.sqrt(d2[inl].mean())) < 1e-12


def test_verify_normal_check_equals_brute_force(orc):
    """Inlier with the normal check: the nearest q within delta among those
    whose normal agrees with R n_p (cosine >= the threshold).  Q is T P plus
    noise with normals R n_p, except a third of them flipped: with the check
    those points are outliers, without it inliers; a transposed rotation (large
    angle) rejects most points.  Random clouds and normals are checked the same
    way against brute force."""
    rng = np.random.default_rng(16)
    delta, cth = 0.006, 0.5
    a = np.array([1.0, -2.0, 0.5]) / np.linalg.norm([1.0, -2.0, 0.5])
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + np.sin(1.2) * K + (1 - np.cos(1.2)) * K @ K   # R^2 turns normals by 2.4 rad
    T[:3, 3] = [0.03, -0.02, 0.04]
    R = T[:3, :3]
    cases = []
    P = rng.uniform(0, 0.25, (3, 1200)).astype(np.float32)
    nP = rng.normal(size=(1200, 3)); nP /= np.linalg.norm(nP, axis=1, keepdims=True)
    Q = ((R @ P.astype(np.float64)) + T[:3, 3:4] + rng.normal(0, 0.001, (3, 1200))).astype(np.float32)
    nQ = nP @ R.T
    flip = rng.random(1200) < 1 / 3
    nQ[flip] *= -1
    cases.append((P, nP, Q, nQ, True))
    P2 = rng.uniform(0, 0.25, (3, 1000)).astype(np.float32)
    Q2 = rng.uniform(0, 0.25, (3, 2200)).astype(np.float32)
    n1 = rng.normal(size=(1000, 3)); n1 /= np.linalg.norm(n1, axis=1, keepdims=True)
    n2 = rng.normal(size=(2200, 3)); n2 /= np.linalg.norm(n2, axis=1, keepdims=True)
    cases.append((P2, n1, Q2, n2, False))
    d2max = np.float64(np.float32(delta)) ** 2
    for P, nP, Q, nQ, constructed in cases:
        ni, ratio, fit = orc.verify(P, nP, Q, nQ, T, delta, normal_check=1, normal_cos=cth)
        tp = (R @ P.astype(np.float64)) + T[:3, 3:4]
        d2 = ((tp[:, :, None] - Q.astype(np.float64)[:, None, :]) ** 2).sum(0)
        agree = (nP @ R.T) @ nQ.T >= np.float64(np.float32(cth))
        d2n = np.where(agree, d2, np.inf).min(1)
        inl = d2n <= d2max
        assert ni == inl.sum() and abs(ratio - inl.mean()) < 1e-15
        assert abs(fit - np.sqrt(d2n[inl].mean())) < 1e-12
        ni0, _, _ = orc.verify(P, nP, Q, nQ, T, delta, normal_check=0, normal_cos=cth)
        assert ni0 == (d2.min(1) <= d2max).sum()
        if constructed:
            wrongR = (np.where((nP @ R) @ nQ.T >= cth, d2, np.inf).min(1) <= d2max).sum()
            assert ni0 > 0.95 * len(flip) and abs(ni - (~flip).sum()) < 0.05 * len(flip) and wrongR < 0.8 * ni


def _copy_pair(seed, n=20000, sigma=0.001):
    """P: a rigidly moved, re-noised subset of Q's samples (a controlled case
    with exact underlying correspondences)."""
    from synth import scenes as S
    rng = np.random.default_rng([seed, 77])
    pr = S.make_pair(5, seed, n_points=n)
    Q = pr.Q.copy()
    sub = rng.permutation(Q.shape[1])[: int(0.7 * Q.shape[1])]
    B = Q[:, sub].astype(np.float64)
    T = _rigid(rng, ang=1.0)
    R, t = T[:3, :3], T[:3, 3:4]
    P = np.concatenate([R.T @ (B[:3] - t) + rng.normal(0, sigma, B[:3].shape), R.T @ B[3:]]).astype(np.float32)
    return P, Q, T


@pytest.mark.slow
def test_end_to_end_recovers_known_transform(orc):
    P, Q, T = _copy_pair(0)
    res, nnQ, cons = orc.register_pair(P, Q)
    d = orc.result_dict(res)
    assert d["status"] == orc.ACCEPTED
    assert _rot_err_deg(d["T"], T) < 0.5 and np.linalg.norm(d["T"][:3, 3] - T[:3, 3]) < 0.02
    R = d["T"][:3, :3]
    assert abs(np.linalg.det(R) - 1) < 1e-12


@pytest.mark.slow
def test_end_to_end_rejects_unrelated_clouds(orc):
    """Q is a different room: nothing can align, so the verdict is not accepted."""
    import synth
    a = synth.make_pair(4, 1, n_points=8000)
    b = synth.make_pair(0, 5, n_points=8000)
    res, _, _ = orc.register_pair(a.P, b.Q, orc.default_params(min_inlier_ratio=0.3))
    assert res.status != orc.ACCEPTED
