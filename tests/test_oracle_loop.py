"""Pins of the oracle's loop verification (Sec. V, eqs. 2-5) against facts
outside its code: edge information against a k-d tree's inlier set and the
second-moment form of sum G^T G; consistent measurements leave the poses and
l = 1; the one-dimensional case against a brute-force minimisation; the
returned poses are a stationary point of E (central differences of an
energy written here with scipy's rotation logarithm); covariance under a
change of world frame; true loops of the chain recipe accepted, false ones
rejected; degenerate and empty cases."""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

import oracle
from synth.chain import make_chain


def _se3(w, v):
    T = np.eye(4)
    T[:3, :3] = Rotation.from_rotvec(w).as_matrix()
    T[:3, 3] = v
    return T


def _inv(T):
    o = np.eye(4)
    o[:3, :3] = T[:3, :3].T
    o[:3, 3] = -T[:3, :3].T @ T[:3, 3]
    return o


def _energy(T, odo, Lo, loop, Ll, lam, mu):
    """E(T) with l eliminated, from the definitions (scipy's SO(3) log)."""
    def f(i, j, A, L):
        D = _inv(A) @ _inv(T[j]) @ T[i]
        xi = np.concatenate([Rotation.from_matrix(D[:3, :3]).as_rotvec(), D[:3, 3]])
        return xi @ L @ xi
    E = sum(lam * f(i, j, A, L) for (i, j, A), L in zip(odo, Lo))
    fl = f(*loop, Ll)
    return E + mu * fl / (mu + fl), fl


@pytest.fixture(scope="module")
def chain():
    return make_chain(24, 3000, n_true=2, n_false=2)


@pytest.fixture(scope="module")
def infos(chain):
    Lo = [oracle.edge_info(chain.frags[i], chain.frags[j], A)[0] for (i, j, A) in chain.odo]
    return np.array(Lo)


def test_edge_info_against_kdtree_and_moments(chain):
    i, j, A = chain.odo[3]
    Pi, Pj = chain.frags[i][:3].astype(np.float64), chain.frags[j][:3].astype(np.float64)
    L, cnt = oracle.edge_info(chain.frags[i], chain.frags[j], A, eps=0.05)
    Ap = A[:3, :3] @ Pi + A[:3, 3:4]
    d, _ = cKDTree(Pj.T).query(Ap.T)
    near = np.abs(d - 0.05) < 1e-9
    assert near.sum() == 0
    inl = d <= 0.05
    assert cnt == inl.sum() > 100
    p = Pi[:, inl]
    M = p @ p.T
    s = p.sum(1)
    S = np.array([[0, -s[2], s[1]], [s[2], 0, -s[0]], [-s[1], s[0], 0]])
    want = np.block([[np.trace(M) * np.eye(3) - M, S], [-S, cnt * np.eye(3)]])
    assert np.allclose(L, want, rtol=1e-12, atol=1e-9 * np.abs(want).max())


def test_consistent_measurements_keep_the_poses(chain, infos):
    T = chain.T_true
    odo = [(i, j, _inv(T[j]) @ T[i]) for (i, j, _) in chain.odo]
    i, j = chain.loops[0][:2]
    loop = (i, j, _inv(T[j]) @ T[i])
    r, To = oracle.loop_solve(T, odo, infos, loop, infos[0], 1000)
    assert r["l"] == 1.0 and r["f_loop"] < 1e-20 and r["status"] == oracle.ACCEPTED
    assert np.abs(To - T).max() < 1e-12


def test_one_dimensional_case_against_brute_force():
    c, d, lam, tau, cnt = 50.0, 0.3, 1000.0, 0.2, 200
    L = c * np.eye(6)
    T0 = np.eye(4)
    odo = [(0, 1, np.eye(4))]
    loop = (0, 1, _se3([0, 0, 0], [d, 0, 0]))
    prm = oracle.loop_params(lambda_=lam, tau=tau)
    r, To = oracle.loop_solve(np.stack([T0, T0]), odo, L[None], loop, L, cnt, prm)
    mu = tau * tau * cnt
    # T_1 = translation u along x: f_odo = c u^2, f_loop = c (u + d)^2
    E = lambda u: lam * c * u * u + mu * c * (u + d) ** 2 / (mu + c * (u + d) ** 2)
    u = minimize_scalar(E, bounds=(-1, 1), method="bounded", options={"xatol": 1e-14}).x
    assert abs(To[1][0, 3] - u) < 1e-9
    assert np.abs(To[1][:3, :3] - np.eye(3)).max() < 1e-12 and abs(To[1][1, 3]) < 1e-12
    fl = c * (u + d) ** 2
    assert abs(r["l"] - (mu / (mu + fl)) ** 2) < 1e-9


@pytest.mark.parametrize("k", [0, 2])
def test_returned_poses_are_stationary(chain, infos, k):
    i, j, A = chain.loops[k]
    Ll, cnt = oracle.edge_info(chain.frags[i], chain.frags[j], A)
    prm = oracle.loop_params()
    r, To = oracle.loop_solve(chain.T_init, chain.odo, infos, (i, j, A), Ll, cnt, prm)
    mu = prm.tau ** 2 * cnt
    E0, _ = _energy(chain.T_init, chain.odo, infos, (i, j, A), Ll, prm.lambda_, mu)
    E1, fl = _energy(To, chain.odo, infos, (i, j, A), Ll, prm.lambda_, mu)
    assert E1 <= E0 and abs(E1 - r["energy"]) <= 1e-9 * (1 + E1) and abs(fl - r["f_loop"]) <= 1e-9 * (1 + fl)
    h = 1e-6
    g = []
    for node in range(1, len(To)):
        for a in range(6):
            e = np.zeros(6)
            e[a] = h
            Tp, Tm = To.copy(), To.copy()
            Tp[node] = _se3(e[:3], e[3:]) @ To[node]
            Tm[node] = _se3(-e[:3], -e[3:]) @ To[node]
            g.append((_energy(Tp, chain.odo, infos, (i, j, A), Ll, prm.lambda_, mu)[0]
                      - _energy(Tm, chain.odo, infos, (i, j, A), Ll, prm.lambda_, mu)[0]) / (2 * h))
    g0 = []
    for a in range(6):          # gradient scale: the first free node at the initial poses
        e = np.zeros(6)
        e[a] = h
        Tp, Tm = chain.T_init.copy(), chain.T_init.copy()
        Tp[1] = _se3(e[:3], e[3:]) @ Tp[1]
        Tm[1] = _se3(-e[:3], -e[3:]) @ Tm[1]
        g0.append((_energy(Tp, chain.odo, infos, (i, j, A), Ll, prm.lambda_, mu)[0]
                   - _energy(Tm, chain.odo, infos, (i, j, A), Ll, prm.lambda_, mu)[0]) / (2 * h))
    assert np.abs(g).max() <= 1e-5 * max(1.0, np.abs(g0).max())


def test_change_of_world_frame_is_covariant(chain, infos):
    i, j, A = chain.loops[1]
    Ll, cnt = oracle.edge_info(chain.frags[i], chain.frags[j], A)
    W = _se3([0.3, -0.2, 1.0], [1.0, 2.0, -0.5])
    r1, T1 = oracle.loop_solve(chain.T_init, chain.odo, infos, (i, j, A), Ll, cnt)
    r2, T2 = oracle.loop_solve(np.einsum("ij,njk->nik", W, chain.T_init), chain.odo, infos, (i, j, A), Ll, cnt)
    assert abs(r1["l"] - r2["l"]) < 1e-9 and r1["status"] == r2["status"]
    assert np.abs(np.einsum("ij,njk->nik", W, T1) - T2).max() < 1e-8


def test_true_loops_accepted_false_rejected(chain, infos):
    for (i, j, A), truth in zip(chain.loops, chain.loop_true):
        Ll, cnt = oracle.edge_info(chain.frags[i], chain.frags[j], A)
        r, _ = oracle.loop_solve(chain.T_init, chain.odo, infos, (i, j, A), Ll, cnt)
        assert cnt > 0
        assert r["status"] == (oracle.ACCEPTED if truth else oracle.REJECTED), (i, j, truth, r)


def test_degenerate_and_empty(chain, infos):
    i, j, A = chain.loops[0]
    Ll, cnt = oracle.edge_info(chain.frags[i], chain.frags[j], A)
    r, To = oracle.loop_solve(chain.T_init, chain.odo, infos, (i, j, A), Ll, 0)
    assert r["status"] == oracle.REJECTED and r["l"] == 0 and r["iters"] == 0
    assert np.array_equal(To, chain.T_init)
    Lz = infos.copy()
    Lz[-1] = 0                # the last odometry edge without correspondences: its node is unconstrained
    r, _ = oracle.loop_solve(chain.T_init, chain.odo, Lz, (i, j, A), Ll, cnt)
    assert r["status"] == oracle.DEGENERATE
