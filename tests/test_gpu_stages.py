"""Stage-by-stage parity of the HIP path against the CPU FP64 oracle, each
stage fed the oracle's own inputs for that stage.  Calls go through the C ABI
(paper_1801_01572_amd -> liblsr.so)."""
import numpy as np
import pytest
import torch

from gpu_helpers import DESC_RTOL, MARGIN, NORMAL_TOL, desc_exempt, dev, pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_1801_01572_amd as lsr
    lsr.lib()
    return lsr


CASES = [(0, 0, None), (4, 1, 12000), (1, 2, 9000)]


@pytest.mark.parametrize("cfg,idx,n", CASES)
def test_normals_parity(L, orc, cfg, idx, n):
    pr = pair(cfg, idx, n)
    print(f"normals cfg={cfg} idx={idx} n={pr.P.shape[1]}", flush=True)
    for cloud in (pr.P, pr.Q):
        want, gap, ori, cnt = orc.normals(cloud, 0.025)
        got = L.stage_normals(dev(cloud), 0.025).cpu().numpy()
        torch.cuda.synchronize()
        ok = ((gap < 0) | (gap > 1e-7)) & (ori > 1e-9)
        assert ok.mean() > 0.999
        err = np.abs(got - want).max(1)
        assert err[ok].max() <= NORMAL_TOL, err[ok].max()
        fb = gap < 0                                   # fewer than 3 points: normalised input normal
        assert np.abs(got[fb] - want[fb]).max(initial=0.0) <= 1e-15


@pytest.mark.parametrize("cfg,idx,n", CASES)
def test_spfh_parity(L, orc, cfg, idx, n):
    """Neighbour counts exact; histograms equal except at points with a
    decision within the margin of its boundary."""
    pr = pair(cfg, idx, n)
    for cloud in (pr.P, pr.Q):
        nrm, *_ = orc.normals(cloud, 0.025)
        S, k, kp, mg = orc.spfh(cloud[:3], nrm, 0.05)
        Sg, kg = L.stage_spfh(dev(cloud[:3]), dev(nrm), 0.05)
        Sg, kg = Sg.cpu().numpy(), kg.cpu().numpy()
        assert np.array_equal(kg, k)
        keep = mg >= MARGIN
        assert keep.mean() > (0.99 if cfg == 0 else 0.9999)
        assert np.abs(Sg[keep] - S[keep]).max() <= 1e-6


@pytest.mark.parametrize("cfg,idx,n", CASES)
def test_fpfh_parity(L, orc, cfg, idx, n):
    pr = pair(cfg, idx, n)
    print(f"fpfh cfg={cfg} idx={idx} n={pr.P.shape[1]}", flush=True)
    for cloud in (pr.P, pr.Q):
        nrm, gap, ori, _ = orc.normals(cloud, 0.025)
        F, v, exempt = desc_exempt(orc, cloud, nrm, gap, ori, 0.05)
        Fg, vg = L.stage_fpfh(dev(cloud[:3]), dev(nrm), 0.05)
        Fg, vg = Fg.cpu().numpy().astype(np.float64), vg.cpu().numpy()
        assert np.array_equal(vg, v)
        keep = (v == 1) & ~exempt
        # sparse clouds (5k points) hold 3-point neighbourhoods whose PCA planes share an edge: the
        # source choice of such a pair is decided by rounding, and the oracle flags it
        assert keep.mean() > (0.9 if cfg == 0 else 0.99)
        rel = np.linalg.norm(Fg[keep] - F[keep], axis=1) / np.linalg.norm(F[keep], axis=1)
        print(f"  max rel {rel.max():.2e}  exempt {exempt.sum()}", flush=True)
        assert rel.max() <= DESC_RTOL


def _oracle_descriptors(orc, pr):
    out = []
    for cloud in (pr.P, pr.Q):
        nrm, *_ = orc.normals(cloud, 0.025)
        F, v, _, _ = orc.fpfh(cloud[:3], nrm, 0.05)
        out += [F, v]
    return out


@pytest.mark.parametrize("cfg,idx,n", CASES)
def test_match_parity_fp32_and_bf16(L, orc, cfg, idx, n):
    """Injected oracle descriptors (rounded to float32): indices equal the
    oracle's outside the near-tie margin; the bf16 screen returns the float32
    scan's bits exactly."""
    pr = pair(cfg, idx, n)
    print(f"match cfg={cfg} idx={idx} n={pr.P.shape[1]}", flush=True)
    F, vF, G, vG = _oracle_descriptors(orc, pr)
    m = orc.match(F, vF, G, vG)
    tP, tQ = orc.tie_flags(F, G, m)
    args = (dev(F.astype(np.float32)), dev(vF), dev(G.astype(np.float32)), dev(vG))
    nnQ, dQ, nnP, dP, _ = [t.cpu().numpy() for t in L.stage_match(*args, precision=L.FP32)]
    okP, okQ = ~tP, ~tQ
    assert np.array_equal(nnQ[okP], m["nnQ"][okP])
    assert np.array_equal(nnP[okQ], m["nnP"][okQ])
    print(f"  tie-exempt rows {tP.mean():.4f}, exempt rows that still agree "
          f"{(nnQ[tP] == m['nnQ'][tP]).mean() if tP.any() else 1.0:.3f}", flush=True)
    b = [t.cpu().numpy() for t in L.stage_match(*args, precision=L.BF16_SCREEN)]
    assert np.array_equal(b[0], nnQ) and np.array_equal(b[2], nnP)
    assert np.array_equal(b[1].view(np.uint32), dQ.view(np.uint32))
    assert np.array_equal(b[3].view(np.uint32), dP.view(np.uint32))
    print(f"  bf16 fallback rows {int(b[4][0])} of {len(nnQ) + len(nnP)}", flush=True)


def test_match_bf16_random_and_edge_sizes(L):
    """bf16 screen == float32 scan on random descriptors, ragged sizes,
    invalid rows, exact duplicates (ties) and an empty side."""
    rng = np.random.default_rng(0)
    for nP, nQ in [(1, 1), (17, 300), (1000, 129), (4099, 2500), (0, 50), (60, 0)]:
        def desc(n):
            x = rng.random((n, 33)) ** 4
            x = x.reshape(n, 3, 11)
            x /= x.sum(2, keepdims=True)
            return x.reshape(n, 33).astype(np.float32)
        F, G = desc(nP), desc(nQ)
        if nP > 10 and nQ > 10:
            G[:5] = F[:5]
            G[5] = G[6]
        vF = (rng.random(nP) > 0.05).astype(np.int32)
        vG = (rng.random(nQ) > 0.05).astype(np.int32)
        args = (dev(F), dev(vF), dev(G), dev(vG))
        a = [t.cpu().numpy() for t in L.stage_match(*args, precision=L.FP32)]
        try:
            for shape in range(L.get_tune()["n_screen_shapes"]):      # every screen tiling the autotuner may pick
                L.set_tune(shape, 0)
                b = [t.cpu().numpy() for t in L.stage_match(*args, precision=L.BF16_SCREEN)]
                for k in range(4):
                    assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), (nP, nQ, shape, k)
        finally:
            L.set_tune(0, 0)
        # float32 scan == brute force in numpy's float64 on non-tied rows
        if nP and nQ:
            D = ((F[:, None, :].astype(np.float64) - G[None].astype(np.float64)) ** 2).sum(2)
            D[:, vG == 0] = np.inf
            srt = np.sort(np.concatenate([D, np.full((nP, 1), np.inf)], 1), 1)
            clear = (vF == 1) & (srt[:, 1] - srt[:, 0] > 1e-5) & np.isfinite(srt[:, 0])
            assert np.array_equal(a[0][clear], np.argmin(D, 1)[clear])
            assert (a[0][vF == 0] == -1).all()


def test_match_bf16_ties_and_extremes(L):
    """bf16 screen == float32 scan where the screen's certificate is hardest:
    1500 identical rows (every query ties with all of them, so the collected
    lists overflow and rows fall back to the float32 rescan), near-duplicates
    differing below bf16 resolution, and one-hot against uniform histograms
    (extreme norms after centring)."""
    rng = np.random.default_rng(5)

    def norm(x):
        x = x.reshape(len(x), 3, 11)
        x = x / x.sum(2, keepdims=True)
        return x.reshape(len(x), 33).astype(np.float32)

    base = norm(rng.random((1, 33)) ** 3)
    G = np.concatenate([np.repeat(base, 1500, 0),
                        norm(rng.random((300, 33)) ** 4),
                        norm(np.eye(11)[rng.integers(0, 11, (200, 3))].reshape(200, 33) + 1e-7),
                        norm(np.ones((20, 33)))])
    near = np.repeat(base, 400, 0) * (1 + rng.normal(scale=2e-4, size=(400, 33)).astype(np.float32))
    F = np.concatenate([np.repeat(base, 50, 0), norm(near), norm(rng.random((300, 33)) ** 4),
                        norm(np.eye(11)[rng.integers(0, 11, (100, 3))].reshape(100, 33) + 1e-7),
                        norm(np.ones((5, 33)))])
    vF = np.ones(len(F), np.int32)
    vG = np.ones(len(G), np.int32)
    print(f"ties nP={len(F)} nQ={len(G)}", flush=True)
    args = (dev(F), dev(vF), dev(G), dev(vG))
    a = [t.cpu().numpy() for t in L.stage_match(*args, precision=L.FP32)]
    try:
        for shape in range(L.get_tune()["n_screen_shapes"]):
            L.set_tune(shape, 0)
            b = [t.cpu().numpy() for t in L.stage_match(*args, precision=L.BF16_SCREEN)]
            for k in range(4):
                assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), (shape, k)
            print(f"  shape {shape}: {int(b[4][0])} rows rescanned in float32", flush=True)
            assert int(b[4][0]) >= 50            # the tie rows overflowed their lists
    finally:
        L.set_tune(0, 0)
    # exact copies of the repeated row match its first copy (lowest index on ties)
    assert (a[0][:50] == 0).all()


def test_consistency_parity(L, orc):
    pr = pair(4, 3, 15000)
    F, vF, G, vG = _oracle_descriptors(orc, pr)
    m = orc.match(F, vF, G, vG)
    mut = orc.mutual(m["nnQ"], m["nnP"])
    for T in (1, 1000, orc.default_trials(pr.P.shape[1])):
        want, npass = orc.consistency(pr.P[:3], pr.Q[:3], m["nnQ"], mut, T, 0.9, 1234)
        flag, passed = L.stage_consistency(dev(pr.P[:3]), dev(pr.Q[:3]), dev(m["nnQ"]),
                                           dev(mut.astype(np.uint8)), T, 0.9, 1234)
        assert np.array_equal(flag.cpu().numpy().astype(bool), want)
        assert int(passed.cpu()[0]) == npass
    # closed form: Q = 2 P rejects everything
    P = pr.P[:3]
    ident = np.arange(P.shape[1], dtype=np.int32)
    flag, passed = L.stage_consistency(dev(P), dev((2 * P).astype(np.float32)), dev(ident),
                                       dev(np.ones(P.shape[1], np.uint8)), 5000, 0.9, 1)
    assert int(passed.cpu()[0]) == 0 and not flag.cpu().numpy().any()


@pytest.mark.parametrize("nC", [0, 3, 4, 5, 7, 12, 40])
def test_consistency_small_c(L, orc, nC):
    # Few reciprocal correspondences: repeated draws are common, so most trials
    # take further attempts per slot, and below four members none can pass.
    rng = np.random.default_rng(100 + nC)
    n = 300
    P = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    Q = (P * 1.02 + rng.normal(0, 0.01, (3, n))).astype(np.float32)
    Q[:, ::3] = rng.uniform(-1, 1, (3, Q[:, ::3].shape[1]))     # a third are outliers
    nnQ = np.arange(n, dtype=np.int32)
    mut = np.zeros(n, np.uint8)
    mut[rng.choice(n, nC, replace=False)] = 1
    for T, seed in ((1, 7), (20000, 99), (8193, 2**64 - 1)):
        want, npass = orc.consistency(P, Q, nnQ, mut, T, 0.9, seed)
        flag, passed = L.stage_consistency(dev(P), dev(Q), dev(nnQ), dev(mut), T, 0.9, seed)
        assert np.array_equal(flag.cpu().numpy().astype(bool), want)
        assert int(passed.cpu()[0]) == npass
        if nC < 4:
            assert npass == 0 and not want.any()


def test_consistency_large_fragment(L, orc):
    """A 230,000-point P: its correspondence words exceed what a block keeps in
    LDS, so the draws read them from global memory; flags and passing-trial
    count still bit-exact."""
    rng = np.random.default_rng(5)
    n = 230000
    P = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    Q = (P * 1.01 + rng.normal(0, 0.005, (3, n))).astype(np.float32)
    Q[:, ::4] = rng.uniform(-1, 1, (3, Q[:, ::4].shape[1]))
    nnQ = rng.permutation(n).astype(np.int32)
    Q = Q[:, np.argsort(nnQ)].copy()                  # q of P point i sits at nnQ[i]
    mut = (rng.random(n) < 0.2).astype(np.uint8)
    for T, seed in ((70001, 3), (4096, 12345)):
        want, npass = orc.consistency(P, Q, nnQ, mut, T, 0.9, seed)
        flag, passed = L.stage_consistency(dev(P), dev(Q), dev(nnQ), dev(mut), T, 0.9, seed)
        assert np.array_equal(flag.cpu().numpy().astype(bool), want)
        assert int(passed.cpu()[0]) == npass and npass > 0


def _corr(rng, n, frac_out=0.5, noise=0.003):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    th = rng.uniform(0.1, 1.0)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    t = rng.uniform(-0.5, 0.5, 3)
    p = rng.uniform(-1.5, 1.5, (n, 3))
    q = p @ R.T + t + rng.normal(0, noise, (n, 3))
    out = rng.random(n) < frac_out
    q[out] = rng.uniform(-2, 2, (out.sum(), 3))
    return p, q


@pytest.mark.parametrize("n,frac", [(3, 0.0), (200, 0.3), (5000, 0.6), (40000, 0.5)])
def test_gnc_parity(L, orc, n, frac):
    rng = np.random.default_rng(n)
    p, q = _corr(rng, n, frac)
    st, T, mu, E, it = orc.gnc(p, q)
    Tg, info = L.stage_gnc(dev(p), dev(q))
    Tg, info = Tg.cpu().numpy(), info.cpu().numpy()
    assert int(info[0]) == st and int(info[1]) == it
    assert np.abs(Tg - T).max() <= 1e-9
    assert abs(info[3] - E) <= 1e-9 * (1 + E)
    R = Tg[:3, :3]
    assert abs(np.linalg.det(R) - 1) < 1e-12


def test_gnc_degenerate(L, orc):
    s = np.linspace(0, 1, 50)[:, None] * np.array([[1.0, 2.0, 3.0]])
    Tg, info = L.stage_gnc(dev(s), dev(s + 0.1))
    assert int(info.cpu()[0]) == 3 == orc.gnc(s, s + 0.1)[0]
    Tg, info = L.stage_gnc(dev(np.zeros((2, 3))), dev(np.zeros((2, 3))))
    assert int(info.cpu()[0]) == 3


@pytest.mark.parametrize("normal_check", [0, 1])
def test_verify_parity(L, orc, normal_check):
    pr = pair(4, 5, 15000)
    nP, *_ = orc.normals(pr.P, 0.025)
    nQ, *_ = orc.normals(pr.Q, 0.025)
    for T in (pr.T_gt, np.eye(4)):
        ni, ratio, fit = orc.verify(pr.P, nP, pr.Q, nQ, T, 0.015, normal_check)
        info = L.stage_verify(dev(pr.P[:3]), dev(nP), dev(pr.Q[:3]), dev(nQ), dev(T), 0.015,
                              normal_check).cpu().numpy()
        assert info[0] == ni                          # one fma order on both sides: exact counts
        assert abs(info[2] - fit) <= 1e-6 * (1 + fit)


@pytest.mark.parametrize("normal_check", [0, 1])
def test_verify_at_the_radius(L, orc, normal_check):
    """Every q placed at distance delta from T p (float32 rounding puts about
    half just inside, half just outside): the exact inlier count, so the
    predicate at the boundary is the oracle's, bit for bit."""
    rng = np.random.default_rng(11)
    n = 20000
    P = rng.uniform(-1, 1, (3, n))
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    th = 0.7
    R = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = [0.1, -0.2, 0.3]
    u = rng.normal(size=(3, n))
    u /= np.linalg.norm(u, axis=0)
    delta = 0.015
    Pf = P.astype(np.float32)
    Q = (R @ Pf.astype(np.float64) + T[:3, 3:4] + delta * u).astype(np.float32)
    nP = rng.normal(size=(n, 3))
    nP /= np.linalg.norm(nP, axis=1, keepdims=True)
    nQ = nP @ R.T + rng.normal(0, 0.3, (n, 3))
    nQ /= np.linalg.norm(nQ, axis=1, keepdims=True)
    ni, _, _ = orc.verify(Pf, nP, Q, nQ, T, delta, normal_check)
    info = L.stage_verify(dev(Pf), dev(nP), dev(Q), dev(nQ), dev(T), delta, normal_check).cpu().numpy()
    print(f"normal_check={normal_check}: oracle {ni} gpu {int(info[0])} inliers of {n}", flush=True)
    assert 0.2 * n < ni < 0.8 * n or normal_check
    assert info[0] == ni


@pytest.mark.parametrize("cfg,idx,n,v", [(0, 0, None, 0.01), (5, 0, 60000, 0.02), (1, 1, 9000, 0.05)])
def test_voxel_parity(L, orc, cfg, idx, n, v):
    """Voxel means and normals bit-identical to the oracle, same voxel order."""
    pr = pair(cfg, idx, n)
    print(f"voxel cfg={cfg} idx={idx} n={pr.P.shape[1]} v={v}", flush=True)
    for cloud in (pr.P, pr.Q):
        want = orc.voxel(cloud, v)
        for _ in range(2):                                   # second call reuses the cached plan
            got = L.voxel_downsample(dev(cloud), v).cpu().numpy()
            assert got.shape == want.shape
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_voxel_edge_cases(L, orc):
    rng = np.random.default_rng(7)
    # duplicates, opposite normals in one voxel (zero mean normal), negative coordinates, ragged size
    n = 4099
    c = rng.normal(size=(6, n)).astype(np.float32)
    c[:3] = np.round(c[:3] * 4) / 4 - 0.125
    c[3:, 1::2] = -c[3:, 0:-1:2]
    c[:3, 1::2] = c[:3, 0:-1:2]
    for v in (0.25, 0.5, 3.0):
        want = orc.voxel(c, v)
        got = L.voxel_downsample(dev(c), v).cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    one = c[:, :1].copy()
    assert np.array_equal(L.voxel_downsample(dev(one), 0.1).cpu().numpy(), orc.voxel(one, 0.1))
    assert L.voxel_downsample(dev(c[:, :0].copy()), 0.1).shape == (6, 0)
    far = c.copy()
    far[0, 17] = 1e9
    with pytest.raises(L.LsrError):
        L.voxel_downsample(dev(far), 0.01)
    with pytest.raises(L.LsrError):
        L.voxel_downsample(dev(c), 0.0)


def _dense_mixed(seed):
    """A dense 6 cm cluster (500-1500 r_f neighbours per point) beside a 1 cm plane
    (~76): neighbourhood sizes far from the room recipe's."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0, 0.06, size=(3, 1500))
    g = np.stack(np.meshgrid(np.arange(60) * 0.01, np.arange(60) * 0.01), 0).reshape(2, -1)
    b = np.vstack([g + 0.5, np.full((1, g.shape[1]), 0.03)]) + rng.normal(0, 0.002, size=(3, g.shape[1]))
    xyz = np.concatenate([a, b], 1)
    n = rng.normal(size=(3, xyz.shape[1]))
    n /= np.linalg.norm(n, axis=0)
    return np.vstack([xyz, n]).astype(np.float32)


def test_spfh_fpfh_dense_cluster(L, orc):
    cloud = _dense_mixed(3)
    print(f"dense+plane n={cloud.shape[1]}", flush=True)
    nrm, gap, ori, _ = orc.normals(cloud, 0.025)
    S, k, kp, mg = orc.spfh(cloud[:3], nrm, 0.05)
    Sg, kg = L.stage_spfh(dev(cloud[:3]), dev(nrm), 0.05)
    Sg, kg = Sg.cpu().numpy(), kg.cpu().numpy()
    assert np.array_equal(kg, k)
    assert k[:1500].min() > 400 and np.median(k[1500:]) < 100
    keep = mg >= MARGIN
    assert keep.mean() > 0.99
    assert np.abs(Sg[keep] - S[keep]).max() <= 1e-6
    F, v, exempt = desc_exempt(orc, cloud, nrm, gap, ori, 0.05)
    Fg, vg = L.stage_fpfh(dev(cloud[:3]), dev(nrm), 0.05)
    Fg, vg = Fg.cpu().numpy().astype(np.float64), vg.cpu().numpy()
    assert np.array_equal(vg, v)
    ok = (v == 1) & ~exempt
    assert ok.mean() > 0.95
    rel = np.linalg.norm(Fg[ok] - F[ok], axis=1) / np.linalg.norm(F[ok], axis=1)
    assert rel.max() <= DESC_RTOL


def _edge_clouds():
    """Clouds that stress the row-group FPFH: tiny sizes around the 16-point group,
    a z-line (every point its own grid row), a diagonal line (groups span cells and
    rows), and a cloud inside one cell."""
    rng = np.random.default_rng(11)
    out = []
    for n in (1, 2, 3, 15, 16, 17, 33, 100):
        out.append((f"box n={n}", rng.uniform(0.0, 0.06, size=(3, n))))
    t = np.arange(400) * 0.004
    out.append(("z-line", np.vstack([np.full_like(t, 0.3), np.full_like(t, 0.2), t])))
    out.append(("diagonal", np.vstack([t, t * 0.7, t * 0.4]) + rng.normal(scale=1e-4, size=(3, t.size))))
    out.append(("one cell", rng.uniform(0.0, 0.02, size=(3, 300))))
    clouds = []
    for name, xyz in out:
        n = rng.normal(size=(3, xyz.shape[1]))
        n /= np.linalg.norm(n, axis=0)
        clouds.append((name, np.vstack([xyz, n]).astype(np.float32)))
    return clouds


@pytest.mark.parametrize("case", range(11))
def test_fpfh_edge_shapes(L, orc, case):
    name, cloud = _edge_clouds()[case]
    print(f"fpfh edge {name} n={cloud.shape[1]}", flush=True)
    # the clouds' own unit normals (lines and blobs have no well-conditioned PCA normal),
    # so only decisions within MARGIN of a bin edge are exempt
    nrm = np.ascontiguousarray(cloud[3:].T.astype(np.float64))
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    ones = np.ones(cloud.shape[1])
    F, v, exempt = desc_exempt(orc, cloud, nrm, ones, ones, 0.05)
    Fg, vg = L.stage_fpfh(dev(cloud[:3]), dev(nrm), 0.05)
    Fg, vg = Fg.cpu().numpy().astype(np.float64), vg.cpu().numpy()
    assert np.array_equal(vg, v)
    ok = (v == 1) & ~exempt
    assert ok.sum() >= 0.9 * v.sum()
    if ok.any():
        rel = np.linalg.norm(Fg[ok] - F[ok], axis=1) / np.linalg.norm(F[ok], axis=1)
        print(f"  valid {int(v.sum())} compared {int(ok.sum())} max rel {rel.max():.2e}", flush=True)
        assert rel.max() <= DESC_RTOL
    assert np.all(Fg[v == 0] == 0)
