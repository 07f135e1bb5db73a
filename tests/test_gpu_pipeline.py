"""End-to-end parity of register_pair / register_batch against the oracle,
batch == per-pair, bf16 == fp32, graph replays, determinism, alignment
energy and its adjoint."""
import numpy as np
import pytest
import torch

from gpu_helpers import POSE_TOL, WORK_KEYS, check_chain, dev, orc_params, pair, rot_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_1801_01572_amd as lsr
    lsr.lib()
    return lsr


@pytest.mark.parametrize("cfg,idx,n", [(0, 0, None), (0, 1, None), (5, 0, None), (4, 2, 15000)])
def test_register_pair_parity(L, orc, cfg, idx, n):
    """A full run checked stage by stage against the oracle (check_chain), and
    against the oracle's own end-to-end result when the correspondence sets
    agree."""
    pr = pair(cfg, idx, n)
    print(f"pair cfg={cfg} idx={idx} nP={pr.P.shape[1]} nQ={pr.Q.shape[1]}", flush=True)
    prm = L.default_params()
    r, tr = L.register_pair(dev(pr.P), dev(pr.Q), prm, trace=True)
    r0 = L.register_pair(dev(pr.P), dev(pr.Q), prm)
    for k in r0:
        assert np.array_equal(np.asarray(r0[k]), np.asarray(r[k])), k
    c = check_chain(orc, pr.P, pr.Q, r, tr, prm, f"cfg{cfg}/{idx}")
    o, _, _ = orc.register_pair(pr.P, pr.Q, orc_params(orc, prm))
    d = orc.result_dict(o)
    print(f"  gpu status {r['status']} recip {r['n_recip']} K {r['n_consistent']} | oracle status {d['status']} "
          f"recip {d['n_recip']} K {d['n_consistent']}; C differs in {c['n_c_diff']}; pose vs oracle on the "
          f"GPU's K {c['pose_err']}; err vs T_gt {rot_err(r['T'], pr.T_gt)}", flush=True)
    if c["n_c_diff"] == 0:
        assert (r["n_recip"], r["n_consistent"], r["status"]) == (d["n_recip"], d["n_consistent"], d["status"])
        if d["status"] != orc.DEGENERATE:
            ang, trn = rot_err(r["T"], d["T"])
            assert ang <= POSE_TOL and trn <= POSE_TOL, (ang, trn)
    R = r["T"][:3, :3]
    assert abs(np.linalg.det(R) - 1) < 1e-12 and np.abs(R.T @ R - np.eye(3)).max() < 1e-12


def test_bf16_equals_fp32_end_to_end(L):
    pr = pair(4, 4, 20000)
    a = L.register_pair(dev(pr.P), dev(pr.Q), L.default_params(precision=L.FP32))
    b = L.register_pair(dev(pr.P), dev(pr.Q), L.default_params(precision=L.BF16_SCREEN))
    for k in a:
        if k not in WORK_KEYS:
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def _batch(prs):
    P = np.concatenate([p.P for p in prs], 1)
    Q = np.concatenate([p.Q for p in prs], 1)
    offP = np.concatenate([[0], np.cumsum([p.P.shape[1] for p in prs])])
    offQ = np.concatenate([[0], np.cumsum([p.Q.shape[1] for p in prs])])
    return P, Q, offP, offQ


def test_batch_equals_pairs_and_replays(L):
    prs = [pair(2, k, (int(n1), int(n2))) for k, (n1, n2) in enumerate([(3000, 5000), (700, 9000), (6000, 200),
                                                                         (0, 100), (4000, 4000)])]
    P, Q, offP, offQ = _batch(prs)
    Pd, Qd = dev(P), dev(Q)
    for prec in (L.FP32, L.BF16_SCREEN):
        prm = L.default_params(precision=prec)
        want = [L.register_pair(dev(p.P), dev(p.Q), prm) for p in prs]
        outs = []
        side = torch.cuda.Stream()                        # a non-default stream: captured once, then replayed
        for rep in range(3):
            with torch.cuda.stream(side):
                outs.append(L.register_batch(Pd, Qd, offP, offQ, prm))
            torch.cuda.synchronize()
            _ = (Pd * 2).sum().item()                     # unrelated eager work between replays
        for res in outs:
            for b in range(len(prs)):
                for k in want[b]:
                    assert np.array_equal(np.asarray(res[b][k]), np.asarray(want[b][k])), (prec, b, k)
    assert want[3]["status"] == L.DEGENERATE


def test_batch_tiny_fragments(L):
    """Fragments of 1-17 points and an empty Q inside one batch (single partial
    blocks, one-point row groups, XCD-ordered grids of one block): batch ==
    per-pair in both precisions."""
    sizes = [(1, 1), (3, 7), (15, 16), (17, 300), (300, 17), (100, 0), (2500, 2500)]
    prs = [pair(2, 20 + k, (int(n1), max(int(n2), 1))) for k, (n1, n2) in enumerate(sizes)]
    for pr, (_, n2) in zip(prs, sizes):
        if n2 == 0:
            pr.Q = pr.Q[:, :0].copy()                     # an empty Q
    P, Q, offP, offQ = _batch(prs)
    for prec in (L.FP32, L.BF16_SCREEN):
        prm = L.default_params(precision=prec)
        want = [L.register_pair(dev(p.P), dev(p.Q), prm) for p in prs]
        got = L.register_batch(dev(P), dev(Q), offP, offQ, prm)
        for b in range(len(prs)):
            for k in want[b]:
                assert np.array_equal(np.asarray(got[b][k]), np.asarray(want[b][k])), (prec, sizes[b], k)
        print(prec, [g["status"] for g in got], flush=True)




def test_pruned_screen_small_and_ragged(L):
    """The pruned screen on fragments of 1-17 points, an empty Q, ragged and
    equal sizes: bf16 == float32 in every result but the fallback count."""
    sizes = [(1, 1), (3, 7), (15, 16), (17, 300), (300, 17), (100, 0), (2500, 2500), (9000, 700), (700, 9000)]
    prs = [pair(2, 40 + k, (int(n1), max(int(n2), 1))) for k, (n1, n2) in enumerate(sizes)]
    for pr, (_, n2) in zip(prs, sizes):
        if n2 == 0:
            pr.Q = pr.Q[:, :0].copy()
    P, Q, offP, offQ = _batch(prs)
    Pd, Qd = dev(P), dev(Q)
    fp = L.register_batch(Pd, Qd, offP, offQ, L.default_params(precision=L.FP32))
    saved = L.get_tune()
    try:
        L.set_tune(L._lib.PRUNED_SCREEN, saved["consistency_shape"])
        bf = L.register_batch(Pd, Qd, offP, offQ, L.default_params(precision=L.BF16_SCREEN))
        bf2 = L.register_batch(Pd, Qd, offP, offQ, L.default_params(precision=L.BF16_SCREEN))
    finally:
        L.set_tune(saved["screen_shape"], saved["consistency_shape"])
    for b in range(len(prs)):
        for k in fp[b]:
            if k not in WORK_KEYS:
                assert np.array_equal(np.asarray(bf[b][k]), np.asarray(fp[b][k])), (sizes[b], k)
            assert np.array_equal(np.asarray(bf2[b][k]), np.asarray(bf[b][k])), (sizes[b], k)
    print("fallback rows", [r["n_fallback_rows"] for r in bf], flush=True)


def test_deterministic(L):
    pr = pair(4, 6, 12000)
    a = L.register_pair(dev(pr.P), dev(pr.Q))
    b = L.register_pair(dev(pr.P.copy()), dev(pr.Q.copy()))
    for k in a:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k


def test_invalid_arguments(L):
    import paper_1801_01572_amd._lib as lib
    pr = pair(0, 2)
    P = dev(pr.P)
    with pytest.raises(lib.LsrError):
        L.register_pair(P, dev(pr.Q), L.default_params(r_feature=-1.0))
    with pytest.raises(lib.LsrError):
        L.register_pair(P, dev(pr.Q), L.default_params(tau=1.5))
    with pytest.raises(lib.LsrError):
        L.register_batch(P, dev(pr.Q), [0, 10 ** 7], [0, 5], L.default_params())


def test_align_loss_and_adjoint(L, orc):
    rng = np.random.default_rng(2)
    nprob = 5
    Ps, Qs, corr, coff, Ts, mus = [], [], [], [0], [], []
    baseP = baseQ = 0
    for k in range(nprob):
        n = int(rng.integers(50, 3000))
        p = rng.uniform(-1, 1, (n, 3))
        th = rng.uniform(0, 1)
        R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
        T = np.eye(4); T[:3, :3] = R; T[:3, 3] = rng.uniform(-0.3, 0.3, 3)
        q = p @ R.T + T[:3, 3] + rng.normal(0, 0.01, (n, 3))
        q[: n // 3] += rng.normal(0, 0.3, (n // 3, 3))
        Ps.append(p); Qs.append(q)
        idx = np.arange(n)
        corr.append(np.stack([baseP + idx, baseQ + idx], 1))
        baseP += n; baseQ += n
        coff.append(coff[-1] + n)
        Ts.append(T); mus.append(rng.uniform(1e-4, 1e-2))
    Pf = np.concatenate(Ps).astype(np.float32)
    Qf = np.concatenate(Qs).astype(np.float32)
    C = np.concatenate(corr).astype(np.int32)
    Td, mud = dev(np.stack(Ts)), dev(np.array(mus))
    E = L.align_loss(dev(Pf.T), dev(Qf.T), dev(C), coff, Td, mud).cpu().numpy()
    dE = rng.uniform(0.5, 2.0, nprob)
    dP, dQ, dxi = [t.cpu().numpy() for t in L.align_loss_backward(dev(Pf.T), dev(Qf.T), dev(C), coff, Td, mud,
                                                                  dev(dE))]
    for k in range(nprob):
        s = slice(coff[k], coff[k + 1])
        Eo, gp, gq, gx = orc.align_loss(Pf[s].astype(np.float64), Qf[s].astype(np.float64), Ts[k], mus[k])
        assert abs(E[k] - Eo) <= 1e-12 * (1 + abs(Eo))
        assert np.abs(dxi[k] - dE[k] * gx).max() <= 1e-10 * (1 + np.abs(dE[k] * gx).max())
        assert np.abs(dP[:, s].T - dE[k] * gp).max() <= 1e-6 * (1 + np.abs(gp).max())
        assert np.abs(dQ[:, s].T - dE[k] * gq).max() <= 1e-6 * (1 + np.abs(gq).max())


def test_autograd_function_fd(L):
    rng = np.random.default_rng(3)
    n = 400
    p = rng.uniform(-1, 1, (n, 3))
    q = p + rng.normal(0, 0.05, (n, 3))
    C = np.stack([np.arange(n), np.arange(n)], 1).astype(np.int32)
    P = dev(p.T.astype(np.float32)).requires_grad_(True)
    Q = dev(q.T.astype(np.float32)).requires_grad_(True)
    T = dev(np.eye(4)[None])
    mu = dev(np.array([0.004]))
    xi = torch.zeros((1, 6), dtype=torch.float64, device="cuda", requires_grad=True)
    E = L.AlignLoss.apply(P, Q, dev(C), [0, n], T, mu, xi)
    E.sum().backward()
    h = 1e-4
    for k in range(6):
        Ts = []
        for s in (1, -1):
            w = np.zeros(3); v = np.zeros(3)
            (w if k < 3 else v)[k % 3] = s * h
            K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
            D = np.eye(4); D[:3, :3] = np.eye(3) + K + 0.5 * K @ K; D[:3, 3] = v
            Ts.append(dev((D @ np.eye(4))[None]))
        Ep = L.align_loss(P.detach(), Q.detach(), dev(C), [0, n], Ts[0], mu).item()
        Em = L.align_loss(P.detach(), Q.detach(), dev(C), [0, n], Ts[1], mu).item()
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - xi.grad[0, k].item()) <= 1e-4 * (1 + abs(fd))


def test_autograd_function_nonzero_xi(L, orc):
    """E at the retracted pose [Rod(w) | v] T equals the oracle's energy at
    that pose (retraction written here with scipy); dE/dxi equals central
    differences of the forward; dP, dQ equal the oracle's gradients there."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(8)
    n = 600
    p = rng.uniform(-1, 1, (n, 3))
    T0 = np.eye(4)
    T0[:3, :3] = Rotation.from_rotvec([0.2, -0.5, 0.3]).as_matrix()
    T0[:3, 3] = [0.3, -0.1, 0.2]
    xi0 = np.array([0.25, -0.1, 0.4, 0.05, 0.3, -0.2])
    Tx = np.eye(4)
    Tx[:3, :3] = Rotation.from_rotvec(xi0[:3]).as_matrix()
    Tx[:3, 3] = xi0[3:]
    Tx = Tx @ T0
    q = (Tx[:3, :3] @ p.T).T + Tx[:3, 3] + rng.normal(0, 0.05, (n, 3))
    p32, q32 = p.astype(np.float32), q.astype(np.float32)
    C = np.stack([np.arange(n), np.arange(n)], 1).astype(np.int32)
    P = dev(p32.T).requires_grad_(True)
    Q = dev(q32.T).requires_grad_(True)
    mu = dev(np.array([0.01]))
    xi = dev(xi0[None]).requires_grad_(True)
    E = L.AlignLoss.apply(P, Q, dev(C), [0, n], dev(T0[None]), mu, xi)
    Eo, dpo, dqo, _ = orc.align_loss(p32.astype(np.float64), q32.astype(np.float64), Tx, 0.01)
    assert abs(E.item() - Eo) <= 1e-10 * (1 + abs(Eo))
    E.sum().backward()
    assert np.abs(P.grad.cpu().numpy().T - dpo).max() <= 1e-6 * (1 + np.abs(dpo).max())
    assert np.abs(Q.grad.cpu().numpy().T - dqo).max() <= 1e-6 * (1 + np.abs(dqo).max())
    h = 1e-6
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        Ep = L.AlignLoss.apply(P.detach(), Q.detach(), dev(C), [0, n], dev(T0[None]), mu, dev((xi0 + e)[None]))
        Em = L.AlignLoss.apply(P.detach(), Q.detach(), dev(C), [0, n], dev(T0[None]), mu, dev((xi0 - e)[None]))
        fd = (Ep.item() - Em.item()) / (2 * h)
        assert abs(fd - xi.grad[0, k].item()) <= 1e-5 * (1 + abs(fd)), (k, fd, xi.grad[0, k].item())


def test_adjoint_deterministic_with_shared_points(L, orc):
    """Points shared by several correspondences (each P point three times,
    Q points twice, across two problems): two backward runs give the same
    bits, and the sums equal the oracle's per-correspondence gradients
    accumulated in FP64."""
    rng = np.random.default_rng(9)
    nP, nQ = 2000, 3000
    P = rng.uniform(-1, 1, (3, nP)).astype(np.float32)
    Q = rng.uniform(-1, 1, (3, nQ)).astype(np.float32)
    m = 6000
    ci = np.tile(np.arange(nP), 3)[rng.permutation(m)]
    cj = np.tile(rng.permutation(nQ), 2)[:m]
    C = np.stack([ci, cj], 1).astype(np.int32)
    coff = [0, 2500, m]
    T = np.stack([np.eye(4), np.eye(4)])
    T[1, :3, 3] = [0.1, 0.0, -0.2]
    mu = np.array([0.05, 0.02])
    dE = np.array([1.0, -0.5])
    outs = []
    for _ in range(2):
        dP, dQ, dxi = L.align_loss_backward(dev(P), dev(Q), dev(C), coff, dev(T), dev(mu), dev(dE))
        outs.append((dP.cpu().numpy(), dQ.cpu().numpy(), dxi.cpu().numpy()))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    wp = np.zeros((nP, 3))
    wq = np.zeros((nQ, 3))
    for k in range(2):
        sl = slice(coff[k], coff[k + 1])
        _, dp, dq, _ = orc.align_loss(P.T[C[sl, 0]].astype(np.float64), Q.T[C[sl, 1]].astype(np.float64), T[k],
                                      mu[k])
        np.add.at(wp, C[sl, 0], dE[k] * dp)
        np.add.at(wq, C[sl, 1], dE[k] * dq)
    assert np.abs(outs[0][0].T - wp).max() <= 1e-6 * (1 + np.abs(wp).max())
    assert np.abs(outs[0][1].T - wq).max() <= 1e-6 * (1 + np.abs(wq).max())


def test_autotune_cache(L, tmp_path):
    """The tune cache: a first autotune times the variants and records the
    choice under the device's architecture and the batch's size bucket; a
    fresh context with the same cache takes that choice without timing; an
    unreadable entry falls back to timing."""
    import json
    prs = [pair(4, k, 3000) for k in range(3)]
    P = np.concatenate([p.P for p in prs], 1)
    Q = np.concatenate([p.Q for p in prs], 1)
    off = np.array([0, 3000, 6000, 9000], np.int64)
    path = str(tmp_path / "tune.json")
    c1 = L.Context(0)
    t1 = L.autotune(dev(P), dev(Q), off, off, L.default_params(), reps=1, ctx=c1, cache=path)
    assert not t1["from_cache"] and max(t1["screen_ms"]) > 0
    data = json.load(open(path))
    assert len(data["entries"]) == 1 and data["entries"][0]["key"].startswith("gfx950|pairs=4|")
    assert data["entries"][0]["screen_shape"] == t1["screen_shape"]
    c2 = L.Context(0)
    t2 = L.autotune(dev(P), dev(Q), off, off, L.default_params(), reps=1, ctx=c2, cache=path)
    assert t2["from_cache"] and (t2["screen_shape"], t2["consistency_shape"]) == \
        (t1["screen_shape"], t1["consistency_shape"]) and max(t2["screen_ms"]) == 0
    assert L.get_tune(c2)["screen_shape"] == t1["screen_shape"]
    data["entries"][0]["screen_shape"] = 99                   # out of range: timed again, entry replaced
    json.dump(data, open(path, "w"))
    t3 = L.autotune(dev(P), dev(Q), off, off, L.default_params(), reps=1, ctx=L.Context(0), cache=path)
    assert not t3["from_cache"] and len(json.load(open(path))["entries"]) == 1


def test_autotune_variants_agree(L):
    """Every launch-shape variant computes the same bits; the autotuner picks one and times all."""
    import paper_1801_01572_amd._lib as lib
    prs = [pair(2, 10 + k, (int(n1), int(n2))) for k, (n1, n2) in enumerate([(4000, 6000), (9000, 700), (2500, 2500)])]
    P, Q, offP, offQ = _batch(prs)
    Pd, Qd = dev(P), dev(Q)
    prm = L.default_params(precision=L.BF16_SCREEN)
    info = L.get_tune()
    ref = None
    try:
        for sv in range(info["n_screen_shapes"]):
            for cv in range(info["n_consistency_shapes"]):
                print(f"tune screen={sv} consistency={cv}", flush=True)
                L.set_tune(sv, cv)
                res = L.register_batch(Pd, Qd, offP, offQ, prm)
                if ref is None:
                    ref = res
                for b in range(len(prs)):
                    for k in ref[b]:
                        if k not in WORK_KEYS:          # the screen's work depends on the variant
                            assert np.array_equal(np.asarray(res[b][k]), np.asarray(ref[b][k])), (sv, cv, b, k)
        t = L.autotune(Pd, Qd, offP, offQ, prm, reps=1)
        assert 0 <= t["screen_shape"] < info["n_screen_shapes"]
        assert 0 <= t["consistency_shape"] < info["n_consistency_shapes"]
        assert all(ms > 0 for ms in t["screen_ms"] + t["consistency_ms"])
        assert t["screen_ms"][t["screen_shape"]] == min(t["screen_ms"])
        g = L.get_tune()
        assert (g["screen_shape"], g["consistency_shape"]) == (t["screen_shape"], t["consistency_shape"])
        res = L.register_batch(Pd, Qd, offP, offQ, prm)
        for b in range(len(prs)):
            for k in ref[b]:
                if k not in WORK_KEYS:
                    assert np.array_equal(np.asarray(res[b][k]), np.asarray(ref[b][k])), ("tuned", b, k)
        with pytest.raises(lib.LsrError):
            L.set_tune(info["n_screen_shapes"], 0)
    finally:
        L.set_tune(0, 0)
