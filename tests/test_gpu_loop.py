"""GPU parity of the loop verification (Sec. V, eqs. 2-5) against the oracle,
through the C ABI: edge correspondence counts exact and information
matrices within 1e-12 (relative to the matrix; moment sums against direct
sums of G^T G), the pose-graph solve on the oracle's own information
(poses within 1e-9, l within 1e-9, the same decision, iteration counts
within one), the combined call equal to the two steps, and edge cases: a
two-node chain, a loop from the fixed node, a loop between neighbours, a
loop ending at the last node, a loop without correspondences, a singular
chain, invalid chains."""
import numpy as np
import pytest
import torch

from gpu_helpers import dev
from synth.chain import make_chain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_1801_01572_amd as lsr
    lsr.lib()
    return lsr


@pytest.fixture(scope="module")
def chain():
    return make_chain(24, 3000, n_true=3, n_false=4)


@pytest.fixture(scope="module")
def frags(chain):
    return [dev(f) for f in chain.frags]


@pytest.fixture(scope="module")
def oracle_info(orc, chain):
    edges = list(chain.odo) + list(chain.loops)
    out = [orc.edge_info(chain.frags[i], chain.frags[j], A) for (i, j, A) in edges]
    return np.array([o[0] for o in out]), np.array([o[1] for o in out])


def _cmp_info(g, o):
    scale = np.abs(o).max(axis=(1, 2), keepdims=True) + 1e-300
    return float((np.abs(g - o) / scale).max())


def test_edge_info_parity(L, chain, frags, oracle_info):
    edges = list(chain.odo) + list(chain.loops)
    print(f"edge info: {len(edges)} edges over {len(frags)} fragments", flush=True)
    info, cnt = L.edge_info(frags, edges, 0.05)
    Lo, co = oracle_info
    assert np.array_equal(cnt.cpu().numpy(), co)
    assert _cmp_info(info.cpu().numpy(), Lo) <= 1e-12


def _solve_both(L, orc, chain, Lo, co, loops, idx, params=None, oparams=None):
    n = len(chain.frags)
    no = n - 1
    info_odo = dev(Lo[:no])
    res, T = L.loop_solve(chain.T_init, chain.odo, info_odo, loops, dev(Lo[idx]), dev(co[idx]), params)
    T = T.cpu().numpy()
    for c, (lp, k) in enumerate(zip(loops, idx)):
        r, To = orc.loop_solve(chain.T_init, chain.odo, Lo[:no], lp, Lo[k], co[k], oparams)
        g = res[c]
        print(f"  loop {lp[0]}-{lp[1]}: gpu l {g['l']:.6f} status {g['status']} iters {g['iters']}; "
              f"oracle l {r['l']:.6f} status {r['status']} iters {r['iters']}", flush=True)
        assert g["n_corr"] == co[k]
        assert abs(g["l"] - r["l"]) <= 1e-9
        assert g["status"] == r["status"] or abs(r["l"] - 0.25) <= 1e-9
        assert abs(g["iters"] - r["iters"]) <= 1
        if r["status"] != orc.DEGENERATE:
            assert np.abs(T[c] - To).max() <= 1e-9
            assert abs(g["energy"] - r["energy"]) <= 1e-9 * (1 + abs(r["energy"]))
    return res


def test_loop_solve_parity(L, orc, chain, oracle_info):
    Lo, co = oracle_info
    no = len(chain.frags) - 1
    idx = list(range(no, no + len(chain.loops)))
    print(f"loop solve: {len(idx)} candidates", flush=True)
    res = _solve_both(L, orc, chain, Lo, co, chain.loops, idx)
    dec = [r["status"] == L.ACCEPTED for r in res]
    assert dec == list(chain.loop_true)


def test_loop_verify_equals_two_steps(L, chain, frags):
    prm = L.loop_params()
    res, T = L.loop_verify(frags, chain.T_init, chain.odo, chain.loops, prm)
    info, cnt = L.edge_info(frags, list(chain.odo) + list(chain.loops), prm.eps)
    no = len(chain.frags) - 1
    res2, T2 = L.loop_solve(chain.T_init, chain.odo, info[:no], chain.loops, info[no:], cnt[no:], prm)
    assert res == res2
    assert torch.equal(T, T2)
    res3, T3 = L.loop_verify(frags, chain.T_init, chain.odo, chain.loops, prm)
    assert res3 == res and torch.equal(T3, T)


def test_loop_edge_cases(L, orc, chain, oracle_info):
    Lo, co = oracle_info
    n = len(chain.frags)
    no = n - 1
    i0, j0, A0 = chain.loops[0]
    # loops from the fixed node, between neighbours, across one node, ending at the last node, reversed (the true
    # transforms, which the drifted initial poses do not satisfy)
    inv = np.linalg.inv
    cases = [(0, 1), (7, 8), (9, 11), (3, n - 1), (4, 2)]
    extra = [(a, b, inv(chain.T_true[b]) @ chain.T_true[a]) for a, b in cases]
    ex = [orc.edge_info(chain.frags[a], chain.frags[b], A) for a, b, A in extra]
    Lx = np.concatenate([Lo, np.array([e[0] for e in ex])])
    cx = np.concatenate([co, np.array([e[1] for e in ex])])
    idx = list(range(len(Lo), len(Lx)))
    print("loop edge cases: fixed node, neighbours, last node, reversed", flush=True)
    assert (cx[idx] > 0).all()
    _solve_both(L, orc, chain, Lx, cx, extra, idx)
    # no correspondences: rejected, poses untouched
    c0 = co.copy()
    c0[no] = 0
    res, T = L.loop_solve(chain.T_init, chain.odo, dev(Lo[:no]), [chain.loops[0]], dev(Lo[no:no + 1]),
                          dev(c0[no:no + 1]))
    assert res[0]["status"] == L.REJECTED and res[0]["l"] == 0.0 and res[0]["iters"] == 0
    assert np.array_equal(T[0].cpu().numpy(), chain.T_init)
    # the last odometry edge without information: singular
    Lz = Lo.copy()
    Lz[no - 1] = 0
    print("loop edge cases: singular chain", flush=True)
    res = _solve_both(L, orc, chain, Lz, co, [chain.loops[0]], [no])
    assert res[0]["status"] == L.DEGENERATE
    # two nodes
    T2 = chain.T_init[:2]
    A = inv(chain.T_true[1]) @ chain.T_true[0]
    L2, c2 = orc.edge_info(chain.frags[0], chain.frags[1], chain.odo[0][2])
    r, To = orc.loop_solve(T2, chain.odo[:1], L2[None], (0, 1, A), L2, c2)
    res, Tg = L.loop_solve(T2, chain.odo[:1], dev(L2[None]), [(0, 1, A)], dev(L2[None]), dev(np.array([c2])))
    assert abs(res[0]["l"] - r["l"]) <= 1e-9 and np.abs(Tg[0].cpu().numpy() - To).max() <= 1e-9
    # invalid: an odometry edge that skips a node
    bad = list(chain.odo)
    bad[3] = (3, 5, bad[3][2])
    with pytest.raises(Exception):
        L.loop_solve(chain.T_init, bad, dev(Lo[:no]), chain.loops[:1], dev(Lo[no:no + 1]), dev(co[no:no + 1]))


def test_loop_verify_at_scale(L, orc):
    ch = make_chain(64, 20000, n_true=8, n_false=8)
    frags = [dev(f) for f in ch.frags]
    print("loop verify: 64 fragments x 20000 points, 16 candidates", flush=True)
    res, T = L.loop_verify(frags, ch.T_init, ch.odo, ch.loops, L.loop_params())
    assert [r["status"] == L.ACCEPTED for r in res] == list(ch.loop_true)
    # sampled edges and candidates against the oracle
    info, cnt = L.edge_info(frags, list(ch.odo) + list(ch.loops), 0.05)
    edges = list(ch.odo) + list(ch.loops)
    for k in (0, 17, 40, 62, 63, 70, 78):
        i, j, A = edges[k]
        Lk, ck = orc.edge_info(ch.frags[i], ch.frags[j], A)
        assert cnt[k].item() == ck
        assert _cmp_info(info[k:k + 1].cpu().numpy(), Lk[None]) <= 1e-12
    Lo = info.cpu().numpy()
    co = cnt.cpu().numpy()
    T = T.cpu().numpy()
    for c in (0, 9):
        r, To = orc.loop_solve(ch.T_init, ch.odo, Lo[:63], ch.loops[c], Lo[63 + c], co[63 + c])
        assert abs(res[c]["l"] - r["l"]) <= 1e-9 and res[c]["status"] == r["status"]
        assert np.abs(T[c] - To).max() <= 1e-9


def test_loop_solve_long_chain(L, orc):
    """A 150-node chain: edges and nodes beyond the wave's 64 lanes (each lane
    takes several), and a chain on one side of the loop's later node longer
    than 64; the solve against the oracle's dense one on the GPU's own edge
    information."""
    ch = make_chain(150, 2000, n_true=2, n_false=2)
    frags = [dev(f) for f in ch.frags]
    n = len(ch.frags)
    print(f"loop solve: {n} fragments x 2000 points, {len(ch.loops)} candidates "
          f"{[(i, j) for i, j, _ in ch.loops]}", flush=True)
    prm = L.loop_params()
    res, T = L.loop_verify(frags, ch.T_init, ch.odo, ch.loops, prm)
    info, cnt = L.edge_info(frags, list(ch.odo) + list(ch.loops), prm.eps)
    Lo = info.cpu().numpy()
    co = cnt.cpu().numpy()
    T = T.cpu().numpy()
    assert max(max(i, j) for i, j, _ in ch.loops) - 1 > 64
    for c in range(len(ch.loops)):
        r, To = orc.loop_solve(ch.T_init, ch.odo, Lo[:n - 1], ch.loops[c], Lo[n - 1 + c], co[n - 1 + c])
        g = res[c]
        print(f"  candidate {c}: gpu l {g['l']:.6f} status {g['status']} iters {g['iters']}; "
              f"oracle l {r['l']:.6f} status {r['status']} iters {r['iters']}", flush=True)
        assert g["n_corr"] == co[n - 1 + c]
        assert abs(g["l"] - r["l"]) <= 1e-9
        assert g["status"] == r["status"]
        assert abs(g["iters"] - r["iters"]) <= 1
        assert np.abs(T[c] - To).max() <= 1e-9
        assert abs(g["energy"] - r["energy"]) <= 1e-9 * (1 + abs(r["energy"]))
