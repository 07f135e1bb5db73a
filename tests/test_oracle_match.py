"""Pins of the oracle's descriptor matching (Algorithm 1 pre-matching cache,
both directions) and quadruple consistency filter (Algorithm 1 pre-rejection,
tau = 0.9)."""
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _desc(n, seed, dup=0):
    rng = np.random.default_rng(seed)
    F = rng.random((n, 33)) ** 3
    F = (F.reshape(n, 3, 11) / F.reshape(n, 3, 11).sum(2, keepdims=True)).reshape(n, 33)
    if dup:
        F[-dup:] = F[:dup]
    return F


def test_match_equals_numpy_brute_force(orc):
    F, G = _desc(700, 0), _desc(900, 1)
    vF = np.ones(700, np.int32); vF[::13] = 0
    vG = np.ones(900, np.int32); vG[::17] = 0
    m = orc.match(F, vF, G, vG)
    D = ((F[:, None, :] - G[None, :, :]) ** 2).sum(2)
    D[:, vG == 0] = np.inf
    D[vF == 0, :] = np.inf
    want_q = np.argmin(D, 1)
    want_p = np.argmin(D, 0)
    ok_r, ok_c = vF == 1, vG == 1
    assert np.array_equal(m["nnQ"][ok_r], want_q[ok_r]) and (m["nnQ"][~ok_r] == -1).all()
    assert np.array_equal(m["nnP"][ok_c], want_p[ok_c]) and (m["nnP"][~ok_c] == -1).all()
    srt = np.sort(D[ok_r], 1)
    assert np.allclose(m["d1Q"][ok_r], srt[:, 0], rtol=1e-12) and np.allclose(m["d2Q"][ok_r], srt[:, 1], rtol=1e-12)


def test_match_symmetry_and_identity(orc):
    F, G = _desc(500, 2), _desc(450, 3)
    v1, v2 = np.ones(500, np.int32), np.ones(450, np.int32)
    a = orc.match(F, v1, G, v2)
    b = orc.match(G, v2, F, v1)
    assert np.array_equal(a["nnQ"], b["nnP"]) and np.array_equal(a["nnP"], b["nnQ"])
    ma = orc.mutual(a["nnQ"], a["nnP"])
    mb = orc.mutual(b["nnQ"], b["nnP"])
    pa = {(i, a["nnQ"][i]) for i in np.nonzero(ma)[0]}
    pb = {(b["nnQ"][j], j) for j in np.nonzero(mb)[0]}
    assert pa == pb                                       # swapping P and Q transposes C
    c = orc.match(F, v1, F, v1)
    assert np.array_equal(c["nnQ"], np.arange(500)) and orc.mutual(c["nnQ"], c["nnP"]).all()


def test_match_ties_lowest_index_and_flags(orc):
    F = _desc(300, 4, dup=20)                             # rows 280.. duplicate rows 0..19
    G = F.copy()
    v = np.ones(300, np.int32)
    m = orc.match(F, v, G, v)
    assert np.array_equal(m["nnQ"][280:], np.arange(20))  # exact tie -> lowest index
    tP, tQ = orc.tie_flags(F, G, m)
    assert tP[280:].all() and tP[:20].all()               # zero gap is always a near tie
    assert not tP[20:280].any()


def test_splitmix64_published_vector(orc):
    rows = [l.split() for l in open(os.path.join(GOLD, "splitmix64_seed1234567.txt")) if not l.startswith("#")]
    for n, v in rows:
        assert orc.splitmix64(1234567, int(n)) == int(v)


def _drawn_quads(orc, nP, mutual, n_trials, seed):
    """The quadruples the sampler draws, reconstructed from its generator:
    uniform P indices, redrawn while the index has no reciprocal
    correspondence or repeats an earlier slot (at most 64 attempts)."""
    quads = []
    for t in range(n_trials):
        ids = []
        for s in range(4):
            got = None
            for a in range(64):
                r = orc.splitmix64(seed, (t << 8) | (s << 6) | a)
                i = ((r >> 32) * nP) >> 32
                if mutual[i] and i not in ids:
                    got = i
                    break
            if got is None:
                break
            ids.append(got)
        quads.append(ids if len(ids) == 4 else None)
    return quads


def test_consistency_closed_forms(orc):
    rng = np.random.default_rng(5)
    n = 400
    P = rng.uniform(0, 1, (3, n)).astype(np.float32)
    ident = np.arange(n, dtype=np.int32)
    mut = np.ones(n, bool)
    mut[::3] = False
    f, passed = orc.consistency(P, P, ident, mut, 2000, 0.9, 11)
    assert passed == 2000 and (f == mut).all()            # P = Q: every trial passes
    f, passed = orc.consistency(P, (2 * P).astype(np.float32), ident, mut, 2000, 0.9, 11)
    assert passed == 0 and not f.any()                    # Q = 2P: every ratio is 0.5 < 0.9
    # rigid motion of P keeps every edge length (up to float rounding)
    th = 0.8
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1]])
    Q = (R @ P.astype(float) + 0.3).astype(np.float32)
    f, passed = orc.consistency(P, Q, ident, mut, 2000, 0.9, 11)
    assert passed == 2000 and (f == mut).all()


def test_consistency_matches_enumeration(orc):
    rng = np.random.default_rng(8)
    n = 12
    P = rng.uniform(0, 1, (3, n)).astype(np.float32)
    Q = (P + rng.normal(0, 0.03, (3, n))).astype(np.float32)
    nnQ = np.arange(n, dtype=np.int32)
    nnQ[[0, 5, 9]] = nnQ[[5, 9, 0]]                          # three wrong correspondences
    mut = np.ones(n, bool)
    mut[[2, 7]] = False
    T, seed, tau = 300, 99, 0.9
    f, passed = orc.consistency(P, Q, nnQ, mut, T, tau, seed)
    Pd, Qd = P.astype(np.float64), Q.astype(np.float64)

    def ok(q):
        for k in range(4):
            a, b = q[k], q[(k + 1) % 4]
            ea = np.sum((Pd[:, a] - Pd[:, b]) ** 2)
            eb = np.sum((Qd[:, nnQ[a]] - Qd[:, nnQ[b]]) ** 2)
            t2 = float(np.float64(np.float32(tau)) ** 2)
            if ea == 0 or eb == 0 or ea < t2 * eb or eb < t2 * ea:
                return False
        return True

    # every 4-subset judged once; the sampler's verdicts must agree with it
    from itertools import combinations
    verdict = {}
    for c in combinations(np.nonzero(mut)[0].tolist(), 4):
        for perm in [(0, 1, 2, 3), (0, 1, 3, 2), (0, 2, 1, 3)]:       # the 3 cyclic orders
            verdict[tuple(c[p] for p in perm)] = ok([c[p] for p in perm])
    want = np.zeros(n, bool)
    npass = 0
    for q in _drawn_quads(orc, n, mut, T, seed):
        if q is None:
            continue
        key = None
        for rot in range(4):                                # canonical rotation/direction
            for seq in (q[rot:] + q[:rot], (q[rot:] + q[:rot])[::-1]):
                if tuple(seq) in verdict:
                    key = tuple(seq)
        assert key is not None
        if verdict[key]:
            npass += 1
            want[q] = True
    assert passed == npass and np.array_equal(f, want) and 0 < npass < T


def test_consistency_draws_are_local(orc):
    """Draws are keyed by P index: removing one correspondence changes only the
    trials that draw its index, so the flags elsewhere follow from the trials
    that never touch it.  Checked against the reconstructed draws: every
    trial that avoids the removed index keeps its verdict."""
    rng = np.random.default_rng(21)
    n = 60
    P = rng.uniform(0, 1, (3, n)).astype(np.float32)
    Q = (P + rng.normal(0, 0.01, (3, n))).astype(np.float32)
    nnQ = np.arange(n, dtype=np.int32)
    mut = rng.random(n) < 0.5
    k = int(np.nonzero(mut)[0][3])
    mut2 = mut.copy()
    mut2[k] = False
    T, seed = 400, 7
    qa = _drawn_quads(orc, n, mut, T, seed)
    qb = _drawn_quads(orc, n, mut2, T, seed)
    touched = [t for t in range(T) if (qa[t] is not None and k in qa[t]) or qa[t] != qb[t]]
    for t in range(T):
        if qa[t] is not None and k not in qa[t]:
            assert qa[t] == qb[t]                           # a trial that avoids k draws the same points
    assert 0 < len(touched) < T // 2
    fa, _ = orc.consistency(P, Q, nnQ, mut, T, 0.9, seed)
    fb, _ = orc.consistency(P, Q, nnQ, mut2, T, 0.9, seed)
    assert not fb[k]
    # a flag can only change at points that appear in a touched trial
    pts = set()
    for t in touched:
        for q in (qa[t], qb[t]):
            if q is not None:
                pts.update(q)
    diff = set(np.nonzero(fa != fb)[0].tolist())
    assert diff <= pts


def test_consistency_draw_distribution(orc):
    """Each slot's accepted index is uniform over the points with a
    correspondence (rejection sampling from a uniform P index): the slot-0
    histogram over 20000 trials passes a chi-square test, and points without a
    correspondence are never drawn."""
    n = 50
    mut = np.zeros(n, bool)
    mut[::3] = True
    counts = np.zeros(n)
    for q in _drawn_quads(orc, n, mut, 20000, 3):
        assert q is not None and all(mut[i] for i in q) and len(set(q)) == 4
        counts[q[0]] += 1
    c = counts[mut]
    e = c.sum() / len(c)
    chi2 = ((c - e) ** 2 / e).sum()
    assert counts[~mut].sum() == 0
    assert chi2 < 45                                        # 16 dof: p ~ 1e-4
