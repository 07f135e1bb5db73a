"""Randomized CPU check of the rounding analysis behind the bf16 screen's
certificate (the inequalities the matcher's slack and screen-error bounds
rest on), with the screen's arithmetic emulated in numpy: float32 Helmert
projections and centring, bf16 round-to-nearest-even splits, exact products
with the worst-case float32 accumulation error added, and the float32
difference-form distance of the exact re-rank.

For every query i and candidate j (realistic histograms, near-duplicates,
peaked and flat descriptors):
  (1) |D^ij - D^y_ij| <= slack(D^ij, delta_i + delta_j): the float32
      distance over the 33 bins against the projected distance of the float
      projections (delta: a row's distance from the exact projection);
  (2) for competitors of i (D^ij <= D*, for every D* drawn from i's row),
      |y_j - y_i| <= Rp(D*) and |s_ij - t_ij - c_i| <= E(D*), where s is the
      exact score in projected space and t the screened score.
"""
import numpy as np
import pytest

U = 2.0 ** -24
NB = 11


def f32(x):
    return np.asarray(x, np.float32)


def bf16(x):
    """Round float32 to bfloat16 (nearest, ties to even), returned as float32."""
    u = f32(x).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def helmert32(X):
    """float32 Helmert contrasts of each 11-bin block (the pack kernel's order,
    its reciprocal square roots taken correctly rounded)."""
    n = X.shape[0]
    H = np.zeros((n, 30), np.float32)
    for k in range(3):
        s = X[:, NB * k].copy()
        for q in range(1, NB):
            r = f32(1.0 / np.sqrt(q * (q + 1)))
            H[:, 10 * k + q - 1] = f32(f32(s - f32(np.float32(q) * X[:, NB * k + q])) * r)
            s = f32(s + X[:, NB * k + q])
    return H


def helmert64(X):
    X = X.astype(np.float64)
    n = X.shape[0]
    H = np.zeros((n, 30))
    for k in range(3):
        s = X[:, NB * k].copy()
        for q in range(1, NB):
            H[:, 10 * k + q - 1] = (s - q * X[:, NB * k + q]) / np.sqrt(q * (q + 1))
            s = s + X[:, NB * k + q]
    return H


def d2_fp32(A, B):
    """The re-rank's float32 difference form: t = a - b (rounded), acc = fma(t, t, acc)."""
    acc = np.zeros((A.shape[0], B.shape[0]), np.float32)
    for c in range(A.shape[1]):
        t = f32(A[:, None, c] - B[None, :, c])
        acc = f32(t.astype(np.float64) ** 2 + acc.astype(np.float64))
    return acc


def slack(D, dl):
    return D * 3e-6 + 2.01 * np.sqrt(D) * dl + 2.0 * dl * dl + 1e-10


def bounds(ny2, dnorm, D, dl):
    yi = np.sqrt(ny2)
    Rp = np.sqrt(D + slack(D, dl)) * 1.0001 + dl + 1e-9
    R = yi * 1.0001 + Rp
    return Rp, dnorm * Rp + 3.0518e-5 * (yi * R + 0.5 * R * R) + 1e-9


def descriptors(rng, n, kind):
    X = np.zeros((n, 33))
    for k in range(3):
        if kind == "peaked":
            a = rng.gamma(0.05, size=(n, NB))
        elif kind == "flat":
            a = 1.0 + 0.01 * rng.random((n, NB))
        else:
            a = rng.gamma(0.6, size=(n, NB))
        a[a.sum(1) == 0, 0] = 1.0
        X[:, NB * k:NB * (k + 1)] = a / a.sum(1, keepdims=True)
    return f32(X)


@pytest.mark.parametrize("kind", ["histogram", "peaked", "flat", "near-duplicate"])
def test_certificate_bounds(kind):
    rng = np.random.default_rng({"histogram": 1, "peaked": 2, "flat": 3, "near-duplicate": 4}[kind])
    nq, nc = 200, 1500
    if kind == "near-duplicate":
        base = descriptors(rng, 40, "histogram")
        X = np.repeat(base, (nq + nc) // 40 + 1, axis=0)[: nq + nc].astype(np.float64)
        X *= 1 + 1e-5 * rng.standard_normal(X.shape)
        for k in range(3):
            X[:, NB * k:NB * (k + 1)] /= X[:, NB * k:NB * (k + 1)].sum(1, keepdims=True)
        X = f32(X)
    else:
        X = descriptors(rng, nq + nc, "peaked" if kind == "peaked" else "flat" if kind == "flat" else "histogram")
    m = f32(helmert64(X[:256]).mean(0))                          # a centre (any centre keeps distances)
    Y = f32(helmert32(X) - m)                                     # the rows' float projections
    delta = np.linalg.norm(Y.astype(np.float64) - (helmert64(X) - m.astype(np.float64)), axis=1)
    delta = delta * (1 + 1e-6) + 1e-15
    Q, C = slice(0, nq), slice(nq, nq + nc)
    Dh = d2_fp32(X[Q], X[C]).astype(np.float64)                  # re-rank distances
    Yq, Yc = Y[Q].astype(np.float64), Y[C].astype(np.float64)
    Dy = ((Yq[:, None, :] - Yc[None, :, :]) ** 2).sum(2)         # projected distances
    dl = delta[Q][:, None] + delta[C][None, :]
    # (1)
    assert (np.abs(Dh - Dy) <= slack(Dh, dl)).all()
    # screen quantities
    ny2 = np.zeros(nq, np.float32)
    for c in range(30):
        ny2 = f32(Y[Q][:, c].astype(np.float64) ** 2 + ny2.astype(np.float64))
    ny2_c = np.zeros(nc, np.float32)
    for c in range(30):
        ny2_c = f32(Y[C][:, c].astype(np.float64) ** 2 + ny2_c.astype(np.float64))
    yh = bf16(Y[Q]).astype(np.float64)                            # query rounded once
    d_i = Yq - yh
    dnorm = np.sqrt((d_i ** 2).sum(1)) * 1.0001
    c_i = (d_i * Yq).sum(1)
    hi = bf16(Y[C])
    lo = bf16(f32(Y[C] - hi))
    cc = f32(-0.5 * ny2_c)
    chi = bf16(cc)
    clo = bf16(f32(cc - chi))
    prod_h = yh @ hi.astype(np.float64).T + yh @ lo.astype(np.float64).T
    t = prod_h + chi.astype(np.float64)[None, :] + clo.astype(np.float64)[None, :]
    acc = np.abs(yh) @ (np.abs(hi.astype(np.float64)) + np.abs(lo.astype(np.float64))).T \
        + np.abs(chi.astype(np.float64))[None, :] + np.abs(clo.astype(np.float64))[None, :]
    s = 0.5 * ((Yq ** 2).sum(1)[:, None] - Dy)
    err = np.abs(s - t - c_i[:, None]) + 64 * U * acc             # worst float32 accumulation of 64 terms
    # (2): every candidate row's D^ taken as the current best D*
    order = np.argsort(Dh, axis=1)
    checked = 0
    for i in range(nq):
        for r in (0, 1, 2, 5, 20, 200):
            Ds = Dh[i, order[i, r]]
            comp = Dh[i] <= Ds
            Rp, E = bounds(float(ny2[i]), dnorm[i], Ds, delta[Q][i] + delta[C].max())
            assert (np.sqrt(Dy[i, comp]) <= Rp).all()
            assert (err[i, comp] <= E).all(), (i, r, err[i, comp].max(), E)
            checked += int(comp.sum())
    assert checked > nq * 200



def _up(x, n):
    """x moved n float32 ulps towards +inf."""
    x = f32(x)
    for _ in range(n):
        x = np.nextafter(x, np.float32(np.inf), dtype=np.float32)
    return x


def _fma32(a, b, c):
    return f32(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def _chunk_bounds(Yc, yh, CR=128, sqrt_scale=1.0):
    """Per (query, chunk): the pruned screen's bound U, with the chunk
    statistics and the bound emulated in float32 as the kernels compute them,
    and the largest screened score of the chunk's rows.  Adversarial
    directions: row scores carry the worst float32 accumulation error of 64
    terms upwards, the centroid score downwards, and the hardware square root
    is taken 4 ulps above the correctly rounded root (times sqrt_scale; the
    instruction errs by about one ulp, the kernel's factor 1 - 2^-19 absorbs
    it).  Also returns the bound's 2^-12 margin term.  Yc: float32 candidate
    rows in packed order; yh: the queries' bf16 rows (float64)."""
    nc = Yc.shape[0]
    hi = bf16(Yc)
    lo = bf16(f32(Yc - hi))
    ny2c = np.zeros(nc, np.float32)
    for c in range(30):
        ny2c = f32(Yc[:, c].astype(np.float64) ** 2 + ny2c.astype(np.float64))
    cc = f32(-0.5 * ny2c)
    chi = bf16(cc)
    clo = bf16(f32(cc - chi))
    yt = f32(hi + lo)                                              # y~ = hi + lo (exact)
    h = f32(-(chi + clo))
    n = np.zeros(yh.shape[0], np.float32)
    for c in range(30):
        n = _fma32(yh[:, c], yh[:, c], n)
    MRG = np.float32(2.0 ** -12)
    SQ_LO = np.float32(1.0 - 2.0 ** -19)
    ga = f32(n - f32(MRG * n))
    ub = f32(f32(f32(np.float32(0.5) * n) * np.float32(1.0 + 1e-6)) + f32(MRG * n))
    rows = hi.astype(np.float64) + lo.astype(np.float64)
    t = yh @ rows.T + (chi.astype(np.float64) + clo.astype(np.float64))[None, :]
    acc = np.abs(yh) @ (np.abs(hi.astype(np.float64)) + np.abs(lo.astype(np.float64))).T \
        + (np.abs(chi.astype(np.float64)) + np.abs(clo.astype(np.float64)))[None, :]
    t_up = t + 64 * U * acc
    Ubs, worsts, margins = [], [], []
    for k0 in range(0, nc, CR):
        sl = slice(k0, k0 + CR)
        y, hh = yt[sl], h[sl]
        mean = f32(y.astype(np.float64).sum(0) / len(y))
        mh = bf16(mean)
        ml = bf16(f32(mean - mh))
        mu = f32(mh + ml)
        mu2 = np.float32(0)
        for c in range(30):
            mu2 = _fma32(mu[c], mu[c], mu2)
        d2 = np.zeros(len(y), np.float32)
        n2f = np.zeros(len(y), np.float32)
        for c in range(30):
            d = f32(y[:, c] - mu[c])
            d2 = _fma32(d, d, d2)
            n2f = _fma32(y[:, c], y[:, c], n2f)
        n2 = (y.astype(np.float64) ** 2).sum(1)
        rho = f32(f32(np.sqrt(d2).max() * np.float32(1.0 + 1e-6)) + np.float32(1e-30))
        df = np.float32((0.5 * n2 - hh.astype(np.float64)).max())
        df = f32(df + f32(abs(df) * np.float32(2.4e-7)) + np.float32(1e-30))
        sz = f32(f32(n2f.max() + hh.max()) * np.float32(1.0 + 1e-6))
        sw = f32(mu2 * np.float32(1.0 + 1e-6))
        ccc = f32(np.float32(-0.5) * mu2)
        cchi = bf16(ccc)
        cclo = bf16(f32(ccc - cchi))
        mrow = mh.astype(np.float64) + ml.astype(np.float64)
        tc = yh @ mrow + float(cchi) + float(cclo)
        tc_acc = np.abs(yh) @ (np.abs(mh.astype(np.float64)) + np.abs(ml.astype(np.float64))) \
            + abs(float(cchi)) + abs(float(cclo))
        tc = f32(tc - 64 * U * tc_acc)
        cw = f32(MRG * sw)
        cy = f32(df + f32(MRG * sz))
        g2 = _fma32(np.float32(-2.0), tc, f32(ga - cw))
        sq = f32(_up(np.sqrt(np.maximum(g2, np.float32(0))), 4) * np.float32(sqrt_scale))
        L = np.maximum(_fma32(sq, SQ_LO, -rho), np.float32(0))
        Ubs.append(_fma32(np.float32(-0.5 * (1.0 - 1e-6)), f32(L * L), f32(ub + cy)).astype(np.float64))
        worsts.append(t_up[:, sl].max(1))
        margins.append(float(MRG) * (n.astype(np.float64) + float(sz)))
    return np.array(Ubs).T, np.array(worsts).T, np.array(margins).T


@pytest.mark.parametrize("kind", ["histogram", "peaked", "near-duplicate"])
def test_chunk_bound(kind):
    """The pruned screen's bound on each 128-row chunk stays above every
    screened score of the chunk's rows, for every query (realistic rows in a
    key order, as packed)."""
    rng = np.random.default_rng({"histogram": 11, "peaked": 12, "near-duplicate": 13}[kind])
    nq, nc = 160, 1536
    if kind == "near-duplicate":
        base = descriptors(rng, 48, "histogram").astype(np.float64)
        X = np.repeat(base, (nq + nc) // 48 + 1, axis=0)[: nq + nc]
        X *= 1 + 1e-5 * rng.standard_normal(X.shape)
        for k in range(3):
            X[:, NB * k:NB * (k + 1)] /= X[:, NB * k:NB * (k + 1)].sum(1, keepdims=True)
        X = f32(X)
    else:
        X = descriptors(rng, nq + nc, kind)
    m = f32(helmert64(X[:256]).mean(0))
    Y = f32(helmert32(X) - m)
    Yc = Y[nq:]
    Yc = Yc[np.argsort(Yc[:, 0] + 0.5 * Yc[:, 1], kind="stable")]
    yh = bf16(Y[:nq]).astype(np.float64)
    Ub, worst, _ = _chunk_bounds(Yc, yh)
    assert Ub.shape == (nq, nc // 128)
    assert (Ub >= worst).all(), float((worst - Ub).max())


def test_chunk_bound_tight():
    """Near-equality cases: each chunk is a ball of radius r around a centre
    with one row on the ball towards the queries, which sit on that ray outside
    the ball, so the nearest row's score comes within the bound's margins of
    it.  The bound holds there, and a square root overstated by 2^-9 breaks it:
    the test resolves errors of that size."""
    rng = np.random.default_rng(21)
    nchunk, CR, nqk = 8, 128, 6
    base = helmert64(descriptors(rng, nchunk, "histogram").astype(np.float64))
    rows, queries, owner = [], [], []
    for k in range(nchunk):
        mu = base[k] - base.mean(0)
        v = rng.standard_normal(30)
        v /= np.linalg.norm(v)
        r = 0.05 * np.linalg.norm(mu) + 1e-3
        u = rng.standard_normal((CR - 1, 30))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        rows.append(np.vstack([mu + u * (r * rng.random((CR - 1, 1))), mu + r * v]))
        for D in np.linspace(1.2, 20.0, nqk):
            queries.append(mu + D * r * v)
            owner.append(k)
    Yc = f32(np.vstack(rows))
    yh = bf16(f32(np.array(queries))).astype(np.float64)
    own = (np.arange(len(owner)), np.array(owner))
    Ub, worst, margin = _chunk_bounds(Yc, yh)
    assert (Ub >= worst).all()
    gap = (Ub - worst)[own]
    assert (gap <= 4 * margin[own]).all(), float((gap / margin[own]).max())
    Ub_over, _, _ = _chunk_bounds(Yc, yh, sqrt_scale=1.0 + 2.0 ** -9)
    assert (Ub_over[own] < worst[own]).any()
