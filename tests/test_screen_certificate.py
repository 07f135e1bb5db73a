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
