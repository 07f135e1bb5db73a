"""GPU parity of the dense surface correction (Sec. VI, eq. 7) against the
oracle, through the C ABI: observation counts and output slots exact, kept
positions and normals within one float32 ulp plus 1e-12 (the FP64 sums
differ only in rounding order), on the map recipe at several sizes (ragged tails of the
256-surfel blocks), at the benchmark's size, and on edge cases: no surfels,
no keyframes, an observation exactly on the image border, equal time stamps,
and unsorted keyframes (rejected)."""
import numpy as np
import pytest
import torch

from gpu_helpers import dev
from synth.surfels import CAMERA, make_surfel_map

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_1801_01572_amd as lsr
    lsr.lib()
    return lsr


def _close(g, o):
    """Kept surfels: the FP64 sums differ only in rounding order (at most 64
    terms of magnitude <= 10 m, or <= 1 for normals: a few 1e-13 apart), then
    round to float32: within one float32 ulp plus 1e-12 absolute."""
    g = np.asarray(g, np.float64)
    o32 = np.asarray(o, np.float32)
    err = np.abs(g - o32.astype(np.float64))
    bound = np.spacing(np.abs(o32)).astype(np.float64) + 1e-12
    return float((err / bound).max())


def _run(L, orc, S, t0, tu, To, Tn, tk, cam):
    out, idx, k, m = L.surfel_correct(dev(S), dev(t0), dev(tu), To, Tn, tk, cam)
    o_out, o_idx, o_k = orc.surfel_correct(S, t0, tu, To, Tn, tk, cam)
    assert np.array_equal(k.cpu().numpy(), o_k)
    assert np.array_equal(idx.cpu().numpy(), o_idx)
    assert m == o_out.shape[1]
    g = out.cpu().numpy()
    if m:
        r = _close(g, o_out)
        if r > 1.0:
            k = np.unravel_index(np.argmax(np.abs(g - o_out) / (np.spacing(np.abs(o_out)) + 1e-12)), g.shape)
            raise AssertionError(f"kept surfels differ: {r} at {k}: gpu {g[k]!r} oracle {o_out[k]!r}")
    return g, o_k


@pytest.mark.parametrize("n,n_kf", [(1, 8), (255, 16), (257, 64), (20011, 128), (200000, 256)])
def test_surfel_parity(L, orc, n, n_kf):
    m = make_surfel_map(n, n_kf, seed=1000 + n)
    print(f"surfels n={n} keyframes={n_kf}", flush=True)
    g, k = _run(L, orc, m.S, m.t0, m.tu, m.T_old, m.T_new, m.t_kf, m.camera)
    print(f"  kept {g.shape[1]} of {n}, mean |F| {k.mean():.2f}", flush=True)


def test_surfel_benchmark_size(L, orc):
    m = make_surfel_map(4_000_000, 512)
    print("surfels n=4000000 keyframes=512", flush=True)
    g, k = _run(L, orc, m.S, m.t0, m.tu, m.T_old, m.T_new, m.t_kf, m.camera)
    assert 0.3 < g.shape[1] / 4_000_000 < 0.95


def test_surfel_edge_cases(L, orc):
    cam = dict(CAMERA)
    m = make_surfel_map(300, 32, seed=7)
    # no surfels
    out, idx, k, cnt = L.surfel_correct(dev(m.S[:, :0]), dev(m.t0[:0]), dev(m.tu[:0]), m.T_old, m.T_new, m.t_kf,
                                        cam)
    assert cnt == 0
    # no keyframes: everything removed
    print("surfels: no keyframes", flush=True)
    _run(L, orc, m.S, m.t0, m.tu, m.T_old[:0], m.T_new[:0], m.t_kf[:0], cam)
    # equal time stamps everywhere, windows that start or end on them
    tk = np.full(32, 100, np.int32)
    t0 = np.where(np.arange(300) % 3 == 0, 100, 99).astype(np.int32)
    tu = np.where(np.arange(300) % 5 == 0, 100, 101).astype(np.int32)
    print("surfels: equal time stamps", flush=True)
    _run(L, orc, m.S, t0, tu, m.T_old, m.T_new, tk, cam)
    # exact image-border and depth-limit decisions (fx x + cx z = 0 exactly, etc.)
    cam2 = {"fx": 500.0, "fy": 500.0, "cx": 250.0, "cy": 250.0, "width": 500, "height": 500, "z_min": 0.5,
            "z_max": 4.0}
    pts = np.array([[-1.0, 2.0 ** -20 - 1.0, -1.0 - 2.0 ** -20, 1.0, 1.0 - 2 ** -22, 0.0, 0.0, 0.0, 0.0],
                    [0.0, 0.0, 0.0, 0.0, 0.0, -1.0, 1.0, 0.0, 0.0],
                    [2.0, 2.0, 2.0, 2.0, 2.0, 2.0, 2.0, 0.5, 4.0]])
    S = np.vstack([pts, np.tile([[0.0], [0.0], [-1.0]], (1, pts.shape[1]))]).astype(np.float32)
    G = np.eye(4)
    G[:3, 3] = [0.01, 0.02, 0.03]
    n = S.shape[1]
    print("surfels: border decisions", flush=True)
    g, k = _run(L, orc, S, np.zeros(n, np.int32), np.full(n, 20, np.int32), np.eye(4)[None], G[None],
                np.array([10], np.int32), cam2)
    # u = 0 and v = 0 are inside, u = W (x = 1 at z = 2) and v = H (y = 1) outside, z_min and z_max inside
    assert k.tolist() == [1, 1, 0, 0, 1, 1, 0, 1, 1]
    # unsorted keyframes are refused
    with pytest.raises(Exception):
        L.surfel_correct(dev(m.S), dev(m.t0), dev(m.tu), m.T_old[:2], m.T_new[:2], np.array([5, 4], np.int32),
                         cam)


def test_surfel_repeat_calls_identical(L):
    m = make_surfel_map(50000, 64, seed=3)
    S, t0, tu = dev(m.S), dev(m.t0), dev(m.tu)
    a = [L.surfel_correct(S, t0, tu, m.T_old, m.T_new, m.t_kf, m.camera) for _ in range(2)]
    assert a[0][3] == a[1][3]
    assert torch.equal(a[0][0], a[1][0]) and torch.equal(a[0][1], a[1][1])
