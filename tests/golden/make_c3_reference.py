"""Writes tests/golden/c3_building_500k.json: the CPU oracle's whole pipeline on
the building-scale pair (3 x 3 rooms with doorways, two 500,000-point
fragments, 40% overlap; synth recipe 3, pair 0), run once and cached, since
its quadratic descriptor matching takes tens of minutes on a host.

Recorded: the returned transform, status, counts, inlier ratio and the share
of valid rows of each fragment whose descriptor neighbour lies within the
near-tie margin.  Calls only the oracle and the input generator.

    OMP_NUM_THREADS=8 python tests/golden/make_c3_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    t0 = time.time()
    pr = synth.make_pair(3, 0)
    prm = oracle.default_params()
    print(f"pair: {pr.P.shape[1]} / {pr.Q.shape[1]} points ({time.time() - t0:.0f} s)", flush=True)
    nP, *_ = oracle.normals(pr.P, prm.r_normal)
    nQ, *_ = oracle.normals(pr.Q, prm.r_normal)
    F, vF = oracle.fpfh(pr.P[:3], nP, prm.r_feature)[:2]
    G, vG = oracle.fpfh(pr.Q[:3], nQ, prm.r_feature)[:2]
    print(f"descriptors ({time.time() - t0:.0f} s)", flush=True)
    m = oracle.match(F, vF, G, vG)
    print(f"matching ({time.time() - t0:.0f} s)", flush=True)
    tP, tQ = oracle.tie_flags(F, G, m)
    r, nnQ, cons = oracle.register_pair(pr.P, pr.Q, prm)
    d = oracle.result_dict(r)
    print(f"pipeline ({time.time() - t0:.0f} s)", flush=True)
    assert np.array_equal(nnQ, m["nnQ"])
    out = {"recipe": 3, "pair": 0, "points": [int(pr.P.shape[1]), int(pr.Q.shape[1])],
           "T": d["T"].reshape(16).tolist(), "status": int(d["status"]), "n_recip": int(d["n_recip"]),
           "n_consistent": int(d["n_consistent"]), "n_inliers": int(d["n_inliers"]),
           "n_valid_P": int(d["n_valid_P"]), "n_valid_Q": int(d["n_valid_Q"]),
           "inlier_ratio": float(d["inlier_ratio"]),
           "tie_exempt_rows_P": float(tP[vF == 1].mean()), "tie_exempt_rows_Q": float(tQ[vG == 1].mean()),
           "min_inlier_ratio": float(prm.min_inlier_ratio), "min_consistent": int(prm.min_consistent),
           "T_gt": pr.T_gt.reshape(16).tolist(), "oracle_seconds": round(time.time() - t0, 1),
           "threads": int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c3_building_500k.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
