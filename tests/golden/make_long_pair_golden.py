"""Write the oracle value used by the full-size parity test of the long-pair workload.

Exact equivalence used (subdivision invariance of the signature kernel: a
linear segment split into pieces has the same affine interpolant):
    k(x_sub, y) == k(x_coarse, y)
where x_coarse = every 1000th point of the long-pair x path (999 segments) and
x_sub splits each of its segments into 1000 equal pieces (999,001 points).  The
GPU evaluates the left side on ~1e12 cells; the oracle evaluates the right
side on ~1e9 cells.  Only the CPU oracle and the seeded generator are used.

Run:  python tests/golden/make_long_pair_golden.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

STRIDE = 1000


def coarse_x():
    x, y = synth.long_pair()
    return x[::STRIDE].copy(), y


def main():
    xc, y = coarse_x()
    t0 = time.time()
    k, diag = oracle.pair_diag(xc, y)
    dt = time.time() - t0
    out = {
        "description": "oracle k(x_coarse, y) for the long-pair workload; x_coarse = "
                       "long_pair x[::1000] (999 segments), y = long_pair y (1e6 points); "
                       "equals k(x_sub, y) with every coarse segment split into 1000",
        "stride": STRIDE, "coarse_points": int(len(xc)), "y_points": int(len(y)),
        "k": k, "oracle_seconds": round(dt, 1), "max_series_length": int(diag[3]),
        "corner_mismatch": float(diag[0]),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_pair_coarse.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
