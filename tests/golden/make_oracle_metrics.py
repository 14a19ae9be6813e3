"""Write the oracle's own accuracy figures on full-size matrices to
tests/golden/oracle_metrics.json.

    python tests/golden/make_oracle_metrics.py [name ...]

For each matrix (seeded, from ``paper_1205_2107_amd.workloads``) the CPU oracle
computes every eigenpair; the file records its orthogonality
max|Z^T Z - I| / (n eps) and residual max_j ||T z_j - lambda_j z_j|| / (n eps
||T||_1) (Sec. 2.3, the two accuracy measures), its status and tree statistics.
A GPU test holds the GPU to these figures where the oracle itself does not
reach the 10 n eps bar.  Nothing here runs on the GPU or imports the GPU
library.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

import oracle  # noqa: E402
from paper_1205_2107_amd import workloads as W  # noqa: E402  (input generators only)

MATRICES = {"glued1_n20000": "glued_wilkinson(20000, 1)"}
EPS = np.finfo(np.float64).eps


def make_input(expr):
    return eval(expr, {}, {k: getattr(W, k) for k in dir(W) if not k.startswith("_")})


def metrics(d, e, w, Z):
    n = d.shape[0]
    tn = np.abs(d).max()
    c = np.abs(d).copy()
    c[:-1] += np.abs(e)
    c[1:] += np.abs(e)
    tn = c.max()
    orth = 0.0
    res = 0.0
    step = 2048
    for c0 in range(0, n, step):
        P = Z[:, c0:c0 + step]
        G = P.T @ Z
        G[:, c0:c0 + step] -= np.eye(P.shape[1])
        orth = max(orth, float(np.abs(G).max()))
        TP = d[:, None] * P
        TP[:-1] += e[:, None] * P[1:]
        TP[1:] += e[:, None] * P[:-1]
        res = max(res, float(np.linalg.norm(TP - P * w[None, c0:c0 + step], axis=0).max()))
    return orth / (n * EPS), res / (n * EPS * tn)


def main():
    names = sys.argv[1:] or list(MATRICES)
    path = os.path.join(HERE, "oracle_metrics.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    for name in names:
        d, e = make_input(MATRICES[name])
        t0 = time.time()
        w, Z, st, stats = oracle.mrrr(d, e, return_stats=True)
        t1 = time.time()
        o, r = metrics(d, e, w, Z)
        out[name] = {"expr": MATRICES[name], "status": int(st), "orth": o, "res": r,
                     "stats": {k: int(v) for k, v in stats.items()}, "oracle_seconds": round(t1 - t0, 1)}
        print(name, out[name], flush=True)
        with open(path, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
