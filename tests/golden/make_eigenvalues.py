"""Write the oracle's eigenvalues of the full-size test matrices to tests/golden/.

    python tests/golden/make_eigenvalues.py [--procs P] [name ...]

Each file ``eigvals_<name>.npy`` holds every eigenvalue (ascending, float64) of
one seeded matrix from ``paper_1205_2107_amd.workloads``, computed by the CPU
oracle alone (``oracle.mrrr`` with an index range and no vectors: bisection on
the root representation to full relative accuracy, Sec. 3.1.1).  The index
range is cut into P contiguous pieces solved in separate processes; each piece
is an ordinary oracle call.  ``eigvals_manifest.json`` records, per matrix, the
order, the generator call and the SHA-256 of the input bytes (d then e), so a
test can tell when a generator no longer produces the matrix the file was
written for.

Nothing here runs on the GPU or imports the GPU library.
"""
import argparse
import hashlib
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1205_2107_amd import workloads as W  # noqa: E402  (input generators only)

# name -> (generator expression, order); the expressions are evaluated against
# the workloads module and are recorded verbatim in the manifest
MATRICES = {
    "c2_random_n20000": ("random_uniform(20000, 2001)", 20000),
    "c2_toeplitz_n20000": ("toeplitz(20000)", 20000),
    "c2_geometric_n20000": ("geometric(20000, 2003)", 20000),
    "glued1_n20000": ("glued_wilkinson(20000, 1)", 20000),
    "c3_glued_n60000": ("glued_wilkinson(60000, 3001)", 60000),
}


def make_input(expr):
    return eval(expr, {}, {k: getattr(W, k) for k in dir(W) if not k.startswith("_")})


def input_sha256(d, e):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(d, dtype="<f8").tobytes())
    h.update(np.ascontiguousarray(e, dtype="<f8").tobytes())
    return h.hexdigest()


def _piece(args):
    expr, il, iu = args
    import oracle
    d, e = make_input(expr)
    w, _, st = oracle.mrrr(d, e, kind=oracle.RANGE_INDEX, il=il, iu=iu, vectors=False)
    if st != 0:
        raise RuntimeError(f"oracle status {st} on {expr} [{il}, {iu}]")
    return il, w


def write(name, procs):
    expr, n = MATRICES[name]
    d, e = make_input(expr)
    assert d.shape[0] == n
    cuts = np.linspace(0, n, procs + 1).round().astype(int)
    jobs = [(expr, int(cuts[k]) + 1, int(cuts[k + 1])) for k in range(procs) if cuts[k + 1] > cuts[k]]
    t0 = time.time()
    w = np.empty(n)
    with Pool(len(jobs)) as pool:
        for il, piece in pool.imap_unordered(_piece, jobs):
            w[il - 1:il - 1 + piece.shape[0]] = piece
    assert np.all(np.diff(w) >= 0), "pieces out of order"
    np.save(os.path.join(HERE, f"eigvals_{name}.npy"), w.astype("<f8"))
    print(f"{name}: n={n} in {time.time() - t0:.0f} s", flush=True)
    return {"expr": expr, "n": n, "input_sha256": input_sha256(d, e), "procs": len(jobs)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("names", nargs="*")
    a = ap.parse_args()
    names = a.names or list(MATRICES)
    man_path = os.path.join(HERE, "eigvals_manifest.json")
    man = json.load(open(man_path)) if os.path.exists(man_path) else {}
    for name in names:
        man[name] = write(name, a.procs)
        with open(man_path, "w") as f:
            json.dump(man, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main()
