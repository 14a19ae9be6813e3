"""Test helpers: accuracy metrics, textbook reference solvers and the eigenvector
comparison rule used by every parity test.

Nothing here is imported by the product path.

Tolerances (eps = 2^-52, ||T|| = 1-norm):
* eigenvalues:   |lambda - lambda_ref| <= 2 n eps ||T||
* residual:      max_j ||T z_j - lambda_j z_j||_2 / (n eps ||T||) <= 10
* orthogonality: max |Z^T Z - I| / (max(n, 1/tol) eps) <= 10, tol = 1e-3: the
  spec bar 10 n eps for n >= 1000 (every full-size case).  Below that the
  constant is floored at 1/tol: a singleton's vector is solved at a shift that
  is exact only to rounding, eps |lambda|, so its component along the nearest
  other eigenvector is of order eps |lambda| / gap = eps / relgap, and the
  method accepts singletons down to relgap = tol (Sec. 3.1.1 classification,
  Eq. errorangle).  For n < 1/tol that floor exceeds n eps whatever the
  implementation: measured max|Z^T Z - I| / (n eps), GPU and oracle, on the
  small cases of tests/test_gpu_parity.py: Wilkinson W21+ 60.2 and 8.9, two
  glued W21+ 22.1 and 3.7, three glued 12.8 and 9.4, graded 12.3 and 5.5, all
  others below 10 for both.
* vectors:       per group G of eigenvalues not separated by the Davis-Kahan
  threshold, the largest principal angle between span Z_ref[:, G] and
  span Z[:, G] has sin <= sin(theta_G) with
  sin(theta_G) = min(1, 20 n eps ||T|| / outer_gap(G)); groups whose bound
  exceeds 0.5 are "parity unpinned" (residual/orthogonality only).
"""
import numpy as np

EPS = np.finfo(np.float64).eps
RELGAP_TOL = 1e-3


def dense(d, e):
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    return np.diag(d) + np.diag(e[: len(d) - 1], 1) + np.diag(e[: len(d) - 1], -1)


def norm1(d, e):
    d = np.abs(np.asarray(d, dtype=np.float64))
    n = d.shape[0]
    c = d.copy()
    if n > 1:
        ea = np.abs(np.asarray(e, dtype=np.float64)[: n - 1])
        c[:-1] += ea
        c[1:] += ea
    return float(c.max()) if n else 0.0


def tmatvec(d, e, Z):
    """T @ Z for tridiagonal T without forming it."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)[: len(d) - 1]
    Y = d[:, None] * Z
    if len(d) > 1:
        Y[:-1] += e[:, None] * Z[1:]
        Y[1:] += e[:, None] * Z[:-1]
    return Y


def residual_ratio(d, e, w, Z):
    n = len(d)
    if Z.shape[1] == 0:
        return 0.0
    R = tmatvec(d, e, Z) - Z * w[None, :]
    return float(np.linalg.norm(R, axis=0).max() / (n * EPS * max(norm1(d, e), np.finfo(float).tiny)))


def orth_ratio(Z):
    n = Z.shape[0]
    m = Z.shape[1]
    if m == 0:
        return 0.0
    G = Z.T @ Z - np.eye(m)
    return float(np.abs(G).max() / (max(n, 1.0 / RELGAP_TOL) * EPS))


def eig_tol(d, e):
    return 2.0 * len(d) * EPS * norm1(d, e)


def sturm_counts_T(d, e, taus):
    """Number of eigenvalues of T below each tau (Sylvester inertia of T - tau I
    through the LDL^T pivots q_i = d_i - tau - e_{i-1}^2 / q_{i-1}), vectorized
    over the shifts."""
    d = np.asarray(d, dtype=np.float64)
    e2 = np.asarray(e, dtype=np.float64)[: len(d) - 1] ** 2
    taus = np.asarray(taus, dtype=np.float64)
    pivmin = np.finfo(np.float64).tiny * max(1.0, float(e2.max()) if e2.size else 1.0)
    q = d[0] - taus
    q = np.where(np.abs(q) < pivmin, -pivmin, q)
    c = (q < 0).astype(np.int64)
    for i in range(1, len(d)):
        q = (d[i] - taus) - e2[i - 1] / q
        q = np.where(np.abs(q) < pivmin, -pivmin, q)
        c += q < 0
    return c


def jacobi_eigh(A, max_sweeps=60):
    """Cyclic Jacobi eigenvalue algorithm (textbook, e.g. Golub & Van Loan 8.5)
    for a small dense symmetric matrix.  Returns ascending (w, V)."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    scale = np.abs(A).max() if n else 0.0
    for _ in range(max_sweeps):
        off = np.sqrt(np.sum(np.tril(A, -1) ** 2))
        if off <= 1e-18 * max(scale, np.finfo(float).tiny) or off == 0.0:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0.0:
                    continue
                theta = (A[q, q] - A[p, p]) / (2.0 * apq)
                if abs(theta) > 1e150:
                    t = 0.5 / theta
                elif theta != 0:
                    t = np.sign(theta) / (abs(theta) + np.sqrt(theta * theta + 1.0))
                else:
                    t = 1.0
                c = 1.0 / np.sqrt(t * t + 1.0)
                s = t * c
                Ap = A[:, p].copy()
                Aq = A[:, q].copy()
                A[:, p] = c * Ap - s * Aq
                A[:, q] = s * Ap + c * Aq
                Ap = A[p, :].copy()
                Aq = A[q, :].copy()
                A[p, :] = c * Ap - s * Aq
                A[q, :] = s * Ap + c * Aq
                Vp = V[:, p].copy()
                Vq = V[:, q].copy()
                V[:, p] = c * Vp - s * Vq
                V[:, q] = s * Vp + c * Vq
    w = np.diag(A).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def sign_normalize(Z):
    """Largest-magnitude entry of each column positive (ties: smallest index)."""
    Z = np.array(Z, dtype=np.float64, copy=True)
    if Z.size == 0:
        return Z
    idx = np.argmax(np.abs(Z), axis=0)
    sgn = np.sign(Z[idx, np.arange(Z.shape[1])])
    sgn[sgn == 0] = 1.0
    return Z * sgn[None, :]


def vector_groups(w, tnorm, n):
    """Split indices into groups of eigenvalues whose consecutive gaps fall below
    the Davis-Kahan threshold (bound > 1e-2); return (groups, outer gaps)."""
    m = len(w)
    thr = 20.0 * n * EPS * tnorm / 1e-2
    groups = []
    start = 0
    for j in range(m - 1):
        if w[j + 1] - w[j] >= thr:
            groups.append((start, j))
            start = j + 1
    if m:
        groups.append((start, m - 1))
    outs = []
    for a, b in groups:
        gl = w[a] - w[a - 1] if a > 0 else np.inf
        gr = w[b + 1] - w[b] if b < m - 1 else np.inf
        outs.append(min(gl, gr))
    return groups, outs


def compare_vectors(d, e, w_ref, Z_ref, Z, full_w=None, sel=None):
    """Check Z against Z_ref group by group; returns (worst ratio, #groups
    checked, #groups unpinned).  A ratio <= 1 passes.  For a subset, pass the
    full spectrum full_w and the selected indices sel (ascending): groups are
    formed on the full spectrum and a group cut by the subset is unpinned."""
    n = len(d)
    tn = norm1(d, e)
    if full_w is None:
        full_w = np.asarray(w_ref)
        sel = np.arange(len(full_w))
    sel = np.asarray(sel)
    pos = {int(s): k for k, s in enumerate(sel)}
    groups, outs = vector_groups(full_w, tn, n)
    worst = 0.0
    checked = unpinned = 0
    for (a, b), go in zip(groups, outs):
        members = [pos.get(i) for i in range(a, b + 1)]
        if all(m is None for m in members):
            continue
        bound = min(1.0, 20.0 * n * EPS * tn / go) if go > 0 else 1.0
        if bound > 0.5 or any(m is None for m in members):
            unpinned += 1
            continue
        cols = np.array(members)
        Zr = Z_ref[:, cols]
        Zg = Z[:, cols]
        Rm = Zg - Zr @ (Zr.T @ Zg)      # component outside the reference subspace
        sin_est = float(np.linalg.norm(Rm, 2))
        worst = max(worst, sin_est / max(bound, 1e-300))
        checked += 1
    return worst, checked, unpinned
