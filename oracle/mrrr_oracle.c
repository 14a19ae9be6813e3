/*
 * oracle/mrrr_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 reference implementation of the MRRR
 * (Multiple Relatively Robust Representations) solver for the real symmetric
 * tridiagonal eigenproblem T z = lambda z, as described in Petschow, Peise and
 * Bientinesi, "High-Performance Solvers for Dense Hermitian Eigenproblems"
 * (arXiv:1205.2107), Sec. 3.1 and Sec. 3.1.1.  Only the test suite, the package
 * smoke check and the benchmark's CPU-baseline leg load this library; the GPU
 * library shares no code, header or constant with it.
 *
 * The steps, in the order Sec. 3.1.1 gives them:
 *   - split T where an off-diagonal is negligible (footnote of Sec. 3.1.1:
 *     threshold eps*||T||, read here with the 1-norm);
 *   - root representation L0 D0 L0^T = T - sigma I with T - sigma I definite;
 *   - every wanted eigenvalue by bisection with Sturm counts on L D L^T, to high
 *     relative accuracy;
 *   - classification: lambda_j is a singleton when its relative gap exceeds
 *     tol = 1e-3 (footnote of Sec. 3.1.1), otherwise it belongs to a cluster;
 *   - singleton: twisted factorization and one step of inverse iteration with a
 *     near-optimal right-hand side e_r (eq. errorangle), with a Rayleigh
 *     quotient correction of lambda;
 *   - cluster: child representation L_c D_c L_c^T = L D L^T - sigma_c I with
 *     sigma_c close to an end of the cluster, refine the cluster's eigenvalues
 *     against it, reclassify, recurse.
 * Accuracy contract (Sec. 2.3, Eq. Tresnorm / Eq. Torthogo): residual
 * O(n eps ||T||), orthogonality O(n eps).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no FMA
 * contraction, so every operation is one correctly rounded IEEE operation).
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define EPS DBL_EPSILON           /* machine epsilon 2^-52 */
#define SAFMIN DBL_MIN            /* smallest normal number */
#define RELGAP_TOL 1.0e-3         /* classification threshold, Sec. 3.1.1 footnote */
#define MAX_DEPTH 64              /* representation-tree depth limit */
#define MAX_BISECT 128            /* bisection step cap per eigenvalue */
#define MAX_RQI 10                /* Rayleigh-quotient iterations per singleton */
#define GROWTH_BOUND 8.0          /* child accepted if max|D_c| <= 8 * spdiam */
#define CHILD_TRIES 2             /* shift margins tried at each cluster end */
#define PERT_SCALE 4.0            /* root perturbation: relative 4*eps*u, u in [-1,1] */

enum { ST_OK = 0, ST_NO_RRR = 1, ST_DEPTH = 2, ST_QUEUE = 3, ST_NONFINITE = 4, ST_NOMEM = 5 };
enum { RANGE_ALL = 0, RANGE_INDEX = 1, RANGE_VALUE = 2 };
/* statistics slots (int64 each) */
enum {
  STAT_NODES = 0,     /* child representations built */
  STAT_MAXDEPTH = 1,  /* deepest node */
  STAT_STURM = 2,     /* Sturm-count steps executed (one per matrix row) */
  STAT_RQI = 3,       /* twisted factorizations executed */
  STAT_FALLBACK = 4,  /* singletons that left the RQI loop unconverged */
  STAT_CHILDTRY = 5,  /* child candidates evaluated */
  STAT_SINGLETONS = 6,
  STAT_CLUSTERS = 7,
  NSTAT = 8
};

/* ------------------------------------------------------------------------- */
/* counter-based random numbers: SplitMix64 finalizer (Steele, Lea, Flood 2014) */

static uint64_t splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* uniform in [-1, 1): top 53 bits scaled */
static double unit_sym(uint64_t seed, uint64_t counter) {
  double u = (double)(splitmix64_at(seed, counter) >> 11) * (1.0 / 9007199254740992.0);
  return 2.0 * u - 1.0;
}

/* ------------------------------------------------------------------------- */
/* representation L D L^T of one unreduced block */

typedef struct {
  int64_t n;
  double *D, *L, *LD, *LLD; /* D[n], L[n-1], LD = L*D, LLD = L*L*D */
  double acc;               /* root shift + child shifts, added root to leaf */
  int depth;
} rep_t;

static int rep_alloc(rep_t* r, int64_t n) {
  r->n = n;
  r->D = (double*)calloc((size_t)(4 * n + 4), sizeof(double));
  if (!r->D) return 0;
  r->L = r->D + n + 1;
  r->LD = r->L + n + 1;
  r->LLD = r->LD + n + 1;
  r->acc = 0.0;
  r->depth = 0;
  return 1;
}

static void rep_free(rep_t* r) {
  free(r->D);
  r->D = r->L = r->LD = r->LLD = NULL;
}

static void rep_products(rep_t* r) {
  for (int64_t i = 0; i + 1 < r->n; i++) {
    r->LD[i] = r->L[i] * r->D[i];
    r->LLD[i] = r->LD[i] * r->L[i];
  }
}

/* ------------------------------------------------------------------------- */
/* Sturm counts */

/* number of eigenvalues of T (diagonal d, squared off-diagonals e2) below tau:
 * negative pivots of T - tau I = L D L^T computed by the plain recurrence
 * q_1 = d_1 - tau, q_i = d_i - tau - e_{i-1}^2 / q_{i-1}; a pivot smaller than
 * pivmin in magnitude is replaced by -pivmin. */
static int64_t count_T(int64_t n, const double* d, const double* e2, double tau, double pivmin) {
  int64_t c = 0;
  double q = d[0] - tau;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) c++;
  for (int64_t i = 1; i < n; i++) {
    q = (d[i] - tau) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) c++;
  }
  return c;
}

/* number of eigenvalues of L D L^T below tau: negative entries of D+ in
 * L D L^T - tau I = L+ D+ L+^T, by the stationary qds transform
 * s_1 = -tau, D+_i = D_i + s_i, s_{i+1} = (s_i / D+_i) * LLD_i - tau.
 * Tiny pivots become -pivmin; an undefined ratio (inf/inf) is taken as 1. */
static int64_t count_ldl(const rep_t* r, double tau, double pivmin, int64_t* st) {
  int64_t c = 0;
  double s = -tau;
  const int64_t n = r->n;
  for (int64_t i = 0; i + 1 < n; i++) {
    double dp = r->D[i] + s;
    if (fabs(dp) < pivmin) dp = -pivmin;
    if (dp < 0.0) c++;
    double t = s / dp;
    if (t != t) t = 1.0;
    s = t * r->LLD[i] - tau;
  }
  double dp = r->D[n - 1] + s;
  if (fabs(dp) < pivmin) dp = -pivmin;
  if (dp < 0.0) c++;
  if (st) st[STAT_STURM] += n;
  return c;
}

/* bisection for eigenvalue j (1-based) of L D L^T inside [*lo, *hi], keeping
 * count(lo) <= j-1 < count(hi); stops at relative width 2 eps or 128 steps. */
static void bisect_ldl(const rep_t* r, int64_t j, double* lo, double* hi, double pivmin, int64_t* st) {
  double a = *lo, b = *hi;
  for (int it = 0; it < MAX_BISECT; it++) {
    double tol = 2.0 * EPS * fmax(fabs(a), fabs(b));
    if (b - a <= tol) break;
    double mid = 0.5 * (a + b);
    if (mid <= a || mid >= b) break;
    if (count_ldl(r, mid, pivmin, st) <= j - 1)
      a = mid;
    else
      b = mid;
  }
  *lo = a;
  *hi = b;
}

/* widen [*lo, *hi] until count(lo) <= j-1 < count(hi) */
static void ensure_bracket(const rep_t* r, int64_t j, double* lo, double* hi, double pad, double pivmin,
                           int64_t* st) {
  if (!(pad > 0.0)) pad = pivmin;
  double p = pad;
  for (int k = 0; k < 2100 && count_ldl(r, *lo, pivmin, st) > j - 1; k++) {
    *lo -= p;
    p *= 2.0;
  }
  p = pad;
  for (int k = 0; k < 2100 && count_ldl(r, *hi, pivmin, st) < j; k++) {
    *hi += p;
    p *= 2.0;
  }
}

/* ------------------------------------------------------------------------- */
/* one unreduced block */

typedef struct {
  int64_t n;        /* block order */
  const double* d;  /* block diagonal */
  const double* e;  /* block off-diagonal, e[n-1] unused */
  double gl, gu, spdiam, pivmin;
  double* lo;       /* per local index: eigenvalue bracket w.r.t. the current node */
  double* hi;
  int64_t wl, wu;   /* wanted local range, 1-based inclusive */
  double* wout;     /* eigenvalues of wanted indices, wout[j - wl] */
  double* zout;     /* vectors of wanted indices, column j - wl, leading dim ldz (or NULL) */
  int64_t ldz;
  int64_t* st;
  int status;
  double* work;     /* 6n scratch for twisted factorizations */
} block_t;

static void gershgorin(int64_t n, const double* d, const double* e, double* gl, double* gu) {
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t i = 0; i < n; i++) {
    double r = 0.0;
    if (i > 0) r += fabs(e[i - 1]);
    if (i + 1 < n) r += fabs(e[i]);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
  }
  *gl = lo;
  *gu = hi;
}

/* root representation: sigma just outside one end of the spectrum of T, so that
 * T - sigma I is definite and L0 D0 L0^T = T - sigma I is an RRR for all of its
 * eigenvalues (Sec. 3.1.1); the extreme eigenvalue comes from bisection on T. */
static int make_root(block_t* B, int left, uint64_t seed, rep_t* r) {
  const int64_t n = B->n;
  const double* d = B->d;
  const double* e = B->e;
  double* e2 = (double*)malloc((size_t)n * sizeof(double));
  if (!e2) return ST_NOMEM;
  for (int64_t i = 0; i + 1 < n; i++) e2[i] = e[i] * e[i];
  double lo = B->gl, hi = B->gu;
  double pad = 2.0 * (double)n * EPS * fmax(fabs(lo), fabs(hi)) + 2.0 * B->pivmin;
  for (int k = 0; k < 64 && count_T(n, d, e2, lo, B->pivmin) > 0; k++) { lo -= pad; pad *= 2.0; }
  pad = 2.0 * (double)n * EPS * fmax(fabs(lo), fabs(hi)) + 2.0 * B->pivmin;
  for (int k = 0; k < 64 && count_T(n, d, e2, hi, B->pivmin) < n; k++) { hi += pad; pad *= 2.0; }
  const int64_t target = left ? 1 : n;
  for (int it = 0; it < MAX_BISECT; it++) {
    double tol = 2.0 * EPS * fmax(fabs(lo), fabs(hi));
    if (hi - lo <= tol) break;
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_T(n, d, e2, mid, B->pivmin) <= target - 1)
      lo = mid;
    else
      hi = mid;
  }
  free(e2);

  double delta = 4.0 * (double)n * EPS * fmax(fabs(B->gl), fabs(B->gu));
  if (!(delta > 0.0)) delta = B->pivmin;
  int ok = 0;
  double sigma = 0.0;
  for (int tries = 0; tries < 64 && !ok; tries++) {
    sigma = left ? lo - delta : hi + delta;
    ok = 1;
    r->D[0] = d[0] - sigma;
    for (int64_t i = 0; i + 1 < n; i++) {
      r->L[i] = e[i] / r->D[i];
      r->D[i + 1] = (d[i + 1] - sigma) - r->L[i] * e[i];
    }
    for (int64_t i = 0; i < n; i++) {
      double v = r->D[i];
      if (!isfinite(v) || (left ? !(v > 0.0) : !(v < 0.0))) { ok = 0; break; }
    }
    for (int64_t i = 0; ok && i + 1 < n; i++)
      if (!isfinite(r->L[i])) ok = 0;
    delta *= 2.0;
  }
  if (!ok) return ST_NO_RRR;
  /* small deterministic relative perturbation of the root: it breaks exact
   * multiplicities of glued matrices without disturbing the RRR property */
  for (int64_t i = 0; i < n; i++) r->D[i] *= 1.0 + PERT_SCALE * EPS * unit_sym(seed, 2u * (uint64_t)i);
  for (int64_t i = 0; i + 1 < n; i++) r->L[i] *= 1.0 + PERT_SCALE * EPS * unit_sym(seed, 2u * (uint64_t)i + 1u);
  rep_products(r);
  r->acc = sigma;
  r->depth = 0;
  return ST_OK;
}

/* child L_c D_c L_c^T = L D L^T - sigma I by the differential stationary qds
 * transform (mixed relatively stable, Sec. 3.1.1):
 *   s_1 = -sigma, D+_i = D_i + s_i, L+_i = LD_i / D+_i, s_{i+1} = L+_i L_i s_i - sigma.
 * Returns max |D+_i| (inf when something is not finite). */
static double dstqds(const rep_t* p, double sigma, rep_t* c) {
  const int64_t n = p->n;
  double s = -sigma;
  double growth = 0.0;
  int finite = 1;
  for (int64_t i = 0; i + 1 < n; i++) {
    double dp = p->D[i] + s;
    double lp = p->LD[i] / dp;
    c->D[i] = dp;
    c->L[i] = lp;
    s = lp * p->L[i] * s - sigma;
    if (!isfinite(dp) || !isfinite(lp)) finite = 0;
    growth = fmax(growth, fabs(dp));
  }
  c->D[n - 1] = p->D[n - 1] + s;
  if (!isfinite(c->D[n - 1])) finite = 0;
  growth = fmax(growth, fabs(c->D[n - 1]));
  return finite ? growth : INFINITY;
}

/* twisted factorization of L D L^T - lam I, twist index r = argmin |gamma_k|
 * (smallest k on ties), and the solution of (L D L^T - lam I) z = gamma_r e_r
 * with z_r = 1.  Returns gamma_r; z gets the unnormalized vector, *ztz its
 * squared norm.  work holds 3n doubles.  Pivots smaller than pivmin become
 * -pivmin; when a ratio vanishes because its predecessor overflowed, the
 * recurrence takes its limiting value (s_{i+1} = LLD_i - lam, p_i = D_i - lam). */
static double twisted_solve(const rep_t* R, double lam, double pivmin, double* z, int64_t* r_out, double* ztz,
                            double* work) {
  const int64_t n = R->n;
  double* s = work;          /* s_k, stationary transform, s_1 = -lam */
  double* lp = work + n;     /* L+_k */
  double* um = work + 2 * n; /* U-_k */
  double sv = -lam;
  for (int64_t i = 0; i + 1 < n; i++) {
    s[i] = sv;
    double dp = R->D[i] + sv;
    if (fabs(dp) < pivmin) dp = -pivmin;
    lp[i] = R->LD[i] / dp;
    double t = lp[i] * R->L[i] * sv;
    if (lp[i] == 0.0) t = R->LLD[i];
    sv = t - lam;
  }
  s[n - 1] = sv;
  /* progressive transform from the bottom: p_n = D_n - lam,
   * D-_{i+1} = LLD_i + p_{i+1}, t = D_i / D-_{i+1}, U-_i = L_i t, p_i = p_{i+1} t - lam.
   * gamma_k = s_k + p_k + lam. */
  double pv = R->D[n - 1] - lam;
  int64_t r = -1;
  double gmin = INFINITY;
  {
    double g = s[n - 1] + pv + lam;
    if (isfinite(g)) { gmin = g; r = n - 1; }
  }
  for (int64_t i = n - 2; i >= 0; i--) {
    double dm = R->LLD[i] + pv;
    if (fabs(dm) < pivmin) dm = -pivmin;
    double t = R->D[i] / dm;
    um[i] = R->L[i] * t;
    double pn = pv * t - lam;
    if (t == 0.0) pn = R->D[i] - lam;
    pv = pn;
    double g = s[i] + pv + lam;
    if (isfinite(g) && !(fabs(g) > fabs(gmin))) { /* ties go to the smaller index */
      gmin = g;
      r = i;
    }
  }
  if (r < 0) { r = 0; gmin = 0.0; }
  /* z_r = 1; upward z_i = -L+_i z_{i+1}; downward z_{i+1} = -U-_i z_i.
   * A zero entry is stepped over with the row equation of the matrix. */
  z[r] = 1.0;
  double nrm = 1.0;
  for (int64_t i = r - 1; i >= 0; i--) {
    if (z[i + 1] != 0.0 || i + 2 > r)
      z[i] = -lp[i] * z[i + 1];
    else
      z[i] = (R->LD[i] != 0.0) ? -(R->LD[i + 1] / R->LD[i]) * z[i + 2] : 0.0;
    if (!isfinite(z[i])) z[i] = 0.0;
    nrm += z[i] * z[i];
  }
  for (int64_t i = r; i + 1 < n; i++) {
    if (z[i] != 0.0 || i == r)
      z[i + 1] = -um[i] * z[i];
    else
      z[i + 1] = (R->LD[i] != 0.0) ? -(R->LD[i - 1] / R->LD[i]) * z[i - 1] : 0.0;
    if (!isfinite(z[i + 1])) z[i + 1] = 0.0;
    nrm += z[i + 1] * z[i + 1];
  }
  *r_out = r;
  *ztz = nrm;
  return gmin;
}

/* eigenvector of singleton j (1-based) of node R: Rayleigh-quotient iteration on
 * the twisted factorization, started from the bisection value. */
static void singleton_vector(block_t* B, const rep_t* R, int64_t j) {
  const int64_t n = B->n;
  double lo = B->lo[j - 1], hi = B->hi[j - 1];
  double lam = 0.5 * (lo + hi);
  double* z = B->work + 3 * n;
  double gamma = 0.0, ztz = 1.0;
  int64_t r = 0;
  int converged = 0;
  for (int it = 0; it < MAX_RQI; it++) {
    gamma = twisted_solve(R, lam, B->pivmin, z, &r, &ztz, B->work);
    B->st[STAT_RQI]++;
    double resid = fabs(gamma) / sqrt(ztz);
    double corr = gamma / ztz;
    if (resid <= 2.0 * (double)n * EPS * fabs(lam) || fabs(corr) <= 2.0 * EPS * fabs(lam)) {
      converged = 1;
      break;
    }
    double nl = lam + corr;
    if (!(nl >= lo && nl <= hi)) break;
    lam = nl;
  }
  if (!converged) {
    /* fall back to bisection to full accuracy and one final solve */
    B->st[STAT_FALLBACK]++;
    bisect_ldl(R, j, &lo, &hi, B->pivmin, B->st);
    lam = 0.5 * (lo + hi);
    gamma = twisted_solve(R, lam, B->pivmin, z, &r, &ztz, B->work);
    B->st[STAT_RQI]++;
  }
  /* Rayleigh quotient of z with respect to L D L^T */
  double lam_out = lam + gamma / ztz;
  if (!(lam_out >= lo && lam_out <= hi)) lam_out = lam;
  B->wout[j - B->wl] = R->acc + lam_out;
  if (B->zout) {
    double inv = 1.0 / sqrt(ztz);
    int64_t imax = 0;
    double vmax = -1.0;
    for (int64_t i = 0; i < n; i++)
      if (fabs(z[i]) > vmax) { vmax = fabs(z[i]); imax = i; }
    if (z[imax] < 0.0) inv = -inv;
    double* col = B->zout + (j - B->wl) * B->ldz;
    for (int64_t i = 0; i < n; i++) col[i] = z[i] * inv;
  }
}

/* relative-gap classification of the indices f..l (1-based) of a node:
 * a break after j iff lo_{j+1} - hi_j >= tol * max(|lambda_j|, |lambda_{j+1}|). */
static int is_break(const block_t* B, int64_t j) {
  double mj = 0.5 * (B->lo[j - 1] + B->hi[j - 1]);
  double mk = 0.5 * (B->lo[j] + B->hi[j]);
  double gap = B->lo[j] - B->hi[j - 1];
  return gap >= RELGAP_TOL * fmax(fabs(mj), fabs(mk));
}

static int any_wanted(const block_t* B, int64_t a, int64_t b) { return !(b < B->wl || a > B->wu); }

static void process_node(block_t* B, const rep_t* R, int64_t f, int64_t l, double gapf, double gapl);

/* cluster a..b of node P with absolute outer gaps gL (below a) and gR (above b):
 * child representation, refined brackets, recursion.  Candidate shifts sit just
 * outside either end of the cluster (margin max(4 eps |lambda_end|, bracket
 * width)); a second try backs off by min(avgap/2, min(gL, gR)/4).  The first
 * candidate with max|D_c| <= 8 spdiam is taken, otherwise the one with the
 * smallest growth. */
static void process_cluster(block_t* B, const rep_t* P, int64_t a, int64_t b, double gL, double gR) {
  const int64_t n = B->n;
  B->st[STAT_CLUSTERS]++;
  if (P->depth + 1 > MAX_DEPTH) {
    if (B->status == ST_OK) B->status = ST_DEPTH;
    for (int64_t j = a; j <= b; j++)
      if (j >= B->wl && j <= B->wu) singleton_vector(B, P, j);
    return;
  }
  rep_t C, best;
  if (!rep_alloc(&C, n) || !rep_alloc(&best, n)) {
    B->status = ST_NOMEM;
    rep_free(&C);
    return;
  }
  double avgap = (B->hi[b - 1] - B->lo[a - 1]) / (double)(b - a);
  double backoff = fmin(0.5 * avgap, 0.25 * fmin(gL, gR));
  if (!(backoff > 0.0)) backoff = 0.0;
  double best_growth = INFINITY, best_sigma = 0.0;
  int accepted = 0;
  double sigma = 0.0;
  for (int t = 0; t < CHILD_TRIES && !accepted; t++) {
    for (int side = 0; side < 2 && !accepted; side++) {
      int64_t j = side == 0 ? a : b;
      double lo = B->lo[j - 1], hi = B->hi[j - 1];
      double mid = 0.5 * (lo + hi);
      double delta = fmax(4.0 * EPS * fabs(mid), hi - lo) + (double)t * backoff;
      sigma = side == 0 ? lo - delta : hi + delta;
      double g = dstqds(P, sigma, &C);
      B->st[STAT_CHILDTRY]++;
      if (g <= GROWTH_BOUND * B->spdiam) {
        accepted = 1;
      } else if (g < best_growth) {
        best_growth = g;
        best_sigma = sigma;
        memcpy(best.D, C.D, (size_t)(2 * n + 2) * sizeof(double));
      }
    }
  }
  if (!accepted) {
    if (!isfinite(best_growth)) {
      if (B->status == ST_OK) B->status = ST_NO_RRR;
      for (int64_t j = a; j <= b; j++)
        if (j >= B->wl && j <= B->wu) singleton_vector(B, P, j);
      rep_free(&C);
      rep_free(&best);
      return;
    }
    memcpy(C.D, best.D, (size_t)(2 * n + 2) * sizeof(double));
    sigma = best_sigma;
  }
  rep_free(&best);
  rep_products(&C);
  C.acc = P->acc + sigma;
  C.depth = P->depth + 1;
  B->st[STAT_NODES]++;
  if (C.depth > B->st[STAT_MAXDEPTH]) B->st[STAT_MAXDEPTH] = C.depth;
  /* brackets in the child's frame, widened and validated by counts, then
   * refined to full relative accuracy against the child */
  for (int64_t j = a; j <= b; j++) {
    double lo = B->lo[j - 1] - sigma, hi = B->hi[j - 1] - sigma;
    double pad = 4.0 * EPS * (fabs(B->lo[j - 1]) + fabs(B->hi[j - 1]) + fabs(sigma));
    lo -= pad;
    hi += pad;
    ensure_bracket(&C, j, &lo, &hi, pad, B->pivmin, B->st);
    bisect_ldl(&C, j, &lo, &hi, B->pivmin, B->st);
    B->lo[j - 1] = lo;
    B->hi[j - 1] = hi;
  }
  process_node(B, &C, a, b, gL, gR);
  rep_free(&C);
}

/* classify indices f..l of node R into singletons and clusters, then handle
 * each (singletons directly, clusters through a child representation).  gapf
 * and gapl are the absolute gaps from f and l to the nearest eigenvalues outside
 * the node's range.  All run boundaries and gaps are taken before any run is
 * processed, because processing a cluster re-expresses its brackets in the
 * child's frame. */
static void process_node(block_t* B, const rep_t* R, int64_t f, int64_t l, double gapf, double gapl) {
  int64_t nruns = 0;
  int64_t* starts = (int64_t*)malloc((size_t)(l - f + 2) * sizeof(int64_t));
  double* gaps = (double*)malloc((size_t)(l - f + 2) * sizeof(double));
  if (!starts || !gaps) { free(starts); free(gaps); B->status = ST_NOMEM; return; }
  gaps[0] = gapf;
  starts[nruns++] = f;
  for (int64_t j = f; j < l; j++)
    if (is_break(B, j)) {
      gaps[nruns] = B->lo[j] - B->hi[j - 1];
      starts[nruns++] = j + 1;
    }
  starts[nruns] = l + 1;
  gaps[nruns] = gapl;
  for (int64_t k = 0; k < nruns; k++) {
    int64_t a = starts[k], b = starts[k + 1] - 1;
    if (!any_wanted(B, a, b)) continue;
    if (a == b) {
      B->st[STAT_SINGLETONS]++;
      singleton_vector(B, R, a);
    } else {
      process_cluster(B, R, a, b, gaps[k], gaps[k + 1]);
    }
  }
  free(starts);
  free(gaps);
}

/* solve one unreduced block for its wanted local range [wl, wu] */
static int solve_block(block_t* B, int left, uint64_t seed) {
  const int64_t n = B->n;
  if (B->wl > B->wu) return ST_OK;
  if (n == 1) {
    B->wout[0] = B->d[0];
    if (B->zout) B->zout[0] = 1.0;
    return ST_OK;
  }
  rep_t R;
  if (!rep_alloc(&R, n)) return ST_NOMEM;
  int s = make_root(B, left, seed, &R);
  if (s != ST_OK) { rep_free(&R); return s; }
  /* common starting bracket for every index, validated once by counts */
  double glo = B->gl - R.acc, ghi = B->gu - R.acc;
  double pad = 2.0 * (double)n * EPS * fmax(fabs(B->gl), fabs(B->gu)) + 2.0 * B->pivmin;
  glo -= pad;
  ghi += pad;
  for (int k = 0; k < 64 && count_ldl(&R, glo, B->pivmin, B->st) > 0; k++) { glo -= pad; pad *= 2.0; }
  for (int k = 0; k < 64 && count_ldl(&R, ghi, B->pivmin, B->st) < n; k++) { ghi += pad; pad *= 2.0; }
  for (int64_t j = B->wl; j <= B->wu; j++) {
    B->lo[j - 1] = glo;
    B->hi[j - 1] = ghi;
    bisect_ldl(&R, j, &B->lo[j - 1], &B->hi[j - 1], B->pivmin, B->st);
  }
  if (!B->zout) {
    for (int64_t j = B->wl; j <= B->wu; j++) B->wout[j - B->wl] = R.acc + 0.5 * (B->lo[j - 1] + B->hi[j - 1]);
    rep_free(&R);
    return ST_OK;
  }
  /* widen the computed range over clusters cut by the wanted range */
  int64_t f = B->wl, l = B->wu;
  while (f > 1) {
    int64_t j = f - 1;
    B->lo[j - 1] = glo;
    B->hi[j - 1] = ghi;
    bisect_ldl(&R, j, &B->lo[j - 1], &B->hi[j - 1], B->pivmin, B->st);
    if (is_break(B, j)) break;
    f = j;
  }
  while (l < n) {
    int64_t j = l + 1;
    B->lo[j - 1] = glo;
    B->hi[j - 1] = ghi;
    bisect_ldl(&R, j, &B->lo[j - 1], &B->hi[j - 1], B->pivmin, B->st);
    if (is_break(B, l)) break;
    l = j;
  }
  double gapf = (f > 1) ? B->lo[f - 1] - B->hi[f - 2] : INFINITY;
  double gapl = (l < n) ? B->lo[l] - B->hi[l - 1] : INFINITY;
  B->status = ST_OK;
  process_node(B, &R, f, l, gapf, gapl);
  rep_free(&R);
  return B->status;
}

/* ------------------------------------------------------------------------- */
/* driver */

typedef struct {
  double w;
  int64_t blk;
  int64_t j;   /* local 1-based index */
  int64_t pos; /* position in the block's output */
} item_t;

static int cmp_item(const void* x, const void* y) {
  const item_t* a = (const item_t*)x;
  const item_t* b = (const item_t*)y;
  if (a->w < b->w) return -1;
  if (a->w > b->w) return 1;
  if (a->blk != b->blk) return a->blk < b->blk ? -1 : 1;
  if (a->j != b->j) return a->j < b->j ? -1 : 1;
  return 0;
}

/*
 * oracle_mrrr: eigenpairs of the symmetric tridiagonal T (diagonal d[n],
 * off-diagonal e[n-1]) for kind 0 = all, 1 = indices il..iu (1-based, inclusive),
 * 2 = values in (vl, vu].  w[m] ascending; Z (n x m, column-major, leading
 * dimension ldz) gets the matching unit eigenvectors, zero outside their split
 * block, largest-magnitude entry positive.  Z == NULL computes values only.
 * Returns a negative argument index on bad arguments, else a status:
 * 0 ok, 1 no acceptable child representation, 2 depth limit, 4 non-finite input,
 * 5 out of host memory.  stats (NSTAT int64, may be NULL) receives counters.
 */
int oracle_mrrr(int64_t n, const double* d, const double* e, int kind, int64_t il, int64_t iu, double vl,
                double vu, double* w, double* Z, int64_t ldz, int64_t* m_out, int64_t* stats) {
  int64_t stloc[NSTAT];
  memset(stloc, 0, sizeof(stloc));
  int64_t* st = stats ? stats : stloc;
  memset(st, 0, NSTAT * sizeof(int64_t));
  if (m_out) *m_out = 0;
  if (n < 0) return -1;
  if (n > 0 && !d) return -2;
  if (n > 1 && !e) return -3;
  if (kind < 0 || kind > 2) return -4;
  if (kind == RANGE_INDEX && n > 0 && (il < 1 || il > iu || iu > n)) return -5;
  if (kind == RANGE_VALUE && !(vl < vu)) return -7;
  if (!w && n > 0) return -9;
  if (Z && ldz < (n > 1 ? n : 1)) return -11;
  if (n == 0) return ST_OK;
  for (int64_t i = 0; i < n; i++)
    if (!isfinite(d[i])) return ST_NONFINITE;
  for (int64_t i = 0; i + 1 < n; i++)
    if (!isfinite(e[i])) return ST_NONFINITE;

  /* scaled copies (power of two, exact) when entries are extreme */
  double* ds = (double*)malloc((size_t)n * sizeof(double));
  double* es = (double*)calloc((size_t)n, sizeof(double));
  if (!ds || !es) { free(ds); free(es); return ST_NOMEM; }
  double tmax = 0.0;
  for (int64_t i = 0; i < n; i++) tmax = fmax(tmax, fabs(d[i]));
  for (int64_t i = 0; i + 1 < n; i++) tmax = fmax(tmax, fabs(e[i]));
  double scale = 1.0;
  if (tmax > 0.0 && (tmax < ldexp(1.0, -500) || tmax > ldexp(1.0, 500))) scale = ldexp(1.0, -ilogb(tmax));
  for (int64_t i = 0; i < n; i++) ds[i] = d[i] * scale;
  for (int64_t i = 0; i + 1 < n; i++) es[i] = e[i] * scale;
  double svl = vl * scale, svu = vu * scale;

  /* 1-norm and splitting */
  double tnorm = 0.0;
  for (int64_t i = 0; i < n; i++) {
    double c = fabs(ds[i]);
    if (i > 0) c += fabs(es[i - 1]);
    if (i + 1 < n) c += fabs(es[i]);
    tnorm = fmax(tnorm, c);
  }
  int64_t nblk = 0;
  int64_t* bstart = (int64_t*)malloc((size_t)(n + 1) * sizeof(int64_t));
  bstart[nblk++] = 0;
  for (int64_t i = 0; i + 1 < n; i++) {
    if (fabs(es[i]) <= EPS * tnorm) {
      es[i] = 0.0;
      bstart[nblk++] = i + 1;
    }
  }
  bstart[nblk] = n;

  /* per block: Gershgorin, pivmin, wanted local range */
  int64_t* bwl = (int64_t*)malloc((size_t)nblk * sizeof(int64_t));
  int64_t* bwu = (int64_t*)malloc((size_t)nblk * sizeof(int64_t));
  double *bgl = (double*)malloc((size_t)nblk * sizeof(double)), *bgu = (double*)malloc((size_t)nblk * sizeof(double));
  double* bpiv = (double*)malloc((size_t)nblk * sizeof(double));
  for (int64_t b = 0; b < nblk; b++) {
    int64_t o = bstart[b], nb = bstart[b + 1] - o;
    gershgorin(nb, ds + o, es + o, &bgl[b], &bgu[b]);
    double emax = 0.0;
    for (int64_t i = 0; i + 1 < nb; i++) emax = fmax(emax, es[o + i] * es[o + i]);
    bpiv[b] = SAFMIN * fmax(1.0, emax);
    bwl[b] = 1;
    bwu[b] = nb;
  }
  if (kind == RANGE_VALUE) {
    for (int64_t b = 0; b < nblk; b++) {
      int64_t o = bstart[b], nb = bstart[b + 1] - o;
      double* e2 = (double*)malloc((size_t)nb * sizeof(double));
      for (int64_t i = 0; i + 1 < nb; i++) e2[i] = es[o + i] * es[o + i];
      bwl[b] = count_T(nb, ds + o, e2, svl, bpiv[b]) + 1;
      bwu[b] = count_T(nb, ds + o, e2, svu, bpiv[b]);
      free(e2);
    }
  } else if (kind == RANGE_INDEX) {
    if (nblk == 1) {
      bwl[0] = il;
      bwu[0] = iu;
    } else {
      /* several blocks: all eigenvalues, global order by (value, block) */
      double* allw = (double*)malloc((size_t)n * sizeof(double));
      double* lo = (double*)malloc((size_t)n * sizeof(double));
      double* hi = (double*)malloc((size_t)n * sizeof(double));
      double* wk = (double*)malloc((size_t)6 * n * sizeof(double));
      item_t* it = (item_t*)malloc((size_t)n * sizeof(item_t));
      int64_t cnt = 0;
      for (int64_t b = 0; b < nblk; b++) {
        int64_t o = bstart[b], nb = bstart[b + 1] - o;
        block_t B = {nb, ds + o, es + o, bgl[b], bgu[b], bgu[b] - bgl[b], bpiv[b], lo + o, hi + o,
                     1, nb, allw + o, NULL, 0, st, ST_OK, wk};
        solve_block(&B, 1, (uint64_t)o);
        for (int64_t j = 1; j <= nb; j++) {
          it[cnt].w = allw[o + j - 1];
          it[cnt].blk = b;
          it[cnt].j = j;
          it[cnt].pos = 0;
          cnt++;
        }
      }
      qsort(it, (size_t)cnt, sizeof(item_t), cmp_item);
      for (int64_t b = 0; b < nblk; b++) { bwl[b] = 1; bwu[b] = 0; }
      int64_t* below = (int64_t*)calloc((size_t)nblk, sizeof(int64_t));
      int64_t* inside = (int64_t*)calloc((size_t)nblk, sizeof(int64_t));
      for (int64_t k = 0; k < cnt; k++) {
        if (k < il - 1) below[it[k].blk]++;
        else if (k < iu) inside[it[k].blk]++;
      }
      for (int64_t b = 0; b < nblk; b++) {
        bwl[b] = below[b] + 1;
        bwu[b] = below[b] + inside[b];
      }
      free(below); free(inside); free(allw); free(lo); free(hi); free(wk); free(it);
    }
  }
  int64_t m = 0;
  for (int64_t b = 0; b < nblk; b++) m += bwu[b] >= bwl[b] ? bwu[b] - bwl[b] + 1 : 0;

  /* solve blocks into per-block buffers, then merge by ascending value */
  double* lo = (double*)malloc((size_t)n * sizeof(double));
  double* hi = (double*)malloc((size_t)n * sizeof(double));
  double* wk = (double*)malloc((size_t)6 * n * sizeof(double));
  double* wb = (double*)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
  item_t* items = (item_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(item_t));
  int64_t zsize = 0;
  for (int64_t b = 0; b < nblk; b++) {
    int64_t nb = bstart[b + 1] - bstart[b];
    if (bwu[b] >= bwl[b]) zsize += nb * (bwu[b] - bwl[b] + 1);
  }
  double* zb = NULL;
  if (Z) zb = (double*)malloc((size_t)(zsize > 0 ? zsize : 1) * sizeof(double));
  int status = ST_OK;
  if (!lo || !hi || !wk || !wb || !items || (Z && !zb)) status = ST_NOMEM;
  int64_t wpos = 0, zpos = 0, k = 0;
  for (int64_t b = 0; b < nblk && status != ST_NOMEM; b++) {
    int64_t o = bstart[b], nb = bstart[b + 1] - o;
    if (bwu[b] < bwl[b]) continue;
    int64_t mb = bwu[b] - bwl[b] + 1;
    /* left end of the spectrum unless the wanted set sits in the upper half */
    int left = (kind == RANGE_ALL) || (bwl[b] + bwu[b] <= nb + 1);
    block_t B = {nb, ds + o, es + o, bgl[b], bgu[b], bgu[b] - bgl[b], bpiv[b], lo + o, hi + o, bwl[b], bwu[b],
                 wb + wpos, Z ? zb + zpos : NULL, nb, st, ST_OK, wk};
    int s = solve_block(&B, left, (uint64_t)o);
    if (s != ST_OK && status == ST_OK) status = s;
    for (int64_t j = 0; j < mb; j++) {
      items[k].w = wb[wpos + j];
      items[k].blk = b;
      items[k].j = bwl[b] + j;
      items[k].pos = zpos + j * nb;
      k++;
    }
    wpos += mb;
    zpos += nb * mb;
  }
  if (status != ST_NOMEM) {
    qsort(items, (size_t)m, sizeof(item_t), cmp_item);
    for (int64_t c = 0; c < m; c++) {
      w[c] = items[c].w / scale;
      if (Z) {
        int64_t b = items[c].blk, o = bstart[b], nb = bstart[b + 1] - o;
        double* col = Z + c * ldz;
        for (int64_t i = 0; i < n; i++) col[i] = 0.0;
        memcpy(col + o, zb + items[c].pos, (size_t)nb * sizeof(double));
      }
    }
    if (m_out) *m_out = m;
  }
  free(lo); free(hi); free(wk); free(wb); free(items); free(zb);
  free(bstart); free(bwl); free(bwu); free(bgl); free(bgu); free(bpiv); free(ds); free(es);
  return status;
}

/* j-th smallest eigenvalue (1-based) of T by plain bisection with Sturm counts
 * on T itself (no representation): the textbook definition used for sampled
 * checks at sizes where the full oracle is too slow.  Returns the bracket. */
int oracle_bisect_T(int64_t n, const double* d, const double* e, int64_t j, double* lo_out, double* hi_out) {
  if (n < 1 || j < 1 || j > n) return -1;
  double* e2 = (double*)calloc((size_t)n, sizeof(double));
  double emax = 0.0;
  for (int64_t i = 0; i + 1 < n; i++) {
    e2[i] = e[i] * e[i];
    emax = fmax(emax, e2[i]);
  }
  double pivmin = SAFMIN * fmax(1.0, emax);
  double gl, gu;
  gershgorin(n, d, e, &gl, &gu);
  double pad = 2.0 * (double)n * EPS * fmax(fabs(gl), fabs(gu)) + 2.0 * pivmin;
  double lo = gl - pad, hi = gu + pad;
  for (int it = 0; it < MAX_BISECT; it++) {
    double tol = 2.0 * EPS * fmax(fabs(lo), fabs(hi));
    if (hi - lo <= tol) break;
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count_T(n, d, e2, mid, pivmin) <= j - 1)
      lo = mid;
    else
      hi = mid;
  }
  free(e2);
  *lo_out = lo;
  *hi_out = hi;
  return 0;
}

/* Sturm count on T (number of eigenvalues below tau), for tests of the counts */
int64_t oracle_count_T(int64_t n, const double* d, const double* e, double tau) {
  double* e2 = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double emax = 0.0;
  for (int64_t i = 0; i + 1 < n; i++) {
    e2[i] = e[i] * e[i];
    emax = fmax(emax, e2[i]);
  }
  int64_t c = count_T(n, d, e2, tau, SAFMIN * fmax(1.0, emax));
  free(e2);
  return c;
}

/* the counter-based generator used for the root perturbation, exposed so the
 * tests can pin it to published SplitMix64 outputs */
uint64_t oracle_splitmix64(uint64_t seed, uint64_t counter) { return splitmix64_at(seed, counter); }
