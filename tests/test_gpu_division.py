"""The reciprocal and quotient forms of the kernels (mrrr_probe_division, the
library's own probe kernel) against IEEE correctly rounded division (numpy's
1/b and a/b on the host), on about 2.9 million seeded operands spread over the
binades the solver meets: the unit binade (mantissa coverage), exponents from
-1000 to 1000, the pivmin range just above the smallest normal (where the
Sturm counts and twisted transforms put guarded pivots), reciprocals near the
overflow threshold (|b| in [2^-1022, 2^-1000]) and subnormal reciprocals
(|b| in [2^1000, 2^1023]).

What each form must give, and where the kernels use it:
* v_rcp_f64 alone: an approximation (relative error below 2^-23);
* one Newton-Raphson step (Sturm counts, twisted transforms, Rayleigh
  correction): a few ulps (the counts' error analysis needs O(eps) relative
  error per operation; bound checked: 16 ulps);
* two steps (multipliers of child representations): correctly rounded on
  every operand here;
* the quotient (two-step reciprocal, product, one residual correction;
  eigenvector recurrence across a zero pivot): correctly rounded on every
  operand here.
Subnormal divisors have no finite reciprocal form: the two-step reciprocal is
NaN there, which the kernels never meet (pivots are replaced by -pivmin, at
least the smallest normal, before a reciprocal, or their results are tested
for finiteness).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def M():
    import paper_1205_2107_amd as pkg
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    return pkg


def operands():
    rng = np.random.default_rng(12345)

    def binades(lo, hi, k):
        ex = np.floor(rng.uniform(lo, hi, k)).astype(int)
        return np.ldexp(1.0 + rng.random(k), ex) * rng.choice([-1.0, 1.0], k)

    tiny = np.finfo(np.float64).tiny
    return {
        "unit": (1.0 + rng.random(1 << 20)) * rng.choice([-1.0, 1.0], 1 << 20),
        "wide": binades(-1000, 1000, 1 << 20),
        "pivmin": tiny * np.exp(rng.uniform(0.0, np.log(1e6), 1 << 18)) * rng.choice([-1.0, 1.0], 1 << 18),
        "near_overflow": binades(-1022, -1000, 1 << 18),
        "subnormal_result": binades(1000, 1023, 1 << 18),
    }, rng


def ulps(x, ref):
    """|x - ref| in units of the spacing of doubles at ref (finite ref only)."""
    return np.abs(x - ref) / np.spacing(np.abs(ref))


@pytest.mark.parametrize("name", ["unit", "wide", "pivmin", "near_overflow", "subnormal_result"])
def test_division_forms_against_correct_rounding(M, name):
    ops, rng = operands()
    b = ops[name]
    a = np.ldexp(1.0 + rng.random(b.size), rng.integers(-400, 400, b.size)) * rng.choice([-1.0, 1.0], b.size)
    r0, r1, r2, q = [t.cpu().numpy() for t in M.probe_division(torch.tensor(a, device="cuda"),
                                                                 torch.tensor(b, device="cuda"))]
    with np.errstate(over="ignore", under="ignore"):
        ref = 1.0 / b
        qref = a / b
    fin = np.isfinite(ref)
    assert fin.all()
    rel0 = np.abs(r0 - ref) / np.abs(ref)
    e1 = ulps(r1, ref)
    e2 = ulps(r2, ref)
    qf = np.isfinite(qref) & (qref != 0)
    eq = ulps(q[qf], qref[qf])
    print(f"{name}: n={b.size} rcp rel {rel0.max():.3g}, one step {e1.max():.0f} ulp "
          f"({(e1 > 0).mean():.1%} not correctly rounded), two steps {e2.max():.0f} ulp, "
          f"quotient {eq.max() if eq.size else 0:.0f} ulp")
    assert rel0.max() < 2.0 ** -23
    assert e1.max() <= 16
    assert e2.max() == 0, "two-step reciprocal not correctly rounded"
    assert eq.size > 0 and eq.max() == 0, "quotient not correctly rounded"


def test_subnormal_divisor_gives_no_finite_reciprocal(M):
    rng = np.random.default_rng(7)
    b = np.ldexp(1.0 + rng.random(4096), -1030) * rng.choice([-1.0, 1.0], 4096)
    a = np.ones_like(b)
    r0, r1, r2, q = [t.cpu().numpy() for t in M.probe_division(torch.tensor(a, device="cuda"),
                                                                 torch.tensor(b, device="cuda"))]
    assert not np.isfinite(r2).any()

