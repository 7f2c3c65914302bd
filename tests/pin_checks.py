"""Pin checks shared by the oracle pin tests and the mutation tests.

Each check takes the function under test as an argument and raises
AssertionError when the function disagrees with what the paper or the
mathematics fixes.  tests/test_oracle_pins.py runs them on the oracle;
tests/test_oracle_mutations.py runs them on copies of the oracle with one
planted mistake each and requires that some check fails.

Nothing here re-types the oracle's formulas:
  * the V map is pinned by monotonicity in u and uniformity;
  * the GEAT key length (App. A bound, App. C terms) is pinned by the
    simplified bound Eq. (1) of Sec. II (a different expression, with xi,
    beta(eps) and gamma(eps) of App. A) and by the two leading terms of its
    large-N expansion, derived here in closed form.
"""

from __future__ import annotations

import math

import numpy as np


# ------------------------------------------------------------- V map ---

def check_v_map(draw_v, splitmix64, n_sub: int, key: int = 0x5A17,
                count: int = 20000) -> None:
    """V_i = map(u_i) with u_i the low (even i) or high (odd i) 32 bits of
    SplitMix64 output i // 2 (outputs pinned by published values).  Sec. III.B
    step 1 only asks for a uniform V_i in [0, N_S); the reading taken is a
    range map that is (a) monotone non-decreasing in u, (b) onto [0, N_S)
    with every value taking about 2^32 / N_S of the u's.  Checked on `count`
    rounds: sorted by u, V never decreases, stays in range, and the values
    are spread evenly (chi-square)."""
    us = np.empty(count, dtype=np.uint64)
    vs = np.empty(count, dtype=np.int64)
    for i in range(count):
        r = splitmix64(key, i // 2)
        us[i] = (r >> 32) if (i & 1) else (r & 0xFFFFFFFF)
        vs[i] = draw_v(key, i, n_sub)
    assert vs.min() >= 0 and vs.max() < n_sub, "V out of range"
    order = np.argsort(us, kind="stable")
    assert np.all(np.diff(vs[order]) >= 0), "V is not monotone in u"
    # Even spread: V / N_S tracks u / 2^32 within one bucket.
    frac_u = us.astype(np.float64) / 2.0 ** 32
    assert np.all(np.abs(vs / n_sub - frac_u) <= 1.0 / n_sub + 1e-12), \
        "V does not track u"
    if count >= 20 * n_sub:
        counts = np.bincount(vs, minlength=n_sub)
        e = count / n_sub
        chi2 = float(((counts - e) ** 2 / e).sum())
        dof = n_sub - 1
        assert chi2 < dof + 6.0 * math.sqrt(2.0 * dof) + 10.0, chi2


# ------------------------------------------------------- GEAT key length ---

def _h2(x: float) -> float:
    return -x * math.log2(x) - (1.0 - x) * math.log2(1.0 - x)


def _app_c_terms(p: dict, e_t: float) -> dict:
    """Max(f), Min(f), Var(f) bound and h of App. C for direct hashing
    (n_sub = 1), read off the appendix."""
    pz = 1.0 - p["p_x"]
    return dict(
        max=pz ** 2 * (1.0 + math.log2(1.0 - e_t)),
        min=pz ** 2 * (1.0 + math.log2(e_t)),
        var=pz ** 4 / p["p_x"] ** 2 * (1.0 + math.log2(1.0 - e_t)) ** 2,
        h=pz ** 2 * p["eta_tol"] * (1.0 - _h2(e_t) - (p["q_tol"] - e_t)
                                     * math.log2(1.0 / e_t - 1.0)))


def _g(eps: float) -> float:
    """g(eps) = -log2(1 - sqrt(1 - eps^2)) of App. A, by 60-digit decimals."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    e = Decimal(eps)
    return float(-(1 - (1 - e * e).sqrt()).ln() / Decimal(2).ln())


def _non_entropy_terms(p: dict) -> float:
    """The App. C key length minus the smooth min-entropy bound: the
    error-correction leakage l_EC = N pZ^2 p_det f_EC h(e_b) and the
    leftover-hash term 1 - log2(1 / (eps_sec - 2 eps_sm))."""
    pz = 1.0 - p["p_x"]
    leak = p["n_rounds"] * pz * pz * p["eta_tol"] * p["f_ec"] * _h2(p["e_bit"])
    return -leak + 1.0 - math.log2(1.0 / (p["eps_sec"] - 2.0 * p["eps_sm"]))


def entropy_bound_best(key_length, p: dict, e_t: float) -> float:
    """max over alpha in (1, 3/2) of the App. A smooth min-entropy bound, got
    from the key length under test by removing the non-entropy terms.  The
    maximum is found over log10(alpha - 1) with a bounded scalar search."""
    from scipy.optimize import minimize_scalar
    r = minimize_scalar(lambda u: -key_length(p, 1.0 + 10.0 ** u, e_t),
                        bounds=(-12.0, math.log10(0.5) - 1e-9),
                        method="bounded", options=dict(xatol=1e-10))
    return -float(r.fun) - _non_entropy_terms(p)


def eq1_bound(p: dict, e_t: float) -> tuple[float, float]:
    """Sec. II Eq. (1): N h - v1 sqrt(N) - v0 with xi, beta(eps) and
    gamma(eps) of App. A.  Returns (bound, v1)."""
    t = _app_c_terms(p, e_t)
    N, dx = p["n_rounds"], p["d_x"]
    g = _g(p["eps_sm"])
    lo = math.log2(1.0 / p["p_omega"])
    ln2 = math.log(2.0)
    xi = 2.0 * ln2 / (1.0 + 2.0 * ln2)
    beta = (((2.0 - xi) * xi ** 2 * lo + xi ** 2 * g)
            / (3.0 * ln2 ** 2 * (2.0 * xi - 1.0) ** 3))
    gamma = math.sqrt(2.0 * ln2 / xi * (g + (2.0 - xi) * lo))
    V = math.log2(2.0 * dx * dx + 1.0) + math.sqrt(2.0 + t["var"])
    nu = 2.0 * math.log2(dx) + t["max"] - t["min"]
    v0 = (beta / V ** 2 * 2.0 ** ((1.0 - xi) / xi * nu)
          * math.log(2.0 ** nu + math.e ** 2) ** 3)
    v1 = gamma * V
    return N * t["h"] - v1 * math.sqrt(N) - v0, v1


def expansion_terms(p: dict, e_t: float) -> tuple[float, float]:
    """Leading terms of N h - max_alpha(App. A bound) = c1 sqrt(N) + c0 + o(1).

    With t = (alpha - 1) / (2 - alpha) the App. A bound reads
        N h - N t ln2 V^2 / 2 - (g + L) / t - (g + 2 L) - N t^2 K(t),
        K(t) = 2^(t nu) ln^3(2^nu + e^2) / (6 (1 - t)^3 ln 2),
    L = log2(1 / p_Omega) (alpha = (1 + 2t) / (1 + t), 3 - 2 alpha =
    (1 - t) / (1 + t)).  The first two terms are smallest at
    t* = sqrt(2 (g + L) / (N ln2 V^2)); since the bound is stationary there,
    moving t* by the K term changes it by O(1 / sqrt(N)), so
        c1 = V sqrt(2 ln2 (g + L)),
        c0 = g + 2 L + N t*^2 K(0) = g + 2 L + 2 (g + L) K(0) / (ln2 V^2)."""
    t = _app_c_terms(p, e_t)
    dx = p["d_x"]
    g = _g(p["eps_sm"])
    lo = math.log2(1.0 / p["p_omega"])
    ln2 = math.log(2.0)
    V = math.log2(2.0 * dx * dx + 1.0) + math.sqrt(2.0 + t["var"])
    nu = 2.0 * math.log2(dx) + t["max"] - t["min"]
    k0 = math.log(2.0 ** nu + math.e ** 2) ** 3 / (6.0 * ln2)
    c1 = V * math.sqrt(2.0 * ln2 * (g + lo))
    c0 = g + 2.0 * lo + 2.0 * (g + lo) * k0 / (ln2 * V * V)
    return c1, c0


GEAT_PIN_BASE = dict(p_x=0.02, q_tol=0.0082, eta_tol=1.0, e_bit=0.058,
                     f_ec=1.16, eps_sec=1e-6, eps_sm=1e-7, eps_abort=0.0,
                     n_sub=1)

GEAT_PIN_GRID = [(n, po, dx, et) for n in (1e6, 1e9, 1e12)
                 for po in (1.0, 1e-3) for dx in (2.0, 3.0)
                 for et in (0.004, 0.01)]


def check_geat_eq1(key_length) -> None:
    """The App. A bound, maximised over alpha, is at least the simplified
    bound Eq. (1) (Sec. II), which comes from one particular alpha; and its
    sqrt(N) coefficient never exceeds Eq. (1)'s v1 = gamma(eps) V."""
    for n, po, dx, et in GEAT_PIN_GRID:
        p = dict(GEAT_PIN_BASE, n_rounds=n, p_omega=po, d_x=dx)
        best = entropy_bound_best(key_length, p, et)
        bound, v1 = eq1_bound(p, et)
        assert best >= bound, (n, po, dx, et, best, bound)
        h = _app_c_terms(p, et)["h"]
        assert (n * h - best) / math.sqrt(n) <= v1, (n, po, dx, et)


def check_geat_expansion(key_length, rel: float = 1e-4) -> None:
    """N h - max_alpha(bound) = c1 sqrt(N) + c0 + o(1): at N = 1e10 and 1e12
    both leading terms match the closed forms of expansion_terms."""
    for n in (1e10, 1e12):
        for po in (1.0, 1e-3):
            for dx in (2.0, 3.0):
                p = dict(GEAT_PIN_BASE, n_rounds=n, p_omega=po, d_x=dx)
                et = 0.01
                best = entropy_bound_best(key_length, p, et)
                h = _app_c_terms(p, et)["h"]
                c1, c0 = expansion_terms(p, et)
                gap = n * h - best
                assert abs(gap / math.sqrt(n) / c1 - 1.0) < rel, \
                    ("sqrt(N) term", n, po, dx, gap / math.sqrt(n), c1)
                r = (gap - c1 * math.sqrt(n)) / c0
                assert abs(r - 1.0) < 1e-3, ("constant term", n, po, dx, r)
