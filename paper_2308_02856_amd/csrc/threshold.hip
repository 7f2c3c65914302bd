// Abort threshold L_S^UB from the binomial tail bound of Sec. III.D (host).
//
// A sifted sub-block has length Binomial(n, p) with p = p_sift.  For
// L >= n p the bound is P(length > L) <= Q(sqrt(2 n H(L/n, p))), where Q is
// the upper normal tail and H the relative entropy of Bernoulli(L/n) to
// Bernoulli(p); over n_sub sub-blocks the abort chance is at most
// n_sub * Q(...).  The bound falls as L grows, so the smallest L meeting a
// target eps is found by bisection.
#include <math.h>

#include "ssbh_internal.hpp"

namespace {

// H(x, p) with d = x - p and log1p: near x = p both logarithms are of size d
// and cancel to a d^2-sized result, which logs of the plain ratios lose.
double rel_entropy(double x, double p) {
    const double d = x - p;
    double h = 0.0;
    if (x > 0.0) h += x * log1p(d / p);
    if (x < 1.0) h += (1.0 - x) * log1p(-d / (1.0 - p));
    return h;
}

double union_tail(uint64_t n, double p, uint32_t n_sub, uint64_t L) {
    if (L >= n) return 0.0;
    const double x = (double)L / (double)n;
    if (x < p) return (double)n_sub;
    const double z = sqrt(2.0 * (double)n * rel_entropy(x, p));
    return (double)n_sub * 0.5 * erfc(z / sqrt(2.0));
}

}  // namespace

using namespace ssbh;

extern "C" ssbh_status ssbh_ub_threshold(uint64_t n_rounds, double p_sift,
                                         uint32_t n_sub, double eps,
                                         uint64_t *l_ub, double *eps_at) {
    clear_error();
    if (!l_ub) SSBH_INVAL("l_ub is null");
    if (!(p_sift > 0.0 && p_sift < 1.0)) SSBH_INVAL("p_sift must be in (0, 1)");
    if (!(eps > 0.0)) SSBH_INVAL("eps must be > 0");
    if (!n_sub || !n_rounds) SSBH_INVAL("n_sub and n_rounds must be >= 1");
    // Invariant: union_tail(hi) <= eps; every L < lo is known to fail.
    uint64_t lo = (uint64_t)ceil((double)n_rounds * p_sift);
    if (lo > n_rounds) lo = n_rounds;
    uint64_t hi = n_rounds;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (union_tail(n_rounds, p_sift, n_sub, mid) <= eps) hi = mid;
        else lo = mid + 1;
    }
    *l_ub = hi;
    if (eps_at) *eps_at = union_tail(n_rounds, p_sift, n_sub, hi);
    return SSBH_OK;
}
