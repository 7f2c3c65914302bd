// Key length of a GEAT-analysed protocol, direct and with sampled sub-block
// hashing (host only).
//
// Generalised entropy accumulation (App. A statement) with the BBM92
// min-tradeoff function of App. C, tangent to the entropy bound at e_t:
//   h      = pZ^2 eta (1 - h2(e_t) - (Q - e_t) log2(1/e_t - 1))
//   Max(f) = pZ^2 (1 + log2(1 - e_t)),  Min(f) = pZ^2 (1 + log2 e_t)
//   Var(f) = pZ^4 / pX^2 (1 + log2(1 - e_t))^2
//   V      = log2(2 dX^2 + 1) + sqrt(2 + Var(f))
//   K'(a)  = (2-a)^3 / (6 (3-2a)^3 ln 2) 2^((a-1)/(2-a) D) ln^3(2^D + e^2),
//            D = 2 log2 dX + Max(f) - Min(f)
//   g(eps) = -log2(1 - sqrt(1 - eps^2))
//   l      = N h - N (a-1) ln 2 / (2 (2-a)) V^2 - N ((a-1)/(2-a))^2 K'(a)
//            - (g(eps_sm) + a log2(1/p_Omega)) / (a - 1)
//            - N pZ^2 eta f_EC h2(e_bit) + 1 - log2(1 / (eps_sec - 2 eps_sm)).
// Sub-block hashing (Claim 1): each of the N_S sub-protocols has f / N_S
// (so h, Max, Min scale by 1/N_S and Var by 1/N_S^2) and key length
// l / N_S, and eps = N_S eps' + eps_Omega'; error correction and smoothing
// are split the same way (leakage / N_S, eps_sm / N_S).  The key length is
// N_S times the sub-protocol's.  g is evaluated as
// -log2(eps^2 / (1 + sqrt(1 - eps^2))), equal and free of cancellation.
#include <math.h>

#include "ssbh_internal.hpp"

namespace {

double h2(double x) {
    if (x <= 0.0 || x >= 1.0) return 0.0;
    return -x * log2(x) - (1.0 - x) * log2(1.0 - x);
}

const char *check(const ssbh_geat_params &p) {
    if (!(p.n_rounds >= 1.0)) return "n_rounds must be >= 1";
    if (!(p.p_x > 0.0 && p.p_x < 1.0)) return "p_x must be in (0, 1)";
    if (!(p.q_tol > 0.0 && p.q_tol < 0.5)) return "q_tol must be in (0, 0.5)";
    if (!(p.eta_tol > 0.0 && p.eta_tol <= 1.0)) return "eta_tol must be in (0, 1]";
    if (!(p.e_bit >= 0.0 && p.e_bit < 0.5)) return "e_bit must be in [0, 0.5)";
    if (!(p.f_ec >= 1.0)) return "f_ec must be >= 1";
    if (!(p.eps_abort >= 0.0)) return "eps_abort must be >= 0";
    if (!(p.eps_sm > 0.0 && 2.0 * p.eps_sm < p.eps_sec - p.eps_abort))
        return "need 0 < 2 eps_sm < eps_sec - eps_abort";
    if (!(p.p_omega > 0.0 && p.p_omega <= 1.0)) return "p_omega must be in (0, 1]";
    if (!(p.d_x >= 2.0)) return "d_x must be >= 2";
    if (p.n_sub < 1) return "n_sub must be >= 1";
    return nullptr;
}

double key_length(const ssbh_geat_params &p, double a, double et) {
    const double ns = (double)p.n_sub, N = p.n_rounds;
    const double pz2 = (1.0 - p.p_x) * (1.0 - p.p_x);
    const double top = 1.0 + log2(1.0 - et);
    const double fmax = pz2 * top / ns;
    const double fmin = pz2 * (1.0 + log2(et)) / ns;
    const double fvar = pz2 * pz2 / (p.p_x * p.p_x) * top * top / (ns * ns);
    const double h = pz2 * p.eta_tol *
                     (1.0 - h2(et) - (p.q_tol - et) * log2(1.0 / et - 1.0)) / ns;
    const double V = log2(2.0 * p.d_x * p.d_x + 1.0) + sqrt(2.0 + fvar);
    const double D = 2.0 * log2(p.d_x) + fmax - fmin;
    const double r = (a - 1.0) / (2.0 - a);
    const double kp = pow(2.0 - a, 3) / (6.0 * pow(3.0 - 2.0 * a, 3) * log(2.0)) *
                      exp2(r * D) * pow(log(exp2(D) + exp(2.0)), 3);
    const double eps_sub = (p.eps_sec - p.eps_abort) / ns;
    const double eps_sm = p.eps_sm / ns;
    const double g = -log2(eps_sm * eps_sm / (1.0 + sqrt(1.0 - eps_sm * eps_sm)));
    const double leak = N * pz2 * p.eta_tol * p.f_ec * h2(p.e_bit) / ns;
    const double l = N * h - N * (a - 1.0) * log(2.0) / (2.0 * (2.0 - a)) * V * V -
                     N * r * r * kp -
                     (g + a * log2(1.0 / p.p_omega)) / (a - 1.0) - leak + 1.0 -
                     log2(1.0 / (eps_sub - 2.0 * eps_sm));
    return ns * l;
}

// Golden-section maximum of f on [lo, hi].
template <class F>
double golden_max(F f, double lo, double hi, int iters, double *arg) {
    const double g = 0.5 * (sqrt(5.0) - 1.0);
    double a = lo, b = hi;
    double c = b - g * (b - a), d = a + g * (b - a);
    double fc = f(c), fd = f(d);
    for (int i = 0; i < iters; ++i) {
        if (fc > fd) { b = d; d = c; fd = fc; c = b - g * (b - a); fc = f(c); }
        else { a = c; c = d; fc = fd; d = a + g * (b - a); fd = f(d); }
    }
    *arg = fc > fd ? c : d;
    return fc > fd ? fc : fd;
}

}  // namespace

using namespace ssbh;

extern "C" ssbh_status ssbh_geat_key_length(const ssbh_geat_params *p,
                                            double alpha, double e_tangent,
                                            double *key_bits) {
    clear_error();
    if (!p || !key_bits) SSBH_INVAL("p and key_bits must be non-null");
    if (const char *m = check(*p)) SSBH_INVAL("%s", m);
    if (!(alpha > 1.0 && alpha < 1.5)) SSBH_INVAL("alpha must be in (1, 1.5)");
    if (!(e_tangent > 0.0 && e_tangent < 0.5))
        SSBH_INVAL("e_tangent must be in (0, 0.5)");
    *key_bits = key_length(*p, alpha, e_tangent);
    return SSBH_OK;
}

// Maximum over alpha in (1, 1.5) and e_t in (0, 0.5): a grid in
// u = log10(alpha - 1) and v = log10(e_t), then alternating golden-section
// searches around the best grid point.
extern "C" ssbh_status ssbh_geat_optimise(const ssbh_geat_params *p,
                                          double *key_bits, double *alpha,
                                          double *e_tangent) {
    clear_error();
    if (!p || !key_bits) SSBH_INVAL("p and key_bits must be non-null");
    if (const char *m = check(*p)) SSBH_INVAL("%s", m);
    const double ulo = -9.0, uhi = log10(0.5) - 1e-9;
    const double vlo = log10(p->q_tol) - 3.0, vhi = log10(0.5) - 1e-9;
    auto F = [&](double u, double v) {
        return key_length(*p, 1.0 + pow(10.0, u), pow(10.0, v));
    };
    double bu = ulo, bv = vlo, best = -INFINITY;
    const int G = 96;
    for (int i = 0; i <= G; ++i)
        for (int j = 0; j <= G; ++j) {
            const double u = ulo + (uhi - ulo) * i / G, v = vlo + (vhi - vlo) * j / G;
            const double f = F(u, v);
            if (f > best) { best = f; bu = u; bv = v; }
        }
    double du = (uhi - ulo) / G, dv = (vhi - vlo) / G;
    for (int round = 0; round < 8; ++round) {
        double nu = bu, nv = bv;
        golden_max([&](double u) { return F(u, bv); }, fmax(ulo, bu - du),
                   fmin(uhi, bu + du), 60, &nu);
        golden_max([&](double v) { return F(nu, v); }, fmax(vlo, bv - dv),
                   fmin(vhi, bv + dv), 60, &nv);
        const double f = F(nu, nv);
        if (f >= best) { best = f; bu = nu; bv = nv; }
        du *= 0.5;
        dv *= 0.5;
    }
    *key_bits = best;
    if (alpha) *alpha = 1.0 + pow(10.0, bu);
    if (e_tangent) *e_tangent = pow(10.0, bv);
    return SSBH_OK;
}
