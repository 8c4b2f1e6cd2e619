// P_K by Chebyshev acceleration of the Jacobi iteration on K_m.
//
// Sec. 5.3 leaves the inner preconditioners P_1 ~ S_1 and P_K ~ K_m free
// (any classical preconditioner of an elliptic or parabolic matrix fits the
// block-LU framework of Def. 2, and its parallel remark asks only for
// parallel inner solves).  K_m = gamma M_H + S_m is the matrix of a
// parabolic step: with the diagonal D of K_m, the spectrum of D^-1 K_m sits
// in a narrow interval [a, b] away from 0, so a fixed polynomial in D^-1 K_m
// is a good approximate inverse that needs only sparse products.
//
// With z_0 = 0 and theta = (a + b) / 2, delta = (b - a) / 2 the method
// (Chebyshev acceleration, e.g. Saad, Iterative Methods for Sparse Linear
// Systems, Sec. 12.1) runs
//     d_0 = D^-1 t / theta,  z_1 = d_0,  r_0 = t,
//     r_k = r_{k-1} - K_m d_{k-1},
//     d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) D^-1 r_k,
//     z_{k+1} = z_k + d_k,
// with rho_0 = delta / theta and rho_k = 1 / (2 theta / delta - rho_{k-1}).
// After m steps the error in each eigencomponent lambda of D^-1 K_m is the
// initial one times T_m((theta - lambda) / delta) / T_m(theta / delta).  The
// map t -> z_m is symmetric and positive definite whenever every eigenvalue
// is below a + b, so plain PCG keeps working.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "host.h"

namespace bido {

namespace {

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal al and off-diagonal be (Sturm sequence of the LDL^T pivots).
int sturm_below(const std::vector<double>& al, const std::vector<double>& be, double x) {
    int count = 0;
    double q = 1.0;
    for (size_t i = 0; i < al.size(); ++i) {
        const double b2 = i > 0 ? be[i - 1] * be[i - 1] : 0.0;
        q = al[i] - x - (i > 0 ? b2 / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++count;
    }
    return count;
}

// k-th smallest eigenvalue (0-based) of the tridiagonal matrix, by bisection.
double tridiag_eig(const std::vector<double>& al, const std::vector<double>& be, int k) {
    double lo = al[0], hi = al[0];
    for (size_t i = 0; i < al.size(); ++i) {
        const double r = (i > 0 ? std::fabs(be[i - 1]) : 0.0) + (i + 1 < al.size() ? std::fabs(be[i]) : 0.0);
        lo = std::min(lo, al[i] - r);
        hi = std::max(hi, al[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_below(al, be, mid) > k) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

bool chebyshev_interval(const Csr& K, const std::vector<double>& gm, int lanczos_steps, ChebInterval& out,
                        std::string& err) {
    const int64_t n = K.n;
    if (n <= 0 || (int64_t)gm.size() != n) { err = "chebyshev_interval: bad sizes"; return false; }
    std::vector<double> d(n), s(n);
    for (int64_t i = 0; i < n; ++i) {
        d[i] = 0.0;
        for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p)
            if (K.col[p] == i) d[i] += K.val[p];
        if (!(d[i] > 0.0)) { err = "chebyshev_interval: K_m has a non-positive diagonal entry"; return false; }
        s[i] = 1.0 / std::sqrt(d[i]);
    }
    // Rigorous bounds on the spectrum of B = D^-1/2 K D^-1/2 (that of D^-1 K):
    // K >= gamma M_H since S_m is positive semi-definite, so
    // lambda_min(B) >= min_i gamma m_i / K_ii; Gershgorin bounds lambda_max.
    double blo = HUGE_VAL, bhi = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        blo = std::min(blo, gm[i] / d[i]);
        double row = 0.0;
        for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p) row += std::fabs(K.val[p]) * s[i] * s[K.col[p]];
        bhi = std::max(bhi, row);
    }
    // Lanczos on B from a fixed pseudo-random start: its extreme Ritz values
    // lie inside the spectrum and approach its ends.
    const int steps = (int)std::min<int64_t>(std::max(1, lanczos_steps), n);
    std::vector<double> v(n), vp(n, 0.0), w(n), al, be;
    uint64_t seed = 0x5eedull;
    double nv = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        v[i] = (double)(splitmix64(seed) >> 11) * 0x1.0p-53 - 0.5;
        nv += v[i] * v[i];
    }
    nv = std::sqrt(nv);
    for (auto& x : v) x /= nv;
    double beta = 0.0;
    for (int j = 0; j < steps; ++j) {
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int64_t p = K.ptr[i]; p < K.ptr[i + 1]; ++p) acc += K.val[p] * s[K.col[p]] * v[K.col[p]];
            w[i] = s[i] * acc - beta * vp[i];
        }
        double a = 0.0;
        for (int64_t i = 0; i < n; ++i) a += w[i] * v[i];
        for (int64_t i = 0; i < n; ++i) w[i] -= a * v[i];
        al.push_back(a);
        double b = 0.0;
        for (int64_t i = 0; i < n; ++i) b += w[i] * w[i];
        b = std::sqrt(b);
        if (j + 1 == steps || b <= 1e-14 * std::fabs(a)) break;   // invariant subspace reached
        be.push_back(b);
        beta = b;
        for (int64_t i = 0; i < n; ++i) { vp[i] = v[i]; v[i] = w[i] / b; }
    }
    out.ritz_lo = tridiag_eig(al, be, 0);
    out.ritz_hi = tridiag_eig(al, be, (int)al.size() - 1);
    out.bound_lo = blo;
    out.bound_hi = bhi;
    // the lower Ritz value only loses accuracy, never definiteness; the top
    // end gets a margin (definiteness needs lambda_max < a + b)
    out.lo = std::max(blo, out.ritz_lo);
    out.hi = std::min(bhi, 1.05 * out.ritz_hi);
    if (out.hi <= out.lo) out.hi = out.lo * (1.0 + 1e-6);
    return true;
}

ChebCoef chebyshev_coefficients(double lo, double hi, int steps) {
    ChebCoef c;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    const double sigma = theta / delta;
    c.inv_theta = 1.0 / theta;
    double rho = 1.0 / sigma;
    for (int k = 1; k < steps; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        c.c1.push_back(rn * rho);
        c.c2.push_back(2.0 * rn / delta);
        rho = rn;
    }
    return c;
}

}  // namespace bido
