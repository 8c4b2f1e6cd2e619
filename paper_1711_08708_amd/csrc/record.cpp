// Probe points of a recording: the potential u at given points (the
// body-surface electrodes of the ECG recordings in Sec. 6) is the P1
// interpolant of the vertex values, so each point needs the element that
// holds it and its barycentric coordinates there.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

#include "host.h"

namespace bido {

namespace {

// Barycentric coordinates of p in the simplex with vertices v[0..dim];
// false for a degenerate simplex.
bool barycentric(int dim, const double* const* v, const double* p, double* lam) {
    if (dim == 2) {
        const double a = v[1][0] - v[0][0], b = v[2][0] - v[0][0];
        const double c = v[1][1] - v[0][1], d = v[2][1] - v[0][1];
        const double det = a * d - b * c;
        if (det == 0.0) return false;
        const double x = p[0] - v[0][0], y = p[1] - v[0][1];
        lam[1] = (d * x - b * y) / det;
        lam[2] = (a * y - c * x) / det;
        lam[0] = 1.0 - lam[1] - lam[2];
        return true;
    }
    double J[3][3], r[3];
    for (int i = 0; i < 3; ++i) {
        for (int k = 0; k < 3; ++k) J[i][k] = v[k + 1][i] - v[0][i];
        r[i] = p[i] - v[0][i];
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (det == 0.0) return false;
    for (int k = 0; k < 3; ++k) {            // Cramer's rule, column k replaced by r
        double M[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = j == k ? r[i] : J[i][j];
        lam[k + 1] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                      M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                      M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
    }
    lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
    return true;
}

}  // namespace

bool locate_points(int dim, const std::vector<double>& xyz, const std::vector<int32_t>& elems, const double* pts,
                   int np, std::vector<int64_t>& ids, std::vector<double>& wts, std::string& err) {
    const int nv = dim + 1;
    const int64_t ne = (int64_t)elems.size() / nv;
    ids.assign((size_t)np * nv, 0);
    wts.assign((size_t)np * nv, 0.0);
    for (int q = 0; q < np; ++q) {
        const double* p = pts + (size_t)q * dim;
        // the element in which the point is deepest (largest smallest
        // coordinate), so that a point on a shared face or vertex gets one
        // well-defined element
        int64_t best = -1;
        double best_min = -1e-9;
        double lam[4], keep[4] = {0, 0, 0, 0};
        for (int64_t e = 0; e < ne; ++e) {
            const double* v[4];
            for (int k = 0; k < nv; ++k) v[k] = &xyz[(size_t)elems[(size_t)e * nv + k] * dim];
            if (!barycentric(dim, v, p, lam)) continue;
            double mn = lam[0];
            for (int k = 1; k < nv; ++k) mn = std::min(mn, lam[k]);
            if (mn > best_min) {
                best_min = mn;
                best = e;
                for (int k = 0; k < nv; ++k) keep[k] = lam[k];
            }
        }
        if (best < 0) {
            err = "probe point " + std::to_string(q) + " lies outside the mesh";
            return false;
        }
        for (int k = 0; k < nv; ++k) {
            ids[(size_t)q * nv + k] = elems[(size_t)best * nv + k];
            wts[(size_t)q * nv + k] = keep[k];
        }
    }
    return true;
}

}  // namespace bido
