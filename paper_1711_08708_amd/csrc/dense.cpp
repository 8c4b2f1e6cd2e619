// Dense FP64 kernels for the host-side multifrontal factorisation.
// Blocked right-looking algorithms; the O(n^3) work goes through one
// register-blocked C -= A B^T kernel (rows of A and B contiguous).
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <vector>

#if defined(__AVX2__) && defined(__FMA__)
#include <immintrin.h>
#define BIDO_HAVE_AVX2 1
#endif

namespace bido {
namespace dense {
namespace {

constexpr int64_t NB = 96;   // algorithmic block size
constexpr int64_t KC = 256;  // k-chunk kept in cache by the micro-kernel

// C[4x4] += alpha * A[4 x k] B[4 x k]^T for rows given by pointers
inline void micro_4x4(int64_t k, const double* const a[4], const double* const b[4],
                      double* c[4], double alpha, bool lower_mask, int64_t i0, int64_t j0) {
    double acc[4][4];
#ifdef BIDO_HAVE_AVX2
    __m256d s[4][4];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) s[i][j] = _mm256_setzero_pd();
    int64_t p = 0;
    for (; p + 4 <= k; p += 4) {
        __m256d av[4], bv[4];
        for (int i = 0; i < 4; ++i) av[i] = _mm256_loadu_pd(a[i] + p);
        for (int j = 0; j < 4; ++j) bv[j] = _mm256_loadu_pd(b[j] + p);
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) s[i][j] = _mm256_fmadd_pd(av[i], bv[j], s[i][j]);
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            alignas(32) double t[4];
            _mm256_store_pd(t, s[i][j]);
            double r = (t[0] + t[1]) + (t[2] + t[3]);
            for (int64_t q = p; q < k; ++q) r += a[i][q] * b[j][q];
            acc[i][j] = r;
        }
#else
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double r = 0.0;
            for (int64_t q = 0; q < k; ++q) r += a[i][q] * b[j][q];
            acc[i][j] = r;
        }
#endif
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            if (!c[i]) continue;
            if (lower_mask && j0 + j > i0 + i) continue;
            c[i][j] += alpha * acc[i][j];
        }
}

void gemm_nt(int64_t m, int64_t n, int64_t k, double alpha, const double* A, int64_t lda,
             const double* B, int64_t ldb, double* C, int64_t ldc, bool lower_only,
             bool par) {
    if (m <= 0 || n <= 0 || k <= 0) return;
    const int64_t mb = (m + 3) / 4;
    static const double zero_row[KC] = {0};
    (void)zero_row;
    std::vector<double> pad;  // rows beyond m / n use a zero row
    pad.assign(KC, 0.0);
    const double* zr = pad.data();
#pragma omp parallel for schedule(dynamic, 1) if (par)
    for (int64_t ib = 0; ib < mb; ++ib) {
        const int64_t i0 = ib * 4;
        for (int64_t kc = 0; kc < k; kc += KC) {
            const int64_t kk = std::min(KC, k - kc);
            const double* a[4];
            double* c[4];
            for (int i = 0; i < 4; ++i) {
                bool ok = i0 + i < m;
                a[i] = ok ? A + (i0 + i) * lda + kc : zr;
                c[i] = ok ? C + (i0 + i) * ldc : nullptr;
            }
            const int64_t jend = lower_only ? std::min(n, i0 + 4) : n;
            for (int64_t j0 = 0; j0 < jend; j0 += 4) {
                const double* b[4];
                double* cc[4];
                bool okj[4];
                for (int j = 0; j < 4; ++j) {
                    okj[j] = j0 + j < n;
                    b[j] = okj[j] ? B + (j0 + j) * ldb + kc : zr;
                }
                for (int i = 0; i < 4; ++i) cc[i] = c[i] ? c[i] + j0 : nullptr;
                if (okj[3]) {
                    micro_4x4(kk, a, b, cc, alpha, lower_only, i0, j0);
                } else {
                    // ragged right edge: scalar
                    for (int i = 0; i < 4; ++i) {
                        if (!c[i]) continue;
                        for (int j = 0; j < 4 && j0 + j < n; ++j) {
                            if (lower_only && j0 + j > i0 + i) continue;
                            double r = 0.0;
                            for (int64_t q = 0; q < kk; ++q) r += a[i][q] * b[j][q];
                            c[i][j0 + j] += alpha * r;
                        }
                    }
                }
            }
        }
    }
}

// X (m x nb block columns) <- X L^-T for a small lower-triangular block L
void trsm_small(int64_t m, int64_t nb, const double* L, int64_t ldl, double* X,
                int64_t ldx, bool par) {
#pragma omp parallel for schedule(static) if (par && m > 256)
    for (int64_t r = 0; r < m; ++r) {
        double* x = X + r * ldx;
        for (int64_t j = 0; j < nb; ++j) {
            const double* l = L + j * ldl;
            double s = x[j];
            for (int64_t q = 0; q < j; ++q) s -= l[q] * x[q];
            x[j] = s / l[j];
        }
    }
}

}  // namespace

void gemm_nt_sub(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                 const double* B, int64_t ldb, double* C, int64_t ldc, bool lower_only,
                 bool par) {
    gemm_nt(m, n, k, -1.0, A, lda, B, ldb, C, ldc, lower_only, par);
}

void trsm_right_lower_t(int64_t m, int64_t n, const double* L, int64_t ldl, double* X,
                        int64_t ldx, bool par) {
    for (int64_t jb = 0; jb < n; jb += NB) {
        const int64_t nb = std::min(NB, n - jb);
        trsm_small(m, nb, L + jb * ldl + jb, ldl, X + jb, ldx, par);
        const int64_t rest = n - jb - nb;
        if (rest > 0)
            gemm_nt(m, rest, nb, -1.0, X + jb, ldx, L + (jb + nb) * ldl + jb, ldl,
                    X + jb + nb, ldx, false, par);
    }
}

int64_t potrf_lower(int64_t n, double* A, int64_t lda, bool par) {
    for (int64_t kb = 0; kb < n; kb += NB) {
        const int64_t nb = std::min(NB, n - kb);
        double* D = A + kb * lda + kb;
        // unblocked Cholesky of the diagonal block
        for (int64_t j = 0; j < nb; ++j) {
            double d = D[j * lda + j];
            for (int64_t q = 0; q < j; ++q) d -= D[j * lda + q] * D[j * lda + q];
            if (!(d > 0.0) || !std::isfinite(d)) return kb + j;
            d = std::sqrt(d);
            D[j * lda + j] = d;
            for (int64_t i = j + 1; i < nb; ++i) {
                double s = D[i * lda + j];
                for (int64_t q = 0; q < j; ++q) s -= D[i * lda + q] * D[j * lda + q];
                D[i * lda + j] = s / d;
            }
        }
        const int64_t rest = n - kb - nb;
        if (rest <= 0) break;
        double* P = A + (kb + nb) * lda + kb;
        trsm_small(rest, nb, D, lda, P, lda, par);
        gemm_nt(rest, rest, nb, -1.0, P, lda, P, lda, A + (kb + nb) * lda + kb + nb, lda,
                true, par);
    }
    return -1;
}

void trtri_lower(int64_t n, const double* L, int64_t lda, double* Linv, bool par) {
    // Y = I L^-T (upper triangular), then Linv = Y^T
    std::vector<double> Y((size_t)n * n, 0.0);
    for (int64_t i = 0; i < n; ++i) Y[i * n + i] = 1.0;
    trsm_right_lower_t(n, n, L, lda, Y.data(), n, par);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) Linv[i * n + j] = (j <= i) ? Y[j * n + i] : 0.0;
}

}  // namespace dense
}  // namespace bido
