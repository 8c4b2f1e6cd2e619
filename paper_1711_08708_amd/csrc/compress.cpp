// Hierarchical compression of the factor panels (placeholder: exact).
#include "host.h"

namespace bido {

void compress(Factor& f, const double* xyz, int dim, double eps, double eta, int n_threads) {
    (void)f; (void)xyz; (void)dim; (void)eps; (void)eta; (void)n_threads;
}

}  // namespace bido
