// Compares the compile-time tabulations used by the kernels (tabulate.hpp) with the host's
// quadrature rules (refelem.cpp, exactness-checked at start-up) and basis gradients.
// Built and run by tests/test_tabulation.py with the host C++ compiler.
#include <cmath>
#include <cstdio>

#include "../paper_2104_08012_amd/csrc/internal.hpp"
#include "../paper_2104_08012_amd/csrc/tabulate.hpp"

template <int P, bool KV>
static double check() {
    constexpr fem::StiffTab<P, KV> tb{};
    const fem::Rule& r = fem::rule_for_degree(KV ? 2 * P - 1 : 2 * P - 2);
    if ((int)r.w.size() != tb.NQ) return 1e300;
    double worst = 0.0;
    const int nl = fem::nloc_of(P);
    double dphi[60];
    for (int q = 0; q < tb.NQ; ++q) {
        worst = std::fmax(worst, std::fabs(tb.w[q] - r.w[q]));
        for (int v = 0; v < 4; ++v) worst = std::fmax(worst, std::fabs(tb.lam[q][v] - r.lam[4 * q + v]));
        fem::eval_basis_grad(P, &r.x[3 * q], nullptr, dphi);
        for (int i = 0; i < nl; ++i)
            for (int d = 0; d < 3; ++d) worst = std::fmax(worst, std::fabs(tb.D[q][d][i] - dphi[i * 3 + d]));
    }
    return worst;
}

int main() {
    const double e[6] = {check<1, false>(), check<1, true>(), check<2, false>(),
                         check<2, true>(), check<3, false>(), check<3, true>()};
    double worst = 0.0;
    for (double v : e) worst = std::fmax(worst, v);
    std::printf("%.3e\n", worst);
    return worst < 1e-14 ? 0 : 1;
}
