// Host check of the face point-to-point maps used by the affine-lattice face
// kernel (one 16-point block, P2/P3): applied to the face traces of every mode
// of either side, the tangential-derivative maps must give the traces of the
// modal derivatives, and the lifting map applied to the jump must give the
// modal averaged-lifting map.  Both fragment orders (FP64 and FP32 MFMA result
// rows) are checked.  Prints one line per order: "order <p> <deriv_err> <lift_err> <scale>".
#include <cmath>
#include <cstdio>

#include "dg_internal.h"

using namespace dgh;

int main() {
  for (int order = 2; order <= 3; ++order) {
    const double h[3] = {0.3, 0.5, 0.7};  // anisotropic spacing: exercises the 2/h_t scaling
    HostTables T = build_tables(3, order, 0, order + 1, h);
    MfmaHost M = build_mfma_tables(T);
    const int nb = T.nb, nfq = T.nfq;
    auto phi = [&](int p, int side, int k, int b) { return T.fPhi[(((size_t)p * 2 + side) * nfq + k) * nb + b]; };
    double derr = 0.0, lerr = 0.0, scale = 0.0;
    for (int prec = 0; prec < 2; ++prec) {
      const std::vector<double>& A = prec ? M.dAf : M.dA;
      auto apply = [&](int p, int slot, int i, auto&& x) {  // sum_k map[i][k] x(k)
        double acc = 0.0;
        for (int ks = 0; ks < 4; ++ks)
          for (int g = 0; g < 4; ++g) {
            const int k = prec ? 4 * g + ks : g + 4 * ks;
            if (k < nfq) acc += A[(((size_t)p * 3 + slot) * 4 + ks) * 64 + i + 16 * g] * x(k);
          }
        return acc;
      };
      for (int p = 0; p < 3; ++p)
        for (int side = 0; side < 2; ++side)
          for (int b = 0; b < nb; ++b)
            for (int i = 0; i < 16; ++i) {
              for (int jt = 0; jt < 2; ++jt) {
                const int t = (jt == 0) ? (p == 0 ? 1 : 0) : (p == 2 ? 1 : 2);
                const double got = apply(p, jt, i, [&](int k) { return phi(p, side, k, b); });
                const double ref = i < nfq ? T.fDphi[((((size_t)p * 2 + side) * 3 + t) * nfq + i) * nb + b] : 0.0;
                derr = std::fmax(derr, std::fabs(got - ref));
                scale = std::fmax(scale, std::fabs(ref));
              }
              // side 0: owner modes, traced on its +p face; side 1: neighbour modes on its -p face
              const double got = apply(p, 2, i, [&](int k) { return side == 0 ? phi(p, 1, k, b) : -phi(p, 0, k, b); });
              const double ref = i < nfq ? T.fLift[(((size_t)p * 2 + side) * nfq + i) * nb + b] : 0.0;
              lerr = std::fmax(lerr, std::fabs(got - ref));
              scale = std::fmax(scale, std::fabs(ref));
            }
    }
    std::printf("order %d %.6e %.6e %.6e\n", order, derr, lerr, scale);
  }
  return 0;
}
