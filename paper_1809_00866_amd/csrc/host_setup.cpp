// Host-side construction of quadrature rules, the hierarchical modal basis
// and the FP64 operator tables of a uniform affine lattice.
//
// Basis: psi_alpha(xi) = prod_i Lt_{alpha_i}(xi_i), Lt_n = sqrt((2n+1)/2) P_n.
// Space P_k (total degree <= k, the paper's broken space, Sec. 2.1) or Q_k.
// Ordering: ascending total degree, then descending alpha_1, then descending
// alpha_2, so that the leading dim P_k' modes span P_k' (restriction to a
// coarser p-level keeps leading modes, Sec. 2.4.1).
#include <algorithm>
#include <array>
#include <cmath>
#include <exception>
#include <stdexcept>
#include <string>
#include <thread>

#include "dg_internal.h"

namespace dgh {

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    // Newton iteration on P_n from the classical cosine guess.
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      if (n == 0) p1 = 1.0;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      // P_n'(t) = n (t P_n - P_{n-1}) / (t^2 - 1)
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = t;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
    }
    x[n - 1 - i] = t;  // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - t * t) * dp * dp);
  }
  if (n == 1) {
    x[0] = 0.0;
    w[0] = 2.0;
  }
}

void legendre_orthonormal(int kmax, double x, double* L, double* dL) {
  // Bonnet recursion for P_n and P'_{n+1} = P'_{n-1} + (2n+1) P_n.
  std::vector<double> P(kmax + 2, 0.0), dP(kmax + 2, 0.0);
  P[0] = 1.0;
  dP[0] = 0.0;
  if (kmax >= 1) {
    P[1] = x;
    dP[1] = 1.0;
  }
  for (int n = 1; n < kmax; ++n) {
    P[n + 1] = ((2.0 * n + 1.0) * x * P[n] - n * P[n - 1]) / (n + 1.0);
    dP[n + 1] = dP[n - 1] + (2.0 * n + 1.0) * P[n];
  }
  for (int n = 0; n <= kmax; ++n) {
    double s = std::sqrt((2.0 * n + 1.0) / 2.0);
    L[n] = s * P[n];
    dL[n] = s * dP[n];
  }
}

std::vector<int> multi_indices(int k, int dim, int basis) {
  std::vector<std::array<int, 3>> all;
  int lim[3] = {k, dim > 1 ? k : 0, dim > 2 ? k : 0};
  for (int a2 = 0; a2 <= lim[2]; ++a2)
    for (int a1 = 0; a1 <= lim[1]; ++a1)
      for (int a0 = 0; a0 <= lim[0]; ++a0) {
        int s = a0 + a1 + a2;
        bool ok = (basis == DG_BASIS_PK) ? (s <= k) : (std::max(a0, std::max(a1, a2)) <= k);
        if (ok) all.push_back({a0, a1, a2});
      }
  std::sort(all.begin(), all.end(), [](const std::array<int, 3>& a, const std::array<int, 3>& b) {
    int sa = a[0] + a[1] + a[2], sb = b[0] + b[1] + b[2];
    if (sa != sb) return sa < sb;
    if (a[0] != b[0]) return a[0] > b[0];
    return a[1] > b[1];
  });
  std::vector<int> out;
  for (auto& a : all)
    for (int i = 0; i < dim; ++i) out.push_back(a[i]);
  return out;
}

namespace {

// psi_b and its reference gradient at a point xi[dim].
void eval_psi(const std::vector<int>& alpha, int dim, int kmax, const double* xi, double* psi, double* dpsi) {
  const int nb = (int)alpha.size() / dim;
  std::vector<double> L(3 * (kmax + 1)), dL(3 * (kmax + 1));
  for (int i = 0; i < dim; ++i) legendre_orthonormal(kmax, xi[i], &L[i * (kmax + 1)], &dL[i * (kmax + 1)]);
  for (int b = 0; b < nb; ++b) {
    double v = 1.0;
    for (int i = 0; i < dim; ++i) v *= L[i * (kmax + 1) + alpha[b * dim + i]];
    psi[b] = v;
    for (int j = 0; j < dim; ++j) {
      double g = 1.0;
      for (int i = 0; i < dim; ++i) {
        int a = alpha[b * dim + i];
        g *= (i == j) ? dL[i * (kmax + 1) + a] : L[i * (kmax + 1) + a];
      }
      dpsi[j * nb + b] = g;
    }
  }
}

}  // namespace

HostTables build_tables(int dim, int order, int basis, int nq1d, const double h[3]) {
  if (dim < 2 || dim > 3) throw std::invalid_argument("dim must be 2 or 3");
  HostTables T;
  T.dim = dim;
  T.alpha = multi_indices(order, dim, basis);
  const int nb = (int)T.alpha.size() / dim;
  T.nb = nb;
  T.nq1 = nq1d;
  int nq = 1, nfq = 1;
  for (int i = 0; i < dim; ++i) nq *= nq1d;
  for (int i = 0; i < dim - 1; ++i) nfq *= nq1d;
  T.nq = nq;
  T.nfq = nfq;
  const int kmax = order;

  std::vector<double> x1, w1;
  gauss_legendre(nq1d, x1, w1);
  T.x1 = x1;
  for (int i = 0; i < dim; ++i) T.h[i] = h[i];

  double detJ = 1.0;
  for (int i = 0; i < dim; ++i) detJ *= 0.5 * h[i];
  const double s = 1.0 / std::sqrt(detJ);

  // ---------------- volume tables
  std::vector<double> vW(nq), vDphi((size_t)dim * nq * nb);
  T.vPhi.assign((size_t)nq * nb, 0.0);
  T.vXi.assign((size_t)nq * dim, 0.0);
  std::vector<double> psi(nb), dpsi((size_t)dim * nb);
  for (int q = 0; q < nq; ++q) {
    int r = q;
    double xi[3] = {0, 0, 0}, wq = 1.0;
    for (int i = 0; i < dim; ++i) {
      int k = r % nq1d;
      r /= nq1d;
      xi[i] = x1[k];
      wq *= w1[k];
    }
    for (int i = 0; i < dim; ++i) T.vXi[q * dim + i] = xi[i];
    vW[q] = wq * detJ;
    eval_psi(T.alpha, dim, kmax, xi, psi.data(), dpsi.data());
    for (int b = 0; b < nb; ++b) {
      T.vPhi[q * nb + b] = s * psi[b];
      for (int j = 0; j < dim; ++j) vDphi[((size_t)j * nq + q) * nb + b] = s * (2.0 / h[j]) * dpsi[j * nb + b];
    }
  }
  T.vWD.assign((size_t)dim * nq * nb, 0.0);
  T.vWPhi.assign((size_t)nq * nb, 0.0);
  for (int q = 0; q < nq; ++q)
    for (int b = 0; b < nb; ++b) {
      T.vWPhi[q * nb + b] = vW[q] * T.vPhi[q * nb + b];
      for (int j = 0; j < dim; ++j)
        T.vWD[((size_t)j * nq + q) * nb + b] = vW[q] * vDphi[((size_t)j * nq + q) * nb + b];
    }
  // modal derivative D_j[a][b] = sum_q w|J| phi_a d_j phi_b (exact on affine elements)
  std::vector<double> D((size_t)dim * nb * nb, 0.0);
  for (int j = 0; j < dim; ++j)
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) {
        double acc = 0.0;
        for (int q = 0; q < nq; ++q) acc += vW[q] * T.vPhi[q * nb + a] * vDphi[((size_t)j * nq + q) * nb + b];
        D[((size_t)j * nb + a) * nb + b] = acc;
      }

  // ---------------- face tables
  T.fPhi.assign((size_t)dim * 2 * nfq * nb, 0.0);
  T.fDphi.assign((size_t)dim * 2 * dim * nfq * nb, 0.0);
  T.fWPhi.assign((size_t)dim * 2 * nfq * nb, 0.0);
  T.fLift.assign((size_t)dim * 2 * nfq * nb, 0.0);
  T.vLift.assign((size_t)dim * 3 * nb * nb, 0.0);
  std::vector<double> fW((size_t)dim * nfq);
  for (int p = 0; p < dim; ++p) {
    double detF = 1.0;
    for (int i = 0; i < dim; ++i)
      if (i != p) detF *= 0.5 * h[i];
    for (int side = 0; side < 2; ++side) {
      for (int fq = 0; fq < nfq; ++fq) {
        double xi[3] = {0, 0, 0}, wf = 1.0;
        int r = fq;
        for (int i = 0; i < dim; ++i) {
          if (i == p) {
            xi[i] = side ? 1.0 : -1.0;
            continue;
          }
          int k = r % nq1d;
          r /= nq1d;
          xi[i] = x1[k];
          wf *= w1[k];
        }
        fW[p * nfq + fq] = wf * detF;
        eval_psi(T.alpha, dim, kmax, xi, psi.data(), dpsi.data());
        for (int b = 0; b < nb; ++b) {
          size_t o = (((size_t)p * 2 + side) * nfq + fq) * nb + b;
          T.fPhi[o] = s * psi[b];
          T.fWPhi[o] = fW[p * nfq + fq] * s * psi[b];
          for (int j = 0; j < dim; ++j)
            T.fDphi[((((size_t)p * 2 + side) * dim + j) * nfq + fq) * nb + b] = s * (2.0 / h[j]) * dpsi[j * nb + b];
        }
      }
    }
    // face mass matrices M[st][b][b'] = sum_f w|J_f| phi^s_b phi^t_b'
    auto fphi = [&](int side, int fq, int b) { return T.fPhi[(((size_t)p * 2 + side) * nfq + fq) * nb + b]; };
    std::vector<double> M(4 * (size_t)nb * nb, 0.0);
    for (int st = 0; st < 4; ++st) {
      int sa = st >> 1, sb = st & 1;
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
          double acc = 0.0;
          for (int fq = 0; fq < nfq; ++fq) acc += fW[p * nfq + fq] * fphi(sa, fq, a) * fphi(sb, fq, b);
          M[((size_t)st * nb + a) * nb + b] = acc;
        }
    }
    auto Mst = [&](int sa, int sb, int a, int b) { return M[((size_t)(sa * 2 + sb) * nb + a) * nb + b]; };
    // Local lifting of face sigma (owner L on side +, neighbour R on side -),
    // int r.tau = -int [[U]] {tau}.n, n = +e_p, [[U]] = U_L - U_R:
    //   rhoL = -1/2 (M_++ U_L - M_+- U_R),  rhoR = -1/2 (M_-+ U_L - M_-- U_R)
    // {r} at the face points = 1/2 (sum_b rhoL_b phi+_b + sum_b rhoR_b phi-_b).
    for (int fq = 0; fq < nfq; ++fq)
      for (int bp = 0; bp < nb; ++bp) {
        double cl = 0.0, cr = 0.0;
        for (int b = 0; b < nb; ++b) {
          cl += fphi(1, fq, b) * (-0.5 * Mst(1, 1, b, bp)) + fphi(0, fq, b) * (-0.5 * Mst(0, 1, b, bp));
          cr += fphi(1, fq, b) * (0.5 * Mst(1, 0, b, bp)) + fphi(0, fq, b) * (0.5 * Mst(0, 0, b, bp));
        }
        T.fLift[(((size_t)p * 2 + 0) * nfq + fq) * nb + bp] = 0.5 * cl;
        T.fLift[(((size_t)p * 2 + 1) * nfq + fq) * nb + bp] = 0.5 * cr;
      }
    // Elemental lifting of element e in direction p: its +p face (e is L) and
    // its -p face (e is R), plus the modal derivative D_p:
    //   Ghat_p = (D_p - M_++/2 + M_--/2) U_e + (M_+-/2) U_{e+p} - (M_-+/2) U_{e-p}
    for (int a = 0; a < nb; ++a)
      for (int b = 0; b < nb; ++b) {
        T.vLift[(((size_t)p * 3 + 0) * nb + a) * nb + b] =
            D[((size_t)p * nb + a) * nb + b] - 0.5 * Mst(1, 1, a, b) + 0.5 * Mst(0, 0, a, b);
        T.vLift[(((size_t)p * 3 + 1) * nb + a) * nb + b] = 0.5 * Mst(1, 0, a, b);
        T.vLift[(((size_t)p * 3 + 2) * nb + a) * nb + b] = -0.5 * Mst(0, 1, a, b);
      }
  }
  return T;
}

// ---------------------------------------------------------------- curved elements
// Every element is the multilinear image of [-1,1]^dim through its 2^dim
// corners (corner v at xi_i = +1 where bit i of v is set).  Its basis is
// phi_K = L_K^{-1} psi with L_K L_K^T = sum_q w_q |J_q| psi psi^T (Cholesky of
// the discrete reference mass matrix): orthonormal in the discrete L2(K)
// product and hierarchical (L_K lower triangular); physical gradients
// J^{-T} grad_xi.  Face (p, e) is the +p face of e; its neighbour er is
// reached through e's +p face and sees the face at xi_p = -1 with the same
// tangential reference coordinates.  Normal and area follow Nanson's formula
// from the owner: n dA = |J| J^{-T} e_p dA_ref.
namespace {

void multilinear(int dim, const double* X, const double* xi, double* x, double* J) {
  const int nv = 1 << dim;
  for (int i = 0; i < dim; ++i) {
    x[i] = 0.0;
    for (int j = 0; j < dim; ++j) J[i * 3 + j] = 0.0;
  }
  for (int v = 0; v < nv; ++v) {
    double f[3], df[3];
    for (int i = 0; i < dim; ++i) {
      const int bit = (v >> i) & 1;
      f[i] = bit ? 0.5 * (1.0 + xi[i]) : 0.5 * (1.0 - xi[i]);
      df[i] = bit ? 0.5 : -0.5;
    }
    double N = 1.0;
    for (int i = 0; i < dim; ++i) N *= f[i];
    for (int i = 0; i < dim; ++i) x[i] += N * X[v * dim + i];
    for (int j = 0; j < dim; ++j) {
      double dN = 1.0;
      for (int i = 0; i < dim; ++i) dN *= (i == j) ? df[i] : f[i];
      for (int i = 0; i < dim; ++i) J[i * 3 + j] += dN * X[v * dim + i];
    }
  }
}

// determinant and inverse of the leading dim x dim block of a 3x3 row-major matrix
double det_inv(int dim, const double* J, double* Ji) {
  if (dim == 2) {
    const double d = J[0] * J[4] - J[1] * J[3];
    Ji[0] = J[4] / d;
    Ji[1] = -J[1] / d;
    Ji[3] = -J[3] / d;
    Ji[4] = J[0] / d;
    return d;
  }
  const double a = J[0], b = J[1], c = J[2], d = J[3], e = J[4], f = J[5], g = J[6], h = J[7], k = J[8];
  const double A = e * k - f * h, B = -(d * k - f * g), C = d * h - e * g;
  const double det = a * A + b * B + c * C;
  Ji[0] = A / det;
  Ji[3] = B / det;
  Ji[6] = C / det;
  Ji[1] = -(b * k - c * h) / det;
  Ji[4] = (a * k - c * g) / det;
  Ji[7] = -(a * h - b * g) / det;
  Ji[2] = (b * f - c * e) / det;
  Ji[5] = -(a * f - c * d) / det;
  Ji[8] = (a * e - b * d) / det;
  return det;
}

}  // namespace

namespace {

// Runs f(i0, i1) over [0, n) in chunks on the host's cores; the first
// exception thrown by any chunk is rethrown after every thread has joined.
template <class F>
void parallel_chunks(int64_t n, F f) {
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw, n / 64));
  std::vector<std::thread> th;
  std::vector<std::exception_ptr> err(nt);
  for (int64_t t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      try {
        f(n * t / nt, n * (t + 1) / nt);
      } catch (...) {
        err[t] = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

}  // namespace

CurvedHost build_curved_tables(const HostTables& T, int order, const double* xyz, const int64_t* nbr, int64_t ne) {
  const int dim = T.dim, nb = T.nb, nq = T.nq, nfq = T.nfq, nq1 = T.nq1;
  const int nvtx = 1 << dim, nbt = nb * (nb + 1) / 2, gv = dim * dim + 1, gf = dim + 1 + 2 * dim * dim;
  CurvedHost C;
  std::vector<double> x1, w1;
  gauss_legendre(nq1, x1, w1);
  // reference points and weights: volume (first coordinate fastest) and face rules
  std::vector<double> vxi((size_t)nq * dim), vw(nq), fxi((size_t)nfq * (dim - 1)), fw(nfq);
  for (int q = 0; q < nq; ++q) {
    int r = q;
    double w = 1.0;
    for (int i = 0; i < dim; ++i) {
      const int k = r % nq1;
      r /= nq1;
      vxi[(size_t)q * dim + i] = x1[k];
      w *= w1[k];
    }
    vw[q] = w;
  }
  for (int f = 0; f < nfq; ++f) {
    int r = f;
    double w = 1.0;
    for (int i = 0; i < dim - 1; ++i) {
      const int k = r % nq1;
      r /= nq1;
      fxi[(size_t)f * (dim - 1) + i] = x1[k];
      w *= w1[k];
    }
    fw[f] = w;
  }
  // reference point of face point fq on local face s (s = 2p: xi_p = -1, s = 2p+1: xi_p = +1)
  auto face_xi = [&](int s, int fq, double* xi) {
    const int p = s / 2;
    for (int i = 0, k = 0; i < dim; ++i) xi[i] = (i == p) ? (s % 2 ? 1.0 : -1.0) : fxi[(size_t)fq * (dim - 1) + k++];
  };

  // shared reference tables
  std::vector<double> psi(nb), dpsi((size_t)dim * nb);
  std::vector<double> vpsi((size_t)nq * nb);
  C.rPsiT.assign((size_t)nb * nq, 0.0);
  C.rDPsiT.assign((size_t)dim * nb * nq, 0.0);
  C.rDPsi.assign((size_t)nq * dim * nb, 0.0);
  for (int q = 0; q < nq; ++q) {
    eval_psi(T.alpha, dim, order, &vxi[(size_t)q * dim], psi.data(), dpsi.data());
    for (int a = 0; a < nb; ++a) {
      vpsi[(size_t)q * nb + a] = psi[a];
      C.rPsiT[(size_t)a * nq + q] = psi[a];
      for (int r = 0; r < dim; ++r) {
        C.rDPsiT[((size_t)r * nb + a) * nq + q] = dpsi[(size_t)r * nb + a];
        C.rDPsi[((size_t)q * dim + r) * nb + a] = dpsi[(size_t)r * nb + a];
      }
    }
  }
  const int nfs = 2 * dim;
  std::vector<double> fpsi((size_t)nfs * nfq * nb);  // [s][fq][a]
  C.rFPsiT.assign((size_t)nfs * nb * nfq, 0.0);
  C.rFDPsiT.assign((size_t)nfs * dim * nb * nfq, 0.0);
  for (int s = 0; s < nfs; ++s)
    for (int fq = 0; fq < nfq; ++fq) {
      double xi[3];
      face_xi(s, fq, xi);
      eval_psi(T.alpha, dim, order, xi, psi.data(), dpsi.data());
      for (int a = 0; a < nb; ++a) {
        fpsi[((size_t)s * nfq + fq) * nb + a] = psi[a];
        C.rFPsiT[((size_t)s * nb + a) * nfq + fq] = psi[a];
        for (int r = 0; r < dim; ++r)
          C.rFDPsiT[(((size_t)s * dim + r) * nb + a) * nfq + fq] = dpsi[(size_t)r * nb + a];
      }
    }
  C.rFPsi = fpsi;

  // per element: geometry at the volume points, L_K^{-1} (packed rows)
  C.Linv.assign((size_t)ne * nbt, 0.0);
  C.vGeo.assign((size_t)ne * gv * nq, 0.0);
  C.vX.assign((size_t)dim * nq * ne, 0.0);
  parallel_chunks(ne, [&](int64_t e0, int64_t e1) {
    std::vector<double> wd(nq), M((size_t)nb * nb), L((size_t)nb * nb);
    for (int64_t e = e0; e < e1; ++e) {
      const double* X = xyz + (size_t)e * nvtx * dim;
      for (int q = 0; q < nq; ++q) {
        double x[3], J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Ji[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        multilinear(dim, X, &vxi[(size_t)q * dim], x, J);
        const double dt = det_inv(dim, J, Ji);
        if (!(dt > 0.0)) throw std::invalid_argument("element " + std::to_string(e) + " has a non-positive Jacobian");
        for (int i = 0; i < dim; ++i) C.vX[((size_t)i * nq + q) * ne + e] = x[i];
        double* g = &C.vGeo[(size_t)e * gv * nq];
        for (int i = 0; i < dim; ++i)  // K[i][r] = d xi_r / d x_i: grad_x = K grad_xi
          for (int r = 0; r < dim; ++r) g[(size_t)(i * dim + r) * nq + q] = Ji[r * 3 + i];
        wd[q] = vw[q] * dt;
        g[(size_t)(dim * dim) * nq + q] = wd[q];
      }
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b <= a; ++b) {
          double s = 0.0;
          for (int q = 0; q < nq; ++q) s += wd[q] * vpsi[(size_t)q * nb + a] * vpsi[(size_t)q * nb + b];
          M[(size_t)a * nb + b] = s;
        }
      std::fill(L.begin(), L.end(), 0.0);  // Cholesky M = L L^T
      for (int j = 0; j < nb; ++j) {
        double s = M[(size_t)j * nb + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * nb + k] * L[(size_t)j * nb + k];
        if (!(s > 0.0)) throw std::invalid_argument("element mass matrix not positive definite");
        const double d = std::sqrt(s);
        L[(size_t)j * nb + j] = d;
        for (int i = j + 1; i < nb; ++i) {
          double t = M[(size_t)i * nb + j];
          for (int k = 0; k < j; ++k) t -= L[(size_t)i * nb + k] * L[(size_t)j * nb + k];
          L[(size_t)i * nb + j] = t / d;
        }
      }
      double* Li = &C.Linv[(size_t)e * nbt];  // L^{-1} by forward substitution, column by column
      for (int c = 0; c < nb; ++c)
        for (int i = c; i < nb; ++i) {
          double s = (i == c) ? 1.0 : 0.0;
          for (int k = c; k < i; ++k) s -= L[(size_t)i * nb + k] * Li[(size_t)k * (k + 1) / 2 + c];
          Li[(size_t)i * (i + 1) / 2 + c] = s / L[(size_t)i * nb + i];
        }
    }
  });

  // faces f = p*ne + e (owner e, neighbour across its +p face): normals,
  // area weights, both sides' K, and P = sum over sides of phi(x_f).phi(x_g)
  const int64_t nfc = (int64_t)dim * ne;
  C.fGeo.assign((size_t)nfc * gf * nfq, 0.0);
  C.fP.assign((size_t)nfc * nfq * nfq, 0.0);
  parallel_chunks(nfc, [&](int64_t f0, int64_t f1) {
    std::vector<double> ph((size_t)nfq * nb), xf((size_t)nfq * 3);
    for (int64_t f = f0; f < f1; ++f) {
      const int p = (int)(f / ne);
      const int64_t e = f % ne;
      const int64_t er = nbr[(size_t)e * 2 * dim + 2 * p + 1];
      double* g = &C.fGeo[(size_t)f * gf * nfq];
      double* P = &C.fP[(size_t)f * nfq * nfq];
      double shift[3] = {0.0, 0.0, 0.0};
      for (int side = 0; side < 2; ++side) {
        const int64_t K = side == 0 ? e : er;
        const int s = side == 0 ? 2 * p + 1 : 2 * p;
        const double* X = xyz + (size_t)K * nvtx * dim;
        const double* Li = &C.Linv[(size_t)K * nbt];
        for (int fq = 0; fq < nfq; ++fq) {
          double xi[3], x[3], J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, Ji[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
          face_xi(s, fq, xi);
          multilinear(dim, X, xi, x, J);
          const double dt = det_inv(dim, J, Ji);
          if (!(dt > 0.0)) throw std::invalid_argument("element " + std::to_string(K) + " has a non-positive Jacobian");
          // conforming faces: both sides map face point fq to the same
          // physical point, up to one periodic shift per face
          if (side == 0) {
            for (int i = 0; i < dim; ++i) xf[(size_t)fq * 3 + i] = x[i];
          } else {
            double dev = 0.0, scale = 0.0;
            for (int i = 0; i < dim; ++i) {
              const double d = xf[(size_t)fq * 3 + i] - x[i];
              if (fq == 0) shift[i] = d;
              dev = std::max(dev, std::fabs(d - shift[i]));
              for (int r = 0; r < dim; ++r) scale = std::max(scale, std::fabs(J[i * 3 + r]));
            }
            if (dev > 1e-9 * scale)
              throw std::invalid_argument("face " + std::to_string(p) + " of element " + std::to_string(e) +
                                          " is not conforming: element " + std::to_string(K) +
                                          " sees it with other corners or another orientation");
          }
          for (int i = 0; i < dim; ++i)
            for (int r = 0; r < dim; ++r)
              g[(size_t)(dim + 1 + side * dim * dim + i * dim + r) * nfq + fq] = Ji[r * 3 + i];
          if (side == 0) {  // Nanson: |J| J^{-T} e_p is the area-weighted normal
            double av[3], area2 = 0.0;
            for (int i = 0; i < dim; ++i) {
              av[i] = dt * Ji[p * 3 + i];
              area2 += av[i] * av[i];
            }
            const double area = std::sqrt(area2);
            for (int i = 0; i < dim; ++i) g[(size_t)i * nfq + fq] = av[i] / area;
            g[(size_t)dim * nfq + fq] = fw[fq] * area;
          }
          const double* ps = &fpsi[((size_t)s * nfq + fq) * nb];
          for (int b = 0; b < nb; ++b) {  // phi_b(x_fq) = sum_{a<=b} L^{-1}[b][a] psi_a
            double v = 0.0;
            for (int a = 0; a <= b; ++a) v += Li[(size_t)b * (b + 1) / 2 + a] * ps[a];
            ph[(size_t)fq * nb + b] = v;
          }
        }
        for (int f1q = 0; f1q < nfq; ++f1q)
          for (int f2q = 0; f2q < nfq; ++f2q) {
            double v = 0.0;
            for (int b = 0; b < nb; ++b) v += ph[(size_t)f1q * nb + b] * ph[(size_t)f2q * nb + b];
            P[(size_t)f1q * nfq + f2q] += v;
          }
      }
    }
  });
  return C;
}

MfmaHost build_mfma_tables(const HostTables& T) {
  MfmaHost M;
  const int dim = T.dim, nb = T.nb, nq = T.nq, nfq = T.nfq;
  const int KSB = (nb + 3) / 4, MB = (nb + 15) / 16, RBQ = (nq + 15) / 16, KSP = dim * 4;
  const int KSF = (nfq + 3) / 4, RBF = (nfq + 15) / 16;
  M.vA.assign((size_t)RBQ * KSB * 64, 0.0);
  for (int rb = 0; rb < RBQ; ++rb)
    for (int ks = 0; ks < KSB; ++ks)
      for (int l = 0; l < 64; ++l) {
        const int q = 16 * rb + (l & 15), b = (l >> 4) + 4 * ks;
        if (q < nq && b < nb) M.vA[((size_t)rb * KSB + ks) * 64 + l] = T.vPhi[(size_t)q * nb + b];
      }
  // FP32 MFMA returns rows 4 (l/16) + r of its 16x16 result in register r of
  // lane l; used unchanged as the B operand of the next MFMA, fragment k-step
  // ks in lane group g then carries mode 16 (ks/4) + 4 g + ks%4, so the
  // interpolation table's columns follow that order (4 k-steps per 16 modes).
  M.vAf.assign((size_t)RBQ * 4 * MB * 64, 0.0);
  for (int rb = 0; rb < RBQ; ++rb)
    for (int ks = 0; ks < 4 * MB; ++ks)
      for (int l = 0; l < 64; ++l) {
        const int q = 16 * rb + (l & 15), b = 16 * (ks / 4) + 4 * (l >> 4) + ks % 4;
        if (q < nq && b < nb) M.vAf[((size_t)rb * 4 * MB + ks) * 64 + l] = T.vPhi[(size_t)q * nb + b];
      }
  M.pA.assign((size_t)RBQ * MB * KSP * 64, 0.0);
  for (int rb = 0; rb < RBQ; ++rb)
    for (int mb = 0; mb < MB; ++mb)
      for (int ks = 0; ks < KSP; ++ks)
        for (int l = 0; l < 64; ++l) {
          const int b = 16 * mb + (l & 15), k = (l >> 4) + 4 * ks, j = k >> 4, q = 16 * rb + (k & 15);
          if (q < nq && b < nb)
            M.pA[(((size_t)rb * MB + mb) * KSP + ks) * 64 + l] = -T.vWD[((size_t)j * nq + q) * nb + b];
        }
  M.fA.assign((size_t)dim * 2 * MB * KSF * 64, 0.0);
  for (int p = 0; p < dim; ++p)
    for (int side = 0; side < 2; ++side)
      for (int mb = 0; mb < MB; ++mb)
        for (int ks = 0; ks < KSF; ++ks)
          for (int l = 0; l < 64; ++l) {
            const int b = 16 * mb + (l & 15), fq = (l >> 4) + 4 * ks;
            if (fq < nfq && b < nb)
              M.fA[((((size_t)p * 2 + side) * MB + mb) * KSF + ks) * 64 + l] =
                  (side ? 1.0 : -1.0) * T.fWPhi[(((size_t)p * 2 + side) * nfq + fq) * nb + b];
          }
  // FP64 copies for the 4-block 4x4x4 MFMA on a last mode block of <= 4 rows:
  // tables of layout [outer][MB][KS][64]; lane l = 16 k + 4 v + w of the
  // instruction's A operand feeds block v with A[w][k], the same rows for
  // every block v (the 16 result columns are the blocks' 4 x 4)
  auto rem_layout = [&](const std::vector<double>& src, int ks) {
    std::vector<double> out = src;
    if (MB < 2 || nb - 16 * (MB - 1) > 4) return out;
    const size_t frag = 64, blk = (size_t)ks * frag, outer = src.size() / (MB * blk);
    for (size_t o = 0; o < outer; ++o)
      for (int k = 0; k < ks; ++k) {
        const size_t base = (o * MB + MB - 1) * blk + (size_t)k * frag;
        for (int l = 0; l < 64; ++l) out[base + l] = src[base + (l & 3) + 16 * (l >> 4)];
      }
    return out;
  };
  M.pA64 = rem_layout(M.pA, KSP);
  M.fA64 = rem_layout(M.fA, KSF);
  M.tA.assign((size_t)dim * RBF * 6 * 2 * KSB * 64, 0.0);
  for (int p = 0; p < dim; ++p)
    for (int rbf = 0; rbf < RBF; ++rbf)
      for (int ch = 0; ch < 6; ++ch)
        for (int ks2 = 0; ks2 < 2 * KSB; ++ks2)
          for (int l = 0; l < 64; ++l) {
            const int fq = 16 * rbf + (l & 15);
            const bool left = ks2 < KSB;
            const int b = (l >> 4) + 4 * (left ? ks2 : ks2 - KSB);
            if (fq >= nfq || b >= nb) continue;
            const int side = left ? 1 : 0;  // owner trace on xi_p = +1, neighbour on xi_p = -1
            double v = 0.0;
            if (ch == 0) v = left ? T.fPhi[(((size_t)p * 2 + 1) * nfq + fq) * nb + b] : 0.0;
            else if (ch == 1) v = left ? 0.0 : T.fPhi[(((size_t)p * 2 + 0) * nfq + fq) * nb + b];
            else if (ch < 5)
              v = 0.5 * T.fDphi[((((size_t)p * 2 + side) * dim + (ch - 2)) * nfq + fq) * nb + b];
            else
              v = T.fLift[(((size_t)p * 2 + (left ? 0 : 1)) * nfq + fq) * nb + b];
            M.tA[((((size_t)p * RBF + rbf) * 6 + ch) * 2 * KSB + ks2) * 64 + l] = v;
          }
  // Point-to-point maps on one face's points (one 16-point block), slots 0-1:
  // tangential derivatives.  The face
  // points are the tensor Gauss grid of the two tangential directions t0 < t1
  // (t0 fastest), so d/dx_t of the interpolating tensor polynomial is the 1D
  // Lagrange derivative along that grid line, scaled by 2/h_t.  Exact on face
  // traces: a trace has degree <= order <= nq1 - 1 in each tangential variable.
  // A[i][k] = D_t[i][k] with k the point in result-row order drow(g, ks), so the
  // 16x16 result of a trace MFMA is directly the B operand of this product.
  if (dim == 3 && nfq <= 16) {
    const int n1 = T.nq1;
    int maxdeg = 0;
    for (int v : T.alpha) maxdeg = std::max(maxdeg, v);
    if (maxdeg > n1 - 1) throw std::logic_error("face points do not resolve the trace degree");
    std::vector<double> Dl((size_t)n1 * n1, 0.0);  // Dl[k][m] = l_m'(x_k)
    std::vector<double> bw(n1, 1.0);
    for (int m = 0; m < n1; ++m)
      for (int n = 0; n < n1; ++n)
        if (n != m) bw[m] /= (T.x1[m] - T.x1[n]);
    for (int k = 0; k < n1; ++k) {
      double diag = 0.0;
      for (int m = 0; m < n1; ++m)
        if (m != k) {
          Dl[k * n1 + m] = (bw[m] / bw[k]) / (T.x1[k] - T.x1[m]);
          diag -= Dl[k * n1 + m];
        }
      Dl[k * n1 + k] = diag;
    }
    auto dt = [&](int p, int jt, int i, int k) {  // D_t[i][k] on face p, tangential index jt
      const int t = (jt == 0) ? (p == 0 ? 1 : 0) : (p == 2 ? 1 : 2);
      const int i0 = i % n1, i1 = i / n1, k0 = k % n1, k1 = k / n1;
      if (jt == 0) return i1 == k1 ? (2.0 / T.h[t]) * Dl[i0 * n1 + k0] : 0.0;
      return i0 == k0 ? (2.0 / T.h[t]) * Dl[i1 * n1 + k1] : 0.0;
    };
    // Slot 2: the averaged lifting from the jump at the face points.  With the
    // face mass matrices written out, {r}(x_f) = -1/4 sum_g P_fg w_g (uL - uR)(x_g),
    // P_fg = sum_b phi+_b(x_f) phi+_b(x_g) + phi-_b(x_f) phi-_b(x_g): the same
    // quadrature as the modal lifting map, so equal to it up to rounding.
    auto lift = [&](int p, int i, int k) {
      double acc = 0.0;
      for (int b = 0; b < nb; ++b)
        for (int side = 0; side < 2; ++side)
          acc += T.fPhi[(((size_t)p * 2 + side) * nfq + i) * nb + b] * T.fWPhi[(((size_t)p * 2 + side) * nfq + k) * nb + b];
      return -0.25 * acc;
    };
    M.dA.assign((size_t)dim * 3 * 4 * 64, 0.0);
    M.dAf.assign((size_t)dim * 3 * 4 * 64, 0.0);
    for (int p = 0; p < dim; ++p)
      for (int jt = 0; jt < 3; ++jt)
        for (int ks = 0; ks < 4; ++ks)
          for (int l = 0; l < 64; ++l) {
            const int i = l & 15, g = l >> 4;
            const size_t o = (((size_t)p * 3 + jt) * 4 + ks) * 64 + l;
            const int k64 = g + 4 * ks, k32 = 4 * g + ks;
            auto val = [&](int k) { return jt < 2 ? dt(p, jt, i, k) : lift(p, i, k); };
            if (i < nfq && k64 < nfq) M.dA[o] = val(k64);
            if (i < nfq && k32 < nfq) M.dAf[o] = val(k32);
          }
  } else {
    M.dA.assign(64, 0.0);
    M.dAf.assign(64, 0.0);
  }
  // modal corrected-gradient maps in A-fragment order, k = (source, mode)
  M.lA.assign((size_t)dim * MB * 3 * KSB * 64, 0.0);
  for (int p = 0; p < dim; ++p)
    for (int mb = 0; mb < MB; ++mb)
      for (int ks3 = 0; ks3 < 3 * KSB; ++ks3)
        for (int l = 0; l < 64; ++l) {
          const int src = ks3 / KSB, b = 16 * mb + (l & 15), bp = (l >> 4) + 4 * (ks3 % KSB);
          if (b < nb && bp < nb)
            M.lA[(((size_t)p * MB + mb) * 3 * KSB + ks3) * 64 + l] =
                T.vLift[(((size_t)p * 3 + src) * nb + b) * nb + bp];
        }
  M.lA64 = rem_layout(M.lA, 3 * KSB);
  // the maps act along tensor lines: at most p+1 nonzeros per row
  double big = 0.0;
  for (double v : T.vLift) big = std::max(big, std::fabs(v));
  int kl = 0;
  for (int r = 0; r < dim * 3 * nb; ++r) {
    int cnt = 0;
    for (int b = 0; b < nb; ++b)
      if (std::fabs(T.vLift[(size_t)r * nb + b]) > 1e-14 * big) ++cnt;
    kl = std::max(kl, cnt);
  }
  M.kl = kl;
  return M;
}

}  // namespace dgh
