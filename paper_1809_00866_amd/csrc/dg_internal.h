// Internal declarations shared by the HIP kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dg.h"

namespace dgk {

// Device tables of a uniform affine lattice (every element the same box of
// edge lengths h).  The physical orthonormal basis is phi = psi / sqrt|J|
// with psi the tensor Legendre basis of the reference cube.  All tables are
// FP64, row-major in the index order written next to them.
struct Tables {
  const double* vPhi;    // [NQ][NB]                 phi_b at volume points
  const double* vWD;     // [DIM][NQ][NB]            w_q|J| d phi_b / d x_j
  const double* vWPhi;   // [NQ][NB]                 w_q|J| phi_b (projection)
  const double* vLift;   // [DIM][3][NB][NB]         modal corrected gradient, see below
  const double* fPhi;    // [DIM][2][NFQ][NB]        traces; side 0: xi_p=-1, 1: xi_p=+1
  const double* fDphi;   // [DIM][2][DIM][NFQ][NB]   trace of d phi_b / d x_j
  const double* fLift;   // [DIM][2][NFQ][NB]        averaged local lifting at face points
  const double* fWPhi;   // [DIM][2][NFQ][NB]        w_f|J_f| phi_b (face projection)
  const double* vXi;     // [NQ][DIM]                reference volume points
};
// vLift[p][0] (self), [p][1] (+p neighbour), [p][2] (-p neighbour) give the
// modal coefficients of G_p = d U/dx_p + R^K_p (R^K the elemental lifting):
//   Ghat_p = vLift[p][0] U_e + vLift[p][1] U_{e+p} + vLift[p][2] U_{e-p}.
// fLift[p][0] / [p][1] map the owner / neighbour modes to {r^sigma} at the
// face points (normal component; the lattice normal is +e_p).

// Curved (multilinear) elements: device tables (layouts as in CurvedHost) and
// the face kernel's outputs read by the volume kernel.
template <class R>
struct CurvedTablesT {
  // shared reference tables (see CurvedHost) and per-element / per-face data
  const R *rPsiT, *rDPsiT, *rDPsi, *rFPsiT, *rFDPsiT, *rFPsi;
  const R *Linv, *vGeo, *fGeo, *fP;
  R *Ut, *Vt;  // [ne][nv][nb]          L^{-T} U and L^{-T} V
  R* fJmp;     // [dim*ne][2][nv][nfq]  [[U]] at the face points (value, tangent)
  R* fHn;      // [dim*ne][nv][nfq]     w_f|J_f| times the normal flux (or its tangent)
  // Probing the diagonal blocks element by element (null: the fields above):
  // the tangent read for every face's +p neighbour (face kernel), and the
  // jump and flux records read on an element's -p faces (volume kernel).
  const R* VtN = nullptr;
  const R* fJmpN = nullptr;
  const R* fHnN = nullptr;
  int diffusion = 0;  // the scalar BR2 Laplacian (nv = 1) instead of the compressible equations
};
using CurvedTables = CurvedTablesT<double>;
using CurvedTablesF = CurvedTablesT<float>;  // the reduced-precision curved operator

// Operator tables pre-permuted into the operand order of the FP64 MFMA
// 16x16x4 instruction (A[i][k] at lane i + 16k, B[k][j] at lane j + 16k,
// D[i][j] at lane j + 16 (i % 4), register i / 4), 64 doubles per fragment.
// MFMA operand tables in A-fragment order (lane l = row + 16 k of each 16x4
// k-step), in the working precision R of the kernels that read them.
template <class R>
struct MTablesT {
  const R* vA;     // [RBQ][KSV][64]            interpolation: phi(q, b); KSV = KSB (FP64) or 4 MB
                   //                           with the FP32 fragment order of the modes
  const R* pA;     // [RBQ][MB][DIM*4][64]      projection: -w|J| d_j phi(q, b), k = (j, q)
  const R* fA;     // [DIM][2][MB][KSF][64]     face projection: +/- w_f|J_f| phi(fq, b)
  const R* tA;     // [DIM][RBF][6][2*KSB][64]  face traces (uL, uR, G_1..3 averaged, {r})
  const R* lA;     // [DIM][MB][3*KSB][64]      modal corrected gradient [L0 | L1 | L2]
                   // (FP64 pA, fA, lA: a last mode block of <= 4 rows in the lane
                   // order of the 4-block 4x4x4 instruction, row l % 4 in lane l)
  const R* dA;     // [DIM][3][4][64]           maps between the points of one face: d/dx_t
                   //                           (t: the two tangential directions) and the
                   //                           averaged lifting from the jump; k = face point in
                   //                           the row order of this precision's MFMA result
  int kl;          // max nonzeros per row of the maps (p+1: they act along tensor lines)
};
using MTables = MTablesT<double>;
using MTablesF = MTablesT<float>;

struct Phys {
  double gamma, prandtl, mu, eta, efix;
  int flux;           // DG_FLUX_LF / DG_FLUX_ROE
  int model = 0;      // DG_PHYS_COMPRESSIBLE / DG_PHYS_INCOMPRESSIBLE
  double beta = 1.0;  // incompressible: artificial compressibility speed of the interface flux
  int stab_only = 0;  // Jv face kernels: keep only the tangent of the face lifting
                      // term eta {r} (the BR2 stabilisation part of the Jacobian)
};

struct Mesh {
  int64_t ne;
  const int64_t* nbr;  // [2*DIM][ne]
  const double* x0;    // [DIM][ne] low corner of every element
  double h[3];
};

// Kernel configuration id -> (dim, nb, nq1d).  Returns -1 if not compiled.
int config_index(int dim, int nb, int nq1d);

// Launchers (asynchronous on `stream`).
hipError_t launch_face(int cfg, bool jvp, const double* U, const double* V, double* H, const Tables& tb,
                       const Mesh& m, const Phys& ph, hipStream_t stream);
hipError_t launch_volume(int cfg, bool jvp, const double* U, const double* V, const double* H, double* out,
                         double shift, const Tables& tb, const Mesh& m, const Phys& ph, hipStream_t stream);
// MFMA kernels (3D); return hipErrorInvalidValue when the configuration has none.
bool has_mfma(int cfg);
// Curved-element kernels compiled for the configuration (the compressible
// equations, or the scalar Laplacian on 2D P2/P3/P6 meshes).
bool has_curved(int cfg, bool diffusion = false);
// occ: minimum waves per SIMD of the face / volume kernel's launch bound (1 or
// 2; 0 = the configuration's default); hipErrorInvalidValue for a shape the
// configuration does not have (mfma_occ_fits).  Every occupancy computes the
// same bits.  fused (volume kernel): form the corrected gradients in the
// kernel from U / V (Gm unused) instead of reading them from Gm written by
// launch_grad_mfma; the same chains, so the same bits.
// Probing the diagonal blocks element by element (the last arguments, null
// for the ordinary operator): Vr (face kernel) the tangent of every face's +p
// neighbour in place of V; Hm (volume kernel) the fluxes read on the
// element's -p faces in place of H, Vn the neighbours' tangents of the
// corrected gradients formed in the kernel in place of V.
bool mfma_occ_fits(int cfg, int prec, int face_occ, int volume_occ);
hipError_t launch_face_mfma(int cfg, bool jvp, const double* U, const double* V, double* H, const MTables& mt,
                            const Mesh& m, const Phys& ph, int occ, hipStream_t stream, const double* Vr = nullptr);
// reduced precision variant: FP32 tables, FP32 face-flux buffer, FP32 MFMA and
// pointwise arithmetic, FP64 inputs and outputs
hipError_t launch_face_mfma_f32(int cfg, bool jvp, const double* U, const double* V, float* H, const MTablesF& mt,
                                const Mesh& m, const Phys& ph, int occ, hipStream_t s, const double* Vr = nullptr);
hipError_t launch_volume_mfma_f32(int cfg, bool jvp, const double* U, const double* V, const float* Gm,
                                  const float* H, double* out, double shift, const MTablesF& mt, const Mesh& m,
                                  const Phys& ph, int occ, bool fused, hipStream_t s, const float* Hm = nullptr,
                                  const double* Vn = nullptr);
// BF16 contractions with FP32 accumulation, otherwise as the FP32 variant
// (FP32 tables and buffers, FP32 pointwise arithmetic)
hipError_t launch_grad_mfma_bf16(int cfg, bool jvp, const double* U, const double* V, float* Gm, const MTablesF& mt,
                                 const Mesh& m, hipStream_t s, const double* Vn = nullptr);
hipError_t launch_face_mfma_bf16(int cfg, bool jvp, const double* U, const double* V, float* H, const MTablesF& mt,
                                 const Mesh& m, const Phys& ph, int occ, hipStream_t s, const double* Vr = nullptr);
hipError_t launch_volume_mfma_bf16(int cfg, bool jvp, const double* U, const double* V, const float* Gm,
                                   const float* H, double* out, double shift, const MTablesF& mt, const Mesh& m,
                                   const Phys& ph, int occ, bool fused, hipStream_t s, const float* Hm = nullptr,
                                  const double* Vn = nullptr);
// modal corrected gradients Gm[s][p][c][b][e] (s = value, tangent); Vn: the
// neighbours' tangent coefficients in place of V (zeros when probing the
// diagonal blocks element by element)
hipError_t launch_grad_mfma(int cfg, bool jvp, const double* U, const double* V, double* Gm, const MTables& mt,
                            const Mesh& m, hipStream_t s, const double* Vn = nullptr);
hipError_t launch_grad_mfma_f32(int cfg, bool jvp, const double* U, const double* V, float* Gm, const MTablesF& mt,
                                const Mesh& m, hipStream_t s, const double* Vn = nullptr);
hipError_t launch_volume_mfma(int cfg, bool jvp, const double* U, const double* V, const double* Gm, const double* H,
                              double* out, double shift, const MTables& mt, const Mesh& m, const Phys& ph, int occ,
                              bool fused, hipStream_t stream,
                              const double* Hm = nullptr, const double* Vn = nullptr);
hipError_t launch_project(int cfg, int nv, const double* f, double* w, const Tables& tb, const Mesh& m,
                          hipStream_t s);
hipError_t launch_points(int cfg, double* xyz, const Tables& tb, const Mesh& m, hipStream_t s);
hipError_t launch_wave_speed(int cfg, const double* w, double* partial, int nblocks, const Tables& tb,
                             const Mesh& m, const Phys& ph, hipStream_t s);

// Vector kernels (FP64, deterministic reductions: fixed block partials + one-block final sum).
constexpr int kRedBlocks = 1024;
hipError_t launch_dot_partials(const double* x, const double* y, int64_t n, double* partial, hipStream_t s);
hipError_t launch_sum_partials(const double* partial, int np, double* out, int sqrt_flag, hipStream_t s);
hipError_t launch_axpby(int64_t n, double a, const double* x, double b, const double* y, double* z, hipStream_t s);
// z = a*x + s*y where s = *dscale (device scalar) times c
hipError_t launch_axpy_dev(int64_t n, const double* x, const double* dscale, double c, const double* y, double* z,
                           hipStream_t s);
hipError_t launch_fd_combine(int64_t n, int64_t nm, const double* rp, const double* r0, const double* dinv,
                             const double* v, double shift, double* out, hipStream_t s);
hipError_t launch_scale_dev(int64_t n, const double* x, const double* dnorm, double* y, hipStream_t s);
// Multi-dot h[j] = V_j . w for j < k (V row-major [k][n]); partial buffer [k][kRedBlocks]
hipError_t launch_mdot(const double* V, int k, int64_t n, const double* w, double* partial, hipStream_t s);
hipError_t launch_msum(const double* partial, int k, double* h, hipStream_t s);
// w -= sum_j h[j] V_j
hipError_t launch_mupdate(const double* V, int k, int64_t n, const double* h, double* w, hipStream_t s);
// x += sum_j y[j] Z_j
hipError_t launch_mupdate_add(const double* Z, int k, int64_t n, const double* y, double* x, hipStream_t s);
hipError_t launch_fill(double* x, int64_t n, double v, hipStream_t s);
hipError_t launch_fd_delta(double* d, double eps, hipStream_t s);
hipError_t launch_max_partials(const double* partial, int np, double* out, hipStream_t s);
hipError_t launch_nonfinite_check(const double* x, int64_t n, int* flag, hipStream_t s);

// Block-Jacobi kernels.  Probe vector: e_l in every element of colour col
// (col < 0: in every element); extraction: column l of the diagonal block of
// the same elements.
hipError_t launch_probe_vector(double* P, const int* color, int col, int l, int nb, int nv, int64_t ne,
                               hipStream_t s);
hipError_t launch_extract_column(const double* Jv, const int* color, int col, int l, int m, int64_t ne,
                                 double shift, double* D, hipStream_t s);
// Stored block inverses use the column stride block_ld(m) (16-byte aligned
// columns for every storage type); D64 holds probed blocks with column
// stride ldd (block_ld(m) for the fine blocks).
constexpr int block_ld(int m) { return (m + 7) / 8 * 8; }
hipError_t launch_block_invert(int storage, double* D64, int ldd, void* Dout, int m, int64_t ne, int* info,
                               hipStream_t s);
// Multicolour block ILU(0) of a block-sparse level operator (m <= 64): factor
// (one launch per colour; D'^{-1} FP64, [ne][m*m]) and apply z = (L U)^{-1} r.
hipError_t launch_ilu_factor(const double* B, const int64_t* nbr, const int* color, int ncolor, int nf, int m,
                             int64_t ne, double* Dinv, int* info, hipStream_t s);
hipError_t launch_ilu_apply(const double* B, const int64_t* nbr, const int* color, int ncolor, int nf, int m,
                            int64_t ne, const double* Dinv, const double* r, double* z, hipStream_t s);
// Launch shape of the block-inverse apply: kApplyRow = one lane per row
// (m <= 64; epw waves = elements per workgroup, 1/2/4/8), kApplyVec =
// 16-byte column loads by `threads` threads per element (64, 128, 256, 512;
// epw elements per workgroup: 1, 2 or 4 with 64 threads, else 1); kind 0 =
// the default for m.  The shapes compute the same products; their sums run
// in shape-dependent order.
enum { kApplyDefault = 0, kApplyRow = 1, kApplyVec = 2 };
struct ApplyShape {
  int kind = kApplyDefault, threads = 0, epw = 0;
};
ApplyShape default_apply_shape(int m);
// The shape exists for blocks of m rows stored as `storage` (kind 0 always).
bool apply_shape_fits(const ApplyShape& sh, int m, int storage);
hipError_t launch_block_apply(int storage, const void* Dinv, int m, int64_t ne, const double* r, double* z,
                              hipStream_t s, const ApplyShape* shape = nullptr);

// p-multigrid kernels (level transfer, inherited BSR operators, fixed-count
// GMRES bookkeeping).  Device scalar block of one smoother, in doubles:
constexpr int kMaxSmooth = 60;  // iterations per smoother call
constexpr int kScBeta = 0, kScHn = 2, kScInv = 3, kScFlag = 4;  // |w|^2 before orthogonalisation: kScH1 + j + 1
constexpr int kScH1 = 8, kScH2 = 72, kScCs = 136, kScSn = 200, kScG = 264, kScY = 336, kScR = 400;
constexpr int kScSize = kScR + (kMaxSmooth + 1) * kMaxSmooth + 64;
hipError_t launch_restrict(const double* f, int nbf, double* cv, int nbc, int nv, int64_t ne, hipStream_t s);
hipError_t launch_prolong_add(const double* cv, int nbc, double* f, int nbf, int nv, int64_t ne, hipStream_t s);
hipError_t launch_extract_bsr(const double* Jv, const int* color, int col, int l, const int64_t* nbr, int nf,
                              int nbf, int nbc, int nv, int64_t ne, double* B, hipStream_t s);
hipError_t launch_truncate_bsr(const double* B1, int nb1, double* B2, int nb2, int nv, int nslot, int64_t ne,
                               hipStream_t s);
// Launch shape of the block-sparse level apply: workgroup size (256, 512 or
// 1024), rows per thread (1, 2, 4 (FP32 blocks only); 0 = the widest vector
// load that m allows) and column slices per row (1, 2, 4 or 8).  Shapes that
// do not fit return hipErrorInvalidValue.
struct BsrShape {
  int bs = 512, rpt = 0, cs = 4;
};
inline int bsr_widest_rpt(int m, size_t elem) { return (elem == 4 && m % 4 == 0) ? 4 : (m % 2 == 0 ? 2 : 1); }
// The shape fits blocks of m rows with entries of elem bytes (8 or 4) and nf
// face neighbours: at least one element row per workgroup, within 64 KB of LDS.
bool bsr_shape_fits(const BsrShape& sh, int m, size_t elem, int nf);
hipError_t launch_bsr_apply(const BsrShape& sh, const double* B, const int64_t* nbr, int nf, int m, int64_t ne,
                            const double* x, double* y, hipStream_t s);
// The same with FP32 blocks (FP64 sums); FP64 -> FP32 copy of n entries.
hipError_t launch_bsr_apply_f32(const BsrShape& sh, const float* B, const int64_t* nbr, int nf, int m, int64_t ne,
                                const double* x, double* y, hipStream_t s);
hipError_t launch_to_f32(const double* x, float* y, int64_t n, hipStream_t s);
hipError_t launch_gmres_init(double* sc, int m, hipStream_t s);
// ||w|| = sqrt(sum of the partials) into kScHn, then the Givens update of column j
hipError_t launch_norm_gmres_step(const double* partial, int np, double* sc, int j, int m, hipStream_t s);
hipError_t launch_gmres_backsolve(double* sc, int m, hipStream_t s);
hipError_t launch_scale_by(int64_t n, double* x, const double* sc, hipStream_t s);

// Curved (multilinear) elements: residual / Jv in two passes (faces, then
// volume and gather), L2 projection and maximal wave speed.
hipError_t launch_modal_curved(int cfg, bool jvp, const double* U, const double* V, const CurvedTables& ct,
                               int64_t ne, hipStream_t s);
hipError_t launch_face_curved(int cfg, bool jvp, const CurvedTables& ct, const Mesh& m, const Phys& ph,
                              hipStream_t s);
hipError_t launch_volume_curved(int cfg, bool jvp, const double* V, const CurvedTables& ct, double* out,
                                double shift, const Mesh& m, const Phys& ph, hipStream_t s);
hipError_t launch_modal_curved_f32(int cfg, bool jvp, const double* U, const double* V, const CurvedTablesF& ct,
                                   int64_t ne, hipStream_t s);
hipError_t launch_face_curved_f32(int cfg, bool jvp, const CurvedTablesF& ct, const Mesh& m, const Phys& ph,
                                  hipStream_t s);
hipError_t launch_volume_curved_f32(int cfg, bool jvp, const double* V, const CurvedTablesF& ct, double* out,
                                    double shift, const Mesh& m, const Phys& ph, hipStream_t s);
hipError_t launch_project_curved(int cfg, const double* f, double* w, const CurvedTables& ct, int64_t ne,
                                 hipStream_t s);
hipError_t launch_wave_speed_curved(int cfg, const double* w, double* partial, int nblocks, const CurvedTables& ct,
                                    const Mesh& m, const Phys& ph, hipStream_t s);

}  // namespace dgk

namespace dgh {

// Host-side table construction (C++, FP64).
struct HostTables {
  int dim = 0, nb = 0, nq1 = 0, nq = 0, nfq = 0;
  std::vector<double> vPhi, vWD, vWPhi, vLift, fPhi, fDphi, fLift, fWPhi, vXi;
  std::vector<double> x1;       // 1D Gauss points (reference coordinate)
  double h[3] = {0, 0, 0};      // lattice spacing per direction
  std::vector<int> alpha;  // [nb][dim]
};

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void legendre_orthonormal(int kmax, double x, double* L, double* dL);
std::vector<int> multi_indices(int k, int dim, int basis);
HostTables build_tables(int dim, int order, int basis, int nq1d, const double h[3]);

// Curved (multilinear) elements.  Each element's orthonormal basis is
// phi = L_K^{-1} psi (M_K = L_K L_K^T, the mass matrix of the reference basis
// psi on K), so every contraction runs against the shared reference tables
// of psi on coefficients transformed by L_K^{-1}; per element and per face
// only L_K^{-1} and the point geometry are stored.
struct CurvedHost {
  std::vector<double> rPsiT;    // [nb][nq]             psi_a(xi_q)
  std::vector<double> rDPsiT;   // [dim][nb][nq]        d psi_a / d xi_r
  std::vector<double> rDPsi;    // [nq][dim][nb]
  std::vector<double> rFPsiT;   // [2dim][nb][nfq]      psi_a on local face s (2p: xi_p=-1, 2p+1: +1)
  std::vector<double> rFDPsiT;  // [2dim][dim][nb][nfq]
  std::vector<double> rFPsi;    // [2dim][nfq][nb]
  std::vector<double> Linv;     // [ne][nb(nb+1)/2]     L_K^{-1}, packed lower rows
  std::vector<double> vGeo;     // [ne][dim*dim+1][nq]  K = J^{-T} (grad_x = K grad_xi), w_q|J_q|
  std::vector<double> vX;       // [dim][nq][ne]        physical volume points
  std::vector<double> fGeo;     // [dim*ne][dim+1+2dim^2][nfq]  n (owner to neighbour), w_f|J_f|, K owner, K neighbour
  std::vector<double> fP;       // [dim*ne][nfq][nfq]   sum over both sides of phi(x_f).phi(x_g)
};
CurvedHost build_curved_tables(const HostTables& T, int order, const double* xyz, const int64_t* nbr, int64_t ne);

struct MfmaHost {
  std::vector<double> vA, pA, fA, tA, lA;
  // FP64 copies of pA, fA, lA whose last mode block, when it holds at most 4
  // live rows (P3, P4), is laid out for the 4-block 4x4x4 FP64 MFMA: lane l
  // of a k-step fragment holds A[row l % 4][k-step row l / 16]
  std::vector<double> pA64, fA64, lA64;
  std::vector<double> vAf;  // interpolation table in the FP32 fragment order (4 MB k-steps per point block)
  std::vector<double> dA, dAf;  // face point-to-point maps, FP64 / FP32 result-row order
  int kl = 0;
};
MfmaHost build_mfma_tables(const HostTables& T);

}  // namespace dgh
