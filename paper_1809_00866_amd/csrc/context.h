// Library context shared by the entry-point translation units (internal
// header; not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace dgc {

// Sets the thread-local message returned by dg_last_error and returns s.
dg_status fail(dg_status s, const std::string& m);

#define HIPCHK(call)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return dgc::fail(DG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Timer {
  double ms = 0.0;
  int64_t n = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
};

// Allocates n elements unless *p is already set.
template <class T>
dg_status dalloc(T** p, size_t n) {
  if (*p) return DG_OK;
  if (hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(DG_ERR_OOM, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  return DG_OK;
}


void dfree(void* p);

// Device address of the static scratch array of dg_jvp_noalloc on the current
// device (looked up once per device; noalloc.hip).
dg_status noalloc_scratch_address(void** out);

// p-multigrid preconditioner state (pmg.cpp)
struct MgState;
void mg_destroy(MgState* m);
void mg_invalidate(MgState* m);  // the fine block factors changed
bool mg_ready(const MgState* m);

// learned preconditioner state (mlp.cpp)
struct MlpState;
void mlp_destroy(MlpState* m);
bool mlp_ready(const MlpState* m);

}  // namespace dgc

// FGMRES read-back slots: one per Arnoldi column of a restart cycle (restart
// <= 60), kRbStride doubles each, then the back-substitution vector.
constexpr int kRbSlots = 64, kRbStride = 160;

struct dg_context {
  dg_params prm{};
  int dim = 0, nv = 0, nb = 0, nq1 = 0, nq = 0, nfq = 0, cfg = -1;
  int nmass = 0;                 // leading variables with a time derivative (mass form)
  int64_t ne = 0, ndof = 0;
  int64_t mass_len = 0;          // nmass*nb*ne: the DOF prefix that "shift" multiplies
  dgk::Tables tb{};
  dgk::MTables mt{};
  bool use_mfma = false;
  bool curved = false;           // multilinear (non-lattice) mesh: curved-element kernels
  dgk::CurvedTables ct{};
  double* d_curved = nullptr;    // packed curved tables
  double* d_cvX = nullptr;       // curved volume points [dim][nq][ne] (inside d_curved)
  double* d_cwork = nullptr;     // curved work buffers (Ut, Vt, face jumps and fluxes)
  dgk::CurvedTablesF ctf{};      // FP32 copies for the reduced-precision curved operator
  float* d_curved_f = nullptr;
  float* d_cwork_f = nullptr;
  double* d_mtab = nullptr;
  dgk::MTablesF mtf{};          // FP32 copies for the reduced-precision operator
  float* d_mtab_f = nullptr;
  float* d_Hf = nullptr;        // FP32 face-flux buffer
  double* d_G = nullptr;        // modal corrected gradients [value/tangent][p][c][b][e]
  float* d_Gf = nullptr;        // the same for the FP32 operator
  dgk::Mesh mesh{};
  dgk::Phys ph{};
  double* d_tab = nullptr;
  int64_t* d_nbr = nullptr;
  double* d_x0 = nullptr;
  double* d_H = nullptr;
  double* d_H2 = nullptr;        // element-local probing: face fluxes of the +face neighbours' tangents
  float* d_Hf2 = nullptr;        // the same for the FP32 / BF16-contraction operators
  double* d_cloc = nullptr;      // the same on curved meshes: jump and flux records [3][dim*ne*nv*nfq]
  float* d_cloc_f = nullptr;     // (FP32 curved operator)
  bool self_nbr = false;         // some element is its own face neighbour (a periodic direction of one element)
  int probe_mode = DG_PROBE_AUTO;
  double* d_t1 = nullptr;
  double* d_t2 = nullptr;
  double* d_t3 = nullptr;
  double* d_rw = nullptr;
  double* d_red = nullptr;
  double* d_scal = nullptr;
  int* d_flag = nullptr;
  int* d_color = nullptr;
  int ncolor = 0;
  double* d_D64 = nullptr;
  void* d_Dinv = nullptr;
  int blk_storage = -1;
  size_t dinv_bytes = 0;  // size of a separate (FP32/BF16) inverse buffer
  bool blk_ready = false;
  double* d_V = nullptr;
  double* d_Z = nullptr;
  int kry_m = 0;
  double* h_pin = nullptr;
  hipEvent_t ev_rb[kRbSlots] = {};  // FGMRES: Hessenberg column j copied to pinned slot j
  double ms_setup_bj = 0.0;        // wall time of the last dg_block_precond_setup
  double ms_setup_mg = 0.0;        // wall time of the last dg_mg_setup
  bool prof = false;
  std::map<std::string, dgc::Timer> timers;
  double* d_zero = nullptr;      // ndof zeros (stabilisation-only Jv)
  double* d_ros = nullptr;       // Rosenbrock step: stage vectors, stage state, right-hand side
  int64_t ros_len = 0;           // entries of d_ros
  dgc::MgState* mg = nullptr;    // p-multigrid preconditioner (dg_mg_setup)
  dgc::MlpState* mlp = nullptr;  // learned preconditioner (dg_mlp_*)
  void* d_scratch = nullptr;     // device address of the static scratch array on this device (dg_jvp_noalloc)
  // launch shapes (autotuner, tune.cpp; 0 / kind 0 = the built-in default)
  int tune_mode = DG_TUNE_AUTO;
  int occ[3][2][2] = {};         // [precision][residual, Jv][face, volume kernel]: waves per SIMD
  bool fuse_grad[3][2] = {};     // [precision][residual, Jv]: corrected gradients formed in the volume kernel
  bool fine_tuned[3] = {};       // the fine operator of this precision has been timed
  dgk::ApplyShape blk_shape{};   // fine block-Jacobi apply
};


namespace dgc {

// Records HIP events around a launch on its stream when profiling is on.
struct ProfScope {
  dg_context* c;
  const char* name;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(dg_context* ctx, const char* nm, hipStream_t st) : c(ctx), name(nm), s(st) {
    if (c->prof) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (c->prof) {
      (void)hipEventRecord(b, s);
      c->timers[name].ev.push_back({a, b});
    }
  }
};

// True when the reduced-precision (FP32) operator exists for this context:
// the 3D P2-P4 MFMA kernels on lattices, the curved kernels on curved meshes.
inline bool has_f32(const dg_context* c) {
  return (c->use_mfma && c->d_mtab_f && c->d_Hf && c->d_Gf) ||
         (c->curved && c->d_curved_f && c->d_cwork_f && !c->ct.diffusion);
}
// True when the operator of precision prec (DG_FP64, DG_FP32 or DG_BF16: BF16
// contractions, the 3D P2-P4 lattice MFMA kernels only) exists.
inline bool has_prec(const dg_context* c, int prec) {
  if (prec == DG_FP64) return true;
  if (prec == DG_FP32) return has_f32(c);
  return prec == DG_BF16 && c->use_mfma && c->d_mtab_f && c->d_Hf && c->d_Gf;
}

// True when the diagonal blocks of the operator of precision prec can be
// probed element-locally (every element perturbed at once): the MFMA kernels
// of 3D P2-P4 lattices and the curved-element kernels, on meshes where no
// element is its own face neighbour.
inline bool local_probe_ok(const dg_context* c, int prec) {
  return c->probe_mode == DG_PROBE_AUTO && (c->use_mfma || c->curved) && !c->self_nbr && has_prec(c, prec);
}

// Residual (jvp = false) or exact Jv plus shift*v (jvp = true) on stream s.
dg_status eval_residual(dg_context* c, bool jvp, const double* w, const double* v, double shift, double* out,
                        hipStream_t s);
// Same with FP32 contractions and FP32 pointwise arithmetic (inputs and
// outputs FP64); 3D P2-P4 configurations only.
dg_status eval_residual_f32(dg_context* c, bool jvp, const double* w, const double* v, double shift, double* out,
                            hipStream_t s);
// The residual / exact Jv of the operator of precision prec (DG_FP64, DG_FP32
// or DG_BF16); DG_ERR_ARG when the context has no such operator.
dg_status eval_op(dg_context* c, int prec, bool jvp, const double* w, const double* v, double shift, double* out,
                  hipStream_t s);
// Element-local Jv of the operator of precision prec (local_probe_ok): out_K =
// shift v_K + (dR_K/dU_K) v_K for every element K, i.e. the Jv with each
// element perturbed alone.  v = e_l in every element gives column l of every
// diagonal block in one pass.
dg_status eval_local(dg_context* c, int prec, const double* w, const double* v, double shift, double* out,
                     hipStream_t s);
// out = STB(w) v: the BR2 stabilisation part of the Jacobian (the tangent of
// the face lifting term eta {r} of the face viscous flux only; no shift),
// FP64 or the FP32 operator.
dg_status eval_stab(dg_context* c, bool f32, const double* w, const double* v, double* out, hipStream_t s);
// Element-block Jacobi setup in two steps: storage for the blocks, then the
// probing (element-local where local_probe_ok allows it, else coloured), with
// the operator of precision probe_prec, of every column whose mode index is at
// least skip_modes (the caller has written the others into d_D64) and the
// inversion.
dg_status block_alloc(dg_context* c, int storage);
dg_status block_probe_invert(dg_context* c, const double* w, double shift, int storage, int skip_modes,
                             int probe_prec, hipStream_t s);
// The probing precision of a plain block setup: FP64 for FP64 factors, the
// FP32 operator (where it exists) for FP32 and BF16 factors.
inline int default_probe_prec(const dg_context* c, int storage) {
  return storage != DG_FP64 && has_f32(c) ? DG_FP32 : DG_FP64;
}
// dout[0] = ||x||_2 over the context's DOF vector length.
dg_status norm2(dg_context* c, const double* x, double* dout, hipStream_t s);
// out = shift*v + J(w) v, exact or finite difference.
dg_status jvp_impl(dg_context* c, const double* w, const double* r_w, const double* v, double shift, int mode,
                   double* out, hipStream_t s);

// Autotuner (tune.cpp).  tune_fine times the waves-per-SIMD candidates of the
// MFMA face and volume kernels of the operator of precision prec (residual and
// Jv, at state w) and stores the fastest in c->occ; tune_apply and tune_bsr
// time the block-inverse and block-sparse apply shapes of an m x m block
// structure.  All do nothing (keeping the defaults) in DG_TUNE_FIXED mode or
// while the stream is being captured, use the context's work vectors d_t1..3,
// synchronise the stream, and reuse a process-wide cache keyed by kernel and
// problem shape.
dg_status tune_fine(dg_context* c, int prec, const double* w, hipStream_t s);
dg_status tune_apply(dg_context* c, int storage, const void* Dinv, int m, dgk::ApplyShape* out, hipStream_t s);
dg_status tune_bsr(dg_context* c, const double* B, const float* B32, int m, dgk::BsrShape* out, hipStream_t s);
std::string apply_shape_name(const dgk::ApplyShape& sh, int m);
std::string bsr_shape_name(const dgk::BsrShape& sh, int m, bool f32);
// one line per p-multigrid level with its shapes (pmg.cpp)
std::string mg_tuning_report(const MgState* m);
// Pins the launch shapes of coarse level `level` (null: keep) and re-captures
// the cycle graph; DG_ERR_ARG for a shape that does not fit.
dg_status mg_set_level_shape(dg_context* c, int level, const dgk::BsrShape* b, const dgk::ApplyShape* a);
// Re-captures the cycle graph of a ready hierarchy (fine-level shapes changed).
dg_status mg_recapture(dg_context* c);

// z = MG_V(0, r, 0) with the context's p-multigrid state (must be ready).
dg_status mg_apply(dg_context* c, const double* r, double* z, hipStream_t s);
// z = s_K MLP(x_K(w, r)) for every element (weights must be set).
dg_status mlp_apply(dg_context* c, const double* w, const double* r, double* z, hipStream_t s);

}  // namespace dgc
