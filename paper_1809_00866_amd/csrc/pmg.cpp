// p-multigrid preconditioner (Sec. 2.4): Alg. vcic or Alg. fullvcic on levels
// k_0 > k_1 (> k_2) with inherited coarse operators (eq. GalProj) and
// fixed-count GMRES smoothers preconditioned by element-wise block Jacobi
// (EWBJ) on every level.
//
// * Level 0 applies the matrix-free operator G_0 = shift*I + J(w) (exact Jv).
// * The first coarse level's operator is probed from G_0: for every colour of
//   a distance-2 colouring (no two elements of a colour share a face
//   neighbour, so every element sees at most one perturbed element among
//   itself and its neighbours) and every coarse mode l, G_0 is applied to the
//   zero-padded unit vectors of that colour; each element's restricted
//   response is one column of the block that couples it to the perturbed
//   element.  Deeper levels keep the leading sub-blocks (eq. GalProj with the
//   unit-diagonal projection matrices of a hierarchical orthonormal basis).
// * The smoothers run entirely on the device (Arnoldi by classical
//   Gram-Schmidt with one re-orthogonalisation, Givens rotations and the
//   triangular solve in one-thread kernels), so one V-cycle is a fixed
//   sequence of kernel launches; setup captures it into a hipGraph that every
//   apply replays on a library stream, ordered against the caller's stream
//   by events.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "context.h"

namespace dgc {

struct MgLevel {
  int order = 0, nb = 0, m = 0, iters = 0;
  int64_t n = 0;               // level vector length ne*nv*nb
  double* B = nullptr;         // coarse levels: BSR blocks [nslot][ne][m*m]
  double* Bs = nullptr;        // rescaled hierarchy, level 1: its stabilisation part (same layout)
  float* B32 = nullptr;        // FP32 copy of B applied inside the cycle (FP32/BF16 storage)
  double* Ilu = nullptr;       // coarsest level with block ILU(0): D'^{-1} [ne][m*m] (FP64)
  void* Dinv = nullptr;        // coarse levels: block-Jacobi inverses
  double* g = nullptr;         // right-hand side
  double* x = nullptr;         // iterate
  double* t = nullptr;         // defect / work
  double* z = nullptr;         // preconditioned vector
  double* h = nullptr;         // full cycle: prolonged coarser solution
  double* V = nullptr;         // Krylov basis [(iters+1)][n]
  double* sc = nullptr;        // smoother scalars (kScSize)
  dgk::BsrShape bshape{};      // coarse levels: launch shape of the block-sparse apply (autotuned)
  dgk::ApplyShape ashape{};    // coarse levels: launch shape of the block-Jacobi apply (autotuned)
};

struct MgState {
  int nlev = 0, nslot = 0, storage = DG_FP64;
  int fine_prec = DG_FP64;  // precision of the fine-level operator inside the cycle (DG_FP64/FP32/BF16)
  bool full = false;      // Alg. fullvcic instead of Alg. vcic
  bool rescale = false;   // rescaled-inherited coarse operators (App. A)
  bool coarse_ilu = false;  // block ILU(0) preconditions the coarsest smoother
  double shift = 0.0;
  bool use_graph = false, ready = false;
  MgLevel lev[3];
  double* w = nullptr;         // linearisation state (own copy)
  double* red = nullptr;       // reduction partials [kMaxSmooth+4][kRedBlocks]
  int* color2 = nullptr;
  int ncolor2 = 0;
  hipStream_t gs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_a = nullptr, ev_b = nullptr;
};

void mg_destroy(MgState* M) {
  if (!M) return;
  if (M->exec) (void)hipGraphExecDestroy(M->exec);
  if (M->graph) (void)hipGraphDestroy(M->graph);
  if (M->gs) (void)hipStreamDestroy(M->gs);
  if (M->ev_a) (void)hipEventDestroy(M->ev_a);
  if (M->ev_b) (void)hipEventDestroy(M->ev_b);
  for (auto& L : M->lev) {
    dfree(L.B);
    dfree(L.Bs);
    dfree(L.B32);
    dfree(L.Ilu);
    dfree(L.Dinv);
    dfree(L.g);
    dfree(L.x);
    dfree(L.t);
    dfree(L.z);
    dfree(L.h);
    dfree(L.V);
    dfree(L.sc);
  }
  dfree(M->w);
  dfree(M->red);
  dfree(M->color2);
  delete M;
}

void mg_invalidate(MgState* M) {
  if (M) M->ready = false;
}

bool mg_ready(const MgState* M) { return M && M->ready; }

std::string mg_tuning_report(const MgState* M) {
  std::string r;
  if (!M) return r;
  for (int l = 1; l < M->nlev; ++l) {
    const MgLevel& L = M->lev[l];
    const char* st = M->storage == DG_FP64 ? "fp64" : (M->storage == DG_FP32 ? "fp32" : "bf16");
    r += "mg level " + std::to_string(l) + " (P" + std::to_string(L.order) + ", m=" + std::to_string(L.m) +
         "): " + bsr_shape_name(L.bshape, L.m, L.B32 != nullptr) + (L.B32 ? " (fp32 blocks)" : " (fp64 blocks)") +
         "; block apply " + st + ": " + apply_shape_name(L.ashape, L.m) + "\n";
  }
  return r;
}

namespace {

int binom(int n, int k) {
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return (int)r;
}

// ---------------------------------------------------------------- level ops
// exact: the FP64 level operator even where the cycle applies an FP32 copy
dg_status level_G(dg_context* c, MgState* M, int l, const double* x, double* y, hipStream_t s, bool exact = false) {
  if (l == 0)
    return eval_op(c, exact ? DG_FP64 : M->fine_prec, true, M->w, x, M->shift, y, s);
  const MgLevel& L = M->lev[l];
  if (L.B32 && !exact)
    HIPCHK(dgk::launch_bsr_apply_f32(L.bshape, L.B32, c->mesh.nbr, 2 * c->dim, L.m, c->ne, x, y, s));
  else if (L.B32)  // the shape was tuned for the FP32 copy: the FP64 blocks take the default
    HIPCHK(dgk::launch_bsr_apply(dgk::BsrShape{}, L.B, c->mesh.nbr, 2 * c->dim, L.m, c->ne, x, y, s));
  else
    HIPCHK(dgk::launch_bsr_apply(L.bshape, L.B, c->mesh.nbr, 2 * c->dim, L.m, c->ne, x, y, s));
  return DG_OK;
}

dg_status level_Minv(dg_context* c, MgState* M, int l, const double* r, double* z, hipStream_t s) {
  if (l == 0) {
    HIPCHK(dgk::launch_block_apply(c->blk_storage, c->d_Dinv, c->nv * c->nb, c->ne, r, z, s, &c->blk_shape));
  } else if (l == M->nlev - 1 && M->coarse_ilu) {
    const MgLevel& L = M->lev[l];
    HIPCHK(dgk::launch_ilu_apply(L.B, c->mesh.nbr, c->d_color, c->ncolor, 2 * c->dim, L.m, c->ne, L.Ilu, r, z, s));
  } else {
    const MgLevel& L = M->lev[l];
    HIPCHK(dgk::launch_block_apply(M->storage, L.Dinv, L.m, c->ne, r, z, s, &L.ashape));
  }
  return DG_OK;
}

dg_status lnorm(MgState* M, const double* x, int64_t n, double* dout, hipStream_t s) {
  HIPCHK(dgk::launch_dot_partials(x, x, n, M->red, s));
  HIPCHK(dgk::launch_sum_partials(M->red, dgk::kRedBlocks, dout, 1, s));
  return DG_OK;
}

// x <- SMOOTH(G_l, g, x): `iters` right-preconditioned GMRES steps, one cycle.
// zero_start: x0 = 0 (x is overwritten, its old content unused).
dg_status smooth(dg_context* c, MgState* M, int l, bool zero_start, hipStream_t s) {
  MgLevel& L = M->lev[l];
  const int m = L.iters;
  const int64_t n = L.n;
  dg_status st;
  if (m == 0) {
    if (zero_start) HIPCHK(dgk::launch_fill(L.x, n, 0.0, s));
    return DG_OK;
  }
  double* V0 = L.V;
  if (zero_start) {
    HIPCHK(dgk::launch_axpby(n, 1.0, L.g, 0.0, L.g, V0, s));
  } else {
    if ((st = level_G(c, M, l, L.x, L.t, s)) != DG_OK) return st;
    HIPCHK(dgk::launch_axpby(n, 1.0, L.g, -1.0, L.t, V0, s));
  }
  if ((st = lnorm(M, V0, n, L.sc + dgk::kScBeta, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_gmres_init(L.sc, m, s));
  HIPCHK(dgk::launch_scale_dev(n, V0, L.sc + dgk::kScBeta, V0, s));
  for (int j = 0; j < m; ++j) {
    double* Vj = L.V + (size_t)j * n;
    double* Wn = L.V + (size_t)(j + 1) * n;
    if ((st = level_Minv(c, M, l, Vj, L.z, s)) != DG_OK) return st;
    if ((st = level_G(c, M, l, L.z, Wn, s)) != DG_OK) return st;
    // first pass: dots with V_0..V_j and, as entry j + 1 (Wn is V_{j+1}), |Wn|^2
    HIPCHK(dgk::launch_mdot(L.V, j + 2, n, Wn, M->red, s));
    HIPCHK(dgk::launch_msum(M->red, j + 2, L.sc + dgk::kScH1, s));
    HIPCHK(dgk::launch_mupdate(L.V, j + 1, n, L.sc + dgk::kScH1, Wn, s));
    HIPCHK(dgk::launch_mdot(L.V, j + 1, n, Wn, M->red, s));
    HIPCHK(dgk::launch_msum(M->red, j + 1, L.sc + dgk::kScH2, s));
    HIPCHK(dgk::launch_mupdate(L.V, j + 1, n, L.sc + dgk::kScH2, Wn, s));
    HIPCHK(dgk::launch_dot_partials(Wn, Wn, n, M->red, s));
    HIPCHK(dgk::launch_norm_gmres_step(M->red, dgk::kRedBlocks, L.sc, j, m, s));
    HIPCHK(dgk::launch_scale_by(n, Wn, L.sc + dgk::kScInv, s));
  }
  HIPCHK(dgk::launch_gmres_backsolve(L.sc, m, s));
  HIPCHK(dgk::launch_fill(L.t, n, 0.0, s));
  HIPCHK(dgk::launch_mupdate_add(L.V, m, n, L.sc + dgk::kScY, L.t, s));
  if ((st = level_Minv(c, M, l, L.t, L.z, s)) != DG_OK) return st;
  if (zero_start) {
    HIPCHK(dgk::launch_axpby(n, 1.0, L.z, 0.0, L.z, L.x, s));
  } else {
    HIPCHK(dgk::launch_axpby(n, 1.0, L.x, 1.0, L.z, L.x, s));
  }
  return DG_OK;
}

// lev[l].x <- MG_V(l, lev[l].g, 0)  (Alg. vcic)
dg_status vcycle(dg_context* c, MgState* M, int l, hipStream_t s) {
  dg_status st;
  MgLevel& L = M->lev[l];
  if (l == M->nlev - 1) return smooth(c, M, l, true, s);  // coarsest-level solve
  if ((st = smooth(c, M, l, true, s)) != DG_OK) return st;  // pre-smoothing
  // coarse-grid correction of the defect d = g - G x
  if ((st = level_G(c, M, l, L.x, L.t, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_axpby(L.n, 1.0, L.g, -1.0, L.t, L.t, s));
  MgLevel& C = M->lev[l + 1];
  HIPCHK(dgk::launch_restrict(L.t, L.nb, C.g, C.nb, c->nv, c->ne, s));
  if ((st = vcycle(c, M, l + 1, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_prolong_add(C.x, C.nb, L.x, L.nb, c->nv, c->ne, s));
  return smooth(c, M, l, false, s);  // post-smoothing
}

// lev[l].x <- MG_full(l, lev[l].g, 0)  (Alg. fullvcic); lev[l].g is consumed
// (it ends as the defect that the V-cycle correction solved for)
dg_status fullcycle(dg_context* c, MgState* M, int l, hipStream_t s) {
  dg_status st;
  MgLevel& L = M->lev[l];
  if (l == M->nlev - 1) return smooth(c, M, l, true, s);  // coarsest-level solve
  MgLevel& C = M->lev[l + 1];
  HIPCHK(dgk::launch_restrict(L.g, L.nb, C.g, C.nb, c->nv, c->ne, s));
  if ((st = fullcycle(c, M, l + 1, s)) != DG_OK) return st;
  // initial iterate: the prolonged coarser solution, then its defect
  HIPCHK(dgk::launch_fill(L.h, L.n, 0.0, s));
  HIPCHK(dgk::launch_prolong_add(C.x, C.nb, L.h, L.nb, c->nv, c->ne, s));
  if ((st = level_G(c, M, l, L.h, L.t, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_axpby(L.n, 1.0, L.g, -1.0, L.t, L.g, s));
  if ((st = vcycle(c, M, l, s)) != DG_OK) return st;  // V-cycle correction
  HIPCHK(dgk::launch_axpby(L.n, 1.0, L.x, 1.0, L.h, L.x, s));
  return DG_OK;
}

dg_status cycle(dg_context* c, MgState* M, hipStream_t s) {
  return M->full ? fullcycle(c, M, 0, s) : vcycle(c, M, 0, s);
}

// (Re)captures one cycle into M->graph / M->exec on the library stream.
dg_status capture(dg_context* c, MgState* M) {
  if (M->exec) (void)hipGraphExecDestroy(M->exec);
  if (M->graph) (void)hipGraphDestroy(M->graph);
  M->exec = nullptr;
  M->graph = nullptr;
  dg_status st = DG_OK;
  const bool prof = c->prof;
  c->prof = false;  // no event records inside the captured graph
  hipError_t e = hipStreamBeginCapture(M->gs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = cycle(c, M, M->gs);
    e = hipStreamEndCapture(M->gs, &M->graph);
  }
  c->prof = prof;
  if (e != hipSuccess) return fail(DG_ERR_HIP, std::string("cycle capture: ") + hipGetErrorString(e));
  if (st != DG_OK) return st;
  HIPCHK(hipGraphInstantiate(&M->exec, M->graph, nullptr, nullptr, 0));
  return DG_OK;
}

// ---------------------------------------------------------------- colouring
// Distance-2 colouring: the lattice colouring (i + 2j + 3k) mod q (2D:
// (i + 2j) mod q) for the smallest q that passes the check, else greedy.
std::vector<int> distance2_colouring(const std::vector<int64_t>& nbrT, int dim, int64_t ne, int* ncolor) {
  const int nf = 2 * dim;
  auto elem = [&](int64_t K, int s) { return s == 0 ? K : nbrT[(size_t)(s - 1) * ne + K]; };
  auto valid = [&](const std::vector<int>& col) {
    // the closed neighbourhood of every element must carry distinct elements' distinct colours
    for (int64_t K = 0; K < ne; ++K)
      for (int a = 0; a <= nf; ++a)
        for (int b = a + 1; b <= nf; ++b) {
          const int64_t A = elem(K, a), Bv = elem(K, b);
          if (A != Bv && col[A] == col[Bv]) return false;
        }
    return true;
  };
  std::vector<int> best;
  // lattice indices from the face-neighbour topology: a breadth-first walk
  // from element 0, one step along +-axis i per face crossed (the check
  // below rejects colourings that do not survive the periodic wrap)
  std::vector<std::array<long, 3>> ijk(ne, std::array<long, 3>{0, 0, 0});
  {
    std::vector<char> seen(ne, 0);
    std::vector<int64_t> queue;
    queue.reserve(ne);
    for (int64_t root = 0; root < ne; ++root) {
      if (seen[root]) continue;
      seen[root] = 1;
      queue.push_back(root);
      for (size_t qh = queue.size() - 1; qh < queue.size(); ++qh) {
        const int64_t K = queue[qh];
        for (int fc = 0; fc < nf; ++fc) {
          const int64_t J = nbrT[(size_t)fc * ne + K];
          if (J < 0 || J >= ne || seen[J]) continue;
          seen[J] = 1;
          ijk[J] = ijk[K];
          ijk[J][fc / 2] += (fc % 2) ? 1 : -1;
          queue.push_back(J);
        }
      }
    }
  }
  for (int q = 2 * dim + 1; q <= 4 * dim && best.empty(); ++q) {
    std::vector<int> col(ne);
    for (int64_t e = 0; e < ne; ++e) {
      long v = 0;
      for (int i = 0; i < dim; ++i) v += (long)(i + 1) * ijk[e][i];
      col[e] = (int)(((v % q) + q) % q);
    }
    if (valid(col)) {
      best = col;
      *ncolor = q;
    }
  }
  // greedy
  std::vector<int> gcol(ne, -1);
  int gn = 0;
  for (int64_t e = 0; e < ne; ++e) {
    std::vector<char> used(64 * 8, 0);
    for (int a = 0; a <= nf; ++a) {
      const int64_t A = elem(e, a);
      for (int b = 0; b <= nf; ++b) {
        const int64_t C = elem(A, b);
        if (C != e && gcol[C] >= 0) used[gcol[C]] = 1;
      }
    }
    int k = 0;
    while (used[k]) ++k;
    gcol[e] = k;
    gn = std::max(gn, k + 1);
  }
  if (best.empty() || gn < *ncolor) {
    *ncolor = gn;
    return gcol;
  }
  return best;
}

}  // namespace

dg_status mg_apply(dg_context* c, const double* r, double* z, hipStream_t s) {
  MgState* M = c->mg;
  MgLevel& L0 = M->lev[0];
  ProfScope ps(c, "mg_vcycle", s);
  HIPCHK(dgk::launch_axpby(L0.n, 1.0, r, 0.0, r, L0.g, s));
  if (M->exec) {
    HIPCHK(hipEventRecord(M->ev_a, s));
    HIPCHK(hipStreamWaitEvent(M->gs, M->ev_a, 0));
    HIPCHK(hipGraphLaunch(M->exec, M->gs));
    HIPCHK(hipEventRecord(M->ev_b, M->gs));
    HIPCHK(hipStreamWaitEvent(s, M->ev_b, 0));
  } else {
    dg_status st;
    if ((st = cycle(c, M, s)) != DG_OK) return st;
  }
  HIPCHK(dgk::launch_axpby(L0.n, 1.0, L0.x, 0.0, L0.x, z, s));
  return DG_OK;
}

dg_status mg_set_level_shape(dg_context* c, int level, const dgk::BsrShape* b, const dgk::ApplyShape* a) {
  MgState* M = c->mg;
  if (!mg_ready(M)) return fail(DG_ERR_STATE, "dg_mg_setup has not succeeded since the last block setup");
  if (level < 1 || level >= M->nlev) return fail(DG_ERR_ARG, "coarse level out of range");
  MgLevel& L = M->lev[level];
  if (b) {
    if (!dgk::bsr_shape_fits(*b, L.m, L.B32 ? 4 : 8, 2 * c->dim))
      return fail(DG_ERR_ARG, "block-sparse apply shape does not fit this level");
    L.bshape = *b;
  }
  if (a) {
    if (!dgk::apply_shape_fits(*a, L.m, M->storage)) return fail(DG_ERR_ARG, "block apply shape does not fit this level");
    L.ashape = *a;
  }
  return mg_recapture(c);
}

dg_status mg_recapture(dg_context* c) {
  MgState* M = c->mg;
  if (!mg_ready(M) || !M->use_graph) return DG_OK;
  return capture(c, M);
}

}  // namespace dgc

using namespace dgc;

extern "C" {

dg_status dg_mg_setup(dg_context* c, const double* w, double shift, const dg_mg_opts* o, void* stream) {
  if (!c || !w || !o) return fail(DG_ERR_ARG, "null argument");
  if (c->prm.basis != DG_BASIS_PK) return fail(DG_ERR_ARG, "p-multigrid needs the total-degree basis");
  if (o->n_levels < 2 || o->n_levels > 3) return fail(DG_ERR_ARG, "n_levels must be 2 or 3");
  if (o->orders[0] != c->prm.order) return fail(DG_ERR_ARG, "orders[0] must equal the context's order");
  for (int l = 1; l < o->n_levels; ++l)
    if (o->orders[l] < 0 || o->orders[l] >= o->orders[l - 1])
      return fail(DG_ERR_ARG, "orders must be strictly decreasing and >= 0");
  for (int l = 0; l < o->n_levels; ++l)
    if (o->smooth_iters[l] < 0 || o->smooth_iters[l] > dgk::kMaxSmooth)
      return fail(DG_ERR_ARG, "smooth_iters must lie in 0..60");
  if (o->smooth_iters[o->n_levels - 1] < 1) return fail(DG_ERR_ARG, "the coarsest level needs >= 1 iteration");
  if (o->storage != DG_FP64 && o->storage != DG_FP32 && o->storage != DG_BF16)
    return fail(DG_ERR_ARG, "storage must be DG_FP64, DG_FP32 or DG_BF16");
  if (o->fine_precision != DG_FP64 && o->fine_precision != DG_FP32 && o->fine_precision != DG_BF16)
    return fail(DG_ERR_ARG, "fine_precision must be DG_FP64, DG_FP32 or DG_BF16");
  if (o->cycle != DG_MG_V && o->cycle != DG_MG_FULL) return fail(DG_ERR_ARG, "cycle must be DG_MG_V or DG_MG_FULL");
  if (o->rescale != 0 && o->rescale != 1) return fail(DG_ERR_ARG, "rescale must be 0 or 1");
  if (o->coarse_ilu != 0 && o->coarse_ilu != 1) return fail(DG_ERR_ARG, "coarse_ilu must be 0 or 1");
  if (o->coarse_ilu && c->nv * binom(o->orders[o->n_levels - 1] + c->dim, c->dim) > 64)
    return fail(DG_ERR_ARG, "block ILU(0) needs coarsest blocks of at most 64 rows");
  if (o->fine_precision == DG_FP32 && !has_f32(c))
    return fail(DG_ERR_ARG, "the FP32 fine operator needs a curved mesh or a 3D P2-P4 lattice configuration");
  if (o->fine_precision == DG_BF16 && !has_prec(c, DG_BF16))
    return fail(DG_ERR_ARG, "the BF16-contraction fine operator needs a 3D P2-P4 lattice configuration");
  hipStream_t s = (hipStream_t)stream;
  const int64_t ne = c->ne;
  const int dim = c->dim, nv = c->nv, nf = 2 * dim;
  dg_status st;
  const auto t_setup = std::chrono::steady_clock::now();

  mg_destroy(c->mg);
  c->mg = nullptr;
  // fine-level block Jacobi (shared with DG_PREC_BJ): the columns of the
  // coarse modes come from the distance-2 probing below, the rest from the
  // face-neighbour colouring
  if (o->storage != DG_FP64 && o->storage != DG_FP32 && o->storage != DG_BF16)
    return fail(DG_ERR_ARG, "storage must be DG_FP64, DG_FP32 or DG_BF16");
  if (nv * c->nb > 256) return fail(DG_ERR_ARG, "block size above 256");
  if ((st = block_alloc(c, o->storage)) != DG_OK) return st;

  auto* M = new MgState();
  c->mg = M;
  auto bail = [&](dg_status e) {
    mg_destroy(M);
    c->mg = nullptr;
    return e;
  };
  M->nlev = o->n_levels;
  M->nslot = nf + 1;
  M->storage = o->storage;
  M->shift = shift;
  M->use_graph = o->use_graph != 0;
  M->fine_prec = o->fine_precision;
  M->full = o->cycle == DG_MG_FULL;
  M->rescale = o->rescale != 0;
  M->coarse_ilu = o->coarse_ilu != 0;
  for (int l = 0; l < M->nlev; ++l) {
    MgLevel& L = M->lev[l];
    L.order = o->orders[l];
    L.nb = binom(L.order + dim, dim);
    L.m = nv * L.nb;
    L.iters = o->smooth_iters[l];
    L.n = ne * L.m;
    if ((st = dalloc(&L.g, (size_t)L.n)) != DG_OK) return bail(st);
    if ((st = dalloc(&L.x, (size_t)L.n)) != DG_OK) return bail(st);
    if ((st = dalloc(&L.t, (size_t)L.n)) != DG_OK) return bail(st);
    if ((st = dalloc(&L.z, (size_t)L.n)) != DG_OK) return bail(st);
    if (M->full && l < M->nlev - 1 && (st = dalloc(&L.h, (size_t)L.n)) != DG_OK) return bail(st);
    if ((st = dalloc(&L.V, (size_t)(L.iters + 1) * L.n)) != DG_OK) return bail(st);
    if ((st = dalloc(&L.sc, (size_t)dgk::kScSize)) != DG_OK) return bail(st);
    HIPCHK(dgk::launch_fill(L.sc, dgk::kScSize, 0.0, s));
  }
  if ((st = dalloc(&M->w, (size_t)c->ndof)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->red, (size_t)(dgk::kMaxSmooth + 4) * dgk::kRedBlocks)) != DG_OK) return bail(st);
  HIPCHK(dgk::launch_axpby(c->ndof, 1.0, w, 0.0, w, M->w, s));

  // distance-2 colouring (host)
  std::vector<int64_t> nbrT((size_t)nf * ne);
  if (hipMemcpy(nbrT.data(), c->d_nbr, nbrT.size() * sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
    return bail(fail(DG_ERR_HIP, "mesh download failed"));
  if (M->coarse_ilu) {
    // the diagonal-only elimination of the block ILU(0) is exact on graphs
    // without triangles (two neighbours of an element that are neighbours
    // of each other: a periodic direction of three elements)
    for (int64_t K = 0; K < ne; ++K)
      for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b) {
          const int64_t J = nbrT[(size_t)a * ne + K], L = nbrT[(size_t)b * ne + K];
          if (J == K || L == K || J == L) continue;
          for (int t = 0; t < nf; ++t)
            if (nbrT[(size_t)t * ne + J] == L)
              return bail(fail(DG_ERR_ARG, "block ILU(0) needs a face-neighbour graph without triangles "
                                           "(no periodic direction of exactly three elements)"));
        }
  }
  std::vector<int> col2 = distance2_colouring(nbrT, dim, ne, &M->ncolor2);
  if ((st = dalloc(&M->color2, (size_t)ne)) != DG_OK) return bail(st);
  if (hipMemcpy(M->color2, col2.data(), ne * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(DG_ERR_HIP, "colour upload failed"));

  // first coarse level probed from G_0, deeper levels by truncation.  Rescaled
  // hierarchy (App. A, eq. GalProjResc): with STB_0 the BR2 stabilisation part
  // of the fine Jacobian, G_1 = R (G_0 - (1 - S_0^1) STB_0) P and
  // STB_1 = S_0^1 R STB_0 P; G_2 = R (G_1 - (1 - S_1^2) STB_1) P, where
  // S_l^{l+1} = k_{l+1} (k_{l+1} + d) / (k_l (k_l + d)).
  auto scale = [&](int l) {
    const double a = M->lev[l].order, b = M->lev[l + 1].order;
    return b * (b + dim) / (a * (a + dim));
  };
  {
    MgLevel& C = M->lev[1];
    const size_t nB = (size_t)M->nslot * ne * C.m * C.m;
    if ((st = dalloc(&C.B, nB)) != DG_OK) return bail(st);
    HIPCHK(dgk::launch_fill(C.B, (int64_t)nB, 0.0, s));
    if (M->rescale) {
      if ((st = dalloc(&C.Bs, nB)) != DG_OK) return bail(st);
      HIPCHK(dgk::launch_fill(C.Bs, (int64_t)nB, 0.0, s));
    }
    const double s01 = scale(0);
    if ((st = tune_fine(c, M->fine_prec, M->w, s)) != DG_OK) return bail(st);
    ProfScope ps(c, "mg_probe", s);
    for (int col = 0; col < M->ncolor2; ++col)
      for (int l = 0; l < C.m; ++l) {
        const int lf = (l / C.nb) * c->nb + l % C.nb;
        HIPCHK(dgk::launch_probe_vector(c->d_t1, M->color2, col, lf, c->nb, nv, ne, s));
        if ((st = eval_op(c, M->fine_prec, true, M->w, c->d_t1, shift, c->d_t2, s)) != DG_OK) return bail(st);
        // the element's own rows: column lf of its fine diagonal block
        HIPCHK(dgk::launch_extract_column(c->d_t2, M->color2, col, lf, nv * c->nb, ne, shift, c->d_D64, s));
        if (M->rescale) {
          if ((st = eval_stab(c, M->fine_prec != DG_FP64, M->w, c->d_t1, c->d_t3, s)) != DG_OK) return bail(st);
          HIPCHK(dgk::launch_axpby(c->ndof, 1.0, c->d_t2, -(1.0 - s01), c->d_t3, c->d_t2, s));
          HIPCHK(dgk::launch_axpby(c->ndof, s01, c->d_t3, 0.0, c->d_t3, c->d_t3, s));
          HIPCHK(dgk::launch_extract_bsr(c->d_t3, M->color2, col, l, c->mesh.nbr, nf, c->nb, C.nb, nv, ne, C.Bs, s));
        }
        HIPCHK(dgk::launch_extract_bsr(c->d_t2, M->color2, col, l, c->mesh.nbr, nf, c->nb, C.nb, nv, ne, C.B, s));
      }
    // the remaining columns of the fine blocks with the same operator
    if ((st = block_probe_invert(c, w, shift, o->storage, C.nb, M->fine_prec, s)) != DG_OK) return bail(st);
  }
  for (int l = 2; l < M->nlev; ++l) {
    MgLevel& P = M->lev[l - 1];
    MgLevel& C = M->lev[l];
    const int64_t nP = (int64_t)M->nslot * ne * P.m * P.m;
    if ((st = dalloc(&C.B, (size_t)M->nslot * ne * C.m * C.m)) != DG_OK) return bail(st);
    if (M->rescale) {
      // P.Bs <- G_{l-1} - (1 - S) STB_{l-1}, truncated into G_l (STB_l is not
      // needed: three levels at most)
      HIPCHK(dgk::launch_axpby(nP, 1.0, P.B, -(1.0 - scale(l - 1)), P.Bs, P.Bs, s));
      HIPCHK(dgk::launch_truncate_bsr(P.Bs, P.nb, C.B, C.nb, nv, M->nslot, ne, s));
    } else {
      HIPCHK(dgk::launch_truncate_bsr(P.B, P.nb, C.B, C.nb, nv, M->nslot, ne, s));
    }
  }
  if (M->rescale) {
    HIPCHK(hipStreamSynchronize(s));
    dfree(M->lev[1].Bs);
    M->lev[1].Bs = nullptr;
  }
  // coarse block-Jacobi factors from the diagonal slot
  for (int l = 1; l < M->nlev; ++l) {
    MgLevel& C = M->lev[l];
    const size_t esz = o->storage == DG_FP64 ? 8 : (o->storage == DG_FP32 ? 4 : 2);
    unsigned char* p = nullptr;
    if ((st = dalloc(&p, (size_t)ne * C.m * dgk::block_ld(C.m) * esz)) != DG_OK) return bail(st);
    C.Dinv = p;
    int zero = 0;
    HIPCHK(hipMemcpyAsync(c->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    {
      ProfScope ps(c, "mg_coarse_invert", s);
      HIPCHK(dgk::launch_block_invert(o->storage, C.B, C.m, C.Dinv, C.m, ne, c->d_flag, s));
    }
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return bail(fail(DG_ERR_SINGULAR_BLOCK, "a coarse diagonal block has a zero or non-finite pivot"));
  }
  // block ILU(0) of the coarsest level (colour by colour)
  if (M->coarse_ilu) {
    MgLevel& C = M->lev[M->nlev - 1];
    if ((st = dalloc(&C.Ilu, (size_t)ne * C.m * C.m)) != DG_OK) return bail(st);
    int zero = 0;
    HIPCHK(hipMemcpyAsync(c->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(dgk::launch_ilu_factor(C.B, c->mesh.nbr, c->d_color, c->ncolor, nf, C.m, ne, C.Ilu, c->d_flag, s));
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) return bail(fail(DG_ERR_SINGULAR_BLOCK, "a block ILU(0) pivot block is singular"));
  }
  // reduced-precision storage: the cycle applies FP32 copies of the coarse
  // operators (the preconditioner only; the level operators stay FP64)
  if (M->storage != DG_FP64)
    for (int l = 1; l < M->nlev; ++l) {
      MgLevel& C = M->lev[l];
      const int64_t nB = (int64_t)M->nslot * ne * C.m * C.m;
      if ((st = dalloc(&C.B32, (size_t)nB)) != DG_OK) return bail(st);
      HIPCHK(dgk::launch_to_f32(C.B, C.B32, nB, s));
    }
  // launch shapes of every coarse level's block-sparse and block-Jacobi applies
  for (int l = 1; l < M->nlev; ++l) {
    MgLevel& C = M->lev[l];
    if ((st = tune_bsr(c, C.B, C.B32, C.m, &C.bshape, s)) != DG_OK) return bail(st);
    if ((st = tune_apply(c, M->storage, C.Dinv, C.m, &C.ashape, s)) != DG_OK) return bail(st);
  }
  HIPCHK(hipEventCreateWithFlags(&M->ev_a, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&M->ev_b, hipEventDisableTiming));
  HIPCHK(hipStreamSynchronize(s));
  if (M->use_graph) {
    HIPCHK(hipStreamCreateWithFlags(&M->gs, hipStreamNonBlocking));
    if ((st = capture(c, M)) != DG_OK) return bail(st);
  }
  M->ready = true;
  c->ms_setup_mg = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_setup).count();
  return DG_OK;
}

dg_status dg_mg_update_fine(dg_context* c, const double* w, double shift, int refresh_blocks, void* stream) {
  if (!c || !w) return fail(DG_ERR_ARG, "null argument");
  MgState* M = c->mg;
  if (!M) return fail(DG_ERR_STATE, "dg_mg_setup has not succeeded");
  if (!M->ready && !refresh_blocks)
    return fail(DG_ERR_STATE, "the fine block factors were replaced since dg_mg_setup: pass refresh_blocks");
  hipStream_t s = (hipStream_t)stream;
  dg_status st;
  M->ready = false;
  if (refresh_blocks) {  // all columns with the cycle's fine operator, as at setup
    if ((st = block_alloc(c, M->storage)) != DG_OK) return st;
    if ((st = block_probe_invert(c, w, shift, M->storage, 0, M->fine_prec, s)) != DG_OK) return st;
  }
  HIPCHK(dgk::launch_axpby(c->ndof, 1.0, w, 0.0, w, M->w, s));
  M->shift = shift;
  HIPCHK(hipStreamSynchronize(s));
  if (M->use_graph && (st = capture(c, M)) != DG_OK) return st;  // the shift is a kernel argument
  M->ready = true;
  return DG_OK;
}

dg_status dg_mg_apply(dg_context* c, const double* r, double* z, void* stream) {
  if (!c || !r || !z) return fail(DG_ERR_ARG, "null argument");
  if (r == z) return fail(DG_ERR_ARG, "r and z may not alias");
  if (!mg_ready(c->mg)) return fail(DG_ERR_STATE, "dg_mg_setup has not succeeded since the last block setup");
  return mg_apply(c, r, z, (hipStream_t)stream);
}

dg_status dg_mg_level_apply(dg_context* c, int level, const double* x, double* y, void* stream) {
  if (!c || !x || !y) return fail(DG_ERR_ARG, "null argument");
  if (x == y) return fail(DG_ERR_ARG, "x and y may not alias");
  if (!mg_ready(c->mg)) return fail(DG_ERR_STATE, "dg_mg_setup has not succeeded since the last block setup");
  if (level < 0 || level >= c->mg->nlev) return fail(DG_ERR_ARG, "level out of range");
  return level_G(c, c->mg, level, x, y, (hipStream_t)stream, true);
}

}  // extern "C"
