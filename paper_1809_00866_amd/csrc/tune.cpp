// Launch-shape autotuner: times the candidate shapes of a kernel family at
// the problem's own size on the caller's stream and keeps the fastest.
//
// Candidate 0 is always the built-in default; another candidate replaces it
// only when it is at least kMargin faster, so timing noise cannot flip a
// choice between equivalent shapes.  A candidate is timed as the best of
// kRounds rounds of kReps back-to-back launches after one warm-up launch;
// candidates whose launch is refused (a shape that does not fit the block
// size, LDS or register budget) are skipped.  Choices are cached per process,
// keyed by kernel family and problem shape (and device), so the timing runs
// once per shape.
#include <array>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "context.h"

namespace dgc {

namespace {

constexpr float kMargin = 0.97f;
constexpr int kRounds = 3, kReps = 3;

enum : int64_t { kFamFine = 1, kFamApply = 2, kFamBsr = 3 };
using Key = std::array<int64_t, 7>;

std::mutex g_mu;
std::map<Key, std::array<int, 3>> g_cache;

bool cached(const Key& k, std::array<int, 3>* v) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cache.find(k);
  if (it == g_cache.end()) return false;
  *v = it->second;
  return true;
}

void store(const Key& k, const std::array<int, 3>& v) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_cache[k] = v;
}

int device_id() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) {
    (void)hipGetLastError();
    return true;  // unknown: leave the defaults
  }
  return st != hipStreamCaptureStatusNone;
}

// Index of the fastest of n candidates; launch(i) enqueues candidate i on s
// and returns false when the candidate is refused.
template <class L>
dg_status pick_fastest(int n, hipStream_t s, L&& launch, int* best) {
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  float t_best = 0.f, t_default = -1.f;
  int i_best = -1;
  dg_status st = DG_OK;
  for (int i = 0; i < n && st == DG_OK; ++i) {
    if (!launch(i)) {
      (void)hipGetLastError();
      continue;
    }
    float t_min = 1e30f;
    for (int r = 0; r < kRounds; ++r) {
      if (hipEventRecord(a, s) != hipSuccess) {
        st = fail(DG_ERR_HIP, "autotuner: hipEventRecord failed");
        break;
      }
      bool ok = true;
      for (int k = 0; k < kReps && ok; ++k) ok = launch(i);
      if (!ok) {
        st = fail(DG_ERR_HIP, "autotuner: a candidate launch failed after its warm-up");
        break;
      }
      float ms = 0.f;
      if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
          hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        st = fail(DG_ERR_HIP, "autotuner: event timing failed");
        break;
      }
      t_min = std::min(t_min, ms);
    }
    if (st != DG_OK) break;
    if (i == 0) t_default = t_min;
    const bool better = i_best < 0 || t_min < t_best;
    const bool clears_margin = i == 0 || t_default < 0.f || t_min < kMargin * t_default;
    if (better && clears_margin) {
      t_best = t_min;
      i_best = i;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != DG_OK) return st;
  if (i_best < 0) return fail(DG_ERR_HIP, "autotuner: no candidate launched");
  *best = i_best;
  return DG_OK;
}

const char* prec_name(int p) { return p == DG_FP64 ? "fp64" : (p == DG_FP32 ? "fp32" : "bf16"); }

}  // namespace

dg_status tune_fine(dg_context* c, int prec, const double* w, hipStream_t s) {
  if (prec < DG_FP64 || prec > DG_BF16) return fail(DG_ERR_ARG, "unknown operator precision");
  if (c->tune_mode != DG_TUNE_AUTO || c->fine_tuned[prec]) return DG_OK;
  if (!c->use_mfma || c->curved || !has_prec(c, prec)) {
    c->fine_tuned[prec] = true;  // no tunable kernels
    return DG_OK;
  }
  if (capturing(s)) return DG_OK;
  // (face occ, volume occ, corrected gradients fused into the volume
  // kernel); occupancy 0 = the configuration's default
  static const int cand[10][3] = {{0, 0, 0}, {1, 1, 0}, {1, 2, 0}, {2, 1, 0}, {2, 2, 0},
                                  {0, 0, 1}, {1, 1, 1}, {1, 2, 1}, {2, 1, 1}, {2, 2, 1}};
  for (int jvp = 0; jvp < 2; ++jvp) {
    const Key k = {kFamFine, c->cfg, prec, jvp, c->ph.model, c->ne, device_id()};
    std::array<int, 3> v{};
    if (!cached(k, &v)) {
      int best = 0;
      auto launch = [&](int i) {
        c->occ[prec][jvp][0] = cand[i][0];
        c->occ[prec][jvp][1] = cand[i][1];
        c->fuse_grad[prec][jvp] = cand[i][2] != 0;
        return eval_op(c, prec, jvp == 1, w, w, 0.0, c->d_t3, s) == DG_OK;
      };
      dg_status st = pick_fastest(10, s, launch, &best);
      if (st != DG_OK) {
        c->occ[prec][jvp][0] = c->occ[prec][jvp][1] = 0;
        c->fuse_grad[prec][jvp] = false;
        return st;
      }
      v = {cand[best][0], cand[best][1], cand[best][2]};
      store(k, v);
    }
    c->occ[prec][jvp][0] = v[0];
    c->occ[prec][jvp][1] = v[1];
    c->fuse_grad[prec][jvp] = v[2] != 0;
  }
  c->fine_tuned[prec] = true;
  return DG_OK;
}

dg_status tune_apply(dg_context* c, int storage, const void* Dinv, int m, dgk::ApplyShape* out, hipStream_t s) {
  *out = dgk::ApplyShape{};
  if (c->tune_mode != DG_TUNE_AUTO || capturing(s)) return DG_OK;
  const Key k = {kFamApply, m, storage, 0, 0, c->ne, device_id()};
  std::array<int, 3> v{};
  if (!cached(k, &v)) {
    std::vector<dgk::ApplyShape> cand = {dgk::default_apply_shape(m)};
    if (m <= 64)
      for (int e : {1, 2, 4, 8}) cand.push_back({dgk::kApplyRow, 64, e});
    for (int e : {1, 2, 4}) cand.push_back({dgk::kApplyVec, 64, e});
    for (int t : {128, 256, 512}) cand.push_back({dgk::kApplyVec, t, 1});
    const int64_t n = (int64_t)m * c->ne;  // <= ndof: the level's vector length
    HIPCHK(dgk::launch_fill(c->d_t1, n, 0.5, s));
    int best = 0;
    auto launch = [&](int i) {
      return dgk::launch_block_apply(storage, Dinv, m, c->ne, c->d_t1, c->d_t2, s, &cand[i]) == hipSuccess;
    };
    dg_status st = pick_fastest((int)cand.size(), s, launch, &best);
    if (st != DG_OK) return st;
    v = {cand[best].kind, cand[best].threads, cand[best].epw};
    store(k, v);
  }
  *out = dgk::ApplyShape{v[0], v[1], v[2]};
  return DG_OK;
}

dg_status tune_bsr(dg_context* c, const double* B, const float* B32, int m, dgk::BsrShape* out, hipStream_t s) {
  *out = dgk::BsrShape{};
  if (c->tune_mode != DG_TUNE_AUTO || capturing(s)) return DG_OK;
  const int nf = 2 * c->dim;
  const Key k = {kFamBsr, m, B32 ? 4 : 8, nf, 0, c->ne, device_id()};
  std::array<int, 3> v{};
  if (!cached(k, &v)) {
    std::vector<dgk::BsrShape> cand = {dgk::BsrShape{}};
    for (int bs : {256, 512, 1024})
      for (int rpt : {1, 2, 4})
        for (int cs : {1, 2, 4, 8}) cand.push_back({bs, rpt, cs});
    const int64_t n = (int64_t)m * c->ne;
    HIPCHK(dgk::launch_fill(c->d_t1, n, 0.5, s));
    int best = 0;
    auto launch = [&](int i) {
      const hipError_t e = B32 ? dgk::launch_bsr_apply_f32(cand[i], B32, c->mesh.nbr, nf, m, c->ne, c->d_t1, c->d_t2, s)
                               : dgk::launch_bsr_apply(cand[i], B, c->mesh.nbr, nf, m, c->ne, c->d_t1, c->d_t2, s);
      return e == hipSuccess;
    };
    dg_status st = pick_fastest((int)cand.size(), s, launch, &best);
    if (st != DG_OK) return st;
    v = {cand[best].bs, cand[best].rpt, cand[best].cs};
    store(k, v);
  }
  *out = dgk::BsrShape{v[0], v[1], v[2]};
  return DG_OK;
}

std::string apply_shape_name(const dgk::ApplyShape& sh0, int m) {
  const dgk::ApplyShape sh = sh0.kind ? sh0 : dgk::default_apply_shape(m);
  char b[96];
  if (sh.kind == dgk::kApplyRow)
    std::snprintf(b, sizeof b, "row x%d%s", sh.epw, sh0.kind ? "" : " (default)");
  else
    std::snprintf(b, sizeof b, "vec %dx%d%s", sh.threads, sh.epw, sh0.kind ? "" : " (default)");
  return b;
}

std::string bsr_shape_name(const dgk::BsrShape& sh, int m, bool f32) {
  char b[96];
  const int rpt = sh.rpt ? sh.rpt : dgk::bsr_widest_rpt(m, f32 ? 4 : 8);
  std::snprintf(b, sizeof b, "bsr wg %d, rows/thread %d, column slices %d", sh.bs, rpt, sh.cs);
  return b;
}

}  // namespace dgc

using namespace dgc;

extern "C" {

dg_status dg_set_tuning(dg_context* c, int mode) {
  if (!c) return fail(DG_ERR_ARG, "null context");
  if (mode != DG_TUNE_FIXED && mode != DG_TUNE_AUTO) return fail(DG_ERR_ARG, "unknown tuning mode");
  c->tune_mode = mode;
  for (int p = 0; p < 3; ++p) {
    c->fine_tuned[p] = false;
    for (int j = 0; j < 2; ++j) {
      c->occ[p][j][0] = c->occ[p][j][1] = 0;
      c->fuse_grad[p][j] = false;
    }
  }
  c->blk_shape = dgk::ApplyShape{};
  return mg_recapture(c);  // a captured cycle follows the fine apply shape
}

dg_status dg_set_fine_shape(dg_context* c, int precision, int jvp, int face_occ, int volume_occ,
                            int fused_gradients) {
  if (!c) return fail(DG_ERR_ARG, "null context");
  if (fused_gradients != 0 && fused_gradients != 1) return fail(DG_ERR_ARG, "fused_gradients must be 0 or 1");
  if (precision < DG_FP64 || precision > DG_BF16 || (jvp != 0 && jvp != 1))
    return fail(DG_ERR_ARG, "precision must be DG_FP64/FP32/BF16 and jvp 0 or 1");
  if (!c->use_mfma || c->curved || !has_prec(c, precision))
    return fail(DG_ERR_ARG, "the context has no MFMA operator of this precision");
  if (!dgk::mfma_occ_fits(c->cfg, precision, face_occ, volume_occ))
    return fail(DG_ERR_ARG, "occupancy not available for this configuration");
  c->occ[precision][jvp][0] = face_occ;
  c->occ[precision][jvp][1] = volume_occ;
  c->fuse_grad[precision][jvp] = fused_gradients != 0;
  c->fine_tuned[precision] = true;
  return mg_recapture(c);
}

dg_status dg_set_apply_shape(dg_context* c, int level, int kind, int threads, int epw) {
  if (!c) return fail(DG_ERR_ARG, "null context");
  const dgk::ApplyShape sh{kind, threads, epw};
  if (level == 0) {
    if (!c->blk_ready) return fail(DG_ERR_STATE, "dg_block_precond_setup has not succeeded");
    if (!dgk::apply_shape_fits(sh, c->nv * c->nb, c->blk_storage))
      return fail(DG_ERR_ARG, "block apply shape does not fit the fine blocks");
    c->blk_shape = sh;
    return mg_recapture(c);
  }
  return mg_set_level_shape(c, level, nullptr, &sh);
}

dg_status dg_set_bsr_shape(dg_context* c, int level, int workgroup, int rows_per_thread, int column_slices) {
  if (!c) return fail(DG_ERR_ARG, "null context");
  const dgk::BsrShape sh{workgroup, rows_per_thread, column_slices};
  return mg_set_level_shape(c, level, &sh, nullptr);
}

dg_status dg_autotune(dg_context* c, const double* w, void* stream) {
  if (!c || !w) return fail(DG_ERR_ARG, "null argument");
  if (c->tune_mode != DG_TUNE_AUTO) return DG_OK;
  hipStream_t s = (hipStream_t)stream;
  dg_status st;
  for (int p = DG_FP64; p <= DG_BF16; ++p)
    if (has_prec(c, p) && (st = tune_fine(c, p, w, s)) != DG_OK) return st;
  if (c->blk_ready) {
    dgk::ApplyShape sh;
    if ((st = tune_apply(c, c->blk_storage, c->d_Dinv, c->nv * c->nb, &sh, s)) != DG_OK) return st;
    c->blk_shape = sh;
  }
  HIPCHK(hipStreamSynchronize(s));
  return DG_OK;
}

dg_status dg_tuning_report(const dg_context* c, char* buf, size_t len) {
  if (!c || !buf) return fail(DG_ERR_ARG, "null argument");
  std::string r = std::string("mode ") + (c->tune_mode == DG_TUNE_AUTO ? "auto" : "fixed") + "\n";
  if (c->use_mfma && !c->curved)
    for (int p = DG_FP64; p <= DG_BF16; ++p) {
      if (!has_prec(c, p)) continue;
      for (int j = 0; j < 2; ++j) {
        char b[160];
        auto occ = [](int o) { return o ? std::to_string(o) : std::string("default"); };
        std::snprintf(b, sizeof b, "fine %s %s: face occ %s, volume occ %s, gradients %s%s\n", prec_name(p),
                      j ? "jv" : "residual", occ(c->occ[p][j][0]).c_str(), occ(c->occ[p][j][1]).c_str(),
                      c->fuse_grad[p][j] ? "fused" : "separate", c->fine_tuned[p] ? "" : " (not tuned)");
        r += b;
      }
    }
  if (c->blk_ready) {
    const int m = c->nv * c->nb;
    r += "block apply m=" + std::to_string(m) + " " + prec_name(c->blk_storage) + ": " +
         apply_shape_name(c->blk_shape, m) + "\n";
  }
  if (c->mg) r += mg_tuning_report(c->mg);
  if (r.size() + 1 > len) return fail(DG_ERR_ARG, "report buffer too small: " + std::to_string(r.size() + 1));
  std::memcpy(buf, r.c_str(), r.size() + 1);
  return DG_OK;
}

}  // extern "C"
