// Learned element-local preconditioner: network state, training step and
// application (the flexible outer solver of Sec. 2.5 accepts it because it
// may change from one application to the next).
//
// Network: n_in = n*Nb + 2d*n features -> 256 -> 256 -> n*Nb, ReLU on the
// hidden layers, BF16 weights/activations/deltas, FP32 biases, FP32 MFMA
// accumulation, FP32 master weights with Adam.  Padded shapes: the input
// width to a multiple of 32 (the MFMA k-step), the output width to a
// multiple of 32 for the backward product through W3; padding is zero.
#include <cmath>
#include <string>

#include "context.h"

namespace dgk {
hipError_t launch_mlp_mref(const double* ss, int nv, int64_t ne, double inv_vol, double* mref, hipStream_t s);
hipError_t launch_mlp_features(const double* w, const double* r, const double* z, const int64_t* nbr,
                               const double* mref, int nv, int nb, int nf, int64_t ne, double inv_sqrt_vol, float* X,
                               int ldx, float* T, double* s_out, hipStream_t s);
hipError_t launch_mlp_pack_rows(const float* X, int ldx, int n_in, const int64_t* rows, int64_t B, int64_t Bp,
                                unsigned short* Xb, int ldb, hipStream_t s);
hipError_t launch_gemm_bf16(bool at, bool bt, int epi, int64_t M, int N, int64_t K, const unsigned short* A,
                            int64_t lda, const unsigned short* B, int64_t ldb, void* out, int64_t ldo,
                            const float* bias, const unsigned short* aux, hipStream_t s);
hipError_t launch_mlp_loss(const float* Y, int ldy, const float* T, const int64_t* rows, int n_out, int64_t B,
                           int64_t Bp, unsigned short* dY, int ldd, double* part, int npart, float* loss,
                           hipStream_t s);
hipError_t launch_colsum_bf16(const unsigned short* D, int ldd, int64_t B, int N, float* g, hipStream_t s);
hipError_t launch_adam(int64_t n, float* th, float* m, float* v, const float* g, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s);
hipError_t launch_pack_weight(const float* W, int rows, int cols, unsigned short* Wb, int prow, int pcol,
                              hipStream_t s);
hipError_t launch_pack_bias(const float* b, int n, float* bp, int np, hipStream_t s);
hipError_t launch_mlp_scatter(const float* Y, int ldy, const double* sc, int m, int64_t ne, double* z, int add,
                              hipStream_t s);
}  // namespace dgk

namespace dgc {

namespace {
constexpr int kH = 256;
constexpr int kLossParts = 256;
int64_t up32(int64_t n) { return (n + 31) / 32 * 32; }
}  // namespace

struct MlpState {
  int n_in = 0, n_out = 0, KP = 0, NP = 0;
  int64_t nparam = 0;
  int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  unsigned short *W1b = nullptr, *W2b = nullptr, *W3b = nullptr;
  float *b1p = nullptr, *b2p = nullptr, *b3p = nullptr;
  int64_t step = 0;
  bool ready = false;
  // batch buffers, capacity cap rows (a multiple of 32)
  int64_t cap = 0;
  unsigned short *Xb = nullptr, *a1 = nullptr, *a2 = nullptr, *dY = nullptr, *d2 = nullptr, *d1 = nullptr;
  float* Y = nullptr;
  double* part = nullptr;
  float* loss = nullptr;
  // application buffers (one row per element)
  float* Xf = nullptr;
  double* s = nullptr;
  double* ss = nullptr;
  double* mref = nullptr;
  // DG_MLP_CORRECT_BJ: z = D^-1 r + s_K MLP(x_K), targets (z - D^-1 r)/s_K
  int mode = DG_MLP_DIRECT;
  double* zt = nullptr;  // ndof: z - D^-1 r for the targets
};

void mlp_destroy(MlpState* M) {
  if (!M) return;
  for (void* p : {(void*)M->theta, (void*)M->m, (void*)M->v, (void*)M->grad, (void*)M->W1b, (void*)M->W2b,
                  (void*)M->W3b, (void*)M->b1p, (void*)M->b2p, (void*)M->b3p, (void*)M->Xb, (void*)M->a1,
                  (void*)M->a2, (void*)M->dY, (void*)M->d2, (void*)M->d1, (void*)M->Y, (void*)M->part,
                  (void*)M->loss, (void*)M->Xf, (void*)M->s, (void*)M->ss, (void*)M->mref, (void*)M->zt})
    dfree(p);
  delete M;
}

bool mlp_ready(const MlpState* M) { return M && M->ready; }

namespace {

dg_status mlp_state(dg_context* c, MlpState** out) {
  if (c->mlp) {
    *out = c->mlp;
    return DG_OK;
  }
  auto* M = new MlpState();
  M->n_out = c->nv * c->nb;
  M->n_in = M->n_out + 2 * c->dim * c->nv;
  M->KP = (int)up32(M->n_in);
  M->NP = (int)up32(M->n_out);
  M->oW1 = 0;
  M->ob1 = M->oW1 + (int64_t)kH * M->n_in;
  M->oW2 = M->ob1 + kH;
  M->ob2 = M->oW2 + (int64_t)kH * kH;
  M->oW3 = M->ob2 + kH;
  M->ob3 = M->oW3 + (int64_t)M->n_out * kH;
  M->nparam = M->ob3 + M->n_out;
  dg_status st;
  auto bail = [&](dg_status e) {
    mlp_destroy(M);
    return e;
  };
  if ((st = dalloc(&M->theta, (size_t)M->nparam)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->m, (size_t)M->nparam)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->v, (size_t)M->nparam)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->grad, (size_t)M->nparam)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->W1b, (size_t)kH * M->KP)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->W2b, (size_t)kH * kH)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->W3b, (size_t)M->NP * kH)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->b1p, (size_t)kH)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->b2p, (size_t)kH)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->b3p, (size_t)M->NP)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->part, (size_t)kLossParts)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->loss, (size_t)1)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->ss, (size_t)8)) != DG_OK) return bail(st);
  if ((st = dalloc(&M->mref, (size_t)8)) != DG_OK) return bail(st);
  c->mlp = M;
  *out = M;
  return DG_OK;
}

// Batch buffers with at least Bp rows (Bp a multiple of 32).
dg_status ensure_rows(MlpState* M, int64_t Bp) {
  if (M->cap >= Bp) return DG_OK;
  for (void* p : {(void*)M->Xb, (void*)M->a1, (void*)M->a2, (void*)M->dY, (void*)M->d2, (void*)M->d1, (void*)M->Y})
    dfree(p);
  M->Xb = M->a1 = M->a2 = M->dY = M->d2 = M->d1 = nullptr;
  M->Y = nullptr;
  M->cap = 0;
  dg_status st;
  if ((st = dalloc(&M->Xb, (size_t)Bp * M->KP)) != DG_OK) return st;
  if ((st = dalloc(&M->a1, (size_t)Bp * kH)) != DG_OK) return st;
  if ((st = dalloc(&M->a2, (size_t)Bp * kH)) != DG_OK) return st;
  if ((st = dalloc(&M->dY, (size_t)Bp * M->NP)) != DG_OK) return st;
  if ((st = dalloc(&M->d2, (size_t)Bp * kH)) != DG_OK) return st;
  if ((st = dalloc(&M->d1, (size_t)Bp * kH)) != DG_OK) return st;
  if ((st = dalloc(&M->Y, (size_t)Bp * M->NP)) != DG_OK) return st;
  M->cap = Bp;
  return DG_OK;
}

dg_status pack_weights(MlpState* M, hipStream_t s) {
  HIPCHK(dgk::launch_pack_weight(M->theta + M->oW1, kH, M->n_in, M->W1b, kH, M->KP, s));
  HIPCHK(dgk::launch_pack_weight(M->theta + M->oW2, kH, kH, M->W2b, kH, kH, s));
  HIPCHK(dgk::launch_pack_weight(M->theta + M->oW3, M->n_out, kH, M->W3b, M->NP, kH, s));
  HIPCHK(dgk::launch_pack_bias(M->theta + M->ob1, kH, M->b1p, kH, s));
  HIPCHK(dgk::launch_pack_bias(M->theta + M->ob2, kH, M->b2p, kH, s));
  HIPCHK(dgk::launch_pack_bias(M->theta + M->ob3, M->n_out, M->b3p, M->NP, s));
  return DG_OK;
}

// Zero rows [B, Bp) of a row-major BF16 buffer of width ld (the K = batch
// products read them).
dg_status zero_tail(unsigned short* p, int64_t B, int64_t Bp, int ld, hipStream_t s) {
  if (Bp > B) HIPCHK(hipMemsetAsync(p + B * ld, 0, (size_t)(Bp - B) * ld * sizeof(unsigned short), s));
  return DG_OK;
}

// a1, a2, Y (ldy) from Xb for rows 0..B-1
dg_status forward_rows(MlpState* M, int64_t B, float* Y, int ldy, int ny, hipStream_t s) {
  HIPCHK(dgk::launch_gemm_bf16(false, true, 1, B, kH, M->KP, M->Xb, M->KP, M->W1b, M->KP, M->a1, kH, M->b1p,
                               nullptr, s));
  HIPCHK(dgk::launch_gemm_bf16(false, true, 1, B, kH, kH, M->a1, kH, M->W2b, kH, M->a2, kH, M->b2p, nullptr, s));
  HIPCHK(dgk::launch_gemm_bf16(false, true, 0, B, ny, kH, M->a2, kH, M->W3b, kH, Y, ldy, M->b3p, nullptr, s));
  return DG_OK;
}

// gradient of the mean squared error into M->grad, loss into lossp (device)
dg_status grad_impl(MlpState* M, const float* X, const float* T, const int64_t* rows, int64_t B, float* lossp,
                    hipStream_t s) {
  const int64_t Bp = up32(B);
  dg_status st;
  if ((st = ensure_rows(M, Bp)) != DG_OK) return st;
  HIPCHK(dgk::launch_mlp_pack_rows(X, M->n_in, M->n_in, rows, B, Bp, M->Xb, M->KP, s));
  if ((st = forward_rows(M, B, M->Y, M->NP, M->n_out, s)) != DG_OK) return st;
  if ((st = zero_tail(M->a1, B, Bp, kH, s)) != DG_OK) return st;
  if ((st = zero_tail(M->a2, B, Bp, kH, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_mlp_loss(M->Y, M->NP, T, rows, M->n_out, B, Bp, M->dY, M->NP, M->part, kLossParts, lossp, s));
  // W3, b3
  HIPCHK(dgk::launch_gemm_bf16(true, false, 0, M->n_out, kH, Bp, M->dY, M->NP, M->a2, kH, M->grad + M->oW3, kH,
                               nullptr, nullptr, s));
  HIPCHK(dgk::launch_colsum_bf16(M->dY, M->NP, B, M->n_out, M->grad + M->ob3, s));
  // delta of layer 2 through W3 and the ReLU
  HIPCHK(dgk::launch_gemm_bf16(false, false, 2, B, kH, M->NP, M->dY, M->NP, M->W3b, kH, M->d2, kH, nullptr, M->a2, s));
  if ((st = zero_tail(M->d2, B, Bp, kH, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_gemm_bf16(true, false, 0, kH, kH, Bp, M->d2, kH, M->a1, kH, M->grad + M->oW2, kH, nullptr,
                               nullptr, s));
  HIPCHK(dgk::launch_colsum_bf16(M->d2, kH, B, kH, M->grad + M->ob2, s));
  // delta of layer 1
  HIPCHK(dgk::launch_gemm_bf16(false, false, 2, B, kH, kH, M->d2, kH, M->W2b, kH, M->d1, kH, nullptr, M->a1, s));
  if ((st = zero_tail(M->d1, B, Bp, kH, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_gemm_bf16(true, false, 0, kH, M->n_in, Bp, M->d1, kH, M->Xb, M->KP, M->grad + M->oW1, M->n_in,
                               nullptr, nullptr, s));
  HIPCHK(dgk::launch_colsum_bf16(M->d1, kH, B, kH, M->grad + M->ob1, s));
  return DG_OK;
}

// X rows (ldx) of features for every element at state w, residual r
dg_status features_impl(dg_context* c, MlpState* M, const double* w, const double* r, const double* z, float* X,
                        int ldx, float* T, double* sK, hipStream_t s) {
  if (c->curved) return fail(DG_ERR_ARG, "the learned preconditioner's features need a uniform lattice");
  double vol = 1.0;
  for (int i = 0; i < c->dim; ++i) vol *= c->mesh.h[i];
  for (int v = 0; v < c->nv; ++v) {
    HIPCHK(dgk::launch_dot_partials(w + (int64_t)v * c->nb * c->ne, w + (int64_t)v * c->nb * c->ne, c->ne, c->d_red,
                                    s));
    HIPCHK(dgk::launch_sum_partials(c->d_red, dgk::kRedBlocks, M->ss + v, 0, s));
  }
  HIPCHK(dgk::launch_mlp_mref(M->ss, c->nv, c->ne, 1.0 / vol, M->mref, s));
  if (z && M->mode == DG_MLP_CORRECT_BJ) {  // the targets are the correction to block Jacobi
    if (!c->blk_ready) return fail(DG_ERR_STATE, "the block-Jacobi correction mode needs a block setup");
    dg_status st;
    if ((st = dalloc(&M->zt, (size_t)c->ndof)) != DG_OK) return st;
    HIPCHK(dgk::launch_block_apply(c->blk_storage, c->d_Dinv, c->nv * c->nb, c->ne, r, M->zt, s, &c->blk_shape));
    HIPCHK(dgk::launch_axpby(c->ndof, 1.0, z, -1.0, M->zt, M->zt, s));
    z = M->zt;
  }
  HIPCHK(dgk::launch_mlp_features(w, r, z, c->mesh.nbr, M->mref, c->nv, c->nb, 2 * c->dim, c->ne, 1.0 / std::sqrt(vol),
                                  X, ldx, T, sK, s));
  return DG_OK;
}

}  // namespace

dg_status mlp_apply(dg_context* c, const double* w, const double* r, double* z, hipStream_t s) {
  MlpState* M = c->mlp;
  ProfScope ps(c, "mlp_apply", s);
  const int64_t ne = c->ne, Bp = up32(ne);
  dg_status st;
  if ((st = ensure_rows(M, Bp)) != DG_OK) return st;
  if ((st = dalloc(&M->Xf, (size_t)ne * M->KP)) != DG_OK) return st;
  if ((st = dalloc(&M->s, (size_t)ne)) != DG_OK) return st;
  if ((st = features_impl(c, M, w, r, nullptr, M->Xf, M->KP, nullptr, M->s, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_mlp_pack_rows(M->Xf, M->KP, M->n_in, nullptr, ne, ne, M->Xb, M->KP, s));
  if ((st = forward_rows(M, ne, M->Y, M->NP, M->n_out, s)) != DG_OK) return st;
  const int add = M->mode == DG_MLP_CORRECT_BJ;
  if (add) {
    if (!c->blk_ready) return fail(DG_ERR_STATE, "the block-Jacobi correction mode needs a block setup");
    HIPCHK(dgk::launch_block_apply(c->blk_storage, c->d_Dinv, c->nv * c->nb, ne, r, z, s, &c->blk_shape));
  }
  HIPCHK(dgk::launch_mlp_scatter(M->Y, M->NP, M->s, M->n_out, ne, z, add, s));
  return DG_OK;
}

}  // namespace dgc

using namespace dgc;

extern "C" {

int64_t dg_mlp_nparams(dg_context* c) {
  if (!c) return -1;
  MlpState* M;
  if (mlp_state(c, &M) != DG_OK) return -1;
  return M->nparam;
}

dg_status dg_mlp_set_weights(dg_context* c, const float* theta, void* stream) {
  if (!c || !theta) return fail(DG_ERR_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  MlpState* M;
  dg_status st;
  if ((st = mlp_state(c, &M)) != DG_OK) return st;
  HIPCHK(hipMemcpyAsync(M->theta, theta, (size_t)M->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemsetAsync(M->m, 0, (size_t)M->nparam * sizeof(float), s));
  HIPCHK(hipMemsetAsync(M->v, 0, (size_t)M->nparam * sizeof(float), s));
  M->step = 0;
  if ((st = pack_weights(M, s)) != DG_OK) return st;
  M->ready = true;
  return DG_OK;
}

dg_status dg_mlp_set_mode(dg_context* c, int mode) {
  if (!c) return fail(DG_ERR_ARG, "null argument");
  if (mode != DG_MLP_DIRECT && mode != DG_MLP_CORRECT_BJ) return fail(DG_ERR_ARG, "unknown network mode");
  MlpState* M;
  dg_status st;
  if ((st = mlp_state(c, &M)) != DG_OK) return st;
  M->mode = mode;
  return DG_OK;
}

dg_status dg_mlp_get_weights(dg_context* c, float* theta, void* stream) {
  if (!c || !theta) return fail(DG_ERR_ARG, "null argument");
  if (!mlp_ready(c->mlp)) return fail(DG_ERR_STATE, "network weights not set");
  HIPCHK(hipMemcpyAsync(theta, c->mlp->theta, (size_t)c->mlp->nparam * sizeof(float), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream));
  return DG_OK;
}

dg_status dg_mlp_features(dg_context* c, const double* w, const double* r, const double* z, float* X, float* T,
                          double* scale, void* stream) {
  if (!c || !w || !r || !X) return fail(DG_ERR_ARG, "null argument");
  if (T && !z) return fail(DG_ERR_ARG, "targets need z");
  MlpState* M;
  dg_status st;
  if ((st = mlp_state(c, &M)) != DG_OK) return st;
  return features_impl(c, M, w, r, z, X, M->n_in, T, scale, (hipStream_t)stream);
}

dg_status dg_mlp_forward(dg_context* c, const float* X, int64_t batch, float* Y, void* stream) {
  if (!c || !X || !Y) return fail(DG_ERR_ARG, "null argument");
  if (batch < 1) return fail(DG_ERR_ARG, "batch must be >= 1");
  if (!mlp_ready(c->mlp)) return fail(DG_ERR_STATE, "network weights not set");
  MlpState* M = c->mlp;
  hipStream_t s = (hipStream_t)stream;
  dg_status st;
  if ((st = ensure_rows(M, up32(batch))) != DG_OK) return st;
  HIPCHK(dgk::launch_mlp_pack_rows(X, M->n_in, M->n_in, nullptr, batch, batch, M->Xb, M->KP, s));
  return forward_rows(M, batch, Y, M->n_out, M->n_out, s);
}

dg_status dg_mlp_grad(dg_context* c, const float* X, const float* T, const int64_t* rows, int64_t batch, float* grad,
                      float* loss, void* stream) {
  if (!c || !X || !T || !grad) return fail(DG_ERR_ARG, "null argument");
  if (batch < 1) return fail(DG_ERR_ARG, "batch must be >= 1");
  if (!mlp_ready(c->mlp)) return fail(DG_ERR_STATE, "network weights not set");
  MlpState* M = c->mlp;
  hipStream_t s = (hipStream_t)stream;
  dg_status st;
  if ((st = grad_impl(M, X, T, rows, batch, loss ? loss : M->loss, s)) != DG_OK) return st;
  HIPCHK(hipMemcpyAsync(grad, M->grad, (size_t)M->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
  return DG_OK;
}

dg_status dg_mlp_train_step(dg_context* c, const float* X, const float* T, const int64_t* rows, int64_t batch,
                            float lr, float* loss, void* stream) {
  if (!c || !X || !T) return fail(DG_ERR_ARG, "null argument");
  if (batch < 1 || !(lr > 0.0f)) return fail(DG_ERR_ARG, "need batch >= 1 and lr > 0");
  if (!mlp_ready(c->mlp)) return fail(DG_ERR_STATE, "network weights not set");
  MlpState* M = c->mlp;
  hipStream_t s = (hipStream_t)stream;
  dg_status st;
  if ((st = grad_impl(M, X, T, rows, batch, loss ? loss : M->loss, s)) != DG_OK) return st;
  M->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)M->step));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)M->step));
  HIPCHK(dgk::launch_adam(M->nparam, M->theta, M->m, M->v, M->grad, lr, b1, b2, 1e-8f, c1, c2, s));
  return pack_weights(M, s);
}

dg_status dg_mlp_apply(dg_context* c, const double* w, const double* r, double* z, void* stream) {
  if (!c || !w || !r || !z) return fail(DG_ERR_ARG, "null argument");
  if (r == z || w == z) return fail(DG_ERR_ARG, "z may not alias w or r");
  if (!mlp_ready(c->mlp)) return fail(DG_ERR_STATE, "network weights not set");
  return mlp_apply(c, w, r, z, (hipStream_t)stream);
}

}  // extern "C"
