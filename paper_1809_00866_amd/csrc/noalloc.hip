// Allocation-free exact Jacobian-vector product.
//
// dg_jvp (exact mode) keeps its intermediate arrays -- the modal corrected
// gradients and the face fluxes (affine lattices), or the transformed
// coefficients, face jumps and face fluxes (curved meshes) -- in buffers the
// context allocated at dg_create.  dg_jvp_noalloc runs the same kernels with
// those arrays placed in one file-scope device array instead, so a call
// allocates nothing, for callers that cannot allocate device memory.
//
// The array is a module global: every GPU the library runs on holds its own
// copy (kScratchBytes) from the load of the library until the process ends,
// at an address that is fixed per device.  In host code the array's name is
// only a host-side stand-in, so its device address is looked up once per
// device with hipGetSymbolAddress (from dg_create, with the context's device
// current) and only that address is passed to kernels.  Every call on one
// GPU shares the array: calls that overlap on one GPU (different streams,
// different threads, different contexts) race and must be serialised by the
// caller.  Nothing needs clearing between calls: the kernels write every
// scratch entry they read before reading it.
#include <mutex>

#include "context.h"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // per GPU
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
constexpr size_t kAlignDoubles = 32;                 // sub-buffers start on 256-byte boundaries
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t round_up(size_t n) { return (n + kAlignDoubles - 1) / kAlignDoubles * kAlignDoubles; }

}  // namespace

namespace dgc {

dg_status noalloc_scratch_address(void** out) {
  *out = nullptr;
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_ERR_ARG, "device index out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(DG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

}  // namespace dgc

using namespace dgc;

extern "C" {

size_t dg_jvp_noalloc_scratch_bytes(void) { return kScratchBytes; }

dg_status dg_jvp_noalloc(dg_context* c, const double* w, const double* v, double shift, double* out,
                         void* stream) {
  if (!c || !w || !v || !out) return fail(DG_ERR_ARG, "null argument");
  if (out == w || out == v) return fail(DG_ERR_ARG, "out may not alias w or v");
  if (!c->d_scratch) return fail(DG_ERR_STATE, "the context has no scratch address");
  const hipStream_t s = (hipStream_t)stream;
  double* S = static_cast<double*>(c->d_scratch);
  const size_t ne = (size_t)c->ne;
  const size_t nfp = (size_t)c->dim * c->nv * c->nfq * ne;  // face points x variables over all faces
  auto too_big = [&](size_t need) {
    return fail(DG_ERR_ARG, "dg_jvp_noalloc needs " + std::to_string(need * sizeof(double)) +
                                " bytes of scratch; the static scratch holds " + std::to_string(kScratchBytes));
  };
  if (c->curved) {
    const size_t nx = ne * c->nv * c->nb;
    const size_t o1 = round_up(nx), o2 = o1 + round_up(nx), o3 = o2 + round_up(2 * nfp);
    const size_t need = o3 + round_up(nfp);
    if (need > kScratchDoubles) return too_big(need);
    dgk::CurvedTables ct = c->ct;
    ct.Ut = S;
    ct.Vt = S + o1;
    ct.fJmp = S + o2;
    ct.fHn = S + o3;
    HIPCHK(dgk::launch_modal_curved(c->cfg, true, w, v, ct, c->ne, s));
    HIPCHK(dgk::launch_face_curved(c->cfg, true, ct, c->mesh, c->ph, s));
    HIPCHK(dgk::launch_volume_curved(c->cfg, true, v, ct, out, shift, c->mesh, c->ph, s));
    return DG_OK;
  }
  if (c->use_mfma) {
    const size_t nG = (size_t)2 * c->dim * c->nv * c->nb * ne;
    const size_t oH = round_up(nG);
    const size_t need = oH + round_up(nfp);
    if (need > kScratchDoubles) return too_big(need);
    double* G = S;
    double* H = S + oH;
    HIPCHK(dgk::launch_grad_mfma(c->cfg, true, w, v, G, c->mt, c->mesh, s));
    HIPCHK(dgk::launch_face_mfma(c->cfg, true, w, v, H, c->mt, c->mesh, c->ph, c->occ[DG_FP64][1][0], s));
    HIPCHK(dgk::launch_volume_mfma(c->cfg, true, w, v, G, H, out, shift, c->mt, c->mesh, c->ph,
                                   c->occ[DG_FP64][1][1], false, s));
    return DG_OK;
  }
  const size_t need = round_up(nfp);
  if (need > kScratchDoubles) return too_big(need);
  HIPCHK(dgk::launch_face(c->cfg, true, w, v, S, c->tb, c->mesh, c->ph, s));
  HIPCHK(dgk::launch_volume(c->cfg, true, w, v, S, out, shift, c->tb, c->mesh, c->ph, s));
  return DG_OK;
}

}  // extern "C"
