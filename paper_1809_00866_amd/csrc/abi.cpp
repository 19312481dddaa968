// extern "C" entry points of the DG library: context management, residual,
// Jacobian-vector products, element block-Jacobi preconditioner and the
// flexible GMRES driver.  Every entry point validates its arguments on the
// host and enqueues HIP kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "context.h"

namespace dgc {

thread_local std::string g_err;

dg_status fail(dg_status s, const std::string& m) {
  g_err = m;
  return s;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

dg_status eval_residual(dg_context* c, bool jvp, const double* w, const double* v, double shift, double* out,
                        hipStream_t s) {
  if (c->curved) {
    {
      ProfScope ps(c, jvp ? "grad_jvp" : "grad_res", s);
      HIPCHK(dgk::launch_modal_curved(c->cfg, jvp, w, v, c->ct, c->ne, s));
    }
    {
      ProfScope ps(c, jvp ? "face_jvp" : "face_res", s);
      HIPCHK(dgk::launch_face_curved(c->cfg, jvp, c->ct, c->mesh, c->ph, s));
    }
    {
      ProfScope ps(c, jvp ? "vol_jvp" : "vol_res", s);
      HIPCHK(dgk::launch_volume_curved(c->cfg, jvp, v, c->ct, out, shift, c->mesh, c->ph, s));
    }
    return DG_OK;
  }
  if (c->use_mfma) {
    const bool fg = c->fuse_grad[DG_FP64][jvp];
    if (!fg) {
      ProfScope ps(c, jvp ? "grad_jvp" : "grad_res", s);
      HIPCHK(dgk::launch_grad_mfma(c->cfg, jvp, w, v, c->d_G, c->mt, c->mesh, s));
    }
    {
      ProfScope ps(c, jvp ? "face_jvp" : "face_res", s);
      HIPCHK(dgk::launch_face_mfma(c->cfg, jvp, w, v, c->d_H, c->mt, c->mesh, c->ph, c->occ[DG_FP64][jvp][0], s));
    }
    {
      ProfScope ps(c, jvp ? "vol_jvp" : "vol_res", s);
      HIPCHK(dgk::launch_volume_mfma(c->cfg, jvp, w, v, c->d_G, c->d_H, out, shift, c->mt, c->mesh, c->ph,
                                     c->occ[DG_FP64][jvp][1], fg, s));
    }
    return DG_OK;
  }
  {
    ProfScope ps(c, jvp ? "face_jvp" : "face_res", s);
    HIPCHK(dgk::launch_face(c->cfg, jvp, w, v, c->d_H, c->tb, c->mesh, c->ph, s));
  }
  {
    ProfScope ps(c, jvp ? "vol_jvp" : "vol_res", s);
    HIPCHK(dgk::launch_volume(c->cfg, jvp, w, v, c->d_H, out, shift, c->tb, c->mesh, c->ph, s));
  }
  return DG_OK;
}

dg_status eval_residual_f32(dg_context* c, bool jvp, const double* w, const double* v, double shift, double* out,
                            hipStream_t s) {
  if (!has_f32(c))
    return fail(DG_ERR_ARG, "the reduced-precision operator needs a curved mesh or a 3D P2-P4 lattice configuration");
  if (c->curved) {
    {
      ProfScope ps(c, jvp ? "grad_jvp_f32" : "grad_res_f32", s);
      HIPCHK(dgk::launch_modal_curved_f32(c->cfg, jvp, w, v, c->ctf, c->ne, s));
    }
    {
      ProfScope ps(c, jvp ? "face_jvp_f32" : "face_res_f32", s);
      HIPCHK(dgk::launch_face_curved_f32(c->cfg, jvp, c->ctf, c->mesh, c->ph, s));
    }
    {
      ProfScope ps(c, jvp ? "vol_jvp_f32" : "vol_res_f32", s);
      HIPCHK(dgk::launch_volume_curved_f32(c->cfg, jvp, v, c->ctf, out, shift, c->mesh, c->ph, s));
    }
    return DG_OK;
  }
  const bool fg = c->fuse_grad[DG_FP32][jvp];
  if (!fg) {
    ProfScope ps(c, jvp ? "grad_jvp_f32" : "grad_res_f32", s);
    HIPCHK(dgk::launch_grad_mfma_f32(c->cfg, jvp, w, v, c->d_Gf, c->mtf, c->mesh, s));
  }
  {
    ProfScope ps(c, jvp ? "face_jvp_f32" : "face_res_f32", s);
    HIPCHK(dgk::launch_face_mfma_f32(c->cfg, jvp, w, v, c->d_Hf, c->mtf, c->mesh, c->ph, c->occ[DG_FP32][jvp][0], s));
  }
  {
    ProfScope ps(c, jvp ? "vol_jvp_f32" : "vol_res_f32", s);
    HIPCHK(dgk::launch_volume_mfma_f32(c->cfg, jvp, w, v, c->d_Gf, c->d_Hf, out, shift, c->mtf, c->mesh, c->ph,
                                       c->occ[DG_FP32][jvp][1], fg, s));
  }
  return DG_OK;
}

dg_status eval_residual_bf16(dg_context* c, bool jvp, const double* w, const double* v, double shift, double* out,
                             hipStream_t s) {
  const bool fg = c->fuse_grad[DG_BF16][jvp];
  if (!fg) {
    ProfScope ps(c, jvp ? "grad_jvp_bf16" : "grad_res_bf16", s);
    HIPCHK(dgk::launch_grad_mfma_bf16(c->cfg, jvp, w, v, c->d_Gf, c->mtf, c->mesh, s));
  }
  {
    ProfScope ps(c, jvp ? "face_jvp_bf16" : "face_res_bf16", s);
    HIPCHK(dgk::launch_face_mfma_bf16(c->cfg, jvp, w, v, c->d_Hf, c->mtf, c->mesh, c->ph, c->occ[DG_BF16][jvp][0], s));
  }
  {
    ProfScope ps(c, jvp ? "vol_jvp_bf16" : "vol_res_bf16", s);
    HIPCHK(dgk::launch_volume_mfma_bf16(c->cfg, jvp, w, v, c->d_Gf, c->d_Hf, out, shift, c->mtf, c->mesh, c->ph,
                                        c->occ[DG_BF16][jvp][1], fg, s));
  }
  return DG_OK;
}

dg_status eval_op(dg_context* c, int prec, bool jvp, const double* w, const double* v, double shift, double* out,
                  hipStream_t s) {
  if (prec == DG_FP64) return eval_residual(c, jvp, w, v, shift, out, s);
  if (prec == DG_FP32) return eval_residual_f32(c, jvp, w, v, shift, out, s);
  if (prec != DG_BF16) return fail(DG_ERR_ARG, "unknown operator precision");
  if (!has_prec(c, DG_BF16))
    return fail(DG_ERR_ARG, "the BF16-contraction operator needs a 3D P2-P4 lattice configuration (MFMA kernels)");
  return eval_residual_bf16(c, jvp, w, v, shift, out, s);
}

// c->d_zero: ndof zeros, allocated and cleared on first use (never written after)
static dg_status zeros(dg_context* c, hipStream_t s) {
  if (c->d_zero) return DG_OK;
  dg_status st;
  if ((st = dalloc(&c->d_zero, (size_t)c->ndof)) != DG_OK) return st;
  HIPCHK(dgk::launch_fill(c->d_zero, c->ndof, 0.0, s));
  return DG_OK;
}

dg_status eval_local(dg_context* c, int prec, const double* w, const double* v, double shift, double* out,
                     hipStream_t s) {
  if (!local_probe_ok(c, prec)) return fail(DG_ERR_ARG, "no element-local probing for this operator");
  dg_status st;
  if ((st = zeros(c, s)) != DG_OK) return st;
  const double* z = c->d_zero;
  // face fluxes of the owners' tangents (read on the +p faces) and of the
  // +p neighbours' tangents (read on the -p faces); gradients without the
  // neighbours' tangents
  if (c->curved) {
    // the same with the curved kernels: the second face pass reads the
    // owner's tangent as zero and writes the jump and flux records that the
    // volume kernel reads on the -p faces
    const size_t nfp = (size_t)c->dim * c->ne * c->nv * c->nfq;
    auto run = [&](auto ct, auto* loc, auto modal, auto face, auto volume, const char* sfx) -> dg_status {
      using R = std::remove_cv_t<std::remove_pointer_t<decltype(loc)>>;
      const R* zr = reinterpret_cast<const R*>(z);  // all-zero bits: +0 in either precision
      auto own = ct, nbr = ct, vol = ct;
      own.VtN = zr;
      nbr.Vt = const_cast<R*>(zr);  // read only by the face kernel
      nbr.VtN = ct.Vt;
      nbr.fJmp = loc;
      nbr.fHn = loc + 2 * nfp;
      vol.fJmpN = nbr.fJmp;
      vol.fHnN = nbr.fHn;
      const std::string g = std::string("grad_probe") + sfx, f = std::string("face_probe") + sfx,
                        v2 = std::string("vol_probe") + sfx;
      {
        ProfScope ps(c, g.c_str(), s);
        HIPCHK(modal(c->cfg, true, w, v, ct, c->ne, s));
      }
      {
        ProfScope ps(c, f.c_str(), s);
        HIPCHK(face(c->cfg, true, own, c->mesh, c->ph, s));
        HIPCHK(face(c->cfg, true, nbr, c->mesh, c->ph, s));
      }
      ProfScope ps(c, v2.c_str(), s);
      HIPCHK(volume(c->cfg, true, v, vol, out, shift, c->mesh, c->ph, s));
      return DG_OK;
    };
    if (prec == DG_FP64) {
      if (!c->d_cloc && (st = dalloc(&c->d_cloc, 3 * nfp)) != DG_OK) return st;
      return run(c->ct, c->d_cloc, dgk::launch_modal_curved, dgk::launch_face_curved, dgk::launch_volume_curved, "");
    }
    if (!c->d_cloc_f && (st = dalloc(&c->d_cloc_f, 3 * nfp)) != DG_OK) return st;
    return run(c->ctf, c->d_cloc_f, dgk::launch_modal_curved_f32, dgk::launch_face_curved_f32,
               dgk::launch_volume_curved_f32, "_f32");
  }
  if (prec == DG_FP64) {
    if (!c->d_H2 && (st = dalloc(&c->d_H2, (size_t)c->dim * c->nv * c->nfq * c->ne)) != DG_OK) return st;
    const bool fg = c->fuse_grad[DG_FP64][1];
    const int* occ = c->occ[DG_FP64][1];
    if (!fg) {
      ProfScope ps(c, "grad_probe", s);
      HIPCHK(dgk::launch_grad_mfma(c->cfg, true, w, v, c->d_G, c->mt, c->mesh, s, z));
    }
    {
      ProfScope ps(c, "face_probe", s);
      HIPCHK(dgk::launch_face_mfma(c->cfg, true, w, v, c->d_H, c->mt, c->mesh, c->ph, occ[0], s, z));
      HIPCHK(dgk::launch_face_mfma(c->cfg, true, w, z, c->d_H2, c->mt, c->mesh, c->ph, occ[0], s, v));
    }
    ProfScope ps(c, "vol_probe", s);
    HIPCHK(dgk::launch_volume_mfma(c->cfg, true, w, v, c->d_G, c->d_H, out, shift, c->mt, c->mesh, c->ph, occ[1], fg,
                                   s, c->d_H2, z));
    return DG_OK;
  }
  if (!c->d_Hf2 && (st = dalloc(&c->d_Hf2, (size_t)c->dim * c->nv * c->nfq * c->ne)) != DG_OK) return st;
  const bool f32 = prec == DG_FP32, fg = c->fuse_grad[prec][1];
  const int* occ = c->occ[prec][1];
  const auto grad = f32 ? dgk::launch_grad_mfma_f32 : dgk::launch_grad_mfma_bf16;
  const auto face = f32 ? dgk::launch_face_mfma_f32 : dgk::launch_face_mfma_bf16;
  const auto vol = f32 ? dgk::launch_volume_mfma_f32 : dgk::launch_volume_mfma_bf16;
  if (!fg) {
    ProfScope ps(c, f32 ? "grad_probe_f32" : "grad_probe_bf16", s);
    HIPCHK(grad(c->cfg, true, w, v, c->d_Gf, c->mtf, c->mesh, s, z));
  }
  {
    ProfScope ps(c, f32 ? "face_probe_f32" : "face_probe_bf16", s);
    HIPCHK(face(c->cfg, true, w, v, c->d_Hf, c->mtf, c->mesh, c->ph, occ[0], s, z));
    HIPCHK(face(c->cfg, true, w, z, c->d_Hf2, c->mtf, c->mesh, c->ph, occ[0], s, v));
  }
  ProfScope ps(c, f32 ? "vol_probe_f32" : "vol_probe_bf16", s);
  HIPCHK(vol(c->cfg, true, w, v, c->d_Gf, c->d_Hf, out, shift, c->mtf, c->mesh, c->ph, occ[1], fg, s, c->d_Hf2, z));
  return DG_OK;
}

dg_status eval_stab(dg_context* c, bool f32, const double* w, const double* v, double* out, hipStream_t s) {
  dg_status st;
  if ((st = zeros(c, s)) != DG_OK) return st;
  dgk::Phys ph = c->ph;
  ph.stab_only = 1;
  const double* z = c->d_zero;  // no tangent in the volume terms and the gradients
  if (c->curved) {
    if (f32) {
      if (!has_f32(c))
        return fail(DG_ERR_ARG, "the reduced-precision operator needs a curved mesh or a 3D P2-P4 lattice configuration");
      HIPCHK(dgk::launch_modal_curved_f32(c->cfg, true, w, v, c->ctf, c->ne, s));
      HIPCHK(dgk::launch_face_curved_f32(c->cfg, true, c->ctf, c->mesh, ph, s));
      HIPCHK(dgk::launch_volume_curved_f32(c->cfg, true, z, c->ctf, out, 0.0, c->mesh, ph, s));
      return DG_OK;
    }
    HIPCHK(dgk::launch_modal_curved(c->cfg, true, w, v, c->ct, c->ne, s));
    HIPCHK(dgk::launch_face_curved(c->cfg, true, c->ct, c->mesh, ph, s));
    HIPCHK(dgk::launch_volume_curved(c->cfg, true, z, c->ct, out, 0.0, c->mesh, ph, s));
    return DG_OK;
  }
  if (f32) {
    if (!c->use_mfma || !c->d_mtab_f || !c->d_Hf || !c->d_Gf)
      return fail(DG_ERR_ARG, "the reduced-precision operator needs a 3D P2-P4 configuration with MFMA kernels");
    HIPCHK(dgk::launch_grad_mfma_f32(c->cfg, true, w, z, c->d_Gf, c->mtf, c->mesh, s));
    HIPCHK(dgk::launch_face_mfma_f32(c->cfg, true, w, v, c->d_Hf, c->mtf, c->mesh, ph, c->occ[DG_FP32][1][0], s));
    HIPCHK(dgk::launch_volume_mfma_f32(c->cfg, true, w, z, c->d_Gf, c->d_Hf, out, 0.0, c->mtf, c->mesh, c->ph,
                                       c->occ[DG_FP32][1][1], false, s));
    return DG_OK;
  }
  if (c->use_mfma) {
    HIPCHK(dgk::launch_grad_mfma(c->cfg, true, w, z, c->d_G, c->mt, c->mesh, s));
    HIPCHK(dgk::launch_face_mfma(c->cfg, true, w, v, c->d_H, c->mt, c->mesh, ph, c->occ[DG_FP64][1][0], s));
    HIPCHK(dgk::launch_volume_mfma(c->cfg, true, w, z, c->d_G, c->d_H, out, 0.0, c->mt, c->mesh, c->ph,
                                   c->occ[DG_FP64][1][1], false, s));
    return DG_OK;
  }
  HIPCHK(dgk::launch_face(c->cfg, true, w, v, c->d_H, c->tb, c->mesh, ph, s));
  HIPCHK(dgk::launch_volume(c->cfg, true, w, z, c->d_H, out, 0.0, c->tb, c->mesh, c->ph, s));
  return DG_OK;
}

dg_status norm2(dg_context* c, const double* x, double* dout, hipStream_t s) {
  HIPCHK(dgk::launch_dot_partials(x, x, c->ndof, c->d_red, s));
  HIPCHK(dgk::launch_sum_partials(c->d_red, dgk::kRedBlocks, dout, 1, s));
  return DG_OK;
}

dg_status jvp_impl(dg_context* c, const double* w, const double* r_w, const double* v, double shift, int mode,
                   double* out, hipStream_t s) {
  if (mode == DG_JVP_EXACT) return eval_residual(c, true, w, v, shift, out, s);
  if (mode == DG_JVP_EXACT_FP32) return eval_residual_f32(c, true, w, v, shift, out, s);
  if (mode == DG_JVP_EXACT_BF16) return eval_op(c, DG_BF16, true, w, v, shift, out, s);
  if (mode == DG_JVP_STAB) {
    dg_status st;
    if ((st = eval_stab(c, false, w, v, out, s)) != DG_OK) return st;
    if (shift != 0.0) HIPCHK(dgk::launch_axpby(c->mass_len, 1.0, out, shift, v, out, s));
    return DG_OK;
  }
  // finite difference of eqs. (matrix-free)/(epsdef)
  const double* r0 = r_w;
  dg_status st;
  if (!r0) {
    if ((st = eval_residual(c, false, w, nullptr, 0.0, c->d_t1, s)) != DG_OK) return st;
    r0 = c->d_t1;
  }
  if ((st = norm2(c, w, c->d_scal + 0, s)) != DG_OK) return st;
  if ((st = norm2(c, v, c->d_scal + 1, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_fd_delta(c->d_scal, 1e-9, s));
  HIPCHK(dgk::launch_axpy_dev(c->ndof, w, c->d_scal + 2, 1.0, v, c->d_t2, s));
  if ((st = eval_residual(c, false, c->d_t2, nullptr, 0.0, c->d_t3, s)) != DG_OK) return st;
  HIPCHK(dgk::launch_fd_combine(c->ndof, c->mass_len, c->d_t3, r0, c->d_scal + 3, v, shift, out, s));
  return DG_OK;
}

}  // namespace dgc

using namespace dgc;

extern "C" {

const char* dg_last_error(void) { return g_err.c_str(); }

dg_status dg_create(const dg_params* prm, const dg_mesh* mesh, dg_context** out) {
  if (!prm || !mesh || !out) return fail(DG_ERR_ARG, "null argument");
  *out = nullptr;
  const int dim = prm->dim;
  if (dim != 2 && dim != 3) return fail(DG_ERR_ARG, "dim must be 2 or 3");
  if (prm->order < 0 || prm->nq1d < 1) return fail(DG_ERR_ARG, "order must be >= 0 and nq1d >= 1");
  if (prm->basis != DG_BASIS_PK && prm->basis != DG_BASIS_QK) return fail(DG_ERR_ARG, "unknown basis");
  if (prm->flux != DG_FLUX_LF && prm->flux != DG_FLUX_ROE) return fail(DG_ERR_ARG, "unknown flux");
  if (prm->physics != DG_PHYS_COMPRESSIBLE && prm->physics != DG_PHYS_INCOMPRESSIBLE &&
      prm->physics != DG_PHYS_DIFFUSION)
    return fail(DG_ERR_ARG, "unknown physics");
  const bool ins = prm->physics == DG_PHYS_INCOMPRESSIBLE;
  const bool diffusion = prm->physics == DG_PHYS_DIFFUSION;
  const bool compressible = !ins && !diffusion;
  if (compressible && (!(prm->gamma > 1.0) || !(prm->prandtl > 0.0)))
    return fail(DG_ERR_ARG, "need gamma > 1, prandtl > 0");
  if (!(prm->mu >= 0.0)) return fail(DG_ERR_ARG, "need mu >= 0");
  const int64_t ne = mesh->n_elem;
  if (ne < 1 || !mesh->elem_xyz || !mesh->elem_nbr) return fail(DG_ERR_ARG, "empty mesh");
  if (ne > (int64_t)1 << 31) return fail(DG_ERR_ARG, "too many elements");
  const int nvtx = 1 << dim;
  // uniform axis-aligned lattice check
  double h[3] = {1.0, 1.0, 1.0};
  for (int i = 0; i < dim; ++i) h[i] = mesh->elem_xyz[(size_t)(1 << i) * dim + i] - mesh->elem_xyz[i];
  for (int i = 0; i < dim; ++i)
    if (!(h[i] > 0.0)) return fail(DG_ERR_ARG, "element 0 is not an axis-aligned box with positive edges");
  // a uniform axis-aligned lattice takes the affine (MFMA / table) kernels;
  // any other mesh of multilinear elements takes the curved-element kernels
  bool lattice = true;
  for (int64_t e = 0; e < ne && lattice; ++e) {
    const double* X = mesh->elem_xyz + (size_t)e * nvtx * dim;
    for (int v = 0; v < nvtx && lattice; ++v)
      for (int i = 0; i < dim; ++i) {
        const double expect = X[i] + (((v >> i) & 1) ? h[i] : 0.0);
        if (std::fabs(X[(size_t)v * dim + i] - expect) > 1e-10 * h[i]) lattice = false;
      }
  }
  for (int64_t e = 0; e < ne; ++e)
    for (int p = 0; p < dim; ++p) {
      const int64_t a = mesh->elem_nbr[e * 2 * dim + 2 * p], b = mesh->elem_nbr[e * 2 * dim + 2 * p + 1];
      if (a < 0 || a >= ne || b < 0 || b >= ne) return fail(DG_ERR_ARG, "neighbour index out of range");
      if (mesh->elem_nbr[b * 2 * dim + 2 * p] != e)
        return fail(DG_ERR_ARG, "inconsistent neighbour table at element " + std::to_string(e));
    }

  dgh::HostTables T;
  try {
    T = dgh::build_tables(dim, prm->order, prm->basis, prm->nq1d, h);
  } catch (const std::exception& ex) {
    return fail(DG_ERR_ARG, ex.what());
  }
  if (ins && !lattice) return fail(DG_ERR_ARG, "the incompressible equations run on uniform lattices only");
  dgh::CurvedHost CH;  // curved (non-lattice) meshes: built before any device work
  if (!lattice) {
    try {
      CH = dgh::build_curved_tables(T, prm->order, mesh->elem_xyz, mesh->elem_nbr, ne);
    } catch (const std::exception& ex) {
      return fail(DG_ERR_ARG, ex.what());
    }
  }
  const int cfg = dgk::config_index(dim, T.nb, prm->nq1d);
  if (cfg < 0 || (!lattice && !dgk::has_curved(cfg, diffusion)))
    return fail(DG_ERR_ARG, std::string("no ") + (lattice ? "" : "curved-element ") + "kernel compiled for dim=" +
                                std::to_string(dim) + " nbasis=" + std::to_string(T.nb) +
                                " nq1d=" + std::to_string(prm->nq1d));

  auto* c = new dg_context();
  c->prm = *prm;
  c->dim = dim;
  c->nv = ins ? dim + 1 : (diffusion ? 1 : dim + 2);
  c->nmass = ins ? dim : c->nv;
  c->nb = T.nb;
  c->nq1 = prm->nq1d;
  c->nq = T.nq;
  c->nfq = T.nfq;
  c->cfg = cfg;
  c->ne = ne;
  c->ndof = ne * c->nv * c->nb;
  c->mass_len = ne * c->nmass * c->nb;
  c->ph.gamma = prm->gamma;
  c->ph.prandtl = prm->prandtl;
  c->ph.mu = prm->mu;
  c->ph.eta = prm->eta_br2 > 0.0 ? prm->eta_br2 : 2.0 * dim + 1.0;
  c->ph.efix = prm->entropy_fix > 0.0 ? prm->entropy_fix : 0.1;
  c->ph.flux = prm->flux;
  c->ph.model = prm->physics;
  c->ph.beta = prm->ac_beta > 0.0 ? prm->ac_beta : 1.0;

  auto cleanup = [&](dg_status st) {
    dg_destroy(c);
    return st;
  };

  // packed tables
  std::vector<const std::vector<double>*> parts = {&T.vPhi, &T.vWD, &T.vWPhi, &T.vLift, &T.fPhi,
                                                   &T.fDphi, &T.fLift, &T.fWPhi, &T.vXi};
  size_t tot = 0;
  for (auto* v : parts) tot += v->size();
  dg_status st;
  if ((st = dalloc(&c->d_tab, tot)) != DG_OK) return cleanup(st);
  std::vector<double> packed;
  packed.reserve(tot);
  std::vector<size_t> off;
  for (auto* v : parts) {
    off.push_back(packed.size());
    packed.insert(packed.end(), v->begin(), v->end());
  }
  if (hipMemcpy(c->d_tab, packed.data(), tot * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(DG_ERR_HIP, "table upload failed"));
  c->tb.vPhi = c->d_tab + off[0];
  c->tb.vWD = c->d_tab + off[1];
  c->tb.vWPhi = c->d_tab + off[2];
  c->tb.vLift = c->d_tab + off[3];
  c->tb.fPhi = c->d_tab + off[4];
  c->tb.fDphi = c->d_tab + off[5];
  c->tb.fLift = c->d_tab + off[6];
  c->tb.fWPhi = c->d_tab + off[7];
  c->tb.vXi = c->d_tab + off[8];

  // curved elements: per-element and per-face tables, face outputs
  if (!lattice) {
    std::vector<const std::vector<double>*> cp = {&CH.rPsiT, &CH.rDPsiT, &CH.rDPsi, &CH.rFPsiT, &CH.rFDPsiT,
                                                  &CH.rFPsi,  &CH.Linv,   &CH.vGeo,  &CH.fGeo,   &CH.fP,
                                                  &CH.vX};
    size_t ctot = 0;
    for (auto* v : cp) ctot += v->size();
    if ((st = dalloc(&c->d_curved, ctot)) != DG_OK) return cleanup(st);
    size_t o = 0;
    std::vector<double*> dst;
    for (auto* v : cp) {
      dst.push_back(c->d_curved + o);
      if (hipMemcpy(c->d_curved + o, v->data(), v->size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(DG_ERR_HIP, "curved table upload failed"));
      o += v->size();
    }
    c->ct.rPsiT = dst[0];
    c->ct.rDPsiT = dst[1];
    c->ct.rDPsi = dst[2];
    c->ct.rFPsiT = dst[3];
    c->ct.rFDPsiT = dst[4];
    c->ct.rFPsi = dst[5];
    c->ct.Linv = dst[6];
    c->ct.vGeo = dst[7];
    c->ct.fGeo = dst[8];
    c->ct.fP = dst[9];
    c->d_cvX = dst[10];
    // work buffers: Ut, Vt, face jumps (value, tangent), face fluxes
    const size_t nx = (size_t)ne * c->nv * T.nb, nfp = (size_t)dim * ne * c->nv * T.nfq;
    if ((st = dalloc(&c->d_cwork, 2 * nx + 3 * nfp)) != DG_OK) return cleanup(st);
    c->ct.Ut = c->d_cwork;
    c->ct.Vt = c->d_cwork + nx;
    c->ct.fJmp = c->d_cwork + 2 * nx;
    c->ct.fHn = c->d_cwork + 2 * nx + 2 * nfp;
    {  // FP32 copies of the tables and FP32 work buffers: the reduced-precision operator
      const size_t ftot = ctot - CH.vX.size();
      std::vector<float> fl(ftot);
      size_t q = 0;
      for (size_t k = 0; k + 1 < cp.size(); ++k)
        for (double x : *cp[k]) fl[q++] = (float)x;
      if ((st = dalloc(&c->d_curved_f, ftot)) != DG_OK) return cleanup(st);
      if (hipMemcpy(c->d_curved_f, fl.data(), ftot * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(DG_ERR_HIP, "curved table upload failed"));
      const float* fp[10];
      size_t of = 0;
      for (int k = 0; k < 10; ++k) {
        fp[k] = c->d_curved_f + of;
        of += cp[k]->size();
      }
      c->ctf.rPsiT = fp[0];
      c->ctf.rDPsiT = fp[1];
      c->ctf.rDPsi = fp[2];
      c->ctf.rFPsiT = fp[3];
      c->ctf.rFDPsiT = fp[4];
      c->ctf.rFPsi = fp[5];
      c->ctf.Linv = fp[6];
      c->ctf.vGeo = fp[7];
      c->ctf.fGeo = fp[8];
      c->ctf.fP = fp[9];
      if ((st = dalloc(&c->d_cwork_f, 2 * nx + 3 * nfp)) != DG_OK) return cleanup(st);
      c->ctf.Ut = c->d_cwork_f;
      c->ctf.Vt = c->d_cwork_f + nx;
      c->ctf.fJmp = c->d_cwork_f + 2 * nx;
      c->ctf.fHn = c->d_cwork_f + 2 * nx + 2 * nfp;
    }
    c->ct.diffusion = c->ctf.diffusion = diffusion ? 1 : 0;
    c->curved = true;
  }

  // MFMA operand tables (3D configurations with MFMA kernels)
  const char* variant = std::getenv("DG_KERNEL_VARIANT");
  // (the MFMA kernels carry the compressible equations only)
  const bool want_mfma = lattice && compressible && !(variant && std::strcmp(variant, "reference") == 0);
  if (want_mfma && dgk::has_mfma(cfg)) {
    dgh::MfmaHost M;
    try {
      M = dgh::build_mfma_tables(T);
    } catch (const std::exception& ex) {
      return cleanup(fail(DG_ERR_ARG, ex.what()));
    }
    std::vector<const std::vector<double>*> mp = {&M.vA, &M.pA64, &M.fA64, &M.tA, &M.lA64, &M.dA};
    size_t mtot = 0;
    for (auto* v : mp) mtot += v->size();
    if ((st = dalloc(&c->d_mtab, mtot)) != DG_OK) return cleanup(st);
    std::vector<double> mpk;
    std::vector<size_t> moff;
    for (auto* v : mp) {
      moff.push_back(mpk.size());
      mpk.insert(mpk.end(), v->begin(), v->end());
    }
    if (hipMemcpy(c->d_mtab, mpk.data(), mtot * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(DG_ERR_HIP, "MFMA table upload failed"));
    c->mt.vA = c->d_mtab + moff[0];
    c->mt.pA = c->d_mtab + moff[1];
    c->mt.fA = c->d_mtab + moff[2];
    c->mt.tA = c->d_mtab + moff[3];
    c->mt.lA = c->d_mtab + moff[4];
    c->mt.dA = c->d_mtab + moff[5];
    c->mt.kl = M.kl;
    c->use_mfma = true;
    // FP32 copies (interpolation table in the FP32 fragment order)
    std::vector<const std::vector<double>*> fp = {&M.vAf, &M.pA, &M.fA, &M.tA, &M.lA, &M.dAf};
    size_t ftot = 0;
    for (auto* v : fp) ftot += v->size();
    if ((st = dalloc(&c->d_mtab_f, ftot)) != DG_OK) return cleanup(st);
    std::vector<float> fpk;
    std::vector<size_t> foff;
    fpk.reserve(ftot);
    for (auto* v : fp) {
      foff.push_back(fpk.size());
      for (double x : *v) fpk.push_back((float)x);
    }
    if (hipMemcpy(c->d_mtab_f, fpk.data(), ftot * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(DG_ERR_HIP, "FP32 MFMA table upload failed"));
    c->mtf.vA = c->d_mtab_f + foff[0];
    c->mtf.pA = c->d_mtab_f + foff[1];
    c->mtf.fA = c->d_mtab_f + foff[2];
    c->mtf.tA = c->d_mtab_f + foff[3];
    c->mtf.lA = c->d_mtab_f + foff[4];
    c->mtf.dA = c->d_mtab_f + foff[5];
    c->mtf.kl = M.kl;
    // allocated here, not on first use: a captured V-cycle may call either operator
    if ((st = dalloc(&c->d_Hf, (size_t)dim * c->nv * T.nfq * ne)) != DG_OK) return cleanup(st);
    if ((st = dalloc(&c->d_G, (size_t)2 * dim * c->nv * T.nb * ne)) != DG_OK) return cleanup(st);
    if ((st = dalloc(&c->d_Gf, (size_t)2 * dim * c->nv * T.nb * ne)) != DG_OK) return cleanup(st);
  }

  // neighbours transposed to [2*dim][ne], low corners [dim][ne]
  std::vector<int64_t> nbrT((size_t)2 * dim * ne);
  std::vector<double> x0((size_t)dim * ne);
  for (int64_t e = 0; e < ne; ++e) {
    for (int k = 0; k < 2 * dim; ++k) nbrT[(size_t)k * ne + e] = mesh->elem_nbr[e * 2 * dim + k];
    for (int i = 0; i < dim; ++i) x0[(size_t)i * ne + e] = mesh->elem_xyz[(size_t)e * nvtx * dim + i];
  }
  if ((st = dalloc(&c->d_nbr, nbrT.size())) != DG_OK) return cleanup(st);
  if ((st = dalloc(&c->d_x0, x0.size())) != DG_OK) return cleanup(st);
  if (hipMemcpy(c->d_nbr, nbrT.data(), nbrT.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_x0, x0.data(), x0.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(DG_ERR_HIP, "mesh upload failed"));
  c->mesh.ne = ne;
  c->mesh.nbr = c->d_nbr;
  c->mesh.x0 = c->d_x0;
  for (int i = 0; i < 3; ++i) c->mesh.h[i] = h[i];

  for (int64_t e = 0; e < ne && !c->self_nbr; ++e)
    for (int k = 0; k < 2 * dim; ++k) c->self_nbr = c->self_nbr || mesh->elem_nbr[e * 2 * dim + k] == e;

  // greedy colouring of the face-neighbour graph (self loops ignored)
  std::vector<int> color(ne, -1);
  int ncol = 0;
  for (int64_t e = 0; e < ne; ++e) {
    uint64_t used = 0;
    for (int k = 0; k < 2 * dim; ++k) {
      const int64_t n = mesh->elem_nbr[e * 2 * dim + k];
      if (n != e && color[n] >= 0 && color[n] < 64) used |= (uint64_t)1 << color[n];
    }
    int col = 0;
    while (used & ((uint64_t)1 << col)) ++col;
    color[e] = col;
    ncol = std::max(ncol, col + 1);
  }
  c->ncolor = ncol;
  if ((st = dalloc(&c->d_color, (size_t)ne)) != DG_OK) return cleanup(st);
  if (hipMemcpy(c->d_color, color.data(), ne * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return cleanup(fail(DG_ERR_HIP, "colour upload failed"));

  if ((st = dalloc(&c->d_H, (size_t)dim * c->nv * c->nfq * ne)) != DG_OK) return cleanup(st);
  if ((st = dalloc(&c->d_t1, (size_t)c->ndof)) != DG_OK) return cleanup(st);
  if ((st = dalloc(&c->d_t2, (size_t)c->ndof)) != DG_OK) return cleanup(st);
  if ((st = dalloc(&c->d_t3, (size_t)c->ndof)) != DG_OK) return cleanup(st);
  if ((st = dalloc(&c->d_red, (size_t)64 * dgk::kRedBlocks)) != DG_OK) return cleanup(st);
  if ((st = dalloc(&c->d_scal, (size_t)256)) != DG_OK) return cleanup(st);
  if ((st = dalloc(&c->d_flag, (size_t)16)) != DG_OK) return cleanup(st);
  if (hipHostMalloc((void**)&c->h_pin, (kRbSlots * kRbStride + 64) * sizeof(double), hipHostMallocDefault) !=
      hipSuccess) {
    c->h_pin = nullptr;
    return cleanup(fail(DG_ERR_OOM, "pinned host allocation failed"));
  }
  if ((st = noalloc_scratch_address(&c->d_scratch)) != DG_OK) return cleanup(st);
  *out = c;
  return DG_OK;
}

void dg_destroy(dg_context* c) {
  if (!c) return;
  for (auto& kv : c->timers)
    for (auto& ab : kv.second.ev) {
      (void)hipEventDestroy(ab.first);
      (void)hipEventDestroy(ab.second);
    }
  dfree(c->d_tab);
  dfree(c->d_mtab);
  dfree(c->d_mtab_f);
  dfree(c->d_Hf);
  dfree(c->d_G);
  dfree(c->d_Gf);
  dfree(c->d_nbr);
  dfree(c->d_x0);
  dfree(c->d_H);
  dfree(c->d_H2);
  dfree(c->d_Hf2);
  dfree(c->d_cloc);
  dfree(c->d_cloc_f);
  dfree(c->d_t1);
  dfree(c->d_t2);
  dfree(c->d_t3);
  dfree(c->d_rw);
  dfree(c->d_red);
  dfree(c->d_scal);
  dfree(c->d_flag);
  dfree(c->d_color);
  dfree(c->d_D64);
  dfree(c->d_ros);
  dfree(c->d_zero);
  dfree(c->d_curved);
  dfree(c->d_cwork);
  dfree(c->d_curved_f);
  dfree(c->d_cwork_f);
  if (c->d_Dinv != c->d_D64) dfree(c->d_Dinv);
  dfree(c->d_V);
  dfree(c->d_Z);
  mg_destroy(c->mg);
  mlp_destroy(c->mlp);
  if (c->h_pin) (void)hipHostFree(c->h_pin);
  for (int i = 0; i < kRbSlots; ++i)
    if (c->ev_rb[i]) (void)hipEventDestroy(c->ev_rb[i]);
  delete c;
}

int64_t dg_ndof(const dg_context* c) { return c ? c->ndof : -1; }
int dg_nbasis(const dg_context* c) { return c ? c->nb : -1; }
int dg_nvar(const dg_context* c) { return c ? c->nv : -1; }
int dg_nq(const dg_context* c) { return c ? c->nq : -1; }

dg_status dg_volume_points(dg_context* c, double* xyz, void* stream) {
  if (!c || !xyz) return fail(DG_ERR_ARG, "null argument");
  if (c->curved) {
    HIPCHK(hipMemcpyAsync(xyz, c->d_cvX, (size_t)c->dim * c->nq * c->ne * sizeof(double), hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
    return DG_OK;
  }
  HIPCHK(dgk::launch_points(c->cfg, xyz, c->tb, c->mesh, (hipStream_t)stream));
  return DG_OK;
}

dg_status dg_project(dg_context* c, const double* f, double* w, void* stream) {
  if (!c || !f || !w) return fail(DG_ERR_ARG, "null argument");
  if (c->curved) {
    HIPCHK(dgk::launch_project_curved(c->cfg, f, w, c->ct, c->ne, (hipStream_t)stream));
    return DG_OK;
  }
  HIPCHK(dgk::launch_project(c->cfg, c->nv, f, w, c->tb, c->mesh, (hipStream_t)stream));
  return DG_OK;
}

dg_status dg_residual(dg_context* c, const double* w, double* r, void* stream) {
  if (!c || !w || !r) return fail(DG_ERR_ARG, "null argument");
  if (w == r) return fail(DG_ERR_ARG, "w and r may not alias");
  return eval_residual(c, false, w, nullptr, 0.0, r, (hipStream_t)stream);
}

dg_status dg_residual_fp32(dg_context* c, const double* w, double* r, void* stream) {
  if (!c || !w || !r) return fail(DG_ERR_ARG, "null argument");
  if (w == r) return fail(DG_ERR_ARG, "w and r may not alias");
  return eval_residual_f32(c, false, w, nullptr, 0.0, r, (hipStream_t)stream);
}

dg_status dg_residual_bf16(dg_context* c, const double* w, double* r, void* stream) {
  if (!c || !w || !r) return fail(DG_ERR_ARG, "null argument");
  if (w == r) return fail(DG_ERR_ARG, "w and r may not alias");
  return eval_op(c, DG_BF16, false, w, nullptr, 0.0, r, (hipStream_t)stream);
}

dg_status dg_jvp(dg_context* c, const double* w, const double* r_w, const double* v, double shift, int mode,
                 double* out, void* stream) {
  if (!c || !w || !v || !out) return fail(DG_ERR_ARG, "null argument");
  if (out == w || out == v || (r_w && out == r_w)) return fail(DG_ERR_ARG, "out may not alias w, v or r_w");
  if (mode != DG_JVP_EXACT && mode != DG_JVP_FD && mode != DG_JVP_EXACT_FP32 && mode != DG_JVP_STAB &&
      mode != DG_JVP_EXACT_BF16)
    return fail(DG_ERR_ARG, "unknown jvp mode");
  return jvp_impl(c, w, r_w, v, shift, mode, out, (hipStream_t)stream);
}

}  // extern "C"

namespace dgc {

dg_status block_alloc(dg_context* c, int storage) {
  const int m = c->nv * c->nb;
  dg_status st;
  c->blk_ready = false;
  const int ld = dgk::block_ld(m);
  if ((st = dalloc(&c->d_D64, (size_t)c->ne * m * ld)) != DG_OK) return st;
  if (storage == DG_FP64) {
    // FP64 inverses overwrite the probed blocks in place
    if (c->d_Dinv && c->d_Dinv != c->d_D64) dfree(c->d_Dinv);
    c->d_Dinv = c->d_D64;
    c->dinv_bytes = 0;
  } else {
    const size_t need = (size_t)c->ne * m * ld * (storage == DG_FP32 ? sizeof(float) : sizeof(uint16_t));
    if (c->d_Dinv == c->d_D64) c->d_Dinv = nullptr;
    if (c->d_Dinv && c->dinv_bytes != need) {
      dfree(c->d_Dinv);
      c->d_Dinv = nullptr;
    }
    if (!c->d_Dinv) {
      unsigned char* f = nullptr;
      if ((st = dalloc(&f, need)) != DG_OK) return st;
      c->d_Dinv = f;
      c->dinv_bytes = need;
    }
  }
  return DG_OK;
}

dg_status block_probe_invert(dg_context* c, const double* w, double shift, int storage, int skip_modes,
                             int probe_prec, hipStream_t s) {
  const int m = c->nv * c->nb, ld = dgk::block_ld(m);
  dg_status st;
  if (!has_prec(c, probe_prec)) return fail(DG_ERR_ARG, "no operator of the probing precision");
  if ((st = tune_fine(c, probe_prec, w, s)) != DG_OK) return st;
  {
    ProfScope ps(c, "block_probe", s);
    // element-local: one pass per column, all elements at once (colour -1);
    // coloured: one Jv per column and colour
    const bool local = local_probe_ok(c, probe_prec);
    for (int col = local ? -1 : 0; col < (local ? 0 : c->ncolor); ++col)
      for (int l = 0; l < m; ++l) {
        if (l % c->nb < skip_modes) continue;  // column already in d_D64
        HIPCHK(dgk::launch_probe_vector(c->d_t1, c->d_color, col, l, c->nb, c->nv, c->ne, s));
        st = local ? eval_local(c, probe_prec, w, c->d_t1, shift, c->d_t2, s)
                   : eval_op(c, probe_prec, true, w, c->d_t1, shift, c->d_t2, s);
        if (st != DG_OK) return st;
        HIPCHK(dgk::launch_extract_column(c->d_t2, c->d_color, col, l, m, c->ne, shift, c->d_D64, s));
      }
  }
  int zero = 0;
  HIPCHK(hipMemcpyAsync(c->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice, s));
  {
    ProfScope ps(c, "block_invert", s);
    HIPCHK(dgk::launch_block_invert(storage, c->d_D64, ld, c->d_Dinv, m, c->ne, c->d_flag, s));
  }
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (bad) return fail(DG_ERR_SINGULAR_BLOCK, "a diagonal block has a zero or non-finite pivot");
  c->blk_storage = storage;
  if ((st = tune_apply(c, storage, c->d_Dinv, m, &c->blk_shape, s)) != DG_OK) return st;
  c->blk_ready = true;
  return DG_OK;
}

}  // namespace dgc

extern "C" {

dg_status dg_set_block_probing(dg_context* c, int mode) {
  if (!c) return fail(DG_ERR_ARG, "null context");
  if (mode != DG_PROBE_AUTO && mode != DG_PROBE_COLOURED) return fail(DG_ERR_ARG, "unknown probing mode");
  c->probe_mode = mode;
  return DG_OK;
}

dg_status dg_block_precond_setup(dg_context* c, const double* w, double shift, int storage, void* stream) {
  if (!c || !w) return fail(DG_ERR_ARG, "null argument");
  if (storage != DG_FP64 && storage != DG_FP32 && storage != DG_BF16)
    return fail(DG_ERR_ARG, "storage must be DG_FP64, DG_FP32 or DG_BF16");
  if (c->nv * c->nb > 256) return fail(DG_ERR_ARG, "block size above 256");
  mg_invalidate(c->mg);
  dg_status st;
  const auto t0 = std::chrono::steady_clock::now();
  if ((st = block_alloc(c, storage)) != DG_OK) return st;
  st = block_probe_invert(c, w, shift, storage, 0, default_probe_prec(c, storage), (hipStream_t)stream);
  c->ms_setup_bj = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

dg_status dg_block_precond_apply(dg_context* c, const double* r, double* z, void* stream) {
  if (!c || !r || !z) return fail(DG_ERR_ARG, "null argument");
  if (r == z) return fail(DG_ERR_ARG, "r and z may not alias");
  if (!c->blk_ready) return fail(DG_ERR_STATE, "dg_block_precond_setup has not succeeded");
  hipStream_t s = (hipStream_t)stream;
  ProfScope ps(c, "block_apply", s);
  HIPCHK(dgk::launch_block_apply(c->blk_storage, c->d_Dinv, c->nv * c->nb, c->ne, r, z, s, &c->blk_shape));
  return DG_OK;
}

dg_status dg_max_wave_speed(dg_context* c, const double* w, double* out, void* stream) {
  if (!c || !w || !out) return fail(DG_ERR_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const int nblk = 1024;
  if (c->curved && c->ct.diffusion)
    return fail(DG_ERR_ARG, "the maximum wave speed is defined for the compressible equations on curved meshes");
  if (c->curved)
    HIPCHK(dgk::launch_wave_speed_curved(c->cfg, w, c->d_red, nblk, c->ct, c->mesh, c->ph, s));
  else
    HIPCHK(dgk::launch_wave_speed(c->cfg, w, c->d_red, nblk, c->tb, c->mesh, c->ph, s));
  HIPCHK(dgk::launch_max_partials(c->d_red, nblk, c->d_scal + 200, s));
  HIPCHK(hipMemcpyAsync(c->h_pin, c->d_scal + 200, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *out = c->h_pin[0];
  return DG_OK;
}

dg_status dg_fgmres_solve(dg_context* c, const double* w, double shift, const double* b, double* x,
                          const dg_solve_opts* opts, dg_solve_stats* stats, void* stream) {
  if (!c || !w || !b || !x || !opts) return fail(DG_ERR_ARG, "null argument");
  if (x == b || x == w) return fail(DG_ERR_ARG, "x may not alias w or b");
  const int m = opts->restart > 0 ? opts->restart : 30;
  if (m > 60) return fail(DG_ERR_ARG, "restart above 60");
  if (opts->precond != DG_PREC_NONE && opts->precond != DG_PREC_BJ && opts->precond != DG_PREC_MG &&
      opts->precond != DG_PREC_MLP)
    return fail(DG_ERR_ARG, "unknown precond");
  if (opts->precond == DG_PREC_MLP && !mlp_ready(c->mlp)) return fail(DG_ERR_STATE, "network weights not set");
  if (opts->precond == DG_PREC_BJ && !c->blk_ready) return fail(DG_ERR_STATE, "block preconditioner not set up");
  if (opts->precond == DG_PREC_MG && !mg_ready(c->mg)) return fail(DG_ERR_STATE, "p-multigrid not set up");
  if (opts->jvp_mode != DG_JVP_EXACT && opts->jvp_mode != DG_JVP_FD)
    return fail(DG_ERR_ARG, "the solve's operator is the exact FP64 or the finite-difference Jv");
  if (opts->orth != DG_ORTH_CGS2 && opts->orth != DG_ORTH_MGS) return fail(DG_ERR_ARG, "unknown orthogonalisation");
  const bool mgs = opts->orth == DG_ORTH_MGS;
  if (opts->check_every < 0) return fail(DG_ERR_ARG, "check_every must be >= 0");
  const int check_every = opts->check_every > 0 ? opts->check_every : 1;
  const double rtol = opts->rtol > 0.0 ? opts->rtol : 1e-8;
  const int max_iter = opts->max_iter > 0 ? opts->max_iter : 1000;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = c->ndof;
  dg_status st;
  auto t0 = std::chrono::steady_clock::now();
  if (c->kry_m < m) {
    dfree(c->d_V);
    dfree(c->d_Z);
    c->d_V = c->d_Z = nullptr;
    c->kry_m = 0;
    if ((st = dalloc(&c->d_V, (size_t)(m + 1) * n)) != DG_OK) return st;
    if ((st = dalloc(&c->d_Z, (size_t)m * n)) != DG_OK) return st;
    c->kry_m = m;
  }
  for (int i = 0; i < m; ++i)
    if (!c->ev_rb[i]) HIPCHK(hipEventCreateWithFlags(&c->ev_rb[i], hipEventDisableTiming));
  const double* rw = nullptr;
  if (opts->jvp_mode == DG_JVP_FD) {
    if ((st = dalloc(&c->d_rw, (size_t)n)) != DG_OK) return st;
    if ((st = eval_residual(c, false, w, nullptr, 0.0, c->d_rw, s)) != DG_OK) return st;
    rw = c->d_rw;
  }
  auto applyG = [&](const double* z, double* outv) { return jvp_impl(c, w, rw, z, shift, opts->jvp_mode, outv, s); };
  int prec = opts->precond;  // the learned preconditioner may fall back to block Jacobi
  const int judge_after = opts->judge_after > 0 ? opts->judge_after : 5;
  int fallbacks = 0;
  auto applyM = [&](const double* v, double* z) -> dg_status {
    if (prec == DG_PREC_MG) return mg_apply(c, v, z, s);
    if (prec == DG_PREC_MLP) return mlp_apply(c, w, v, z, s);
    if (prec == DG_PREC_BJ) {
      ProfScope ps(c, "block_apply", s);
      HIPCHK(dgk::launch_block_apply(c->blk_storage, c->d_Dinv, c->nv * c->nb, c->ne, v, z, s, &c->blk_shape));
      return DG_OK;
    }
    HIPCHK(dgk::launch_axpby(n, 1.0, v, 0.0, v, z, s));
    return DG_OK;
  };
  auto readback = [&](const double* dptr, int cnt) -> dg_status {
    HIPCHK(hipMemcpyAsync(c->h_pin, dptr, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return DG_OK;
  };
  // device scalars: [0] |b|, [1] beta, [2] |w| before orthogonalisation (MGS; CGS2: |w|^2 at
  // [16 + j + 1]), [3] h_{j+1,j}; [16..] h pass 1; [80..] h pass 2; [144..] y
  double* dS = c->d_scal;
  if ((st = norm2(c, b, dS + 0, s)) != DG_OK) return st;
  if ((st = readback(dS + 0, 1)) != DG_OK) return st;
  const double bnorm = c->h_pin[0];
  dg_solve_stats S{};
  if (!std::isfinite(bnorm)) return fail(DG_ERR_NONFINITE, "right-hand side is not finite");
  if (bnorm == 0.0) {
    HIPCHK(dgk::launch_fill(x, n, 0.0, s));
    S.converged = 1;
    if (stats) *stats = S;
    return DG_OK;
  }
  double* V = c->d_V;
  double* Z = c->d_Z;
  // r0 = b - G x
  if ((st = applyG(x, c->d_t1)) != DG_OK) return st;
  HIPCHK(dgk::launch_axpby(n, 1.0, b, -1.0, c->d_t1, V, s));
  if ((st = norm2(c, V, dS + 1, s)) != DG_OK) return st;
  if ((st = readback(dS + 1, 1)) != DG_OK) return st;
  double beta = c->h_pin[0];
  const double d0 = beta;
  int iters = 0;
  double est = beta;
  bool converged = false;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  while (true) {
    if (!std::isfinite(beta)) return fail(DG_ERR_NONFINITE, "residual is not finite");
    if (beta <= rtol * bnorm) {
      converged = true;
      break;
    }
    if (iters >= max_iter) break;
    HIPCHK(dgk::launch_scale_dev(n, V, dS + 1, V, s));
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    // The Hessenberg column of iteration j travels to the host asynchronously
    // (pinned slot j, event ev_rb[j]); every check_every iterations the host
    // applies the Givens rotations of the columns that arrived and tests
    // convergence, keeping the newest iteration in flight on the GPU.
    // Iterations enqueued past the stopping point are discarded (with the
    // V-cycle as preconditioner no iteration is left in flight at a check).
    int k = 0;
    std::vector<int> pend;
    bool stop = false;
    auto process = [&](int jj) -> dg_status {
      HIPCHK(hipEventSynchronize(c->ev_rb[jj]));
      const double* hp = c->h_pin + (size_t)kRbStride * jj;
      const double w0 = mgs ? hp[2] : std::sqrt(hp[16 + jj + 1]), hn = hp[3];
      if (!std::isfinite(hn)) return fail(DG_ERR_NONFINITE, "Arnoldi vector is not finite");
      double* Hc = &H[(size_t)jj * (m + 1)];  // column jj, rows 0..jj+1
      for (int i = 0; i <= jj; ++i) Hc[i] = mgs ? hp[16 + i] : hp[16 + i] + hp[80 + i];
      Hc[jj + 1] = hn;
      for (int i = 0; i < jj; ++i) {
        const double t = cs[i] * Hc[i] + sn[i] * Hc[i + 1];
        Hc[i + 1] = -sn[i] * Hc[i] + cs[i] * Hc[i + 1];
        Hc[i] = t;
      }
      const double den = std::hypot(Hc[jj], Hc[jj + 1]);
      cs[jj] = den > 0.0 ? Hc[jj] / den : 1.0;
      sn[jj] = den > 0.0 ? Hc[jj + 1] / den : 0.0;
      Hc[jj] = den;
      Hc[jj + 1] = 0.0;
      g[jj + 1] = -sn[jj] * g[jj];
      g[jj] = cs[jj] * g[jj];
      k = jj + 1;
      ++iters;
      est = std::fabs(g[jj + 1]);
      // judge of the learned preconditioner: a convergence factor above the
      // reference one after judge_after iterations switches to block Jacobi
      // (legal in flexible GMRES: every z_j is stored)
      if (prec == DG_PREC_MLP && opts->rho_ref > 0.0 && iters == judge_after && c->blk_ready && d0 > 0.0) {
        const double rho_now = std::exp(std::log(std::max(est, 1e-300) / d0) / iters);
        if (rho_now > opts->rho_ref) {
          prec = DG_PREC_BJ;
          ++fallbacks;
        }
      }
      const bool brk = hn <= 1e-14 * w0;
      stop = est <= rtol * bnorm || brk || iters >= max_iter;
      return DG_OK;
    };
    for (int j = 0; j < m && !stop; ++j) {
      double* Vj = V + (size_t)j * n;
      double* Zj = Z + (size_t)j * n;
      double* Wn = V + (size_t)(j + 1) * n;
      if ((st = applyM(Vj, Zj)) != DG_OK) return st;
      if ((st = applyG(Zj, Wn)) != DG_OK) return st;
      if (mgs && (st = norm2(c, Wn, dS + 2, s)) != DG_OK) return st;
      {
        ProfScope ps(c, "arnoldi", s);
        if (mgs) {  // modified Gram-Schmidt: one basis vector at a time
          for (int i = 0; i <= j; ++i) {
            HIPCHK(dgk::launch_mdot(V + (size_t)i * n, 1, n, Wn, c->d_red, s));
            HIPCHK(dgk::launch_msum(c->d_red, 1, dS + 16 + i, s));
            HIPCHK(dgk::launch_mupdate(V + (size_t)i * n, 1, n, dS + 16 + i, Wn, s));
          }
        } else {  // classical Gram-Schmidt with one re-orthogonalisation; the first
                  // pass also gives |Wn|^2 (Wn is V_{j+1}) as entry j + 1
          HIPCHK(dgk::launch_mdot(V, j + 2, n, Wn, c->d_red, s));
          HIPCHK(dgk::launch_msum(c->d_red, j + 2, dS + 16, s));
          HIPCHK(dgk::launch_mupdate(V, j + 1, n, dS + 16, Wn, s));
          HIPCHK(dgk::launch_mdot(V, j + 1, n, Wn, c->d_red, s));
          HIPCHK(dgk::launch_msum(c->d_red, j + 1, dS + 80, s));
          HIPCHK(dgk::launch_mupdate(V, j + 1, n, dS + 80, Wn, s));
        }
      }
      if ((st = norm2(c, Wn, dS + 3, s)) != DG_OK) return st;
      HIPCHK(hipMemcpyAsync(c->h_pin + (size_t)kRbStride * j, dS, 144 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipEventRecord(c->ev_rb[j], s));
      HIPCHK(dgk::launch_scale_dev(n, Wn, dS + 3, Wn, s));
      pend.push_back(j);
      if ((j + 1) % check_every == 0 || j == m - 1) {
        // a V-cycle per iteration is too costly to run past the stop speculatively
        const size_t keep = (prec == DG_PREC_MG || j == m - 1) ? 0 : 1;
        size_t done = 0;
        while (pend.size() - done > keep && !stop)
          if ((st = process(pend[done++])) != DG_OK) return st;
        pend.erase(pend.begin(), pend.begin() + done);
      }
    }
    for (size_t i = 0; i < pend.size() && !stop; ++i)
      if ((st = process(pend[i])) != DG_OK) return st;
    // y = H_k^{-1} g (upper triangular back substitution)
    for (int i = k - 1; i >= 0; --i) {
      double a = g[i];
      for (int l = i + 1; l < k; ++l) a -= H[(size_t)l * (m + 1) + i] * y[l];
      const double d = H[(size_t)i * (m + 1) + i];
      y[i] = d != 0.0 ? a / d : 0.0;
    }
    double* hy = c->h_pin + (size_t)kRbSlots * kRbStride;
    for (int i = 0; i < k; ++i) hy[i] = y[i];
    HIPCHK(hipMemcpyAsync(dS + 144, hy, k * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(dgk::launch_mupdate_add(Z, k, n, dS + 144, x, s));
    if ((st = applyG(x, c->d_t1)) != DG_OK) return st;
    HIPCHK(dgk::launch_axpby(n, 1.0, b, -1.0, c->d_t1, V, s));
    if ((st = norm2(c, V, dS + 1, s)) != DG_OK) return st;
    if ((st = readback(dS + 1, 1)) != DG_OK) return st;
    beta = c->h_pin[0];
    ++S.restarts;
  }
  S.iters = iters;
  S.fallbacks = fallbacks;
  S.converged = converged ? 1 : 0;
  S.rel_res_est = est / bnorm;
  S.rel_res_true = beta / bnorm;
  S.rho = (iters > 0 && beta > 0.0 && d0 > 0.0) ? std::exp(std::log(beta / d0) / iters) : 0.0;
  S.ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  S.ms_setup = opts->precond == DG_PREC_BJ ? c->ms_setup_bj : (opts->precond == DG_PREC_MG ? c->ms_setup_mg : 0.0);
  if (stats) *stats = S;
  return converged ? DG_OK : DG_NOT_CONVERGED;
}

dg_status dg_set_profiling(dg_context* c, int on) {
  if (!c) return fail(DG_ERR_ARG, "null context");
  c->prof = on != 0;
  return DG_OK;
}

dg_status dg_kernel_time(dg_context* c, const char* name, double* ms, int64_t* launches) {
  if (!c || !name) return fail(DG_ERR_ARG, "null argument");
  auto it = c->timers.find(name);
  double tot = 0.0;
  int64_t cnt = 0;
  if (it != c->timers.end()) {
    for (auto& ab : it->second.ev) {
      HIPCHK(hipEventSynchronize(ab.second));
      float t = 0.0f;
      HIPCHK(hipEventElapsedTime(&t, ab.first, ab.second));
      tot += t;
      ++cnt;
      (void)hipEventDestroy(ab.first);
      (void)hipEventDestroy(ab.second);
    }
    it->second.ev.clear();
  }
  if (ms) *ms = tot;
  if (launches) *launches = cnt;
  return DG_OK;
}

dg_status dg_sync(dg_context* c) {
  (void)c;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipGetLastError());
  return DG_OK;
}

}  // extern "C"
