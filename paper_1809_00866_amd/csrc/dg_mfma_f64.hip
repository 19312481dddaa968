// Launchers of the MFMA residual / Jv kernels of dg_mfma.h: FP64 MFMA (v_mfma_f64_16x16x4).
#include "dg_mfma.h"

namespace dgk {

bool has_mfma(int cfg) {
#define X(id, nb_, nq_, kl_) \
  if (cfg == id) return true;
  DG_MFMA_CONFIGS(X)
#undef X
  return false;
}

bool mfma_occ_fits(int cfg, int prec, int face_occ, int volume_occ) {
  if (face_occ < 0 || face_occ > 2 || volume_occ < 0 || volume_occ > 2) return false;
#define X(id, nb_, nq_, kl_)                                                                          \
  if (cfg == id)                                                                                      \
    return face_occ != 2 || !(prec == DG_FP64 ? FaceTab<double, nb_>::only_default : FaceTab<float, nb_>::only_default);
  DG_MFMA_CONFIGS(X)
#undef X
  return false;
}

hipError_t launch_face_mfma(int cfg, bool jvp, const double* U, const double* V, double* H, const MTables& mt,
                            const Mesh& m, const Phys& ph, int occ, hipStream_t s, const double* Vr) {
  return face_mfma_dispatch<double, MP<double>>(cfg, jvp, U, V, H, mt, m, ph, occ, s, Vr);
}

hipError_t launch_volume_mfma(int cfg, bool jvp, const double* U, const double* V, const double* Gm, const double* H,
                              double* out, double shift, const MTables& mt, const Mesh& m, const Phys& ph, int occ,
                              bool fused, hipStream_t s, const double* Hm,
                                  const double* Vn) {
  return volume_mfma_dispatch<double, MP<double>>(cfg, jvp, U, V, Gm, H, out, shift, mt, m, ph, occ, fused, s, Hm, Vn);
}

hipError_t launch_grad_mfma(int cfg, bool jvp, const double* U, const double* V, double* Gm, const MTables& mt,
                            const Mesh& m, hipStream_t s, const double* Vn) {
  return grad_mfma_dispatch<double, MP<double>>(cfg, jvp, U, V, Gm, mt, m, s, Vn);
}

}  // namespace dgk
