// Launchers of the MFMA residual / Jv kernels of dg_mfma.h: the FP32
// operator (v_mfma_f32_16x16x4; FP32 tables, buffers and pointwise
// arithmetic).
#include "dg_mfma.h"

namespace dgk {

hipError_t launch_grad_mfma_f32(int cfg, bool jvp, const double* U, const double* V, float* Gm, const MTablesF& mt,
                                const Mesh& m, hipStream_t s, const double* Vn) {
  return grad_mfma_dispatch<float, MP<float>>(cfg, jvp, U, V, Gm, mt, m, s, Vn);
}

hipError_t launch_face_mfma_f32(int cfg, bool jvp, const double* U, const double* V, float* H, const MTablesF& mt,
                                const Mesh& m, const Phys& ph, int occ, hipStream_t s, const double* Vr) {
  return face_mfma_dispatch<float, MP<float>>(cfg, jvp, U, V, H, mt, m, ph, occ, s, Vr);
}

hipError_t launch_volume_mfma_f32(int cfg, bool jvp, const double* U, const double* V, const float* Gm,
                                  const float* H, double* out, double shift, const MTablesF& mt, const Mesh& m,
                                  const Phys& ph, int occ, bool fused, hipStream_t s, const float* Hm,
                                  const double* Vn) {
  return volume_mfma_dispatch<float, MP<float>>(cfg, jvp, U, V, Gm, H, out, shift, mt, m, ph, occ, fused, s, Hm, Vn);
}

}  // namespace dgk
