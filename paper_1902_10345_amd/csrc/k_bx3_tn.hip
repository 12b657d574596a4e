// k_bx3_tn.hip -- one-pass MFMA GEMM tiles with A transposed.
#include "bx3_launch.hpp"

namespace mm {

gemm_status bx3_run_tn(const GemmArgs &g, int cfg, hipStream_t s) {
  return bx3::bx3_run_trans<true, false>(g, cfg, s);
}

gemm_status f32mfma_run_tn(const GemmArgs &g, int which, hipStream_t s) {
  return bx3::f32mfma_run_trans<true, false>(g, which, s);
}

}  // namespace mm
