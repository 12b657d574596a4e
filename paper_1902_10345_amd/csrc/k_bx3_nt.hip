// k_bx3_nt.hip -- one-pass MFMA GEMM tiles with B transposed.
#include "bx3_launch.hpp"

namespace mm {

gemm_status bx3_run_nt(const GemmArgs &g, int cfg, hipStream_t s) {
  return bx3::bx3_run_trans<false, true>(g, cfg, s);
}

gemm_status f32mfma_run_nt(const GemmArgs &g, int which, hipStream_t s) {
  return bx3::f32mfma_run_trans<false, true>(g, which, s);
}

}  // namespace mm
