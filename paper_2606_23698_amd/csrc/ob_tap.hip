// The debug variants of the stage kernels (residue tap and the epilogue
// record of one line); the same tile code as the production kernels.
#include "ob_stage.h"

namespace obfft {

hipError_t launch_stage_tap(int sub, int tgt, bool h0, const StageParams& P, dim3 grid, hipStream_t st) {
  if (sub == SUB_FP16) {
    if (h0) return tgt == 0 ? launch_stage_k<SUB_FP16, 0, true, true>(P, grid, st) : hipErrorInvalidValue;
    return tgt == 0 ? launch_stage_k<SUB_FP16, 0, false, true>(P, grid, st)
                    : launch_stage_k<SUB_FP16, 1, false, true>(P, grid, st);
  }
  if (h0) return hipErrorInvalidValue;
  if (sub == SUB_INT8)
    return tgt == 0 ? launch_stage_k<SUB_INT8, 0, false, true>(P, grid, st)
                    : launch_stage_k<SUB_INT8, 1, false, true>(P, grid, st);
  return tgt == 0 ? launch_stage_k<SUB_FP8, 0, false, true>(P, grid, st)
                  : launch_stage_k<SUB_FP8, 1, false, true>(P, grid, st);
}

}  // namespace obfft
