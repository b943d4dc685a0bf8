// One instance set of the matrix-core step kernel: GEMM precision, optimiser
// and workgroup width fixed by the build (PMKLC_BF16, PMKLC_ADAM, PMKLC_NT),
// all row-tile counts and F1 unit shapes.  The build compiles this file once
// per combination, side by side; step_mfma.hip dispatches to them.
#include "step_mfma.h"

namespace pmklc {

hipError_t PMKLC_VARIANT(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st) {
#if PMKLC_BF16
  typedef MmaBf16 P;
#else
  typedef MmaF32 P;
#endif
  return launch_f1<PMKLC_NT, P, PMKLC_ADAM != 0>(a_dev, grid, mt, f1_fours, lds, st);
}

}  // namespace pmklc
