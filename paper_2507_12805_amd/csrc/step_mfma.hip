// Dispatch to the matrix-core step kernel instances (step_mfma_inst.hip,
// compiled once per precision, optimiser and workgroup width), and the BF16
// fragment-order conversion of a first-layer weight matrix.
#include "pmklc_internal.h"

namespace pmklc {

hipError_t launch_mfma_bf16_sgd_256(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);
hipError_t launch_mfma_bf16_sgd_512(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);
hipError_t launch_mfma_bf16_adam_256(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);
hipError_t launch_mfma_bf16_adam_512(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);
hipError_t launch_mfma_f32_sgd_256(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);
hipError_t launch_mfma_f32_sgd_512(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);
hipError_t launch_mfma_f32_adam_256(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);
hipError_t launch_mfma_f32_adam_512(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st);

// W1 (D x H, FP32) -> BF16 in the first layer's fragment order
__global__ void w1_frag_kernel(const float *__restrict__ W1, int D, int H, uint16_t *__restrict__ out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= D * H) return;
  const int dd = q / H, h = q - dd * H;
  __bf16 v = (__bf16)W1[q];
  out[w1_frag_index(dd, h, D)] = __builtin_bit_cast(uint16_t, v);
}

hipError_t launch_w1_frag(const float *W1, int D, int H, uint16_t *out, hipStream_t st) {
  const int n = D * H;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(w1_frag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, W1, D, H, out);
  return hipGetLastError();
}


// a_dev: a device copy of `a` (kernel arguments are read through it).
// nt: 256 or 512 threads per workgroup; the choice never changes a value.
hipError_t launch_step_mfma(const StepArgs &a, const StepArgs *a_dev, int grid, bool bf16, int nt, int f1,
                            hipStream_t st) {
  // the BF16 kernel reads and writes W1 through its BF16 copies: refuse to
  // launch without them
  if (bf16 && (!a.w1f || (a.d.static_on && (!a.s1f || !a.stat)))) return hipErrorInvalidValue;
  const size_t lds = (size_t)a.lay.total;
  const int mt = a.d.bs / 16;
  const bool adam = a.d.optimizer == 1;
  const bool f1_fours = (a.d.H[0] / 16) % 4 == 0 && f1 != 0;
  if (nt != 256 && nt != 512) return hipErrorInvalidValue;
  const bool w = nt == 512;
  if (bf16) {
    if (adam) return (w ? launch_mfma_bf16_adam_512 : launch_mfma_bf16_adam_256)(a_dev, grid, mt, f1_fours, lds, st);
    return (w ? launch_mfma_bf16_sgd_512 : launch_mfma_bf16_sgd_256)(a_dev, grid, mt, f1_fours, lds, st);
  }
  if (adam) return (w ? launch_mfma_f32_adam_512 : launch_mfma_f32_adam_256)(a_dev, grid, mt, f1_fours, lds, st);
  return (w ? launch_mfma_f32_sgd_512 : launch_mfma_f32_sgd_256)(a_dev, grid, mt, f1_fours, lds, st);
}

}  // namespace pmklc
