// The dynamic model as a stand-alone differentiable op (forward, and a
// hand-written backward that recomputes the activations from the contexts
// instead of storing them), for use under torch.autograd and for gradient
// checks.  Same model as the step kernels: x = concat(Emb[ctx_0..ctx_{t-1}]),
// h_{l+1} = ReLU(h_l W_l + b_l), logits = h_nh W_nh + b_nh (Sec. 4.2.4 with
// the MLP reading; gradient of Eq. 2 flows in as dlogits).
//
// Every GEMM output element is computed by one thread with a fixed k order;
// the embedding gradient is summed in 64-bit fixed point with integer
// atomics, so results do not depend on scheduling.
#include "pmklc_internal.h"

namespace pmklc {

namespace {

constexpr int TILE = 32;

// C[M][N] = op(A) op(B) (+ bias[n]) (ReLU); A is [M][K] (or [K][M] when TA),
// B is [K][N] (or [N][K] when TB). If mask != null, C *= (mask[m][n] > 0).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const float *__restrict__ A,
                                                   const float *__restrict__ B, float *__restrict__ C,
                                                   const float *__restrict__ bias, int relu,
                                                   const float *__restrict__ mask) {
  __shared__ float As[TILE][TILE + 1], Bs[TILE][TILE + 1];
  const int tx = threadIdx.x % TILE, ty = threadIdx.x / TILE;   // 32 x 8 threads, 4 rows each
  const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += TILE) {
    for (int q = 0; q < 4; q++) {
      const int rr = ty + 8 * q;
      // As[m][k], Bs[k][n]
      {
        const int m = m0 + rr, k = k0 + tx;
        float v = 0.0f;
        if (m < M && k < K) v = TA ? A[(size_t)k * M + m] : A[(size_t)m * K + k];
        As[rr][tx] = v;
      }
      {
        const int k = k0 + rr, n = n0 + tx;
        float v = 0.0f;
        if (k < K && n < N) v = TB ? B[(size_t)n * K + k] : B[(size_t)k * N + n];
        Bs[rr][tx] = v;
      }
    }
    __syncthreads();
    for (int kk = 0; kk < TILE; kk++) {
      const float b = Bs[kk][tx];
#pragma unroll
      for (int q = 0; q < 4; q++) acc[q] = fmaf(As[ty + 8 * q][kk], b, acc[q]);
    }
    __syncthreads();
  }
  for (int q = 0; q < 4; q++) {
    const int m = m0 + ty + 8 * q, n = n0 + tx;
    if (m < M && n < N) {
      float v = acc[q] + (bias ? bias[n] : 0.0f);
      if (relu) v = fmaxf(v, 0.0f);
      if (mask) v = mask[(size_t)m * N + n] > 0.0f ? v : 0.0f;
      C[(size_t)m * N + n] = v;
    }
  }
}

template <bool TA, bool TB>
hipError_t gemm(int M, int N, int K, const float *A, const float *B, float *C, const float *bias, bool relu,
                const float *mask, hipStream_t st) {
  if (M == 0 || N == 0) return hipSuccess;
  dim3 grid((N + TILE - 1) / TILE, (M + TILE - 1) / TILE);
  hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(256), 0, st, M, N, K, A, B, C, bias, relu ? 1 : 0, mask);
  return hipGetLastError();
}

__global__ void gather_x_kernel(const float *emb, const uint8_t *ctx, int rows, int t, int E, int V, float *X,
                                int *err) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t D = (size_t)t * E;
  if (i >= (size_t)rows * D) return;
  const size_t j = i / D, dd = i % D, p = dd / E, e = dd % E;
  const int tok = ctx[j * t + p];
  if (tok >= V) { atomicOr(err, 1); X[i] = 0.0f; return; }
  X[i] = emb[(size_t)tok * E + e];
}

// column sums in fixed order (one thread per column)
__global__ void colsum_kernel(const float *G, int rows, int N, float *out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int j = 0; j < rows; j++) s += G[(size_t)j * N + n];
  out[n] = s;
}

__device__ __forceinline__ long long fixed(float x) {
  double y = (double)x * (double)(1ull << kFixShift);
  y = fmin(fmax(y, -4.0e18), 4.0e18);
  return (long long)rint(y);
}

// (a token >= V has no embedding row: the gather flagged it and it is skipped here)
__global__ void scatter_emb_kernel(const float *dX, const uint8_t *ctx, int rows, int t, int E, int V, long long *acc) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t D = (size_t)t * E;
  if (i >= (size_t)rows * D) return;
  const size_t j = i / D, dd = i % D, p = dd / E, e = dd % E;
  const int tok = ctx[j * t + p];
  if (tok >= V) return;
  atomicAdd(reinterpret_cast<unsigned long long *>(acc + (size_t)tok * E + e), (unsigned long long)fixed(dX[i]));
}

__global__ void fixed_to_float_kernel(const long long *acc, int n, float *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)((double)acc[i] * (1.0 / (double)(1ull << kFixShift)));
}

}  // namespace

// Workspace: X, activations per layer, two gradient buffers, fixed-point
// embedding accumulator, error word.
uint64_t dm_op_workspace(const Dims &d, int rows) {
  uint64_t f = (uint64_t)rows * d.D;
  for (int l = 0; l < d.nh; l++) f += (uint64_t)rows * d.dim[l + 1];
  int maxd = d.D;
  for (int l = 0; l <= d.nh + 1; l++) maxd = maxd > d.dim[l] ? maxd : d.dim[l];
  f += 2ull * rows * maxd;
  return 4 * f + 8ull * d.V * d.E + 256 + 64;
}

namespace {
struct DmBufs {
  float *X, *act[2], *g0, *g1;
  long long *eacc;
  int *err;
};
DmBufs carve(const Dims &d, int rows, void *ws) {
  DmBufs b;
  float *p = static_cast<float *>(ws);
  b.X = p;
  p += (size_t)rows * d.D;
  for (int l = 0; l < 2; l++) {
    b.act[l] = p;
    if (l < d.nh) p += (size_t)rows * d.dim[l + 1];
  }
  int maxd = d.D;
  for (int l = 0; l <= d.nh + 1; l++) maxd = maxd > d.dim[l] ? maxd : d.dim[l];
  b.g0 = p;
  p += (size_t)rows * maxd;
  b.g1 = p;
  p += (size_t)rows * maxd;
  uintptr_t q = (reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255);
  b.eacc = reinterpret_cast<long long *>(q);
  b.err = reinterpret_cast<int *>(b.eacc + (size_t)d.V * d.E);
  return b;
}

hipError_t forward_into(const Dims &d, const float *W, const uint8_t *ctx, int rows, float *logits, DmBufs &b,
                        hipStream_t st) {
  const size_t nx = (size_t)rows * d.D;
  hipLaunchKernelGGL(gather_x_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, W + d.off_emb, ctx, rows,
                     d.t, d.E, d.V, b.X, b.err);
  hipError_t e = hipGetLastError();
  const float *in = b.X;
  for (int l = 0; l <= d.nh && e == hipSuccess; l++) {
    float *out = l == d.nh ? logits : b.act[l];
    e = gemm<false, false>(rows, d.dim[l + 1], d.dim[l], in, W + d.off_W[l], out, W + d.off_b[l], l < d.nh, nullptr,
                           st);
    in = out;
  }
  return e;
}
}  // namespace

hipError_t dm_forward(const Dims &d, const float *W, const uint8_t *ctx, int rows, float *logits, void *ws,
                      int *err_host, hipStream_t st) {
  DmBufs b = carve(d, rows, ws);
  hipError_t e = hipMemsetAsync(b.err, 0, sizeof(int), st);
  if (e == hipSuccess) e = forward_into(d, W, ctx, rows, logits, b, st);
  if (e == hipSuccess) e = hipMemcpyAsync(err_host, b.err, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

// grad (flat parameter layout, P floats) of sum(dlogits * logits)
hipError_t dm_backward(const Dims &d, const float *W, const uint8_t *ctx, int rows, const float *dlogits,
                       float *grad, void *ws, int *err_host, hipStream_t st) {
  DmBufs b = carve(d, rows, ws);
  hipError_t e = hipMemsetAsync(b.err, 0, sizeof(int), st);
  if (e == hipSuccess) e = hipMemsetAsync(b.eacc, 0, 8ull * d.V * d.E, st);
  // recompute the activations (the logits themselves are not needed)
  float *scratch_logits = b.g1;
  if (e == hipSuccess) e = forward_into(d, W, ctx, rows, scratch_logits, b, st);
  const float *dout = dlogits;
  float *bufs[2] = {b.g0, b.g1};
  for (int l = d.nh; l >= 0 && e == hipSuccess; l--) {
    const int Din = d.dim[l], Dout = d.dim[l + 1];
    const float *in = l == 0 ? b.X : b.act[l - 1];
    // dW_l = in^T dout, db_l = colsum(dout)
    e = gemm<true, false>(Din, Dout, rows, in, dout, grad + d.off_W[l], nullptr, false, nullptr, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(colsum_kernel, dim3((Dout + 255) / 256), dim3(256), 0, st, dout, rows, Dout,
                         grad + d.off_b[l]);
      e = hipGetLastError();
    }
    // dIn = dout W_l^T (* ReLU' of the layer input for hidden layers)
    float *din = bufs[(d.nh - l) & 1];
    if (din == dout) din = bufs[((d.nh - l) & 1) ^ 1];
    if (e == hipSuccess)
      e = gemm<false, true>(rows, Din, Dout, dout, W + d.off_W[l], din, nullptr, false, l > 0 ? in : nullptr, st);
    dout = din;
  }
  if (e == hipSuccess) {
    const size_t nx = (size_t)rows * d.D;
    hipLaunchKernelGGL(scatter_emb_kernel, dim3((unsigned)((nx + 255) / 256)), dim3(256), 0, st, dout, ctx, rows, d.t,
                       d.E, d.V, b.eacc);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    const int n = d.V * d.E;
    hipLaunchKernelGGL(fixed_to_float_kernel, dim3((n + 255) / 256), dim3(256), 0, st, b.eacc, n, grad + d.off_emb);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(err_host, b.err, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

}  // namespace pmklc
