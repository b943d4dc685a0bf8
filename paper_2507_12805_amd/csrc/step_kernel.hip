// Per-block online learning + arithmetic coding: the PMKLC model loop,
// generic FP32 variant (any shape the LDS holds).
//
// One workgroup owns one data block for its whole life (Sec. 4.3: blocks are
// independent apart from step-wise model passing) and loops over the
// block's steps inside the kernel, so no launch or host round trip sits
// between steps.  A step i handles token i of every one of the bs segments
// of the block (one row per segment):
//   forward (Sec. 2 step (3)): context of the previous t tokens -> embedding
//     -> MLP -> logits L^m; with the static model on, its logits L^u too;
//   mixer (Eq. 1): z = alpha*L^u + (1-alpha)*L^m (or z = L^m), P = softmax(z);
//   quantiser: integer CDF with total 2^16 (f = 1 + floor(p*(2^16-V)),
//     residual to the most probable symbol, lowest index on ties);
//   coder: one Witten-Neal-Cleary arithmetic coder per segment (lane j);
//   backward (Sec. 2 step (4), Eq. 2): mean cross-entropy over the bs rows,
//     back-propagated through the MLP, the embedding and alpha; then SGD or
//     Adam on the FP32 parameters.
// The first t steps of every segment use the uniform distribution and do
// not train (Sec. 2).  The loop itself lives in step_common.h; this file
// supplies the MLP as per-thread 4x4 FMA tiles.
//
// Numerics are fixed by construction so that encode and decode (the same
// kernel, selected by a runtime flag) produce bit-identical probabilities:
// every dot product is a sequential FMA chain in a fixed k order inside one
// thread, wave reductions are xor butterflies (commutative at every level,
// so all lanes agree), and the embedding gradient, whose scatter has
// data-dependent collisions, is summed in 64-bit fixed point with integer
// atomics, which are order-independent.  Launch shape (threads, grid) never
// changes any value.
#include "step_common.h"

namespace pmklc {

namespace {

// ------------------------------------------------------------ GEMM tiles
struct Ctx {   // context-window gather for the first layer
  const uint8_t *ring;
  int rows, mask, base;   // ring positions are rows bytes apart (one byte per row); RS-1; (i - t)
  const float *emb;
  int E, EP;            // embedding width, LDS row pitch
};

// out[j][o] = b[o] + sum_d in[j][d] W[d][o]   (optionally ReLU)
// layer 0 gathers in[j][p*E+e] = emb[ring[j][(base+p)&mask]][e]
__device__ __forceinline__ void fwd_tile(int r0, int c0, int Din, int Dout, const float *__restrict__ W,
                                         const float *__restrict__ b, const float *in, const Ctx *g, float *out,
                                         int ldo, bool relu) {
  float acc[4][4];
  float4 bb = *reinterpret_cast<const float4 *>(b + c0);
#pragma unroll
  for (int r = 0; r < 4; r++) { acc[r][0] = bb.x; acc[r][1] = bb.y; acc[r][2] = bb.z; acc[r][3] = bb.w; }
  if (g) {
    const int t = Din / g->E;
    for (int p = 0; p < t; p++) {
      int tk[4];
#pragma unroll
      for (int r = 0; r < 4; r++) tk[r] = g->ring[((g->base + p) & g->mask) * g->rows + (r0 + r)];
      for (int e = 0; e < g->E; e += 4) {
        float4 a[4], w[4];
#pragma unroll
        for (int r = 0; r < 4; r++) a[r] = *reinterpret_cast<const float4 *>(g->emb + tk[r] * g->EP + e);
#pragma unroll
        for (int q = 0; q < 4; q++) w[q] = *reinterpret_cast<const float4 *>(W + (size_t)(p * g->E + e + q) * Dout + c0);
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const float av[4] = {a[r].x, a[r].y, a[r].z, a[r].w};
#pragma unroll
          for (int q = 0; q < 4; q++) {
            acc[r][0] = fmaf(av[q], w[q].x, acc[r][0]);
            acc[r][1] = fmaf(av[q], w[q].y, acc[r][1]);
            acc[r][2] = fmaf(av[q], w[q].z, acc[r][2]);
            acc[r][3] = fmaf(av[q], w[q].w, acc[r][3]);
          }
        }
      }
    }
  } else {
    for (int d = 0; d < Din; d += 4) {
      float4 a[4], w[4];
#pragma unroll
      for (int r = 0; r < 4; r++) a[r] = *reinterpret_cast<const float4 *>(in + (r0 + r) * Din + d);
#pragma unroll
      for (int q = 0; q < 4; q++) w[q] = *reinterpret_cast<const float4 *>(W + (size_t)(d + q) * Dout + c0);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const float av[4] = {a[r].x, a[r].y, a[r].z, a[r].w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
          acc[r][0] = fmaf(av[q], w[q].x, acc[r][0]);
          acc[r][1] = fmaf(av[q], w[q].y, acc[r][1]);
          acc[r][2] = fmaf(av[q], w[q].z, acc[r][2]);
          acc[r][3] = fmaf(av[q], w[q].w, acc[r][3]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < 4; r++) {
    float4 o;
    o.x = relu ? fmaxf(acc[r][0], 0.0f) : acc[r][0];
    o.y = relu ? fmaxf(acc[r][1], 0.0f) : acc[r][1];
    o.z = relu ? fmaxf(acc[r][2], 0.0f) : acc[r][2];
    o.w = relu ? fmaxf(acc[r][3], 0.0f) : acc[r][3];
    *reinterpret_cast<float4 *>(out + (r0 + r) * ldo + c0) = o;
  }
}

// dIn[j][d] = sum_o dOut[j][o] W[d][o]; rows j0..j0+3, columns d0..d0+3
__device__ __forceinline__ void bwd_in_tile(int r0, int d0, int Dout, const float *__restrict__ W,
                                            const float *dOut, int ldo, float acc[4][4]) {
#pragma unroll
  for (int r = 0; r < 4; r++)
#pragma unroll
    for (int q = 0; q < 4; q++) acc[r][q] = 0.0f;
  for (int o = 0; o < Dout; o += 4) {
    float4 a[4], w[4];
#pragma unroll
    for (int r = 0; r < 4; r++) a[r] = *reinterpret_cast<const float4 *>(dOut + (r0 + r) * ldo + o);
#pragma unroll
    for (int q = 0; q < 4; q++) w[q] = *reinterpret_cast<const float4 *>(W + (size_t)(d0 + q) * Dout + o);
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        acc[r][q] = fmaf(a[r].x, w[q].x, acc[r][q]);
        acc[r][q] = fmaf(a[r].y, w[q].y, acc[r][q]);
        acc[r][q] = fmaf(a[r].z, w[q].z, acc[r][q]);
        acc[r][q] = fmaf(a[r].w, w[q].w, acc[r][q]);
      }
  }
}

// dW[d][o] = sum_j In[j][d] dOut[j][o], then the optimiser update of W.
__device__ __forceinline__ void bwd_w_tile(int d0, int o0, int rows, int Dout, float *W, float *M, float *Vv,
                                           const float *in, int Din, const Ctx *g, const float *dOut, int ldo,
                                           const Opt &opt) {
  float acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; q++)
#pragma unroll
    for (int c = 0; c < 4; c++) acc[q][c] = 0.0f;
  int p = 0, e = 0;
  if (g) { p = d0 / g->E; e = d0 % g->E; }
  for (int j = 0; j < rows; j++) {
    float4 a;
    if (g) {
      int tk = g->ring[((g->base + p) & g->mask) * g->rows + j];
      a = *reinterpret_cast<const float4 *>(g->emb + tk * g->EP + e);
    } else {
      a = *reinterpret_cast<const float4 *>(in + j * Din + d0);
    }
    float4 bv = *reinterpret_cast<const float4 *>(dOut + j * ldo + o0);
    const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int q = 0; q < 4; q++) {
      acc[q][0] = fmaf(av[q], bv.x, acc[q][0]);
      acc[q][1] = fmaf(av[q], bv.y, acc[q][1]);
      acc[q][2] = fmaf(av[q], bv.z, acc[q][2]);
      acc[q][3] = fmaf(av[q], bv.w, acc[q][3]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; q++) {
    size_t idx = (size_t)(d0 + q) * Dout + o0;
    float4 w = *reinterpret_cast<float4 *>(W + idx);
    float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int c = 0; c < 4; c++) wv[c] = wv[c] - opt_delta(opt, acc[q][c], M ? M + idx + c : nullptr, Vv ? Vv + idx + c : nullptr);
    *reinterpret_cast<float4 *>(W + idx) = make_float4(wv[0], wv[1], wv[2], wv[3]);
  }
}


}  // namespace

template <int NT>
struct NetGeneric {
  static constexpr bool kOnChip = false;
  static constexpr int kSpl = 0;   // softmax symbols per lane: chosen at run time
  const StepArgs &a;
  const Dims &d;
  float *emb, *embs, *act[2], *lm, *lu, *dh[2];
  uint8_t *ring;
  long long *demb;
  int tid;
  PhaseClock *pc = nullptr;
  __device__ NetGeneric(const StepArgs &a_, unsigned char *lds) : a(a_), d(a_.d) {
    emb = reinterpret_cast<float *>(lds + a.lay.emb);
    embs = reinterpret_cast<float *>(lds + a.lay.embs);
    if (a.lay.act_global) {
      // activations too large for the LDS live in this workgroup's slab
      float *slab = a.act_scratch + (size_t)blockIdx.x * a.lay.act_slot;
      act[0] = slab + a.lay.act[0];
      act[1] = slab + a.lay.act[1];
      dh[0] = slab + a.lay.dh[0];
      dh[1] = slab + a.lay.dh[1];
    } else {
      act[0] = reinterpret_cast<float *>(lds + a.lay.act[0]);
      act[1] = reinterpret_cast<float *>(lds + a.lay.act[1]);
      dh[0] = reinterpret_cast<float *>(lds + a.lay.dh[0]);
      dh[1] = reinterpret_cast<float *>(lds + a.lay.dh[1]);
    }
    lm = reinterpret_cast<float *>(lds + a.lay.lm);
    lu = reinterpret_cast<float *>(lds + a.lay.lu);
    ring = lds + a.lay.ring;
    demb = reinterpret_cast<long long *>(lds + a.lay.demb);
    tid = threadIdx.x;
  }

  __device__ void begin_block(const float *) {}

  // forward, layer by layer; DM and static tiles share one pass
  __device__ void forward(float *W, uint64_t i, float alpha) {
    (void)alpha;
    const int bs = d.bs, nh = d.nh, mask = d.RS - 1, t = d.t, E = d.E;
    Ctx g{ring, bs, mask, (int)(i - (uint64_t)t), emb, E, d.EP};
    Ctx gs{ring, bs, mask, (int)(i - (uint64_t)t), embs, E, d.EP};
    for (int l = 0; l <= nh; l++) {
      const int Din = d.dim[l], Dout = d.dim[l + 1];
      const bool last = (l == nh);
      const int tiles = (bs / 4) * (Dout / 4);
      const int total = d.static_on ? 2 * tiles : tiles;
      for (int tile = tid; tile < total; tile += NT) {
        const bool st = tile >= tiles;
        const int tt = st ? tile - tiles : tile;
        const int r0 = (tt / (Dout / 4)) * 4, c0 = (tt % (Dout / 4)) * 4;
        const float *Wp = st ? a.stat : W;
        const float *in = l == 0 ? nullptr : (st ? dh[(l - 1) & 1] : act[l - 1]);
        float *out = last ? (st ? lu : lm) : (st ? dh[l & 1] : act[l]);
        fwd_tile(r0, c0, Din, Dout, Wp + d.off_W[l], Wp + d.off_b[l], in, l == 0 ? (st ? &gs : &g) : nullptr, out,
                 last ? d.VS : Dout, !last);
      }
      __syncthreads();
    }
  }

  // lm holds dL/dL^m; gradients of every layer with the old weights, then
  // the optimiser update, layer by layer from the output down
  __device__ void backward(float *W, float *M, float *Vs, uint64_t i, const Opt &opt) {
    const int bs = d.bs, nh = d.nh, mask = d.RS - 1, t = d.t, E = d.E;
    const Ctx g{ring, bs, mask, (int)(i - (uint64_t)t), emb, E, d.EP};
    const float *dout = lm;
    int ldo = d.VS;
    for (int l = nh; l >= 0; l--) {
      const int Din = d.dim[l], Dout = d.dim[l + 1];
      float *Wl = W + d.off_W[l];
      float *dIn = dh[(nh - l) & 1];
      // (a) gradient of this layer's input, with the old weights
      const int tiles_a = (bs / 4) * (Din / 4);
      for (int tile = tid; tile < tiles_a; tile += NT) {
        const int r0 = (tile / (Din / 4)) * 4, c0 = (tile % (Din / 4)) * 4;
        float acc[4][4];
        bwd_in_tile(r0, c0, Dout, Wl, dout, ldo, acc);
        if (l > 0) {
          const float *ain = act[l - 1];
#pragma unroll
          for (int r = 0; r < 4; r++) {
            float4 o;
            o.x = ain[(r0 + r) * Din + c0 + 0] > 0.0f ? acc[r][0] : 0.0f;
            o.y = ain[(r0 + r) * Din + c0 + 1] > 0.0f ? acc[r][1] : 0.0f;
            o.z = ain[(r0 + r) * Din + c0 + 2] > 0.0f ? acc[r][2] : 0.0f;
            o.w = ain[(r0 + r) * Din + c0 + 3] > 0.0f ? acc[r][3] : 0.0f;
            *reinterpret_cast<float4 *>(dIn + (r0 + r) * Din + c0) = o;
          }
        } else {
          // embedding rows: d = p*E + e of row j scatters into emb[token]
#pragma unroll
          for (int r = 0; r < 4; r++) {
            const int j = r0 + r;
#pragma unroll
            for (int q = 0; q < 4; q++) {
              const int dd = c0 + q, p = dd / E, e = dd % E;
              const int tk = ring[((((int)(i - (uint64_t)t) + p) & mask)) * bs + j];
              atomicAdd(reinterpret_cast<unsigned long long *>(demb + tk * d.ES + e),
                        (unsigned long long)to_fixed(acc[r][q]));
            }
          }
        }
      }
      __syncthreads();
      // (b) weight gradient and update
      const int tiles_b = (Din / 4) * (Dout / 4);
      float *Ml = M ? M + d.off_W[l] : nullptr;
      float *Vl = Vs ? Vs + d.off_W[l] : nullptr;
      for (int tile = tid; tile < tiles_b; tile += NT) {
        const int d0 = (tile / (Dout / 4)) * 4, o0 = (tile % (Dout / 4)) * 4;
        bwd_w_tile(d0, o0, bs, Dout, Wl, Ml, Vl, l == 0 ? nullptr : act[l - 1], Din, l == 0 ? &g : nullptr, dout, ldo,
                   opt);
      }
      for (int o = tid; o < Dout; o += NT) {
        float gsum = 0.0f;
        for (int j = 0; j < bs; j++) gsum += dout[j * ldo + o];
        const int bi = d.off_b[l] + o;
        W[bi] = W[bi] - opt_delta(opt, gsum, M ? M + bi : nullptr, Vs ? Vs + bi : nullptr);
      }
      dout = dIn;
      ldo = Din;
    }
    __syncthreads();
  }
};

template <int NT>
__global__ __launch_bounds__(NT) void step_kernel(StepArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  NetGeneric<NT> net(a, lds);
  run_blocks<NT>(a, lds, net);
}

hipError_t launch_step(const StepArgs &a, int grid, int nt, hipStream_t st) {
  size_t lds = (size_t)a.lay.total;
  if (nt == 256) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_kernel<256>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(step_kernel<256>, dim3(grid), dim3(256), lds, st, a);
  } else if (nt == 512) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_kernel<512>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(step_kernel<512>, dim3(grid), dim3(512), lds, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// --------------------------------------------------------- parameter init
// SplitMix64 (Steele, Lea, Flood 2014) in counter form: draw i is
// mix(seed + (i+1) * 0x9E3779B97F4A7C15).  w_i = fp32((2u - 1) * a) with
// u = top 24 bits / 2^24 and a the tensor's scale (1 for the embedding,
// 1/sqrt(fan_in) for linear weights and biases, computed on the host).
struct InitScales {
  int n_tensors;
  int end[2 * kMaxLayers + 1];    // exclusive end offsets, in parameter order
  double a[2 * kMaxLayers + 1];
};

__global__ void init_params_kernel(uint64_t seed, int P, InitScales sc, float *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > P) return;
  if (i == P) { out[i] = 0.0f; return; }   // mixing weight a = 0, alpha = 1/2
  uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  double u = (double)(z >> 40) * (1.0 / 16777216.0);
  double a = sc.a[sc.n_tensors - 1];
  for (int q = 0; q < sc.n_tensors; q++)
    if (i < sc.end[q]) { a = sc.a[q]; break; }
  out[i] = (float)((2.0 * u - 1.0) * a);
}

// the same draws for a model given as consecutive tensors (exclusive end
// offsets) with their scales (at most 2 kMaxLayers + 1 tensors)
hipError_t launch_init_scaled(uint64_t seed, int P, int n_tensors, const int *end, const double *scale, float *out,
                              hipStream_t st) {
  InitScales sc;
  if (n_tensors < 1 || n_tensors > 2 * kMaxLayers + 1) return hipErrorInvalidValue;
  sc.n_tensors = n_tensors;
  for (int q = 0; q < n_tensors; q++) {
    sc.end[q] = end[q];
    sc.a[q] = scale[q];
  }
  hipLaunchKernelGGL(init_params_kernel, dim3((P + 1 + 255) / 256), dim3(256), 0, st, seed, P, sc, out);
  return hipGetLastError();
}

hipError_t launch_init_params(const Dims &d, uint64_t seed, float *out, hipStream_t st) {
  InitScales sc;
  sc.n_tensors = 0;
  sc.end[sc.n_tensors] = d.off_emb + d.V * d.E;
  sc.a[sc.n_tensors++] = 1.0;
  for (int l = 0; l <= d.nh; l++) {
    double a = 1.0 / sqrt((double)d.dim[l]);
    sc.end[sc.n_tensors] = d.off_W[l] + d.dim[l] * d.dim[l + 1];
    sc.a[sc.n_tensors++] = a;
    sc.end[sc.n_tensors] = d.off_b[l] + d.dim[l + 1];
    sc.a[sc.n_tensors++] = a;
  }
  int n = d.P + 1;
  hipLaunchKernelGGL(init_params_kernel, dim3((n + 255) / 256), dim3(256), 0, st, seed, d.P, sc, out);
  return hipGetLastError();
}

// ------------------------------------------------------- test exports
// the step kernels' quantiser (G lanes per row, as in the step loop)
__global__ void quantise_kernel(const float *P, uint32_t rows, uint32_t V, uint32_t *cdf) {
  const int spl = row_spl((int)V), G = (int)V / spl;
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t row = gid / (uint64_t)G;
  if (row >= rows) return;   // whole groups leave together (G divides the block)
  row_quantise_group(P + row * V, (int)V, spl, G, (int)(gid % (uint64_t)G), cdf + row * (V + 1));
}

hipError_t launch_quantise(const float *P, uint32_t rows, uint32_t V, uint32_t *cdf, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  const uint64_t G = V / (uint64_t)(V >= 32 ? V / 8 : 4);
  const uint64_t threads = (uint64_t)rows * G;
  hipLaunchKernelGGL(quantise_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, P, rows, V, cdf);
  return hipGetLastError();
}

__global__ void wnc_encode_kernel(const uint32_t *lo, const uint32_t *hi, uint64_t m, uint32_t *out,
                                  uint32_t cap, uint64_t *nbits, int *err) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Enc e;
  enc_init(e);
  int ovf = 0;
  gu32 *o = (gu32 *)out;
  for (uint64_t i = 0; i < m; i++) enc_symbol(e, o, cap, lo[i], hi[i], ovf);
  enc_finish(e, o, cap, ovf);
  *nbits = e.nbits;
  if (ovf) *err = 2;
}

hipError_t launch_wnc_encode(const uint32_t *lo, const uint32_t *hi, uint64_t m, uint32_t *out_words,
                             uint32_t cap_words, uint64_t *nbits_dev, int *err, hipStream_t st) {
  hipLaunchKernelGGL(wnc_encode_kernel, dim3(1), dim3(64), 0, st, lo, hi, m, out_words, cap_words, nbits_dev, err);
  return hipGetLastError();
}

__global__ void wnc_decode_kernel(const uint32_t *words, uint32_t nwords, const uint32_t *cdfs, uint32_t V,
                                  uint64_t m, uint32_t *sym) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Dec d;
  const gu32 *w = (const gu32 *)words;
  dec_init(d, w, nwords);
  for (uint64_t i = 0; i < m; i++) {
    const uint32_t *c = cdfs + i * (V + 1);
    sym[i] = (uint32_t)dec_symbol(d, w, nwords, (int)V, [&](int s) { return c[s]; });
  }
}

hipError_t launch_wnc_decode(const uint32_t *words, uint32_t nwords, const uint32_t *cdfs, uint32_t V,
                             uint64_t m, uint32_t *sym, hipStream_t st) {
  hipLaunchKernelGGL(wnc_decode_kernel, dim3(1), dim3(64), 0, st, words, nwords, cdfs, V, m, sym);
  return hipGetLastError();
}

}  // namespace pmklc
