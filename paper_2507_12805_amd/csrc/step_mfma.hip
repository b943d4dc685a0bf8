// Step kernel with the MLP on the matrix cores (CDNA4 MFMA), one hidden
// layer, FP32 accumulation.  Two precisions of the GEMM inputs:
//   MmaBf16: v_mfma_f32_16x16x32_bf16 — operands rounded to BF16 (RNE),
//   MmaF32:  v_mfma_f32_16x16x4_f32   — FP32 operands.
// Everything else (softmax, mixing weight, quantiser, coder, optimiser
// state and master weights) stays FP32; the loop around the network is the
// shared one in step_common.h.
//
// Operand layout of a 16x16 tile (lane l, r = l % 16, g = l / 16): the A
// fragment holds A[r][k0 + g*KL .. + KL-1], the B fragment B[k0 + g*KL ..][r],
// and the accumulator C[4g + i][r] for i = 0..3 (KL = 8 for BF16, 1 for
// FP32).  Per step, for bs rows (j), input width D = t*E (d), hidden H (h),
// V symbols (v):
//   F1  H1[j][h]   = ReLU(X W1 + b1)       X gathered from the embedding
//   F2  L[j][v]    = H1 W2 + b2            (dynamic model and static model)
//   B1  dpre[j][h] = (dL W2^T) * [H1 > 0]
//   B2  dW2^T[v][h] = dL^T H1               -> W2 update (4 consecutive v per lane)
//   B3  dX^T[d][j] = W1 dpre^T             -> embedding-gradient scatter
//   B4  dW1^T[h][d] = dpre^T X              -> W1 update (4 consecutive h per lane)
// Each output element is one MFMA accumulation chain over k in a fixed
// order, so encode and decode agree bit for bit; which wave computes a tile
// never changes its value.
#include "step_common.h"

namespace pmklc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct MmaF32 {
  static constexpr int KS = 4, KL = 1;
  typedef float frag;
  __device__ static frag pack(const float *v) { return v[0]; }
  __device__ static f32x4 mma(frag a, frag b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
struct MmaBf16 {
  static constexpr int KS = 32, KL = 8;
  typedef bf16x8 frag;
  __device__ static frag pack(const float *v) {
    frag f;
#pragma unroll
    for (int q = 0; q < 8; q++) f[q] = (__bf16)v[q];
    return f;
  }
  __device__ static f32x4 mma(frag a, frag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// KL consecutive floats (16-byte aligned when KL >= 4)
template <int KL>
__device__ __forceinline__ void load_run(const float *p, float *v) {
  if constexpr (KL >= 4) {
#pragma unroll
    for (int q = 0; q < KL; q += 4) {
      float4 x = *reinterpret_cast<const float4 *>(p + q);
      v[q] = x.x; v[q + 1] = x.y; v[q + 2] = x.z; v[q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < KL; q++) v[q] = p[q];
  }
}
// KL floats with a stride
template <int KL>
__device__ __forceinline__ void load_strided(const float *p, int stride, float *v) {
#pragma unroll
  for (int q = 0; q < KL; q++) v[q] = p[q * stride];
}

// Distributes `groups` groups of Mt tiles over NW waves: a wave gets whole
// groups when there are enough, else a contiguous part of one group.
template <int NW, class F>
__device__ __forceinline__ void split_groups(int groups, int Mt, int wave, F &&f) {
  if (groups >= NW) {
    for (int g = wave; g < groups; g += NW) f(g, 0, Mt);
  } else {
    const int per = NW / groups;
    const int g = wave / per, part = wave % per;
    if (g < groups) {
      const int mb = Mt * part / per, me = Mt * (part + 1) / per;
      if (mb < me) f(g, mb, me);
    }
  }
}

}  // namespace

template <int NT, class P, int MAXT>
struct NetMfma {
  static constexpr int NW = NT / 64;
  static constexpr int KS = P::KS, KL = P::KL;   // MAXT = bs / 16 row tiles
  const StepArgs &a;
  const Dims &d;
  float *emb, *embs, *h1, *hs, *lm, *lu;
  uint8_t *ring;
  long long *demb;
  int tid, lane, wave, r, g;
  PhaseClock *pc = nullptr;
  __device__ NetMfma(const StepArgs &a_, unsigned char *lds) : a(a_), d(a_.d) {
    emb = reinterpret_cast<float *>(lds + a.lay.emb);
    embs = reinterpret_cast<float *>(lds + a.lay.embs);
    h1 = reinterpret_cast<float *>(lds + a.lay.act[0]);
    hs = reinterpret_cast<float *>(lds + a.lay.dh[0]);    // static hidden; later dpre
    lm = reinterpret_cast<float *>(lds + a.lay.lm);
    lu = reinterpret_cast<float *>(lds + a.lay.lu);
    ring = lds + a.lay.ring;
    demb = reinterpret_cast<long long *>(lds + a.lay.demb);
    tid = threadIdx.x;
    lane = tid & 63;
    wave = tid >> 6;
    r = lane & 15;
    g = lane >> 4;
  }

  __device__ __forceinline__ int token(int j, int p, uint64_t i) const {
    return ring[j * d.RS + (((int)(i - (uint64_t)d.t) + p) & (d.RS - 1))];
  }

  __device__ void forward(float *W, uint64_t i, float alpha) {
    (void)alpha;
    const int bs = d.bs, H = d.H[0], V = d.V, E = d.E, D = d.D;
    const int nmod = d.static_on ? 2 : 1;
    const int Mt = bs / 16;
    // F1: X W1 + b1, ReLU; a wave owns a column tile n and all its rows
    split_groups<NW>(nmod * (H / 16), Mt, wave, [&](int grp, int mb, int me) {
      const int model = grp / (H / 16), n = grp % (H / 16);
      const float *Wm = model ? a.stat : W;
      const float *W1 = Wm + d.off_W[0];
      const float *em = model ? embs : emb;
      f32x4 acc[MAXT];
#pragma unroll
      for (int m = 0; m < MAXT; m++) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      // B fragments are fetched two k-steps ahead
      const float *wcol = W1 + 16 * n + r + (size_t)(g * KL) * H;
      float b0[KL], b1[KL];
      load_strided<KL>(wcol, H, b0);
      if (KS < D) load_strided<KL>(wcol + (size_t)KS * H, H, b1);
      auto step = [&](int k0, float *bcur) {
        const typename P::frag bf = P::pack(bcur);
        if (k0 + 2 * KS < D) load_strided<KL>(wcol + (size_t)(k0 + 2 * KS) * H, H, bcur);
        const int kk = k0 + g * KL;
        const int p = kk / E, e = kk % E;
#pragma unroll
        for (int m = 0; m < MAXT; m++) {
          if (m < mb || m >= me) continue;
          float av[KL];
          load_run<KL>(em + token(16 * m + r, p, i) * E + e, av);
          acc[m] = P::mma(P::pack(av), bf, acc[m]);
        }
      };
      int k0 = 0;
      for (; k0 + 2 * KS <= D; k0 += 2 * KS) {
        step(k0, b0);
        step(k0 + KS, b1);
      }
      if (k0 < D) step(k0, b0);
      const float bias = Wm[d.off_b[0] + 16 * n + r];
      float *out = model ? hs : h1;
#pragma unroll
      for (int m = 0; m < MAXT; m++) {
        if (m < mb || m >= me) continue;
#pragma unroll
        for (int q = 0; q < 4; q++) out[(16 * m + 4 * g + q) * H + 16 * n + r] = fmaxf(acc[m][q] + bias, 0.0f);
      }
    });
    __syncthreads();
    // F2: H1 W2 + b2 -> logits
    split_groups<NW>(nmod * (V / 16), Mt, wave, [&](int grp, int mb, int me) {
      const int model = grp / (V / 16), n = grp % (V / 16);
      const float *Wm = model ? a.stat : W;
      const float *W2 = Wm + d.off_W[1];
      const float *hin = model ? hs : h1;
      f32x4 acc[MAXT];
#pragma unroll
      for (int m = 0; m < MAXT; m++) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      const float *wcol = W2 + 16 * n + r + (size_t)(g * KL) * V;
      float b0[KL], b1[KL];
      load_strided<KL>(wcol, V, b0);
      if (KS < H) load_strided<KL>(wcol + (size_t)KS * V, V, b1);
      auto step = [&](int k0, float *bcur) {
        const typename P::frag bf = P::pack(bcur);
        if (k0 + 2 * KS < H) load_strided<KL>(wcol + (size_t)(k0 + 2 * KS) * V, V, bcur);
        const int kk = k0 + g * KL;
#pragma unroll
        for (int m = 0; m < MAXT; m++) {
          if (m < mb || m >= me) continue;
          float av[KL];
          load_run<KL>(hin + (16 * m + r) * H + kk, av);
          acc[m] = P::mma(P::pack(av), bf, acc[m]);
        }
      };
      int k0 = 0;
      for (; k0 + 2 * KS <= H; k0 += 2 * KS) {
        step(k0, b0);
        step(k0 + KS, b1);
      }
      if (k0 < H) step(k0, b0);
      const float bias = Wm[d.off_b[1] + 16 * n + r];
      float *out = model ? lu : lm;
#pragma unroll
      for (int m = 0; m < MAXT; m++) {
        if (m < mb || m >= me) continue;
#pragma unroll
        for (int q = 0; q < 4; q++) out[(16 * m + 4 * g + q) * d.VS + 16 * n + r] = acc[m][q] + bias;
      }
    });
    __syncthreads();
  }

  __device__ void backward(float *W, float *M, float *Vs, uint64_t i, const Opt &opt) {
    const int bs = d.bs, H = d.H[0], V = d.V, E = d.E, D = d.D;
    const int Mt = bs / 16;
    float *W1 = W + d.off_W[0], *W2 = W + d.off_W[1];
    float *dpre = hs;
    // B1: dpre = (dL W2^T) * [H1 > 0]
    split_groups<NW>(H / 16, Mt, wave, [&](int n, int mb, int me) {
      f32x4 acc[MAXT];
#pragma unroll
      for (int m = 0; m < MAXT; m++) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      for (int k0 = 0; k0 < V; k0 += KS) {
        const int kk = k0 + g * KL;
        float bv[KL];
        load_run<KL>(W2 + (size_t)(16 * n + r) * V + kk, bv);
        const typename P::frag bf = P::pack(bv);
#pragma unroll
        for (int m = 0; m < MAXT; m++) {
          if (m < mb || m >= me) continue;
          float av[KL];
          load_run<KL>(lm + (16 * m + r) * d.VS + kk, av);
          acc[m] = P::mma(P::pack(av), bf, acc[m]);
        }
      }
#pragma unroll
      for (int m = 0; m < MAXT; m++) {
        if (m < mb || m >= me) continue;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int idx = (16 * m + 4 * g + q) * H + 16 * n + r;
          dpre[idx] = h1[idx] > 0.0f ? acc[m][q] : 0.0f;
        }
      }
    });
    __syncthreads();
    pc->mark(8);
    // B2: dW2^T = dL^T H1 -> W2 update; db2.   B3: dX^T = W1 dpre^T -> embedding scatter.
    float *M2 = M ? M + d.off_W[1] : nullptr, *V2 = Vs ? Vs + d.off_W[1] : nullptr;
    split_groups<NW>(H / 16, V / 16, wave, [&](int n, int mb, int me) {
      f32x4 acc[MAXT];
#pragma unroll
      for (int m = 0; m < MAXT; m++) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      for (int k0 = 0; k0 < bs; k0 += KS) {
        const int kk = k0 + g * KL;
        float bv[KL];
        load_strided<KL>(h1 + kk * H + 16 * n + r, H, bv);
        const typename P::frag bf = P::pack(bv);
#pragma unroll
        for (int m = 0; m < MAXT; m++) {
          if (m < mb || m >= me) continue;
          float av[KL];
          load_strided<KL>(lm + kk * d.VS + 16 * m + r, d.VS, av);
          acc[m] = P::mma(P::pack(av), bf, acc[m]);
        }
      }
#pragma unroll
      for (int m = 0; m < MAXT; m++) {
        if (m < mb || m >= me) continue;
        const size_t idx = (size_t)(16 * n + r) * V + 16 * m + 4 * g;   // W2[h][v .. v+3]
        float4 w = *reinterpret_cast<float4 *>(W2 + idx);
        float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int q = 0; q < 4; q++)
          wv[q] = wv[q] - opt_delta(opt, acc[m][q], M2 ? M2 + idx + q : nullptr, V2 ? V2 + idx + q : nullptr);
        *reinterpret_cast<float4 *>(W2 + idx) = make_float4(wv[0], wv[1], wv[2], wv[3]);
      }
    });
    for (int v = tid; v < V; v += NT) {
      float gsum = 0.0f;
      for (int j = 0; j < bs; j++) gsum += lm[j * d.VS + v];
      const int bi = d.off_b[1] + v;
      W[bi] = W[bi] - opt_delta(opt, gsum, M ? M + bi : nullptr, Vs ? Vs + bi : nullptr);
    }
    // B3: rows d of W1 (A operand, contiguous h), columns j from dpre
    for (int mt = wave; mt < D / 16; mt += NW) {
      f32x4 acc[MAXT];
#pragma unroll
      for (int n = 0; n < MAXT; n++) acc[n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      const float *wrow = W1 + (size_t)(16 * mt + r) * H + g * KL;
      float a0[KL], a1[KL];
      load_run<KL>(wrow, a0);
      if (KS < H) load_run<KL>(wrow + KS, a1);
      auto step = [&](int k0, float *acur) {
        const typename P::frag af = P::pack(acur);
        if (k0 + 2 * KS < H) load_run<KL>(wrow + k0 + 2 * KS, acur);
        const int kk = k0 + g * KL;
#pragma unroll
        for (int n = 0; n < MAXT; n++) {
          if (n >= Mt) continue;
          float bv[KL];
          load_run<KL>(dpre + (16 * n + r) * H + kk, bv);
          acc[n] = P::mma(af, P::pack(bv), acc[n]);
        }
      };
      int k0 = 0;
      for (; k0 + 2 * KS <= H; k0 += 2 * KS) {
        step(k0, a0);
        step(k0 + KS, a1);
      }
      if (k0 < H) step(k0, a0);
#pragma unroll
      for (int n = 0; n < MAXT; n++) {
        if (n >= Mt) continue;
        const int j = 16 * n + r;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int dd = 16 * mt + 4 * g + q, p = dd / E, e = dd % E;
          atomicAdd(reinterpret_cast<unsigned long long *>(demb + token(j, p, i) * d.ES + e),
                    (unsigned long long)to_fixed(acc[n][q]));
        }
      }
    }
    __syncthreads();
    pc->mark(9);
    // B4: dW1^T = dpre^T X -> W1 update (a wave owns column tiles over d); db1
    float *M1 = M ? M + d.off_W[0] : nullptr, *V1 = Vs ? Vs + d.off_W[0] : nullptr;
    const int Ht = H / 16;
    for (int nt = wave; nt < D / 16; nt += NW) {
      const int dd = 16 * nt + r, p = dd / E, e = dd % E;
      for (int m0 = 0; m0 < Ht; m0 += MAXT) {
        f32x4 acc[MAXT];
#pragma unroll
        for (int m = 0; m < MAXT; m++) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int k0 = 0; k0 < bs; k0 += KS) {
          const int kk = k0 + g * KL;
          float bv[KL];
#pragma unroll
          for (int q = 0; q < KL; q++) bv[q] = emb[token(kk + q, p, i) * E + e];
          const typename P::frag bf = P::pack(bv);
#pragma unroll
          for (int m = 0; m < MAXT; m++) {
            if (m0 + m >= Ht) continue;
            float av[KL];
            load_strided<KL>(dpre + kk * H + 16 * (m0 + m) + r, H, av);
            acc[m] = P::mma(P::pack(av), bf, acc[m]);
          }
        }
#pragma unroll
        for (int m = 0; m < MAXT; m++) {
          if (m0 + m >= Ht) continue;
          const size_t idx = (size_t)dd * H + 16 * (m0 + m) + 4 * g;   // W1[d][h .. h+3]
          float4 w = *reinterpret_cast<float4 *>(W1 + idx);
          float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int q = 0; q < 4; q++)
            wv[q] = wv[q] - opt_delta(opt, acc[m][q], M1 ? M1 + idx + q : nullptr, V1 ? V1 + idx + q : nullptr);
          *reinterpret_cast<float4 *>(W1 + idx) = make_float4(wv[0], wv[1], wv[2], wv[3]);
        }
      }
    }
    for (int h = tid; h < H; h += NT) {
      float gsum = 0.0f;
      for (int j = 0; j < bs; j++) gsum += dpre[j * H + h];
      const int bi = d.off_b[0] + h;
      W[bi] = W[bi] - opt_delta(opt, gsum, M ? M + bi : nullptr, Vs ? Vs + bi : nullptr);
    }
    __syncthreads();
    pc->mark(10);
  }
};

template <int NT, class P, int MT>
__global__ __launch_bounds__(NT) void step_mfma_kernel(const StepArgs *__restrict__ args) {
  extern __shared__ __align__(16) unsigned char lds[];
  const StepArgs &a = *args;
  NetMfma<NT, P, MT> net(a, lds);
  run_blocks<NT>(a, lds, net);
}

template <int NT, class P, int MT>
hipError_t launch_one(const StepArgs *a_dev, int grid, size_t lds, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_mfma_kernel<NT, P, MT>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((step_mfma_kernel<NT, P, MT>), dim3(grid), dim3(NT), lds, st, a_dev);
  return hipGetLastError();
}

template <int NT>
hipError_t launch_nt(const StepArgs *a_dev, int grid, bool bf16, int mt, size_t lds, hipStream_t st) {
  if (mt == 2) return bf16 ? launch_one<NT, MmaBf16, 2>(a_dev, grid, lds, st) : launch_one<NT, MmaF32, 2>(a_dev, grid, lds, st);
  if (mt == 4) return bf16 ? launch_one<NT, MmaBf16, 4>(a_dev, grid, lds, st) : launch_one<NT, MmaF32, 4>(a_dev, grid, lds, st);
  if (mt == 6) return bf16 ? launch_one<NT, MmaBf16, 6>(a_dev, grid, lds, st) : launch_one<NT, MmaF32, 6>(a_dev, grid, lds, st);
  if (mt == 8) return bf16 ? launch_one<NT, MmaBf16, 8>(a_dev, grid, lds, st) : launch_one<NT, MmaF32, 8>(a_dev, grid, lds, st);
  return hipErrorInvalidValue;
}

// a_dev: a device copy of `a` (kernel arguments are read through it).
// nt: 256 or 512 threads per workgroup; the choice never changes a value.
hipError_t launch_step_mfma(const StepArgs &a, const StepArgs *a_dev, int grid, bool bf16, int nt, hipStream_t st) {
  const size_t lds = (size_t)a.lay.total;
  const int mt = a.d.bs / 16;
  if (nt == 256) return launch_nt<256>(a_dev, grid, bf16, mt, lds, st);
  if (nt == 512) return launch_nt<512>(a_dev, grid, bf16, mt, lds, st);
  return hipErrorInvalidValue;
}

}  // namespace pmklc
