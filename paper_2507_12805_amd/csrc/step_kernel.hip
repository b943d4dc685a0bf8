// Per-block online learning + arithmetic coding: the PMKLC model loop.
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
// not train (Sec. 2).
//
// Numerics are fixed by construction so that encode and decode (the same
// kernel, selected by a runtime flag) produce bit-identical probabilities:
// every dot product is a sequential FMA chain in a fixed k order inside one
// thread, wave reductions are xor butterflies (commutative at every level,
// so all lanes agree), and the embedding gradient, whose scatter has
// data-dependent collisions, is summed in 64-bit fixed point with integer
// atomics, which are order-independent.  Launch shape (threads, grid) never
// changes any value.
#include "pmklc_internal.h"

namespace pmklc {

namespace {

constexpr uint32_t kHalf = 0x80000000u;
constexpr uint32_t kQuarter = 0x40000000u;

__device__ __forceinline__ float wave_max(float x) {
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o));
  return x;
}
__device__ __forceinline__ float wave_sum(float x) {
  for (int o = 32; o > 0; o >>= 1) x = x + __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ int wave_sum_i(int x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ void wave_argmax(float &v, int &i) {
  for (int o = 32; o > 0; o >>= 1) {
    float ov = __shfl_xor(v, o);
    int oi = __shfl_xor(i, o);
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
  }
}
// inclusive scan of ints over the 64 lanes (lane order)
__device__ __forceinline__ int wave_scan_incl(int x, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  return x;
}

// ---------------------------------------------------------------- coder
struct Enc {
  uint32_t low, high, pending, widx;
  uint64_t buf, nbits;
  int nbuf;
};
__device__ __forceinline__ void enc_init(Enc &e) {
  e.low = 0; e.high = 0xFFFFFFFFu; e.pending = 0; e.widx = 0; e.buf = 0; e.nbits = 0; e.nbuf = 0;
}
__device__ __forceinline__ void enc_emit(Enc &e, uint32_t *slot, uint32_t cap, uint32_t bits, int n, int &ovf) {
  e.buf = (e.buf << n) | (uint64_t)bits;
  e.nbuf += n;
  e.nbits += (uint64_t)n;
  if (e.nbuf >= 32) {
    e.nbuf -= 32;
    uint32_t w = (uint32_t)(e.buf >> e.nbuf);
    if (e.widx < cap) slot[e.widx] = __builtin_bswap32(w);
    else ovf = 1;
    e.widx++;
    e.buf &= (1ull << e.nbuf) - 1ull;
  }
}
__device__ __forceinline__ void enc_run(Enc &e, uint32_t *slot, uint32_t cap, int bit, uint32_t count, int &ovf) {
  while (count) {
    int n = count > 32u ? 32 : (int)count;
    uint32_t bits = bit ? (n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)) : 0u;
    enc_emit(e, slot, cap, bits, n, ovf);
    count -= (uint32_t)n;
  }
}
__device__ __forceinline__ void enc_symbol(Enc &e, uint32_t *slot, uint32_t cap, uint32_t lo, uint32_t hi, int &ovf) {
  uint64_t r = (uint64_t)e.high - e.low + 1u;
  uint32_t l0 = e.low;
  e.high = l0 + (uint32_t)((r * hi) >> kTotalBits) - 1u;
  e.low = l0 + (uint32_t)((r * lo) >> kTotalBits);
  for (;;) {
    if (e.high < kHalf) {
      enc_emit(e, slot, cap, 0u, 1, ovf);
      enc_run(e, slot, cap, 1, e.pending, ovf);
      e.pending = 0;
    } else if (e.low >= kHalf) {
      enc_emit(e, slot, cap, 1u, 1, ovf);
      enc_run(e, slot, cap, 0, e.pending, ovf);
      e.pending = 0;
      e.low -= kHalf;
      e.high -= kHalf;
    } else if (e.low >= kQuarter && e.high < 3u * kQuarter) {
      e.pending++;
      e.low -= kQuarter;
      e.high -= kQuarter;
    } else {
      break;
    }
    e.low <<= 1;
    e.high = (e.high << 1) | 1u;
  }
}
__device__ __forceinline__ void enc_finish(Enc &e, uint32_t *slot, uint32_t cap, int &ovf) {
  e.pending++;
  int bit = e.low < kQuarter ? 0 : 1;
  enc_emit(e, slot, cap, (uint32_t)bit, 1, ovf);
  enc_run(e, slot, cap, !bit, e.pending, ovf);
  e.pending = 0;
  if (e.nbuf > 0) {
    uint32_t w = (uint32_t)(e.buf << (32 - e.nbuf));
    if (e.widx < cap) slot[e.widx] = __builtin_bswap32(w);
    else ovf = 1;
    e.widx++;
    e.nbuf = 0;
    e.buf = 0;
  }
}

struct Dec {
  uint32_t low, high, value, widx;
  uint32_t buf;
  int nbuf;
};
__device__ __forceinline__ int dec_bit(Dec &d, const uint32_t *w, uint32_t nw) {
  if (d.nbuf == 0) {
    d.buf = d.widx < nw ? __builtin_bswap32(w[d.widx]) : 0u;
    d.widx++;
    d.nbuf = 32;
  }
  d.nbuf--;
  return (int)((d.buf >> d.nbuf) & 1u);
}
__device__ __forceinline__ void dec_init(Dec &d, const uint32_t *w, uint32_t nw) {
  d.low = 0; d.high = 0xFFFFFFFFu; d.value = 0; d.widx = 0; d.buf = 0; d.nbuf = 0;
  for (int i = 0; i < 32; i++) d.value = (d.value << 1) | (uint32_t)dec_bit(d, w, nw);
}
// cum(s) is the cumulative count below symbol s (cum(0) = 0, cum(V) = 2^16).
template <class Cum>
__device__ __forceinline__ int dec_symbol(Dec &d, const uint32_t *w, uint32_t nw, int V, Cum cum) {
  uint64_t r = (uint64_t)d.high - d.low + 1u;
  uint32_t target = d.value - d.low;
  int a = 0, b = V;
  while (b - a > 1) {
    int m = (a + b) >> 1;
    if ((uint32_t)((r * cum(m)) >> kTotalBits) <= target) a = m;
    else b = m;
  }
  uint32_t l0 = d.low;
  d.high = l0 + (uint32_t)((r * cum(a + 1)) >> kTotalBits) - 1u;
  d.low = l0 + (uint32_t)((r * cum(a)) >> kTotalBits);
  for (;;) {
    if (d.high < kHalf) {
    } else if (d.low >= kHalf) {
      d.low -= kHalf; d.high -= kHalf; d.value -= kHalf;
    } else if (d.low >= kQuarter && d.high < 3u * kQuarter) {
      d.low -= kQuarter; d.high -= kQuarter; d.value -= kQuarter;
    } else {
      break;
    }
    d.low <<= 1;
    d.high = (d.high << 1) | 1u;
    d.value = (d.value << 1) | (uint32_t)dec_bit(d, w, nw);
  }
  return a;
}

// -------------------------------------------------- softmax + quantiser
// One wave turns the V logits of a row into probabilities and an integer
// CDF.  Lane l holds symbols l, l+64, ... (V <= 256).
__device__ __forceinline__ void row_quantise(const float *p_in, int V, int lane, uint32_t *cdf) {
  int f[4];
  float pq[4];
  int fsum = 0;
  float best = -1.0f;
  int besti = 0x7fffffff;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    int v = lane + 64 * q;
    f[q] = 0;
    pq[q] = 0.0f;
    if (v < V) {
      float p = p_in[q];
      p = (p >= 0.0f && p <= 1.0f) ? p : 0.0f;
      pq[q] = p;
      // exact: a 24-bit mantissa times a 16-bit integer fits FP64
      f[q] = 1 + (int)floor((double)p * (double)(kTotal - (uint32_t)V));
      fsum += f[q];
      if (p > best) { best = p; besti = v; }
    }
  }
  fsum = wave_sum_i(fsum);
  wave_argmax(best, besti);
  besti = __builtin_amdgcn_readfirstlane(besti);
  int resid = (int)kTotal - fsum;
  int run = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (64 * q >= V) break;
    int v = lane + 64 * q;
    int fv = (v < V) ? f[q] + (v == besti ? resid : 0) : 0;
    int incl = wave_scan_incl(fv, lane);
    if (v < V) cdf[v] = (uint32_t)(run + incl - fv);
    run += __shfl(incl, 63);
  }
  if (lane == 0) cdf[V] = kTotal;
  (void)pq;
}

__device__ __forceinline__ long long to_fixed(float x) {
  double y = (double)x * (double)(1ull << kFixShift);
  y = fmin(fmax(y, -4.0e18), 4.0e18);
  return (long long)rint(y);
}

// ------------------------------------------------------------ GEMM tiles
struct Ctx {   // context-window gather for the first layer
  const uint8_t *ring;
  int RS, mask, base;   // ring row length, RS-1, (i - t)
  const float *emb;
  int E;
};

// out[j][o] = b[o] + sum_d in[j][d] W[d][o]   (optionally ReLU)
// layer 0 gathers in[j][p*E+e] = emb[ring[j][(base+p)&mask]][e]
__device__ __forceinline__ void fwd_tile(int r0, int c0, int Din, int Dout, const float *__restrict__ W,
                                         const float *__restrict__ b, const float *in, const Ctx *g, float *out,
                                         bool relu) {
  float acc[4][4];
  float4 bb = *reinterpret_cast<const float4 *>(b + c0);
#pragma unroll
  for (int r = 0; r < 4; r++) { acc[r][0] = bb.x; acc[r][1] = bb.y; acc[r][2] = bb.z; acc[r][3] = bb.w; }
  if (g) {
    const int t = Din / g->E;
    for (int p = 0; p < t; p++) {
      int tk[4];
#pragma unroll
      for (int r = 0; r < 4; r++) tk[r] = g->ring[(r0 + r) * g->RS + ((g->base + p) & g->mask)];
      for (int e = 0; e < g->E; e += 4) {
        float4 a[4], w[4];
#pragma unroll
        for (int r = 0; r < 4; r++) a[r] = *reinterpret_cast<const float4 *>(g->emb + tk[r] * g->E + e);
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
    *reinterpret_cast<float4 *>(out + (r0 + r) * Dout + c0) = o;
  }
}

// dIn[j][d] = sum_o dOut[j][o] W[d][o]; rows j0..j0+3, columns d0..d0+3
__device__ __forceinline__ void bwd_in_tile(int r0, int d0, int Dout, const float *__restrict__ W,
                                            const float *dOut, float acc[4][4]) {
#pragma unroll
  for (int r = 0; r < 4; r++)
#pragma unroll
    for (int q = 0; q < 4; q++) acc[r][q] = 0.0f;
  for (int o = 0; o < Dout; o += 4) {
    float4 a[4], w[4];
#pragma unroll
    for (int r = 0; r < 4; r++) a[r] = *reinterpret_cast<const float4 *>(dOut + (r0 + r) * Dout + o);
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

struct Opt {
  int kind;
  float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^tau, c2 = 1 - b2^tau
};
__device__ __forceinline__ float opt_delta(const Opt &o, float g, float *m, float *v) {
  if (o.kind == 0) return o.lr * g;
  float mm = o.b1 * (*m) + (1.0f - o.b1) * g;
  float vv = o.b2 * (*v) + (1.0f - o.b2) * (g * g);
  *m = mm;
  *v = vv;
  float mh = mm / o.c1, vh = vv / o.c2;
  return o.lr * mh / (sqrtf(vh) + o.eps);
}

// dW[d][o] = sum_j In[j][d] dOut[j][o], then the optimiser update of W.
__device__ __forceinline__ void bwd_w_tile(int d0, int o0, int rows, int Dout, float *W, float *M, float *Vv,
                                           const float *in, int Din, const Ctx *g, const float *dOut,
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
      int tk = g->ring[j * g->RS + ((g->base + p) & g->mask)];
      a = *reinterpret_cast<const float4 *>(g->emb + tk * g->E + e);
    } else {
      a = *reinterpret_cast<const float4 *>(in + j * Din + d0);
    }
    float4 bv = *reinterpret_cast<const float4 *>(dOut + j * Dout + o0);
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
__global__ __launch_bounds__(NT) void step_kernel(StepArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int sh_b;
  __shared__ float sh_ga;
  const Dims &d = a.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bs = d.bs, V = d.V, E = d.E, t = d.t, nh = d.nh, RS = d.RS, mask = d.RS - 1;
  float *emb = reinterpret_cast<float *>(lds + a.lay.emb);
  float *embs = reinterpret_cast<float *>(lds + a.lay.embs);
  uint8_t *ring = lds + a.lay.ring;
  float *act[2] = {reinterpret_cast<float *>(lds + a.lay.act[0]), reinterpret_cast<float *>(lds + a.lay.act[1])};
  float *lm = reinterpret_cast<float *>(lds + a.lay.lm);
  float *lu = reinterpret_cast<float *>(lds + a.lay.lu);
  uint32_t *cdf = reinterpret_cast<uint32_t *>(lds + a.lay.cdf);
  uint8_t *tgt = lds + a.lay.tgt;
  float *dh[2] = {reinterpret_cast<float *>(lds + a.lay.dh[0]), reinterpret_cast<float *>(lds + a.lay.dh[1])};
  long long *demb = reinterpret_cast<long long *>(lds + a.lay.demb);
  float *misc = reinterpret_cast<float *>(lds + a.lay.misc);   // [bs] row sums for the alpha gradient
  const int stride = d.stride;
  const float inv_bs = 1.0f / (float)bs;

  for (;;) {
    if (tid == 0) sh_b = atomicAdd(a.queue, 1);
    __syncthreads();
    const int b = sh_b;
    __syncthreads();
    if (b >= a.n_blocks) break;
    const BlockDesc bd = a.blocks[b];
    float *W = a.params + (size_t)b * stride;
    float *M = a.adam_m ? a.adam_m + (size_t)b * stride : nullptr;
    float *Vs = a.adam_v ? a.adam_v + (size_t)b * stride : nullptr;
    uint64_t Lrun = bd.L;
    if (a.stop && a.stop < Lrun) Lrun = a.stop;

    // ---- initial parameters: seeded, or the predecessor's snapshot (Sec. 4.3)
    const float *src = a.init;
    if (bd.pred >= 0) {
      if (tid == 0) {
        long long spins = 0;
        while (__hip_atomic_load(a.snap_flag + bd.pred, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
          __builtin_amdgcn_s_sleep(8);
          if (++spins > a.spin_limit) { atomicOr(a.err, 4); break; }
        }
      }
      __syncthreads();
      src = a.snap + (size_t)bd.pred * stride;
    }
    for (int q = tid; q < stride; q += NT) {
      W[q] = __builtin_nontemporal_load(src + q);
      if (M) { M[q] = 0.0f; Vs[q] = 0.0f; }
    }
    __syncthreads();
    for (int q = tid; q < V * E; q += NT) {
      emb[q] = W[d.off_emb + q];
      if (d.static_on) embs[q] = a.stat[d.off_emb + q];
      demb[q] = 0;
    }
    __syncthreads();

    auto snapshot = [&]() {
      float *dst = a.snap + (size_t)b * stride;
      for (int q = tid; q < stride; q += NT) dst[q] = (q >= d.off_emb && q < d.off_emb + V * E) ? emb[q - d.off_emb] : W[q];
      __threadfence();
      __syncthreads();
      if (tid == 0) __hip_atomic_store(a.snap_flag + b, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    };
    if (bd.has_snap && bd.S == 0) snapshot();

    // ---- coders: lane j < bs owns segment j
    Enc enc;
    Dec dec;
    int ovf = 0;
    uint32_t *slot = a.slots + bd.slot_off + (size_t)tid * bd.slot_words;
    uint32_t nwords = 0;
    if (tid < bs) {
      if (a.mode == 0) enc_init(enc);
      else {
        nwords = a.seg_words[(size_t)b * bs + tid];
        if (nwords > bd.slot_words) nwords = bd.slot_words;
        dec_init(dec, slot, nwords);
      }
    }
    Opt opt;
    opt.kind = d.optimizer;
    opt.lr = d.lr; opt.b1 = d.b1; opt.b2 = d.b2; opt.eps = d.eps;
    float b1t = 1.0f, b2t = 1.0f;
    int probe_i = 0;
    const size_t tok0 = bd.tok_off;

    for (uint64_t i = 0; i < Lrun; i++) {
      const bool uniform = !d.model_on || i < (uint64_t)t;
      // stage the true tokens of the next CH steps (encode)
      if (a.mode == 0 && (i % (uint64_t)d.CH) == 0) {
        const int CH = d.CH;
        for (int q = tid; q < bs * CH; q += NT) {
          int j = q / CH, c = q % CH;
          uint64_t pos = i + (uint64_t)c;
          if (pos < bd.L) ring[j * RS + (int)(pos & (uint64_t)mask)] = a.tokens[tok0 + (size_t)j * bd.L + pos];
        }
        __syncthreads();
      }
      float alpha = 0.0f;
      if (!uniform) {
        if (d.static_on) alpha = 1.0f / (1.0f + expf(-W[d.P]));
        Ctx g{ring, RS, mask, (int)(i - (uint64_t)t), emb, E};
        Ctx gs{ring, RS, mask, (int)(i - (uint64_t)t), embs, E};
        // forward, layer by layer; DM and static tiles share one pass
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
            fwd_tile(r0, c0, Din, Dout, Wp + d.off_W[l], Wp + d.off_b[l], in, l == 0 ? (st ? &gs : &g) : nullptr,
                     out, !last);
          }
          __syncthreads();
        }
        // mixer (Eq. 1) + softmax + quantiser, one wave per row
        for (int j = wave; j < bs; j += NT / 64) {
          float z[4], p[4];
          float mx = -INFINITY;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            int v = lane + 64 * q;
            z[q] = -INFINITY;
            if (v < V) {
              float m = lm[j * V + v];
              z[q] = d.static_on ? (alpha * lu[j * V + v] + (1.0f - alpha) * m) : m;
              mx = fmaxf(mx, z[q]);
            }
          }
          mx = wave_max(mx);
          float se = 0.0f;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            int v = lane + 64 * q;
            p[q] = (v < V) ? expf(z[q] - mx) : 0.0f;
            se += p[q];
          }
          se = wave_sum(se);
          float srow = 0.0f;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            int v = lane + 64 * q;
            if (v < V) {
              p[q] = p[q] / se;
              if (d.static_on) {
                float diff = lu[j * V + v] - lm[j * V + v];
                lu[j * V + v] = diff;
                srow = fmaf(p[q], diff, srow);
              }
              lm[j * V + v] = p[q];
            }
          }
          if (d.static_on) {
            srow = wave_sum(srow);
            if (lane == 0) misc[j] = srow;
          }
          row_quantise(p, V, lane, cdf + j * (V + 1));
          if (a.probe_P && b == 0 && probe_i < a.n_probe && a.probe_steps[probe_i] == i) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
              int v = lane + 64 * q;
              if (v < V) a.probe_P[((size_t)probe_i * bs + j) * V + v] = p[q];
            }
          }
        }
        __syncthreads();
      } else if (a.probe_P && b == 0 && probe_i < a.n_probe && a.probe_steps[probe_i] == i) {
        for (int q = tid; q < bs * V; q += NT) a.probe_P[(size_t)probe_i * bs * V + q] = 1.0f / (float)V;
      }
      if (a.probe_P && b == 0 && probe_i < a.n_probe && a.probe_steps[probe_i] == i) probe_i++;

      // ---- coding: lane j codes token i of segment j
      if (tid < bs) {
        const int j = tid;
        const int rp = j * RS + (int)(i & (uint64_t)mask);
        const uint32_t unit = kTotal / (uint32_t)V;
        if (a.mode == 0) {
          int e = ring[rp];
          uint32_t lo, hi;
          if (uniform) { lo = (uint32_t)e * unit; hi = lo + unit; }
          else { lo = cdf[j * (V + 1) + e]; hi = cdf[j * (V + 1) + e + 1]; }
          enc_symbol(enc, slot, bd.slot_words, lo, hi, ovf);
          tgt[j] = (uint8_t)e;
        } else {
          int e;
          if (uniform) e = dec_symbol(dec, slot, nwords, V, [&](int s) { return (uint32_t)s * unit; });
          else {
            const uint32_t *c = cdf + j * (V + 1);
            e = dec_symbol(dec, slot, nwords, V, [&](int s) { return c[s]; });
          }
          ring[rp] = (uint8_t)e;
          tgt[j] = (uint8_t)e;
          a.tokens[tok0 + (size_t)j * bd.L + i] = (uint8_t)e;
        }
      }
      __syncthreads();

      if (!uniform) {
        // dz = (P - onehot)/bs (mean loss over the step's rows); dL^m = (1-alpha) dz
        for (int q = tid; q < bs * V; q += NT) {
          int j = q / V, v = q % V;
          float dz = (lm[q] - (v == tgt[j] ? 1.0f : 0.0f)) * inv_bs;
          lm[q] = d.static_on ? dz * (1.0f - alpha) : dz;
        }
        if (d.static_on && tid == 0) {
          float acc = 0.0f;
          for (int j = 0; j < bs; j++) acc += misc[j] - lu[j * V + tgt[j]];
          sh_ga = acc * inv_bs * (alpha * (1.0f - alpha));
        }
        __syncthreads();
        opt.c1 = 1.0f;
        opt.c2 = 1.0f;
        if (opt.kind == 1) {
          b1t *= d.b1;
          b2t *= d.b2;
          opt.c1 = 1.0f - b1t;
          opt.c2 = 1.0f - b2t;
        }
        const Ctx g{ring, RS, mask, (int)(i - (uint64_t)t), emb, E};
        const float *dout = lm;
        for (int l = nh; l >= 0; l--) {
          const int Din = d.dim[l], Dout = d.dim[l + 1];
          float *Wl = W + d.off_W[l];
          float *dIn = dh[(nh - l) & 1];
          // (a) gradient of this layer's input, with the old weights
          const int tiles_a = (bs / 4) * (Din / 4);
          for (int tile = tid; tile < tiles_a; tile += NT) {
            const int r0 = (tile / (Din / 4)) * 4, c0 = (tile % (Din / 4)) * 4;
            float acc[4][4];
            bwd_in_tile(r0, c0, Dout, Wl, dout, acc);
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
                  const int tk = ring[j * RS + (((int)(i - (uint64_t)t) + p) & mask)];
                  atomicAdd(reinterpret_cast<unsigned long long *>(demb + tk * E + e),
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
            bwd_w_tile(d0, o0, bs, Dout, Wl, Ml, Vl, l == 0 ? nullptr : act[l - 1], Din, l == 0 ? &g : nullptr,
                       dout, opt);
          }
          for (int o = tid; o < Dout; o += NT) {
            float gsum = 0.0f;
            for (int j = 0; j < bs; j++) gsum += dout[j * Dout + o];
            const int bi = d.off_b[l] + o;
            W[bi] = W[bi] - opt_delta(opt, gsum, M ? M + bi : nullptr, Vs ? Vs + bi : nullptr);
          }
          dout = dIn;
        }
        __syncthreads();
        // embedding update from the fixed-point sums
        for (int q = tid; q < V * E; q += NT) {
          float gq = (float)((double)demb[q] * (1.0 / (double)(1ull << kFixShift)));
          demb[q] = 0;
          const int pi = d.off_emb + q;
          emb[q] = emb[q] - opt_delta(opt, gq, M ? M + pi : nullptr, Vs ? Vs + pi : nullptr);
        }
        if (d.static_on && tid == 0) {
          W[d.P] = W[d.P] - opt_delta(opt, sh_ga, M ? M + d.P : nullptr, Vs ? Vs + d.P : nullptr);
        }
        __syncthreads();
      }
      if (bd.has_snap && i + 1 == (uint64_t)bd.S) snapshot();
    }

    if (tid < bs) {
      if (a.mode == 0) {
        enc_finish(enc, slot, bd.slot_words, ovf);
        a.seg_bits[(size_t)b * bs + tid] = (uint32_t)enc.nbits;
      }
      if (ovf) atomicOr(a.err, 2);
    }
    // final parameters (embedding lives in LDS during the loop)
    for (int q = tid; q < V * E; q += NT) W[d.off_emb + q] = emb[q];
    __syncthreads();
    if (a.params_out && b == 0)
      for (int q = tid; q < d.P + 1; q += NT) a.params_out[q] = W[q];
    __syncthreads();
  }
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
__global__ void quantise_kernel(const float *P, uint32_t rows, uint32_t V, uint32_t *cdf) {
  const int lane = threadIdx.x & 63;
  const uint32_t row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (row >= rows) return;
  float p[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    int v = lane + 64 * q;
    p[q] = v < (int)V ? P[(size_t)row * V + v] : 0.0f;
  }
  row_quantise(p, (int)V, lane, cdf + (size_t)row * (V + 1));
}

hipError_t launch_quantise(const float *P, uint32_t rows, uint32_t V, uint32_t *cdf, hipStream_t st) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(quantise_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, P, rows, V, cdf);
  return hipGetLastError();
}

__global__ void wnc_encode_kernel(const uint32_t *lo, const uint32_t *hi, uint64_t m, uint32_t *out,
                                  uint32_t cap, uint64_t *nbits, int *err) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Enc e;
  enc_init(e);
  int ovf = 0;
  for (uint64_t i = 0; i < m; i++) enc_symbol(e, out, cap, lo[i], hi[i], ovf);
  enc_finish(e, out, cap, ovf);
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
  dec_init(d, words, nwords);
  for (uint64_t i = 0; i < m; i++) {
    const uint32_t *c = cdfs + i * (V + 1);
    sym[i] = (uint32_t)dec_symbol(d, words, nwords, (int)V, [&](int s) { return c[s]; });
  }
}

hipError_t launch_wnc_decode(const uint32_t *words, uint32_t nwords, const uint32_t *cdfs, uint32_t V,
                             uint64_t m, uint32_t *sym, hipStream_t st) {
  hipLaunchKernelGGL(wnc_decode_kernel, dim3(1), dim3(64), 0, st, words, nwords, cdfs, V, m, sym);
  return hipGetLastError();
}

}  // namespace pmklc
