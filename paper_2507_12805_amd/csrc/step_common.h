// Device code shared by the step kernels (library-private).
#pragma once
#include "pmklc_internal.h"

namespace pmklc {
namespace detail {

// Global-memory views.  Pointers read out of the argument block are generic
// (flat) to the compiler, and a flat load also counts as LDS traffic: every
// wait for an LDS read would then wait for the outstanding weight loads too.
// Hot loops address weights through these address-space-1 views instead.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) uint8_t gu8;
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) fvec4 gfvec4;
// Waits until this wave's outstanding global loads and stores are done.
// Loads and stores share one counter, and with stores outstanding the
// compiler can only wait for everything; draining the stores of an earlier
// phase once (they are long done) lets the loads of the next phase be waited
// for one chunk at a time.  (gfx9 encoding: vmcnt 0, expcnt 7, lgkmcnt 15.)
__device__ __forceinline__ void drain_stores() { __builtin_amdgcn_s_waitcnt(0x0F70); }
__device__ __forceinline__ gfloat *glb(float *p) { return (gfloat *)p; }
__device__ __forceinline__ const gfloat *glb(const float *p) { return (const gfloat *)p; }
// four consecutive floats, 16-byte aligned
__device__ __forceinline__ fvec4 ld4(const gfloat *p) { return *(const gfvec4 *)p; }
__device__ __forceinline__ void st4(gfloat *p, fvec4 v) { *(gfvec4 *)p = v; }


constexpr uint32_t kHalf = 0x80000000u;
constexpr uint32_t kQuarter = 0x40000000u;

// Lane exchanges inside aligned groups of G lanes (G a power of two), the
// first three levels by DPP lane permutations, which are register moves,
// the wider ones through the LDS crossbar.  Level 1 pairs lane i with
// i ^ 1, level 2 with i ^ 2 (quad permutations), level 3 with 7 - i inside
// its 8 (row half-mirror); level o >= 8 pairs i with i ^ o.  Every level
// pairs lanes symmetrically, so a reduction ends with the same value, in the
// same order of operations, in every lane of the group.
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(dpp_mov<CTRL>(__float_as_int(x)));
}
template <class T, class Op>
__device__ __forceinline__ T group_reduce(T x, int G, Op op) {
  if (G >= 2) x = op(x, dpp_mov<0xB1>(x));    // quad_perm [1, 0, 3, 2]
  if (G >= 4) x = op(x, dpp_mov<0x4E>(x));    // quad_perm [2, 3, 0, 1]
  if (G >= 8) x = op(x, dpp_mov<0x141>(x));   // row_half_mirror
  for (int o = 8; o < G; o <<= 1) x = op(x, __shfl_xor(x, o));
  return x;
}
// the partner's value at each level, for reductions over several values
template <class F>
__device__ __forceinline__ void group_levels(int G, F &&level) {
  if (G >= 2) level([](auto v) { return dpp_mov<0xB1>(v); });
  if (G >= 4) level([](auto v) { return dpp_mov<0x4E>(v); });
  if (G >= 8) level([](auto v) { return dpp_mov<0x141>(v); });
  for (int o = 8; o < G; o <<= 1) level([o](auto v) { return __shfl_xor(v, o); });
}
// inclusive prefix sum over the G lanes of a group (gl: index in the group);
// a row shift brings lane i - o, taken only when it is in the same group
__device__ __forceinline__ int group_scan(int x, int G, int gl) {
  if (G >= 2) { const int y = dpp_mov<0x111>(x); if (gl >= 1) x += y; }   // row_shr:1
  if (G >= 4) { const int y = dpp_mov<0x112>(x); if (gl >= 2) x += y; }   // row_shr:2
  if (G >= 8) { const int y = dpp_mov<0x114>(x); if (gl >= 4) x += y; }   // row_shr:4
  for (int o = 8; o < G; o <<= 1) { const int y = __shfl_up(x, o, G); if (gl >= o) x += y; }
  return x;
}
__device__ __forceinline__ float wave_sum(float x) {
  return group_reduce(x, 64, [](float a, float b) { return a + b; });
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
__device__ __forceinline__ void enc_emit(Enc &e, gu32 *slot, uint32_t cap, uint32_t bits, int n, int &ovf) {
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
__device__ __forceinline__ void enc_run(Enc &e, gu32 *slot, uint32_t cap, int bit, uint32_t count, int &ovf) {
  while (count) {
    int n = count > 32u ? 32 : (int)count;
    uint32_t bits = bit ? (n == 32 ? 0xFFFFFFFFu : ((1u << n) - 1u)) : 0u;
    enc_emit(e, slot, cap, bits, n, ovf);
    count -= (uint32_t)n;
  }
}
// Renormalisation of the WNC coder (Witten, Neal and Cleary 1987) in two
// bulk moves that give exactly what its one-bit loop gives.  While the top
// bits of low and high agree the loop outputs that bit (E1 for 0, E2 for 1)
// and shifts both left (high taking a 1): the k1 = clz(low ^ high) agreed
// leading bits go out together, the first followed by the pending opposite
// bits.  Then, while low has 1 and high has 0 in bit 30 (E3), the loop counts
// a pending bit and maps x -> 2 (x - 2^30): over k3 such positions that is
// x << k3 with bit 31 flipped, mod 2^32, high again taking 1s.  After E3 the
// top bits still differ, so no E1/E2 follows.  With the coding range above
// 2^30 before a symbol and every frequency at least 1, the new range exceeds
// 2^14, so k1 and k3 stay far below 32 (k1 is clamped to 31 for an empty
// interval, which only a caller's invalid table can give).
__device__ __forceinline__ void enc_symbol(Enc &e, gu32 *slot, uint32_t cap, uint32_t lo, uint32_t hi, int &ovf) {
  uint64_t r = (uint64_t)e.high - e.low + 1u;
  uint32_t l0 = e.low;
  uint32_t high = l0 + (uint32_t)((r * hi) >> kTotalBits) - 1u;
  uint32_t low = l0 + (uint32_t)((r * lo) >> kTotalBits);
  const int k1 = min(__clz(low ^ high), 31);   // (31 only for an empty interval)
  if (k1 > 0) {
    const uint32_t top = low >> (32 - k1);   // the agreed bits, first one highest
    if (e.pending) {
      const uint32_t first = top >> (k1 - 1);
      enc_emit(e, slot, cap, first, 1, ovf);
      enc_run(e, slot, cap, first ^ 1u, e.pending, ovf);
      e.pending = 0;
      if (k1 > 1) enc_emit(e, slot, cap, top & ((1u << (k1 - 1)) - 1u), k1 - 1, ovf);
    } else {
      enc_emit(e, slot, cap, top, k1, ovf);
    }
    low <<= k1;
    high = (high << k1) | ((1u << k1) - 1u);
  }
  const int k3 = __clz(~((low & ~high) << 1));
  if (k3 > 0) {
    e.pending += (uint32_t)k3;
    low = (low << k3) ^ kHalf;
    high = ((high << k3) ^ kHalf) | ((1u << k3) - 1u);
  }
  e.low = low;
  e.high = high;
}
__device__ __forceinline__ void enc_finish(Enc &e, gu32 *slot, uint32_t cap, int &ovf) {
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
  uint64_t buf;   // the low nbuf bits are the next stream bits, first one highest
  int nbuf;
};
// the next n stream bits (1 <= n <= 32) as an integer, first bit highest;
// bits past the last word are 0
__device__ __forceinline__ uint32_t dec_bits(Dec &d, const gu32 *w, uint32_t nw, int n) {
  if (d.nbuf < n) {
    const uint32_t x = d.widx < nw ? __builtin_bswap32(w[d.widx]) : 0u;
    d.widx++;
    d.buf = (d.buf << 32) | x;
    d.nbuf += 32;
  }
  d.nbuf -= n;
  return (uint32_t)(d.buf >> d.nbuf) & (uint32_t)((1ull << n) - 1ull);
}
__device__ __forceinline__ void dec_init(Dec &d, const gu32 *w, uint32_t nw) {
  d.low = 0; d.high = 0xFFFFFFFFu; d.widx = 0; d.buf = 0; d.nbuf = 0;
  d.value = dec_bits(d, w, nw, 32);
}
// cum(s) is the cumulative count below symbol s (cum(0) = 0, cum(V) = 2^16).
// The renormalisation mirrors enc_symbol's, value taking the stream bits.
template <class Cum>
__device__ __forceinline__ int dec_symbol(Dec &d, const gu32 *w, uint32_t nw, int V, Cum cum) {
  uint64_t r = (uint64_t)d.high - d.low + 1u;
  uint32_t target = d.value - d.low;
  int a = 0, b = V;
  while (b - a > 1) {
    int m = (a + b) >> 1;
    if ((uint32_t)((r * cum(m)) >> kTotalBits) <= target) a = m;
    else b = m;
  }
  uint32_t l0 = d.low;
  uint32_t high = l0 + (uint32_t)((r * cum(a + 1)) >> kTotalBits) - 1u;
  uint32_t low = l0 + (uint32_t)((r * cum(a)) >> kTotalBits);
  uint32_t value = d.value;
  const int k1 = min(__clz(low ^ high), 31);   // (31 only for an empty interval)
  if (k1 > 0) {
    low <<= k1;
    high = (high << k1) | ((1u << k1) - 1u);
    value = (value << k1) | dec_bits(d, w, nw, k1);
  }
  const int k3 = __clz(~((low & ~high) << 1));
  if (k3 > 0) {
    low = (low << k3) ^ kHalf;
    high = ((high << k3) ^ kHalf) | ((1u << k3) - 1u);
    value = ((value << k3) ^ kHalf) | dec_bits(d, w, nw, k3);
  }
  d.low = low;
  d.high = high;
  d.value = value;
  return a;
}

// One segment's coder between steps.  It is kept in LDS and loaded and
// stored around each use, so that none of it is live (and spilled) across
// the rest of the step.
struct CoderState {
  union {
    Enc enc;
    Dec dec;
  };
  uint32_t nwords;   // decode: words in the segment's stream
  int ovf;           // encode: the slot overflowed
};
static_assert(sizeof(CoderState) == 48, "the LDS plan reserves 48 bytes per segment");

// ------------------------------------------------------------ quantiser
// floor(p * c) of the exact real product, for 0 <= p <= 1 and an integer
// 0 < c < 2^24, in FP32: y = fl(p c) and the FMA residual p c - y (exact for
// a product) decide the only ambiguous case, y integral with p c < y.  If y
// is not an integer, no integer lies between p c and y (integers below 2^24
// are representable and rounding is monotone), so floor(y) is exact.
__device__ __forceinline__ int floor_mul_exact(float p, float c) {
  const float y = p * c;
  const float err = fmaf(p, c, -y);
  float fy = floorf(y);
  if (fy == y && err < 0.0f) fy -= 1.0f;
  return (int)fy;
}

// Lanes per row of the mixer/softmax/quantiser and symbols per lane: V/8
// symbols per lane (at least 4, a float4 run); G = V/spl divides 64 for
// every V = 4^k, so a row's lanes sit in one wave, aligned.
__device__ __forceinline__ int row_spl(int V) { return V >= 32 ? V >> 3 : 4; }

// Frequency quantisation of one row by its G lanes (lane gl holds the SPL
// probabilities of symbols [gl*SPL, gl*SPL + SPL) in registers):
// f_v = 1 + floor(p_v * (2^16 - V)) with the product exact, the residual
// 2^16 - sum f added to the most probable symbol (lowest index on ties), and
// the V+1 cumulative counts written.  Integer sums and a fixed-order scan: the
// result does not depend on G.  Invalid probabilities (NaN, outside [0, 1])
// count as 0.
template <int SPL>
__device__ __forceinline__ void row_quantise_regs(const float (&p)[SPL], int V, int G, int gl, uint32_t *cdf) {
  const float qc = (float)(kTotal - (uint32_t)V);
  const int v0 = gl * SPL;
  int f[SPL];
  int fs = 0, bi = v0;
  float best = -1.0f;
#pragma unroll
  for (int q = 0; q < SPL; q++) {
    const float pv = (p[q] >= 0.0f && p[q] <= 1.0f) ? p[q] : 0.0f;
    f[q] = 1 + floor_mul_exact(pv, qc);
    fs += f[q];
    if (pv > best) { best = pv; bi = v0 + q; }
  }
  int tot = fs;
  group_levels(G, [&](auto other) {
    tot += other(tot);
    const float ob = other(best);
    const int oi = other(bi);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  });
  const int resid = (int)kTotal - tot;
  const int mine = fs + ((bi >= v0 && bi < v0 + SPL) ? resid : 0);
  const int incl = group_scan(mine, G, gl);
  uint32_t run = (uint32_t)(incl - mine);
#pragma unroll
  for (int q = 0; q < SPL; q++) {
    cdf[v0 + q] = run;
    run += (uint32_t)(f[q] + (v0 + q == bi ? resid : 0));
  }
  if (gl == G - 1) cdf[V] = kTotal;
}

// the same from a row in memory (symbols per lane: 4, 8 or 32 for V = 4^k)
template <int SPL>
__device__ __forceinline__ void row_quantise_mem(const float *p, int V, int G, int gl, uint32_t *cdf) {
  float r[SPL];
#pragma unroll
  for (int q = 0; q < SPL; q++) r[q] = p[gl * SPL + q];
  row_quantise_regs<SPL>(r, V, G, gl, cdf);
}
__device__ __forceinline__ void row_quantise_group(const float *p, int V, int spl, int G, int gl, uint32_t *cdf) {
  if (spl == 4) row_quantise_mem<4>(p, V, G, gl, cdf);
  else if (spl == 8) row_quantise_mem<8>(p, V, G, gl, cdf);
  else row_quantise_mem<32>(p, V, G, gl, cdf);
}

// Mixer (Eq. 1), softmax and quantiser of one row by its G lanes, SPL
// symbols per lane held in registers.  lr: the dynamic logits, replaced by
// the probabilities; ur: the static logits, replaced by L^u - L^m (for the
// mixing-weight gradient).  Returns this row's sum_v p_v (L^u_v - L^m_v)
// (static model on) in every lane of the row.
template <int SPL>
__device__ __forceinline__ float row_softmax_regs(float *lr, float *ur, bool mix, float alpha, int V, int G, int gl,
                                                  uint32_t *cdf, float (&pr)[SPL]) {
  const int v0 = gl * SPL;
  float z[SPL], df[SPL];
  float mx = -INFINITY;
#pragma unroll
  for (int q = 0; q < SPL; q += 4) {
    const float4 m4 = *reinterpret_cast<const float4 *>(lr + v0 + q);
    const float mm[4] = {m4.x, m4.y, m4.z, m4.w};
    if (mix) {
      const float4 u4 = *reinterpret_cast<const float4 *>(ur + v0 + q);
      const float uu[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
      for (int c = 0; c < 4; c++) {
        z[q + c] = alpha * uu[c] + (1.0f - alpha) * mm[c];
        df[q + c] = uu[c] - mm[c];
      }
      *reinterpret_cast<float4 *>(ur + v0 + q) = make_float4(df[q], df[q + 1], df[q + 2], df[q + 3]);
    } else {
#pragma unroll
      for (int c = 0; c < 4; c++) z[q + c] = mm[c];
    }
    mx = fmaxf(mx, fmaxf(fmaxf(z[q], z[q + 1]), fmaxf(z[q + 2], z[q + 3])));
  }
  mx = group_reduce(mx, G, [](float a, float b) { return fmaxf(a, b); });
  // hardware exp2-based exponential and one reciprocal per row: both
  // deterministic, within a few ulp of the correctly rounded values
  float se = 0.0f;
#pragma unroll
  for (int q = 0; q < SPL; q += 4) {
#pragma unroll
    for (int c = 0; c < 4; c++) z[q + c] = __expf(z[q + c] - mx);
    se = se + z[q] + z[q + 1] + z[q + 2] + z[q + 3];
  }
  se = group_reduce(se, G, [](float a, float b) { return a + b; });
  const float rse = 1.0f / se;
  float srow = 0.0f;
#pragma unroll
  for (int q = 0; q < SPL; q += 4) {
#pragma unroll
    for (int c = 0; c < 4; c++) pr[q + c] = z[q + c] * rse;
    *reinterpret_cast<float4 *>(lr + v0 + q) = make_float4(pr[q], pr[q + 1], pr[q + 2], pr[q + 3]);
    if (mix) {
#pragma unroll
      for (int c = 0; c < 4; c++) srow = fmaf(pr[q + c], df[q + c], srow);
    }
  }
  if (mix) srow = group_reduce(srow, G, [](float a, float b) { return a + b; });
  row_quantise_regs<SPL>(pr, V, G, gl, cdf);
  return srow;
}

__device__ __forceinline__ long long to_fixed(float x) {
  double y = (double)x * (double)(1ull << kFixShift);
  y = fmin(fmax(y, -4.0e18), 4.0e18);
  return (long long)rint(y);
}

struct Opt {
  int kind;
  float lr, b1, b2, eps, c1, c2;   // c1 = 1 - b1^tau, c2 = 1 - b2^tau
};
// m, v: optimiser state in LDS/registers (float) or global memory (gfloat);
// untouched by SGD.  opt_delta_c fixes the optimiser at compile time (no
// branch in the caller's loop); opt_delta picks it at run time.
template <bool ADAM, class F>
__device__ __forceinline__ float opt_delta_c(const Opt &o, float g, F *m, F *v) {
  if constexpr (!ADAM) {
    return o.lr * g;
  } else {
    float mm = o.b1 * (*m) + (1.0f - o.b1) * g;
    float vv = o.b2 * (*v) + (1.0f - o.b2) * (g * g);
    *m = mm;
    *v = vv;
    float mh = mm / o.c1, vh = vv / o.c2;
    return o.lr * mh / (sqrtf(vh) + o.eps);
  }
}
template <class F>
__device__ __forceinline__ float opt_delta(const Opt &o, float g, F *m, F *v) {
  return o.kind == 1 ? opt_delta_c<true>(o, g, m, v) : opt_delta_c<false>(o, g, m, v);
}


// Per-phase wall-clock accounting of one block's loop (block 0, thread 0):
// phases 0 staging, 1 forward, 2 softmax+quantiser, 3 coder, 4 loss
// gradient, 5 network backward, 6 embedding update; the network may split
// its backward into 8.. (B1, B2+B3, B4). Enabled when a sink is given.
// The sums live in LDS (acc, 12 entries, touched by the one active thread
// only), so that a disabled clock holds no registers through the loop.
struct PhaseClock {
  unsigned long long *sink;
  unsigned long long *acc;
  unsigned long long t0;
  bool on;
  __device__ void init(unsigned long long *s, unsigned long long *acc_lds, bool active) {
    sink = s;
    acc = acc_lds;
    on = s && active;
    if (on)
      for (int q = 0; q < 12; q++) acc[q] = 0;
    t0 = on ? wall_clock64() : 0;
  }
  __device__ __forceinline__ void mark(int phase) {
    if (!on) return;
    unsigned long long t = wall_clock64();
    acc[phase] += t - t0;
    t0 = t;
  }
  __device__ void flush() {
    if (!on) return;
    for (int q = 0; q < 12; q++) sink[q] = acc[q];
  }
};

}  // namespace detail

using namespace detail;

// The per-block loop shared by every step kernel: block queue, model
// passing, token staging, mixer + softmax + quantiser, coders, loss
// gradient, embedding and mixing-weight updates.  `Net` supplies the
// forward (logits into lm, and lu when the static model is on) and the
// backward of the MLP layers (weight updates and the embedding gradient);
// both end with a workgroup barrier.  A Net with kOnChip keeps its layer
// parameters in registers and LDS during a block: it writes them back to
// the parameter slab with flush() (before a snapshot and at the block's
// end), hands over the embedding gradient through emb_grad(), sees every
// embedding value written (emb_set(), for a copy of its own), and updates
// what it keeps on chip besides the weight matrices in after_update(),
// during the embedding-update phase.  The others sum the embedding
// gradient into the fixed-point table demb.
template <int NT, class Net>
__device__ __forceinline__ void run_blocks(const StepArgs &a, unsigned char *lds, Net &net) {
  __shared__ int sh_b;
  __shared__ float sh_ga;
  __shared__ float sh_a;   // the mixing weight's raw parameter a (Eq. 1), kept beside its global copy
  __shared__ unsigned long long sh_pc[12];   // phase clock sums (block 0, thread 0)
  const Dims &d = a.d;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int bs = d.bs, V = d.V, E = d.E, t = d.t, mask = d.RS - 1, VS = d.VS;
  float *emb = reinterpret_cast<float *>(lds + a.lay.emb);
  float *embs = reinterpret_cast<float *>(lds + a.lay.embs);
  uint8_t *ring = lds + a.lay.ring;
  float *lm = reinterpret_cast<float *>(lds + a.lay.lm);
  float *lu = reinterpret_cast<float *>(lds + a.lay.lu);
  uint32_t *cdf = reinterpret_cast<uint32_t *>(lds + a.lay.cdf);
  uint8_t *tgt = lds + a.lay.tgt;
  long long *demb = reinterpret_cast<long long *>(lds + a.lay.demb);
  float *misc = reinterpret_cast<float *>(lds + a.lay.misc);   // [bs] row sums for the alpha gradient
  const int stride = d.stride;
  const float inv_bs = 1.0f / (float)bs;

  __shared__ int sh_ok;
  for (;;) {
    if (tid == 0) {
      const int q = atomicAdd(a.queue, 1);
      sh_b = q < a.n_blocks && a.order ? a.order[q] : q;
    }
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
    // The predecessor was dequeued before this block, so it is running or
    // done.  The wait ends when its snapshot is published (flag 1).  It fails
    // only if the predecessor gave up (flag 2) or, while running, made no
    // step for spin_limit sleeps; a predecessor that is itself waiting
    // (progress 0) keeps the wait alive.  A block that fails skips its work
    // and passes the failure on to its own successor.
    const float *src = a.init;
    if (bd.pred >= 0) {
      if (tid == 0) {
        int ok = 1;
        uint32_t last = 0;
        long long idle = 0;
        for (;;) {
          const int f = __hip_atomic_load(a.snap_flag + bd.pred, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
          if (f == 1) break;
          if (f != 0) { ok = 0; break; }
          const uint32_t pg = __hip_atomic_load(a.progress + bd.pred, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (pg == 0 || pg != last) { last = pg; idle = 0; }
          else if (++idle > a.spin_limit) { ok = 0; break; }
          __builtin_amdgcn_s_sleep(8);
        }
        if (!ok) {
          atomicOr(a.err, 4);
          if (bd.has_snap) __hip_atomic_store(a.snap_flag + b, 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        sh_ok = ok;
      }
      __syncthreads();
      const int ok = sh_ok;
      __syncthreads();
      if (!ok) continue;
      src = a.snap + (size_t)bd.pred * stride;
    }
    for (int q = tid; q < stride; q += NT) {
      W[q] = __builtin_nontemporal_load(src + q);
      if (M) { M[q] = 0.0f; Vs[q] = 0.0f; }
    }
    net.begin_block(src);
    if (tid == 0) sh_a = d.static_on ? src[d.P] : 0.0f;
    __syncthreads();
    for (int q = tid; q < V * E; q += NT) {
      const int v = (int)__umulhi((uint32_t)q, d.Emag), qp = q + v * (d.EP - E);   // row v, pitch EP
      emb[qp] = W[d.off_emb + q];
      if constexpr (Net::kOnChip) net.emb_set(v, q - v * E, emb[qp]);
      if (d.static_on) embs[qp] = a.stat[d.off_emb + q];
    }
    if constexpr (!Net::kOnChip)
      for (int q = tid; q < V * d.ES; q += NT) demb[q] = 0;
    __syncthreads();

    auto snapshot = [&]() {
      if constexpr (Net::kOnChip) {
        net.flush(W);
        __syncthreads();
      }
      float *dst = a.snap + (size_t)b * stride;
      for (int q = tid; q < stride; q += NT) {
        const int qe = q - d.off_emb;
        dst[q] = (qe >= 0 && qe < V * E) ? emb[qe + (int)__umulhi((uint32_t)qe, d.Emag) * (d.EP - E)] : W[q];
      }
      __threadfence();
      __syncthreads();
      if (tid == 0) __hip_atomic_store(a.snap_flag + b, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    };
    if (bd.has_snap && bd.S == 0) snapshot();

    // ---- coders: lane j < bs owns segment j; its state lives in cst[j].
    // (global-space views: a generic access would also hold up every LDS wait)
    CoderState *cst = reinterpret_cast<CoderState *>(lds + a.lay.cst);
    auto slot_of = [&](int j) { return (gu32 *)(a.slots + bd.slot_off + (size_t)j * bd.slot_words); };
    gu8 *toks = (gu8 *)a.tokens;
    if (tid < bs) {
      CoderState c;
      c.ovf = 0;
      c.nwords = 0;
      if (a.mode == 0) enc_init(c.enc);
      else {
        c.nwords = a.seg_words[(size_t)b * bs + tid];
        if (c.nwords > bd.slot_words) c.nwords = bd.slot_words;
        dec_init(c.dec, slot_of(tid), c.nwords);
      }
      cst[tid] = c;
    }
    Opt opt;
    opt.kind = d.optimizer;
    opt.lr = d.lr; opt.b1 = d.b1; opt.b2 = d.b2; opt.eps = d.eps;
    float b1t = 1.0f, b2t = 1.0f;
    int probe_i = 0;
    const size_t tok0 = bd.tok_off;
    PhaseClock pc;
    pc.init(a.phase_clk, sh_pc, b == 0 && tid == 0);
    net.pc = &pc;

    for (uint64_t i = 0; i < Lrun; i++) {
      const bool uniform = !d.model_on || i < (uint64_t)t;
      // stage the true tokens of the next CH steps (encode)
      if (a.mode == 0 && (i & (uint64_t)(d.CH - 1)) == 0) {   // (CH a power of two)
        const int CH = d.CH, chs = __builtin_ctz((unsigned)CH);
        for (int q = tid; q < bs * CH; q += NT) {
          const int j = q >> chs, c = q & (CH - 1);
          uint64_t pos = i + (uint64_t)c;
          if (pos < bd.L) ring[(int)(pos & (uint64_t)mask) * bs + j] = toks[tok0 + (size_t)j * bd.L + pos];
        }
        __syncthreads();
      }
      pc.mark(0);
      float alpha = 0.0f;
      if (!uniform) {
        if (d.static_on) alpha = 1.0f / (1.0f + expf(-sh_a));
        net.forward(W, i, alpha);
        pc.mark(1);
        // mixer (Eq. 1) + softmax + quantiser: G aligned lanes of one wave per
        // row, spl symbols each (float4 runs); row reductions are symmetric
        // lane exchanges over the G lanes after a sequential per-lane sum, so
        // the order is fixed.  Rows are VS = V + 4 floats apart.  (spl and G
        // are powers of two.)
        const int spl = row_spl(V), G = V / spl, gs = __builtin_ctz((unsigned)G);
        for (int j0 = 0; j0 < bs; j0 += NT >> gs) {
          const int j = j0 + (tid >> gs), gl = tid & (G - 1);
          if (j >= bs) continue;   // a row's lanes are all in or all out
          float *lr = lm + j * VS;
          float *ur = lu + j * VS;
          uint32_t *crow = cdf + j * (V + 1);
          float srow;
          const bool probe = a.probe_P && b == 0 && probe_i < a.n_probe && a.probe_steps[probe_i] == i;
          float *pp = probe ? a.probe_P + ((size_t)probe_i * bs + j) * V + gl * spl : nullptr;
          if (Net::kSpl == 8 || (Net::kSpl == 0 && spl == 8)) {
            float pr[8];
            srow = row_softmax_regs<8>(lr, ur, d.static_on, alpha, V, G, gl, crow, pr);
            if (pp) for (int q = 0; q < 8; q++) pp[q] = pr[q];
          } else if (Net::kSpl != 0) {
            __builtin_unreachable();
          } else if (spl == 4) {
            float pr[4];
            srow = row_softmax_regs<4>(lr, ur, d.static_on, alpha, V, G, gl, crow, pr);
            if (pp) for (int q = 0; q < 4; q++) pp[q] = pr[q];
          } else {
            float pr[32];
            srow = row_softmax_regs<32>(lr, ur, d.static_on, alpha, V, G, gl, crow, pr);
            if (pp) for (int q = 0; q < 32; q++) pp[q] = pr[q];
          }
          if (d.static_on && gl == 0) misc[j] = srow;
        }
        __syncthreads();
      } else if (a.probe_P && b == 0 && probe_i < a.n_probe && a.probe_steps[probe_i] == i) {
        for (int q = tid; q < bs * V; q += NT) a.probe_P[(size_t)probe_i * bs * V + q] = 1.0f / (float)V;
      }
      if (a.probe_P && b == 0 && probe_i < a.n_probe && a.probe_steps[probe_i] == i) probe_i++;

      pc.mark(2);
      // ---- coding: lane j codes token i of segment j
      if (tid < bs) {
        const int j = tid;
        const int rp = (int)(i & (uint64_t)mask) * bs + j;
        const uint32_t unit = kTotal / (uint32_t)V;
        CoderState cs = cst[j];
        gu32 *slot = slot_of(j);
        if (a.mode == 0) {
          int e = ring[rp];
          uint32_t lo, hi;
          if (uniform) { lo = (uint32_t)e * unit; hi = lo + unit; }
          else { lo = cdf[j * (V + 1) + e]; hi = cdf[j * (V + 1) + e + 1]; }
          enc_symbol(cs.enc, slot, bd.slot_words, lo, hi, cs.ovf);
          tgt[j] = (uint8_t)e;
        } else {
          int e;
          if (uniform) e = dec_symbol(cs.dec, slot, cs.nwords, V, [&](int s) { return (uint32_t)s * unit; });
          else {
            const uint32_t *c = cdf + j * (V + 1);
            e = dec_symbol(cs.dec, slot, cs.nwords, V, [&](int s) { return c[s]; });
          }
          ring[rp] = (uint8_t)e;
          tgt[j] = (uint8_t)e;
          toks[tok0 + (size_t)j * bd.L + i] = (uint8_t)e;
        }
        cst[j] = cs;
      }
      // mixing-weight gradient: per-row terms summed by a wave butterfly,
      // then the wave partials in order by thread 0
      if (d.static_on && !uniform && wave < (bs + 63) / 64) {
        float gt = 0.0f;
        if (tid < bs) gt = misc[tid] - lu[tid * VS + tgt[tid]];
        gt = wave_sum(gt);
        if (lane == 0) misc[bs + wave] = gt;
      }
      __syncthreads();

      if (!uniform) {
        pc.mark(3);
        // dz = (P - onehot)/bs (mean loss over the step's rows); dL^m = (1-alpha) dz
        // (four symbols per item; V = 4^k, so rows hold a power-of-two count of items)
        const int vq = V >> 2, vqs = __builtin_ctz((unsigned)vq);
        for (int q = tid; q < bs * vq; q += NT) {
          const int j = q >> vqs, v0 = (q & (vq - 1)) << 2, idx = j * VS + v0;
          const int tj = tgt[j];
          const float4 x4 = *reinterpret_cast<const float4 *>(lm + idx);
          float x[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
          for (int c = 0; c < 4; c++) {
            const float dz = (x[c] - (v0 + c == tj ? 1.0f : 0.0f)) * inv_bs;
            x[c] = d.static_on ? dz * (1.0f - alpha) : dz;
          }
          *reinterpret_cast<float4 *>(lm + idx) = make_float4(x[0], x[1], x[2], x[3]);
        }
        if (d.static_on && tid == 0) {
          float acc = 0.0f;
          for (int w = 0; w < (bs + 63) / 64; w++) acc += misc[bs + w];
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
        pc.mark(4);
        net.backward(W, M, Vs, i, opt);
        pc.mark(5);
        // embedding update from the fixed-point sums
        for (int q = tid; q < V * E; q += NT) {
          const int v = (int)__umulhi((uint32_t)q, d.Emag);
          const int qi = q + v * (d.ES - E), qp = q + v * (d.EP - E);
          float gq;
          if constexpr (Net::kOnChip) {
            (void)qi;
            gq = net.emb_grad(v, q - v * E);
          } else {
            gq = (float)((double)demb[qi] * (1.0 / (double)(1ull << kFixShift)));
            demb[qi] = 0;
          }
          const int pi = d.off_emb + q;
          emb[qp] = emb[qp] - opt_delta(opt, gq, M ? glb(M) + pi : nullptr, Vs ? glb(Vs) + pi : nullptr);
          if constexpr (Net::kOnChip) net.emb_set(v, q - v * E, emb[qp]);
        }
        if constexpr (Net::kOnChip) net.after_update(opt);
        if (d.static_on && tid == 0) {
          const float an = sh_a - opt_delta(opt, sh_ga, M ? glb(M) + d.P : nullptr, Vs ? glb(Vs) + d.P : nullptr);
          sh_a = an;
          glb(W)[d.P] = an;
        }
        __syncthreads();
      }
      pc.mark(6);
      if (bd.has_snap && i + 1 == (uint64_t)bd.S) snapshot();
      if (bd.has_snap && tid == 0)
        __hip_atomic_store(a.progress + b, (uint32_t)(i + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

    pc.flush();
    if constexpr (Net::kOnChip) net.flush(W);
    if (tid < bs) {
      CoderState cs = cst[tid];
      if (a.mode == 0) {
        enc_finish(cs.enc, slot_of(tid), bd.slot_words, cs.ovf);
        a.seg_bits[(size_t)b * bs + tid] = (uint32_t)cs.enc.nbits;
      }
      if (cs.ovf) atomicOr(a.err, 2);
    }
    // final parameters (embedding lives in LDS during the loop)
    for (int q = tid; q < V * E; q += NT) W[d.off_emb + q] = emb[q + (int)__umulhi((uint32_t)q, d.Emag) * (d.EP - E)];
    __syncthreads();
    if (a.params_out && b == 0)
      for (int q = tid; q < d.P + 1; q += NT) a.params_out[q] = W[q];
    __syncthreads();
  }
}


}  // namespace pmklc
