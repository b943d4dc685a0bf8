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
#pragma once
#include "step_common.h"

#include <type_traits>

namespace pmklc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) u32x2 gu32x2;

// the BF16 roundings (nearest even) of lo and hi as one 32-bit word, lo in
// the low half (one packed conversion)
__device__ __forceinline__ uint32_t bf16x2_bits(float lo, float hi) {
  typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
  const bf16x2 v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}

// x taken from the lane of this lane's quad that the DPP quad_perm pattern
// PAT (four 2-bit source indices, lowest first) names
template <int PAT>
__device__ __forceinline__ uint32_t quad_perm(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, PAT, 0xF, 0xF, true);
}

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

// four consecutive floats (16-byte aligned) from LDS or global memory
__device__ __forceinline__ fvec4 vec4_at(const float *p) { return *reinterpret_cast<const fvec4 *>(p); }
__device__ __forceinline__ fvec4 vec4_at(const gfloat *p) { return ld4(p); }

// KL consecutive floats (16-byte aligned when KL >= 4) from LDS (F = float)
// or global memory (F = gfloat)
template <int KL, class F>
__device__ __forceinline__ void load_run(const F *p, float *v) {
  if constexpr (KL >= 4) {
#pragma unroll
    for (int q = 0; q < KL; q += 4) {
      const fvec4 x = vec4_at(p + q);
      v[q] = x.x; v[q + 1] = x.y; v[q + 2] = x.z; v[q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int q = 0; q < KL; q++) v[q] = p[q];
  }
}
// KL floats with a stride
template <int KL, class F>
__device__ __forceinline__ void load_strided(const F *p, int stride, float *v) {
#pragma unroll
  for (int q = 0; q < KL; q++) v[q] = p[q * stride];
}

}  // namespace

// F1N: the F1 unit shape, 4 column tiles x MR1 row tiles (F1N = 4, for hidden
// widths in multiples of 64) or 2 x 1 (F1N = 2); one shape per kernel keeps
// the other's registers out of its allocation
template <int NT, class P, int MAXT, bool ADAM, int F1N>
struct NetMfma {
  static constexpr bool kOnChip = false;
  static constexpr int kSpl = 0;   // softmax symbols per lane: chosen at run time
  static constexpr int NW = NT / 64;
  static constexpr int KS = P::KS, KL = P::KL;   // MAXT = bs / 16 row tiles
  static constexpr int KC = 16 / KL;             // k-steps per streamed chunk (16 raw floats per lane)
  static constexpr int KB = 16 * MAXT / KS;      // k-steps over the bs rows
  // hidden tiles whose dpre^T fragments B4 keeps in registers (at most 4
  // tiles and about 32 VGPRs, next to two 4-tile W1 prefetch buffers)
  static constexpr int HB0 = 32 / (KB * (KL == 8 ? 4 : 1));
  static constexpr int HB = HB0 < 1 ? 1 : HB0 > 4 ? 4 : HB0;
  static constexpr int TB = NT >= 512 ? 2 : 4;   // B4 d tiles whose W1 values are loaded together
  static constexpr int NC1 = 4;                  // F1 column tiles per unit
  static constexpr int HCH = NT >= 512 ? 4 : 8;  // hidden tiles per chunk of the fused B3/B4
  static constexpr int MR1 = MAXT % 2 == 0 ? 2 : 1;   // F1 row tiles per unit
  typedef typename P::frag frag;
  typedef __attribute__((address_space(1))) frag gfrag;
  typedef __attribute__((address_space(1))) __bf16 gbf16;
  const StepArgs &a;
  const Dims &d;
  unsigned char *lds;
  float *emb, *embs, *h1, *hs, *lm, *lu;
  uint8_t *ring;
  long long *demb;
  __bf16 *dpt;     // BF16 dpre^T in B4's A-fragment order (LDS), BF16 only
  __bf16 *dpb;     // BF16 dpre in B3's B-fragment order (LDS), BF16 only
  uint16_t *w1f;   // this workgroup's BF16 copy of W1 (fragment order), BF16 only
  int tid, lane, wave, r, g;
  PhaseClock *pc = nullptr;
  __device__ NetMfma(const StepArgs &a_, unsigned char *lds_) : a(a_), d(a_.d), lds(lds_) {
    emb = reinterpret_cast<float *>(lds + a.lay.emb);
    embs = reinterpret_cast<float *>(lds + a.lay.embs);
    h1 = reinterpret_cast<float *>(lds + a.lay.act[0]);
    hs = reinterpret_cast<float *>(lds + a.lay.dh[0]);    // static hidden; later dpre
    lm = reinterpret_cast<float *>(lds + a.lay.lm);
    lu = reinterpret_cast<float *>(lds + a.lay.lu);
    ring = lds + a.lay.ring;
    demb = reinterpret_cast<long long *>(lds + a.lay.demb);
    dpt = reinterpret_cast<__bf16 *>(lds + a.lay.dpt);
    dpb = a.lay.dpb >= 0 ? reinterpret_cast<__bf16 *>(lds + a.lay.dpb) : nullptr;
    tid = threadIdx.x;
    lane = tid & 63;
    wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: branches on it stay scalar
    r = lane & 15;
    g = lane >> 4;
    w1f = a.w1f ? a.w1f + (size_t)blockIdx.x * d.D * d.H[0] : nullptr;
  }

  // a block starts from the parameters at src: fill the BF16 W1 copy (the
  // caller's barrier orders it before the first forward)
  __device__ void begin_block(const float *src) {
    if constexpr (KL == 8) {
      const int D = d.D, H = d.H[0];
      const gfloat *W1 = glb(src) + d.off_W[0];
      gbf16 *out = (gbf16 *)w1f;
      for (int q = tid; q < D * H; q += NT) {
        const int dd = q / H, h = q - dd * H;
        out[w1_frag_index(dd, h, D)] = (__bf16)W1[q];
      }
    }
  }

  // B4's A fragment of dpre^T: hidden tile ht, k-step kb of the rows j
  __device__ __forceinline__ frag dpre_frag(int ht, int kb) const {
    if constexpr (KL == 8) {
      return *reinterpret_cast<const bf16x8 *>(dpt + (((size_t)ht * KB + kb) * 64 + lane) * 8);
    } else {
      return hs[(kb * KS + g) * d.HP + 16 * ht + r];
    }
  }
  __device__ __forceinline__ frag ones_frag() const {
    float o[KL];
#pragma unroll
    for (int q = 0; q < KL; q++) o[q] = 1.0f;
    return P::pack(o);
  }
  __device__ __forceinline__ frag zero_frag() const {
    float z[KL];
#pragma unroll
    for (int q = 0; q < KL; q++) z[q] = 0.0f;
    return P::pack(z);
  }

  // a k-step of the streamed operand as loaded: KL raw floats (packed at
  // use) or a ready fragment (the BF16 W1 copy)
  struct RawF { float v[KL]; };
  __device__ static frag to_frag(const RawF &x) { return P::pack(x.v); }
  __device__ static frag to_frag(const frag &x) { return x; }

  // acc[m][n] += A_m(ks) B_n(ks) over k-steps 0..ksteps-1, with the NN
  // streamed operands (B_n, or A_n when SA) fetched from global memory in
  // chunks of KCX k-steps, the next chunk in flight while the current one is
  // used.  load(ks, n, buf) issues the loads of k-step ks of operand n;
  // reg(m, ks) gives the register operand of tile m (gathered a few k-steps
  // at a time before their MFMAs, so the LDS round trips overlap, and each
  // used for NN MFMAs).  Every fetch is issued unconditionally (addresses
  // clamped to the last k-step), which keeps the in-order memory counter
  // exact (a scheduling barrier pins each chunk's loads ahead of the
  // previous chunk's MFMAs); chunks go in pairs, and k-steps past the end
  // multiply a zero fragment, leaving acc exact.
  template <int NM, int NN, bool SA, int KCX, class Buf, class LD, class RG>
  __device__ __forceinline__ void stream2(int ksteps, f32x4 (*acc)[NN], LD &&load, RG &&reg) const {
    Buf bufA[KCX][NN], bufB[KCX][NN];
    const int nch = (ksteps + KCX - 1) / KCX;
    const bool ragged = (ksteps % (2 * KCX)) != 0;
    auto fetch = [&](int ch, Buf (&buf)[KCX][NN]) {
#pragma unroll
      for (int c = 0; c < KCX; c++)
#pragma unroll
        for (int n = 0; n < NN; n++) load(min(ch * KCX + c, ksteps - 1), n, buf[c][n]);
      __builtin_amdgcn_sched_barrier(0);
    };
    // register operands are gathered GC k-steps at a time (about 8 fragments)
    constexpr int GC0 = NM >= 8 ? 1 : 8 / NM, GC = GC0 < KCX ? GC0 : KCX;
    static_assert(KCX % GC == 0, "gather groups must tile the chunk");
    // CHK: this chunk may hold k-steps past the end (only the last pair of a
    // ragged stream), whose streamed fragments are zeroed
    auto use = [&](auto chk, int ch, Buf (&buf)[KCX][NN]) {
      constexpr bool CHK = decltype(chk)::value;
#pragma unroll
      for (int c0 = 0; c0 < KCX; c0 += GC) {
        frag o[GC][NM];
#pragma unroll
        for (int c = 0; c < GC; c++)
#pragma unroll
          for (int m = 0; m < NM; m++) o[c][m] = reg(m, min(ch * KCX + c0 + c, ksteps - 1));
#pragma unroll
        for (int c = 0; c < GC; c++) {
          const bool past = CHK && ch * KCX + c0 + c >= ksteps;
#pragma unroll
          for (int n = 0; n < NN; n++) {
            frag sf = to_frag(buf[c0 + c][n]);
            if (past) sf = zero_frag();
#pragma unroll
            for (int m = 0; m < NM; m++)
              acc[m][n] = SA ? P::mma(sf, o[c][m], acc[m][n]) : P::mma(o[c][m], sf, acc[m][n]);
          }
        }
      }
    };
    fetch(0, bufA);
    for (int ch = 0; ch < nch; ch += 2) {
      const bool tail = ragged && ch + 2 >= nch;   // uniform
      fetch(ch + 1, bufB);
      if (tail) use(std::true_type{}, ch, bufA);
      else use(std::false_type{}, ch, bufA);
      fetch(ch + 2, bufA);
      if (tail) use(std::true_type{}, ch + 1, bufB);
      else use(std::false_type{}, ch + 1, bufB);
    }
  }
  // one streamed operand
  template <int NM, bool SA, int KCX, class Buf, class LD, class RG>
  __device__ __forceinline__ void stream(int ksteps, f32x4 *acc, LD &&load, RG &&reg) const {
    stream2<NM, 1, SA, KCX, Buf>(ksteps, reinterpret_cast<f32x4 (*)[1]>(acc),
                                 [&](int ks, int, Buf &b) { load(ks, b); }, reg);
  }
  // the common case: KC k-steps of raw floats per chunk
  template <int NM, bool SA, class LD, class RG>
  __device__ __forceinline__ void stream(int ksteps, f32x4 *acc, LD &&load, RG &&reg) const {
    stream<NM, SA, KC, RawF>(ksteps, acc, [&](int ks, RawF &b) { load(ks, b.v); }, reg);
  }

  // an LDS array by byte offset (selecting offsets, not pointers, keeps the
  // compiler from building a pointer table in scratch)
  __device__ __forceinline__ float *lds_f(int off) const { return reinterpret_cast<float *>(lds + off); }

  // token of context position p (0..t-1) of row j at step i
  __device__ __forceinline__ int token(int j, int p, uint64_t i) const {
    return ring[((((int)(i - (uint64_t)d.t) + p) & (d.RS - 1))) * d.bs + j];
  }
  __device__ __forceinline__ void split_k(int kk, int &p, int &e) const {
    p = (int)__umulhi((uint32_t)kk, d.Emag);
    e = kk - p * d.E;
  }

  __device__ void forward(float *W, uint64_t i, float alpha) {
    (void)alpha;
    const int H = d.H[0], HP = d.HP, V = d.V, D = d.D;
    const int nmod = d.static_on ? 2 : 1;
    drain_stores();
    // F1: X W1 + b1, ReLU.  A unit is NC column tiles x MR row tiles of one
    // model: each gathered X fragment feeds NC MFMAs, so X is gathered
    // H/(16 NC) times per model.  NC = 4, MR = MR1 when the column tiles come
    // in fours (F1N = 4), else NC = 2, MR = 1 (more units, no repeated columns); column
    // tiles past the end repeat the last one and are not stored.  Each output
    // tile is one chain over the k-steps in order, whatever the unit shape.
    auto f1 = [&](auto nc_c, auto mr_c) {
      constexpr int NC = decltype(nc_c)::value, MR = decltype(mr_c)::value;
      const int HT = H / 16, CG = (HT + NC - 1) / NC, RG = MAXT / MR;
      const int units = nmod * CG * RG;
      for (int u = wave; u < units; u += NW) {
        const int model = u / (CG * RG), rem = u - model * (CG * RG), cg = rem / RG, rg = rem - cg * RG;
        const gfloat *Wm = glb(model ? a.stat : W);
        const float *em = lds_f(model ? a.lay.embs : a.lay.emb);
        int ncol[NC];
        float bias[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) {
          ncol[c] = min(cg * NC + c, HT - 1);
          bias[c] = Wm[d.off_b[0] + 16 * ncol[c] + r];
        }
        f32x4 acc[MR][NC];
#pragma unroll
        for (int mm = 0; mm < MR; mm++)
#pragma unroll
          for (int c = 0; c < NC; c++) acc[mm][c] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        auto xfrag = [&](int mm, int ks) {
          int p, e;
          split_k(ks * KS + g * KL, p, e);
          float av[KL];
          load_run<KL>(em + token(16 * (rg * MR + mm) + r, p, i) * d.EP + e, av);
          return P::pack(av);
        };
        if constexpr (KL == 8) {
          // BF16: one 16-byte load per lane, k-step and column tile from the
          // fragment-ordered copy, through a buffer descriptor over the copy
          // (the lane's slot as the vector offset, the tile and k-step as a
          // scalar one; a load past the copy would read 0)
          const uint16_t *copy = model ? a.s1f : w1f;
          const __amdgpu_buffer_rsrc_t rs =
              __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t *>(copy), (short)0, D * H * 2, 0x00020000);
          const int kst = D / KS, voff = lane * 16;
          stream2<MR, NC, false, 2, frag>(kst, acc,
              [&](int ks, int c, frag &b) {
                b = __builtin_bit_cast(frag, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, (ncol[c] * kst + ks) * 1024, 0));
              }, xfrag);
        } else {
          const gfloat *W1 = Wm + d.off_W[0] + r + (size_t)(g * KL) * H;
          stream2<MR, NC, false, 4, RawF>(D / KS, acc,
              [&](int ks, int c, RawF &b) { load_strided<KL>(W1 + 16 * ncol[c] + (size_t)ks * KS * H, H, b.v); }, xfrag);
        }
        float *out = lds_f(model ? a.lay.dh[0] : a.lay.act[0]);
#pragma unroll
        for (int c = 0; c < NC; c++) {
          if (cg * NC + c >= HT) break;
#pragma unroll
          for (int mm = 0; mm < MR; mm++)
#pragma unroll
            for (int q = 0; q < 4; q++)
              out[(16 * (rg * MR + mm) + 4 * g + q) * HP + 16 * ncol[c] + r] = fmaxf(acc[mm][c][q] + bias[c], 0.0f);
        }
      }
    };
    if constexpr (F1N == 4) f1(std::integral_constant<int, NC1>{}, std::integral_constant<int, MR1>{});
    else f1(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{});
    __syncthreads();
    pc->mark(7);
    // F2: H1 W2 + b2 -> logits
    for (int grp = wave; grp < nmod * (V / 16); grp += NW) {
      const int model = grp / (V / 16), n = grp % (V / 16);
      const gfloat *Wm = glb(model ? a.stat : W);
      const gfloat *wcol = Wm + d.off_W[1] + 16 * n + r + (size_t)(g * KL) * V;
      const float *hin = lds_f(model ? a.lay.dh[0] : a.lay.act[0]);
      const float bias = Wm[d.off_b[1] + 16 * n + r];   // issued before the k-loop
      f32x4 acc[MAXT];
#pragma unroll
      for (int m = 0; m < MAXT; m++) acc[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      stream<MAXT, false>(H / KS, acc,
          [&](int ks, float *v) { load_strided<KL>(wcol + (size_t)ks * KS * V, V, v); },
          [&](int m, int ks) {
            float av[KL];
            load_run<KL>(hin + (16 * m + r) * HP + ks * KS + g * KL, av);
            return P::pack(av);
          });
      float *out = lds_f(model ? a.lay.lu : a.lay.lm);
#pragma unroll
      for (int m = 0; m < MAXT; m++)
#pragma unroll
        for (int q = 0; q < 4; q++) out[(16 * m + 4 * g + q) * d.VS + 16 * n + r] = acc[m][q] + bias;
    }
    __syncthreads();
  }

  __device__ void backward(float *Wf, float *Mf, float *Vf, uint64_t i, const Opt &opt) {
    const int bs = d.bs, H = d.H[0], HP = d.HP, V = d.V, D = d.D;
    gfloat *W = glb(Wf), *M = Mf ? glb(Mf) : nullptr, *Vs = Vf ? glb(Vf) : nullptr;
    gfloat *W1 = W + d.off_W[0], *W2 = W + d.off_W[1];
    float *dpre = hs;
    constexpr bool adam = ADAM;   // fixed per kernel: no optimiser branch in the update loops
    drain_stores();
    // BF16: the biases are updated after the backward from gradients gathered
    // in LDS (gb below, hidden first); each thread's first one is loaded now
    // so that its latency hides behind the backward
    auto bias_at = [&](int c) { return c < H ? d.off_b[0] + c : d.off_b[1] + (c - H); };
    float b_old = 0.0f;
    if (KL == 8 && tid < V + H) b_old = W[bias_at(tid)];
    // B1 + B2, fused per hidden tile n (a wave per tile).  Lane (r, g) loads
    // W2[16n + r][16m + 4g .. +3] for a chunk of 4 symbol tiles m: these are
    // the values its B2 output tile updates, and, with the contraction index v
    // of B1 permuted to match (BF16 k-slot q: v = 32k + 4g + q for q < 4,
    // 32k + 16 + 4g + q - 4 otherwise; FP32 k-step 4m + i: v = 16m + 4g + i;
    // dz gathered the same way), B1's B operand, so W2 is read once.
    //   B1: dpre = (dz W2^T) * [H1 > 0]   (old W2; all chunks)
    //   B2: dW2^T = dz^T H1 -> W2 update  (per chunk, after B1 has used it)
    {
      gfloat *M2 = M ? M + d.off_W[1] : nullptr, *V2 = Vs ? Vs + d.off_W[1] : nullptr;
      const int VT = V / 16;
      for (int n = wave; n < H / 16; n += NW) {
        f32x4 acc1[MAXT];
#pragma unroll
        for (int m = 0; m < MAXT; m++) acc1[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        // H1 columns of this tile as B2's B operand (k = rows j), all k-steps
        frag hb[KB];
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
          float bv[KL];
          load_strided<KL>(h1 + (kb * KS + g * KL) * HP + 16 * n + r, HP, bv);
          hb[kb] = P::pack(bv);
        }
        for (int vc = 0; vc < VT; vc += 4) {
          fvec4 w[4];
#pragma unroll
          for (int m = 0; m < 4; m++)   // W2[h][v .. v+3]
            w[m] = ld4(W2 + (size_t)(16 * n + r) * V + 16 * min(vc + m, VT - 1) + 4 * g);
          // B2 (LDS operands only) while the loads are in flight
          f32x4 acc2[4];
#pragma unroll
          for (int m = 0; m < 4; m++) {
            acc2[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int kb = 0; kb < KB; kb++) {
              float av[KL];
              load_strided<KL>(lm + (kb * KS + g * KL) * d.VS + 16 * min(vc + m, VT - 1) + r, d.VS, av);
              acc2[m] = P::mma(P::pack(av), hb[kb], acc2[m]);
            }
          }
          // B1 over this chunk's symbols (tiles past the end contribute zero)
          if constexpr (KL == 8) {
#pragma unroll
            for (int k = 0; k < 2; k++) {
              const bool v0 = vc + 2 * k < VT, v1 = vc + 2 * k + 1 < VT;
              float bv[8] = {v0 ? w[2 * k].x : 0.0f, v0 ? w[2 * k].y : 0.0f, v0 ? w[2 * k].z : 0.0f,
                             v0 ? w[2 * k].w : 0.0f, v1 ? w[2 * k + 1].x : 0.0f, v1 ? w[2 * k + 1].y : 0.0f,
                             v1 ? w[2 * k + 1].z : 0.0f, v1 ? w[2 * k + 1].w : 0.0f};
              const frag b1f = P::pack(bv);
              const int c0 = 16 * min(vc + 2 * k, VT - 1) + 4 * g, c1 = 16 * min(vc + 2 * k + 1, VT - 1) + 4 * g;
#pragma unroll
              for (int m = 0; m < MAXT; m++) {
                float av[8];
                load_run<4>(lm + (16 * m + r) * d.VS + c0, av);
                load_run<4>(lm + (16 * m + r) * d.VS + c1, av + 4);
                acc1[m] = P::mma(P::pack(av), b1f, acc1[m]);
              }
            }
          } else {
#pragma unroll
            for (int mv = 0; mv < 4; mv++) {
              const bool ok = vc + mv < VT;
              const int cb = 16 * min(vc + mv, VT - 1) + 4 * g;
#pragma unroll
              for (int q = 0; q < 4; q++) {
                const float bv = ok ? w[mv][q] : 0.0f;
#pragma unroll
                for (int m = 0; m < MAXT; m++) acc1[m] = P::mma(lm[(16 * m + r) * d.VS + cb + q], bv, acc1[m]);
              }
            }
          }
          // W2 update of this chunk
#pragma unroll
          for (int m = 0; m < 4; m++) {
            if (vc + m >= VT) break;
            const size_t idx = (size_t)(16 * n + r) * V + 16 * (vc + m) + 4 * g;
            float wv[4] = {w[m].x, w[m].y, w[m].z, w[m].w};
            fvec4 mo = fvec4{0.0f, 0.0f, 0.0f, 0.0f}, vo = mo;
            if constexpr (adam) {
              mo = ld4(M2 + idx);
              vo = ld4(V2 + idx);
            }
            float mv[4] = {mo.x, mo.y, mo.z, mo.w};
            float vv[4] = {vo.x, vo.y, vo.z, vo.w};
#pragma unroll
            for (int q = 0; q < 4; q++) wv[q] = wv[q] - opt_delta_c<ADAM>(opt, acc2[m][q], &mv[q], &vv[q]);
            st4(W2 + idx, fvec4{wv[0], wv[1], wv[2], wv[3]});
            if constexpr (adam) {
              st4(M2 + idx, fvec4{mv[0], mv[1], mv[2], mv[3]});
              st4(V2 + idx, fvec4{vv[0], vv[1], vv[2], vv[3]});
            }
          }
        }
        // dpre = B1 * [H1 > 0] (and its BF16 transpose for B4)
#pragma unroll
        for (int m = 0; m < MAXT; m++) {
          float dv[4];
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const int idx = (16 * m + 4 * g + q) * HP + 16 * n + r;
            dv[q] = h1[idx] > 0.0f ? acc1[m][q] : 0.0f;
            dpre[idx] = dv[q];
          }
          if constexpr (KL == 8) {
            // BF16 dpre^T as B4's A fragments: tile n of h, k-step m/2 of j;
            // this lane's 4 rows j are 4 consecutive slots of lane r + 16 (2 (m%2) + g/2)
            bf16x4 pk;
#pragma unroll
            for (int q = 0; q < 4; q++) pk[q] = (__bf16)dv[q];
            const int slot = r + 16 * (2 * (m & 1) + (g >> 1));
            *reinterpret_cast<bf16x4 *>(dpt + (((size_t)n * KB + (m >> 1)) * 64 + slot) * 8 + 4 * (g & 1)) = pk;
            // and dpre as B3's B fragments: row tile m of j, k-step n/2 of h with
            // B3's slot order (q < 4: h = 32k + 4g' + q; q >= 4: h = 32k + 16 + 4g' + q - 4),
            // so h = 16n + r sits in lane (4g + i) + 16 (r/4), slot 4 (n%2) + r%4
            if (dpb) {
              __bf16 *pb = dpb + ((m * (H / 32) + (n >> 1)) * 64 + 4 * g + 16 * (r >> 2)) * 8 + 4 * (n & 1) + (r & 3);
#pragma unroll
              for (int q = 0; q < 4; q++) pb[8 * q] = pk[q];
            }
          }
        }
      }
    }
    __syncthreads();
    pc->mark(8);
    pc->mark(11);
    // (no store drain here: the W2 update's stores complete behind the first
    // chunk's B4 MFMAs, and every later wait of this phase follows W1 stores)
    // bias gradients (BF16): H1 is dead from here to the next forward
    float *gb = h1;
    // B3 + B4, fused per tile of 16 rows d of W1 (a wave takes d tiles
    // wave, wave + NW, ...).  Lane (r, g) loads W1[d][16m + 4g .. +3] for the
    // hidden tiles m of a chunk of HCH: these are the values its B4 output tile
    // updates, and, with the contraction index h of B3 permuted to match
    // (k-slot q of a BF16 k-step: h = 32k + 4g + q for q < 4, 32k + 16 + 4g +
    // q - 4 otherwise; FP32 k-step 4m + i: h = 16m + 4g + i, gathered the same
    // way from dpre), also B3's A operand, so W1 is read once.  B4's MFMAs
    // need only LDS operands and run while the loads are in flight.
    //   B3: dX^T[d][j] = sum_h W1[d][h] dpre[j][h] -> embedding-gradient scatter
    //   B4: dW1^T[h][d] = sum_j dpre^T[h][j] X[j][d] -> W1 update
    {
      gfloat *M1 = M ? M + d.off_W[0] : nullptr, *V1 = Vs ? Vs + d.off_W[0] : nullptr;
      const int HT = H / 16, DT = D / 16, NHC = (HT + HCH - 1) / HCH;
      // output-bias gradient sum_j dz[j][v] (BF16, as an MFMA against a ones
      // fragment): symbol tiles from the last wave down
      if constexpr (KL == 8) {
        for (int vt = NW - 1 - wave; vt < V / 16; vt += NW) {
          f32x4 accb = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int kb = 0; kb < KB; kb++) {
            float av[KL];
            load_strided<KL>(lm + (kb * KS + g * KL) * d.VS + 16 * vt + r, d.VS, av);
            accb = P::mma(P::pack(av), ones_frag(), accb);
          }
          if (r == 0) {
#pragma unroll
            for (int q = 0; q < 4; q++) gb[H + 16 * vt + 4 * g + q] = accb[q];
          }
        }
      }
      for (int mt = wave; mt < DT; mt += NW) {
        const int dd = 16 * mt + r;
        // BF16 copy offset of this lane's quad-transposed store for hidden tile
        // 0; tile ht adds 16 D (the copy's column tiles are D/32 k-steps of 512)
        const uint32_t w1f_base = KL == 8 ? w1_frag_index(16 * mt + (r & ~3), 4 * g + (lane & 3), D) : 0u;
        int p, e;
        split_k(dd, p, e);
        // X^T fragments of this d tile (B4's B operand)
        frag bf[KB];
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
          float bv[KL];
#pragma unroll
          for (int q = 0; q < KL; q++) bv[q] = emb[token(kb * KS + g * KL + q, p, i) * d.EP + e];
          bf[kb] = P::pack(bv);
        }
        f32x4 acc3[MAXT];
#pragma unroll
        for (int n = 0; n < MAXT; n++) acc3[n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int hc = 0; hc < NHC; hc++) {
          fvec4 w[HCH];
#pragma unroll
          for (int m = 0; m < HCH; m++)
            w[m] = ld4(W1 + (size_t)dd * H + 16 * min(HCH * hc + m, HT - 1) + 4 * g);
          __builtin_amdgcn_sched_barrier(0);
          // B4 (LDS operands only)
          f32x4 acc4[HCH];
#pragma unroll
          for (int m = 0; m < HCH; m++) acc4[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
          auto b4 = [&](auto full_chunk) {
            constexpr bool FULL = decltype(full_chunk)::value;
#pragma unroll
            for (int m = 0; m < HCH; m++) {
              if (!FULL && HCH * hc + m >= HT) break;   // (tiles past the end are neither used nor stored)
              const int ht = HCH * hc + m;
#pragma unroll
              for (int kb = 0; kb < KB; kb++) acc4[m] = P::mma(dpre_frag(ht, kb), bf[kb], acc4[m]);
            }
          };
          if (HCH * (hc + 1) <= HT) b4(std::true_type{});
          else b4(std::false_type{});
          // hidden-bias gradient sum_j dpre[j][h] (BF16): the wave of d tile 0
          // multiplies the dpre^T fragments by a ones fragment (column 0)
          if (KL == 8 && mt == 0) {
#pragma unroll
            for (int m = 0; m < HCH; m++) {
              if (HCH * hc + m >= HT) break;
              f32x4 accb = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
              for (int kb = 0; kb < KB; kb++) accb = P::mma(dpre_frag(HCH * hc + m, kb), ones_frag(), accb);
              if (r == 0) {
#pragma unroll
                for (int q = 0; q < 4; q++) gb[16 * (HCH * hc + m) + 4 * g + q] = accb[q];
              }
            }
          }
          // B3 over this chunk's hidden units (tiles past the end contribute
          // zero; a full chunk needs no test)
          if constexpr (KL == 8) {
            auto b3_bf16 = [&](auto full_chunk) {
              constexpr bool FULL = decltype(full_chunk)::value;
#pragma unroll
              for (int k = 0; k < HCH / 2; k++) {
                const bool v0 = FULL || HCH * hc + 2 * k < HT, v1 = FULL || HCH * hc + 2 * k + 1 < HT;
                if (!v0) break;   // both tiles past the end
                float av[8] = {v0 ? w[2 * k].x : 0.0f, v0 ? w[2 * k].y : 0.0f, v0 ? w[2 * k].z : 0.0f,
                               v0 ? w[2 * k].w : 0.0f, v1 ? w[2 * k + 1].x : 0.0f, v1 ? w[2 * k + 1].y : 0.0f,
                               v1 ? w[2 * k + 1].z : 0.0f, v1 ? w[2 * k + 1].w : 0.0f};
                const frag a3 = P::pack(av);
                if (dpb) {
                  // B3's B fragments from the BF16 copy of dpre (k-steps past the end
                  // clamped; their A operand is zero)
                  const int ks3 = min((HCH * hc) / 2 + k, H / 32 - 1);
#pragma unroll
                  for (int n = 0; n < MAXT; n++)
                    acc3[n] = P::mma(a3, *reinterpret_cast<const bf16x8 *>(dpb + ((n * (H / 32) + ks3) * 64 + lane) * 8),
                                     acc3[n]);
                } else {
                  const int h0 = 16 * min(HCH * hc + 2 * k, HT - 1) + 4 * g, h1c = 16 * min(HCH * hc + 2 * k + 1, HT - 1) + 4 * g;
#pragma unroll
                  for (int n = 0; n < MAXT; n++) {
                    float bv[8];
                    load_run<4>(dpre + (16 * n + r) * HP + h0, bv);
                    load_run<4>(dpre + (16 * n + r) * HP + h1c, bv + 4);
                    acc3[n] = P::mma(a3, P::pack(bv), acc3[n]);
                  }
                }
              }
            };
            if (HCH * (hc + 1) <= HT) b3_bf16(std::true_type{});
            else b3_bf16(std::false_type{});
          } else {
#pragma unroll
            for (int m = 0; m < HCH; m++) {
              const bool vm = HCH * hc + m < HT;
              const int hb = 16 * min(HCH * hc + m, HT - 1) + 4 * g;
#pragma unroll
              for (int q = 0; q < 4; q++) {
                const float av = vm ? w[m][q] : 0.0f;
#pragma unroll
                for (int n = 0; n < MAXT; n++) acc3[n] = P::mma(av, dpre[(16 * n + r) * HP + hb + q], acc3[n]);
              }
            }
          }
          // B4 update of this chunk
#pragma unroll
          for (int m = 0; m < HCH; m++) {
            if (HCH * hc + m >= HT) break;
            const size_t idx = (size_t)dd * H + 16 * (HCH * hc + m) + 4 * g;
            float wv[4] = {w[m].x, w[m].y, w[m].z, w[m].w};
            fvec4 mo = fvec4{0.0f, 0.0f, 0.0f, 0.0f}, vo = mo;
            if constexpr (adam) {
              mo = ld4(M1 + idx);
              vo = ld4(V1 + idx);
            }
            float mv[4] = {mo.x, mo.y, mo.z, mo.w};
            float vv[4] = {vo.x, vo.y, vo.z, vo.w};
#pragma unroll
            for (int q = 0; q < 4; q++) wv[q] = wv[q] - opt_delta_c<ADAM>(opt, acc4[m][q], &mv[q], &vv[q]);
            st4(W1 + idx, fvec4{wv[0], wv[1], wv[2], wv[3]});
            if constexpr (KL == 8) {
              // BF16 copy: the four lanes of a quad hold 4 consecutive d and
              // each the same 4 consecutive h; a 4x4 transpose of the 16-bit
              // values inside the quad leaves lane c with h = 4g + c at those
              // 4 d, which are 8 contiguous bytes of the fragment-ordered copy
              const uint32_t c = lane & 3u;
              const uint32_t p01 = bf16x2_bits(wv[0], wv[1]), p23 = bf16x2_bits(wv[2], wv[3]);
              // lanes c and c ^ 2 swap a dword: afterwards lane c = 2s + t holds
              // A = (x[t][2s], x[t][2s+1]) and B = (x[2+t][2s], x[2+t][2s+1]),
              // x[c'][q] being value q of quad lane c'
              const uint32_t x2 = quad_perm<0x4E>(c < 2 ? p23 : p01);
              const uint32_t A = c < 2 ? p01 : x2, B = c < 2 ? x2 : p23;
              // lanes c and c ^ 1 swap a half of each: an odd lane sends its low
              // half and keeps its high one, an even lane the reverse; one byte
              // permutation then joins kept and received halves into
              // E = (x[0][c], x[1][c]), F = (x[2][c], x[3][c])
              const uint32_t sh = (c & 1u) ? 0u : 16u, sel = (c & 1u) ? 0x03020504u : 0x05040100u;
              const uint32_t ya = quad_perm<0xB1>(A >> sh), yb = quad_perm<0xB1>(B >> sh);
              const uint32_t E = __builtin_amdgcn_perm(ya, A, sel), F = __builtin_amdgcn_perm(yb, B, sel);
              gu32x2 *cp = (gu32x2 *)(w1f + w1f_base + (uint32_t)(HCH * hc + m) * ((uint32_t)D << 4));
              *cp = u32x2{E, F};
            }
            if constexpr (adam) {
              st4(M1 + idx, fvec4{mv[0], mv[1], mv[2], mv[3]});
              st4(V1 + idx, fvec4{vv[0], vv[1], vv[2], vv[3]});
            }
          }
        }
        // embedding-gradient scatter of dX^T[d][j] in 64-bit fixed point; this
        // lane's 4 consecutive d are 4 consecutive embedding columns of one
        // context position (E is a multiple of 8), so one token per row
        {
          int p0, e0;
          split_k(16 * mt + 4 * g, p0, e0);
#pragma unroll
          for (int n = 0; n < MAXT; n++) {
            unsigned long long *row =
                reinterpret_cast<unsigned long long *>(demb + token(16 * n + r, p0, i) * d.ES + e0);
#pragma unroll
            for (int q = 0; q < 4; q++) atomicAdd(row + q, (unsigned long long)to_fixed(acc3[n][q]));
          }
        }
      }
    }
    if constexpr (KL != 8) {
      // FP32: bias gradients as plain column sums of dz and dpre
      for (int c = tid; c < V + H; c += NT) {
        const bool out = c < V;
        const float *src = out ? lm + c : dpre + (c - V);
        const int pitch = out ? d.VS : HP;
        float gsum = 0.0f;
        for (int j = 0; j < bs; j++) gsum += src[j * pitch];
        const int bi = out ? d.off_b[1] + c : d.off_b[0] + (c - V);
        W[bi] = W[bi] - opt_delta_c<ADAM>(opt, gsum, M ? M + bi : nullptr, Vs ? Vs + bi : nullptr);
      }
    }
    __syncthreads();
    if constexpr (KL == 8) {
      // BF16 bias updates (nothing reads the biases or H1 before the next
      // step's forward, so no barrier follows)
      for (int c = tid; c < V + H; c += NT) {
        const int bi = bias_at(c);
        const float old = c == tid ? b_old : W[bi];
        W[bi] = old - opt_delta_c<ADAM>(opt, gb[c], M ? M + bi : nullptr, Vs ? Vs + bi : nullptr);
      }
    }
    pc->mark(10);
  }
};

template <int NT, class P, int MT, bool ADAM, int F1N>
__global__ __launch_bounds__(NT) void step_mfma_kernel(const StepArgs *__restrict__ args) {
  extern __shared__ __align__(16) unsigned char lds[];
  const StepArgs &a = *args;
  NetMfma<NT, P, MT, ADAM, F1N> net(a, lds);
  run_blocks<NT>(a, lds, net);
}

template <int NT, class P, int MT, bool ADAM, int F1N>
hipError_t launch_one(const StepArgs *a_dev, int grid, size_t lds, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_mfma_kernel<NT, P, MT, ADAM, F1N>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((step_mfma_kernel<NT, P, MT, ADAM, F1N>), dim3(grid), dim3(NT), lds, st, a_dev);
  return hipGetLastError();
}

template <int NT, class P, bool ADAM, int F1N>
hipError_t launch_mt(const StepArgs *a_dev, int grid, int mt, size_t lds, hipStream_t st) {
  if (mt == 2) return launch_one<NT, P, 2, ADAM, F1N>(a_dev, grid, lds, st);
  if (mt == 4) return launch_one<NT, P, 4, ADAM, F1N>(a_dev, grid, lds, st);
  if (mt == 6) return launch_one<NT, P, 6, ADAM, F1N>(a_dev, grid, lds, st);
  if (mt == 8) return launch_one<NT, P, 8, ADAM, F1N>(a_dev, grid, lds, st);
  return hipErrorInvalidValue;
}

template <int NT, class P, bool ADAM>
hipError_t launch_f1(const StepArgs *a_dev, int grid, int mt, bool f1_fours, size_t lds, hipStream_t st) {
  return f1_fours ? launch_mt<NT, P, ADAM, 4>(a_dev, grid, mt, lds, st) : launch_mt<NT, P, ADAM, 2>(a_dev, grid, mt, lds, st);
}

}  // namespace pmklc
