// Step kernel for small dynamic models with the whole network on chip for
// the life of a block: one hidden layer, SGD, no static model, the shape
// fixed at compile time (one instance per supported shape, 512 threads).
//
// The model GEMMs run on the matrix cores in BF16 with FP32 accumulation
// (Sec. 4.2.4 with the MLP reading; Sec. 2 steps (3)-(4)); softmax,
// quantiser, coder and the FP32 master weights are as in the other step
// kernels (the loop around the network is run_blocks in step_common.h).
// Where the weights live during a block:
//   W1 (D x H) FP32 master: registers.  Lane (r, g) of wave w owns
//     W1[16 mt + r][16 m + 4 g + c] for its d tiles mt = w, w + 8, ... and
//     every hidden tile m: exactly the elements its B4 output tiles update,
//     and, read as B3's B operand, the W1^T fragments B3 needs.
//   W1 BF16 copy: LDS, in F1's B-fragment order (w1_frag_index), rewritten
//     next to the master by the update.
//   W2 (H x V) FP32, transposed (V x H): LDS; biases: LDS.
// So a step reads and writes no weight in global memory; the parameter slab
// is written back only for a model-passing snapshot and at the block's end.
//
// Operand layout of a 16x16 tile (lane l, r = l % 16, g = l / 16):
//   16x16x32 BF16: A[r][8g .. 8g+7], B[8g .. 8g+7][r], C[4g+c][r] (c = 0..3)
// Per step, rows j (BS), inputs d (D = T E), hidden h (H), symbols v (V):
//   F1  H1 = ReLU(X W1 + b1)              units: row tiles (all hidden tiles)
//   F2  L  = H1 W2 + b2                   units (row tile, symbol tile)
//   B1  dpre = (dz W2^T) * [H1 > 0]       units (row tile, hidden tile)
//   B2  dW2^T = dz^T H1 -> W2 update      units (symbol tile, hidden tile)
//   B3  dX = dpre W1^T                    per d tile, by the tile's W1 owner
//   B4  dW1^T = dpre^T X -> W1 update     per d tile
//   EG  dEmb = onehot(ctx)^T dX           per d tile: with E = 16 a d tile is
//       one context position p, and sum_j [ctx_j,p = v] dX[j][16p + e] is a
//       product of one-hot fragments and B3's output as it lies in the
//       accumulators (two row tiles' C layouts make one B fragment)
// Every output element is one MFMA accumulation chain in a fixed order; the
// embedding gradient is one chain per wave (its d tiles in order) and the
// eight wave partials are added in wave order, so encode and decode agree
// bit for bit.
#include "step_mfma.h"

namespace pmklc {

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 bf8(const float *v) {
  bf16x8 f;
#pragma unroll
  for (int q = 0; q < 8; q++) f[q] = (__bf16)v[q];
  return f;
}
constexpr int ring_len(int t) {   // smallest power of two >= t + 32 (the staging width)
  int rs = 1;
  while (rs < t + 32) rs <<= 1;
  return rs;
}

template <int BS, int T, int E, int H, int V>
struct NetChip {
  static constexpr bool kOnChip = true;
  static constexpr int kSpl = V / 8;   // softmax symbols per lane (V >= 32)
  static constexpr int NT = 512, NW = NT / 64;
  static constexpr int D = T * E, DT = D / 16, MT = BS / 16, HT = H / 16, VT = V / 16;
  static constexpr int KD = D / 32, KB = BS / 32, KH = H / 32, KV = V / 32;
  static constexpr int DTW = DT / NW;                       // d tiles per wave
  static constexpr int HP = H + 4, VS = V + 4, EP = E + 4;  // LDS row pitches (floats), as in the layout
  static constexpr int W2P = H + 4;                          // pitch of W2^T rows
  static constexpr int EPH = E + 8;                          // pitch of the BF16 embedding rows (16-byte runs)
  static constexpr int RS = ring_len(T);
  static_assert(E == 16, "a d tile is one context position");
  static_assert(H % 32 == 0 && V % 32 == 0 && BS % 32 == 0 && DT % NW == 0, "tile multiples");

  const StepArgs &a;
  const Dims &d;
  unsigned char *lds;
  float *emb, *h1, *lm, *w2t, *bias, *gb, *eg;
  uint8_t *ring;
  __bf16 *dpt, *dpb, *w1c, *embh;
  int tid, lane, wave, r, g;
  float w1m[DTW][HT][4];
  PhaseClock *pc = nullptr;

  __device__ NetChip(const StepArgs &a_, unsigned char *lds_) : a(a_), d(a_.d), lds(lds_) {
    emb = reinterpret_cast<float *>(lds + a.lay.emb);
    h1 = reinterpret_cast<float *>(lds + a.lay.act[0]);
    lm = reinterpret_cast<float *>(lds + a.lay.lm);
    w2t = reinterpret_cast<float *>(lds + a.lay.w2t);
    bias = reinterpret_cast<float *>(lds + a.lay.bias);
    gb = reinterpret_cast<float *>(lds + a.lay.gb);
    eg = reinterpret_cast<float *>(lds + a.lay.eg);
    ring = lds + a.lay.ring;
    dpt = reinterpret_cast<__bf16 *>(lds + a.lay.dpt);
    dpb = reinterpret_cast<__bf16 *>(lds + a.lay.dpb);
    w1c = reinterpret_cast<__bf16 *>(lds + a.lay.w1c);
    embh = reinterpret_cast<__bf16 *>(lds + a.lay.embh);
    tid = threadIdx.x;
    lane = tid & 63;
    wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    r = lane & 15;
    g = lane >> 4;
  }

  // token of context position p (0..T-1) of row j at step i
  __device__ __forceinline__ int token(int j, int p, uint64_t i) const {
    return ring[((((int)(i - (uint64_t)T) + p) & (RS - 1))) * BS + j];
  }
  __device__ __forceinline__ size_t w1_at(int q, int m) const {   // W1 index of this lane's run (q, m)
    return (size_t)(16 * (wave + NW * q) + r) * H + 16 * m + 4 * g;
  }

  __device__ void begin_block(const float *src) {
    const gfloat *s = glb(src);
#pragma unroll
    for (int q = 0; q < DTW; q++)
#pragma unroll
      for (int m = 0; m < HT; m++) {
        const fvec4 v = ld4(s + d.off_W[0] + w1_at(q, m));
        w1m[q][m][0] = v.x; w1m[q][m][1] = v.y; w1m[q][m][2] = v.z; w1m[q][m][3] = v.w;
      }
    for (int x = tid; x < D * H; x += NT) {
      const int dd = x / H, h = x - dd * H;
      w1c[w1_frag_index(dd, h, D)] = (__bf16)s[d.off_W[0] + x];
    }
    for (int x = tid; x < H * V; x += NT) {
      const int h = x / V, v = x - h * V;
      w2t[v * W2P + h] = s[d.off_W[1] + x];
    }
    for (int x = tid; x < H + V; x += NT) bias[x] = s[x < H ? d.off_b[0] + x : d.off_b[1] + (x - H)];
  }

  // the layer parameters back into the slab (W1 from registers, W2 and the
  // biases from LDS); every thread calls it
  __device__ void flush(float *Wf) {
    gfloat *W = glb(Wf);
#pragma unroll
    for (int q = 0; q < DTW; q++)
#pragma unroll
      for (int m = 0; m < HT; m++)
        st4(W + d.off_W[0] + w1_at(q, m), fvec4{w1m[q][m][0], w1m[q][m][1], w1m[q][m][2], w1m[q][m][3]});
    for (int x = tid; x < H * V; x += NT) {
      const int h = x / V, v = x - h * V;
      W[d.off_W[1] + x] = w2t[v * W2P + h];
    }
    for (int x = tid; x < H + V; x += NT) W[x < H ? d.off_b[0] + x : d.off_b[1] + (x - H)] = bias[x];
  }

  // gradient of embedding element (v, e): the wave partials in wave order
  __device__ __forceinline__ float emb_grad(int v, int e) const {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < NW; w++) s += eg[(w * V + v) * E + e];
    return s;
  }
  // the BF16 embedding copy follows every write of the FP32 embedding
  __device__ __forceinline__ void emb_set(int v, int e, float x) { embh[v * EPH + e] = (__bf16)x; }
  // bias updates from the gradients gathered by the backward
  __device__ void after_update(const Opt &opt) {
    for (int c = tid; c < H + V; c += NT) bias[c] = bias[c] - opt_delta_c<false>(opt, gb[c], (float *)nullptr, (float *)nullptr);
  }

  __device__ void forward(float *, uint64_t i, float) {
    // F1: X W1 + b1, ReLU.  A unit is one row tile and every hidden tile:
    // each X fragment (8 consecutive inputs = 8 columns of one position, one
    // 16-byte read of the BF16 embedding) feeds HT MFMAs; W1 fragments come
    // from the LDS copy (one 16-byte read each)
    for (int rt = wave; rt < MT; rt += NW) {
      const int j = 16 * rt + r;
      f32x4 acc[HT];
#pragma unroll
      for (int n = 0; n < HT; n++) acc[n] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
      // every k-step's token first (independent reads, one wait), then the
      // fragments a few k-steps at a time
      int tk[KD];
#pragma unroll
      for (int ks = 0; ks < KD; ks++) tk[ks] = token(j, (32 * ks + 8 * g) / E, i);
      constexpr int KG = 4;
#pragma unroll
      for (int k0 = 0; k0 < KD; k0 += KG) {
        bf16x8 xa[KG], wf[KG][HT];
#pragma unroll
        for (int c = 0; c < KG; c++) {
          xa[c] = *reinterpret_cast<const bf16x8 *>(embh + tk[k0 + c] * EPH + (32 * (k0 + c) + 8 * g) % E);
#pragma unroll
          for (int n = 0; n < HT; n++)
            wf[c][n] = *reinterpret_cast<const bf16x8 *>(w1c + ((n * KD + k0 + c) * 64 + lane) * 8);
        }
#pragma unroll
        for (int c = 0; c < KG; c++)
#pragma unroll
          for (int n = 0; n < HT; n++) acc[n] = mma32(xa[c], wf[c][n], acc[n]);
      }
#pragma unroll
      for (int n = 0; n < HT; n++) {
        const float b = bias[16 * n + r];
#pragma unroll
        for (int c = 0; c < 4; c++) h1[(16 * rt + 4 * g + c) * HP + 16 * n + r] = fmaxf(acc[n][c] + b, 0.0f);
      }
    }
    __syncthreads();
    pc->mark(7);
    // F2: H1 W2 + b2 -> logits (W2 fragments are rows of W2^T)
    for (int u = wave; u < MT * VT; u += NW) {
      const int rt = u / VT, vt = u - rt * VT;
      f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kh = 0; kh < KH; kh++) {
        const float *ha = h1 + (16 * rt + r) * HP + 32 * kh + 8 * g;
        const float *wb = w2t + (16 * vt + r) * W2P + 32 * kh + 8 * g;
        const fvec4 a0 = *reinterpret_cast<const fvec4 *>(ha), a1 = *reinterpret_cast<const fvec4 *>(ha + 4);
        const fvec4 b0 = *reinterpret_cast<const fvec4 *>(wb), b1 = *reinterpret_cast<const fvec4 *>(wb + 4);
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
        acc = mma32(bf8(av), bf8(bv), acc);
      }
      const float b = bias[H + 16 * vt + r];
#pragma unroll
      for (int c = 0; c < 4; c++) lm[(16 * rt + 4 * g + c) * VS + 16 * vt + r] = acc[c] + b;
    }
    __syncthreads();
  }

  __device__ void backward(float *, float *, float *, uint64_t i, const Opt &opt) {
    float ones[8];
#pragma unroll
    for (int q = 0; q < 8; q++) ones[q] = 1.0f;
    const bf16x8 onef = bf8(ones);
    // B1: dpre = (dz W2^T) * [H1 > 0] (contraction over v in plain order),
    // stored in BF16 twice: dpre^T as B4's A fragments (dpt: hidden tile n,
    // k-step rt/2 of the rows) and dpre as B3's A fragments (dpb: row tile
    // rt, k-step n/2 of h in B3's slot order: slot q < 4 is h = 32k + 4g + q,
    // q >= 4 is h = 32k + 16 + 4g + q - 4)
    for (int u = wave; u < MT * HT; u += NW) {
      const int rt = u / HT, n = u - rt * HT;
      f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kv = 0; kv < KV; kv++) {
        const float *za = lm + (16 * rt + r) * VS + 32 * kv + 8 * g;
        const fvec4 a0 = *reinterpret_cast<const fvec4 *>(za), a1 = *reinterpret_cast<const fvec4 *>(za + 4);
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        float bv[8];
#pragma unroll
        for (int q = 0; q < 8; q++) bv[q] = w2t[(32 * kv + 8 * g + q) * W2P + 16 * n + r];
        acc = mma32(bf8(av), bf8(bv), acc);
      }
      bf16x4 pk;
#pragma unroll
      for (int c = 0; c < 4; c++) pk[c] = (__bf16)(h1[(16 * rt + 4 * g + c) * HP + 16 * n + r] > 0.0f ? acc[c] : 0.0f);
      const int slot = r + 16 * (2 * (rt & 1) + (g >> 1));
      *reinterpret_cast<bf16x4 *>(dpt + ((n * KB + (rt >> 1)) * 64 + slot) * 8 + 4 * (g & 1)) = pk;
      __bf16 *pb = dpb + ((rt * KH + (n >> 1)) * 64 + 4 * g + 16 * (r >> 2)) * 8 + 4 * (n & 1) + (r & 3);
#pragma unroll
      for (int c = 0; c < 4; c++) pb[8 * c] = pk[c];
    }
    __syncthreads();
    pc->mark(8);
    pc->mark(11);
    // B2 and the W2 update, with the output-bias gradient sum_j dz[j][v] as
    // an MFMA against a ones fragment (kept by hidden tile 0's units); B2 is
    // the only reader of W2 in this phase.  (No branch separates an MFMA from
    // the first use of its result anywhere in this kernel: the wait states a
    // matrix result needs before a vector read are not kept over a branch.)
    for (int u = wave; u < VT * HT; u += NW) {
      const int vt = u / HT, n = u - vt * HT;
      f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f}, accb = acc;
#pragma unroll
      for (int kb = 0; kb < KB; kb++) {
        float av[8], bv[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
          av[q] = lm[(32 * kb + 8 * g + q) * VS + 16 * vt + r];
          bv[q] = h1[(32 * kb + 8 * g + q) * HP + 16 * n + r];
        }
        const bf16x8 af = bf8(av);
        acc = mma32(af, bf8(bv), acc);
        accb = mma32(af, onef, accb);
      }
#pragma unroll
      for (int c = 0; c < 4; c++) {
        float *w = w2t + (16 * vt + 4 * g + c) * W2P + 16 * n + r;
        *w = *w - opt_delta_c<false>(opt, acc[c], (float *)nullptr, (float *)nullptr);
      }
      if (n == 0 && r == 0) {
#pragma unroll
        for (int c = 0; c < 4; c++) gb[H + 16 * vt + 4 * g + c] = accb[c];
      }
    }
    // B3 + B4 + embedding gradient, per d tile of this wave (the tile's W1
    // owner), in the same phase
    f32x4 acce[VT], accb1[HT];
#pragma unroll
    for (int vt = 0; vt < VT; vt++) acce[vt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < DTW; q++) {
      const int mt = wave + NW * q, p = mt;   // E = 16: d tile mt is context position mt, e = r
      // this tile's tokens first: the ring is position-major, so the tokens
      // of 8 (4) consecutive rows at this position are one 8-byte (4-byte)
      // read; B3, which needs none of them, covers their latency
      const uint8_t *tp = ring + ((((int)(i - (uint64_t)T) + p) & (RS - 1))) * BS;
      u32x2 t8[KB];
#pragma unroll
      for (int kb = 0; kb < KB; kb++) t8[kb] = *reinterpret_cast<const u32x2 *>(tp + 32 * kb + 8 * g);
      uint32_t t4[MT];
#pragma unroll
      for (int rt = 0; rt < MT; rt++) t4[rt] = *reinterpret_cast<const uint32_t *>(tp + 16 * rt + 4 * g);
      // B3 with the old W1: dX[j][d] = sum_h dpre[j][h] W1[d][h]; the
      // lane's own master values are the W1^T fragment in B3's slot order
      bf16x8 wb[KH];
#pragma unroll
      for (int kh = 0; kh < KH; kh++) {
        const float wv[8] = {w1m[q][2 * kh][0], w1m[q][2 * kh][1], w1m[q][2 * kh][2], w1m[q][2 * kh][3],
                             w1m[q][2 * kh + 1][0], w1m[q][2 * kh + 1][1], w1m[q][2 * kh + 1][2], w1m[q][2 * kh + 1][3]};
        wb[kh] = bf8(wv);
      }
      f32x4 acc3[MT];
#pragma unroll
      for (int rt = 0; rt < MT; rt++) {
        acc3[rt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kh = 0; kh < KH; kh++)
          acc3[rt] = mma32(*reinterpret_cast<const bf16x8 *>(dpb + ((rt * KH + kh) * 64 + lane) * 8), wb[kh], acc3[rt]);
      }
      // X fragments (B4's B operand): X[32 kb + 8 g + c][16 mt + r] from the
      // BF16 embedding
      bf16x8 xb[KB];
#pragma unroll
      for (int kb = 0; kb < KB; kb++)
#pragma unroll
        for (int c = 0; c < 8; c++) xb[kb][c] = embh[((t8[kb][c >> 2] >> (8 * (c & 3))) & 0xFFu) * EPH + r];
      // B4: dW1^T[h][d] for every hidden tile m (C: h = 16 m + 4 g + c, d = 16 mt + r)
      f32x4 acc4[HT];
#pragma unroll
      for (int m = 0; m < HT; m++) {
        acc4[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kb = 0; kb < KB; kb++)
          acc4[m] = mma32(*reinterpret_cast<const bf16x8 *>(dpt + ((m * KB + kb) * 64 + lane) * 8), xb[kb], acc4[m]);
      }
      // hidden-bias gradient sum_j dpre[j][h]: every wave's first d tile
      // computes it, wave 0 stores it at the end
      if (q == 0) {
#pragma unroll
        for (int m = 0; m < HT; m++) {
          accb1[m] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
          for (int kb = 0; kb < KB; kb++)
            accb1[m] = mma32(*reinterpret_cast<const bf16x8 *>(dpt + ((m * KB + kb) * 64 + lane) * 8), onef, accb1[m]);
        }
      }
      // embedding gradient over row-tile pairs (2k, 2k+1), K = 32 rows in the
      // slot order s < 4: row 32k + 4g + s, s >= 4: row 32k + 16 + 4g + s - 4,
      // which is how the two dX tiles lie in the accumulators (C layout: rows
      // 4g + c, column e = r).  B = those dX values; A = one-hot rows of the
      // same rows' tokens at this position (BF16 1.0 where token = 16 vt + r).
      // Built per slot s as one 64-bit word holding the slot's value for all
      // four symbol tiles (BF16 1.0 in 16-bit lane tok / 16 when tok % 16 =
      // r, else 0); a byte permutation then gathers each tile's slot pairs.
      static_assert(V == 64, "four symbol tiles per 64-bit slot word");
#pragma unroll
      for (int k = 0; k < MT / 2; k++) {
        uint32_t wlo[8], whi[8];
#pragma unroll
        for (int s2 = 0; s2 < 8; s2++) {
          const uint32_t tok = (t4[2 * k + (s2 >> 2)] >> (8 * (s2 & 3))) & 0xFFu;
          const uint64_t w = (tok & 15u) == (uint32_t)r ? (0x3F80ull << (16u * (tok >> 4))) : 0ull;
          wlo[s2] = (uint32_t)w;
          whi[s2] = (uint32_t)(w >> 32);
        }
        const float dv[8] = {acc3[2 * k][0], acc3[2 * k][1], acc3[2 * k][2], acc3[2 * k][3],
                             acc3[2 * k + 1][0], acc3[2 * k + 1][1], acc3[2 * k + 1][2], acc3[2 * k + 1][3]};
        const bf16x8 bx = bf8(dv);
#pragma unroll
        for (int vt = 0; vt < VT; vt++) {
          // bytes 2h, 2h+1 of slot 2s2's word (low half) and of slot 2s2+1's
          // (high half), h = vt % 2, from the low (vt < 2) or high dwords
          const uint32_t sel = (vt & 1) ? 0x07060302u : 0x05040100u;
          u32x4 wv;
#pragma unroll
          for (int s2 = 0; s2 < 4; s2++)
            wv[s2] = vt < 2 ? __builtin_amdgcn_perm(wlo[2 * s2 + 1], wlo[2 * s2], sel)
                            : __builtin_amdgcn_perm(whi[2 * s2 + 1], whi[2 * s2], sel);
          acce[vt] = mma32(__builtin_bit_cast(bf16x8, wv), bx, acce[vt]);
        }
      }
      // W1 update, and the BF16 copy: this lane's 4 consecutive h at d are 4
      // lanes of one k-step in the fragment order, 16 bytes apart
      const uint32_t base = w1_frag_index(16 * mt + r, 4 * g, D);
#pragma unroll
      for (int m = 0; m < HT; m++) {
#pragma unroll
        for (int x = 0; x < 4; x++) {
          w1m[q][m][x] = w1m[q][m][x] - opt_delta_c<false>(opt, acc4[m][x], (float *)nullptr, (float *)nullptr);
          w1c[base + (uint32_t)m * ((uint32_t)D << 4) + 8u * (uint32_t)x] = (__bf16)w1m[q][m][x];
        }
      }
    }
    // this wave's embedding-gradient partial (C: v = 16 vt + 4 g + c, e = r)
#pragma unroll
    for (int vt = 0; vt < VT; vt++)
#pragma unroll
      for (int c = 0; c < 4; c++) eg[(wave * V + 16 * vt + 4 * g + c) * E + r] = acce[vt][c];
    if (wave == 0 && r == 0) {
#pragma unroll
      for (int m = 0; m < HT; m++)
#pragma unroll
        for (int c = 0; c < 4; c++) gb[16 * m + 4 * g + c] = accb1[m][c];
    }
    __syncthreads();
    pc->mark(10);
  }
};

template <int BS, int T, int E, int H, int V>
__global__ __launch_bounds__(512) void step_chip_kernel(const StepArgs *__restrict__ args) {
  extern __shared__ __align__(16) unsigned char lds[];
  const StepArgs &a = *args;
  NetChip<BS, T, E, H, V> net(a, lds);
  run_blocks<512>(a, lds, net);
}

template <int BS, int T, int E, int H, int V>
hipError_t launch_chip(const StepArgs *a_dev, int grid, size_t lds, hipStream_t st) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&step_chip_kernel<BS, T, E, H, V>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((step_chip_kernel<BS, T, E, H, V>), dim3(grid), dim3(512), lds, st, a_dev);
  return hipGetLastError();
}

// the compiled shapes: (bs, t, E, H, V) of the 16-wide embedding,
// 32-wide hidden, (3,3)-mer model
bool is_shape(const Dims &d, int bs, int t, int E, int H, int V) {
  return d.bs == bs && d.t == t && d.E == E && d.nh == 1 && d.H[0] == H && d.V == V;
}

}  // namespace

bool chip_supports(const Dims &d) {
  if (!d.model_on || d.static_on || d.optimizer != 0) return false;
  if (d.EP != d.E + 4 || d.VS != d.V + 4 || d.HP != d.H[0] + 4) return false;
  if (is_shape(d, 64, 32, 16, 32, 64)) return d.RS == ring_len(32);
  return false;
}

hipError_t launch_step_chip(const StepArgs &a, const StepArgs *a_dev, int grid, hipStream_t st) {
  if (!chip_supports(a.d)) return hipErrorInvalidValue;
  const size_t lds = (size_t)a.lay.total;
  if (is_shape(a.d, 64, 32, 16, 32, 64)) return launch_chip<64, 32, 16, 32, 64>(a_dev, grid, lds, st);
  return hipErrorInvalidValue;
}

}  // namespace pmklc
