// The paper's Transformer dynamic model (Sec. 4.2.4) trained online, on the
// matrix cores.
//
// A step of every active block is a fixed sequence of launches, each over
// all active blocks at once (one batch entry per block): the context
// gather, the products of the forward, the attention, the softmax +
// quantiser + coder (the step_common.h routines of the MLP kernels), and the
// backward, whose weight-gradient products update the weights in their
// epilogue.  The model's weights (2.2 M for the paper's shape) do not fit on
// chip, so unlike the MLP kernels the step is not one persistent workgroup
// per block: the products are ordinary tiled GEMMs spread over the whole
// GPU.
//
// Every output element is summed by one workgroup in a fixed order (split-K
// partial sums are added in slice order by a second pass), and the split is
// a function of the product's shape only, so the probabilities do not depend
// on the number of blocks, the batch or the launch shape: the decoder and
// every single-block run reproduce the encoder bit for bit.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pmklc_internal.h"
#include "seq_loop.h"
#include "step_common.h"

namespace pmklc {

namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kGT = 256;   // GEMM tile and workgroup
enum Epi { kStore = 0, kUpdate = 1, kGrad = 2, kPartial = 3, kAccum = 4 };

// One strided-batched product C = op(A) op(B), batch entry = slot.
//   op(A) is M x K: A[m lda + k], or (TA) A[k lda + m];
//   op(B) is K x N: B[k ldb + n], or (TB) B[n ldb + k].
struct Gemm {
  const float *A, *B;
  float *C;
  int64_t lda, ldb, ldc, sA, sB, sC;
  int M, N, K;
  const float *bias;   // kStore: bias[n] (per slot, stride sB2), or null
  int64_t sBias;
  const float *mask;   // kStore: C = 0 where mask[m ldm + n] <= 0, or null
  int64_t ldm, sMask;
  int relu;            // kStore: max(., 0)
  float *m, *v;        // kUpdate (Adam): moments laid out like C
  int64_t sMV;
  float *part;         // kPartial: part[slot][slice][M][N]
  int64_t sPart;
  int split;           // K slices
  // TA only: A may be virtual.  aug: one more row of ones (row M of the
  // product is then the column sums of op(B), a bias gradient, stored at
  // C + M ldc, where each layer's bias follows its weight).  One-hot:
  // A[k][m] = (key(k) == m), key = oh[k] (per slot, stride sOh) or k % oh_mod.
  int aug;
  const uint8_t *oh;
  int64_t sOh;
  int oh_mod;
  // virtual X (the MLP's first-layer input, either layout; A is null): X[r][k]
  // = emb[slot sEmb + key(r, k / xE) xE + k % xE], key = oh[slot sOh + r xt + k / xE]
  // (the step's context tokens): the concatenated context embeddings,
  // never written out
  const float *emb;
  int64_t sEmb;
  int xE, xt;
  const TfState *st;
  int opt;
  float lr, b1, b2, eps;
  // 16-byte accesses allowed (base 16-byte aligned, every stride a multiple
  // of 4 floats): va / vb for the operands' loads, vc for the epilogue's
  int va, vb, vc;
  // BF16 storage (element strides unchanged, the pointers reinterpreted):
  // hc, kStore writes C rounded to BF16 (to nearest even, as the operand
  // staging rounds); hb, the BF16 product reads B (not TB) from BF16.  A
  // product that rounds its operands to BF16 anyway reads the same values
  // from half the bytes.
  int hb, hc;
};

__device__ __forceinline__ Opt make_opt(const Gemm &g) {
  Opt o;
  o.kind = g.opt;
  o.lr = g.lr; o.b1 = g.b1; o.b2 = g.b2; o.eps = g.eps;
  o.c1 = g.st->c1;
  o.c2 = g.st->c2;
  return o;
}

// the epilogue of one output element: x is the sum over K (or a slice)
template <int EPI>
__device__ __forceinline__ void epilogue(const Gemm &g, int slot, int slice, int row, int col, float x) {
  if constexpr (EPI == kPartial) {
    g.part[slot * g.sPart + ((int64_t)slice * (g.M + g.aug) + row) * g.N + col] = x;
  } else if constexpr (EPI == kStore) {
    if (g.bias) x += g.bias[slot * g.sBias + col];
    if (g.relu) x = x > 0.0f ? x : 0.0f;
    if (g.mask && !(g.mask[slot * g.sMask + (int64_t)row * g.ldm + col] > 0.0f)) x = 0.0f;
    if (g.hc)
      reinterpret_cast<__bf16 *>(g.C)[slot * g.sC + (int64_t)row * g.ldc + col] = (__bf16)x;
    else
      g.C[slot * g.sC + (int64_t)row * g.ldc + col] = x;
  } else if constexpr (EPI == kGrad) {
    g.C[slot * g.sC + (int64_t)row * g.ldc + col] = x;
  } else if constexpr (EPI == kAccum) {
    g.C[slot * g.sC + (int64_t)row * g.ldc + col] += x;
  } else {
    const int64_t at = (int64_t)row * g.ldc + col;
    const Opt o = make_opt(g);
    float *mm = g.m ? g.m + slot * g.sMV + at : nullptr;
    float *vv = g.v ? g.v + slot * g.sMV + at : nullptr;
    g.C[slot * g.sC + at] -= opt_delta(o, x, mm, vv);
  }
}

// the same for 4 consecutive columns col..col+3 < N, when g.vc allows
// 16-byte accesses: the same operations per element, four at a time
template <int EPI>
__device__ __forceinline__ void epilogue4(const Gemm &g, int slot, int slice, int row, int col, const float *x) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  f4 y = {x[0], x[1], x[2], x[3]};
  if constexpr (EPI == kPartial) {
    *reinterpret_cast<f4 *>(g.part + slot * g.sPart + ((int64_t)slice * (g.M + g.aug) + row) * g.N + col) = y;
  } else if constexpr (EPI == kStore) {
    if (g.bias) {
      const f4 b = *reinterpret_cast<const f4 *>(g.bias + slot * g.sBias + col);
#pragma unroll
      for (int c = 0; c < 4; c++) y[c] += b[c];
    }
    if (g.relu) {
#pragma unroll
      for (int c = 0; c < 4; c++) y[c] = y[c] > 0.0f ? y[c] : 0.0f;
    }
    if (g.mask) {
      const f4 k = *reinterpret_cast<const f4 *>(g.mask + slot * g.sMask + (int64_t)row * g.ldm + col);
#pragma unroll
      for (int c = 0; c < 4; c++)
        if (!(k[c] > 0.0f)) y[c] = 0.0f;
    }
    if (g.hc) {
      typedef __bf16 h4 __attribute__((ext_vector_type(4)));
      h4 z;
#pragma unroll
      for (int c = 0; c < 4; c++) z[c] = (__bf16)y[c];
      *reinterpret_cast<h4 *>(reinterpret_cast<__bf16 *>(g.C) + slot * g.sC + (int64_t)row * g.ldc + col) = z;
    } else {
      *reinterpret_cast<f4 *>(g.C + slot * g.sC + (int64_t)row * g.ldc + col) = y;
    }
  } else if constexpr (EPI == kGrad) {
    *reinterpret_cast<f4 *>(g.C + slot * g.sC + (int64_t)row * g.ldc + col) = y;
  } else if constexpr (EPI == kAccum) {
    f4 *c4 = reinterpret_cast<f4 *>(g.C + slot * g.sC + (int64_t)row * g.ldc + col);
    f4 z = *c4;
#pragma unroll
    for (int c = 0; c < 4; c++) z[c] += y[c];
    *c4 = z;
  } else {
    const int64_t at = (int64_t)row * g.ldc + col;
    const Opt o = make_opt(g);
    f4 *w4 = reinterpret_cast<f4 *>(g.C + slot * g.sC + at);
    f4 w = *w4;
    if (g.m) {
      f4 *m4 = reinterpret_cast<f4 *>(g.m + slot * g.sMV + at), *v4 = reinterpret_cast<f4 *>(g.v + slot * g.sMV + at);
      f4 mm = *m4, vv = *v4;
#pragma unroll
      for (int c = 0; c < 4; c++) {
        float mc = mm[c], vc = vv[c];
        w[c] -= opt_delta(o, y[c], &mc, &vc);
        mm[c] = mc;
        vv[c] = vc;
      }
      *m4 = mm;
      *v4 = vv;
    } else {
#pragma unroll
      for (int c = 0; c < 4; c++) w[c] -= opt_delta(o, y[c], (float *)nullptr, (float *)nullptr);
    }
    *w4 = w;
  }
}

// 64 x 64 output tile per workgroup of four waves, 32 x 32 per wave (2 x 2
// MFMA tiles of 16 x 16); K in chunks of 64.  A chunk is read from global
// memory into registers while the previous one is multiplied, then stored
// to LDS: BF16 (rounded to nearest even once, on the way in) as A[m][k] and
// B transposed, B^T[n][k], rows padded to 72, so that every fragment is one
// 16-byte read; FP32 as A[m][k] and B^T[n][k] rows of 65.
// BF16: v_mfma_f32_16x16x32_bf16, lane l (r = l % 16, q = l / 16) holding
// A[r][8q..8q+7] and B[8q..8q+7][r]; FP32: v_mfma_f32_16x16x4f32 with A[r][q]
// and B[q][r] per 4-wide k-step.  The accumulator holds C[4q + c][r].
constexpr int kCK = 64;                 // K chunk
constexpr int kLdB = kCK + 8;           // BF16 LDS row (elements)
constexpr int kLdF = kCK + 1;           // FP32 LDS row (elements)
constexpr int kPer = kBM * kCK / kGT;   // elements of each operand per thread and chunk (16)

// Compiled for at least 4 waves per SIMD: at most 128 registers per lane
// (vector and accumulation together, no spills), so that four workgroups
// share a CU and hide each other's memory latency on grids of many blocks.
template <bool BF16, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(kGT, 4) void gemm_kernel(Gemm g) {
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs (each with its
  // own L2) round robin by linear id; logical tile `tile` gives XCD k one
  // contiguous range of tiles, so neighbouring tiles (the N tiles of one M
  // row, which read the same A tile) share an L2.  A bijection of the grid:
  // every tile is still computed once, the same way.
  const uint32_t gx = gridDim.x, gy = gridDim.y, total = gx * gy * gridDim.z;
  const uint32_t lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), xcd = lin % 8, full = total / 8;
  const uint32_t tile = xcd * full + min(xcd, total % 8) + lin / 8;
  const int tz = (int)(tile / (gx * gy)), ty = (int)((tile / gx) % gy), tx = (int)(tile % gx);
  const int slot = tz / g.split, slice = tz % g.split;
  if (slot >= g.st->nact) return;
  const int m0 = ty * kBM, n0 = tx * kBN;
  const int M = g.M + (TA ? g.aug : 0);
  typedef float f4 __attribute__((ext_vector_type(4)));
  const float *A = g.emb || (TA && (g.oh || g.oh_mod)) ? nullptr : g.A + slot * g.sA;
  const float *emb = g.emb ? g.emb + slot * g.sEmb : nullptr;
  const uint8_t *oh = g.oh ? g.oh + slot * g.sOh : nullptr;
  // element (r, k) of the virtual X
  auto xv = [&](int r, int k) -> float { return emb[(int)oh[(int64_t)r * g.xt + k / g.xE] * g.xE + k % g.xE]; };
  // 4 of them along k (one embedding row: xE % 4 == 0 when g.va)
  auto xv4 = [&](int r, int k, float *x) {
    const f4 v = *reinterpret_cast<const f4 *>(emb + (int)oh[(int64_t)r * g.xt + k / g.xE] * g.xE + k % g.xE);
#pragma unroll
    for (int c = 0; c < 4; c++) x[c] = v[c];
  };
  const float *B = g.B + slot * g.sB;
  int kbeg = 0, kend = g.K;
  if (g.split > 1) {
    const int ks = ((g.K + g.split - 1) / g.split + kCK - 1) / kCK * kCK;
    kbeg = slice * ks;
    kend = min(g.K, kbeg + ks);
  }
  typedef typename std::conditional<BF16, __bf16, float>::type T;
  constexpr int LD = BF16 ? kLdB : kLdF;
  // the two operand tiles, and after the products the output tile (FP32,
  // rows of 65) for a coalesced epilogue
  constexpr int kTile = (kBM + kBN) * LD * (int)sizeof(T);
  constexpr int kOut = kBM * (kBN + 1) * 4;
  __shared__ __attribute__((aligned(16))) unsigned char smem[kTile > kOut ? kTile : kOut];
  T *As = reinterpret_cast<T *>(smem);        // 16-byte fragment reads
  T *Bs = As + kBM * LD;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32, r = lane & 15, q = lane >> 4;
  // a chunk's operands, 16 elements of each per thread.  An operand stored
  // with k contiguous (A, or B^T when TB) is read in groups of 4 along k:
  // group e = tid + 256 u (u < 4), 16 groups per 64-wide line.  One stored
  // transposed (A^T when TA, B otherwise) is read as one 4 x 4 sub-block
  // per thread: 4 consecutive m (n) from 4 (tid % 16) at the 4 consecutive
  // k from 4 (tid / 16), one 4-wide load per k, so that both go to LDS as
  // runs of 4 along k.  In-bounds loads whose layout allows it are 16-byte
  // loads, the others element by element.  pa / pb[4 u + c]: element c of
  // group u, or of sub-block row k = 4 (tid / 16) + u.
  auto kgroup = [&](int u, int &line, int &kk) {
    const int e = tid + kGT * u;
    line = e >> 4;
    kk = (e & 15) * 4;
  };
  const int sub_mn = (tid & 15) * 4, sub_k = (tid >> 4) * 4;
  float pa[kPer], pb[kPer];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < kPer / 4; u++) {
      float *x = pa + 4 * u;
      if (!TA) {
        int mm, kk;
        kgroup(u, mm, kk);
        const int gm = m0 + mm, gk = k0 + kk;
        if (emb) {
          if (g.va && gm < M && gk + 3 < kend) {
            xv4(gm, gk, x);
          } else {
#pragma unroll
            for (int c = 0; c < 4; c++) x[c] = gm < M && gk + c < kend ? xv(gm, gk + c) : 0.0f;
          }
        } else if (g.va && gm < M && gk + 3 < kend) {
          const f4 v = *reinterpret_cast<const f4 *>(A + (int64_t)gm * g.lda + gk);
#pragma unroll
          for (int c = 0; c < 4; c++) x[c] = v[c];
        } else {
#pragma unroll
          for (int c = 0; c < 4; c++) x[c] = gm < M && gk + c < kend ? A[(int64_t)gm * g.lda + gk + c] : 0.0f;
        }
      } else {
        const int gm = m0 + sub_mn, gk = k0 + sub_k + u;
        if (emb) {
          if (g.va && gk < kend && gm + 3 < g.M) {
            xv4(gk, gm, x);
          } else {
#pragma unroll
            for (int c = 0; c < 4; c++) {
              const int gmc = gm + c;
              x[c] = gmc < M && gk < kend ? (gmc == g.M ? 1.0f : xv(gk, gmc)) : 0.0f;
            }
          }
        } else if (oh || g.oh_mod) {
          const int key = gk < kend ? (oh ? (int)oh[gk] : gk % g.oh_mod) : -1;
#pragma unroll
          for (int c = 0; c < 4; c++) x[c] = gm + c < M && key == gm + c ? 1.0f : 0.0f;
        } else if (g.va && gk < kend && gm + 3 < g.M) {
          const f4 v = *reinterpret_cast<const f4 *>(A + (int64_t)gk * g.lda + gm);
#pragma unroll
          for (int c = 0; c < 4; c++) x[c] = v[c];
        } else {
#pragma unroll
          for (int c = 0; c < 4; c++) {
            const int gmc = gm + c;
            x[c] = gmc < M && gk < kend ? (gmc == g.M ? 1.0f : A[(int64_t)gk * g.lda + gmc]) : 0.0f;
          }
        }
      }
      float *y = pb + 4 * u;
      if (TB) {
        int nn, kk;
        kgroup(u, nn, kk);
        const int gn = n0 + nn, gk = k0 + kk;
        if (g.vb && gn < g.N && gk + 3 < kend) {
          const f4 v = *reinterpret_cast<const f4 *>(B + (int64_t)gn * g.ldb + gk);
#pragma unroll
          for (int c = 0; c < 4; c++) y[c] = v[c];
        } else {
#pragma unroll
          for (int c = 0; c < 4; c++) y[c] = gn < g.N && gk + c < kend ? B[(int64_t)gn * g.ldb + gk + c] : 0.0f;
        }
      } else if (BF16 && g.hb) {
        const int gn = n0 + sub_mn, gk = k0 + sub_k + u;
        const __bf16 *Bh = reinterpret_cast<const __bf16 *>(g.B) + slot * g.sB;
        if (g.vb && gk < kend && gn + 3 < g.N) {
          typedef __bf16 h4 __attribute__((ext_vector_type(4)));
          const h4 v = *reinterpret_cast<const h4 *>(Bh + (int64_t)gk * g.ldb + gn);
#pragma unroll
          for (int c = 0; c < 4; c++) y[c] = (float)v[c];
        } else {
#pragma unroll
          for (int c = 0; c < 4; c++) y[c] = gn + c < g.N && gk < kend ? (float)Bh[(int64_t)gk * g.ldb + gn + c] : 0.0f;
        }
      } else {
        const int gn = n0 + sub_mn, gk = k0 + sub_k + u;
        if (g.vb && gk < kend && gn + 3 < g.N) {
          const f4 v = *reinterpret_cast<const f4 *>(B + (int64_t)gk * g.ldb + gn);
#pragma unroll
          for (int c = 0; c < 4; c++) y[c] = v[c];
        } else {
#pragma unroll
          for (int c = 0; c < 4; c++) y[c] = gn + c < g.N && gk < kend ? B[(int64_t)gk * g.ldb + gn + c] : 0.0f;
        }
      }
    }
  };
  // one operand's 16 elements to LDS, row-major [m or n][k]: a group's 4
  // values are adjacent along k; a sub-block's column c is the run of 4
  // along k at row sub_mn + c (BF16: one 8-byte store per run)
  auto stage = [&](T *S, const float *v, bool kcontig) {
    if (kcontig) {
#pragma unroll
      for (int u = 0; u < kPer / 4; u++) {
        int line, kk;
        kgroup(u, line, kk);
#pragma unroll
        for (int c = 0; c < 4; c++) S[line * LD + kk + c] = (T)v[4 * u + c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; c++) {
        if constexpr (BF16) {
          typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
          bf4 run;
#pragma unroll
          for (int u = 0; u < 4; u++) run[u] = (__bf16)v[4 * u + c];
          *reinterpret_cast<bf4 *>(&S[(sub_mn + c) * LD + sub_k]) = run;
        } else {
#pragma unroll
          for (int u = 0; u < 4; u++) S[(sub_mn + c) * LD + sub_k + u] = v[4 * u + c];
        }
      }
    }
  };
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) acc[i][j] = f32x4_t{0.0f, 0.0f, 0.0f, 0.0f};
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kCK) {
    stage(As, pa, !TA);
    stage(Bs, pb, TB);
    __syncthreads();
    if (k0 + kCK < kend) fetch(k0 + kCK);   // in flight during the products
    if constexpr (BF16) {
#pragma unroll
      for (int ks = 0; ks < kCK / 32; ks++) {
        bf16x8_t a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; i++)
          a[i] = *reinterpret_cast<const bf16x8_t *>(&As[(wm + 16 * i + r) * LD + 32 * ks + 8 * q]);
#pragma unroll
        for (int j = 0; j < 2; j++)
          b[j] = *reinterpret_cast<const bf16x8_t *>(&Bs[(wn + 16 * j + r) * LD + 32 * ks + 8 * q]);
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < kCK / 4; ks++) {
        const float a0 = As[(wm + r) * LD + 4 * ks + q], a1 = As[(wm + 16 + r) * LD + 4 * ks + q];
        const float b0 = Bs[(wn + r) * LD + 4 * ks + q], b1 = Bs[(wn + 16 + r) * LD + 4 * ks + q];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // the accumulators are read after the loop's branch: keep the matrix-core
  // results' wait states explicit rather than relying on the scheduler
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" ::: "memory");
  __builtin_amdgcn_sched_barrier(0);
  // the tile through LDS, then 4 consecutive outputs per thread, 16 threads
  // per 64-wide row: the epilogue's loads and stores (the optimiser's weight
  // and moments above all) move whole 256-byte rows, 16 bytes per thread
  // where the layout allows
  float *Cs = reinterpret_cast<float *>(smem);
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int c = 0; c < 4; c++) Cs[(wm + 16 * i + 4 * q + c) * (kBN + 1) + wn + 16 * j + r] = acc[i][j][c];
  __syncthreads();
  constexpr int kU = kBM * kBN / (4 * kGT);   // 4-column groups per thread
  if constexpr (EPI == kUpdate) {
    // Adam over a tile whose columns are all in range: every group's
    // weight and moments are loaded before the first is updated, so a
    // thread has 12 16-byte loads in flight instead of 3 (the stores of one
    // group would otherwise order the next group's loads behind them).
    // Each element is updated by the same operations as in epilogue4.
    if (g.vc && g.m && n0 + kBN <= g.N) {
      float *Cb = g.C + slot * g.sC, *Mb = g.m + slot * g.sMV, *Vb = g.v + slot * g.sMV;
      f4 wt[kU], mm[kU], vv[kU];
#pragma unroll
      for (int u = 0; u < kU; u++) {
        const int e = tid + kGT * u, row = m0 + (e >> 4);
        const int64_t at = (int64_t)row * g.ldc + n0 + (e & 15) * 4;
        if (row < M) {
          wt[u] = *reinterpret_cast<const f4 *>(Cb + at);
          mm[u] = *reinterpret_cast<const f4 *>(Mb + at);
          vv[u] = *reinterpret_cast<const f4 *>(Vb + at);
        }
      }
      const Opt o = make_opt(g);
#pragma unroll
      for (int u = 0; u < kU; u++) {
        const int e = tid + kGT * u, rl = e >> 4, cl = (e & 15) * 4, row = m0 + rl;
        if (row >= M) continue;
        const int64_t at = (int64_t)row * g.ldc + n0 + cl;
#pragma unroll
        for (int c = 0; c < 4; c++) {
          float mc = mm[u][c], vc = vv[u][c];
          wt[u][c] -= opt_delta(o, Cs[rl * (kBN + 1) + cl + c], &mc, &vc);
          mm[u][c] = mc;
          vv[u][c] = vc;
        }
        *reinterpret_cast<f4 *>(Cb + at) = wt[u];
        *reinterpret_cast<f4 *>(Mb + at) = mm[u];
        *reinterpret_cast<f4 *>(Vb + at) = vv[u];
      }
      return;
    }
  }
#pragma unroll
  for (int u = 0; u < kU; u++) {
    const int e = tid + kGT * u, rl = e >> 4, cl = (e & 15) * 4, row = m0 + rl, col = n0 + cl;
    if (row >= M) continue;
    float x[4];
#pragma unroll
    for (int c = 0; c < 4; c++) x[c] = Cs[rl * (kBN + 1) + cl + c];
    if (g.vc && col + 3 < g.N) {
      epilogue4<EPI>(g, slot, slice, row, col, x);
    } else {
#pragma unroll
      for (int c = 0; c < 4; c++)
        if (col + c < g.N) epilogue<EPI>(g, slot, slice, row, col + c, x[c]);
    }
  }
}

// second pass of a split product: the slices' partial sums added in slice
// order, then the product's own epilogue
template <int EPI>
__global__ __launch_bounds__(256) void reduce_kernel(Gemm g) {
  const int slot = blockIdx.y;
  if (slot >= g.st->nact) return;
  const int M = g.M + g.aug;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * g.N) return;
  const int row = (int)(e / g.N), col = (int)(e % g.N);
  const float *p = g.part + slot * g.sPart + e;
  float x = 0.0f;
  for (int s = 0; s < g.split; s++) x += p[(int64_t)s * M * g.N];
  epilogue<EPI>(g, slot, 0, row, col, x);
}

// Fixed split per product shape (never per batch): the long-K products
// whose tiles alone would leave most of the GPU idle get about one slice
// per 512 of K, as many as the slot's partial-sum buffer (cap floats) holds.
int split_for(int M, int N, int K, int64_t cap) {
  const int64_t tiles = (int64_t)((M + kBM - 1) / kBM) * ((N + kBN - 1) / kBN);
  if (K < 1024 || tiles > 64) return 1;
  int64_t sp = std::min<int64_t>(32, K / 512);
  sp = std::min<int64_t>(sp, cap / ((int64_t)M * N));
  return (int)std::max<int64_t>(sp, 1);
}

template <bool BF16, bool TA, bool TB, int EPI>
hipError_t gemm_go(Gemm g, int nslots, hipStream_t st) {
  if (nslots <= 0 || g.M <= 0 || g.N <= 0) return hipSuccess;
  const int M = g.M + g.aug;
  dim3 grid((g.N + kBN - 1) / kBN, (M + kBM - 1) / kBM, nslots * g.split);
  if (g.split > 1) {
    hipLaunchKernelGGL((gemm_kernel<BF16, TA, TB, kPartial>), grid, dim3(kGT), 0, st, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t mn = (int64_t)M * g.N;
    hipLaunchKernelGGL((reduce_kernel<EPI>), dim3((unsigned)((mn + 255) / 256), nslots), dim3(256), 0, st, g);
  } else {
    hipLaunchKernelGGL((gemm_kernel<BF16, TA, TB, EPI>), grid, dim3(kGT), 0, st, g);
  }
  return hipGetLastError();
}

// C[M x N] = op(A) op(B) (+ epilogue) over nslots batch entries
template <bool TA, bool TB, int EPI>
hipError_t gemm(const TfShape &s, Gemm g, int nslots, hipStream_t st) {
  if ((g.hb && (TB || !s.bf16)) || (g.hc && EPI != kStore)) return hipErrorInvalidValue;
  // the partial sums must fit the slot's buffer (sized from the shape, so
  // the choice still depends on the shape alone)
  g.split = split_for(g.M + g.aug, g.N, g.K, g.sPart);
  auto al = [](const void *p, std::initializer_list<int64_t> strides) {
    if (reinterpret_cast<uintptr_t>(p) % 16) return false;
    for (int64_t x : strides)
      if (x % 4) return false;
    return true;
  };
  g.va = g.emb ? al(g.emb, {g.sEmb, g.xE}) : g.A && al(g.A, {g.lda, g.sA});
  g.vb = al(g.B, {g.ldb, g.sB});
  g.vc = al(g.C, {g.ldc, g.sC}) && (!g.bias || al(g.bias, {g.sBias})) && (!g.mask || al(g.mask, {g.ldm, g.sMask})) &&
         (!g.m || (al(g.m, {g.sMV}) && g.v && al(g.v, {g.sMV}))) &&
         (g.split == 1 || (al(g.part, {g.sPart}) && g.N % 4 == 0));
  return s.bf16 ? gemm_go<true, TA, TB, EPI>(g, nslots, st) : gemm_go<false, TA, TB, EPI>(g, nslots, st);
}

// ----------------------------------------------------------- small kernels
// the context token (row, p) of slot `slot` at step i: the stream's
// tok_off + row L + i - t + p, or (op) ctx[row t + p]
__device__ __forceinline__ int ctx_token(const TfShape &s, const TfSlot &d, const uint8_t *toks, const uint8_t *ctx,
                                         int i, int row, int p) {
  if (ctx) return ctx[(int64_t)row * s.t + p];
  return toks[d.tok_off + (uint64_t)row * d.L + (uint64_t)(i - s.t + p)];
}

// X[slot][(row t + p) E + e] = Emb[c][e] + Pos[p][e] (for the MLP, without
// Pos: the concatenated context embeddings, row-major)
__global__ __launch_bounds__(256) void gather_kernel(TfShape s, const TfState *st, const TfSlot *desc,
                                                     const uint8_t *toks, const uint8_t *ctx, const float *params,
                                                     float *X, int64_t sX, uint8_t *tokstep, int64_t sTok,
                                                     int *err) {
  const int slot = blockIdx.y;
  if (slot >= st->nact) return;
  const int64_t n = (int64_t)s.bs * s.t * s.E;
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n) return;
  const int e = (int)(q % s.E);
  const int64_t rp = q / s.E;
  const int p = (int)(rp % s.t), row = (int)(rp / s.t);
  int c = ctx_token(s, desc[slot], toks, ctx, st->i, row, p);
  if (c >= s.V) {
    atomicOr(err, 1);
    c = 0;
  }
  const float *W = params + slot * s.stride;
  const float pe = s.off_pos >= 0 ? W[s.off_pos + (int64_t)p * s.E + e] : 0.0f;   // the MLP has none
  X[slot * sX + q] = W[s.off_emb + (int64_t)c * s.E + e] + pe;
  if (e == 0) tokstep[slot * sTok + rp] = (uint8_t)c;   // the embedding gradient's one-hot keys
}

// the step's context tokens only (the MLP reads its X virtually):
// tokstep[slot][row t + p]
__global__ __launch_bounds__(256) void tokstep_kernel(TfShape s, const TfState *st, const TfSlot *desc,
                                                      const uint8_t *toks, const uint8_t *ctx, uint8_t *tokstep,
                                                      int64_t sTok, int *err) {
  const int slot = blockIdx.y;
  if (slot >= st->nact) return;
  const int64_t rp = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (rp >= (int64_t)s.bs * s.t) return;
  const int p = (int)(rp % s.t), row = (int)(rp / s.t);
  int c = ctx_token(s, desc[slot], toks, ctx, st->i, row, p);
  if (c >= s.V) {
    atomicOr(err, 1);
    c = 0;
  }
  tokstep[slot * sTok + rp] = (uint8_t)c;
}

// Attention at the last position, one workgroup per (row, slot), one thread
// per column x = h dh + d of the A-wide projections:
// s_p = q_h . k_{p,h} / sqrt(dh), a = softmax(s), o_h = sum_p a_p v_{p,h}.
// KV rows hold [k | v] (2A), Q rows q (A).  The probabilities a are kept
// for the backward.  The row's keys pass through LDS pc positions at a time
// (rows padded to A + 1), where one thread per (head, position) adds its
// dh products in order; the softmax and the weighted sum of values are per
// column.  LDS: scores [H][t], q [A], key chunk [pc][A + 1].
__global__ void attn_fwd_kernel(TfShape s, const TfState *st, const float *Q, const float *KV, float *att,
                                float *O, int64_t sQ, int64_t sKV, int64_t sAtt, int pc) {
  const int slot = blockIdx.y;
  if (slot >= st->nact) return;
  extern __shared__ float sm[];
  const int A = s.A, t = s.t, H = s.H, dh = s.dh, LA = A + 1;
  float *sc = sm, *qs = sc + H * t, *ks = qs + A;
  const int row = blockIdx.x, x = threadIdx.x, h = x / dh, d = x % dh;
  const float scale = 1.0f / sqrtf((float)dh);
  const float *kv = KV + slot * sKV + (int64_t)row * t * 2 * A;
  qs[x] = Q[slot * sQ + (int64_t)row * A + x];
  for (int p0 = 0; p0 < t; p0 += pc) {
    const int np = min(pc, t - p0);
    __syncthreads();   // q written; the previous chunk read
#pragma unroll 32
    for (int p = 0; p < np; p++) ks[p * LA + x] = kv[(int64_t)(p0 + p) * 2 * A + x];
    __syncthreads();
    for (int u = x; u < H * np; u += A) {
      const int hh = u / np, p = u - hh * np;
      const float *qa = qs + hh * dh, *ka = ks + p * LA + hh * dh;
      float acc = 0.0f;
      for (int e = 0; e < dh; e++) acc += qa[e] * ka[e];
      sc[hh * t + p0 + p] = acc * scale;
    }
  }
  __syncthreads();
  const float *sh = sc + h * t;
  float mx = -INFINITY;
  for (int p = 0; p < t; p++) mx = fmaxf(mx, sh[p]);
  float sum = 0.0f;
  for (int p = 0; p < t; p++) sum += __expf(sh[p] - mx);
  const float inv = 1.0f / sum;
  float o = 0.0f;
  float *arow = att + slot * sAtt + ((int64_t)row * H + h) * t;
#pragma unroll 32
  for (int p = 0; p < t; p++) {
    const float a = __expf(sh[p] - mx) * inv;
    o += a * kv[(int64_t)p * 2 * A + A + x];
    if (d == 0) arow[p] = a;
  }
  O[slot * sQ + (int64_t)row * A + x] = o;
}

// Backward of the attention: dv_p = a_p do, da_p = do . v_p,
// ds_p = a_p (da_p - sum_r a_r da_r) / sqrt(dh), dq = sum_p ds_p k_p,
// dk_p = ds_p q (per head).  The values pass through LDS as the keys do in
// the forward (da_p by one thread per (head, position)); LDS: da [H][t],
// do [A], value chunk [pc][A + 1].
__global__ void attn_bwd_kernel(TfShape s, const TfState *st, const float *Q, const float *KV, const float *att,
                                const float *dO, float *dQ, float *dKV, int64_t sQ, int64_t sKV, int64_t sAtt, int pc) {
  const int slot = blockIdx.y;
  if (slot >= st->nact) return;
  extern __shared__ float sm[];
  const int A = s.A, t = s.t, H = s.H, dh = s.dh, LA = A + 1;
  float *da = sm, *ds_ = da + H * t, *vs = ds_ + A;
  const int row = blockIdx.x, x = threadIdx.x, h = x / dh;
  const float scale = 1.0f / sqrtf((float)dh);
  const float *kv = KV + slot * sKV + (int64_t)row * t * 2 * A;
  float *dkv = dKV + slot * sKV + (int64_t)row * t * 2 * A;
  const float *arow = att + slot * sAtt + ((int64_t)row * H + h) * t;
  const float qx = Q[slot * sQ + (int64_t)row * A + x];
  const float dox = dO[slot * sQ + (int64_t)row * A + x];
  ds_[x] = dox;
  for (int p0 = 0; p0 < t; p0 += pc) {
    const int np = min(pc, t - p0);
    __syncthreads();
#pragma unroll 32
    for (int p = 0; p < np; p++) {
      vs[p * LA + x] = kv[(int64_t)(p0 + p) * 2 * A + A + x];
      dkv[(int64_t)(p0 + p) * 2 * A + A + x] = arow[p0 + p] * dox;
    }
    __syncthreads();
    for (int u = x; u < H * np; u += A) {
      const int hh = u / np, p = u - hh * np;
      const float *oa = ds_ + hh * dh, *va = vs + p * LA + hh * dh;
      float acc = 0.0f;
      for (int e = 0; e < dh; e++) acc += oa[e] * va[e];
      da[hh * t + p0 + p] = acc;
    }
  }
  __syncthreads();
  const float *dh_ = da + h * t;
  float dot = 0.0f;
  for (int p = 0; p < t; p++) dot += arow[p] * dh_[p];
  float dq = 0.0f;
#pragma unroll 32
  for (int p = 0; p < t; p++) {
    const float ds = arow[p] * (dh_[p] - dot) * scale;
    dq += ds * kv[(int64_t)p * 2 * A + x];
    dkv[(int64_t)p * 2 * A + x] = ds * qx;
  }
  dQ[slot * sQ + (int64_t)row * A + x] = dq;
}

// LDS of the attention kernels: H t scores, A of q (do), a chunk of pc
// positions of keys (values) in rows of A + 1, pc as many as 36 KB holds
int attn_chunk(const TfShape &s) { return std::max(1, std::min(s.t, 9216 / (s.A + 1))); }
size_t attn_lds(const TfShape &s) {
  return ((size_t)s.H * s.t + s.A + (size_t)attn_chunk(s) * (s.A + 1)) * sizeof(float);
}
hipError_t attn_allow_lds(const TfShape &s) {
  static bool done = false;
  if (done || attn_lds(s) <= 65536) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&attn_fwd_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&attn_bwd_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  done = e == hipSuccess;
  return e;
}

// Step bookkeeping (one thread): the step index, the active slots and, for
// an update step, Adam's bias corrections as running FP32 powers.
__global__ void begin_step_kernel(TfShape s, TfState *st, int i, int nact) {
  st->i = i;
  st->nact = nact;
  if (i >= s.t) {
    st->b1t *= s.b1;
    st->b2t *= s.b2;
    st->c1 = 1.0f - st->b1t;
    st->c2 = 1.0f - st->b2t;
  }
}
__global__ void init_state_kernel(TfState *st, int nact) {
  st->i = -1;
  st->nact = nact;
  st->c1 = st->c2 = 1.0f;
  st->b1t = st->b2t = 1.0f;
  st->pad[0] = st->pad[1] = 0;
}

// every slot starts from the seeded parameters; Adam moments at zero
__global__ __launch_bounds__(256) void slot_init_kernel(TfShape s, int n, const float *init, float *params,
                                                        float *m, float *v) {
  const int slot = blockIdx.y;
  if (slot >= n) return;
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < s.stride; q += (int64_t)gridDim.x * 256) {
    params[slot * s.stride + q] = q <= s.P ? init[q] : 0.0f;
    if (m) m[slot * s.stride + q] = 0.0f;
    if (v) v[slot * s.stride + q] = 0.0f;
  }
}

__global__ void coder_init_kernel(TfShape s, int n, const TfSlot *desc, CoderState *coder, const uint32_t *sslots,
                                  const uint32_t *seg_words, int mode) {
  const int slot = blockIdx.x;
  if (slot >= n) return;
  const TfSlot d = desc[slot];
  for (int j = threadIdx.x; j < s.bs; j += blockDim.x) {
    CoderState c;
    c.ovf = 0;
    c.nwords = 0;
    if (mode == 0) {
      enc_init(c.enc);
    } else {
      uint32_t nw = seg_words[(int64_t)d.block * s.bs + j];
      c.nwords = nw > d.slot_words ? d.slot_words : nw;
      dec_init(c.dec, (const gu32 *)(sslots + d.slot_off + (uint64_t)j * d.slot_words), c.nwords);
    }
    coder[(int64_t)slot * s.bs + j] = c;
  }
}

__global__ void coder_finish_kernel(TfShape s, int n, const TfSlot *desc, CoderState *coder, uint32_t *sslots,
                                    uint32_t *seg_bits, int *err) {
  const int slot = blockIdx.x;
  if (slot >= n) return;
  const TfSlot d = desc[slot];
  for (int j = threadIdx.x; j < s.bs; j += blockDim.x) {
    CoderState c = coder[(int64_t)slot * s.bs + j];
    enc_finish(c.enc, (gu32 *)(sslots + d.slot_off + (uint64_t)j * d.slot_words), d.slot_words, c.ovf);
    seg_bits[(int64_t)d.block * s.bs + j] = (uint32_t)c.enc.nbits;
    if (c.ovf) atomicOr(err, 2);
  }
}

// Softmax + quantiser + coder + loss gradient of one slot's step (one
// workgroup per slot): the logits rows become probabilities, lane j < bs
// codes token i of segment j with its row's table (the uniform table before
// step t), and the rows become dL/dlogits = (P - onehot) / bs.
constexpr int kCodeT = 256;
// With the static model (lu given): Eq. 1 mixes alpha L^u + (1 - alpha) L^m,
// alpha = sigmoid(a) with a the slot's parameter P; the rows of lu become
// L^u - L^m, the loss gradient of the dynamic model is scaled by 1 - alpha,
// and a takes its own optimiser step from sum_rows (sum_v P_v (L^u_v - L^m_v)
// - (L^u_e - L^m_e)) / bs * alpha (1 - alpha), rows summed in order.
__global__ __launch_bounds__(kCodeT) void code_kernel(TfShape s, const TfState *st, const TfSlot *desc,
                                                      uint8_t *toks, uint32_t *sslots, float *logits, int64_t sLog,
                                                      uint32_t *cdf, int64_t sCdf, CoderState *coder, int mode,
                                                      float *probe, float *lu, float *params, float *adam_m,
                                                      float *adam_v) {
  const int slot = blockIdx.x;
  if (slot >= st->nact) return;
  __shared__ uint8_t tgt[1024];
  __shared__ float srow_s[1024];
  const TfSlot d = desc[slot];
  const int i = st->i, V = s.V, bs = s.bs, tid = threadIdx.x;
  const bool uniform = i < s.t;
  float *lg = logits + slot * sLog;
  float *ul = lu ? lu + slot * sLog : nullptr;
  uint32_t *cd = cdf + slot * sCdf;
  const bool mix = ul != nullptr;
  float *ap = mix ? params + slot * s.stride + s.P : nullptr;
  const float alpha = mix ? 1.0f / (1.0f + expf(-*ap)) : 0.0f;
  if (!uniform) {
    const int spl = row_spl(V), G = V / spl, gs = __builtin_ctz((unsigned)G);
    for (int j0 = 0; j0 < bs; j0 += kCodeT >> gs) {
      const int j = j0 + (tid >> gs), gl = tid & (G - 1);
      if (j >= bs) continue;
      float *lr = lg + (int64_t)j * V;
      float *ur = mix ? ul + (int64_t)j * V : nullptr;
      uint32_t *crow = cd + (int64_t)j * (V + 1);
      float *pp = probe ? probe + (int64_t)j * V + gl * spl : nullptr;
      float sr;
      if (spl == 4) {
        float pr[4];
        sr = row_softmax_regs<4>(lr, ur, mix, alpha, V, G, gl, crow, pr);
        if (pp) for (int c = 0; c < 4; c++) pp[c] = pr[c];
      } else if (spl == 8) {
        float pr[8];
        sr = row_softmax_regs<8>(lr, ur, mix, alpha, V, G, gl, crow, pr);
        if (pp) for (int c = 0; c < 8; c++) pp[c] = pr[c];
      } else {
        float pr[32];
        sr = row_softmax_regs<32>(lr, ur, mix, alpha, V, G, gl, crow, pr);
        if (pp) for (int c = 0; c < 32; c++) pp[c] = pr[c];
      }
      if (mix && gl == 0) srow_s[j] = sr;
    }
  } else if (probe) {
    for (int q = tid; q < bs * V; q += kCodeT) probe[q] = 1.0f / (float)V;
  }
  __syncthreads();
  const uint32_t unit = kTotal / (uint32_t)V;
  for (int j = tid; j < bs; j += kCodeT) {
    CoderState cs = coder[(int64_t)slot * bs + j];
    gu32 *sl = (gu32 *)(sslots + d.slot_off + (uint64_t)j * d.slot_words);
    const uint64_t pos = d.tok_off + (uint64_t)j * d.L + (uint64_t)i;
    const uint32_t *c = cd + (int64_t)j * (V + 1);
    int e;
    if (mode == 0) {
      e = toks[pos];
      uint32_t lo, hi;
      if (uniform) { lo = (uint32_t)e * unit; hi = lo + unit; }
      else { lo = c[e]; hi = c[e + 1]; }
      enc_symbol(cs.enc, sl, d.slot_words, lo, hi, cs.ovf);
    } else {
      if (uniform) e = dec_symbol(cs.dec, sl, cs.nwords, V, [&](int q) { return (uint32_t)q * unit; });
      else e = dec_symbol(cs.dec, sl, cs.nwords, V, [&](int q) { return c[q]; });
      toks[pos] = (uint8_t)e;
    }
    tgt[j] = (uint8_t)e;
    coder[(int64_t)slot * bs + j] = cs;
  }
  __syncthreads();
  if (uniform) return;
  const float inv_bs = 1.0f / (float)bs;
  const float scale = mix ? inv_bs * (1.0f - alpha) : inv_bs;
  for (int q = tid; q < bs * V; q += kCodeT) {
    const int j = q / V, v = q % V;
    lg[q] = (lg[q] - (v == tgt[j] ? 1.0f : 0.0f)) * scale;
  }
  if (mix && tid == 0) {
    float acc = 0.0f;
    for (int j = 0; j < bs; j++) acc += srow_s[j] - ul[(int64_t)j * V + tgt[j]];
    Opt o;
    o.kind = s.optimizer;
    o.lr = s.lr; o.b1 = s.b1; o.b2 = s.b2; o.eps = s.eps;
    o.c1 = st->c1;
    o.c2 = st->c2;
    float *mm = adam_m ? adam_m + slot * s.stride + s.P : nullptr;
    float *vv = adam_v ? adam_v + slot * s.stride + s.P : nullptr;
    *ap -= opt_delta(o, acc * inv_bs * (alpha * (1.0f - alpha)), mm, vv);
  }
}

// The BiGRU static model's logits for every row of a slot's step: one
// workgroup per R rows, one thread per (direction, gate row); the current
// layer's weights in LDS, the rows' hidden states, gate parts, context
// embeddings and (two layers) the first layer's output sequence beside
// them.  Per position the
// threads form the 3h input and hidden parts of their gate row for the R
// rows, then h threads per direction combine them (r, z, n, h'); the two
// directions run side by side.  FP32 throughout; every sum in order.
__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ float tanh_f(float x) { return 1.0f - 2.0f / (__expf(2.0f * x) + 1.0f); }

__global__ void bigru_kernel(TfShape s, const TfState *st, const float *W, const uint8_t *tokstep, int64_t sTok,
                             float *lu, int64_t sLu, int R) {
  const int slot = blockIdx.y;
  if (slot >= st->nact) return;
  extern __shared__ float sm[];
  const int h = s.gh, G = 3 * h, t = s.t, V = s.V, E = s.sE;
  const int IN = s.gl == 2 && 2 * h > E ? 2 * h : E;    // widest layer input
  const int tid = threadIdx.x, d = tid / G, g = tid % G;   // direction, gate row (blockDim = 2G)
  const int row0 = blockIdx.x * R, rows = min(R, s.bs - row0);
  // weight rows padded to an odd stride: a thread reading its own row and
  // lanes reading one column both hit distinct banks
  const int LI = IN + 1, LH = h + 1;
  float *wih = sm;                              // [2][G][IN + 1]
  float *whh = wih + 2 * G * LI;                // [2][G][h + 1]
  float *hs = whh + 2 * G * LH;                 // [R][2][h]
  float *ga = hs + R * 2 * h;                   // [R][2][G]
  float *gb = ga + R * 2 * G;                   // [R][2][G]
  float *seq = gb + R * 2 * G;                  // [R][t][2h] first layer's outputs (two layers)
  float *dn = seq + (s.gl == 2 ? R * t * 2 * h : 0);   // [R][gd]
  float *xs = dn + R * s.gd;                    // [R][t][E] the rows' context embeddings
  const uint8_t *tk = tokstep + slot * sTok;
  // the first layer's inputs, read once per step instead of once per position
  for (int q = tid; q < rows * t * E; q += blockDim.x) {
    const int r = q / (t * E), p = (q / E) % t;
    xs[q] = W[s.s_emb + (int64_t)tk[(int64_t)(row0 + r) * t + p] * E + q % E];
  }
  for (int l = 0; l < s.gl; l++) {
    const int in = l == 0 ? E : 2 * h;
    __syncthreads();
    for (int q = tid; q < 2 * G * in; q += blockDim.x) {
      const int dd = q / (G * in), rr = q % (G * in);
      wih[dd * G * LI + (rr / in) * LI + rr % in] = W[s.s_wih[l][dd] + rr];
    }
    for (int q = tid; q < 2 * G * h; q += blockDim.x) {
      const int dd = q / (G * h), rr = q % (G * h);
      whh[dd * G * LH + (rr / h) * LH + rr % h] = W[s.s_whh[l][dd] + rr];
    }
    for (int q = tid; q < R * 2 * h; q += blockDim.x) hs[q] = 0.0f;
    const float bi = W[s.s_bih[l][d] + g], bh = W[s.s_bhh[l][d] + g];
    const float *wi = wih + (d * G + g) * LI, *wh = whh + (d * G + g) * LH;
    __syncthreads();
    for (int step = 0; step < t; step++) {
      const int p = d == 0 ? step : t - 1 - step;
      for (int r = 0; r < rows; r++) {
        float a = bi, b = bh;
        if (l == 0) {
          const float *x = xs + (r * t + p) * E;
#pragma unroll 8
          for (int k = 0; k < E; k++) a += wi[k] * x[k];
        } else {
          const float *x = seq + (r * t + p) * 2 * h;
#pragma unroll 8
          for (int k = 0; k < 2 * h; k++) a += wi[k] * x[k];
        }
        const float *hp = hs + (r * 2 + d) * h;
#pragma unroll 8
        for (int k = 0; k < h; k++) b += wh[k] * hp[k];
        ga[(r * 2 + d) * G + g] = a;
        gb[(r * 2 + d) * G + g] = b;
      }
      __syncthreads();
      if (g < h) {
        for (int r = 0; r < rows; r++) {
          const float *xa = ga + (r * 2 + d) * G, *xb = gb + (r * 2 + d) * G;
          const float rg = sigm(xa[g] + xb[g]);
          const float zg = sigm(xa[h + g] + xb[h + g]);
          const float ng = tanh_f(xa[2 * h + g] + rg * xb[2 * h + g]);
          float *hp = hs + (r * 2 + d) * h;
          const float hn = (1.0f - zg) * ng + zg * hp[g];
          hp[g] = hn;
          if (l == 0 && s.gl == 2) seq[(r * t + p) * 2 * h + d * h + g] = hn;
        }
      }
      __syncthreads();
    }
  }
  // head: final states [forward | backward] -> Dense + ReLU -> linear
  for (int q = tid; q < rows * s.gd; q += blockDim.x) {
    const int r = q / s.gd, o = q % s.gd;
    float a = W[s.s_db + o];
    const float *hr = hs + r * 2 * h;
#pragma unroll 8
    for (int k = 0; k < 2 * h; k++) a += hr[k] * W[s.s_dw + (int64_t)k * s.gd + o];
    dn[r * s.gd + o] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  for (int q = tid; q < rows * V; q += blockDim.x) {
    const int r = q / V, v = q % V;
    float a = W[s.s_lb + v];
    const float *dr = dn + r * s.gd;
#pragma unroll 8
    for (int o = 0; o < s.gd; o++) a += dr[o] * W[s.s_lw + (int64_t)o * V + v];
    lu[slot * sLu + (int64_t)(row0 + r) * V + v] = a;
  }
}

// rows per workgroup of bigru_kernel and its LDS bytes (0: does not fit):
// at most 2 rows, so that a step's grid holds bs / 2 workgroups per block
// (measured faster than 1 or 8 rows per workgroup; the rows of a workgroup
// run one after another, and no value depends on how they are grouped)
int bigru_rows(const TfShape &s, size_t &bytes) {
  const int h = s.gh, G = 3 * h, IN = s.gl == 2 && 2 * h > s.sE ? 2 * h : s.sE;
  for (int R = 2; R >= 1; R >>= 1) {
    const size_t f = (size_t)2 * G * (IN + 1) + 2 * G * (h + 1) + R * 2 * h + 2 * R * 2 * G +
                     (s.gl == 2 ? (size_t)R * s.t * 2 * h : 0) + R * s.gd + (size_t)R * s.t * s.sE;
    if (f * 4 <= 150 * 1024) {
      bytes = f * 4;
      return R;
    }
  }
  bytes = 0;
  return 0;
}

// the op's own loss gradient is given: copy it into the logits rows
__global__ __launch_bounds__(256) void copy_kernel(const float *src, float *dst, int64_t n) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) dst[q] = src[q];
}

// ------------------------------------------------------------- host side
struct Ctx {
  const TfShape &s;
  const TfBufs &b;
  float *W;            // parameters of slot 0 (slot stride s.stride)
  float *gW;           // kGrad: gradient slab (one slot) or null
  const uint8_t *toks, *ctx;
  int n;               // slots launched
  hipStream_t st;
};

Gemm base_gemm(const Ctx &c) {
  Gemm g;
  memset(&g, 0, sizeof g);
  g.st = c.b.state;
  g.split = 1;
  g.opt = c.s.optimizer;
  g.lr = c.s.lr; g.b1 = c.s.b1; g.b2 = c.s.b2; g.eps = c.s.eps;
  return g;
}
Gemm mk(const Ctx &c, const float *A, int64_t lda, int64_t sA, const float *B, int64_t ldb, int64_t sB, float *C,
        int64_t ldc, int64_t sC, int M, int N, int K) {
  Gemm g = base_gemm(c);
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = B; g.ldb = ldb; g.sB = sB;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.M = M; g.N = N; g.K = K;
  g.part = c.b.part;
  g.sPart = c.b.sPart;
  return g;
}
// a weight-gradient product or column sum whose epilogue updates the
// weight at parameter offset `off` (kUpdate) or stores its gradient (kGrad)
// the MLP's first-layer input X read virtually from the embedding and the
// step's context tokens (see Gemm::emb) instead of from a gathered copy
void virtual_x(const Ctx &c, Gemm &g) {
  g.A = nullptr;
  g.sA = 0;
  g.emb = c.W + c.s.off_emb;
  g.sEmb = c.s.stride;
  g.xE = c.s.E;
  g.xt = c.s.t;
  g.oh = c.b.tokstep;
  g.sOh = c.b.sTok;
}

Gemm wgt(const Ctx &c, Gemm g, int64_t off) {
  if (c.gW) {
    g.C = c.gW + off;
    g.sC = 0;
  } else {
    g.C = c.W + off;
    g.sC = c.s.stride;
    g.m = c.b.adam_m ? c.b.adam_m + off : nullptr;
    g.v = c.b.adam_v ? c.b.adam_v + off : nullptr;
    g.sMV = c.s.stride;
  }
  return g;
}

#define TRY(x)                        \
  do {                                \
    hipError_t e_ = (x);              \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

hipError_t forward(const Ctx &c, int *err) {
  const TfShape &s = c.s;
  const TfBufs &b = c.b;
  const int bs = s.bs, t = s.t, E = s.E, A = s.A, F = s.F, V = s.V;
  const int64_t S = s.stride;
  float *W = c.W;
  const int64_t nx = (int64_t)bs * t * E;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((nx + 255) / 256), c.n), dim3(256), 0, c.st, s, b.state,
                     b.slots_desc, c.toks, c.ctx, W, b.X, b.sX, b.tokstep, b.sTok, err);
  TRY(hipGetLastError());
  // [k | v] for every position, q at the last
  Gemm g = mk(c, b.X, E, b.sX, W + s.off_W[0] + A, 3 * A, S, b.KV, 2 * A, b.sKV, bs * t, 2 * A, E);
  g.bias = W + s.off_b[0] + A;
  g.sBias = S;
  TRY((gemm<false, false, kStore>(s, g, c.n, c.st)));
  g = mk(c, b.X + (int64_t)(t - 1) * E, (int64_t)t * E, b.sX, W + s.off_W[0], 3 * A, S, b.Q, A, b.sQ, bs, A, E);
  g.bias = W + s.off_b[0];
  g.sBias = S;
  TRY((gemm<false, false, kStore>(s, g, c.n, c.st)));
  TRY(attn_allow_lds(s));
  hipLaunchKernelGGL(attn_fwd_kernel, dim3(bs, c.n), dim3(A), attn_lds(s), c.st, s, b.state, b.Q, b.KV, b.att,
                     b.O, b.sQ, b.sKV, b.sAtt, attn_chunk(s));
  TRY(hipGetLastError());
  struct L { const float *in; int64_t ldi, si; int K; int li; float *out; int N; int64_t so; int relu; };
  const L layers[4] = {{b.O, A, b.sQ, A, 1, b.Z, A, b.sQ, 0},
                       {b.Z, A, b.sQ, A, 2, b.U, F, b.sU, 1},
                       {b.U, F, b.sU, F, 3, b.G, A, b.sQ, 0},
                       {b.G, A, b.sQ, A, 4, b.logits, V, b.sLog, 0}};
  for (const L &l : layers) {
    g = mk(c, l.in, l.ldi, l.si, W + s.off_W[l.li], l.N, S, l.out, l.N, l.so, bs, l.N, l.K);
    g.bias = W + s.off_b[l.li];
    g.sBias = S;
    g.relu = l.relu;
    TRY((gemm<false, false, kStore>(s, g, c.n, c.st)));
  }
  return hipSuccess;
}

template <int EPI>
hipError_t backward(const Ctx &c) {
  const TfShape &s = c.s;
  const TfBufs &b = c.b;
  const int bs = s.bs, t = s.t, E = s.E, A = s.A, F = s.F, V = s.V;
  const int64_t S = s.stride;
  float *W = c.W;
  // one dense layer out = in W + b, given dout: din = dout W^T (masked by
  // the ReLU that produced `in` when given), then W and b together: the
  // product in^T dout with a row of ones appended to in^T gives b's
  // gradient as its last row, which lands on b (b follows W, same width)
  struct L { const float *in; int64_t ldi, si; int din_n; float *din; int64_t sdin; const float *mask;
             const float *dout; int64_t ldo, so; int N; int li; };
  const L layers[4] = {{b.G, A, b.sQ, A, b.dG, b.sQ, nullptr, b.logits, V, b.sLog, V, 4},
                       {b.U, F, b.sU, F, b.dU, b.sU, b.U, b.dG, A, b.sQ, A, 3},
                       {b.Z, A, b.sQ, A, b.dZ, b.sQ, nullptr, b.dU, F, b.sU, F, 2},
                       {b.O, A, b.sQ, A, b.dO, b.sQ, nullptr, b.dZ, A, b.sQ, A, 1}};
  for (const L &l : layers) {
    // din = dout W^T: W is [din_n][N], read transposed
    Gemm g = mk(c, l.dout, l.ldo, l.so, W + s.off_W[l.li], l.N, S, l.din, l.din_n, l.sdin, bs, l.din_n, l.N);
    if (l.mask) {
      g.mask = l.mask;
      g.ldm = l.din_n;
      g.sMask = l.sdin;
    }
    TRY((gemm<false, true, kStore>(s, g, c.n, c.st)));
    g = wgt(c, mk(c, l.in, l.ldi, l.si, l.dout, l.ldo, l.so, nullptr, l.N, 0, l.din_n, l.N, bs), s.off_W[l.li]);
    g.aug = 1;
    TRY((gemm<true, false, EPI>(s, g, c.n, c.st)));
  }
  TRY(attn_allow_lds(s));
  hipLaunchKernelGGL(attn_bwd_kernel, dim3(bs, c.n), dim3(A), attn_lds(s), c.st, s, b.state, b.Q, b.KV, b.att,
                     b.dO, b.dQ, b.dKV, b.sQ, b.sKV, b.sAtt, attn_chunk(s));
  TRY(hipGetLastError());
  // dX = dKV Wkv^T, then dX[row t + t - 1] += dQ Wq^T (before either weight changes)
  Gemm g = mk(c, b.dKV, 2 * A, b.sKV, W + s.off_W[0] + A, 3 * A, S, b.dX, E, b.sX, bs * t, E, 2 * A);
  TRY((gemm<false, true, kStore>(s, g, c.n, c.st)));
  g = mk(c, b.dQ, A, b.sQ, W + s.off_W[0], 3 * A, S, b.dX + (int64_t)(t - 1) * E, (int64_t)t * E, b.sX, bs, E, A);
  TRY((gemm<false, true, kAccum>(s, g, c.n, c.st)));
  // Wkv and bkv from X^T dKV (+ ones row), Wq and bq from Xlast^T dQ (+ ones
  // row): columns A..3A and 0..A of Wqkv, whose bias row follows it
  g = wgt(c, mk(c, b.X, E, b.sX, b.dKV, 2 * A, b.sKV, nullptr, 3 * A, 0, E, 2 * A, bs * t), s.off_W[0] + A);
  g.aug = 1;
  TRY((gemm<true, false, EPI>(s, g, c.n, c.st)));
  g = wgt(c, mk(c, b.X + (int64_t)(t - 1) * E, (int64_t)t * E, b.sX, b.dQ, A, b.sQ, nullptr, 3 * A, 0, E, A, bs),
          s.off_W[0]);
  g.aug = 1;
  TRY((gemm<true, false, EPI>(s, g, c.n, c.st)));
  // embeddings: dEmb = onehot(tokens)^T dX, dPos = onehot(position)^T dX
  g = wgt(c, mk(c, nullptr, 0, 0, b.dX, E, b.sX, nullptr, E, 0, V, E, bs * t), s.off_emb);
  g.oh = b.tokstep;
  g.sOh = b.sTok;
  TRY((gemm<true, false, EPI>(s, g, c.n, c.st)));
  g = wgt(c, mk(c, nullptr, 0, 0, b.dX, E, b.sX, nullptr, E, 0, t, E, bs * t), s.off_pos);
  g.oh_mod = t;
  return gemm<true, false, EPI>(s, g, c.n, c.st);
}

// The configurations' MLP on the launch sequence: x = concat(Emb[c_p]),
// h_{l+1} = ReLU(h_l W_l + b_l), logits = h_nh W_nh + b_nh.
hipError_t mlp_forward(const Ctx &c, int *err) {
  const TfShape &s = c.s;
  const TfBufs &b = c.b;
  const int bs = s.bs, t = s.t, E = s.E;
  const int64_t S = s.stride;
  float *W = c.W;
  const int64_t nrp = (int64_t)bs * t;
  hipLaunchKernelGGL(tokstep_kernel, dim3((unsigned)((nrp + 255) / 256), c.n), dim3(256), 0, c.st, s, b.state,
                     b.slots_desc, c.toks, c.ctx, b.tokstep, b.sTok, err);
  TRY(hipGetLastError());
  const int dims[4] = {t * E, s.H0, s.H1, s.V};
  const float *in = nullptr;   // the first layer reads X virtually
  int64_t ldi = t * E, si = 0;
  for (int l = 0; l <= s.nh; l++) {
    const int N = l == s.nh ? s.V : dims[l + 1];
    float *out = l == s.nh ? b.logits : b.act[l];
    const int64_t so = l == s.nh ? b.sLog : b.sAct[l];
    Gemm g = mk(c, in, ldi, si, W + s.off_W[l], N, S, out, N, so, bs, N, (int)ldi);
    if (l == 0) virtual_x(c, g);
    g.bias = W + s.off_b[l];
    g.sBias = S;
    g.relu = l < s.nh;
    TRY((gemm<false, false, kStore>(s, g, c.n, c.st)));
    in = out;
    ldi = N;
    si = so;
  }
  return hipSuccess;
}

template <int EPI>
hipError_t mlp_backward(const Ctx &c) {
  const TfShape &s = c.s;
  const TfBufs &b = c.b;
  const int bs = s.bs, t = s.t, E = s.E, V = s.V;
  const int64_t S = s.stride;
  float *W = c.W;
  const int dims[3] = {t * E, s.H0, s.H1};
  for (int l = s.nh; l >= 0; l--) {
    const int din_n = dims[l], N = l == s.nh ? V : dims[l + 1];
    const float *dout = l == s.nh ? b.logits : b.dact[l];
    const int64_t so = l == s.nh ? b.sLog : b.sAct[l];
    const float *in = l == 0 ? nullptr : b.act[l - 1];   // layer 0: X, read virtually
    const int64_t si = l == 0 ? 0 : b.sAct[l - 1];
    float *din = l == 0 ? b.dX : b.dact[l - 1];
    const int64_t sdin = l == 0 ? b.sX : b.sAct[l - 1];
    // din = dout W_l^T, masked by the ReLU that produced `in` (not for x)
    Gemm g = mk(c, dout, N, so, W + s.off_W[l], N, S, din, din_n, sdin, bs, din_n, N);
    if (l > 0) {
      g.mask = in;
      g.ldm = din_n;
      g.sMask = si;
    } else {
      g.hc = s.bf16;   // dX: read only by the embedding product below
    }
    TRY((gemm<false, true, kStore>(s, g, c.n, c.st)));
    // W_l and b_l: in^T dout with a ones row for the bias, which follows W_l
    g = wgt(c, mk(c, in, din_n, si, dout, N, so, nullptr, N, 0, din_n, N, bs), s.off_W[l]);
    if (l == 0) virtual_x(c, g);
    g.aug = 1;
    TRY((gemm<true, false, EPI>(s, g, c.n, c.st)));
  }
  // dEmb = onehot(tokens)^T dX, dX viewed as [bs t][E]; in BF16 it was
  // stored rounded as this product would round it
  Gemm g = wgt(c, mk(c, nullptr, 0, 0, b.dX, E, b.sX, nullptr, E, 0, V, E, bs * t), s.off_emb);
  g.oh = b.tokstep;
  g.sOh = b.sTok;
  g.hb = s.bf16;
  return gemm<true, false, EPI>(s, g, c.n, c.st);
}

}  // namespace

bool bigru_shape(int sE, int gh, int gl, int gd, TfShape &s) {
  if (sE < 1 || sE > 256 || gh < 1 || gh > 128 || gl < 1 || gl > 2 || gd < 1) return false;
  s.sarch = 1;
  s.sE = sE; s.gh = gh; s.gl = gl; s.gd = gd;
  int64_t off = 0;
  s.s_emb = off;
  off += (int64_t)s.V * sE;
  for (int l = 0; l < gl; l++) {
    const int64_t in = l == 0 ? sE : 2 * gh;
    for (int d = 0; d < 2; d++) {
      s.s_wih[l][d] = off; off += 3ll * gh * in;
      s.s_whh[l][d] = off; off += 3ll * gh * gh;
      s.s_bih[l][d] = off; off += 3ll * gh;
      s.s_bhh[l][d] = off; off += 3ll * gh;
    }
  }
  s.s_dw = off; off += 2ll * gh * gd;
  s.s_db = off; off += gd;
  s.s_lw = off; off += (int64_t)gd * s.V;
  s.s_lb = off; off += s.V;
  s.sP = off;
  size_t lds;
  return bigru_rows(s, lds) > 0;
}

bool mlp_seq_shape(const Dims &d, TfShape &s) {
  memset(&s, 0, sizeof s);
  if (d.nh > 2 || d.V > 256 || d.bs < 1 || d.bs > 1024 || d.E > 1024 || d.t > 65535) return false;
  s.arch = 0;
  s.nh = d.nh;
  s.H0 = d.nh >= 1 ? d.H[0] : 0;
  s.H1 = d.nh >= 2 ? d.H[1] : 0;
  s.V = d.V; s.E = d.E; s.t = d.t; s.bs = d.bs;
  s.H = 1; s.dh = 1;
  s.off_emb = d.off_emb;
  s.off_pos = -1;
  for (int l = 0; l <= d.nh; l++) {
    s.off_W[l] = d.off_W[l];
    s.off_b[l] = d.off_b[l];
  }
  s.P = d.P;
  s.stride = d.stride;
  s.optimizer = d.optimizer;
  s.lr = d.lr; s.b1 = d.b1; s.b2 = d.b2; s.eps = d.eps;
  return true;
}

bool tf_shape(int k, int t, int E, int A, int F, int H, TfShape &s) {
  memset(&s, 0, sizeof s);
  s.arch = 1;
  if (k < 1 || k > 4 || t < 1 || t > 256 || E < 1 || E > 1024 || A < 1 || A > 1024 || F < 1 || H < 1 || A % H)
    return false;
  const int dh = A / H;
  if (dh > 64 || (dh & (dh - 1)) || H * t > 16384) return false;
  s.V = 1 << (2 * k);
  s.E = E; s.t = t; s.A = A; s.F = F; s.H = H; s.dh = dh;
  const int64_t rows[5] = {E, A, A, F, A}, cols[5] = {3ll * A, A, F, A, s.V};
  int64_t off = 0;
  s.off_emb = off;
  off += (int64_t)s.V * E;
  s.off_pos = off;
  off += (int64_t)t * E;
  for (int l = 0; l < 5; l++) {
    s.off_W[l] = off;
    off += rows[l] * cols[l];
    s.off_b[l] = off;
    off += cols[l];
  }
  s.P = off;
  s.stride = (off + 1 + 63) / 64 * 64;
  return off < (1ll << 31);
}

uint64_t tf_bufs_carve(const TfShape &s, int n, float *base, TfBufs &b) {
  const int64_t bs = s.bs, t = s.t, E = s.E, A = s.A, F = s.F, V = s.V, H = s.H;
  uint64_t used = 0;
  auto take = [&](int64_t per, int64_t &stride) -> float * {
    stride = (per + 63) / 64 * 64;   // 256-byte aligned slots
    float *p = base ? base + used : nullptr;
    used += (uint64_t)stride * (uint64_t)n;
    return p;
  };
  int64_t dummy;
  if (s.arch == 0) {
    // the MLP reads its X virtually (Gemm::emb): only dX is kept, and sX
    // is its slot stride
    b.X = nullptr;
    b.dX = take(bs * t * E, b.sX);
    const int64_t hw[2] = {s.H0, s.H1};
    for (int l = 0; l < 2; l++) {
      b.act[l] = take(l < s.nh ? bs * hw[l] : 0, b.sAct[l]);
      b.dact[l] = take(l < s.nh ? bs * hw[l] : 0, dummy);
    }
    b.logits = take(bs * V, b.sLog);
    b.lu = take(s.sarch ? bs * V : 0, dummy);
    b.part = take(std::max<int64_t>(8 * bs * std::max<int64_t>(std::max<int64_t>(s.H0, s.H1), V), 16 * V * E),
                  b.sPart);
    b.cdf = reinterpret_cast<uint32_t *>(take(bs * (V + 1), b.sCdf));
    b.coder = take(bs * (int64_t)(sizeof(CoderState) / 4), dummy);
    int64_t stok;
    b.tokstep = reinterpret_cast<uint8_t *>(take((bs * t + 3) / 4, stok));
    b.sTok = stok * 4;
    return used;
  }
  b.X = take(bs * t * E, b.sX);
  b.dX = take(bs * t * E, dummy);
  b.KV = take(bs * t * 2 * A, b.sKV);
  b.dKV = take(bs * t * 2 * A, dummy);
  b.Q = take(bs * A, b.sQ);
  b.O = take(bs * A, dummy);
  b.Z = take(bs * A, dummy);
  b.G = take(bs * A, dummy);
  b.dG = take(bs * A, dummy);
  b.dZ = take(bs * A, dummy);
  b.dO = take(bs * A, dummy);
  b.dQ = take(bs * A, dummy);
  b.att = take(bs * H * t, b.sAtt);
  b.U = take(bs * F, b.sU);
  b.dU = take(bs * F, dummy);
  b.logits = take(bs * V, b.sLog);
  b.part = take((int64_t)kTfSplit * std::max<int64_t>(bs * A, E * 2 * A), b.sPart);
  b.cdf = reinterpret_cast<uint32_t *>(take(bs * (V + 1), b.sCdf));
  b.coder = take(bs * (int64_t)(sizeof(CoderState) / 4), dummy);
  int64_t stok;
  b.tokstep = reinterpret_cast<uint8_t *>(take((bs * t + 3) / 4, stok));
  b.sTok = stok * 4;
  b.sA = b.sQ;
  return used;
}

hipError_t tf_init_params(const TfShape &s, uint64_t seed, float *out, hipStream_t st) {
  // the same SplitMix64 draws and scales as the MLP's initialiser: 1 for
  // the embeddings, 1/sqrt(fan_in) for each linear layer's weight and bias
  int end[6];
  double sc[6];
  const int64_t fan[5] = {s.E, s.A, s.A, s.F, s.A};
  end[0] = (int)s.off_W[0];
  sc[0] = 1.0;
  for (int l = 0; l < 5; l++) {
    end[l + 1] = (int)(l + 1 < 5 ? s.off_W[l + 1] : s.P);
    sc[l + 1] = 1.0 / sqrt((double)fan[l]);
  }
  return launch_init_scaled(seed, (int)s.P, 6, end, sc, out, st);
}

hipError_t tf_run(const TfShape &s, const TfBufs &b, const TfRun &r, hipStream_t st) {
  if (r.n <= 0) return hipSuccess;
  int *err = &b.state->pad[0];
  Ctx c{s, b, b.params, nullptr, r.tokens, nullptr, r.n, st};
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, st, b.state, r.n);
  TRY(hipGetLastError());
  hipLaunchKernelGGL(slot_init_kernel, dim3((unsigned)std::min<int64_t>((s.stride + 255) / 256, 1024), r.n),
                     dim3(256), 0, st, s, r.n, b.init, b.params, b.adam_m, b.adam_v);
  TRY(hipGetLastError());
  hipLaunchKernelGGL(coder_init_kernel, dim3(r.n), dim3(256), 0, st, s, r.n, b.slots_desc,
                     reinterpret_cast<CoderState *>(b.coder), r.stream_slots, r.seg_words, r.mode);
  TRY(hipGetLastError());
  const TfSlot *desc = r.desc_host;   // slot lengths, longest first
  const uint64_t steps = r.stop ? std::min<uint64_t>(r.stop, r.max_L) : r.max_L;
  int probe_i = 0;
  int nact = r.n;
  for (uint64_t i = 0; i < steps; i++) {
    while (nact > 0 && desc[nact - 1].L <= i) nact--;
    if (nact == 0) break;
    c.n = nact;
    hipLaunchKernelGGL(begin_step_kernel, dim3(1), dim3(1), 0, st, s, b.state, (int)i, nact);
    TRY(hipGetLastError());
    if (i >= (uint64_t)s.t) {
      TRY(s.arch == 1 ? forward(c, err) : mlp_forward(c, err));
      if (s.sarch == 1) {
        size_t lds = 0;
        const int R = bigru_rows(s, lds);
        static bool lds_set = false;   // dynamic LDS beyond 64 KB needs the kernel's attribute once
        if (!lds_set) {
          TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(&bigru_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024));
          lds_set = true;
        }
        hipLaunchKernelGGL(bigru_kernel, dim3((s.bs + R - 1) / R, nact), dim3(6 * s.gh), lds, st, s, b.state, b.stat,
                           b.tokstep, b.sTok, b.lu, b.sLog, R);
        TRY(hipGetLastError());
      }
    }
    float *probe = nullptr;
    if (r.probe_P && probe_i < r.n_probe && r.probe_steps_host[probe_i] == i)
      probe = r.probe_P + (int64_t)(probe_i++) * s.bs * s.V;
    hipLaunchKernelGGL(code_kernel, dim3(nact), dim3(kCodeT), 0, st, s, b.state, b.slots_desc, r.tokens,
                       r.stream_slots, b.logits, b.sLog, b.cdf, b.sCdf, reinterpret_cast<CoderState *>(b.coder),
                       r.mode, probe, s.sarch == 1 ? b.lu : nullptr, b.params, b.adam_m, b.adam_v);
    TRY(hipGetLastError());
    if (i >= (uint64_t)s.t) TRY(s.arch == 1 ? backward<kUpdate>(c) : mlp_backward<kUpdate>(c));
    if (r.progress && (i + 1) % r.progress == 0) {
      TRY(hipStreamSynchronize(st));
      fprintf(stderr, "[pmklc] %s: step %llu of %llu, %d blocks active\n", r.mode ? "decompress" : "compress",
              (unsigned long long)(i + 1), (unsigned long long)steps, nact);
      fflush(stderr);
    }
  }
  if (r.mode == 0) {
    hipLaunchKernelGGL(coder_finish_kernel, dim3(r.n), dim3(256), 0, st, s, r.n, b.slots_desc,
                       reinterpret_cast<CoderState *>(b.coder), r.stream_slots, r.seg_bits, err);
    TRY(hipGetLastError());
  }
  if (r.params_out) TRY(hipMemcpyAsync(r.params_out, b.params, sizeof(float) * (s.P + 1), hipMemcpyDeviceToDevice, st));
  return hipSuccess;
}

hipError_t tf_forward_op(const TfShape &s, const TfBufs &b, const float *params, const uint8_t *ctx, float *logits,
                         hipStream_t st) {
  int *err = &b.state->pad[0];
  Ctx c{s, b, const_cast<float *>(params), nullptr, nullptr, ctx, 1, st};
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, st, b.state, 1);
  TRY(hipGetLastError());
  hipLaunchKernelGGL(begin_step_kernel, dim3(1), dim3(1), 0, st, s, b.state, s.t, 1);
  TRY(hipGetLastError());
  TRY(s.arch == 1 ? forward(c, err) : mlp_forward(c, err));
  const int64_t n = (int64_t)s.bs * s.V;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, b.logits, logits, n);
  return hipGetLastError();
}

hipError_t tf_backward_op(const TfShape &s, const TfBufs &b, const float *params, const uint8_t *ctx,
                          const float *dlogits, float *grad, hipStream_t st) {
  int *err = &b.state->pad[0];
  Ctx c{s, b, const_cast<float *>(params), grad, nullptr, ctx, 1, st};
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(1), 0, st, b.state, 1);
  TRY(hipGetLastError());
  hipLaunchKernelGGL(begin_step_kernel, dim3(1), dim3(1), 0, st, s, b.state, s.t, 1);
  TRY(hipGetLastError());
  // activations recomputed from the contexts, then the backward
  TRY(s.arch == 1 ? forward(c, err) : mlp_forward(c, err));
  const int64_t n = (int64_t)s.bs * s.V;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dlogits, b.logits, n);
  TRY(hipGetLastError());
  return s.arch == 1 ? backward<kGrad>(c) : mlp_backward<kGrad>(c);
}

}  // namespace pmklc
