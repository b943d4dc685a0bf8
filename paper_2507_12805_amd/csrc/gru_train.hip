// Training of the one-layer BiGRU static private model on the input
// (Sec. 4.2.3, the static model of Sec. 4.2.2 as the private one): the
// dynamic model's learning steps (Sec. 2 steps (2)-(4), its optimiser and
// learning rate, no other model mixed in) over the gathered training block
// of bs segments of Lp tokens; steps t..Lp-1 each make one update from the
// mean cross-entropy of the bs rows.  FP32 throughout.
//
// One learned step i is six launches on the caller's stream:
//   gru_fwd_kernel    the recurrence of both directions per R rows (one
//                     thread per (direction, gate row), as the inference
//                     kernel), every position's state kept for the backward,
//                     the Dense (ReLU) output and the logits;
//   gru_loss_kernel   softmax and dL/dlogits = (P - onehot) / bs;
//   gru_du_kernel, gru_dgrad_kernel
//                     the head and Dense layers' gradients and dL/dfeat
//                     (one output per thread, sums over the rows in order);
//   gru_bptt_kernel   back-propagation through time per R rows (one thread
//                     per (direction, gate row), its weight-gradient rows in
//                     registers; gates recomputed from the kept states; the
//                     embedding gradient per direction in LDS, rows in order)
//                     into one partial gradient per workgroup;
//   gru_update_kernel the partials summed in workgroup order, then the
//                     optimiser step of every parameter.
// Every value is computed in a fixed order, so the trained model does not
// depend on scheduling.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "pmklc_internal.h"
#include "seq_loop.h"
#include "step_common.h"

namespace pmklc {

namespace {

constexpr int kEmax = 32, kHmax = 64;   // embedding width and units per direction the training kernels hold

__device__ __forceinline__ float sg(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ float th(float x) { return 1.0f - 2.0f / (__expf(2.0f * x) + 1.0f); }

// context token (row, p) of step i: the training block holds row j's
// segment at j Lp
__device__ __forceinline__ int ctx_tok(const uint8_t *tok, uint64_t Lp, int i, int t, int row, int p) {
  return tok[(uint64_t)row * Lp + (uint64_t)(i - t + p)];
}

// Forward of the rows [row0, row0 + R) of step i.  seq[row][p][2h] receives
// the state after position p of each direction (forward half, backward
// half); dn[row][gd] the post-ReLU Dense output; lg[row][V] the logits.
// LDS: W_ih [2][G][E + 1], W_hh [2][G][h + 1] (rows padded), states
// [R][2][h], pre-activations [R][2][G] twice, the rows' context embeddings
// [R][t][E].
__global__ __launch_bounds__(384) void gru_fwd_kernel(TfShape s, const uint8_t *tok, uint64_t Lp, int i,
                                                      const float *W, float *seq, float *dn, float *lg, int R) {
  extern __shared__ float sm[];
  const int h = s.gh, G = 3 * h, t = s.t, E = s.sE, V = s.V, gd = s.gd;
  const int tid = threadIdx.x, d = tid / G, g = tid % G;
  const int row0 = blockIdx.x * R, rows = min(R, s.bs - row0);
  const int LE = E + 1, LH = h + 1;   // weight rows padded to an odd stride (no bank conflicts)
  float *wih = sm, *whh = wih + 2 * G * LE, *hs = whh + 2 * G * LH, *ga = hs + R * 2 * h, *gb = ga + R * 2 * G,
        *xs = gb + R * 2 * G;
  for (int q = tid; q < 2 * G * E; q += blockDim.x)
    wih[(q / E) * LE + q % E] = W[s.s_wih[0][q / (G * E)] + q % (G * E)];
  for (int q = tid; q < 2 * G * h; q += blockDim.x)
    whh[(q / h) * LH + q % h] = W[s.s_whh[0][q / (G * h)] + q % (G * h)];
  for (int q = tid; q < R * 2 * h; q += blockDim.x) hs[q] = 0.0f;
  for (int q = tid; q < rows * t * E; q += blockDim.x) {
    const int r = q / (t * E), p = (q / E) % t;
    xs[q] = W[s.s_emb + (int64_t)ctx_tok(tok, Lp, i, t, row0 + r, p) * E + q % E];
  }
  const float bi = W[s.s_bih[0][d] + g], bh = W[s.s_bhh[0][d] + g];
  const float *wi = wih + (d * G + g) * LE, *wh = whh + (d * G + g) * LH;
  __syncthreads();
  for (int step = 0; step < t; step++) {
    const int p = d == 0 ? step : t - 1 - step;
    for (int r = 0; r < rows; r++) {
      const float *x = xs + (r * t + p) * E;
      float a = bi, b = bh;
#pragma unroll 8
      for (int k = 0; k < E; k++) a += wi[k] * x[k];
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
        const float rg = sg(xa[g] + xb[g]);
        const float zg = sg(xa[h + g] + xb[h + g]);
        const float ng = th(xa[2 * h + g] + rg * xb[2 * h + g]);
        float *hp = hs + (r * 2 + d) * h;
        const float hn = (1.0f - zg) * ng + zg * hp[g];
        hp[g] = hn;
        seq[((int64_t)(row0 + r) * t + p) * 2 * h + d * h + g] = hn;
      }
    }
    __syncthreads();
  }
  // final states [forward after t-1 | backward after 0] -> Dense + ReLU -> head
  for (int q = tid; q < rows * gd; q += blockDim.x) {
    const int r = q / gd, o = q % gd;
    float a = W[s.s_db + o];
    const float *hr = hs + r * 2 * h;
#pragma unroll 8
    for (int k = 0; k < 2 * h; k++) a += hr[k] * W[s.s_dw + (int64_t)k * gd + o];
    dn[(int64_t)(row0 + r) * gd + o] = a > 0.0f ? a : 0.0f;
  }
  __syncthreads();
  for (int q = tid; q < rows * V; q += blockDim.x) {
    const int r = q / V, v = q % V;
    float a = W[s.s_lb + v];
    const float *dr = dn + (int64_t)(row0 + r) * gd;
#pragma unroll 8
    for (int o = 0; o < gd; o++) a += dr[o] * W[s.s_lw + (int64_t)o * V + v];
    lg[(int64_t)(row0 + r) * V + v] = a;
  }
}

// lg[row] (logits) becomes (softmax - onehot(target)) / bs; one thread per row
__global__ __launch_bounds__(256) void gru_loss_kernel(TfShape s, const uint8_t *tok, uint64_t Lp, int i, float *lg) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= s.bs) return;
  const int V = s.V;
  float *z = lg + (int64_t)row * V;
  float mx = z[0];
  for (int v = 1; v < V; v++) mx = fmaxf(mx, z[v]);
  float sum = 0.0f;
  for (int v = 0; v < V; v++) sum += __expf(z[v] - mx);
  const float inv = 1.0f / sum, scale = 1.0f / (float)s.bs;
  const int e = tok[(uint64_t)row * Lp + (uint64_t)i];
  for (int v = 0; v < V; v++) z[v] = (__expf(z[v] - mx) * inv - (v == e ? 1.0f : 0.0f)) * scale;
}

// The head and Dense layers' backward, one output per thread: du = (dz
// Wl^T) * [dn > 0]; then the gradients of Wl, bl, Wd, bd into gr (the
// parameter layout) and dfeat = du Wd^T.  Sums over rows run in row order.
__global__ __launch_bounds__(256) void gru_du_kernel(TfShape s, const float *W, const float *dn, const float *dz,
                                                     float *du) {
  const int V = s.V, gd = s.gd;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= s.bs * gd) return;
  const int j = q / gd, o = q % gd;
  float a = 0.0f;
#pragma unroll 8
  for (int v = 0; v < V; v++) a += dz[(int64_t)j * V + v] * W[s.s_lw + (int64_t)o * V + v];
  du[q] = dn[q] > 0.0f ? a : 0.0f;
}
__global__ __launch_bounds__(256) void gru_dgrad_kernel(TfShape s, const float *W, const float *seq, const float *dn,
                                                        const float *dz, const float *du, float *gr, float *dfeat) {
  const int h = s.gh, t = s.t, V = s.V, gd = s.gd, bs = s.bs, F = 2 * h;
  const int n_lw = gd * V, n_lb = V, n_dw = F * gd, n_db = gd, n_df = bs * F;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= n_lw + n_lb + n_dw + n_db + n_df) return;
  auto feat = [&](int j, int k) {
    return k < h ? seq[((int64_t)j * t + t - 1) * F + k] : seq[((int64_t)j * t) * F + k];
  };
  float a = 0.0f;
  if (q < n_lw) {
    const int o = q / V, v = q % V;
#pragma unroll 8
    for (int j = 0; j < bs; j++) a += dn[(int64_t)j * gd + o] * dz[(int64_t)j * V + v];
    gr[s.s_lw + q] = a;
  } else if (q < n_lw + n_lb) {
    const int v = q - n_lw;
    for (int j = 0; j < bs; j++) a += dz[(int64_t)j * V + v];
    gr[s.s_lb + v] = a;
  } else if (q < n_lw + n_lb + n_dw) {
    const int r = q - n_lw - n_lb, k = r / gd, o = r % gd;
#pragma unroll 8
    for (int j = 0; j < bs; j++) a += feat(j, k) * du[(int64_t)j * gd + o];
    gr[s.s_dw + r] = a;
  } else if (q < n_lw + n_lb + n_dw + n_db) {
    const int o = q - n_lw - n_lb - n_dw;
    for (int j = 0; j < bs; j++) a += du[(int64_t)j * gd + o];
    gr[s.s_db + o] = a;
  } else {
    const int r = q - n_lw - n_lb - n_dw - n_db, j = r / F, k = r % F;
#pragma unroll 8
    for (int o = 0; o < gd; o++) a += du[(int64_t)j * gd + o] * W[s.s_dw + (int64_t)k * gd + o];
    dfeat[r] = a;
  }
}

// Back-propagation through time for the rows [row0, row0 + R) of step i,
// each direction from its final state (dL/dfeat) back to its first
// position, the gates recomputed from the kept states.  With a = W_i x +
// b_i, b = W_h h + b_h per gate row: dn = dh' (1 - z), dz = dh' (h - n),
// dA_n = dn (1 - n^2), dA_r = dA_n b_n r (1 - r), dA_z = dz z (1 - z);
// input rows (dA_r, dA_z, dA_n), hidden rows (dA_r, dA_z, dA_n r);
// dh = dh' z + W_h^T (hidden rows), dx = W_i^T (input rows) onto the
// position's embedding row.  part[blockIdx.x] receives this workgroup's
// gradient of the GRU tensors (their layout from s_wih[0][0]) and, after
// them, of the embedding per direction [2][V][E].
// LDS: W_ih [2][G][E + 1], W_hh [2][G][h + 1] (rows padded), pre-activations
// [R][2][G] twice, input and hidden rows [R][2][G] twice, dh [R][2][h],
// embedding [2][V][E], the rows' context embeddings [R][t][E] and kept
// states [R][t][2h].
__global__ __launch_bounds__(384) void gru_bptt_kernel(TfShape s, const uint8_t *tok, uint64_t Lp, int i,
                                                       const float *W, const float *seq, const float *dfeat,
                                                       float *part, int64_t part_stride, int R) {
  extern __shared__ float sm[];
  const int h = s.gh, G = 3 * h, t = s.t, E = s.sE, V = s.V, F = 2 * h;
  const int tid = threadIdx.x, d = tid / G, g = tid % G;
  const int row0 = blockIdx.x * R, rows = min(R, s.bs - row0);
  const int LE = E + 1, LH = h + 1;   // weight rows padded to an odd stride (no bank conflicts)
  float *wih = sm, *whh = wih + 2 * G * LE, *ga = whh + 2 * G * LH, *gb = ga + R * 2 * G, *gi = gb + R * 2 * G,
        *gh = gi + R * 2 * G, *dh = gh + R * 2 * G, *de = dh + R * 2 * h, *xs = de + 2 * V * E,
        *hsq = xs + R * t * E;
  for (int q = tid; q < 2 * G * E; q += blockDim.x)
    wih[(q / E) * LE + q % E] = W[s.s_wih[0][q / (G * E)] + q % (G * E)];
  for (int q = tid; q < 2 * G * h; q += blockDim.x)
    whh[(q / h) * LH + q % h] = W[s.s_whh[0][q / (G * h)] + q % (G * h)];
  for (int q = tid; q < 2 * V * E; q += blockDim.x) de[q] = 0.0f;
  for (int q = tid; q < rows * t * E; q += blockDim.x) {
    const int r = q / (t * E), p = (q / E) % t;
    xs[q] = W[s.s_emb + (int64_t)ctx_tok(tok, Lp, i, t, row0 + r, p) * E + q % E];
  }
  for (int q = tid; q < rows * t * F; q += blockDim.x) hsq[q] = seq[(int64_t)row0 * t * F + q];
  for (int q = tid; q < R * 2 * h; q += blockDim.x) {
    const int r = q / F, dd = (q / h) % 2, u = q % h;
    dh[q] = r < rows ? dfeat[(int64_t)(row0 + r) * F + dd * h + u] : 0.0f;
  }
  const float bi = W[s.s_bih[0][d] + g], bh = W[s.s_bhh[0][d] + g];
  const float *wi = wih + (d * G + g) * LE, *wh = whh + (d * G + g) * LH;
  float awi[kEmax], awh[kHmax], abi = 0.0f, abh = 0.0f;
#pragma unroll
  for (int k = 0; k < kEmax; k++) awi[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < kHmax; k++) awh[k] = 0.0f;
  __syncthreads();
  for (int step = t - 1; step >= 0; step--) {
    const int p = d == 0 ? step : t - 1 - step;
    const int pp = d == 0 ? p - 1 : p + 1;    // the position processed before p (step > 0)
    // pre-activations of this position from the kept states
    for (int r = 0; r < rows; r++) {
      const float *x = xs + (r * t + p) * E;
      float a = bi, b = bh;
#pragma unroll 8
      for (int k = 0; k < E; k++) a += wi[k] * x[k];
      if (step > 0) {
        const float *hp = hsq + (r * t + pp) * F + d * h;
#pragma unroll 8
        for (int k = 0; k < h; k++) b += wh[k] * hp[k];
      }
      ga[(r * 2 + d) * G + g] = a;
      gb[(r * 2 + d) * G + g] = b;
    }
    __syncthreads();
    if (g < h) {
      for (int r = 0; r < rows; r++) {
        const int o = (r * 2 + d) * G;
        const float rg = sg(ga[o + g] + gb[o + g]);
        const float zg = sg(ga[o + h + g] + gb[o + h + g]);
        const float ng = th(ga[o + 2 * h + g] + rg * gb[o + 2 * h + g]);
        const float hprev = step > 0 ? hsq[(r * t + pp) * F + d * h + g] : 0.0f;
        float *dhr = dh + (r * 2 + d) * h;
        const float dhu = dhr[g];
        const float dnn = dhu * (1.0f - zg), dzz = dhu * (hprev - ng);
        const float dan = dnn * (1.0f - ng * ng);
        const float dar = dan * gb[o + 2 * h + g] * rg * (1.0f - rg), daz = dzz * zg * (1.0f - zg);
        gi[o + g] = dar;
        gi[o + h + g] = daz;
        gi[o + 2 * h + g] = dan;
        gh[o + g] = dar;
        gh[o + h + g] = daz;
        gh[o + 2 * h + g] = dan * rg;
        dhr[g] = dhu * zg;   // the direct part; the hidden rows' part is added below
      }
    }
    __syncthreads();
    for (int r = 0; r < rows; r++) {
      const int o = (r * 2 + d) * G;
      const int tk = ctx_tok(tok, Lp, i, t, row0 + r, p);
      const float *x = xs + (r * t + p) * E;
      // this thread's gate row: weight and bias gradients
      const float vi = gi[o + g], vh = gh[o + g];
      abi += vi;
      abh += vh;
#pragma unroll
      for (int k = 0; k < kEmax; k++)
        if (k < E) awi[k] += vi * x[k];
      if (step > 0) {
        const float *hp = hsq + (r * t + pp) * F + d * h;
#pragma unroll
        for (int k = 0; k < kHmax; k++)
          if (k < h) awh[k] += vh * hp[k];
      }
      // dh of the previous position (unit g) and dx (component g) of this one
      if (g < h && step > 0) {
        float a = 0.0f;
#pragma unroll 8
        for (int q = 0; q < G; q++) a += whh[(d * G + q) * LH + g] * gh[o + q];
        dh[(r * 2 + d) * h + g] += a;
      }
      for (int e = g; e < E; e += G) {
        float a = 0.0f;
#pragma unroll 8
        for (int q = 0; q < G; q++) a += wih[(d * G + q) * LE + e] * gi[o + q];
        de[(d * V + tk) * E + e] += a;
      }
    }
    __syncthreads();
  }
  float *pw = part + (int64_t)blockIdx.x * part_stride;
  const int64_t base = s.s_wih[0][0];
#pragma unroll
  for (int k = 0; k < kEmax; k++)
    if (k < E) pw[s.s_wih[0][d] - base + (int64_t)g * E + k] = awi[k];
#pragma unroll
  for (int k = 0; k < kHmax; k++)
    if (k < h) pw[s.s_whh[0][d] - base + (int64_t)g * h + k] = awh[k];
  pw[s.s_bih[0][d] - base + g] = abi;
  pw[s.s_bhh[0][d] - base + g] = abh;
  const int64_t ne = s.s_dw - base;   // the GRU tensors' length
  for (int q = tid; q < 2 * V * E; q += blockDim.x) pw[ne + q] = de[q];
}

// every parameter: its gradient (embedding and GRU tensors: the partials in
// workgroup order, the embedding's two directions in order; the dense
// layers: gr), then the optimiser step
__global__ __launch_bounds__(256) void gru_update_kernel(TfShape s, float *W, const float *gr, const float *part,
                                                         int64_t part_stride, int nwg, float *m, float *v, float c1,
                                                         float c2) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= s.sP) return;
  const int64_t base = s.s_wih[0][0], ne = s.s_dw - base, VE = (int64_t)s.V * s.sE;
  float g = 0.0f;
  if (q < base) {
    for (int w = 0; w < nwg; w++)
      for (int dd = 0; dd < 2; dd++) g += part[(int64_t)w * part_stride + ne + dd * VE + q];
  } else if (q < s.s_dw) {
    for (int w = 0; w < nwg; w++) g += part[(int64_t)w * part_stride + q - base];
  } else {
    g = gr[q];
  }
  Opt o;
  o.kind = s.optimizer;
  o.lr = s.lr; o.b1 = s.b1; o.b2 = s.b2; o.eps = s.eps;
  o.c1 = c1;
  o.c2 = c2;
  W[q] -= opt_delta(o, g, m ? m + q : (float *)nullptr, v ? v + q : (float *)nullptr);
}

// rows per workgroup (one: the training runs one block of bs rows, so a
// workgroup per row fills more of the chip; measured faster than two) and
// LDS bytes of the two recurrent kernels
size_t fwd_lds(const TfShape &s, int R) {
  const int h = s.gh, G = 3 * h;
  return ((size_t)2 * G * (s.sE + 1) + 2 * G * (h + 1) + (size_t)R * 2 * h + 2 * (size_t)R * 2 * G +
          (size_t)R * s.t * s.sE) * 4;
}
size_t bptt_lds(const TfShape &s, int R) {
  const int h = s.gh, G = 3 * h;
  return ((size_t)2 * G * (s.sE + 1) + 2 * G * (h + 1) + 4 * (size_t)R * 2 * G + (size_t)R * 2 * h +
          2 * (size_t)s.V * s.sE +
          (size_t)R * s.t * s.sE + (size_t)R * s.t * 2 * h) * 4;
}
int pick_rows(const TfShape &s, size_t (*lds)(const TfShape &, int)) {
  for (int R = 1; R >= 1; R >>= 1)
    if (lds(s, R) <= 150 * 1024) return R;
  return 0;
}

}  // namespace

// the seeded initialisation of the BiGRU shape: U(-a, a) from the same
// SplitMix64 draws as every model's initialiser, a = 1 for the embedding,
// 1/sqrt(gh) for the GRU tensors, 1/sqrt(2 gh) for the Dense layer,
// 1/sqrt(gd) for the head
hipError_t gru_init_params(const TfShape &s, uint64_t seed, float *out, hipStream_t st) {
  const int end[4] = {(int)s.s_wih[0][0], (int)s.s_dw, (int)s.s_lw, (int)s.sP};
  const double sc[4] = {1.0, 1.0 / std::sqrt((double)s.gh), 1.0 / std::sqrt(2.0 * s.gh), 1.0 / std::sqrt((double)s.gd)};
  return launch_init_scaled(seed, (int)s.sP, 4, end, sc, out, st);
}

bool gru_train_supported(const TfShape &s) {
  return s.sarch == 1 && s.gl == 1 && s.sE >= 1 && s.sE <= kEmax && s.gh >= 1 && s.gh <= kHmax &&
         pick_rows(s, fwd_lds) > 0 && pick_rows(s, bptt_lds) > 0;
}

uint64_t gru_train_floats(const TfShape &s, uint64_t &part_stride, int &nwg) {
  const int R = pick_rows(s, bptt_lds);
  nwg = R ? (s.bs + R - 1) / R : 0;
  part_stride = ((uint64_t)(s.s_dw - s.s_wih[0][0]) + 2ull * s.V * s.sE + 63) / 64 * 64;
  const uint64_t bs = (uint64_t)s.bs;
  return bs * s.t * 2 * s.gh      // seq
         + bs * s.gd * 2          // dn, du
         + bs * s.V               // logits / loss gradient
         + bs * 2 * s.gh          // dfeat
         + (uint64_t)s.sP         // dense gradients
         + part_stride * nwg      // partials
         + 64 * 8;                // alignment slack
}

hipError_t gru_train(const TfShape &s, const uint8_t *tok, uint64_t Lp, float *W, float *buf, float *adam_m,
                     float *adam_v, hipStream_t st) {
  if (!gru_train_supported(s)) return hipErrorInvalidValue;
  uint64_t ps;
  int nwg;
  gru_train_floats(s, ps, nwg);
  const int Rf = pick_rows(s, fwd_lds), Rb = pick_rows(s, bptt_lds);
  auto take = [&](uint64_t n) {
    float *p = buf;
    buf += (n + 63) / 64 * 64;
    return p;
  };
  const uint64_t bs = (uint64_t)s.bs;
  float *seq = take(bs * s.t * 2 * s.gh), *dn = take(bs * s.gd), *du = take(bs * s.gd), *lg = take(bs * s.V),
        *dfeat = take(bs * 2 * s.gh), *gr = take((uint64_t)s.sP), *part = take(ps * nwg);
  static bool lds_set = false;   // dynamic LDS beyond 64 KB needs the kernels' attribute once
  if (!lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&gru_fwd_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute(reinterpret_cast<const void *>(&gru_bptt_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    if (e != hipSuccess) return e;
    lds_set = true;
  }
  if (adam_m) {
    hipError_t e = hipMemsetAsync(adam_m, 0, sizeof(float) * s.sP, st);
    if (e == hipSuccess) e = hipMemsetAsync(adam_v, 0, sizeof(float) * s.sP, st);
    if (e != hipSuccess) return e;
  }
  const int threads = 6 * s.gh;
  const int gfwd = (s.bs + Rf - 1) / Rf;
  const unsigned nup = (unsigned)((s.sP + 255) / 256);
  const unsigned ngrad =
      (unsigned)(((int64_t)s.gd * s.V + s.V + 2ll * s.gh * s.gd + s.gd + (int64_t)s.bs * 2 * s.gh + 255) / 256);
  uint64_t tau = 0;
  for (uint64_t i = (uint64_t)s.t; i < Lp; i++) {
    tau++;
    // Adam's bias corrections in double, as the optimiser's definition
    const float c1 = (float)(1.0 - std::pow((double)s.b1, (double)tau));
    const float c2 = (float)(1.0 - std::pow((double)s.b2, (double)tau));
    hipLaunchKernelGGL(gru_fwd_kernel, dim3(gfwd), dim3(threads), fwd_lds(s, Rf), st, s, tok, Lp, (int)i, W, seq, dn,
                       lg, Rf);
    hipLaunchKernelGGL(gru_loss_kernel, dim3((s.bs + 255) / 256), dim3(256), 0, st, s, tok, Lp, (int)i, lg);
    hipLaunchKernelGGL(gru_du_kernel, dim3((unsigned)((s.bs * s.gd + 255) / 256)), dim3(256), 0, st, s, W, dn, lg,
                       du);
    hipLaunchKernelGGL(gru_dgrad_kernel, dim3(ngrad), dim3(256), 0, st, s, W, seq, dn, lg, du, gr, dfeat);
    hipLaunchKernelGGL(gru_bptt_kernel, dim3(nwg), dim3(threads), bptt_lds(s, Rb), st, s, tok, Lp, (int)i, W, seq,
                       dfeat, part, (int64_t)ps, Rb);
    hipLaunchKernelGGL(gru_update_kernel, dim3(nup), dim3(256), 0, st, s, W, gr, part, (int64_t)ps, nwg,
                       s.optimizer == 1 ? adam_m : nullptr, s.optimizer == 1 ? adam_v : nullptr, c1, c2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace pmklc
