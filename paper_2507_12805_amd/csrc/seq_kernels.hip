// Sequence-side kernels: the GPU (s,k)-mer encoder (Sec. 4.1, Fig. 3),
// input scan with N-run extraction, the inverse (tokens -> ASCII) used by
// decompression (Sec. 2), and stream compaction.
//
// Bases map A0 C1 G2 T3 (Sec. 4.1).  For an ASCII byte c in {A,C,G,T} the
// 2-bit code is ((c >> 1) ^ (c >> 2)) & 3 (A 0x41 -> 0, C 0x43 -> 1,
// G 0x47 -> 2, T 0x54 -> 3).  A token is e_j = sum_m 4^(k-1-m) b_{js+m},
// i.e. the window's codes read as a base-4 number, first base most
// significant.
#include "pmklc_internal.h"

namespace pmklc {

namespace {

__device__ __forceinline__ uint32_t code_of(uint32_t c) { return ((c >> 1) ^ (c >> 2)) & 3u; }
__device__ __forceinline__ bool is_acgt(uint32_t c) { return c == 'A' || c == 'C' || c == 'G' || c == 'T'; }

constexpr int kTokPerThread = 4;   // per-block tokeniser
constexpr int kTokPerWG = 256 * kTokPerThread;

}  // namespace

// ---------------------------------------------------------------- GskE
// Direct ASCII -> tokens (no N allowed), one instance per (S, K).  A
// workgroup owns 4096 tokens: it stages their bytes in LDS with 16-byte
// loads in a 16-byte aligned frame (bytes outside [0, n) are never read; a
// word that crosses either end is read byte by byte), validates them, then
// every thread builds 16 tokens from the dwords of its window and writes them
// with one 16-byte store when the destination run is whole and aligned.
// Validation of a whole word: the 2-bit codes of its 4 bytes mapped back to
// ASCII by one byte permutation ('A' 'C' 'G' 'T' at selectors 0..3) must give
// the word again.
constexpr int kSkTokPerThread = 16;
constexpr int kSkTokPerWG = 256 * kSkTokPerThread;
constexpr int kSkBuf = kSkTokPerWG * 4 + 32;   // s <= 4, plus the k - s tail and the frame offset

__device__ __forceinline__ uint32_t codes4(uint32_t w) { return ((w >> 1) ^ (w >> 2)) & 0x03030303u; }
__device__ __forceinline__ bool acgt4(uint32_t w) { return __builtin_amdgcn_perm(0u, 0x54474341u, codes4(w)) == w; }

template <int S, int K>
__global__ __launch_bounds__(256) void skmer_direct_kernel(const uint8_t *__restrict__ in, uint64_t n,
                                                           uint8_t *__restrict__ tok, uint64_t l, int *err) {
  __shared__ __align__(16) uint8_t buf[kSkBuf + 16];
  const uint64_t j0 = (uint64_t)blockIdx.x * kSkTokPerWG;
  const uint64_t b0 = j0 * (uint64_t)S;
  uint64_t b1 = (j0 + kSkTokPerWG) * (uint64_t)S + (uint64_t)(K - S);
  if (b1 > n || blockIdx.x == gridDim.x - 1) b1 = n;
  // frame: buf[i] holds input byte a0 + i, a0 = b0 rounded down to 16 bytes
  // of the input address; bytes of the frame outside [b0, b1) are not used
  const int pre = (int)(reinterpret_cast<uintptr_t>(in + b0) & 15u);
  const int64_t a0 = (int64_t)b0 - pre;   // may be < 0 only when pre > b0
  const int span = pre + (int)(b1 - b0);
  const int nq = (span + 15) >> 4;
  int bad = 0;
  for (int w = threadIdx.x; w < nq; w += 256) {
    const int64_t addr = a0 + 16 * (int64_t)w;
    uint32_t v[4];
    const bool whole = addr >= 0 && (uint64_t)addr + 16 <= n;
    if (whole) {
      const uint4 x = *reinterpret_cast<const uint4 *>(in + addr);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
      for (int q = 0; q < 4; q++) {
        v[q] = 0;
        for (int c = 0; c < 4; c++) {
          const int64_t ad = addr + 4 * q + c;
          if (ad >= 0 && (uint64_t)ad < n) v[q] |= (uint32_t)in[ad] << (8 * c);
        }
      }
    }
    *reinterpret_cast<uint4 *>(buf + 16 * w) = make_uint4(v[0], v[1], v[2], v[3]);
    if (whole && 16 * w >= pre && 16 * w + 16 <= span) {
#pragma unroll
      for (int q = 0; q < 4; q++) bad |= !acgt4(v[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 16; q++) {
        const int pos = 16 * w + q;   // frame index
        if (pos >= pre && pos < span) bad |= !is_acgt((v[q >> 2] >> (8 * (q & 3))) & 0xFFu);
      }
    }
  }
  if (bad) atomicOr(err, 1);
  __syncthreads();
  // this thread's 16 tokens: bytes [first, first + 15 S + K) of the frame
  const int t16 = threadIdx.x * kSkTokPerThread;
  const uint64_t jt = j0 + (uint64_t)t16;
  if (jt >= l) return;
  const int cnt = (int)min((uint64_t)kSkTokPerThread, l - jt);
  const int first = pre + t16 * S;
  const int fw = first >> 2, sh0 = first & 3;
  // dwords covering any sh0 (at least 6 for S = 1: its realignment reads one past the last needed)
  constexpr int NW0 = ((kSkTokPerThread - 1) * S + K + 3 + 3) / 4;
  constexpr int NW = (S == 1 && NW0 < 6) ? 6 : NW0;
  uint32_t cw[NW];
  const uint32_t *bw = reinterpret_cast<const uint32_t *>(buf);
#pragma unroll
  for (int q = 0; q < NW; q++) cw[q] = codes4(bw[fw + q]);
  auto code_at = [&](int i) {   // i relative to `first`
    const int bi = sh0 + i;
    return (cw[bi >> 2] >> (8 * (bi & 3))) & 3u;
  };
  uint32_t packed[4] = {0u, 0u, 0u, 0u};
  if constexpr (S == 1) {
    // consecutive tokens: realign the code bytes to the first base, then
    // the 4 tokens of output dword i are sum_m (codes i*4 + m .. + 3) << 2 (K - 1 - m),
    // each byte's token staying below 256 (no carries between bytes)
    uint32_t al[5];
#pragma unroll
    for (int q = 0; q < 5; q++) al[q] = __builtin_amdgcn_alignbyte(cw[q + 1], cw[q], (uint32_t)sh0);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      uint32_t v = 0;
#pragma unroll
      for (int m = 0; m < K; m++) v |= __builtin_amdgcn_alignbyte(al[i + 1], al[i], (uint32_t)m) << (2 * (K - 1 - m));
      packed[i] = v;
    }
  } else {
#pragma unroll
    for (int q = 0; q < kSkTokPerThread; q++) {
      uint32_t e = 0;
#pragma unroll
      for (int m = 0; m < K; m++) e = (e << 2) | code_at(q * S + m);
      packed[q >> 2] |= e << (8 * (q & 3));
    }
  }
  if (cnt == kSkTokPerThread && ((reinterpret_cast<uintptr_t>(tok + jt) & 15u) == 0)) {
    *reinterpret_cast<uint4 *>(tok + jt) = make_uint4(packed[0], packed[1], packed[2], packed[3]);
  } else {
    for (int q = 0; q < cnt; q++) tok[jt + q] = (uint8_t)(packed[q >> 2] >> (8 * (q & 3)));
  }
}

template <int S, int K>
hipError_t launch_sk(const uint8_t *in, uint64_t n, uint8_t *tok, uint64_t l, int *err, hipStream_t st) {
  const uint64_t grid = l ? (l + kSkTokPerWG - 1) / kSkTokPerWG : 1;
  hipLaunchKernelGGL((skmer_direct_kernel<S, K>), dim3((unsigned)grid), dim3(256), 0, st, in, n, tok, l, err);
  return hipGetLastError();
}

hipError_t launch_skmer_direct(const uint8_t *in, uint64_t n, int s, int k, uint8_t *tok, uint64_t l, int *err,
                               hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (k * 8 + s) {
    case 1 * 8 + 1: return launch_sk<1, 1>(in, n, tok, l, err, st);
    case 2 * 8 + 1: return launch_sk<1, 2>(in, n, tok, l, err, st);
    case 2 * 8 + 2: return launch_sk<2, 2>(in, n, tok, l, err, st);
    case 3 * 8 + 1: return launch_sk<1, 3>(in, n, tok, l, err, st);
    case 3 * 8 + 2: return launch_sk<2, 3>(in, n, tok, l, err, st);
    case 3 * 8 + 3: return launch_sk<3, 3>(in, n, tok, l, err, st);
    case 4 * 8 + 1: return launch_sk<1, 4>(in, n, tok, l, err, st);
    case 4 * 8 + 2: return launch_sk<2, 4>(in, n, tok, l, err, st);
    case 4 * 8 + 3: return launch_sk<3, 4>(in, n, tok, l, err, st);
    case 4 * 8 + 4: return launch_sk<4, 4>(in, n, tok, l, err, st);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------- input scan
// One workgroup per 4096-byte chunk of a block (chunks never straddle
// blocks).  Counts N bytes, N-run starts and bytes outside {A,C,G,T,N}.
__global__ __launch_bounds__(256) void scan_kernel(const uint8_t *__restrict__ in, const SeqBlock *blk,
                                                   const uint64_t *chunk_block, ChunkStat *stats) {
  __shared__ uint32_t sN, sR, sB;
  const uint64_t c = blockIdx.x;
  const SeqBlock b = blk[chunk_block[c]];
  const uint64_t cstart = (c - b.chunk0) * kScanChunk;
  const uint64_t cend = min(cstart + kScanChunk, b.raw_len);
  if (threadIdx.x == 0) { sN = 0; sR = 0; sB = 0; }
  __syncthreads();
  uint32_t nN = 0, nR = 0, bad = 0;
  for (uint64_t p = cstart + threadIdx.x; p < cend; p += 256) {
    uint32_t ch = in[b.raw_off + p];
    bool isN = ch == 'N';
    nN += isN;
    bad |= !(isN || is_acgt(ch));
    if (isN && (p == 0 || in[b.raw_off + p - 1] != 'N')) nR++;
  }
  if (nN) atomicAdd(&sN, nN);
  if (nR) atomicAdd(&sR, nR);
  if (bad) atomicOr(&sB, 1u);
  __syncthreads();
  if (threadIdx.x == 0) stats[c] = ChunkStat{sN, sR, sB, 0};
}

hipError_t launch_scan(const uint8_t *in, const SeqBlock *blk, const uint64_t *chunk_block, uint64_t n_chunks,
                       ChunkStat *stats, hipStream_t st) {
  if (n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_kernel, dim3((unsigned)n_chunks), dim3(256), 0, st, in, blk, chunk_block, stats);
  return hipGetLastError();
}

// Writes the runs (block-relative raw start, length) of chunks that have
// any.  Thread q of the chunk takes bytes [16q, 16q+16); a workgroup scan
// of the per-thread start counts keeps the runs in ascending order.  The
// length is found from the matching run end (N followed by non-N or the
// block end), counted the same way, so no thread walks a long run.
__global__ __launch_bounds__(256) void runs_kernel(const uint8_t *__restrict__ in, const SeqBlock *blk,
                                                   const uint64_t *chunk_block, const ChunkStat *stats,
                                                   const uint64_t *chunk_run0, uint32_t *run_start,
                                                   uint32_t *run_len) {
  __shared__ uint32_t scan_s[256], scan_e[256];
  const uint64_t c = blockIdx.x;
  if (stats[c].n_N == 0) return;
  const SeqBlock b = blk[chunk_block[c]];
  const uint64_t cstart = (c - b.chunk0) * kScanChunk;
  const uint64_t cend = min(cstart + kScanChunk, b.raw_len);
  const uint64_t p0 = cstart + 16ull * threadIdx.x, p1 = min(p0 + 16ull, cend);
  uint32_t ns = 0, ne = 0;
  for (uint64_t p = p0; p < p1; p++) {
    bool isN = in[b.raw_off + p] == 'N';
    if (isN && (p == 0 || in[b.raw_off + p - 1] != 'N')) ns++;
    if (isN && (p + 1 == b.raw_len || in[b.raw_off + p + 1] != 'N')) ne++;
  }
  scan_s[threadIdx.x] = ns;
  scan_e[threadIdx.x] = ne;
  __syncthreads();
  // Hillis-Steele inclusive scans
  for (int o = 1; o < 256; o <<= 1) {
    uint32_t vs = threadIdx.x >= (unsigned)o ? scan_s[threadIdx.x - o] : 0;
    uint32_t ve = threadIdx.x >= (unsigned)o ? scan_e[threadIdx.x - o] : 0;
    __syncthreads();
    scan_s[threadIdx.x] += vs;
    scan_e[threadIdx.x] += ve;
    __syncthreads();
  }
  // runs starting in this chunk get global indices chunk_run0[c] + ...;
  // run ends are paired with their start: the number of run ends before a
  // position equals the number of starts before it minus (1 if inside a run)
  uint64_t rs = chunk_run0[c] + scan_s[threadIdx.x] - ns;
  // index of the first run that ends in this thread's range: all runs that
  // started before this chunk and are still open end here or later
  uint64_t open_before = 0;
  if (cstart > 0 && in[b.raw_off + cstart - 1] == 'N') open_before = 1;
  uint64_t re = chunk_run0[c] - open_before + scan_e[threadIdx.x] - ne;
  for (uint64_t p = p0; p < p1; p++) {
    bool isN = in[b.raw_off + p] == 'N';
    if (isN && (p == 0 || in[b.raw_off + p - 1] != 'N')) run_start[b.run0 + rs++] = (uint32_t)p;
    if (isN && (p + 1 == b.raw_len || in[b.raw_off + p + 1] != 'N')) run_len[b.run0 + re++] = (uint32_t)(p + 1);
  }
}

hipError_t launch_runs(const uint8_t *in, const SeqBlock *blk, const uint64_t *chunk_block, uint64_t n_chunks,
                       const ChunkStat *stats, const uint64_t *chunk_run0, uint32_t *run_start,
                       uint32_t *run_len, hipStream_t st) {
  if (n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(runs_kernel, dim3((unsigned)n_chunks), dim3(256), 0, st, in, blk, chunk_block, stats,
                     chunk_run0, run_start, run_len);
  return hipGetLastError();
}

// Per block, in run order: run_len holds run ends on entry and lengths on
// exit; run_sp[r] = start_r - (N bases before run r) is the stripped
// position before which run r sits; run_cum[r] = N bases of runs 0..r.
__global__ void run_sp_kernel(const SeqBlock *blk, int n_blocks, const uint32_t *run_start, uint32_t *run_len,
                              uint32_t *run_sp, uint32_t *run_cum) {
  int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= n_blocks) return;
  const SeqBlock b = blk[bi];
  uint32_t cum = 0;
  for (uint64_t r = 0; r < b.n_runs; r++) {
    uint64_t g = b.run0 + r;
    uint32_t len = run_len[g] - run_start[g];
    run_len[g] = len;
    run_sp[g] = run_start[g] - cum;
    cum += len;
    run_cum[g] = cum;
  }
}

hipError_t launch_run_sp(const SeqBlock *blk, int n_blocks, const uint32_t *run_start, uint32_t *run_len,
                         uint32_t *run_sp, uint32_t *run_cum, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(run_sp_kernel, dim3((n_blocks + 63) / 64), dim3(64), 0, st, blk, n_blocks, run_start, run_len,
                     run_sp, run_cum);
  return hipGetLastError();
}

namespace {
// Stripped position q of a block sits at raw position q + cum[r-1], where r
// is the number of runs whose stripped position is <= q (the runs that
// come before it).
struct RunMap {
  const uint32_t *sp, *cum;
  uint64_t n;
  __device__ uint64_t count_le(uint64_t q) const {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
      uint64_t m = (lo + hi) >> 1;
      if ((uint64_t)sp[m] <= q) lo = m + 1; else hi = m;
    }
    return lo;
  }
  __device__ uint64_t raw(uint64_t q, uint64_t &r) const {   // r: running count, only grows with q
    while (r < n && (uint64_t)sp[r] <= q) r++;
    return q + (r ? (uint64_t)cum[r - 1] : 0);
  }
};
}  // namespace

// Per block tokenisation of the N-stripped bases (Sec. 4.1).  Grid:
// (token chunk, block); each thread builds 4 tokens.
__global__ __launch_bounds__(256) void tokenise_kernel(const uint8_t *__restrict__ in, const SeqBlock *blk,
                                                       const uint32_t *run_sp, const uint32_t *run_cum, int s, int k,
                                                       uint8_t *__restrict__ tok) {
  const SeqBlock b = blk[blockIdx.y];
  const uint64_t jt = (uint64_t)blockIdx.x * kTokPerWG + (uint64_t)threadIdx.x * kTokPerThread;
  if (jt >= b.l) return;
  const RunMap rm{run_sp + b.run0, run_cum + b.run0, b.n_runs};
  const uint8_t *raw = in + b.raw_off;
  uint64_t r0 = b.n_runs ? rm.count_le(jt * (uint64_t)s) : 0;
  for (int t = 0; t < kTokPerThread; t++) {
    const uint64_t j = jt + (uint64_t)t;
    if (j >= b.l) break;
    const uint64_t q0 = j * (uint64_t)s;
    rm.raw(q0, r0);
    uint64_t r = r0;
    uint32_t e = 0;
    for (int m = 0; m < k; m++) e = (e << 2) | code_of(raw[rm.raw(q0 + (uint64_t)m, r)]);
    tok[b.tok_off + j] = (uint8_t)e;
  }
}

hipError_t launch_tokenise(const uint8_t *in, const SeqBlock *blk, int n_blocks, uint64_t max_l,
                           const uint32_t *run_sp, const uint32_t *run_cum, int s, int k, uint8_t *tok,
                           hipStream_t st) {
  if (n_blocks == 0 || max_l == 0) return hipSuccess;
  uint64_t gx = (max_l + kTokPerWG - 1) / kTokPerWG;
  hipLaunchKernelGGL(tokenise_kernel, dim3((unsigned)gx, (unsigned)n_blocks), dim3(256), 0, st, in, blk, run_sp,
                     run_cum, s, k, tok);
  return hipGetLastError();
}

// Per block: the tail bases the last window leaves over (2-bit codes) and
// the remainder tokens that do not fill a step, copied to extras[ex_off..]
// (tail codes first).  One thread per block.
__global__ void extras_kernel(const uint8_t *__restrict__ in, const SeqBlock *blk, int n_blocks,
                              const uint32_t *run_sp, const uint32_t *run_cum, int bs, const uint8_t *tok,
                              uint8_t *extras) {
  int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= n_blocks) return;
  const SeqBlock b = blk[bi];
  const RunMap rm{run_sp + b.run0, run_cum + b.run0, b.n_runs};
  uint8_t *ex = extras + b.ex_off;
  uint64_t r = 0;
  uint64_t o = 0;
  for (uint64_t q = b.tail_off; q < b.nb; q++) ex[o++] = (uint8_t)code_of(in[b.raw_off + rm.raw(q, r)]);
  for (uint64_t j = b.L * (uint64_t)bs; j < b.l; j++) ex[o++] = tok[b.tok_off + j];
}

hipError_t launch_extras(const uint8_t *in, const SeqBlock *blk, int n_blocks, const uint32_t *run_sp,
                         const uint32_t *run_cum, int s, int k, int bs, const uint8_t *tok, uint8_t *extras,
                         hipStream_t st) {
  (void)s; (void)k;
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(extras_kernel, dim3((n_blocks + 63) / 64), dim3(64), 0, st, in, blk, n_blocks, run_sp, run_cum,
                     bs, tok, extras);
  return hipGetLastError();
}

// ------------------------------------------------------------- inverse
// Decompression's last step (Sec. 2): tokens -> bases -> ASCII with the N
// runs put back.  Stripped base q comes from token 0 (q < k, digit q) or
// from token j = (q-k)/s + 1 (digit k-s + (q-k) % s), the digit read as
// (e >> 2(k-1-m)) & 3; bases past the last window are the tail codes.
// Tokens at or past bs*L are the remainder tokens kept in extras.
__global__ __launch_bounds__(256) void detok_kernel(const SeqBlock *blk, const uint32_t *run_start,
                                                    const uint32_t *run_len, const uint32_t *run_cum, int s, int k,
                                                    int bs, const uint8_t *__restrict__ tok,
                                                    const uint8_t *__restrict__ extras, uint8_t *__restrict__ out) {
  const SeqBlock b = blk[blockIdx.y];
  const uint64_t r0 = (uint64_t)blockIdx.x * 4096 + (uint64_t)threadIdx.x * 16;
  if (r0 >= b.raw_len) return;
  const uint32_t *rs = run_start + b.run0, *rl = run_len + b.run0, *rc = run_cum + b.run0;
  // #runs starting at or before r0
  uint64_t lo = 0, hi = b.n_runs;
  while (lo < hi) {
    uint64_t m = (lo + hi) >> 1;
    if ((uint64_t)rs[m] <= r0) lo = m + 1; else hi = m;
  }
  uint64_t r = lo;
  const uint64_t covered = b.tail_off;
  const uint64_t nseg = b.L * (uint64_t)bs;
  const uint8_t *ex = extras + b.ex_off;
  const uint64_t ntail = b.nb - b.tail_off;
  const char letter[4] = {'A', 'C', 'G', 'T'};
  uint8_t o16[16];
  int cnt = 0;
  for (uint64_t p = r0; p < r0 + 16 && p < b.raw_len; p++, cnt++) {
    while (r < b.n_runs && (uint64_t)rs[r] <= p) r++;
    if (r > 0 && p < (uint64_t)rs[r - 1] + rl[r - 1]) { o16[cnt] = 'N'; continue; }
    uint64_t q = p - (r ? (uint64_t)rc[r - 1] : 0);
    uint32_t code;
    if (q < covered) {
      uint64_t j;
      int m;
      if (q < (uint64_t)k) { j = 0; m = (int)q; }
      else { j = (q - (uint64_t)k) / (uint64_t)s + 1; m = k - s + (int)((q - (uint64_t)k) % (uint64_t)s); }
      uint32_t e = j < nseg ? tok[b.tok_off + j] : ex[ntail + (j - nseg)];
      code = (e >> (2 * (k - 1 - m))) & 3u;
    } else {
      code = ex[q - covered];
    }
    o16[cnt] = (uint8_t)letter[code];
  }
  for (int q = 0; q < cnt; q++) out[b.raw_off + r0 + q] = o16[q];
}

hipError_t launch_detok(const SeqBlock *blk, int n_blocks, uint64_t max_raw, const uint32_t *run_start,
                        const uint32_t *run_len, const uint32_t *run_cum, int s, int k, int bs, const uint8_t *tok,
                        const uint8_t *extras, uint8_t *out, hipStream_t st) {
  if (n_blocks == 0 || max_raw == 0) return hipSuccess;
  uint64_t gx = (max_raw + 4095) / 4096;
  hipLaunchKernelGGL(detok_kernel, dim3((unsigned)gx, (unsigned)n_blocks), dim3(256), 0, st, blk, run_start, run_len,
                     run_cum, s, k, bs, tok, extras, out);
  return hipGetLastError();
}

// ------------------------------------------------------- stream copies
// One workgroup per segment stream: slot words (stored in stream byte
// order) -> packed bytes at dst + seg_dst[i].
__global__ __launch_bounds__(256) void gather_streams_kernel(const uint32_t *slots, const uint64_t *seg_src_word,
                                                             const uint64_t *seg_dst, const uint32_t *seg_bytes,
                                                             uint8_t *dst) {
  const uint64_t i = blockIdx.x;
  const uint8_t *src = reinterpret_cast<const uint8_t *>(slots + seg_src_word[i]);
  uint8_t *d = dst + seg_dst[i];
  const uint32_t n = seg_bytes[i];
  for (uint32_t q = threadIdx.x; q < n; q += 256) d[q] = src[q];
}

hipError_t launch_gather_streams(const uint32_t *slots, const uint64_t *seg_src_word, const uint64_t *seg_dst,
                                 const uint32_t *seg_bytes, uint64_t n_seg, uint8_t *dst, hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_streams_kernel, dim3((unsigned)n_seg), dim3(256), 0, st, slots, seg_src_word, seg_dst,
                     seg_bytes, dst);
  return hipGetLastError();
}

// Inverse: packed bytes -> word-aligned slots, zero-padded to seg_words.
__global__ __launch_bounds__(256) void scatter_streams_kernel(const uint8_t *src, const uint64_t *seg_src,
                                                              const uint64_t *seg_dst_word, const uint32_t *seg_bytes,
                                                              const uint32_t *seg_words, uint32_t *slots) {
  const uint64_t i = blockIdx.x;
  const uint8_t *s8 = src + seg_src[i];
  uint8_t *d = reinterpret_cast<uint8_t *>(slots + seg_dst_word[i]);
  const uint32_t n = seg_bytes[i], nw = seg_words[i];
  for (uint32_t q = threadIdx.x; q < 4 * nw; q += 256) d[q] = q < n ? s8[q] : 0;
}

hipError_t launch_scatter_streams(const uint8_t *src, const uint64_t *seg_src, const uint64_t *seg_dst_word,
                                  const uint32_t *seg_bytes, const uint32_t *seg_words, uint64_t n_seg,
                                  uint32_t *slots, hipStream_t st) {
  if (n_seg == 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_streams_kernel, dim3((unsigned)n_seg), dim3(256), 0, st, src, seg_src, seg_dst_word,
                     seg_bytes, seg_words, slots);
  return hipGetLastError();
}

}  // namespace pmklc
