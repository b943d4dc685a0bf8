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

// the block whose tiles (first tile blk[b].*F) contain `tile`: the last
// block whose first tile is <= tile (blocks with no tiles share their
// first tile with the next block)
template <uint64_t SeqBlock::*F>
__device__ __forceinline__ int block_of_tile(const SeqBlock *blk, int n, uint64_t tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int m = (lo + hi + 1) >> 1;
    if (blk[m].*F <= tile) lo = m; else hi = m - 1;
  }
  return lo;
}

}  // namespace

void assign_tiles_impl(SeqBlock *sb, int n_blocks, uint64_t &n_sk, uint64_t &n_tk, uint64_t &n_raw, int sk_tile) {
  n_sk = n_tk = n_raw = 0;
  for (int b = 0; b < n_blocks; b++) {
    SeqBlock &q = sb[b];
    q.t_sk = n_sk;
    q.t_tk = n_tk;
    q.t_raw = n_raw;
    if (q.n_runs == 0) n_sk += (q.l + sk_tile - 1) / sk_tile;
    else n_tk += (q.l + kTokPerWG - 1) / kTokPerWG;
    n_raw += (q.raw_len + 4095) / 4096;
  }
}

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

// One workgroup's tile (4096 tokens starting at token 4096 * tile) of the
// tokens of bases in[0, n); `last`: the sequence's last tile.  VALIDATE:
// flag bytes outside {A,C,G,T} in err (the per-block tokeniser's input was
// validated by the scan already).
template <int S, int K, bool VALIDATE>
__device__ __forceinline__ void skmer_tile(const uint8_t *__restrict__ in, uint64_t n, uint8_t *__restrict__ tok,
                                           uint64_t l, int *err, uint64_t tile, bool last, uint8_t *buf) {
  const uint64_t j0 = tile * kSkTokPerWG;
  const uint64_t b0 = j0 * (uint64_t)S;
  uint64_t b1 = (j0 + kSkTokPerWG) * (uint64_t)S + (uint64_t)(K - S);
  if (b1 > n || last) b1 = n;
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
    if constexpr (!VALIDATE) continue;
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
  if (VALIDATE && bad) atomicOr(err, 1);
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
__global__ __launch_bounds__(256) void skmer_direct_kernel(const uint8_t *__restrict__ in, uint64_t n,
                                                           uint8_t *__restrict__ tok, uint64_t l, int *err) {
  __shared__ __align__(16) uint8_t buf[kSkBuf + 16];
  skmer_tile<S, K, true>(in, n, tok, l, err, blockIdx.x, blockIdx.x == gridDim.x - 1, buf);
}

// The same over the blocks of a compress call (grid: tile, block): a block
// without N runs is tokenised straight from its raw bytes, already
// validated by the scan; blocks with N runs are left to tokenise_kernel.
template <int S, int K>
__global__ __launch_bounds__(256) void skmer_blocks_kernel(const uint8_t *__restrict__ in, const SeqBlock *blk,
                                                           int n_blocks, uint8_t *__restrict__ tok) {
  __shared__ __align__(16) uint8_t buf[kSkBuf + 16];
  const int bi = block_of_tile<&SeqBlock::t_sk>(blk, n_blocks, blockIdx.x);
  const SeqBlock b = blk[bi];
  const uint64_t tile = blockIdx.x - b.t_sk, tiles = (b.l + kSkTokPerWG - 1) / kSkTokPerWG;
  skmer_tile<S, K, false>(in + b.raw_off, b.nb, tok + b.tok_off, b.l, nullptr, tile, tile + 1 == tiles, buf);
}

void assign_tiles(SeqBlock *sb, int n_blocks, uint64_t &n_sk, uint64_t &n_tk, uint64_t &n_raw) {
  assign_tiles_impl(sb, n_blocks, n_sk, n_tk, n_raw, kSkTokPerWG);
}

template <int S, int K>
hipError_t launch_sk(const uint8_t *in, uint64_t n, uint8_t *tok, uint64_t l, int *err, hipStream_t st) {
  const uint64_t grid = l ? (l + kSkTokPerWG - 1) / kSkTokPerWG : 1;
  hipLaunchKernelGGL((skmer_direct_kernel<S, K>), dim3((unsigned)grid), dim3(256), 0, st, in, n, tok, l, err);
  return hipGetLastError();
}

template <int S, int K>
hipError_t launch_skb(const uint8_t *in, const SeqBlock *blk, int n_blocks, uint64_t n_sk, uint8_t *tok,
                      hipStream_t st) {
  hipLaunchKernelGGL((skmer_blocks_kernel<S, K>), dim3((unsigned)n_sk), dim3(256), 0, st, in, blk, n_blocks, tok);
  return hipGetLastError();
}

hipError_t launch_skmer_blocks(const uint8_t *in, const SeqBlock *blk, int n_blocks, uint64_t n_sk, int s, int k,
                               uint8_t *tok, hipStream_t st) {
  if (n_blocks == 0 || n_sk == 0) return hipSuccess;
  switch (k * 8 + s) {
    case 1 * 8 + 1: return launch_skb<1, 1>(in, blk, n_blocks, n_sk, tok, st);
    case 2 * 8 + 1: return launch_skb<1, 2>(in, blk, n_blocks, n_sk, tok, st);
    case 2 * 8 + 2: return launch_skb<2, 2>(in, blk, n_blocks, n_sk, tok, st);
    case 3 * 8 + 1: return launch_skb<1, 3>(in, blk, n_blocks, n_sk, tok, st);
    case 3 * 8 + 2: return launch_skb<2, 3>(in, blk, n_blocks, n_sk, tok, st);
    case 3 * 8 + 3: return launch_skb<3, 3>(in, blk, n_blocks, n_sk, tok, st);
    case 4 * 8 + 1: return launch_skb<1, 4>(in, blk, n_blocks, n_sk, tok, st);
    case 4 * 8 + 2: return launch_skb<2, 4>(in, blk, n_blocks, n_sk, tok, st);
    case 4 * 8 + 3: return launch_skb<3, 4>(in, blk, n_blocks, n_sk, tok, st);
    case 4 * 8 + 4: return launch_skb<4, 4>(in, blk, n_blocks, n_sk, tok, st);
    default: return hipErrorInvalidValue;
  }
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
// Four 4096-byte chunks per workgroup, one after the other (chunks never
// straddle blocks).  Counts N bytes, N-run starts and bytes outside
// {A,C,G,T,N} per chunk.  A chunk is read as 16-byte words of a 16-byte aligned frame (a word
// that crosses either end of the chunk has its outside bytes masked off);
// each dword is classified four bytes at a time: byte == 'N' by the exact
// zero-byte test on w ^ 'NNNN' (bit 7 of each byte), ACGT by the
// code-permutation test, run starts as N bytes whose previous byte is not N.
__device__ __forceinline__ uint32_t n_bits4(uint32_t w) {   // 0x80 in each byte equal to 'N'
  const uint32_t y = w ^ 0x4E4E4E4Eu;
  return ~(((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y | 0x7F7F7F7Fu) & 0x80808080u;
}
constexpr int kScanChunksPerWG = 4;
__global__ __launch_bounds__(256) void scan_kernel(const uint8_t *__restrict__ in, const SeqBlock *blk,
                                                   const uint64_t *chunk_block, uint64_t n_chunks, ChunkStat *stats) {
  __shared__ uint32_t red[kScanChunksPerWG][3];   // per chunk: N bytes, run starts, bad bytes
  if (threadIdx.x < kScanChunksPerWG * 3) (&red[0][0])[threadIdx.x] = 0;
  __syncthreads();
  // every chunk's word for this thread first (the loads in flight
  // together), then the counting; a chunk has at most 257 words in its
  // frame, so thread 0 may own one more per chunk
  uint4 wv[kScanChunksPerWG];
  uint32_t prevbyte[kScanChunksPerWG];
  const SeqBlock *bp[kScanChunksPerWG];
  for (int cc = 0; cc < kScanChunksPerWG; cc++) {
    const uint64_t c = (uint64_t)blockIdx.x * kScanChunksPerWG + cc;
    wv[cc] = make_uint4(0u, 0u, 0u, 0u);
    prevbyte[cc] = 0;
    if (c >= n_chunks) continue;
    const SeqBlock &b = blk[chunk_block[c]];
    bp[cc] = &b;
    const uint64_t cstart = (c - b.chunk0) * kScanChunk;
    const uint64_t cend = min(cstart + kScanChunk, b.raw_len);
    const uint8_t *base = in + b.raw_off;
    const int pre = (int)(reinterpret_cast<uintptr_t>(base + cstart) & 15u);
    const int span = pre + (int)(cend - cstart);
    const int f0 = 16 * (int)threadIdx.x;
    if (f0 >= pre && f0 + 16 <= span) wv[cc] = *reinterpret_cast<const uint4 *>(base + cstart - pre + f0);
    const int64_t p0 = (int64_t)cstart - pre + f0;
    if (p0 >= 1 && f0 < span) prevbyte[cc] = base[p0 - 1];
  }
  for (int cc = 0; cc < kScanChunksPerWG; cc++) {
  const uint64_t c = (uint64_t)blockIdx.x * kScanChunksPerWG + cc;
  if (c >= n_chunks) break;
  const SeqBlock b = *bp[cc];
  const uint64_t cstart = (c - b.chunk0) * kScanChunk;
  const uint64_t cend = min(cstart + kScanChunk, b.raw_len);
  const uint8_t *base = in + b.raw_off;
  const int pre = (int)(reinterpret_cast<uintptr_t>(base + cstart) & 15u);
  const int span = pre + (int)(cend - cstart);          // frame bytes [pre, span) are the chunk
  const int nq = (span + 15) >> 4;
  const uint8_t *frame = base + cstart - pre;           // 16-byte aligned
  // bytes loaded: the chunk and the one before it (the first byte's
  // predecessor), block positions [lo, cend)
  const int flo = cstart > 0 ? pre - 1 : pre;
  uint32_t nN = 0, nR = 0, bad = 0;
  for (int q = threadIdx.x; q < nq; q += 256) {
    const int f0 = 16 * q;
    const bool whole = f0 >= pre && f0 + 16 <= span;
    uint32_t v[4];
    if (whole && q == (int)threadIdx.x) {
      v[0] = wv[cc].x; v[1] = wv[cc].y; v[2] = wv[cc].z; v[3] = wv[cc].w;
    } else if (whole) {
      const uint4 x = *reinterpret_cast<const uint4 *>(frame + f0);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    } else {
#pragma unroll
      for (int d = 0; d < 4; d++) {
        v[d] = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int f = f0 + 4 * d + e;
          if (f >= flo && f < span) v[d] |= (uint32_t)frame[f] << (8 * e);
        }
      }
    }
    // N bit of the byte before this word (block position p0 - 1)
    const int64_t p0 = (int64_t)cstart - pre + f0;
    uint32_t prevN;
    if (q == (int)threadIdx.x) prevN = prevbyte[cc] == 'N' ? 0x80u : 0u;
    else prevN = (p0 >= 1 && base[p0 - 1] == 'N') ? 0x80u : 0u;
#pragma unroll
    for (int d = 0; d < 4; d++) {
      uint32_t inb = 0x80808080u;   // in-chunk bytes (bit 7 of each)
      if (!whole) {
        inb = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const int f = f0 + 4 * d + e;
          if (f >= pre && f < span) inb |= 0x80u << (8 * e);
        }
      }
      const uint32_t nbu = n_bits4(v[d]);               // N bits of the loaded bytes
      const uint32_t prevb = (nbu << 8) | prevN;        // each byte's predecessor's N bit
      const uint32_t nb = nbu & inb;
      nN += __popc(nb);
      nR += __popc(nb & ~prevb);
      prevN = (nbu >> 24) & 0x80u;
      if (!(inb == 0x80808080u && acgt4(v[d]))) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
          const uint32_t ch = (v[d] >> (8 * e)) & 0xFFu;
          if (((inb >> (8 * e)) & 0x80u) && !(ch == 'N' || is_acgt(ch))) bad = 1;
        }
      }
    }
  }
  // workgroup sums by LDS atomics from the threads that saw anything
  // (integer sums: the order does not matter); most DNA has no N at all
  if (nN) atomicAdd(&red[cc][0], nN);
  if (nR) atomicAdd(&red[cc][1], nR);
  if (bad) atomicOr(&red[cc][2], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kScanChunksPerWG) {
    const uint64_t c = (uint64_t)blockIdx.x * kScanChunksPerWG + threadIdx.x;
    if (c < n_chunks) stats[c] = ChunkStat{red[threadIdx.x][0], red[threadIdx.x][1], red[threadIdx.x][2], 0};
  }
}

hipError_t launch_scan(const uint8_t *in, const SeqBlock *blk, const uint64_t *chunk_block, uint64_t n_chunks,
                       ChunkStat *stats, hipStream_t st) {
  if (n_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(scan_kernel, dim3((unsigned)((n_chunks + kScanChunksPerWG - 1) / kScanChunksPerWG)), dim3(256), 0,
                     st, in, blk, chunk_block, n_chunks, stats);
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

// Per block tokenisation of the N-stripped bases (Sec. 4.1) for blocks with
// N runs (each base located through the run map).  Grid: the blocks'
// 1024-token tiles, compact; each thread builds 4 tokens.
__global__ __launch_bounds__(256) void tokenise_kernel(const uint8_t *__restrict__ in, const SeqBlock *blk,
                                                       int n_blocks, const uint32_t *run_sp, const uint32_t *run_cum,
                                                       int s, int k, uint8_t *__restrict__ tok) {
  const SeqBlock b = blk[block_of_tile<&SeqBlock::t_tk>(blk, n_blocks, blockIdx.x)];
  const uint64_t jt = (blockIdx.x - b.t_tk) * kTokPerWG + (uint64_t)threadIdx.x * kTokPerThread;
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

hipError_t launch_tokenise(const uint8_t *in, const SeqBlock *blk, int n_blocks, uint64_t n_sk, uint64_t n_tk,
                           const uint32_t *run_sp, const uint32_t *run_cum, int s, int k, uint8_t *tok,
                           hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  if (n_tk) {
    hipLaunchKernelGGL(tokenise_kernel, dim3((unsigned)n_tk), dim3(256), 0, st, in, blk, n_blocks, run_sp, run_cum, s,
                       k, tok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return launch_skmer_blocks(in, blk, n_blocks, n_sk, s, k, tok, st);
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
__global__ __launch_bounds__(256) void detok_kernel(const SeqBlock *blk, int n_blocks, const uint32_t *run_start,
                                                    const uint32_t *run_len, const uint32_t *run_cum, int s, int k,
                                                    int bs, const uint8_t *__restrict__ tok,
                                                    const uint8_t *__restrict__ extras, uint8_t *__restrict__ out) {
  const SeqBlock b = blk[block_of_tile<&SeqBlock::t_raw>(blk, n_blocks, blockIdx.x)];
  const uint64_t tile = blockIdx.x - b.t_raw;   // this workgroup's 4096 raw bytes of the block
  if (b.n_runs == 0) {
    // no N runs: raw position = stripped position.  Thread t writes bytes
    // t, t + 256, ... of the workgroup's 4096, so each store instruction
    // covers consecutive bytes
    // (block positions fit 32 bits; division by s = 1..4 by shifts or the
    // exact 32-bit reciprocal of 3)
    const uint32_t w0 = (uint32_t)tile * 4096u, len = (uint32_t)b.raw_len;
    const uint32_t nseg = (uint32_t)(b.L * (uint64_t)bs), covered = (uint32_t)b.tail_off;
    const uint32_t ntail = (uint32_t)(b.nb - b.tail_off);
    const uint8_t *ex = extras + b.ex_off;
    const uint8_t *tk = tok + b.tok_off;
    uint8_t *o = out + b.raw_off;
    auto div_s = [&](uint32_t x) {
      return s == 3 ? __umulhi(x, 0xAAAAAAABu) >> 1 : x >> (s == 4 ? 2 : s == 2 ? 1 : 0);
    };
#pragma unroll 4
    for (int x = 0; x < 16; x++) {
      const uint32_t q = w0 + (uint32_t)(x * 256) + threadIdx.x;
      if (q >= len) break;
      uint32_t code;
      if (q < covered) {
        uint32_t j;
        int m;
        if (q < (uint32_t)k) { j = 0; m = (int)q; }
        else {
          const uint32_t dq = q - (uint32_t)k, qq = div_s(dq);
          j = qq + 1;
          m = k - s + (int)(dq - qq * (uint32_t)s);
        }
        const uint32_t e = j < nseg ? tk[j] : ex[ntail + (j - nseg)];
        code = (e >> (2 * (k - 1 - m))) & 3u;
      } else {
        code = ex[q - covered];
      }
      o[q] = (uint8_t)(0x54474341u >> (8 * code));   // 'A' 'C' 'G' 'T'
    }
    return;
  }
  const uint64_t r0 = tile * 4096 + (uint64_t)threadIdx.x * 16;
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

hipError_t launch_detok(const SeqBlock *blk, int n_blocks, uint64_t n_raw, const uint32_t *run_start,
                        const uint32_t *run_len, const uint32_t *run_cum, int s, int k, int bs, const uint8_t *tok,
                        const uint8_t *extras, uint8_t *out, hipStream_t st) {
  if (n_blocks == 0 || n_raw == 0) return hipSuccess;
  hipLaunchKernelGGL(detok_kernel, dim3((unsigned)n_raw), dim3(256), 0, st, blk, n_blocks, run_start, run_len,
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


// Training block of the static private model (Sec. 4.2.3): segment j is the
// Lp tokens that start at token floor(j * l / bs) of the whole token array.
// One workgroup per segment; floor(j l / bs) + Lp <= l since Lp <= l / bs.
__global__ __launch_bounds__(256) void sprm_gather_kernel(const uint8_t *tok, uint64_t l, uint32_t bs, uint32_t Lp,
                                                          uint8_t *dst) {
  const uint32_t j = blockIdx.x;
  const uint64_t start = (uint64_t)j * l / bs;
  const uint8_t *s8 = tok + start;
  uint8_t *d = dst + (uint64_t)j * Lp;
  for (uint32_t q = threadIdx.x; q < Lp; q += 256) d[q] = s8[q];
}

hipError_t launch_sprm_gather(const uint8_t *tok, uint64_t l, uint32_t bs, uint32_t Lp, uint8_t *dst,
                              hipStream_t st) {
  if (Lp == 0) return hipSuccess;
  if (bs == 0 || (uint64_t)Lp * bs > l || l > ~0ull / bs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sprm_gather_kernel, dim3(bs), dim3(256), 0, st, tok, l, bs, Lp, dst);
  return hipGetLastError();
}

}  // namespace pmklc
