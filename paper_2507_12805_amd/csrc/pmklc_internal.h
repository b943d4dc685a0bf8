// Library-private declarations shared by the HIP sources of libpmklc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmklc {

constexpr int kTotalBits = 16;
constexpr uint32_t kTotal = 1u << kTotalBits;  // frequency total of the coder
constexpr int kMaxLayers = 3;                  // up to two hidden layers + output
constexpr int kFixShift = 44;                  // fixed-point scale of the embedding-gradient sums

// Runtime shape of one model (dynamic or static, which share a shape).
struct Dims {
  int V, E, t, D, bs, nh;
  int H[2];
  int dim[kMaxLayers + 1];      // dim[0] = D, ..., dim[nh+1] = V
  int off_emb;
  int off_W[kMaxLayers], off_b[kMaxLayers];
  int P;                        // parameters without the mixing weight
  int stride;                   // floats per block parameter slab (>= P+1, multiple of 64)
  int VS;                       // row stride (floats) of the logits / probability rows in LDS (V + 4)
  int ES;                       // row stride (entries) of the fixed-point embedding gradient (E + 1)
  int EP;                       // row pitch (floats) of the embedding tables in LDS (E + 4: rows of
                                // 16 tokens fall in distinct banks, float4 runs stay aligned)
  int HP;                       // row pitch (floats) of the hidden activations of the matrix-core
                                // kernel in LDS (H[0] + 4, same reason)
  int RS;                       // context ring length in positions (power of two >= t + CH); the ring is
                                // position-major: position q of row j is byte (q mod RS) * bs + j
  int CH;                       // tokens staged per row at a time (encode)
  uint32_t Emag;                // ceil(2^32 / E): k / E = umulhi(k, Emag) for k < 2^20, E < 4096
  int static_on;                // frozen static model mixed in (Eq. 1)
  int model_on;                 // dynamic model present (else every token is uniform)
  int optimizer;                // 0 SGD, 1 Adam
  float lr, b1, b2, eps;
};

// LDS layout (byte offsets into dynamic shared memory).
struct LdsLayout {
  int emb, embs, ring, act[2], lm, lu, cdf, tgt, dh[2], demb, misc, total;
  int cst;            // per-segment coder states (CoderState, one per row)
  int dpt;            // matrix-core kernel: BF16 dpre^T fragments (aliases cdf, dead in the backward, when it fits)
  int dpb;            // BF16 matrix-core kernel: dpre as B3's B fragments (aliases lu, dead in the backward, when
                      // it fits), or -1 when absent
  int act_global;     // 1: act[] and dh[] are float offsets into a per-workgroup global slab
  int act_slot;       // floats per workgroup slab
  // on-chip kernel only (step_chip.hip): BF16 W1 copy in F1 fragment order,
  // FP32 W2^T [V][H+4], biases [H+V], their gradients [H+V], the eight
  // wave partials of the embedding gradient [8][V][E], and a BF16 copy of
  // the embedding [V][E+8]
  int w1c, w2t, bias, gb, eg, embh;
};
constexpr int kMaxGrid = 1024;   // upper bound on step-kernel workgroups (global slabs)

// One data block as the step kernel sees it.
struct BlockDesc {
  uint64_t tok_off;      // first token of the block in the token array
  uint64_t slot_off;     // first 32-bit word of the block's segment slots
  uint32_t L;            // steps = tokens per segment
  uint32_t slot_words;   // words per segment slot
  uint32_t S;            // model passing point (steps); used when has_snap
  int32_t pred;          // block whose snapshot initialises this one, or -1
  int32_t has_snap;      // a successor waits on this block's snapshot
  int32_t pad;
};

struct StepArgs {
  Dims d;
  LdsLayout lay;
  int mode;                       // 0 encode, 1 decode
  int n_blocks;
  const BlockDesc *blocks;
  uint8_t *tokens;                // encode: input; decode: output
  float *params;                  // [n_blocks][stride] live parameters (+ a at index P)
  float *adam_m, *adam_v;         // [n_blocks][stride] or null
  const float *init;              // [stride] seeded initial parameters (+ a)
  const float *stat;              // [P] static parameters or null
  float *snap;                    // [n_blocks][stride] model-passing snapshots or null
  int *snap_flag;                 // [n_blocks] 1 when the snapshot is written, 2 when the block gave up
  uint32_t *progress;             // [n_blocks] steps done by a block whose successor may wait on it
                                  // (0 before its first step; zeroed before launch)
  const int *order;               // [n_blocks] queue position -> block, or null (block order); a block's
                                  // model-passing predecessor always comes before it
  int *queue;                     // work counter (zeroed before launch)
  int *err;                       // error word (0 = ok)
  uint32_t *slots;                // encode: segment slots; decode: aligned streams
  uint32_t *seg_bits;             // encode: bits per segment [n_blocks][bs]
  uint32_t *seg_words;            // decode: words available per segment [n_blocks][bs]
  // trace/probe (block 0 only)
  uint64_t stop;                  // 0 = all steps
  const uint64_t *probe_steps;    // device, sorted
  int n_probe;
  float *probe_P;                 // [n_probe][bs][V]
  float *params_out;              // [P+1] parameters after the last step, or null
  long long spin_limit;           // model-passing wait: sleeps without progress of a running predecessor
                                  // before the waiting block gives up (error bit 4)
  float *act_scratch;             // [grid][act_slot] activations when lay.act_global
  unsigned long long *phase_clk;  // [12] per-phase wall-clock ticks of block 0, or null
  // BF16 matrix-core kernel: W1 rounded to BF16 in the first layer's
  // B-fragment order (see w1_frag_index), one slab per workgroup for the
  // dynamic model (kept in step with the FP32 master by the update) and one
  // for the static model; null otherwise
  uint16_t *w1f;
  const uint16_t *s1f;
};

// Offset of W1[d][h] (D x H) in the fragment-ordered BF16 copy: 16-column
// tiles n of h, 32-row k-steps ks of d, then the 64 lanes (r = h % 16,
// g = (d % 32) / 8) and 8 consecutive d per lane, so a wave reads one k-step
// of a column tile as 1 KB of contiguous memory.
__host__ __device__ inline uint32_t w1_frag_index(int d, int h, int D) {
  const uint32_t n = (uint32_t)h >> 4, ks = (uint32_t)d >> 5;
  const uint32_t lane = ((uint32_t)h & 15u) + 16u * (((uint32_t)d & 31u) >> 3);
  return ((n * ((uint32_t)D >> 5) + ks) * 64u + lane) * 8u + ((uint32_t)d & 7u);
}
hipError_t launch_w1_frag(const float *W1, int D, int H, uint16_t *out, hipStream_t st);

hipError_t launch_step(const StepArgs &a, int grid, int nt, hipStream_t st);
// f1: the first layer's MFMA unit, 1 = four hidden tiles per unit (hidden
// widths in multiples of 64), 0 = two, -1 = four where the width allows;
// like nt it never changes a value
hipError_t launch_step_mfma(const StepArgs &a, const StepArgs *a_dev, int grid, bool bf16, int nt, int f1,
                            hipStream_t st);
// the on-chip BF16 kernel: shapes compiled in, and its launch (512 threads)
bool chip_supports(const Dims &d);
hipError_t launch_step_chip(const StepArgs &a, const StepArgs *a_dev, int grid, hipStream_t st);
hipError_t launch_init_params(const Dims &d, uint64_t seed, float *out, hipStream_t st);
hipError_t launch_init_scaled(uint64_t seed, int P, int n_tensors, const int *end, const double *scale, float *out,
                              hipStream_t st);
hipError_t launch_quantise(const float *P, uint32_t rows, uint32_t V, uint32_t *cdf, hipStream_t st);
hipError_t launch_wnc_encode(const uint32_t *lo, const uint32_t *hi, uint64_t m, uint32_t *out_words,
                             uint32_t cap_words, uint64_t *nbits_dev, int *err, hipStream_t st);
hipError_t launch_wnc_decode(const uint32_t *words, uint32_t nwords, const uint32_t *cdfs, uint32_t V,
                             uint64_t m, uint32_t *sym, hipStream_t st);

// ---- the dynamic model as a stand-alone differentiable op ----
uint64_t dm_op_workspace(const Dims &d, int rows);
hipError_t dm_forward(const Dims &d, const float *W, const uint8_t *ctx, int rows, float *logits, void *ws,
                      int *err_host, hipStream_t st);
hipError_t dm_backward(const Dims &d, const float *W, const uint8_t *ctx, int rows, const float *dlogits,
                       float *grad, void *ws, int *err_host, hipStream_t st);

// ---- sequence kernels (tokeniser, scan, inverse) ----
struct SeqBlock {              // per block, shared by the scan / tokenise / inverse kernels
  uint64_t raw_off, raw_len;   // raw input bytes
  uint64_t chunk0;             // first scan chunk of the block
  uint64_t run0, n_runs;       // first run in the run table, count
  uint64_t nb;                 // bases after N removal
  uint64_t tok_off, l;         // token array offset, token count
  uint64_t tail_off;           // first tail base (stripped coordinates)
  uint64_t ex_off;             // offset of the block's extras (tail codes then remainder tokens)
  uint64_t L;                  // steps
  // first workgroup of this block in the compact grids of the tokenisers
  // and the inverse (prefix sums over the blocks before it; a block with no
  // work there has as many workgroups as zero)
  uint64_t t_sk;               // GskE tiles (4096 tokens) of a block without N runs
  uint64_t t_tk;               // run-map tokeniser tiles (1024 tokens) of a block with N runs
  uint64_t t_raw;              // inverse tiles (4096 raw bytes)
};
// sets t_sk, t_tk, t_raw and returns the grids' sizes
void assign_tiles(SeqBlock *sb, int n_blocks, uint64_t &n_sk, uint64_t &n_tk, uint64_t &n_raw);

constexpr int kScanChunk = 4096;   // raw bytes per scan chunk

struct ChunkStat {             // per scan chunk
  uint32_t n_N, n_runs, bad, pad;
};

hipError_t launch_skmer_direct(const uint8_t *in, uint64_t n, int s, int k, uint8_t *tok, uint64_t l, int *err,
                               hipStream_t st);
hipError_t launch_scan(const uint8_t *in, const SeqBlock *blk, const uint64_t *chunk_block, uint64_t n_chunks,
                       ChunkStat *stats, hipStream_t st);
// run_end: filled with run ends; run_sp_kernel turns them into lengths
hipError_t launch_runs(const uint8_t *in, const SeqBlock *blk, const uint64_t *chunk_block, uint64_t n_chunks,
                       const ChunkStat *stats, const uint64_t *chunk_run0, uint32_t *run_start, uint32_t *run_len,
                       hipStream_t st);
hipError_t launch_run_sp(const SeqBlock *blk, int n_blocks, const uint32_t *run_start, uint32_t *run_len,
                         uint32_t *run_sp, uint32_t *run_cum, hipStream_t st);
hipError_t launch_tokenise(const uint8_t *in, const SeqBlock *blk, int n_blocks, uint64_t n_sk, uint64_t n_tk,
                           const uint32_t *run_sp, const uint32_t *run_cum, int s, int k, uint8_t *tok,
                           hipStream_t st);
hipError_t launch_extras(const uint8_t *in, const SeqBlock *blk, int n_blocks, const uint32_t *run_sp,
                         const uint32_t *run_cum, int s, int k, int bs, const uint8_t *tok, uint8_t *extras,
                         hipStream_t st);
hipError_t launch_detok(const SeqBlock *blk, int n_blocks, uint64_t n_raw, const uint32_t *run_start,
                        const uint32_t *run_len, const uint32_t *run_cum, int s, int k, int bs, const uint8_t *tok,
                        const uint8_t *extras, uint8_t *out, hipStream_t st);
// streams: segment i is seg_bytes[i] bytes at byte offset src[i] (or words
// src_word[i]) -> dst
hipError_t launch_gather_streams(const uint32_t *slots, const uint64_t *seg_src_word, const uint64_t *seg_dst,
                                 const uint32_t *seg_bytes, uint64_t n_seg, uint8_t *dst, hipStream_t st);
hipError_t launch_scatter_streams(const uint8_t *src, const uint64_t *seg_src, const uint64_t *seg_dst_word,
                                  const uint32_t *seg_bytes, const uint32_t *seg_words, uint64_t n_seg,
                                  uint32_t *slots, hipStream_t st);
// static private model (Sec. 4.2.3): training block of bs segments of Lp
// tokens, segment j from token floor(j * l / bs) of tok[0, l)
hipError_t launch_sprm_gather(const uint8_t *tok, uint64_t l, uint32_t bs, uint32_t Lp, uint8_t *dst,
                              hipStream_t st);

}  // namespace pmklc
