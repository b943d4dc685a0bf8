/*
 * pmklc.h — C ABI of the MI355X PMKLC hot path (arXiv 2507.12805).
 *
 * The library compresses DNA (ASCII A/C/G/T/N) losslessly with the paper's
 * pipeline: the GPU (s,k)-mer encoder (Sec. 4.1), per-block online-learned
 * probability prediction (dynamic model, optionally mixed with a frozen
 * static model by Eq. (1), trained every step on the cross-entropy of
 * Eq. (2), Sec. 2 steps (1)-(4)), and an arithmetic coder driven by the
 * quantised probabilities, over many data blocks at once (Sec. 4.3).
 *
 * Conventions for every call:
 *   - Pointers named *_dev are device pointers (HBM of the current HIP
 *     device); *_host are host pointers. The caller owns and allocates every
 *     buffer; the library keeps no pointer after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Calls are synchronous with respect to the host: they return after the
 *     work they queued has finished (output sizes depend on the data).
 *   - Every call returns a pmklc_status and never aborts. On
 *     PMKLC_ERR_BUFFER_TOO_SMALL the size out-parameter receives the size
 *     that is needed; on any other error out-parameters are left unchanged.
 *   - Output bytes are a pure function of (input, configuration, static
 *     weights, library version): they do not depend on the stream, buffer
 *     addresses, launch shapes or timing.
 *   - Layout of model parameters (flat FP32, little-endian): Emb[V][E], then
 *     per linear layer l = 0..n_hidden: W_l[d_l][d_{l+1}] (input-major) and
 *     b_l[d_{l+1}], with d_0 = t*E, d_l = hidden[l-1], d_{n_hidden+1} = V,
 *     V = 4^k. Where a parameter vector carries the mixing weight, the
 *     pre-sigmoid value a (alpha = 1/(1+exp(-a))) follows as one more float.
 */
#ifndef PMKLC_H
#define PMKLC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PMKLC_OK = 0,
  PMKLC_ERR_INVALID_ARG = -1,      /* bad configuration or argument */
  PMKLC_ERR_INVALID_BASE = -2,     /* input byte outside the accepted alphabet */
  PMKLC_ERR_BUFFER_TOO_SMALL = -3, /* a caller buffer is too small (size reported) */
  PMKLC_ERR_CORRUPT = -4,          /* container malformed or truncated */
  PMKLC_ERR_MODEL_MISMATCH = -5,   /* static weights or numeric path differ from the container's */
  PMKLC_ERR_DEVICE = -6,           /* a HIP call failed */
  PMKLC_ERR_UNSUPPORTED = -7,      /* valid configuration that this build has no kernel for */
  PMKLC_ERR_SCRATCH_LIMIT = -8     /* input needs more than pmklc_compress_noalloc's fixed buffer */
} pmklc_status;

enum { PMKLC_SGD = 0, PMKLC_ADAM = 1 };
/* Arithmetic of the model GEMMs. PMKLC_FP32 uses the FP32 matrix-core kernel
 * when the model shape allows it (one hidden layer; bs, hidden and V multiples
 * of 32, E of 8) and the per-thread FMA kernel otherwise; PMKLC_FP32_VALU
 * always uses the per-thread FMA kernel; PMKLC_BF16 rounds GEMM inputs to
 * BF16 on the matrix cores (FP32 accumulation; softmax, mixing weight,
 * quantiser and optimiser state stay FP32). The container records which
 * numeric path made it, and only that path decodes it. */
enum { PMKLC_FP32 = 0, PMKLC_BF16 = 1, PMKLC_FP32_VALU = 2 };
enum { PMKLC_BATCHED = 0, PMKLC_PLAIN = 1 };      /* all blocks in one launch | one block per launch */
/* Dynamic model. PMKLC_ARCH_MLP: embedding E, concatenation of the t
 * context embeddings, n_hidden Dense + ReLU layers, linear head (the
 * configurations' model). PMKLC_ARCH_TRANSFORMER, the paper's DM
 * (Sec. 4.2.4): embedding E plus a learned position embedding, one
 * attention layer of `heads` heads and width A = hidden[0] whose query is
 * the last context position, a shared ReLU FFN of width F = hidden[1],
 * linear head; n_hidden = 2. Its parameter layout (FP32): Emb[V][E],
 * Pos[t][E], Wqkv[E][3A], bqkv[3A], Wo[A][A], bo[A], W1[A][F], b1[F],
 * W2[F][A], b2[A], Wh[A][V], bh[V]. It runs without a static model and
 * without model passing (PMKLC_ERR_INVALID_ARG / PMKLC_ERR_UNSUPPORTED), in
 * PMKLC_FP32 (FP32 matrix cores) or PMKLC_BF16, for A / heads a power of two
 * <= 64, A <= 1024, E <= 1024, t <= 256, bs <= 1024, bs * t <= 65536. */
enum { PMKLC_ARCH_MLP = 0, PMKLC_ARCH_TRANSFORMER = 1 };
/* Static model (Sec. 4.2.2; the public one, or the private one of Sec.
 * 4.2.3, which has the same shape). PMKLC_STATIC_MLP: the dynamic model's
 * own shape. PMKLC_STATIC_BIGRU: an embedding of static_embed (paper: 16),
 * gru_layers (1 or 2; paper: 2) bidirectional GRU layers of gru_hidden units
 * per direction (gates r, z, n with n = tanh(W_in x + b_in + r (W_hn h +
 * b_hn)), h' = (1 - z) n + z h), the last layer's final states of both
 * directions (forward after the last context position, backward after the
 * first) concatenated, Dense of `dense` units (paper: 128) with ReLU, linear
 * head to V. Layout (FP32): Emb[V][static_embed]; per layer, forward then
 * backward direction: W_ih[3h][in] (in = static_embed, then 2h),
 * W_hh[3h][h], b_ih[3h], b_hh[3h]; Wd[2h][dense], bd; Wl[dense][V], bl.
 * Mixed by Eq. 1 with an MLP dynamic model on the launch-sequence loop
 * (numeric path 7 / 8); the recurrence runs in FP32 on both precisions.
 * gru_hidden <= 128, static_embed <= 256. As the private model (selector
 * SPRM|DM, or the Model Selector's choice above its bound) the BiGRU has one
 * layer (paper: 1; gru_layers = 2 gives PMKLC_ERR_INVALID_ARG) and is trained
 * on the input in FP32 before coding (the training block and steps of
 * pmklc_config.selector's SPRM), for static_embed <= 32 and gru_hidden <= 64
 * (else PMKLC_ERR_UNSUPPORTED); the container stores it in this layout. */
enum { PMKLC_STATIC_MLP = 0, PMKLC_STATIC_BIGRU = 1 };
/* Model selector S = {S0, S1, S2} of Sec. 4.2.1 as a bit mask. Accepted:
 * 0, DM, SPUM|DM, SPRM|DM (the selector enables one static model at most),
 * or AUTO.
 *
 * SPRM (Sec. 4.2.3, stage (b) of Fig. 2): before coding, the call trains a
 * static private model on the input and stores it in the container (4 P
 * bytes of FP32 after the file table; the header's static CRC-32 covers
 * them). It has the static model's shape (static_arch: the dynamic model's,
 * or the one-layer BiGRU), starts from the seeded
 * initialisation under seed ^ 0x5350524D and takes the dynamic model's
 * learning steps (its optimiser and rate, no mixing) over one
 * training block of bs segments of Lp = min(floor(l / bs), 8192) tokens,
 * segment j starting at token floor(j * l / bs) of the input's token
 * sequence (all blocks' tokens in block order, l in all). The coding pass
 * then mixes it by Eq. (1) exactly as it mixes a public static model.
 *
 * AUTO (the Model Selector, Sec. 4.2.1): resolved per call from the input
 * size n in bytes: SPRM|DM when n > ms_threshold (0 = 500 * 10^6), else
 * SPUM|DM when static_host is given, else DM. The container records the
 * resolved selector. */
enum {
  PMKLC_SEL_UNIFORM = 0,   /* no model: every token coded with the uniform distribution */
  PMKLC_SEL_SPUM = 1,      /* S0: frozen static public model, supplied in static_host */
  PMKLC_SEL_SPRM = 2,      /* S1: static private model, trained on the input, stored in the container */
  PMKLC_SEL_DM = 4,        /* S2: dynamic model */
  PMKLC_SEL_AUTO = 8       /* the Model Selector's choice by input size (see above) */
};

typedef struct pmklc_config {
  uint32_t struct_size;     /* sizeof(pmklc_config) */
  uint32_t s, k;            /* (s,k)-mer step and window, 1 <= s <= k <= 4 (Sec. 4.1) */
  uint32_t t;               /* context length in tokens (Sec. 2 step (2)) */
  uint32_t bs;              /* tokens per step = contiguous segments per block */
  uint32_t embed;           /* embedding width E */
  uint32_t n_hidden;        /* hidden layers, 0..2 */
  uint32_t hidden[4];       /* hidden widths */
  uint32_t optimizer;       /* PMKLC_SGD | PMKLC_ADAM */
  float lr, beta1, beta2, eps;
  uint32_t precision;       /* PMKLC_FP32 | PMKLC_BF16 | PMKLC_FP32_VALU */
  uint32_t schedule;        /* PMKLC_BATCHED | PMKLC_PLAIN */
  uint32_t selector;        /* PMKLC_SEL_*: 0, DM, SPUM|DM, SPRM|DM or AUTO */
  uint32_t smp_ppm;         /* step-wise model passing point in parts per million of a
                               block's steps (paper: 5% = 50000); 0 = off (Sec. 4.3) */
  uint64_t seed;            /* seed of the dynamic model's initial weights */
  uint32_t n_blocks;        /* data blocks (Sec. 4.3 data chunker) */
  const uint64_t *block_len_host;   /* raw bytes per block, or NULL = equal split */
  uint32_t n_files;         /* files in the input; model passing never crosses a file */
  const uint64_t *file_blocks_host; /* blocks per file, or NULL = one file */
  const float *static_host; /* frozen static public model (parameter layout above, no alpha) */
  uint64_t static_len;      /* number of floats in static_host */
  uint64_t ms_threshold;    /* PMKLC_SEL_AUTO's size bound in input bytes; 0 = 500 * 10^6 */
  uint32_t arch;            /* dynamic model: PMKLC_ARCH_MLP or PMKLC_ARCH_TRANSFORMER */
  uint32_t heads;           /* attention heads (PMKLC_ARCH_TRANSFORMER) */
  uint32_t static_arch;     /* static model: PMKLC_STATIC_MLP or PMKLC_STATIC_BIGRU */
  uint32_t static_embed, gru_hidden, gru_layers, dense;   /* PMKLC_STATIC_BIGRU's widths */
} pmklc_config;

/* Sec. 4.1 (GskE): maps ASCII bases A,C,G,T (0,1,2,3) to (s,k)-mer ids
 * e_j = sum_{m<k} 4^(k-1-m) * b_{j*s+m}, j = 0 .. floor((n-k)/s), one byte
 * per id. bases_dev: n bytes; tokens_dev: capacity `cap` bytes. *n_tokens
 * receives floor((n-k)/s)+1 (0 if n < k). Any byte other than A,C,G,T
 * (including N) gives PMKLC_ERR_INVALID_BASE. */
pmklc_status pmklc_encode_skmer(const uint8_t *bases_dev, uint64_t n, uint32_t s, uint32_t k,
                                uint8_t *tokens_dev, uint64_t cap, uint64_t *n_tokens, void *stream);

/* Upper bounds for pmklc_compress on n input bytes: *max_out = container
 * bytes, *ws_bytes = device workspace bytes. */
pmklc_status pmklc_compress_bound(const pmklc_config *cfg, uint64_t n, uint64_t *max_out,
                                  uint64_t *ws_bytes);

/* Sec. 2 (compression steps (1)-(4)) over the blocks of Sec. 4.3.
 * in_dev: n bytes of ASCII A/C/G/T/N (N runs are stored aside; any other
 * byte gives PMKLC_ERR_INVALID_BASE). ws_dev: workspace of at least the
 * bound's ws_bytes. out_host: container, capacity out_cap; *out_len its
 * length. With PMKLC_PROGRESS=<k> in the environment, the models run as a
 * sequence of launches per step (the Transformer, the BiGRU static model,
 * the MLPs too large for one CU) wait for the stream every k steps and
 * print the step reached to stderr (pmklc_decompress too). */
pmklc_status pmklc_compress(const pmklc_config *cfg, const uint8_t *in_dev, uint64_t n, void *ws_dev,
                            uint64_t ws_bytes, uint8_t *out_host, uint64_t out_cap, uint64_t *out_len,
                            void *stream);

/* pmklc_compress for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and the same container bytes as
 * pmklc_compress, with the workspace taken from a fixed buffer that the
 * library holds in device memory (64 MiB per device, reserved when the
 * library's code is loaded on that device and held until the process ends)
 * instead of a caller's ws_dev. The call makes no device allocation: no
 * hipMalloc/hipFree, no timing events, no autotuner trial runs (the
 * workgroup width is the cached choice for the model shape, else the
 * default; no width changes a value). Inputs whose pmklc_compress_bound
 * workspace exceeds 64 MiB give PMKLC_ERR_SCRATCH_LIMIT before any device
 * work (about 6.5 million bases for the 16-wide embedding, 32-wide hidden
 * model). The buffer is shared by every call on the device and keeps the
 * last call's contents; the call clears what must start at zero. Calls
 * from threads of one process are serialised per device by a lock; calls
 * that overlap on one device through other means (another copy of the
 * library in the same process) would race. in_dev, out_host, out_cap,
 * out_len, stream and the errors are those of pmklc_compress. */
pmklc_status pmklc_compress_noalloc(const pmklc_config *cfg, const uint8_t *in_dev, uint64_t n,
                                    uint8_t *out_host, uint64_t out_cap, uint64_t *out_len, void *stream);

/* Reads a container's header: *n_bases = decompressed size, *ws_bytes =
 * device workspace needed by pmklc_decompress. */
pmklc_status pmklc_decompress_info(const uint8_t *cbf_host, uint64_t len, uint64_t *n_bases,
                                   uint64_t *ws_bytes);

/* Sec. 2 (decompression): the same models, updated the same way, restore
 * the input from the container. For a container made with the public
 * static model, static_host must be that model (checked by CRC-32), else
 * PMKLC_ERR_MODEL_MISMATCH; a private model is read from the container
 * (checked by CRC-32, else PMKLC_ERR_CORRUPT) and static_host is ignored.
 * out_dev receives n_bases bytes. */
pmklc_status pmklc_decompress(const uint8_t *cbf_host, uint64_t len, const float *static_host,
                              uint64_t static_len, void *ws_dev, uint64_t ws_bytes, uint8_t *out_dev,
                              uint64_t out_cap, uint64_t *out_len, void *stream);

const char *pmklc_status_string(pmklc_status s);

/* ---- Exports for parity tests (same device code as the hot path) ---- */

/* Frequency quantisation of probabilities: for each of `rows` rows of V
 * FP32 probabilities, f_v = 1 + floor(p_v * (2^16 - V)) with the product
 * taken exactly, the residual 2^16 - sum(f) added to the largest p (lowest
 * index on ties); cdf_dev receives rows x (V+1) cumulative counts (u32).
 * V is a vocabulary size 4^k: 4, 16, 64 or 256 (else ERR_INVALID_ARG). */
pmklc_status pmklc_quantise(const float *probs_dev, uint32_t rows, uint32_t V, uint32_t *cdf_dev,
                            void *stream);

/* Arithmetic coder (Witten, Neal, Cleary 1987; 32-bit, total 2^16) over m
 * symbols given as [cum_lo, cum_hi) pairs (u32 device arrays). out_dev:
 * capacity `cap` bytes, bits most significant first; *nbits receives the
 * stream length in bits. */
pmklc_status pmklc_wnc_encode(const uint32_t *cum_lo_dev, const uint32_t *cum_hi_dev, uint64_t m,
                              uint8_t *out_dev, uint64_t cap, uint64_t *nbits, void *stream);

/* Inverse of pmklc_wnc_encode: cdfs_dev holds m rows of V+1 cumulative
 * counts; symbols_dev receives m u32 symbols. */
pmklc_status pmklc_wnc_decode(const uint8_t *in_dev, uint64_t nbytes, const uint32_t *cdfs_dev, uint32_t V,
                              uint64_t m, uint32_t *symbols_dev, void *stream);

/* Runs the learning loop of one block over l tokens (tokens_dev), exactly
 * as pmklc_compress does for a block (Sec. 2 steps (2)-(4)), coding into
 * its own streams. init_dev: initial parameters + a (n_params+1 floats) or
 * NULL for the seeded ones. static_dev: static parameters (device) or NULL.
 * stop: run only the first `stop` steps (0 = all). probe_steps_host:
 * sorted step indices whose FP32 probabilities [bs][V] are written to
 * probs_dev (n_probe x bs x V). params_dev receives the parameters + a
 * after the last step run (n_params+1 floats). If streams_len is not NULL,
 * *streams_len receives the byte length of the bs segment streams,
 * byte-aligned and concatenated in segment order (the block's payload in
 * a container), and streams_host (capacity streams_cap bytes) receives them
 * (PMKLC_ERR_BUFFER_TOO_SMALL if it is smaller). Allocates its own
 * temporary device memory (a test export). */
pmklc_status pmklc_model_trace(const pmklc_config *cfg, const uint8_t *tokens_dev, uint64_t l,
                               const float *static_dev, const float *init_dev, uint64_t stop,
                               const uint64_t *probe_steps_host, uint32_t n_probe, float *probs_dev,
                               float *params_dev, uint8_t *streams_host, uint64_t streams_cap,
                               uint64_t *streams_len, void *stream);

/* Timing of the last pmklc_compress / pmklc_decompress on this thread,
 * measured with HIP events on the call's stream around the step kernel
 * (the per-block learning + coding loop), plus the work it did. */
typedef struct pmklc_timing {
  float step_ms;          /* step kernel(s): first launch start to last launch end */
  float call_ms;          /* whole call, host entry to return */
  uint64_t model_rows;    /* rows (tokens) that went through the model: sum_b bs * max(0, L_b - t) */
  uint64_t coded_tokens;  /* tokens coded by the arithmetic coders: sum_b bs * L_b */
  uint64_t max_steps;     /* longest block's step count (the critical path) */
  uint32_t launches;      /* step-kernel launches */
  uint32_t threads;       /* threads per workgroup the autotuner chose */
  uint32_t wall_khz;      /* device wall-clock rate for phase_ticks */
  /* With PMKLC_PHASES=1 in the environment: wall-clock ticks block 0 spent
   * per phase of its loop (0 staging, 1 forward, 2 softmax + quantiser,
   * 3 coder, 4 loss gradient, 5 backward, 6 embedding update; matrix-core
   * backward split into 8 input gradient, 9 output-layer update + embedding
   * scatter, 10 first-layer update). Zero otherwise. */
  uint64_t phase_ticks[12];
  uint32_t f1_units;      /* hidden tiles per first-layer MFMA unit the autotuner chose for the
                             global-weight matrix-core kernel (4 or 2); 0 for the other kernels */
  uint32_t reserved;
} pmklc_timing;
pmklc_status pmklc_last_timing(pmklc_timing *t);

/* The dynamic model as a differentiable op (Sec. 4.2.4; Sec. 2 step (4)),
 * for autograd use and gradient checks. MLP: uses cfg's k, t, embed,
 * n_hidden (0..2) and hidden; any widths.
 *   params_dev: n_params FP32 (layout above, no mixing weight);
 *   ctx_dev: rows x t token ids (u8, < 4^k; oldest first);
 *   logits_dev: rows x V FP32 output.
 * pmklc_dm_backward writes grad_dev (n_params FP32, same layout) = the
 * gradient of sum(dlogits * logits) with respect to the parameters; the
 * activations are recomputed from ctx_dev, not stored. The embedding
 * gradient is summed in 64-bit fixed point (scale 2^44), so results do not
 * depend on scheduling. ws_dev must hold pmklc_dm_workspace bytes. A token
 * >= 4^k gives PMKLC_ERR_INVALID_ARG.
 * With arch = PMKLC_ARCH_TRANSFORMER the op is the Transformer DM (same
 * argument meanings, its own parameter layout above; rows <= 1024), run by
 * the matrix-core kernels of the compression loop in cfg->precision (FP32 or
 * BF16 GEMM inputs); its backward recomputes the activations and sums every
 * gradient in a fixed order. */
pmklc_status pmklc_dm_workspace(const pmklc_config *cfg, uint32_t rows, uint64_t *ws_bytes);
pmklc_status pmklc_dm_forward(const pmklc_config *cfg, const float *params_dev, const uint8_t *ctx_dev,
                              uint32_t rows, float *logits_dev, void *ws_dev, uint64_t ws_bytes,
                              void *stream);
pmklc_status pmklc_dm_backward(const pmklc_config *cfg, const float *params_dev, const uint8_t *ctx_dev,
                               uint32_t rows, const float *dlogits_dev, float *grad_dev, void *ws_dev,
                               uint64_t ws_bytes, void *stream);

/* Number of model parameters (without the mixing weight) for cfg. */
uint64_t pmklc_param_count(const pmklc_config *cfg);

#ifdef __cplusplus
}
#endif
#endif
