// Library-private declarations of the launch-sequence loop (tf_kernels.hip):
// the paper's Transformer dynamic model and the MLP when it does not fit
// one compute unit.
#pragma once
#include "pmklc_internal.h"

namespace pmklc {

// ---- the paper's Transformer dynamic model (Sec. 4.2.4), arch 1 ----
// x_p = Emb[c_p] + Pos[p]; [q|k|v]_p = x_p Wqkv + bqkv; per head (dh = A/H
// columns) the last position's query attends over the t positions with
// scale 1/sqrt(dh); z = o Wo + bo; u = ReLU(z W1 + b1); g = u W2 + b2;
// logits = g Wh + bh.  Parameters in that order: Emb[V][E], Pos[t][E],
// Wqkv[E][3A], bqkv, Wo[A][A], bo, W1[A][F], b1, W2[F][A], b2, Wh[A][V], bh.
struct TfShape {
  int arch;                                        // 1 Transformer; 0 the MLP on the same launch sequence
  int nh, H0, H1;                                  // MLP: hidden layers and widths (input t E)
  int V, E, t, A, F, H, dh, bs;
  int64_t off_emb, off_pos, off_W[5], off_b[5];   // W: Wqkv, Wo, W1, W2, Wh (MLP: its layers; no Pos)
  int64_t P, stride;                               // parameters; floats per block slab (>= P + 1)
  int optimizer;                                   // 0 SGD, 1 Adam
  float lr, b1, b2, eps;
  int bf16;                                        // GEMM inputs rounded to BF16 (else FP32 MFMA)
  // the BiGRU static public model mixed in by Eq. 1 (sarch 1), or none (0):
  // embedding sE, gl layers of gh units per direction, Dense gd; offsets in
  // its own parameter vector (sP floats), layer l, direction d
  int sarch, sE, gh, gl, gd;
  int64_t s_emb, s_wih[2][2], s_whh[2][2], s_bih[2][2], s_bhh[2][2], s_dw, s_db, s_lw, s_lb, sP;
};
// the BiGRU static model's shape into s (false outside the kernel's limits:
// gh <= 128, 1 <= gl <= 2, sE <= 256, gd >= 1)
bool bigru_shape(int sE, int gh, int gl, int gd, TfShape &s);
// fills everything but bs/optimiser/bf16 from the widths; false when the
// shape is outside what the kernels take (A = H dh with dh a power of two
// <= 64, A <= 1024, t <= 256)
bool tf_shape(int k, int t, int E, int A, int F, int H, TfShape &s);
// the configurations' MLP (Dims' shape and parameter layout) on the same
// launch sequence: its layers as strided-batched matrix-core GEMMs, the
// embedding gradient as a one-hot GEMM; false when outside (nh <= 2,
// bs <= 1024)
bool mlp_seq_shape(const Dims &d, TfShape &s);

// Device state of a running loop, read by every kernel of a step so the
// launches of one step are the same every step.
struct TfState {
  int i;          // step
  int nact;       // active slots (blocks with L > i; slots hold blocks longest first)
  float c1, c2;   // Adam: 1 - b1^tau, 1 - b2^tau of this step's update
  float b1t, b2t; // running powers
  int pad[2];
};
struct TfSlot {   // one block as the Transformer loop sees it (slot order)
  uint64_t tok_off;     // first token of the block
  uint64_t slot_off;    // first word of its segment slots
  uint32_t L;           // steps
  uint32_t slot_words;  // words per segment slot
  int32_t block;        // block number (seg_bits / seg_words index)
  int32_t pad;
};
// Buffers of the loop, per slot unless noted (floats).
struct TfBufs {
  TfState *state;                 // [1]
  TfSlot *slots_desc;             // [n]
  float *params, *adam_m, *adam_v;   // [n][stride]
  const float *init;              // [stride] seeded parameters, copied into every slot
  float *X, *KV, *Q, *att, *O, *Z, *U, *G, *logits;   // activations
  float *dG, *dU, *dZ, *dO, *dQ, *dKV, *dX;          // gradients of activations
  float *act[2], *dact[2];        // MLP: hidden activations and their gradients
  int64_t sAct[2];
  float *part;                    // split-K partial sums [n][kSplit][max M N]
  uint32_t *cdf;                  // [n][bs][V+1]
  uint8_t *tokstep;               // [n][bs t] the step's context tokens (row-major)
  const float *stat;              // the BiGRU static model's parameters (sP floats, shared), or null
  float *lu;                      // [n][bs][V] its logits, then L^u - L^m for the mixing weight
  void *coder;                    // [n][bs] coder states
  int64_t sX, sKV, sQ, sAtt, sA, sU, sLog, sPart, sCdf, sTok;   // per-slot strides (elements)
};
constexpr int kTfSplit = 8;   // split-K slices of the long-K weight gradients

// runs the whole learning/coding loop of n blocks (encode: mode 0, decode: 1)
struct TfRun {
  int mode, n;                    // n slots
  const TfSlot *desc_host;        // host copy of the slot descriptors (longest first)
  uint8_t *tokens;
  uint32_t *stream_slots, *seg_bits;
  const uint32_t *seg_words;
  uint64_t max_L;
  // probes (slot 0): P at sorted steps, parameters after the last step
  const uint64_t *probe_steps_host;
  int n_probe;
  float *probe_P;
  float *params_out;
  uint64_t stop;                  // 0 = all steps
  // > 0: every `progress` steps the host waits for the stream and prints
  // the step reached to stderr (long runs report their own progress)
  uint64_t progress;
};
// carves the per-slot buffers of n slots out of `base` (null: sizes only);
// returns the floats used.  state, slots_desc, params, adam_m/v and init
// are the caller's.
uint64_t tf_bufs_carve(const TfShape &s, int n, float *base, TfBufs &b);
hipError_t tf_run(const TfShape &s, const TfBufs &b, const TfRun &r, hipStream_t st);
hipError_t tf_init_params(const TfShape &s, uint64_t seed, float *out, hipStream_t st);
// The one-layer BiGRU static private model (gru_train.hip): its seeded
// initialisation; whether the training kernels take the shape (embedding
// <= 32, units per direction <= 64, one layer); the training scratch in
// floats (part_stride, nwg: the per-workgroup partial gradients); the
// training itself on the gathered block tok [bs][Lp], W updated in place
// (adam_m / adam_v: sP floats each for Adam, else null).
hipError_t gru_init_params(const TfShape &s, uint64_t seed, float *out, hipStream_t st);
bool gru_train_supported(const TfShape &s);
uint64_t gru_train_floats(const TfShape &s, uint64_t &part_stride, int &nwg);
hipError_t gru_train(const TfShape &s, const uint8_t *tok, uint64_t Lp, float *W, float *buf, float *adam_m,
                     float *adam_v, hipStream_t st);
// the model as a differentiable op over `rows` contexts (one slot of bs = rows)
hipError_t tf_forward_op(const TfShape &s, const TfBufs &b, const float *params, const uint8_t *ctx,
                         float *logits, hipStream_t st);
hipError_t tf_backward_op(const TfShape &s, const TfBufs &b, const float *params, const uint8_t *ctx,
                          const float *dlogits, float *grad, hipStream_t st);

}  // namespace pmklc
