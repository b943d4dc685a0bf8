// Host side of libpmklc: configuration checks, block planning (Sec. 4.3),
// workspace layout, container writing/parsing, and the orchestration of
// the HIP kernels behind the C ABI in include/pmklc.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/pmklc.h"
#include "pmklc_internal.h"
#include "seq_loop.h"

using namespace pmklc;

// Status words of the calls that take no workspace (the encoder's error flag,
// the coder export's bit count and error flag): a fixed pool in device memory
// owned by the library, 32 bytes per call in flight on a device, so that no
// call allocates.  Each device holds its own copy (its address is looked up
// once per device).
namespace pmklc {
constexpr int kStatusSlots = 64;
__device__ __align__(256) unsigned long long g_status_words[kStatusSlots * 4];

// The workspace of pmklc_compress_noalloc (callers that cannot allocate
// device memory): a fixed buffer per device, held until the process ends.
// Host code never passes the array's name to a kernel or copy: it uses the
// device address looked up with hipGetSymbolAddress.
constexpr uint64_t kScratchBytes = 64ull << 20;
__device__ __align__(256) uint8_t scratch[kScratchBytes];
}  // namespace pmklc

namespace {

struct StatusPool {
  std::mutex mu;
  std::condition_variable cv;
  unsigned long long *base = nullptr;   // this device's g_status_words
  uint64_t busy = 0;                    // bit i: slot i in use
};
constexpr int kMaxDevices = 64;
StatusPool g_status_pool[kMaxDevices];

// One slot of the pool on the current device for the length of a call; a
// call waits while all slots are taken.  Released only after the call's
// stream has drained, so no kernel can still write it.
struct StatusSlot {
  StatusPool *pool = nullptr;
  hipStream_t st = nullptr;
  int idx = -1;
  unsigned long long *ptr = nullptr;   // 4 words of device memory
  hipError_t acquire(hipStream_t stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    pool = &g_status_pool[dev];
    std::unique_lock<std::mutex> lk(pool->mu);
    if (!pool->base) {
      void *p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(pmklc::g_status_words));
      if (e != hipSuccess) return e;
      pool->base = static_cast<unsigned long long *>(p);
    }
    pool->cv.wait(lk, [&] { return pool->busy != ~0ull >> (64 - kStatusSlots); });
    idx = __builtin_ctzll(~pool->busy);
    pool->busy |= 1ull << idx;
    ptr = pool->base + 4 * idx;
    st = stream;
    return hipSuccess;
  }
  ~StatusSlot() {
    if (idx < 0) return;
    (void)hipStreamSynchronize(st);
    {
      std::lock_guard<std::mutex> lk(pool->mu);
      pool->busy &= ~(1ull << idx);
    }
    pool->cv.notify_one();
  }
};

// numeric path of a container: which kernel computed its probabilities
constexpr uint8_t kPathFP32Valu = 1, kPathBF16 = 2, kPathFP32Mfma = 3, kPathBF16Chip = 4, kPathTfBF16 = 5,
                  kPathTfFP32 = 6, kPathSeqBF16 = 7, kPathSeqFP32 = 8, kPathUniform = 255;
// kTf*: the Transformer DM; kSeq*: the MLP on the same launch sequence
enum Kind { kGeneric = 0, kMfmaF32 = 1, kMfmaBf16 = 2, kChipBf16 = 3, kTfF32 = 4, kTfBf16 = 5, kSeqF32 = 6, kSeqBf16 = 7 };
bool is_tf(int kind) { return kind >= kTfF32 && kind <= kSeqBf16; }   // runs the launch-sequence loop
bool is_transformer(int kind) { return kind == kTfF32 || kind == kTfBf16; }
constexpr int kHeaderBytes = 80;
// Sec. 4.2.1: the Model Selector's size bound (500 MB, read as 10^6 bytes)
constexpr uint64_t kMsBytes = 500000000ull;
// training of the static private model (Sec. 4.2.3): at most this many
// steps, seeded initialisation under seed ^ kSprmSeedXor
constexpr uint32_t kSprmSteps = 8192;
constexpr uint64_t kSprmSeedXor = 0x5350524Dull;

#define HIP_TRY(x)                                     \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return PMKLC_ERR_DEVICE;     \
  } while (0)

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------- CRC-32
// IEEE 802.3 polynomial, reflected (the zlib value), table-driven.
struct Crc32Table {
  uint32_t t[256];
  Crc32Table() {
    for (uint32_t i = 0; i < 256; i++) {
      uint32_t c = i;
      for (int b = 0; b < 8; b++) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      t[i] = c;
    }
  }
};
uint32_t crc32(const void *p, uint64_t n) {
  static const Crc32Table tab;
  const uint8_t *s = static_cast<const uint8_t *>(p);
  uint32_t c = 0xFFFFFFFFu;
  for (uint64_t i = 0; i < n; i++) c = tab.t[(c ^ s[i]) & 0xFFu] ^ (c >> 8);
  return c ^ 0xFFFFFFFFu;
}

// ------------------------------------------------------------ byte I/O
struct Writer {
  uint8_t *p;
  uint64_t cap, n = 0;
  bool over = false;
  void put(const void *src, uint64_t len) {
    if (n + len > cap) { over = true; n += len; return; }
    memcpy(p + n, src, len);
    n += len;
  }
  void le(uint64_t v, int bytes) {
    uint8_t b[8];
    for (int i = 0; i < bytes; i++) b[i] = (uint8_t)(v >> (8 * i));
    put(b, (uint64_t)bytes);
  }
  void f32(float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    le(u, 4);
  }
  void varint(uint64_t v) {
    uint8_t b[10];
    int k = 0;
    while (v >= 0x80) { b[k++] = (uint8_t)(v | 0x80); v >>= 7; }
    b[k++] = (uint8_t)v;
    put(b, (uint64_t)k);
  }
};
int varint_len(uint64_t v) {
  int k = 1;
  while (v >= 0x80) { v >>= 7; k++; }
  return k;
}
struct Reader {
  const uint8_t *p;
  uint64_t n, pos = 0;
  bool bad = false;
  uint64_t le(int bytes) {
    if (pos + (uint64_t)bytes > n) { bad = true; return 0; }
    uint64_t v = 0;
    for (int i = 0; i < bytes; i++) v |= (uint64_t)p[pos + i] << (8 * i);
    pos += (uint64_t)bytes;
    return v;
  }
  float f32() {
    uint32_t u = (uint32_t)le(4);
    float f;
    memcpy(&f, &u, 4);
    return f;
  }
  uint64_t varint() {
    uint64_t v = 0;
    for (int sh = 0; sh < 64; sh += 7) {
      if (pos >= n) { bad = true; return 0; }
      uint8_t c = p[pos++];
      v |= (uint64_t)(c & 0x7F) << sh;
      if (!(c & 0x80)) return v;
    }
    bad = true;
    return 0;
  }
};

// ------------------------------------------------------- configuration
struct Model {
  Dims d;
  LdsLayout lay;
  int nt;
  int f1 = -1;   // the global-weight kernel's F1 unit (launch_step_mfma), chosen with nt
  int kind;
  TfShape tf;   // the Transformer DM's shape (is_tf(kind))
};

pmklc_status check_cfg(const pmklc_config *c) {
  if (!c || c->struct_size != sizeof(pmklc_config)) return PMKLC_ERR_INVALID_ARG;
  if (c->s < 1 || c->k < 1 || c->k > 4 || c->s > c->k) return PMKLC_ERR_INVALID_ARG;
  if (c->t < 1 || c->t > 65535 || c->bs < 1 || c->bs > 65535 || c->embed < 1 || c->embed > 65535)
    return PMKLC_ERR_INVALID_ARG;
  if (c->n_hidden > 4) return PMKLC_ERR_INVALID_ARG;
  for (uint32_t l = 0; l < c->n_hidden; l++)
    if (c->hidden[l] < 1 || c->hidden[l] > 65535) return PMKLC_ERR_INVALID_ARG;
  if (c->optimizer > 1 || c->precision > 2 || c->schedule > 1) return PMKLC_ERR_INVALID_ARG;
  // one static model at most, always with the dynamic model (Sec. 4.2.1)
  if (c->selector != PMKLC_SEL_UNIFORM && c->selector != PMKLC_SEL_DM &&
      c->selector != (PMKLC_SEL_SPUM | PMKLC_SEL_DM) && c->selector != (PMKLC_SEL_SPRM | PMKLC_SEL_DM) &&
      c->selector != PMKLC_SEL_AUTO)
    return PMKLC_ERR_INVALID_ARG;
  if (c->smp_ppm > 1000000u) return PMKLC_ERR_INVALID_ARG;
  if (c->n_blocks < 1) return PMKLC_ERR_INVALID_ARG;
  if (c->arch > PMKLC_ARCH_TRANSFORMER) return PMKLC_ERR_INVALID_ARG;
  if (c->static_arch > PMKLC_STATIC_BIGRU) return PMKLC_ERR_INVALID_ARG;
  if (c->static_arch == PMKLC_STATIC_BIGRU) {
    // the BiGRU model mixed with the MLP dynamic model: the public one (one
    // or two layers), or the private one (one layer, trained on the input)
    if (c->arch != PMKLC_ARCH_MLP) return PMKLC_ERR_INVALID_ARG;
    if ((c->selector & PMKLC_SEL_SPRM) && c->gru_layers != 1) return PMKLC_ERR_INVALID_ARG;
    if (c->static_embed < 1 || c->gru_hidden < 1 || c->gru_layers < 1 || c->gru_layers > 2 || c->dense < 1 ||
        c->static_embed > 255 || c->gru_hidden > 255 || c->dense > 65535)
      return PMKLC_ERR_INVALID_ARG;
  }
  if (c->arch == PMKLC_ARCH_TRANSFORMER) {
    // hidden = {A, F}; no static model (Sec. 4.2.4's DM stands alone here)
    if (c->n_hidden != 2 || c->heads < 1 || c->hidden[0] % c->heads) return PMKLC_ERR_INVALID_ARG;
    if (c->selector & (PMKLC_SEL_SPUM | PMKLC_SEL_SPRM)) return PMKLC_ERR_INVALID_ARG;
  }
  return PMKLC_OK;
}

uint64_t param_count(uint32_t k, uint32_t t, uint32_t E, uint32_t nh, const uint32_t *hidden, uint32_t arch = 0) {
  if (arch == PMKLC_ARCH_TRANSFORMER) {
    const uint64_t V = 1ull << (2 * k), A = hidden[0], F = hidden[1];
    return V * E + (uint64_t)t * E + E * 3 * A + 3 * A + A * A + A + A * F + F + F * A + A + A * V + V;
  }
  uint64_t V = 1ull << (2 * k);
  uint64_t prev = (uint64_t)t * E, n = V * E;
  for (uint32_t l = 0; l < nh; l++) { n += prev * hidden[l] + hidden[l]; prev = hidden[l]; }
  n += prev * V + V;
  return n;
}

// parameters of the BiGRU static model a configuration names
uint64_t bigru_param_count(const pmklc_config &c) {
  const uint64_t V = 1ull << (2 * c.k), E = c.static_embed, h = c.gru_hidden, gd = c.dense;
  uint64_t n = V * E;
  for (uint32_t l = 0; l < c.gru_layers; l++) n += 2 * (3 * h * (l == 0 ? E : 2 * h) + 3 * h * h + 6 * h);
  return n + 2 * h * gd + gd + gd * V + V;
}

// Shape and parameter offsets of the model (no kernel-support checks).
pmklc_status fill_dims(uint32_t k, uint32_t t, uint32_t bs, uint32_t E, uint32_t nh, const uint32_t *hidden,
                       uint32_t selector, uint32_t opt, float lr, float b1, float b2, float eps, Dims &d) {
  memset(&d, 0, sizeof d);
  if (nh > 2) return PMKLC_ERR_UNSUPPORTED;
  d.V = 1 << (2 * k);
  d.E = (int)E;
  d.t = (int)t;
  d.D = (int)(t * E);
  d.bs = (int)bs;
  d.nh = (int)nh;
  d.model_on = (selector & PMKLC_SEL_DM) ? 1 : 0;
  d.static_on = (selector & (PMKLC_SEL_SPUM | PMKLC_SEL_SPRM)) ? 1 : 0;
  d.optimizer = (int)opt;
  d.lr = lr; d.b1 = b1; d.b2 = b2; d.eps = eps;
  if (!d.model_on) d.nh = 0;   // uniform coding needs no model
  if ((uint64_t)t * E > (1u << 20) || E >= 4096) return PMKLC_ERR_UNSUPPORTED;
  d.dim[0] = d.D;
  d.Emag = E ? (uint32_t)(((1ull << 32) + E - 1) / E) : 0;
  for (int l = 0; l < d.nh; l++) { d.H[l] = (int)hidden[l]; d.dim[l + 1] = (int)hidden[l]; }
  d.dim[d.nh + 1] = d.V;
  uint64_t off = 0;
  d.off_emb = 0;
  off += (uint64_t)d.V * E;
  for (int l = 0; l <= d.nh; l++) {
    d.off_W[l] = (int)off;
    off += (uint64_t)d.dim[l] * d.dim[l + 1];
    d.off_b[l] = (int)off;
    off += (uint64_t)d.dim[l + 1];
  }
  if (off > (1ull << 30)) return PMKLC_ERR_UNSUPPORTED;
  d.P = (int)off;
  d.stride = (int)align_up(off + 1, 64);
  return PMKLC_OK;
}

// Shape + LDS plan of the step kernel; UNSUPPORTED when this build's kernels
// cannot hold it (tile multiples of 4, LDS <= 160 KB, at most two hidden
// layers).
// seq: the launch-sequence form of the MLP: -1 where the persistent kernels
// cannot hold a BF16 model (or with PMKLC_SEQ_MLP=1 in the environment for
// FP32), 1 always (decoding a container it made), 0 never
pmklc_status make_model(uint32_t s, uint32_t k, uint32_t t, uint32_t bs, uint32_t E, uint32_t nh,
                        const uint32_t *hidden, uint32_t selector, uint32_t opt, float lr, float b1, float b2,
                        float eps, uint32_t precision, Model &m, bool allow_chip, int seq) {
  (void)s;
  Dims &d = m.d;
  pmklc_status rc = fill_dims(k, t, bs, E, nh, hidden, selector, opt, lr, b1, b2, eps, d);
  if (rc) return rc;
  auto make_seq = [&]() -> pmklc_status {
    if (!d.model_on || d.static_on || precision == PMKLC_FP32_VALU || !mlp_seq_shape(d, m.tf))
      return PMKLC_ERR_UNSUPPORTED;
    m.tf.bf16 = precision == PMKLC_BF16;
    memset(&m.lay, 0, sizeof m.lay);
    m.kind = m.tf.bf16 ? kSeqBf16 : kSeqF32;
    m.nt = 256;
    return PMKLC_OK;
  };
  const char *env_seq = getenv("PMKLC_SEQ_MLP");
  if (seq == 1 || (seq < 0 && precision == PMKLC_FP32 && env_seq && env_seq[0] == '1' && d.model_on &&
                   !d.static_on))
    return make_seq();
  if (d.model_on) {
    if (E % 4 || bs % 4 || d.V % 4) return PMKLC_ERR_UNSUPPORTED;
    for (uint32_t l = 0; l < nh; l++) if (hidden[l] % 4) return PMKLC_ERR_UNSUPPORTED;
  }

  d.VS = d.V + 4;
  d.ES = d.E + 1;
  d.EP = d.E + 4;
  d.HP = d.H[0] + 4;
  d.CH = 32;   // staging width in steps (a power of two)
  int rs = 1;
  while (rs < d.t + d.CH) rs <<= 1;
  d.RS = rs;
  // LDS plan; when the activations do not fit, they move to a global slab
  // per workgroup (act/dh offsets then count floats in that slab)
  LdsLayout &L = m.lay;
  int hmax = 0;
  for (int l = 0; l < d.nh; l++) hmax = std::max(hmax, d.H[l]);
  for (int glob = 0; glob < 2; glob++) {
    memset(&L, 0, sizeof L);
    uint64_t o = 0, g = 0;
    auto take = [&](uint64_t bytes) { uint64_t at = o; o = align_up(o + bytes, 16); return (int)at; };
    auto act = [&](uint64_t bytes) {
      if (!glob) return take(bytes);
      uint64_t at = g;
      g = align_up(g + bytes / 4, 64);
      return (int)at;
    };
    L.emb = take(4ull * d.V * d.EP);
    L.embs = take(d.static_on ? 4ull * d.V * d.EP : 0);
    L.ring = take((uint64_t)bs * d.RS);
    L.act[0] = act(d.nh >= 1 ? 4ull * bs * d.HP : 0);
    L.act[1] = act(d.nh >= 2 ? 4ull * bs * d.H[1] : 0);
    L.lm = take(4ull * bs * d.VS);
    L.lu = take(d.static_on ? 4ull * bs * d.VS : 0);
    L.cdf = take(4ull * bs * (d.V + 1));
    L.tgt = take(bs);
    L.dh[0] = act(d.nh >= 1 ? 4ull * bs * (hmax + 4) : 0);
    L.dh[1] = act(d.nh >= 2 ? 4ull * bs * hmax : 0);
    L.demb = take(8ull * d.V * d.ES);
    L.misc = take(4ull * bs + 64);
    L.cst = take(48ull * bs);
    {
      // BF16 copy of dpre^T for the fused backward (one hidden layer)
      const uint64_t need = d.nh == 1 ? 2ull * bs * d.H[0] : 0;
      const uint64_t cdf_bytes = 4ull * bs * (d.V + 1);
      L.dpt = need <= cdf_bytes ? L.cdf : take(need);
      // dpre in BF16 as B3's B fragments (BF16 kernel only): in the static
      // logits when they are there and large enough, else its own region if
      // the total still fits, else absent (-1: B3 reads the FP32 dpre)
      const uint64_t lu_bytes = d.static_on ? 4ull * bs * d.VS : 0;
      if (precision != PMKLC_BF16 || need == 0) L.dpb = -1;
      else if (need <= lu_bytes) L.dpb = L.lu;
      else if (o + need <= 160 * 1024) L.dpb = take(need);
      else L.dpb = -1;
    }
    L.total = (int)o;
    L.act_global = glob;
    L.act_slot = (int)g;
    if (o <= 160 * 1024) break;
    if (glob) return (seq < 0 && precision == PMKLC_BF16) ? make_seq() : PMKLC_ERR_UNSUPPORTED;
  }
  m.nt = bs <= 256 ? 256 : 512;
  if (bs > 512) return PMKLC_ERR_UNSUPPORTED;
  // matrix-core kernel: one hidden layer, tile-friendly shapes
  const bool mfma_ok = d.model_on && !L.act_global && d.nh == 1 && bs % 32 == 0 && bs <= 128 && d.H[0] % 32 == 0 && d.V % 32 == 0 &&
                       E % 8 == 0 && E < 4096 && d.D % 32 == 0;
  m.kind = kGeneric;
  if (precision == PMKLC_BF16) {
    if (d.model_on && !mfma_ok) return seq < 0 ? make_seq() : PMKLC_ERR_UNSUPPORTED;
    m.kind = kMfmaBf16;
  } else if (precision == PMKLC_FP32 && mfma_ok) {
    m.kind = kMfmaF32;
  }
  if (m.kind != kGeneric) m.nt = 512;
  // BF16 with a shape the on-chip kernel is compiled for: its extra LDS
  // regions (weights and gradient partials), when they fit
  if (m.kind == kMfmaBf16 && allow_chip && L.dpb >= 0 && chip_supports(d)) {
    LdsLayout C = L;
    uint64_t o = (uint64_t)C.total;
    auto take = [&](uint64_t bytes) { uint64_t at = o; o = align_up(o + bytes, 16); return (int)at; };
    C.w1c = take(2ull * d.D * d.H[0]);
    C.w2t = take(4ull * d.V * (d.H[0] + 4));
    C.bias = take(4ull * (d.H[0] + d.V));
    C.gb = take(4ull * (d.H[0] + d.V));
    C.eg = take(4ull * 8 * d.V * d.E);
    C.embh = take(2ull * d.V * (d.E + 8));
    if (o <= 160 * 1024) {
      C.total = (int)o;
      L = C;
      m.kind = kChipBf16;
    }
  }
  return PMKLC_OK;
}

// the on-chip kernel is the BF16 default for the shapes it has; PMKLC_NO_CHIP=1
// selects the global-weight BF16 kernel instead (a different numeric path)
bool chip_default() {
  const char *e = getenv("PMKLC_NO_CHIP");
  return !(e && e[0] == '1');
}

// The Transformer DM (arch 1, dynamic model on): its shape, and the Dims
// fields the shared host code reads (parameter slab, optimiser, sizes).
pmklc_status make_tf_model(const pmklc_config *c, Model &m) {
  memset(&m, 0, sizeof m);
  TfShape &s = m.tf;
  if (!tf_shape((int)c->k, (int)c->t, (int)c->embed, (int)c->hidden[0], (int)c->hidden[1], (int)c->heads, s))
    return PMKLC_ERR_UNSUPPORTED;
  if (c->precision == PMKLC_FP32_VALU || c->schedule != PMKLC_BATCHED || c->smp_ppm > 0 || c->bs > 1024 ||
      (uint64_t)c->bs * c->t > 65536)
    return PMKLC_ERR_UNSUPPORTED;
  s.bs = (int)c->bs;
  s.optimizer = (int)c->optimizer;
  s.lr = c->lr; s.b1 = c->beta1; s.b2 = c->beta2; s.eps = c->eps;
  s.bf16 = c->precision == PMKLC_BF16;
  Dims &d = m.d;
  d.V = s.V; d.E = s.E; d.t = s.t; d.bs = s.bs; d.nh = 2;
  d.H[0] = s.A; d.H[1] = s.F;
  d.P = (int)s.P;
  d.stride = (int)s.stride;
  d.model_on = 1;
  d.optimizer = s.optimizer;
  d.lr = s.lr; d.b1 = s.b1; d.b2 = s.b2; d.eps = s.eps;
  d.CH = 32;
  m.kind = s.bf16 ? kTfBf16 : kTfF32;
  m.nt = 256;
  return PMKLC_OK;
}

pmklc_status make_model(const pmklc_config *c, Model &m, bool allow_chip, int seq = -1) {
  if (c->arch == PMKLC_ARCH_TRANSFORMER && (c->selector & PMKLC_SEL_DM)) return make_tf_model(c, m);
  if (c->static_arch == PMKLC_STATIC_BIGRU && (c->selector & PMKLC_SEL_DM) &&
      (c->selector & (PMKLC_SEL_SPUM | PMKLC_SEL_SPRM))) {
    // the MLP on the launch-sequence loop, the BiGRU model beside it
    pmklc_status rc = make_model(c->s, c->k, c->t, c->bs, c->embed, c->n_hidden, c->hidden, PMKLC_SEL_DM,
                                 c->optimizer, c->lr, c->beta1, c->beta2, c->eps, c->precision, m, false, 1);
    if (rc) return rc;
    if (c->schedule != PMKLC_BATCHED || c->smp_ppm > 0) return PMKLC_ERR_UNSUPPORTED;
    if (!bigru_shape((int)c->static_embed, (int)c->gru_hidden, (int)c->gru_layers, (int)c->dense, m.tf))
      return PMKLC_ERR_UNSUPPORTED;
    if ((c->selector & PMKLC_SEL_SPRM) && !gru_train_supported(m.tf)) return PMKLC_ERR_UNSUPPORTED;
    return PMKLC_OK;
  }
  pmklc_status rc = make_model(c->s, c->k, c->t, c->bs, c->embed, c->arch == PMKLC_ARCH_TRANSFORMER ? 0 : c->n_hidden,
                               c->hidden, c->selector, c->optimizer, c->lr, c->beta1, c->beta2, c->eps, c->precision,
                               m, allow_chip, seq);
  if (rc == PMKLC_OK && is_tf(m.kind)) {
    if (c->schedule != PMKLC_BATCHED || c->smp_ppm > 0) return PMKLC_ERR_UNSUPPORTED;
  }
  return rc;
}
pmklc_status make_model(const pmklc_config *c, Model &m) { return make_model(c, m, chip_default()); }

// the static public model: present, and its parameter count
bool bigru_on(const Model &m) { return is_tf(m.kind) && m.tf.sarch == 1; }
bool has_static(const Model &m) { return m.d.static_on || bigru_on(m); }
uint64_t static_count(const Model &m) { return bigru_on(m) ? (uint64_t)m.tf.sP : (uint64_t)m.d.P; }

// Sec. 4.2.1, the Model Selector: the configuration with S chosen for an
// input of n bytes when the caller asked for the selector's choice (the
// private static model above the size bound; else the public one when the
// caller supplies it; else the dynamic model alone).
pmklc_config ms_resolve(const pmklc_config *c, uint64_t n) {
  pmklc_config r = *c;
  if (c->selector == PMKLC_SEL_AUTO) {
    const uint64_t bound = c->ms_threshold ? c->ms_threshold : kMsBytes;
    r.selector = n > bound ? (PMKLC_SEL_SPRM | PMKLC_SEL_DM)
                 : c->static_host ? (PMKLC_SEL_SPUM | PMKLC_SEL_DM) : PMKLC_SEL_DM;
  }
  return r;
}

// -------------------------------------------------------------- planning
struct Plan {
  std::vector<uint64_t> raw_len, raw_off;
  std::vector<int32_t> pred;       // SMP predecessor or -1
  std::vector<uint64_t> file_blocks;
};

pmklc_status plan_blocks(uint64_t n, uint32_t n_blocks, const uint64_t *block_len, uint32_t n_files,
                         const uint64_t *file_blocks, bool smp, Plan &p) {
  p.raw_len.resize(n_blocks);
  p.raw_off.resize(n_blocks);
  uint64_t off = 0;
  for (uint32_t b = 0; b < n_blocks; b++) {
    uint64_t len = block_len ? block_len[b] : (b + 1 == n_blocks ? n - (n / n_blocks) * (n_blocks - 1) : n / n_blocks);
    if (len > 0xFFFFFFFFull) return PMKLC_ERR_INVALID_ARG;   // run tables are 32-bit per block
    p.raw_off[b] = off;
    p.raw_len[b] = len;
    off += len;
  }
  if (off != n) return PMKLC_ERR_INVALID_ARG;
  if (file_blocks && n_files > 0) p.file_blocks.assign(file_blocks, file_blocks + n_files);
  else p.file_blocks.assign(1, n_blocks);
  uint64_t tot = 0;
  for (uint64_t v : p.file_blocks) tot += v;
  if (tot != n_blocks) return PMKLC_ERR_INVALID_ARG;
  p.pred.assign(n_blocks, -1);
  uint64_t b = 0;
  for (uint64_t fb : p.file_blocks) {
    for (uint64_t q = 0; q < fb; q++, b++)
      if (smp && q > 0) p.pred[b] = (int32_t)(b - 1);
  }
  return PMKLC_OK;
}

uint64_t smp_steps(uint32_t ppm, uint64_t L) { return (uint64_t)(((unsigned __int128)ppm * L + 999999u) / 1000000u); }
uint64_t tokens_of(uint64_t nb, uint32_t s, uint32_t k) { return nb >= k ? (nb - k) / s + 1 : 0; }
uint32_t slot_words_for(uint64_t L) { return (uint32_t)((17 * L + 2 + 31) / 32 + 1); }

// ------------------------------------------------------------ workspace
struct Arena {
  uint8_t *base;
  uint64_t cap, used = 0;
  bool over = false;
  template <class T>
  T *take(uint64_t count) {
    uint64_t at = align_up(used, 256);
    used = at + align_up(count * sizeof(T), 256);
    if (used > cap) over = true;
    return base ? reinterpret_cast<T *>(base + at) : nullptr;
  }
};

struct Work {
  uint64_t *chunk_block, *chunk_run0;
  ChunkStat *stats;
  SeqBlock *seq;
  BlockDesc *desc;
  uint32_t *run_start, *run_len, *run_sp, *run_cum;
  uint8_t *tok, *extras;
  float *params, *adam_m, *adam_v, *init, *stat, *snap;
  int *snap_flag, *ctr;   // ctr[0] queue, ctr[1] err
  uint32_t *progress;     // steps done per block (model-passing waits)
  int *order;             // queue order of the blocks
  uint32_t *slots, *seg_bits, *seg_words;
  uint64_t *seg_src, *seg_dst;
  uint32_t *seg_bytes;
  uint8_t *staging;
  StepArgs *args;         // device copies of the step-kernel arguments (one per launch)
  float *act;             // activation slabs (models whose activations exceed the LDS)
  uint16_t *w1f, *s1f;
  unsigned long long *phase;   // [16] phase clock of block 0
  uint8_t *tune;          // the autotuner's trial block (inside the caller's workspace)
  uint64_t tune_bytes;
  // the Transformer DM's loop: state, per-slot descriptors and buffers
  TfState *tf_state;
  TfSlot *tf_desc;
  float *tf_f;
  float *tf_stat;         // the BiGRU static model's parameters
};

struct Sizes {
  uint64_t n_chunks, runs, tokens, slot_words, staging;
};

uint64_t trial_bytes(const Model &m);

// trial: the autotuner's own one-block layout (which holds no trial region)
void layout(Arena &A, const Model &m, uint32_t n_blocks, const Sizes &z, bool adam, bool smp, Work &w,
            bool trial = false) {
  const uint64_t stride = (uint64_t)m.d.stride;
  w.ctr = A.take<int>(64);
  w.chunk_block = A.take<uint64_t>(z.n_chunks + 1);
  w.chunk_run0 = A.take<uint64_t>(z.n_chunks + 1);
  w.stats = A.take<ChunkStat>(z.n_chunks + 1);
  w.seq = A.take<SeqBlock>(n_blocks);
  w.desc = A.take<BlockDesc>(n_blocks);
  w.run_start = A.take<uint32_t>(z.runs + 1);
  w.run_len = A.take<uint32_t>(z.runs + 1);
  w.run_sp = A.take<uint32_t>(z.runs + 1);
  w.run_cum = A.take<uint32_t>(z.runs + 1);
  w.tok = A.take<uint8_t>(z.tokens + 16);
  w.extras = A.take<uint8_t>((uint64_t)n_blocks * ((uint64_t)m.d.bs + 8));
  w.params = A.take<float>((uint64_t)n_blocks * stride);
  w.adam_m = adam ? A.take<float>((uint64_t)n_blocks * stride) : nullptr;
  w.adam_v = adam ? A.take<float>((uint64_t)n_blocks * stride) : nullptr;
  w.init = A.take<float>(stride);
  w.stat = m.d.static_on ? A.take<float>(stride) : nullptr;
  w.snap = smp ? A.take<float>((uint64_t)n_blocks * stride) : nullptr;
  w.snap_flag = A.take<int>(n_blocks);
  w.progress = A.take<uint32_t>(n_blocks);
  w.order = A.take<int>(n_blocks);
  w.slots = A.take<uint32_t>(z.slot_words + 1);
  w.seg_bits = A.take<uint32_t>((uint64_t)n_blocks * m.d.bs);
  w.seg_words = A.take<uint32_t>((uint64_t)n_blocks * m.d.bs);
  w.seg_src = A.take<uint64_t>((uint64_t)n_blocks * m.d.bs);
  w.seg_dst = A.take<uint64_t>((uint64_t)n_blocks * m.d.bs);
  w.seg_bytes = A.take<uint32_t>((uint64_t)n_blocks * m.d.bs);
  w.staging = A.take<uint8_t>(z.staging + 16);
  w.args = A.take<StepArgs>((uint64_t)n_blocks + 1);
  w.act = m.lay.act_global ? A.take<float>((uint64_t)std::min<uint32_t>(n_blocks, kMaxGrid) * m.lay.act_slot) : nullptr;
  w.phase = A.take<unsigned long long>(16);
  const uint64_t w1n = m.kind == kMfmaBf16 ? (uint64_t)m.d.D * m.d.H[0] : 0;
  w.w1f = w1n ? A.take<uint16_t>((uint64_t)std::min<uint32_t>(n_blocks, kMaxGrid) * w1n) : nullptr;
  w.s1f = (w1n && m.d.static_on) ? A.take<uint16_t>(w1n) : nullptr;
  w.tune_bytes = (!trial && m.d.model_on && !is_tf(m.kind)) ? trial_bytes(m) : 0;
  w.tune = w.tune_bytes ? A.take<uint8_t>(w.tune_bytes) : nullptr;
  w.tf_state = nullptr;
  w.tf_desc = nullptr;
  w.tf_f = nullptr;
  w.tf_stat = nullptr;
  if (is_tf(m.kind)) {
    TfBufs tb;
    w.tf_state = A.take<TfState>(1);
    w.tf_desc = A.take<TfSlot>(n_blocks);
    w.tf_f = A.take<float>(tf_bufs_carve(m.tf, (int)n_blocks, nullptr, tb));
    w.tf_stat = m.tf.sarch ? A.take<float>((uint64_t)m.tf.sP) : nullptr;
  }
}

// The autotuner's trial: one synthetic block of t + 64 steps.
Sizes trial_sizes(const Model &m) {
  const uint32_t L = (uint32_t)m.d.t + 64;
  Sizes z{};
  z.tokens = (uint64_t)L * m.d.bs;
  z.slot_words = (uint64_t)slot_words_for(L) * m.d.bs;
  return z;
}
uint64_t trial_bytes(const Model &m) {
  Arena A{nullptr, ~0ull};
  Work w;
  layout(A, m, 1, trial_sizes(m), m.d.optimizer == 1, false, w, true);
  return A.used + 256;
}

// The static private model's training run (Sec. 4.2.3): the dynamic model
// alone (its own kernel choice) on one block of bs segments of at most
// Lp_max steps, laid out after the compression's own workspace.
struct SprmRun {
  Model m;
  Work w;
  uint32_t Lp_max = 0;
  // the BiGRU private model: its training block, scratch, Adam moments
  bool gru = false;
  uint8_t *gtok = nullptr;
  float *gbuf = nullptr, *gm = nullptr, *gv = nullptr;
};
pmklc_status sprm_layout(Arena &A, const pmklc_config *c, uint64_t tokens_max, SprmRun &r, const Model &cm) {
  if (bigru_on(cm)) {
    r.gru = true;
    r.Lp_max = (uint32_t)std::min<uint64_t>(tokens_max / c->bs, kSprmSteps);
    uint64_t ps;
    int nwg;
    r.gtok = A.take<uint8_t>((uint64_t)r.Lp_max * c->bs + 1);
    r.gbuf = A.take<float>(gru_train_floats(cm.tf, ps, nwg));
    if (c->optimizer == PMKLC_ADAM) {
      r.gm = A.take<float>((uint64_t)cm.tf.sP);
      r.gv = A.take<float>((uint64_t)cm.tf.sP);
    }
    return PMKLC_OK;
  }
  pmklc_config cd = *c;
  cd.selector = PMKLC_SEL_DM;
  pmklc_status rc = make_model(&cd, r.m);
  if (rc) return rc;
  r.Lp_max = (uint32_t)std::min<uint64_t>(tokens_max / c->bs, kSprmSteps);
  Sizes z{};
  z.tokens = (uint64_t)r.Lp_max * c->bs;
  z.slot_words = (uint64_t)slot_words_for(r.Lp_max) * c->bs;
  layout(A, r.m, 1, z, c->optimizer == PMKLC_ADAM, false, r.w, true);
  return PMKLC_OK;
}

hipError_t launch_kind(const Model &m, const StepArgs &a, const StepArgs *a_dev, int grid, int nt, hipStream_t st) {
  if (m.kind == kGeneric) return launch_step(a, grid, nt, st);
  if (m.kind == kChipBf16) return launch_step_chip(a, a_dev, grid, st);
  return launch_step_mfma(a, a_dev, grid, m.kind == kMfmaBf16, nt, m.f1, st);
}

// One synthetic block of t + 64 steps (constant tokens) in encode mode,
// best of two runs, with the candidate width, in the trial region of the
// caller's workspace (region: trial_bytes(m) bytes).
hipError_t time_candidate(Model m, int nt, int f1, uint8_t *region, uint64_t cap, hipStream_t st, float *ms) {
  m.nt = nt;
  m.f1 = f1;
  const uint32_t L = (uint32_t)m.d.t + 64;
  const Sizes z = trial_sizes(m);
  Work w;
  Arena B{reinterpret_cast<uint8_t *>(align_up(reinterpret_cast<uintptr_t>(region), 256)), cap - 256};
  if (!region || cap < 256) return hipErrorInvalidValue;
  layout(B, m, 1, z, m.d.optimizer == 1, false, w, true);
  if (B.over) return hipErrorInvalidValue;
  hipError_t e = hipSuccess;
  BlockDesc bd{0, 0, L, slot_words_for(L), 0, -1, 0, 0};
  StepArgs a;
  memset(&a, 0, sizeof a);
  a.d = m.d;
  a.lay = m.lay;
  a.n_blocks = 1;
  a.blocks = w.desc;
  a.tokens = w.tok;
  a.params = w.params;
  a.adam_m = w.adam_m;
  a.adam_v = w.adam_v;
  a.init = w.init;
  a.stat = m.d.static_on ? w.init : nullptr;
  a.snap_flag = w.snap_flag;
  a.progress = w.progress;
  a.queue = w.ctr;
  a.err = w.ctr + 1;
  a.slots = w.slots;
  a.seg_bits = w.seg_bits;
  a.seg_words = w.seg_words;
  a.act_scratch = w.act;
  a.spin_limit = 1;
  a.w1f = w.w1f;
  a.s1f = w.s1f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = 1e30f;
  if (e == hipSuccess) e = hipMemcpyAsync(w.desc, &bd, sizeof bd, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(w.tok, 1, z.tokens, st);
  if (e == hipSuccess) e = launch_init_params(m.d, 1, w.init, st);
  if (e == hipSuccess && w.s1f) e = launch_w1_frag(w.init + m.d.off_W[0], m.d.D, m.d.H[0], w.s1f, st);
  if (e == hipSuccess) e = hipMemcpyAsync(w.args, &a, sizeof a, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {
    e = hipMemsetAsync(w.ctr, 0, 64 * sizeof(int), st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess)
      e = launch_kind(m, a, w.args, 1, nt, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e == hipSuccess) best = std::min(best, t);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  *ms = best;
  return e;
}

template <class T>
hipError_t h2d(T *dst, const std::vector<T> &v, hipStream_t st) {
  if (v.empty()) return hipSuccess;
  return hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st);
}
template <class T>
hipError_t d2h(std::vector<T> &v, const T *src, uint64_t count, hipStream_t st) {
  v.resize(count);
  if (!count) return hipSuccess;
  return hipMemcpyAsync(v.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, st);
}

uint8_t path_of(uint32_t selector, int kind) {
  if (!(selector & PMKLC_SEL_DM)) return kPathUniform;
  if (is_transformer(kind)) return kind == kTfBf16 ? kPathTfBF16 : kPathTfFP32;
  if (is_tf(kind)) return kind == kSeqBf16 ? kPathSeqBF16 : kPathSeqFP32;
  return kind == kChipBf16 ? kPathBF16Chip : kind == kMfmaBf16 ? kPathBF16 : kind == kMfmaF32 ? kPathFP32Mfma
                                                                                       : kPathFP32Valu;
}

void write_header(Writer &o, const pmklc_config *c, uint8_t path, uint32_t scrc, uint64_t n, uint32_t n_files) {
  o.put("PMKC", 4);
  o.le(1, 1);
  o.le(path, 1);
  o.le(c->s, 1);
  o.le(c->k, 1);
  o.le(c->t, 2);
  o.le(c->bs, 2);
  o.le(c->embed, 2);
  o.le(c->n_hidden, 1);
  o.le(c->optimizer, 1);
  for (uint32_t l = 0; l < 4; l++) o.le(l < c->n_hidden ? c->hidden[l] : 0, 2);
  o.f32(c->lr);
  o.f32(c->beta1);
  o.f32(c->beta2);
  o.f32(c->eps);
  o.le(c->selector, 1);
  o.le(c->arch, 1);
  o.le(c->arch == PMKLC_ARCH_TRANSFORMER ? c->heads : 0, 1);
  const bool gru = c->static_arch == PMKLC_STATIC_BIGRU && (c->selector & (PMKLC_SEL_SPUM | PMKLC_SEL_SPRM));
  o.le(gru ? 1 | (c->gru_layers << 4) : 0, 1);
  o.le(c->smp_ppm, 4);
  o.le(c->seed, 8);
  o.le(scrc, 4);
  o.le(gru ? c->static_embed : 0, 1);
  o.le(gru ? c->gru_hidden : 0, 1);
  o.le(gru ? c->dense : 0, 2);
  o.le(n, 8);
  o.le(c->n_blocks, 4);
  o.le(n_files, 4);
}

// MSB-first bit packer for the per-block extras
struct BitPack {
  std::vector<uint8_t> b;
  uint64_t nbits = 0;
  void put(uint32_t v, int n) {
    for (int i = n - 1; i >= 0; i--) {
      if ((nbits >> 3) >= b.size()) b.push_back(0);
      if ((v >> i) & 1u) b[nbits >> 3] |= (uint8_t)(0x80u >> (nbits & 7));
      nbits++;
    }
  }
};
uint32_t get_bits(const uint8_t *p, uint64_t &bit, int n) {
  uint32_t v = 0;
  for (int i = 0; i < n; i++, bit++) v = (v << 1) | ((p[bit >> 3] >> (7 - (bit & 7))) & 1u);
  return v;
}

void fill_blockdesc(const Model &m, const std::vector<SeqBlock> &sb, const Plan &p, uint32_t smp_ppm,
                    std::vector<BlockDesc> &bd, uint64_t &slot_total) {
  const uint32_t nb = (uint32_t)sb.size();
  bd.resize(nb);
  slot_total = 0;
  std::vector<int> has_succ(nb, 0);
  for (uint32_t b = 0; b < nb; b++) if (p.pred[b] >= 0) has_succ[p.pred[b]] = 1;
  for (uint32_t b = 0; b < nb; b++) {
    BlockDesc &d = bd[b];
    d.tok_off = sb[b].tok_off;
    d.L = (uint32_t)sb[b].L;
    d.slot_words = slot_words_for(sb[b].L);
    d.slot_off = slot_total;
    slot_total += (uint64_t)d.slot_words * (uint64_t)m.d.bs;
    d.S = (uint32_t)smp_steps(smp_ppm, sb[b].L);
    d.pred = p.pred[b];
    d.has_snap = has_succ[b];
    d.pad = 0;
  }
}

thread_local pmklc_timing g_last = {};

// ------------------------------------------------------------- autotuner
// Picks the step kernel's launch shape for a model shape by timing a short
// synthetic block with each candidate, and caches the choice for the
// process: the threads per workgroup (4 or 8 waves, which also fix the
// fused B3/B4 chunking, HCH and TB) and, for the global-weight matrix-core
// kernel with hidden widths in multiples of 64, the F1 unit (four or two
// hidden tiles per gathered context fragment). No choice changes a value:
// every output element is computed by one thread or wave in a fixed order
// whatever the launch shape. PMKLC_NT=256|512 and PMKLC_F1=4|2 force them.
struct TuneEntry {
  int kind, bs, H0, H1, V, E, t, nh, stat, opt;
  int nt, f1;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

// tune = false (the no-allocation entry point): no trial runs, which would
// create timing events; the cached choice, else the widest candidate.
int choose_nt(Model &m, const Work &w, hipStream_t st, bool tune = true) {
  const char *env = getenv("PMKLC_NT"), *env_f1 = getenv("PMKLC_F1");
  std::vector<int> nts;
  if (m.kind == kGeneric) {
    nts = {256};
    if (m.d.bs <= 512) nts.push_back(512);
  } else if (m.kind == kChipBf16) {
    nts = {512};   // its register-resident weights are laid out for 8 waves
  } else {
    nts = {256, 512};
  }
  if (m.d.bs > 256) nts.erase(std::remove(nts.begin(), nts.end(), 256), nts.end());
  if (env) {
    const int f = atoi(env);
    if (std::find(nts.begin(), nts.end(), f) != nts.end()) nts = {f};
  }
  // the F1 unit: a choice only for the global-weight kernel at hidden widths
  // in multiples of 64 (four hidden tiles per unit need them)
  std::vector<int> f1s = {-1};
  if ((m.kind == kMfmaBf16 || m.kind == kMfmaF32) && (m.d.H[0] / 16) % 4 == 0) {
    f1s = {1, 0};
    if (env_f1) f1s = {atoi(env_f1) == 2 ? 0 : 1};
  }
  m.f1 = f1s[0];
  if ((nts.size() == 1 && f1s.size() == 1) || !m.d.model_on) return nts.back();
  TuneEntry key{m.kind, m.d.bs, m.d.H[0], m.d.H[1], m.d.V, m.d.E, m.d.t, m.d.nh, m.d.static_on, m.d.optimizer, 0, 0};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (const TuneEntry &e : g_tune)
    if (e.kind == key.kind && e.bs == key.bs && e.H0 == key.H0 && e.H1 == key.H1 && e.V == key.V && e.E == key.E &&
        e.t == key.t && e.nh == key.nh && e.stat == key.stat && e.opt == key.opt &&
        std::find(nts.begin(), nts.end(), e.nt) != nts.end() && std::find(f1s.begin(), f1s.end(), e.f1) != f1s.end()) {
      m.f1 = e.f1;
      return e.nt;
    }
  if (!tune) return nts.back();
  int best = nts.back(), best_f1 = f1s[0];
  float best_ms = 1e30f;
  for (int nt : nts)
    for (int f1 : f1s) {
      float ms = 0.0f;
      if (time_candidate(m, nt, f1, w.tune, w.tune_bytes, st, &ms) != hipSuccess) continue;
      if (ms < best_ms) { best_ms = ms; best = nt; best_f1 = f1; }
    }
  key.nt = best;
  key.f1 = best_f1;
  g_tune.push_back(key);
  m.f1 = best_f1;
  return best;
}

struct StepTimer {
  hipEvent_t a = nullptr, b = nullptr;
  ~StepTimer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

void count_work(const Model &m, const std::vector<BlockDesc> &bd, pmklc_timing &t) {
  t.model_rows = t.coded_tokens = t.max_steps = 0;
  for (const BlockDesc &d : bd) {
    t.coded_tokens += (uint64_t)d.L * m.d.bs;
    if (m.d.model_on && d.L > (uint32_t)m.d.t) t.model_rows += (uint64_t)(d.L - m.d.t) * m.d.bs;
    t.max_steps = std::max<uint64_t>(t.max_steps, d.L);
  }
}

// Queue order of the persistent kernel: longest critical path first, where a
// block's path is its own steps or, with a successor in its file, the steps
// up to its snapshot plus the successor's path.  A predecessor's path is at
// least its successor's, and ties keep block order, so a block is never
// dequeued before the block it waits on.
std::vector<int> queue_order(const std::vector<BlockDesc> &bd) {
  const size_t n = bd.size();
  std::vector<int> succ(n, -1), ord(n);
  std::vector<uint64_t> key(n, 0);
  for (size_t b = 0; b < n; b++) if (bd[b].pred >= 0) succ[bd[b].pred] = (int)b;
  for (size_t q = n; q-- > 0;) {
    key[q] = bd[q].L;
    if (succ[q] >= 0) key[q] = std::max<uint64_t>(key[q], (uint64_t)bd[q].S + key[succ[q]]);
  }
  for (size_t b = 0; b < n; b++) ord[b] = (int)b;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key[x] > key[y]; });
  return ord;
}

// params_out: when given, block 0 writes its final parameters (+ a) there
pmklc_status run_step(Model m, const Work &w, int mode, const std::vector<BlockDesc> &bd, uint32_t schedule,
                      hipStream_t st, StepTimer *tm = nullptr, bool tune = true, float *params_out = nullptr) {
  m.nt = choose_nt(m, w, st, tune);
  g_last.threads = (uint32_t)m.nt;
  g_last.f1_units = m.kind == kMfmaBf16 || m.kind == kMfmaF32 ? ((m.d.H[0] / 16) % 4 == 0 && m.f1 != 0 ? 4u : 2u) : 0u;
  StepArgs a;
  memset(&a, 0, sizeof a);
  a.d = m.d;
  a.lay = m.lay;
  a.mode = mode;
  a.n_blocks = (int)bd.size();
  a.blocks = w.desc;
  a.tokens = w.tok;
  a.params = w.params;
  a.adam_m = w.adam_m;
  a.adam_v = w.adam_v;
  a.init = w.init;
  a.stat = w.stat;
  a.snap = w.snap;
  a.snap_flag = w.snap_flag;
  a.progress = w.progress;
  a.queue = w.ctr;
  a.err = w.ctr + 1;
  a.slots = w.slots;
  a.seg_bits = w.seg_bits;
  a.seg_words = w.seg_words;
  a.act_scratch = w.act;
  a.w1f = w.w1f;
  a.s1f = w.s1f;
  a.params_out = params_out;
  // a waiting block gives up only after ~10 s without a step of its running
  // predecessor (a hardware fault, not a slow model); PMKLC_SPIN_LIMIT
  // overrides the bound (tests of the give-up path)
  a.spin_limit = 1ll << 26;
  if (const char *sl = getenv("PMKLC_SPIN_LIMIT")) a.spin_limit = atoll(sl);
  const char *ph = getenv("PMKLC_PHASES");
  a.phase_clk = (ph && ph[0] == '1') ? w.phase : nullptr;
  if (a.phase_clk) HIP_TRY(hipMemsetAsync(w.phase, 0, 16 * sizeof(unsigned long long), st));
  HIP_TRY(hipMemsetAsync(w.ctr, 0, 64 * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(w.snap_flag, 0, bd.size() * sizeof(int), st));
  HIP_TRY(hipMemsetAsync(w.progress, 0, bd.size() * sizeof(uint32_t), st));
  if (bd.empty()) return PMKLC_OK;
  std::vector<int> order;
  if (schedule != PMKLC_PLAIN) {
    order = queue_order(bd);
    HIP_TRY(h2d(w.order, order, st));
    a.order = w.order;
  }
  if (w.s1f) HIP_TRY(launch_w1_frag(w.stat + m.d.off_W[0], m.d.D, m.d.H[0], w.s1f, st));
  if (tm) {
    HIP_TRY(hipEventCreate(&tm->a));
    HIP_TRY(hipEventCreate(&tm->b));
    HIP_TRY(hipEventRecord(tm->a, st));
  }
  g_last.launches = schedule == PMKLC_PLAIN ? (uint32_t)bd.size() : 1;
  // host copies of the kernel arguments stay alive until the stream has
  // consumed them (synchronised before returning)
  std::vector<StepArgs> hold(schedule == PMKLC_PLAIN ? bd.size() : 1);
  if (schedule == PMKLC_PLAIN) {
    // one block per launch, in block order (the per-block baseline)
    for (size_t b = 0; b < bd.size(); b++) {
      StepArgs &one = hold[b];
      one = a;
      one.n_blocks = 1;
      one.blocks = w.desc + b;
      // parameters/slots/bits are indexed by the block number: offset them
      one.params = w.params + b * (size_t)m.d.stride;
      one.adam_m = w.adam_m ? w.adam_m + b * (size_t)m.d.stride : nullptr;
      one.adam_v = w.adam_v ? w.adam_v + b * (size_t)m.d.stride : nullptr;
      one.seg_bits = w.seg_bits + b * (size_t)m.d.bs;
      one.seg_words = w.seg_words + b * (size_t)m.d.bs;
      one.queue = w.ctr + 2 + (int)(b % 60);
      if (bd[b].pred >= 0 || bd[b].has_snap) return PMKLC_ERR_UNSUPPORTED;
      HIP_TRY(hipMemsetAsync(one.queue, 0, sizeof(int), st));
      HIP_TRY(hipMemcpyAsync(w.args + b, &one, sizeof(StepArgs), hipMemcpyHostToDevice, st));
      HIP_TRY(launch_kind(m, one, w.args + b, 1, m.nt, st));
    }
  } else {
    int dev = 0, ncu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    int grid = (int)std::min<uint64_t>(std::min<uint64_t>(bd.size(), (uint64_t)std::max(ncu, 1)), kMaxGrid);
    hold[0] = a;
    HIP_TRY(hipMemcpyAsync(w.args, &hold[0], sizeof(StepArgs), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_kind(m, a, w.args, grid, m.nt, st));
  }
  if (tm) HIP_TRY(hipEventRecord(tm->b, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (a.phase_clk) {
    HIP_TRY(hipMemcpy(g_last.phase_ticks, w.phase, 12 * sizeof(uint64_t), hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    g_last.wall_khz = (uint32_t)khz;
  }
  return PMKLC_OK;
}

// The Transformer DM's loop over all blocks, slots holding the blocks
// longest first (a stable order, so slot contents are a function of the
// block lengths alone).
pmklc_status run_tf(const Model &m, const Work &w, int mode, const std::vector<BlockDesc> &bd, hipStream_t st,
                    StepTimer *tm, const uint8_t *tokens_override = nullptr, TfRun *extra = nullptr) {
  const int n = (int)bd.size();
  g_last.threads = 256;
  g_last.launches = 0;
  if (n == 0) return PMKLC_OK;
  std::vector<int> ord(n);
  for (int b = 0; b < n; b++) ord[b] = b;
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return bd[x].L > bd[y].L; });
  std::vector<TfSlot> sl(n);
  uint64_t maxL = 0;
  for (int q = 0; q < n; q++) {
    const BlockDesc &d = bd[ord[q]];
    sl[q] = TfSlot{d.tok_off, d.slot_off, d.L, d.slot_words, ord[q], 0};
    maxL = std::max<uint64_t>(maxL, d.L);
  }
  HIP_TRY(h2d(w.tf_desc, sl, st));
  // the error word the callers read after the loop (shared with the MLP kernels)
  if (w.ctr) HIP_TRY(hipMemsetAsync(w.ctr, 0, 64 * sizeof(int), st));
  TfBufs b;
  tf_bufs_carve(m.tf, n, w.tf_f, b);
  b.state = w.tf_state;
  b.slots_desc = w.tf_desc;
  b.params = w.params;
  b.adam_m = w.adam_m;
  b.adam_v = w.adam_v;
  b.init = w.init;
  b.stat = w.tf_stat;
  TfRun r;
  if (extra) r = *extra;
  else memset(&r, 0, sizeof r);
  r.mode = mode;
  r.n = n;
  r.desc_host = sl.data();
  r.tokens = const_cast<uint8_t *>(tokens_override ? tokens_override : w.tok);
  r.stream_slots = w.slots;
  r.seg_bits = w.seg_bits;
  r.seg_words = w.seg_words;
  r.max_L = maxL;
  if (const char *pg = getenv("PMKLC_PROGRESS")) r.progress = strtoull(pg, nullptr, 10);
  if (tm) {
    HIP_TRY(hipEventCreate(&tm->a));
    HIP_TRY(hipEventCreate(&tm->b));
    HIP_TRY(hipEventRecord(tm->a, st));
  }
  HIP_TRY(tf_run(m.tf, b, r, st));
  if (tm) HIP_TRY(hipEventRecord(tm->b, st));
  TfState hs;
  HIP_TRY(hipMemcpyAsync(&hs, w.tf_state, sizeof hs, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return hs.pad[0] ? PMKLC_ERR_DEVICE : PMKLC_OK;
}

// after the stream has been synchronised
void finish_timing(StepTimer &tm, std::chrono::steady_clock::time_point t0) {
  float ms = 0.0f;
  if (tm.a && tm.b && hipEventElapsedTime(&ms, tm.a, tm.b) == hipSuccess) g_last.step_ms = ms;
  g_last.call_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

// ====================================================================== ABI
extern "C" {

const char *pmklc_status_string(pmklc_status s) {
  switch (s) {
    case PMKLC_OK: return "ok";
    case PMKLC_ERR_INVALID_ARG: return "invalid argument";
    case PMKLC_ERR_INVALID_BASE: return "invalid base";
    case PMKLC_ERR_BUFFER_TOO_SMALL: return "buffer too small";
    case PMKLC_ERR_CORRUPT: return "corrupt container";
    case PMKLC_ERR_MODEL_MISMATCH: return "model mismatch";
    case PMKLC_ERR_DEVICE: return "device error";
    case PMKLC_ERR_UNSUPPORTED: return "unsupported configuration";
    case PMKLC_ERR_SCRATCH_LIMIT: return "input exceeds the no-allocation scratch buffer";
  }
  return "unknown";
}

uint64_t pmklc_param_count(const pmklc_config *c) {
  if (!c || c->k < 1 || c->k > 4 || c->n_hidden > 4) return 0;
  return param_count(c->k, c->t, c->embed, c->n_hidden, c->hidden, c->arch);
}

pmklc_status pmklc_encode_skmer(const uint8_t *bases_dev, uint64_t n, uint32_t s, uint32_t k, uint8_t *tokens_dev,
                                uint64_t cap, uint64_t *n_tokens, void *stream) {
  if (s < 1 || k < 1 || k > 4 || s > k || !n_tokens || (n && !bases_dev)) return PMKLC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t l = tokens_of(n, s, k);
  if (l > cap) { *n_tokens = l; return PMKLC_ERR_BUFFER_TOO_SMALL; }
  if (l && !tokens_dev) return PMKLC_ERR_INVALID_ARG;
  if (n == 0) { *n_tokens = 0; return PMKLC_OK; }
  StatusSlot slot;
  HIP_TRY(slot.acquire(st));
  int *err = reinterpret_cast<int *>(slot.ptr);
  int herr = 0;
  hipError_t e = hipMemsetAsync(err, 0, sizeof(int), st);
  if (e == hipSuccess) e = launch_skmer_direct(bases_dev, n, (int)s, (int)k, tokens_dev, l, err, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return PMKLC_ERR_DEVICE;
  if (herr) return PMKLC_ERR_INVALID_BASE;
  *n_tokens = l;
  return PMKLC_OK;
}

pmklc_status pmklc_compress_bound(const pmklc_config *cfg_in, uint64_t n, uint64_t *max_out, uint64_t *ws_bytes) {
  pmklc_status rc = check_cfg(cfg_in);
  if (rc) return rc;
  const pmklc_config cr = ms_resolve(cfg_in, n);
  const pmklc_config *cfg = &cr;
  rc = check_cfg(cfg);   // the selector's choice must be a valid configuration too
  if (rc) return rc;
  Model m;
  rc = make_model(cfg, m);
  if (rc) return rc;
  Plan p;
  rc = plan_blocks(n, cfg->n_blocks, cfg->block_len_host, cfg->n_files, cfg->file_blocks_host,
                   cfg->smp_ppm > 0 && (cfg->selector & PMKLC_SEL_DM), p);
  if (rc) return rc;
  Sizes z{};
  uint64_t meta = kHeaderBytes + 10ull * p.file_blocks.size();
  for (uint32_t b = 0; b < cfg->n_blocks; b++) {
    uint64_t rl = p.raw_len[b];
    z.n_chunks += (rl + kScanChunk - 1) / kScanChunk;
    z.runs += (rl + 1) / 2;
    uint64_t l = tokens_of(rl, cfg->s, cfg->k);
    uint64_t L = l / cfg->bs;
    z.tokens += l;
    z.slot_words += (uint64_t)slot_words_for(L) * cfg->bs;
    uint64_t runs = (rl + 1) / 2;
    meta += 10 + 10 + 20 * runs + (2ull * cfg->k * cfg->bs + 8 + 7) / 8 + 1 + 10ull * cfg->bs;
  }
  z.staging = 4 * z.slot_words;
  Arena A{nullptr, ~0ull};
  Work w;
  layout(A, m, cfg->n_blocks, z, cfg->optimizer == PMKLC_ADAM, cfg->smp_ppm > 0, w);
  if (cfg->selector & PMKLC_SEL_SPRM) {
    SprmRun pr;
    rc = sprm_layout(A, cfg, z.tokens, pr, m);
    if (rc) return rc;
    meta += 4ull * static_count(m);
  }
  if (max_out) *max_out = meta + z.staging;
  if (ws_bytes) *ws_bytes = A.used + 256;
  return PMKLC_OK;
}

}  // extern "C"

namespace {
// pmklc_compress on a given workspace. noalloc: the no-allocation entry
// point's call (no timing events, no autotuner trial runs).
pmklc_status compress_impl(const pmklc_config *cfg_in, const uint8_t *in_dev, uint64_t n, void *ws_dev,
                           uint64_t ws_bytes, uint8_t *out_host, uint64_t out_cap, uint64_t *out_len,
                           void *stream, bool noalloc) {
  const auto t0 = std::chrono::steady_clock::now();
  g_last = pmklc_timing{};
  StepTimer tm;
  pmklc_status rc = check_cfg(cfg_in);
  if (rc) return rc;
  const pmklc_config cr = ms_resolve(cfg_in, n);
  const pmklc_config *cfg = &cr;
  rc = check_cfg(cfg);   // the selector's choice must be a valid configuration too
  if (rc) return rc;
  const bool sprm = (cfg->selector & PMKLC_SEL_SPRM) != 0;
  if (!out_len || (n && !in_dev) || !ws_dev) return PMKLC_ERR_INVALID_ARG;
  Model m;
  rc = make_model(cfg, m);
  if (rc) return rc;
  if ((cfg->selector & PMKLC_SEL_SPUM) && (!cfg->static_host || cfg->static_len != static_count(m)))
    return PMKLC_ERR_MODEL_MISMATCH;
  const bool smp = cfg->smp_ppm > 0 && (cfg->selector & PMKLC_SEL_DM);
  Plan p;
  rc = plan_blocks(n, cfg->n_blocks, cfg->block_len_host, cfg->n_files, cfg->file_blocks_host, smp, p);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t nblk = cfg->n_blocks;
  const uint32_t s = cfg->s, k = cfg->k, bs = cfg->bs;

  // worst-case sizes (same as the bound), so the layout is fixed before the scan
  Sizes z{};
  std::vector<SeqBlock> sb(nblk);
  std::vector<uint64_t> chunk_block;
  for (uint32_t b = 0; b < nblk; b++) {
    sb[b] = SeqBlock{};
    sb[b].raw_off = p.raw_off[b];
    sb[b].raw_len = p.raw_len[b];
    sb[b].chunk0 = z.n_chunks;
    uint64_t nc = (p.raw_len[b] + kScanChunk - 1) / kScanChunk;
    for (uint64_t c = 0; c < nc; c++) chunk_block.push_back(b);
    z.n_chunks += nc;
    z.runs += (p.raw_len[b] + 1) / 2;
    uint64_t l = tokens_of(p.raw_len[b], s, k);
    z.tokens += l;
    z.slot_words += (uint64_t)slot_words_for(l / bs) * bs;
  }
  z.staging = 4 * z.slot_words;
  Arena A{static_cast<uint8_t *>(ws_dev), ws_bytes};
  Work w;
  layout(A, m, nblk, z, cfg->optimizer == PMKLC_ADAM, smp, w);
  SprmRun pr;
  if (sprm) {
    rc = sprm_layout(A, cfg, z.tokens, pr, m);
    if (rc) return rc;
  }
  if (A.over) return PMKLC_ERR_BUFFER_TOO_SMALL;

  // ---- A1: scan (validate, count N runs)
  std::vector<ChunkStat> stats;
  HIP_TRY(h2d(w.chunk_block, chunk_block, st));
  HIP_TRY(h2d(w.seq, sb, st));
  HIP_TRY(launch_scan(in_dev, w.seq, w.chunk_block, z.n_chunks, w.stats, st));
  HIP_TRY(d2h(stats, w.stats, z.n_chunks, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::vector<uint64_t> chunk_run0(z.n_chunks);
  uint64_t run_total = 0, tok_total = 0, ex_total = 0;
  for (uint32_t b = 0; b < nblk; b++) {
    uint64_t nN = 0, nr = 0;
    uint64_t nc = (p.raw_len[b] + kScanChunk - 1) / kScanChunk;
    for (uint64_t c = sb[b].chunk0; c < sb[b].chunk0 + nc; c++) {
      if (stats[c].bad) return PMKLC_ERR_INVALID_BASE;
      chunk_run0[c] = nr;
      nr += stats[c].n_runs;
      nN += stats[c].n_N;
    }
    SeqBlock &q = sb[b];
    q.run0 = run_total;
    q.n_runs = nr;
    run_total += nr;
    q.nb = q.raw_len - nN;
    q.l = tokens_of(q.nb, s, k);
    q.tok_off = tok_total;
    tok_total += q.l;
    q.L = q.l / bs;
    q.tail_off = q.l ? (q.l - 1) * s + k : 0;
    q.ex_off = ex_total;
    ex_total += bs + 8;
  }
  // ---- A1/A2: runs, tokens, extras
  uint64_t n_sk = 0, n_tk = 0, n_raw = 0;
  assign_tiles(sb.data(), (int)nblk, n_sk, n_tk, n_raw);
  HIP_TRY(h2d(w.seq, sb, st));
  HIP_TRY(h2d(w.chunk_run0, chunk_run0, st));
  if (run_total) {
    HIP_TRY(launch_runs(in_dev, w.seq, w.chunk_block, z.n_chunks, w.stats, w.chunk_run0, w.run_start, w.run_len, st));
    HIP_TRY(launch_run_sp(w.seq, (int)nblk, w.run_start, w.run_len, w.run_sp, w.run_cum, st));
  }
  HIP_TRY(launch_tokenise(in_dev, w.seq, (int)nblk, n_sk, n_tk, w.run_sp, w.run_cum, (int)s, (int)k, w.tok, st));
  HIP_TRY(launch_extras(in_dev, w.seq, (int)nblk, w.run_sp, w.run_cum, (int)s, (int)k, (int)bs, w.tok, w.extras, st));

  // ---- A3-A11: model loop + coder
  std::vector<BlockDesc> bd;
  uint64_t slot_total = 0;
  fill_blockdesc(m, sb, p, cfg->smp_ppm, bd, slot_total);
  HIP_TRY(h2d(w.desc, bd, st));
  uint32_t scrc = 0;
  std::vector<float> priv;   // the static private model, as stored
  if (m.d.model_on) {
    HIP_TRY(is_transformer(m.kind) ? tf_init_params(m.tf, cfg->seed, w.init, st)
                                   : launch_init_params(m.d, cfg->seed, w.init, st));
    if (has_static(m) && !sprm) {
      scrc = crc32(cfg->static_host, 4 * static_count(m));
      HIP_TRY(hipMemcpyAsync(bigru_on(m) ? w.tf_stat : w.stat, cfg->static_host, 4 * static_count(m),
                             hipMemcpyHostToDevice, st));
    }
  }
  if (sprm) {
    // Sec. 4.2.3 / stage (b): train the private model on the input's own
    // tokens, straight into the static-model slab of the coding pass
    const uint64_t Lp = std::min<uint64_t>(tok_total / bs, kSprmSteps);
    if (Lp > pr.Lp_max) return PMKLC_ERR_DEVICE;
    if (pr.gru) {
      // the one-layer BiGRU private model, trained in place in the static slab
      HIP_TRY(gru_init_params(m.tf, cfg->seed ^ kSprmSeedXor, w.tf_stat, st));
      if (Lp > 0) {
        HIP_TRY(launch_sprm_gather(w.tok, tok_total, bs, (uint32_t)Lp, pr.gtok, st));
        HIP_TRY(gru_train(m.tf, pr.gtok, Lp, w.tf_stat, pr.gbuf, pr.gm, pr.gv, st));
      }
      HIP_TRY(d2h(priv, w.tf_stat, (uint64_t)m.tf.sP, st));
    } else {
    HIP_TRY(launch_init_params(pr.m.d, cfg->seed ^ kSprmSeedXor, pr.w.init, st));
    if (Lp > 0) {
      HIP_TRY(launch_sprm_gather(w.tok, tok_total, bs, (uint32_t)Lp, pr.w.tok, st));
      std::vector<BlockDesc> one(1);
      one[0] = BlockDesc{};
      one[0].L = (uint32_t)Lp;
      one[0].slot_words = slot_words_for(Lp);
      one[0].pred = -1;
      HIP_TRY(h2d(pr.w.desc, one, st));
      rc = run_step(pr.m, pr.w, 0, one, PMKLC_BATCHED, st, nullptr, false, w.stat);
      if (rc) return rc;
      std::vector<int> pctr;
      HIP_TRY(d2h(pctr, pr.w.ctr, 2, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (pctr[1]) return PMKLC_ERR_DEVICE;
    } else {
      HIP_TRY(hipMemcpyAsync(w.stat, pr.w.init, 4ull * m.d.P, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(d2h(priv, w.stat, (uint64_t)m.d.P, st));
    }
    HIP_TRY(hipStreamSynchronize(st));
    scrc = crc32(priv.data(), 4ull * static_count(m));
  }
  count_work(m, bd, g_last);
  rc = is_tf(m.kind) ? run_tf(m, w, 0, bd, st, noalloc ? nullptr : &tm)
                     : run_step(m, w, 0, bd, cfg->schedule, st, noalloc ? nullptr : &tm, !noalloc);
  if (rc) return rc;
  std::vector<uint32_t> seg_bits, run_start, run_len;
  std::vector<uint8_t> extras;
  std::vector<int> ctr;
  HIP_TRY(d2h(seg_bits, w.seg_bits, (uint64_t)nblk * bs, st));
  HIP_TRY(d2h(extras, w.extras, ex_total, st));
  HIP_TRY(d2h(run_start, w.run_start, run_total, st));
  HIP_TRY(d2h(run_len, w.run_len, run_total, st));
  HIP_TRY(d2h(ctr, w.ctr, 2, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ctr[1]) return PMKLC_ERR_DEVICE;

  // ---- A12: container
  Writer meta{out_host, out_cap};
  write_header(meta, cfg, path_of(cfg->selector, m.kind), scrc, n, (uint32_t)p.file_blocks.size());
  for (uint64_t fb : p.file_blocks) meta.varint(fb);
  if (sprm) meta.put(priv.data(), 4ull * static_count(m));   // the private model travels in the file
  std::vector<uint64_t> seg_src, seg_dst;
  std::vector<uint32_t> seg_bytes;
  uint64_t stream_total = 0;
  for (uint32_t b = 0; b < nblk; b++) {
    const SeqBlock &q = sb[b];
    meta.varint(q.raw_len);
    meta.varint(q.n_runs);
    uint64_t prev_end = 0;
    for (uint64_t r = 0; r < q.n_runs; r++) {
      uint64_t st0 = run_start[q.run0 + r], ln = run_len[q.run0 + r];
      meta.varint(st0 - prev_end);
      meta.varint(ln);
      prev_end = st0 + ln;
    }
    BitPack bp;
    const uint8_t *ex = extras.data() + q.ex_off;
    uint64_t ntail = q.nb - q.tail_off, nrem = q.l - q.L * bs;
    for (uint64_t i = 0; i < ntail; i++) bp.put(ex[i], 2);
    for (uint64_t i = 0; i < nrem; i++) bp.put(ex[ntail + i], 2 * (int)k);
    meta.put(bp.b.data(), (bp.nbits + 7) / 8);
    if (q.L > 0) {
      for (uint32_t j = 0; j < bs; j++) {
        uint32_t nbytes = (seg_bits[(uint64_t)b * bs + j] + 7) / 8;
        meta.varint(nbytes);
        seg_src.push_back(bd[b].slot_off + (uint64_t)j * bd[b].slot_words);
        seg_dst.push_back(stream_total);
        seg_bytes.push_back(nbytes);
        stream_total += nbytes;
      }
    }
  }
  const uint64_t total = meta.n + stream_total;
  if (total > out_cap || meta.over) { *out_len = total; return PMKLC_ERR_BUFFER_TOO_SMALL; }
  if (stream_total) {
    HIP_TRY(h2d(w.seg_src, seg_src, st));
    HIP_TRY(h2d(w.seg_dst, seg_dst, st));
    HIP_TRY(h2d(w.seg_bytes, seg_bytes, st));
    HIP_TRY(launch_gather_streams(w.slots, w.seg_src, w.seg_dst, w.seg_bytes, seg_src.size(), w.staging, st));
    HIP_TRY(hipMemcpyAsync(out_host + meta.n, w.staging, stream_total, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  *out_len = total;
  finish_timing(tm, t0);
  return PMKLC_OK;
}

// Per device: the address of its copy of `scratch` (looked up once, with
// that device current) and the lock that serialises this process's
// no-allocation calls on it.
struct ScratchDev {
  std::mutex mu;
  void *ptr = nullptr;
};
ScratchDev g_scratch[kMaxDevices];
}  // namespace

extern "C" {

pmklc_status pmklc_compress(const pmklc_config *cfg, const uint8_t *in_dev, uint64_t n, void *ws_dev,
                            uint64_t ws_bytes, uint8_t *out_host, uint64_t out_cap, uint64_t *out_len,
                            void *stream) {
  return compress_impl(cfg, in_dev, n, ws_dev, ws_bytes, out_host, out_cap, out_len, stream, false);
}

pmklc_status pmklc_compress_noalloc(const pmklc_config *cfg, const uint8_t *in_dev, uint64_t n, uint8_t *out_host,
                                    uint64_t out_cap, uint64_t *out_len, void *stream) {
  uint64_t need = 0;
  pmklc_status rc = pmklc_compress_bound(cfg, n, nullptr, &need);
  if (rc) return rc;
  if (need > kScratchBytes) return PMKLC_ERR_SCRATCH_LIMIT;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return PMKLC_ERR_DEVICE;
  ScratchDev &sd = g_scratch[dev];
  std::lock_guard<std::mutex> lk(sd.mu);
  if (!sd.ptr) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(pmklc::scratch)) != hipSuccess || !p) return PMKLC_ERR_DEVICE;
    sd.ptr = p;
  }
  return compress_impl(cfg, in_dev, n, sd.ptr, kScratchBytes, out_host, out_cap, out_len, stream, true);
}

// --------------------------------------------------------------- decode
namespace {
struct Parsed {
  pmklc_config c;
  uint32_t hidden[4];
  uint8_t path;
  uint32_t scrc;
  uint64_t n;
  std::vector<uint64_t> file_blocks;
  std::vector<SeqBlock> sb;
  std::vector<uint32_t> run_start, run_len, run_cum;
  std::vector<uint8_t> extras;        // per block: tail codes then remainder tokens (bs + 8 bytes each)
  std::vector<uint32_t> seg_bytes;    // [blocks with L>0][bs] in block order, flat per block b at b*bs
  uint64_t stream_off;                // first stream byte in the container
  uint64_t private_off = 0;           // the stored static private model (4 P bytes), if any
};

pmklc_status parse(const uint8_t *p, uint64_t len, Parsed &o, bool full) {
  if (!p || len < (uint64_t)kHeaderBytes || memcmp(p, "PMKC", 4) != 0) return PMKLC_ERR_CORRUPT;
  Reader r{p, len};
  r.pos = 4;
  if (r.le(1) != 1) return PMKLC_ERR_CORRUPT;
  pmklc_config &c = o.c;
  memset(&c, 0, sizeof c);
  c.struct_size = sizeof(pmklc_config);
  o.path = (uint8_t)r.le(1);
  c.s = (uint32_t)r.le(1);
  c.k = (uint32_t)r.le(1);
  c.t = (uint32_t)r.le(2);
  c.bs = (uint32_t)r.le(2);
  c.embed = (uint32_t)r.le(2);
  c.n_hidden = (uint32_t)r.le(1);
  c.optimizer = (uint32_t)r.le(1);
  for (int l = 0; l < 4; l++) c.hidden[l] = (uint32_t)r.le(2);
  c.lr = r.f32();
  c.beta1 = r.f32();
  c.beta2 = r.f32();
  c.eps = r.f32();
  c.selector = (uint32_t)r.le(1);
  c.arch = (uint32_t)r.le(1);
  c.heads = (uint32_t)r.le(1);
  {
    const uint32_t sb = (uint32_t)r.le(1);
    c.static_arch = sb & 15;
    c.gru_layers = sb >> 4;
  }
  c.smp_ppm = (uint32_t)r.le(4);
  c.seed = r.le(8);
  o.scrc = (uint32_t)r.le(4);
  c.static_embed = (uint32_t)r.le(1);
  c.gru_hidden = (uint32_t)r.le(1);
  c.dense = (uint32_t)r.le(2);
  o.n = r.le(8);
  c.n_blocks = (uint32_t)r.le(4);
  uint32_t nf = (uint32_t)r.le(4);
  if (r.bad) return PMKLC_ERR_CORRUPT;
  c.precision = (o.path == kPathBF16 || o.path == kPathBF16Chip || o.path == kPathTfBF16 || o.path == kPathSeqBF16)
                    ? PMKLC_BF16
                : o.path == kPathFP32Valu ? PMKLC_FP32_VALU : PMKLC_FP32;
  if (check_cfg(&c) || c.selector == PMKLC_SEL_AUTO) return PMKLC_ERR_CORRUPT;
  if (o.path != kPathUniform && o.path != kPathBF16 && o.path != kPathFP32Valu && o.path != kPathFP32Mfma &&
      o.path != kPathBF16Chip && o.path != kPathTfBF16 && o.path != kPathTfFP32 && o.path != kPathSeqBF16 &&
      o.path != kPathSeqFP32)
    return PMKLC_ERR_MODEL_MISMATCH;
  if (nf < 1 || (uint64_t)nf > len || (uint64_t)c.n_blocks * 2 > len) return PMKLC_ERR_CORRUPT;
  o.file_blocks.resize(nf);
  uint64_t tot = 0;
  for (uint32_t f = 0; f < nf; f++) { o.file_blocks[f] = r.varint(); tot += o.file_blocks[f]; }
  if (r.bad || tot != c.n_blocks) return PMKLC_ERR_CORRUPT;
  c.n_files = nf;
  if (c.selector & PMKLC_SEL_SPRM) {
    // the private static model, checked against the header's CRC-32
    const uint64_t P = c.static_arch == PMKLC_STATIC_BIGRU
                           ? bigru_param_count(c)
                           : param_count(c.k, c.t, c.embed, c.n_hidden, c.hidden, c.arch);
    if (P > (len - r.pos) / 4 || crc32(p + r.pos, 4 * P) != o.scrc) return PMKLC_ERR_CORRUPT;
    o.private_off = r.pos;
    r.pos += 4 * P;
  }
  if (!full) return PMKLC_OK;
  const uint32_t nblk = c.n_blocks, bs = c.bs, s = c.s, k = c.k;
  o.sb.resize(nblk);
  o.extras.assign((uint64_t)nblk * (bs + 8), 0);
  o.seg_bytes.assign((uint64_t)nblk * bs, 0);
  uint64_t off = 0, tok_total = 0;
  for (uint32_t b = 0; b < nblk; b++) {
    SeqBlock &q = o.sb[b];
    q = SeqBlock{};
    q.raw_off = off;
    q.raw_len = r.varint();
    if (r.bad || q.raw_len > o.n - off || q.raw_len > 0xFFFFFFFFull) return PMKLC_ERR_CORRUPT;
    off += q.raw_len;
    q.n_runs = r.varint();
    if (r.bad || q.n_runs > q.raw_len) return PMKLC_ERR_CORRUPT;
    q.run0 = o.run_start.size();
    uint64_t prev_end = 0, nN = 0;
    for (uint64_t i = 0; i < q.n_runs; i++) {
      uint64_t gap = r.varint(), ln = r.varint();
      uint64_t st0 = prev_end + gap;
      if (r.bad || ln == 0 || st0 + ln > q.raw_len || (i > 0 && gap == 0)) return PMKLC_ERR_CORRUPT;
      nN += ln;
      o.run_start.push_back((uint32_t)st0);
      o.run_len.push_back((uint32_t)ln);
      o.run_cum.push_back((uint32_t)nN);
      prev_end = st0 + ln;
    }
    q.nb = q.raw_len - nN;
    q.l = tokens_of(q.nb, s, k);
    q.L = q.l / bs;
    q.tail_off = q.l ? (q.l - 1) * s + k : 0;
    q.tok_off = tok_total;
    tok_total += q.l;
    q.ex_off = (uint64_t)b * (bs + 8);
    uint64_t ntail = q.nb - q.tail_off, nrem = q.l - q.L * bs;
    uint64_t bits = 2 * ntail + 2ull * k * nrem;
    uint64_t eb = (bits + 7) / 8;
    if (r.pos + eb > len) return PMKLC_ERR_CORRUPT;
    uint64_t bit = 0;
    const uint8_t *src = p + r.pos;
    for (uint64_t i = 0; i < ntail; i++) o.extras[q.ex_off + i] = (uint8_t)get_bits(src, bit, 2);
    for (uint64_t i = 0; i < nrem; i++) o.extras[q.ex_off + ntail + i] = (uint8_t)get_bits(src, bit, 2 * (int)k);
    r.pos += eb;
    if (q.L > 0) {
      for (uint32_t j = 0; j < bs; j++) {
        uint64_t v = r.varint();
        if (r.bad || v > len) return PMKLC_ERR_CORRUPT;
        o.seg_bytes[(uint64_t)b * bs + j] = (uint32_t)v;
      }
      if (q.L > 0xFFFFFFFFull) return PMKLC_ERR_CORRUPT;
    }
  }
  if (off != o.n) return PMKLC_ERR_CORRUPT;
  o.stream_off = r.pos;
  uint64_t sum = 0;
  for (uint32_t v : o.seg_bytes) sum += v;
  if (o.stream_off + sum != len) return PMKLC_ERR_CORRUPT;
  for (uint32_t b = 0; b < nblk; b++) {
    if (o.sb[b].L == 0) continue;
    for (uint32_t j = 0; j < bs; j++)
      if (o.seg_bytes[(uint64_t)b * bs + j] > 4ull * slot_words_for(o.sb[b].L)) return PMKLC_ERR_CORRUPT;
  }
  return PMKLC_OK;
}

Sizes dec_sizes(const Parsed &o) {
  Sizes z{};
  z.runs = o.run_start.size();
  for (const SeqBlock &q : o.sb) {
    z.tokens += q.l;
    z.slot_words += (uint64_t)slot_words_for(q.L) * o.c.bs;
  }
  for (uint32_t v : o.seg_bytes) z.staging += v;
  return z;
}
}  // namespace

pmklc_status pmklc_decompress_info(const uint8_t *cbf_host, uint64_t len, uint64_t *n_bases, uint64_t *ws_bytes) {
  Parsed o;
  pmklc_status rc = parse(cbf_host, len, o, true);
  if (rc) return rc;
  Model m;
  rc = make_model(&o.c, m, o.path == kPathBF16Chip, o.path == kPathSeqBF16 || o.path == kPathSeqFP32 ? 1 : 0);
  if (rc) return rc;
  Plan p;
  rc = plan_blocks(o.n, o.c.n_blocks, nullptr, 0, nullptr, false, p);
  (void)p;
  Arena A{nullptr, ~0ull};
  Work w;
  layout(A, m, o.c.n_blocks, dec_sizes(o), o.c.optimizer == PMKLC_ADAM, o.c.smp_ppm > 0, w);
  if (n_bases) *n_bases = o.n;
  if (ws_bytes) *ws_bytes = A.used + 256;
  return PMKLC_OK;
}

pmklc_status pmklc_decompress(const uint8_t *cbf_host, uint64_t len, const float *static_host, uint64_t static_len,
                              void *ws_dev, uint64_t ws_bytes, uint8_t *out_dev, uint64_t out_cap, uint64_t *out_len,
                              void *stream) {
  const auto t0 = std::chrono::steady_clock::now();
  g_last = pmklc_timing{};
  StepTimer tm;
  if (!out_len || !ws_dev) return PMKLC_ERR_INVALID_ARG;
  Parsed o;
  pmklc_status rc = parse(cbf_host, len, o, true);
  if (rc) return rc;
  Model m;
  rc = make_model(&o.c, m, o.path == kPathBF16Chip, o.path == kPathSeqBF16 || o.path == kPathSeqFP32 ? 1 : 0);
  if (rc) return rc;
  if (path_of(o.c.selector, m.kind) != o.path) return PMKLC_ERR_MODEL_MISMATCH;
  const bool sprm = (o.c.selector & PMKLC_SEL_SPRM) != 0;
  if (has_static(m) && !sprm) {
    if (!static_host || static_len != static_count(m) || crc32(static_host, 4 * static_count(m)) != o.scrc)
      return PMKLC_ERR_MODEL_MISMATCH;
  }
  if (o.n > out_cap) { *out_len = o.n; return PMKLC_ERR_BUFFER_TOO_SMALL; }
  if (o.n && !out_dev) return PMKLC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint32_t nblk = o.c.n_blocks, bs = o.c.bs;
  const bool smp = o.c.smp_ppm > 0 && m.d.model_on;
  Sizes z = dec_sizes(o);
  Arena A{static_cast<uint8_t *>(ws_dev), ws_bytes};
  Work w;
  layout(A, m, nblk, z, o.c.optimizer == PMKLC_ADAM, smp, w);
  if (A.over) return PMKLC_ERR_BUFFER_TOO_SMALL;
  Plan p;
  std::vector<uint64_t> bl(nblk);
  for (uint32_t b = 0; b < nblk; b++) bl[b] = o.sb[b].raw_len;
  rc = plan_blocks(o.n, nblk, bl.data(), (uint32_t)o.file_blocks.size(), o.file_blocks.data(), smp, p);
  if (rc) return PMKLC_ERR_CORRUPT;
  std::vector<BlockDesc> bd;
  uint64_t slot_total = 0;
  fill_blockdesc(m, o.sb, p, o.c.smp_ppm, bd, slot_total);
  // streams -> aligned slots
  std::vector<uint64_t> seg_src, seg_dst;
  std::vector<uint32_t> seg_bytes, seg_words((uint64_t)nblk * bs, 0);
  uint64_t so = 0;
  for (uint32_t b = 0; b < nblk; b++) {
    if (o.sb[b].L == 0) continue;
    for (uint32_t j = 0; j < bs; j++) {
      uint32_t nbt = o.seg_bytes[(uint64_t)b * bs + j];
      seg_src.push_back(so);
      seg_dst.push_back(bd[b].slot_off + (uint64_t)j * bd[b].slot_words);
      seg_bytes.push_back(nbt);
      seg_words[(uint64_t)b * bs + j] = (nbt + 3) / 4;
      so += nbt;
    }
  }
  std::vector<uint32_t> seg_words_c;
  for (uint32_t b = 0; b < nblk; b++) {
    if (o.sb[b].L == 0) continue;
    for (uint32_t j = 0; j < bs; j++) seg_words_c.push_back(seg_words[(uint64_t)b * bs + j]);
  }
  if (so) {
    HIP_TRY(hipMemcpyAsync(w.staging, cbf_host + o.stream_off, so, hipMemcpyHostToDevice, st));
    HIP_TRY(h2d(w.seg_src, seg_src, st));
    HIP_TRY(h2d(w.seg_dst, seg_dst, st));
    HIP_TRY(h2d(w.seg_bytes, seg_bytes, st));
    HIP_TRY(h2d(w.seg_bits, seg_words_c, st));   // per listed segment: words to fill
    HIP_TRY(launch_scatter_streams(w.staging, w.seg_src, w.seg_dst, w.seg_bytes, w.seg_bits, seg_src.size(), w.slots,
                                   st));
  }
  HIP_TRY(h2d(w.seg_words, seg_words, st));
  HIP_TRY(h2d(w.desc, bd, st));
  uint64_t n_sk = 0, n_tk = 0, n_raw = 0;
  assign_tiles(o.sb.data(), (int)nblk, n_sk, n_tk, n_raw);
  HIP_TRY(h2d(w.seq, o.sb, st));
  HIP_TRY(h2d(w.extras, o.extras, st));
  HIP_TRY(h2d(w.run_start, o.run_start, st));
  HIP_TRY(h2d(w.run_len, o.run_len, st));
  HIP_TRY(h2d(w.run_cum, o.run_cum, st));
  if (m.d.model_on) {
    HIP_TRY(is_transformer(m.kind) ? tf_init_params(m.tf, o.c.seed, w.init, st)
                                   : launch_init_params(m.d, o.c.seed, w.init, st));
    if (has_static(m)) {
      const void *src = sprm ? static_cast<const void *>(cbf_host + o.private_off) : static_host;
      HIP_TRY(hipMemcpyAsync(bigru_on(m) ? w.tf_stat : w.stat, src, 4 * static_count(m), hipMemcpyHostToDevice,
                             st));
    }
  }
  count_work(m, bd, g_last);
  rc = is_tf(m.kind) ? run_tf(m, w, 1, bd, st, &tm) : run_step(m, w, 1, bd, PMKLC_BATCHED, st, &tm);
  if (rc) return rc;
  HIP_TRY(launch_detok(w.seq, (int)nblk, n_raw, w.run_start, w.run_len, w.run_cum, (int)o.c.s, (int)o.c.k, (int)bs,
                       w.tok, w.extras, out_dev, st));
  std::vector<int> ctr;
  HIP_TRY(d2h(ctr, w.ctr, 2, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ctr[1]) return PMKLC_ERR_DEVICE;
  *out_len = o.n;
  finish_timing(tm, t0);
  return PMKLC_OK;
}

// ------------------------------------------------ differentiable DM op
// the Transformer op: one slot of bs = rows; workspace = state, one slot
// descriptor, then the slot's buffers
static pmklc_status tf_op_shape(const pmklc_config *cfg, uint32_t rows, TfShape &s) {
  pmklc_status rc = check_cfg(cfg);
  if (rc) return rc;
  if (!tf_shape((int)cfg->k, (int)cfg->t, (int)cfg->embed, (int)cfg->hidden[0], (int)cfg->hidden[1],
                (int)cfg->heads, s) ||
      cfg->precision == PMKLC_FP32_VALU || rows > 1024 || (uint64_t)rows * cfg->t > 65536)
    return PMKLC_ERR_UNSUPPORTED;
  s.bs = (int)rows;
  s.bf16 = cfg->precision == PMKLC_BF16;
  return PMKLC_OK;
}
// the MLP op on the same kernels (matrix cores, FP32 or BF16 inputs); false
// for PMKLC_FP32_VALU or shapes outside them (the per-thread op then runs)
static bool mlp_op_shape(const pmklc_config *cfg, uint32_t rows, TfShape &s) {
  if (cfg->precision == PMKLC_FP32_VALU || cfg->arch != PMKLC_ARCH_MLP || rows < 1) return false;
  Dims d;
  if (fill_dims(cfg->k, cfg->t, rows, cfg->embed, cfg->n_hidden, cfg->hidden, PMKLC_SEL_DM, cfg->optimizer, cfg->lr,
                cfg->beta1, cfg->beta2, cfg->eps, d))
    return false;
  if (!mlp_seq_shape(d, s)) return false;
  s.bf16 = cfg->precision == PMKLC_BF16;
  return true;
}
static uint64_t tf_op_bytes(const TfShape &s) {
  TfBufs b;
  return 512 + 4 * tf_bufs_carve(s, 1, nullptr, b) + 256;
}
static TfBufs tf_op_bufs(const TfShape &s, void *ws) {
  TfBufs b;
  memset(&b, 0, sizeof b);
  uint8_t *p = static_cast<uint8_t *>(ws);
  tf_bufs_carve(s, 1, reinterpret_cast<float *>(p + 512), b);
  b.state = reinterpret_cast<TfState *>(p);
  b.slots_desc = reinterpret_cast<TfSlot *>(p + 256);
  return b;
}
static pmklc_status tf_op_err(const TfBufs &b, hipStream_t st) {
  TfState hs;
  HIP_TRY(hipMemcpyAsync(&hs, b.state, sizeof hs, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return hs.pad[0] ? PMKLC_ERR_INVALID_ARG : PMKLC_OK;
}

static pmklc_status dm_dims(const pmklc_config *cfg, Dims &d) {
  pmklc_status rc = check_cfg(cfg);
  if (rc) return rc;
  return fill_dims(cfg->k, cfg->t, cfg->bs, cfg->embed, cfg->n_hidden, cfg->hidden, PMKLC_SEL_DM, cfg->optimizer,
                   cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, d);
}

pmklc_status pmklc_dm_workspace(const pmklc_config *cfg, uint32_t rows, uint64_t *ws_bytes) {
  if (cfg && cfg->struct_size == sizeof(pmklc_config) && cfg->arch == PMKLC_ARCH_TRANSFORMER) {
    TfShape s;
    pmklc_status rc = tf_op_shape(cfg, rows, s);
    if (rc) return rc;
    if (!ws_bytes) return PMKLC_ERR_INVALID_ARG;
    *ws_bytes = tf_op_bytes(s);
    return PMKLC_OK;
  }
  TfShape ms;
  if (cfg && cfg->struct_size == sizeof(pmklc_config) && !check_cfg(cfg) && mlp_op_shape(cfg, rows, ms)) {
    if (!ws_bytes) return PMKLC_ERR_INVALID_ARG;
    *ws_bytes = tf_op_bytes(ms);
    return PMKLC_OK;
  }
  Dims d;
  pmklc_status rc = dm_dims(cfg, d);
  if (rc) return rc;
  if (!ws_bytes) return PMKLC_ERR_INVALID_ARG;
  *ws_bytes = dm_op_workspace(d, (int)rows);
  return PMKLC_OK;
}

pmklc_status pmklc_dm_forward(const pmklc_config *cfg, const float *params_dev, const uint8_t *ctx_dev, uint32_t rows,
                              float *logits_dev, void *ws_dev, uint64_t ws_bytes, void *stream) {
  if (cfg && cfg->struct_size == sizeof(pmklc_config) && cfg->arch == PMKLC_ARCH_TRANSFORMER) {
    TfShape s;
    pmklc_status rc = tf_op_shape(cfg, rows, s);
    if (rc) return rc;
    if (rows == 0) return PMKLC_OK;
    if (!params_dev || !ctx_dev || !logits_dev || !ws_dev) return PMKLC_ERR_INVALID_ARG;
    if (ws_bytes < tf_op_bytes(s)) return PMKLC_ERR_BUFFER_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TfBufs b = tf_op_bufs(s, ws_dev);
    HIP_TRY(tf_forward_op(s, b, params_dev, ctx_dev, logits_dev, st));
    return tf_op_err(b, st);
  }
  TfShape ms;
  if (cfg && cfg->struct_size == sizeof(pmklc_config) && !check_cfg(cfg) && mlp_op_shape(cfg, rows, ms)) {
    if (!params_dev || !ctx_dev || !logits_dev || !ws_dev) return PMKLC_ERR_INVALID_ARG;
    if (ws_bytes < tf_op_bytes(ms)) return PMKLC_ERR_BUFFER_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TfBufs b = tf_op_bufs(ms, ws_dev);
    HIP_TRY(tf_forward_op(ms, b, params_dev, ctx_dev, logits_dev, st));
    return tf_op_err(b, st);
  }
  Dims d;
  pmklc_status rc = dm_dims(cfg, d);
  if (rc) return rc;
  if (rows == 0) return PMKLC_OK;
  if (!params_dev || !ctx_dev || !logits_dev || !ws_dev) return PMKLC_ERR_INVALID_ARG;
  if (ws_bytes < dm_op_workspace(d, (int)rows)) return PMKLC_ERR_BUFFER_TOO_SMALL;
  int err = 0;
  HIP_TRY(dm_forward(d, params_dev, ctx_dev, (int)rows, logits_dev, ws_dev, &err, static_cast<hipStream_t>(stream)));
  return err ? PMKLC_ERR_INVALID_ARG : PMKLC_OK;
}

pmklc_status pmklc_dm_backward(const pmklc_config *cfg, const float *params_dev, const uint8_t *ctx_dev, uint32_t rows,
                               const float *dlogits_dev, float *grad_dev, void *ws_dev, uint64_t ws_bytes,
                               void *stream) {
  if (cfg && cfg->struct_size == sizeof(pmklc_config) && cfg->arch == PMKLC_ARCH_TRANSFORMER) {
    TfShape s;
    pmklc_status rc = tf_op_shape(cfg, rows, s);
    if (rc) return rc;
    if (!params_dev || !ctx_dev || !dlogits_dev || !grad_dev || !ws_dev || rows == 0) return PMKLC_ERR_INVALID_ARG;
    if (ws_bytes < tf_op_bytes(s)) return PMKLC_ERR_BUFFER_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TfBufs b = tf_op_bufs(s, ws_dev);
    HIP_TRY(tf_backward_op(s, b, params_dev, ctx_dev, dlogits_dev, grad_dev, st));
    return tf_op_err(b, st);
  }
  TfShape ms;
  if (cfg && cfg->struct_size == sizeof(pmklc_config) && !check_cfg(cfg) && mlp_op_shape(cfg, rows, ms)) {
    if (!params_dev || !ctx_dev || !dlogits_dev || !grad_dev || !ws_dev) return PMKLC_ERR_INVALID_ARG;
    if (ws_bytes < tf_op_bytes(ms)) return PMKLC_ERR_BUFFER_TOO_SMALL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const TfBufs b = tf_op_bufs(ms, ws_dev);
    HIP_TRY(tf_backward_op(ms, b, params_dev, ctx_dev, dlogits_dev, grad_dev, st));
    return tf_op_err(b, st);
  }
  Dims d;
  pmklc_status rc = dm_dims(cfg, d);
  if (rc) return rc;
  if (!params_dev || !ctx_dev || !dlogits_dev || !grad_dev || !ws_dev) return PMKLC_ERR_INVALID_ARG;
  if (ws_bytes < dm_op_workspace(d, (int)rows)) return PMKLC_ERR_BUFFER_TOO_SMALL;
  int err = 0;
  HIP_TRY(dm_backward(d, params_dev, ctx_dev, (int)rows, dlogits_dev, grad_dev, ws_dev, &err,
                      static_cast<hipStream_t>(stream)));
  return err ? PMKLC_ERR_INVALID_ARG : PMKLC_OK;
}

pmklc_status pmklc_last_timing(pmklc_timing *t) {
  if (!t) return PMKLC_ERR_INVALID_ARG;
  *t = g_last;
  return PMKLC_OK;
}

// ------------------------------------------------------------ test exports
pmklc_status pmklc_quantise(const float *probs_dev, uint32_t rows, uint32_t V, uint32_t *cdf_dev, void *stream) {
  if ((V != 4 && V != 16 && V != 64 && V != 256) || (rows && (!probs_dev || !cdf_dev))) return PMKLC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_quantise(probs_dev, rows, V, cdf_dev, st));
  HIP_TRY(hipStreamSynchronize(st));
  return PMKLC_OK;
}

pmklc_status pmklc_wnc_encode(const uint32_t *cum_lo_dev, const uint32_t *cum_hi_dev, uint64_t m, uint8_t *out_dev,
                              uint64_t cap, uint64_t *nbits, void *stream) {
  if (!nbits || !out_dev || (m && (!cum_lo_dev || !cum_hi_dev)) || (reinterpret_cast<uintptr_t>(out_dev) & 3u))
    return PMKLC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  uint64_t need = (17 * m + 2 + 7) / 8;
  uint64_t need_words = (17 * m + 2 + 31) / 32;
  if (cap / 4 < need_words) { *nbits = 8 * need; return PMKLC_ERR_BUFFER_TOO_SMALL; }
  StatusSlot slot;
  HIP_TRY(slot.acquire(st));
  uint64_t *nb_dev = reinterpret_cast<uint64_t *>(slot.ptr);
  int *err = reinterpret_cast<int *>(nb_dev + 1);
  uint64_t hb = 0;
  int herr = 0;
  hipError_t e = hipMemsetAsync(nb_dev, 0, 16, st);
  if (e == hipSuccess)
    e = launch_wnc_encode(cum_lo_dev, cum_hi_dev, m, reinterpret_cast<uint32_t *>(out_dev),
                          (uint32_t)std::min<uint64_t>(cap / 4, 0xFFFFFFFFu), nb_dev, err, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&hb, nb_dev, 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return PMKLC_ERR_DEVICE;
  if (herr) return PMKLC_ERR_DEVICE;
  *nbits = hb;
  return PMKLC_OK;
}

pmklc_status pmklc_wnc_decode(const uint8_t *in_dev, uint64_t nbytes, const uint32_t *cdfs_dev, uint32_t V,
                              uint64_t m, uint32_t *symbols_dev, void *stream) {
  if (V < 2 || V > 256 || (m && (!cdfs_dev || !symbols_dev)) || (nbytes && !in_dev) ||
      (reinterpret_cast<uintptr_t>(in_dev) & 3u) || (nbytes & 3u))
    return PMKLC_ERR_INVALID_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(launch_wnc_decode(reinterpret_cast<const uint32_t *>(in_dev), (uint32_t)(nbytes / 4), cdfs_dev, V, m,
                            symbols_dev, st));
  HIP_TRY(hipStreamSynchronize(st));
  return PMKLC_OK;
}

// pmklc_model_trace for the Transformer DM: the compression loop's own
// launches on one block, with probes and the final parameters
static pmklc_status model_trace_tf(const pmklc_config *cfg, const Model &m, const uint8_t *tokens_dev, uint64_t l,
                                   const float *static_dev, const float *init_dev, uint64_t stop, const uint64_t *probe_steps_host,
                                   uint32_t n_probe, float *probs_dev, float *params_dev, uint8_t *streams_host,
                                   uint64_t streams_cap, uint64_t *streams_len, hipStream_t st) {
  const uint32_t bs = cfg->bs;
  const uint64_t L = l / bs;
  if (L > 0xFFFFFFFFull) return PMKLC_ERR_UNSUPPORTED;
  for (uint32_t q = 1; q < n_probe; q++)
    if (probe_steps_host[q] <= probe_steps_host[q - 1]) return PMKLC_ERR_INVALID_ARG;
  Sizes z{};
  z.slot_words = (uint64_t)slot_words_for(L) * bs;
  Arena A{nullptr, ~0ull};
  Work w;
  layout(A, m, 1, z, cfg->optimizer == PMKLC_ADAM, false, w);
  uint8_t *base = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&base), A.used + 256, st));
  Arena B{base, A.used + 256};
  layout(B, m, 1, z, cfg->optimizer == PMKLC_ADAM, false, w);
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  if (init_dev) chk(hipMemcpyAsync(w.init, init_dev, 4ull * (m.d.P + 1), hipMemcpyDeviceToDevice, st));
  else chk(is_transformer(m.kind) ? tf_init_params(m.tf, cfg->seed, w.init, st)
                                  : launch_init_params(m.d, cfg->seed, w.init, st));
  if (bigru_on(m)) {
    if (!static_dev) e = hipErrorInvalidValue;
    else chk(hipMemcpyAsync(w.tf_stat, static_dev, 4ull * m.tf.sP, hipMemcpyDeviceToDevice, st));
  }
  std::vector<BlockDesc> bd(1);
  bd[0] = BlockDesc{};
  bd[0].L = (uint32_t)L;
  bd[0].slot_words = slot_words_for(L);
  bd[0].pred = -1;
  TfRun r;
  memset(&r, 0, sizeof r);
  r.probe_steps_host = probe_steps_host;
  r.n_probe = (int)n_probe;
  r.probe_P = probs_dev;
  r.params_out = params_dev;
  r.stop = stop;
  pmklc_status rc = PMKLC_OK;
  if (e == hipSuccess) rc = run_tf(m, w, 0, bd, st, nullptr, tokens_dev, &r);
  std::vector<uint32_t> bits, slots;
  if (e == hipSuccess && rc == PMKLC_OK && streams_len && L > 0) {
    chk(d2h(bits, w.seg_bits, bs, st));
    chk(d2h(slots, w.slots, (uint64_t)slot_words_for(L) * bs, st));
  }
  chk(hipStreamSynchronize(st));
  (void)hipFreeAsync(base, st);
  (void)hipStreamSynchronize(st);
  if (e != hipSuccess) return PMKLC_ERR_DEVICE;
  if (rc) return rc;
  if (streams_len) {
    uint64_t total = 0;
    for (uint32_t b : bits) total += (b + 7) / 8;
    *streams_len = total;
    if (total > streams_cap) return PMKLC_ERR_BUFFER_TOO_SMALL;
    uint64_t at = 0;
    for (uint32_t j = 0; j < bits.size(); j++) {
      const uint64_t nb = (bits[j] + 7) / 8;
      memcpy(streams_host + at, reinterpret_cast<const uint8_t *>(slots.data() + (uint64_t)j * slot_words_for(L)), nb);
      at += nb;
    }
  }
  return PMKLC_OK;
}

pmklc_status pmklc_model_trace(const pmklc_config *cfg, const uint8_t *tokens_dev, uint64_t l, const float *static_dev,
                               const float *init_dev, uint64_t stop, const uint64_t *probe_steps_host, uint32_t n_probe,
                               float *probs_dev, float *params_dev, uint8_t *streams_host, uint64_t streams_cap,
                               uint64_t *streams_len, void *stream) {
  pmklc_status rc = check_cfg(cfg);
  if (rc) return rc;
  if (!(cfg->selector & PMKLC_SEL_DM) || !tokens_dev) return PMKLC_ERR_INVALID_ARG;
  Model m;
  rc = make_model(cfg, m);
  if (rc) return rc;
  if (has_static(m) && !static_dev) return PMKLC_ERR_MODEL_MISMATCH;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (is_tf(m.kind))
    return model_trace_tf(cfg, m, tokens_dev, l, static_dev, init_dev, stop, probe_steps_host, n_probe, probs_dev, params_dev,
                          streams_host, streams_cap, streams_len, st);
  const uint32_t bs = cfg->bs;
  uint64_t L = l / bs;
  if (L > 0xFFFFFFFFull) return PMKLC_ERR_UNSUPPORTED;
  Sizes z{};
  z.tokens = 0;
  z.slot_words = (uint64_t)slot_words_for(L) * bs;
  Arena A{nullptr, ~0ull};
  Work w;
  layout(A, m, 1, z, cfg->optimizer == PMKLC_ADAM, false, w);
  uint8_t *base = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&base), A.used + 256, st));
  Arena B{base, A.used + 256};
  layout(B, m, 1, z, cfg->optimizer == PMKLC_ADAM, false, w);
  m.nt = choose_nt(m, w, st);
  uint64_t *probe_dev = nullptr;
  StepArgs a;
  memset(&a, 0, sizeof a);
  std::vector<BlockDesc> bd(1);
  bd[0] = BlockDesc{0, 0, (uint32_t)L, slot_words_for(L), 0, -1, 0, 0};
  std::vector<uint64_t> probe(probe_steps_host, probe_steps_host + n_probe);
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  if (n_probe) {
    chk(hipMallocAsync(reinterpret_cast<void **>(&probe_dev), 8ull * n_probe, st));
    chk(h2d(probe_dev, probe, st));
  }
  chk(h2d(w.desc, bd, st));
  if (init_dev) chk(hipMemcpyAsync(w.init, init_dev, 4ull * (m.d.P + 1), hipMemcpyDeviceToDevice, st));
  else chk(launch_init_params(m.d, cfg->seed, w.init, st));
  chk(hipMemsetAsync(w.ctr, 0, 64 * sizeof(int), st));
  a.d = m.d;
  a.lay = m.lay;
  a.mode = 0;
  a.n_blocks = 1;
  a.blocks = w.desc;
  a.tokens = const_cast<uint8_t *>(tokens_dev);
  a.params = w.params;
  a.adam_m = w.adam_m;
  a.adam_v = w.adam_v;
  a.init = w.init;
  a.stat = static_dev;
  a.snap_flag = w.snap_flag;
  a.progress = w.progress;
  a.queue = w.ctr;
  a.err = w.ctr + 1;
  a.slots = w.slots;
  a.seg_bits = w.seg_bits;
  a.seg_words = w.seg_words;
  a.stop = stop;
  a.probe_steps = probe_dev;
  a.n_probe = (int)n_probe;
  a.probe_P = probs_dev;
  a.params_out = params_dev;
  a.act_scratch = w.act;
  a.w1f = w.w1f;
  a.s1f = w.s1f;
  a.spin_limit = 1ll << 30;
  if (w.s1f && static_dev) chk(launch_w1_frag(static_dev + m.d.off_W[0], m.d.D, m.d.H[0], w.s1f, st));
  chk(hipMemcpyAsync(w.args, &a, sizeof(StepArgs), hipMemcpyHostToDevice, st));
  if (e == hipSuccess) {
    chk(launch_kind(m, a, w.args, 1, m.nt, st));
  }
  int herr[2] = {0, 0};
  chk(hipMemcpyAsync(herr, w.ctr, 8, hipMemcpyDeviceToHost, st));
  // the segment streams, byte-aligned and concatenated in segment order (a
  // block's payload in the container)
  std::vector<uint32_t> bits, slots;
  if (streams_len && L > 0) {
    chk(d2h(bits, w.seg_bits, bs, st));
    chk(d2h(slots, w.slots, (uint64_t)slot_words_for(L) * bs, st));
  }
  chk(hipStreamSynchronize(st));
  uint64_t total = 0;
  for (uint32_t b : bits) total += (b + 7) / 8;
  if (e == hipSuccess && streams_len && total <= streams_cap && (streams_host || !total)) {
    uint64_t at = 0;
    for (uint32_t j = 0; j < bits.size(); j++) {
      const uint64_t nb = (bits[j] + 7) / 8;
      memcpy(streams_host + at, reinterpret_cast<const uint8_t *>(slots.data() + (uint64_t)j * slot_words_for(L)),
             nb);
      at += nb;
    }
  }
  (void)hipFreeAsync(base, st);
  if (probe_dev) (void)hipFreeAsync(probe_dev, st);
  (void)hipStreamSynchronize(st);
  if (e != hipSuccess || herr[1]) return PMKLC_ERR_DEVICE;
  if (streams_len) {
    *streams_len = total;
    if (total > streams_cap) return PMKLC_ERR_BUFFER_TOO_SMALL;
  }
  return PMKLC_OK;
}

}  // extern "C"
