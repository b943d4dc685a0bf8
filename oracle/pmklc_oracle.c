/*
 * PMKLC CPU oracle — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of what the PMKLC hot path computes,
 * written from the paper (arXiv 2507.12805).  Only the tests, the smoke
 * check and the bench's CPU-baseline leg may load it; the GPU library never
 * does, and the two share no code, header, table or helper.
 *
 * What each part follows:
 *   - (s,k)-mer encoding: Sec. 4.1 and Fig. 3 (bases A0 C1 G2 T3, window k,
 *     step s, first base most significant: "CGG" -> 26).
 *   - Online learning loop: Sec. 2 steps (1)-(4): context of t symbols,
 *     model -> distribution -> entropy coder, then cross-entropy and
 *     back-propagation; the first t symbols use a uniform distribution.
 *   - Mixer: Eq. (1), P = softmax(alpha*(S0*Lu + S1*Lr) + (1-alpha)*S2*Lm),
 *     alpha self-learned (Sec. 4.2.5).
 *   - Loss: Eq. (2), cross-entropy against the one-hot target (Sec. 4.2.6).
 *   - Blocks and step-wise model passing: Sec. 4.3 (even partition; after
 *     5% of a block the dynamic model seeds the next block).
 *   - Entropy coder: the paper names an entropy encoder only (Sec. 4); this
 *     oracle uses the integer arithmetic coder of Witten, Neal and Cleary
 *     (CACM 30(6), 1987) with 32-bit registers and a 2^16 frequency total.
 * Readings of points the paper leaves open (segment layout of a block,
 * MLP model shape, frequency quantisation, container layout) are the ones
 * listed with the design notes of this repository; each is restated at the
 * function that implements it.
 *
 * Parity status: every function here is pinned by a test against something
 * other than itself (brute force, closed forms, torch FP64 autograd, finite
 * differences, zlib), except the learned-model compression ratio on the
 * synthetic data, which the paper cannot pin (its datasets are not
 * available): parity unpinned for that value.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_ERR_ARG -1
#define OR_ERR_BASE -2
#define OR_ERR_SMALL -3
#define OR_ERR_CORRUPT -4
#define OR_ERR_MODEL -5
#define OR_ERR_NOMEM -8

#define TOTAL_BITS 16
#define TOTAL (1u << TOTAL_BITS)

/* ------------------------------------------------------------------ */
/* Bases and (s,k)-mers (Sec. 4.1, Fig. 3)                             */
/* ------------------------------------------------------------------ */

/* A->0 C->1 G->2 T->3; N -> 4; anything else -> 255. */
static int base_code(uint8_t c) {
    switch (c) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    case 'N': return 4;
    default: return 255;
    }
}
static const uint8_t LETTER[4] = {'A', 'C', 'G', 'T'};

/* Number of (s,k)-mers in n bases: windows start at 0, s, 2s, ... and must
 * fit entirely (a window never runs past the end). */
uint64_t or_skmer_count(uint64_t n, int s, int k) {
    if (s < 1 || k < 1 || n < (uint64_t)k) return 0;
    return (n - (uint64_t)k) / (uint64_t)s + 1;
}

/* Sec. 4.1: e_j = sum_{m<k} 4^(k-1-m) * b_{j*s+m}.  Input is ASCII ACGT only
 * (the paper's GD alphabet); anything else is an error. */
int or_encode_skmer(const uint8_t *ascii, uint64_t n, int s, int k, uint8_t *tokens,
                    uint64_t cap, uint64_t *n_tokens) {
    if (s < 1 || k < 1 || k > 4 || s > k) return OR_ERR_ARG;
    for (uint64_t i = 0; i < n; i++)
        if (base_code(ascii[i]) > 3) return OR_ERR_BASE;
    uint64_t l = or_skmer_count(n, s, k);
    if (n_tokens) *n_tokens = l;
    if (l > cap) return OR_ERR_SMALL;
    for (uint64_t j = 0; j < l; j++) {
        uint32_t e = 0;
        for (int m = 0; m < k; m++) {
            uint32_t pw = 1;
            for (int q = 0; q < k - 1 - m; q++) pw *= 4;
            e += pw * (uint32_t)base_code(ascii[j * (uint64_t)s + (uint64_t)m]);
        }
        tokens[j] = (uint8_t)e;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Frequency quantisation: probabilities -> integer CDF, total 2^16.     */
/* The paper only says that the mixed probability drives the entropy     */
/* coder.  Reading: f_v = 1 + floor(p_v * (2^16 - V)), the residual      */
/* 2^16 - sum f goes to the most probable symbol (lowest index on ties). */
/* ------------------------------------------------------------------ */
void or_quantise(const double *p, int V, uint32_t *cum) {
    int64_t sum = 0;
    int amax = 0;
    int64_t f[256];
    for (int v = 0; v < V; v++) {
        f[v] = 1 + (int64_t)floor(p[v] * (double)(TOTAL - (uint32_t)V));
        sum += f[v];
        if (p[v] > p[amax]) amax = v;
    }
    f[amax] += (int64_t)TOTAL - sum;
    cum[0] = 0;
    for (int v = 0; v < V; v++) cum[v + 1] = cum[v] + (uint32_t)f[v];
}

/* ------------------------------------------------------------------ */
/* Arithmetic coder (Witten-Neal-Cleary 1987), 32-bit, total 2^16.      */
/* Bits are written most significant first within each byte.           */
/* ------------------------------------------------------------------ */
#define HALF 0x80000000u
#define QUARTER 0x40000000u

typedef struct {
    uint32_t low, high;
    uint64_t pending;
    uint8_t *buf;
    uint64_t cap;   /* bytes */
    uint64_t nbits;
} or_enc;

static int enc_bit(or_enc *e, int bit) {
    uint64_t byte = e->nbits >> 3;
    if (byte >= e->cap) {
        uint64_t nc = e->cap ? 2 * e->cap : 64;
        uint8_t *nb = (uint8_t *)realloc(e->buf, nc);
        if (!nb) return OR_ERR_NOMEM;
        memset(nb + e->cap, 0, nc - e->cap);
        e->buf = nb;
        e->cap = nc;
    }
    if (bit) e->buf[byte] |= (uint8_t)(0x80u >> (e->nbits & 7));
    e->nbits++;
    return OR_OK;
}
static int enc_bit_plus_pending(or_enc *e, int bit) {
    int rc = enc_bit(e, bit);
    for (; rc == OR_OK && e->pending; e->pending--) rc = enc_bit(e, !bit);
    return rc;
}
static void enc_init(or_enc *e) { memset(e, 0, sizeof *e); e->high = 0xFFFFFFFFu; }

static int enc_symbol(or_enc *e, uint32_t cum_lo, uint32_t cum_hi) {
    uint64_t r = (uint64_t)e->high - e->low + 1;
    uint32_t lo = e->low;
    e->high = lo + (uint32_t)((r * cum_hi) >> TOTAL_BITS) - 1;
    e->low = lo + (uint32_t)((r * cum_lo) >> TOTAL_BITS);
    for (;;) {
        int rc = OR_OK;
        if (e->high < HALF) {
            rc = enc_bit_plus_pending(e, 0);
        } else if (e->low >= HALF) {
            rc = enc_bit_plus_pending(e, 1);
            e->low -= HALF;
            e->high -= HALF;
        } else if (e->low >= QUARTER && e->high < 3u * QUARTER) {
            e->pending++;
            e->low -= QUARTER;
            e->high -= QUARTER;
        } else {
            break;
        }
        if (rc) return rc;
        e->low <<= 1;
        e->high = (e->high << 1) | 1u;
    }
    return OR_OK;
}
static int enc_finish(or_enc *e) {
    e->pending++;
    return enc_bit_plus_pending(e, e->low < QUARTER ? 0 : 1);
}

typedef struct {
    uint32_t low, high, value;
    const uint8_t *buf;
    uint64_t nbytes, pos;
} or_dec;

static int dec_bit(or_dec *d) {
    uint64_t byte = d->pos >> 3;
    int b = byte < d->nbytes ? (d->buf[byte] >> (7 - (d->pos & 7))) & 1 : 0;
    d->pos++;
    return b;
}
static void dec_init(or_dec *d, const uint8_t *buf, uint64_t nbytes) {
    d->low = 0;
    d->high = 0xFFFFFFFFu;
    d->buf = buf;
    d->nbytes = nbytes;
    d->pos = 0;
    d->value = 0;
    for (int i = 0; i < 32; i++) d->value = (d->value << 1) | (uint32_t)dec_bit(d);
}
/* cum has V+1 entries. Returns the symbol. */
static int dec_symbol(or_dec *d, const uint32_t *cum, int V) {
    uint64_t r = (uint64_t)d->high - d->low + 1;
    uint32_t lo = d->low;
    /* largest s with lo + floor(r*cum[s]/T) <= value */
    int a = 0, b = V; /* invariant: bound(a) <= value < bound(b) */
    while (b - a > 1) {
        int m = (a + b) / 2;
        uint32_t bm = lo + (uint32_t)((r * cum[m]) >> TOTAL_BITS);
        if (bm <= d->value) a = m; else b = m;
    }
    int s = a;
    d->high = lo + (uint32_t)((r * cum[s + 1]) >> TOTAL_BITS) - 1;
    d->low = lo + (uint32_t)((r * cum[s]) >> TOTAL_BITS);
    for (;;) {
        if (d->high < HALF) {
        } else if (d->low >= HALF) {
            d->low -= HALF;
            d->high -= HALF;
            d->value -= HALF;
        } else if (d->low >= QUARTER && d->high < 3u * QUARTER) {
            d->low -= QUARTER;
            d->high -= QUARTER;
            d->value -= QUARTER;
        } else {
            break;
        }
        d->low <<= 1;
        d->high = (d->high << 1) | 1u;
        d->value = (d->value << 1) | (uint32_t)dec_bit(d);
    }
    return s;
}

/* Standalone coder entry points (used by the coder pins). */
int or_wnc_encode(const uint32_t *cum_lo, const uint32_t *cum_hi, uint64_t m, uint8_t **out,
                  uint64_t *nbits) {
    or_enc e;
    enc_init(&e);
    for (uint64_t i = 0; i < m; i++) {
        if (cum_hi[i] <= cum_lo[i] || cum_hi[i] > TOTAL) { free(e.buf); return OR_ERR_ARG; }
        int rc = enc_symbol(&e, cum_lo[i], cum_hi[i]);
        if (rc) { free(e.buf); return rc; }
    }
    int rc = enc_finish(&e);
    if (rc) { free(e.buf); return rc; }
    *out = e.buf;
    *nbits = e.nbits;
    return OR_OK;
}
/* cdfs: m rows of V+1 cumulative counts. */
int or_wnc_decode(const uint8_t *in, uint64_t nbytes, const uint32_t *cdfs, int V, uint64_t m,
                  uint32_t *symbols) {
    or_dec d;
    dec_init(&d, in, nbytes);
    for (uint64_t i = 0; i < m; i++) symbols[i] = (uint32_t)dec_symbol(&d, cdfs + i * (uint64_t)(V + 1), V);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* CRC-32 (IEEE 802.3 polynomial, reflected; same value as zlib.crc32).  */
/* ------------------------------------------------------------------ */
uint32_t or_crc32(const uint8_t *p, uint64_t n) {
    uint32_t c = 0xFFFFFFFFu;
    for (uint64_t i = 0; i < n; i++) {
        c ^= p[i];
        for (int b = 0; b < 8; b++) c = (c >> 1) ^ (0xEDB88320u & (0u - (c & 1u)));
    }
    return c ^ 0xFFFFFFFFu;
}

/* ------------------------------------------------------------------ */
/* Model: embedding + MLP (the configuration's reading of DM / SPuM).    */
/* Flat parameter order: Emb[V][E], then per layer l: W_l[d_l][d_{l+1}]   */
/* (input-major) and b_l[d_{l+1}]; d_0 = t*E, d_{nh+1} = V.              */
/* ------------------------------------------------------------------ */
/* arch 0: the MLP of the configurations (embedding, concatenation, hidden
 * Dense + ReLU layers, linear head).  arch 1: the paper's Transformer DM
 * (Sec. 4.2.4): embedding E plus a learned position embedding, one
 * attention layer of `heads` heads and width A = hidden[0], a shared FFN of
 * width F = hidden[1] with ReLU, a linear head to V, read at the last
 * context position.  Parameter order for arch 1: Emb[V][E], Pos[t][E],
 * Wqkv[E][3A], bqkv[3A], Wo[A][A], bo[A], W1[A][F], b1[F], W2[F][A], b2[A],
 * Wh[A][V], bh[V] (off_W / off_b 0..4 in that order, fan[l] their fan-in). */
typedef struct or_shape_s {
    int V, E, t, D, nh;
    int dims[6];
    uint64_t off_emb, off_W[5], off_b[5], n;
    int arch, heads, A, F;
    int fan[5];
    uint64_t off_pos;
    /* arch 2, the BiGRU static model: gh units per direction, gl layers,
     * gd-wide Dense; per layer l and direction d (0 forward, 1 backward):
     * W_ih [3gh][in_l], W_hh [3gh][gh], b_ih [3gh], b_hh [3gh] (gate rows
     * r, z, n), in_0 = E, in_1 = 2gh; then Wd [2gh][gd], bd, Wl [gd][V], bl */
    int gh, gl, gd;
    uint64_t off_wih[2][2], off_whh[2][2], off_bih[2][2], off_bhh[2][2], off_dw, off_db, off_lw, off_lb;
    /* the static model's shape when it differs from this (DM) shape, or NULL */
    const struct or_shape_s *ssh;
} or_shape;

/* The static model of Sec. 4.2.2 (reading): a 16-d embedding (E here),
 * gl bidirectional GRU layers (Cho et al. 2014, the gate form with the reset
 * gate applied to W_hn h + b_hn), the last layer's final states of both
 * directions (forward after position t-1, backward after position 0)
 * concatenated, a Dense layer of width gd with ReLU, a linear head to V. */
static int shape_init_gru(or_shape *sh, int k, int t, int E, int gh, int gl, int gd) {
    if (k < 1 || k > 4 || t < 1 || E < 1 || gh < 1 || gh > 256 || gl < 1 || gl > 2 || gd < 1) return OR_ERR_ARG;
    memset(sh, 0, sizeof *sh);
    sh->arch = 2;
    sh->V = 1 << (2 * k);
    sh->E = E;
    sh->t = t;
    sh->gh = gh;
    sh->gl = gl;
    sh->gd = gd;
    uint64_t off = 0;
    sh->off_emb = off;
    off += (uint64_t)sh->V * E;
    for (int l = 0; l < gl; l++) {
        int in = l == 0 ? E : 2 * gh;
        for (int d = 0; d < 2; d++) {
            sh->off_wih[l][d] = off; off += 3ull * gh * in;
            sh->off_whh[l][d] = off; off += 3ull * gh * gh;
            sh->off_bih[l][d] = off; off += 3ull * gh;
            sh->off_bhh[l][d] = off; off += 3ull * gh;
        }
    }
    sh->off_dw = off; off += 2ull * gh * gd;
    sh->off_db = off; off += (uint64_t)gd;
    sh->off_lw = off; off += (uint64_t)gd * sh->V;
    sh->off_lb = off; off += (uint64_t)sh->V;
    sh->n = off;
    return OR_OK;
}

static int shape_init_tf(or_shape *sh, int k, int t, int E, int nh, const int32_t *hidden, int heads) {
    if (nh != 2 || heads < 1 || hidden[0] < 1 || hidden[1] < 1 || hidden[0] % heads) return OR_ERR_ARG;
    int A = hidden[0], F = hidden[1];
    sh->V = 1 << (2 * k);
    sh->E = E;
    sh->t = t;
    sh->D = E;
    sh->nh = nh;
    sh->arch = 1;
    sh->heads = heads;
    sh->A = A;
    sh->F = F;
    int rows[5] = {E, A, A, F, A}, cols[5] = {3 * A, A, F, A, sh->V};
    uint64_t off = 0;
    sh->off_emb = off;
    off += (uint64_t)sh->V * E;
    sh->off_pos = off;
    off += (uint64_t)t * E;
    for (int l = 0; l < 5; l++) {
        sh->fan[l] = rows[l];
        sh->off_W[l] = off;
        off += (uint64_t)rows[l] * cols[l];
        sh->off_b[l] = off;
        off += (uint64_t)cols[l];
    }
    sh->n = off;
    return OR_OK;
}

static int shape_init(or_shape *sh, int k, int t, int E, int nh, const int32_t *hidden, int arch, int heads) {
    if (k < 1 || k > 4 || t < 1 || E < 1 || nh < 0 || nh > 4) return OR_ERR_ARG;
    memset(sh, 0, sizeof *sh);
    if (arch == 1) return shape_init_tf(sh, k, t, E, nh, hidden, heads);
    if (arch != 0) return OR_ERR_ARG;
    sh->V = 1 << (2 * k);
    sh->E = E;
    sh->t = t;
    sh->D = t * E;
    sh->nh = nh;
    sh->dims[0] = sh->D;
    for (int l = 0; l < nh; l++) {
        if (hidden[l] < 1) return OR_ERR_ARG;
        sh->dims[l + 1] = hidden[l];
    }
    sh->dims[nh + 1] = sh->V;
    uint64_t off = 0;
    sh->off_emb = off;
    off += (uint64_t)sh->V * E;
    for (int l = 0; l <= nh; l++) {
        sh->off_W[l] = off;
        off += (uint64_t)sh->dims[l] * sh->dims[l + 1];
        sh->off_b[l] = off;
        off += (uint64_t)sh->dims[l + 1];
    }
    sh->n = off;
    return OR_OK;
}

uint64_t or_param_count(int k, int t, int E, int nh, const int32_t *hidden, int arch, int heads) {
    or_shape sh;
    if (shape_init(&sh, k, t, E, nh, hidden, arch, heads)) return 0;
    return sh.n;
}

/* SplitMix64 (Steele, Lea, Flood 2014) in counter form: the i-th draw is
 * mix(seed + (i+1) * golden_gamma). */
static uint64_t splitmix_at(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* Initial weights: u = top 24 bits / 2^24, w = fp32((2u - 1) * a) with
 * a = 1 for the embeddings (token and, for arch 1, position) and
 * a = 1/sqrt(fan_in) for every linear weight and bias.  The oracle keeps
 * the FP64 value of the FP32 number. */
static void init_params(const or_shape *sh, uint64_t seed, double *w) {
    if (sh->arch == 2) {
        /* U(-a, a): a = 1 for the embedding, 1/sqrt(gh) for the GRU weights
         * and biases (the usual GRU range), 1/sqrt(fan_in) for the two
         * dense layers */
        for (uint64_t i = 0; i < sh->n; i++) {
            double a = 1.0;
            if (i >= sh->off_wih[0][0] && i < sh->off_dw) a = 1.0 / sqrt((double)sh->gh);
            else if (i >= sh->off_dw && i < sh->off_lw) a = 1.0 / sqrt(2.0 * sh->gh);
            else if (i >= sh->off_lw) a = 1.0 / sqrt((double)sh->gd);
            double u = (double)(splitmix_at(seed, i) >> 40) * (1.0 / 16777216.0);
            w[i] = (double)(float)((2.0 * u - 1.0) * a);
        }
        return;
    }
    int nl = sh->arch == 1 ? 5 : sh->nh + 1;
    for (uint64_t i = 0; i < sh->n; i++) {
        double a = 1.0;
        for (int l = 0; l < nl; l++) {
            uint64_t end = sh->arch == 1 ? (l + 1 < nl ? sh->off_W[l + 1] : sh->n)
                                         : sh->off_b[l] + (uint64_t)sh->dims[l + 1];
            if (i >= sh->off_W[l] && i < end)
                a = 1.0 / sqrt((double)(sh->arch == 1 ? sh->fan[l] : sh->dims[l]));
        }
        double u = (double)(splitmix_at(seed, i) >> 40) * (1.0 / 16777216.0);
        w[i] = (double)(float)((2.0 * u - 1.0) * a);
    }
}
int or_init_params(int k, int t, int E, int nh, const int32_t *hidden, int arch, int heads, uint64_t seed,
                   double *w) {
    or_shape sh;
    int rc = shape_init(&sh, k, t, E, nh, hidden, arch, heads);
    if (rc) return rc;
    init_params(&sh, seed, w);
    return OR_OK;
}

/* Forward of one row: x = concat(Emb[ctx_0..ctx_{t-1}]) (oldest first),
 * h_{l+1} = ReLU(h_l W_l + b_l), logits = h_nh W_nh + b_nh.
 * acts must hold sum_{l<=nh} dims[l] doubles (layer inputs), logits V. */
static void mlp_forward_row(const or_shape *sh, const double *w, const uint8_t *ctx, double *acts,
                            double *logits) {
    double *x = acts;
    for (int p = 0; p < sh->t; p++)
        for (int e = 0; e < sh->E; e++) x[p * sh->E + e] = w[sh->off_emb + (uint64_t)ctx[p] * sh->E + e];
    double *in = acts;
    for (int l = 0; l <= sh->nh; l++) {
        int di = sh->dims[l], dn = sh->dims[l + 1];
        double *out = (l == sh->nh) ? logits : in + di;
        const double *W = w + sh->off_W[l];
        const double *b = w + sh->off_b[l];
        for (int o = 0; o < dn; o++) out[o] = b[o];
        for (int d = 0; d < di; d++) {
            double xv = in[d];
            const double *Wr = W + (uint64_t)d * dn;
            for (int o = 0; o < dn; o++) out[o] += xv * Wr[o];
        }
        if (l < sh->nh)
            for (int o = 0; o < dn; o++) out[o] = out[o] > 0.0 ? out[o] : 0.0;
        in = out;
    }
}
/* Transformer DM forward of one row (Sec. 4.2.4, reading): with context
 * tokens c_0..c_{t-1} (oldest first),
 *   x_p = Emb[c_p] + Pos[p],  [q_p | k_p | v_p] = x_p Wqkv + bqkv,
 *   per head h over its dh = A/heads columns, at the last position:
 *     s_p = q_{t-1,h} . k_{p,h} / sqrt(dh),  a = softmax(s),  o_h = sum_p a_p v_{p,h},
 *   z = o Wo + bo,  u = ReLU(z W1 + b1),  g = u W2 + b2,  logits = g Wh + bh.
 * The prediction reads the last position only, so the position-wise FFN
 * is needed there alone.  act layout: X[t][E], QKV[t][3A], att[heads][t],
 * O[A], Z[A], U[F], G[A]. */
static uint64_t tf_act_len(const or_shape *sh) {
    return (uint64_t)sh->t * sh->E + (uint64_t)sh->t * 3 * sh->A + (uint64_t)sh->heads * sh->t + 3ull * sh->A +
           (uint64_t)sh->F + (uint64_t)sh->A;
}
static void linear_fwd(const double *in, int di, const double *W, const double *b, int dn, double *out) {
    for (int o = 0; o < dn; o++) out[o] = b[o];
    for (int d = 0; d < di; d++) {
        const double *Wr = W + (uint64_t)d * dn;
        for (int o = 0; o < dn; o++) out[o] += in[d] * Wr[o];
    }
}
static void tf_forward_row(const or_shape *sh, const double *w, const uint8_t *ctx, double *act, double *logits) {
    int t = sh->t, E = sh->E, A = sh->A, F = sh->F, H = sh->heads, dh = A / H;
    double *X = act, *QKV = X + (uint64_t)t * E, *att = QKV + (uint64_t)t * 3 * A, *O = att + (uint64_t)H * t;
    double *Z = O + A, *U = Z + A, *G = U + F;
    for (int p = 0; p < t; p++)
        for (int e = 0; e < E; e++)
            X[p * E + e] = w[sh->off_emb + (uint64_t)ctx[p] * E + e] + w[sh->off_pos + (uint64_t)p * E + e];
    for (int p = 0; p < t; p++)
        linear_fwd(X + (uint64_t)p * E, E, w + sh->off_W[0], w + sh->off_b[0], 3 * A, QKV + (uint64_t)p * 3 * A);
    const double *q = QKV + (uint64_t)(t - 1) * 3 * A;
    double scale = 1.0 / sqrt((double)dh);
    for (int h = 0; h < H; h++) {
        double *a = att + (uint64_t)h * t;
        for (int p = 0; p < t; p++) {
            const double *k = QKV + (uint64_t)p * 3 * A + A;
            double dot = 0.0;
            for (int d = 0; d < dh; d++) dot += q[h * dh + d] * k[h * dh + d];
            a[p] = dot * scale;
        }
        double mx = a[0];
        for (int p = 1; p < t; p++) if (a[p] > mx) mx = a[p];
        double sum = 0.0;
        for (int p = 0; p < t; p++) { a[p] = exp(a[p] - mx); sum += a[p]; }
        for (int p = 0; p < t; p++) a[p] /= sum;
        for (int d = 0; d < dh; d++) {
            double o = 0.0;
            for (int p = 0; p < t; p++) o += a[p] * QKV[(uint64_t)p * 3 * A + 2 * A + h * dh + d];
            O[h * dh + d] = o;
        }
    }
    linear_fwd(O, A, w + sh->off_W[1], w + sh->off_b[1], A, Z);
    linear_fwd(Z, A, w + sh->off_W[2], w + sh->off_b[2], F, U);
    for (int f = 0; f < F; f++) U[f] = U[f] > 0.0 ? U[f] : 0.0;
    linear_fwd(U, F, w + sh->off_W[3], w + sh->off_b[3], A, G);
    linear_fwd(G, A, w + sh->off_W[4], w + sh->off_b[4], sh->V, logits);
}
/* Backward of a linear layer out = in W + b given dout: accumulates the
 * weight and bias gradients and returns din = W dout (din may be NULL). */
static void linear_bwd(const double *in, int di, const double *W, int dn, const double *dout, double *gW, double *gb,
                       double *din) {
    for (int o = 0; o < dn; o++) gb[o] += dout[o];
    for (int d = 0; d < di; d++) {
        const double *Wr = W + (uint64_t)d * dn;
        double *gWr = gW + (uint64_t)d * dn;
        double s = 0.0;
        for (int o = 0; o < dn; o++) {
            gWr[o] += in[d] * dout[o];
            s += Wr[o] * dout[o];
        }
        if (din) din[d] = s;
    }
}
static uint64_t tf_scratch_len(const or_shape *sh) {
    return 3ull * sh->A + (uint64_t)sh->F + (uint64_t)sh->t * 3 * sh->A + (uint64_t)sh->t * sh->E + (uint64_t)sh->t;
}
/* Backward of one row through the forward above (pre-update weights),
 * accumulating into grad; scratch holds tf_scratch_len doubles. */
static void tf_backward_row(const or_shape *sh, const double *w, const uint8_t *ctx, const double *act,
                            const double *dlogits, double *grad, double *scratch) {
    int t = sh->t, E = sh->E, A = sh->A, F = sh->F, H = sh->heads, dh = A / H;
    const double *X = act, *QKV = X + (uint64_t)t * E, *att = QKV + (uint64_t)t * 3 * A, *O = att + (uint64_t)H * t;
    const double *Z = O + A, *U = Z + A, *G = U + F;
    double *dG = scratch, *dU = dG + A, *dZ = dU + F, *dO = dZ + A, *dQKV = dO + A, *dX = dQKV + (uint64_t)t * 3 * A;
    double *da = dX + (uint64_t)t * E;
    linear_bwd(G, A, w + sh->off_W[4], sh->V, dlogits, grad + sh->off_W[4], grad + sh->off_b[4], dG);
    linear_bwd(U, F, w + sh->off_W[3], A, dG, grad + sh->off_W[3], grad + sh->off_b[3], dU);
    for (int f = 0; f < F; f++) dU[f] = U[f] > 0.0 ? dU[f] : 0.0;   /* ReLU'(0) = 0 */
    linear_bwd(Z, A, w + sh->off_W[2], F, dU, grad + sh->off_W[2], grad + sh->off_b[2], dZ);
    linear_bwd(O, A, w + sh->off_W[1], A, dZ, grad + sh->off_W[1], grad + sh->off_b[1], dO);
    memset(dQKV, 0, sizeof(double) * (uint64_t)t * 3 * A);
    const double *q = QKV + (uint64_t)(t - 1) * 3 * A;
    double *dq = dQKV + (uint64_t)(t - 1) * 3 * A;
    double scale = 1.0 / sqrt((double)dh);
    for (int h = 0; h < H; h++) {
        const double *a = att + (uint64_t)h * t;
        double dot = 0.0;
        for (int p = 0; p < t; p++) {
            const double *v = QKV + (uint64_t)p * 3 * A + 2 * A + h * dh;
            double *dv = dQKV + (uint64_t)p * 3 * A + 2 * A + h * dh;
            da[p] = 0.0;
            for (int d = 0; d < dh; d++) {
                dv[d] = a[p] * dO[h * dh + d];
                da[p] += dO[h * dh + d] * v[d];
            }
            dot += a[p] * da[p];
        }
        for (int p = 0; p < t; p++) {
            double ds = a[p] * (da[p] - dot) * scale;   /* softmax backward, then the 1/sqrt(dh) */
            const double *k = QKV + (uint64_t)p * 3 * A + A + h * dh;
            double *dk = dQKV + (uint64_t)p * 3 * A + A + h * dh;
            for (int d = 0; d < dh; d++) {
                dq[h * dh + d] += ds * k[d];
                dk[d] = ds * q[h * dh + d];
            }
        }
    }
    for (int p = 0; p < t; p++)
        linear_bwd(X + (uint64_t)p * E, E, w + sh->off_W[0], 3 * A, dQKV + (uint64_t)p * 3 * A, grad + sh->off_W[0],
                   grad + sh->off_b[0], dX + (uint64_t)p * E);
    for (int p = 0; p < t; p++)
        for (int e = 0; e < E; e++) {
            grad[sh->off_emb + (uint64_t)ctx[p] * E + e] += dX[p * E + e];
            grad[sh->off_pos + (uint64_t)p * E + e] += dX[p * E + e];
        }
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* BiGRU static model forward of one row; act holds gl t 2gh + 6gh + gd
 * doubles: each layer's output sequence [t][2gh] (forward half, backward
 * half), the gate scratch, the Dense output. */
static uint64_t gru_act_len(const or_shape *sh) {
    return (uint64_t)sh->gl * sh->t * 2 * sh->gh + 6ull * sh->gh + (uint64_t)sh->gd;
}
static void gru_forward_row(const or_shape *sh, const double *w, const uint8_t *ctx, double *act, double *logits) {
    int t = sh->t, E = sh->E, h = sh->gh;
    double *gx = act + (uint64_t)sh->gl * t * 2 * h, *gh_ = gx + 3 * h, *dense = gh_ + 3 * h;
    const double *last = NULL;
    for (int l = 0; l < sh->gl; l++) {
        int in = l == 0 ? E : 2 * h;
        double *out = act + (uint64_t)l * t * 2 * h;
        for (int d = 0; d < 2; d++) {
            const double *Wih = w + sh->off_wih[l][d], *Whh = w + sh->off_whh[l][d];
            const double *bih = w + sh->off_bih[l][d], *bhh = w + sh->off_bhh[l][d];
            double hs[256];
            for (int u = 0; u < h; u++) hs[u] = 0.0;
            for (int step = 0; step < t; step++) {
                int p = d == 0 ? step : t - 1 - step;
                const double *x = l == 0 ? w + sh->off_emb + (uint64_t)ctx[p] * E : last + (uint64_t)p * 2 * h;
                for (int g = 0; g < 3 * h; g++) {
                    double a = bih[g], b = bhh[g];
                    for (int i = 0; i < in; i++) a += Wih[(uint64_t)g * in + i] * x[i];
                    for (int i = 0; i < h; i++) b += Whh[(uint64_t)g * h + i] * hs[i];
                    gx[g] = a;
                    gh_[g] = b;
                }
                for (int u = 0; u < h; u++) {
                    double r = sigmoid(gx[u] + gh_[u]);
                    double z = sigmoid(gx[h + u] + gh_[h + u]);
                    double nn = tanh(gx[2 * h + u] + r * gh_[2 * h + u]);
                    hs[u] = (1.0 - z) * nn + z * hs[u];
                    out[(uint64_t)p * 2 * h + d * h + u] = hs[u];
                }
            }
        }
        last = out;
    }
    /* final states: forward after position t-1, backward after position 0 */
    double feat[512];
    for (int u = 0; u < h; u++) {
        feat[u] = last[(uint64_t)(t - 1) * 2 * h + u];
        feat[h + u] = last[h + u];
    }
    linear_fwd(feat, 2 * h, w + sh->off_dw, w + sh->off_db, sh->gd, dense);
    for (int o = 0; o < sh->gd; o++) dense[o] = dense[o] > 0.0 ? dense[o] : 0.0;
    linear_fwd(dense, sh->gd, w + sh->off_lw, w + sh->off_lb, sh->V, logits);
}

/* Backward of the one-layer BiGRU static model for one row, given dlogits
 * (used when the private static model has this shape and is trained on the
 * input).  act is the row's forward (gru_forward_row): the layer's output
 * sequence and the post-ReLU Dense output.  Back-propagation through time,
 * written from the gate equations of gru_forward_row: for each direction,
 * from its final state back to its first position, with the gates of a
 * position recomputed from the stored states.  With s the pre-activations
 * (a = W_i x + b_i, b = W_h h + b_h per gate row):
 *   r = sig(a_r + b_r), z = sig(a_z + b_z), n = tanh(a_n + r b_n),
 *   h' = (1 - z) n + z h;
 *   dn = dh' (1 - z), dz = dh' (h - n), dh = dh' z (direct part);
 *   dA_n = dn (1 - n^2), dA_r = dA_n b_n r (1 - r), dA_z = dz z (1 - z);
 *   input rows (dA_r, dA_z, dA_n) -> dW_i += . x, db_i, dx += W_i^T .;
 *   hidden rows (dA_r, dA_z, dA_n r) -> dW_h += . h, db_h, dh += W_h^T .;
 * dx lands on the embedding row of the position's token. */
static uint64_t gru_scratch_len(const or_shape *sh) {
    return (uint64_t)sh->gd + 13ull * sh->gh + (uint64_t)sh->E + 8;
}
static void gru_backward_row(const or_shape *sh, const double *w, const uint8_t *ctx, const double *act,
                             const double *dlogits, double *grad, double *scratch) {
    int t = sh->t, E = sh->E, h = sh->gh, gd = sh->gd, V = sh->V;
    const double *out = act, *dense = act + (uint64_t)t * 2 * h + 6ull * h;
    double *dd = scratch, *dfeat = dd + gd, *ga = dfeat + 2 * h, *gb = ga + 3 * h, *gi = gb + 3 * h,
           *dh = gi + 3 * h, *dx = dh + h;   /* gd + 12 h + E doubles */
    double feat[512];
    for (int u = 0; u < h; u++) {
        feat[u] = out[(uint64_t)(t - 1) * 2 * h + u];
        feat[h + u] = out[h + u];
    }
    /* head and Dense (ReLU) */
    for (int o = 0; o < gd; o++) {
        double sacc = 0.0;
        for (int v = 0; v < V; v++) {
            grad[sh->off_lw + (uint64_t)o * V + v] += dense[o] * dlogits[v];
            sacc += w[sh->off_lw + (uint64_t)o * V + v] * dlogits[v];
        }
        dd[o] = dense[o] > 0.0 ? sacc : 0.0;
    }
    for (int v = 0; v < V; v++) grad[sh->off_lb + v] += dlogits[v];
    for (int i = 0; i < 2 * h; i++) {
        double sacc = 0.0;
        for (int o = 0; o < gd; o++) {
            grad[sh->off_dw + (uint64_t)i * gd + o] += feat[i] * dd[o];
            sacc += w[sh->off_dw + (uint64_t)i * gd + o] * dd[o];
        }
        dfeat[i] = sacc;
    }
    for (int o = 0; o < gd; o++) grad[sh->off_db + o] += dd[o];
    /* through time, each direction from its final state */
    for (int d = 0; d < 2; d++) {
        const double *Wih = w + sh->off_wih[0][d], *Whh = w + sh->off_whh[0][d];
        const double *bih = w + sh->off_bih[0][d], *bhh = w + sh->off_bhh[0][d];
        double *gWih = grad + sh->off_wih[0][d], *gWhh = grad + sh->off_whh[0][d];
        double *gbih = grad + sh->off_bih[0][d], *gbhh = grad + sh->off_bhh[0][d];
        for (int u = 0; u < h; u++) dh[u] = dfeat[d * h + u];
        for (int step = t - 1; step >= 0; step--) {
            int p = d == 0 ? step : t - 1 - step;
            int pp = d == 0 ? p - 1 : p + 1;          /* the position processed before p */
            const double *hp = step > 0 ? out + (uint64_t)pp * 2 * h + d * h : NULL;
            const double *x = w + sh->off_emb + (uint64_t)ctx[p] * E;
            for (int g = 0; g < 3 * h; g++) {
                double a = bih[g], b = bhh[g];
                for (int i = 0; i < E; i++) a += Wih[(uint64_t)g * E + i] * x[i];
                if (hp)
                    for (int i = 0; i < h; i++) b += Whh[(uint64_t)g * h + i] * hp[i];
                ga[g] = a;
                gb[g] = b;
            }
            for (int u = 0; u < h; u++) {
                double r = sigmoid(ga[u] + gb[u]);
                double z = sigmoid(ga[h + u] + gb[h + u]);
                double nn = tanh(ga[2 * h + u] + r * gb[2 * h + u]);
                double hprev = hp ? hp[u] : 0.0;
                double dn = dh[u] * (1.0 - z), dz = dh[u] * (hprev - nn);
                double dan = dn * (1.0 - nn * nn);
                gi[u] = dan * gb[2 * h + u] * r * (1.0 - r);
                gi[h + u] = dz * z * (1.0 - z);
                gi[2 * h + u] = dan;
                dh[u] = dh[u] * z;                     /* direct part of dh */
                ga[u] = r;                             /* keep r for the hidden rows */
            }
            /* input rows */
            for (int e = 0; e < E; e++) dx[e] = 0.0;
            for (int g = 0; g < 3 * h; g++) {
                gbih[g] += gi[g];
                for (int i = 0; i < E; i++) {
                    gWih[(uint64_t)g * E + i] += gi[g] * x[i];
                    dx[i] += Wih[(uint64_t)g * E + i] * gi[g];
                }
            }
            for (int e = 0; e < E; e++) grad[sh->off_emb + (uint64_t)ctx[p] * E + e] += dx[e];
            /* hidden rows: (dA_r, dA_z, dA_n r) */
            for (int g = 0; g < 3 * h; g++) {
                double gh = g < 2 * h ? gi[g] : gi[g] * ga[g - 2 * h];
                gbhh[g] += gh;
                if (hp)
                    for (int i = 0; i < h; i++) {
                        gWhh[(uint64_t)g * h + i] += gh * hp[i];
                        dh[i] += Whh[(uint64_t)g * h + i] * gh;
                    }
            }
        }
    }
}

static uint64_t acts_len(const or_shape *sh) {
    if (sh->arch == 2) return gru_act_len(sh);
    if (sh->arch == 1) return tf_act_len(sh);
    uint64_t s = 0;
    for (int l = 0; l <= sh->nh; l++) s += (uint64_t)sh->dims[l];
    return s;
}
static void forward_row(const or_shape *sh, const double *w, const uint8_t *ctx, double *acts, double *logits) {
    if (sh->arch == 2) gru_forward_row(sh, w, ctx, acts, logits);
    else if (sh->arch == 1) tf_forward_row(sh, w, ctx, acts, logits);
    else mlp_forward_row(sh, w, ctx, acts, logits);
}

/* Backward of one row given dlogits; accumulates into grad (same layout as
 * the parameters).  ReLU'(0) = 0. Uses the pre-update weights. */
static void mlp_backward_row(const or_shape *sh, const double *w, const uint8_t *ctx, const double *acts,
                             const double *dlogits, double *grad, double *scratch) {
    /* scratch: two buffers of max dim */
    int maxd = 0;
    for (int l = 0; l <= sh->nh + 1; l++) if (sh->dims[l] > maxd) maxd = sh->dims[l];
    double *dout = scratch, *din = scratch + maxd;
    memcpy(dout, dlogits, sizeof(double) * (size_t)sh->V);
    /* layer inputs: layer l input starts at acts + sum_{q<l} dims[q] */
    uint64_t in_off[6];
    in_off[0] = 0;
    for (int l = 1; l <= sh->nh; l++) in_off[l] = in_off[l - 1] + (uint64_t)sh->dims[l - 1];
    for (int l = sh->nh; l >= 0; l--) {
        int di = sh->dims[l], dn = sh->dims[l + 1];
        const double *in = acts + in_off[l];
        const double *W = w + sh->off_W[l];
        double *gW = grad + sh->off_W[l];
        double *gb = grad + sh->off_b[l];
        for (int o = 0; o < dn; o++) gb[o] += dout[o];
        for (int d = 0; d < di; d++) {
            double s = 0.0;
            const double *Wr = W + (uint64_t)d * dn;
            double *gWr = gW + (uint64_t)d * dn;
            for (int o = 0; o < dn; o++) {
                gWr[o] += in[d] * dout[o];
                s += Wr[o] * dout[o];
            }
            din[d] = s;
        }
        if (l > 0) /* through the ReLU that produced this layer's input */
            for (int d = 0; d < di; d++) din[d] = in[d] > 0.0 ? din[d] : 0.0;
        double *tmp = dout; dout = din; din = tmp;
    }
    /* dout now holds dL/dx (t*E); scatter into the embedding rows */
    for (int p = 0; p < sh->t; p++)
        for (int e = 0; e < sh->E; e++) grad[sh->off_emb + (uint64_t)ctx[p] * sh->E + e] += dout[p * sh->E + e];
}

/* One learning step over bs rows (Sec. 2 steps (3)-(4); Eq. (1), Eq. (2)).
 *   ctx: bs x t tokens (oldest first), tgt: bs targets.
 *   w: DM parameters; ws: static parameters or NULL (S0 = 0).
 *   a_alpha: pre-sigmoid mixing parameter (used only when ws != NULL).
 * Outputs: P (bs x V, may be NULL), grad (n params, zeroed here, may be
 * NULL = forward only), *g_alpha, *loss = mean cross-entropy in nats.
 * The per-step loss is the mean over the bs rows (Eq. (2) summed over one
 * step, divided by bs). */
static int step_grad(const or_shape *sh, const double *w, const double *ws, double a_alpha, const uint8_t *ctx,
                     const uint8_t *tgt, int bs, double *P, double *grad, double *g_alpha, double *loss) {
    int V = sh->V;
    const or_shape *ssh = sh->ssh ? sh->ssh : sh;   /* the static model's shape */
    uint64_t al = acts_len(sh), als = acts_len(ssh);
    uint64_t maxd = 0;
    for (int l = 0; l <= sh->nh + 1; l++) if ((uint64_t)sh->dims[l] > maxd) maxd = (uint64_t)sh->dims[l];
    uint64_t scr = sh->arch == 1 ? tf_scratch_len(sh) : sh->arch == 2 ? gru_scratch_len(sh) : 2 * maxd;
    double *acts = (double *)malloc(sizeof(double) * (al + als + 4 * (uint64_t)V + scr));
    if (!acts) return OR_ERR_NOMEM;
    double *acts_s = acts + al;
    double *lm = acts_s + als, *lu = lm + V, *z = lu + V, *dz = z + V, *scratch = dz + V;
    double alpha = 1.0 / (1.0 + exp(-a_alpha));
    if (grad) memset(grad, 0, sizeof(double) * sh->n);
    double ga = 0.0, L = 0.0;
    for (int j = 0; j < bs; j++) {
        const uint8_t *c = ctx + (uint64_t)j * sh->t;
        forward_row(sh, w, c, acts, lm);
        if (ws) {
            forward_row(ssh, ws, c, acts_s, lu);
            for (int v = 0; v < V; v++) z[v] = alpha * lu[v] + (1.0 - alpha) * lm[v];
        } else {
            for (int v = 0; v < V; v++) z[v] = lm[v];
        }
        double mx = z[0];
        for (int v = 1; v < V; v++) if (z[v] > mx) mx = z[v];
        double sum = 0.0;
        for (int v = 0; v < V; v++) sum += exp(z[v] - mx);
        double *Pj = P ? P + (uint64_t)j * V : dz;
        for (int v = 0; v < V; v++) Pj[v] = exp(z[v] - mx) / sum;
        if (loss) L += -log(Pj[tgt[j]]);
        if (grad) {
            for (int v = 0; v < V; v++) dz[v] = (Pj[v] - (v == tgt[j] ? 1.0 : 0.0)) / (double)bs;
            if (ws) {
                for (int v = 0; v < V; v++) ga += dz[v] * (lu[v] - lm[v]);
                for (int v = 0; v < V; v++) dz[v] *= (1.0 - alpha);
            }
            if (sh->arch == 1) tf_backward_row(sh, w, c, acts, dz, grad, scratch);
            else if (sh->arch == 2) gru_backward_row(sh, w, c, acts, dz, grad, scratch);
            else mlp_backward_row(sh, w, c, acts, dz, grad, scratch);
        }
    }
    if (g_alpha) *g_alpha = ws ? ga * alpha * (1.0 - alpha) : 0.0;
    if (loss) *loss = L / (double)bs;
    free(acts);
    return OR_OK;
}

/* Exported single step for the forward/backward pins. */
int or_step(int k, int t, int E, int nh, const int32_t *hidden, int arch, int heads, const double *w,
            const double *ws, double a_alpha, const uint8_t *ctx, const uint8_t *tgt, int bs, double *P,
            double *grad, double *g_alpha, double *loss) {
    or_shape sh;
    int rc = shape_init(&sh, k, t, E, nh, hidden, arch, heads);
    if (rc) return rc;
    return step_grad(&sh, w, ws, a_alpha, ctx, tgt, bs, P, grad, g_alpha, loss);
}

/* ------------------------------------------------------------------ */
/* Optimisers.  The paper says only "back-propagation" (Sec. 2 (4)); the  */
/* configurations fix plain SGD, or Adam with bias correction.           */
/* ------------------------------------------------------------------ */
typedef struct {
    int kind; /* 0 SGD, 1 Adam */
    double lr, b1, b2, eps;
} or_opt;

static void opt_apply(const or_opt *o, double *w, const double *g, double *m, double *v, uint64_t n, uint64_t tau) {
    if (o->kind == 0) {
        for (uint64_t i = 0; i < n; i++) w[i] -= o->lr * g[i];
    } else {
        double c1 = 1.0 - pow(o->b1, (double)tau), c2 = 1.0 - pow(o->b2, (double)tau);
        for (uint64_t i = 0; i < n; i++) {
            m[i] = o->b1 * m[i] + (1.0 - o->b1) * g[i];
            v[i] = o->b2 * v[i] + (1.0 - o->b2) * g[i] * g[i];
            double mh = m[i] / c1, vh = v[i] / c2;
            w[i] -= o->lr * mh / (sqrt(vh) + o->eps);
        }
    }
}
/* Exported for the optimiser pins (tau = 1-based update count). */
void or_opt_step(int kind, double lr, double b1, double b2, double eps, double *w, const double *g, double *m,
                 double *v, uint64_t n, uint64_t tau) {
    or_opt o = {kind, lr, b1, b2, eps};
    opt_apply(&o, w, g, m, v, n, tau);
}

/* ------------------------------------------------------------------ */
/* Configuration and block plan.                                       */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t s, k, t, bs, E, nh;
    int32_t hidden[4];
    int32_t optimizer;
    float lr, beta1, beta2, eps;
    int32_t selector;        /* bit0: static public model, bit1: static private model, bit2: dynamic
                                model; 0 = uniform; 8 = chosen by the Model Selector */
    uint32_t smp_ppm;        /* step-wise model passing point, parts per million of the block's steps; 0 = off */
    uint64_t seed;
    int32_t n_blocks;
    const uint64_t *block_len; /* raw bytes per block, or NULL = equal split */
    int32_t n_files;
    const uint64_t *file_blocks; /* blocks per file, or NULL = one file */
    const double *init_override; /* test hook: initial DM parameters (+ a_alpha) of every chain head, or NULL */
    uint64_t ms_threshold;   /* Model Selector size bound in input bytes; 0 = 500 * 10^6 */
    int32_t arch;            /* dynamic model: 0 MLP, 1 Transformer (hidden = {A, F}, nh = 2) */
    int32_t heads;           /* attention heads (arch 1) */
    int32_t static_arch;     /* static public model: 0 the DM's shape, 1 BiGRU (Sec. 4.2.2) */
    int32_t static_E, gru_h, gru_layers, dense;   /* BiGRU: embedding, units per direction, layers, Dense */
} or_config;

#define SEL_SPUM 1
#define SEL_SPRM 2
#define SEL_DM 4
#define SEL_AUTO 8

/* Sec. 4.2.1: the selector enables the public static model for inputs of at
 * most 500 MB and the private one above (MB read as 10^6 bytes). */
#define MS_BYTES_DEFAULT 500000000ull
/* Training of the private static model (Sec. 4.2.3, pipeline stage (b));
 * the paper gives no budget or seed, these are this implementation's. */
#define SPRM_STEPS 8192u
#define SPRM_SEED_XOR 0x5350524Dull

typedef struct {
    uint64_t raw_off, raw_len;
    /* derived */
    uint64_t n_runs;
    uint64_t *run_start, *run_len; /* block-relative raw coordinates */
    uint64_t nb;                    /* stripped bases */
    uint8_t *codes;                 /* stripped bases 0..3 */
    uint64_t l, L, rem, tail;
    uint8_t *tok;
    int has_pred;                   /* previous block of the same file exists */
    /* coded output */
    uint8_t **seg_buf;
    uint64_t *seg_bytes;
    uint8_t *extras;
    uint64_t extras_bytes;
    double *snap;                   /* parameters (+ alpha) after the SMP step */
} or_block;

static int model_on(const or_config *c) { return (c->selector & SEL_DM) != 0; }
static int static_on(const or_config *c) { return (c->selector & (SEL_SPUM | SEL_SPRM)) != 0; }
static int private_on(const or_config *c) { return (c->selector & SEL_SPRM) != 0; }

/* Sec. 4.2.1: S for an input of n bytes.  Above the size bound the private
 * model and DM; otherwise the public model and DM when a public model is
 * supplied (the paper's is built in; here the caller holds it), else DM. */
/* The static public model's shape when it is not the DM's (BiGRU); sh->ssh
 * then points to it.  ssh must outlive sh's use. */
static int static_shape(const or_config *c, or_shape *sh, or_shape *ssh) {
    sh->ssh = NULL;
    if (c->static_arch != 1) return OR_OK;
    int rc = shape_init_gru(ssh, c->k, c->t, c->static_E, c->gru_h, c->gru_layers, c->dense);
    if (rc) return rc;
    sh->ssh = ssh;
    return OR_OK;
}

static int32_t ms_select(const or_config *c, uint64_t n, int have_public) {
    uint64_t bound = c->ms_threshold ? c->ms_threshold : MS_BYTES_DEFAULT;
    if (n > bound) return SEL_SPRM | SEL_DM;
    return have_public ? (SEL_SPUM | SEL_DM) : SEL_DM;
}

static uint64_t smp_steps(uint32_t ppm, uint64_t L) {
    return (uint64_t)(((unsigned __int128)ppm * L + 999999u) / 1000000u);
}

/* Run one block's learning/coding loop.  Sec. 2: for each target, the
 * model predicts from the previous t tokens, the coder codes it, then the
 * cross-entropy gradient updates the model.  Reading of the batch size bs:
 * the block's first bs*L tokens form bs contiguous segments of L tokens;
 * step i predicts token i of every segment at once (one row per segment)
 * and makes one update with the mean loss of those bs rows.  The first t
 * tokens of every segment are coded with the uniform distribution and do
 * not train the model.
 *   mode 0: encode (blk->tok known), mode 1: decode (fills blk->tok).
 *   init: initial DM parameters followed by a_alpha.
 *   probe: optional callback storage for P of sampled steps (trace API). */
typedef struct {
    uint64_t stop;        /* run only this many steps (0 = all) */
    double *P_out;        /* (n_steps_probe) x bs x V, or NULL */
    const uint64_t *steps;
    uint64_t n_steps;
    double *w_final;      /* n params + 1, or NULL */
    double *loss_out;     /* L values, or NULL */
} or_probe;

static int run_block(const or_config *cfg, const or_shape *sh, const double *ws, or_block *blk, const double *init,
                     int mode, const uint8_t *stream_region, or_probe *probe) {
    int V = sh->V, bs = cfg->bs, t = cfg->t;
    uint64_t L = blk->L, n = sh->n;
    uint32_t ucum[257];
    for (int v = 0; v <= V; v++) ucum[v] = (uint32_t)((uint64_t)v * TOTAL / (uint64_t)V);
    or_opt opt = {cfg->optimizer, (double)cfg->lr, (double)cfg->beta1, (double)cfg->beta2, (double)cfg->eps};
    int rc = OR_OK;
    double *w = NULL, *g = NULL, *m = NULL, *vv = NULL, *P = NULL;
    uint8_t *ctx = NULL, *tgt = NULL;
    uint32_t *cum = NULL;
    or_enc *enc = NULL;
    or_dec *dec = NULL;
    if (L == 0) {
        if (blk->snap && init) memcpy(blk->snap, init, sizeof(double) * (n + 1));
        return OR_OK;
    }
    w = (double *)malloc(sizeof(double) * (n + 1));
    g = (double *)malloc(sizeof(double) * (n + 1));
    m = (double *)calloc(n + 1, sizeof(double));
    vv = (double *)calloc(n + 1, sizeof(double));
    P = (double *)malloc(sizeof(double) * (uint64_t)bs * V);
    ctx = (uint8_t *)malloc((uint64_t)bs * t);
    tgt = (uint8_t *)malloc((uint64_t)bs);
    cum = (uint32_t *)malloc(sizeof(uint32_t) * (uint64_t)(V + 1) * bs);
    if (mode == 0) enc = (or_enc *)calloc((uint64_t)bs, sizeof(or_enc));
    else dec = (or_dec *)calloc((uint64_t)bs, sizeof(or_dec));
    if (!w || !g || !m || !vv || !P || !ctx || !tgt || !cum || (!enc && !dec)) { rc = OR_ERR_NOMEM; goto done; }
    if (init) memcpy(w, init, sizeof(double) * (n + 1));
    else memset(w, 0, sizeof(double) * (n + 1));
    if (mode == 0) {
        for (int j = 0; j < bs; j++) enc_init(&enc[j]);
    } else {
        const uint8_t *p = stream_region;
        for (int j = 0; j < bs; j++) {
            dec_init(&dec[j], p, blk->seg_bytes[j]);
            p += blk->seg_bytes[j];
        }
    }
    uint64_t S = smp_steps(cfg->smp_ppm, L);
    if (blk->snap && S == 0) memcpy(blk->snap, w, sizeof(double) * (n + 1));
    uint64_t tau = 0, probe_i = 0;
    int use_model = model_on(cfg);
    uint64_t L_run = (probe && probe->stop && probe->stop < L) ? probe->stop : L;
    for (uint64_t i = 0; i < L_run; i++) {
        int uniform = !use_model || i < (uint64_t)t;
        double loss = 0.0, ga = 0.0;
        if (!uniform) {
            for (int j = 0; j < bs; j++)
                for (int p = 0; p < t; p++) ctx[(uint64_t)j * t + p] = blk->tok[(uint64_t)j * L + i - (uint64_t)t + (uint64_t)p];
            /* forward (and, for encode, the gradient needs the target: do the
             * forward first, code, then the backward with the known target) */
            rc = step_grad(sh, w, ws, w[n], ctx, tgt, bs, P, NULL, NULL, NULL);
            if (rc) goto done;
            for (int j = 0; j < bs; j++) or_quantise(P + (uint64_t)j * V, V, cum + (uint64_t)j * (V + 1));
        }
        for (int j = 0; j < bs; j++) {
            const uint32_t *c = uniform ? ucum : cum + (uint64_t)j * (V + 1);
            uint64_t pos = (uint64_t)j * L + i;
            if (mode == 0) {
                int e = blk->tok[pos];
                rc = enc_symbol(&enc[j], c[e], c[e + 1]);
                if (rc) goto done;
            } else {
                blk->tok[pos] = (uint8_t)dec_symbol(&dec[j], c, V);
            }
            tgt[j] = blk->tok[pos];
        }
        if (!uniform) {
            rc = step_grad(sh, w, ws, w[n], ctx, tgt, bs, P, g, &ga, &loss);
            if (rc) goto done;
            g[n] = ga;
            tau++;
            opt_apply(&opt, w, g, m, vv, ws ? n + 1 : n, tau);
            if (probe && probe->loss_out) probe->loss_out[i] = loss;
        }
        if (probe && probe->P_out && probe_i < probe->n_steps && probe->steps[probe_i] == i) {
            double *dst = probe->P_out + probe_i * (uint64_t)bs * V;
            if (uniform)
                for (uint64_t q = 0; q < (uint64_t)bs * V; q++) dst[q] = 1.0 / V;
            else
                memcpy(dst, P, sizeof(double) * (uint64_t)bs * V);
            probe_i++;
        }
        if (blk->snap && i + 1 == S) memcpy(blk->snap, w, sizeof(double) * (n + 1));
    }
    if (mode == 0) {
        blk->seg_buf = (uint8_t **)calloc((uint64_t)bs, sizeof(uint8_t *));
        blk->seg_bytes = (uint64_t *)calloc((uint64_t)bs, sizeof(uint64_t));
        if (!blk->seg_buf || !blk->seg_bytes) { rc = OR_ERR_NOMEM; goto done; }
        for (int j = 0; j < bs; j++) {
            rc = enc_finish(&enc[j]);
            if (rc) goto done;
            blk->seg_buf[j] = enc[j].buf;
            blk->seg_bytes[j] = (enc[j].nbits + 7) / 8;
            enc[j].buf = NULL;
        }
    }
    if (probe && probe->w_final) memcpy(probe->w_final, w, sizeof(double) * (n + 1));
done:
    if (enc) { for (int j = 0; j < bs; j++) free(enc[j].buf); free(enc); }
    free(dec);
    free(w); free(g); free(m); free(vv); free(P); free(ctx); free(tgt); free(cum);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Container (compressed binary file).  All integers little-endian;     */
/* varints are unsigned LEB128.                                         */
/* ------------------------------------------------------------------ */
typedef struct { uint8_t *p; uint64_t n, cap; int err; } or_buf;

static void buf_put(or_buf *b, const void *src, uint64_t n) {
    if (b->err) return;
    if (b->n + n > b->cap) {
        uint64_t nc = b->cap ? b->cap : 256;
        while (nc < b->n + n) nc *= 2;
        uint8_t *np = (uint8_t *)realloc(b->p, nc);
        if (!np) { b->err = 1; return; }
        b->p = np;
        b->cap = nc;
    }
    memcpy(b->p + b->n, src, n);
    b->n += n;
}
static void put_le(or_buf *b, uint64_t v, int nbytes) {
    uint8_t t[8];
    for (int i = 0; i < nbytes; i++) t[i] = (uint8_t)(v >> (8 * i));
    buf_put(b, t, (uint64_t)nbytes);
}
static void put_varint(or_buf *b, uint64_t v) {
    uint8_t t[10];
    int n = 0;
    do {
        uint8_t c = v & 0x7F;
        v >>= 7;
        t[n++] = (uint8_t)(c | (v ? 0x80 : 0));
    } while (v);
    buf_put(b, t, (uint64_t)n);
}
static void put_f32(or_buf *b, float f) {
    uint32_t u;
    memcpy(&u, &f, 4);
    put_le(b, u, 4);
}

typedef struct { const uint8_t *p; uint64_t n, pos; int err; } or_rd;
static uint64_t get_le(or_rd *r, int nbytes) {
    if (r->pos + (uint64_t)nbytes > r->n) { r->err = 1; return 0; }
    uint64_t v = 0;
    for (int i = 0; i < nbytes; i++) v |= (uint64_t)r->p[r->pos + i] << (8 * i);
    r->pos += (uint64_t)nbytes;
    return v;
}
static uint64_t get_varint(or_rd *r) {
    uint64_t v = 0;
    for (int sh = 0; sh < 64; sh += 7) {
        if (r->pos >= r->n) { r->err = 1; return 0; }
        uint8_t c = r->p[r->pos++];
        v |= (uint64_t)(c & 0x7F) << sh;
        if (!(c & 0x80)) return v;
    }
    r->err = 1;
    return 0;
}
static float get_f32(or_rd *r) {
    uint32_t u = (uint32_t)get_le(r, 4);
    float f;
    memcpy(&f, &u, 4);
    return f;
}

#define PATH_ORACLE 0
#define PATH_UNIFORM 255

static int cfg_check(const or_config *c, or_shape *sh) {
    if (c->s < 1 || c->k < 1 || c->k > 4 || c->s > c->k) return OR_ERR_ARG;
    if (c->bs < 1 || c->bs > 65535 || c->t < 1 || c->t > 65535 || c->E < 1 || c->E > 65535) return OR_ERR_ARG;
    if (c->n_blocks < 1) return OR_ERR_ARG;
    if (c->selector & ~(SEL_SPUM | SEL_SPRM | SEL_DM)) return OR_ERR_ARG;
    if (c->selector && !(c->selector & SEL_DM)) return OR_ERR_ARG;
    /* the selector enables one of the two static models, never both */
    if ((c->selector & SEL_SPUM) && (c->selector & SEL_SPRM)) return OR_ERR_ARG;
    /* the Transformer DM runs without a static model */
    if (c->arch == 1 && (c->selector & (SEL_SPUM | SEL_SPRM))) return OR_ERR_ARG;
    /* a BiGRU static model: the public one (1 or 2 layers), or the private
     * one with one layer (Sec. 4.2.2 / 4.2.3) */
    if (c->static_arch < 0 || c->static_arch > 1) return OR_ERR_ARG;
    if (c->static_arch == 1 && (c->selector & SEL_SPRM) && c->gru_layers != 1) return OR_ERR_ARG;
    if (c->smp_ppm > 1000000u) return OR_ERR_ARG;
    return shape_init(sh, c->k, c->t, c->E, c->nh, c->hidden, c->arch, c->arch == 1 ? c->heads : 0);
}

/* Split the N runs out of a block and map ACGT to 0..3. */
static int block_strip(const uint8_t *raw, or_block *b) {
    uint64_t runs = 0, nn = 0;
    for (uint64_t i = 0; i < b->raw_len; i++) {
        int c = base_code(raw[i]);
        if (c == 255) return OR_ERR_BASE;
        if (c == 4) {
            nn++;
            if (i == 0 || raw[i - 1] != 'N') runs++;
        }
    }
    b->n_runs = runs;
    b->nb = b->raw_len - nn;
    b->run_start = (uint64_t *)malloc(sizeof(uint64_t) * (runs + 1));
    b->run_len = (uint64_t *)malloc(sizeof(uint64_t) * (runs + 1));
    b->codes = (uint8_t *)malloc(b->nb + 1);
    if (!b->run_start || !b->run_len || !b->codes) return OR_ERR_NOMEM;
    uint64_t r = 0, q = 0;
    for (uint64_t i = 0; i < b->raw_len; i++) {
        int c = base_code(raw[i]);
        if (c == 4) {
            if (i == 0 || raw[i - 1] != 'N') { b->run_start[r] = i; b->run_len[r] = 0; r++; }
            b->run_len[r - 1]++;
        } else {
            b->codes[q++] = (uint8_t)c;
        }
    }
    return OR_OK;
}

static void block_geometry(const or_config *c, or_block *b) {
    b->l = or_skmer_count(b->nb, c->s, c->k);
    b->L = b->l / (uint64_t)c->bs;
    b->rem = b->l - b->L * (uint64_t)c->bs;
    uint64_t covered = b->l ? (b->l - 1) * (uint64_t)c->s + (uint64_t)c->k : 0;
    b->tail = b->nb - covered;
}

static void block_free(or_block *b, int bs) {
    free(b->run_start); free(b->run_len); free(b->codes); free(b->tok); free(b->extras); free(b->snap);
    if (b->seg_buf) for (int j = 0; j < bs; j++) free(b->seg_buf[j]);
    free(b->seg_buf); free(b->seg_bytes);
}

/* Extras: tail bases (2 bits each) then remainder tokens (2k bits each),
 * most significant bit first. */
static void pack_bits(uint8_t *dst, uint64_t *bitpos, uint32_t val, int nbits) {
    for (int i = nbits - 1; i >= 0; i--) {
        if ((val >> i) & 1u) dst[*bitpos >> 3] |= (uint8_t)(0x80u >> (*bitpos & 7));
        (*bitpos)++;
    }
}
static uint32_t unpack_bits(const uint8_t *src, uint64_t *bitpos, int nbits) {
    uint32_t v = 0;
    for (int i = 0; i < nbits; i++) {
        v = (v << 1) | (uint32_t)((src[*bitpos >> 3] >> (7 - (*bitpos & 7))) & 1u);
        (*bitpos)++;
    }
    return v;
}

static int plan_blocks(const or_config *cfg, uint64_t n, or_block **out) {
    int nb = cfg->n_blocks;
    or_block *B = (or_block *)calloc((uint64_t)nb, sizeof(or_block));
    if (!B) return OR_ERR_NOMEM;
    uint64_t off = 0;
    for (int b = 0; b < nb; b++) {
        uint64_t len;
        if (cfg->block_len) len = cfg->block_len[b];
        else len = (b == nb - 1) ? n - (n / (uint64_t)nb) * (uint64_t)(nb - 1) : n / (uint64_t)nb;
        B[b].raw_off = off;
        B[b].raw_len = len;
        off += len;
    }
    if (off != n) { free(B); return OR_ERR_ARG; }
    /* file membership: a block has an SMP predecessor when the previous
     * block belongs to the same file */
    int fb = 0, f = 0, left = cfg->file_blocks ? (int)cfg->file_blocks[0] : nb;
    int nf = cfg->file_blocks ? cfg->n_files : 1;
    uint64_t tot = 0;
    for (int q = 0; q < nf; q++) tot += cfg->file_blocks ? cfg->file_blocks[q] : (uint64_t)nb;
    if (tot != (uint64_t)nb) { free(B); return OR_ERR_ARG; }
    for (int b = 0; b < nb; b++) {
        while (left == 0 && f + 1 < nf) { f++; left = (int)cfg->file_blocks[f]; fb = 0; }
        B[b].has_pred = fb > 0;
        fb++;
        left--;
    }
    *out = B;
    return OR_OK;
}

static void write_header(or_buf *o, const or_config *cfg, int path, uint32_t static_crc, uint64_t n) {
    const uint8_t magic[4] = {'P', 'M', 'K', 'C'};
    buf_put(o, magic, 4);
    put_le(o, 1, 1);
    put_le(o, (uint64_t)path, 1);
    put_le(o, (uint64_t)cfg->s, 1);
    put_le(o, (uint64_t)cfg->k, 1);
    put_le(o, (uint64_t)cfg->t, 2);
    put_le(o, (uint64_t)cfg->bs, 2);
    put_le(o, (uint64_t)cfg->E, 2);
    put_le(o, (uint64_t)cfg->nh, 1);
    put_le(o, (uint64_t)cfg->optimizer, 1);
    for (int l = 0; l < 4; l++) put_le(o, l < cfg->nh ? (uint64_t)cfg->hidden[l] : 0, 2);
    put_f32(o, cfg->lr);
    put_f32(o, cfg->beta1);
    put_f32(o, cfg->beta2);
    put_f32(o, cfg->eps);
    put_le(o, (uint64_t)cfg->selector, 1);
    put_le(o, (uint64_t)cfg->arch, 1);
    put_le(o, cfg->arch == 1 ? (uint64_t)cfg->heads : 0, 1);
    put_le(o, cfg->static_arch == 1 ? (uint64_t)(1 | (cfg->gru_layers << 4)) : 0, 1);
    put_le(o, cfg->smp_ppm, 4);
    put_le(o, cfg->seed, 8);
    put_le(o, static_crc, 4);
    if (cfg->static_arch == 1) {
        put_le(o, (uint64_t)cfg->static_E, 1);
        put_le(o, (uint64_t)cfg->gru_h, 1);
        put_le(o, (uint64_t)cfg->dense, 2);
    } else {
        put_le(o, 0, 4);
    }
    put_le(o, n, 8);
    put_le(o, (uint64_t)cfg->n_blocks, 4);
    put_le(o, (uint64_t)(cfg->file_blocks ? cfg->n_files : 1), 4);
}

/* Process all blocks: DM-only or static+DM, SMP chains within files.
 * Blocks without SMP run in parallel (OpenMP); with SMP each file's chain
 * runs in order (block b+1 starts from block b's snapshot). */
static int process_blocks(const or_config *cfg, const or_shape *sh, const double *ws, or_block *B, int mode,
                          const uint8_t *const *stream_ptr) {
    int nb = cfg->n_blocks;
    uint64_t n = sh->n;
    double *init = (double *)malloc(sizeof(double) * (n + 1));
    if (!init) return OR_ERR_NOMEM;
    if (cfg->init_override) {
        memcpy(init, cfg->init_override, sizeof(double) * (n + 1));
    } else {
        init_params(sh, cfg->seed, init);
        init[n] = 0.0; /* a_alpha: alpha = sigmoid(0) = 1/2 */
    }
    int smp = cfg->smp_ppm > 0 && model_on(cfg);
    int rc_all = OR_OK;
    if (!smp) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int b = 0; b < nb; b++) {
            int rc = run_block(cfg, sh, ws, &B[b], init, mode, stream_ptr ? stream_ptr[b] : NULL, NULL);
            if (rc) {
#pragma omp critical
                rc_all = rc;
            }
        }
    } else {
        /* chain heads */
        int nheads = 0;
        for (int b = 0; b < nb; b++) nheads += !B[b].has_pred;
        int *heads = (int *)malloc(sizeof(int) * (uint64_t)(nheads + 1));
        if (!heads) { free(init); return OR_ERR_NOMEM; }
        for (int b = 0, q = 0; b < nb; b++) if (!B[b].has_pred) heads[q++] = b;
#pragma omp parallel for schedule(dynamic, 1)
        for (int h = 0; h < nheads; h++) {
            const double *cur = init;
            for (int b = heads[h]; b < nb && (b == heads[h] || B[b].has_pred); b++) {
                B[b].snap = (double *)malloc(sizeof(double) * (n + 1));
                int rc = B[b].snap ? run_block(cfg, sh, ws, &B[b], cur, mode, stream_ptr ? stream_ptr[b] : NULL, NULL)
                                   : OR_ERR_NOMEM;
                if (rc) {
#pragma omp critical
                    rc_all = rc;
                    break;
                }
                cur = B[b].snap;
            }
        }
        free(heads);
    }
    free(init);
    return rc_all;
}

/* Sec. 4.2.3 with stage (b) of the pipeline (Fig. 2): the static private
 * model is learned from the input itself before compression and stored in
 * the compressed file.  Reading (the paper fixes neither the training data
 * nor its length): the model has the static model's shape (the one-layer
 * BiGRU of Sec. 4.2.2 when configured, else the dynamic model's); it starts from
 * the seeded initialisation under seed ^ SPRM_SEED_XOR and takes the
 * dynamic model's learning steps (Sec. 2 steps (2) and (4), its optimiser
 * and learning rate, no static model mixed in) over one training block of
 * bs segments of Lp tokens, segment j starting at token floor(j * l / bs)
 * of the input's whole token sequence (the blocks' tokens in block order,
 * l in all), Lp = min(floor(l / bs), SPRM_STEPS).  Spreading the segments
 * over the whole input is what makes the model learn its global features.
 * The result, rounded to FP32, is what the container stores and what both
 * sides mix in as L^r. */
static int sprm_train(const or_config *cfg, const or_shape *sh, const or_block *B, float *out) {
    uint64_t n = sh->n, l = 0;
    int nb = cfg->n_blocks, bs = cfg->bs;
    for (int b = 0; b < nb; b++) l += B[b].l;
    uint64_t Lp = l / (uint64_t)bs;
    if (Lp > SPRM_STEPS) Lp = SPRM_STEPS;
    double *w = (double *)malloc(sizeof(double) * (n + 1));
    double *wf = (double *)malloc(sizeof(double) * (n + 1));
    or_block pb;
    memset(&pb, 0, sizeof pb);
    pb.l = Lp * (uint64_t)bs;
    pb.L = Lp;
    pb.tok = (uint8_t *)malloc(pb.l + 1);
    if (!w || !wf || !pb.tok) { free(w); free(wf); free(pb.tok); return OR_ERR_NOMEM; }
    /* segment j: global tokens [floor(j l / bs), + Lp), read across blocks */
    for (int j = 0; j < bs; j++) {
        uint64_t g = (uint64_t)(((unsigned __int128)j * l) / (uint64_t)bs);
        int b = 0;
        uint64_t base = 0;
        while (b < nb && g >= base + B[b].l) { base += B[b].l; b++; }
        for (uint64_t p = 0; p < Lp; p++, g++) {
            while (g >= base + B[b].l) { base += B[b].l; b++; }
            pb.tok[(uint64_t)j * Lp + p] = B[b].tok[g - base];
        }
    }
    init_params(sh, cfg->seed ^ SPRM_SEED_XOR, w);
    w[n] = 0.0;
    memcpy(wf, w, sizeof(double) * (n + 1));
    or_config cd = *cfg;
    cd.selector = SEL_DM;
    cd.smp_ppm = 0;
    or_probe pr = {0, NULL, NULL, 0, wf, NULL};
    int rc = Lp ? run_block(&cd, sh, NULL, &pb, w, 0, NULL, &pr) : OR_OK;
    if (!rc)
        for (uint64_t i = 0; i < n; i++) out[i] = (float)wf[i];
    block_free(&pb, bs);
    free(w);
    free(wf);
    return rc;
}

int or_compress(const or_config *cfg_in, const uint8_t *in, uint64_t n, const float *static_w, uint64_t static_len,
                uint8_t **out, uint64_t *out_len) {
    or_config cfg_sel = *cfg_in;
    const or_config *cfg = &cfg_sel;
    if (cfg_sel.selector == SEL_AUTO) cfg_sel.selector = ms_select(cfg_in, n, static_w != NULL);
    or_shape sh, ssh;
    int rc = cfg_check(cfg, &sh);
    if (!rc) rc = static_shape(cfg, &sh, &ssh);
    if (rc) return rc;
    const uint64_t sn = sh.ssh ? sh.ssh->n : sh.n;   /* static parameters */
    double *ws = NULL;
    float *priv = NULL;     /* the private static model, once trained */
    uint32_t scrc = 0;
    if (static_on(cfg)) {
        ws = (double *)malloc(sizeof(double) * sn);
        if (!ws) return OR_ERR_NOMEM;
    }
    if (static_on(cfg) && !private_on(cfg)) {
        if (!static_w || static_len != sn) { free(ws); return OR_ERR_MODEL; }
        for (uint64_t i = 0; i < sn; i++) ws[i] = (double)static_w[i];
        scrc = or_crc32((const uint8_t *)static_w, sn * 4);
    }
    or_block *B = NULL;
    rc = plan_blocks(cfg, n, &B);
    if (rc) { free(ws); return rc; }
    int nb = cfg->n_blocks;
    for (int b = 0; b < nb && !rc; b++) {
        rc = block_strip(in + B[b].raw_off, &B[b]);
        if (rc) break;
        block_geometry(cfg, &B[b]);
        B[b].tok = (uint8_t *)malloc(B[b].l + 1);
        if (!B[b].tok) { rc = OR_ERR_NOMEM; break; }
        /* tokenise the stripped bases of this block (Sec. 4.1) */
        for (uint64_t j = 0; j < B[b].l; j++) {
            uint32_t e = 0;
            for (int m = 0; m < cfg->k; m++) e = e * 4u + B[b].codes[j * (uint64_t)cfg->s + (uint64_t)m];
            B[b].tok[j] = (uint8_t)e;
        }
    }
    if (!rc && private_on(cfg)) {
        /* the private model has the static model's shape: the BiGRU one when
         * configured, else the dynamic model's */
        priv = (float *)malloc(sizeof(float) * (sn + 1));
        rc = priv ? sprm_train(cfg, sh.ssh ? sh.ssh : &sh, B, priv) : OR_ERR_NOMEM;
        if (!rc) {
            for (uint64_t i = 0; i < sn; i++) ws[i] = (double)priv[i];
            scrc = or_crc32((const uint8_t *)priv, sn * 4);
        }
    }
    if (!rc) rc = process_blocks(cfg, &sh, ws, B, 0, NULL);
    if (!rc) {
        or_buf o = {0};
        int path = cfg->selector ? PATH_ORACLE : PATH_UNIFORM;
        write_header(&o, cfg, path, scrc, n);
        if (cfg->file_blocks) for (int f = 0; f < cfg->n_files; f++) put_varint(&o, cfg->file_blocks[f]);
        else put_varint(&o, (uint64_t)nb);
        /* the private static model travels in the file (Sec. 4.2.3) */
        if (priv) for (uint64_t i = 0; i < sn; i++) put_f32(&o, priv[i]);
        for (int b = 0; b < nb; b++) {
            or_block *k = &B[b];
            put_varint(&o, k->raw_len);
            put_varint(&o, k->n_runs);
            uint64_t prev_end = 0;
            for (uint64_t r = 0; r < k->n_runs; r++) {
                put_varint(&o, k->run_start[r] - prev_end);
                put_varint(&o, k->run_len[r]);
                prev_end = k->run_start[r] + k->run_len[r];
            }
            uint64_t bits = 2 * k->tail + 2 * (uint64_t)cfg->k * k->rem;
            uint8_t *ex = (uint8_t *)calloc((bits + 7) / 8 + 1, 1);
            if (!ex) { o.err = 1; break; }
            uint64_t bp = 0;
            for (uint64_t q = k->nb - k->tail; q < k->nb; q++) pack_bits(ex, &bp, k->codes[q], 2);
            for (uint64_t q = k->L * (uint64_t)cfg->bs; q < k->l; q++) pack_bits(ex, &bp, k->tok[q], 2 * cfg->k);
            buf_put(&o, ex, (bits + 7) / 8);
            free(ex);
            if (k->L > 0)
                for (int j = 0; j < cfg->bs; j++) put_varint(&o, k->seg_bytes[j]);
        }
        for (int b = 0; b < nb; b++)
            if (B[b].L > 0)
                for (int j = 0; j < cfg->bs; j++) buf_put(&o, B[b].seg_buf[j], B[b].seg_bytes[j]);
        if (o.err) { free(o.p); rc = OR_ERR_NOMEM; }
        else { *out = o.p; *out_len = o.n; }
    }
    for (int b = 0; b < nb; b++) block_free(&B[b], cfg->bs);
    free(B);
    free(ws);
    free(priv);
    return rc;
}

int or_decompress(const uint8_t *cbf, uint64_t len, const float *static_w, uint64_t static_len, uint8_t **out,
                  uint64_t *out_len) {
    or_rd r = {cbf, len, 0, 0};
    if (len < 80 || memcmp(cbf, "PMKC", 4) != 0) return OR_ERR_CORRUPT;
    r.pos = 4;
    if (get_le(&r, 1) != 1) return OR_ERR_CORRUPT;
    int path = (int)get_le(&r, 1);
    or_config c;
    memset(&c, 0, sizeof c);
    c.s = (int32_t)get_le(&r, 1);
    c.k = (int32_t)get_le(&r, 1);
    c.t = (int32_t)get_le(&r, 2);
    c.bs = (int32_t)get_le(&r, 2);
    c.E = (int32_t)get_le(&r, 2);
    c.nh = (int32_t)get_le(&r, 1);
    c.optimizer = (int32_t)get_le(&r, 1);
    for (int l = 0; l < 4; l++) c.hidden[l] = (int32_t)get_le(&r, 2);
    c.lr = get_f32(&r);
    c.beta1 = get_f32(&r);
    c.beta2 = get_f32(&r);
    c.eps = get_f32(&r);
    c.selector = (int32_t)get_le(&r, 1);
    c.arch = (int32_t)get_le(&r, 1);
    c.heads = (int32_t)get_le(&r, 1);
    {
        int sb = (int)get_le(&r, 1);
        c.static_arch = sb & 15;
        c.gru_layers = sb >> 4;
    }
    c.smp_ppm = (uint32_t)get_le(&r, 4);
    c.seed = get_le(&r, 8);
    uint32_t scrc = (uint32_t)get_le(&r, 4);
    c.static_E = (int32_t)get_le(&r, 1);
    c.gru_h = (int32_t)get_le(&r, 1);
    c.dense = (int32_t)get_le(&r, 2);
    uint64_t n = get_le(&r, 8);
    c.n_blocks = (int32_t)get_le(&r, 4);
    c.n_files = (int32_t)get_le(&r, 4);
    if (r.err) return OR_ERR_CORRUPT;
    if (c.nh > 4) return OR_ERR_CORRUPT;
    if (!(path == PATH_ORACLE && c.selector) && !(path == PATH_UNIFORM && !c.selector)) return OR_ERR_MODEL;
    or_shape sh, ssh;
    if (cfg_check(&c, &sh) || static_shape(&c, &sh, &ssh)) return OR_ERR_CORRUPT;
    const uint64_t sn = sh.ssh ? sh.ssh->n : sh.n;
    if (c.n_files < 1 || (uint64_t)c.n_files > len || (uint64_t)c.n_blocks * 2 > len) return OR_ERR_CORRUPT;
    uint64_t *fblocks = (uint64_t *)malloc(sizeof(uint64_t) * (uint64_t)c.n_files);
    uint64_t *blen = (uint64_t *)malloc(sizeof(uint64_t) * (uint64_t)c.n_blocks);
    if (!fblocks || !blen) { free(fblocks); free(blen); return OR_ERR_NOMEM; }
    for (int f = 0; f < c.n_files; f++) fblocks[f] = get_varint(&r);
    c.file_blocks = fblocks;
    if (r.err) { free(fblocks); free(blen); return OR_ERR_CORRUPT; }
    double *ws = NULL;
    int rc = OR_OK;
    if (private_on(&c)) {
        /* the stored private model: its FP32 values after the file table */
        if (sn > (len - r.pos) / 4 || or_crc32(cbf + r.pos, sn * 4) != scrc) {
            free(fblocks); free(blen);
            return OR_ERR_CORRUPT;
        }
        ws = (double *)malloc(sizeof(double) * sn);
        if (!ws) { free(fblocks); free(blen); return OR_ERR_NOMEM; }
        for (uint64_t i = 0; i < sn; i++) ws[i] = (double)get_f32(&r);
    } else if (static_on(&c)) {
        if (!static_w || static_len != sn || or_crc32((const uint8_t *)static_w, sn * 4) != scrc) {
            free(fblocks); free(blen);
            return OR_ERR_MODEL;
        }
        ws = (double *)malloc(sizeof(double) * sn);
        if (!ws) { free(fblocks); free(blen); return OR_ERR_NOMEM; }
        for (uint64_t i = 0; i < sn; i++) ws[i] = (double)static_w[i];
    }
    /* first pass over the block table to learn raw lengths */
    or_block *B = (or_block *)calloc((uint64_t)c.n_blocks, sizeof(or_block));
    const uint8_t **sp = (const uint8_t **)calloc((uint64_t)c.n_blocks, sizeof(uint8_t *));
    uint8_t *dst = NULL;
    if (!B || !sp) { rc = OR_ERR_NOMEM; goto fail; }
    uint64_t off = 0;
    for (int b = 0; b < c.n_blocks; b++) {
        or_block *k = &B[b];
        k->raw_off = off;
        k->raw_len = get_varint(&r);
        if (r.err || k->raw_len > n - off) { rc = OR_ERR_CORRUPT; goto fail; }
        off += k->raw_len;
        blen[b] = k->raw_len;
        k->n_runs = get_varint(&r);
        if (r.err || k->n_runs > k->raw_len) { rc = OR_ERR_CORRUPT; goto fail; }
        k->run_start = (uint64_t *)malloc(sizeof(uint64_t) * (k->n_runs + 1));
        k->run_len = (uint64_t *)malloc(sizeof(uint64_t) * (k->n_runs + 1));
        if (!k->run_start || !k->run_len) { rc = OR_ERR_NOMEM; goto fail; }
        uint64_t prev_end = 0, nn = 0;
        for (uint64_t q = 0; q < k->n_runs; q++) {
            uint64_t gap = get_varint(&r), rl = get_varint(&r);
            k->run_start[q] = prev_end + gap;
            k->run_len[q] = rl;
            prev_end = k->run_start[q] + rl;
            nn += rl;
            if (r.err || prev_end > k->raw_len || rl == 0) { rc = OR_ERR_CORRUPT; goto fail; }
        }
        k->nb = k->raw_len - nn;
        block_geometry(&c, k);
        uint64_t bits = 2 * k->tail + 2 * (uint64_t)c.k * k->rem;
        uint64_t eb = (bits + 7) / 8;
        if (r.pos + eb > len) { rc = OR_ERR_CORRUPT; goto fail; }
        k->extras = (uint8_t *)malloc(eb + 1);
        k->codes = (uint8_t *)malloc(k->nb + 1);
        k->tok = (uint8_t *)malloc(k->l + 1);
        if (!k->extras || !k->codes || !k->tok) { rc = OR_ERR_NOMEM; goto fail; }
        memcpy(k->extras, cbf + r.pos, eb);
        k->extras_bytes = eb;
        r.pos += eb;
        if (k->L > 0) {
            k->seg_bytes = (uint64_t *)calloc((uint64_t)c.bs, sizeof(uint64_t));
            if (!k->seg_bytes) { rc = OR_ERR_NOMEM; goto fail; }
            for (int j = 0; j < c.bs; j++) k->seg_bytes[j] = get_varint(&r);
            if (r.err) { rc = OR_ERR_CORRUPT; goto fail; }
        }
    }
    if (off != n) { rc = OR_ERR_CORRUPT; goto fail; }
    {
        uint64_t p = r.pos;
        for (int b = 0; b < c.n_blocks; b++) {
            sp[b] = cbf + p;
            if (B[b].L > 0)
                for (int j = 0; j < c.bs; j++) {
                    if (B[b].seg_bytes[j] > len - p) { rc = OR_ERR_CORRUPT; goto fail; }
                    p += B[b].seg_bytes[j];
                }
        }
        if (p != len) { rc = OR_ERR_CORRUPT; goto fail; }
    }
    {
        int fb_tot = 0;
        for (int f = 0; f < c.n_files; f++) fb_tot += (int)fblocks[f];
        if (fb_tot != c.n_blocks) { rc = OR_ERR_CORRUPT; goto fail; }
        /* recompute SMP predecessor flags */
        int f = 0, left = (int)fblocks[0], fbi = 0;
        for (int b = 0; b < c.n_blocks; b++) {
            while (left == 0 && f + 1 < c.n_files) { f++; left = (int)fblocks[f]; fbi = 0; }
            B[b].has_pred = fbi > 0;
            fbi++;
            left--;
        }
    }
    rc = process_blocks(&c, &sh, ws, B, 1, sp);
    if (rc) goto fail;
    dst = (uint8_t *)malloc(n + 1);
    if (!dst) { rc = OR_ERR_NOMEM; goto fail; }
    for (int b = 0; b < c.n_blocks; b++) {
        or_block *k = &B[b];
        /* remainder tokens and tail bases from the extras */
        uint64_t bp = 0;
        uint8_t tailc[8];
        for (uint64_t q = 0; q < k->tail; q++) tailc[q] = (uint8_t)unpack_bits(k->extras, &bp, 2);
        for (uint64_t q = k->L * (uint64_t)c.bs; q < k->l; q++) k->tok[q] = (uint8_t)unpack_bits(k->extras, &bp, 2 * c.k);
        /* tokens -> bases: the first token gives k bases, each later one its last s */
        uint64_t qb = 0;
        for (uint64_t j = 0; j < k->l; j++) {
            int from = j == 0 ? 0 : c.k - c.s;
            for (int m = from; m < c.k; m++) k->codes[qb++] = (uint8_t)((k->tok[j] >> (2 * (c.k - 1 - m))) & 3u);
        }
        for (uint64_t q = 0; q < k->tail; q++) k->codes[qb++] = tailc[q];
        /* re-insert N runs */
        uint8_t *o = dst + k->raw_off;
        uint64_t ri = 0, ci = 0;
        for (uint64_t i = 0; i < k->raw_len; i++) {
            if (ri < k->n_runs && i >= k->run_start[ri] && i < k->run_start[ri] + k->run_len[ri]) {
                o[i] = 'N';
                if (i + 1 == k->run_start[ri] + k->run_len[ri]) ri++;
            } else {
                o[i] = LETTER[k->codes[ci++]];
            }
        }
    }
    *out = dst;
    *out_len = n;
    dst = NULL;
fail:
    free(dst);
    if (B) for (int b = 0; b < c.n_blocks; b++) block_free(&B[b], c.bs);
    free(B);
    free(sp);
    free(ws);
    free(fblocks);
    free(blen);
    return rc;
}

/* Trace of one block's compression: P for the requested steps (sorted),
 * per-step loss, and the parameters (+ a_alpha) after `stop` steps (0 = all
 * L steps).  The segment length L is that of the whole block.  The block is
 * tokenised from ACGT-only input; init = seeded parameters, or `init`
 * when not NULL (n params + a_alpha). */
int or_trace_block(const or_config *cfg, const uint8_t *tokens, uint64_t l, const float *static_w,
                   const double *init, uint64_t stop, const uint64_t *steps, uint64_t n_steps, double *P_out,
                   double *loss_out, double *w_final) {
    or_shape sh, ssh;
    int rc = cfg_check(cfg, &sh);
    if (!rc) rc = static_shape(cfg, &sh, &ssh);
    if (rc) return rc;
    const uint64_t sn = sh.ssh ? sh.ssh->n : sh.n;
    double *ws = NULL;
    if (static_on(cfg)) {
        ws = (double *)malloc(sizeof(double) * sn);
        if (!ws) return OR_ERR_NOMEM;
        for (uint64_t i = 0; i < sn; i++) ws[i] = (double)static_w[i];
    }
    or_block blk;
    memset(&blk, 0, sizeof blk);
    blk.l = l;
    blk.L = l / (uint64_t)cfg->bs;
    blk.tok = (uint8_t *)malloc(l + 1);
    double *w0 = (double *)malloc(sizeof(double) * (sh.n + 1));
    if (!blk.tok || !w0) { free(blk.tok); free(w0); free(ws); return OR_ERR_NOMEM; }
    memcpy(blk.tok, tokens, l);
    if (init) memcpy(w0, init, sizeof(double) * (sh.n + 1));
    else { init_params(&sh, cfg->seed, w0); w0[sh.n] = 0.0; }
    or_probe pr = {stop, P_out, steps, n_steps, w_final, loss_out};
    rc = run_block(cfg, &sh, ws, &blk, w0, 0, NULL, &pr);
    block_free(&blk, cfg->bs);
    free(w0);
    free(ws);
    return rc;
}

void or_free(void *p) { free(p); }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* The static public model alone, for its pins: parameter count, seeded
 * initialisation and the logits L^u of `rows` contexts (cfg's static_arch
 * and BiGRU fields; static_arch 0 is the DM's own MLP shape). */
static int static_only_shape(const or_config *c, or_shape *s) {
    if (c->static_arch == 1) return shape_init_gru(s, c->k, c->t, c->static_E, c->gru_h, c->gru_layers, c->dense);
    return shape_init(s, c->k, c->t, c->E, c->nh, c->hidden, 0, 0);
}

uint64_t or_static_param_count(const void *cfg) {
    or_shape s;
    return static_only_shape((const or_config *)cfg, &s) ? 0 : s.n;
}
int or_static_init(const void *cfg, uint64_t seed, double *w) {
    or_shape s;
    int rc = static_only_shape((const or_config *)cfg, &s);
    if (rc) return rc;
    init_params(&s, seed, w);
    return OR_OK;
}
/* One learning step of the static model as a standalone model (the private
 * model's training step): P, the gradient of the mean cross-entropy of the
 * rows' targets, the loss (Sec. 2 steps (3)-(4)). */
int or_static_step(const void *cfg, const double *ws, const uint8_t *ctx, const uint8_t *tgt, int rows, double *P,
                   double *grad, double *loss) {
    or_shape s;
    int rc = static_only_shape((const or_config *)cfg, &s);
    if (rc) return rc;
    if (s.arch == 2 && grad && s.gl != 1) return OR_ERR_ARG;   /* training: one BiGRU layer */
    return step_grad(&s, ws, NULL, 0.0, ctx, tgt, rows, P, grad, NULL, loss);
}
int or_static_forward(const void *cfg, const double *ws, const uint8_t *ctx, int rows, double *logits) {
    or_shape s;
    int rc = static_only_shape((const or_config *)cfg, &s);
    if (rc) return rc;
    double *act = (double *)malloc(sizeof(double) * (acts_len(&s) + 1));
    if (!act) return OR_ERR_NOMEM;
    for (int j = 0; j < rows; j++)
        forward_row(&s, ws, ctx + (uint64_t)j * s.t, act, logits + (uint64_t)j * s.V);
    free(act);
    return OR_OK;
}
