/*
 * Seeded synthetic DNA source used as the stand-in for the paper's genome
 * datasets (which are real genomes and are not available here).
 *
 * This file holds no part of the compression method: it only draws ASCII
 * bases.  Both the oracle tests and the GPU tests/bench take their inputs
 * from here.  Recipe (all draws from one SplitMix64 stream per call):
 *   1. order-m Markov chain; the caller passes the 4^m x 4 transition rows
 *      (drawn from Dirichlet(0.5) in Python); the first m bases are uniform;
 *      optional GC tilt per segment: p'(b|c) ~ p(b|c) * w_b with
 *      w_C = w_G = gc/0.5, w_A = w_T = (1-gc)/0.5;
 *   2. planted repeats: until a fraction rho of the sequence is covered,
 *      copy a length U{lmin..lmax} piece from an earlier position to a
 *      destination that overlaps no earlier destination; with probability
 *      p_rc the copy is reverse-complemented;
 *   3. N runs: each position starts a run with probability rate/mean_len,
 *      length U{1..nmax}.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t sm_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static double sm_unit(uint64_t *s) { return (double)(sm_next(s) >> 11) * (1.0 / 9007199254740992.0); }
static uint64_t sm_below(uint64_t *s, uint64_t n) { return n ? sm_next(s) % n : 0; }

static const uint8_t ACGT[4] = {'A', 'C', 'G', 'T'};

/* rows: 4^order x 4 probabilities (row-major). gc: n_seg values or NULL.
 * Per GC segment the tilted rows are turned into three cumulative
 * thresholds once; each base then costs one draw and three compares. */
void synth_markov(uint8_t *out, uint64_t n, int order, const double *rows,
                  const double *gc, uint64_t seg_len, uint64_t seed) {
    uint64_t st = seed ^ 0x5DEECE66Dull;
    uint64_t nrows = 1ull << (2 * order);
    uint64_t mask = (order > 0) ? (nrows - 1) : 0;
    double *thr = (double *)malloc(sizeof(double) * 3 * nrows);
    if (!thr) return;
    uint64_t ctx = 0, cur_seg = ~0ull;
    for (uint64_t i = 0; i < n; i++) {
        int b;
        double u = sm_unit(&st);
        uint64_t seg = (gc && seg_len) ? i / seg_len : 0;
        if (seg != cur_seg) {
            cur_seg = seg;
            double wat = 1.0, wcg = 1.0;
            if (gc) { wat = (1.0 - gc[seg]) / 0.5; wcg = gc[seg] / 0.5; }
            for (uint64_t r = 0; r < nrows; r++) {
                const double *q = rows + 4 * r;
                double p0 = q[0] * wat, p1 = q[1] * wcg, p2 = q[2] * wcg, p3 = q[3] * wat;
                double tot = p0 + p1 + p2 + p3;
                thr[3 * r] = p0 / tot;
                thr[3 * r + 1] = (p0 + p1) / tot;
                thr[3 * r + 2] = (p0 + p1 + p2) / tot;
            }
        }
        if (i < (uint64_t)order) {
            b = (int)(u * 4.0);
            if (b > 3) b = 3;
        } else {
            const double *t3 = thr + 3 * ctx;
            b = (u < t3[0]) ? 0 : (u < t3[1]) ? 1 : (u < t3[2]) ? 2 : 3;
        }
        out[i] = ACGT[b];
        ctx = ((ctx << 2) | (uint64_t)b) & mask;
    }
    free(thr);
}

static uint8_t comp(uint8_t c) {
    switch (c) { case 'A': return 'T'; case 'C': return 'G'; case 'G': return 'C'; case 'T': return 'A'; }
    return c;
}

/* Returns the number of bases covered by planted repeats. */
uint64_t synth_repeats(uint8_t *seq, uint64_t n, double rho, uint64_t lmin, uint64_t lmax,
                       double p_rc, uint64_t seed) {
    if (rho <= 0.0 || n < 4 * lmax) return 0;
    uint64_t st = seed ^ 0xA5A5A5A5DEADBEEFull;
    uint64_t target = (uint64_t)(rho * (double)n);
    uint64_t words = (n + 63) / 64;
    uint64_t *cov = (uint64_t *)calloc(words, 8);
    if (!cov) return 0;
    uint64_t covered = 0, tries = 0, max_tries = 64 * (target / lmin + 16);
    while (covered < target && tries < max_tries) {
        tries++;
        uint64_t len = lmin + sm_below(&st, lmax - lmin + 1);
        uint64_t d = len + sm_below(&st, n - 2 * len);  /* dest in [len, n-len) */
        int clash = 0;
        for (uint64_t q = d; q < d + len; q++)
            if (cov[q >> 6] >> (q & 63) & 1) { clash = 1; break; }
        if (clash) continue;
        uint64_t src = sm_below(&st, d - len + 1);       /* src in [0, d-len] */
        int rc = sm_unit(&st) < p_rc;
        for (uint64_t q = 0; q < len; q++) {
            uint8_t c = rc ? comp(seq[src + len - 1 - q]) : seq[src + q];
            seq[d + q] = c;
            cov[(d + q) >> 6] |= 1ull << ((d + q) & 63);
        }
        covered += len;
    }
    free(cov);
    return covered;
}

/* Returns the number of N bases written. */
uint64_t synth_nruns(uint8_t *seq, uint64_t n, double rate, uint64_t nmax, uint64_t seed) {
    if (rate <= 0.0) return 0;
    uint64_t st = seed ^ 0x0123456789ABCDEFull;
    double mean = 0.5 * (double)(nmax + 1);
    double p = rate / mean;
    uint64_t total = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (sm_unit(&st) < p) {
            uint64_t len = 1 + sm_below(&st, nmax);
            for (uint64_t q = 0; q < len && i + q < n; q++, total++) seq[i + q] = 'N';
            i += len;
        }
    }
    return total;
}
