/* Plain C oracle of the FS2D HLF stage-2 enumeration, sampling and membership
 * -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this file's shared object.  It shares nothing with the HIP library.
 *
 * Every function is the direct per-index definition, with OpenMP over the
 * index range and no other restructuring:
 *
 *   z_i = l XOR ( XOR over k < r with bit k of g(i) set of B_k ),
 *   g(i) = i XOR (i >> 1),
 *
 * which is the paper's second stage (Section 2, Eq. (3) restricted to the
 * pivot inputs, followed by the final CNOT layer with z^a = l), traversed in
 * Gray order.  Vectors are W little-endian 64-bit words; bit j of the vector
 * is z_{j+1}.
 *
 * Hash of one solution (a project convention): h_0 = 0,
 * h_{w+1} = mix13(h_w ^ z_w ^ GAMMA), h(z) = h_W; the hash of a set is the sum
 * of h(z) mod 2^64.  mix13 is the output function of Vigna's public-domain
 * SplitMix64 (Stafford's Mix13); GAMMA is SplitMix64's increment.
 *
 * Samples use the same combination with a coefficient vector drawn from the
 * project's counter-based SplitMix64 stream (or passed in); membership checks
 * the problem's definition on the Ker(A) basis.
 *
 * Parity pins: tests compare these functions with the Python oracle on small
 * ranges and with closed forms (per-qubit counts, full-rank identity hash,
 * samples satisfying every kernel equation, membership against brute force).
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 0x9E3779B97F4A7C15ULL

static uint64_t mix13(uint64_t x) {
    x ^= x >> 30;
    x *= 0xBF58476D1CE4E5B9ULL;
    x ^= x >> 27;
    x *= 0x94D049BB133111EBULL;
    x ^= x >> 31;
    return x;
}

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

uint64_t oracle_mix13(uint64_t x) { return mix13(x); }

/* l XOR (XOR over k < r with bit k of the coefficient vector c set of B_k)
 * into z[0..W-1]; c is given as ceil(r/64) words.  Each term is B_k ANDed with
 * an all-ones or all-zeros mask made from its coefficient bit (the same sum
 * as "if bit k is set, add B_k", without a data-dependent branch). */
static void combine(const uint64_t *basis, int r, int W, const uint64_t *shift,
                    const uint64_t *c, uint64_t *z) {
    if (W == 1) {  /* the same sum, written for one-word vectors */
        uint64_t acc = shift[0];
        for (int k = 0; k < r; ++k) acc ^= basis[k] & (0ULL - ((c[k >> 6] >> (k & 63)) & 1ULL));
        z[0] = acc;
        return;
    }
    for (int w = 0; w < W; ++w) z[w] = shift[w];
    for (int k = 0; k < r; ++k) {
        const uint64_t m = 0ULL - ((c[k >> 6] >> (k & 63)) & 1ULL);
        for (int w = 0; w < W; ++w) z[w] ^= basis[(size_t)k * W + w] & m;
    }
}

/* z_i into z[0..W-1] by the direct definition (coefficients g(i), r <= 62). */
static void solution_at(const uint64_t *basis, int r, int W, const uint64_t *shift,
                        uint64_t i, uint64_t *z) {
    const uint64_t g = i ^ (i >> 1);
    combine(basis, r, W, shift, &g, z);
}

static uint64_t hash_words(const uint64_t *z, int W) {
    uint64_t h = 0;
    for (int w = 0; w < W; ++w) h = mix13(h ^ z[w] ^ GAMMA);
    return h;
}

/* out[(i - begin) * W + w] = word w of z_i, i in [begin, begin + count). */
int oracle_enumerate(const uint64_t *basis, int r, int W, const uint64_t *shift,
                     uint64_t begin, uint64_t count, uint64_t *out) {
    if (r < 0 || r > 62 || W < 1 || W > 16) return -1;
    if (begin > (1ULL << r) || count > (1ULL << r) - begin) return -3;
    int64_t cnt = (int64_t)count;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < cnt; ++t) {
        solution_at(basis, r, W, shift, begin + (uint64_t)t, out + (size_t)t * W);
    }
    return 0;
}

/* Counter order (the FPGA's binary counter, Section 4): solution number i is
 * l XOR (XOR over k < r with bit k of i set of B_k), by the direct
 * definition; out as oracle_enumerate. */
int oracle_enumerate_counter(const uint64_t *basis, int r, int W, const uint64_t *shift,
                             uint64_t begin, uint64_t count, uint64_t *out) {
    if (r < 0 || r > 62 || W < 1 || W > 16) return -1;
    if (begin > (1ULL << r) || count > (1ULL << r) - begin) return -3;
    int64_t cnt = (int64_t)count;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < cnt; ++t) {
        const uint64_t i = begin + (uint64_t)t;
        uint64_t *z = out + (size_t)t * W;
        for (int w = 0; w < W; ++w) z[w] = shift[w];
        for (int k = 0; k < r; ++k)
            if ((i >> k) & 1ULL)
                for (int w = 0; w < W; ++w) z[w] ^= basis[(size_t)k * W + w];
    }
    return 0;
}

/* counts[j] = #solutions with bit j set (j < n; counts may be NULL when only
 * the hash is wanted); *hash = sum of h(z); xorfold[w] = XOR of all solutions
 * (may be NULL). */
int oracle_reduce(const uint64_t *basis, int r, int W, int n, const uint64_t *shift,
                  uint64_t begin, uint64_t count, uint64_t *counts, uint64_t *hash,
                  uint64_t *xorfold) {
    if (r < 0 || r > 62 || W < 1 || W > 16 || n < 1 || n > 64 * W) return -1;
    if (begin > (1ULL << r) || count > (1ULL << r) - begin) return -3;
    int64_t cnt = (int64_t)count;
    int nt = oracle_threads();
    uint64_t *part_counts = (uint64_t *)calloc((size_t)nt * n, sizeof(uint64_t));
    uint64_t *part_hash = (uint64_t *)calloc((size_t)nt, sizeof(uint64_t));
    uint64_t *part_xor = (uint64_t *)calloc((size_t)nt * W, sizeof(uint64_t));
    if (!part_counts || !part_hash || !part_xor) {
        free(part_counts); free(part_hash); free(part_xor);
        return -4;
    }
#pragma omp parallel
    {
#ifdef _OPENMP
        int tid = omp_get_thread_num();
#else
        int tid = 0;
#endif
        uint64_t z[16];
        uint64_t *pc = part_counts + (size_t)tid * n;
        uint64_t *px = part_xor + (size_t)tid * W;
        uint64_t ph = 0;
#pragma omp for schedule(static)
        for (int64_t t = 0; t < cnt; ++t) {
            solution_at(basis, r, W, shift, begin + (uint64_t)t, z);
            if (counts)
                for (int j = 0; j < n; ++j) pc[j] += (z[j >> 6] >> (j & 63)) & 1ULL;
            ph += hash_words(z, W);
            for (int w = 0; w < W; ++w) px[w] ^= z[w];
        }
        part_hash[tid] = ph;
    }
    if (counts) for (int j = 0; j < n; ++j) counts[j] = 0;
    *hash = 0;
    if (xorfold) for (int w = 0; w < W; ++w) xorfold[w] = 0;
    for (int t = 0; t < nt; ++t) {
        if (counts) for (int j = 0; j < n; ++j) counts[j] += part_counts[(size_t)t * n + j];
        *hash += part_hash[t];
        if (xorfold) for (int w = 0; w < W; ++w) xorfold[w] ^= part_xor[(size_t)t * W + w];
    }
    free(part_counts); free(part_hash); free(part_xor);
    return 0;
}

/* Samples (uniform single solutions, App. A): for s in [0, num),
 *   c_s = coeffs[s*R64 .. s*R64+R64-1] if coeffs is not NULL, else the
 *         SplitMix64 outputs number s*R64 .. s*R64+R64-1 of the generator whose
 *         state starts at seed (output k = mix13(seed + (k+1)*GAMMA), Steele,
 *         Lea and Flood 2014), R64 = ceil(r/64), bits at positions >= r cleared;
 *   out[s*W .. s*W+W-1] = l XOR (XOR over set bits k of c_s of B_k).
 * Any r in [0, 64W]; OpenMP over the samples. */
int oracle_sample(const uint64_t *basis, int r, int W, const uint64_t *shift, uint64_t seed,
                  uint64_t num, const uint64_t *coeffs, uint64_t *out) {
    if (W < 1 || W > 16 || r < 0 || r > 64 * W) return -1;
    const int R64 = (r + 63) / 64;
    int64_t cnt = (int64_t)num;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < cnt; ++t) {
        const uint64_t s = (uint64_t)t;
        uint64_t c[16] = {0};
        for (int w = 0; w < R64; ++w) {
            const uint64_t k = s * (uint64_t)R64 + (uint64_t)w;
            c[w] = coeffs ? coeffs[k] : mix13(seed + (k + 1ULL) * GAMMA);
        }
        if (r & 63) c[R64 - 1] &= (1ULL << (r & 63)) - 1ULL;
        combine(basis, r, W, shift, c, out + (size_t)t * W);
    }
    return 0;
}

/* Membership by the problem's definition (Section 1) on a basis of Ker(A):
 * member[s] = 1 iff q_f = 2 <z_s, k_f> (mod 4) for every kernel vector k_f,
 * f < nk, with <z, k> the integer count of common ones and q_f = q(k_f) mod 4
 * (the values of the quadratic form on the basis, passed in).  q is linear on
 * Ker(A), so the basis vectors suffice.  OpenMP over the strings. */
int oracle_membership(const uint64_t *kernel, int nk, const int *q, int W,
                      const uint64_t *z, uint64_t num, uint8_t *member) {
    if (W < 1 || W > 16 || nk < 0) return -1;
    int64_t cnt = (int64_t)num;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < cnt; ++t) {
        const uint64_t *zs = z + (size_t)t * W;
        int ok = 1;
        for (int f = 0; f < nk; ++f) {
            int64_t dot = 0;
            for (int w = 0; w < W; ++w)
                dot += __builtin_popcountll(zs[w] & kernel[(size_t)f * W + w]);
            if ((((int64_t)q[f] - 2 * dot) % 4 + 4) % 4 != 0) ok = 0;
        }
        member[t] = (uint8_t)ok;
    }
    return 0;
}

/* Sum of h(z) over every 64-bit value z in [lo, hi): the hash of the whole
 * solution set {0,1}^n of a full-rank instance (r = n <= 62), independent of
 * the basis and of the enumeration order. */
uint64_t oracle_identity_hash(uint64_t lo, uint64_t hi) {
    int64_t cnt = (int64_t)(hi - lo);
    uint64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t t = 0; t < cnt; ++t) {
        uint64_t z = lo + (uint64_t)t;
        total += mix13(z ^ GAMMA);
    }
    return total;
}
