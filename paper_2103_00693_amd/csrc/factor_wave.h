// Stage 1 (the paper's CLA module, Section 2, tasks (1)-(4)) for one
// instance with n <= 64*WMAX (WMAX in {1,2,3}) on one wavefront.
//
// Lane l holds rows l, l+64, l+128 ("slots") in VGPRs.  Gauss-Jordan over
// GF(2) takes a ballot per slot to find the candidate rows of a column, picks
// the lowest, broadcasts it with readlane and XORs it into every other row
// that has the column set -- no barriers, no LDS in the elimination.  The
// reduced rows then give the Ker(A) basis (task (2)), q on it (task (3)) and
// the canonical shift (task (4)).
//
// Only the calling wave takes part (LDS ordering by wave_lds_sync), so the
// routine can run on one wave of a larger workgroup.
#pragma once

#include "hlf_device.h"
#include "hlf_internal.h"

namespace hlf {

template <int WMAX>
struct WaveSmem {
    uint64_t orig[64 * WMAX * WMAX];  // A, packed rows of W words
    uint64_t rref[64 * WMAX * WMAX];  // RREF row k at k*W
    int piv[64 * WMAX];
    int freec[64 * WMAX];
    unsigned long long shiftw[WMAX];
    int internal;
};

template <int WMAX>
__device__ __forceinline__ void set_bit(uint64_t (&v)[WMAX], int pos) {
#pragma unroll
    for (int w = 0; w < WMAX; ++w)
        if (w == (pos >> 6)) v[w] |= 1ull << (pos & 63);
}

// Packed rows from global memory into sm.orig.
template <int WMAX>
__device__ __forceinline__ void wave_load_rows(const uint64_t *__restrict__ rows, int n, int W,
                                               WaveSmem<WMAX> &sm) {
    for (int idx = lane_id(); idx < n * W; idx += 64) sm.orig[idx] = rows[idx];
}

// Dense row-major uint8 matrix into sm.orig: lane l reads column 64*w + l of
// 16 rows at once (independent loads, one memory latency per group), and the
// ballot over the 64 lanes of each row gives its packed word.  Returns true
// on every lane if an entry is not 0/1.
template <int WMAX>
__device__ __forceinline__ bool wave_load_dense(const uint8_t *__restrict__ A, int n, int W,
                                                WaveSmem<WMAX> &sm) {
    constexpr int G = 16;
    const int lane = lane_id();
    bool bad = false;
    for (int w = 0; w < W; ++w) {
        const int j = 64 * w + lane;
        const bool jin = j < n;
        for (int i0 = 0; i0 < n; i0 += G) {
            uint32_t v[G];
#pragma unroll
            for (int k = 0; k < G; ++k)
                v[k] = (jin && i0 + k < n) ? (uint32_t)A[(size_t)(i0 + k) * n + j] : 0u;
#pragma unroll
            for (int k = 0; k < G; ++k) {
                if (i0 + k >= n) break;
                bad |= v[k] > 1u;
                const uint64_t word = __ballot(v[k] == 1u);
                if (lane == 0) sm.orig[(i0 + k) * W + w] = word;
            }
        }
    }
    return __ballot(bad) != 0;
}

// Factor the matrix in sm.orig.  `bad_input` forces HLF_ENOTSYM.  Returns the
// rank, or -1 if the record was marked invalid.
template <int WMAX>
__device__ int factor_wave_core(int n, int W, bool bad_input, const FactorOut &out,
                                WaveSmem<WMAX> &sm) {
    const int lane = lane_id();
    if (lane < WMAX) sm.shiftw[lane] = 0;
    if (lane == 0) sm.internal = 0;
    wave_lds_sync();

    uint64_t row[WMAX][WMAX];
    bool used[WMAX];
    int rk[WMAX], pc[WMAX];  // rank and pivot column of a pivot row
#pragma unroll
    for (int s = 0; s < WMAX; ++s) {
        const int i = s * 64 + lane;
#pragma unroll
        for (int w = 0; w < WMAX; ++w) row[s][w] = (i < n && w < W) ? sm.orig[i * W + w] : 0ull;
        used[s] = false;
        rk[s] = -1;
        pc[s] = -1;
    }

    // Validation: pad bits zero, A = A^T (slot s of word cw, transposed across
    // the wave, gives lane l word s of column 64cw + l, which must equal word
    // s of row 64cw + l).
    bool bad = bad_input;
    const uint64_t lm = last_word_mask(n);
#pragma unroll
    for (int s = 0; s < WMAX; ++s)
#pragma unroll
        for (int w = 0; w < WMAX; ++w)
            if (w == W - 1 && (row[s][w] & ~lm)) bad = true;
#pragma unroll
    for (int cw = 0; cw < WMAX; ++cw) {
        if (cw >= W) break;
        const int c = 64 * cw + lane;
#pragma unroll
        for (int s = 0; s < WMAX; ++s) {
            if (s >= W) break;
            const uint64_t col = wave_transpose64(row[s][cw]);
            if (c < n && col != sm.orig[c * W + s]) bad = true;
        }
    }
    if (__ballot(bad)) {
        if (lane == 0) {
            *out.rank = 0;
            *out.status = HLF_ENOTSYM;
        }
        return -1;
    }

    // Gauss-Jordan over GF(2), column by column.
    int r = 0, nfree = 0;
#pragma unroll
    for (int cw = 0; cw < WMAX; ++cw) {
        if (cw >= W) break;
        for (int cb = 0; cb < 64; ++cb) {
            const int c = 64 * cw + cb;
            if (c >= n) break;
            int ps = -1, pl = 0;
#pragma unroll
            for (int s = 0; s < WMAX; ++s) {
                const bool cand = (s < W) && !used[s] && ((row[s][cw] >> cb) & 1ull);
                const uint64_t m = __ballot(cand);
                if (ps < 0 && m) {
                    ps = s;
                    pl = __builtin_ctzll(m);
                }
            }
            if (ps < 0) {
                if (lane == 0) sm.freec[nfree] = c;
                ++nfree;
                continue;
            }
            pl = __builtin_amdgcn_readfirstlane(pl);
            uint64_t prow[WMAX];
#pragma unroll
            for (int w = 0; w < WMAX; ++w) prow[w] = 0;
#pragma unroll
            for (int s = 0; s < WMAX; ++s)
                if (s == ps)
#pragma unroll
                    for (int w = 0; w < WMAX; ++w) prow[w] = readlane64(row[s][w], pl);
#pragma unroll
            for (int s = 0; s < WMAX; ++s) {
                const bool is_p = (s == ps) && (lane == pl);
                if (((row[s][cw] >> cb) & 1ull) && !is_p)
#pragma unroll
                    for (int w = 0; w < WMAX; ++w) row[s][w] ^= prow[w];
                if (is_p) {
                    used[s] = true;
                    rk[s] = r;
                    pc[s] = c;
                }
            }
            if (lane == 0) sm.piv[r] = c;
            ++r;
        }
    }
    if constexpr (WMAX == 1) {
        // One word per row (n <= 64).  P[c] = the reduced pivot row whose
        // pivot column is c, 0 at free columns; transposed across the wave,
        // lane f holds column f of P, whose bit c is that row's entry f, so
        // k_f = e_f | column f of P for a free column f.
        sm.rref[lane] = 0ull;
        wave_lds_sync();
        if (used[0]) sm.rref[pc[0]] = row[0][0];
        wave_lds_sync();
        const uint64_t P = sm.rref[lane];
        if (lane < n) out.pivots[lane] = (lane < r) ? sm.piv[lane] : -1;
        if (lane < r) out.basis[lane] = sm.orig[sm.piv[lane]];
        const uint64_t pivmask = __ballot(P != 0ull);  // a pivot row is never 0
        const uint64_t freemask = __ballot(lane < n) & ~pivmask;
        const bool is_free = (freemask >> lane) & 1ull;
        const uint64_t T = wave_transpose64(P);  // every lane takes part in the exchanges
        const uint64_t kv = is_free ? (T | (1ull << lane)) : 0ull;
        if (out.kernel && is_free) out.kernel[__builtin_popcountll(freemask & ((1ull << lane) - 1ull))] = kv;
        // q(k_f) = sum over i in supp k_f of popcount(A_i & k_f), one uniform
        // step per free column: every term is even (A k_f = 0 mod 2), so bit
        // 1 of the sum is the parity of the terms = 2 mod 4.
        const uint64_t Ai = lane < n ? sm.orig[lane] : 0ull;
        uint64_t shiftbits = 0ull;
        bool internal = false;
        for (uint64_t fm = freemask; fm; fm &= fm - 1ull) {
            const int f = __builtin_ctzll(fm);
            const uint64_t x = readlane64(kv, f);
            const uint32_t term = ((x >> lane) & 1ull) ? (uint32_t)__builtin_popcountll(Ai & x) : 0u;
            if (__ballot(term & 1u)) internal = true;
            if (__builtin_popcountll(__ballot(term & 2u)) & 1) shiftbits |= 1ull << f;
        }
        if (lane == 0) sm.shiftw[0] = shiftbits;
        wave_lds_sync();
        if (lane == 0) {
            out.shift[0] = shiftbits;
            *out.rank = r;
            *out.status = internal ? HLF_EINTERNAL : HLF_OK;
        }
        return internal ? -1 : r;
    } else {
#pragma unroll
        for (int s = 0; s < WMAX; ++s)
            if (used[s])
#pragma unroll
                for (int w = 0; w < WMAX; ++w)
                    if (w < W) sm.rref[rk[s] * W + w] = row[s][w];
        wave_lds_sync();

        for (int k = lane; k < n; k += 64) out.pivots[k] = (k < r) ? sm.piv[k] : -1;
        for (int idx = lane; idx < r * W; idx += 64) {
            const int k = idx / W, w = idx - k * W;
            out.basis[idx] = sm.orig[sm.piv[k] * W + w];
        }

        // Kernel vectors k_f and q(k_f) = sum_{i in supp k_f} popcount(A_i & k_f).
        const int nk = n - r;
        for (int j = lane; j < nk; j += 64) {
            const int f = sm.freec[j];
            uint64_t kv[WMAX];
#pragma unroll
            for (int w = 0; w < WMAX; ++w) kv[w] = 0;
            set_bit<WMAX>(kv, f);
            for (int k = 0; k < r; ++k) {
                if ((sm.rref[k * W + (f >> 6)] >> (f & 63)) & 1ull) set_bit<WMAX>(kv, sm.piv[k]);
            }
            if (out.kernel)
#pragma unroll
                for (int w = 0; w < WMAX; ++w)
                    if (w < W) out.kernel[j * W + w] = kv[w];
            uint32_t q = 0;
#pragma unroll
            for (int iw = 0; iw < WMAX; ++iw) {
                uint64_t bits = kv[iw];
                while (bits) {
                    const int i = iw * 64 + __builtin_ctzll(bits);
                    bits &= bits - 1;
#pragma unroll
                    for (int w = 0; w < WMAX; ++w)
                        if (w < W) q += __builtin_popcountll(sm.orig[i * W + w] & kv[w]);
                }
            }
            if (q & 1u) sm.internal = 1;
            if (q & 2u) atomicOr(&sm.shiftw[f >> 6], 1ull << (f & 63));
        }
        wave_lds_sync();
        if (lane < W) out.shift[lane] = sm.shiftw[lane];
        const bool internal = sm.internal != 0;
        if (lane == 0) {
            *out.rank = r;
            *out.status = internal ? HLF_EINTERNAL : HLF_OK;
        }
        return internal ? -1 : r;
    }
}

}  // namespace hlf
