// Stage 2 of the two-stage scheme (the paper's classical parallel circuit,
// Section 2, Eqs. (1)-(3) and the final CNOT layer): device code shared by the
// single-instance and the batched kernels.
//
// Solution i is z_i = l ^ XOR_{bit k of g(i)} B_k with g(i) = i ^ (i >> 1).
// Writing E_j = B_j ^ B_{j-1} (B_{-1} = 0) turns this into an affine map of
// the bits of i itself:  z_i = l ^ F(i),  F(i) = XOR_{bit j of i} E_j.
// For an index split i = (T << S) | x with x < 2^S,
//     z_i = (l ^ F(x)) ^ F(T << S):
// a per-lane constant XOR a per-tile constant.  Moving from tile T to T+1
// changes the tile constant by F(((T+1) ^ T) << S) = B_{S-1} ^ B_{S+ctz(T+1)}
// (the sum telescopes): the Gray-code step lifted to whole tiles.
//
// Over a tile that lies inside [0, 2^r) the solutions form the coset
// z(T << S) ^ span(B_0 .. B_{S-1}).  Bit j is therefore set in exactly half of
// them when some B_k (k < S) has bit j set, and otherwise in all or none of
// them according to bit j of z(T << S); the XOR of the coset is zero (S >= 2).
// The reduce routines use this for the per-qubit counts of whole tiles; the
// hash is evaluated on every solution.
#pragma once

#include "hlf_device.h"
#include "hlf_internal.h"

namespace hlf {


// Status/range gate of every stage-2 kernel.  Returns false (and the caller
// writes nothing) if the record is bad or [begin, begin+count) is not inside
// [0, 2^r); the verdict is the same for every block.
__device__ __forceinline__ bool gate(int32_t *status, const int32_t *rank, uint64_t begin,
                                     uint64_t count, int &r) {
    if (*(volatile int32_t *)status != HLF_OK) return false;
    r = *rank;
    if (r > HLF_MAX_ENUM_RANK || begin > (1ull << r) || count > (1ull << r) - begin) {
        if (threadIdx.x == 0) *status = HLF_ERANGE;
        return false;
    }
    return true;
}

// Bx[j*WW + w] = word w of B_j for j < r, zero for r <= j < 64.
template <int WW>
__device__ __forceinline__ void load_basis_padded(const uint64_t *__restrict__ basis, int r,
                                                  uint64_t *Bx, int tid, int nthreads) {
    for (int idx = tid; idx < 64 * WW; idx += nthreads) {
        const int j = idx / WW;
        Bx[idx] = (j < r) ? basis[idx] : 0ull;
    }
}

template <int WW>
__device__ __forceinline__ uint64_t E_at(const uint64_t *Bx, int j, int w) {
    return Bx[j * WW + w] ^ (j ? Bx[(j - 1) * WW + w] : 0ull);
}

// Word w of F(x) for x < 2^bits.
template <int WW>
__device__ __forceinline__ uint64_t F_low(const uint64_t *Bx, uint64_t x, int bits, int w) {
    uint64_t v = 0;
    for (int j = 0; j < bits; ++j)
        if ((x >> j) & 1ull) v ^= E_at<WW>(Bx, j, w);
    return v;
}

// Word w of F(T << S).
template <int WW>
__device__ __forceinline__ uint64_t F_tile(const uint64_t *Bx, uint64_t T, int S, int w) {
    uint64_t v = 0;
    for (int j = 0; j + S < 64 && (T >> j); ++j)
        if ((T >> j) & 1ull) v ^= E_at<WW>(Bx, S + j, w);
    return v;
}

// Word w of the tile-constant step from T to T+1.
template <int WW>
__device__ __forceinline__ uint64_t tile_step(const uint64_t *Bx, uint64_t T, int S, int w) {
    const int c = S + __builtin_ctzll(T + 1);
    return Bx[(S - 1) * WW + w] ^ Bx[(c < 63 ? c : 63) * WW + w];
}

// ---------------------------------------------------------------------------
// Materialise, W = 1, 16/32/64-bit words: V values per 16-byte store.
// ---------------------------------------------------------------------------
template <typename T>
struct Vec {
    static constexpr int V = 16 / (int)sizeof(T);  // values per 16-byte store
    static constexpr int LOGV = (V == 8) ? 3 : (V == 4) ? 2 : 1;
};

// Materialise workgroups: 1024 threads, one 16-byte store per thread per
// tile, so a tile holds 1024*V solutions.
constexpr int kTileThreads = 1024;
constexpr int kLogTileThreads = 10;
// Workgroups per CU of the one-launch solve kernel (more workgroups than
// resident slots: the dispatcher balances the tail).
constexpr int kTileBlocksPerCU = 16;
// Materialise kernels give each workgroup a short contiguous range of about
// kBlockBytes of output, and a launch holds many more workgroups than fit on
// the device, so the resident ones are at different points of their ranges
// (resident workgroups that write in step at a fixed stride lose 5-15% of
// the write bandwidth).  Longer ranges only for grids beyond kMaxTileBlocks.
constexpr uint64_t kBlockBytes = 128ull << 10;
constexpr uint64_t kMaxTileBlocks = 1ull << 30;

// Tiles per workgroup for a materialise launch over ntiles tiles of
// tile_bytes bytes each; a launch too small to give every CU two workgroups
// at that size is spread thinner.
inline uint64_t materialise_tiles_per_block(uint64_t ntiles, uint64_t tile_bytes) {
    uint64_t want = kBlockBytes / tile_bytes ? kBlockBytes / tile_bytes : 1;
    const uint64_t spread = 2ull * (uint64_t)device_cu_count();
    const uint64_t thin = (ntiles + spread - 1) / spread;
    if (thin < want) want = thin ? thin : 1;
    const uint64_t need = (ntiles + kMaxTileBlocks - 1) / kMaxTileBlocks;
    return need > want ? need : want;
}

// Bytes of one tile of the W = 1 materialise kernels (one 16-byte store per
// thread).
constexpr uint64_t kTileBytes = 16ull * kTileThreads;
// Grids up to this many workgroups seed their lane constants the short way.
constexpr unsigned kShortSeedGrid = 512;

// Workgroups are dealt to the 8 XCDs in turn, so dispatch index b runs on XCD
// b % 8.  xcd_block maps b (of n) to the block index it materialises such that
// each XCD's workgroups take one contiguous run of blocks, in order: XCD x
// takes the q or q + 1 blocks from x*q + min(x, n % 8) on, q = n / 8.  Stores
// from one XCD then stay in one region instead of interleaving with the other
// seven XCDs' every 128 KiB, which the HBM write rate favours.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t n) {
    const uint32_t x = b & 7u, q = n >> 3, rem = n & 7u;
    return x * q + (x < rem ? x : rem) + (b >> 3);
}

template <typename T>
__host__ __device__ constexpr int tile_shift() {
    return kLogTileThreads + Vec<T>::LOGV;
}

template <typename T>
__device__ __forceinline__ void pack16(const uint64_t *v, uint32_t (&w)[4]) {
    if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            w[k] = (uint32_t)(v[2 * k] & 0xFFFFu) | ((uint32_t)v[2 * k + 1] << 16);
    } else if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = (uint32_t)v[k];
    } else {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            w[2 * k] = (uint32_t)v[k];
            w[2 * k + 1] = (uint32_t)(v[k] >> 32);
        }
    }
}

template <typename T>
__device__ __forceinline__ void spread16(uint64_t h, uint32_t (&w)[4]) {
    if constexpr (sizeof(T) == 2) {
        const uint32_t x = (uint32_t)(h & 0xFFFFu) * 0x10001u;
        w[0] = w[1] = w[2] = w[3] = x;
    } else if constexpr (sizeof(T) == 4) {
        w[0] = w[1] = w[2] = w[3] = (uint32_t)h;
    } else {
        w[0] = w[2] = (uint32_t)h;
        w[1] = w[3] = (uint32_t)(h >> 32);
    }
}

// Tiles [t0, t1) (relative to the first tile of [begin, begin+count)) of one
// instance, by a kTileThreads workgroup; out[i - begin] = z_i.  Requires
// begin % V == 0 and a 16-byte aligned `out`.  Bx: LDS basis (WW = 1).
template <typename T>
__device__ void enum_tiles_w1(const uint64_t *Bx, uint64_t l, uint64_t begin, uint64_t count,
                              T *__restrict__ out, uint64_t t0, uint64_t t1) {
    constexpr int V = Vec<T>::V;
    constexpr int S = tile_shift<T>();
    constexpr int LOGV = Vec<T>::LOGV;
    const int tid = threadIdx.x;
    // Lane constants l ^ F(tid*V + e).  F is linear in the bits of the index,
    // so F(tid*V + e) = F(tid << LOGV) ^ F(e): about LOGV + 10 lookups instead
    // of V * S.  The workgroups that start with the launch (all of a launch
    // that fits on the device at once) take the short form: their start-up
    // is the launch's ramp.  The later ones keep the per-index form, whose
    // longer start-up spreads their first stores (measured about 1% faster
    // than the short form everywhere).
    uint64_t lo[V];
    if (gridDim.x <= kShortSeedGrid || blockIdx.x < kShortSeedGrid) {
        uint64_t base = l;
#pragma unroll
        for (int j = 0; j < kLogTileThreads; ++j)
            if ((tid >> j) & 1) base ^= E_at<1>(Bx, LOGV + j, 0);
#pragma unroll
        for (int e = 0; e < V; ++e) lo[e] = base ^ F_low<1>(Bx, (uint64_t)e, LOGV, 0);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) lo[e] = l ^ F_low<1>(Bx, (uint64_t)(tid * V + e), S, 0);
    }
    uint32_t lw[4];
    pack16<T>(lo, lw);

    const uint64_t end = begin + count;
    uint64_t Tt = (begin >> S) + t0;
    uint64_t hi = F_tile<1>(Bx, Tt, S, 0);
    for (uint64_t t = t0; t < t1; ++t, ++Tt) {
        const uint64_t i0 = (Tt << S) + (uint64_t)(tid * V);
        if (i0 >= begin && i0 + V <= end) {
            uint32_t hw[4];
            spread16<T>(hi, hw);
            u32x4 val;
            val.x = lw[0] ^ hw[0];
            val.y = lw[1] ^ hw[1];
            val.z = lw[2] ^ hw[2];
            val.w = lw[3] ^ hw[3];
            __builtin_nontemporal_store(val, (u32x4 *)(out + (i0 - begin)));
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const uint64_t i = i0 + e;
                if (i >= begin && i < end) out[i - begin] = (T)(lo[e] ^ hi);
            }
        }
        hi ^= tile_step<1>(Bx, Tt, S, 0);
    }
}

// ---------------------------------------------------------------------------
// Reduce on one wavefront, W = WW words (n <= 64*WW).  Tiles of 64*U indices.
// ---------------------------------------------------------------------------
template <int WW>
struct WaveReduce {
    static constexpr int U = (WW == 1) ? 16 : 8;
    static constexpr int S = (WW == 1) ? 10 : 9;  // log2(64 * U)
};

template <int WW>
struct WavePartial {
    uint64_t hash;     // wave total (same on every lane)
    uint64_t cnt[WW];  // this lane's count of bit 64*w + lane
    uint64_t xf[WW];   // wave XOR (same on every lane)
};

// Counts, hash and XOR-fold over the solutions z_i, i in [c0, c1) of one
// instance (c1 <= 2^r, r <= 62).  Bx: basis words, padded; l: shift words.
template <int WW>
__device__ WavePartial<WW> wave_reduce_range(const uint64_t *Bx, const uint64_t (&l)[WW], int n,
                                             int r, uint64_t c0, uint64_t c1) {
    constexpr int U = WaveReduce<WW>::U;
    constexpr int S = WaveReduce<WW>::S;
    const int lane = lane_id();
    WavePartial<WW> p;
    p.hash = 0;
#pragma unroll
    for (int w = 0; w < WW; ++w) p.cnt[w] = p.xf[w] = 0;
    if (c0 >= c1) return p;

    uint64_t lo[U][WW];
    uint64_t loh[U];  // mix13_head of word 0 (the first step of mix13 is GF(2)-linear)
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int w = 0; w < WW; ++w) lo[u][w] = l[w] ^ F_low<WW>(Bx, (uint64_t)(u * 64 + lane), S, w);
        loh[u] = mix13_head(lo[u][0]);
    }

    uint64_t acc = 0, nfull = 0;
    uint64_t ones[WW], pc[WW], xacc[WW];
#pragma unroll
    for (int w = 0; w < WW; ++w) ones[w] = pc[w] = xacc[w] = 0;
    uint64_t Tt = c0 >> S;
    const uint64_t Tend = ((c1 - 1) >> S) + 1;
    uint64_t hi[WW];
#pragma unroll
    for (int w = 0; w < WW; ++w) hi[w] = F_tile<WW>(Bx, Tt, S, w);

    for (; Tt < Tend; ++Tt) {
        const uint64_t tb = Tt << S;
        if (tb >= c0 && tb + (1ull << S) <= c1) {
            // h(z) = chain over words of mix13(h ^ z_w ^ GAMMA), z = lo ^ hi
            const uint64_t hgh = uniform64(mix13_head(hi[0] ^ kGamma));
            uint64_t hg[WW];
#pragma unroll
            for (int w = 1; w < WW; ++w) hg[w] = uniform64(hi[w] ^ kGamma);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint64_t h = mix13_tail(loh[u] ^ hgh);
#pragma unroll
                for (int w = 1; w < WW; ++w) h = mix13(h ^ lo[u][w] ^ hg[w]);
                acc += h;
            }
            ++nfull;
#pragma unroll
            for (int w = 0; w < WW; ++w) ones[w] += ((l[w] ^ hi[w]) >> lane) & 1ull;
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i = tb + (uint64_t)(u * 64 + lane);
                const bool valid = (i >= c0) && (i < c1);
                uint64_t z[WW];
#pragma unroll
                for (int w = 0; w < WW; ++w) z[w] = lo[u][w] ^ hi[w];
                if (valid) {
                    uint64_t h = 0;
#pragma unroll
                    for (int w = 0; w < WW; ++w) {
                        h = mix13(h ^ z[w] ^ kGamma);
                        xacc[w] ^= z[w];
                    }
                    acc += h;
                }
                // Lane b counts bit 64w + b over the valid lanes: bit b of z[w]
                // across the lanes is lane b's word after the wave transpose
                // (bits at or past n are zero in every solution).
                const uint64_t vm = __ballot(valid);
#pragma unroll
                for (int w = 0; w < WW; ++w)
                    pc[w] += (uint64_t)__builtin_popcountll(wave_transpose64(z[w]) & vm);
            }
        }
#pragma unroll
        for (int w = 0; w < WW; ++w) hi[w] ^= tile_step<WW>(Bx, Tt, S, w);
    }

    p.hash = wave_sum_u64(acc);
#pragma unroll
    for (int w = 0; w < WW; ++w) {
        p.xf[w] = wave_xor_u64(xacc[w]);
        uint64_t orS = 0;
        for (int k = 0; k < S && k < r; ++k) orS |= Bx[k * WW + w];
        uint64_t c = pc[w];
        if (nfull) c += ((orS >> lane) & 1ull) ? (nfull << (S - 1)) : (ones[w] << S);
        p.cnt[w] = c;
    }
    return p;
}

}  // namespace hlf
