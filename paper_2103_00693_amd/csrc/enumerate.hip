// Stage 2 of the two-stage scheme (the paper's classical parallel circuit,
// Section 2, Eqs. (1)-(3) and the final CNOT layer) on gfx950.
//
// Solution i is z_i = l ^ XOR_{bit k of g(i)} B_k with g(i) = i ^ (i >> 1).
// Writing E_j = B_j ^ B_{j-1} (B_{-1} = 0) turns this into an affine map of
// the bits of i itself:  z_i = l ^ F(i),  F(i) = XOR_{bit j of i} E_j.
// Consequently, for an index split i = (T << S) | x with x < 2^S,
//     z_i = (l ^ F(x)) ^ F(T << S):
// a per-lane constant XOR a per-tile constant.  Moving from tile T to T+1
// changes the tile constant by F(((T+1) ^ T) << S) = B_{S-1} ^ B_{S+ctz(T+1)}
// (the sum telescopes) -- the Gray-code step lifted to whole tiles.
//
// Kernels:
//   enum_tile_kernel<T>    W = 1, 16/32/64-bit words, begin a multiple of
//                          the 16-byte vector: every lane keeps its V
//                          per-lane constants in VGPRs and emits one 16-byte
//                          nontemporal store per tile; blocks walk contiguous
//                          tile ranges.
//   enum_general_kernel    any W, any begin/alignment: z_i from LDS lookup
//                          tables over the bytes (W = 1) or nibbles (W > 1)
//                          of i (method of four Russians).
//   reduce_tile_kernel<U>  W = 1: per-qubit ones-counts, order-independent
//                          hash and XOR-fold over [begin, begin+count).  The
//                          hash is evaluated per solution; counts and XOR-fold
//                          of a whole tile follow in closed form from the
//                          tile's coset structure (below); partial tiles are
//                          counted element by element with wave ballots.
//   reduce_general_kernel  W > 1: element by element.
#include "hlf_device.h"
#include "hlf_internal.h"

namespace hlf {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Status/range gate shared by every stage-2 kernel.  Returns false (and the
// caller does nothing) if the record is bad or the range lies outside
// [0, 2^r); the range verdict is the same for every block.
__device__ __forceinline__ bool gate(const FactorIn &f, uint64_t begin, uint64_t count, int &r) {
    if (*(volatile int32_t *)f.status != HLF_OK) return false;
    r = *f.rank;
    if (r > HLF_MAX_ENUM_RANK || begin > (1ull << r) || count > (1ull << r) - begin) {
        if (threadIdx.x == 0) *f.status = HLF_ERANGE;
        return false;
    }
    return true;
}

// B_j for j < r, zero above: Bx[j] ^ Bx[j-1] is E_j.
__device__ __forceinline__ void load_basis_w1(const FactorIn &f, int r, uint64_t *Bx) {
    if (threadIdx.x < 64) Bx[threadIdx.x] = ((int)threadIdx.x < r) ? f.basis[threadIdx.x] : 0ull;
}

__device__ __forceinline__ uint64_t E_at(const uint64_t *Bx, int j) {
    return Bx[j] ^ (j ? Bx[j - 1] : 0ull);
}

// F(x) for x < 2^bits, W = 1.
__device__ __forceinline__ uint64_t F_low(const uint64_t *Bx, uint64_t x, int bits) {
    uint64_t v = 0;
    for (int j = 0; j < bits; ++j)
        if ((x >> j) & 1ull) v ^= E_at(Bx, j);
    return v;
}

// F(T << S) for a tile index T.
__device__ __forceinline__ uint64_t F_tile(const uint64_t *Bx, uint64_t T, int S) {
    uint64_t v = 0;
    for (int j = 0; j + S < 64 && (T >> j); ++j)
        if ((T >> j) & 1ull) v ^= E_at(Bx, S + j);
    return v;
}

template <typename T>
struct Vec;
template <>
struct Vec<uint16_t> {
    static constexpr int V = 8;
    static constexpr int S = 11;  // log2(256 * 8)
};
template <>
struct Vec<uint32_t> {
    static constexpr int V = 4;
    static constexpr int S = 10;
};
template <>
struct Vec<uint64_t> {
    static constexpr int V = 2;
    static constexpr int S = 9;
};

// 32-bit lanes of a 16-byte vector of V values v[0..V-1].
template <typename T>
__device__ __forceinline__ void pack16(const uint64_t *v, uint32_t (&w)[4]) {
    if constexpr (sizeof(T) == 2) {
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = (uint32_t)(v[2 * k] & 0xFFFFu) | ((uint32_t)v[2 * k + 1] << 16);
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

// The tile constant replicated over the 32-bit lanes of a 16-byte vector.
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

constexpr int kTileThreads = 256;

template <typename T>
__global__ __launch_bounds__(kTileThreads) void enum_tile_kernel(FactorIn f, uint64_t begin,
                                                                 uint64_t count,
                                                                 T *__restrict__ out,
                                                                 uint64_t tiles_per_block) {
    constexpr int V = Vec<T>::V;
    constexpr int S = Vec<T>::S;
    __shared__ uint64_t Bx[64];
    int r;
    if (!gate(f, begin, count, r)) return;
    load_basis_w1(f, r, Bx);
    __syncthreads();

    const int tid = threadIdx.x;
    const uint64_t l = f.shift[0];
    uint64_t lo[V];
#pragma unroll
    for (int e = 0; e < V; ++e) lo[e] = l ^ F_low(Bx, (uint64_t)(tid * V + e), S);
    uint32_t lw[4];
    pack16<T>(lo, lw);

    const uint64_t end = begin + count;
    const uint64_t first_tile = begin >> S;
    const uint64_t ntiles = ((end - 1) >> S) - first_tile + 1;
    const uint64_t t0 = (uint64_t)blockIdx.x * tiles_per_block;
    if (t0 >= ntiles) return;
    const uint64_t t1 = (t0 + tiles_per_block < ntiles) ? t0 + tiles_per_block : ntiles;
    uint64_t Tt = first_tile + t0;
    uint64_t hi = F_tile(Bx, Tt, S);
    const uint64_t step_lo = Bx[S - 1];

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
        const int c = __builtin_ctzll(Tt + 1);
        hi ^= step_lo ^ Bx[(S + c) < 63 ? (S + c) : 63];
    }
}

// ---------------------------------------------------------------------------
// General materialise: z_i = l ^ XOR_m Tab[m][digit m of i].
// W = 1: 8 byte tables of 256 entries (16 KiB); W > 1: 16 nibble tables of
// 16 entries, W words each (<= 32 KiB).
// ---------------------------------------------------------------------------
template <int WMAX>
struct GenTables {
    static constexpr int kDigitBits = (WMAX == 1) ? 8 : 4;
    static constexpr int kDigits = 64 / kDigitBits;
    static constexpr int kEntries = 1 << kDigitBits;
    uint64_t tab[kDigits * kEntries * WMAX];
    uint64_t l[WMAX];
};

// Build tables from E_j = B_j ^ B_{j-1}; returns the number of digits in use.
template <int WMAX>
__device__ int build_tables(const FactorIn &f, int r, int W, GenTables<WMAX> &g) {
    using G = GenTables<WMAX>;
    const int ndig = (r + G::kDigitBits - 1) / G::kDigitBits;
    for (int idx = threadIdx.x; idx < ndig * G::kEntries; idx += blockDim.x) {
        const int m = idx / G::kEntries, v = idx - m * G::kEntries;
        for (int w = 0; w < W; ++w) {
            uint64_t acc = 0;
            for (int q = 0; q < G::kDigitBits; ++q) {
                const int j = m * G::kDigitBits + q;
                if (((v >> q) & 1) && j < r) {
                    acc ^= f.basis[(size_t)j * W + w];
                    if (j > 0) acc ^= f.basis[(size_t)(j - 1) * W + w];
                }
            }
            g.tab[idx * WMAX + w] = acc;
        }
    }
    if ((int)threadIdx.x < W) g.l[threadIdx.x] = f.shift[threadIdx.x];
    return ndig;
}

template <int WMAX, typename T>
__global__ __launch_bounds__(256) void enum_general_kernel(FactorIn f, uint64_t begin,
                                                           uint64_t count, T *__restrict__ out) {
    using G = GenTables<WMAX>;
    __shared__ G g;
    int r;
    if (!gate(f, begin, count, r)) return;
    const int W = f.words;
    const int ndig = build_tables<WMAX>(f, r, W, g);
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride) {
        const uint64_t i = begin + j;
        uint64_t z[WMAX];
#pragma unroll
        for (int w = 0; w < WMAX; ++w) z[w] = (w < W) ? g.l[w] : 0ull;
        for (int m = 0; m < ndig; ++m) {
            const int d = (int)((i >> (m * G::kDigitBits)) & (G::kEntries - 1));
            const uint64_t *e = &g.tab[(m * G::kEntries + d) * WMAX];
#pragma unroll
            for (int w = 0; w < WMAX; ++w) z[w] ^= e[w];
        }
        if constexpr (WMAX == 1) {
            out[j] = (T)z[0];
        } else {
#pragma unroll
            for (int w = 0; w < WMAX; ++w)
                if (w < W) out[j * W + w] = z[w];
        }
    }
}

// ---------------------------------------------------------------------------
// Reduce, W = 1.  Tiles are aligned in absolute index space: tile T covers
// [T << S, (T+1) << S), S = log2(256 * U).  Thread t handles x = u*256 + t.
// Over a tile that lies inside [begin, end) and [0, 2^r), the solutions form
// the coset z(T << S) ^ span(B_0 .. B_{S-1}); so bit j is set in exactly half
// of them when some B_k (k < S) has bit j set, and otherwise in all or none
// of them according to bit j of z(T << S).  The XOR of a coset of dimension
// S >= 2 is zero.  The hash needs every solution: h(z) = mix13(z ^ GAMMA).
// ---------------------------------------------------------------------------
template <int U>
struct ReduceShape {
    static constexpr int S = (U == 8) ? 11 : (U == 16) ? 12 : (U == 4) ? 10 : 13;
};

template <int U>
__global__ __launch_bounds__(kTileThreads) void reduce_tile_kernel(
    FactorIn f, uint64_t begin, uint64_t count, uint64_t tiles_per_block,
    uint64_t *__restrict__ counts, uint64_t *__restrict__ hash, uint64_t *__restrict__ xorfold) {
    constexpr int S = ReduceShape<U>::S;
    static_assert((kTileThreads * U) == (1 << S), "tile shape");
    __shared__ uint64_t Bx[64];
    __shared__ unsigned long long part[64];
    int r;
    if (!gate(f, begin, count, r)) return;
    load_basis_w1(f, r, Bx);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (tid < 64) part[tid] = 0;
    __syncthreads();

    const int n = f.n;
    const uint64_t l = f.shift[0];
    uint64_t lo[U];
#pragma unroll
    for (int u = 0; u < U; ++u) lo[u] = l ^ F_low(Bx, (uint64_t)(u * kTileThreads + tid), S);

    const uint64_t end = begin + count;
    const uint64_t first_tile = begin >> S;
    const uint64_t ntiles = ((end - 1) >> S) - first_tile + 1;
    const uint64_t t0 = (uint64_t)blockIdx.x * tiles_per_block;
    uint64_t acc = 0;       // sum of h(z), this thread
    uint64_t xacc = 0;      // XOR of z over partial tiles, this thread
    uint64_t nfull = 0;     // full tiles of this block
    uint64_t ones = 0;      // thread j < n: full tiles whose first solution has bit j
    uint64_t pcnt = 0;      // lane j < n: bit-j count over partial tiles, this wave
    if (t0 < ntiles) {
        const uint64_t t1 = (t0 + tiles_per_block < ntiles) ? t0 + tiles_per_block : ntiles;
        uint64_t Tt = first_tile + t0;
        uint64_t hi = F_tile(Bx, Tt, S);
        const uint64_t step_lo = Bx[S - 1];
        for (uint64_t t = t0; t < t1; ++t, ++Tt) {
            const uint64_t tb = Tt << S;
            if (tb >= begin && tb + (1ull << S) <= end) {
                const uint64_t hg = hi ^ kGamma;
#pragma unroll
                for (int u = 0; u < U; ++u) acc += mix13(lo[u] ^ hg);
                ++nfull;
                if (tid < n) ones += ((l ^ hi) >> tid) & 1ull;
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const uint64_t i = tb + (uint64_t)(u * kTileThreads + tid);
                    const bool valid = (i >= begin) && (i < end);
                    const uint64_t z = lo[u] ^ hi;
                    if (valid) {
                        acc += mix13(z ^ kGamma);
                        xacc ^= z;
                    }
                    for (int j = 0; j < n; ++j) {
                        const uint64_t m = __ballot(valid && ((z >> j) & 1ull));
                        if (lane == j) pcnt += (uint64_t)__builtin_popcountll(m);
                    }
                }
            }
            const int c = __builtin_ctzll(Tt + 1);
            hi ^= step_lo ^ Bx[(S + c) < 63 ? (S + c) : 63];
        }
    }

    // hash and XOR-fold: wave sums, one atomic per wave
    const uint64_t wsum = wave_sum_u64(acc);
    const uint64_t wx = wave_xor_u64(xacc);
    if (lane == 0) {
        if (wsum) atomicAdd((unsigned long long *)hash, (unsigned long long)wsum);
        if (xorfold && wx) atomicXor((unsigned long long *)xorfold, (unsigned long long)wx);
    }
    if (lane < n && pcnt) atomicAdd(&part[lane], (unsigned long long)pcnt);
    __syncthreads();
    if (tid < n) {
        uint64_t orS = 0;
        for (int k = 0; k < S && k < r; ++k) orS |= Bx[k];
        uint64_t c = part[tid];
        if (nfull) c += ((orS >> tid) & 1ull) ? (nfull << (S - 1)) : (ones << S);
        if (c) atomicAdd((unsigned long long *)&counts[tid], (unsigned long long)c);
    }
}

// Reduce for W > 1, element by element (tables as in enum_general_kernel).
template <int WMAX>
__global__ __launch_bounds__(256) void reduce_general_kernel(FactorIn f, uint64_t begin,
                                                             uint64_t count,
                                                             uint64_t *__restrict__ counts,
                                                             uint64_t *__restrict__ hash,
                                                             uint64_t *__restrict__ xorfold) {
    using G = GenTables<WMAX>;
    __shared__ G g;
    __shared__ unsigned long long part[64 * WMAX];
    int r;
    if (!gate(f, begin, count, r)) return;
    const int W = f.words;
    const int n = f.n;
    const int ndig = build_tables<WMAX>(f, r, W, g);
    for (int j = threadIdx.x; j < 64 * WMAX; j += blockDim.x) part[j] = 0;
    __syncthreads();
    const int lane = lane_id();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    uint64_t xacc[WMAX];
    uint64_t pc[WMAX];  // lane j: count of bit 64*w + j
#pragma unroll
    for (int w = 0; w < WMAX; ++w) xacc[w] = pc[w] = 0;
    // Every lane of a wave runs the same number of iterations (ballots).
    const uint64_t base0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u);
    for (uint64_t jb = base0; jb < count; jb += stride) {
        const uint64_t j = jb + lane;
        const bool valid = j < count;
        const uint64_t i = begin + (valid ? j : 0);
        uint64_t z[WMAX];
#pragma unroll
        for (int w = 0; w < WMAX; ++w) z[w] = (w < W) ? g.l[w] : 0ull;
        for (int m = 0; m < ndig; ++m) {
            const int d = (int)((i >> (m * G::kDigitBits)) & (G::kEntries - 1));
            const uint64_t *e = &g.tab[(m * G::kEntries + d) * WMAX];
#pragma unroll
            for (int w = 0; w < WMAX; ++w) z[w] ^= e[w];
        }
        if (valid) {
            uint64_t h = 0;
#pragma unroll
            for (int w = 0; w < WMAX; ++w)
                if (w < W) h = mix13(h ^ z[w] ^ kGamma);
            acc += h;
#pragma unroll
            for (int w = 0; w < WMAX; ++w) xacc[w] ^= z[w];
        }
#pragma unroll
        for (int w = 0; w < WMAX; ++w) {
            if (w >= W) break;
            for (int b = 0; b < 64; ++b) {
                const uint64_t m = __ballot(valid && ((z[w] >> b) & 1ull));
                if (lane == b) pc[w] += (uint64_t)__builtin_popcountll(m);
            }
        }
    }
    const uint64_t wsum = wave_sum_u64(acc);
    if (lane == 0 && wsum) atomicAdd((unsigned long long *)hash, (unsigned long long)wsum);
#pragma unroll
    for (int w = 0; w < WMAX; ++w) {
        if (w >= W) break;
        const uint64_t wx = wave_xor_u64(xacc[w]);
        if (xorfold && lane == 0 && wx) atomicXor((unsigned long long *)&xorfold[w], (unsigned long long)wx);
        const int bit = 64 * w + lane;
        if (bit < n && pc[w]) atomicAdd(&part[bit], (unsigned long long)pc[w]);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x)
        if (part[j]) atomicAdd((unsigned long long *)&counts[j], part[j]);
}

// Overwrite mode: zero the outputs first (a kernel, so the call stays
// capturable in a graph).
__global__ void zero_outputs_kernel(FactorIn f, uint64_t begin, uint64_t count, int n, int W,
                                    uint64_t *counts, uint64_t *hash, uint64_t *xorfold) {
    int r;
    if (!gate(f, begin, count, r)) return;
    for (int j = threadIdx.x; j < n; j += blockDim.x) counts[j] = 0;
    if (threadIdx.x == 0) *hash = 0;
    if (xorfold)
        for (int w = threadIdx.x; w < W; w += blockDim.x) xorfold[w] = 0;
}

uint64_t tiles_per_block_for(uint64_t ntiles, uint64_t max_blocks, uint64_t *blocks) {
    uint64_t b = ntiles < max_blocks ? ntiles : max_blocks;
    if (b == 0) b = 1;
    const uint64_t tpb = (ntiles + b - 1) / b;
    *blocks = (ntiles + tpb - 1) / tpb;
    return tpb;
}

template <typename T>
hlf_status launch_tile(const FactorIn &f, uint64_t begin, uint64_t count, T *out,
                       hipStream_t stream) {
    constexpr int S = Vec<T>::S;
    const uint64_t end = begin + count;  // host: may wrap only for invalid ranges
    uint64_t ntiles;
    if (end < begin) {
        ntiles = 1;  // invalid range: the device gate reports HLF_ERANGE
    } else {
        ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    }
    uint64_t blocks;
    const uint64_t tpb = tiles_per_block_for(ntiles, (uint64_t)device_cu_count() * 8, &blocks);
    hipLaunchKernelGGL(enum_tile_kernel<T>, dim3((unsigned)blocks), dim3(kTileThreads), 0, stream,
                       f, begin, count, out, tpb);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int WMAX, typename T>
hlf_status launch_general(const FactorIn &f, uint64_t begin, uint64_t count, T *out,
                          hipStream_t stream) {
    uint64_t blocks = (count + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL((enum_general_kernel<WMAX, T>), dim3((unsigned)blocks), dim3(256), 0,
                       stream, f, begin, count, out);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int WMAX>
hlf_status launch_reduce_general(const FactorIn &f, uint64_t begin, uint64_t count,
                                 uint64_t *counts, uint64_t *hash, uint64_t *xorfold,
                                 hipStream_t stream) {
    uint64_t blocks = (count + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(reduce_general_kernel<WMAX>, dim3((unsigned)blocks), dim3(256), 0, stream,
                       f, begin, count, counts, hash, xorfold);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

constexpr int kReduceU = 8;

}  // namespace

hlf_status launch_enumerate(const FactorIn &f, uint64_t begin, uint64_t count, int word_bits,
                            void *out, hipStream_t stream) {
    const int W = f.words;
    const bool aligned16 = ((uintptr_t)out & 15u) == 0;
    if (W == 1 && word_bits <= 64) {
        if (word_bits == 16) {
            if (aligned16 && begin % Vec<uint16_t>::V == 0)
                return launch_tile<uint16_t>(f, begin, count, (uint16_t *)out, stream);
            return launch_general<1, uint16_t>(f, begin, count, (uint16_t *)out, stream);
        }
        if (word_bits == 32) {
            if (aligned16 && begin % Vec<uint32_t>::V == 0)
                return launch_tile<uint32_t>(f, begin, count, (uint32_t *)out, stream);
            return launch_general<1, uint32_t>(f, begin, count, (uint32_t *)out, stream);
        }
        if (aligned16 && begin % Vec<uint64_t>::V == 0)
            return launch_tile<uint64_t>(f, begin, count, (uint64_t *)out, stream);
        return launch_general<1, uint64_t>(f, begin, count, (uint64_t *)out, stream);
    }
    uint64_t *o = (uint64_t *)out;
    if (W <= 2) return launch_general<2, uint64_t>(f, begin, count, o, stream);
    if (W <= 4) return launch_general<4, uint64_t>(f, begin, count, o, stream);
    if (W <= 8) return launch_general<8, uint64_t>(f, begin, count, o, stream);
    return launch_general<16, uint64_t>(f, begin, count, o, stream);
}

hlf_status launch_reduce(const FactorIn &f, uint64_t begin, uint64_t count, bool accumulate,
                         uint64_t *counts, uint64_t *hash, uint64_t *xorfold,
                         hipStream_t stream) {
    const int W = f.words;
    if (!accumulate) {
        hipLaunchKernelGGL(zero_outputs_kernel, dim3(1), dim3(256), 0, stream, f, begin, count,
                           f.n, W, counts, hash, xorfold);
        if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    }
    if (count == 0) return HLF_OK;
    if (W == 1) {
        constexpr int S = ReduceShape<kReduceU>::S;
        const uint64_t end = begin + count;
        uint64_t ntiles = (end < begin) ? 1 : ((end - 1) >> S) - (begin >> S) + 1;
        uint64_t blocks;
        const uint64_t tpb =
            tiles_per_block_for(ntiles, (uint64_t)device_cu_count() * 8, &blocks);
        hipLaunchKernelGGL(reduce_tile_kernel<kReduceU>, dim3((unsigned)blocks),
                           dim3(kTileThreads), 0, stream, f, begin, count, tpb, counts, hash,
                           xorfold);
        return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
    }
    if (W <= 2) return launch_reduce_general<2>(f, begin, count, counts, hash, xorfold, stream);
    if (W <= 4) return launch_reduce_general<4>(f, begin, count, counts, hash, xorfold, stream);
    if (W <= 8) return launch_reduce_general<8>(f, begin, count, counts, hash, xorfold, stream);
    return launch_reduce_general<16>(f, begin, count, counts, hash, xorfold, stream);
}

}  // namespace hlf
