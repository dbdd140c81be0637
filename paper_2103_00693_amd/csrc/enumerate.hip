// Single-instance stage-2 kernels (materialise and reduce) for gfx950; the
// tile algebra they share with the batched kernels is in stage2.h.
//
//   enum_tile_kernel<T>     W = 1, 16/32/64-bit words, begin a multiple of
//                           the 16-byte vector: per-lane constants in VGPRs,
//                           one 16-byte nontemporal store per lane per tile,
//                           blocks walk contiguous tile ranges.
//   enum_general_kernel     any W, any begin/alignment: z_i from LDS lookup
//                           tables over the bytes (W = 1) or nibbles (W > 1)
//                           of i (method of four Russians).
//   reduce_wave_kernel<WW>  W <= 3: every wavefront reduces a contiguous tile
//                           range (stage2.h); the block combines its waves in
//                           LDS and adds to the outputs with one atomic each.
//   reduce_general_kernel   W > 3: element by element.
#include <type_traits>

#include "hlf_device.h"
#include "hlf_internal.h"
#include "stage2.h"

namespace hlf {
namespace {

__device__ __forceinline__ bool gate(const FactorIn &f, uint64_t begin, uint64_t count, int &r) {
    return hlf::gate(f.status, f.rank, begin, count, r);
}

// Counter order (one word per basis vector): Bx[j] <- B_0 ^ ... ^ B_j for
// j < r, by an inclusive prefix-XOR scan across the 64 lanes of wave 0.  The
// Gray-order walk over these prefix sums visits l ^ XOR_{bit j of i} B_j at
// index i, since g^-1 maps y to its prefix parities (bit j = XOR of y_k,
// k >= j).  The caller synchronises the workgroup afterwards.
__device__ __forceinline__ void prefix_xor_basis_w1(uint64_t *Bx, int r) {
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    uint64_t v = Bx[lane];
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t t = __shfl_up(v, d);
        if (lane >= d) v ^= t;
    }
    if (lane < r) Bx[lane] = v;
}

template <typename T>
__global__ __launch_bounds__(kTileThreads) void enum_tile_kernel(FactorIn f, uint64_t begin,
                                                                 uint64_t count,
                                                                 T *__restrict__ out,
                                                                 uint64_t tiles_per_block,
                                                                 int counter) {
    constexpr int S = tile_shift<T>();
    __shared__ uint64_t Bx[64];
    int r;
    if (!gate(f, begin, count, r)) return;
    load_basis_padded<1>(f.basis, r, Bx, threadIdx.x, blockDim.x);
    __syncthreads();
    if (counter) {
        prefix_xor_basis_w1(Bx, r);
        __syncthreads();
    }
    const uint64_t end = begin + count;
    const uint64_t ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    const uint64_t t0 = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * tiles_per_block;
    if (t0 >= ntiles) return;
    const uint64_t t1 = (t0 + tiles_per_block < ntiles) ? t0 + tiles_per_block : ntiles;
    enum_tiles_w1<T>(Bx, f.shift[0], begin, count, out, t0, t1);
}

// ---------------------------------------------------------------------------
// Materialise, W > 1 words per solution: the tile algebra of the one-word
// kernel with one lane per word.  A tile is 1024 consecutive indices; thread
// (slot, w) = (tid / WMAX, tid % WMAX) holds word w of the per-lane constants
// l ^ F(slot + P*u), u < WMAX, P = 1024 / WMAX, and word w of the tile constant
// F(T << 10); every output word is one XOR and one 8-byte store, and the
// active lanes of a wave store one contiguous run of words.
// ---------------------------------------------------------------------------
template <int WMAX>
__global__ __launch_bounds__(kTileThreads) void enum_wide_tile_kernel(FactorIn f, uint64_t begin,
                                                                      uint64_t count,
                                                                      uint64_t *__restrict__ out,
                                                                      uint64_t tiles_per_block,
                                                                      int counter) {
    constexpr int P = kTileThreads / WMAX;  // solutions per row of the tile
    constexpr int U = WMAX;                 // rows per tile
    constexpr int S = kLogTileThreads;      // log2(P * U)
    constexpr int LOGP = S - (WMAX == 2 ? 1 : WMAX == 4 ? 2 : WMAX == 8 ? 3 : 4);
    __shared__ uint64_t Bx[64 * WMAX];
    int r;
    if (!gate(f, begin, count, r)) return;
    const int W = f.words;
    for (int idx = threadIdx.x; idx < 64 * WMAX; idx += blockDim.x) {
        const int j = idx / WMAX, w = idx - j * WMAX;
        Bx[idx] = (j < r && w < W) ? f.basis[(size_t)j * W + w] : 0ull;
    }
    __syncthreads();
    if (counter) {
        // Prefix sums B_0 ^ ... ^ B_j (j < r) of word w, by wave w.
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (wv < W) {
            uint64_t v = Bx[lane * WMAX + wv];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint64_t t = __shfl_up(v, d);
                if (lane >= d) v ^= t;
            }
            if (lane < r) Bx[lane * WMAX + wv] = v;
        }
        __syncthreads();
    }
    const uint64_t end = begin + count;
    const uint64_t ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    const uint64_t t0 = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * tiles_per_block;
    if (t0 >= ntiles) return;
    const uint64_t t1 = (t0 + tiles_per_block < ntiles) ? t0 + tiles_per_block : ntiles;

    const int w = (int)(threadIdx.x & (WMAX - 1));
    const int slot = (int)(threadIdx.x / WMAX);
    // lo[u] = l ^ F(slot + P*u): F(P * 2^k) = E_{LOGP + k}, built along u.
    uint64_t lo[U];
    lo[0] = ((w < W) ? f.shift[w] : 0ull) ^ F_low<WMAX>(Bx, (uint64_t)slot, LOGP, w);
#pragma unroll
    for (int u = 1; u < U; ++u)
        lo[u] = lo[u & (u - 1)] ^ E_at<WMAX>(Bx, LOGP + __builtin_ctz(u), w);
    uint64_t Tt = (begin >> S) + t0;
    uint64_t hi = F_tile<WMAX>(Bx, Tt, S, w);
    const bool act = w < W;
    for (uint64_t t = t0; t < t1; ++t, ++Tt) {
        const uint64_t base = Tt << S;
        if (base >= begin && base + (1u << S) <= end) {
            if (act) {
                uint64_t *o = out + (base - begin + (uint64_t)slot) * W + w;
#pragma unroll
                for (int u = 0; u < U; ++u)
                    __builtin_nontemporal_store(lo[u] ^ hi, o + (uint64_t)u * P * W);
            }
        } else if (act) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t i = base + (uint64_t)slot + (uint64_t)u * P;
                if (i >= begin && i < end) out[(i - begin) * W + w] = lo[u] ^ hi;
            }
        }
        hi ^= tile_step<WMAX>(Bx, Tt, S, w);
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

// Build tables from E_j = B_j ^ B_{j-1} (Gray order) or E_j = B_j (counter
// order); returns the number of digits in use.
template <int WMAX>
__device__ int build_tables(const FactorIn &f, int r, int W, bool counter, GenTables<WMAX> &g) {
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
                    if (j > 0 && !counter) acc ^= f.basis[(size_t)(j - 1) * W + w];
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
                                                           uint64_t count, T *__restrict__ out,
                                                           int counter) {
    using G = GenTables<WMAX>;
    __shared__ G g;
    int r;
    if (!gate(f, begin, count, r)) return;
    const int W = f.words;
    const int ndig = build_tables<WMAX>(f, r, W, counter != 0, g);
    __syncthreads();
    if constexpr (WMAX == 1) {
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride) {
            const uint64_t i = begin + j;
            uint64_t z = g.l[0];
            for (int m = 0; m < ndig; ++m) {
                const int d = (int)((i >> (m * G::kDigitBits)) & (G::kEntries - 1));
                z ^= g.tab[m * G::kEntries + d];
            }
            out[j] = (T)z;
        }
    } else {
        // WMAX lanes per solution, lane w computes and stores word w: the
        // active lanes of a wave store one contiguous run of words.
        const int w = (int)(threadIdx.x & (WMAX - 1));
        const uint64_t stride = ((uint64_t)gridDim.x * blockDim.x) / WMAX;
        for (uint64_t j = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) / WMAX; j < count;
             j += stride) {
            const uint64_t i = begin + j;
            uint64_t z = (w < W) ? g.l[w] : 0ull;
            for (int m = 0; m < ndig; ++m) {
                const int d = (int)((i >> (m * G::kDigitBits)) & (G::kEntries - 1));
                z ^= g.tab[(m * G::kEntries + d) * WMAX + w];
            }
            if (w < W) out[j * W + w] = z;
        }
    }
}

// ---------------------------------------------------------------------------
// The paper's circuit, evaluated literally (Section 2, Eqs. (1)-(2), Fig. 1(c))
// and fed by the binary counter of the FPGA design (Section 4).  Solution
// number i:
//   R = the bits of i scattered onto the pivot positions (R_{p_k} = bit k),
//   y = ((R & H) << 1) ^ ((R >> 1) & H)        horizontal-edge ROU layers
//     ^ ((R & Vm) << N) ^ ((R >> N) & Vm)      vertical-edge ROU layers
//     ^ (R & b)                                Toffoli layer (colours b)
//   z = y ^ l                                  final CNOT layer
// H has bit v set when the edge (v, v+1) exists, Vm when (v, v+N) exists.
// The scatter is linear in the bits of i, so R = R_lo(x) ^ R_hi(T) for
// i = (T << S) | x; the circuit itself runs for every solution.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kTileThreads) void circuit_tile_kernel(
    FactorIn f, const int32_t *__restrict__ pivots, const uint64_t *__restrict__ rows, int N,
    uint64_t begin, uint64_t count, T *__restrict__ out, uint64_t tiles_per_block) {
    constexpr int V = Vec<T>::V;
    constexpr int S = tile_shift<T>();
    __shared__ uint64_t PM[65];  // PM[k] = OR of e_{p_j}, j < min(k, r)
    __shared__ uint64_t masks[3];
    __shared__ int grid_ok;
    int r;
    if (!gate(f, begin, count, r)) return;
    const int tid = threadIdx.x;
    const int n = f.n;
    if (tid < 64) {
        const int v = tid;
        const uint64_t row = (v < n) ? rows[v] : 0ull;
        const int gr = v / N, gc = v - (v / N) * N;
        uint64_t allowed = 0;
        if (v < n) {
            allowed |= 1ull << v;
            if (gc > 0) allowed |= 1ull << (v - 1);
            if (gc < N - 1) allowed |= 1ull << (v + 1);
            if (gr > 0) allowed |= 1ull << (v - N);
            if (gr < N - 1) allowed |= 1ull << (v + N);
        }
        const bool off_grid = (row & ~allowed) != 0;
        const uint64_t H = __ballot(v < n && gc < N - 1 && ((row >> (v + 1)) & 1ull));
        const uint64_t Vm = __ballot(v < n && gr < N - 1 && ((row >> (v + N)) & 1ull));
        const uint64_t bb = __ballot(v < n && ((row >> v) & 1ull));
        const bool any_off = __ballot(off_grid) != 0;
        if (tid == 0) {
            masks[0] = H;
            masks[1] = Vm;
            masks[2] = bb;
            grid_ok = any_off ? 0 : 1;
            uint64_t acc = 0;
            PM[0] = 0;
            for (int k = 0; k < 64; ++k) {
                if (k < r) acc |= 1ull << pivots[k];
                PM[k + 1] = acc;
            }
        }
    }
    __syncthreads();
    if (!grid_ok) {
        if (tid == 0) *f.status = HLF_EINVAL;
        return;
    }
    // The layers in the output width: n <= 32 bits fit one dword.
    using U = typename std::conditional<sizeof(T) <= 4, uint32_t, uint64_t>::type;
    const U H = (U)masks[0], Vm = (U)masks[1], bb = (U)masks[2];
    const U l = (U)f.shift[0];
    U Rlo[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const uint64_t x = (uint64_t)(tid * V + e);
        U R = 0;
        for (int j = 0; j < S; ++j)
            if ((x >> j) & 1ull) R ^= (U)(PM[j + 1] ^ PM[j]);
        Rlo[e] = R;
    }
    const uint64_t end = begin + count;
    const uint64_t ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    const uint64_t t0 = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * tiles_per_block;
    if (t0 >= ntiles) return;
    const uint64_t t1 = (t0 + tiles_per_block < ntiles) ? t0 + tiles_per_block : ntiles;
    uint64_t Tt = (begin >> S) + t0;
    U Rhi = 0;
    for (int j = 0; j + S < 64 && (Tt >> j); ++j)
        if ((Tt >> j) & 1ull) Rhi ^= (U)(PM[S + j + 1] ^ PM[S + j]);
    for (uint64_t t = t0; t < t1; ++t, ++Tt) {
        uint64_t zv[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
            const U R = Rlo[e] ^ Rhi;
            const U y = ((R & H) << 1) ^ ((R >> 1) & H) ^ ((R & Vm) << N) ^ ((R >> N) & Vm) ^ (R & bb);
            zv[e] = (uint64_t)(U)(y ^ l);
        }
        const uint64_t i0 = (Tt << S) + (uint64_t)(tid * V);
        if (i0 >= begin && i0 + V <= end) {
            uint32_t w[4];
            pack16<T>(zv, w);
            u32x4 val;
            val.x = w[0];
            val.y = w[1];
            val.z = w[2];
            val.w = w[3];
            __builtin_nontemporal_store(val, (u32x4 *)(out + (i0 - begin)));
        } else {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const uint64_t i = i0 + e;
                if (i >= begin && i < end) out[i - begin] = (T)zv[e];
            }
        }
        const int c = S + __builtin_ctzll(Tt + 1) + 1;
        Rhi ^= (U)(PM[c < 64 ? c : 64] ^ PM[S]);
    }
}

// ---------------------------------------------------------------------------
// Reduce, W <= 3: 4 waves per block, each on a contiguous range of tiles.
// ---------------------------------------------------------------------------
template <int WW>
__global__ __launch_bounds__(256) void reduce_wave_kernel(FactorIn f, uint64_t begin,
                                                          uint64_t count, uint64_t tiles_per_wave,
                                                          uint64_t *__restrict__ counts,
                                                          uint64_t *__restrict__ hash,
                                                          uint64_t *__restrict__ xorfold) {
    constexpr int S = WaveReduce<WW>::S;
    __shared__ uint64_t Bx[64 * WW];
    __shared__ unsigned long long part_cnt[64 * WW];
    __shared__ unsigned long long part_hash;
    __shared__ unsigned long long part_xf[WW];
    int r;
    if (!gate(f, begin, count, r)) return;
    const int tid = threadIdx.x;
    load_basis_padded<WW>(f.basis, r, Bx, tid, blockDim.x);
    for (int j = tid; j < 64 * WW; j += blockDim.x) part_cnt[j] = 0;
    if (tid == 0) part_hash = 0;
    if (tid < WW) part_xf[tid] = 0;
    uint64_t l[WW];
#pragma unroll
    for (int w = 0; w < WW; ++w) l[w] = f.shift[w];
    __syncthreads();

    const int lane = tid & 63;
    const uint64_t end = begin + count;
    const uint64_t first_tile = begin >> S;
    const uint64_t ntiles = ((end - 1) >> S) - first_tile + 1;
    const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (tid >> 6);
    const uint64_t t0 = gw * tiles_per_wave;
    if (t0 < ntiles) {
        const uint64_t t1 = (t0 + tiles_per_wave < ntiles) ? t0 + tiles_per_wave : ntiles;
        uint64_t c0 = (first_tile + t0) << S;
        uint64_t c1 = (first_tile + t1) << S;
        if (c0 < begin) c0 = begin;
        if (c1 > end) c1 = end;
        const WavePartial<WW> p = wave_reduce_range<WW>(Bx, l, f.n, r, c0, c1);
        if (lane == 0) {
            if (p.hash) atomicAdd(&part_hash, (unsigned long long)p.hash);
#pragma unroll
            for (int w = 0; w < WW; ++w)
                if (p.xf[w]) atomicXor(&part_xf[w], (unsigned long long)p.xf[w]);
        }
#pragma unroll
        for (int w = 0; w < WW; ++w)
            if (p.cnt[w]) atomicAdd(&part_cnt[64 * w + lane], (unsigned long long)p.cnt[w]);
    }
    __syncthreads();
    for (int j = tid; j < f.n; j += blockDim.x)
        if (part_cnt[j]) atomicAdd((unsigned long long *)&counts[j], part_cnt[j]);
    if (tid == 0 && part_hash) atomicAdd((unsigned long long *)hash, part_hash);
    if (xorfold && tid < WW && part_xf[tid])
        atomicXor((unsigned long long *)&xorfold[tid], part_xf[tid]);
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
    const int ndig = build_tables<WMAX>(f, r, W, false, g);
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
        // Lane b counts bit 64w + b over the wave's valid solutions: bit b of
        // z[w] across the lanes is lane b's word after the wave transpose.
        const uint64_t vm = __ballot(valid);
#pragma unroll
        for (int w = 0; w < WMAX; ++w)
            if (w < W) pc[w] += (uint64_t)__builtin_popcountll(wave_transpose64(z[w]) & vm);
    }
    const uint64_t wsum = wave_sum_u64(acc);
    if (lane == 0 && wsum) atomicAdd((unsigned long long *)hash, (unsigned long long)wsum);
#pragma unroll
    for (int w = 0; w < WMAX; ++w) {
        if (w < W) {
            const uint64_t wx = wave_xor_u64(xacc[w]);
            if (xorfold && lane == 0 && wx) atomicXor((unsigned long long *)&xorfold[w], (unsigned long long)wx);
            const int bit = 64 * w + lane;
            if (bit < n && pc[w]) atomicAdd(&part[bit], (unsigned long long)pc[w]);
        }
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

// Even split of ntiles over at most max_units units: tiles per unit.
uint64_t tiles_per_unit_for(uint64_t ntiles, uint64_t max_units, uint64_t *units) {
    uint64_t b = ntiles < max_units ? ntiles : max_units;
    if (b == 0) b = 1;
    const uint64_t tpu = (ntiles + b - 1) / b;
    *units = (ntiles + tpu - 1) / tpu;
    return tpu;
}

// Materialise launches: materialise_tiles_per_block tiles per workgroup.
uint64_t tiles_per_block_for(uint64_t ntiles, uint64_t tile_bytes, uint64_t *blocks) {
    const uint64_t tpb = materialise_tiles_per_block(ntiles, tile_bytes);
    *blocks = ntiles ? (ntiles + tpb - 1) / tpb : 1;
    return tpb;
}

template <typename T>
hlf_status launch_tile(const FactorIn &f, uint64_t begin, uint64_t count, T *out, int counter,
                       hipStream_t stream) {
    constexpr int S = tile_shift<T>();
    const uint64_t end = begin + count;  // host: may wrap only for invalid ranges
    uint64_t ntiles;
    if (end < begin) {
        ntiles = 1;  // invalid range: the device gate reports HLF_ERANGE
    } else {
        ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    }
    uint64_t blocks;
    const uint64_t tpb = tiles_per_block_for(ntiles, kTileBytes, &blocks);
    hipLaunchKernelGGL(enum_tile_kernel<T>, dim3((unsigned)blocks), dim3(kTileThreads), 0, stream,
                       f, begin, count, out, tpb, counter);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

// The multi-word kernel's workgroups build per-word tables before their first
// store, so they take ranges kWideRangeFactor times longer than the W = 1
// kernels (passed as a smaller nominal tile size).
constexpr uint64_t kWideRangeFactor = 2;

template <int WMAX>
hlf_status launch_wide_tile(const FactorIn &f, uint64_t begin, uint64_t count, uint64_t *out,
                            int counter, hipStream_t stream) {
    constexpr int S = kLogTileThreads;
    const uint64_t end = begin + count;
    const uint64_t ntiles = (end < begin) ? 1 : ((end - 1) >> S) - (begin >> S) + 1;
    uint64_t blocks;
    const uint64_t tpb = tiles_per_block_for(ntiles, (8ull * (uint64_t)f.words << S) / kWideRangeFactor, &blocks);
    hipLaunchKernelGGL(enum_wide_tile_kernel<WMAX>, dim3((unsigned)blocks), dim3(kTileThreads), 0,
                       stream, f, begin, count, out, tpb, counter);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int WMAX, typename T>
hlf_status launch_general(const FactorIn &f, uint64_t begin, uint64_t count, T *out, int counter,
                          hipStream_t stream) {
    const uint64_t per_block = 256 / WMAX;  // solutions per workgroup pass
    uint64_t blocks = (count + per_block - 1) / per_block;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL((enum_general_kernel<WMAX, T>), dim3((unsigned)blocks), dim3(256), 0,
                       stream, f, begin, count, out, counter);
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

template <int WW>
hlf_status launch_reduce_wave(const FactorIn &f, uint64_t begin, uint64_t count,
                              uint64_t *counts, uint64_t *hash, uint64_t *xorfold,
                              hipStream_t stream) {
    constexpr int S = WaveReduce<WW>::S;
    const uint64_t end = begin + count;
    const uint64_t ntiles = (end < begin) ? 1 : ((end - 1) >> S) - (begin >> S) + 1;
    uint64_t waves;
    const uint64_t tpw = tiles_per_unit_for(ntiles, (uint64_t)device_cu_count() * 32, &waves);
    const uint64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(reduce_wave_kernel<WW>, dim3((unsigned)blocks), dim3(256), 0, stream, f,
                       begin, count, tpw, counts, hash, xorfold);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

}  // namespace

hlf_status launch_enumerate(const FactorIn &f, uint64_t begin, uint64_t count, int word_bits,
                            bool counter_order, void *out, hipStream_t stream) {
    const int W = f.words;
    const int c = counter_order ? 1 : 0;
    const bool aligned16 = ((uintptr_t)out & 15u) == 0;
    if (W == 1 && word_bits <= 64) {
        if (word_bits == 16) {
            if (aligned16 && begin % Vec<uint16_t>::V == 0)
                return launch_tile<uint16_t>(f, begin, count, (uint16_t *)out, c, stream);
            return launch_general<1, uint16_t>(f, begin, count, (uint16_t *)out, c, stream);
        }
        if (word_bits == 32) {
            if (aligned16 && begin % Vec<uint32_t>::V == 0)
                return launch_tile<uint32_t>(f, begin, count, (uint32_t *)out, c, stream);
            return launch_general<1, uint32_t>(f, begin, count, (uint32_t *)out, c, stream);
        }
        if (aligned16 && begin % Vec<uint64_t>::V == 0)
            return launch_tile<uint64_t>(f, begin, count, (uint64_t *)out, c, stream);
        return launch_general<1, uint64_t>(f, begin, count, (uint64_t *)out, c, stream);
    }
    uint64_t *o = (uint64_t *)out;
    if (((uintptr_t)out & 7u) == 0) {
        if (W <= 2) return launch_wide_tile<2>(f, begin, count, o, c, stream);
        if (W <= 4) return launch_wide_tile<4>(f, begin, count, o, c, stream);
        if (W <= 8) return launch_wide_tile<8>(f, begin, count, o, c, stream);
        return launch_wide_tile<16>(f, begin, count, o, c, stream);
    }
    if (W <= 2) return launch_general<2, uint64_t>(f, begin, count, o, c, stream);
    if (W <= 4) return launch_general<4, uint64_t>(f, begin, count, o, c, stream);
    if (W <= 8) return launch_general<8, uint64_t>(f, begin, count, o, c, stream);
    return launch_general<16, uint64_t>(f, begin, count, o, c, stream);
}

// ---------------------------------------------------------------------------
// The paper's circuit for grids of more than 64 vertices (W > 1 words per
// vector; the same layers as circuit_tile_kernel).  First one workgroup checks
// that A is a subgraph of the N x N grid (every row's bits lie on the vertex
// itself and its grid neighbours) and writes HLF_EINVAL otherwise, so the
// materialising launch behind it on the stream writes nothing.  The
// materialising kernel takes one lane per word, as enum_wide_tile_kernel:
// thread (slot, w) holds word w of solutions base + slot + u*P, u < WMAX,
// P = 1024 / WMAX.  R, the counter bits scattered onto the pivots, is linear
// in the index: R = Rlo(slot + u*P) ^ Rhi(T) for a tile T of 1024 indices.
// The edge layers shift R by 1 and by N bits across words; a lane takes the
// neighbouring words of its solution from lanes w - 1 and w + 1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void circuit_check_kernel(int32_t *status, const uint64_t *__restrict__ rows,
                                                             int n, int W, int N) {
    if (*(volatile int32_t *)status != HLF_OK) return;
    int bad = 0;
    for (int v = threadIdx.x; v < n; v += blockDim.x) {
        const int gr = v / N, gc = v - (v / N) * N;
        for (int w = 0; w < W; ++w) {
            uint64_t allowed = 0;
            auto allow = [&](int u) {
                if ((u >> 6) == w) allowed |= 1ull << (u & 63);
            };
            allow(v);
            if (gc > 0) allow(v - 1);
            if (gc < N - 1) allow(v + 1);
            if (gr > 0) allow(v - N);
            if (gr < N - 1) allow(v + N);
            if (rows[(size_t)v * W + w] & ~allowed) bad = 1;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) *status = HLF_EINVAL;
}

namespace {

// x of lane - 1 / lane + 1 within the lane's 16-lane row (0 at the row edge).
__device__ __forceinline__ uint64_t dpp_row_shr1(uint64_t x) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, 0x111, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), 0x111, 0xf, 0xf, true);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
__device__ __forceinline__ uint64_t dpp_row_shl1(uint64_t x) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, 0x101, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), 0x101, 0xf, 0xf, true);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

template <int WMAX>
__global__ __launch_bounds__(kTileThreads) void circuit_wide_kernel(
    FactorIn f, const int32_t *__restrict__ pivots, const uint64_t *__restrict__ rows, int N,
    uint64_t begin, uint64_t count, uint64_t *__restrict__ out, uint64_t tiles_per_block) {
    constexpr int P = kTileThreads / WMAX;
    constexpr int U = WMAX;
    constexpr int S = kLogTileThreads;
    constexpr int LOGP = S - (WMAX == 2 ? 1 : WMAX == 4 ? 2 : WMAX == 8 ? 3 : 4);
    __shared__ uint64_t E[64 * WMAX];     // E[k][w] = word w of e_{p_k}, k < r
    __shared__ uint64_t M[3 * WMAX];      // H, V (edge masks), b (colours)
    int r;
    if (!gate(f, begin, count, r)) return;
    const int n = f.n, W = f.words;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < 64 * WMAX; idx += blockDim.x) {
        const int k = idx / WMAX, w = idx - k * WMAX;
        uint64_t e = 0;
        if (k < r) {
            const int p = pivots[k];
            if ((p >> 6) == w) e = 1ull << (p & 63);
        }
        E[idx] = e;
    }
    // masks from three words per row: A[v][v+1], A[v][v+N], A[v][v]
    {
        const int v = tid;  // n <= 1024 = blockDim.x
        bool h = false, vv = false, bb = false;
        if (v < n) {
            const int gr = v / N, gc = v - (v / N) * N;
            const uint64_t *row = rows + (size_t)v * W;
            if (gc < N - 1) h = (row[(v + 1) >> 6] >> ((v + 1) & 63)) & 1ull;
            if (gr < N - 1) vv = (row[(v + N) >> 6] >> ((v + N) & 63)) & 1ull;
            bb = (row[v >> 6] >> (v & 63)) & 1ull;
        }
        const uint64_t H = __ballot(h), V = __ballot(vv), B = __ballot(bb);
        const int wave = tid >> 6;
        if ((tid & 63) == 0 && wave < WMAX) {
            M[wave] = H;
            M[WMAX + wave] = V;
            M[2 * WMAX + wave] = B;
        }
    }
    __syncthreads();
    const uint64_t end = begin + count;
    const uint64_t ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    const uint64_t t0 = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * tiles_per_block;
    if (t0 >= ntiles) return;
    const uint64_t t1 = (t0 + tiles_per_block < ntiles) ? t0 + tiles_per_block : ntiles;
    const int w = tid & (WMAX - 1);
    const int slot = tid / WMAX;
    const bool act = w < W;
    const uint64_t Hw = M[w], Vw = M[WMAX + w], Bw = M[2 * WMAX + w];
    const uint64_t Hm = w ? M[w - 1] : 0ull, Vm = w ? M[WMAX + w - 1] : 0ull;
    const uint64_t lw = act ? f.shift[w] : 0ull;
    // Rlo[u] = scatter of slot + u*P; bit j of slot is e_{p_j}, u*P adds LOGP + bits of u
    uint64_t Rlo[U];
    {
        uint64_t x = 0;
        for (int j = 0; j < LOGP; ++j)
            if ((slot >> j) & 1) x ^= E[j * WMAX + w];
        Rlo[0] = x;
    }
#pragma unroll
    for (int u = 1; u < U; ++u) Rlo[u] = Rlo[u & (u - 1)] ^ E[(LOGP + __builtin_ctz(u)) * WMAX + w];
    uint64_t Tt = (begin >> S) + t0;
    uint64_t Rhi = 0;
    for (int j = 0; j + S < 64 && (Tt >> j); ++j)
        if ((Tt >> j) & 1ull) Rhi ^= E[(S + j) * WMAX + w];
    const int Nr = 64 - N;
    for (uint64_t t = t0; t < t1; ++t, ++Tt) {
        const uint64_t base = Tt << S;
        const bool full = base >= begin && base + (1u << S) <= end;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t R = Rlo[u] ^ Rhi;
            // neighbouring words of the same solution (0 beyond the vector):
            // DPP row shifts by one lane (a solution's WMAX lanes lie in one
            // 16-lane row)
            uint64_t Rd = dpp_row_shr1(R);
            uint64_t Ru = dpp_row_shl1(R);
            if (w == 0) Rd = 0;
            if (w == WMAX - 1) Ru = 0;
            const uint64_t X1 = R & Hw, X1d = Rd & Hm, X2 = R & Vw, X2d = Rd & Vm;
            const uint64_t y = ((X1 << 1) | (X1d >> 63)) ^ (((R >> 1) | (Ru << 63)) & Hw) ^
                               ((X2 << N) | (X2d >> Nr)) ^ (((R >> N) | (Ru << Nr)) & Vw) ^ (R & Bw);
            const uint64_t z = y ^ lw;
            const uint64_t i = base + (uint64_t)slot + (uint64_t)u * P;
            if (act) {
                if (full)
                    __builtin_nontemporal_store(z, out + (i - begin) * W + w);
                else if (i >= begin && i < end)
                    out[(i - begin) * W + w] = z;
            }
        }
        // next tile: the counter's carry flips bits S .. S + ctz(T + 1)
        const int c = __builtin_ctzll(Tt + 1);
        for (int j = 0; j <= c && S + j < 64; ++j) Rhi ^= E[(S + j) * WMAX + w];
    }
}

}  // namespace

hlf_status launch_circuit(const FactorIn &f, const int32_t *pivots, const uint64_t *rows, int N,
                          uint64_t begin, uint64_t count, int word_bits, void *out,
                          hipStream_t stream) {
    const uint64_t end = begin + count;
    auto go = [&](auto tag) -> hlf_status {
        using T = decltype(tag);
        constexpr int S = tile_shift<T>();
        const uint64_t ntiles = (end < begin) ? 1 : ((end - 1) >> S) - (begin >> S) + 1;
        uint64_t blocks;
        const uint64_t tpb = tiles_per_block_for(ntiles, kTileBytes, &blocks);
        hipLaunchKernelGGL(circuit_tile_kernel<T>, dim3((unsigned)blocks), dim3(kTileThreads), 0,
                           stream, f, pivots, rows, N, begin, count, (T *)out, tpb);
        return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
    };
    if (word_bits == 16) return go(uint16_t{});
    if (word_bits == 32) return go(uint32_t{});
    if (word_bits == 64 && f.words == 1) return go(uint64_t{});
    // W > 1 words per solution
    const int W = f.words;
    hipLaunchKernelGGL(circuit_check_kernel, dim3(1), dim3(1024), 0, stream, f.status, rows, f.n, W, N);
    if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    auto wide = [&](auto wm) -> hlf_status {
        constexpr int WMAX = decltype(wm)::value;
        constexpr int S = kLogTileThreads;
        const uint64_t ntiles = (end < begin) ? 1 : ((end - 1) >> S) - (begin >> S) + 1;
        uint64_t blocks;
        const uint64_t tpb = tiles_per_block_for(ntiles, (8ull * (uint64_t)W << S) / kWideRangeFactor, &blocks);
        hipLaunchKernelGGL(circuit_wide_kernel<WMAX>, dim3((unsigned)blocks), dim3(kTileThreads), 0, stream,
                           f, pivots, rows, N, begin, count, (uint64_t *)out, tpb);
        return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
    };
    if (W <= 2) return wide(std::integral_constant<int, 2>{});
    if (W <= 4) return wide(std::integral_constant<int, 4>{});
    if (W <= 8) return wide(std::integral_constant<int, 8>{});
    return wide(std::integral_constant<int, 16>{});
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
    if (W == 1) return launch_reduce_wave<1>(f, begin, count, counts, hash, xorfold, stream);
    if (W == 2) return launch_reduce_wave<2>(f, begin, count, counts, hash, xorfold, stream);
    if (W == 3) return launch_reduce_wave<3>(f, begin, count, counts, hash, xorfold, stream);
    if (W <= 4) return launch_reduce_general<4>(f, begin, count, counts, hash, xorfold, stream);
    if (W <= 8) return launch_reduce_general<8>(f, begin, count, counts, hash, xorfold, stream);
    return launch_reduce_general<16>(f, begin, count, counts, hash, xorfold, stream);
}

}  // namespace hlf
