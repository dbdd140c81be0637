// Stage 1 of the two-stage scheme (the paper's CLA module, Section 2,
// tasks (1)-(4)) on gfx950:
//   * pack_dense_kernel (n <= 64), pack_rows_kernel + pack_check_kernel
//     (n > 64): dense 0/1 matrix -> packed uint64 rows, with the symmetry /
//     0-1 validation of the problem statement (Section 1);
//   * factor_wave_kernel: one wavefront per instance (used for n <= 64; the
//     batch path runs the same elimination for n <= 192); every lane keeps
//     its rows in VGPRs, pivots are found with a ballot and the pivot row is
//     broadcast with readlane -- no barriers in the elimination;
//   * factor_workgroup_kernel: one workgroup per instance for n <= 1024, one
//     row per thread in VGPRs, Gauss-Jordan in blocks of 8 columns: the
//     pivot search runs on bit-planes of the rows' 8-bit slices in one wave,
//     then every row applies its block update with two lookups per word in
//     tables of XOR combinations of the block's pivot rows (LDS).
// Both variants produce the canonical record defined in hlf.h (the RREF is
// unique, so the pivot rows chosen do not matter).
#include "factor_wave.h"
#include "hlf_device.h"
#include "hlf_internal.h"

#include <climits>

namespace hlf {
namespace {

// ---------------------------------------------------------------------------
// A0: pack + validate for n <= 64 (larger n: the two launches above).  One
// workgroup of 64*W threads packs A into bit rows in LDS, then checks A = A^T:
// for column c, the ballot of bit c over the 64 rows held by wave v is word v
// of column c, which must equal word v of row c.
//
// Packing: when n is a multiple of 16 and A is 16-byte aligned, each thread
// loads 16 bytes (columns 16q..16q+15 of one row) per request, kPackU rows in
// flight, and gathers them into 16 bits.  For a 32-bit word x holding four
// 0/1 bytes b0..b3, (x * 0x10204080) >> 28 = b0 | b1<<1 | b2<<2 | b3<<3: the
// partial product of b_k with 2^(28-7k) lands on bit 28+k, and every other
// partial product lands on a distinct bit below 28 or above 31, so there are
// no carries into bits 28..31.  Any other n falls back to byte loads (lane l
// loads column 64w+l of G rows, one ballot per row).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t gather4(uint32_t x) { return (x * 0x10204080u) >> 28; }

// Symmetry of one pair of 64x64 tiles: lane l holds x = word J of row 64I+l
// and y = word I of row 64J+l.  Column b of tile (I, J), which lane b of the
// transposed tile holds, must equal y in lane b (row 64J+b restricted to
// columns 64I..64I+63).  Returns true, wave-uniform, if some
// A[64I+l][64J+b] != A[64J+b][64I+l].  Needs all lanes active.
__device__ __forceinline__ bool tile_pair_asym(uint64_t x, uint64_t y) {
    return __ballot(wave_transpose64(x) != y) != 0;
}

// A0 for n > 64: two launches.  pack_rows_kernel packs 16 rows per
// workgroup (16-byte loads and gather4 when n is a multiple of 16 and A is
// 16-byte aligned, else byte loads and one ballot per row word) and checks
// that every byte is 0 or 1.  gather4 is only meaningful on 0/1 bytes, so a
// row holding another value may pack to arbitrary bits; the workgroup then
// marks it so that the check below must fail whatever those bits are.  When
// n is not a multiple of 64 the row gets pad bit 63 of its last word.  When
// it is, every block is 16 full rows, and the asymmetry goes inside one of
// the workgroup's own row pairs (i, i^1): if one row of the pair is bad, its
// entry towards the other becomes the complement of the other's entry back,
// if both are, the two entries become 1 and 0.  pack_check_kernel checks the
// pad bits and A = A^T on the packed rows, tile pair by tile pair, and is the
// only writer of the status.
constexpr int kPackRowsPerBlock = 16;
constexpr int kPackRowsThreads = 256;

__global__ __launch_bounds__(kPackRowsThreads) void pack_rows_kernel(const uint8_t *__restrict__ A,
                                                                     int n, int W, int vec16,
                                                                     uint64_t *__restrict__ rows) {
    __shared__ uint64_t lds[kPackRowsPerBlock * HLF_MAX_WORDS];
    __shared__ int badrow[kPackRowsPerBlock];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x * kPackRowsPerBlock;
    const int cpr = n >> 4;  // 16-byte chunks per row
    if (tid < kPackRowsPerBlock) badrow[tid] = 0;
    for (int idx = tid; idx < kPackRowsPerBlock * W; idx += kPackRowsThreads) lds[idx] = 0;
    __syncthreads();
    if (!vec16) {
        // (row, word) items per wave: lane l loads byte 64w + l of the row, a
        // ballot gives the packed word; eight items' loads go out together.
        const int lane = tid & 63, wave = tid >> 6;
        constexpr int kWaves = kPackRowsThreads / 64, kBatch = 8;
        const int items = kPackRowsPerBlock * W;
        for (int it0 = wave * kBatch; it0 < items; it0 += kWaves * kBatch) {
            uint32_t byte[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int it = it0 + u, lr = it / W, w = it - lr * W;
                const int i = i0 + lr, c = 64 * w + lane;
                byte[u] = (it < items && i < n && c < n) ? (uint32_t)A[(size_t)i * n + c] : 0u;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int it = it0 + u, lr = it / W;
                const uint64_t word = __ballot(byte[u] & 1u);
                const bool badb = __ballot(byte[u] > 1u) != 0;
                if (lane == 0 && it < items) {
                    lds[it] = word;  // it = lr * W + w
                    if (badb) badrow[lr] = 1;
                }
            }
        }
    } else {
    uint16_t *l16 = reinterpret_cast<uint16_t *>(lds);
    const u32x4 *A16 = reinterpret_cast<const u32x4 *>(A);
    // at most 16 rows x 64 chunks = 4 chunks per thread, all loads first
    constexpr int kPer = kPackRowsPerBlock * (HLF_MAX_N / 16) / kPackRowsThreads;
    u32x4 v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int idx = tid + k * kPackRowsThreads;
        const int lr = idx / cpr, c = idx - lr * cpr;
        const bool ok = lr < kPackRowsPerBlock && i0 + lr < n;
        v[k] = ok ? __builtin_nontemporal_load(&A16[(size_t)(i0 + lr) * cpr + c]) : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int idx = tid + k * kPackRowsThreads;
        const int lr = idx / cpr, c = idx - lr * cpr;
        if (lr < kPackRowsPerBlock && i0 + lr < n) {
            if (((v[k].x | v[k].y | v[k].z | v[k].w) & 0xFEFEFEFEu) != 0u) badrow[lr] = 1;
            l16[lr * 4 * W + c] = (uint16_t)(gather4(v[k].x) | (gather4(v[k].y) << 4) |
                                             (gather4(v[k].z) << 8) | (gather4(v[k].w) << 12));
        }
    }
    }
    __syncthreads();
    if ((n & 63) != 0) {  // pad bit 63 of the last word of a bad row
        if (tid < kPackRowsPerBlock && i0 + tid < n && badrow[tid]) lds[tid * W + W - 1] |= 1ull << 63;
    } else if (tid < kPackRowsPerBlock / 2) {  // row pair (a, a + 1): full blocks
        const int a = 2 * tid, b = a + 1, ia = i0 + a, ib = i0 + b;
        if (ib < n && (badrow[a] || badrow[b])) {
            uint64_t &ab = lds[a * W + (ib >> 6)];  // holds entry (ia, ib)
            uint64_t &ba = lds[b * W + (ia >> 6)];  // holds entry (ib, ia)
            const uint64_t mab = 1ull << (ib & 63), mba = 1ull << (ia & 63);
            if (badrow[a] && badrow[b]) {
                ab |= mab;
                ba &= ~mba;
            } else if (badrow[a]) {
                ab = (ba & mba) ? (ab & ~mab) : (ab | mab);
            } else {
                ba = (ab & mab) ? (ba & ~mba) : (ba | mba);
            }
        }
    }
    __syncthreads();
    for (int idx = tid; idx < kPackRowsPerBlock * W; idx += kPackRowsThreads) {
        const int lr = idx / W, w = idx - lr * W;
        const int i = i0 + lr;
        if (i < n) rows[(size_t)i * W + w] = lds[lr * W + w];
    }
}

__global__ __launch_bounds__(1024) void pack_check_kernel(const uint64_t *__restrict__ rows, int n,
                                                          int W, int32_t *__restrict__ status) {
    __shared__ int bad;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    if (tid == 0) bad = 0;
    __syncthreads();
    const uint64_t lm = last_word_mask(n);
    for (int i = tid; i < n; i += blockDim.x)
        if (rows[(size_t)i * W + W - 1] & ~lm) bad = 1;
    for (int t = wave; t < W * W; t += nwaves) {  // wave-uniform
        const int I = t / W, J = t - I * W;
        if (J < I) continue;
        const int ri = 64 * I + lane, rj = 64 * J + lane;
        const uint64_t x = ri < n ? rows[(size_t)ri * W + J] : 0ull;
        const uint64_t y = rj < n ? rows[(size_t)rj * W + I] : 0ull;
        if (tile_pair_asym(x, y) && lane == 0) bad = 1;
    }
    __syncthreads();
    if (tid == 0) *status = bad ? HLF_ENOTSYM : HLF_OK;
}

template <int WMAX>
__global__ __launch_bounds__(64 * WMAX) void pack_dense_kernel(const uint8_t *__restrict__ A, int n,
                                                               int W, uint64_t *__restrict__ rows,
                                                               int32_t *__restrict__ status) {
    __shared__ uint64_t lds[64 * WMAX * WMAX];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int nthr = blockDim.x;
    const int nwaves = nthr >> 6;
    int mybad = 0;

    if ((n & 15) == 0 && ((uintptr_t)A & 15u) == 0) {
        // Pieces of 16 bits; pieces past column n-1 of the last word stay 0.
        for (int idx = tid; idx < n * W; idx += nthr) lds[idx] = 0;
        if (tid == 0) bad = 0;
        __syncthreads();
        uint16_t *l16 = reinterpret_cast<uint16_t *>(lds);
        const int cpr = n >> 4;             // 16-byte chunks per row, <= 4W
        const int rpp = nthr / cpr;         // rows per pass, >= 16
        const int ri = tid / cpr, q = tid - ri * cpr;
        const u32x4 *A16 = reinterpret_cast<const u32x4 *>(A);
        constexpr int kPackU = 16;
        if (ri < rpp) {
            for (int i0 = ri; i0 < n; i0 += kPackU * rpp) {
                u32x4 v[kPackU];
#pragma unroll
                for (int u = 0; u < kPackU; ++u) {
                    const int i = i0 + u * rpp;
                    v[u] = (i < n) ? __builtin_nontemporal_load(&A16[(size_t)i * cpr + q])
                                   : u32x4{0u, 0u, 0u, 0u};
                }
#pragma unroll
                for (int u = 0; u < kPackU; ++u) {
                    const int i = i0 + u * rpp;
                    if (i < n) {
                        mybad |= ((v[u].x | v[u].y | v[u].z | v[u].w) & 0xFEFEFEFEu) != 0u;
                        const uint32_t m = gather4(v[u].x) | (gather4(v[u].y) << 4) |
                                           (gather4(v[u].z) << 8) | (gather4(v[u].w) << 12);
                        l16[i * 4 * W + q] = (uint16_t)m;
                    }
                }
            }
        }
    } else {
        if (tid == 0) bad = 0;
        __syncthreads();
        // Wave v packs row groups v, v + nwaves, ... of G rows: lane l loads
        // byte 64*w + l of the G rows at once (independent loads), then one
        // ballot per row gives the packed word.
        constexpr int G = 16;
        for (int i0 = wave * G; i0 < n; i0 += nwaves * G) {
            for (int w = 0; w < W; ++w) {
                const int j = 64 * w + lane;
                uint32_t v[G];
#pragma unroll
                for (int k = 0; k < G; ++k)
                    v[k] = (j < n && i0 + k < n) ? (uint32_t)A[(size_t)(i0 + k) * n + j] : 0u;
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    if (i0 + k >= n) break;
                    mybad |= (v[k] > 1u);
                    const uint64_t word = __ballot(v[k] == 1u);
                    if (lane == 0) lds[(i0 + k) * W + w] = word;
                }
            }
        }
    }
    __syncthreads();

    // Symmetry: tile pairs (I, J), I <= J < W, spread over the waves.
    {
        int pidx = 0;
        for (int I = 0; I < W; ++I)
            for (int J = I; J < W; ++J, ++pidx) {
                if (pidx % nwaves != wave) continue;
                const int ri = 64 * I + lane, rj = 64 * J + lane;
                const uint64_t x = (ri < n) ? lds[ri * W + J] : 0ull;
                const uint64_t y = (rj < n) ? lds[rj * W + I] : 0ull;
                if (tile_pair_asym(x, y)) mybad = 1;
            }
    }
    if (mybad) bad = 1;
    __syncthreads();
    for (int idx = tid; idx < n * W; idx += nthr) rows[idx] = lds[idx];
    if (tid == 0) *status = bad ? HLF_ENOTSYM : HLF_OK;
}

// keep_bad: out.status already holds the pack verdict for these rows; a
// verdict other than HLF_OK stays and nothing else is written.
template <int WMAX>
__global__ __launch_bounds__(64) void factor_wave_kernel(const uint64_t *__restrict__ rows, int n,
                                                         int W, FactorOut out, int keep_bad) {
    if (keep_bad && *(volatile int32_t *)out.status != HLF_OK) return;
    __shared__ WaveSmem<WMAX> sm;
    wave_load_rows<WMAX>(rows, n, W, sm);
    factor_wave_core<WMAX>(n, W, false, out, sm);
}

// ---------------------------------------------------------------------------
// A1-A4, workgroup variant: n <= 64*WMAX <= 1024, 64*W threads, thread i
// holds row i.  The LDS matrix `mat` (n rows of W words) first holds A for
// the symmetry check, then the RREF rows (0..r-1) and the kernel vectors
// (r..n-1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lower_bound_int(const int *a, int len, int key) {
    int lo = 0, hi = len;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int WMAX>
__global__ __launch_bounds__(1024) void factor_workgroup_kernel(const uint64_t *__restrict__ rows,
                                                                int n, int W, FactorOut out,
                                                                int keep_bad) {
    if (keep_bad && *(volatile int32_t *)out.status != HLF_OK) return;
    constexpr int NP = 64 * WMAX;
    constexpr int kMatWords = 64 * WMAX * WMAX > 256 * WMAX ? 64 * WMAX * WMAX : 256 * WMAX;
    __shared__ uint64_t mat[kMatWords];
    __shared__ uint64_t prow[8 * WMAX];
    __shared__ int piv[64 * WMAX];
    __shared__ int freec[64 * WMAX];
    __shared__ int qacc[64 * WMAX];
    __shared__ __align__(16) uint8_t sl8[1024];
    __shared__ uint16_t pivmark[64 * WMAX];  // block * 8 + j for the block's j-th pivot row
    __shared__ uint32_t ttab[32];            // tag of a slice: ttab[low nibble] ^ ttab[16 + high]
    __shared__ __align__(16) uint32_t blkstate[16];
    __shared__ int blk[2];
    __shared__ uint32_t wmask;
    __shared__ unsigned long long shiftw[WMAX];
    __shared__ int flag_bad, flag_internal;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nthr = blockDim.x;

    // `mat` holds, in turn: A word-major (word w of row i at w*NP + i) for the
    // symmetry check; the block tables of the elimination; the RREF rows and
    // the kernel vectors, row-major.
    uint64_t row[WMAX];
#pragma unroll
    for (int w = 0; w < WMAX; ++w) {
        row[w] = (tid < n && w < W) ? rows[tid * W + w] : 0ull;
        mat[w * NP + tid] = row[w];
    }
    if (tid < WMAX) shiftw[tid] = 0;
    pivmark[tid] = 0xFFFFu;
    if (tid == 0) {
        flag_bad = 0;
        flag_internal = 0;
    }
    __syncthreads();

    bool bad = false;
    const uint64_t lm = last_word_mask(n);
#pragma unroll
    for (int w = 0; w < WMAX; ++w)
        if (w == W - 1 && (row[w] & ~lm)) bad = true;
    // Symmetry: tile pairs (I, J), I <= J < W, spread over the waves.
    {
        const int nwaves = nthr >> 6;
        int pidx = 0;
        for (int I = 0; I < W; ++I)
            for (int J = I; J < W; ++J, ++pidx) {
                if (pidx % nwaves != wave) continue;
                if (tile_pair_asym(mat[J * NP + 64 * I + lane], mat[I * NP + 64 * J + lane]))
                    bad = true;
            }
    }
    if (bad) flag_bad = 1;
    __syncthreads();
    if (flag_bad) {
        if (tid == 0) {
            *out.status = HLF_ENOTSYM;
            *out.rank = 0;
        }
        return;
    }

    // Gauss-Jordan in blocks of 8 columns (the blocking of Arlazarov,
    // Dinic, Kronrod and Faradzev, the "Four Russians").  Within a block only
    // the 8-bit slice s of every row takes part in the elimination: the
    // pivot of column c is the lowest-index row that is not yet a pivot and
    // has bit c of its current slice set, and every row keeps a tag tau (bit
    // j set: the block's j-th pivot row, as it stood when the block began,
    // has been added to it).  One column step maps the state (slice, tag) of
    // every row other than that column's pivot by a linear map over GF(2)
    // (add the pivot's state, plus bit j to the tag, if bit c is set), so
    // the state of such a row is a linear function of its starting slice:
    // the XOR of the states reached from the 8 unit slices.  Wave 0 holds the
    // current slices of all rows as 8 bit-planes, 16 rows per lane, so the
    // candidates of column c are one plane ANDed with the not-yet-pivot mask
    // and the pivot is its lowest set bit (a ballot and a readlane); the rows
    // with bit c then take the pivot's current slice, one XOR per later
    // plane.  For the tags, lanes 0-7 track the states of the 8 unit slices
    // and lanes 8-15 the pivots' own states; a pivot's state is the XOR of
    // the unit states over its starting slice (a DPP reduction).  The block
    // ends with every row's tag; the current value of every row is then its
    // start-of-block value plus the XOR of the pivot rows in its tag, so two
    // lookups per word in 16-entry tables (one per half of the tag) update
    // every row, pivot rows included.
    int r = 0, nfree = 0;
    bool used = false;
    int myk = -1;
    uint32_t unused16 = 0;  // wave 0: bit b of lane l <=> row 16l+b is not a pivot
    if (wave == 0)
        for (int b = 0; b < 16; ++b)
            if (16 * lane + b < n) unused16 |= 1u << b;
    uint64_t cur = row[0];  // word c0 / 64 of this row, kept current
    for (int c0 = 0; c0 < n; c0 += 8) {
        const int kb = (n - c0) < 8 ? (n - c0) : 8;
        const int cw = c0 >> 6;
        const int blkno = c0 >> 3;
        if (cw && (c0 & 63) == 0) {
#pragma unroll
            for (int w = 0; w < WMAX; ++w)
                if (w == cw) cur = row[w];
        }
        const uint32_t sl = (uint32_t)(cur >> (c0 & 63)) & 0xFFu;
        sl8[tid] = (uint8_t)sl;
        __syncthreads();

        if (wave == 0) {
            // cp[u]: bit b of lane l <=> bit u of the current slice of row
            // 16l+b: the 16 slices of the lane, as two 8x8 bit matrices (byte
            // = row, bit = column), transposed with three delta swaps.  Lanes
            // past the last row hold stale bytes; their rows are never
            // candidates (unused16 is 0 there).
            const u32x4 sq = *reinterpret_cast<const u32x4 *>(&sl8[16 * lane]);
            auto transpose8 = [](uint64_t x) {
                uint64_t t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
                x ^= t ^ (t << 7);
                t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
                x ^= t ^ (t << 14);
                t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
                x ^= t ^ (t << 28);
                return x;
            };
            const uint64_t p0 = transpose8(((uint64_t)sq.y << 32) | sq.x);
            const uint64_t p1 = transpose8(((uint64_t)sq.w << 32) | sq.z);
            uint32_t cp[8];
#pragma unroll
            for (int k = 0; k < 8; ++k)
                cp[k] = (uint32_t)((p0 >> (8 * k)) & 0xFFu) | ((uint32_t)((p1 >> (8 * k)) & 0xFFu) << 8);
            // Lane k < 8: state of unit slice e_k (slice | tag << 8); lane 8+j:
            // state of pivot j after its own step.
            uint32_t st = (lane < 8) ? (1u << lane) : 0u;
            int m = 0;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (t >= kb) break;
                const uint32_t cm = cp[t] & unused16;
                const uint64_t bm = __ballot(cm != 0u);
                if (bm == 0) {
                    if (lane == 0) freec[nfree] = c0 + t;
                    ++nfree;
                    continue;
                }
                const int L = __builtin_ctzll(bm);
                const int b = __builtin_ctz((uint32_t)__builtin_amdgcn_readlane((int)cm, L));
                const uint32_t rbit = (lane == L) ? (1u << b) : 0u;
                // Rows with bit t set, the pivot excluded, add the pivot's
                // current slice; its bit t+1 is read directly so the next
                // column's candidates do not wait for the unit states.
                const uint32_t cpx = cp[t] & ~rbit;
                unused16 &= ~rbit;
                if (t + 1 < 8) {
                    const uint32_t c1 =
                        ((uint32_t)__builtin_amdgcn_readlane((int)cp[t + 1 < 8 ? t + 1 : 7], L) >> b) & 1u;
                    if (c1) cp[t + 1 < 8 ? t + 1 : 7] ^= cpx;
                }
                const int q = b >> 2;
                const uint32_t sw = q == 0 ? sq.x : q == 1 ? sq.y : q == 2 ? sq.z : sq.w;
                const uint32_t sp =
                    ((uint32_t)__builtin_amdgcn_readlane((int)sw, L) >> (8 * (b & 3))) & 0xFFu;
                const uint32_t xr =
                    xor_lanes0to7((lane < 8 && ((sp >> lane) & 1u)) ? st : 0u);
#pragma unroll
                for (int u = t + 2; u < 8; ++u)
                    if ((xr >> u) & 1u) cp[u] ^= cpx;
                const uint32_t upd = xr ^ (1u << (8 + m));
                if (lane < 8 + m && ((st >> t) & 1u)) st ^= upd;
                if (lane == 8 + m) st = xr;
                if (lane == 0) {
                    piv[r + m] = c0 + t;
                    pivmark[16 * L + b] = (uint16_t)(8 * blkno + m);
                }
                ++m;
            }
            // Tag of a row = XOR of the unit tags over its starting slice,
            // as two 16-entry tables (low and high nibble): lane l < 32 fills
            // entry l & 15 of table l >> 4.
            uint32_t us[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) us[k] = ((uint32_t)__builtin_amdgcn_readlane((int)st, k) >> 8) & 0xFFu;
            if (lane < 32) {
                const int hi = lane >> 4, e = lane & 15;
                uint32_t v = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if ((e >> k) & 1) v ^= hi ? us[4 + k] : us[k];
                ttab[lane] = v;
            }
            if (lane >= 8 && lane < 16) blkstate[lane] = (st >> 8) & 0xFFu;
            if (lane == 0) {
                blk[0] = m;
                blk[1] = nfree;
            }
        }
        __syncthreads();
        const int m = blk[0];
        nfree = blk[1];
        uint32_t tau = 0;
        if (m > 0 && tid < n) {
            tau = ttab[sl & 15u] ^ ttab[16 + (sl >> 4)];
            const uint32_t mk = pivmark[tid];
            if ((int)(mk >> 3) == blkno) {
                const int j = (int)(mk & 7u);
                used = true;
                myk = r + j;
                tau = blkstate[8 + j];
#pragma unroll
                for (int w = 0; w < WMAX; ++w) prow[j * WMAX + w] = row[w];
            }
        }
        if (tid == 0) wmask = 0;
        r += m;
        if (m == 0) continue;
        __syncthreads();
        // Two tables per word w of the block's pivot rows (as they stood when
        // the block began): L[e] = XOR of pivot rows j < 4 with bit j of e
        // set at mat[w*32 + e], H[e] the same for pivot rows 4 + j at
        // mat[w*32 + 16 + e]; word w of a row's update is L[tau & 15] ^
        // H[tau >> 4].  Thread (w, e) = (tid / 32, tid % 32) fills one entry.
        // Words that are zero in every pivot row (all words left of the
        // block's word, since a row that is not yet a pivot is zero in every
        // column already eliminated or found free) are skipped in the lookup;
        // wmask records the others, one ballot per wave for its two words.
        {
            const int w = tid >> 5, e = tid & 31;
            const int half = e >> 4, idx = e & 15;
            uint64_t v = 0;
            if (w < W) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (4 * half + k < m && ((idx >> k) & 1)) v ^= prow[(4 * half + k) * WMAX + w];
                mat[w * 32 + e] = v;
            }
            const uint64_t nzb = __ballot(v != 0ull);
            if (lane == 0 && nzb)
                atomicOr(&wmask, ((uint32_t)nzb ? 1u << (2 * wave) : 0u) |
                                     ((uint32_t)(nzb >> 32) ? 1u << (2 * wave + 1) : 0u));
        }
        __syncthreads();
        const uint32_t wm = (uint32_t)__builtin_amdgcn_readfirstlane((int)wmask);
        if (tau) {
            const uint32_t tl = tau & 15u, th = 16u + (tau >> 4);
            uint64_t tv[WMAX];
#pragma unroll
            for (int w = 0; w < WMAX; ++w)
                tv[w] = ((wm >> w) & 1u) ? (mat[w * 32 + tl] ^ mat[w * 32 + th]) : 0ull;
#pragma unroll
            for (int w = 0; w < WMAX; ++w) row[w] ^= tv[w];
            if ((wm >> cw) & 1u) cur ^= mat[cw * 32 + tl] ^ mat[cw * 32 + th];
        }
        // The next block's first write to sl8, the block state or the table
        // comes after at least one more barrier.
    }
    __syncthreads();
    if (used)
#pragma unroll
        for (int w = 0; w < WMAX; ++w)
            if (w < W) mat[myk * W + w] = row[w];
    const int nk = n - r;
    if (tid < nk) qacc[tid] = 0;
    __syncthreads();

    // Kernel vectors: word w of k_f collects RREF[k][f] at the pivots of word w.
    for (int idx = tid; idx < nk * W; idx += nthr) {
        const int j = idx / W, w = idx - j * W;
        const int f = freec[j];
        uint64_t v = ((f >> 6) == w) ? (1ull << (f & 63)) : 0ull;
        const int klo = lower_bound_int(piv, r, 64 * w);
        const int khi = lower_bound_int(piv, r, 64 * w + 64);
        for (int k = klo; k < khi; ++k)
            if ((mat[k * W + (f >> 6)] >> (f & 63)) & 1ull) v |= 1ull << (piv[k] & 63);
        mat[(r + j) * W + w] = v;
        if (out.kernel) out.kernel[j * W + w] = v;
    }
    __syncthreads();

    // q(k_f): thread i adds popcount(A_i & k_f) when bit i of k_f is set.
    if (tid < n) {
        uint64_t arow[WMAX];
#pragma unroll
        for (int w = 0; w < WMAX; ++w) arow[w] = (w < W) ? rows[tid * W + w] : 0ull;
        for (int j = 0; j < nk; ++j) {
            const uint64_t *kv = &mat[(r + j) * W];
            if ((kv[tid >> 6] >> (tid & 63)) & 1ull) {
                int cnt = 0;
#pragma unroll
                for (int w = 0; w < WMAX; ++w)
                    if (w < W) cnt += __builtin_popcountll(arow[w] & kv[w]);
                atomicAdd(&qacc[j], cnt);
            }
        }
    }
    __syncthreads();
    if (tid < nk) {
        const int q = qacc[tid];
        const int f = freec[tid];
        if (q & 1) flag_internal = 1;
        if (q & 2) atomicOr(&shiftw[f >> 6], 1ull << (f & 63));
    }
    __syncthreads();

    for (int k = tid; k < n; k += nthr) out.pivots[k] = (k < r) ? piv[k] : -1;
    for (int idx0 = tid; idx0 < r * W; idx0 += 4 * nthr) {
        uint64_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int idx = idx0 + u * nthr;
            const int k = idx / W, w = idx - k * W;
            v[u] = (idx < r * W) ? rows[piv[k] * W + w] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (idx0 + u * nthr < r * W) out.basis[idx0 + u * nthr] = v[u];
    }
    if (tid < W) out.shift[tid] = shiftw[tid];
    if (tid == 0) {
        *out.rank = r;
        *out.status = flag_internal ? HLF_EINTERNAL : HLF_OK;
    }
}

template <int WMAX>
hlf_status launch_pack_t(const uint8_t *A, int n, int W, uint64_t *rows, int32_t *status,
                         hipStream_t stream) {
    hipLaunchKernelGGL(pack_dense_kernel<WMAX>, dim3(1), dim3(64 * W), 0, stream, A, n, W, rows,
                       status);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int WMAX>
hlf_status launch_wave_t(const uint64_t *rows, int n, int W, const FactorOut &out, int keep_bad,
                         hipStream_t stream) {
    hipLaunchKernelGGL(factor_wave_kernel<WMAX>, dim3(1), dim3(64), 0, stream, rows, n, W, out,
                       keep_bad);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int WMAX>
hlf_status launch_workgroup_t(const uint64_t *rows, int n, int W, const FactorOut &out,
                              int keep_bad, hipStream_t stream) {
    hipLaunchKernelGGL(factor_workgroup_kernel<WMAX>, dim3(1), dim3(64 * W), 0, stream, rows, n,
                       W, out, keep_bad);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

}  // namespace

hlf_status launch_pack(const uint8_t *A, int n, int W, uint64_t *rows, int32_t *status,
                       hipStream_t stream) {
    if (W >= 2) {
        const int vec16 = ((n & 15) == 0 && ((uintptr_t)A & 15u) == 0) ? 1 : 0;
        const unsigned blocks = (unsigned)((n + kPackRowsPerBlock - 1) / kPackRowsPerBlock);
        hipLaunchKernelGGL(pack_rows_kernel, dim3(blocks), dim3(kPackRowsThreads), 0, stream, A, n, W,
                           vec16, rows);
        if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
        hipLaunchKernelGGL(pack_check_kernel, dim3(1), dim3(1024), 0, stream, rows, n, W, status);
        return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
    }
    return launch_pack_t<1>(A, n, W, rows, status, stream);
}

hlf_status launch_factor(const uint64_t *rows, int n, int W, const FactorOut &out,
                         bool force_workgroup, bool keep_pack_status, hipStream_t stream) {
    const int kb = keep_pack_status ? 1 : 0;
    // One wave is faster up to n = 64; from two words on, the blocked
    // workgroup elimination is.
    if (!force_workgroup && W == 1) return launch_wave_t<1>(rows, n, W, out, kb, stream);
    if (W <= 1) return launch_workgroup_t<1>(rows, n, W, out, kb, stream);
    if (W <= 2) return launch_workgroup_t<2>(rows, n, W, out, kb, stream);
    if (W <= 4) return launch_workgroup_t<4>(rows, n, W, out, kb, stream);
    if (W <= 8) return launch_workgroup_t<8>(rows, n, W, out, kb, stream);
    return launch_workgroup_t<16>(rows, n, W, out, kb, stream);
}

}  // namespace hlf
