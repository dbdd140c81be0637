// Uniform single solutions (the quantum circuit's output distribution,
// Section 1 and Appendix A): sample s is z_s = l ^ XOR_{bit k of c_s} B_k with
// c_s uniform on {0,1}^r.  The coefficient words come from the SplitMix64
// stream of the caller's seed (or from the caller), so every sample depends
// only on (seed, s) -- never on the launch shape.
//
// n <= 64 (one word): the basis (at most 64 words) is staged in LDS once per
// workgroup; each thread produces whole samples, reading every basis row at a
// wave-uniform address (an LDS broadcast) and applying it under a mask, so no
// lane diverges.  Larger n run in sample_mfma_kernel (below): a sparse path
// for the sparse bases of the paper's grids, the matrix cores otherwise.

#include "hlf_device.h"
#include "hlf_internal.h"

namespace hlf {
namespace {

// A sample's W words are split over TPS threads (at most 4 words each); only
// the one-word shape is launched.
template <int WMAX>
struct SampleShape {
    static constexpr int kThreads = (WMAX >= 8) ? 1024 : 256;
    static constexpr int kTPS = (WMAX + 3) / 4;            // threads per sample
    static constexpr int kWPT = (WMAX + kTPS - 1) / kTPS;  // words per thread
};

template <int WMAX>
__global__ __launch_bounds__(SampleShape<WMAX>::kThreads) void sample_kernel(
    FactorIn f, uint64_t seed, uint64_t num, const uint64_t *__restrict__ coeffs,
    uint64_t *__restrict__ out) {
    using Sh = SampleShape<WMAX>;
    __shared__ uint64_t Bs[64 * WMAX * WMAX];
    __shared__ uint64_t ls[WMAX];
    if (*(volatile int32_t *)f.status != HLF_OK) return;
    const int r = *f.rank;
    const int W = f.words;
    for (int idx = threadIdx.x; idx < r * W; idx += blockDim.x) Bs[idx] = f.basis[idx];
    if ((int)threadIdx.x < W) ls[threadIdx.x] = f.shift[threadIdx.x];
    __syncthreads();

    const int R64 = (r + 63) >> 6;
    const int g = (int)threadIdx.x % Sh::kTPS;  // word group of this thread
    const int w0 = g * Sh::kWPT;
    const uint64_t per_block = blockDim.x / Sh::kTPS;
    const uint64_t stride = (uint64_t)gridDim.x * per_block;
    for (uint64_t s = (uint64_t)blockIdx.x * per_block + threadIdx.x / Sh::kTPS; s < num;
         s += stride) {
        uint64_t z[Sh::kWPT];
#pragma unroll
        for (int q = 0; q < Sh::kWPT; ++q) z[q] = (w0 + q < W) ? ls[w0 + q] : 0ull;
        for (int kw = 0; kw < R64; ++kw) {
            const uint64_t ctr = s * (uint64_t)R64 + (uint64_t)kw;
            const uint64_t c = coeffs ? coeffs[ctr] : mix13(seed + (ctr + 1) * kGamma);
            const int nb = (r - 64 * kw) < 64 ? (r - 64 * kw) : 64;
            const uint64_t *B = &Bs[(size_t)(64 * kw) * W + w0];
            for (int kb = 0; kb < nb; ++kb) {
                const uint64_t mask = 0ull - ((c >> kb) & 1ull);
#pragma unroll
                for (int q = 0; q < Sh::kWPT; ++q)
                    if (w0 + q < W) z[q] ^= B[kb * W + q] & mask;
            }
        }
#pragma unroll
        for (int q = 0; q < Sh::kWPT; ++q)
            if (w0 + q < W) out[s * W + w0 + q] = z[q];
    }
}

// ---------------------------------------------------------------------------
// Large n: sampling as a dense product over GF(2) on the matrix cores.
// Z = C * Bm mod 2, C the num x r coefficient bits, Bm the r x n basis bits,
// on v_mfma_scale_f32_32x32x64_f8f6f4 with 4-bit E2M1 operands (scale 1):
// fp32 sums of products that are 0 or exactly 1.  A workgroup owns one group
// of 32*JC output bits (JC column chunks of 32); its B operands, in the
// register layout of the instruction, are built once in LDS (ceil(r/64) x JC
// chunks of 64 lanes x 16 bytes).  Each wave multiplies blocks of 32 samples
// by them, the A operand coming straight from the coefficient words, which
// a wave generates once per block for all JC chunks.
//
// K chunk kc is coefficient word kc: lane l covers sample row l % 32 and the
// 32-bit half h = l / 32 of the word, y.  Nibble t of operand dword d stands
// for k = 64kc + 32h + 4t + d, for A and B alike.  A single set bit of an
// E2M1 nibble reads 0.5, 1 or 2 at positions 0, 1, 2 (position 3 is the
// sign), so the A dwords are y & 0x11111111, y & 0x22222222, y & 0x44444444
// and (y >> 1) & 0x44444444 (positions 0, 1, 2, 2), and the B nibbles, built
// once, put their bits at positions 2, 1, 0, 0: every product of two set
// bits is 1.  The product is taken as Z^T = Bm^T * C^T (the basis operand
// first), so accumulator register i of lane l holds output bit 8*(i/4) +
// 4*(l/32) + i%4 of a column chunk for sample l % 32: a lane assembles 16
// bits of its sample's word and takes the other 16 from lane l ^ 32.
//
// Parity without a conversion, two chunks per accumulator: the first K chunk
// adds its products to 2^23 (a constant accumulator operand) instead of 0,
// and the products of the second column chunk of a pair carry the scale
// 2^11, so every sum is 2^23 + c + 2^11 c' with c, c' <= r <= 1024 the two
// counts.  fp32 holds it exactly (below 2^24, unit spacing), so bit 0 of its
// raw bits is the parity of c and bit 11 that of c'.  The raw bits are read
// with __float_as_uint on each element: __builtin_bit_cast applied to an
// element of an ext_vector_type value read element 0 for every index in this
// compiler (the generated IR extracted lane 0 sixteen times).
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kMfmaMaxKC = HLF_MAX_N / 64;
constexpr int kE2M1 = 4;         // operand format code of the instruction
constexpr int kScaleOne = 127;   // E8M0 scale 2^0
constexpr int kScaleHigh = 138;  // E8M0 scale 2^11
constexpr float kTwo23 = 8388608.0f;

// a ^ b ^ c in one instruction (a three-input bitwise op, truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// 32x32 bit transposes within each half of the wave, on the VALU alone:
// lane l of a half holds row l of each matrix and gets its column l.  Step j
// exchanges, between lanes l and l ^ j, the bits whose row and column indices
// differ in bit j (the lane with bit j clear keeps the columns with bit j
// clear and takes its partner's, moved up by j; the other keeps the columns
// with bit j set and takes its partner's, moved down).  Partners: j = 16 by
// a permlane16 swap of the two rows of 16, j = 8 by a row mirror then a half
// mirror, j = 4 by a half mirror then a quad mirror, j = 2 and 1 by quad
// permutations (DPP).  Byte and halfword steps merge with one byte permute,
// the others with a masked rotate and an and-or.
template <int N>
__device__ __forceinline__ void half_transpose32_n(uint32_t (&x)[N]) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    {   // j = 16: after the swap, the first result holds the lane's own value
        // in rows 0 and 2 and its partner's in rows 1 and 3, the second the
        // other way round, so one byte permute with a per-row selector merges
        const bool up = lane & 16;
        const uint32_t sel = up ? 0x07060302u : 0x05040100u;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const auto sw = __builtin_amdgcn_permlane16_swap(x[i], x[i], false, false);
            x[i] = __builtin_amdgcn_perm(sw[1], sw[0], sel);
        }
    }
    {   // j = 8
        const uint32_t sel = (lane & 8) ? 0x03070105u : 0x06020400u;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const int t = __builtin_amdgcn_mov_dpp((int)x[i], 0x140, 0xF, 0xF, false);   // row mirror
            const uint32_t y = (uint32_t)__builtin_amdgcn_mov_dpp(t, 0x141, 0xF, 0xF, false);  // half mirror
            x[i] = __builtin_amdgcn_perm(y, x[i], sel);
        }
    }
#pragma unroll
    for (int step = 2; step >= 0; --step) {
        const int j = 1 << step;
        const uint32_t mj = j == 4 ? 0x0F0F0F0Fu : j == 2 ? 0x33333333u : 0x55555555u;
        const uint32_t M = (lane & j) ? ~mj : mj;
        const uint32_t R = (lane & j) ? (uint32_t)j : (uint32_t)(32 - j);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            int y;
            if (j == 4) {
                const int t = __builtin_amdgcn_mov_dpp((int)x[i], 0x141, 0xF, 0xF, false);  // half mirror
                y = __builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, true);                     // quad [3,2,1,0]
            } else if (j == 2) {
                y = __builtin_amdgcn_mov_dpp((int)x[i], 0x4E, 0xF, 0xF, true);  // quad [2,3,0,1]
            } else {
                y = __builtin_amdgcn_mov_dpp((int)x[i], 0xB1, 0xF, 0xF, true);  // quad [1,0,3,2]
            }
            const uint32_t t = (uint32_t)y & M;
            x[i] = (x[i] & M) | __builtin_amdgcn_alignbit(t, t, R);
        }
    }
}

// ---------------------------------------------------------------------------
// Sparse bases.  B_k is column p_k of A, so on the paper's 2D grids every
// basis row and every basis column has at most five set bits (a vertex and
// its neighbours), and sampling is a sparse product: bit j of z_s is l_j XOR
// the coefficient bits c_{s,k} of the rows k with B_k[j] = 1.  A workgroup
// whose basis words (64 of its columns in one row) have at most kSparseMaxW
// set bits, and whose columns have at most kSparseMaxW rows, takes this path
// instead of the matrix cores.  Per 32-sample block, the
// coefficient words of the K chunks that touch its columns are transposed
// into bit slices (slice k holds c_{s,k} of the block's 32 samples, one bit
// per sample) in a per-wave LDS table; each output column XORs the slices of
// the rows in its list, and the output slices are transposed back into the
// samples' words.  The lists hold byte offsets into a wave's table, so a
// gather is one add and one LDS read.
// ---------------------------------------------------------------------------
constexpr int kSparseMaxW = 16;  // set bits per basis word, rows per column, at most

// LDS layout of the sparse path, in dwords from the start of the workgroup's
// buffer (it aliases the matrix-core operands, which are not built then).
// RMAX bounds the rows (64 ceil(n/64)); NCOL = 64 * words per group.
constexpr int kSpVotes = 0;                       // [wave] K-chunk pairs in use << 1 | heavy word
constexpr int kSpColCnt = 32;                     // [NCOL] column weights
constexpr int kSpLists = kSpColCnt + 256;         // [NCOL][kSparseMaxW] row lists: 4k (16-byte aligned)
constexpr int kSpSlices = kSpLists + 256 * kSparseMaxW;  // per wave: [RMAX + 4] slices
static_assert(kSpLists % 4 == 0 && kSpSlices % 4 == 0, "16-byte aligned lists");

// Slices per wave: every k the K-chunk pairs reach, 64 * 2 * ceil(KC/2)
// (the JC = 4 kernel serves W <= 3, so KC <= 3), then a zero slice.
template <int JC>
constexpr int sparse_rmax() { return JC == 4 ? 256 : HLF_MAX_N; }

// The 32-sample blocks of the sparse path.
template <int JC, int WAVES, int MWB>
__device__ __forceinline__ void sample_sparse_blocks(const FactorIn &f, int r, uint32_t pairs, uint64_t seed,
                                                     uint64_t num, const uint64_t *__restrict__ coeffs,
                                                     uint64_t *__restrict__ out, uint32_t *lds) {
    constexpr int QW = JC / 2;
    constexpr int RMAX = sparse_rmax<JC>();
    const int W = f.words;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, m = lane & 31;
    const int KC = (r + 63) >> 6;
    const int w0 = QW * (int)blockIdx.x;
    const int nq = min(QW, W - w0);
    const uint32_t *lists = lds + kSpLists;
    uint32_t *cs = lds + kSpSlices + wave * (RMAX + 4);  // cs[RMAX] stays zero
    const char *csb = reinterpret_cast<const char *>(cs);
    // Lane (h, m) gathers the output columns 64c + 32h + m: their row lists
    // (unused entries point at the zero slice) and bits of l.
    uint32_t lbit[QW];
#pragma unroll
    for (int c = 0; c < QW; ++c) {
        const uint32_t lw = c < nq ? reinterpret_cast<const uint32_t *>(f.shift)[2 * (w0 + c) + h] : 0u;
        lbit[c] = 0u - ((lw >> m) & 1u);
    }
    // Row lists of the lane's columns: byte offsets into the wave's table.
    // Short lists stay in registers for the whole launch; longer ones are
    // read per block and column.
    constexpr bool kHoist = MWB <= 8;
    auto load_list = [&](int c, uint32_t (&e)[MWB]) {
        const uint32_t *lp = lists + (64 * c + 32 * h + m) * kSparseMaxW;
#pragma unroll
        for (int i = 0; i < MWB; i += 4) {
            if (i + 4 <= MWB) {
                const uint4 q4 = *reinterpret_cast<const uint4 *>(lp + i);
                e[i] = q4.x;
                e[i + 1] = q4.y;
                e[i + 2] = q4.z;
                e[i + 3] = q4.w;
            } else {
#pragma unroll
                for (int j = i; j < MWB; ++j) e[j] = lp[j];
            }
        }
    };
    uint32_t kk[kHoist ? QW : 1][MWB];
    if constexpr (kHoist) {
#pragma unroll
        for (int c = 0; c < QW; ++c) load_list(c, kk[c]);
    }
    uint32_t *out32 = reinterpret_cast<uint32_t *>(out);
    const uint64_t nblk = (num + 31) >> 5;
    const uint64_t per_wg = (nblk + gridDim.y - 1) / gridDim.y;
    const uint64_t blk_end = min(nblk, (uint64_t)(blockIdx.y + 1) * per_wg);
    for (uint64_t blk = (uint64_t)blockIdx.y * per_wg + wave; blk < blk_end; blk += WAVES) {
        const uint64_t s = 32ull * blk + (uint64_t)m;  // lane (h, m): sample m of the block
        const bool live = s < num;
        const uint64_t ctr0 = s * (uint64_t)KC + (uint64_t)h;  // word h of the sample
        uint64_t state = seed + (ctr0 + 1) * kGamma;  // SplitMix64 state of word 2p + h
        for (int p = 0; 2 * p < KC; ++p, state += 2 * kGamma) {
            if (!((pairs >> p) & 1u)) continue;  // wave-uniform
            // Lane half h makes coefficient word 2p + h of its sample; within
            // each half, the low and high dwords transposed give lane (h, m)
            // the slices of k = 64(2p+h) + m and 64(2p+h) + 32 + m.  Words of
            // samples >= num and beyond the last one are left unmasked: they
            // only reach bits of samples that are not stored and slices of
            // rows >= r, which no list holds.
            const int kc = 2 * p + h;
            uint64_t word;
            if (coeffs) {  // wave-uniform
                word = (live && kc < KC) ? coeffs[ctr0 + 2 * p] : 0ull;
            } else {
                word = mix13(state);
            }
            uint32_t y[2] = {(uint32_t)word, (uint32_t)(word >> 32)};
            half_transpose32_n<2>(y);
            cs[64 * kc + m] = y[0];
            cs[64 * kc + 32 + m] = y[1];
        }
        // Per column: the slices of its rows, XORed onto the bits of l.
        uint32_t v[QW];
#pragma unroll
        for (int c = 0; c < QW; ++c) {
            uint32_t e[MWB];
            if constexpr (kHoist) {
#pragma unroll
                for (int i = 0; i < MWB; ++i) e[i] = kk[c][i];
            } else {
                load_list(c, e);
            }
            uint32_t sv[MWB];
#pragma unroll
            for (int i = 0; i < MWB; ++i) sv[i] = *reinterpret_cast<const uint32_t *>(csb + e[i]);
            uint32_t acc = lbit[c];
#pragma unroll
            for (int i = 0; i + 1 < MWB; i += 2) acc = xor3(acc, sv[i], sv[i + 1]);
            if (MWB & 1) acc ^= sv[MWB - 1];
            v[c] = acc;
        }
        // Slice of column 64c + 32h + m, transposed within the half: lane
        // (h, m) gets dword h of word c of sample m.
        half_transpose32_n<QW>(v);
#pragma unroll
        for (int c = 0; c < QW; ++c)
            if (live && c < nq) out32[(s * (uint64_t)W + (uint64_t)(w0 + c)) * 2 + h] = v[c];
    }
}

// JC column chunks (JC/2 words of every sample) per workgroup, WAVES waves.
template <int JC, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void sample_mfma_kernel(
    FactorIn f, uint64_t seed, uint64_t num, const uint64_t *__restrict__ coeffs,
    uint64_t *__restrict__ out) {
    constexpr int QW = JC / 2;  // words per workgroup
    constexpr int TPW = (kMfmaMaxKC * QW + WAVES - 1) / WAVES;  // basis tiles per wave, at most
    __shared__ __align__(16) uint32_t Bop[kMfmaMaxKC * JC * 64 * 4];
    static_assert(kSpSlices + WAVES * (sparse_rmax<JC>() + 4) <= kMfmaMaxKC * JC * 64 * 4, "sparse layout fits");
    static_assert(64 * QW <= 256 && 64 * QW <= 64 * WAVES, "one column per thread");
    static_assert(WAVES <= 16, "one vote word per wave");
    const int W = f.words;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, m = lane & 31;
    const int w0 = QW * (int)blockIdx.x;
    const int nq = min(QW, W - w0);   // words of this group that exist
    // The group's basis words are staged in LDS ([word q][row k], at the
    // top of the buffer): consecutive lanes load consecutive words of a row,
    // so a row's words arrive in one request.  The basis array has n rows,
    // so the loads go out with those of the status and the rank; rows k >= r
    // are cleared once the rank has arrived.  (The record was written by an
    // earlier launch: plain loads see it.)
    constexpr int RS = sparse_rmax<JC>();  // rows staged, at most
    constexpr int kStage = kMfmaMaxKC * JC * 64 * 4 - 2 * QW * RS;  // dwords
    constexpr int SPT = (RS * QW + 64 * WAVES - 1) / (64 * WAVES);  // staged words per thread
    static_assert(kSpSlices + WAVES * (RS + 4) <= kStage && kStage % 2 == 0, "staging above the sparse tables");
    uint64_t *stage = reinterpret_cast<uint64_t *>(Bop + kStage);
    const int status = *f.status;
    const int r = *f.rank;
    {
        uint64_t sw[SPT];
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            const int e = tid + i * 64 * WAVES;
            const int k = e / QW, q = e % QW;
            sw[i] = (k < f.n && q < nq) ? f.basis[(size_t)k * W + w0 + q] : 0ull;
        }
#pragma unroll
        for (int i = 0; i < SPT; ++i) {
            const int e = tid + i * 64 * WAVES;
            if (e < RS * QW) stage[(e % QW) * RS + e / QW] = sw[i];
        }
    }
    if (status != HLF_OK) return;
    const int KC = (r + 63) >> 6;     // K chunks of 64 = coefficient words
    // Path choice, by votes of the waves (one LDS word per wave): the
    // sparse path needs every basis word of the group (64 columns of a row)
    // to have at most kSparseMaxW set bits, and then every column at most
    // kSparseMaxW rows.
    constexpr int NCOL = 64 * QW;
    int *colcnt = reinterpret_cast<int *>(Bop + kSpColCnt);
    if (tid < NCOL) colcnt[tid] = 0;
    {   // row lists start as RMAX (the zero slice) in every entry
        constexpr uint32_t kFill = 4u * (uint32_t)sparse_rmax<JC>();
        for (int i = tid; i < NCOL * kSparseMaxW; i += 64 * WAVES) Bop[kSpLists + i] = kFill;
    }
    __syncthreads();  // staged words written
    // The basis tiles: a wave takes (kc, word q) tiles, lane t the word of
    // B_{64kc+t}.
    uint64_t x[TPW];
    {
        uint32_t pm = 0u;  // K-chunk pairs with a set bit in the group's columns
        bool heavy = false;
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int t = wave + i * WAVES;
            const int kc = t / QW, q = t - kc * QW;
            const int k = 64 * kc + lane;
            x[i] = (t < KC * QW && k < r) ? stage[q * RS + k] : 0ull;
            if (__ballot(x[i] != 0ull)) pm |= 1u << (kc >> 1);  // kc is wave-uniform
            heavy |= __popcll(x[i]) > kSparseMaxW;
        }
        const bool heavy_w = __ballot(heavy) != 0ull;
        if (lane == 0) Bop[kSpVotes + wave] = pm << 1 | (heavy_w ? 1u : 0u);
    }
    __syncthreads();
    uint32_t votes = 0u;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) votes |= Bop[kSpVotes + w];
    votes = __builtin_amdgcn_readfirstlane(votes);  // workgroup-uniform
    if (!(votes & 1u)) {
        // Row lists per column (at most kSparseMaxW kept; a longer one sends
        // the workgroup to the matrix cores).
        uint32_t *lists = Bop + kSpLists;
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int t = wave + i * WAVES;
            const int kc = t / QW, q = t - kc * QW;
            const uint32_t entry = 4u * (uint32_t)(64 * kc + lane);
            uint64_t v = x[i];
            while (v) {
                const int col = 64 * q + __builtin_ctzll(v);
                v &= v - 1;
                const int slot = atomicAdd(&colcnt[col], 1);
                if (slot < kSparseMaxW) lists[col * kSparseMaxW + slot] = entry;
            }
        }
        __syncthreads();
        // Every wave reads all column weights, so all reach the same flags
        // (columns above 5, 8, kSparseMaxW rows) without another barrier.
        uint32_t cf;
        {
            int cw = 0;
#pragma unroll
            for (int c = lane; c < NCOL; c += 64) cw = max(cw, colcnt[c]);
            cf = (__ballot(cw > 5) ? 1u : 0u) | (__ballot(cw > 8) ? 2u : 0u) |
                 (__ballot(cw > kSparseMaxW) ? 4u : 0u);
        }
        if (!(cf & 4u)) {
            constexpr int RMAX = sparse_rmax<JC>();
            if (lane == 0) Bop[kSpSlices + wave * (RMAX + 4) + RMAX] = 0u;  // the zero slice
            const uint32_t pairs = votes >> 1;
            if (!(cf & 1u)) sample_sparse_blocks<JC, WAVES, 5>(f, r, pairs, seed, num, coeffs, out, Bop);
            else if (!(cf & 2u)) sample_sparse_blocks<JC, WAVES, 8>(f, r, pairs, seed, num, coeffs, out, Bop);
            else sample_sparse_blocks<JC, WAVES, kSparseMaxW>(f, r, pairs, seed, num, coeffs, out, Bop);
            return;
        }
    }
    __syncthreads();  // the weights are read; the operands overwrite them
    // B operands.  Lanes 32h .. 32h+31 of a tile hold rows 64kc + 32h +
    // 0..31; their low dwords (columns 64q + 0..31) and high dwords (64q +
    // 32..63), each transposed within the half, give lane (h, m) half h of
    // column 64q + m (chunk 2q, first) and of column 64q + 32 + m (chunk
    // 2q + 1, second).  Nibble t of dword d holds k = 32h + 4t + d at
    // position 2, 1, 0, 0 for d = 0..3.
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int t = wave + i * WAVES;
        if (t >= KC * QW) break;  // wave-uniform
        const int kc = t / QW, q = t - kc * QW;
        uint32_t y2[2] = {(uint32_t)x[i], (uint32_t)(x[i] >> 32)};
        half_transpose32_n<2>(y2);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const uint32_t y = y2[e];
            const v4i d = {(int)((y & 0x11111111u) << 2), (int)(y & 0x22222222u),
                           (int)((y & 0x44444444u) >> 2), (int)((y & 0x88888888u) >> 3)};
            *reinterpret_cast<v4i *>(&Bop[((size_t)(kc * JC + 2 * q + e) * 64 + lane) * 4]) = d;
        }
    }
    __syncthreads();

    // Lane (h, m) stores dword h of each word of sample m: chunk 2q + h.
    uint32_t *out32 = reinterpret_cast<uint32_t *>(out);
    uint32_t lh[QW];
#pragma unroll
    for (int q = 0; q < QW; ++q) {
        const uint64_t lw = q < nq ? f.shift[w0 + q] : 0ull;
        lh[q] = h ? (uint32_t)(lw >> 32) : (uint32_t)lw;
    }
    v16f magic;
#pragma unroll
    for (int i = 0; i < 16; ++i) magic[i] = kTwo23;
    // Bit extraction (below): the parity bits of register 4t + u sit at bit 0
    // (chunk 2q) and bit 11 (chunk 2q + 1); they go to bit 8t + 4h + u of the
    // lane's two words.  Per u, a mask and two rotations.
    uint32_t emask[4], erot0[4], erot1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t sh = (uint32_t)(u + 4 * h);
        emask[u] = 0x01010101u << sh;
        erot0[u] = (32u - sh) & 31u;  // rotate right: bit 0 of each byte to bit sh
        erot1[u] = (35u - sh) & 31u;  // bit 3 of each byte to bit sh
    }
    // This workgroup's samples: a contiguous run of 32-sample blocks, taken by
    // its waves in turn (every SIMD of the CU gets the same number of blocks).
    const uint64_t nblk = (num + 31) >> 5;
    const uint64_t per_wg = (nblk + gridDim.y - 1) / gridDim.y;
    const uint64_t blk_end = min(nblk, (uint64_t)(blockIdx.y + 1) * per_wg);
    for (uint64_t blk = (uint64_t)blockIdx.y * per_wg + wave; blk < blk_end; blk += WAVES) {
        const uint64_t s = 32ull * blk + (uint64_t)m;  // this lane's A row
        const bool live = s < num;
        // (Bits k >= r of the last word meet B operand rows k >= r, which are
        // zero, so they need no mask.)
        // Coefficient words 2p, 2p+1 of this row are K chunks 2p, 2p+1: lane
        // half h generates word 2p+h (SplitMix64 state seed + (ctr+1) gamma,
        // advanced by 2 gamma per step).  One swap of the upper 32 lanes of
        // its low dword with the lower 32 lanes of its high dword then leaves
        // every lane the 32-bit half h of word 2p (first) and of word 2p+1
        // (second); lanes m and m + 32 cover the same row.
        const uint64_t ctr0 = s * (uint64_t)KC + (uint64_t)h;
        uint64_t state = seed + (ctr0 + 1) * kGamma;
        auto words = [&](int p) {
            const int q = 2 * p + h;
            uint64_t mine = 0ull;
            if (live && q < KC) mine = coeffs ? coeffs[ctr0 + 2 * p] : mix13(state);
            state += 2 * kGamma;
            return __builtin_amdgcn_permlane32_swap((uint32_t)mine, (uint32_t)(mine >> 32), false, false);
        };
        // Accumulator q takes the products of chunk 2q with scale 1 and those
        // of chunk 2q + 1 with scale 2^11: every sum is 2^23 + c + 2^11 c'
        // (counts c, c' <= r <= 1024, below 2^24 and exact in fp32), so the
        // raw bits hold the parity of c at bit 0 and that of c' at bit 11.
        v16f acc[QW];
        auto chunk = [&](int kc, uint32_t y, bool first) {
            const v8i a = {(int)(y & 0x11111111u), (int)(y & 0x22222222u),
                           (int)(y & 0x44444444u), (int)((y >> 1) & 0x44444444u), 0, 0, 0, 0};
#pragma unroll
            for (int q = 0; q < QW; ++q) {
                const v4i b0 = *reinterpret_cast<const v4i *>(&Bop[((size_t)(kc * JC + 2 * q) * 64 + lane) * 4]);
                const v4i b1 = *reinterpret_cast<const v4i *>(&Bop[((size_t)(kc * JC + 2 * q + 1) * 64 + lane) * 4]);
                const v8i bl = {b0[0], b0[1], b0[2], b0[3], 0, 0, 0, 0};
                const v8i bh = {b1[0], b1[1], b1[2], b1[3], 0, 0, 0, 0};
                acc[q] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    bl, a, first ? magic : acc[q], kE2M1, kE2M1, 0, kScaleOne, 0, kScaleOne);
                acc[q] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                    bh, a, acc[q], kE2M1, kE2M1, 0, kScaleHigh, 0, kScaleOne);
            }
        };
        if (KC == 0) {
#pragma unroll
            for (int q = 0; q < QW; ++q) acc[q] = magic;
        } else {
            auto ys = words(0);
            chunk(0, ys[0], true);
            if (KC > 1) chunk(1, ys[1], false);
            for (int p = 1; 2 * p < KC; ++p) {
                ys = words(p);
                chunk(2 * p, ys[0], false);
                if (2 * p + 1 < KC) chunk(2 * p + 1, ys[1], false);
            }
        }
        // Register i = 4t + u holds the bits of column 8t + 4h + u of both
        // chunks.  Byte permutes gather bytes 0 (bit 0: chunk 2q) and 1 (bit
        // 11 = bit 3 of byte 1: chunk 2q + 1) of registers u, 4+u, 8+u, 12+u
        // into bytes 0..3; a rotation and a mask put each bit in place.  One
        // swap then gives the lanes of half 0 their partner's bits of chunk 2q
        // and those of half 1 their partner's bits of chunk 2q + 1.
#pragma unroll
        for (int q = 0; q < QW; ++q) {
            uint32_t c[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) c[i] = __float_as_uint(acc[q][i]);
            uint32_t lo = 0u, hi = 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t P = __builtin_amdgcn_perm(c[4 + u], c[u], 0x05010400u);
                const uint32_t Q = __builtin_amdgcn_perm(c[12 + u], c[8 + u], 0x05010400u);
                const uint32_t R = __builtin_amdgcn_perm(Q, P, 0x05040100u);  // bytes 0
                const uint32_t S = __builtin_amdgcn_perm(Q, P, 0x07060302u);  // bytes 1
                lo |= __builtin_amdgcn_alignbit(R, R, erot0[u]) & emask[u];
                hi |= __builtin_amdgcn_alignbit(S, S, erot1[u]) & emask[u];
            }
            const auto sw = __builtin_amdgcn_permlane32_swap(lo, hi, false, false);
            if (live && q < nq) out32[(s * (uint64_t)W + (uint64_t)(w0 + q)) * 2 + h] = (sw[0] | sw[1]) ^ lh[q];
        }
    }
}

template <int JC, int WAVES>
hlf_status launch_sample_mfma_t(const FactorIn &f, uint64_t seed, uint64_t num,
                                const uint64_t *coeffs, uint64_t *out, hipStream_t stream) {
    const int W = f.words;
    const unsigned groups = (unsigned)((W + JC / 2 - 1) / (JC / 2));
    const uint64_t blocks32 = (num + 31) / 32;
    // One workgroup per CU; every workgroup builds the operands once and
    // takes a contiguous run of 32-sample blocks, at least one per wave.
    uint64_t y = (uint64_t)device_cu_count() / groups;
    const uint64_t most = (blocks32 + WAVES - 1) / WAVES;
    if (y > most) y = most;
    if (y == 0) y = 1;
    if (y > 0xFFFFull) return HLF_EINVAL;
    hipLaunchKernelGGL((sample_mfma_kernel<JC, WAVES>), dim3(groups, (unsigned)y),
                       dim3(64 * WAVES), 0, stream, f, seed, num, coeffs, out);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

hlf_status launch_sample_mfma(const FactorIn &f, uint64_t seed, uint64_t num,
                              const uint64_t *coeffs, uint64_t *out, hipStream_t stream) {
    // Four words (256 output bits) per workgroup from W = 4: the coefficient
    // words and A operands of a block then serve 8 products per K chunk, and
    // 12 waves (three per SIMD) share the 128 KiB of operands (four waves per
    // SIMD measured slower).
    if (f.words >= 4) return launch_sample_mfma_t<8, 12>(f, seed, num, coeffs, out, stream);
    return launch_sample_mfma_t<4, 16>(f, seed, num, coeffs, out, stream);
}

template <int WMAX>
hlf_status launch_sample_t(const FactorIn &f, uint64_t seed, uint64_t num,
                           const uint64_t *coeffs, uint64_t *out, hipStream_t stream) {
    using Sh = SampleShape<WMAX>;
    constexpr int T = Sh::kThreads;
    const uint64_t per_block = T / Sh::kTPS;
    uint64_t blocks = (num + per_block - 1) / per_block;
    const uint64_t cap = (uint64_t)device_cu_count() * ((WMAX >= 8) ? 1 : 4);
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(sample_kernel<WMAX>, dim3((unsigned)blocks), dim3(T), 0, stream, f, seed,
                       num, coeffs, out);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

}  // namespace

hlf_status launch_sample(const FactorIn &f, uint64_t seed, uint64_t num, const uint64_t *coeffs,
                         uint64_t *out, hipStream_t stream) {
    const int W = f.words;
    // n > 64 on the matrix cores: at n = 81..169 they took 7.3-8.0 us for 65536
    // samples where one sample per thread took 12-31 us.
    if (W >= 2) return launch_sample_mfma(f, seed, num, coeffs, out, stream);
    return launch_sample_t<1>(f, seed, num, coeffs, out, stream);
}

}  // namespace hlf
