// Verification data for a cross-entropy benchmark of a device that runs the
// circuit (Section 5): exact pair statistics of a uniform solution, and the
// membership test that gives the ideal probability 2^-r of a sampled string
// (Section 1's definition of a solution, App. A's output distribution).
#include <utility>

#include "hlf_device.h"
#include "hlf_internal.h"

namespace hlf {
namespace {

// Row i per workgroup: quarters[i*n + j] = 0 if A_i = 0 or A_j = 0, 2 if
// A_i = A_j != 0, else 1.  z = l ^ XOR_k c_k B_k with c uniform makes
// coordinate i the functional c -> l_i ^ <c, beta_i>, beta_i = row i of A at
// the pivot columns; the pivot columns are an information set of the row
// space, so beta_i = beta_j exactly when A_i = A_j, and beta_i = 0 exactly
// when A_i = 0 (then l_i = 0: e_i is in Ker(A) with q(e_i) = A_ii = 0).
template <int WMAX>
__global__ __launch_bounds__(256) void pair_stats_kernel(FactorIn f, const uint64_t *__restrict__ rows,
                                                         uint8_t *__restrict__ quarters) {
    if (*(volatile int32_t *)f.status != HLF_OK) return;
    const int n = f.n, W = f.words;
    const int i = blockIdx.x;
    __shared__ uint64_t ri[WMAX];
    __shared__ int nz_i;
    if (threadIdx.x == 0) nz_i = 0;
    __syncthreads();
    if ((int)threadIdx.x < W) {
        const uint64_t v = rows[(size_t)i * W + threadIdx.x];
        ri[threadIdx.x] = v;
        if (v) atomicOr(&nz_i, 1);
    }
    __syncthreads();
    const bool nzi = nz_i != 0;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        uint64_t diff = 0, orj = 0;
#pragma unroll
        for (int w = 0; w < WMAX; ++w) {
            if (w < W) {
                const uint64_t x = rows[(size_t)j * W + w];
                diff |= x ^ ri[w];
                orj |= x;
            }
        }
        quarters[(size_t)i * n + j] = (!nzi || !orj) ? 0 : (diff == 0 ? 2 : 1);
    }
}

typedef int m4i __attribute__((ext_vector_type(4)));
typedef int m8i __attribute__((ext_vector_type(8)));
typedef float m16f __attribute__((ext_vector_type(16)));

// Pair statistics on the matrix cores (n > 64): quarters[i][j] needs |A_i|,
// |A_j| and the integer dot product popcount(A_i & A_j) (rows equal exactly
// when all three agree), and the dot products of all row pairs are the
// product of the packed rows with their transpose.  One wave per 32 x 32 tile
// of (i, j): v_mfma_scale_f32_32x32x64_f8f6f4 with E2M1 operands whose
// set-bit products are exactly 1 (the i rows at nibble positions 2, 1, 0, 0,
// the j rows at 0, 1, 2, 2 for bits 4t + 0..3), so the fp32 sums are the
// counts.  K chunk w is row word w; lane half h takes its 32-bit half.
// Accumulator register q of lane l holds the count of rows i = 32bi + 8(q/4)
// + 4(l/32) + q%4 and j = 32bj + l%32.
constexpr int kPairWaves = 4;

__global__ __launch_bounds__(64 * kPairWaves) void pair_stats_mfma_kernel(
    FactorIn f, const uint64_t *__restrict__ rows, uint8_t *__restrict__ quarters) {
    __shared__ uint32_t pci[kPairWaves][32];
    if (*(volatile int32_t *)f.status != HLF_OK) return;
    const int n = f.n, W = f.words;
    const int nb = (n + 31) >> 5;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, m = lane & 31;
    const int t = blockIdx.x * kPairWaves + wave;  // tile index, wave-uniform
    if (t >= nb * nb) return;                      // no barrier below
    const int bi = t / nb, bj = t - bi * nb;
    const int i = 32 * bi + m, j = 32 * bj + m;    // this lane's rows
    // words 2p + h of rows i and j, all loads at once
    uint64_t xi[HLF_MAX_N / 128], xj[HLF_MAX_N / 128];
    uint32_t pi = 0, pj = 0;
#pragma unroll
    for (int p = 0; p < HLF_MAX_N / 128; ++p) {
        const int w = 2 * p + h;
        xi[p] = (i < n && w < W) ? rows[(size_t)i * W + w] : 0ull;
        xj[p] = (j < n && w < W) ? rows[(size_t)j * W + w] : 0ull;
        pi += (uint32_t)__builtin_popcountll(xi[p]);
        pj += (uint32_t)__builtin_popcountll(xj[p]);
    }
    // whole-row popcounts: add the other half's words (lane l ^ 32)
    pi += __builtin_amdgcn_permlane32_swap(pi, pi, false, false)[h ? 0 : 1];
    pj += __builtin_amdgcn_permlane32_swap(pj, pj, false, false)[h ? 0 : 1];
    if (lane < 32) pci[wave][m] = pi;
    m16f acc;
    auto chunk = [&](int w, uint32_t yi, uint32_t yj) {
        const m8i a = {(int)((yi & 0x11111111u) << 2), (int)(yi & 0x22222222u),
                       (int)((yi & 0x44444444u) >> 2), (int)((yi & 0x88888888u) >> 3), 0, 0, 0, 0};
        const m8i b = {(int)(yj & 0x11111111u), (int)(yj & 0x22222222u),
                       (int)(yj & 0x44444444u), (int)((yj >> 1) & 0x44444444u), 0, 0, 0, 0};
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, w == 0 ? m16f{} : acc, 4, 4, 0, 127,
                                                             0, 127);
    };
#pragma unroll
    for (int p = 0; p < HLF_MAX_N / 128; ++p) {
        if (2 * p < W) {
            const auto yi = __builtin_amdgcn_permlane32_swap((uint32_t)xi[p], (uint32_t)(xi[p] >> 32), false, false);
            const auto yj = __builtin_amdgcn_permlane32_swap((uint32_t)xj[p], (uint32_t)(xj[p] >> 32), false, false);
            chunk(2 * p, yi[0], yj[0]);
            if (2 * p + 1 < W) chunk(2 * p + 1, yi[1], yj[1]);
        }
    }
    wave_lds_sync();  // pci of this wave written above
    if (j < n) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int mi = 8 * (q >> 2) + 4 * h + (q & 3);
            const int ii = 32 * bi + mi;
            if (ii < n) {
                const uint32_t c = (uint32_t)acc[q], ni = pci[wave][mi];
                quarters[(size_t)ii * n + j] = (ni == 0u || pj == 0u) ? 0 : (ni == pj && c == ni) ? 2 : 1;
            }
        }
    }
}

// Membership on the matrix cores (n > 192, 1 <= n - r <= 128): the parities
// <k_j, z_s> for all kernel vectors at once are the GF(2) product of the
// strings (num x n) and the kernel basis transposed (n x (n - r)), computed
// as in the sampler: v_mfma_scale_f32_32x32x64_f8f6f4 with E2M1 operands
// whose set-bit products are exactly 1, fp32 sums that are integer counts,
// bit 0 their parity.  K chunk w is string word w; lane half h takes its
// 32-bit half, and nibble t of operand dword d stands for bit 4t + d of it.
// The kernel vectors are already rows of n bits, the layout the basis operand
// needs (lane = kernel vector), so they are encoded once into LDS without a
// transpose.  A workgroup holds all (up to 128) of them; its 16 waves take
// contiguous blocks of 32 strings.  The product is taken with the kernel
// operand first, so accumulator register i of lane l holds the count of
// kernel vector 8(i/4) + 4(l/32) + i%4 of its 32-chunk for string l % 32.
// Two chunks share an accumulator, as in the sampler: the first K chunk adds
// to 2^23 and the second chunk of a pair carries the scale 2^11, so a sum is
// 2^23 + c + 2^11 c' (c, c' <= n <= 1024) and its raw bits 0 and 11 are the
// two parities.
constexpr int kMemMfmaMinWords = 4;
constexpr int kMemMfmaMaxVectors = 128;
constexpr int kMemWaves = 16;


__global__ __launch_bounds__(64 * kMemWaves) void membership_mfma_kernel(
    FactorIn f, const uint64_t *__restrict__ kernel, const uint64_t *__restrict__ z, uint64_t num,
    uint8_t *__restrict__ member) {
    constexpr int JC = kMemMfmaMaxVectors / 32;
    __shared__ __align__(16) uint32_t Bop[(HLF_MAX_N / 64) * JC * 64 * 4];  // 64 KiB
    __shared__ uint32_t target[JC];
    if (*(volatile int32_t *)f.status != HLF_OK) return;
    const int W = f.words;
    const int nk = f.n - *f.rank;
    if (nk < 1 || nk > kMemMfmaMaxVectors) return;  // the VALU kernel's case
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int h = lane >> 5, m = lane & 31;
    const int jcs = (nk + 31) >> 5;  // 32-vector chunks in use
    if (tid < JC) target[tid] = 0;
    __syncthreads();
    // target bit j = <k_j, l> (mod 2)
    if (tid < nk) {
        uint64_t acc = 0;
        for (int w = 0; w < W; ++w) acc ^= kernel[(size_t)tid * W + w] & f.shift[w];
        if (__builtin_popcountll(acc) & 1) atomicOr(&target[tid >> 5], 1u << (tid & 31));
    }
    // Kernel operand of chunk (w, jc): lane (h, n), dword d, nibble t holds
    // bit 64w + 32h + 4t + d of k_{32jc+n} at nibble position 2, 1, 0, 0 for
    // d = 0, 1, 2, 3 (0 beyond n - r).
    for (int t = wave; t < W * jcs; t += kMemWaves) {
        const int w = t / jcs, jc = t - w * jcs;
        const int j = 32 * jc + m;
        const uint32_t y = j < nk ? (uint32_t)(kernel[(size_t)j * W + w] >> (32 * h)) : 0u;
        uint32_t *dst = &Bop[((size_t)(w * JC + jc) * 64 + lane) * 4];
        dst[0] = (y & 0x11111111u) << 2;
        dst[1] = y & 0x22222222u;
        dst[2] = (y & 0x44444444u) >> 2;
        dst[3] = (y & 0x88888888u) >> 3;
    }
    __syncthreads();
    // After the extraction lane (h, m) holds the parities of chunk 2a + h
    // for string m: its targets and valid vectors.
    constexpr int JA = JC / 2;
    uint32_t valid[JA], tgt[JA];
#pragma unroll
    for (int a = 0; a < JA; ++a) {
        const int left = nk - 32 * (2 * a + h);
        valid[a] = left >= 32 ? ~0u : left > 0 ? (1u << left) - 1u : 0u;
        tgt[a] = target[2 * a + h];
    }
    m16f magic;
#pragma unroll
    for (int i = 0; i < 16; ++i) magic[i] = 8388608.0f;  // 2^23
    uint32_t emask[4], erot0[4], erot1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const uint32_t sh = (uint32_t)(u + 4 * h);
        emask[u] = 0x01010101u << sh;
        erot0[u] = (32u - sh) & 31u;  // rotate right: bit 0 of each byte to bit sh
        erot1[u] = (35u - sh) & 31u;  // bit 3 of each byte to bit sh
    }
    const uint64_t nblk = (num + 31) >> 5;
    const uint64_t per_wg = (nblk + gridDim.x - 1) / gridDim.x;
    const uint64_t blk_end = min(nblk, (uint64_t)(blockIdx.x + 1) * per_wg);
    for (uint64_t blk = (uint64_t)blockIdx.x * per_wg + wave; blk < blk_end; blk += kMemWaves) {
        const uint64_t s = 32ull * blk + (uint64_t)m;  // this lane's string
        const bool live = s < num;
        // Lane half h loads words 2p + h of its string, all at once; one swap
        // of the upper 32 lanes of a word's low dword with the lower 32 lanes
        // of its high dword then leaves every lane the 32-bit half h of words
        // 2p and 2p + 1 (lanes m and m + 32 hold the same string).
        uint64_t zw[HLF_MAX_N / 128];
#pragma unroll
        for (int p = 0; p < HLF_MAX_N / 128; ++p) {
            const int w = 2 * p + h;
            zw[p] = (live && w < W) ? z[s * (uint64_t)W + (uint64_t)w] : 0ull;
        }
        m16f acc[JA];
        auto chunk = [&](int w, uint32_t y) {
            const m8i a = {(int)(y & 0x11111111u), (int)(y & 0x22222222u),
                           (int)(y & 0x44444444u), (int)((y >> 1) & 0x44444444u), 0, 0, 0, 0};
#pragma unroll
            for (int jc = 0; jc < JC; ++jc) {
                if (jc < jcs) {
                    const m4i b4 = *reinterpret_cast<const m4i *>(&Bop[((size_t)(w * JC + jc) * 64 + lane) * 4]);
                    const m8i b = {b4[0], b4[1], b4[2], b4[3], 0, 0, 0, 0};
                    const int ja = jc >> 1;
                    if (jc & 1)
                        acc[ja] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(b, a, acc[ja], 4, 4, 0, 138, 0, 127);
                    else
                        acc[ja] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
                            b, a, w == 0 ? magic : acc[ja], 4, 4, 0, 127, 0, 127);
                }
            }
        };
#pragma unroll
        for (int p = 0; p < HLF_MAX_N / 128; ++p) {
            if (2 * p < W) {
                const auto ys = __builtin_amdgcn_permlane32_swap((uint32_t)zw[p], (uint32_t)(zw[p] >> 32),
                                                                 false, false);
                chunk(2 * p, ys[0]);
                if (2 * p + 1 < W) chunk(2 * p + 1, ys[1]);
            }
        }
        // Register i = 4t + u holds the counts of vector 8t + 4h + u of both
        // chunks of a pair: byte permutes gather bytes 0 (bit 0) and 1 (bit
        // 11 = bit 3 of byte 1) of registers u, 4+u, 8+u, 12+u, a rotation and
        // a mask put each parity at bit 8t + 4h + u, and one swap leaves lane
        // (h, m) the 32 parities of chunk 2a + h for string m.
        uint32_t bad = 0;
#pragma unroll
        for (int a = 0; a < JA; ++a) {
            if (2 * a < jcs) {
                uint32_t c[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) c[i] = __float_as_uint(acc[a][i]);
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
                bad |= ((sw[0] | sw[1]) ^ tgt[a]) & valid[a];
            }
        }
        // lanes 0..31 (the ones that store) take the verdict of lane + 32
        bad |= __builtin_amdgcn_permlane32_swap(bad, bad, false, false)[1];
        const uint64_t so = 32ull * blk + (uint64_t)lane;  // string `lane` for lanes < 32
        if (lane < 32 && so < num) member[so] = bad ? 0 : 1;
    }
}

// One thread per string: member[s] = 1 iff <k_j, z_s> = <k_j, l> (mod 2) for
// every kernel vector k_j, j < n - r.  <k_j, l> = l_{f_j} because k_j is 1 at
// its free column f_j, 0 at the other free columns, and l is 0 on the pivots.
// The word count W is a compile-time constant, so each kernel vector is one
// wide wave-uniform (scalar) load and one wait; the targets <k_j, l> are
// staged once per workgroup as a bit mask in LDS.
template <int W>
__global__ __launch_bounds__(256) void membership_kernel(FactorIn f, const uint64_t *__restrict__ kernel,
                                                         const uint64_t *__restrict__ z,
                                                         uint64_t num, uint8_t *__restrict__ member) {
    if (*(volatile int32_t *)f.status != HLF_OK) return;
    const int n = f.n;
    const int nk = n - *f.rank;
    if (W >= kMemMfmaMinWords && nk >= 1 && nk <= kMemMfmaMaxVectors) return;  // matrix-core kernel
    __shared__ uint32_t target[HLF_MAX_N / 32];
    for (int t = threadIdx.x; t < HLF_MAX_N / 32; t += blockDim.x) target[t] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < nk; j += blockDim.x) {
        uint64_t acc = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) acc ^= kernel[(size_t)j * W + w] & f.shift[w];
        if (__builtin_popcountll(acc) & 1) atomicOr(&target[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < num; s += stride) {
        uint64_t zv[W];
#pragma unroll
        for (int w = 0; w < W; ++w) zv[w] = z[s * W + w];
        bool ok = true;
        for (int j = 0; j < nk; ++j) {
            const uint64_t *kj = kernel + (size_t)j * W;
            uint64_t acc = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) acc ^= kj[w] & zv[w];
            const uint32_t par = (uint32_t)__builtin_popcountll(acc) & 1u;
            if (par != ((target[j >> 5] >> (j & 31)) & 1u)) {
                ok = false;
                break;
            }
        }
        member[s] = ok ? 1 : 0;
    }
}

template <int WMAX>
hlf_status launch_pair_stats_t(const FactorIn &f, const uint64_t *rows, uint8_t *quarters,
                               hipStream_t stream) {
    hipLaunchKernelGGL(pair_stats_kernel<WMAX>, dim3((unsigned)f.n), dim3(256), 0, stream, f, rows,
                       quarters);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int W>
hlf_status launch_membership_t(const FactorIn &f, const uint64_t *kernel, const uint64_t *z,
                               uint64_t num, uint8_t *member, hipStream_t stream) {
    uint64_t blocks = (num + 255) / 256;
    const uint64_t cap = (uint64_t)device_cu_count() * 8;
    if (blocks > cap) blocks = cap;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(membership_kernel<W>, dim3((unsigned)blocks), dim3(256), 0, stream, f,
                       kernel, z, num, member);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int... Ws>
hlf_status launch_membership_w(int W, const FactorIn &f, const uint64_t *kernel, const uint64_t *z,
                               uint64_t num, uint8_t *member, hipStream_t stream,
                               std::integer_sequence<int, Ws...>) {
    hlf_status st = HLF_EINVAL;
    ((W == Ws + 1 ? (st = launch_membership_t<Ws + 1>(f, kernel, z, num, member, stream), 0) : 0), ...);
    return st;
}

}  // namespace

hlf_status launch_pair_stats(const FactorIn &f, const uint64_t *rows, uint8_t *quarters,
                             hipStream_t stream) {
    const int W = f.words;
    if (W >= 2) {
        const int nb = (f.n + 31) / 32;
        const unsigned blocks = (unsigned)((nb * nb + kPairWaves - 1) / kPairWaves);
        hipLaunchKernelGGL(pair_stats_mfma_kernel, dim3(blocks), dim3(64 * kPairWaves), 0, stream, f,
                           rows, quarters);
        return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
    }
    return launch_pair_stats_t<1>(f, rows, quarters, stream);
}

hlf_status launch_membership(const FactorIn &f, const uint64_t *kernel, const uint64_t *z,
                             uint64_t num, uint8_t *member, hipStream_t stream) {
    // n - r is on the device: for n > 192 both kernels are launched and each
    // returns at once unless the case is its own (1 <= n - r <= 128 for the
    // matrix cores, every other one for the VALU kernel).
    if (f.words >= kMemMfmaMinWords) {
        const uint64_t blocks32 = (num + 31) / 32;
        uint64_t g = (uint64_t)device_cu_count();
        const uint64_t most = (blocks32 + kMemWaves - 1) / kMemWaves;
        if (g > most) g = most;
        if (g == 0) g = 1;
        hipLaunchKernelGGL(membership_mfma_kernel, dim3((unsigned)g), dim3(64 * kMemWaves), 0, stream,
                           f, kernel, z, num, member);
        if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    }
    return launch_membership_w(f.words, f, kernel, z, num, member, stream,
                               std::make_integer_sequence<int, HLF_MAX_N / 64>{});
}

}  // namespace hlf
