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
    if (W <= 1) return launch_pair_stats_t<1>(f, rows, quarters, stream);
    if (W <= 2) return launch_pair_stats_t<2>(f, rows, quarters, stream);
    if (W <= 4) return launch_pair_stats_t<4>(f, rows, quarters, stream);
    if (W <= 8) return launch_pair_stats_t<8>(f, rows, quarters, stream);
    return launch_pair_stats_t<16>(f, rows, quarters, stream);
}

hlf_status launch_membership(const FactorIn &f, const uint64_t *kernel, const uint64_t *z,
                             uint64_t num, uint8_t *member, hipStream_t stream) {
    return launch_membership_w(f.words, f, kernel, z, num, member, stream,
                               std::make_integer_sequence<int, HLF_MAX_N / 64>{});
}

}  // namespace hlf
