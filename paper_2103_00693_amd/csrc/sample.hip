// Uniform single solutions (the quantum circuit's output distribution,
// Section 1 and Appendix A): sample s is z_s = l ^ XOR_{bit k of c_s} B_k with
// c_s uniform on {0,1}^r.  The coefficient words come from the SplitMix64
// stream of the caller's seed (or from the caller), so every sample depends
// only on (seed, s) -- never on the launch shape.
//
// The basis (r rows of W words, <= 128 KiB) is staged in LDS once per
// workgroup; each thread produces whole samples, reading every basis row at a
// wave-uniform address (an LDS broadcast) and applying it under a mask, so no
// lane diverges.
#include "hlf_device.h"
#include "hlf_internal.h"

namespace hlf {
namespace {

// A sample's W words are split over TPS threads (at most 4 words each), so
// that large-n launches still spread over every CU.
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
    if (W <= 1) return launch_sample_t<1>(f, seed, num, coeffs, out, stream);
    if (W <= 2) return launch_sample_t<2>(f, seed, num, coeffs, out, stream);
    if (W <= 4) return launch_sample_t<4>(f, seed, num, coeffs, out, stream);
    if (W <= 8) return launch_sample_t<8>(f, seed, num, coeffs, out, stream);
    return launch_sample_t<16>(f, seed, num, coeffs, out, stream);
}

}  // namespace hlf
