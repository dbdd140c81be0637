// Stage 1 of the two-stage scheme (the paper's CLA module, Section 2,
// tasks (1)-(4)) on gfx950:
//   * pack_dense_kernel: dense 0/1 matrix -> packed uint64 rows, with the
//     symmetry / 0-1 validation of the problem statement (Section 1);
//   * factor_wave_kernel: one wavefront per instance for n <= 192; every
//     lane keeps its rows in VGPRs, pivots are found with a ballot and the
//     pivot row is broadcast with readlane -- no barriers in the elimination;
//   * factor_workgroup_kernel: one workgroup per instance for n <= 1024, one
//     row per thread (VGPRs, mirrored in LDS), pivot choice by an LDS
//     atomicMin over per-wave ballots, one barrier per column.
// Both variants produce the canonical record defined in hlf.h (the RREF is
// unique, so the pivot rows chosen do not matter).
#include "factor_wave.h"
#include "hlf_device.h"
#include "hlf_internal.h"

#include <climits>

namespace hlf {
namespace {

// ---------------------------------------------------------------------------
// A0: pack + validate.  One workgroup of 64*W threads; each wave packs groups
// of rows by ballot over 64 consecutive bytes, then checks A = A^T: for
// column c, the ballot of bit c over the 64 rows held by wave v is word v of
// column c, which must equal word v of row c.
// ---------------------------------------------------------------------------
template <int WMAX>
__global__ __launch_bounds__(64 * WMAX) void pack_dense_kernel(const uint8_t *__restrict__ A, int n,
                                                               int W, uint64_t *__restrict__ rows,
                                                               int32_t *__restrict__ status) {
    __shared__ uint64_t lds[64 * WMAX * WMAX];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int nwaves = blockDim.x >> 6;
    if (tid == 0) bad = 0;
    __syncthreads();

    // Wave v packs row groups v, v + nwaves, ... of G rows: lane l loads byte
    // 64*w + l of the G rows at once (independent loads), then one ballot per
    // row gives the packed word.
    constexpr int G = 16;
    int mybad = 0;
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
    __syncthreads();

    const int i = tid;
    uint64_t row[WMAX];
#pragma unroll
    for (int w = 0; w < WMAX; ++w) row[w] = (i < n && w < W) ? lds[i * W + w] : 0ull;
#pragma unroll
    for (int cw = 0; cw < WMAX; ++cw) {
        if (cw >= W) break;
        for (int cb = 0; cb < 64; ++cb) {
            const int c = 64 * cw + cb;
            if (c >= n) break;
            const uint64_t col = __ballot((row[cw] >> cb) & 1ull);
            if (col != lds[c * W + wave]) mybad = 1;
        }
    }
    if (mybad) bad = 1;
    __syncthreads();
    for (int idx = tid; idx < n * W; idx += blockDim.x) rows[idx] = lds[idx];
    if (tid == 0) *status = bad ? HLF_ENOTSYM : HLF_OK;
}

template <int WMAX>
__global__ __launch_bounds__(64) void factor_wave_kernel(const uint64_t *__restrict__ rows, int n,
                                                         int W, FactorOut out) {
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
                                                                int n, int W, FactorOut out) {
    __shared__ uint64_t mat[64 * WMAX * WMAX];
    __shared__ int piv[64 * WMAX];
    __shared__ int freec[64 * WMAX];
    __shared__ int qacc[64 * WMAX];
    __shared__ int cand[3];
    __shared__ unsigned long long shiftw[WMAX];
    __shared__ int flag_bad, flag_internal;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nthr = blockDim.x;

    // During validation and elimination `mat` is word-major (word w of row i
    // at w*NP + i), so the 64 lanes of a wave store to consecutive addresses;
    // afterwards it is reused row-major for the RREF and the kernel vectors.
    constexpr int NP = 64 * WMAX;
    uint64_t row[WMAX];
#pragma unroll
    for (int w = 0; w < WMAX; ++w) {
        row[w] = (tid < n && w < W) ? rows[tid * W + w] : 0ull;
        if (tid < n && w < W) mat[w * NP + tid] = row[w];
    }
    if (tid < WMAX) shiftw[tid] = 0;
    if (tid < 3) cand[tid] = INT_MAX;
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
#pragma unroll
    for (int cw = 0; cw < WMAX; ++cw) {
        if (cw >= W) break;
        for (int cb = 0; cb < 64; ++cb) {
            const int c = 64 * cw + cb;
            if (c >= n) break;
            const uint64_t col = __ballot((row[cw] >> cb) & 1ull);
            if (col != mat[wave * NP + c]) bad = true;
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

    // Gauss-Jordan with one barrier per column.  `mat` holds every current row
    // (word-major, kept equal to thread i's registers).  Phase c: every
    // thread reads the pivot p of column c chosen before the barrier, XORs row
    // p (read from LDS) into its own row if it has bit c, stores its row back,
    // and offers itself as a candidate for column c+1 (atomicMin over
    // per-wave ballots).  Row p is not written in phase c, so all reads of it
    // see one value; a candidate slot is reset two columns before its reuse,
    // after every thread has read it.
    int r = 0, nfree = 0, slot = 0;
    bool used = false;
    int myk = -1;
    {
        const uint64_t m = __ballot(tid < n && (row[0] & 1ull));
        if (lane == 0 && m) atomicMin(&cand[0], wave * 64 + __builtin_ctzll(m));
    }
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        const int p = cand[slot];
        if (tid == 0) cand[slot == 0 ? 2 : slot - 1] = INT_MAX;
        const int cw = c >> 6, cb = c & 63;
        if (p != INT_MAX) {
            uint64_t word = 0;
#pragma unroll
            for (int w = 0; w < WMAX; ++w)
                if (w == cw) word = row[w];
            if (tid == p) {
                used = true;
                myk = r;
            }
            if (tid == 0) piv[r] = c;
            if (((word >> cb) & 1ull) && tid != p) {
#pragma unroll
                for (int w = 0; w < WMAX; ++w)
                    if (w < W) {
                        row[w] ^= mat[w * NP + p];
                        mat[w * NP + tid] = row[w];
                    }
            }
            ++r;
        } else {
            if (tid == 0) freec[nfree] = c;
            ++nfree;
        }
        const int nslot = (slot == 2) ? 0 : slot + 1;
        if (c + 1 < n) {
            const int c1 = c + 1;
            uint64_t word1 = 0;
#pragma unroll
            for (int w = 0; w < WMAX; ++w)
                if (w == (c1 >> 6)) word1 = row[w];
            const uint64_t m = __ballot(tid < n && !used && ((word1 >> (c1 & 63)) & 1ull));
            if (lane == 0 && m) atomicMin(&cand[nslot], wave * 64 + __builtin_ctzll(m));
        }
        slot = nslot;
        __syncthreads();
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
    for (int idx = tid; idx < r * W; idx += nthr) {
        const int k = idx / W, w = idx - k * W;
        out.basis[idx] = rows[piv[k] * W + w];
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
hlf_status launch_wave_t(const uint64_t *rows, int n, int W, const FactorOut &out,
                         hipStream_t stream) {
    hipLaunchKernelGGL(factor_wave_kernel<WMAX>, dim3(1), dim3(64), 0, stream, rows, n, W, out);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int WMAX>
hlf_status launch_workgroup_t(const uint64_t *rows, int n, int W, const FactorOut &out,
                              hipStream_t stream) {
    hipLaunchKernelGGL(factor_workgroup_kernel<WMAX>, dim3(1), dim3(64 * W), 0, stream, rows, n,
                       W, out);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

}  // namespace

hlf_status launch_pack(const uint8_t *A, int n, int W, uint64_t *rows, int32_t *status,
                       hipStream_t stream) {
    if (W <= 1) return launch_pack_t<1>(A, n, W, rows, status, stream);
    if (W <= 2) return launch_pack_t<2>(A, n, W, rows, status, stream);
    if (W <= 3) return launch_pack_t<3>(A, n, W, rows, status, stream);
    if (W <= 4) return launch_pack_t<4>(A, n, W, rows, status, stream);
    if (W <= 8) return launch_pack_t<8>(A, n, W, rows, status, stream);
    return launch_pack_t<16>(A, n, W, rows, status, stream);
}

hlf_status launch_factor(const uint64_t *rows, int n, int W, const FactorOut &out,
                         bool force_workgroup, hipStream_t stream) {
    if (!force_workgroup) {
        if (W == 1) return launch_wave_t<1>(rows, n, W, out, stream);
        if (W == 2) return launch_wave_t<2>(rows, n, W, out, stream);
        if (W == 3) return launch_wave_t<3>(rows, n, W, out, stream);
    }
    if (W <= 1) return launch_workgroup_t<1>(rows, n, W, out, stream);
    if (W <= 2) return launch_workgroup_t<2>(rows, n, W, out, stream);
    if (W <= 4) return launch_workgroup_t<4>(rows, n, W, out, stream);
    if (W <= 8) return launch_workgroup_t<8>(rows, n, W, out, stream);
    return launch_workgroup_t<16>(rows, n, W, out, stream);
}

}  // namespace hlf
