// Stage 1 and stage 2 of one small instance in ONE launch (n <= 64): every
// workgroup packs and validates A and factors it on its first wave (the
// paper's Section 2 tasks (1)-(4): a few microseconds of one wave at this
// size), then materialises its own tiles of [begin, begin + count) (Eq. (3)
// and the final CNOT layer, as in stage2.h).  Workgroup 0 writes the caller's
// record; every other workgroup writes a private copy in LDS, so the record
// has a single writer and a range error cannot race with another
// workgroup's verdict.  The redundant factorisations run side by side and no
// workgroup waits for another: this is the latency path for small instances.
#include "factor_wave.h"
#include "hlf_device.h"
#include "hlf_internal.h"
#include "stage2.h"

namespace hlf {
namespace {

template <typename T>
__global__ __launch_bounds__(kTileThreads) void solve_dense_kernel(const uint8_t *__restrict__ A,
                                                                   int n, FactorOut rec,
                                                                   uint64_t begin, uint64_t count,
                                                                   T *__restrict__ out,
                                                                   uint64_t tiles_per_block) {
    constexpr int S = tile_shift<T>();
    __shared__ WaveSmem<1> sm;
    __shared__ uint64_t Bx[64];
    __shared__ int32_t own_status, own_rank, own_piv[64];
    __shared__ uint64_t own_basis[64], own_shift[1];
    __shared__ int go;
    if (threadIdx.x < 64) {
        FactorOut o = rec;
        if (blockIdx.x != 0) {  // generic pointers into this workgroup's LDS
            o.status = &own_status;
            o.rank = &own_rank;
            o.pivots = own_piv;
            o.basis = own_basis;
            o.shift = own_shift;
            o.kernel = nullptr;
        }
        const bool badv = wave_load_dense<1>(A, n, 1, sm);
        const int r = factor_wave_core<1>(n, 1, badv, o, sm);  // -1: invalid matrix
        const bool ok = r >= 0 && r <= HLF_MAX_ENUM_RANK && begin <= (1ull << r) &&
                        count <= (1ull << r) - begin;
        // After this lane's own status write in factor_wave_core.
        if (r >= 0 && !ok && blockIdx.x == 0 && threadIdx.x == 0) *rec.status = HLF_ERANGE;
        if (ok) Bx[threadIdx.x] = ((int)threadIdx.x < r) ? sm.orig[sm.piv[threadIdx.x]] : 0ull;
        if (threadIdx.x == 0) go = (ok && count > 0) ? 1 : 0;
    }
    __syncthreads();
    if (!go) return;
    const uint64_t end = begin + count;
    const uint64_t ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    const uint64_t t0 = (uint64_t)blockIdx.x * tiles_per_block;
    if (t0 >= ntiles) return;
    const uint64_t t1 = (t0 + tiles_per_block < ntiles) ? t0 + tiles_per_block : ntiles;
    enum_tiles_w1<T>(Bx, sm.shiftw[0], begin, count, out, t0, t1);
}

template <typename T>
hlf_status launch_solve_dense_t(const uint8_t *A, int n, const FactorOut &rec, uint64_t begin,
                                uint64_t count, T *out, hipStream_t stream) {
    constexpr int S = tile_shift<T>();
    const uint64_t end = begin + count;
    uint64_t ntiles = 1;  // count = 0 or a wrapping range: one workgroup (stage 1 only)
    if (count > 0 && end > begin) ntiles = ((end - 1) >> S) - (begin >> S) + 1;
    const uint64_t tpb = materialise_tiles_per_block(ntiles, kTileBytes);
    const uint64_t blocks = (ntiles + tpb - 1) / tpb;
    hipLaunchKernelGGL(solve_dense_kernel<T>, dim3((unsigned)blocks), dim3(kTileThreads), 0, stream,
                       A, n, rec, begin, count, out, tpb);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

}  // namespace

hlf_status launch_solve_dense(const uint8_t *A, int n, const FactorOut &rec, uint64_t begin,
                              uint64_t count, int word_bits, void *out, hipStream_t stream) {
    if (word_bits == 16)
        return launch_solve_dense_t<uint16_t>(A, n, rec, begin, count, (uint16_t *)out, stream);
    if (word_bits == 32)
        return launch_solve_dense_t<uint32_t>(A, n, rec, begin, count, (uint32_t *)out, stream);
    return launch_solve_dense_t<uint64_t>(A, n, rec, begin, count, (uint64_t *)out, stream);
}

}  // namespace hlf
