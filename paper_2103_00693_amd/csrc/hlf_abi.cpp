// extern "C" entry points of libhlf.so: argument validation (host-detectable
// errors return before anything is enqueued) and dispatch to the launchers.
#include <hip/hip_runtime.h>

#include <atomic>

#include "hlf.h"
#include "hlf_internal.h"

namespace hlf {

int device_cu_count() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cu <= 0)
            cu = 256;
        cache[dev].store(cu, std::memory_order_relaxed);
        v = cu;
    }
    return v;
}

}  // namespace hlf

namespace {

bool record_ok(const hlf_factors *f) {
    if (!f) return false;
    if (f->n < 1 || f->n > HLF_MAX_N) return false;
    if (f->words != hlf_words_for(f->n)) return false;
    if (!f->status || !f->rank || !f->pivots || !f->basis || !f->shift) return false;
    return true;
}

hlf::FactorIn view(const hlf_factors *f) {
    hlf::FactorIn in;
    in.n = f->n;
    in.words = f->words;
    in.status = f->status;
    in.rank = f->rank;
    in.basis = f->basis;
    in.shift = f->shift;
    return in;
}

}  // namespace

extern "C" {

int32_t hlf_version(void) { return (1 << 16) | 0; }

const char *hlf_status_string(int32_t status) {
    switch (status) {
        case HLF_OK: return "HLF_OK";
        case HLF_EINVAL: return "HLF_EINVAL: invalid argument";
        case HLF_ENOTSYM: return "HLF_ENOTSYM: matrix is not a symmetric 0/1 matrix";
        case HLF_ERANGE: return "HLF_ERANGE: index range outside [0, 2^r) or r > 62";
        case HLF_ENOMEM: return "HLF_ENOMEM: capacity exceeded";
        case HLF_EDEVICE: return "HLF_EDEVICE: HIP launch failed";
        case HLF_EINTERNAL: return "HLF_EINTERNAL: internal invariant failed";
        default: return "unknown hlf_status";
    }
}

int32_t hlf_words_for(int32_t n) { return n <= 0 ? 0 : (n + 63) / 64; }

hlf_status hlf_pack_dense(const uint8_t *A_dev, int32_t n, uint64_t *rows_dev,
                          int32_t *status_dev, hipStream_t stream) {
    if (!A_dev || !rows_dev || !status_dev) return HLF_EINVAL;
    if (n < 1 || n > HLF_MAX_N) return HLF_EINVAL;
    return hlf::launch_pack(A_dev, n, hlf_words_for(n), rows_dev, status_dev, stream);
}

hlf_status hlf_factor_ex(const uint64_t *rows_dev, const hlf_factors *f, uint32_t flags,
                         hipStream_t stream) {
    if (!rows_dev || !record_ok(f)) return HLF_EINVAL;
    if (flags & ~(HLF_FACTOR_WORKGROUP | HLF_FACTOR_PACK_STATUS)) return HLF_EINVAL;
    hlf::FactorOut out;
    out.status = f->status;
    out.rank = f->rank;
    out.pivots = f->pivots;
    out.basis = f->basis;
    out.shift = f->shift;
    out.kernel = f->kernel;
    return hlf::launch_factor(rows_dev, f->n, f->words, out, (flags & HLF_FACTOR_WORKGROUP) != 0,
                              (flags & HLF_FACTOR_PACK_STATUS) != 0, stream);
}

hlf_status hlf_factor(const uint64_t *rows_dev, const hlf_factors *f, hipStream_t stream) {
    return hlf_factor_ex(rows_dev, f, 0u, stream);
}

hlf_status hlf_enumerate(const hlf_factors *f, uint64_t begin, uint64_t count, int32_t word_bits,
                         void *out_dev, hipStream_t stream) {
    return hlf_enumerate_ex(f, begin, count, word_bits, 0u, out_dev, stream);
}

hlf_status hlf_enumerate_ex(const hlf_factors *f, uint64_t begin, uint64_t count,
                            int32_t word_bits, uint32_t flags, void *out_dev, hipStream_t stream) {
    if (!record_ok(f)) return HLF_EINVAL;
    if (flags & ~HLF_ORDER_COUNTER) return HLF_EINVAL;
    const int W = f->words;
    const bool narrow = (word_bits == 16 || word_bits == 32 || word_bits == 64) &&
                        f->n <= word_bits;
    const bool wide = word_bits == 64 * W;
    if (!narrow && !wide) return HLF_EINVAL;
    if (count == 0) return HLF_OK;
    if (!out_dev) return HLF_EINVAL;
    return hlf::launch_enumerate(view(f), begin, count, word_bits, (flags & HLF_ORDER_COUNTER) != 0,
                                 out_dev, stream);
}

hlf_status hlf_solve_dense(const uint8_t *A_dev, const hlf_factors *f, uint64_t begin,
                           uint64_t count, int32_t word_bits, void *out_dev, hipStream_t stream) {
    if (!A_dev || !record_ok(f)) return HLF_EINVAL;
    if (f->words != 1) return HLF_EINVAL;  // n <= 64
    if ((word_bits != 16 && word_bits != 32 && word_bits != 64) || f->n > word_bits)
        return HLF_EINVAL;
    const uint64_t V = 16 / (uint64_t)(word_bits / 8);
    if (count > 0 && (!out_dev || ((uintptr_t)out_dev & 15u) != 0 || begin % V != 0))
        return HLF_EINVAL;
    hlf::FactorOut out;
    out.status = f->status;
    out.rank = f->rank;
    out.pivots = f->pivots;
    out.basis = f->basis;
    out.shift = f->shift;
    out.kernel = f->kernel;
    return hlf::launch_solve_dense(A_dev, f->n, out, begin, count, word_bits, out_dev, stream);
}

hlf_status hlf_enumerate_circuit(const hlf_factors *f, const uint64_t *rows_dev, int32_t grid_N,
                                 uint64_t begin, uint64_t count, int32_t word_bits, void *out_dev,
                                 hipStream_t stream) {
    if (!record_ok(f) || !rows_dev) return HLF_EINVAL;
    if (grid_N < 1 || grid_N * grid_N != f->n) return HLF_EINVAL;
    if (f->words == 1) {
        if ((word_bits != 16 && word_bits != 32 && word_bits != 64) || f->n > word_bits)
            return HLF_EINVAL;
    } else if (word_bits != 64 * f->words) {
        return HLF_EINVAL;
    }
    if (count == 0) return HLF_OK;
    if (!out_dev) return HLF_EINVAL;
    if (f->words == 1) {
        const uint64_t V = 16 / (uint64_t)(word_bits / 8);
        if (((uintptr_t)out_dev & 15u) != 0 || begin % V != 0) return HLF_EINVAL;
    } else if (((uintptr_t)out_dev & 7u) != 0) {
        return HLF_EINVAL;
    }
    return hlf::launch_circuit(view(f), f->pivots, rows_dev, grid_N, begin, count, word_bits,
                               out_dev, stream);
}

hlf_status hlf_enumerate_reduce(const hlf_factors *f, uint64_t begin, uint64_t count,
                                uint32_t flags, uint64_t *counts_dev, uint64_t *hash_dev,
                                uint64_t *xorfold_dev, hipStream_t stream) {
    if (!record_ok(f) || !counts_dev || !hash_dev) return HLF_EINVAL;
    if (flags & ~HLF_ACCUMULATE) return HLF_EINVAL;
    return hlf::launch_reduce(view(f), begin, count, (flags & HLF_ACCUMULATE) != 0, counts_dev,
                              hash_dev, xorfold_dev, stream);
}

hlf_status hlf_sample(const hlf_factors *f, uint64_t seed, uint64_t num,
                      const uint64_t *coeffs_dev, uint64_t *out_dev, hipStream_t stream) {
    if (!record_ok(f)) return HLF_EINVAL;
    if (num == 0) return HLF_OK;
    if (!out_dev) return HLF_EINVAL;
    return hlf::launch_sample(view(f), seed, num, coeffs_dev, out_dev, stream);
}

hlf_status hlf_pair_stats(const hlf_factors *f, const uint64_t *rows_dev, uint8_t *quarters_dev,
                          hipStream_t stream) {
    if (!record_ok(f) || !rows_dev || !quarters_dev) return HLF_EINVAL;
    return hlf::launch_pair_stats(view(f), rows_dev, quarters_dev, stream);
}

hlf_status hlf_membership(const hlf_factors *f, const uint64_t *z_dev, uint64_t num,
                          uint8_t *member_dev, hipStream_t stream) {
    if (!record_ok(f) || !f->kernel) return HLF_EINVAL;
    if (num == 0) return HLF_OK;
    if (!z_dev || !member_dev) return HLF_EINVAL;
    return hlf::launch_membership(view(f), f->kernel, z_dev, num, member_dev, stream);
}

}  // extern "C"
