// Host-side internal interface between the C ABI (hlf_abi.cpp) and the
// kernel launchers (one per .hip file).
#pragma once

#include <stdint.h>

#include "hlf.h"

namespace hlf {

// Output pointers of one factor record.
struct FactorOut {
    int32_t *status;
    int32_t *rank;
    int32_t *pivots;
    uint64_t *basis;
    uint64_t *shift;
    uint64_t *kernel;  // may be null
};

// Read-only view of a factor record for the stage-2 kernels.
struct FactorIn {
    int32_t n;
    int32_t words;
    int32_t *status;        // read, and set to HLF_ERANGE on a bad range
    const int32_t *rank;
    const uint64_t *basis;
    const uint64_t *shift;
};

int device_cu_count();

hlf_status launch_pack(const uint8_t *A, int n, int W, uint64_t *rows, int32_t *status,
                       hipStream_t stream);
// Pack + factor + materialise of one instance with n <= 64 in one launch
// (word_bits 16/32/64 >= n, begin a multiple of the 16-byte vector, out
// 16-byte aligned).
hlf_status launch_solve_dense(const uint8_t *A, int n, const FactorOut &rec, uint64_t begin,
                              uint64_t count, int word_bits, void *out, hipStream_t stream);
hlf_status launch_factor(const uint64_t *rows, int n, int W, const FactorOut &out,
                         bool force_workgroup, bool keep_pack_status, hipStream_t stream);
hlf_status launch_enumerate(const FactorIn &f, uint64_t begin, uint64_t count, int word_bits,
                            bool counter_order, void *out, hipStream_t stream);
// Gray order.
inline hlf_status launch_enumerate(const FactorIn &f, uint64_t begin, uint64_t count,
                                   int word_bits, void *out, hipStream_t stream) {
    return launch_enumerate(f, begin, count, word_bits, false, out, stream);
}
hlf_status launch_pair_stats(const FactorIn &f, const uint64_t *rows, uint8_t *quarters,
                             hipStream_t stream);
hlf_status launch_membership(const FactorIn &f, const uint64_t *kernel, const uint64_t *z,
                             uint64_t num, uint8_t *member, hipStream_t stream);
hlf_status launch_circuit(const FactorIn &f, const int32_t *pivots, const uint64_t *rows, int N,
                          uint64_t begin, uint64_t count, int word_bits, void *out,
                          hipStream_t stream);
hlf_status launch_reduce(const FactorIn &f, uint64_t begin, uint64_t count, bool accumulate,
                         uint64_t *counts, uint64_t *hash, uint64_t *xorfold,
                         hipStream_t stream);
hlf_status launch_sample(const FactorIn &f, uint64_t seed, uint64_t num, const uint64_t *coeffs,
                         uint64_t *out, hipStream_t stream);

}  // namespace hlf
