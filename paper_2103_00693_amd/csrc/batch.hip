// Batches of instances on gfx950: the whole FS2D pipeline (Sections 1-2) for
// many grid instances of mixed size with one launch per stage.
//
//   batch_factor_kernel<WMAX>   pack + validate + factor, one wavefront (a
//                               64-thread workgroup) per instance, n <= 64*WMAX.
//   batch_enum_kernel<T>        materialise for up to kMaxEnumTasks instances
//                               in one launch; each workgroup takes a short
//                               contiguous tile range of one instance.
//   batch_reduce_kernel<WMAX>   persistent: each wavefront first takes factor
//                               tasks from a device counter; an instance with
//                               r <= max_rank then claims a contiguous block of
//                               chunk indices with ONE 64-bit atomic that returns
//                               both its slot and its first chunk, writes the
//                               slot and releases it; wavefronts then take chunk
//                               indices from a second counter and find the slot
//                               by binary search.  A wave only waits for a slot
//                               that was already claimed (its writer is running)
//                               or for factor tasks that running waves hold, so
//                               every wait ends and the grid drains.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "factor_wave.h"
#include "hlf.h"
#include "hlf_device.h"
#include "hlf_internal.h"
#include "stage2.h"

namespace hlf {
namespace {

struct BatchDev {
    int32_t count;
    const int32_t *n;
    const int64_t *dense_off;
    const int64_t *mat_off;
    const int64_t *vec_off;
    const int64_t *piv_off;
    const int32_t *order;  // instance ids grouped by word count
    int32_t *status;
    int32_t *rank;
    int32_t *pivots;
    uint64_t *basis;
    uint64_t *shift;
    uint64_t *kernel;
    uint64_t *counts;
    uint64_t *hash;
};

__device__ __forceinline__ FactorOut record_of(const BatchDev &b, int i) {
    FactorOut out;
    out.status = &b.status[i];
    out.rank = &b.rank[i];
    out.pivots = b.pivots + b.piv_off[i];
    out.basis = b.basis + b.mat_off[i];
    out.shift = b.shift + b.vec_off[i];
    out.kernel = b.kernel ? b.kernel + b.mat_off[i] : nullptr;
    return out;
}

// ---------------------------------------------------------------------------
// Stage 1 for the instances order[first .. first + gridDim.x).
// ---------------------------------------------------------------------------
template <int WMAX>
__global__ __launch_bounds__(64) void batch_factor_kernel(BatchDev b, const uint8_t *__restrict__ A,
                                                          int first) {
    __shared__ WaveSmem<WMAX> sm;
    const int i = b.order[first + blockIdx.x];
    const int n = b.n[i];
    const int W = (n + 63) >> 6;
    const bool badv = wave_load_dense<WMAX>(A + b.dense_off[i], n, W, sm);
    factor_wave_core<WMAX>(n, W, badv, record_of(b, i), sm);
}

// A failed pack (an entry other than 0/1) overrides the factor's verdict.
__global__ void merge_pack_status_kernel(int32_t *status, const int32_t *pack_status) {
    if (threadIdx.x == 0 && *pack_status != HLF_OK) *status = *pack_status;
}

// ---------------------------------------------------------------------------
// Materialise for several instances.
// ---------------------------------------------------------------------------
constexpr int kMaxEnumTasks = 16;

struct EnumTask {
    int32_t *status;
    const int32_t *rank;
    const uint64_t *basis;
    const uint64_t *shift;
    void *out;
    uint64_t begin;
    uint64_t count;
    uint32_t block0;           // first block of this task
    uint32_t tiles_per_block;
};

struct EnumTasks {
    EnumTask t[kMaxEnumTasks];
    int32_t num;
};

// Optional stage-1 work carried by a materialise launch: the first `blocks`
// workgroups factor instances order[first .. first + num) of another batch,
// one instance per wavefront (W = 1).  The records it writes are not read by
// the same launch, so there is no dependency inside the launch.
struct FactorJob {
    BatchDev d;
    const uint8_t *A;
    int32_t first;
    int32_t num;
    uint32_t blocks;
};

constexpr int kWavesPerTileBlock = kTileThreads / 64;

template <typename T, bool kFactor>
__global__ __launch_bounds__(kTileThreads, 8) void batch_enum_kernel(EnumTasks tasks, FactorJob job) {
    constexpr int S = tile_shift<T>();
    __shared__ uint64_t Bx[64];
    unsigned int bid = blockIdx.x;
    if constexpr (kFactor) {
        __shared__ WaveSmem<1> sm[kWavesPerTileBlock];
        if (bid < job.blocks) {
            const int w = threadIdx.x >> 6;
            const int idx = (int)bid * kWavesPerTileBlock + w;
            if (idx < job.num) {
                const int i = job.d.order[job.first + idx];
                const int n = job.d.n[i];
                const bool badv = wave_load_dense<1>(job.A + job.d.dense_off[i], n, 1, sm[w]);
                factor_wave_core<1>(n, 1, badv, record_of(job.d, i), sm[w]);
            }
            return;
        }
        bid -= job.blocks;
    }
    bid = xcd_block(bid, gridDim.x - (kFactor ? job.blocks : 0u));
    int k = 0;
    for (int j = 1; j < tasks.num; ++j)
        if (tasks.t[j].block0 <= bid) k = j;
    const EnumTask &t = tasks.t[k];
    int r;
    if (!gate(t.status, t.rank, t.begin, t.count, r)) return;
    load_basis_padded<1>(t.basis, r, Bx, threadIdx.x, blockDim.x);
    __syncthreads();
    const uint64_t end = t.begin + t.count;
    const uint64_t ntiles = ((end - 1) >> S) - (t.begin >> S) + 1;
    const uint64_t t0 = (uint64_t)(bid - t.block0) * t.tiles_per_block;
    if (t0 >= ntiles) return;
    const uint64_t t1 = (t0 + t.tiles_per_block < ntiles) ? t0 + t.tiles_per_block : ntiles;
    enum_tiles_w1<T>(Bx, t.shift[0], t.begin, t.count, (T *)t.out, t0, t1);
}

// ---------------------------------------------------------------------------
// Stage 1 + stage 2 materialise in one launch (instances with n <= 64).
// The first workgroup of an instance to start claims its factorisation with a
// CAS on flags[inst] (0 idle, 1 claimed, 2 done) and runs it on its first wave;
// the instance's other workgroups wait for 2 -- a claim is only ever held by a
// running workgroup, so every wait ends.  The last workgroup to finish resets
// the flags of the launch, so each launch starts from idle flags.  Every
// workgroup reaches the final counter (no early return).
// ---------------------------------------------------------------------------
struct SolveTasks {
    EnumTask t[kMaxEnumTasks];
    int32_t inst[kMaxEnumTasks];
    int32_t num;
};

template <typename T>
__global__ __launch_bounds__(kTileThreads) void batch_solve_kernel(BatchDev b,
                                                                   const uint8_t *__restrict__ A,
                                                                   SolveTasks tasks, int32_t *flags,
                                                                   unsigned int *blocks_done) {
    constexpr int S = tile_shift<T>();
    __shared__ WaveSmem<1> sm;
    __shared__ uint64_t Bx[64];
    __shared__ int role;
    __shared__ int ok;
    __shared__ int rank_s;
    const int tid = threadIdx.x;
    int k = 0;
    for (int j = 1; j < tasks.num; ++j)
        if (tasks.t[j].block0 <= blockIdx.x) k = j;
    const EnumTask &t = tasks.t[k];
    const int i = tasks.inst[k];

    // Agent-scope acquire/release fences invalidate / write back the XCD's L2,
    // so the claim and the wait use relaxed atomics and each workgroup takes
    // exactly one acquire (thread 0) after it has seen the flag at 2.
    if (tid == 0) {
        int mine = 0;
        if (__hip_atomic_load(&flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            int expected = 0;
            mine = __hip_atomic_compare_exchange_strong(&flags[i], &expected, 1, __ATOMIC_RELAXED,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       ? 1 : 0;
        }
        role = mine;
    }
    __syncthreads();
    if (role) {
        if (tid < 64) {
            const int n = b.n[i];
            const bool badv = wave_load_dense<1>(A + b.dense_off[i], n, 1, sm);
            factor_wave_core<1>(n, 1, badv, record_of(b, i), sm);
            if (tid == 0) __hip_atomic_store(&flags[i], 2, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (tid == 0) {
        while (__hip_atomic_load(&flags[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 2)
            __builtin_amdgcn_s_sleep(8);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (tid == 0) {
        int r = 0;
        ok = gate(t.status, t.rank, t.begin, t.count, r) ? 1 : 0;
        rank_s = r;
    }
    __syncthreads();
    if (ok) {
        load_basis_padded<1>(t.basis, rank_s, Bx, tid, blockDim.x);
        __syncthreads();
        const uint64_t end = t.begin + t.count;
        const uint64_t ntiles = ((end - 1) >> S) - (t.begin >> S) + 1;
        const uint64_t t0 = (uint64_t)(blockIdx.x - t.block0) * t.tiles_per_block;
        if (t0 < ntiles) {
            const uint64_t t1 = (t0 + t.tiles_per_block < ntiles) ? t0 + t.tiles_per_block : ntiles;
            enum_tiles_w1<T>(Bx, t.shift[0], t.begin, t.count, (T *)t.out, t0, t1);
        }
    }
    __syncthreads();
    // Thread 0's flag accesses have all returned before its increment is
    // issued, so the last workgroup can reset the flags; the end of the kernel
    // makes the reset visible to the next launch.
    if (tid == 0) {
        const unsigned int prev =
            __hip_atomic_fetch_add(blocks_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            for (int j = 0; j < tasks.num; ++j)
                __hip_atomic_store(&flags[tasks.inst[j]], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(blocks_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent factor + reduce.
// ---------------------------------------------------------------------------
constexpr int kClaimShift = 40;  // claim word: (slots << 40) | chunks
constexpr unsigned long long kChunkMask = (1ull << kClaimShift) - 1;

struct QueueHead {
    unsigned int fnext;        // next factor task
    unsigned int fdone;        // factor tasks finished
    unsigned long long cnext;  // next chunk index
    unsigned long long claim;  // published slots and chunks
};

struct ChunkSlot {
    unsigned long long base;  // first chunk index of the instance
    int inst;
    int ready;
};

__global__ void batch_queue_reset_kernel(QueueHead *q, ChunkSlot *slots, int count) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        q->fnext = 0;
        q->fdone = 0;
        q->cnext = 0;
        q->claim = 0;
    }
    if (t < count) {
        slots[t].base = 0;
        slots[t].inst = 0;
        slots[t].ready = 0;
    }
}

// Offsets of the batch layout (prefix sums over the instance sizes) for the
// allocation-free reduce: one workgroup of 1024 threads, count <= 1024 * kPer.
// An n outside [1, max_n] counts as 0 (no space; its factor task reports
// HLF_EINVAL).  n_eff receives the sizes the other kernels use.
constexpr int kLayoutPer = 16;

__global__ __launch_bounds__(1024) void noalloc_layout_kernel(const int32_t *__restrict__ n_in,
                                                              int count, int max_n, int32_t *n_eff,
                                                              int64_t *dense_off, int64_t *mat_off,
                                                              int64_t *vec_off, int64_t *piv_off) {
    __shared__ int64_t part[4][1024];
    const int t = threadIdx.x;
    const int i0 = t * kLayoutPer;
    int64_t loc[4] = {0, 0, 0, 0};
    for (int i = i0; i < min(count, i0 + kLayoutPer); ++i) {
        const int n = n_in[i];
        const int64_t ne = (n >= 1 && n <= max_n) ? n : 0;
        const int64_t W = (ne + 63) >> 6;
        loc[0] += ne * ne;
        loc[1] += ne * W;
        loc[2] += W;
        loc[3] += ne;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) part[q][t] = loc[q];
    __syncthreads();
    // inclusive scan over the 1024 partial sums (Hillis-Steele)
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = t >= d ? part[q][t - d] : 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) part[q][t] += v[q];
        __syncthreads();
    }
    int64_t run[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) run[q] = part[q][t] - loc[q];  // exclusive
    for (int i = i0; i < min(count, i0 + kLayoutPer); ++i) {
        const int n = n_in[i];
        const int64_t ne = (n >= 1 && n <= max_n) ? n : 0;
        const int64_t W = (ne + 63) >> 6;
        n_eff[i] = (int32_t)ne;
        dense_off[i] = run[0];
        mat_off[i] = run[1];
        vec_off[i] = run[2];
        piv_off[i] = run[3];
        run[0] += ne * ne;
        run[1] += ne * W;
        run[2] += W;
        run[3] += ne;
    }
}

__device__ __forceinline__ unsigned long long slot_base(ChunkSlot *slots, int s) {
    while (__builtin_amdgcn_readfirstlane(
               __hip_atomic_load(&slots[s].ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) == 0)
        __builtin_amdgcn_s_sleep(2);
    return uniform64(__hip_atomic_load(&slots[s].base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Last slot whose first chunk is <= c (slot bases increase with the slot).
__device__ int find_slot(ChunkSlot *slots, int nslots, unsigned long long c) {
    int lo = 0, hi = nslots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (slot_base(slots, mid) <= c) lo = mid; else hi = mid - 1;
    }
    (void)slot_base(slots, lo);
    return lo;
}

template <int WW, int WMAX>
__device__ void reduce_chunk(const BatchDev &b, int inst, int n, int r, unsigned long long c0,
                             unsigned long long c1, uint64_t *Bx) {
    const int lane = lane_id();
    load_basis_padded<WW>(b.basis + b.mat_off[inst], r, Bx, lane, 64);
    uint64_t l[WW];
    const uint64_t *sh = b.shift + b.vec_off[inst];
#pragma unroll
    for (int w = 0; w < WW; ++w) l[w] = sh[w];
    __syncthreads();
    const WavePartial<WW> p = wave_reduce_range<WW>(Bx, l, n, r, c0, c1);
    uint64_t *cnt = b.counts + b.piv_off[inst];
#pragma unroll
    for (int w = 0; w < WW; ++w) {
        const int j = 64 * w + lane;
        if (j < n && p.cnt[w]) atomicAdd((unsigned long long *)&cnt[j], (unsigned long long)p.cnt[w]);
    }
    if (lane == 0 && p.hash) atomicAdd((unsigned long long *)&b.hash[inst], (unsigned long long)p.hash);
    __syncthreads();  // Bx is reused by the next chunk
}

template <int WMAX>
__global__ __launch_bounds__(64) void batch_reduce_kernel(BatchDev b, const uint8_t *__restrict__ A,
                                                          int max_rank, int chunk_log2,
                                                          QueueHead *q, ChunkSlot *slots) {
    __shared__ WaveSmem<WMAX> sm;
    __shared__ uint64_t Bx[64 * WMAX];
    const int lane = lane_id();

    // Phase 1: factor tasks.
    for (;;) {
        unsigned int f = 0;
        if (lane == 0) f = atomicAdd(&q->fnext, 1u);
        f = (unsigned int)__builtin_amdgcn_readfirstlane((int)f);
        if (f >= (unsigned int)b.count) break;
        const int n = b.n[f];
        const int W = (n + 63) >> 6;
        const FactorOut out = record_of(b, (int)f);
        int r = -1;
        if (n >= 1 && W <= WMAX) {
            const bool badv = wave_load_dense<WMAX>(A + b.dense_off[f], n, W, sm);
            r = factor_wave_core<WMAX>(n, W, badv, out, sm);
        } else if (lane == 0) {
            *out.rank = 0;
            *out.status = HLF_EINVAL;
        }
        uint64_t *cnt = b.counts + b.piv_off[f];
        for (int j = lane; j < n; j += 64) cnt[j] = 0;
        if (lane == 0) b.hash[f] = 0;
        __threadfence();  // the record and the zeroed results precede publication
        if (lane == 0) {
            if (r >= 0 && r <= max_rank) {
                const unsigned long long nch =
                    (r > chunk_log2) ? (1ull << (r - chunk_log2)) : 1ull;
                const unsigned long long old =
                    atomicAdd(&q->claim, (1ull << kClaimShift) | nch);
                const int s = (int)(old >> kClaimShift);
                slots[s].base = old & kChunkMask;
                slots[s].inst = (int)f;
                __hip_atomic_store(&slots[s].ready, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            __hip_atomic_fetch_add(&q->fdone, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();  // LDS is reused by the next factor task
    }

    // Phase 2: chunk tasks.
    for (;;) {
        unsigned long long c = 0;
        if (lane == 0) c = atomicAdd(&q->cnext, 1ull);
        c = uniform64(c);
        int s = -1;
        for (;;) {
            const unsigned long long cl = uniform64(
                __hip_atomic_load(&q->claim, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
            if (c < (cl & kChunkMask)) {
                s = find_slot(slots, (int)(cl >> kClaimShift), c);
                break;
            }
            const unsigned int done = (unsigned int)__builtin_amdgcn_readfirstlane((int)
                __hip_atomic_load(&q->fdone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
            if (done >= (unsigned int)b.count) {
                // every claim happened before its fdone increment
                const unsigned long long cl2 = uniform64(
                    __hip_atomic_load(&q->claim, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT));
                if (c < (cl2 & kChunkMask)) continue;
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        if (s < 0) break;
        const int inst = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&slots[s].inst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const unsigned long long local = c - slot_base(slots, s);
        const int n = b.n[inst];
        const int W = (n + 63) >> 6;
        const int r = b.rank[inst];
        const unsigned long long total = 1ull << r;
        const unsigned long long c0 = local << chunk_log2;
        unsigned long long c1 = c0 + (1ull << chunk_log2);
        if (c1 > total) c1 = total;
        if (W == 1) reduce_chunk<1, WMAX>(b, inst, n, r, c0, c1, Bx);
        if constexpr (WMAX >= 2)
            if (W == 2) reduce_chunk<2, WMAX>(b, inst, n, r, c0, c1, Bx);
        if constexpr (WMAX >= 3)
            if (W == 3) reduce_chunk<3, WMAX>(b, inst, n, r, c0, c1, Bx);
    }
}

}  // namespace
}  // namespace hlf

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct hlf_batch_s {
    int device = 0;
    int32_t count = 0;
    int32_t max_n = 0;
    std::vector<int32_t> n;
    std::vector<int64_t> dense_off, mat_off, vec_off, piv_off;
    int64_t dense_bytes = 0, mat_words = 0, vec_words = 0, piv_entries = 0;
    // instances ordered by word count: W = 1, 2, 3, then larger
    std::vector<int32_t> order;
    int bucket_start[5] = {0, 0, 0, 0, 0};
    // device arrays
    int32_t *d_n = nullptr;
    int64_t *d_dense_off = nullptr, *d_mat_off = nullptr, *d_vec_off = nullptr, *d_piv_off = nullptr;
    int32_t *d_order = nullptr;
    int32_t *status = nullptr, *rank = nullptr, *pivots = nullptr;
    uint64_t *basis = nullptr, *shift = nullptr, *kernel = nullptr, *counts = nullptr, *hash = nullptr;
    uint64_t *rows = nullptr;  // packed rows of instances with n > 192
    int32_t *pack_status = nullptr;
    int32_t *solve_flags = nullptr;        // per instance, idle between launches
    unsigned int *solve_done = nullptr;    // workgroups finished in a solve launch
    hlf::QueueHead *queue = nullptr;
    hlf::ChunkSlot *slots = nullptr;
    hlf_batch_params tuned = {20, 8};
    bool has_tuned = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<void *> allocations;
};

namespace {

template <typename T>
hlf_status dev_alloc(hlf_batch_s *b, T **p, size_t elems) {
    void *q = nullptr;
    const size_t bytes = std::max<size_t>(elems, 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) return HLF_ENOMEM;
    b->allocations.push_back(q);
    *p = (T *)q;
    return HLF_OK;
}

hlf::BatchDev view_of(const hlf_batch_s *b) {
    hlf::BatchDev d;
    d.count = b->count;
    d.n = b->d_n;
    d.dense_off = b->d_dense_off;
    d.mat_off = b->d_mat_off;
    d.vec_off = b->d_vec_off;
    d.piv_off = b->d_piv_off;
    d.order = b->d_order;
    d.status = b->status;
    d.rank = b->rank;
    d.pivots = b->pivots;
    d.basis = b->basis;
    d.shift = b->shift;
    d.kernel = b->kernel;
    d.counts = b->counts;
    d.hash = b->hash;
    return d;
}

hlf::FactorIn instance_view(const hlf_batch_s *b, int i) {
    hlf::FactorIn f;
    f.n = b->n[i];
    f.words = (b->n[i] + 63) / 64;
    f.status = b->status + i;
    f.rank = b->rank + i;
    f.basis = b->basis + b->mat_off[i];
    f.shift = b->shift + b->vec_off[i];
    return f;
}

bool params_ok(const hlf_batch_params &p) {
    return p.chunk_log2 >= 10 && p.chunk_log2 <= 30 && p.waves_per_cu >= 1 && p.waves_per_cu <= 16;
}

// The claim word keeps the running chunk total in its low kClaimShift bits:
// every instance with r <= max_rank claims max(1, 2^(r - chunk_log2)) chunks,
// so the total over the batch must stay below 2^kClaimShift (else it would
// carry into the slot field).
bool claims_fit_count(int count, int max_rank, int chunk_log2) {
    const int e = max_rank > chunk_log2 ? max_rank - chunk_log2 : 0;
    if (e >= hlf::kClaimShift) return false;
    const unsigned long long per = 1ull << e;
    return (unsigned long long)count < ((1ull << hlf::kClaimShift) / per);
}

bool claims_fit(const hlf_batch_s *b, int max_rank, int chunk_log2) {
    return claims_fit_count(b->count, max_rank, chunk_log2);
}

// Queue reset + the persistent factor/reduce kernel over the instances of a
// device view, with the given queue and slot arrays.
template <int WMAX>
hlf_status launch_reduce_view(const hlf::BatchDev &d, const uint8_t *A, int max_rank,
                              const hlf_batch_params &p, hlf::QueueHead *queue,
                              hlf::ChunkSlot *slots, hipStream_t stream) {
    auto kern = hlf::batch_reduce_kernel<WMAX>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const int waves = std::min(p.waves_per_cu, per_cu);
    const int grid = hlf::device_cu_count() * waves;
    const int reset_blocks = (d.count + 255) / 256;
    hipLaunchKernelGGL(hlf::batch_queue_reset_kernel, dim3(reset_blocks), dim3(256), 0, stream,
                       queue, slots, d.count);
    if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64), 0, stream, d, A, max_rank, p.chunk_log2, queue,
                       slots);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

template <int WMAX>
hlf_status launch_batch_reduce_t(hlf_batch_s *b, const uint8_t *A, int max_rank,
                                 const hlf_batch_params &p, hipStream_t stream) {
    return launch_reduce_view<WMAX>(view_of(b), A, max_rank, p, b->queue, b->slots, stream);
}

hlf_status batch_reduce_impl(hlf_batch_s *b, const uint8_t *A, int max_rank,
                             const hlf_batch_params &p, hipStream_t stream) {
    if (b->max_n <= 64) return launch_batch_reduce_t<1>(b, A, max_rank, p, stream);
    return launch_batch_reduce_t<3>(b, A, max_rank, p, stream);
}

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t, int>, std::pair<hlf_batch_params, float>> g_tune_cache;

}  // namespace

extern "C" {

hlf_status hlf_batch_create(int32_t count, const int32_t *n_host, hlf_batch *out) {
    if (!out || !n_host || count < 1 || count > (1 << 20)) return HLF_EINVAL;
    *out = nullptr;
    for (int i = 0; i < count; ++i)
        if (n_host[i] < 1 || n_host[i] > HLF_MAX_N) return HLF_EINVAL;
    hlf_batch_s *b = new hlf_batch_s();
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return HLF_EDEVICE;
    }
    b->count = count;
    b->n.assign(n_host, n_host + count);
    b->dense_off.resize(count);
    b->mat_off.resize(count);
    b->vec_off.resize(count);
    b->piv_off.resize(count);
    std::vector<std::vector<int32_t>> buckets(4);
    for (int i = 0; i < count; ++i) {
        const int64_t n = b->n[i], W = (n + 63) / 64;
        b->dense_off[i] = b->dense_bytes;
        b->mat_off[i] = b->mat_words;
        b->vec_off[i] = b->vec_words;
        b->piv_off[i] = b->piv_entries;
        b->dense_bytes += n * n;
        b->mat_words += n * W;
        b->vec_words += W;
        b->piv_entries += n;
        b->max_n = std::max<int32_t>(b->max_n, (int32_t)n);
        buckets[W <= 3 ? W - 1 : 3].push_back(i);
    }
    for (int k = 0; k < 4; ++k) {
        b->bucket_start[k] = (int)b->order.size();
        b->order.insert(b->order.end(), buckets[k].begin(), buckets[k].end());
    }
    b->bucket_start[4] = (int)b->order.size();
    int64_t big_words = 0;
    for (int i : buckets[3]) big_words = std::max<int64_t>(big_words, (int64_t)b->n[i] * ((b->n[i] + 63) / 64));

    hlf_status st = HLF_OK;
    auto chk = [&](hlf_status s) { if (st == HLF_OK) st = s; };
    chk(dev_alloc(b, &b->d_n, count));
    chk(dev_alloc(b, &b->d_dense_off, count));
    chk(dev_alloc(b, &b->d_mat_off, count));
    chk(dev_alloc(b, &b->d_vec_off, count));
    chk(dev_alloc(b, &b->d_piv_off, count));
    chk(dev_alloc(b, &b->d_order, count));
    chk(dev_alloc(b, &b->status, count));
    chk(dev_alloc(b, &b->rank, count));
    chk(dev_alloc(b, &b->pivots, b->piv_entries));
    chk(dev_alloc(b, &b->basis, b->mat_words));
    chk(dev_alloc(b, &b->shift, b->vec_words));
    chk(dev_alloc(b, &b->kernel, b->mat_words));
    chk(dev_alloc(b, &b->counts, b->piv_entries));
    chk(dev_alloc(b, &b->hash, count));
    chk(dev_alloc(b, &b->rows, big_words));
    chk(dev_alloc(b, &b->pack_status, 1));
    chk(dev_alloc(b, &b->solve_flags, count));
    chk(dev_alloc(b, &b->solve_done, 1));
    chk(dev_alloc(b, &b->queue, 1));
    chk(dev_alloc(b, &b->slots, count));
    if (st == HLF_OK) {
        auto up = [&](void *dst, const void *src, size_t bytes) {
            if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) st = HLF_EDEVICE;
        };
        up(b->d_n, b->n.data(), count * sizeof(int32_t));
        up(b->d_dense_off, b->dense_off.data(), count * sizeof(int64_t));
        up(b->d_mat_off, b->mat_off.data(), count * sizeof(int64_t));
        up(b->d_vec_off, b->vec_off.data(), count * sizeof(int64_t));
        up(b->d_piv_off, b->piv_off.data(), count * sizeof(int64_t));
        up(b->d_order, b->order.data(), count * sizeof(int32_t));
        std::vector<int32_t> init(count, HLF_EINVAL);  // not factored yet
        up(b->status, init.data(), count * sizeof(int32_t));
        std::vector<int32_t> zero(count, 0);
        up(b->solve_flags, zero.data(), count * sizeof(int32_t));
        const unsigned int zero_u = 0;
        up(b->solve_done, &zero_u, sizeof(zero_u));
    }
    if (st != HLF_OK) {
        hlf_batch_destroy(b);
        return st;
    }
    *out = b;
    return HLF_OK;
}

hlf_status hlf_batch_destroy(hlf_batch b) {
    if (!b) return HLF_OK;
    // Best-effort teardown: the handle is gone whatever these return.
    (void)hipDeviceSynchronize();
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (void *p : b->allocations) (void)hipFree(p);
    delete b;
    return HLF_OK;
}

hlf_status hlf_batch_get_layout(hlf_batch b, hlf_batch_layout *L) {
    if (!b || !L) return HLF_EINVAL;
    L->count = b->count;
    L->max_n = b->max_n;
    L->dense_bytes = b->dense_bytes;
    L->mat_words = b->mat_words;
    L->vec_words = b->vec_words;
    L->piv_entries = b->piv_entries;
    L->dense_off = b->dense_off.data();
    L->mat_off = b->mat_off.data();
    L->vec_off = b->vec_off.data();
    L->piv_off = b->piv_off.data();
    L->status = b->status;
    L->rank = b->rank;
    L->pivots = b->pivots;
    L->basis = b->basis;
    L->shift = b->shift;
    L->kernel = b->kernel;
    L->counts = b->counts;
    L->hash = b->hash;
    return HLF_OK;
}

hlf_status hlf_batch_factor_dense(hlf_batch b, const uint8_t *A_dev, hipStream_t stream) {
    if (!b || !A_dev) return HLF_EINVAL;
    const hlf::BatchDev d = view_of(b);
    for (int k = 0; k < 3; ++k) {
        const int first = b->bucket_start[k];
        const int num = b->bucket_start[k + 1] - first;
        if (num == 0) continue;
        if (k == 0) hipLaunchKernelGGL(hlf::batch_factor_kernel<1>, dim3(num), dim3(64), 0, stream, d, A_dev, first);
        if (k == 1) hipLaunchKernelGGL(hlf::batch_factor_kernel<2>, dim3(num), dim3(64), 0, stream, d, A_dev, first);
        if (k == 2) hipLaunchKernelGGL(hlf::batch_factor_kernel<3>, dim3(num), dim3(64), 0, stream, d, A_dev, first);
        if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    }
    for (int idx = b->bucket_start[3]; idx < b->bucket_start[4]; ++idx) {
        const int i = b->order[idx];
        const int n = b->n[i], W = (n + 63) / 64;
        hlf::FactorOut out;
        out.status = b->status + i;
        out.rank = b->rank + i;
        out.pivots = b->pivots + b->piv_off[i];
        out.basis = b->basis + b->mat_off[i];
        out.shift = b->shift + b->vec_off[i];
        out.kernel = b->kernel + b->mat_off[i];
        hlf_status s = hlf::launch_pack(A_dev + b->dense_off[i], n, W, b->rows, b->pack_status, stream);
        if (s != HLF_OK) return s;
        s = hlf::launch_factor(b->rows, n, W, out, false, false, stream);
        if (s != HLF_OK) return s;
        hipLaunchKernelGGL(hlf::merge_pack_status_kernel, dim3(1), dim3(64), 0, stream, out.status,
                           b->pack_status);
        if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    }
    return HLF_OK;
}

}  // extern "C"

namespace {

template <typename T>
void launch_enum_group(unsigned blocks, const hlf::EnumTasks &tasks, const hlf::FactorJob *job,
                       hipStream_t stream) {
    if (job) {
        hipLaunchKernelGGL((hlf::batch_enum_kernel<T, true>), dim3(blocks + job->blocks),
                           dim3(hlf::kTileThreads), 0, stream, tasks, *job);
    } else {
        hipLaunchKernelGGL((hlf::batch_enum_kernel<T, false>), dim3(blocks),
                           dim3(hlf::kTileThreads), 0, stream, tasks, hlf::FactorJob{});
    }
}

hlf_status batch_enumerate_impl(hlf_batch b, int32_t num, const int32_t *inst,
                                const uint64_t *begin, const uint64_t *count, void *const *out,
                                int32_t word_bits, const hlf::FactorJob *job, hipStream_t stream) {
    if (!b || num < 0 || (num > 0 && (!inst || !begin || !count || !out))) return HLF_EINVAL;
    if (word_bits != 16 && word_bits != 32 && word_bits != 64) return HLF_EINVAL;
    for (int k = 0; k < num; ++k) {
        if (inst[k] < 0 || inst[k] >= b->count) return HLF_EINVAL;
        if (b->n[inst[k]] > word_bits) return HLF_EINVAL;
        if (count[k] > 0 && !out[k]) return HLF_EINVAL;
    }
    const int V = 16 / (word_bits / 8);
    const int S = word_bits == 16 ? hlf::tile_shift<uint16_t>()
                  : word_bits == 32 ? hlf::tile_shift<uint32_t>() : hlf::tile_shift<uint64_t>();
    // Fast tasks go into multi-instance launches; the rest take the general path.
    std::vector<int> fast;
    for (int k = 0; k < num; ++k) {
        if (count[k] == 0) continue;
        const bool ok = begin[k] % V == 0 && ((uintptr_t)out[k] & 15u) == 0 &&
                        begin[k] + count[k] >= begin[k];
        if (ok) {
            fast.push_back(k);
        } else {
            hlf_status s = hlf::launch_enumerate(instance_view(b, inst[k]), begin[k], count[k],
                                                 word_bits, out[k], stream);
            if (s != HLF_OK) return s;
        }
    }
    bool job_done = job == nullptr;
    for (size_t g = 0; g < fast.size() || !job_done; g += hlf::kMaxEnumTasks) {
        const size_t m = g < fast.size() ? std::min<size_t>(hlf::kMaxEnumTasks, fast.size() - g) : 0;
        std::vector<uint64_t> tiles(m);
        uint64_t total = 0;
        for (size_t j = 0; j < m; ++j) {
            const int k = fast[g + j];
            const uint64_t end = begin[k] + count[k];
            tiles[j] = ((end - 1) >> S) - (begin[k] >> S) + 1;
            total += tiles[j];
        }
        const uint64_t tpb = hlf::materialise_tiles_per_block(total, hlf::kTileBytes);
        hlf::EnumTasks tasks;
        std::memset(&tasks, 0, sizeof(tasks));
        tasks.num = (int)m;
        uint64_t block = 0;
        for (size_t j = 0; j < m; ++j) {
            const int k = fast[g + j];
            const int i = inst[k];
            hlf::EnumTask &t = tasks.t[j];
            t.status = b->status + i;
            t.rank = b->rank + i;
            t.basis = b->basis + b->mat_off[i];
            t.shift = b->shift + b->vec_off[i];
            t.out = out[k];
            t.begin = begin[k];
            t.count = count[k];
            t.block0 = (uint32_t)block;
            t.tiles_per_block = (uint32_t)tpb;
            block += (tiles[j] + tpb - 1) / tpb;
        }
        if (block > 0xFFFF0000ull) return HLF_EINVAL;
        const hlf::FactorJob *jb = job_done ? nullptr : job;
        job_done = true;
        if (word_bits == 16) launch_enum_group<uint16_t>((unsigned)block, tasks, jb, stream);
        else if (word_bits == 32) launch_enum_group<uint32_t>((unsigned)block, tasks, jb, stream);
        else launch_enum_group<uint64_t>((unsigned)block, tasks, jb, stream);
        if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    }
    return HLF_OK;
}

}  // namespace

extern "C" {

hlf_status hlf_batch_enumerate(hlf_batch b, int32_t num, const int32_t *inst,
                               const uint64_t *begin, const uint64_t *count, void *const *out,
                               int32_t word_bits, hipStream_t stream) {
    return batch_enumerate_impl(b, num, inst, begin, count, out, word_bits, nullptr, stream);
}

hlf_status hlf_batch_enumerate_overlap(hlf_batch b, int32_t num, const int32_t *inst,
                                       const uint64_t *begin, const uint64_t *count,
                                       void *const *out, int32_t word_bits, hlf_batch next,
                                       const uint8_t *A_next_dev, hipStream_t stream) {
    if (!next || !A_next_dev || next == b || next->max_n > 64) return HLF_EINVAL;
    hlf::FactorJob job;
    job.d = view_of(next);
    job.A = A_next_dev;
    job.first = 0;
    job.num = next->count;
    job.blocks = (uint32_t)((next->count + hlf::kWavesPerTileBlock - 1) / hlf::kWavesPerTileBlock);
    return batch_enumerate_impl(b, num, inst, begin, count, out, word_bits, &job, stream);
}

hlf_status hlf_batch_solve(hlf_batch b, const uint8_t *A_dev, int32_t num, const int32_t *inst,
                           const uint64_t *begin, const uint64_t *count, void *const *out,
                           int32_t word_bits, hipStream_t stream) {
    if (!b || !A_dev || num < 1 || num > hlf::kMaxEnumTasks || !inst || !begin || !count || !out)
        return HLF_EINVAL;
    if (word_bits != 16 && word_bits != 32 && word_bits != 64) return HLF_EINVAL;
    const int V = 16 / (word_bits / 8);
    const int S = word_bits == 16 ? hlf::tile_shift<uint16_t>()
                  : word_bits == 32 ? hlf::tile_shift<uint32_t>() : hlf::tile_shift<uint64_t>();
    std::vector<uint64_t> tiles(num);
    uint64_t total = 0;
    for (int k = 0; k < num; ++k) {
        const int i = inst[k];
        if (i < 0 || i >= b->count || b->n[i] > word_bits) return HLF_EINVAL;
        if (count[k] == 0 || !out[k] || begin[k] % V != 0 || ((uintptr_t)out[k] & 15u) != 0 ||
            begin[k] + count[k] < begin[k])
            return HLF_EINVAL;
        const uint64_t end = begin[k] + count[k];
        tiles[k] = ((end - 1) >> S) - (begin[k] >> S) + 1;
        total += tiles[k];
    }
    const uint64_t target_blocks = (uint64_t)hlf::device_cu_count() * hlf::kTileBlocksPerCU;
    const uint64_t tpb = std::max<uint64_t>(1, (total + target_blocks - 1) / target_blocks);
    hlf::SolveTasks tasks;
    std::memset(&tasks, 0, sizeof(tasks));
    tasks.num = num;
    uint64_t block = 0;
    for (int k = 0; k < num; ++k) {
        const int i = inst[k];
        hlf::EnumTask &t = tasks.t[k];
        t.status = b->status + i;
        t.rank = b->rank + i;
        t.basis = b->basis + b->mat_off[i];
        t.shift = b->shift + b->vec_off[i];
        t.out = out[k];
        t.begin = begin[k];
        t.count = count[k];
        t.block0 = (uint32_t)block;
        t.tiles_per_block = (uint32_t)tpb;
        tasks.inst[k] = i;
        block += (tiles[k] + tpb - 1) / tpb;
    }
    if (block > 0xFFFFFFFFull) return HLF_EINVAL;
    const hlf::BatchDev d = view_of(b);
    if (word_bits == 16)
        hipLaunchKernelGGL(hlf::batch_solve_kernel<uint16_t>, dim3((unsigned)block), dim3(hlf::kTileThreads), 0, stream, d, A_dev, tasks, b->solve_flags, b->solve_done);
    else if (word_bits == 32)
        hipLaunchKernelGGL(hlf::batch_solve_kernel<uint32_t>, dim3((unsigned)block), dim3(hlf::kTileThreads), 0, stream, d, A_dev, tasks, b->solve_flags, b->solve_done);
    else
        hipLaunchKernelGGL(hlf::batch_solve_kernel<uint64_t>, dim3((unsigned)block), dim3(hlf::kTileThreads), 0, stream, d, A_dev, tasks, b->solve_flags, b->solve_done);
    return hipGetLastError() == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

hlf_status hlf_batch_reduce(hlf_batch b, const uint8_t *A_dev, int32_t max_rank,
                            const hlf_batch_params *params, hipStream_t stream) {
    if (!b || !A_dev || max_rank < 0 || max_rank > HLF_MAX_ENUM_RANK) return HLF_EINVAL;
    if (b->max_n > 192) return HLF_EINVAL;
    const hlf_batch_params p = params ? *params : b->tuned;
    if (!params_ok(p) || !claims_fit(b, max_rank, p.chunk_log2)) return HLF_EINVAL;
    return batch_reduce_impl(b, A_dev, max_rank, p, stream);
}

hlf_status hlf_batch_tune(hlf_batch b, const uint8_t *A_dev, int32_t max_rank,
                          hlf_batch_params *best, float *best_ms, hipStream_t stream) {
    if (!b || !A_dev || max_rank < 0 || max_rank > HLF_MAX_ENUM_RANK) return HLF_EINVAL;
    if (b->max_n > 192) return HLF_EINVAL;
    const auto key = std::make_tuple(b->count, b->max_n, b->piv_entries, (int)max_rank);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            b->tuned = it->second.first;
            b->has_tuned = true;
            if (best) *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return HLF_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return HLF_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return HLF_EDEVICE;
    }
    const int chunks[] = {14, 16, 18, 20, 22};
    const int waves[] = {2, 4, 8, 12};
    hlf_batch_params bestp = b->tuned;
    float bestt = 1e30f;
    hlf_status st = HLF_OK;
    bool any = false;
    for (int c : chunks) {
        if (!claims_fit(b, max_rank, c)) continue;
        any = true;
        for (int w : waves) {
            const hlf_batch_params p = {c, w};
            st = batch_reduce_impl(b, A_dev, max_rank, p, stream);  // warm
            if (st != HLF_OK) break;
            float tsum = 0;
            for (int rep = 0; rep < 2 && st == HLF_OK; ++rep) {
                if (hipEventRecord(e0, stream) != hipSuccess) st = HLF_EDEVICE;
                if (st == HLF_OK) st = batch_reduce_impl(b, A_dev, max_rank, p, stream);
                if (st == HLF_OK && hipEventRecord(e1, stream) != hipSuccess) st = HLF_EDEVICE;
                if (st == HLF_OK && hipEventSynchronize(e1) != hipSuccess) st = HLF_EDEVICE;
                float ms = 0;
                if (st == HLF_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) st = HLF_EDEVICE;
                tsum += ms;
            }
            if (st != HLF_OK) break;
            if (tsum / 2 < bestt) {
                bestt = tsum / 2;
                bestp = p;
            }
        }
        if (st != HLF_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != HLF_OK) return st;
    if (!any) return HLF_EINVAL;
    b->tuned = bestp;
    b->has_tuned = true;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = {bestp, bestt};
    }
    if (best) *best = bestp;
    if (best_ms) *best_ms = bestt;
    return HLF_OK;
}

hlf_status hlf_batch_graph_capture(hlf_batch b, const uint8_t *A_dev, int32_t max_rank,
                                   const hlf_batch_params *params) {
    if (!b || !A_dev || max_rank < 0 || max_rank > HLF_MAX_ENUM_RANK) return HLF_EINVAL;
    if (b->max_n > 192) return HLF_EINVAL;
    const hlf_batch_params p = params ? *params : b->tuned;
    if (!params_ok(p) || !claims_fit(b, max_rank, p.chunk_log2)) return HLF_EINVAL;
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return HLF_EDEVICE;
    hlf_status st = HLF_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) st = HLF_EDEVICE;
    if (st == HLF_OK) {
        st = batch_reduce_impl(b, A_dev, max_rank, p, s);
        if (hipStreamEndCapture(s, &g) != hipSuccess) st = HLF_EDEVICE;
    }
    hipGraphExec_t exec = nullptr;
    if (st == HLF_OK && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) != hipSuccess)
        st = HLF_EDEVICE;
    (void)hipStreamDestroy(s);
    if (st != HLF_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph = g;
    b->graph_exec = exec;
    return HLF_OK;
}

hlf_status hlf_batch_graph_launch(hlf_batch b, hipStream_t stream) {
    if (!b || !b->graph_exec) return HLF_EINVAL;
    return hipGraphLaunch(b->graph_exec, stream) == hipSuccess ? HLF_OK : HLF_EDEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free batched reduce.  Its scratch -- the work queue, the chunk
// slots, the layout offsets and the checked sizes -- is one file-scope device
// array; each device holds its own copy, located once per device with
// hipGetSymbolAddress and used through that address only.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocMaxCount = 16384;
constexpr size_t kNoAllocQueueBytes = 256;
constexpr size_t kNoAllocSlotBytes = sizeof(hlf::ChunkSlot) * kNoAllocMaxCount;
constexpr size_t kNoAllocOffBytes = sizeof(int64_t) * kNoAllocMaxCount;
constexpr size_t kNoAllocScratchBytes =
    kNoAllocQueueBytes + kNoAllocSlotBytes + 4 * kNoAllocOffBytes + sizeof(int32_t) * kNoAllocMaxCount;
static_assert(sizeof(hlf::QueueHead) <= kNoAllocQueueBytes, "queue head fits its space");
static_assert(kNoAllocMaxCount <= 1024 * hlf::kLayoutPer, "one layout workgroup covers every instance");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

// Device address of this device's scratch array (looked up once per device).
hlf_status scratch_address(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return HLF_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return HLF_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HLF_OK;
}
}  // namespace

extern "C" {

hlf_status hlf_batch_reduce_noalloc(int32_t count, int32_t max_n, const int32_t *n_dev,
                                    const uint8_t *A_dev, int32_t max_rank,
                                    const hlf_batch_params *params, int32_t *status_dev,
                                    int32_t *rank_dev, int32_t *pivots_dev, uint64_t *basis_dev,
                                    uint64_t *shift_dev, uint64_t *kernel_dev,
                                    uint64_t *counts_dev, uint64_t *hash_dev, hipStream_t stream) {
    if (count < 1 || count > kNoAllocMaxCount || max_n < 1 || max_n > 192) return HLF_EINVAL;
    if (!n_dev || !A_dev || !status_dev || !rank_dev || !pivots_dev || !basis_dev || !shift_dev ||
        !counts_dev || !hash_dev)
        return HLF_EINVAL;
    if (max_rank < 0 || max_rank > HLF_MAX_ENUM_RANK) return HLF_EINVAL;
    const hlf_batch_params p = params ? *params : hlf_batch_params{20, 8};
    if (!params_ok(p) || !claims_fit_count(count, max_rank, p.chunk_log2)) return HLF_EINVAL;
    void *base = nullptr;
    const hlf_status st = scratch_address(&base);
    if (st != HLF_OK) return st;
    unsigned char *sb = static_cast<unsigned char *>(base);
    auto *queue = reinterpret_cast<hlf::QueueHead *>(sb);
    auto *slots = reinterpret_cast<hlf::ChunkSlot *>(sb + kNoAllocQueueBytes);
    auto *offs = reinterpret_cast<int64_t *>(sb + kNoAllocQueueBytes + kNoAllocSlotBytes);
    auto *n_eff = reinterpret_cast<int32_t *>(offs + 4 * kNoAllocMaxCount);
    hlf::BatchDev d;
    d.count = count;
    d.n = n_eff;
    d.dense_off = offs;
    d.mat_off = offs + kNoAllocMaxCount;
    d.vec_off = offs + 2 * kNoAllocMaxCount;
    d.piv_off = offs + 3 * kNoAllocMaxCount;
    d.order = nullptr;
    d.status = status_dev;
    d.rank = rank_dev;
    d.pivots = pivots_dev;
    d.basis = basis_dev;
    d.shift = shift_dev;
    d.kernel = kernel_dev;
    d.counts = counts_dev;
    d.hash = hash_dev;
    hipLaunchKernelGGL(hlf::noalloc_layout_kernel, dim3(1), dim3(1024), 0, stream, n_dev, count,
                       max_n, n_eff, offs, offs + kNoAllocMaxCount, offs + 2 * kNoAllocMaxCount,
                       offs + 3 * kNoAllocMaxCount);
    if (hipGetLastError() != hipSuccess) return HLF_EDEVICE;
    if (max_n <= 64) return launch_reduce_view<1>(d, A_dev, max_rank, p, queue, slots, stream);
    return launch_reduce_view<3>(d, A_dev, max_rank, p, queue, slots, stream);
}

}  // extern "C"
