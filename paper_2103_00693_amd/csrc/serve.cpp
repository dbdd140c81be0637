// Serving engine: continuous admission of FS2D HLF requests onto one GPU
// (the workload of Section 1 per request: stage 1, the CLA module of
// Section 2, then either every solution -- the circuit's traversal of
// Section 2 -- or uniform single solutions, the quantum circuit's output of
// Appendix A).
//
// One worker thread owns the device side.  Requests wait in arrival order; a
// request is admitted when a slot (a HIP stream) is free, its arrival time has
// come and its stage-1 memory can be carved from the server's arena, a single
// allocation of the configured HBM budget made at creation: every device byte
// the server touches (inputs, packed rows, stage-1 records, outputs, the
// stage-1 cache) lies in that arena, so the budget is exact.  Each admitted
// request advances on its slot's stream as soon as its previous phase's event
// has fired:
//   phase 1: host staging -> device copy, pack, factor, status and rank to
//            pinned memory;
//   phase 2: with r known, carve the exact output from the arena (waiting
//            for memory if needed), enumerate all 2^r solutions (n <= 64,
//            r <= enum_max_rank) or sample num_samples solutions, copy to the
//            pinned result arena;
//   done:    the result (a pointer into the pinned arena, held until the
//            caller releases it) goes to the completion queue.
// Results depend only on (A, seed): the sampling stream is keyed by (seed,
// sample index), never by slot, timing or cache state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hlf.h"

namespace {

// First-fit allocator over one contiguous region, with coalescing.  Offsets
// and sizes are multiples of kAlign.
class Arena {
public:
    static constexpr int64_t kAlign = 256;
    void reset(int64_t bytes) {
        free_.clear();
        size_ = bytes / kAlign * kAlign;
        if (size_ > 0) free_[0] = size_;
        used_ = peak_ = 0;
    }
    // Offset of a block of `bytes`, or -1.
    int64_t alloc(int64_t bytes) {
        const int64_t need = std::max<int64_t>(kAlign, (bytes + kAlign - 1) / kAlign * kAlign);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const int64_t off = it->first, rest = it->second - need;
                free_.erase(it);
                if (rest > 0) free_[off + need] = rest;
                sizes_[off] = need;
                used_ += need;
                peak_ = std::max(peak_, used_);
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off) {
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return;
        int64_t start = off, len = s->second;
        sizes_.erase(s);
        used_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = len;
    }
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
    int64_t size() const { return size_; }

private:
    std::map<int64_t, int64_t> free_;                 // offset -> length
    std::unordered_map<int64_t, int64_t> sizes_;      // offset -> length of live blocks
    int64_t size_ = 0, used_ = 0, peak_ = 0;
};

int32_t words_of(int32_t n) { return (n + 63) / 64; }

// Device bytes of a stage-1 record: status, rank, pivots[n], then (8-byte
// aligned) basis[n*W] and shift[W].
int64_t record_bytes(int32_t n) {
    const int64_t head = ((8 + 4 * (int64_t)n) + 7) / 8 * 8;
    return head + 8 * ((int64_t)n * words_of(n) + words_of(n));
}

struct Record {
    int64_t off = -1;   // arena offset
    int32_t n = 0;
    int32_t status = 0, rank = 0;
};

struct Key {
    uint64_t hi, lo;
    int32_t n;
    bool operator==(const Key &o) const { return hi == o.hi && lo == o.lo && n == o.n; }
};
struct KeyHash {
    size_t operator()(const Key &k) const { return (size_t)(k.hi ^ (k.lo * 0x9E3779B97F4A7C15ull) ^ (uint64_t)k.n); }
};

struct CacheEntry {
    Record rec;
    int refs = 0;
    std::list<Key>::iterator lru;
};

struct Pending {
    hlf_request req;   // req.A is the caller's matrix, valid until the result is polled
};

struct Active {
    Pending p;
    int phase = 0;
    bool cache_hit = false;
    Key key{};
    bool keyed = false;
    Record rec;              // own record (not cached yet) or the cached one
    bool rec_cached = false; // rec belongs to the cache (holds a reference)
    int64_t a_off = -1, rows_off = -1, out_off = -1;
    int64_t out_bytes = 0, out_count = 0;
    int32_t word_bytes = 0, kind = 0;
    int64_t host_off = -1;
    int64_t admitted_ns = 0;
};

}  // namespace

struct hlf_server_s {
    hlf_server_config cfg{};
    int device = 0;
    char *dev_base = nullptr;
    char *host_base = nullptr;
    Arena dev, host;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    std::vector<uint8_t *> staging;     // pinned, n*n bytes at most per slot
    int32_t *heads = nullptr;           // pinned (status, rank) per slot
    std::vector<Active *> slot_job;
    std::chrono::steady_clock::time_point epoch;

    std::mutex mu;                      // guards `incoming`, `done`, `host`, `stop`
    std::condition_variable cv_in, cv_done;
    std::deque<Pending> incoming;
    std::deque<hlf_result> done;
    bool stop = false;
    std::atomic<int64_t> admitted{0}, cache_hits{0}, completed{0};
    std::atomic<int64_t> dev_peak{0};   // copy of dev.peak() for other threads

    // worker-only state
    std::deque<Pending> pending;
    std::unordered_map<Key, CacheEntry, KeyHash> cache;
    std::list<Key> lru;                 // front = least recently used
    std::thread worker;
    hlf_status worker_error = HLF_OK;

    int64_t now_ns() const {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now() - epoch).count();
    }
};

namespace {

hlf_factors factors_at(hlf_server_s *s, const Record &r) {
    hlf_factors f;
    const int32_t n = r.n, W = words_of(n);
    char *b = s->dev_base + r.off;
    f.n = n;
    f.words = W;
    f.status = reinterpret_cast<int32_t *>(b);
    f.rank = reinterpret_cast<int32_t *>(b + 4);
    f.pivots = reinterpret_cast<int32_t *>(b + 8);
    const int64_t head = ((8 + 4 * (int64_t)n) + 7) / 8 * 8;
    f.basis = reinterpret_cast<uint64_t *>(b + head);
    f.shift = f.basis + (int64_t)n * W;
    f.kernel = nullptr;
    return f;
}

// Evict least recently used cache entries that no request holds until `bytes`
// can be allocated from the device arena; offset or -1.
int64_t dev_alloc_evicting(hlf_server_s *s, int64_t bytes) {
    int64_t off = s->dev.alloc(bytes);
    auto it = s->lru.begin();
    while (off < 0 && it != s->lru.end()) {
        auto e = s->cache.find(*it);
        if (e != s->cache.end() && e->second.refs == 0) {
            s->dev.release(e->second.rec.off);
            s->cache.erase(e);
            it = s->lru.erase(it);
            off = s->dev.alloc(bytes);
        } else {
            ++it;
        }
    }
    return off;
}

void finish(hlf_server_s *s, Active *a, int32_t status) {
    hlf_result r;
    std::memset(&r, 0, sizeof(r));
    r.id = a->p.req.id;
    r.status = status;
    r.n = a->p.req.n;
    r.rank = a->rec.rank;
    r.kind = status == HLF_OK ? a->kind : 0;
    r.word_bytes = a->word_bytes;
    r.count = status == HLF_OK ? a->out_count : 0;
    r.data = (status == HLF_OK && a->host_off >= 0) ? s->host_base + a->host_off : nullptr;
    r.arrival_ns = a->p.req.arrival_ns;
    r.admitted_ns = a->admitted_ns;
    r.finished_ns = s->now_ns();
    r.cache_hit = a->cache_hit ? 1 : 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (status != HLF_OK && a->host_off >= 0) s->host.release(a->host_off);
        s->done.push_back(r);
    }
    s->cv_done.notify_all();
    s->completed.fetch_add(1);
}

// Releases the device memory of a finished or failed request and files its
// stage-1 record in the cache when it is keyed and valid.
void retire(hlf_server_s *s, Active *a) {
    if (a->a_off >= 0) s->dev.release(a->a_off);
    if (a->rows_off >= 0) s->dev.release(a->rows_off);
    if (a->out_off >= 0) s->dev.release(a->out_off);
    a->a_off = a->rows_off = a->out_off = -1;
    if (a->rec_cached) {
        auto e = s->cache.find(a->key);
        if (e != s->cache.end()) e->second.refs--;
    } else if (a->rec.off >= 0) {
        const bool keep = a->keyed && s->cfg.cache_entries > 0 && a->rec.status == HLF_OK &&
                          s->cache.find(a->key) == s->cache.end();
        if (keep) {
            while ((int)s->cache.size() >= s->cfg.cache_entries) {
                auto it = s->lru.begin();
                while (it != s->lru.end() && s->cache[*it].refs > 0) ++it;
                if (it == s->lru.end()) break;
                s->dev.release(s->cache[*it].rec.off);
                s->cache.erase(*it);
                s->lru.erase(it);
            }
        }
        if (keep && (int)s->cache.size() < s->cfg.cache_entries) {
            CacheEntry ce;
            ce.rec = a->rec;
            s->lru.push_back(a->key);
            ce.lru = std::prev(s->lru.end());
            s->cache.emplace(a->key, ce);
        } else {
            s->dev.release(a->rec.off);
        }
    }
    a->rec.off = -1;
}

// Phase 2 launch (after stage 1, or at once on a cache hit).  Returns false
// if the pinned result arena is full (the request waits and retries).
bool launch_phase2(hlf_server_s *s, int slot, Active *a) {
    const int32_t n = a->p.req.n;
    hipStream_t st = s->streams[slot];
    if (a->rec.status != HLF_OK) {
        retire(s, a);
        finish(s, a, a->rec.status);
        return true;
    }
    const int32_t r = a->rec.rank;
    int64_t bytes;
    if (n <= 64 && r <= s->cfg.enum_max_rank) {
        a->kind = 1;
        a->word_bytes = n <= 16 ? 2 : n <= 32 ? 4 : 8;
        a->out_count = (int64_t)1 << r;
    } else {
        a->kind = 2;
        a->word_bytes = 8 * words_of(n);
        a->out_count = s->cfg.num_samples;
    }
    bytes = a->out_count * a->word_bytes;
    if (bytes + Arena::kAlign > s->host.size() ||
        bytes + record_bytes(n) + 2 * Arena::kAlign > s->dev.size()) {  // can never fit
        retire(s, a);
        finish(s, a, HLF_ENOMEM);
        return true;
    }
    if (a->out_off < 0) {
        a->out_off = dev_alloc_evicting(s, bytes);
        if (a->out_off < 0) return false;  // waits for device memory
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        a->host_off = s->host.alloc(bytes);
    }
    if (a->host_off < 0) return false;    // waits for result memory
    a->out_bytes = bytes;
    hlf_factors f = factors_at(s, a->rec);
    void *out = s->dev_base + a->out_off;
    hlf_status rc = a->kind == 1 ? hlf_enumerate(&f, 0, (uint64_t)a->out_count, 8 * a->word_bytes, out, st)
                                 : hlf_sample(&f, a->p.req.seed, (uint64_t)a->out_count, nullptr,
                                              (uint64_t *)out, st);
    if (rc == HLF_OK && hipMemcpyAsync(s->host_base + a->host_off, out, bytes, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = HLF_EDEVICE;
    if (rc == HLF_OK && hipEventRecord(s->events[slot], st) != hipSuccess) rc = HLF_EDEVICE;
    if (rc != HLF_OK) {
        s->worker_error = rc;
        retire(s, a);
        finish(s, a, rc);
        return true;
    }
    a->phase = 2;
    return true;
}

// Admission of the next pending request on a free slot: false if it does not
// fit the device arena now.
bool admit(hlf_server_s *s, int slot) {
    Pending &p = s->pending.front();
    const int32_t n = p.req.n, W = words_of(n);
    auto *a = new Active();
    a->key = Key{p.req.key[0], p.req.key[1], n};
    a->keyed = (p.req.key[0] | p.req.key[1]) != 0;
    // stage-1 cache
    if (a->keyed) {
        auto e = s->cache.find(a->key);
        if (e != s->cache.end()) {
            e->second.refs++;
            s->lru.splice(s->lru.end(), s->lru, e->second.lru);
            a->rec = e->second.rec;
            a->rec_cached = true;
            a->cache_hit = true;
            a->p = std::move(p);
            s->pending.pop_front();
            a->admitted_ns = s->now_ns();
            s->admitted.fetch_add(1);
            s->cache_hits.fetch_add(1);
            s->slot_job[slot] = a;
            if (!launch_phase2(s, slot, a)) a->phase = 3;  // waits for memory
            if (a->phase != 2 && a->phase != 3) {            // finished at once
                s->slot_job[slot] = nullptr;
                delete a;
            }
            return true;
        }
    }
    const int64_t need[3] = {(int64_t)n * n, 8 * (int64_t)n * W, record_bytes(n)};
    int64_t off[3] = {-1, -1, -1};
    for (int k = 0; k < 3; ++k) {
        off[k] = dev_alloc_evicting(s, need[k]);
        if (off[k] < 0) {
            for (int j = 0; j < k; ++j) s->dev.release(off[j]);
            delete a;
            return false;
        }
    }
    a->a_off = off[0];
    a->rows_off = off[1];
    a->rec.off = off[2];
    a->rec.n = n;
    a->p = std::move(p);
    s->pending.pop_front();
    a->admitted_ns = s->now_ns();
    s->admitted.fetch_add(1);
    hipStream_t st = s->streams[slot];
    std::memcpy(s->staging[slot], a->p.req.A, (size_t)n * n);
    hlf_factors f = factors_at(s, a->rec);
    uint8_t *A_dev = reinterpret_cast<uint8_t *>(s->dev_base + a->a_off);
    uint64_t *rows = reinterpret_cast<uint64_t *>(s->dev_base + a->rows_off);
    hlf_status rc = HLF_OK;
    if (hipMemcpyAsync(A_dev, s->staging[slot], (size_t)n * n, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = HLF_EDEVICE;
    if (rc == HLF_OK) rc = hlf_pack_dense(A_dev, n, rows, f.status, st);
    if (rc == HLF_OK) rc = hlf_factor_ex(rows, &f, HLF_FACTOR_PACK_STATUS, st);
    if (rc == HLF_OK && hipMemcpyAsync(s->heads + 2 * slot, f.status, 8, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = HLF_EDEVICE;
    if (rc == HLF_OK && hipEventRecord(s->events[slot], st) != hipSuccess) rc = HLF_EDEVICE;
    if (rc != HLF_OK) {
        s->worker_error = rc;
        a->rec.status = rc;
        retire(s, a);
        finish(s, a, rc);
        delete a;
        return true;
    }
    a->phase = 1;
    s->slot_job[slot] = a;
    return true;
}

void worker_main(hlf_server_s *s) {
    if (hipSetDevice(s->device) != hipSuccess) {
        s->worker_error = HLF_EDEVICE;
        return;
    }
    const int slots = s->cfg.slots;
    for (;;) {
        bool stopping = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            bool idle = s->pending.empty();
            for (int k = 0; k < slots && idle; ++k) idle = s->slot_job[k] == nullptr;
            if (idle && s->incoming.empty() && !s->stop)
                s->cv_in.wait_for(lk, std::chrono::milliseconds(50));
            if (s->stop) {
                stopping = true;
                bool busy = false;
                for (int k = 0; k < slots; ++k) busy = busy || s->slot_job[k] != nullptr;
                if (!busy) return;
            }
            while (!s->incoming.empty()) {
                s->pending.push_back(std::move(s->incoming.front()));
                s->incoming.pop_front();
            }
        }
        bool progressed = false;
        // advance admitted requests whose last phase has finished
        for (int k = 0; k < slots; ++k) {
            Active *a = s->slot_job[k];
            if (!a) continue;
            if (a->phase == 3) {  // waiting for output (device) or result (pinned) memory
                if (stopping) {   // the caller no longer releases results: give up
                    retire(s, a);
                    finish(s, a, HLF_ENOMEM);
                    s->slot_job[k] = nullptr;
                    delete a;
                    progressed = true;
                    continue;
                }
                if (launch_phase2(s, k, a)) {
                    progressed = true;
                    if (a->phase != 2) {
                        s->slot_job[k] = nullptr;
                        delete a;
                    }
                }
                continue;
            }
            const hipError_t q = hipEventQuery(s->events[k]);
            if (q == hipErrorNotReady) continue;
            progressed = true;
            if (q != hipSuccess) {
                s->worker_error = HLF_EDEVICE;
                retire(s, a);
                finish(s, a, HLF_EDEVICE);
                s->slot_job[k] = nullptr;
                delete a;
                continue;
            }
            if (a->phase == 1) {
                a->rec.status = s->heads[2 * k];
                a->rec.rank = s->heads[2 * k + 1];
                // the dense input and packed rows are no longer needed
                s->dev.release(a->a_off);
                s->dev.release(a->rows_off);
                a->a_off = a->rows_off = -1;
                if (!launch_phase2(s, k, a)) {
                    a->phase = 3;
                } else if (a->phase != 2) {
                    s->slot_job[k] = nullptr;
                    delete a;
                }
            } else {  // phase 2 done: the result is in pinned memory
                retire(s, a);
                finish(s, a, HLF_OK);
                s->slot_job[k] = nullptr;
                delete a;
            }
        }
        // admission: arrived requests, free slots, device memory
        const int64_t now = s->now_ns();
        for (int k = 0; k < slots && !s->pending.empty() && !stopping; ++k) {
            if (s->slot_job[k] != nullptr) continue;
            Pending &p = s->pending.front();
            if (p.req.arrival_ns > now) break;
            const int32_t n = p.req.n;
            const int64_t total = (int64_t)n * n + 8 * (int64_t)n * words_of(n) + record_bytes(n) +
                                  3 * Arena::kAlign;
            if (total > s->dev.size()) {  // can never fit: fail it
                auto *a = new Active();
                a->p = std::move(p);
                s->pending.pop_front();
                a->rec.n = n;
                a->admitted_ns = now;
                finish(s, a, HLF_ENOMEM);
                delete a;
                progressed = true;
                continue;
            }
            if (!admit(s, k)) break;
            progressed = true;
        }
        s->dev_peak.store(s->dev.peak(), std::memory_order_relaxed);
        if (!progressed) {
            bool active = false;
            for (int k = 0; k < slots; ++k) active = active || s->slot_job[k] != nullptr;
            if (active) {
                std::this_thread::yield();
            } else if (!s->pending.empty()) {
                const int64_t wait = s->pending.front().req.arrival_ns - s->now_ns();
                if (wait > 0)
                    std::this_thread::sleep_for(std::chrono::nanoseconds(std::min<int64_t>(wait, 200000)));
            }
        }
    }
}

void destroy_resources(hlf_server_s *s) {
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto ev : s->events) (void)hipEventDestroy(ev);
    for (auto p : s->staging) (void)hipHostFree(p);
    if (s->heads) (void)hipHostFree(s->heads);
    if (s->host_base) (void)hipHostFree(s->host_base);
    if (s->dev_base) (void)hipFree(s->dev_base);
}

}  // namespace

extern "C" {

hlf_status hlf_server_create(const hlf_server_config *cfg, hlf_server *out) {
    if (!cfg || !out) return HLF_EINVAL;
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > 64 || cfg->hbm_bytes < (1 << 20) || cfg->host_bytes < (1 << 20) ||
        cfg->num_samples < 1 || cfg->enum_max_rank < 0 || cfg->enum_max_rank > 30 || cfg->cache_entries < 0)
        return HLF_EINVAL;
    auto *s = new hlf_server_s();
    s->cfg = *cfg;
    s->epoch = std::chrono::steady_clock::now();
    hlf_status st = HLF_OK;
    if (hipGetDevice(&s->device) != hipSuccess) st = HLF_EDEVICE;
    if (st == HLF_OK && hipMalloc((void **)&s->dev_base, (size_t)cfg->hbm_bytes) != hipSuccess) st = HLF_ENOMEM;
    if (st == HLF_OK && hipHostMalloc((void **)&s->host_base, (size_t)cfg->host_bytes, hipHostMallocDefault) != hipSuccess)
        st = HLF_ENOMEM;
    if (st == HLF_OK && hipHostMalloc((void **)&s->heads, 8 * (size_t)cfg->slots, hipHostMallocDefault) != hipSuccess)
        st = HLF_ENOMEM;
    for (int k = 0; k < cfg->slots && st == HLF_OK; ++k) {
        hipStream_t stream;
        hipEvent_t ev;
        uint8_t *stg = nullptr;
        if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) { st = HLF_EDEVICE; break; }
        s->streams.push_back(stream);
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) { st = HLF_EDEVICE; break; }
        s->events.push_back(ev);
        if (hipHostMalloc((void **)&stg, (size_t)HLF_MAX_N * HLF_MAX_N, hipHostMallocDefault) != hipSuccess) {
            st = HLF_ENOMEM;
            break;
        }
        s->staging.push_back(stg);
    }
    if (st != HLF_OK) {
        destroy_resources(s);
        delete s;
        return st;
    }
    s->dev.reset(cfg->hbm_bytes);
    s->host.reset(cfg->host_bytes);
    s->slot_job.assign(cfg->slots, nullptr);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return HLF_OK;
}

int64_t hlf_server_now(hlf_server s) { return s ? s->now_ns() : -1; }

hlf_status hlf_server_submit(hlf_server s, const hlf_request *reqs, int32_t count) {
    if (!s || (!reqs && count > 0) || count < 0) return HLF_EINVAL;
    for (int i = 0; i < count; ++i)
        if (reqs[i].n < 1 || reqs[i].n > HLF_MAX_N || !reqs[i].A) return HLF_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (int i = 0; i < count; ++i) s->incoming.push_back(Pending{reqs[i]});
    }
    s->cv_in.notify_all();
    return HLF_OK;
}

hlf_status hlf_server_poll(hlf_server s, hlf_result *out, int32_t max, int32_t *got, int32_t wait_ms) {
    if (!s || !out || !got || max < 1) return HLF_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_ms > 0)
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
    int k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *got = k;
    return HLF_OK;
}

hlf_status hlf_server_release(hlf_server s, const void *data) {
    if (!s) return HLF_EINVAL;
    if (!data) return HLF_OK;
    const int64_t off = static_cast<const char *>(data) - s->host_base;
    if (off < 0 || off >= s->cfg.host_bytes) return HLF_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    s->host.release(off);
    return HLF_OK;
}

hlf_status hlf_server_get_stats(hlf_server s, hlf_server_stats *out) {
    if (!s || !out) return HLF_EINVAL;
    out->admitted = s->admitted.load();
    out->completed = s->completed.load();
    out->cache_hits = s->cache_hits.load();
    out->hbm_bytes = s->cfg.hbm_bytes;
    out->hbm_peak_bytes = s->dev_peak.load(std::memory_order_relaxed);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        out->host_peak_bytes = s->host.peak();
    }
    out->worker_status = s->worker_error;
    return HLF_OK;
}

hlf_status hlf_server_destroy(hlf_server s) {
    if (!s) return HLF_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->incoming.clear();
    }
    s->cv_in.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    destroy_resources(s);
    delete s;
    return HLF_OK;
}

}  // extern "C"
