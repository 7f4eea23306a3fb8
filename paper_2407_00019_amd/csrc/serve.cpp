// Continuous-batching SpMV server: the auto-tuner of section 2.2 applied per
// request, with the transformation amortised over the request's declared
// number of SpMVs (the iteration-count discussion after the on-line phase).
//
// A dispatcher thread makes jobs visible at their arrival time and admits
// them in FIFO order: the head job waits until a slot is free and its CRS
// block fits in the device arena.  Each slot (one HIP stream) has its own
// worker thread, so the host work of one job (copies, launches, waits)
// never holds up another's.  A worker carries its job through:
//   INGEST  host-to-device copies, row statistics written straight into
//           pinned memory, an event after them;
//   RUN     format choice from D_mat, the bandwidth, the row lengths and k
//           (the transformed format is allocated only if it fits now, else
//           the job stays in CRS), the optional transformation, the chain of
//           k SpMVs x_{t+1} = 2^-shift A x_t, and the copy of y_k back.
// The device work of a job is the same whatever runs beside it, so its
// result is too.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/spmvat.h"
#include "kernels.h"
#include "plan_internal.h"

#define SPMV_API extern "C" __attribute__((visibility("default")))

using namespace spmvat;

// ------------------------------------------------------------- arena

struct spmv_arena {
    // free blocks: offset -> size, kept coalesced
    std::map<size_t, size_t> free_;
    size_t cap = 0;
    size_t free_bytes = 0;
    static constexpr size_t kGrain = 256;

    explicit spmv_arena(size_t bytes) : cap(bytes / kGrain * kGrain), free_bytes(cap) {
        if (cap) free_[0] = cap;
    }
    static size_t round(size_t b) { return (std::max<size_t>(b, 1) + kGrain - 1) / kGrain * kGrain; }
    int64_t alloc(size_t bytes) {
        const size_t need = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const size_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > need) free_[off + need] = sz - need;
                free_bytes -= need;
                return (int64_t)off;
            }
        }
        return -1;
    }
    void release(int64_t off, size_t bytes) {
        size_t o = (size_t)off, sz = round(bytes);
        free_bytes += sz;
        auto next = free_.lower_bound(o);
        if (next != free_.end() && o + sz == next->first) {
            sz += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == o) {
                prev->second += sz;
                return;
            }
        }
        free_[o] = sz;
    }
    size_t largest() const {
        size_t m = 0;
        for (auto& kv : free_) m = std::max(m, kv.second);
        return m;
    }
};

SPMV_API spmv_arena* spmv_arena_create(size_t bytes) { return new (std::nothrow) spmv_arena(bytes); }
SPMV_API int64_t spmv_arena_alloc(spmv_arena* a, size_t bytes) { return a ? a->alloc(bytes) : -1; }
SPMV_API void spmv_arena_free(spmv_arena* a, int64_t off, size_t bytes) {
    if (a && off >= 0) a->release(off, bytes);
}
SPMV_API size_t spmv_arena_free_bytes(const spmv_arena* a) { return a ? a->free_bytes : 0; }
SPMV_API size_t spmv_arena_largest(const spmv_arena* a) { return a ? a->largest() : 0; }
SPMV_API void spmv_arena_destroy(spmv_arena* a) { delete a; }

// ------------------------------------------------------------- server

namespace {

using Clock = std::chrono::steady_clock;

struct Block {
    int64_t off = -1;
    size_t bytes = 0;
};

// One slot = one HIP stream and one worker thread that carries a job from
// its copies to its result.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    RowStats* host_stats = nullptr;   // pinned, written by the statistics kernel
    std::thread worker;
    bool busy = false;                // a job is assigned (guarded by the server's mutex)
    spmv_job job{};
    spmv_job_result res{};
    spmv_plan plan;
    Block crs, fmt;
    int32_t *irp = nullptr, *icol = nullptr;
    float *val = nullptr, *x = nullptr, *y = nullptr;
    void* pwork = nullptr;
    size_t pwork_bytes = 0;
};

inline size_t r256(size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; }

// Device bytes of a job in CRS: the arrays, x, y and the plan workspace.
size_t crs_footprint(const spmv_job& j) {
    return r256(4 * ((size_t)j.n + 1)) + 2 * r256(4 * (size_t)j.nnz) + 2 * r256(4 * (size_t)j.n) +
           r256(spmv_plan_workspace_bytes(j.n, j.nnz));
}

}  // namespace

struct spmv_server {
    spmv_server_config cfg{};
    int device = 0;
    char* base = nullptr;
    spmv_arena arena{0};
    std::mutex arena_mu;              // the arena is shared by the dispatcher and the workers
    std::vector<Slot> slots;
    std::thread dispatcher;
    std::mutex mu;                    // queues, results, slot assignment
    std::condition_variable cv;       // completions (spmv_server_wait, the dispatcher)
    std::condition_variable work_cv;  // assignments (the workers)
    std::deque<spmv_job> pending;     // submitted, sorted by arrival
    std::deque<spmv_job> ready;       // arrived, FIFO
    std::vector<spmv_job_result> done;
    int64_t submitted = 0, completed = 0;
    std::atomic<bool> stop{false};
    bool started = false;
    Clock::time_point t0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    int64_t arena_alloc(size_t bytes) {
        std::lock_guard<std::mutex> g(arena_mu);
        return arena.alloc(bytes);
    }
    void arena_release(Block& b) {
        if (b.off >= 0) {
            std::lock_guard<std::mutex> g(arena_mu);
            arena.release(b.off, b.bytes);
        }
        b = Block{};
    }

    void report(const spmv_job_result& r) {
        std::lock_guard<std::mutex> g(mu);
        done.push_back(r);
        ++completed;
        cv.notify_all();
    }

    // Ends the slot's job: frees its memory, records the result, frees the slot.
    void finish(Slot& s, int32_t status) {
        arena_release(s.fmt);
        arena_release(s.crs);
        s.res.status = status;
        s.res.done_s = now();
        {
            std::lock_guard<std::mutex> g(mu);
            done.push_back(s.res);
            ++completed;
            s.busy = false;
        }
        cv.notify_all();
    }

    void fail_unadmitted(const spmv_job& j, int32_t status) {
        spmv_job_result r{};
        r.id = j.id;
        r.status = status;
        r.arrival_s = j.arrival_s;
        r.admit_s = r.ready_s = r.done_s = now();
        r.format = -1;
        report(r);
    }

    bool wait_event(Slot& s) { return hipEventSynchronize(s.event) == hipSuccess; }

    // INGEST: copies in (the CRS block was reserved at admission), row
    // statistics written to pinned memory, an event after them.
    spmv_status ingest(Slot& s) {
        const spmv_job& j = s.job;
        char* p = base + s.crs.off;
        s.irp = reinterpret_cast<int32_t*>(p); p += r256(4 * ((size_t)j.n + 1));
        s.icol = reinterpret_cast<int32_t*>(p); p += r256(4 * (size_t)j.nnz);
        s.val = reinterpret_cast<float*>(p); p += r256(4 * (size_t)j.nnz);
        s.x = reinterpret_cast<float*>(p); p += r256(4 * (size_t)j.n);
        s.y = reinterpret_cast<float*>(p); p += r256(4 * (size_t)j.n);
        s.pwork = p;
        s.pwork_bytes = spmv_plan_workspace_bytes(j.n, j.nnz);
        hipError_t e = hipMemcpyAsync(s.irp, j.irp, 4 * ((size_t)j.n + 1), hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && j.nnz > 0)
            e = hipMemcpyAsync(s.icol, j.icol, 4 * (size_t)j.nnz, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && j.nnz > 0)
            e = hipMemcpyAsync(s.val, j.val, 4 * (size_t)j.nnz, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(s.x, j.x0, 4 * (size_t)j.n, hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) return SPMV_E_HIP;
        s.plan = spmv_plan();
        spmv_status st = plan_begin(&s.plan, j.n, j.nnz, s.irp, s.icol, s.val, SPMV_F32, s.pwork, s.pwork_bytes,
                                    s.host_stats, s.stream);
        if (st == SPMV_OK && hipEventRecord(s.event, s.stream) != hipSuccess) st = SPMV_E_HIP;
        return st;
    }

    // RUN: format choice from D_mat, the row lengths and k (the transformed
    // format is allocated only if it fits now, else the job stays in CRS),
    // the optional transformation, the chain, the copy of y_k back.
    spmv_status run(Slot& s) {
        spmv_status st = plan_finish(&s.plan, *s.host_stats);
        if (st != SPMV_OK) return st;
        s.res.ready_s = now();
        s.res.d_mat = s.plan.st.d_mat;
        spmv_format f = SPMV_CRS;
        int v = 1;
        if (cfg.policy == 0) {
            at_decision why{};
            size_t largest;
            {
                std::lock_guard<std::mutex> g(arena_mu);
                largest = arena.largest();
            }
            const size_t limit = std::min(s.plan.limit, largest);
            if (at_choose_format_stats(&s.plan.st, SPMV_F32, limit, &cfg.table, s.job.k, &f, &v, &why) != SPMV_OK) {
                f = SPMV_CRS;
                v = 1;
            }
        }
        if (f != SPMV_CRS) {
            spmv_sizes sz{};
            if (spmv_buffer_sizes(&s.plan, f, &sz) != SPMV_OK) {
                f = SPMV_CRS;
                v = 1;
            } else {
                const size_t need = r256(sz.bytes[0]) + r256(sz.bytes[1]);
                const int64_t off = arena_alloc(need);
                if (off < 0) {
                    f = SPMV_CRS;   // not enough memory now: stay in CRS
                    v = 1;
                } else {
                    s.fmt = Block{off, need};
                    s.res.device_bytes += need;
                    spmv_buffers b{};
                    b.ptr[0] = base + off;
                    b.bytes[0] = sz.bytes[0];
                    b.ptr[1] = base + off + r256(sz.bytes[0]);
                    b.bytes[1] = sz.bytes[1];
                    st = f == SPMV_ELL_ROW ? csr_to_ell(&s.plan, 0, &b, nullptr, 0, s.stream)
                                           : csr_to_coo(&s.plan, 0, &b, nullptr, 0, s.stream);
                    if (st != SPMV_OK) return st;
                }
            }
        }
        s.res.format = (int32_t)f;
        s.res.variant = v;
        // the chain x_{t+1} = 2^-shift A x_t, y_k = A x_k.  CRS and ELL-Row
        // store the scaled product directly (one launch per step, x and y
        // taking turns as input and output); COO-Row adds its carries after
        // the main pass, so it keeps a separate scaling launch
        const bool fused = f == SPMV_CRS || f == SPMV_ELL_ROW;
        const double scale = std::ldexp(1.0, -s.job.shift);
        float* in = s.x;
        float* out = s.y;
        for (int32_t t = 0; t < s.job.k; ++t) {
            const bool last = t + 1 == s.job.k;
            if (fused) {
                st = plan_exec(&s.plan, f, v, in, out, last ? 1.0 : scale, s.stream);
                std::swap(in, out);
            } else {
                st = plan_exec(&s.plan, f, v, s.x, s.y, 1.0, s.stream);
                if (st == SPMV_OK && !last &&
                    launch_scale_pow2(1, s.job.n, s.job.shift, s.y, s.x, s.stream) != hipSuccess)
                    st = SPMV_E_HIP;
                in = s.y;
            }
            if (st != SPMV_OK) return st;
        }
        // `in` holds y_k after the last step in either scheme
        hipError_t e = hipMemcpyAsync(s.job.y_out, in, 4 * (size_t)s.job.n, hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess) e = hipEventRecord(s.event, s.stream);
        return e == hipSuccess ? SPMV_OK : SPMV_E_HIP;
    }

    void work(Slot& s) {
        (void)hipSetDevice(device);
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                work_cv.wait(lk, [&] { return s.busy || stop.load(); });
                if (!s.busy) return;   // stopping, nothing assigned
            }
            spmv_status st = ingest(s);
            if (st == SPMV_OK && !wait_event(s)) st = SPMV_E_HIP;
            if (st == SPMV_OK) st = run(s);
            if (st == SPMV_OK && !wait_event(s)) st = SPMV_E_HIP;
            if (st != SPMV_OK) (void)hipStreamSynchronize(s.stream);
            finish(s, st);
        }
    }

    // Arrivals and admission in arrival order: the head job waits until a
    // slot is free and its CRS block fits in the arena.
    void dispatch() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop.load()) {
            const double t = now();
            while (!pending.empty() && pending.front().arrival_s <= t) {
                ready.push_back(pending.front());
                pending.pop_front();
            }
            bool admitted = false;
            while (!ready.empty()) {
                const spmv_job j = ready.front();
                if (crs_footprint(j) > arena.cap) {
                    ready.pop_front();
                    lk.unlock();
                    fail_unadmitted(j, SPMV_E_TOO_LARGE);
                    lk.lock();
                    continue;
                }
                Slot* free_slot = nullptr;
                for (Slot& sl : slots)
                    if (!sl.busy) { free_slot = &sl; break; }
                if (!free_slot) break;
                const size_t need = crs_footprint(j);
                const int64_t off = arena_alloc(need);
                if (off < 0) break;
                ready.pop_front();
                Slot& sl = *free_slot;
                sl.job = j;
                sl.res = spmv_job_result{};
                sl.res.id = j.id;
                sl.res.arrival_s = j.arrival_s;
                sl.res.admit_s = t;
                sl.res.format = -1;
                sl.res.device_bytes = need;
                sl.crs = Block{off, need};
                sl.fmt = Block{};
                sl.busy = true;
                admitted = true;
            }
            if (admitted) work_cv.notify_all();
            // wake at the next arrival, at a completion, or after a short wait
            double wait_s = 2e-4;
            if (!pending.empty()) wait_s = std::min(wait_s, std::max(0.0, pending.front().arrival_s - now()));
            cv.wait_for(lk, std::chrono::duration<double>(wait_s));
        }
    }
};

SPMV_API spmv_status spmv_server_create(const spmv_server_config* cfg, spmv_server** out) {
    if (!cfg || !out || cfg->slots < 1 || cfg->slots > 64 || cfg->hbm_cap < 4096 || cfg->policy < 0 ||
        cfg->policy > 1)
        return SPMV_E_ARG;
    *out = nullptr;
    spmv_server* s = new (std::nothrow) spmv_server();
    if (!s) return SPMV_E_ARG;
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return SPMV_E_HIP; }
    if (hipMalloc(&s->base, cfg->hbm_cap) != hipSuccess) { delete s; return SPMV_E_TOO_LARGE; }
    s->arena.~spmv_arena();
    new (&s->arena) spmv_arena(cfg->hbm_cap);
    s->slots.resize((size_t)cfg->slots);
    for (Slot& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.event, hipEventDisableTiming | hipEventBlockingSync) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&sl.host_stats), sizeof(RowStats), hipHostMallocCoherent) != hipSuccess) {
            spmv_server_destroy(s);
            return SPMV_E_HIP;
        }
    }
    *out = s;
    return SPMV_OK;
}

SPMV_API spmv_status spmv_server_start(spmv_server* s) {
    if (!s || s->started) return SPMV_E_ARG;
    s->t0 = Clock::now();
    s->started = true;
    for (Slot& sl : s->slots) sl.worker = std::thread([s, &sl] { s->work(sl); });
    s->dispatcher = std::thread([s] { s->dispatch(); });
    return SPMV_OK;
}

SPMV_API spmv_status spmv_server_submit(spmv_server* s, const spmv_job* job) {
    if (!s || !job || job->n < 1 || job->nnz < 0 || job->nnz > SPMV_MAX_NNZ || job->k < 1 || job->shift < 0 ||
        job->shift > 126 || !job->irp || !job->x0 || !job->y_out || (job->nnz > 0 && (!job->icol || !job->val)))
        return SPMV_E_ARG;
    spmv_job j = *job;
    std::lock_guard<std::mutex> g(s->mu);
    if (j.arrival_s < 0) j.arrival_s = s->started ? s->now() : 0.0;
    // keep pending sorted by arrival (submissions normally come in order)
    auto it = s->pending.end();
    while (it != s->pending.begin() && std::prev(it)->arrival_s > j.arrival_s) --it;
    s->pending.insert(it, j);
    ++s->submitted;
    s->cv.notify_all();   // the dispatcher re-reads the queue
    return SPMV_OK;
}

SPMV_API spmv_status spmv_server_wait(spmv_server* s, double timeout_s) {
    if (!s || !s->started) return SPMV_E_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->cv.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                   [s] { return s->completed == s->submitted; });
    return ok ? SPMV_OK : SPMV_E_NOT_READY;
}

SPMV_API int32_t spmv_server_results(spmv_server* s, spmv_job_result* out, int32_t cap) {
    if (!s || !out || cap <= 0) return 0;
    std::lock_guard<std::mutex> g(s->mu);
    const int32_t m = (int32_t)std::min<size_t>((size_t)cap, s->done.size());
    std::memcpy(out, s->done.data(), sizeof(spmv_job_result) * (size_t)m);
    return m;
}

SPMV_API void spmv_server_destroy(spmv_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop.store(true);
    }
    s->cv.notify_all();
    s->work_cv.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    // a worker finishes the job it holds, then sees the stop flag
    for (Slot& sl : s->slots)
        if (sl.worker.joinable()) sl.worker.join();
    for (Slot& sl : s->slots) {
        if (sl.stream) { (void)hipStreamSynchronize(sl.stream); (void)hipStreamDestroy(sl.stream); }
        if (sl.event) (void)hipEventDestroy(sl.event);
        if (sl.host_stats) (void)hipHostFree(sl.host_stats);
    }
    if (s->base) (void)hipFree(s->base);
    delete s;
}
