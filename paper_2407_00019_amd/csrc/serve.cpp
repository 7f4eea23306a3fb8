// Continuous-batching SpMV server: the auto-tuner of section 2.2 applied per
// request, with the transformation amortised over the request's declared
// number of SpMVs (the iteration-count discussion after the on-line phase).
//
// A dispatcher thread makes jobs visible at their arrival time and admits
// them in FIFO order: the head job waits until an ingest slot is free and
// its CRS and vector blocks fit in the device arena.  Each slot (one HIP
// stream, one worker thread) carries its job through
//   INGEST  host-to-device copies, row statistics written straight into
//           pinned memory, an event after them;
//   PREPARE format choice from D_mat, the bandwidth, the row lengths and k
//           (CRS or ELL-Row; the converted format is allocated only if it
//           fits now, else the job stays in CRS) and the conversion; under
//           policy 2 a converted job then gives back its CRS arrays;
// and hands it to the engine.  The engine thread runs every job it holds in
// lock step: each tick is one launch of the batched step kernel, which
// advances the chain x_{t+1} = 2^-shift A x_t of every running job by one
// SpMV, each job in its own format; jobs join and leave between ticks.  A
// job's last tick also copies y_k back; a reaper thread waits for the
// ticks in order, reports the jobs they finished and frees their memory.
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
#include "host_core.h"
#include "kernels.h"
#include "plan_internal.h"

#define SPMV_API extern "C" __attribute__((visibility("default")))

using namespace spmvat;

// ------------------------------------------------------------- server

namespace {

using Clock = std::chrono::steady_clock;

struct Block {
    int64_t off = -1;
    size_t bytes = 0;
};

inline size_t r256(size_t b) { return (std::max<size_t>(b, 1) + 255) / 256 * 256; }

// Device bytes of a job's CRS block (the arrays and the plan workspace) and
// of its vector block (x and y).
size_t mat_footprint(const spmv_job& j) {
    return r256(4 * ((size_t)j.n + 1)) + 2 * r256(4 * (size_t)j.nnz) + r256(spmv_plan_workspace_bytes(j.n, j.nnz));
}
size_t vec_footprint(const spmv_job& j) { return 2 * r256(4 * (size_t)j.n); }

// One job from admission to its report.
struct JobState {
    spmv_job job{};
    spmv_job_result res{};
    Block mat, vec, fmt;
    int32_t *irp = nullptr, *icol = nullptr;
    float *val = nullptr, *x = nullptr, *y = nullptr;
    void* pwork = nullptr;
    size_t pwork_bytes = 0;
    spmv_plan plan;
    // the chain in the engine
    int kind = kServeCrs, param = 1, rows_per_item = kServeThreads;
    const int32_t* a0 = nullptr;
    const int32_t* a1 = nullptr;
    const float* v = nullptr;
    int32_t step = 0;
};

// One ingest slot: a HIP stream and a worker thread.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t event = nullptr;
    RowStats* host_stats = nullptr;   // pinned, written by the statistics kernel
    std::thread worker;
    JobState* job = nullptr;          // assigned job (guarded by the server's mutex)
};

// A tick handed to the reaper: its event and the jobs it finished.
struct Tick {
    int64_t index;
    std::vector<JobState*> finished;
};

constexpr int kTickEvents = 64;          // events of the ticks, reused in a ring
constexpr int kRing = 3;                 // host descriptor buffers (at most 2 ticks in flight)
constexpr int kMaxTickJobs = 4096;       // jobs one tick advances at most
constexpr int kMaxCoarse = 1 << 16;      // coarse map entries: 4M work items per tick at most
constexpr size_t kDescBytes = (size_t)kMaxTickJobs * sizeof(ServeStep) + (size_t)kMaxCoarse * 4;

}  // namespace

struct spmv_server {
    spmv_server_config cfg{};
    at_table table{};                 // cfg.table without the COO-Row rates (the step kernel runs CRS and ELL-Row)
    int device = 0;
    char* base = nullptr;
    spmv_arena arena{0};
    std::mutex arena_mu;              // the arena is shared by every thread
    std::vector<Slot> slots;
    std::thread dispatcher, engine, reaper;
    std::mutex mu;                    // queues, results, slot assignment
    std::condition_variable cv;       // completions and freed slots (spmv_server_wait, the dispatcher)
    std::condition_variable work_cv;  // assignments (the slot workers)
    std::condition_variable engine_cv;
    std::condition_variable reap_cv;
    std::deque<spmv_job> pending;     // submitted, sorted by arrival
    std::deque<spmv_job> ready;       // arrived, FIFO
    std::deque<JobState*> inbox;      // prepared jobs waiting for the engine
    std::deque<Tick> reap;            // ticks waiting for the reaper
    std::vector<spmv_job_result> done;
    int64_t submitted = 0, completed = 0;
    int64_t reaped_ticks = 0;         // ticks the reaper has finished with
    std::atomic<bool> stop{false};    // dispatcher and slots
    bool engine_drain = false;        // the slots are gone: the engine ends once its jobs are done
    bool reaper_drain = false;        // the engine is gone: the reaper ends once its ticks are done
    bool started = false;
    Clock::time_point t0;
    // engine resources
    hipStream_t estream = nullptr;
    hipEvent_t tick_ev[kTickEvents] = {};
    char* host_ring[kRing] = {};
    char* dev_desc = nullptr;

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

    // Frees a job's memory and records its result.
    void finish(JobState* js, int32_t status) {
        arena_release(js->fmt);
        arena_release(js->mat);
        arena_release(js->vec);
        js->res.status = status;
        js->res.done_s = now();
        {
            std::lock_guard<std::mutex> g(mu);
            done.push_back(js->res);
            ++completed;
        }
        cv.notify_all();
        delete js;
    }

    void fail_unadmitted(const spmv_job& j, int32_t status) {
        spmv_job_result r{};
        r.id = j.id;
        r.status = status;
        r.arrival_s = j.arrival_s;
        r.admit_s = r.ready_s = r.done_s = now();
        r.format = -1;
        std::lock_guard<std::mutex> g(mu);
        done.push_back(r);
        ++completed;
        cv.notify_all();
    }

    // INGEST: copies in (the blocks were reserved at admission), row
    // statistics written to pinned memory; waits for them.
    spmv_status ingest(Slot& s, JobState& js) {
        const spmv_job& j = js.job;
        char* p = base + js.mat.off;
        js.irp = reinterpret_cast<int32_t*>(p); p += r256(4 * ((size_t)j.n + 1));
        js.icol = reinterpret_cast<int32_t*>(p); p += r256(4 * (size_t)j.nnz);
        js.val = reinterpret_cast<float*>(p); p += r256(4 * (size_t)j.nnz);
        js.pwork = p;
        js.pwork_bytes = spmv_plan_workspace_bytes(j.n, j.nnz);
        char* q = base + js.vec.off;
        js.x = reinterpret_cast<float*>(q); q += r256(4 * (size_t)j.n);
        js.y = reinterpret_cast<float*>(q);
        hipError_t e = hipMemcpyAsync(js.irp, j.irp, 4 * ((size_t)j.n + 1), hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && j.nnz > 0)
            e = hipMemcpyAsync(js.icol, j.icol, 4 * (size_t)j.nnz, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && j.nnz > 0)
            e = hipMemcpyAsync(js.val, j.val, 4 * (size_t)j.nnz, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(js.x, j.x0, 4 * (size_t)j.n, hipMemcpyHostToDevice, s.stream);
        if (e != hipSuccess) return SPMV_E_HIP;
        js.plan = spmv_plan();
        spmv_status st = plan_begin(&js.plan, j.n, j.nnz, js.irp, js.icol, js.val, SPMV_F32, js.pwork,
                                    js.pwork_bytes, s.host_stats, s.stream);
        if (st == SPMV_OK && hipEventRecord(s.event, s.stream) != hipSuccess) st = SPMV_E_HIP;
        if (st == SPMV_OK && hipEventSynchronize(s.event) != hipSuccess) st = SPMV_E_HIP;
        return st;
    }

    // PREPARE: the format (CRS or ELL-Row) and its conversion; under
    // policy 2 a converted job gives back its CRS block.
    spmv_status prepare(Slot& s, JobState& js) {
        spmv_status st = plan_finish(&js.plan, *s.host_stats);
        if (st != SPMV_OK) return st;
        js.res.d_mat = js.plan.st.d_mat;
        spmv_format f = SPMV_CRS;
        int v = 1;
        if (cfg.policy != 1) {
            at_decision why{};
            size_t largest;
            {
                std::lock_guard<std::mutex> g(arena_mu);
                largest = arena.largest();
            }
            const size_t limit = std::min(js.plan.limit, largest);
            if (at_choose_format_stats(&js.plan.st, SPMV_F32, limit, &table, js.job.k, &f, &v, &why) != SPMV_OK ||
                f != SPMV_ELL_ROW) {
                f = SPMV_CRS;
                v = 1;
            }
        }
        if (f == SPMV_ELL_ROW) {
            spmv_sizes sz{};
            if (spmv_buffer_sizes(&js.plan, f, &sz) != SPMV_OK) {
                f = SPMV_CRS;
            } else {
                const size_t need = r256(sz.bytes[0]) + r256(sz.bytes[1]);
                const int64_t off = arena_alloc(need);
                if (off < 0) {
                    f = SPMV_CRS;   // not enough memory now: stay in CRS
                } else {
                    js.fmt = Block{off, need};
                    spmv_buffers b{};
                    b.ptr[0] = base + off;
                    b.bytes[0] = sz.bytes[0];
                    b.ptr[1] = base + off + r256(sz.bytes[0]);
                    b.bytes[1] = sz.bytes[1];
                    st = csr_to_ell(&js.plan, 0, &b, nullptr, 0, s.stream);
                    if (st != SPMV_OK) return st;
                    if (hipEventRecord(s.event, s.stream) != hipSuccess || hipEventSynchronize(s.event) != hipSuccess)
                        return SPMV_E_HIP;
                    js.kind = kServeEll;
                    js.param = sz.width;
                    js.rows_per_item = kServeThreads;
                    js.a0 = static_cast<const int32_t*>(b.ptr[1]);
                    js.v = static_cast<const float*>(b.ptr[0]);
                    js.res.device_bytes = js.mat.bytes + js.vec.bytes + js.fmt.bytes;
                    if (cfg.policy == 2) arena_release(js.mat);   // the memory policy: CRS is no longer needed
                }
            }
        }
        if (f == SPMV_CRS) {
            js.kind = kServeCrs;
            js.param = serve_crs_lanes(js.job.n, js.job.nnz);
            js.rows_per_item = kServeThreads / js.param;
            js.a0 = js.irp;
            js.a1 = js.icol;
            js.v = js.val;
        }
        js.res.format = (int32_t)f;
        js.res.variant = f == SPMV_CRS ? 1 : 0;
        if (f == SPMV_CRS) js.res.device_bytes = js.mat.bytes + js.vec.bytes;
        // a job whose step alone exceeds a tick's work items could never run
        const int64_t items = ((int64_t)js.job.n + js.rows_per_item - 1) / js.rows_per_item;
        if (items > ((int64_t)kMaxCoarse << kServeCoarseBits)) return SPMV_E_TOO_LARGE;
        js.res.ready_s = now();   // its format is built: the job goes to the engine
        return SPMV_OK;
    }

    void work(Slot& s) {
        (void)hipSetDevice(device);
        for (;;) {
            JobState* js;
            {
                std::unique_lock<std::mutex> lk(mu);
                work_cv.wait(lk, [&] { return s.job != nullptr || stop.load(); });
                if (!s.job) return;   // stopping, nothing assigned
                js = s.job;
            }
            spmv_status st = ingest(s, *js);
            if (st == SPMV_OK) st = prepare(s, *js);
            if (st != SPMV_OK) {
                (void)hipStreamSynchronize(s.stream);
                finish(js, st);
            } else {
                std::lock_guard<std::mutex> g(mu);
                inbox.push_back(js);
            }
            {
                std::lock_guard<std::mutex> g(mu);
                s.job = nullptr;
            }
            engine_cv.notify_all();
            cv.notify_all();   // the dispatcher may admit the next job
        }
    }

    // The engine: one batched step per tick over every job it holds.
    void run_engine() {
        (void)hipSetDevice(device);
        std::vector<JobState*> active;
        int64_t tick = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                engine_cv.wait(lk, [&] { return !inbox.empty() || !active.empty() || engine_drain; });
                while (!inbox.empty()) {
                    active.push_back(inbox.front());
                    inbox.pop_front();
                }
                if (active.empty()) return;   // draining and nothing left
                // the event of tick - kTickEvents is reused below: the reaper must be past it
                engine_cv.wait(lk, [&] { return reaped_ticks > tick - kTickEvents; });
            }
            // at most two ticks in flight; the descriptor buffer of tick - 3 is free
            if (tick >= 2 && hipEventSynchronize(tick_ev[(tick - 2) % kTickEvents]) != hipSuccess) {
                fail_all(active);
                return;
            }
            char* hb = host_ring[tick % kRing];
            ServeStep* desc = reinterpret_cast<ServeStep*>(hb);
            int* coarse = reinterpret_cast<int*>(hb + (size_t)kMaxTickJobs * sizeof(ServeStep));
            // the jobs of this tick, in the order they joined, within the capacities
            int nj = 0;
            int64_t items = 0;
            std::vector<JobState*> in_tick, later;
            for (JobState* js : active) {
                const int64_t it = ((int64_t)js->job.n + js->rows_per_item - 1) / js->rows_per_item;
                if (nj >= kMaxTickJobs || items + it > ((int64_t)kMaxCoarse << kServeCoarseBits)) {
                    later.push_back(js);
                    continue;
                }
                const int t = js->step;
                const bool last = t + 1 == js->job.k;
                ServeStep& d = desc[nj];
                d.a0 = js->a0;
                d.a1 = js->a1;
                d.val = js->v;
                d.x = (t & 1) ? js->y : js->x;
                d.y = (t & 1) ? js->x : js->y;
                d.n = js->job.n;
                d.kind = js->kind;
                d.param = js->param;
                d.item0 = (int32_t)items;
                d.rows_per_item = js->rows_per_item;
                d.alpha = last ? 1.0f : std::ldexp(1.0f, -js->job.shift);
                items += it;
                ++nj;
                in_tick.push_back(js);
            }
            int ji = 0;
            const int ncoarse = (int)((items + (1 << kServeCoarseBits) - 1) >> kServeCoarseBits);
            for (int g = 0; g < ncoarse; ++g) {
                const int64_t first = (int64_t)g << kServeCoarseBits;
                while (ji + 1 < nj && desc[ji + 1].item0 <= first) ++ji;
                coarse[g] = ji;
            }
            ServeStep* ddesc = reinterpret_cast<ServeStep*>(dev_desc);
            int* dcoarse = reinterpret_cast<int*>(dev_desc + (size_t)kMaxTickJobs * sizeof(ServeStep));
            hipError_t e = hipMemcpyAsync(ddesc, desc, (size_t)nj * sizeof(ServeStep), hipMemcpyHostToDevice, estream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(dcoarse, coarse, (size_t)ncoarse * 4, hipMemcpyHostToDevice, estream);
            if (e == hipSuccess) e = launch_serve_step(ddesc, nj, dcoarse, (int)items, estream);
            Tick tk{tick, {}};
            std::vector<JobState*> next = later;
            for (JobState* js : in_tick) {
                const int t = js->step++;
                if (js->step == js->job.k) {
                    float* out = (t & 1) ? js->x : js->y;
                    if (e == hipSuccess)
                        e = hipMemcpyAsync(js->job.y_out, out, 4 * (size_t)js->job.n, hipMemcpyDeviceToHost, estream);
                    tk.finished.push_back(js);
                } else {
                    next.push_back(js);
                }
            }
            if (e == hipSuccess) e = hipEventRecord(tick_ev[tick % kTickEvents], estream);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(estream);
                for (JobState* js : tk.finished) finish(js, SPMV_E_HIP);
                fail_all(next);
                return;
            }
            active.swap(next);
            {
                std::lock_guard<std::mutex> g(mu);
                reap.push_back(std::move(tk));
            }
            reap_cv.notify_all();
            ++tick;
        }
    }

    // Ends jobs the engine can no longer run (a HIP error), and every job
    // still waiting for it.
    void fail_all(std::vector<JobState*>& jobs) {
        for (JobState* js : jobs) finish(js, SPMV_E_HIP);
        jobs.clear();
        std::deque<JobState*> rest;
        {
            std::lock_guard<std::mutex> g(mu);
            rest.swap(inbox);
            engine_failed = true;
        }
        for (JobState* js : rest) finish(js, SPMV_E_HIP);
    }
    bool engine_failed = false;

    // The reaper: ticks in order; each one's jobs are done when its event is.
    void run_reaper() {
        (void)hipSetDevice(device);
        for (;;) {
            Tick tk;
            {
                std::unique_lock<std::mutex> lk(mu);
                reap_cv.wait(lk, [&] { return !reap.empty() || reaper_drain; });
                if (reap.empty()) return;
                tk = std::move(reap.front());
                reap.pop_front();
            }
            const bool ok = hipEventSynchronize(tick_ev[tk.index % kTickEvents]) == hipSuccess;
            for (JobState* js : tk.finished) finish(js, ok ? SPMV_OK : SPMV_E_HIP);
            {
                std::lock_guard<std::mutex> g(mu);
                reaped_ticks = tk.index + 1;
            }
            engine_cv.notify_all();
        }
    }

    // Arrivals and admission in arrival order: the head job waits until a
    // slot is free and its CRS and vector blocks fit in the arena.
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
                const size_t need_mat = mat_footprint(j), need_vec = vec_footprint(j);
                if (r256(need_mat) + r256(need_vec) > arena.cap || engine_failed) {
                    ready.pop_front();
                    lk.unlock();
                    fail_unadmitted(j, engine_failed ? SPMV_E_HIP : SPMV_E_TOO_LARGE);
                    lk.lock();
                    continue;
                }
                Slot* free_slot = nullptr;
                for (Slot& sl : slots)
                    if (!sl.job) { free_slot = &sl; break; }
                if (!free_slot) break;
                const int64_t om = arena_alloc(need_mat);
                if (om < 0) break;
                const int64_t ov = arena_alloc(need_vec);
                if (ov < 0) {
                    Block b{om, need_mat};
                    arena_release(b);
                    break;
                }
                ready.pop_front();
                JobState* js = new JobState();
                js->job = j;
                js->res.id = j.id;
                js->res.arrival_s = j.arrival_s;
                js->res.admit_s = t;
                js->res.format = -1;
                js->mat = Block{om, need_mat};
                js->vec = Block{ov, need_vec};
                free_slot->job = js;
                admitted = true;
            }
            if (admitted) work_cv.notify_all();
            // wake at the next arrival, at a completion or a freed slot, or after a short wait
            double wait_s = 2e-4;
            if (!pending.empty()) wait_s = std::min(wait_s, std::max(0.0, pending.front().arrival_s - now()));
            cv.wait_for(lk, std::chrono::duration<double>(wait_s));
        }
    }
};

SPMV_API spmv_status spmv_server_create(const spmv_server_config* cfg, spmv_server** out) {
    if (!cfg || !out || cfg->slots < 1 || cfg->slots > 64 || cfg->hbm_cap < 4096 || cfg->policy < 0 ||
        cfg->policy > 2)
        return SPMV_E_ARG;
    *out = nullptr;
    spmv_server* s = new (std::nothrow) spmv_server();
    if (!s) return SPMV_E_ARG;
    s->cfg = *cfg;
    // the step kernel runs CRS and ELL-Row: the chooser sees no COO-Row rates
    s->table = cfg->table;
    for (int loc = 0; loc < 2; ++loc) {
        for (int v = 0; v < 2; ++v)
            for (int b = 0; b < AT_DBUCKETS; ++b) s->table.spmv_bps[loc][SPMV_COO_ROW][v][b] = 0.0;
        for (int b = 0; b < AT_DBUCKETS; ++b) s->table.trans_bps[loc][SPMV_COO_ROW][b] = 0.0;
    }
    if (hipGetDevice(&s->device) != hipSuccess) { delete s; return SPMV_E_HIP; }
    if (hipMalloc(&s->base, cfg->hbm_cap) != hipSuccess) { delete s; return SPMV_E_TOO_LARGE; }
    s->arena.~spmv_arena();
    new (&s->arena) spmv_arena(cfg->hbm_cap);
    bool ok = hipStreamCreateWithFlags(&s->estream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc(&s->dev_desc, kDescBytes) == hipSuccess;
    for (int i = 0; ok && i < kTickEvents; ++i)
        ok = hipEventCreateWithFlags(&s->tick_ev[i], hipEventDisableTiming | hipEventBlockingSync) == hipSuccess;
    for (int i = 0; ok && i < kRing; ++i)
        ok = hipHostMalloc(reinterpret_cast<void**>(&s->host_ring[i]), kDescBytes, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
        spmv_server_destroy(s);
        return SPMV_E_HIP;
    }
    s->slots = std::vector<Slot>((size_t)cfg->slots);
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
    s->engine = std::thread([s] { s->run_engine(); });
    s->reaper = std::thread([s] { s->run_reaper(); });
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
    // a slot finishes the job it holds (handing it to the engine), then sees the stop flag
    for (Slot& sl : s->slots)
        if (sl.worker.joinable()) sl.worker.join();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->engine_drain = true;
    }
    s->engine_cv.notify_all();
    if (s->engine.joinable()) s->engine.join();
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->reaper_drain = true;
    }
    s->reap_cv.notify_all();
    if (s->reaper.joinable()) s->reaper.join();
    for (Slot& sl : s->slots) {
        if (sl.stream) { (void)hipStreamSynchronize(sl.stream); (void)hipStreamDestroy(sl.stream); }
        if (sl.event) (void)hipEventDestroy(sl.event);
        if (sl.host_stats) (void)hipHostFree(sl.host_stats);
    }
    if (s->estream) { (void)hipStreamSynchronize(s->estream); (void)hipStreamDestroy(s->estream); }
    for (int i = 0; i < kTickEvents; ++i)
        if (s->tick_ev[i]) (void)hipEventDestroy(s->tick_ev[i]);
    for (int i = 0; i < kRing; ++i)
        if (s->host_ring[i]) (void)hipHostFree(s->host_ring[i]);
    if (s->dev_desc) (void)hipFree(s->dev_desc);
    if (s->base) (void)hipFree(s->base);
    delete s;
}
