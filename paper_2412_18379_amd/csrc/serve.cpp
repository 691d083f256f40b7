// Serving loop: CNN-SNS tracking jobs on resident meshes, continuous batching.
//
// A job is one CNN forward pass over its mesh's overlay (the prediction step
// of Alg. 2) followed by the CNN-SNS walk of its points (Alg. 1 from the
// predicted start), exactly what cnnsns_predict + cnnsns_locate compute.
// Meshes (elements, neighbours, overlay lookups) stay resident; the weights
// are copied and prepared once when the server is created.
//
// Scheduling: jobs wait in a FIFO queue.  A scheduler thread admits them in
// arrival order while their device footprint (the displacement grid, plus
// the FP32 activation workspace when the CNN runs in FP32) can be carved out
// of a device arena of hbm_budget bytes and fewer than max_inflight jobs are
// on the device.  Each scheduling round captures the newly admitted jobs
// into one hipGraph, one parallel branch per job (forward pass, then walk),
// and launches it on the next stream of a small pool; rounds overlap with
// earlier rounds still running, so jobs that arrive while others execute are
// admitted as soon as memory and slots free up.  Completion is observed with
// events; it releases the job's arena block and stamps its latency.
#include "serve.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <vector>

namespace cnnsns {
namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;

inline size_t align_up(size_t n)
{
    return (n + kAlign - 1) / kAlign * kAlign;
}

// First-fit allocator over one device allocation.
class Arena {
public:
    Arena(char* base, size_t size) : base_(base) { free_[0] = size; }
    // offset of a block of n bytes, or -1 when nothing fits
    int64_t alloc(size_t n)
    {
        n = align_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const size_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return (int64_t)off;
            }
        }
        return -1;
    }
    void release(size_t off, size_t n)
    {
        n = align_up(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char* at(size_t off) const { return base_ + off; }

private:
    char* base_;
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Job {
    uint64_t id = 0;
    cnnsns_mesh mesh = nullptr;
    const float* vel = nullptr;
    int64_t n = 0;
    const double* xp = nullptr;
    const double* origin = nullptr;
    const int32_t* start = nullptr;
    int32_t* host = nullptr;
    int32_t* iters = nullptr;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream: the job's inputs are written
    size_t footprint = 0;
    int64_t arena_off = -1;
    Clock::time_point t_submit, t_done;
    bool done = false;
    int error = CNNSNS_OK;
};

struct Batch {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    std::vector<uint64_t> jobs;
};

}  // namespace
}  // namespace cnnsns

struct cnnsns_server_s {
    int device = 0;
    int32_t precision = CNNSNS_BF16;
    int32_t max_inflight = 1;
    int32_t queue_depth = 1;
    // weights: device copies of the caller's FP32 tensors, and the prepared form
    float* wbuf = nullptr;
    cnnsns_cnn w{};
    void* packed = nullptr;  // BF16 packed weights (prepared once)
    char* arena_mem = nullptr;
    int64_t budget = 0;
    std::unique_ptr<cnnsns::Arena> arena;
    std::vector<hipStream_t> streams;
    hipStream_t capture = nullptr;
    std::vector<hipStream_t> branch;  // fork streams used while capturing
    hipEvent_t fork = nullptr;        // fork / join events of a capture (created once)
    std::vector<hipEvent_t> joins;
    size_t next_stream = 0;

    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::deque<uint64_t> queue;
    std::map<uint64_t, cnnsns::Job> jobs;
    std::deque<cnnsns::Batch> running;
    int32_t inflight = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread thread;
    std::string thread_error;
};

namespace cnnsns {
namespace {

size_t job_footprint(const cnnsns_server_s& s, const cnnsns_mesh_s& m)
{
    size_t b = align_up(sizeof(float) * 2 * (size_t)m.G * (size_t)m.G);  // displacement grid
    if (s.precision == CNNSNS_F32) b += align_up(cnn_workspace_bytes(m.G, CNNSNS_F32));
    return b;
}

// Record the forward pass and walk of one job on stream st (inside a capture).
void enqueue_job(cnnsns_server_s& s, const Job& j, hipStream_t st)
{
    char* base = s.arena->at((size_t)j.arena_off);
    float* disp = reinterpret_cast<float*>(base);
    const cnnsns_mesh_s& m = *j.mesh;
    if (s.precision == CNNSNS_BF16) {
        cnn_bf16_forward(m.G, j.vel, s.packed, s.w, disp, cnn_persistent_grid(), st);
    } else {
        void* ws = base + align_up(sizeof(float) * 2 * (size_t)m.G * (size_t)m.G);
        run_cnn(m.G, j.vel, s.w, CNNSNS_F32, disp, ws, st);
    }
    if (j.n > 0) launch_locate(m, j.n, j.xp, j.start, j.origin, disp, 0, j.host, j.iters, nullptr, st);
}

// Capture the jobs into one graph, one parallel branch per job, and launch it.
void launch_batch(cnnsns_server_s& s, const std::vector<uint64_t>& ids)
{
    Batch b;
    b.jobs = ids;
    struct Guard {  // frees the batch's graph objects unless it was handed to the running list
        Batch& b;
        bool armed = true;
        ~Guard()
        {
            if (!armed) return;
            if (b.exec) (void)hipGraphExecDestroy(b.exec);
            if (b.graph) (void)hipGraphDestroy(b.graph);
            if (b.done) (void)hipEventDestroy(b.done);
        }
    } guard{ b };
    const size_t nb = std::min(ids.size(), s.branch.size());
    hip_check(hipStreamBeginCapture(s.capture, hipStreamCaptureModeRelaxed), "begin capture");
    try {
        hip_check(hipEventRecord(s.fork, s.capture), "fork");
        for (size_t k = 0; k < nb; ++k) hip_check(hipStreamWaitEvent(s.branch[k], s.fork, 0), "fork wait");
        for (size_t k = 0; k < ids.size(); ++k) enqueue_job(s, s.jobs.at(ids[k]), s.branch[k % s.branch.size()]);
        for (size_t k = 0; k < nb; ++k) {
            hip_check(hipEventRecord(s.joins[k], s.branch[k]), "join record");
            hip_check(hipStreamWaitEvent(s.capture, s.joins[k], 0), "join wait");
        }
        hip_check(hipStreamEndCapture(s.capture, &b.graph), "end capture");
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(s.capture, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hip_check(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0), "graph instantiate");
    hip_check(hipEventCreateWithFlags(&b.done, hipEventDisableTiming), "event");
    hipStream_t st = s.streams[s.next_stream++ % s.streams.size()];
    // the batch starts once every job's inputs, written on its submitter's stream, are ready
    for (uint64_t id : ids) hip_check(hipStreamWaitEvent(st, s.jobs.at(id).ready, 0), "wait for job inputs");
    hip_check(hipGraphLaunch(b.exec, st), "graph launch");
    if (hipEventRecord(b.done, st) != hipSuccess) {
        // the graph is running: its jobs' memory may only be released once it has finished
        (void)hipStreamSynchronize(st);
        fail(CNNSNS_EHIP, "serve: cannot record the completion event of a batch");
    }
    s.running.push_back(b);
    guard.armed = false;
}

void release_batch(cnnsns_server_s& s, Batch& b, Clock::time_point now, int err)
{
    for (uint64_t id : b.jobs) {
        Job& j = s.jobs.at(id);
        s.arena->release((size_t)j.arena_off, j.footprint);
        if (j.ready) (void)hipEventDestroy(j.ready);
        j.ready = nullptr;
        j.mesh->pending_jobs.fetch_sub(1);
        j.done = true;
        j.error = err;
        j.t_done = now;
        --s.inflight;
    }
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    if (b.done) (void)hipEventDestroy(b.done);
}

void scheduler(cnnsns_server_s* sp)
{
    cnnsns_server_s& s = *sp;
    (void)hipSetDevice(s.device);
    std::unique_lock<std::mutex> lock(s.mu);
    for (;;) {
        // completions, oldest first (they may also finish out of order)
        bool progressed = false;
        for (auto it = s.running.begin(); it != s.running.end();) {
            hipError_t q = hipEventQuery(it->done);
            if (q == hipErrorNotReady) {
                ++it;
                continue;
            }
            release_batch(s, *it, Clock::now(), q == hipSuccess ? CNNSNS_OK : CNNSNS_EHIP);
            it = s.running.erase(it);
            progressed = true;
        }
        if (progressed) s.cv_done.notify_all();
        // admission in arrival order
        std::vector<uint64_t> admit;
        while (!s.queue.empty() && s.inflight < s.max_inflight) {
            Job& j = s.jobs.at(s.queue.front());
            const int64_t off = s.arena->alloc(j.footprint);
            if (off < 0) break;  // wait for memory to free up
            j.arena_off = off;
            admit.push_back(j.id);
            s.queue.pop_front();
            ++s.inflight;
        }
        if (!admit.empty()) {
            try {
                launch_batch(s, admit);
            } catch (const Error& e) {
                s.thread_error = e.msg;
                Batch b;
                b.jobs = admit;
                release_batch(s, b, Clock::now(), e.code);
                s.cv_done.notify_all();
            }
            continue;
        }
        if (s.stop && s.queue.empty() && s.running.empty()) break;
        if (s.running.empty())
            s.cv_sched.wait(lock, [&] { return s.stop || !s.queue.empty(); });
        else
            s.cv_sched.wait_for(lock, std::chrono::microseconds(20));
    }
}

}  // namespace

cnnsns_server server_create(int64_t hbm_budget_bytes, int32_t max_inflight, int32_t queue_depth, int32_t precision,
                            const cnnsns_cnn* w)
{
    if (!w) fail(CNNSNS_EINVAL, "server_create: NULL weights");
    for (int l = 0; l < 4; ++l)
        if (!w->w[l] || !w->b[l]) fail(CNNSNS_EINVAL, "server_create: NULL weight or bias pointer");
    if (hbm_budget_bytes <= 0 || max_inflight < 1 || queue_depth < 1)
        fail(CNNSNS_EINVAL, "server_create: budget, max_inflight and queue_depth must be positive");
    if (precision != CNNSNS_F32 && precision != CNNSNS_BF16)
        fail(CNNSNS_EINVAL, "server_create: precision must be CNNSNS_F32 or CNNSNS_BF16");
    auto s = std::make_unique<cnnsns_server_s>();
    hip_check(hipGetDevice(&s->device), "hipGetDevice");
    s->precision = precision;
    s->max_inflight = max_inflight;
    s->queue_depth = queue_depth;
    s->budget = hbm_budget_bytes;
    const size_t wsz[4] = { 32 * 2 * 9, 32 * 32 * 9, 32 * 32 * 9, 2 * 32 * 9 }, bsz[4] = { 32, 32, 32, 2 };
    size_t total = 0;
    for (int l = 0; l < 4; ++l) total += wsz[l] + bsz[l];
    struct Cleanup {
        cnnsns_server_s* s;
        bool armed = true;
        ~Cleanup()
        {
            if (!armed) return;
            if (s->wbuf) (void)hipFree(s->wbuf);
            if (s->packed) (void)hipFree(s->packed);
            if (s->arena_mem) (void)hipFree(s->arena_mem);
            for (auto st : s->streams) (void)hipStreamDestroy(st);
            for (auto st : s->branch) (void)hipStreamDestroy(st);
            if (s->capture) (void)hipStreamDestroy(s->capture);
            if (s->fork) (void)hipEventDestroy(s->fork);
            for (auto e : s->joins) (void)hipEventDestroy(e);
        }
    } cleanup{ s.get() };
    hip_check(hipMalloc(&s->wbuf, total * sizeof(float)), "weights");
    float* p = s->wbuf;
    for (int l = 0; l < 4; ++l) {
        hip_check(hipMemcpy(p, w->w[l], wsz[l] * sizeof(float), hipMemcpyDeviceToDevice), "copy weights");
        s->w.w[l] = p;
        p += wsz[l];
        hip_check(hipMemcpy(p, w->b[l], bsz[l] * sizeof(float), hipMemcpyDeviceToDevice), "copy biases");
        s->w.b[l] = p;
        p += bsz[l];
    }
    if (precision == CNNSNS_BF16) {
        hip_check(hipMalloc(&s->packed, cnn_bf16_workspace_bytes()), "packed weights");
        cnn_bf16_pack(s->w, s->packed, nullptr);
    }
    if (hipMalloc(&s->arena_mem, (size_t)hbm_budget_bytes) != hipSuccess) {
        (void)hipGetLastError();
        fail(CNNSNS_ENOMEM, "server_create: cannot allocate the device budget");
    }
    s->arena = std::make_unique<Arena>(s->arena_mem, (size_t)hbm_budget_bytes);
    const int nstreams = std::max(2, std::min(4, (int)max_inflight));
    for (int k = 0; k < nstreams; ++k) {
        hipStream_t st;
        hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
        s->streams.push_back(st);
    }
    const int nbranch = std::max(1, std::min(8, (int)max_inflight));
    for (int k = 0; k < nbranch; ++k) {
        hipStream_t st;
        hip_check(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream");
        s->branch.push_back(st);
    }
    hip_check(hipStreamCreateWithFlags(&s->capture, hipStreamNonBlocking), "stream");
    hip_check(hipEventCreateWithFlags(&s->fork, hipEventDisableTiming), "event");
    for (int k = 0; k < nbranch; ++k) {
        hipEvent_t e;
        hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
        s->joins.push_back(e);
    }
    hip_check(hipDeviceSynchronize(), "server setup");
    s->thread = std::thread(scheduler, s.get());
    cleanup.armed = false;
    return s.release();
}

uint64_t server_submit(cnnsns_server s, cnnsns_mesh m, const float* vel, int64_t n, const double* xp,
                       const double* origin, const int32_t* start, int32_t* host, int32_t* iters,
                       hipStream_t stream)
{
    if (m->device != s->device) fail(CNNSNS_EINVAL, "submit: mesh and server are on different devices");
    Job j;
    j.mesh = m;
    j.vel = vel;
    j.n = n;
    j.xp = xp;
    j.origin = origin;
    j.start = start;
    j.host = host;
    j.iters = iters;
    j.footprint = job_footprint(*s, *m);
    if ((int64_t)j.footprint > s->budget)
        fail(CNNSNS_ENOMEM, "submit: the job's device footprint (" + std::to_string(j.footprint) +
                                " bytes) exceeds the server budget");
    // order the job after the caller's work on its stream (inputs written, outputs initialised)
    struct EventGuard {
        hipEvent_t e = nullptr;
        ~EventGuard() { if (e) (void)hipEventDestroy(e); }
    } ready;
    hip_check(hipEventCreateWithFlags(&ready.e, hipEventDisableTiming), "submit event");
    hip_check(hipEventRecord(ready.e, stream), "submit: event on the caller's stream");
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) fail(CNNSNS_EINVAL, "submit: server is shutting down");
    if ((int32_t)s->queue.size() >= s->queue_depth) fail(CNNSNS_EBUSY, "submit: queue full");
    j.ready = ready.e;
    ready.e = nullptr;
    m->pending_jobs.fetch_add(1);
    j.id = s->next_id++;
    j.t_submit = Clock::now();
    s->jobs.emplace(j.id, j);
    s->queue.push_back(j.id);
    s->cv_sched.notify_one();
    return j.id;
}

static bool finished(cnnsns_server s, uint64_t job_id, double* latency_ms)
{
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) fail(CNNSNS_EINVAL, "unknown job id " + std::to_string(job_id));
    const Job& j = it->second;
    if (!j.done) return false;
    const double lat = std::chrono::duration<double, std::milli>(j.t_done - j.t_submit).count();
    const int err = j.error;
    s->jobs.erase(it);  // a completed job is reported once
    if (latency_ms) *latency_ms = lat;
    if (err != CNNSNS_OK) fail(err, "job " + std::to_string(job_id) + " failed: " + s->thread_error);
    return true;
}

bool server_poll(cnnsns_server s, uint64_t job_id, double* latency_ms)
{
    std::lock_guard<std::mutex> lock(s->mu);
    return finished(s, job_id, latency_ms);
}

void server_wait(cnnsns_server s, uint64_t job_id, double* latency_ms)
{
    std::unique_lock<std::mutex> lock(s->mu);
    for (;;) {
        if (finished(s, job_id, latency_ms)) return;
        s->cv_done.wait(lock);
    }
}

void server_destroy(cnnsns_server s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv_sched.notify_all();
    }
    if (s->thread.joinable()) s->thread.join();
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto st : s->branch) (void)hipStreamDestroy(st);
    if (s->capture) (void)hipStreamDestroy(s->capture);
    if (s->fork) (void)hipEventDestroy(s->fork);
    for (auto e : s->joins) (void)hipEventDestroy(e);
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    if (s->packed) (void)hipFree(s->packed);
    if (s->wbuf) (void)hipFree(s->wbuf);
    delete s;
}

}  // namespace cnnsns
