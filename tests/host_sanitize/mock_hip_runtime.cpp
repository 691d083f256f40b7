// A host-only stand-in for the HIP runtime, linked in place of libamdhip64 so
// that the library's real host code (api.cpp, serve.cpp and the host halves
// of every .hip file, compiled with --offload-host-only) runs on a CPU under
// AddressSanitizer/UndefinedBehaviorSanitizer or ThreadSanitizer.
//
// What it models, and checks:
//  * device memory: hipMalloc returns host memory; every copy, fill and free
//    is checked against the live allocations (a copy that runs past its
//    allocation, a free of an unknown pointer, a leak at exit are failures);
//  * asynchrony: copies, fills and kernel launches are queued per stream and
//    executed by a separate "device" thread in stream order; a copy to host
//    memory lands only when the host synchronises with its stream (stream,
//    event or device synchronisation, an event query, or another stream's
//    wait); until then its destination holds a 0xa5 pattern and, under
//    AddressSanitizer, is poisoned, so reading it early, or copying into a
//    frame that has returned, gives wrong values or a report;
//  * the legacy null stream, which waits for and is waited on by blocking
//    streams; events (record, query, synchronise, cross-stream waits);
//  * stream capture in relaxed mode: work on a capturing stream is recorded,
//    streams join a capture by waiting on an event recorded inside it, every
//    forked stream must join back before the capture ends, a capturing stream
//    may not wait on an event recorded outside its capture, and a device-wide
//    synchronisation while a capture is open is a failure; graphs replay
//    their recorded work in capture order when launched;
//  * kernel launches: the configuration (grid, block, dynamic LDS) is checked
//    against the device limits; the kernels themselves do nothing.
// Failures are counted and printed; mock_failures() returns the count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#include <sanitizer/asan_interface.h>
#endif
#endif
#ifndef ASAN_POISON_MEMORY_REGION
#define ASAN_POISON_MEMORY_REGION(a, n) ((void)(a), (void)(n))
#define ASAN_UNPOISON_MEMORY_REGION(a, n) ((void)(a), (void)(n))
#endif

namespace {

struct Capture;

// A stream's progress: ops completed, and how far held ops may run.  Shared so
// that an event or a wait outlives the stream it refers to.
struct Progress {
    uint64_t done = 0;
    uint64_t flush = 0;  // held ops with an index below this may run
};
using Counter = std::shared_ptr<Progress>;

struct Op {
    std::function<void()> run;  // host work done when the op executes (copies, fills)
    std::string what;           // for messages
    Counter wait_on;            // a wait: until wait_on->done >= wait_seq
    uint64_t wait_seq = 0;
    bool hold = false;          // runs only once the host synchronises with it
    uint64_t idx = 0;           // position in its stream
};

struct MStream {
    unsigned flags = 0;
    std::deque<Op> q;
    uint64_t enq = 0;  // ops enqueued
    Counter done = std::make_shared<Progress>();
    Capture* cap = nullptr;
    uint64_t cap_count = 0;      // ops this stream recorded into its capture
    bool origin = false;         // began the capture it is in
};

struct MEvent {
    Counter done;                // null: never recorded (complete)
    uint64_t seq = 0;            // complete when *done >= seq
    Capture* cap = nullptr;      // recorded inside this capture
    MStream* cap_stream = nullptr;
    uint64_t cap_pos = 0;        // cap_count of cap_stream when recorded
};

struct Capture {
    MStream* origin = nullptr;
    std::vector<Op> ops;
    std::map<MStream*, uint64_t> joined;  // forked stream -> ops of it the origin has waited for
    bool failed = false;
};

struct MGraph {
    std::vector<Op> ops;
};

// All state lives in one object built on first use: module constructors
// register kernels before this file's own globals would be initialised.
struct State {
    std::mutex mu;                   // guards everything below
    std::condition_variable cv;      // signalled on every state change
    std::map<char*, size_t> allocs;  // device allocations
    std::set<MStream*> streams;
    std::set<MEvent*> events;
    std::set<MGraph*> graphs;
    std::set<Capture*> captures;     // open captures
    MStream null_stream;             // the legacy null stream
    std::map<const void*, std::string> kernels;  // host stub -> kernel name
    std::map<const void*, size_t> vars;          // device variable shadow -> size
    std::map<const void*, char*> var_copies;     // its device copy (looked up once)
    long static_bytes = 0;                       // held by device variables until exit
    long mallocs = 0;                            // hipMalloc calls
    bool stop = false;
    std::thread device;
    State();
    ~State();
};

State& mock_state()
{
    static State s;
    return s;
}

#define g_mu (mock_state().mu)
#define g_cv (mock_state().cv)
#define g_allocs (mock_state().allocs)
#define g_streams (mock_state().streams)
#define g_events (mock_state().events)
#define g_graphs (mock_state().graphs)
#define g_captures (mock_state().captures)
#define g_null (mock_state().null_stream)
#define g_kernels (mock_state().kernels)
#define g_stop (mock_state().stop)

std::atomic<int> g_failures{ 0 };
std::atomic<long> g_launches{ 0 };

thread_local hipError_t t_last = hipSuccess;
thread_local struct {
    dim3 grid, block;
    size_t shmem = 0;
    hipStream_t stream = nullptr;
} t_cfg;

void failure(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::fprintf(stderr, "MOCK FAILURE: ");
    std::vfprintf(stderr, fmt, ap);
    std::fprintf(stderr, "\n");
    va_end(ap);
    ++g_failures;
}

hipError_t set_err(hipError_t e)
{
    if (e != hipSuccess) t_last = e;
    return e;
}

MStream* S(hipStream_t s)
{
    return s ? reinterpret_cast<MStream*>(s) : &g_null;
}

// the allocation holding [p, p + n), or false
bool in_alloc(const void* p, size_t n)
{
    auto c = static_cast<const char*>(p);
    auto it = g_allocs.upper_bound(const_cast<char*>(c));
    if (it == g_allocs.begin()) return false;
    --it;
    return c >= it->first && c + n <= it->first + it->second;
}

bool is_device(const void* p)
{
    return in_alloc(p, 1);
}

void device_loop()
{
    std::unique_lock<std::mutex> lk(g_mu);  // st() returns once the state is built
    for (;;) {
        bool progressed = false;
        std::vector<MStream*> all(g_streams.begin(), g_streams.end());
        all.push_back(&g_null);
        for (MStream* s : all) {
            if (s->q.empty()) continue;
            Op& op = s->q.front();
            if (op.wait_on && op.wait_on->done < op.wait_seq) {
                // a wait makes the work it waits for runnable, as a synchronisation would
                if (op.wait_on->flush < op.wait_seq) op.wait_on->flush = op.wait_seq, progressed = true;
                continue;
            }
            if (op.hold && op.idx >= s->done->flush) continue;
            Op mine = std::move(op);
            if (mine.run) {
                // the op stays at the front (so the stream cannot be destroyed) while it runs unlocked
                lk.unlock();
                mine.run();
                lk.lock();
            }
            s->q.pop_front();
            ++s->done->done;
            progressed = true;
            if (mine.run) break;  // streams may have come and gone meanwhile: rescan
        }
        if (progressed) {
            g_cv.notify_all();
            continue;
        }
        if (g_stop) return;
        g_cv.wait(lk);
    }
}

State::State()
{
    device = std::thread(device_loop);
}

State::~State()
{
    {
        std::lock_guard<std::mutex> lk(mu);
        stop = true;
    }
    cv.notify_all();
    device.join();
}

// Enqueue an op on s (recording it instead when s is capturing).  The legacy
// null stream orders itself with every blocking stream.  Caller holds g_mu.
void enqueue(MStream* s, Op op)
{
    if (s->cap) {
        if (!op.wait_on) {
            s->cap->ops.push_back(op);
            ++s->cap_count;
        }
        return;
    }
    for (Capture* c : g_captures)
        if (s == &g_null && !(c->origin->flags & hipStreamNonBlocking))
            failure("null-stream work while a blocking stream is capturing (%s)", op.what.c_str());
    if (s == &g_null) {
        for (MStream* o : g_streams)
            if (!(o->flags & hipStreamNonBlocking) && o->enq > 0)
                s->q.push_back(Op{ nullptr, "null waits for blocking", o->done, o->enq, false, s->enq }), ++s->enq;
    } else if (!(s->flags & hipStreamNonBlocking) && g_null.enq > 0) {
        s->q.push_back(Op{ nullptr, "blocking waits for null", g_null.done, g_null.enq, false, s->enq });
        ++s->enq;
    }
    op.idx = s->enq;
    s->q.push_back(std::move(op));
    ++s->enq;
    g_cv.notify_all();
}

void wait_stream(std::unique_lock<std::mutex>& lk, MStream* s)
{
    const uint64_t target = s->enq;
    s->done->flush = std::max(s->done->flush, target);
    g_cv.notify_all();
    g_cv.wait(lk, [&] { return s->done->done >= target; });
}

bool any_capture_open()
{
    return !g_captures.empty();
}

void wait_all(std::unique_lock<std::mutex>& lk, const char* who)
{
    if (any_capture_open()) failure("%s while a stream capture is open", who);
    std::vector<std::pair<MStream*, uint64_t>> targets;
    for (MStream* s : g_streams) targets.push_back({ s, s->enq });
    targets.push_back({ &g_null, g_null.enq });
    for (auto& t : targets) t.first->done->flush = std::max(t.first->done->flush, t.second);
    g_cv.notify_all();
    g_cv.wait(lk, [&] {
        for (auto& t : targets)
            if (t.first->done->done < t.second) return false;
        return true;
    });
}

}  // namespace

extern "C" int mock_failures()
{
    return g_failures.load();
}

extern "C" long mock_live_device_bytes()
{
    std::lock_guard<std::mutex> lk(g_mu);
    long b = 0;
    for (auto& a : g_allocs) b += (long)a.second;
    return b - mock_state().static_bytes;
}

extern "C" long mock_live_handles()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return (long)(g_streams.size() + g_events.size() + g_graphs.size());
}

extern "C" long mock_mallocs()
{
    std::lock_guard<std::mutex> lk(g_mu);
    return mock_state().mallocs;
}

extern "C" long mock_launches()
{
    return g_launches.load();
}

// ----------------------------------------------------------------------------- registration, launches

extern "C" void** __hipRegisterFatBinary(const void*)
{
    static void* handle = nullptr;
    return &handle;
}

extern "C" void __hipRegisterFunction(void**, const void* hostFunction, char*, const char* deviceName, unsigned int,
                                      uint3*, uint3*, dim3*, dim3*, int*)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_kernels[hostFunction] = deviceName ? deviceName : "?";
}

extern "C" void __hipUnregisterFatBinary(void**) {}

// device variables: host shadow address -> size; their device copies, made on first lookup
extern "C" void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int)
{
    std::lock_guard<std::mutex> lk(g_mu);
    mock_state().vars[var] = size;
}

hipError_t hipGetSymbolAddress(void** p, const void* symbol)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = mock_state().vars.find(symbol);
    if (it == mock_state().vars.end()) {
        failure("hipGetSymbolAddress of an unregistered symbol");
        return set_err(hipErrorInvalidSymbol);
    }
    auto& copy = mock_state().var_copies[symbol];
    if (!copy) {
        copy = static_cast<char*>(std::aligned_alloc(256, (it->second + 255) / 256 * 256));
        g_allocs[copy] = it->second;
        mock_state().static_bytes += (long)it->second;
    }
    *p = copy;
    return hipSuccess;
}

hipError_t __hipPushCallConfiguration(dim3 gridDim, dim3 blockDim, size_t sharedMem, hipStream_t stream)
{
    t_cfg.grid = gridDim;
    t_cfg.block = blockDim;
    t_cfg.shmem = sharedMem;
    t_cfg.stream = stream;
    return hipSuccess;
}

hipError_t __hipPopCallConfiguration(dim3* gridDim, dim3* blockDim, size_t* sharedMem, hipStream_t* stream)
{
    *gridDim = t_cfg.grid;
    *blockDim = t_cfg.block;
    *sharedMem = t_cfg.shmem;
    *stream = t_cfg.stream;
    return hipSuccess;
}

hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t shmem, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_kernels.find(f);
    const std::string name = it == g_kernels.end() ? "unregistered kernel" : it->second;
    const unsigned long threads = (unsigned long)block.x * block.y * block.z;
    if (threads == 0 || threads > 1024 || grid.x == 0 || grid.y == 0 || grid.z == 0 || grid.y > 65535 ||
        grid.z > 65535 || shmem > 160 * 1024) {
        failure("bad launch of %s: grid (%u,%u,%u) block (%u,%u,%u) lds %zu", name.c_str(), grid.x, grid.y, grid.z,
                block.x, block.y, block.z, shmem);
        return set_err(hipErrorInvalidConfiguration);
    }
    if (!args) failure("launch of %s without arguments", name.c_str());
    if (stream && !g_streams.count(S(stream))) {
        failure("launch of %s on a destroyed or unknown stream", name.c_str());
        return set_err(hipErrorInvalidHandle);
    }
    ++g_launches;
    enqueue(S(stream), Op{ nullptr, name });
    return hipSuccess;
}

// ----------------------------------------------------------------------------- device, errors

hipError_t hipGetDevice(int* d)
{
    *d = 0;
    return hipSuccess;
}

hipError_t hipSetDevice(int d)
{
    return d == 0 ? hipSuccess : set_err(hipErrorInvalidDevice);
}

hipError_t hipGetDeviceCount(int* n)
{
    *n = 1;
    return hipSuccess;
}

int hipGetStreamDeviceId(hipStream_t)
{
    return 0;
}

hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t attr, int)
{
    switch (attr) {
    case hipDeviceAttributeMultiprocessorCount: *v = 256; break;
    case hipDeviceAttributeWarpSize: *v = 64; break;
    case hipDeviceAttributeMaxThreadsPerBlock: *v = 1024; break;
    case hipDeviceAttributeMaxSharedMemoryPerBlock: *v = 160 * 1024; break;
    default: *v = 0;
    }
    return hipSuccess;
}

hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int)
{
    std::memset(p, 0, sizeof(*p));
    std::strcpy(p->name, "mock MI355X");
    std::strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
    p->totalGlobalMem = (size_t)288 << 30;
    p->sharedMemPerBlock = 160 * 1024;
    p->warpSize = 64;
    p->maxThreadsPerBlock = 1024;
    p->maxThreadsDim[0] = p->maxThreadsDim[1] = p->maxThreadsDim[2] = 1024;
    p->maxGridSize[0] = 0x7fffffff;
    p->maxGridSize[1] = p->maxGridSize[2] = 65535;
    p->multiProcessorCount = 256;
    p->major = 9;
    p->minor = 5;
    return hipSuccess;
}

hipError_t hipGetLastError()
{
    const hipError_t e = t_last;
    t_last = hipSuccess;
    return e;
}

hipError_t hipPeekAtLastError()
{
    return t_last;
}

const char* hipGetErrorString(hipError_t e)
{
    return e == hipSuccess ? "no error" : "mock runtime error";
}

hipError_t hipDeviceSynchronize()
{
    std::unique_lock<std::mutex> lk(g_mu);
    wait_all(lk, "hipDeviceSynchronize");
    return hipSuccess;
}

// ----------------------------------------------------------------------------- memory

hipError_t hipMalloc(void** p, size_t n)
{
    if (!p) return set_err(hipErrorInvalidValue);
    char* q = static_cast<char*>(std::aligned_alloc(256, (std::max<size_t>(n, 1) + 255) / 256 * 256));
    if (!q) return set_err(hipErrorOutOfMemory);
    std::lock_guard<std::mutex> lk(g_mu);
    g_allocs[q] = std::max<size_t>(n, 1);
    ++mock_state().mallocs;
    *p = q;
    return hipSuccess;
}

hipError_t hipFree(void* p)
{
    if (!p) return hipSuccess;
    std::unique_lock<std::mutex> lk(g_mu);
    wait_all(lk, "hipFree");  // frees synchronise the device
    auto it = g_allocs.find(static_cast<char*>(p));
    if (it == g_allocs.end()) {
        failure("hipFree of a pointer that is not a live allocation (%p)", p);
        return set_err(hipErrorInvalidValue);
    }
    g_allocs.erase(it);
    std::free(p);
    return hipSuccess;
}

static hipError_t check_copy(void* dst, const void* src, size_t n, hipMemcpyKind kind, const char* who)
{
    const bool dd = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyHostToDevice || kind == hipMemcpyDefault;
    const bool sd = kind == hipMemcpyDeviceToDevice || kind == hipMemcpyDeviceToHost || kind == hipMemcpyDefault;
    if (n == 0) return hipSuccess;
    if (kind != hipMemcpyDefault) {
        if (dd && !in_alloc(dst, n)) {
            failure("%s: %zu bytes to %p run outside a device allocation", who, n, dst);
            return hipErrorInvalidValue;
        }
        if (sd && !in_alloc(src, n)) {
            failure("%s: %zu bytes from %p run outside a device allocation", who, n, src);
            return hipErrorInvalidValue;
        }
        if (kind == hipMemcpyHostToDevice && is_device(src)) failure("%s: host source is device memory", who);
        if (kind == hipMemcpyDeviceToHost && is_device(dst)) failure("%s: host destination is device memory", who);
    }
    return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind kind, hipStream_t stream)
{
    std::unique_lock<std::mutex> lk(g_mu);
    if (hipError_t e = check_copy(dst, src, n, kind, "hipMemcpyAsync")) return set_err(e);
    if (n == 0) return hipSuccess;
    if (kind == hipMemcpyHostToDevice) {
        // pageable host memory: the copy takes the source before the call returns
        auto staged = std::make_shared<std::vector<char>>(static_cast<const char*>(src),
                                                           static_cast<const char*>(src) + n);
        enqueue(S(stream), Op{ [=] { std::memcpy(dst, staged->data(), n); }, "memcpy H2D" });
        return hipSuccess;
    }
    if (kind == hipMemcpyDeviceToHost) {
        // lands when the host synchronises with the stream; until then the destination is
        // poisoned, so reading it early (or a copy into a frame that has returned) is reported
        std::memset(dst, 0xa5, n);  // what an early read sees (poisoning works on 8-byte granules only)
        ASAN_POISON_MEMORY_REGION(dst, n);
        Op op{ [=] {
                  ASAN_UNPOISON_MEMORY_REGION(dst, n);
                  std::memcpy(dst, src, n);
              },
               "memcpy D2H" };
        op.hold = true;
        enqueue(S(stream), std::move(op));
        return hipSuccess;
    }
    enqueue(S(stream), Op{ [=] { std::memcpy(dst, src, n); }, "memcpy" });
    return hipSuccess;
}

hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind kind)
{
    {
        std::unique_lock<std::mutex> lk(g_mu);
        if (hipError_t e = check_copy(dst, src, n, kind, "hipMemcpy")) return set_err(e);
        if (n == 0) return hipSuccess;
        enqueue(&g_null, Op{ [=] { std::memcpy(dst, src, n); }, "memcpy (sync)" });
        wait_stream(lk, &g_null);
    }
    return hipSuccess;
}

hipError_t hipMemsetAsync(void* dst, int value, size_t n, hipStream_t stream)
{
    std::unique_lock<std::mutex> lk(g_mu);
    if (n && !in_alloc(dst, n)) {
        failure("hipMemsetAsync: %zu bytes at %p run outside a device allocation", n, dst);
        return set_err(hipErrorInvalidValue);
    }
    enqueue(S(stream), Op{ [=] { std::memset(dst, value, n); }, "memset" });
    return hipSuccess;
}

// ----------------------------------------------------------------------------- streams, events

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned flags)
{
    auto* m = new MStream();
    m->flags = flags;
    std::lock_guard<std::mutex> lk(g_mu);
    g_streams.insert(m);
    *s = reinterpret_cast<hipStream_t>(m);
    return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t* s)
{
    return hipStreamCreateWithFlags(s, 0);
}

hipError_t hipStreamDestroy(hipStream_t s)
{
    std::unique_lock<std::mutex> lk(g_mu);
    MStream* m = S(s);
    if (!s || !g_streams.count(m)) {
        failure("hipStreamDestroy of an unknown stream");
        return set_err(hipErrorInvalidHandle);
    }
    if (m->cap) {
        failure("hipStreamDestroy of a capturing stream");
        return set_err(hipErrorStreamCaptureUnsupported);
    }
    wait_stream(lk, m);
    g_streams.erase(m);
    delete m;
    return hipSuccess;
}

hipError_t hipStreamSynchronize(hipStream_t s)
{
    std::unique_lock<std::mutex> lk(g_mu);
    MStream* m = S(s);
    if (s && !g_streams.count(m)) {
        failure("hipStreamSynchronize of an unknown stream");
        return set_err(hipErrorInvalidHandle);
    }
    if (m->cap) {
        failure("hipStreamSynchronize of a capturing stream");
        return set_err(hipErrorStreamCaptureUnsupported);
    }
    if (m == &g_null) {
        wait_all(lk, "hipStreamSynchronize(null)");
    } else {
        wait_stream(lk, m);
    }
    return hipSuccess;
}

hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned)
{
    auto* m = new MEvent();
    std::lock_guard<std::mutex> lk(g_mu);
    g_events.insert(m);
    *e = reinterpret_cast<hipEvent_t>(m);
    return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e)
{
    return hipEventCreateWithFlags(e, 0);
}

hipError_t hipEventDestroy(hipEvent_t e)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto* m = reinterpret_cast<MEvent*>(e);
    if (!g_events.count(m)) {
        failure("hipEventDestroy of an unknown event");
        return set_err(hipErrorInvalidHandle);
    }
    g_events.erase(m);
    delete m;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto* m = reinterpret_cast<MEvent*>(e);
    MStream* st = S(s);
    if (!g_events.count(m)) {
        failure("hipEventRecord of an unknown event");
        return set_err(hipErrorInvalidHandle);
    }
    if (s && !g_streams.count(st)) {
        failure("hipEventRecord on an unknown stream");
        return set_err(hipErrorInvalidHandle);
    }
    if (st->cap) {
        m->cap = st->cap;
        m->cap_stream = st;
        m->cap_pos = st->cap_count;
        m->done = nullptr;
        return hipSuccess;
    }
    m->cap = nullptr;
    // the event completes once everything enqueued so far on st (and, on the null stream, on the
    // blocking streams it waits for) has run: mark it with a no-op
    enqueue(st, Op{ nullptr, "event" });
    m->done = st->done;
    m->seq = st->enq;
    return hipSuccess;
}

hipError_t hipEventQuery(hipEvent_t e)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto* m = reinterpret_cast<MEvent*>(e);
    if (!g_events.count(m)) {
        failure("hipEventQuery of an unknown event");
        return set_err(hipErrorInvalidHandle);
    }
    if (m->cap) {
        failure("hipEventQuery of an event recorded in a capture");
        return set_err(hipErrorStreamCaptureUnsupported);
    }
    if (!m->done) return hipSuccess;
    m->done->flush = std::max(m->done->flush, m->seq);
    g_cv.notify_all();
    return m->done->done >= m->seq ? hipSuccess : hipErrorNotReady;
}

hipError_t hipEventSynchronize(hipEvent_t e)
{
    std::unique_lock<std::mutex> lk(g_mu);
    auto* m = reinterpret_cast<MEvent*>(e);
    if (!g_events.count(m)) {
        failure("hipEventSynchronize of an unknown event");
        return set_err(hipErrorInvalidHandle);
    }
    if (!m->done) return hipSuccess;
    const Counter done = m->done;
    const uint64_t seq = m->seq;
    done->flush = std::max(done->flush, seq);
    g_cv.notify_all();
    g_cv.wait(lk, [&] { return done->done >= seq; });
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto* m = reinterpret_cast<MEvent*>(e);
    MStream* st = S(s);
    if (!g_events.count(m) || (s && !g_streams.count(st))) {
        failure("hipStreamWaitEvent with an unknown stream or event");
        return set_err(hipErrorInvalidHandle);
    }
    if (m->cap) {
        Capture* c = m->cap;
        if (st->cap && st->cap != c) {
            failure("a stream of one capture waits on an event of another");
            return set_err(hipErrorStreamCaptureIsolation);
        }
        if (!st->cap) {  // fork: st joins the capture
            st->cap = c;
            st->cap_count = 0;
            st->origin = false;
            c->joined[st] = 0;
        } else if (st == c->origin && m->cap_stream != c->origin) {  // join back
            auto it = c->joined.find(m->cap_stream);
            if (it != c->joined.end()) it->second = std::max(it->second, m->cap_pos);
        }
        return hipSuccess;
    }
    if (st->cap) {
        failure("a capturing stream waits on an event recorded outside its capture");
        return set_err(hipErrorStreamCaptureIsolation);
    }
    if (m->done) enqueue(st, Op{ nullptr, "wait event", m->done, m->seq });
    return hipSuccess;
}

// ----------------------------------------------------------------------------- capture, graphs

hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode)
{
    std::lock_guard<std::mutex> lk(g_mu);
    MStream* st = S(s);
    if (!s || !g_streams.count(st)) {
        failure("hipStreamBeginCapture on the null or an unknown stream");
        return set_err(hipErrorInvalidValue);
    }
    if (st->cap) {
        failure("hipStreamBeginCapture on a stream that is capturing");
        return set_err(hipErrorIllegalState);
    }
    auto* c = new Capture();
    c->origin = st;
    st->cap = c;
    st->cap_count = 0;
    st->origin = true;
    g_captures.insert(c);
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g)
{
    std::lock_guard<std::mutex> lk(g_mu);
    MStream* st = S(s);
    *g = nullptr;
    if (!st->cap || !st->origin) {
        failure("hipStreamEndCapture on a stream that did not begin a capture");
        return set_err(hipErrorIllegalState);
    }
    Capture* c = st->cap;
    hipError_t rc = hipSuccess;
    for (auto& [fs, pos] : c->joined) {
        if (fs->cap_count > pos) {
            failure("a forked stream did not join back before the capture ended (%llu of %llu ops joined)",
                    (unsigned long long)pos, (unsigned long long)fs->cap_count);
            rc = hipErrorStreamCaptureUnjoined;
        }
        fs->cap = nullptr;
    }
    for (MEvent* e : g_events)
        if (e->cap == c) e->cap = nullptr, e->done = nullptr;
    st->cap = nullptr;
    st->origin = false;
    g_captures.erase(c);
    if (rc == hipSuccess) {
        auto* gr = new MGraph();
        gr->ops = std::move(c->ops);
        g_graphs.insert(gr);
        *g = reinterpret_cast<hipGraph_t>(gr);
    }
    delete c;
    return set_err(rc);
}

hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto* gr = reinterpret_cast<MGraph*>(g);
    if (!g_graphs.count(gr)) {
        failure("hipGraphInstantiate of an unknown graph");
        return set_err(hipErrorInvalidValue);
    }
    auto* ex = new MGraph(*gr);
    g_graphs.insert(ex);
    *e = reinterpret_cast<hipGraphExec_t>(ex);
    return hipSuccess;
}

hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t s)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto* ex = reinterpret_cast<MGraph*>(e);
    if (!g_graphs.count(ex)) {
        failure("hipGraphLaunch of an unknown graph");
        return set_err(hipErrorInvalidValue);
    }
    for (const Op& op : ex->ops) enqueue(S(s), op);
    return hipSuccess;
}

hipError_t hipGraphDestroy(hipGraph_t g)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto* gr = reinterpret_cast<MGraph*>(g);
    if (!g_graphs.erase(gr)) {
        failure("hipGraphDestroy of an unknown graph");
        return set_err(hipErrorInvalidValue);
    }
    delete gr;
    return hipSuccess;
}

hipError_t hipGraphExecDestroy(hipGraphExec_t e)
{
    return hipGraphDestroy(reinterpret_cast<hipGraph_t>(e));
}
