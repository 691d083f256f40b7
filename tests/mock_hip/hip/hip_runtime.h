// Host-only stand-in for the subset of the HIP runtime API the serving loop
// uses, so that its scheduling logic (admission, arena, batches, completion)
// can be tested on a CPU under AddressSanitizer.  Events complete a few
// polls after they are recorded; graphs are plain host objects.
#pragma once
#include <atomic>
#include <cstddef>
#include <cstdlib>
#include <cstring>

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorOutOfMemory = 2, hipErrorInvalidValue = 1 };
enum { hipStreamNonBlocking = 1, hipEventDisableTiming = 2 };
typedef int hipStreamCaptureMode;
enum { hipStreamCaptureModeRelaxed = 2 };
typedef int hipDeviceAttribute_t;
enum { hipDeviceAttributeMultiprocessorCount = 1 };
enum hipMemcpyKind { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };

struct MockStream { int capturing = 0; int work = 0; };
struct MockEvent { std::atomic<int> countdown{0}; };
struct MockGraph { int nodes = 0; };
struct MockExec { int nodes = 0; };
typedef MockStream* hipStream_t;
typedef MockEvent* hipEvent_t;
typedef MockGraph* hipGraph_t;
typedef MockExec* hipGraphExec_t;

extern std::atomic<long> mock_live_objects;
extern std::atomic<long> mock_bytes;

inline hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
inline hipError_t hipSetDevice(int) { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char* hipGetErrorString(hipError_t) { return "mock error"; }
inline hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) { *v = 256; return hipSuccess; }
inline hipError_t hipMalloc(void** p, size_t n) { *p = std::malloc(n ? n : 1); mock_bytes += (long)n; return *p ? hipSuccess : hipErrorOutOfMemory; }
template <class T> inline hipError_t hipMalloc(T** p, size_t n) { return hipMalloc(reinterpret_cast<void**>(p), n); }
inline hipError_t hipFree(void* p) { std::free(p); return hipSuccess; }
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { std::memcpy(d, s, n); return hipSuccess; }
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) { *s = new MockStream(); ++mock_live_objects; return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipStreamDestroy(hipStream_t s) { delete s; --mock_live_objects; return hipSuccess; }
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { *e = new MockEvent(); ++mock_live_objects; return hipSuccess; }
inline hipError_t hipEventDestroy(hipEvent_t e) { delete e; --mock_live_objects; return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) { e->countdown = 1 + std::rand() % 4; return hipSuccess; }
inline hipError_t hipEventQuery(hipEvent_t e) { return e->countdown.fetch_sub(1) <= 1 ? hipSuccess : hipErrorNotReady; }
inline hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
inline hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) { s->capturing = 1; return hipSuccess; }
inline hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g)
{
    if (!s->capturing) { *g = nullptr; return hipErrorInvalidValue; }
    s->capturing = 0; *g = new MockGraph(); ++mock_live_objects; return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, void*, void*, size_t) { *e = new MockExec(); ++mock_live_objects; return hipSuccess; }
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t g) { delete g; --mock_live_objects; return hipSuccess; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete e; --mock_live_objects; return hipSuccess; }
