// The C ABI: argument checks, error codes and the thread-local error message.
// Every exported function catches everything; nothing propagates to C.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include "common.h"
#include "serve.h"

namespace cnnsns {

static thread_local std::string g_last_error;

void fail(int code, const std::string& msg)
{
    throw Error{ code, msg };
}

void hip_check(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? CNNSNS_ENOMEM : CNNSNS_EHIP,
             std::string(what) + ": " + hipGetErrorString(e));
    }
}

void workspace_acquire(Workspace& ws, size_t need, hipStream_t stream, const char* what)
{
    if (ws.bytes < need) {
        if (ws.ptr) {
            // every pass enqueued with the old buffer must finish before it is freed
            hip_check(hipDeviceSynchronize(), what);
            hip_check(hipFree(ws.ptr), what);
            ws.ptr = nullptr;
            ws.bytes = 0;
        }
        if (hipMalloc(&ws.ptr, need) != hipSuccess) {
            ws.ptr = nullptr;
            (void)hipGetLastError();
            fail(CNNSNS_ENOMEM, std::string(what) + ": workspace of " + std::to_string(need) + " bytes");
        }
        ws.bytes = need;
    }
    // (also on the same stream handle: a destroyed stream's handle may be reused by a new one)
    if (ws.last_use) hip_check(hipStreamWaitEvent(stream, ws.last_use, 0), what);
}

void workspace_used(Workspace& ws, hipStream_t stream)
{
    if (!ws.last_use) hip_check(hipEventCreateWithFlags(&ws.last_use, hipEventDisableTiming), "workspace event");
    hip_check(hipEventRecord(ws.last_use, stream), "workspace event");
}

void workspace_release(Workspace& ws)
{
    if (ws.ptr) (void)hipFree(ws.ptr);
    if (ws.last_use) (void)hipEventDestroy(ws.last_use);
    ws.ptr = nullptr;
    ws.bytes = 0;
    ws.last_use = nullptr;
}

template <class F>
static int guarded(F&& f)
{
    try {
        f();
        g_last_error.clear();
        return CNNSNS_OK;
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return CNNSNS_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return CNNSNS_EINVAL;
    } catch (...) {
        g_last_error = "unknown error";
        return CNNSNS_EINVAL;
    }
}

// Run on the mesh's device, restoring the caller's current device afterwards.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        hip_check(hipGetDevice(&prev), "hipGetDevice");
        if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace cnnsns

using namespace cnnsns;

extern "C" {

int cnnsns_build_mesh(const double* xy, int64_t n_nodes, const int32_t* tri, int64_t n_tri, int32_t overlay_side,
                      void* stream, cnnsns_mesh* out)
{
    return guarded([&] {
        if (!out) fail(CNNSNS_EINVAL, "build_mesh: out must not be NULL");
        *out = nullptr;
        *out = build_mesh(xy, n_nodes, tri, n_tri, overlay_side, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_mesh_info(cnnsns_mesh m, int64_t* n_tri, int32_t* overlay_side, int64_t* device_bytes, double* mean_diam)
{
    return guarded([&] {
        if (!m) fail(CNNSNS_EINVAL, "mesh_info: NULL mesh");
        if (n_tri) *n_tri = m->n_tri;
        if (overlay_side) *overlay_side = m->G;
        if (device_bytes) *device_bytes = m->device_bytes;
        if (mean_diam) *mean_diam = m->mean_diam;
    });
}

int cnnsns_destroy_mesh(cnnsns_mesh m)
{
    return guarded([&] { destroy_mesh(m); });
}

int cnnsns_predict(cnnsns_mesh m, const float* vel, const cnnsns_cnn* w, int32_t precision, float* disp, void* stream)
{
    return guarded([&] {
        if (!m || !vel || !w || !disp) fail(CNNSNS_EINVAL, "predict: NULL argument");
        for (int l = 0; l < 4; ++l)
            if (!w->w[l] || !w->b[l]) fail(CNNSNS_EINVAL, "predict: NULL weight or bias pointer");
        if (precision != CNNSNS_F32 && precision != CNNSNS_BF16 && precision != CNNSNS_FP8E4M3)
            fail(CNNSNS_EINVAL, "predict: unknown precision");
        DeviceScope ds(m->device);
        run_predict(*m, vel, *w, precision, disp, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_predict_noalloc(cnnsns_mesh m, const float* vel, const cnnsns_cnn* w, int32_t precision, float* disp,
                           void* stream)
{
    return guarded([&] {
        if (!m || !vel || !w || !disp) fail(CNNSNS_EINVAL, "predict_noalloc: NULL argument");
        for (int l = 0; l < 4; ++l)
            if (!w->w[l] || !w->b[l]) fail(CNNSNS_EINVAL, "predict_noalloc: NULL weight or bias pointer");
        DeviceScope ds(m->device);
        run_predict_noalloc(*m, vel, *w, precision, disp, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_classify(cnnsns_mesh m, int64_t n, const double* xp, const cnnsns_cls* w, const int32_t* fallback,
                    int32_t* start, int32_t* cls, float* logits, void* stream)
{
    return guarded([&] {
        if (!m || !w) fail(CNNSNS_EINVAL, "classify: NULL mesh or weights");
        if (n < 0) fail(CNNSNS_EINVAL, "classify: n must be >= 0");
        if (n == 0) return;
        if (!xp || !start) fail(CNNSNS_EINVAL, "classify: xp and start must not be NULL");
        for (int l = 0; l < 6; ++l)
            if (!w->w[l] || !w->b[l]) fail(CNNSNS_EINVAL, "classify: NULL weight or bias pointer");
        DeviceScope ds(m->device);
        run_classify(*m, n, xp, *w, fallback, start, cls, logits, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_locate(cnnsns_mesh m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                  const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status, void* stream)
{
    return guarded([&] {
        if (!m) fail(CNNSNS_EINVAL, "locate: NULL mesh");
        if (n < 0) fail(CNNSNS_EINVAL, "locate: n must be >= 0");
        if (n == 0) return;
        if (!xp || !host) fail(CNNSNS_EINVAL, "locate: xp and host must not be NULL");
        if (disp && !origin) fail(CNNSNS_EINVAL, "locate: disp given without origin");
        DeviceScope ds(m->device);
        launch_locate(*m, n, xp, start, origin, disp, max_iter, host, iters, status, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_locate_interpolate(cnnsns_mesh m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                              const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status,
                              const double* nodal, double* out, void* stream)
{
    return guarded([&] {
        if (!m) fail(CNNSNS_EINVAL, "locate_interpolate: NULL mesh");
        if (n < 0) fail(CNNSNS_EINVAL, "locate_interpolate: n must be >= 0");
        if (n == 0) return;
        if (!xp || !host || !nodal || !out) fail(CNNSNS_EINVAL, "locate_interpolate: NULL argument");
        if (disp && !origin) fail(CNNSNS_EINVAL, "locate_interpolate: disp given without origin");
        DeviceScope ds(m->device);
        launch_locate(*m, n, xp, start, origin, disp, max_iter, host, iters, status, static_cast<hipStream_t>(stream),
                      nodal, out);
    });
}

int cnnsns_build_mesh3d(const double* xyz, int64_t n_nodes, const int32_t* tet, int64_t n_tet, int32_t overlay_side,
                        void* stream, cnnsns_mesh3* out)
{
    return guarded([&] {
        if (!xyz || !tet || !out) fail(CNNSNS_EINVAL, "build_mesh3d: NULL argument");
        *out = nullptr;
        if (n_nodes < 4 || n_tet < 1) fail(CNNSNS_EINVAL, "build_mesh3d: need n_nodes >= 4 and n_tet >= 1");
        if (n_tet > (int64_t)INT32_MAX / 4 || n_nodes >= (int64_t)INT32_MAX)
            fail(CNNSNS_EINVAL, "build_mesh3d: ids must fit in int32");
        if (overlay_side < 0 || overlay_side > 1024) fail(CNNSNS_EINVAL, "build_mesh3d: overlay_side out of range");
        *out = build_mesh3(xyz, n_nodes, tet, n_tet, overlay_side, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_mesh3d_info(cnnsns_mesh3 m, int64_t* n_tet, int32_t* overlay_side, int64_t* device_bytes)
{
    return guarded([&] {
        if (!m) fail(CNNSNS_EINVAL, "mesh3d_info: NULL mesh");
        if (n_tet) *n_tet = m->n_tet;
        if (overlay_side) *overlay_side = m->G;
        if (device_bytes) *device_bytes = m->device_bytes;
    });
}

int cnnsns_destroy_mesh3d(cnnsns_mesh3 m)
{
    return guarded([&] { destroy_mesh3(m); });
}

int cnnsns_predict3d(cnnsns_mesh3 m, const float* vel, const cnnsns_cnn* w, int32_t precision, float* disp,
                     void* stream)
{
    return guarded([&] {
        if (!m || !vel || !w || !disp) fail(CNNSNS_EINVAL, "predict3d: NULL argument");
        for (int l = 0; l < 4; ++l)
            if (!w->w[l] || !w->b[l]) fail(CNNSNS_EINVAL, "predict3d: NULL weight or bias pointer");
        if (precision != CNNSNS_F32 && precision != CNNSNS_BF16)
            fail(CNNSNS_EINVAL, "predict3d: CNNSNS_F32 and CNNSNS_BF16 are implemented in 3D");
        DeviceScope ds(m->device);
        run_predict3(*m, vel, *w, precision, disp, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_locate3d(cnnsns_mesh3 m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                    const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status, void* stream)
{
    return guarded([&] {
        if (!m) fail(CNNSNS_EINVAL, "locate3d: NULL mesh");
        if (n < 0) fail(CNNSNS_EINVAL, "locate3d: n must be >= 0");
        if (n == 0) return;
        if (!xp || !host) fail(CNNSNS_EINVAL, "locate3d: xp and host must not be NULL");
        if (disp && !origin) fail(CNNSNS_EINVAL, "locate3d: disp given without origin");
        DeviceScope ds(m->device);
        launch_locate3(*m, n, xp, start, origin, disp, max_iter, host, iters, status,
                       static_cast<hipStream_t>(stream));
    });
}

int cnnsns_interpolate3d(cnnsns_mesh3 m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                         double* out, void* stream)
{
    return guarded([&] {
        if (!m) fail(CNNSNS_EINVAL, "interpolate3d: NULL mesh");
        if (n < 0) fail(CNNSNS_EINVAL, "interpolate3d: n must be >= 0");
        if (n == 0) return;
        if (!xp || !host || !nodal || !out) fail(CNNSNS_EINVAL, "interpolate3d: NULL argument");
        DeviceScope ds(m->device);
        launch_interp3(*m, n, xp, host, nodal, out, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_interpolate(cnnsns_mesh m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                       double* out, void* stream)
{
    return guarded([&] {
        if (!m) fail(CNNSNS_EINVAL, "interpolate: NULL mesh");
        if (n < 0) fail(CNNSNS_EINVAL, "interpolate: n must be >= 0");
        if (n == 0) return;
        if (!xp || !host || !nodal || !out) fail(CNNSNS_EINVAL, "interpolate: NULL argument");
        DeviceScope ds(m->device);
        launch_interp(*m, n, xp, host, nodal, out, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_server_create(int64_t hbm_budget_bytes, int32_t max_inflight, int32_t queue_depth, int32_t precision,
                         const cnnsns_cnn* w, cnnsns_server* out)
{
    return guarded([&] {
        if (!out) fail(CNNSNS_EINVAL, "server_create: out must not be NULL");
        *out = nullptr;
        // Switched off unless asked for: runs of the serving loop on the GPU have ended, now and
        // then, in a host-side segmentation fault whose cause has not been found.
        const char* on = std::getenv("CNNSNS_ENABLE_SERVING");
        if (!on || std::strcmp(on, "1") != 0)
            fail(CNNSNS_EINVAL, "server_create: the serving loop is switched off (an intermittent host "
                                "crash in it is unexplained); set CNNSNS_ENABLE_SERVING=1 to enable it");
        *out = server_create(hbm_budget_bytes, max_inflight, queue_depth, precision, w);
    });
}

int cnnsns_submit(cnnsns_server s, cnnsns_mesh m, const float* vel, int64_t n, const double* xp, const double* origin,
                  const int32_t* start, int32_t* host, int32_t* iters, void* stream, uint64_t* job_id)
{
    return guarded([&] {
        if (!s || !m || !vel || !job_id) fail(CNNSNS_EINVAL, "submit: NULL argument");
        if (n < 0) fail(CNNSNS_EINVAL, "submit: n must be >= 0");
        if (n > 0 && (!xp || !origin || !host)) fail(CNNSNS_EINVAL, "submit: NULL point buffer");
        *job_id = server_submit(s, m, vel, n, xp, origin, start, host, iters, static_cast<hipStream_t>(stream));
    });
}

int cnnsns_poll(cnnsns_server s, uint64_t job_id, int32_t* done, double* latency_ms)
{
    return guarded([&] {
        if (!s || !done) fail(CNNSNS_EINVAL, "poll: NULL argument");
        *done = server_poll(s, job_id, latency_ms) ? 1 : 0;
    });
}

int cnnsns_wait(cnnsns_server s, uint64_t job_id, double* latency_ms)
{
    return guarded([&] {
        if (!s) fail(CNNSNS_EINVAL, "wait: NULL server");
        server_wait(s, job_id, latency_ms);
    });
}

int cnnsns_server_destroy(cnnsns_server s)
{
    return guarded([&] { server_destroy(s); });
}

const char* cnnsns_last_error(void)
{
    return g_last_error.c_str();
}

}  // extern "C"
