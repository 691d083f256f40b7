// Replays the library's call sequences through the C ABI against the mock HIP
// runtime (the kernels do nothing; everything the host code does is real).
//
// usage: host_driver <scenario> [args]
//   c5ref  <n_meshes> <scale> <seed>
//          the served-mix benchmark's pass without a server: meshes of
//          log-uniform size (triangle counts in [1e4, 4e6] divided by scale,
//          overlay side from the unscaled count), each with a BF16 predict and
//          a CNN-SNS locate into fresh buffers, then a plain locate of every
//          mesh, then the meshes destroyed
//   serve  <seed>
//          the serving tests' sequence: six meshes, each job alone (predict +
//          locate + synchronise), then servers of three configurations taking
//          30 jobs each with outputs initialised on the submitter's stream,
//          waits in order; then a one-job budget, a full queue, polling,
//          invalid arguments, and a mesh destroyed while its jobs are pending
//   predict_mt <iters>
//          two threads predicting on one mesh on their own streams,
//          alternating BF16 and FP32 (so the shared workspace grows while the
//          other thread uses it), while a third locates
//   mesh3d  building, predicting on and locating in a small tetrahedral mesh
// Prints "<n> failures" and exits non-zero on any failure, including those the
// mock runtime reports and device memory or handles left behind.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/cnnsns.h"

extern "C" int mock_failures();
extern "C" long mock_live_device_bytes();
extern "C" long mock_live_handles();
extern "C" long mock_launches();
extern "C" long mock_mallocs();

namespace {

int g_fail = 0;

#define EXPECT(cond, what)                                                                                       \
    do {                                                                                                         \
        if (!(cond)) {                                                                                           \
            std::fprintf(stderr, "FAILED %s:%d: %s (%s)\n", __FILE__, __LINE__, what, cnnsns_last_error());      \
            ++g_fail;                                                                                            \
        }                                                                                                        \
    } while (0)

template <class T>
T* dev_alloc(size_t n)
{
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (n ? n : 1)) != hipSuccess) {
        std::fprintf(stderr, "device allocation failed\n");
        std::exit(3);
    }
    return static_cast<T*>(p);
}

template <class T>
T* dev_copy(const std::vector<T>& h)
{
    T* d = dev_alloc<T>(h.size());
    if (!h.empty()) (void)hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
    return d;
}

// An n x n node grid on the unit square, two triangles per cell.
struct HostMesh {
    int64_t n_nodes = 0, n_tri = 0;
    std::vector<double> xy;
    std::vector<int32_t> tri;
};

HostMesh grid_mesh(int n)
{
    HostMesh m;
    m.n_nodes = (int64_t)n * n;
    m.xy.resize(2 * m.n_nodes);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            m.xy[2 * ((int64_t)j * n + i)] = (double)i / (n - 1);
            m.xy[2 * ((int64_t)j * n + i) + 1] = (double)j / (n - 1);
        }
    for (int j = 0; j + 1 < n; ++j)
        for (int i = 0; i + 1 < n; ++i) {
            const int32_t a = j * n + i, b = a + 1, c = a + n + 1, d = a + n;
            m.tri.insert(m.tri.end(), { a, b, c, a, c, d });
        }
    m.n_tri = (int64_t)m.tri.size() / 3;
    return m;
}

int overlay_side_for(double n_tri)
{
    return 1 << (int)std::ceil(std::log2(std::sqrt(n_tri)));
}

struct Weights {
    float* buf = nullptr;
    cnnsns_cnn w{};
    explicit Weights(int dim)  // dim 2: 2-32-32-32-2 with 3x3 kernels; 3: 3-32-32-32-3 with 3x3x3
    {
        const size_t taps = dim == 2 ? 9 : 27, c0 = dim == 2 ? 2 : 3;
        const size_t wsz[4] = { 32 * c0 * taps, 32 * 32 * taps, 32 * 32 * taps, c0 * 32 * taps };
        const size_t bsz[4] = { 32, 32, 32, c0 };
        size_t total = 0;
        for (int l = 0; l < 4; ++l) total += wsz[l] + bsz[l];
        std::vector<float> h(total, 0.01f);
        buf = dev_copy(h);
        float* p = buf;
        for (int l = 0; l < 4; ++l) {
            w.w[l] = p;
            p += wsz[l];
            w.b[l] = p;
            p += bsz[l];
        }
    }
    ~Weights() { (void)hipFree(buf); }
};

struct Job {
    cnnsns_mesh m = nullptr;
    int64_t n = 0;
    int32_t G = 0;
    float* vel = nullptr;
    double *xp = nullptr, *origin = nullptr;
    int32_t* start = nullptr;
};

Job make_job(const HostMesh& hm, int32_t G, hipStream_t st)
{
    Job j;
    EXPECT(cnnsns_build_mesh(hm.xy.data(), hm.n_nodes, hm.tri.data(), hm.n_tri, G, st, &j.m) == CNNSNS_OK,
           "build_mesh");
    int64_t nt = 0;
    EXPECT(cnnsns_mesh_info(j.m, &nt, &j.G, nullptr, nullptr) == CNNSNS_OK && nt == hm.n_tri && j.G == G,
           "mesh_info");
    j.n = hm.n_nodes;
    j.vel = dev_copy(std::vector<float>(2 * (size_t)G * G, 0.5f));
    j.xp = dev_copy(hm.xy);
    j.origin = dev_copy(hm.xy);
    std::vector<int32_t> s(j.n);
    for (int64_t i = 0; i < j.n; ++i) s[i] = (int32_t)(i % hm.n_tri);
    j.start = dev_copy(s);
    return j;
}

void free_job(Job& j)
{
    EXPECT(cnnsns_destroy_mesh(j.m) == CNNSNS_OK, "destroy_mesh");
    for (void* p : { (void*)j.vel, (void*)j.xp, (void*)j.origin, (void*)j.start }) (void)hipFree(p);
    j = Job{};
}

// -------------------------------------------------------------------------------------------------

void scenario_c5ref(int n_meshes, double scale, unsigned seed)
{
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(std::log(1e4), std::log(4e6));
    Weights W(2);
    std::vector<Job> jobs;
    for (int k = 0; k < n_meshes; ++k) {
        const double nt = std::exp(U(rng));
        const int n_side = std::max(3, (int)std::lround(std::sqrt(nt / scale / 2.0)) + 1);
        const HostMesh hm = grid_mesh(n_side);
        jobs.push_back(make_job(hm, overlay_side_for(nt), nullptr));
    }
    (void)hipDeviceSynchronize();
    // each job alone: BF16 forward pass, then the CNN-SNS locate, into fresh buffers
    std::vector<std::vector<void*>> bufs;
    for (Job& j : jobs) {
        float* disp = dev_alloc<float>(2 * (size_t)j.G * j.G);
        int32_t* host = dev_alloc<int32_t>(j.n);
        int32_t* iters = dev_alloc<int32_t>(j.n);
        uint8_t* status = dev_alloc<uint8_t>(j.n);
        EXPECT(cnnsns_predict(j.m, j.vel, &W.w, CNNSNS_BF16, disp, nullptr) == CNNSNS_OK, "predict bf16");
        EXPECT(cnnsns_locate(j.m, j.n, j.xp, nullptr, j.origin, disp, 0, host, iters, status, nullptr) == CNNSNS_OK,
               "locate cnn");
        (void)hipFree(status);  // as the binding's dropped status tensor
        (void)hipFree(disp);
        bufs.push_back({ host, iters });
    }
    (void)hipDeviceSynchronize();
    for (Job& j : jobs) {
        int32_t* host = dev_alloc<int32_t>(j.n);
        int32_t* iters = dev_alloc<int32_t>(j.n);
        EXPECT(cnnsns_locate(j.m, j.n, j.xp, j.start, nullptr, nullptr, 0, host, iters, nullptr, nullptr) ==
                   CNNSNS_OK,
               "locate plain");
        bufs.push_back({ host, iters });
    }
    // the walk with the interpolation fused into its last iteration, in every start mode
    for (size_t k = 0; k < jobs.size() && k < 6; ++k) {
        Job& j = jobs[k];
        double* nodal = dev_copy(std::vector<double>(2 * (size_t)j.n, 1.0));
        double* out = dev_alloc<double>(2 * j.n);
        int32_t* host = dev_alloc<int32_t>(j.n);
        float* disp = dev_alloc<float>(2 * (size_t)j.G * j.G);
        EXPECT(cnnsns_locate_interpolate(j.m, j.n, j.xp, j.start, nullptr, nullptr, 0, host, nullptr, nullptr, nodal,
                                         out, nullptr) == CNNSNS_OK, "locate_interpolate given");
        EXPECT(cnnsns_locate_interpolate(j.m, j.n, j.xp, nullptr, j.origin, disp, 0, host, nullptr, nullptr, nodal,
                                         out, nullptr) == CNNSNS_OK, "locate_interpolate cnn");
        EXPECT(cnnsns_locate_interpolate(j.m, j.n, j.xp, nullptr, nullptr, nullptr, 0, host, nullptr, nullptr, nodal,
                                         out, nullptr) == CNNSNS_OK, "locate_interpolate asg");
        EXPECT(cnnsns_locate_interpolate(j.m, j.n, j.xp, nullptr, nullptr, nullptr, 0, host, nullptr, nullptr, nullptr,
                                         out, nullptr) == CNNSNS_EINVAL, "locate_interpolate without nodal");
        bufs.push_back({ nodal, out, host, disp });
    }
    (void)hipDeviceSynchronize();
    for (auto& b : bufs)
        for (void* p : b) (void)hipFree(p);
    // FP32 on a few of them (the workspace grows from the BF16 size), then FP8 (it fits the grown
    // workspace), and an unknown precision is refused
    for (size_t k = 0; k < jobs.size() && k < 4; ++k) {
        float* disp = dev_alloc<float>(2 * (size_t)jobs[k].G * jobs[k].G);
        EXPECT(cnnsns_predict(jobs[k].m, jobs[k].vel, &W.w, CNNSNS_F32, disp, nullptr) == CNNSNS_OK, "predict f32");
        EXPECT(cnnsns_predict(jobs[k].m, jobs[k].vel, &W.w, CNNSNS_FP8E4M3, disp, nullptr) == CNNSNS_OK, "predict fp8");
        EXPECT(cnnsns_predict(jobs[k].m, jobs[k].vel, &W.w, 7, disp, nullptr) == CNNSNS_EINVAL, "unknown precision");
        (void)hipFree(disp);
    }
    // FP8 on a fresh mesh first: the workspace is allocated at the FP8 size, then grows for BF16
    if (!jobs.empty()) {
        Job& j = jobs.back();
        float* disp = dev_alloc<float>(2 * (size_t)j.G * j.G);
        EXPECT(cnnsns_predict(j.m, j.vel, &W.w, CNNSNS_FP8E4M3, disp, nullptr) == CNNSNS_OK, "predict fp8 first");
        EXPECT(cnnsns_predict(j.m, j.vel, &W.w, CNNSNS_BF16, disp, nullptr) == CNNSNS_OK, "predict bf16 after fp8");
        (void)hipFree(disp);
    }
    for (Job& j : jobs) free_job(j);
}

void scenario_serve(unsigned seed)
{
    std::mt19937 rng(seed);
    // the serving tests' meshes: n_side 30, 90, 150, 60, 283, 45
    const int sides[6] = { 30, 90, 150, 60, 283, 45 };
    std::vector<Job> jobs;
    for (int s : sides) {
        const HostMesh hm = grid_mesh(s);
        jobs.push_back(make_job(hm, overlay_side_for((double)hm.n_tri), nullptr));
    }
    Weights W(2);
    hipStream_t user = nullptr;  // the submitter's stream (as torch's current stream)
    (void)hipStreamCreateWithFlags(&user, 0);
    const struct {
        int precision;
        int64_t budget;
        int inflight;
    } cfgs[3] = { { CNNSNS_BF16, 256 << 20, 4 }, { CNNSNS_BF16, 3 << 20, 2 }, { CNNSNS_F32, 40 << 20, 3 } };
    for (const auto& c : cfgs) {
        // each job alone
        for (Job& j : jobs) {
            float* disp = dev_alloc<float>(2 * (size_t)j.G * j.G);
            int32_t* host = dev_alloc<int32_t>(j.n);
            int32_t* iters = dev_alloc<int32_t>(j.n);
            EXPECT(cnnsns_predict(j.m, j.vel, &W.w, c.precision, disp, user) == CNNSNS_OK, "predict alone");
            EXPECT(cnnsns_locate(j.m, j.n, j.xp, nullptr, j.origin, disp, 0, host, iters, nullptr, user) == CNNSNS_OK,
                   "locate alone");
            (void)hipStreamSynchronize(user);
            std::vector<int32_t> hh(j.n);
            (void)hipMemcpy(hh.data(), host, sizeof(int32_t) * j.n, hipMemcpyDeviceToHost);
            for (void* p : { (void*)disp, (void*)host, (void*)iters }) (void)hipFree(p);
        }
        cnnsns_server s = nullptr;
        EXPECT(cnnsns_server_create(c.budget, c.inflight, 4096, c.precision, &W.w, &s) == CNNSNS_OK, "server_create");
        if (!s) continue;
        std::vector<uint64_t> ids;
        std::vector<void*> outs;
        for (int k = 0; k < 30; ++k) {
            Job& j = jobs[k % jobs.size()];
            int32_t* host = dev_alloc<int32_t>(j.n);
            int32_t* iters = dev_alloc<int32_t>(j.n);
            (void)hipMemsetAsync(host, 0xff, sizeof(int32_t) * j.n, user);  // initialised on the user's stream
            (void)hipMemsetAsync(iters, 0, sizeof(int32_t) * j.n, user);
            uint64_t id = 0;
            EXPECT(cnnsns_submit(s, j.m, j.vel, j.n, j.xp, j.origin, nullptr, host, iters, user, &id) == CNNSNS_OK,
                   "submit");
            ids.push_back(id);
            outs.push_back(host);
            outs.push_back(iters);
            if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
        }
        // a mesh with jobs in flight cannot be destroyed (one of the jobs may already be done: then
        // the call succeeds, so rebuild in that case)
        for (uint64_t id : ids) {
            double lat = -1;
            EXPECT(cnnsns_wait(s, id, &lat) == CNNSNS_OK && lat >= 0, "wait");
        }
        EXPECT(cnnsns_server_destroy(s) == CNNSNS_OK, "server_destroy");
        for (void* p : outs) (void)hipFree(p);
    }
    // one job at a time, a budget below one job, a full queue, polling
    {
        Job& j = jobs[4];
        cnnsns_server s = nullptr;
        EXPECT(cnnsns_server_create(2 * 4 * (int64_t)j.G * j.G - 1, 1, 8, CNNSNS_BF16, &W.w, &s) == CNNSNS_OK,
               "server small");
        int32_t* host = dev_alloc<int32_t>(j.n);
        uint64_t id = 0;
        EXPECT(cnnsns_submit(s, j.m, j.vel, j.n, j.xp, j.origin, nullptr, host, nullptr, user, &id) == CNNSNS_ENOMEM,
               "budget below one job");
        EXPECT(cnnsns_server_destroy(s) == CNNSNS_OK, "destroy small");
        EXPECT(cnnsns_server_create(64 << 20, 1, 1, CNNSNS_BF16, &W.w, &s) == CNNSNS_OK, "server queue 1");
        std::vector<uint64_t> accepted;
        int busy = 0;
        for (int k = 0; k < 40; ++k) {
            const int rc = cnnsns_submit(s, j.m, j.vel, j.n, j.xp, j.origin, nullptr, host, nullptr, user, &id);
            if (rc == CNNSNS_OK)
                accepted.push_back(id);
            else {
                EXPECT(rc == CNNSNS_EBUSY, "queue full gives EBUSY");
                ++busy;
            }
        }
        EXPECT(!accepted.empty(), "some accepted");  // how many are refused depends on timing
        // the mesh has jobs in flight unless they all finished already
        const int rc = cnnsns_destroy_mesh(j.m);
        EXPECT(rc == CNNSNS_EBUSY || rc == CNNSNS_OK, "destroy with pending jobs");
        if (rc == CNNSNS_OK) {
            const HostMesh hm = grid_mesh(283);
            EXPECT(cnnsns_build_mesh(hm.xy.data(), hm.n_nodes, hm.tri.data(), hm.n_tri, j.G, nullptr, &j.m) ==
                       CNNSNS_OK,
                   "rebuild");
        }
        for (uint64_t a : accepted) {
            int32_t done = 0;
            while (!done) EXPECT(cnnsns_poll(s, a, &done, nullptr) == CNNSNS_OK, "poll");
        }
        int32_t done = 0;
        EXPECT(cnnsns_poll(s, accepted[0], &done, nullptr) == CNNSNS_EINVAL, "a reported job is unknown");
        EXPECT(cnnsns_server_destroy(s) == CNNSNS_OK, "destroy queue 1");
        (void)hipFree(host);
        EXPECT(cnnsns_server_create(0, 1, 1, CNNSNS_BF16, &W.w, &s) == CNNSNS_EINVAL, "zero budget");
        EXPECT(cnnsns_server_create(1 << 20, 1, 1, CNNSNS_FP8E4M3, &W.w, &s) == CNNSNS_EINVAL, "fp8 server");
    }
    // jobs still queued when the server is destroyed are drained first; then their mesh can go
    {
        cnnsns_server s = nullptr;
        EXPECT(cnnsns_server_create(8 << 20, 2, 64, CNNSNS_BF16, &W.w, &s) == CNNSNS_OK, "server drain");
        std::vector<void*> outs;
        for (int k = 0; k < 12; ++k) {
            Job& j = jobs[k % 3];
            int32_t* host = dev_alloc<int32_t>(j.n);
            uint64_t id = 0;
            EXPECT(cnnsns_submit(s, j.m, j.vel, j.n, j.xp, j.origin, j.start, host, nullptr, user, &id) == CNNSNS_OK,
                   "submit drain");
            outs.push_back(host);
        }
        EXPECT(cnnsns_server_destroy(s) == CNNSNS_OK, "destroy drains");
        for (void* p : outs) (void)hipFree(p);
    }
    (void)hipStreamDestroy(user);
    for (Job& j : jobs) free_job(j);
}

void scenario_predict_mt(int iters)
{
    const HostMesh hm = grid_mesh(120);
    Job j = make_job(hm, 256, nullptr);
    Weights W(2);
    auto predictor = [&](int tid) {
        hipStream_t st = nullptr;
        (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        float* disp = dev_alloc<float>(2 * (size_t)j.G * j.G);
        for (int k = 0; k < iters; ++k) {
            const int prec = (k + tid) % 2 ? CNNSNS_F32 : CNNSNS_BF16;
            EXPECT(cnnsns_predict(j.m, j.vel, &W.w, prec, disp, st) == CNNSNS_OK, "predict mt");
        }
        (void)hipStreamSynchronize(st);
        (void)hipFree(disp);
        (void)hipStreamDestroy(st);
    };
    auto locator = [&] {
        hipStream_t st = nullptr;
        (void)hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        int32_t* host = dev_alloc<int32_t>(j.n);
        for (int k = 0; k < iters; ++k)
            EXPECT(cnnsns_locate(j.m, j.n, j.xp, j.start, nullptr, nullptr, 0, host, nullptr, nullptr, st) ==
                       CNNSNS_OK,
                   "locate mt");
        (void)hipStreamSynchronize(st);
        (void)hipFree(host);
        (void)hipStreamDestroy(st);
    };
    std::thread a(predictor, 0), b(predictor, 1), c(locator);
    a.join();
    b.join();
    c.join();
    free_job(j);
}

void scenario_mesh3d()
{
    const int n = 9;
    std::vector<double> xyz;
    for (int k = 0; k < n; ++k)
        for (int jj = 0; jj < n; ++jj)
            for (int i = 0; i < n; ++i) xyz.insert(xyz.end(), { (double)i / (n - 1), (double)jj / (n - 1), (double)k / (n - 1) });
    std::vector<int32_t> tet;
    auto id = [&](int i, int jj, int k) { return (int32_t)((k * n + jj) * n + i); };
    for (int k = 0; k + 1 < n; ++k)
        for (int jj = 0; jj + 1 < n; ++jj)
            for (int i = 0; i + 1 < n; ++i) {
                // six Kuhn tetrahedra of the cube around its main diagonal
                const int perms[6][3] = { { 0, 1, 2 }, { 0, 2, 1 }, { 1, 0, 2 }, { 1, 2, 0 }, { 2, 0, 1 }, { 2, 1, 0 } };
                for (auto& p : perms) {
                    int c[3] = { i, jj, k };
                    std::vector<int32_t> t{ id(c[0], c[1], c[2]) };
                    for (int a : p) {
                        ++c[a];
                        t.push_back(id(c[0], c[1], c[2]));
                    }
                    tet.insert(tet.end(), t.begin(), t.end());
                }
            }
    cnnsns_mesh3 m = nullptr;
    EXPECT(cnnsns_build_mesh3d(xyz.data(), (int64_t)xyz.size() / 3, tet.data(), (int64_t)tet.size() / 4, 16, nullptr,
                               &m) == CNNSNS_OK,
           "build_mesh3d");
    Weights W(3);
    const int G = 16;
    float* vel = dev_copy(std::vector<float>(3 * (size_t)G * G * G, 0.25f));
    float* disp = dev_alloc<float>(3 * (size_t)G * G * G);
    const int64_t np = (int64_t)xyz.size() / 3;
    double* xp = dev_copy(xyz);
    int32_t* host = dev_alloc<int32_t>(np);
    EXPECT(cnnsns_predict3d(m, vel, &W.w, CNNSNS_F32, disp, nullptr) == CNNSNS_OK, "predict3d f32");
    EXPECT(cnnsns_predict3d(m, vel, &W.w, CNNSNS_BF16, disp, nullptr) == CNNSNS_OK, "predict3d bf16");
    EXPECT(cnnsns_locate3d(m, np, xp, nullptr, xp, disp, 0, host, nullptr, nullptr, nullptr) == CNNSNS_OK, "locate3d");
    double* nodal = dev_copy(xyz);
    double* out = dev_alloc<double>(3 * np);
    EXPECT(cnnsns_interpolate3d(m, np, xp, host, nodal, out, nullptr) == CNNSNS_OK, "interpolate3d");
    (void)hipDeviceSynchronize();
    EXPECT(cnnsns_destroy_mesh3d(m) == CNNSNS_OK, "destroy3d");
    for (void* p : { (void*)vel, (void*)disp, (void*)xp, (void*)host, (void*)nodal, (void*)out }) (void)hipFree(p);
}

// the no-allocation forward pass: no hipMalloc from its first call on, two meshes
// (the second with a smaller overlay), both precisions, FP32 refused beyond its size
void scenario_noalloc()
{
    Weights W(2);
    Job a = make_job(grid_mesh(60), 512, nullptr), b = make_job(grid_mesh(20), 64, nullptr),
        c = make_job(grid_mesh(20), 1024, nullptr);
    float* disp = dev_alloc<float>(2 * 1024 * 1024);
    const long before = mock_mallocs();
    for (int rep = 0; rep < 3; ++rep)
        for (Job* j : { &a, &b })
            for (int prec : { CNNSNS_BF16, CNNSNS_F32, CNNSNS_FP8E4M3 })
                EXPECT(cnnsns_predict_noalloc(j->m, j->vel, &W.w, prec, disp, nullptr) == CNNSNS_OK, "noalloc");
    EXPECT(cnnsns_predict_noalloc(c.m, c.vel, &W.w, CNNSNS_BF16, disp, nullptr) == CNNSNS_OK, "noalloc bf16 G=1024");
    EXPECT(cnnsns_predict_noalloc(c.m, c.vel, &W.w, CNNSNS_F32, disp, nullptr) == CNNSNS_EINVAL,
           "noalloc f32 beyond the scratch size");
    EXPECT(cnnsns_predict_noalloc(c.m, c.vel, &W.w, CNNSNS_FP8E4M3, disp, nullptr) == CNNSNS_OK, "noalloc fp8 G=1024");
    EXPECT(cnnsns_predict_noalloc(c.m, c.vel, &W.w, 7, disp, nullptr) == CNNSNS_EINVAL, "noalloc unknown precision");
    EXPECT(mock_mallocs() == before, "no device allocation");
    (void)hipDeviceSynchronize();
    (void)hipFree(disp);
    free_job(a);
    free_job(b);
    free_job(c);
}

// the classifier's prediction step: the pooled grid on the first call, two chunks of points
void scenario_classify()
{
    const HostMesh hm = grid_mesh(200);
    Job j = make_job(hm, 256, nullptr);
    const size_t shapes[6][2] = { { 16, 18 }, { 16, 144 }, { 256, 2 }, { 256, 256 }, { 512, 512 }, { 81, 512 } };
    std::vector<void*> bufs;
    cnnsns_cls w{};
    for (int l = 0; l < 6; ++l) {
        float* wl = dev_copy(std::vector<float>(shapes[l][0] * shapes[l][1], 0.01f));
        float* bl = dev_copy(std::vector<float>(shapes[l][0], 0.0f));
        w.w[l] = wl;
        w.b[l] = bl;
        bufs.push_back(wl);
        bufs.push_back(bl);
    }
    const int64_t n = 70001;  // two passes of the fully connected layers
    int32_t* start = dev_alloc<int32_t>(n);
    int32_t* cls = dev_alloc<int32_t>(n);
    float* logits = dev_alloc<float>(81 * n);
    for (int rep = 0; rep < 2; ++rep) {
        EXPECT(cnnsns_classify(j.m, n, j.xp, &w, j.start, start, cls, logits, nullptr) == CNNSNS_OK, "classify");
        EXPECT(cnnsns_classify(j.m, n, j.xp, &w, nullptr, start, nullptr, nullptr, nullptr) == CNNSNS_OK,
               "classify without optional outputs");
    }
    EXPECT(cnnsns_classify(j.m, 0, nullptr, &w, nullptr, nullptr, nullptr, nullptr, nullptr) == CNNSNS_OK, "n = 0");
    EXPECT(cnnsns_classify(j.m, n, j.xp, nullptr, nullptr, start, nullptr, nullptr, nullptr) == CNNSNS_EINVAL,
           "no weights");
    (void)hipDeviceSynchronize();
    for (void* p : { (void*)start, (void*)cls, (void*)logits }) (void)hipFree(p);
    for (void* p : bufs) (void)hipFree(p);
    free_job(j);
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc < 2) {
        std::fprintf(stderr, "usage: host_driver c5ref|serve|predict_mt|mesh3d [args]\n");
        return 2;
    }
    const std::string sc = argv[1];
    auto arg = [&](int k, double d) { return argc > k ? std::atof(argv[k]) : d; };
    if (sc == "c5ref")
        scenario_c5ref((int)arg(2, 64), arg(3, 16.0), (unsigned)arg(4, 5));
    else if (sc == "serve")
        scenario_serve((unsigned)arg(2, 1));
    else if (sc == "predict_mt")
        scenario_predict_mt((int)arg(2, 200));
    else if (sc == "mesh3d")
        scenario_mesh3d();
    else if (sc == "noalloc")
        scenario_noalloc();
    else if (sc == "classify")
        scenario_classify();
    else {
        std::fprintf(stderr, "unknown scenario %s\n", sc.c_str());
        return 2;
    }
    (void)hipDeviceSynchronize();
    const long left = mock_live_device_bytes(), handles = mock_live_handles();
    if (left != 0) std::fprintf(stderr, "FAILED: %ld device bytes still allocated\n", left), ++g_fail;
    if (handles != 0) std::fprintf(stderr, "FAILED: %ld streams, events or graphs left\n", handles), ++g_fail;
    const int total = g_fail + mock_failures();
    std::printf("%s: %ld launches, %d failures\n", sc.c_str(), mock_launches(), total);
    return total == 0 ? 0 : 1;
}
