// Drives the serving loop through the C ABI on the host (mock HIP runtime):
// uneven meshes, batches of submissions, waits in and out of order, polling,
// Poisson-like arrivals, budget-bound admission and error paths.  Every job's
// output is checked against what its own launch must have written.
//
// usage: serve_driver <precision 0|1> <budget bytes> <max_inflight> <n_meshes> <n_jobs> <seed>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

#include "../../include/cnnsns.h"
#include <hip/hip_runtime.h>

extern std::atomic<long> mock_live_objects;

namespace {

struct MeshData {
    cnnsns_mesh m = nullptr;
    int64_t n = 0;
    int32_t G = 0;
    std::vector<float> vel;
    std::vector<double> xp, origin;
};

struct Out {
    int mesh;
    uint64_t id;
    std::vector<int32_t> host, iters;
};

int g_failures = 0;

void expect(bool ok, const char* what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s (%s)\n", what, cnnsns_last_error());
        ++g_failures;
    }
}

bool check_out(const MeshData& d, const Out& o)
{
    for (int64_t i = 0; i < d.n; ++i) {
        const int32_t want = (int32_t)(d.n + 1000 + i) + (int32_t)(d.xp[2 * i] + d.origin[2 * i + 1]);
        if (o.host[i] != want || o.iters[i] != 1) return false;
    }
    return true;
}

}  // namespace

int main(int argc, char** argv)
{
    if (argc != 7) {
        std::fprintf(stderr, "usage: serve_driver precision budget max_inflight n_meshes n_jobs seed\n");
        return 2;
    }
    const int precision = std::atoi(argv[1]);
    const int64_t budget = std::atoll(argv[2]);
    const int inflight = std::atoi(argv[3]);
    const int n_meshes = std::atoi(argv[4]);
    const int n_jobs = std::atoi(argv[5]);
    std::mt19937_64 rng(std::atoi(argv[6]));

    std::vector<float> wts(32 * 32 * 9, 0.5f);
    cnnsns_cnn w{};
    for (int l = 0; l < 4; ++l) {
        w.w[l] = wts.data();
        w.b[l] = wts.data();
    }
    // meshes: overlay sides 16 .. 512, point counts 0 .. 3000 (0 exercises the empty job)
    std::vector<MeshData> meshes(n_meshes);
    for (int k = 0; k < n_meshes; ++k) {
        MeshData& d = meshes[k];
        d.G = 16 << (rng() % 6);
        d.n = (k % 17 == 5) ? 0 : (int64_t)(rng() % 3000) + 1;
        d.vel.assign(2 * (size_t)d.G * d.G, (float)k);
        d.xp.resize(2 * d.n);
        d.origin.resize(2 * d.n);
        for (int64_t i = 0; i < 2 * d.n; ++i) {
            d.xp[i] = (double)(rng() % 7);
            d.origin[i] = (double)(rng() % 5);
        }
        expect(cnnsns_build_mesh(nullptr, d.n + 1000, nullptr, 2 * d.n, d.G, nullptr, &d.m) == CNNSNS_OK, "mesh");
    }
    cnnsns_server s = nullptr;
    expect(cnnsns_server_create(budget, inflight, 1 << 16, precision, &w, &s) == CNNSNS_OK, "create");
    if (!s) return 1;

    auto submit = [&](int mi) {
        MeshData& d = meshes[mi];
        Out o{ mi, 0, std::vector<int32_t>(d.n + 1, -7), std::vector<int32_t>(d.n + 1, 0) };  // never empty: host must not be NULL
        const bool empty = d.n == 0;  // an empty job may pass NULL point buffers
        const int rc = cnnsns_submit(s, d.m, d.vel.data(), d.n, empty ? nullptr : d.xp.data(),
                                     empty ? nullptr : d.origin.data(), nullptr, empty ? nullptr : o.host.data(),
                                     empty ? nullptr : o.iters.data(), nullptr, &o.id);
        expect(rc == CNNSNS_OK, "submit");
        return o;
    };

    // 1. warm-up then all meshes once, waits in submission order
    for (int pass = 0; pass < 2; ++pass) {
        const int count = pass == 0 ? std::min(16, n_meshes) : n_meshes;
        std::vector<Out> outs;
        outs.reserve(count);
        for (int k = 0; k < count; ++k) outs.push_back(submit(k));
        for (auto& o : outs) {
            double lat = -1;
            expect(cnnsns_wait(s, o.id, &lat) == CNNSNS_OK, "wait");
            expect(lat >= 0, "latency");
            expect(check_out(meshes[o.mesh], o), "output (in-order waits)");
        }
    }
    // 2. random order, arrivals spread in time, waits in reverse order, some by polling
    std::vector<Out> outs;
    outs.reserve(n_jobs);
    for (int k = 0; k < n_jobs; ++k) {
        outs.push_back(submit((int)(rng() % n_meshes)));
        if (rng() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 200));
    }
    for (int k = n_jobs - 1; k >= 0; --k) {
        Out& o = outs[k];
        if (k % 3 == 0) {
            int32_t done = 0;
            double lat = 0;
            for (;;) {
                const int rc = cnnsns_poll(s, o.id, &done, &lat);
                expect(rc == CNNSNS_OK, "poll");
                if (done || rc != CNNSNS_OK) break;
                std::this_thread::yield();
            }
        } else {
            expect(cnnsns_wait(s, o.id, nullptr) == CNNSNS_OK, "wait");
        }
        expect(check_out(meshes[o.mesh], o), "output (reverse waits)");
    }
    // 3. a reported job is unknown afterwards
    int32_t done = 0;
    expect(cnnsns_poll(s, outs.empty() ? 1 : outs[0].id, &done, nullptr) == CNNSNS_EINVAL, "second report");
    // 4. jobs left unreported at destroy time are drained
    for (int k = 0; k < std::min(n_meshes, 8); ++k) outs.push_back(submit(k));
    expect(cnnsns_server_destroy(s) == CNNSNS_OK, "destroy");
    for (auto& d : meshes) expect(cnnsns_destroy_mesh(d.m) == CNNSNS_OK, "destroy mesh");
    expect(mock_live_objects.load() == 0, "streams, events and graphs all destroyed");
    std::printf("serve_driver: %d failures\n", g_failures);
    return g_failures == 0 ? 0 : 1;
}
