// Host stand-ins for the library's mesh build and kernel launchers, so that
// api.cpp and serve.cpp link without a GPU.  "Launches" run at once on the host:
// the walk writes host[i] = mesh tag + i and iters[i] = 1, the forward pass
// fills the displacement grid, so a test can tell which job wrote what and
// AddressSanitizer sees every arena access.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "../../paper_2412_18379_amd/csrc/common.h"

std::atomic<long> mock_live_objects{0};
std::atomic<long> mock_bytes{0};

namespace cnnsns {

cnnsns_mesh build_mesh(const double*, int64_t n_nodes, const int32_t*, int64_t n_tri, int32_t G, hipStream_t)
{
    auto* m = new cnnsns_mesh_s();
    m->n_nodes = n_nodes;
    m->n_tri = n_tri;
    m->G = G;
    return m;
}

void destroy_mesh(cnnsns_mesh m)
{
    delete m;
}

void run_predict(cnnsns_mesh_s& m, const float* vel, const cnnsns_cnn&, int32_t, float* disp, hipStream_t)
{
    std::memcpy(disp, vel, sizeof(float) * 2 * (size_t)m.G * (size_t)m.G);
}

unsigned cnn_persistent_grid()
{
    return 256;
}

size_t cnn_workspace_bytes(int32_t G, int32_t precision)
{
    if (precision == CNNSNS_BF16) return cnn_bf16_workspace_bytes();
    return sizeof(float) * (2 * 9216 + 32 * (size_t)G * (size_t)G);
}

size_t cnn_bf16_workspace_bytes()
{
    return 1 << 16;
}

void cnn_bf16_pack(const cnnsns_cnn&, void* packed, hipStream_t)
{
    std::memset(packed, 0, cnn_bf16_workspace_bytes());
}

void cnn_bf16_forward(int32_t G, const float* vel, const void*, const cnnsns_cnn&, float* disp, unsigned,
                      hipStream_t)
{
    std::memcpy(disp, vel, sizeof(float) * 2 * (size_t)G * (size_t)G);
}

void run_cnn(int32_t G, const float* vel, const cnnsns_cnn&, int32_t, float* disp, void* ws, hipStream_t)
{
    std::memset(ws, 0, cnn_workspace_bytes(G, CNNSNS_F32));
    std::memcpy(disp, vel, sizeof(float) * 2 * (size_t)G * (size_t)G);
}

void launch_interp(const cnnsns_mesh_s&, int64_t, const double*, const int32_t*, const double*, double*, hipStream_t)
{
}

size_t cnn_scratch_bytes()
{
    return 0;
}

void run_predict_noalloc(const cnnsns_mesh_s&, const float*, const cnnsns_cnn&, int32_t, float*, hipStream_t)
{
    fail(CNNSNS_EINVAL, "the mock runtime has no preallocated workspace");
}

void run_classify(cnnsns_mesh_s&, int64_t, const double*, const cnnsns_cls&, const int32_t*, int32_t*, int32_t*,
                  float*, hipStream_t)
{
    fail(CNNSNS_EINVAL, "the mock runtime has no classifier");
}

cnnsns_mesh3 build_mesh3(const double*, int64_t, const int32_t*, int64_t, int32_t, hipStream_t)
{
    fail(CNNSNS_EINVAL, "the mock runtime has no 3D meshes");
}

void destroy_mesh3(cnnsns_mesh3) {}

void launch_locate3(const cnnsns_mesh3_s&, int64_t, const double*, const int32_t*, const double*, const float*,
                    int32_t, int32_t*, int32_t*, uint8_t*, hipStream_t)
{
}

size_t cnn3_workspace_bytes(int32_t) { return 0; }

void launch_interp3(const cnnsns_mesh3_s&, int64_t, const double*, const int32_t*, const double*, double*, hipStream_t)
{
}

void run_predict3(cnnsns_mesh3_s&, const float*, const cnnsns_cnn&, int32_t, float*, hipStream_t) {}

void launch_locate(const cnnsns_mesh_s& m, int64_t n, const double* xp, const int32_t*, const double* origin,
                   const float* disp, int32_t, int32_t* host, int32_t* iters, uint8_t*, hipStream_t, const double*,
                   double*)
{
    volatile float sink = disp[2 * (size_t)m.G * (size_t)m.G - 1];
    (void)sink;
    for (int64_t i = 0; i < n; ++i) {
        host[i] = (int32_t)(m.n_nodes + i) + (int32_t)(xp[2 * i] + origin[2 * i + 1]);
        if (iters) iters[i] = 1;
    }
}

}  // namespace cnnsns
