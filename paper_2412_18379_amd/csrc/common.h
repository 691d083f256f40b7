// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/cnnsns.h"

namespace cnnsns {

// One mesh element as the walk reads it: the three counter-clockwise vertex
// coordinates and the three neighbour ids (neighbour j across the edge
// opposite vertex j, -1 on the boundary), packed into one 64-byte aligned
// record so that a hop is a single 64-byte gather.
struct alignas(64) ElemRec {
    double ax, ay, bx, by, cx, cy;
    int32_t n0, n1, n2, pad;
};
static_assert(sizeof(ElemRec) == 64, "element record must be 64 bytes");

// One tetrahedron as the 3D walk reads it, in one 128-byte record (one line
// per hop): its vertices in ascending node-id order, the neighbour across the
// face opposite each (-1 on the boundary), the orientation of that vertex
// order (+1 or -1), and each vertex's position in the positively oriented
// element order (one byte per vertex, low byte first).
struct alignas(128) TetRec {
    double v[4][3];
    int32_t nbr[4];
    int32_t orient;
    uint32_t pos;
    int32_t pad[2];
};
static_assert(sizeof(TetRec) == 128, "tetrahedron record must be 128 bytes");

// Error with a status code; thrown inside the library and turned into a
// return code plus a thread-local message at the C boundary.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);
void hip_check(hipError_t e, const char* what);

// Device workspace a mesh keeps for its CNN forward passes, allocated on the
// first pass and grown when a larger one is needed.  Passes on one mesh share
// it, so each pass is ordered on the device after the previous one (an event
// recorded after the last pass, waited on by the next pass's stream);
// growing frees the old buffer only after the device has drained.
struct Workspace {
    std::mutex mu;
    void* ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t last_use = nullptr;  // recorded after the last pass that used ptr
};

// Makes ws.ptr at least `need` bytes and orders `stream` after the previous
// pass that used it.  Call with ws.mu held; after enqueueing the pass, call
// workspace_used with the lock still held.
void workspace_acquire(Workspace& ws, size_t need, hipStream_t stream, const char* what);
void workspace_used(Workspace& ws, hipStream_t stream);
// Frees the buffer and the event (the caller has synchronised the device).
void workspace_release(Workspace& ws);

}  // namespace cnnsns

struct cnnsns_mesh_s {
    int device = 0;
    int64_t n_nodes = 0;
    int64_t n_tri = 0;
    int32_t G = 0;
    double mean_diam = 0.0;
    cnnsns::ElemRec* rec = nullptr;  // device [n_tri]
    int32_t* tri = nullptr;          // device [n_tri][3] node ids, in the records' counter-clockwise order
    int32_t* lookup = nullptr;       // device [G][G]
    int64_t device_bytes = 0;
    // CNN workspace, allocated on the first cnnsns_predict of this mesh
    cnnsns::Workspace ws;
    // serving jobs submitted on this mesh and not yet complete (destroy refuses while > 0)
    std::atomic<int64_t> pending_jobs{ 0 };
    // classifier CNN: the average-pooled overlay of element centroids (FP64 [G][G][2], built on the first
    // cnnsns_classify) and the workspace of its layers
    void* cls_pool = nullptr;
    cnnsns::Workspace cls_ws;
};

struct cnnsns_mesh3_s {
    int device = 0;
    int64_t n_nodes = 0;
    int64_t n_tet = 0;
    int32_t G = 0;
    cnnsns::TetRec* rec = nullptr;  // device [n_tet]
    int32_t* ids = nullptr;         // device [n_tet][4] node ids, in the records' (ascending id) order
    int32_t* lookup = nullptr;      // device [G][G][G]
    int64_t device_bytes = 0;
    // 3D CNN workspace, allocated on the first cnnsns_predict3d of this mesh
    cnnsns::Workspace ws;
};

namespace cnnsns {

// mesh3d.hip
cnnsns_mesh3 build_mesh3(const double* xyz, int64_t n_nodes, const int32_t* tet, int64_t n_tet, int32_t G,
                         hipStream_t stream);
void destroy_mesh3(cnnsns_mesh3 m);
void launch_locate3(const cnnsns_mesh3_s& m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                    const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status,
                    hipStream_t stream);
void launch_interp3(const cnnsns_mesh3_s& m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                    double* out, hipStream_t stream);
// cnn3d.hip
size_t cnn3_workspace_bytes(int32_t G);
void run_predict3(cnnsns_mesh3_s& m, const float* vel, const cnnsns_cnn& w, int32_t precision, float* disp,
                  hipStream_t stream);

// mesh.hip
cnnsns_mesh build_mesh(const double* xy, int64_t n_nodes, const int32_t* tri, int64_t n_tri, int32_t G,
                       hipStream_t stream);
void destroy_mesh(cnnsns_mesh m);

// sns_walk.hip
enum StartMode { START_GIVEN = 0, START_CNN = 1, START_ASG = 2 };
void launch_interp(const cnnsns_mesh_s& m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                   double* out, hipStream_t stream);
// with nodal (FP64 [n_nodes][2]) and out (FP64 [n][2]), also the P1 interpolant at x_p in the host
void launch_locate(const cnnsns_mesh_s& m, int64_t n, const double* xp, const int32_t* start,
                   const double* origin, const float* disp, int32_t max_iter, int32_t* host, int32_t* iters,
                   uint8_t* status, hipStream_t stream, const double* nodal = nullptr, double* out = nullptr);

// classifier.hip
size_t cls_workspace_bytes(int64_t n);
void run_classify(cnnsns_mesh_s& m, int64_t n, const double* xp, const cnnsns_cls& w, const int32_t* fallback,
                  int32_t* start, int32_t* cls, float* logits, hipStream_t stream);

// cnn.hip
unsigned cnn_persistent_grid();  // one block per compute unit
size_t cnn_workspace_bytes(int32_t G, int32_t precision);
void run_cnn(int32_t G, const float* vel, const cnnsns_cnn& w, int32_t precision, float* disp, void* ws,
             hipStream_t stream);
// cnn_bf16.hip
size_t cnn_fp8_workspace_bytes();
void cnn_fp8_forward(int32_t G, const float* vel, const cnnsns_cnn& w, float* disp, void* ws, unsigned grid,
                     hipStream_t stream);
size_t cnn_bf16_workspace_bytes();
void cnn_bf16_pack(const cnnsns_cnn& w, void* packed, hipStream_t stream);
void cnn_bf16_forward(int32_t G, const float* vel, const void* packed, const cnnsns_cnn& w, float* disp,
                      unsigned grid, hipStream_t stream);
void run_predict(cnnsns_mesh_s& m, const float* vel, const cnnsns_cnn& w, int32_t precision, float* disp,
                 hipStream_t stream);
// the same pass with the preallocated per-device workspace (no allocation)
size_t cnn_scratch_bytes();
void run_predict_noalloc(const cnnsns_mesh_s& m, const float* vel, const cnnsns_cnn& w, int32_t precision,
                         float* disp, hipStream_t stream);

}  // namespace cnnsns
