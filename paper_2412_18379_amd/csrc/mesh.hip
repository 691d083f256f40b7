// Mesh residency: orientation, neighbour table, packed element records and
// the overlay cell -> element lookup, all built on the device.
//
// The element list {K_l} and neighbour table {m_j^l} are the inputs of the
// SNS walk (Sec. 2.2, eq. 6).  The overlay lookup is the auxiliary
// structured grid of Sec. 1 / Alg. 2: for each cell of a G x G grid on the
// unit square, the smallest id of an element whose closed region contains
// the cell centre.
#pragma clang fp contract(off)

#include <hipcub/hipcub.hpp>

#include <climits>
#include <cmath>
#include <vector>

#include "common.h"

namespace cnnsns {
namespace {

constexpr int kBlock = 256;

enum : int { ERR_INDEX = 1, ERR_AREA = 2, ERR_EDGE3 = 4, ERR_OVERLAP = 8 };

// Counter-clockwise order: swap the 2nd and 3rd vertex when the signed area
// (b - a) x (c - a) is negative.  Zero area and out-of-range ids are errors.
__global__ void k_canonicalise(int64_t n_tri, int64_t n_nodes, const double2* __restrict__ xy,
                               const int32_t* __restrict__ tri_in, int32_t* __restrict__ tri, int* err)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    int32_t a = tri_in[3 * t], b = tri_in[3 * t + 1], c = tri_in[3 * t + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n_nodes || b >= n_nodes || c >= n_nodes) {
        atomicOr(err, ERR_INDEX);
        tri[3 * t] = 0; tri[3 * t + 1] = 0; tri[3 * t + 2] = 0;
        return;
    }
    double2 A = xy[a], B = xy[b], C = xy[c];
    double d = (B.x - A.x) * (C.y - A.y) - (B.y - A.y) * (C.x - A.x);
    if (!(d > 0.0 || d < 0.0) || !isfinite(d)) atomicOr(err, ERR_AREA);  // zero, NaN or infinite
    tri[3 * t] = a;
    tri[3 * t + 1] = d < 0.0 ? c : b;
    tri[3 * t + 2] = d < 0.0 ? b : c;
}

__global__ void k_degree(int64_t n_tri, const int32_t* __restrict__ tri, unsigned long long* deg)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 3 * n_tri) return;
    atomicAdd(&deg[tri[k]], 1ull);
}

// Incidence lists: the triangles around each node, at inc[first[v] .. first[v+1]).
// The order inside a list is whatever the atomics give; only membership is used.
__global__ void k_fill(int64_t n_tri, const int32_t* __restrict__ tri, unsigned long long* cursor,
                       int32_t* __restrict__ inc)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 3 * n_tri) return;
    unsigned long long pos = atomicAdd(&cursor[tri[k]], 1ull);
    inc[pos] = (int32_t)(k / 3);
}

// Neighbour across the edge opposite vertex j of triangle t: the one other
// triangle around node u = v[(j+1)%3] that also holds w = v[(j+2)%3].
// With both triangles counter-clockwise, a proper neighbour traverses the
// edge w -> u; a second triangle holding u -> w overlaps t.
__global__ void k_neighbours(int64_t n_tri, const int32_t* __restrict__ tri,
                             const unsigned long long* __restrict__ first, const int32_t* __restrict__ inc,
                             int32_t* __restrict__ nbr, int* err)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 3 * n_tri) return;
    int64_t t = k / 3;
    int j = (int)(k - 3 * t);
    int32_t u = tri[3 * t + (j + 1) % 3], w = tri[3 * t + (j + 2) % 3];
    int32_t found = -1;
    int bad = 0;
    for (unsigned long long q = first[u]; q < first[u + 1]; ++q) {
        int32_t s = inc[q];
        if (s == t) continue;
        int32_t s0 = tri[3 * (int64_t)s], s1 = tri[3 * (int64_t)s + 1], s2 = tri[3 * (int64_t)s + 2];
        int iw = s0 == w ? 0 : (s1 == w ? 1 : (s2 == w ? 2 : -1));
        if (iw < 0) continue;
        int iu = s0 == u ? 0 : (s1 == u ? 1 : 2);
        if (found >= 0) bad |= ERR_EDGE3;
        if ((iu + 1) % 3 == iw) bad |= ERR_OVERLAP;
        found = s;
    }
    if (bad) atomicOr(err, bad);
    nbr[k] = found;
}

__global__ void k_pack(int64_t n_tri, const double2* __restrict__ xy, const int32_t* __restrict__ tri,
                       const int32_t* __restrict__ nbr, ElemRec* __restrict__ rec)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    double2 A = xy[tri[3 * t]], B = xy[tri[3 * t + 1]], C = xy[tri[3 * t + 2]];
    ElemRec r;
    r.ax = A.x; r.ay = A.y; r.bx = B.x; r.by = B.y; r.cx = C.x; r.cy = C.y;
    r.n0 = nbr[3 * t]; r.n1 = nbr[3 * t + 1]; r.n2 = nbr[3 * t + 2]; r.pad = 0;
    rec[t] = r;
}

__global__ void k_fill_i32(int64_t n, int32_t* p, int32_t v)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

__global__ void k_lookup_finish(int64_t n, int32_t* p)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && p[k] == INT_MAX) p[k] = -1;
}

// Overlay cells tested for one triangle: the cell centres inside its bounding
// box, grown by one cell (a conservative superset; the containment test
// decides).  Returns false when the box misses the grid.
struct CellBox {
    int32_t cx0, cy0, cx1, cy1;
};
__device__ __forceinline__ CellBox cell_box(const ElemRec& r, int32_t G)
{
    const double g = (double)G;
    double xmin = fmin(r.ax, fmin(r.bx, r.cx)), xmax = fmax(r.ax, fmax(r.bx, r.cx));
    double ymin = fmin(r.ay, fmin(r.by, r.cy)), ymax = fmax(r.ay, fmax(r.by, r.cy));
    // clamped before conversion (fmax and fmin return the number when the other is NaN)
    const double fx0 = fmax(floor(xmin * g - 0.5) - 1.0, 0.0), fx1 = fmin(ceil(xmax * g - 0.5) + 1.0, g - 1.0);
    const double fy0 = fmax(floor(ymin * g - 0.5) - 1.0, 0.0), fy1 = fmin(ceil(ymax * g - 0.5) + 1.0, g - 1.0);
    CellBox b;
    b.cx0 = fx0 > g - 1.0 ? G : (int32_t)fx0;
    b.cy0 = fy0 > g - 1.0 ? G : (int32_t)fy0;
    b.cx1 = fx1 < 0.0 ? -1 : (int32_t)fx1;
    b.cy1 = fy1 < 0.0 ? -1 : (int32_t)fy1;
    return b;
}

// Closed containment of the centre of cell (cx, cy), with the same
// barycentric numerators the walk uses.
__device__ __forceinline__ bool holds_centre(const ElemRec& r, int32_t cx, int32_t cy, int32_t G)
{
    const double g = (double)G;
    const double px = ((double)cx + 0.5) / g, py = ((double)cy + 0.5) / g;
    const double adx = r.ax - px, bdx = r.bx - px, cdx = r.cx - px;
    const double ady = r.ay - py, bdy = r.by - py, cdy = r.cy - py;
    const double s0 = bdx * cdy - bdy * cdx;
    const double s1 = cdx * ady - cdy * adx;
    const double s2 = adx * bdy - ady * bdx;
    return s0 >= 0.0 && s1 >= 0.0 && s2 >= 0.0;
}

constexpr int64_t kBigBox = 256;  // cells; larger boxes go to the block-parallel pass

// Rasterise one triangle per thread over its cell box, keeping the smallest
// containing id per cell.  Triangles with large boxes (a coarse mesh under a
// fine overlay) are listed for k_lookup_raster_big instead.
__global__ void k_lookup_raster(int64_t n_tri, const ElemRec* __restrict__ rec, int32_t G, int32_t* lookup,
                                int32_t* big, unsigned* n_big)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    const ElemRec r = rec[t];
    const CellBox b = cell_box(r, G);
    if (b.cx1 < b.cx0 || b.cy1 < b.cy0) return;
    if ((int64_t)(b.cx1 - b.cx0 + 1) * (b.cy1 - b.cy0 + 1) > kBigBox) {
        big[atomicAdd(n_big, 1u)] = (int32_t)t;
        return;
    }
    for (int32_t cy = b.cy0; cy <= b.cy1; ++cy)
        for (int32_t cx = b.cx0; cx <= b.cx1; ++cx)
            if (holds_centre(r, cx, cy, G)) atomicMin(&lookup[(int64_t)cy * G + cx], (int32_t)t);
}

// Listed triangles: blockIdx.y picks the triangle, all blocks along x and
// their threads stride over its cells.
__global__ void k_lookup_raster_big(const ElemRec* __restrict__ rec, const int32_t* __restrict__ big, unsigned n_big,
                                    int32_t G, int32_t* lookup)
{
    for (unsigned k = blockIdx.y; k < n_big; k += gridDim.y) {
        const int32_t t = big[k];
        const ElemRec r = rec[t];
        const CellBox b = cell_box(r, G);
        const int64_t w = b.cx1 - b.cx0 + 1, n = w * (b.cy1 - b.cy0 + 1);
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
            const int32_t cy = b.cy0 + (int32_t)(c / w), cx = b.cx0 + (int32_t)(c % w);
            if (holds_centre(r, cx, cy, G)) atomicMin(&lookup[(int64_t)cy * G + cx], t);
        }
    }
}

inline unsigned grid_for(int64_t n)
{
    return (unsigned)((n + kBlock - 1) / kBlock);
}

// Device allocation owned by one build step; freed on scope exit.
template <class T>
struct DevBuf {
    T* p = nullptr;
    explicit DevBuf(size_t count)
    {
        if (count == 0) count = 1;
        if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            fail(CNNSNS_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
        }
    }
    ~DevBuf() { if (p) (void)hipFree(p); }
    T* release() { T* q = p; p = nullptr; return q; }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
};

}  // namespace

cnnsns_mesh build_mesh(const double* xy, int64_t n_nodes, const int32_t* tri, int64_t n_tri, int32_t G,
                       hipStream_t stream)
{
    if (!xy || !tri) fail(CNNSNS_EINVAL, "build_mesh: xy and tri must not be NULL");
    if (n_nodes < 3) fail(CNNSNS_EINVAL, "build_mesh: n_nodes must be >= 3");
    if (n_tri < 1) fail(CNNSNS_EINVAL, "build_mesh: n_tri must be >= 1");
    if (n_tri > (int64_t)INT32_MAX / 3 || n_nodes > (int64_t)INT32_MAX)
        fail(CNNSNS_EINVAL, "build_mesh: mesh too large for int32 element / node ids");
    if (G < 0 || G > 65536) fail(CNNSNS_EINVAL, "build_mesh: overlay_side must be in [0, 65536]");
    if (G == 0) {
        int e = (int)std::ceil(std::log2(std::sqrt((double)n_tri)));
        G = 1 << (e < 0 ? 0 : (e > 16 ? 16 : e));
    }

    // mean element diameter (longest edge), on the host from the caller's arrays
    double sum = 0.0;
    for (int64_t t = 0; t < n_tri; ++t) {
        int32_t v[3] = { tri[3 * t], tri[3 * t + 1], tri[3 * t + 2] };
        double best = 0.0;
        for (int k = 0; k < 3; ++k) {
            int32_t a = v[k], b = v[(k + 1) % 3];
            if (a < 0 || b < 0 || a >= n_nodes || b >= n_nodes) fail(CNNSNS_EMESH, "build_mesh: node index out of range");
            double dx = xy[2 * (int64_t)b] - xy[2 * (int64_t)a], dy = xy[2 * (int64_t)b + 1] - xy[2 * (int64_t)a + 1];
            best = std::fmax(best, std::sqrt(dx * dx + dy * dy));
        }
        sum += best;
    }

    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    DevBuf<double2> d_xy((size_t)n_nodes);
    DevBuf<int32_t> d_tri_in((size_t)(3 * n_tri)), d_tri((size_t)(3 * n_tri)), d_nbr((size_t)(3 * n_tri));
    DevBuf<int32_t> d_inc((size_t)(3 * n_tri));
    DevBuf<unsigned long long> d_deg((size_t)n_nodes + 1), d_first((size_t)n_nodes + 1), d_cursor((size_t)n_nodes + 1);
    DevBuf<int> d_err(1);
    DevBuf<ElemRec> d_rec((size_t)n_tri);
    DevBuf<int32_t> d_lookup((size_t)G * (size_t)G);

    hip_check(hipMemcpyAsync(d_xy.p, xy, sizeof(double2) * (size_t)n_nodes, hipMemcpyHostToDevice, stream), "copy xy");
    hip_check(hipMemcpyAsync(d_tri_in.p, tri, sizeof(int32_t) * 3 * (size_t)n_tri, hipMemcpyHostToDevice, stream),
              "copy tri");
    hip_check(hipMemsetAsync(d_err.p, 0, sizeof(int), stream), "memset");
    hip_check(hipMemsetAsync(d_deg.p, 0, sizeof(unsigned long long) * ((size_t)n_nodes + 1), stream), "memset");

    k_canonicalise<<<grid_for(n_tri), kBlock, 0, stream>>>(n_tri, n_nodes, d_xy.p, d_tri_in.p, d_tri.p, d_err.p);
    k_degree<<<grid_for(3 * n_tri), kBlock, 0, stream>>>(n_tri, d_tri.p, d_deg.p);
    size_t tmp_bytes = 0;
    hip_check(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, d_deg.p, d_first.p, (int)(n_nodes + 1), stream),
              "scan size");
    {
        DevBuf<unsigned char> d_tmp(tmp_bytes);
        hip_check(hipcub::DeviceScan::ExclusiveSum(d_tmp.p, tmp_bytes, d_deg.p, d_first.p, (int)(n_nodes + 1), stream),
                  "scan");
        hip_check(hipMemcpyAsync(d_cursor.p, d_first.p, sizeof(unsigned long long) * ((size_t)n_nodes + 1),
                                 hipMemcpyDeviceToDevice, stream), "copy cursor");
        k_fill<<<grid_for(3 * n_tri), kBlock, 0, stream>>>(n_tri, d_tri.p, d_cursor.p, d_inc.p);
        k_neighbours<<<grid_for(3 * n_tri), kBlock, 0, stream>>>(n_tri, d_tri.p, d_first.p, d_inc.p, d_nbr.p,
                                                                 d_err.p);
        k_pack<<<grid_for(n_tri), kBlock, 0, stream>>>(n_tri, d_xy.p, d_tri.p, d_nbr.p, d_rec.p);
        const int64_t ncell = (int64_t)G * G;
        k_fill_i32<<<grid_for(ncell), kBlock, 0, stream>>>(ncell, d_lookup.p, INT_MAX);
        DevBuf<int32_t> d_big((size_t)n_tri);
        DevBuf<unsigned> d_nbig(1);
        hip_check(hipMemsetAsync(d_nbig.p, 0, sizeof(unsigned), stream), "memset");
        k_lookup_raster<<<grid_for(n_tri), kBlock, 0, stream>>>(n_tri, d_rec.p, G, d_lookup.p, d_big.p, d_nbig.p);
        unsigned n_big = 0;
        hip_check(hipMemcpyAsync(&n_big, d_nbig.p, sizeof(unsigned), hipMemcpyDeviceToHost, stream), "copy n_big");
        hip_check(hipStreamSynchronize(stream), "lookup raster");
        if (n_big > 0) {
            const dim3 grid(64, n_big < 4096u ? n_big : 4096u);
            k_lookup_raster_big<<<grid, kBlock, 0, stream>>>(d_rec.p, d_big.p, n_big, G, d_lookup.p);
        }
        k_lookup_finish<<<grid_for(ncell), kBlock, 0, stream>>>(ncell, d_lookup.p);
        hip_check(hipGetLastError(), "mesh build kernels");
        int err = 0;
        hip_check(hipMemcpyAsync(&err, d_err.p, sizeof(int), hipMemcpyDeviceToHost, stream), "copy err");
        hip_check(hipStreamSynchronize(stream), "mesh build");
        if (err & ERR_INDEX) fail(CNNSNS_EMESH, "build_mesh: node index out of range");
        if (err & ERR_AREA) fail(CNNSNS_EMESH, "build_mesh: a triangle of zero or non-finite area");
        if (err & ERR_EDGE3) fail(CNNSNS_EMESH, "build_mesh: an edge is shared by more than two triangles");
        if (err & ERR_OVERLAP) fail(CNNSNS_EMESH, "build_mesh: two triangles overlap across an edge");
    }

    auto* m = new cnnsns_mesh_s();
    m->device = dev;
    m->n_nodes = n_nodes;
    m->n_tri = n_tri;
    m->G = G;
    m->mean_diam = sum / (double)n_tri;
    m->rec = d_rec.release();
    m->tri = d_tri.release();
    m->lookup = d_lookup.release();
    m->device_bytes = (int64_t)(sizeof(ElemRec) * (size_t)n_tri + sizeof(int32_t) * 3 * (size_t)n_tri +
                                sizeof(int32_t) * (size_t)G * (size_t)G);
    return m;
}

void destroy_mesh(cnnsns_mesh m)
{
    if (!m) return;
    if (m->pending_jobs.load() > 0)
        fail(CNNSNS_EBUSY, "destroy_mesh: serving jobs on this mesh are not complete");
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(m->rec);
    (void)hipFree(m->tri);
    (void)hipFree(m->lookup);
    workspace_release(m->ws);
    workspace_release(m->cls_ws);
    if (m->cls_pool) (void)hipFree(m->cls_pool);
    (void)hipSetDevice(cur);
    delete m;
}

}  // namespace cnnsns
