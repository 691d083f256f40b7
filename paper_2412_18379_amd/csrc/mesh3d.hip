// The SNS walk on tetrahedral meshes: the paper's own setting (Sec. 2.2 with
// four nodes and four neighbours per element; Alg. 1), with the starts of the
// 2D build: the element before movement, or the overlay lookup of the cell
// holding x_p (a G x G x G grid on the unit cube).
//
// Mesh residency is built on the device as in 2D: positive orientation,
// node -> tetrahedron incidence lists, the neighbour across each face, one
// 128-byte record per tetrahedron (one hop is one 128-byte line) and the
// overlay lookup.
//
// Barycentric numerators: s_j = |S_j| is the volume determinant with vertex
// j replaced by x_p.  Moving x_p to the front gives s_j = sigma_j det[F - p]
// with F the other three vertices in order and sigma = (+, -, +, -) for a
// positively oriented vertex order, all signs flipped for a negative one.
// Each face is evaluated with its vertices in node-id order, so the two
// elements that share a face compute the same number for it and their
// numerators are exact negatives (FP64, no fused multiply-add, expressions as
// written).  The record stores the vertices already in node-id order: every
// face's vertices are then in order with fixed register indices, and the
// record keeps the orientation of that order and each vertex's position in the
// positively oriented element order, which breaks ties of eq. (5) by the
// lowest position there.
#pragma clang fp contract(off)

#include <hipcub/hipcub.hpp>

#include <climits>
#include <cmath>

#include "common.h"

namespace cnnsns {
namespace {

constexpr int kBlock = 256;

enum : int { ERR_INDEX = 1, ERR_VOLUME = 2, ERR_FACE3 = 4, ERR_OVERLAP = 8 };

inline unsigned grid_for(int64_t n)
{
    return (unsigned)((n + kBlock - 1) / kBlock);
}

// det[a - p, b - p, c - p] = ax (by cz - bz cy) - ay (bx cz - bz cx) + az (bx cy - by cx)
__device__ __forceinline__ double orient3(const double3& p, const double3& a, const double3& b, const double3& c)
{
    const double ax = a.x - p.x, ay = a.y - p.y, az = a.z - p.z;
    const double bx = b.x - p.x, by = b.y - p.y, bz = b.z - p.z;
    const double cx = c.x - p.x, cy = c.y - p.y, cz = c.z - p.z;
    const double t1 = by * cz - bz * cy, t2 = bx * cz - bz * cx, t3 = bx * cy - by * cx;
    return ax * t1 - ay * t2 + az * t3;
}

// The four numerators of a record's element (vertices in node-id order, orientation o): the
// face opposite vertex k is the other three in order, signed sigma_k o.
__device__ __forceinline__ void numerators(const double3& p, const double3* v, int32_t o, double* s)
{
    const double a = orient3(p, v[1], v[2], v[3]), b = orient3(p, v[0], v[2], v[3]);
    const double c = orient3(p, v[0], v[1], v[3]), d = orient3(p, v[0], v[1], v[2]);
    s[0] = o > 0 ? a : -a;
    s[1] = o > 0 ? -b : b;
    s[2] = o > 0 ? c : -c;
    s[3] = o > 0 ? -d : d;
}

__device__ __forceinline__ double3 d3(const double* q)
{
    return double3{ q[0], q[1], q[2] };
}

// Positive orientation (det[b - a, c - a, d - a] > 0): swap the 3rd and 4th vertex when negative.
__global__ void k3_canonicalise(int64_t n_tet, int64_t n_nodes, const double* __restrict__ xyz,
                                const int32_t* __restrict__ tet_in, int32_t* __restrict__ tet, int* err)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tet) return;
    int32_t q[4];
    for (int k = 0; k < 4; ++k) q[k] = tet_in[4 * t + k];
    for (int k = 0; k < 4; ++k)
        if (q[k] < 0 || q[k] >= n_nodes) {
            atomicOr(err, ERR_INDEX);
            for (int m = 0; m < 4; ++m) tet[4 * t + m] = 0;
            return;
        }
    const double vol = orient3(d3(xyz + 3 * (int64_t)q[0]), d3(xyz + 3 * (int64_t)q[1]), d3(xyz + 3 * (int64_t)q[2]),
                               d3(xyz + 3 * (int64_t)q[3]));
    if (!(vol > 0.0 || vol < 0.0) || !isfinite(vol)) atomicOr(err, ERR_VOLUME);  // zero, NaN or infinite
    tet[4 * t] = q[0];
    tet[4 * t + 1] = q[1];
    tet[4 * t + 2] = vol < 0.0 ? q[3] : q[2];
    tet[4 * t + 3] = vol < 0.0 ? q[2] : q[3];
}

__global__ void k3_degree(int64_t n_tet, const int32_t* __restrict__ tet, unsigned long long* deg)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * n_tet) return;
    atomicAdd(&deg[tet[k]], 1ull);
}

__global__ void k3_fill(int64_t n_tet, const int32_t* __restrict__ tet, unsigned long long* cursor,
                        int32_t* __restrict__ inc)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * n_tet) return;
    const unsigned long long pos = atomicAdd(&cursor[tet[k]], 1ull);
    inc[pos] = (int32_t)(k / 4);
}

// Neighbour across the face opposite vertex j of t: the one other tetrahedron around the face's
// smallest node that holds all three face nodes.  A third holder is an error, and so is a
// neighbour on the same side of the face as t (the two would overlap).
__global__ void k3_neighbours(int64_t n_tet, const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                              const unsigned long long* __restrict__ first, const int32_t* __restrict__ inc,
                              int32_t* __restrict__ nbr, int* err)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * n_tet) return;
    const int64_t t = k / 4;
    const int j = (int)(k - 4 * t);
    int32_t f[3], m = 0;
    for (int a = 0; a < 4; ++a)
        if (a != j) f[m++] = tet[4 * t + a];
    int32_t lo = f[0] < f[1] ? (f[0] < f[2] ? f[0] : f[2]) : (f[1] < f[2] ? f[1] : f[2]);
    int32_t found = -1;
    int bad = 0;
    for (unsigned long long q = first[lo]; q < first[lo + 1]; ++q) {
        const int32_t s = inc[q];
        if (s == t) continue;
        int hits = 0, other = -1;
        for (int a = 0; a < 4; ++a) {
            const int32_t x = tet[4 * (int64_t)s + a];
            if (x == f[0] || x == f[1] || x == f[2]) ++hits;
            else other = x;
        }
        if (hits != 3) continue;
        if (found >= 0) bad |= ERR_FACE3;
        found = s;
        // the neighbour's fourth node must lie on the other side of the face from t's own
        const double3 A = d3(xyz + 3 * (int64_t)f[0]), B = d3(xyz + 3 * (int64_t)f[1]), C = d3(xyz + 3 * (int64_t)f[2]);
        const double own = orient3(d3(xyz + 3 * (int64_t)tet[4 * t + j]), A, B, C);
        const double opp = orient3(d3(xyz + 3 * (int64_t)other), A, B, C);
        if ((own > 0.0 && opp > 0.0) || (own < 0.0 && opp < 0.0)) bad |= ERR_OVERLAP;
    }
    if (bad) atomicOr(err, bad);
    nbr[k] = found;
}

// Record of tetrahedron t: its vertices sorted by node id (five compare-exchanges, the parity
// of the permutation gives the orientation of the sorted order, the element order being
// positive), with the neighbours and positions carried along.
__global__ void k3_pack(int64_t n_tet, const double* __restrict__ xyz, const int32_t* __restrict__ tet,
                        const int32_t* __restrict__ nbr, TetRec* __restrict__ rec, int4* __restrict__ ids)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tet) return;
    int32_t id[4], nb[4], ps[4];
    for (int k = 0; k < 4; ++k) {
        id[k] = tet[4 * t + k];
        nb[k] = nbr[4 * t + k];
        ps[k] = k;
    }
    int32_t o = 1;
    const int net[5][2] = { { 0, 1 }, { 2, 3 }, { 0, 2 }, { 1, 3 }, { 1, 2 } };
    for (int e = 0; e < 5; ++e) {
        const int i = net[e][0], j = net[e][1];
        if (id[i] > id[j]) {
            int32_t x = id[i]; id[i] = id[j]; id[j] = x;
            x = nb[i]; nb[i] = nb[j]; nb[j] = x;
            x = ps[i]; ps[i] = ps[j]; ps[j] = x;
            o = -o;
        }
    }
    TetRec r;
    for (int k = 0; k < 4; ++k) {
        r.v[k][0] = xyz[3 * (int64_t)id[k]];
        r.v[k][1] = xyz[3 * (int64_t)id[k] + 1];
        r.v[k][2] = xyz[3 * (int64_t)id[k] + 2];
        r.nbr[k] = nb[k];
    }
    r.orient = o;
    r.pos = (uint32_t)ps[0] | ((uint32_t)ps[1] << 8) | ((uint32_t)ps[2] << 16) | ((uint32_t)ps[3] << 24);
    r.pad[0] = r.pad[1] = 0;
    rec[t] = r;
    ids[t] = int4{ id[0], id[1], id[2], id[3] };
}

__device__ __forceinline__ void load_tet(const TetRec* __restrict__ rec, int64_t t, double3* v, int32_t* nb,
                                         int32_t& orient, uint32_t& pos)
{
    const double2* q = reinterpret_cast<const double2*>(rec + t);
    const double2 a = q[0], b = q[1], c = q[2], d = q[3], e = q[4], f = q[5];
    v[0] = double3{ a.x, a.y, b.x };
    v[1] = double3{ b.y, c.x, c.y };
    v[2] = double3{ d.x, d.y, e.x };
    v[3] = double3{ e.y, f.x, f.y };
    const int4 n4 = reinterpret_cast<const int4*>(rec + t)[6];
    const int2 m2 = reinterpret_cast<const int2*>(rec + t)[14];
    nb[0] = n4.x; nb[1] = n4.y; nb[2] = n4.z; nb[3] = n4.w;
    orient = m2.x;
    pos = (uint32_t)m2.y;
}

__global__ void k3_fill_i32(int64_t n, int32_t* p, int32_t v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

__global__ void k3_lookup_finish(int64_t n, int32_t* p)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n && p[k] == INT_MAX) p[k] = -1;
}

__device__ __forceinline__ int32_t cell3(double x, int32_t G)
{
    return (int32_t)fmin(fmax(floor(x * (double)G), 0.0), (double)(G - 1));
}

// The overlay cells a tetrahedron's centres can lie in: its bounding box grown by one cell,
// clipped to the grid (lo > hi on an axis when it misses the grid).
__device__ __forceinline__ void tet_box(const double3* v, int32_t G, int32_t (&lo)[3], int32_t (&hi)[3])
{
    const double g = (double)G;
    for (int d = 0; d < 3; ++d) {
        double mn = d == 0 ? v[0].x : (d == 1 ? v[0].y : v[0].z), mx = mn;
        for (int k = 1; k < 4; ++k) {
            const double c = d == 0 ? v[k].x : (d == 1 ? v[k].y : v[k].z);
            mn = fmin(mn, c);
            mx = fmax(mx, c);
        }
        // clamped before conversion (fmax and fmin return the number when the other is NaN)
        const double f0 = fmax(floor(mn * g - 0.5) - 1.0, 0.0), f1 = fmin(ceil(mx * g - 0.5) + 1.0, g - 1.0);
        lo[d] = f0 > g - 1.0 ? G : (int32_t)f0;
        hi[d] = f1 < 0.0 ? -1 : (int32_t)f1;
    }
}

__device__ __forceinline__ bool holds_centre3(const double3* v, int32_t o, int32_t cx, int32_t cy, int32_t cz,
                                              int32_t G)
{
    const double g = (double)G;
    const double3 p{ ((double)cx + 0.5) / g, ((double)cy + 0.5) / g, ((double)cz + 0.5) / g };
    double sn[4];
    numerators(p, v, o, sn);
    return sn[0] >= 0.0 && sn[1] >= 0.0 && sn[2] >= 0.0 && sn[3] >= 0.0;
}

constexpr int64_t kBigBox = 512;  // cells; larger boxes go to the block-parallel pass

// The overlay cells whose centres a tetrahedron contains, one tetrahedron per thread over its
// cell box (the walk's numerators at each centre); the smallest containing id wins.
// Tetrahedra with large boxes (a coarse mesh under a fine overlay) are listed for
// k3_lookup_raster_big instead.
__global__ void k3_lookup_raster(int64_t n_tet, const TetRec* __restrict__ rec, int32_t G, int32_t* lookup,
                                 int32_t* big, unsigned* n_big)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tet) return;
    double3 v[4];
    int32_t nb[4], o;
    uint32_t pos;
    load_tet(rec, t, v, nb, o, pos);
    int32_t lo[3], hi[3];
    tet_box(v, G, lo, hi);
    if (hi[0] < lo[0] || hi[1] < lo[1] || hi[2] < lo[2]) return;
    if ((int64_t)(hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1) > kBigBox) {
        big[atomicAdd(n_big, 1u)] = (int32_t)t;
        return;
    }
    for (int32_t cz = lo[2]; cz <= hi[2]; ++cz)
        for (int32_t cy = lo[1]; cy <= hi[1]; ++cy)
            for (int32_t cx = lo[0]; cx <= hi[0]; ++cx)
                if (holds_centre3(v, o, cx, cy, cz, G))
                    atomicMin(&lookup[((int64_t)cz * G + cy) * G + cx], (int32_t)t);
}

// Listed tetrahedra: blockIdx.y picks the tetrahedron, all blocks along x and their threads
// stride over its cells.
__global__ void k3_lookup_raster_big(const TetRec* __restrict__ rec, const int32_t* __restrict__ big, unsigned n_big,
                                     int32_t G, int32_t* lookup)
{
    for (unsigned k = blockIdx.y; k < n_big; k += gridDim.y) {
        const int32_t t = big[k];
        double3 v[4];
        int32_t nb[4], o;
        uint32_t pos;
        load_tet(rec, t, v, nb, o, pos);
        int32_t lo[3], hi[3];
        tet_box(v, G, lo, hi);
        const int64_t wx = hi[0] - lo[0] + 1, wy = hi[1] - lo[1] + 1, n = wx * wy * (hi[2] - lo[2] + 1);
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
            const int32_t cx = lo[0] + (int32_t)(c % wx), cy = lo[1] + (int32_t)((c / wx) % wy),
                          cz = lo[2] + (int32_t)(c / (wx * wy));
            if (holds_centre3(v, o, cx, cy, cz, G)) atomicMin(&lookup[((int64_t)cz * G + cy) * G + cx], t);
        }
    }
}

__device__ __forceinline__ double clamp01(double v)
{
    return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

enum { S3_GIVEN = 0, S3_LOOKUP = 1, S3_CNN = 2 };

// Alg. 1 for a batch of points, one lane per point.  (The wave-local refill of the 2D walk,
// with 2, 4 or 8 points per lane, measured 8 to 37 % slower on 1M and 8M points in 5.8M
// tetrahedra: neighbouring points walk alike, and the refill costs parallelism.)
// Starts: given (K_m); the overlay lookup of x_p's cell; or CNN-SNS (Alg. 2): the lookup of
// the cell holding x_hat = clamp(x_i + D[cell(x_i)], 0, 1), falling back to the given start
// (else element 0) where that cell holds no element.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k3_locate(const TetRec* __restrict__ rec, int64_t n_tet, int64_t n,
                                                    const double* __restrict__ xp, const int32_t* __restrict__ start,
                                                    const double* __restrict__ origin, const float* __restrict__ disp,
                                                    const int32_t* __restrict__ lookup, int32_t G, int32_t max_iter,
                                                    int32_t* __restrict__ host, int32_t* __restrict__ iters,
                                                    uint8_t* __restrict__ status)
{
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n) return;
    const double3 p{ xp[3 * idx], xp[3 * idx + 1], xp[3 * idx + 2] };
    int32_t K;
    if (MODE == S3_GIVEN) {
        K = start[idx];
    } else {
        double3 q = p;
        if (MODE == S3_CNN) {
            const double3 o{ origin[3 * idx], origin[3 * idx + 1], origin[3 * idx + 2] };
            const int64_t nc = (int64_t)G * G * G;
            const int64_t c = ((int64_t)cell3(o.z, G) * G + cell3(o.y, G)) * G + cell3(o.x, G);
            q = double3{ clamp01(o.x + (double)disp[c]), clamp01(o.y + (double)disp[nc + c]),
                         clamp01(o.z + (double)disp[2 * nc + c]) };
        }
        K = lookup[((int64_t)cell3(q.z, G) * G + cell3(q.y, G)) * G + cell3(q.x, G)];
        if (K < 0) K = (MODE == S3_CNN && start) ? start[idx] : 0;  // a cell with no element
    }
    if (K < 0 || K >= n_tet) {
        host[idx] = -1;
        if (iters) iters[idx] = 0;
        if (status) status[idx] = CNNSNS_BADSTART;
        return;
    }
    int32_t I = 0;
    int fin;
    for (;;) {
        I = I + 1;
        double3 v[4];
        int32_t nb[4], o;
        uint32_t pos;
        load_tet(rec, K, v, nb, o, pos);
        double s[4];
        numerators(p, v, o, s);
        if (s[0] >= 0.0 && s[1] >= 0.0 && s[2] >= 0.0 && s[3] >= 0.0) {
            fin = CNNSNS_FOUND;
            break;
        }
        // eq. (5): the smallest coordinate, ties to the lowest position in the element order
        double sm = s[0];
        uint32_t pm = pos & 0xffu;
        int32_t m = nb[0];
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            const uint32_t pk = (pos >> (8 * k)) & 0xffu;
            if (s[k] < sm || (s[k] == sm && pk < pm)) {
                sm = s[k];
                pm = pk;
                m = nb[k];
            }
        }
        if (m == -1) {
            fin = CNNSNS_OUTSIDE;
            break;
        }
        K = m;
        if (I >= max_iter) {
            fin = CNNSNS_MAXITER;
            break;
        }
    }
    host[idx] = K;
    if (iters) iters[idx] = I;
    if (status) status[idx] = (uint8_t)fin;
}

// P1 interpolation at x_p in its host tetrahedron (Sec. 2.1 after eq. 4): u(x_p) = sum_k
// (s_k / V) u(n_k) over the vertices in ascending node id (the record's order), with s_k the
// walk's numerators and V = det[v1 - v0, v2 - v0, v3 - v0] in that order times its orientation
// (six times the volume, > 0).  A host outside [0, n_tet) gives NaN.
__global__ __launch_bounds__(kBlock) void k3_interp(const TetRec* __restrict__ rec, const int4* __restrict__ ids,
                                                    int64_t n_tet, int64_t n, const double* __restrict__ xp,
                                                    const int32_t* __restrict__ host,
                                                    const double* __restrict__ nodal, double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t K = host[i];
    if (K < 0 || K >= n_tet) {
        out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = __builtin_nan("");
        return;
    }
    const double3 p{ xp[3 * i], xp[3 * i + 1], xp[3 * i + 2] };
    double3 v[4];
    int32_t nb[4], o;
    uint32_t pos;
    load_tet(rec, K, v, nb, o, pos);
    double s[4];
    numerators(p, v, o, s);
    const double d = orient3(v[0], v[1], v[2], v[3]);
    const double V = o > 0 ? d : -d;
    const int4 id = ids[K];
    const int32_t nid[4] = { id.x, id.y, id.z, id.w };
    double f[3] = { 0.0, 0.0, 0.0 };
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double l = s[k] / V;
        const double* u = nodal + 3 * (int64_t)nid[k];
        f[0] = f[0] + l * u[0];
        f[1] = f[1] + l * u[1];
        f[2] = f[2] + l * u[2];
    }
    out[3 * i] = f[0];
    out[3 * i + 1] = f[1];
    out[3 * i + 2] = f[2];
}

template <class T>
struct DevBuf3 {
    T* p = nullptr;
    explicit DevBuf3(size_t count)
    {
        if (count == 0) count = 1;
        if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            fail(CNNSNS_ENOMEM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
        }
    }
    ~DevBuf3() { if (p) (void)hipFree(p); }
    T* release() { T* q = p; p = nullptr; return q; }
    DevBuf3(const DevBuf3&) = delete;
    DevBuf3& operator=(const DevBuf3&) = delete;
};

}  // namespace

cnnsns_mesh3 build_mesh3(const double* xyz, int64_t n_nodes, const int32_t* tet, int64_t n_tet, int32_t G,
                         hipStream_t stream)
{
    if (G == 0) {
        const int e = (int)std::ceil(std::log2(std::cbrt((double)n_tet)));
        G = 1 << (e < 0 ? 0 : (e > 10 ? 10 : e));
    }
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    DevBuf3<double> d_xyz((size_t)(3 * n_nodes));
    DevBuf3<int32_t> d_in((size_t)(4 * n_tet)), d_tet((size_t)(4 * n_tet)), d_nbr((size_t)(4 * n_tet)),
        d_inc((size_t)(4 * n_tet));
    DevBuf3<unsigned long long> d_deg((size_t)n_nodes + 1), d_first((size_t)n_nodes + 1), d_cursor((size_t)n_nodes + 1);
    DevBuf3<int> d_err(1);
    DevBuf3<TetRec> d_rec((size_t)n_tet);
    DevBuf3<int4> d_ids((size_t)n_tet);
    const int64_t ncell = (int64_t)G * G * G;
    DevBuf3<int32_t> d_lookup((size_t)ncell);

    hip_check(hipMemcpyAsync(d_xyz.p, xyz, sizeof(double) * 3 * (size_t)n_nodes, hipMemcpyHostToDevice, stream),
              "copy xyz");
    hip_check(hipMemcpyAsync(d_in.p, tet, sizeof(int32_t) * 4 * (size_t)n_tet, hipMemcpyHostToDevice, stream),
              "copy tet");
    hip_check(hipMemsetAsync(d_err.p, 0, sizeof(int), stream), "memset");
    hip_check(hipMemsetAsync(d_deg.p, 0, sizeof(unsigned long long) * ((size_t)n_nodes + 1), stream), "memset");
    k3_canonicalise<<<grid_for(n_tet), kBlock, 0, stream>>>(n_tet, n_nodes, d_xyz.p, d_in.p, d_tet.p, d_err.p);
    k3_degree<<<grid_for(4 * n_tet), kBlock, 0, stream>>>(n_tet, d_tet.p, d_deg.p);
    size_t tmp_bytes = 0;
    hip_check(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, d_deg.p, d_first.p, (int)(n_nodes + 1), stream),
              "scan size");
    {
        DevBuf3<unsigned char> d_tmp(tmp_bytes);
        hip_check(hipcub::DeviceScan::ExclusiveSum(d_tmp.p, tmp_bytes, d_deg.p, d_first.p, (int)(n_nodes + 1), stream),
                  "scan");
        hip_check(hipMemcpyAsync(d_cursor.p, d_first.p, sizeof(unsigned long long) * ((size_t)n_nodes + 1),
                                 hipMemcpyDeviceToDevice, stream), "copy cursor");
        k3_fill<<<grid_for(4 * n_tet), kBlock, 0, stream>>>(n_tet, d_tet.p, d_cursor.p, d_inc.p);
        k3_neighbours<<<grid_for(4 * n_tet), kBlock, 0, stream>>>(n_tet, d_xyz.p, d_tet.p, d_first.p, d_inc.p,
                                                                  d_nbr.p, d_err.p);
        k3_pack<<<grid_for(n_tet), kBlock, 0, stream>>>(n_tet, d_xyz.p, d_tet.p, d_nbr.p, d_rec.p, d_ids.p);
        k3_fill_i32<<<grid_for(ncell), kBlock, 0, stream>>>(ncell, d_lookup.p, INT_MAX);
        DevBuf3<int32_t> d_big((size_t)n_tet);
        DevBuf3<unsigned> d_nbig(1);
        hip_check(hipMemsetAsync(d_nbig.p, 0, sizeof(unsigned), stream), "memset");
        k3_lookup_raster<<<grid_for(n_tet), kBlock, 0, stream>>>(n_tet, d_rec.p, G, d_lookup.p, d_big.p, d_nbig.p);
        unsigned n_big = 0;
        hip_check(hipMemcpyAsync(&n_big, d_nbig.p, sizeof(unsigned), hipMemcpyDeviceToHost, stream), "copy n_big");
        hip_check(hipStreamSynchronize(stream), "3D lookup raster");
        if (n_big > 0) {
            const dim3 grid(64, n_big < 4096u ? n_big : 4096u);
            k3_lookup_raster_big<<<grid, kBlock, 0, stream>>>(d_rec.p, d_big.p, n_big, G, d_lookup.p);
        }
        k3_lookup_finish<<<grid_for(ncell), kBlock, 0, stream>>>(ncell, d_lookup.p);
        hip_check(hipGetLastError(), "3D mesh build kernels");
        int err = 0;
        hip_check(hipMemcpyAsync(&err, d_err.p, sizeof(int), hipMemcpyDeviceToHost, stream), "copy err");
        hip_check(hipStreamSynchronize(stream), "3D mesh build");
        if (err & ERR_INDEX) fail(CNNSNS_EMESH, "build_mesh3d: node index out of range");
        if (err & ERR_VOLUME) fail(CNNSNS_EMESH, "build_mesh3d: a tetrahedron of zero or non-finite volume");
        if (err & ERR_FACE3) fail(CNNSNS_EMESH, "build_mesh3d: a face is shared by more than two tetrahedra");
        if (err & ERR_OVERLAP) fail(CNNSNS_EMESH, "build_mesh3d: two tetrahedra overlap across a face");
    }
    auto* m = new cnnsns_mesh3_s();
    m->device = dev;
    m->n_nodes = n_nodes;
    m->n_tet = n_tet;
    m->G = G;
    m->rec = d_rec.release();
    m->ids = reinterpret_cast<int32_t*>(d_ids.release());
    m->lookup = d_lookup.release();
    m->device_bytes = (int64_t)((sizeof(TetRec) + sizeof(int4)) * (size_t)n_tet + sizeof(int32_t) * (size_t)ncell);
    return m;
}

void destroy_mesh3(cnnsns_mesh3 m)
{
    if (!m) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(m->rec);
    (void)hipFree(m->ids);
    (void)hipFree(m->lookup);
    workspace_release(m->ws);
    (void)hipSetDevice(cur);
    delete m;
}

void launch_locate3(const cnnsns_mesh3_s& m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                    const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status,
                    hipStream_t stream)
{
    if (n == 0) return;
    if (max_iter <= 0) max_iter = 1 << 20;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > (int64_t)INT32_MAX) fail(CNNSNS_EINVAL, "locate3d: too many points");
    const unsigned g = (unsigned)blocks;
    if (disp)
        k3_locate<S3_CNN><<<g, kBlock, 0, stream>>>(m.rec, m.n_tet, n, xp, start, origin, disp, m.lookup, m.G,
                                                    max_iter, host, iters, status);
    else if (start)
        k3_locate<S3_GIVEN><<<g, kBlock, 0, stream>>>(m.rec, m.n_tet, n, xp, start, origin, disp, m.lookup, m.G,
                                                      max_iter, host, iters, status);
    else
        k3_locate<S3_LOOKUP><<<g, kBlock, 0, stream>>>(m.rec, m.n_tet, n, xp, start, origin, disp, m.lookup, m.G,
                                                       max_iter, host, iters, status);
    hip_check(hipGetLastError(), "locate3d launch");
}

void launch_interp3(const cnnsns_mesh3_s& m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                    double* out, hipStream_t stream)
{
    if (n == 0) return;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > (int64_t)INT32_MAX) fail(CNNSNS_EINVAL, "interpolate3d: too many points");
    k3_interp<<<(unsigned)blocks, kBlock, 0, stream>>>(m.rec, reinterpret_cast<const int4*>(m.ids), m.n_tet, n, xp,
                                                       host, nodal, out);
    hip_check(hipGetLastError(), "interpolate3d launch");
}

}  // namespace cnnsns
