// The successive neighbour search (Alg. 1) for a batch of points, with the
// CNN-SNS start element of Alg. 2 selected in the same kernel.
//
// One lane walks one point.  A wavefront owns a contiguous chunk of points
// and keeps all 64 lanes busy: whenever lanes finish their walks, the wave
// hands them the chunk's next unstarted points (ballot + lane prefix count),
// so a long walk does not leave the rest of its wave idle.  Each hop is one
// 64-byte gather of the current element's record; the geometry is FP64 with
// no fused multiply-add, exactly as written.
#pragma clang fp contract(off)

#include "common.h"

namespace cnnsns {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int64_t kChunk = 512;  // points per wavefront

__device__ __forceinline__ int32_t cell_of(double x, int32_t G)
{
    double f = floor(x * (double)G);
    if (!(f >= 0.0)) return 0;  // negative or NaN
    if (f > (double)(G - 1)) return G - 1;
    return (int32_t)f;
}

__device__ __forceinline__ double clamp01(double v)
{
    return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

template <int MODE>
__device__ __forceinline__ int32_t start_of(int64_t i, double px, double py, const int32_t* __restrict__ start,
                                            const double2* __restrict__ origin, const float* __restrict__ disp,
                                            const int32_t* __restrict__ lookup, int32_t G)
{
    if (MODE == START_GIVEN) return start[i];
    if (MODE == START_ASG) {
        int32_t k = lookup[(int64_t)cell_of(py, G) * G + cell_of(px, G)];
        return k < 0 ? 0 : k;
    }
    // CNN-SNS: predicted departure point from the displacement of the origin's cell
    const double2 o = origin[i];
    const int64_t c = (int64_t)cell_of(o.y, G) * G + cell_of(o.x, G);
    const double hx = clamp01(o.x + (double)disp[c]);
    const double hy = clamp01(o.y + (double)disp[(int64_t)G * G + c]);
    int32_t k = lookup[(int64_t)cell_of(hy, G) * G + cell_of(hx, G)];
    if (k < 0) k = start ? start[i] : 0;
    return k;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_locate(const ElemRec* __restrict__ rec, int64_t n_tri, int64_t n,
                                                   const double2* __restrict__ xp, const int32_t* __restrict__ start,
                                                   const double2* __restrict__ origin,
                                                   const float* __restrict__ disp,
                                                   const int32_t* __restrict__ lookup, int32_t G, int32_t max_iter,
                                                   int32_t* __restrict__ host, int32_t* __restrict__ iters,
                                                   uint8_t* __restrict__ status)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    int64_t next = wave * kChunk;           // wave-uniform: next unstarted point of the chunk
    const int64_t end = next + kChunk < n ? next + kChunk : n;
    if (next >= end) return;

    bool active = false;
    int64_t idx = 0;
    double px = 0.0, py = 0.0;
    int32_t K = 0, I = 0;

    for (;;) {
        // hand unstarted points of the chunk to idle lanes
        const uint64_t idle = __ballot(!active);
        if (idle != 0 && next < end) {
            const uint32_t lo = (uint32_t)idle, hi = (uint32_t)(idle >> 32);
            const int rank = (int)__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            if (!active && next + rank < end) {
                idx = next + rank;
                const double2 p = xp[idx];
                px = p.x;
                py = p.y;
                K = start_of<MODE>(idx, px, py, start, origin, disp, lookup, G);
                I = 0;
                if (K < 0 || K >= n_tri) {
                    host[idx] = -1;
                    if (iters) iters[idx] = 0;
                    if (status) status[idx] = CNNSNS_BADSTART;
                } else {
                    active = true;
                }
            }
            next += __popcll(idle);
        }
        if (__ballot(active) == 0) {
            if (next >= end) break;
            continue;
        }
        if (active) {
            I = I + 1;
            const double2* r2 = reinterpret_cast<const double2*>(rec + K);
            const double2 A = r2[0], B = r2[1], C = r2[2];
            const int4 nb = reinterpret_cast<const int4*>(rec + K)[3];
            // barycentric numerators s_j = |S_j| (Sec. 2.2), vertex j's column replaced by x_p
            const double adx = A.x - px, ady = A.y - py;
            const double bdx = B.x - px, bdy = B.y - py;
            const double cdx = C.x - px, cdy = C.y - py;
            const double s0 = bdx * cdy - bdy * cdx;
            const double s1 = cdx * ady - cdy * adx;
            const double s2 = adx * bdy - ady * bdx;
            int fin = -1;
            if (s0 >= 0.0 && s1 >= 0.0 && s2 >= 0.0) {
                fin = CNNSNS_FOUND;  // closed containment: all coordinates >= 0
            } else {
                // eq. (5): smallest coordinate, ties to the lowest index
                int32_t m = nb.x;
                double smin = s0;
                if (s1 < smin) { smin = s1; m = nb.y; }
                if (s2 < smin) { m = nb.z; }
                if (m == -1) {
                    fin = CNNSNS_OUTSIDE;
                } else {
                    K = m;
                    if (I >= max_iter) fin = CNNSNS_MAXITER;
                }
            }
            if (fin >= 0) {
                host[idx] = K;
                if (iters) iters[idx] = I;
                if (status) status[idx] = (uint8_t)fin;
                active = false;
            }
        }
    }
}

}  // namespace

void launch_locate(const cnnsns_mesh_s& m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                   const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status,
                   hipStream_t stream)
{
    if (n == 0) return;
    if (max_iter <= 0) max_iter = 1 << 20;
    const int64_t waves = (n + kChunk - 1) / kChunk;
    const int64_t blocks = (waves * kWave + kBlock - 1) / kBlock;
    if (blocks > (int64_t)INT32_MAX) fail(CNNSNS_EINVAL, "locate: too many points");
    const auto* xp2 = reinterpret_cast<const double2*>(xp);
    const auto* or2 = reinterpret_cast<const double2*>(origin);
    if (disp) {
        k_locate<START_CNN><<<(unsigned)blocks, kBlock, 0, stream>>>(m.rec, m.n_tri, n, xp2, start, or2, disp, m.lookup,
                                                                     m.G, max_iter, host, iters, status);
    } else if (start) {
        k_locate<START_GIVEN><<<(unsigned)blocks, kBlock, 0, stream>>>(m.rec, m.n_tri, n, xp2, start, or2, disp,
                                                                       m.lookup, m.G, max_iter, host, iters, status);
    } else {
        k_locate<START_ASG><<<(unsigned)blocks, kBlock, 0, stream>>>(m.rec, m.n_tri, n, xp2, start, or2, disp,
                                                                     m.lookup, m.G, max_iter, host, iters, status);
    }
    hip_check(hipGetLastError(), "locate launch");
}

}  // namespace cnnsns
