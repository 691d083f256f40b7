// The successive neighbour search (Alg. 1) for a batch of points, with the
// CNN-SNS start element of Alg. 2 selected in the same kernel.
//
// One lane walks one point.  With looked-up starts (short walks, a few long
// ones) a wavefront owns 128 points and keeps all 64 lanes busy: whenever
// lanes finish their walks, the wave hands them its next unstarted points
// (ballot + lane prefix count), so a long walk does not leave the rest of its
// wave idle (on 8M points in 16M triangles, 128 points per wavefront walk 7 %
// faster than 512 and 3.5 % faster than 256).  From given starts (long walks
// of similar length for neighbouring points) a wavefront takes 64 points, one
// per lane: 20 % faster than chunks of 512 and 7 % faster than 128, the wider
// grid hiding more of each hop's latency.  Each hop is one 64-byte gather of
// the current element's record; the geometry is FP64 with no fused
// multiply-add, exactly as written.
#pragma clang fp contract(off)

#include "common.h"

namespace cnnsns {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int64_t kChunk = 128;      // points per wavefront, looked-up starts (two per lane at least)
constexpr int64_t kChunkGiven = 64;  // points per wavefront, given starts

__device__ __forceinline__ int32_t cell_of(double x, int32_t G)
{
    // floor(x G) clamped to [0, G-1]; fmax takes 0 for a NaN
    return (int32_t)fmin(fmax(floor(x * (double)G), 0.0), (double)(G - 1));
}

__device__ __forceinline__ double clamp01(double v)
{
    return v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
}

// With INTERP, a finished point also gets the P1 interpolant of a nodal field at x_p in its host
// element (the step after eq. 4 of Sec. 2.1), from the barycentric numerators of the last iteration:
// out = sum_j (s_j / |S_0|) nodal[node j], summed in the element's counter-clockwise node order,
// exactly as cnnsns_interpolate computes it.
template <int MODE, bool INTERP>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_locate(const ElemRec* __restrict__ rec, int64_t n_tri, int64_t n,
                                                   const double2* __restrict__ xp, const int32_t* __restrict__ start,
                                                   const double2* __restrict__ origin,
                                                   const float* __restrict__ disp,
                                                   const int32_t* __restrict__ lookup, int32_t G, int32_t max_iter,
                                                   int32_t* __restrict__ host, int32_t* __restrict__ iters,
                                                   uint8_t* __restrict__ status, const int3* __restrict__ tri,
                                                   const double2* __restrict__ nodal, double2* __restrict__ out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    const int64_t n_waves = (int64_t)gridDim.x * (kBlock / kWave);
    // From the element before movement (long paths, where neighbouring points share elements)
    // a wave owns kChunkGiven slots: slot v is point wave kChunkGiven + v, a contiguous chunk.
    // From a looked-up start (short paths, whose rare long ones cluster at the two ends of the
    // point order, the domain boundary) a wave owns kChunk slots, R = kChunk / 64 runs of 64
    // consecutive points strided across all points, so the long walks of one region spread over
    // many waves: run u is 64-point block b + u n_waves with b = wave for even u and
    // n_waves - 1 - wave for odd u, so both ends of the point order fall to the first waves,
    // which walk them first (runs in the order 0, R - 1, 1, R - 2, ...).
    auto point_of = [&](int64_t v) -> int64_t {
        if (MODE == START_GIVEN) return wave * kChunkGiven + v;
        const int k = (int)(v >> 6);
        const int u = (k & 1) ? (int)(kChunk / 64) - 1 - (k >> 1) : (k >> 1);
        const int64_t b = (u & 1) ? n_waves - 1 - wave : wave;
        return ((b + u * n_waves) << 6) + (v & (kWave - 1));
    };
    int64_t next = 0;  // wave-uniform: next unstarted slot
    const int64_t n_slots =
        MODE == START_GIVEN ? (n - wave * kChunkGiven < kChunkGiven ? n - wave * kChunkGiven : kChunkGiven) : kChunk;
    if (MODE == START_GIVEN && n_slots <= 0) return;

    // Start elements that depend on a lookup (CNN-SNS, ASG) are computed for the whole chunk
    // first, eight independent load chains per lane, and kept in LDS: a lane that takes a new
    // point then waits for one load (x_p) instead of a chain of three.
    __shared__ int32_t s_start[MODE == START_GIVEN ? 1 : kBlock / kWave][MODE == START_GIVEN ? 1 : kChunk];
    int32_t* const my_start = s_start[MODE == START_GIVEN ? 0 : (threadIdx.x / kWave)];
    // Results of the lookup-started modes, whose lanes take new points as they finish, wait in LDS until
    // the wave's chunk is done and are then written run by run, 64 consecutive points at a time (the
    // start slot of a point is reused for its host).  From given starts a lane keeps its one point's
    // results in registers and writes them when the whole wave is done.
    constexpr int kStage = MODE == START_GIVEN ? 1 : kBlock / kWave;
    constexpr int kSlots = MODE == START_GIVEN ? 1 : kChunk;
    __shared__ int32_t s_iters[kStage][kSlots];
    __shared__ uint8_t s_status[kStage][kSlots];
    // with INTERP, the barycentric coordinates of x_p in the host: the interpolant is formed after the
    // loop, for all of the wave's points at once, instead of a chain of dependent gathers per finishing lane
    __shared__ double s_lam[INTERP ? kStage : 1][3][INTERP ? kSlots : 1];
    const int wslot = MODE == START_GIVEN ? 0 : (int)(threadIdx.x / kWave);
    if (MODE != START_GIVEN) {
        // in two halves of four points per lane, staged so that the four chains' loads of each
        // level issue together (eight at once would cost occupancy)
        constexpr int PER_LANE = (int)(kChunk / kWave), H = PER_LANE / 2;
        static_assert(H >= 1 && PER_LANE == 2 * H, "looked-up starts need an even number (>= 2) of points per lane");
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            int64_t pt[H];
            double2 o[H];
            int32_t k0[H];
#pragma unroll
            for (int u = 0; u < H; ++u) {
                const int64_t i = point_of((half * H + u) * kWave + lane);
                pt[u] = i < n ? i : n - 1;  // slots past the last point repeat it
                o[u] = MODE == START_CNN ? origin[pt[u]] : xp[pt[u]];
            }
            if (MODE == START_CNN) {
                float dx[H], dy[H];
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    const int64_t c = (int64_t)cell_of(o[u].y, G) * G + cell_of(o[u].x, G);
                    dx[u] = disp[c];
                    dy[u] = disp[(int64_t)G * G + c];
                }
#pragma unroll
                for (int u = 0; u < H; ++u) {
                    // predicted departure point of the origin's cell (Alg. 2)
                    o[u].x = clamp01(o[u].x + (double)dx[u]);
                    o[u].y = clamp01(o[u].y + (double)dy[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < H; ++u) k0[u] = lookup[(int64_t)cell_of(o[u].y, G) * G + cell_of(o[u].x, G)];
#pragma unroll
            for (int u = 0; u < H; ++u) {
                if (k0[u] < 0) k0[u] = (MODE == START_CNN && start) ? start[pt[u]] : 0;  // uncovered cell
                my_start[(half * H + u) * kWave + lane] = k0[u];
            }
        }
        __builtin_amdgcn_wave_barrier();  // LDS operations of one wavefront complete in order
    }

    bool active = false;
    int64_t idx = 0;
    int64_t slot = 0;  // the lane's current slot (lookup-started modes)
    double px = 0.0, py = 0.0;
    int32_t K = 0, I = 0;
    int fin_given = -1;          // given starts: the lane's outcome, written after the loop
    double lam_given[3] = { 0.0, 0.0, 0.0 };

    for (;;) {
        // hand unstarted points of the chunk to idle lanes
        const uint64_t idle = __ballot(!active);
        if (idle != 0 && next < n_slots) {
            const uint32_t lo = (uint32_t)idle, hi = (uint32_t)(idle >> 32);
            const int rank = (int)__builtin_amdgcn_mbcnt_hi(hi, __builtin_amdgcn_mbcnt_lo(lo, 0u));
            if (!active && next + rank < n_slots) {
                const int64_t v = next + rank;
                idx = point_of(v);
                slot = v;
                if (idx < n) {
                    const double2 p = xp[idx];
                    px = p.x;
                    py = p.y;
                    K = MODE == START_GIVEN ? start[idx] : my_start[v];
                    I = 0;
                    if (K < 0 || K >= n_tri) {  // no element: host -1, path 0 (and a NaN interpolant)
                        if (MODE == START_GIVEN) {
                            fin_given = CNNSNS_BADSTART;
                            K = -1;
                        } else {
                            my_start[v] = -1;
                            s_iters[wslot][v] = 0;
                            s_status[wslot][v] = CNNSNS_BADSTART;
                        }
                    } else {
                        active = true;
                    }
                }
            }
            next += __popcll(idle);
        }
        if (__ballot(active) == 0) {
            if (next >= n_slots) break;
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
            // the neighbour ids arrive with the coordinates (one 64-byte line): keep their load beside
            // the others, not sunk behind the containment test as a second dependent access
            asm volatile("" : : "v"(nb.x), "v"(nb.y), "v"(nb.z));
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
                double lam[3] = { 0.0, 0.0, 0.0 };
                if (INTERP) {  // barycentric coordinates s_j / |S_0| of x_p in the host
                    double2 a = A, b = B, c = C;
                    double t0 = s0, t1 = s1, t2 = s2;
                    if (fin == CNNSNS_MAXITER) {  // the host is the element just moved to
                        const double2* q2 = reinterpret_cast<const double2*>(rec + K);
                        a = q2[0];
                        b = q2[1];
                        c = q2[2];
                        const double ax_ = a.x - px, ay_ = a.y - py, bx_ = b.x - px, by_ = b.y - py;
                        const double cx_ = c.x - px, cy_ = c.y - py;
                        t0 = bx_ * cy_ - by_ * cx_;
                        t1 = cx_ * ay_ - cy_ * ax_;
                        t2 = ax_ * by_ - ay_ * bx_;
                    }
                    const double area2 = (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
                    lam[0] = t0 / area2;
                    lam[1] = t1 / area2;
                    lam[2] = t2 / area2;
                }
                if (MODE == START_GIVEN) {
                    fin_given = fin;
                    if (INTERP)
                        for (int j = 0; j < 3; ++j) lam_given[j] = lam[j];
                } else {
                    my_start[slot] = K;
                    s_iters[wslot][slot] = I;
                    s_status[wslot][slot] = (uint8_t)fin;
                    if (INTERP)
                        for (int j = 0; j < 3; ++j) s_lam[wslot][j][slot] = lam[j];
                }
                active = false;
            }
        }
    }
    // the interpolant at x_p: sum_j lambda_j nodal[node j] over the host's nodes in counter-clockwise
    // order, NaN where there is no host
    auto interpolant = [&](int32_t k, const double (&l)[3]) -> double2 {
        if (k < 0) return double2{ __builtin_nan(""), __builtin_nan("") };
        const int3 v = tri[k];
        const double2 u0 = nodal[v.x], u1 = nodal[v.y], u2 = nodal[v.z];
        return double2{ l[0] * u0.x + l[1] * u1.x + l[2] * u2.x, l[0] * u0.y + l[1] * u1.y + l[2] * u2.y };
    };
    // the wave's results, coalesced
    if (MODE == START_GIVEN) {
        const int64_t i = wave * kChunkGiven + lane;
        if (fin_given >= 0 && i < n) {
            host[i] = K;
            if (iters) iters[i] = fin_given == CNNSNS_BADSTART ? 0 : I;
            if (status) status[i] = (uint8_t)fin_given;
            if (INTERP) out[i] = interpolant(K, lam_given);
        }
    } else {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int r = 0; r < (int)(kChunk / kWave); ++r) {
            const int64_t v = r * kWave + lane, i = point_of(v);
            if (i < n) {
                const int32_t k = my_start[v];
                host[i] = k;
                if (iters) iters[i] = s_iters[wslot][v];
                if (status) status[i] = s_status[wslot][v];
                if (INTERP) {
                    const double l[3] = { s_lam[wslot][0][v], s_lam[wslot][1][v], s_lam[wslot][2][v] };
                    out[i] = interpolant(k, l);
                }
            }
        }
    }
}

// P1 interpolation at x_p in its host element (the approximation that follows
// eq. 4 in Sec. 2.1): the element's nodal basis functions are its barycentric
// coordinates (Sec. 2.2), lambda_j = s_j / |S_0| with s_j the numerators the
// walk uses and |S_0| the doubled area, and the value is sum_j lambda_j u(n_j)
// over the element's nodes, summed in node order.  One thread per point;
// FP64, no fused multiply-add.
__global__ __launch_bounds__(kBlock) void k_interp(const ElemRec* __restrict__ rec, const int3* __restrict__ tri,
                                                   int64_t n_tri, int64_t n, const double2* __restrict__ xp,
                                                   const int32_t* __restrict__ host, const double2* __restrict__ nodal,
                                                   double2* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t K = host[i];
    if (K < 0 || K >= n_tri) {  // no element (a start outside the mesh)
        out[i] = double2{ __builtin_nan(""), __builtin_nan("") };
        return;
    }
    const double2* r2 = reinterpret_cast<const double2*>(rec + K);
    const double2 A = r2[0], B = r2[1], C = r2[2], p = xp[i];
    const double adx = A.x - p.x, ady = A.y - p.y;
    const double bdx = B.x - p.x, bdy = B.y - p.y;
    const double cdx = C.x - p.x, cdy = C.y - p.y;
    const double s0 = bdx * cdy - bdy * cdx;
    const double s1 = cdx * ady - cdy * adx;
    const double s2 = adx * bdy - ady * bdx;
    const double area2 = (B.x - A.x) * (C.y - A.y) - (B.y - A.y) * (C.x - A.x);
    const double l0 = s0 / area2, l1 = s1 / area2, l2 = s2 / area2;
    const int3 v = tri[K];
    const double2 u0 = nodal[v.x], u1 = nodal[v.y], u2 = nodal[v.z];
    out[i] = double2{ l0 * u0.x + l1 * u1.x + l2 * u2.x, l0 * u0.y + l1 * u1.y + l2 * u2.y };
}

}  // namespace

void launch_interp(const cnnsns_mesh_s& m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                   double* out, hipStream_t stream)
{
    if (n == 0) return;
    const int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > (int64_t)INT32_MAX) fail(CNNSNS_EINVAL, "interpolate: too many points");
    k_interp<<<(unsigned)blocks, kBlock, 0, stream>>>(m.rec, reinterpret_cast<const int3*>(m.tri), m.n_tri, n,
                                                       reinterpret_cast<const double2*>(xp), host,
                                                       reinterpret_cast<const double2*>(nodal),
                                                       reinterpret_cast<double2*>(out));
    hip_check(hipGetLastError(), "interpolate launch");
}

template <int MODE, bool INTERP>
static void launch_mode(const cnnsns_mesh_s& m, int64_t n, const double2* xp2, const int32_t* start,
                        const double2* or2, const float* disp, int32_t max_iter, int32_t* host, int32_t* iters,
                        uint8_t* status, const double* nodal, double* out, unsigned blocks, hipStream_t stream)
{
    k_locate<MODE, INTERP><<<blocks, kBlock, 0, stream>>>(m.rec, m.n_tri, n, xp2, start, or2, disp, m.lookup, m.G,
                                                           max_iter, host, iters, status,
                                                           reinterpret_cast<const int3*>(m.tri),
                                                           reinterpret_cast<const double2*>(nodal),
                                                           reinterpret_cast<double2*>(out));
}

void launch_locate(const cnnsns_mesh_s& m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                   const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status,
                   hipStream_t stream, const double* nodal, double* out)
{
    if (n == 0) return;
    if (max_iter <= 0) max_iter = 1 << 20;
    const int64_t chunk = (!disp && start) ? kChunkGiven : kChunk;
    const int64_t waves = (n + chunk - 1) / chunk;
    const int64_t blocks = (waves * kWave + kBlock - 1) / kBlock;
    if (blocks > (int64_t)INT32_MAX) fail(CNNSNS_EINVAL, "locate: too many points");
    const auto* xp2 = reinterpret_cast<const double2*>(xp);
    const auto* or2 = reinterpret_cast<const double2*>(origin);
    const unsigned g = (unsigned)blocks;
    const bool interp = nodal != nullptr;
    if (disp) {
        if (interp)
            launch_mode<START_CNN, true>(m, n, xp2, start, or2, disp, max_iter, host, iters, status, nodal, out, g, stream);
        else
            launch_mode<START_CNN, false>(m, n, xp2, start, or2, disp, max_iter, host, iters, status, nodal, out, g, stream);
    } else if (start) {
        if (interp)
            launch_mode<START_GIVEN, true>(m, n, xp2, start, or2, disp, max_iter, host, iters, status, nodal, out, g, stream);
        else
            launch_mode<START_GIVEN, false>(m, n, xp2, start, or2, disp, max_iter, host, iters, status, nodal, out, g, stream);
    } else {
        if (interp)
            launch_mode<START_ASG, true>(m, n, xp2, start, or2, disp, max_iter, host, iters, status, nodal, out, g, stream);
        else
            launch_mode<START_ASG, false>(m, n, xp2, start, or2, disp, max_iter, host, iters, status, nodal, out, g, stream);
    }
    hip_check(hipGetLastError(), "locate launch");
}

}  // namespace cnnsns
