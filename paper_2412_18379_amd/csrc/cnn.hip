// Displacement CNN over the G x G overlay grid: four 3x3 convolution layers
// 2 -> 32 -> 32 -> 32 -> 2 with zero "same" padding, bias, and ReLU between
// layers (the CNN of Sec. 2.3, here a per-cell displacement regressor fed
// with the overlay velocity).  Cross-correlation with OIHW weights:
//   y[o][r][c] = b[o] + sum_i sum_{dy,dx} w[o][i][dy+1][dx+1] x[i][r+dy][c+dx].
//
// Two fused FP32 kernels per forward pass, both persistent (one block per
// compute unit) looping over tiles:
//   conv12: 8 wavefronts, two per SIMD, each owning one row of conv2's 2 x 2
//           output blocks (under 256 registers each): conv1 (K = 18 padded
//           to 20) on the matrix cores into LDS on the 16 x 32 tile plus a
//           one-pixel border, then conv2, stored from registers as the
//           32-channel activation, pixel-major ([G][G][32]).
//   conv34: 8 wavefronts, two per SIMD, each owning one 16-channel block of
//           conv3's output for two rows of 2 x 2 blocks: conv3 on a 16 x 32
//           region (a 14 x 30 output tile plus a one-pixel border; tiles
//           walk down column strips, and a tile that continues a strip
//           reuses the two region rows above it and writes 16 x 30); its
//           results feed conv4 (N = 2) in registers: per region pixel, the
//           block's partial sums of its 18 (output channel, tap)
//           contributions on the matrix cores, kept in LDS, then a 9-term sum
//           of both blocks' partials per output pixel; writes the 2-channel
//           displacement.
// The two 32 -> 32 layers use the Winograd minimal filtering algorithm
// F(2x2, 3x3) (Lavin and Gray, 2016): per 2 x 2 output block and channel
// pair, 16 products in a transformed domain replace 36 direct ones, so the
// layer becomes 16 independent 32 x 32 channel contractions, run in FP32 on
// the matrix cores (v_mfma_f32_16x16x4f32).  Transforms are exact-coefficient
// FP32 additions; the transformed weights are computed once per call in FP64
// and rounded to FP32.  LDS tiles are pixel-major with a 36-float pixel
// stride, so a lane fetches 4 channels of one pixel with one 16-byte read.
// The next tile's input is fetched into registers while the current tile
// computes.
#include "common.h"
#include "strip.h"

namespace cnnsns {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int RH = 16, RW = 32;          // MFMA region per block
constexpr int IH = RH + 2, IW = RW + 2;  // its input tile (one-pixel border)
constexpr int NIN = IH * IW;             // 612 input pixels
constexpr int NREG = RH * RW;            // 512 region pixels
constexpr int C = 32;                    // hidden channels
constexpr int PS = 36;                   // LDS floats per pixel (32 channels + 4 pad)
constexpr int OH34 = RH - 2, OW34 = RW - 2;  // conv34 output tile (region minus its border)
constexpr int NU = 16 * 2 * 2 * 64 * 4;  // Winograd-domain 32->32 weights (floats)
constexpr int VH = IH + 2, VW = IW + 2;  // velocity tile (two-pixel border) 20 x 36
constexpr int CHUNKS = NIN * C / 4;      // float4 chunks of an input tile
constexpr int L1_MBLOCKS = (NIN + 15) / 16;
constexpr int NIN_PAD = L1_MBLOCKS * 16;     // conv1's 39 M-blocks write whole blocks

static_assert(NU == 16 * C * C, "transformed weights cover the whole layer");
static_assert(NREG * PS <= NIN * PS, "output tile aliases the input tile");
constexpr int kThreads12 = 512;  // conv12: 8 wavefronts, two per SIMD, one row of 2 x 2 blocks each
constexpr int kWaves12 = kThreads12 / 64;
static_assert(kWaves12 * 2 == RH, "one row of 2 x 2 output blocks per wavefront");
constexpr int VEL_PER_THREAD12 = (2 * VH * VW + kThreads12 - 1) / kThreads12;
static_assert(RW == 32, "a row of 2 x 2 output blocks is one 16-row matrix block");

// Winograd F(2x2, 3x3) for one 2 x 2 output block:
//   Y = A^T [ (G g G^T) (.) (B^T d B) ] A
// with d the 4 x 4 input patch, g the 3 x 3 filter, and
//   B^T = [1 0 -1 0; 0 1 1 0; 0 -1 1 0; 0 1 0 -1],
//   G   = [1 0 0; 1/2 1/2 1/2; 1/2 -1/2 1/2; 0 0 1],
//   A^T = [1 1 1 0; 0 1 -1 -1].
// Summed over input channels, the 16 elementwise products of position
// (xi, nu) form a contraction M[xi][nu] = U[xi][nu] V[xi][nu] over channels,
// U = G g G^T per (output, input) channel pair.
//
// Matrix-core operand order (v_mfma_f32_16x16x4f32, D = A B with A the
// weights and B the transformed inputs): A row = output channel, B column =
// one of the 16 output blocks of a block row, k = input channel.  Lane l
// supplies output channel 16 nb + l%16 (A) and block l%16 (B), both for input
// channel 8 (l/16) + 4h + j in k-step j of channel half h, and receives
// output channels 16 nb + 4 (l/16) + r (r = 0..3) of block l%16, four
// consecutive channels of one block.
// u[(((xn * 2 + nb) * 2 + h) * 64 + l) * 4 + j] holds
//   U[xn = 4 xi + nu][output channel 16 nb + l%16][input channel 8 (l/16) + 4h + j],
// so a lane reads the A operands of four k-steps as one float4.
__global__ void k_wino_weights(const float* __restrict__ w, float* __restrict__ u)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NU) return;
    const int j = k & 3, l = (k >> 2) & 63, h = (k >> 8) & 1, nb = (k >> 9) & 1, xn = k >> 10;
    const int xi = xn >> 2, nu = xn & 3;
    const int o = nb * 16 + (l & 15), ci = 8 * (l >> 4) + 4 * h + j;
    const double gm[4][3] = { { 1.0, 0.0, 0.0 }, { 0.5, 0.5, 0.5 }, { 0.5, -0.5, 0.5 }, { 0.0, 0.0, 1.0 } };
    const float* g = w + (o * C + ci) * 9;
    double acc = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) acc += gm[xi][a] * (double)g[a * 3 + b] * gm[nu][b];
    u[k] = (float)acc;
}

// The 4 x 4 input patch of output block (ty, tx) of the region, channels
// 8 g + 4 h .. +3, from the input tile in LDS (region pixel (y, x) is tile
// pixel (y + 1, x + 1), so the patch starts at tile pixel (2 ty, 2 tx)).
__device__ __forceinline__ void wino_patch(const float* __restrict__ s_in, int ty, int tx, int g, int h,
                                           v4f (&d)[4][4])
{
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            d[a][b] = *reinterpret_cast<const v4f*>(s_in + ((2 * ty + a) * IW + 2 * tx + b) * PS + 8 * g + 4 * h);
}

// d <- B^T d B, in place (four channels at once), in four parts: the row
// pass over columns 2 part, 2 part + 1 (parts 0, 1), then the column pass over
// rows 2 (part - 2), 2 (part - 2) + 1 (parts 2, 3).
__device__ __forceinline__ void wino_input_transform_part(v4f (&d)[4][4], int part)
{
    if (part < 2) {
#pragma unroll
        for (int b = 2 * part; b < 2 * part + 2; ++b) {
            const v4f t0 = d[0][b] - d[2][b], t1 = d[1][b] + d[2][b], t2 = d[2][b] - d[1][b], t3 = d[1][b] - d[3][b];
            d[0][b] = t0;
            d[1][b] = t1;
            d[2][b] = t2;
            d[3][b] = t3;
        }
    } else {
#pragma unroll
        for (int a = 2 * (part - 2); a < 2 * (part - 2) + 2; ++a) {
            const v4f t0 = d[a][0] - d[a][2], t1 = d[a][1] + d[a][2], t2 = d[a][2] - d[a][1], t3 = d[a][1] - d[a][3];
            d[a][0] = t0;
            d[a][1] = t1;
            d[a][2] = t2;
            d[a][3] = t3;
        }
    }
}

__device__ __forceinline__ void wino_input_transform(v4f (&d)[4][4])
{
#pragma unroll
    for (int part = 0; part < 4; ++part) wino_input_transform_part(d, part);
}

// Weight operands of four transformed positions (xn = 4 grp .. 4 grp + 3) for
// channel half h: b[x][nb][j] = U[4 grp + x][16 nb + l%16][8 (l/16) + 4h + j].
__device__ __forceinline__ void wino_weights(const v4f* __restrict__ su, int grp, int h, v4f (&b)[4][2])
{
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        b[x][0] = su[(((4 * grp + x) * 2 + 0) * 2 + h) * 64];
        b[x][1] = su[(((4 * grp + x) * 2 + 1) * 2 + h) * 64];
    }
}

// conv 32 -> 32 (no bias) for the single block row ty of the region (region
// rows 2 ty, 2 ty + 1), each of eight wavefronts owning one row, with no
// prefetch across rows (the second wavefront of the SIMD covers the waits), so
// that a wavefront needs under 256 registers.  emit(y) receives y[e][nb][r'],
// e = 2a + b: region pixel (2 ty + a, 2 (l%16) + b), output channel
// 16 nb + 4 (l/16) + r'.
template <class Emit>
__device__ __forceinline__ void conv32_wino_row(const float* __restrict__ s_in, const float* __restrict__ s_u,
                                                int ty, int lane, Emit&& emit)
{
    const int tx = lane & 15, g = lane >> 4;
    const v4f* su = reinterpret_cast<const v4f*>(s_u) + lane;
    v4f acc[16][2];
#pragma unroll
    for (int xn = 0; xn < 16; ++xn) {
        acc[xn][0] = v4f{ 0.f, 0.f, 0.f, 0.f };
        acc[xn][1] = v4f{ 0.f, 0.f, 0.f, 0.f };
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        v4f d[4][4];
        wino_patch(s_in, ty, tx, g, h, d);
        wino_input_transform(d);
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
            v4f bc[4][2];
            wino_weights(su, grp, h, bc);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int xn = 4 * grp + x;
                    const float a = d[xn >> 2][xn & 3][j];
                    acc[xn][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(bc[x][0][j], a, acc[xn][0], 0, 0, 0);
                    acc[xn][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(bc[x][1][j], a, acc[xn][1], 0, 0, 0);
                }
        }
    }
    v4f y[4][2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        v4f m0[4], m1[4];
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            m0[nu] = acc[nu][nb] + acc[4 + nu][nb] + acc[8 + nu][nb];
            m1[nu] = acc[4 + nu][nb] - acc[8 + nu][nb] - acc[12 + nu][nb];
        }
        y[0][nb] = m0[0] + m0[1] + m0[2];
        y[1][nb] = m0[1] - m0[2] - m0[3];
        y[2][nb] = m1[0] + m1[1] + m1[2];
        y[3][nb] = m1[1] - m1[2] - m1[3];
    }
    emit(y);
}

// conv 32 -> 32 (no bias) for block row ty of the region and the 16 output channels of block nb:
// conv32_wino_row's contraction for one output-channel block, so that a wavefront holds 16
// accumulators and two wavefronts per SIMD fit their registers.  emit(y) receives y[e], e = 2a + b:
// region pixel (2 ty + a, 2 (l%16) + b), output channels 16 nb + 4 (l/16) + r.
template <class Emit>
__device__ __forceinline__ void conv32_wino_nb(const float* __restrict__ s_in, const float* __restrict__ s_u, int ty,
                                               int nb, int lane, Emit&& emit)
{
    const int tx = lane & 15, g = lane >> 4;
    const v4f* su = reinterpret_cast<const v4f*>(s_u) + lane;
    v4f acc[16];
#pragma unroll
    for (int xn = 0; xn < 16; ++xn) acc[xn] = v4f{ 0.f, 0.f, 0.f, 0.f };
    // the weights of the next group of four transformed positions are read while this group's
    // matrix instructions issue
    v4f bc[2][4];
    auto wload = [&](int stage, v4f (&b)[4]) {
        const int hh = stage >> 2, gg = stage & 3;
#pragma unroll
        for (int x = 0; x < 4; ++x) b[x] = su[(((4 * gg + x) * 2 + nb) * 2 + hh) * 64];
    };
    wload(0, bc[0]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        v4f d[4][4];
        wino_patch(s_in, ty, tx, g, h, d);
        wino_input_transform(d);
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
            const int stage = 4 * h + grp;
            if (stage + 1 < 8) wload(stage + 1, bc[(stage + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            const v4f(&cur)[4] = bc[stage & 1];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    const int xn = 4 * grp + x;
                    acc[xn] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[x][j], d[xn >> 2][xn & 3][j], acc[xn], 0, 0, 0);
                }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    v4f m0[4], m1[4], y[4];
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
        m0[nu] = acc[nu] + acc[4 + nu] + acc[8 + nu];
        m1[nu] = acc[4 + nu] - acc[8 + nu] - acc[12 + nu];
    }
    y[0] = m0[0] + m0[1] + m0[2];
    y[1] = m0[1] - m0[2] - m0[3];
    y[2] = m1[0] + m1[1] + m1[2];
    y[3] = m1[1] - m1[2] - m1[3];
    emit(y);
}

// x summed over the four lanes l % 16 + 16 k of its 16-lane column: x + (x of lane l ^ 16), then the
// same with lane l ^ 32, through the lane-swap instructions (no trip through the LDS).  With both
// operands x, the swap returns x of lane l in one half and of its partner in the other, so their sum
// is x_l + x_(l ^ 16); the two addends may come in either order, which leaves the sum unchanged.
__device__ __forceinline__ float sum_lane_column(float x)
{
    const auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    const auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}

// Block loads of the transformed 32->32 weights into LDS.
__device__ __forceinline__ void load_u(const float* __restrict__ u, float* __restrict__ s_u)
{
    const v4f* src = reinterpret_cast<const v4f*>(u);
    v4f* dst = reinterpret_cast<v4f*>(s_u);
    for (int k = threadIdx.x; k < NU / 4; k += blockDim.x) dst[k] = src[k];
}

// Persistent tile loop.  Tiles (row-major) are split into 8 contiguous
// ranges, one per XCD: workgroups are dispatched to the 8 XCDs round-robin
// by id, so the blocks of one XCD walk one range together and neighbouring
// tiles, whose halos overlap, are read through the same L2.
struct TileIter {
    int t, step, end;
    __device__ explicit TileIter(int ntiles)
    {
        const int nx = 8;
        const int xcd = blockIdx.x % nx, slot = blockIdx.x / nx, per = gridDim.x / nx;
        t = (int)((int64_t)ntiles * xcd / nx) + slot;
        end = (int)((int64_t)ntiles * (xcd + 1) / nx);
        step = per;
    }
};

// conv1 + ReLU (matrix cores, into LDS) then conv2 + ReLU -> act2 [G][G][32].
__global__ __launch_bounds__(kThreads12) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_conv12_f32(
    int32_t G, int tiles_x, int ntiles, const float* __restrict__ vel, const float* __restrict__ w1,
    const float* __restrict__ b1, const float* __restrict__ u2, const float* __restrict__ b2,
    float* __restrict__ act2)
{
    __shared__ __attribute__((aligned(16))) float s_in[NIN_PAD * PS];
    __shared__ __attribute__((aligned(16))) float s_u[NU];
    __shared__ float s_vel[2 * VH * VW];
    // conv1's weights (OIHW, 18 per output channel) and the biases of conv1 and conv2: read per
    // tile from LDS rather than from global memory, so their latency is an LDS read's
    __shared__ float s_w1[C * 18];
    __shared__ __attribute__((aligned(16))) float s_b12[2][C];

    const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, q = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t GG = (int64_t)G * G;

    TileIter it(ntiles);
    if (it.t >= it.end) return;

    load_u(u2, s_u);
    for (int k = tid; k < C * 18; k += kThreads12) s_w1[k] = w1[k];
    if (tid < 2 * C) s_b12[tid / C][tid % C] = (tid < C ? b1 : b2)[tid % C];
    // conv1's operands and conv2's biases are (re)loaded on every tile, from an index the
    // compiler cannot see through, so that none of them occupies registers during conv2
    auto conv1_setup = [&](float (&bw1)[5][2], v4f (&bias1)[2], int (&l1_off)[5], bool (&l1_on)[5]) {
        int qq = q;
        asm volatile("" : "+v"(qq));
        // A operands (the weights): in k-step s lane (i, q) supplies output channel 16 nb + i at
        // k = 4s + q = 9 ci + tap (zero for k >= 18).  The gathered inputs are the B operands,
        // so a lane receives four consecutive output channels 16 nb + 4q + r of one pixel, and
        // the accumulators start from those channels' biases.
#pragma unroll
        for (int s = 0; s < 5; ++s)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int k = 4 * s + qq, o = nb * 16 + i;
                bw1[s][nb] = k < 18 ? s_w1[o * 18 + k] : 0.f;
            }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) bias1[nb] = *reinterpret_cast<const v4f*>(&s_b12[0][16 * nb + 4 * qq]);
        // B operands: k-step s of lane (i, q) reads s_vel at the pixel's base plus a per-lane
        // constant offset (channel k / 9, tap k % 9); slots k >= 18 read the pixel itself and
        // are zeroed by a select
#pragma unroll
        for (int s = 0; s < 5; ++s) {
            const int k = 4 * s + qq, t = k % 9;
            l1_on[s] = k < 18;
            l1_off[s] = k < 18 ? (k / 9) * VH * VW + (t / 3) * VW + t % 3 : VW + 1;
        }
    };

    // The next tile's velocity is loaded unconditionally, from clamped (valid) positions, and what
    // lies outside the grid is zeroed when it is stashed: with no branch between the loads and their
    // use, the compiled code waits for them only at the stash, not at the start of the tile (where
    // it would also wait for the previous tile's activation stores).
    float pv[VEL_PER_THREAD12];
    bool pin[VEL_PER_THREAD12];
    auto fetch_vel = [&](int t) {
        const int y0 = (t / tiles_x) * RH, x0 = (t % tiles_x) * RW;
#pragma unroll
        for (int k = 0; k < VEL_PER_THREAD12; ++k) {
            // opaque to the compiler, so the positions are not kept in registers across tiles
            int e = tid + k * kThreads12;
            asm volatile("" : "+v"(e));
            const int ec = min(e, 2 * VH * VW - 1);
            const int c = ec / (VH * VW), rem = ec % (VH * VW);
            const int gy = y0 - 2 + rem / VW, gx = x0 - 2 + rem % VW;
            pin[k] = gy >= 0 && gy < G && gx >= 0 && gx < G;
            pv[k] = vel[c * GG + (int64_t)min(max(gy, 0), G - 1) * G + min(max(gx, 0), G - 1)];
        }
    };
    auto stash_vel = [&]() {
#pragma unroll
        for (int k = 0; k < VEL_PER_THREAD12; ++k) {
            // threads past the end write the last element again, the value its owner writes (their
            // loads were clamped to it): every store is unconditional, so no load sinks to it
            const int e = min(tid + k * kThreads12, 2 * VH * VW - 1);
            s_vel[e] = pin[k] ? pv[k] : 0.f;
        }
    };
    // conv1 of tile t from s_vel into s_in
    auto conv1 = [&](int t) {
        const int y0 = (t / tiles_x) * RH, x0 = (t % tiles_x) * RW;
        float bw1[5][2];
        v4f bias1[2];
        int l1_off[5];
        bool l1_on[5];
        conv1_setup(bw1, bias1, l1_off, l1_on);

        // conv1 on the 18 x 34 input tile of conv2; zero outside the grid (conv2's padding).
        // Wave w takes blocks w, w + 4, ....
        auto conv1_gather = [&](int mb, float (&a)[5]) {
            const int p = min(mb * 16 + i, NIN - 1);
            const int py = p / IW, base = py * VW + (p - py * IW);
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                const float v = s_vel[base + l1_off[s]];
                a[s] = l1_on[s] ? v : 0.f;
            }
        };
        // result of a block: lane (i, q) holds channels 16 nb + 4q .. +3 of tile pixel 16 mb + i,
        // written as two 16-byte runs (the last block's pixels past the tile land in the padding
        // of s_in)
        auto conv1_store = [&](int mb, const v4f& d0, const v4f& d1) {
            const int p = mb * 16 + i, oy = p / IW, ox = p - oy * IW;
            const int gy = y0 - 1 + oy, gx = x0 - 1 + ox;
            const bool in = (unsigned)gy < (unsigned)G && (unsigned)gx < (unsigned)G;
            v4f v0, v1;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v0[r] = in ? fmaxf(d0[r], 0.f) : 0.f;
                v1[r] = in ? fmaxf(d1[r], 0.f) : 0.f;
            }
            *reinterpret_cast<v4f*>(s_in + p * PS + 4 * q) = v0;
            *reinterpret_cast<v4f*>(s_in + p * PS + 16 + 4 * q) = v1;
        };
        {
            // all of the wave's blocks at once (w, w + 8, ..., at most 5): every gather issues
            // first, then 10 independent accumulation chains
            constexpr int NB1 = (L1_MBLOCKS + kWaves12 - 1) / kWaves12;
            float a[NB1][5];
#pragma unroll
            for (int u = 0; u < NB1; ++u) conv1_gather(min(wave + u * kWaves12, L1_MBLOCKS - 1), a[u]);
            v4f d[NB1][2];
#pragma unroll
            for (int u = 0; u < NB1; ++u) {
                d[u][0] = bias1[0];
                d[u][1] = bias1[1];
            }
#pragma unroll
            for (int s = 0; s < 5; ++s)
#pragma unroll
                for (int u = 0; u < NB1; ++u) {
                    d[u][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(bw1[s][0], a[u][s], d[u][0], 0, 0, 0);
                    d[u][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(bw1[s][1], a[u][s], d[u][1], 0, 0, 0);
                }
#pragma unroll
            for (int u = 0; u < NB1; ++u)
                if (wave + u * kWaves12 < L1_MBLOCKS) conv1_store(wave + u * kWaves12, d[u][0], d[u][1]);
        }
    };

    fetch_vel(it.t);
    stash_vel();
    __syncthreads();
    conv1(it.t);
    __syncthreads();

    for (; it.t < it.end; it.t += it.step) {
        const int y0 = (it.t / tiles_x) * RH, x0 = (it.t % tiles_x) * RW;
        const int next = it.t + it.step;
        fetch_vel(next < it.end ? next : it.t);  // lands while conv2 runs (after the last tile: unused)
        __builtin_amdgcn_sched_barrier(0);  // the loads stay here (the scheduler would sink them to their use)

        // A tile takes two phases.  First conv2's matrix instructions and output transform on block
        // row ty = wave (reading s_in) and the next tile's velocity into s_vel; then the next tile's
        // conv1 (writing s_in) and this tile's stores, whose address work and issue run while
        // conv1's matrix instructions execute (with the stores first, the pass ran 1.2% slower).
        // The results go straight to act2, not through LDS: each lane stores them (bias, ReLU) as
        // two 16-byte runs of channels per pixel that L2 merges into whole lines.
        v4f yk[4][2];
        conv32_wino_row(s_in, s_u, wave, lane, [&](const v4f (&y)[4][2]) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                yk[e][0] = y[e][0];
                yk[e][1] = y[e][1];
            }
        });
        stash_vel();  // conv1 of this tile is done with s_vel
        __syncthreads();                 // every wave is done reading this tile's s_in
        if (next < it.end) conv1(next);
        {
            const v4f(&y)[4][2] = yk;
            int qq = q;
            asm volatile("" : "+v"(qq));
            v4f bias2[2];  // of the lane's output channels 16 nb + 4q + r
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
                bias2[nb] = *reinterpret_cast<const v4f*>(&s_b12[1][16 * nb + 4 * qq]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int gy = y0 + 2 * wave + (e >> 1), gx = x0 + 2 * i + (e & 1);
                if (gy < G && gx < G) {
                    float* dst = act2 + ((int64_t)gy * G + gx) * C + 4 * q;
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) {
                        v4f v = y[e][nb] + bias2[nb];
#pragma unroll
                        for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r], 0.f);
                        *reinterpret_cast<v4f*>(dst + 16 * nb) = v;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// conv3 + ReLU then conv4 on a 14 x 30 output tile: eight wavefronts, two per SIMD.  Wavefront w takes
// output-channel block nb = w / 4 of conv3 for block rows w % 4 and w % 4 + 4 (two rounds), so each
// holds 16 accumulators; conv4's contraction is split the same way (each block's 16 channels give a
// partial sum) and the two partials are added in the tap sums.
constexpr int kThreads34 = 512;
constexpr int CHUNKS_PER_THREAD34 = (CHUNKS + kThreads34 - 1) / kThreads34;
constexpr int ZS34 = 18;                  // floats per pixel of a partial: the 18 (output, tap) columns
constexpr int ZAREA = NREG / 2 * ZS34;    // one round's 256 pixels, one partial
constexpr int ZOFF1 = 8 * IW * PS;        // round 1's partials: past the input rows 0 .. 7 that hold round 0's
static_assert(2 * ZAREA <= ZOFF1, "round 0's partials fit in the input rows that round 1 does not read");
static_assert(ZOFF1 + 2 * ZAREA <= NIN * PS, "round 1's partials fit after them");
constexpr int OHB = RH;                   // output rows of a tile that continues a strip

// conv34 walks down column strips (strip.h): the first tile of a segment computes conv3 on its 16 x 32
// region and writes OH34 = 14 output rows; every further tile computes conv3 on the 16 rows below the
// previous region only and writes OHB = 16 rows, taking the conv4 products of the two region rows
// above it (the previous region's last two, kept in LDS as the sum of both channel blocks' partials).
using Strip34 = StripIter<OH34, OHB, OW34>;

__global__ __launch_bounds__(kThreads34) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_conv34_f32(
    int32_t G, int tiles_x, int nseg, int seg_rows, const float* __restrict__ act2, const float* __restrict__ u3,
    const float* __restrict__ b3, const float* __restrict__ w4, const float* __restrict__ b4,
    float* __restrict__ disp)
{
    __shared__ __attribute__((aligned(16))) float s_in[NIN * PS];
    __shared__ __attribute__((aligned(16))) float s_u[NU];
    __shared__ __attribute__((aligned(16))) float s_w17[2][C];  // w4[1][c][7], w4[1][c][8]
    // conv4 products (both channel blocks summed) of the last two region rows of the previous tile,
    // double-buffered: a tile reads one and writes the other
    __shared__ float s_zs[2][2][RW][ZS34];

    const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, q = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nb = wave >> 2, wr = wave & 3;
    const int64_t GG = (int64_t)G * G;

    Strip34 it(nseg, tiles_x, seg_rows, G);
    if (!it.valid()) return;

    load_u(u3, s_u);
    // conv3 biases of the lane's output channels 16 nb + 4q + r
    v4f bias3;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias3[r] = b3[16 * nb + 4 * q + r];
    // conv4 A operands (rows n = i = 9 o + tap, the first 16 of the 18 columns): in k-step s, lane
    // (i, q) supplies input channel 16 nb + 4q + s, the channels the Winograd result places in it
    float aw4[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const int n = i, c = 16 * nb + 4 * q + st;
        aw4[st] = w4[((n / 9) * C + c) * 9 + n % 9];
    }
    // the last two columns (n = 16, 17: output channel 1, taps 7 and 8) are vector dot products
    for (int k = tid; k < 2 * C; k += kThreads34) s_w17[k / C][k % C] = w4[(C + k % C) * 9 + 7 + k / C];
    const float bias4[2] = { b4[0], b4[1] };

    // next tile's input, as float4 chunks (8 per pixel) of the 18 x 34 tile
    v4f pa[CHUNKS_PER_THREAD34];
    // the conv3 region of a tile starts one row above its outputs, or (continuing a strip) one below
    auto region_y = [](const Strip34& t) { return t.y() + (t.continues() ? 1 : -1); };
    auto fetch_act = [&](const Strip34& t) {
        const int y0 = region_y(t), x0 = t.x() - 1;  // conv3 region origin
#pragma unroll
        for (int k = 0; k < CHUNKS_PER_THREAD34; ++k) {
            int e = tid + k * kThreads34;
            asm volatile("" : "+v"(e));  // positions recomputed per tile, not held in registers
            const int px = e >> 3, part = e & 7;
            const int gy = y0 - 1 + px / IW, gx = x0 - 1 + px % IW;
            v4f v = v4f{ 0.f, 0.f, 0.f, 0.f };
            if (e < CHUNKS && (unsigned)gy < (unsigned)G && (unsigned)gx < (unsigned)G)
                v = *reinterpret_cast<const v4f*>(act2 + ((int64_t)gy * G + gx) * C + part * 4);
            pa[k] = v;
        }
    };
    auto stash_act = [&]() {
#pragma unroll
        for (int k = 0; k < CHUNKS_PER_THREAD34; ++k) {
            const int e = tid + k * kThreads34;
            if (e < CHUNKS) *reinterpret_cast<v4f*>(s_in + (e >> 3) * PS + (e & 7) * 4) = pa[k];
        }
    };
    fetch_act(it);
    stash_act();
    __syncthreads();

    for (int k = 0; it.valid(); ++k) {
        const int ty0 = it.y(), tx0 = it.x();                 // output tile origin
        const int y0 = region_y(it), x0 = tx0 - 1;            // conv3 region origin
        const bool cont = it.continues();
        Strip34 nx = it;
        nx.advance();
        const bool more = nx.valid();

#pragma unroll 1
        for (int round = 0; round < 2; ++round) {
            // the next tile's input is requested at the start of the second round, so that the
            // address work and the issue of its loads share the round with the matrix instructions
            if (round == 1 && more) fetch_act(nx);
            // each round's results go straight into conv4: for every pixel p of the round,
            // Z_nb[p][n] = sum over block nb's channels c of act3[p][c] w4[n / 9][c][n % 9] (n < 18), stored
            // over input rows that the remaining reads no longer need, after every wave has read them
            conv32_wino_nb(s_in, s_u, wr + 4 * round, nb, lane, [&](const v4f (&y)[4]) {
                __syncthreads();
                v4f act[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int gy = y0 + 2 * (wr + 4 * round) + (e >> 1), gx = x0 + 2 * i + (e & 1);
                    const bool in = (unsigned)gy < (unsigned)G && (unsigned)gx < (unsigned)G;  // conv4's zero padding
                    act[e] = y[e] + bias3;
#pragma unroll
                    for (int r = 0; r < 4; ++r) act[e][r] = in ? fmaxf(act[e][r], 0.f) : 0.f;
                }
                v4f z0[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) z0[e] = v4f{ 0.f, 0.f, 0.f, 0.f };
#pragma unroll
                for (int st = 0; st < 4; ++st)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        z0[e] = __builtin_amdgcn_mfma_f32_16x16x4f32(aw4[st], act[e][st], z0[e], 0, 0, 0);
                float z16[4] = { 0.f, 0.f, 0.f, 0.f }, z17[4] = { 0.f, 0.f, 0.f, 0.f };
                const v4f u = *reinterpret_cast<const v4f*>(&s_w17[0][16 * nb + 4 * q]);
                const v4f v = *reinterpret_cast<const v4f*>(&s_w17[1][16 * nb + 4 * q]);
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        z16[e] += u[r] * act[e][r];
                        z17[e] += v[r] * act[e][r];
                    }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    z16[e] = sum_lane_column(z16[e]);
                    z17[e] = sum_lane_column(z17[e]);
                }
                // lane (i, q) holds the partial Z of its pixels for n = 4q + r, and 16, 17
                float* zbase = s_in + (round ? ZOFF1 : 0) + nb * ZAREA;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = 2 * wr + (e >> 1), col = 2 * i + (e & 1);
                    float* zp = zbase + (row * RW + col) * ZS34;
                    *reinterpret_cast<float2*>(zp + 4 * q) = float2{ z0[e][0], z0[e][1] };
                    *reinterpret_cast<float2*>(zp + 4 * q + 2) = float2{ z0[e][2], z0[e][3] };
                    if (q == 0) *reinterpret_cast<float2*>(zp + 16) = float2{ z16[e], z17[e] };
                }
            });
        }
        __syncthreads();
        // each output pixel sums its 9 taps of both partials: disp[o] = b4[o] + sum_t Z[pixel + tap t][9 o + t].
        // Tap rows are counted from the row above the outputs; continuing a strip, the first two of
        // them are the previous region's last two (kept summed), the rest this region's rows 0, 1, ...
        const int oh = cont ? OHB : OH34, rshift = cont ? 2 : 0;
        const float(*zs_prev)[RW][ZS34] = s_zs[(k & 1) ^ 1];
        for (int e = tid; e < oh * OW34; e += kThreads34) {
            const int oy = e / OW34, ox = e - oy * OW34;
            float d0 = bias4[0], d1 = bias4[1];
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int zr = oy + t / 3, pc = ox + t % 3;
                if (zr < rshift) {
                    d0 += zs_prev[zr][pc][t];
                    d1 += zs_prev[zr][pc][9 + t];
                } else {
                    const int pr = zr - rshift;
                    const float* zp = s_in + (pr < 8 ? 0 : ZOFF1) + ((pr & 7) * RW + pc) * ZS34;
                    d0 += zp[t] + zp[ZAREA + t];
                    d1 += zp[9 + t] + zp[ZAREA + 9 + t];
                }
            }
            const int gy = ty0 + oy, gx = tx0 + ox;
            if (gy < G && gx < G) {
                disp[(int64_t)gy * G + gx] = d0;
                disp[GG + (int64_t)gy * G + gx] = d1;
            }
        }
        // this region's last two rows (14, 15) for the next tile of the strip
        for (int e = tid; e < 2 * RW * ZS34; e += kThreads34) {
            const int rr = e / (RW * ZS34), rem = e - rr * (RW * ZS34), pc = rem / ZS34, n = rem - pc * ZS34;
            const float* zp = s_in + ZOFF1 + ((6 + rr) * RW + pc) * ZS34;
            s_zs[k & 1][rr][pc][n] = zp[n] + zp[ZAREA + n];
        }
        __syncthreads();
        if (more) stash_act();
        __syncthreads();
        it = nx;
    }
}

inline unsigned cdiv(int64_t a, int64_t b)
{
    return (unsigned)((a + b - 1) / b);
}

// One block per compute unit (the LDS footprint allows one), a multiple of the 8 XCDs.
unsigned persistent_grid(int ntiles)
{
    int dev = 0, cus = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CU count");
    int g = cus < ntiles ? cus : ntiles;
    g = (g + 7) / 8 * 8;
    return (unsigned)(g < 8 ? 8 : g);
}

}  // namespace

unsigned cnn_persistent_grid()
{
    return persistent_grid(1 << 30);
}

size_t cnn_workspace_bytes(int32_t G, int32_t precision)
{
    if (precision == CNNSNS_BF16) return cnn_bf16_workspace_bytes();
    if (precision == CNNSNS_FP8E4M3) return cnn_fp8_workspace_bytes();
    return sizeof(float) * (2 * (size_t)NU + (size_t)C * (size_t)G * (size_t)G);
}

void run_cnn(int32_t G, const float* vel, const cnnsns_cnn& w, int32_t precision, float* disp, void* ws,
             hipStream_t stream)
{
    if (precision == CNNSNS_BF16) {
        cnn_bf16_pack(w, ws, stream);
        cnn_bf16_forward(G, vel, ws, w, disp, persistent_grid(1 << 30), stream);
        return;
    }
    if (precision == CNNSNS_FP8E4M3) {
        cnn_fp8_forward(G, vel, w, disp, ws, persistent_grid(1 << 30), stream);
        return;
    }
    if (precision != CNNSNS_F32) fail(CNNSNS_EINVAL, "predict: unknown precision");
    float* u2 = static_cast<float*>(ws);
    float* u3 = u2 + NU;
    float* act2 = u3 + NU;
    k_wino_weights<<<cdiv(NU, 256), 256, 0, stream>>>(w.w[1], u2);
    k_wino_weights<<<cdiv(NU, 256), 256, 0, stream>>>(w.w[2], u3);
    const int tx12 = (int)cdiv(G, RW), n12 = tx12 * (int)cdiv(G, RH);
    const int tx34 = (int)cdiv(G, OW34);
    int n34 = 0;
    const int kb34 = strip_plan(G, OH34, OHB, OW34, persistent_grid(1 << 30), &n34);
    k_conv12_f32<<<persistent_grid(n12), kThreads12, 0, stream>>>(G, tx12, n12, vel, w.w[0], w.b[0], u2, w.b[1], act2);
    k_conv34_f32<<<persistent_grid(n34), kThreads34, 0, stream>>>(G, tx34, n34, OH34 + OHB * kb34, act2, u3,
                                                                 w.b[2], w.w[3], w.b[3], disp);
    hip_check(hipGetLastError(), "predict launch");
}

// Workspace of the forward passes that may not allocate (cnnsns_predict_noalloc): one
// array per GPU, held until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress returns for the current device, never by its name.
constexpr size_t kScratchBytes = ((size_t)32 << 20) + ((size_t)128 << 10);  // the FP32 pass at G = 512
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The calling thread's current device's copy of `scratch`, looked up once per device.
void* scratch_for_current_device()
{
    int dev = 0;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) fail(CNNSNS_EINVAL, "predict_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "predict_noalloc: scratch address");
        if (!p) fail(CNNSNS_EHIP, "predict_noalloc: scratch address is NULL");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

size_t cnn_scratch_bytes()
{
    return kScratchBytes;
}

void run_predict_noalloc(const cnnsns_mesh_s& m, const float* vel, const cnnsns_cnn& w, int32_t precision,
                         float* disp, hipStream_t stream)
{
    if (precision != CNNSNS_F32 && precision != CNNSNS_BF16 && precision != CNNSNS_FP8E4M3)
        fail(CNNSNS_EINVAL, "predict_noalloc: unknown precision");
    const size_t need = cnn_workspace_bytes(m.G, precision);
    if (need > kScratchBytes)
        fail(CNNSNS_EINVAL, "predict_noalloc: this overlay needs a workspace of " + std::to_string(need) +
                                " bytes, more than the " + std::to_string(kScratchBytes) +
                                " bytes of the preallocated one (FP32 takes G <= 512; BF16 and FP8 any G)");
    run_cnn(m.G, vel, w, precision, disp, scratch_for_current_device(), stream);
}

void run_predict(cnnsns_mesh_s& m, const float* vel, const cnnsns_cnn& w, int32_t precision, float* disp,
                 hipStream_t stream)
{
    if (precision != CNNSNS_F32 && precision != CNNSNS_BF16 && precision != CNNSNS_FP8E4M3)
        fail(CNNSNS_EINVAL, "predict: unsupported precision");
    std::lock_guard<std::mutex> lock(m.ws.mu);
    workspace_acquire(m.ws, cnn_workspace_bytes(m.G, precision), stream, "predict");
    run_cnn(m.G, vel, w, precision, disp, m.ws.ptr, stream);
    workspace_used(m.ws, stream);
}

}  // namespace cnnsns
