// Displacement CNN with FP8 e4m3 operands on the matrix cores, all four layers fused.
//
// The network and the tiling are those of the BF16 pass (3x3 convolutions
// 2 -> 32 -> 32 -> 32 -> 2, zero "same" padding, ReLU between layers, one
// 14 x 30 output tile per iteration with the halo recomputed), with the
// operands of every layer in FP8 e4m3 (OCP format: 4 exponent bits, 3
// mantissa bits, largest finite value 448) and FP32 accumulation on
// v_mfma_f32_16x16x32_fp8_fp8, K = 32 per instruction as in the BF16 pass,
// half the bytes per operand.
//
// Scales, all powers of two so that applying them is exact:
//   * weights: one scale per output channel and layer, s_w = 2^ceil(log2(max|w| / 448));
//   * the velocity: s_v from max|u, v| over the grid (a reduction pass before the forward pass);
//   * the activations after layers 1-3: from a bound on their magnitude that follows from the
//     weights alone, |z_o| <= sum_{i,t} |w_oit| * A_in + |b_o| (with A_in the previous layer's
//     bound, and a margin of 1.25 for the rounding of the operands), so no value can overflow
//     the format whatever the input.
// A layer's accumulator starts at b_o / (s_w,o s_in) and is multiplied by s_w,o s_in / s_out
// before ReLU and rounding to e4m3 (round to nearest even) for the next layer; the last layer's
// nine tap products per output channel are summed in FP32 and multiplied by s_w,o s_in.
#include "common.h"

namespace cnnsns {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef long fp8x8;  // eight e4m3 values, the k = 8 (l/16) + j operand slots of lane l

constexpr int kThreads = 512;  // 8 wavefronts, two per SIMD
constexpr int kWaves = kThreads / 64;
constexpr int C = 32;
constexpr int OH = 14, OW = 30;            // output tile
constexpr int H1 = OH + 6, W1 = OW + 6;    // conv1 region (20 x 36)
constexpr int H2 = OH + 4, W2 = OW + 4;    // conv2 region (18 x 34)
constexpr int H3 = OH + 2, W3 = OW + 2;    // conv3 region (16 x 32)
constexpr int HV = OH + 8, WV = OW + 8;    // velocity tile (22 x 38)
constexpr int PXB = 40;                    // bytes per pixel in LDS (32 channels + 8 pad)
constexpr int VEL_PER_THREAD = (HV * WV + kThreads - 1) / kThreads;
constexpr int NMB1 = H1 * W1 / 16, BPW1 = (NMB1 + kWaves - 1) / kWaves, MB1 = BPW1;
constexpr int NMB2 = (H2 * W2 + 15) / 16, BPW2 = (NMB2 + kWaves - 1) / kWaves, MB2 = BPW2;
constexpr int NMB3 = H3 * W3 / 16, BPW3 = NMB3 / kWaves, MB3 = BPW3;
static_assert(H1 * W1 % 16 == 0 && H3 * W3 % 16 == 0 && NMB3 % kWaves == 0, "whole M-blocks");
constexpr int ZC = 532;  // column stride of the conv4 tap products (floats)
static_assert(ZC >= H3 * W3 && ZC % 4 == 0, "Z columns");

// Hidden activations are stored pair-interleaved as in the BF16 pass: byte 2c + h of a pixel
// holds channel c + 16 h, so a lane that owns channels c and c + 16 writes them as one 16-bit word.
__device__ __forceinline__ int chan_at(int pos)
{
    return (pos >> 1) + 16 * (pos & 1);
}

// packed weights (fp8x8 per lane, the layout of the BF16 pass): w1 [nb][lane], w2/w3
// [tap][nb][lane], w4 [nb][lane] with column n = 16 nb + l%16 = 9 o + tap
constexpr int P1 = 2 * 64, P2 = 9 * 2 * 64, P4 = 2 * 64;
constexpr int PACKED = P1 + 2 * P2 + P4;

// Scales and the per-channel epilogue factors, written by k_fp8_prep
struct Fp8Scales {
    unsigned vmax_bits;       // max |u|, |v| over the grid (bit pattern of a non-negative float)
    float s_v;                // velocity scale
    float s_a[3];             // activation scales after layers 1..3
    float s_w[4][C];          // weight scale per layer and output channel (layer 4: channels 0, 1)
    float init[3][C];         // accumulator start b_o / (s_w,o s_in) of layers 1..3
    float fac[3][C];          // s_w,o s_in / s_out of layers 1..3
    float out4[2];            // s_w4,o s_a3
};

__device__ __forceinline__ float pow2_at_least(float x)
{
    // the smallest power of two >= x (x > 0 and finite), else 1
    if (!(x > 0.f) || !(x < 3.0e38f)) return 1.f;
    int e;
    const float m = frexpf(x, &e);  // x = m 2^e, m in [0.5, 1)
    return ldexpf(1.f, m == 0.5f ? e - 1 : e);
}

__device__ __forceinline__ uint32_t to_e4m3_pair(float lo, float hi)
{
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(lo, hi, 0, false) & 0xffffu;
}

__global__ void k_fp8_clear(Fp8Scales* s)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) s->vmax_bits = 0u;
}

// max |u|, |v| over the 2 G^2 velocity values: a block reduces its share through LDS and makes one
// atomic update (one per wavefront on a single word serialises thousands of updates)
constexpr int kMaxThreads = 512;
__global__ __launch_bounds__(kMaxThreads) void k_fp8_absmax(int64_t count, const float* __restrict__ vel, Fp8Scales* s)
{
    __shared__ float s_m[kMaxThreads / 64];
    float m = 0.f;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(vel[k]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kMaxThreads / 64; ++w) m = fmaxf(m, s_m[w]);
        atomicMax(&s->vmax_bits, __float_as_uint(m));
    }
}

// Weight scales, activation scales and the packed e4m3 weights; one block of 1024 threads.  The
// FP32 weights are staged in LDS (78 KiB), each wavefront reduces the max and the sum of |w| of
// its output channels, the first wavefront chains the layer bounds (one lane per channel), and
// all threads pack.
constexpr int NW1 = C * 2 * 9, NW23 = C * C * 9, NW4 = 2 * C * 9;
__global__ __launch_bounds__(1024) void k_fp8_prep(const float* __restrict__ w1, const float* __restrict__ w2,
                                                   const float* __restrict__ w3, const float* __restrict__ w4,
                                                   const float* __restrict__ b1, const float* __restrict__ b2,
                                                   const float* __restrict__ b3, Fp8Scales* s,
                                                   fp8x8* __restrict__ packed)
{
    __shared__ float s_w[NW1 + 2 * NW23 + NW4];
    __shared__ float s_rsum[3][C];   // sum of |w| over inputs and taps per output channel, layers 1..3
    __shared__ float s_scale[4][C];  // weight scale per layer and output channel
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    float* const sw1 = s_w;
    float* const sw2 = sw1 + NW1;
    float* const sw3 = sw2 + NW23;
    float* const sw4 = sw3 + NW23;
    for (int k = tid; k < NW1; k += 1024) sw1[k] = w1[k];
    for (int k = tid; k < NW23; k += 1024) {
        sw2[k] = w2[k];
        sw3[k] = w3[k];
    }
    for (int k = tid; k < NW4; k += 1024) sw4[k] = w4[k];
    __syncthreads();
    // channel c = 0 .. 97: layer c / 32 (layer 4: c = 96, 97), output channel c % 32
    for (int c = wave; c < 3 * C + 2; c += 16) {
        const int l = c < 3 * C ? c / C : 3, o = c < 3 * C ? c % C : c - 3 * C;
        const float* w = l == 0 ? sw1 : (l == 1 ? sw2 : (l == 2 ? sw3 : sw4));
        const int per = (l == 0 ? 2 : C) * 9;
        float mx = 0.f, sm = 0.f;
        for (int k = lane; k < per; k += 64) {
            const float a = fabsf(w[o * per + k]);
            mx = fmaxf(mx, a);
            sm += a;
        }
        for (int off = 32; off > 0; off >>= 1) {
            mx = fmaxf(mx, __shfl_xor(mx, off));
            sm += __shfl_xor(sm, off);
        }
        if (lane == 0) {
            s_scale[l][o] = pow2_at_least(mx / 448.f);
            if (l < 3) s_rsum[l][o] = sm;
        }
    }
    __syncthreads();
    if (wave == 0) {
        const float margin = 1.25f;  // covers the rounding of operands (at most 2^-4 each)
        const int o = lane & (C - 1);
        const float bl[3] = { b1[o], b2[o], b3[o] };
        float A = __uint_as_float(s->vmax_bits);
        float s_in = pow2_at_least(A / 448.f);
        if (lane == 0) s->s_v = s_in;
        for (int l = 0; l < 3; ++l) {
            float P = margin * s_rsum[l][o] * A + fabsf(bl[l]);
            for (int off = 16; off > 0; off >>= 1) P = fmaxf(P, __shfl_xor(P, off));
            const float s_out = pow2_at_least(P / 448.f);
            if (lane < C) {
                const float sc = s_scale[l][o] * s_in;
                s->s_w[l][o] = s_scale[l][o];
                s->init[l][o] = bl[l] / sc;
                s->fac[l][o] = sc / s_out;
            }
            if (lane == 0) s->s_a[l] = s_out;
            A = P;
            s_in = s_out;
        }
        if (lane < 2) {
            s->s_w[3][lane] = s_scale[3][lane];
            s->out4[lane] = s_scale[3][lane] * s_in;
        }
    }
    for (int e = tid; e < PACKED; e += 1024) {
        const int l = e & 63, i = l & 15, q = l >> 4;
        float v[8];
        if (e < P1) {
            const int o = (e >> 6) * 16 + i;
            const float r = 1.f / s_scale[0][o];
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * q + j;
                v[j] = k < 18 ? sw1[(o * 2 + (k & 1)) * 9 + (k >> 1)] * r : 0.f;
            }
        } else if (e < P1 + 2 * P2) {
            const int f = e - P1;
            const int layer = f < P2 ? 1 : 2;
            const float* w = f < P2 ? sw2 : sw3;
            const int g = f % P2, t = g / 128, o = ((g >> 6) & 1) * 16 + i;
            const float r = 1.f / s_scale[layer][o];
            for (int j = 0; j < 8; ++j) v[j] = w[(o * C + chan_at(8 * q + j)) * 9 + t] * r;
        } else {
            const int n = 16 * ((e - P1 - 2 * P2) >> 6) + i;
            const float r = n < 18 ? 1.f / s_scale[3][n / 9] : 0.f;
            for (int j = 0; j < 8; ++j)
                v[j] = n < 18 ? sw4[((n / 9) * C + chan_at(8 * q + j)) * 9 + n % 9] * r : 0.f;
        }
        uint64_t word = 0;
        for (int j = 0; j < 8; j += 2) word |= (uint64_t)to_e4m3_pair(v[j], v[j + 1]) << (8 * j);
        packed[e] = (fp8x8)word;
    }
}

struct TileIter {
    int t, step, end;
    __device__ explicit TileIter(int ntiles)
    {
        const int nx = 8;  // XCDs; workgroups are dispatched to them round-robin
        const int xcd = blockIdx.x % nx, slot = blockIdx.x / nx;
        t = (int)((int64_t)ntiles * xcd / nx) + slot;
        end = (int)((int64_t)ntiles * (xcd + 1) / nx);
        step = gridDim.x / nx;
    }
};

__device__ __forceinline__ bool inside(int gy, int gx, int G)
{
    return gy >= 0 && gy < G && gx >= 0 && gx < G;
}

// Writes the 4 pixels (p0 .. p0 + 3 of an HO x WO region with grid origin (oy0, ox0)) that lane
// (i, q) holds after a layer's M-block: channels i and 16 + i scaled to the next layer's operand
// scale, ReLU, rounded to e4m3; zero for pixels outside the grid (the next layer's zero padding).
template <int WO, bool EDGE>
__device__ __forceinline__ void store_block(uint8_t* __restrict__ out, int p0, int i, const v4f& d0, const v4f& d1,
                                            float f0, float f1, int oy0, int ox0, int G)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        uint32_t v = to_e4m3_pair(fmaxf(d0[r] * f0, 0.f), fmaxf(d1[r] * f1, 0.f));
        if (EDGE) {
            const int p = p0 + r, gy = oy0 + p / WO, gx = ox0 + p % WO;
            if (!inside(gy, gx, G)) v = 0;
        }
        *reinterpret_cast<uint16_t*>(out + (p0 + r) * PXB + 2 * i) = (uint16_t)v;
    }
}

// One 32 -> 32 layer over an HO x WO region reading an (HO+2) x (WO+2) input region, in LDS.
template <int HO, int WO, int BPW, int MB, bool EDGE>
__device__ __forceinline__ void conv32_fp8(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                           const fp8x8* __restrict__ sw, float ilo, float ihi, float flo, float fhi,
                                           int oy0, int ox0, int G, int wave, int lane)
{
    constexpr int WI = WO + 2, N = HO * WO, NMB = (N + 15) / 16;
    const int i = lane & 15, q = lane >> 4;
    int wl = lane;
    asm volatile("" : "+v"(wl));
    int g0 = wave * BPW;
    asm volatile("" : "+s"(g0));
#pragma unroll 1
    for (int g = g0; g < g0 + BPW; g += MB) {
        v4f acc[MB][2];
        int base[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int p = min((g + m) * 16 + i, N - 1);
            base[m] = ((p / WO) * WI + p % WO) * PXB + 8 * q;
            acc[m][0] = v4f{ ilo, ilo, ilo, ilo };
            acc[m][1] = v4f{ ihi, ihi, ihi, ihi };
        }
        constexpr int PF = 2;
        auto tap_off = [](int t) { return ((t / 3) * WI + t % 3) * PXB; };
        fp8x8 a[PF + 1][MB], w[PF + 1][2];
        auto fetch = [&](int t, int slot) {
#pragma unroll
            for (int m = 0; m < MB; ++m) a[slot][m] = *reinterpret_cast<const fp8x8*>(in + base[m] + tap_off(t));
            w[slot][0] = sw[(t * 2) * 64 + wl];
            w[slot][1] = sw[(t * 2 + 1) * 64 + wl];
        };
#pragma unroll
        for (int t = 0; t < PF; ++t) fetch(t, t);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int cur = t % (PF + 1);
            if (t + PF < 9) fetch(t + PF, (t + PF) % (PF + 1));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[cur][m], w[cur][0], acc[m][0], 0, 0, 0);
                acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[cur][m], w[cur][1], acc[m][1], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int m = 0; m < MB; ++m)
            if (NMB == BPW * kWaves || g + m < NMB)
                store_block<WO, EDGE>(out, (g + m) * 16 + 4 * q, i, acc[m][0], acc[m][1], flo, fhi, oy0, ox0, G);
    }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_cnn_fp8(
    int32_t G, int tiles_x, int ntiles, const float* __restrict__ vel, const fp8x8* __restrict__ packed,
    const Fp8Scales* __restrict__ sc, const float* __restrict__ b4, float* __restrict__ disp)
{
    __shared__ __attribute__((aligned(16))) uint8_t bufA[H1 * W1 * PXB];  // conv1 out, then conv3 out
    static_assert(H1 * W1 >= NMB3 * 16, "conv3 output fits in bufA");
    __shared__ __attribute__((aligned(16))) uint8_t bufB[NMB2 * 16 * PXB];  // conv2 out
    __shared__ __attribute__((aligned(16))) float zb[18 * ZC];             // conv4 tap products
    __shared__ uint16_t s_vel[HV * WV];  // (u, v) of each velocity pixel as an e4m3 pair
    __shared__ fp8x8 s_w1[P1];
    __shared__ fp8x8 s_w4[P4];
    __shared__ fp8x8 s_w23[2 * P2];

    const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, q = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t GG = (int64_t)G * G;

    TileIter it(ntiles);
    if (it.t >= it.end) return;

    for (int k = tid; k < P1; k += kThreads) s_w1[k] = packed[k];
    for (int k = tid; k < P4; k += kThreads) s_w4[k] = packed[P1 + 2 * P2 + k];
    for (int k = tid; k < 2 * P2; k += kThreads) s_w23[k] = packed[P1 + k];
    // the lane's two output channels (i, 16 + i): accumulator start and epilogue factor per layer
    const float i1lo = sc->init[0][i], i1hi = sc->init[0][16 + i], f1lo = sc->fac[0][i], f1hi = sc->fac[0][16 + i];
    const float i2lo = sc->init[1][i], i2hi = sc->init[1][16 + i], f2lo = sc->fac[1][i], f2hi = sc->fac[1][16 + i];
    const float i3lo = sc->init[2][i], i3hi = sc->init[2][16 + i], f3lo = sc->fac[2][i], f3hi = sc->fac[2][16 + i];
    const float rv = 1.f / sc->s_v;
    const float o40 = sc->out4[0], o41 = sc->out4[1], b40 = b4[0], b41 = b4[1];

    // conv1 operand: slots j = 2 jj + ci of lane group q hold channel ci of tap 4q + jj
    int l1_off[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int t = 4 * q + jj;
        l1_off[jj] = t < 9 ? (t / 3) * WV + t % 3 : 0;
    }

    float pu[VEL_PER_THREAD], pw[VEL_PER_THREAD];
    bool pin[VEL_PER_THREAD];
    auto fetch_vel = [&](int t) {  // unconditional loads from clamped positions, as in the BF16 pass
        const int y0 = (t / tiles_x) * OH - 4, x0 = (t % tiles_x) * OW - 4;
#pragma unroll
        for (int k = 0; k < VEL_PER_THREAD; ++k) {
            const int e = min(tid + k * kThreads, HV * WV - 1);
            const int gy = y0 + e / WV, gx = x0 + e % WV;
            pin[k] = inside(gy, gx, G);
            const int64_t o = (int64_t)min(max(gy, 0), G - 1) * G + min(max(gx, 0), G - 1);
            pu[k] = vel[o];
            pw[k] = vel[GG + o];
        }
    };
    auto stash_vel = [&]() {
#pragma unroll
        for (int k = 0; k < VEL_PER_THREAD; ++k) {
            const int e = tid + k * kThreads;
            const float u = pin[k] ? pu[k] : 0.f, v = pin[k] ? pw[k] : 0.f;
            if (e < HV * WV) s_vel[e] = (uint16_t)to_e4m3_pair(u * rv, v * rv);
        }
    };
    auto conv1 = [&](int t) {
        const int ty0 = (t / tiles_x) * OH, tx0 = (t % tiles_x) * OW;
        const bool edge = ty0 < 4 || tx0 < 4 || ty0 + OH + 4 > G || tx0 + OW + 4 > G;
        int g1 = wave * BPW1;
        asm volatile("" : "+s"(g1));
#pragma unroll 1
        for (int g = g1; g < g1 + BPW1; g += MB1) {
            fp8x8 a[MB1];
#pragma unroll
            for (int m = 0; m < MB1; ++m) {
                const int p = min((g + m) * 16 + i, H1 * W1 - 1);
                const int pbase = (p / W1) * WV + p % W1;
                uint64_t v = 0;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) v |= (uint64_t)s_vel[pbase + l1_off[jj]] << (16 * jj);
                a[m] = (fp8x8)v;
            }
            const fp8x8 w1lo = s_w1[lane], w1hi = s_w1[64 + lane];
            v4f d[MB1][2];
#pragma unroll
            for (int m = 0; m < MB1; ++m) {
                d[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[m], w1lo, v4f{ i1lo, i1lo, i1lo, i1lo }, 0, 0, 0);
                d[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a[m], w1hi, v4f{ i1hi, i1hi, i1hi, i1hi }, 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < MB1; ++m) {
                if (NMB1 == BPW1 * kWaves || g + m < NMB1) {
                    if (edge)
                        store_block<W1, true>(bufA, (g + m) * 16 + 4 * q, i, d[m][0], d[m][1], f1lo, f1hi, ty0 - 3,
                                              tx0 - 3, G);
                    else
                        store_block<W1, false>(bufA, (g + m) * 16 + 4 * q, i, d[m][0], d[m][1], f1lo, f1hi, 0, 0, G);
                }
            }
        }
    };

    fetch_vel(it.t);
    stash_vel();
    __syncthreads();
    conv1(it.t);
    __syncthreads();

    for (; it.t < it.end; it.t += it.step) {
        const int ty0 = (it.t / tiles_x) * OH, tx0 = (it.t % tiles_x) * OW;
        const bool edge = ty0 < 4 || tx0 < 4 || ty0 + OH + 4 > G || tx0 + OW + 4 > G;
        const int next = it.t + it.step;
        fetch_vel(next < it.end ? next : it.t);  // after the last tile: unused

        if (edge)
            conv32_fp8<H2, W2, BPW2, MB2, true>(bufA, bufB, s_w23, i2lo, i2hi, f2lo, f2hi, ty0 - 2, tx0 - 2, G, wave,
                                                lane);
        else
            conv32_fp8<H2, W2, BPW2, MB2, false>(bufA, bufB, s_w23, i2lo, i2hi, f2lo, f2hi, ty0 - 2, tx0 - 2, G, wave,
                                                 lane);
        __syncthreads();
        stash_vel();
        if (edge)
            conv32_fp8<H3, W3, BPW3, MB3, true>(bufB, bufA, s_w23 + P2, i3lo, i3hi, f3lo, f3hi, ty0 - 1, tx0 - 1, G,
                                                wave, lane);
        else
            conv32_fp8<H3, W3, BPW3, MB3, false>(bufB, bufA, s_w23 + P2, i3lo, i3hi, f3lo, f3hi, ty0 - 1, tx0 - 1, G,
                                                 wave, lane);
        __syncthreads();

        // conv4: Z[9 o + t][p] = sum_c act3[p][c] w4q[o][c][t] for every pixel of the conv3 region,
        // then each output pixel sums its 9 taps and applies the scale s_w4,o s_a3
        for (int mb = wave; mb < NMB3; mb += kWaves) {
            const fp8x8 a = *reinterpret_cast<const fp8x8*>(bufA + (mb * 16 + i) * PXB + 8 * q);
            const v4f z0 = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, s_w4[lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0, 0, 0);
            const v4f z1 =
                __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, s_w4[64 + lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0, 0, 0);
            *reinterpret_cast<v4f*>(zb + i * ZC + mb * 16 + 4 * q) = z0;
            if (i < 2) *reinterpret_cast<v4f*>(zb + (16 + i) * ZC + mb * 16 + 4 * q) = z1;
        }
        __syncthreads();
        for (int e = tid; e < OH * OW; e += kThreads) {
            const int oy = e / OW, ox = e - oy * OW;
            const float* zp = zb + oy * W3 + ox;
            float s0 = 0.f, s1 = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                s0 += zp[t * ZC + (t / 3) * W3 + t % 3];
                s1 += zp[(9 + t) * ZC + (t / 3) * W3 + t % 3];
            }
            const int gy = ty0 + oy, gx = tx0 + ox;
            if (gy < G && gx < G) {
                disp[(int64_t)gy * G + gx] = b40 + o40 * s0;
                disp[GG + (int64_t)gy * G + gx] = b41 + o41 * s1;
            }
        }
        // the next tile's conv1: bufA was last read before the barrier above, the tap sums read zb
        if (next < it.end) conv1(next);
        __syncthreads();
    }
}

inline unsigned cdiv(int64_t a, int64_t b)
{
    return (unsigned)((a + b - 1) / b);
}

}  // namespace

size_t cnn_fp8_workspace_bytes()
{
    return sizeof(fp8x8) * (size_t)PACKED + ((sizeof(Fp8Scales) + 255) / 256) * 256;
}

void cnn_fp8_forward(int32_t G, const float* vel, const cnnsns_cnn& w, float* disp, void* ws, unsigned grid,
                     hipStream_t stream)
{
    fp8x8* packed = static_cast<fp8x8*>(ws);
    Fp8Scales* sc = reinterpret_cast<Fp8Scales*>(static_cast<char*>(ws) + sizeof(fp8x8) * (size_t)PACKED);
    const int64_t count = 2 * (int64_t)G * G;
    k_fp8_clear<<<1, 64, 0, stream>>>(sc);
    const unsigned rb = (unsigned)std::min<int64_t>(512, std::max<int64_t>(1, (count + kMaxThreads - 1) / kMaxThreads));
    k_fp8_absmax<<<rb, kMaxThreads, 0, stream>>>(count, vel, sc);
    k_fp8_prep<<<1, 1024, 0, stream>>>(w.w[0], w.w[1], w.w[2], w.w[3], w.b[0], w.b[1], w.b[2], sc, packed);
    const int tx = (int)cdiv(G, OW), nt = tx * (int)cdiv(G, OH);
    unsigned g = grid < (unsigned)nt ? grid : (unsigned)nt;
    g = (g + 7) / 8 * 8;
    k_cnn_fp8<<<g, kThreads, 0, stream>>>(G, tx, nt, vel, packed, sc, w.b[3], disp);
    hip_check(hipGetLastError(), "fp8 cnn launch");
}

}  // namespace cnnsns
