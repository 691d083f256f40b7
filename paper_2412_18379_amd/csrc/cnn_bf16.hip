// Displacement CNN in BF16 on the matrix cores, all four layers fused.
//
// Same network as the FP32 path (3x3 convolutions 2 -> 32 -> 32 -> 32 -> 2,
// zero "same" padding, ReLU between layers, the CNN of Sec. 2.3 in its
// displacement form), computed with BF16 operands (inputs, weights and the
// activations between layers, rounded to nearest even) and FP32
// accumulation; the output displacement is FP32.
//
// v_mfma_f32_16x16x32_bf16 takes K = 32, one tap of 32 channels per
// instruction, so a layer costs 9 instructions per 16 pixels x 16 output
// channels.  Being 16x cheaper than FP32 on the matrix cores, the whole net
// is fused per 14 x 30 output tile, recomputing the halo (conv1 on 20 x 36,
// conv2 on 18 x 34, conv3 on 16 x 32, conv4 on 14 x 30): a pass reads only
// the 2-channel velocity and writes only the 2-channel displacement, and
// needs no device workspace beyond the packed weights.  conv1 (K = 18) is
// padded to one K = 32 step; conv4 (N = 2) computes, per conv3 pixel, its 18
// (output channel, tap) contributions (two N-blocks of one K = 32
// instruction each) and then sums 9 taps per output pixel.
#include "common.h"

namespace cnnsns {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // 4 wavefronts, one per SIMD
constexpr int kWaves = kThreads / 64;
constexpr int C = 32;
constexpr int OH = 14, OW = 30;            // output tile
constexpr int H1 = OH + 6, W1 = OW + 6;    // conv1 region (20 x 36)
constexpr int H2 = OH + 4, W2 = OW + 4;    // conv2 region (18 x 34)
constexpr int H3 = OH + 2, W3 = OW + 2;    // conv3 region (16 x 32)
constexpr int HV = OH + 8, WV = OW + 8;    // velocity tile (22 x 38)
constexpr int PXS = 40;                    // bf16 per pixel in LDS (32 channels + 8 pad: 80 bytes)
constexpr int VEL_PER_THREAD = (2 * HV * WV + kThreads - 1) / kThreads;

// Hidden activations are stored pair-interleaved: LDS position 2c + h of a
// pixel holds channel c + 16 h, so a lane that owns channels c and c + 16 of
// the matrix-core result writes them with one packed 32-bit store.
__device__ __forceinline__ int chan_at(int pos)
{
    return (pos >> 1) + 16 * (pos & 1);
}

// packed weights, one bf16x8 B operand per lane:
//   w1p[nb][lane]: k = 8 (l/16) + j = 9 ci + tap (< 18, else 0) of output channel 16 nb + l%16
//   w2p/w3p[tap][nb][lane]: input channel chan_at(8 (l/16) + j), output channel 16 nb + l%16
//   w4p[nb][lane]: input channel chan_at(8 (l/16) + j), column n = 16 nb + l%16 = 9 o + tap
//                  (output channel o = n / 9, tap n % 9) for n < 18, else 0
constexpr int P1 = 2 * 64, P2 = 9 * 2 * 64, P4 = 2 * 64;
constexpr int PACKED = P1 + 2 * P2 + P4;  // bf16x8 entries

__global__ void k_pack_bf16(const float* __restrict__ w1, const float* __restrict__ w2, const float* __restrict__ w3,
                            const float* __restrict__ w4, bf16x8* __restrict__ out)
{
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= PACKED) return;
    const int l = e & 63, i = l & 15, q = l >> 4;
    bf16x8 v;
    if (e < P1) {
        const int nb = e >> 6;
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * q + j;
            v[j] = (bf16)(k < 18 ? w1[((nb * 16 + i) * 2 + k / 9) * 9 + k % 9] : 0.f);
        }
    } else if (e < P1 + 2 * P2) {
        const int f = e - P1;
        const float* w = f < P2 ? w2 : w3;
        const int g = f % P2, t = g / 128, nb = (g >> 6) & 1;
        for (int j = 0; j < 8; ++j) v[j] = (bf16)w[((nb * 16 + i) * C + chan_at(8 * q + j)) * 9 + t];
    } else {
        const int n = 16 * ((e - P1 - 2 * P2) >> 6) + i;
        for (int j = 0; j < 8; ++j) v[j] = (bf16)(n < 18 ? w4[((n / 9) * C + chan_at(8 * q + j)) * 9 + n % 9] : 0.f);
    }
    out[e] = v;
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

// Packed store of channels (i, 16 + i) of one pixel: bias, ReLU, and zero when
// the pixel lies outside the grid (the next layer's zero padding).
template <bool EDGE>
__device__ __forceinline__ void store_pair(bf16* __restrict__ out, int pp, int i, float v0, float v1,
                                           const float* __restrict__ bias, int gy, int gx, int G)
{
    float a = fmaxf(v0 + bias[i], 0.f), b = fmaxf(v1 + bias[16 + i], 0.f);
    if (EDGE && !inside(gy, gx, G)) a = b = 0.f;
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 pk;
    pk[0] = (bf16)a;
    pk[1] = (bf16)b;
    *reinterpret_cast<bf16x2*>(out + pp * PXS + 2 * i) = pk;
}

// One 32 -> 32 layer over an HO x WO region (output origin (oy0, ox0) in the
// grid) reading an (HO+2) x (WO+2) input region, all in LDS, pixel-major.
// Wavefront w takes the contiguous M-blocks [w NMB / 4, (w+1) NMB / 4) and
// works through them four at a time; the A operands of tap t+1 are read
// while the matrix instructions of tap t issue.
template <int HO, int WO, bool EDGE>
__device__ __forceinline__ void conv32_bf16(const bf16* __restrict__ in, bf16* __restrict__ out,
                                            const bf16x8 (&w)[9][2], const float* __restrict__ bias, int oy0,
                                            int ox0, int G, int wave, int lane)
{
    constexpr int WI = WO + 2, N = HO * WO, NMB = (N + 15) / 16;
    const int i = lane & 15, q = lane >> 4;
    const int lo = wave * NMB / kWaves, hi = (wave + 1) * NMB / kWaves;
    for (int g = lo; g < hi; g += 4) {
        v4f acc[4][2];
        int base[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int p = min((g + m) * 16 + i, N - 1);
            base[m] = ((p / WO) * WI + p % WO) * PXS + 8 * q;
            acc[m][0] = v4f{ 0.f, 0.f, 0.f, 0.f };
            acc[m][1] = acc[m][0];
        }
        bf16x8 a[2][4];
#pragma unroll
        for (int m = 0; m < 4; ++m) a[0][m] = *reinterpret_cast<const bf16x8*>(in + base[m]);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int cur = t & 1;
            if (t + 1 < 9) {
                const int off = (((t + 1) / 3) * WI + (t + 1) % 3) * PXS;
#pragma unroll
                for (int m = 0; m < 4; ++m) a[cur ^ 1][m] = *reinterpret_cast<const bf16x8*>(in + base[m] + off);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cur][m], w[t][0], acc[m][0], 0, 0, 0);
                acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cur][m], w[t][1], acc[m][1], 0, 0, 0);
            }
        }
        // result: lane (i, q) holds region pixels (g + m) 16 + 4q + r, channels i and 16 + i
        const int p0 = g * 16 + 4 * q;
        int oy = p0 / WO, ox = p0 % WO;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            if (g + m < hi) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    store_pair<EDGE>(out, p0 + m * 16 + r, i, acc[m][0][r], acc[m][1][r], bias, oy0 + oy, ox0 + ox,
                                     G);
                    if (EDGE) {
                        if (++ox == WO) { ox = 0; ++oy; }
                    }
                }
                if (EDGE) {
                    ox += 12;
                    if (ox >= WO) { ox -= WO; ++oy; }
                }
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_cnn_bf16(
    int32_t G, int tiles_x, int ntiles, const float* __restrict__ vel, const bf16x8* __restrict__ packed,
    const float* __restrict__ b1, const float* __restrict__ b2, const float* __restrict__ b3,
    const float* __restrict__ b4, float* __restrict__ disp)
{
    __shared__ __attribute__((aligned(16))) bf16 bufA[H1 * W1 * PXS];  // conv1 out, then conv3 out
    static_assert(H1 * W1 >= (H3 * W3 + 63) / 64 * 64, "conv3 output fits in bufA");
    // conv2 out, padded to whole groups of four M-blocks (conv32_bf16 stores them unguarded)
    __shared__ __attribute__((aligned(16))) bf16 bufB[(H2 * W2 + 63) / 64 * 64 * PXS];
    __shared__ float s_vel[2 * HV * WV];
    __shared__ bf16x8 s_w1[P1];
    __shared__ bf16x8 s_w4[P4];
    __shared__ float s_b[3 * C + 2];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, i = lane & 15, q = lane >> 4;
    const int64_t GG = (int64_t)G * G;

    TileIter it(ntiles);
    if (it.t >= it.end) return;

    for (int k = tid; k < P1; k += kThreads) s_w1[k] = packed[k];
    for (int k = tid; k < P4; k += kThreads) s_w4[k] = packed[P1 + 2 * P2 + k];
    for (int k = tid; k < C; k += kThreads) {
        s_b[k] = b1[k];
        s_b[C + k] = b2[k];
        s_b[2 * C + k] = b3[k];
    }
    if (tid < 2) s_b[3 * C + tid] = b4[tid];
    bf16x8 w2[9][2], w3[9][2];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            w2[t][nb] = packed[P1 + (t * 2 + nb) * 64 + lane];
            w3[t][nb] = packed[P1 + P2 + (t * 2 + nb) * 64 + lane];
        }

    // conv1 gather: slot j of lane group q is k = 8q + j = 9 ci + tap, read at this offset from the
    // pixel's top-left velocity sample; k >= 18 is a zero slot
    // (zero slots read offset 0 and are scaled by 0: no branches around the loads)
    int l1_off[8];
    float l1_on[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 8 * q + j, ci = k / 9, t = k % 9;
        l1_off[j] = k < 18 ? (ci * HV + t / 3) * WV + t % 3 : 0;
        l1_on[j] = k < 18 ? 1.f : 0.f;
    }

    float pv[VEL_PER_THREAD];
    auto fetch_vel = [&](int t) {
        const int y0 = (t / tiles_x) * OH - 4, x0 = (t % tiles_x) * OW - 4;
#pragma unroll
        for (int k = 0; k < VEL_PER_THREAD; ++k) {
            const int e = tid + k * kThreads;
            float v = 0.f;
            if (e < 2 * HV * WV) {
                const int c = e / (HV * WV), rem = e % (HV * WV);
                const int gy = y0 + rem / WV, gx = x0 + rem % WV;
                if (inside(gy, gx, G)) v = vel[c * GG + (int64_t)gy * G + gx];
            }
            pv[k] = v;
        }
    };
    auto stash_vel = [&]() {
#pragma unroll
        for (int k = 0; k < VEL_PER_THREAD; ++k) {
            const int e = tid + k * kThreads;
            if (e < 2 * HV * WV) s_vel[e] = pv[k];
        }
    };
    fetch_vel(it.t);
    stash_vel();
    __syncthreads();

    for (; it.t < it.end; it.t += it.step) {
        const int ty0 = (it.t / tiles_x) * OH, tx0 = (it.t % tiles_x) * OW;

        // tiles whose velocity halo lies inside the grid need no zero-padding tests
        const bool edge = ty0 < 4 || tx0 < 4 || ty0 + OH + 4 > G || tx0 + OW + 4 > G;

        // conv1 on the 20 x 36 region: K = 18 (2 channels x 9 taps) padded to 32
        {
            constexpr int N = H1 * W1, NMB = N / 16;
            static_assert(N % 16 == 0, "conv1 region is whole M-blocks");
            const int lo = wave * NMB / kWaves, hi = (wave + 1) * NMB / kWaves;
            for (int g = lo; g < hi; g += 4) {
                // four M-blocks at once: all gathers issue before the first matrix instruction
                bf16x8 a[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int p = min((g + m) * 16 + i, N - 1);
                    const int pbase = (p / W1) * WV + p % W1;
#pragma unroll
                    for (int j = 0; j < 8; ++j) a[m][j] = (bf16)(s_vel[pbase + l1_off[j]] * l1_on[j]);
                }
                v4f d[4][2];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    d[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], s_w1[lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0, 0, 0);
                    d[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], s_w1[64 + lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0,
                                                                      0, 0);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (g + m >= hi) break;
                    const int p0 = (g + m) * 16 + 4 * q;
                    int oy = p0 / W1, ox = p0 % W1;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (edge)
                            store_pair<true>(bufA, p0 + r, i, d[m][0][r], d[m][1][r], s_b, ty0 - 3 + oy, tx0 - 3 + ox, G);
                        else
                            store_pair<false>(bufA, p0 + r, i, d[m][0][r], d[m][1][r], s_b, 0, 0, G);
                        if (++ox == W1) { ox = 0; ++oy; }
                    }
                }
            }
        }
        __syncthreads();

        const int next = it.t + it.step;
        if (next < it.end) fetch_vel(next);  // lands while conv2-conv4 run

        if (edge)
            conv32_bf16<H2, W2, true>(bufA, bufB, w2, s_b + C, ty0 - 2, tx0 - 2, G, wave, lane);
        else
            conv32_bf16<H2, W2, false>(bufA, bufB, w2, s_b + C, ty0 - 2, tx0 - 2, G, wave, lane);
        __syncthreads();
        if (next < it.end) stash_vel();
        if (edge)
            conv32_bf16<H3, W3, true>(bufB, bufA, w3, s_b + 2 * C, ty0 - 1, tx0 - 1, G, wave, lane);
        else
            conv32_bf16<H3, W3, false>(bufB, bufA, w3, s_b + 2 * C, ty0 - 1, tx0 - 1, G, wave, lane);
        __syncthreads();

        // conv4 as a contraction: for every pixel p of the 16 x 32 conv3 region,
        // Z[p][9 o + t] = sum_c act3[p][c] w4[o][c][t] (one K = 32 instruction per 16 pixels and
        // N-block), written in FP32 over the pixel's own 80 bytes: a block's pixels are read
        // only by the wave that computes the block, before its results exist.  Then each output
        // pixel sums its 9 taps.
        {
            constexpr int NMB3 = H3 * W3 / 16, ZS = PXS / 2;  // 32 blocks; floats per pixel
            static_assert(H3 * W3 % 16 == 0, "conv3 region is whole M-blocks");
            float* zf = reinterpret_cast<float*>(bufA);
            for (int mb = wave; mb < NMB3; mb += kWaves) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(bufA + (mb * 16 + i) * PXS + 8 * q);
                const v4f z0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, s_w4[lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0, 0, 0);
                const v4f z1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, s_w4[64 + lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0,
                                                                       0, 0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    float* zp = zf + (mb * 16 + 4 * q + r) * ZS;
                    zp[i] = z0[r];
                    if (i < 2) zp[16 + i] = z1[r];
                }
            }
            __syncthreads();
            for (int e = tid; e < OH * OW; e += kThreads) {
                const int oy = e / OW, ox = e - oy * OW;
                float d0 = s_b[3 * C], d1 = s_b[3 * C + 1];
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    const float* zp = zf + ((oy + t / 3) * W3 + ox + t % 3) * ZS;
                    d0 += zp[t];
                    d1 += zp[9 + t];
                }
                const int gy = ty0 + oy, gx = tx0 + ox;
                if (gy < G && gx < G) {
                    disp[(int64_t)gy * G + gx] = d0;
                    disp[GG + (int64_t)gy * G + gx] = d1;
                }
            }
        }
        __syncthreads();
    }
}

inline unsigned cdiv(int64_t a, int64_t b)
{
    return (unsigned)((a + b - 1) / b);
}

}  // namespace

size_t cnn_bf16_workspace_bytes()
{
    return sizeof(bf16x8) * (size_t)PACKED;
}

void cnn_bf16_pack(const cnnsns_cnn& w, void* packed, hipStream_t stream)
{
    k_pack_bf16<<<cdiv(PACKED, 256), 256, 0, stream>>>(w.w[0], w.w[1], w.w[2], w.w[3],
                                                      static_cast<bf16x8*>(packed));
    hip_check(hipGetLastError(), "bf16 weight packing");
}

void cnn_bf16_forward(int32_t G, const float* vel, const void* packed, const cnnsns_cnn& w, float* disp,
                      unsigned grid, hipStream_t stream)
{
    const int tx = (int)cdiv(G, OW), nt = tx * (int)cdiv(G, OH);
    unsigned g = grid < (unsigned)nt ? grid : (unsigned)nt;
    g = (g + 7) / 8 * 8;
    k_cnn_bf16<<<g, kThreads, 0, stream>>>(G, tx, nt, vel, static_cast<const bf16x8*>(packed), w.b[0], w.b[1],
                                           w.b[2], w.b[3], disp);
    hip_check(hipGetLastError(), "bf16 cnn launch");
}

}  // namespace cnnsns
