// The displacement CNN in 3D (Sec. 2.3 with 3 x 3 x 3 kernels on a G x G x G
// overlay): 3 -> 32 -> 32 -> 32 -> 3 channels, zero padding of one cell, bias,
// ReLU after layers 1-3, FP32.
//
// Layers 2 and 3 (32 -> 32, 94 % of the work) are dense contractions over
// 27 taps x 32 input channels per output cell and run on the matrix cores
// (v_mfma_f32_16x16x4f32, D = A B): A holds the weights (row = output
// channel, k = input channel), B the input activations (column = one of 16
// consecutive cells along x, k = input channel).  Lane l supplies output
// channel 16 nb + l%16 (A) and cell l%16 (B), both for input channel
// 8 (l/16) + 4h + j in k-step j of channel half h, and receives output
// channels 16 nb + 4 (l/16) + r (r = 0..3) of cell l%16: four consecutive
// channels, stored as one 16-byte write.  A wavefront computes 64 cells of one
// x row (four 16-cell blocks) for all 32 output channels; the 27 taps' weights
// sit in LDS in operand order (108 KiB, loaded once per block), the
// activations come through the caches (a cell's 32 channels are one 128-byte
// line).  Layers 1 and 4 (3 -> 32, 32 -> 3) are 9 % of the work.  Layer 1 runs
// on the vector ALUs, one cell per lane; layer 4 reads its input as the matrix
// layers do and runs on the vector ALUs in FP32 (four lanes per cell, 8 of the
// 32 input channels each) or, in the BF16 pass, on the matrix cores with its
// 3 outputs padded to 16.
//
// Activations between layers: FP32 [G^3][32], cell-major (z, y, x; x fastest),
// 32 channels per cell.  Input velocity and output displacement: FP32
// [3][G][G][G] (component, z, y, x).
#include <mutex>

#include "common.h"

namespace cnnsns {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v8f __attribute__((ext_vector_type(8)));
typedef __bf16 bf16;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int C = 32;             // hidden channels
constexpr int CIO = 3;            // velocity / displacement components
constexpr int TAPS = 27;
constexpr int NWT = TAPS * 4 * 64 * 4;  // operand-ordered weights of one 32 -> 32 layer (floats)
constexpr int NWB = TAPS * 2 * 64;      // the same in BF16 (bf16x8 entries)
constexpr int kBlock = 256;       // vector-ALU layers
constexpr int kWaves32 = 12;      // matrix layers: waves per block (three per SIMD, at most 170 registers)
constexpr int kWaves4 = 16;       // layer 4: waves per block
constexpr int kSeg = 64;          // cells per wavefront work item (four 16-cell blocks)

// wt[((tap * 2 + nb) * 2 + h) * 64 + l) * 4 + j] = W[16 nb + l%16][8 (l/16) + 4h + j][tap]
__global__ void k3c_wprep(const float* __restrict__ w, float* __restrict__ wt)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NWT) return;
    const int j = k & 3, l = (k >> 2) & 63, h = (k >> 8) & 1, nb = (k >> 9) & 1, tap = k >> 10;
    const int o = 16 * nb + (l & 15), ci = 8 * (l >> 4) + 4 * h + j;
    wt[k] = w[(o * C + ci) * TAPS + tap];
}

// Layer 1: 3 -> 32 with ReLU, one cell per lane; weights in LDS as [cin][tap][32].  A block of
// 256 threads takes 4 rows x 64 cells of one plane and first stages their 3 x 3 x 3 neighbourhood
// of the velocity (3 components x 3 planes x 6 rows x 66 cells, zero outside the grid) in LDS,
// so each input value is read from memory once per block instead of once per tap.  The output
// activations are FP32, or BF16 rounded to nearest even for the BF16 pass.
constexpr int kC1R = 4, kC1W = 64;  // rows and cells of a block
template <class T>
__global__ __launch_bounds__(kC1R * kC1W) void k3c_conv1(int32_t G, const float* __restrict__ vel,
                                                         const float* __restrict__ w, const float* __restrict__ b,
                                                         T* __restrict__ out)
{
    constexpr int VR = kC1R + 2, VW = kC1W + 2, VP = VR * VW;  // one staged plane
    __shared__ float s_w[CIO * TAPS * C];
    __shared__ float s_b[C];
    __shared__ float s_v[CIO * 3 * VP];
    const int tid = threadIdx.x;
    for (int k = tid; k < CIO * TAPS * C; k += kC1R * kC1W) {
        const int o = k % C, ct = k / C;  // ct = cin * 27 + tap
        s_w[k] = w[o * CIO * TAPS + ct];
    }
    if (tid < C) s_b[tid] = b[tid];
    const int segs = (G + kC1W - 1) / kC1W, bands = (G + kC1R - 1) / kC1R;
    const int64_t blk = blockIdx.x;
    const int x0 = (int)(blk % segs) * kC1W, y0 = (int)((blk / segs) % bands) * kC1R;
    const int z = (int)(blk / ((int64_t)segs * bands));
    const int64_t n = (int64_t)G * G * G;
    for (int e = tid; e < CIO * 3 * VP; e += kC1R * kC1W) {
        const int c = e % VW, r = (e / VW) % VR, dz = (e / VP) % 3, ci = e / (3 * VP);
        const int Z = z + dz - 1, Y = y0 + r - 1, X = x0 + c - 1;
        s_v[e] = (Z >= 0 && Z < G && Y >= 0 && Y < G && X >= 0 && X < G)
                     ? vel[(int64_t)ci * n + ((int64_t)Z * G + Y) * G + X]
                     : 0.f;
    }
    __syncthreads();
    const int tx = tid % kC1W, ty = tid / kC1W;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= G || y >= G) return;
    float acc[C];
#pragma unroll
    for (int o = 0; o < C; ++o) acc[o] = s_b[o];
    for (int ci = 0; ci < CIO; ++ci) {
        for (int t = 0; t < TAPS; ++t) {
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            const float a = s_v[((ci * 3 + dz) * VR + ty + dy) * VW + tx + dx];
            const v4f* wr = reinterpret_cast<const v4f*>(s_w + (ci * TAPS + t) * C);
#pragma unroll
            for (int q = 0; q < C / 4; ++q) {
                const v4f wq = wr[q];
                acc[4 * q] += wq.x * a;
                acc[4 * q + 1] += wq.y * a;
                acc[4 * q + 2] += wq.z * a;
                acc[4 * q + 3] += wq.w * a;
            }
        }
    }
    const int64_t v = ((int64_t)z * G + y) * G + x;
    if constexpr (sizeof(T) == 4) {
        v4f* dst = reinterpret_cast<v4f*>(out + v * C);
#pragma unroll
        for (int q = 0; q < C / 4; ++q)
            dst[q] = v4f{ fmaxf(acc[4 * q], 0.f), fmaxf(acc[4 * q + 1], 0.f), fmaxf(acc[4 * q + 2], 0.f),
                          fmaxf(acc[4 * q + 3], 0.f) };
    } else {
        bf16x8* dst = reinterpret_cast<bf16x8*>(out + v * C);
#pragma unroll
        for (int q = 0; q < C / 8; ++q) {
            v8f r;
#pragma unroll
            for (int j = 0; j < 8; ++j) r[j] = fmaxf(acc[8 * q + j], 0.f);
            dst[q] = __builtin_convertvector(r, bf16x8);
        }
    }
}

// The work items (64 cells of an x row) of a persistent block: the blocks of one XCD (block id
// mod 8) take neighbouring contiguous ranges, so the rows above and below and the neighbouring
// planes, which the taps read, are shared in that XCD's L2.
__device__ __forceinline__ void item_range(int64_t n_items, int64_t& i0, int64_t& i1)
{
    const int64_t nblk = gridDim.x;
    int64_t lb = blockIdx.x;
    if (nblk % 8 == 0) lb = (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8;
    const int64_t per = (n_items + nblk - 1) / nblk;
    i0 = lb * per;
    i1 = i0 + per < n_items ? i0 + per : n_items;
}

// Layers 2 and 3: 32 -> 32 with ReLU on the matrix cores, persistent blocks of 12 wavefronts
// (three per SIMD).  The next tap's activations are loaded while this tap's 64 matrix
// instructions run: that needs 160 registers, so three wavefronts per SIMD instead of four
// without the prefetch (whole pass at G = 128: 3.43 ms without it, 3.25 ms with it at two
// wavefronts per SIMD, 3.12 ms at three; four wavefronts with the prefetch spill).
__global__ __launch_bounds__(kWaves32 * 64) void k3c_conv32(int32_t G, const float* __restrict__ in,
                                                            const float* __restrict__ wt,
                                                            const float* __restrict__ bias,
                                                            float* __restrict__ out)
{
    __shared__ v4f s_w[NWT / 4];
    for (int k = threadIdx.x; k < NWT / 4; k += kWaves32 * 64) s_w[k] = reinterpret_cast<const v4f*>(wt)[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int segs = (G + kSeg - 1) / kSeg;
    const int64_t n_items = (int64_t)G * G * segs;
    int64_t i0, i1;
    item_range(n_items, i0, i1);
    v4f bv[2];
    bv[0] = *reinterpret_cast<const v4f*>(bias + 4 * grp);
    bv[1] = *reinterpret_cast<const v4f*>(bias + 16 + 4 * grp);
    for (int64_t item = i0 + wave; item < i1; item += kWaves32) {
        const int seg = (int)(item % segs);
        const int64_t row = item / segs;  // z G + y
        const int y = (int)(row % G), z = (int)(row / G);
        const int x0 = seg * kSeg;
        v4f acc[4][2];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            acc[mb][0] = bv[0];
            acc[mb][1] = bv[1];
        }
        auto load = [&](int t, v4f (&bo)[4][2]) {
            const int Z = z + t / 9 - 1, Y = y + (t / 3) % 3 - 1, dx = t % 3 - 1;
            const bool ok = Z >= 0 && Z < G && Y >= 0 && Y < G;
            const float* src = in + ((int64_t)(ok ? Z : 0) * G + (ok ? Y : 0)) * G * C + 8 * grp;
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const int X = x0 + 16 * mb + col + dx;
                if (ok && X >= 0 && X < G) {
                    const v4f* p = reinterpret_cast<const v4f*>(src + (int64_t)X * C);
                    bo[mb][0] = p[0];
                    bo[mb][1] = p[1];
                } else {
                    bo[mb][0] = v4f{ 0.f, 0.f, 0.f, 0.f };
                    bo[mb][1] = v4f{ 0.f, 0.f, 0.f, 0.f };
                }
            }
        };
        v4f bop[4][2], bnx[4][2];
        load(0, bop);
        for (int t = 0; t < TAPS; ++t) {
            if (t + 1 < TAPS) load(t + 1, bnx);
            v4f aop[2][2];
#pragma unroll
            for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                for (int h = 0; h < 2; ++h) aop[nb][h] = s_w[((t * 2 + nb) * 2 + h) * 64 + lane];
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
                        for (int nb = 0; nb < 2; ++nb)
                            acc[mb][nb] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(aop[nb][h][j], bop[mb][h][j], acc[mb][nb], 0, 0, 0);
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                bop[mb][0] = bnx[mb][0];
                bop[mb][1] = bnx[mb][1];
            }
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int X = x0 + 16 * mb + col;
            if (X >= G) continue;
            v4f* dst = reinterpret_cast<v4f*>(out + (row * G + X) * C + 4 * grp);
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const v4f a = acc[mb][nb];
                dst[4 * nb] = v4f{ fmaxf(a.x, 0.f), fmaxf(a.y, 0.f), fmaxf(a.z, 0.f), fmaxf(a.w, 0.f) };
            }
        }
    }
}

// BF16 operand-ordered weights: wb[(tap * 2 + nb) * 64 + l] holds, as 8 BF16 (rounded to
// nearest even), W[16 nb + l%16][8 (l/16) + j][tap] for j = 0..7: the A operand of
// v_mfma_f32_16x16x32_bf16 (row = output channel, k = input channel 8 (l/16) + j).
__global__ void k3c_wprep_bf16(const float* __restrict__ w, bf16x8* __restrict__ wb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NWB) return;
    const int l = k & 63, nb = (k >> 6) & 1, tap = k >> 7;
    const int o = 16 * nb + (l & 15), c0 = 8 * (l >> 4);
    v8f v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = w[(o * C + c0 + j) * TAPS + tap];
    wb[k] = __builtin_convertvector(v, bf16x8);
}

// Layers 2 and 3 in BF16 (BF16 activations and weights, FP32 accumulation): one
// v_mfma_f32_16x16x32_bf16 per tap covers all 32 input channels of 16 cells x 16 output
// channels.  Lane l's B operand is channels 8 (l/16) .. +7 of cell l%16 (one 16-byte load), and
// it receives output channels 16 nb + 4 (l/16) + r of cell l%16, stored as four BF16 after ReLU.
// Persistent blocks of 16 wavefronts, the next tap loaded while this tap's 8 instructions run.
__global__ __launch_bounds__(16 * 64) void k3c_conv32_bf16(int32_t G, const bf16* __restrict__ in,
                                                          const bf16x8* __restrict__ wb,
                                                          const float* __restrict__ bias, bf16* __restrict__ out)
{
    __shared__ bf16x8 s_w[NWB];
    for (int k = threadIdx.x; k < NWB; k += 16 * 64) s_w[k] = wb[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int segs = (G + kSeg - 1) / kSeg;
    int64_t i0, i1;
    item_range((int64_t)G * G * segs, i0, i1);
    const v4f bv0 = *reinterpret_cast<const v4f*>(bias + 4 * grp);
    const v4f bv1 = *reinterpret_cast<const v4f*>(bias + 16 + 4 * grp);
    for (int64_t item = i0 + wave; item < i1; item += 16) {
        const int seg = (int)(item % segs);
        const int64_t row = item / segs;
        const int y = (int)(row % G), z = (int)(row / G);
        const int x0 = seg * kSeg;
        v4f acc[4][2];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            acc[mb][0] = bv0;
            acc[mb][1] = bv1;
        }
        auto load = [&](int t, bf16x8 (&bo)[4]) {
            const int Z = z + t / 9 - 1, Y = y + (t / 3) % 3 - 1, dx = t % 3 - 1;
            const bool ok = Z >= 0 && Z < G && Y >= 0 && Y < G;
            const bf16* src = in + ((int64_t)(ok ? Z : 0) * G + (ok ? Y : 0)) * G * C + 8 * grp;
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const int X = x0 + 16 * mb + col + dx;
                if (ok && X >= 0 && X < G)
                    bo[mb] = *reinterpret_cast<const bf16x8*>(src + (int64_t)X * C);
                else
                    bo[mb] = bf16x8{ 0, 0, 0, 0, 0, 0, 0, 0 };
            }
        };
        bf16x8 bop[4], bnx[4];
        load(0, bop);
#pragma unroll 1
        for (int t = 0; t < TAPS; ++t) {
            if (t + 1 < TAPS) load(t + 1, bnx);
            const bf16x8 a0 = s_w[(t * 2) * 64 + lane], a1 = s_w[(t * 2 + 1) * 64 + lane];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                acc[mb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, bop[mb], acc[mb][0], 0, 0, 0);
                acc[mb][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, bop[mb], acc[mb][1], 0, 0, 0);
            }
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) bop[mb] = bnx[mb];
        }
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int X = x0 + 16 * mb + col;
            if (X >= G) continue;
            bf16* dst = out + (row * G + X) * C + 4 * grp;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const v4f a = acc[mb][nb];
                const v4f r{ fmaxf(a.x, 0.f), fmaxf(a.y, 0.f), fmaxf(a.z, 0.f), fmaxf(a.w, 0.f) };
                *reinterpret_cast<bf16x4*>(dst + 16 * nb) = __builtin_convertvector(r, bf16x4);
            }
        }
    }
}

// Layer 4 in the BF16 pass on the matrix cores: the 3 output channels padded to one 16-row A
// block, wb4[tap * 64 + l] = W4[l%16][8 (l/16) + j][tap] as BF16 (zero for rows >= 3), so a tap is
// one v_mfma_f32_16x16x32_bf16 per 16 cells.  Lanes 0..15 receive output channels 0..3 of
// their cell, the first three of which are written with the bias added.
__global__ void k3c_wprep4_bf16(const float* __restrict__ w, bf16x8* __restrict__ wb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= TAPS * 64) return;
    const int l = k & 63, tap = k >> 6;
    const int o = l & 15, c0 = 8 * (l >> 4);
    v8f v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = o < CIO ? w[(o * C + c0 + j) * TAPS + tap] : 0.f;
    wb[k] = __builtin_convertvector(v, bf16x8);
}

__global__ __launch_bounds__(16 * 64) void k3c_conv4_bf16(int32_t G, const bf16* __restrict__ in,
                                                         const bf16x8* __restrict__ wb, const float* __restrict__ b,
                                                         float* __restrict__ disp)
{
    __shared__ bf16x8 s_w[TAPS * 64];
    for (int k = threadIdx.x; k < TAPS * 64; k += 16 * 64) s_w[k] = wb[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int segs = (G + kSeg - 1) / kSeg;
    const int64_t n = (int64_t)G * G * G;
    const float b0 = b[0], b1 = b[1], b2 = b[2];
    int64_t i0, i1;
    item_range((int64_t)G * G * segs, i0, i1);
    for (int64_t item = i0 + wave; item < i1; item += 16) {
        const int seg = (int)(item % segs);
        const int64_t row = item / segs;
        const int y = (int)(row % G), z = (int)(row / G);
        const int x0 = seg * kSeg;
        v4f acc[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) acc[mb] = v4f{ 0.f, 0.f, 0.f, 0.f };
        auto load = [&](int t, bf16x8 (&bo)[4]) {
            const int Z = z + t / 9 - 1, Y = y + (t / 3) % 3 - 1, dx = t % 3 - 1;
            const bool ok = Z >= 0 && Z < G && Y >= 0 && Y < G;
            const bf16* src = in + ((int64_t)(ok ? Z : 0) * G + (ok ? Y : 0)) * G * C + 8 * grp;
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const int X = x0 + 16 * mb + col + dx;
                if (ok && X >= 0 && X < G)
                    bo[mb] = *reinterpret_cast<const bf16x8*>(src + (int64_t)X * C);
                else
                    bo[mb] = bf16x8{ 0, 0, 0, 0, 0, 0, 0, 0 };
            }
        };
        bf16x8 bop[4], bnx[4];
        load(0, bop);
        for (int t = 0; t < TAPS; ++t) {
            if (t + 1 < TAPS) load(t + 1, bnx);
            const bf16x8 a = s_w[t * 64 + lane];
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bop[mb], acc[mb], 0, 0, 0);
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) bop[mb] = bnx[mb];
        }
        if (grp == 0) {
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) {
                const int X = x0 + 16 * mb + col;
                if (X >= G) continue;
                const int64_t c = row * G + X;
                disp[c] = acc[mb].x + b0;
                disp[n + c] = acc[mb].y + b1;
                disp[2 * n + c] = acc[mb].z + b2;
            }
        }
    }
}

__device__ __forceinline__ void conv4_item(int32_t G, const float* __restrict__ in, const v4f* s_w, int segs,
                                           int64_t item, int col, int grp, int64_t n, float bias,
                                           float* __restrict__ disp)
{
    const int seg = (int)(item % segs);
    const int64_t row = item / segs;
    const int y = (int)(row % G), z = (int)(row / G);
    const int x0 = seg * kSeg;
    float acc[4][CIO];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int o = 0; o < CIO; ++o) acc[mb][o] = 0.f;
    for (int t = 0; t < TAPS; ++t) {
        const int Z = z + t / 9 - 1, Y = y + (t / 3) % 3 - 1, dx = t % 3 - 1;
        if (Z < 0 || Z >= G || Y < 0 || Y >= G) continue;
        const float* src = in + ((int64_t)Z * G + Y) * G * C + 8 * grp;
        const v4f* wq = s_w + (t * 4 + grp) * 6;  // 24 floats: [channel][output]
        const v4f w0 = wq[0], w1 = wq[1], w2 = wq[2], w3 = wq[3], w4 = wq[4], w5 = wq[5];
        const float wv[24] = { w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w, w2.x, w2.y, w2.z, w2.w,
                               w3.x, w3.y, w3.z, w3.w, w4.x, w4.y, w4.z, w4.w, w5.x, w5.y, w5.z, w5.w };
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int X = x0 + 16 * mb + col + dx;
            if (X < 0 || X >= G) continue;
            const v4f* p = reinterpret_cast<const v4f*>(src + (int64_t)X * C);
            const v4f a0 = p[0], a1 = p[1];
            const float av[8] = { a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w };
#pragma unroll
            for (int c = 0; c < 8; ++c)
#pragma unroll
                for (int o = 0; o < CIO; ++o) acc[mb][o] += wv[c * CIO + o] * av[c];
        }
    }
    // add the four lane groups (lanes l, l ^ 16, l ^ 32, l ^ 48 hold the same cell)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int o = 0; o < CIO; ++o) {
            float v = acc[mb][o];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            acc[mb][o] = v;
        }
    // lane group g < 3 writes output component g for the 64 cells
    if (grp < CIO) {
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            const int X = x0 + 16 * mb + col;
            if (X >= G) continue;
            const float v = grp == 0 ? acc[mb][0] : (grp == 1 ? acc[mb][1] : acc[mb][2]);
            disp[(int64_t)grp * n + row * G + X] = v + bias;
        }
    }
}


// Layer 4: 32 -> 3, no ReLU.  A wavefront takes a work item of 64 cells of an x row as the
// matrix layers do, and reads activations the same way: lane l loads channels 8 (l/16) .. +7 of
// cell l%16 of each 16-cell block (four lanes cover a cell's 128-byte line), forms the partial
// sums of its 8 channels for the 3 outputs, and the four lane groups' sums are added across lanes.
// Weights in LDS as [tap][lane group][8 channels][3].
__global__ __launch_bounds__(kWaves4 * 64) void k3c_conv4(int32_t G, const float* __restrict__ in,
                                                           const float* __restrict__ w, const float* __restrict__ b,
                                                           float* __restrict__ disp)
{
    __shared__ v4f s_w[TAPS * C * CIO / 4];
    float* const sw = reinterpret_cast<float*>(s_w);
    for (int k = threadIdx.x; k < TAPS * C * CIO; k += kWaves4 * 64) {
        const int o = k % CIO, ci = (k / CIO) % C, t = k / (CIO * C);  // ci = 8 group + channel
        sw[k] = w[(o * C + ci) * TAPS + t];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    const int segs = (G + kSeg - 1) / kSeg;
    const int64_t n = (int64_t)G * G * G;
    const float bias = b[grp < CIO ? grp : 0];
    int64_t i0, i1;
    item_range((int64_t)G * G * segs, i0, i1);
    for (int64_t item = i0 + (threadIdx.x >> 6); item < i1; item += kWaves4)
        conv4_item(G, in, s_w, segs, item, col, grp, n, bias, disp);
}

}  // namespace

size_t cnn3_workspace_bytes(int32_t G)
{
    const size_t cells = (size_t)G * G * G;
    return 2 * cells * C * sizeof(float) + 2 * (size_t)NWT * sizeof(float);
}

void run_predict3(cnnsns_mesh3_s& m, const float* vel, const cnnsns_cnn& w, int32_t precision, float* disp,
                  hipStream_t stream)
{
    if (precision != CNNSNS_F32 && precision != CNNSNS_BF16) fail(CNNSNS_EINVAL, "predict3d: unsupported precision");
    std::lock_guard<std::mutex> lock(m.ws.mu);
    workspace_acquire(m.ws, cnn3_workspace_bytes(m.G), stream, "predict3d");
    const int32_t G = m.G;
    const int64_t cells = (int64_t)G * G * G;
    const unsigned grid = cnn_persistent_grid();
    const int64_t c1blocks = (int64_t)G * ((G + kC1R - 1) / kC1R) * ((G + kC1W - 1) / kC1W);
    if (c1blocks > (int64_t)UINT32_MAX) fail(CNNSNS_EINVAL, "predict3d: overlay too large");
    const unsigned c1grid = (unsigned)c1blocks;
    float* act0 = static_cast<float*>(m.ws.ptr);
    float* act1 = act0 + cells * C;
    float* wt2 = act1 + cells * C;
    float* wt3 = wt2 + NWT;
    if (precision == CNNSNS_BF16) {
        bf16* b0 = reinterpret_cast<bf16*>(act0);
        bf16* b1 = reinterpret_cast<bf16*>(act1);
        bf16x8* wb2 = reinterpret_cast<bf16x8*>(wt2);
        bf16x8* wb3 = reinterpret_cast<bf16x8*>(wt3);
        k3c_wprep_bf16<<<(NWB + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[1], wb2);
        k3c_wprep_bf16<<<(NWB + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[2], wb3);
        k3c_conv1<bf16><<<c1grid, kC1R * kC1W, 0, stream>>>(G, vel, w.w[0], w.b[0], b0);
        k3c_conv32_bf16<<<grid, 16 * 64, 0, stream>>>(G, b0, wb2, w.b[1], b1);
        k3c_conv32_bf16<<<grid, 16 * 64, 0, stream>>>(G, b1, wb3, w.b[2], b0);
        bf16x8* wb4 = wb3 + NWB;
        k3c_wprep4_bf16<<<(TAPS * 64 + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[3], wb4);
        k3c_conv4_bf16<<<grid, 16 * 64, 0, stream>>>(G, b0, wb4, w.b[3], disp);
    } else {
        k3c_wprep<<<(NWT + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[1], wt2);
        k3c_wprep<<<(NWT + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[2], wt3);
        k3c_conv1<float><<<c1grid, kC1R * kC1W, 0, stream>>>(G, vel, w.w[0], w.b[0], act0);
        k3c_conv32<<<grid, kWaves32 * 64, 0, stream>>>(G, act0, wt2, w.b[1], act1);
        k3c_conv32<<<grid, kWaves32 * 64, 0, stream>>>(G, act1, wt3, w.b[2], act0);
        k3c_conv4<<<grid, kWaves4 * 64, 0, stream>>>(G, act0, w.w[3], w.b[3], disp);
    }
    hip_check(hipGetLastError(), "predict3d launch");
    workspace_used(m.ws, stream);
}

}  // namespace cnnsns
