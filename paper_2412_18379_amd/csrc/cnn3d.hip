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
// on the matrix cores in FP32 as a z-sweep (k3c_zconv1: three velocity planes
// staged in LDS, K = one tap's three components and a zero); layer 4 reads its
// input once per plane in a z-sweep and runs on the vector ALUs in FP32
// (k3c_zconv4_f32).  The BF16 pass (BF16
// operands after layer 1, FP32 accumulation) runs layers 2-4 as z-sweeps that
// stage three input planes at a time in LDS (described before
// k3c_zsweep_bf16), layer 4 with its 3 outputs padded to 16.
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

// Layer 4 in the BF16 pass on the matrix cores: the 3 output channels padded to one 16-row A
// block, wb4[tap * 64 + l] = W4[l%16][8 (l/16) + j][tap] as BF16 (zero for rows >= 3), so a tap is
// one v_mfma_f32_16x16x32_bf16 per 16 cells; lanes 0..15 receive output channels 0..3 of their
// cell, the first three of which are written with the bias added.
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

// Layers 2-4 of the BF16 pass as z-sweeps through LDS.  A block owns a column of ZY x ZX cells
// and ZP consecutive planes; it keeps the three input planes that its current output plane reads,
// each as a (ZY + 2) x (ZX + 2) slab with the one-cell border (zero outside the grid), in a ring
// in LDS, so every input cell is read from memory once per block (plus the borders) instead of
// once per tap.  While a plane's 27 taps run on the matrix cores, the plane after next is loaded
// into registers; it replaces the oldest slab after the plane is done.  Eight wavefronts take two
// 16-cell M-blocks each (the 256 cells of a plane; sixteen wavefronts of one M-block each ran
// 10% slower); a tap is one v_mfma_f32_16x16x32_bf16 per M-block and 16 output channels (NB such
// blocks: two for 32 -> 32, one for 32 -> 3 with the outputs padded to 16).
constexpr int ZY = 8, ZX = 32, ZP = 32;           // cells per block: rows, columns, planes
constexpr int ZSY = ZY + 2, ZSX = ZX + 2;         // slab with its border
// bf16 per slab cell: 32 channels + 16 pad, 96 bytes.  The LDS serves a 16-byte read in groups of
// 16 lanes over 64 four-byte banks, a group joining lanes 0-7 with 56-63 (8-15 with 48-55, ...): here
// eight consecutive cells at one 16-byte channel chunk and eight others at the mirrored chunk.  With
// a 96-byte pitch those sixteen reads fall in distinct bank groups; with 80 bytes half of them collide.
constexpr int ZCS = 48;
constexpr int ZSLAB = ZSY * ZSX * ZCS;            // bf16 per slab
constexpr int kZThreads = 512;
constexpr int ZCHUNKS = ZSY * ZSX * 4;            // 16-byte pieces of a slab
constexpr int ZCH_PER_THREAD = (ZCHUNKS + kZThreads - 1) / kZThreads;
static_assert(ZY * ZX == (kZThreads / 64) * 2 * 16, "two M-blocks per wavefront cover a plane");

template <int NB>
__global__ __launch_bounds__(kZThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k3c_zsweep_bf16(
    int32_t G, const bf16* __restrict__ in, const bf16x8* __restrict__ wb, const float* __restrict__ bias,
    bf16* __restrict__ out, float* __restrict__ disp)
{
    __shared__ __attribute__((aligned(16))) bf16 s_slab[3 * ZSLAB];
    __shared__ bf16x8 s_w[TAPS * NB * 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    for (int k = tid; k < TAPS * NB * 64; k += kZThreads) s_w[k] = wb[k];
    const int tiles_x = (G + ZX - 1) / ZX, tiles_y = (G + ZY - 1) / ZY;
    const int64_t b = blockIdx.x;
    const int tx0 = (int)(b % tiles_x) * ZX, ty0 = (int)((b / tiles_x) % tiles_y) * ZY;
    const int z0 = (int)(b / ((int64_t)tiles_x * tiles_y)) * ZP;
    const int z1 = min(z0 + ZP, G);
    const int64_t GG = (int64_t)G * G;

    // the wavefront's M-blocks: cells (ty0 + r, tx0 + 16 h + col) with r = wave, h = 0, 1
    const int r = wave;
    // slab offsets (bf16) of the lane's operand for tap (dy, dx) = (0, 0), per M-block
    int base[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) base[h] = (r * ZSX + 16 * h + col) * ZCS + 8 * grp;

    // Plane p of the slab into registers: unconditional loads from clamped positions (a chunk past
    // the end loads the last one again); the zero padding is applied when the plane is stashed,
    // every store unconditional (a thread past the end writes the last chunk again, the value its
    // owner writes).  So the loads stay in flight while a plane's taps run; with a branch around them
    // the compiled code had waited for them before the plane's first matrix instruction.
    bf16x8 pf[ZCH_PER_THREAD];
    auto fetch = [&](int p) {
        const int pc = min(max(p, 0), G - 1);
#pragma unroll
        for (int k = 0; k < ZCH_PER_THREAD; ++k) {
            const int e = min(tid + k * kZThreads, ZCHUNKS - 1);
            const int cell = e >> 2, part = e & 3;
            const int gy = min(max(ty0 + cell / ZSX - 1, 0), G - 1), gx = min(max(tx0 + cell % ZSX - 1, 0), G - 1);
            pf[k] = *reinterpret_cast<const bf16x8*>(in + ((int64_t)pc * GG + (int64_t)gy * G + gx) * C + 8 * part);
        }
    };
    auto stash = [&](int p) {
        bf16* dst = s_slab + ((p + 3) % 3) * ZSLAB;
        const bool pin = p >= 0 && p < G;
#pragma unroll
        for (int k = 0; k < ZCH_PER_THREAD; ++k) {
            const int e = min(tid + k * kZThreads, ZCHUNKS - 1);
            const int cell = e >> 2;
            const int gy = ty0 + cell / ZSX - 1, gx = tx0 + cell % ZSX - 1;
            const bool on = pin && gy >= 0 && gy < G && gx >= 0 && gx < G;
            *reinterpret_cast<bf16x8*>(dst + cell * ZCS + 8 * (e & 3)) = on ? pf[k] : bf16x8{ 0, 0, 0, 0, 0, 0, 0, 0 };
        }
    };
    fetch(z0 - 1);
    stash(z0 - 1);
    fetch(z0);
    stash(z0);
    fetch(z0 + 1);
    stash(z0 + 1);
    __syncthreads();
    // the first 16 output channels' weights stay in registers for the whole sweep (all of the
    // layer's weights do not fit beside the operands at two wavefronts per SIMD); the other block's
    // are read from LDS per tap
    bf16x8 wr[TAPS];
#pragma unroll
    for (int t = 0; t < TAPS; ++t) wr[t] = s_w[(t * NB) * 64 + lane];

    v4f bl[2];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        if (NB == 2) {
            bl[nb] = *reinterpret_cast<const v4f*>(bias + 16 * nb + 4 * grp);
        } else {  // rows 4 grp + j of the single output block: channels 0..2 are real
            bl[nb] = v4f{ 0.f, 0.f, 0.f, 0.f };
        }
    }
    for (int z = z0; z < z1; ++z) {
        fetch(z + 2);  // lands while this plane computes (after the block's last plane: unused)
        __builtin_amdgcn_sched_barrier(0);  // the loads stay ahead of the plane's taps
        v4f acc[2][NB];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[h][nb] = bl[nb];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            const bf16* sl = s_slab + ((z + dz - 1 + 3) % 3) * ZSLAB;
#pragma unroll
            for (int t9 = 0; t9 < 9; ++t9) {
                const int t = dz * 9 + t9, off = ((t9 / 3) * ZSX + t9 % 3) * ZCS;
                const bf16x8 a0 = *reinterpret_cast<const bf16x8*>(sl + base[0] + off);
                const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(sl + base[1] + off);
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const bf16x8 w = nb == 0 ? wr[t] : s_w[(t * NB + nb) * 64 + lane];
                    acc[0][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, a0, acc[0][nb], 0, 0, 0);
                    acc[1][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, a1, acc[1][nb], 0, 0, 0);
                }
            }
        }
        // results: lane (col, grp) holds rows 4 grp + j (output channels 16 nb + 4 grp + j) of cell col
        const int gy = ty0 + r;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int gx = tx0 + 16 * h + col;
            if (gy >= G || gx >= G) continue;
            const int64_t c = (int64_t)z * GG + (int64_t)gy * G + gx;
            if (NB == 2) {
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) {
                    const v4f a = acc[h][nb];
                    const v4f v{ fmaxf(a.x, 0.f), fmaxf(a.y, 0.f), fmaxf(a.z, 0.f), fmaxf(a.w, 0.f) };
                    *reinterpret_cast<bf16x4*>(out + c * C + 16 * nb + 4 * grp) = __builtin_convertvector(v, bf16x4);
                }
            } else if (grp == 0) {
                disp[c] = acc[h][0].x + bias[0];
                disp[GG * G + c] = acc[h][0].y + bias[1];
                disp[2 * GG * G + c] = acc[h][0].z + bias[2];
            }
        }
        __syncthreads();           // every wavefront is done with the slab of plane z - 1
        stash(z + 2);  // after the last plane it replaces a plane no longer read
        __syncthreads();
    }
}

// Layer 1 (3 -> 32) as a z-sweep on the matrix cores in FP32 (both passes; the BF16 pass rounds
// its output): the velocity's three planes in LDS as (u, v, w, 0) per cell, one
// v_mfma_f32_16x16x4f32 per tap and 16 output channels with K = the three components and a zero,
// the weights (one float per lane, tap and block of 16 output channels) held in registers.
constexpr int Z1CS = 4;  // floats per slab cell

constexpr int kZ1Threads = 1024;  // one 16-cell M-block per wavefront
template <class T>
__global__ __launch_bounds__(kZ1Threads) void k3c_zconv1(int32_t G, const float* __restrict__ vel,
                                                        const float* __restrict__ w, const float* __restrict__ bias,
                                                        T* __restrict__ out)
{
    constexpr int NCELL = ZSY * ZSX;
    static_assert(NCELL <= kZ1Threads && ZY * ZX == (kZ1Threads / 64) * 16, "one slab cell per thread");
    __shared__ __attribute__((aligned(16))) float s_v[3 * NCELL * Z1CS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    // A operands: lane (col, grp) holds W[16 nb + col][grp][tap] (zero for grp = 3)
    float wa[TAPS][2];
#pragma unroll
    for (int t = 0; t < TAPS; ++t)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) wa[t][nb] = grp < CIO ? w[((16 * nb + col) * CIO + grp) * TAPS + t] : 0.f;
    const int tiles_x = (G + ZX - 1) / ZX, tiles_y = (G + ZY - 1) / ZY;
    const int64_t b = blockIdx.x;
    const int tx0 = (int)(b % tiles_x) * ZX, ty0 = (int)((b / tiles_x) % tiles_y) * ZY;
    const int z0 = (int)(b / ((int64_t)tiles_x * tiles_y)) * ZP;
    const int z1 = min(z0 + ZP, G);
    const int64_t GG = (int64_t)G * G, n = GG * G;
    const int r = wave >> 1, h = wave & 1;

    v4f pf;
    auto fetch = [&](int p) {  // thread tid < NCELL: its slab cell of plane p (zero outside the grid)
        pf = v4f{ 0.f, 0.f, 0.f, 0.f };
        if (tid < NCELL) {
            const int gy = ty0 + tid / ZSX - 1, gx = tx0 + tid % ZSX - 1;
            if (p >= 0 && p < G && gy >= 0 && gy < G && gx >= 0 && gx < G) {
                const int64_t c = (int64_t)p * GG + (int64_t)gy * G + gx;
                pf = v4f{ vel[c], vel[n + c], vel[2 * n + c], 0.f };
            }
        }
    };
    auto stash = [&](int p) {
        if (tid < NCELL) *reinterpret_cast<v4f*>(s_v + (((p + 3) % 3) * NCELL + tid) * Z1CS) = pf;
    };
    fetch(z0 - 1);
    stash(z0 - 1);
    fetch(z0);
    stash(z0);
    fetch(z0 + 1);
    stash(z0 + 1);
    __syncthreads();
    const v4f bl0 = *reinterpret_cast<const v4f*>(bias + 4 * grp);
    const v4f bl1 = *reinterpret_cast<const v4f*>(bias + 16 + 4 * grp);
    const int cell0 = r * ZSX + 16 * h + col;  // the lane's output cell in the slab, and its channel
    for (int z = z0; z < z1; ++z) {
        if (z + 2 < z1 + 1) fetch(z + 2);
        v4f acc0 = bl0, acc1 = bl1;
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            const float* sl = s_v + ((z + dz - 1 + 3) % 3) * NCELL * Z1CS + cell0 * Z1CS + grp;
#pragma unroll
            for (int t9 = 0; t9 < 9; ++t9) {
                const float a = sl[((t9 / 3) * ZSX + t9 % 3) * Z1CS];
                acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[dz * 9 + t9][0], a, acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(wa[dz * 9 + t9][1], a, acc1, 0, 0, 0);
            }
        }
        const int gy = ty0 + r, gx = tx0 + 16 * h + col;
        if (gy < G && gx < G) {
            T* dst = out + ((int64_t)z * GG + (int64_t)gy * G + gx) * C + 4 * grp;
            const v4f v0{ fmaxf(acc0.x, 0.f), fmaxf(acc0.y, 0.f), fmaxf(acc0.z, 0.f), fmaxf(acc0.w, 0.f) };
            const v4f v1{ fmaxf(acc1.x, 0.f), fmaxf(acc1.y, 0.f), fmaxf(acc1.z, 0.f), fmaxf(acc1.w, 0.f) };
            if constexpr (sizeof(T) == 4) {
                *reinterpret_cast<v4f*>(dst) = v0;
                *reinterpret_cast<v4f*>(dst + 16) = v1;
            } else {
                *reinterpret_cast<bf16x4*>(dst) = __builtin_convertvector(v0, bf16x4);
                *reinterpret_cast<bf16x4*>(dst + 16) = __builtin_convertvector(v1, bf16x4);
            }
        }
        __syncthreads();
        if (z + 2 < z1 + 1) stash(z + 2);
        __syncthreads();
    }
}

// Layer 1 of the BF16 pass on the BF16 matrix cores with split operands: each velocity value
// v = v_h + v_l and each weight w = w_h + w_l as a BF16 pair (v_h, w_h rounded to nearest, the
// rest rounded again), and w v taken as w_h v_h + w_h v_l + w_l v_h, which is within about 2^-16
// of it, far below the BF16 rounding of the layer's output.  A slab cell holds
// (v_h0, v_h1, v_h2, v_l0, v_l1, v_l2, 0, 0); a tap takes K = 16 (two lane groups that both read
// that cell): weights (w_h, w_h, 0) against it for the first group, (w_l, 0, 0) for the second,
// so a K = 32 step covers two taps (14 steps for 27 taps, the last half empty).
constexpr int NW1S = 14 * 2 * 64;  // bf16x8 operands of the split layer 1

// wb[(s * 2 + nb) * 64 + l]: output channel 16 nb + l%16; lane group g = l/16 takes tap 2 s + g/2
__global__ void k3c_wprep1_split(const float* __restrict__ w, bf16x8* __restrict__ wb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NW1S) return;
    const int l = k & 63, nb = (k >> 6) & 1, st = k >> 7, g = l >> 4;
    const int o = 16 * nb + (l & 15), t = 2 * st + (g >> 1);
    bf16x8 v = bf16x8{ 0, 0, 0, 0, 0, 0, 0, 0 };
    if (t < TAPS) {
#pragma unroll
        for (int ci = 0; ci < CIO; ++ci) {
            const float x = w[(o * CIO + ci) * TAPS + t];
            const bf16 hi = (bf16)x;
            const bf16 lo = (bf16)(x - (float)hi);
            if ((g & 1) == 0) {
                v[ci] = hi;
                v[3 + ci] = hi;
            } else {
                v[ci] = lo;
            }
        }
    }
    wb[k] = v;
}

__global__ __launch_bounds__(kZ1Threads) void k3c_zconv1_split(int32_t G, const float* __restrict__ vel,
                                                               const bf16x8* __restrict__ wb,
                                                               const float* __restrict__ bias, bf16* __restrict__ out)
{
    constexpr int NCELL = ZSY * ZSX;
    static_assert(NCELL <= kZ1Threads && ZY * ZX == (kZ1Threads / 64) * 16, "one slab cell per thread");
    static_assert((NWB + NW1S) * sizeof(bf16x8) <= NWT * sizeof(float), "layer 1's operands fit after layer 2's");
    __shared__ __attribute__((aligned(16))) bf16x8 s_v[3 * NCELL];
    __shared__ bf16x8 s_w[NW1S];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    for (int k = tid; k < NW1S; k += kZ1Threads) s_w[k] = wb[k];
    const int tiles_x = (G + ZX - 1) / ZX, tiles_y = (G + ZY - 1) / ZY;
    const int64_t b = blockIdx.x;
    const int tx0 = (int)(b % tiles_x) * ZX, ty0 = (int)((b / tiles_x) % tiles_y) * ZY;
    const int z0 = (int)(b / ((int64_t)tiles_x * tiles_y)) * ZP;
    const int z1 = min(z0 + ZP, G);
    const int64_t GG = (int64_t)G * G, n = GG * G;
    const int r = wave >> 1, h = wave & 1;

    bf16x8 pf;
    auto fetch = [&](int p) {  // thread tid < NCELL: its slab cell of plane p (zero outside the grid)
        float v[3] = { 0.f, 0.f, 0.f };
        if (tid < NCELL) {
            const int gy = ty0 + tid / ZSX - 1, gx = tx0 + tid % ZSX - 1;
            if (p >= 0 && p < G && gy >= 0 && gy < G && gx >= 0 && gx < G) {
                const int64_t c = (int64_t)p * GG + (int64_t)gy * G + gx;
                v[0] = vel[c];
                v[1] = vel[n + c];
                v[2] = vel[2 * n + c];
            }
        }
        pf = bf16x8{ 0, 0, 0, 0, 0, 0, 0, 0 };
#pragma unroll
        for (int ci = 0; ci < CIO; ++ci) {
            const bf16 hi = (bf16)v[ci];
            pf[ci] = hi;
            pf[3 + ci] = (bf16)(v[ci] - (float)hi);
        }
    };
    auto stash = [&](int p) {
        if (tid < NCELL) s_v[((p + 3) % 3) * NCELL + tid] = pf;
    };
    fetch(z0 - 1);
    stash(z0 - 1);
    fetch(z0);
    stash(z0);
    fetch(z0 + 1);
    stash(z0 + 1);
    __syncthreads();
    const v4f bl0 = *reinterpret_cast<const v4f*>(bias + 4 * grp);
    const v4f bl1 = *reinterpret_cast<const v4f*>(bias + 16 + 4 * grp);
    const int cell0 = r * ZSX + 16 * h + col;
    for (int z = z0; z < z1; ++z) {
        if (z + 2 < z1 + 1) fetch(z + 2);
        v4f acc0 = bl0, acc1 = bl1;
#pragma unroll
        for (int st = 0; st < 14; ++st) {
            int t = 2 * st + (grp >> 1);
            t = t < TAPS ? t : 13;  // zero weights: any finite operand serves
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
            const bf16x8 a = s_v[((z + dz - 1 + 3) % 3) * NCELL + cell0 + dy * ZSX + dx];
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[(st * 2) * 64 + lane], a, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(s_w[(st * 2 + 1) * 64 + lane], a, acc1, 0, 0, 0);
        }
        const int gy = ty0 + r, gx = tx0 + 16 * h + col;
        if (gy < G && gx < G) {
            bf16* dst = out + ((int64_t)z * GG + (int64_t)gy * G + gx) * C + 4 * grp;
            const v4f v0{ fmaxf(acc0.x, 0.f), fmaxf(acc0.y, 0.f), fmaxf(acc0.z, 0.f), fmaxf(acc0.w, 0.f) };
            const v4f v1{ fmaxf(acc1.x, 0.f), fmaxf(acc1.y, 0.f), fmaxf(acc1.z, 0.f), fmaxf(acc1.w, 0.f) };
            *reinterpret_cast<bf16x4*>(dst) = __builtin_convertvector(v0, bf16x4);
            *reinterpret_cast<bf16x4*>(dst + 16) = __builtin_convertvector(v1, bf16x4);
        }
        __syncthreads();
        if (z + 2 < z1 + 1) stash(z + 2);
        __syncthreads();
    }
}

// Layer 4 of the FP32 pass (32 -> 3) as a z-sweep on the vector ALUs: a block owns a column of
// Z4Y x Z4X cells (one per thread) and Z4P output planes, and reads each input plane once, as one
// slab with its one-cell border in LDS.  An input plane p feeds output planes p + 1, p and p - 1
// (kernel depth index 0, 1, 2), so a thread keeps the partial sums of three output planes; after
// plane p, output plane p - 1 is complete and written.  The weights are uniform across the block
// (scalar loads); the next plane's slab is loaded into registers while this one is used.
constexpr int Z4Y = 8, Z4X = 64, Z4P = 16;
constexpr int Z4SY = Z4Y + 2, Z4SX = Z4X + 2;
constexpr int Z4CS = C + 4;  // floats per slab cell (32 channels + 4 pad)
constexpr int kZ4Threads = Z4Y * Z4X;
constexpr int Z4CHUNKS = Z4SY * Z4SX * (C / 4);
constexpr int Z4CH_PER_THREAD = (Z4CHUNKS + kZ4Threads - 1) / kZ4Threads;

// w4t[(t9 * C + ci) * 9 + d * 3 + o] = W4[o][ci][d * 9 + t9]: for one (dy, dx) the 288 weights
// of all channels, depths and outputs are contiguous (scalar loads of whole lines)
__global__ void k3c_wprep4_f32(const float* __restrict__ w, float* __restrict__ w4t)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= TAPS * C * CIO) return;
    const int o = k % 3, d = (k / 3) % 3, ci = (k / 9) % C, t9 = k / (9 * C);
    w4t[k] = w[(o * C + ci) * TAPS + d * 9 + t9];
}

__global__ __launch_bounds__(kZ4Threads) void k3c_zconv4_f32(int32_t G, const float* __restrict__ in,
                                                              const float* __restrict__ w,
                                                              const float* __restrict__ bias, float* __restrict__ disp)
{
    __shared__ __attribute__((aligned(16))) float s_a[Z4SY * Z4SX * Z4CS];
    const int tid = threadIdx.x;
    const int tiles_x = (G + Z4X - 1) / Z4X, tiles_y = (G + Z4Y - 1) / Z4Y;
    const int64_t b = blockIdx.x;
    const int tx0 = (int)(b % tiles_x) * Z4X, ty0 = (int)((b / tiles_x) % tiles_y) * Z4Y;
    const int z0 = (int)(b / ((int64_t)tiles_x * tiles_y)) * Z4P;
    const int z1 = min(z0 + Z4P, G);
    const int64_t GG = (int64_t)G * G, n = GG * G;
    const int r = tid / Z4X, c = tid % Z4X;
    const int gy = ty0 + r, gx = tx0 + c;
    const float b0 = bias[0], b1 = bias[1], b2 = bias[2];

    v4f pf[Z4CH_PER_THREAD];
    auto fetch = [&](int p) {
#pragma unroll
        for (int k = 0; k < Z4CH_PER_THREAD; ++k) {
            const int e = tid + k * kZ4Threads;
            v4f v{ 0.f, 0.f, 0.f, 0.f };
            if (e < Z4CHUNKS) {
                const int cell = e / (C / 4), part = e % (C / 4);
                const int y = ty0 + cell / Z4SX - 1, x = tx0 + cell % Z4SX - 1;
                if (p >= 0 && p < G && y >= 0 && y < G && x >= 0 && x < G)
                    v = *reinterpret_cast<const v4f*>(in + ((int64_t)p * GG + (int64_t)y * G + x) * C + 4 * part);
            }
            pf[k] = v;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int k = 0; k < Z4CH_PER_THREAD; ++k) {
            const int e = tid + k * kZ4Threads;
            if (e < Z4CHUNKS) *reinterpret_cast<v4f*>(s_a + (e / (C / 4)) * Z4CS + 4 * (e % (C / 4))) = pf[k];
        }
    };
    // acc[d][o]: output plane p + 1 - d, component o
    float acc[3][CIO];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int o = 0; o < CIO; ++o) acc[d][o] = 0.f;
    fetch(z0 - 1);
    for (int p = z0 - 1; p <= z1; ++p) {
        __syncthreads();  // every thread is done with the previous plane's slab
        stash();
        __syncthreads();
        if (p + 1 <= z1) fetch(p + 1);  // lands while this plane is used
#pragma unroll 1
        for (int t9 = 0; t9 < 9; ++t9) {
            const int dy = t9 / 3, dx = t9 % 3;
            const v4f* a4 = reinterpret_cast<const v4f*>(s_a + ((r + dy) * Z4SX + c + dx) * Z4CS);
#pragma unroll 2
            for (int q = 0; q < C / 4; ++q) {
                const v4f a = a4[q];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int ci = 4 * q + j;
#pragma unroll
                    for (int d = 0; d < 3; ++d)
#pragma unroll
                        for (int o = 0; o < CIO; ++o) acc[d][o] += w[(t9 * C + ci) * 9 + d * 3 + o] * a[j];
                }
            }
        }
        const int zo = p - 1;  // complete now: its last input plane was p
        if (zo >= z0 && zo < z1 && gy < G && gx < G) {
            const int64_t cell = (int64_t)zo * GG + (int64_t)gy * G + gx;
            disp[cell] = acc[2][0] + b0;
            disp[n + cell] = acc[2][1] + b1;
            disp[2 * n + cell] = acc[2][2] + b2;
        }
#pragma unroll
        for (int o = 0; o < CIO; ++o) {
            acc[2][o] = acc[1][o];
            acc[1][o] = acc[0][o];
            acc[0][o] = 0.f;
        }
    }
}

}  // namespace

size_t cnn3_workspace_bytes(int32_t G)
{
    const size_t cells = (size_t)G * G * G;
    return 2 * cells * C * sizeof(float) + 2 * (size_t)NWT * sizeof(float) + (size_t)TAPS * C * CIO * sizeof(float);
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
    const int64_t zblocks = (int64_t)((G + ZX - 1) / ZX) * ((G + ZY - 1) / ZY) * ((G + ZP - 1) / ZP);
    if (zblocks > (int64_t)UINT32_MAX) fail(CNNSNS_EINVAL, "predict3d: overlay too large");
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
        bf16x8* wb1 = wb2 + NWB;  // after layer 2's operands in their 108 KiB region
        k3c_wprep1_split<<<(NW1S + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[0], wb1);
        k3c_zconv1_split<<<(unsigned)zblocks, kZ1Threads, 0, stream>>>(G, vel, wb1, w.b[0], b0);
        k3c_zsweep_bf16<2><<<(unsigned)zblocks, kZThreads, 0, stream>>>(G, b0, wb2, w.b[1], b1, nullptr);
        k3c_zsweep_bf16<2><<<(unsigned)zblocks, kZThreads, 0, stream>>>(G, b1, wb3, w.b[2], b0, nullptr);
        bf16x8* wb4 = wb3 + NWB;
        k3c_wprep4_bf16<<<(TAPS * 64 + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[3], wb4);
        k3c_zsweep_bf16<1><<<(unsigned)zblocks, kZThreads, 0, stream>>>(G, b0, wb4, w.b[3], nullptr, disp);
    } else {
        k3c_wprep<<<(NWT + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[1], wt2);
        k3c_wprep<<<(NWT + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[2], wt3);
        k3c_zconv1<float><<<(unsigned)zblocks, kZ1Threads, 0, stream>>>(G, vel, w.w[0], w.b[0], act0);
        k3c_conv32<<<grid, kWaves32 * 64, 0, stream>>>(G, act0, wt2, w.b[1], act1);
        k3c_conv32<<<grid, kWaves32 * 64, 0, stream>>>(G, act1, wt3, w.b[2], act0);
        const int64_t z4blocks = (int64_t)((G + Z4X - 1) / Z4X) * ((G + Z4Y - 1) / Z4Y) * ((G + Z4P - 1) / Z4P);
        if (z4blocks > (int64_t)UINT32_MAX) fail(CNNSNS_EINVAL, "predict3d: overlay too large");
        float* w4t = wt3 + NWT;
        k3c_wprep4_f32<<<(TAPS * C * CIO + kBlock - 1) / kBlock, kBlock, 0, stream>>>(w.w[3], w4t);
        k3c_zconv4_f32<<<(unsigned)z4blocks, kZ4Threads, 0, stream>>>(G, act0, w4t, w.b[3], disp);
    }
    hip_check(hipGetLastError(), "predict3d launch");
    workspace_used(m.ws, stream);
}

}  // namespace cnnsns
