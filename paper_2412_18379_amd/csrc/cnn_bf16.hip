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
// padded to one K = 32 step, its K ordered tap-major so that a lane's operand
// is four (u, v) pairs read straight from LDS; conv4 (N = 2) computes, per
// conv3 pixel, its 18 (output channel, tap) contributions (two N-blocks of one
// K = 32 instruction each) into the conv2 buffer, free by then, and sums 9
// taps per output pixel.  Biases
// enter as the accumulators' initial values, and ReLU acts on the rounded
// BF16 pair (rounding to nearest keeps the sign, so the order of the two does
// not change the result).
#include "common.h"

namespace cnnsns {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;  // 8 wavefronts, two per SIMD
constexpr int kWaves = kThreads / 64;
constexpr int C = 32;
constexpr int OH = 14, OW = 30;            // output tile
constexpr int H1 = OH + 6, W1 = OW + 6;    // conv1 region (20 x 36)
constexpr int H2 = OH + 4, W2 = OW + 4;    // conv2 region (18 x 34)
constexpr int H3 = OH + 2, W3 = OW + 2;    // conv3 region (16 x 32)
constexpr int HV = OH + 8, WV = OW + 8;    // velocity tile (22 x 38)
// bf16 per pixel of the conv1 and conv3 outputs (96 bytes) and of the conv2 output (80 bytes).  The
// LDS serves a 16-byte read in groups of 16 lanes over 64 four-byte banks, a group joining lanes 0-7
// with 56-63 (8-15 with 48-55, ...): for the operand reads, eight consecutive pixels at one channel
// chunk and eight others at the mirrored chunk.  At a 96-byte pitch those reads fall in distinct bank
// groups; at 80 bytes half of them collide.  The LDS holds only one of the two layer buffers at 96:
// it goes to conv2's input, the layer with the more operand reads per tile.  conv3 reads the 80-byte
// buffer conflict-free all the same: its M-blocks take every second pixel of a 32-pixel row (one
// block the even pixels, the next the odd ones), so at a 5-slot pitch all 16 pixels of a block sit in
// 16-byte slots of one parity and the mirrored chunk (3 slots on) in the other.
constexpr int PXS = 48;
constexpr int PXS2 = 40;
constexpr int VEL_PER_THREAD = (HV * WV + kThreads - 1) / kThreads;  // velocity pixels per thread
// M-blocks of 16 pixels per wavefront, and how many of them are in flight at once
constexpr int NMB1 = H1 * W1 / 16, BPW1 = (NMB1 + kWaves - 1) / kWaves, MB1 = BPW1;
constexpr int NMB2 = (H2 * W2 + 15) / 16, BPW2 = (NMB2 + kWaves - 1) / kWaves, MB2 = BPW2;
constexpr int NMB3 = H3 * W3 / 16, BPW3 = NMB3 / kWaves, MB3 = BPW3;
static_assert(H1 * W1 % 16 == 0 && H3 * W3 % 16 == 0 && NMB3 % kWaves == 0, "whole M-blocks");
static_assert(BPW1 % MB1 == 0 && BPW2 % MB2 == 0 && BPW3 % MB3 == 0, "whole groups per wavefront");

// Hidden activations are stored pair-interleaved: LDS position 2c + h of a
// pixel holds channel c + 16 h, so a lane that owns channels c and c + 16 of
// the matrix-core result writes them with one packed 32-bit store.
__device__ __forceinline__ int chan_at(int pos)
{
    return (pos >> 1) + 16 * (pos & 1);
}

// packed weights, one bf16x8 B operand per lane:
//   w1p[nb][lane]: k = 8 (l/16) + j = 2 tap + ci (< 18, else 0) of output channel 16 nb + l%16
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
            v[j] = (bf16)(k < 18 ? w1[((nb * 16 + i) * 2 + (k & 1)) * 9 + (k >> 1)] : 0.f);
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

// Channels (i, 16 + i) of one pixel as a packed BF16 pair after ReLU: the
// pair is rounded to nearest even, then every half whose sign bit is set
// (negative, or -0) becomes +0, which is the integer maximum of the bit
// pattern with 0.  The result is ReLU of the rounded value, which equals the
// rounded ReLU.
__device__ __forceinline__ uint32_t relu_pair(float v0, float v1)
{
    const bf16x2 pk = __builtin_convertvector(f32x2{ v0, v1 }, bf16x2);
    const s16x2 r = __builtin_elementwise_max(__builtin_bit_cast(s16x2, pk), s16x2{ 0, 0 });
    return __builtin_bit_cast(uint32_t, r);
}

// Writes the 4 pixels (p0 .. p0 + 3 of an HO x WO region with grid origin
// (oy0, ox0)) that lane (i, q) holds after a layer's M-block: ReLU pairs, and
// zero for pixels outside the grid (the next layer's zero padding).
template <int WO, int OPXS, bool EDGE, int S = 1>
__device__ __forceinline__ void store_block(bf16* __restrict__ out, int p0, int i, const v4f& d0, const v4f& d1,
                                            int oy0, int ox0, int G)
{
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        uint32_t v = relu_pair(d0[r], d1[r]);
        const int p = p0 + S * r;
        if (EDGE) {
            const int gy = oy0 + p / WO, gx = ox0 + p % WO;
            if (!inside(gy, gx, G)) v = 0;
        }
        *reinterpret_cast<uint32_t*>(out + p * OPXS + 2 * i) = v;
    }
}

// One 32 -> 32 layer over an HO x WO region (output origin (oy0, ox0) in the
// grid) reading an (HO+2) x (WO+2) input region, all in LDS, pixel-major.
// Wavefront w takes the BPW M-blocks [w BPW, (w+1) BPW) and works through
// them MB at a time; the A and B operands of the next two taps are read while
// the matrix instructions of the current one issue.  STRIDE2: block 2k + e holds
// pixels 32k + e, 32k + e + 2, ..., 32k + e + 30 (rows of 32 pixels).  Blocks past the region's last one are
// computed on clamped pixels and not stored.
template <int HO, int WO, int IPXS, int OPXS, int BPW, int MB, bool EDGE, bool STRIDE2 = false>
__device__ __forceinline__ void conv32_bf16(const bf16* __restrict__ in, bf16* __restrict__ out,
                                            const bf16x8* __restrict__ sw, float blo, float bhi, int oy0, int ox0,
                                            int G, int wave, int lane)
{
    constexpr int WI = WO + 2, N = HO * WO, NMB = (N + 15) / 16;
    static_assert(!STRIDE2 || (WO == 32 && BPW % 2 == 0 && MB % 2 == 0 && N % 32 == 0),
                  "strided M-blocks pair up the two halves of one 32-pixel row");
    const int i = lane & 15, q = lane >> 4;
    int wl = lane;  // opaque to the compiler: the weights are read per tap, not held across calls
    asm volatile("" : "+v"(wl));
    // first block, opaque so that its addresses are recomputed per call, not held across tiles
    int g0 = wave * BPW;
    asm volatile("" : "+s"(g0));
#pragma unroll 1
    for (int g = g0; g < g0 + BPW; g += MB) {
        v4f acc[MB][2];
        int base[MB];
#pragma unroll
        for (int m = 0; m < MB; ++m) {
            const int p = STRIDE2 ? ((g + m) >> 1) * 32 + 2 * i + ((g + m) & 1) : min((g + m) * 16 + i, N - 1);
            base[m] = ((p / WO) * WI + p % WO) * IPXS + 8 * q;
            acc[m][0] = v4f{ blo, blo, blo, blo };
            acc[m][1] = v4f{ bhi, bhi, bhi, bhi };
        }
        // operands (and weights) of taps t+1 and t+2 are in flight while tap t's instructions issue
        constexpr int PF = 2;
        static_assert(PF * (MB + 2) <= 15, "outstanding LDS reads fit the wait counter");
        auto tap_off = [](int t) { return ((t / 3) * WI + t % 3) * IPXS; };
        bf16x8 a[PF + 1][MB], w[PF + 1][2];
        auto fetch = [&](int t, int slot) {
#pragma unroll
            for (int m = 0; m < MB; ++m) a[slot][m] = *reinterpret_cast<const bf16x8*>(in + base[m] + tap_off(t));
            w[slot][0] = sw[(t * 2) * 64 + wl];
            w[slot][1] = sw[(t * 2 + 1) * 64 + wl];
        };
#pragma unroll
        for (int t = 0; t < PF; ++t) fetch(t, t);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int cur = t % (PF + 1);
            if (t + PF < 9) fetch(t + PF, (t + PF) % (PF + 1));
            // keep the reads ahead of the instructions (the scheduler would sink them to their use)
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int m = 0; m < MB; ++m) {
                acc[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cur][m], w[cur][0], acc[m][0], 0, 0, 0);
                acc[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[cur][m], w[cur][1], acc[m][1], 0, 0, 0);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // result: lane (i, q) holds region pixels (g + m) 16 + 4q + r, channels i and 16 + i
#pragma unroll
        for (int m = 0; m < MB; ++m)
            if (NMB == BPW * kWaves || g + m < NMB)
            {
                if (STRIDE2)
                    store_block<WO, OPXS, EDGE, 2>(out, ((g + m) >> 1) * 32 + 8 * q + ((g + m) & 1), i, acc[m][0],
                                                   acc[m][1], oy0, ox0, G);
                else
                    store_block<WO, OPXS, EDGE>(out, (g + m) * 16 + 4 * q, i, acc[m][0], acc[m][1], oy0, ox0, G);
            }
    }
}

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_cnn_bf16(
    int32_t G, int tiles_x, int ntiles, const float* __restrict__ vel, const bf16x8* __restrict__ packed,
    const float* __restrict__ b1, const float* __restrict__ b2, const float* __restrict__ b3,
    const float* __restrict__ b4, float* __restrict__ disp)
{
    __shared__ __attribute__((aligned(16))) bf16 bufA[H1 * W1 * PXS];  // conv1 out, then conv3 out
    static_assert(H1 * W1 >= NMB3 * 16, "conv3 output fits in bufA");
    // conv2 out, padded to the last stored M-block
    __shared__ __attribute__((aligned(16))) bf16 bufB[NMB2 * 16 * PXS2];
    __shared__ uint32_t s_vel[HV * WV];  // (u, v) of each velocity pixel as a packed BF16 pair
    __shared__ bf16x8 s_w1[P1];
    __shared__ bf16x8 s_w4[P4];
    __shared__ bf16x8 s_w23[2 * P2];  // conv2 then conv3: [layer][tap][nb][lane]

    const int tid = threadIdx.x, lane = tid & 63, i = lane & 15, q = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: block ranges stay scalar
    const int64_t GG = (int64_t)G * G;

    TileIter it(ntiles);
    if (it.t >= it.end) return;

    for (int k = tid; k < P1; k += kThreads) s_w1[k] = packed[k];
    for (int k = tid; k < P4; k += kThreads) s_w4[k] = packed[P1 + 2 * P2 + k];
    for (int k = tid; k < 2 * P2; k += kThreads) s_w23[k] = packed[P1 + k];
    // the bias of the lane's two output channels (i, 16 + i) in each hidden layer
    const float b1lo = b1[i], b1hi = b1[16 + i], b2lo = b2[i], b2hi = b2[16 + i], b3lo = b3[i], b3hi = b3[16 + i];
    const float b40 = b4[0], b41 = b4[1];

    // conv1 operand: slots j = 2 jj + ci of lane group q hold channel ci of tap 4q + jj, so the
    // lane reads the packed (u, v) pair of four taps; taps past 8 meet zero weights and read the
    // pixel itself (any finite value gives the same result)
    int l1_off[4];
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
        const int t = 4 * q + jj;
        l1_off[jj] = t < 9 ? (t / 3) * WV + t % 3 : 0;
    }

    // The next tile's velocity is loaded unconditionally, from clamped (valid) positions, and what
    // lies outside the grid is zeroed when it is stashed: with no branch between the loads and their
    // use, the compiled code waits for them at the stash and not before conv2's first matrix
    // instruction (which a register shared with a pending load had made it do).
    float pu[VEL_PER_THREAD], pw[VEL_PER_THREAD];
    bool pin[VEL_PER_THREAD];
    auto fetch_vel = [&](int t) {
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
            if (e < HV * WV) s_vel[e] = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{ u, v }, bf16x2));
        }
    };
    // conv1 of tile t on its 20 x 36 region into bufA: K = 18 (9 taps x 2 channels) padded to 32
    auto conv1 = [&](int t) {
        const int ty0 = (t / tiles_x) * OH, tx0 = (t % tiles_x) * OW;
        // tiles whose velocity halo lies inside the grid need no zero-padding tests
        const bool edge = ty0 < 4 || tx0 < 4 || ty0 + OH + 4 > G || tx0 + OW + 4 > G;
        int g1 = wave * BPW1;  // opaque, as in conv32_bf16
        asm volatile("" : "+s"(g1));
#pragma unroll 1
        for (int g = g1; g < g1 + BPW1; g += MB1) {
            // MB1 M-blocks at once: all reads issue before the first matrix instruction
            bf16x8 a[MB1];
#pragma unroll
            for (int m = 0; m < MB1; ++m) {
                const int p = min((g + m) * 16 + i, H1 * W1 - 1);
                const int pbase = (p / W1) * WV + p % W1;
                u32x4 v;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) v[jj] = s_vel[pbase + l1_off[jj]];
                a[m] = __builtin_bit_cast(bf16x8, v);
            }
            const bf16x8 w1lo = s_w1[lane], w1hi = s_w1[64 + lane];
            // every block's instructions issue before the first result is read back
            v4f d[MB1][2];
#pragma unroll
            for (int m = 0; m < MB1; ++m) {
                d[m][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], w1lo, v4f{ b1lo, b1lo, b1lo, b1lo }, 0, 0, 0);
                d[m][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], w1hi, v4f{ b1hi, b1hi, b1hi, b1hi }, 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < MB1; ++m) {
                if (NMB1 == BPW1 * kWaves || g + m < NMB1) {
                    if (edge)
                        store_block<W1, PXS, true>(bufA, (g + m) * 16 + 4 * q, i, d[m][0], d[m][1], ty0 - 3, tx0 - 3,
                                                   G);
                    else
                        store_block<W1, PXS, false>(bufA, (g + m) * 16 + 4 * q, i, d[m][0], d[m][1], 0, 0, G);
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

        // tiles whose velocity halo lies inside the grid need no zero-padding tests
        const bool edge = ty0 < 4 || tx0 < 4 || ty0 + OH + 4 > G || tx0 + OW + 4 > G;

        const int next = it.t + it.step;
        fetch_vel(next < it.end ? next : it.t);  // lands while conv2-conv4 run (after the last tile: unused)

        if (edge)
            conv32_bf16<H2, W2, PXS, PXS2, BPW2, MB2, true>(bufA, bufB, s_w23, b2lo, b2hi, ty0 - 2, tx0 - 2, G, wave,
                                                            lane);
        else
            conv32_bf16<H2, W2, PXS, PXS2, BPW2, MB2, false>(bufA, bufB, s_w23, b2lo, b2hi, ty0 - 2, tx0 - 2, G, wave,
                                                             lane);
        __syncthreads();
        stash_vel();
        if (edge)
            conv32_bf16<H3, W3, PXS2, PXS, BPW3, MB3, true, true>(bufB, bufA, s_w23 + P2, b3lo, b3hi, ty0 - 1, tx0 - 1, G,
                                                            wave, lane);
        else
            conv32_bf16<H3, W3, PXS2, PXS, BPW3, MB3, false, true>(bufB, bufA, s_w23 + P2, b3lo, b3hi, ty0 - 1, tx0 - 1, G,
                                                             wave, lane);
        __syncthreads();

        // conv4 as a contraction: for every pixel p of the 16 x 32 conv3 region,
        // Z[9 o + t][p] = sum_c act3[p][c] w4[o][c][t] (one K = 32 instruction per 16 pixels and
        // N-block), in FP32, column-major in the conv2 buffer (no longer read): a lane's four
        // results are four consecutive pixels of one column, one 16-byte store.  Then each output
        // pixel sums its 9 taps; the lanes of a wavefront read consecutive pixels of one column,
        // and the column stride (532 floats) spreads a store's 16 columns over distinct banks.
        {
            constexpr int ZC = 532;
            static_assert(18 * ZC * sizeof(float) <= sizeof(bufB) && ZC >= H3 * W3 && ZC % 4 == 0, "Z fits");
            float* zb = reinterpret_cast<float*>(bufB);
            for (int mb = wave; mb < NMB3; mb += kWaves) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(bufA + (mb * 16 + i) * PXS + 8 * q);
                const v4f z0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, s_w4[lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0, 0, 0);
                const v4f z1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, s_w4[64 + lane], v4f{ 0.f, 0.f, 0.f, 0.f }, 0,
                                                                       0, 0);
                *reinterpret_cast<v4f*>(zb + i * ZC + mb * 16 + 4 * q) = z0;
                if (i < 2) *reinterpret_cast<v4f*>(zb + (16 + i) * ZC + mb * 16 + 4 * q) = z1;
            }
            __syncthreads();
            for (int e = tid; e < OH * OW; e += kThreads) {
                const int oy = e / OW, ox = e - oy * OW;
                const float* zp = zb + oy * W3 + ox;
                float d0 = b40, d1 = b41;
#pragma unroll
                for (int t = 0; t < 9; ++t) {
                    d0 += zp[t * ZC + (t / 3) * W3 + t % 3];
                    d1 += zp[(9 + t) * ZC + (t / 3) * W3 + t % 3];
                }
                const int gy = ty0 + oy, gx = tx0 + ox;
                if (gy < G && gx < G) {
                    disp[(int64_t)gy * G + gx] = d0;
                    disp[GG + (int64_t)gy * G + gx] = d1;
                }
            }
        }
        // the next tile's conv1 in the same phase: bufA (this tile's conv3 output) was last read
        // before the barrier above, the tap sums read only the conv2 buffer, and the next
        // tile's velocity was stashed after conv2
        if (next < it.end) conv1(next);
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
