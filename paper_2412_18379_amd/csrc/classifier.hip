// The paper's classifier CNN (Sec. 2.3, eq. 7-8): the prediction step of
// Alg. 2 as a per-particle multiclass classification, in 2D on the overlay.
//
// Input preparation (Sec. 2.3).  Elements are represented by their centroids
// (vertices summed in ascending node id, then divided by 3); the ASG filter
// assigns each element to the overlay cell holding its centroid, and average
// pooling gives every cell the mean of its elements' centroids (summed in
// ascending element id), or the cell centre when it has none.  This grid is
// built once per mesh.  For a point x_p the filtered region is the 9 x 9 block
// of cells centred on the cell of x_p, extended at the grid boundary by the
// nearest cell (the padding layer); its input is G (pooled centroid - x_p) per
// cell, and x_p's own offset in its cell, x_p G - (cell + 1/2).  Both are
// formed in FP64 and rounded to FP32.
//
// Network (FP32 weights in PyTorch layouts): module 1, conv 3x3 2 -> 16, ReLU,
// conv 3x3 16 -> 16, ReLU, 2 x 2 average pooling (4 x 4, flattened
// [channel][row][col]); module 2, FC 2 -> 256, ReLU, FC 256 -> 256, ReLU; then
// FC 512 -> 512, ReLU, and FC 512 -> 81: the logits.  The class is the argmax
// of the logits (the softmax of eq. 7 is monotone, so it has the same
// argmax), the lowest class on ties; class (dy + 4) 9 + (dx + 4) is the window
// cell at offset (dx, dy) and K_p is that cell's overlay lookup element.
//
// On the GPU: one wavefront per particle for module 1 (window gather and
// conv1 on the vector ALUs, conv2 on v_mfma_f32_16x16x4f32 with K ordered
// tap-major, pooling) and module 2's first layer; the three wide FC layers as
// batched FP32 matrix products over a chunk of particles
// (v_mfma_f32_16x16x4f32, 64 x 64 output tiles); then the argmax and start.
#pragma clang fp contract(off)

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace cnnsns {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kW = 9, kR = 4, kNA = kW * kW;  // window side, radius, classes
constexpr int kC = 16;                         // conv channels
constexpr int kPW = kW + 2;                    // the window with a one-cell zero border (conv padding)
constexpr int kNF = kC * 4 * 4;                // module 1 features (256)
constexpr int kH1 = 256, kH2 = 512, kNZ = kNF + kH1;
constexpr int kBlock = 256;
constexpr int64_t kChunk = 65536;  // particles per pass of the fully connected layers

__device__ __forceinline__ int32_t cell_of(double x, int32_t G)
{
    const double f = floor(x * (double)G);
    if (!(f >= 0.0)) return 0;  // negative or NaN
    if (f > (double)(G - 1)) return G - 1;
    return (int32_t)f;
}

__device__ __forceinline__ int32_t clamp_cell(int32_t c, int32_t G)
{
    return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

// centroid of element t with its vertices summed in ascending node id
__device__ __forceinline__ void centroid_by_id(const ElemRec* __restrict__ rec, const int32_t* __restrict__ tri,
                                               int64_t t, double& x, double& y)
{
    const ElemRec r = rec[t];
    int32_t id[3] = { tri[3 * t], tri[3 * t + 1], tri[3 * t + 2] };
    double px[3] = { r.ax, r.bx, r.cx }, py[3] = { r.ay, r.by, r.cy };
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2 - i; ++j)
            if (id[j] > id[j + 1]) {
                const int32_t s = id[j];
                id[j] = id[j + 1];
                id[j + 1] = s;
                const double sx = px[j], sy = py[j];
                px[j] = px[j + 1];
                py[j] = py[j + 1];
                px[j + 1] = sx;
                py[j + 1] = sy;
            }
    x = ((px[0] + px[1]) + px[2]) / 3.0;
    y = ((py[0] + py[1]) + py[2]) / 3.0;
}

// pass 1 of the pooled grid: each element's cell (the sort key) and the cell counts
__global__ void k_pool_cells(int64_t n_tri, const ElemRec* __restrict__ rec, const int32_t* __restrict__ tri,
                             int32_t G, uint32_t* __restrict__ key, int32_t* __restrict__ val,
                             uint32_t* __restrict__ count)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tri) return;
    double x, y;
    centroid_by_id(rec, tri, t, x, y);
    const uint32_t c = (uint32_t)cell_of(y, G) * (uint32_t)G + (uint32_t)cell_of(x, G);
    key[t] = c;
    val[t] = (int32_t)t;
    atomicAdd(&count[c], 1u);
}

// pass 2: per cell, the mean of its elements' centroids in ascending element id (the stable sort keeps the
// ids of a cell ascending), or the cell centre
__global__ void k_pool_mean(int32_t G, const ElemRec* __restrict__ rec, const int32_t* __restrict__ tri,
                            const int32_t* __restrict__ sorted, const uint32_t* __restrict__ first,
                            const uint32_t* __restrict__ count, double2* __restrict__ pool)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)G * G) return;
    const uint32_t k0 = first[c], k = count[c];
    double2 p;
    if (k == 0) {
        p.x = ((double)(c % G) + 0.5) / (double)G;
        p.y = ((double)(c / G) + 0.5) / (double)G;
    } else {
        double sx = 0.0, sy = 0.0;
        for (uint32_t q = 0; q < k; ++q) {
            double x, y;
            centroid_by_id(rec, tri, sorted[k0 + q], x, y);
            sx += x;
            sy += y;
        }
        p.x = sx / (double)k;
        p.y = sy / (double)k;
    }
    pool[c] = p;
}

// Module 1 (window, conv1, conv2, pooling) and module 2's first layer, one wavefront per particle at a time
// (persistent blocks loop over the particles with the weights staged once): writes
// z[i][0 .. 255] and m1[i][0 .. 255] (row strides ldz, ldm).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_cls_module1(
    int64_t n, const double2* __restrict__ xp, int32_t G, const double2* __restrict__ pool,
    const float* __restrict__ w1, const float* __restrict__ b1, const float* __restrict__ w2,
    const float* __restrict__ b2, const float* __restrict__ wx1, const float* __restrict__ bx1,
    float* __restrict__ z, int ldz, float* __restrict__ m1, int ldm)
{
    constexpr int kWaves = kBlock / 64;
    __shared__ float s_w1[kC * 2 * 9], s_b1[kC], s_b2[kC];
    __shared__ float s_w2[9][kC][kC + 1];  // [tap][in channel][out channel], padded
    __shared__ float s_in[kWaves][2][kPW * kPW];
    // conv1's output on the bordered window; conv2's output goes to its interior once conv2 has read it
    __shared__ float s_a1[kWaves][kPW * kPW][kC + 1];
    __shared__ float s_x1[kH1][3];  // module 2's first layer: (w0, w1, bias) per output

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k < kC * 2 * 9; k += kBlock) s_w1[k] = w1[k];
    for (int k = tid; k < kC * kC * 9; k += kBlock) {
        const int o = k / (kC * 9), i = (k / 9) % kC, t = k % 9;  // PyTorch [out][in][3][3]
        s_w2[t][i][o] = w2[k];
    }
    if (tid < kC) {
        s_b1[tid] = b1[tid];
        s_b2[tid] = b2[tid];
    }
    for (int j = tid; j < kH1; j += kBlock) {
        s_x1[j][0] = wx1[2 * j];
        s_x1[j][1] = wx1[2 * j + 1];
        s_x1[j][2] = bx1[j];
    }
    float* in = &s_in[wave][0][0];
    for (int k = lane; k < 2 * kPW * kPW; k += 64) in[k] = 0.f;
    for (int k = lane; k < kPW * kPW * (kC + 1); k += 64) (&s_a1[wave][0][0])[k] = 0.f;
    __syncthreads();  // the weights and the zero borders, which no point's writes touch
    // a wavefront takes points i, i + the grid's wavefront count, ...: its window, conv1 output and
    // conv2 output are its own LDS regions, so only the wavefront's own accesses need ordering
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    };
    const int row = lane & 15, kq = lane >> 4;
    int base[6];
#pragma unroll
    for (int mb = 0; mb < 6; ++mb) {
        const int px = min(mb * 16 + row, kNA - 1), r = px / kW, c = px % kW;
        base[mb] = r * kPW + c;  // top-left tap in the bordered window
    }
    // conv1's B operands: lane (row, kq) supplies output channel `row` at k = 4 st + kq = 9 ci + tap
    float w1k[5];
#pragma unroll
    for (int st = 0; st < 5; ++st) {
        const int k = 4 * st + kq;
        w1k[st] = k < 18 ? s_w1[(row * 2 + k / 9) * 9 + k % 9] : 0.f;
    }
    // the window's pooled values of the wavefront's next particle are gathered into registers while
    // the current one computes (lane o holds window cells o and o + 64)
    const int64_t stride = (int64_t)gridDim.x * kWaves;
    double2 pn = double2{ 0.0, 0.0 };
    double2 qn[2] = { double2{ 0.0, 0.0 }, double2{ 0.0, 0.0 } };
    auto gather = [&](int64_t k) {
        pn = xp[k];
        const int32_t gx = cell_of(pn.x, G), gy = cell_of(pn.y, G);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int o = lane + 64 * u;
            if (o < kNA) {
                const int dy = o / kW - kR, dx = o % kW - kR;
                qn[u] = pool[(int64_t)clamp_cell(gy + dy, G) * G + clamp_cell(gx + dx, G)];
            }
        }
    };
    int64_t i = (int64_t)blockIdx.x * kWaves + wave;
    if (i < n) gather(i);
    for (; i < n; i += stride) {
        const double2 p = pn;
        const int32_t cx = cell_of(p.x, G), cy = cell_of(p.y, G);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int o = lane + 64 * u;
            if (o < kNA) {
                const int dy = o / kW - kR, dx = o % kW - kR;
                const int at = (dy + kR + 1) * kPW + (dx + kR + 1);
                in[at] = (float)((qn[u].x - p.x) * (double)G);
                in[kPW * kPW + at] = (float)((qn[u].y - p.y) * (double)G);
            }
        }
        const float xo0 = (float)(p.x * (double)G - ((double)cx + 0.5));
        const float xo1 = (float)(p.y * (double)G - ((double)cy + 0.5));
        wave_sync();
        if (i + stride < n) gather(i + stride);
        // conv1 (2 -> 16) on the matrix cores: rows = pixels (6 blocks of 16, the last partly repeated),
        // columns = output channels, k = 9 channel + tap (18, padded to 20: five steps of 4)
        {
            v4f a1[6];
#pragma unroll
            for (int mb = 0; mb < 6; ++mb) a1[mb] = v4f{ 0.f, 0.f, 0.f, 0.f };
#pragma unroll
            for (int st = 0; st < 5; ++st) {
                const int k = 4 * st + kq, ci = k / 9, t = k % 9;
                const int off = ci * kPW * kPW + (t / 3) * kPW + t % 3;
#pragma unroll
                for (int mb = 0; mb < 6; ++mb) {
                    const float av = k < 18 ? in[base[mb] + off] : 0.f;
                    a1[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, w1k[st], a1[mb], 0, 0, 0);
                }
            }
            // lane holds pixels 16 mb + 4 kq + e of output channel `row`
#pragma unroll
            for (int mb = 0; mb < 6; ++mb)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int px = mb * 16 + 4 * kq + e;
                    if (px < kNA)
                        s_a1[wave][(px / kW + 1) * kPW + px % kW + 1][row] = fmaxf(a1[mb][e] + s_b1[row], 0.f);
                }
        }
        wave_sync();
        // conv2 (16 -> 16) on the matrix cores: rows = pixels (6 blocks of 16, the last partly
        // repeated), columns = output channels, k = 16 tap + input channel in 36 steps of 4
        v4f acc[6];
#pragma unroll
        for (int mb = 0; mb < 6; ++mb) acc[mb] = v4f{ 0.f, 0.f, 0.f, 0.f };
        for (int s = 0; s < 36; ++s) {
            const int t = s >> 2, ch = 4 * (s & 3) + kq;
            const int off = (t / 3) * kPW + t % 3;
            const float bw = s_w2[t][ch][row];
#pragma unroll
            for (int mb = 0; mb < 6; ++mb)
                acc[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(s_a1[wave][base[mb] + off][ch], bw, acc[mb], 0, 0, 0);
        }
        wave_sync();  // conv2 has read all of conv1's output
        // lane holds pixels 16 mb + 4 kq + e of output channel `row`: into the interior of the window
#pragma unroll
        for (int mb = 0; mb < 6; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int px = mb * 16 + 4 * kq + e;
                if (px < kNA) s_a1[wave][(px / kW + 1) * kPW + px % kW + 1][row] = fmaxf(acc[mb][e] + s_b2[row], 0.f);
            }
        wave_sync();
        // 2 x 2 average pooling, [channel][row][col] order
        for (int f = lane; f < kNF; f += 64) {
            const int ch = f >> 4, pr = (f >> 2) & 3, pc = f & 3;
            const int p0 = (2 * pr + 1) * kPW + 2 * pc + 1;
            const float q = ((s_a1[wave][p0][ch] + s_a1[wave][p0 + 1][ch]) + s_a1[wave][p0 + kPW][ch]) +
                            s_a1[wave][p0 + kPW + 1][ch];
            z[i * ldz + f] = q * 0.25f;
        }
        // module 2, first layer: FC 2 -> 256 on x_p's offset
        for (int j = lane; j < kH1; j += 64)
            m1[i * ldm + j] = fmaxf(s_x1[j][2] + s_x1[j][0] * xo0 + s_x1[j][1] * xo1, 0.f);
        wave_sync();  // the next point's window and conv1 output replace these
    }
}

// C[m][n] = act(bias[n] + sum_k A[m][k] W[n][k]) for m < M, n < N (W in [out][in] layout); K a multiple of 16,
// rows of A and W 16-byte aligned.  128 x 128 output tiles, four wavefronts of 64 x 64 each (4 x 4 blocks of
// v_mfma_f32_16x16x4f32, so each operand read from LDS feeds four instructions); the next 16-wide K slice
// is loaded into registers while this one's products issue.
constexpr int kDT = 128;  // dense tile side
template <bool RELU>
__global__ __launch_bounds__(kBlock) void k_dense_f32(int M, int N, int K, const float* __restrict__ A, int lda,
                                                      const float* __restrict__ Wt, const float* __restrict__ bias,
                                                      float* __restrict__ Cm, int ldc)
{
    __shared__ float sA[2][kDT][17], sB[2][kDT][17];
    const int m0 = blockIdx.x * kDT, n0 = blockIdx.y * kDT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int row = lane & 15, kq = lane >> 4;
    // the two float4 of each operand tile this thread stages: rows tid / 4 and tid / 4 + 64
    const int sr = tid >> 2, sc = (tid & 3) * 4;
    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{ 0.f, 0.f, 0.f, 0.f };
    auto fetch = [&](int k0, v4f (&va)[2], v4f (&vb)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = sr + 64 * h;
            va[h] = m0 + r < M ? *reinterpret_cast<const v4f*>(A + (int64_t)(m0 + r) * lda + k0 + sc)
                               : v4f{ 0.f, 0.f, 0.f, 0.f };
            vb[h] = n0 + r < N ? *reinterpret_cast<const v4f*>(Wt + (int64_t)(n0 + r) * K + k0 + sc)
                               : v4f{ 0.f, 0.f, 0.f, 0.f };
        }
    };
    auto stash = [&](int buf, const v4f (&va)[2], const v4f (&vb)[2]) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sA[buf][sr + 64 * h][sc + e] = va[h][e];
                sB[buf][sr + 64 * h][sc + e] = vb[h][e];
            }
    };
    v4f va[2], vb[2];
    fetch(0, va, vb);
    stash(0, va, vb);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        const bool more = k0 + 16 < K;
        if (more) fetch(k0 + 16, va, vb);  // lands while this slice's products issue
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            float a[4], b[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[x] = sA[buf][wm + 16 * x + row][kk + kq];
                b[x] = sB[buf][wn + 16 * x + row][kk + kq];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        if (more) stash(buf ^ 1, va, vb);
        __syncthreads();
        buf ^= 1;
    }
    // lane holds rows 4 kq + e of column `row` of each 16 x 16 block
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int n = n0 + wn + 16 * y + row;
            if (n >= N) continue;
            const float bn = bias[n];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wm + 16 * x + 4 * kq + e;
                if (m >= M) continue;
                float v = acc[x][y][e] + bn;
                if (RELU) v = fmaxf(v, 0.f);
                Cm[(int64_t)m * ldc + n] = v;
            }
        }
}

// The argmax of each particle's logits (the lowest class on ties) and its start element: the lookup element
// of that window cell, else the fallback start, else element 0.
__global__ void k_cls_argmax(int64_t n, const double2* __restrict__ xp, int32_t G, const int32_t* __restrict__ lookup,
                             const float* __restrict__ logits, int ldl, const int32_t* __restrict__ fallback,
                             int32_t* __restrict__ start, int32_t* __restrict__ cls)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float* h = logits + i * ldl;
    int best = 0;
    float hb = h[0];
    for (int l = 1; l < kNA; ++l) {
        const float v = h[l];
        if (v > hb) {
            hb = v;
            best = l;
        }
    }
    const double2 p = xp[i];
    const int32_t cx = clamp_cell(cell_of(p.x, G) + best % kW - kR, G);
    const int32_t cy = clamp_cell(cell_of(p.y, G) + best / kW - kR, G);
    int32_t k = lookup[(int64_t)cy * G + cx];
    if (k < 0) k = fallback ? fallback[i] : 0;
    start[i] = k;
    if (cls) cls[i] = best;
}

inline unsigned blocks_for(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

// The pooled grid of a mesh, built on its first classification.
void build_pool(cnnsns_mesh_s& m, hipStream_t stream)
{
    const int64_t nt = m.n_tri, GG = (int64_t)m.G * m.G;
    if (GG > (int64_t)UINT32_MAX || nt > (int64_t)UINT32_MAX) fail(CNNSNS_EINVAL, "classify: overlay too large");
    void* tmp = nullptr;
    auto dmalloc = [&](size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes ? bytes : 1) != hipSuccess) {
            (void)hipGetLastError();
            fail(CNNSNS_ENOMEM, "classify: pooled grid allocation of " + std::to_string(bytes) + " bytes");
        }
        return p;
    };
    struct Bufs {
        void* p[7] = {};
        ~Bufs()
        {
            for (void* q : p)
                if (q) (void)hipFree(q);
        }
    } b;
    auto* key = static_cast<uint32_t*>(b.p[0] = dmalloc(sizeof(uint32_t) * nt));
    auto* key2 = static_cast<uint32_t*>(b.p[1] = dmalloc(sizeof(uint32_t) * nt));
    auto* val = static_cast<int32_t*>(b.p[2] = dmalloc(sizeof(int32_t) * nt));
    auto* val2 = static_cast<int32_t*>(b.p[3] = dmalloc(sizeof(int32_t) * nt));
    auto* count = static_cast<uint32_t*>(b.p[4] = dmalloc(sizeof(uint32_t) * GG));
    auto* first = static_cast<uint32_t*>(b.p[5] = dmalloc(sizeof(uint32_t) * GG));
    auto* pool = static_cast<double2*>(dmalloc(sizeof(double2) * GG));
    try {
        hip_check(hipMemsetAsync(count, 0, sizeof(uint32_t) * GG, stream), "classify: pool counts");
        k_pool_cells<<<blocks_for(nt, kBlock), kBlock, 0, stream>>>(nt, m.rec, m.tri, m.G, key, val, count);
        int end_bit = 1;
        while (end_bit < 32 && ((uint64_t)1 << end_bit) < (uint64_t)GG) ++end_bit;
        size_t sort_bytes = 0, scan_bytes = 0;
        hip_check(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, key, key2, val, val2, (int)nt, 0, end_bit,
                                                     stream),
                  "classify: sort size");
        hip_check(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, count, first, (int)GG, stream),
                  "classify: scan size");
        tmp = b.p[6] = dmalloc(std::max(sort_bytes, scan_bytes));
        hip_check(hipcub::DeviceRadixSort::SortPairs(tmp, sort_bytes, key, key2, val, val2, (int)nt, 0, end_bit, stream),
                  "classify: sort");
        hip_check(hipcub::DeviceScan::ExclusiveSum(tmp, scan_bytes, count, first, (int)GG, stream), "classify: scan");
        k_pool_mean<<<blocks_for(GG, kBlock), kBlock, 0, stream>>>(m.G, m.rec, m.tri, val2, first, count, pool);
        hip_check(hipGetLastError(), "classify: pool kernels");
        hip_check(hipStreamSynchronize(stream), "classify: pooled grid");
    } catch (...) {
        (void)hipFree(pool);
        throw;
    }
    m.cls_pool = pool;
    m.device_bytes += (int64_t)(sizeof(double2) * GG);
}

}  // namespace

size_t cls_workspace_bytes(int64_t n)
{
    const int64_t ch = n < kChunk ? n : kChunk;
    return sizeof(float) * (size_t)ch * (size_t)(kNZ + kH2 + kNA);
}

void run_classify(cnnsns_mesh_s& m, int64_t n, const double* xp, const cnnsns_cls& w, const int32_t* fallback,
                  int32_t* start, int32_t* cls, float* logits, hipStream_t stream)
{
    if (n == 0) return;
    std::lock_guard<std::mutex> lock(m.cls_ws.mu);
    if (!m.cls_pool) build_pool(m, stream);
    workspace_acquire(m.cls_ws, cls_workspace_bytes(n), stream, "classify");
    const int64_t ch = n < kChunk ? n : kChunk;
    float* Z = static_cast<float*>(m.cls_ws.ptr);     // [ch][512]: module 1 | module 2
    float* Hb = Z + ch * kNZ;                          // [ch][512]: module 2's first layer, then FC h2
    float* Lw = Hb + ch * kH2;                         // [ch][81] logits when the caller keeps none
    const auto* xp2 = reinterpret_cast<const double2*>(xp);
    for (int64_t c0 = 0; c0 < n; c0 += ch) {
        const int mc = (int)(n - c0 < ch ? n - c0 : ch);
        float* L = logits ? logits + c0 * kNA : Lw;
        // persistent: three blocks per compute unit fit its LDS
        const unsigned mblocks = std::min<unsigned>(blocks_for(mc, kBlock / 64), cnn_persistent_grid() * 3);
        k_cls_module1<<<mblocks, kBlock, 0, stream>>>(
            mc, xp2 + c0, m.G, static_cast<const double2*>(m.cls_pool), w.w[0], w.b[0], w.w[1], w.b[1], w.w[2], w.b[2],
            Z, kNZ, Hb, kH2);
        const dim3 g256(blocks_for(mc, kDT), kH1 / kDT), g512(blocks_for(mc, kDT), kH2 / kDT),
            g81(blocks_for(mc, kDT), (kNA + kDT - 1) / kDT);
        k_dense_f32<true><<<g256, kBlock, 0, stream>>>(mc, kH1, kH1, Hb, kH2, w.w[3], w.b[3], Z + kNF, kNZ);
        k_dense_f32<true><<<g512, kBlock, 0, stream>>>(mc, kH2, kNZ, Z, kNZ, w.w[4], w.b[4], Hb, kH2);
        k_dense_f32<false><<<g81, kBlock, 0, stream>>>(mc, kNA, kH2, Hb, kH2, w.w[5], w.b[5], L, kNA);
        k_cls_argmax<<<blocks_for(mc, kBlock), kBlock, 0, stream>>>(mc, xp2 + c0, m.G, m.lookup, L, kNA,
                                                                    fallback ? fallback + c0 : nullptr, start + c0,
                                                                    cls ? cls + c0 : nullptr);
    }
    hip_check(hipGetLastError(), "classify launch");
    workspace_used(m.cls_ws, stream);
}

}  // namespace cnnsns
