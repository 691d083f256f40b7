// Column-strip tiling of the 2D CNN passes whose tiles recompute a vertical halo.
//
// Output tiles are W columns wide.  Blocks walk down column strips in segments of seg_rows output
// rows: the first tile of a segment writes FIRST rows; every further tile writes NEXT rows and takes
// the rows it shares with the tile above it from that tile's results (kept on chip) instead of
// recomputing them.  Segments are numbered row-major over (segment row, strip) and split into 8
// contiguous ranges, one per XCD (workgroups are dispatched to the 8 XCDs round-robin by id), so the
// blocks of one XCD work on neighbouring strips, whose halo columns meet in the same L2.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

namespace cnnsns {

template <int FIRST, int NEXT, int W>
struct StripIter {
    int s, end, step, j, tiles_x, seg_rows, G;
    // the tiles of block `block` of `grid` (the host-side form lets the plan be checked on the CPU)
    __host__ __device__ StripIter(int nseg, int tiles_x_, int seg_rows_, int G_, unsigned block, unsigned grid)
        : j(0), tiles_x(tiles_x_), seg_rows(seg_rows_), G(G_)
    {
        const int nx = 8;
        const int xcd = block % nx, slot = block / nx;
        s = (int)((int64_t)nseg * xcd / nx) + slot;
        end = (int)((int64_t)nseg * (xcd + 1) / nx);
        step = grid / nx;
    }
    __device__ StripIter(int nseg, int tiles_x_, int seg_rows_, int G_)
        : StripIter(nseg, tiles_x_, seg_rows_, G_, blockIdx.x, gridDim.x)
    {
    }
    __host__ __device__ bool valid() const { return s < end; }
    __host__ __device__ bool continues() const { return j > 0; }           // not the segment's first tile
    __host__ __device__ int rows() const { return j > 0 ? NEXT : FIRST; }  // output rows it writes
    __host__ __device__ int y() const { return (s / tiles_x) * seg_rows + (j == 0 ? 0 : FIRST + NEXT * (j - 1)); }
    __host__ __device__ int x() const { return (s % tiles_x) * W; }
    __host__ __device__ void advance()
    {
        const int yend = (s / tiles_x + 1) * seg_rows, ylim = yend < G ? yend : G;
        if ((s / tiles_x) * seg_rows + FIRST + NEXT * j < ylim) {
            ++j;
        } else {
            s += step;
            j = 0;
        }
    }
};

// The segment plan for a G x G grid and at most gmax blocks: the number kb of continuing tiles per
// segment (seg_rows = first + next kb) that minimises the tiles of the busiest block; *nseg gets the
// number of segments.
inline int strip_plan(int G, int first, int next, int width, unsigned gmax, int* nseg)
{
    auto cdiv = [](int64_t a, int64_t b) { return (a + b - 1) / b; };
    const int tx = (int)cdiv(G, width);
    int64_t best = -1;
    int kb_best = 0;
    for (int kb = 0; kb <= 64; ++kb) {
        const int seg = first + next * kb, n = tx * (int)cdiv(G, seg);
        const unsigned grid = n < (int)gmax ? (unsigned)std::max(8, (n + 7) / 8 * 8) : gmax;
        const int64_t cost = cdiv(n, grid) * (kb + 1);
        if (best < 0 || cost <= best) {
            best = cost;
            kb_best = kb;
            *nseg = n;
        }
        if (seg >= G) break;
    }
    return kb_best;
}

}  // namespace cnnsns
