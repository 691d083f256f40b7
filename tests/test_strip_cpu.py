"""CPU: the column-strip tiling of the FP32 conv3 + conv4 pass (csrc/strip.h) writes every output
pixel exactly once.

The test compiles strip.h itself for the host (its iterator takes the block and grid explicitly
there) with the tile sizes of that pass: first tiles of a segment write 14 rows, continuing tiles
16, strips are 30 columns wide.  For every overlay side G up to 1024, a sample up to 4096, and
several compute-unit counts, it plans the segments as the launcher does (strip_plan, then a grid of
min(units, segments) blocks rounded up to a multiple of 8), walks every block's tiles, and checks
that in every strip the tiles' row spans partition [0, G) in order, none starting past the grid,
that a continuing tile follows its block's previous tile directly, and that no block walks more
tiles than the plan's cost.  The benchmark's count of the pass's issued matrix work plans the tiles
in Python; its tile totals must equal the walked ones.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_18379_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include "strip.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <utility>
#include <vector>

using namespace cnnsns;
constexpr int FIRST = 14, NEXT = 16, W = 30;

static long long total_tiles = 0;

static int check(int G, unsigned cus)
{
    total_tiles = 0;
    const unsigned gmax = std::max(8u, (cus + 7) / 8 * 8);
    int nseg = 0;
    const int kb = strip_plan(G, FIRST, NEXT, W, gmax, &nseg);
    const int seg_rows = FIRST + NEXT * kb, tx = (G + W - 1) / W;
    unsigned g = cus < (unsigned)nseg ? cus : (unsigned)nseg;
    g = std::max(8u, (g + 7) / 8 * 8);
    const long long cost = (long long)((nseg + g - 1) / g) * (kb + 1);
    std::vector<std::vector<std::pair<int, int>>> spans(tx);
    for (unsigned b = 0; b < g; ++b) {
        StripIter<FIRST, NEXT, W> it(nseg, tx, seg_rows, G, b, g);
        long long n = 0;
        int prev_end = -1, prev_x = -1;
        for (; it.valid(); it.advance()) {
            const int x = it.x(), y = it.y(), r = it.rows();
            if (x % W != 0 || x / W >= tx) return printf("G=%d cus=%u: tile column %d\n", G, cus, x), 1;
            if (y >= G) return printf("G=%d cus=%u: tile starts at row %d\n", G, cus, y), 1;
            if (it.continues() && (prev_x != x || prev_end != y))
                return printf("G=%d cus=%u: continuing tile at (%d, %d) does not follow its block's previous tile\n",
                              G, cus, x, y), 1;
            if (r != (it.continues() ? NEXT : FIRST)) return printf("G=%d cus=%u: rows %d\n", G, cus, r), 1;
            spans[x / W].push_back({ y, y + r });
            prev_end = y + r;
            prev_x = x;
            ++n;
            ++total_tiles;
        }
        if (n > cost) return printf("G=%d cus=%u: block %u walks %lld tiles, plan %lld\n", G, cus, b, n, cost), 1;
    }
    for (int s = 0; s < tx; ++s) {
        auto& v = spans[s];
        std::sort(v.begin(), v.end());
        int at = 0;
        for (auto& p : v) {
            if (p.first != at) return printf("G=%d cus=%u: strip %d row %d covered from %d\n", G, cus, s, at, p.first), 1;
            at = p.second;
        }
        if (at < G) return printf("G=%d cus=%u: strip %d ends at row %d\n", G, cus, s, at), 1;
    }
    return 0;
}

int main(int argc, char** argv)
{
    if (argc > 1) {  // "G cus" pairs: the tiles the pass runs for each
        for (int a = 1; a + 1 < argc; a += 2) {
            const int G = atoi(argv[a]);
            const unsigned cus = (unsigned)atoi(argv[a + 1]);
            if (check(G, cus)) return 1;
            printf("%d %u %lld\n", G, cus, total_tiles);
        }
        return 0;
    }
    std::vector<int> sides;
    for (int G = 1; G <= 1024; ++G) sides.push_back(G);
    for (int G = 1031; G < 4096; G += 37) sides.push_back(G);
    sides.push_back(4095);
    sides.push_back(4096);
    const unsigned units[] = { 8, 104, 248, 256, 304 };
    long long cases = 0;
    for (int G : sides)
        for (unsigned cus : units) {
            if (check(G, cus)) return 1;
            ++cases;
        }
    printf("ok %lld\n", cases);
    return 0;
}
"""


def test_strip_tiling_covers_every_pixel_once(tmp_path):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    src = tmp_path / "strip_check.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "strip_check"
    r = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "--offload-host-only", "-O2", "-std=c++17",
                        "-I", CSRC, str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stdout.startswith("ok"), r.stdout

    # the benchmark's count of the matrix work this pass issues uses its own copy of the plan: it must
    # give the tiles the kernel runs
    import sys
    sys.path.insert(0, ROOT)
    import bench
    cases = [(G, cus) for G in (1, 14, 30, 64, 601, 777, 1024, 2000, 4096) for cus in (8, 248, 256)]
    r = subprocess.run([str(exe), *[str(v) for c in cases for v in c]], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout[-2000:]
    got = {(int(a), int(b)): int(t) for a, b, t in (line.split() for line in r.stdout.strip().splitlines())}
    for G, cus in cases:
        assert bench.conv34_tiles(G, cus) == got[(G, cus)], (G, cus, bench.conv34_tiles(G, cus), got[(G, cus)])
