/*
 * CPU oracle for 2D CNN-SNS particle location (Luo et al., "A CNN-based
 * particle tracking method for large-scale fluid simulations with
 * Lagrangian-Eulerian approaches").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it;
 * the GPU library never links, imports or falls back to it, and it shares no
 * code with the GPU library.
 *
 * Arithmetic: IEEE FP64 throughout for geometry, compiled with
 * -ffp-contract=off (no fused multiply-add) and no fast-math, so every
 * expression below is evaluated exactly as written, operation by operation.
 * The CNN is accumulated in FP64 from FP32 inputs and weights widened exactly.
 *
 * Paper -> 2D: the paper works with tetrahedra (4 barycentric coordinates,
 * 4 neighbours).  Here elements are triangles: 3 barycentric coordinates from
 * 3x3 determinants and 3 neighbours, one across each edge.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC oracle.c
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EMESH (-4)

/* per-point outcome of a walk */
#define ORC_FOUND 0
#define ORC_OUTSIDE 1
#define ORC_MAXITER 2
#define ORC_BADSTART 3

/* Number of threads used by the parallel loops (n <= 0 only queries). */
int orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* ------------------------------------------------------------------------ */
/* Element geometry.                                                         */

/*
 * Twice the signed area of triangle (a, b, c): the determinant |S_0| of the
 * matrix of homogeneous vertex coordinates (Sec. 2.2, definition of the
 * barycentric coordinates), in 2D.  Positive for counter-clockwise order.
 */
static double area2(const double* a, const double* b, const double* c)
{
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/*
 * The three barycentric numerators of p in the triangle with vertices
 * v[0], v[1], v[2] (Sec. 2.2): s_j = |S_j| is the determinant with vertex j's
 * column replaced by p, so lambda_j = s_j / |S_0|.  Written out, with indices
 * taken mod 3:
 *     s_j = (x_{j+1} - px) (y_{j+2} - py) - (y_{j+1} - py) (x_{j+2} - px).
 * For a counter-clockwise triangle |S_0| > 0, so sign(lambda_j) = sign(s_j)
 * and the smallest lambda_j is at the smallest s_j; the walk compares the
 * numerators and never divides.  Because IEEE multiplication commutes and
 * fl(b - a) = -fl(a - b), the numerator for a shared edge evaluated in the
 * two triangles that share it (which traverse the edge in opposite
 * directions) are exact negatives of each other.
 */
static void bary_numerators(const double* const v[3], const double* p, double s[3])
{
    for (int j = 0; j < 3; ++j) {
        const double* u = v[(j + 1) % 3];
        const double* w = v[(j + 2) % 3];
        s[j] = (u[0] - p[0]) * (w[1] - p[1]) - (u[1] - p[1]) * (w[0] - p[0]);
    }
}

/* ------------------------------------------------------------------------ */
/* Mesh preparation: the element list {K_l} and neighbour table {m^l}.      */

/*
 * Put every triangle in counter-clockwise order (swap its 2nd and 3rd vertex
 * when |S_0| < 0), keeping triangle ids.  Zero-area triangles and vertex
 * indices outside [0, n_nodes) are mesh errors.
 */
int orc_canonicalise(int64_t n_nodes, const double* xy, int64_t n_tri, const int32_t* tri_in, int32_t* tri_out)
{
    if (n_nodes < 0 || n_tri < 0 || (n_tri > 0 && (!xy || !tri_in || !tri_out))) return ORC_EINVAL;
    for (int64_t t = 0; t < n_tri; ++t) {
        int32_t a = tri_in[3 * t], b = tri_in[3 * t + 1], c = tri_in[3 * t + 2];
        if (a < 0 || b < 0 || c < 0 || a >= n_nodes || b >= n_nodes || c >= n_nodes) return ORC_EMESH;
        double d = area2(xy + 2 * (int64_t)a, xy + 2 * (int64_t)b, xy + 2 * (int64_t)c);
        if (d == 0.0) return ORC_EMESH;
        tri_out[3 * t] = a;
        tri_out[3 * t + 1] = d > 0 ? b : c;
        tri_out[3 * t + 2] = d > 0 ? c : b;
    }
    return ORC_OK;
}

/*
 * Neighbour table (Sec. 2.2): nbr[3t + j] is the triangle across the edge
 * opposite vertex j of triangle t, i.e. the other triangle containing both
 * vertices (j+1)%3 and (j+2)%3, or -1 when that edge is on the boundary.
 * Mesh errors: an edge in more than two triangles, or an edge whose two
 * triangles traverse it in the same direction (overlapping triangles).
 * The triangles must already be counter-clockwise.
 */
int orc_neighbours(int64_t n_nodes, int64_t n_tri, const int32_t* tri, int32_t* nbr)
{
    if (n_nodes < 0 || n_tri < 0) return ORC_EINVAL;
    int64_t* first = (int64_t*)calloc((size_t)n_nodes + 1, sizeof(int64_t));
    int64_t* cursor = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_nodes + 1));
    int32_t* inc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * n_tri + 1));
    if (!first || !cursor || !inc) { free(first); free(cursor); free(inc); return ORC_ENOMEM; }
    /* triangles incident to each node */
    for (int64_t k = 0; k < 3 * n_tri; ++k) first[tri[k] + 1]++;
    for (int64_t v = 0; v < n_nodes; ++v) first[v + 1] += first[v];
    memcpy(cursor, first, sizeof(int64_t) * ((size_t)n_nodes + 1));
    for (int64_t t = 0; t < n_tri; ++t)
        for (int j = 0; j < 3; ++j) inc[cursor[tri[3 * t + j]]++] = (int32_t)t;
    int rc = ORC_OK;
    for (int64_t t = 0; t < n_tri && rc == ORC_OK; ++t) {
        for (int j = 0; j < 3 && rc == ORC_OK; ++j) {
            int32_t u = tri[3 * t + (j + 1) % 3], w = tri[3 * t + (j + 2) % 3];
            int32_t found = -1;
            for (int64_t k = first[u]; k < first[u + 1]; ++k) {
                int32_t s = inc[k];
                if (s == t) continue;
                const int32_t* S = tri + 3 * (int64_t)s;
                int iu = -1, iw = -1;
                for (int q = 0; q < 3; ++q) {
                    if (S[q] == u) iu = q;
                    if (S[q] == w) iw = q;
                }
                if (iw < 0) continue;
                if (found >= 0) { rc = ORC_EMESH; break; }       /* edge in 3+ triangles */
                if ((iu + 1) % 3 == iw) { rc = ORC_EMESH; break; } /* same direction u->w */
                found = s;
            }
            nbr[3 * t + j] = found;
        }
    }
    free(first); free(cursor); free(inc);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1: successive neighbour search.                                */

/*
 * SNS walk for one point (Alg. 1 / eq. 6), from the start element k0:
 *   I <- 0; loop { I <- I + 1; compute the barycentric coordinates of x_p in
 *   the current element; if all are >= 0 the element contains x_p (closed
 *   test, Sec. 2.2) -> stop; otherwise take j with the smallest coordinate
 *   (eq. 5; ties go to the lowest j); if the neighbour m_j of the current
 *   element is -1 the walk has reached the domain boundary and x_p lies
 *   outside -> stop; else move to m_j }.
 * The paper's loop has no bound; max_iter caps it (status MAXITER, returned
 * with the element just moved to).  A start outside [0, n_tri) is reported
 * as BADSTART with host -1 and zero iterations.
 */
static void sns_one(int64_t n_tri, const double* xy, const int32_t* tri, const int32_t* nbr,
                    const double* p, int32_t k0, int32_t max_iter,
                    int32_t* host, int32_t* iters, uint8_t* status)
{
    if (k0 < 0 || k0 >= n_tri) { *host = -1; *iters = 0; *status = ORC_BADSTART; return; }
    int32_t K = k0, I = 0;
    for (;;) {
        I = I + 1;
        const double* v[3] = { xy + 2 * (int64_t)tri[3 * (int64_t)K], xy + 2 * (int64_t)tri[3 * (int64_t)K + 1],
                               xy + 2 * (int64_t)tri[3 * (int64_t)K + 2] };
        double s[3];
        bary_numerators(v, p, s);
        if (s[0] >= 0.0 && s[1] >= 0.0 && s[2] >= 0.0) { *host = K; *iters = I; *status = ORC_FOUND; return; }
        int j = 0;
        if (s[1] < s[j]) j = 1;
        if (s[2] < s[j]) j = 2;
        int32_t m = nbr[3 * (int64_t)K + j];
        if (m == -1) { *host = K; *iters = I; *status = ORC_OUTSIDE; return; }
        K = m;
        if (I >= max_iter) { *host = K; *iters = I; *status = ORC_MAXITER; return; }
    }
}

/*
 * Locate n points: host[i] = SNS(xp[i], start[i]).  max_iter <= 0 selects
 * the default cap 2^20.  tri must be counter-clockwise and nbr its
 * neighbour table.  Points are independent; they are split over threads.
 */
int orc_sns(int64_t n_tri, const double* xy, const int32_t* tri, const int32_t* nbr,
            int64_t n, const double* xp, const int32_t* start, int32_t max_iter,
            int32_t* host, int32_t* iters, uint8_t* status)
{
    if (n < 0 || n_tri < 0) return ORC_EINVAL;
    if (max_iter <= 0) max_iter = 1 << 20;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i)
        sns_one(n_tri, xy, tri, nbr, xp + 2 * i, start[i], max_iter, host + i, iters + i, status + i);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Interpolation at the departure point (Sec. 2.1).                          */

/*
 * After eq. 4, the velocity at the departure point x_p is approximated by
 * interpolation in its host element with the element's nodal basis functions
 * phi_j (phi_i(n_j) = 1 for i = j, 0 otherwise).  For a linear triangle these
 * are its barycentric coordinates (Sec. 2.2), lambda_j = |S_j| / |S_0|, so a
 * nodal field f takes at p the value
 *     f(p) = lambda_0 f(n_0) + lambda_1 f(n_1) + lambda_2 f(n_2)
 * over the nodes of the counter-clockwise host triangle, added in that order.
 * nodal holds two components per node and out two per point.  A host id
 * outside [0, n_tri) (a point whose start was invalid) gives NaN.
 */
int orc_interp(int64_t n_tri, const double* xy, const int32_t* tri, const double* nodal, int64_t n,
               const double* xp, const int32_t* host, double* out)
{
    if (n < 0 || n_tri < 0) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t t = host[i];
        if (t < 0 || t >= n_tri) {
            out[2 * i] = NAN;
            out[2 * i + 1] = NAN;
            continue;
        }
        const int32_t* nd = tri + 3 * t;
        const double* v[3] = { xy + 2 * (int64_t)nd[0], xy + 2 * (int64_t)nd[1], xy + 2 * (int64_t)nd[2] };
        double s[3];
        bary_numerators(v, xp + 2 * i, s);
        const double a = area2(v[0], v[1], v[2]);
        for (int c = 0; c < 2; ++c) {
            double f = 0.0;
            for (int j = 0; j < 3; ++j) f += (s[j] / a) * nodal[2 * (int64_t)nd[j] + c];
            out[2 * i + c] = f;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* ASG overlay: cell -> element lookup.                                      */

/*
 * The auxiliary structured grid (Sec. 1, Alg. 2): a G x G Cartesian grid over
 * the unit square.  lookup[cy*G + cx] is the smallest id of a triangle whose
 * closed region contains the cell centre ((cx + 1/2)/G, (cy + 1/2)/G), or -1
 * when no triangle contains it.  Triangles are visited in increasing id, and
 * each tests the centres inside its bounding box (a conservative superset of
 * the centres it can contain); the first triangle to claim a cell is the
 * smallest containing id.  tri must be counter-clockwise.
 */
int orc_lookup(int64_t n_tri, const double* xy, const int32_t* tri, int32_t G, int32_t* lookup)
{
    if (G <= 0 || n_tri < 0) return ORC_EINVAL;
    for (int64_t c = 0; c < (int64_t)G * G; ++c) lookup[c] = -1;
    for (int64_t t = 0; t < n_tri; ++t) {
        const double* v[3] = { xy + 2 * (int64_t)tri[3 * t], xy + 2 * (int64_t)tri[3 * t + 1],
                               xy + 2 * (int64_t)tri[3 * t + 2] };
        double xmin = fmin(v[0][0], fmin(v[1][0], v[2][0])), xmax = fmax(v[0][0], fmax(v[1][0], v[2][0]));
        double ymin = fmin(v[0][1], fmin(v[1][1], v[2][1])), ymax = fmax(v[0][1], fmax(v[1][1], v[2][1]));
        /* centre (c + 1/2)/G in [min, max]  <=>  c in [min*G - 1/2, max*G - 1/2]; widened by one */
        int64_t cx0 = (int64_t)floor(xmin * G - 0.5) - 1, cx1 = (int64_t)ceil(xmax * G - 0.5) + 1;
        int64_t cy0 = (int64_t)floor(ymin * G - 0.5) - 1, cy1 = (int64_t)ceil(ymax * G - 0.5) + 1;
        if (cx0 < 0) cx0 = 0;
        if (cy0 < 0) cy0 = 0;
        if (cx1 > G - 1) cx1 = G - 1;
        if (cy1 > G - 1) cy1 = G - 1;
        for (int64_t cy = cy0; cy <= cy1; ++cy) {
            for (int64_t cx = cx0; cx <= cx1; ++cx) {
                if (lookup[cy * G + cx] != -1) continue;
                double p[2] = { ((double)cx + 0.5) / (double)G, ((double)cy + 0.5) / (double)G };
                double s[3];
                bary_numerators(v, p, s);
                if (s[0] >= 0.0 && s[1] >= 0.0 && s[2] >= 0.0) lookup[cy * G + cx] = (int32_t)t;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* CNN: displacement predictor over the overlay grid.                        */

/*
 * One 3x3 convolution layer (stride 1, "same" zero padding, cross-correlation
 * with weights in [out][in][ky][kx] order, bias, optional ReLU; the layers of
 * Sec. 2.3 with ReLU between layers), evaluated on a window of the G x G grid:
 *   y[o][r][c] = b[o] + sum_i sum_{dy,dx in -1..1} W[o][i][dy+1][dx+1] * x[i][r+dy][c+dx],
 * where x is zero outside [0, G)^2.  The input window covers global rows
 * [ir0, ir0 + ih) and columns [ic0, ic0 + iw); the output window
 * [or0, or0 + oh) x [oc0, oc0 + ow) must be such that every in-grid tap falls
 * inside the input window.
 */
static void conv3x3(int32_t G, const double* x, int32_t cin, int64_t ir0, int64_t ic0, int64_t ih, int64_t iw,
                    double* y, int32_t cout, int64_t or0, int64_t oc0, int64_t oh, int64_t ow,
                    const double* W, const double* b, int relu)
{
#pragma omp parallel for schedule(static)
    for (int64_t rr = 0; rr < oh; ++rr) {
        for (int32_t o = 0; o < cout; ++o) {
            for (int64_t cc = 0; cc < ow; ++cc) {
                int64_t r = or0 + rr, c = oc0 + cc;
                double acc = b[o];
                for (int32_t i = 0; i < cin; ++i) {
                    for (int dy = -1; dy <= 1; ++dy) {
                        for (int dx = -1; dx <= 1; ++dx) {
                            int64_t R = r + dy, C = c + dx;
                            if (R < 0 || R >= G || C < 0 || C >= G) continue;
                            double xv = x[((int64_t)i * ih + (R - ir0)) * iw + (C - ic0)];
                            acc += W[(((int64_t)o * cin + i) * 3 + (dy + 1)) * 3 + (dx + 1)] * xv;
                        }
                    }
                }
                if (relu && acc < 0.0) acc = 0.0;
                y[((int64_t)o * oh + rr) * ow + cc] = acc;
            }
        }
    }
}

/*
 * Four-layer displacement CNN, channels chan[0] -> chan[1] -> ... -> chan[4]
 * (2 -> 32 -> 32 -> 32 -> 2 for the velocity-to-displacement net), ReLU after
 * layers 1-3 and none after the last.  Evaluates the output on rows
 * [r0, r0+h) and columns [c0, c0+w) of the G x G grid; with r0 = c0 = 0 and
 * h = w = G this is the whole forward pass.  Each inner layer is computed on
 * the output window grown by one cell per remaining layer (clipped to the
 * grid), so that the result equals the full-grid forward pass restricted to
 * the window.
 *   vel: FP32 [chan0][G][G]; w[l]: FP32 [chan(l+1)][chan(l)][3][3]; b[l]: FP32;
 *   out: FP64 [chan4][h][w].
 */
int orc_cnn_window(int32_t G, const float* vel, const int32_t* chan, const float* const* w, const float* const* b,
                   int64_t r0, int64_t c0, int64_t h, int64_t wd, double* out)
{
    if (G <= 0 || h <= 0 || wd <= 0 || r0 < 0 || c0 < 0 || r0 + h > G || c0 + wd > G) return ORC_EINVAL;
    /* window of each activation: act 0 = input, act 4 = output */
    int64_t wr0[5], wc0[5], wh[5], ww[5];
    for (int l = 0; l <= 4; ++l) {
        int64_t grow = 4 - l;
        int64_t ra = r0 - grow, rb = r0 + h + grow, ca = c0 - grow, cb = c0 + wd + grow;
        if (ra < 0) ra = 0;
        if (ca < 0) ca = 0;
        if (rb > G) rb = G;
        if (cb > G) cb = G;
        wr0[l] = ra; wc0[l] = ca; wh[l] = rb - ra; ww[l] = cb - ca;
    }
    double* act[5] = { 0 };
    double* Wd[4] = { 0 };
    double* bd[4] = { 0 };
    int rc = ORC_OK;
    for (int l = 0; l <= 4; ++l) {
        act[l] = (double*)malloc(sizeof(double) * (size_t)(chan[l] * wh[l] * ww[l]));
        if (!act[l]) rc = ORC_ENOMEM;
    }
    for (int l = 0; l < 4; ++l) {
        Wd[l] = (double*)malloc(sizeof(double) * (size_t)(chan[l + 1] * chan[l] * 9));
        bd[l] = (double*)malloc(sizeof(double) * (size_t)chan[l + 1]);
        if (!Wd[l] || !bd[l]) rc = ORC_ENOMEM;
    }
    if (rc == ORC_OK) {
        for (int l = 0; l < 4; ++l) {
            for (int64_t k = 0; k < (int64_t)chan[l + 1] * chan[l] * 9; ++k) Wd[l][k] = (double)w[l][k];
            for (int32_t k = 0; k < chan[l + 1]; ++k) bd[l][k] = (double)b[l][k];
        }
        for (int32_t i = 0; i < chan[0]; ++i)
            for (int64_t r = 0; r < wh[0]; ++r)
                for (int64_t c = 0; c < ww[0]; ++c)
                    act[0][((int64_t)i * wh[0] + r) * ww[0] + c] =
                        (double)vel[((int64_t)i * G + (wr0[0] + r)) * G + (wc0[0] + c)];
        for (int l = 0; l < 4; ++l)
            conv3x3(G, act[l], chan[l], wr0[l], wc0[l], wh[l], ww[l], act[l + 1], chan[l + 1], wr0[l + 1],
                    wc0[l + 1], wh[l + 1], ww[l + 1], Wd[l], bd[l], l < 3);
        memcpy(out, act[4], sizeof(double) * (size_t)(chan[4] * h * wd));
    }
    for (int l = 0; l <= 4; ++l) free(act[l]);
    for (int l = 0; l < 4; ++l) { free(Wd[l]); free(bd[l]); }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2: the CNN-SNS start element.                                   */

/* overlay cell index of a coordinate: min(G-1, floor(x G)), clamped to >= 0 */
static int64_t cell_of(double x, int32_t G)
{
    double f = floor(x * (double)G);
    if (!(f >= 0.0)) return 0; /* negative or NaN */
    if (f > (double)(G - 1)) return G - 1;
    return (int64_t)f;
}

/*
 * Start element K_p of CNN-SNS (Alg. 2): the predicted departure point is
 * x_hat = clamp(x_i + D, 0, 1), with D the predicted displacement of the
 * overlay cell holding the origin x_i, and K_p is the overlay lookup of the
 * cell holding x_hat.  When that cell has no element (-1), the fallback
 * start[i] is used if given, else element 0.
 *   origin: [n][2]; disp: [2][G][G] (x then y component); lookup: [G][G].
 */
int orc_cnnsns_start(int64_t n, const double* origin, int32_t G, const double* disp, const int32_t* lookup,
                     const int32_t* fallback, int32_t* start_out)
{
    if (n < 0 || G <= 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = cell_of(origin[2 * i], G), cy = cell_of(origin[2 * i + 1], G);
        double dx = disp[(0 * (int64_t)G + cy) * G + cx];
        double dy = disp[(1 * (int64_t)G + cy) * G + cx];
        double hx = origin[2 * i] + dx, hy = origin[2 * i + 1] + dy;
        hx = hx < 0.0 ? 0.0 : (hx > 1.0 ? 1.0 : hx);
        hy = hy < 0.0 ? 0.0 : (hy > 1.0 ? 1.0 : hy);
        int32_t k = lookup[cell_of(hy, G) * G + cell_of(hx, G)];
        if (k < 0) k = fallback ? fallback[i] : 0;
        start_out[i] = k;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive containment (the definition of the host element).              */

/*
 * For each point, the smallest id of a triangle whose closed region contains
 * it, testing every triangle (Sec. 2.2: x_p lies in K_l iff all barycentric
 * coordinates are >= 0), or -1.  O(n * n_tri): small meshes only.
 */
int orc_brute_force(int64_t n_tri, const double* xy, const int32_t* tri, int64_t n, const double* xp,
                    int32_t* host)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        host[i] = -1;
        for (int64_t t = 0; t < n_tri; ++t) {
            const double* v[3] = { xy + 2 * (int64_t)tri[3 * t], xy + 2 * (int64_t)tri[3 * t + 1],
                                   xy + 2 * (int64_t)tri[3 * t + 2] };
            double s[3];
            bary_numerators(v, xp + 2 * i, s);
            if (s[0] >= 0.0 && s[1] >= 0.0 && s[2] >= 0.0) { host[i] = (int32_t)t; break; }
        }
    }
    return ORC_OK;
}

/* ======================================================================== */
/* 3D: tetrahedral meshes, the paper's own setting (Sec. 2.2 with 4 nodes).  */
/* ======================================================================== */

/*
 * det[a - p, b - p, c - p]: six times the signed volume of tetrahedron
 * (p, a, b, c), positive when (a, b, c) turn counter-clockwise seen from p's
 * opposite side, i.e. the determinant |S| of Sec. 2.2 with the homogeneous
 * row removed by subtracting p's column.  Evaluated as written:
 *   det = ax (by cz - bz cy) - ay (bx cz - bz cx) + az (bx cy - by cx).
 */
static double orient3(const double* p, const double* a, const double* b, const double* c)
{
    const double ax = a[0] - p[0], ay = a[1] - p[1], az = a[2] - p[2];
    const double bx = b[0] - p[0], by = b[1] - p[1], bz = b[2] - p[2];
    const double cx = c[0] - p[0], cy = c[1] - p[1], cz = c[2] - p[2];
    const double t1 = by * cz - bz * cy, t2 = bx * cz - bz * cx, t3 = bx * cy - by * cx;
    return ax * t1 - ay * t2 + az * t3;
}

/*
 * The four barycentric numerators s_j = |S_j| of p in the positively
 * oriented tetrahedron v[0..3] (node ids id[0..3]): the volume determinant
 * with vertex j replaced by p.  Moving p to the front gives
 *   s_j = sigma_j det[F_j - p], sigma = (+, -, +, -),
 * with F_j the other three vertices in the tetrahedron's order.  The face is
 * evaluated with its vertices sorted by node id (and the sign of that
 * permutation applied), so the two tetrahedra that share a face compute the
 * very same number for it and their numerators are exact negatives.
 */
static void bary3_numerators(const double* const v[4], const int32_t id[4], const double* p, double s[4])
{
    for (int j = 0; j < 4; ++j) {
        int f[3], k = 0;
        for (int m = 0; m < 4; ++m)
            if (m != j) f[k++] = m;
        int sign = (j & 1) ? -1 : 1;
        /* sort the three face vertices by node id, flipping the sign per swap */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2 - a; ++b)
                if (id[f[b]] > id[f[b + 1]]) {
                    const int t = f[b];
                    f[b] = f[b + 1];
                    f[b + 1] = t;
                    sign = -sign;
                }
        const double d = orient3(p, v[f[0]], v[f[1]], v[f[2]]);
        s[j] = sign > 0 ? d : -d;
    }
}

static void tet_vertices(const double* xyz, const int32_t* tet, int64_t t, const double* v[4], int32_t id[4])
{
    for (int k = 0; k < 4; ++k) {
        id[k] = tet[4 * t + k];
        v[k] = xyz + 3 * (int64_t)id[k];
    }
}

/*
 * Put every tetrahedron in positive orientation (det[b - a, c - a, d - a] > 0;
 * swap its 3rd and 4th vertex when negative), keeping ids.  Zero volume and
 * vertex indices outside [0, n_nodes) are mesh errors.
 */
int orc3_canonicalise(int64_t n_nodes, const double* xyz, int64_t n_tet, const int32_t* tet_in, int32_t* tet_out)
{
    for (int64_t t = 0; t < n_tet; ++t) {
        const int32_t* q = tet_in + 4 * t;
        for (int k = 0; k < 4; ++k)
            if (q[k] < 0 || q[k] >= n_nodes) return ORC_EMESH;
        const double vol = orient3(xyz + 3 * (int64_t)q[0], xyz + 3 * (int64_t)q[1], xyz + 3 * (int64_t)q[2],
                                   xyz + 3 * (int64_t)q[3]);
        if (vol == 0.0) return ORC_EMESH;
        tet_out[4 * t] = q[0];
        tet_out[4 * t + 1] = q[1];
        tet_out[4 * t + 2] = vol < 0.0 ? q[3] : q[2];
        tet_out[4 * t + 3] = vol < 0.0 ? q[2] : q[3];
    }
    return ORC_OK;
}

typedef struct {
    int32_t k[3];
    int64_t slot; /* 4 t + j */
} Face3;

static int face3_cmp(const void* x, const void* y)
{
    const Face3* a = (const Face3*)x;
    const Face3* b = (const Face3*)y;
    for (int i = 0; i < 3; ++i)
        if (a->k[i] != b->k[i]) return a->k[i] < b->k[i] ? -1 : 1;
    return a->slot < b->slot ? -1 : (a->slot > b->slot ? 1 : 0);
}

/*
 * Neighbour table: nbr[4t + j] is the tetrahedron sharing the face opposite
 * vertex j of t, or -1 on the boundary.  A face in more than two tetrahedra
 * is a mesh error.  (Sorted list of faces keyed by their node ids.)
 */
int orc3_neighbours(int64_t n_tet, const int32_t* tet, int32_t* nbr)
{
    Face3* f = (Face3*)malloc(sizeof(Face3) * 4 * (size_t)n_tet);
    if (!f) return ORC_ENOMEM;
    for (int64_t t = 0; t < n_tet; ++t)
        for (int j = 0; j < 4; ++j) {
            Face3* e = f + 4 * t + j;
            int k = 0;
            for (int m = 0; m < 4; ++m)
                if (m != j) e->k[k++] = tet[4 * t + m];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2 - a; ++b)
                    if (e->k[b] > e->k[b + 1]) {
                        const int32_t x = e->k[b];
                        e->k[b] = e->k[b + 1];
                        e->k[b + 1] = x;
                    }
            e->slot = 4 * t + j;
            nbr[4 * t + j] = -1;
        }
    qsort(f, 4 * (size_t)n_tet, sizeof(Face3), face3_cmp);
    int rc = ORC_OK;
    for (int64_t i = 0; i < 4 * n_tet;) {
        int64_t e = i + 1;
        while (e < 4 * n_tet && f[e].k[0] == f[i].k[0] && f[e].k[1] == f[i].k[1] && f[e].k[2] == f[i].k[2]) ++e;
        if (e - i > 2) rc = ORC_EMESH;
        if (e - i == 2) {
            nbr[f[i].slot] = (int32_t)(f[i + 1].slot / 4);
            nbr[f[i + 1].slot] = (int32_t)(f[i].slot / 4);
        }
        i = e;
    }
    free(f);
    return rc;
}

/* Alg. 1 in 3D for one point: as sns_one with four numerators and neighbours. */
static void sns3_one(int64_t n_tet, const double* xyz, const int32_t* tet, const int32_t* nbr, const double* p,
                     int32_t start, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status)
{
    if (start < 0 || start >= n_tet) {
        *host = -1;
        *iters = 0;
        *status = ORC_BADSTART;
        return;
    }
    int32_t K = start, I = 0;
    for (;;) {
        I += 1;
        const double* v[4];
        int32_t id[4];
        double s[4];
        tet_vertices(xyz, tet, K, v, id);
        bary3_numerators(v, id, p, s);
        if (s[0] >= 0.0 && s[1] >= 0.0 && s[2] >= 0.0 && s[3] >= 0.0) {
            *host = K;
            *iters = I;
            *status = ORC_FOUND;
            return;
        }
        int jmin = 0;
        for (int j = 1; j < 4; ++j)
            if (s[j] < s[jmin]) jmin = j;
        const int32_t m = nbr[4 * (int64_t)K + jmin];
        if (m == -1) {
            *host = K;
            *iters = I;
            *status = ORC_OUTSIDE;
            return;
        }
        K = m;
        if (I >= max_iter) {
            *host = K;
            *iters = I;
            *status = ORC_MAXITER;
            return;
        }
    }
}

int orc3_sns(int64_t n_tet, const double* xyz, const int32_t* tet, const int32_t* nbr, int64_t n, const double* xp,
             const int32_t* start, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status)
{
    if (n < 0 || n_tet < 0) return ORC_EINVAL;
    if (max_iter <= 0) max_iter = 1 << 20;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i)
        sns3_one(n_tet, xyz, tet, nbr, xp + 3 * i, start[i], max_iter, host + i, iters + i, status + i);
    return ORC_OK;
}

/*
 * P1 interpolation at x_p in its host tetrahedron (Sec. 2.1 after eq. 4 with
 * the nodal basis of Sec. 2.2): u(x_p) = sum_j (s_j / V) u(n_j), with s_j the
 * four barycentric numerators and V = det[b - a, c - a, d - a] > 0 six times
 * the volume.  V is evaluated with the vertices in ascending node id (the sign
 * of that permutation applied) and the sum runs over the vertices in
 * ascending node id, so the value does not depend on the element's vertex
 * order.  nodal: [n_nodes][3]; out: [n][3]; a host outside [0, n_tet) gives NaN.
 */
int orc3_interp(int64_t n_tet, const double* xyz, const int32_t* tet, const double* nodal, int64_t n,
                const double* xp, const int32_t* host, double* out)
{
    if (n < 0 || n_tet < 0) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const int64_t t = host[i];
        if (t < 0 || t >= n_tet) {
            out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = NAN;
            continue;
        }
        const double* v[4];
        int32_t id[4];
        double s[4];
        tet_vertices(xyz, tet, t, v, id);
        bary3_numerators(v, id, xp + 3 * i, s);
        int ord[4] = { 0, 1, 2, 3 }, sign = 1;
        for (int a = 1; a < 4; ++a) /* insertion sort by node id, one sign flip per swap */
            for (int b = a; b > 0 && id[ord[b - 1]] > id[ord[b]]; --b) {
                const int x = ord[b];
                ord[b] = ord[b - 1];
                ord[b - 1] = x;
                sign = -sign;
            }
        double V = orient3(v[ord[0]], v[ord[1]], v[ord[2]], v[ord[3]]);
        if (sign < 0) V = -V;
        for (int c = 0; c < 3; ++c) {
            double f = 0.0;
            for (int k = 0; k < 4; ++k) f += (s[ord[k]] / V) * nodal[3 * (int64_t)id[ord[k]] + c];
            out[3 * i + c] = f;
        }
    }
    return ORC_OK;
}

/*
 * 3D overlay: lookup[(cz G + cy) G + cx] is the smallest id of a tetrahedron
 * whose closed region contains the cell centre ((c + 1/2) / G per axis), or
 * -1.  Tetrahedra in increasing id test the centres in their bounding box;
 * the first to claim a cell is the smallest containing id.
 */
int orc3_lookup(int64_t n_tet, const double* xyz, const int32_t* tet, int32_t G, int32_t* lookup)
{
    if (G <= 0 || n_tet < 0) return ORC_EINVAL;
    const int64_t nc = (int64_t)G * G * G;
    for (int64_t c = 0; c < nc; ++c) lookup[c] = -1;
    /* each thread owns a range of cell planes z and visits every tetrahedron in increasing id
       for the cells of its planes, so the result is the serial one */
#pragma omp parallel
    {
        const int tid = omp_get_thread_num(), nth = omp_get_num_threads();
        const int z_lo = (int)((int64_t)G * tid / nth), z_hi = (int)((int64_t)G * (tid + 1) / nth) - 1;
        for (int64_t t = 0; t < n_tet; ++t) {
            const double* v[4];
            int32_t id[4];
            tet_vertices(xyz, tet, t, v, id);
            int lo[3], hi[3];
            for (int d = 0; d < 3; ++d) {
                double mn = v[0][d], mx = v[0][d];
                for (int k = 1; k < 4; ++k) {
                    mn = v[k][d] < mn ? v[k][d] : mn;
                    mx = v[k][d] > mx ? v[k][d] : mx;
                }
                lo[d] = (int)floor(mn * G - 0.5) - 1;
                hi[d] = (int)ceil(mx * G - 0.5) + 1;
                if (lo[d] < 0) lo[d] = 0;
                if (hi[d] > G - 1) hi[d] = G - 1;
            }
            if (lo[2] < z_lo) lo[2] = z_lo;
            if (hi[2] > z_hi) hi[2] = z_hi;
            for (int cz = lo[2]; cz <= hi[2]; ++cz)
                for (int cy = lo[1]; cy <= hi[1]; ++cy)
                    for (int cx = lo[0]; cx <= hi[0]; ++cx) {
                        int32_t* cell = lookup + ((int64_t)cz * G + cy) * G + cx;
                        if (*cell != -1) continue;
                        const double p[3] = { (cx + 0.5) / G, (cy + 0.5) / G, (cz + 0.5) / G };
                        double s[4];
                        bary3_numerators(v, id, p, s);
                        if (s[0] >= 0.0 && s[1] >= 0.0 && s[2] >= 0.0 && s[3] >= 0.0) *cell = (int32_t)t;
                    }
        }
    }
    return ORC_OK;
}

/* Smallest id of a tetrahedron containing each point (closed), or -1: by trying all of them. */
int orc3_brute_force(int64_t n_tet, const double* xyz, const int32_t* tet, int64_t n, const double* xp, int32_t* host)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        host[i] = -1;
        for (int64_t t = 0; t < n_tet; ++t) {
            const double* v[4];
            int32_t id[4];
            double s[4];
            tet_vertices(xyz, tet, t, v, id);
            bary3_numerators(v, id, xp + 3 * i, s);
            if (s[0] >= 0.0 && s[1] >= 0.0 && s[2] >= 0.0 && s[3] >= 0.0) {
                host[i] = (int32_t)t;
                break;
            }
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* 3D displacement CNN (Sec. 2.3 with 3 x 3 x 3 kernels on a G x G x G grid) */

/*
 * One layer of 3 x 3 x 3 convolution with zero padding of one cell, on
 * windows of the G^3 grid (axes z, y, x, x fastest):
 *   y[o][z][y][x] = b[o] + sum_i sum_{dz,dy,dx in -1..1}
 *                   W[o][i][dz+1][dy+1][dx+1] * x[i][z+dz][y+dy][x+dx],
 * with x zero outside [0, G)^3.  The input window starts at iw0 = (z, y, x)
 * with sizes in_ = (d, h, w); the output window at ow0 with sizes on_, and
 * every in-grid tap of an output cell falls inside the input window.
 */
static void conv3x3x3(int32_t G, const double* x, int32_t cin, const int64_t iw0[3], const int64_t in_[3],
                      double* y, int32_t cout, const int64_t ow0[3], const int64_t on_[3], const double* W,
                      const double* b, int relu)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t zz = 0; zz < on_[0]; ++zz) {
        for (int64_t yy = 0; yy < on_[1]; ++yy) {
            for (int32_t o = 0; o < cout; ++o) {
                for (int64_t xx = 0; xx < on_[2]; ++xx) {
                    const int64_t z = ow0[0] + zz, yv = ow0[1] + yy, xv = ow0[2] + xx;
                    double acc = b[o];
                    for (int32_t i = 0; i < cin; ++i)
                        for (int dz = -1; dz <= 1; ++dz)
                            for (int dy = -1; dy <= 1; ++dy)
                                for (int dx = -1; dx <= 1; ++dx) {
                                    const int64_t Z = z + dz, Y = yv + dy, X = xv + dx;
                                    if (Z < 0 || Z >= G || Y < 0 || Y >= G || X < 0 || X >= G) continue;
                                    const double v =
                                        x[(((int64_t)i * in_[0] + (Z - iw0[0])) * in_[1] + (Y - iw0[1])) * in_[2] +
                                          (X - iw0[2])];
                                    acc += W[((((int64_t)o * cin + i) * 3 + (dz + 1)) * 3 + (dy + 1)) * 3 + (dx + 1)] * v;
                                }
                    if (relu && acc < 0.0) acc = 0.0;
                    y[(((int64_t)o * on_[0] + zz) * on_[1] + yy) * on_[2] + xx] = acc;
                }
            }
        }
    }
}

/*
 * Four-layer 3D displacement CNN, channels chan[0] -> ... -> chan[4]
 * (3 -> 32 -> 32 -> 32 -> 3 for velocity to displacement), ReLU after layers
 * 1-3.  Output on the window starting at (z0, y0, x0) of sizes (d, h, w) of
 * the G^3 grid; each inner layer is evaluated on the window grown by one cell
 * per remaining layer (clipped to the grid), so the result equals the
 * full-grid pass restricted to the window.
 *   vel: FP32 [chan0][G][G][G]; w[l]: FP32 [chan(l+1)][chan(l)][3][3][3];
 *   b[l]: FP32 [chan(l+1)]; out: FP64 [chan4][d][h][w].
 */
int orc3_cnn_window(int32_t G, const float* vel, const int32_t* chan, const float* const* w, const float* const* b,
                    const int64_t* origin3, const int64_t* size3, double* out)
{
    if (G <= 0) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (size3[a] <= 0 || origin3[a] < 0 || origin3[a] + size3[a] > G) return ORC_EINVAL;
    int64_t w0[5][3], wn[5][3];
    for (int l = 0; l <= 4; ++l)
        for (int a = 0; a < 3; ++a) {
            const int64_t grow = 4 - l;
            int64_t lo = origin3[a] - grow, hi = origin3[a] + size3[a] + grow;
            if (lo < 0) lo = 0;
            if (hi > G) hi = G;
            w0[l][a] = lo;
            wn[l][a] = hi - lo;
        }
    double* act[5] = { 0 };
    double* Wd[4] = { 0 };
    double* bd[4] = { 0 };
    int rc = ORC_OK;
    for (int l = 0; l <= 4; ++l) {
        act[l] = (double*)malloc(sizeof(double) * (size_t)(chan[l] * wn[l][0] * wn[l][1] * wn[l][2]));
        if (!act[l]) rc = ORC_ENOMEM;
    }
    for (int l = 0; l < 4; ++l) {
        Wd[l] = (double*)malloc(sizeof(double) * (size_t)(chan[l + 1] * chan[l] * 27));
        bd[l] = (double*)malloc(sizeof(double) * (size_t)chan[l + 1]);
        if (!Wd[l] || !bd[l]) rc = ORC_ENOMEM;
    }
    if (rc == ORC_OK) {
        for (int l = 0; l < 4; ++l) {
            for (int64_t k = 0; k < (int64_t)chan[l + 1] * chan[l] * 27; ++k) Wd[l][k] = (double)w[l][k];
            for (int32_t k = 0; k < chan[l + 1]; ++k) bd[l][k] = (double)b[l][k];
        }
        for (int32_t i = 0; i < chan[0]; ++i)
            for (int64_t z = 0; z < wn[0][0]; ++z)
                for (int64_t y = 0; y < wn[0][1]; ++y)
                    for (int64_t x = 0; x < wn[0][2]; ++x)
                        act[0][(((int64_t)i * wn[0][0] + z) * wn[0][1] + y) * wn[0][2] + x] =
                            (double)vel[(((int64_t)i * G + (w0[0][0] + z)) * G + (w0[0][1] + y)) * G + (w0[0][2] + x)];
        for (int l = 0; l < 4; ++l)
            conv3x3x3(G, act[l], chan[l], w0[l], wn[l], act[l + 1], chan[l + 1], w0[l + 1], wn[l + 1], Wd[l], bd[l],
                      l < 3);
        memcpy(out, act[4], sizeof(double) * (size_t)(chan[4] * size3[0] * size3[1] * size3[2]));
    }
    for (int l = 0; l <= 4; ++l) free(act[l]);
    for (int l = 0; l < 4; ++l) { free(Wd[l]); free(bd[l]); }
    return rc;
}

/*
 * CNN-SNS start element in 3D (Alg. 2): x_hat = clamp(x_i + D, 0, 1) per axis,
 * D the predicted displacement of the overlay cell holding x_i, and K_p the
 * 3D overlay lookup of the cell holding x_hat (fallback[i], else element 0,
 * where that cell has no element).
 *   origin: [n][3]; disp: [3][G][G][G] (x, y, z components); lookup: [G][G][G].
 */
int orc3_cnnsns_start(int64_t n, const double* origin, int32_t G, const double* disp, const int32_t* lookup,
                      const int32_t* fallback, int32_t* start_out)
{
    if (n < 0 || G <= 0) return ORC_EINVAL;
    const int64_t nc = (int64_t)G * G * G;
    for (int64_t i = 0; i < n; ++i) {
        const double* o = origin + 3 * i;
        const int64_t c = (cell_of(o[2], G) * G + cell_of(o[1], G)) * G + cell_of(o[0], G);
        double h[3];
        for (int a = 0; a < 3; ++a) {
            h[a] = o[a] + disp[a * nc + c];
            h[a] = h[a] < 0.0 ? 0.0 : (h[a] > 1.0 ? 1.0 : h[a]);
        }
        int32_t k = lookup[(cell_of(h[2], G) * G + cell_of(h[1], G)) * G + cell_of(h[0], G)];
        if (k < 0) k = fallback ? fallback[i] : 0;
        start_out[i] = k;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The paper's classifier CNN (Sec. 2.3, eq. 7-8, Alg. 2's prediction step), */
/* in 2D on the overlay grid.                                                */
/*
 * Input preparation (Sec. 2.3):
 *  - each element is represented by its centroid (the paper's "barycentric
 *    coordinates" x_l^*): the mean of its vertices, summed with the vertices
 *    in ascending node id, ((x_a + x_b) + x_c) / 3;
 *  - the ASG filter assigns each element to the overlay cell holding its
 *    centroid, and average pooling gives each cell one value: the mean of the
 *    centroids assigned to it (summed in ascending element id, divided by
 *    their count), or the cell centre when none is;
 *  - the filtered region around x_p is the W x W block of cells centred on
 *    the cell of x_p (W = 9, N_a = 81 classes); the padding layer extends the
 *    grid at its boundary (a cell index outside [0, G) takes the nearest
 *    cell's value);
 *  - network input: per window cell, G (pooled centroid - x_p), both
 *    components, rounded to FP32 (channel 0 x, channel 1 y, [2][9][9]); and
 *    x_p's offset in its own cell, x_p G - (cell + 1/2) per axis, rounded to
 *    FP32.
 * Network (Fig. 2's sizes are missing; chosen here): module 1: conv 3x3
 * 2 -> 16, ReLU, conv 3x3 16 -> 16, ReLU (zero "same" padding), 2 x 2 average
 * pooling (stride 2, the last row and column dropped: 4 x 4), flattened in
 * [channel][row][col] order (256); module 2: FC 2 -> h1 = 256, ReLU, FC
 * 256 -> 256, ReLU; concatenation [module 1, module 2] (512); FC 512 -> h2 =
 * 512, ReLU; FC 512 -> N_a = 81: the logits H_l; B_l = softmax(H)_l; the class
 * is the l of the largest B_l, the lowest l on ties (eq. 8's "max" read as
 * argmax).  Class l = (dy + 4) 9 + (dx + 4) is the window cell at offset
 * (dx, dy) from the cell of x_p, and K_p is the overlay lookup element of that
 * cell (clamped to the grid), or the fallback start (else element 0) where the
 * cell has none.
 * Weights are FP32 in PyTorch layouts (conv [out][in][3][3], FC [out][in]),
 * widened exactly to FP64.
 */
#define CLS_W 9
#define CLS_R 4
#define CLS_NA (CLS_W * CLS_W)
#define CLS_C 16
#define CLS_P 4
#define CLS_H1 256
#define CLS_H2 512
#define CLS_F (CLS_C * CLS_P * CLS_P)

static int64_t clamp_cell(int64_t c, int32_t G)
{
    return c < 0 ? 0 : (c >= G ? G - 1 : c);
}

/* centroid of triangle t, vertices summed in ascending node id */
static void centroid_by_id(const double* xy, const int32_t* tri, int64_t t, double c[2])
{
    int32_t v[3] = { tri[3 * t], tri[3 * t + 1], tri[3 * t + 2] };
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (v[j] > v[j + 1]) {
                int32_t s = v[j];
                v[j] = v[j + 1];
                v[j + 1] = s;
            }
    for (int k = 0; k < 2; ++k)
        c[k] = ((xy[2 * (int64_t)v[0] + k] + xy[2 * (int64_t)v[1] + k]) + xy[2 * (int64_t)v[2] + k]) / 3.0;
}

/* The average-pooled ASG grid: pool [G][G][2] (x, y), as described above. */
int orc_cls_pool(int64_t n_nodes, const double* xy, int64_t n_tri, const int32_t* tri, int32_t G, double* pool)
{
    if (n_tri < 0 || G <= 0 || n_nodes < 0) return ORC_EINVAL;
    const int64_t GG = (int64_t)G * G;
    int64_t* count = (int64_t*)calloc((size_t)GG, sizeof(int64_t));
    if (!count) return ORC_ENOMEM;
    for (int64_t k = 0; k < 2 * GG; ++k) pool[k] = 0.0;
    for (int64_t t = 0; t < n_tri; ++t) { /* ascending element id */
        double c[2];
        centroid_by_id(xy, tri, t, c);
        const int64_t cell = cell_of(c[1], G) * G + cell_of(c[0], G);
        pool[2 * cell] += c[0];
        pool[2 * cell + 1] += c[1];
        ++count[cell];
    }
    for (int64_t cy = 0; cy < G; ++cy)
        for (int64_t cx = 0; cx < G; ++cx) {
            const int64_t cell = cy * G + cx;
            if (count[cell] > 0) {
                pool[2 * cell] /= (double)count[cell];
                pool[2 * cell + 1] /= (double)count[cell];
            } else {
                pool[2 * cell] = ((double)cx + 0.5) / (double)G;
                pool[2 * cell + 1] = ((double)cy + 0.5) / (double)G;
            }
        }
    free(count);
    return ORC_OK;
}

/* Network inputs of n points: feat [n][2][9][9] and xoff [n][2], FP32. */
int orc_cls_features(int64_t n, const double* xp, int32_t G, const double* pool, float* feat, float* xoff)
{
    if (n < 0 || G <= 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        const double px = xp[2 * i], py = xp[2 * i + 1];
        const int64_t cx = cell_of(px, G), cy = cell_of(py, G);
        for (int dy = -CLS_R; dy <= CLS_R; ++dy)
            for (int dx = -CLS_R; dx <= CLS_R; ++dx) {
                const int64_t cell = clamp_cell(cy + dy, G) * G + clamp_cell(cx + dx, G);
                const int64_t o = (dy + CLS_R) * CLS_W + (dx + CLS_R);
                feat[(i * 2 + 0) * CLS_NA + o] = (float)((pool[2 * cell] - px) * (double)G);
                feat[(i * 2 + 1) * CLS_NA + o] = (float)((pool[2 * cell + 1] - py) * (double)G);
            }
        xoff[2 * i] = (float)(px * (double)G - ((double)cx + 0.5));
        xoff[2 * i + 1] = (float)(py * (double)G - ((double)cy + 0.5));
    }
    return ORC_OK;
}

/* one 3x3 "same" convolution on a 9 x 9 image, FP64, optional ReLU */
static void cls_conv(const double* x, int cin, const float* w, const float* b, int cout, double* y)
{
    for (int o = 0; o < cout; ++o)
        for (int r = 0; r < CLS_W; ++r)
            for (int c = 0; c < CLS_W; ++c) {
                double s = (double)b[o];
                for (int i = 0; i < cin; ++i)
                    for (int u = 0; u < 3; ++u)
                        for (int v = 0; v < 3; ++v) {
                            const int rr = r + u - 1, cc = c + v - 1;
                            if (rr < 0 || rr >= CLS_W || cc < 0 || cc >= CLS_W) continue;
                            s += (double)w[((o * cin + i) * 3 + u) * 3 + v] * x[(i * CLS_W + rr) * CLS_W + cc];
                        }
                y[(o * CLS_W + r) * CLS_W + c] = s > 0.0 ? s : 0.0;
            }
}

/* a fully connected layer y = W x + b ([out][in] weights), FP64, optional ReLU */
static void cls_fc(const double* x, int nin, const float* w, const float* b, int nout, int relu, double* y)
{
    for (int o = 0; o < nout; ++o) {
        double s = (double)b[o];
        for (int k = 0; k < nin; ++k) s += (double)w[(int64_t)o * nin + k] * x[k];
        y[o] = relu && !(s > 0.0) ? 0.0 : s;
    }
}

/*
 * The classifier on n prepared inputs.  w[0..5] / b[0..5]: conv1, conv2,
 * module-2 FC1, module-2 FC2, FC h2, FC N_a.  Outputs (each may be NULL):
 * logits [n][81] (FP64), prob [n][81] (the softmax, FP64), cls [n].
 */
int orc_cls_forward(int64_t n, const float* feat, const float* xoff, const float* const* w, const float* const* b,
                    double* logits, double* prob, int32_t* cls)
{
    if (n < 0) return ORC_EINVAL;
    int rc = ORC_OK;
#pragma omp parallel
    {
        double* x0 = (double*)malloc(sizeof(double) * 2 * CLS_NA);
        double* y1 = (double*)malloc(sizeof(double) * CLS_C * CLS_NA);
        double* y2 = (double*)malloc(sizeof(double) * CLS_C * CLS_NA);
        double* z = (double*)malloc(sizeof(double) * (CLS_F + CLS_H1));
        double* m1 = (double*)malloc(sizeof(double) * CLS_H1);
        double* h = (double*)malloc(sizeof(double) * CLS_H2);
        double H[CLS_NA], B[CLS_NA];
        if (!x0 || !y1 || !y2 || !z || !m1 || !h) {
#pragma omp atomic write
            rc = ORC_ENOMEM;
        } else {
#pragma omp for schedule(dynamic, 64)
            for (int64_t i = 0; i < n; ++i) {
                for (int k = 0; k < 2 * CLS_NA; ++k) x0[k] = (double)feat[i * 2 * CLS_NA + k];
                /* module 1: two convolutions with ReLU, 2 x 2 average pooling, flattened */
                cls_conv(x0, 2, w[0], b[0], CLS_C, y1);
                cls_conv(y1, CLS_C, w[1], b[1], CLS_C, y2);
                for (int o = 0; o < CLS_C; ++o)
                    for (int r = 0; r < CLS_P; ++r)
                        for (int c = 0; c < CLS_P; ++c) {
                            const double* q = y2 + (o * CLS_W + 2 * r) * CLS_W + 2 * c;
                            z[(o * CLS_P + r) * CLS_P + c] = (((q[0] + q[1]) + q[CLS_W]) + q[CLS_W + 1]) / 4.0;
                        }
                /* module 2: two fully connected layers on x_p's offset */
                const double xo[2] = { (double)xoff[2 * i], (double)xoff[2 * i + 1] };
                cls_fc(xo, 2, w[2], b[2], CLS_H1, 1, m1);
                cls_fc(m1, CLS_H1, w[3], b[3], CLS_H1, 1, z + CLS_F);
                /* fusion: two fully connected layers to the logits */
                cls_fc(z, CLS_F + CLS_H1, w[4], b[4], CLS_H2, 1, h);
                cls_fc(h, CLS_H2, w[5], b[5], CLS_NA, 0, H);
                /* softmax and its argmax (lowest index on ties) */
                double mx = H[0];
                for (int l = 1; l < CLS_NA; ++l)
                    if (H[l] > mx) mx = H[l];
                double sum = 0.0;
                for (int l = 0; l < CLS_NA; ++l) sum += (B[l] = exp(H[l] - mx));
                int best = 0;
                for (int l = 0; l < CLS_NA; ++l) {
                    B[l] /= sum;
                    if (B[l] > B[best]) best = l;
                }
                if (logits) memcpy(logits + i * CLS_NA, H, sizeof(H));
                if (prob) memcpy(prob + i * CLS_NA, B, sizeof(B));
                if (cls) cls[i] = best;
            }
        }
        free(x0); free(y1); free(y2); free(z); free(m1); free(h);
    }
    return rc;
}

/* K_p of each point: the lookup element of its class's window cell (clamped to the grid), else the fallback
 * start (else element 0). */
int orc_cls_start(int64_t n, const double* xp, int32_t G, const int32_t* lookup, const int32_t* cls,
                  const int32_t* fallback, int32_t* start)
{
    if (n < 0 || G <= 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        if (cls[i] < 0 || cls[i] >= CLS_NA) return ORC_EINVAL;
        const int64_t dy = cls[i] / CLS_W - CLS_R, dx = cls[i] % CLS_W - CLS_R;
        const int64_t cell = clamp_cell(cell_of(xp[2 * i + 1], G) + dy, G) * G + clamp_cell(cell_of(xp[2 * i], G) + dx, G);
        int32_t k = lookup[cell];
        if (k < 0) k = fallback ? fallback[i] : 0;
        start[i] = k;
    }
    return ORC_OK;
}

/*
 * Training label of each point (Sec. 2.3: B'_l = 1 for the class of the host
 * K_t found by SNS): the window cell holding the centroid of the host
 * element, its offset from the cell of x_p clamped to the window; -1 where
 * the host is not an element.
 */
int orc_cls_label(int64_t n, const double* xp, int32_t G, const double* xy, int64_t n_tri, const int32_t* tri,
                  const int32_t* host, int32_t* label)
{
    if (n < 0 || G <= 0) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        if (host[i] < 0 || host[i] >= n_tri) {
            label[i] = -1;
            continue;
        }
        double c[2];
        centroid_by_id(xy, tri, host[i], c);
        int64_t dx = cell_of(c[0], G) - cell_of(xp[2 * i], G), dy = cell_of(c[1], G) - cell_of(xp[2 * i + 1], G);
        dx = dx < -CLS_R ? -CLS_R : (dx > CLS_R ? CLS_R : dx);
        dy = dy < -CLS_R ? -CLS_R : (dy > CLS_R ? CLS_R : dy);
        label[i] = (int32_t)((dy + CLS_R) * CLS_W + (dx + CLS_R));
    }
    return ORC_OK;
}
