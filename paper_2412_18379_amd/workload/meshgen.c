/*
 * Seeded synthetic mesh generation: triangulation of a (jittered, possibly
 * graded) n x n point grid on the unit square, made Delaunay by Lawson edge
 * flips.  This is input generation only; it is used to produce the meshes
 * that both the located-point library and its checker receive, and it holds
 * none of the point-location arithmetic.
 *
 * Build: gcc -O2 -shared -fPIC meshgen.c -o _meshgen.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* > 0 when d lies strictly inside the circumcircle of the CCW triangle abc. */
static long double incircle(const double* a, const double* b, const double* c, const double* d)
{
    long double adx = (long double)a[0] - d[0], ady = (long double)a[1] - d[1];
    long double bdx = (long double)b[0] - d[0], bdy = (long double)b[1] - d[1];
    long double cdx = (long double)c[0] - d[0], cdy = (long double)c[1] - d[1];
    long double ad = adx * adx + ady * ady;
    long double bd = bdx * bdx + bdy * bdy;
    long double cd = cdx * cdx + cdy * cdy;
    return adx * (bdy * cd - bd * cdy) - ady * (bdx * cd - bd * cdx) + ad * (bdx * cdy - bdy * cdx);
}

static double orient(const double* a, const double* b, const double* c)
{
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

/*
 * Two CCW triangles per grid cell, cells in row-major order (y outer).  The
 * cell diagonal is the one that is locally Delaunay for the cell's quad.
 * Node (i, j) (x index i, y index j) is node j*n + i.
 */
int mg_triangulate_grid(int32_t n, const double* xy, int32_t* tri)
{
    if (n < 2) return -1;
    int64_t t = 0;
    for (int32_t j = 0; j + 1 < n; ++j) {
        for (int32_t i = 0; i + 1 < n; ++i) {
            int32_t p00 = j * n + i, p10 = p00 + 1, p01 = p00 + n, p11 = p01 + 1;
            const double *a = xy + 2 * (int64_t)p00, *b = xy + 2 * (int64_t)p10;
            const double *c = xy + 2 * (int64_t)p11, *d = xy + 2 * (int64_t)p01;
            /* main diagonal p00-p11 vs anti-diagonal p10-p01; a diagonal is
               usable when both of its triangles are CCW (always true for at
               least one of them in a simple quad) */
            int main_ok = orient(a, b, c) > 0 && orient(a, c, d) > 0;
            int anti_ok = orient(a, b, d) > 0 && orient(b, c, d) > 0;
            int main_diag = main_ok;
            if (main_ok && anti_ok) main_diag = !(incircle(a, b, c, d) > 0);
            if (main_diag) {
                tri[3 * t + 0] = p00; tri[3 * t + 1] = p10; tri[3 * t + 2] = p11; ++t;
                tri[3 * t + 0] = p00; tri[3 * t + 1] = p11; tri[3 * t + 2] = p01; ++t;
            } else {
                tri[3 * t + 0] = p00; tri[3 * t + 1] = p10; tri[3 * t + 2] = p01; ++t;
                tri[3 * t + 0] = p10; tri[3 * t + 1] = p11; tri[3 * t + 2] = p01; ++t;
            }
        }
    }
    return 0;
}

/* Edge-adjacency: nbr[3t+j] = triangle across the edge opposite vertex j, or -1. */
static int build_adjacency(int64_t nv, int64_t nt, const int32_t* tri, int32_t* nbr)
{
    int64_t* start = (int64_t*)calloc((size_t)nv + 1, sizeof(int64_t));
    int32_t* inc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * nt));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nv + 1));
    if (!start || !inc || !fill) { free(start); free(inc); free(fill); return -2; }
    for (int64_t k = 0; k < 3 * nt; ++k) start[tri[k] + 1]++;
    for (int64_t v = 0; v < nv; ++v) start[v + 1] += start[v];
    memcpy(fill, start, sizeof(int64_t) * (size_t)(nv + 1));
    for (int64_t t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j) inc[fill[tri[3 * t + j]]++] = (int32_t)t;
    int rc = 0;
    for (int64_t t = 0; t < nt && rc == 0; ++t) {
        for (int j = 0; j < 3; ++j) {
            int32_t u = tri[3 * t + (j + 1) % 3], v = tri[3 * t + (j + 2) % 3];
            int32_t found = -1;
            for (int64_t k = start[u]; k < start[u + 1]; ++k) {
                int32_t s = inc[k];
                if (s == t) continue;
                const int32_t* S = tri + 3 * (int64_t)s;
                if (S[0] == v || S[1] == v || S[2] == v) {
                    if (found >= 0) { rc = -3; break; }
                    found = s;
                }
            }
            nbr[3 * t + j] = found;
        }
    }
    free(start); free(inc); free(fill);
    return rc;
}

/*
 * Lawson flipping until every interior edge is locally Delaunay.  tri must be
 * a valid CCW triangulation; it is modified in place (triangle count and ids
 * are kept).  Returns 0 on success, <0 on failure; *nflips gets the count.
 */
int mg_lawson(int64_t nv, const double* xy, int64_t nt, int32_t* tri, int64_t* nflips)
{
    int32_t* nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(3 * nt));
    if (!nbr) return -2;
    int rc = build_adjacency(nv, nt, tri, nbr);
    if (rc) { free(nbr); return rc; }
    int64_t cap = 3 * nt + 16, top = 0;
    int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    if (!stack) { free(nbr); return -2; }
    for (int64_t t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j)
            if (nbr[3 * t + j] > t) stack[top++] = 3 * t + j;
    int64_t flips = 0, limit = 20 * nt + 1000;
    while (top > 0) {
        int64_t e = stack[--top];
        int64_t t = e / 3;
        int j = (int)(e % 3);
        int32_t t2 = nbr[e];
        if (t2 < 0) continue;
        int32_t* T1 = tri + 3 * t;
        int32_t* T2 = tri + 3 * (int64_t)t2;
        int j2 = -1;
        for (int k = 0; k < 3; ++k)
            if (nbr[3 * (int64_t)t2 + k] == t) j2 = k;
        if (j2 < 0) { rc = -4; break; }
        int32_t p = T1[j], u = T1[(j + 1) % 3], v = T1[(j + 2) % 3], q = T2[j2];
        if (incircle(xy + 2 * (int64_t)p, xy + 2 * (int64_t)u, xy + 2 * (int64_t)v, xy + 2 * (int64_t)q) <= 0)
            continue;
        /* convexity of the quad p,u,q,v is implied for a valid triangulation; check anyway */
        if (orient(xy + 2 * (int64_t)p, xy + 2 * (int64_t)u, xy + 2 * (int64_t)q) <= 0 ||
            orient(xy + 2 * (int64_t)q, xy + 2 * (int64_t)v, xy + 2 * (int64_t)p) <= 0)
            continue;
        int32_t A = nbr[3 * t + (j + 1) % 3];            /* edge v-p */
        int32_t B = nbr[3 * t + (j + 2) % 3];            /* edge p-u */
        int32_t C = nbr[3 * (int64_t)t2 + (j2 + 1) % 3]; /* edge u-q */
        int32_t D = nbr[3 * (int64_t)t2 + (j2 + 2) % 3]; /* edge q-v */
        T1[0] = p; T1[1] = u; T1[2] = q;
        T2[0] = q; T2[1] = v; T2[2] = p;
        nbr[3 * t + 0] = C; nbr[3 * t + 1] = t2; nbr[3 * t + 2] = B;
        nbr[3 * (int64_t)t2 + 0] = A; nbr[3 * (int64_t)t2 + 1] = (int32_t)t; nbr[3 * (int64_t)t2 + 2] = D;
        if (A >= 0)
            for (int k = 0; k < 3; ++k)
                if (nbr[3 * (int64_t)A + k] == t) nbr[3 * (int64_t)A + k] = t2;
        if (C >= 0)
            for (int k = 0; k < 3; ++k)
                if (nbr[3 * (int64_t)C + k] == t2) nbr[3 * (int64_t)C + k] = (int32_t)t;
        if (top + 4 > cap) { rc = -5; break; }
        stack[top++] = 3 * t + 0;
        stack[top++] = 3 * t + 2;
        stack[top++] = 3 * (int64_t)t2 + 0;
        stack[top++] = 3 * (int64_t)t2 + 2;
        if (++flips > limit) { rc = -6; break; }
    }
    if (nflips) *nflips = flips;
    free(stack); free(nbr);
    return rc;
}
