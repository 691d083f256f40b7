/*
 * cnnsns.h - CNN-accelerated successive-neighbour-search particle location on
 * unstructured 2D triangle meshes, for AMD Instinct MI355X (gfx950).
 *
 * Method: Luo et al., "A CNN-based particle tracking method for large-scale
 * fluid simulations with Lagrangian-Eulerian approaches" (arXiv 2412.18379).
 * For every Lagrangian point x_p the library finds its host element K_t, the
 * mesh element whose closed region contains x_p (Sec. 2.1-2.2).  The search is
 * the successive neighbour search (SNS, Alg. 1, eq. 6): from a start element,
 * compute the barycentric coordinates of x_p, stop when all are >= 0,
 * otherwise step to the neighbour across the edge with the smallest
 * coordinate (eq. 5).  CNN-SNS (Alg. 2) starts the same walk from an element
 * predicted by a CNN instead of the host element before movement.  The
 * paper's elements are tetrahedra; here they are triangles (3 barycentric
 * coordinates, 3 neighbours), and the CNN predicts, for every cell of a
 * G x G overlay grid on the unit square (the auxiliary structured grid of
 * Sec. 1 / Alg. 2), the displacement from a point's position before movement
 * to its departure point, from the Eulerian velocity sampled on that grid.
 *
 * Conventions shared by every call:
 *  - Every function is extern "C", never throws, and returns an int32 status:
 *    CNNSNS_OK (0) or a negative error code.  cnnsns_last_error() returns a
 *    thread-local message describing the last non-OK return of this thread.
 *  - "host" pointers point to CPU memory, "device" pointers to GPU memory of
 *    the device that was current when the mesh was built.  The library never
 *    takes ownership of caller memory; caller buffers passed to asynchronous
 *    calls must stay valid until the stream has been synchronised (predict,
 *    locate) or the job is complete (submit).
 *  - Streams are hipStream_t passed as void* (NULL = the null stream).
 *  - Element ids are the caller's triangle indices (0-based).
 *  - Geometry is FP64 everywhere: the walk's containment and direction tests
 *    are exact IEEE double evaluations with no fused multiply-add, so results
 *    are bitwise reproducible and independent of batching.
 */
#ifndef CNNSNS_H
#define CNNSNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Call-level status codes. */
enum {
    CNNSNS_OK = 0,
    CNNSNS_EINVAL = -1, /* invalid argument (null pointer, negative size, bad enum, ...) */
    CNNSNS_ENOMEM = -2, /* device or host allocation failed, or a memory budget is exceeded */
    CNNSNS_EHIP = -3,   /* a HIP runtime call failed */
    CNNSNS_EMESH = -4,  /* the mesh is invalid (see cnnsns_build_mesh) */
    CNNSNS_EBUSY = -5,  /* the serving queue is full (retry later), or a mesh still has jobs in flight */
};

/* Per-point outcome of a walk (not an error). */
enum {
    CNNSNS_FOUND = 0,    /* host[i] contains x_p (all barycentric coordinates >= 0) */
    CNNSNS_OUTSIDE = 1,  /* the walk reached a boundary edge (neighbour -1): x_p lies outside
                            the mesh (Alg. 1's second exit); host[i] is the last element */
    CNNSNS_MAXITER = 2,  /* max_iter iterations were used up; host[i] is the element reached */
    CNNSNS_BADSTART = 3, /* the start element id was outside [0, n_tri); host[i] = -1, iters 0 */
};

/* CNN arithmetic precision for cnnsns_predict / the serving loop. */
enum {
    CNNSNS_F32 = 0,     /* FP32 operands and activations, FP32 accumulation (the 32 -> 32 layers
                           as Winograd F(2x2,3x3) contractions: within 1e-5 of the exact result) */
    CNNSNS_BF16 = 1,    /* BF16 operands and activations, FP32 accumulation */
    CNNSNS_FP8E4M3 = 2, /* FP8 e4m3 (OCP: 3 mantissa bits, largest finite 448) operands with
                           FP32 accumulation: a power-of-two scale per layer and output channel
                           for the weights, per layer for the activations (cnnsns_predict only:
                           the serving loop and the 3D pass return EINVAL for it) */
};

typedef struct cnnsns_mesh_s* cnnsns_mesh;
typedef struct cnnsns_mesh3_s* cnnsns_mesh3; /* a tetrahedral mesh (the 3D walk) */
typedef struct cnnsns_server_s* cnnsns_server;

/*
 * Weights of the displacement CNN: four 3x3 convolution layers with channel
 * counts 2 -> 32 -> 32 -> 32 -> 2, stride 1, zero "same" padding (the padding
 * layer of Sec. 2.3), bias, and ReLU between layers (Sec. 2.3: after layers
 * 1-3, none after the last).  The operation is cross-correlation:
 *   y[o][r][c] = b[o] + sum_i sum_{dy,dx=-1..1} w[o][i][dy+1][dx+1] * x[i][r+dy][c+dx].
 * w[l] is a DEVICE pointer to FP32 [C_out][C_in][3][3] (OIHW), b[l] a DEVICE
 * pointer to FP32 [C_out].  Lower precisions are derived from these FP32
 * weights by the library on each call.
 */
typedef struct {
    const float* w[4];
    const float* b[4];
} cnnsns_cnn;

/*
 * Build a device-resident mesh: the element list {K_l} and the neighbour
 * table {m_j^l} that the SNS walk reads (Sec. 2.2, eq. 6), plus the overlay
 * lookup lookup[cy][cx] = the smallest id of an element whose closed region
 * contains the cell centre ((cx + 1/2)/G, (cy + 1/2)/G), or -1 when none does
 * (the ASG overlay of Sec. 1 / Alg. 2, over the unit square).
 *
 *   xy           HOST FP64 [n_nodes][2] node coordinates.
 *   tri          HOST int32 [n_tri][3] node indices per triangle, 0-based, any
 *                orientation (the library orders each triangle counter-clockwise;
 *                neighbour j of a triangle is across the edge opposite its
 *                j-th counter-clockwise vertex).
 *   overlay_side G >= 1, or 0 to choose 2^ceil(log2(sqrt(n_tri))).
 *   stream       stream for the upload and build kernels; the call waits for it.
 *   out          receives the handle (owned by the library until cnnsns_destroy_mesh).
 *
 * The inputs are copied; the caller keeps its arrays.  Errors: EINVAL (null
 * pointer, n_nodes < 3, n_tri < 1, overlay_side < 0 or > 65536), EMESH (a
 * node index out of range, a triangle of zero or non-finite area, an edge in more than two
 * triangles, or two triangles that overlap across an edge), ENOMEM, EHIP.
 */
int cnnsns_build_mesh(const double* xy, int64_t n_nodes, const int32_t* tri, int64_t n_tri,
                      int32_t overlay_side, void* stream, cnnsns_mesh* out);

/*
 * Facts about a built mesh; any output pointer may be NULL.  device_bytes is
 * the device memory the handle holds; mean_diam the mean over triangles of
 * the longest edge.
 */
int cnnsns_mesh_info(cnnsns_mesh m, int64_t* n_tri, int32_t* overlay_side, int64_t* device_bytes,
                     double* mean_diam);

/* Free a mesh and its device memory (synchronises the device first). NULL is a
 * no-op.  EBUSY while serving jobs submitted on the mesh are not complete. */
int cnnsns_destroy_mesh(cnnsns_mesh m);

/*
 * CNN forward pass over the mesh's G x G overlay (the prediction step of
 * Alg. 2, in the displacement-regression form described above):
 *   vel   DEVICE FP32 [2][G][G], (u, v) at the cell centres, row = y index.
 *   w     the weights (device pointers, see cnnsns_cnn).
 *   precision  CNNSNS_F32, CNNSNS_BF16 or CNNSNS_FP8E4M3.
 *   disp  DEVICE FP32 [2][G][G] output (caller-owned): predicted (dx, dy).
 * The mesh keeps a workspace for the forward pass, allocated on first use and
 * grown when needed (FP32: one 32-channel FP32 activation of 128 G^2 bytes
 * plus 128 KiB of transformed weights; BF16: 40 KiB of packed weights; FP8:
 * 20 KiB of packed weights and 2 KiB of scales) until it is destroyed.
 * FP8: the weight scale of output channel o of a layer is the smallest power of
 * two s with max|w_o| / s <= 448; the velocity's is that of max|u, v| over the
 * grid (a reduction pass before the forward pass); the scale of the
 * activations after layer l bounds them for any input of that magnitude:
 * P_l = max_o (1.25 sum_{i,t} |w_oit| P_{l-1} + |b_o|) with P_0 = max|u, v|,
 * scale the smallest power of two s with P_l / s <= 448.  Values are rounded
 * to nearest even; none can exceed the format.  Passes on one mesh share it: a pass is ordered on the
 * device after the previous pass on that mesh, also across streams and
 * threads (growing it synchronises the device).  Asynchronous on `stream`.
 * Errors: EINVAL (an unknown precision before any allocation), ENOMEM, EHIP.
 */
int cnnsns_predict(cnnsns_mesh m, const float* vel, const cnnsns_cnn* w, int32_t precision, float* disp,
                   void* stream);

/*
 * cnnsns_predict for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same forward pass, same kernels and same results, with its workspace
 * in a preallocated array of 32 MiB + 128 KiB per GPU that the library holds until the
 * process ends, instead of the mesh's workspace.  Makes no hipMalloc,
 * hipFree or other allocating call.  Every call on one GPU uses that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and give wrong results; a call may follow another on the same stream.
 *   precision  CNNSNS_F32 (workspace 128 G^2 bytes + 128 KiB: G <= 512),
 *              CNNSNS_BF16 (40 KiB: any G) or CNNSNS_FP8E4M3 (22 KiB: any G).
 * Other arguments as in cnnsns_predict.  Asynchronous on `stream`.  Errors:
 * EINVAL (null argument, precision, or a workspace beyond the array's
 * size), EHIP.
 */
int cnnsns_predict_noalloc(cnnsns_mesh m, const float* vel, const cnnsns_cnn* w, int32_t precision, float* disp,
                           void* stream);

/*
 * Weights of the paper's classifier CNN (Sec. 2.3, Fig. 2), as DEVICE FP32
 * arrays in PyTorch layouts:
 *   w[0] conv1 [16][2][3][3],   b[0] [16]   module 1: 3x3, zero padding, ReLU
 *   w[1] conv2 [16][16][3][3],  b[1] [16]   then ReLU and 2 x 2 average pooling
 *   w[2] fc    [256][2],        b[2] [256]  module 2 (x_p): FC, ReLU (h1 = 256)
 *   w[3] fc    [256][256],      b[3] [256]  FC, ReLU
 *   w[4] fc    [512][512],      b[4] [512]  [module 1 (256), module 2 (256)]: FC, ReLU (h2 = 512)
 *   w[5] fc    [81][512],       b[5] [81]   the logits of the N_a = 81 classes
 */
typedef struct {
    const float* w[6];
    const float* b[6];
} cnnsns_cls;

/*
 * The prediction step of Alg. 2 with the paper's classifier CNN (Sec. 2.3,
 * eq. 7-8), per point, in 2D on the mesh's G x G overlay.  The element data
 * fed to the network are the elements' centroids (vertices summed in
 * ascending node id, divided by 3); each overlay cell holds the mean of the
 * centroids lying in it (average pooling, summed in ascending element id), or
 * its centre when none does, built once per mesh on the first call (16 G^2
 * bytes, counted in the mesh's device bytes).  For a point x_p the network
 * sees the 9 x 9 cells centred on the cell of x_p (cells outside the grid
 * take the nearest cell's value: the padding layer), as G (cell value - x_p)
 * in two channels, and x_p's offset in its own cell, x_p G - (cell + 1/2),
 * both formed in FP64 and rounded to FP32; the network itself runs in FP32
 * (convolutions and the fully connected layers on the matrix cores).  The
 * class is the argmax of the 81 logits (the softmax of eq. 7 does not change
 * it; ties go to the lowest class); class (dy + 4) 9 + (dx + 4) is the window
 * cell at offset (dx, dy) from the cell of x_p, clamped to the grid, and the
 * start element K_p is that cell's overlay lookup element.  The walk is then
 * cnnsns_locate with these starts (Alg. 2's SNS from K_p).  DEVICE arrays:
 *   xp        FP64 [n][2] the points x_p.
 *   w         the weights (device pointers).
 *   fallback  int32 [n] start where the chosen cell has no element, or NULL
 *             (then element 0).
 *   start     int32 [n] output K_p.
 *   cls       int32 [n] output class, or NULL.
 *   logits    FP32 [n][81] output logits, or NULL.
 * Uses a workspace of the mesh (at most 4.4 KB per point, for up to 65,536
 * points at a time), ordered after the previous classification on the mesh
 * like cnnsns_predict.  Asynchronous on `stream` (the first call on a mesh
 * synchronises it once, to build the pooled grid).  n == 0 is a no-op.
 * Errors: EINVAL (null mesh, weights, xp or start, n < 0), ENOMEM, EHIP.
 */
int cnnsns_classify(cnnsns_mesh m, int64_t n, const double* xp, const cnnsns_cls* w, const int32_t* fallback,
                    int32_t* start, int32_t* cls, float* logits, void* stream);

/*
 * Locate n points (Alg. 1 for every point; Alg. 2 when a displacement grid is
 * given).  All arrays are DEVICE memory:
 *   xp      FP64 [n][2] query points x_p (departure points).
 *   start   int32 [n] start elements, or NULL.
 *   origin  FP64 [n][2] positions before movement x_i, or NULL.
 *   disp    FP32 [2][G][G] predicted displacements (from cnnsns_predict), or NULL.
 *   max_iter  iteration cap per point; <= 0 selects 2^20.
 *   host    int32 [n] output host element ids.
 *   iters   int32 [n] output path lengths I_t (Alg. 1's counter; 1 when the
 *           start contains x_p), or NULL.
 *   status  uint8 [n] output per-point outcome (CNNSNS_FOUND ...), or NULL.
 * Start element per point:
 *   disp and origin given (CNN-SNS, Alg. 2): x_hat = clamp(x_i + D, 0, 1) with
 *     D the displacement of the overlay cell holding x_i, and the start is the
 *     overlay lookup of the cell holding x_hat; if that cell has no element,
 *     start[i] when start is given, else element 0.  Cell of a coordinate:
 *     min(G-1, max(0, floor(coord * G))).
 *   else start given (plain SNS, Alg. 1 from K_m): start[i].
 *   else (neither): the overlay lookup of the cell holding x_p itself (the
 *     ASG locator of Sec. 1), element 0 where that cell has no element.
 * Asynchronous on `stream`.  n == 0 is a no-op.  Errors: EINVAL (null mesh,
 * xp or host, n < 0, disp without origin), EHIP.
 */
int cnnsns_locate(cnnsns_mesh m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                  const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status,
                  void* stream);

/*
 * Interpolate a nodal field at located points: the step the host element is
 * found for (Sec. 2.1, the approximation after eq. 4).  For point i with host
 * element K = host[i] and its nodes n_0, n_1, n_2 (in the counter-clockwise
 * order the library stores), the value is sum_j lambda_j nodal[n_j], where
 * lambda_j = s_j / |S_0| are the barycentric coordinates of Sec. 2.2 (s_j the
 * numerators of cnnsns_locate, |S_0| the doubled element area), i.e. the P1
 * (linear) interpolant, exact for fields linear in x and y.  All arrays are
 * DEVICE memory:
 *   xp     FP64 [n][2] the points (as given to cnnsns_locate).
 *   host   int32 [n] their host elements (as returned by cnnsns_locate).
 *   nodal  FP64 [n_nodes][2] the field at the mesh nodes (node ids of
 *          cnnsns_build_mesh), e.g. the Eulerian velocity u(n_j).
 *   out    FP64 [n][2] output.
 * FP64 with no fused multiply-add; the sum runs over j = 0, 1, 2 in order.  A
 * host id outside [0, n_tri) (a BADSTART point) gives NaN; for an OUTSIDE
 * point (x_p beyond the mesh, host = the boundary element reached) the same
 * formula extrapolates.  Asynchronous on `stream`; n == 0 is a no-op.
 * Errors: EINVAL (null mesh or array, n < 0), EHIP.
 */
int cnnsns_interpolate(cnnsns_mesh m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                       double* out, void* stream);

/*
 * cnnsns_locate followed, in the same pass, by the interpolation of
 * cnnsns_interpolate at each point's x_p in the host the walk ends in (the
 * step after eq. 4 of Sec. 2.1, fused into the walk's final iteration: the
 * barycentric numerators of that iteration are reused, so x_p, the host and
 * the element's coordinates are not read again).  Arguments as in
 * cnnsns_locate, plus (DEVICE, as in cnnsns_interpolate):
 *   nodal  FP64 [n_nodes][2] the field at the mesh nodes.
 *   out    FP64 [n][2] output: sum_j lambda_j nodal[n_j], bit for bit what
 *          cnnsns_interpolate returns for the same host (NaN for BADSTART).
 * Asynchronous on `stream`.  n == 0 is a no-op.  Errors: those of
 * cnnsns_locate, and EINVAL for a NULL nodal or out.
 */
int cnnsns_locate_interpolate(cnnsns_mesh m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                              const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status,
                              const double* nodal, double* out, void* stream);

/*
 * Build a device-resident tetrahedral mesh for the 3D walk (the paper's own
 * setting: Sec. 2.2 with four nodes and four neighbours per element).
 *   xyz          HOST FP64 [n_nodes][3] node coordinates.
 *   tet          HOST int32 [n_tet][4] node indices per tetrahedron, 0-based,
 *                either orientation (the library makes det[b-a, c-a, d-a] > 0
 *                by swapping the 3rd and 4th node where it is negative;
 *                neighbour j is across the face opposite the j-th node).
 *   overlay_side G >= 1 for a G x G x G overlay lookup over the unit cube
 *                (cell centre ((c + 1/2) / G per axis -> the smallest id of a
 *                tetrahedron containing it, -1 if none), or 0 to choose
 *                2^ceil(log2(cbrt(n_tet))) (at most 1024).
 *   stream       stream for the upload and build kernels; the call waits for it.
 *   out          receives the handle (owned by the library until
 *                cnnsns_destroy_mesh3d).
 * Inputs are copied.  Errors: EINVAL (null pointer, n_nodes < 4, n_tet < 1,
 * overlay_side < 0 or > 1024), EMESH (a node index out of range, a
 * tetrahedron of zero or non-finite volume, a face in more than two tetrahedra, or two
 * tetrahedra overlapping across a face), ENOMEM, EHIP.
 */
int cnnsns_build_mesh3d(const double* xyz, int64_t n_nodes, const int32_t* tet, int64_t n_tet, int32_t overlay_side,
                        void* stream, cnnsns_mesh3* out);

/* Facts about a tetrahedral mesh; any output pointer may be NULL. */
int cnnsns_mesh3d_info(cnnsns_mesh3 m, int64_t* n_tet, int32_t* overlay_side, int64_t* device_bytes);

/* Free a tetrahedral mesh (synchronises the device first).  NULL is a no-op. */
int cnnsns_destroy_mesh3d(cnnsns_mesh3 m);

/*
 * The 3D displacement CNN (Sec. 2.3 with 3 x 3 x 3 kernels) on the mesh's
 * G x G x G overlay: 3 -> 32 -> 32 -> 32 -> 3 channels, zero padding of one
 * cell, bias, ReLU after layers 1-3, cross-correlation.  DEVICE arrays:
 *   vel   FP32 [3][G][G][G] (component, z, y, x) velocity at the cell centres.
 *   w     weights as in cnnsns_predict, with 3 x 3 x 3 kernels: w[0] FP32
 *         [32][3][3][3][3], w[1], w[2] [32][32][3][3][3], w[3] [3][32][3][3][3]
 *         (OIDHW); b[0..2] [32], b[3] [3].
 *   precision  CNNSNS_F32, or CNNSNS_BF16: layers 2 and 3 with BF16 weights
 *              and activations (rounded to nearest even) on the matrix cores,
 *              FP32 accumulation; layer 1 writes BF16 activations and layer 4
 *              reads them, both computing in FP32.  CNNSNS_FP8E4M3: EINVAL.
 *   disp  FP32 [3][G][G][G] out: the predicted displacement per cell.
 * Uses a workspace of the mesh (2 G^3 x 32 FP32 activations plus 216 KiB),
 * allocated on the first call; a pass is ordered on the device after the
 * previous pass on that mesh, also across streams.
 * Asynchronous on `stream`.  Errors: EINVAL (null argument, precision not
 * CNNSNS_F32 or CNNSNS_BF16), ENOMEM (workspace), EHIP.
 */
int cnnsns_predict3d(cnnsns_mesh3 m, const float* vel, const cnnsns_cnn* w, int32_t precision, float* disp,
                     void* stream);

/*
 * Locate n points in a tetrahedral mesh (Alg. 1 with four barycentric
 * coordinates).  The numerator of coordinate j is the volume determinant of
 * the tetrahedron with node j replaced by x_p, det[F - p] over the other three
 * nodes F taken in node-id order with the sign of that permutation applied,
 * so both tetrahedra of a face compute it identically; containment is closed
 * (all >= 0), the smallest coordinate picks the face (ties to the lowest j of
 * the positively oriented node order) and the walk steps across it.  DEVICE
 * arrays:
 *   xp      FP64 [n][3] query points.
 *   start   int32 [n] start elements (plain SNS), or NULL.
 *   origin  FP64 [n][3] positions before movement x_i, with disp, or NULL.
 *   disp    FP32 [3][G][G][G] from cnnsns_predict3d, or NULL.  With disp the
 *           start is CNN-SNS (Alg. 2): the overlay lookup of the cell holding
 *           clamp(x_i + D[cell(x_i)], 0, 1), or start[i] (else element 0)
 *           where that cell has no element.  Without disp and start: the
 *           overlay lookup of the cell holding x_p (element 0 for an empty
 *           cell).  Cell of a coordinate: min(G-1, max(0, floor(x G))).
 *   max_iter, host, iters, status as in cnnsns_locate.
 * Asynchronous on `stream`.  n == 0 is a no-op.  Errors: EINVAL (null mesh,
 * xp or host, n < 0, disp without origin), EHIP.
 */
int cnnsns_locate3d(cnnsns_mesh3 m, int64_t n, const double* xp, const int32_t* start, const double* origin,
                    const float* disp, int32_t max_iter, int32_t* host, int32_t* iters, uint8_t* status, void* stream);

/*
 * P1 interpolation of a nodal field at points in their host tetrahedra
 * (Sec. 2.1 after eq. 4; the nodal basis functions are the barycentric
 * coordinates of Sec. 2.2): u(x_p) = sum_j (s_j / V) u(n_j), with s_j the
 * numerators of cnnsns_locate3d and V six times the element's volume,
 * evaluated with the nodes in ascending id, the sum taken over the nodes in
 * ascending id (FP64, no fused multiply-add).  DEVICE arrays:
 *   xp     FP64 [n][3] points.
 *   host   int32 [n] host tetrahedra (from cnnsns_locate3d); an id outside
 *          [0, n_tet) gives NaN in all three components.
 *   nodal  FP64 [n_nodes][3] field values at the mesh nodes.
 *   out    FP64 [n][3] interpolated values.
 * Asynchronous on `stream`.  n == 0 is a no-op.  Errors: EINVAL (null mesh or
 * array, n < 0), EHIP.
 */
int cnnsns_interpolate3d(cnnsns_mesh3 m, int64_t n, const double* xp, const int32_t* host, const double* nodal,
                         double* out, void* stream);

/*
 * Serving loop: a host scheduler that takes CNN-SNS tracking jobs on
 * resident meshes as they arrive and runs them with continuous batching.
 * Each job is one CNN forward pass over its mesh's overlay (in `precision`)
 * followed by the CNN-SNS locate of its points, exactly as cnnsns_predict +
 * cnnsns_locate would compute them (results do not depend on what else is
 * in flight).  Jobs are admitted in arrival order while their device
 * footprint (the displacement grid and CNN activations) fits in
 * hbm_budget_bytes and fewer than max_inflight jobs are running; admitted
 * jobs run concurrently on several streams.
 *   hbm_budget_bytes  budget for per-job device memory (> 0).
 *   max_inflight      jobs on the device at once (>= 1).
 *   queue_depth       jobs waiting for admission at most (>= 1).
 *   w                 CNN weights (device pointers; copied at creation).
 * Switched off: returns EINVAL unless the environment variable
 * CNNSNS_ENABLE_SERVING is "1", because runs of the serving loop on the GPU
 * have occasionally ended in a host-side segmentation fault whose cause has
 * not been found.
 */
int cnnsns_server_create(int64_t hbm_budget_bytes, int32_t max_inflight, int32_t queue_depth,
                         int32_t precision, const cnnsns_cnn* w, cnnsns_server* out);

/*
 * Submit a job: locate n points of mesh m whose overlay velocity is vel
 * (DEVICE FP32 [2][G][G]), with x_p = xp (DEVICE FP64 [n][2]) and positions
 * before movement origin (DEVICE FP64 [n][2]); results go to host / iters
 * (DEVICE int32 [n], iters may be NULL).  start (DEVICE int32 [n]) may be
 * NULL; it is only the fallback for uncovered overlay cells.  With n == 0
 * the point buffers may be NULL (the job is the forward pass alone).
 *   stream  the caller's stream (NULL = the null stream): the job runs after
 *           the work enqueued on it before this call (an event is recorded
 *           on it here), so inputs and output buffers written there are
 *           ready; to consume the results, wait for completion (poll/wait).
 * Buffers and the mesh must stay valid until the job completes; while a
 * mesh has jobs that are not complete, cnnsns_destroy_mesh refuses it
 * (EBUSY).  Returns at once with *job_id.  Errors: EINVAL, EBUSY (queue
 * full), ENOMEM (the job alone exceeds the budget), EHIP.
 */
int cnnsns_submit(cnnsns_server s, cnnsns_mesh m, const float* vel, int64_t n, const double* xp,
                  const double* origin, const int32_t* start, int32_t* host, int32_t* iters, void* stream,
                  uint64_t* job_id);

/*
 * Completion of a job: *done = 1 when its results are in device memory.
 * latency_ms (may be NULL) gets submit-to-completion time once done.
 */
int cnnsns_poll(cnnsns_server s, uint64_t job_id, int32_t* done, double* latency_ms);

/* Block until the job is complete. */
int cnnsns_wait(cnnsns_server s, uint64_t job_id, double* latency_ms);

/* Drain every submitted job, then free the server.  NULL is a no-op. */
int cnnsns_server_destroy(cnnsns_server s);

/* Message for the last non-OK return on the calling thread ("" if none). */
const char* cnnsns_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CNNSNS_H */
