/*
 * gl_dca.h -- C ABI of the MI355X (gfx950) preconditioned-DCA library for the
 * graph Ginzburg-Landau model of Shen, Sun and Tai, "Preconditioned Algorithm
 * for Difference of Convex Functions with applications to Graph
 * Ginzburg-Landau Model" (arXiv 2303.14495).  Citations name the paper's
 * sections, propositions (Prop. 1: the preconditioned iteration of the
 * proximal DCA; Prop. 3: 2I >= L_s), Lemma 1 (step size k) and Theorem 1
 * (energy decay).
 *
 * The library computes the inner linear solve of every DCA step,
 *     (eps L_s + eta Lambda + c I) u^{t+1} = c u^t - (u^t^3 - u^t)/eps + eta Lambda y,
 * by a fixed number of diagonal-preconditioned sweeps (Section 3, Prop. 1,
 * and Section 3.1), on the normalized graph Laplacian
 * L_s = I - D^{-1/2} W D^{-1/2} (Section 2.2), for an N x K label field.
 *
 * Conventions shared by every entry point
 *   - Pointers named "device" point to GPU memory on the current HIP device;
 *     pointers named "host" point to CPU memory.  The caller owns every buffer
 *     it passes; the library never frees a caller buffer.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls that do not say otherwise only enqueue work on `stream` and
 *     return without synchronising.
 *   - Dense N x K arrays are row-major: element (i, k) at i*K + k, and must be
 *     16-byte aligned.
 *   - Every entry point returns a gl_status; nothing aborts or throws across
 *     the ABI.  On a non-OK status, gl_last_error() returns a message for the
 *     calling thread.  Argument checks happen on the host before any launch.
 *   - Arithmetic: storage in F64/F32/BF16/F16; accumulation in F32 (F64 when
 *     the field is stored in F64).  BF16/F16 stores round to nearest even.
 *   - Reductions have a fixed order: two runs with the same inputs give
 *     bitwise identical outputs.
 */
#ifndef GL_DCA_H
#define GL_DCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gl_status {
    GL_OK = 0,
    GL_E_INVALID_ARG = 1,  /* a pointer, size, parameter or alignment is invalid */
    GL_E_BAD_GRAPH = 2,    /* CSR malformed, not symmetric, self-loop, bad weight or degree */
    GL_E_DTYPE = 3,        /* unsupported storage type or combination */
    GL_E_NOMEM = 4,        /* a device or pinned-host allocation failed */
    GL_E_BUDGET = 5,       /* (server) request larger than the HBM budget */
    GL_E_NONFINITE = 6,    /* (server) a residual or energy became NaN/Inf */
    GL_E_HIP = 7,          /* a HIP runtime call failed */
    GL_E_QUEUE_FULL = 8,   /* (server) the pending queue is full */
    GL_E_NOT_READY = 9,    /* (server) the result is not ready yet */
    GL_E_CANCELLED = 10    /* (server) the request was cancelled */
} gl_status;

typedef enum gl_dtype { GL_F64 = 0, GL_F32 = 1, GL_BF16 = 2, GL_F16 = 3 } gl_dtype;

/* Diagonal preconditioners G for T = eps L_s + eta Lambda + c I (Section 3.1):
 *   DAMPED_JACOBI     G_Jd,s = 2(eps + c + eta Lambda)
 *   PERTURBED_JACOBI  G_Jp,s = 2 eps + c + eta Lambda + delta0
 *   RICHARDSON        G_R,s  = eps lambda_max + c + eta Lambda + delta0
 * and, for a finite step size k, the preconditioners of T_k = I + k T of the
 * same section (G_Jd,ks, G_Jp,ks, G_R,ks).  With the unnormalized Laplacian
 * (T = eps L + eta Lambda + c I) the same names select G_Jd = 2(eps D + eta
 * Lambda + c), G_Jp = 2 eps D + eta Lambda + c + delta0, G_R = eps lambda_max
 * + eta Lambda + c + delta0 and their step-size-k versions G_Jd,k, G_Jp,k,
 * G_R,k (Section 3.1). */
typedef enum gl_precond {
    GL_PC_DAMPED_JACOBI = 0,
    GL_PC_PERTURBED_JACOBI = 1,
    GL_PC_RICHARDSON = 2
} gl_precond;

/* Storage layout of the operator (chosen once, at creation, from the graph
 * alone, so every K and every solve sums each row in the same order).
 *   AUTO    tile layout when `order` is given and every block of 256 rows
 *           references few enough distinct columns, else direct
 *   DIRECT  CSR rows (in `order`, if given) with 32-bit columns; gathers from
 *           global memory
 *   TILE    rows in `order` cut into blocks of 256; each block's distinct
 *           columns (its halo) are staged in LDS and every entry stores a
 *           16-bit index into the halo; rows padded to 4-entry multiples.
 *           Fails with GL_E_INVALID_ARG when a halo exceeds the limit. */
typedef enum gl_layout {
    GL_LAYOUT_AUTO = 0,
    GL_LAYOUT_DIRECT = 1,
    GL_LAYOUT_TILE = 2,
    GL_LAYOUT_WINDOW = 3, /* reported for operators of gl_window_operator_create; not a request */
    GL_LAYOUT_GRID = 4    /* nodes are the pixels of a grid_height x grid_width image (see gl_graph) */
} gl_layout;

/* Graph Laplacian of the operator (Section 2.2):
 *   NORMALIZED    L_s = I - D^{-1/2} W D^{-1/2} (the default);
 *   UNNORMALIZED  L = D - W.  The operator stores w_ij rounded to its storage
 *                 type and, as the diagonal, the row sums of those stored
 *                 weights (so L 1 = 0 holds for the weights the sweeps use). */
typedef enum gl_laplacian { GL_LAP_NORMALIZED = 0, GL_LAP_UNNORMALIZED = 1 } gl_laplacian;

/* Weighted undirected graph in CSR form (Section 2.2), device memory.
 *   row_ptr  int64 [n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col_idx  int32 [nnz], strictly increasing within a row, in [0, n),
 *            no self-loops (w_ii = 0, so diag(L_s) = 1)
 *   weight   [nnz] of weight_dtype (GL_F64 or GL_F32), finite, > 0,
 *            symmetric: w_ij == w_ji bit for bit with the same pattern
 *   order    int32 [n] or NULL: a permutation of 0..n-1 giving the order in
 *            which rows are processed (position p handles node order[p]).
 *            It changes nothing in the result but the rounding order of the
 *            sums; a locality-preserving order (e.g. the Z-order of an image's
 *            pixel grid) lets the tile layout keep each block's gathers in LDS.
 *            The operator is renumbered into this order: its sweeps read and
 *            write the field in position order, and gl_solve,
 *            gl_laplacian_apply, gl_power_max_eig and gl_time_sweeps move
 *            their node-ordered inputs and outputs in and out once per call
 *            (their workspaces grow accordingly).
 *   layout   gl_layout request.
 *   laplacian gl_laplacian: L_s or L.
 *   grid_height, grid_width  for GL_LAYOUT_GRID: node i is the pixel
 *            (i / grid_width, i % grid_width) of an image (n = height *
 *            width) and every edge joins pixels at most 7 rows and 7 columns
 *            apart (within the paper's default 15 x 15 search window, Section
 *            2.2); 0 otherwise.  The grid layout stores, per pixel, its
 *            entries as one byte of window offset (dy, dx) and the weight, in
 *            chunks of 8, and stages each 64 x 8 pixel tile's 15 x 15 window
 *            halo of the field in LDS; it takes no `order` and is built on
 *            the device.  One call with K
 *            columns needs K * 78 * 22 * (field element size: 2, 4 or 8
 *            bytes) <= 147456 of LDS and 22 * grid_width * K * (element
 *            size) < 2^32 bytes, both checked per call (GL_E_INVALID_ARG);
 *            grid_width < 2^24.
 * Every degree d_i = sum_j w_ij must be > 0. */
typedef struct gl_graph {
    int64_t n;
    int64_t nnz;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    const void *weight;
    gl_dtype weight_dtype;
    const int32_t *order;
    int32_t layout;
    int32_t laplacian;
    int32_t grid_height;
    int32_t grid_width;
} gl_graph;

/* Solver parameters (Section 3 and Section 3.1).
 *   eps > 0, c > 0, eta >= 0: the model's diffuse parameter, the convex-split
 *     constant and the fidelity weight;
 *   delta0 >= 0: the perturbation of G_Jp,s and G_R,s;
 *   lambda_max > 0: the estimate of the largest eigenvalue of the operator's
 *     Laplacian (L_s: at most 2; L: at most 2 max d_i, Prop. 3) used by
 *     RICHARDSON (see gl_power_max_eig), ignored otherwise; it must not be
 *     below the true largest eigenvalue for G_R to be feasible;
 *   step_k: INFINITY for the DCA without step size (Prop. 1), or a finite
 *     k > 0 for the step-size form T_k u = b_k, T_k = I + k T,
 *     b_k = u^t + k b^t (Lemma 1);
 *   outer_steps >= 0 DCA steps of inner_sweeps >= 1 sweeps each. */
typedef struct gl_params {
    double eps;
    double c;
    double eta;
    double delta0;
    double lambda_max;
    double step_k;
    int32_t precond;      /* gl_precond */
    int32_t outer_steps;  /* T */
    int32_t inner_sweeps; /* m */
    int32_t reserved;     /* must be 0 */
} gl_params;

typedef struct gl_operator gl_operator;

/* Build the operator of `graph` (Section 2.2): validates the CSR (see
 * gl_graph), computes d_i = sum_j w_ij in F64 and stores, for L_s,
 * what_ij = w_ij / (sqrt(d_i) sqrt(d_j)) rounded to `store_w` (GL_F64, GL_F32,
 * GL_BF16 or GL_F16), for L the rounded w_ij and the row sums of the stored
 * weights as the diagonal, in library-owned device memory, with its own copy of the
 * index arrays; the caller may free `graph`'s arrays after return.  Every
 * index layout (direct, ordered, tile, grid) is built on the device; with an
 * order or a tile request it takes about 16 bytes per nonzero of temporary
 * device memory.  Synchronises `stream`.  Errors: GL_E_INVALID_ARG, GL_E_BAD_GRAPH (message
 * names the first defect), GL_E_DTYPE, GL_E_NOMEM, GL_E_HIP. */
gl_status gl_operator_create(const gl_graph *graph, gl_dtype store_w, void *stream,
                             gl_operator **out);

/* The paper's image graph (Section 2.2): pixel i is joined to every other
 * pixel j of its search window, max(|x_i - x_j|, |y_i - y_j|) <= window_radius
 * (the proximity N_s with dist = window_radius + 1; the 15 x 15 window is
 * radius 7, 55 x 55 is 27), with the patch-similarity weight
 *     w_ij = exp(-sum_n alpha_n |C(p_i + n) - C(p_j + n)|^2 / sigma^2),
 * n over the (2 patch_radius + 1)^2 offsets of the patch (5 x 5: radius 2),
 * C the pixel's colour vector.  The paper fixes neither alpha nor the border:
 * here alpha_(a,b) = g(a) g(b) / (sum_t g(t))^2 with g(t) = exp(-t^2 / (2
 * patch_radius^2)) (weights falling with the distance from the patch centre,
 * summing to 1; alpha = 1 for patch_radius 0), and a patch position outside
 * the image takes the colour of the nearest border pixel.
 *   image          device float [height * width * channels]: pixel (y, x) at
 *                  (y * width + x) * channels, channels interleaved; pixels are
 *                  the graph's nodes in that row-major order
 *   height, width  >= 1, height * width < 2^31
 *   channels       1..4
 *   window_radius  1..27;  patch_radius 0..4
 *   sigma          finite, > 0 (the paper takes it of the order log(N) + 1)
 *   laplacian      gl_laplacian, as in gl_graph;  reserved  0
 */
typedef struct gl_window_graph {
    const float *image;
    int32_t height;
    int32_t width;
    int32_t channels;
    int32_t window_radius;
    int32_t patch_radius;
    int32_t laplacian;
    double sigma;
    int32_t reserved;
} gl_window_graph;

/* Build the operator of a window graph on the device, with implicit columns
 * (layout GL_LAYOUT_WINDOW): the weights are computed in F64 once, the degrees
 * d_i summed in F64 in increasing neighbour order, and the stored weights
 * (what_ij for L_s, w_ij for L, rounded to `store_w`) kept once per pair: each
 * pixel keeps the first half of its window in scan order (dy < 0, or dy = 0
 * and dx < 0), and W being symmetric, the other half is its neighbours';
 * neighbours outside the image store 0.  Sweeps stream ((2r+1)^2 - 1) / 2
 * weights per pixel and no column indices.  The operator serves gl_solve,
 * gl_laplacian_apply, gl_power_max_eig, gl_second_eigenpair and gl_time_sweeps
 * like any other; their workspace sizes include the per-tile region sums of
 * one product (about (4 + r)(64 + 2r) / 256 x K x (4 or 8) bytes per pixel),
 * and gl_laplacian_apply takes that buffer from the stream-ordered allocator
 * for the call.  One call with K columns needs
 * 2 K * (64 + 2r) * (4 + r) * (4 or 8 bytes) <= 147456 of LDS, checked per
 * call (GL_E_INVALID_ARG).  Construction holds 8 bytes per pixel and window
 * offset of temporary device memory.  Synchronises `stream`.  Errors: GL_E_INVALID_ARG,
 * GL_E_BAD_GRAPH (a pixel whose weights all underflow to zero: a degree of
 * 0), GL_E_DTYPE, GL_E_NOMEM, GL_E_HIP. */
gl_status gl_window_operator_create(const gl_window_graph *graph, gl_dtype store_w, void *stream,
                                    gl_operator **out);

/* Release an operator (waits for nothing: the caller must not destroy an
 * operator while work that uses it is still queued). NULL is accepted. */
gl_status gl_operator_destroy(gl_operator *op);

/* Host: number of nodes, stored nonzeros, weight storage type, lanes per
 * row of the sparse product, and device bytes held.  Any pointer may be NULL. */
gl_status gl_operator_info(const gl_operator *op, int64_t *n, int64_t *nnz,
                           gl_dtype *store_w, int32_t *lanes_per_row, size_t *device_bytes);

/* Host: layout chosen (GL_LAYOUT_DIRECT, GL_LAYOUT_TILE, GL_LAYOUT_WINDOW or GL_LAYOUT_GRID),
 * entries stored (with padding), largest halo and total halo entries (tile:
 * distinct columns per block; window, grid: staged cells per block), and the bytes
 * of index/weight arrays one sweep streams.  Any pointer may be NULL. */
gl_status gl_operator_layout(const gl_operator *op, int32_t *layout, int64_t *stored_entries,
                             int32_t *halo_max, int64_t *halo_total, int64_t *stream_bytes);

/* Y = L_s X = X - D^{-1/2} W D^{-1/2} X (Section 2.2) for device X, Y of
 * n x K elements of `dtype` (1 <= K <= 16); X and Y must not overlap.  On a
 * renumbered operator and on the window layout the call allocates its scratch
 * from the stream-ordered allocator (hipMallocAsync) and frees it on `stream`. */
gl_status gl_laplacian_apply(const gl_operator *op, int32_t K, gl_dtype dtype,
                             const void *X, void *Y, void *stream);

/* Device bytes of workspace that gl_power_max_eig needs (host out). */
gl_status gl_power_workspace_size(const gl_operator *op, size_t *bytes);

/* Power method for the largest eigenvalue of the operator's Laplacian
 * (Section 3.1; Section 5.1.1 uses 150 iterations): x <- x0/|x0|, then
 * `iters` times x <- L x / |L x|, in F32 with F64 norms.  Host outputs:
 * *rayleigh = x^T L x of the final unit vector (L_s or L, as the operator's),
 * *lambda_hat = min(2 dmax, 1.01 * rayleigh) with dmax = 1 for L_s and the
 * largest stored diagonal for L, an upper estimate kept feasible by
 * 2I >= L_s and 2D >= L (Prop. 3).  x0: device float [n], not all zero.
 * Synchronises `stream`. */
gl_status gl_power_max_eig(const gl_operator *op, int32_t iters, const float *x0,
                           void *workspace, size_t workspace_bytes,
                           double *rayleigh, double *lambda_hat, void *stream);

/* The clustering graph of Section 2.2 from kNN lists (e.g. gl_knn's): i and
 * j are joined when either is among the other's k nearest neighbours (N_c,
 * symmetrised by union), with the local-scaling Gaussian weight of
 * Zelnik-Manor and Perona
 *     w_ij = exp(-|x_i - x_j|^2 / (s_i s_j)),  s_i = sqrt(d2[i][scale_rank-1])
 * (s_i = 2^-256 when that distance is 0), computed in F64.  Edges whose
 * weight is 0 are left out.
 *   idx       device int32 [n x k], each row ascending by distance, no self
 *   d2        device float [n x k], squared distances; symmetric (|x_i-x_j|^2
 *             computed alike from both ends, as gl_knn does); when an edge is
 *             in both lists the lower row's entry is used
 *   row_ptr   device int64 [n+1] (out);  col device int32, weight device
 *             double [capacity] (out, first *nnz entries; columns ascending per
 *             row, no self-loops): a gl_graph ready for gl_operator_create
 *   capacity  >= 2 n k;  *nnz (host out)
 * 2 <= n < 2^31, 1 <= k <= min(n-1, 1024), 2 n k < 2^31, 1 <= scale_rank <= k.
 * Allocates about 48 n k bytes of stream-ordered temporaries; synchronises
 * `stream`.  Errors: GL_E_INVALID_ARG (also an index out of range or equal
 * to its row, a negative or non-finite distance), GL_E_BAD_GRAPH (a point
 * whose weights are all 0), GL_E_NOMEM, GL_E_HIP. */
gl_status gl_knn_graph(int64_t n, int32_t k, const int32_t *idx, const float *d2, int32_t scale_rank,
                       int64_t *row_ptr, int32_t *col, double *weight, int64_t capacity, int64_t *nnz,
                       void *stream);

/* Unsupervised initialisation (Section 5.2 starts the unsupervised runs from
 * the second eigenvector of the normalized graph Laplacian): the second
 * smallest eigenvalue lambda_2 of the operator's Laplacian (L_s or L) and a
 * unit eigenvector, by Lanczos with full reorthogonalisation on the
 * operator's own product, deflated against the null vector (D^{1/2} 1 for L_s,
 * 1 for L), restarted from the Ritz vector until |L v - lambda_2 v| <= tol or
 * `max_restarts` restarts have run.
 *   krylov        Lanczos steps per restart, 2..512 (capped at n - 1)
 *   x0            device float [n], node order: start vector, not parallel
 *                 to the null vector
 *   v_out         device float [n], node order: the eigenvector, unit norm,
 *                 its entry of largest magnitude positive
 *   *lambda2, *residual, *restarts_used (may be NULL): host outputs
 * Vectors and products are float, inner products double.  With L_s the
 * deflation uses the exact degrees, so weights stored in BF16/F16 leave a
 * small null-space component; F32 weights are recommended.  Synchronises
 * `stream`.  Errors: GL_E_INVALID_ARG (also for an x0 parallel to the null
 * vector), GL_E_DTYPE (F64 weights), GL_E_NONFINITE (x0 zero or not finite),
 * GL_E_HIP. */
gl_status gl_second_eigenpair_workspace_size(const gl_operator *op, int32_t krylov, size_t *bytes);
gl_status gl_second_eigenpair(const gl_operator *op, int32_t krylov, int32_t max_restarts, double tol,
                              const float *x0, float *v_out, void *workspace, size_t workspace_bytes,
                              double *lambda2, double *residual, int32_t *restarts_used, void *stream);

/* Device bytes of workspace that gl_solve needs for K columns stored as
 * `store_u` (host out). */
gl_status gl_solve_workspace_size(const gl_operator *op, int32_t K, gl_dtype store_u,
                                  size_t *bytes);

/* Number of doubles gl_solve writes to `stats` for these parameters. */
int64_t gl_stats_length(int32_t K, int32_t outer_steps, int32_t inner_sweeps);

/* The preconditioned DCA (Prop. 1 with `inner_sweeps` diagonal sweeps per
 * step, Section 3.1).  For t = 0 .. T-1:
 *     b = c u^t - (u^t^3 - u^t)/eps + eta Lambda y          (right-hand side)
 *     v = u^t; repeat m times: r = b - T v, v = v + r / g   (all old values)
 *     u^{t+1} = v
 * with T = eps L_s + eta Lambda + c I and g the diagonal of `precond`; for a
 * finite step k, r = (u^t + k b) - (v + k T v) and g the T_k version.
 *   labels  device int32 [n]: -1 unlabelled (Lambda_i = 0); otherwise
 *           Lambda_i = 1 and, for K == 1, 1 -> y = +1 and 0 -> y = -1;
 *           for K >= 2, y_ik = +1 if labels[i] == k else -1.
 *   U       device [n x K] of `store_u`: u^0 on entry, u^T on return.
 *   workspace  device, >= gl_solve_workspace_size bytes, 256-byte aligned.
 *   stats   device double [gl_stats_length] or NULL (skips the reductions):
 *           [0, (T+1)K)          F(u^t) per column, t = 0..T (Section 2.1)
 *           [(T+1)K, +T m K)     |r|^2 per column for sweep s of step t
 *           last element         1.0 if any of them is NaN/Inf, else 0.0
 * Supported (store_w, store_u): F64 with F64; {F32, BF16, F16} with
 * {F32, BF16, F16}.  Asynchronous; allocates nothing. */
gl_status gl_solve(const gl_operator *op, const gl_params *params, int32_t K,
                   const int32_t *labels, gl_dtype store_u, void *U,
                   void *workspace, size_t workspace_bytes, double *stats, void *stream);

/* gl_solve without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Arguments, results and errors as gl_solve; the
 * workspace is a static device array of the library (128 MiB, one copy on
 * each GPU the library's kernels are loaded on, held until the process
 * ends).  The call itself allocates nothing and never synchronises; its
 * first call on a device resolves the array's address (make it outside a
 * graph capture).  Solves whose gl_solve_workspace_size exceeds 128 MiB fail
 * with GL_E_INVALID_ARG before any launch (use gl_solve for them).  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two threads) race and give wrong results, so serialise them.
 * Nothing in the array needs to start at zero (every call writes each part
 * before it reads it); the array keeps the last call's contents.  Results
 * are bitwise equal to gl_solve's for the same inputs (same kernels). */
gl_status gl_solve_noalloc(const gl_operator *op, const gl_params *params, int32_t K,
                           const int32_t *labels, gl_dtype store_u, void *U, double *stats,
                           void *stream);

/* Measurement helper: the practical HBM ceiling that the sweep kernels are
 * held against.  kind 0: a plain read-only streaming kernel reads all `bytes`
 * of `buf` (16-byte non-temporal vector loads, four in flight per lane,
 * grid-stride over 4096 workgroups of 256 lanes); kind 1: a plain copy kernel
 * reads the first half of `buf` and writes the second half (bytes moved =
 * `bytes`).  `reps` launches back to back between one pair of HIP events on
 * `stream`; *avg_ms (host) receives the mean time per launch.
 *   buf    device, 256-byte aligned, `bytes` long (contents: read, and for
 *          kind 1 the second half overwritten); bytes a multiple of 256,
 *          >= 1 MiB; use several GiB to measure HBM rather than the caches.
 * Synchronises `stream`.  Errors: GL_E_INVALID_ARG, GL_E_HIP. */
gl_status gl_time_stream(int32_t kind, void *buf, size_t bytes, int32_t reps, double *avg_ms,
                         void *stream);

/* Host-only check of a parameter block (the same checks gl_solve applies
 * before launching anything).  GL_OK or GL_E_INVALID_ARG with a message. */
gl_status gl_params_validate(const gl_params *params);

/* Measurement helper: launch `reps` sweep kernels exactly as gl_solve launches
 * its sweeps s >= 1 (gathering from one workspace buffer, writing the other,
 * reading u^t = U on the own row, block partial sums on), back to back
 * between one pair of HIP events on `stream`, as a solve issues them; *avg_ms
 * (host) receives the span divided by reps: the mean time per launch, gaps
 * between launches included.  1 <= reps <= 10000.
 * U is read, not changed; the workspace contents are overwritten.
 * Synchronises `stream`. */
gl_status gl_time_sweeps(const gl_operator *op, const gl_params *params, int32_t K,
                         const int32_t *labels, gl_dtype store_u, const void *U,
                         void *workspace, size_t workspace_bytes, int32_t reps,
                         double *avg_ms, void *stream);

/* Class per node from an n x K field: K == 1 -> 1 iff u_i >= 0, else 0;
 * K >= 2 -> argmax_k u_ik, ties to the lowest k.  labels_out: device int32 [n]. */
gl_status gl_assign_labels(int64_t n, int32_t K, gl_dtype dtype, const void *U,
                           int32_t *labels_out, void *stream);

/* ------------------------------------------------------------------------
 * Continuous-batching server.  Requests (host arrays) are queued by
 * gl_server_submit; a loader thread admits them in arrival order while a
 * solve slot is free and the request's device footprint fits in the server's
 * HBM arena, copies them to the GPU and builds their operators (direct
 * layout); a scheduler thread advances every admitted solve by one sweep per
 * "tick" with ONE batched kernel launch over all of them (plus one batched
 * statistics launch), so requests that arrive while others run join at the
 * next tick; a finisher thread copies results back and frees the slot and
 * memory.  Each solve computes exactly what gl_solve computes for it (same
 * kernels, same per-row order): results are bitwise equal to a gl_solve of
 * the same request, alone or in any mix.
 * ------------------------------------------------------------------------ */
typedef struct gl_server gl_server;

typedef struct gl_server_config {
    size_t hbm_budget_bytes;  /* device arena for admitted solves, allocated at creation */
    int32_t max_slots;        /* solves on the GPU at once, 1..64 */
    int32_t max_pending;      /* queued, not yet admitted requests (>= 1) */
    int32_t store_w;          /* gl_dtype of the weights: GL_F32, GL_BF16 or GL_F16 */
    int32_t store_u;          /* gl_dtype of the field: GL_F32, GL_BF16 or GL_F16 */
    int32_t ticks_in_flight;  /* batched launches queued ahead of the GPU, 1..8 */
    int32_t reserved;         /* must be 0 */
} gl_server_config;

/* gl_request.flags */
#define GL_REQ_BORROW 1 /* read the host arrays in place instead of copying them */

typedef struct gl_request {   /* HOST arrays */
    int64_t n;
    int64_t nnz;
    const int64_t *row_ptr;   /* as in gl_graph */
    const int32_t *col_idx;
    const double *weight;
    const int32_t *labels;    /* n, as in gl_solve */
    const float *u0;          /* n x K */
    int32_t K;                /* 1..10 */
    int32_t flags;            /* 0: gl_server_submit copies the arrays and the caller may
                                 reuse them at once.  GL_REQ_BORROW: the server reads them
                                 in place; they must stay alive and unchanged until
                                 gl_server_poll has returned this ticket's result.  Page-
                                 locked memory (hipHostMalloc) then moves at DMA speed. */
    gl_params params;
} gl_request;

typedef struct gl_result {    /* filled by gl_server_poll */
    float *U;                 /* caller's host n x K buffer for u^T, or NULL */
    int32_t *labels;          /* caller's host n buffer for the classes, or NULL */
    double *stats;            /* caller's host gl_stats_length(K, T, m) buffer, or NULL */
    double t_submit;          /* seconds since the server was created */
    double t_admit;
    double t_done;
    int32_t status;           /* gl_status of this solve (GL_E_NONFINITE, GL_E_BAD_GRAPH, ...) */
    int32_t reserved;
} gl_result;

/* Create a server on the current device.  Errors: GL_E_INVALID_ARG, GL_E_NOMEM. */
gl_status gl_server_create(const gl_server_config *cfg, gl_server **out);

/* Queue a request; *ticket identifies it.  GL_E_QUEUE_FULL when max_pending
 * requests wait; GL_E_BUDGET when its footprint exceeds the whole arena;
 * GL_E_INVALID_ARG for malformed sizes/params (graph content is checked on
 * the GPU at admission and reported through the result status). */
gl_status gl_server_submit(gl_server *srv, const gl_request *req, uint64_t *ticket);

/* Result of a ticket.  wait = 0: GL_E_NOT_READY while it runs; wait != 0:
 * block until done.  On GL_OK the ticket is consumed and out->status holds
 * the solve's own status. */
gl_status gl_server_poll(gl_server *srv, uint64_t ticket, int32_t wait, gl_result *out);

/* Cancel a ticket: a queued request ends at once, an admitted one stops at
 * the next tick; its result status becomes GL_E_CANCELLED.  A request that has
 * already finished keeps its result.  The ticket must still be polled. */
gl_status gl_server_cancel(gl_server *srv, uint64_t ticket);

/* Arena bytes a request of these sizes takes in a server with this storage:
 * `peak` while it is being admitted (graph copy included), `held` from then
 * until it finishes (host out).  A request is refused with GL_E_BUDGET when
 * `peak` exceeds hbm_budget_bytes.  Touches no GPU.  Errors: GL_E_INVALID_ARG,
 * GL_E_DTYPE. */
gl_status gl_server_request_bytes(int64_t n, int64_t nnz, int32_t K, int32_t outer_steps,
                                  int32_t inner_sweeps, gl_dtype store_w, gl_dtype store_u,
                                  size_t *peak, size_t *held);

/* Host counters: queued, on the GPU, finished-unpolled, arena bytes in use,
 * batched ticks launched.  Any pointer may be NULL. */
gl_status gl_server_info(gl_server *srv, int64_t *pending, int64_t *active, int64_t *finished,
                         size_t *arena_used, int64_t *ticks);

/* Drain: queued requests are cancelled, admitted ones finish; then free all. */
gl_status gl_server_destroy(gl_server *srv);

/* ------------------------------------------------------------------------
 * Graph construction: exact k nearest neighbours (Section 2.2 builds the
 * clustering graphs from the k nearest neighbours in Euclidean distance;
 * Section 6 names a parallel kNN as the missing piece for clustering).
 *   x        device f32 [n x d], row-major feature vectors (caller-owned)
 *   idx_out  device int32 [n x k]: for each point its k nearest other points
 *            by ascending squared distance, ties to the lower index
 *   d2_out   device f32 [n x k] or NULL: those squared distances, computed
 *            as sum_c (x_ic - x_jc)^2 in f32 in coordinate order
 * 1 <= d <= 4096, 1 <= k <= 32, k < n < 2^31.
 * d <= 64: one register-resident scan per query, asynchronous on `stream`; a
 * point with a non-finite coordinate is never chosen as a neighbour, and a
 * list that cannot be filled ends with index -1 and distance +inf.
 * d > 64 (wide features, e.g. 784 pixels): the same result, found through
 * the matrix cores: <x_i, x_j> of the centred points rounded to f16 (scaled
 * by a power of two), f32 accumulation, in one fused kernel that filters
 * every block of products into per-query candidate lists without storing
 * them; per query 64 candidates get their exact distances recomputed, and a
 * certificate from the rounding-error bound proves that no other point can
 * enter or tie the k best; queries without it are rescanned exactly
 * (gl_knn_fallback_rows).  Non-finite coordinates are rejected
 * (GL_E_INVALID_ARG).  Allocates about n (2 d + 300) bytes as
 * stream-ordered temporaries and synchronises `stream`.
 * Errors: GL_E_INVALID_ARG, GL_E_NOMEM, GL_E_HIP. */
gl_status gl_knn(const float *x, int64_t n, int32_t d, int32_t k, int32_t *idx_out,
                 float *d2_out, void *stream);

/* Host: queries of the calling thread's last gl_knn call with d > 64 that
 * needed the exact rescan (0 after a call with d <= 64, -1 after an error). */
int64_t gl_knn_fallback_rows(void);

/* Message of the last non-OK status returned to the calling thread. */
const char *gl_last_error(void);

/* Library version string. */
const char *gl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GL_DCA_H */
