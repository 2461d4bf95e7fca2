/*
 * Plain C float64 oracle of the preconditioned DCA inner solve for the graph
 * Ginzburg-Landau model (arXiv 2303.14495).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product library, and it shares no
 * code with it.  The algorithm and its readings are those of gl_oracle.py:
 *
 *   Laplacian            written as diag(dd) - A (Section 2.2):
 *                        L_s = I - D^{-1/2} W D^{-1/2}: A_ij = w_ij / (sqrt(d_i) sqrt(d_j)), dd = 1;
 *                        L   = D - W:                   A = W,                      dd = d;
 *                        d_i = sum_j w_ij
 *   DCA right-hand side  b = c u - (u^3 - u)/eps + eta Lambda y      (Prop. 1)
 *   operator             T v = eps (dd v - A v) + eta Lambda v + c v  (Section 3)
 *   sweep                v <- v + (b - T v) / g, all old values       (Section 3.1)
 *                        finite step k: r = (u + k b) - (v + k T v)   (Lemma 1)
 *   preconditioners      g from G_Jd,s / G_Jp,s / G_R,s (L_s) or G_Jd / G_Jp / G_R (L),
 *                        or their step-size-k versions                (Section 3.1)
 *   energy               (eps/2) u.L u + sum (u^2-1)^2/(4 eps)
 *                        + (eta/2) sum Lambda (u - y)^2               (Section 2.1)
 *
 * Rows are split over OpenMP threads; every row is summed in CSR order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { GLO_DAMPED_JACOBI = 0, GLO_PERTURBED_JACOBI = 1, GLO_RICHARDSON = 2 };

/* The off-diagonal part A and the diagonal dd of the chosen Laplacian; both
   arrays are malloc'ed (freed by the caller). */
static int operator_parts(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                          int32_t unnormalized, double **A_out, double **dd_out)
{
    int64_t nnz = rp[n];
    double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *A = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!d || !A) { free(d); free(A); return 1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) s += w[p];
        d[i] = s;
    }
    if (unnormalized) {
        memcpy(A, w, sizeof(double) * (size_t)nnz);
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++)
            for (int64_t p = rp[i]; p < rp[i + 1]; p++)
                A[p] = w[p] / (sqrt(d[i]) * sqrt(d[col[p]]));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) d[i] = 1.0;
    }
    *A_out = A;
    *dd_out = d;
    return 0;
}

/* y_ik of node i (0 when unlabelled; K == 1: class 1 -> +1, class 0 -> -1). */
static double target(int32_t label, int32_t K, int32_t k)
{
    if (label < 0) return 0.0;
    if (K == 1) return label == 1 ? 1.0 : -1.0;
    return label == k ? 1.0 : -1.0;
}

/* Diagonal preconditioner of node i with diagonal dd_i of the Laplacian
   (dd_i = 1 for L_s: G_Jd,s, G_Jp,s, G_R,s and their k versions; dd_i = d_i
   for L: G_Jd, G_Jp, G_R and their k versions; Section 3.1). */
static double gdiag(int kind, double lam, double dd, double eps, double c, double eta,
                    double delta0, double lmax, double k)
{
    double el = eta * lam;
    if (isinf(k)) {
        if (kind == GLO_DAMPED_JACOBI) return 2.0 * (eps * dd + el + c);
        if (kind == GLO_PERTURBED_JACOBI) return 2.0 * eps * dd + el + c + delta0;
        return eps * lmax + el + c + delta0;
    }
    if (kind == GLO_DAMPED_JACOBI) return 2.0 * (1.0 + k * (eps * dd + el + c));
    if (kind == GLO_PERTURBED_JACOBI) return 1.0 + k * (2.0 * eps * dd + el + c) + delta0;
    return 1.0 + k * (eps * lmax + el + c) + delta0;
}

/* Y = L_s X or L X for n x K row-major X. */
int glo_laplacian_apply(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
                        int32_t K, const double *X, double *Y, int32_t unnormalized)
{
    double *A, *dd;
    if (operator_parts(n, rp, col, w, unnormalized, &A, &dd)) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        for (int32_t k = 0; k < K; k++) {
            double z = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; p++) z += A[p] * X[(int64_t)col[p] * K + k];
            Y[i * K + k] = dd[i] * X[i * K + k] - z;
        }
    }
    free(A); free(dd);
    return 0;
}

static void energy_cols(int64_t n, const int64_t *rp, const int32_t *col, const double *wh,
                        const double *dd, int32_t K, const int32_t *labels, const double *U,
                        double eps, double eta, double *out)
{
    double *lap = (double *)calloc((size_t)K, sizeof(double));
    double *well = (double *)calloc((size_t)K, sizeof(double));
    double *fid = (double *)calloc((size_t)K, sizeof(double));
#pragma omp parallel for schedule(static) reduction(+ : lap[:K], well[:K], fid[:K])
    for (int64_t i = 0; i < n; i++) {
        for (int32_t k = 0; k < K; k++) {
            double u = U[i * K + k], z = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; p++) z += wh[p] * U[(int64_t)col[p] * K + k];
            lap[k] += u * (dd[i] * u - z);
            well[k] += (u * u - 1.0) * (u * u - 1.0);
            if (labels[i] >= 0) {
                double e = u - target(labels[i], K, k);
                fid[k] += e * e;
            }
        }
    }
    for (int32_t k = 0; k < K; k++) out[k] = 0.5 * eps * lap[k] + well[k] / (4.0 * eps) + 0.5 * eta * fid[k];
    free(lap); free(well); free(fid);
}

/*
 * outer DCA steps of `sweeps` preconditioned sweeps.  U (n x K) holds u^0 on
 * entry and u^T on exit.  energies ((outer+1) x K) and res_sq
 * (outer x sweeps x K) may be NULL.  Returns 0 on success.
 */
int glo_solve(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
              int32_t K, const int32_t *labels, double *U,
              double eps, double c, double eta, int32_t precond,
              int32_t outer, int32_t sweeps, double delta0, double lambda_max, double step_k,
              double *energies, double *res_sq, int32_t unnormalized)
{
    double *wh = NULL, *dd = NULL;
    if (operator_parts(n, rp, col, w, unnormalized, &wh, &dd)) return 1;
    size_t cells = (size_t)n * (size_t)K;
    double *b = (double *)malloc(sizeof(double) * (cells ? cells : 1));
    double *V = (double *)malloc(sizeof(double) * (cells ? cells : 1));
    double *Vn = (double *)malloc(sizeof(double) * (cells ? cells : 1));
    double *rs = (double *)calloc((size_t)K, sizeof(double));
    if (!b || !V || !Vn || !rs) {
        free(wh); free(dd); free(b); free(V); free(Vn); free(rs);
        return 1;
    }
    int finite_k = !isinf(step_k);
    for (int32_t t = 0; t < outer; t++) {
        if (energies) energy_cols(n, rp, col, wh, dd, K, labels, U, eps, eta, energies + (int64_t)t * K);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            double lam = labels[i] >= 0 ? 1.0 : 0.0;
            for (int32_t k = 0; k < K; k++) {
                double u = U[i * K + k];
                b[i * K + k] = c * u - (u * u * u - u) / eps + eta * lam * target(labels[i], K, k);
                V[i * K + k] = u;
            }
        }
        for (int32_t s = 0; s < sweeps; s++) {
            for (int32_t k = 0; k < K; k++) rs[k] = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : rs[:K])
            for (int64_t i = 0; i < n; i++) {
                double lam = labels[i] >= 0 ? 1.0 : 0.0;
                double g = gdiag(precond, lam, dd[i], eps, c, eta, delta0, lambda_max, step_k);
                for (int32_t k = 0; k < K; k++) {
                    double z = 0.0;
                    for (int64_t p = rp[i]; p < rp[i + 1]; p++) z += wh[p] * V[(int64_t)col[p] * K + k];
                    double v = V[i * K + k];
                    double Tv = eps * (dd[i] * v - z) + eta * lam * v + c * v;
                    double r = finite_k ? (U[i * K + k] + step_k * b[i * K + k]) - (v + step_k * Tv)
                                        : b[i * K + k] - Tv;
                    rs[k] += r * r;
                    Vn[i * K + k] = v + r / g;
                }
            }
            if (res_sq)
                for (int32_t k = 0; k < K; k++) res_sq[((int64_t)t * sweeps + s) * K + k] = rs[k];
            double *tmp = V; V = Vn; Vn = tmp;
        }
        memcpy(U, V, sizeof(double) * cells);
    }
    if (energies) energy_cols(n, rp, col, wh, dd, K, labels, U, eps, eta, energies + (int64_t)outer * K);
    free(wh); free(dd); free(b); free(V); free(Vn); free(rs);
    return 0;
}

/* Power method on L_s (or L) from x0 (n); writes the Rayleigh quotient of the
   final unit vector to *rq and min(2 max dd, 1.01 rq) to *lambda_hat. */
int glo_power(int64_t n, const int64_t *rp, const int32_t *col, const double *w,
              const double *x0, int32_t iters, double *rq, double *lambda_hat, int32_t unnormalized)
{
    double *wh = NULL, *dd = NULL;
    if (operator_parts(n, rp, col, w, unnormalized, &wh, &dd)) return 1;
    double *x = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    if (!x || !y) { free(wh); free(dd); free(x); free(y); return 1; }
    double ddmax = 0.0;
    for (int64_t i = 0; i < n; i++) ddmax = dd[i] > ddmax ? dd[i] : ddmax;
    double nrm = 0.0;
    for (int64_t i = 0; i < n; i++) nrm += x0[i] * x0[i];
    nrm = sqrt(nrm);
    for (int64_t i = 0; i < n; i++) x[i] = x0[i] / nrm;
    for (int32_t it = 0; it <= iters; it++) {
        double ss = 0.0, xy = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : ss, xy)
        for (int64_t i = 0; i < n; i++) {
            double z = 0.0;
            for (int64_t p = rp[i]; p < rp[i + 1]; p++) z += wh[p] * x[col[p]];
            y[i] = dd[i] * x[i] - z;
            ss += y[i] * y[i];
            xy += x[i] * y[i];
        }
        if (it == iters) {
            *rq = xy;
            break;
        }
        double inv = 1.0 / sqrt(ss);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) x[i] = y[i] * inv;
    }
    *lambda_hat = fmin(2.0 * ddmax, 1.01 * *rq);
    free(wh); free(dd); free(x); free(y);
    return 0;
}

/* The paper's image graph (Section 2.2) in CSR, with the readings of
 * window_oracle.py: pixel i (row-major, h x w, C channels, img[(y w + x) C + c])
 * is joined to every other pixel j with max(|dy|, |dx|) <= rw, weight
 *     w_ij = exp(-sum_n alpha_n |C(p_i + n) - C(p_j + n)|^2 / sigma^2)
 * over the (2 rp + 1)^2 patch offsets n, alpha_n = g(a) g(b) / (sum g)^2 with
 * g(t) = exp(-t^2 / (2 rp^2)) (1 for rp = 0), colours outside the image taken
 * from the nearest border pixel.  Columns ascend within a row (window offsets
 * in scan order); row_ptr has n + 1 entries; returns the number of stored
 * entries, or -1 when `cap` is too small. */
int64_t glo_window_graph(int32_t h, int32_t w, int32_t C, const double *img, int32_t rw, int32_t rp,
                         double sigma, int64_t *row_ptr, int32_t *col, double *wout, int64_t cap)
{
    const int64_t n = (int64_t)h * w;
    const int32_t P = 2 * rp + 1;
    double g[64], gs = 0.0, alpha[64 * 64];
    for (int32_t a = -rp; a <= rp; a++) {
        g[a + rp] = rp > 0 ? exp(-(double)(a * a) / (2.0 * rp * rp)) : 1.0;
        gs += g[a + rp];
    }
    for (int32_t a = 0; a < P; a++)
        for (int32_t b = 0; b < P; b++) alpha[a * P + b] = g[a] * g[b] / (gs * gs);
    /* row offsets: the count of in-image window cells of every pixel */
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        const int32_t y = (int32_t)(i / w), x = (int32_t)(i % w);
        const int32_t y0 = y - rw < 0 ? 0 : y - rw, y1 = y + rw >= h ? h - 1 : y + rw;
        const int32_t x0 = x - rw < 0 ? 0 : x - rw, x1 = x + rw >= w ? w - 1 : x + rw;
        row_ptr[i + 1] = row_ptr[i] + (int64_t)(y1 - y0 + 1) * (x1 - x0 + 1) - 1;
    }
    if (row_ptr[n] > cap) return -1;
    const double inv_s2 = 1.0 / (sigma * sigma);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        const int32_t y = (int32_t)(i / w), x = (int32_t)(i % w);
        int64_t q = row_ptr[i];
        for (int32_t dy = -rw; dy <= rw; dy++) {
            for (int32_t dx = -rw; dx <= rw; dx++) {
                const int32_t yj = y + dy, xj = x + dx;
                if ((dy == 0 && dx == 0) || yj < 0 || yj >= h || xj < 0 || xj >= w) continue;
                double s = 0.0;
                for (int32_t a = -rp; a <= rp; a++) {
                    for (int32_t b = -rp; b <= rp; b++) {
                        int32_t yi2 = y + a, xi2 = x + b, yj2 = yj + a, xj2 = xj + b;
                        yi2 = yi2 < 0 ? 0 : (yi2 >= h ? h - 1 : yi2);
                        xi2 = xi2 < 0 ? 0 : (xi2 >= w ? w - 1 : xi2);
                        yj2 = yj2 < 0 ? 0 : (yj2 >= h ? h - 1 : yj2);
                        xj2 = xj2 < 0 ? 0 : (xj2 >= w ? w - 1 : xj2);
                        const double *ci = img + ((int64_t)yi2 * w + xi2) * C;
                        const double *cj = img + ((int64_t)yj2 * w + xj2) * C;
                        double d2 = 0.0;
                        for (int32_t c = 0; c < C; c++) d2 += (ci[c] - cj[c]) * (ci[c] - cj[c]);
                        s += alpha[(a + rp) * P + (b + rp)] * d2;
                    }
                }
                col[q] = (int32_t)((int64_t)yj * w + xj);
                wout[q] = exp(-s * inv_s2);
                q++;
            }
        }
    }
    return row_ptr[n];
}

int glo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
