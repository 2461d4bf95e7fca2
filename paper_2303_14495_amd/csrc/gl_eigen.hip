// Second eigenpair of the operator's Laplacian, the start of the unsupervised
// runs (Section 5.2 initialises them with the second eigenvector of the
// normalized graph Laplacian).
//
// Lanczos with full reorthogonalisation on the operator's own sparse product,
// deflated against the known null vector (D^{1/2} 1 for L_s, 1 for L):
//   q_0 = x_0 - (z.x_0) z, normalised; for j = 0 .. m-1:
//   w = L q_j; alpha_j = q_j.w; w -= [z, q_0 .. q_j] c twice (classical
//   Gram-Schmidt, c = [z, q_0 .. q_j]^T w); beta_j = |w|; q_{j+1} = w / beta_j.
// The smallest eigenpair (theta, y) of the tridiagonal T_m (bisection on the
// Sturm count, then inverse iteration) gives the Ritz vector x = Q y; the run
// restarts from x until |L x - theta x| <= tol.  Vectors are float in the
// operator's position order; every inner product is summed in double in a
// fixed order, so results are reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "gl_internal.hpp"
#include "gl_kernels.hpp"

namespace gl {

constexpr int kDotRows = 2048;  // rows per workgroup of the inner-product kernel (8 per thread)

// z_p = sqrt(d_i) (L_s) or 1 (L), i the node of position p.
__global__ void null_vector_kernel(int64_t n, const double* __restrict__ degree, const int32_t* __restrict__ order,
                                   int32_t normalized, float* __restrict__ z) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = order ? (int64_t)order[p] : p;
    z[p] = normalized ? (float)sqrt(degree[i]) : 1.0f;
}

// partials[j * nb + b] = sum over the rows of block b of V_j[i] * w[i] for the
// cnt vectors V_j = V + j * ldv (fixed order: thread, then wavefront, then the
// four wavefronts of the block).
__global__ __launch_bounds__(kBlock) void multi_dot_kernel(int64_t n, const float* __restrict__ V, int64_t ldv,
                                                           int32_t cnt, const float* __restrict__ w,
                                                           double* __restrict__ partials, int64_t nb) {
    __shared__ double sh[kBlock / 64];
    const int64_t b = blockIdx.x;
    const int64_t base = b * kDotRows + threadIdx.x;
    float wv[kDotRows / kBlock];
#pragma unroll
    for (int e = 0; e < kDotRows / kBlock; ++e) {
        const int64_t i = base + (int64_t)e * kBlock;
        wv[e] = i < n ? w[i] : 0.0f;
    }
    for (int32_t j = 0; j < cnt; ++j) {
        const float* v = V + (int64_t)j * ldv;
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < kDotRows / kBlock; ++e) {
            const int64_t i = base + (int64_t)e * kBlock;
            if (i < n) acc += (double)v[i] * (double)wv[e];
        }
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) partials[(int64_t)j * nb + b] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
        __syncthreads();
    }
}

// out[j] = sum of partials[j * nb .. j * nb + nb) in a fixed order (block j).
__global__ __launch_bounds__(kBlock) void sum_partials_kernel(const double* __restrict__ partials, int64_t nb,
                                                              double* __restrict__ out) {
    const double v = block_sum(partials + (int64_t)blockIdx.x * nb, nb);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// w -= sum_j c_j V_j (sum in double).
__global__ void combine_kernel(int64_t n, const float* __restrict__ V, int64_t ldv, int32_t cnt,
                               const double* __restrict__ c, float* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int32_t j = 0; j < cnt; ++j) acc += c[j] * (double)V[(int64_t)j * ldv + i];
    w[i] = (float)((double)w[i] - acc);
}

// x = sum_j y_j V_j (sum in double).
__global__ void ritz_kernel(int64_t n, const float* __restrict__ V, int64_t ldv, int32_t cnt,
                            const double* __restrict__ y, float* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int32_t j = 0; j < cnt; ++j) acc += y[j] * (double)V[(int64_t)j * ldv + i];
    x[i] = (float)acc;
}

// y = s x; with order, y lands at the node of each position (scatter).
__global__ void scale_kernel(int64_t n, const float* __restrict__ x, float* __restrict__ y, double s,
                             const int32_t* __restrict__ scatter_order) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t o = scatter_order ? (int64_t)scatter_order[i] : i;
    y[o] = (float)((double)x[i] * s);
}

// y = x gathered from node order into position order.
__global__ void gather_kernel(int64_t n, const float* __restrict__ x, const int32_t* __restrict__ order,
                              float* __restrict__ y) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    y[p] = x[order ? (int64_t)order[p] : p];
}

// r = w - theta x.
__global__ void residual_kernel(int64_t n, const float* __restrict__ w, const float* __restrict__ x, double theta,
                                float* __restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    r[i] = (float)((double)w[i] - theta * (double)x[i]);
}

}  // namespace gl

namespace {

gl_status efail(gl_status st, const std::string& m) {
    gl::set_last_error(m);
    return st;
}

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct EigWs {
    int64_t ldv = 0, nb = 0;
    float* Q = nullptr;  // [m + 1] Lanczos vectors
    float* z = nullptr;  // null vector (unit)
    float* w = nullptr;
    float* x = nullptr;
    double* partials = nullptr;  // [(m + 2) * nb]
    double* dots = nullptr;      // [m + 2]
    double* y = nullptr;         // [m]
    float* wpart = nullptr;      // window layout: region sums of one product
    size_t bytes = 0;
};

EigWs carve(const gl_operator* op, int32_t m, char* base) {
    EigWs e;
    e.ldv = (op->n + 63) / 64 * 64;
    e.nb = (op->n + gl::kDotRows - 1) / gl::kDotRows;
    const size_t vec = al256((size_t)e.ldv * 4);
    size_t o = 0;
    auto take = [&](size_t b) {
        char* p = base ? base + o : nullptr;
        o += al256(b);
        return p;
    };
    e.Q = (float*)take((size_t)(m + 1) * e.ldv * 4);
    e.z = (float*)take(vec);
    e.w = (float*)take(vec);
    e.x = (float*)take(vec);
    e.partials = (double*)take((size_t)(m + 2) * e.nb * 8);
    e.dots = (double*)take((size_t)(m + 2) * 8);
    e.y = (double*)take((size_t)m * 8);
    e.wpart = (float*)take(gl::window_part_bytes(op, 1, 4));
    e.bytes = o;
    return e;
}

// Smallest eigenpair of the symmetric tridiagonal matrix (a, b): bisection on
// the Sturm count for the eigenvalue, inverse iteration (dense elimination with
// partial pivoting; m is small) for the unit eigenvector.
void tridiag_smallest(const std::vector<double>& a, const std::vector<double>& b, double& theta,
                      std::vector<double>& y) {
    const int m = (int)a.size();
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    const double scale = std::max(std::fabs(lo), std::fabs(hi)) + 1e-300;
    auto count_below = [&](double x) {  // eigenvalues < x
        int c = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0) d = -1e-300;
            if (d < 0.0) ++c;
        }
        return c;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * scale; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= 1) hi = mid;
        else lo = mid;
    }
    theta = 0.5 * (lo + hi);
    // inverse iteration on T - (theta - tiny) I
    const double shift = theta - 1e-12 * scale;
    y.assign(m, 1.0 / std::sqrt((double)m));
    for (int it = 0; it < 3; ++it) {
        std::vector<double> A((size_t)m * m, 0.0), rhs = y;
        for (int i = 0; i < m; ++i) {
            A[(size_t)i * m + i] = a[i] - shift;
            if (i + 1 < m) A[(size_t)i * m + i + 1] = A[(size_t)(i + 1) * m + i] = b[i];
        }
        for (int k = 0; k < m; ++k) {
            int piv = k;
            for (int i = k + 1; i < m; ++i)
                if (std::fabs(A[(size_t)i * m + k]) > std::fabs(A[(size_t)piv * m + k])) piv = i;
            if (piv != k) {
                for (int j = 0; j < m; ++j) std::swap(A[(size_t)k * m + j], A[(size_t)piv * m + j]);
                std::swap(rhs[k], rhs[piv]);
            }
            double p = A[(size_t)k * m + k];
            if (p == 0.0) p = A[(size_t)k * m + k] = 1e-300;
            for (int i = k + 1; i < m; ++i) {
                const double f = A[(size_t)i * m + k] / p;
                if (f == 0.0) continue;
                for (int j = k; j < m; ++j) A[(size_t)i * m + j] -= f * A[(size_t)k * m + j];
                rhs[i] -= f * rhs[k];
            }
        }
        for (int i = m - 1; i >= 0; --i) {
            double s = rhs[i];
            for (int j = i + 1; j < m; ++j) s -= A[(size_t)i * m + j] * y[j];
            y[i] = s / A[(size_t)i * m + i];
        }
        double nrm = 0.0;
        for (double v : y) nrm += v * v;
        nrm = std::sqrt(nrm);
        for (double& v : y) v /= nrm;
    }
}

}  // namespace

extern "C" {

gl_status gl_second_eigenpair_workspace_size(const gl_operator* op, int32_t krylov, size_t* bytes) {
    if (!gl::valid(op) || !bytes) return efail(GL_E_INVALID_ARG, "operator (a live operator handle) and bytes must not be NULL");
    if (krylov < 2 || krylov > 512) return efail(GL_E_INVALID_ARG, "krylov must lie in [2, 512]");
    *bytes = carve(op, krylov, nullptr).bytes;
    return GL_OK;
}

gl_status gl_second_eigenpair(const gl_operator* op, int32_t krylov, int32_t max_restarts, double tol,
                              const float* x0, float* v_out, void* ws, size_t ws_bytes, double* lambda2,
                              double* residual, int32_t* restarts_used, void* stream) {
    if (!gl::valid(op) || !x0 || !v_out || !ws || !lambda2 || !residual)
        return efail(GL_E_INVALID_ARG, "operator, x0, v_out, workspace and outputs must not be NULL");
    if (krylov < 2 || krylov > 512) return efail(GL_E_INVALID_ARG, "krylov must lie in [2, 512]");
    if (max_restarts < 0) return efail(GL_E_INVALID_ARG, "max_restarts must be >= 0");
    if (!(tol > 0.0) || !std::isfinite(tol)) return efail(GL_E_INVALID_ARG, "tol must be finite and > 0");
    if (op->store_w == GL_F64) return efail(GL_E_DTYPE, "the eigen-solver runs on F32/BF16/F16 weights");
    if ((uintptr_t)ws % 256) return efail(GL_E_INVALID_ARG, "workspace must be 256-byte aligned");
    const int32_t m = (int32_t)std::min<int64_t>(krylov, op->n - 1);
    if (m < 2) return efail(GL_E_INVALID_ARG, "the graph is too small");
    EigWs e = carve(op, m, (char*)ws);
    if (ws_bytes < e.bytes) return efail(GL_E_INVALID_ARG, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->n;
    const unsigned g256 = (unsigned)((n + 255) / 256);
    gl::RowLaunch rows = gl::operator_rows(op);
    rows.wpart = e.wpart;
    hipError_t err = hipSuccess;
#define GE_CHECK(what)                                                                  \
    do {                                                                                \
        if (err == hipSuccess) err = hipGetLastError();                                 \
        if (err != hipSuccess)                                                          \
            return efail(GL_E_HIP, std::string(what) + ": " + hipGetErrorString(err)); \
    } while (0)

    // inner products of cnt vectors starting at V with w, copied to host
    std::vector<double> hd(m + 2);
    auto dots = [&](const float* V, int32_t cnt, const float* w) -> hipError_t {
        hipLaunchKernelGGL(gl::multi_dot_kernel, dim3((unsigned)e.nb), dim3(gl::kBlock), 0, s, n, V, e.ldv, cnt, w,
                           e.partials, e.nb);
        hipLaunchKernelGGL(gl::sum_partials_kernel, dim3((unsigned)cnt), dim3(gl::kBlock), 0, s, e.partials, e.nb,
                           e.dots);
        hipError_t r = hipGetLastError();
        if (r == hipSuccess) r = hipMemcpyAsync(hd.data(), e.dots, (size_t)cnt * 8, hipMemcpyDeviceToHost, s);
        if (r == hipSuccess) r = hipStreamSynchronize(s);
        return r;
    };
    // w -= [z, Q_0 .. Q_{cnt-1}] c with c the host coefficients
    std::vector<double> hc(m + 2);
    auto subtract = [&](const float* V, int32_t cnt, const double* c, float* w) -> hipError_t {
        hipError_t r = hipMemcpyAsync(e.dots, c, (size_t)cnt * 8, hipMemcpyHostToDevice, s);
        if (r != hipSuccess) return r;
        hipLaunchKernelGGL(gl::combine_kernel, dim3(g256), dim3(256), 0, s, n, V, e.ldv, cnt, e.dots, w);
        return hipGetLastError();
    };
    // Gram-Schmidt of w against z and Q_0 .. Q_{j}; returns the first-pass coefficient on Q_j
    auto orthogonalise = [&](float* w, int32_t j, double* coef_j) -> hipError_t {
        for (int pass = 0; pass < 2; ++pass) {
            hipError_t r = dots(e.z, 1, w);
            if (r != hipSuccess) return r;
            hc[0] = hd[0];
            r = subtract(e.z, 1, hc.data(), w);
            if (r != hipSuccess) return r;
            if (j >= 0) {
                r = dots(e.Q, j + 1, w);
                if (r != hipSuccess) return r;
                if (pass == 0 && coef_j) *coef_j = hd[j];
                r = subtract(e.Q, j + 1, hd.data(), w);
                if (r != hipSuccess) return r;
            }
        }
        return hipSuccess;
    };

    // null vector z, unit norm
    hipLaunchKernelGGL(gl::null_vector_kernel, dim3(g256), dim3(256), 0, s, n, op->degree, op->order,
                       op->lap == GL_LAP_NORMALIZED ? 1 : 0, e.z);
    GE_CHECK("null vector");
    err = dots(e.z, 1, e.z);
    GE_CHECK("null vector norm");
    hipLaunchKernelGGL(gl::scale_kernel, dim3(g256), dim3(256), 0, s, n, e.z, e.z, 1.0 / std::sqrt(hd[0]),
                       (const int32_t*)nullptr);
    GE_CHECK("null vector scale");
    // start vector in position order
    hipLaunchKernelGGL(gl::gather_kernel, dim3(g256), dim3(256), 0, s, n, x0, op->order, e.x);
    GE_CHECK("start vector");

    double theta = 0.0, res = INFINITY;
    int32_t restart = 0;
    std::vector<double> a, b, y;
    for (;; ++restart) {
        // q_0 = x - (z.x) z, normalised
        err = dots(e.x, 1, e.x);
        GE_CHECK("start norm");
        const double before = hd[0];
        if (!(before > 0.0) || !std::isfinite(before))
            return efail(GL_E_NONFINITE, "the start vector is zero or not finite");
        err = orthogonalise(e.x, -1, nullptr);
        GE_CHECK("start orthogonalisation");
        err = dots(e.x, 1, e.x);
        GE_CHECK("start norm");
        if (!(hd[0] > 1e-10 * before))
            return efail(GL_E_INVALID_ARG, "the start vector is parallel to the null vector");
        hipLaunchKernelGGL(gl::scale_kernel, dim3(g256), dim3(256), 0, s, n, e.x, e.Q, 1.0 / std::sqrt(hd[0]),
                           (const int32_t*)nullptr);
        GE_CHECK("start scale");
        a.clear();
        b.clear();
        for (int32_t j = 0; j < m; ++j) {
            float* qj = e.Q + (int64_t)j * e.ldv;
            err = gl::launch_laplacian_f32(1, rows, qj, e.w, s);
            GE_CHECK("Lanczos product");
            double alpha = 0.0;
            err = orthogonalise(e.w, j, &alpha);
            GE_CHECK("reorthogonalisation");
            a.push_back(alpha);
            if (j + 1 == m) break;
            err = dots(e.w, 1, e.w);
            GE_CHECK("Lanczos norm");
            const double beta = std::sqrt(std::max(hd[0], 0.0));
            if (!(beta > 1e-30 * (std::fabs(alpha) + 1.0))) break;  // invariant subspace
            b.push_back(beta);
            hipLaunchKernelGGL(gl::scale_kernel, dim3(g256), dim3(256), 0, s, n, e.w,
                               e.Q + (int64_t)(j + 1) * e.ldv, 1.0 / beta, (const int32_t*)nullptr);
            GE_CHECK("Lanczos scale");
        }
        tridiag_smallest(a, b, theta, y);
        const int32_t k = (int32_t)a.size();
        err = hipMemcpyAsync(e.y, y.data(), (size_t)k * 8, hipMemcpyHostToDevice, s);
        GE_CHECK("Ritz coefficients");
        hipLaunchKernelGGL(gl::ritz_kernel, dim3(g256), dim3(256), 0, s, n, e.Q, e.ldv, k, e.y, e.x);
        GE_CHECK("Ritz vector");
        // residual |L x - theta x| of the unit Ritz vector
        err = dots(e.x, 1, e.x);
        GE_CHECK("Ritz norm");
        const double xn = std::sqrt(hd[0]);
        hipLaunchKernelGGL(gl::scale_kernel, dim3(g256), dim3(256), 0, s, n, e.x, e.x, 1.0 / xn,
                           (const int32_t*)nullptr);
        err = gl::launch_laplacian_f32(1, rows, e.x, e.w, s);
        GE_CHECK("residual product");
        hipLaunchKernelGGL(gl::residual_kernel, dim3(g256), dim3(256), 0, s, n, e.w, e.x, theta, e.w);
        GE_CHECK("residual");
        err = dots(e.w, 1, e.w);
        GE_CHECK("residual norm");
        res = std::sqrt(std::max(hd[0], 0.0));
        if (res <= tol || restart >= max_restarts) break;
    }
    // sign: the entry of largest magnitude is positive
    std::vector<float> hx(n);
    err = hipMemcpyAsync(hx.data(), e.x, (size_t)n * 4, hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    GE_CHECK("eigenvector copy");
    int64_t imax = 0;
    for (int64_t i = 1; i < n; ++i)
        if (std::fabs(hx[i]) > std::fabs(hx[imax])) imax = i;
    const double sgn = hx[imax] < 0.0f ? -1.0 : 1.0;
    hipLaunchKernelGGL(gl::scale_kernel, dim3(g256), dim3(256), 0, s, n, e.x, v_out, sgn, op->order);
    GE_CHECK("eigenvector output");
    err = hipStreamSynchronize(s);
    GE_CHECK("eigen-solver");
#undef GE_CHECK
    *lambda2 = theta;
    *residual = res;
    if (restarts_used) *restarts_used = restart;
    return GL_OK;
}

}  // extern "C"
