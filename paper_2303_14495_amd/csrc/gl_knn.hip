// Exact k-nearest-neighbour search in R^d, the step that builds a clustering
// graph before the method runs (Section 2.2 uses the k nearest neighbours in
// Euclidean distance of the feature vectors; Section 6 names a parallel kNN as
// the missing piece for clustering).
//
// One thread per query: the query's coordinates and its k best (distance,
// index) pairs live in registers; the block streams every point through an LDS
// tile and each thread scans it with broadcast reads.  Nothing of size n x n
// is ever formed.  Distances are sum_c (q_c - p_c)^2 accumulated in f32 with
// FMA in coordinate order; ties go to the lower index.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "gl_internal.hpp"

namespace gl {

constexpr int kKnnBlock = 256;

template <int D>
struct KnnTile {
    static constexpr int points = D <= 32 ? 256 : 128;  // LDS: points * D * 4 bytes <= 32 KB
};

template <int D, int KM>
__global__ __launch_bounds__(kKnnBlock) void knn_kernel(const float* __restrict__ x, int64_t n, int32_t d,
                                                        int32_t k, int32_t* __restrict__ idx_out,
                                                        float* __restrict__ d2_out) {
    constexpr int TP = KnnTile<D>::points;
    __shared__ float tile[TP * D];
    const int64_t q = (int64_t)blockIdx.x * kKnnBlock + threadIdx.x;
    const bool active = q < n;
    float qc[D];
#pragma unroll
    for (int c = 0; c < D; ++c) qc[c] = (active && c < d) ? x[q * d + c] : 0.0f;
    float best[KM];
    int32_t bi[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) {
        best[i] = INFINITY;
        bi[i] = -1;
    }
    float thr = INFINITY;  // k-th best so far
    for (int64_t base = 0; base < n; base += TP) {
        const int cnt = (int)(n - base < TP ? n - base : TP);
        __syncthreads();
        for (int e = threadIdx.x; e < TP * D; e += kKnnBlock) {
            const int p = e / D, c = e - p * D;
            tile[e] = (p < cnt && c < d) ? x[(base + p) * d + c] : 0.0f;
        }
        __syncthreads();
        for (int p = 0; p < cnt; ++p) {
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const float t = qc[c] - tile[p * D + c];
                acc = fmaf(t, t, acc);
            }
            const int64_t j = base + p;
            if (acc < thr && j != q) {
                // insert after every entry <= acc and shift the rest down one
                // place (compile-time indices keep the lists in registers;
                // descending i reads each old entry before it is overwritten)
                const int32_t vi = (int32_t)j;
#pragma unroll
                for (int i = KM - 1; i >= 1; --i) {
                    const bool shift = acc < best[i - 1];
                    const bool here = acc < best[i];
                    best[i] = shift ? best[i - 1] : (here ? acc : best[i]);
                    bi[i] = shift ? bi[i - 1] : (here ? vi : bi[i]);
                }
                if (acc < best[0]) {
                    best[0] = acc;
                    bi[0] = vi;
                }
                float t = best[0];
#pragma unroll
                for (int i = 1; i < KM; ++i) t = (i == k - 1) ? best[i] : t;
                thr = t;
            }
        }
    }
    if (!active) return;
#pragma unroll
    for (int i = 0; i < KM; ++i) {
        if (i < k) {
            idx_out[q * k + i] = bi[i];
            if (d2_out) d2_out[q * k + i] = best[i];
        }
    }
}

template <int D>
static hipError_t knn_launch_d(const float* x, int64_t n, int32_t d, int32_t k, int32_t* idx, float* d2,
                               hipStream_t s) {
    const dim3 grid((unsigned)((n + kKnnBlock - 1) / kKnnBlock)), block(kKnnBlock);
    if (k <= 8)
        hipLaunchKernelGGL((knn_kernel<D, 8>), grid, block, 0, s, x, n, d, k, idx, d2);
    else if (k <= 16)
        hipLaunchKernelGGL((knn_kernel<D, 16>), grid, block, 0, s, x, n, d, k, idx, d2);
    else if (k <= 24)
        hipLaunchKernelGGL((knn_kernel<D, 24>), grid, block, 0, s, x, n, d, k, idx, d2);
    else
        hipLaunchKernelGGL((knn_kernel<D, 32>), grid, block, 0, s, x, n, d, k, idx, d2);
    return hipGetLastError();
}

static hipError_t knn_launch(const float* x, int64_t n, int32_t d, int32_t k, int32_t* idx, float* d2,
                             hipStream_t s) {
    switch (d) {
#define GL_KNN_D(DD) \
    case DD:         \
        return knn_launch_d<DD>(x, n, d, k, idx, d2, s);
        GL_KNN_D(1) GL_KNN_D(2) GL_KNN_D(3) GL_KNN_D(4) GL_KNN_D(5) GL_KNN_D(6) GL_KNN_D(7) GL_KNN_D(8)
        GL_KNN_D(9) GL_KNN_D(10) GL_KNN_D(11) GL_KNN_D(12) GL_KNN_D(13) GL_KNN_D(14) GL_KNN_D(15)
        GL_KNN_D(16)
#undef GL_KNN_D
        default:
            break;
    }
    // wider features: pad to the next supported width with zero coordinates
    if (d <= 24) return knn_launch_d<24>(x, n, d, k, idx, d2, s);
    if (d <= 32) return knn_launch_d<32>(x, n, d, k, idx, d2, s);
    if (d <= 48) return knn_launch_d<48>(x, n, d, k, idx, d2, s);
    return knn_launch_d<64>(x, n, d, k, idx, d2, s);
}

}  // namespace gl

namespace {
thread_local int64_t g_knn_fallback = 0;
}

extern "C" int64_t gl_knn_fallback_rows(void) { return g_knn_fallback; }

extern "C" gl_status gl_knn(const float* x, int64_t n, int32_t d, int32_t k, int32_t* idx_out, float* d2_out,
                            void* stream) {
    if (!x || !idx_out) {
        gl::set_last_error("x and idx_out must not be NULL");
        return GL_E_INVALID_ARG;
    }
    if (d < 1 || d > 4096) {
        gl::set_last_error("d must lie in [1, 4096]");
        return GL_E_INVALID_ARG;
    }
    if (k < 1 || k > 32) {
        gl::set_last_error("k must lie in [1, 32]");
        return GL_E_INVALID_ARG;
    }
    if (n <= k || n > INT32_MAX) {
        gl::set_last_error("need k < n < 2^31");
        return GL_E_INVALID_ARG;
    }
    if (d > 64) {
        int64_t fb = 0;
        const gl_status st = gl::knn_wide(x, n, d, k, idx_out, d2_out, (hipStream_t)stream, &fb);
        g_knn_fallback = st == GL_OK ? fb : -1;
        return st;
    }
    g_knn_fallback = 0;
    const hipError_t e = gl::knn_launch(x, n, d, k, idx_out, d2_out, (hipStream_t)stream);
    if (e != hipSuccess) {
        gl::set_last_error(std::string("knn launch: ") + hipGetErrorString(e));
        return GL_E_HIP;
    }
    return GL_OK;
}
