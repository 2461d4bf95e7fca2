// Symmetric kNN graph with local-scaling weights from kNN lists (the
// clustering graph of Section 2.2): union of the lists, Gaussian weights with
// the bandwidth product s_i s_j, CSR out.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <string>

#include "gl_internal.hpp"

namespace {

constexpr double kScaleFloor = 0x1p-256;  // s_i of a point whose scale neighbour is at distance 0

enum : int32_t { KG_BAD_INDEX = 1, KG_BAD_DIST = 2, KG_ISOLATED = 4 };

// Both orientations of every list entry t = i * k + e: key (row << 32 | col),
// value t (the entry whose distance gives the weight).
__global__ void kg_emit_kernel(int64_t n, int32_t k, const int32_t* __restrict__ idx,
                               const float* __restrict__ d2, unsigned long long* __restrict__ keys,
                               int64_t* __restrict__ vals, int32_t* flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * k) return;
    const int64_t i = t / k;
    const int64_t j = idx[t];
    const float dv = d2[t];
    int32_t f = 0;
    if (j < 0 || j >= n || j == i) f |= KG_BAD_INDEX;
    if (!(dv >= 0.0f) || !(dv <= 3.4028234663852886e38f)) f |= KG_BAD_DIST;
    if (f) {
        atomicOr(flags, f);
        keys[2 * t] = keys[2 * t + 1] = 0ull;  // keeps the sort defined; the call fails
    } else {
        keys[2 * t] = ((unsigned long long)i << 32) | (unsigned long long)j;
        keys[2 * t + 1] = ((unsigned long long)j << 32) | (unsigned long long)i;
    }
    vals[2 * t] = vals[2 * t + 1] = t;
}

__device__ __forceinline__ double kg_scale(const float* d2, int64_t node, int32_t k, int32_t rank) {
    const double s = sqrt((double)d2[node * k + rank - 1]);
    return s > 0.0 ? s : kScaleFloor;
}

// keep[p] = 1 for the first occurrence of a key whose weight is > 0;
// wts[p] = that weight.
__global__ void kg_weight_kernel(int64_t m2, int32_t k, int32_t rank, const unsigned long long* __restrict__ keys,
                                 const int64_t* __restrict__ vals, const float* __restrict__ d2,
                                 int32_t* __restrict__ keep, double* __restrict__ wts) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m2) return;
    const unsigned long long key = keys[p];
    int32_t kp = 0;
    double w = 0.0;
    if (p == 0 || keys[p - 1] != key) {
        const int64_t i = (int64_t)(key >> 32), j = (int64_t)(key & 0xffffffffull);
        w = exp(-(double)d2[vals[p]] / (kg_scale(d2, i, k, rank) * kg_scale(d2, j, k, rank)));
        kp = w > 0.0 ? 1 : 0;
    }
    keep[p] = kp;
    wts[p] = w;
}

__global__ void kg_scatter_kernel(int64_t m2, const unsigned long long* __restrict__ keys,
                                  const int32_t* __restrict__ keep, const int32_t* __restrict__ pos,
                                  const double* __restrict__ wts, int32_t* __restrict__ col,
                                  double* __restrict__ weight, int32_t* __restrict__ rows) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m2 || !keep[p]) return;
    const int64_t q = pos[p];
    col[q] = (int32_t)(keys[p] & 0xffffffffull);
    rows[q] = (int32_t)(keys[p] >> 32);
    weight[q] = wts[p];
}

// row_ptr[i] = first kept entry of row >= i (rows sorted); isolated rows flagged.
__global__ void kg_rowptr_kernel(int64_t n, int64_t nnz, const int32_t* __restrict__ rows,
                                 int64_t* __restrict__ row_ptr, int32_t* flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (rows[mid] < i) lo = mid + 1; else hi = mid;
    }
    row_ptr[i] = lo;
    if (i < n) {
        const bool has = lo < nnz && rows[lo] == i;
        if (!has) atomicOr(flags, (int32_t)KG_ISOLATED);
    }
}

gl_status kfail(gl_status st, const std::string& m) {
    gl::set_last_error(m);
    return st;
}

}  // namespace

extern "C" gl_status gl_knn_graph(int64_t n, int32_t k, const int32_t* idx, const float* d2, int32_t scale_rank,
                                  int64_t* row_ptr, int32_t* col, double* weight, int64_t capacity, int64_t* nnz,
                                  void* stream) {
    if (!idx || !d2 || !row_ptr || !col || !weight || !nnz)
        return kfail(GL_E_INVALID_ARG, "arrays and nnz must not be NULL");
    if (n < 2 || n >= ((int64_t)1 << 31)) return kfail(GL_E_INVALID_ARG, "n must lie in [2, 2^31)");
    if (k < 1 || (int64_t)k >= n || k > 1024) return kfail(GL_E_INVALID_ARG, "k must lie in [1, min(n - 1, 1024)]");
    if (scale_rank < 1 || scale_rank > k) return kfail(GL_E_INVALID_ARG, "scale_rank must lie in [1, k]");
    const int64_t m = n * k, m2 = 2 * m;
    if (capacity < m2) return kfail(GL_E_INVALID_ARG, "capacity must be >= 2 n k");
    hipStream_t s = (hipStream_t)stream;
    // temporaries: keys (2 buffers), values (2), keep, positions, weights, rows, flags, sort storage
    int nbits = 32;
    while (nbits < 64 && ((unsigned long long)(n - 1) >> (nbits - 32)) != 0ull) ++nbits;
    size_t sort_bytes = 0;
    hipcub::DoubleBuffer<unsigned long long> kb(nullptr, nullptr);
    hipcub::DoubleBuffer<int64_t> vb(nullptr, nullptr);
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, kb, vb, (int)0, 0, nbits, s) != hipSuccess)
        return kfail(GL_E_HIP, "radix sort size query failed");
    if (m2 > (int64_t)INT32_MAX) return kfail(GL_E_INVALID_ARG, "2 n k must be < 2^31");
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, kb, vb, (int)m2, 0, nbits, s);
    size_t scan_bytes = 0;
    if (e == hipSuccess)
        e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (const int32_t*)nullptr, (int32_t*)nullptr,
                                             (int)m2, s);
    if (e != hipSuccess) return kfail(GL_E_HIP, std::string("temporary size query: ") + hipGetErrorString(e));
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_keys = al((size_t)m2 * 8), b_vals = al((size_t)m2 * 8), b_i32 = al((size_t)m2 * 4),
                 b_w = al((size_t)m2 * 8);
    const size_t total = 2 * b_keys + 2 * b_vals + 3 * b_i32 + b_w + 256 + al(sort_bytes) + al(scan_bytes);
    char* base = nullptr;
    if (hipMallocAsync((void**)&base, total, s) != hipSuccess) {
        (void)hipGetLastError();
        return kfail(GL_E_NOMEM, "temporary device memory for the kNN graph");
    }
    char* q = base;
    auto take = [&](size_t b) { char* r = q; q += b; return r; };
    unsigned long long* k0 = (unsigned long long*)take(b_keys);
    unsigned long long* k1 = (unsigned long long*)take(b_keys);
    int64_t* v0 = (int64_t*)take(b_vals);
    int64_t* v1 = (int64_t*)take(b_vals);
    int32_t* keep = (int32_t*)take(b_i32);
    int32_t* pos = (int32_t*)take(b_i32);
    int32_t* rows = (int32_t*)take(b_i32);
    double* wts = (double*)take(b_w);
    int32_t* flags = (int32_t*)take(256);
    void* sort_tmp = take(al(sort_bytes));
    void* scan_tmp = take(al(scan_bytes));

    const unsigned g_m = (unsigned)((m + 255) / 256), g_m2 = (unsigned)((m2 + 255) / 256);
    int32_t hflags = 0, hlast[2] = {0, 0};
    int64_t count = 0;
    e = hipMemsetAsync(flags, 0, 4, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kg_emit_kernel, dim3(g_m), dim3(256), 0, s, n, k, idx, d2, k0, v0, flags);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    gl_status st = GL_OK;
    if (e == hipSuccess && hflags) {
        st = kfail(GL_E_INVALID_ARG, (hflags & KG_BAD_INDEX) ? "a neighbour index is out of [0, n) or the point itself"
                                                              : "a squared distance is negative or not finite");
    }
    if (e == hipSuccess && st == GL_OK) {
        hipcub::DoubleBuffer<unsigned long long> keys(k0, k1);
        hipcub::DoubleBuffer<int64_t> vals(v0, v1);
        e = hipcub::DeviceRadixSort::SortPairs(sort_tmp, sort_bytes, keys, vals, (int)m2, 0, nbits, s);
        const unsigned long long* ks = keys.Current();
        const int64_t* vs = vals.Current();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(kg_weight_kernel, dim3(g_m2), dim3(256), 0, s, m2, k, scale_rank, ks, vs, d2, keep, wts);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(scan_tmp, scan_bytes, keep, pos, (int)m2, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hlast[0], pos + (m2 - 1), 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hlast[1], keep + (m2 - 1), 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        count = (int64_t)hlast[0] + hlast[1];
        if (e == hipSuccess) {
            hipLaunchKernelGGL(kg_scatter_kernel, dim3(g_m2), dim3(256), 0, s, m2, ks, keep, pos, wts, col, weight,
                               rows);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(kg_rowptr_kernel, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, n, count,
                               rows, row_ptr, flags);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&hflags, flags, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e == hipSuccess && (hflags & KG_ISOLATED))
            st = kfail(GL_E_BAD_GRAPH, "a point has no edge of positive weight (isolated)");
    }
    const hipError_t ef = hipFreeAsync(base, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (st != GL_OK) return st;
    if (e != hipSuccess || ef != hipSuccess || es != hipSuccess)
        return kfail(GL_E_HIP, std::string("kNN graph: ") + hipGetErrorString(e != hipSuccess ? e : (ef != hipSuccess ? ef : es)));
    *nnz = count;
    return GL_OK;
}
