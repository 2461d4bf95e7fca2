// Kernels of the gfx950 preconditioned-DCA library and their launch helpers.
#pragma once

#include "gl_device.hpp"

namespace gl {

constexpr int kBlock = 256;  // 4 wavefronts of 64 lanes

// Per-launch geometry shared by the row kernels: block b (after the XCD remap)
// owns rows [b * rows_per_block, (b + 1) * rows_per_block), processed as `tiles`
// passes of 256 / G rows.
struct RowGeom {
    int64_t n;
    int64_t rows_per_block;
    int32_t G;
    int32_t log2G;
    int32_t tiles;
    int32_t remap;
};

template <typename A> struct SweepCoef {
    A eps, c, eta;          // model parameters
    A inv_eps;              // 1 / eps
    A half_eps, quarter_inv_eps, half_eta;  // energy prefactors
    A ginv0, ginv1;         // 1 / g for unlabelled (Lambda = 0) and labelled rows (L_s)
    A alpha, kappa;         // r = alpha (u^t - v) + kappa (b - T v)
    A ga, gd, gl;           // unnormalized L: g_i = ga + gd d_i + gl Lambda_i
};

template <typename TW, typename TU, typename OffT> struct SweepArgs {
    typedef typename acc_of<TU>::type A;
    const OffT* rp;
    const int32_t* col;
    const TW* w;
    const TU* ut;      // u^t, read on the own row for b
    const TU* vin;     // v^s, gathered
    TU* vout;          // v^{s+1}; nullptr for the energy-only pass
    const int32_t* labels;
    const int32_t* order;  // node of each row position, or nullptr (identity)
    const A* dd;       // diagonal d_i of L = D - W, or nullptr for L_s (diagonal 1)
    A* partials;       // [2K][grid] block partial sums, or nullptr
    RowGeom g;
    int32_t energy;    // also accumulate the energy terms (vin == ut)
    SweepCoef<A> k;
    const int32_t* heavy;  // direct layout: rows longer than 16 G, summed by workgroups of their own
    int32_t nheavy;        // number of heavy rows
    int32_t hblocks;       // their workgroups (nheavy rounded up to a multiple of 8), first in the launch
};

// Fixed-order double reduction of one statistic per block: block s sums
// partials[s * nb .. s * nb + nb).
template <typename P>
__device__ __forceinline__ double block_sum(const P* __restrict__ src, int64_t nb) {
    __shared__ double sh[kBlock / 64];
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += kBlock) acc += (double)src[i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

// Solve statistics of up to kStatGroup sweeps, reduced by one launch: set j
// (block column j) holds the 2K statistics of one sweep at partials + j *
// stride; block s < K sums energy column s into energy_dst[j][s] (nullptr:
// none), block K + k the |r|^2 of column k into res_dst[j][k], each in the
// fixed order of block_sum.  A non-finite sum sets *flag to 1.
constexpr int kStatGroup = 16;
struct StatGroup {
    double* energy_dst[kStatGroup];
    double* res_dst[kStatGroup];
};

template <typename P>
__global__ __launch_bounds__(kBlock) void finalize_group_kernel(const P* partials, int64_t nb, int64_t stride,
                                                                int32_t K, StatGroup g, double* flag) {
    const int s = blockIdx.x, j = blockIdx.y;
    double* dst = s < K ? g.energy_dst[j] : g.res_dst[j];
    if (dst == nullptr) return;  // uniform per block
    const double v = block_sum(partials + (int64_t)j * stride + (int64_t)s * nb, nb);
    if (threadIdx.x == 0) {
        dst[s < K ? s : s - K] = v;
        if (!(fabs(v) <= 1.7976931348623157e308)) *flag = 1.0;
    }
}

// Power method: scale_out = 1 / sqrt(sum partial[scale_stat]); sums_out (optional)
// gets both sums in double.
static __global__ __launch_bounds__(kBlock) void power_finalize_kernel(const float* partials, int64_t nb,
                                                                int32_t scale_stat, float* scale_out,
                                                                double* sums_out) {
    const double s0 = block_sum(partials, nb);
    __syncthreads();
    const double s1 = block_sum(partials + nb, nb);
    if (threadIdx.x == 0) {
        if (scale_out) *scale_out = (float)(1.0 / sqrt(scale_stat ? s1 : s0));
        if (sums_out) {
            sums_out[0] = s0;
            sums_out[1] = s1;
        }
    }
}

static __global__ void fill_double_kernel(double* p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static __global__ void copy_bytes_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst, int64_t n16,
                                  const uint8_t* __restrict__ src_tail, uint8_t* __restrict__ dst_tail,
                                  int32_t tail) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) dst[i] = src[i];
    if (i < tail) dst_tail[i] = src_tail[i];
}

// Move whole rows between node order and position order:
//   gather  (scatter = 0): dst[p] = src[order[p]]
//   scatter (scatter = 1): dst[order[p]] = src[p]
// Rows are `words` units of W (a row of K field values).
template <typename W>
__global__ void permute_rows_kernel(int64_t n, int32_t words, const int32_t* __restrict__ order,
                                    const W* __restrict__ src, W* __restrict__ dst, int32_t scatter) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * words) return;
    const int64_t p = i / words, j = i - p * words;
    const int64_t o = (int64_t)order[p] * words + j;
    if (scatter)
        dst[o] = src[i];
    else
        dst[i] = src[o];
}

// Bandwidth ceilings (measurement helpers).  Each thread moves four 16-byte
// vectors per step (non-temporal, grid-stride); the read-only kernel folds
// what it reads into a value it stores only if it matches `never`, so the
// loads cannot be dropped and nothing is written in practice.
static __global__ __launch_bounds__(256) void stream_read_kernel(const u32x4* __restrict__ src, int64_t n16,
                                                                 uint32_t never, u32x4* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    u32x4 acc = {0u, 0u, 0u, 0u};
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(src + i);
        const u32x4 b = __builtin_nontemporal_load(src + i + stride);
        const u32x4 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(src + i + 3 * stride);
        acc ^= (a ^ b) ^ (c ^ d);
    }
    for (; i < n16; i += stride) acc ^= __builtin_nontemporal_load(src + i);
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == never) sink[0] = acc;
}

static __global__ __launch_bounds__(256) void stream_copy_kernel(const u32x4* __restrict__ src,
                                                                 u32x4* __restrict__ dst, int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(src + i);
        const u32x4 b = __builtin_nontemporal_load(src + i + stride);
        const u32x4 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const u32x4 d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n16; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

template <typename TU>
__global__ void labels_kernel(int64_t n, int32_t K, const TU* __restrict__ U, int32_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    typedef typename acc_of<TU>::type A;
    if (K == 1) {
        out[i] = cvt<A>(U[i]) >= (A)0 ? 1 : 0;
        return;
    }
    A best = cvt<A>(U[i * K]);
    int32_t arg = 0;
    for (int k = 1; k < K; ++k) {
        const A v = cvt<A>(U[i * K + k]);
        if (v > best) {
            best = v;
            arg = k;
        }
    }
    out[i] = arg;
}

// ---------------------------------------------------------------------------
// operator construction (once per graph)
// ---------------------------------------------------------------------------
enum : int32_t {
    BAD_ROWPTR = 1,
    BAD_COL_RANGE = 2,
    BAD_COL_ORDER = 4,
    BAD_SELF_LOOP = 8,
    BAD_WEIGHT = 16,
    BAD_ASYMMETRIC = 32,
    BAD_DEGREE = 64
};

template <typename TIN>
__global__ void validate_kernel(int64_t n, int64_t nnz, const int64_t* __restrict__ rp,
                                const int32_t* __restrict__ col, const TIN* __restrict__ w,
                                int32_t* flags, unsigned long long* first_bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t f = 0;
    const int64_t beg = rp[i], end = rp[i + 1];
    if (beg < 0 || end < beg || end > nnz) {
        f |= BAD_ROWPTR;
    } else {
        int64_t prev = -1;
        for (int64_t p = beg; p < end; ++p) {
            const int64_t j = col[p];
            if (j < 0 || j >= n) {
                f |= BAD_COL_RANGE;
                break;
            }
            if (j <= prev) f |= BAD_COL_ORDER;
            prev = j;
            if (j == i) f |= BAD_SELF_LOOP;
            const double wv = (double)w[p];
            if (!(wv > 0.0) || !(wv <= 1.7976931348623157e308)) f |= BAD_WEIGHT;
            // symmetry: find i in row j by binary search and compare the weight bits
            const int64_t jb = rp[j], je = rp[j + 1];
            if (jb < 0 || je < jb || je > nnz) {
                f |= BAD_ROWPTR;
                continue;
            }
            int64_t lo = jb, hi = je;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < i) lo = mid + 1; else hi = mid;
            }
            if (lo >= je || col[lo] != i || !(w[lo] == w[p])) f |= BAD_ASYMMETRIC;
        }
    }
    if (f) {
        atomicOr(flags, f);
        atomicMin(first_bad, (unsigned long long)i);
    }
}

template <typename TIN>
__global__ void degree_kernel(int64_t n, const int64_t* __restrict__ rp, const TIN* __restrict__ w,
                              double* __restrict__ d, int32_t* flags, unsigned long long* first_bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += (double)w[p];
    d[i] = s;
    if (!(s > 0.0) || !(s <= 1.7976931348623157e308)) {
        atomicOr(flags, (int32_t)BAD_DEGREE);
        atomicMin(first_bad, (unsigned long long)i);
    }
}

// what_ij = w_ij / (sqrt(d_i) sqrt(d_j)) in double, rounded once to TOUT; the index
// arrays are copied (row offsets narrowed to OffT) in the same pass.
// raw != 0 (unnormalized L = D - W): w_ij itself, rounded once to TOUT.
template <typename TIN, typename TOUT, typename OffT>
__global__ void normalize_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 const TIN* __restrict__ w, const double* __restrict__ d,
                                 OffT* __restrict__ rp_out, int32_t* __restrict__ col_out,
                                 TOUT* __restrict__ w_out, int32_t raw) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    rp_out[i] = (OffT)rp[i];
    if (i == n) return;
    const double di = d[i];
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
        const int32_t j = col[p];
        col_out[p] = j;
        w_out[p] = store_as<TOUT>::from(raw ? (double)w[p] : (double)w[p] / (sqrt(di) * sqrt(d[j])));
    }
}

// Diagonal of the unnormalized operator as stored: dd_p = sum of the row's
// stored (rounded) weights, summed in double in storage order, rounded to A.
// Keeps L 1 = 0 for the weights the sweeps actually use.
template <typename TW, typename OffT, typename A>
__global__ void rowsum_kernel(int64_t n, const OffT* __restrict__ rp, const TW* __restrict__ w,
                              A* __restrict__ dd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t p = rp[i]; p < rp[i + 1]; ++p) s += cvt<double>(w[p]);
    dd[i] = (A)s;
}

}  // namespace gl
