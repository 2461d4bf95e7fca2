// Direct layout (CSR rows with 32- or 64-bit offsets and 32-bit columns):
// the row gather and the sweep, Laplacian and power-method kernels built on it.
//
// Work mapping (CDNA4, 64-lane wavefronts): a group of G lanes (G a power of
// two, 4..64, chosen from the mean row length) owns one CSR row.  Lane q of the
// group streams nonzeros q, q+G, q+2G, ... so one load instruction of the
// wavefront reads 64/G consecutive rows' index and weight runs; each nonzero
// gathers the whole K-wide row of V with one or a few vector loads.  The G
// partial sums are combined by a butterfly of cross-lane swaps, which leaves
// the same bits in every lane of the group; lane q then finishes columns q,
// q+G, ...  Every sum has a fixed order, independent of K and of the launch, so
// results are bitwise reproducible.
#pragma once

#include "gl_kernels.hpp"

namespace gl {

// z += sum of what_ij V[j, :] over entries p, p + S, p + 2S, ... < end, added
// in that order (four entries' index, weight and V loads in flight at once for
// K <= 4; two for wider rows, whose four V rows would cost too many registers).
template <int K, typename TW, typename TU, typename OffT, typename A>
__device__ __forceinline__ void row_accumulate(const int32_t* __restrict__ col, const TW* __restrict__ w,
                                               const TU* __restrict__ V, OffT p, OffT end, int S, A (&z)[K]) {
    const OffT s = (OffT)S;
    if constexpr (K <= 4)
    for (; p + 3 * s < end; p += 4 * s) {
        const int32_t j0 = col[p], j1 = col[p + s], j2 = col[p + 2 * s], j3 = col[p + 3 * s];
        const A w0 = cvt<A>(w[p]), w1 = cvt<A>(w[p + s]), w2 = cvt<A>(w[p + 2 * s]), w3 = cvt<A>(w[p + 3 * s]);
        A v0[K], v1[K], v2[K], v3[K];
        load_row<K>(V + (int64_t)j0 * K, v0);
        load_row<K>(V + (int64_t)j1 * K, v1);
        load_row<K>(V + (int64_t)j2 * K, v2);
        load_row<K>(V + (int64_t)j3 * K, v3);
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += w0 * v0[k];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += w1 * v1[k];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += w2 * v2[k];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += w3 * v3[k];
    }
    for (; p + s < end; p += 2 * s) {
        const int32_t j0 = col[p], j1 = col[p + s];
        const A w0 = cvt<A>(w[p]), w1 = cvt<A>(w[p + s]);
        A v0[K], v1[K];
        load_row<K>(V + (int64_t)j0 * K, v0);
        load_row<K>(V + (int64_t)j1 * K, v1);
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += w0 * v0[k];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += w1 * v1[k];
    }
    if (p < end) {
        const int32_t j0 = col[p];
        const A w0 = cvt<A>(w[p]);
        A v0[K];
        load_row<K>(V + (int64_t)j0 * K, v0);
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] += w0 * v0[k];
    }
}

// z = sum_j what_ij V[j, :] for `row`, completed in every lane of its G-lane group.
// Rows >= n contribute zeros but still take part in the cross-lane swaps.
template <int K, typename TW, typename TU, typename OffT, typename A>
__device__ __forceinline__ void row_gather(const OffT* __restrict__ rp, const int32_t* __restrict__ col,
                                           const TW* __restrict__ w, const TU* __restrict__ V,
                                           int64_t row, int64_t n, int q, int G, A (&z)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = (A)0;
    if (row < n) row_accumulate<K>(col, w, V, rp[row] + (OffT)q, rp[row + 1], G, z);
    group_butterfly<K>(z, __builtin_ctz((unsigned)G));
}

// The fused update of column k of row `node` (Prop. 1, Section 3.1) from
// zk = (What v)_{node,k}, the row's u^t and v and its label: writes v' (unless
// this is the energy-only pass) and adds |r|^2 and the energy terms of u^t
// (Section 2.1) to the lane's accumulators.
template <int K, typename TW, typename TU, typename OffT, typename A>
__device__ __forceinline__ void update_column(const SweepArgs<TW, TU, OffT>& a, int64_t node, int k, int32_t lab,
                                              A dl, A u, A v, A zk, A& e_acc, A& r_acc) {
    const A lam = lab >= 0 ? (A)1 : (A)0;
    const A ginv = a.dd ? (A)1 / (a.k.ga + a.k.gd * dl + a.k.gl * lam) : (lab >= 0 ? a.k.ginv1 : a.k.ginv0);
    const A y = lab < 0 ? (A)0 : (K == 1 ? (lab == 1 ? (A)1 : (A)-1) : (lab == k ? (A)1 : (A)-1));
    const A rhs = a.k.c * u - (u * u * u - u) * a.k.inv_eps + a.k.eta * lam * y;
    const A lv = a.dd ? dl * v - zk : v - zk;  // (L v)_i or (L_s v)_i
    const A tv = a.k.eps * lv + (a.k.eta * lam + a.k.c) * v;
    const A r = a.k.alpha * (u - v) + a.k.kappa * (rhs - tv);
    if (a.vout) a.vout[node * K + k] = store_as<TU>::from(v + r * ginv);
    r_acc += r * r;
    if (a.energy) {
        const A u2m1 = u * u - (A)1, dy = u - y;
        const A ulu = fma_acc(u, a.dd ? dl * u : u, -(u * zk));  // u (L u)_i, one rounding
        e_acc += a.k.half_eps * ulu + a.k.quarter_inv_eps * u2m1 * u2m1 + a.k.half_eta * lam * dy * dy;
    }
}

// One sweep (or the energy-only pass) over logical row block b, writing its
// statistics to partial slot `slot` of nb.  The rows' offsets are loaded for
// all passes first, and each row's own inputs (label, u^t, v) are requested
// before its gather, so a wavefront waits on memory about twice per pass.
// Heavy rows (longer than 16 G) are skipped here: heavy_block sums them.
template <int K, typename TW, typename TU, typename OffT>
__device__ __forceinline__ void sweep_block(const SweepArgs<TW, TU, OffT>& a, int64_t b, int64_t slot, int64_t nb) {
    typedef typename acc_of<TU>::type A;
    constexpr int CPL = (K + 3) / 4;  // columns per lane (G >= 4)
    constexpr int kMaxPasses = 4;
    const int G = a.g.G;
    const int q = threadIdx.x & (G - 1);
    const int grp = threadIdx.x >> a.g.log2G;
    const int rows_per_tile = kBlock >> a.g.log2G;
    const int64_t row0 = b * a.g.rows_per_block;
    const OffT heavy_min = a.nheavy > 0 ? (OffT)(16 * G) : (OffT)-1;
    A e_acc[CPL], r_acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) e_acc[c] = r_acc[c] = (A)0;
    OffT beg[kMaxPasses], end[kMaxPasses];
#pragma unroll
    for (int t = 0; t < kMaxPasses; ++t) {
        const int64_t row = row0 + (int64_t)t * rows_per_tile + grp;
        beg[t] = end[t] = 0;
        if (t < a.g.tiles && row < a.g.n) {
            beg[t] = a.rp[row];
            end[t] = a.rp[row + 1];
        }
    }
#pragma unroll
    for (int t = 0; t < kMaxPasses; ++t) {
        if (t >= a.g.tiles) break;
        const int64_t row = row0 + (int64_t)t * rows_per_tile + grp;
        const bool live = row < a.g.n && !(heavy_min >= 0 && end[t] - beg[t] > heavy_min);
        const int64_t node = live ? (a.order ? (int64_t)a.order[row] : row) : 0;
        int32_t lab = -1;
        A dl = (A)1;
        // own-row inputs as stored: converted only after the gathers are
        // issued, so that their loads are in flight together
        TU ur[CPL], vr[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) ur[c] = vr[c] = store_as<TU>::from((A)0);
        if (live) {
            lab = a.labels[node];
            if (a.dd) dl = a.dd[node];
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int k = q + c * G;
                if (k < K) {
                    ur[c] = a.ut[node * K + k];
                    vr[c] = a.vin[node * K + k];
                }
            }
        }
        A z[K];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] = (A)0;
        if (live) row_accumulate<K>(a.col, a.w, a.vin, beg[t] + (OffT)q, end[t], G, z);
        group_butterfly<K>(z, a.g.log2G);
        if (live) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int k = q + c * G;
                if (k < K)
                    update_column<K>(a, node, k, lab, dl, cvt<A>(late(ur[c])), cvt<A>(late(vr[c])), pick<K>(z, k),
                                     e_acc[c], r_acc[c]);
            }
        }
    }
    if (a.partials) block_stats<K, CPL>(e_acc, r_acc, G, a.partials, nb, slot);
}

// One heavy row (h < nheavy; workgroups up to the multiple of 8 are idle) with
// the whole workgroup: lane l adds entries l, l + 256, ... in order, the
// wavefronts reduce in a fixed order (DPP), then the four wavefronts in order,
// so the sum does not depend on K or on the launch.  Thread k < K finishes
// column k and writes statistic k (energy) and K + k (|r|^2) of slot `slot`.
template <int K, typename TW, typename TU, typename OffT>
__device__ __forceinline__ void heavy_block(const SweepArgs<TW, TU, OffT>& a, int64_t h, int64_t slot, int64_t nb) {
    typedef typename acc_of<TU>::type A;
    __shared__ A sh[kBlock / 64][K];
    const bool live = h < a.nheavy;
    const int64_t row = live ? (int64_t)a.heavy[h] : 0;
    const int k = threadIdx.x;
    const int64_t node = live ? (a.order ? (int64_t)a.order[row] : row) : 0;
    int32_t lab = -1;
    A dl = (A)1, u = (A)0, v = (A)0;
    if (live && k < K) {
        lab = a.labels[node];
        if (a.dd) dl = a.dd[node];
        u = cvt<A>(a.ut[node * K + k]);
        v = cvt<A>(a.vin[node * K + k]);
    }
    A z[K];
#pragma unroll
    for (int c = 0; c < K; ++c) z[c] = (A)0;
    if (live) row_accumulate<K>(a.col, a.w, a.vin, a.rp[row] + (OffT)threadIdx.x, a.rp[row + 1], kBlock, z);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        const A s = wave_sum63(z[c]);
        if (lane == 63) sh[wave][c] = s;
    }
    __syncthreads();
    A e = (A)0, r2 = (A)0;
    if (live && k < K) {
        const A zk = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
        update_column<K>(a, node, k, lab, dl, u, v, zk, e, r2);
    }
    if (a.partials && k < K) {
        a.partials[(int64_t)k * nb + slot] = e;
        a.partials[(int64_t)(K + k) * nb + slot] = r2;
    }
}

// One sweep (or the energy-only pass) for K columns: the heavy rows'
// workgroups first, then the row blocks (XCD-aware order).
template <int K, typename TW, typename TU, typename OffT>
__global__ __launch_bounds__(kBlock) void sweep_kernel(SweepArgs<TW, TU, OffT> a) {
    const int64_t hb = a.hblocks, nb = (int64_t)gridDim.x;
    const int64_t x = (int64_t)blockIdx.x;
    if (x < hb) {
        heavy_block<K>(a, x, x, nb);
        return;
    }
    const int64_t b = a.g.remap ? xcd_remap(x - hb, nb - hb) : x - hb;
    sweep_block<K>(a, b, hb + b, nb);
}

// Y = X - What X (L_s X) or Y = D X - W X (L X), Section 2.2
template <typename TW, typename TU, typename OffT> struct LapArgs {
    const OffT* rp;
    const int32_t* col;
    const TW* w;
    const TU* x;
    TU* y;
    const int32_t* order;
    const typename acc_of<TU>::type* dd;  // d_i of L, or nullptr for L_s
    RowGeom g;
};

template <int K, typename TW, typename TU, typename OffT>
__global__ __launch_bounds__(kBlock) void laplacian_kernel(LapArgs<TW, TU, OffT> a) {
    typedef typename acc_of<TU>::type A;
    constexpr int CPL = (K + 3) / 4;
    const int G = a.g.G;
    const int q = threadIdx.x & (G - 1);
    const int grp = threadIdx.x >> a.g.log2G;
    const int rows_per_tile = kBlock >> a.g.log2G;
    const int64_t b = a.g.remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t row0 = b * a.g.rows_per_block;
    for (int t = 0; t < a.g.tiles; ++t) {
        const int64_t row = row0 + (int64_t)t * rows_per_tile + grp;
        A z[K];
        row_gather<K>(a.rp, a.col, a.w, a.x, row, a.g.n, q, G, z);
        if (row < a.g.n) {
            const int64_t node = a.order ? (int64_t)a.order[row] : row;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int k = q + c * G;
                if (k < K) {
                    const int64_t at = node * K + k;
                    const A xv = cvt<A>(a.x[at]);
                    a.y[at] = store_as<TU>::from((a.dd ? a.dd[node] * xv : xv) - pick<K>(z, k));
                }
            }
        }
    }
}

// Power-method pass on float vectors with lx = L_s x = x - What x (or L x =
// d x - W x).  mode 0: y = s lx with s = *scale, partial[0] = sum y^2.
// mode 1: partial[0] = sum x lx, partial[1] = sum x^2.
template <typename TW, typename OffT> struct PowerArgs {
    const OffT* rp;
    const int32_t* col;
    const TW* w;
    const float* x;
    float* y;
    const float* scale;
    float* partials;  // [2][grid]
    const int32_t* order;
    const float* dd;  // d_i of L, or nullptr for L_s
    RowGeom g;
    int32_t mode;
};

template <typename TW, typename OffT>
__global__ __launch_bounds__(kBlock) void power_kernel(PowerArgs<TW, OffT> a) {
    const int G = a.g.G;
    const int q = threadIdx.x & (G - 1);
    const int grp = threadIdx.x >> a.g.log2G;
    const int rows_per_tile = kBlock >> a.g.log2G;
    const int64_t b = a.g.remap ? xcd_remap(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    const int64_t row0 = b * a.g.rows_per_block;
    const float s = a.mode == 0 ? *a.scale : 1.0f;
    float p0 = 0.f, p1 = 0.f;
    for (int t = 0; t < a.g.tiles; ++t) {
        const int64_t row = row0 + (int64_t)t * rows_per_tile + grp;
        float z[1];
        row_gather<1>(a.rp, a.col, a.w, a.x, row, a.g.n, q, G, z);
        if (row < a.g.n && q == 0) {
            const int64_t node = a.order ? (int64_t)a.order[row] : row;
            const float xv = a.x[node];
            const float lx = (a.dd ? a.dd[node] * xv : xv) - z[0];
            if (a.mode == 0) {
                const float yv = s * lx;
                a.y[node] = yv;
                p0 += yv * yv;
            } else {
                p0 += xv * lx;
                p1 += xv * xv;
            }
        }
    }
    float e[1] = {p0}, r[1] = {p1};
    block_stats<1, 1>(e, r, G, a.partials, (int64_t)gridDim.x, b);
}

}  // namespace gl
