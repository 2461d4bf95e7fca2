// Halo-staged ("tile") kernels of the gfx950 preconditioned-DCA library.
//
// Operator layout: the rows are visited in a caller-chosen processing order
// (for an image graph, the Z-order of the pixel grid) and cut into blocks of
// 256 consecutive positions.  Block b lists the distinct columns its rows
// reference -- its halo, halo[hp[b] .. hp[b+1]) -- and every stored nonzero
// carries a 16-bit index into that list instead of a 32-bit column.  Rows are
// padded to a multiple of 4 entries (index 0xFFFF marks padding) so that one
// lane reads 4 consecutive entries with a single vector load.
//
// Kernel plan (one 256-thread workgroup per block, no dependent global loads
// beyond two levels):
//   1. halo ids and each lane group's row offsets -> registers;
//   2. issue the gathers of the halo rows of V, then the first 4-entry chunk of
//      every row's index/weight stream;
//   3. halo rows -> LDS, barrier, own-row inputs of the epilogue, products from
//      LDS, butterfly over the 4 lanes of each row (fixed order), epilogue on
//      lanes q = column (mod 4).
// Gathers thus hit LDS instead of the vector L1, and the index stream shrinks
// from 4 to 2 bytes per nonzero.
#pragma once

#include <type_traits>

#include "gl_kernels.hpp"

namespace gl {

constexpr int kTileRows = 256;   // positions per block
constexpr int kTileG = 4;        // lanes per row
// 4-entry chunks per lane loaded before the halo is staged: one for 2-byte
// weights (fewer live registers, more resident blocks), two for 4- and 8-byte
// weights; with 2-byte weights the second chunk is loaded right after the
// halo rows have gone to LDS (their registers are free by then), close enough
// to the first to find its cache lines still in L2.
template <typename TW> constexpr int tile_unr() { return sizeof(TW) == 2 ? 1 : 2; }
template <typename TW> constexpr int tile_late() { return sizeof(TW) == 2 ? 1 : 0; }
constexpr int kTileRPT = 256 / kTileG;            // rows per pass of the block
constexpr int kTilePasses = kTileRows / kTileRPT;  // 4
constexpr int kTileHPT = 4;      // halo entries per thread held in registers
constexpr int kTileHaloMax = 960;  // halo limit: 960 * 16 columns * 4 B + offsets < 64 KB

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

struct u32x8 {
    u32x4 lo, hi;
};
template <typename TW> struct wvec4;
template <> struct wvec4<double> { typedef u32x8 type; };
template <> struct wvec4<float> { typedef u32x4 type; };
template <> struct wvec4<bf16> { typedef u32x2 type; };
template <> struct wvec4<f16> { typedef u32x2 type; };

struct TileOp {
    const int32_t* rp;      // [n + 1] padded entry offsets per position
    const uint16_t* lcol;   // [padded nnz] halo-local column, 0xFFFF = padding
    const void* w;          // [padded nnz] normalized weights (0 on padding)
    const int32_t* halo;    // [total halo] node ids, sorted within a block
    const int32_t* hp;      // [blocks + 1] halo offsets
    const int32_t* order;   // [n] node of each position, or nullptr (identity)
    int64_t n;
};

// Rows of the block handled by this lane's group: pass tt covers position
// b * 256 + tt * 64 + group.
struct TileRows {
    int64_t node[kTilePasses];
    bool ok[kTilePasses];
};

// Phases 1-3 for one block.  Order of the loads: halo ids and row offsets,
// then the gathers of the halo rows of V (so that they return first and the
// halo can be staged in LDS while the index/weight stream is still in flight),
// then the first chunk of every row.  `prefetch(rows)` runs after the barrier
// (the caller's own-row loads); `finish(tt, zs)` receives the completed sums of
// pass tt for the columns q, q + 4, ... that lane q finishes.
template <int K, typename TW, typename TU, typename A, typename Prefetch, typename Finish>
__device__ __forceinline__ void tile_products(const TileOp& op, const TU* __restrict__ V, int64_t b, A* hv,
                                              TileRows& rows, Prefetch&& prefetch, Finish&& finish) {
    typedef typename wvec4<TW>::type WV;
    const TW* __restrict__ w = static_cast<const TW*>(op.w);
    const int t = threadIdx.x;
    const int64_t n = op.n;
    const int64_t row0 = b * kTileRows;
    const int q = t & (kTileG - 1), grp = t / kTileG;
    const int32_t hb = op.hp[b], he = op.hp[b + 1];
    int32_t hid[kTileHPT];
#pragma unroll
    for (int i = 0; i < kTileHPT; ++i) hid[i] = (hb + t + 256 * i < he) ? op.halo[hb + t + 256 * i] : -1;
    int32_t beg[kTilePasses], end[kTilePasses];
#pragma unroll
    for (int tt = 0; tt < kTilePasses; ++tt) {
        const int64_t p = row0 + tt * kTileRPT + grp;
        const int64_t p0 = p < n ? p : n, p1 = p + 1 < n ? p + 1 : n;
        beg[tt] = op.rp[p0];
        end[tt] = op.rp[p1];
        rows.ok[tt] = p < n;
        rows.node[tt] = rows.ok[tt] ? (op.order ? (int64_t)op.order[p] : p) : 0;
    }
    A hvr[kTileHPT][K];
#pragma unroll
    for (int i = 0; i < kTileHPT; ++i)
        if (hid[i] >= 0) load_row<K>(V + (int64_t)hid[i] * K, hvr[i]);
    constexpr int kTileUnr = tile_unr<TW>();
    u32x2 lr[kTilePasses][kTileUnr];
    WV wr[kTilePasses][kTileUnr];
#pragma unroll
    for (int tt = 0; tt < kTilePasses; ++tt) {
#pragma unroll
        for (int u = 0; u < kTileUnr; ++u) {
            const int32_t pp = beg[tt] + 4 * q + 4 * kTileG * u;
            if (pp < end[tt]) {
                lr[tt][u] = *reinterpret_cast<const u32x2*>(op.lcol + pp);
                wr[tt][u] = *reinterpret_cast<const WV*>(w + pp);
            } else {
                lr[tt][u] = u32x2{0xFFFFFFFFu, 0xFFFFFFFFu};
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kTileHPT; ++i) {
        if (hid[i] >= 0) {
#pragma unroll
            for (int k = 0; k < K; ++k) hv[(t + 256 * i) * K + k] = hvr[i][k];
        }
    }
    for (int32_t idx = t + 256 * kTileHPT; idx < he - hb; idx += 256) {
        A v[K];
        load_row<K>(V + (int64_t)op.halo[hb + idx] * K, v);
#pragma unroll
        for (int k = 0; k < K; ++k) hv[idx * K + k] = v[k];
    }
    constexpr int kTileLate = tile_late<TW>();
    u32x2 lr2[kTilePasses][kTileLate > 0 ? kTileLate : 1];
    WV wr2[kTilePasses][kTileLate > 0 ? kTileLate : 1];
#pragma unroll
    for (int tt = 0; tt < kTilePasses; ++tt) {
#pragma unroll
        for (int u = 0; u < kTileLate; ++u) {
            const int32_t pp = beg[tt] + 4 * q + 4 * kTileG * (kTileUnr + u);
            if (pp < end[tt]) {
                lr2[tt][u] = *reinterpret_cast<const u32x2*>(op.lcol + pp);
                wr2[tt][u] = *reinterpret_cast<const WV*>(w + pp);
            } else {
                lr2[tt][u] = u32x2{0xFFFFFFFFu, 0xFFFFFFFFu};
            }
        }
    }
    __syncthreads();  // halo visible
    prefetch(rows);
    static_for<0, kTilePasses>([&](auto TT) {
        constexpr int tt = decltype(TT)::value;
        A z[K];
#pragma unroll
        for (int k = 0; k < K; ++k) z[k] = (A)0;
#pragma unroll
        for (int u = 0; u < kTileUnr; ++u) {
            uint16_t li[4];
            TW wi[4];
            __builtin_memcpy(li, &lr[tt][u], 8);
            __builtin_memcpy(wi, &wr[tt][u], sizeof(WV));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (li[e] != 0xFFFFu) {
                    const A we = cvt<A>(wi[e]);
#pragma unroll
                    for (int k = 0; k < K; ++k) z[k] += we * hv[(int32_t)li[e] * K + k];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kTileLate; ++u) {
            uint16_t li[4];
            TW wi[4];
            __builtin_memcpy(li, &lr2[tt][u], 8);
            __builtin_memcpy(wi, &wr2[tt][u], sizeof(WV));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (li[e] != 0xFFFFu) {
                    const A we = cvt<A>(wi[e]);
#pragma unroll
                    for (int k = 0; k < K; ++k) z[k] += we * hv[(int32_t)li[e] * K + k];
                }
            }
        }
        // the rest of the row, one 4-entry chunk per lane at a time
        for (int32_t pp = beg[tt] + 4 * q + 4 * kTileG * (kTileUnr + kTileLate); pp < end[tt];
             pp += 4 * kTileG) {
            const u32x2 l2 = *reinterpret_cast<const u32x2*>(op.lcol + pp);
            const WV w2 = *reinterpret_cast<const WV*>(w + pp);
            uint16_t li[4];
            TW wi[4];
            __builtin_memcpy(li, &l2, 8);
            __builtin_memcpy(wi, &w2, sizeof(WV));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if (li[e] != 0xFFFFu) {
                    const A we = cvt<A>(wi[e]);
#pragma unroll
                    for (int k = 0; k < K; ++k) z[k] += we * hv[(int32_t)li[e] * K + k];
                }
            }
        }
        for (int off = kTileG >> 1; off > 0; off >>= 1) {
#pragma unroll
            for (int k = 0; k < K; ++k) z[k] = xor_add(z[k], off);
        }
        // this lane finishes columns q, q + 4, ...
        constexpr int CPL = (K + kTileG - 1) / kTileG;
        A zs[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            // select z[4c + q] by the two bits of q from compile-time-indexed values
            const A c0 = z[(4 * c + 0) < K ? 4 * c + 0 : K - 1];
            const A c1 = z[(4 * c + 1) < K ? 4 * c + 1 : K - 1];
            const A c2 = z[(4 * c + 2) < K ? 4 * c + 2 : K - 1];
            const A c3 = z[(4 * c + 3) < K ? 4 * c + 3 : K - 1];
            zs[c] = (q & 2) ? ((q & 1) ? c3 : c2) : ((q & 1) ? c1 : c0);
        }
        finish(TT, zs);
    });
}

// ---------------------------------------------------------------------------
// sweep (and energy-only pass) on the tile layout
// ---------------------------------------------------------------------------
template <typename TU, typename A> struct TileSweepArgs {
    TileOp op;
    const TU* ut;
    const TU* vin;
    TU* vout;  // nullptr: energy-only pass
    const int32_t* labels;
    const A* dd;  // d_i of L = D - W by position, or nullptr for L_s
    A* partials;
    int32_t energy;
    SweepCoef<A> k;
};

template <int K, typename TW, typename TU>
__global__ __launch_bounds__(256) void tile_sweep_kernel(TileSweepArgs<TU, typename acc_of<TU>::type> a) {
    typedef typename acc_of<TU>::type A;
    constexpr int CPL = (K + kTileG - 1) / kTileG;
    extern __shared__ unsigned char smem_raw[];
    A* hv = reinterpret_cast<A*>(smem_raw);
    const int64_t b = blockIdx.x;
    const int q = threadIdx.x & (kTileG - 1);
    TileRows rows;
    int32_t lab[kTilePasses];
    A uu[kTilePasses][CPL], vv[kTilePasses][CPL];
    A dls[kTilePasses];
    A e_acc[CPL], r_acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) e_acc[c] = r_acc[c] = (A)0;
    auto prefetch = [&](TileRows& r) {
#pragma unroll
        for (int tt = 0; tt < kTilePasses; ++tt) {
            lab[tt] = r.ok[tt] ? a.labels[r.node[tt]] : -1;
            dls[tt] = (a.dd && r.ok[tt]) ? a.dd[r.node[tt]] : (A)1;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int k = q + c * kTileG;
                if (r.ok[tt] && k < K) {
                    uu[tt][c] = cvt<A>(a.ut[r.node[tt] * K + k]);
                    vv[tt][c] = cvt<A>(a.vin[r.node[tt] * K + k]);
                }
            }
        }
    };
    auto finish = [&](auto TT, const A (&zs)[CPL]) {
        constexpr int tt = decltype(TT)::value;
        if (!rows.ok[tt]) return;
        const int32_t l = lab[tt];
        const A lam = l >= 0 ? (A)1 : (A)0;
        const A dl = dls[tt];
        const A ginv = a.dd ? (A)1 / (a.k.ga + a.k.gd * dl + a.k.gl * lam) : (l >= 0 ? a.k.ginv1 : a.k.ginv0);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int k = q + c * kTileG;
            if (k < K) {
                const A zk = zs[c];
                const A u = uu[tt][c], v = vv[tt][c];
                const A y = l < 0 ? (A)0 : (K == 1 ? (l == 1 ? (A)1 : (A)-1) : (l == k ? (A)1 : (A)-1));
                const A rhs = a.k.c * u - (u * u * u - u) * a.k.inv_eps + a.k.eta * lam * y;
                const A lv = a.dd ? dl * v - zk : v - zk;
                const A tv = a.k.eps * lv + (a.k.eta * lam + a.k.c) * v;
                const A r = a.k.alpha * (u - v) + a.k.kappa * (rhs - tv);
                if (a.vout) a.vout[rows.node[tt] * K + k] = store_as<TU>::from(v + r * ginv);
                r_acc[c] += r * r;
                if (a.energy) {
                    const A u2m1 = u * u - (A)1, dy = u - y;
                    const A ulu = fma_acc(u, a.dd ? dl * u : u, -(u * zk));  // u (L u)_i, one rounding
                    e_acc[c] += a.k.half_eps * ulu + a.k.quarter_inv_eps * u2m1 * u2m1 +
                                a.k.half_eta * lam * dy * dy;
                }
            }
        }
    };
    tile_products<K, TW, TU, A>(a.op, a.vin, b, hv, rows, prefetch, finish);
    if (a.partials) block_stats<K, CPL>(e_acc, r_acc, kTileG, a.partials, (int64_t)gridDim.x, b);
}

// Y = X - What X (or D X - W X) on the tile layout
template <typename TU> struct TileLapArgs {
    TileOp op;
    const TU* x;
    TU* y;
    const typename acc_of<TU>::type* dd;  // d_i of L by position, or nullptr for L_s
};

template <int K, typename TW, typename TU>
__global__ __launch_bounds__(256) void tile_laplacian_kernel(TileLapArgs<TU> a) {
    typedef typename acc_of<TU>::type A;
    constexpr int CPL = (K + kTileG - 1) / kTileG;
    extern __shared__ unsigned char smem_raw[];
    A* hv = reinterpret_cast<A*>(smem_raw);
    const int q = threadIdx.x & (kTileG - 1);
    TileRows rows;
    A xx[kTilePasses][CPL];
    auto prefetch = [&](TileRows& r) {
#pragma unroll
        for (int tt = 0; tt < kTilePasses; ++tt)
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int k = q + c * kTileG;
                if (r.ok[tt] && k < K) {
                    const A xv = cvt<A>(a.x[r.node[tt] * K + k]);
                    xx[tt][c] = a.dd ? a.dd[r.node[tt]] * xv : xv;
                }
            }
    };
    auto finish = [&](auto TT, const A (&zs)[CPL]) {
        constexpr int tt = decltype(TT)::value;
        if (!rows.ok[tt]) return;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int k = q + c * kTileG;
            if (k < K) a.y[rows.node[tt] * K + k] = store_as<TU>::from(xx[tt][c] - zs[c]);
        }
    };
    tile_products<K, TW, TU, A>(a.op, a.x, (int64_t)blockIdx.x, hv, rows, prefetch, finish);
}

// Power-method pass on the tile layout (float vectors; see power_kernel).
struct TilePowerArgs {
    TileOp op;
    const float* x;
    float* y;
    const float* scale;
    float* partials;
    const float* dd;  // d_i of L by position, or nullptr for L_s
    int32_t mode;
};

template <typename TW>
__global__ __launch_bounds__(256) void tile_power_kernel(TilePowerArgs a) {
    extern __shared__ unsigned char smem_raw[];
    float* hv = reinterpret_cast<float*>(smem_raw);
    const int q = threadIdx.x & (kTileG - 1);
    TileRows rows;
    float xx[kTilePasses], dx[kTilePasses];
    const float s = a.mode == 0 ? *a.scale : 1.0f;
    float p0 = 0.f, p1 = 0.f;
    auto prefetch = [&](TileRows& r) {
#pragma unroll
        for (int tt = 0; tt < kTilePasses; ++tt) {
            xx[tt] = (r.ok[tt] && q == 0) ? a.x[r.node[tt]] : 0.f;
            dx[tt] = (a.dd && r.ok[tt] && q == 0) ? a.dd[r.node[tt]] * xx[tt] : xx[tt];
        }
    };
    auto finish = [&](auto TT, const float (&z)[1]) {
        constexpr int tt = decltype(TT)::value;
        if (!rows.ok[tt] || q != 0) return;
        const float lx = dx[tt] - z[0];
        if (a.mode == 0) {
            const float yv = s * lx;
            a.y[rows.node[tt]] = yv;
            p0 += yv * yv;
        } else {
            p0 += xx[tt] * lx;
            p1 += xx[tt] * xx[tt];
        }
    };
    tile_products<1, TW, float, float>(a.op, a.x, (int64_t)blockIdx.x, hv, rows, prefetch, finish);
    float e[1] = {p0}, r[1] = {p1};
    block_stats<1, 1>(e, r, kTileG, a.partials, (int64_t)gridDim.x, (int64_t)blockIdx.x);
}

// Fill the tile (or direct) weight array: entry e of position p takes the
// normalized weight of source entry src[e] (w / (sqrt(d_i) sqrt(d_j)), i the node of p),
// or 0 when src[e] < 0 (padding).  col_out (direct layout only) receives the
// source column, mapped through pos_of (node -> position) when ordered.
// raw != 0 (unnormalized L = D - W): the weight itself, rounded once.
template <typename TIN, typename TOUT>
__global__ void fill_layout_kernel(int64_t n, const int32_t* __restrict__ rp_out, const int32_t* __restrict__ src,
                                   const int32_t* __restrict__ order, const int32_t* __restrict__ pos_of,
                                   const int32_t* __restrict__ col, const TIN* __restrict__ w,
                                   const double* __restrict__ d, TOUT* __restrict__ w_out,
                                   int32_t* __restrict__ col_out, int32_t raw) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t i = order ? (int64_t)order[p] : p;
    const double di = d[i];
    for (int64_t e = rp_out[p]; e < rp_out[p + 1]; ++e) {
        const int32_t s = src[e];
        if (s >= 0) {
            const int32_t j = col[s];
            w_out[e] = store_as<TOUT>::from(raw ? (double)w[s] : (double)w[s] / (sqrt(di) * sqrt(d[j])));
            if (col_out) col_out[e] = pos_of ? pos_of[j] : j;
        } else {
            w_out[e] = store_as<TOUT>::from(0.0);
            if (col_out) col_out[e] = 0;
        }
    }
}

}  // namespace gl
