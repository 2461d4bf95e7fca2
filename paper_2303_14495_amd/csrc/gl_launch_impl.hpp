// Typed launch of the sweep and Laplacian kernels for one field storage type TU.
// Included by one translation unit per TU so the K x weight-type x index-width
// instantiations compile in parallel.
#pragma once

#include <type_traits>

#include "gl_internal.hpp"
#include "gl_kernels.hpp"
#include "gl_direct.hpp"
#include "gl_tile.hpp"
#include "gl_window.hpp"
#include "gl_grid.hpp"

namespace gl {

template <typename TW, typename TU, typename OffT>
static SweepArgs<TW, TU, OffT> make_sweep_args(const SweepLaunch& L) {
    typedef typename acc_of<TU>::type A;
    SweepArgs<TW, TU, OffT> a;
    a.rp = static_cast<const OffT*>(L.r.rp);
    a.col = L.r.col;
    a.w = static_cast<const TW*>(L.r.w);
    a.ut = static_cast<const TU*>(L.ut);
    a.vin = static_cast<const TU*>(L.vin);
    a.vout = static_cast<TU*>(L.vout);
    a.labels = L.labels;
    a.order = L.r.order;
    a.dd = static_cast<const A*>(L.r.dd);
    a.partials = static_cast<A*>(L.partials);
    a.g = RowGeom{L.r.n, L.r.rows_per_block, L.r.G, L.r.log2G, L.r.tiles, L.r.remap};
    a.energy = L.energy;
    a.k.eps = (A)L.coef[0];
    a.k.c = (A)L.coef[1];
    a.k.eta = (A)L.coef[2];
    a.k.inv_eps = (A)L.coef[3];
    a.k.half_eps = (A)L.coef[4];
    a.k.quarter_inv_eps = (A)L.coef[5];
    a.k.half_eta = (A)L.coef[6];
    a.k.ginv0 = (A)L.coef[7];
    a.k.ginv1 = (A)L.coef[8];
    a.k.alpha = (A)L.coef[9];
    a.k.kappa = (A)L.coef[10];
    a.k.ga = (A)L.coef[11];
    a.k.gd = (A)L.coef[12];
    a.k.gl = (A)L.coef[13];
    a.heavy = L.r.heavy;
    a.nheavy = L.r.layout == LAYOUT_DIRECT ? L.r.nheavy : 0;
    a.hblocks = (int32_t)(sweep_grid(L.r) - L.r.grid);
    return a;
}

#define GL_K_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

static TileOp tile_op(const RowLaunch& r) {
    TileOp op;
    op.rp = r.trp;
    op.lcol = r.lcol;
    op.w = r.w;
    op.halo = r.halo;
    op.hp = r.hp;
    op.order = r.order;
    op.n = r.n;
    return op;
}

template <typename TW, typename TU>
static hipError_t tile_sweep_k(int K, const SweepLaunch& L, hipStream_t s) {
    typedef typename acc_of<TU>::type A;
    TileSweepArgs<TU, A> a;
    a.op = tile_op(L.r);
    a.ut = static_cast<const TU*>(L.ut);
    a.vin = static_cast<const TU*>(L.vin);
    a.vout = static_cast<TU*>(L.vout);
    a.labels = L.labels;
    a.dd = static_cast<const A*>(L.r.dd);
    a.partials = static_cast<A*>(L.partials);
    a.energy = L.energy;
    const SweepArgs<TW, TU, int32_t> d = make_sweep_args<TW, TU, int32_t>(L);
    a.k = d.k;
    const dim3 grid((unsigned)L.r.grid), block(kBlock);
    const size_t lds = (size_t)L.r.hmax * K * sizeof(A);
    switch (K) {
#define GL_CASE(KK)                                                                       \
    case KK:                                                                              \
        hipLaunchKernelGGL((tile_sweep_kernel<KK, TW, TU>), grid, block, lds, s, a);     \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TW, typename TU>
static hipError_t tile_laplacian_k(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s) {
    typedef typename acc_of<TU>::type A;
    TileLapArgs<TU> a;
    a.op = tile_op(r);
    a.x = static_cast<const TU*>(x);
    a.y = static_cast<TU*>(y);
    a.dd = static_cast<const A*>(r.dd);
    const dim3 grid((unsigned)r.grid), block(kBlock);
    const size_t lds = (size_t)r.hmax * K * sizeof(A);
    switch (K) {
#define GL_CASE(KK)                                                                        \
    case KK:                                                                               \
        hipLaunchKernelGGL((tile_laplacian_kernel<KK, TW, TU>), grid, block, lds, s, a);  \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static WinOp window_op(const RowLaunch& r) {
    WinOp op;
    op.w = r.w;
    op.height = r.wheight;
    op.width = r.wwidth;
    op.r = r.wr;
    op.M = r.wM;
    op.tiles_x = r.wtiles_x;
    return op;
}

// LDS of window_part_kernel: V and the accumulator over one tile's region.
static size_t window_lds(const RowLaunch& r, int K, size_t acc) {
    return 2 * (size_t)K * window_region(r.wr) * acc;
}

// Region sums of W X over every tile into r.wpart (the first pass of each
// window product).
template <int K, typename TW, typename TU>
static void window_part_launch(const RowLaunch& r, const void* x, hipStream_t s) {
    typedef typename acc_of<TU>::type A;
    WinPartArgs<TU> a;
    a.op = window_op(r);
    a.v = static_cast<const TU*>(x);
    a.part = static_cast<A*>(r.wpart);
    hipLaunchKernelGGL((window_part_kernel<K, TW, TU>), dim3((unsigned)r.grid), dim3(256), window_lds(r, K, sizeof(A)),
                       s, a);
}

template <typename TW, typename TU>
static hipError_t window_sweep_k(int K, const SweepLaunch& L, hipStream_t s) {
    typedef typename acc_of<TU>::type A;
    if (!L.r.wpart) return hipErrorInvalidValue;
    WinSweepArgs<TU, A> a;
    a.op = window_op(L.r);
    a.part = static_cast<const A*>(L.r.wpart);
    a.ut = static_cast<const TU*>(L.ut);
    a.vin = static_cast<const TU*>(L.vin);
    a.vout = static_cast<TU*>(L.vout);
    a.labels = L.labels;
    a.dd = static_cast<const A*>(L.r.dd);
    a.partials = static_cast<A*>(L.partials);
    a.energy = L.energy;
    a.k = make_sweep_args<TW, TU, int32_t>(L).k;
    const dim3 grid((unsigned)L.r.grid), block(256);
    switch (K) {
#define GL_CASE(KK)                                                                 \
    case KK:                                                                        \
        window_part_launch<KK, TW, TU>(L.r, L.vin, s);                              \
        hipLaunchKernelGGL((window_sweep_kernel<KK, TW, TU>), grid, block, 0, s, a); \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TW, typename TU>
static hipError_t window_laplacian_k(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s) {
    typedef typename acc_of<TU>::type A;
    if (!r.wpart) return hipErrorInvalidValue;
    WinLapArgs<TU> a;
    a.op = window_op(r);
    a.part = static_cast<const A*>(r.wpart);
    a.x = static_cast<const TU*>(x);
    a.y = static_cast<TU*>(y);
    a.dd = static_cast<const A*>(r.dd);
    const dim3 grid((unsigned)r.grid), block(256);
    switch (K) {
#define GL_CASE(KK)                                                                     \
    case KK:                                                                            \
        window_part_launch<KK, TW, TU>(r, x, s);                                        \
        hipLaunchKernelGGL((window_laplacian_kernel<KK, TW, TU>), grid, block, 0, s, a); \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static GridOp grid_op(const RowLaunch& r) {
    GridOp op;
    op.w = r.w;
    op.offs = r.goffs;
    op.wbase = r.gwbase;
    op.cnt = r.gcnt;
    op.n = r.n;
    op.dense = r.gdense;
    op.height = r.wheight;
    op.width = r.wwidth;
    op.tiles_x = r.wtiles_x;
    return op;
}

template <typename TW, typename TU>
static hipError_t grid_sweep_k(int K, const SweepLaunch& L, hipStream_t s) {
    typedef typename acc_of<TU>::type A;
    GridSweepArgs<TU, A> a;
    a.op = grid_op(L.r);
    a.ut = static_cast<const TU*>(L.ut);
    a.vin = static_cast<const TU*>(L.vin);
    a.vout = static_cast<TU*>(L.vout);
    a.labels = L.labels;
    a.dd = static_cast<const A*>(L.r.dd);
    a.partials = static_cast<A*>(L.partials);
    a.energy = L.energy;
    a.k = make_sweep_args<TW, TU, int32_t>(L).k;
    const dim3 grid((unsigned)L.r.grid), block(kGridThreads);
    const size_t lds = grid_lds_bytes<TU, A>(K);
    const bool en = L.energy != 0 || L.vout == nullptr;
    switch (K) {
#define GL_CASE(KK)                                                                               \
    case KK:                                                                                      \
        if (en)                                                                                   \
            hipLaunchKernelGGL((grid_energy_sweep_kernel<KK, TW, TU>), grid, block, lds, s, a);  \
        else                                                                                      \
            hipLaunchKernelGGL((grid_sweep_kernel<KK, TW, TU>), grid, block, lds, s, a);         \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Grid-layout sweeps of every weight type for field type TU (compiled in the
// gl_unit_grid_* units, so they build in parallel with the other kernels).
template <typename TU>
static hipError_t grid_sweep_typed(int K, const SweepLaunch& L, hipStream_t s) {
    if constexpr (std::is_same<TU, double>::value) {
        if (L.r.wdt != GL_F64) return hipErrorInvalidValue;
        return grid_sweep_k<double, double>(K, L, s);
    } else {
        switch (L.r.wdt) {
            case GL_F32: return grid_sweep_k<float, TU>(K, L, s);
            case GL_BF16: return grid_sweep_k<bf16, TU>(K, L, s);
            case GL_F16: return grid_sweep_k<f16, TU>(K, L, s);
            default: return hipErrorInvalidValue;
        }
    }
}

template <typename TU>
static hipError_t grid_sweep_extern(int K, const SweepLaunch& L, hipStream_t s) {
    if constexpr (std::is_same<TU, double>::value) return launch_grid_sweep_f64(K, L, s);
    else if constexpr (std::is_same<TU, float>::value) return launch_grid_sweep_f32(K, L, s);
    else if constexpr (std::is_same<TU, bf16>::value) return launch_grid_sweep_bf16(K, L, s);
    else return launch_grid_sweep_f16(K, L, s);
}

template <typename TW, typename TU>
static hipError_t grid_laplacian_k(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s) {
    typedef typename acc_of<TU>::type A;
    GridLapArgs<TU> a;
    a.op = grid_op(r);
    a.x = static_cast<const TU*>(x);
    a.y = static_cast<TU*>(y);
    a.dd = static_cast<const A*>(r.dd);
    const dim3 grid((unsigned)r.grid), block(kGridThreads);
    const size_t lds = grid_lds_bytes<TU, A>(K);
    switch (K) {
#define GL_CASE(KK)                                                                        \
    case KK:                                                                               \
        hipLaunchKernelGGL((grid_laplacian_kernel<KK, TW, TU>), grid, block, lds, s, a);  \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TW, typename TU, typename OffT>
static hipError_t sweep_k(int K, const SweepLaunch& L, hipStream_t s) {
    if (L.r.layout == LAYOUT_GRID) return grid_sweep_extern<TU>(K, L, s);
    if (L.r.layout == LAYOUT_TILE) return tile_sweep_k<TW, TU>(K, L, s);
    if (L.r.layout == LAYOUT_WINDOW) return window_sweep_k<TW, TU>(K, L, s);
    const SweepArgs<TW, TU, OffT> a = make_sweep_args<TW, TU, OffT>(L);
    const dim3 grid((unsigned)sweep_grid(L.r)), block(kBlock);
    switch (K) {
#define GL_CASE(KK)                                                           \
    case KK:                                                                  \
        hipLaunchKernelGGL((sweep_kernel<KK, TW, TU, OffT>), grid, block, 0, s, a); \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename TW, typename TU, typename OffT>
static hipError_t laplacian_k(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s) {
    if (r.layout == LAYOUT_TILE) return tile_laplacian_k<TW, TU>(K, r, x, y, s);
    if (r.layout == LAYOUT_WINDOW) return window_laplacian_k<TW, TU>(K, r, x, y, s);
    if (r.layout == LAYOUT_GRID) return grid_laplacian_k<TW, TU>(K, r, x, y, s);
    LapArgs<TW, TU, OffT> a;
    a.rp = static_cast<const OffT*>(r.rp);
    a.col = r.col;
    a.w = static_cast<const TW*>(r.w);
    a.x = static_cast<const TU*>(x);
    a.y = static_cast<TU*>(y);
    a.order = r.order;
    a.dd = static_cast<const typename acc_of<TU>::type*>(r.dd);
    a.g = RowGeom{r.n, r.rows_per_block, r.G, r.log2G, r.tiles, r.remap};
    const dim3 grid((unsigned)r.grid), block(kBlock);
    switch (K) {
#define GL_CASE(KK)                                                                  \
    case KK:                                                                         \
        hipLaunchKernelGGL((laplacian_kernel<KK, TW, TU, OffT>), grid, block, 0, s, a); \
        break;
        GL_K_CASES(GL_CASE)
#undef GL_CASE
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Weight types paired with a reduced-precision or float field.
template <typename TU>
static hipError_t sweep_lowp(int K, const SweepLaunch& L, hipStream_t s) {
    switch (L.r.wdt) {
        case GL_F32:
            return L.r.idx64 ? sweep_k<float, TU, int64_t>(K, L, s) : sweep_k<float, TU, int32_t>(K, L, s);
        case GL_BF16:
            return L.r.idx64 ? sweep_k<bf16, TU, int64_t>(K, L, s) : sweep_k<bf16, TU, int32_t>(K, L, s);
        case GL_F16:
            return L.r.idx64 ? sweep_k<f16, TU, int64_t>(K, L, s) : sweep_k<f16, TU, int32_t>(K, L, s);
        default:
            return hipErrorInvalidValue;
    }
}

template <typename TU>
static hipError_t laplacian_lowp(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s) {
    switch (r.wdt) {
        case GL_F32:
            return r.idx64 ? laplacian_k<float, TU, int64_t>(K, r, x, y, s)
                           : laplacian_k<float, TU, int32_t>(K, r, x, y, s);
        case GL_BF16:
            return r.idx64 ? laplacian_k<bf16, TU, int64_t>(K, r, x, y, s)
                           : laplacian_k<bf16, TU, int32_t>(K, r, x, y, s);
        case GL_F16:
            return r.idx64 ? laplacian_k<f16, TU, int64_t>(K, r, x, y, s)
                           : laplacian_k<f16, TU, int32_t>(K, r, x, y, s);
        default:
            return hipErrorInvalidValue;
    }
}

}  // namespace gl
