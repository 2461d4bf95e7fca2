// Window layout: the paper's image graph (Section 2.2) with implicit columns.
//
// Pixel i is joined to every pixel j of its (2r+1) x (2r+1) search window
// (the proximity term N_s), j != i.  The neighbour at window offset o = (dy, dx)
// is pixel i + dy * width + dx, so no column index is stored: a sweep streams
// only the weights, one value per (pixel, offset), which is 2 bytes per
// nonzero in BF16/F16 against 6 for a CSR row with 32-bit columns.
//
// Work mapping: a block of 256 lanes owns a 64 x 4 pixel tile, one pixel per
// lane and one image row per wavefront.  The block stages V over the tile and
// its r-wide halo in LDS (zeros outside the image), then every lane walks the
// M = (2r+1)^2 - 1 offsets of its pixel in scan order (row-major over (dy, dx),
// the centre skipped).  Its weights for GS consecutive offsets form one
// 16-byte vector, and the vectors of the block's 256 pixels are contiguous, so
// each wavefront load reads 1 KB in one piece:
//     w[((tile * (M / GS) + g) * 256 + lane) * GS + e]   (offset m = g * GS + e).
// The LDS reads of one wavefront are 64 consecutive words of one halo row,
// free of bank conflicts for every offset.  Offsets whose neighbour falls
// outside the image, and pixels of a ragged tile outside it, store weight 0.
// Each lane sums its row in a fixed order (two interleaved partial sums added
// at the end), so results are bitwise reproducible.
#pragma once

#include "gl_kernels.hpp"

namespace gl {

constexpr int kWinTX = 64;    // tile width: one wavefront per image row
constexpr int kWinTY = 4;     // tile height: four wavefronts
constexpr int kWinMaxR = 27;  // largest window radius (55 x 55 window)
constexpr int kWinMaxRp = 4;  // largest patch radius (9 x 9 patch)
constexpr size_t kWinLdsMax = 147456;  // LDS one block may stage (the device allows 160 KB; room for static LDS)

struct WinOp {
    const void* w;          // weights, layout above
    const int32_t* woff;    // [M] LDS offset dy * S + dx of window offset m
    int32_t height, width;  // image
    int32_t r;              // window radius
    int32_t M;              // offsets per pixel, (2r+1)^2 - 1
    int32_t tiles_x;        // tiles per image row
};

// Z = W V for the pixel of this lane (W: the stored weights, normalized for
// L_s or raw for L); also returns the pixel's own V row from the staged tile.
//   prefetch(ok, p): issue the loads of the pixel's own data
//   finish(ok, p, z, v): consume the product
template <int K, typename TW, typename TU, typename A, typename Pre, typename Fin>
__device__ __forceinline__ void window_products(const WinOp& op, const TU* __restrict__ V, int64_t b, A* hv,
                                                Pre&& prefetch, Fin&& finish) {
    constexpr int GS = 16 / (int)sizeof(TW);
    const int S = kWinTX + 2 * op.r, HY = kWinTY + 2 * op.r, plane = S * HY;
    const int ty = (int)(b / op.tiles_x), tx = (int)(b - (int64_t)ty * op.tiles_x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = tx * kWinTX + lane, y = ty * kWinTY + wave;
    const bool ok = x < op.width && y < op.height;
    const int64_t p = (int64_t)y * op.width + x;
    prefetch(ok, p);

    // stage V over the tile and its halo, kStage cells per lane in flight
    constexpr int kStage = 4;
    const int gx0 = tx * kWinTX - op.r, gy0 = ty * kWinTY - op.r;
    const float invS = 1.0f / (float)S;
    for (int c0 = 0; c0 < plane; c0 += 256 * kStage) {
        A vals[kStage][K];
        int cell[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int c = c0 + u * 256 + (int)threadIdx.x;
            int hy = (int)((float)c * invS);  // exact after the two corrections (c < 2^16)
            hy -= hy * S > c ? 1 : 0;
            hy += (hy + 1) * S <= c ? 1 : 0;
            const int gy = gy0 + hy, gx = gx0 + (c - hy * S);
            cell[u] = c;
            if (c < plane && gy >= 0 && gy < op.height && gx >= 0 && gx < op.width) {
                load_row<K>(V + ((int64_t)gy * op.width + gx) * K, vals[u]);
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) vals[u][k] = (A)0;
            }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            if (cell[u] < plane) {
#pragma unroll
                for (int k = 0; k < K; ++k) hv[k * plane + cell[u]] = vals[u][k];
            }
        }
    }
    __syncthreads();

    const int base = (wave + op.r) * S + lane + op.r;
    const int ng = op.M / GS;
    const u32x4* wp = static_cast<const u32x4*>(op.w) + b * (int64_t)ng * 256 + threadIdx.x;
    A z0[K], z1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) z0[k] = z1[k] = (A)0;
#pragma unroll 4
    for (int g = 0; g < ng; ++g) {
        // streamed once per sweep: a non-temporal load keeps the weights from
        // evicting the V halos that neighbouring tiles re-read from L2
        const u32x4 wq = __builtin_nontemporal_load(wp + (int64_t)g * 256);
        TW we[GS];
        __builtin_memcpy(we, &wq, 16);
#pragma unroll
        for (int e = 0; e < GS; ++e) {
            const int at = base + op.woff[g * GS + e];
            const A wv = cvt<A>(we[e]);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (e & 1) z1[k] += wv * hv[k * plane + at];
                else z0[k] += wv * hv[k * plane + at];
            }
        }
    }
    A z[K], vc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        z[k] = z0[k] + z1[k];
        vc[k] = hv[k * plane + base];
    }
    finish(ok, p, z, vc);
}

template <typename TU, typename A> struct WinSweepArgs {
    WinOp op;
    const TU* ut;
    const TU* vin;
    TU* vout;  // nullptr: energy-only pass
    const int32_t* labels;
    const A* dd;  // d_i of L = D - W, or nullptr for L_s
    A* partials;
    int32_t energy;
    SweepCoef<A> k;
};

// One sweep (or the energy-only pass) on the window layout; the update is the
// one of sweep_block, for all K columns of the lane's pixel.
template <int K, typename TW, typename TU>
__global__ __launch_bounds__(256) void window_sweep_kernel(WinSweepArgs<TU, typename acc_of<TU>::type> a) {
    typedef typename acc_of<TU>::type A;
    extern __shared__ unsigned char smem_raw[];
    A* hv = reinterpret_cast<A*>(smem_raw);
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    int32_t lab = -1;
    A dl = (A)1;
    A uu[K], e_acc[K], r_acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) uu[k] = e_acc[k] = r_acc[k] = (A)0;
    auto prefetch = [&](bool ok, int64_t p) {
        if (!ok) return;
        lab = a.labels[p];
        if (a.dd) dl = a.dd[p];
        load_row<K>(a.ut + p * K, uu);
    };
    auto finish = [&](bool ok, int64_t p, const A (&z)[K], const A (&vc)[K]) {
        if (!ok) return;
        const A lam = lab >= 0 ? (A)1 : (A)0;
        const A ginv = a.dd ? (A)1 / (a.k.ga + a.k.gd * dl + a.k.gl * lam) : (lab >= 0 ? a.k.ginv1 : a.k.ginv0);
        TU vnew[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const A zk = z[k], u = uu[k], v = vc[k];
            const A y = lab < 0 ? (A)0 : (K == 1 ? (lab == 1 ? (A)1 : (A)-1) : (lab == k ? (A)1 : (A)-1));
            const A rhs = a.k.c * u - (u * u * u - u) * a.k.inv_eps + a.k.eta * lam * y;
            const A lv = a.dd ? dl * v - zk : v - zk;
            const A tv = a.k.eps * lv + (a.k.eta * lam + a.k.c) * v;
            const A r = a.k.alpha * (u - v) + a.k.kappa * (rhs - tv);
            vnew[k] = store_as<TU>::from(v + r * ginv);
            r_acc[k] += r * r;
            if (a.energy) {
                const A u2m1 = u * u - (A)1, dy = u - y;
                const A ulu = fma_acc(u, a.dd ? dl * u : u, -(u * zk));  // u (L u)_i, one rounding
                e_acc[k] += a.k.half_eps * ulu + a.k.quarter_inv_eps * u2m1 * u2m1 + a.k.half_eta * lam * dy * dy;
            }
        }
        if (a.vout) store_raw<K>(a.vout + p * K, vnew);
    };
    window_products<K, TW, TU, A>(a.op, a.vin, b, hv, prefetch, finish);
    if (a.partials) block_stats<K, K>(e_acc, r_acc, 1, a.partials, (int64_t)gridDim.x, b);
}

// Y = X - What X (L_s X) or D X - W X (L X) on the window layout
template <typename TU> struct WinLapArgs {
    WinOp op;
    const TU* x;
    TU* y;
    const typename acc_of<TU>::type* dd;
};

template <int K, typename TW, typename TU>
__global__ __launch_bounds__(256) void window_laplacian_kernel(WinLapArgs<TU> a) {
    typedef typename acc_of<TU>::type A;
    extern __shared__ unsigned char smem_raw[];
    A* hv = reinterpret_cast<A*>(smem_raw);
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    A dl = (A)1;
    auto prefetch = [&](bool ok, int64_t p) {
        if (ok && a.dd) dl = a.dd[p];
    };
    auto finish = [&](bool ok, int64_t p, const A (&z)[K], const A (&vc)[K]) {
        if (!ok) return;
#pragma unroll
        for (int k = 0; k < K; ++k) a.y[p * K + k] = store_as<TU>::from((a.dd ? dl * vc[k] : vc[k]) - z[k]);
    };
    window_products<K, TW, TU, A>(a.op, a.x, b, hv, prefetch, finish);
}

// Power-method pass on the window layout (float vectors; see power_kernel).
struct WinPowerArgs {
    WinOp op;
    const float* x;
    float* y;
    const float* scale;
    float* partials;
    const float* dd;
    int32_t mode;
};

template <typename TW>
__global__ __launch_bounds__(256) void window_power_kernel(WinPowerArgs a) {
    extern __shared__ unsigned char smem_raw[];
    float* hv = reinterpret_cast<float*>(smem_raw);
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const float s = a.mode == 0 ? *a.scale : 1.0f;
    float dl = 1.f, p0 = 0.f, p1 = 0.f;
    auto prefetch = [&](bool ok, int64_t p) {
        if (ok && a.dd) dl = a.dd[p];
    };
    auto finish = [&](bool ok, int64_t p, const float (&z)[1], const float (&vc)[1]) {
        if (!ok) return;
        const float xv = vc[0];
        const float lx = (a.dd ? dl * xv : xv) - z[0];
        if (a.mode == 0) {
            const float yv = s * lx;
            a.y[p] = yv;
            p0 += yv * yv;
        } else {
            p0 += xv * lx;
            p1 += xv * xv;
        }
    };
    window_products<1, TW, float, float>(a.op, a.x, b, hv, prefetch, finish);
    float e[1] = {p0}, r[1] = {p1};
    block_stats<1, 1>(e, r, 1, a.partials, (int64_t)gridDim.x, b);
}

}  // namespace gl
