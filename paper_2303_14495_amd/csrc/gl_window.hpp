// Window layout: the paper's image graph (Section 2.2) with implicit columns.
//
// Pixel i is joined to every pixel j of its (2r+1) x (2r+1) search window
// (the proximity term N_s), j != i.  The neighbour at window offset o = (dy, dx)
// is pixel i + dy * width + dx, so no column index is stored.  W is symmetric,
// and each pair is stored once: pixel i keeps the weights of the first half of
// its window in scan order (row-major over (dy, dx)), the Mh = M / 2 offsets
// with dy < 0, or dy = 0 and dx < 0 (M = (2r+1)^2 - 1); the weight of (i, j)
// for an offset of the second half is the one j keeps for the offset -o.  A
// sweep streams Mh weights per pixel, 1 byte per nonzero in BF16/F16 against
// 6 for a CSR row with 32-bit columns.
//
// Work mapping: a block of 256 lanes owns a 64 x 4 pixel tile, one pixel per
// lane and one image row per wavefront, and a region of (4 + r) x (64 + 2r)
// cells: the tile, the r image rows above it and r columns on each side.  The
// block stages V over the region in LDS (zeros outside the image), then every
// lane walks the Mh stored offsets of its pixel in scan order.  For the stored
// weight w of (i, i + o) it adds w V[i + o] to its own sum (a register) and
// w V[i] to the cell of i + o (an LDS accumulator over the region), so each
// weight is read once and used in both directions.  The offsets of one window
// row (one dy) form a phase, and the block synchronises between phases: the
// four wavefronts then add into four different image rows, and every cell
// receives its contributions in a fixed order.  The block writes the region
// (its own pixels' sums included) to a partial buffer, and the consumer kernel
// sums, for each pixel, the regions of the tiles that cover it, in a fixed
// order: (W V)_i is bitwise reproducible.
//
// Stored weights: GS = 16 / sizeof(weight) consecutive offsets of one pixel
// form one 16-byte vector, and the vectors of a tile's 256 pixels are
// contiguous, so each wavefront load reads 1 KB in one piece:
//     w[((tile * NG + g) * 256 + lane) * GS + e]   (offset m = g * GS + e < Mh),
// NG = ceil(Mh / GS), padding zero.  Offsets whose neighbour falls outside the
// image, and pixels of a ragged tile outside it, store weight 0.
#pragma once

#include <type_traits>

#include "gl_kernels.hpp"

namespace gl {

constexpr int kWinTX = 64;    // tile width: one wavefront per image row
constexpr int kWinTY = 4;     // tile height: four wavefronts
constexpr int kWinMaxR = 27;  // largest window radius (55 x 55 window)
constexpr int kWinMaxRp = 4;  // largest patch radius (9 x 9 patch)
constexpr size_t kWinLdsMax = 147456;  // LDS one block may stage (the device allows 160 KB; room for static LDS)

struct WinOp {
    const void* w;          // stored weights, layout above
    int32_t height, width;  // image
    int32_t r;              // window radius
    int32_t M;              // offsets per pixel, (2r+1)^2 - 1
    int32_t tiles_x;        // tiles per image row
};

// Cells of one tile's region: (4 + r) rows of 64 + 2r.
__host__ __device__ __forceinline__ int window_region(int r) { return (kWinTY + r) * (kWinTX + 2 * r); }

// Stored vectors per pixel for GS offsets per vector.
__host__ __device__ __forceinline__ int window_groups(int M, int GS) { return (M / 2 + GS - 1) / GS; }

template <typename TU> struct WinPartArgs {
    WinOp op;
    const TU* v;                          // V, n x K
    typename acc_of<TU>::type* part;      // [tile][region cell][K]
};

// First pass of every window product: the region sums of one tile (above).
template <int K, typename TW, typename TU>
__global__ __launch_bounds__(256) void window_part_kernel(WinPartArgs<TU> a) {
    typedef typename acc_of<TU>::type A;
    // V at the cell and the contributions added to it, read by one 64-bit LDS
    // load (two 32-bit loads 8 bytes apart conflict on half the banks)
    struct alignas(2 * sizeof(A)) A2 {
        A v, s;
    };
    constexpr int GS = 16 / (int)sizeof(TW);
    extern __shared__ unsigned char smem_raw[];
    const WinOp& op = a.op;
    const int S = kWinTX + 2 * op.r, plane = window_region(op.r);
    A2* hl = reinterpret_cast<A2*>(smem_raw);  // [cell][k]: one read returns both halves
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int ty = (int)(b / op.tiles_x), tx = (int)(b - (int64_t)ty * op.tiles_x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // stage V over the region, kStage cells per lane in flight; clear the sums
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
                load_row<K>(a.v + ((int64_t)gy * op.width + gx) * K, vals[u]);
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) vals[u][k] = (A)0;
            }
        }
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            if (cell[u] < plane) {
#pragma unroll
                for (int k = 0; k < K; ++k) hl[cell[u] * K + k] = A2{vals[u][k], (A)0};
            }
        }
    }
    __syncthreads();

    const int base = (wave + op.r) * S + lane + op.r;  // the lane's own cell
    A vp[K];
#pragma unroll
    for (int k = 0; k < K; ++k) vp[k] = hl[base * K + k].v;
    const int ng = window_groups(op.M, GS), mh = op.M / 2, side = 2 * op.r + 1;
    const u32x4* wp = static_cast<const u32x4*>(op.w) + b * (int64_t)ng * 256 + threadIdx.x;
    A z0[K], z1[K];
#pragma unroll
    for (int k = 0; k < K; ++k) z0[k] = z1[k] = (A)0;
    // offset m of the first half: window row `row` and column `col` (dy = row - r,
    // dx = col - r), the cell vbase + rc with rc = row * S + col
    A2* const vb = hl + (wave * S + lane) * K;
    int m = 0, rc = 0, col = 0;
    auto ld = [&](int g) { return __builtin_nontemporal_load(wp + (int64_t)(g < ng ? g : ng - 1) * 256); };
    // MASK: the vector may hold padding (offsets m >= mh: weight 0, added at the own cell)
    auto step = [&](const u32x4& wq, auto mask) {
        TW we[GS];
        __builtin_memcpy(we, &wq, 16);
#pragma unroll
        for (int e = 0; e < GS; ++e) {
            const bool live = !decltype(mask)::value || m < mh;
            A2* const c = live ? vb + rc * K : hl + base * K;
            const A wv = live ? cvt<A>(we[e]) : (A)0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const A2 t = c[k];
                if (e & 1) z1[k] += wv * t.v;
                else z0[k] += wv * t.v;
                c[k].s = t.s + wv * vp[k];
                // keep the own sum's FMA here: left to the scheduler, the FMAs of
                // a whole vector wait at its end, and their operands held in
                // registers cost three of the eight wavefronts a SIMD can hold
                if (e & 1) asm volatile("" : "+v"(z1[k]));
                else asm volatile("" : "+v"(z0[k]));
            }
            ++m;
            ++rc;
            if (++col == side) {  // end of a phase: one window row done by all four wavefronts
                col = 0;
                rc += S - side;
                __syncthreads();
            }
        }
    };
    typedef std::integral_constant<bool, false> Full;
    typedef std::integral_constant<bool, true> Masked;
    u32x4 w0 = ld(0), w1 = ld(1), w2 = ld(2), w3 = ld(3);
    int g = 0;
    for (const int gq = (ng - 1) & ~3; g < gq; g += 4) {  // vectors without padding, four at a time
        step(w0, Full());
        w0 = ld(g + 4);
        step(w1, Full());
        w1 = ld(g + 5);
        step(w2, Full());
        w2 = ld(g + 6);
        step(w3, Full());
        w3 = ld(g + 7);
    }
    // the last one to four vectors, already loaded
    step(w0, Masked());
    if (g + 1 < ng) step(w1, Masked());
    if (g + 2 < ng) step(w2, Masked());
    if (g + 3 < ng) step(w3, Masked());
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) hl[base * K + k].s += z0[k] + z1[k];
    __syncthreads();
    A* out = a.part + b * (int64_t)plane * K;
    for (int i = threadIdx.x; i < plane * K; i += 256) out[i] = hl[i].s;
}

// (W V) at pixel (y, x): the sum of the regions of the tiles that cover it
// (tile rows from the pixel's own down, columns left to right).
template <int K, typename A>
__device__ __forceinline__ void window_gather(const WinOp& op, const A* __restrict__ part, int y, int x, A (&z)[K]) {
    // a pixel lies in the regions of its own tile, of the tiles below it whose
    // r rows above reach it, and of at most one horizontal neighbour of each
    // (the left one when x mod 64 < r, the right one when x mod 64 >= 64 - r)
    static_assert(2 * kWinMaxR < kWinTX, "one horizontal neighbour at most");
    constexpr int NT = (kWinMaxR + 2 * kWinTY - 1) / kWinTY;  // tile rows that can cover a pixel
    constexpr int B = K <= 4 ? 4 : (K <= 8 ? 2 : 1);           // tile rows requested at once
    const int S = kWinTX + 2 * op.r, plane = window_region(op.r);
    const int tiles_y = (op.height + kWinTY - 1) / kWinTY;
    const int ty = y / kWinTY, tx = x / kWinTX, xl = x - tx * kWinTX;
    const int ty1 = min(tiles_y - 1, (y + op.r) / kWinTY);
    const bool left = xl < op.r && tx > 0, right = xl >= kWinTX - op.r && tx + 1 < op.tiles_x;
    const int ts = left ? tx - 1 : tx + 1;                        // the horizontal neighbour, if any
    const int rxo = xl + op.r, rxs = left ? xl + kWinTX + op.r : xl - kWinTX + op.r;
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = (A)0;
    for (int t0 = 0; t0 < NT; t0 += B) {
        // every request of the batch is issued before any is added; rows past
        // the last covering one read the pixel's own cell and are not added
        A own[B][K], side[B][K];
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int t2 = ty + t0 + i;
            const bool v = t2 <= ty1;
            const int tr = v ? t2 : ty;
            const int ry = y - (tr * kWinTY - op.r);
            const int64_t rb = (int64_t)tr * op.tiles_x;
            load_raw<K>(part + ((rb + tx) * plane + ry * S + rxo) * K, own[i]);
            const bool vs = v && (left || right);
            load_raw<K>(part + ((vs ? rb + ts : rb + tx) * plane + ry * S + (vs ? rxs : rxo)) * K, side[i]);
        }
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const bool v = ty + t0 + i <= ty1;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                A t = z[k];
                t = v && left ? t + side[i][k] : t;
                t = v ? t + own[i][k] : t;
                t = v && right ? t + side[i][k] : t;
                z[k] = t;
            }
        }
        if (ty + t0 + B > ty1) break;
    }
}

// The pixel of this lane in the second pass (same tiles and block order as the first).
struct WinPixel {
    int64_t b, p;
    int y, x;
    bool ok;
};

__device__ __forceinline__ WinPixel window_pixel(const WinOp& op) {
    WinPixel q;
    q.b = xcd_remap(blockIdx.x, gridDim.x);
    const int ty = (int)(q.b / op.tiles_x), tx = (int)(q.b - (int64_t)ty * op.tiles_x);
    q.x = tx * kWinTX + (int)(threadIdx.x & 63);
    q.y = ty * kWinTY + (int)(threadIdx.x >> 6);
    q.ok = q.x < op.width && q.y < op.height;
    q.p = (int64_t)q.y * op.width + q.x;
    return q;
}

template <typename TU, typename A> struct WinSweepArgs {
    WinOp op;
    const A* part;  // region sums of W vin (window_part_kernel)
    const TU* ut;
    const TU* vin;
    TU* vout;  // nullptr: energy-only pass
    const int32_t* labels;
    const A* dd;  // d_i of L = D - W, or nullptr for L_s
    A* partials;
    int32_t energy;
    SweepCoef<A> k;
};

// One sweep (or the energy-only pass) on the window layout, after
// window_part_kernel over vin; the update is the one of sweep_block, for all K
// columns of the lane's pixel.
template <int K, typename TW, typename TU>
__global__ __launch_bounds__(256) void window_sweep_kernel(WinSweepArgs<TU, typename acc_of<TU>::type> a) {
    typedef typename acc_of<TU>::type A;
    const WinPixel q = window_pixel(a.op);
    A e_acc[K], r_acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) e_acc[k] = r_acc[k] = (A)0;
    if (q.ok) {
        const int64_t p = q.p;
        const int32_t lab = a.labels[p];
        const A dl = a.dd ? a.dd[p] : (A)1;
        A uu[K], vc[K], z[K];
        load_row<K>(a.ut + p * K, uu);
        load_row<K>(a.vin + p * K, vc);
        window_gather<K, A>(a.op, a.part, q.y, q.x, z);
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
    }
    if (a.partials) block_stats<K, K>(e_acc, r_acc, 1, a.partials, (int64_t)gridDim.x, q.b);
}

// Y = X - What X (L_s X) or D X - W X (L X) on the window layout, after
// window_part_kernel over X.
template <typename TU> struct WinLapArgs {
    WinOp op;
    const typename acc_of<TU>::type* part;
    const TU* x;
    TU* y;
    const typename acc_of<TU>::type* dd;
};

template <int K, typename TW, typename TU>
__global__ __launch_bounds__(256) void window_laplacian_kernel(WinLapArgs<TU> a) {
    typedef typename acc_of<TU>::type A;
    const WinPixel q = window_pixel(a.op);
    if (!q.ok) return;
    const A dl = a.dd ? a.dd[q.p] : (A)1;
    A vc[K], z[K];
    load_row<K>(a.x + q.p * K, vc);
    window_gather<K, A>(a.op, a.part, q.y, q.x, z);
#pragma unroll
    for (int k = 0; k < K; ++k) a.y[q.p * K + k] = store_as<TU>::from((a.dd ? dl * vc[k] : vc[k]) - z[k]);
}

// Power-method pass on the window layout (float vectors; see power_kernel),
// after window_part_kernel over x.
struct WinPowerArgs {
    WinOp op;
    const float* part;
    const float* x;
    float* y;
    const float* scale;
    float* partials;
    const float* dd;
    int32_t mode;
};

template <typename TW>
__global__ __launch_bounds__(256) void window_power_kernel(WinPowerArgs a) {
    const WinPixel q = window_pixel(a.op);
    const float s = a.mode == 0 ? *a.scale : 1.0f;
    float p0 = 0.f, p1 = 0.f;
    if (q.ok) {
        const float dl = a.dd ? a.dd[q.p] : 1.f;
        const float xv = a.x[q.p];
        float z[1];
        window_gather<1, float>(a.op, a.part, q.y, q.x, z);
        const float lx = (a.dd ? dl * xv : xv) - z[0];
        if (a.mode == 0) {
            const float yv = s * lx;
            a.y[q.p] = yv;
            p0 += yv * yv;
        } else {
            p0 += xv * lx;
            p1 += xv * xv;
        }
    }
    float e[1] = {p0}, r[1] = {p1};
    block_stats<1, 1>(e, r, 1, a.partials, (int64_t)gridDim.x, q.b);
}

}  // namespace gl
