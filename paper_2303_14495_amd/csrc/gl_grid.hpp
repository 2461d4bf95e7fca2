// Grid layout: a sparse graph on the pixels of an image whose edges stay
// within the 15 x 15 search window (Section 2.2), with window-relative
// one-byte columns.
//
// Entry (i, j) stores the byte (dy + 7) << 4 | (dx + 7), where (dy, dx) is
// pixel j's offset from pixel i, and its weight.  A pixel's entries, in CSR
// order, form chunks of 8 (the last one padded with the byte 0x77, the pixel
// itself, and weight 0, so padding needs no branch).  Work mapping: a block of
// 512 lanes owns a 64 x 8 pixel tile, one pixel per lane and one image row per
// wavefront; the block stages V over the tile and its 7-pixel halo in LDS,
// K values per cell side by side (one vector LDS read per entry), zeros
// outside the image.  Chunks are stored so that every wavefront load is
// contiguous.  The first `dense` chunks of every pixel (dense = the smallest
// chunk count of the graph, at most 4) are stored tile by tile, chunk r of lane
// l of tile t at (t * dense + r) * 512 + l, so a lane can request them before it
// knows its chunk count and a workgroup reads them as `dense` contiguous spans
// (long DRAM bursts, as for a plain stream).  The others follow by row
// segment, the segments of a tile one after another: within a wavefront (a
// 64-pixel row segment), chunk c of all lanes that have more than c chunks
// follows chunk c - 1 of all lanes, in lane order; a lane finds its chunk from
// the segment's first chunk, a ballot of the lanes still active and a
// population count.  A sweep thus
// streams 3 bytes per entry in BF16/F16 (1 + 2), plus padding, and no row
// offsets or halo lists.
#pragma once

#include "gl_kernels.hpp"

namespace gl {

constexpr int kGridTX = 64;                       // tile width: one wavefront per image row
constexpr int kGridTY = 8;                        // tile height: eight wavefronts
constexpr int kGridThreads = kGridTX * kGridTY;   // 512
constexpr int kGridR = 7;                         // window radius (15 x 15)
constexpr int kGridS = kGridTX + 2 * kGridR + 2;  // staged row length, 80: image columns 64 tx - 8 .. 64 tx + 71
constexpr int kGridHY = kGridTY + 2 * kGridR;     // staged rows, 22
constexpr int kGridCells = kGridS * kGridHY;      // 1716
constexpr int kGridChunk = 8;                     // entries per chunk
constexpr int kGridGroup = 4;                     // chunks a lane requests at once
constexpr uint8_t kGridPad = 0x77;                // offset byte of the pixel itself
constexpr size_t kGridLdsMax = 147456;  // staged tile per block (the device allows 160 KB; room for static LDS)

struct GridOp {
    const void* w;          // [chunks][8] weights
    const uint64_t* offs;   // [chunks] 8 offset bytes
    const int64_t* wbase;   // [height * tiles_x] first chunk of each wavefront
    const uint8_t* cnt;     // [n] chunks per pixel
    int64_t n;              // pixels
    int32_t dense;          // chunk rounds stored by tile (<= kGridGroup): chunk r of lane l of tile t is (t dense + r) 512 + l
    int32_t height, width, tiles_x;
};

// Fixed-order block reduction of per-lane column statistics for NW wavefronts
// (as block_stats, every lane holding all K columns).  with_e = false: the e
// statistics are known to be zero and are written as such.
template <int K, int NW, typename A>
__device__ __forceinline__ void block_stats_lanes(A (&e)[K], A (&r)[K], A* __restrict__ partials, int64_t nb,
                                                  int64_t b, bool with_e = true) {
    __shared__ A sh[NW][2][K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        r[k] = wave_sum63(r[k]);
        e[k] = with_e ? wave_sum63(e[k]) : (A)0;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            sh[wave][0][k] = e[k];
            sh[wave][1][k] = r[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * K) {
        const int kind = threadIdx.x / K, k = threadIdx.x - kind * K;
        A s = sh[0][kind][k];
#pragma unroll
        for (int w = 1; w < NW; ++w) s += sh[w][kind][k];
        partials[(int64_t)threadIdx.x * nb + b] = s;
    }
}

// Type of the staged field: 16-bit fields are staged as stored (half the LDS
// bytes and traffic of float, converted on read); wider ones in the
// accumulator type.
template <typename TU, typename A> struct grid_lds { typedef A type; };
template <typename A> struct grid_lds<bf16, A> { typedef bf16 type; };
template <typename A> struct grid_lds<f16, A> { typedef f16 type; };

template <typename TU, typename A>
constexpr size_t grid_lds_bytes(int K) { return (size_t)K * kGridCells * sizeof(typename grid_lds<TU, A>::type); }

// LDS byte offsets, from the start of the staged tile, of the 8 entries of a
// chunk (offset bytes ob) for a lane whose window corner is at byte rowb.
// Entry byte x = (dy + 7) * 16 + (dx + 7) sits (dy + 7) * S + (dx + 7) =
// x + (S - 16) * (x >> 4) cells from the corner.  Two entries are decoded at
// once in the 16-bit halves of a register (packed integer arithmetic); this
// needs every offset below 2^16, i.e. a staged tile of at most 64 KB, which
// is the LDS limit the host enforces.  Offsets come out in entry order.
template <int CB>
__device__ __forceinline__ void grid_chunk_offsets(uint64_t ob, uint32_t rowb, uint32_t (&at)[kGridChunk]) {
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    static_assert((size_t)kGridCells * CB <= 65536, "16-bit LDS offsets");
    // the multipliers are hidden from the optimizer so that each pair costs two
    // multiply-adds rather than shifts and adds
    uint32_t cbw = (uint32_t)CB * 0x10001u, rbw = (uint32_t)(CB * (kGridS - 16)) * 0x10001u;
    asm("" : "+s"(cbw));
    asm("" : "+s"(rbw));
    u16x2 cb, cbrow;
    __builtin_memcpy(&cb, &cbw, 4);
    __builtin_memcpy(&cbrow, &rbw, 4);
    const u16x2 base = {(unsigned short)rowb, (unsigned short)rowb};
    const u16x2 four = {4, 4};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t wd = (uint32_t)(ob >> (32 * h));
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            // bytes q and q + 2 of the word, zero-extended into the two halves:
            // entries 4h + q (low half) and 4h + q + 2 (high half)
            const uint32_t pr = __builtin_amdgcn_perm(wd, wd, q == 0 ? 0x0c020c00u : 0x0c030c01u);
            u16x2 x;
            __builtin_memcpy(&x, &pr, 4);
            const u16x2 a = x * cb + ((x >> four) * cbrow + base);
            uint32_t av;
            __builtin_memcpy(&av, &a, 4);
            at[4 * h + q] = av & 0xffffu;
            at[4 * h + q + 2] = av >> 16;
        }
    }
}

// Z = W V for the lane's pixel; the pixel's own V row comes from the staged tile.
//   prefetch(ok, p): issue the loads of the pixel's own data
//   finish(ok, p, z, v): consume the product
template <int K, typename TW, typename TU, typename A, typename Pre, typename Fin>
__device__ __forceinline__ void grid_products(const GridOp& op, const TU* __restrict__ V, int64_t b, void* lds,
                                              Pre&& prefetch, Fin&& finish) {
    typedef typename grid_lds<TU, A>::type L;
    L* hv = static_cast<L*>(lds);
    constexpr int NV = kGridChunk * (int)sizeof(TW) / 16;  // 16-byte vectors per chunk
    const int bi = (int)b;  // tiles < 2^31: 2^31 tiles of 512 pixels would not fit in memory
    const int ty = bi / op.tiles_x, tx = bi - ty * op.tiles_x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = tx * kGridTX + lane, y = ty * kGridTY + wave;
    const bool ok = x < op.width && y < op.height;
    const int64_t p = (int64_t)y * op.width + x;
    const int cnt = ok ? (int)op.cnt[p] : 0;
    const int64_t wb = y < op.height ? op.wbase[(int64_t)y * op.tiles_x + tx] : 0;
    prefetch(ok, p);

    // chunks stream in groups of kGridGroup per lane; the dense rounds of the
    // first group need only the pixel index and are requested at once
    constexpr int U = kGridGroup;
    const u32x4* wv4 = static_cast<const u32x4*>(op.w);
    uint64_t ob[U];
    u32x4 wq[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (u < op.dense && ok) {
            const int64_t id = ((int64_t)bi * op.dense + u) * kGridThreads + (int)threadIdx.x;
            // streamed once per sweep: keep the staged V halos of other tiles in L2
            ob[u] = __builtin_nontemporal_load(op.offs + id);
#pragma unroll
            for (int v = 0; v < NV; ++v) wq[u][v] = __builtin_nontemporal_load(wv4 + id * NV + v);
        }
    }

    // stage V over the tile and its halo, in two halves around the first
    // chunk fetch: lane t < 440 issues the loads of cells t % 20 + 20 u,
    // u = 0..3, of staged row t / 20 at once (before waiting for its chunk
    // count; neighbouring lanes take neighbouring cells), and writes them to
    // LDS afterwards, cells outside the image zeroed.  Loads use
    // 32-bit byte offsets from the first image row of the halo (the host keeps
    // 22 rows of V below 2^32 bytes); a cell outside the image loads that
    // row's first pixel, a valid address.
    constexpr int kSL = kGridS / 4;  // lanes per staged row, 4 cells each
    static_assert(kSL * kGridHY <= kGridThreads && kGridS % 4 == 0, "one staging pass");
    const int gx0 = tx * kGridTX - kGridR - 1, gy0 = ty * kGridTY - kGridR;
    const int gyb = gy0 < 0 ? 0 : gy0;
    const unsigned char* vb = reinterpret_cast<const unsigned char*>(V + (int64_t)gyb * op.width * K);
    const bool stager = (int)threadIdx.x < kSL * kGridHY;
    const int shy = (int)threadIdx.x / kSL, shx = (int)threadIdx.x - shy * kSL;
    const int sgy = gy0 + shy;
    const bool row_in = stager && (unsigned)sgy < (unsigned)op.height;
    // row distance <= 21 and width < 2^24 (host checks): 24-bit multiply
    const uint32_t rowcell = row_in ? __umul24((uint32_t)(sgy - gyb), (uint32_t)op.width) : 0u;
    L vals[4][K];
    bool in[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int gx = gx0 + shx + kSL * u;
        in[u] = row_in && (unsigned)gx < (unsigned)op.width;
        const uint32_t cell = in[u] ? rowcell + (uint32_t)gx : 0u;
        const TU* src = reinterpret_cast<const TU*>(vb + cell * (uint32_t)(K * sizeof(TU)));
        if constexpr (sizeof(L) == sizeof(TU)) {
            load_raw<K>(src, vals[u]);
        } else {
            load_row<K>(src, vals[u]);
        }
    }

    const int maxc = wave_max_nonneg(cnt);
    const int rowbase = wave * kGridS + lane + 1;  // staged cell of window offset (-7, -7)
    constexpr int kCB = K * (int)sizeof(L);    // bytes per staged cell
    // tiles beyond 64 KB (wide fields, e.g. 16 float columns) keep the 32-bit
    // offset decode
    constexpr bool kPacked = (size_t)kGridCells * kCB <= 65536;
    const uint32_t rowb = (uint32_t)rowbase * kCB;
    const unsigned char* hb = static_cast<const unsigned char*>(lds);
    // a row segment's chunks are contiguous: address them by 32-bit byte
    // offsets from the segment's first chunk (at most 64 x 255 chunks)
    const int64_t wbs = ((int64_t)__builtin_amdgcn_readfirstlane((int)(wb >> 32)) << 32) |
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)wb);
    const unsigned char* offs_seg = reinterpret_cast<const unsigned char*>(op.offs + wbs);
    const unsigned char* w_seg = reinterpret_cast<const unsigned char*>(wv4 + wbs * NV);
    uint32_t next = 0;  // chunks of the segment dealt so far
    A z[K];
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = (A)0;
    // the rounds of group c that are stored by segment; their requests wait
    // for the chunk count, and are in flight while the first group's dense
    // rounds are consumed
    auto fetch = [&](int c) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (c + u < op.dense) continue;
            const bool act = c + u < cnt;
            const uint64_t m = __ballot(act);
            // rank of this lane among the active ones (mask bits below it)
            const uint32_t id = next + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            next += (uint32_t)__popcll(m);
            if (act) {
                ob[u] = __builtin_nontemporal_load(reinterpret_cast<const uint64_t*>(offs_seg + id * 8u));
                const u32x4* wp = reinterpret_cast<const u32x4*>(w_seg + id * (uint32_t)(16 * NV));
#pragma unroll
                for (int v = 0; v < NV; ++v) wq[u][v] = __builtin_nontemporal_load(wp + v);
            }
        }
    };
    fetch(0);

    if (stager) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = shy * kGridS + shx + kSL * u;
            if constexpr ((K * sizeof(L)) % 4 == 0) {
                // select whole words: all-zero bits are +0 in every field type
                uint32_t wv[K * sizeof(L) / 4];
                __builtin_memcpy(wv, vals[u], sizeof(wv));
#pragma unroll
                for (int i = 0; i < (int)(K * sizeof(L) / 4); ++i) wv[i] = in[u] ? wv[i] : 0u;
                __builtin_memcpy(&hv[c * K], wv, sizeof(wv));
            } else {
#pragma unroll
                for (int k = 0; k < K; ++k) hv[c * K + k] = in[u] ? vals[u][k] : store_as<L>::from((A)0);
            }
        }
    }
    __syncthreads();

    for (int c = 0; c < maxc; c += U) {
        if (c > 0) fetch(c);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (c + u < cnt) {
                TW we[kGridChunk];
                __builtin_memcpy(we, &wq[u][0], sizeof(we));
                uint32_t at[kGridChunk];
                if constexpr (kPacked) {
                    grid_chunk_offsets<kCB>(ob[u], rowb, at);
                } else {
#pragma unroll
                    for (int e = 0; e < kGridChunk; ++e) {
                        const uint32_t byte = (uint32_t)(ob[u] >> (8 * e)) & 0xffu;
                        at[e] = (uint32_t)(rowbase + (int)(byte >> 4) * kGridS + (int)(byte & 15u)) * kCB;
                    }
                }
#pragma unroll
                for (int e = 0; e < kGridChunk; ++e) {
                    const A w = cvt<A>(we[e]);
                    L hvv[K];
                    constexpr int kAl = kCB % 16 == 0 ? 16 : kCB % 8 == 0 ? 8 : kCB % 4 == 0 ? 4 : 2;
                    __builtin_memcpy(hvv, __builtin_assume_aligned(hb + at[e], kAl), sizeof(hvv));
#pragma unroll
                    for (int k = 0; k < K; ++k) z[k] += w * cvt<A>(hvv[k]);
                }
            }
        }
    }
    const int center = (wave + kGridR) * kGridS + lane + kGridR + 1;
    A vc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) vc[k] = cvt<A>(hv[center * K + k]);
    finish(ok, p, z, vc);
}

template <typename TU, typename A> struct GridSweepArgs {
    GridOp op;
    const TU* ut;
    const TU* vin;
    TU* vout;  // nullptr: energy-only pass
    const int32_t* labels;
    const A* dd;  // d_i of L = D - W, or nullptr for L_s
    A* partials;
    int32_t energy;
    SweepCoef<A> k;
};

// One sweep (or the energy-only pass) on the grid layout; the update is the
// one of sweep_block, for all K columns of the lane's pixel.  EN: the energy
// terms are accumulated (a.energy is ignored); two kernel names below, so the
// sweeps that carry the energy reduction (sweep 0 of every DCA step and the
// energy-only pass) are timed apart from the plain sweeps.
template <int K, typename TW, typename TU, bool EN>
__device__ __forceinline__ void grid_sweep_body(const GridSweepArgs<TU, typename acc_of<TU>::type>& a) {
    typedef typename acc_of<TU>::type A;
    extern __shared__ unsigned char smem_raw[];
    void* hv = smem_raw;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    int32_t lab = -1;
    A dl = (A)1;
    A e_acc[K], r_acc[K];
    // u^t as stored: converted at the update, so that its load does not hold
    // back the chunk requests issued after it
    TU ur[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        e_acc[k] = r_acc[k] = (A)0;
        ur[k] = store_as<TU>::from((A)0);
    }
    auto prefetch = [&](bool ok, int64_t p) {
        if (!ok) return;
        lab = a.labels[p];
        if (a.dd) dl = a.dd[p];
        load_raw<K>(a.ut + p * K, ur);
    };
    auto finish = [&](bool ok, int64_t p, const A (&z)[K], const A (&vc)[K]) {
        if (!ok) return;
        const A lam = lab >= 0 ? (A)1 : (A)0;
        const A ginv = a.dd ? (A)1 / (a.k.ga + a.k.gd * dl + a.k.gl * lam) : (lab >= 0 ? a.k.ginv1 : a.k.ginv0);
        TU vnew[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const A zk = z[k], u = cvt<A>(ur[k]), v = vc[k];
            const A y = lab < 0 ? (A)0 : (K == 1 ? (lab == 1 ? (A)1 : (A)-1) : (lab == k ? (A)1 : (A)-1));
            const A rhs = a.k.c * u - (u * u * u - u) * a.k.inv_eps + a.k.eta * lam * y;
            const A lv = a.dd ? dl * v - zk : v - zk;
            const A tv = a.k.eps * lv + (a.k.eta * lam + a.k.c) * v;
            const A r = a.k.alpha * (u - v) + a.k.kappa * (rhs - tv);
            vnew[k] = store_as<TU>::from(v + r * ginv);
            r_acc[k] += r * r;
            if constexpr (EN) {
                const A u2m1 = u * u - (A)1, dy = u - y;
                const A ulu = fma_acc(u, a.dd ? dl * u : u, -(u * zk));  // u (L u)_i, one rounding
                e_acc[k] += a.k.half_eps * ulu + a.k.quarter_inv_eps * u2m1 * u2m1 + a.k.half_eta * lam * dy * dy;
            }
        }
        if (!EN || a.vout) store_raw<K>(a.vout + p * K, vnew);
    };
    grid_products<K, TW, TU, A>(a.op, a.vin, b, hv, prefetch, finish);
    if (a.partials) block_stats_lanes<K, kGridTY>(e_acc, r_acc, a.partials, (int64_t)gridDim.x, b, EN);
}

// A plain sweep: no energy terms, always stores the new field.
template <int K, typename TW, typename TU>
__global__ __launch_bounds__(kGridThreads) void grid_sweep_kernel(GridSweepArgs<TU, typename acc_of<TU>::type> a) {
    grid_sweep_body<K, TW, TU, false>(a);
}

// Sweep 0 of a DCA step with the energy terms of u^t, or (vout == nullptr) the
// energy-only pass after the last step.
template <int K, typename TW, typename TU>
__global__ __launch_bounds__(kGridThreads) void grid_energy_sweep_kernel(GridSweepArgs<TU, typename acc_of<TU>::type> a) {
    grid_sweep_body<K, TW, TU, true>(a);
}

// Y = X - What X (L_s X) or D X - W X (L X) on the grid layout
template <typename TU> struct GridLapArgs {
    GridOp op;
    const TU* x;
    TU* y;
    const typename acc_of<TU>::type* dd;
};

template <int K, typename TW, typename TU>
__global__ __launch_bounds__(kGridThreads) void grid_laplacian_kernel(GridLapArgs<TU> a) {
    typedef typename acc_of<TU>::type A;
    extern __shared__ unsigned char smem_raw[];
    void* hv = smem_raw;
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
    grid_products<K, TW, TU, A>(a.op, a.x, b, hv, prefetch, finish);
}

// Power-method pass on the grid layout (float vectors; see power_kernel).
struct GridPowerArgs {
    GridOp op;
    const float* x;
    float* y;
    const float* scale;
    float* partials;
    const float* dd;
    int32_t mode;
};

template <typename TW>
__global__ __launch_bounds__(kGridThreads) void grid_power_kernel(GridPowerArgs a) {
    extern __shared__ unsigned char smem_raw[];
    void* hv = smem_raw;
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
    grid_products<1, TW, float, float>(a.op, a.x, b, hv, prefetch, finish);
    float e[1] = {p0}, r[1] = {p1};
    block_stats_lanes<1, kGridTY>(e, r, a.partials, (int64_t)gridDim.x, b);
}

// Unnormalized L on the grid layout: dd_i = sum over row i of the weights as
// stored (rounded to TW), in CSR order (the storage order), summed in double.
template <typename TIN, typename TW, typename A>
__global__ void grid_rowsum_kernel(int64_t n, const int64_t* __restrict__ rp, const TIN* __restrict__ w,
                                   A* __restrict__ dd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) s += cvt<double>(store_as<TW>::from((double)w[e]));
    dd[i] = (A)s;
}

}  // namespace gl
