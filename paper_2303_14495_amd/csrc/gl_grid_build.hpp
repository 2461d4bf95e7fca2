// Construction of the grid layout on the device (see gl_grid.hpp for the
// layout and the sweep that reads it), from the validated CSR graph and its
// degrees:
//   grid_count_kernel    chunks per pixel (its entries in chunks of 8), the
//                        window check of every edge, the smallest count;
//   grid_segrest_kernel  per row segment, its chunks beyond the dense rounds;
//   (exclusive scan of those counts over the segments in tile order)
//   grid_emit_kernel     one wavefront per row segment writes the offset bytes
//                        and the normalized weights of every chunk, the dense
//                        rounds at (t * dense + r) * 512 + l and the rest after
//                        the segment's scanned offset, ranked by the same
//                        ballot the sweep uses to find them.
#pragma once

#include "gl_grid.hpp"

namespace gl {

// Chunks per pixel; flags |= 1 (first bad pixel in *first) for an edge more
// than 7 rows or columns away; *mincnt = the smallest chunk count.
static __global__ void grid_count_kernel(int64_t n, int32_t width, const int64_t* __restrict__ rp,
                                         const int32_t* __restrict__ col, uint8_t* __restrict__ cnt,
                                         int32_t* flags, unsigned long long* first, int32_t* mincnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // n < 2^31 and width < 2^24: 32-bit arithmetic
    const int32_t yi = (int32_t)i / width, xi = (int32_t)i - yi * width;
    const int64_t beg = rp[i], end = rp[i + 1];
    bool bad = false;
    for (int64_t e = beg; e < end; ++e) {
        const int32_t j = col[e], yj = j / width, xj = j - yj * width;
        if (yj - yi < -kGridR || yj - yi > kGridR || xj - xi < -kGridR || xj - xi > kGridR) bad = true;
    }
    if (bad) {
        atomicOr(flags, 1);
        atomicMin(first, (unsigned long long)i);
    }
    // at most 224 distinct window cells (columns are strictly increasing)
    const int c = (int)((end - beg + kGridChunk - 1) / kGridChunk);
    cnt[i] = (uint8_t)(c < 255 ? c : 255);
    atomicMin(mincnt, c);
}

// Row segment s (tile-major: s = tile * 8 + row in tile): its chunks beyond
// the first `dense` rounds.
static __global__ void grid_segrest_kernel(int64_t nseg, int32_t height, int32_t width, int32_t tiles_x,
                                           const uint8_t* __restrict__ cnt, int32_t dense,
                                           int64_t* __restrict__ seg_rest) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int64_t t = s / kGridTY;
    const int32_t ty = (int32_t)(t / tiles_x), tx = (int32_t)(t - (int64_t)ty * tiles_x);
    const int32_t y = ty * kGridTY + (int32_t)(s - t * kGridTY);
    int64_t r = 0;
    if (y < height) {
        const int32_t x1 = min(width, tx * kGridTX + kGridTX);
        for (int32_t x = tx * kGridTX; x < x1; ++x) {
            const int c = cnt[(int64_t)y * width + x];
            r += c > dense ? c - dense : 0;
        }
    }
    seg_rest[s] = r;
}

// One wavefront per row segment (4 per workgroup of 256 lanes): lane = column
// in the segment.  Chunk c of the lane's pixel holds its CSR entries 8c ..
// 8c + 7: offset byte (dy + 7) << 4 | (dx + 7) and weight w_ij / (sqrt(d_i)
// sqrt(d_j)) (w_ij itself when raw), rounded once to TOUT; missing entries are
// the padding byte 0x77 (the pixel itself) with weight 0.
template <typename TIN, typename TOUT>
__global__ __launch_bounds__(256) void grid_emit_kernel(int64_t nseg, int32_t height, int32_t width, int32_t tiles_x,
                                                        int32_t dense, const int64_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col, const TIN* __restrict__ w,
                                                        const double* __restrict__ d, int32_t raw,
                                                        const uint8_t* __restrict__ cnt,
                                                        const int64_t* __restrict__ seg_off, int64_t rest_base,
                                                        uint64_t* __restrict__ offs, TOUT* __restrict__ w_out,
                                                        int64_t* __restrict__ wbase) {
    const int64_t s = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (s >= nseg) return;  // uniform per wavefront
    const int lane = threadIdx.x & 63;
    const int64_t t = s / kGridTY;
    const int32_t row = (int32_t)(s - t * kGridTY);
    const int32_t ty = (int32_t)(t / tiles_x), tx = (int32_t)(t - (int64_t)ty * tiles_x);
    const int32_t y = ty * kGridTY + row, x = tx * kGridTX + lane;
    const bool ok = y < height && x < width;
    const int64_t p = ok ? (int64_t)y * width + x : 0;
    const int c_have = ok ? (int)cnt[p] : 0;
    const int64_t beg = ok ? rp[p] : 0, end = ok ? rp[p + 1] : 0;
    const double dp = ok && !raw ? sqrt(d[p]) : 1.0;

    auto write_chunk = [&](int64_t id, int c) {
        uint64_t ob = 0;
        TOUT wv[kGridChunk];
#pragma unroll
        for (int e = 0; e < kGridChunk; ++e) {
            const int64_t k = beg + (int64_t)c * kGridChunk + e;
            uint64_t byte = kGridPad;
            double val = 0.0;
            if (k < end) {
                const int32_t j = col[k], yj = j / width, xj = j - yj * width;
                byte = (uint64_t)(((yj - y + kGridR) << 4) | (xj - x + kGridR));
                const double wk = (double)w[k];
                val = raw ? wk : wk / (dp * sqrt(d[j]));
            }
            ob |= byte << (8 * e);
            wv[e] = store_as<TOUT>::from(val);
        }
        offs[id] = ob;
#pragma unroll
        for (int e = 0; e < kGridChunk; ++e) w_out[id * kGridChunk + e] = wv[e];
    };

    // dense rounds, by tile; slots of pixels outside the image are padding
    for (int r = 0; r < dense; ++r) write_chunk((t * dense + r) * kGridThreads + row * kGridTX + lane, r);
    // the rest of the segment, round by round in lane order
    const int64_t base = rest_base + seg_off[s];
    if (lane == 0 && y < height) wbase[(int64_t)y * tiles_x + tx] = base;
    const int maxc = wave_max_nonneg(c_have);
    int64_t next = 0;
    for (int c = dense; c < maxc; ++c) {
        const bool act = c < c_have;
        const uint64_t m = __ballot(act);
        const int64_t id = base + next +
                           __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        next += __popcll(m);
        if (act) write_chunk(id, c);
    }
}

// Exclusive prefix sums of n values by one workgroup of 1024 lanes: lane l
// sums its contiguous range, the 1024 range sums are scanned in LDS, then each
// lane writes its range's prefixes; *total = the sum of all.
static __global__ __launch_bounds__(1024) void scan_exclusive_kernel(const int64_t* __restrict__ in,
                                                                     int64_t* __restrict__ out, int64_t n,
                                                                     int64_t* total) {
    __shared__ int64_t sh[1024];
    const int l = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b0 = min(n, (int64_t)l * per), b1 = min(n, b0 + per);
    int64_t acc = 0;
    for (int64_t i = b0; i < b1; ++i) acc += in[i];
    sh[l] = acc;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = l >= off ? sh[l - off] : 0;
        __syncthreads();
        sh[l] += v;
        __syncthreads();
    }
    int64_t run = sh[l] - acc;  // exclusive prefix of this lane's range
    for (int64_t i = b0; i < b1; ++i) {
        const int64_t v = in[i];
        out[i] = run;
        run += v;
    }
    if (l == 1023) *total = sh[1023];
}

}  // namespace gl
