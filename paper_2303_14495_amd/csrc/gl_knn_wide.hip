// k nearest neighbours for wide features (64 < d <= 4096), with the same
// result as the exact kernel: the k smallest f32 distances
// sum_c (q_c - p_c)^2 (FMA, coordinate order), ties to the lower index.
//
// The n^2 d work is a Gram matrix, so it runs on the matrix cores: the points
// are centred, scaled by a power of two and rounded to f16, and one fused
// kernel multiplies a block of 128 queries by blocks of 128 points with
// v_mfma_f32_32x32x16_f16 (f32 accumulation), staging both operand tiles
// through LDS, and turns every block of products straight into approximate
// distances |q|^2 + |p|^2 - 2 <q, p> that it filters into per-query candidate
// lists; no product leaves the chip.  A query's points are dealt to four
// lists (two halves of every point block, two workgroups each sweeping half
// of the point blocks), each keeping its 16 smallest approximate distances,
// so 64 candidates per query, and nu = the smallest approximate distance any
// list had to drop or reject: every point outside the candidates is at least
// nu away, approximately.  A second kernel recomputes the candidates' exact
// f32 distances, keeps the k best, and checks a certificate: the
// approximation error is at most E_q (a bound from the f16 rounding, the f32
// accumulation and the norms), so if nu - E_q exceeds the exact k-th distance
// no other point can enter or tie.  Rows without the certificate are
// recomputed by an exact scan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gl_internal.hpp"

namespace {


gl_status wfail(gl_status st, const std::string& m) {
    gl::set_last_error(m);
    return st;
}

// Column means, so the approximate distances are formed from centred points,
// whose smaller norms shrink the error bound: double partial sums over the
// rows r = slice, slice + kMeanSlices, ... (one block row per slice), then the
// slices added in order.
constexpr int kMeanSlices = 256;

__global__ void kw_mean_partial_kernel(const float* __restrict__ x, int64_t n, int32_t d,
                                       double* __restrict__ part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d) return;
    double s = 0.0;
    for (int64_t i = blockIdx.y; i < n; i += kMeanSlices) s += (double)x[i * d + c];
    part[(int64_t)blockIdx.y * d + c] = s;
}

__global__ void kw_mean_final_kernel(const double* __restrict__ part, int64_t n, int32_t d,
                                     float* __restrict__ mu) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d) return;
    double s = 0.0;
    for (int r = 0; r < kMeanSlices; ++r) s += part[(int64_t)r * d + c];
    mu[c] = (float)(s / (double)n);
}

// |x_i - mu|^2 (f32, fixed-order wave reduction), and max |x_ic - mu_c| over
// all points as the bits of a non-negative float (monotone as unsigned).
__global__ __launch_bounds__(256) void kw_norms_kernel(const float* __restrict__ x, const float* __restrict__ mu,
                                                      int64_t n, int32_t d, float* __restrict__ norm2,
                                                      unsigned int* amax) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (i >= n) return;
    float s = 0.f, m = 0.f;
    for (int c = lane; c < d; c += 64) {
        const float v = x[i * d + c] - mu[c];
        s = fmaf(v, v, s);
        m = fmaxf(m, fabsf(v));
    }
    for (int off = 32; off > 0; off >>= 1) {
        s += __shfl_xor(s, off, 64);
        m = fmaxf(m, __shfl_xor(m, off, 64));
    }
    if (lane == 0) {
        norm2[i] = s;
        atomicMax(amax, __float_as_uint(m));
    }
}

// xh[i][c] = f16(scale * (x[i][c] - mu[c])), zero padded to dp columns.
__global__ void kw_half_kernel(const float* __restrict__ x, const float* __restrict__ mu, int64_t n, int32_t d,
                               int32_t dp, float scale, _Float16* __restrict__ xh) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * dp) return;
    const int64_t i = e / dp;
    const int c = (int)(e - i * dp);
    xh[e] = c < d ? (_Float16)(scale * (x[i * d + c] - mu[c])) : (_Float16)0.0f;
}

// Insert (v, j) into an ascending list of T entries (ties by index); returns
// the entry pushed out at the end.
template <int T>
__device__ __forceinline__ void kw_insert(float (&bv)[T], int32_t (&bj)[T], float v, int32_t j, float& out_v) {
    out_v = bv[T - 1];
#pragma unroll
    for (int t = T - 1; t > 0; --t) {
        const bool mv = v < bv[t - 1] || (v == bv[t - 1] && j < bj[t - 1]);
        const bool here = !mv && (v < bv[t] || (v == bv[t] && j < bj[t]));
        if (mv) {
            bv[t] = bv[t - 1];
            bj[t] = bj[t - 1];
        } else if (here) {
            bv[t] = v;
            bj[t] = j;
        }
    }
    if (v < bv[0] || (v == bv[0] && j < bj[0])) {
        bv[0] = v;
        bj[0] = j;
    }
}

// Pop the wave-wide smallest (v, j) head among the lanes' ascending lists;
// every lane receives it, and the owning lane advances its list.
template <int T>
__device__ __forceinline__ void kw_pop_min(float (&bv)[T], int32_t (&bj)[T], float& v, int32_t& j) {
    float hv = bv[0];
    int32_t hj = bj[0];
    for (int off = 32; off > 0; off >>= 1) {
        const float ov = __shfl_xor(hv, off, 64);
        const int32_t oj = __shfl_xor(hj, off, 64);
        if (ov < hv || (ov == hv && oj < hj)) {
            hv = ov;
            hj = oj;
        }
    }
    v = hv;
    j = hj;
    if (bj[0] == hj && bv[0] == hv && hj >= 0) {
#pragma unroll
        for (int t = 0; t < T - 1; ++t) {
            bv[t] = bv[t + 1];
            bj[t] = bj[t + 1];
        }
        bv[T - 1] = INFINITY;
        bj[T - 1] = INT32_MAX;
    }
}

typedef _Float16 kw_h8 __attribute__((ext_vector_type(8)));
typedef float kw_f16v __attribute__((ext_vector_type(16)));
typedef uint32_t kw_u4 __attribute__((ext_vector_type(4)));

constexpr int kFQ = 128;           // queries per workgroup
constexpr int kFP = 128;           // points per block
constexpr int kFK = 64;            // coordinates per staging step (four MFMA k-steps of 16)
constexpr int kFPitch = kFK + 8;   // f16 per staged row: 144-byte rows, conflict-free 16-byte reads
constexpr int kFThreads = 512;     // 8 wavefronts: 4 query quarters x 2 point halves
constexpr int kFKc = 64;           // candidates per query: 2 H SEG lists of T = 32 / (H SEG)
constexpr int kFRow = 68;          // floats per row of a wavefront's distance block (64 + 4)
constexpr size_t kFStageBytes = (size_t)2 * 2 * kFQ * kFPitch * 2;      // A and B tiles, two buffers
constexpr size_t kFEpiBytes = (size_t)8 * 32 * kFRow * 4;               // eight 32 x 64 blocks
constexpr size_t kFLds = kFStageBytes > kFEpiBytes ? kFStageBytes : kFEpiBytes;

// Workgroup (query block qb, point segment seg of SEG), 8 wavefronts.
// Wavefront w computes the 32 x 64 products of queries 32 (w & 3) .. and
// points 64 (w >> 2) .. of each 128 x 128 block with two MFMA tiles of
// 32 x 32 (lane l of a tile: A row / B column l % 32, coordinates
// 8 (l / 32) .. + 7; result r: row 8 (r / 4) + 4 (l / 32) + r % 4, column
// l % 32), writes |p|^2 - 2 <q, p> into its LDS block as query rows, and
// lanes 2i and 2i + 1 then filter row i into their lists: with H = 2 one
// half of the row each, with H = 1 lane 2i all of it.  A query's points are
// thus dealt to 2 H SEG lists (H lanes x 2 point halves x SEG segments) of
// T = 32 / (H SEG) candidates: (SEG, H) = (2, 2) gives eight lists of 8 for
// small k, (1, 1) two lists of 32 for k up to 32.  Operand tiles are staged
// through LDS, the loads of step s + 2 in flight while step s is multiplied.
// xh: n x dp f16 (dp a multiple of kFK, zero padded); m2inv = -2 / scale^2.
// cand: [n][2 H SEG][T] indices (INT32_MAX: empty), nu: [n][2 H SEG].
template <int SEG, int H>
__global__ __launch_bounds__(kFThreads) __attribute__((amdgpu_waves_per_eu(H == 2 ? 4 : 2))) void kw_fused_kernel(const _Float16* __restrict__ xh,
                                                               const float* __restrict__ norm2, int64_t n,
                                                               int32_t dp, float m2inv, int32_t* __restrict__ cand,
                                                               float* __restrict__ nu_out) {
    constexpr int kL = 2 * H * SEG, kT = kFKc / kL;
    extern __shared__ __attribute__((aligned(16))) unsigned char kw_smem[];
    _Float16* stage = reinterpret_cast<_Float16*>(kw_smem);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wq = wave & 3, wp = wave >> 2;
    const int64_t qb = blockIdx.x / SEG;
    const int seg = blockIdx.x - (int)qb * SEG;
    const int64_t q_base = qb * kFQ;
    const int64_t nblk = (n + kFP - 1) / kFP;
    const int64_t b0 = nblk * seg / SEG, b1 = nblk * (seg + 1) / SEG;

    // the list of this lane: query 32 wq + lane / 2, point half lane & 1 (the
    // whole row, for lane & 1 == 0, when H = 1)
    const int ql = lane >> 1, half = lane & 1;
    const bool lister = H == 2 || half == 0;
    const int64_t myq = q_base + wq * 32 + ql;
    const float nq = myq < n ? norm2[myq] : 0.f;
    float bv[kT];
    int32_t bj[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        bv[t] = INFINITY;
        bj[t] = INT32_MAX;
    }
    float dropped = INFINITY;

    // staging: per step, thread t copies 16 bytes (coordinates 8 (t % 8) ..)
    // of rows t / 8 and t / 8 + 64 of each tile: every wavefront load reads
    // 8 whole 128-byte row segments
    constexpr int kV = kFQ * kFK / 8 / kFThreads;  // 16-byte vectors per thread and tile (2)
    static_assert(kFK == 64, "8 threads per staged row");
    const int sr = tid >> 3, sc = (tid & 7) * 8;
    int64_t qrow[kV];
#pragma unroll
    for (int v = 0; v < kV; ++v) qrow[v] = min(q_base + sr + 64 * v, n - 1) * dp + sc;
    const int nk = dp / kFK;
    auto tileA = [&](int buf) { return stage + (size_t)buf * 2 * kFQ * kFPitch; };
    auto tileB = [&](int buf) { return stage + (size_t)buf * 2 * kFQ * kFPitch + kFQ * kFPitch; };
    auto put = [&](int buf, const kw_u4 (&ra)[kV], const kw_u4 (&rb)[kV]) {
#pragma unroll
        for (int v = 0; v < kV; ++v) {
            *reinterpret_cast<kw_u4*>(tileA(buf) + (sr + 64 * v) * kFPitch + sc) = ra[v];
            *reinterpret_cast<kw_u4*>(tileB(buf) + (sr + 64 * v) * kFPitch + sc) = rb[v];
        }
    };
    const int fr = lane & 31, fk = 8 * (lane >> 5);  // fragment row and first coordinate

    for (int64_t blk = b0; blk < b1; ++blk) {
        const int64_t p_base = blk * kFP;
        int64_t prow[kV];
#pragma unroll
        for (int v = 0; v < kV; ++v) prow[v] = min(p_base + sr + 64 * v, n - 1) * dp + sc;
        kw_f16v acc[2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[j][r] = 0.f;
        // two register sets of staged loads: step s + 2 is requested while step
        // s is multiplied and step s + 1 waits to be written to LDS (a request
        // past the last step re-reads it, so every step issues the same loads)
        kw_u4 ra0[kV], rb0[kV], ra1[kV], rb1[kV];
        auto fetch = [&](kw_u4 (&ra)[kV], kw_u4 (&rb)[kV], int st) {
            const int o = min(st, nk - 1) * kFK;
#pragma unroll
            for (int v = 0; v < kV; ++v) {
                ra[v] = *reinterpret_cast<const kw_u4*>(xh + qrow[v] + o);
                rb[v] = *reinterpret_cast<const kw_u4*>(xh + prow[v] + o);
            }
        };
        fetch(ra0, rb0, 0);
        fetch(ra1, rb1, 1);
        __syncthreads();  // the previous block's distance blocks have been read
        put(0, ra0, rb0);
        __syncthreads();
        // step st: multiply buffer st % 2; (ia, ib) take step st + 2, (ha, hb)
        // hold step st + 1
        auto step = [&](int st, kw_u4 (&ia)[kV], kw_u4 (&ib)[kV], kw_u4 (&ha)[kV], kw_u4 (&hb)[kV]) {
            fetch(ia, ib, st + 2);
            const _Float16* A = tileA(st & 1);
            const _Float16* B = tileB(st & 1);
#pragma unroll
            for (int ks = 0; ks < kFK; ks += 16) {
                const kw_h8 fa = *reinterpret_cast<const kw_h8*>(A + (wq * 32 + fr) * kFPitch + ks + fk);
                kw_h8 fb[2];
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    fb[j] = *reinterpret_cast<const kw_h8*>(B + (wp * 64 + j * 32 + fr) * kFPitch + ks + fk);
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(fa, fb[j], acc[j], 0, 0, 0);
            }
            if (st + 1 < nk) put((st + 1) & 1, ha, hb);
            __syncthreads();
        };
        int st = 0;
        for (; st + 1 < nk; st += 2) {
            step(st, ra0, rb0, ra1, rb1);
            step(st + 1, ra1, rb1, ra0, rb0);
        }
        if (st < nk) step(st, ra0, rb0, ra1, rb1);

        // |p|^2 - 2 <q, p> as query rows of this wavefront's block
        float* blkd = reinterpret_cast<float*>(kw_smem) + (size_t)wave * 32 * kFRow;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int64_t p = p_base + wp * 64 + j * 32 + fr;
            const float np = norm2[p < n ? p : n - 1];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                blkd[row * kFRow + j * 32 + fr] = fmaf(m2inv, acc[j][r], np);
            }
        }
        // lanes 2i, 2i + 1: the two halves of row i (query 32 wq + i), in order
        constexpr int kC = 64 / H;  // points per list and block
        const float4* rowv = reinterpret_cast<const float4*>(blkd + ql * kFRow + (H == 2 ? half * 32 : 0));
        const int64_t pj0 = p_base + wp * 64 + (H == 2 ? half * 32 : 0);
#pragma unroll 2
        for (int c4 = 0; c4 < (lister ? kC / 4 : 0); ++c4) {
            const float4 v4 = rowv[c4];
            const float vv[4] = {v4.x, v4.y, v4.z, v4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t j = pj0 + c4 * 4 + e;
                if (j >= n || j == myq) continue;
                const float a = nq + vv[e];
                if (a < bv[kT - 1] || (a == bv[kT - 1] && (int32_t)j < bj[kT - 1])) {
                    float out;
                    kw_insert<kT>(bv, bj, a, (int32_t)j, out);
                    dropped = fminf(dropped, out);
                } else {
                    dropped = fminf(dropped, a);
                }
            }
        }
    }
    if (myq < n && lister) {
        const int list = (seg * 2 + wp) * H + (H == 2 ? half : 0);
        int32_t* cq = cand + (myq * kL + list) * kT;
#pragma unroll
        for (int t = 0; t < kT; ++t) cq[t] = bj[t];
        nu_out[myq * kL + list] = dropped;
    }
}

// Exact f32 distance as the exact kernel forms it (one FMA per coordinate,
// in order); rows whose length is a multiple of 4 are read 16 bytes at a time.
__device__ __forceinline__ float kw_exact(const float* __restrict__ a, const float* __restrict__ b, int32_t d) {
    float acc = 0.f;
    int c = 0;
    if ((d & 3) == 0) {
        const float4* a4 = reinterpret_cast<const float4*>(a);
        const float4* b4 = reinterpret_cast<const float4*>(b);
#pragma unroll 4
        for (int c4 = 0; c4 < d / 4; ++c4) {
            const float4 u = a4[c4], v = b4[c4];
            float t = u.x - v.x;
            acc = fmaf(t, t, acc);
            t = u.y - v.y;
            acc = fmaf(t, t, acc);
            t = u.z - v.z;
            acc = fmaf(t, t, acc);
            t = u.w - v.w;
            acc = fmaf(t, t, acc);
        }
        c = d;
    }
    for (; c < d; ++c) {
        const float t = a[c] - b[c];
        acc = fmaf(t, t, acc);
    }
    return acc;
}

// Bitonic sort of one (v, j) pair per lane across the wavefront, ascending.
__device__ __forceinline__ void kw_wave_sort(float& v, int32_t& j) {
    const int lane = threadIdx.x & 63;
    for (int size = 2; size <= 64; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const float ov = __shfl_xor(v, stride, 64);
            const int32_t oj = __shfl_xor(j, stride, 64);
            const bool up = (lane & size) == 0;
            const bool lower = (lane & stride) == 0;
            const bool other_less = ov < v || (ov == v && oj < j);
            const bool take = (lower == up) ? other_less : !other_less;
            if (take && !(ov == v && oj == j)) {
                v = ov;
                j = oj;
            }
        }
    }
}

// One wavefront per query: exact distances of the candidates, the k best
// written out, and the certificate nu - E_q > d_k checked (nu: the smallest of
// the query's `lists` list bounds); failures listed.
__global__ __launch_bounds__(256) void kw_refine_kernel(const float* __restrict__ x, int64_t n, int32_t d,
                                                       int32_t k, const int32_t* __restrict__ cand,
                                                       const float* __restrict__ nu, int32_t lists,
                                                       const float* __restrict__ norm2,
                                                       float err_a, float err_b, float err_c, float rel_exact,
                                                       int32_t* __restrict__ idx_out, float* __restrict__ d2_out,
                                                       int32_t* fail_list, unsigned int* fail_count) {
    const int64_t q = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (q >= n) return;
    static_assert(kFKc == 64, "one candidate per lane");
    int32_t j = cand[q * kFKc + lane];
    float v = INFINITY;
    if (j >= 0 && j < n) v = kw_exact(x + q * d, x + (int64_t)j * d, d);
    else j = INT32_MAX;
    kw_wave_sort(v, j);
    if (lane < k) {
        idx_out[q * k + lane] = j;
        if (d2_out) d2_out[q * k + lane] = v;
    }
    const float dk = __shfl(v, k - 1, 64);
    if (lane == 0) {
        // every other point's approximate distance is >= nu, its real distance
        // >= nu - E_q, its exact f32 distance >= (nu - E_q)(1 - rel_exact)
        float nuq = nu[q * lists];
        for (int t = 1; t < lists; ++t) nuq = fminf(nuq, nu[q * lists + t]);
        const float nq = norm2[q], aq = sqrtf(nq);
        const float eq = err_a * aq + err_b * nq + err_c;
        if (!((nuq - eq) * (1.0f - rel_exact) > dk)) {
            const unsigned int slot = atomicAdd(fail_count, 1u);
            fail_list[slot] = (int32_t)q;
        }
    }
}

// Exact scan for the rows without a certificate.  Block (slice, row) takes
// the points j = slice * per, ... (per = points per slice, at most 8 per lane)
// and writes the k best of them, ascending with ties by index; a second
// kernel merges a row's slices.
constexpr int kScanLane = 8;  // points per lane and slice

__global__ __launch_bounds__(256) void kw_scan_slice_kernel(const float* __restrict__ x, int64_t n, int32_t d,
                                                           int32_t k, int64_t per, int32_t slices,
                                                           const int32_t* __restrict__ rows,
                                                           float* __restrict__ pv, int32_t* __restrict__ pj) {
    __shared__ float sv[4][32];
    __shared__ int32_t sj[4][32];
    const int64_t q = rows[blockIdx.y];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float bv[kScanLane];
    int32_t bj[kScanLane];
#pragma unroll
    for (int t = 0; t < kScanLane; ++t) {
        bv[t] = INFINITY;
        bj[t] = INT32_MAX;
    }
    const int64_t j0 = (int64_t)blockIdx.x * per, j1 = j0 + per < n ? j0 + per : n;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += 256) {
        if (j == q) continue;
        float out;
        kw_insert<kScanLane>(bv, bj, kw_exact(x + q * d, x + j * d, d), (int32_t)j, out);
    }
    for (int t = 0; t < k; ++t) {
        float v;
        int32_t j;
        kw_pop_min<kScanLane>(bv, bj, v, j);
        if (lane == 0) {
            sv[wave][t] = v;
            sj[wave][t] = j;
        }
    }
    __syncthreads();
    if (wave == 0) {
        // merge the four sorted wavefront lists: lane w < 4 walks list w
        int pos = 0;
        const int64_t o = ((int64_t)blockIdx.y * slices + blockIdx.x) * k;
        for (int t = 0; t < k; ++t) {
            const float hv = (lane < 4 && pos < k) ? sv[lane][pos] : INFINITY;
            const int32_t hj = (lane < 4 && pos < k) ? sj[lane][pos] : INT32_MAX;
            float mv = hv;
            int32_t mj = hj;
            for (int off = 32; off > 0; off >>= 1) {
                const float ov = __shfl_xor(mv, off, 64);
                const int32_t oj = __shfl_xor(mj, off, 64);
                if (ov < mv || (ov == mv && oj < mj)) {
                    mv = ov;
                    mj = oj;
                }
            }
            if (lane < 4 && hj == mj && hv == mv) ++pos;
            if (lane == 0) {
                pv[o + t] = mv;
                pj[o + t] = mj;
            }
        }
    }
}

// One wavefront per rescanned row: lane l keeps the k best of the slices
// l, l + 64, ...; the wavefront then pops the row's k best.
__global__ __launch_bounds__(64) void kw_scan_merge_kernel(int32_t k, int32_t slices,
                                                          const int32_t* __restrict__ rows,
                                                          const float* __restrict__ pv,
                                                          const int32_t* __restrict__ pj,
                                                          int32_t* __restrict__ idx_out,
                                                          float* __restrict__ d2_out) {
    constexpr int KM = 32;
    const int64_t q = rows[blockIdx.x];
    const int lane = threadIdx.x;
    float bv[KM];
    int32_t bj[KM];
#pragma unroll
    for (int t = 0; t < KM; ++t) {
        bv[t] = INFINITY;
        bj[t] = INT32_MAX;
    }
    for (int sl = lane; sl < slices; sl += 64) {
        const int64_t o = ((int64_t)blockIdx.x * slices + sl) * k;
        for (int t = 0; t < k; ++t) {
            float out;
            kw_insert<KM>(bv, bj, pv[o + t], pj[o + t], out);
        }
    }
    for (int t = 0; t < k; ++t) {
        float v;
        int32_t j;
        kw_pop_min<KM>(bv, bj, v, j);
        if (lane == 0) {
            idx_out[q * k + t] = j;
            if (d2_out) d2_out[q * k + t] = v;
        }
    }
}

}  // namespace

namespace gl {

// Wide-feature path of gl_knn; arguments already checked (64 < d <= 4096).
gl_status knn_wide(const float* x, int64_t n, int32_t d, int32_t k, int32_t* idx_out, float* d2_out,
                   hipStream_t s, int64_t* fallback_rows) {
    const int32_t dp = (d + kFK - 1) / kFK * kFK;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_xh = al((size_t)n * dp * 2), b_n = al((size_t)n * 4), b_c = al((size_t)n * kFKc * 4),
                 b_nu = al((size_t)n * 8 * 4), b_f = al((size_t)n * 4);
    const size_t b_mu = al((size_t)d * 4) + al((size_t)kMeanSlices * d * 8);
    char* base = nullptr;
    if (hipMallocAsync((void**)&base, b_xh + b_n + b_c + b_nu + b_f + b_mu + 256, s) != hipSuccess) {
        (void)hipGetLastError();
        return wfail(GL_E_NOMEM, "temporary device memory for the wide kNN");
    }
    char* p = base;
    _Float16* xh = (_Float16*)p;
    p += b_xh;
    float* norm2 = (float*)p;
    p += b_n;
    int32_t* cand = (int32_t*)p;
    p += b_c;
    float* nu = (float*)p;
    p += b_nu;
    int32_t* fails = (int32_t*)p;
    p += b_f;
    float* mu = (float*)p;
    double* mu_part = (double*)(p + al((size_t)d * 4));
    p += b_mu;
    unsigned int* counters = (unsigned int*)p;  // [0] max |x| bits, [1] failures

    gl_status st = GL_OK;
    hipError_t e = hipMemsetAsync(counters, 0, 8, s);
    unsigned int hc[2] = {0, 0};
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kw_mean_partial_kernel, dim3((unsigned)((d + 255) / 256), kMeanSlices), dim3(256), 0, s,
                           x, n, d, mu_part);
        e = hipGetLastError();
        if (e == hipSuccess) {
            hipLaunchKernelGGL(kw_mean_final_kernel, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s,
                               (const double*)mu_part, n, d, mu);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(kw_norms_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, x, (const float*)mu, n,
                           d, norm2, counters);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hc, counters, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float amax = 0.f;
    if (e == hipSuccess) {
        std::memcpy(&amax, &hc[0], 4);
        if (!std::isfinite(amax)) st = wfail(GL_E_INVALID_ARG, "x holds a non-finite coordinate");
    }
    // scale by a power of two so that the largest coordinate is in [2^13, 2^14)
    const int ex = amax > 0.f ? 13 - (int)std::floor(std::log2((double)amax)) : 0;
    const double scale = std::ldexp(1.0, ex);
    if (e == hipSuccess && st == GL_OK) {
        const int64_t tot = n * dp;
        hipLaunchKernelGGL(kw_half_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x,
                           (const float*)mu, n, d, dp, (float)scale, xh);
        e = hipGetLastError();
    }
    // Error of an approximate distance |q|^2 + |p|^2 - 2 <q~, p~> (tilde: f16):
    //   f16 rounding of both factors, |<q~,p~> - <q,p>| <= (2u + u^2) |q| |p|
    //   (u = 2^-11) plus the range below the smallest normal f16 (2^-14, which
    //   the matrix cores may flush to zero), sub = 2^-14 sqrt(d) / scale, times
    //   (|q| + |p|); f32 accumulation over dp terms, the f32 norms and the final
    //   combination: g |q| |p| and g (|q|^2 + |p|^2) with a generous
    //   g = 4 (dp + 8) 2^-24; the f32 rounding of the centring changes a
    //   distance by at most h (|q| + |p|)^2, h = 2^-22.  Norms are those of the
    //   centred points; with |p| <= P:
    //   E_q = A |q| + B |q|^2 + C,  A = 2 (2u + u^2 + g) P + 2 sub + 2 h P,
    //   B = g + h,  C = 2 sub P + (g + h) P^2, each raised by 1 %.
    double maxn2 = 0.0;
    if (st == GL_OK && e == hipSuccess) {
        std::vector<float> hn(n);
        e = hipMemcpyAsync(hn.data(), norm2, (size_t)n * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        for (int64_t i = 0; i < n && e == hipSuccess; ++i) {
            if (!std::isfinite(hn[i])) {
                st = wfail(GL_E_INVALID_ARG, "x holds a non-finite coordinate");
                break;
            }
            maxn2 = std::max(maxn2, (double)hn[i]);
        }
    }
    const double P = std::sqrt(maxn2) * (1.0 + 1e-6);
    const double u = std::ldexp(1.0, -11), g = 4.0 * (dp + 8) * std::ldexp(1.0, -24);
    const double sub = std::ldexp(1.0, -14) * std::sqrt((double)d) / scale;
    const double hcen = std::ldexp(1.0, -22);
    const float err_a = (float)(1.01 * (2.0 * (2.0 * u + u * u + g) * P + 2.0 * sub + 2.0 * hcen * P));
    const float err_b = (float)(1.01 * (g + hcen));
    const float err_c = (float)(1.01 * (2.0 * sub * P + (g + hcen) * maxn2));
    // the exact f32 distance (d fused multiply-adds) is within d 2^-24 of the real one, relatively
    const float rel_exact = (float)(1.01 * (d + 2) * std::ldexp(1.0, -24));
    const float m2inv = (float)(-2.0 / (scale * scale));
    // eight lists of 8 candidates per query while a list cannot be expected to
    // need more than 8 of the k best; two of 32 for larger k
    const bool small_k = k <= 12;
    if (st == GL_OK && e == hipSuccess) {
        const unsigned nqb = (unsigned)((n + kFQ - 1) / kFQ);
        if (small_k)
            hipLaunchKernelGGL((kw_fused_kernel<2, 2>), dim3(nqb * 2), dim3(kFThreads), kFLds, s,
                               (const _Float16*)xh, (const float*)norm2, n, dp, m2inv, cand, nu);
        else
            hipLaunchKernelGGL((kw_fused_kernel<1, 1>), dim3(nqb), dim3(kFThreads), kFLds, s, (const _Float16*)xh,
                               (const float*)norm2, n, dp, m2inv, cand, nu);
        e = hipGetLastError();
    }
    if (st == GL_OK && e == hipSuccess) {
        hipLaunchKernelGGL(kw_refine_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, x, n, d, k,
                           (const int32_t*)cand, (const float*)nu, small_k ? 8 : 2, (const float*)norm2, err_a, err_b, err_c,
                           rel_exact, idx_out, d2_out, fails, counters + 1);
        e = hipGetLastError();
    }
    if (st == GL_OK && e == hipSuccess) e = hipMemcpyAsync(&hc[1], counters + 1, 4, hipMemcpyDeviceToHost, s);
    if (st == GL_OK && e == hipSuccess) e = hipStreamSynchronize(s);
    if (st == GL_OK && e == hipSuccess && hc[1] > 0) {
        const int64_t per = 256 * kScanLane;
        const int32_t slices = (int32_t)((n + per - 1) / per);
        float* pv = nullptr;
        const size_t pb = (size_t)hc[1] * slices * k;
        e = hipMallocAsync((void**)&pv, pb * 8, s);
        if (e == hipSuccess) {
            int32_t* pj = (int32_t*)(pv + pb);
            hipLaunchKernelGGL(kw_scan_slice_kernel, dim3((unsigned)slices, hc[1]), dim3(256), 0, s, x, n, d, k, per,
                               slices, fails, pv, pj);
            e = hipGetLastError();
            if (e == hipSuccess) {
                hipLaunchKernelGGL(kw_scan_merge_kernel, dim3(hc[1]), dim3(64), 0, s, k, slices, fails,
                                   (const float*)pv, (const int32_t*)pj, idx_out, d2_out);
                e = hipGetLastError();
            }
            const hipError_t e2 = hipFreeAsync(pv, s);
            if (e == hipSuccess) e = e2;
        } else {
            st = wfail(GL_E_NOMEM, "temporary device memory for the exact rescan");
        }
    }
    if (fallback_rows) *fallback_rows = hc[1];
    const hipError_t ef = hipFreeAsync(base, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (st != GL_OK) return st;
    if (e != hipSuccess || ef != hipSuccess || es != hipSuccess)
        return wfail(GL_E_HIP, std::string("wide kNN: ") +
                                   hipGetErrorString(e != hipSuccess ? e : (ef != hipSuccess ? ef : es)));
    return GL_OK;
}

}  // namespace gl
