// Construction of the window operator (the image graph of Section 2.2) and the
// host side of its power-method pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "gl_internal.hpp"
#include "gl_window.hpp"

namespace gl {
namespace {

struct WinAlpha {
    double a[(2 * kWinMaxRp + 1) * (2 * kWinMaxRp + 1)];  // row-major over the patch offsets
};

// Colours with a border of rp pixels replicated from the nearest edge pixel,
// channels padded to four: J[(y + rp) * (width + 2 rp) + x + rp] = C(clamp(y), clamp(x)).
__global__ void window_pad_kernel(const float* __restrict__ img, int32_t h, int32_t w, int32_t C, int32_t rp,
                                  float4* __restrict__ J) {
    const int64_t Jw = (int64_t)w + 2 * rp, Jh = (int64_t)h + 2 * rp;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Jw * Jh) return;
    const int64_t yy = i / Jw, xx = i - yy * Jw;
    const int64_t y = yy - rp < 0 ? 0 : (yy - rp >= h ? h - 1 : yy - rp);
    const int64_t x = xx - rp < 0 ? 0 : (xx - rp >= w ? w - 1 : xx - rp);
    const float* c = img + (y * w + x) * C;
    float4 v;
    v.x = c[0];
    v.y = C > 1 ? c[1] : 0.f;
    v.z = C > 2 ? c[2] : 0.f;
    v.w = C > 3 ? c[3] : 0.f;
    J[i] = v;
}

// Raw weights in double, one block per (tile, offset m of the first half of
// the scan order); the weight of the pair (p, q = p + o_m) is written to p's
// slot m and to q's slot M - 1 - m (offset -o_m), so the stored W is
// symmetric bit for bit.  raw[(tile * M + m) * 256 + lane], zero-initialised.
__global__ __launch_bounds__(256) void window_raw_kernel(const float4* __restrict__ J, int32_t h, int32_t w,
                                                         int32_t r, int32_t rp, int32_t tiles_x, int32_t M,
                                                         WinAlpha al, double inv_s2, double* __restrict__ raw) {
    const int64_t b = blockIdx.x;
    const int m = blockIdx.y;  // < M / 2: the cell index of the scan equals m
    const int side = 2 * r + 1;
    const int dy = m / side - r, dx = m - (m / side) * side - r;
    const int ty = (int)(b / tiles_x), tx = (int)(b - (int64_t)ty * tiles_x);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = tx * kWinTX + lane, y = ty * kWinTY + wave;
    const int qx = x + dx, qy = y + dy;
    if (x >= w || y >= h || qx < 0 || qx >= w || qy < 0 || qy >= h) return;
    const int64_t Jw = (int64_t)w + 2 * rp;
    const int pw = 2 * rp + 1;
    double s = 0.0;
    for (int a = 0; a < pw; ++a) {
        const float4* rowp = J + (int64_t)(y + a) * Jw + x;
        const float4* rowq = J + (int64_t)(qy + a) * Jw + qx;
        for (int c = 0; c < pw; ++c) {
            const float4 cp = rowp[c], cq = rowq[c];
            const double d0 = (double)cp.x - (double)cq.x, d1 = (double)cp.y - (double)cq.y;
            const double d2 = (double)cp.z - (double)cq.z, d3 = (double)cp.w - (double)cq.w;
            s += al.a[a * pw + c] * (((d0 * d0 + d1 * d1) + d2 * d2) + d3 * d3);
        }
    }
    const double wgt = exp(-s * inv_s2);
    raw[(b * M + m) * 256 + threadIdx.x] = wgt;
    const int64_t qb = (int64_t)(qy / kWinTY) * tiles_x + qx / kWinTX;
    const int ql = (qy % kWinTY) * kWinTX + qx % kWinTX;
    raw[(qb * M + (M - 1 - m)) * 256 + ql] = wgt;
}

// d_p = sum over the window of w_pq in double, in increasing offset order
// (increasing neighbour index), into the pixel-ordered degree array.
__global__ __launch_bounds__(256) void window_degree_kernel(const double* __restrict__ raw, int32_t h, int32_t w,
                                                            int32_t tiles_x, int32_t M, double* __restrict__ d,
                                                            int32_t* flags, unsigned long long* first_bad) {
    const int64_t b = blockIdx.x;
    const int ty = (int)(b / tiles_x), tx = (int)(b - (int64_t)ty * tiles_x);
    const int x = tx * kWinTX + (threadIdx.x & 63), y = ty * kWinTY + (threadIdx.x >> 6);
    if (x >= w || y >= h) return;
    double s = 0.0;
    for (int m = 0; m < M; ++m) s += raw[(b * M + m) * 256 + threadIdx.x];
    const int64_t p = (int64_t)y * w + x;
    d[p] = s;
    if (!(s > 0.0) || !(s <= 1.7976931348623157e308)) {
        atomicOr(flags, (int32_t)BAD_DEGREE);
        atomicMin(first_bad, (unsigned long long)p);
    }
}

// Stored weights: what_pq = w_pq / sqrt(d_p d_q) (raw = 0) or w_pq (raw != 0),
// rounded once to TW, for the first half of each pixel's window; one block per
// (tile, vector of GS offsets).
template <typename TW>
__global__ __launch_bounds__(256) void window_fill_kernel(const double* __restrict__ raw,
                                                          const double* __restrict__ d, int32_t h, int32_t w,
                                                          int32_t r, int32_t tiles_x, int32_t M, int32_t raw_mode,
                                                          u32x4* __restrict__ out) {
    constexpr int GS = 16 / (int)sizeof(TW);
    const int64_t b = blockIdx.x;
    const int g = blockIdx.y, ng = window_groups(M, GS);
    const int side = 2 * r + 1;
    const int ty = (int)(b / tiles_x), tx = (int)(b - (int64_t)ty * tiles_x);
    const int x = tx * kWinTX + (threadIdx.x & 63), y = ty * kWinTY + (threadIdx.x >> 6);
    const bool ok = x < w && y < h;
    const double dp = ok ? d[(int64_t)y * w + x] : 1.0;
    TW vals[GS];
#pragma unroll
    for (int e = 0; e < GS; ++e) {
        const int m = g * GS + e;
        double o = 0.0;
        if (m < M / 2) {
            const double wv = raw[(b * M + m) * 256 + threadIdx.x];
            if (ok && wv != 0.0) {
                const int dy = m / side - r, dx = m - (m / side) * side - r;  // the cell index of the scan equals m
                const double dq = d[(int64_t)(y + dy) * w + (x + dx)];
                o = raw_mode ? wv : wv / (sqrt(dp) * sqrt(dq));
            }
        }
        vals[e] = store_as<TW>::from(o);
    }
    u32x4 v;
    __builtin_memcpy(&v, vals, 16);
    out[(b * ng + g) * 256 + threadIdx.x] = v;
}

// Unnormalized L: diagonal dd_p = sum of the stored weights of p's whole window
// (double, offset order: the first half from p's vectors, the second half
// from the neighbours', which keep the weight of the mirrored offset),
// rounded to the accumulator type A.
template <typename TW, typename A>
__global__ __launch_bounds__(256) void window_rowsum_kernel(const TW* __restrict__ wst, int32_t h, int32_t w,
                                                            int32_t r, int32_t tiles_x, int32_t M,
                                                            A* __restrict__ dd) {
    constexpr int GS = 16 / (int)sizeof(TW);
    const int64_t b = blockIdx.x;
    const int ty = (int)(b / tiles_x), tx = (int)(b - (int64_t)ty * tiles_x);
    const int x = tx * kWinTX + (threadIdx.x & 63), y = ty * kWinTY + (threadIdx.x >> 6);
    if (x >= w || y >= h) return;
    const int ng = window_groups(M, GS), side = 2 * r + 1;
    auto stored = [&](int qy, int qx, int m) {
        const int64_t qb = (int64_t)(qy / kWinTY) * tiles_x + qx / kWinTX;
        const int ql = (qy % kWinTY) * kWinTX + qx % kWinTX;
        return cvt<double>(wst[((qb * ng + m / GS) * 256 + ql) * GS + m % GS]);
    };
    double s = 0.0;
    for (int m = 0; m < M; ++m) {
        if (m < M / 2) {
            s += stored(y, x, m);
        } else {
            const int cell = m + 1;
            const int qy = y + cell / side - r, qx = x + cell % side - r;
            if (qy < h && qx >= 0 && qx < w) s += stored(qy, qx, M - 1 - m);
        }
    }
    dd[(int64_t)y * w + x] = (A)s;
}

template <typename TW>
hipError_t launch_fill_t(const double* raw, const double* d, const gl_operator* op, int raw_mode, hipStream_t s) {
    const int GS = 16 / (int)sizeof(TW);
    const dim3 grid((unsigned)op->nblocks, (unsigned)window_groups(op->wM, GS));
    hipLaunchKernelGGL(window_fill_kernel<TW>, grid, dim3(256), 0, s, raw, d, op->wheight, op->wwidth, op->wr,
                       op->wtiles_x, op->wM, raw_mode, (u32x4*)op->w);
    return hipGetLastError();
}

template <typename TW, typename A>
hipError_t launch_rowsum_t(const gl_operator* op, hipStream_t s) {
    hipLaunchKernelGGL((window_rowsum_kernel<TW, A>), dim3((unsigned)op->nblocks), dim3(256), 0, s,
                       (const TW*)op->w, op->wheight, op->wwidth, op->wr, op->wtiles_x, op->wM, (A*)op->dd);
    return hipGetLastError();
}

size_t wdtype_size(gl_dtype d) {
    switch (d) {
        case GL_F64: return 8;
        case GL_F32: return 4;
        case GL_BF16:
        case GL_F16: return 2;
    }
    return 0;
}

gl_status wfail(gl_status st, const std::string& msg) {
    set_last_error(msg);
    return st;
}

}  // namespace

size_t window_lds_bytes(const gl_operator* op, int K, size_t acc) {
    return 2 * (size_t)K * window_region(op->wr) * acc;
}

size_t window_part_bytes(const gl_operator* op, int K, size_t acc) {
    if (op->layout != LAYOUT_WINDOW) return 0;
    return (size_t)op->nblocks * window_region(op->wr) * K * acc;
}

template <typename TW>
static void window_power_t(const WinPowerArgs& a, const gl_operator* op, hipStream_t s) {
    WinPartArgs<float> pa;
    pa.op = a.op;
    pa.v = a.x;
    pa.part = const_cast<float*>(a.part);
    const dim3 grid((unsigned)op->nblocks), block(256);
    hipLaunchKernelGGL((window_part_kernel<1, TW, float>), grid, block, window_lds_bytes(op, 1, 4), s, pa);
    hipLaunchKernelGGL(window_power_kernel<TW>, grid, block, 0, s, a);
}

hipError_t launch_window_power(const gl_operator* op, const float* x, float* y, int mode, const float* scale,
                               float* partials, float* part, hipStream_t s) {
    WinPowerArgs a;
    a.op.w = op->w;
    a.op.height = op->wheight;
    a.op.width = op->wwidth;
    a.op.r = op->wr;
    a.op.M = op->wM;
    a.op.tiles_x = op->wtiles_x;
    a.part = part;
    a.x = x;
    a.y = y;
    a.scale = scale;
    a.partials = partials;
    a.dd = (const float*)op->dd;
    a.mode = mode;
    switch (op->store_w) {
        case GL_F32: window_power_t<float>(a, op, s); break;
        case GL_BF16: window_power_t<bf16>(a, op, s); break;
        case GL_F16: window_power_t<f16>(a, op, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gl

extern "C" gl_status gl_window_operator_create(const gl_window_graph* g, gl_dtype store_w, void* stream,
                                               gl_operator** out) {
    using namespace gl;
    if (!g || !out) return wfail(GL_E_INVALID_ARG, "graph and out must not be NULL");
    *out = nullptr;
    if (!g->image) return wfail(GL_E_INVALID_ARG, "image must not be NULL");
    if (((uintptr_t)g->image) % 4) return wfail(GL_E_INVALID_ARG, "image must be 4-byte aligned");
    if (g->height < 1 || g->width < 1 || (int64_t)g->height * g->width >= ((int64_t)1 << 31))
        return wfail(GL_E_INVALID_ARG, "height and width must be >= 1 with height * width < 2^31");
    if (g->channels < 1 || g->channels > 4) return wfail(GL_E_INVALID_ARG, "channels must lie in [1, 4]");
    if (g->window_radius < 1 || g->window_radius > kWinMaxR)
        return wfail(GL_E_INVALID_ARG, "window_radius must lie in [1, 27]");
    if (g->patch_radius < 0 || g->patch_radius > kWinMaxRp)
        return wfail(GL_E_INVALID_ARG, "patch_radius must lie in [0, 4]");
    if (!(g->sigma > 0.0) || !std::isfinite(g->sigma)) return wfail(GL_E_INVALID_ARG, "sigma must be finite and > 0");
    if (g->laplacian != GL_LAP_NORMALIZED && g->laplacian != GL_LAP_UNNORMALIZED)
        return wfail(GL_E_INVALID_ARG, "unknown laplacian");
    if (g->reserved != 0) return wfail(GL_E_INVALID_ARG, "reserved must be 0");
    if (wdtype_size(store_w) == 0) return wfail(GL_E_DTYPE, "unknown weight storage type");
    hipStream_t s = (hipStream_t)stream;

    const int32_t h = g->height, w = g->width, r = g->window_radius, rp = g->patch_radius;
    const int32_t side = 2 * r + 1, M = side * side - 1;
    const int32_t tiles_x = (w + kWinTX - 1) / kWinTX, tiles_y = (h + kWinTY - 1) / kWinTY;
    const int64_t ntiles = (int64_t)tiles_x * tiles_y;
    const int64_t n = (int64_t)h * w;
    const int GS = 16 / (int)wdtype_size(store_w);
    const int64_t stored = ntiles * 256 * window_groups(M, GS) * GS;  // first half of each window, padded
    const int64_t rawn = ntiles * 256 * M;                             // F64 weights of the whole windows

    gl_operator* op = new gl_operator();
    op->n = n;
    op->store_w = store_w;
    op->layout = LAYOUT_WINDOW;
    op->lap = g->laplacian;
    op->G = 1;
    op->wheight = h;
    op->wwidth = w;
    op->wr = r;
    op->wM = M;
    op->wtiles_x = tiles_x;
    op->nblocks = ntiles;
    op->stored = stored;
    // edges: the window clipped to the image, minus the pixel itself
    int64_t sy = 0, sx = 0;
    for (int32_t y = 0; y < h; ++y) sy += std::min(y + r, h - 1) - std::max(y - r, 0) + 1;
    for (int32_t x = 0; x < w; ++x) sx += std::min(x + r, w - 1) - std::max(x - r, 0) + 1;
    op->nnz = sy * sx - n;
    (void)hipGetDevice(&op->device);

    // patch weights: separable Gaussian normalised to sum 1
    WinAlpha al = {};
    {
        const int pw = 2 * rp + 1;
        std::vector<double> gg(pw);
        double gs = 0.0;
        for (int t = -rp; t <= rp; ++t) {
            gg[t + rp] = rp > 0 ? std::exp(-(double)t * t / (2.0 * rp * rp)) : 1.0;
            gs += gg[t + rp];
        }
        for (int a = 0; a < pw; ++a)
            for (int c = 0; c < pw; ++c) al.a[a * pw + c] = gg[a] * gg[c] / (gs * gs);
    }

    const size_t wbytes = (size_t)stored * wdtype_size(store_w);
    const size_t Jn = (size_t)(h + 2 * rp) * (size_t)(w + 2 * rp);
    float4* J = nullptr;
    double* raw = nullptr;
    int32_t* flags = nullptr;
    std::string what;
    hipError_t e = hipMalloc(&op->w, wbytes);
    if (e == hipSuccess) e = hipMalloc((void**)&op->degree, (size_t)n * 8);
    if (e == hipSuccess) e = hipMalloc((void**)&J, Jn * sizeof(float4));
    if (e == hipSuccess) e = hipMalloc((void**)&raw, (size_t)rawn * 8);
    if (e == hipSuccess) e = hipMalloc((void**)&flags, 16);
    if (e != hipSuccess) {
        (void)hipFree(J);
        (void)hipFree(raw);
        (void)hipFree(flags);
        gl_operator_destroy(op);
        (void)hipGetLastError();
        return wfail(GL_E_NOMEM, "device allocation for the window operator failed");
    }
    op->bytes = wbytes + (size_t)n * 8;
    unsigned long long* first_bad = (unsigned long long*)(flags + 2);
    const unsigned long long none = ~0ull;
    int32_t hflags[4] = {0, 0, 0, 0};
    __builtin_memcpy(&hflags[2], &none, 8);

    e = hipMemcpyAsync(flags, hflags, 16, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(raw, 0, (size_t)rawn * 8, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(window_pad_kernel, dim3((unsigned)((Jn + 255) / 256)), dim3(256), 0, s, g->image, h, w,
                           g->channels, rp, J);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(window_raw_kernel, dim3((unsigned)ntiles, (unsigned)(M / 2)), dim3(256), 0, s,
                           (const float4*)J, h, w, r, rp, tiles_x, M, al, 1.0 / (g->sigma * g->sigma), raw);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(window_degree_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, (const double*)raw, h, w,
                           tiles_x, M, op->degree, flags, first_bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(hflags, flags, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    gl_status st = GL_OK;
    if (e != hipSuccess) {
        st = wfail(GL_E_HIP, std::string("window weights: ") + hipGetErrorString(e));
    } else if (hflags[0]) {
        unsigned long long bad = 0;
        __builtin_memcpy(&bad, &hflags[2], 8);
        st = wfail(GL_E_BAD_GRAPH, "window graph: pixel (" + std::to_string(bad / (unsigned long long)w) + ", " +
                                       std::to_string(bad % (unsigned long long)w) +
                                       ") has degree 0 (no neighbour, or every weight underflows)");
    }
    if (st == GL_OK) {
        const int raw_mode = op->lap == GL_LAP_UNNORMALIZED ? 1 : 0;
        switch (store_w) {
            case GL_F64: e = launch_fill_t<double>(raw, op->degree, op, raw_mode, s); break;
            case GL_F32: e = launch_fill_t<float>(raw, op->degree, op, raw_mode, s); break;
            case GL_BF16: e = launch_fill_t<bf16>(raw, op->degree, op, raw_mode, s); break;
            default: e = launch_fill_t<f16>(raw, op->degree, op, raw_mode, s); break;
        }
        if (e == hipSuccess && raw_mode) {
            const size_t es = store_w == GL_F64 ? 8 : 4;
            e = hipMalloc(&op->dd, (size_t)n * es);
            if (e == hipSuccess) {
                op->bytes += (size_t)n * es;
                switch (store_w) {
                    case GL_F64: e = launch_rowsum_t<double, double>(op, s); break;
                    case GL_F32: e = launch_rowsum_t<float, float>(op, s); break;
                    case GL_BF16: e = launch_rowsum_t<bf16, float>(op, s); break;
                    default: e = launch_rowsum_t<f16, float>(op, s); break;
                }
            }
            std::vector<char> hd;
            if (e == hipSuccess) {
                hd.resize((size_t)n * es);
                e = hipMemcpyAsync(hd.data(), op->dd, hd.size(), hipMemcpyDeviceToHost, s);
            }
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            double mx = 0.0;
            for (int64_t i = 0; e == hipSuccess && i < n; ++i) {
                const double v = es == 8 ? ((const double*)hd.data())[i] : (double)((const float*)hd.data())[i];
                if (!(v > 0.0) || !std::isfinite(v)) {
                    st = wfail(GL_E_BAD_GRAPH, "window graph: a stored row sums to a non-positive degree");
                    break;
                }
                mx = v > mx ? v : mx;
            }
            op->dmax = mx;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess && st == GL_OK) st = wfail(GL_E_HIP, std::string("window fill: ") + hipGetErrorString(e));
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(J);
    (void)hipFree(raw);
    (void)hipFree(flags);
    if (st != GL_OK) {
        gl_operator_destroy(op);
        return st;
    }
    *out = op;
    return GL_OK;
}
