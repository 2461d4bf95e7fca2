// C ABI of the gfx950 preconditioned-DCA library: operator construction,
// Laplacian product, power method, the preconditioned DCA solve and labelling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include <vector>

#include "gl_internal.hpp"
#include "gl_kernels.hpp"
#include "gl_direct.hpp"
#include "gl_layout.hpp"
#include "gl_sched.hpp"
#include "gl_tile.hpp"
#include "gl_window.hpp"
#include "gl_grid.hpp"
#include "gl_grid_build.hpp"


namespace {

thread_local std::string g_err;

gl_status fail(gl_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

}  // namespace

void gl::set_last_error(const std::string& msg) { g_err = msg; }

namespace {

#define GL_HIP(expr, what)                                                                \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(GL_E_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t dtype_size(int d) {
    switch (d) {
        case GL_F64: return 8;
        case GL_F32: return 4;
        case GL_BF16:
        case GL_F16: return 2;
        default: return 0;
    }
}

typedef gl::u32x4 u32x4_alias;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }


}  // namespace

static_assert(gl::kGridDenseMax <= gl::kGridGroup, "the sweep requests the dense chunk rounds as one group");

gl::RowLaunch gl::operator_rows(const gl_operator* op) {
    gl::RowLaunch r = {};
    r.layout = op->layout;
    r.w = op->w;
    r.wdt = op->store_w;
    r.order = nullptr;  // an ordered operator is renumbered: kernels index positions
    r.dd = op->dd;
    r.n = op->n;
    if (op->layout == gl::LAYOUT_GRID) {
        r.goffs = op->goffs;
        r.gwbase = op->gwbase;
        r.gcnt = op->gcnt;
        r.gdense = op->gdense;
        r.wheight = op->wheight;
        r.wwidth = op->wwidth;
        r.wtiles_x = op->wtiles_x;
        r.grid = op->nblocks;
        r.rows_per_block = gl::kGridThreads;
        r.idx64 = false;
        r.G = 1;
        return r;
    }
    if (op->layout == gl::LAYOUT_WINDOW) {
        r.wheight = op->wheight;
        r.wwidth = op->wwidth;
        r.wr = op->wr;
        r.wM = op->wM;
        r.wtiles_x = op->wtiles_x;
        r.grid = op->nblocks;
        r.rows_per_block = gl::kWinTX * gl::kWinTY;
        r.idx64 = false;
        r.G = 1;
        return r;
    }
    if (op->layout == gl::LAYOUT_TILE) {
        r.trp = (const int32_t*)op->rp;
        r.lcol = op->lcol;
        r.halo = op->halo;
        r.hp = op->hp;
        r.hmax = op->hmax;
        r.grid = op->nblocks;
        r.rows_per_block = gl::kTileRows;
        r.idx64 = false;
        r.G = gl::kTileG;
        return r;
    }
    r.rp = op->rp;
    r.col = op->col;
    r.idx64 = op->idx64;
    r.G = op->G;
    r.log2G = op->log2G;
    r.tiles = op->tiles;
    r.remap = op->remap;
    r.heavy = op->heavy;
    r.nheavy = op->nheavy;
    r.rows_per_block = (int64_t)(gl::kBlock >> op->log2G) * op->tiles;
    r.grid = (op->n + r.rows_per_block - 1) / r.rows_per_block;
    return r;
}

namespace {

gl::RowLaunch row_launch(const gl_operator* op) { return gl::operator_rows(op); }

// Storage pairs the kernels are compiled for: F64 weights with an F64 field;
// F32/BF16/F16 weights with an F32/BF16/F16 field.
bool pair_ok(gl_dtype w, gl_dtype u) {
    if (w == GL_F64 || u == GL_F64) return w == GL_F64 && u == GL_F64;
    return dtype_size(w) != 0 && dtype_size(u) != 0;
}

// The window layout stages K columns of V and of the accumulator over its
// tile's region in LDS.
gl_status window_fits(const gl_operator* op, int K, gl_dtype u) {
    if (op->layout == gl::LAYOUT_GRID) {
        const size_t need = (size_t)K * gl::kGridCells * (u == GL_F64 ? 8 : u == GL_F32 ? 4 : 2);
        if (need > gl::kGridLdsMax)
            return fail(GL_E_INVALID_ARG, "grid operator: K = " + std::to_string(K) + " columns need " +
                                              std::to_string(need) + " B of LDS per block (limit " +
                                              std::to_string(gl::kGridLdsMax) + "); use fewer columns per call");
        // the staging loads address a block's halo rows with 32-bit byte offsets
        const uint64_t rows = (uint64_t)gl::kGridHY * (uint64_t)op->wwidth * K * (u == GL_F64 ? 8 : u == GL_F32 ? 4 : 2);
        if (rows >= (1ull << 32))
            return fail(GL_E_INVALID_ARG, "grid operator: " + std::to_string(gl::kGridHY) + " image rows of " +
                                              std::to_string(K) + " columns exceed 4 GiB; use fewer columns per call");
        return GL_OK;
    }
    if (op->layout != gl::LAYOUT_WINDOW) return GL_OK;
    const size_t need = gl::window_lds_bytes(op, K, u == GL_F64 ? 8 : 4);
    if (need > gl::kWinLdsMax)
        return fail(GL_E_INVALID_ARG, "window operator: K = " + std::to_string(K) + " columns need " +
                                          std::to_string(need) + " B of LDS per block (limit " +
                                          std::to_string(gl::kWinLdsMax) + "); use fewer columns per call");
    return GL_OK;
}

hipError_t launch_sweep(gl_dtype u, int K, const gl::SweepLaunch& L, hipStream_t s) {
    switch (u) {
        case GL_F64: return gl::launch_sweep_f64(K, L, s);
        case GL_F32: return gl::launch_sweep_f32(K, L, s);
        case GL_BF16: return gl::launch_sweep_bf16(K, L, s);
        case GL_F16: return gl::launch_sweep_f16(K, L, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_laplacian(gl_dtype u, int K, const gl::RowLaunch& r, const void* x, void* y, hipStream_t s) {
    switch (u) {
        case GL_F64: return gl::launch_laplacian_f64(K, r, x, y, s);
        case GL_F32: return gl::launch_laplacian_f32(K, r, x, y, s);
        case GL_BF16: return gl::launch_laplacian_bf16(K, r, x, y, s);
        case GL_F16: return gl::launch_laplacian_f16(K, r, x, y, s);
    }
    return hipErrorInvalidValue;
}

hipError_t copy_bytes(const void* src, void* dst, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    const int64_t n16 = (int64_t)(bytes / 16);
    const int32_t tail = (int32_t)(bytes % 16);
    const int64_t work = n16 > tail ? n16 : tail;
    const unsigned grid = (unsigned)((work + 255) / 256);
    hipLaunchKernelGGL(gl::copy_bytes_kernel, dim3(grid), dim3(256), 0, s, (const gl::u32x4*)src,
                       (gl::u32x4*)dst, n16, (const uint8_t*)src + n16 * 16, (uint8_t*)dst + n16 * 16, tail);
    return hipGetLastError();
}

hipError_t fill_double(double* p, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gl::fill_double_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Coefficients of g_i = ga + gd dd_i + gl Lambda_i for every preconditioner of
// Section 3.1 (dd_i = 1 for L_s, d_i for L): step size infinite / finite k.
void precond_affine(int kind, const gl_params& p, double& ga, double& gd, double& gl_) {
    if (std::isinf(p.step_k)) {
        if (kind == GL_PC_DAMPED_JACOBI) { ga = 2.0 * p.c; gd = 2.0 * p.eps; gl_ = 2.0 * p.eta; }
        else if (kind == GL_PC_PERTURBED_JACOBI) { ga = p.c + p.delta0; gd = 2.0 * p.eps; gl_ = p.eta; }
        else { ga = p.eps * p.lambda_max + p.c + p.delta0; gd = 0.0; gl_ = p.eta; }
        return;
    }
    const double k = p.step_k;
    if (kind == GL_PC_DAMPED_JACOBI) { ga = 2.0 * (1.0 + k * p.c); gd = 2.0 * k * p.eps; gl_ = 2.0 * k * p.eta; }
    else if (kind == GL_PC_PERTURBED_JACOBI) { ga = 1.0 + k * p.c + p.delta0; gd = 2.0 * k * p.eps; gl_ = k * p.eta; }
    else { ga = 1.0 + k * (p.eps * p.lambda_max + p.c) + p.delta0; gd = 0.0; gl_ = k * p.eta; }
}

// g for unlabelled (lam = 0) and labelled (lam = 1) rows (Section 3.1).
double precond_g(int kind, double lam, const gl_params& p) {
    const double el = p.eta * lam;
    if (std::isinf(p.step_k)) {
        if (kind == GL_PC_DAMPED_JACOBI) return 2.0 * (p.eps + el + p.c);
        if (kind == GL_PC_PERTURBED_JACOBI) return 2.0 * p.eps + el + p.c + p.delta0;
        return p.eps * p.lambda_max + el + p.c + p.delta0;
    }
    const double k = p.step_k;
    if (kind == GL_PC_DAMPED_JACOBI) return 2.0 * (1.0 + k * (p.eps + p.c) + k * el);
    if (kind == GL_PC_PERTURBED_JACOBI) return (2.0 * k * p.eps + 1.0) + k * (el + p.c) + p.delta0;
    return 1.0 + k * (p.eps * p.lambda_max + el + p.c) + p.delta0;
}

gl_status check_params(const gl_params* p) {
    if (!p) return fail(GL_E_INVALID_ARG, "params is NULL");
    auto fin = [](double x) { return std::isfinite(x); };
    if (!fin(p->eps) || p->eps <= 0) return fail(GL_E_INVALID_ARG, "eps must be finite and > 0");
    if (!fin(p->c) || p->c <= 0) return fail(GL_E_INVALID_ARG, "c must be finite and > 0");
    if (!fin(p->eta) || p->eta < 0) return fail(GL_E_INVALID_ARG, "eta must be finite and >= 0");
    if (!fin(p->delta0) || p->delta0 < 0) return fail(GL_E_INVALID_ARG, "delta0 must be finite and >= 0");
    if (p->precond < GL_PC_DAMPED_JACOBI || p->precond > GL_PC_RICHARDSON)
        return fail(GL_E_INVALID_ARG, "unknown preconditioner");
    if (p->precond == GL_PC_RICHARDSON && (!fin(p->lambda_max) || p->lambda_max <= 0))
        return fail(GL_E_INVALID_ARG, "lambda_max must be finite and > 0 for the Richardson preconditioner");
    if (std::isnan(p->step_k) || p->step_k <= 0 || (std::isinf(p->step_k) && p->step_k < 0))
        return fail(GL_E_INVALID_ARG, "step_k must be > 0 or +INFINITY");
    if (p->outer_steps < 0) return fail(GL_E_INVALID_ARG, "outer_steps must be >= 0");
    if (p->inner_sweeps < 1) return fail(GL_E_INVALID_ARG, "inner_sweeps must be >= 1");
    if (p->reserved != 0) return fail(GL_E_INVALID_ARG, "reserved must be 0");
    return GL_OK;
}

template <typename TIN, typename TOUT, typename OffT>
void launch_normalize(gl_operator* op, const gl_graph* g, hipStream_t s) {
    const unsigned grid = (unsigned)((op->n + 1 + 255) / 256);
    hipLaunchKernelGGL((gl::normalize_kernel<TIN, TOUT, OffT>), dim3(grid), dim3(256), 0, s, op->n, g->row_ptr,
                       g->col_idx, static_cast<const TIN*>(g->weight), op->degree, static_cast<OffT*>(op->rp),
                       op->col, static_cast<TOUT*>(op->w), op->lap == GL_LAP_UNNORMALIZED ? 1 : 0);
}

template <typename TIN, typename TOUT>
void launch_normalize_idx(gl_operator* op, const gl_graph* g, hipStream_t s) {
    if (op->idx64) launch_normalize<TIN, TOUT, int64_t>(op, g, s);
    else launch_normalize<TIN, TOUT, int32_t>(op, g, s);
}

template <typename TIN>
void launch_normalize_out(gl_operator* op, const gl_graph* g, hipStream_t s) {
    switch (op->store_w) {
        case GL_F64: launch_normalize_idx<TIN, double>(op, g, s); break;
        case GL_F32: launch_normalize_idx<TIN, float>(op, g, s); break;
        case GL_BF16: launch_normalize_idx<TIN, gl::bf16>(op, g, s); break;
        case GL_F16: launch_normalize_idx<TIN, gl::f16>(op, g, s); break;
    }
}

void free_op(gl_operator* op) {
    if (!op) return;
    op->magic = 0;
    (void)hipFree(op->order);
    (void)hipFree(op->rp);
    (void)hipFree(op->col);
    (void)hipFree(op->lcol);
    (void)hipFree(op->halo);
    (void)hipFree(op->hp);
    (void)hipFree(op->w);
    (void)hipFree(op->degree);
    (void)hipFree(op->dd);
    (void)hipFree(op->goffs);
    (void)hipFree(op->gwbase);
    (void)hipFree(op->gcnt);
    (void)hipFree(op->heavy);
    delete op;
}

template <typename TIN, typename TOUT>
void launch_fill(gl_operator* op, const gl_graph* g, const int32_t* src, const int32_t* pos_of, hipStream_t s) {
    const unsigned grid = (unsigned)((op->n + 255) / 256);
    hipLaunchKernelGGL((gl::fill_layout_kernel<TIN, TOUT>), dim3(grid), dim3(256), 0, s, op->n,
                       (const int32_t*)op->rp, src, op->order, pos_of, g->col_idx,
                       static_cast<const TIN*>(g->weight), op->degree, static_cast<TOUT*>(op->w), op->col,
                       op->lap == GL_LAP_UNNORMALIZED ? 1 : 0);
}

// Unnormalized operator: diagonal d of L = D - W as the row sums of the stored
// weights (position order, accumulator type of the storage) and its maximum.
template <typename TW, typename A>
hipError_t launch_rowsum(gl_operator* op, hipStream_t s) {
    const unsigned grid = (unsigned)((op->n + 255) / 256);
    if (op->layout == gl::LAYOUT_DIRECT && op->idx64)
        hipLaunchKernelGGL((gl::rowsum_kernel<TW, int64_t, A>), dim3(grid), dim3(256), 0, s, op->n,
                           (const int64_t*)op->rp, (const TW*)op->w, (A*)op->dd);
    else
        hipLaunchKernelGGL((gl::rowsum_kernel<TW, int32_t, A>), dim3(grid), dim3(256), 0, s, op->n,
                           (const int32_t*)op->rp, (const TW*)op->w, (A*)op->dd);
    return hipGetLastError();
}

// Grid layout: the same row sums, taken over the input CSR rows (whose order
// is the storage order) with every weight rounded as stored.
template <typename TW, typename A>
hipError_t launch_grid_rowsum(gl_operator* op, const gl_graph* g, hipStream_t s) {
    const unsigned grid = (unsigned)((op->n + 255) / 256);
    if (g->weight_dtype == GL_F64)
        hipLaunchKernelGGL((gl::grid_rowsum_kernel<double, TW, A>), dim3(grid), dim3(256), 0, s, op->n, g->row_ptr,
                           (const double*)g->weight, (A*)op->dd);
    else
        hipLaunchKernelGGL((gl::grid_rowsum_kernel<float, TW, A>), dim3(grid), dim3(256), 0, s, op->n, g->row_ptr,
                           (const float*)g->weight, (A*)op->dd);
    return hipGetLastError();
}

gl_status finish_unnormalized(gl_operator* op, hipStream_t s, const gl_graph* g = nullptr) {
    if (op->lap != GL_LAP_UNNORMALIZED) return GL_OK;
    const size_t es = op->store_w == GL_F64 ? 8 : 4;
    if (hipMalloc(&op->dd, (size_t)op->n * es) != hipSuccess)
        return fail(GL_E_NOMEM, "device allocation for the operator failed");
    op->bytes += (size_t)op->n * es;
    hipError_t e = hipSuccess;
    if (op->layout == gl::LAYOUT_GRID) {
        switch (op->store_w) {
            case GL_F64: e = launch_grid_rowsum<double, double>(op, g, s); break;
            case GL_F32: e = launch_grid_rowsum<float, float>(op, g, s); break;
            case GL_BF16: e = launch_grid_rowsum<gl::bf16, float>(op, g, s); break;
            default: e = launch_grid_rowsum<gl::f16, float>(op, g, s); break;
        }
    } else {
        switch (op->store_w) {
            case GL_F64: e = launch_rowsum<double, double>(op, s); break;
            case GL_F32: e = launch_rowsum<float, float>(op, s); break;
            case GL_BF16: e = launch_rowsum<gl::bf16, float>(op, s); break;
            default: e = launch_rowsum<gl::f16, float>(op, s); break;
        }
    }
    std::vector<char> h((size_t)op->n * es);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), op->dd, h.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(GL_E_HIP, std::string("operator diagonal: ") + hipGetErrorString(e));
    double m = 0.0;
    for (int64_t i = 0; i < op->n; ++i) {
        const double v = es == 8 ? ((const double*)h.data())[i] : (double)((const float*)h.data())[i];
        if (!(v > 0.0) || !std::isfinite(v)) return fail(GL_E_BAD_GRAPH, "a stored row sums to a non-positive degree");
        m = v > m ? v : m;
    }
    op->dmax = m;
    return GL_OK;
}

template <typename TIN>
void launch_fill_out(gl_operator* op, const gl_graph* g, const int32_t* src, const int32_t* pos_of,
                     hipStream_t s) {
    switch (op->store_w) {
        case GL_F64: launch_fill<TIN, double>(op, g, src, pos_of, s); break;
        case GL_F32: launch_fill<TIN, float>(op, g, src, pos_of, s); break;
        case GL_BF16: launch_fill<TIN, gl::bf16>(op, g, src, pos_of, s); break;
        case GL_F16: launch_fill<TIN, gl::f16>(op, g, src, pos_of, s); break;
    }
}

// Rows of `row_bytes` between node order (caller's arrays) and position order
// (the renumbered operator's space): gather dst[p] = src[order[p]], or scatter
// dst[order[p]] = src[p].
hipError_t permute_rows(const gl_operator* op, size_t row_bytes, const void* src, void* dst, bool scatter,
                        hipStream_t s) {
    const int64_t n = op->n;
    auto go = [&](auto unit) -> hipError_t {
        typedef decltype(unit) W;
        const int32_t words = (int32_t)(row_bytes / sizeof(W));
        const unsigned grid = (unsigned)((n * words + 255) / 256);
        hipLaunchKernelGGL(gl::permute_rows_kernel<W>, dim3(grid), dim3(256), 0, s, n, words, op->order,
                           (const W*)src, (W*)dst, scatter ? 1 : 0);
        return hipGetLastError();
    };
    if (row_bytes % 8 == 0) return go(uint64_t{});
    if (row_bytes % 4 == 0) return go(uint32_t{});
    return go(uint16_t{});
}

template <typename T>
hipError_t upload(T** dst, const std::vector<T>& v, hipStream_t s) {
    const size_t bytes = v.size() * sizeof(T);
    hipError_t e = hipMalloc((void**)dst, bytes ? bytes : sizeof(T));
    if (e != hipSuccess) return e;
    if (bytes) e = hipMemcpyAsync(*dst, v.data(), bytes, hipMemcpyHostToDevice, s);
    return e;
}

// The heavy rows of a direct-layout operator (rows longer than 16 G, summed by
// workgroups of their own in the sweep), from host row offsets in the
// operator's row order.
template <typename OffT>
hipError_t set_heavy_rows(gl_operator* op, const OffT* h_rp, hipStream_t s) {
    const std::vector<int32_t> hv = gl::heavy_rows(op->n, h_rp, op->G);
    if (hv.empty()) return hipSuccess;
    hipError_t e = upload(&op->heavy, hv, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
        op->nheavy = (int32_t)hv.size();
        op->bytes += hv.size() * 4;
    }
    return e;
}

std::string bad_graph_message(int32_t flags, unsigned long long row) {
    std::string m = "bad graph (first offending row " + std::to_string(row) + "):";
    if (flags & gl::BAD_ROWPTR) m += " row_ptr not monotone or out of [0, nnz];";
    if (flags & gl::BAD_COL_RANGE) m += " column index out of [0, n);";
    if (flags & gl::BAD_COL_ORDER) m += " columns not strictly increasing within a row;";
    if (flags & gl::BAD_SELF_LOOP) m += " self-loop;";
    if (flags & gl::BAD_WEIGHT) m += " weight not finite and > 0;";
    if (flags & gl::BAD_ASYMMETRIC) m += " W not symmetric (pattern or weight);";
    if (flags & gl::BAD_DEGREE) m += " degree not finite and > 0;";
    return m;
}

}  // namespace

namespace {

// The solve behind gl_solve and gl_solve_noalloc (arguments as gl_solve).
gl_status solve_impl(const gl_operator* op, const gl_params* params, int32_t K, const int32_t* labels,
                     gl_dtype store_u, void* U, void* ws, size_t ws_bytes, double* stats, void* stream);

// Workspace of gl_solve_noalloc: a file-scope device array, one copy per GPU
// the library's code is loaded on, held until the process ends.  Host code
// never uses its name as an address: static_workspace() resolves the device
// address once per device (hipGetSymbolAddress, with that device current)
// and every launch takes that pointer.
constexpr size_t kStaticWorkspaceBytes = (size_t)128 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {

gl_status static_workspace(void** out) {
    int dev = -1;
    GL_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GL_E_INVALID_ARG, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        GL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "resolving the static workspace");
        if (!ptr || !aligned(ptr, 256)) return fail(GL_E_HIP, "static workspace address is not 256-byte aligned");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return GL_OK;
}

}  // namespace

extern "C" {

const char* gl_last_error(void) { return g_err.c_str(); }

const char* gl_version(void) { return "gl_dca 0.1 (gfx950)"; }

int64_t gl_stats_length(int32_t K, int32_t outer, int32_t sweeps) {
    if (K < 1 || outer < 0 || sweeps < 1) return 0;
    return (int64_t)(outer + 1) * K + (int64_t)outer * sweeps * K + 1;
}

gl_status gl_operator_create(const gl_graph* g, gl_dtype store_w, void* stream, gl_operator** out) {
    if (!g || !out) return fail(GL_E_INVALID_ARG, "graph and out must not be NULL");
    *out = nullptr;
    if (!g->row_ptr || !g->col_idx || !g->weight) return fail(GL_E_INVALID_ARG, "graph arrays must not be NULL");
    if (g->n < 2 || g->n > INT32_MAX) return fail(GL_E_INVALID_ARG, "n must lie in [2, 2^31 - 1]");
    if (g->nnz < 1 || g->nnz > ((int64_t)1 << 62)) return fail(GL_E_INVALID_ARG, "nnz must be >= 1");
    if (g->weight_dtype != GL_F64 && g->weight_dtype != GL_F32)
        return fail(GL_E_DTYPE, "input weights must be GL_F64 or GL_F32");
    if (dtype_size(store_w) == 0) return fail(GL_E_DTYPE, "unknown store_w");
    if (!(g->layout >= GL_LAYOUT_AUTO && g->layout <= GL_LAYOUT_TILE) && g->layout != GL_LAYOUT_GRID)
        return fail(GL_E_INVALID_ARG, "unknown layout");
    const bool grid_req = g->layout == GL_LAYOUT_GRID;
    if (grid_req) {
        if (g->grid_height < 1 || g->grid_width < 1 || (int64_t)g->grid_height * g->grid_width != g->n)
            return fail(GL_E_INVALID_ARG, "the grid layout needs grid_height * grid_width == n");
        if (g->grid_width >= (1 << 24))
            return fail(GL_E_INVALID_ARG, "the grid layout needs grid_width < 2^24");
        if (g->order) return fail(GL_E_INVALID_ARG, "the grid layout takes no order");
    }
    if (g->laplacian != GL_LAP_NORMALIZED && g->laplacian != GL_LAP_UNNORMALIZED)
        return fail(GL_E_INVALID_ARG, "unknown laplacian");
    const bool host_layout = g->order != nullptr || g->layout == GL_LAYOUT_TILE || grid_req;
    if (host_layout && g->nnz > (int64_t)INT32_MAX)
        return fail(GL_E_INVALID_ARG, "an order or the tile layout needs nnz < 2^31");
    hipStream_t s = (hipStream_t)stream;

    gl_operator* op = new gl_operator();
    op->n = g->n;
    op->nnz = g->nnz;
    op->stored = g->nnz;
    op->store_w = store_w;
    op->lap = g->laplacian;
    op->idx64 = g->nnz > (int64_t)INT32_MAX;
    if (hipGetDevice(&op->device) != hipSuccess) {
        delete op;
        return fail(GL_E_HIP, "hipGetDevice failed");
    }
    // geometry of the direct row kernels: the same function as the server's,
    // so a served solve sums every row and block in the order gl_solve does
    const gl::DirectGeom geom = gl::direct_geometry(g->n, g->nnz);
    op->G = geom.G;
    op->log2G = geom.log2G;
    op->tiles = geom.tiles;
    op->remap = 1;

    void* scratch = nullptr;  // [int32 flags][pad][u64 first_bad]
    if (hipMalloc((void**)&op->degree, (size_t)g->n * 8) != hipSuccess || hipMalloc(&scratch, 64) != hipSuccess) {
        (void)hipFree(scratch);
        free_op(op);
        return fail(GL_E_NOMEM, "device allocation for the operator failed");
    }
    int32_t* d_flags = (int32_t*)scratch;
    unsigned long long* d_first = (unsigned long long*)((char*)scratch + 8);
    struct {
        int32_t flags, pad;
        unsigned long long first;
    } init = {0, 0, ~0ull};
    int64_t ends[2] = {-1, -1};
    int32_t* d_src = nullptr;
    auto cleanup_fail = [&](gl_status st, const std::string& m) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(scratch);
        (void)hipFree(d_src);
        free_op(op);
        return fail(st, m);
    };
    if (hipMemcpyAsync(scratch, &init, sizeof(init), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(&ends[0], g->row_ptr, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&ends[1], g->row_ptr + g->n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup_fail(GL_E_HIP, "copying row_ptr ends failed");
    if (ends[0] != 0 || ends[1] != g->nnz)
        return cleanup_fail(GL_E_BAD_GRAPH, "bad graph: row_ptr[0] must be 0 and row_ptr[n] must equal nnz");

    const unsigned grid = (unsigned)((g->n + 255) / 256);
    if (g->weight_dtype == GL_F64) {
        hipLaunchKernelGGL(gl::validate_kernel<double>, dim3(grid), dim3(256), 0, s, g->n, g->nnz, g->row_ptr,
                           g->col_idx, (const double*)g->weight, d_flags, d_first);
    } else {
        hipLaunchKernelGGL(gl::validate_kernel<float>, dim3(grid), dim3(256), 0, s, g->n, g->nnz, g->row_ptr,
                           g->col_idx, (const float*)g->weight, d_flags, d_first);
    }
    if (hipGetLastError() != hipSuccess) return cleanup_fail(GL_E_HIP, "validate launch failed");
    if (hipMemcpyAsync(&init, scratch, sizeof(init), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup_fail(GL_E_HIP, "graph validation failed");
    if (init.flags) return cleanup_fail(GL_E_BAD_GRAPH, bad_graph_message(init.flags, init.first));

    if (g->weight_dtype == GL_F64) {
        hipLaunchKernelGGL(gl::degree_kernel<double>, dim3(grid), dim3(256), 0, s, g->n, g->row_ptr,
                           (const double*)g->weight, op->degree, d_flags, d_first);
    } else {
        hipLaunchKernelGGL(gl::degree_kernel<float>, dim3(grid), dim3(256), 0, s, g->n, g->row_ptr,
                           (const float*)g->weight, op->degree, d_flags, d_first);
    }
    if (hipMemcpyAsync(&init, scratch, sizeof(init), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup_fail(GL_E_HIP, "degree computation failed");
    if (init.flags) return cleanup_fail(GL_E_BAD_GRAPH, bad_graph_message(init.flags, init.first));

    const size_t sw = dtype_size(store_w);
    if (grid_req) {
        // grid layout, built on the device from the CSR graph and the degrees
        const int32_t H = g->grid_height, W = g->grid_width;
        const int32_t tiles_x = (W + gl::kGridTX - 1) / gl::kGridTX;
        const int64_t ntiles = (int64_t)tiles_x * ((H + gl::kGridTY - 1) / gl::kGridTY);
        const int64_t nseg = ntiles * gl::kGridTY;
        op->layout = gl::LAYOUT_GRID;
        op->idx64 = false;
        op->G = 1;
        op->wheight = H;
        op->wwidth = W;
        op->wtiles_x = tiles_x;
        op->nblocks = ntiles;
        int64_t* seg = nullptr;  // [nseg] rest chunks per segment, [nseg] their offsets, [1] total
        struct {
            int32_t flags, mincnt;
            unsigned long long first;
        } st = {0, 1 << 30, ~0ull};
        int64_t rest = 0;
        auto grid_fail = [&](gl_status code, const std::string& m) {
            (void)hipStreamSynchronize(s);
            (void)hipFree(seg);
            return cleanup_fail(code, m);
        };
        if (hipMalloc((void**)&op->gcnt, (size_t)g->n) != hipSuccess ||
            hipMalloc((void**)&op->gwbase, (size_t)H * tiles_x * 8) != hipSuccess ||
            hipMalloc((void**)&seg, (size_t)(2 * nseg + 1) * 8) != hipSuccess)
            return grid_fail(GL_E_NOMEM, "device allocation for the operator failed");
        int32_t* d_st = (int32_t*)scratch;  // flags, mincnt, first bad pixel
        if (hipMemcpyAsync(scratch, &st, sizeof(st), hipMemcpyHostToDevice, s) != hipSuccess)
            return grid_fail(GL_E_HIP, "grid layout: copy failed");
        hipLaunchKernelGGL(gl::grid_count_kernel, dim3(grid), dim3(256), 0, s, g->n, W, g->row_ptr, g->col_idx,
                           op->gcnt, d_st, (unsigned long long*)((char*)scratch + 8), d_st + 1);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&st, scratch, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return grid_fail(GL_E_HIP, "grid layout: chunk counts failed");
        if (st.flags)
            return grid_fail(GL_E_INVALID_ARG, "grid layout: pixel " + std::to_string(st.first) +
                                                   " has an edge more than 7 rows or columns away");
        const int32_t dense = std::min(st.mincnt, gl::kGridDenseMax);
        hipLaunchKernelGGL(gl::grid_segrest_kernel, dim3((unsigned)((nseg + 255) / 256)), dim3(256), 0, s, nseg, H,
                           W, tiles_x, op->gcnt, dense, seg);
        hipLaunchKernelGGL(gl::scan_exclusive_kernel, dim3(1), dim3(1024), 0, s, seg, seg + nseg, nseg,
                           seg + 2 * nseg);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(&rest, seg + 2 * nseg, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return grid_fail(GL_E_HIP, "grid layout: segment offsets failed");
        const int64_t chunks = ntiles * dense * gl::kGridThreads + rest;
        op->gchunks = chunks;
        op->gdense = dense;
        op->stored = chunks * gl::kGridChunk;
        if (hipMalloc((void**)&op->goffs, (size_t)chunks * 8) != hipSuccess ||
            hipMalloc(&op->w, (size_t)op->stored * sw + 64) != hipSuccess)
            return grid_fail(GL_E_NOMEM, "device allocation for the operator failed");
        op->bytes = (size_t)op->stored * sw + (size_t)chunks * 8 + (size_t)H * tiles_x * 8 + (size_t)g->n +
                    (size_t)g->n * 8;
        const int raw = op->lap == GL_LAP_UNNORMALIZED ? 1 : 0;
        const dim3 eg((unsigned)((nseg + 3) / 4)), eb(256);
        auto emit = [&](auto tin, auto tout) {
            typedef decltype(tin) TIN;
            typedef decltype(tout) TOUT;
            hipLaunchKernelGGL((gl::grid_emit_kernel<TIN, TOUT>), eg, eb, 0, s, nseg, H, W, tiles_x, dense,
                               g->row_ptr, g->col_idx, (const TIN*)g->weight, op->degree, raw, op->gcnt, seg + nseg,
                               ntiles * dense * gl::kGridThreads, op->goffs, (TOUT*)op->w, op->gwbase);
        };
        auto emit_in = [&](auto tin) {
            switch (store_w) {
                case GL_F64: emit(tin, double{}); break;
                case GL_F32: emit(tin, float{}); break;
                case GL_BF16: emit(tin, gl::bf16{}); break;
                default: emit(tin, gl::f16{}); break;
            }
        };
        if (g->weight_dtype == GL_F64) emit_in(double{});
        else emit_in(float{});
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return grid_fail(GL_E_HIP, "grid layout: chunk emission failed");
        (void)hipFree(seg);
        seg = nullptr;
        const gl_status su = finish_unnormalized(op, s, g);
        if (su != GL_OK) {
            const std::string m = gl_last_error();
            return cleanup_fail(su, m);
        }
        (void)hipFree(scratch);
        *out = op;
        return GL_OK;
    }
    if (!host_layout) {
        // direct layout in natural order, built on the device
        const size_t rp_bytes = (size_t)(g->n + 1) * (op->idx64 ? 8 : 4);
        if (hipMalloc(&op->rp, rp_bytes) != hipSuccess || hipMalloc((void**)&op->col, (size_t)g->nnz * 4) != hipSuccess ||
            hipMalloc(&op->w, (size_t)g->nnz * sw) != hipSuccess)
            return cleanup_fail(GL_E_NOMEM, "device allocation for the operator failed");
        op->bytes = rp_bytes + (size_t)g->nnz * (4 + sw) + (size_t)g->n * 8;
        if (g->weight_dtype == GL_F64) launch_normalize_out<double>(op, g, s);
        else launch_normalize_out<float>(op, g, s);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return cleanup_fail(GL_E_HIP, "weight normalization failed");
        {
            std::vector<int64_t> h_rp(g->n + 1);
            if (hipMemcpy(h_rp.data(), g->row_ptr, h_rp.size() * 8, hipMemcpyDeviceToHost) != hipSuccess ||
                set_heavy_rows(op, h_rp.data(), s) != hipSuccess)
                return cleanup_fail(GL_E_HIP, "heavy-row list failed");
        }
        const gl_status su = finish_unnormalized(op, s);
        if (su != GL_OK) {
            const std::string m = gl_last_error();
            return cleanup_fail(su, m);
        }
        (void)hipFree(scratch);
        *out = op;
        return GL_OK;
    }

    // processing order and/or tile layout: index layout built on the device
    gl::DeviceLayout L;
    std::string err;
    const int32_t halo_limit = store_w == GL_F64 ? 480 : gl::kTileHaloMax;
    const gl::LayoutStatus ls = gl::build_layout(g->n, g->nnz, g->row_ptr, g->col_idx, g->order,
                                                 g->layout != GL_LAYOUT_DIRECT, g->layout == GL_LAYOUT_TILE,
                                                 halo_limit, s, L, err);
    if (ls != gl::kLayoutOk) return cleanup_fail(ls == gl::kLayoutInvalid ? GL_E_INVALID_ARG : GL_E_HIP, err);
    op->layout = L.layout == 1 ? gl::LAYOUT_TILE : gl::LAYOUT_DIRECT;
    op->idx64 = false;
    op->stored = L.stored;
    op->rp = L.rp;
    d_src = L.src;
    int32_t* d_pos_of = L.pos_of;
    if (op->layout == gl::LAYOUT_TILE) {
        op->lcol = L.lcol;
        op->halo = L.halo;
        op->hp = L.hp;
        op->hmax = L.hmax;
        op->halo_total = L.halo_total;
        op->nblocks = L.nblocks;
    }
    hipError_t e = hipSuccess;
    if (g->order) {
        e = hipMalloc((void**)&op->order, (size_t)g->n * 4);
        if (e == hipSuccess) e = hipMemcpyAsync(op->order, g->order, (size_t)g->n * 4, hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess && op->layout == gl::LAYOUT_DIRECT)
        e = hipMalloc((void**)&op->col, (size_t)op->stored * 4 + 4);
    if (e == hipSuccess) e = hipMalloc(&op->w, (size_t)op->stored * sw + 16);
    if (e != hipSuccess) {
        (void)hipFree(d_pos_of);
        return cleanup_fail(GL_E_NOMEM, "device allocation for the operator failed");
    }
    op->bytes = (size_t)(g->n + 1) * 4 + (size_t)op->stored * sw + (size_t)g->n * 8 +
                (g->order ? (size_t)g->n * 4 : 0) +
                (op->layout == gl::LAYOUT_TILE ? (size_t)op->stored * 2 + (size_t)op->halo_total * 4 +
                                                     (size_t)(op->nblocks + 1) * 4
                                               : (size_t)op->stored * 4);
    // the fill reads columns through pos_of only on the direct layout (the tile
    // layout's halo already names positions)
    if (op->layout == gl::LAYOUT_TILE) {
        (void)hipFree(d_pos_of);
        d_pos_of = nullptr;
    }
    if (g->weight_dtype == GL_F64) launch_fill_out<double>(op, g, d_src, d_pos_of, s);
    else launch_fill_out<float>(op, g, d_src, d_pos_of, s);
    const bool fill_ok = hipGetLastError() == hipSuccess && hipStreamSynchronize(s) == hipSuccess;
    (void)hipFree(d_pos_of);
    if (!fill_ok) return cleanup_fail(GL_E_HIP, "weight normalization failed");
    if (op->layout == gl::LAYOUT_DIRECT) {
        std::vector<int32_t> h_srp(g->n + 1);
        if (hipMemcpy(h_srp.data(), op->rp, h_srp.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            set_heavy_rows(op, h_srp.data(), s) != hipSuccess)
            return cleanup_fail(GL_E_HIP, "heavy-row list failed");
    }
    const gl_status su = finish_unnormalized(op, s);
    if (su != GL_OK) {
        const std::string m = gl_last_error();
        return cleanup_fail(su, m);
    }
    (void)hipFree(d_src);
    (void)hipFree(scratch);
    *out = op;
    return GL_OK;
}

gl_status gl_params_validate(const gl_params* params) { return check_params(params); }

gl_status gl_operator_destroy(gl_operator* op) {
    if (!op) return GL_OK;
    if (!gl::valid(op)) return fail(GL_E_INVALID_ARG, "not an operator handle");
    free_op(op);
    return GL_OK;
}

gl_status gl_operator_info(const gl_operator* op, int64_t* n, int64_t* nnz, gl_dtype* store_w,
                           int32_t* lanes_per_row, size_t* device_bytes) {
    if (!gl::valid(op)) return fail(GL_E_INVALID_ARG, "operator is NULL or not an operator handle");
    if (n) *n = op->n;
    if (nnz) *nnz = op->nnz;
    if (store_w) *store_w = op->store_w;
    if (lanes_per_row) *lanes_per_row = op->G;
    if (device_bytes) *device_bytes = op->bytes;
    return GL_OK;
}

gl_status gl_operator_layout(const gl_operator* op, int32_t* layout, int64_t* stored, int32_t* halo_max,
                             int64_t* halo_total, int64_t* stream_bytes) {
    if (!gl::valid(op)) return fail(GL_E_INVALID_ARG, "operator is NULL or not an operator handle");
    const bool tile = op->layout == gl::LAYOUT_TILE;
    if (op->layout == gl::LAYOUT_GRID) {
        if (layout) *layout = GL_LAYOUT_GRID;
        if (stored) *stored = op->stored;
        if (halo_max) *halo_max = gl::kGridCells;
        if (halo_total) *halo_total = (int64_t)gl::kGridCells * op->nblocks;
        if (stream_bytes)
            *stream_bytes = op->gchunks * (8 + 8 * (int64_t)dtype_size(op->store_w)) + op->n +
                            (int64_t)op->wheight * op->wtiles_x * 8 +
                            (op->dd ? op->n * (op->store_w == GL_F64 ? 8 : 4) : 0);
        return GL_OK;
    }
    if (op->layout == gl::LAYOUT_WINDOW) {
        const int64_t cells = gl::window_region(op->wr);
        if (layout) *layout = GL_LAYOUT_WINDOW;
        if (stored) *stored = op->stored;
        if (halo_max) *halo_max = (int32_t)cells;
        if (halo_total) *halo_total = cells * op->nblocks;
        if (stream_bytes)
            *stream_bytes = op->stored * (int64_t)dtype_size(op->store_w) +
                            (op->dd ? op->n * (op->store_w == GL_F64 ? 8 : 4) : 0);
        return GL_OK;
    }
    if (layout) *layout = tile ? GL_LAYOUT_TILE : GL_LAYOUT_DIRECT;
    if (stored) *stored = op->stored;
    if (halo_max) *halo_max = tile ? op->hmax : 0;
    if (halo_total) *halo_total = tile ? op->halo_total : 0;
    if (stream_bytes) {
        const int64_t rp = (op->n + 1) * (op->idx64 ? 8 : 4);
        const int64_t idx = tile ? op->stored * 2 + op->halo_total * 4 + (op->nblocks + 1) * 4 : op->stored * 4;
        *stream_bytes = rp + idx + op->stored * (int64_t)dtype_size(op->store_w) +
                        (op->dd ? op->n * (op->store_w == GL_F64 ? 8 : 4) : 0);
    }
    return GL_OK;
}

gl_status gl_laplacian_apply(const gl_operator* op, int32_t K, gl_dtype dtype, const void* X, void* Y,
                             void* stream) {
    if (!gl::valid(op) || !X || !Y) return fail(GL_E_INVALID_ARG, "operator (a live operator handle), X and Y must not be NULL");
    if (K < 1 || K > 16) return fail(GL_E_INVALID_ARG, "K must lie in [1, 16]");
    if (!pair_ok(op->store_w, dtype)) return fail(GL_E_DTYPE, "unsupported (weight, field) storage pair");
    if (!aligned(X, 16) || !aligned(Y, 16)) return fail(GL_E_INVALID_ARG, "X and Y must be 16-byte aligned");
    if (window_fits(op, K, dtype) != GL_OK) return GL_E_INVALID_ARG;
    const size_t bytes = (size_t)op->n * K * dtype_size(dtype);
    const char *x = (const char*)X, *y = (const char*)Y;
    if (x < y + bytes && y < x + bytes) return fail(GL_E_INVALID_ARG, "X and Y overlap");
    hipStream_t s = (hipStream_t)stream;
    if (op->layout == gl::LAYOUT_WINDOW) {
        // region sums of the window product (stream-ordered scratch)
        gl::RowLaunch r = row_launch(op);
        GL_HIP(hipMallocAsync(&r.wpart, gl::window_part_bytes(op, K, dtype == GL_F64 ? 8 : 4), s),
               "laplacian scratch");
        const hipError_t e = launch_laplacian(dtype, K, r, X, Y, s);
        const hipError_t ef = hipFreeAsync(r.wpart, s);
        GL_HIP(e, "laplacian launch");
        GL_HIP(ef, "laplacian scratch");
        return GL_OK;
    }
    if (!op->order) {
        GL_HIP(launch_laplacian(dtype, K, row_launch(op), X, Y, s), "laplacian launch");
        return GL_OK;
    }
    // renumbered operator: X -> position order, apply, scatter back (stream-ordered scratch)
    const size_t row = (size_t)K * dtype_size(dtype);
    void* tmp = nullptr;
    GL_HIP(hipMallocAsync(&tmp, 2 * align256(bytes), s), "laplacian scratch");
    char* tx = (char*)tmp;
    char* ty = tx + align256(bytes);
    hipError_t e = permute_rows(op, row, X, tx, false, s);
    if (e == hipSuccess) e = launch_laplacian(dtype, K, row_launch(op), tx, ty, s);
    if (e == hipSuccess) e = permute_rows(op, row, ty, Y, true, s);
    const hipError_t ef = hipFreeAsync(tmp, s);
    GL_HIP(e, "laplacian launch");
    GL_HIP(ef, "laplacian scratch");
    return GL_OK;
}

gl_status gl_power_workspace_size(const gl_operator* op, size_t* bytes) {
    if (!gl::valid(op) || !bytes) return fail(GL_E_INVALID_ARG, "operator (a live operator handle) and bytes must not be NULL");
    const gl::RowLaunch r = row_launch(op);
    *bytes = (op->order ? 3 : 2) * align256((size_t)op->n * 4) + align256((size_t)2 * r.grid * 4) + 256 +
             align256(gl::window_part_bytes(op, 1, 4));
    return GL_OK;
}

gl_status gl_power_max_eig(const gl_operator* op, int32_t iters, const float* x0, void* ws, size_t ws_bytes,
                           double* rayleigh, double* lambda_hat, void* stream) {
    if (!gl::valid(op) || !x0 || !ws || !rayleigh || !lambda_hat)
        return fail(GL_E_INVALID_ARG, "operator, x0, workspace and outputs must not be NULL");
    if (iters < 0) return fail(GL_E_INVALID_ARG, "iters must be >= 0");
    if (op->store_w == GL_F64) return fail(GL_E_DTYPE, "the power method runs on F32/BF16/F16 weights");
    if (!aligned(ws, 256)) return fail(GL_E_INVALID_ARG, "workspace must be 256-byte aligned");
    size_t need = 0;
    gl_power_workspace_size(op, &need);
    if (ws_bytes < need) return fail(GL_E_INVALID_ARG, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    const gl::RowLaunch r = row_launch(op);
    char* base = (char*)ws;
    const size_t vec = align256((size_t)op->n * 4);
    float* buf[2] = {(float*)base, (float*)(base + vec)};
    float* partials = (float*)(base + (op->order ? 3 : 2) * vec);
    char* tail = (char*)partials + align256((size_t)2 * r.grid * 4);
    float* scale = (float*)tail;
    double* sums = (double*)(tail + 64);
    float* wpart = (float*)(tail + 256);  // window layout: region sums of one product

    auto pass = [&](const float* x, float* y, int mode, const float* sc) -> hipError_t {
        if (op->layout == gl::LAYOUT_WINDOW) return gl::launch_window_power(op, x, y, mode, sc, partials, wpart, s);
        if (op->layout == gl::LAYOUT_GRID) {
            gl::GridPowerArgs a;
            a.op.w = op->w;
            a.op.offs = op->goffs;
            a.op.wbase = op->gwbase;
            a.op.cnt = op->gcnt;
            a.op.n = op->n;
            a.op.dense = op->gdense;
            a.op.height = op->wheight;
            a.op.width = op->wwidth;
            a.op.tiles_x = op->wtiles_x;
            a.x = x;
            a.y = y;
            a.scale = sc;
            a.partials = partials;
            a.dd = (const float*)op->dd;
            a.mode = mode;
            const size_t lds = (size_t)gl::kGridCells * 4;
            const dim3 gg((unsigned)r.grid), bb(gl::kGridThreads);
            switch (op->store_w) {
                case GL_F32: hipLaunchKernelGGL(gl::grid_power_kernel<float>, gg, bb, lds, s, a); break;
                case GL_BF16: hipLaunchKernelGGL(gl::grid_power_kernel<gl::bf16>, gg, bb, lds, s, a); break;
                case GL_F16: hipLaunchKernelGGL(gl::grid_power_kernel<gl::f16>, gg, bb, lds, s, a); break;
                default: return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
        if (op->layout == gl::LAYOUT_TILE) {
            gl::TilePowerArgs a;
            a.op.rp = (const int32_t*)op->rp;
            a.op.lcol = op->lcol;
            a.op.w = op->w;
            a.op.halo = op->halo;
            a.op.hp = op->hp;
            a.op.order = nullptr;
            a.op.n = op->n;
            a.dd = (const float*)op->dd;
            a.x = x;
            a.y = y;
            a.scale = sc;
            a.partials = partials;
            a.mode = mode;
            const size_t lds = (size_t)op->hmax * 4;
            switch (op->store_w) {
                case GL_F32:
                    hipLaunchKernelGGL(gl::tile_power_kernel<float>, dim3((unsigned)r.grid), dim3(256), lds, s, a);
                    break;
                case GL_BF16:
                    hipLaunchKernelGGL(gl::tile_power_kernel<gl::bf16>, dim3((unsigned)r.grid), dim3(256), lds, s, a);
                    break;
                case GL_F16:
                    hipLaunchKernelGGL(gl::tile_power_kernel<gl::f16>, dim3((unsigned)r.grid), dim3(256), lds, s, a);
                    break;
                default:
                    return hipErrorInvalidValue;
            }
            return hipGetLastError();
        }
        const gl::RowGeom geo{r.n, r.rows_per_block, r.G, r.log2G, r.tiles, r.remap};
        switch (op->store_w) {
#define GL_POW(T)                                                                                   \
    if (op->idx64) {                                                                                \
        gl::PowerArgs<T, int64_t> a{(const int64_t*)op->rp, op->col, (const T*)op->w, x, y, sc, partials, nullptr, (const float*)op->dd, geo, mode}; \
        hipLaunchKernelGGL((gl::power_kernel<T, int64_t>), dim3((unsigned)r.grid), dim3(256), 0, s, a); \
    } else {                                                                                        \
        gl::PowerArgs<T, int32_t> a{(const int32_t*)op->rp, op->col, (const T*)op->w, x, y, sc, partials, nullptr, (const float*)op->dd, geo, mode}; \
        hipLaunchKernelGGL((gl::power_kernel<T, int32_t>), dim3((unsigned)r.grid), dim3(256), 0, s, a); \
    }
            case GL_F32: GL_POW(float) break;
            case GL_BF16: GL_POW(gl::bf16) break;
            case GL_F16: GL_POW(gl::f16) break;
            default: return hipErrorInvalidValue;
#undef GL_POW
        }
        return hipGetLastError();
    };
    auto finalize = [&](int scale_stat) -> hipError_t {
        hipLaunchKernelGGL(gl::power_finalize_kernel, dim3(1), dim3(256), 0, s, partials, r.grid, scale_stat,
                           scale, sums);
        return hipGetLastError();
    };
    if (op->order) {
        // renumbered operator: iterate on x0 in position order
        float* xp = (float*)(base + 2 * vec);
        GL_HIP(permute_rows(op, 4, x0, xp, false, s), "power permute");
        x0 = xp;
    }
    // s_0 = 1/|x0| from the mode-1 pass over x0
    GL_HIP(pass(x0, nullptr, 1, nullptr), "power launch");
    GL_HIP(finalize(1), "power finalize");
    const float* x = x0;
    for (int it = 0; it < iters; ++it) {
        float* y = buf[it & 1];
        GL_HIP(pass(x, y, 0, scale), "power launch");
        GL_HIP(finalize(0), "power finalize");
        x = y;
    }
    GL_HIP(pass(x, nullptr, 1, nullptr), "power launch");
    GL_HIP(finalize(1), "power finalize");
    double h[2] = {0, 0};
    GL_HIP(hipMemcpyAsync(h, sums, sizeof(h), hipMemcpyDeviceToHost, s), "copy power sums");
    GL_HIP(hipStreamSynchronize(s), "power method");
    if (!(h[1] > 0) || !std::isfinite(h[0]) || !std::isfinite(h[1]))
        return fail(GL_E_NONFINITE, "power method: x0 is zero or the iteration is not finite");
    *rayleigh = h[0] / h[1];
    *lambda_hat = std::fmin(2.0 * op->dmax, 1.01 * *rayleigh);  // 2D >= L, 2I >= L_s (Prop. 3)
    return GL_OK;
}

gl_status gl_solve_workspace_size(const gl_operator* op, int32_t K, gl_dtype store_u, size_t* bytes) {
    if (!gl::valid(op) || !bytes) return fail(GL_E_INVALID_ARG, "operator (a live operator handle) and bytes must not be NULL");
    if (K < 1 || K > 16) return fail(GL_E_INVALID_ARG, "K must lie in [1, 16]");
    if (!pair_ok(op->store_w, store_u)) return fail(GL_E_DTYPE, "unsupported (weight, field) storage pair");
    const gl::RowLaunch r = row_launch(op);
    const size_t field = align256((size_t)op->n * K * dtype_size(store_u));
    const size_t acc = store_u == GL_F64 ? 8 : 4;
    // ordered operators keep all three field buffers and the labels in position order
    // the block partial sums of up to kStatGroup sweeps wait for one reduction
    // the window layout's region sums of one product
    *bytes = (op->order ? 3 * field + align256((size_t)op->n * 4) : 2 * field) +
             (size_t)gl::kStatGroup * align256((size_t)2 * K * gl::sweep_grid(r) * acc) +
             align256(gl::window_part_bytes(op, K, acc));
    return GL_OK;
}

gl_status gl_solve(const gl_operator* op, const gl_params* params, int32_t K, const int32_t* labels,
                   gl_dtype store_u, void* U, void* ws, size_t ws_bytes, double* stats, void* stream) {
    return solve_impl(op, params, K, labels, store_u, U, ws, ws_bytes, stats, stream);
}

gl_status gl_solve_noalloc(const gl_operator* op, const gl_params* params, int32_t K, const int32_t* labels,
                           gl_dtype store_u, void* U, double* stats, void* stream) {
    if (!gl::valid(op) || !labels || !U)
        return fail(GL_E_INVALID_ARG, "operator (a live operator handle), labels and U must not be NULL");
    if (K < 1 || K > 16) return fail(GL_E_INVALID_ARG, "K must lie in [1, 16]");
    if (!pair_ok(op->store_w, store_u)) return fail(GL_E_DTYPE, "unsupported (weight, field) storage pair");
    size_t need = 0;
    const gl_status sz = gl_solve_workspace_size(op, K, store_u, &need);
    if (sz != GL_OK) return sz;
    if (need > kStaticWorkspaceBytes)
        return fail(GL_E_INVALID_ARG, "this solve needs " + std::to_string(need) +
                                          " bytes of workspace, more than the " +
                                          std::to_string(kStaticWorkspaceBytes) +
                                          "-byte static workspace of gl_solve_noalloc; use gl_solve");
    void* ws = nullptr;
    const gl_status st = static_workspace(&ws);
    if (st != GL_OK) return st;
    return solve_impl(op, params, K, labels, store_u, U, ws, kStaticWorkspaceBytes, stats, stream);
}

}  // extern "C"

namespace {

gl_status solve_impl(const gl_operator* op, const gl_params* params, int32_t K, const int32_t* labels,
                     gl_dtype store_u, void* U, void* ws, size_t ws_bytes, double* stats, void* stream) {
    if (!gl::valid(op) || !labels || !U || !ws) return fail(GL_E_INVALID_ARG, "operator (a live operator handle), labels, U and workspace must not be NULL");
    gl_status st = check_params(params);
    if (st != GL_OK) return st;
    if (K < 1 || K > 16) return fail(GL_E_INVALID_ARG, "K must lie in [1, 16]");
    if (!pair_ok(op->store_w, store_u)) return fail(GL_E_DTYPE, "unsupported (weight, field) storage pair");
    if (!aligned(U, 16)) return fail(GL_E_INVALID_ARG, "U must be 16-byte aligned");
    if (!aligned(ws, 256)) return fail(GL_E_INVALID_ARG, "workspace must be 256-byte aligned");
    if (window_fits(op, K, store_u) != GL_OK) return GL_E_INVALID_ARG;
    if (stats && !aligned(stats, 8)) return fail(GL_E_INVALID_ARG, "stats must be 8-byte aligned");
    size_t need = 0;
    gl_solve_workspace_size(op, K, store_u, &need);
    if (ws_bytes < need) return fail(GL_E_INVALID_ARG, "workspace too small");
    const gl_params& p = *params;
    const int T = p.outer_steps, m = p.inner_sweeps;
    hipStream_t s = (hipStream_t)stream;

    const size_t field = align256((size_t)op->n * K * dtype_size(store_u));
    const size_t row = (size_t)K * dtype_size(store_u);
    char* bufs[3] = {(char*)U, (char*)ws, (char*)ws + field};
    void* partials = (char*)ws + 2 * field;
    if (op->order) {
        // renumbered operator: u^0 and the labels move to position order once
        bufs[0] = (char*)ws;
        bufs[1] = (char*)ws + field;
        bufs[2] = (char*)ws + 2 * field;
        int32_t* lab_pos = (int32_t*)((char*)ws + 3 * field);
        partials = (char*)lab_pos + align256((size_t)op->n * 4);
        GL_HIP(permute_rows(op, row, U, bufs[0], false, s), "permute u0");
        GL_HIP(permute_rows(op, 4, labels, lab_pos, false, s), "permute labels");
        labels = lab_pos;
    }

    gl::SweepLaunch L;
    L.r = row_launch(op);
    // the window layout's region sums sit at the end of the workspace
    L.r.wpart = (char*)ws + (need - align256(gl::window_part_bytes(op, K, store_u == GL_F64 ? 8 : 4)));
    L.labels = labels;
    L.partials = stats ? partials : nullptr;
    const double g0 = precond_g(p.precond, 0.0, p), g1 = precond_g(p.precond, 1.0, p);
    const bool inf_k = std::isinf(p.step_k);
    double ga = 0, gd = 0, gll = 0;
    precond_affine(p.precond, p, ga, gd, gll);
    const double coef[14] = {p.eps, p.c, p.eta, 1.0 / p.eps, 0.5 * p.eps, 0.25 / p.eps, 0.5 * p.eta,
                             1.0 / g0, 1.0 / g1, inf_k ? 0.0 : 1.0, inf_k ? 1.0 : p.step_k, ga, gd, gll};
    std::memcpy(L.coef, coef, sizeof(coef));

    const int64_t slen = gl_stats_length(K, T, m);
    double* flag = stats ? stats + slen - 1 : nullptr;
    double* res_base = stats ? stats + (int64_t)(T + 1) * K : nullptr;
    if (stats) GL_HIP(fill_double(stats, slen, 0.0, s), "stats init");

    // The statistics of each sweep are reduced later, kStatGroup sweeps per
    // launch: sweep j of a group writes its block partial sums to set j.
    const size_t acc = store_u == GL_F64 ? 8 : 4;
    const size_t set_bytes = align256((size_t)2 * K * gl::sweep_grid(L.r) * acc);
    gl::StatGroup group = {};
    int pending = 0;
    auto flush = [&]() -> hipError_t {
        if (!stats || pending == 0) return hipSuccess;
        const dim3 grid((unsigned)(2 * K), (unsigned)pending);
        const int64_t stride = (int64_t)(set_bytes / acc);
        if (store_u == GL_F64) {
            hipLaunchKernelGGL(gl::finalize_group_kernel<double>, grid, dim3(256), 0, s,
                               (const double*)partials, gl::sweep_grid(L.r), stride, K, group, flag);
        } else {
            hipLaunchKernelGGL(gl::finalize_group_kernel<float>, grid, dim3(256), 0, s,
                               (const float*)partials, gl::sweep_grid(L.r), stride, K, group, flag);
        }
        pending = 0;
        group = {};
        return hipGetLastError();
    };
    // before a sweep: point it at the next free set (reducing a full group first)
    auto next_set = [&](double* e_dst, double* r_dst) -> hipError_t {
        if (!stats) return hipSuccess;
        if (pending == gl::kStatGroup) {
            hipError_t e = flush();
            if (e != hipSuccess) return e;
        }
        L.partials = (char*)partials + (size_t)pending * set_bytes;
        group.energy_dst[pending] = e_dst;
        group.res_dst[pending] = r_dst;
        ++pending;
        return hipSuccess;
    };

    int cur = 0;  // buffer holding u^t
    for (int t = 0; t < T; ++t) {
        const int a = (cur + 1) % 3, b = (cur + 2) % 3;
        int prev = cur;
        for (int sw = 0; sw < m; ++sw) {
            const int outb = (sw & 1) ? b : a;
            L.ut = bufs[cur];
            L.vin = bufs[prev];
            L.vout = bufs[outb];
            L.energy = (stats && sw == 0) ? 1 : 0;
            GL_HIP(next_set(sw == 0 ? stats + (int64_t)t * K : nullptr,
                            res_base ? res_base + ((int64_t)t * m + sw) * K : nullptr),
                   "stats set");
            GL_HIP(launch_sweep(store_u, K, L, s), "sweep launch");
            prev = outb;
        }
        cur = prev;
    }
    if (stats) {
        // F(u^T): one more product, no update
        L.ut = bufs[cur];
        L.vin = bufs[cur];
        L.vout = nullptr;
        L.energy = 1;
        GL_HIP(next_set(stats + (int64_t)T * K, nullptr), "stats set");
        GL_HIP(launch_sweep(store_u, K, L, s), "energy launch");
    }
    GL_HIP(flush(), "stats launch");
    if (op->order)
        GL_HIP(permute_rows(op, row, bufs[cur], U, true, s), "result scatter");
    else if (cur != 0)
        GL_HIP(copy_bytes(bufs[cur], U, (size_t)op->n * K * dtype_size(store_u), s), "result copy");
    return GL_OK;
}

}  // namespace

extern "C" {

gl_status gl_time_sweeps(const gl_operator* op, const gl_params* params, int32_t K, const int32_t* labels,
                         gl_dtype store_u, const void* U, void* ws, size_t ws_bytes, int32_t reps, double* avg_ms,
                         void* stream) {
    if (!gl::valid(op) || !labels || !U || !ws || !avg_ms) return fail(GL_E_INVALID_ARG, "NULL argument or not an operator handle");
    gl_status st = check_params(params);
    if (st != GL_OK) return st;
    if (K < 1 || K > 16) return fail(GL_E_INVALID_ARG, "K must lie in [1, 16]");
    if (reps < 1 || reps > 10000) return fail(GL_E_INVALID_ARG, "reps must lie in [1, 10000]");
    if (!pair_ok(op->store_w, store_u)) return fail(GL_E_DTYPE, "unsupported (weight, field) storage pair");
    if (!aligned(U, 16) || !aligned(ws, 256)) return fail(GL_E_INVALID_ARG, "U / workspace misaligned");
    if (window_fits(op, K, store_u) != GL_OK) return GL_E_INVALID_ARG;
    size_t need = 0;
    gl_solve_workspace_size(op, K, store_u, &need);
    if (ws_bytes < need) return fail(GL_E_INVALID_ARG, "workspace too small");
    const gl_params& p = *params;
    hipStream_t s = (hipStream_t)stream;
    const size_t field = align256((size_t)op->n * K * dtype_size(store_u));
    char* P = (char*)ws;
    char* Q = (char*)ws + field;
    gl::SweepLaunch L;
    L.r = row_launch(op);
    // the window layout's region sums sit at the end of the workspace
    L.r.wpart = (char*)ws + (need - align256(gl::window_part_bytes(op, K, store_u == GL_F64 ? 8 : 4)));
    L.labels = labels;
    L.partials = (char*)ws + 2 * field;
    L.energy = 0;
    const void* ut = U;
    if (op->order) {
        // renumbered operator: time the sweep on position-ordered inputs
        char* R = (char*)ws + 2 * field;
        int32_t* lab_pos = (int32_t*)((char*)ws + 3 * field);
        L.partials = (char*)lab_pos + align256((size_t)op->n * 4);
        GL_HIP(permute_rows(op, (size_t)K * dtype_size(store_u), U, R, false, s), "permute u");
        GL_HIP(permute_rows(op, 4, labels, lab_pos, false, s), "permute labels");
        L.labels = lab_pos;
        ut = R;
    }
    const double g0 = precond_g(p.precond, 0.0, p), g1 = precond_g(p.precond, 1.0, p);
    const bool inf_k = std::isinf(p.step_k);
    double ga = 0, gd = 0, gll = 0;
    precond_affine(p.precond, p, ga, gd, gll);
    const double coef[14] = {p.eps, p.c, p.eta, 1.0 / p.eps, 0.5 * p.eps, 0.25 / p.eps, 0.5 * p.eta,
                             1.0 / g0, 1.0 / g1, inf_k ? 0.0 : 1.0, inf_k ? 1.0 : p.step_k, ga, gd, gll};
    std::memcpy(L.coef, coef, sizeof(coef));
    L.ut = ut;
    // seed P with u^t so every timed sweep gathers finite values
    GL_HIP(copy_bytes(ut, P, (size_t)op->n * K * dtype_size(store_u), s), "copy");
    // back-to-back launches between one event pair, as a solve issues them:
    // the mean per launch includes the gaps between launches (an event pair
    // around every launch would add its own completion work to every span)
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t err = hipEventCreate(&ev[0]);
    if (err == hipSuccess) err = hipEventCreate(&ev[1]);
    if (err == hipSuccess) err = hipEventRecord(ev[0], s);
    for (int i = 0; i < reps && err == hipSuccess; ++i) {
        L.vin = (i & 1) ? Q : P;
        L.vout = (i & 1) ? P : Q;
        err = launch_sweep(store_u, K, L, s);
    }
    if (err == hipSuccess) err = hipEventRecord(ev[1], s);
    if (err == hipSuccess) err = hipEventSynchronize(ev[1]);
    float total = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&total, ev[0], ev[1]);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    GL_HIP(err, "timed sweeps");
    const double ms = total;
    *avg_ms = (double)ms / reps;
    return GL_OK;
}

gl_status gl_time_stream(int32_t kind, void* buf, size_t bytes, int32_t reps, double* avg_ms, void* stream) {
    if (!buf || !avg_ms) return fail(GL_E_INVALID_ARG, "buf and avg_ms must not be NULL");
    if (kind != 0 && kind != 1) return fail(GL_E_INVALID_ARG, "kind must be 0 (read) or 1 (copy)");
    if (reps < 1 || reps > 10000) return fail(GL_E_INVALID_ARG, "reps must lie in [1, 10000]");
    if (!aligned(buf, 256)) return fail(GL_E_INVALID_ARG, "buf must be 256-byte aligned");
    if (bytes < ((size_t)1 << 20) || bytes % 256) return fail(GL_E_INVALID_ARG, "bytes must be a multiple of 256, >= 1 MiB");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n16 = (int64_t)(kind == 0 ? bytes : bytes / 2) / 16;
    const u32x4_alias* src = (const u32x4_alias*)buf;
    u32x4_alias* dst = (u32x4_alias*)((char*)buf + bytes / 2);
    // 16 workgroups of 256 lanes per compute unit
    const dim3 grid(4096), block(256);
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipError_t err = hipEventCreate(&ev[0]);
    if (err == hipSuccess) err = hipEventCreate(&ev[1]);
    if (err == hipSuccess) err = hipEventRecord(ev[0], s);
    for (int i = 0; i < reps && err == hipSuccess; ++i) {
        if (kind == 0)
            hipLaunchKernelGGL(gl::stream_read_kernel, grid, block, 0, s, src, n16, 0x9e3779b9u,
                               (u32x4_alias*)buf);
        else
            hipLaunchKernelGGL(gl::stream_copy_kernel, grid, block, 0, s, src, dst, n16);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipEventRecord(ev[1], s);
    if (err == hipSuccess) err = hipEventSynchronize(ev[1]);
    float total = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&total, ev[0], ev[1]);
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    GL_HIP(err, "timed streaming");
    *avg_ms = (double)total / reps;
    return GL_OK;
}

gl_status gl_assign_labels(int64_t n, int32_t K, gl_dtype dtype, const void* U, int32_t* out, void* stream) {
    if (!U || !out || n < 0) return fail(GL_E_INVALID_ARG, "U and labels_out must not be NULL, n >= 0");
    if (K < 1 || K > 16) return fail(GL_E_INVALID_ARG, "K must lie in [1, 16]");
    if (n == 0) return GL_OK;
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (dtype) {
        case GL_F64: hipLaunchKernelGGL(gl::labels_kernel<double>, grid, block, 0, s, n, K, (const double*)U, out); break;
        case GL_F32: hipLaunchKernelGGL(gl::labels_kernel<float>, grid, block, 0, s, n, K, (const float*)U, out); break;
        case GL_BF16: hipLaunchKernelGGL(gl::labels_kernel<gl::bf16>, grid, block, 0, s, n, K, (const gl::bf16*)U, out); break;
        case GL_F16: hipLaunchKernelGGL(gl::labels_kernel<gl::f16>, grid, block, 0, s, n, K, (const gl::f16*)U, out); break;
        default: return fail(GL_E_DTYPE, "unknown dtype");
    }
    GL_HIP(hipGetLastError(), "labels launch");
    return GL_OK;
}

}  // extern "C"
