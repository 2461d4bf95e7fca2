// Continuous-batching server of the preconditioned-DCA library (see the
// gl_server_* declarations in gl_dca.h).
//
// Threads:
//   loader    admits queued requests in arrival order while a slot is free and
//             the request fits in the HBM arena; copies it to the GPU, validates
//             the graph and builds the direct-layout operator on its own stream.
//   scheduler advances every admitted solve by one sweep per tick: one batched
//             sweep launch over all of them, then one batched statistics launch.
//   finisher  waits for a finished solve's tick, copies U, classes and stats
//             back, releases its slot and arena memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "gl_internal.hpp"
#include "gl_kernels.hpp"
#include "gl_direct.hpp"
#include "gl_sched.hpp"

namespace gl {

constexpr int kServedKMax = 10;
constexpr int kServedMaxSlots = 64;
constexpr int kServedMaxTicks = 8;

// One active solve as the batched kernels see it.
struct ServedDesc {
    const int32_t* rp;
    const int32_t* col;
    const void* w;
    const void* ut;
    const void* vin;
    void* vout;
    const int32_t* labels;
    void* partials;
    double* energy_dst;  // K doubles or nullptr
    double* res_dst;     // K doubles or nullptr
    double* flag;
    const int32_t* heavy;  // rows longer than 16 G, each summed by a workgroup of its own
    int64_t n;
    int64_t rows_per_block;
    int64_t blocks;       // workgroups of this solve: hblocks heavy-row ones, then the row blocks
    int64_t block_begin;  // prefix over the descriptors of `blocks`
    int32_t stat_begin;   // prefix over the descriptors of 2K
    int32_t G, log2G, tiles, K, energy;
    int32_t nheavy, hblocks;
    float coef[11];
};

template <typename TW, typename TU>
__device__ __forceinline__ SweepArgs<TW, TU, int32_t> served_args(const ServedDesc& d) {
    SweepArgs<TW, TU, int32_t> a;
    // every array of a descriptor is device memory of the arena
    a.rp = as_global(d.rp);
    a.col = as_global(d.col);
    a.w = as_global(static_cast<const TW*>(d.w));
    a.ut = as_global(static_cast<const TU*>(d.ut));
    a.vin = as_global(static_cast<const TU*>(d.vin));
    a.vout = d.vout ? as_global(static_cast<TU*>(d.vout)) : nullptr;
    a.labels = as_global(d.labels);
    a.order = nullptr;
    a.dd = nullptr;  // served solves use L_s
    a.partials = d.partials ? as_global(static_cast<float*>(d.partials)) : nullptr;
    a.g = RowGeom{d.n, d.rows_per_block, d.G, d.log2G, d.tiles, 0};
    a.energy = d.energy;
    a.k.eps = d.coef[0];
    a.k.c = d.coef[1];
    a.k.eta = d.coef[2];
    a.k.inv_eps = d.coef[3];
    a.k.half_eps = d.coef[4];
    a.k.quarter_inv_eps = d.coef[5];
    a.k.half_eta = d.coef[6];
    a.k.ginv0 = d.coef[7];
    a.k.ginv1 = d.coef[8];
    a.k.alpha = d.coef[9];
    a.k.kappa = d.coef[10];
    a.k.ga = a.k.gd = a.k.gl = 0.f;
    a.heavy = d.heavy ? as_global(d.heavy) : nullptr;
    a.nheavy = d.nheavy;
    a.hblocks = d.hblocks;
    return a;
}

// One tick, for the solves of one K: workgroup x runs workgroup
// (x - block_begin) of the solve whose block range contains x: a heavy row or
// a row block, exactly as sweep_kernel numbers them for that solve alone (so
// the partial sums land in the same slots and the results are bitwise those of
// gl_solve).  One instantiation per K keeps each K's register budget its own.
template <int K, typename TW, typename TU>
__global__ __launch_bounds__(kBlock) void served_sweep_kernel(const ServedDesc* __restrict__ descs, int32_t count) {
    __shared__ int32_t s_idx;
    if (threadIdx.x == 0) {
        int lo = 0, hi = count - 1;
        const int64_t x = blockIdx.x;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (descs[mid].block_begin <= x) lo = mid; else hi = mid - 1;
        }
        s_idx = lo;
    }
    __syncthreads();
    const ServedDesc& d = descs[s_idx];
    const int64_t b = (int64_t)blockIdx.x - d.block_begin;
    const SweepArgs<TW, TU, int32_t> a = served_args<TW, TU>(d);
    if (b < d.hblocks)
        heavy_block<K>(a, b, b, d.blocks);
    else
        sweep_block<K>(a, b - d.hblocks, b, d.blocks);
}

// Statistics of one tick: workgroup x reduces statistic (x - stat_begin) of its solve.
__global__ __launch_bounds__(kBlock) void served_stats_kernel(const ServedDesc* __restrict__ descs, int32_t count) {
    __shared__ int32_t s_idx;
    if (threadIdx.x == 0) {
        int lo = 0, hi = count - 1;
        const int32_t x = blockIdx.x;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (descs[mid].stat_begin <= x) lo = mid; else hi = mid - 1;
        }
        s_idx = lo;
    }
    __syncthreads();
    const ServedDesc& d = descs[s_idx];
    const int st = (int)blockIdx.x - d.stat_begin;
    double* dst = st < d.K ? d.energy_dst : d.res_dst;
    if (dst == nullptr) return;  // uniform per block
    const double v = block_sum(static_cast<const float*>(d.partials) + (int64_t)st * d.blocks, d.blocks);
    if (threadIdx.x == 0) {
        dst[st < d.K ? st : st - d.K] = v;
        if (!(fabs(v) <= 1.7976931348623157e308)) *d.flag = 1.0;
    }
}

template <typename TU>
__global__ void f32_to_field_kernel(const float* __restrict__ src, TU* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = store_as<TU>::from(src[i]);
}

template <typename TU>
__global__ void field_to_f32_kernel(const TU* __restrict__ src, float* __restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)cvt<double>(src[i]);
}

__global__ void served_fill_kernel(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace gl

using gl::Arena;

namespace {

gl_status sfail(gl_status st, const std::string& m) {
    gl::set_last_error(m);
    return st;
}

double now_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

size_t dsize(int d) { return d == GL_F64 ? 8 : d == GL_F32 ? 4 : (d == GL_BF16 || d == GL_F16) ? 2 : 0; }

struct Solve {
    uint64_t ticket = 0;
    int64_t n = 0, nnz = 0;
    int32_t K = 1;
    gl_params p{};
    std::vector<int64_t> rp;  // host copies (empty when the request is borrowed)
    std::vector<int32_t> col;
    std::vector<double> w;
    std::vector<int32_t> labels;
    std::vector<float> u0;
    const int64_t* h_rp = nullptr;  // what the loader reads: the copies or the caller's arrays
    const int32_t* h_col = nullptr;
    const double* h_w = nullptr;
    const int32_t* h_labels = nullptr;
    const float* h_u0 = nullptr;
    gl::Footprint fp{};
    size_t off_raw = Arena::kNone, off_held = Arena::kNone;
    // device pointers inside the arena
    int64_t* d_rp64 = nullptr;
    int32_t* d_colin = nullptr;
    double* d_win = nullptr;
    float* d_u0 = nullptr;
    int32_t* d_rp = nullptr;
    int32_t* d_col = nullptr;
    void* d_w = nullptr;
    double* d_deg = nullptr;
    int32_t* d_labels = nullptr;
    int32_t* d_classes = nullptr;
    void* d_buf[3] = {nullptr, nullptr, nullptr};
    float* d_partials = nullptr;
    int32_t* d_heavy = nullptr;
    int32_t nheavy = 0, hblocks = 0;
    double* d_stats = nullptr;
    int32_t* d_flags = nullptr;
    gl::DirectGeom geom{};
    float coef[11]{};
    gl::SweepCursor cur;
    int64_t stats_len = 0;
    // bookkeeping
    double t_submit = 0, t_admit = -1, t_done = -1;
    gl_status status = GL_OK;
    bool cancelled = false;
    hipEvent_t done_event = nullptr;
    // results
    std::vector<float> U_out;
    std::vector<int32_t> classes_out;
    std::vector<double> stats_out;
};

// The solves of one K within a tick: descriptors [first, first + count), their
// workgroups numbered from 0 within the group.
struct TickGroup {
    int32_t K, first, count;
    int64_t blocks;
};

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

}  // namespace

constexpr uint64_t kServerMagic = 0x7365727665722121ull;  // "server!!"

struct gl_server {
    // tag checked by every entry point that takes a server (an operator
    // handle, or a destroyed server, passed in its place is rejected)
    uint64_t magic = kServerMagic;
    gl_server_config cfg{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    char* arena_base = nullptr;
    std::unique_ptr<Arena> arena;
    hipStream_t s_load = nullptr, s_comp = nullptr, s_fin = nullptr;
    // descriptor rings
    gl::ServedDesc* h_desc = nullptr;  // pinned [ticks][slots]
    gl::ServedDesc* d_desc = nullptr;  // device [ticks][slots]
    hipEvent_t tick_ev[gl::kServedMaxTicks] = {};
    bool tick_used[gl::kServedMaxTicks] = {};
    int64_t ticks = 0;

    std::mutex mu;
    std::condition_variable cv_load, cv_sched, cv_fin, cv_done;
    std::deque<std::shared_ptr<Solve>> pending, ready, finishing;
    std::vector<std::shared_ptr<Solve>> active;  // owned by the scheduler
    std::unordered_map<uint64_t, std::shared_ptr<Solve>> all;
    int64_t slots_used = 0, n_finished = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::string fatal;
    std::thread th_load, th_sched, th_fin;

    void set_fatal(const std::string& m) {
        std::lock_guard<std::mutex> g(mu);
        if (fatal.empty()) fatal = m;
    }

    void* at(size_t off) { return arena_base + off; }

    // ---------------------------------------------------------------- loader
    void loader() {
        (void)hipSetDevice(device);
        for (;;) {
            std::shared_ptr<Solve> s;
            {
                std::unique_lock<std::mutex> g(mu);
                cv_load.wait(g, [&] {
                    if (stop) return true;
                    if (pending.empty() || slots_used >= cfg.max_slots) return false;
                    return true;
                });
                if (stop && pending.empty()) return;
                if (stop) {
                    // drain: cancel everything still queued
                    while (!pending.empty()) {
                        auto c = pending.front();
                        pending.pop_front();
                        c->status = GL_E_CANCELLED;
                        c->t_done = now_since(t0);
                        ++n_finished;
                    }
                    cv_done.notify_all();
                    return;
                }
                auto head = pending.front();
                if (head->cancelled) {
                    pending.pop_front();
                    head->status = GL_E_CANCELLED;
                    head->t_done = now_since(t0);
                    ++n_finished;
                    cv_done.notify_all();
                    continue;
                }
                const size_t off_held = arena->alloc(head->fp.held);
                if (off_held == Arena::kNone) {
                    cv_load.wait(g);  // memory is released by the finisher
                    continue;
                }
                const size_t off_raw = arena->alloc(head->fp.raw);
                if (off_raw == Arena::kNone) {
                    arena->release(off_held);
                    cv_load.wait(g);
                    continue;
                }
                pending.pop_front();
                head->off_held = off_held;
                head->off_raw = off_raw;
                head->t_admit = now_since(t0);
                ++slots_used;
                s = head;
            }
            const gl_status st = prepare(*s);
            std::lock_guard<std::mutex> g(mu);
            arena->release(s->off_raw);
            s->off_raw = Arena::kNone;
            if (st != GL_OK) {
                s->status = st;
                arena->release(s->off_held);
                s->off_held = Arena::kNone;
                --slots_used;
                s->t_done = now_since(t0);
                ++n_finished;
                s->rp.clear();
                s->col.clear();
                s->w.clear();
                cv_done.notify_all();
                cv_load.notify_all();
                continue;
            }
            ready.push_back(s);
            cv_sched.notify_all();
        }
    }

    // copy a request to the GPU and build its operator (direct layout)
    gl_status prepare(Solve& s) {
        const size_t sw = dsize(cfg.store_w), su = dsize(cfg.store_u);
        char* raw = (char*)at(s.off_raw);
        char* held = (char*)at(s.off_held);
        size_t o = 0;
        auto take = [&](char* base, size_t bytes) {
            char* p = base + o;
            o += gl::align256(bytes);
            return p;
        };
        s.d_rp64 = (int64_t*)take(raw, (size_t)(s.n + 1) * 8);
        s.d_colin = (int32_t*)take(raw, (size_t)s.nnz * 4);
        s.d_win = (double*)take(raw, (size_t)s.nnz * 8);
        s.d_u0 = (float*)take(raw, (size_t)s.n * s.K * 4);
        o = 0;
        s.d_rp = (int32_t*)take(held, (size_t)(s.n + 1) * 4);
        s.d_col = (int32_t*)take(held, (size_t)s.nnz * 4);
        s.d_w = take(held, (size_t)s.nnz * sw);
        s.d_deg = (double*)take(held, (size_t)s.n * 8);
        s.d_labels = (int32_t*)take(held, (size_t)s.n * 4);
        s.d_classes = (int32_t*)take(held, (size_t)s.n * 4);
        for (int i = 0; i < 3; ++i) s.d_buf[i] = take(held, (size_t)s.n * s.K * su);
        // heavy rows from the request's own row offsets (host), before the copies
        const std::vector<int32_t> hv = gl::heavy_rows(s.n, s.h_rp, s.geom.G);
        if ((int64_t)hv.size() > gl::heavy_bound(s.nnz, s.geom.G)) {
            // only a malformed row_ptr (not non-decreasing) gets here; the
            // validation kernel would reject it too
            return GL_E_BAD_GRAPH;
        }
        s.nheavy = (int32_t)hv.size();
        s.hblocks = (int32_t)gl::heavy_blocks(s.nheavy);
        s.d_heavy = (int32_t*)take(held, (size_t)gl::heavy_bound(s.nnz, s.geom.G) * 4);
        s.d_partials = (float*)take(held, (size_t)2 * s.K * (s.geom.blocks + gl::heavy_blocks(gl::heavy_bound(s.nnz, s.geom.G))) * 4);
        s.d_stats = (double*)take(held, (size_t)s.stats_len * 8);
        s.d_flags = (int32_t*)take(held, 256);

        hipStream_t st = s_load;
        struct {
            int32_t flags, pad;
            unsigned long long first;
        } fl = {0, 0, ~0ull};
        hipError_t e = hipMemcpyAsync(s.d_rp64, s.h_rp, (s.n + 1) * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_colin, s.h_col, s.nnz * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_win, s.h_w, s.nnz * 8, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_labels, s.h_labels, s.n * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_u0, s.h_u0, s.n * s.K * 4, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(s.d_flags, &fl, sizeof(fl), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !hv.empty())
            e = hipMemcpyAsync(s.d_heavy, hv.data(), hv.size() * 4, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            set_fatal(std::string("server copy: ") + hipGetErrorString(e));
            return GL_E_HIP;
        }
        // Validation, degrees and normalisation run one after another with a
        // host check in between: the later kernels trust the row offsets and
        // columns, so they only run on a graph that passed the previous step.
        const unsigned grid = (unsigned)((s.n + 255) / 256);
        unsigned long long* first = (unsigned long long*)((char*)s.d_flags + 8);
        auto read_flags = [&]() {
            hipError_t e2 = hipGetLastError();
            if (e2 == hipSuccess) e2 = hipMemcpyAsync(&fl, s.d_flags, sizeof(fl), hipMemcpyDeviceToHost, st);
            if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
            return e2;
        };
        auto drop_host_copies = [&]() {
            s.h_rp = nullptr;
            s.h_col = nullptr;
            s.h_w = nullptr;
            s.h_labels = nullptr;
            s.h_u0 = nullptr;
            s.labels.clear();
            s.labels.shrink_to_fit();
            s.rp.clear();
            s.rp.shrink_to_fit();
            s.col.clear();
            s.col.shrink_to_fit();
            s.w.clear();
            s.w.shrink_to_fit();
            s.u0.clear();
            s.u0.shrink_to_fit();
        };
        hipLaunchKernelGGL(gl::validate_kernel<double>, dim3(grid), dim3(256), 0, st, s.n, s.nnz, s.d_rp64,
                           s.d_colin, s.d_win, s.d_flags, first);
        e = read_flags();
        if (e == hipSuccess && fl.flags == 0) {
            hipLaunchKernelGGL(gl::degree_kernel<double>, dim3(grid), dim3(256), 0, st, s.n, s.d_rp64, s.d_win,
                               s.d_deg, s.d_flags, first);
            e = read_flags();
        }
        if (e != hipSuccess) {
            set_fatal(std::string("server validation: ") + hipGetErrorString(e));
            return GL_E_HIP;
        }
        if (fl.flags) {
            drop_host_copies();
            return GL_E_BAD_GRAPH;
        }
        const unsigned grid1 = (unsigned)((s.n + 1 + 255) / 256);
        switch (cfg.store_w) {
            case GL_F32:
                hipLaunchKernelGGL((gl::normalize_kernel<double, float, int32_t>), dim3(grid1), dim3(256), 0, st, s.n,
                                   s.d_rp64, s.d_colin, s.d_win, s.d_deg, s.d_rp, s.d_col, (float*)s.d_w, 0);
                break;
            case GL_BF16:
                hipLaunchKernelGGL((gl::normalize_kernel<double, gl::bf16, int32_t>), dim3(grid1), dim3(256), 0, st,
                                   s.n, s.d_rp64, s.d_colin, s.d_win, s.d_deg, s.d_rp, s.d_col, (gl::bf16*)s.d_w, 0);
                break;
            default:
                hipLaunchKernelGGL((gl::normalize_kernel<double, gl::f16, int32_t>), dim3(grid1), dim3(256), 0, st,
                                   s.n, s.d_rp64, s.d_colin, s.d_win, s.d_deg, s.d_rp, s.d_col, (gl::f16*)s.d_w, 0);
                break;
        }
        const int64_t cells = s.n * s.K;
        const unsigned gc = (unsigned)((cells + 255) / 256);
        switch (cfg.store_u) {
            case GL_F32:
                hipLaunchKernelGGL(gl::f32_to_field_kernel<float>, dim3(gc), dim3(256), 0, st, s.d_u0,
                                   (float*)s.d_buf[0], cells);
                break;
            case GL_BF16:
                hipLaunchKernelGGL(gl::f32_to_field_kernel<gl::bf16>, dim3(gc), dim3(256), 0, st, s.d_u0,
                                   (gl::bf16*)s.d_buf[0], cells);
                break;
            default:
                hipLaunchKernelGGL(gl::f32_to_field_kernel<gl::f16>, dim3(gc), dim3(256), 0, st, s.d_u0,
                                   (gl::f16*)s.d_buf[0], cells);
                break;
        }
        hipLaunchKernelGGL(gl::served_fill_kernel, dim3((unsigned)((s.stats_len + 255) / 256)), dim3(256), 0, st,
                           s.d_stats, s.stats_len);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            set_fatal(std::string("server prepare: ") + hipGetErrorString(e));
            return GL_E_HIP;
        }
        drop_host_copies();
        const double g0 = precond_g(s.p.precond, 0.0, s.p), g1 = precond_g(s.p.precond, 1.0, s.p);
        const bool inf_k = std::isinf(s.p.step_k);
        const double c[11] = {s.p.eps, s.p.c, s.p.eta, 1.0 / s.p.eps, 0.5 * s.p.eps, 0.25 / s.p.eps, 0.5 * s.p.eta,
                              1.0 / g0, 1.0 / g1, inf_k ? 0.0 : 1.0, inf_k ? 1.0 : s.p.step_k};
        for (int i = 0; i < 11; ++i) s.coef[i] = (float)c[i];
        s.cur.start(s.p.outer_steps, s.p.inner_sweeps);
        return GL_OK;
    }

    // ------------------------------------------------------------- scheduler
    void scheduler() {
        (void)hipSetDevice(device);
        int slot = 0;
        for (;;) {
            {
                std::unique_lock<std::mutex> g(mu);
                cv_sched.wait(g, [&] { return !ready.empty() || !active.empty() || (stop && slots_used == 0); });
                while (!ready.empty()) {
                    active.push_back(ready.front());
                    ready.pop_front();
                }
                if (active.empty()) return;  // stop requested and nothing left
            }
            // drop cancelled solves at the tick boundary
            std::vector<std::shared_ptr<Solve>> done_now;
            {
                std::lock_guard<std::mutex> g(mu);
                for (auto& s : active)
                    if (s->cancelled && !s->cur.done) {
                        s->status = GL_E_CANCELLED;
                        s->cur.done = true;
                    }
            }
            // descriptor slot must be free of the launch it last served
            if (tick_used[slot]) {
                if (hipEventSynchronize(tick_ev[slot]) != hipSuccess) set_fatal("tick wait failed");
            }
            gl::ServedDesc* hd = h_desc + (size_t)slot * cfg.max_slots;
            gl::ServedDesc* dd = d_desc + (size_t)slot * cfg.max_slots;
            int count = 0;
            int64_t blocks = 0;  // within the current K group
            int32_t stats = 0;
            // solves grouped by K (one sweep launch per K), in admission order within a group
            std::vector<Solve*> order;
            for (auto& s : active)
                if (!s->cur.done) order.push_back(s.get());
            std::stable_sort(order.begin(), order.end(), [](const Solve* a, const Solve* b) { return a->K < b->K; });
            std::vector<TickGroup> groups;
            for (Solve* s : order) {
                if (groups.empty() || groups.back().K != s->K) {
                    groups.push_back(TickGroup{s->K, count, 0, 0});
                    blocks = 0;
                }
                gl::ServedDesc& d = hd[count++];
                d.rp = s->d_rp;
                d.col = s->d_col;
                d.w = s->d_w;
                d.labels = s->d_labels;
                d.partials = s->d_partials;
                d.heavy = s->d_heavy;
                d.nheavy = s->nheavy;
                d.hblocks = s->hblocks;
                d.n = s->n;
                d.rows_per_block = s->geom.rows_per_block;
                d.blocks = s->geom.blocks + s->hblocks;
                d.block_begin = blocks;
                d.stat_begin = stats;
                d.G = s->geom.G;
                d.log2G = s->geom.log2G;
                d.tiles = s->geom.tiles;
                d.K = s->K;
                std::memcpy(d.coef, s->coef, sizeof(d.coef));
                const int64_t E = (int64_t)(s->cur.T + 1) * s->K;
                d.flag = s->d_stats + s->stats_len - 1;
                if (s->cur.final_pass) {
                    d.ut = d.vin = s->d_buf[s->cur.cur];
                    d.vout = nullptr;
                    d.energy = 1;
                    d.energy_dst = s->d_stats + (int64_t)s->cur.T * s->K;
                    d.res_dst = nullptr;
                } else {
                    d.ut = s->d_buf[s->cur.cur];
                    d.vin = s->d_buf[s->cur.s == 0 ? s->cur.cur : s->cur.prev];
                    d.vout = s->d_buf[s->cur.out()];
                    d.energy = s->cur.s == 0 ? 1 : 0;
                    d.energy_dst = s->cur.s == 0 ? s->d_stats + (int64_t)s->cur.t * s->K : nullptr;
                    d.res_dst = s->d_stats + E + ((int64_t)s->cur.t * s->cur.m + s->cur.s) * s->K;
                }
                blocks += d.blocks;
                stats += 2 * s->K;
                groups.back().count += 1;
                groups.back().blocks = blocks;
            }
            if (count > 0) {
                hipError_t e = hipMemcpyAsync(dd, hd, sizeof(gl::ServedDesc) * count, hipMemcpyHostToDevice, s_comp);
                if (e == hipSuccess) e = launch_tick(dd, count, groups, stats);
                if (e == hipSuccess) e = hipEventRecord(tick_ev[slot], s_comp);
                if (e != hipSuccess) set_fatal(std::string("tick launch: ") + hipGetErrorString(e));
                tick_used[slot] = true;
                ++ticks;
            }
            // advance; finished solves get their classes and a completion event
            for (auto& s : active) {
                if (s->cur.done) {
                    done_now.push_back(s);
                    continue;
                }
                const bool was_final = s->cur.final_pass;
                s->cur.advance();
                if (was_final) {
                    const unsigned gl_ = (unsigned)((s->n + 255) / 256);
                    const void* u = s->d_buf[s->cur.cur];
                    switch (cfg.store_u) {
                        case GL_F32:
                            hipLaunchKernelGGL(gl::labels_kernel<float>, dim3(gl_), dim3(256), 0, s_comp, s->n, s->K,
                                               (const float*)u, s->d_classes);
                            break;
                        case GL_BF16:
                            hipLaunchKernelGGL(gl::labels_kernel<gl::bf16>, dim3(gl_), dim3(256), 0, s_comp, s->n,
                                               s->K, (const gl::bf16*)u, s->d_classes);
                            break;
                        default:
                            hipLaunchKernelGGL(gl::labels_kernel<gl::f16>, dim3(gl_), dim3(256), 0, s_comp, s->n,
                                               s->K, (const gl::f16*)u, s->d_classes);
                            break;
                    }
                    done_now.push_back(s);
                }
            }
            if (!done_now.empty()) {
                for (auto& s : done_now) {
                    if (hipEventCreateWithFlags(&s->done_event, hipEventDisableTiming) != hipSuccess ||
                        hipEventRecord(s->done_event, s_comp) != hipSuccess)
                        set_fatal("event record failed");
                }
                std::lock_guard<std::mutex> g(mu);
                active.erase(std::remove_if(active.begin(), active.end(),
                                            [&](const std::shared_ptr<Solve>& s) {
                                                return std::find(done_now.begin(), done_now.end(), s) !=
                                                       done_now.end();
                                            }),
                             active.end());
                for (auto& s : done_now) finishing.push_back(s);
                cv_fin.notify_all();
            }
            slot = (slot + 1) % cfg.ticks_in_flight;
        }
    }

    template <typename TW, typename TU>
    hipError_t launch_group(const gl::ServedDesc* dd, const TickGroup& g) {
        const dim3 grid((unsigned)g.blocks), block(gl::kBlock);
        const gl::ServedDesc* d = dd + g.first;
        switch (g.K) {
#define GL_SK(KK)                                                                                        \
    case KK:                                                                                             \
        hipLaunchKernelGGL((gl::served_sweep_kernel<KK, TW, TU>), grid, block, 0, s_comp, d, g.count);   \
        break;
            GL_SK(1) GL_SK(2) GL_SK(3) GL_SK(4) GL_SK(5) GL_SK(6) GL_SK(7) GL_SK(8) GL_SK(9) GL_SK(10)
#undef GL_SK
            default:
                return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }

    hipError_t launch_tick(const gl::ServedDesc* dd, int count, const std::vector<TickGroup>& groups, int32_t stats) {
        for (const TickGroup& g : groups) {
            hipError_t e = hipErrorInvalidValue;
            switch (cfg.store_w * 4 + cfg.store_u) {
#define GL_TICK(WD, UD, TW, TU) \
    case WD * 4 + UD:           \
        e = launch_group<TW, TU>(dd, g); \
        break;
                GL_TICK(GL_F32, GL_F32, float, float)
                GL_TICK(GL_F32, GL_BF16, float, gl::bf16)
                GL_TICK(GL_F32, GL_F16, float, gl::f16)
                GL_TICK(GL_BF16, GL_F32, gl::bf16, float)
                GL_TICK(GL_BF16, GL_BF16, gl::bf16, gl::bf16)
                GL_TICK(GL_BF16, GL_F16, gl::bf16, gl::f16)
                GL_TICK(GL_F16, GL_F32, gl::f16, float)
                GL_TICK(GL_F16, GL_BF16, gl::f16, gl::bf16)
                GL_TICK(GL_F16, GL_F16, gl::f16, gl::f16)
#undef GL_TICK
                default:
                    break;
            }
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(gl::served_stats_kernel, dim3((unsigned)stats), dim3(gl::kBlock), 0, s_comp, dd,
                           (int32_t)count);
        return hipGetLastError();
    }

    // -------------------------------------------------------------- finisher
    void finisher() {
        (void)hipSetDevice(device);
        for (;;) {
            std::shared_ptr<Solve> s;
            {
                std::unique_lock<std::mutex> g(mu);
                cv_fin.wait(g, [&] { return !finishing.empty() || (stop && slots_used == 0); });
                if (finishing.empty()) return;
                s = finishing.front();
                finishing.pop_front();
            }
            hipError_t e = hipEventSynchronize(s->done_event);
            (void)hipEventDestroy(s->done_event);
            s->done_event = nullptr;
            if (e == hipSuccess && s->status == GL_OK) {
                const int64_t cells = s->n * s->K;
                const size_t su = dsize(cfg.store_u);
                std::vector<uint8_t> raw((size_t)cells * su);
                s->classes_out.resize(s->n);
                s->stats_out.resize(s->stats_len);
                e = hipMemcpyAsync(raw.data(), s->d_buf[s->cur.cur], raw.size(), hipMemcpyDeviceToHost, s_fin);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(s->classes_out.data(), s->d_classes, s->n * 4, hipMemcpyDeviceToHost, s_fin);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(s->stats_out.data(), s->d_stats, s->stats_len * 8, hipMemcpyDeviceToHost,
                                       s_fin);
                if (e == hipSuccess) e = hipStreamSynchronize(s_fin);
                if (e != hipSuccess) {
                    set_fatal(std::string("server readback: ") + hipGetErrorString(e));
                    s->status = GL_E_HIP;
                } else {
                    s->U_out.resize(cells);
                    for (int64_t i = 0; i < cells; ++i) {
                        if (cfg.store_u == GL_F32) {
                            std::memcpy(&s->U_out[i], &raw[(size_t)i * 4], 4);
                        } else if (cfg.store_u == GL_BF16) {
                            uint16_t h;
                            std::memcpy(&h, &raw[(size_t)i * 2], 2);
                            const uint32_t bits = (uint32_t)h << 16;
                            std::memcpy(&s->U_out[i], &bits, 4);
                        } else {
                            _Float16 h;
                            std::memcpy(&h, &raw[(size_t)i * 2], 2);
                            s->U_out[i] = (float)h;
                        }
                    }
                    if (s->stats_out.back() != 0.0) s->status = GL_E_NONFINITE;
                }
            } else if (e != hipSuccess) {
                s->status = GL_E_HIP;
            }
            std::lock_guard<std::mutex> g(mu);
            arena->release(s->off_held);
            s->off_held = Arena::kNone;
            --slots_used;
            ++n_finished;
            s->t_done = now_since(t0);
            cv_done.notify_all();
            cv_load.notify_all();
            cv_sched.notify_all();
        }
    }
};

namespace {
bool srv_ok(const gl_server* srv) { return srv != nullptr && srv->magic == kServerMagic; }
}  // namespace

extern "C" {

gl_status gl_server_create(const gl_server_config* cfg, gl_server** out) {
    if (!cfg || !out) return sfail(GL_E_INVALID_ARG, "config and out must not be NULL");
    *out = nullptr;
    if (cfg->hbm_budget_bytes < (1u << 20)) return sfail(GL_E_INVALID_ARG, "hbm_budget_bytes must be >= 1 MiB");
    if (cfg->max_slots < 1 || cfg->max_slots > gl::kServedMaxSlots) return sfail(GL_E_INVALID_ARG, "max_slots in 1..64");
    if (cfg->max_pending < 1) return sfail(GL_E_INVALID_ARG, "max_pending must be >= 1");
    auto lowp = [](int d) { return d == GL_F32 || d == GL_BF16 || d == GL_F16; };
    if (!lowp(cfg->store_w) || !lowp(cfg->store_u)) return sfail(GL_E_DTYPE, "server storage must be F32/BF16/F16");
    if (cfg->ticks_in_flight < 1 || cfg->ticks_in_flight > gl::kServedMaxTicks)
        return sfail(GL_E_INVALID_ARG, "ticks_in_flight in 1..8");
    if (cfg->reserved != 0) return sfail(GL_E_INVALID_ARG, "reserved must be 0");
    gl_server* s = new gl_server();
    s->cfg = *cfg;
    s->t0 = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return sfail(GL_E_HIP, "hipGetDevice failed");
    }
    const size_t ring = sizeof(gl::ServedDesc) * cfg->max_slots * cfg->ticks_in_flight;
    bool ok = hipMalloc((void**)&s->arena_base, cfg->hbm_budget_bytes) == hipSuccess &&
              hipMalloc((void**)&s->d_desc, ring) == hipSuccess &&
              hipHostMalloc((void**)&s->h_desc, ring, hipHostMallocDefault) == hipSuccess &&
              hipStreamCreateWithFlags(&s->s_load, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->s_fin, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; ok && i < cfg->ticks_in_flight; ++i)
        ok = hipEventCreateWithFlags(&s->tick_ev[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        (void)hipFree(s->arena_base);
        (void)hipFree(s->d_desc);
        (void)hipHostFree(s->h_desc);
        if (s->s_load) (void)hipStreamDestroy(s->s_load);
        if (s->s_comp) (void)hipStreamDestroy(s->s_comp);
        if (s->s_fin) (void)hipStreamDestroy(s->s_fin);
        for (int i = 0; i < gl::kServedMaxTicks; ++i)
            if (s->tick_ev[i]) (void)hipEventDestroy(s->tick_ev[i]);
        delete s;
        return sfail(GL_E_NOMEM, "server allocation failed");
    }
    s->arena.reset(new Arena(cfg->hbm_budget_bytes));
    s->th_load = std::thread([s] { s->loader(); });
    s->th_sched = std::thread([s] { s->scheduler(); });
    s->th_fin = std::thread([s] { s->finisher(); });
    *out = s;
    return GL_OK;
}

gl_status gl_server_submit(gl_server* srv, const gl_request* r, uint64_t* ticket) {
    if (!srv_ok(srv) || !r || !ticket)
        return sfail(GL_E_INVALID_ARG, "server (a live server handle), request and ticket must not be NULL");
    if (!r->row_ptr || !r->col_idx || !r->weight || !r->labels || !r->u0)
        return sfail(GL_E_INVALID_ARG, "request arrays must not be NULL");
    if (r->n < 2 || r->n > INT32_MAX || r->nnz < 1 || r->nnz > INT32_MAX)
        return sfail(GL_E_INVALID_ARG, "served graphs need 2 <= n and 1 <= nnz < 2^31");
    if (r->K < 1 || r->K > gl::kServedKMax) return sfail(GL_E_INVALID_ARG, "served K must lie in [1, 10]");
    if (r->flags & ~GL_REQ_BORROW) return sfail(GL_E_INVALID_ARG, "unknown request flags");
    if (gl_params_validate(&r->params) != GL_OK) return sfail(GL_E_INVALID_ARG, gl_last_error());
    if (r->row_ptr[0] != 0 || r->row_ptr[r->n] != r->nnz)
        return sfail(GL_E_INVALID_ARG, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    auto s = std::make_shared<Solve>();
    s->n = r->n;
    s->nnz = r->nnz;
    s->K = r->K;
    s->p = r->params;
    s->geom = gl::direct_geometry(r->n, r->nnz);
    s->stats_len = gl_stats_length(r->K, r->params.outer_steps, r->params.inner_sweeps);
    s->fp = gl::served_footprint(r->n, r->nnz, r->K, r->params.outer_steps, r->params.inner_sweeps,
                                 dsize(srv->cfg.store_w), dsize(srv->cfg.store_u));
    {
        std::lock_guard<std::mutex> g(srv->mu);
        if (s->fp.held + s->fp.raw > srv->arena->capacity())
            return sfail(GL_E_BUDGET, "request footprint exceeds the server's HBM arena");
        if ((int64_t)srv->pending.size() >= srv->cfg.max_pending) return sfail(GL_E_QUEUE_FULL, "pending queue is full");
        if (srv->stop) return sfail(GL_E_INVALID_ARG, "server is shutting down");
    }
    if (r->flags & GL_REQ_BORROW) {
        s->h_rp = r->row_ptr;
        s->h_col = r->col_idx;
        s->h_w = r->weight;
        s->h_labels = r->labels;
        s->h_u0 = r->u0;
    } else {
        s->rp.assign(r->row_ptr, r->row_ptr + r->n + 1);
        s->col.assign(r->col_idx, r->col_idx + r->nnz);
        s->w.assign(r->weight, r->weight + r->nnz);
        s->labels.assign(r->labels, r->labels + r->n);
        s->u0.assign(r->u0, r->u0 + r->n * r->K);
        s->h_rp = s->rp.data();
        s->h_col = s->col.data();
        s->h_w = s->w.data();
        s->h_labels = s->labels.data();
        s->h_u0 = s->u0.data();
    }
    std::lock_guard<std::mutex> g(srv->mu);
    s->ticket = srv->next_ticket++;
    s->t_submit = now_since(srv->t0);
    srv->pending.push_back(s);
    srv->all[s->ticket] = s;
    *ticket = s->ticket;
    srv->cv_load.notify_all();
    return GL_OK;
}

gl_status gl_server_poll(gl_server* srv, uint64_t ticket, int32_t wait, gl_result* out) {
    if (!srv_ok(srv) || !out) return sfail(GL_E_INVALID_ARG, "server (a live server handle) and result must not be NULL");
    std::shared_ptr<Solve> s;
    {
        std::unique_lock<std::mutex> g(srv->mu);
        auto it = srv->all.find(ticket);
        if (it == srv->all.end()) return sfail(GL_E_INVALID_ARG, "unknown or consumed ticket");
        s = it->second;
        if (s->t_done < 0) {
            if (!wait) return sfail(GL_E_NOT_READY, "not finished");
            srv->cv_done.wait(g, [&] { return s->t_done >= 0; });
        }
        srv->all.erase(it);
        --srv->n_finished;
    }
    out->t_submit = s->t_submit;
    out->t_admit = s->t_admit;
    out->t_done = s->t_done;
    out->status = s->status;
    if (s->status == GL_OK || s->status == GL_E_NONFINITE) {
        if (out->U) std::memcpy(out->U, s->U_out.data(), s->U_out.size() * 4);
        if (out->labels) std::memcpy(out->labels, s->classes_out.data(), s->classes_out.size() * 4);
        if (out->stats) std::memcpy(out->stats, s->stats_out.data(), s->stats_out.size() * 8);
    }
    return GL_OK;
}

gl_status gl_server_cancel(gl_server* srv, uint64_t ticket) {
    if (!srv_ok(srv)) return sfail(GL_E_INVALID_ARG, "server must be a live server handle");
    std::lock_guard<std::mutex> g(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) return sfail(GL_E_INVALID_ARG, "unknown or consumed ticket");
    const std::shared_ptr<Solve>& s = it->second;
    s->cancelled = true;
    auto q = std::find(srv->pending.begin(), srv->pending.end(), s);
    if (q != srv->pending.end()) {
        // still queued: it ends here, without ever reaching the GPU
        srv->pending.erase(q);
        s->status = GL_E_CANCELLED;
        s->t_done = now_since(srv->t0);
        ++srv->n_finished;
        srv->cv_done.notify_all();
    }
    srv->cv_load.notify_all();
    return GL_OK;
}

gl_status gl_server_request_bytes(int64_t n, int64_t nnz, int32_t K, int32_t outer_steps, int32_t inner_sweeps,
                                  gl_dtype store_w, gl_dtype store_u, size_t* peak, size_t* held) {
    if (!peak || !held) return sfail(GL_E_INVALID_ARG, "peak and held must not be NULL");
    if (n < 2 || nnz < 1 || K < 1 || K > gl::kServedKMax || outer_steps < 0 || inner_sweeps < 1)
        return sfail(GL_E_INVALID_ARG, "sizes out of range");
    const size_t sw = dsize(store_w), su = dsize(store_u);
    if (store_w == GL_F64 || store_u == GL_F64 || !sw || !su)
        return sfail(GL_E_DTYPE, "server storage must be F32/BF16/F16");
    const gl::Footprint f = gl::served_footprint(n, nnz, K, outer_steps, inner_sweeps, sw, su);
    *peak = f.total();
    *held = f.held;
    return GL_OK;
}

gl_status gl_server_info(gl_server* srv, int64_t* pending, int64_t* active, int64_t* finished, size_t* arena_used,
                         int64_t* ticks) {
    if (!srv_ok(srv)) return sfail(GL_E_INVALID_ARG, "server must be a live server handle");
    std::lock_guard<std::mutex> g(srv->mu);
    if (pending) *pending = (int64_t)srv->pending.size();
    if (active) *active = srv->slots_used;
    if (finished) *finished = srv->n_finished;
    if (arena_used) *arena_used = srv->arena->used();
    if (ticks) *ticks = srv->ticks;
    if (!srv->fatal.empty()) return sfail(GL_E_HIP, srv->fatal);
    return GL_OK;
}

gl_status gl_server_destroy(gl_server* srv) {
    if (!srv) return GL_OK;
    if (!srv_ok(srv)) return sfail(GL_E_INVALID_ARG, "not a server handle");
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
        srv->cv_load.notify_all();
    }
    srv->th_load.join();
    // the loader has cancelled the queue; wait for admitted solves to finish
    {
        std::unique_lock<std::mutex> g(srv->mu);
        srv->cv_sched.notify_all();
        srv->cv_done.wait(g, [&] { return srv->slots_used == 0; });
        srv->cv_sched.notify_all();
        srv->cv_fin.notify_all();
    }
    srv->th_sched.join();
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->cv_fin.notify_all();
    }
    srv->th_fin.join();
    (void)hipStreamSynchronize(srv->s_comp);
    (void)hipFree(srv->arena_base);
    (void)hipFree(srv->d_desc);
    (void)hipHostFree(srv->h_desc);
    (void)hipStreamDestroy(srv->s_load);
    (void)hipStreamDestroy(srv->s_comp);
    (void)hipStreamDestroy(srv->s_fin);
    for (int i = 0; i < gl::kServedMaxTicks; ++i)
        if (srv->tick_ev[i]) (void)hipEventDestroy(srv->tick_ev[i]);
    srv->magic = 0;
    delete srv;
    return GL_OK;
}

}  // extern "C"
