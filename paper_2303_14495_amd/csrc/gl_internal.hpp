// Host-side interfaces between the C ABI and the per-storage-type kernel units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/gl_dca.h"

namespace gl {

enum Layout : int32_t { LAYOUT_DIRECT = 0, LAYOUT_TILE = 1, LAYOUT_WINDOW = 2, LAYOUT_GRID = 3 };

// Untyped description of one row-kernel launch; the unit compiled for the
// field's storage type casts the pointers and picks the K instantiation.
struct RowLaunch {
    int32_t layout;
    const void* w;        // normalized weights in the operator's storage type
    gl_dtype wdt;
    const int32_t* order; // node of each position, or nullptr
    const void* dd;       // diagonal of L = D - W in the accumulator type, or nullptr (L_s)
    int64_t n;
    int64_t grid;
    // direct layout
    const void* rp;       // int32 or int64 row offsets
    const int32_t* col;
    bool idx64;
    int64_t rows_per_block;
    int32_t G, log2G, tiles, remap;
    const int32_t* heavy;  // rows longer than 16 G (summed by workgroups of their own in the sweep)
    int32_t nheavy;
    // tile layout
    const int32_t* trp;
    const uint16_t* lcol;
    const int32_t* halo;
    const int32_t* hp;
    int32_t hmax;
    // window layout (implicit columns of an image's search window); wpart: the
    // caller's buffer for the region sums of one product (window_part_bytes)
    void* wpart;
    int32_t wheight, wwidth, wr, wM, wtiles_x;
    // grid layout (window-relative one-byte columns); image size and tiles_x
    // share wheight, wwidth, wtiles_x
    const uint64_t* goffs;
    const int64_t* gwbase;
    const uint8_t* gcnt;
    int32_t gdense;
};

struct SweepLaunch {
    RowLaunch r;
    const void* ut;
    const void* vin;
    void* vout;
    const int32_t* labels;
    void* partials;
    int32_t energy;
    // eps, c, eta, 1/eps, eps/2, 1/(4 eps), eta/2, 1/g0, 1/g1, alpha, kappa, ga, gd, gl
    double coef[14];
};

}  // namespace gl

// The operator behind the gl_operator handle (library-owned device memory).
struct gl_operator {
    // tag checked by every entry point that takes an operator, so that a
    // server handle (or a destroyed operator) passed in its place is rejected
    uint64_t magic = 0x6f70657261746f72ull;  // "operator"
    int64_t n = 0, nnz = 0, stored = 0;
    int device = 0;
    gl_dtype store_w = GL_F32;
    int32_t layout = gl::LAYOUT_DIRECT;
    bool idx64 = false;
    int32_t* order = nullptr;   // node of each position (nullptr = natural order)
    void* rp = nullptr;         // direct: int32/int64 offsets; tile: int32 padded offsets
    int32_t* col = nullptr;     // direct only
    uint16_t* lcol = nullptr;   // tile only
    int32_t* halo = nullptr;    // tile only
    int32_t* hp = nullptr;      // tile only
    int32_t hmax = 0;
    int64_t halo_total = 0, nblocks = 0;
    void* w = nullptr;
    double* degree = nullptr;   // d_i of the input weights, node order
    int32_t lap = GL_LAP_NORMALIZED;
    void* dd = nullptr;   // unnormalized L: diagonal d (accumulator type, position order)
    double dmax = 1.0;    // largest diagonal entry of the Laplacian (1 for L_s)
    int32_t G = 16, log2G = 4, tiles = 4, remap = 1;
    int32_t* heavy = nullptr;  // direct layout: rows longer than 16 G, in position order
    int32_t nheavy = 0;
    // window layout: image height x width, window radius, offsets per pixel,
    // tiles per image row
    int32_t wheight = 0, wwidth = 0, wr = 0, wM = 0, wtiles_x = 0;
    // grid layout: offset bytes, first chunk per row segment, chunks per pixel
    // (image size and tiles per row in wheight, wwidth, wtiles_x)
    uint64_t* goffs = nullptr;
    int64_t* gwbase = nullptr;
    uint8_t* gcnt = nullptr;
    int64_t gchunks = 0;
    int32_t gdense = 0;  // chunk rounds stored by pixel
    size_t bytes = 0;
};

namespace gl {

constexpr uint64_t kOperatorMagic = 0x6f70657261746f72ull;

// True for a live operator handle (not NULL, not another handle type).
inline bool valid(const gl_operator* op) { return op != nullptr && op->magic == kOperatorMagic; }

// Row-kernel launch description of an operator.
RowLaunch operator_rows(const gl_operator* op);

// Workgroups of one sweep launch: the row blocks, and on the direct layout the
// heavy rows' workgroups (a multiple of 8) before them.  The sweep's block
// partial sums have one slot per workgroup.
inline int64_t sweep_grid(const RowLaunch& r) {
    return r.grid + (r.layout == LAYOUT_DIRECT ? ((int64_t)r.nheavy + 7) / 8 * 8 : 0);
}

// Power-method pass on the window layout (see gl::window_power_kernel); part:
// window_part_bytes(op, 1, 4) bytes.
hipError_t launch_window_power(const gl_operator* op, const float* x, float* y, int mode, const float* scale,
                               float* partials, float* part, hipStream_t s);

// gl_knn for 64 < d <= 4096 (arguments checked by the caller); *fallback_rows
// receives the number of rows recomputed by the exact scan.
gl_status knn_wide(const float* x, int64_t n, int32_t d, int32_t k, int32_t* idx_out, float* d2_out,
                   hipStream_t s, int64_t* fallback_rows);

// LDS bytes one window-layout block needs for K columns of accumulator size acc.
size_t window_lds_bytes(const gl_operator* op, int K, size_t acc);

// Bytes of the region-sum buffer of one window product with K columns of
// accumulator size acc (0 for other layouts).
size_t window_part_bytes(const gl_operator* op, int K, size_t acc);

// Thread-local message returned by gl_last_error().
void set_last_error(const std::string& msg);

// Each returns hipSuccess or the launch error; hipErrorInvalidValue when the
// (weight type, K) combination is not compiled for this field type.
hipError_t launch_sweep_f64(int K, const SweepLaunch& L, hipStream_t s);
hipError_t launch_sweep_f32(int K, const SweepLaunch& L, hipStream_t s);
hipError_t launch_sweep_bf16(int K, const SweepLaunch& L, hipStream_t s);
hipError_t launch_sweep_f16(int K, const SweepLaunch& L, hipStream_t s);

// Grid-layout sweeps (their own compile units), dispatched by launch_sweep_*.
hipError_t launch_grid_sweep_f64(int K, const SweepLaunch& L, hipStream_t s);
hipError_t launch_grid_sweep_f32(int K, const SweepLaunch& L, hipStream_t s);
hipError_t launch_grid_sweep_bf16(int K, const SweepLaunch& L, hipStream_t s);
hipError_t launch_grid_sweep_f16(int K, const SweepLaunch& L, hipStream_t s);

hipError_t launch_laplacian_f64(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s);
hipError_t launch_laplacian_f32(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s);
hipError_t launch_laplacian_bf16(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s);
hipError_t launch_laplacian_f16(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s);

}  // namespace gl
