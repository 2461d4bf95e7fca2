// Index layouts the operator builder constructs on the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace gl {

constexpr int64_t kLayoutRows = 256;  // positions per tile block (equals kTileRows)

// Device arrays of an ordered direct or tile layout (gl_layout.hip); the
// operator takes ownership of them.
struct DeviceLayout {
    int32_t layout = 0;          // 0 direct, 1 tile
    int32_t* rp = nullptr;       // [n + 1] stored-entry offsets per position
    int32_t* src = nullptr;      // [stored] source CSR entry, -1 = padding
    uint16_t* lcol = nullptr;    // tile: [stored] halo-local column, 0xFFFF = padding
    int32_t* halo = nullptr;     // tile: columns per block (positions when ordered), sorted
    int32_t* hp = nullptr;       // tile: [blocks + 1] halo offsets
    int32_t* pos_of = nullptr;   // with an order: position of each node
    int32_t hmax = 0;            // tile: largest halo
    int64_t halo_total = 0, nblocks = 0, stored = 0;
    void release();              // free every array
};

// Build the layout of rows visited in `order` (nullptr = natural order) from
// the device CSR pattern rp[n + 1] (int64), col[nnz] (nnz < 2^31), and check
// that `order` is a permutation.  With an order, halo entries and columns name
// positions (pos_of[column]), i.e. the operator is renumbered into processing
// order.  try_tile: attempt the tile layout (falls back to direct when a halo
// exceeds halo_limit, unless require_tile).  Synchronises `s`.  Returns
// kLayoutOk, or kLayoutInvalid (the order or the sizes) / kLayoutDevice (an
// allocation or launch failed) with `err` set and nothing allocated.
enum LayoutStatus { kLayoutOk = 0, kLayoutInvalid = 1, kLayoutDevice = 2 };
LayoutStatus build_layout(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col, const int32_t* order,
                  bool try_tile, bool require_tile, int32_t halo_limit, hipStream_t s, DeviceLayout& out,
                  std::string& err);

// Grid layout (gl_grid.hpp, built on the device by gl_grid_build.hpp): the
// chunk rounds every pixel has (at most the sweep's first chunk group, which a
// lane requests at once) are stored tile by tile.
constexpr int kGridDenseMax = 4;

}  // namespace gl
