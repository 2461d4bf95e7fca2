// Host-side layout construction shared by the operator builder.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace gl {

constexpr int64_t kLayoutRows = 256;  // positions per tile block (equals kTileRows)

struct HostLayout {
    int32_t layout = 0;              // 0 direct, 1 tile
    std::vector<int32_t> rp;         // [n + 1] stored-entry offsets per position
    std::vector<int32_t> src;        // [stored] source CSR entry, -1 = padding
    std::vector<uint16_t> lcol;      // tile: [stored] halo-local column, 0xFFFF = padding
    std::vector<int32_t> halo;       // tile: columns per block (positions when ordered), sorted
    std::vector<int32_t> hp;         // tile: [blocks + 1] halo offsets
    int32_t hmax = 0;                // tile: largest halo
};

// Build the layout of rows visited in `order` (nullptr = natural order).  With
// an order, halo entries are positions (pos_of[column]), i.e. the operator is
// renumbered into processing order.
// try_tile: attempt the tile layout (falls back to direct when a halo exceeds
// halo_limit, unless require_tile).  Returns false with `err` set on failure.
bool build_layout(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* order, bool try_tile,
                  bool require_tile, int32_t halo_limit, HostLayout& out, std::string& err);

// Grid layout (gl_grid.hpp, built on the device by gl_grid_build.hpp): the
// chunk rounds every pixel has (at most the sweep's first chunk group, which a
// lane requests at once) are stored tile by tile.
constexpr int kGridDenseMax = 4;

}  // namespace gl
