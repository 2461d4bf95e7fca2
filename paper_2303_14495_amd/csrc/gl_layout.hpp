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

// Grid layout (nodes = pixels of a height x width image, row-major; every
// edge within 7 rows and 7 columns).  Per pixel, its CSR entries in chunks of
// 8; within each 64-pixel row segment (one wavefront), chunk c of every pixel
// that has more than c chunks follows all chunks c - 1, in pixel order.
// Chunk rounds of every pixel stored by pixel (at most the sweep's first chunk
// group, which a lane requests at once).
constexpr int kGridDenseMax = 4;

struct GridLayout {
    int64_t chunks = 0;
    int32_t tiles_x = 0;
    int32_t dense = 0;            // rounds stored by pixel: chunk r < dense of pixel i is chunk r * n + i
    std::vector<uint8_t> offs;    // [chunks * 8] (dy + 7) << 4 | (dx + 7); 0x77 = padding
    std::vector<int32_t> src;     // [chunks * 8] source CSR entry, -1 = padding
    std::vector<uint8_t> cnt;     // [n] chunks per pixel
    std::vector<int64_t> wbase;   // [height * tiles_x] first chunk of each row segment (rounds >= dense)
};

bool build_grid_layout(int64_t n, int32_t height, int32_t width, const int64_t* rp, const int32_t* col,
                       GridLayout& out, std::string& err);

}  // namespace gl
