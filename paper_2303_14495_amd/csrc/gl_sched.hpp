// Host-side pieces of the continuous-batching server that do not touch the
// GPU: the device-arena allocator, the per-request footprint, the direct-layout
// geometry and the per-solve sweep schedule.  Header-only so that the CPU tests
// compile it with a plain C++ compiler.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <vector>

namespace gl {

// First-fit allocator over [0, capacity) with aligned offsets; adjacent free
// ranges are merged on release.  Not thread-safe (the server holds a lock).
class Arena {
  public:
    static constexpr size_t kNone = ~(size_t)0;

    explicit Arena(size_t capacity, size_t align = 256) : cap_(capacity), align_(align), used_(0) {
        if (cap_) free_[0] = cap_;
    }

    size_t alloc(size_t bytes) {
        const size_t need = round_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                const size_t off = it->first, rest = it->second - need;
                free_.erase(it);
                if (rest) free_[off + need] = rest;
                live_[off] = need;
                used_ += need;
                return off;
            }
        }
        return kNone;
    }

    // Returns false if `off` is not a live allocation.
    bool release(size_t off) {
        auto it = live_.find(off);
        if (it == live_.end()) return false;
        size_t start = off, size = it->second;
        used_ -= size;
        live_.erase(it);
        auto nxt = free_.lower_bound(start);
        if (nxt != free_.end() && start + size == nxt->first) {
            size += nxt->second;
            nxt = free_.erase(nxt);
        }
        if (nxt != free_.begin()) {
            auto prv = std::prev(nxt);
            if (prv->first + prv->second == start) {
                start = prv->first;
                size += prv->second;
                free_.erase(prv);
            }
        }
        free_[start] = size;
        return true;
    }

    size_t used() const { return used_; }
    size_t capacity() const { return cap_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }
    size_t round_up(size_t b) const { return (b + align_ - 1) / align_ * align_; }

  private:
    std::map<size_t, size_t> free_;  // offset -> size
    std::map<size_t, size_t> live_;  // offset -> size
    size_t cap_, align_, used_;
};

// Direct-layout geometry for a graph: G lanes per row (smallest power of two
// with 2G > mean row length, 4..64), 4 passes of 256/G rows per block, or 2
// or 1 when that would leave fewer than 256 blocks (one per compute unit)
// for a small graph (more, shorter blocks cost the batched server more than
// they gain above that).  Every row is summed in the same order whatever the
// geometry; the block partial sums of the statistics follow it, so gl_solve
// and the server share this function.
struct DirectGeom {
    int32_t G, log2G, tiles;
    int64_t rows_per_block, blocks;
};

inline DirectGeom direct_geometry(int64_t n, int64_t nnz) {
    DirectGeom g;
    const double avg = n > 0 ? (double)nnz / (double)n : 0.0;
    int G = 4;
    while (G < 64 && 2.0 * G <= avg) G *= 2;
    g.G = G;
    g.log2G = 0;
    while ((1 << g.log2G) < G) ++g.log2G;
    const int64_t rows_per_tile = (int64_t)(256 >> g.log2G);
    g.tiles = 4;
    while (g.tiles > 1 && (n + rows_per_tile * g.tiles - 1) / (rows_per_tile * g.tiles) < 256) g.tiles /= 2;
    g.rows_per_block = rows_per_tile * g.tiles;
    g.blocks = (n + g.rows_per_block - 1) / g.rows_per_block;
    return g;
}

// Rows longer than heavy_threshold(G) entries ("heavy" rows: the hubs of kNN
// graphs in high dimension) are left out of the row passes of the sweep and
// summed by a workgroup of their own (each of its 256 lanes takes every 256th
// entry), so no lane walks a long row alone.  Their workgroups come first in
// the launch, padded to a multiple of 8 (one per XCD), so the row passes that
// follow keep their XCD-aligned numbering.
inline int64_t heavy_threshold(int G) { return 16 * (int64_t)G; }

inline int64_t heavy_blocks(int64_t nheavy) { return (nheavy + 7) / 8 * 8; }

// Upper bound of the heavy rows of a graph (each holds more than
// heavy_threshold(G) of the nnz entries).
inline int64_t heavy_bound(int64_t nnz, int G) { return nnz / (heavy_threshold(G) + 1) + 1; }

// The heavy rows of a CSR graph, in increasing row order.
template <typename OffT>
inline std::vector<int32_t> heavy_rows(int64_t n, const OffT* rp, int G) {
    std::vector<int32_t> out;
    const int64_t h = heavy_threshold(G);
    for (int64_t i = 0; i < n; ++i)
        if ((int64_t)(rp[i + 1] - rp[i]) > h) out.push_back((int32_t)i);
    return out;
}

// Device bytes of one served solve, split into the part released once its
// operator is built (the raw CSR copy) and the part held until it finishes.
struct Footprint {
    size_t raw, held;
    size_t total() const { return raw + held; }
};

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline Footprint served_footprint(int64_t n, int64_t nnz, int32_t K, int32_t T, int32_t m, size_t sw,
                                  size_t su) {
    const DirectGeom g = direct_geometry(n, nnz);
    Footprint f;
    f.raw = align256((size_t)(n + 1) * 8) + align256((size_t)nnz * 4) + align256((size_t)nnz * 8) +
            align256((size_t)n * K * 4);  // row_ptr, col, f64 weights, f32 u0
    const size_t stats = (size_t)((T + 1) * K + (int64_t)T * m * K + 1) * 8;
    f.held = align256((size_t)(n + 1) * 4) + align256((size_t)nnz * 4) + align256((size_t)nnz * sw) +
             align256((size_t)n * 8) +                       // degrees
             align256((size_t)n * 4) * 2 +                    // labels in, classes out
             3 * align256((size_t)n * K * su) +               // field buffers
             align256((size_t)heavy_bound(nnz, g.G) * 4) +    // heavy rows
             align256((size_t)2 * K * (g.blocks + heavy_blocks(heavy_bound(nnz, g.G))) * 4) +  // block partials
             align256(stats) + 256;                           // stats + flags
    return f;
}

// Position of a solve in its schedule: outer step t, sweep s of m; after the
// T steps one energy-only pass, then done.
struct SweepCursor {
    int32_t t = 0, s = 0, T = 0, m = 1;
    bool final_pass = false, done = false;
    int cur = 0, prev = 0;  // buffer holding u^t, buffer gathered by the next sweep

    void start(int32_t T_, int32_t m_) {
        T = T_;
        m = m_;
        t = s = 0;
        cur = prev = 0;
        done = false;
        final_pass = (T == 0);
    }
    // buffer written by the current sweep
    int out() const { return (s & 1) ? (cur + 2) % 3 : (cur + 1) % 3; }
    // advance past the sweep (or final pass) just launched
    void advance() {
        if (final_pass) {
            done = true;
            return;
        }
        prev = out();
        if (++s == m) {
            s = 0;
            cur = prev;
            if (++t == T) final_pass = true;
        }
    }
};

}  // namespace gl
