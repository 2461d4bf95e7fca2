// Host construction of the operator's index layout (once per graph).
//
// Given the CSR pattern and a processing order of the rows, build either
//   - the tile layout: rows in processing order padded to multiples of 4,
//     per-256-row halo lists and 16-bit halo-local indices, or
//   - the direct layout: rows in processing order with their own columns,
// plus, for every stored entry, the index of the CSR entry whose normalized
// weight it holds (-1 for padding).  The weights themselves are computed on
// the GPU from that map.
#include <algorithm>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "gl_layout.hpp"

namespace gl {

namespace {

template <typename F>
void parallel_for(int64_t count, F&& fn) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t threads = hw ? (int64_t)hw : 4;
    if (threads > 16) threads = 16;
    if (count < 64) threads = 1;
    if (threads <= 1) {
        fn((int64_t)0, count);
        return;
    }
    std::vector<std::thread> pool;
    const int64_t chunk = (count + threads - 1) / threads;
    for (int64_t t = 0; t < threads; ++t) {
        const int64_t lo = t * chunk, hi = std::min(count, lo + chunk);
        if (lo >= hi) break;
        pool.emplace_back([&fn, lo, hi]() { fn(lo, hi); });
    }
    for (auto& th : pool) th.join();
}

}  // namespace

bool build_layout(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* order, bool try_tile,
                  bool require_tile, int32_t halo_limit, HostLayout& out, std::string& err) {
    auto node = [&](int64_t p) -> int64_t { return order ? (int64_t)order[p] : p; };
    out = HostLayout();
    // With an order the operator works in position space: halo entries and
    // columns name positions, so the field is read in processing order.
    std::vector<int32_t> pos_of;
    if (order) {
        pos_of.resize(n);
        for (int64_t p = 0; p < n; ++p) pos_of[order[p]] = (int32_t)p;
    }
    auto cpos = [&](int32_t j) -> int32_t { return order ? pos_of[j] : j; };
    if (try_tile) {
        const int64_t nb = (n + kLayoutRows - 1) / kLayoutRows;
        std::vector<int64_t> plen(n + 1, 0);
        for (int64_t p = 0; p < n; ++p) {
            const int64_t deg = rp[node(p) + 1] - rp[node(p)];
            plen[p + 1] = plen[p] + ((deg + 3) & ~(int64_t)3);
        }
        if (plen[n] >= ((int64_t)1 << 31)) {
            err = "too many stored entries for the tile layout";
            return false;
        }
        std::vector<std::vector<int32_t>> halos(nb);
        std::vector<int64_t> hsize(nb, 0);
        parallel_for(nb, [&](int64_t lo, int64_t hi) {
            std::vector<int32_t> cols;
            for (int64_t b = lo; b < hi; ++b) {
                cols.clear();
                const int64_t p0 = b * kLayoutRows, p1 = std::min(n, p0 + kLayoutRows);
                for (int64_t p = p0; p < p1; ++p) {
                    const int64_t i = node(p);
                    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) cols.push_back(cpos(col[e]));
                }
                std::sort(cols.begin(), cols.end());
                cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
                hsize[b] = (int64_t)cols.size();
                halos[b] = cols;
            }
        });
        int64_t hmax = 0, htot = 0;
        int64_t worst = 0;
        for (int64_t b = 0; b < nb; ++b) {
            if (hsize[b] > hmax) {
                hmax = hsize[b];
                worst = b;
            }
            htot += hsize[b];
        }
        if (hmax <= halo_limit) {
            out.layout = 1;
            out.hmax = (int32_t)hmax;
            out.rp.resize(n + 1);
            for (int64_t p = 0; p <= n; ++p) out.rp[p] = (int32_t)plen[p];
            out.hp.resize(nb + 1);
            out.hp[0] = 0;
            for (int64_t b = 0; b < nb; ++b) out.hp[b + 1] = out.hp[b] + (int32_t)hsize[b];
            out.halo.resize(htot);
            out.lcol.assign(plen[n], (uint16_t)0xFFFF);
            out.src.assign(plen[n], -1);
            parallel_for(nb, [&](int64_t lo, int64_t hi) {
                for (int64_t b = lo; b < hi; ++b) {
                    const std::vector<int32_t>& h = halos[b];
                    std::copy(h.begin(), h.end(), out.halo.begin() + out.hp[b]);
                    const int64_t p0 = b * kLayoutRows, p1 = std::min(n, p0 + kLayoutRows);
                    for (int64_t p = p0; p < p1; ++p) {
                        const int64_t i = node(p);
                        int64_t dst = plen[p];
                        for (int64_t e = rp[i]; e < rp[i + 1]; ++e, ++dst) {
                            const auto it = std::lower_bound(h.begin(), h.end(), cpos(col[e]));
                            out.lcol[dst] = (uint16_t)(it - h.begin());
                            out.src[dst] = (int32_t)e;
                        }
                    }
                }
            });
            return true;
        }
        if (require_tile) {
            err = "block " + std::to_string(worst) + " references " + std::to_string(hmax) +
                  " distinct columns, above the tile limit of " + std::to_string(halo_limit) +
                  "; pass a locality-preserving order or use the direct layout";
            return false;
        }
    }
    // direct layout in processing order
    out.layout = 0;
    out.rp.resize(n + 1);
    int64_t acc = 0;
    out.rp[0] = 0;
    for (int64_t p = 0; p < n; ++p) {
        acc += rp[node(p) + 1] - rp[node(p)];
        if (acc >= ((int64_t)1 << 31)) {
            err = "a processing order needs fewer than 2^31 stored entries";
            return false;
        }
        out.rp[p + 1] = (int32_t)acc;
    }
    out.src.resize(acc);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        for (int64_t p = lo; p < hi; ++p) {
            const int64_t i = node(p);
            int64_t dst = out.rp[p];
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e, ++dst) out.src[dst] = (int32_t)e;
        }
    });
    return true;
}

}  // namespace gl
