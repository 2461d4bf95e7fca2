// Device construction of the operator's index layout when a processing order
// or the tile layout is asked for (once per graph).
//
// Given the validated CSR pattern on the device and a processing order of the
// rows, build either
//   - the tile layout: rows in processing order padded to multiples of 4,
//     per-256-row halo lists (the sorted distinct columns the block's rows
//     reference) and 16-bit halo-local indices, or
//   - the direct layout: rows in processing order with their own columns,
// plus, for every stored entry, the index of the CSR entry whose normalized
// weight it holds (-1 for padding).  The weights themselves are filled by the
// caller from that map.
//
// Steps: the order's inverse (and its check), stored lengths per position and
// their exclusive scan; for the tile layout one radix sort of the keys
// (block << 32 | column) of all entries, whose distinct keys are the halos in
// block order, and per entry a binary search of its column in its block's
// halo.  The result is the same, entry for entry, as sorting and deduplicating
// each block's columns on its own.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <string>

#include "gl_layout.hpp"

namespace gl {
namespace {

constexpr unsigned kB = 256;

unsigned blocks_for(int64_t n) { return (unsigned)((n + kB - 1) / kB); }

// first[i] = the smallest position that names node i; out-of-range names flag
// their position
__global__ void order_first_kernel(int64_t n, const int32_t* __restrict__ order, int32_t* __restrict__ first,
                                   unsigned long long* __restrict__ bad) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= n) return;
    const int32_t i = order[p];
    if (i < 0 || (int64_t)i >= n) atomicMin(bad, (unsigned long long)p);
    else atomicMin(&first[i], (int32_t)p);
}

// pos_of[i] = p for the first position naming i; a later position naming the
// same node flags itself (the order is then not a permutation)
__global__ void order_inverse_kernel(int64_t n, const int32_t* __restrict__ order, const int32_t* __restrict__ first,
                                     int32_t* __restrict__ pos_of, unsigned long long* __restrict__ bad) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= n) return;
    const int32_t i = order[p];
    if (i < 0 || (int64_t)i >= n) return;
    if (first[i] == (int32_t)p) pos_of[i] = (int32_t)p;
    else atomicMin(bad, (unsigned long long)p);
}

// Entries of the row at each position: stored (padded to 4 for the tile
// layout) and actual.
__global__ void position_lengths_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ order,
                                        int pad4, int64_t* __restrict__ plen, int64_t* __restrict__ dlen) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= n) return;
    const int64_t i = order ? (int64_t)order[p] : p;
    const int64_t deg = rp[i + 1] - rp[i];
    plen[p] = pad4 ? (deg + 3) & ~(int64_t)3 : deg;
    dlen[p] = deg;
}

__global__ void to_int32_kernel(int64_t m, const int64_t* __restrict__ a, int32_t* __restrict__ b) {
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k < m) b[k] = (int32_t)a[k];
}

// keys[eoff[p] + j] = (block of p) << 32 | position of column j of the row at p
__global__ void halo_keys_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 const int32_t* __restrict__ order, const int32_t* __restrict__ pos_of,
                                 const int64_t* __restrict__ eoff, unsigned long long* __restrict__ keys) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= n) return;
    const int64_t i = order ? (int64_t)order[p] : p;
    const unsigned long long hi = (unsigned long long)(p / kLayoutRows) << 32;
    unsigned long long* out = keys + eoff[p];
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t c = pos_of ? pos_of[col[e]] : col[e];
        *out++ = hi | (uint32_t)c;
    }
}

// distinct keys: the first of each run of equal sorted keys
__global__ void key_heads_kernel(int64_t m, const unsigned long long* __restrict__ keys, int32_t* __restrict__ head,
                                 int32_t* __restrict__ per_block) {
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k >= m) return;
    const bool h = k == 0 || keys[k] != keys[k - 1];
    head[k] = h ? 1 : 0;
    if (h) atomicAdd(&per_block[keys[k] >> 32], 1);
}

__global__ void halo_write_kernel(int64_t m, const unsigned long long* __restrict__ keys,
                                  const int32_t* __restrict__ head, const int32_t* __restrict__ slot,
                                  int32_t* __restrict__ halo) {
    const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (k < m && head[k]) halo[slot[k]] = (int32_t)(uint32_t)keys[k];
}

// Per position: the stored entries' source CSR entry and, for the tile layout,
// the column's index in the block's halo (padding keeps its -1 / 0xFFFF fill).
__global__ void entry_map_kernel(int64_t n, const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                 const int32_t* __restrict__ order, const int32_t* __restrict__ pos_of,
                                 const int32_t* __restrict__ srp, const int32_t* __restrict__ halo,
                                 const int32_t* __restrict__ hp, int32_t* __restrict__ src,
                                 uint16_t* __restrict__ lcol) {
    const int64_t p = (int64_t)blockIdx.x * kB + threadIdx.x;
    if (p >= n) return;
    const int64_t i = order ? (int64_t)order[p] : p;
    int64_t dst = srp[p];
    const int32_t* h = nullptr;
    int32_t hn = 0;
    if (lcol) {
        const int64_t b = p / kLayoutRows;
        h = halo + hp[b];
        hn = hp[b + 1] - hp[b];
    }
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e, ++dst) {
        src[dst] = (int32_t)e;
        if (lcol) {
            const int32_t c = pos_of ? pos_of[col[e]] : col[e];
            int32_t lo = 0, hi = hn;  // first halo entry >= c (present: the halo holds every column)
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (h[mid] < c) lo = mid + 1;
                else hi = mid;
            }
            lcol[dst] = (uint16_t)lo;
        }
    }
}

template <typename T> hipError_t dalloc(T** p, size_t count) {
    return hipMalloc((void**)p, (count ? count : 1) * sizeof(T));
}

}  // namespace

void DeviceLayout::release() {
    (void)hipFree(rp);
    (void)hipFree(src);
    (void)hipFree(lcol);
    (void)hipFree(halo);
    (void)hipFree(hp);
    (void)hipFree(pos_of);
    rp = src = halo = hp = pos_of = nullptr;
    lcol = nullptr;
}

LayoutStatus build_layout(int64_t n, int64_t nnz, const int64_t* rp, const int32_t* col, const int32_t* order,
                  bool try_tile, bool require_tile, int32_t halo_limit, hipStream_t s, DeviceLayout& out,
                  std::string& err) {
    out = DeviceLayout();
    int64_t *plen = nullptr, *dlen = nullptr, *sum = nullptr, *eoff = nullptr;
    int32_t* first = nullptr;
    unsigned long long* bad = nullptr;
    unsigned long long *k0 = nullptr, *k1 = nullptr;
    int32_t *head = nullptr, *slot = nullptr, *per_block = nullptr;
    void* tmp = nullptr;
    bool ok = false, invalid = false;
    auto hip = [&](hipError_t e, const char* what) {
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess && err.empty()) err = std::string(what) + ": " + hipGetErrorString(e);
        return e == hipSuccess;
    };
    // exclusive scan of m int64 values into m + 1 offsets
    auto scan = [&](const int64_t* in, int64_t* outp, int64_t m) {
        size_t bytes = 0;
        if (!hip(hipcub::DeviceScan::InclusiveSum(nullptr, bytes, in, outp + 1, (int)m, s), "layout scan")) return false;
        void* t = nullptr;
        if (!hip(hipMalloc(&t, bytes ? bytes : 1), "layout scan")) return false;
        const bool r = hip(hipMemsetAsync(outp, 0, sizeof(int64_t), s), "layout scan") &&
                       hip(hipcub::DeviceScan::InclusiveSum(t, bytes, in, outp + 1, (int)m, s), "layout scan");
        (void)hipFree(t);
        return r;
    };
    const unsigned gn = blocks_for(n);
    do {
        if (!hip(dalloc(&bad, 1), "layout allocation")) break;
        const unsigned long long none = ~0ull;
        if (!hip(hipMemcpyAsync(bad, &none, 8, hipMemcpyHostToDevice, s), "layout set-up")) break;
        // the inverse of the order, and its check
        if (order) {
            if (!hip(dalloc(&first, n), "layout allocation") || !hip(dalloc(&out.pos_of, n), "layout allocation"))
                break;
            if (!hip(hipMemsetAsync(first, 0x7f, (size_t)n * 4, s), "layout set-up")) break;
            hipLaunchKernelGGL(order_first_kernel, dim3(gn), dim3(kB), 0, s, n, order, first, bad);
            if (!hip(hipSuccess, "order check")) break;
            hipLaunchKernelGGL(order_inverse_kernel, dim3(gn), dim3(kB), 0, s, n, order, first, out.pos_of, bad);
            unsigned long long hbad = 0;
            if (!hip(hipMemcpyAsync(&hbad, bad, 8, hipMemcpyDeviceToHost, s), "order check") ||
                !hip(hipStreamSynchronize(s), "order check"))
                break;
            if (hbad != none) {
                err = "order is not a permutation of 0..n-1 (position " + std::to_string(hbad) + ")";
                invalid = true;
                break;
            }
        }
        // stored lengths per position and their offsets
        if (!hip(dalloc(&plen, n), "layout allocation") || !hip(dalloc(&dlen, n), "layout allocation") ||
            !hip(dalloc(&sum, n + 1), "layout allocation") || !hip(dalloc(&eoff, n + 1), "layout allocation"))
            break;
        bool tile = try_tile;
        hipLaunchKernelGGL(position_lengths_kernel, dim3(gn), dim3(kB), 0, s, n, rp, order, tile ? 1 : 0, plen, dlen);
        if (!hip(hipSuccess, "layout lengths") || !scan(dlen, eoff, n)) break;
        if (tile) {
            if (!scan(plen, sum, n)) break;
            int64_t total = 0;
            if (!hip(hipMemcpyAsync(&total, sum + n, 8, hipMemcpyDeviceToHost, s), "layout lengths") ||
                !hip(hipStreamSynchronize(s), "layout lengths"))
                break;
            if (total >= ((int64_t)1 << 31)) {
                err = "too many stored entries for the tile layout";
                invalid = true;
                break;
            }
            // the halos: distinct (block, column) keys of all entries, sorted
            const int64_t nb = (n + kLayoutRows - 1) / kLayoutRows;
            int nbits = 32;
            while (nbits < 64 && ((unsigned long long)nb >> (nbits - 32)) != 0) ++nbits;
            if (!hip(dalloc(&k0, nnz), "layout allocation") || !hip(dalloc(&k1, nnz), "layout allocation") ||
                !hip(dalloc(&head, nnz), "layout allocation") || !hip(dalloc(&slot, nnz), "layout allocation") ||
                !hip(dalloc(&per_block, nb), "layout allocation") || !hip(dalloc(&out.hp, nb + 1), "layout allocation"))
                break;
            hipLaunchKernelGGL(halo_keys_kernel, dim3(gn), dim3(kB), 0, s, n, rp, col, order, out.pos_of,
                               (const int64_t*)eoff, k0);
            if (!hip(hipSuccess, "halo keys")) break;
            hipcub::DoubleBuffer<unsigned long long> keys(k0, k1);
            size_t sort_bytes = 0;
            if (!hip(hipcub::DeviceRadixSort::SortKeys(nullptr, sort_bytes, keys, (int)nnz, 0, nbits, s), "halo sort"))
                break;
            if (!hip(hipMalloc(&tmp, sort_bytes ? sort_bytes : 1), "layout allocation")) break;
            if (!hip(hipcub::DeviceRadixSort::SortKeys(tmp, sort_bytes, keys, (int)nnz, 0, nbits, s), "halo sort"))
                break;
            (void)hipFree(tmp);
            tmp = nullptr;
            const unsigned long long* sorted = keys.Current();
            const unsigned ge = blocks_for(nnz);
            if (!hip(hipMemsetAsync(per_block, 0, (size_t)nb * 4, s), "halo counts")) break;
            hipLaunchKernelGGL(key_heads_kernel, dim3(ge), dim3(kB), 0, s, nnz, sorted, head, per_block);
            if (!hip(hipSuccess, "halo counts")) break;
            size_t scan_bytes = 0;
            if (!hip(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, head, slot, (int)nnz, s), "halo scan"))
                break;
            if (!hip(hipMalloc(&tmp, scan_bytes ? scan_bytes : 1), "layout allocation")) break;
            if (!hip(hipcub::DeviceScan::ExclusiveSum(tmp, scan_bytes, head, slot, (int)nnz, s), "halo scan")) break;
            (void)hipFree(tmp);
            tmp = nullptr;
            // block sizes to the host: the largest halo decides the layout
            std::vector<int32_t> hcount(nb);
            if (!hip(hipMemcpyAsync(hcount.data(), per_block, (size_t)nb * 4, hipMemcpyDeviceToHost, s),
                     "halo counts") ||
                !hip(hipStreamSynchronize(s), "halo counts"))
                break;
            int64_t hmax = 0, htot = 0, worst = 0;
            std::vector<int32_t> hp(nb + 1, 0);
            for (int64_t b = 0; b < nb; ++b) {
                if (hcount[b] > hmax) {
                    hmax = hcount[b];
                    worst = b;
                }
                htot += hcount[b];
                hp[b + 1] = (int32_t)htot;
            }
            if (hmax <= halo_limit) {
                out.layout = 1;
                out.hmax = (int32_t)hmax;
                out.halo_total = htot;
                out.nblocks = nb;
                out.stored = total;
                if (!hip(hipMemcpyAsync(out.hp, hp.data(), (size_t)(nb + 1) * 4, hipMemcpyHostToDevice, s),
                         "halo offsets") ||
                    !hip(dalloc(&out.halo, htot), "layout allocation") ||
                    !hip(dalloc(&out.rp, n + 1), "layout allocation") ||
                    !hip(dalloc(&out.src, total), "layout allocation") ||
                    !hip(dalloc(&out.lcol, total), "layout allocation"))
                    break;
                hipLaunchKernelGGL(halo_write_kernel, dim3(ge), dim3(kB), 0, s, nnz, sorted, head, slot, out.halo);
                hipLaunchKernelGGL(to_int32_kernel, dim3(blocks_for(n + 1)), dim3(kB), 0, s, n + 1, sum, out.rp);
                if (!hip(hipMemsetAsync(out.src, 0xff, (size_t)total * 4, s), "layout fill") ||
                    !hip(hipMemsetAsync(out.lcol, 0xff, (size_t)total * 2, s), "layout fill"))
                    break;
                hipLaunchKernelGGL(entry_map_kernel, dim3(gn), dim3(kB), 0, s, n, rp, col, order, out.pos_of, out.rp,
                                   out.halo, out.hp, out.src, out.lcol);
                if (!hip(hipSuccess, "layout entries")) break;
                ok = true;
                break;
            }
            if (require_tile) {
                err = "block " + std::to_string(worst) + " references " + std::to_string(hmax) +
                      " distinct columns, above the tile limit of " + std::to_string(halo_limit) +
                      "; pass a locality-preserving order or use the direct layout";
                invalid = true;
                break;
            }
            (void)hipFree(out.hp);
            out.hp = nullptr;
        }
        // direct layout in processing order
        int64_t total = 0;
        if (!hip(hipMemcpyAsync(&total, eoff + n, 8, hipMemcpyDeviceToHost, s), "layout lengths") ||
            !hip(hipStreamSynchronize(s), "layout lengths"))
            break;
        if (total >= ((int64_t)1 << 31)) {
            err = "a processing order needs fewer than 2^31 stored entries";
            invalid = true;
            break;
        }
        out.layout = 0;
        out.stored = total;
        if (!hip(dalloc(&out.rp, n + 1), "layout allocation") || !hip(dalloc(&out.src, total), "layout allocation"))
            break;
        hipLaunchKernelGGL(to_int32_kernel, dim3(blocks_for(n + 1)), dim3(kB), 0, s, n + 1, eoff, out.rp);
        hipLaunchKernelGGL(entry_map_kernel, dim3(gn), dim3(kB), 0, s, n, rp, col, order, out.pos_of, out.rp,
                           (const int32_t*)nullptr, (const int32_t*)nullptr, out.src, (uint16_t*)nullptr);
        ok = hip(hipSuccess, "layout entries");
    } while (false);
    if (ok) ok = hip(hipStreamSynchronize(s), "layout construction");
    (void)hipFree(tmp);
    (void)hipFree(plen);
    (void)hipFree(dlen);
    (void)hipFree(sum);
    (void)hipFree(eoff);
    (void)hipFree(first);
    (void)hipFree(bad);
    (void)hipFree(k0);
    (void)hipFree(k1);
    (void)hipFree(head);
    (void)hipFree(slot);
    (void)hipFree(per_block);
    if (!ok) {
        out.release();
        if (err.empty()) err = "layout construction failed";
        return invalid ? kLayoutInvalid : kLayoutDevice;
    }
    return kLayoutOk;
}

}  // namespace gl
