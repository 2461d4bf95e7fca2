// CPU test of the server's host-side logic: arena allocator, footprint,
// direct geometry and the per-solve sweep schedule (buffer rotation).
#include <cassert>
#include <cstdio>
#include <random>
#include <set>
#include <vector>

#include "../paper_2303_14495_amd/csrc/gl_sched.hpp"

static int fails = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                                \
        }                                                           \
    } while (0)

int main() {
    // arena: alignment, exhaustion, coalescing, reuse
    gl::Arena a(1 << 20);
    size_t x = a.alloc(1000), y = a.alloc(5000), z = a.alloc(100);
    CHECK(x == 0 && y == 1024 && z == 1024 + 5120);
    CHECK(a.used() == 1024 + 5120 + 256);
    CHECK(a.alloc(2u << 20) == gl::Arena::kNone);
    CHECK(a.release(y) && !a.release(y) && !a.release(12345));
    CHECK(a.alloc(5000) == 1024);  // first fit reuses the hole
    CHECK(a.release(x) && a.release(1024) && a.release(z));
    CHECK(a.used() == 0 && a.largest_free() == (1u << 20));
    // random alloc/free never overlaps and returns everything
    std::mt19937 rng(7);
    std::vector<std::pair<size_t, size_t>> live;
    gl::Arena b(64 << 20);
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 3) {
            size_t sz = 1 + rng() % 200000;
            size_t off = b.alloc(sz);
            if (off != gl::Arena::kNone) {
                CHECK(off % 256 == 0 && off + sz <= b.capacity());
                for (auto& l : live) CHECK(off + sz <= l.first || l.first + l.second <= off);
                live.push_back({off, sz});
            }
        } else {
            size_t k = rng() % live.size();
            CHECK(b.release(live[k].first));
            live.erase(live.begin() + k);
        }
    }
    for (auto& l : live) CHECK(b.release(l.first));
    CHECK(b.used() == 0 && b.largest_free() == b.capacity());

    // geometry
    gl::DirectGeom g = gl::direct_geometry(1000, 15000);
    CHECK(g.G == 4 || g.G == 8);
    // a small graph: one pass per block, so that there are as many blocks as rows allow
    CHECK(g.tiles == 1 && g.rows_per_block == 256 / g.G && g.blocks * g.rows_per_block >= 1000);
    CHECK(gl::direct_geometry(100, 3000).G == 16);
    // a large one keeps 4 passes per block (>= 1024 blocks either way)
    gl::DirectGeom big = gl::direct_geometry(4194304, 92865744);
    CHECK(big.G == 16 && big.tiles == 4 && big.rows_per_block == 64 && big.blocks == 65536);
    gl::DirectGeom mid = gl::direct_geometry(70000, 1000000);  // 32 rows per pass
    CHECK(mid.G == 8 && mid.tiles == 4 && mid.blocks == 547);
    gl::DirectGeom small = gl::direct_geometry(4096, 61000);  // 4 passes: 32 blocks
    CHECK(small.G == 8 && small.tiles == 1 && small.blocks == 128);

    // footprint grows with every size and separates the raw CSR copy
    gl::Footprint f1 = gl::served_footprint(10000, 150000, 3, 20, 4, 2, 2);
    gl::Footprint f2 = gl::served_footprint(20000, 150000, 3, 20, 4, 2, 2);
    gl::Footprint f3 = gl::served_footprint(10000, 150000, 6, 20, 4, 2, 2);
    CHECK(f2.total() > f1.total() && f3.held > f1.held && f1.raw >= 150000 * 12);

    // schedule: matches the host rotation of gl_solve, never writes the buffer it
    // gathers from or the buffer holding u^t, ends with one energy-only pass
    for (int T = 0; T <= 4; ++T) {
        for (int m = 1; m <= 5; ++m) {
            gl::SweepCursor c;
            c.start(T, m);
            int sweeps = 0, finals = 0;
            int cur = 0;  // reference rotation
            int prev = 0, ref_sweep = 0;
            while (!c.done) {
                if (c.final_pass) {
                    ++finals;
                    CHECK(c.cur == cur);
                } else {
                    const int a_ = (cur + 1) % 3, b_ = (cur + 2) % 3;
                    const int outb = (ref_sweep & 1) ? b_ : a_;
                    const int vin = c.s == 0 ? c.cur : c.prev;
                    CHECK(vin == prev && c.out() == outb && c.out() != vin && c.out() != c.cur);
                    prev = outb;
                    if (++ref_sweep == m) {
                        ref_sweep = 0;
                        cur = prev;
                    }
                    ++sweeps;
                }
                c.advance();
            }
            CHECK(sweeps == T * m && finals == 1 && c.cur == cur);
        }
    }
    std::printf("%s (%d failures)\n", fails ? "FAILED" : "ok", fails);
    return fails ? 1 : 0;
}
