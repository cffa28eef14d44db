// Host check of the sweep pass orders used by the staged-gather and batched
// sweeps.  batch::Slabs (random access, integer division) defines the slab
// order; the kernels walk it incrementally with batch::SlabWalk (host-built
// SlabGeom, multiply-high division by kpm::FastDiv).  Checked here:
//   * Slabs visits every row exactly once and no pass exceeds its budget;
//   * SlabWalk from any start pass with any stride visits exactly the passes
//     p0, p0 + stride, ... of Slabs, in order, and reports the end;
//   * FastDiv equals integer division for edge-case and random dividends.
// Built and run by tests/test_host_logic.py.
#include "kpm_batched.h"

#include <cstdio>
#include <random>
#include <vector>

int main() {
    int bad = 0, cases = 0;
    for (int Lx : {2, 3, 4, 5, 6, 7, 16}) for (int Ly : {2, 3, 4, 6, 9, 16}) for (int Lz : {3, 5, 8})
    for (int lines : {0, 1, 2, 3, 4, 8, 20}) for (int rpw : {1, 2, 4, 8, 16, 64, 128}) {
        kpm::batch::Slabs s;
        s.init(Lx, Ly, Lz, lines, rpw);
        const long N = 4L * Lx * Ly * Lz;
        std::vector<int> seen(N, 0);
        for (long p = 0; p < s.npass + 3; ++p) {
            int64_t r0, nr;
            s.pass(p, r0, nr);
            if (p >= s.npass) {
                if (nr != 0 || r0 != N) ++bad;
                continue;
            }
            if (nr <= 0 || nr > rpw) ++bad;
            for (long r = r0; r < r0 + nr; ++r) {
                if (r < 0 || r >= N) { ++bad; break; }
                ++seen[r];
            }
        }
        for (long r = 0; r < N; ++r)
            if (seen[r] != 1) { ++bad; break; }
        // the walk with the block height the kernels use (a divisor of Ly)
        const kpm::SlabGeom g = kpm::SlabGeom::make(Lx, Ly, Lz, lines, rpw);
        int eff = (lines <= 0 || lines > Ly) ? Ly : lines;
        while (Ly % eff) --eff;
        kpm::batch::Slabs ref;
        ref.init(Lx, Ly, Lz, eff, rpw);
        if (g.npass != ref.npass) ++bad;
        for (int64_t stride : {1, 2, 3, 7, 64, 1000}) for (int64_t p0 : {0, 1, 5, 63}) {
            kpm::batch::SlabWalk w;
            w.init(g, p0, stride);
            for (int64_t p = p0; p < ref.npass + 2 * stride; p += stride) {
                int64_t a0, an, b0, bn;
                w.cur(a0, an);
                ref.pass(p, b0, bn);
                if (a0 != b0 || an != bn) { ++bad; break; }
                w.advance();
            }
        }
        ++cases;
    }
    std::mt19937_64 rng(1);
    long checks = 0;
    std::vector<uint32_t> ds = {1, 2, 3, 5, 7, 10, 16, 17, 64, 100, 255, 256, 1000, 4096, 65535, 65536,
                                1u << 20, (1u << 31) - 1, 1u << 31, 0xFFFFFFFFu};
    for (int i = 0; i < 500; ++i) ds.push_back(1 + static_cast<uint32_t>(rng() % 0xFFFFFFFFull));
    for (uint32_t d : ds) {
        kpm::FastDiv f;
        f.init(d);
        std::vector<uint32_t> ns = {0, 1, d - 1, d, d + 1, 2 * d - 1, 2 * d, 0x7FFFFFFFu, 0x80000000u,
                                    0xFFFFFFFEu, 0xFFFFFFFFu};
        for (int k = 0; k < 500; ++k) ns.push_back(static_cast<uint32_t>(rng()));
        for (uint32_t x : ns) {
            ++checks;
            if (f.div(x) != x / d) ++bad;
        }
    }
    printf("slabs %d cases, fastdiv %ld checks, %d bad\n", cases, checks, bad);
    return bad != 0;
}
