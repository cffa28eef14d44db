// Host check of the pencil order of the staged-gather sweep (TileGeom,
// batch::TileWalk).  For lattices whose sides are and are not multiples of
// the tile side, every pass size the order is used with (rpw 1, 2, 4), grids
// that do and do not split over the 8 dies and several waves per workgroup,
// the passes of all waves of all workgroups together cover every row
// exactly once, each pass is whole (rpw rows inside one line of one tile),
// and every wave reports its end.  Built and run by tests/test_host_logic.py.
#include "kpm_batched.h"

#include <cstdio>
#include <vector>

int main() {
    int bad = 0, cases = 0;
    long passes = 0;
    for (int Lx : {3, 4, 5, 8, 13, 16}) for (int Ly : {2, 4, 7, 8, 16}) for (int Lz : {3, 4, 9, 16})
    for (int side : {1, 2, 3, 4, 8}) for (int rpw : {1, 2, 4}) for (int grid : {1, 7, 8, 16, 40, 64})
    for (int waves : {1, 3, 8}) {
        const kpm::TileGeom g = kpm::TileGeom::make(Lx, Ly, Lz, side, rpw, grid, 8);
        const long N = 4L * Lx * Ly * Lz;
        if (g.nrows != N) { ++bad; continue; }
        std::vector<int> seen(N, 0);
        for (int b = 0; b < grid; ++b) for (int w = 0; w < waves; ++w) {
            kpm::batch::TileWalk t;
            t.init(g, b, grid, 8, w, waves);
            for (long it = 0;; ++it) {
                int64_t r0, nr;
                t.cur(r0, nr);
                if (nr == 0) {
                    if (r0 != N) ++bad;
                    t.advance();          // past the end stays at the end
                    t.cur(r0, nr);
                    if (nr != 0 || r0 != N) ++bad;
                    break;
                }
                if (nr != rpw || r0 < 0 || r0 + nr > N) { ++bad; break; }
                // a pass lies inside one line of one tile: same site line, same tile column
                const long s0 = r0 / 4, s1 = (r0 + nr - 1) / 4;
                if (s0 / Lx != s1 / Lx || (s0 % Lx) / side != (s1 % Lx) / side) ++bad;
                for (long r = r0; r < r0 + nr; ++r) ++seen[r];
                ++passes;
                if (it > 4 * N) { ++bad; break; }
                t.advance();
            }
        }
        for (long r = 0; r < N; ++r)
            if (seen[r] != 1) { ++bad; break; }
        ++cases;
    }
    printf("tile walk %d cases, %ld passes, %d bad\n", cases, passes, bad);
    return bad != 0;
}
