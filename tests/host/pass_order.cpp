// Host check of the sweep pass order (batch::Slabs) used by the staged-gather
// and batched sweeps: for lattices of many shapes, slab heights and pass
// sizes, every row is visited exactly once, no pass exceeds its row budget,
// and passes past the end are empty.  Built and run by tests/test_host_logic.py.
#include "kpm_batched.h"

#include <cstdio>
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
        ++cases;
    }
    printf("slabs %d cases, %d bad\n", cases, bad);
    return bad != 0;
}
