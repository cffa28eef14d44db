// The batched solver derives the 13 gather offsets of a row from its lattice
// site (batch::gather_offsets) instead of reading column indices.  Checked
// here, for the host, against the column rule of the lattice builder (row
// 4 n + o; slot 0 the row itself; per axis x, y, z the sites n - e_j and
// n + e_j, each with orbital o and the partner orbital, o ^ 3 for x and y,
// o ^ 2 for z; a neighbour beyond an open side is a padding slot of value
// zero, for which any row inside the block is acceptable).
#include <cstdio>
#include <cstdint>

#include "kpm_batched.h"

using namespace kpm;

static void builder_columns(int64_t row, const int L[3], const int per[3], int64_t c[13], bool pad[13]) {
    const int64_t n = row >> 2;
    const int o = static_cast<int>(row & 3);
    const int xyz[3] = {static_cast<int>(n % L[0]), static_cast<int>((n / L[0]) % L[1]),
                        static_cast<int>(n / (static_cast<int64_t>(L[0]) * L[1]))};
    int slot = 0;
    pad[slot] = false;
    c[slot++] = row;
    for (int j = 0; j < 3; ++j) {
        const int partner = (j == 2) ? (o ^ 2) : (o ^ 3);
        for (int dir = -1; dir <= 1; dir += 2) {
            int q[3] = {xyz[0], xyz[1], xyz[2]};
            int v = q[j] + dir;
            bool ok = true;
            if (v < 0 || v >= L[j]) {
                if (per[j]) v = (v + L[j]) % L[j];
                else ok = false;
            }
            q[j] = v;
            const int64_t m = q[0] + static_cast<int64_t>(L[0]) * (q[1] + static_cast<int64_t>(L[1]) * q[2]);
            pad[slot] = !ok;
            c[slot++] = 4 * m + o;
            pad[slot] = !ok;
            c[slot++] = 4 * m + partner;
        }
    }
}

template <int R, unsigned CB>
static long check(const int L[3], const int per[3], long* rows) {
    BatchInst d{};
    for (int j = 0; j < 3; ++j) d.L[j] = L[j];
    d.by_lx.init(static_cast<uint32_t>(L[0]));
    d.by_lxy.init(static_cast<uint32_t>(L[0]) * static_cast<uint32_t>(L[1]));
    const int64_t N = 4LL * L[0] * L[1] * L[2];
    const uint32_t RB = R * CB;
    const int64_t step = N > 2000000 ? 7 : 1;
    long bad = 0;
    for (int64_t row = 0; row < N; row += step) {
        int64_t c[13];
        bool pad[13];
        builder_columns(row, L, per, c, pad);
        for (uint32_t lp : {0u, RB - CB}) {
            uint32_t off[13];
            batch::gather_offsets<R, CB>(static_cast<uint32_t>(row), d, lp, off);
            ++*rows;
            for (int k = 0; k < 13; ++k) {
                const bool ok = pad[k] ? (off[k] >= lp && (off[k] - lp) % RB == 0 && (off[k] - lp) / RB < static_cast<uint64_t>(N))
                                       : static_cast<int64_t>(off[k]) == c[k] * RB + lp;
                if (!ok) {
                    if (bad < 5)
                        std::printf("L %d %d %d row %lld slot %d: offset %u, builder column %lld\n", L[0], L[1], L[2],
                                    static_cast<long long>(row), k, off[k], static_cast<long long>(c[k]));
                    ++bad;
                }
            }
        }
    }
    return bad;
}

int main() {
    const int shapes[][6] = {{3, 3, 3, 1, 1, 1},    {4, 4, 4, 1, 1, 1},   {5, 4, 3, 1, 1, 1},  {6, 6, 7, 1, 1, 1},
                             {3, 5, 4, 1, 0, 1},    {2, 3, 5, 0, 1, 0},   {1, 4, 3, 0, 1, 1},  {4, 2, 1, 1, 0, 0},
                             {1, 1, 1, 0, 0, 0},    {7, 6, 5, 1, 1, 0},   {12, 12, 12, 1, 1, 1}, {24, 24, 24, 1, 1, 1},
                             {100, 100, 40, 1, 1, 0}, {64, 64, 64, 1, 1, 1}};
    long rows = 0, bad = 0;
    for (const auto& sh : shapes) {
        const int L[3] = {sh[0], sh[1], sh[2]}, per[3] = {sh[3], sh[4], sh[5]};
        bad += check<8, 8>(L, per, &rows);     // complex64, R = 8 (the batched family)
        bad += check<32, 16>(L, per, &rows);   // complex128, R = 32
    }
    std::printf("gather offsets: %ld rows, %ld bad\n", rows, bad);
    return bad != 0;
}
