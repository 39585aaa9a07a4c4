// Host-side table construction (grid and blockwise Hilbert ordering, row
// neighbour table, projector supports, per-row entries, block atom lists)
// run under AddressSanitizer and UndefinedBehaviorSanitizer, with consistency
// checks between the gather-side and scatter-side projector tables.  Built and
// run by tests/test_host_sanitizers.py with the host compiler only; nothing
// here touches a GPU.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.hpp"

namespace chf {
// the library's error path lives in the C-ABI unit; a host-only stand-in
[[noreturn]] void fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "fail(%d): %s\n", code, buf);
    std::exit(3);
}
}  // namespace chf

using namespace chf;

#define EXPECT(c)                                                          \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                      \
        }                                                                  \
    } while (0)

static double lcg(uint64_t& s) {
    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
    return double(s >> 11) * (1.0 / 9007199254740992.0);
}

static int run(double h, double radius, int ordering, int n_atoms, uint64_t seed) {
    HostGrid g;
    build_grid(g, h, radius, ordering);
    EXPECT(g.n > 0 && g.n_rows >= g.n);
    std::vector<int32_t> nbr;
    build_row_neighbours(g, nbr);
    EXPECT(int64_t(nbr.size()) == g.n_rows * 36);
    for (int64_t r = 0; r < g.n_rows; ++r)
        for (int k = 0; k < 36; ++k) EXPECT(nbr[size_t(r * 36 + k)] >= -1 && nbr[size_t(r * 36 + k)] < g.n_rows);
    for (int64_t r = 0; r < g.n_rows; ++r)        // padding rows have no neighbours
        if (g.rank_of_row[size_t(r)] < 0)
            for (int k = 0; k < 36; ++k) EXPECT(nbr[size_t(r * 36 + k)] == -1);
    if (ordering == CHF_ORDER_HILBERT) {
        for (int64_t q = 0; q < g.n; ++q) {
            const int i = g.ijk[size_t(3 * q)], j = g.ijk[size_t(3 * q + 1)], k = g.ijk[size_t(3 * q + 2)];
            const int64_t row = g.row_of_rank[size_t(q)], s = row / kBlockPts;
            // the point's block coordinates, and its bit in the block's inside mask
            EXPECT(g.blocks[size_t(3 * s)] == (i + g.n_r) / kBlock);
            EXPECT(g.blocks[size_t(3 * s + 1)] == (j + g.n_r) / kBlock);
            EXPECT(g.blocks[size_t(3 * s + 2)] == (k + g.n_r) / kBlock);
            const int l = int(row % kBlockPts);
            EXPECT((g.block_mask[size_t(s * 8 + l / 64)] >> (l % 64)) & 1);
            // every stencil offset that leaves the block through a face lands, when
            // inside the sphere, in the block the face table names
            for (int axis = 0; axis < 3; ++axis)
                for (int d = -6; d <= 6; ++d) {
                    if (d == 0) continue;
                    int c[3] = {i, j, k};
                    c[axis] += d;
                    const int64_t nr_ = g.row_of(c[0], c[1], c[2]);
                    const int64_t ns = nr_ < 0 ? -1 : nr_ / kBlockPts;
                    if (ns < 0 || ns == s) continue;
                    const int f = 2 * axis + (d > 0 ? 1 : 0);
                    EXPECT(g.block_nbr[size_t(6 * s + f)] == ns);
                }
        }
        for (int64_t s = 0; s < g.n_blocks; ++s)      // mask bits are exactly the inside rows
            for (int l = 0; l < kBlockPts; ++l)
                EXPECT((((g.block_mask[size_t(s * 8 + l / 64)] >> (l % 64)) & 1) != 0) ==
                       (g.rank_of_row[size_t(s * kBlockPts + l)] >= 0));
    }
    // atoms inside the sphere, two thirds Si
    std::vector<double> pos(size_t(3 * n_atoms));
    std::vector<int> species(static_cast<size_t>(n_atoms), 0);
    for (int a = 0; a < n_atoms; ++a) {
        double x, y, z;
        do {
            x = (2 * lcg(seed) - 1) * radius;
            y = (2 * lcg(seed) - 1) * radius;
            z = (2 * lcg(seed) - 1) * radius;
        } while (x * x + y * y + z * z > 0.6 * radius * radius);
        pos[size_t(3 * a)] = x, pos[size_t(3 * a + 1)] = y, pos[size_t(3 * a + 2)] = z;
        species[size_t(a)] = (a % 3 == 2) ? 1 : 0;
    }
    chf_atoms atoms{n_atoms, pos.data(), species.data()};
    chf_pp pp{4.0, 1.0, 0.7, 0.5, 1.2, 4.8, 3.0, 0.0};
    HostProj P;
    build_projectors(g, atoms, pp, P);
    EXPECT(P.sup_off.back() == int64_t(P.sup_row.size()));
    EXPECT(P.ent_off.back() == int64_t(P.sup_row.size()));
    for (int64_t r = 0; r < g.n_rows; ++r) EXPECT(P.ent_off[size_t(r)] <= P.ent_off[size_t(r) + 1]);
    for (size_t j = 0; j < P.sup_row.size(); ++j) EXPECT(P.sup_row[j] >= 0 && P.sup_row[j] < g.n_rows);
    // the per-row entries are the transpose of the per-atom supports: walking the
    // atoms in order and appending each support pair to its row reproduces every
    // row's entry list (atoms ascending) with the same projector values, bit for bit
    {
        std::vector<int64_t> fill(P.ent_off.begin(), P.ent_off.end() - 1);
        for (int64_t a = 0; a < P.n_proj; ++a) {
            for (int64_t j = P.sup_off[size_t(a)]; j < P.sup_off[size_t(a) + 1]; ++j) {
                if (j > P.sup_off[size_t(a)]) EXPECT(P.sup_row[size_t(j)] > P.sup_row[size_t(j - 1)]);
                const int64_t e = fill[size_t(P.sup_row[size_t(j)])]++;
                EXPECT(e < P.ent_off[size_t(P.sup_row[size_t(j)]) + 1]);
                EXPECT(P.ent_atom[size_t(e)] == a);
                for (int m = 0; m < 4; ++m) EXPECT(P.ent_beta[size_t(4 * e + m)] == P.sup_beta[size_t(4 * j + m)]);
            }
        }
        for (int64_t r = 0; r < g.n_rows; ++r) EXPECT(fill[size_t(r)] == P.ent_off[size_t(r) + 1]);
    }
    if (ordering == CHF_ORDER_HILBERT) {
        build_block_atoms(g, P);
        EXPECT(int64_t(P.blk_atom_off.size()) == g.n_blocks + 1);
        int max_na = 0;
        for (int64_t b = 0; b < g.n_blocks; ++b) {
            const int64_t e0 = P.ent_off[size_t(b * kBlockPts)], e1 = P.ent_off[size_t((b + 1) * kBlockPts)];
            const int64_t a0 = P.blk_atom_off[size_t(b)], na = P.blk_atom_off[size_t(b) + 1] - a0;
            max_na = std::max(max_na, int(na));
            // the block's list holds exactly the atoms with an entry in its rows, ascending
            std::vector<int32_t> seen;
            for (int64_t e = e0; e < e1; ++e) seen.push_back(P.ent_atom[size_t(e)]);
            std::sort(seen.begin(), seen.end());
            seen.erase(std::unique(seen.begin(), seen.end()), seen.end());
            EXPECT(int64_t(seen.size()) == na);
            for (int64_t i = 0; i < na; ++i) EXPECT(P.blk_atoms[size_t(a0 + i)] == seen[size_t(i)]);
            // and every entry's slot names its own atom in that list
            for (int64_t e = e0; e < e1; ++e) {
                EXPECT(P.ent_slot[size_t(e)] < na || na > 255);
                if (na <= 255) EXPECT(P.blk_atoms[size_t(a0 + P.ent_slot[size_t(e)])] == P.ent_atom[size_t(e)]);
            }
        }
        EXPECT(P.max_block_atoms == max_na);
    }
    std::printf("h %.2f radius %.1f ordering %d: %lld points, %lld rows, %zu support entries\n", h, radius, ordering,
                (long long)g.n, (long long)g.n_rows, P.sup_row.size());
    return 0;
}

int main() {
    int rc = 0;
    rc |= run(0.7, 9.0, CHF_ORDER_HILBERT, 30, 1);
    rc |= run(0.7, 9.0, CHF_ORDER_LEX, 30, 2);
    rc |= run(0.45, 6.3, CHF_ORDER_HILBERT, 12, 3);
    rc |= run(1.0, 5.61, CHF_ORDER_HILBERT, 5, 4);
    if (rc == 0) std::printf("ok\n");
    return rc;
}
