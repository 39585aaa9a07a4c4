// Host-side construction of the spherical grid, its blockwise Hilbert (or
// lexicographic) ordering, the neighbour / block tables and the
// Kleinman-Bylander projector tables.
//
// Paper: the spherical confined domain with wavefunctions vanishing outside;
// the partitioning of grid points along blockwise Hilbert space-filling
// curves that speeds up the sparse H-times-vector products; norm-conserving
// pseudopotentials in Kleinman-Bylander (separable) form.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <numeric>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "internal.hpp"

namespace chf {

// Hilbert index of a cell by Skilling's transpose method (J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004): undo the
// excess work level by level (high bit first) by inverting or exchanging the
// low bits of the first axis, Gray-encode across the axes, then interleave
// the bits with the x axis most significant at every level.
uint64_t hilbert_index3(uint32_t x, uint32_t y, uint32_t z, int nbits) {
    uint32_t v[3] = {x, y, z};
    const uint32_t top = 1u << (nbits - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t lowmask = q - 1;
        for (int a = 0; a < 3; ++a) {
            if (v[a] & q) {
                v[0] ^= lowmask;
            } else {
                const uint32_t swap = (v[0] ^ v[a]) & lowmask;
                v[0] ^= swap;
                v[a] ^= swap;
            }
        }
    }
    v[1] ^= v[0];
    v[2] ^= v[1];
    uint32_t flip = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (v[2] & q) flip ^= q - 1;
    for (int a = 0; a < 3; ++a) v[a] ^= flip;
    uint64_t key = 0;
    for (int lvl = nbits - 1; lvl >= 0; --lvl)
        for (int a = 0; a < 3; ++a) key = (key << 1) | ((v[a] >> lvl) & 1u);
    return key;
}

static int bit_length(int64_t v) {
    int n = 0;
    while (v > 0) {
        ++n;
        v >>= 1;
    }
    return n;
}

bool HostGrid::inside(int i, int j, int k) const {
    if (i < -n_r || i > n_r || j < -n_r || j > n_r || k < -n_r || k > n_r) return false;
    return int64_t(i) * i + int64_t(j) * j + int64_t(k) * k <= thr;
}

int64_t HostGrid::row_of(int i, int j, int k) const {
    if (!inside(i, j, k)) return -1;
    const int I = i + n_r, J = j + n_r, K = k + n_r;
    if (ordering == CHF_ORDER_LEX) {
        const int64_t e = 2 * int64_t(n_r) + 1;
        return lex_cube[(int64_t(K) * e + J) * e + I];
    }
    const int64_t blin = (int64_t(K / kBlock) * nb + J / kBlock) * nb + I / kBlock;
    const int64_t slot = slot_of_block[blin];
    return slot * kBlockPts + (I % kBlock) + kBlock * (J % kBlock) + kBlock * kBlock * (K % kBlock);
}

void build_grid(HostGrid& g, double h, double radius, int ordering) {
    g.h = h;
    g.radius = radius;
    g.ordering = ordering;
    g.n_r = int(std::floor(radius / h));
    const double q = radius / h;
    g.thr = int64_t(std::floor(q * q + 1e-9));
    const int nr = g.n_r;
    const int64_t e = 2 * int64_t(nr) + 1;
    if (ordering == CHF_ORDER_LEX) {
        g.lex_cube.assign(size_t(e * e * e), -1);
        int64_t rank = 0;
        for (int k = -nr; k <= nr; ++k)
            for (int j = -nr; j <= nr; ++j)
                for (int i = -nr; i <= nr; ++i)
                    if (g.inside(i, j, k)) {
                        g.lex_cube[(int64_t(k + nr) * e + (j + nr)) * e + (i + nr)] = int32_t(rank);
                        g.ijk.push_back(i);
                        g.ijk.push_back(j);
                        g.ijk.push_back(k);
                        ++rank;
                    }
        g.n = rank;
        g.n_rows = rank;
        g.n_blocks = 0;
        g.row_of_rank.resize(size_t(rank));
        std::iota(g.row_of_rank.begin(), g.row_of_rank.end(), int64_t(0));
        g.rank_of_row.resize(size_t(rank));
        std::iota(g.rank_of_row.begin(), g.rank_of_row.end(), 0);
        return;
    }
    g.nb = int((2 * nr) / kBlock + 1);
    const int nb = g.nb;
    const int nbits = std::max(1, bit_length(nb - 1));
    std::vector<uint8_t> occ(size_t(nb) * nb * nb, 0);
    for (int k = -nr; k <= nr; ++k)
        for (int j = -nr; j <= nr; ++j)
            for (int i = -nr; i <= nr; ++i)
                if (g.inside(i, j, k))
                    occ[(size_t((k + nr) / kBlock) * nb + (j + nr) / kBlock) * nb + (i + nr) / kBlock] = 1;
    std::vector<std::pair<uint64_t, int64_t>> keyed;
    for (int bz = 0; bz < nb; ++bz)
        for (int by = 0; by < nb; ++by)
            for (int bx = 0; bx < nb; ++bx) {
                const int64_t lin = (int64_t(bz) * nb + by) * nb + bx;
                if (occ[size_t(lin)]) keyed.emplace_back(hilbert_index3(bx, by, bz, nbits), lin);
            }
    std::sort(keyed.begin(), keyed.end());
    g.n_blocks = int64_t(keyed.size());
    g.n_rows = g.n_blocks * kBlockPts;
    g.slot_of_block.assign(occ.size(), -1);
    g.blocks.resize(size_t(g.n_blocks) * 3);
    for (int64_t s = 0; s < g.n_blocks; ++s) {
        const int64_t lin = keyed[size_t(s)].second;
        g.slot_of_block[size_t(lin)] = int32_t(s);
        g.blocks[size_t(3 * s + 0)] = int32_t(lin % nb);
        g.blocks[size_t(3 * s + 1)] = int32_t((lin / nb) % nb);
        g.blocks[size_t(3 * s + 2)] = int32_t(lin / (int64_t(nb) * nb));
    }
    // ranks follow rows; rows of a block are its x-fastest local indices
    g.rank_of_row.assign(size_t(g.n_rows), -1);
    g.block_mask.assign(size_t(g.n_blocks) * 8, 0);
    for (int64_t s = 0; s < g.n_blocks; ++s) {
        const int bx = g.blocks[size_t(3 * s)], by = g.blocks[size_t(3 * s + 1)], bz = g.blocks[size_t(3 * s + 2)];
        for (int l = 0; l < kBlockPts; ++l) {
            const int i = bx * kBlock + (l % kBlock) - nr;
            const int j = by * kBlock + ((l / kBlock) % kBlock) - nr;
            const int k = bz * kBlock + (l / (kBlock * kBlock)) - nr;
            if (g.inside(i, j, k)) {
                g.rank_of_row[size_t(s * kBlockPts + l)] = 0;
                g.block_mask[size_t(s * 8 + l / 64)] |= uint64_t(1) << (l % 64);
            }
        }
    }
    int64_t rank = 0;
    for (int64_t r = 0; r < g.n_rows; ++r) {
        if (g.rank_of_row[size_t(r)] < 0) continue;
        g.rank_of_row[size_t(r)] = int32_t(rank++);
        const int64_t s = r / kBlockPts;
        const int l = int(r % kBlockPts);
        g.row_of_rank.push_back(r);
        g.ijk.push_back(g.blocks[size_t(3 * s)] * kBlock + (l % kBlock) - nr);
        g.ijk.push_back(g.blocks[size_t(3 * s + 1)] * kBlock + ((l / kBlock) % kBlock) - nr);
        g.ijk.push_back(g.blocks[size_t(3 * s + 2)] * kBlock + (l / (kBlock * kBlock)) - nr);
    }
    g.n = rank;
    g.block_nbr.assign(size_t(g.n_blocks) * 6, -1);
    for (int64_t s = 0; s < g.n_blocks; ++s) {
        const int b[3] = {g.blocks[size_t(3 * s)], g.blocks[size_t(3 * s + 1)], g.blocks[size_t(3 * s + 2)]};
        for (int f = 0; f < 6; ++f) {
            int c[3] = {b[0], b[1], b[2]};
            c[f / 2] += (f % 2) ? 1 : -1;
            if (c[0] < 0 || c[1] < 0 || c[2] < 0 || c[0] >= nb || c[1] >= nb || c[2] >= nb) continue;
            g.block_nbr[size_t(6 * s + f)] = g.slot_of_block[(size_t(c[2]) * nb + c[1]) * nb + c[0]];
        }
    }
}

void build_row_neighbours(const HostGrid& g, std::vector<int32_t>& nbr_rows) {
    nbr_rows.assign(size_t(g.n_rows) * kNbr, -1);
    for (int64_t p = 0; p < g.n; ++p) {
        const int i = g.ijk[size_t(3 * p)], j = g.ijk[size_t(3 * p + 1)], k = g.ijk[size_t(3 * p + 2)];
        int32_t* out = &nbr_rows[size_t(g.row_of_rank[size_t(p)]) * kNbr];
        int c = 0;
        for (int axis = 0; axis < 3; ++axis)
            for (int s = -kHalf; s <= kHalf; ++s) {
                if (s == 0) continue;
                const int64_t r = g.row_of(i + (axis == 0 ? s : 0), j + (axis == 1 ? s : 0), k + (axis == 2 ? s : 0));
                out[c++] = int32_t(r);
            }
    }
}

void build_projectors(const HostGrid& g, const chf_atoms& atoms, const chf_pp& pp, HostProj& out) {
    const double h = g.h;
    const double rc = pp.r_c;
    const double rcut2 = pp.r_cut * pp.r_cut;
    const double pi = 3.14159265358979323846;
    const double ns = std::sqrt(4.0 / (std::sqrt(pi) * rc * rc * rc));
    const double np = std::sqrt(8.0 / (3.0 * std::sqrt(pi) * rc * rc * rc * rc * rc));
    const double y00 = 1.0 / std::sqrt(4.0 * pi);
    const double y1 = std::sqrt(3.0 / (4.0 * pi));
    out = HostProj{};
    for (int a = 0; a < atoms.n_atoms; ++a)
        if (atoms.species_host[a] == 0) out.atom_index.push_back(a);
    out.n_proj = int64_t(out.atom_index.size());
    const int64_t np_atoms = out.n_proj;
    // per projector atom: support rows ascending and the four projector values
    std::vector<std::vector<int32_t>> rows_of(static_cast<size_t>(np_atoms));
    std::vector<std::vector<double>> beta_of(static_cast<size_t>(np_atoms));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t pa = 0; pa < np_atoms; ++pa) {
        const double* X = atoms.pos_host + 3 * out.atom_index[size_t(pa)];
        int lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::max(-g.n_r, int(std::floor((X[d] - pp.r_cut) / h)) - 1);
            hi[d] = std::min(g.n_r, int(std::ceil((X[d] + pp.r_cut) / h)) + 1);
        }
        std::vector<std::pair<int32_t, int>> tmp;
        std::vector<double> tmpb;
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    if (!g.inside(i, j, k)) continue;
                    const double dx = double(i) * h - X[0];
                    const double dy = double(j) * h - X[1];
                    const double dz = double(k) * h - X[2];
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    if (!(d2 <= rcut2)) continue;
                    const double gauss = std::exp(-d2 / (2.0 * rc * rc));
                    tmp.emplace_back(int32_t(g.row_of(i, j, k)), int(tmp.size()));
                    tmpb.push_back(ns * y00 * gauss);
                    tmpb.push_back(np * y1 * gauss * dx);
                    tmpb.push_back(np * y1 * gauss * dy);
                    tmpb.push_back(np * y1 * gauss * dz);
                }
        std::sort(tmp.begin(), tmp.end());
        auto& R = rows_of[size_t(pa)];
        auto& Bv = beta_of[size_t(pa)];
        R.reserve(tmp.size());
        Bv.reserve(4 * tmp.size());
        for (auto& rl : tmp) {
            R.push_back(rl.first);
            for (int m = 0; m < 4; ++m) Bv.push_back(tmpb[size_t(4 * rl.second + m)]);
        }
    }
    out.sup_off.assign(size_t(np_atoms) + 1, 0);
    for (int64_t pa = 0; pa < np_atoms; ++pa)
        out.sup_off[size_t(pa) + 1] = out.sup_off[size_t(pa)] + int64_t(rows_of[size_t(pa)].size());
    const int64_t pairs = out.sup_off.back();
    out.sup_row.resize(size_t(pairs));
    out.sup_beta.resize(size_t(pairs) * 4);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t pa = 0; pa < np_atoms; ++pa) {
        std::copy(rows_of[size_t(pa)].begin(), rows_of[size_t(pa)].end(), out.sup_row.begin() + out.sup_off[size_t(pa)]);
        std::copy(beta_of[size_t(pa)].begin(), beta_of[size_t(pa)].end(),
                  out.sup_beta.begin() + 4 * out.sup_off[size_t(pa)]);
        std::vector<int32_t>().swap(rows_of[size_t(pa)]);
        std::vector<double>().swap(beta_of[size_t(pa)]);
    }
    // scatter entries bucketed by row, atoms ascending within a row
    out.ent_off.assign(size_t(g.n_rows) + 1, 0);
    for (int64_t e = 0; e < pairs; ++e) out.ent_off[size_t(out.sup_row[size_t(e)]) + 1]++;
    for (int64_t r = 0; r < g.n_rows; ++r) out.ent_off[size_t(r) + 1] += out.ent_off[size_t(r)];
    out.ent_atom.assign(size_t(pairs), 0);
    out.ent_beta.assign(size_t(pairs) * 4, 0.0);
    // each thread owns a contiguous range of rows and scans all pairs in
    // atom order, so the entries of a row stay atom-ascending
#pragma omp parallel
    {
        int nt = 1, tid = 0;
#ifdef _OPENMP
        nt = omp_get_num_threads();
        tid = omp_get_thread_num();
#endif
        const int64_t r0 = g.n_rows * tid / nt, r1 = g.n_rows * (tid + 1) / nt;
        std::vector<int64_t> fill(out.ent_off.begin() + r0, out.ent_off.begin() + r1);
        for (int64_t pa = 0; pa < np_atoms; ++pa)
            for (int64_t e = out.sup_off[size_t(pa)]; e < out.sup_off[size_t(pa) + 1]; ++e) {
                const int64_t r = out.sup_row[size_t(e)];
                if (r < r0 || r >= r1) continue;
                const int64_t dst = fill[size_t(r - r0)]++;
                out.ent_atom[size_t(dst)] = int32_t(pa);
                for (int m = 0; m < 4; ++m) out.ent_beta[size_t(4 * dst + m)] = out.sup_beta[size_t(4 * e + m)];
            }
    }
}

void build_block_atoms(const HostGrid& g, HostProj& P) {
    P.blk_atom_off.assign(size_t(g.n_blocks) + 1, 0);
    P.blk_atoms.clear();
    P.ent_slot.assign(P.ent_atom.size(), 0);
    P.max_block_atoms = 0;
    std::vector<int32_t> list;
    for (int64_t b = 0; b < g.n_blocks; ++b) {
        const int64_t e0 = P.ent_off[size_t(b * kBlockPts)], e1 = P.ent_off[size_t((b + 1) * kBlockPts)];
        list.assign(P.ent_atom.begin() + e0, P.ent_atom.begin() + e1);
        std::sort(list.begin(), list.end());
        list.erase(std::unique(list.begin(), list.end()), list.end());
        P.max_block_atoms = std::max(P.max_block_atoms, int(list.size()));
        for (int64_t e = e0; e < e1; ++e) {
            const auto it = std::lower_bound(list.begin(), list.end(), P.ent_atom[size_t(e)]);
            P.ent_slot[size_t(e)] = uint8_t(std::min<ptrdiff_t>(255, it - list.begin()));
        }
        P.blk_atoms.insert(P.blk_atoms.end(), list.begin(), list.end());
        P.blk_atom_off[size_t(b) + 1] = int64_t(P.blk_atoms.size());
    }
}

}  // namespace chf
