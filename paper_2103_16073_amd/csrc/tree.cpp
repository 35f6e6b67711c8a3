// Host octree and interaction lists (Section 3.3: space partitioned by an octree whose
// smallest boxes are larger than the near cutoff r_c).
//
// Uniform-depth octree over the bounding cube of the mesh: the leaf level L is the smallest
// depth whose non-empty leaves hold at most `leaf_max` element centroids on average, subject to
// the leaf side staying above r_c (so every near pair lies in neighbouring leaves).  Elements are sorted by
// the Morton code of their centroid; only non-empty boxes are kept at every level.
//   P2P list of a leaf: the non-empty leaves of its 3x3x3 neighbourhood (itself included).
//   M2L list of a box at level l >= 2: children of its parent's neighbours that are not its own
//   neighbours; the translation t = c_target - c_source is (dx,dy,dz) * d_l with
//   max(|dx|,|dy|,|dz|) in {2,3}: 316 directions, 15 distinct lengths.
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"

namespace fmm {

static inline uint64_t spread3(uint64_t v) {
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}
static inline uint64_t compact3(uint64_t v) {
    v &= 0x1249249249249249ULL;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ULL;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00fULL;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffULL;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffULL;
    v = (v ^ (v >> 32)) & 0x1fffff;
    return v;
}
static inline uint64_t morton(uint64_t x, uint64_t y, uint64_t z) { return spread3(x) | spread3(y) << 1 | spread3(z) << 2; }
static inline void demorton(uint64_t c, int64_t &x, int64_t &y, int64_t &z) {
    x = (int64_t)compact3(c);
    y = (int64_t)compact3(c >> 1);
    z = (int64_t)compact3(c >> 2);
}

static int64_t find_code(const std::vector<uint64_t> &codes, uint64_t c) {
    auto it = std::lower_bound(codes.begin(), codes.end(), c);
    if (it == codes.end() || *it != c) return -1;
    return it - codes.begin();
}

void build_tree(const double *cen, int64_t n, const double *vlo, const double *vhi, double rc, int leaf_max,
                int max_depth, double min_leaf, TreeHost &T) {
    const int DMAX = 21;
    max_depth = std::min(std::max(max_depth, 2), DMAX);
    double ext = 0.0, mid[3];
    for (int d = 0; d < 3; ++d) {
        ext = std::max(ext, vhi[d] - vlo[d]);
        mid[d] = 0.5 * (vlo[d] + vhi[d]);
    }
    T.side = ext * (1.0 + 1e-6) + 1e-9;
    for (int d = 0; d < 3; ++d) T.lo[d] = mid[d] - 0.5 * T.side;

    // finest integer coordinates and codes at DMAX
    std::vector<uint64_t> fine(n);
    const double scale = (double)(1u << DMAX) / T.side;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t ic[3];
        for (int d = 0; d < 3; ++d) {
            double q = std::floor((cen[3 * i + d] - T.lo[d]) * scale);
            q = std::min(std::max(q, 0.0), (double)((1u << DMAX) - 1));
            ic[d] = (uint64_t)q;
        }
        fine[i] = morton(ic[0], ic[1], ic[2]);
    }
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return fine[a] < fine[b]; });

    // choose the depth
    int L = 2, best = -1, best_occ = 0;
    for (L = 2; L <= max_depth; ++L) {
        double dl = T.side / (double)(1u << L);
        if (dl <= rc && L > 2) break;
        if (dl < min_leaf && L > 2) break;  // leaves no smaller than min_leaf (the wavelength bound)
        int shift = 3 * (DMAX - L), occ = 0, run = 0;
        int64_t nbox = 0;
        uint64_t prev = ~0ULL;
        for (int64_t i = 0; i < n; ++i) {
            uint64_t c = fine[order[i]] >> shift;
            if (c != prev) ++nbox;
            run = (c == prev) ? run + 1 : 1;
            prev = c;
            occ = std::max(occ, run);
        }
        best = L;
        best_occ = occ;
        if ((double)n / (double)nbox <= (double)leaf_max) break;
    }
    L = best;
    T.depth = L;
    T.max_occ = best_occ;
    T.perm = order;

    // levels
    T.lv.assign(L + 1, LevelHost());
    for (int l = 0; l <= L; ++l) {
        T.lv[l].level = l;
        T.lv[l].side = T.side / (double)(1u << l);
    }
    {
        int shift = 3 * (DMAX - L);
        auto &leaf = T.lv[L];
        T.leaf_start.clear();
        uint64_t prev = ~0ULL;
        for (int64_t i = 0; i < n; ++i) {
            uint64_t c = fine[order[i]] >> shift;
            if (c != prev) {
                leaf.code.push_back(c);
                T.leaf_start.push_back((int32_t)i);
                prev = c;
            }
        }
        T.leaf_start.push_back((int32_t)n);
    }
    for (int l = L - 1; l >= 0; --l) {
        auto &up = T.lv[l];
        auto &dn = T.lv[l + 1];
        for (uint64_t c : dn.code) {
            uint64_t pc = c >> 3;
            if (up.code.empty() || up.code.back() != pc) up.code.push_back(pc);
        }
        dn.parent.resize(dn.code.size());
        dn.octant.resize(dn.code.size());
        up.child_start.assign(up.code.size() + 1, 0);
        for (size_t i = 0; i < dn.code.size(); ++i) {
            int64_t pi = find_code(up.code, dn.code[i] >> 3);
            dn.parent[i] = (int32_t)pi;
            dn.octant[i] = (int8_t)(dn.code[i] & 7);
            up.child_start[pi + 1]++;
        }
        for (size_t i = 0; i < up.code.size(); ++i) up.child_start[i + 1] += up.child_start[i];
        up.child_list.resize(dn.code.size());
        std::iota(up.child_list.begin(), up.child_list.end(), 0);  // children are contiguous
    }

    // P2P neighbour lists at the leaf level
    {
        auto &leaf = T.lv[L];
        const int64_t nb = (int64_t)leaf.code.size(), lim = (int64_t)1 << L;
        T.nbr_start.assign(nb + 1, 0);
        T.nbr_list.clear();
        for (int64_t b = 0; b < nb; ++b) {
            int64_t x, y, z;
            demorton(leaf.code[b], x, y, z);
            std::vector<int32_t> tmp;
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int64_t X = x + dx, Y = y + dy, Z = z + dz;
                        if (X < 0 || Y < 0 || Z < 0 || X >= lim || Y >= lim || Z >= lim) continue;
                        int64_t s = find_code(leaf.code, morton(X, Y, Z));
                        if (s >= 0) tmp.push_back((int32_t)s);
                    }
            std::sort(tmp.begin(), tmp.end());
            T.nbr_list.insert(T.nbr_list.end(), tmp.begin(), tmp.end());
            T.nbr_start[b + 1] = (int32_t)T.nbr_list.size();
        }
    }

    // distinct |t|^2 of the M2L offsets
    std::vector<int> t2;
    for (int dx = -3; dx <= 3; ++dx)
        for (int dy = -3; dy <= 3; ++dy)
            for (int dz = -3; dz <= 3; ++dz)
                if (std::max({std::abs(dx), std::abs(dy), std::abs(dz)}) >= 2) t2.push_back(dx * dx + dy * dy + dz * dz);
    std::sort(t2.begin(), t2.end());
    t2.erase(std::unique(t2.begin(), t2.end()), t2.end());

    // M2L lists at levels 2..L
    for (int l = 2; l <= L; ++l) {
        auto &lv = T.lv[l];
        auto &pl = T.lv[l - 1];
        const int64_t lim_p = (int64_t)1 << (l - 1);
        lv.m2l_tau_of_dir.assign(343, -1);
        lv.m2l_taus.clear();
        for (int v : t2) lv.m2l_taus.push_back(std::sqrt((double)v) * lv.side);
        for (int dx = -3; dx <= 3; ++dx)
            for (int dy = -3; dy <= 3; ++dy)
                for (int dz = -3; dz <= 3; ++dz)
                    if (std::max({std::abs(dx), std::abs(dy), std::abs(dz)}) >= 2) {
                        int v = dx * dx + dy * dy + dz * dz;
                        lv.m2l_tau_of_dir[dir_of_offset(dx, dy, dz)] =
                            (int)(std::lower_bound(t2.begin(), t2.end(), v) - t2.begin());
                    }
        const int64_t nb = (int64_t)lv.code.size();
        lv.m2l_start.assign(nb + 1, 0);
        lv.m2l_src.clear();
        lv.m2l_dir.clear();
        for (int64_t b = 0; b < nb; ++b) {
            int64_t x, y, z, px, py, pz;
            demorton(lv.code[b], x, y, z);
            demorton(pl.code[lv.parent[b]], px, py, pz);
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int64_t X = px + dx, Y = py + dy, Z = pz + dz;
                        if (X < 0 || Y < 0 || Z < 0 || X >= lim_p || Y >= lim_p || Z >= lim_p) continue;
                        int64_t q = find_code(pl.code, morton(X, Y, Z));
                        if (q < 0) continue;
                        for (int32_t c = pl.child_start[q]; c < pl.child_start[q + 1]; ++c) {
                            int64_t cx, cy, cz;
                            demorton(lv.code[c], cx, cy, cz);
                            int64_t ox = x - cx, oy = y - cy, oz = z - cz;
                            if (std::max({std::llabs(ox), std::llabs(oy), std::llabs(oz)}) < 2) continue;
                            lv.m2l_src.push_back(c);
                            lv.m2l_dir.push_back((int16_t)dir_of_offset((int)ox, (int)oy, (int)oz));
                        }
                    }
            lv.m2l_start[b + 1] = (int32_t)lv.m2l_src.size();
        }
    }
}

// box centre of a level-l box from its Morton code
void box_center(const TreeHost &T, int l, uint64_t code, double *c) {
    int64_t x, y, z;
    demorton(code, x, y, z);
    double d = T.side / (double)(1u << l);
    c[0] = T.lo[0] + (x + 0.5) * d;
    c[1] = T.lo[1] + (y + 0.5) * d;
    c[2] = T.lo[2] + (z + 0.5) * d;
}

}  // namespace fmm
