// Host mesh builder: conformal base grid plus recursive 3x3x3 refinement of
// selected leaves (the paper's Assumption 1 with 3-partitioning, Sec. 2.3),
// flattened into the arrays the kernels consume.
//
//   * cells sorted by (level, k, j, i);
//   * conforming faces (same level on both sides) grouped by normal axis;
//   * hanging child faces: one per (fine cell, side) whose neighbour is a
//     coarser leaf; the Riemann problem is solved there (Sec. 2.3: on the
//     finest resolution, against a virtual cell);
//   * coarse sides: every (cell, side) covered by finer leaves, with the list
//     of its child faces in increasing fine-cell order (restriction order);
//   * skeleton: cells on either side of a resolution transition (Sec. 3);
//     enclave: the rest.
#include <algorithm>
#include <iterator>
#include <cstdio>
#include <unordered_map>

#include "adg_internal.h"

namespace adg {
namespace {

struct Key {
    int l, i, j, k;
};

inline bool key_less(const Key &a, const Key &b)
{
    if (a.l != b.l) return a.l < b.l;
    if (a.k != b.k) return a.k < b.k;
    if (a.j != b.j) return a.j < b.j;
    return a.i < b.i;
}

inline uint64_t pack(int l, int i, int j, int k)
{
    // 2 bits of level, 20 bits per coordinate (up to 1,048,575 cells per axis)
    return (uint64_t(l) << 60) | (uint64_t(uint32_t(k)) << 40) | (uint64_t(uint32_t(j)) << 20) |
           uint64_t(uint32_t(i));
}

inline int64_t pow3(int e)
{
    int64_t r = 1;
    while (e-- > 0) r *= 3;
    return r;
}

}  // namespace

std::string build_host_mesh(const adg_instance_desc &d, HostMesh &m, bool leaves_only)
{
    char buf[256];
    if (d.order < 0 || d.order > NMAX - 1) return "unsupported: order must be in [0, 7]";
    if (d.max_level < 0 || d.max_level > LMAX) return "unsupported: max_level must be in [0, 3]";
    if ((d.periodic_mask & 7u) != 7u) return "unsupported: only fully periodic boxes";
    for (int a = 0; a < 3; ++a) {
        if (d.n[a] < 1) return "base cell counts must be >= 1";
        if (!(d.hi[a] > d.lo[a])) return "domain box needs hi > lo";
        if (int64_t(d.n[a]) * pow3(d.max_level) >= (1 << 20)) return "unsupported: mesh too fine for the cell index";
    }
    if (!(d.gamma > 1.0)) return "gamma must be > 1";
    if (!(d.cfl > 0.0)) return "cfl must be > 0";
    if (d.picard_iters < 0) return "picard_iters must be >= 0";
    if (d.n_refine < 0 || (d.n_refine > 0 && d.refine == nullptr)) return "refine list missing";

    m.N = d.order + 1;
    for (int a = 0; a < 3; ++a) { m.n[a] = d.n[a]; m.lo[a] = d.lo[a]; m.hi[a] = d.hi[a]; }
    m.max_level = d.max_level;

    // refine rows grouped per level
    std::vector<std::vector<Key>> ref(LMAX + 1);
    for (int64_t r = 0; r < d.n_refine; ++r) {
        Key k{d.refine[4 * r], d.refine[4 * r + 1], d.refine[4 * r + 2], d.refine[4 * r + 3]};
        if (k.l < 0 || k.l >= d.max_level) {
            std::snprintf(buf, sizeof buf, "refine row %lld: level %d not below max_level", (long long)r, k.l);
            return buf;
        }
        ref[k.l].push_back(k);
    }

    // Leaves level by level: level 0 is the base grid, level l+1 the children
    // of the cells refined at level l, and each level loses its refined
    // cells.  Every list is kept sorted by packed key, i.e. by (level, k, j, i),
    // so the checks are binary searches, the removal is a merge, and the
    // children are emitted in order (no hashing, no global sort).
    auto ki = [](uint64_t p) { return int(p & 0xFFFFF); };
    auto kj = [](uint64_t p) { return int((p >> 20) & 0xFFFFF); };
    auto kk = [](uint64_t p) { return int((p >> 40) & 0xFFFFF); };
    std::vector<std::vector<uint64_t>> rk(LMAX + 1);
    for (int l = 0; l < d.max_level; ++l) {
        const int64_t ext[3] = {d.n[0] * pow3(l), d.n[1] * pow3(l), d.n[2] * pow3(l)};
        rk[l].reserve(ref[l].size());
        for (const Key &k : ref[l]) {
            if (k.i < 0 || k.j < 0 || k.k < 0 || k.i >= ext[0] || k.j >= ext[1] || k.k >= ext[2])
                return "refine row outside the grid";
            rk[l].push_back(pack(l, k.i, k.j, k.k));
        }
        std::sort(rk[l].begin(), rk[l].end());
        if (std::adjacent_find(rk[l].begin(), rk[l].end()) != rk[l].end())
            return "refine row names a cell that is not a leaf (or a duplicate)";
        if (l > 0)
            for (uint64_t key : rk[l])
                if (!std::binary_search(rk[l - 1].begin(), rk[l - 1].end(),
                                        pack(l - 1, ki(key) / 3, kj(key) / 3, kk(key) / 3)))
                    return "refine row names a cell that is not a leaf (or a duplicate)";
    }
    std::vector<uint64_t> all, lev, next;
    lev.reserve(size_t(d.n[0]) * d.n[1] * d.n[2]);
    for (int k = 0; k < d.n[2]; ++k)
        for (int j = 0; j < d.n[1]; ++j)
            for (int i = 0; i < d.n[0]; ++i) lev.push_back(pack(0, i, j, k));
    for (int l = 0;; ++l) {
        const std::vector<uint64_t> &r = rk[l];  // empty at max_level
        std::set_difference(lev.begin(), lev.end(), r.begin(), r.end(), std::back_inserter(all));
        if (l >= d.max_level) break;
        // children of the refined cells, in (k, j, i) order: parents grouped by
        // their k, then j; child rows 3 kp + c, 3 jp + b, then 3 ip + a
        next.clear();
        next.reserve(27 * r.size());
        for (size_t p = 0; p < r.size();) {
            size_t q = p;
            while (q < r.size() && kk(r[q]) == kk(r[p])) ++q;
            for (int c = 0; c < 3; ++c)
                for (size_t s0 = p; s0 < q;) {
                    size_t e = s0;
                    while (e < q && kj(r[e]) == kj(r[s0])) ++e;
                    for (int b = 0; b < 3; ++b)
                        for (size_t t = s0; t < e; ++t)
                            for (int a = 0; a < 3; ++a)
                                next.push_back(pack(l + 1, 3 * ki(r[t]) + a, 3 * kj(r[t]) + b, 3 * kk(r[t]) + c));
                    s0 = e;
                }
            p = q;
        }
        lev.swap(next);
    }
    std::vector<Key> cells;
    cells.reserve(all.size());
    for (uint64_t p : all) cells.push_back(Key{int(p >> 60), ki(p), kj(p), kk(p)});
    if (cells.size() > size_t(INT32_MAX) / 8) return "too many cells";
    m.nc = int64_t(cells.size());
    m.level.resize(m.nc);
    m.ijk.resize(3 * m.nc);
    for (int64_t c = 0; c < m.nc; ++c) {
        m.level[c] = int8_t(cells[c].l);
        m.ijk[3 * c] = cells[c].i;
        m.ijk[3 * c + 1] = cells[c].j;
        m.ijk[3 * c + 2] = cells[c].k;
    }
    if (leaves_only) return "";
    std::unordered_map<uint64_t, int32_t> index;
    index.reserve(cells.size() * 2);
    for (int64_t c = 0; c < m.nc; ++c) index.emplace(all[size_t(c)], int32_t(c));

    // side classification
    std::vector<int8_t> kind(6 * m.nc);
    std::vector<int32_t> nbr(6 * m.nc, -1);
    for (int64_t c = 0; c < m.nc; ++c) {
        int l = m.level[c];
        for (int s = 0; s < 6; ++s) {
            int ax = s / 2, dir = (s & 1) ? 1 : -1;
            int q[3] = {m.ijk[3 * c], m.ijk[3 * c + 1], m.ijk[3 * c + 2]};
            int64_t ext = d.n[ax] * pow3(l);
            q[ax] = int((q[ax] + dir + ext) % ext);
            auto it = index.find(pack(l, q[0], q[1], q[2]));
            if (it != index.end()) {
                kind[6 * c + s] = SIDE_CONFORMING;
                nbr[6 * c + s] = it->second;
                continue;
            }
            kind[6 * c + s] = SIDE_COARSE;
            for (int lc = l - 1; lc >= 0; --lc) {
                int64_t f = pow3(l - lc);
                auto jt = index.find(pack(lc, int(q[0] / f), int(q[1] / f), int(q[2] / f)));
                if (jt != index.end()) {
                    kind[6 * c + s] = SIDE_FINE;
                    nbr[6 * c + s] = jt->second;
                    break;
                }
            }
        }
    }

    // conforming faces from the minus cell's plus side
    for (int a = 0; a < 3; ++a) { m.face_m[a].clear(); m.face_p[a].clear(); }
    for (int64_t c = 0; c < m.nc; ++c)
        for (int a = 0; a < 3; ++a)
            if (kind[6 * c + 2 * a + 1] == SIDE_CONFORMING) {
                m.face_m[a].push_back(int32_t(c));
                m.face_p[a].push_back(nbr[6 * c + 2 * a + 1]);
            }

    // hanging child faces in increasing fine-cell order
    m.hang.clear();
    std::vector<char> is_skel(m.nc, 0);
    for (int64_t c = 0; c < m.nc; ++c)
        for (int s = 0; s < 6; ++s) {
            if (kind[6 * c + s] != SIDE_FINE) continue;
            int ax = s / 2;
            int t1 = (ax == 0) ? 1 : 0, t2 = (ax == 2) ? 1 : 2;
            int32_t C = nbr[6 * c + s];
            int dl = m.level[c] - m.level[C];
            int64_t r = pow3(dl);
            HostMesh::Hang h;
            h.fine = int32_t(c);
            h.coarse = C;
            h.d = int8_t(ax);
            h.fine_minus = int8_t(s & 1);  // fine cell on the minus side if its plus side hangs
            h.dl = int8_t(dl);
            h.s1 = int8_t(m.ijk[3 * c + t1] - r * m.ijk[3 * C + t1]);
            h.s2 = int8_t(m.ijk[3 * c + t2] - r * m.ijk[3 * C + t2]);
            m.hang.push_back(h);
            is_skel[c] = 1;
            is_skel[C] = 1;
        }
    // coarse sides and their children (CSR), children sorted by fine cell
    std::unordered_map<int64_t, int32_t> cs_index;  // 6*cell+side -> coarse slot
    m.coarse_cell.clear();
    m.coarse_side.clear();
    for (int64_t c = 0; c < m.nc; ++c)
        for (int s = 0; s < 6; ++s)
            if (kind[6 * c + s] == SIDE_COARSE) {
                cs_index.emplace(6 * c + s, int32_t(m.coarse_cell.size()));
                m.coarse_cell.push_back(int32_t(c));
                m.coarse_side.push_back(int8_t(s));
            }
    std::vector<int32_t> count(m.coarse_cell.size() + 1, 0);
    std::vector<int32_t> slot_of(m.hang.size());
    for (size_t h = 0; h < m.hang.size(); ++h) {
        const auto &H = m.hang[h];
        int coarse_side = 2 * H.d + (H.fine_minus ? 0 : 1);
        auto it = cs_index.find(6 * int64_t(H.coarse) + coarse_side);
        if (it == cs_index.end()) return "internal: hanging face without a coarse side";
        slot_of[h] = it->second;
        count[it->second + 1]++;
    }
    for (size_t i = 1; i < count.size(); ++i) count[i] += count[i - 1];
    m.coarse_ptr = count;
    m.coarse_child.assign(m.hang.size(), 0);
    std::vector<int32_t> fill(count.begin(), count.end() - 1);
    for (size_t h = 0; h < m.hang.size(); ++h) m.coarse_child[fill[slot_of[h]]++] = int32_t(h);
    for (size_t i = 0; i + 1 < m.coarse_ptr.size(); ++i)
        if (m.coarse_ptr[i] == m.coarse_ptr[i + 1]) return "internal: coarse side without children";

    m.skeleton.clear();
    m.enclave.clear();
    for (int64_t c = 0; c < m.nc; ++c) (is_skel[c] ? m.skeleton : m.enclave).push_back(int32_t(c));
    return "";
}

}  // namespace adg
