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
#include <memory>
#include <cstdio>
#include <thread>

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
    {
        size_t leaves = size_t(d.n[0]) * d.n[1] * d.n[2];
        for (int l = 0; l < d.max_level; ++l) leaves += 26 * rk[l].size();
        all.reserve(leaves);
    }
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
    if (all.size() > size_t(INT32_MAX) / 8) return "too many cells";
    m.nc = int64_t(all.size());
    m.level.resize(size_t(m.nc));
    m.ijk.resize(size_t(3 * m.nc));
    parallel_for(m.nc, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            const uint64_t p = all[size_t(c)];
            m.level[size_t(c)] = int8_t(p >> 60);
            m.ijk[size_t(3 * c)] = ki(p);
            m.ijk[size_t(3 * c + 1)] = kj(p);
            m.ijk[size_t(3 * c + 2)] = kk(p);
        }
    });
    std::vector<uint64_t>().swap(all);
    if (leaves_only) return "";
    CellIndex index;
    index.build(m);

    // side classification: the same-level neighbour, else the coarser leaf
    // that covers the side (fine side), else finer leaves (coarse side).  The
    // x neighbour of a leaf is usually the next or previous entry of the table.
    // every entry is written by the loop below (first touch on its threads)
    std::unique_ptr<int8_t[]> kind(new int8_t[size_t(std::max<int64_t>(6 * m.nc, 1))]);
    std::unique_ptr<int32_t[]> nbr(new int32_t[size_t(std::max<int64_t>(6 * m.nc, 1))]);
    parallel_for(m.nc, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            const int l = m.level[size_t(c)];
            const int32_t *p = &m.ijk[size_t(3 * c)];
            for (int s = 0; s < 6; ++s) {
                const int ax = s / 2, dir = (s & 1) ? 1 : -1;
                int64_t q[3] = {p[0], p[1], p[2]};
                const int64_t ext = d.n[ax] * pow3(l);
                q[ax] += dir;
                if (q[ax] < 0) q[ax] += ext;
                else if (q[ax] >= ext) q[ax] -= ext;
                int32_t f = -1;
                const int64_t g = c + dir;
                if (ax == 0 && g >= 0 && g < m.nc && m.level[size_t(g)] == l && m.ijk[size_t(3 * g)] == q[0] &&
                    m.ijk[size_t(3 * g + 1)] == q[1] && m.ijk[size_t(3 * g + 2)] == q[2])
                    f = int32_t(g);
                if (f < 0) f = index.find(l, q[0], q[1], q[2]);
                if (f >= 0) {
                    kind[size_t(6 * c + s)] = SIDE_CONFORMING;
                    nbr[size_t(6 * c + s)] = f;
                    continue;
                }
                kind[size_t(6 * c + s)] = SIDE_COARSE;
                nbr[size_t(6 * c + s)] = -1;
                for (int lc = l - 1; lc >= 0; --lc) {
                    const int64_t r = pow3(l - lc);
                    f = index.find(lc, q[0] / r, q[1] / r, q[2] / r);
                    if (f >= 0) {
                        kind[size_t(6 * c + s)] = SIDE_FINE;
                        nbr[size_t(6 * c + s)] = f;
                        break;
                    }
                }
            }
        }
    });

    // Lists, each in increasing cell order, then side order: conforming faces
    // (from the minus cell's plus side) per axis, hanging child faces (one per
    // fine side), coarse sides, skeleton cells (a side that is not
    // conforming: the fine or the coarse cell of a hanging face) and enclave
    // cells.  Counted per chunk of cells, then written at the chunk offsets.
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(1024, m.nc / 2048));
    auto cbeg = [&](int64_t t) { return m.nc * t / nch; };
    struct Count { int64_t face[3], hang, coarse, skel; };
    std::vector<Count> cnt(size_t(nch) + 1, Count{{0, 0, 0}, 0, 0, 0});
    auto skeletal = [&](int64_t c) {
        for (int s = 0; s < 6; ++s)
            if (kind[size_t(6 * c + s)] != SIDE_CONFORMING) return true;
        return false;
    };
    parallel_for(nch, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            Count &n = cnt[size_t(t) + 1];
            for (int64_t c = cbeg(t); c < cbeg(t + 1); ++c) {
                for (int a = 0; a < 3; ++a) n.face[a] += kind[size_t(6 * c + 2 * a + 1)] == SIDE_CONFORMING;
                for (int s = 0; s < 6; ++s) {
                    n.hang += kind[size_t(6 * c + s)] == SIDE_FINE;
                    n.coarse += kind[size_t(6 * c + s)] == SIDE_COARSE;
                }
                n.skel += skeletal(c);
            }
        }
    }, 1);
    for (int64_t t = 0; t < nch; ++t) {
        Count &a = cnt[size_t(t) + 1];
        const Count &b = cnt[size_t(t)];
        for (int x = 0; x < 3; ++x) a.face[x] += b.face[x];
        a.hang += b.hang;
        a.coarse += b.coarse;
        a.skel += b.skel;
    }
    const Count &tot = cnt[size_t(nch)];
    for (int a = 0; a < 3; ++a) {
        m.face_m[a].resize(size_t(tot.face[a]));
        m.face_p[a].resize(size_t(tot.face[a]));
    }
    m.hang.resize(size_t(tot.hang));
    m.coarse_cell.resize(size_t(tot.coarse));
    m.coarse_side.resize(size_t(tot.coarse));
    m.skeleton.resize(size_t(tot.skel));
    m.enclave.resize(size_t(m.nc - tot.skel));
    parallel_for(nch, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            Count o = cnt[size_t(t)];
            int64_t enc = cbeg(t) - o.skel;
            for (int64_t c = cbeg(t); c < cbeg(t + 1); ++c) {
                for (int a = 0; a < 3; ++a)
                    if (kind[size_t(6 * c + 2 * a + 1)] == SIDE_CONFORMING) {
                        m.face_m[a][size_t(o.face[a])] = int32_t(c);
                        m.face_p[a][size_t(o.face[a]++)] = nbr[size_t(6 * c + 2 * a + 1)];
                    }
                for (int s = 0; s < 6; ++s) {
                    const int8_t k = kind[size_t(6 * c + s)];
                    if (k == SIDE_FINE) {
                        const int ax = s / 2;
                        const int t1a = (ax == 0) ? 1 : 0, t2a = (ax == 2) ? 1 : 2;
                        const int32_t C = nbr[size_t(6 * c + s)];
                        const int dl = m.level[size_t(c)] - m.level[size_t(C)];
                        const int64_t r = pow3(dl);
                        HostMesh::Hang &h = m.hang[size_t(o.hang++)];
                        h.fine = int32_t(c);
                        h.coarse = C;
                        h.d = int8_t(ax);
                        h.fine_minus = int8_t(s & 1);  // fine cell on the minus side if its plus side hangs
                        h.dl = int8_t(dl);
                        h.s1 = int8_t(m.ijk[size_t(3 * c + t1a)] - r * m.ijk[size_t(3 * C + t1a)]);
                        h.s2 = int8_t(m.ijk[size_t(3 * c + t2a)] - r * m.ijk[size_t(3 * C + t2a)]);
                    } else if (k == SIDE_COARSE) {
                        // the slot is kept in the coarse side's (otherwise unused) nbr entry
                        nbr[size_t(6 * c + s)] = int32_t(o.coarse);
                        m.coarse_cell[size_t(o.coarse)] = int32_t(c);
                        m.coarse_side[size_t(o.coarse++)] = int8_t(s);
                    }
                }
                if (skeletal(c)) m.skeleton[size_t(o.skel++)] = int32_t(c);
                else m.enclave[size_t(enc++)] = int32_t(c);
            }
        }
    }, 1);

    // coarse sides' children (CSR), children sorted by fine cell
    std::vector<int32_t> count(m.coarse_cell.size() + 1, 0);
    std::vector<int32_t> slot_of(m.hang.size());
    for (size_t h = 0; h < m.hang.size(); ++h) {
        const auto &H = m.hang[h];
        const int64_t cs = 6 * int64_t(H.coarse) + 2 * H.d + (H.fine_minus ? 0 : 1);
        if (kind[cs] != SIDE_COARSE) return "internal: hanging face without a coarse side";
        slot_of[h] = nbr[cs];
        count[nbr[cs] + 1]++;
    }
    for (size_t i = 1; i < count.size(); ++i) count[i] += count[i - 1];
    m.coarse_ptr = count;
    m.coarse_child.assign(m.hang.size(), 0);
    std::vector<int32_t> fill(count.begin(), count.end() - 1);
    for (size_t h = 0; h < m.hang.size(); ++h) m.coarse_child[fill[slot_of[h]]++] = int32_t(h);
    for (size_t i = 0; i + 1 < m.coarse_ptr.size(); ++i)
        if (m.coarse_ptr[i] == m.coarse_ptr[i + 1]) return "internal: coarse side without children";

    return "";
}

void CellIndex::build(const HostMesh &m)
{
    ijk_ = m.ijk.data();
    max_level_ = m.max_level;
    int64_t c = 0;
    for (int l = 0; l <= LMAX; ++l) {
        start_[l].clear();
        rowkey_[l].clear();
        if (l > m.max_level) continue;
        for (int a = 0; a < 3; ++a) ext_[l][a] = m.n[a] * pow3(l);
        const int64_t lb = c;
        while (c < m.nc && m.level[c] == l) ++c;
        const int64_t le = c, rows = ext_[l][1] * ext_[l][2];
        auto row_of = [&](int64_t x) { return int64_t(m.ijk[3 * x + 2]) * ext_[l][1] + m.ijk[3 * x + 1]; };
        dense_[l] = rows <= 4 * (le - lb) + 65536;
        if (dense_[l]) {
            start_[l].resize(size_t(rows) + 1);
            int64_t p = lb;
            for (int64_t r = 0; r < rows; ++r) {
                start_[l][size_t(r)] = int32_t(p);
                while (p < le && row_of(p) == r) ++p;
            }
            start_[l][size_t(rows)] = int32_t(le);
        } else {
            for (int64_t p = lb; p < le; ++p)
                if (p == lb || row_of(p) != row_of(p - 1)) {
                    rowkey_[l].push_back(row_of(p));
                    start_[l].push_back(int32_t(p));
                }
            start_[l].push_back(int32_t(le));
        }
    }
}

int32_t CellIndex::find(int l, int64_t i, int64_t j, int64_t k) const
{
    if (l < 0 || l > max_level_) return -1;
    const int64_t *e = ext_[l];
    if (i < 0 || j < 0 || k < 0 || i >= e[0] || j >= e[1] || k >= e[2]) return -1;
    const int64_t row = k * e[1] + j;
    int64_t s, t;
    if (dense_[l]) {
        s = start_[l][size_t(row)];
        t = start_[l][size_t(row) + 1];
    } else {
        auto it = std::lower_bound(rowkey_[l].begin(), rowkey_[l].end(), row);
        if (it == rowkey_[l].end() || *it != row) return -1;
        const size_t r = size_t(it - rowkey_[l].begin());
        s = start_[l][r];
        t = start_[l][r + 1];
    }
    const int64_t end = t;
    while (s < t) {  // first leaf of the row with i' >= i
        const int64_t mid = (s + t) >> 1;
        if (ijk_[3 * mid] < i) s = mid + 1;
        else t = mid;
    }
    return (s < end && ijk_[3 * s] == i) ? int32_t(s) : -1;
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t min_chunk)
{
    if (n <= 0) return;
    const unsigned hw = std::thread::hardware_concurrency();
    const int64_t nt = std::max<int64_t>(
        1, std::min<int64_t>({int64_t(hw ? hw : 1), 16, (n + min_chunk - 1) / std::max<int64_t>(1, min_chunk)}));
    if (nt == 1) {
        fn(0, n);
        return;
    }
    const int64_t per = (n + nt - 1) / nt;
    std::vector<std::thread> th;
    th.reserve(size_t(nt - 1));
    for (int64_t t = 1; t < nt; ++t) {
        const int64_t b = t * per, e = std::min(n, b + per);
        if (b < e) th.emplace_back(fn, b, e);
    }
    fn(0, std::min(n, per));
    for (auto &x : th) x.join();
}

}  // namespace adg
