// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "adg.h"

namespace adg {

constexpr int NV = 5;       // conserved variables (rho, m1, m2, m3, E)
constexpr int NMAX = 8;     // largest supported N = p + 1
constexpr int LMAX = 3;     // deepest refinement level
constexpr int RMAX = 27;    // 3^LMAX sub-intervals per parent interval

// 1-D operators of one order on [0,1] Gauss-Legendre nodes (host-computed).
struct Basis {
    int N;
    double xi[NMAX], w[NMAX];
    double D[NMAX * NMAX];    // D[a][e] = phi_e'(xi_a)
    double KW[NMAX * NMAX];   // KW[l][j] = (K1^{-1})[l][j] * w_j
    double Kw[NMAX * NMAX];   // Kw[a][e] = int phi_a' phi_e = w_e D[e][a]
    double L[NMAX], R[NMAX];  // phi_e(0), phi_e(1)
};

// Compute the basis of order N (Golub-Welsch nodes, barycentric Lagrange).
bool make_basis(int N, Basis &b);
// Interpolation P[k][e] = phi_e((s + xi_k)/r) and its quadrature-weighted
// transpose Rm[k][e] = (w_e / w_k) P[e][k] / r.
void make_transfer(const Basis &b, int r, int s, double *P, double *Rm);

// Device-side constant table, one entry per N (index N).
struct DevBasis {
    double D[NMAX * NMAX];
    double KW[NMAX * NMAX];
    double Kw[NMAX * NMAX];
    double w[NMAX], winv[NMAX], L[NMAX], R[NMAX], xi[NMAX];
    double KWsum[NMAX];  // row sums sum_j KW[l][j] (time solve from a time-constant state)
};

// Subcell limiter operators of one order (ns = 2N - 1 equal subintervals):
//   A[s][k]   average of phi_k over subinterval s
//   Ap[k][s]  least-squares inverse (A^T A)^{-1} A^T
//   Bf[k][s]  L2 projection of piecewise constants onto the polynomials,
//             A[s][k] / (ns w_k)
constexpr int LIM_NMAX = 7;                 // largest N of the limiter (LDS)
constexpr int LIM_NS = 2 * LIM_NMAX - 1;
struct DevSub {
    double A[LIM_NS * LIM_NMAX], Ap[LIM_NMAX * LIM_NS], Bf[LIM_NMAX * LIM_NS];
};
bool make_subcell(const Basis &b, DevSub &out);

// Per-mesh geometry passed to kernels by value.
struct Geo {
    double inv_dx[LMAX + 1][3];  // 1/dx per level and axis
};

enum SideKind : int8_t { SIDE_CONFORMING = 0, SIDE_FINE = 1, SIDE_COARSE = 2 };

// Host-built mesh of one instance.
struct HostMesh {
    int N = 0;
    int n[3] = {0, 0, 0};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int max_level = 0;
    int64_t nc = 0;
    std::vector<int8_t> level;            // [nc]
    std::vector<int32_t> ijk;             // [3 nc]
    // conforming faces grouped by axis: minus cell, plus cell
    std::vector<int32_t> face_m[3], face_p[3];
    // hanging child faces: fine cell, coarse cell, axis, fine-is-minus,
    // ratio index (r = 3^dl), sub-positions s1 (axis t1), s2 (axis t2)
    struct Hang { int32_t fine, coarse; int8_t d, fine_minus, dl; int8_t s1, s2; };
    std::vector<Hang> hang;
    // coarse sides: (cell, side) with the CSR range of child faces (indices
    // into hang, increasing fine cell) restricted into them
    std::vector<int32_t> coarse_cell;
    std::vector<int8_t> coarse_side;
    std::vector<int32_t> coarse_ptr;      // [n_coarse + 1]
    std::vector<int32_t> coarse_child;    // indices into hang
    std::vector<int32_t> skeleton, enclave;  // cell lists
};

// Returns an empty string on success, otherwise the error text.
// leaves_only: stop after the sorted cell table (level, ijk)
std::string build_host_mesh(const adg_instance_desc &d, HostMesh &m, bool leaves_only = false);

// Leaves of a host mesh looked up by (level, i, j, k).  The cell table is
// sorted by (level, k, j, i), so every level is one block of it and every
// (level, k, j) row one run inside that block, sorted by i.  The index keeps
// the start of every row (a dense table over the level's rows when there are
// at most a few times as many rows as cells, else the sorted list of the
// non-empty rows) and finds i by binary search along the row.
class CellIndex {
  public:
    void build(const HostMesh &m);
    // cell index of the leaf, or -1 (also for coordinates outside the grid)
    int32_t find(int l, int64_t i, int64_t j, int64_t k) const;

  private:
    const int32_t *ijk_ = nullptr;
    int max_level_ = -1;
    int64_t ext_[LMAX + 1][3] = {};
    bool dense_[LMAX + 1] = {};
    std::vector<int32_t> start_[LMAX + 1];   // row starts (+ the block end)
    std::vector<int64_t> rowkey_[LMAX + 1];  // sparse levels: k ext_j + j of each non-empty row
};

// fn(begin, end) over [0, n) in contiguous chunks on up to 16 host threads
// (the caller runs the first chunk); chunks hold at least min_chunk items.
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t min_chunk = 32768);

void set_error(const std::string &msg);

}  // namespace adg
