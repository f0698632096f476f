/*
 * adg_oracle.c -- plain, slow, FP64 CPU oracle for one ADER-DG time step of the
 * 3-D compressible Euler equations on (adaptive) Cartesian meshes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP path.
 *
 * What it follows (Charrier, Hazelwood, Weinzierl, "Enclave tasking for DG
 * methods on dynamically adaptive meshes", arXiv:1806.07984):
 *   - the conservation law dQ/dt + div F(Q) = 0 with m = 5 Euler variables
 *     (Sec. 2, Eq. 1; source and point terms absent);
 *   - the Lagrange basis on Gauss-Legendre points, same order in time (Sec. 2.1);
 *   - the space-time predictor C_STP, element-local, jump terms dropped, solved
 *     by Picard iterations, partial integration in time injecting Q_h(T)
 *     (Sec. 2.1, Eq. 2 and the STP paragraph; Eq. 3);
 *   - keep only the time-integrated face projections id|dc and the volume
 *     data (Sec. 2.2, text after Eq. 3);
 *   - one Rusanov solve per face over the whole time span (Sec. 2.4, Alg. 1);
 *   - the corrector C_Corr that merges predictor and Riemann results (Eq. 4);
 *   - adaptive meshes: virtual cells filled by interpolation from the coarse
 *     cell (only their face projections are needed), Riemann solves on the
 *     finest resolution, restriction (transpose of the interpolation) into the
 *     parent face (Sec. 2.3, Assumption 1), 3-partitioning.
 * Where the paper leaves a detail open (node family, Picard start and count,
 * CFL formula, what the Riemann solver sees, the weighting of the
 * restriction), this file takes the readings stated next to each function.
 *
 * Style: loops follow the definitions directly; no blocking, no fusion beyond
 * what the definitions state.  OpenMP only distributes independent cells.
 *
 * Layouts (all arrays FP64 unless noted, cells ordered by (level, k, j, i)):
 *   volume node  a = a0 + N*a1 + N*N*a2   (a0 along x fastest)
 *   face node    b = a_t1 + N*a_t2 with (t1 < t2) the two tangential axes
 *   sides        s = 2*d + (0: minus, 1: plus), d = 0,1,2
 *   u, ustar     [5][ncell][N^3]
 *   traces       [6 sides][2: (time-averaged Q, time-averaged normal flux)][5][ncell][N^2]
 *   fside        [6 sides][5][ncell][N^2]  the face flux each cell side sees
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NV 5
#define MAXN 10

/* ------------------------------------------------------------------------- */
/* 1-D basis on [0,1]                                                        */
/* ------------------------------------------------------------------------- */

/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence
 * (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static void legendre_eval(int n, double x, double *P, double *dP)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *P = p1;
    /* (1 - x^2) P_n' = n (P_{n-1} - x P_n) */
    *dP = n * (p0 - x * p1) / (1.0 - x * x);
}

/* Gauss-Legendre nodes (ascending) and weights on [0,1], weights summing to 1.
 * Roots of P_N by Newton's method from the Chebyshev-like initial guess. */
int orc_gauss_legendre(int N, double *xi, double *w)
{
    if (N < 1 || N > MAXN) return 1;
    for (int k = 0; k < N; ++k) {
        double x = cos(M_PI * (k + 0.75) / (N + 0.5));
        double P, dP;
        for (int it = 0; it < 100; ++it) {
            legendre_eval(N, x, &P, &dP);
            double dx = P / dP;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        legendre_eval(N, x, &P, &dP);
        /* x runs from near +1 down to near -1 as k increases */
        xi[k] = 0.5 * (1.0 - x);
        w[k] = 1.0 / ((1.0 - x * x) * dP * dP); /* = (2/((1-x^2)P'^2)) / 2 */
    }
    return 0;
}

/* Lagrange basis polynomial phi_e on the nodes xi, evaluated at x. */
static double lagrange(int N, const double *xi, int e, double x)
{
    double v = 1.0;
    for (int m = 0; m < N; ++m)
        if (m != e) v *= (x - xi[m]) / (xi[e] - xi[m]);
    return v;
}

/* Derivative of phi_e at x (product rule written out). */
static double lagrange_deriv(int N, const double *xi, int e, double x)
{
    double s = 0.0;
    for (int k = 0; k < N; ++k) {
        if (k == e) continue;
        double t = 1.0 / (xi[e] - xi[k]);
        for (int m = 0; m < N; ++m)
            if (m != e && m != k) t *= (x - xi[m]) / (xi[e] - xi[m]);
        s += t;
    }
    return s;
}

/* Inverse of an n x n matrix by Gauss-Jordan elimination with partial
 * pivoting.  Returns nonzero if singular. */
static int invert(int n, const double *A, double *Ainv)
{
    double M[MAXN][2 * MAXN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            M[i][j] = A[i * n + j];
            M[i][n + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (fabs(M[i][c]) > fabs(M[piv][c])) piv = i;
        if (M[piv][c] == 0.0) return 1;
        if (piv != c)
            for (int j = 0; j < 2 * n; ++j) {
                double t = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = t;
            }
        double d = M[c][c];
        for (int j = 0; j < 2 * n; ++j) M[c][j] /= d;
        for (int i = 0; i < n; ++i) {
            if (i == c) continue;
            double f = M[i][c];
            for (int j = 0; j < 2 * n; ++j) M[i][j] -= f * M[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = M[i][n + j];
    return 0;
}

/* The 1-D operators of one order (N = p+1 nodes):
 *   D[a][e]   = phi_e'(xi_a)                     derivative at the nodes
 *   L[e], R[e]= phi_e(0), phi_e(1)               extrapolation to the faces
 *   K1[k][l]  = phi_k(1) phi_l(1) - int phi_k' phi_l
 *             = R_k R_l - w_l D[l][k]            time operator after partial
 *               integration in time with Q_h(T) injected at tau = 0
 *   Kinv      = K1^{-1}
 *   Kw[a][e]  = int phi_a' phi_e = w_e D[e][a]   weak stiffness (exact by GL)
 */
int orc_basis(int N, double *xi, double *w, double *D, double *L, double *R,
              double *Kinv, double *Kw)
{
    if (orc_gauss_legendre(N, xi, w)) return 1;
    for (int a = 0; a < N; ++a)
        for (int e = 0; e < N; ++e) D[a * N + e] = lagrange_deriv(N, xi, e, xi[a]);
    for (int e = 0; e < N; ++e) {
        L[e] = lagrange(N, xi, e, 0.0);
        R[e] = lagrange(N, xi, e, 1.0);
    }
    double K1[MAXN * MAXN];
    for (int k = 0; k < N; ++k)
        for (int l = 0; l < N; ++l) K1[k * N + l] = R[k] * R[l] - w[l] * D[l * N + k];
    if (invert(N, K1, Kinv)) return 2;
    for (int a = 0; a < N; ++a)
        for (int e = 0; e < N; ++e) Kw[a * N + e] = w[e] * D[e * N + a];
    return 0;
}

/* Inter-grid transfer along one axis for a child interval s of a parent
 * interval split into r equal parts (r = 3^dl with 3-partitioning):
 *   P[k][e] = phi_e((s + xi_k)/r)      interpolation coarse -> child nodes
 *   Rm[k][e] = (1/r)(w_e/w_k) phi_k((s + xi_e)/r)
 * Rm is the transpose of P taken in the quadrature-weighted inner product
 * (Rm = r^{-1} W^{-1} P^T W), which makes the restriction conservative and
 * sum_s Rm^(s) P^(s) = I. */
int orc_transfer(int N, int r, int s, double *P, double *Rm)
{
    double xi[MAXN], w[MAXN];
    if (orc_gauss_legendre(N, xi, w)) return 1;
    if (r < 1 || s < 0 || s >= r) return 2;
    for (int k = 0; k < N; ++k)
        for (int e = 0; e < N; ++e) {
            P[k * N + e] = lagrange(N, xi, e, (s + xi[k]) / r);
            Rm[k * N + e] = (w[e] / w[k]) * lagrange(N, xi, k, (s + xi[e]) / r) / r;
        }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Euler equations                                                           */
/* ------------------------------------------------------------------------- */

static double pressure(double g, const double q[NV])
{
    return (g - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

/* Flux along axis d: (m_d, m_d m/rho + p e_d, m_d (E + p)/rho). */
static void euler_flux(double g, const double q[NV], int d, double f[NV])
{
    double p = pressure(g, q);
    double vd = q[1 + d] / q[0];
    f[0] = q[1 + d];
    f[1] = vd * q[1];
    f[2] = vd * q[2];
    f[3] = vd * q[3];
    f[1 + d] += p;
    f[4] = vd * (q[4] + p);
}

/* Largest characteristic speed along d: |u_d| + c, c = sqrt(gamma p / rho). */
static double euler_speed(double g, const double q[NV], int d)
{
    double p = pressure(g, q);
    return fabs(q[1 + d] / q[0]) + sqrt(g * p / q[0]);
}

static int unphysical(double g, const double q[NV])
{
    for (int v = 0; v < NV; ++v)
        if (!isfinite(q[v])) return 1;
    if (!(q[0] > 0.0)) return 1;
    if (!(pressure(g, q) > 0.0)) return 1;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Mesh: conformal base grid, recursive 3x3x3 refinement (Assumption 1)      */
/* ------------------------------------------------------------------------- */

enum { SIDE_CONFORMING = 0, SIDE_FINE = 1, SIDE_COARSE = 2 };

typedef struct {
    int N;
    int n[3];
    double lo[3], hi[3];
    int max_level;
    long nc;
    int *lev;     /* [nc] */
    int *ijk;     /* [3*nc] integer cell coordinates at the cell's level */
    /* per cell side (6 per cell):
     *   kind[6*c+s]  SIDE_CONFORMING: same-level neighbour nbr
     *                SIDE_FINE: neighbour nbr is coarser (hanging face, this
     *                           cell is the fine side)
     *                SIDE_COARSE: the region beyond is refined further   */
    int *kind;
    long *nbr;
} orc_mesh;

static long ipow3(int e)
{
    long r = 1;
    while (e-- > 0) r *= 3;
    return r;
}

/* lexicographic key compare: (level, k, j, i) */
static int key_cmp(int la, const int *a, int lb, const int *b)
{
    if (la != lb) return la < lb ? -1 : 1;
    for (int d = 2; d >= 0; --d)
        if (a[d] != b[d]) return a[d] < b[d] ? -1 : 1;
    return 0;
}

static long find_cell(const orc_mesh *m, int l, const int *c)
{
    long lo = 0, hi = m->nc - 1;
    while (lo <= hi) {
        long mid = (lo + hi) / 2;
        int r = key_cmp(m->lev[mid], &m->ijk[3 * mid], l, c);
        if (r == 0) return mid;
        if (r < 0) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

typedef struct { int l, i[3]; } cellkey;

static int cellkey_cmp(const void *pa, const void *pb)
{
    const cellkey *a = (const cellkey *)pa, *b = (const cellkey *)pb;
    return key_cmp(a->l, a->i, b->l, b->i);
}

void orc_mesh_free(orc_mesh *m)
{
    if (!m) return;
    free(m->lev); free(m->ijk); free(m->kind); free(m->nbr);
    free(m);
}

/* Build the leaf mesh.  refine holds n_refine entries (level, i, j, k); each
 * names a leaf that is split into 27 children.  Entries of level l must refer
 * to leaves that exist once all entries of levels < l are applied.  Only fully
 * periodic domains are represented.  Returns NULL on invalid input. */
orc_mesh *orc_mesh_build(int N, const int *n, const double *lo, const double *hi,
                         int max_level, long n_refine, const int *refine)
{
    if (N < 1 || N > MAXN || max_level < 0 || max_level > 4) return NULL;
    for (int d = 0; d < 3; ++d)
        if (n[d] < 1 || !(hi[d] > lo[d])) return NULL;
    /* current leaves, as keys */
    long cap = (long)n[0] * n[1] * n[2];
    cellkey *leaves = (cellkey *)malloc(sizeof(cellkey) * cap);
    long nl = 0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                leaves[nl].l = 0;
                leaves[nl].i[0] = i; leaves[nl].i[1] = j; leaves[nl].i[2] = k;
                ++nl;
            }
    /* sorted refine list */
    cellkey *ref = (cellkey *)malloc(sizeof(cellkey) * (n_refine > 0 ? n_refine : 1));
    for (long r = 0; r < n_refine; ++r) {
        ref[r].l = refine[4 * r];
        for (int d = 0; d < 3; ++d) ref[r].i[d] = refine[4 * r + 1 + d];
        if (ref[r].l < 0 || ref[r].l >= max_level) { free(leaves); free(ref); return NULL; }
    }
    qsort(ref, n_refine, sizeof(cellkey), cellkey_cmp);
    for (long r = 1; r < n_refine; ++r)
        if (cellkey_cmp(&ref[r - 1], &ref[r]) == 0) { free(leaves); free(ref); return NULL; }
    /* apply level by level; leaves stay sorted because children are appended
     * at a strictly greater level and re-sorted */
    long used = 0;
    for (int l = 0; l < max_level; ++l) {
        long first = used;
        while (used < n_refine && ref[used].l == l) ++used;
        long nr = used - first;
        if (nr == 0) continue;
        cellkey *next = (cellkey *)malloc(sizeof(cellkey) * (nl - nr + 27 * nr));
        long nn = 0, found = 0;
        for (long q = 0; q < nl; ++q) {
            cellkey *c = &leaves[q];
            int is_ref = 0;
            if (c->l == l) {
                cellkey *hit = (cellkey *)bsearch(c, ref + first, nr, sizeof(cellkey), cellkey_cmp);
                is_ref = hit != NULL;
            }
            if (!is_ref) { next[nn++] = *c; continue; }
            ++found;
            for (int dz = 0; dz < 3; ++dz)
                for (int dy = 0; dy < 3; ++dy)
                    for (int dx = 0; dx < 3; ++dx) {
                        next[nn].l = l + 1;
                        next[nn].i[0] = 3 * c->i[0] + dx;
                        next[nn].i[1] = 3 * c->i[1] + dy;
                        next[nn].i[2] = 3 * c->i[2] + dz;
                        ++nn;
                    }
        }
        free(leaves);
        leaves = next;
        nl = nn;
        if (found != nr) { free(leaves); free(ref); return NULL; }
        qsort(leaves, nl, sizeof(cellkey), cellkey_cmp);
    }
    free(ref);

    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    m->N = N;
    for (int d = 0; d < 3; ++d) { m->n[d] = n[d]; m->lo[d] = lo[d]; m->hi[d] = hi[d]; }
    m->max_level = max_level;
    m->nc = nl;
    m->lev = (int *)malloc(sizeof(int) * nl);
    m->ijk = (int *)malloc(sizeof(int) * 3 * nl);
    m->kind = (int *)malloc(sizeof(int) * 6 * nl);
    m->nbr = (long *)malloc(sizeof(long) * 6 * nl);
    for (long c = 0; c < nl; ++c) {
        m->lev[c] = leaves[c].l;
        for (int d = 0; d < 3; ++d) m->ijk[3 * c + d] = leaves[c].i[d];
    }
    free(leaves);

    /* neighbour search: same level first, then coarser levels; otherwise the
     * region beyond the face is refined further */
    for (long c = 0; c < nl; ++c) {
        int l = m->lev[c];
        for (int s = 0; s < 6; ++s) {
            int d = s / 2, dir = (s % 2) ? 1 : -1;
            int q[3] = { m->ijk[3 * c], m->ijk[3 * c + 1], m->ijk[3 * c + 2] };
            long extent = n[d] * ipow3(l);
            q[d] = (int)(((long)q[d] + dir + extent) % extent);
            long hit = find_cell(m, l, q);
            if (hit >= 0) { m->kind[6 * c + s] = SIDE_CONFORMING; m->nbr[6 * c + s] = hit; continue; }
            m->kind[6 * c + s] = SIDE_COARSE;
            m->nbr[6 * c + s] = -1;
            for (int lc = l - 1; lc >= 0; --lc) {
                long f = ipow3(l - lc);
                int qc[3] = { (int)(q[0] / f), (int)(q[1] / f), (int)(q[2] / f) };
                hit = find_cell(m, lc, qc);
                if (hit >= 0) { m->kind[6 * c + s] = SIDE_FINE; m->nbr[6 * c + s] = hit; break; }
            }
        }
    }
    return m;
}

long orc_mesh_ncells(const orc_mesh *m) { return m->nc; }

/* level, i, j, k of every cell */
void orc_mesh_cells(const orc_mesh *m, int *out)
{
    for (long c = 0; c < m->nc; ++c) {
        out[4 * c] = m->lev[c];
        for (int d = 0; d < 3; ++d) out[4 * c + 1 + d] = m->ijk[3 * c + d];
    }
}

/* kind and neighbour of every cell side: kind[6*nc], nbr[6*nc] */
void orc_mesh_sides(const orc_mesh *m, int *kind, long *nbr)
{
    memcpy(kind, m->kind, sizeof(int) * 6 * m->nc);
    memcpy(nbr, m->nbr, sizeof(long) * 6 * m->nc);
}

static void cell_dx(const orc_mesh *m, long c, double dx[3])
{
    double f = (double)ipow3(m->lev[c]);
    for (int d = 0; d < 3; ++d) dx[d] = (m->hi[d] - m->lo[d]) / (m->n[d] * f);
}

/* Physical coordinates of every node: xyz[3][nc][N^3]. */
void orc_node_coords(const orc_mesh *m, double *xyz)
{
    int N = m->N, N3 = N * N * N;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    for (long c = 0; c < m->nc; ++c) {
        double dx[3];
        cell_dx(m, c, dx);
        for (int a2 = 0; a2 < N; ++a2)
            for (int a1 = 0; a1 < N; ++a1)
                for (int a0 = 0; a0 < N; ++a0) {
                    int a = a0 + N * a1 + N * N * a2;
                    int aa[3] = { a0, a1, a2 };
                    for (int d = 0; d < 3; ++d)
                        xyz[((long)d * m->nc + c) * N3 + a] =
                            m->lo[d] + (m->ijk[3 * c + d] + xi[aa[d]]) * dx[d];
                }
    }
}

/* ------------------------------------------------------------------------- */
/* Index helpers                                                             */
/* ------------------------------------------------------------------------- */

/* volume node index with the index along axis d replaced by e */
static int node_with(int N, int a, int d, int e)
{
    int aa[3] = { a % N, (a / N) % N, a / (N * N) };
    aa[d] = e;
    return aa[0] + N * aa[1] + N * N * aa[2];
}

/* face node index b of volume node a for a face normal to d */
static int face_index(int N, int a, int d)
{
    int aa[3] = { a % N, (a / N) % N, a / (N * N) };
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    return aa[t1] + N * aa[t2];
}

/* volume node with index e along d and face index b on the tangential axes */
static int node_from_face(int N, int d, int e, int b)
{
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    int aa[3];
    aa[d] = e;
    aa[t1] = b % N;
    aa[t2] = b / N;
    return aa[0] + N * aa[1] + N * N * aa[2];
}

/* ------------------------------------------------------------------------- */
/* Time step size (global time stepping, one dt for all cells)               */
/* ------------------------------------------------------------------------- */

/* dt = cfl / ((2p+1) * max_{cells,nodes} sum_d lambda_d(u)/dx_d), lambda_d =
 * |u_d| + c.  Sets *status = 1 if any node is unphysical (rho <= 0, p <= 0 or
 * a non-finite value). */
double orc_cfl(const orc_mesh *m, double g, double cfl, const double *u, int *status)
{
    int N = m->N, N3 = N * N * N;
    long nc = m->nc;
    double lam = 0.0;
    int bad = 0;
#pragma omp parallel for reduction(max : lam) reduction(| : bad) schedule(static)
    for (long c = 0; c < nc; ++c) {
        double dx[3];
        cell_dx(m, c, dx);
        for (int a = 0; a < N3; ++a) {
            double q[NV];
            for (int v = 0; v < NV; ++v) q[v] = u[((long)v * nc + c) * N3 + a];
            if (unphysical(g, q)) { bad = 1; continue; }
            double s = 0.0;
            for (int d = 0; d < 3; ++d) s += euler_speed(g, q, d) / dx[d];
            if (s > lam) lam = s;
        }
    }
    *status = bad;
    if (bad || !(lam > 0.0)) return 0.0;
    return cfl / ((2.0 * (N - 1) + 1.0) * lam);
}

/* ------------------------------------------------------------------------- */
/* Space-time predictor + volume term + face projections                     */
/* ------------------------------------------------------------------------- */

/* Per cell, with tau in [0,1] mapped to (T, T+dt) and reference coordinates:
 *   q_l  (l = time node) starts as u at every time node,
 *   repeat npic times:
 *     G_j   = sum_d (dt/dx_d) (D along axis d) f_d(q_j)
 *     q_l  <- u - sum_j Kinv[l][j] w_j G_j
 *   qbar  = sum_j w_j q_j,  Fbar_d = sum_j w_j f_d(q_j)   (final iterate)
 *   ustar = u + sum_d (dt/dx_d) (1/w_{a_d}) sum_e Kw[a_d][e] Fbar_d(..e..)
 *   traces: qbar and Fbar_d extrapolated with L (minus side) or R (plus side)
 *   along d; only the normal flux component d is kept. */
void orc_predictor(const orc_mesh *m, double g, int npic, double dt,
                   const double *u, double *ustar, double *traces)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    double xi[MAXN], w[MAXN], D[MAXN * MAXN], L[MAXN], R[MAXN], Kinv[MAXN * MAXN], Kw[MAXN * MAXN];
    orc_basis(N, xi, w, D, L, R, Kinv, Kw);

#pragma omp parallel
    {
        double *q = (double *)malloc(sizeof(double) * N * NV * N3);      /* [l][v][a] */
        double *qn = (double *)malloc(sizeof(double) * N * NV * N3);
        double *F = (double *)malloc(sizeof(double) * N * 3 * NV * N3);  /* [j][d][v][a] */
        double *G = (double *)malloc(sizeof(double) * N * NV * N3);      /* [j][v][a] */
        double *qbar = (double *)malloc(sizeof(double) * NV * N3);
        double *Fbar = (double *)malloc(sizeof(double) * 3 * NV * N3);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            double dx[3];
            cell_dx(m, c, dx);
            double uc[NV][MAXN * MAXN * MAXN];
            for (int v = 0; v < NV; ++v)
                for (int a = 0; a < N3; ++a) uc[v][a] = u[((long)v * nc + c) * N3 + a];

            for (int l = 0; l < N; ++l)
                for (int v = 0; v < NV; ++v)
                    for (int a = 0; a < N3; ++a) q[(l * NV + v) * N3 + a] = uc[v][a];

            for (int it = 0; it <= npic; ++it) {
                /* fluxes of the current iterate */
                for (int j = 0; j < N; ++j)
                    for (int a = 0; a < N3; ++a) {
                        double qq[NV], f[NV];
                        for (int v = 0; v < NV; ++v) qq[v] = q[(j * NV + v) * N3 + a];
                        for (int d = 0; d < 3; ++d) {
                            euler_flux(g, qq, d, f);
                            for (int v = 0; v < NV; ++v) F[((j * 3 + d) * NV + v) * N3 + a] = f[v];
                        }
                    }
                if (it == npic) break; /* the final fluxes feed the time averages */
                /* G_j = sum_d (dt/dx_d) D_d f_d(q_j) */
                for (int j = 0; j < N; ++j)
                    for (int v = 0; v < NV; ++v)
                        for (int a = 0; a < N3; ++a) {
                            int aa[3] = { a % N, (a / N) % N, a / N2 };
                            double s = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                double sd = 0.0;
                                for (int e = 0; e < N; ++e)
                                    sd += D[aa[d] * N + e] * F[((j * 3 + d) * NV + v) * N3 + node_with(N, a, d, e)];
                                s += (dt / dx[d]) * sd;
                            }
                            G[(j * NV + v) * N3 + a] = s;
                        }
                /* q_l = u - sum_j Kinv[l][j] w_j G_j */
                for (int l = 0; l < N; ++l)
                    for (int v = 0; v < NV; ++v)
                        for (int a = 0; a < N3; ++a) {
                            double s = 0.0;
                            for (int j = 0; j < N; ++j) s += Kinv[l * N + j] * w[j] * G[(j * NV + v) * N3 + a];
                            qn[(l * NV + v) * N3 + a] = uc[v][a] - s;
                        }
                double *t = q; q = qn; qn = t;
            }
            /* time averages of the final iterate */
            for (int v = 0; v < NV; ++v)
                for (int a = 0; a < N3; ++a) {
                    double s = 0.0;
                    for (int j = 0; j < N; ++j) s += w[j] * q[(j * NV + v) * N3 + a];
                    qbar[v * N3 + a] = s;
                    for (int d = 0; d < 3; ++d) {
                        double sf = 0.0;
                        for (int j = 0; j < N; ++j) sf += w[j] * F[((j * 3 + d) * NV + v) * N3 + a];
                        Fbar[(d * NV + v) * N3 + a] = sf;
                    }
                }
            /* volume term */
            for (int v = 0; v < NV; ++v)
                for (int a = 0; a < N3; ++a) {
                    int aa[3] = { a % N, (a / N) % N, a / N2 };
                    double s = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        double sd = 0.0;
                        for (int e = 0; e < N; ++e)
                            sd += Kw[aa[d] * N + e] * Fbar[(d * NV + v) * N3 + node_with(N, a, d, e)];
                        s += (dt / dx[d]) * sd / w[aa[d]];
                    }
                    ustar[((long)v * nc + c) * N3 + a] = uc[v][a] + s;
                }
            /* face projections of the time-averaged data */
            for (int s = 0; s < 6; ++s) {
                int d = s / 2;
                const double *E = (s % 2) ? R : L;
                for (int v = 0; v < NV; ++v)
                    for (int b = 0; b < N2; ++b) {
                        double sq = 0.0, sf = 0.0;
                        for (int e = 0; e < N; ++e) {
                            int a = node_from_face(N, d, e, b);
                            sq += E[e] * qbar[v * N3 + a];
                            sf += E[e] * Fbar[(d * NV + v) * N3 + a];
                        }
                        traces[(((long)(s * 2 + 0) * NV + v) * nc + c) * N2 + b] = sq;
                        traces[(((long)(s * 2 + 1) * NV + v) * nc + c) * N2 + b] = sf;
                    }
            }
        }
        free(q); free(qn); free(F); free(G); free(qbar); free(Fbar);
    }
}

/* ------------------------------------------------------------------------- */
/* Riemann solves (Rusanov), with virtual cells and restriction on AMR       */
/* ------------------------------------------------------------------------- */

/* Rusanov flux on one face with N2 nodes, normal axis d, left state (QL, FL)
 * on the minus side and right state (QR, FR) on the plus side; one wave
 * speed s per face, the largest |u_d| + c over the face nodes of both sides.
 * Arrays are [5][N2]. Returns 1 if a node is unphysical. */
static int rusanov(double g, int d, int N2, const double *QL, const double *FL,
                   const double *QR, const double *FR, double *Fs)
{
    double smax = 0.0;
    int bad = 0;
    for (int b = 0; b < N2; ++b) {
        double ql[NV], qr[NV];
        for (int v = 0; v < NV; ++v) { ql[v] = QL[v * N2 + b]; qr[v] = QR[v * N2 + b]; }
        if (unphysical(g, ql) || unphysical(g, qr)) bad = 1;
        double sl = euler_speed(g, ql, d), sr = euler_speed(g, qr, d);
        if (sl > smax) smax = sl;
        if (sr > smax) smax = sr;
    }
    for (int v = 0; v < NV; ++v)
        for (int b = 0; b < N2; ++b)
            Fs[v * N2 + b] = 0.5 * (FL[v * N2 + b] + FR[v * N2 + b])
                             - 0.5 * smax * (QR[v * N2 + b] - QL[v * N2 + b]);
    return bad;
}

static void get_trace(const orc_mesh *m, const double *traces, long c, int s, int arr, double *out)
{
    int N2 = m->N * m->N;
    for (int v = 0; v < NV; ++v)
        for (int b = 0; b < N2; ++b)
            out[v * N2 + b] = traces[(((long)(s * 2 + arr) * NV + v) * m->nc + c) * N2 + b];
}

static void put_side(const orc_mesh *m, double *fside, long c, int s, const double *F)
{
    int N2 = m->N * m->N;
    for (int v = 0; v < NV; ++v)
        for (int b = 0; b < N2; ++b)
            fside[((long)(s * NV + v) * m->nc + c) * N2 + b] = F[v * N2 + b];
}

/* tangential axes of a face normal to d, increasing */
static void tangential(int d, int *t1, int *t2)
{
    *t1 = (d == 0) ? 1 : 0;
    *t2 = (d == 2) ? 1 : 2;
}

/* Virtual-cell face data: the coarse cell's face projection interpolated to
 * the child face (s1, s2) with 1-D interpolation P along each tangential
 * axis (the exact restriction of the coarse polynomial to the child face). */
static void prolong_face(int N, int r, int s1, int s2, const double *coarse, double *fine)
{
    int N2 = N * N;
    double P1[MAXN * MAXN], P2[MAXN * MAXN], Rm[MAXN * MAXN];
    orc_transfer(N, r, s1, P1, Rm);
    orc_transfer(N, r, s2, P2, Rm);
    for (int v = 0; v < NV; ++v)
        for (int k2 = 0; k2 < N; ++k2)
            for (int k1 = 0; k1 < N; ++k1) {
                double s = 0.0;
                for (int e2 = 0; e2 < N; ++e2)
                    for (int e1 = 0; e1 < N; ++e1)
                        s += P1[k1 * N + e1] * P2[k2 * N + e2] * coarse[v * N2 + e1 + N * e2];
                fine[v * N2 + k1 + N * k2] = s;
            }
}

/* child sub-position of fine cell f inside the coarse cell, along axis t */
static int sub_position(const orc_mesh *m, long f, long cc, int t)
{
    long r = ipow3(m->lev[f] - m->lev[cc]);
    return (int)(m->ijk[3 * f + t] - r * m->ijk[3 * cc + t]);
}

/* Fills fside for every cell side.  Conforming faces: one Rusanov solve,
 * written to both sides.  Hanging faces: the Rusanov solve runs on the child
 * face between the fine cell and the virtual cell; the fine cell sees the
 * result; the coarse side receives the sum over its child faces of the
 * restricted results (accumulated in increasing fine-cell order).
 * Returns 1 if an unphysical state was met. */
int orc_riemann(const orc_mesh *m, double g, const double *traces, double *fside)
{
    int N = m->N, N2 = N * N;
    long nc = m->nc;
    int bad = 0;
#pragma omp parallel reduction(| : bad)
    {
        double *QL = (double *)malloc(sizeof(double) * NV * N2 * 6);
        double *FL = QL + NV * N2, *QR = FL + NV * N2, *FR = QR + NV * N2;
        double *Fs = FR + NV * N2, *tmp = Fs + NV * N2;
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            for (int s = 0; s < 6; ++s) {
                int d = s / 2, plus = s % 2;
                int kind = m->kind[6 * c + s];
                long o = m->nbr[6 * c + s];
                if (kind == SIDE_COARSE) continue;
                int so = 2 * d + (1 - plus); /* the neighbour's side facing c */
                double *Qc = plus ? QL : QR, *Fc = plus ? FL : FR;
                double *Qo = plus ? QR : QL, *Fo = plus ? FR : FL;
                get_trace(m, traces, c, s, 0, Qc);
                get_trace(m, traces, c, s, 1, Fc);
                if (kind == SIDE_CONFORMING) {
                    get_trace(m, traces, o, so, 0, Qo);
                    get_trace(m, traces, o, so, 1, Fo);
                } else {
                    int t1, t2;
                    tangential(d, &t1, &t2);
                    int r = (int)ipow3(m->lev[c] - m->lev[o]);
                    int s1 = sub_position(m, c, o, t1), s2 = sub_position(m, c, o, t2);
                    get_trace(m, traces, o, so, 0, tmp);
                    prolong_face(N, r, s1, s2, tmp, Qo);
                    get_trace(m, traces, o, so, 1, tmp);
                    prolong_face(N, r, s1, s2, tmp, Fo);
                }
                bad |= rusanov(g, d, N2, QL, FL, QR, FR, Fs);
                put_side(m, fside, c, s, Fs);
            }
        }
        free(QL);
    }
    /* restriction into coarse sides: zero, then accumulate child results */
    for (long c = 0; c < nc; ++c)
        for (int s = 0; s < 6; ++s)
            if (m->kind[6 * c + s] == SIDE_COARSE)
                for (int v = 0; v < NV; ++v)
                    for (int b = 0; b < N2; ++b) fside[((long)(s * NV + v) * nc + c) * N2 + b] = 0.0;
    for (long f = 0; f < nc; ++f) {
        for (int s = 0; s < 6; ++s) {
            if (m->kind[6 * f + s] != SIDE_FINE) continue;
            int d = s / 2, plus = s % 2;
            long cc = m->nbr[6 * f + s];
            int sc = 2 * d + (1 - plus);
            int t1, t2;
            tangential(d, &t1, &t2);
            int r = (int)ipow3(m->lev[f] - m->lev[cc]);
            int s1 = sub_position(m, f, cc, t1), s2 = sub_position(m, f, cc, t2);
            double P[MAXN * MAXN], R1[MAXN * MAXN], R2[MAXN * MAXN];
            orc_transfer(N, r, s1, P, R1);
            orc_transfer(N, r, s2, P, R2);
            for (int v = 0; v < NV; ++v)
                for (int k2 = 0; k2 < N; ++k2)
                    for (int k1 = 0; k1 < N; ++k1) {
                        double acc = 0.0;
                        for (int e2 = 0; e2 < N; ++e2)
                            for (int e1 = 0; e1 < N; ++e1)
                                acc += R1[k1 * N + e1] * R2[k2 * N + e2] *
                                       fside[((long)(s * NV + v) * nc + f) * N2 + e1 + N * e2];
                        fside[((long)(sc * NV + v) * nc + cc) * N2 + k1 + N * k2] += acc;
                    }
        }
    }
    return bad;
}

/* ------------------------------------------------------------------------- */
/* Corrector                                                                 */
/* ------------------------------------------------------------------------- */

/* u_new = ustar - sum_d (dt/dx_d)(1/w_{a_d}) [R_{a_d} F*_{d+} - L_{a_d} F*_{d-}]
 * with F*_{d+-} the face flux of the cell side at the node's face index. */
void orc_corrector(const orc_mesh *m, double dt, const double *ustar, const double *fside, double *unew)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    double xi[MAXN], w[MAXN], D[MAXN * MAXN], L[MAXN], R[MAXN], Kinv[MAXN * MAXN], Kw[MAXN * MAXN];
    orc_basis(N, xi, w, D, L, R, Kinv, Kw);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double dx[3];
        cell_dx(m, c, dx);
        for (int v = 0; v < NV; ++v)
            for (int a = 0; a < N3; ++a) {
                int aa[3] = { a % N, (a / N) % N, a / N2 };
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int b = face_index(N, a, d);
                    double fm = fside[((long)((2 * d) * NV + v) * nc + c) * N2 + b];
                    double fp = fside[((long)((2 * d + 1) * NV + v) * nc + c) * N2 + b];
                    s += (dt / dx[d]) * (R[aa[d]] * fp - L[aa[d]] * fm) / w[aa[d]];
                }
                unew[((long)v * nc + c) * N3 + a] = ustar[((long)v * nc + c) * N3 + a] - s;
            }
    }
}

/* ------------------------------------------------------------------------- */
/* Whole steps                                                               */
/* ------------------------------------------------------------------------- */

/* Runs nsteps ADER-DG steps in place on u.  dt per step from orc_cfl, or the
 * fixed value dt_fixed when dt_fixed > 0; t_end > 0 clamps the last step and
 * ends the run once t_end is reached (later dt_hist entries stay untouched).
 * Writes the dt of every step to dt_hist (may be NULL).  Returns 0 on success,
 * 1 if an unphysical state was met (u then holds the last valid state),
 * 2 on allocation failure. */
int orc_run(const orc_mesh *m, double g, double cfl, int npic, double dt_fixed, double t_end,
            double *u, int nsteps, double *dt_hist)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    double *us = (double *)malloc(sizeof(double) * NV * nc * N3);
    double *tr = (double *)malloc(sizeof(double) * 6 * 2 * NV * nc * N2);
    double *fs = (double *)malloc(sizeof(double) * 6 * NV * nc * N2);
    if (!us || !tr || !fs) { free(us); free(tr); free(fs); return 2; }
    double t = 0.0;
    int rc = 0;
    for (int n = 0; n < nsteps; ++n) {
        if (t_end > 0.0 && t >= t_end) break; /* final time reached */
        int st = 0;
        double dt = dt_fixed > 0.0 ? dt_fixed : orc_cfl(m, g, cfl, u, &st);
        if (st) { rc = 1; break; }
        if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
        if (dt_hist) dt_hist[n] = dt;
        orc_predictor(m, g, npic, dt, u, us, tr);
        if (orc_riemann(m, g, tr, fs)) { rc = 1; break; }
        orc_corrector(m, dt, us, fs, u);
        t += dt;
    }
    free(us); free(tr); free(fs);
    return rc;
}

/* Runs nsteps steps with a prescribed dt per step (dt_sched[n]); the CFL
 * reduction is skipped.  Returns 0, or 1 if an unphysical state was met. */
int orc_run_sched(const orc_mesh *m, double g, int npic, const double *dt_sched, double *u, int nsteps)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    double *us = (double *)malloc(sizeof(double) * NV * nc * N3);
    double *tr = (double *)malloc(sizeof(double) * 6 * 2 * NV * nc * N2);
    double *fs = (double *)malloc(sizeof(double) * 6 * NV * nc * N2);
    if (!us || !tr || !fs) { free(us); free(tr); free(fs); return 2; }
    int rc = 0;
    for (int n = 0; n < nsteps; ++n) {
        orc_predictor(m, g, npic, dt_sched[n], u, us, tr);
        if (orc_riemann(m, g, tr, fs)) { rc = 1; break; }
        orc_corrector(m, dt_sched[n], us, fs, u);
    }
    free(us); free(tr); free(fs);
    return rc;
}

/* Density of the discrete solution at points (base-level meshes only):
 * rho_h(x) = sum_a rho_{c,a} phi_a0(xi0) phi_a1(xi1) phi_a2(xi2) with c the
 * cell containing x (floor of the cell coordinate, clamped into the grid). */
int orc_sample(const orc_mesh *m, const double *u, const double *pts, long n, double *out)
{
    if (m->max_level != 0) return 1;
    int N = m->N, N3 = N * N * N;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    for (long s = 0; s < n; ++s) {
        int ijk[3];
        double phi[3][MAXN];
        for (int d = 0; d < 3; ++d) {
            double y = (pts[3 * s + d] - m->lo[d]) / (m->hi[d] - m->lo[d]) * m->n[d];
            int i = (int)floor(y);
            if (i < 0) i = 0;
            if (i >= m->n[d]) i = m->n[d] - 1;
            ijk[d] = i;
            for (int e = 0; e < N; ++e) phi[d][e] = lagrange(N, xi, e, y - i);
        }
        long c = ijk[0] + (long)m->n[0] * (ijk[1] + (long)m->n[1] * ijk[2]);
        double acc = 0.0;
        for (int a2 = 0; a2 < N; ++a2)
            for (int a1 = 0; a1 < N; ++a1)
                for (int a0 = 0; a0 < N; ++a0)
                    acc += u[c * N3 + a0 + N * a1 + N * N * a2] * phi[0][a0] * phi[1][a1] * phi[2][a2];
        out[s] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Dynamic adaptivity: refinement indicator and volumetric transfer          */
/* ------------------------------------------------------------------------- */

/* Feature-based criterion read in the corrector's epilogue (Sec. 2.3,
 * dynamic-adaptivity paragraph; Sec. 2.4: criteria study first or second
 * derivatives of the solution, cell by cell).  Reading: the indicator of a
 * cell is the largest change of the density across the cell along any axis,
 *   eta_c = max_{nodes a, axes d} | d rho_h / d xi_d (x_a) |,
 * the derivative in the cell's reference coordinate xi_d in [0,1] (so
 * eta_c = dx_d * |d rho / dx_d| for a linear density). */
void orc_indicator(const orc_mesh *m, const double *u, double *eta)
{
    int N = m->N, N3 = N * N * N;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    for (long c = 0; c < m->nc; ++c) {
        double best = 0.0;
        for (int a = 0; a < N3; ++a) {
            int aa[3] = { a % N, (a / N) % N, a / (N * N) };
            for (int d = 0; d < 3; ++d) {
                double g = 0.0;
                for (int e = 0; e < N; ++e)
                    g += lagrange_deriv(N, xi, e, xi[aa[d]]) * u[c * N3 + node_with(N, a, d, e)];
                if (fabs(g) > best) best = fabs(g);
            }
        }
        eta[c] = best;
    }
}

/* Value of cell c's polynomial (all 5 variables) at reference point y. */
static void eval_cell(const orc_mesh *m, const double *u, long c, const double *xi, const double y[3],
                      double out[NV])
{
    int N = m->N, N3 = N * N * N;
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    for (int b = 0; b < N3; ++b) {
        double phi = lagrange(N, xi, b % N, y[0]) * lagrange(N, xi, (b / N) % N, y[1]) *
                     lagrange(N, xi, b / (N * N), y[2]);
        for (int v = 0; v < NV; ++v) out[v] += phi * u[((long)v * m->nc + c) * N3 + b];
    }
}

/* Accumulate into acc[v][a] the integral over the part of cell C (level lc,
 * coordinates kc) covered by the leaves of `from` inside region (l, q) of
 * the u_from polynomials times phi_a of C, in units of C's volume; the
 * covered volume fraction goes to *vol.  Each leaf is integrated with its own
 * Gauss rule, exact for the degree-2p integrands. */
static void project_region(const orc_mesh *from, const double *u, int lc, const int *kc, int l, const int *q,
                           const double *xi, const double *w, double *acc, double *vol)
{
    int N = from->N, N3 = N * N * N;
    long f = find_cell(from, l, q);
    if (f >= 0) {
        double r = (double)ipow3(l - lc);
        for (int b = 0; b < N3; ++b) {
            int bb[3] = { b % N, (b / N) % N, b / (N * N) };
            double wt = w[bb[0]] * w[bb[1]] * w[bb[2]] / (r * r * r);
            double y[3];
            for (int d = 0; d < 3; ++d) y[d] = (q[d] + xi[bb[d]]) / r - kc[d];
            *vol += wt;
            for (int a = 0; a < N3; ++a) {
                double phi = lagrange(N, xi, a % N, y[0]) * lagrange(N, xi, (a / N) % N, y[1]) *
                             lagrange(N, xi, a / (N * N), y[2]);
                for (int v = 0; v < NV; ++v)
                    acc[v * N3 + a] += wt * phi * u[((long)v * from->nc + f) * N3 + b];
            }
        }
        return;
    }
    if (l >= from->max_level) return;
    for (int c2 = 0; c2 < 3; ++c2)
        for (int c1 = 0; c1 < 3; ++c1)
            for (int c0 = 0; c0 < 3; ++c0) {
                int q2[3] = { 3 * q[0] + c0, 3 * q[1] + c1, 3 * q[2] + c2 };
                project_region(from, u, lc, kc, l + 1, q2, xi, w, acc, vol);
            }
}

/* Volumetric data of a new mesh from an old one of the same box and order,
 * u [5][nc][N^3] on both (Sec. 2.3: refinement interpolates volumetric data,
 * coarsening merges cells).  For every cell C of `to`:
 *   - C is a leaf of `from`: copied;
 *   - C lies in a coarser leaf P of `from`: P's polynomial evaluated at C's
 *     nodes (exact: the space of C contains P's polynomial restricted to C);
 *   - C is covered by finer leaves of `from`: the L2 projection onto C's
 *     polynomials, u_C(a) = (1 / (|C| w_a0 w_a1 w_a2)) * int_C u phi_a.
 * Returns 1 if a cell of `to` is only partly covered by `from`. */
int orc_volume_transfer(const orc_mesh *from, const double *u_from, const orc_mesh *to, double *u_to)
{
    int N = to->N, N3 = N * N * N;
    if (from->N != N) return 1;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    int rc = 0;
    double *acc = (double *)malloc(sizeof(double) * NV * N3);
    for (long c = 0; c < to->nc; ++c) {
        int l = to->lev[c];
        const int *k = &to->ijk[3 * c];
        long s = find_cell(from, l, k);
        if (s >= 0) {
            for (int v = 0; v < NV; ++v)
                for (int a = 0; a < N3; ++a)
                    u_to[((long)v * to->nc + c) * N3 + a] = u_from[((long)v * from->nc + s) * N3 + a];
            continue;
        }
        long p = -1;
        int lp = -1, kp[3];
        for (int l2 = l - 1; l2 >= 0 && p < 0; --l2) {
            long r = ipow3(l - l2);
            for (int d = 0; d < 3; ++d) kp[d] = (int)(k[d] / r);
            p = find_cell(from, l2, kp);
            lp = l2;
        }
        if (p >= 0) {
            double r = (double)ipow3(l - lp);
            for (int a = 0; a < N3; ++a) {
                int aa[3] = { a % N, (a / N) % N, a / (N * N) };
                double y[3], val[NV];
                for (int d = 0; d < 3; ++d) y[d] = (k[d] + xi[aa[d]]) / r - kp[d];
                eval_cell(from, u_from, p, xi, y, val);
                for (int v = 0; v < NV; ++v) u_to[((long)v * to->nc + c) * N3 + a] = val[v];
            }
            continue;
        }
        memset(acc, 0, sizeof(double) * NV * N3);
        double vol = 0.0;
        project_region(from, u_from, l, k, l, k, xi, w, acc, &vol);
        if (fabs(vol - 1.0) > 1e-12) rc = 1;
        for (int a = 0; a < N3; ++a) {
            double wa = w[a % N] * w[(a / N) % N] * w[a / (N * N)];
            for (int v = 0; v < NV; ++v) u_to[((long)v * to->nc + c) * N3 + a] = acc[v * N3 + a] / wa;
        }
    }
    free(acc);
    return rc;
}

/* Integral of every variable over the box: sum over cells of |cell| times
 * the Gauss rule of the cell. */
void orc_integral(const orc_mesh *m, const double *u, double *out)
{
    int N = m->N, N3 = N * N * N;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    for (int v = 0; v < NV; ++v) out[v] = 0.0;
    for (long c = 0; c < m->nc; ++c) {
        double dx[3];
        cell_dx(m, c, dx);
        double vol = dx[0] * dx[1] * dx[2];
        for (int a = 0; a < N3; ++a) {
            double wa = w[a % N] * w[(a / N) % N] * w[a / (N * N)];
            for (int v = 0; v < NV; ++v) out[v] += vol * wa * u[((long)v * m->nc + c) * N3 + a];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* A-posteriori finite-volume subcell limiter                                */
/* ------------------------------------------------------------------------- */

/* The limiter of Sec. 5.3 (block-structured methods) and Sec. 6 (Euler
 * with shocks): after the ADER-DG update, a cell whose new solution is physically
 * wrong or oscillates is rolled back and advanced over the same dt by a
 * finite-volume scheme on (2p+1)^3 equal subcells.  Readings (the paper
 * leaves the details to the limiter's own literature):
 *   - the old subcell data of a cell are the subcell averages of its
 *     polynomial; if one of them is unphysical, every subcell takes the cell
 *     mean instead (a convex combination of the physical nodal states);
 *   - the FV scheme is first order (piecewise constant data, Sec. 3: FV is
 *     ADER-DG with a degenerate predictor) with the Rusanov flux on every
 *     subcell face, the speed being the larger |u_d| + c of its two states;
 *   - a cell is troubled if its candidate has a non-finite value, rho <= 0
 *     or p <= 0 at a node or in a subcell average, or if a subcell average
 *     of a variable leaves [m - delta, M + delta], where m and M are the
 *     smallest and largest old subcell averages of that variable in the cell
 *     and its face neighbours, delta = max(delta0, eps (M - m));
 *   - the limited cell's new polynomial is the least-squares fit to its new
 *     subcell averages (it keeps the cell mean); if that polynomial is
 *     unphysical at a node or in a subcell average, the cell takes the
 *     constant state of the mean;
 *   - on a face between a limited cell and an unlimited one, the unlimited
 *     cell's face flux is replaced by the L2 projection of the subcell face
 *     fluxes onto the face polynomials and its corrector is run again, so
 *     that both sides see the same flux (conservation).
 * On adaptive meshes (Sec. 6: the solution is refined down to the FV level
 * near shocks, so no resolution transition cuts an FV region) only cells
 * whose six sides are conforming can be limited.  A troubled cell with a
 * hanging side keeps its unlimited candidate and is reported (flag 3); the
 * bounds of the relaxed maximum principle run over the cell and its
 * conforming face neighbours. */

/* 1 if every side of cell c is conforming (a same-level face neighbour). */
static int all_conforming(const orc_mesh *m, long c)
{
    for (int s = 0; s < 6; ++s)
        if (m->kind[6 * c + s] != SIDE_CONFORMING) return 0;
    return 1;
}

/* 1-D subcell operators for N = p+1 nodes and ns = 2p+1 subintervals:
 *   A[s][k]    average of phi_k over subinterval s
 *              = sum_q w_q phi_k((s + xi_q)/ns)  (N-point Gauss, exact);
 *   Ap[k][s]   least-squares inverse (A^T A)^{-1} A^T;
 *   B[k][s]    L2 projection of piecewise constants onto the polynomials:
 *              (B F)_k = (1/w_k) int phi_k F = sum_s F_s A[s][k] / (ns w_k).
 * Any pointer may be NULL.  Returns nonzero on bad N. */
int orc_subcell_ops(int N, double *A, double *Ap, double *B)
{
    if (N < 1 || N > MAXN) return 1;
    int ns = 2 * N - 1;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    double Aloc[(2 * MAXN - 1) * MAXN];
    for (int s = 0; s < ns; ++s)
        for (int k = 0; k < N; ++k) {
            double acc = 0.0;
            for (int q = 0; q < N; ++q) acc += w[q] * lagrange(N, xi, k, (s + xi[q]) / ns);
            Aloc[s * N + k] = acc;
        }
    if (A) memcpy(A, Aloc, sizeof(double) * ns * N);
    if (B)
        for (int k = 0; k < N; ++k)
            for (int s = 0; s < ns; ++s) B[k * ns + s] = Aloc[s * N + k] / (ns * w[k]);
    if (Ap) {
        double AtA[MAXN * MAXN], inv[MAXN * MAXN];
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
                double acc = 0.0;
                for (int s = 0; s < ns; ++s) acc += Aloc[s * N + i] * Aloc[s * N + j];
                AtA[i * N + j] = acc;
            }
        if (invert(N, AtA, inv)) return 1;
        for (int k = 0; k < N; ++k)
            for (int s = 0; s < ns; ++s) {
                double acc = 0.0;
                for (int j = 0; j < N; ++j) acc += inv[k * N + j] * Aloc[s * N + j];
                Ap[k * ns + s] = acc;
            }
    }
    return 0;
}

/* Subcell averages v[5][ns^3] (subcell index s0 + ns s1 + ns^2 s2) of cell c:
 * v_s = sum_a A[s0][a0] A[s1][a1] A[s2][a2] u_a. */
static void subcell_averages(int N, long nc, const double *A, const double *u, long c, double *v)
{
    int ns = 2 * N - 1, N3 = N * N * N, S3 = ns * ns * ns;
    for (int vv = 0; vv < NV; ++vv)
        for (int s = 0; s < S3; ++s) {
            int ss[3] = { s % ns, (s / ns) % ns, s / (ns * ns) };
            double acc = 0.0;
            for (int a = 0; a < N3; ++a)
                acc += A[ss[0] * N + a % N] * A[ss[1] * N + (a / N) % N] * A[ss[2] * N + a / (N * N)] *
                       u[((long)vv * nc + c) * N3 + a];
            v[vv * S3 + s] = acc;
        }
}

/* Old subcell data of cell c: the subcell averages, or the cell mean in
 * every subcell if an average is unphysical. */
static void subcell_data(int N, long nc, double g, const double *A, const double *u, long c, double *v)
{
    int ns = 2 * N - 1, N3 = N * N * N, S3 = ns * ns * ns;
    subcell_averages(N, nc, A, u, c, v);
    int bad = 0;
    for (int s = 0; s < S3 && !bad; ++s) {
        double q[NV];
        for (int vv = 0; vv < NV; ++vv) q[vv] = v[vv * S3 + s];
        bad = unphysical(g, q);
    }
    if (!bad) return;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    for (int vv = 0; vv < NV; ++vv) {
        double mean = 0.0;
        for (int a = 0; a < N3; ++a)
            mean += w[a % N] * w[(a / N) % N] * w[a / (N * N)] * u[((long)vv * nc + c) * N3 + a];
        for (int s = 0; s < S3; ++s) v[vv * S3 + s] = mean;
    }
}

/* Rusanov flux along d between subcell states ql (minus side) and qr. */
static void rusanov_point(double g, int d, const double ql[NV], const double qr[NV], double f[NV])
{
    double fl[NV], fr[NV];
    euler_flux(g, ql, d, fl);
    euler_flux(g, qr, d, fr);
    double sl = euler_speed(g, ql, d), sr = euler_speed(g, qr, d);
    double smax = sl > sr ? sl : sr;
    for (int v = 0; v < NV; ++v) f[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * smax * (qr[v] - ql[v]);
}

/* Troubled-cell test of one cell (see the readings above).  ucand: candidate
 * polynomial of the whole mesh; vcand: the cell's candidate subcell averages;
 * lo, hi: [5] neighbourhood bounds of the old averages. */
static int is_troubled(int N, long nc, double g, const double *ucand, long c, const double *vcand,
                       const double *lo, const double *hi, double delta0, double eps)
{
    int ns = 2 * N - 1, N3 = N * N * N, S3 = ns * ns * ns;
    for (int a = 0; a < N3; ++a) {
        double q[NV];
        for (int v = 0; v < NV; ++v) q[v] = ucand[((long)v * nc + c) * N3 + a];
        if (unphysical(g, q)) return 1;
    }
    for (int s = 0; s < S3; ++s) {
        double q[NV];
        for (int v = 0; v < NV; ++v) q[v] = vcand[v * S3 + s];
        if (unphysical(g, q)) return 1;
    }
    for (int v = 0; v < NV; ++v) {
        double delta = eps * (hi[v] - lo[v]);
        if (delta < delta0) delta = delta0;
        for (int s = 0; s < S3; ++s) {
            double x = vcand[v * S3 + s];
            if (!(x >= lo[v] - delta && x <= hi[v] + delta)) return 1;
        }
    }
    return 0;
}

/* Troubled-cell flags (1 troubled, 0 not) of candidate ucand given the old
 * solution uold, both [5][nc][N^3].  Returns 3 if the mesh has a hanging
 * face, 2 on allocation failure, else 0. */
int orc_limiter_detect(const orc_mesh *m, double g, double delta0, double eps, const double *uold,
                       const double *ucand, int *flags)
{
    int N = m->N, ns = 2 * N - 1, S3 = ns * ns * ns;
    long nc = m->nc;
    double A[(2 * MAXN - 1) * MAXN];
    if (orc_subcell_ops(N, A, NULL, NULL)) return 2;
    double *bnd = (double *)malloc(sizeof(double) * nc * 2 * NV);
    if (!bnd) return 2;
    /* per-cell extremes of the old subcell averages */
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * NV * S3);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            subcell_data(N, nc, g, A, uold, c, tmp);
            for (int v = 0; v < NV; ++v) {
                double lo = tmp[v * S3], hi = tmp[v * S3];
                for (int s = 0; s < S3; ++s) {
                    if (tmp[v * S3 + s] < lo) lo = tmp[v * S3 + s];
                    if (tmp[v * S3 + s] > hi) hi = tmp[v * S3 + s];
                }
                bnd[(c * 2 + 0) * NV + v] = lo;
                bnd[(c * 2 + 1) * NV + v] = hi;
            }
        }
        free(tmp);
    }
    /* bounds over the cell and its face neighbours; test the candidate */
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * NV * S3);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            double lo[NV], hi[NV];
            for (int v = 0; v < NV; ++v) {
                lo[v] = bnd[(c * 2 + 0) * NV + v];
                hi[v] = bnd[(c * 2 + 1) * NV + v];
            }
            for (int s = 0; s < 6; ++s) {
                if (m->kind[6 * c + s] != SIDE_CONFORMING) continue;
                long o = m->nbr[6 * c + s];
                for (int v = 0; v < NV; ++v) {
                    if (bnd[(o * 2 + 0) * NV + v] < lo[v]) lo[v] = bnd[(o * 2 + 0) * NV + v];
                    if (bnd[(o * 2 + 1) * NV + v] > hi[v]) hi[v] = bnd[(o * 2 + 1) * NV + v];
                }
            }
            subcell_averages(N, nc, A, ucand, c, tmp);
            flags[c] = is_troubled(N, nc, g, ucand, c, tmp, lo, hi, delta0, eps);
            if (flags[c] && !all_conforming(m, c)) flags[c] = 3;
        }
        free(tmp);
    }
    free(bnd);
    return 0;
}

/* Old subcell average of neighbour/own data at subcell (s0,s1,s2), variable v. */
#define VOLD(cell, v, s) vold[((long)(cell) * NV + (v)) * S3 + (s)]

/* One limited ADER-DG step of size dt in place on u.  flags[nc] receives 1
 * for limited cells, 2 for unlimited cells whose corrector ran again, 3 for
 * troubled cells that cannot be limited (a hanging side), 0 otherwise.
 * force != 0 limits every cell that can be limited (test hook).  Returns 0,
 * 1 if the final state is unphysical somewhere, 2 on allocation failure. */
int orc_limited_step(const orc_mesh *m, double g, int npic, double dt, double delta0, double eps, int force,
                     double *u, int *flags)
{
    int N = m->N, N2 = N * N, N3 = N2 * N, ns = 2 * N - 1, S2 = ns * ns, S3 = S2 * ns;
    long nc = m->nc;
    double A[(2 * MAXN - 1) * MAXN], Ap[MAXN * (2 * MAXN - 1)], B[MAXN * (2 * MAXN - 1)];
    if (orc_subcell_ops(N, A, Ap, B)) return 2;
    double xi[MAXN], w[MAXN], D[MAXN * MAXN], L[MAXN], R[MAXN], Kinv[MAXN * MAXN], Kw[MAXN * MAXN];
    orc_basis(N, xi, w, D, L, R, Kinv, Kw);
    double *vold = (double *)malloc(sizeof(double) * nc * NV * S3);
    double *us = (double *)malloc(sizeof(double) * NV * nc * N3);
    double *tr = (double *)malloc(sizeof(double) * 6 * 2 * NV * nc * N2);
    double *fs = (double *)malloc(sizeof(double) * 6 * NV * nc * N2);
    double *un = (double *)malloc(sizeof(double) * NV * nc * N3);
    if (!vold || !us || !tr || !fs || !un) {
        free(vold); free(us); free(tr); free(fs); free(un);
        return 2;
    }
    /* old subcell data */
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * NV * S3);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            subcell_data(N, nc, g, A, u, c, tmp);
            for (int v = 0; v < NV; ++v)
                for (int s = 0; s < S3; ++s) VOLD(c, v, s) = tmp[v * S3 + s];
        }
        free(tmp);
    }
    /* the unlimited candidate (unphysical states are what the limiter is for) */
    orc_predictor(m, g, npic, dt, u, us, tr);
    (void)orc_riemann(m, g, tr, fs);
    orc_corrector(m, dt, us, fs, un);
    /* detection (u still holds the old solution) */
    if (force) {
        for (long c = 0; c < nc; ++c) flags[c] = all_conforming(m, c) ? 1 : 3;
    } else if (orc_limiter_detect(m, g, delta0, eps, u, un, flags)) {
        free(vold); free(us); free(tr); free(fs); free(un);
        return 2;
    }
    /* finite-volume update of the limited cells; projected face fluxes for
     * their unlimited neighbours */
#pragma omp parallel
    {
        double *vn = (double *)malloc(sizeof(double) * NV * S3);
        double *vfit = (double *)malloc(sizeof(double) * NV * S3);
        double *Fsub = (double *)malloc(sizeof(double) * NV * S2);
#pragma omp for schedule(dynamic)
        for (long c = 0; c < nc; ++c) {
            if (flags[c] != 1) continue;
            double dx[3];
            cell_dx(m, c, dx);
            for (int s = 0; s < S3; ++s) {
                int ss[3] = { s % ns, (s / ns) % ns, s / S2 };
                double q[NV], acc[NV] = { 0 };
                for (int v = 0; v < NV; ++v) q[v] = VOLD(c, v, s);
                for (int d = 0; d < 3; ++d) {
                    double h = dx[d] / ns;
                    for (int side = 0; side < 2; ++side) {
                        /* state across the subcell face on this side */
                        double qo[NV];
                        int sn[3] = { ss[0], ss[1], ss[2] };
                        long co = c;
                        sn[d] += side ? 1 : -1;
                        if (sn[d] < 0 || sn[d] >= ns) {
                            co = m->nbr[6 * c + 2 * d + side];
                            sn[d] = side ? 0 : ns - 1;
                        }
                        int so = sn[0] + ns * sn[1] + S2 * sn[2];
                        for (int v = 0; v < NV; ++v) qo[v] = VOLD(co, v, so);
                        double f[NV];
                        if (side) rusanov_point(g, d, q, qo, f);
                        else rusanov_point(g, d, qo, q, f);
                        for (int v = 0; v < NV; ++v) acc[v] += (side ? 1.0 : -1.0) * f[v] / h;
                    }
                }
                for (int v = 0; v < NV; ++v) vn[v * S3 + s] = q[v] - dt * acc[v];
            }
            /* least-squares polynomial of the new averages */
            for (int v = 0; v < NV; ++v)
                for (int a = 0; a < N3; ++a) {
                    int aa[3] = { a % N, (a / N) % N, a / N2 };
                    double acc = 0.0;
                    for (int s = 0; s < S3; ++s)
                        acc += Ap[aa[0] * ns + s % ns] * Ap[aa[1] * ns + (s / ns) % ns] * Ap[aa[2] * ns + s / S2] *
                               vn[v * S3 + s];
                    un[((long)v * nc + c) * N3 + a] = acc;
                }
            /* an unphysical fit falls back to the constant mean state */
            int bad = 0;
            for (int a = 0; a < N3 && !bad; ++a) {
                double q[NV];
                for (int v = 0; v < NV; ++v) q[v] = un[((long)v * nc + c) * N3 + a];
                bad = unphysical(g, q);
            }
            if (!bad) {
                subcell_averages(N, nc, A, un, c, vfit);
                for (int s = 0; s < S3 && !bad; ++s) {
                    double q[NV];
                    for (int v = 0; v < NV; ++v) q[v] = vfit[v * S3 + s];
                    bad = unphysical(g, q);
                }
            }
            if (bad)
                for (int v = 0; v < NV; ++v) {
                    double mean = 0.0;
                    for (int s = 0; s < S3; ++s) mean += vn[v * S3 + s];
                    mean /= S3;
                    for (int a = 0; a < N3; ++a) un[((long)v * nc + c) * N3 + a] = mean;
                }
            /* subcell fluxes on the faces shared with unlimited cells */
            for (int side6 = 0; side6 < 6; ++side6) {
                int d = side6 / 2, plus = side6 % 2;
                long o = m->nbr[6 * c + side6];
                if (flags[o] == 1) continue;
                int t1, t2;
                tangential(d, &t1, &t2);
                for (int j2 = 0; j2 < ns; ++j2)
                    for (int j1 = 0; j1 < ns; ++j1) {
                        int sc[3], so[3];
                        sc[t1] = so[t1] = j1;
                        sc[t2] = so[t2] = j2;
                        sc[d] = plus ? ns - 1 : 0;
                        so[d] = plus ? 0 : ns - 1;
                        int ic = sc[0] + ns * sc[1] + S2 * sc[2], io = so[0] + ns * so[1] + S2 * so[2];
                        double qc[NV], qo[NV], f[NV];
                        for (int v = 0; v < NV; ++v) {
                            qc[v] = VOLD(c, v, ic);
                            qo[v] = VOLD(o, v, io);
                        }
                        if (plus) rusanov_point(g, d, qc, qo, f);
                        else rusanov_point(g, d, qo, qc, f);
                        for (int v = 0; v < NV; ++v) Fsub[v * S2 + j1 + ns * j2] = f[v];
                    }
                int sopp = 2 * d + (1 - plus);
                for (int v = 0; v < NV; ++v)
                    for (int b = 0; b < N2; ++b) {
                        int b1 = b % N, b2 = b / N;
                        double acc = 0.0;
                        for (int j = 0; j < S2; ++j)
                            acc += B[b1 * ns + j % ns] * B[b2 * ns + j / ns] * Fsub[v * S2 + j];
                        fs[((long)(sopp * NV + v) * nc + o) * N2 + b] = acc;
                    }
            }
        }
        free(vn);
        free(vfit);
        free(Fsub);
    }
    /* unlimited cells next to a limited one (flag 2, or 3 kept for a
     * troubled cell that cannot be limited): corrector again with the new
     * face fluxes (written out as in orc_corrector) */
    unsigned char *rerun = (unsigned char *)calloc(nc > 0 ? nc : 1, 1);
    if (!rerun) {
        free(vold); free(us); free(tr); free(fs); free(un);
        return 2;
    }
    for (long c = 0; c < nc; ++c) {
        if (flags[c] == 1) continue;
        int near = 0;
        for (int s = 0; s < 6; ++s)
            if (m->kind[6 * c + s] == SIDE_CONFORMING && flags[m->nbr[6 * c + s]] == 1) near = 1;
        if (near) {
            rerun[c] = 1;
            if (flags[c] == 0) flags[c] = 2;
        }
    }
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        if (!rerun[c]) continue;
        double dx[3];
        cell_dx(m, c, dx);
        for (int v = 0; v < NV; ++v)
            for (int a = 0; a < N3; ++a) {
                int aa[3] = { a % N, (a / N) % N, a / N2 };
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int b = face_index(N, a, d);
                    double fm = fs[((long)((2 * d) * NV + v) * nc + c) * N2 + b];
                    double fp = fs[((long)((2 * d + 1) * NV + v) * nc + c) * N2 + b];
                    s += (dt / dx[d]) * (R[aa[d]] * fp - L[aa[d]] * fm) / w[aa[d]];
                }
                un[((long)v * nc + c) * N3 + a] = us[((long)v * nc + c) * N3 + a] - s;
            }
    }
    free(rerun);
    memcpy(u, un, sizeof(double) * NV * nc * N3);
    int rc = 0;
    for (long c = 0; c < nc && !rc; ++c)
        for (int a = 0; a < N3; ++a) {
            double q[NV];
            for (int v = 0; v < NV; ++v) q[v] = u[((long)v * nc + c) * N3 + a];
            if (unphysical(g, q)) { rc = 1; break; }
        }
    free(vold); free(us); free(tr); free(fs); free(un);
    return rc;
}
#undef VOLD

/* nsteps limited steps in place on u, dt from orc_cfl (or dt_fixed > 0).
 * dt_hist[n] and ntroubled[n] (may be NULL) receive each step's dt and its
 * number of limited cells; flags holds the last step's flags.  Returns the
 * first nonzero orc_limited_step code (u then holds that step's result), or
 * 1 if a CFL evaluation meets an unphysical state. */
int orc_run_limited(const orc_mesh *m, double g, double cfl, int npic, double dt_fixed, double delta0, double eps,
                    int force, double *u, int nsteps, double *dt_hist, long *ntroubled, int *flags)
{
    for (int n = 0; n < nsteps; ++n) {
        int st = 0;
        double dt = dt_fixed > 0.0 ? dt_fixed : orc_cfl(m, g, cfl, u, &st);
        if (st) return 1;
        if (dt_hist) dt_hist[n] = dt;
        int rc = orc_limited_step(m, g, npic, dt, delta0, eps, force, u, flags);
        if (ntroubled) {
            long k = 0;
            for (long c = 0; c < m->nc; ++c) k += flags[c] == 1;
            ntroubled[n] = k;
        }
        if (rc) return rc;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Linear PDE: elastic waves, space-time predictor by Cauchy-Kowalevski      */
/* ------------------------------------------------------------------------- */

/* The seismic variant (Sec. 2.4: a linear PDE is integrated in time by the
 * Cauchy-Kowalevski procedure instead of an iterative predictor; Sec. 6: the
 * seismic benchmark is elastic wave propagation with the material carried
 * along as time-constant unknowns).  Readings:
 *   - 3-D linear elasticity in velocity-stress form, 9 unknowns
 *     q = (s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, v_x, v_y, v_z):
 *       d_t s_ij = lambda delta_ij div v + mu (d_i v_j + d_j v_i),
 *       rho d_t v_i = sum_j d_j s_ij,
 *     written as d_t q + sum_d d_d (A_d q) = 0;
 *   - the material (rho, lambda, mu) is constant inside each cell (the
 *     paper's time-constant material unknowns, stored once per cell);
 *   - Cauchy-Kowalevski: d_t^k q = L^k q with L q = -sum_d (1/dx_d) A_d D_d q
 *     on the nodal polynomial; L lowers the degree, so the series ends after
 *     p+1 terms and the time average is exact:
 *       qbar = sum_{k=0}^{p} dt^k / (k+1)! L^k u;
 *   - the rest of the step is the one of the Euler path with the flux A_d q:
 *     volume term, face projections, one Rusanov solve per face with the
 *     larger P-wave speed of its two cells, corrector;
 *   - dt = cfl / ((2p+1) max_c c_p(c) sum_d 1/dx_d), c_p = sqrt((lambda+2mu)/rho).
 * Layouts: u [9][nc][N^3], traces [6][2][9][nc][N^2], fside [6][9][nc][N^2],
 * material [3][nc] (rho, lambda, mu).  Uniform meshes. */
#define NL 9
enum { SXX = 0, SYY, SZZ, SXY, SYZ, SXZ, VX, VY, VZ };

/* f = A_d q for material (rho, lambda, mu) */
static void elastic_flux(const double mat[3], const double q[NL], int d, double f[NL])
{
    double rho = mat[0], lam = mat[1], mu = mat[2];
    for (int v = 0; v < NL; ++v) f[v] = 0.0;
    if (d == 0) {
        f[SXX] = -(lam + 2 * mu) * q[VX];
        f[SYY] = -lam * q[VX];
        f[SZZ] = -lam * q[VX];
        f[SXY] = -mu * q[VY];
        f[SXZ] = -mu * q[VZ];
        f[VX] = -q[SXX] / rho;
        f[VY] = -q[SXY] / rho;
        f[VZ] = -q[SXZ] / rho;
    } else if (d == 1) {
        f[SXX] = -lam * q[VY];
        f[SYY] = -(lam + 2 * mu) * q[VY];
        f[SZZ] = -lam * q[VY];
        f[SXY] = -mu * q[VX];
        f[SYZ] = -mu * q[VZ];
        f[VX] = -q[SXY] / rho;
        f[VY] = -q[SYY] / rho;
        f[VZ] = -q[SYZ] / rho;
    } else {
        f[SXX] = -lam * q[VZ];
        f[SYY] = -lam * q[VZ];
        f[SZZ] = -(lam + 2 * mu) * q[VZ];
        f[SYZ] = -mu * q[VY];
        f[SXZ] = -mu * q[VX];
        f[VX] = -q[SXZ] / rho;
        f[VY] = -q[SYZ] / rho;
        f[VZ] = -q[SZZ] / rho;
    }
}

static double p_speed(const double mat[3]) { return sqrt((mat[1] + 2 * mat[2]) / mat[0]); }

static void cell_mat(const orc_mesh *m, const double *mat, long c, double out[3])
{
    for (int k = 0; k < 3; ++k) out[k] = mat[(long)k * m->nc + c];
}

/* A_d as a 9 x 9 matrix (row-major), column k = A_d e_k */
void orc_lin_flux_matrix(const double mat[3], int d, double *A)
{
    for (int k = 0; k < NL; ++k) {
        double e[NL] = { 0 }, f[NL];
        e[k] = 1.0;
        elastic_flux(mat, e, d, f);
        for (int r = 0; r < NL; ++r) A[r * NL + k] = f[r];
    }
}

/* Shared epilogue: from qbar (one cell, [9][N^3]) the volume term into ustar
 * and the face projections of qbar and of the normal flux into traces. */
static void lin_epilogue(const orc_mesh *m, long c, const double *cm, double dt, const double *uc,
                         const double *qbar, const double *D, const double *L, const double *R,
                         const double *w, const double *Kw, double *ustar, double *traces)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    double dx[3];
    cell_dx(m, c, dx);
    double *Fbar = (double *)malloc(sizeof(double) * 3 * NL * N3);
    for (int a = 0; a < N3; ++a) {
        double qq[NL], f[NL];
        for (int v = 0; v < NL; ++v) qq[v] = qbar[v * N3 + a];
        for (int d = 0; d < 3; ++d) {
            elastic_flux(cm, qq, d, f);
            for (int v = 0; v < NL; ++v) Fbar[(d * NL + v) * N3 + a] = f[v];
        }
    }
    (void)D;
    for (int v = 0; v < NL; ++v)
        for (int a = 0; a < N3; ++a) {
            int aa[3] = { a % N, (a / N) % N, a / N2 };
            double s = 0.0;
            for (int d = 0; d < 3; ++d) {
                double sd = 0.0;
                for (int e = 0; e < N; ++e) sd += Kw[aa[d] * N + e] * Fbar[(d * NL + v) * N3 + node_with(N, a, d, e)];
                s += (dt / dx[d]) * sd / w[aa[d]];
            }
            ustar[((long)v * nc + c) * N3 + a] = uc[v * N3 + a] + s;
        }
    for (int s = 0; s < 6; ++s) {
        int d = s / 2;
        const double *E = (s % 2) ? R : L;
        for (int v = 0; v < NL; ++v)
            for (int b = 0; b < N2; ++b) {
                double sq = 0.0, sf = 0.0;
                for (int e = 0; e < N; ++e) {
                    int a = node_from_face(N, d, e, b);
                    sq += E[e] * qbar[v * N3 + a];
                    sf += E[e] * Fbar[(d * NL + v) * N3 + a];
                }
                traces[(((long)(s * 2 + 0) * NL + v) * nc + c) * N2 + b] = sq;
                traces[(((long)(s * 2 + 1) * NL + v) * nc + c) * N2 + b] = sf;
            }
    }
    free(Fbar);
}

/* Predictor of the elastic system.  ck != 0: Cauchy-Kowalevski as above;
 * ck == 0: the Picard iteration of orc_predictor with the flux A_d q and
 * npic iterations (test reference: for a linear PDE, p+1 iterations reach
 * the same space-time polynomial). */
void orc_lin_predictor(const orc_mesh *m, const double *mat, double dt, int ck, int npic, const double *u,
                       double *ustar, double *traces)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    double xi[MAXN], w[MAXN], D[MAXN * MAXN], L[MAXN], R[MAXN], Kinv[MAXN * MAXN], Kw[MAXN * MAXN];
    orc_basis(N, xi, w, D, L, R, Kinv, Kw);
#pragma omp parallel
    {
        double *uc = (double *)malloc(sizeof(double) * NL * N3);
        double *qbar = (double *)malloc(sizeof(double) * NL * N3);
        double *dk = (double *)malloc(sizeof(double) * NL * N3);
        double *dn = (double *)malloc(sizeof(double) * NL * N3);
        double *q = (double *)malloc(sizeof(double) * N * NL * N3);
        double *qn = (double *)malloc(sizeof(double) * N * NL * N3);
        double *F = (double *)malloc(sizeof(double) * N * 3 * NL * N3);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            double cm[3], dx[3];
            cell_mat(m, mat, c, cm);
            cell_dx(m, c, dx);
            for (int v = 0; v < NL; ++v)
                for (int a = 0; a < N3; ++a) uc[v * N3 + a] = u[((long)v * nc + c) * N3 + a];
            if (ck) {
                memcpy(dk, uc, sizeof(double) * NL * N3);
                memcpy(qbar, uc, sizeof(double) * NL * N3);
                double fac = 1.0;
                for (int k = 1; k < N; ++k) {
                    /* dn = L dk = -sum_d (1/dx_d) D_d (A_d dk) */
                    for (int v = 0; v < NL; ++v)
                        for (int a = 0; a < N3; ++a) {
                            int aa[3] = { a % N, (a / N) % N, a / N2 };
                            double s = 0.0;
                            for (int d = 0; d < 3; ++d) {
                                double sd = 0.0;
                                for (int e = 0; e < N; ++e) {
                                    int b = node_with(N, a, d, e);
                                    double qq[NL], f[NL];
                                    for (int vv = 0; vv < NL; ++vv) qq[vv] = dk[vv * N3 + b];
                                    elastic_flux(cm, qq, d, f);
                                    sd += D[aa[d] * N + e] * f[v];
                                }
                                s += sd / dx[d];
                            }
                            dn[v * N3 + a] = -s;
                        }
                    memcpy(dk, dn, sizeof(double) * NL * N3);
                    fac *= dt / (k + 1);
                    for (int i = 0; i < NL * N3; ++i) qbar[i] += fac * dk[i];
                }
            } else {
                for (int l = 0; l < N; ++l) memcpy(q + l * NL * N3, uc, sizeof(double) * NL * N3);
                for (int it = 0; it < npic; ++it) {
                    for (int j = 0; j < N; ++j)
                        for (int a = 0; a < N3; ++a) {
                            double qq[NL], f[NL];
                            for (int v = 0; v < NL; ++v) qq[v] = q[(j * NL + v) * N3 + a];
                            for (int d = 0; d < 3; ++d) {
                                elastic_flux(cm, qq, d, f);
                                for (int v = 0; v < NL; ++v) F[((j * 3 + d) * NL + v) * N3 + a] = f[v];
                            }
                        }
                    for (int l = 0; l < N; ++l)
                        for (int v = 0; v < NL; ++v)
                            for (int a = 0; a < N3; ++a) {
                                int aa[3] = { a % N, (a / N) % N, a / N2 };
                                double s = 0.0;
                                for (int j = 0; j < N; ++j) {
                                    double g = 0.0;
                                    for (int d = 0; d < 3; ++d) {
                                        double sd = 0.0;
                                        for (int e = 0; e < N; ++e)
                                            sd += D[aa[d] * N + e] * F[((j * 3 + d) * NL + v) * N3 + node_with(N, a, d, e)];
                                        g += (dt / dx[d]) * sd;
                                    }
                                    s += Kinv[l * N + j] * w[j] * g;
                                }
                                qn[(l * NL + v) * N3 + a] = uc[v * N3 + a] - s;
                            }
                    double *t = q; q = qn; qn = t;
                }
                for (int v = 0; v < NL; ++v)
                    for (int a = 0; a < N3; ++a) {
                        double s = 0.0;
                        for (int j = 0; j < N; ++j) s += w[j] * q[(j * NL + v) * N3 + a];
                        qbar[v * N3 + a] = s;
                    }
            }
            lin_epilogue(m, c, cm, dt, uc, qbar, D, L, R, w, Kw, ustar, traces);
        }
        free(uc); free(qbar); free(dk); free(dn); free(q); free(qn); free(F);
    }
}

/* Rusanov on every face (uniform mesh): F = (F_L + F_R)/2 - s (Q_R - Q_L)/2
 * with s the larger P-wave speed of the two cells; both sides get F. */
void orc_lin_riemann(const orc_mesh *m, const double *mat, const double *traces, double *fside)
{
    int N = m->N, N2 = N * N;
    long nc = m->nc;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c)
        for (int s = 0; s < 6; ++s) {
            int d = s / 2, plus = s % 2;
            long o = m->nbr[6 * c + s];
            int so = 2 * d + (1 - plus);
            long cl = plus ? c : o, cr = plus ? o : c;
            int sl = plus ? s : so, sr = plus ? so : s;
            double ml[3], mr[3];
            cell_mat(m, mat, cl, ml);
            cell_mat(m, mat, cr, mr);
            double sp = p_speed(ml) > p_speed(mr) ? p_speed(ml) : p_speed(mr);
            for (int v = 0; v < NL; ++v)
                for (int b = 0; b < N2; ++b) {
                    double QL = traces[(((long)(sl * 2 + 0) * NL + v) * nc + cl) * N2 + b];
                    double FL = traces[(((long)(sl * 2 + 1) * NL + v) * nc + cl) * N2 + b];
                    double QR = traces[(((long)(sr * 2 + 0) * NL + v) * nc + cr) * N2 + b];
                    double FR = traces[(((long)(sr * 2 + 1) * NL + v) * nc + cr) * N2 + b];
                    fside[((long)(s * NL + v) * nc + c) * N2 + b] = 0.5 * (FL + FR) - 0.5 * sp * (QR - QL);
                }
        }
}

void orc_lin_corrector(const orc_mesh *m, double dt, const double *ustar, const double *fside, double *unew)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    double xi[MAXN], w[MAXN], D[MAXN * MAXN], L[MAXN], R[MAXN], Kinv[MAXN * MAXN], Kw[MAXN * MAXN];
    orc_basis(N, xi, w, D, L, R, Kinv, Kw);
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nc; ++c) {
        double dx[3];
        cell_dx(m, c, dx);
        for (int v = 0; v < NL; ++v)
            for (int a = 0; a < N3; ++a) {
                int aa[3] = { a % N, (a / N) % N, a / N2 };
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int b = face_index(N, a, d);
                    double fm = fside[((long)((2 * d) * NL + v) * nc + c) * N2 + b];
                    double fp = fside[((long)((2 * d + 1) * NL + v) * nc + c) * N2 + b];
                    s += (dt / dx[d]) * (R[aa[d]] * fp - L[aa[d]] * fm) / w[aa[d]];
                }
                unew[((long)v * nc + c) * N3 + a] = ustar[((long)v * nc + c) * N3 + a] - s;
            }
    }
}

double orc_lin_cfl(const orc_mesh *m, const double *mat, double cfl)
{
    double best = 0.0;
    for (long c = 0; c < m->nc; ++c) {
        double cm[3], dx[3];
        cell_mat(m, mat, c, cm);
        cell_dx(m, c, dx);
        double r = p_speed(cm) * (1.0 / dx[0] + 1.0 / dx[1] + 1.0 / dx[2]);
        if (r > best) best = r;
    }
    return cfl / ((2.0 * (m->N - 1) + 1.0) * best);
}

/* Steps in place; dt from orc_lin_cfl (or dt_fixed > 0).  Returns 0, 2 on
 * allocation failure, 3 on a mesh with hanging faces. */
int orc_lin_run(const orc_mesh *m, const double *mat, double cfl, double dt_fixed, double *u, int nsteps,
                double *dt_out)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    for (long k = 0; k < 6 * nc; ++k)
        if (m->kind[k] != SIDE_CONFORMING) return 3;
    double *us = (double *)malloc(sizeof(double) * NL * nc * N3);
    double *tr = (double *)malloc(sizeof(double) * 6 * 2 * NL * nc * N2);
    double *fs = (double *)malloc(sizeof(double) * 6 * NL * nc * N2);
    if (!us || !tr || !fs) { free(us); free(tr); free(fs); return 2; }
    double dt = dt_fixed > 0.0 ? dt_fixed : orc_lin_cfl(m, mat, cfl);
    if (dt_out) *dt_out = dt;
    for (int n = 0; n < nsteps; ++n) {
        orc_lin_predictor(m, mat, dt, 1, 0, u, us, tr);
        orc_lin_riemann(m, mat, tr, fs);
        orc_lin_corrector(m, dt, us, fs, u);
    }
    free(us); free(tr); free(fs);
    return 0;
}

/* Elastic energy: sum over cells of |cell| sum_a W_a e(q_a),
 * e = rho |v|^2 / 2 + (s:s)/(4 mu) - lambda (tr s)^2 / (4 mu (3 lambda + 2 mu)). */
double orc_lin_energy(const orc_mesh *m, const double *mat, const double *u)
{
    int N = m->N, N3 = N * N * N;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    double total = 0.0;
    for (long c = 0; c < m->nc; ++c) {
        double cm[3], dx[3];
        cell_mat(m, mat, c, cm);
        cell_dx(m, c, dx);
        double rho = cm[0], lam = cm[1], mu = cm[2];
        for (int a = 0; a < N3; ++a) {
            double q[NL];
            for (int v = 0; v < NL; ++v) q[v] = u[((long)v * m->nc + c) * N3 + a];
            double ss = q[SXX] * q[SXX] + q[SYY] * q[SYY] + q[SZZ] * q[SZZ] +
                        2 * (q[SXY] * q[SXY] + q[SYZ] * q[SYZ] + q[SXZ] * q[SXZ]);
            double tr = q[SXX] + q[SYY] + q[SZZ];
            double e = 0.5 * rho * (q[VX] * q[VX] + q[VY] * q[VY] + q[VZ] * q[VZ]) + ss / (4 * mu) -
                       lam * tr * tr / (4 * mu * (3 * lam + 2 * mu));
            total += dx[0] * dx[1] * dx[2] * w[a % N] * w[(a / N) % N] * w[a / (N * N)] * e;
        }
    }
    return total;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Tangent-linear model and adjoint of one step at a fixed dt                */
/* ------------------------------------------------------------------------- */
/* At a fixed time step size the step u^n -> u^{n+1} (Eq. 3-4, Alg. 1) is a
 * piecewise-smooth map.  Its derivative goes through the same phases:
 *   - predictor: every Picard iterate, the time averages, the volume term and
 *     the face projections differentiate term by term (chain rule through the
 *     Euler flux);
 *   - Rusanov: F* = (F_L + F_R)/2 - s (Q_R - Q_L)/2 with s a maximum; s is
 *     differentiated at its FIRST maximiser in the order (face node, minus
 *     side first), and d|x|/dx is taken as 0 at x = 0;
 *   - virtual-cell interpolation, restriction and corrector are linear.
 * dt is held fixed: the CFL reduction is not differentiated.
 * The tangent (forward mode) carries K directions at once; the adjoint is the
 * transpose of the same phases in reverse order.  Both exist to check the
 * GPU adjoint; they are written plainly from the definitions above. */

/* d f_d(q)[dq]: directional derivative of the flux along axis d. */
static void euler_flux_tan(double g, const double q[NV], const double dq[NV], int d, double df[NV])
{
    double r = q[0], dr = dq[0];
    double mm = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    double mdm = q[1] * dq[1] + q[2] * dq[2] + q[3] * dq[3];
    double p = (g - 1.0) * (q[4] - 0.5 * mm / r);
    double dp = (g - 1.0) * (dq[4] - mdm / r + 0.5 * mm * dr / (r * r));
    double vd = q[1 + d] / r;
    double dvd = (dq[1 + d] - vd * dr) / r;
    df[0] = dq[1 + d];
    for (int i = 1; i <= 3; ++i) df[i] = dvd * q[i] + vd * dq[i];
    df[1 + d] += dp;
    df[4] = dvd * (q[4] + p) + vd * (dq[4] + dp);
}

/* d lambda_d(q)[dq] for lambda_d = |u_d| + c, with d|x|/dx = 0 at 0. */
static double euler_speed_tan(double g, const double q[NV], const double dq[NV], int d)
{
    double r = q[0], dr = dq[0];
    double mm = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    double mdm = q[1] * dq[1] + q[2] * dq[2] + q[3] * dq[3];
    double p = (g - 1.0) * (q[4] - 0.5 * mm / r);
    double dp = (g - 1.0) * (dq[4] - mdm / r + 0.5 * mm * dr / (r * r));
    double vd = q[1 + d] / r;
    double dvd = (dq[1 + d] - vd * dr) / r;
    double c = sqrt(g * p / r);
    double dc = g * (dp * r - p * dr) / (r * r) / (2.0 * c);
    double sg = vd > 0.0 ? 1.0 : (vd < 0.0 ? -1.0 : 0.0);
    return sg * dvd + dc;
}

/* f_d'(q)^T y, built column by column from the directional derivative. */
static void euler_flux_vjp(double g, const double q[NV], int d, const double y[NV], double out[NV])
{
    for (int k = 0; k < NV; ++k) {
        double e[NV] = { 0, 0, 0, 0, 0 }, df[NV];
        e[k] = 1.0;
        euler_flux_tan(g, q, e, d, df);
        double s = 0.0;
        for (int v = 0; v < NV; ++v) s += y[v] * df[v];
        out[k] = s;
    }
}

/* Face speed of the Rusanov flux and where it is attained: the first
 * maximiser in (node b, minus side first) order. */
static double rusanov_speed(double g, int d, int N2, const double *QL, const double *QR, int *bstar, int *side)
{
    double smax = 0.0;
    *bstar = -1;
    *side = 0;
    for (int b = 0; b < N2; ++b) {
        double ql[NV], qr[NV];
        for (int v = 0; v < NV; ++v) { ql[v] = QL[v * N2 + b]; qr[v] = QR[v * N2 + b]; }
        double sl = euler_speed(g, ql, d), sr = euler_speed(g, qr, d);
        if (sl > smax) { smax = sl; *bstar = b; *side = 0; }
        if (sr > smax) { smax = sr; *bstar = b; *side = 1; }
    }
    return smax;
}

/* Predictor with K tangent directions: the forward results (ustar, traces)
 * and their directional derivatives (dus, dtr: [K][...] of the same layout)
 * along du ([K][5][nc][N^3]). */
static void predictor_tlm(const orc_mesh *m, double g, int npic, double dt, const double *u, int K,
                          const double *du, double *ustar, double *traces, double *dus, double *dtr)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    long usz = (long)NV * nc * N3, tsz = (long)6 * 2 * NV * nc * N2;
    double xi[MAXN], w[MAXN], D[MAXN * MAXN], L[MAXN], R[MAXN], Kinv[MAXN * MAXN], Kw[MAXN * MAXN];
    orc_basis(N, xi, w, D, L, R, Kinv, Kw);
    int K1 = K + 1; /* slot 0: the forward state, slots 1..K: the tangents */
#pragma omp parallel
    {
        double *q = (double *)malloc(sizeof(double) * K1 * N * NV * N3);      /* [k][l][v][a] */
        double *qn = (double *)malloc(sizeof(double) * K1 * N * NV * N3);
        double *F = (double *)malloc(sizeof(double) * K1 * N * 3 * NV * N3);  /* [k][j][d][v][a] */
        double *G = (double *)malloc(sizeof(double) * N * NV * N3);
        double *uc = (double *)malloc(sizeof(double) * K1 * NV * N3);
        double *qbar = (double *)malloc(sizeof(double) * NV * N3);
        double *Fbar = (double *)malloc(sizeof(double) * 3 * NV * N3);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            double dx[3];
            cell_dx(m, c, dx);
            for (int k = 0; k < K1; ++k)
                for (int v = 0; v < NV; ++v)
                    for (int a = 0; a < N3; ++a)
                        uc[((long)k * NV + v) * N3 + a] =
                            k == 0 ? u[((long)v * nc + c) * N3 + a] : du[(k - 1) * usz + ((long)v * nc + c) * N3 + a];
            for (int k = 0; k < K1; ++k)
                for (int l = 0; l < N; ++l)
                    for (int v = 0; v < NV; ++v)
                        for (int a = 0; a < N3; ++a)
                            q[(((long)k * N + l) * NV + v) * N3 + a] = uc[((long)k * NV + v) * N3 + a];
            for (int it = 0; it <= npic; ++it) {
                /* fluxes of the iterate and their derivatives */
                for (int j = 0; j < N; ++j)
                    for (int a = 0; a < N3; ++a) {
                        double qq[NV], f[NV];
                        for (int v = 0; v < NV; ++v) qq[v] = q[((long)j * NV + v) * N3 + a];
                        for (int d = 0; d < 3; ++d) {
                            euler_flux(g, qq, d, f);
                            for (int v = 0; v < NV; ++v) F[((long)(j * 3 + d) * NV + v) * N3 + a] = f[v];
                            for (int k = 1; k < K1; ++k) {
                                double dq[NV], df[NV];
                                for (int v = 0; v < NV; ++v) dq[v] = q[(((long)k * N + j) * NV + v) * N3 + a];
                                euler_flux_tan(g, qq, dq, d, df);
                                for (int v = 0; v < NV; ++v)
                                    F[(((long)k * N + j) * 3 + d) * NV * N3 + (long)v * N3 + a] = df[v];
                            }
                        }
                    }
                if (it == npic) break;
                /* the iteration is linear in (u, F): the same operators act on
                 * the forward data and on every tangent */
                for (int k = 0; k < K1; ++k) {
                    const double *Fk = F + (long)k * N * 3 * NV * N3;
                    for (int j = 0; j < N; ++j)
                        for (int v = 0; v < NV; ++v)
                            for (int a = 0; a < N3; ++a) {
                                int aa[3] = { a % N, (a / N) % N, a / N2 };
                                double s = 0.0;
                                for (int d = 0; d < 3; ++d) {
                                    double sd = 0.0;
                                    for (int e = 0; e < N; ++e)
                                        sd += D[aa[d] * N + e] * Fk[((j * 3 + d) * NV + v) * N3 + node_with(N, a, d, e)];
                                    s += (dt / dx[d]) * sd;
                                }
                                G[(j * NV + v) * N3 + a] = s;
                            }
                    for (int l = 0; l < N; ++l)
                        for (int v = 0; v < NV; ++v)
                            for (int a = 0; a < N3; ++a) {
                                double s = 0.0;
                                for (int j = 0; j < N; ++j) s += Kinv[l * N + j] * w[j] * G[(j * NV + v) * N3 + a];
                                qn[(((long)k * N + l) * NV + v) * N3 + a] = uc[((long)k * NV + v) * N3 + a] - s;
                            }
                }
                double *t = q; q = qn; qn = t;
            }
            /* time averages, volume term and face projections (linear in q, F) */
            for (int k = 0; k < K1; ++k) {
                const double *qk = q + (long)k * N * NV * N3;
                const double *Fk = F + (long)k * N * 3 * NV * N3;
                for (int v = 0; v < NV; ++v)
                    for (int a = 0; a < N3; ++a) {
                        double s = 0.0;
                        for (int j = 0; j < N; ++j) s += w[j] * qk[(j * NV + v) * N3 + a];
                        qbar[v * N3 + a] = s;
                        for (int d = 0; d < 3; ++d) {
                            double sf = 0.0;
                            for (int j = 0; j < N; ++j) sf += w[j] * Fk[((j * 3 + d) * NV + v) * N3 + a];
                            Fbar[(d * NV + v) * N3 + a] = sf;
                        }
                    }
                double *uo = k == 0 ? ustar : dus + (k - 1) * usz;
                double *to = k == 0 ? traces : dtr + (k - 1) * tsz;
                for (int v = 0; v < NV; ++v)
                    for (int a = 0; a < N3; ++a) {
                        int aa[3] = { a % N, (a / N) % N, a / N2 };
                        double s = 0.0;
                        for (int d = 0; d < 3; ++d) {
                            double sd = 0.0;
                            for (int e = 0; e < N; ++e)
                                sd += Kw[aa[d] * N + e] * Fbar[(d * NV + v) * N3 + node_with(N, a, d, e)];
                            s += (dt / dx[d]) * sd / w[aa[d]];
                        }
                        uo[((long)v * nc + c) * N3 + a] = uc[((long)k * NV + v) * N3 + a] + s;
                    }
                for (int s = 0; s < 6; ++s) {
                    int d = s / 2;
                    const double *E = (s % 2) ? R : L;
                    for (int v = 0; v < NV; ++v)
                        for (int b = 0; b < N2; ++b) {
                            double sq = 0.0, sf = 0.0;
                            for (int e = 0; e < N; ++e) {
                                int a = node_from_face(N, d, e, b);
                                sq += E[e] * qbar[v * N3 + a];
                                sf += E[e] * Fbar[(d * NV + v) * N3 + a];
                            }
                            to[(((long)(s * 2 + 0) * NV + v) * nc + c) * N2 + b] = sq;
                            to[(((long)(s * 2 + 1) * NV + v) * nc + c) * N2 + b] = sf;
                        }
                }
            }
        }
        free(q); free(qn); free(F); free(G); free(uc); free(qbar); free(Fbar);
    }
}

/* Riemann phase with K tangents: fside and dfs ([K] x fside layout) from the
 * traces and their tangents dtr.  Returns 1 if a node is unphysical. */
static int riemann_tlm(const orc_mesh *m, double g, const double *traces, int K, const double *dtr,
                       double *fside, double *dfs)
{
    int N = m->N, N2 = N * N;
    long nc = m->nc;
    long tsz = (long)6 * 2 * NV * nc * N2, fsz = (long)6 * NV * nc * N2;
    int bad = orc_riemann(m, g, traces, fside);
#pragma omp parallel
    {
        double *QL = (double *)malloc(sizeof(double) * NV * N2 * 9);
        double *QR = QL + NV * N2, *dQL = QR + NV * N2, *dFL = dQL + NV * N2, *dQR = dFL + NV * N2;
        double *dFR = dQR + NV * N2, *tmp = dFR + NV * N2, *Fs = tmp + NV * N2, *Qtmp = Fs + NV * N2;
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            for (int s = 0; s < 6; ++s) {
                int d = s / 2, plus = s % 2;
                int kind = m->kind[6 * c + s];
                long o = m->nbr[6 * c + s];
                if (kind == SIDE_COARSE) continue;
                int so = 2 * d + (1 - plus);
                int r = 1, s1 = 0, s2 = 0;
                if (kind == SIDE_FINE) {
                    int t1, t2;
                    tangential(d, &t1, &t2);
                    r = (int)ipow3(m->lev[c] - m->lev[o]);
                    s1 = sub_position(m, c, o, t1);
                    s2 = sub_position(m, c, o, t2);
                }
                /* forward states of the face: this cell's trace and the
                 * neighbour's (interpolated to the child face if coarser) */
                double *Qc = plus ? QL : QR, *Qo = plus ? QR : QL;
                get_trace(m, traces, c, s, 0, Qc);
                if (kind == SIDE_CONFORMING) {
                    get_trace(m, traces, o, so, 0, Qo);
                } else {
                    get_trace(m, traces, o, so, 0, Qtmp);
                    prolong_face(N, r, s1, s2, Qtmp, Qo);
                }
                int bs, side;
                double smax = rusanov_speed(g, d, N2, QL, QR, &bs, &side);
                for (int k = 0; k < K; ++k) {
                    const double *dt_k = dtr + k * tsz;
                    double *dQc = plus ? dQL : dQR, *dFc = plus ? dFL : dFR;
                    double *dQo = plus ? dQR : dQL, *dFo = plus ? dFR : dFL;
                    get_trace(m, dt_k, c, s, 0, dQc);
                    get_trace(m, dt_k, c, s, 1, dFc);
                    if (kind == SIDE_CONFORMING) {
                        get_trace(m, dt_k, o, so, 0, dQo);
                        get_trace(m, dt_k, o, so, 1, dFo);
                    } else {
                        get_trace(m, dt_k, o, so, 0, tmp);
                        prolong_face(N, r, s1, s2, tmp, dQo);
                        get_trace(m, dt_k, o, so, 1, tmp);
                        prolong_face(N, r, s1, s2, tmp, dFo);
                    }
                    double ds = 0.0;
                    if (bs >= 0) {
                        double q[NV], dq[NV];
                        const double *Qa = side ? QR : QL, *dQa = side ? dQR : dQL;
                        for (int v = 0; v < NV; ++v) { q[v] = Qa[v * N2 + bs]; dq[v] = dQa[v * N2 + bs]; }
                        ds = euler_speed_tan(g, q, dq, d);
                    }
                    for (int v = 0; v < NV; ++v)
                        for (int b = 0; b < N2; ++b)
                            Fs[v * N2 + b] = 0.5 * (dFL[v * N2 + b] + dFR[v * N2 + b])
                                             - 0.5 * ds * (QR[v * N2 + b] - QL[v * N2 + b])
                                             - 0.5 * smax * (dQR[v * N2 + b] - dQL[v * N2 + b]);
                    put_side(m, dfs + k * fsz, c, s, Fs);
                }
            }
        }
        free(QL);
    }
    /* restriction of the tangents into the coarse sides (linear) */
    for (int k = 0; k < K; ++k) {
        double *dk = dfs + k * fsz;
        for (long c = 0; c < nc; ++c)
            for (int s = 0; s < 6; ++s)
                if (m->kind[6 * c + s] == SIDE_COARSE)
                    for (int v = 0; v < NV; ++v)
                        for (int b = 0; b < N2; ++b) dk[((long)(s * NV + v) * nc + c) * N2 + b] = 0.0;
        for (long f = 0; f < nc; ++f)
            for (int s = 0; s < 6; ++s) {
                if (m->kind[6 * f + s] != SIDE_FINE) continue;
                int d = s / 2, plus = s % 2;
                long cc = m->nbr[6 * f + s];
                int sc = 2 * d + (1 - plus);
                int t1, t2;
                tangential(d, &t1, &t2);
                int r = (int)ipow3(m->lev[f] - m->lev[cc]);
                int s1 = sub_position(m, f, cc, t1), s2 = sub_position(m, f, cc, t2);
                double P[MAXN * MAXN], R1[MAXN * MAXN], R2[MAXN * MAXN];
                orc_transfer(N, r, s1, P, R1);
                orc_transfer(N, r, s2, P, R2);
                for (int v = 0; v < NV; ++v)
                    for (int k2 = 0; k2 < N; ++k2)
                        for (int k1 = 0; k1 < N; ++k1) {
                            double acc = 0.0;
                            for (int e2 = 0; e2 < N; ++e2)
                                for (int e1 = 0; e1 < N; ++e1)
                                    acc += R1[k1 * N + e1] * R2[k2 * N + e2] *
                                           dk[((long)(s * NV + v) * nc + f) * N2 + e1 + N * e2];
                            dk[((long)(sc * NV + v) * nc + cc) * N2 + k1 + N * k2] += acc;
                        }
            }
    }
    return bad;
}

/* One step at the fixed dt with K tangent directions: u <- u^{n+1} and
 * du[k] <- (d u^{n+1} / d u^n) du[k] (du is [K][5][nc][N^3]).  Returns 0,
 * 1 if an unphysical state was met, 2 on allocation failure. */
int orc_step_tlm(const orc_mesh *m, double g, int npic, double dt, double *u, int K, double *du)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    long usz = (long)NV * nc * N3, tsz = (long)6 * 2 * NV * nc * N2, fsz = (long)6 * NV * nc * N2;
    double *us = (double *)malloc(sizeof(double) * usz);
    double *tr = (double *)malloc(sizeof(double) * tsz);
    double *fs = (double *)malloc(sizeof(double) * fsz);
    double *dus = (double *)malloc(sizeof(double) * usz * (K > 0 ? K : 1));
    double *dtr = (double *)malloc(sizeof(double) * tsz * (K > 0 ? K : 1));
    double *dfs = (double *)malloc(sizeof(double) * fsz * (K > 0 ? K : 1));
    int rc = 0;
    if (!us || !tr || !fs || !dus || !dtr || !dfs) {
        rc = 2;
    } else {
        predictor_tlm(m, g, npic, dt, u, K, du, us, tr, dus, dtr);
        if (riemann_tlm(m, g, tr, K, dtr, fs, dfs)) {
            rc = 1;
        } else {
            /* the corrector is linear in (ustar, fside) */
            orc_corrector(m, dt, us, fs, u);
            for (int k = 0; k < K; ++k) orc_corrector(m, dt, dus + k * usz, dfs + k * fsz, du + k * usz);
        }
    }
    free(us); free(tr); free(fs); free(dus); free(dtr); free(dfs);
    return rc;
}

/* Adjoint of one step at the fixed dt: ubar_n = (d u^{n+1} / d u^n)^T
 * ubar_np1 at the state u (unchanged).  The phases are transposed in reverse
 * order: corrector, restriction, Rusanov (with the virtual-cell
 * interpolation), predictor (face projections, volume term, time averages,
 * then the Picard iterations backwards with the forward iterates
 * recomputed per cell).  Returns 0, 1 if an unphysical state was met, 2 on
 * allocation failure. */
int orc_step_adj(const orc_mesh *m, double g, int npic, double dt, const double *u, const double *ubar_np1,
                 double *ubar_n)
{
    int N = m->N, N2 = N * N, N3 = N2 * N;
    long nc = m->nc;
    long usz = (long)NV * nc * N3, tsz = (long)6 * 2 * NV * nc * N2, fsz = (long)6 * NV * nc * N2;
    double xi[MAXN], w[MAXN], D[MAXN * MAXN], L[MAXN], R[MAXN], Kinv[MAXN * MAXN], Kw[MAXN * MAXN];
    orc_basis(N, xi, w, D, L, R, Kinv, Kw);
    double *us = (double *)malloc(sizeof(double) * usz);
    double *tr = (double *)malloc(sizeof(double) * tsz);
    double *trb = (double *)calloc(tsz, sizeof(double));
    double *fsb = (double *)calloc(fsz, sizeof(double));
    if (!us || !tr || !trb || !fsb) { free(us); free(tr); free(trb); free(fsb); return 2; }
    orc_predictor(m, g, npic, dt, u, us, tr);

    /* corrector: u^{n+1} = ustar - sum_d (dt/dx_d)(1/w)(R F*_{d+} - L F*_{d-}) */
    for (long c = 0; c < nc; ++c) {
        double dx[3];
        cell_dx(m, c, dx);
        for (int v = 0; v < NV; ++v)
            for (int a = 0; a < N3; ++a) {
                int aa[3] = { a % N, (a / N) % N, a / N2 };
                double y = ubar_np1[((long)v * nc + c) * N3 + a];
                for (int d = 0; d < 3; ++d) {
                    int b = face_index(N, a, d);
                    double k = (dt / dx[d]) / w[aa[d]];
                    fsb[((long)((2 * d + 1) * NV + v) * nc + c) * N2 + b] -= k * R[aa[d]] * y;
                    fsb[((long)((2 * d) * NV + v) * nc + c) * N2 + b] += k * L[aa[d]] * y;
                }
            }
    }
    /* restriction: coarse side = sum over child faces of (R1 x R2) fine side */
    for (long f = 0; f < nc; ++f)
        for (int s = 0; s < 6; ++s) {
            if (m->kind[6 * f + s] != SIDE_FINE) continue;
            int d = s / 2, plus = s % 2;
            long cc = m->nbr[6 * f + s];
            int sc = 2 * d + (1 - plus);
            int t1, t2;
            tangential(d, &t1, &t2);
            int r = (int)ipow3(m->lev[f] - m->lev[cc]);
            int s1 = sub_position(m, f, cc, t1), s2 = sub_position(m, f, cc, t2);
            double P[MAXN * MAXN], R1[MAXN * MAXN], R2[MAXN * MAXN];
            orc_transfer(N, r, s1, P, R1);
            orc_transfer(N, r, s2, P, R2);
            for (int v = 0; v < NV; ++v)
                for (int k2 = 0; k2 < N; ++k2)
                    for (int k1 = 0; k1 < N; ++k1) {
                        double y = fsb[((long)(sc * NV + v) * nc + cc) * N2 + k1 + N * k2];
                        for (int e2 = 0; e2 < N; ++e2)
                            for (int e1 = 0; e1 < N; ++e1)
                                fsb[((long)(s * NV + v) * nc + f) * N2 + e1 + N * e2] +=
                                    R1[k1 * N + e1] * R2[k2 * N + e2] * y;
                    }
        }
    /* Rusanov per (cell, non-coarse side); the bars go to both traces (through
     * the transposed interpolation on hanging faces) */
    int bad = 0;
    {
        double *QL = (double *)malloc(sizeof(double) * NV * N2 * 8);
        double *QR = QL + NV * N2, *bQL = QR + NV * N2, *bFL = bQL + NV * N2, *bQR = bFL + NV * N2;
        double *bFR = bQR + NV * N2, *Qtmp = bFR + NV * N2;
        for (long c = 0; c < nc; ++c)
            for (int s = 0; s < 6; ++s) {
                int d = s / 2, plus = s % 2;
                int kind = m->kind[6 * c + s];
                long o = m->nbr[6 * c + s];
                if (kind == SIDE_COARSE) continue;
                int so = 2 * d + (1 - plus);
                int r = 1, s1 = 0, s2 = 0;
                if (kind == SIDE_FINE) {
                    int t1, t2;
                    tangential(d, &t1, &t2);
                    r = (int)ipow3(m->lev[c] - m->lev[o]);
                    s1 = sub_position(m, c, o, t1);
                    s2 = sub_position(m, c, o, t2);
                }
                double *Qc = plus ? QL : QR, *Qo = plus ? QR : QL;
                get_trace(m, tr, c, s, 0, Qc);
                if (kind == SIDE_CONFORMING) {
                    get_trace(m, tr, o, so, 0, Qo);
                } else {
                    get_trace(m, tr, o, so, 0, Qtmp);
                    prolong_face(N, r, s1, s2, Qtmp, Qo);
                }
                for (int b = 0; b < N2; ++b) {
                    double ql[NV], qr[NV];
                    for (int v = 0; v < NV; ++v) { ql[v] = QL[v * N2 + b]; qr[v] = QR[v * N2 + b]; }
                    if (unphysical(g, ql) || unphysical(g, qr)) bad = 1;
                }
                int bs, side;
                double smax = rusanov_speed(g, d, N2, QL, QR, &bs, &side);
                double sbar = 0.0;
                for (int v = 0; v < NV; ++v)
                    for (int b = 0; b < N2; ++b) {
                        double y = fsb[((long)(s * NV + v) * nc + c) * N2 + b];
                        bFL[v * N2 + b] = 0.5 * y;
                        bFR[v * N2 + b] = 0.5 * y;
                        bQL[v * N2 + b] = 0.5 * smax * y;
                        bQR[v * N2 + b] = -0.5 * smax * y;
                        sbar += -0.5 * (QR[v * N2 + b] - QL[v * N2 + b]) * y;
                    }
                if (bs >= 0) {
                    const double *Qa = side ? QR : QL;
                    double *bQa = side ? bQR : bQL;
                    double q[NV];
                    for (int v = 0; v < NV; ++v) q[v] = Qa[v * N2 + bs];
                    for (int kk = 0; kk < NV; ++kk) {
                        double e[NV] = { 0, 0, 0, 0, 0 };
                        e[kk] = 1.0;
                        bQa[kk * N2 + bs] += sbar * euler_speed_tan(g, q, e, d);
                    }
                }
                double *bQc = plus ? bQL : bQR, *bFc = plus ? bFL : bFR;
                double *bQo = plus ? bQR : bQL, *bFo = plus ? bFR : bFL;
                for (int v = 0; v < NV; ++v)
                    for (int b = 0; b < N2; ++b) {
                        trb[(((long)(s * 2 + 0) * NV + v) * nc + c) * N2 + b] += bQc[v * N2 + b];
                        trb[(((long)(s * 2 + 1) * NV + v) * nc + c) * N2 + b] += bFc[v * N2 + b];
                    }
                if (kind == SIDE_CONFORMING) {
                    for (int v = 0; v < NV; ++v)
                        for (int b = 0; b < N2; ++b) {
                            trb[(((long)(so * 2 + 0) * NV + v) * nc + o) * N2 + b] += bQo[v * N2 + b];
                            trb[(((long)(so * 2 + 1) * NV + v) * nc + o) * N2 + b] += bFo[v * N2 + b];
                        }
                } else {
                    /* fine[k1 + N k2] = sum_e P1[k1][e1] P2[k2][e2] coarse[e1 + N e2] */
                    double P1[MAXN * MAXN], P2[MAXN * MAXN], Rm[MAXN * MAXN];
                    orc_transfer(N, r, s1, P1, Rm);
                    orc_transfer(N, r, s2, P2, Rm);
                    for (int arr = 0; arr < 2; ++arr) {
                        const double *bo = arr ? bFo : bQo;
                        for (int v = 0; v < NV; ++v)
                            for (int k2 = 0; k2 < N; ++k2)
                                for (int k1 = 0; k1 < N; ++k1) {
                                    double y = bo[v * N2 + k1 + N * k2];
                                    for (int e2 = 0; e2 < N; ++e2)
                                        for (int e1 = 0; e1 < N; ++e1)
                                            trb[(((long)(so * 2 + arr) * NV + v) * nc + o) * N2 + e1 + N * e2] +=
                                                P1[k1 * N + e1] * P2[k2 * N + e2] * y;
                                }
                    }
                }
            }
        free(QL);
    }
    /* predictor, cell by cell: ustar = u + volume term, traces from the time
     * averages, Picard iterations backwards */
    const double *usb = ubar_np1; /* ustar enters the corrector with weight 1 */
#pragma omp parallel
    {
        double *qs = (double *)malloc(sizeof(double) * (npic + 1) * N * NV * N3); /* [it][j][v][a] */
        double *Fs = (double *)malloc(sizeof(double) * (npic + 1) * N * 3 * NV * N3);
        double *qb = (double *)malloc(sizeof(double) * N * NV * N3);
        double *Fb = (double *)malloc(sizeof(double) * N * 3 * NV * N3);
        double *Gb = (double *)malloc(sizeof(double) * N * NV * N3);
        double *qbarb = (double *)malloc(sizeof(double) * NV * N3);
        double *Fbarb = (double *)malloc(sizeof(double) * 3 * NV * N3);
        double *ub = (double *)malloc(sizeof(double) * NV * N3);
#pragma omp for schedule(static)
        for (long c = 0; c < nc; ++c) {
            double dx[3];
            cell_dx(m, c, dx);
            /* forward iterates q^(0..npic) and their fluxes */
            for (int j = 0; j < N; ++j)
                for (int v = 0; v < NV; ++v)
                    for (int a = 0; a < N3; ++a) qs[(j * NV + v) * N3 + a] = u[((long)v * nc + c) * N3 + a];
            for (int it = 0; it <= npic; ++it) {
                double *q = qs + (long)it * N * NV * N3;
                double *F = Fs + (long)it * N * 3 * NV * N3;
                for (int j = 0; j < N; ++j)
                    for (int a = 0; a < N3; ++a) {
                        double qq[NV], f[NV];
                        for (int v = 0; v < NV; ++v) qq[v] = q[(j * NV + v) * N3 + a];
                        for (int d = 0; d < 3; ++d) {
                            euler_flux(g, qq, d, f);
                            for (int v = 0; v < NV; ++v) F[((j * 3 + d) * NV + v) * N3 + a] = f[v];
                        }
                    }
                if (it == npic) break;
                double *qn = qs + (long)(it + 1) * N * NV * N3;
                for (int l = 0; l < N; ++l)
                    for (int v = 0; v < NV; ++v)
                        for (int a = 0; a < N3; ++a) {
                            int aa[3] = { a % N, (a / N) % N, a / N2 };
                            double s = 0.0;
                            for (int j = 0; j < N; ++j) {
                                double Gj = 0.0;
                                for (int d = 0; d < 3; ++d) {
                                    double sd = 0.0;
                                    for (int e = 0; e < N; ++e)
                                        sd += D[aa[d] * N + e] * F[((j * 3 + d) * NV + v) * N3 + node_with(N, a, d, e)];
                                    Gj += (dt / dx[d]) * sd;
                                }
                                s += Kinv[l * N + j] * w[j] * Gj;
                            }
                            qn[(l * NV + v) * N3 + a] = u[((long)v * nc + c) * N3 + a] - s;
                        }
            }
            /* bars of the time averages from ustar and the traces */
            for (int i = 0; i < NV * N3; ++i) qbarb[i] = 0.0;
            for (int i = 0; i < 3 * NV * N3; ++i) Fbarb[i] = 0.0;
            for (int v = 0; v < NV; ++v)
                for (int a = 0; a < N3; ++a) {
                    int aa[3] = { a % N, (a / N) % N, a / N2 };
                    double y = usb[((long)v * nc + c) * N3 + a];
                    ub[v * N3 + a] = y;
                    for (int d = 0; d < 3; ++d)
                        for (int e = 0; e < N; ++e)
                            Fbarb[(d * NV + v) * N3 + node_with(N, a, d, e)] +=
                                (dt / dx[d]) / w[aa[d]] * Kw[aa[d] * N + e] * y;
                }
            for (int s = 0; s < 6; ++s) {
                int d = s / 2;
                const double *E = (s % 2) ? R : L;
                for (int v = 0; v < NV; ++v)
                    for (int b = 0; b < N2; ++b) {
                        double yq = trb[(((long)(s * 2 + 0) * NV + v) * nc + c) * N2 + b];
                        double yf = trb[(((long)(s * 2 + 1) * NV + v) * nc + c) * N2 + b];
                        for (int e = 0; e < N; ++e) {
                            int a = node_from_face(N, d, e, b);
                            qbarb[v * N3 + a] += E[e] * yq;
                            Fbarb[(d * NV + v) * N3 + a] += E[e] * yf;
                        }
                    }
            }
            /* qbar = sum_j w_j q_j, Fbar_d = sum_j w_j f_d(q_j) of the final iterate */
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < NV * N3; ++i) qb[j * NV * N3 + i] = w[j] * qbarb[i];
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < 3 * NV * N3; ++i) Fb[(long)j * 3 * NV * N3 + i] = w[j] * Fbarb[i];
            for (int it = npic; it >= 0; --it) {
                /* q^(it) -> F^(it) */
                const double *q = qs + (long)it * N * NV * N3;
                for (int j = 0; j < N; ++j)
                    for (int a = 0; a < N3; ++a) {
                        double qq[NV], y[NV], o[NV];
                        for (int v = 0; v < NV; ++v) qq[v] = q[(j * NV + v) * N3 + a];
                        for (int d = 0; d < 3; ++d) {
                            for (int v = 0; v < NV; ++v) y[v] = Fb[((j * 3 + d) * NV + v) * N3 + a];
                            euler_flux_vjp(g, qq, d, y, o);
                            for (int v = 0; v < NV; ++v) qb[(j * NV + v) * N3 + a] += o[v];
                        }
                    }
                if (it == 0) {
                    /* q^(0)_j = u for every time node */
                    for (int j = 0; j < N; ++j)
                        for (int i = 0; i < NV * N3; ++i) ub[i] += qb[j * NV * N3 + i];
                    break;
                }
                /* q^(it)_l = u - sum_j Kinv[l][j] w_j G_j,
                 * G_j = sum_d (dt/dx_d) D_d F^(it-1)[j][d] */
                for (int l = 0; l < N; ++l)
                    for (int i = 0; i < NV * N3; ++i) ub[i] += qb[l * NV * N3 + i];
                for (int j = 0; j < N; ++j)
                    for (int i = 0; i < NV * N3; ++i) {
                        double s = 0.0;
                        for (int l = 0; l < N; ++l) s += Kinv[l * N + j] * qb[l * NV * N3 + i];
                        Gb[j * NV * N3 + i] = -w[j] * s;
                    }
                for (int i = 0; i < N * 3 * NV * N3; ++i) Fb[i] = 0.0;
                for (int j = 0; j < N; ++j)
                    for (int v = 0; v < NV; ++v)
                        for (int a = 0; a < N3; ++a) {
                            int aa[3] = { a % N, (a / N) % N, a / N2 };
                            double y = Gb[(j * NV + v) * N3 + a];
                            for (int d = 0; d < 3; ++d)
                                for (int e = 0; e < N; ++e)
                                    Fb[((j * 3 + d) * NV + v) * N3 + node_with(N, a, d, e)] +=
                                        (dt / dx[d]) * D[aa[d] * N + e] * y;
                        }
                for (int i = 0; i < N * NV * N3; ++i) qb[i] = 0.0;
            }
            for (int v = 0; v < NV; ++v)
                for (int a = 0; a < N3; ++a) ubar_n[((long)v * nc + c) * N3 + a] = ub[v * N3 + a];
        }
        free(qs); free(Fs); free(qb); free(Fb); free(Gb); free(qbarb); free(Fbarb); free(ub);
    }
    free(us); free(tr); free(trb); free(fsb);
    return bad;
}

/* Transpose of orc_sample: ubar[rho][c_s][a] += wbar_s phi_a(x_s) for every
 * point in order (base-level meshes only).  The sample is linear in u, so
 * this is its adjoint. */
int orc_sample_adj(const orc_mesh *m, const double *pts, long n, const double *wbar, double *ubar)
{
    if (m->max_level != 0) return 1;
    int N = m->N, N3 = N * N * N;
    double xi[MAXN], w[MAXN];
    orc_gauss_legendre(N, xi, w);
    for (long s = 0; s < n; ++s) {
        int ijk[3];
        double phi[3][MAXN];
        for (int d = 0; d < 3; ++d) {
            double y = (pts[3 * s + d] - m->lo[d]) / (m->hi[d] - m->lo[d]) * m->n[d];
            int i = (int)floor(y);
            if (i < 0) i = 0;
            if (i >= m->n[d]) i = m->n[d] - 1;
            ijk[d] = i;
            for (int e = 0; e < N; ++e) phi[d][e] = lagrange(N, xi, e, y - i);
        }
        long c = ijk[0] + (long)m->n[0] * (ijk[1] + (long)m->n[1] * ijk[2]);
        for (int a2 = 0; a2 < N; ++a2)
            for (int a1 = 0; a1 < N; ++a1)
                for (int a0 = 0; a0 < N; ++a0)
                    ubar[c * N3 + a0 + N * a1 + N * N * a2] += wbar[s] * phi[0][a0] * phi[1][a1] * phi[2][a2];
    }
    return 0;
}
