// Host computation of the 1-D ADER-DG operators on Gauss-Legendre nodes.
//
// Nodes and weights: Golub-Welsch (eigen-decomposition of the symmetric
// Jacobi matrix of the Legendre recurrence, cyclic Jacobi rotations).
// Lagrange values and derivatives: barycentric formulas.
// These are the operators of the paper's Sec. 2.1 (Lagrange polynomials over
// Gauss-Legendre points, the same order in time) and Sec. 2.3 (interpolation
// to virtual cells and its transpose for the restriction).
#include <cmath>
#include <cstring>

#include "adg_internal.h"

namespace adg {
namespace {

// Symmetric eigen-decomposition by cyclic Jacobi rotations; A is n x n
// (row-major), overwritten; V receives eigenvectors as columns.
void jacobi_eig(int n, double *A, double *V)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-34) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {  // columns p, q
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // rows p, q
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
}

// Legendre P_n and derivative (used for one Newton polish of each node).
void legendre(int n, double x, double &P, double &dP)
{
    double a = 1.0, b = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    P = b;
    dP = n * (a - x * b) / (1.0 - x * x);
}

// Barycentric Lagrange evaluation of all phi_e at x.
void lagrange_all(int N, const double *xi, const double *lam, double x, double *out)
{
    for (int e = 0; e < N; ++e)
        if (std::fabs(x - xi[e]) < 1e-15) {
            for (int k = 0; k < N; ++k) out[k] = (k == e) ? 1.0 : 0.0;
            return;
        }
    double den = 0.0;
    for (int k = 0; k < N; ++k) den += lam[k] / (x - xi[k]);
    for (int e = 0; e < N; ++e) out[e] = lam[e] / (x - xi[e]) / den;
}

// Solve A X = B for X (n x n, row-major) by LU with partial pivoting.
bool lu_solve(int n, const double *A_in, const double *B_in, double *X)
{
    double A[NMAX * NMAX], B[NMAX * NMAX];
    std::memcpy(A, A_in, sizeof(double) * n * n);
    std::memcpy(B, B_in, sizeof(double) * n * n);
    int piv[NMAX];
    for (int i = 0; i < n; ++i) piv[i] = i;
    for (int k = 0; k < n; ++k) {
        int m = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[i * n + k]) > std::fabs(A[m * n + k])) m = i;
        if (A[m * n + k] == 0.0) return false;
        if (m != k) {
            for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[m * n + j]);
            std::swap(piv[k], piv[m]);
        }
        for (int i = k + 1; i < n; ++i) {
            A[i * n + k] /= A[k * n + k];
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= A[i * n + k] * A[k * n + j];
        }
    }
    for (int col = 0; col < n; ++col) {
        double y[NMAX];
        for (int i = 0; i < n; ++i) {
            double s = B[piv[i] * n + col];
            for (int j = 0; j < i; ++j) s -= A[i * n + j] * y[j];
            y[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * X[j * n + col];
            X[i * n + col] = s / A[i * n + i];
        }
    }
    return true;
}

void bary_weights(int N, const double *xi, double *lam)
{
    for (int e = 0; e < N; ++e) {
        double p = 1.0;
        for (int k = 0; k < N; ++k)
            if (k != e) p *= (xi[e] - xi[k]);
        lam[e] = 1.0 / p;
    }
}

}  // namespace

bool make_basis(int N, Basis &b)
{
    if (N < 1 || N > NMAX) return false;
    std::memset(&b, 0, sizeof(b));
    b.N = N;
    // Jacobi matrix of monic-normalised Legendre: off-diagonal k/sqrt(4k^2-1)
    double J[NMAX * NMAX] = {0}, V[NMAX * NMAX];
    for (int k = 1; k < N; ++k) {
        double beta = k / std::sqrt(4.0 * k * k - 1.0);
        J[(k - 1) * N + k] = beta;
        J[k * N + (k - 1)] = beta;
    }
    jacobi_eig(N, J, V);
    // sort eigenpairs ascending
    int idx[NMAX];
    for (int i = 0; i < N; ++i) idx[i] = i;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j)
            if (J[idx[j] * N + idx[j]] < J[idx[i] * N + idx[i]]) std::swap(idx[i], idx[j]);
    for (int i = 0; i < N; ++i) {
        double x = J[idx[i] * N + idx[i]];
        if (N > 1) {  // one Newton polish on P_N
            double P, dP;
            legendre(N, x, P, dP);
            x -= P / dP;
        }
        double v0 = V[0 * N + idx[i]];
        b.xi[i] = 0.5 * (x + 1.0);
        b.w[i] = v0 * v0;  // 2 v0^2 on [-1,1], halved on [0,1]
    }
    double lam[NMAX];
    bary_weights(N, b.xi, lam);
    // differentiation matrix (barycentric)
    for (int a = 0; a < N; ++a) {
        double diag = 0.0;
        for (int e = 0; e < N; ++e) {
            if (e == a) continue;
            double v = (lam[e] / lam[a]) / (b.xi[a] - b.xi[e]);
            b.D[a * N + e] = v;
            diag -= v;
        }
        b.D[a * N + a] = diag;
    }
    lagrange_all(N, b.xi, lam, 0.0, b.L);
    lagrange_all(N, b.xi, lam, 1.0, b.R);
    // K1[k][l] = R_k R_l - w_l D[l][k]; KW = K1^{-1} diag(w)
    double K1[NMAX * NMAX], Wd[NMAX * NMAX] = {0};
    for (int k = 0; k < N; ++k)
        for (int l = 0; l < N; ++l) K1[k * N + l] = b.R[k] * b.R[l] - b.w[l] * b.D[l * N + k];
    for (int j = 0; j < N; ++j) Wd[j * N + j] = b.w[j];
    if (!lu_solve(N, K1, Wd, b.KW)) return false;
    for (int a = 0; a < N; ++a)
        for (int e = 0; e < N; ++e) b.Kw[a * N + e] = b.w[e] * b.D[e * N + a];
    return true;
}

bool make_subcell(const Basis &b, DevSub &out)
{
    const int N = b.N, ns = 2 * N - 1;
    if (N < 1 || N > LIM_NMAX) return false;
    std::memset(&out, 0, sizeof(out));
    double lam[NMAX], row[NMAX];
    bary_weights(N, b.xi, lam);
    // subinterval averages by the N-point Gauss rule on each subinterval
    for (int s = 0; s < ns; ++s)
        for (int q = 0; q < N; ++q) {
            lagrange_all(N, b.xi, lam, (s + b.xi[q]) / ns, row);
            for (int k = 0; k < N; ++k) out.A[s * N + k] += b.w[q] * row[k];
        }
    // (A^T A)^{-1} by LU, then times A^T
    double G[NMAX * NMAX], I[NMAX * NMAX] = {0}, Gi[NMAX * NMAX];
    for (int i = 0; i < N; ++i) {
        I[i * N + i] = 1.0;
        for (int j = 0; j < N; ++j) {
            double acc = 0.0;
            for (int s = 0; s < ns; ++s) acc += out.A[s * N + i] * out.A[s * N + j];
            G[i * N + j] = acc;
        }
    }
    if (!lu_solve(N, G, I, Gi)) return false;
    for (int k = 0; k < N; ++k)
        for (int s = 0; s < ns; ++s) {
            double acc = 0.0;
            for (int j = 0; j < N; ++j) acc += Gi[k * N + j] * out.A[s * N + j];
            out.Ap[k * ns + s] = acc;
            out.Bf[k * ns + s] = out.A[s * N + k] / (ns * b.w[k]);
        }
    return true;
}

void make_transfer(const Basis &b, int r, int s, double *P, double *Rm)
{
    int N = b.N;
    double lam[NMAX];
    bary_weights(N, b.xi, lam);
    for (int k = 0; k < N; ++k) lagrange_all(N, b.xi, lam, (s + b.xi[k]) / r, &P[k * N]);
    for (int k = 0; k < N; ++k)
        for (int e = 0; e < N; ++e) Rm[k * N + e] = (b.w[e] / b.w[k]) * P[e * N + k] / r;
}

}  // namespace adg
