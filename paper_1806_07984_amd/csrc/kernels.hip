// HIP kernels of the ADER-DG step for gfx950 (MI355X).
//
// Data layouts are the ones documented in include/adg.h (structure of arrays:
// variable-major, then cell, then node), so that consecutive lanes touch
// consecutive doubles in every global load and store.
//
// Kernels (template parameters: real type T, N = p + 1):
//   k_predictor   C_STP by Picard iterations + time averages + volume term +
//                 face projections (paper Eq. 3-4, Sec. 2.1-2.2).  One lane per
//                 spatial node holds the whole time history of its node in
//                 registers; flux values are exchanged through LDS once per
//                 time node for the three derivative contractions.
//   k_riemann     Rusanov solve on conforming faces (Alg. 1, Sec. 2.4).
//   k_hang        virtual-cell face data (interpolation of the coarse cell's
//                 face projection) + Rusanov on hanging child faces (Sec. 2.3).
//   k_restrict    restriction of child face results into the coarse side, in
//                 a fixed order (no atomics).
//   k_corrector   C_Corr (Eq. 4), FP64 accumulation.
//   k_cfl_*       global time step size: block maxima then one final block.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "adg_internal.h"
#include "kernels.h"

namespace adg {

__constant__ DevBasis c_basis[NMAX + 1];

// Per-lane coefficient rows of the N = 4 FP32 predictor (one wavefront per
// cell, lane l = node a0 + 4 a1 + 16 a2), LANE4 floats per lane, in the order
// the rotations of the x (quad), y (row) and z (row group) sums visit them:
//   [0,4)   D[a0][(a0+e)&3]          [4,8)   D[a1][(a1-e)&3]
//   [8,12)  D[a2][(a2+k)&3]          [12,16) KW[a0][e]
//   [16,20) Kw[a0][(a0+e)&3]/w[a0]   [20,24) Kw[a1][(a1-e)&3]/w[a1]
//   [24,28) Kw[a2][(a2+k)&3]/w[a2]
//   [28,32) P(a0)[(a0+e)&3], [32,36) P(a1)[(a1-e)&3], [36,40) P(a2)[(a2+k)&3]
//           with P(t) = L for t = 0, R otherwise (only the face lanes store)
constexpr int LANE4 = 40;
__constant__ float c_lane4[64 * LANE4];
// row sums sum_l KW[j][l] of the N = 4 time solve (first Picard iteration)
__constant__ float c_kwsum4[4];
// lift weights of the N = 4 corrector per lane (node): R[a_d]/w[a_d] for
// d = 0, 1, 2, then L[a_d]/w[a_d]
__constant__ double c_corr4[64 * 6];

namespace {

template <typename T>
__device__ __forceinline__ T rcp(T x) { return T(1) / x; }

// 1/x in FP64 from the hardware estimate and one Newton step: within an ulp
// or so of the quotient, for about a third of the instructions of the IEEE
// division sequence
__device__ __forceinline__ double rcp_newton(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// Euler fluxes along the three axes of the state q (FAST: FP64 reciprocal of
// the density by rcp_newton, for the predictor's Picard iterations).
template <typename T, bool FAST = false>
__device__ __forceinline__ void euler_flux3(T gm1, const T q[NV], T f[3][NV])
{
    // velocities once; the momentum flux m_de = rho v_d v_e is symmetric
    T inv;
    if constexpr (FAST && std::is_same<T, double>::value)
        inv = rcp_newton(q[0]);
    else
        inv = rcp(q[0]);
    const T v0 = q[1] * inv, v1 = q[2] * inv, v2 = q[3] * inv;
    const T m00 = v0 * q[1], m11 = v1 * q[2], m22 = v2 * q[3];
    const T m01 = v0 * q[2], m02 = v0 * q[3], m12 = v1 * q[3];
    const T p = gm1 * (q[4] - T(0.5) * (m00 + m11 + m22));
    const T Ep = q[4] + p;
    f[0][0] = q[1]; f[0][1] = m00 + p; f[0][2] = m01; f[0][3] = m02; f[0][4] = v0 * Ep;
    f[1][0] = q[2]; f[1][1] = m01; f[1][2] = m11 + p; f[1][3] = m12; f[1][4] = v1 * Ep;
    f[2][0] = q[3]; f[2][1] = m02; f[2][2] = m12; f[2][3] = m22 + p; f[2][4] = v2 * Ep;
}

// |u_d| + c and a physical-state check.
template <typename T>
__device__ __forceinline__ T wave_speed(T gamma, T gm1, const T q[NV], int d, bool &bad)
{
    const T inv = rcp(q[0]);
    const T p = gm1 * (q[4] - T(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) * inv);
    bool ok = q[0] > T(0) && p > T(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) ok = ok && isfinite(q[v]);
    bad = !ok;
    return fabs(q[1 + d] * inv) + sqrt(gamma * p * inv);
}

// volume node index from (index e along axis d, face index b)
template <int N>
__device__ __forceinline__ int node_from_face(int d, int e, int b)
{
    const int b1 = b % N, b2 = b / N;
    if (d == 0) return e + N * b1 + N * N * b2;
    if (d == 1) return b1 + N * e + N * N * b2;
    return b1 + N * b2 + N * N * e;
}

constexpr int round64(int x) { return (x + 63) / 64 * 64; }

}  // namespace

// Default cells per block of the per-order predictor kernel, chosen so one
// block is close to a multiple of 64 lanes (the autotuner may pick others).
template <int N> struct PredCfg;
template <> struct PredCfg<1> { static constexpr int CPB = 64; };
template <> struct PredCfg<2> { static constexpr int CPB = 32; };
template <> struct PredCfg<3> { static constexpr int CPB = 9; };
template <> struct PredCfg<4> { static constexpr int CPB = 4; };
template <> struct PredCfg<5> { static constexpr int CPB = 2; };
template <> struct PredCfg<6> { static constexpr int CPB = 1; };
template <> struct PredCfg<7> { static constexpr int CPB = 1; };

// wavefront-per-cell FP32 predictor for N = 4 (defined below); KEEP_U holds
// the FP64 state in registers for u* = u + V instead of reading it again
template <bool KEEP_U = false>
__device__ __forceinline__ void pred4_wave(const double *__restrict__ u, double *__restrict__ ustar,
                                           float *__restrict__ traces, int64_t c, int64_t nc, int lev,
                                           const Geo &geo, double dt, double gamma, int npic);
// the LDS-free N = 4 FP32 kernels are always used (kept as a constant so the
// generic path stays compiled for the FP64 form and other orders)
constexpr bool g_pred4_mfma_dev = true;

// a scheduling fence: keeps the compiler from hoisting the loads of later
// work above it (bounds the live registers of long unrolled sequences)
#ifndef SCHED_SPLIT
#define SCHED_SPLIT() __builtin_amdgcn_sched_barrier(0)
#endif

// LDS of the generic predictor: NBUF buffers of 15 planes (3 axes x 5
// variables).  A plane holds one value per thread of the block (thread t =
// cell t / N^3 of the block, node t % N^3) and is padded to whole wavefronts,
// so every lane writes its slot without a branch.  A fibre read is a
// broadcast across the lanes that share the fibre (cheaper in LDS bandwidth
// than wide loads, which move all their bytes per lane).  With two buffers,
// consecutive flux exchanges alternate and need one barrier each.
constexpr int pred_plane(int N, int CPB) { return round64(CPB * N * N * N); }
constexpr int pred_nbuf(int N, int CPB, int real_bytes)
{
    return 2 * 15 * pred_plane(N, CPB) * real_bytes <= 65536 ? 2 : 1;
}
constexpr int pred_lds_elems(int N, int CPB, int real_bytes)
{
    return pred_nbuf(N, CPB, real_bytes) * 15 * pred_plane(N, CPB);
}

// Write planes (f[d][v] into plane d NV + v, or q[v] into plane v, at this
// thread's slot) of the next buffer, one barrier, and return that buffer.
// With a single buffer, a barrier first lets every lane finish reading the
// previous exchange.
template <typename T, int P, int NBUF, int ND>
__device__ __forceinline__ const T *pred_exchange(T *lds, int &buf, int tid, const T (&f)[ND][NV])
{
    T *w = lds + buf * (15 * P);
    if constexpr (NBUF == 1) __syncthreads();
    if (tid < P) {
#pragma unroll
        for (int d = 0; d < ND; ++d)
#pragma unroll
            for (int v = 0; v < NV; ++v) w[(d * NV + v) * P + tid] = f[d][v];
    }
    __syncthreads();
    if constexpr (NBUF == 2) buf ^= 1;
    return w;
}

// Euler fluxes in FP32: hardware reciprocal for 1/rho, and the symmetric
// momentum flux formed once
__device__ __forceinline__ void euler_flux3_fast(float gm1, const float q[NV], float f[3][NV])
{
    // velocities once; the momentum flux m_de = rho v_d v_e is symmetric
    const float inv = __builtin_amdgcn_rcpf(q[0]);
    const float v0 = q[1] * inv, v1 = q[2] * inv, v2 = q[3] * inv;
    const float m00 = v0 * q[1], m11 = v1 * q[2], m22 = v2 * q[3];
    const float m01 = v0 * q[2], m02 = v0 * q[3], m12 = v1 * q[3];
    // p = (gamma - 1) (E - rho |v|^2 / 2)
    const float p = fmaf(-0.5f * gm1, m00 + m11 + m22, gm1 * q[4]);
    const float Ep = q[4] + p;
    f[0][0] = q[1]; f[0][1] = m00 + p; f[0][2] = m01; f[0][3] = m02; f[0][4] = v0 * Ep;
    f[1][0] = q[2]; f[1][1] = m01; f[1][2] = m11 + p; f[1][3] = m12; f[1][4] = v1 * Ep;
    f[2][0] = q[3]; f[2][1] = m02; f[2][2] = m12; f[2][3] = m22 + p; f[2][4] = v2 * Ep;
}

template <typename T>
__device__ __forceinline__ void flux3(T gm1, const T q[NV], T f[3][NV])
{
    if constexpr (std::is_same<T, float>::value)
        euler_flux3_fast(gm1, q, f);
    else
        euler_flux3<T, true>(gm1, q, f);
}

// Predictor of CPB cells (list entries first .. first+CPB-1) by one block of
// at least pred_plane(N, CPB) threads; lds holds NBUF x 15 planes
// (pred_lds_elems(N, CPB, sizeof(T)) reals with the default NBUF).
template <typename T, int N, int CPB, bool STORE = false, int NBUF = pred_nbuf(N, CPB, int(sizeof(T)))>
__device__ __forceinline__ void predictor_body(T *__restrict__ lds, const double *__restrict__ u,
                                               double *__restrict__ ustar, T *__restrict__ traces,
                                               const int32_t *__restrict__ list, int64_t nlist, int64_t nc,
                                               const int8_t *__restrict__ level, const Geo &geo, double dt,
                                               double gamma, int npic, int64_t first,
                                               T *__restrict__ iters = nullptr)
{
    constexpr int N2 = N * N, N3 = N2 * N, NT = CPB * N3;
    constexpr int P = pred_plane(N, CPB);
    const DevBasis &B = c_basis[N];

    // opaque: in the persistent kernels nothing derived from the lane index is
    // hoisted out of the loop over work items to hold registers through it
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const bool lane_ok = tid < NT;
    // lanes past the block's cells read cell 0's values and store nothing
    const int cl = lane_ok ? tid / N3 : 0, a = lane_ok ? tid % N3 : 0;
    const int64_t idx = first + cl;
    const bool active = lane_ok && idx < nlist;
    const int64_t c = active ? (list ? int64_t(list[idx]) : idx) : 0;
    const int aa[3] = {a % N, (a / N) % N, a / N2};
    // first node of this lane's fibre along each axis (in the block's planes)
    const int fo[3] = {cl * N3 + a - aa[0], cl * N3 + a - N * aa[1], cl * N3 + a - N2 * aa[2]};

    const int lev = level ? level[c] : 0;
    const double cdd[3] = {dt * geo.inv_dx[lev][0], dt * geo.inv_dx[lev][1], dt * geo.inv_dx[lev][2]};
    const T gm1 = T(gamma - 1.0);

    double ud[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) ud[v] = active ? u[(int64_t(v) * nc + c) * N3 + a] : (v == 0 ? 1.0 : (v == 4 ? 2.5 : 0.0));
    T uu[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uu[v] = T(ud[v]);

    // derivative rows of this lane's node along each axis, scaled by dt/dx_d
    T Dc[3][N];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int e = 0; e < N; ++e) Dc[d][e] = T(cdd[d] * B.D[aa[d] * N + e]);

    T q[N][NV];
#pragma unroll
    for (int l = 0; l < N; ++l)
#pragma unroll
        for (int v = 0; v < NV; ++v) q[l][v] = uu[v];

    int buf = 0;
    // the N values of this lane's fibre along d in plane k of buffer w
    auto fibre = [&](const T *w, int k, int d, T out[N]) {
        const T *src = w + k * P + fo[d];
        const int st = d == 0 ? 1 : (d == 1 ? N : N2);
#pragma unroll
        for (int e = 0; e < N; ++e) out[e] = src[e * st];
    };

    // scaled divergence sum_d (dt/dx_d) D_d F_d(qn) at this lane's node
    auto divergence = [&](const T qn[NV], T G[NV]) {
        T f[3][NV];
        flux3(gm1, qn, f);
        const T *w = pred_exchange<T, P, NBUF>(lds, buf, tid, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T s = T(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                T fib[N];
                fibre(w, d * NV + v, d, fib);
#pragma unroll
                for (int e = 0; e < N; ++e) s += Dc[d][e] * fib[e];
            }
            // pinned here: otherwise the compiler sinks the contraction to
            // the time solve at the end of the Picard iteration and keeps
            // every fibre value of every time node live until then
            asm volatile("" : "+v"(s));
            G[v] = s;
        }
    };
    // iterate it+1, kept for the adjoint: [slot][l][v][cell][N^3]
    auto store_iterate = [&](int it) {
        if (STORE && active) {
#pragma unroll
            for (int l = 0; l < N; ++l)
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    iters[(((int64_t(it) * N + l) * NV + v) * nc + c) * N3 + a] = q[l][v];
        }
    };

    if (npic > 0) {
        // first iteration from q = u at every time node: one flux and one
        // divergence serve all time nodes, and the row sums of KW finish the
        // time solve
        T G[NV];
        divergence(uu, G);
#pragma unroll
        for (int l = 0; l < N; ++l)
#pragma unroll
            for (int v = 0; v < NV; ++v) q[l][v] = uu[v] - T(B.KWsum[l]) * G[v];
        store_iterate(0);
    }
    for (int it = 1; it < npic; ++it) {
        T acc[N][NV];
#pragma unroll
        for (int l = 0; l < N; ++l)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[l][v] = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T G[NV];
            divergence(q[j], G);
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int l = 0; l < N; ++l) acc[l][v] += T(B.KW[l * N + j]) * G[v];
        }
#pragma unroll
        for (int l = 0; l < N; ++l)
#pragma unroll
            for (int v = 0; v < NV; ++v) q[l][v] = uu[v] - acc[l][v];
        store_iterate(it);
    }

    // time averages of the state and of the fluxes of the final iterate
    T qb[NV], Fb[3][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        qb[v] = T(0);
        Fb[0][v] = Fb[1][v] = Fb[2][v] = T(0);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T f[3][NV];
        flux3(gm1, q[j], f);
        const T wj = T(B.w[j]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qb[v] += wj * q[j][v];
#pragma unroll
            for (int d = 0; d < 3; ++d) Fb[d][v] += wj * f[d][v];
        }
    }
    const T *wF = pred_exchange<T, P, NBUF>(lds, buf, tid, Fb);

    // volume term of the corrector: u* = u + sum_d (dt/dx_d)/w_{a_d} sum_e Kw[a_d][e] Fbar_d
    if (active) {
        T Kc[3][N];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int e = 0; e < N; ++e) Kc[d][e] = T(cdd[d] * B.winv[aa[d]] * B.Kw[aa[d] * N + e]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            T V = T(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                T fib[N];
                fibre(wF, d * NV + v, d, fib);
#pragma unroll
                for (int e = 0; e < N; ++e) V += Kc[d][e] * fib[e];
            }
            ustar[(int64_t(v) * nc + c) * N3 + a] = ud[v] + double(V);
            SCHED_SPLIT();
        }
    }

    // face projections: lane (cell, node a) takes face node b = a mod N^2 of
    // the (axis, variable) pairs k = a / N^2, a / N^2 + N, ... (k = d NV + v)
    // and projects the fibre through it onto both faces of the axis; the
    // normal flux (array 1) comes from the flux planes, the state (array 0)
    // from the state planes (plane v for every axis)
    T Lf[N], Rf[N];
#pragma unroll
    for (int e = 0; e < N; ++e) {
        Lf[e] = T(B.L[e]);
        Rf[e] = T(B.R[e]);
    }
    const int fb_node = a % N2, g0 = a / N2;
    const int64_t face_plane = nc * N2;
    auto project = [&](const T *w, int arr, bool state) {
        if (!active) return;
        for (int k = g0; k < 3 * NV; k += N) {
            const int d = k / NV, v = k - NV * (k / NV);
            const int st = d == 0 ? 1 : (d == 1 ? N : N2);
            const int b1 = fb_node % N, b2 = fb_node / N;
            const int node0 = d == 0 ? N * b1 + N2 * b2 : (d == 1 ? b1 + N2 * b2 : b1 + N * b2);
            const T *src = w + (state ? v : k) * P + cl * N3 + node0;
            T sl = T(0), sr = T(0);
#pragma unroll
            for (int e = 0; e < N; ++e) {
                const T x = src[e * st];
                sl += Lf[e] * x;
                sr += Rf[e] * x;
            }
            const int64_t o = (int64_t((2 * d) * 2 + arr) * NV + v) * face_plane + c * N2 + fb_node;
            traces[o] = sl;
            traces[o + int64_t(2 * NV) * face_plane] = sr;  // side 2d+1
        }
    };
    project(wF, 1, false);
    T qb1[1][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) qb1[0][v] = qb[v];
    const T *wq = pred_exchange<T, P, NBUF>(lds, buf, tid, qb1);
    project(wq, 0, true);
}

// waves per SIMD asked of the register allocator for the per-launch predictor
#ifndef ADG_PRED_WAVES5
#define ADG_PRED_WAVES5 3
#endif
// At N = 5 (not recording) three waves per SIMD.  In FP64 that also takes one
// plane buffer (30 KB instead of 61 KB per block, so that three blocks fit a
// CU) and spills 9 registers: the uniform p = 4 step at 65^3 went from 11.78
// to 11.25 ms (one buffer at two waves: 12.0 ms).
template <typename T, int N, bool STORE> struct PredWaves {
    static constexpr int MIN = (N == 5 && !STORE) ? ADG_PRED_WAVES5 : 1;
    static constexpr int NBUF = (!std::is_same<T, float>::value && N == 5 && !STORE)
                                    ? 1 : pred_nbuf(N, PredCfg<N>::CPB, int(sizeof(T)));
};

template <typename T, int N, int CPB, bool STORE>
__global__ void __launch_bounds__(round64(CPB * N * N * N))
__attribute__((amdgpu_waves_per_eu(PredWaves<T, N, STORE>::MIN, 8)))
k_predictor(const double *__restrict__ u, double *__restrict__ ustar, T *__restrict__ traces,
            const int32_t *__restrict__ list, int64_t nlist, int64_t nc,
            const int8_t *__restrict__ level, Geo geo, const double *__restrict__ dt_dev,
            double gamma, int npic, T *__restrict__ iters)
{
    constexpr int NBUF = CPB == PredCfg<N>::CPB ? PredWaves<T, N, STORE>::NBUF : pred_nbuf(N, CPB, int(sizeof(T)));
    __shared__ __align__(16) T lds[NBUF * 15 * pred_plane(N, CPB)];
    predictor_body<T, N, CPB, STORE, NBUF>(lds, u, ustar, traces, list, nlist, nc, level, geo, dt_dev[0], gamma,
                                           npic, int64_t(blockIdx.x) * CPB, iters);
}

// One variant of the batched predictor on one work item.
template <typename T, int N, int CPB>
__device__ __forceinline__ void predictor_item(T *lds, const double *u, double *ustar, T *traces, int64_t nc,
                                            const int8_t *level, const Geo *geo, double dt, double gamma,
                                            int npic, int64_t first)
{
    if constexpr (std::is_same<T, float>::value && N == 4) {
        // the FP32 N = 4 items use the same wavefront-per-cell kernel as the
        // other launch modes (results identical across modes)
        if (g_pred4_mfma_dev) {
            for (int k = int(threadIdx.x >> 6); k < CPB; k += int(blockDim.x >> 6)) {
                if (first + k >= nc) break;
                pred4_wave<true>(u, ustar, traces, first + k, nc, level ? level[first + k] : 0, *geo, dt, gamma,
                                 npic);
            }
            return;
        }
    }
    predictor_body<T, N, CPB>(lds, u, ustar, traces, nullptr, nc, nc, level, *geo, dt, gamma, npic, first);
}

// waves per SIMD asked of the register allocator for the per-order
// persistent predictor (FP32 N = 5 and 6 run faster with a few spills at the
// higher occupancy; N = 7 does not)
#ifndef ADG_ORDER_WAVES5
#define ADG_ORDER_WAVES5 3
#endif
#ifndef ADG_ORDER_WAVES6
#define ADG_ORDER_WAVES6 2
#endif
template <typename T, int N> struct PredOrderWaves {
    static constexpr int MIN = !std::is_same<T, float>::value ? 1 : N == 5 ? ADG_ORDER_WAVES5 : N == 6 ? ADG_ORDER_WAVES6 : 1;
};

// Persistent predictor over the work items of ONE order (all instances of
// that order): block b processes items b, b + gridDim, ...
template <typename T, int N, int CPB>
__global__ void __launch_bounds__(round64(CPB * N * N * N))
__attribute__((amdgpu_waves_per_eu(PredOrderWaves<T, N>::MIN, 8)))
k_predictor_order(const PredItem *__restrict__ items, int64_t nitems, const PredInst *__restrict__ insts,
                  const double *__restrict__ u, double *__restrict__ ustar, T *__restrict__ traces,
                  const double *__restrict__ dt)
{
    __shared__ __align__(16) T lds[pred_lds_elems(N, CPB, int(sizeof(T)))];
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const PredItem w = items[it];
        const PredInst &I = insts[w.inst];
        predictor_body<T, N, CPB>(lds, u + I.u_off, ustar + I.u_off, traces + I.tr_off, nullptr, I.nc, I.nc, I.level,
                                  I.geo, dt[w.inst], I.gamma, I.npic, w.first);
        __syncthreads();
    }
}

// Predictor variants compiled into the batched kernel: (N, CPB) per code.
#define ADG_PRED_VARIANTS(X) \
    X(0, 1, 64) X(1, 2, 16) X(2, 2, 32) X(3, 2, 64) X(4, 3, 4) X(5, 3, 9) X(6, 3, 18) \
    X(7, 4, 2) X(8, 4, 4) X(9, 4, 8) X(10, 5, 1) X(11, 5, 2) X(12, 5, 4) X(13, 6, 1) X(14, 6, 2) \
    X(15, 7, 1)

// One persistent launch over the work items of many instances of any order:
// block b processes items b, b + gridDim, ... ; each item is CPB cells of one
// instance, run by the (N, CPB) variant its code names.
template <typename T>
__global__ void __launch_bounds__(512)
k_predictor_batch(const PredItem *__restrict__ items, int64_t nitems, const PredInst *__restrict__ insts,
                  const double *__restrict__ u, double *__restrict__ ustar, T *__restrict__ traces,
                  const double *__restrict__ dt)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *lds = reinterpret_cast<T *>(smem);
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const PredItem w = items[it];
        const PredInst &I = insts[w.inst];
        const double dti = dt[w.inst];
        switch (w.code) {
#define ADG_CASE(code, NN, CC)                                                                                \
    case code:                                                                                                \
        predictor_item<T, NN, CC>(lds, u + I.u_off, ustar + I.u_off, traces + I.tr_off, I.nc, I.level, &I.geo, \
                                  dti, I.gamma, I.npic, w.first);                                             \
        break;
            ADG_PRED_VARIANTS(ADG_CASE)
#undef ADG_CASE
        default:
            break;
        }
        __syncthreads();
    }
}


// ---------------------------------------------------------------------------
// Predictor for N = 4 in FP32 on one wavefront per cell, without LDS.
// Lane l holds node a = l (a0 = l%4, a1 = (l/4)%4, a2 = l/16) and the whole
// time history of that node in registers.
//   x contraction: the x fibre is a lane quad -> DPP quad broadcasts fused
//                  into the FMAs;
//   y contraction: the y fibre is lanes a0 + 4 k of a 16-lane row -> DPP row
//                  rotations by 4 k;
//   z contraction: the z fibre is the four 16-lane row groups; DPP does not
//                  cross rows, so the three other values come through
//                  ds_bpermute (the LDS crossbar, which issues beside the
//                  VALU) and plain FMAs.  (A 16x16x4 MFMA with three of four
//                  A rows zero does the same sum, but matrix-core and VALU
//                  work do not overlap here, and it costs 32 cycles against
//                  16 for the FMAs);
//   time solve:    q_l -= sum_j KW[l][j] G_j is a register-axis contraction,
//                  done by v_mfma_f32_4x4x1f32 (16 blocks of 4 lanes: lane
//                  4b+i supplies KW[i][j], every lane its own G_j; register
//                  l of every lane accumulates KW[l][j] G_j).
// ---------------------------------------------------------------------------

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Fused DPP multiply-adds: acc += c[k] * x(from the lane selected by the
// DPP pattern).  The compiler does not fold DPP moves into v_fmac_f32 here,
// so the fused forms are written directly.  The hazard recognizer does not
// look inside the block, so it carries its own wait states: s_nop 1 before
// (a DPP read after a VALU write of its source).  Results feed ordinary VALU
// code or stores only, never an MFMA directly.  The blocks are volatile so
// that they are never moved into a branch with a partial EXEC mask.
//
// x fibre (a lane quad): c[k] multiplies x from the lane with a0' = (a0+k)&3.
__device__ __forceinline__ float quad_sum(const float c[4], float x, float acc)
{
    acc = fmaf(c[0], x, acc);
    asm volatile("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %1, %2 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf"
        : "+v"(acc)
        : "v"(x), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}

// y fibre (lanes a0 + 4 a1 of a 16-lane row): c[k] multiplies x from the lane
// with a1' = (a1 - k)&3 (row rotation by 4 k lanes).
__device__ __forceinline__ float row_sum(const float c[4], float x, float acc)
{
    acc = fmaf(c[0], x, acc);
    asm volatile("s_nop 1\n\t"
        "v_fmac_f32_dpp %0, %1, %2 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %3 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %1, %4 row_ror:12 row_mask:0xf bank_mask:0xf"
        : "+v"(acc)
        : "v"(x), "v"(c[1]), "v"(c[2]), "v"(c[3]));
    return acc;
}

// x and y derivative sums of the five flux components of one time node.  On
// entry G[v] holds the lane's own x term; adds the lane's own y term, then the
// three neighbour terms of x (quad rotations) and of y (row rotations by 4, 8,
// 12 lanes).  The five plain FMAs ahead of the first DPP read give the DPP
// sources their required distance from any earlier write.  G is read next by
// ordinary (compiler-scheduled) VALU code only.
__device__ __forceinline__ void xy_sums5(float G[NV], const float fx[NV], const float fy[NV], const float Cx[4],
                                         const float Cy[4])
{
    asm volatile(
        "v_fmac_f32 %0, %10, %15\n\t"
        "v_fmac_f32 %1, %11, %15\n\t"
        "v_fmac_f32 %2, %12, %15\n\t"
        "v_fmac_f32 %3, %13, %15\n\t"
        "v_fmac_f32 %4, %14, %15\n\t"
        "v_fmac_f32_dpp %0, %5, %16 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %6, %16 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %7, %16 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %8, %16 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %9, %16 quad_perm:[1,2,3,0] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %5, %17 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %6, %17 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %7, %17 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %8, %17 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %9, %17 quad_perm:[2,3,0,1] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %5, %18 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %6, %18 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %7, %18 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %8, %18 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %9, %18 quad_perm:[3,0,1,2] row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %10, %19 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %11, %19 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %12, %19 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %13, %19 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %14, %19 row_ror:4 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %10, %20 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %11, %20 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %12, %20 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %13, %20 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %14, %20 row_ror:8 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %0, %10, %21 row_ror:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %1, %11, %21 row_ror:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %2, %12, %21 row_ror:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %3, %13, %21 row_ror:12 row_mask:0xf bank_mask:0xf\n\t"
        "v_fmac_f32_dpp %4, %14, %21 row_ror:12 row_mask:0xf bank_mask:0xf"
        : "+v"(G[0]), "+v"(G[1]), "+v"(G[2]), "+v"(G[3]), "+v"(G[4])
        : "v"(fx[0]), "v"(fx[1]), "v"(fx[2]), "v"(fx[3]), "v"(fx[4]), "v"(fy[0]), "v"(fy[1]), "v"(fy[2]),
          "v"(fy[3]), "v"(fy[4]), "v"(Cy[0]), "v"(Cx[1]), "v"(Cx[2]), "v"(Cx[3]), "v"(Cy[1]), "v"(Cy[2]),
          "v"(Cy[3]));
}

// Raw buffer views: a wave-uniform base (in scalar registers) of a given byte
// size, addressed by a 32-bit lane offset.  Offsets beyond the size read as
// zero and drop stores (buffer range checking), which is also how lanes skip
// a store without a branch.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_view(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, 0x00020000);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, double x)
{
    using b64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(b64, x), r, off, 0, 0);
}

// x of the lane whose byte address (4 x lane index) is addr, through the LDS
// crossbar (no LDS memory is used)
__device__ __forceinline__ float from_row(int addr, float x)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
}

// base + byte offset, with the offset a 32-bit unsigned value: a wave-uniform
// base then stays in scalar registers and the access uses scalar-base addressing
template <typename T> __device__ __forceinline__ T *lane_at(T *base, unsigned byte_off)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off);
}
template <typename T> __device__ __forceinline__ const T *lane_at(const T *base, unsigned byte_off)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// One cell per wavefront; work item w covers cells first + w.
template <bool KEEP_U>
__device__ __forceinline__ void pred4_wave(const double *__restrict__ u, double *__restrict__ ustar,
                                           float *__restrict__ traces, int64_t c, int64_t nc, int lev,
                                           const Geo &geo, double dt, double gamma, int npic)
{
    constexpr int N = 4, N2 = 16, N3 = 64;
    const DevBasis &B = c_basis[N];
    const int l = threadIdx.x & 63;
    const int a0 = l & 3, a1 = (l >> 2) & 3, a2 = l >> 4;
    const float cx = float(dt * geo.inv_dx[lev][0]);
    const float cy = float(dt * geo.inv_dx[lev][1]);
    const float cz = float(dt * geo.inv_dx[lev][2]);
    const float gm1 = float(gamma - 1.0);

    // wave-uniform bases plus a 32-bit lane byte offset (scalar-base addressing)
    const unsigned lu = unsigned(l) * unsigned(sizeof(double));
    float uu[NV];
    double ud[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        ud[v] = *lane_at(u + (int64_t(v) * nc + c) * N3, lu);
        uu[v] = float(ud[v]);
    }

    // per-lane coefficients (one scalar base, one lane offset)
    const float *Tl = lane_at(static_cast<const float *>(c_lane4), unsigned(l) * unsigned(LANE4 * sizeof(float)));
    float Cx[4], Cy[4], Cz[4], KWa[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        Cx[e] = cx * Tl[e];
        Cy[e] = cy * Tl[4 + e];
        Cz[e] = cz * Tl[8 + e];
        KWa[e] = Tl[12 + e];  // lane 4b+i supplies KW[i][j], i = a0
    }
    // z neighbours come through the LDS crossbar: from_row(pz[k], x) is x of
    // the lane with a2' = (a2 + k) & 3 (same a0, a1)
    int pz[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pz[k] = ((l + 16 * k) & 63) * 4;

    // scaled divergence sum_d (dt/dx_d) D_d F_d(qn) at this lane's node
    auto spatial = [&](const float qn[NV], float g[NV]) {
        float f[3][NV];
        euler_flux3_fast(gm1, qn, f);
        float zn[3][NV];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int k = 1; k < 4; ++k) zn[k - 1][v] = from_row(pz[k], f[2][v]);
        SCHED_SPLIT();
#pragma unroll
        for (int v = 0; v < NV; ++v) g[v] = Cx[0] * f[0][v];
        xy_sums5(g, f[0], f[1], Cx, Cy);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            g[v] = fmaf(Cz[0], f[2][v], g[v]);
#pragma unroll
            for (int k = 1; k < 4; ++k) g[v] = fmaf(Cz[k], zn[k - 1][v], g[v]);
        }
    };

    float q[N][NV];
    if (npic > 0) {
        // first iteration from q = u at every time node: one flux and one
        // spatial sum serve all time nodes, and the row sums of KW finish
        // the time solve
        float g[NV];
        spatial(uu, g);
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) q[j][v] = fmaf(-c_kwsum4[j], g[v], uu[v]);
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) q[j][v] = uu[v];
    }

    for (int it = 1; it < npic; ++it) {
        f32x4 acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < N; ++j) {
            float g[NV];
            spatial(q[j], g);
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = __builtin_amdgcn_mfma_f32_4x4x1f32(KWa[j], g[v], acc[v], 0, 0, 0);
            SCHED_SPLIT();
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int j = 0; j < N; ++j) q[j][v] = uu[v] - acc[v][j];
    }

    // time averages of the final iterate
    float qb[NV], Fb[3][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        qb[v] = 0.f;
        Fb[0][v] = Fb[1][v] = Fb[2][v] = 0.f;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        float f[3][NV];
        euler_flux3_fast(gm1, q[j], f);
        const float wj = float(B.w[j]);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qb[v] = fmaf(wj, q[j][v], qb[v]);
#pragma unroll
            for (int d = 0; d < 3; ++d) Fb[d][v] = fmaf(wj, f[d][v], Fb[d][v]);
        }
    }

    // volume term with the weak stiffness Kw (same three mechanisms)
    {
        float Vx[4], Vy[4], Vz[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Vx[e] = cx * Tl[16 + e];
            Vy[e] = cy * Tl[20 + e];
            Vz[e] = cz * Tl[24 + e];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            float V = Vz[0] * Fb[2][v];
#pragma unroll
            for (int k = 1; k < 4; ++k) V = fmaf(Vz[k], from_row(pz[k], Fb[2][v]), V);
            V = quad_sum(Vx, Fb[0][v], V);
            V = row_sum(Vy, Fb[1][v], V);
            const int64_t o = (int64_t(v) * nc + c) * N3;
            *lane_at(ustar + o, lu) = (KEEP_U ? ud[v] : *lane_at(u + o, lu)) + double(V);
        }
    }

    // face projections: L (minus) and R (plus) along each axis.  The x sum
    // runs with L weights in lanes a0 = 0 and R weights in the other lanes, so
    // lane a0 = 0 holds the minus-face value and lane a0 = 3 the plus-face
    // value of one sum (y likewise over a1).  Stores go through 64-byte raw
    // buffer views of one face plane each; lanes that do not store get an
    // offset beyond the view, which buffer range checking drops.
    {
        float Px[4], Py[4], Pz[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Px[e] = Tl[28 + e];
            Py[e] = Tl[32 + e];
            Pz[e] = Tl[36 + e];
        }
        constexpr unsigned F = sizeof(float), OUT = 0x80000000u;
        const unsigned bx = (a1 + 4 * a2) * F, by = (a0 + 4 * a2) * F, bz = (a0 + 4 * a1) * F;
        const unsigned o0 = a0 == 0 ? bx : OUT, o1 = a0 == 3 ? bx : OUT;
        const unsigned o2 = a1 == 0 ? by : OUT, o3 = a1 == 3 ? by : OUT;
        const unsigned o4 = a2 == 0 ? bz : OUT, o5 = a2 == 3 ? bz : OUT;
        auto put = [&](int s, int arr, int v, unsigned off, float x) {
            float *plane = traces + ((int64_t(s * 2 + arr) * NV + v) * nc + c) * N2;
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x),
                                                  __builtin_amdgcn_make_buffer_rsrc(plane, 0, N2 * F, 0x00020000),
                                                  off, 0, 0);
        };
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int arr = 0; arr < 2; ++arr) {
                // x faces: state or normal flux Fx
                const float px = quad_sum(Px, arr == 0 ? qb[v] : Fb[0][v], 0.f);
                put(0, arr, v, o0, px);
                put(1, arr, v, o1, px);
                const float py = row_sum(Py, arr == 0 ? qb[v] : Fb[1][v], 0.f);
                put(2, arr, v, o2, py);
                put(3, arr, v, o3, py);
                const float zv = arr == 0 ? qb[v] : Fb[2][v];
                float pz_ = Pz[0] * zv;
#pragma unroll
                for (int k = 1; k < 4; ++k) pz_ = fmaf(Pz[k], from_row(pz[k], zv), pz_);
                put(4, arr, v, o4, pz_);
                put(5, arr, v, o5, pz_);
            }
        }
    }
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_predictor4_mfma(const double *__restrict__ u, double *__restrict__ ustar, float *__restrict__ traces,
                  const int32_t *__restrict__ list, int64_t nlist, int64_t nc, const int8_t *__restrict__ level,
                  Geo geo, const double *__restrict__ dt_dev, double gamma, int npic)
{
    // the wave index is uniform across the wavefront: saying so keeps the cell
    // index and every address derived from it in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t idx = int64_t(blockIdx.x) * (blockDim.x >> 6) + wave;
    if (idx >= nlist) return;  // whole wavefront leaves together
    const int64_t c = list ? int64_t(list[idx]) : idx;
    pred4_wave<true>(u, ustar, traces, c, nc, level ? level[c] : 0, geo, dt_dev[0], gamma, npic);
}

// persistent form over batched work items of order 4 (items of CPB cells)
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_predictor4_mfma_order(const PredItem *__restrict__ items, int64_t nitems, const PredInst *__restrict__ insts,
                        const double *__restrict__ u, double *__restrict__ ustar, float *__restrict__ traces,
                        const double *__restrict__ dt, int cpb)
{
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), nwaves = blockDim.x >> 6;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const PredItem w = items[it];
        const PredInst &I = insts[w.inst];
        for (int k = wave; k < cpb; k += nwaves) {
            const int64_t c = w.first + k;
            if (c >= I.nc) break;
            pred4_wave<true>(u + I.u_off, ustar + I.u_off, traces + I.tr_off, c, I.nc, I.level ? I.level[c] : 0,
                             I.geo, dt[w.inst], I.gamma, I.npic);
        }
    }
}

// ---------------------------------------------------------------------------
// Predictor for N = 4 in FP64 on one wavefront per cell, without LDS memory.
// The same lane layout as the FP32 kernel above (lane l = node a = l, the
// whole time history of the node in registers).
//   x contraction: DPP quad permutations (a double moves as two 32-bit
//                  DPP moves into a register pair), then FMAs;
//   y contraction: DPP row rotations by 4 k lanes;
//   z contraction: one v_mfma_f64_4x4x4f64 per variable.  Its 4 blocks are
//                  the lane groups of equal a1; block b takes A[i][k] from
//                  lane 4b + i + 16k and B[k][j] from lane 4b + j + 16k and
//                  puts D[i][j] in lane 4b + j + 16i (measured on gfx950).
//                  With the node layout, B[k][j] is the flux at node
//                  (a0 = j, a1 = b, a2 = k) and D[i][j] lands on node
//                  (j, b, i): the matrix core contracts over a2 in place,
//                  given A[i][k] = (dt/dz) D_ik in lane i + 16k (any block),
//                  and accumulates onto the x and y sums (C operand);
//   time solve:    q_l = u - sum_j KW[l][j] G_j with the KW entries
//                  wave-uniform (scalar operands of the FMAs).
// ---------------------------------------------------------------------------

// x from the lane that the DPP control CTRL selects (two 32-bit DPP moves
// into a register pair; every source lane exists for these controls)
template <int CTRL> __device__ __forceinline__ double dpp64(double x)
{
    return __longlong_as_double(__builtin_amdgcn_mov_dpp(__double_as_longlong(x), CTRL, 0xf, 0xf, true));
}
// DPP controls: quad_perm [1,2,3,0], [2,3,0,1], [3,0,1,2]; row_ror by 4, 8, 12
constexpr int DPP_QP1 = 0x39, DPP_QP2 = 0x4E, DPP_QP3 = 0x93;
constexpr int DPP_ROR4 = 0x124, DPP_ROR8 = 0x128, DPP_ROR12 = 0x12C;

// sum_e c[e] x(lane of the e-th neighbour along the axis): x through quad
// permutations (axis 0) or row rotations (axis 1)
template <int AXIS>
__device__ __forceinline__ double fibre_sum64(const double c[4], double x, double acc)
{
    acc = fma(c[0], x, acc);
    if constexpr (AXIS == 0) {
        acc = fma(c[1], dpp64<DPP_QP1>(x), acc);
        acc = fma(c[2], dpp64<DPP_QP2>(x), acc);
        acc = fma(c[3], dpp64<DPP_QP3>(x), acc);
    } else {
        acc = fma(c[1], dpp64<DPP_ROR4>(x), acc);
        acc = fma(c[2], dpp64<DPP_ROR8>(x), acc);
        acc = fma(c[3], dpp64<DPP_ROR12>(x), acc);
    }
    return acc;
}

// acc + sum_k A[a2][k] x(node a0, a1, k) on the matrix cores; a is this
// lane's A entry (row lane & 3, column lane >> 4)
__device__ __forceinline__ double zsum64(double a, double x, double acc)
{
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, x, acc, 0, 0, 0);
}

// STORE: also write what the adjoint reads, in planes [v][c][node] of one
// time node each: the final iterate (time node j in plane j), the first
// iteration's divergence G(u) in plane N (npic >= 2; the first iterate is
// u - KWsum_j G(u), which the adjoint rebuilds with the same fma), and
// iterate r = 2 .. npic-1 at time node j in plane N + 1 + (r-2) N + j.
// At most npic N planes.  The tape is read once, by the adjoint step, and
// goes out with non-temporal stores: at 27^3 its 650 MB per step otherwise
// pushed the step's own projections out of the 256 MB Infinity Cache before
// the face kernel read them (that kernel took 89 instead of 56 us).
template <bool STORE>
__device__ __forceinline__ void pred4_wave_f64(const double *__restrict__ u, double *__restrict__ ustar,
                                               double *__restrict__ traces, int64_t c, int64_t nc, int lev,
                                               const Geo &geo, double dt, double gamma, int npic,
                                               double *__restrict__ iters)
{
    constexpr int N = 4, N2 = 16, N3 = 64;
    const DevBasis &B = c_basis[N];
    const int l = threadIdx.x & 63;
    const int a0 = l & 3, a1 = (l >> 2) & 3, a2 = l >> 4;
    const double cd[3] = {dt * geo.inv_dx[lev][0], dt * geo.inv_dx[lev][1], dt * geo.inv_dx[lev][2]};
    const double gm1 = gamma - 1.0;
    const unsigned lu = unsigned(l) * unsigned(sizeof(double));
    double uu[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uu[v] = *lane_at(u + (int64_t(v) * nc + c) * N3, lu);

    // neighbour e of this lane along x and y: a0 + e (quad permutation),
    // a1 - e (row rotation), mod 4; the z operator as this lane's MFMA A
    // entry, row zi = l & 3, column zk = l >> 4
    const int nx[4] = {a0, (a0 + 1) & 3, (a0 + 2) & 3, (a0 + 3) & 3};
    const int ny[4] = {a1, (a1 + 3) & 3, (a1 + 2) & 3, (a1 + 1) & 3};
    const int zi = l & 3, zk = l >> 4;
    double Cx[4], Cy[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        Cx[e] = cd[0] * B.D[a0 * N + nx[e]];
        Cy[e] = cd[1] * B.D[a1 * N + ny[e]];
    }
    const double Az = cd[2] * B.D[zi * N + zk];

    // scaled divergence sum_d (dt/dx_d) D_d F_d(qn) at this lane's node
    auto spatial = [&](const double qn[NV], double g[NV]) {
        double f[3][NV];
        euler_flux3<double, true>(gm1, qn, f);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = fibre_sum64<0>(Cx, f[0][v], 0.0);
            s = fibre_sum64<1>(Cy, f[1][v], s);
            g[v] = zsum64(Az, f[2][v], s);
        }
    };

    double q[N][NV];
    // time node j of the current iterate into plane p0 + j
    auto store_iterate = [&](int64_t p0) {
        if constexpr (STORE) {
#pragma unroll
            for (int j = 0; j < N; ++j)
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    __builtin_nontemporal_store(q[j][v], lane_at(iters + (((p0 + j) * NV + v) * nc + c) * N3, lu));
        }
    };
    if (npic > 0) {
        // first iteration from q = u at every time node: one flux and one
        // divergence serve all time nodes; the row sums of KW finish it
        double g[NV];
        spatial(uu, g);
        if constexpr (STORE) {
            if (npic >= 2)
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    __builtin_nontemporal_store(g[v], lane_at(iters + ((int64_t(N) * NV + v) * nc + c) * N3, lu));
        }
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) q[j][v] = fma(-B.KWsum[j], g[v], uu[v]);
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) q[j][v] = uu[v];
    }
    for (int it = 1; it < npic; ++it) {
        // G_j replaces q_j as soon as it is formed (q_j is not needed
        // again), so the iterate and the divergences share registers; the
        // time solve then sums over j in order
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double g[NV];
            spatial(q[j], g);
#pragma unroll
            for (int v = 0; v < NV; ++v) q[j][v] = g[v];
        }
        double qn[N][NV];
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) acc = fma(B.KW[i * N + j], q[j][v], acc);
                qn[i][v] = uu[v] - acc;
            }
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int v = 0; v < NV; ++v) q[i][v] = qn[i][v];
        if (it + 1 < npic) store_iterate(N + 1 + int64_t(it - 1) * N);  // iterate it + 1
    }
    if (npic > 0) store_iterate(0);  // the final iterate

    // time averages of the final iterate
    double qb[NV], Fb[3][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        qb[v] = 0.0;
        Fb[0][v] = Fb[1][v] = Fb[2][v] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double f[3][NV];
        euler_flux3<double, true>(gm1, q[j], f);
        const double wj = B.w[j];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qb[v] = fma(wj, q[j][v], qb[v]);
#pragma unroll
            for (int d = 0; d < 3; ++d) Fb[d][v] = fma(wj, f[d][v], Fb[d][v]);
        }
    }

    // volume term of the corrector with the weak stiffness Kw
    {
        double Vx[4], Vy[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Vx[e] = cd[0] * B.winv[a0] * B.Kw[a0 * N + nx[e]];
            Vy[e] = cd[1] * B.winv[a1] * B.Kw[a1 * N + ny[e]];
        }
        const double Vz = cd[2] * B.winv[zi] * B.Kw[zi * N + zk];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double V = fibre_sum64<0>(Vx, Fb[0][v], 0.0);
            V = fibre_sum64<1>(Vy, Fb[1][v], V);
            V = zsum64(Vz, Fb[2][v], V);
            *lane_at(ustar + (int64_t(v) * nc + c) * N3, lu) = uu[v] + V;
        }
    }

    // face projections: along each axis the lanes at index 0 hold the minus
    // face (L weights) and the lanes at index 3 the plus face (R weights) of
    // one sum; the others' stores get an offset beyond the 128-byte plane
    // view, which buffer range checking drops
    {
        double Px[4], Py[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Px[e] = a0 == 0 ? B.L[nx[e]] : B.R[nx[e]];
            Py[e] = a1 == 0 ? B.L[ny[e]] : B.R[ny[e]];
        }
        // rows 0 (minus face) and 3 (plus face) of the z projection
        const double Pz = zi == 0 ? B.L[zk] : B.R[zk];
        constexpr unsigned F = sizeof(double), OUT = 0x80000000u;
        const unsigned bx = (a1 + 4 * a2) * F, by = (a0 + 4 * a2) * F, bz = (a0 + 4 * a1) * F;
        const unsigned o0 = a0 == 0 ? bx : OUT, o1 = a0 == 3 ? bx : OUT;
        const unsigned o2 = a1 == 0 ? by : OUT, o3 = a1 == 3 ? by : OUT;
        const unsigned o4 = a2 == 0 ? bz : OUT, o5 = a2 == 3 ? bz : OUT;
        auto put = [&](int s, int arr, int v, unsigned off, double x) {
            double *plane = traces + ((int64_t(s * 2 + arr) * NV + v) * nc + c) * N2;
            buf_st(buf_view(plane, N2 * F), off, x);
        };
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int arr = 0; arr < 2; ++arr) {
                const double px = fibre_sum64<0>(Px, arr == 0 ? qb[v] : Fb[0][v], 0.0);
                put(0, arr, v, o0, px);
                put(1, arr, v, o1, px);
                const double py = fibre_sum64<1>(Py, arr == 0 ? qb[v] : Fb[1][v], 0.0);
                put(2, arr, v, o2, py);
                put(3, arr, v, o3, py);
                const double pzv = zsum64(Pz, arr == 0 ? qb[v] : Fb[2][v], 0.0);
                put(4, arr, v, o4, pzv);
                put(5, arr, v, o5, pzv);
            }
        }
    }
}

template <bool STORE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_predictor4_f64(const double *__restrict__ u, double *__restrict__ ustar, double *__restrict__ traces,
                 const int32_t *__restrict__ list, int64_t nlist, int64_t nc, const int8_t *__restrict__ level,
                 Geo geo, const double *__restrict__ dt_dev, double gamma, int npic, double *__restrict__ iters)
{
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t idx = int64_t(blockIdx.x) * (blockDim.x >> 6) + wave;
    if (idx >= nlist) return;  // whole wavefront leaves together
    const int64_t c = list ? int64_t(list[idx]) : idx;
    pred4_wave_f64<STORE>(u, ustar, traces, c, nc, level ? level[c] : 0, geo, dt_dev[0], gamma, npic, iters);
}

// sum_d (d f_d / d q)^T fb[d] added to qb, for the Euler fluxes of the three
// axes at once (their common terms formed once).  With v = m / rho,
// H = (E + p) / rho, fb[d] = (a_d, b_d1, b_d2, b_d3, c_d) and
// S = sum_d (b_dd + v_d c_d), the weight every p-term carries:
//   qb_rho += -sum_d v_d (sum_k b_dk v_k + H c_d) + S (gamma-1) |v|^2 / 2
//   qb_m_j += a_j + sum_k b_jk v_k + sum_d b_dj v_d + c_j H - S (gamma-1) v_j
//   qb_E   += sum_d c_d v_d + S (gamma-1)
__device__ __forceinline__ void flux3_vjp(double gm1, const double q[NV], const double fb[3][NV], double qb[NV])
{
    const double inv = 1.0 / q[0];
    const double v[3] = {q[1] * inv, q[2] * inv, q[3] * inv};
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double p = gm1 * (q[4] - 0.5 * q[0] * v2);
    const double H = (q[4] + p) * inv;
    double S = 0.0, r = 0.0, e = 0.0;
    double bv[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        bv[d] = fb[d][1] * v[0] + fb[d][2] * v[1] + fb[d][3] * v[2];
        S += fb[d][1 + d] + v[d] * fb[d][4];
        r -= v[d] * (bv[d] + H * fb[d][4]);
        e += fb[d][4] * v[d];
    }
    qb[0] += r + S * gm1 * 0.5 * v2;
#pragma unroll
    for (int j = 0; j < 3; ++j)
        qb[1 + j] += fb[j][0] + bv[j] + (fb[0][1 + j] * v[0] + fb[1][1 + j] * v[1] + fb[2][1 + j] * v[2]) +
                     fb[j][4] * H - S * gm1 * v[j];
    qb[4] += e + S * gm1;
}

// Adjoint of the FP64 N = 4 predictor (the forward kernel above) on one
// wavefront per cell, lane = node.  The transposed contractions use the same
// exchanges as the forward ones with transposed coefficients (x and y by
// DPP, z on the matrix cores with A[i][k] = transposed operator); the
// Picard iterates come from the forward run (iters, slots 0..npic-1 =
// iterates 1..npic).
__device__ __forceinline__ void pred4_adj_wave(const double *__restrict__ u, const double *__restrict__ iters,
                                               const double *__restrict__ ubar_next, const double *__restrict__ tbar,
                                               double *__restrict__ ubar, int64_t c, int64_t nc, int lev,
                                               const Geo &geo, double dt, double gamma, int npic)
{
    constexpr int N = 4, N2 = 16, N3 = 64;
    const DevBasis &B = c_basis[N];
    const int l = threadIdx.x & 63;
    const int a0 = l & 3, a1 = (l >> 2) & 3, a2 = l >> 4;
    const int bf[3] = {a1 + N * a2, a0 + N * a2, a0 + N * a1};
    const double cd[3] = {dt * geo.inv_dx[lev][0], dt * geo.inv_dx[lev][1], dt * geo.inv_dx[lev][2]};
    const double gm1 = gamma - 1.0;
    const unsigned lu = unsigned(l) * unsigned(sizeof(double));
    const int nx[4] = {a0, (a0 + 1) & 3, (a0 + 2) & 3, (a0 + 3) & 3};
    const int ny[4] = {a1, (a1 + 3) & 3, (a1 + 2) & 3, (a1 + 1) & 3};
    const int zi = l & 3, zk = l >> 4;
    // the iterates from the forward kernel's planes (the launch requires
    // npic >= 1, so none of them is the state u itself; a select between the
    // state and the tape had the compiler split the kernel into branches,
    // across which the exchanged values stayed live: 330 registers, not 168)
    auto load_plane = [&](int64_t pl, double q[NV]) {  // read once: non-temporal
        const double *base = iters + (pl * NV * nc + c) * N3;
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = __builtin_nontemporal_load(lane_at(base + int64_t(v) * nc * N3, lu));
    };

    // adjoint of u* = u + volume term: identity, and the transposed volume
    // term into the time-averaged fluxes
    double ub[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        ub[v] = *lane_at(ubar_next + (int64_t(v) * nc + c) * N3, lu);
        acc[v] = ub[v];
    }
    double Fbb[3][NV], qbb[NV];
    {
        double Vx[4], Vy[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Vx[e] = cd[0] * B.winv[nx[e]] * B.Kw[nx[e] * N + a0];
            Vy[e] = cd[1] * B.winv[ny[e]] * B.Kw[ny[e] * N + a1];
        }
        const double Vz = cd[2] * B.winv[zk] * B.Kw[zk * N + zi];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Fbb[0][v] = fibre_sum64<0>(Vx, ub[v], 0.0);
            Fbb[1][v] = fibre_sum64<1>(Vy, ub[v], 0.0);
            Fbb[2][v] = zsum64(Vz, ub[v], 0.0);
            SCHED_SPLIT();
        }
    }
    // adjoint of the face projections (each node reads its own face entries)
#pragma unroll
    for (int v = 0; v < NV; ++v) qbb[v] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int ad = d == 0 ? a0 : (d == 1 ? a1 : a2);
        const double Lk = B.L[ad], Rk = B.R[ad];
        const unsigned fo = unsigned(bf[d]) * unsigned(sizeof(double));
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double *qm = tbar + ((int64_t((2 * d) * 2 + 0) * NV + v) * nc + c) * N2;
            const double *qp = tbar + ((int64_t((2 * d + 1) * 2 + 0) * NV + v) * nc + c) * N2;
            const double *fm = tbar + ((int64_t((2 * d) * 2 + 1) * NV + v) * nc + c) * N2;
            const double *fp = tbar + ((int64_t((2 * d + 1) * 2 + 1) * NV + v) * nc + c) * N2;
            qbb[v] += Lk * *lane_at(qm, fo) + Rk * *lane_at(qp, fo);
            Fbb[d][v] += Lk * *lane_at(fm, fo) + Rk * *lane_at(fp, fo);
        }
        SCHED_SPLIT();  // one axis of loads in flight at a time
    }
    // adjoint of the time averages of the final iterate
    double qbar[N][NV];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double q[NV], fbw[3][NV];
        load_plane(j, q);  // the final iterate
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            qbar[j][v] = B.w[j] * qbb[v];
#pragma unroll
            for (int d = 0; d < 3; ++d) fbw[d][v] = B.w[j] * Fbb[d][v];
        }
        flux3_vjp(gm1, q, fbw, qbar[j]);
        SCHED_SPLIT();
    }
    // transposed derivative operators (dt/dx_d) D_d^T
    double Dx[4], Dy[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        Dx[e] = cd[0] * B.D[nx[e] * N + a0];
        Dy[e] = cd[1] * B.D[ny[e] * N + a1];
    }
    const double Dz = cd[2] * B.D[zk * N + zi];
    // Picard iterations in reverse: q^(r) = u - sum_j KW[l][j] G_j(q^(r-1)),
    // r = npic .. 2; the divergences' adjoints Gb_j replace the iterate
    // adjoints, which are then rebuilt time node by time node
    auto divergence_vjp = [&](const double q[NV], const double gb[NV], double nb[NV]) {
        double fb[3][NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            fb[0][v] = fibre_sum64<0>(Dx, gb[v], 0.0);
            fb[1][v] = fibre_sum64<1>(Dy, gb[v], 0.0);
            fb[2][v] = zsum64(Dz, gb[v], 0.0);
            nb[v] = 0.0;
        }
        flux3_vjp(gm1, q, fb, nb);
    };
    // one reverse iteration, given the iterate it was formed from
    auto reverse_iteration = [&](auto &&load_prev) {
        double Gb[N][NV];
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) s = fma(B.KW[i * N + j], qbar[i][v], s);
                Gb[j][v] = -s;
            }
#pragma unroll
        for (int i = 0; i < N; ++i)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += qbar[i][v];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double q[NV];
            load_prev(j, q);
            divergence_vjp(q, Gb[j], qbar[j]);
            SCHED_SPLIT();  // one time node at a time: bounds the live registers
        }
    };
    for (int r = npic; r >= 3; --r)  // iterate r - 1 >= 2 is stored
        reverse_iteration([&](int j, double q[NV]) { load_plane(N + 1 + int64_t(r - 3) * N + j, q); });
    if (npic >= 2)  // iterate 1 = u - KWsum_j G(u), as the forward kernel formed it
        reverse_iteration([&](int j, double q[NV]) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                q[v] = fma(-B.KWsum[j], *lane_at(iters + ((int64_t(N) * NV + v) * nc + c) * N3, lu),
                           *lane_at(u + (int64_t(v) * nc + c) * N3, lu));
        });
    // r = 1: every q^(0)_j is u, and one divergence served all time nodes
    // with the row sums of KW; q^(0) = u adds the rest
    {
        double gs[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                s = fma(B.KWsum[i], qbar[i][v], s);
                acc[v] += qbar[i][v];
            }
            gs[v] = -s;
        }
        double q[NV], nb[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = *lane_at(u + (int64_t(v) * nc + c) * N3, lu);
        divergence_vjp(q, gs, nb);
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += nb[v];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) *lane_at(ubar + (int64_t(v) * nc + c) * N3, lu) = acc[v];
}

// three waves per SIMD (168 VGPRs, 14 of them spilled around the rebuilt
// first iterate); at two waves (176 VGPRs, no spills) the gradient of 20
// steps at 27^3 took 1 % longer
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_predictor4_adj_f64(const double *__restrict__ u, const double *__restrict__ iters,
                     const double *__restrict__ ubar_next, const double *__restrict__ tbar,
                     const double *__restrict__ dt_dev, double *__restrict__ ubar, int64_t nc,
                     const int8_t *__restrict__ level, Geo geo, double gamma, int npic)
{
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t c = int64_t(blockIdx.x) * (blockDim.x >> 6) + wave;
    if (c >= nc) return;  // whole wavefront leaves together
    pred4_adj_wave(u, iters, ubar_next, tbar, ubar, c, nc, level ? level[c] : 0, geo, dt_dev[0], gamma, npic);
}

// ---------------------------------------------------------------------------
// Riemann solves on conforming faces of one axis
// ---------------------------------------------------------------------------

// maximum over the 16 lanes of each DPP row, in every lane (rotations by 8,
// 4, 2, 1 lanes); doubles move as two 32-bit halves
template <int K> __device__ __forceinline__ float ror_max(float x)
{
    return fmaxf(x, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x120 + K, 0xf, 0xf, false)));
}
template <int K> __device__ __forceinline__ double ror_max(double x)
{
    const long long bits = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, int(bits & 0xffffffff), 0x120 + K, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(bits >> 32), 0x120 + K, 0xf, 0xf, false);
    return fmax(x, __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo)));
}
template <typename T> __device__ __forceinline__ T row_max16(T x)
{
    return ror_max<1>(ror_max<2>(ror_max<4>(ror_max<8>(x))));
}

template <int N> struct FaceCfg {
    static constexpr int FPB = (256 / (N * N)) > 0 ? 256 / (N * N) : 1;
    static constexpr int THREADS = round64(FPB * N * N);
};

// B32: every trace and face plane (one side, array and variable over all
// cells) is below 2 GiB, so accesses are buffer loads and stores from a
// scalar plane base with a 32-bit per-lane offset
// Rusanov flux of one face node from both sides' projections and the face
// speed s: one fixed chain of operations, shared by every kernel that solves
// conforming faces, so they all give the same bits.
template <typename T>
__device__ __forceinline__ T rusanov(T FL, T FR, T QL, T QR, T s)
{
    return fma(T(-0.5) * s, QR - QL, T(0.5) * (FL + FR));
}

template <typename T, int N, bool B32>
__global__ void __launch_bounds__(FaceCfg<N>::THREADS)
k_riemann(const T *__restrict__ traces, T *__restrict__ fside, const int32_t *__restrict__ fm,
          const int32_t *__restrict__ fp, int64_t nf, int d, int64_t nc, double gamma,
          int *__restrict__ status, int16_t *__restrict__ tape, int tape_mode)
{
    constexpr int N2 = N * N, FPB = FaceCfg<N>::FPB;
    __shared__ T slam[FPB * N2 * 2];
    const int tid = threadIdx.x;
    const int fl = tid / N2, b = tid % N2;
    const int64_t f = int64_t(blockIdx.x) * FPB + fl;
    const bool lane_ok = tid < FPB * N2;
    const bool active = lane_ok && f < nf;
    const T g = T(gamma), gm1 = T(gamma - 1.0);
    const int sL = 2 * d + 1, sR = 2 * d;
    T QL[NV], FL[NV], QR[NV], FR[NV];
    int64_t cL = 0, cR = 0;
    T lL = T(0), lR = T(0);
    if (active) {
        cL = fm[f];
        cR = fp[f];
        if constexpr (B32) {
            const int pb = int(nc * N2 * int64_t(sizeof(T)));
            const unsigned oL = unsigned(cL * N2 + b) * unsigned(sizeof(T));
            const unsigned oR = unsigned(cR * N2 + b) * unsigned(sizeof(T));
            auto plane = [&](int side, int arr, int v) {
                return buf_view(traces + (int64_t(side * 2 + arr) * NV + v) * nc * N2, pb);
            };
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                QL[v] = buf_ld(plane(sL, 0, v), oL, T(0));
                FL[v] = buf_ld(plane(sL, 1, v), oL, T(0));
                QR[v] = buf_ld(plane(sR, 0, v), oR, T(0));
                FR[v] = buf_ld(plane(sR, 1, v), oR, T(0));
            }
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                QL[v] = traces[((int64_t(sL * 2 + 0) * NV + v) * nc + cL) * N2 + b];
                FL[v] = traces[((int64_t(sL * 2 + 1) * NV + v) * nc + cL) * N2 + b];
                QR[v] = traces[((int64_t(sR * 2 + 0) * NV + v) * nc + cR) * N2 + b];
                FR[v] = traces[((int64_t(sR * 2 + 1) * NV + v) * nc + cR) * N2 + b];
            }
        }
        bool badL, badR;
        lL = wave_speed(g, gm1, QL, d, badL);
        lR = wave_speed(g, gm1, QR, d, badR);
        if (badL || badR) *status = 1;
    }
    T s;
    if (N2 == 16 && tape_mode == TAPE_OFF) {
        // one face per 16-lane row: the maximum over (node, side) by row
        // rotations (a maximum is exact, so this equals the serial scan)
        s = row_max16(lL > lR ? lL : lR);  // speeds are >= 0 and finite unless flagged
        if (!active) return;
    } else {
    if (lane_ok) {
        slam[2 * tid] = lL;
        slam[2 * tid + 1] = lR;
    }
    __syncthreads();
    if (!active) return;
    // s = the largest speed over (node, side); its first maximiser in
    // (node, minus side first) order can be recorded or replayed
    if (tape_mode == TAPE_REPLAY) {
        s = slam[2 * fl * N2 + tape[f]];
    } else {
        s = T(-1);
        int arg = 0;
        for (int k = 0; k < 2 * N2; ++k) {
            const T x = slam[2 * fl * N2 + k];
            if (x > s) {
                s = x;
                arg = k;
            }
        }
        if (tape_mode == TAPE_RECORD && b == 0) tape[f] = int16_t(arg);
    }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const T F = rusanov(FL[v], FR[v], QL[v], QR[v], s);
        if constexpr (B32) {
            const int pb = int(nc * N2 * int64_t(sizeof(T)));
            buf_st(buf_view(fside + (int64_t(sL) * NV + v) * nc * N2, pb), unsigned(cL * N2 + b) * unsigned(sizeof(T)), F);
            buf_st(buf_view(fside + (int64_t(sR) * NV + v) * nc * N2, pb), unsigned(cR * N2 + b) * unsigned(sizeof(T)), F);
        } else {
            fside[(int64_t(sL * NV + v) * nc + cL) * N2 + b] = F;
            fside[(int64_t(sR * NV + v) * nc + cR) * N2 + b] = F;
        }
    }
}

// ---------------------------------------------------------------------------
// Hanging faces: virtual-cell data by interpolation, Rusanov on the child face
// ---------------------------------------------------------------------------

template <typename T, int N>
__global__ void __launch_bounds__(FaceCfg<N>::THREADS)
k_hang(const T *__restrict__ traces, T *__restrict__ fside, const HangDev *__restrict__ hang,
       int64_t nh, int64_t nc, const double *__restrict__ ptab, double gamma,
       int *__restrict__ status)
{
    constexpr int N2 = N * N, FPB = FaceCfg<N>::FPB;
    __shared__ T smax[FPB * N2];
    const int tid = threadIdx.x;
    const int fl = tid / N2, b = tid % N2;
    const int64_t h = int64_t(blockIdx.x) * FPB + fl;
    const bool lane_ok = tid < FPB * N2;
    const bool active = lane_ok && h < nh;
    const T g = T(gamma), gm1 = T(gamma - 1.0);
    T Qf[NV], Ff[NV], Qv[NV], Fv[NV];
    T lam = T(0);
    int64_t fine = 0;
    int sf = 0, d = 0, fine_minus = 0;
    if (active) {
        const HangDev H = hang[h];
        fine = H.fine;
        d = H.d;
        fine_minus = H.fine_minus;
        sf = 2 * d + (fine_minus ? 1 : 0);
        const int sc = 2 * d + (fine_minus ? 0 : 1);
        const double *P1 = ptab + (transfer_base(H.dl) + H.s1) * 2 * N2;  // P block
        const double *P2 = ptab + (transfer_base(H.dl) + H.s2) * 2 * N2;
        const int k1 = b % N, k2 = b / N;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Qf[v] = traces[((int64_t(sf * 2 + 0) * NV + v) * nc + fine) * N2 + b];
            Ff[v] = traces[((int64_t(sf * 2 + 1) * NV + v) * nc + fine) * N2 + b];
            const T *cq = traces + ((int64_t(sc * 2 + 0) * NV + v) * nc + H.coarse) * N2;
            const T *cf = traces + ((int64_t(sc * 2 + 1) * NV + v) * nc + H.coarse) * N2;
            T sq = T(0), sfl = T(0);
#pragma unroll
            for (int e2 = 0; e2 < N; ++e2) {
                T rq = T(0), rf = T(0);
#pragma unroll
                for (int e1 = 0; e1 < N; ++e1) {
                    const T p1 = T(P1[k1 * N + e1]);
                    rq += p1 * cq[e1 + N * e2];
                    rf += p1 * cf[e1 + N * e2];
                }
                const T p2 = T(P2[k2 * N + e2]);
                sq += p2 * rq;
                sfl += p2 * rf;
            }
            Qv[v] = sq;
            Fv[v] = sfl;
        }
        bool b1, b2;
        lam = fmax(wave_speed(g, gm1, Qf, d, b1), wave_speed(g, gm1, Qv, d, b2));
        if (b1 || b2) *status = 1;
    }
    if (lane_ok) smax[tid] = lam;
    __syncthreads();
    if (!active) return;
    T s = T(0);
    for (int k = 0; k < N2; ++k) s = fmax(s, smax[fl * N2 + k]);
    const T *QL = fine_minus ? Qf : Qv, *FL = fine_minus ? Ff : Fv;
    const T *QR = fine_minus ? Qv : Qf, *FR = fine_minus ? Fv : Ff;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const T F = rusanov(FL[v], FR[v], QL[v], QR[v], s);
        fside[(int64_t(sf * NV + v) * nc + fine) * N2 + b] = F;
    }
}

// Restriction into coarse sides: F_C[k] = sum_children (R1 x R2) F_child,
// children in increasing fine-cell order, FP64 accumulation.
template <typename T, int N>
__global__ void __launch_bounds__(256)
k_restrict(T *__restrict__ fside, const HangDev *__restrict__ hang, const int32_t *__restrict__ ccell,
           const int8_t *__restrict__ cside, const int32_t *__restrict__ cptr,
           const int32_t *__restrict__ cchild, int64_t ncs, int64_t nc, const double *__restrict__ ptab)
{
    constexpr int N2 = N * N;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ncs * N2) return;
    const int64_t i = t / N2;
    const int k = int(t % N2), k1 = k % N, k2 = k / N;
    const int64_t C = ccell[i];
    const int s = cside[i];
    double acc[NV] = {0, 0, 0, 0, 0};
    for (int q = cptr[i]; q < cptr[i + 1]; ++q) {
        const HangDev H = hang[cchild[q]];
        const int sf = 2 * H.d + (H.fine_minus ? 1 : 0);
        const double *R1 = ptab + (transfer_base(H.dl) + H.s1) * 2 * N2 + N2;  // R block
        const double *R2 = ptab + (transfer_base(H.dl) + H.s2) * 2 * N2 + N2;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const T *src = fside + (int64_t(sf * NV + v) * nc + H.fine) * N2;
            double sum = 0.0;
#pragma unroll
            for (int e2 = 0; e2 < N; ++e2) {
                double r = 0.0;
#pragma unroll
                for (int e1 = 0; e1 < N; ++e1) r += R1[k1 * N + e1] * double(src[e1 + N * e2]);
                sum += R2[k2 * N + e2] * r;
            }
            acc[v] += sum;
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) fside[(int64_t(s * NV + v) * nc + C) * N2 + k] = T(acc[v]);
}

// ---------------------------------------------------------------------------
// Corrector
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_max(double x, double *sh);

// Sum over the axes of (|u_d| + c)/dx_d at one node; +inf (and the status
// flag) for a non-physical state.  Shared by the CFL kernels and the fused
// corrector epilogue, so both give the same bits.
__device__ __forceinline__ double cfl_rate(double gamma, const double q[NV], const Geo &geo, int lev,
                                           int *__restrict__ status)
{
    const double gm1 = gamma - 1.0;
    bool bad = false, b2;
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s += wave_speed(gamma, gm1, q, d, b2) * geo.inv_dx[lev][d];
        bad = bad || b2;
    }
    if (bad) {
        *status = 1;
        s = INFINITY;
    }
    return s;
}

// FUSE: also reduce the CFL rate of the new state to one maximum per block
// (partial[blockIdx.x]), which the next step's k_cfl_final consumes.
template <typename T, int N, bool FUSE>
__global__ void __launch_bounds__(256)
k_corrector(const double *__restrict__ ustar, const T *__restrict__ fside, const double *__restrict__ dt_dev,
            double *__restrict__ uout, int64_t nc, const int8_t *__restrict__ level, Geo geo, double gamma,
            double *__restrict__ partial, int *__restrict__ status, int64_t c0, int64_t c1)
{
    constexpr int N2 = N * N, N3 = N2 * N;
    const DevBasis &B = c_basis[N];
    const double dt = dt_dev[0];
    double rate = 0.0;
    const int64_t total = c1 * N3;
    // grid-stride over the nodes of cells c0 .. c1-1 (the grid is capped so
    // that the fused CFL leaves few block maxima)
    for (int64_t t = c0 * N3 + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t c = t / N3;
        const int a = int(t % N3), a0 = a % N, a1 = (a / N) % N, a2 = a / N2;
        const int lev = level ? level[c] : 0;
        const double sx = dt * geo.inv_dx[lev][0] * B.winv[a0];
        const double sy = dt * geo.inv_dx[lev][1] * B.winv[a1];
        const double sz = dt * geo.inv_dx[lev][2] * B.winv[a2];
        const int bx = a1 + N * a2, by = a0 + N * a2, bz = a0 + N * a1;
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double fxm = fside[(int64_t(0 * NV + v) * nc + c) * N2 + bx];
            const double fxp = fside[(int64_t(1 * NV + v) * nc + c) * N2 + bx];
            const double fym = fside[(int64_t(2 * NV + v) * nc + c) * N2 + by];
            const double fyp = fside[(int64_t(3 * NV + v) * nc + c) * N2 + by];
            const double fzm = fside[(int64_t(4 * NV + v) * nc + c) * N2 + bz];
            const double fzp = fside[(int64_t(5 * NV + v) * nc + c) * N2 + bz];
            const double s = sx * (B.R[a0] * fxp - B.L[a0] * fxm) + sy * (B.R[a1] * fyp - B.L[a1] * fym) +
                             sz * (B.R[a2] * fzp - B.L[a2] * fzm);
            const int64_t o = (int64_t(v) * nc + c) * N3 + a;
            q[v] = ustar[o] - s;
            uout[o] = q[v];
        }
        if (FUSE) rate = fmax(rate, cfl_rate(gamma, q, geo, lev, status));
    }
    if (FUSE) {
        __shared__ double sh[4];
        rate = block_max(rate, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = rate;
    }
}

// ---------------------------------------------------------------------------
// Time step size
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_max(double x, double *sh)
{
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sh[0];
        for (int i = 1; i < int(blockDim.x >> 6); ++i) m = fmax(m, sh[i]);
        sh[0] = m;
    }
    __syncthreads();
    return sh[0];
}

// N = 4: one wavefront per cell (lane = node), so the cell index is uniform
// and every address is a scalar base plus a 32-bit lane offset.  Grid-stride
// over cells with the same block count as the generic form.
template <typename T, bool FUSE>
__global__ void __launch_bounds__(256)
k_corrector4(const double *__restrict__ ustar, const T *__restrict__ fside, const double *__restrict__ dt_dev,
             double *__restrict__ uout, int64_t nc, const int8_t *__restrict__ level, Geo geo, double gamma,
             double *__restrict__ partial, int *__restrict__ status, int64_t c0, int64_t c1)
{
    constexpr int N2 = 16, N3 = 64;
    const int l = threadIdx.x & 63;
    const int a0 = l & 3, a1 = (l >> 2) & 3, a2 = l >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const unsigned lu = unsigned(l) * unsigned(sizeof(double));
    const unsigned bx = unsigned(a1 + 4 * a2) * unsigned(sizeof(T)), by = unsigned(a0 + 4 * a2) * unsigned(sizeof(T)),
                   bz = unsigned(a0 + 4 * a1) * unsigned(sizeof(T));
    const double *Wl = lane_at(static_cast<const double *>(c_corr4), unsigned(l) * unsigned(6 * sizeof(double)));
    const double Rx = Wl[0], Ry = Wl[1], Rz = Wl[2], Lx = Wl[3], Ly = Wl[4], Lz = Wl[5];
    const double dt = dt_dev[0];
    double rate = 0.0;
    for (int64_t c = c0 + int64_t(blockIdx.x) * (blockDim.x >> 6) + wave; c < c1;
         c += int64_t(gridDim.x) * (blockDim.x >> 6)) {
        const int lev = level ? __builtin_amdgcn_readfirstlane(int(level[c])) : 0;
        const double cx = dt * geo.inv_dx[lev][0], cy = dt * geo.inv_dx[lev][1], cz = dt * geo.inv_dx[lev][2];
        // every load of the cell first (the stores below could alias them for
        // all the compiler knows, which would serialise the variables)
        T f[NV][6];
        double us[NV], q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
#pragma unroll
            for (int side = 0; side < 6; ++side)
                f[v][side] = buf_ld(buf_view(fside + ((int64_t(side) * NV + v) * nc + c) * N2, N2 * sizeof(T)),
                                    side < 2 ? bx : (side < 4 ? by : bz), T(0));
            us[v] = buf_ld(buf_view(ustar + (int64_t(v) * nc + c) * N3, N3 * sizeof(double)), lu, 0.0);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            // explicit fused operations: the same bits in every variant of
            // the kernel (the compiler may contract a plain expression
            // differently in the fused-CFL variant)
            const double tx = fma(Rx, double(f[v][1]), -(Lx * double(f[v][0])));
            const double ty = fma(Ry, double(f[v][3]), -(Ly * double(f[v][2])));
            const double tz = fma(Rz, double(f[v][5]), -(Lz * double(f[v][4])));
            const double sv = fma(cx, tx, fma(cy, ty, cz * tz));
            q[v] = us[v] - sv;
            buf_st(buf_view(uout + (int64_t(v) * nc + c) * N3, N3 * sizeof(double)), lu, q[v]);
        }
        if (FUSE) rate = fmax(rate, cfl_rate(gamma, q, geo, lev, status));
    }
    if (FUSE) {
        __shared__ double sh[4];
        rate = block_max(rate, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = rate;
    }
}

// Cells of an nx x ny x nz mesh visited in tiles of tx x ty x tz (tx a
// multiple of 4, so the four cells of a block are neighbours along x), x
// fastest inside a tile and over the tiles: the cells in flight at one time
// form about a tile, and most face neighbours along all three axes are read
// while the cell that owns them is also being read.  Workgroups go to the 8
// XCDs in turn (workgroup i to XCD i mod 8), each with its own L2, and each
// XCD walks one contiguous eighth of the blocks of four slots.
struct TileWalk {
    int64_t nx, ny, nz, tx, ty, tz, ntx, nty, tsz, ub, ue, stride, first;
    __device__ TileWalk(int nx_, int ny_, int nz_, int tx_, int ty_, int tz_)
        : nx(nx_), ny(ny_), nz(nz_), tx(tx_), ty(ty_), tz(tz_)
    {
        ntx = (nx + tx - 1) / tx;
        nty = (ny + ty - 1) / ty;
        const int64_t ntz = (nz + tz - 1) / tz;
        tsz = tx * ty * tz;
        const int64_t units = ntx * nty * ntz * tsz / 4;
        const bool by_xcd = gridDim.x % 8 == 0;
        const int xcd = by_xcd ? int(blockIdx.x % 8) : 0;
        stride = by_xcd ? gridDim.x / 8 : gridDim.x;
        ub = by_xcd ? units * xcd / 8 : 0;
        ue = by_xcd ? units * (xcd + 1) / 8 : units;
        first = ub + (by_xcd ? blockIdx.x / 8 : blockIdx.x);
    }
    // slot `wave` of block-unit `unit`: its cell and coordinates, false past the mesh's edge
    __device__ bool cell(int64_t unit, int wave, int64_t &c, int64_t ijk[3]) const
    {
        const int64_t slot = unit * 4 + wave, t = slot / tsz, o = slot % tsz;
        ijk[0] = (t % ntx) * tx + o % tx;
        ijk[1] = ((t / ntx) % nty) * ty + (o / tx) % ty;
        ijk[2] = (t / (ntx * nty)) * tz + o / (tx * ty);
        const bool ok = ijk[0] < nx && ijk[1] < ny && ijk[2] < nz;
        c = ok ? ijk[0] + nx * (ijk[1] + ny * ijk[2]) : 0;
        return ok;
    }
};

// The Riemann problems of a cell's six faces and the cell's corrector in one
// pass, for one uniform periodic instance at N = 4 (cells in (k, j, i) order,
// one wavefront per cell, four cells per block, cells visited tile by tile).  Rows of 16 lanes take one
// face each: faces 0-3 in a first round, 4-5 in a second (lanes 32-63 idle);
// lane b of a row is face node b, reads its own side's and the neighbour's
// projections, and the row's maximum is the face speed.  Both cells of a face
// solve it, with the same operands in the same order as k_riemann, so the
// flux is bit for bit the one k_riemann stores; the six faces' fluxes go
// through the block's LDS to the nodes, and the update is that of
// k_corrector4.  No face-flux array is written or read.
template <typename T, bool FUSE>
__global__ void __launch_bounds__(256)
k_face_corrector4(const double *__restrict__ ustar, const T *__restrict__ traces, const double *__restrict__ dt_dev,
                  double *__restrict__ uout, int64_t nc, int nx, int ny, int nz, int tx, int ty, int tz, Geo geo,
                  double gamma, double *__restrict__ partial, int *__restrict__ status)
{
    constexpr int N2 = 16, N3 = 64;
    __shared__ T fs[4 * 6 * NV * N2];
    const int l = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    T *fw = fs + wave * (6 * NV * N2);
    const unsigned lu = unsigned(l) * unsigned(sizeof(double));
    const int bxi = (l >> 2) & 15, byi = (l & 3) + 4 * (l >> 4), bzi = l & 15;
    const double *Wl = lane_at(static_cast<const double *>(c_corr4), unsigned(l) * unsigned(6 * sizeof(double)));
    const double Rx = Wl[0], Ry = Wl[1], Rz = Wl[2], Lx = Wl[3], Ly = Wl[4], Lz = Wl[5];
    const T g = T(gamma), gm1 = T(gamma - 1.0);
    const int64_t nxy = int64_t(nx) * ny, plane = nc * N2;
    const int b = l & 15;
    const double dt = dt_dev[0];
    const double cx = dt * geo.inv_dx[0][0], cy = dt * geo.inv_dx[0][1], cz = dt * geo.inv_dx[0][2];
    double rate = 0.0;
    const TileWalk walk(nx, ny, nz, tx, ty, tz);  // slots past the mesh's edge are idle wavefronts
    for (int64_t unit = walk.first; unit < walk.ue; unit += walk.stride) {
        int64_t c, ijk[3];
        const bool cell_ok = walk.cell(unit, wave, c, ijk);  // uniform per wavefront
        if (cell_ok) {
            const int64_t ext[3] = {nx, ny, nz}, str[3] = {1, nx, nxy};
#pragma unroll 1
            for (int r = 0; r < 2; ++r) {  // one round's loads in flight: bounds the registers
                const int side = 4 * r + (l >> 4);
                const bool face_ok = side < 6;
                const int sd = face_ok ? side : 0, d = sd >> 1, plus = sd & 1;
                // the neighbour across this side (periodic)
                const int64_t q = ijk[d] + (plus ? 1 : -1);
                const int64_t qn = q < 0 ? q + ext[d] : (q >= ext[d] ? q - ext[d] : q);
                const int64_t n = c + (qn - ijk[d]) * str[d];
                // minus cell's plus side on the left, plus cell's minus side on the right
                const int64_t cL = plus ? c : n, cR = plus ? n : c;
                const int sL = 2 * d + 1, sR = 2 * d;
                T QL[NV], FL[NV], QR[NV], FR[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    QL[v] = traces[(int64_t(sL * 2 + 0) * NV + v) * plane + cL * N2 + b];
                    FL[v] = traces[(int64_t(sL * 2 + 1) * NV + v) * plane + cL * N2 + b];
                    QR[v] = traces[(int64_t(sR * 2 + 0) * NV + v) * plane + cR * N2 + b];
                    FR[v] = traces[(int64_t(sR * 2 + 1) * NV + v) * plane + cR * N2 + b];
                }
                bool badL, badR;
                const T lL = wave_speed(g, gm1, QL, d, badL);
                const T lR = wave_speed(g, gm1, QR, d, badR);
                if (face_ok && (badL || badR)) *status = 1;
                const T sf = row_max16(lL > lR ? lL : lR);
                if (face_ok) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) fw[(sd * NV + v) * N2 + b] = rusanov(FL[v], FR[v], QL[v], QR[v], sf);
                }
            }
        }
        __syncthreads();
        if (cell_ok) {
            double q[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double f0 = double(fw[(0 * NV + v) * N2 + bxi]), f1 = double(fw[(1 * NV + v) * N2 + bxi]);
                const double f2 = double(fw[(2 * NV + v) * N2 + byi]), f3 = double(fw[(3 * NV + v) * N2 + byi]);
                const double f4 = double(fw[(4 * NV + v) * N2 + bzi]), f5 = double(fw[(5 * NV + v) * N2 + bzi]);
                const double us = buf_ld(buf_view(ustar + (int64_t(v) * nc + c) * N3, N3 * sizeof(double)), lu, 0.0);
                // the update of k_corrector4, operation for operation
                const double tx = fma(Rx, f1, -(Lx * f0));
                const double ty = fma(Ry, f3, -(Ly * f2));
                const double tz = fma(Rz, f5, -(Lz * f4));
                const double sv = fma(cx, tx, fma(cy, ty, cz * tz));
                q[v] = us - sv;
                buf_st(buf_view(uout + (int64_t(v) * nc + c) * N3, N3 * sizeof(double)), lu, q[v]);
            }
            if (FUSE) rate = fmax(rate, cfl_rate(gamma, q, geo, 0, status));
        }
        __syncthreads();  // the next cells overwrite the fluxes
    }
    if (FUSE) {
        __shared__ double sh[4];
        rate = block_max(rate, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = rate;
    }
}

// N >= 5: a cell spans W = ceil(N^3 / 64) wavefronts (node a = 64 w + lane),
// so the cell index is again uniform per wavefront and all accesses are
// buffer accesses from scalar bases.  Lanes past N^3 use out-of-range offsets
// (loads read zero, stores are dropped) and stay out of the CFL maximum.
template <int N> struct CorrW {
    static constexpr int W = (N * N * N + 63) / 64;
    static constexpr int CPB = W >= 4 ? 1 : 4 / W;  // cells per block
    static constexpr int THREADS = 64 * W * CPB;
};

template <typename T, int N, bool FUSE>
__global__ void __launch_bounds__(CorrW<N>::THREADS)
k_correctorW(const double *__restrict__ ustar, const T *__restrict__ fside, const double *__restrict__ dt_dev,
             double *__restrict__ uout, int64_t nc, const int8_t *__restrict__ level, Geo geo, double gamma,
             double *__restrict__ partial, int *__restrict__ status, int64_t c0, int64_t c1)
{
    constexpr int N2 = N * N, N3 = N2 * N, W = CorrW<N>::W, CPB = CorrW<N>::CPB;
    constexpr unsigned OUT = 0x80000000u;
    const DevBasis &B = c_basis[N];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int a = (wave % W) * 64 + lane, cl = wave / W;
    const bool node_ok = a < N3;
    const int a0 = node_ok ? a % N : 0, a1 = node_ok ? (a / N) % N : 0, a2 = node_ok ? a / N2 : 0;
    const unsigned lu = node_ok ? unsigned(a) * unsigned(sizeof(double)) : OUT;
    const unsigned bx = node_ok ? unsigned(a1 + N * a2) * unsigned(sizeof(T)) : OUT;
    const unsigned by = node_ok ? unsigned(a0 + N * a2) * unsigned(sizeof(T)) : OUT;
    const unsigned bz = node_ok ? unsigned(a0 + N * a1) * unsigned(sizeof(T)) : OUT;
    const double Rx = B.R[a0] * B.winv[a0], Ry = B.R[a1] * B.winv[a1], Rz = B.R[a2] * B.winv[a2];
    const double Lx = B.L[a0] * B.winv[a0], Ly = B.L[a1] * B.winv[a1], Lz = B.L[a2] * B.winv[a2];
    const double dt = dt_dev[0];
    double rate = 0.0;
    for (int64_t c = c0 + int64_t(blockIdx.x) * CPB + cl; c < c1; c += int64_t(gridDim.x) * CPB) {
        const int lev = level ? __builtin_amdgcn_readfirstlane(int(level[c])) : 0;
        const double cx = dt * geo.inv_dx[lev][0], cy = dt * geo.inv_dx[lev][1], cz = dt * geo.inv_dx[lev][2];
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            auto face = [&](int side, unsigned off) {
                return double(buf_ld(buf_view(fside + ((int64_t(side) * NV + v) * nc + c) * N2, N2 * sizeof(T)), off,
                                     T(0)));
            };
            const double fxm = face(0, bx), fxp = face(1, bx);
            const double fym = face(2, by), fyp = face(3, by);
            const double fzm = face(4, bz), fzp = face(5, bz);
            const double sv = cx * (Rx * fxp - Lx * fxm) + cy * (Ry * fyp - Ly * fym) + cz * (Rz * fzp - Lz * fzm);
            const int64_t o = (int64_t(v) * nc + c) * N3;
            q[v] = buf_ld(buf_view(ustar + o, N3 * sizeof(double)), lu, 0.0) - sv;
            buf_st(buf_view(uout + o, N3 * sizeof(double)), lu, q[v]);
        }
        if (FUSE && node_ok) rate = fmax(rate, cfl_rate(gamma, q, geo, lev, status));
    }
    if (FUSE) {
        __shared__ double sh[CorrW<N>::THREADS / 64];
        rate = block_max(rate, sh);
        if (threadIdx.x == 0) partial[blockIdx.x] = rate;
    }
}

template <int N>
__global__ void __launch_bounds__(256)
k_cfl_partial(const double *__restrict__ u, int64_t nc, const int8_t *__restrict__ level, Geo geo,
              double gamma, double *__restrict__ partial, int *__restrict__ status)
{
    constexpr int N3 = N * N * N;
    __shared__ double sh[4];
    double m = 0.0;
    const int64_t total = nc * N3;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t c = t / N3;
        const int a = int(t % N3);
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = u[(int64_t(v) * nc + c) * N3 + a];
        m = fmax(m, cfl_rate(gamma, q, geo, level ? level[c] : 0, status));
    }
    m = block_max(m, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

__global__ void __launch_bounds__(1024)
k_cfl_final(const double *__restrict__ partial, int nparts, double factor, double *__restrict__ dt_out,
            double *__restrict__ hist, double t_end, double *__restrict__ clock)
{
    __shared__ double sh[16];
    double m = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmax(m, partial[i]);
    m = block_max(m, sh);
    if (threadIdx.x == 0) {
        double dt = (m > 0.0 && m < INFINITY) ? factor / m : 0.0;
        if (clock) {
            // the last step ends at t_end exactly; later steps have dt = 0
            const double rest = fmax(t_end - clock[0], 0.0);
            if (dt >= rest) {
                dt = rest;
                clock[0] = t_end;
            } else {
                clock[0] += dt;
            }
        }
        dt_out[0] = dt;
        if (hist) hist[0] = dt;
    }
}

// p[0 .. n-1] = x (a kernel rather than a memset, so that graph captures
// hold no memset node)
__global__ void __launch_bounds__(256) k_fill(double *__restrict__ p, int64_t n, double x)
{
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) p[i] = x;
}

// ---------------------------------------------------------------------------
// Node coordinates
// ---------------------------------------------------------------------------

template <int N>
__global__ void __launch_bounds__(256)
k_node_coords(double *__restrict__ xyz, const int32_t *__restrict__ ijk, const int8_t *__restrict__ level,
              int64_t nc, Geo geo, double lo0, double lo1, double lo2)
{
    constexpr int N3 = N * N * N;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nc * N3) return;
    const int64_t c = t / N3;
    const int a = int(t % N3);
    const int aa[3] = {a % N, (a / N) % N, a / (N * N)};
    const double lo[3] = {lo0, lo1, lo2};
    const int lev = level ? level[c] : 0;
    const DevBasis &B = c_basis[N];
#pragma unroll
    for (int d = 0; d < 3; ++d)
        xyz[(int64_t(d) * nc + c) * N3 + a] = lo[d] + (double(ijk[3 * c + d]) + B.xi[aa[d]]) / geo.inv_dx[lev][d];
}


// ---------------------------------------------------------------------------
// Discrete adjoint of one step at a fixed time step size (FP64, uniform
// meshes).  Forward: u* = u + V(Fbar(q)), traces = E(qbar, Fbar), F* =
// Rusanov(traces), u_next = u* - C(F*).  The kernels apply the transposes in
// reverse order: k_corrector_adj, k_riemann_adj, k_predictor_adj.
// ---------------------------------------------------------------------------

// qbar += (df_d/dq)^T fbar for the Euler flux along d at state q.
__device__ __forceinline__ void flux_vjp(double gm1, const double q[NV], int d, const double fb[NV], double qb[NV])
{
    const double inv = 1.0 / q[0];
    const double v[3] = {q[1] * inv, q[2] * inv, q[3] * inv};
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double p = gm1 * (q[4] - 0.5 * q[0] * v2);
    const double H = (q[4] + p) * inv;  // (E + p)/rho
    // partials of p
    const double dp_r = gm1 * 0.5 * v2;
    const double dp_m[3] = {-gm1 * v[0], -gm1 * v[1], -gm1 * v[2]};
    const double dp_E = gm1;
    const double vd = v[d];
    // f0 = m_d
    qb[1 + d] += fb[0];
    // f_k = m_d m_k / rho + delta_kd p
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double g = fb[1 + k];
        qb[0] += g * (-vd * v[k] + (k == d ? dp_r : 0.0));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double dm = (j == d ? v[k] : 0.0) + (j == k ? vd : 0.0) + (k == d ? dp_m[j] : 0.0);
            qb[1 + j] += g * dm;
        }
        if (k == d) qb[4] += g * dp_E;
    }
    // f4 = m_d (E + p) / rho
    const double g4 = fb[4];
    qb[0] += g4 * (-vd * H + vd * dp_r);
#pragma unroll
    for (int j = 0; j < 3; ++j) qb[1 + j] += g4 * ((j == d ? H : 0.0) + vd * dp_m[j]);
    qb[4] += g4 * vd * (1.0 + dp_E);
}

// qbar += sbar * d(|u_d| + c)/dq  (abs'(0) = 0)
__device__ __forceinline__ void speed_vjp(double gamma, const double q[NV], int d, double sbar, double qb[NV])
{
    const double gm1 = gamma - 1.0;
    const double inv = 1.0 / q[0];
    const double v[3] = {q[1] * inv, q[2] * inv, q[3] * inv};
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double p = gm1 * (q[4] - 0.5 * q[0] * v2);
    const double c = sqrt(gamma * p * inv);
    const double sg = v[d] > 0.0 ? 1.0 : (v[d] < 0.0 ? -1.0 : 0.0);
    // |v_d|
    qb[0] += sbar * (-sg * v[d] * inv);
    qb[1 + d] += sbar * sg * inv;
    // c = sqrt(gamma p / rho): dc = gamma/(2 c rho) (dp - p/rho drho)
    const double k = gamma / (2.0 * c * q[0]);
    qb[0] += sbar * k * (gm1 * 0.5 * v2 - p * inv);
#pragma unroll
    for (int j = 0; j < 3; ++j) qb[1 + j] += sbar * k * (-gm1 * v[j]);
    qb[4] += sbar * k * gm1;
}

// fbar of every cell side from the corrector: u_next = u* - sum_d s_d(a)
// [R_{a_d} F_{d+}(b) - L_{a_d} F_{d-}(b)], s_d(a) = dt/dx_d/w_{a_d}.
template <int N>
__global__ void __launch_bounds__(256)
k_corrector_adj(const double *__restrict__ ubar, double *__restrict__ fbar, const double *__restrict__ dt_dev,
                int64_t nc, const int8_t *__restrict__ level, Geo geo)
{
    constexpr int N2 = N * N, N3 = N2 * N;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= 6 * NV * nc * N2) return;
    const int b = int(t % N2);
    const int64_t c = (t / N2) % nc;
    const int sv = int(t / (N2 * nc));
    const int s = sv / NV, v = sv % NV, d = s >> 1;
    const DevBasis &B = c_basis[N];
    const double sc = dt_dev[0] * geo.inv_dx[level ? level[c] : 0][d];
    const double *E = (s & 1) ? B.R : B.L;
    const double sign = (s & 1) ? -1.0 : 1.0;
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < N; ++e)
        acc += B.winv[e] * E[e] * ubar[(int64_t(v) * nc + c) * N3 + node_from_face<N>(d, e, b)];
    fbar[t] = sign * sc * acc;
}

// The same at N = 4 with one wavefront per cell: the cell's cotangent is read
// once, coalesced (lane = node), into LDS, and the lanes form the 6 x 5 x 16
// side sums from there with the operations of k_corrector_adj (same bits).
// The thread-per-output form reads every cell once per side.
__global__ void __launch_bounds__(256)
k_corrector_adj4(const double *__restrict__ ubar, double *__restrict__ fbar, const double *__restrict__ dt_dev,
                 int64_t nc, const int8_t *__restrict__ level, Geo geo)
{
    constexpr int N = 4, N2 = 16, N3 = 64, OUT = 6 * NV * N2;
    __shared__ double ls[4][NV * N3];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int64_t c = int64_t(blockIdx.x) * 4 + wave;
    const bool ok = c < nc;  // uniform per wavefront; every wavefront reaches the barrier
    if (ok)
#pragma unroll
        for (int v = 0; v < NV; ++v) ls[wave][v * N3 + l] = ubar[(int64_t(v) * nc + c) * N3 + l];
    __syncthreads();
    if (!ok) return;
    const DevBasis &B = c_basis[N];
    const int lev = level ? level[c] : 0;
    for (int o = l; o < OUT; o += 64) {
        const int s = o / (NV * N2), v = (o / N2) % NV, b = o % N2, d = s >> 1;
        const double sc = dt_dev[0] * geo.inv_dx[lev][d];
        const double *E = (s & 1) ? B.R : B.L;
        const double sign = (s & 1) ? -1.0 : 1.0;
        double acc = 0.0;
#pragma unroll
        for (int e = 0; e < N; ++e) acc += B.winv[e] * E[e] * ls[wave][v * N3 + node_from_face<N>(d, e, b)];
        fbar[(int64_t(s * NV + v) * nc + c) * N2 + b] = sign * sc * acc;
    }
}

// Transpose of the Rusanov solve on the conforming faces of one axis: writes
// the adjoint of both cells' face projections (state and normal flux).
template <int N>
__global__ void __launch_bounds__(FaceCfg<N>::THREADS)
k_riemann_adj(const double *__restrict__ traces, const double *__restrict__ fbar, double *__restrict__ tbar,
              const int32_t *__restrict__ fm, const int32_t *__restrict__ fp, int64_t nf, int d, int64_t nc,
              double gamma)
{
    constexpr int N2 = N * N, FPB = FaceCfg<N>::FPB;
    __shared__ double lam[FPB * N2 * 2];
    __shared__ double part[FPB * N2];
    const int tid = threadIdx.x;
    const int fl = tid / N2, b = tid % N2;
    const int64_t f = int64_t(blockIdx.x) * FPB + fl;
    const bool lane_ok = tid < FPB * N2;
    const bool active = lane_ok && f < nf;
    const double gm1 = gamma - 1.0;
    const int sL = 2 * d + 1, sR = 2 * d;
    double QL[NV], FL[NV], QR[NV], FR[NV], Fb[NV];
    int64_t cL = 0, cR = 0;
    double lL = 0.0, lR = 0.0, sb = 0.0;
    bool dummy;
    if (active) {
        cL = fm[f];
        cR = fp[f];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            QL[v] = traces[((int64_t(sL * 2 + 0) * NV + v) * nc + cL) * N2 + b];
            FL[v] = traces[((int64_t(sL * 2 + 1) * NV + v) * nc + cL) * N2 + b];
            QR[v] = traces[((int64_t(sR * 2 + 0) * NV + v) * nc + cR) * N2 + b];
            FR[v] = traces[((int64_t(sR * 2 + 1) * NV + v) * nc + cR) * N2 + b];
            Fb[v] = fbar[(int64_t(sL * NV + v) * nc + cL) * N2 + b] + fbar[(int64_t(sR * NV + v) * nc + cR) * N2 + b];
            sb += -0.5 * (QR[v] - QL[v]) * Fb[v];
        }
        lL = wave_speed(gamma, gm1, QL, d, dummy);
        lR = wave_speed(gamma, gm1, QR, d, dummy);
    }
    if (lane_ok) {
        lam[2 * tid] = lL;
        lam[2 * tid + 1] = lR;
        part[tid] = sb;
    }
    __syncthreads();
    if (!active) return;
    // s and its (lowest-index) argmax over (node, side), and sbar of the face
    double s = -1.0, sbar = 0.0;
    int arg = 0;
    for (int k = 0; k < 2 * N2; ++k) {
        const double x = lam[2 * fl * N2 + k];
        if (x > s) {
            s = x;
            arg = k;
        }
    }
    for (int k = 0; k < N2; ++k) sbar += part[fl * N2 + k];
    double QLb[NV], QRb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        QLb[v] = 0.5 * s * Fb[v];
        QRb[v] = -0.5 * s * Fb[v];
    }
    if (arg / 2 == b) {
        if (arg % 2 == 0) speed_vjp(gamma, QL, d, sbar, QLb);
        else speed_vjp(gamma, QR, d, sbar, QRb);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        tbar[((int64_t(sL * 2 + 0) * NV + v) * nc + cL) * N2 + b] = QLb[v];
        tbar[((int64_t(sL * 2 + 1) * NV + v) * nc + cL) * N2 + b] = 0.5 * Fb[v];
        tbar[((int64_t(sR * 2 + 0) * NV + v) * nc + cR) * N2 + b] = QRb[v];
        tbar[((int64_t(sR * 2 + 1) * NV + v) * nc + cR) * N2 + b] = 0.5 * Fb[v];
    }
}

// Transpose of the restriction (coarse side = sum over its child faces of
// (R1 x R2) applied to the fine side's flux): the fine side of every hanging
// child face also receives (R1 x R2)^T of its coarse side's adjoint.  Every
// fine side belongs to one hanging record, so each lane owns its output.
template <int N>
__global__ void __launch_bounds__(256)
k_restrict_adj(double *__restrict__ fbar, const HangDev *__restrict__ hang, int64_t nh, int64_t nc,
               const double *__restrict__ ptab)
{
    constexpr int N2 = N * N;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nh * N2) return;
    const int64_t h = t / N2;
    const int e = int(t % N2), e1 = e % N, e2 = e / N;
    const HangDev H = hang[h];
    const int sf = 2 * H.d + (H.fine_minus ? 1 : 0), sc = 2 * H.d + (H.fine_minus ? 0 : 1);
    const double *R1 = ptab + (transfer_base(H.dl) + H.s1) * 2 * N2 + N2;
    const double *R2 = ptab + (transfer_base(H.dl) + H.s2) * 2 * N2 + N2;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double *cb = fbar + (int64_t(sc * NV + v) * nc + H.coarse) * N2;
        double sum = 0.0;
#pragma unroll
        for (int k2 = 0; k2 < N; ++k2) {
            double r = 0.0;
#pragma unroll
            for (int k1 = 0; k1 < N; ++k1) r += R1[k1 * N + e1] * cb[k1 + N * k2];
            sum += R2[k2 * N + e2] * r;
        }
        fbar[(int64_t(sf * NV + v) * nc + H.fine) * N2 + e] += sum;
    }
}

// Transpose of the Rusanov solve on hanging child faces between the fine
// cell's projection and the coarse projection interpolated to the child face
// (virtual cell).  The fine side's adjoint goes to tbar; the virtual side's
// adjoint (state and normal flux) goes to vbar [nh][2][5][N^2], from which
// k_prolong_adj gathers the coarse side.  The face speed takes the
// subgradient at its first maximiser in (node, minus side first) order.
template <int N>
__global__ void __launch_bounds__(FaceCfg<N>::THREADS)
k_hang_adj(const double *__restrict__ traces, const double *__restrict__ fbar, double *__restrict__ tbar,
           double *__restrict__ vbar, const HangDev *__restrict__ hang, int64_t nh, int64_t nc,
           const double *__restrict__ ptab, double gamma)
{
    constexpr int N2 = N * N, FPB = FaceCfg<N>::FPB;
    __shared__ double lam[FPB * N2 * 2];
    __shared__ double part[FPB * N2];
    const int tid = threadIdx.x;
    const int fl = tid / N2, b = tid % N2;
    const int64_t h = int64_t(blockIdx.x) * FPB + fl;
    const bool lane_ok = tid < FPB * N2;
    const bool active = lane_ok && h < nh;
    const double gm1 = gamma - 1.0;
    double Qf[NV], Ff[NV], Qv[NV], Fv[NV], Fb[NV];
    HangDev H{};
    int sf = 0;
    double lL = 0.0, lR = 0.0, sb = 0.0;
    bool dummy;
    if (active) {
        H = hang[h];
        sf = 2 * H.d + (H.fine_minus ? 1 : 0);
        const int sc = 2 * H.d + (H.fine_minus ? 0 : 1);
        const double *P1 = ptab + (transfer_base(H.dl) + H.s1) * 2 * N2;
        const double *P2 = ptab + (transfer_base(H.dl) + H.s2) * 2 * N2;
        const int k1 = b % N, k2 = b / N;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Qf[v] = traces[((int64_t(sf * 2 + 0) * NV + v) * nc + H.fine) * N2 + b];
            Ff[v] = traces[((int64_t(sf * 2 + 1) * NV + v) * nc + H.fine) * N2 + b];
            const double *cq = traces + ((int64_t(sc * 2 + 0) * NV + v) * nc + H.coarse) * N2;
            const double *cf = traces + ((int64_t(sc * 2 + 1) * NV + v) * nc + H.coarse) * N2;
            double sq = 0.0, sfl = 0.0;
#pragma unroll
            for (int e2 = 0; e2 < N; ++e2) {
                double rq = 0.0, rf = 0.0;
#pragma unroll
                for (int e1 = 0; e1 < N; ++e1) {
                    rq += P1[k1 * N + e1] * cq[e1 + N * e2];
                    rf += P1[k1 * N + e1] * cf[e1 + N * e2];
                }
                sq += P2[k2 * N + e2] * rq;
                sfl += P2[k2 * N + e2] * rf;
            }
            Qv[v] = sq;
            Fv[v] = sfl;
            Fb[v] = fbar[(int64_t(sf * NV + v) * nc + H.fine) * N2 + b];
        }
        const double *QL = H.fine_minus ? Qf : Qv, *QR = H.fine_minus ? Qv : Qf;
#pragma unroll
        for (int v = 0; v < NV; ++v) sb += -0.5 * (QR[v] - QL[v]) * Fb[v];
        lL = wave_speed(gamma, gm1, QL, H.d, dummy);
        lR = wave_speed(gamma, gm1, QR, H.d, dummy);
    }
    if (lane_ok) {
        lam[2 * tid] = lL;
        lam[2 * tid + 1] = lR;
        part[tid] = sb;
    }
    __syncthreads();
    if (!active) return;
    double s = -1.0, sbar = 0.0;
    int arg = 0;
    for (int k = 0; k < 2 * N2; ++k) {
        const double x = lam[2 * fl * N2 + k];
        if (x > s) {
            s = x;
            arg = k;
        }
    }
    for (int k = 0; k < N2; ++k) sbar += part[fl * N2 + k];
    double QLb[NV], QRb[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        QLb[v] = 0.5 * s * Fb[v];
        QRb[v] = -0.5 * s * Fb[v];
    }
    if (arg / 2 == b) {
        if (arg % 2 == 0) speed_vjp(gamma, H.fine_minus ? Qf : Qv, H.d, sbar, QLb);
        else speed_vjp(gamma, H.fine_minus ? Qv : Qf, H.d, sbar, QRb);
    }
    const double *Qfb = H.fine_minus ? QLb : QRb, *Qvb = H.fine_minus ? QRb : QLb;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        tbar[((int64_t(sf * 2 + 0) * NV + v) * nc + H.fine) * N2 + b] = Qfb[v];
        tbar[((int64_t(sf * 2 + 1) * NV + v) * nc + H.fine) * N2 + b] = 0.5 * Fb[v];
        vbar[((h * 2 + 0) * NV + v) * N2 + b] = Qvb[v];
        vbar[((h * 2 + 1) * NV + v) * N2 + b] = 0.5 * Fb[v];
    }
}

// Transpose of the interpolation to virtual cells: every coarse side with
// hanging children gets sum over its children of (P1 x P2)^T applied to the
// virtual side's adjoint, children in the restriction lists' fixed order.
template <int N>
__global__ void __launch_bounds__(256)
k_prolong_adj(double *__restrict__ tbar, const double *__restrict__ vbar, const HangDev *__restrict__ hang,
              const int32_t *__restrict__ ccell, const int8_t *__restrict__ cside, const int32_t *__restrict__ cptr,
              const int32_t *__restrict__ cchild, int64_t ncs, int64_t nc, const double *__restrict__ ptab)
{
    constexpr int N2 = N * N;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ncs * N2) return;
    const int64_t i = t / N2;
    const int e = int(t % N2), e1 = e % N, e2 = e / N;
    const int64_t C = ccell[i];
    const int sc = cside[i];
    double acc[2][NV] = {{0, 0, 0, 0, 0}, {0, 0, 0, 0, 0}};
    for (int q = cptr[i]; q < cptr[i + 1]; ++q) {
        const int64_t h = cchild[q];
        const HangDev H = hang[h];
        const double *P1 = ptab + (transfer_base(H.dl) + H.s1) * 2 * N2;
        const double *P2 = ptab + (transfer_base(H.dl) + H.s2) * 2 * N2;
#pragma unroll
        for (int arr = 0; arr < 2; ++arr)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double *src = vbar + ((h * 2 + arr) * NV + v) * N2;
                double sum = 0.0;
#pragma unroll
                for (int k2 = 0; k2 < N; ++k2) {
                    double r = 0.0;
#pragma unroll
                    for (int k1 = 0; k1 < N; ++k1) r += P1[k1 * N + e1] * src[k1 + N * k2];
                    sum += P2[k2 * N + e2] * r;
                }
                acc[arr][v] += sum;
            }
    }
#pragma unroll
    for (int arr = 0; arr < 2; ++arr)
#pragma unroll
        for (int v = 0; v < NV; ++v) tbar[((int64_t(sc * 2 + arr) * NV + v) * nc + C) * N2 + e] = acc[arr][v];
}

// Transpose of the predictor (Picard iterations, time averages, volume term,
// face projections).  One lane per node as in the forward kernel; iterates
// come from the forward run (iters, slots 0..npic-1 = iterates 1..npic).
template <int N, int CPB>
__global__ void __launch_bounds__(round64(CPB * N * N * N))
k_predictor_adj(const double *__restrict__ u, const double *__restrict__ iters, const double *__restrict__ ubar_next,
                const double *__restrict__ tbar, const double *__restrict__ dt_dev, double *__restrict__ ubar,
                int64_t nc, const int8_t *__restrict__ level, Geo geo, double gamma, int npic)
{
    constexpr int N2 = N * N, N3 = N2 * N, NT = CPB * N3;
    // per cell: the adjoint divergence inputs Gb_j of all N time nodes
    __shared__ double lds[CPB * N * NV * N3];
    const DevBasis &B = c_basis[N];
    const int tid = threadIdx.x;
    const int cl = tid / N3, a = tid % N3;
    const int64_t c = int64_t(blockIdx.x) * CPB + cl;
    const bool lane_ok = tid < NT;
    const bool active = lane_ok && c < nc;
    const int aa[3] = {a % N, (a / N) % N, a / N2};
    const int bf[3] = {aa[1] + N * aa[2], aa[0] + N * aa[2], aa[0] + N * aa[1]};
    const double dt = dt_dev[0];
    const int lev = level && active ? level[c] : 0;
    const double cd[3] = {dt * geo.inv_dx[lev][0], dt * geo.inv_dx[lev][1], dt * geo.inv_dx[lev][2]};
    const double gm1 = gamma - 1.0;
    double *my = lds + (lane_ok ? cl : 0) * N * NV * N3;
    auto node_with = [&](int d, int k) {
        return d == 0 ? k + N * aa[1] + N2 * aa[2] : (d == 1 ? aa[0] + N * k + N2 * aa[2] : aa[0] + N * aa[1] + N2 * k);
    };
    auto load_q = [&](int r, int j, double q[NV]) {  // iterate r (0 = u) at time node j
#pragma unroll
        for (int v = 0; v < NV; ++v)
            q[v] = !active ? (v == 0 ? 1.0 : (v == 4 ? 2.5 : 0.0))
                 : (r == 0 ? u[(int64_t(v) * nc + c) * N3 + a]
                           : iters[(((int64_t(r - 1) * N + j) * NV + v) * nc + c) * N3 + a]);
    };

    // adjoint of u* (identity part and the volume term)
    double ub[NV], acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        ub[v] = active ? ubar_next[(int64_t(v) * nc + c) * N3 + a] : 0.0;
        acc[v] = ub[v];
    }
    if (lane_ok)
#pragma unroll
        for (int v = 0; v < NV; ++v) my[v * N3 + a] = ub[v];
    __syncthreads();
    double Fbb[3][NV], qbb[NV];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double sacc = 0.0;
#pragma unroll
            for (int k = 0; k < N; ++k) sacc += B.winv[k] * B.Kw[k * N + aa[d]] * my[v * N3 + node_with(d, k)];
            Fbb[d][v] = cd[d] * sacc;
        }
    // adjoint of the face projections
#pragma unroll
    for (int v = 0; v < NV; ++v) qbb[v] = 0.0;
    if (active) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int sm = 2 * d, sp = 2 * d + 1;
            const double Lk = B.L[aa[d]], Rk = B.R[aa[d]];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                qbb[v] += Lk * tbar[((int64_t(sm * 2 + 0) * NV + v) * nc + c) * N2 + bf[d]] +
                          Rk * tbar[((int64_t(sp * 2 + 0) * NV + v) * nc + c) * N2 + bf[d]];
                Fbb[d][v] += Lk * tbar[((int64_t(sm * 2 + 1) * NV + v) * nc + c) * N2 + bf[d]] +
                             Rk * tbar[((int64_t(sp * 2 + 1) * NV + v) * nc + c) * N2 + bf[d]];
            }
        }
    }
    // adjoint of the time averages of the final iterate
    double qbar[N][NV];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double q[NV];
        load_q(npic, j, q);
#pragma unroll
        for (int v = 0; v < NV; ++v) qbar[j][v] = B.w[j] * qbb[v];
        double fbw[NV];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
#pragma unroll
            for (int v = 0; v < NV; ++v) fbw[v] = B.w[j] * Fbb[d][v];
            flux_vjp(gm1, q, d, fbw, qbar[j]);
        }
    }
    // Picard iterations in reverse: q^(r) = u - sum_j KW[l][j] G_j(q^(r-1)).
    // Gb_j = -sum_l KW[l][j] qbar_l of every time node goes to LDS at once.
    // At r = 1 every q^(0)_j is u, so the Gb_j are summed first and one
    // transposed divergence and flux VJP serve all time nodes.
    for (int r = npic; r >= 1; --r) {
        const bool first = r == 1;
        __syncthreads();
        if (lane_ok) {
            double gs[NV] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int j = 0; j < N; ++j)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double sacc = 0.0;
#pragma unroll
                    for (int l = 0; l < N; ++l) sacc += B.KW[l * N + j] * qbar[l][v];
                    if (first)
                        gs[v] -= sacc;
                    else
                        my[(j * NV + v) * N3 + a] = -sacc;
                }
            if (first)
#pragma unroll
                for (int v = 0; v < NV; ++v) my[v * N3 + a] = gs[v];
        }
#pragma unroll
        for (int l = 0; l < N; ++l)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] += qbar[l][v];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (first && j > 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v) qbar[j][v] = 0.0;
                continue;
            }
            double q[NV];
            load_q(r - 1, j, q);
            double nb[NV] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                double fb[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double sacc = 0.0;
#pragma unroll
                    for (int k = 0; k < N; ++k) sacc += B.D[k * N + aa[d]] * my[(j * NV + v) * N3 + node_with(d, k)];
                    fb[v] = cd[d] * sacc;
                }
                flux_vjp(gm1, q, d, fb, nb);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) qbar[j][v] = nb[v];
        }
    }
    // q^(0) = u at every time node
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] += qbar[j][v];
    if (active)
#pragma unroll
        for (int v = 0; v < NV; ++v) ubar[(int64_t(v) * nc + c) * N3 + a] = acc[v];
}

// ---------------------------------------------------------------------------
// Point sampling of the density and its adjoint (uniform meshes)
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ void locate(const double *x, const int *n, const double *lo, const double *inv_h,
                                       int64_t &cell, double phi[3][N])
{
    const DevBasis &B = c_basis[N];
    int ijk[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double y = (x[d] - lo[d]) * inv_h[d];
        int i = int(floor(y));
        i = i < 0 ? 0 : (i >= n[d] ? n[d] - 1 : i);
        ijk[d] = i;
        const double xi = y - i;
#pragma unroll
        for (int e = 0; e < N; ++e) {
            double p = 1.0;
#pragma unroll
            for (int m = 0; m < N; ++m)
                if (m != e) p *= (xi - B.xi[m]) / (B.xi[e] - B.xi[m]);
            phi[d][e] = p;
        }
    }
    cell = ijk[0] + int64_t(n[0]) * (ijk[1] + int64_t(n[1]) * ijk[2]);
}

template <int N>
__global__ void __launch_bounds__(256)
k_sample(const double *__restrict__ u, int64_t nc, SampleGeo sg, const double *__restrict__ pts, int64_t npts,
         double *__restrict__ out)
{
    constexpr int N3 = N * N * N;
    const int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (s >= npts) return;
    int64_t cell;
    double phi[3][N];
    locate<N>(pts + 3 * s, sg.n, sg.lo, sg.inv_h, cell, phi);
    double acc = 0.0;
    for (int a = 0; a < N3; ++a) acc += u[cell * N3 + a] * phi[0][a % N] * phi[1][(a / N) % N] * phi[2][a / (N * N)];
    out[s] = acc;
}

// cell index of a point (floor of the cell coordinate, clamped into the grid)
__device__ __forceinline__ int64_t cell_of(const double *x, const int *n, const double *lo, const double *inv_h)
{
    int ijk[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        int i = int(floor((x[d] - lo[d]) * inv_h[d]));
        ijk[d] = i < 0 ? 0 : (i >= n[d] ? n[d] - 1 : i);
    }
    return ijk[0] + int64_t(n[0]) * (ijk[1] + int64_t(n[1]) * ijk[2]);
}

// ubar_rho[c][a] += sum over the points s in cell c, in increasing s, of
// wbar[s] phi_a(x_s).  One block per point; the block of the lowest-index
// point of a cell forms that cell's sum (lane = node) and the others leave,
// so every cell is written once and the order of the sum is fixed.  The
// leader test scans the earlier points, so the work grows with the square
// of the number of points (meant for up to about 10^4 points).
template <int N>
__global__ void __launch_bounds__(round64(N * N * N))
k_sample_adj(const double *__restrict__ pts, const double *__restrict__ wbar, int64_t npts, SampleGeo sg,
             double *__restrict__ ubar)
{
    constexpr int N3 = N * N * N;
    const int64_t s = blockIdx.x;
    const int a = threadIdx.x;
    const int64_t cs = cell_of(pts + 3 * s, sg.n, sg.lo, sg.inv_h);
    int earlier = 0;
    for (int64_t t = a; t < s; t += blockDim.x) earlier |= cell_of(pts + 3 * t, sg.n, sg.lo, sg.inv_h) == cs;
    if (__syncthreads_or(earlier)) return;  // the same decision in every lane of the block
    if (a >= N3) return;
    double acc = 0.0;
    for (int64_t t = s; t < npts; ++t) {
        if (cell_of(pts + 3 * t, sg.n, sg.lo, sg.inv_h) != cs) continue;
        int64_t cell;
        double phi[3][N];
        locate<N>(pts + 3 * t, sg.n, sg.lo, sg.inv_h, cell, phi);
        acc += wbar[t] * phi[0][a % N] * phi[1][(a / N) % N] * phi[2][a / (N * N)];
    }
    ubar[cs * N3 + a] += acc;
}

// ---------------------------------------------------------------------------
// Dynamic adaptivity: refinement indicator and volumetric transfer
// ---------------------------------------------------------------------------

// Indicator of one cell per block (lane = node): the largest change of the
// density across the cell along any axis, max_{a,d} |d rho_h / d xi_d (x_a)|
// (derivative in the cell's reference coordinate).
template <int N>
__global__ void __launch_bounds__(round64(N * N * N))
k_indicator(const double *__restrict__ u, int64_t nc, double *__restrict__ eta)
{
    constexpr int N2 = N * N, N3 = N2 * N, W = round64(N3) / 64;
    __shared__ double sh[W];
    const DevBasis &B = c_basis[N];
    const int64_t c = blockIdx.x;
    const int a = threadIdx.x;
    double m = 0.0;
    if (a < N3) {
        const double *rho = u + c * N3;  // variable 0
        const int aa[3] = {a % N, (a / N) % N, a / N2};
        const int stride[3] = {1, N, N2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int base = a - aa[d] * stride[d];
            double g = 0.0;
#pragma unroll
            for (int e = 0; e < N; ++e) g += B.D[aa[d] * N + e] * rho[base + e * stride[d]];
            m = fmax(m, fabs(g));
        }
    }
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((a & 63) == 0) sh[a >> 6] = m;
    __syncthreads();
    if (a == 0) {
        double r = sh[0];
        for (int w = 1; w < W; ++w) r = fmax(r, sh[w]);
        eta[c] = r;
    }
}

// Volumetric data of one target cell per block (lane = node): copy, the
// coarser source cell's polynomial at the target nodes (tensor product of the
// 1-D evaluation blocks P), or the L2 projection of the finer source cells
// (tensor product of the 1-D projection blocks R, one term per source cell in
// list order).
template <int N>
__global__ void __launch_bounds__(round64(N * N * N))
k_vtransfer(const double *__restrict__ uf, int64_t ncf, double *__restrict__ ut, int64_t nct,
            const VOp *__restrict__ ops, const VKid *__restrict__ kids, const double *__restrict__ ptab)
{
    constexpr int N2 = N * N, N3 = N2 * N;
    __shared__ double src[NV * N3], t1[NV * N3], t2[NV * N3];
    const int64_t c = blockIdx.x;
    const int a = threadIdx.x;
    const bool node = a < N3;
    const VOp op = ops[c];
    const int aa[3] = {a % N, (a / N) % N, a / N2};
    double acc[NV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (op.kind == 0) {
        if (node)
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = uf[(int64_t(v) * ncf + op.src) * N3 + a];
    } else {
        // the tensor product M0 x M1 x M2 of one source cell applied axis by
        // axis (x, then y, then z), accumulated over the source cells
        const int n = op.kind == 1 ? 1 : op.nkid;
        for (int t = 0; t < n; ++t) {
            int64_t sc;
            int dl, sp[3], half;
            if (op.kind == 1) {
                sc = op.src; dl = op.dl; sp[0] = op.s[0]; sp[1] = op.s[1]; sp[2] = op.s[2]; half = 0;
            } else {
                const VKid k = kids[op.kid0 + t];
                sc = k.cell; dl = k.dl; sp[0] = k.s[0]; sp[1] = k.s[1]; sp[2] = k.s[2]; half = N2;
            }
            const double *M[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) M[d] = ptab + int64_t(transfer_base(dl) + sp[d]) * 2 * N2 + half;
            for (int i = a; i < NV * N3; i += blockDim.x) src[i] = uf[(int64_t(i / N3) * ncf + sc) * N3 + i % N3];
            __syncthreads();
            for (int i = a; i < NV * N3; i += blockDim.x) {
                const int v = i / N3, r = i % N3, o0 = r % N, b12 = r / N;
                double s = 0.0;
#pragma unroll
                for (int b0 = 0; b0 < N; ++b0) s += M[0][o0 * N + b0] * src[v * N3 + b0 + N * b12];
                t1[i] = s;  // (o0, b1, b2)
            }
            __syncthreads();
            for (int i = a; i < NV * N3; i += blockDim.x) {
                const int v = i / N3, r = i % N3, o0 = r % N, o1 = (r / N) % N, b2 = r / N2;
                double s = 0.0;
#pragma unroll
                for (int b1 = 0; b1 < N; ++b1) s += M[1][o1 * N + b1] * t1[v * N3 + o0 + N * b1 + N2 * b2];
                t2[i] = s;  // (o0, o1, b2)
            }
            __syncthreads();
            if (node)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double s = 0.0;
#pragma unroll
                    for (int b2 = 0; b2 < N; ++b2)
                        s += M[2][aa[2] * N + b2] * t2[v * N3 + aa[0] + N * aa[1] + N2 * b2];
                    acc[v] += s;
                }
        }
    }
    if (node)
#pragma unroll
        for (int v = 0; v < NV; ++v) ut[(int64_t(v) * nct + c) * N3 + a] = acc[v];
}

// ---------------------------------------------------------------------------
// A-posteriori finite-volume subcell limiter
// ---------------------------------------------------------------------------
// A cell whose ADER-DG update is unphysical or leaves the relaxed bounds of
// its neighbourhood is advanced instead by first-order finite volumes on
// (2p+1)^3 subcells of the old solution, then fitted back to a polynomial;
// its unlimited face neighbours take the projected subcell fluxes on the
// shared face and run their corrector again (conservation).  The subcell
// averages are tensor-product contractions staged through LDS; every average
// is one fixed chain of fused multiply-adds, so a face layer computed for a
// neighbour's halo equals the same layer of the full computation bit for
// bit, and two limited cells see identical fluxes on their common face.

__constant__ DevSub c_sub[LIM_NMAX + 1];

template <int N> struct LimCfg {
    static constexpr int NS = 2 * N - 1, N2 = N * N, N3 = N2 * N, S2 = NS * NS, S3 = S2 * NS;
    static constexpr int T1 = NS * N2, T2 = S2 * N;  // per-variable contraction temporaries
    // variables contracted together in the FV kernel (all five while they fit in LDS)
    static constexpr int NVB = N <= 6 ? NV : 1;
    static constexpr int TMP = (NVB * (T1 + T2) > NV * S2) ? NVB * (T1 + T2) : NV * S2;
    // threads of the FV kernel; each keeps PT subcells' new data in registers
    static constexpr int THREADS = N >= 6 ? 512 : 256;
    static constexpr int PT = (S3 + THREADS - 1) / THREADS;
};

// rho <= 0 or p <= 0, the pressure test written without a division: for
// rho > 0, p > 0 exactly when 2 rho E > |m|^2 (also false for NaN)
__device__ __forceinline__ bool lim_nonpositive(const double q[NV])
{
    return !(q[0] > 0.0) || !(2.0 * q[0] * q[4] - (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) > 0.0);
}

// non-finite, rho <= 0 or p <= 0
__device__ __forceinline__ bool lim_bad(double, const double q[NV])
{
    bool fin = true;
#pragma unroll
    for (int v = 0; v < NV; ++v) fin = fin && isfinite(q[v]);
    return !fin || lim_nonpositive(q);
}

// Subcell averages of NVAR variables x[var N^3 + a] (node a0 + N a1 + N^2 a2).
// axis < 0: all subcells, out[var ostride + s0 + NS s1 + NS^2 s2]; axis = d:
// only the layer s_d = layer, out[var ostride + j1 + NS j2] over the other two
// axes in increasing order.  t1, t2: NVAR LimCfg<N>::T1 and ::T2 doubles.
// Every value is the same chain of fused multiply-adds whatever NVAR and
// whichever outputs are asked for, so a layer matches the full result bit for
// bit.  Block-wide (contains barriers).
template <int N, int NVAR = 1>
__device__ void sub_avg(const double *__restrict__ A, const double *x, double *t1, double *t2, double *out, int ostride,
                        int axis, int layer)
{
    using C = LimCfg<N>;
    constexpr int NS = C::NS, N2 = N * N, N3 = N2 * N;
    const int lo0 = axis == 0 ? layer : 0, n0 = axis == 0 ? 1 : NS;
    const int lo1 = axis == 1 ? layer : 0, n1 = axis == 1 ? 1 : NS;
    const int lo2 = axis == 2 ? layer : 0, n2 = axis == 2 ? 1 : NS;
    const int m1 = n0 * N2, m2 = n0 * n1 * N, m3 = n0 * n1 * n2;
    for (int i = threadIdx.x; i < NVAR * m1; i += blockDim.x) {
        const int var = i / m1, r = i % m1;
        const int s0 = lo0 + r % n0, a12 = r / n0;
        double acc = 0.0;
#pragma unroll
        for (int a0 = 0; a0 < N; ++a0) acc = fma(A[s0 * N + a0], x[var * N3 + a0 + N * a12], acc);
        t1[var * C::T1 + s0 + NS * a12] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NVAR * m2; i += blockDim.x) {
        const int var = i / m2, r = i % m2;
        const int s0 = lo0 + r % n0, s1 = lo1 + (r / n0) % n1, a2 = r / (n0 * n1);
        double acc = 0.0;
#pragma unroll
        for (int a1 = 0; a1 < N; ++a1)
            acc = fma(A[s1 * N + a1], t1[var * C::T1 + s0 + NS * (a1 + N * a2)], acc);
        t2[var * C::T2 + s0 + NS * (s1 + NS * a2)] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NVAR * m3; i += blockDim.x) {
        const int var = i / m3, r = i % m3;
        const int j0 = r % n0, j1 = (r / n0) % n1, j2 = r / (n0 * n1);
        const int s0 = lo0 + j0, s1 = lo1 + j1, s2 = lo2 + j2;
        double acc = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2) acc = fma(A[s2 * N + a2], t2[var * C::T2 + s0 + NS * (s1 + NS * a2)], acc);
        out[var * ostride + r] = acc;
    }
    __syncthreads();
}

// Least-squares polynomials x[var N^3 + a] of NVAR variables' subcell data
// v[var NS^3 + s] (r1: NVAR T2 doubles, r2: NVAR T1 doubles).  Block-wide.
template <int N, int NVAR = 1>
__device__ void sub_fit(const double *__restrict__ Ap, const double *v, double *r1, double *r2, double *x)
{
    using C = LimCfg<N>;
    constexpr int NS = C::NS, S2 = NS * NS, S3 = S2 * NS, N2 = N * N, N3 = N2 * N;
    for (int i = threadIdx.x; i < NVAR * N * S2; i += blockDim.x) {
        const int var = i / (N * S2), r = i % (N * S2);
        const int k0 = r % N, s12 = r / N;
        double acc = 0.0;
        for (int s0 = 0; s0 < NS; ++s0) acc = fma(Ap[k0 * NS + s0], v[var * S3 + s0 + NS * s12], acc);
        r1[var * C::T2 + r] = acc;  // k0 + N (s1 + NS s2)
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NVAR * N2 * NS; i += blockDim.x) {
        const int var = i / (N2 * NS), r = i % (N2 * NS);
        const int k0 = r % N, k1 = (r / N) % N, s2 = r / N2;
        double acc = 0.0;
        for (int s1 = 0; s1 < NS; ++s1) acc = fma(Ap[k1 * NS + s1], r1[var * C::T2 + k0 + N * (s1 + NS * s2)], acc);
        r2[var * C::T1 + r] = acc;  // k0 + N (k1 + N s2)
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NVAR * N3; i += blockDim.x) {
        const int var = i / N3, r = i % N3;
        const int k01 = r % N2, k2 = r / N2;
        double acc = 0.0;
        for (int s2 = 0; s2 < NS; ++s2) acc = fma(Ap[k2 * NS + s2], r2[var * C::T1 + k01 + N2 * s2], acc);
        x[var * N3 + r] = acc;
    }
    __syncthreads();
}

// Cell mean of one variable (Gauss rule), one fixed sequential order.
template <int N>
__device__ double lim_mean(const double *x)
{
    const DevBasis &B = c_basis[N];
    double acc = 0.0;
    for (int a = 0; a < N * N * N; ++a) acc = fma(B.w[a % N] * B.w[(a / N) % N] * B.w[a / (N * N)], x[a], acc);
    return acc;
}

// Rusanov flux along d between subcell states ql (minus side) and qr.
__device__ __forceinline__ void lim_rusanov(double gamma, int d, const double ql[NV], const double qr[NV],
                                            double f[NV])
{
    const double gm1 = gamma - 1.0;
    const double pl = gm1 * (ql[4] - 0.5 * (ql[1] * ql[1] + ql[2] * ql[2] + ql[3] * ql[3]) / ql[0]);
    const double pr = gm1 * (qr[4] - 0.5 * (qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]) / qr[0]);
    const double vl = ql[1 + d] / ql[0], vr = qr[1 + d] / qr[0];
    const double sl = fabs(vl) + sqrt(gamma * pl / ql[0]), sr = fabs(vr) + sqrt(gamma * pr / qr[0]);
    const double smax = fmax(sl, sr);
    double fl[NV], fr[NV];
    fl[0] = ql[1 + d];
    fr[0] = qr[1 + d];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        fl[1 + k] = vl * ql[1 + k];
        fr[1 + k] = vr * qr[1 + k];
    }
    fl[1 + d] += pl;
    fr[1 + d] += pr;
    fl[4] = vl * (ql[4] + pl);
    fr[4] = vr * (qr[4] + pr);
#pragma unroll
    for (int v = 0; v < NV; ++v) f[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * smax * (qr[v] - ql[v]);
}

__global__ void __launch_bounds__(256)
k_lim_nbr(const int32_t *__restrict__ fm, const int32_t *__restrict__ fp, int64_t nf, int d, int64_t nc,
          int32_t *__restrict__ nbr)
{
    const int64_t f = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    nbr[(2 * d + 1) * nc + fm[f]] = fp[f];
    nbr[(2 * d) * nc + fp[f]] = fm[f];
}

// One wavefront per cell: loads the cell's u (NV N^3 doubles, coalesced)
// into LDS x and scans its subcell
// averages: per variable min / max, whether an average is unphysical,
// whether one leaves the relaxed bounds and whether a node is unphysical (if
// BND; ext[k NV + var] and ext[7 NV + k NV + var] hold the old extremes of
// the cell (k = 0) and its face neighbours, written by the caller before the
// first barrier).  Stage 1 contracts x-pencils into t1 (NV NS N^2 doubles);
// stages 2 and 3 are fused per
// (s0, s1) column: the NV x N stage-2 values of a column stay in registers
// and the column's subcells are produced one at a time.  Each average is the
// same chain of fused multiply-adds as in sub_avg.  Results are valid in
// every lane.
template <int N, bool BND>
__device__ void lim_cell_scan(const double *__restrict__ u, int64_t nc, int64_t c, double gm1, double *x,
                              double *t1, const double *ext, double delta0, double eps,
                              double lo[NV], double hi[NV], bool &bad_avg, bool &bad_node, bool &outside)
{
    using C = LimCfg<N>;
    constexpr int NS = C::NS, N2 = C::N2, N3 = C::N3, S2 = C::S2;
    const double *__restrict__ A = c_sub[N].A;
    const int lane = threadIdx.x;
    for (int i = lane; i < NV * N3; i += 64) {
        const int64_t o = (int64_t(i / N3) * nc + c) * N3 + i % N3;
        x[i] = u[o];
    }
    __syncthreads();
    for (int t = lane; t < NV * N2; t += 64) {
        const int var = t / N2, a12 = t % N2;
        double xv[N];
#pragma unroll
        for (int a0 = 0; a0 < N; ++a0) xv[a0] = x[var * N3 + N * a12 + a0];
#pragma unroll
        for (int s0 = 0; s0 < NS; ++s0) {
            double acc = 0.0;
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0) acc = fma(A[s0 * N + a0], xv[a0], acc);
            t1[var * C::T1 + s0 + NS * a12] = acc;
        }
    }
    __syncthreads();
    bool bn = false;
    if (BND)
        for (int a = lane; a < N3; a += 64) {
            double q[NV];
#pragma unroll
            for (int var = 0; var < NV; ++var) q[var] = x[var * N3 + a];
            bn = bn || lim_bad(gm1, q);
        }
    double bl[NV], bh[NV];
#pragma unroll
    for (int var = 0; var < NV; ++var) {
        lo[var] = INFINITY;
        hi[var] = -INFINITY;
        bl[var] = 0.0;
        bh[var] = 0.0;
        if (BND) {
            double l = ext[var], h = ext[7 * NV + var];
            for (int k = 1; k < 7; ++k) {
                l = fmin(l, ext[k * NV + var]);
                h = fmax(h, ext[7 * NV + k * NV + var]);
            }
            double delta = eps * (h - l);
            if (delta < delta0) delta = delta0;
            bl[var] = l - delta;
            bh[var] = h + delta;
        }
    }
    bool ba = false, bo = false;
    for (int t = lane; t < S2; t += 64) {
        const int s0 = t % NS, s1 = t / NS;
        double t2[NV][N];
#pragma unroll
        for (int var = 0; var < NV; ++var)
#pragma unroll
            for (int a2 = 0; a2 < N; ++a2) {
                double acc = 0.0;
#pragma unroll
                for (int a1 = 0; a1 < N; ++a1)
                    acc = fma(A[s1 * N + a1], t1[var * C::T1 + s0 + NS * (a1 + N * a2)], acc);
                t2[var][a2] = acc;
            }
#pragma unroll 1
        for (int s2 = 0; s2 < NS; ++s2) {
            double q[NV];
#pragma unroll
            for (int var = 0; var < NV; ++var) {
                double acc = 0.0;
#pragma unroll
                for (int a2 = 0; a2 < N; ++a2) acc = fma(A[s2 * N + a2], t2[var][a2], acc);
                q[var] = acc;
                lo[var] = fmin(lo[var], acc);
                hi[var] = fmax(hi[var], acc);
                if (BND) bo = bo || !(acc >= bl[var] && acc <= bh[var]);
            }
            // with bounds, a non-finite average already fails them
            ba = ba || (BND ? lim_nonpositive(q) : lim_bad(gm1, q));
        }
    }
#pragma unroll
    for (int var = 0; var < NV; ++var)
        for (int off = 32; off > 0; off >>= 1) {
            lo[var] = fmin(lo[var], __shfl_xor(lo[var], off));
            hi[var] = fmax(hi[var], __shfl_xor(hi[var], off));
        }
    bad_avg = __any(ba);
    bad_node = __any(bn);
    outside = __any(bo);
}

// Subcell bounds of one cell's u (the subcell averages' extremes, or the
// cell mean if an average is unphysical) into mm2 / fb2 (one wavefront).
template <int N>
__device__ void lim_scan_cell(const double *__restrict__ u, int64_t nc, int64_t c, double gm1, double *x, double *t1,
                              double *__restrict__ mm2, int32_t *__restrict__ fb2)
{
    double lo[NV], hi[NV];
    bool bad, bn, bo;
    lim_cell_scan<N, false>(u, nc, c, gm1, x, t1, nullptr, 0.0, 0.0, lo, hi, bad, bn, bo);
    const int lane = threadIdx.x;
    if (bad) {
        const double m = lane < NV ? lim_mean<N>(x + lane * N * N * N) : 0.0;
        if (lane < NV) {
            mm2[c * 2 * NV + lane] = m;
            mm2[c * 2 * NV + NV + lane] = m;
        }
    } else if (lane < NV) {
        double l = lo[0], h = hi[0];
#pragma unroll
        for (int var = 1; var < NV; ++var)
            if (lane == var) {
                l = lo[var];
                h = hi[var];
            }
        mm2[c * 2 * NV + lane] = l;
        mm2[c * 2 * NV + NV + lane] = h;
    }
    if (lane == 0) fb2[c] = bad ? 1 : 0;
    __syncthreads();
}

// LISTED = false: one wavefront per cell; true: persistent over the cells
// whose corrector ran again.
template <int N, bool LISTED>
__global__ void __launch_bounds__(64)
k_lim_scan(const double *__restrict__ u, int64_t nc, double gamma, double *__restrict__ mm2,
           int32_t *__restrict__ fb2, const int32_t *__restrict__ rlist, const int32_t *__restrict__ cnt)
{
    using C = LimCfg<N>;
    __shared__ double x[NV * C::N3], t1[NV * C::T1];
    if (!LISTED) {
        lim_scan_cell<N>(u, nc, blockIdx.x, gamma - 1.0, x, t1, mm2, fb2);
        return;
    }
    const int n = cnt[1];
    for (int it = blockIdx.x; it < n; it += gridDim.x) lim_scan_cell<N>(u, nc, rlist[it], gamma - 1.0, x, t1, mm2, fb2);
}

// Start of a limited step: copy of u, the carried bounds become the old ones,
// counters cleared.
__global__ void __launch_bounds__(256)
k_lim_copy(const double *__restrict__ u, int64_t n_u, int64_t nc, double *__restrict__ uold,
           const double *__restrict__ mm2, double *__restrict__ mm, const int32_t *__restrict__ fb2,
           int32_t *__restrict__ fb, int32_t *__restrict__ cnt)
{
    const int64_t i0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x, stride = int64_t(gridDim.x) * blockDim.x;
    if (i0 == 0) {
        cnt[0] = 0;
        cnt[1] = 0;
    }
    for (int64_t i = i0; i < n_u; i += stride) uold[i] = u[i];
    for (int64_t i = i0; i < 2 * NV * nc; i += stride) mm[i] = mm2[i];
    for (int64_t i = i0; i < nc; i += stride) fb[i] = fb2[i];
}

// One wavefront per cell: troubled-cell test of the candidate u.  Lanes
// 0..34 fetch the old extremes of (cell or face neighbour k, variable) while
// the cell's data loads; every lane combines them after the first barrier.
template <int N>
__global__ void __launch_bounds__(64)
k_lim_detect(const double *__restrict__ u, int64_t nc, double gamma, double delta0, double eps, int force,
             const double *__restrict__ mm, const int32_t *__restrict__ nbr, int32_t *__restrict__ flag,
             int32_t *__restrict__ list, int32_t *__restrict__ cnt, double *__restrict__ mm2,
             int32_t *__restrict__ fb2)
{
    using C = LimCfg<N>;
    __shared__ double x[NV * C::N3], t1[NV * C::T1], ext[2 * 7 * NV];
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    // a hanging side (no same-level neighbour) adds no bounds; such a cell
    // cannot be limited
    if (lane < 7 * NV) {
        const int k = lane / NV, var = lane % NV;
        const int64_t n = k == 0 ? c : nbr[(k - 1) * nc + c];
        const int64_t o = n < 0 ? c : n;
        ext[lane] = mm[o * 2 * NV + var];
        ext[7 * NV + lane] = mm[o * 2 * NV + NV + var];
    }
    double lo[NV], hi[NV];
    bool ba, bn, bo;
    lim_cell_scan<N, true>(u, nc, c, gamma - 1.0, x, t1, ext, delta0, eps, lo, hi, ba, bn, bo);
    const bool troubled = ba || bn || bo || force;
    if (lane == 0) {
        bool hang = false;
        for (int k = 0; k < 6; ++k) hang = hang || nbr[k * nc + c] < 0;
        flag[c] = troubled ? (hang ? 3 : 1) : 0;
        if (troubled && !hang) list[atomicAdd(cnt, 1)] = int32_t(c);
        fb2[c] = 0;  // an unlimited cell's averages are physical; limited cells are rewritten
    }
    // the bounds an unlimited cell carries into the next step (as lim_scan_cell)
    if (lane < NV) {
        double l = lo[0], h = hi[0];
#pragma unroll
        for (int var = 1; var < NV; ++var)
            if (lane == var) {
                l = lo[var];
                h = hi[var];
            }
        mm2[c * 2 * NV + lane] = l;
        mm2[c * 2 * NV + NV + lane] = h;
    }
}

// Persistent over the limited cells: FV step on the subcells, least-squares
// fit (or the constant mean), projected subcell fluxes for the unlimited face
// neighbours.
template <typename T, int N>
__global__ void __launch_bounds__(LimCfg<N>::THREADS)
k_lim_fv(double *__restrict__ u, T *__restrict__ fside, int64_t nc, Geo geo, const double *__restrict__ dt_dev,
         double gamma, const double *__restrict__ uold, const int32_t *__restrict__ fb,
         const int32_t *__restrict__ nbr, int32_t *__restrict__ flag, const int32_t *__restrict__ list,
         int32_t *__restrict__ rlist, int32_t *__restrict__ cnt, double *__restrict__ mm2, int32_t *__restrict__ fb2,
         const int8_t *__restrict__ level)
{
    using C = LimCfg<N>;
    constexpr int NS = C::NS, N2 = C::N2, N3 = C::N3, S2 = C::S2, S3 = C::S3, PT = C::PT, TH = C::THREADS;
    __shared__ double v[NV * S3], halo[6 * NV * S2], x[NV * N3], tmp[C::TMP], mean[NV], red[2 * NV * (TH / 64)];
    __shared__ double err[NV * N2], dlt[6 * NV];
    const DevSub &S = c_sub[N];
    const double dt = dt_dev[0], gm1 = gamma - 1.0;
    const int n_lim = cnt[0];
    constexpr int NVB = C::NVB;
    double *t1 = tmp, *t2 = tmp + NVB * C::T1;
    for (int it = blockIdx.x; it < n_lim; it += gridDim.x) {
        const int64_t c = list[it];
        // old subcell data of the cell and the face layers of its neighbours
        for (int k = -1; k < 6; ++k) {
            const int64_t o = k < 0 ? c : nbr[k * nc + c];
            for (int i = threadIdx.x; i < NV * N3; i += blockDim.x)
                x[i] = uold[(int64_t(i / N3) * nc + o) * N3 + i % N3];
            __syncthreads();
            const int cnt_out = k < 0 ? S3 : S2;
            double *dst = k < 0 ? v : halo + k * NV * S2;
            if (fb[o]) {
                if (threadIdx.x < NV) mean[threadIdx.x] = lim_mean<N>(x + threadIdx.x * N3);
                __syncthreads();
                for (int i = threadIdx.x; i < NV * cnt_out; i += blockDim.x) dst[i] = mean[i / cnt_out];
            } else {
                const int axis = k < 0 ? -1 : k / 2, layer = (k & 1) ? 0 : NS - 1;
                for (int var = 0; var < NV; var += NVB)
                    sub_avg<N, NVB>(S.A, x + var * N3, t1, t2, dst + var * cnt_out, cnt_out, axis, layer);
            }
            __syncthreads();
        }
        // subcell fluxes on faces shared with unlimited cells, projected onto
        // the face nodes of the neighbour's side.  The FP32 form stores face
        // fluxes in FP32: dlt[k] = sum_b W_b (stored - exact) is added to this
        // cell's subcell fluxes on face k, so that both sides exchange the
        // same total (conservation to FP64 rounding).
        if (threadIdx.x < 6 * NV) dlt[threadIdx.x] = 0.0;
        __syncthreads();
        for (int k = 0; k < 6; ++k) {
            const int64_t o = nbr[k * nc + c];
            if (flag[o] == 1) continue;  // never 1 for every reader: uniform
            const int d = k / 2, plus = k & 1;
            const int t1a = d == 0 ? 1 : 0, t2a = d == 2 ? 1 : 2;
            for (int j = threadIdx.x; j < S2; j += blockDim.x) {
                int sc[3];
                sc[t1a] = j % NS;
                sc[t2a] = j / NS;
                sc[d] = plus ? NS - 1 : 0;
                const int is = sc[0] + NS * sc[1] + S2 * sc[2];
                double qc[NV], qo[NV], f[NV];
#pragma unroll
                for (int var = 0; var < NV; ++var) {
                    qc[var] = v[var * S3 + is];
                    qo[var] = halo[(k * NV + var) * S2 + j];
                }
                if (plus) lim_rusanov(gamma, d, qc, qo, f);
                else lim_rusanov(gamma, d, qo, qc, f);
#pragma unroll
                for (int var = 0; var < NV; ++var) tmp[var * S2 + j] = f[var];
            }
            __syncthreads();
            const int sopp = 2 * d + (1 - plus);
            for (int i = threadIdx.x; i < NV * N2; i += blockDim.x) {
                const int var = i / N2, b = i % N2, b1 = b % N, b2 = b / N;
                double acc = 0.0;
                for (int j2 = 0; j2 < NS; ++j2) {
                    double r = 0.0;
                    for (int j1 = 0; j1 < NS; ++j1) r = fma(S.Bf[b1 * NS + j1], tmp[var * S2 + j1 + NS * j2], r);
                    acc = fma(S.Bf[b2 * NS + j2], r, acc);
                }
                const T stored = T(acc);
                fside[(int64_t(sopp * NV + var) * nc + o) * N2 + b] = stored;
                err[i] = c_basis[N].w[b1] * c_basis[N].w[b2] * (double(stored) - acc);
            }
            __syncthreads();
            if (!std::is_same<T, double>::value && threadIdx.x < NV) {
                double sum = 0.0;
                for (int b = 0; b < N2; ++b) sum += err[threadIdx.x * N2 + b];
                dlt[k * NV + threadIdx.x] = sum;
            }
            if (threadIdx.x == 0 && (atomicCAS(&flag[o], 0, 2) == 0 || atomicCAS(&flag[o], 3, 4) == 3))
                rlist[atomicAdd(&cnt[1], 1)] = int32_t(o);
            __syncthreads();
        }
        // first-order update of every subcell (kept in registers)
        double vn[PT][NV];
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const int s = threadIdx.x + k * TH;
            if (s >= S3) break;
            const int ss[3] = {s % NS, (s / NS) % NS, s / S2};
            double q[NV], acc[NV] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int var = 0; var < NV; ++var) q[var] = v[var * S3 + s];
#pragma unroll 1
            for (int d = 0; d < 3; ++d) {
                const double inv_h = geo.inv_dx[level ? level[c] : 0][d] * NS;
                const int t1a = d == 0 ? 1 : 0, t2a = d == 2 ? 1 : 2;
#pragma unroll 1
                for (int side = 0; side < 2; ++side) {
                    double qo[NV], f[NV];
                    const int sn = ss[d] + (side ? 1 : -1);
                    if (sn >= 0 && sn < NS) {
                        const int idx = s + (side ? 1 : -1) * (d == 0 ? 1 : (d == 1 ? NS : S2));
#pragma unroll
                        for (int var = 0; var < NV; ++var) qo[var] = v[var * S3 + idx];
                    } else {
                        const int j = ss[t1a] + NS * ss[t2a];
#pragma unroll
                        for (int var = 0; var < NV; ++var) qo[var] = halo[((2 * d + side) * NV + var) * S2 + j];
                    }
                    if (side) lim_rusanov(gamma, d, q, qo, f);
                    else lim_rusanov(gamma, d, qo, q, f);
                    if (sn < 0 || sn >= NS)
#pragma unroll
                        for (int var = 0; var < NV; ++var) f[var] += dlt[(2 * d + side) * NV + var];
#pragma unroll
                    for (int var = 0; var < NV; ++var) acc[var] += (side ? 1.0 : -1.0) * f[var] * inv_h;
                }
            }
#pragma unroll
            for (int var = 0; var < NV; ++var) vn[k][var] = q[var] - dt * acc[var];
        }
        // new subcell data (every read of the old data is done), their means
        __syncthreads();
        double part[NV] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const int s = threadIdx.x + k * TH;
            if (s >= S3) break;
#pragma unroll
            for (int var = 0; var < NV; ++var) {
                v[var * S3 + s] = vn[k][var];
                part[var] += vn[k][var];
            }
        }
        {
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
            for (int var = 0; var < NV; ++var) {
                for (int off = 32; off > 0; off >>= 1) part[var] += __shfl_xor(part[var], off);
                if (lane == 0) red[var * (TH / 64) + wv] = part[var];
            }
        }
        __syncthreads();
        if (threadIdx.x < NV) {
            double sum = 0.0;
            for (int w = 0; w < TH / 64; ++w) sum += red[threadIdx.x * (TH / 64) + w];
            mean[threadIdx.x] = sum / S3;
        }
        // least-squares fit into x, its subcell averages back into v
        for (int var = 0; var < NV; var += NVB) sub_fit<N, NVB>(S.Ap, v + var * S3, t2, t1, x + var * N3);
        bool bad = false;
        for (int a = threadIdx.x; a < N3; a += blockDim.x) {
            double q[NV];
#pragma unroll
            for (int var = 0; var < NV; ++var) q[var] = x[var * N3 + a];
            bad = bad || lim_bad(gm1, q);
        }
        for (int var = 0; var < NV; var += NVB) sub_avg<N, NVB>(S.A, x + var * N3, t1, t2, v + var * S3, S3, -1, 0);
        for (int s = threadIdx.x; s < S3; s += blockDim.x) {
            double q[NV];
#pragma unroll
            for (int var = 0; var < NV; ++var) q[var] = v[var * S3 + s];
            bad = bad || lim_bad(gm1, q);
        }
        bad = __syncthreads_or(bad);
        for (int i = threadIdx.x; i < NV * N3; i += blockDim.x) {
            if (bad) x[i] = mean[i / N3];
            u[(int64_t(i / N3) * nc + c) * N3 + i % N3] = x[i];
        }
        __syncthreads();
        // bounds of the new state for the next step, as lim_scan_cell gives
        // them (same averages, exact extremes, the same mean)
        if (bad)
            for (int var = 0; var < NV; var += NVB) sub_avg<N, NVB>(S.A, x + var * N3, t1, t2, v + var * S3, S3, -1, 0);
        double lo[NV], hi[NV];
        bool badv = false;
#pragma unroll
        for (int var = 0; var < NV; ++var) {
            lo[var] = INFINITY;
            hi[var] = -INFINITY;
        }
        for (int s = threadIdx.x; s < S3; s += blockDim.x) {
            double q[NV];
#pragma unroll
            for (int var = 0; var < NV; ++var) {
                q[var] = v[var * S3 + s];
                lo[var] = fmin(lo[var], q[var]);
                hi[var] = fmax(hi[var], q[var]);
            }
            badv = badv || lim_bad(gm1, q);
        }
        {
            const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
            for (int var = 0; var < NV; ++var) {
                for (int off = 32; off > 0; off >>= 1) {
                    lo[var] = fmin(lo[var], __shfl_xor(lo[var], off));
                    hi[var] = fmax(hi[var], __shfl_xor(hi[var], off));
                }
                if (lane == 0) {
                    red[var * (TH / 64) + wv] = lo[var];
                    red[(NV + var) * (TH / 64) + wv] = hi[var];
                }
            }
        }
        badv = __syncthreads_or(badv);
        if (threadIdx.x < NV) {
            const int var = threadIdx.x;
            double l = red[var * (TH / 64)], h = red[(NV + var) * (TH / 64)];
            for (int w = 1; w < TH / 64; ++w) {
                l = fmin(l, red[var * (TH / 64) + w]);
                h = fmax(h, red[(NV + var) * (TH / 64) + w]);
            }
            if (badv) l = h = lim_mean<N>(x + var * N3);
            mm2[c * 2 * NV + var] = l;
            mm2[c * 2 * NV + NV + var] = h;
        }
        if (threadIdx.x == 0) fb2[c] = badv ? 1 : 0;
        __syncthreads();
    }
}

// Persistent over the listed cells: the corrector again with the face fluxes
// the limited neighbours left in fside.
template <typename T, int N>
__global__ void __launch_bounds__(round64(N * N * N))
k_lim_recorrect(const double *__restrict__ ustar, const T *__restrict__ fside, const double *__restrict__ dt_dev,
                double *__restrict__ u, int64_t nc, Geo geo, const int32_t *__restrict__ rlist,
                const int32_t *__restrict__ cnt, const int8_t *__restrict__ level)
{
    constexpr int N2 = N * N, N3 = N2 * N;
    const DevBasis &B = c_basis[N];
    const int a = threadIdx.x;
    if (a >= N3) return;
    const int a0 = a % N, a1 = (a / N) % N, a2 = a / N2;
    const int bx = a1 + N * a2, by = a0 + N * a2, bz = a0 + N * a1;
    const double dt = dt_dev[0];
    const int n = cnt[1];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int64_t c = rlist[it];
        const int lev = level ? level[c] : 0;
        const double sx = dt * geo.inv_dx[lev][0] * B.winv[a0];
        const double sy = dt * geo.inv_dx[lev][1] * B.winv[a1];
        const double sz = dt * geo.inv_dx[lev][2] * B.winv[a2];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double fxm = fside[(int64_t(0 * NV + v) * nc + c) * N2 + bx];
            const double fxp = fside[(int64_t(1 * NV + v) * nc + c) * N2 + bx];
            const double fym = fside[(int64_t(2 * NV + v) * nc + c) * N2 + by];
            const double fyp = fside[(int64_t(3 * NV + v) * nc + c) * N2 + by];
            const double fzm = fside[(int64_t(4 * NV + v) * nc + c) * N2 + bz];
            const double fzp = fside[(int64_t(5 * NV + v) * nc + c) * N2 + bz];
            const double s = sx * (B.R[a0] * fxp - B.L[a0] * fxm) + sy * (B.R[a1] * fyp - B.L[a1] * fym) +
                             sz * (B.R[a2] * fzp - B.L[a2] * fzm);
            const int64_t o = (int64_t(v) * nc + c) * N3 + a;
            u[o] = ustar[o] - s;
        }
    }
}

// ---------------------------------------------------------------------------
// Linear variant: elastic waves with the Cauchy-Kowalevski predictor
// ---------------------------------------------------------------------------
// 9 unknowns (s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, v_x, v_y, v_z), material
// (rho, lambda, mu) constant per cell, flux A_d q.  Uniform periodic meshes
// (neighbours by index arithmetic), FP64.  The predictor keeps the k-th time
// derivative L^k u of every node in LDS for the derivative contractions and
// accumulates qbar = sum_k dt^k/(k+1)! L^k u in registers; L lowers the
// polynomial degree and is applied p times.

constexpr int NLV = 9;
enum { LSXX = 0, LSYY, LSZZ, LSXY, LSYZ, LSXZ, LVX, LVY, LVZ };

// f = A_d q (lam2 = lambda + 2 mu, irho = 1/rho)
__device__ __forceinline__ void lin_flux(int d, double lam, double mu, double lam2, double irho, const double q[NLV],
                                         double f[NLV])
{
    if (d == 0) {
        f[LSXX] = -lam2 * q[LVX];
        f[LSYY] = -lam * q[LVX];
        f[LSZZ] = -lam * q[LVX];
        f[LSXY] = -mu * q[LVY];
        f[LSYZ] = 0.0;
        f[LSXZ] = -mu * q[LVZ];
        f[LVX] = -q[LSXX] * irho;
        f[LVY] = -q[LSXY] * irho;
        f[LVZ] = -q[LSXZ] * irho;
    } else if (d == 1) {
        f[LSXX] = -lam * q[LVY];
        f[LSYY] = -lam2 * q[LVY];
        f[LSZZ] = -lam * q[LVY];
        f[LSXY] = -mu * q[LVX];
        f[LSYZ] = -mu * q[LVZ];
        f[LSXZ] = 0.0;
        f[LVX] = -q[LSXY] * irho;
        f[LVY] = -q[LSYY] * irho;
        f[LVZ] = -q[LSYZ] * irho;
    } else {
        f[LSXX] = -lam * q[LVZ];
        f[LSYY] = -lam * q[LVZ];
        f[LSZZ] = -lam2 * q[LVZ];
        f[LSXY] = 0.0;
        f[LSYZ] = -mu * q[LVY];
        f[LSXZ] = -mu * q[LVX];
        f[LVX] = -q[LSXZ] * irho;
        f[LVY] = -q[LSYZ] * irho;
        f[LVZ] = -q[LSZZ] * irho;
    }
}

// Cells per block of the elastic predictor: CPB cells of N^3 threads each.
template <int N> struct LinCfg {
    static constexpr int N3 = N * N * N;
    static constexpr int CPB = N3 >= 256 ? 1 : 256 / N3;
    static constexpr int THREADS = round64(CPB * N3);
    // waves per SIMD asked of the register allocator (fits without spills for N <= 4)
    static constexpr int MIN_WAVES = N <= 4 ? 4 : 1;
};

// CPB cells per block, one thread per node.  FTR: also write the normal-flux
// traces (the flux of the state trace, lin_flux); the fused elastic step
// forms them again from the state traces and needs only those.
template <int N, bool FTR = true>
__global__ void __launch_bounds__(LinCfg<N>::THREADS) __attribute__((amdgpu_waves_per_eu(LinCfg<N>::MIN_WAVES, 8)))
k_lin_predictor(const double *__restrict__ u, const double *__restrict__ mat, const double *__restrict__ dt_dev,
                double *__restrict__ ustar, double *__restrict__ traces, int64_t nc, double idx0, double idx1,
                double idx2)
{
    constexpr int N2 = N * N, N3 = N2 * N, CPB = LinCfg<N>::CPB;
    __shared__ double lds[CPB * NLV * N3];
    const DevBasis &B = c_basis[N];
    const int lc = threadIdx.x / N3, a = threadIdx.x % N3;
    const int64_t c = int64_t(blockIdx.x) * CPB + lc;
    const bool node = lc < CPB && c < nc;
    double *dk = lds + (lc < CPB ? lc : 0) * NLV * N3;
    const int aa[3] = {a % N, (a / N) % N, a / N2};
    const int64_t cm = node ? c : 0;
    const double rho = mat[cm], lam = mat[nc + cm], mu = mat[2 * nc + cm];
    const double lam2 = lam + 2.0 * mu, irho = 1.0 / rho;
    const double idx[3] = {idx0, idx1, idx2};
    const double dt = dt_dev[0];
    double uc[NLV], qbar[NLV];
#pragma unroll
    for (int v = 0; v < NLV; ++v) {
        uc[v] = node ? u[(int64_t(v) * nc + c) * N3 + a] : 0.0;
        qbar[v] = uc[v];
        if (node) dk[v * N3 + a] = uc[v];
    }
    __syncthreads();
    double fac = 1.0;
    for (int k = 1; k < N; ++k) {
        // L dk at this node: -sum_d (1/dx_d) A_d (D_d dk)
        double nd[NLV] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (node)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int stride = d == 0 ? 1 : (d == 1 ? N : N2);
                const int base = a - aa[d] * stride;
                double g[NLV];
#pragma unroll
                for (int v = 0; v < NLV; ++v) {
                    double s = 0.0;
#pragma unroll
                    for (int e = 0; e < N; ++e) s = fma(B.D[aa[d] * N + e], dk[v * N3 + base + e * stride], s);
                    g[v] = s;
                }
                double f[NLV];
                lin_flux(d, lam, mu, lam2, irho, g, f);
#pragma unroll
                for (int v = 0; v < NLV; ++v) nd[v] = fma(-idx[d], f[v], nd[v]);
            }
        __syncthreads();
        fac *= dt / (k + 1);
#pragma unroll
        for (int v = 0; v < NLV; ++v) {
            if (node) dk[v * N3 + a] = nd[v];
            qbar[v] = fma(fac, nd[v], qbar[v]);
        }
        __syncthreads();
    }
    // qbar into LDS for the volume term and the face projections
#pragma unroll
    for (int v = 0; v < NLV; ++v)
        if (node) dk[v * N3 + a] = qbar[v];
    __syncthreads();
    if (!node) return;
    // volume term: u + sum_d (dt/dx_d) (1/w) A_d (Kw_d qbar)
    double us[NLV];
#pragma unroll
    for (int v = 0; v < NLV; ++v) us[v] = uc[v];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int stride = d == 0 ? 1 : (d == 1 ? N : N2);
        const int base = a - aa[d] * stride;
        double g[NLV], f[NLV];
#pragma unroll
        for (int v = 0; v < NLV; ++v) {
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < N; ++e) s = fma(B.Kw[aa[d] * N + e], dk[v * N3 + base + e * stride], s);
            g[v] = s;
        }
        lin_flux(d, lam, mu, lam2, irho, g, f);
        const double sc = dt * idx[d] * B.winv[aa[d]];
#pragma unroll
        for (int v = 0; v < NLV; ++v) us[v] = fma(sc, f[v], us[v]);
    }
#pragma unroll
    for (int v = 0; v < NLV; ++v) ustar[(int64_t(v) * nc + c) * N3 + a] = us[v];
    // face projections: threads with a_d = 0 write side 2d, a_d = N-1 side 2d+1
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int stride = d == 0 ? 1 : (d == 1 ? N : N2);
        const int base = a - aa[d] * stride;
        const int b = d == 0 ? aa[1] + N * aa[2] : (d == 1 ? aa[0] + N * aa[2] : aa[0] + N * aa[1]);
        for (int plus = 0; plus < 2; ++plus) {
            if (aa[d] != (plus ? N - 1 : 0)) continue;
            const double *E = plus ? B.R : B.L;
            double qf[NLV], f[NLV];
#pragma unroll
            for (int v = 0; v < NLV; ++v) {
                double s = 0.0;
#pragma unroll
                for (int e = 0; e < N; ++e) s = fma(E[e], dk[v * N3 + base + e * stride], s);
                qf[v] = s;
            }
            lin_flux(d, lam, mu, lam2, irho, qf, f);
            const int side = 2 * d + plus;
#pragma unroll
            for (int v = 0; v < NLV; ++v) {
                traces[((int64_t(side * 2 + 0) * NLV + v) * nc + c) * N2 + b] = qf[v];
                if constexpr (FTR) traces[((int64_t(side * 2 + 1) * NLV + v) * nc + c) * N2 + b] = f[v];
            }
        }
    }
}

// The elastic predictor at N = 4 on one wavefront per cell (lane = node
// a = a0 + 4 a1 + 16 a2, as the FP64 Euler predictor), with nothing staged in
// LDS: x and y contractions by DPP, z on v_mfma_f64_4x4x4f64.  The material
// is constant in a cell, so the flux matrix A_d commutes with the derivative
// along d: each application of L forms A_d of the node's state first and then
// contracts, -sum_d (1/dx_d) D_d (A_d dk); the volume term likewise contracts
// A_d qbar with the weak stiffness.  The same quantities as k_lin_predictor,
// in another order of rounding.  FTR as there.  Three waves per SIMD (144
// VGPRs; at two, 172 VGPRs, the 81^3 step took 4.73 instead of 4.48 ms; at
// four it spills).
template <bool FTR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_lin_predictor4(const double *__restrict__ u, const double *__restrict__ mat, const double *__restrict__ dt_dev,
                 double *__restrict__ ustar, double *__restrict__ traces, int64_t nc, double idx0, double idx1,
                 double idx2)
{
    constexpr int N = 4, N2 = 16, N3 = 64;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t c = int64_t(blockIdx.x) * 4 + wave;
    if (c >= nc) return;  // whole wavefront leaves together
    const DevBasis &B = c_basis[N];
    const int l = threadIdx.x & 63;
    const int a0 = l & 3, a1 = (l >> 2) & 3, a2 = l >> 4;
    // neighbour e of this lane along x (quad permutation) and y (row
    // rotation), as in the FP64 Euler predictor; the z operator as this
    // lane's MFMA A entry (row zi, column zk)
    const int nx[4] = {a0, (a0 + 1) & 3, (a0 + 2) & 3, (a0 + 3) & 3};
    const int ny[4] = {a1, (a1 + 3) & 3, (a1 + 2) & 3, (a1 + 1) & 3};
    const int zi = l & 3, zk = l >> 4;
    const double rho = mat[c], lam = mat[nc + c], mu = mat[2 * nc + c];
    const double lam2 = lam + 2.0 * mu, irho = 1.0 / rho;
    const double dt = dt_dev[0];
    const double idx[3] = {idx0, idx1, idx2};
    double uc[NLV], dk[NLV], qbar[NLV];
#pragma unroll
    for (int v = 0; v < NLV; ++v) {
        uc[v] = u[(int64_t(v) * nc + c) * N3 + l];
        dk[v] = uc[v];
        qbar[v] = uc[v];
    }
    // -(1/dx_d) D_d rows of this lane
    double Cx[4], Cy[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        Cx[e] = -idx[0] * B.D[a0 * N + nx[e]];
        Cy[e] = -idx[1] * B.D[a1 * N + ny[e]];
    }
    const double Az = -idx[2] * B.D[zi * N + zk];
    double fac = 1.0;
    for (int k = 1; k < N; ++k) {
        double nd[NLV], f[NLV];
        lin_flux(0, lam, mu, lam2, irho, dk, f);
#pragma unroll
        for (int v = 0; v < NLV; ++v) nd[v] = fibre_sum64<0>(Cx, f[v], 0.0);
        lin_flux(1, lam, mu, lam2, irho, dk, f);
#pragma unroll
        for (int v = 0; v < NLV; ++v) nd[v] = fibre_sum64<1>(Cy, f[v], nd[v]);
        lin_flux(2, lam, mu, lam2, irho, dk, f);
#pragma unroll
        for (int v = 0; v < NLV; ++v) nd[v] = zsum64(Az, f[v], nd[v]);
        fac *= dt / (k + 1);
#pragma unroll
        for (int v = 0; v < NLV; ++v) {
            dk[v] = nd[v];
            qbar[v] = fma(fac, nd[v], qbar[v]);
        }
    }
    // volume term: u + sum_d (dt/dx_d) (1/w_{a_d}) Kw_d (A_d qbar)
    {
        double Vx[4], Vy[4], us[NLV], f[NLV];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Vx[e] = dt * idx[0] * B.winv[a0] * B.Kw[a0 * N + nx[e]];
            Vy[e] = dt * idx[1] * B.winv[a1] * B.Kw[a1 * N + ny[e]];
        }
        const double Vz = dt * idx[2] * B.winv[zi] * B.Kw[zi * N + zk];
        lin_flux(0, lam, mu, lam2, irho, qbar, f);
#pragma unroll
        for (int v = 0; v < NLV; ++v) us[v] = fibre_sum64<0>(Vx, f[v], 0.0);
        lin_flux(1, lam, mu, lam2, irho, qbar, f);
#pragma unroll
        for (int v = 0; v < NLV; ++v) us[v] = fibre_sum64<1>(Vy, f[v], us[v]);
        lin_flux(2, lam, mu, lam2, irho, qbar, f);
#pragma unroll
        for (int v = 0; v < NLV; ++v) {
            us[v] = zsum64(Vz, f[v], us[v]);
            ustar[(int64_t(v) * nc + c) * N3 + l] = uc[v] + us[v];
        }
    }
    // face projections: along each axis the lanes at index 0 hold the minus
    // face (L weights) and those at index 3 the plus face (R weights) of one
    // sum, then the normal flux of that state
    double Px[4], Py[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        Px[e] = a0 == 0 ? B.L[nx[e]] : B.R[nx[e]];
        Py[e] = a1 == 0 ? B.L[ny[e]] : B.R[ny[e]];
    }
    const double Pz = zi == 0 ? B.L[zk] : B.R[zk];
    const int bf[3] = {a1 + N * a2, a0 + N * a2, a0 + N * a1};
    const int ad[3] = {a0, a1, a2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double qf[NLV], f[NLV];
#pragma unroll
        for (int v = 0; v < NLV; ++v)
            qf[v] = d == 0 ? fibre_sum64<0>(Px, qbar[v], 0.0)
                           : (d == 1 ? fibre_sum64<1>(Py, qbar[v], 0.0) : zsum64(Pz, qbar[v], 0.0));
        if (ad[d] == 0 || ad[d] == N - 1) {
            const int side = 2 * d + (ad[d] == 0 ? 0 : 1);
            if constexpr (FTR) lin_flux(d, lam, mu, lam2, irho, qf, f);
#pragma unroll
            for (int v = 0; v < NLV; ++v) {
                traces[((int64_t(side * 2 + 0) * NLV + v) * nc + c) * N2 + bf[d]] = qf[v];
                if constexpr (FTR) traces[((int64_t(side * 2 + 1) * NLV + v) * nc + c) * N2 + bf[d]] = f[v];
            }
        }
    }
}

// Rusanov on the +d faces: thread per (cell, face node); both sides written.
template <int N>
__global__ void __launch_bounds__(256)
k_lin_riemann(const double *__restrict__ traces, const double *__restrict__ mat, double *__restrict__ fside, int64_t nc,
              int d, int n0, int n1, int n2)
{
    constexpr int N2 = N * N;
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nc * N2) return;
    const int64_t c = t / N2;
    const int b = int(t % N2);
    const int64_t i = c % n0, j = (c / n0) % n1, k = c / (int64_t(n0) * n1);
    const int64_t cp = d == 0 ? ((i + 1) % n0) + n0 * (j + int64_t(n1) * k)
                              : (d == 1 ? i + n0 * (((j + 1) % n1) + int64_t(n1) * k)
                                        : i + n0 * (j + int64_t(n1) * ((k + 1) % n2)));
    const double sl = sqrt((mat[nc + c] + 2.0 * mat[2 * nc + c]) / mat[c]);
    const double sr = sqrt((mat[nc + cp] + 2.0 * mat[2 * nc + cp]) / mat[cp]);
    const double s = fmax(sl, sr);
    const int side_l = 2 * d + 1, side_r = 2 * d;
#pragma unroll
    for (int v = 0; v < NLV; ++v) {
        const double QL = traces[((int64_t(side_l * 2 + 0) * NLV + v) * nc + c) * N2 + b];
        const double FL = traces[((int64_t(side_l * 2 + 1) * NLV + v) * nc + c) * N2 + b];
        const double QR = traces[((int64_t(side_r * 2 + 0) * NLV + v) * nc + cp) * N2 + b];
        const double FR = traces[((int64_t(side_r * 2 + 1) * NLV + v) * nc + cp) * N2 + b];
        const double F = 0.5 * (FL + FR) - 0.5 * s * (QR - QL);
        fside[(int64_t(side_l * NLV + v) * nc + c) * N2 + b] = F;
        fside[(int64_t(side_r * NLV + v) * nc + cp) * N2 + b] = F;
    }
}

template <int N>
__global__ void __launch_bounds__(256)
k_lin_corrector(const double *__restrict__ ustar, const double *__restrict__ fside, const double *__restrict__ dt_dev,
                double *__restrict__ u, int64_t nc, double idx0, double idx1, double idx2)
{
    constexpr int N2 = N * N, N3 = N2 * N;
    const DevBasis &B = c_basis[N];
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nc * N3) return;
    const int64_t c = t / N3;
    const int a = int(t % N3), a0 = a % N, a1 = (a / N) % N, a2 = a / N2;
    const double dt = dt_dev[0];
    const double sx = dt * idx0 * B.winv[a0], sy = dt * idx1 * B.winv[a1], sz = dt * idx2 * B.winv[a2];
    const int bx = a1 + N * a2, by = a0 + N * a2, bz = a0 + N * a1;
#pragma unroll
    for (int v = 0; v < NLV; ++v) {
        auto F = [&](int side, int b) { return fside[(int64_t(side * NLV + v) * nc + c) * N2 + b]; };
        const double s = sx * (B.R[a0] * F(1, bx) - B.L[a0] * F(0, bx)) + sy * (B.R[a1] * F(3, by) - B.L[a1] * F(2, by)) +
                         sz * (B.R[a2] * F(5, bz) - B.L[a2] * F(4, bz));
        const int64_t o = (int64_t(v) * nc + c) * N3 + a;
        u[o] = ustar[o] - s;
    }
}

// The elastic step's faces inside its corrector at N = 4: one wavefront per
// cell, four cells per block, cells visited by TileWalk.  Rows of 16 lanes
// take one face each (faces 0-3, then 4-5), lane b of a row face node b; the
// face's flux is that of k_lin_riemann (same operands, same operations), so
// both cells of a face get its bits, and the update through the block's LDS
// is that of k_lin_corrector.  No face-flux array is written or read, and
// the normal-flux traces are formed from the state traces with the
// predictor's lin_flux and material terms (the values it would have stored),
// so only the state traces are read.
__global__ void __launch_bounds__(256)
k_lin_face_corrector4(const double *__restrict__ ustar, const double *__restrict__ traces,
                      const double *__restrict__ mat, const double *__restrict__ dt_dev, double *__restrict__ u,
                      int64_t nc, int nx, int ny, int nz, int tx, int ty, int tz, double idx0, double idx1,
                      double idx2)
{
    constexpr int N = 4, N2 = 16, N3 = 64;
    __shared__ double fs[4 * 6 * NLV * N2];
    const int l = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    double *fw = fs + wave * (6 * NLV * N2);
    const DevBasis &B = c_basis[N];
    const int b = l & 15;
    const int a0 = l % N, a1 = (l / N) % N, a2 = l / N2;
    const int bx = a1 + N * a2, by = a0 + N * a2, bz = a0 + N * a1;
    const double dt = dt_dev[0];
    const double sx = dt * idx0 * B.winv[a0], sy = dt * idx1 * B.winv[a1], sz = dt * idx2 * B.winv[a2];
    const int64_t nxy = int64_t(nx) * ny;
    const TileWalk walk(nx, ny, nz, tx, ty, tz);  // slots past the mesh's edge are idle wavefronts
    for (int64_t unit = walk.first; unit < walk.ue; unit += walk.stride) {
        int64_t c, ijk[3];
        const bool cell_ok = walk.cell(unit, wave, c, ijk);  // uniform per wavefront
        if (cell_ok) {
            const int64_t ext[3] = {nx, ny, nz}, str[3] = {1, nx, nxy};
#pragma unroll 1
            for (int r = 0; r < 2; ++r) {
                const int side = 4 * r + (l >> 4);
                if (side < 6) {
                    const int d = side >> 1, plus = side & 1;
                    // the neighbour across this side (periodic)
                    const int64_t q = ijk[d] + (plus ? 1 : -1);
                    const int64_t qn = q < 0 ? q + ext[d] : (q >= ext[d] ? q - ext[d] : q);
                    const int64_t n = c + (qn - ijk[d]) * str[d];
                    // the minus cell's plus side on the left, the plus cell's minus side on the right
                    const int64_t cl = plus ? c : n, cr = plus ? n : c;
                    const double sl = sqrt((mat[nc + cl] + 2.0 * mat[2 * nc + cl]) / mat[cl]);
                    const double sr = sqrt((mat[nc + cr] + 2.0 * mat[2 * nc + cr]) / mat[cr]);
                    const double sp = fmax(sl, sr);
                    const int side_l = 2 * d + 1, side_r = 2 * d;
                    double QL[NLV], QR[NLV], FL[NLV], FR[NLV];
#pragma unroll
                    for (int v = 0; v < NLV; ++v) {
                        QL[v] = traces[((int64_t(side_l * 2 + 0) * NLV + v) * nc + cl) * N2 + b];
                        QR[v] = traces[((int64_t(side_r * 2 + 0) * NLV + v) * nc + cr) * N2 + b];
                    }
                    {
                        const double rho = mat[cl], lam = mat[nc + cl], mu = mat[2 * nc + cl];
                        const double lam2 = lam + 2.0 * mu, irho = 1.0 / rho;
                        lin_flux(d, lam, mu, lam2, irho, QL, FL);
                    }
                    {
                        const double rho = mat[cr], lam = mat[nc + cr], mu = mat[2 * nc + cr];
                        const double lam2 = lam + 2.0 * mu, irho = 1.0 / rho;
                        lin_flux(d, lam, mu, lam2, irho, QR, FR);
                    }
                    // rounded as the predictor stores them: without the pin the compiler
                    // fuses the flux products into the sum below (other bits)
#pragma unroll
                    for (int v = 0; v < NLV; ++v) asm volatile("" : "+v"(FL[v]), "+v"(FR[v]));
#pragma unroll
                    for (int v = 0; v < NLV; ++v)
                        fw[(side * NLV + v) * N2 + b] = 0.5 * (FL[v] + FR[v]) - 0.5 * sp * (QR[v] - QL[v]);
                }
            }
        }
        __syncthreads();
        if (cell_ok) {
#pragma unroll
            for (int v = 0; v < NLV; ++v) {
                auto F = [&](int side, int bb) { return fw[(side * NLV + v) * N2 + bb]; };
                const double s = sx * (B.R[a0] * F(1, bx) - B.L[a0] * F(0, bx)) +
                                 sy * (B.R[a1] * F(3, by) - B.L[a1] * F(2, by)) +
                                 sz * (B.R[a2] * F(5, bz) - B.L[a2] * F(4, bz));
                const int64_t o = (int64_t(v) * nc + c) * N3 + l;
                u[o] = ustar[o] - s;
            }
        }
        __syncthreads();  // the next cells overwrite the fluxes
    }
}

// dt = factor / max_c c_p(c) (one block); factor = cfl / ((2p+1) sum_d 1/dx_d)
__global__ void __launch_bounds__(1024)
k_lin_cfl(const double *__restrict__ mat, int64_t nc, double factor, double *__restrict__ dt_out)
{
    __shared__ double sh[16];
    double m = 0.0;
    for (int64_t c = threadIdx.x; c < nc; c += blockDim.x)
        m = fmax(m, sqrt((mat[nc + c] + 2.0 * mat[2 * nc + c]) / mat[c]));
    m = block_max(m, sh);
    if (threadIdx.x == 0) dt_out[0] = (m > 0.0 && m < INFINITY) ? factor / m : 0.0;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

#define ADG_DISPATCH_N(N_, ...)                      \
    switch (N_) {                                    \
    case 1: { constexpr int NN = 1; __VA_ARGS__; } break; \
    case 2: { constexpr int NN = 2; __VA_ARGS__; } break; \
    case 3: { constexpr int NN = 3; __VA_ARGS__; } break; \
    case 4: { constexpr int NN = 4; __VA_ARGS__; } break; \
    case 5: { constexpr int NN = 5; __VA_ARGS__; } break; \
    case 6: { constexpr int NN = 6; __VA_ARGS__; } break; \
    case 7: { constexpr int NN = 7; __VA_ARGS__; } break; \
    default: return hipErrorInvalidValue;            \
    }

bool g_pred4_mfma = true;
bool g_pred4_f64 = true;
bool g_lin_pred4 = true;

hipError_t upload_basis(const DevBasis *tab)
{
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_basis), tab, sizeof(DevBasis) * (NMAX + 1));
    if (e != hipSuccess) return e;
    // lane rows of the N = 4 FP32 predictor (layout at c_lane4)
    const DevBasis &B = tab[4];
    constexpr int N = 4;
    std::vector<float> lane(64 * LANE4);
    for (int l = 0; l < 64; ++l) {
        const int a[3] = {l & 3, (l >> 2) & 3, l >> 4};
        float *r = &lane[l * LANE4];
        for (int e = 0; e < 4; ++e) {
            // neighbour visited at step e of each axis' rotation
            const int nx = (a[0] + e) & 3, ny = (a[1] - e) & 3, nz = (a[2] + e) & 3;
            r[e] = float(B.D[a[0] * N + nx]);
            r[4 + e] = float(B.D[a[1] * N + ny]);
            r[8 + e] = float(B.D[a[2] * N + nz]);
            r[12 + e] = float(B.KW[a[0] * N + e]);
            r[16 + e] = float(B.Kw[a[0] * N + nx] * B.winv[a[0]]);
            r[20 + e] = float(B.Kw[a[1] * N + ny] * B.winv[a[1]]);
            r[24 + e] = float(B.Kw[a[2] * N + nz] * B.winv[a[2]]);
            r[28 + e] = float(a[0] == 0 ? B.L[nx] : B.R[nx]);
            r[32 + e] = float(a[1] == 0 ? B.L[ny] : B.R[ny]);
            r[36 + e] = float(a[2] == 0 ? B.L[nz] : B.R[nz]);
        }
    }
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_lane4), lane.data(), sizeof(float) * lane.size());
    if (e != hipSuccess) return e;
    float kws[4];
    for (int j = 0; j < 4; ++j) kws[j] = float(B.KWsum[j]);
    e = hipMemcpyToSymbol(HIP_SYMBOL(c_kwsum4), kws, sizeof(kws));
    if (e != hipSuccess) return e;
    std::vector<double> corr(64 * 6);
    for (int l = 0; l < 64; ++l) {
        const int a[3] = {l & 3, (l >> 2) & 3, l >> 4};
        for (int d = 0; d < 3; ++d) {
            corr[l * 6 + d] = B.R[a[d]] * B.winv[a[d]];
            corr[l * 6 + 3 + d] = B.L[a[d]] * B.winv[a[d]];
        }
    }
    return hipMemcpyToSymbol(HIP_SYMBOL(c_corr4), corr.data(), sizeof(double) * corr.size());
}

template <typename T>
hipError_t launch_predictor(int N, const double *u, double *ustar, T *traces, const int32_t *list,
                            int64_t nlist, int64_t nc, const int8_t *level, const Geo &geo,
                            const double *dt, double gamma, int npic, hipStream_t st, T *iters)
{
    if (nlist <= 0) return hipSuccess;
    if constexpr (std::is_same<T, float>::value) {
        if (N == 4 && iters == nullptr && g_pred4_mfma) {
            const int64_t blocks = (nlist + 3) / 4;
            hipLaunchKernelGGL(k_predictor4_mfma, dim3(unsigned(blocks)), dim3(256), 0, st, u, ustar, traces, list,
                               nlist, nc, level, geo, dt, gamma, npic);
            return hipGetLastError();
        }
    } else {
        if (N == 4 && g_pred4_f64) {
            const int64_t blocks = (nlist + 3) / 4;
            if (iters)
                hipLaunchKernelGGL(k_predictor4_f64<true>, dim3(unsigned(blocks)), dim3(256), 0, st, u, ustar, traces,
                                   list, nlist, nc, level, geo, dt, gamma, npic, iters);
            else
                hipLaunchKernelGGL(k_predictor4_f64<false>, dim3(unsigned(blocks)), dim3(256), 0, st, u, ustar,
                                   traces, list, nlist, nc, level, geo, dt, gamma, npic, iters);
            return hipGetLastError();
        }
    }
    ADG_DISPATCH_N(N, {
        constexpr int CPB = PredCfg<NN>::CPB;
        const int64_t blocks = (nlist + CPB - 1) / CPB;
        if (iters)
            hipLaunchKernelGGL((k_predictor<T, NN, CPB, true>), dim3(unsigned(blocks)),
                               dim3(round64(CPB * NN * NN * NN)), 0, st, u, ustar, traces, list, nlist, nc, level, geo,
                               dt, gamma, npic, iters);
        else
            hipLaunchKernelGGL((k_predictor<T, NN, CPB, false>), dim3(unsigned(blocks)),
                               dim3(round64(CPB * NN * NN * NN)), 0, st, u, ustar, traces, list, nlist, nc, level, geo,
                               dt, gamma, npic, iters);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_riemann(int N, const T *traces, T *fside, const int32_t *fm, const int32_t *fp,
                          int64_t nf, int d, int64_t nc, double gamma, int *status, hipStream_t st,
                          int16_t *tape, int tape_mode)
{
    if (nf <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        constexpr int FPB = FaceCfg<NN>::FPB;
        const int64_t blocks = (nf + FPB - 1) / FPB;
        if (nc * NN * NN * int64_t(sizeof(T)) < (int64_t(1) << 31))
            hipLaunchKernelGGL((k_riemann<T, NN, true>), dim3(unsigned(blocks)), dim3(FaceCfg<NN>::THREADS), 0, st,
                               traces, fside, fm, fp, nf, d, nc, gamma, status, tape, tape_mode);
        else
            hipLaunchKernelGGL((k_riemann<T, NN, false>), dim3(unsigned(blocks)), dim3(FaceCfg<NN>::THREADS), 0, st,
                               traces, fside, fm, fp, nf, d, nc, gamma, status, tape, tape_mode);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_hang(int N, const T *traces, T *fside, const HangDev *hang, int64_t nh, int64_t nc,
                       const double *ptab, double gamma, int *status, hipStream_t st)
{
    if (nh <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        constexpr int FPB = FaceCfg<NN>::FPB;
        const int64_t blocks = (nh + FPB - 1) / FPB;
        hipLaunchKernelGGL((k_hang<T, NN>), dim3(unsigned(blocks)), dim3(FaceCfg<NN>::THREADS), 0, st,
                           traces, fside, hang, nh, nc, ptab, gamma, status);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(int N, T *fside, const HangDev *hang, const int32_t *ccell, const int8_t *cside,
                           const int32_t *cptr, const int32_t *cchild, int64_t ncs, int64_t nc,
                           const double *ptab, hipStream_t st)
{
    if (ncs <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        const int64_t blocks = (ncs * NN * NN + 255) / 256;
        hipLaunchKernelGGL((k_restrict<T, NN>), dim3(unsigned(blocks)), dim3(256), 0, st,
                           fside, hang, ccell, cside, cptr, cchild, ncs, nc, ptab);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_corrector(int N, const double *ustar, const T *fside, const double *dt, double *uout,
                            int64_t nc, const int8_t *level, const Geo &geo, hipStream_t st, double gamma,
                            double *partial, int *status, int64_t c0, int64_t c1)
{
    if (c1 < 0) c1 = nc;
    if (c1 <= c0) return hipSuccess;
    const int64_t blocks = corrector_blocks(N, c1 - c0);
    ADG_DISPATCH_N(N, {
        if constexpr (NN == 4) {
            if (partial)
                hipLaunchKernelGGL((k_corrector4<T, true>), dim3(unsigned(blocks)), dim3(256), 0, st, ustar, fside,
                                   dt, uout, nc, level, geo, gamma, partial, status, c0, c1);
            else
                hipLaunchKernelGGL((k_corrector4<T, false>), dim3(unsigned(blocks)), dim3(256), 0, st, ustar, fside,
                                   dt, uout, nc, level, geo, gamma, partial, status, c0, c1);
        } else if constexpr (NN >= 5) {
            if (partial)
                hipLaunchKernelGGL((k_correctorW<T, NN, true>), dim3(unsigned(blocks)), dim3(CorrW<NN>::THREADS), 0,
                                   st, ustar, fside, dt, uout, nc, level, geo, gamma, partial, status, c0, c1);
            else
                hipLaunchKernelGGL((k_correctorW<T, NN, false>), dim3(unsigned(blocks)), dim3(CorrW<NN>::THREADS), 0,
                                   st, ustar, fside, dt, uout, nc, level, geo, gamma, partial, status, c0, c1);
        } else {
            if (partial)
                hipLaunchKernelGGL((k_corrector<T, NN, true>), dim3(unsigned(blocks)), dim3(256), 0, st, ustar,
                                   fside, dt, uout, nc, level, geo, gamma, partial, status, c0, c1);
            else
                hipLaunchKernelGGL((k_corrector<T, NN, false>), dim3(unsigned(blocks)), dim3(256), 0, st, ustar,
                                   fside, dt, uout, nc, level, geo, gamma, partial, status, c0, c1);
        }
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_face_corrector4(const double *ustar, const T *traces, const double *dt, double *uout, int64_t nc,
                                  const int n[3], const Geo &geo, double gamma, double *partial, int *status,
                                  hipStream_t st)
{
    const int64_t blocks = corrector_blocks(4, nc);
    int tx, ty, tz;
    face_tiles(n, tx, ty, tz);
    if (partial)
        hipLaunchKernelGGL((k_face_corrector4<T, true>), dim3(unsigned(blocks)), dim3(256), 0, st, ustar, traces, dt,
                           uout, nc, n[0], n[1], n[2], tx, ty, tz, geo, gamma, partial, status);
    else
        hipLaunchKernelGGL((k_face_corrector4<T, false>), dim3(unsigned(blocks)), dim3(256), 0, st, ustar, traces, dt,
                           uout, nc, n[0], n[1], n[2], tx, ty, tz, geo, gamma, partial, status);
    return hipGetLastError();
}

int pred_variant_count() { return PRED_VARIANTS; }

void pred_variant_shape(int code, int *N, int *CPB)
{
    switch (code) {
#define ADG_SHAPE(code_, NN, CC) \
    case code_: *N = NN; *CPB = CC; return;
        ADG_PRED_VARIANTS(ADG_SHAPE)
#undef ADG_SHAPE
    default: *N = 0; *CPB = 0;
    }
}


template <typename T>
hipError_t launch_predictor_batch(const PredItem *items, int64_t nitems, const PredInst *insts, const double *u,
                                  double *ustar, T *traces, const double *dt, int threads, int grid,
                                  hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    size_t lds = 0;
    for (int c = 0; c < PRED_VARIANTS; ++c) {
        int N, CPB;
        pred_variant_shape(c, &N, &CPB);
        if (round64(CPB * N * N * N) <= threads) lds = std::max(lds, size_t(pred_lds_elems(N, CPB, int(sizeof(T)))) * sizeof(T));
    }
    hipLaunchKernelGGL(k_predictor_batch<T>, dim3(grid), dim3(threads), lds, st, items, nitems, insts, u, ustar,
                       traces, dt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_predictor_order(int code, const PredItem *items, int64_t nitems, const PredInst *insts,
                                  const double *u, double *ustar, T *traces, const double *dt, int n_cu,
                                  hipStream_t st)
{
    if (nitems <= 0) return hipSuccess;
    if constexpr (std::is_same<T, float>::value) {
        int vn, cpb;
        pred_variant_shape(code, &vn, &cpb);
        if (vn == 4 && g_pred4_mfma) {
            int occ = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_predictor4_mfma_order, 256, 0) != hipSuccess ||
                occ < 1)
                occ = 1;
            const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nitems, int64_t(occ) * n_cu));
            hipLaunchKernelGGL(k_predictor4_mfma_order, dim3(unsigned(grid)), dim3(256), 0, st, items, nitems, insts,
                               u, ustar, traces, dt, cpb);
            return hipGetLastError();
        }
    }
    switch (code) {
#define ADG_ORDER_CASE(code_, NN, CC)                                                                            \
    case code_: {                                                                                                \
        constexpr int TH = round64(CC * NN * NN * NN);                                                           \
        int occ = 0;                                                                                             \
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_predictor_order<T, NN, CC>, TH, 0) != hipSuccess \
            || occ < 1)                                                                                          \
            occ = 1;                                                                                             \
        const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(nitems, int64_t(occ) * n_cu));              \
        hipLaunchKernelGGL((k_predictor_order<T, NN, CC>), dim3(unsigned(grid)), dim3(TH), 0, st, items, nitems, \
                           insts, u, ustar, traces, dt);                                                         \
        break;                                                                                                   \
    }
        ADG_PRED_VARIANTS(ADG_ORDER_CASE)
#undef ADG_ORDER_CASE
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
int predictor_batch_occupancy(int threads)
{
    size_t lds = 0;
    for (int c = 0; c < PRED_VARIANTS; ++c) {
        int N, CPB;
        pred_variant_shape(c, &N, &CPB);
        if (round64(CPB * N * N * N) <= threads) lds = std::max(lds, size_t(pred_lds_elems(N, CPB, int(sizeof(T)))) * sizeof(T));
    }
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_predictor_batch<T>, threads, lds) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

int cfl_blocks(int N, int64_t nc)
{
    const int64_t total = nc * int64_t(N) * N * N;
    int64_t b = (total + 255) / 256;
    if (b > CFL_MAX_BLOCKS) b = CFL_MAX_BLOCKS;
    if (b < 1) b = 1;
    return int(b);
}

hipError_t launch_cfl(int N, const double *u, int64_t nc, const int8_t *level, const Geo &geo, double gamma,
                      double factor, double *partial, int *status, double *dt_out, double *hist,
                      hipStream_t st)
{
    const int nb = cfl_blocks(N, nc);
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_cfl_partial<NN>), dim3(nb), dim3(256), 0, st, u, nc, level, geo, gamma, partial,
                           status);
    });
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, st, partial, nb, factor, dt_out, hist, 0.0,
                       static_cast<double *>(nullptr));
    return hipGetLastError();
}

// Tiles of the fused face kernels' cell walk: about 12 x 9 x 9 cells (about
// what the chip holds in flight); tx, a multiple of 4, leaves the fewest idle
// slots along x (closest to 12 among equals: 12 at 81 cells, 4 at 27).
void face_tiles(const int n[3], int &tx, int &ty, int &tz)
{
    tx = 4;
    for (int t = 4, best = 1 << 30; t <= 28; t += 4) {
        const int padded = (n[0] + t - 1) / t * t;
        if (padded < best || (padded == best && std::abs(t - 12) < std::abs(tx - 12))) best = padded, tx = t;
    }
    ty = std::min(9, n[1]);
    tz = std::min(9, n[2]);
}

int corrector_blocks(int N, int64_t nc)
{
    const int64_t b = (nc * N * N * N + 255) / 256;
    return int(std::max<int64_t>(1, std::min<int64_t>(b, CORRECTOR_MAX_BLOCKS)));
}

hipError_t launch_cfl_prime(int N, const double *u, int64_t nc, const int8_t *level, const Geo &geo, double gamma,
                            double *partial, int nb, int *status, hipStream_t st)
{
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_cfl_partial<NN>), dim3(nb), dim3(256), 0, st, u, nc, level, geo, gamma, partial,
                           status);
    });
    return hipGetLastError();
}

hipError_t launch_cfl_final(const double *partial, int nparts, double factor, double *dt_out, double *hist,
                            hipStream_t st, double t_end, double *clock)
{
    hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(1024), 0, st, partial, nparts, factor, dt_out, hist, t_end, clock);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double x, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, p, n, x);
    return hipGetLastError();
}

hipError_t launch_node_coords(int N, double *xyz, const int32_t *ijk, const int8_t *level, int64_t nc,
                              const Geo &geo, const double *lo, hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        const int64_t blocks = (nc * NN * NN * NN + 255) / 256;
        hipLaunchKernelGGL((k_node_coords<NN>), dim3(unsigned(blocks)), dim3(256), 0, st, xyz, ijk, level, nc,
                           geo, lo[0], lo[1], lo[2]);
    });
    return hipGetLastError();
}


hipError_t launch_adjoint_step(int N, const double *u, const double *dt, const double *ubar_next, double *ubar,
                               double *ustar, double *traces, double *tbar, double *fbar, double *iters,
                               const int32_t *const fm[3], const int32_t *const fp[3], const int64_t nf[3],
                               int64_t nc, const int8_t *level, const Geo &geo, double gamma, int npic,
                               const AdjHang &ah, hipStream_t st, bool forward)
{
    // the forward predictor with its iterates, unless the caller recorded them
    if (forward) {
        hipError_t e = launch_predictor<double>(N, u, ustar, traces, nullptr, nc, nc, level, geo, dt, gamma, npic,
                                                st, iters);
        if (e != hipSuccess) return e;
    }
    ADG_DISPATCH_N(N, {
        constexpr int N2 = NN * NN;
        constexpr int FPB = FaceCfg<NN>::FPB;
        const int64_t items = 6 * int64_t(NV) * nc * N2;
        if (NN == 4)
            hipLaunchKernelGGL(k_corrector_adj4, dim3(unsigned((nc + 3) / 4)), dim3(256), 0, st, ubar_next, fbar, dt,
                               nc, level, geo);
        else
            hipLaunchKernelGGL((k_corrector_adj<NN>), dim3(unsigned((items + 255) / 256)), dim3(256), 0, st,
                               ubar_next, fbar, dt, nc, level, geo);
        if (ah.nh > 0)
            hipLaunchKernelGGL((k_restrict_adj<NN>), dim3(unsigned((ah.nh * N2 + 255) / 256)), dim3(256), 0, st,
                               fbar, ah.hang, ah.nh, nc, ah.ptab);
        for (int d = 0; d < 3; ++d) {
            if (nf[d] <= 0) continue;
            hipLaunchKernelGGL((k_riemann_adj<NN>), dim3(unsigned((nf[d] + FPB - 1) / FPB)), dim3(FaceCfg<NN>::THREADS),
                               0, st, traces, fbar, tbar, fm[d], fp[d], nf[d], d, nc, gamma);
        }
        if (ah.nh > 0)
            hipLaunchKernelGGL((k_hang_adj<NN>), dim3(unsigned((ah.nh + FPB - 1) / FPB)), dim3(FaceCfg<NN>::THREADS),
                               0, st, traces, fbar, tbar, ah.vbar, ah.hang, ah.nh, nc, ah.ptab, gamma);
        if (ah.ncs > 0)
            hipLaunchKernelGGL((k_prolong_adj<NN>), dim3(unsigned((ah.ncs * N2 + 255) / 256)), dim3(256), 0, st,
                               tbar, ah.vbar, ah.hang, ah.ccell, ah.cside, ah.cptr, ah.cchild, ah.ncs, nc, ah.ptab);
        constexpr int CPB = PredCfg<NN>::CPB;
        if (NN == 4 && g_pred4_f64 && npic >= 1)
            hipLaunchKernelGGL(k_predictor4_adj_f64, dim3(unsigned((nc + 3) / 4)), dim3(256), 0, st, u, iters,
                               ubar_next, tbar, dt, ubar, nc, level, geo, gamma, npic);
        else
            hipLaunchKernelGGL((k_predictor_adj<NN, CPB>), dim3(unsigned((nc + CPB - 1) / CPB)),
                               dim3(round64(CPB * NN * NN * NN)), 0, st, u, iters, ubar_next, tbar, dt, ubar, nc,
                               level, geo, gamma, npic);
    });
    return hipGetLastError();
}

hipError_t launch_sample(int N, const double *u, int64_t nc, const SampleGeo &sg, const double *pts, int64_t npts,
                         double *out, hipStream_t st)
{
    if (npts <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_sample<NN>), dim3(unsigned((npts + 255) / 256)), dim3(256), 0, st, u, nc, sg, pts, npts,
                           out);
    });
    return hipGetLastError();
}

hipError_t launch_sample_adjoint(int N, const double *pts, const double *wbar, int64_t npts, const SampleGeo &sg,
                                 double *ubar, hipStream_t st)
{
    if (npts <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_sample_adj<NN>), dim3(unsigned(npts)), dim3(round64(NN * NN * NN)), 0, st, pts, wbar,
                           npts, sg, ubar);
    });
    return hipGetLastError();
}

hipError_t launch_indicator(int N, const double *u, int64_t nc, double *eta, hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_indicator<NN>), dim3(unsigned(nc)), dim3(round64(NN * NN * NN)), 0, st, u, nc, eta);
    });
    return hipGetLastError();
}

hipError_t launch_vtransfer(int N, const double *u_from, int64_t nc_from, double *u_to, int64_t nc_to,
                            const VOp *ops, const VKid *kids, const double *ptab, hipStream_t st)
{
    if (nc_to <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_vtransfer<NN>), dim3(unsigned(nc_to)), dim3(round64(NN * NN * NN)), 0, st, u_from,
                           nc_from, u_to, nc_to, ops, kids, ptab);
    });
    return hipGetLastError();
}

hipError_t upload_subcell(const DevSub *tab)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_sub), tab, sizeof(DevSub) * (LIM_NMAX + 1));
}

hipError_t launch_lim_nbr(const int32_t *fm, const int32_t *fp, int64_t nf, int d, int64_t nc, int32_t *nbr,
                          hipStream_t st)
{
    if (nf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lim_nbr, dim3(unsigned((nf + 255) / 256)), dim3(256), 0, st, fm, fp, nf, d, nc, nbr);
    return hipGetLastError();
}

hipError_t launch_lim_scan(int N, const double *u, int64_t nc, double gamma, const LimDev &L, bool listed,
                           hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        if (listed)
            hipLaunchKernelGGL((k_lim_scan<NN, true>), dim3(LIM_GRID), dim3(64), 0, st, u, nc, gamma, L.mm2, L.fb2,
                               L.rlist, L.cnt);
        else
            hipLaunchKernelGGL((k_lim_scan<NN, false>), dim3(unsigned(nc)), dim3(64), 0, st, u, nc, gamma, L.mm2,
                               L.fb2, L.rlist, L.cnt);
    });
    return hipGetLastError();
}

hipError_t launch_lim_copy(const double *u, int64_t n_u, int64_t nc, const LimDev &L, hipStream_t st)
{
    hipLaunchKernelGGL(k_lim_copy, dim3(4096), dim3(256), 0, st, u, n_u, nc, L.uold, L.mm2, L.mm, L.fb2, L.fb, L.cnt);
    return hipGetLastError();
}

hipError_t launch_lim_detect(int N, const double *u, int64_t nc, double gamma, double delta0, double eps, int force,
                             const LimDev &L, hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_lim_detect<NN>), dim3(unsigned(nc)), dim3(64), 0, st, u, nc, gamma, delta0, eps, force,
                           L.mm, L.nbr, L.flag, L.list, L.cnt, L.mm2, L.fb2);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lim_fv(int N, double *u, T *fside, int64_t nc, const Geo &geo, const double *dt, double gamma,
                         const LimDev &L, hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_lim_fv<T, NN>), dim3(LIM_GRID), dim3(LimCfg<NN>::THREADS), 0, st, u, fside, nc, geo, dt,
                           gamma, L.uold, L.fb, L.nbr, L.flag, L.list, L.rlist, L.cnt, L.mm2, L.fb2, L.level);
    });
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lim_recorrect(int N, const double *ustar, const T *fside, double *u, int64_t nc, const Geo &geo,
                                const double *dt, const LimDev &L, hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        hipLaunchKernelGGL((k_lim_recorrect<T, NN>), dim3(LIM_GRID), dim3(round64(NN * NN * NN)), 0, st, ustar, fside,
                           dt, u, nc, geo, L.rlist, L.cnt, L.level);
    });
    return hipGetLastError();
}

hipError_t launch_lin_face_corrector4(const double *ustar, const double *traces, const double *mat, const double *dt,
                                      double *u, int64_t nc, const int n[3], const double inv_dx[3], hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    int tx, ty, tz;
    face_tiles(n, tx, ty, tz);
    hipLaunchKernelGGL(k_lin_face_corrector4, dim3(unsigned(corrector_blocks(4, nc))), dim3(256), 0, st, ustar, traces,
                       mat, dt, u, nc, n[0], n[1], n[2], tx, ty, tz, inv_dx[0], inv_dx[1], inv_dx[2]);
    return hipGetLastError();
}

hipError_t launch_lin_cfl(const double *mat, int64_t nc, double factor, double *dt, hipStream_t st)
{
    hipLaunchKernelGGL(k_lin_cfl, dim3(1), dim3(1024), 0, st, mat, nc, factor, dt);
    return hipGetLastError();
}

hipError_t launch_lin_predictor(int N, const double *u, const double *mat, const double *dt, double *ustar,
                                double *traces, int64_t nc, const double inv_dx[3], hipStream_t st, bool flux_traces)
{
    if (nc <= 0) return hipSuccess;
    if (N == 4 && g_lin_pred4) {
        if (flux_traces)
            hipLaunchKernelGGL(k_lin_predictor4<true>, dim3(unsigned((nc + 3) / 4)), dim3(256), 0, st, u, mat, dt,
                               ustar, traces, nc, inv_dx[0], inv_dx[1], inv_dx[2]);
        else
            hipLaunchKernelGGL(k_lin_predictor4<false>, dim3(unsigned((nc + 3) / 4)), dim3(256), 0, st, u, mat, dt,
                               ustar, traces, nc, inv_dx[0], inv_dx[1], inv_dx[2]);
        return hipGetLastError();
    }
    ADG_DISPATCH_N(N, {
        constexpr int CPB = LinCfg<NN>::CPB;
        if (flux_traces)
            hipLaunchKernelGGL((k_lin_predictor<NN, true>), dim3(unsigned((nc + CPB - 1) / CPB)),
                               dim3(LinCfg<NN>::THREADS), 0, st, u, mat, dt, ustar, traces, nc, inv_dx[0], inv_dx[1],
                               inv_dx[2]);
        else
            hipLaunchKernelGGL((k_lin_predictor<NN, false>), dim3(unsigned((nc + CPB - 1) / CPB)),
                               dim3(LinCfg<NN>::THREADS), 0, st, u, mat, dt, ustar, traces, nc, inv_dx[0], inv_dx[1],
                               inv_dx[2]);
    });
    return hipGetLastError();
}

hipError_t launch_lin_riemann(int N, const double *traces, const double *mat, double *fside, int64_t nc,
                              const int n[3], hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        const int64_t work = nc * NN * NN;
        for (int d = 0; d < 3; ++d)
            hipLaunchKernelGGL((k_lin_riemann<NN>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, st, traces, mat,
                               fside, nc, d, n[0], n[1], n[2]);
    });
    return hipGetLastError();
}

hipError_t launch_lin_corrector(int N, const double *ustar, const double *fside, const double *dt, double *u,
                                int64_t nc, const double inv_dx[3], hipStream_t st)
{
    if (nc <= 0) return hipSuccess;
    ADG_DISPATCH_N(N, {
        const int64_t work = nc * NN * NN * NN;
        hipLaunchKernelGGL((k_lin_corrector<NN>), dim3(unsigned((work + 255) / 256)), dim3(256), 0, st, ustar, fside,
                           dt, u, nc, inv_dx[0], inv_dx[1], inv_dx[2]);
    });
    return hipGetLastError();
}

#define ADG_INSTANTIATE(T)                                                                              \
    template hipError_t launch_predictor<T>(int, const double *, double *, T *, const int32_t *, int64_t,  \
                                            int64_t, const int8_t *, const Geo &, const double *, double, \
                                            int, hipStream_t, T *);                                      \
    template hipError_t launch_riemann<T>(int, const T *, T *, const int32_t *, const int32_t *, int64_t, \
                                          int, int64_t, double, int *, hipStream_t, int16_t *, int);     \
    template hipError_t launch_hang<T>(int, const T *, T *, const HangDev *, int64_t, int64_t,           \
                                       const double *, double, int *, hipStream_t);                      \
    template hipError_t launch_restrict<T>(int, T *, const HangDev *, const int32_t *, const int8_t *,   \
                                           const int32_t *, const int32_t *, int64_t, int64_t,           \
                                           const double *, hipStream_t);                                 \
    template hipError_t launch_corrector<T>(int, const double *, const T *, const double *, double *,    \
                                            int64_t, const int8_t *, const Geo &, hipStream_t, double,    \
                                            double *, int *, int64_t, int64_t);                           \
    template hipError_t launch_face_corrector4<T>(const double *, const T *, const double *, double *,   \
                                                  int64_t, const int[3], const Geo &, double, double *,    \
                                                  int *, hipStream_t);

ADG_INSTANTIATE(double)
ADG_INSTANTIATE(float)
template hipError_t launch_lim_fv<double>(int, double *, double *, int64_t, const Geo &, const double *, double,
                                          const LimDev &, hipStream_t);
template hipError_t launch_lim_fv<float>(int, double *, float *, int64_t, const Geo &, const double *, double,
                                         const LimDev &, hipStream_t);
template hipError_t launch_lim_recorrect<double>(int, const double *, const double *, double *, int64_t,
                                                 const Geo &, const double *, const LimDev &, hipStream_t);
template hipError_t launch_lim_recorrect<float>(int, const double *, const float *, double *, int64_t, const Geo &,
                                                const double *, const LimDev &, hipStream_t);
template hipError_t launch_predictor_batch<double>(const PredItem *, int64_t, const PredInst *, const double *,
                                                  double *, double *, const double *, int, int, hipStream_t);
template hipError_t launch_predictor_batch<float>(const PredItem *, int64_t, const PredInst *, const double *,
                                                 double *, float *, const double *, int, int, hipStream_t);
template int predictor_batch_occupancy<double>(int);
template hipError_t launch_predictor_order<double>(int, const PredItem *, int64_t, const PredInst *, const double *,
                                                  double *, double *, const double *, int, hipStream_t);
template hipError_t launch_predictor_order<float>(int, const PredItem *, int64_t, const PredInst *, const double *,
                                                 double *, float *, const double *, int, hipStream_t);
template int predictor_batch_occupancy<float>(int);

}  // namespace adg
