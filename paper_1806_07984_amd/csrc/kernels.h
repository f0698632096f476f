// Launch wrappers of the HIP kernels (kernels.hip).  Every wrapper enqueues on
// the given stream and returns the launch status; none synchronises.
#pragma once

#include "adg_internal.h"

namespace adg {

constexpr int CFL_MAX_BLOCKS = 2048;
constexpr int CORRECTOR_MAX_BLOCKS = 16384;

// Hanging child face as the kernels read it.
struct HangDev {
    int32_t fine, coarse;
    int8_t d, fine_minus, dl, s1, s2, pad[3];
};

// first transfer block of level jump dl (blocks of 2 N^2 doubles: P then Rm,
// one per sub-position s < 3^dl)
__host__ __device__ constexpr int transfer_base(int dl)
{
    return dl == 1 ? 0 : (dl == 2 ? 3 : 12);
}
constexpr int TRANSFER_BLOCKS = 3 + 9 + 27;

hipError_t upload_basis(const DevBasis *tab);

// FP32, N = 4: use the LDS-free DPP/MFMA predictor (default) or the generic one
extern bool g_pred4_mfma;
extern bool g_pred4_f64;

// Batched predictor: one work item = CPB cells of one instance.
struct PredItem {
    int32_t inst;   // index into the PredInst table
    int32_t code;   // (N, CPB) variant, see pred_variant_shape
    int64_t first;  // first cell of the item
};
// per instance: offsets into the concatenated u / u* / traces arrays
struct PredInst {
    int64_t u_off, tr_off, nc;
    const int8_t *level;
    double gamma;
    int32_t npic, N;
    Geo geo;
};
constexpr int PRED_VARIANTS = 16;
int pred_variant_count();
void pred_variant_shape(int code, int *N, int *CPB);
template <typename T>
hipError_t launch_predictor_batch(const PredItem *items, int64_t nitems, const PredInst *insts, const double *u,
                                  double *ustar, T *traces, const double *dt, int threads, int grid,
                                  hipStream_t st);
template <typename T>
int predictor_batch_occupancy(int threads);
// persistent predictor over the items of one order (variant code)
template <typename T>
hipError_t launch_predictor_order(int code, const PredItem *items, int64_t nitems, const PredInst *insts,
                                  const double *u, double *ustar, T *traces, const double *dt, int n_cu,
                                  hipStream_t st);

template <typename T>
hipError_t launch_predictor(int N, const double *u, double *ustar, T *traces, const int32_t *list,
                            int64_t nlist, int64_t nc, const int8_t *level, const Geo &geo,
                            const double *dt, double gamma, int npic, hipStream_t st, T *iters = nullptr);
// Rusanov switch tape: TAPE_RECORD stores each face's maximiser (2 node +
// side) of the wave speed, TAPE_REPLAY uses the stored one instead of the max.
enum { TAPE_OFF = 0, TAPE_RECORD = 1, TAPE_REPLAY = 2 };
template <typename T>
hipError_t launch_riemann(int N, const T *traces, T *fside, const int32_t *fm, const int32_t *fp,
                          int64_t nf, int d, int64_t nc, double gamma, int *status, hipStream_t st,
                          int16_t *tape = nullptr, int tape_mode = TAPE_OFF);
template <typename T>
hipError_t launch_hang(int N, const T *traces, T *fside, const HangDev *hang, int64_t nh, int64_t nc,
                       const double *ptab, double gamma, int *status, hipStream_t st);
template <typename T>
hipError_t launch_restrict(int N, T *fside, const HangDev *hang, const int32_t *ccell, const int8_t *cside,
                           const int32_t *cptr, const int32_t *cchild, int64_t ncs, int64_t nc,
                           const double *ptab, hipStream_t st);
// Cells c0 .. c1-1 (c1 < 0: all nc cells).  partial != nullptr: also write
// the CFL maximum of the new state per block (corrector_blocks(N, c1 - c0)
// values) for the next step's launch_cfl_final.
template <typename T>
hipError_t launch_corrector(int N, const double *ustar, const T *fside, const double *dt, double *uout,
                            int64_t nc, const int8_t *level, const Geo &geo, hipStream_t st, double gamma = 0.0,
                            double *partial = nullptr, int *status = nullptr, int64_t c0 = 0, int64_t c1 = -1);
int corrector_blocks(int N, int64_t nc);
// tiles (tx x ty x tz cells) in which the fused face kernels visit an
// n[0] x n[1] x n[2] mesh
void face_tiles(const int n[3], int &tx, int &ty, int &tz);
// The conforming Riemann problems and the corrector in one kernel, for one
// uniform periodic instance at N = 4 with n[0] x n[1] x n[2] cells: the same
// bits as launch_riemann on every axis followed by launch_corrector (partial
// as there), without the face-flux array.
template <typename T>
hipError_t launch_face_corrector4(const double *ustar, const T *traces, const double *dt, double *uout, int64_t nc,
                                  const int n[3], const Geo &geo, double gamma, double *partial, int *status,
                                  hipStream_t st);
// block maxima of the CFL rate of u, nb blocks (the number of maxima the next
// launch_cfl_final reads)
hipError_t launch_cfl_prime(int N, const double *u, int64_t nc, const int8_t *level, const Geo &geo, double gamma,
                            double *partial, int nb, int *status, hipStream_t st);
// clock != nullptr: dt = min(dt, t_end - clock), then clock += dt (the
// last step of a run to t_end lands on it exactly)
hipError_t launch_cfl_final(const double *partial, int nparts, double factor, double *dt_out, double *hist,
                            hipStream_t st, double t_end = 0.0, double *clock = nullptr);
// p[0 .. n-1] = x
hipError_t launch_fill(double *p, int64_t n, double x, hipStream_t st);

// Dynamic adaptivity.  One target cell's relation to the source mesh:
// kind 0 copy of cell src; 1 evaluation of the coarser source cell src (dl
// levels up, sub-position s per axis); 2 L2 projection of the finer source
// cells kids[kid0 .. kid0+nkid) (each with its own dl and sub-position).
struct VOp {
    int32_t kind, src, kid0, nkid;
    int8_t dl, s[3];
};
struct VKid {
    int32_t cell;
    int8_t dl, s[3];
};
// refinement indicator per cell: max over nodes and axes of |d rho/d xi_d|
hipError_t launch_indicator(int N, const double *u, int64_t nc, double *eta, hipStream_t st);
hipError_t launch_vtransfer(int N, const double *u_from, int64_t nc_from, double *u_to, int64_t nc_to,
                            const VOp *ops, const VKid *kids, const double *ptab, hipStream_t st);

// A-posteriori subcell limiter (single-level meshes, N <= LIM_NMAX).
hipError_t upload_subcell(const DevSub *tab);
// Device buffers of the limiter of one mesh.
struct LimDev {
    double *uold;     // [5][nc][N^3] copy of the step's input
    double *mm;       // [nc][2][5] smallest / largest old subcell datum per variable
    int32_t *fb;      // [nc] 1: old subcell data replaced by the cell mean
    double *mm2;      // the same of the step's result (carried to the next step)
    int32_t *fb2;
    int32_t *nbr;     // [6][nc] same-level face neighbour of every cell side, -1 at a hanging side
    int32_t *flag;    // [nc] 1 limited, 2 corrector re-run, 3 troubled with a hanging
                      // side (not limited), 4 the same with its corrector re-run, 0 else
    int32_t *list;    // [nc] limited cells (first cnt[0] entries)
    int32_t *rlist;   // [nc] cells whose corrector runs again (first cnt[1])
    int32_t *cnt;     // [2]
    const int8_t *level;  // [nc] cell levels (adaptive meshes), else nullptr
};
constexpr int LIM_GRID = 2048;  // blocks of the persistent limiter kernels
hipError_t launch_lim_nbr(const int32_t *fm, const int32_t *fp, int64_t nf, int d, int64_t nc, int32_t *nbr,
                          hipStream_t st);
// subcell bounds and fall-back flags of u into mm2 / fb2: every cell, or
// (listed) the cells whose corrector ran again
hipError_t launch_lim_scan(int N, const double *u, int64_t nc, double gamma, const LimDev &L, bool listed,
                           hipStream_t st);
// start of a step: u -> uold, mm2 -> mm, fb2 -> fb; clears the counters
hipError_t launch_lim_copy(const double *u, int64_t n_u, int64_t nc, const LimDev &L, hipStream_t st);
// troubled-cell flags and list of the candidate u (force: every cell); the
// candidate's subcell bounds into mm2 / fb2
hipError_t launch_lim_detect(int N, const double *u, int64_t nc, double gamma, double delta0, double eps, int force,
                             const LimDev &L, hipStream_t st);
// FV update of the listed cells into u (and their new bounds into mm2 / fb2);
// projected face fluxes for their unlimited neighbours into fside, which are
// listed for the corrector re-run
template <typename T>
hipError_t launch_lim_fv(int N, double *u, T *fside, int64_t nc, const Geo &geo, const double *dt, double gamma,
                         const LimDev &L, hipStream_t st);
template <typename T>
hipError_t launch_lim_recorrect(int N, const double *ustar, const T *fside, double *u, int64_t nc, const Geo &geo,
                                const double *dt, const LimDev &L, hipStream_t st);

// Linear variant (elastic waves, 9 unknowns, uniform periodic mesh, FP64).
// mat: [3][nc] (rho, lambda, mu); factor = cfl / ((2p+1) sum_d 1/dx_d).
hipError_t launch_lin_cfl(const double *mat, int64_t nc, double factor, double *dt, hipStream_t st);
// flux_traces = false: only the state traces (array 0 of each side) are written
hipError_t launch_lin_predictor(int N, const double *u, const double *mat, const double *dt, double *ustar,
                                double *traces, int64_t nc, const double inv_dx[3], hipStream_t st,
                                bool flux_traces = true);
hipError_t launch_lin_riemann(int N, const double *traces, const double *mat, double *fside, int64_t nc,
                              const int n[3], hipStream_t st);
hipError_t launch_lin_corrector(int N, const double *ustar, const double *fside, const double *dt, double *u,
                                int64_t nc, const double inv_dx[3], hipStream_t st);
// N = 4: launch_lin_riemann followed by launch_lin_corrector in one kernel,
// the same bits, without the face-flux array; reads only the state traces.
hipError_t launch_lin_face_corrector4(const double *ustar, const double *traces, const double *mat, const double *dt,
                                      double *u, int64_t nc, const int n[3], const double inv_dx[3], hipStream_t st);

int cfl_blocks(int N, int64_t nc);
// factor = cfl / (2p + 1); writes dt_out[0] (and hist[0] if not null)
hipError_t launch_cfl(int N, const double *u, int64_t nc, const int8_t *level, const Geo &geo, double gamma,
                      double factor, double *partial, int *status, double *dt_out, double *hist,
                      hipStream_t st);
// Geometry of a uniform mesh for point location.
struct SampleGeo {
    int n[3];
    double lo[3], inv_h[3];
};

// Hanging-face tables of an adaptive instance for the adjoint step (nh = 0
// and ncs = 0 on uniform meshes); vbar is scratch of nh * 2 * 5 * N^2 doubles.
struct AdjHang {
    const HangDev *hang = nullptr;
    int64_t nh = 0;
    const int32_t *ccell = nullptr, *cptr = nullptr, *cchild = nullptr;
    const int8_t *cside = nullptr;
    int64_t ncs = 0;
    const double *ptab = nullptr;
    double *vbar = nullptr;
};

// One adjoint step (FP64): recomputes the predictor storing its iterates,
// then applies the transposed corrector, restriction, Riemann solves
// (conforming and hanging faces), interpolation to virtual cells and
// predictor.
hipError_t launch_adjoint_step(int N, const double *u, const double *dt, const double *ubar_next, double *ubar,
                               double *ustar, double *traces, double *tbar, double *fbar, double *iters,
                               const int32_t *const fm[3], const int32_t *const fp[3], const int64_t nf[3],
                               int64_t nc, const int8_t *level, const Geo &geo, double gamma, int npic,
                               const AdjHang &ah, hipStream_t st, bool forward = true);
hipError_t launch_sample(int N, const double *u, int64_t nc, const SampleGeo &sg, const double *pts, int64_t npts,
                         double *out, hipStream_t st);
hipError_t launch_sample_adjoint(int N, const double *pts, const double *wbar, int64_t npts, const SampleGeo &sg,
                                 double *ubar, hipStream_t st);
hipError_t launch_node_coords(int N, double *xyz, const int32_t *ijk, const int8_t *level, int64_t nc,
                              const Geo &geo, const double *lo, hipStream_t st);

}  // namespace adg
