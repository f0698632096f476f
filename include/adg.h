/*
 * adg.h -- C ABI of the MI355X (gfx950) ADER-DG time-step library.
 *
 * The library advances the 3-D compressible Euler equations
 *     dQ/dt + div F(Q) = 0,  Q = (rho, m1, m2, m3, E),  p = (gamma-1)(E - |m|^2/(2 rho))
 * (Charrier, Hazelwood, Weinzierl, arXiv:1806.07984, Sec. 2, Eq. 1 without
 * source and point terms) with the ADER-DG scheme of Eq. 4: a cell-local
 * space-time predictor C_STP (Eq. 3, Picard iterations), projections of its
 * time average onto the faces (id|dc, Sec. 2.2), one Rusanov solve per face
 * over the whole time step (F_R, Alg. 1, Sec. 2.4) and the corrector C_Corr.
 * On adaptive meshes (Sec. 2.3, Assumption 1, 3-partitioning) hanging faces
 * are solved on the fine side against data interpolated from the coarse cell
 * (virtual cells) and the results are restricted into the coarse face.
 *
 * Conventions for every call
 *   - Every function returns adg_status and never throws.  On a non-OK return
 *     adg_last_error() gives a message (thread-local).
 *   - Pointers named *_dev are HIP device memory OWNED BY THE CALLER.  The
 *     mesh handle owns only connectivity, basis constants and small scratch.
 *   - All device work is enqueued asynchronously on the given stream(s); no
 *     call synchronises the host unless its comment says so.  The time step
 *     size lives in device memory and is never read back by the step loop.
 *   - Argument errors are detected on the host before anything is enqueued.
 *     Non-physical states met on the device (rho <= 0, p <= 0, non-finite) are
 *     latched in the handle and reported by adg_get_status().
 *   - A handle is not thread-safe; distinct handles are independent.
 *
 * Numbering and layouts (shared with every array argument)
 *   N = p + 1 Gauss-Legendre nodes per axis on [0,1]; m = 5 variables.
 *   cells      ordered by (level, k, j, i), i fastest; level 0 = base grid.
 *   volume     node a = a0 + N a1 + N^2 a2 (a0 along x).
 *   sides      s = 2 d + (0: minus, 1: plus), d = 0 (x), 1 (y), 2 (z).
 *   face node  b = a_t1 + N a_t2, t1 < t2 the two axes tangential to d.
 *   u, u*      double [5][n_cells][N^3]            ("solution layout")
 *   traces     real   [6][2][5][n_cells][N^2]      [side][0: time-averaged Q,
 *                                                  1: time-averaged normal flux]
 *   fside      real   [6][5][n_cells][N^2]         face flux seen by each side
 *   real = double for ADG_FP64, float for ADG_FP32_MFMA.
 *   Batched handles (n_instances > 1) concatenate the instances' arrays: the
 *   offsets of instance i are reported by adg_instance_info().
 */
#ifndef ADG_H
#define ADG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adg_mesh adg_mesh;

typedef enum {
    ADG_OK = 0,
    ADG_ERR_INVALID_ARG = 1,  /* bad descriptor, null pointer, size mismatch  */
    ADG_ERR_UNSUPPORTED = 2,  /* order, level count or boundary not supported */
    ADG_ERR_OOM = 3,          /* device or host allocation failed             */
    ADG_ERR_HIP = 4,          /* a HIP runtime call failed                    */
    ADG_ERR_NONPHYSICAL = 5,  /* rho <= 0, p <= 0 or non-finite state met     */
    ADG_ERR_WORKSPACE = 6     /* workspace smaller than adg_mesh_info reports */
} adg_status;

typedef enum {
    ADG_FP64 = 0,       /* every step in FP64                                    */
    ADG_FP32_MFMA = 1   /* predictor, traces, Riemann in FP32; for p = 3 the
                           predictor's time solve runs on MFMA (4x4x1 FP32
                           blocks) and its spatial derivative contractions on
                           the vector units (DPP and ds_bpermute); other orders
                           run wholly on the vector units; u, u*, dt and the
                           corrector accumulation stay FP64                        */
} adg_precision;

/* One periodic box with an optional static 3:1 refinement (Assumption 1). */
typedef struct {
    int32_t order;           /* p in [0, 7]; N = p+1 nodes per axis                */
    int32_t n[3];            /* base cells per axis, >= 1                          */
    double lo[3], hi[3];     /* domain box, hi > lo                                */
    uint32_t periodic_mask;  /* must be 7 (periodic along x, y and z)              */
    int32_t max_level;       /* 0 = uniform; at most 3 refinement levels           */
    int64_t n_refine;        /* number of (level, i, j, k) rows in refine          */
    const int32_t *refine;   /* host array; each row names a leaf to split 3x3x3.
                                Rows of level l must name leaves that exist once
                                all rows of lower levels are applied; l < max_level */
    double gamma;            /* ratio of specific heats, > 1                       */
    double cfl;              /* dt = cfl / ((2p+1) max sum_d (|u_d|+c)/dx_d)       */
    int32_t picard_iters;    /* predictor iterations; 0 selects p+1                */
} adg_instance_desc;

typedef struct {
    int32_t n_instances;
    int64_t n_cells;          /* total over instances                            */
    int64_t n_dofs;           /* 5 * sum_i n_cells_i * N_i^3                      */
    int64_t u_elems;          /* doubles in a solution array (= n_dofs)           */
    int64_t trace_elems;      /* reals in a traces array                          */
    int64_t fside_elems;      /* reals in an fside array                          */
    int64_t workspace_bytes;  /* device bytes adg_step needs in ws                */
    int64_t n_conforming_faces, n_hanging_faces, n_skeleton_cells;
    int32_t real_bytes;       /* 8 (FP64) or 4 (FP32_MFMA)                        */
    int64_t adjoint_workspace_bytes;  /* device bytes adg_step_adjoint needs      */
    int64_t adjoint_tape_bytes;       /* device bytes of one adg_step_record tape */
} adg_info;

typedef struct {
    int32_t order;
    int64_t n_cells;
    int64_t cell_offset;      /* first cell of the instance                       */
    int64_t u_offset;         /* first double of the instance in u / u*           */
    int64_t trace_offset;     /* first real of the instance in traces             */
    int64_t fside_offset;     /* first real of the instance in fside              */
} adg_instance_geom;

/* Builds the leaf meshes, face lists, skeleton/enclave lists and basis
 * constants of n_instances descriptors (desc[0..n_instances-1]) on the current
 * HIP device.  All instances of one handle use the same precision.
 * Returns ADG_ERR_INVALID_ARG for inconsistent descriptors (including refine
 * rows naming non-leaves), ADG_ERR_UNSUPPORTED for p > 7, max_level > 3 or a
 * non-periodic box.  *out is set only on success; free with adg_free_mesh. */
adg_status adg_init_mesh(const adg_instance_desc *desc, int32_t n_instances,
                         adg_precision prec, adg_mesh **out);
void adg_free_mesh(adg_mesh *mesh);

adg_status adg_mesh_info(const adg_mesh *mesh, adg_info *info);
adg_status adg_instance_info(const adg_mesh *mesh, int32_t instance, adg_instance_geom *info);

/* Host copy of the cell table: level, i, j, k per cell (4 * n_cells int32). */
adg_status adg_mesh_cells(const adg_mesh *mesh, int32_t *cells_host);

/* Physical coordinates of every node, xyz_dev = double [3][u_elems / 5]
 * (per instance: [3][n_cells][N^3] at offset 3 * u_offset / 5). */
adg_status adg_node_coords(const adg_mesh *mesh, double *xyz_dev, hipStream_t stream);

/* Global time step size per instance (Sec. 2.2: global time stepping, one dt
 * for all cells): dt_dev[i] = cfl / ((2p+1) max_{cells,nodes} sum_d
 * (|u_d| + c)/dx_d), c = sqrt(gamma p / rho).  Non-physical nodes latch
 * ADG_ERR_NONPHYSICAL and give dt = 0.  dt_dev holds n_instances doubles. */
adg_status adg_cfl(adg_mesh *mesh, const double *u_dev, double *dt_dev, hipStream_t stream);

/* C_STP plus id|dc and the volume part of C_Corr (Eq. 3-4): for every cell,
 * Picard iterations of the element-local space-time problem starting from
 * u at every time node, then u* = u + volume term of the time-averaged flux,
 * and the face projections of the time-averaged state and normal flux. */
adg_status adg_predictor(adg_mesh *mesh, const double *u_dev, const double *dt_dev,
                         double *ustar_dev, void *traces_dev, hipStream_t stream);

/* F_R (Alg. 1, Sec. 2.4): one Rusanov solve per face, F* = (F_L + F_R)/2 -
 * s (Q_R - Q_L)/2 with s the largest |u_d| + c over the face's nodes on both
 * sides; hanging faces (Sec. 2.3) are solved on each child face against the
 * coarse cell's projection interpolated to it, and the coarse side receives
 * the restriction (quadrature-weighted transpose of the interpolation) of
 * its child results.  Writes the flux every cell side sees into fside. */
adg_status adg_riemann(adg_mesh *mesh, const void *traces_dev, void *fside_dev, hipStream_t stream);

/* C_Corr (Eq. 4): u_out = u* - sum_d (dt/dx_d)(1/w_{a_d})
 * [phi_{a_d}(1) F*_{d+} - phi_{a_d}(0) F*_{d-}], accumulated in FP64.
 * u_out may alias ustar. */
adg_status adg_corrector(adg_mesh *mesh, const double *ustar_dev, const void *fside_dev,
                         const double *dt_dev, double *u_out_dev, hipStream_t stream);

/* n_steps whole steps in place on u_dev (cfl -> predictor -> riemann ->
 * corrector per step).  t_end > 0 is an end time, measured from the state
 * the call starts from: every step takes dt = min(dt_cfl, t_end - t), so the
 * last step lands on t_end exactly and any further steps of the call have
 * dt = 0 and leave u unchanged (per instance; the clock stays on the device).
 * t_end <= 0: no end time.  ws_dev must hold workspace_bytes.  dt_hist_dev,
 * if not NULL, receives n_steps * n_instances doubles (step-major).
 * Passing two different streams splits each step (Sec. 3): the skeleton
 * cells (cells at a resolution transition) run their predictor first and the
 * hanging-face work follows them on one of the handle's two streams, the
 * enclave cells' predictor runs on the other, and the two join before the
 * conforming faces and the corrector.  The handle's streams are created one
 * after the other at init, so the runtime gives them different hardware
 * queues (a caller's streams may share one); they are ordered after both
 * caller streams at the start and both caller streams after them at the
 * end.  Passing the same stream twice runs every phase on that stream.
 * Results do not depend on the schedule. */
adg_status adg_step(adg_mesh *mesh, double *u_dev, int32_t n_steps, double t_end, double *dt_hist_dev,
                    void *ws_dev, hipStream_t stream_skeleton, hipStream_t stream_enclave);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): adg_step with its
 * workspace taken from a static device array of the library instead of a
 * caller buffer.  The array holds ADG_NOALLOC_WORKSPACE_BYTES (64 MiB) on
 * every GPU the library runs on, from the first adg_init_mesh on that GPU
 * until the process ends; handles whose workspace_bytes exceed it get
 * ADG_ERR_WORKSPACE (uniform FP64 meshes of up to about 5,800 cells at
 * p = 3 fit).  The call allocates nothing: plain launches on `stream` (no
 * graph), both predictor parts on that stream; ADG_ERR_UNSUPPORTED while
 * adg_profile is on.  Nothing in the array needs to start at zero, and its
 * contents after a call are unspecified.  All calls on one GPU share the
 * array: calls that may overlap in time on one GPU (other streams, other
 * host threads) race and give wrong results; calls ordered on one stream
 * are safe.  Results are those of adg_step on the same handle. */
#define ADG_NOALLOC_WORKSPACE_BYTES (64LL * 1024 * 1024)
adg_status adg_step_noalloc(adg_mesh *mesh, double *u_dev, int32_t n_steps, double t_end, double *dt_hist_dev,
                            hipStream_t stream);

/* Batched handles (more than one instance, none with hanging faces) run the
 * predictors of all instances from a work list whose items are groups of
 * cells of one instance: either one persistent launch per order over the
 * items of all instances of that order (default), or ONE persistent launch
 * over all items of all orders.  The cells per item of each order come from
 * a table that adg_autotune fills by timing every candidate on the handle's
 * largest instance of that order (u_dev is the state to time on, ws_dev a
 * workspace of workspace_bytes; both are only read/overwritten as scratch;
 * synchronises).  adg_tuning returns the cells per group chosen for
 * N = 1..8 (8 int32).  Results do not depend on the choice. */
adg_status adg_autotune(adg_mesh *mesh, const double *u_dev, void *ws_dev, hipStream_t stream);
adg_status adg_tuning(const adg_mesh *mesh, int32_t *cells_per_block);

/* use_graph = 1 (default for handles with more than one instance):
 * adg_step captures one step into a hipGraph on the handle's own streams and
 * replays it (re-captured when u_dev or ws_dev change); 0 (default for a
 * single instance, whose few large launches ran about 2 % faster without
 * the graph at 81^3, p = 3): plain launches.  batched = 0: one predictor launch per
 * instance; 1: one persistent launch per order (default for handles with
 * more than one instance and no hanging faces); 2: one persistent launch for
 * all orders.  Results are identical either way. */
adg_status adg_set_options(adg_mesh *mesh, int32_t use_graph, int32_t batched);

/* Pipelined step for a handle with a single instance and no hanging faces
 * (off by default).  The cells form 8 contiguous chunks;
 * adg_step runs the predictors chunk by chunk on one of the handle's streams
 * and, on the other, the Riemann solves of the faces whose two cells are
 * done, followed by the correctors of chunks whose faces are all solved, so
 * the bandwidth-bound face and corrector work overlaps the compute-bound
 * predictor.  The per-cell and per-face arithmetic is unchanged, so results
 * are identical with the pipeline on or off.  The caller's streams are joined
 * by events before and after.  ADG_ERR_UNSUPPORTED for other handles when
 * enable != 0.  Waits for the device before switching.  On one MI355X at
 * 81^3, p = 3 it is not faster than the sequential step (3.21 against
 * 3.19 ms, plain launches): the face and corrector kernels also issue VALU
 * work, and running beside the VALU-bound predictor they slow it by about as
 * much as they save.  enable = 2 runs the same chunk order on one stream
 * (locality only); it is slower (3.26 ms). */
adg_status adg_set_pipeline(adg_mesh *mesh, int32_t enable);

/* Face fusion (on by default): for a handle of one uniform instance at p = 3,
 * adg_step solves the Riemann problems of each cell's six faces (Eq. 3, the
 * Rusanov flux with one speed per face, Sec. 2.4) inside that cell's corrector
 * (Eq. 4) instead of in separate per-axis face kernels: each face is solved
 * by both of its cells, with the same operands in the same order, and the
 * fluxes stay on chip, so no face-flux array goes through device memory.
 * Results are the same bits either way.  Not used while a switch tape is on,
 * with the limiter or the pipelined step, or for other handles; the phase
 * entry points adg_riemann and adg_corrector are unaffected.  enable = 0
 * switches it off. */
adg_status adg_set_face_fusion(adg_mesh *mesh, int32_t enable);

/* A-posteriori finite-volume subcell limiter (Sec. 5.3, block-structured
 * methods; Sec. 6, Euler with shocks: a cell whose ADER-DG update is
 * physically wrong or oscillates is rolled back and advanced over the same dt
 * by FV on (2p+1)^3 subcells).  With the limiter on, every adg_step step:
 *   1. takes the old subcell data of every cell: the averages of its
 *      polynomial over (2p+1)^3 equal subcells, or the cell mean in every
 *      subcell if one average is unphysical;
 *   2. computes the unlimited ADER-DG candidate;
 *   3. limits a cell if the candidate has a non-finite value, rho <= 0 or
 *      p <= 0 at a node or in a subcell average, or a subcell average of a
 *      variable outside [m - delta, M + delta], with m, M the extremes of the
 *      old subcell data of that variable over the cell and its six face
 *      neighbours and delta = max(delta0, eps (M - m));
 *   4. advances a limited cell's old subcell data by one first-order
 *      finite-volume step with the Rusanov flux (speed: the larger
 *      |u_d| + c of the two subcell states), and takes the least-squares
 *      polynomial of the result, or the constant state of its mean if that
 *      polynomial is unphysical at a node or in a subcell average;
 *   5. on each face between a limited and an unlimited cell, replaces the
 *      unlimited cell's face flux by the L2 projection of the subcell fluxes
 *      onto the face polynomials and runs its corrector again (the scheme
 *      stays conservative).
 * On adaptive meshes only cells whose six sides are conforming (same-level
 * face neighbours) can be limited: the paper refines down to the FV level
 * near shocks, so no resolution transition cuts an FV region (Sec. 6).  A
 * troubled cell with a hanging side keeps its unlimited candidate (flag 3,
 * or 4 when its corrector ran again next to a limited cell); the relaxed
 * bounds use the cell and its same-level face neighbours.
 * mode: 0 off, 1 on, 2 every cell limited (test hook; every cell that can
 * be).  delta0, eps >= 0 (1e-4 and 1e-3 are usual).  The first enable
 * allocates the limiter's device buffers (about one more state array); they
 * live until adg_free_mesh.  ADG_ERR_UNSUPPORTED unless the handle has one
 * instance and p <= 6.  While on, adg_set_pipeline has no effect, the step
 * runs on s_skel only, and the candidate's inadmissible states are not
 * errors: only an unphysical final state sets the status adg_get_status
 * reports.  Synchronises the device. */
adg_status adg_set_limiter(adg_mesh *mesh, int32_t mode, double delta0, double eps);
/* Of the last limited step: the number of limited cells and of cells whose
 * corrector ran again; flags_dev (device, nc int32, may be NULL) receives per
 * cell 1 limited, 2 corrector re-run, 3 troubled but not limitable (a
 * hanging side), 4 the same with its corrector re-run, 0 otherwise.  Synchronises stream.
 * ADG_ERR_INVALID_ARG if the limiter was never enabled on the handle. */
adg_status adg_limiter_stats(adg_mesh *mesh, int64_t *n_limited, int64_t *n_recorrected, int32_t *flags_dev,
                             hipStream_t stream);

/* Phase timing for measurement.  While enabled, every launch made by the
 * handle's calls is bracketed by HIP events recorded on the stream the launch
 * goes to.  adg_profile(mesh, 1) enables (every phase) and clears the
 * accumulators, adg_profile(mesh, 2) likewise but records the predictor
 * launches only (the fewest events in a timed run), adg_profile(mesh, 0)
 * disables.  adg_profile_read synchronises on the
 * recorded events and returns, per phase (ADG_PHASE_*), the summed kernel
 * time in milliseconds and the number of launches (arrays of ADG_NPHASES).
 * Enabling adds an event pair per launch; results are unchanged. */
enum { ADG_PHASE_CFL = 0, ADG_PHASE_PREDICTOR = 1, ADG_PHASE_HANGING = 2, ADG_PHASE_RIEMANN = 3,
       ADG_PHASE_CORRECTOR = 4, ADG_PHASE_LIMITER = 5, ADG_NPHASES = 6 };
adg_status adg_profile(adg_mesh *mesh, int32_t enable);
adg_status adg_profile_read(adg_mesh *mesh, double *ms, int64_t *launches);

/* Vector-Jacobian product of one step at a FIXED time step size:
 * ubar_n = (d u_{n+1} / d u_n)^T ubar_np1, where u_{n+1} = corrector(riemann(
 * predictor(u_n, dt)), dt) with dt_dev[i] held constant (the CFL reduction is
 * not differentiated).  The transposes run in reverse order: corrector,
 * Rusanov (the face speed s takes the subgradient of the max at its first
 * maximiser in (node, minus side first) order; |x|' = 0 at 0), then the
 * predictor (time averages, volume term and face projections, then the
 * Picard iterations in reverse, with the forward iterates recomputed and
 * stored in ws_dev).  On adaptive meshes (Sec. 2.3) the restriction's
 * transpose sends each coarse side's adjoint to its child faces, and the
 * transpose of the interpolation to virtual cells gathers the child faces'
 * virtual-side adjoints into the coarse side in a fixed order.  FP64 handles
 * with the limiter off only (ADG_ERR_UNSUPPORTED otherwise).  ws_dev holds
 * adjoint_workspace_bytes;
 * ubar_n_dev must not alias ubar_np1_dev. */
adg_status adg_step_adjoint(adg_mesh *mesh, const double *u_n_dev, const double *dt_dev,
                            const double *ubar_np1_dev, double *ubar_n_dev, void *ws_dev,
                            hipStream_t stream);

/* A recorded step, for reverse sweeps that recompute the forward run from a
 * checkpoint anyway: adg_step_record advances u_n_dev by one step at the
 * fixed dt_dev (the predictor, Riemann and corrector of adg_predictor,
 * adg_riemann and adg_corrector, Eq. 4) into u_np1_dev (which may alias
 * u_n_dev; NULL: only the tape is written) and keeps in tape_dev what the
 * step's adjoint reads from its forward run: the predictor's face projections
 * and Picard iterates (at p = 3 the first iterate as the divergence it is
 * formed from, rebuilt from u_n_dev by the adjoint; adjoint_tape_bytes,
 * device memory the caller owns).
 * tape_dev NULL: a plain step at the fixed dt (then u_np1_dev is required).
 * adg_step_adjoint_tape then gives the result of adg_step_adjoint(u_n_dev,
 * dt_dev, ...) bit for bit, reading the tape instead of running the
 * predictor again; u_n_dev and dt_dev must be those of the recording.  Both
 * take an adjoint workspace (adjoint_workspace_bytes), FP64 handles with the
 * limiter off (ADG_ERR_UNSUPPORTED otherwise). */
adg_status adg_step_record(adg_mesh *mesh, const double *u_n_dev, const double *dt_dev, double *u_np1_dev,
                           void *tape_dev, void *ws_dev, hipStream_t stream);
adg_status adg_step_adjoint_tape(adg_mesh *mesh, const double *u_n_dev, const double *dt_dev,
                                 const void *tape_dev, const double *ubar_np1_dev, double *ubar_n_dev,
                                 void *ws_dev, hipStream_t stream);

/* Switch tape of the Rusanov face speed on conforming faces (for checking
 * derivatives of the piecewise-smooth step).  mode 1 (record): every
 * following adg_riemann stores, per conforming face, the first maximiser of
 * |u_d| + c in (node, minus side first) order as 2*node + side into tape_dev;
 * mode 2 (replay): the face speed is taken at the stored maximiser instead of
 * the maximum; mode 0: off (tape_dev may be NULL).  tape_dev holds
 * n_conforming_faces int16 (faces of axis 0, 1, 2 per instance, instances in
 * order) and must stay valid while the mode is on. */
adg_status adg_set_switch_tape(adg_mesh *mesh, int16_t *tape_dev, int32_t mode);

/* Point values of the density of a single-instance uniform handle:
 * out_dev[s] = sum_a rho_{c,a} phi_a0(xi0) phi_a1(xi1) phi_a2(xi2), where c
 * is the cell containing pts_dev[3s..3s+2] (floor of the cell coordinate,
 * clamped into the grid, so a point on a face goes to the upper cell).
 * adg_sample_adjoint ADDS wbar_dev[s] phi_a(x_s) into the density part of
 * ubar_dev: the points of one cell are summed in increasing s, then added
 * (deterministic).  Its work grows with the square of n_pts (meant for up
 * to about 10^4 points); n_pts below 2^31. */
adg_status adg_sample(adg_mesh *mesh, const double *u_dev, const double *pts_dev, int64_t n_pts,
                      double *out_dev, hipStream_t stream);
adg_status adg_sample_adjoint(adg_mesh *mesh, const double *pts_dev, const double *wbar_dev, int64_t n_pts,
                              double *ubar_dev, hipStream_t stream);

/* Dynamic adaptivity (Sec. 2.3, dynamic-adaptivity paragraph: a cell-wise,
 * feature-based criterion reads the new solution in the corrector's
 * epilogue; refinement interpolates volumetric data onto new cells and
 * coarsening merges a cluster of 27 cells; both complete before the next
 * predictor).  A step of adaptation is: adg_indicator on the state,
 * adg_adapt_plan (or adg_adapt_plan_mesh) on the host, adg_init_mesh with the new refine rows,
 * adg_transfer of the state, adg_free_mesh of the old handle.
 *
 * adg_indicator: eta_dev[c] (FP64, one per cell of the handle, cells in the
 * handle's order) = max over nodes a and axes d of |d rho_h / d xi_d (x_a)|,
 * the density derivative in the cell's reference coordinate xi_d in [0, 1],
 * i.e. the largest change of density across the cell.  Reads u_dev. */
adg_status adg_indicator(adg_mesh *mesh, const double *u_dev, double *eta_dev, hipStream_t stream);

/* adg_adapt_plan (host only, no device work): the refine rows of the next
 * mesh from the instance `desc` (whose refine rows describe the current
 * mesh) and eta_host (one value per cell, cells in the handle's order).  A
 * leaf with eta > theta_refine below desc->max_level is split; a refined
 * cell whose 27 children are all leaves, none of them split now, all with
 * eta < theta_coarsen, is merged.  Rows (level, i, j, k) sorted by (level,
 * k, j, i) go to refine_out (host, 4 * capacity int32); *n_refine_out gets
 * their number in any case, and ADG_ERR_WORKSPACE is returned when capacity
 * is smaller (call again with a larger buffer). */
adg_status adg_adapt_plan(const adg_instance_desc *desc, const double *eta_host, double theta_refine,
                          double theta_coarsen, int32_t *refine_out, int64_t capacity, int64_t *n_refine_out);

/* adg_adapt_plan_mesh (host only): adg_adapt_plan for the mesh of a
 * single-instance handle, from the leaves and refine rows the handle keeps
 * since adg_init_mesh, so the current mesh is not built again.  Same rule,
 * output and errors; ADG_ERR_UNSUPPORTED for handles of several instances. */
adg_status adg_adapt_plan_mesh(const adg_mesh *mesh, const double *eta_host, double theta_refine,
                               double theta_coarsen, int32_t *refine_out, int64_t capacity, int64_t *n_refine_out);

/* adg_transfer: the state u_to_dev of handle `to` from u_from_dev of handle
 * `from` (one instance each, same order and base box; refinement levels may
 * differ).  For every cell of `to`: a copy if `from` has the same cell; the
 * polynomial of the coarser `from` cell that contains it, evaluated at its
 * nodes; or the L2 projection of the finer `from` cells that cover it
 * (exact Gauss rules, so mass is conserved to rounding either way).
 * ADG_ERR_INVALID_ARG if the meshes differ or a cell is only partly covered.
 * Allocates and frees a small device table and synchronises `stream`. */
adg_status adg_transfer(const adg_mesh *from, const double *u_from_dev, adg_mesh *to, double *u_to_dev,
                        hipStream_t stream);

/* Synchronises the handle's device work and returns ADG_ERR_NONPHYSICAL if a
 * non-physical state was met since the last call (then clears the latch). */
adg_status adg_get_status(adg_mesh *mesh);

/* ------------------------------------------------------------------------ */
/* Linear variant: elastic waves, Cauchy-Kowalevski predictor                */
/* ------------------------------------------------------------------------ */
/* The seismic variant of the method (Sec. 2.4: for a linear PDE the
 * space-time predictor is the Cauchy-Kowalevski procedure instead of an
 * iteration; Sec. 6: elastic wave propagation with the material carried as
 * time-constant unknowns).  3-D linear elasticity in velocity-stress form,
 * 9 unknowns q = (s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, v_x, v_y, v_z),
 *   d_t s_ij = lambda delta_ij div v + mu (d_i v_j + d_j v_i),
 *   rho d_t v_i = sum_j d_j s_ij,
 * i.e. d_t q + sum_d d_d (A_d q) = 0 with the material constant per cell.
 * One step: qbar = sum_{k=0}^{p} dt^k / (k+1)! L^k u with
 * L q = -sum_d (1/dx_d) A_d D_d q (the Taylor series in time of degree p;
 * it equals p Picard iterations from the time-constant start); then the
 * Euler path's volume term, face projections, one Rusanov solve per face
 * with the larger P-wave speed c_p = sqrt((lambda + 2 mu)/rho) of its two
 * cells, and the corrector.  dt = cfl / ((2p+1) max_c c_p sum_d 1/dx_d),
 * fixed by the material.  Uniform fully periodic boxes, p <= 6, FP64.
 * Layouts (device, caller-owned): u, ustar [9][n_cells][N^3]; traces
 * [6][2][9][n_cells][N^2]; face fluxes [6][9][n_cells][N^2]; material
 * [3][n_cells] (rho, lambda, mu), cells ordered i + n0 (j + n1 k). */
typedef struct adg_lin adg_lin;
typedef struct {
    int32_t order;    /* p, 0..6 */
    int32_t n[3];     /* cells per axis */
    double lo[3], hi[3];
    double cfl;       /* e.g. 0.4 */
} adg_lin_desc;
/* Handle of one uniform periodic mesh on the current device.
 * ADG_ERR_UNSUPPORTED for p > 6 or too many cells; ADG_ERR_INVALID_ARG for
 * bad sizes. */
adg_status adg_lin_init(const adg_lin_desc *desc, adg_lin **out);
adg_status adg_lin_free(adg_lin *lin);
/* Element counts of the arrays above and the adg_lin_step workspace size
 * (any pointer may be NULL). */
adg_status adg_lin_info(adg_lin *lin, int64_t *n_cells, int64_t *u_elems, int64_t *trace_elems,
                        int64_t *fside_elems, int64_t *workspace_bytes);
/* dt of the material into dt_dev (device, one double). */
adg_status adg_lin_dt(adg_lin *lin, const double *material, double *dt_dev, hipStream_t stream);
/* Cauchy-Kowalevski predictor with the dt in dt_dev: ustar (u plus the
 * volume term) and the face projections of the time-averaged state and of
 * its normal flux. */
adg_status adg_lin_predictor(adg_lin *lin, const double *material, const double *u, const double *dt_dev,
                             double *ustar, double *traces, hipStream_t stream);
/* n_steps whole steps in place on u; dt_out (device, may be NULL) receives
 * dt.  ws holds workspace_bytes.  Enqueued on stream, no synchronisation. */
adg_status adg_lin_step(adg_lin *lin, const double *material, double *u, int32_t n_steps, double *dt_out,
                        void *ws, hipStream_t stream);
/* Face fusion of the elastic step (on by default, p = 3 only): adg_lin_step
 * solves each cell's six face problems (the flux of Sec. 2.4 with the larger
 * P-wave speed of the two cells) inside that cell's corrector (Eq. 4), each
 * face by both of its cells with the same operands in the same order, so no
 * face-flux array goes through device memory; the same bits either way.
 * enable = 0 switches it off.  ADG_ERR_INVALID_ARG for a bad handle. */
adg_status adg_lin_set_face_fusion(adg_lin *lin, int32_t enable);

const char *adg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ADG_H */
