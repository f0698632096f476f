// C ABI of the ADER-DG library: handle management, argument checking and the
// launch sequences of the phases and of whole steps.
#include <algorithm>
#include <iterator>
#include <memory>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "adg_internal.h"
#include "kernels.h"

// Workspace of adg_step_noalloc: one copy of this array per GPU, held until
// the process ends.  In host code the name is only a stand-in for the
// symbol, not a device address: host code uses the per-device addresses
// that ensure_scratch takes with hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[ADG_NOALLOC_WORKSPACE_BYTES];

namespace adg {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

namespace {

// pipelined step: number of cell chunks (off by default: measured slower)
constexpr int PIPE_CHUNKS = 8;

struct Instance {
    HostMesh hm;
    std::vector<int32_t> refine;  // the refine rows the handle was built from (4 per row)
    CellIndex index;              // leaves by (level, i, j, k), over hm's cell table
    int N = 0, order = 0, npic = 0;
    double gamma = 1.4, cfl = 0.4;
    int64_t nc = 0, cell_off = 0, u_off = 0, tr_off = 0, fs_off = 0;
    Geo geo{};
    int8_t *level = nullptr;   // null on uniform meshes
    int32_t *ijk = nullptr;
    int32_t *face_m[3] = {nullptr, nullptr, nullptr}, *face_p[3] = {nullptr, nullptr, nullptr};
    int64_t nf[3] = {0, 0, 0};
    HangDev *hang = nullptr;
    int64_t nh = 0;
    int32_t *ccell = nullptr, *cptr = nullptr, *cchild = nullptr;
    int8_t *cside = nullptr;
    int64_t ncs = 0;
    int32_t *skel = nullptr, *encl = nullptr;
    int64_t nskel = 0, nencl = 0;
    double *ptab = nullptr;
    double *partial = nullptr;
    // pipelined step (one instance without hanging faces): the cells form ps
    // contiguous chunks and the faces of every axis are sorted by owner
    // chunk, the later chunk of their two cells
    int ps = 0;                            // chunks (0: not available)
    std::vector<int64_t> pcb;              // [ps + 1] chunk cell boundaries
    std::vector<int64_t> pfo[3];           // [ps + 1] face offsets per axis
    std::vector<std::vector<int>> pcorr;   // chunks whose corrector follows chunk k's faces
    std::vector<int64_t> ppoff;            // [ps + 1] offsets of the chunks' CFL block maxima
    int32_t *ident = nullptr;              // cell list 0 .. nc-1
};

}  // namespace
}  // namespace adg

struct adg_mesh {
    int device = 0;
    adg_precision prec = ADG_FP64;
    std::vector<adg::Instance> inst;
    std::vector<void *> allocs;
    int *status_dev = nullptr;
    double *dt_dev = nullptr;  // one per instance
    // end time of the current adg_step call (0: none) and the time reached
    // since the call started, per instance (device)
    double t_end = 0.0;
    double *clock_dev = nullptr;
    hipEvent_t ev_dt = nullptr, ev_skel = nullptr, ev_encl = nullptr;
    adg_info info{};
    // phase timing (adg_profile)
    int prof = 0;  // 0 off, 1 every phase, 2 predictor launches only
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Rec { int phase; hipEvent_t a, b; };
    std::vector<Rec> recs;
    // batched predictor: every instance in one persistent launch (handles
    // without hanging faces and with more than one instance)
    int batched = 0;                  // 0 per instance, 1 per order, 2 one launch
    int codes[adg::NMAX + 1] = {0};  // predictor variant per N
    int64_t order_begin[adg::NMAX + 2] = {0};  // first item of every N (items grouped by N)
    int64_t order_count[adg::NMAX + 2] = {0};
    adg::PredInst *insts_dev = nullptr;
    adg::PredItem *items_dev = nullptr;
    int64_t nitems = 0;
    int batch_threads = 0, batch_grid = 0, n_cu = 0;
    bool autotuned = false;
    // Rusanov switch tape (conforming faces, axis-major per instance)
    int16_t *tape = nullptr;
    int tape_mode = 0;
    // uniform N = 4 instances: Riemann problems fused into the corrector
    bool fuse_faces = true;
    // captured step (hipGraph) replayed by adg_step
    bool use_graph = false;  // set at init: on for handles with more than one instance
    hipStream_t gs_a = nullptr, gs_b = nullptr;
    hipEvent_t ev_in = nullptr, ev_in2 = nullptr, ev_out = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    const void *gkey_u = nullptr, *gkey_ws = nullptr;
    bool gkey_two = false;
    double gkey_tend = 0.0;
    // pipelined step: predictors chunk by chunk on one stream, the faces and
    // correctors of finished chunks on another
    int pipeline = 0;                 // 0 off, 1 two streams, 2 one stream (chunk by chunk)
    std::vector<hipEvent_t> ev_chunk;
    hipEvent_t ev_join = nullptr;
    // a-posteriori subcell limiter (one instance, uniform mesh)
    int lim_mode = 0;  // 0 off, 1 on, 2 every cell limited
    double lim_delta0 = 1e-4, lim_eps = 1e-3;
    adg::LimDev lim{};
    int *lim_status = nullptr;  // sink of the candidate's admissibility flags
};

namespace adg {
namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

template <typename P>
bool dev_alloc(adg_mesh *m, P *&ptr, size_t count)
{
    ptr = nullptr;
    if (count == 0) return true;
    void *p = nullptr;
    if (hipMalloc(&p, count * sizeof(P)) != hipSuccess) return false;
    m->allocs.push_back(p);
    ptr = static_cast<P *>(p);
    return true;
}

template <typename P>
bool upload(adg_mesh *m, P *&dst, const P *src, size_t count)
{
    if (!dev_alloc(m, dst, count)) return false;
    if (count == 0) return true;
    return hipMemcpy(dst, src, count * sizeof(P), hipMemcpyHostToDevice) == hipSuccess;
}

std::mutex g_basis_mutex;
bool g_basis_uploaded[64] = {false};

adg_status ensure_basis(int device)
{
    std::lock_guard<std::mutex> lk(g_basis_mutex);
    if (device < 0 || device >= 64) {
        set_error("device index out of range");
        return ADG_ERR_UNSUPPORTED;
    }
    if (g_basis_uploaded[device]) return ADG_OK;
    static DevBasis tab[NMAX + 1];
    std::memset(tab, 0, sizeof(tab));
    for (int N = 1; N <= NMAX; ++N) {
        Basis b;
        if (!make_basis(N, b)) {
            set_error("basis construction failed");
            return ADG_ERR_INVALID_ARG;
        }
        std::memcpy(tab[N].D, b.D, sizeof(b.D));
        std::memcpy(tab[N].KW, b.KW, sizeof(b.KW));
        std::memcpy(tab[N].Kw, b.Kw, sizeof(b.Kw));
        for (int e = 0; e < NMAX; ++e) {
            tab[N].w[e] = b.w[e];
            tab[N].winv[e] = e < N ? 1.0 / b.w[e] : 0.0;
            tab[N].L[e] = b.L[e];
            tab[N].R[e] = b.R[e];
            tab[N].xi[e] = b.xi[e];
            double rs = 0.0;
            for (int j = 0; j < N && e < N; ++j) rs += b.KW[e * N + j];
            tab[N].KWsum[e] = rs;
        }
    }
    static DevSub sub[LIM_NMAX + 1];
    std::memset(sub, 0, sizeof(sub));
    for (int N = 1; N <= LIM_NMAX; ++N) {
        Basis b;
        if (!make_basis(N, b) || !make_subcell(b, sub[N])) {
            set_error("subcell operator construction failed");
            return ADG_ERR_INVALID_ARG;
        }
    }
    if (upload_subcell(sub) != hipSuccess) {
        set_error("uploading subcell constants failed");
        return ADG_ERR_HIP;
    }
    if (upload_basis(tab) != hipSuccess) {
        set_error("uploading basis constants failed");
        return ADG_ERR_HIP;
    }
    g_basis_uploaded[device] = true;
    return ADG_OK;
}

std::mutex g_scratch_mutex;
void *g_scratch_ptr[64] = {nullptr};

// Device address of this device's copy of `scratch`; taken once per device
// with the device current (the handle's init call).
adg_status ensure_scratch(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mutex);
    if (device < 0 || device >= 64) {
        set_error("device index out of range");
        return ADG_ERR_UNSUPPORTED;
    }
    if (g_scratch_ptr[device]) return ADG_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error(std::string("address of the static workspace: ") + hipGetErrorString(e));
        return ADG_ERR_HIP;
    }
    g_scratch_ptr[device] = p;
    return ADG_OK;
}

adg_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return ADG_ERR_HIP;
}

#define ADG_HIP(call, what)                       \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

void drop_graph(adg_mesh *m)
{
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    m->gexec = nullptr;
    m->graph = nullptr;
    m->gkey_u = m->gkey_ws = nullptr;
}

void free_all(adg_mesh *m)
{
    drop_graph(m);
    if (m->items_dev) (void)hipFree(m->items_dev);
    if (m->insts_dev) (void)hipFree(m->insts_dev);
    m->items_dev = nullptr;
    m->insts_dev = nullptr;
    for (hipEvent_t *e : {&m->ev_in, &m->ev_in2, &m->ev_out, &m->ev_join})
        if (*e) (void)hipEventDestroy(*e);
    for (hipEvent_t e : m->ev_chunk)
        if (e) (void)hipEventDestroy(e);
    m->ev_chunk.clear();
    if (m->gs_a) (void)hipStreamDestroy(m->gs_a);
    if (m->gs_b) (void)hipStreamDestroy(m->gs_b);
    for (void *p : m->allocs) (void)hipFree(p);
    m->allocs.clear();
    if (m->ev_dt) (void)hipEventDestroy(m->ev_dt);
    if (m->ev_skel) (void)hipEventDestroy(m->ev_skel);
    if (m->ev_encl) (void)hipEventDestroy(m->ev_encl);
    for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
    m->ev_pool.clear();
}

// Event pair around the launches of one phase on one stream (no-op unless
// profiling is enabled).
struct PhaseTimer {
    adg_mesh *m;
    int phase;
    hipStream_t st;
    hipEvent_t a = nullptr;
    PhaseTimer(adg_mesh *m_, int phase_, hipStream_t st_) : m(m_), phase(phase_), st(st_)
    {
        if (!m->prof || (m->prof == 2 && phase != ADG_PHASE_PREDICTOR)) return;
        a = take();
        if (a) (void)hipEventRecord(a, st);
    }
    ~PhaseTimer()
    {
        if (!a) return;
        hipEvent_t b = take();
        if (!b) return;
        (void)hipEventRecord(b, st);
        m->recs.push_back({phase, a, b});
    }
    hipEvent_t take()
    {
        if (m->ev_used == m->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            m->ev_pool.push_back(e);
        }
        return m->ev_pool[m->ev_used++];
    }
};

// doubles of the Picard iterates the adjoint step stores (all instances)
int64_t adjoint_iter_elems(const adg_mesh *m)
{
    int64_t n = 0;
    for (const auto &I : m->inst) n += int64_t(I.npic) * I.N * NV * I.nc * I.N * I.N * I.N;
    return n;
}

bool valid_mesh(const adg_mesh *m)
{
    if (!m) {
        set_error("null mesh handle");
        return false;
    }
    return true;
}

// default predictor variant per N (cells per block as PredCfg)
int default_code(int N)
{
    static const int tab[NMAX + 1] = {0, 0, 2, 5, 8, 11, 13, 15, 15};
    return tab[N];
}

int variant_threads(int code)
{
    int N, CPB;
    pred_variant_shape(code, &N, &CPB);
    int t = CPB * N * N * N;
    return (t + 63) / 64 * 64;
}

// (Re)build the work items of the batched predictor from m->codes: one item
// per CPB cells of every instance, ordered by decreasing cost per item so
// that the static round-robin of the persistent grid balances the load.
adg_status build_batch(adg_mesh *m)
{
    std::vector<PredItem> items;
    int threads = 64;
    for (size_t i = 0; i < m->inst.size(); ++i) {
        const Instance &I = m->inst[i];
        const int code = m->codes[I.N];
        int N, CPB;
        pred_variant_shape(code, &N, &CPB);
        threads = std::max(threads, variant_threads(code));
        for (int64_t c = 0; c < I.nc; c += CPB) items.push_back(PredItem{int32_t(i), code, c});
    }
    auto cost = [&](const PredItem &w) {
        int N, CPB;
        pred_variant_shape(w.code, &N, &CPB);
        return double(CPB) * N * N * N * N;
    };
    // grouped by order (largest first), each group in instance order; the
    // per-order launches take contiguous ranges, the single launch the whole
    // list (cost per item decreases along it)
    std::stable_sort(items.begin(), items.end(),
                     [&](const PredItem &a, const PredItem &b) { return cost(a) > cost(b); });
    std::stable_sort(items.begin(), items.end(), [&](const PredItem &a, const PredItem &b) {
        return m->inst[a.inst].N > m->inst[b.inst].N;
    });
    for (int N = 0; N <= NMAX + 1; ++N) m->order_begin[N] = 0;
    {
        // order_begin[N] .. order_begin[N] + count: items of order N
        std::vector<int64_t> cnt(NMAX + 2, 0);
        for (const auto &w : items) cnt[m->inst[w.inst].N]++;
        int64_t pos = 0;
        for (int N = NMAX; N >= 1; --N) {
            m->order_begin[N] = pos;
            pos += cnt[N];
        }
        m->order_begin[NMAX + 1] = pos;  // unused sentinel
        for (int N = 1; N <= NMAX; ++N) m->order_count[N] = cnt[N];
    }
    if (m->items_dev) (void)hipFree(m->items_dev);
    m->items_dev = nullptr;
    ADG_HIP(hipMalloc(&m->items_dev, sizeof(PredItem) * std::max<size_t>(items.size(), 1)), "batch items");
    ADG_HIP(hipMemcpy(m->items_dev, items.data(), sizeof(PredItem) * items.size(), hipMemcpyHostToDevice),
            "batch items upload");
    m->nitems = int64_t(items.size());
    m->batch_threads = threads;
    const int occ = m->prec == ADG_FP64 ? predictor_batch_occupancy<double>(threads)
                                        : predictor_batch_occupancy<float>(threads);
    const int64_t grid = std::min<int64_t>(m->nitems, int64_t(occ) * m->n_cu);
    m->batch_grid = int(std::max<int64_t>(grid, 1));
    drop_graph(m);
    return ADG_OK;
}

template <typename T>
adg_status do_predictor(adg_mesh *m, const double *u, const double *dt, double *ustar, T *traces,
                        hipStream_t st_skel, hipStream_t st_encl, bool split)
{
    if (m->batched == 2) {
        PhaseTimer tm(m, ADG_PHASE_PREDICTOR, st_encl);
        ADG_HIP(launch_predictor_batch<T>(m->items_dev, m->nitems, m->insts_dev, u, ustar, traces, dt,
                                          m->batch_threads, m->batch_grid, st_encl), "batched predictor");
        return ADG_OK;
    }
    if (m->batched == 1) {
        PhaseTimer tm(m, ADG_PHASE_PREDICTOR, st_encl);
        for (int N = NMAX; N >= 1; --N) {
            if (m->order_count[N] == 0) continue;
            ADG_HIP(launch_predictor_order<T>(m->codes[N], m->items_dev + m->order_begin[N], m->order_count[N],
                                              m->insts_dev, u, ustar, traces, dt, m->n_cu, st_encl),
                    "per-order batched predictor");
        }
        return ADG_OK;
    }
    for (size_t i = 0; i < m->inst.size(); ++i) {
        Instance &I = m->inst[i];
        const double *ui = u + I.u_off;
        double *usi = ustar + I.u_off;
        T *tri = traces + I.tr_off;
        if (split && I.nskel > 0) {
            {
                PhaseTimer tm(m, ADG_PHASE_PREDICTOR, st_skel);
                ADG_HIP(launch_predictor<T>(I.N, ui, usi, tri, I.skel, I.nskel, I.nc, I.level, I.geo, dt + i,
                                            I.gamma, I.npic, st_skel), "predictor (skeleton)");
            }
            PhaseTimer tm(m, ADG_PHASE_PREDICTOR, st_encl);
            ADG_HIP(launch_predictor<T>(I.N, ui, usi, tri, I.encl, I.nencl, I.nc, I.level, I.geo, dt + i,
                                        I.gamma, I.npic, st_encl), "predictor (enclave)");
        } else {
            PhaseTimer tm(m, ADG_PHASE_PREDICTOR, st_encl);
            ADG_HIP(launch_predictor<T>(I.N, ui, usi, tri, nullptr, I.nc, I.nc, I.level, I.geo, dt + i, I.gamma,
                                        I.npic, st_encl), "predictor");
        }
    }
    return ADG_OK;
}

template <typename T>
adg_status do_hanging(adg_mesh *m, const T *traces, T *fside, hipStream_t st)
{
    for (auto &I : m->inst) {
        if (I.nh == 0) continue;
        PhaseTimer tm(m, ADG_PHASE_HANGING, st);
        ADG_HIP(launch_hang<T>(I.N, traces + I.tr_off, fside + I.fs_off, I.hang, I.nh, I.nc, I.ptab, I.gamma,
                               m->status_dev, st), "hanging faces");
        ADG_HIP(launch_restrict<T>(I.N, fside + I.fs_off, I.hang, I.ccell, I.cside, I.cptr, I.cchild, I.ncs, I.nc,
                                   I.ptab, st), "restriction");
    }
    return ADG_OK;
}

template <typename T>
adg_status do_conforming(adg_mesh *m, const T *traces, T *fside, hipStream_t st)
{
    PhaseTimer tm(m, ADG_PHASE_RIEMANN, st);
    int64_t toff = 0;
    for (auto &I : m->inst)
        for (int d = 0; d < 3; ++d) {
            ADG_HIP(launch_riemann<T>(I.N, traces + I.tr_off, fside + I.fs_off, I.face_m[d], I.face_p[d], I.nf[d],
                                      d, I.nc, I.gamma, m->status_dev, st, m->tape ? m->tape + toff : nullptr,
                                      m->tape ? m->tape_mode : 0),
                    "riemann");
            toff += I.nf[d];
        }
    return ADG_OK;
}

// fuse_cfl: the corrector also leaves the block maxima of the new state's
// CFL rate in each instance's partial buffer (consumed by do_cfl_fused).
template <typename T>
adg_status do_corrector(adg_mesh *m, const double *ustar, const T *fside, const double *dt, double *uout,
                        hipStream_t st, bool fuse_cfl = false)
{
    PhaseTimer tm(m, ADG_PHASE_CORRECTOR, st);
    for (size_t i = 0; i < m->inst.size(); ++i) {
        Instance &I = m->inst[i];
        ADG_HIP(launch_corrector<T>(I.N, ustar + I.u_off, fside + I.fs_off, dt + i, uout + I.u_off, I.nc, I.level,
                                    I.geo, st, I.gamma, fuse_cfl ? I.partial : nullptr, m->status_dev),
                "corrector");
    }
    return ADG_OK;
}

// The Riemann problems of every cell's faces inside its corrector (one
// uniform periodic instance at N = 4, no switch tape): the same bits as
// do_conforming then do_corrector with fuse_cfl, without the face fluxes.
bool can_fuse_faces(const adg_mesh *m)
{
    return m->fuse_faces && m->inst.size() == 1 && m->inst[0].N == 4 && m->inst[0].hm.max_level == 0 &&
           m->inst[0].nh == 0 && m->tape_mode == 0;
}

template <typename T>
adg_status do_face_corrector(adg_mesh *m, const double *ustar, const T *traces, const double *dt, double *u,
                             hipStream_t st, bool fuse_cfl)
{
    PhaseTimer tm(m, ADG_PHASE_CORRECTOR, st);
    Instance &I = m->inst[0];
    ADG_HIP(launch_face_corrector4<T>(ustar, traces, dt, u, I.nc, I.hm.n, I.geo, I.gamma,
                                      fuse_cfl ? I.partial : nullptr, m->status_dev, st),
            "riemann + corrector");
    return ADG_OK;
}

// number of CFL block maxima the corrector leaves for the next step
int nparts(const adg_mesh *m, const Instance &I)
{
    return m->pipeline && !m->lim_mode && I.ps > 0 ? int(I.ppoff[I.ps]) : corrector_blocks(I.N, I.nc);
}

adg_status do_cfl(adg_mesh *m, const double *u, double *dt, double *hist, hipStream_t st)
{
    PhaseTimer tm(m, ADG_PHASE_CFL, st);
    for (size_t i = 0; i < m->inst.size(); ++i) {
        Instance &I = m->inst[i];
        const double factor = I.cfl / (2.0 * I.order + 1.0);
        ADG_HIP(launch_cfl(I.N, u + I.u_off, I.nc, I.level, I.geo, I.gamma, factor, I.partial, m->status_dev,
                           dt + i, hist ? hist + i : nullptr, st), "cfl");
    }
    return ADG_OK;
}

// Block maxima of the CFL rate of u in the corrector's layout (starts a run
// of fused steps).
adg_status do_cfl_prime(adg_mesh *m, const double *u, hipStream_t st)
{
    PhaseTimer tm(m, ADG_PHASE_CFL, st);
    for (auto &I : m->inst)
        ADG_HIP(launch_cfl_prime(I.N, u + I.u_off, I.nc, I.level, I.geo, I.gamma, I.partial, nparts(m, I),
                                 m->status_dev, st),
                "cfl block maxima");
    return ADG_OK;
}

// dt from the block maxima left by do_cfl_prime or the previous corrector.
adg_status do_cfl_fused(adg_mesh *m, double *dt, double *hist, hipStream_t st)
{
    PhaseTimer tm(m, ADG_PHASE_CFL, st);
    for (size_t i = 0; i < m->inst.size(); ++i) {
        Instance &I = m->inst[i];
        ADG_HIP(launch_cfl_final(I.partial, nparts(m, I), I.cfl / (2.0 * I.order + 1.0), dt + i,
                                 hist ? hist + i : nullptr, st, m->t_end, m->t_end > 0.0 ? m->clock_dev + i : nullptr),
                "cfl final");
    }
    return ADG_OK;
}

// Chunks of the pipelined step: ps contiguous cell ranges; the faces of every
// axis stably sorted by owner chunk (the later chunk of their two cells); the
// corrector of chunk j follows the faces of the latest chunk that owns a face
// of j; the CFL block maxima of chunk j start at ppoff[j].
void build_chunks(Instance &I)
{
    HostMesh &h = I.hm;
    const int S = PIPE_CHUNKS;
    I.ps = S;
    I.pcb.resize(S + 1);
    for (int k = 0; k <= S; ++k) I.pcb[k] = h.nc * k / S;
    auto chunk = [&](int32_t c) {
        return int(std::upper_bound(I.pcb.begin(), I.pcb.end(), int64_t(c)) - I.pcb.begin()) - 1;
    };
    std::vector<int> dep(S);
    for (int k = 0; k < S; ++k) dep[k] = k;
    for (int a = 0; a < 3; ++a) {
        const size_t nf = h.face_m[a].size();
        std::vector<int> own(nf);
        std::vector<int64_t> cnt(S + 1, 0);
        for (size_t f = 0; f < nf; ++f) {
            const int cm = chunk(h.face_m[a][f]), cp = chunk(h.face_p[a][f]);
            own[f] = std::max(cm, cp);
            dep[cm] = std::max(dep[cm], own[f]);
            dep[cp] = std::max(dep[cp], own[f]);
            ++cnt[own[f] + 1];
        }
        for (int k = 0; k < S; ++k) cnt[k + 1] += cnt[k];
        I.pfo[a] = cnt;
        std::vector<int32_t> fm(nf), fp(nf);
        for (size_t f = 0; f < nf; ++f) {
            const int64_t at = cnt[own[f]]++;
            fm[size_t(at)] = h.face_m[a][f];
            fp[size_t(at)] = h.face_p[a][f];
        }
        h.face_m[a].swap(fm);
        h.face_p[a].swap(fp);
    }
    I.pcorr.assign(S, {});
    for (int j = 0; j < S; ++j) I.pcorr[dep[j]].push_back(j);
    I.ppoff.assign(S + 1, 0);
    for (int j = 0; j < S; ++j) I.ppoff[j + 1] = I.ppoff[j] + corrector_blocks(I.N, I.pcb[j + 1] - I.pcb[j]);
}

// Enqueues one whole step (CFL, predictor, faces, corrector) on the streams.
// The block maxima of the CFL rate must be current (do_cfl_prime, or the
// previous step's corrector); the corrector leaves them for the next step.
// While alive, the launches of the handle report inadmissible states to a
// scratch flag instead of the handle's status (the limited step's candidate
// may be unphysical; its final state is checked by the CFL reduction).
struct StatusSink {
    adg_mesh *m;
    int *keep;
    explicit StatusSink(adg_mesh *mm) : m(mm), keep(mm->status_dev) { m->status_dev = m->lim_status; }
    ~StatusSink() { m->status_dev = keep; }
};

// Subcell bounds of u for the first limited step of a call (later steps
// carry them from the previous step's kernels).
adg_status do_lim_prime(adg_mesh *m, const double *u, hipStream_t st)
{
    if (!m->lim_mode) return ADG_OK;
    PhaseTimer tm(m, ADG_PHASE_LIMITER, st);
    const Instance &I = m->inst[0];
    ADG_HIP(launch_lim_scan(I.N, u, I.nc, I.gamma, m->lim, false, st), "limiter bounds");
    return ADG_OK;
}

// One step with the a-posteriori subcell limiter (one instance, uniform
// mesh, one stream): CFL, a copy of u and of the carried bounds, the
// unlimited candidate (predictor, faces, corrector), detection, the FV step
// of the limited cells with the flux replacement on their faces, the
// corrector again for their unlimited neighbours, then the CFL block maxima
// of the final state (which also flags an unphysical result).
template <typename T>
adg_status enqueue_step_limited(adg_mesh *m, double *u, double *hist, void *ws, hipStream_t st)
{
    char *w = static_cast<char *>(ws);
    double *ustar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * m->info.u_elems);
    T *traces = reinterpret_cast<T *>(w);
    w += align_up(sizeof(T) * m->info.trace_elems);
    T *fside = reinterpret_cast<T *>(w);
    Instance &I = m->inst[0];
    adg_status s = do_cfl_fused(m, m->dt_dev, hist, st);
    if (s != ADG_OK) return s;
    {
        PhaseTimer tm(m, ADG_PHASE_LIMITER, st);
        ADG_HIP(launch_lim_copy(u, int64_t(m->info.u_elems), I.nc, m->lim, st), "limiter copy");
    }
    {
        StatusSink sink(m);
        s = do_predictor<T>(m, u, m->dt_dev, ustar, traces, st, st, false);
        if (s != ADG_OK) return s;
        s = do_hanging<T>(m, traces, fside, st);
        if (s != ADG_OK) return s;
        s = do_conforming<T>(m, traces, fside, st);
        if (s != ADG_OK) return s;
        s = do_corrector<T>(m, ustar, fside, m->dt_dev, u, st, false);
        if (s != ADG_OK) return s;
    }
    {
        PhaseTimer tm(m, ADG_PHASE_LIMITER, st);
        ADG_HIP(launch_lim_detect(I.N, u, I.nc, I.gamma, m->lim_delta0, m->lim_eps, m->lim_mode == 2 ? 1 : 0, m->lim,
                                  st),
                "limiter detection");
    }
    {
        PhaseTimer tm(m, ADG_PHASE_LIMITER, st);
        ADG_HIP(launch_lim_fv<T>(I.N, u, fside, I.nc, I.geo, m->dt_dev, I.gamma, m->lim, st), "limiter FV step");
    }
    {
        PhaseTimer tm(m, ADG_PHASE_LIMITER, st);
        ADG_HIP(launch_lim_recorrect<T>(I.N, ustar, fside, u, I.nc, I.geo, m->dt_dev, m->lim, st),
                "limiter corrector re-run");
        ADG_HIP(launch_lim_scan(I.N, u, I.nc, I.gamma, m->lim, true, st), "limiter bounds (re-run cells)");
    }
    return do_cfl_prime(m, u, st);
}

template <typename T>
adg_status enqueue_step(adg_mesh *m, double *u, double *hist, void *ws, hipStream_t s_skel, hipStream_t s_encl)
{
    if (m->lim_mode) return enqueue_step_limited<T>(m, u, hist, ws, s_skel);
    char *w = static_cast<char *>(ws);
    double *ustar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * m->info.u_elems);
    T *traces = reinterpret_cast<T *>(w);
    w += align_up(sizeof(T) * m->info.trace_elems);
    T *fside = reinterpret_cast<T *>(w);
    const bool two = s_skel != s_encl;
    {
        adg_status st = do_cfl_fused(m, m->dt_dev, hist, s_skel);
        if (st != ADG_OK) return st;
        if (two) {
            ADG_HIP(hipEventRecord(m->ev_dt, s_skel), "event record");
            ADG_HIP(hipStreamWaitEvent(s_encl, m->ev_dt, 0), "stream wait");
        }
        st = do_predictor<T>(m, u, m->dt_dev, ustar, traces, s_skel, s_encl, true);
        if (st != ADG_OK) return st;
        st = do_hanging<T>(m, traces, fside, s_skel);
        if (st != ADG_OK) return st;
        if (two) {
            ADG_HIP(hipEventRecord(m->ev_encl, s_encl), "event record");
            ADG_HIP(hipStreamWaitEvent(s_skel, m->ev_encl, 0), "stream wait");
        }
        if (can_fuse_faces(m)) {
            st = do_face_corrector<T>(m, ustar, traces, m->dt_dev, u, s_skel, true);
            if (st != ADG_OK) return st;
        } else {
            st = do_conforming<T>(m, traces, fside, s_skel);
            if (st != ADG_OK) return st;
            st = do_corrector<T>(m, ustar, fside, m->dt_dev, u, s_skel, true);
            if (st != ADG_OK) return st;
        }
    }
    return ADG_OK;
}

// One whole step, pipelined over cell chunks (single instance, no hanging
// faces).  Stream A: dt, then the predictor of chunk 0, 1, ...  Stream B: as
// soon as chunk k's predictor is done, the faces chunk k owns (both cells'
// predictors are then done), then the corrector of every chunk whose faces
// are now all solved.  B joins A at the end.  Per-cell and per-face
// arithmetic is that of enqueue_step, so the results are identical.
template <typename T>
adg_status enqueue_step_pipe(adg_mesh *m, double *u, double *hist, void *ws, hipStream_t A, hipStream_t B)
{
    char *w = static_cast<char *>(ws);
    double *ustar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * m->info.u_elems);
    T *traces = reinterpret_cast<T *>(w);
    w += align_up(sizeof(T) * m->info.trace_elems);
    T *fside = reinterpret_cast<T *>(w);
    Instance &I = m->inst[0];
    const int S = I.ps;
    adg_status st = do_cfl_fused(m, m->dt_dev, hist, A);
    if (st != ADG_OK) return st;
    if (A != B) {
        ADG_HIP(hipEventRecord(m->ev_dt, A), "event record");
        ADG_HIP(hipStreamWaitEvent(B, m->ev_dt, 0), "stream wait");
    }
    for (int k = 0; k < S; ++k) {
        {
            PhaseTimer tm(m, ADG_PHASE_PREDICTOR, A);
            ADG_HIP(launch_predictor<T>(I.N, u, ustar, traces, I.ident + I.pcb[k], I.pcb[k + 1] - I.pcb[k], I.nc,
                                        I.level, I.geo, m->dt_dev, I.gamma, I.npic, A),
                    "predictor (chunk)");
        }
        if (A != B) {
            ADG_HIP(hipEventRecord(m->ev_chunk[k], A), "event record");
            ADG_HIP(hipStreamWaitEvent(B, m->ev_chunk[k], 0), "stream wait");
        }
        {
            PhaseTimer tm(m, ADG_PHASE_RIEMANN, B);
            for (int d = 0; d < 3; ++d)
                ADG_HIP(launch_riemann<T>(I.N, traces, fside, I.face_m[d] + I.pfo[d][k], I.face_p[d] + I.pfo[d][k],
                                          I.pfo[d][k + 1] - I.pfo[d][k], d, I.nc, I.gamma, m->status_dev, B),
                        "riemann (chunk)");
        }
        for (int j : I.pcorr[k]) {
            PhaseTimer tm(m, ADG_PHASE_CORRECTOR, B);
            ADG_HIP(launch_corrector<T>(I.N, ustar, fside, m->dt_dev, u, I.nc, I.level, I.geo, B, I.gamma,
                                        I.partial + I.ppoff[j], m->status_dev, I.pcb[j], I.pcb[j + 1]),
                    "corrector (chunk)");
        }
    }
    if (A != B) {
        ADG_HIP(hipEventRecord(m->ev_join, B), "event record");
        ADG_HIP(hipStreamWaitEvent(A, m->ev_join, 0), "stream wait");
    }
    return ADG_OK;
}

template <typename T>
adg_status step_eager(adg_mesh *m, double *u, int32_t n_steps, double *hist, void *ws, hipStream_t s_skel,
                      hipStream_t s_encl)
{
    if (m->pipeline && !m->lim_mode) {
        // the handle's two streams, joined with the caller's before and after
        hipStream_t A = m->gs_a, B = m->pipeline == 2 ? m->gs_a : m->gs_b;
        ADG_HIP(hipEventRecord(m->ev_in, s_skel), "event record");
        ADG_HIP(hipStreamWaitEvent(A, m->ev_in, 0), "stream wait");
        if (s_skel != s_encl) {
            ADG_HIP(hipEventRecord(m->ev_in2, s_encl), "event record");
            ADG_HIP(hipStreamWaitEvent(A, m->ev_in2, 0), "stream wait");
        }
        const int ni = int(m->inst.size());
        adg_status st0 = do_cfl_prime(m, u, A);
        if (st0 != ADG_OK) return st0;
        for (int n = 0; n < n_steps; ++n) {
            adg_status st = enqueue_step_pipe<T>(m, u, hist ? hist + int64_t(n) * ni : nullptr, ws, A, B);
            if (st != ADG_OK) return st;
        }
        ADG_HIP(hipEventRecord(m->ev_out, A), "event record");
        ADG_HIP(hipStreamWaitEvent(s_skel, m->ev_out, 0), "stream wait");
        if (s_skel != s_encl) ADG_HIP(hipStreamWaitEvent(s_encl, m->ev_out, 0), "stream wait");
        return ADG_OK;
    }
    const int ni = int(m->inst.size());
    if (s_skel != s_encl && !m->lim_mode) {
        // Skeleton/enclave split on the handle's two streams, created at
        // init one after the other, so that the runtime gives them different
        // hardware queues (a caller's streams may share one); joined with
        // the caller's streams by events before and after.
        hipStream_t A = m->gs_a, B = m->gs_b;
        ADG_HIP(hipEventRecord(m->ev_in, s_skel), "event record");
        ADG_HIP(hipStreamWaitEvent(A, m->ev_in, 0), "stream wait");
        ADG_HIP(hipEventRecord(m->ev_in2, s_encl), "event record");
        ADG_HIP(hipStreamWaitEvent(A, m->ev_in2, 0), "stream wait");
        adg_status st0 = do_cfl_prime(m, u, A);
        if (st0 != ADG_OK) return st0;
        for (int n = 0; n < n_steps; ++n) {
            adg_status st = enqueue_step<T>(m, u, hist ? hist + int64_t(n) * ni : nullptr, ws, A, B);
            if (st != ADG_OK) return st;
        }
        ADG_HIP(hipEventRecord(m->ev_out, A), "event record");
        ADG_HIP(hipStreamWaitEvent(s_skel, m->ev_out, 0), "stream wait");
        ADG_HIP(hipStreamWaitEvent(s_encl, m->ev_out, 0), "stream wait");
        return ADG_OK;
    }
    adg_status st0 = do_cfl_prime(m, u, s_skel);
    if (st0 != ADG_OK) return st0;
    st0 = do_lim_prime(m, u, s_skel);
    if (st0 != ADG_OK) return st0;
    for (int n = 0; n < n_steps; ++n) {
        adg_status st = enqueue_step<T>(m, u, hist ? hist + int64_t(n) * ni : nullptr, ws, s_skel, s_encl);
        if (st != ADG_OK) return st;
    }
    if (s_skel != s_encl) {
        // the limited step runs on s_skel only: leave s_encl ordered after it
        ADG_HIP(hipEventRecord(m->ev_skel, s_skel), "event record");
        ADG_HIP(hipStreamWaitEvent(s_encl, m->ev_skel, 0), "stream wait");
    }
    return ADG_OK;
}

// Captures one step into a hipGraph on the handle's private streams (default
// priority) and replays it n_steps times; the caller's streams are joined by
// events before and after.  dt stays on the device; the history, if asked
// for, is copied after each replay.
template <typename T>
adg_status step_graph(adg_mesh *m, double *u, int32_t n_steps, double *hist, void *ws, hipStream_t s_skel,
                      hipStream_t s_encl)
{
    const bool two = s_skel != s_encl;
    hipStream_t A = m->gs_a, B = (two || m->pipeline == 1) ? m->gs_b : m->gs_a;
    ADG_HIP(hipEventRecord(m->ev_in, s_skel), "event record");
    ADG_HIP(hipStreamWaitEvent(A, m->ev_in, 0), "stream wait");
    if (two) {
        ADG_HIP(hipEventRecord(m->ev_in2, s_encl), "event record");
        ADG_HIP(hipStreamWaitEvent(A, m->ev_in2, 0), "stream wait");
    }
    {
        adg_status st0 = do_cfl_prime(m, u, A);
        if (st0 != ADG_OK) return st0;
        st0 = do_lim_prime(m, u, A);
        if (st0 != ADG_OK) return st0;
    }
    if (!m->gexec || m->gkey_u != u || m->gkey_ws != ws || m->gkey_two != two || m->gkey_tend != m->t_end) {
        drop_graph(m);
        ADG_HIP(hipStreamBeginCapture(A, hipStreamCaptureModeThreadLocal), "begin capture");
        adg_status st = m->pipeline && !m->lim_mode ? enqueue_step_pipe<T>(m, u, nullptr, ws, A, B)
                                                    : enqueue_step<T>(m, u, nullptr, ws, A, B);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(A, &g);
        if (st != ADG_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        m->graph = g;
        ADG_HIP(hipGraphInstantiate(&m->gexec, m->graph, nullptr, nullptr, 0), "graph instantiate");
        m->gkey_u = u;
        m->gkey_ws = ws;
        m->gkey_two = two;
        m->gkey_tend = m->t_end;
    }
    const int ni = int(m->inst.size());
    for (int n = 0; n < n_steps; ++n) {
        ADG_HIP(hipGraphLaunch(m->gexec, A), "graph launch");
        if (hist)
            ADG_HIP(hipMemcpyAsync(hist + int64_t(n) * ni, m->dt_dev, sizeof(double) * ni, hipMemcpyDeviceToDevice, A),
                    "dt history copy");
    }
    ADG_HIP(hipEventRecord(m->ev_out, A), "event record");
    ADG_HIP(hipStreamWaitEvent(s_skel, m->ev_out, 0), "stream wait");
    if (two) ADG_HIP(hipStreamWaitEvent(s_encl, m->ev_out, 0), "stream wait");
    return ADG_OK;
}

// Starts the clock of a run to t_end (t_end <= 0: no end time) on s_skel,
// ahead of everything the step sequence enqueues.
adg_status start_clock(adg_mesh *m, double t_end, hipStream_t s_skel)
{
    m->t_end = t_end > 0.0 ? t_end : 0.0;
    if (m->t_end > 0.0)
        ADG_HIP(launch_fill(m->clock_dev, int64_t(m->inst.size()), 0.0, s_skel), "clock reset");
    return ADG_OK;
}

template <typename T>
adg_status step_impl(adg_mesh *m, double *u, int32_t n_steps, double t_end, double *hist, void *ws,
                     hipStream_t s_skel, hipStream_t s_encl)
{
    if (n_steps == 0) return ADG_OK;
    adg_status st = start_clock(m, t_end, s_skel);
    if (st != ADG_OK) return st;
    if (m->use_graph && !m->prof && m->tape_mode == 0) return step_graph<T>(m, u, n_steps, hist, ws, s_skel, s_encl);
    return step_eager<T>(m, u, n_steps, hist, ws, s_skel, s_encl);
}

// Times one predictor variant on one instance (the per-order persistent
// kernel restricted to that instance); returns milliseconds per cell, or a
// negative value.
template <typename T>
double time_variant(adg_mesh *m, int inst, int code, const double *u, double *ustar, T *traces, hipStream_t st)
{
    const Instance &I = m->inst[inst];
    int N, CPB;
    pred_variant_shape(code, &N, &CPB);
    std::vector<PredItem> items;
    for (int64_t c = 0; c < I.nc; c += CPB) items.push_back(PredItem{int32_t(inst), code, c});
    PredItem *dev = nullptr;
    if (hipMalloc(&dev, sizeof(PredItem) * items.size()) != hipSuccess) return -1.0;
    double best = -1.0;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipMemcpy(dev, items.data(), sizeof(PredItem) * items.size(), hipMemcpyHostToDevice) == hipSuccess &&
        hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess) {
        for (int rep = 0; rep < 4; ++rep) {
            (void)hipEventRecord(a, st);
            (void)launch_predictor_order<T>(code, dev, int64_t(items.size()), m->insts_dev, u, ustar, traces,
                                            m->dt_dev, m->n_cu, st);
            (void)hipEventRecord(b, st);
            (void)hipEventSynchronize(b);
            float ms = 0.0f;
            if (rep > 0 && hipEventElapsedTime(&ms, a, b) == hipSuccess) {
                const double per = double(ms) / double(I.nc);
                if (best < 0.0 || per < best) best = per;
            }
        }
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(dev);
    return best;
}

template <typename T>
adg_status autotune_impl(adg_mesh *m, const double *u, void *ws, hipStream_t st)
{
    char *w = static_cast<char *>(ws);
    double *ustar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * m->info.u_elems);
    T *traces = reinterpret_cast<T *>(w);
    // dt for the trials: the CFL value of the current state
    adg_status s0 = do_cfl(m, u, m->dt_dev, nullptr, st);
    if (s0 != ADG_OK) return s0;
    for (int N = 1; N <= NMAX; ++N) {
        int rep = -1;  // the largest instance of this order stands for it
        for (size_t i = 0; i < m->inst.size(); ++i)
            if (m->inst[i].N == N && (rep < 0 || m->inst[i].nc > m->inst[rep].nc)) rep = int(i);
        if (rep < 0) continue;
        double best = -1.0;
        int best_code = default_code(N);
        for (int code = 0; code < PRED_VARIANTS; ++code) {
            int vn, cpb;
            pred_variant_shape(code, &vn, &cpb);
            if (vn != N) continue;
            const double t = time_variant<T>(m, rep, code, u, ustar, traces, st);
            if (t > 0.0 && (best < 0.0 || t < best)) {
                best = t;
                best_code = code;
            }
        }
        m->codes[N] = best_code;
    }
    m->autotuned = true;
    return build_batch(m);
}

}  // namespace
}  // namespace adg

using namespace adg;

namespace {
// Makes `device` current for the lifetime of the guard and then restores the
// caller's current device.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int device)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != device) (void)hipSetDevice(device);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};
}  // namespace

extern "C" {

const char *adg_last_error(void) { return g_last_error.c_str(); }

adg_status adg_init_mesh(const adg_instance_desc *desc, int32_t n_instances, adg_precision prec, adg_mesh **out)
{
    if (!desc || !out || n_instances < 1) {
        set_error("adg_init_mesh: null argument or n_instances < 1");
        return ADG_ERR_INVALID_ARG;
    }
    if (prec != ADG_FP64 && prec != ADG_FP32_MFMA) {
        set_error("adg_init_mesh: unknown precision");
        return ADG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    adg_mesh *m = new (std::nothrow) adg_mesh();
    if (!m) {
        set_error("out of host memory");
        return ADG_ERR_OOM;
    }
    m->prec = prec;
    const int rb = prec == ADG_FP64 ? 8 : 4;
    m->inst.resize(n_instances);
    int64_t cell_off = 0, u_off = 0, tr_off = 0, fs_off = 0;
    int64_t ncf = 0, nhang = 0, nskel = 0;
    for (int i = 0; i < n_instances; ++i) {
        const adg_instance_desc &d = desc[i];
        Instance &I = m->inst[i];
        std::string err = build_host_mesh(d, I.hm);
        if (!err.empty()) {
            set_error("instance " + std::to_string(i) + ": " + err);
            delete m;
            return err.rfind("unsupported", 0) == 0 ? ADG_ERR_UNSUPPORTED : ADG_ERR_INVALID_ARG;
        }
        I.refine.assign(d.refine, d.refine + 4 * d.n_refine);
        I.index.build(I.hm);
        I.N = I.hm.N;
        I.order = d.order;
        I.npic = d.picard_iters > 0 ? d.picard_iters : d.order + 1;
        I.gamma = d.gamma;
        I.cfl = d.cfl;
        I.nc = I.hm.nc;
        I.cell_off = cell_off;
        I.u_off = u_off;
        I.tr_off = tr_off;
        I.fs_off = fs_off;
        const int64_t N2 = int64_t(I.N) * I.N, N3 = N2 * I.N;
        cell_off += I.nc;
        u_off += NV * I.nc * N3;
        tr_off += 12 * NV * I.nc * N2;
        fs_off += 6 * NV * I.nc * N2;
        for (int l = 0; l <= LMAX; ++l)
            for (int a = 0; a < 3; ++a) {
                double f = 1.0;
                for (int k = 0; k < l; ++k) f *= 3.0;
                I.geo.inv_dx[l][a] = (d.n[a] * f) / (d.hi[a] - d.lo[a]);
            }
        for (int a = 0; a < 3; ++a) ncf += int64_t(I.hm.face_m[a].size());
        nhang += int64_t(I.hm.hang.size());
        nskel += int64_t(I.hm.skeleton.size());
    }
    if (hipGetDevice(&m->device) != hipSuccess) {
        set_error("no HIP device");
        delete m;
        return ADG_ERR_HIP;
    }
    adg_status bs = ensure_basis(m->device);
    if (bs == ADG_OK) bs = ensure_scratch(m->device);
    if (bs != ADG_OK) {
        delete m;
        return bs;
    }
    bool ok = true;
    for (auto &I : m->inst) {
        HostMesh &h = I.hm;
        if (n_instances == 1 && h.hang.empty() && h.nc >= 2 * PIPE_CHUNKS) build_chunks(I);
        if (h.max_level > 0) ok = ok && upload(m, I.level, h.level.data(), h.level.size());
        ok = ok && upload(m, I.ijk, h.ijk.data(), h.ijk.size());
        if (I.ps > 0) {
            std::vector<int32_t> id(size_t(I.nc));
            for (int64_t c = 0; c < I.nc; ++c) id[size_t(c)] = int32_t(c);
            ok = ok && upload(m, I.ident, id.data(), id.size());
        }
        for (int a = 0; a < 3; ++a) {
            I.nf[a] = int64_t(h.face_m[a].size());
            ok = ok && upload(m, I.face_m[a], h.face_m[a].data(), h.face_m[a].size());
            ok = ok && upload(m, I.face_p[a], h.face_p[a].data(), h.face_p[a].size());
        }
        std::vector<HangDev> hd(h.hang.size());
        for (size_t k = 0; k < h.hang.size(); ++k) {
            const auto &H = h.hang[k];
            hd[k] = HangDev{H.fine, H.coarse, H.d, H.fine_minus, H.dl, H.s1, H.s2, {0, 0, 0}};
        }
        I.nh = int64_t(hd.size());
        ok = ok && upload(m, I.hang, hd.data(), hd.size());
        I.ncs = int64_t(h.coarse_cell.size());
        ok = ok && upload(m, I.ccell, h.coarse_cell.data(), h.coarse_cell.size());
        ok = ok && upload(m, I.cside, h.coarse_side.data(), h.coarse_side.size());
        ok = ok && upload(m, I.cptr, h.coarse_ptr.data(), I.ncs > 0 ? h.coarse_ptr.size() : 0);
        ok = ok && upload(m, I.cchild, h.coarse_child.data(), h.coarse_child.size());
        I.nskel = int64_t(h.skeleton.size());
        I.nencl = int64_t(h.enclave.size());
        ok = ok && upload(m, I.skel, h.skeleton.data(), h.skeleton.size());
        ok = ok && upload(m, I.encl, h.enclave.data(), h.enclave.size());
        // transfer table
        Basis b;
        make_basis(I.N, b);
        const int N2 = I.N * I.N;
        std::vector<double> pt(size_t(TRANSFER_BLOCKS) * 2 * N2, 0.0);
        for (int dl = 1; dl <= LMAX; ++dl) {
            int r = 1;
            for (int k = 0; k < dl; ++k) r *= 3;
            for (int s = 0; s < r; ++s) {
                double *blk = &pt[size_t(transfer_base(dl) + s) * 2 * N2];
                make_transfer(b, r, s, blk, blk + N2);
            }
        }
        ok = ok && upload(m, I.ptab, pt.data(), pt.size());
        ok = ok && dev_alloc(m, I.partial, size_t(std::max<int64_t>({CFL_MAX_BLOCKS, corrector_blocks(I.N, I.nc),
                                                                      I.ps > 0 ? I.ppoff[I.ps] : 0})));
        // the host copy of the cell table is kept (adg_mesh_cells); face lists are not needed
        for (int a = 0; a < 3; ++a) {
            std::vector<int32_t>().swap(h.face_m[a]);
            std::vector<int32_t>().swap(h.face_p[a]);
        }
    }
    ok = ok && dev_alloc(m, m->status_dev, 1) && dev_alloc(m, m->dt_dev, size_t(n_instances)) &&
         dev_alloc(m, m->clock_dev, size_t(n_instances));
    if (ok) {
        // one attribute, not the whole property record (a handle is made per adaptation)
        int ncu = 1;
        ok = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, m->device) == hipSuccess;
        m->n_cu = ok ? ncu : 1;
        ok = ok && hipStreamCreateWithFlags(&m->gs_a, hipStreamNonBlocking) == hipSuccess &&
             hipStreamCreateWithFlags(&m->gs_b, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&m->ev_in2, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming) == hipSuccess;
    }
    if (ok) {
        // batched predictor table (used when there is more than one instance
        // and no instance has hanging faces)
        bool any_skel = false;
        std::vector<PredInst> pis;
        for (auto &I : m->inst) {
            any_skel = any_skel || I.nskel > 0;
            pis.push_back(PredInst{I.u_off, I.tr_off, I.nc, I.level, I.gamma, int32_t(I.npic), int32_t(I.N), I.geo});
        }
        for (int N = 0; N <= NMAX; ++N) m->codes[N] = default_code(N);
        m->batched = (n_instances > 1 && !any_skel) ? 1 : 0;
        m->use_graph = n_instances > 1;
        ok = hipMalloc(&m->insts_dev, sizeof(PredInst) * pis.size()) == hipSuccess &&
             hipMemcpy(m->insts_dev, pis.data(), sizeof(PredInst) * pis.size(), hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && (!any_skel ? build_batch(m) == ADG_OK : true);
    }
    if (ok) {
        int zero = 0;
        ok = hipMemcpy(m->status_dev, &zero, sizeof(int), hipMemcpyHostToDevice) == hipSuccess;
    }
    if (ok)
        ok = hipEventCreateWithFlags(&m->ev_dt, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&m->ev_skel, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&m->ev_encl, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming) == hipSuccess;
    if (ok && m->inst[0].ps > 0) {
        m->ev_chunk.assign(size_t(m->inst[0].ps), nullptr);
        for (auto &e : m->ev_chunk) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        set_error("device allocation or upload failed");
        free_all(m);
        delete m;
        return ADG_ERR_OOM;
    }
    adg_info &inf = m->info;
    inf.n_instances = n_instances;
    inf.n_cells = cell_off;
    inf.n_dofs = u_off;
    inf.u_elems = u_off;
    inf.trace_elems = tr_off;
    inf.fside_elems = fs_off;
    inf.workspace_bytes = int64_t(align_up(sizeof(double) * u_off) + align_up(size_t(rb) * tr_off) +
                                  align_up(size_t(rb) * fs_off));
    inf.n_conforming_faces = ncf;
    inf.n_hanging_faces = nhang;
    inf.n_skeleton_cells = nskel;
    inf.real_bytes = rb;
    {
        // adjoint workspace: u*, traces, their adjoint, face-flux adjoint (FP64), Picard iterates, the
        // virtual-cell adjoints of the hanging faces
        int64_t vb = 0;
        for (auto &I : m->inst) vb += I.nh * 2 * NV * I.N * I.N;
        inf.adjoint_workspace_bytes =
            int64_t(align_up(sizeof(double) * u_off) + 2 * align_up(sizeof(double) * tr_off) +
                    align_up(sizeof(double) * fs_off) +
                    align_up(sizeof(double) * std::max<int64_t>(adjoint_iter_elems(m), 1)) +
                    align_up(sizeof(double) * std::max<int64_t>(vb, 1)));
        inf.adjoint_tape_bytes = int64_t(align_up(sizeof(double) * tr_off) +
                                         align_up(sizeof(double) * std::max<int64_t>(adjoint_iter_elems(m), 1)));
    }
    *out = m;
    return ADG_OK;
}

void adg_free_mesh(adg_mesh *mesh)
{
    if (!mesh) return;
    (void)hipDeviceSynchronize();
    free_all(mesh);
    delete mesh;
}

adg_status adg_mesh_info(const adg_mesh *mesh, adg_info *info)
{
    if (!valid_mesh(mesh) || !info) {
        set_error("adg_mesh_info: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    *info = mesh->info;
    return ADG_OK;
}

adg_status adg_instance_info(const adg_mesh *mesh, int32_t instance, adg_instance_geom *info)
{
    if (!valid_mesh(mesh) || !info || instance < 0 || instance >= int32_t(mesh->inst.size())) {
        set_error("adg_instance_info: bad argument");
        return ADG_ERR_INVALID_ARG;
    }
    const Instance &I = mesh->inst[instance];
    info->order = I.order;
    info->n_cells = I.nc;
    info->cell_offset = I.cell_off;
    info->u_offset = I.u_off;
    info->trace_offset = I.tr_off;
    info->fside_offset = I.fs_off;
    return ADG_OK;
}

adg_status adg_mesh_cells(const adg_mesh *mesh, int32_t *cells)
{
    if (!valid_mesh(mesh) || !cells) {
        set_error("adg_mesh_cells: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    for (const auto &I : mesh->inst)
        for (int64_t c = 0; c < I.nc; ++c) {
            int32_t *o = cells + 4 * (I.cell_off + c);
            o[0] = I.hm.level[c];
            o[1] = I.hm.ijk[3 * c];
            o[2] = I.hm.ijk[3 * c + 1];
            o[3] = I.hm.ijk[3 * c + 2];
        }
    return ADG_OK;
}

adg_status adg_node_coords(const adg_mesh *mesh, double *xyz, hipStream_t stream)
{
    if (!valid_mesh(mesh) || !xyz) {
        set_error("adg_node_coords: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    for (const auto &I : mesh->inst)
        ADG_HIP(launch_node_coords(I.N, xyz + 3 * (I.u_off / NV), I.ijk, I.level, I.nc, I.geo, I.hm.lo, stream),
                "node coords");
    return ADG_OK;
}

adg_status adg_cfl(adg_mesh *mesh, const double *u, double *dt, hipStream_t stream)
{
    if (!valid_mesh(mesh) || !u || !dt) {
        set_error("adg_cfl: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    return do_cfl(mesh, u, dt, nullptr, stream);
}

adg_status adg_predictor(adg_mesh *mesh, const double *u, const double *dt, double *ustar, void *traces,
                         hipStream_t stream)
{
    if (!valid_mesh(mesh) || !u || !dt || !ustar || !traces) {
        set_error("adg_predictor: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    if (mesh->prec == ADG_FP64)
        return do_predictor<double>(mesh, u, dt, ustar, static_cast<double *>(traces), stream, stream, false);
    return do_predictor<float>(mesh, u, dt, ustar, static_cast<float *>(traces), stream, stream, false);
}

adg_status adg_riemann(adg_mesh *mesh, const void *traces, void *fside, hipStream_t stream)
{
    if (!valid_mesh(mesh) || !traces || !fside) {
        set_error("adg_riemann: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    adg_status st;
    if (mesh->prec == ADG_FP64) {
        st = do_conforming<double>(mesh, static_cast<const double *>(traces), static_cast<double *>(fside), stream);
        if (st == ADG_OK)
            st = do_hanging<double>(mesh, static_cast<const double *>(traces), static_cast<double *>(fside), stream);
    } else {
        st = do_conforming<float>(mesh, static_cast<const float *>(traces), static_cast<float *>(fside), stream);
        if (st == ADG_OK)
            st = do_hanging<float>(mesh, static_cast<const float *>(traces), static_cast<float *>(fside), stream);
    }
    return st;
}

adg_status adg_corrector(adg_mesh *mesh, const double *ustar, const void *fside, const double *dt, double *uout,
                         hipStream_t stream)
{
    if (!valid_mesh(mesh) || !ustar || !fside || !dt || !uout) {
        set_error("adg_corrector: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    if (mesh->prec == ADG_FP64)
        return do_corrector<double>(mesh, ustar, static_cast<const double *>(fside), dt, uout, stream);
    return do_corrector<float>(mesh, ustar, static_cast<const float *>(fside), dt, uout, stream);
}

adg_status adg_step(adg_mesh *mesh, double *u, int32_t n_steps, double t_end, double *dt_hist, void *ws,
                    hipStream_t s_skel, hipStream_t s_encl)
{
    if (!valid_mesh(mesh) || !u || !ws || n_steps < 0) {
        set_error("adg_step: null argument or negative step count");
        return ADG_ERR_INVALID_ARG;
    }
    if (reinterpret_cast<uintptr_t>(ws) % ALIGN != 0) {
        set_error("adg_step: workspace must be 256-byte aligned");
        return ADG_ERR_WORKSPACE;
    }
    if (mesh->prec == ADG_FP64) return step_impl<double>(mesh, u, n_steps, t_end, dt_hist, ws, s_skel, s_encl);
    return step_impl<float>(mesh, u, n_steps, t_end, dt_hist, ws, s_skel, s_encl);
}

adg_status adg_step_noalloc(adg_mesh *mesh, double *u, int32_t n_steps, double t_end, double *dt_hist,
                            hipStream_t stream)
{
    if (!valid_mesh(mesh) || !u || n_steps < 0) {
        set_error("adg_step_noalloc: null argument or negative step count");
        return ADG_ERR_INVALID_ARG;
    }
    if (mesh->info.workspace_bytes > ADG_NOALLOC_WORKSPACE_BYTES) {
        set_error("adg_step_noalloc: the mesh needs " + std::to_string(mesh->info.workspace_bytes) +
                  " workspace bytes, more than the static " + std::to_string(ADG_NOALLOC_WORKSPACE_BYTES) +
                  "; use adg_step with a caller workspace");
        return ADG_ERR_WORKSPACE;
    }
    if (mesh->prof) {
        set_error("adg_step_noalloc: phase timing creates events; switch adg_profile off");
        return ADG_ERR_UNSUPPORTED;
    }
    void *ws = g_scratch_ptr[mesh->device];
    if (!ws) {
        set_error("adg_step_noalloc: static workspace not set up on the handle's device");
        return ADG_ERR_HIP;
    }
    if (n_steps == 0) return ADG_OK;
    adg_status st = start_clock(mesh, t_end, stream);
    if (st != ADG_OK) return st;
    // plain launches on one stream: no graph is instantiated
    if (mesh->prec == ADG_FP64) return step_eager<double>(mesh, u, n_steps, dt_hist, ws, stream, stream);
    return step_eager<float>(mesh, u, n_steps, dt_hist, ws, stream, stream);
}

adg_status adg_autotune(adg_mesh *mesh, const double *u, void *ws, hipStream_t stream)
{
    if (!valid_mesh(mesh) || !u || !ws) {
        set_error("adg_autotune: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    if (mesh->nitems == 0) {
        set_error("adg_autotune: the handle has hanging faces; only uniform instances are batched");
        return ADG_ERR_UNSUPPORTED;
    }
    if (mesh->prec == ADG_FP64) return autotune_impl<double>(mesh, u, ws, stream);
    return autotune_impl<float>(mesh, u, ws, stream);
}

adg_status adg_tuning(const adg_mesh *mesh, int32_t *cells_per_block)
{
    if (!valid_mesh(mesh) || !cells_per_block) {
        set_error("adg_tuning: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    for (int N = 1; N <= NMAX; ++N) {
        int vn, cpb;
        pred_variant_shape(mesh->codes[N], &vn, &cpb);
        cells_per_block[N - 1] = cpb;
    }
    return ADG_OK;
}

adg_status adg_set_options(adg_mesh *mesh, int32_t use_graph, int32_t batched)
{
    if (!valid_mesh(mesh)) return ADG_ERR_INVALID_ARG;
    if (batched < 0 || batched > 2) {
        set_error("adg_set_options: batched must be 0, 1 or 2");
        return ADG_ERR_INVALID_ARG;
    }
    if (batched && mesh->nitems == 0) {
        set_error("adg_set_options: batching needs instances without hanging faces");
        return ADG_ERR_UNSUPPORTED;
    }
    mesh->use_graph = use_graph != 0;
    mesh->batched = batched;
    drop_graph(mesh);
    return ADG_OK;
}

adg_status adg_set_face_fusion(adg_mesh *mesh, int32_t enable)
{
    if (!valid_mesh(mesh)) return ADG_ERR_INVALID_ARG;
    mesh->fuse_faces = enable != 0;
    drop_graph(mesh);
    return ADG_OK;
}

adg_status adg_set_pipeline(adg_mesh *mesh, int32_t enable)
{
    if (!valid_mesh(mesh)) return ADG_ERR_INVALID_ARG;
    if (enable && mesh->inst[0].ps == 0) {
        set_error("adg_set_pipeline: the pipelined step needs a single instance without hanging faces");
        return ADG_ERR_UNSUPPORTED;
    }
    if (enable < 0 || enable > 2) {
        set_error("adg_set_pipeline: mode must be 0, 1 or 2");
        return ADG_ERR_INVALID_ARG;
    }
    ADG_HIP(hipDeviceSynchronize(), "synchronize");
    mesh->pipeline = enable;
    drop_graph(mesh);
    return ADG_OK;
}

adg_status adg_set_limiter(adg_mesh *mesh, int32_t mode, double delta0, double eps)
{
    if (!valid_mesh(mesh)) return ADG_ERR_INVALID_ARG;
    if (mode < 0 || mode > 2 || !(delta0 >= 0.0) || !(eps >= 0.0)) {
        set_error("adg_set_limiter: mode must be 0, 1 or 2 and delta0, eps non-negative");
        return ADG_ERR_INVALID_ARG;
    }
    if (mode && (mesh->inst.size() != 1 || mesh->inst[0].N > LIM_NMAX)) {
        set_error("adg_set_limiter: the limiter needs a single instance with p <= 6");
        return ADG_ERR_UNSUPPORTED;
    }
    DeviceGuard dg(mesh->device);
    ADG_HIP(hipDeviceSynchronize(), "synchronize");
    if (mode && !mesh->lim.uold) {
        Instance &I = mesh->inst[0];
        const size_t nc = size_t(I.nc);
        LimDev L{};
        bool ok = dev_alloc(mesh, L.uold, size_t(mesh->info.u_elems)) && dev_alloc(mesh, L.mm, nc * 2 * NV) &&
                  dev_alloc(mesh, L.fb, nc) && dev_alloc(mesh, L.mm2, nc * 2 * NV) && dev_alloc(mesh, L.fb2, nc) && dev_alloc(mesh, L.nbr, 6 * nc) && dev_alloc(mesh, L.flag, nc) &&
                  dev_alloc(mesh, L.list, nc) && dev_alloc(mesh, L.rlist, nc) && dev_alloc(mesh, L.cnt, 2) &&
                  dev_alloc(mesh, mesh->lim_status, 1);
        if (!ok) {
            set_error("adg_set_limiter: device allocation failed");
            return ADG_ERR_OOM;
        }
        ADG_HIP(hipMemset(L.flag, 0, nc * sizeof(int32_t)), "limiter flags");
        ADG_HIP(hipMemset(L.cnt, 0, 2 * sizeof(int32_t)), "limiter counters");
        ADG_HIP(hipMemset(mesh->lim_status, 0, sizeof(int)), "limiter status sink");
        // same-level neighbours from the conforming faces; -1 marks a hanging side
        ADG_HIP(hipMemset(L.nbr, 0xff, 6 * nc * sizeof(int32_t)), "neighbour table");
        L.level = I.level;
        for (int d = 0; d < 3; ++d)
            ADG_HIP(launch_lim_nbr(I.face_m[d], I.face_p[d], I.nf[d], d, I.nc, L.nbr, nullptr), "neighbour table");
        ADG_HIP(hipDeviceSynchronize(), "synchronize");
        mesh->lim = L;
    }
    mesh->lim_mode = mode;
    mesh->lim_delta0 = delta0;
    mesh->lim_eps = eps;
    drop_graph(mesh);
    return ADG_OK;
}

adg_status adg_limiter_stats(adg_mesh *mesh, int64_t *n_limited, int64_t *n_recorrected, int32_t *flags_dev,
                             hipStream_t stream)
{
    if (!valid_mesh(mesh)) return ADG_ERR_INVALID_ARG;
    if (!mesh->lim.uold) {
        set_error("adg_limiter_stats: the limiter was never enabled on this handle");
        return ADG_ERR_INVALID_ARG;
    }
    int32_t cnt[2] = {0, 0};
    ADG_HIP(hipMemcpyAsync(cnt, mesh->lim.cnt, sizeof(cnt), hipMemcpyDeviceToHost, stream), "counter read");
    if (flags_dev)
        ADG_HIP(hipMemcpyAsync(flags_dev, mesh->lim.flag, size_t(mesh->inst[0].nc) * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, stream),
                "flag copy");
    ADG_HIP(hipStreamSynchronize(stream), "synchronize");
    if (n_limited) *n_limited = cnt[0];
    if (n_recorrected) *n_recorrected = cnt[1];
    return ADG_OK;
}

adg_status adg_profile(adg_mesh *mesh, int32_t enable)
{
    if (!valid_mesh(mesh)) return ADG_ERR_INVALID_ARG;
    if (enable) {
        ADG_HIP(hipDeviceSynchronize(), "synchronize");
        mesh->recs.clear();
        mesh->ev_used = 0;
    }
    if (enable < 0 || enable > 2) {
        set_error("adg_profile: enable must be 0, 1 or 2");
        return ADG_ERR_INVALID_ARG;
    }
    mesh->prof = enable;
    return ADG_OK;
}

adg_status adg_profile_read(adg_mesh *mesh, double *ms, int64_t *launches)
{
    if (!valid_mesh(mesh) || !ms || !launches) {
        set_error("adg_profile_read: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    for (int k = 0; k < ADG_NPHASES; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (const auto &r : mesh->recs) {
        ADG_HIP(hipEventSynchronize(r.b), "event synchronize");
        float t = 0.0f;
        ADG_HIP(hipEventElapsedTime(&t, r.a, r.b), "event elapsed");
        ms[r.phase] += double(t);
        launches[r.phase] += 1;
    }
    return ADG_OK;
}

adg_status adg_set_switch_tape(adg_mesh *mesh, int16_t *tape, int32_t mode)
{
    if (!valid_mesh(mesh) || mode < 0 || mode > 2 || (mode != 0 && !tape)) {
        set_error("adg_set_switch_tape: bad argument");
        return ADG_ERR_INVALID_ARG;
    }
    mesh->tape = mode ? tape : nullptr;
    mesh->tape_mode = mode;
    drop_graph(mesh);
    return ADG_OK;
}

// The adjoint of one step; with a tape (recorded by adg_step_record) the
// forward predictor's face projections and iterates come from it instead of
// a new predictor run.
static adg_status adjoint_impl(adg_mesh *mesh, const double *u, const double *dt, const double *ubar_next,
                               double *ubar, void *ws, const void *tape, hipStream_t stream, const char *who)
{
    if (!valid_mesh(mesh) || !u || !dt || !ubar_next || !ubar || !ws) {
        set_error(std::string(who) + ": null argument");
        return ADG_ERR_INVALID_ARG;
    }
    if (ubar == ubar_next) {
        set_error(std::string(who) + ": ubar_n must not alias ubar_np1");
        return ADG_ERR_INVALID_ARG;
    }
    if (mesh->prec != ADG_FP64) {
        set_error(std::string(who) + ": needs an FP64 handle");
        return ADG_ERR_UNSUPPORTED;
    }
    if (mesh->lim_mode) {
        set_error(std::string(who) + ": the adjoint is that of the unlimited step; switch the limiter off");
        return ADG_ERR_UNSUPPORTED;
    }
    char *w = static_cast<char *>(ws);
    double *ustar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * mesh->info.u_elems);
    double *traces = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * mesh->info.trace_elems);
    double *tbar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * mesh->info.trace_elems);
    double *fbar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * mesh->info.fside_elems);
    double *iters = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * std::max<int64_t>(adjoint_iter_elems(mesh), 1));
    double *vbar = reinterpret_cast<double *>(w);
    if (tape) {
        char *t = static_cast<char *>(const_cast<void *>(tape));
        traces = reinterpret_cast<double *>(t);
        iters = reinterpret_cast<double *>(t + align_up(sizeof(double) * mesh->info.trace_elems));
    }
    for (size_t i = 0; i < mesh->inst.size(); ++i) {
        Instance &I = mesh->inst[i];
        const int32_t *fm[3] = {I.face_m[0], I.face_m[1], I.face_m[2]};
        const int32_t *fp[3] = {I.face_p[0], I.face_p[1], I.face_p[2]};
        AdjHang ah;
        ah.hang = I.hang;
        ah.nh = I.nh;
        ah.ccell = I.ccell;
        ah.cptr = I.cptr;
        ah.cchild = I.cchild;
        ah.cside = I.cside;
        ah.ncs = I.ncs;
        ah.ptab = I.ptab;
        ah.vbar = vbar;
        ADG_HIP(launch_adjoint_step(I.N, u + I.u_off, dt + i, ubar_next + I.u_off, ubar + I.u_off, ustar + I.u_off,
                                    traces + I.tr_off, tbar + I.tr_off, fbar + I.fs_off, iters, fm, fp, I.nf, I.nc,
                                    I.level, I.geo, I.gamma, I.npic, ah, stream, tape == nullptr),
                "adjoint step");
        iters += int64_t(I.npic) * I.N * NV * I.nc * I.N * I.N * I.N;
        vbar += I.nh * 2 * NV * I.N * I.N;
    }
    return ADG_OK;
}

adg_status adg_step_adjoint(adg_mesh *mesh, const double *u, const double *dt, const double *ubar_next,
                            double *ubar, void *ws, hipStream_t stream)
{
    return adjoint_impl(mesh, u, dt, ubar_next, ubar, ws, nullptr, stream, "adg_step_adjoint");
}

adg_status adg_step_adjoint_tape(adg_mesh *mesh, const double *u, const double *dt, const void *tape,
                                 const double *ubar_next, double *ubar, void *ws, hipStream_t stream)
{
    if (!tape) {
        set_error("adg_step_adjoint_tape: null tape");
        return ADG_ERR_INVALID_ARG;
    }
    return adjoint_impl(mesh, u, dt, ubar_next, ubar, ws, tape, stream, "adg_step_adjoint_tape");
}

adg_status adg_step_record(adg_mesh *mesh, const double *u, const double *dt, double *u_next, void *tape, void *ws,
                           hipStream_t stream)
{
    if (!valid_mesh(mesh) || !u || !dt || !ws || (!tape && !u_next)) {
        set_error("adg_step_record: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    if (mesh->prec != ADG_FP64) {
        set_error("adg_step_record: needs an FP64 handle");
        return ADG_ERR_UNSUPPORTED;
    }
    if (mesh->lim_mode) {
        set_error("adg_step_record: the recorded step is the unlimited one; switch the limiter off");
        return ADG_ERR_UNSUPPORTED;
    }
    // u* and the face fluxes in the adjoint workspace's u* and fbar slots
    char *w = static_cast<char *>(ws);
    double *ustar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * mesh->info.u_elems) + 2 * align_up(sizeof(double) * mesh->info.trace_elems);
    double *fside = reinterpret_cast<double *>(w);
    // no tape: a plain step at the fixed dt, its face projections in the
    // workspace's trace slot
    double *traces = reinterpret_cast<double *>(static_cast<char *>(ws) + align_up(sizeof(double) * mesh->info.u_elems));
    double *iters = nullptr;
    if (tape) {
        char *t = static_cast<char *>(tape);
        traces = reinterpret_cast<double *>(t);
        iters = reinterpret_cast<double *>(t + align_up(sizeof(double) * mesh->info.trace_elems));
    }
    for (size_t i = 0; i < mesh->inst.size(); ++i) {
        Instance &I = mesh->inst[i];
        ADG_HIP(launch_predictor<double>(I.N, u + I.u_off, ustar + I.u_off, traces + I.tr_off, nullptr, I.nc, I.nc,
                                         I.level, I.geo, dt + i, I.gamma, I.npic, stream, iters),
                "recorded predictor");
        if (iters) iters += int64_t(I.npic) * I.N * NV * I.nc * I.N * I.N * I.N;
    }
    if (!u_next) return ADG_OK;
    if (can_fuse_faces(mesh)) return do_face_corrector<double>(mesh, ustar, traces, dt, u_next, stream, false);
    adg_status st = do_conforming<double>(mesh, traces, fside, stream);
    if (st == ADG_OK) st = do_hanging<double>(mesh, traces, fside, stream);
    if (st == ADG_OK) st = do_corrector<double>(mesh, ustar, fside, dt, u_next, stream);
    return st;
}

static adg_status sample_geo(adg_mesh *mesh, SampleGeo &sg)
{
    if (mesh->inst.size() != 1 || mesh->inst[0].hm.max_level > 0) {
        set_error("point sampling needs a single-instance uniform handle");
        return ADG_ERR_UNSUPPORTED;
    }
    const Instance &I = mesh->inst[0];
    for (int d = 0; d < 3; ++d) {
        sg.n[d] = I.hm.n[d];
        sg.lo[d] = I.hm.lo[d];
        sg.inv_h[d] = I.geo.inv_dx[0][d];
    }
    return ADG_OK;
}

adg_status adg_sample(adg_mesh *mesh, const double *u, const double *pts, int64_t n_pts, double *out,
                      hipStream_t stream)
{
    if (!valid_mesh(mesh) || !u || (n_pts > 0 && (!pts || !out)) || n_pts < 0) {
        set_error("adg_sample: bad argument");
        return ADG_ERR_INVALID_ARG;
    }
    SampleGeo sg;
    adg_status st = sample_geo(mesh, sg);
    if (st != ADG_OK) return st;
    const Instance &I = mesh->inst[0];
    ADG_HIP(launch_sample(I.N, u, I.nc, sg, pts, n_pts, out, stream), "sample");
    return ADG_OK;
}

adg_status adg_sample_adjoint(adg_mesh *mesh, const double *pts, const double *wbar, int64_t n_pts, double *ubar,
                              hipStream_t stream)
{
    if (!valid_mesh(mesh) || !ubar || (n_pts > 0 && (!pts || !wbar)) || n_pts < 0 || n_pts >= (int64_t(1) << 31)) {
        set_error("adg_sample_adjoint: bad argument");
        return ADG_ERR_INVALID_ARG;
    }
    SampleGeo sg;
    adg_status st = sample_geo(mesh, sg);
    if (st != ADG_OK) return st;
    const Instance &I = mesh->inst[0];
    ADG_HIP(launch_sample_adjoint(I.N, pts, wbar, n_pts, sg, ubar, stream), "sample adjoint");
    return ADG_OK;
}

adg_status adg_get_status(adg_mesh *mesh)
{
    if (!valid_mesh(mesh)) return ADG_ERR_INVALID_ARG;
    ADG_HIP(hipDeviceSynchronize(), "synchronize");
    int flag = 0;
    ADG_HIP(hipMemcpy(&flag, mesh->status_dev, sizeof(int), hipMemcpyDeviceToHost), "status read");
    if (flag) {
        int zero = 0;
        ADG_HIP(hipMemcpy(mesh->status_dev, &zero, sizeof(int), hipMemcpyHostToDevice), "status reset");
        set_error("non-physical state (rho <= 0, p <= 0 or non-finite) met on the device");
        return ADG_ERR_NONPHYSICAL;
    }
    return ADG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Dynamic adaptivity (Sec. 2.3, dynamic-adaptivity paragraph)
// ---------------------------------------------------------------------------

namespace {

int64_t pow3i(int e)
{
    int64_t r = 1;
    while (e-- > 0) r *= 3;
    return r;
}

// Leaves of `from` inside region (l, q) of target cell (lc, kc), in the order
// z, y, x of the sub-cells at every level; adds 27^(depth - dl) per leaf to
// *cover (depth = max_level - lc), which sums to 27^depth when covered.
void collect_kids(const adg::CellIndex &index, int max_level, int lc, const int64_t *kc,
                  int l, const int64_t *q, std::vector<adg::VKid> &kids, int64_t &cover)
{
    const int32_t f = index.find(l, q[0], q[1], q[2]);
    if (f >= 0) {
        const int dl = l - lc;
        const int64_t r = pow3i(dl);
        adg::VKid k{f, int8_t(dl), {int8_t(q[0] - r * kc[0]), int8_t(q[1] - r * kc[1]),
                                    int8_t(q[2] - r * kc[2])}};
        kids.push_back(k);
        cover += pow3i(3 * (max_level - lc - dl));
        return;
    }
    if (l >= max_level) return;
    for (int c2 = 0; c2 < 3; ++c2)
        for (int c1 = 0; c1 < 3; ++c1)
            for (int c0 = 0; c0 < 3; ++c0) {
                const int64_t q2[3] = {3 * q[0] + c0, 3 * q[1] + c1, 3 * q[2] + c2};
                collect_kids(index, max_level, lc, kc, l + 1, q2, kids, cover);
            }
}

// The next refine rows from the current leaves hm (built from the rows
// refine[0 .. 4 n_refine)) and the indicator eta per leaf: the current rows
// minus the merged parents, plus the split leaves, sorted by (level, k, j, i).
adg_status plan_rows(const adg::HostMesh &hm, const adg::CellIndex &index, const int32_t *refine, int64_t n_refine,
                     const double *eta, double theta_refine, double theta_coarsen, int32_t *refine_out,
                     int64_t capacity, int64_t *n_refine_out, const char *who)
{
    using namespace adg;
    auto split = [&](int64_t c) { return eta[c] > theta_refine && hm.level[c] < hm.max_level; };
    // current rows minus the merged parents, plus the split leaves
    struct Row { int32_t l, i, j, k; };
    // a row merges when its 27 children are leaves, none split, all quiet;
    // the three children along x of one (k, j) row of children are
    // consecutive in the cell table, so one lookup finds them
    std::vector<char> keep(static_cast<size_t>(std::max<int64_t>(n_refine, 1)));
    parallel_for(n_refine, [&](int64_t r0, int64_t r1) {
        for (int64_t r = r0; r < r1; ++r) {
            const int32_t *q = refine + 4 * r;
            const int lc = q[0] + 1;
            const int64_t i0 = 3 * int64_t(q[1]);
            bool merge = true;
            for (int c2 = 0; c2 < 3 && merge; ++c2)
                for (int c1 = 0; c1 < 3 && merge; ++c1) {
                    const int64_t j = 3 * int64_t(q[2]) + c1, k = 3 * int64_t(q[3]) + c2;
                    const int64_t f = index.find(lc, i0, j, k);
                    for (int c0 = 0; c0 < 3 && merge; ++c0) {
                        const int64_t g = f + c0;
                        merge = f >= 0 && g < hm.nc && hm.level[g] == lc && hm.ijk[3 * g] == i0 + c0 &&
                                hm.ijk[3 * g + 1] == j && hm.ijk[3 * g + 2] == k && !split(g) &&
                                eta[g] < theta_coarsen;
                    }
                }
            keep[size_t(r)] = !merge;
        }
    }, 4096);
    std::vector<Row> rows;
    for (int64_t r = 0; r < n_refine; ++r)
        if (keep[size_t(r)]) {
            const int32_t *q = refine + 4 * r;
            rows.push_back(Row{q[0], q[1], q[2], q[3]});
        }
    auto less = [](const Row &a, const Row &b) {
        if (a.l != b.l) return a.l < b.l;
        if (a.k != b.k) return a.k < b.k;
        if (a.j != b.j) return a.j < b.j;
        return a.i < b.i;
    };
    if (!std::is_sorted(rows.begin(), rows.end(), less)) std::sort(rows.begin(), rows.end(), less);
    // the split leaves, gathered per chunk in cell order, which is (level, k,
    // j, i) order: a merge with the kept rows sorts the plan
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(256, hm.nc / 8192));
    std::vector<std::vector<Row>> part(static_cast<size_t>(nch));
    parallel_for(nch, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t)
            for (int64_t c = hm.nc * t / nch; c < hm.nc * (t + 1) / nch; ++c)
                if (split(c))
                    part[size_t(t)].push_back(Row{hm.level[c], hm.ijk[3 * c], hm.ijk[3 * c + 1], hm.ijk[3 * c + 2]});
    }, 1);
    std::vector<Row> splits;
    for (auto &p : part) splits.insert(splits.end(), p.begin(), p.end());
    std::vector<Row> merged;
    merged.reserve(rows.size() + splits.size());
    std::merge(rows.begin(), rows.end(), splits.begin(), splits.end(), std::back_inserter(merged), less);
    rows.swap(merged);
    *n_refine_out = int64_t(rows.size());
    if (!refine_out || capacity < int64_t(rows.size())) {
        set_error(std::string(who) + ": refine_out holds fewer rows than the plan (count returned in n_refine_out)");
        return ADG_ERR_WORKSPACE;
    }
    for (size_t r = 0; r < rows.size(); ++r) {
        refine_out[4 * r] = rows[r].l;
        refine_out[4 * r + 1] = rows[r].i;
        refine_out[4 * r + 2] = rows[r].j;
        refine_out[4 * r + 3] = rows[r].k;
    }
    return ADG_OK;
}

}  // namespace

extern "C" {

adg_status adg_indicator(adg_mesh *mesh, const double *u, double *eta, hipStream_t stream)
{
    if (!valid_mesh(mesh) || !u || !eta) {
        set_error("adg_indicator: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    for (auto &I : mesh->inst)
        ADG_HIP(launch_indicator(I.N, u + I.u_off, I.nc, eta + I.cell_off, stream), "indicator");
    return ADG_OK;
}

adg_status adg_transfer(const adg_mesh *from, const double *u_from, adg_mesh *to, double *u_to, hipStream_t stream)
{
    if (!valid_mesh(from) || !valid_mesh(to) || !u_from || !u_to) {
        set_error("adg_transfer: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    if (from->inst.size() != 1 || to->inst.size() != 1) {
        set_error("adg_transfer: handles must hold one instance each");
        return ADG_ERR_UNSUPPORTED;
    }
    const Instance &F = from->inst[0];
    Instance &T = to->inst[0];
    bool same = F.N == T.N;
    for (int a = 0; a < 3; ++a)
        same = same && F.hm.n[a] == T.hm.n[a] && F.hm.lo[a] == T.hm.lo[a] && F.hm.hi[a] == T.hm.hi[a];
    if (!same) {
        set_error("adg_transfer: the meshes differ in order or base grid");
        return ADG_ERR_INVALID_ARG;
    }
    const CellIndex &index = F.index;
    // copy (the same leaf) or prolongation (a coarser leaf covers the cell),
    // in parallel; the rest are coarsened cells, gathered in order afterwards
    // every entry is written by the loop below (first touch on its threads)
    std::unique_ptr<VOp[]> ops(new VOp[size_t(std::max<int64_t>(T.nc, 1))]);
    parallel_for(T.nc, [&](int64_t c0, int64_t c1) {
        for (int64_t c = c0; c < c1; ++c) {
            const int l = T.hm.level[size_t(c)];
            const int64_t k[3] = {T.hm.ijk[size_t(3 * c)], T.hm.ijk[size_t(3 * c + 1)], T.hm.ijk[size_t(3 * c + 2)]};
            VOp op{};
            op.kind = 2;
            int32_t f = index.find(l, k[0], k[1], k[2]);
            if (f >= 0) {
                op.kind = 0;
                op.src = f;
            }
            for (int lp = l - 1; lp >= 0 && op.kind == 2; --lp) {
                const int64_t r = pow3i(l - lp);
                f = index.find(lp, k[0] / r, k[1] / r, k[2] / r);
                if (f < 0) continue;
                op.kind = 1;
                op.src = f;
                op.dl = int8_t(l - lp);
                for (int d = 0; d < 3; ++d) op.s[d] = int8_t(k[d] % r);
            }
            ops[size_t(c)] = op;
        }
    });
    // the source leaves of every coarsened cell, gathered per chunk of the
    // coarsened cells (they cluster in the cell table) and concatenated in
    // cell order
    std::vector<int32_t> coarsened;
    for (int64_t c = 0; c < T.nc; ++c)
        if (ops[size_t(c)].kind == 2) coarsened.push_back(int32_t(c));
    const int64_t ncs = int64_t(coarsened.size());
    const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(256, ncs / 64));
    auto cbeg = [&](int64_t t) { return ncs * t / nch; };
    std::vector<std::vector<VKid>> part(static_cast<size_t>(nch));
    std::vector<char> partial_cover(static_cast<size_t>(nch), 0);
    parallel_for(nch, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t)
            for (int64_t x = cbeg(t); x < cbeg(t + 1); ++x) {
                const int64_t c = coarsened[size_t(x)];
                VOp &op = ops[size_t(c)];
                const int l = T.hm.level[size_t(c)];
                const int64_t k[3] = {T.hm.ijk[size_t(3 * c)], T.hm.ijk[size_t(3 * c + 1)],
                                      T.hm.ijk[size_t(3 * c + 2)]};
                int64_t cover = 0;
                op.kid0 = int32_t(part[size_t(t)].size());  // within the chunk for now
                collect_kids(index, F.hm.max_level, l, k, l, k, part[size_t(t)], cover);
                op.nkid = int32_t(part[size_t(t)].size()) - op.kid0;
                if (op.nkid == 0 || cover != pow3i(3 * (F.hm.max_level - l))) partial_cover[size_t(t)] = 1;
            }
    }, 1);
    std::vector<int64_t> kid_off(size_t(nch) + 1, 0);
    for (int64_t t = 0; t < nch; ++t) {
        if (partial_cover[size_t(t)]) {
            set_error("adg_transfer: a cell of the target mesh is only partly covered by the source mesh");
            return ADG_ERR_INVALID_ARG;
        }
        kid_off[size_t(t) + 1] = kid_off[size_t(t)] + int64_t(part[size_t(t)].size());
    }
    if (kid_off[size_t(nch)] > INT32_MAX) {
        set_error("adg_transfer: too many source cells under coarsened cells");
        return ADG_ERR_UNSUPPORTED;
    }
    std::vector<VKid> kids(static_cast<size_t>(kid_off[static_cast<size_t>(nch)]));
    parallel_for(nch, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            std::copy(part[size_t(t)].begin(), part[size_t(t)].end(), kids.begin() + kid_off[size_t(t)]);
            for (int64_t x = cbeg(t); x < cbeg(t + 1); ++x)
                ops[size_t(coarsened[size_t(x)])].kid0 += int32_t(kid_off[size_t(t)]);
        }
    }, 1);
    VOp *ops_dev = nullptr;
    VKid *kids_dev = nullptr;
    DeviceGuard dg(to->device);
    ADG_HIP(hipMalloc(&ops_dev, sizeof(VOp) * size_t(T.nc)), "transfer table");
    hipError_t e = hipMalloc(&kids_dev, sizeof(VKid) * std::max<size_t>(1, kids.size()));
    if (e == hipSuccess) e = hipMemcpyAsync(ops_dev, ops.get(), sizeof(VOp) * size_t(T.nc), hipMemcpyHostToDevice,
                                            stream);
    if (e == hipSuccess && !kids.empty())
        e = hipMemcpyAsync(kids_dev, kids.data(), sizeof(VKid) * kids.size(), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_vtransfer(T.N, u_from, F.nc, u_to, T.nc, ops_dev, kids_dev, T.ptab, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    (void)hipFree(ops_dev);
    if (kids_dev) (void)hipFree(kids_dev);
    if (e != hipSuccess) return hip_fail(e, "volumetric transfer");
    return ADG_OK;
}

adg_status adg_adapt_plan(const adg_instance_desc *desc, const double *eta, double theta_refine, double theta_coarsen,
                          int32_t *refine_out, int64_t capacity, int64_t *n_refine_out)
{
    if (!desc || !eta || !n_refine_out) {
        set_error("adg_adapt_plan: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    HostMesh hm;
    std::string err = build_host_mesh(*desc, hm, true);
    if (!err.empty()) {
        set_error("adg_adapt_plan: " + err);
        return err.rfind("unsupported", 0) == 0 ? ADG_ERR_UNSUPPORTED : ADG_ERR_INVALID_ARG;
    }
    CellIndex index;
    index.build(hm);
    return plan_rows(hm, index, desc->refine, desc->n_refine, eta, theta_refine, theta_coarsen, refine_out, capacity,
                     n_refine_out, "adg_adapt_plan");
}

adg_status adg_adapt_plan_mesh(const adg_mesh *mesh, const double *eta, double theta_refine, double theta_coarsen,
                               int32_t *refine_out, int64_t capacity, int64_t *n_refine_out)
{
    if (!valid_mesh(mesh) || !eta || !n_refine_out) {
        set_error("adg_adapt_plan_mesh: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    if (mesh->inst.size() != 1) {
        set_error("adg_adapt_plan_mesh: the handle must hold one instance");
        return ADG_ERR_UNSUPPORTED;
    }
    const Instance &I = mesh->inst[0];
    return plan_rows(I.hm, I.index, I.refine.data(), int64_t(I.refine.size() / 4), eta, theta_refine, theta_coarsen,
                     refine_out, capacity, n_refine_out, "adg_adapt_plan_mesh");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Linear variant: elastic waves with the Cauchy-Kowalevski predictor
// ---------------------------------------------------------------------------

struct adg_lin {
    int device = 0;
    int N = 0;
    int n[3] = {0, 0, 0};
    double inv_dx[3] = {0, 0, 0};
    double cfl = 0.0;
    int64_t nc = 0;
    double *dt_dev = nullptr;
    bool fuse_faces = true;  // N = 4: faces inside the corrector
};

namespace {

bool valid_lin(const adg_lin *l) { return l && l->nc > 0 && l->dt_dev; }

size_t lin_u_elems(const adg_lin *l) { return size_t(9) * size_t(l->nc) * size_t(l->N * l->N * l->N); }
size_t lin_trace_elems(const adg_lin *l) { return size_t(6 * 2 * 9) * size_t(l->nc) * size_t(l->N * l->N); }
size_t lin_fside_elems(const adg_lin *l) { return size_t(6 * 9) * size_t(l->nc) * size_t(l->N * l->N); }

adg_status lin_dt(adg_lin *l, const double *material, hipStream_t st)
{
    const double sum_inv = l->inv_dx[0] + l->inv_dx[1] + l->inv_dx[2];
    const double factor = l->cfl / ((2.0 * (l->N - 1) + 1.0) * sum_inv);
    ADG_HIP(launch_lin_cfl(material, l->nc, factor, l->dt_dev, st), "linear time step");
    return ADG_OK;
}

}  // namespace

extern "C" {

adg_status adg_lin_init(const adg_lin_desc *desc, adg_lin **out)
{
    if (!desc || !out) {
        set_error("adg_lin_init: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    if (desc->order < 0 || desc->order > 6) {
        set_error("adg_lin_init: order must be in [0, 6]");
        return ADG_ERR_UNSUPPORTED;
    }
    for (int a = 0; a < 3; ++a)
        if (desc->n[a] < 1 || !(desc->hi[a] > desc->lo[a])) {
            set_error("adg_lin_init: need n >= 1 and hi > lo on every axis");
            return ADG_ERR_INVALID_ARG;
        }
    if (!(desc->cfl > 0.0)) {
        set_error("adg_lin_init: cfl must be > 0");
        return ADG_ERR_INVALID_ARG;
    }
    const int64_t nc = int64_t(desc->n[0]) * desc->n[1] * desc->n[2];
    if (nc * (desc->order + 1) * (desc->order + 1) >= (int64_t(1) << 31) / 2) {
        set_error("adg_lin_init: mesh too large for one launch");
        return ADG_ERR_UNSUPPORTED;
    }
    int dev = 0;
    ADG_HIP(hipGetDevice(&dev), "get device");
    adg_status bs = ensure_basis(dev);
    if (bs != ADG_OK) return bs;
    auto *l = new adg_lin;
    l->device = dev;
    l->N = desc->order + 1;
    l->nc = nc;
    l->cfl = desc->cfl;
    for (int a = 0; a < 3; ++a) {
        l->n[a] = desc->n[a];
        l->inv_dx[a] = desc->n[a] / (desc->hi[a] - desc->lo[a]);
    }
    if (hipMalloc(&l->dt_dev, sizeof(double)) != hipSuccess) {
        delete l;
        set_error("adg_lin_init: device allocation failed");
        return ADG_ERR_OOM;
    }
    *out = l;
    return ADG_OK;
}

adg_status adg_lin_free(adg_lin *lin)
{
    if (!lin) return ADG_OK;
    if (lin->dt_dev) (void)hipFree(lin->dt_dev);
    delete lin;
    return ADG_OK;
}

adg_status adg_lin_info(adg_lin *lin, int64_t *n_cells, int64_t *u_elems, int64_t *trace_elems, int64_t *fside_elems,
                        int64_t *workspace_bytes)
{
    if (!valid_lin(lin)) return ADG_ERR_INVALID_ARG;
    if (n_cells) *n_cells = lin->nc;
    if (u_elems) *u_elems = int64_t(lin_u_elems(lin));
    if (trace_elems) *trace_elems = int64_t(lin_trace_elems(lin));
    if (fside_elems) *fside_elems = int64_t(lin_fside_elems(lin));
    if (workspace_bytes)
        *workspace_bytes = int64_t(align_up(sizeof(double) * lin_u_elems(lin)) +
                                   align_up(sizeof(double) * lin_trace_elems(lin)) +
                                   align_up(sizeof(double) * lin_fside_elems(lin)));
    return ADG_OK;
}

adg_status adg_lin_dt(adg_lin *lin, const double *material, double *dt_dev, hipStream_t stream)
{
    if (!valid_lin(lin) || !material || !dt_dev) {
        set_error("adg_lin_dt: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    adg_status s = lin_dt(lin, material, stream);
    if (s != ADG_OK) return s;
    ADG_HIP(hipMemcpyAsync(dt_dev, lin->dt_dev, sizeof(double), hipMemcpyDeviceToDevice, stream), "dt copy");
    return ADG_OK;
}

adg_status adg_lin_predictor(adg_lin *lin, const double *material, const double *u, const double *dt_dev,
                             double *ustar, double *traces, hipStream_t stream)
{
    if (!valid_lin(lin) || !material || !u || !dt_dev || !ustar || !traces) {
        set_error("adg_lin_predictor: null argument");
        return ADG_ERR_INVALID_ARG;
    }
    ADG_HIP(launch_lin_predictor(lin->N, u, material, dt_dev, ustar, traces, lin->nc, lin->inv_dx, stream),
            "linear predictor");
    return ADG_OK;
}

adg_status adg_lin_set_face_fusion(adg_lin *lin, int32_t enable)
{
    if (!valid_lin(lin)) {
        set_error("adg_lin_set_face_fusion: invalid handle");
        return ADG_ERR_INVALID_ARG;
    }
    lin->fuse_faces = enable != 0;
    return ADG_OK;
}

adg_status adg_lin_step(adg_lin *lin, const double *material, double *u, int32_t n_steps, double *dt_out, void *ws,
                        hipStream_t stream)
{
    if (!valid_lin(lin) || !material || !u || !ws || n_steps < 0) {
        set_error("adg_lin_step: null argument or n_steps < 0");
        return ADG_ERR_INVALID_ARG;
    }
    char *w = static_cast<char *>(ws);
    double *ustar = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * lin_u_elems(lin));
    double *traces = reinterpret_cast<double *>(w);
    w += align_up(sizeof(double) * lin_trace_elems(lin));
    double *fside = reinterpret_cast<double *>(w);
    adg_status s = lin_dt(lin, material, stream);
    if (s != ADG_OK) return s;
    const bool fused = lin->N == 4 && lin->fuse_faces;
    for (int32_t k = 0; k < n_steps; ++k) {
        // the fused faces form the flux traces from the state traces
        ADG_HIP(launch_lin_predictor(lin->N, u, material, lin->dt_dev, ustar, traces, lin->nc, lin->inv_dx, stream,
                                     !fused),
                "linear predictor");
        if (fused) {
            ADG_HIP(launch_lin_face_corrector4(ustar, traces, material, lin->dt_dev, u, lin->nc, lin->n, lin->inv_dx,
                                               stream),
                    "linear faces and corrector");
            continue;
        }
        ADG_HIP(launch_lin_riemann(lin->N, traces, material, fside, lin->nc, lin->n, stream), "linear riemann");
        ADG_HIP(launch_lin_corrector(lin->N, ustar, fside, lin->dt_dev, u, lin->nc, lin->inv_dx, stream),
                "linear corrector");
    }
    if (dt_out) ADG_HIP(hipMemcpyAsync(dt_out, lin->dt_dev, sizeof(double), hipMemcpyDeviceToDevice, stream), "dt copy");
    return ADG_OK;
}

}  // extern "C"
