// Host runtime and C-ABI of librbl (see include/rbl.h).
//
// A context owns the cell-sorted particle state, the cell list, the sliced
// ELL neighbour lists, the pre-drawn batches and the reduction buffers, all in
// HBM.  Every call queues kernels on the context's stream; the only host
// synchronisations are the capacity check after a list build and the flag
// read-back at the end of rbl_step / rbl_sync.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rbl.h"
#include "kernels.h"

using namespace rbl;

namespace {

thread_local std::string g_err;

rbl_status fail(rbl_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? RBL_E_NOMEM : RBL_E_HIP,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define RBL_TRY(expr)                      \
    do {                                   \
        rbl_status s_ = (expr);            \
        if (s_ < 0) return s_;             \
    } while (0)

constexpr int kBlock = 256;
constexpr int kKinds = 7;
enum { kKForceRbl = 0, kKForceFull = 1, kKBuild = 2, kKBin = 3, kKIntegrate = 4, kKReduce = 5,
       kKPredraw = 6 };

inline unsigned grid_for(int64_t n, int block = kBlock)
{
    return (unsigned)((n + block - 1) / block);
}

template <typename T>
rbl_status dalloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(e == hipErrorOutOfMemory ? RBL_E_NOMEM : RBL_E_HIP,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return RBL_OK;
}

template <typename T>
void dfree(T*& p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

// Device memory of rbl_forces_noalloc: one static array per device (each GPU
// holds its own copy for the life of the process).  Host code never passes
// the array's name to a kernel: its device address is taken once per device
// with hipGetSymbolAddress (rbl_create, with that device current) and kept
// in scratch_dev[device].  Calls on one device share the array.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kScratchDevices] = {};
bool scratch_tried[kScratchDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Address of the scratch array on the current device (null if unavailable).
void* scratch_setup(int dev)
{
    if (dev < 0 || dev >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_tried[dev]) {
        scratch_tried[dev] = true;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) scratch_dev[dev] = p;
        else (void)hipGetLastError();
    }
    return scratch_dev[dev];
}

}  // namespace

struct rbl_ctx {
    rbl_config cfg;
    hipStream_t stream = nullptr;  // the caller's stream
    hipStream_t ls = nullptr;      // stream the helpers launch on (the caller's, or gs)
    hipStream_t gs = nullptr;      // internal stream for captured step blocks
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::vector<unsigned char> gsig;  // parameters the captured blocks were made with
    // device words of the MD loop: [0] step counter read by captured kernels;
    // [1] pending half-kick flag of a captured lifetime's first step; [2] step
    // of the last list build and [3] builds in the run (written by the build
    // kernels); [4] rebuild gate of the displacement criterion; [5] gate of
    // the filtered core rows
    uint64_t* d_step = nullptr;
    uint64_t h_marks[2] = {0, 0};
    int R = 1;
    int64_t n = 0, n_slots = 0, n_slices = 0;
    std::vector<int64_t> id_base, rep_n, slot_base;

    // geometry of the last build
    bool built = false;
    int built_mask = 0;
    bool shell_counts = false;  // shell_len valid (explicit shell list or fused build)
    bool fused_ok = true;       // false once a stencil outgrew the fused kernel's LDS lists
    int cap_list = 0;           // fused kernel: LDS shell-list room per centre particle
    bool stencil = false;       // batches drawn from the stencil cells (N_I in d_nI)
    int* d_nI = nullptr;        // stencil draw population size per slot
    // the paper's own grid (shell_source RBL_SHELL_PAPER): per-replica grids,
    // per-cell counts and starts, per-slot cell and rank, members by cell
    bool paper = false;
    bool pop_valid = false;     // d_nI holds N_I of the last build (a draw ran on it)
    int64_t n_pcells = 0;
    int64_t pcells_alloc = 0;
    PaperGrid* d_pgrid = nullptr;
    int* d_pcell_rep = nullptr;
    int* d_pcount = nullptr;
    int* d_pstart = nullptr;
    int* d_ptile = nullptr;
    int* d_pcell_of_slot = nullptr;
    int* d_prank = nullptr;
    int* d_pmember = nullptr;

    // Langevin thermostat (rbl_set_thermostat) and the continuous trajectory
    double gamma = 0.0;              // friction; 0: NVE
    std::vector<double> kT;          // bath temperature per replica
    double* d_osig = nullptr;        // per replica sqrt(kT (1 - c^2)) of the last run
    std::vector<double> h_osig;      // its host copy (source of the upload)
    int* d_img = nullptr;            // [3][n] box lengths the builds of rbl_step took off
    int* d_img_delta = nullptr;      // the same for the run in progress
    bool track_images = false;       // binning inside rbl_step counts wraps
    double* d_sq_part = nullptr;     // partial sums of k_sumsq
    int sq_nb = 0;
    double r_s = 0, r_c = 0;
    // particle types (n_types > 0): the type of each particle as a double in
    // caller order (the w word of the position records), the pair table of
    // the last build, and the extremes of sigma_ab
    bool typed = false;
    double* d_tcol = nullptr;
    TypeTable* d_tt = nullptr;
    std::vector<double> eps_sig;    // [n_types][n_types][2]
    double sig_min = 1.0, sig_max = 1.0;
    std::vector<DevReplica> h_rep;
    int64_t n_cells = 0, cells_alloc = 0;

    DevReplica* d_rep = nullptr;
    int* d_id_rep = nullptr;
    int* d_slice_rep = nullptr;
    int* d_cell_rep = nullptr;
    int* d_cell_count = nullptr;
    int* d_cell_start = nullptr;
    int* d_tile_sum = nullptr;
    int* d_cell_of_src = nullptr;
    int* d_rank_of_src = nullptr;
    int* d_src_of_slot = nullptr;
    int* d_perm[2] = {nullptr, nullptr};
    int cur = 0;
    int* d_slot_of_id = nullptr;
    double4* d_xs[2] = {nullptr, nullptr};
    int4* d_xq = nullptr;           // mixed precision: fixed-point copy of the current positions
    double guard_q = 0.0;           // bound on |r^2 fixed-point - r^2 FP64| of the mixed kernels
    double* d_vs[2] = {nullptr, nullptr};
    double* d_xb = nullptr;
    double* d_f = nullptr;
    // filtered core rows of runs with rebuilds on displacement (one lane per
    // particle): rows of cap[0] entries, their lengths, the positions at the
    // filtering; filt_run while a run uses them, with the thresholds below
    int* d_fcore = nullptr;
    int* d_fcore_len = nullptr;
    float* d_xf = nullptr;
    int64_t fcore_alloc = 0;
    bool filt_run = false;
    double filt2 = 0.0;
    float fhalf2 = 0.0f;

    int cap[3] = {0, 0, 0};
    int* d_list[3] = {nullptr, nullptr, nullptr};
    int* d_len[3] = {nullptr, nullptr, nullptr};

    int* d_batch = nullptr;
    size_t batch_alloc = 0;
    // what d_batch holds: batches of P partners for force evaluations
    // draw_step0 .. draw_step0 + draw_steps - 1 (0 steps: none)
    int draw_steps = 0, draw_P = 0;
    int64_t draw_step0 = 0;

    double* d_partial = nullptr;    // [5][n_slices * 4] wavefront partial sums
    int part_per = 1;               // partial entries per slice of the last force launch
    int lpp_rbl = 4, lpp_full = 4;  // lanes per particle of the force kernels
    bool persist[2] = {false, false};  // persistent force grid (RBL, full list)
    double persist_us[2][2] = {{0, 0}, {0, 0}};  // per launch: one block per tile, persistent
    int device = 0;                 // device the context was created on
    int n_cu = 256;                 // compute units of the device
    int64_t lds_per_cu = 160 * 1024;  // bytes of LDS per compute unit
    int64_t fused_static_lds = -1;    // static LDS of the fused build (queried once)
    bool tuned_rbl = false, tuned_full = false;
    // core_filter == 2: decided once per context by timing (filt_tuned);
    // filt_us: unfiltered step, filtered step, filtering launch
    bool filt_tuned = false, filt_auto_on = false;
    bool filt_last = false;  // the last run read filtered rows
    double filt_us[3] = {0, 0, 0};
    double tune_us[2][3] = {{0, 0, 0}, {0, 0, 0}};  // measured force time per LPP 1, 2, 4
    double* d_part2 = nullptr;
    int red_blocks = 1;
    double* d_rep_sum = nullptr;
    int* d_flags = nullptr;
    int h_flags[kNumFlags];

    // The last completed rbl_step / rbl_continue: the state it left in the
    // buffers above (positions, complete velocities, F at end_step, lists
    // built at build_step with the batches of their whole lifetime) is what
    // rbl_continue resumes.  Calls that load other positions or draws clear
    // `valid`.
    struct RunState {
        bool valid = false;
        int P = 0;
        uint64_t seed = 0;
        int64_t K = 1;
        double dt = 0.0;
        bool full = false;
        int64_t end_step = 0;
        int64_t build_step = 0;
        int attempts = 0;  // md_run passes the last call took (more than 1 after a capacity regrow)
        int64_t builds = 0;  // list builds in the last pass
    } run;
    double* d_ckpt = nullptr;  // [6][n] caller-order positions and velocities at a continued run's start

    bool profiling = false;
    // profiling: events the next launch_k hands to the dispatch itself
    hipEvent_t lt_a = nullptr, lt_b = nullptr;
    bool lt_used = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending[kKinds];
    std::vector<hipEvent_t> ev_pool;
    int64_t stat_launches[kKinds] = {0};
    double stat_ms[kKinds] = {0};

    int* cur_perm() { return d_perm[cur]; }
    // the w words of the position records: charges, or the particle types
    const double* wcol() const { return typed ? d_tcol : cfg.charges; }
    double4* cur_xs() { return d_xs[cur]; }
    double* cur_vs() { return d_vs[cur]; }
};

namespace {

hipEvent_t take_event(rbl_ctx* c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Queues `kernel` on the context's stream.  While profiling with events
// armed by timed(..., dispatch = true), the launch carries them itself
// (hipExtLaunchKernelGGL), so they hold the kernel's own start and end.
template <typename K, typename... A>
void launch_k(rbl_ctx* c, K kernel, unsigned grid, size_t shmem, A... args)
{
    if (c->lt_a && c->lt_b && !c->lt_used) {
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), (uint32_t)shmem, c->ls, c->lt_a, c->lt_b, 0u,
                              args...);
        c->lt_used = true;
    } else {
        kernel<<<grid, kBlock, shmem, c->ls>>>(args...);
    }
}

// Two dispatches timed as one (the start of the first to the end of the
// second), e.g. the two instances of a force step of which one returns at once.
template <typename K1, typename K2, typename... A>
void launch_k2(rbl_ctx* c, K1 k1, unsigned g1, size_t sh1, K2 k2, unsigned g2, size_t sh2, A... args)
{
    if (c->lt_a && c->lt_b && !c->lt_used) {
        hipExtLaunchKernelGGL(k1, dim3(g1), dim3(kBlock), (uint32_t)sh1, c->ls, c->lt_a, nullptr, 0u, args...);
        hipExtLaunchKernelGGL(k2, dim3(g2), dim3(kBlock), (uint32_t)sh2, c->ls, nullptr, c->lt_b, 0u, args...);
        c->lt_used = true;
    } else {
        k1<<<g1, kBlock, sh1, c->ls>>>(args...);
        k2<<<g2, kBlock, sh2, c->ls>>>(args...);
    }
}

// Runs `fn` (which queues one kernel) and, when profiling, times it: between
// two events recorded around it, or (dispatch = true, for an fn that
// launches through launch_k) with the events the launch itself records,
// which leave out the dispatch latency that stream events take in.
template <typename F>
rbl_status timed(rbl_ctx* c, int kind, F&& fn, bool dispatch = false)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->profiling) {
        a = take_event(c);
        b = take_event(c);
        if (a && b) {
            if (dispatch) {
                c->lt_a = a;
                c->lt_b = b;
                c->lt_used = false;
            } else {
                HIP_TRY(hipEventRecord(a, c->ls));
            }
        }
    }
    fn();
    c->lt_a = c->lt_b = nullptr;
    HIP_TRY(hipGetLastError());
    if (c->profiling && a && b) {
        if (dispatch && !c->lt_used) {
            // nothing went through launch_k: no time for this call
            c->ev_pool.push_back(a);
            c->ev_pool.push_back(b);
            return RBL_OK;
        }
        if (!dispatch) HIP_TRY(hipEventRecord(b, c->ls));
        c->ev_pending[kind].push_back({a, b});
    }
    return RBL_OK;
}

rbl_status resolve_events(rbl_ctx* c)
{
    for (int k = 0; k < kKinds; ++k) {
        for (auto& pr : c->ev_pending[k]) {
            HIP_TRY(hipEventSynchronize(pr.second));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
            c->stat_ms[k] += ms;
            c->stat_launches[k] += 1;
            c->ev_pool.push_back(pr.first);
            c->ev_pool.push_back(pr.second);
        }
        c->ev_pending[k].clear();
    }
    return RBL_OK;
}

rbl_status fill_i32(rbl_ctx* c, int* p, int64_t n, int v)
{
    if (n <= 0) return RBL_OK;
    k_fill_i32<<<grid_for(n), kBlock, 0, c->ls>>>(p, n, v);
    HIP_TRY(hipGetLastError());
    return RBL_OK;
}

rbl_status read_flags(rbl_ctx* c)
{
    HIP_TRY(hipMemcpyAsync(c->h_flags, c->d_flags, sizeof(int) * kNumFlags, hipMemcpyDeviceToHost,
                           c->ls));
    HIP_TRY(hipStreamSynchronize(c->ls));
    return RBL_OK;
}

rbl_status clear_flags(rbl_ctx* c) { return fill_i32(c, c->d_flags, kNumFlags, 0); }

// Clears only the list-capacity flags (overflow and longest rows), keeping
// the error flags raised by the binning of the same build.
rbl_status clear_list_flags(rbl_ctx* c) { return fill_i32(c, c->d_flags, kFlagMaxFull + 1, 0); }

// ---------------------------------------------------------------------------
// geometry

// The paper's own grid (Sec. II): cells of edge w = (r_s + skin)(1 + 1e-6)
// per replica, stencil half-width h = floor((r_c + skin)/w) + 1.  The x-runs
// of one stencil, 2 (2h+1)^2 at most, must fit the draw kernel's table.
rbl_status setup_paper_grid(rbl_ctx* c, double r_s, double r_c)
{
    const double skin = c->cfg.skin;
    const double w = (r_s + skin) * 1.000001;
    const int h = (int)std::floor((r_c + skin) / w) + 1;
    std::vector<PaperGrid> g(c->R);
    int64_t base = 0;
    for (int r = 0; r < c->R; ++r) {
        PaperGrid& G = g[r];
        std::memset(&G, 0, sizeof(G));
        int64_t runs = 1, cells = 1;
        for (int a = 0; a < 3; ++a) {
            const double L = c->h_rep[r].L[a];
            double nc = std::floor(L / w);
            if (nc < 1.0) nc = 1.0;
            if (nc > 4096) return fail(RBL_E_BOX, "box too large for the paper's cell grid");
            G.nc[a] = (int)nc;
            G.scale[a] = (double)G.nc[a] / L;
            const int64_t span = std::min<int64_t>(2 * h + 1, G.nc[a]);
            runs *= a == 0 ? (2 * h + 1 < G.nc[a] ? 2 : 1) : span;
            cells *= G.nc[a];
        }
        if (runs > kPaperRuns)
            return fail(RBL_E_ARG, "the paper's stencil (half-width " + std::to_string(h) +
                                       " cells) exceeds the draw kernel's run table");
        G.h = h;
        G.cell_base = base;
        base += cells;
    }
    if (base > (int64_t)1 << 30) return fail(RBL_E_BOX, "too many cells in the paper's grid");
    if ((base + kScanTile - 1) / kScanTile > 1024 * kScanPerThread)
        return fail(RBL_E_BOX, "the paper's grid exceeds the scan capacity");
    if (base > c->pcells_alloc) {
        dfree(c->d_pcell_rep);
        dfree(c->d_pcount);
        dfree(c->d_pstart);
        dfree(c->d_ptile);
        RBL_TRY(dalloc(&c->d_pcell_rep, base));
        RBL_TRY(dalloc(&c->d_pcount, base));
        RBL_TRY(dalloc(&c->d_pstart, base));
        RBL_TRY(dalloc(&c->d_ptile, (base + kScanTile - 1) / kScanTile + 1));
        c->pcells_alloc = base;
    }
    std::vector<int> cell_rep(base);
    for (int r = 0; r < c->R; ++r) {
        const int64_t nc = (int64_t)g[r].nc[0] * g[r].nc[1] * g[r].nc[2];
        std::fill(cell_rep.begin() + g[r].cell_base, cell_rep.begin() + g[r].cell_base + nc, r);
    }
    HIP_TRY(hipMemcpyAsync(c->d_pgrid, g.data(), sizeof(PaperGrid) * c->R, hipMemcpyHostToDevice, c->ls));
    HIP_TRY(hipMemcpyAsync(c->d_pcell_rep, cell_rep.data(), sizeof(int) * base, hipMemcpyHostToDevice, c->ls));
    HIP_TRY(hipStreamSynchronize(c->ls));
    c->n_pcells = base;
    return RBL_OK;
}

// The pair table of a typed context for radii r_s, r_c (in units of sigma)
// on the cell grid of `reps`: per pair (a, b) the LJ constants of eps_ab and
// sigma_ab, the radii r_s sigma_ab and r_c sigma_ab with the energy at the
// cut-off, the list thresholds with the skin, and per centre type the
// stencil half-width: the cell edges (times 1 + 1e-6) that its largest pair
// cut-off plus the skin spans, on the narrowest edge of any replica.
rbl_status setup_types(rbl_ctx* c, const std::vector<DevReplica>& reps, double r_s, double r_c)
{
    const int T = c->cfg.n_types;
    const double skin = c->cfg.skin;
    TypeTable t;
    std::memset(&t, 0, sizeof(t));
    t.n_types = T;
    double edge = std::numeric_limits<double>::infinity();
    for (const auto& d : reps)
        for (int ax = 0; ax < 3; ++ax) edge = std::min(edge, d.L[ax] / d.nc[ax]);
    for (int a = 0; a < T; ++a) {
        double smax = 0.0;
        for (int b = 0; b < T; ++b) {
            const double eps = c->eps_sig[(a * T + b) * 2 + 0];
            const double sig = c->eps_sig[(a * T + b) * 2 + 1];
            smax = std::max(smax, sig);
            TypePair& p = t.p[a * kMaxTypes + b];
            p.eps24 = 24.0 * eps;
            p.eps4 = 4.0 * eps;
            p.sig2 = sig * sig;
            const double rs = r_s * sig, rc = r_c * sig;
            p.rs2 = rs * rs;
            p.rc2 = rc * rc;
            p.uc = 0.0;
            if (c->cfg.shift) {
                const double r2i = 1.0 / p.rc2;
                const double s2 = p.sig2 * r2i;
                const double sr6 = s2 * s2 * s2;
                p.uc = p.eps4 * sr6 * (sr6 - 1.0);
            }
            const double ca = rs + skin;
            double cb = rs - skin;
            if (cb < 0.0) cb = 0.0;
            const double co = rc + skin;
            p.thr_core = ca * ca;
            p.thr_in = cb * cb;
            p.thr_out = co * co;
            const double cf = rs + 0.5 * skin;
            p.filt2 = cf * cf;
        }
        const double h = std::ceil((r_c * smax + skin) * 1.000001 / edge);
        if (!(h <= 15.0))
            return fail(RBL_E_BOX, "the stencil of particle type " + std::to_string(a) + " spans " +
                                       std::to_string((int)h) + " cells, more than 15: use fewer, wider cells "
                                       "(a smaller disparity of cut-offs)");
        t.h[a] = (int)h;
    }
    if (!c->d_tt) RBL_TRY(dalloc(&c->d_tt, 1));
    HIP_TRY(hipMemcpyAsync(c->d_tt, &t, sizeof(t), hipMemcpyHostToDevice, c->ls));
    HIP_TRY(hipStreamSynchronize(c->ls));
    return RBL_OK;
}

rbl_status setup_geometry(rbl_ctx* c, const double* box, double r_s, double r_c)
{
    const double skin = c->cfg.skin;
    // the largest pair cut-off decides the box check; the smallest sizes the
    // cells (one type: both are r_c)
    const double reach = r_c * c->sig_max + skin;
    const double r_cell = r_c * c->sig_min;
    std::vector<DevReplica> reps(c->R);
    int64_t cell_base = 0;
    for (int r = 0; r < c->R; ++r) {
        DevReplica& d = reps[r];
        std::memset(&d, 0, sizeof(d));
        // cells of edge >= (r_c + skin)/2 with a small margin, so that any pair
        // closer than r_c + skin lies within two cells along every axis (with
        // particle types: r_c of the smallest pair cut-off, and each type's
        // stencil reaches its own largest one)
        const double w = 0.5 * (r_cell + skin) * 1.000001;
        int64_t ncell = 1;
        for (int a = 0; a < 3; ++a) {
            const double L = box[3 * r + a];
            if (!(std::isfinite(L) && L > 2.0 * reach))
                return fail(RBL_E_BOX, "box edge " + std::to_string(L) + " of replica " +
                                           std::to_string(r) + " must exceed 2 (r_c + skin) = " +
                                           std::to_string(2.0 * reach) +
                                           (c->typed ? " (largest pair cut-off)" : ""));
            double nc = std::floor(L / w);
            if (nc < 1.0) nc = 1.0;
            if (nc > 1 << 20) return fail(RBL_E_BOX, "box too large for the cell grid");
            d.L[a] = L;
            d.inv[a] = 1.0 / L;
            d.nc[a] = (int)nc;
            d.cscale[a] = (double)d.nc[a] / L;
            ncell *= d.nc[a];
        }
        d.id_base = c->id_base[r];
        d.n = c->rep_n[r];
        d.slot_base = c->slot_base[r];
        d.cell_base = cell_base;
        cell_base += ncell;
    }
    if (cell_base > (int64_t)1 << 30) return fail(RBL_E_BOX, "too many cells");
    c->n_cells = cell_base;
    if (c->n_cells > c->cells_alloc) {
        dfree(c->d_cell_rep);
        dfree(c->d_cell_count);
        dfree(c->d_cell_start);
        dfree(c->d_tile_sum);
        RBL_TRY(dalloc(&c->d_cell_rep, c->n_cells));
        RBL_TRY(dalloc(&c->d_cell_count, c->n_cells));
        RBL_TRY(dalloc(&c->d_cell_start, c->n_cells + 1));
        RBL_TRY(dalloc(&c->d_tile_sum, (c->n_cells + kScanTile - 1) / kScanTile + 1));
        c->cells_alloc = c->n_cells;
    }
    if ((c->n_cells + kScanTile - 1) / kScanTile > 1024 * kScanPerThread)
        return fail(RBL_E_BOX, "cell grid exceeds the scan capacity");
    bool same = c->h_rep.size() == reps.size();
    for (size_t r = 0; same && r < reps.size(); ++r)
        same = std::memcmp(&reps[r], &c->h_rep[r], sizeof(DevReplica)) == 0;
    if (!same) {
        std::vector<int> cell_rep(c->n_cells);
        for (int r = 0; r < c->R; ++r) {
            const int64_t nc = (int64_t)reps[r].nc[0] * reps[r].nc[1] * reps[r].nc[2];
            std::fill(cell_rep.begin() + reps[r].cell_base, cell_rep.begin() + reps[r].cell_base + nc, r);
        }
        HIP_TRY(hipMemcpyAsync(c->d_rep, reps.data(), sizeof(DevReplica) * c->R, hipMemcpyHostToDevice,
                               c->ls));
        HIP_TRY(hipMemcpyAsync(c->d_cell_rep, cell_rep.data(), sizeof(int) * c->n_cells,
                               hipMemcpyHostToDevice, c->ls));
        HIP_TRY(hipStreamSynchronize(c->ls));
        c->h_rep = reps;
    }
    c->r_s = r_s;
    c->r_c = r_c;
    if (c->paper) RBL_TRY(setup_paper_grid(c, r_s, r_c));
    if (c->typed) RBL_TRY(setup_types(c, reps, r_s, r_c));
    // Mixed-precision forces classify from fixed-point copies of the
    // positions (x / L mod 1 in units of 2^-32).  With u = 2^-53 and
    // coordinates below X = 1024 (L_max + r_c) in magnitude, a stored word
    // is off by at most half a unit plus u X twice (1/L and x/L rounded), so
    // the scaled difference of two is off from the true displacement by
    // L 2^-32 + u (4 X + r) per component, and the FP64 path's min-image
    // difference by u (4 X + 3 L_max + r); with e the sum of the two, the
    // two r^2 (three roundings each) differ by at most
    // 2 sqrt(3) r e + 3 e^2 + 8 u r^2, r <= r_c + 1 near a bound; the guard
    // doubles that.
    {
        double lmax = 0.0;
        for (const auto& d : reps)
            for (int a = 0; a < 3; ++a) lmax = std::max(lmax, d.L[a]);
        const double u = std::ldexp(1.0, -53);
        const double X = 1024.0 * (lmax + r_c * c->sig_max);
        const double r = r_c * c->sig_max + 1.0;
        const double e = std::ldexp(lmax, -32) + u * (8.0 * X + 3.0 * lmax + 2.0 * r);
        c->guard_q = 2.0 * (2.0 * std::sqrt(3.0) * r * e + 3.0 * e * e + 8.0 * u * r * r);
    }
    return RBL_OK;
}

struct Thresholds {
    double core, shell_in, out, rs2, rc2, uc, uce;
};

Thresholds thresholds(const rbl_ctx* c)
{
    Thresholds t;
    const double skin = c->cfg.skin;
    const double a = c->r_s + skin;
    double b = c->r_s - skin;
    if (b < 0.0) b = 0.0;
    const double o = c->r_c + skin;
    t.core = a * a;
    t.shell_in = b * b;
    t.out = o * o;
    t.rs2 = c->r_s * c->r_s;
    t.rc2 = c->r_c * c->r_c;
    t.uc = 0.0;
    t.uce = 0.0;
    if (c->cfg.shift) {
        const double r2i = 1.0 / t.rc2;
        const double sr6 = r2i * r2i * r2i;
        t.uc = 4.0 * sr6 * (sr6 - 1.0);
        // erfc(alpha r)/r at the cut-off, per unit charge product
        if (c->cfg.pair == RBL_PAIR_LJ_ERFC) t.uce = std::erfc(c->cfg.alpha * c->r_c) / c->r_c;
    }
    return t;
}

// ---------------------------------------------------------------------------
// binning: histogram, scan, scatter, per-cell ID sort, gather into new buffers

// With `gate` (a rebuild decided on the device) every kernel returns at once
// while *gate is 0, and the new state lands in the current buffer set, which
// captured kernels address: the counting pass saves the old state into the
// other set, from which the scatter and the gather read.  The skin monitor is
// then off: the rebuild happens because the displacement reached skin/2.
template <int SRC>
rbl_status bin_particles(rbl_ctx* c, const double* pos, const double* vel, bool with_vel,
                         const uint64_t* gate = nullptr)
{
    const int nxt = 1 - c->cur;
    BinArgs b;
    b.rep = c->d_rep;
    b.id_rep = c->d_id_rep;
    b.slice_rep = c->d_slice_rep;
    b.pos = pos;
    b.xs = c->cur_xs();
    b.perm_old = c->cur_perm();
    b.xb = c->d_xb;
    {
        const double hs = 0.5 * c->cfg.skin;
        b.half_skin2 = gate ? std::numeric_limits<double>::infinity() : hs * hs;
    }
    b.gate = gate;
    b.xs_save = nullptr;
    b.vs_src = nullptr;
    b.vs_save = nullptr;
    b.perm_save = nullptr;
    b.n = c->n;
    b.n_src = SRC == kSrcCaller ? c->n : c->n_slots;
    b.cell_of_src = c->d_cell_of_src;
    b.rank_of_src = c->d_rank_of_src;
    b.cell_count = c->d_cell_count;
    b.flags = c->d_flags;
    const int64_t ntiles = (c->n_cells + kScanTile - 1) / kScanTile;
    RBL_TRY(timed(c, kKBin, [&] {
        k_clear_counts<<<grid_for(c->n_cells), kBlock, 0, c->ls>>>(c->d_cell_count, c->n_cells, gate);
    }));
    const bool in_place = gate != nullptr && SRC == kSrcSorted;
    const int dst = in_place ? c->cur : nxt;
    {
        BinArgs bc = b;
        if (in_place) {
            bc.xs_save = c->d_xs[nxt];
            bc.vs_src = c->d_vs[c->cur];
            bc.vs_save = c->d_vs[nxt];
            bc.perm_save = c->d_perm[nxt];
        }
        RBL_TRY(timed(c, kKBin, [&] { k_bin_count<SRC><<<grid_for(b.n_src), kBlock, 0, c->ls>>>(bc); }));
    }
    if (in_place) b.perm_old = c->d_perm[nxt];
    RBL_TRY(timed(c, kKBin, [&] {
        k_scan_tiles<<<(unsigned)ntiles, kScanBlock, 0, c->ls>>>(c->d_cell_count, c->n_cells,
                                                                     c->d_tile_sum, gate);
    }));
    RBL_TRY(timed(c, kKBin, [&] {
        k_scan_tile_sums<<<1, 1024, 0, c->ls>>>(c->d_tile_sum, (int)ntiles, gate);
    }));
    RBL_TRY(timed(c, kKBin, [&] {
        k_scan_final<<<(unsigned)ntiles, kScanBlock, 0, c->ls>>>(
            c->d_cell_count, c->n_cells, c->d_tile_sum, c->d_cell_rep, c->d_rep, c->d_cell_start, gate);
    }));
    RBL_TRY(timed(c, kKBin, [&] {
        k_bin_scatter<SRC><<<grid_for(b.n_src), kBlock, 0, c->ls>>>(
            b, c->d_cell_start, c->d_perm[dst], c->d_src_of_slot, c->n_slots);
    }));
    RBL_TRY(timed(c, kKBin, [&] {
        k_cell_sort<<<grid_for(c->n_cells), kBlock, 0, c->ls>>>(
            c->d_cell_start, c->d_cell_count, c->n_cells, c->n_slots, c->d_perm[dst],
            c->d_src_of_slot, c->d_flags, gate);
    }));
    GatherArgs g;
    g.rep = c->d_rep;
    g.slice_rep = c->d_slice_rep;
    g.perm = c->d_perm[dst];
    g.src_of_slot = c->d_src_of_slot;
    g.pos = pos;
    g.vel = vel;
    g.charges = c->wcol();
    g.xs_old = in_place ? c->d_xs[nxt] : c->cur_xs();
    g.vs_old = in_place ? c->d_vs[nxt] : c->cur_vs();
    g.n = c->n;
    g.n_src = b.n_src;
    g.n_slots = c->n_slots;
    g.flags = c->d_flags;
    g.xs = c->d_xs[dst];
    g.vs = c->d_vs[dst];
    g.xb = c->d_xb;
    g.slot_of_id = c->d_slot_of_id;
    g.img_delta = c->track_images ? c->d_img_delta : nullptr;
    g.gate = gate;
    g.xq = c->d_xq;
    RBL_TRY(timed(c, kKBin, [&] {
        if (with_vel)
            k_gather<SRC, true><<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(g);
        else
            k_gather<SRC, false><<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(g);
    }));
    c->cur = dst;
    return RBL_OK;
}

// ---------------------------------------------------------------------------
// list build

BuildArgs build_args(rbl_ctx* c)
{
    const Thresholds t = thresholds(c);
    BuildArgs a;
    a.rep = c->d_rep;
    a.cell_rep = c->d_cell_rep;
    a.cell_start = c->d_cell_start;
    a.cell_count = c->d_cell_count;
    a.xs = c->cur_xs();
    a.n_cells = c->n_cells;
    a.n_slots = c->n_slots;
    a.thr_core = t.core;
    a.thr_shell_in = t.shell_in;
    a.thr_out = t.out;
    a.cap_core = c->cap[0];
    a.cap_shell = c->cap[1];
    a.cap_full = c->cap[2];
    a.core = c->d_list[0];
    a.shell = c->d_list[1];
    a.full = c->d_list[2];
    a.core_len = c->d_len[0];
    a.shell_len = c->d_len[1];
    a.full_len = c->d_len[2];
    a.flags = c->d_flags;
    a.gate = nullptr;
    a.types = c->typed ? c->d_tt : nullptr;
    a.mark = nullptr;
    a.mark_step = 0;
    a.mark_step_dev = nullptr;
    return a;
}

// Build arguments of a list build of the MD loop: gated by `gate`, and
// recording its step (*step_dev + step, or step) and count on the device.
BuildArgs loop_build_args(rbl_ctx* c, uint64_t step, const uint64_t* step_dev, const uint64_t* gate)
{
    BuildArgs a = build_args(c);
    a.gate = gate;
    a.mark = c->d_step + 2;
    a.mark_step = step;
    a.mark_step_dev = step_dev;
    return a;
}

template <bool COUNT_ONLY>
void launch_build(rbl_ctx* c, const BuildArgs& a, int mask)
{
    const unsigned g = grid_for(c->n_cells, 4);
    const bool wc = mask & RBL_LIST_CORE, ws = mask & RBL_LIST_SHELL, wf = mask & RBL_LIST_FULL;
    if (c->typed) {
#define RBL_B(C, S, F) k_build_typed<COUNT_ONLY, C, S, F><<<g, kBlock, 0, c->ls>>>(a)
        if (wc && ws && wf) RBL_B(true, true, true);
        else if (wc && ws) RBL_B(true, true, false);
        else if (wc && wf) RBL_B(true, false, true);
        else if (ws && wf) RBL_B(false, true, true);
        else if (wc) RBL_B(true, false, false);
        else if (ws) RBL_B(false, true, false);
        else RBL_B(false, false, true);
#undef RBL_B
        return;
    }
#define RBL_B(C, S, F) k_build<COUNT_ONLY, C, S, F><<<g, kBlock, 0, c->ls>>>(a)
    if (wc && ws && wf) RBL_B(true, true, true);
    else if (wc && ws) RBL_B(true, true, false);
    else if (wc && wf) RBL_B(true, false, true);
    else if (ws && wf) RBL_B(false, true, true);
    else if (wc) RBL_B(true, false, false);
    else if (ws) RBL_B(false, true, false);
    else RBL_B(false, false, true);
#undef RBL_B
}

// Row capacity of list q for rows of up to `need` entries.  The first
// sizing applies capacity_factor (values below 1 size rows short on
// purpose); after an overflow rows grow to at least 1.5x the longest row
// seen and by at least 16 entries, so a run regrows a bounded number of
// times.
rbl_status ensure_list_storage(rbl_ctx* c, int q, int need, bool regrow = false)
{
    int cap;
    if (regrow) {
        cap = std::max((int)std::ceil(need * std::max(1.5, c->cfg.capacity_factor)) + 8, c->cap[q] + 16);
    } else {
        cap = (int)std::ceil(need * c->cfg.capacity_factor) + 8;
    }
    cap = (cap + 3) & ~3;
    if (cap <= c->cap[q] && c->d_list[q]) return RBL_OK;
    dfree(c->d_list[q]);
    c->cap[q] = 0;
    RBL_TRY(dalloc(&c->d_list[q], (size_t)c->n_slots * cap));
    c->cap[q] = cap;
    return RBL_OK;
}

// Builds the lists in `mask` at the current sorted positions.  The first
// build of a list (or one that overflowed) runs a counting pass, sizes the
// rows to the longest one times capacity_factor, and fills.
rbl_status build_lists(rbl_ctx* c, int mask)
{
    for (int q = 0; q < 3; ++q)
        if ((mask >> q) & 1)
            if (!c->d_len[q]) RBL_TRY(dalloc(&c->d_len[q], c->n_slots));
    bool need_count = false;
    for (int q = 0; q < 3; ++q)
        if (((mask >> q) & 1) && c->cap[q] == 0) need_count = true;
    for (int attempt = 0; attempt < 3; ++attempt) {
        RBL_TRY(clear_list_flags(c));
        if (need_count) {
            BuildArgs a = build_args(c);
            RBL_TRY(timed(c, kKBuild, [&] { launch_build<true>(c, a, mask); }));
            RBL_TRY(read_flags(c));
            if (c->h_flags[kFlagBadSlot]) return fail(RBL_E_HIP, "inconsistent cell binning");
            for (int q = 0; q < 3; ++q)
                if ((mask >> q) & 1) RBL_TRY(ensure_list_storage(c, q, c->h_flags[kFlagMaxCore + q]));
            RBL_TRY(clear_list_flags(c));
        }
        BuildArgs a = build_args(c);
        RBL_TRY(timed(c, kKBuild, [&] { launch_build<false>(c, a, mask); }));
        RBL_TRY(read_flags(c));
        if (c->h_flags[kFlagBadSlot]) return fail(RBL_E_HIP, "inconsistent cell binning");
        if (c->h_flags[kFlagNonfinite]) {
            c->built = false;
            return fail(RBL_E_NONFINITE, "non-finite particle position at list build");
        }
        if (!c->h_flags[kFlagOverflow]) {
            c->built_mask = mask;
            c->shell_counts = (mask & RBL_LIST_SHELL) != 0;
            return RBL_OK;
        }
        for (int q = 0; q < 3; ++q)
            if ((mask >> q) & 1) RBL_TRY(ensure_list_storage(c, q, c->h_flags[kFlagMaxCore + q], true));
        need_count = false;
    }
    return fail(RBL_E_CAPACITY, "neighbour rows kept overflowing their capacity");
}


// Core rows + shell counts + the batches of force evaluations step0 ..
// step0+K-1 in one pass (no shell rows in HBM).
rbl_status ensure_batch(rbl_ctx* c, int K, int P);

PaperArgs paper_args(rbl_ctx* c, const uint64_t* gate)
{
    PaperArgs a;
    a.grid = c->d_pgrid;
    a.rep = c->d_rep;
    a.slice_rep = c->d_slice_rep;
    a.cell_rep = c->d_pcell_rep;
    a.xs = c->cur_xs();
    a.perm = c->cur_perm();
    a.n_slots = c->n_slots;
    a.n_cells = c->n_pcells;
    a.cell_of_slot = c->d_pcell_of_slot;
    a.rank = c->d_prank;
    a.count = c->d_pcount;
    a.start = c->d_pstart;
    a.member = c->d_pmember;
    a.flags = c->d_flags;
    a.gate = gate;
    return a;
}

// Bins the current (build) positions into the paper's grid: counts, an
// exclusive scan into member positions, scatter, and the in-cell order by
// ID.  Gated like the rest of a build.
void paper_bin(rbl_ctx* c, const uint64_t* gate)
{
    const PaperArgs a = paper_args(c, gate);
    const int64_t tiles = (c->n_pcells + kScanTile - 1) / kScanTile;
    k_clear_counts<<<grid_for(c->n_pcells), kBlock, 0, c->ls>>>(c->d_pcount, c->n_pcells, gate);
    k_paper_count<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(a);
    k_scan_tiles<<<(unsigned)tiles, kScanBlock, 0, c->ls>>>(c->d_pcount, c->n_pcells, c->d_ptile, gate);
    k_scan_tile_sums<<<1, 1024, 0, c->ls>>>(c->d_ptile, (int)tiles, gate);
    k_scan_final<<<(unsigned)tiles, kScanBlock, 0, c->ls>>>(c->d_pcount, c->n_pcells, c->d_ptile, nullptr,
                                                          nullptr, c->d_pstart, gate);
    k_paper_scatter<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(a);
    k_paper_sort<<<grid_for(c->n_pcells), kBlock, 0, c->ls>>>(a);
}

// The batches of K force evaluations from step0 (or *step_dev + step0),
// drawn from the paper-grid stencils of the last build, and N_I per slot.
void paper_draw(rbl_ctx* c, int P, uint64_t seed, uint64_t step0, int K, const uint64_t* step_dev,
                const uint64_t* gate)
{
    PaperDrawArgs d;
    d.p = paper_args(c, gate);
    d.batch = c->d_batch;
    d.n_pop = c->d_nI;
    d.seed = seed;
    d.step0 = step0;
    d.step_dev = step_dev;
    d.K = K;
    d.P = P;
    const unsigned g = grid_for(c->n_pcells, 4);
#define RBL_PD(PM) k_paper_draw<PM><<<g, kBlock, 0, c->ls>>>(d)
    if (P <= 8) RBL_PD(8);
    else if (P <= 12) RBL_PD(12);
    else if (P <= 16) RBL_PD(16);
    else if (P <= 24) RBL_PD(24);
    else if (P <= 32) RBL_PD(32);
    else if (P <= 64) RBL_PD(64);
    else RBL_PD(128);
#undef RBL_PD
}

// Queues the fused build (core rows, shell counts, batches of K force
// evaluations from step0, or from *step_dev + step0 when step_dev is set).
rbl_status launch_fused(rbl_ctx* c, int P, uint64_t seed, uint64_t step0, int K,
                        const uint64_t* step_dev, bool draw_only = false, bool loop = false,
                        const uint64_t* gate = nullptr)
{
    FusedArgs fa;
    fa.b = loop ? loop_build_args(c, step0, step_dev, gate) : build_args(c);
    fa.core_reach = c->r_s + c->cfg.skin;
    fa.draw_only = draw_only ? 1 : 0;
    if (c->stencil) fa.b.shell_len = c->d_nI;
    fa.perm = c->cur_perm();
    fa.batch = c->d_batch;
    fa.seed = seed;
    fa.step0 = step0;
    fa.step_dev = step_dev;
    fa.K = K;
    fa.P = P;
    fa.cap_list = c->cap_list;
    // LDS list budget per wavefront: the largest with which the blocks the
    // kernel's registers allow (kFusedWavesPerEu for P <= 32) still fit in
    // a CU's LDS, but at least two list rooms.  Occupancy outweighs group
    // size: a cell with more particles than fit one group walks its stencil
    // once per group, and that costs less than fewer resident blocks (at
    // N = 1e6: 2112 entries, groups of 8, 7 blocks per CU).
    if (c->fused_static_lds < 0) {
        hipFuncAttributes fattr{};
        c->fused_static_lds = hipFuncGetAttributes(&fattr, reinterpret_cast<const void*>(k_build_draw<12, false>))
                                      == hipSuccess
                                  ? (int64_t)fattr.sharedSizeBytes
                                  : 8192;
    }
    const int64_t blocks_per_cu = P <= 32 ? kFusedWavesPerEu : 2;
    const int64_t per_wave = (c->lds_per_cu / blocks_per_cu - c->fused_static_lds) / (4 * (int64_t)sizeof(unsigned short));
    const int64_t fit = std::max<int64_t>(64, (per_wave - 64) / 64 * 64);
    fa.list_budget = (int)std::min<int64_t>(kListBudgetMax,
                                            std::max<int64_t>(fit, ((int64_t)2 * c->cap_list + 63) / 64 * 64));
    const size_t lds = c->stencil ? 0 : (size_t)4 * (fa.list_budget + 64) * sizeof(unsigned short);
    const unsigned g = grid_for(c->n_cells, 4);
    if (c->paper) {
        // core rows on the binning grid (no draws there), then the paper
        // grid's binning at a build, and the draws from its stencils
        if (!draw_only) {
            FusedArgs fc = fa;
            fc.K = 0;
            RBL_TRY(timed(c, kKBuild, [&] { launch_k(c, k_build_draw<8, true>, g, 0, fc); }, true));
            RBL_TRY(timed(c, kKBuild, [&] { paper_bin(c, fa.b.gate); }));
        }
        c->pop_valid = true;
        return timed(c, kKBuild, [&] { paper_draw(c, P, seed, step0, K, step_dev, fa.b.gate); });
    }
    if (c->stencil) c->pop_valid = true;
    return timed(c, kKBuild, [&] {
#define RBL_BD(PM)                                                    \
    do {                                                              \
        if (c->stencil) launch_k(c, k_build_draw<PM, true>, g, 0, fa); \
        else launch_k(c, k_build_draw<PM, false>, g, lds, fa);         \
    } while (0)
        if (P <= 8) RBL_BD(8);
        else if (P <= 12) RBL_BD(12);
        else if (P <= 16) RBL_BD(16);
        else if (P <= 24) RBL_BD(24);
        else if (P <= 32) RBL_BD(32);
        else if (P <= 64) RBL_BD(64);
        else RBL_BD(128);
#undef RBL_BD
    }, true);
}

// LDS shell-list room per centre particle of the fused kernel: the longest
// shell row seen, with the context's headroom but at most kListRoomFactor
// (at least 1.5x after an overflow), rounded up to 8 entries.  The room
// sets how many particles share a wavefront's list budget, so a tighter
// first room means fewer cells split into two groups; a row that outgrows
// it is caught and the run repeated with a larger room.  (At N = 1e6 the
// longest shell row grows from 199 to 210 over 2000 steps as the lattice
// start melts, against a first room of 232.)
constexpr double kListRoomFactor = 1.1;

void grow_cap_list(rbl_ctx* c, int need, bool regrow)
{
    const double f = regrow ? std::max(1.5, c->cfg.capacity_factor)
                            : std::min(c->cfg.capacity_factor, kListRoomFactor);
    int64_t cap = (int64_t)std::ceil(std::max(need, 1) * f) + 8;
    if (regrow) cap = std::max<int64_t>(cap, (int64_t)c->cap_list + 16);
    cap = (cap + 7) / 8 * 8;
    c->cap_list = (int)std::min<int64_t>(cap, 1 << 20);
}

rbl_status prepare_lists(rbl_ctx* c, int mask);

// Sizes the core rows if needed (a counting pass and one synchronisation,
// the first time only) and makes sure the shell-count and batch buffers
// exist for `K` steps of batch size P.
rbl_status prepare_fused(rbl_ctx* c, int P, int K)
{
    for (int q = 0; q < 2; ++q)
        if (!c->d_len[q]) RBL_TRY(dalloc(&c->d_len[q], c->n_slots));
    RBL_TRY(ensure_batch(c, K, P));
    if (c->stencil) {
        // no shell list: the core rows alone are sized
        if (!c->d_nI) RBL_TRY(dalloc(&c->d_nI, c->n_slots));
        return prepare_lists(c, RBL_LIST_CORE);
    }
    if (c->cap[0] == 0 || c->cap_list == 0) {
        RBL_TRY(clear_list_flags(c));
        BuildArgs a = build_args(c);
        RBL_TRY(timed(c, kKBuild, [&] { launch_build<true>(c, a, RBL_LIST_CORE | RBL_LIST_SHELL); }));
        RBL_TRY(read_flags(c));
        if (c->h_flags[kFlagBadSlot]) return fail(RBL_E_HIP, "inconsistent cell binning");
        if (c->cap[0] == 0) RBL_TRY(ensure_list_storage(c, 0, c->h_flags[kFlagMaxCore]));
        if (c->cap_list == 0) grow_cap_list(c, c->h_flags[kFlagMaxShell], false);
    }
    return RBL_OK;
}

// Sizes the rows of `mask` if needed (counting pass + one synchronisation).
rbl_status prepare_lists(rbl_ctx* c, int mask)
{
    for (int q = 0; q < 3; ++q)
        if (((mask >> q) & 1) && !c->d_len[q]) RBL_TRY(dalloc(&c->d_len[q], c->n_slots));
    bool need = false;
    for (int q = 0; q < 3; ++q)
        if (((mask >> q) & 1) && c->cap[q] == 0) need = true;
    if (!need) return RBL_OK;
    RBL_TRY(clear_list_flags(c));
    BuildArgs a = build_args(c);
    RBL_TRY(timed(c, kKBuild, [&] { launch_build<true>(c, a, mask); }));
    RBL_TRY(read_flags(c));
    if (c->h_flags[kFlagBadSlot]) return fail(RBL_E_HIP, "inconsistent cell binning");
    for (int q = 0; q < 3; ++q)
        if ((mask >> q) & 1) RBL_TRY(ensure_list_storage(c, q, c->h_flags[kFlagMaxCore + q]));
    return RBL_OK;
}

// ---------------------------------------------------------------------------
// forces

ForceArgs force_args(rbl_ctx* c, int P, uint64_t seed, uint64_t step, bool full)
{
    const Thresholds t = thresholds(c);
    ForceArgs a;
    a.rep = c->d_rep;
    a.slice_rep = c->d_slice_rep;
    a.perm = c->cur_perm();
    a.xs = c->cur_xs();
    a.core = full ? c->d_list[2] : c->d_list[0];
    a.core_len = full ? c->d_len[2] : c->d_len[0];
    a.cap_core = full ? c->cap[2] : c->cap[0];
    a.shell = c->d_list[1];
    a.shell_len = c->stencil ? c->d_nI : c->d_len[1];
    a.cap_shell = c->cap[1];
    a.batch = nullptr;
    a.n_slots = c->n_slots;
    a.n_slices = c->n_slices;
    a.rs2 = t.rs2;
    a.rc2 = t.rc2;
    a.uc = t.uc;
    a.uce = t.uce;
    a.alpha = c->cfg.alpha;
    a.seed = seed;
    a.step = step;
    a.step_dev = nullptr;
    a.P = P;
    a.f = c->d_f;
    a.partial = c->d_partial;
    a.bstep = nullptr;
    a.gate_clear = nullptr;
    a.xq = c->d_xq;
    a.guard = c->guard_q;
    a.types = c->typed ? c->d_tt : nullptr;
    a.fgate = nullptr;
    a.fcore = nullptr;
    a.fcore_len = nullptr;
    a.xf = nullptr;
    a.filt2 = 0.0;
    return a;
}

// Blocks of a force launch: one per work tile, or (persistent) as many as
// the device keeps resident, a multiple of 8 so that every block stays on
// the tiles the XCD map gives its XCD.
template <typename Kernel>
unsigned force_grid(rbl_ctx* c, Kernel kernel, int64_t vblocks, bool persistent)
{
    if (!persistent) return (unsigned)vblocks;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    int64_t g = (int64_t)c->n_cu * per_cu / 8 * 8;
    if (g < 8) g = 8;
    return (unsigned)std::min<int64_t>(g, vblocks);
}

template <int PREC, int MODE, bool EN, int PAIR>
void launch_force_p(rbl_ctx* c, const ForceArgs& a0)
{
    ForceArgs a = a0;
    const bool pers = c->persist[MODE == kShellNone ? 1 : 0];
    // filtering instance: LDS column of cap_core entries per lane
    const size_t keep_lds = (size_t)kBlock * std::min(a.cap_core, kKeepLds) * sizeof(int);
    if constexpr (MODE == kShellInline) {
        a.vblocks = grid_for(c->n_slots);
        c->part_per = 1;
        if (a.P <= 16) {
            auto k = k_forces<PREC, MODE, EN, PAIR, 16>;
            auto kf = k_forces<PREC, MODE, EN, PAIR, 16, true>;
            if (a.fgate)
                launch_k2(c, kf, force_grid(c, kf, a.vblocks, pers), keep_lds, k,
                          force_grid(c, k, a.vblocks, pers), 0, a);
            else launch_k(c, k, force_grid(c, k, a.vblocks, pers), 0, a);
        } else {
            auto k = k_forces<PREC, MODE, EN, PAIR, 32>;
            auto kf = k_forces<PREC, MODE, EN, PAIR, 32, true>;
            if (a.fgate)
                launch_k2(c, kf, force_grid(c, kf, a.vblocks, pers), keep_lds, k,
                          force_grid(c, k, a.vblocks, pers), 0, a);
            else launch_k(c, k, force_grid(c, k, a.vblocks, pers), 0, a);
        }
    } else {
        const int lpp = MODE == kShellNone ? c->lpp_full : c->lpp_rbl;
        c->part_per = lpp;
        if (lpp == 4 || lpp == 2) {
            a.vblocks = grid_for(c->n_slots * lpp);
            auto k = lpp == 4 ? k_forces_lpp<PREC, MODE, EN, PAIR, 4> : k_forces_lpp<PREC, MODE, EN, PAIR, 2>;
            launch_k(c, k, force_grid(c, k, a.vblocks, pers), 0, a);
        } else {
            a.vblocks = grid_for(c->n_slots);
            auto k = k_forces<PREC, MODE, EN, PAIR, 1>;
            if constexpr (MODE != kShellNone) {
                if (a.fgate) {
                    auto kf = k_forces<PREC, MODE, EN, PAIR, 1, true>;
                    launch_k2(c, kf, force_grid(c, kf, a.vblocks, pers), keep_lds, k,
                              force_grid(c, k, a.vblocks, pers), 0, a);
                    return;
                }
            }
            launch_k(c, k, force_grid(c, k, a.vblocks, pers), 0, a);
        }
    }
}

template <int MODE>
void launch_force(rbl_ctx* c, const ForceArgs& a, bool energy)
{
    const bool mixed = c->cfg.precision == RBL_PREC_MIXED;
    const int pair = c->typed ? kPairTyped : (c->cfg.pair == RBL_PAIR_LJ_ERFC ? kPairErfc : kPairLJ);
#define RBL_F(P, E, X) launch_force_p<P, MODE, E, X>(c, a)
#define RBL_FP(X)                                       \
    do {                                                \
        if (!mixed && !energy) RBL_F(kFP64, false, X);  \
        else if (!mixed) RBL_F(kFP64, true, X);         \
        else if (!energy) RBL_F(kMixed, false, X);      \
        else RBL_F(kMixed, true, X);                    \
    } while (0)
    if (pair == kPairLJ) RBL_FP(kPairLJ);
    else if (pair == kPairErfc) RBL_FP(kPairErfc);
    else RBL_FP(kPairTyped);
#undef RBL_FP
#undef RBL_F
}

rbl_status ensure_batch(rbl_ctx* c, int K, int P)
{
    const size_t need = (size_t)K * P * c->n_slots;
    if (need <= c->batch_alloc) return RBL_OK;
    dfree(c->d_batch);
    c->batch_alloc = 0;
    RBL_TRY(dalloc(&c->d_batch, need));
    c->batch_alloc = need;
    return RBL_OK;
}

rbl_status predraw(rbl_ctx* c, int P, uint64_t seed, uint64_t step0, int K)
{
    RBL_TRY(ensure_batch(c, K, P));
    DrawArgs d;
    d.rep = c->d_rep;
    d.slice_rep = c->d_slice_rep;
    d.perm = c->cur_perm();
    d.shell = c->d_list[1];
    d.shell_len = c->d_len[1];
    d.cap_shell = c->cap[1];
    d.n_slots = c->n_slots;
    d.n_slices = c->n_slices;
    d.seed = seed;
    d.step0 = step0;
    d.K = K;
    d.P = P;
    d.batch = c->d_batch;
    const unsigned g = grid_for(c->n_slots);
    return timed(c, kKPredraw, [&] {
        if (P <= 16) k_predraw<16><<<g, kBlock, 0, c->ls>>>(d);
        else if (P <= 32) k_predraw<32><<<g, kBlock, 0, c->ls>>>(d);
        else if (P <= 64) k_predraw<64><<<g, kBlock, 0, c->ls>>>(d);
        else k_predraw<128><<<g, kBlock, 0, c->ls>>>(d);
    });
}

rbl_status reduce(rbl_ctx* c, bool gated = false)
{
    uint64_t* fclear = gated && c->filt_run ? c->d_step + 5 : nullptr;
    return timed(c, kKReduce, [&] {
        k_reduce<<<dim3(c->red_blocks, c->R), kBlock, 0, c->ls>>>(
            c->d_rep, c->d_partial, c->n_slices, c->part_per, c->red_blocks, c->d_part2, fclear);
        k_reduce_final<<<c->R, kBlock, 0, c->ls>>>(c->d_rep, c->part_per, c->red_blocks, c->d_part2,
                                                   c->d_rep_sum);
    });
}

// RBL force at the current sorted positions (raw; per-replica sums reduced).
// batch_rel >= 0 selects pre-drawn batches of that relative step.
// gated: a step of a run with rebuilds on displacement (the force resets the
// gate; pre-drawn batches are addressed through the device's build step).
rbl_status rbl_force_sorted(rbl_ctx* c, int P, uint64_t seed, uint64_t step, int batch_rel,
                            bool energy, const uint64_t* step_dev = nullptr, bool gated = false)
{
    ForceArgs a = force_args(c, P, seed, step, false);
    a.step_dev = step_dev;
    if (gated) a.gate_clear = c->d_step + 4;
    if (gated && c->filt_run) {
        a.fgate = c->d_step + 5;
        a.fcore = c->d_fcore;
        a.fcore_len = c->d_fcore_len;
        a.xf = c->d_xf;
        a.filt2 = c->filt2;
    }
    if (batch_rel >= 0 && gated) {
        a.batch = c->d_batch;
        a.bstep = c->d_step + 2;
        RBL_TRY(timed(c, kKForceRbl, [&] { launch_force<kShellPredraw>(c, a, energy); }, true));
    } else if (batch_rel >= 0) {
        a.batch = c->d_batch + (size_t)batch_rel * P * c->n_slots;
        RBL_TRY(timed(c, kKForceRbl, [&] { launch_force<kShellPredraw>(c, a, energy); }, true));
    } else {
        RBL_TRY(timed(c, kKForceRbl, [&] { launch_force<kShellInline>(c, a, energy); }, true));
    }
    return reduce(c, gated);
}

rbl_status full_force_sorted(rbl_ctx* c, bool energy, bool gated = false)
{
    ForceArgs a = force_args(c, 0, 0, 0, true);
    if (gated) a.gate_clear = c->d_step + 4;
    RBL_TRY(timed(c, kKForceFull, [&] { launch_force<kShellNone>(c, a, energy); }, true));
    return reduce(c);
}

IoArgs io_args(rbl_ctx* c, bool momentum_fix)
{
    IoArgs io;
    io.rep = c->d_rep;
    io.slice_rep = c->d_slice_rep;
    io.perm = c->cur_perm();
    io.rep_sum = c->d_rep_sum;
    io.charges = c->wcol();
    io.n = c->n;
    io.n_slots = c->n_slots;
    io.n_slices = c->n_slices;
    io.momentum_fix = momentum_fix ? 1 : 0;
    io.xs = c->cur_xs();
    io.vs = c->cur_vs();
    io.f = c->d_f;
    io.pos_in = nullptr;
    io.pos_out = nullptr;
    io.vel_out = nullptr;
    io.f_out = nullptr;
    io.img_delta = nullptr;
    io.img = nullptr;
    io.xq = c->d_xq;
    return io;
}

rbl_status emit_ev(rbl_ctx* c, double* ev)
{
    if (!ev) return RBL_OK;
    k_ev_out<<<grid_for(c->R), kBlock, 0, c->ls>>>(c->d_rep_sum, c->R, ev);
    HIP_TRY(hipGetLastError());
    return RBL_OK;
}

// Velocity-Verlet kick/drift, or with a thermostat the BAOAB step (its
// noise keyed by the force evaluation `step` the step leads to, or
// *step_dev + step).
rbl_status integrate(rbl_ctx* c, int mode, double dt, bool momentum_fix, uint64_t seed = 0,
                     uint64_t step = 0, const uint64_t* step_dev = nullptr,
                     const uint64_t* pending = nullptr, int64_t gate_life = 0)
{
    IntArgs a;
    a.langevin = c->gamma > 0.0 ? 1 : 0;
    a.oc = std::exp(-c->gamma * dt);
    a.osig = c->d_osig;
    a.perm = c->cur_perm();
    a.seed = seed;
    a.step = step;
    a.step_dev = step_dev;
    a.pending = pending;
    // gate_life > 0: rebuilds on displacement, lifetimes of at most gate_life steps
    a.gate = gate_life > 0 ? c->d_step + 4 : nullptr;
    a.bstep = c->d_step + 2;
    a.max_life = gate_life;
    a.fgate = gate_life > 0 && c->filt_run ? c->d_step + 5 : nullptr;
    a.xf = c->d_xf;
    a.fhalf2 = c->fhalf2;
    a.xq = c->d_xq;
    a.rep = c->d_rep;
    a.slice_rep = c->d_slice_rep;
    a.rep_sum = c->d_rep_sum;
    a.xs = c->cur_xs();
    a.vs = c->cur_vs();
    a.f = c->d_f;
    a.xb = c->d_xb;
    a.n_slots = c->n_slots;
    a.n_slices = c->n_slices;
    a.h = 0.5 * dt;
    a.dt = dt;
    a.momentum_fix = momentum_fix ? 1 : 0;
    const double hs = 0.5 * c->cfg.skin;
    a.half_skin2 = hs * hs;
    a.flags = c->d_flags;
    const unsigned g = grid_for(c->n_slots);
    return timed(c, kKIntegrate, [&] {
        if (mode == kIntFirst) k_integrate<kIntFirst><<<g, kBlock, 0, c->ls>>>(a);
        else if (mode == kIntMid) k_integrate<kIntMid><<<g, kBlock, 0, c->ls>>>(a);
        else k_integrate<kIntLast><<<g, kBlock, 0, c->ls>>>(a);
    });
}

rbl_status check_p(int P)
{
    if (P < 1 || P > RBL_MAX_P)
        return fail(RBL_E_ARG, "batch size P must be in [1, " + std::to_string(RBL_MAX_P) + "]");
    return RBL_OK;
}


// ---------------------------------------------------------------------------
// molecular-dynamics driver and captured step blocks

__global__ void k_set_block(uint64_t* p, uint64_t step, uint64_t pending)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        p[0] = step;
        p[1] = pending;
    }
}

// Start of a run: build count and rebuild gate cleared, the filter gate
// raised (the first gated force filters the rows it is given), and (entry
// build at `step`, set_build) the step of the last build.
__global__ void k_run_marks(uint64_t* p, uint64_t step, int set_build)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (set_build) p[2] = step;
        p[3] = 0;
        p[4] = 0;
        p[5] = 1;
    }
}

void drop_graphs(rbl_ctx* c)
{
    for (int q = 0; q < 2; ++q)
        if (c->gexec[q]) {
            (void)hipGraphExecDestroy(c->gexec[q]);
            c->gexec[q] = nullptr;
        }
    c->gsig.clear();
}

struct StepParams {
    int P;
    uint64_t seed;
    int64_t K;
    double dt;
    bool full, pre, fix;
    bool check;  // lists rebuilt on displacement (decided on the device)
};

template <typename T>
void sig_put(std::vector<unsigned char>& v, const T& x)
{
    const unsigned char* p = reinterpret_cast<const unsigned char*>(&x);
    v.insert(v.end(), p, p + sizeof(T));
}

std::vector<unsigned char> block_signature(const rbl_ctx* c, const StepParams& sp)
{
    std::vector<unsigned char> v;
    sig_put(v, sp.P);
    sig_put(v, sp.seed);
    sig_put(v, sp.K);
    sig_put(v, sp.dt);
    sig_put(v, (int)sp.full);
    sig_put(v, (int)sp.pre);
    sig_put(v, (int)sp.fix);
    sig_put(v, (int)sp.check);
    sig_put(v, c->r_s);
    sig_put(v, c->r_c);
    sig_put(v, c->n_cells);
    sig_put(v, c->cap_list);
    for (int q = 0; q < 3; ++q) {
        sig_put(v, c->cap[q]);
        sig_put(v, (const void*)c->d_list[q]);
        sig_put(v, (const void*)c->d_len[q]);
    }
    sig_put(v, (const void*)c->d_batch);
    sig_put(v, (const void*)c->d_nI);
    sig_put(v, (const void*)c->d_cell_start);
    sig_put(v, (const void*)c->d_cell_rep);
    sig_put(v, c->profiling);
    sig_put(v, c->gamma);
    sig_put(v, (const void*)c->d_osig);
    sig_put(v, (const void*)c->d_img_delta);
    sig_put(v, (int)c->filt_run);
    sig_put(v, (const void*)c->d_fcore);
    sig_put(v, c->filt2);
    sig_put(v, c->fhalf2);
    return v;
}

// One step of a run whose lists are rebuilt on displacement: kick and drift
// (setting the rebuild gate when some particle has moved more than skin/2
// since the last build, or the lifetime reached K steps), the gated binning
// and list build (lists, and the batches of the K steps from this one), the
// force (which resets the gate) and its reduction.  The step is
// *step_dev + step, or step without a device counter.
rbl_status queue_gated_step(rbl_ctx* c, const StepParams& sp, int mode, uint64_t step,
                            const uint64_t* step_dev, const uint64_t* pending, bool energy)
{
    const uint64_t* gate = c->d_step + 4;
    const int mask = sp.full ? RBL_LIST_FULL : (RBL_LIST_CORE | RBL_LIST_SHELL);
    RBL_TRY(integrate(c, mode, sp.dt, sp.fix, sp.seed, step, step_dev, pending, sp.K));
    RBL_TRY(bin_particles<kSrcSorted>(c, nullptr, nullptr, true, gate));
    if (sp.pre) {
        RBL_TRY(launch_fused(c, sp.P, sp.seed, step, (int)sp.K, step_dev, false, true, gate));
    } else {
        BuildArgs a = loop_build_args(c, step, step_dev, gate);
        RBL_TRY(timed(c, kKBuild, [&] { launch_build<false>(c, a, mask); }));
    }
    if (sp.full) return full_force_sorted(c, energy, true);
    return rbl_force_sorted(c, sp.P, sp.seed, step, sp.pre ? 0 : -1, energy, step_dev, true);
}

// Steps of a captured block of gated steps (rebuilds on displacement): any
// length serves, since every gated step decides its own rebuild.
constexpr int64_t kGatedBlock = 10;

// Queues steps s_b+1 .. s_b+K for replay.  Step-dependent values come from
// the device counter d_step[0] = s_b, so the same queue serves every block;
// d_step[1] says whether the velocities await the closing half-kick of step
// s_b.  Fixed lifetimes: s_b is a multiple of K whose lists and batches are
// built, and the block ends with the rebuild at s_b+K (binning, lists, and
// the batches of s_b+K .. s_b+2K-1).  Rebuilds on displacement:
// kGatedBlock gated steps.
rbl_status queue_block(rbl_ctx* c, const StepParams& sp)
{
    if (sp.check) {
        for (int64_t r = 1; r <= kGatedBlock; ++r)
            RBL_TRY(queue_gated_step(c, sp, kIntMid, (uint64_t)r, c->d_step, r == 1 ? c->d_step + 1 : nullptr,
                                     false));
        return RBL_OK;
    }
    const int mask = sp.full ? RBL_LIST_FULL : (RBL_LIST_CORE | RBL_LIST_SHELL);
    for (int64_t r = 1; r <= sp.K; ++r) {
        RBL_TRY(integrate(c, kIntMid, sp.dt, sp.fix, sp.seed, (uint64_t)r, c->d_step,
                          r == 1 ? c->d_step + 1 : nullptr));
        if (r == sp.K) {
            RBL_TRY(bin_particles<kSrcSorted>(c, nullptr, nullptr, true));
            if (sp.pre) {
                RBL_TRY(launch_fused(c, sp.P, sp.seed, (uint64_t)sp.K, (int)sp.K, c->d_step, false, true));
            } else {
                BuildArgs a = loop_build_args(c, (uint64_t)sp.K, c->d_step, nullptr);
                RBL_TRY(timed(c, kKBuild, [&] { launch_build<false>(c, a, mask); }));
            }
        }
        if (sp.full) RBL_TRY(full_force_sorted(c, false));
        else if (sp.pre) RBL_TRY(rbl_force_sorted(c, sp.P, sp.seed, 0, r == sp.K ? 0 : (int)r, false));
        else RBL_TRY(rbl_force_sorted(c, sp.P, sp.seed, (uint64_t)r, -1, false, c->d_step));
    }
    return RBL_OK;
}

__global__ void k_set_u64(uint64_t* p, uint64_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Filtered core rows for a run with rebuilds on displacement (RBL, one lane
// per particle, core rows of at most 64 entries).  Rows keep the partners
// within r_s + d_f, d_f = skin/2 (with types r_s sigma_ab + d_f, from the
// pair table), and are filtered again once a
// particle has moved d_f/2 - m from its position then.  The positions are
// compared in FP32: stored and current values each round by at most
// 2^-24 (L + skin) (coordinates drift less than skin/2 out of the box
// between rebuilds), and m = 4 2^-24 (L_max + skin) + 1e-6 bounds both with
// room to spare.  A dropped partner was at r >= r_s + d_f and both
// particles have since moved less than d_f/2, so it stays beyond r_s (by at
// least m, far above the rounding of r^2).
// Whether the filter can serve this run, and if so its buffers and
// thresholds (*ok).
// any_lanes: the decision of core_filter = 2 with autotuned lanes, which may
// move a pre-drawn RBL kernel of 2 or 4 lanes to one lane with the filter.
rbl_status prepare_core_filter(rbl_ctx* c, const StepParams& sp, bool& ok, bool any_lanes = false)
{
    ok = false;
    if (!c->cfg.core_filter || sp.full || (sp.pre && c->lpp_rbl != 1 && !any_lanes) || c->cap[0] > 64)
        return RBL_OK;
    if (c->cfg.core_filter == 2 && c->paper) return RBL_OK;
    double lmax = 0.0;
    for (int r = 0; r < c->R; ++r)
        for (int a = 0; a < 3; ++a) lmax = std::max(lmax, c->h_rep[r].L[a]);
    const double df = 0.5 * c->cfg.skin;
    const double m = 4.0 * std::ldexp(lmax + c->cfg.skin, -24) + 1e-6;
    if (!(df > 0.0) || m >= 0.25 * df) return RBL_OK;
    const int64_t need = (int64_t)c->cap[0] * c->n_slots;
    if (need > c->fcore_alloc) {
        dfree(c->d_fcore);
        c->fcore_alloc = 0;
        RBL_TRY(dalloc(&c->d_fcore, (size_t)need));
        c->fcore_alloc = need;
    }
    if (!c->d_fcore_len) RBL_TRY(dalloc(&c->d_fcore_len, (size_t)c->n_slots));
    if (!c->d_xf) RBL_TRY(dalloc(&c->d_xf, 3 * (size_t)c->n_slots));
    const double rf = c->r_s + df;
    const double hf = 0.5 * df - m;
    c->filt2 = rf * rf;
    c->fhalf2 = (float)(hf * hf);
    ok = true;
    return RBL_OK;
}

// At a run's start: core_filter 1 filters whenever it can; 2 once the
// decision (taken at the end of the context's first such run) says so.
rbl_status setup_core_filter(rbl_ctx* c, const StepParams& sp)
{
    c->filt_run = false;
    if (c->cfg.core_filter == 2 && !(c->filt_tuned && c->filt_auto_on)) return RBL_OK;
    bool ok = false;
    RBL_TRY(prepare_core_filter(c, sp, ok));
    c->filt_run = ok;
    return RBL_OK;
}

// core_filter == 2, at the end of the context's first run with rebuilds on
// displacement (a first run often starts from a lattice, whose regular
// neighbourhoods time the kernels unlike the fluid it becomes): times, on
// the final state and its lists, an unfiltered force launch (t_u), the
// filtering launch (t_F) and a launch on the filtered rows (t_f), each
// after 64 MB of stores that push the lists and positions out of L2 as the
// integrator does in a step, and keeps the filter if a filtered step saves
// enough to repay a filtering within R = 0.4 K steps (a filtering comes
// about every half list lifetime, and lifetimes end before the longest, K):
// (t_u - t_f - o) R > t_F - t_f, o being the per-step cost of the gate (the
// FP32 position compare in the integrator and the launch that returns at
// once).  The state and the run's results are left as they are.
rbl_status tune_core_filter(rbl_ctx* c, const StepParams& sp)
{
    c->filt_tuned = true;
    c->filt_auto_on = false;
    // with autotuned lanes a kernel of 2 or 4 lanes per particle competes
    // with one lane on filtered rows
    const bool relane = c->cfg.lanes == 0 && sp.pre;
    bool ok = false;
    RBL_TRY(prepare_core_filter(c, sp, ok, relane));
    if (!ok) return RBL_OK;
    const int lpp0 = c->lpp_rbl;
    // the timed launches write forces and partial sums of their own: the
    // context's hold the run's state (the force the first half-kick takes)
    struct Scratch {
        double* f = nullptr;
        double* part = nullptr;
        int* flush = nullptr;
        ~Scratch()
        {
            dfree(f);
            dfree(part);
            dfree(flush);
        }
    } tmp;
    constexpr int64_t kFlushInts = 16 << 20;  // 64 MB
    RBL_TRY(dalloc(&tmp.f, 3 * (size_t)c->n_slots));
    RBL_TRY(dalloc(&tmp.part, 5 * 4 * (size_t)c->n_slices));
    RBL_TRY(dalloc(&tmp.flush, (size_t)kFlushInts));
    hipEvent_t e0 = take_event(c), e1 = take_event(c);
    if (!e0 || !e1) return fail(RBL_E_HIP, "event creation failed");
    const bool prof = c->profiling;
    c->profiling = false;
    // microseconds per launch (mean of the second and third of three); gate
    // < 0: unfiltered, else the filter gate's value for the launch
    auto time_force = [&](int gate, double& us) -> rbl_status {
        float total = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            ForceArgs a = force_args(c, sp.P, sp.seed, 0, false);
            a.f = tmp.f;
            a.partial = tmp.part;
            if (gate >= 0) {
                k_set_u64<<<1, 64, 0, c->ls>>>(c->d_step + 5, (uint64_t)gate);
                a.fgate = c->d_step + 5;
                a.fcore = c->d_fcore;
                a.fcore_len = c->d_fcore_len;
                a.xf = c->d_xf;
                a.filt2 = c->filt2;
            }
            k_fill_i32<<<grid_for(kFlushInts), kBlock, 0, c->ls>>>(tmp.flush, kFlushInts, rep);
            HIP_TRY(hipEventRecord(e0, c->ls));
            if (sp.pre) {
                a.batch = c->d_batch;
                launch_force<kShellPredraw>(c, a, false);
            } else {
                launch_force<kShellInline>(c, a, false);
            }
            HIP_TRY(hipEventRecord(e1, c->ls));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) total += ms;
        }
        us = 1e3 * total / 2.0;
        return RBL_OK;
    };
    // the layout in use, unfiltered; then one lane per particle with the
    // filter (the filtered kernels are one-lane)
    RBL_TRY(time_force(-1, c->filt_us[0]));
    c->lpp_rbl = 1;
    RBL_TRY(time_force(1, c->filt_us[2]));
    RBL_TRY(time_force(0, c->filt_us[1]));
    c->profiling = prof;
    c->ev_pool.push_back(e0);
    c->ev_pool.push_back(e1);
    const double o = 1.6 + 12.0 * (double)c->n_slots / 5.0e6;  // us: launch + 12 bytes per slot at 5 TB/s
    const double R = 0.4 * (double)sp.K;
    // per step: t_f + o + (t_F - t_f) / R against t_u
    c->filt_auto_on = (c->filt_us[0] - c->filt_us[1] - o) * R > c->filt_us[2] - c->filt_us[1];
    if (!c->filt_auto_on) c->lpp_rbl = lpp0;
    // the run's first gated force filters again
    k_set_u64<<<1, 64, 0, c->ls>>>(c->d_step + 5, 1);
    HIP_TRY(hipGetLastError());
    if (!c->filt_auto_on) {
        // declined for good: the rows' memory goes back (hipFree waits for
        // the launches above)
        dfree(c->d_fcore);
        dfree(c->d_fcore_len);
        dfree(c->d_xf);
        c->fcore_alloc = 0;
    }
    return RBL_OK;
}

rbl_status capture_block(rbl_ctx* c, int parity, const StepParams& sp)
{
    const int saved = c->cur;
    c->cur = parity;
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->ls, hipStreamCaptureModeThreadLocal));
    const rbl_status st = queue_block(c, sp);
    const hipError_t e = hipStreamEndCapture(c->ls, &g);
    c->cur = saved;
    if (st < 0) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(RBL_E_HIP, std::string("stream capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(RBL_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e2));
    c->gexec[parity] = exec;
    return RBL_OK;
}

// Replays the captured lifetime s_b+1 .. s_b+K (capturing it first for the
// current buffer parity if needed).
rbl_status run_block(rbl_ctx* c, int64_t s_b, bool pending, const StepParams& sp)
{
    std::vector<unsigned char> sig = block_signature(c, sp);
    if (sig != c->gsig) {
        drop_graphs(c);
        c->gsig = sig;
    }
    const int parity = c->cur;
    if (!c->gexec[parity]) RBL_TRY(capture_block(c, parity, sp));
    k_set_block<<<1, 64, 0, c->ls>>>(c->d_step, (uint64_t)s_b, pending ? 1u : 0u);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipGraphLaunch(c->gexec[parity], c->ls));
    // a gated block copies each rebuild back into the same buffer set
    if (!sp.check) c->cur = 1 - parity;
    return RBL_OK;
}

// Autotuner: times the force kernel at 1, 2 and 4 lanes per particle on
// the state at hand (lists and batches built) and keeps the fastest for the
// context.  Runs once per context and force kind, outside any capture.
rbl_status autotune_forces(rbl_ctx* c, const StepParams& sp)
{
    const int kind = sp.full ? 1 : 0;
    if (sp.full ? c->tuned_full : c->tuned_rbl) return RBL_OK;
    hipEvent_t e0 = take_event(c), e1 = take_event(c);
    if (!e0 || !e1) return fail(RBL_E_HIP, "event creation failed");
    const bool prof = c->profiling;
    c->profiling = false;
    // microseconds per launch: mean of the second and third of three
    auto time_force = [&](double& us) -> rbl_status {
        float total = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
            HIP_TRY(hipEventRecord(e0, c->ls));
            if (sp.full) RBL_TRY(full_force_sorted(c, false));
            else if (sp.pre) RBL_TRY(rbl_force_sorted(c, sp.P, sp.seed, 0, 0, false));
            else RBL_TRY(rbl_force_sorted(c, sp.P, sp.seed, 0, -1, false));
            HIP_TRY(hipEventRecord(e1, c->ls));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) total += ms;
        }
        us = 1e3 * total / 2.0;
        return RBL_OK;
    };
    // lanes per particle (the inline-draw kernel has one lane per particle)
    if (c->cfg.lanes == 0 && (sp.full || sp.pre)) {
        const int cand[3] = {1, 2, 4};
        double best = 1e30;
        int best_lpp = 4;
        for (int q = 0; q < 3; ++q) {
            (sp.full ? c->lpp_full : c->lpp_rbl) = cand[q];
            RBL_TRY(time_force(c->tune_us[kind][q]));
            if (c->tune_us[kind][q] < best) {
                best = c->tune_us[kind][q];
                best_lpp = cand[q];
            }
        }
        (sp.full ? c->lpp_full : c->lpp_rbl) = best_lpp;
    }
    // one block per tile or a persistent grid (same results either way)
    if (c->cfg.persistent == 0) {
        for (int q = 0; q < 2; ++q) {
            c->persist[kind] = q == 1;
            RBL_TRY(time_force(c->persist_us[kind][q]));
        }
        c->persist[kind] = c->persist_us[kind][1] < c->persist_us[kind][0];
    }
    c->profiling = prof;
    c->ev_pool.push_back(e0);
    c->ev_pool.push_back(e1);
    (sp.full ? c->tuned_full : c->tuned_rbl) = true;
    return RBL_OK;
}

struct LaunchStreamGuard {
    rbl_ctx* c;
    ~LaunchStreamGuard() { c->ls = c->stream; }
};

void set_draw(rbl_ctx* c, int64_t step0, int steps, int P)
{
    c->draw_step0 = step0;
    c->draw_steps = steps;
    c->draw_P = P;
}

// One run of Algorithm 1 (readings of the step schedule in include/rbl.h):
// from the caller's arrays (pos_in, vel_in; a list build at step0) or, with
// `resume`, from the state the last run left in the context.  Writes the
// final positions, velocities and forces to whichever of pos_out, vel_out
// and force are given.  `overflow` reports a list that outgrew its room;
// the run's results are then void and it has to be repeated.
rbl_status md_run(rbl_ctx* c, const double* pos_in, const double* vel_in, double* pos_out, double* vel_out,
                  double* force, int64_t nsteps, double dt, int P, uint64_t seed, int64_t step0, int64_t K,
                  bool full, double* ev, bool resume, bool& overflow)
{
    overflow = false;
    StepParams sp;
    sp.P = P;
    sp.seed = seed;
    sp.K = K;
    sp.dt = dt;
    sp.full = full;
    sp.fix = !full && c->cfg.momentum_fix;
    sp.pre = !full && ((c->cfg.predraw && c->fused_ok) || c->stencil);
    sp.check = c->cfg.rebuild_check != 0;
    if (!full && !sp.pre && P > 32)
        return fail(RBL_E_ARG, "this context draws its batches in the force kernel (explicit shell rows: "
                               "particle types, predraw off, or a stencil beyond the fused build), "
                               "which takes P <= 32");
    const int mask = full ? RBL_LIST_FULL : (RBL_LIST_CORE | RBL_LIST_SHELL);
    const bool use_graph = c->cfg.graphs && !c->profiling && c->gs;
    LaunchStreamGuard guard{c};
    if (use_graph) {
        HIP_TRY(hipEventRecord(c->ev_in, c->stream));
        HIP_TRY(hipStreamWaitEvent(c->gs, c->ev_in, 0));
        c->ls = c->gs;
    }
    const int64_t resume_build = c->run.build_step;
    c->run.valid = false;
    RBL_TRY(clear_flags(c));
    k_run_marks<<<1, 64, 0, c->ls>>>(c->d_step, 0, 0);
    HIP_TRY(hipGetLastError());
    // wraps of this run's builds are counted apart and added to the
    // trajectory's image counters only when the run completes
    if (!c->d_img) {
        RBL_TRY(dalloc(&c->d_img, 3 * (size_t)c->n));
        RBL_TRY(fill_i32(c, c->d_img, 3 * c->n, 0));
    }
    if (!c->d_img_delta) RBL_TRY(dalloc(&c->d_img_delta, 3 * (size_t)c->n));
    RBL_TRY(fill_i32(c, c->d_img_delta, 3 * c->n, 0));
    struct TrackGuard {
        rbl_ctx* c;
        ~TrackGuard() { c->track_images = false; }
    } track{c};
    c->track_images = true;
    if (c->gamma > 0.0) {
        if (!c->d_osig) RBL_TRY(dalloc(&c->d_osig, (size_t)c->R));
        const double oc = std::exp(-c->gamma * dt);
        c->h_osig.resize(c->R);
        for (int r = 0; r < c->R; ++r) c->h_osig[r] = std::sqrt(c->kT[r] * (1.0 - oc * oc));
        HIP_TRY(hipMemcpyAsync(c->d_osig, c->h_osig.data(), sizeof(double) * c->R, hipMemcpyHostToDevice,
                               c->ls));
    }
    const int64_t last = step0 + nsteps;
    int64_t build_step = resume ? resume_build : step0;

    auto do_build = [&](int64_t s, bool from_caller) -> rbl_status {
        if (from_caller) RBL_TRY(bin_particles<kSrcCaller>(c, pos_in, vel_in, true));
        else RBL_TRY(bin_particles<kSrcSorted>(c, nullptr, nullptr, true));
        c->built = false;
        build_step = s;
        if (sp.pre) {
            // batches for every force evaluation of the list lifetime, also
            // those past this run's end (a continued run uses them); a
            // lifetime ends at the next multiple of K, or with rebuilds on
            // displacement at most K steps on
            const int64_t cnt = sp.check ? K : (s / K + 1) * K - s;
            RBL_TRY(prepare_fused(c, P, (int)K));
            RBL_TRY(launch_fused(c, P, seed, (uint64_t)s, (int)cnt, nullptr, false, true));
            set_draw(c, s, (int)cnt, P);
            c->built_mask = RBL_LIST_CORE;
            c->shell_counts = !c->stencil;
        } else {
            RBL_TRY(prepare_lists(c, mask));
            BuildArgs a = loop_build_args(c, (uint64_t)s, nullptr, nullptr);
            RBL_TRY(timed(c, kKBuild, [&] { launch_build<false>(c, a, mask); }));
            set_draw(c, 0, 0, 0);
            c->built_mask = mask;
            c->shell_counts = (mask & RBL_LIST_SHELL) != 0;
        }
        c->built = true;
        return RBL_OK;
    };
    auto do_force = [&](int64_t s, bool energy) -> rbl_status {
        if (full) return full_force_sorted(c, energy);
        return rbl_force_sorted(c, P, seed, (uint64_t)s, sp.pre ? (int)(s - build_step) : -1, energy);
    };

    if (!resume) {
        RBL_TRY(do_build(step0, true));
        if (c->cfg.lanes == 0 || c->cfg.persistent == 0) RBL_TRY(autotune_forces(c, sp));
        RBL_TRY(do_force(step0, ev != nullptr && nsteps == 0));
    }
    struct FilterGuard {
        rbl_ctx* c;
        ~FilterGuard() { c->filt_run = false; }
    } fguard{c};
    if (sp.check) RBL_TRY(setup_core_filter(c, sp));
    else c->filt_run = false;
    c->filt_last = c->filt_run;
    // pending: the velocities await the closing half-kick of the last force
    bool pending = false;
    int64_t it = 1;
    while (sp.check && it <= nsteps) {
        // rebuilds decided on the device: blocks of kGatedBlock gated steps
        // (not the run's last block when its energy is asked for)
        const int64_t s = step0 + it;
        const int64_t G = kGatedBlock;
        if (use_graph && it + G - 1 <= nsteps && !(ev && it + G - 1 == nsteps)) {
            RBL_TRY(run_block(c, s - 1, pending, sp));
            it += G;
        } else {
            RBL_TRY(queue_gated_step(c, sp, pending ? kIntMid : kIntFirst, (uint64_t)s, nullptr, nullptr,
                                     ev != nullptr && it == nsteps));
            ++it;
        }
        pending = true;
        c->built = true;
        c->built_mask = sp.full ? RBL_LIST_FULL : (sp.pre ? RBL_LIST_CORE : mask);
        c->shell_counts = !sp.full && !c->stencil;
    }
    while (!sp.check && it <= nsteps) {
        const int64_t s = step0 + it;
        const int64_t s_b = s - 1;
        // A whole list lifetime s_b+1 .. s_b+K whose lists were built at s_b
        // replays as a captured block (not the run's last lifetime when its
        // energy is asked for: that force is queued with the energy sums).
        if (use_graph && s_b % K == 0 && build_step == s_b && (s_b + K < last || (s_b + K == last && !ev))) {
            RBL_TRY(run_block(c, s_b, pending, sp));
            build_step = s_b + K;
            if (sp.pre) set_draw(c, build_step, (int)K, P);
            else set_draw(c, 0, 0, 0);
            c->built = true;
            c->built_mask = sp.full ? RBL_LIST_FULL : (sp.pre ? RBL_LIST_CORE : mask);
            c->shell_counts = !sp.full && !c->stencil;
            pending = true;
            it += K;
            continue;
        }
        RBL_TRY(integrate(c, pending ? kIntMid : kIntFirst, dt, sp.fix, seed, (uint64_t)s));
        if (s % K == 0) RBL_TRY(do_build(s, false));
        RBL_TRY(do_force(s, ev != nullptr && it == nsteps));
        pending = true;
        ++it;
    }
    if (pending) RBL_TRY(integrate(c, kIntLast, dt, sp.fix));
    HIP_TRY(hipMemcpyAsync(c->h_marks, c->d_step + 2, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, c->ls));
    RBL_TRY(read_flags(c));
    c->run.builds = (int64_t)c->h_marks[1];
    if (sp.check) {
        // the step of the last build is known on the device only
        build_step = (int64_t)c->h_marks[0];
        if (sp.pre) set_draw(c, build_step, (int)K, P);
    }
    if (c->h_flags[kFlagStencil]) {
        // a stencil held more candidates than the fused kernel's LDS lists:
        // the run is repeated on explicit core and shell rows
        c->fused_ok = false;
        overflow = true;
        return RBL_OK;
    }
    if (c->h_flags[kFlagOverflow]) {
        if (sp.pre && c->h_flags[kFlagMaxShell] > c->cap_list) grow_cap_list(c, c->h_flags[kFlagMaxShell], true);
        overflow = true;
        return RBL_OK;
    }
    if (c->h_flags[kFlagNonfinite]) return fail(RBL_E_NONFINITE, "non-finite position during the run");
    if (c->h_flags[kFlagBadSlot]) return fail(RBL_E_HIP, "inconsistent cell binning");
    if (sp.check && c->cfg.core_filter == 2 && !c->filt_tuned) RBL_TRY(tune_core_filter(c, sp));
    IoArgs io = io_args(c, sp.fix);
    io.pos_out = pos_out;
    io.vel_out = vel_out;
    io.f_out = force;
    io.img_delta = c->d_img_delta;
    io.img = c->d_img;
    k_scatter_out<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(io);
    HIP_TRY(hipGetLastError());
    RBL_TRY(emit_ev(c, ev));
    if (use_graph) {
        HIP_TRY(hipEventRecord(c->ev_out, c->gs));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->ev_out, 0));
    }
    c->run.valid = true;
    c->run.P = P;
    c->run.seed = seed;
    c->run.K = K;
    c->run.dt = dt;
    c->run.full = full;
    c->run.end_step = last;
    c->run.build_step = build_step;
    if (c->h_flags[kFlagSkin]) {
        g_err = "a particle moved more than skin/2 within one list lifetime";
        return RBL_W_SKIN;
    }
    return RBL_OK;
}

// After a run whose rows outgrew their room: grows the rows of the lists
// the repeat will build (the fused kernel's LDS room grew in md_run).
rbl_status grow_after_overflow(rbl_ctx* c, bool full)
{
    drop_graphs(c);
    if (c->h_flags[kFlagStencil]) return RBL_OK;  // rows of the explicit path get counted afresh
    const int mask = full ? RBL_LIST_FULL
                          : (((c->cfg.predraw && c->fused_ok) || c->stencil) ? RBL_LIST_CORE
                                                                            : (RBL_LIST_CORE | RBL_LIST_SHELL));
    for (int q = 0; q < 3; ++q)
        if ((mask >> q) & 1) RBL_TRY(ensure_list_storage(c, q, c->h_flags[kFlagMaxCore + q], true));
    return RBL_OK;
}

// out[r] = (1 / n_r) sum over replica r of |x - y|^2 (y may be null)
rbl_status mean_sq(rbl_ctx* c, const double* x, const double* y, double* out)
{
    int64_t most = 1;
    for (int r = 0; r < c->R; ++r) most = std::max(most, c->rep_n[r]);
    const int nb = (int)((most + 256 * kSqIter - 1) / (256 * kSqIter));
    if (nb > c->sq_nb) {
        dfree(c->d_sq_part);
        c->sq_nb = 0;
        RBL_TRY(dalloc(&c->d_sq_part, (size_t)nb * c->R));
        c->sq_nb = nb;
    }
    k_sumsq<<<dim3(nb, c->R), 256, 0, c->ls>>>(c->d_rep, x, y, c->n, nb, c->d_sq_part);
    HIP_TRY(hipGetLastError());
    k_sumsq_final<<<(c->R + 63) / 64, 64, 0, c->ls>>>(c->d_rep, c->d_sq_part, nb, c->R, 1.0, out);
    HIP_TRY(hipGetLastError());
    return RBL_OK;
}
// Parameters of the run rbl_continue resumes.
struct RbRun {
    int P;
    uint64_t seed;
    int64_t K;
    double dt;
    bool full;
    int64_t step0;
};
}  // namespace

// ===========================================================================
// C-ABI

extern "C" {

void rbl_config_init(rbl_config* cfg, int64_t n)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->n = n;
    cfg->n_replicas = 1;
    cfg->precision = RBL_PREC_FP64;
    cfg->pair = RBL_PAIR_LJ;
    cfg->lists = RBL_LIST_CORE | RBL_LIST_SHELL;
    cfg->skin = 0.3;
    cfg->alpha = 0.0;
    cfg->shift = 1;
    cfg->momentum_fix = 1;
    cfg->predraw = 1;
    cfg->graphs = 1;
    cfg->lanes = 0;
    cfg->persistent = 0;
    cfg->capacity_factor = 1.25;
    cfg->replica_offsets = nullptr;
    cfg->charges = nullptr;
    cfg->shell_source = RBL_SHELL_LIST;
    cfg->rebuild_check = 0;
    cfg->core_filter = 2;
    cfg->n_types = 0;
    cfg->types = nullptr;
    cfg->pair_coeffs = nullptr;
}

const char* rbl_last_error(void) { return g_err.c_str(); }

const char* rbl_version(void) { return "librbl 0.1 (gfx950)"; }

rbl_status rbl_destroy(rbl_ctx* c)
{
    if (!c) return RBL_OK;
    (void)hipStreamSynchronize(c->stream);
    if (c->gs) (void)hipStreamSynchronize(c->gs);
    for (int q = 0; q < 2; ++q)
        if (c->gexec[q]) (void)hipGraphExecDestroy(c->gexec[q]);
    if (c->gs) (void)hipStreamDestroy(c->gs);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    dfree(c->d_step);
    for (int k = 0; k < kKinds; ++k)
        for (auto& pr : c->ev_pending[k]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    dfree(c->d_rep);
    dfree(c->d_id_rep);
    dfree(c->d_slice_rep);
    dfree(c->d_cell_rep);
    dfree(c->d_cell_count);
    dfree(c->d_cell_start);
    dfree(c->d_tile_sum);
    dfree(c->d_cell_of_src);
    dfree(c->d_rank_of_src);
    dfree(c->d_src_of_slot);
    dfree(c->d_perm[0]);
    dfree(c->d_perm[1]);
    dfree(c->d_slot_of_id);
    dfree(c->d_xs[0]);
    dfree(c->d_xs[1]);
    dfree(c->d_xq);
    dfree(c->d_tcol);
    dfree(c->d_tt);
    dfree(c->d_vs[0]);
    dfree(c->d_vs[1]);
    dfree(c->d_xb);
    dfree(c->d_f);
    dfree(c->d_fcore);
    dfree(c->d_fcore_len);
    dfree(c->d_xf);
    for (int q = 0; q < 3; ++q) {
        dfree(c->d_list[q]);
        dfree(c->d_len[q]);
    }
    dfree(c->d_batch);
    dfree(c->d_nI);
    dfree(c->d_pgrid);
    dfree(c->d_pcell_rep);
    dfree(c->d_pcount);
    dfree(c->d_pstart);
    dfree(c->d_ptile);
    dfree(c->d_pcell_of_slot);
    dfree(c->d_prank);
    dfree(c->d_pmember);
    dfree(c->d_osig);
    dfree(c->d_img);
    dfree(c->d_img_delta);
    dfree(c->d_ckpt);
    dfree(c->d_sq_part);
    dfree(c->d_partial);
    dfree(c->d_part2);
    dfree(c->d_rep_sum);
    dfree(c->d_flags);
    delete c;
    return RBL_OK;
}

rbl_status rbl_create(const rbl_config* cfg, void* hip_stream, rbl_ctx** out)
{
    if (!cfg || !out) return fail(RBL_E_ARG, "NULL config or output pointer");
    *out = nullptr;
    if (cfg->n < 1 || cfg->n > 0x7fffffff - 64 * (int64_t)std::max(cfg->n_replicas, 1))
        return fail(RBL_E_ARG, "particle count out of range");
    if (cfg->n_replicas < 1) return fail(RBL_E_ARG, "n_replicas must be >= 1");
    if (cfg->n_replicas > 1 && !cfg->replica_offsets)
        return fail(RBL_E_ARG, "replica_offsets required for n_replicas > 1");
    if (cfg->precision != RBL_PREC_FP64 && cfg->precision != RBL_PREC_MIXED)
        return fail(RBL_E_ARG, "unknown precision");
    if (cfg->pair != RBL_PAIR_LJ && cfg->pair != RBL_PAIR_LJ_ERFC) return fail(RBL_E_ARG, "unknown pair");
    if (cfg->lists <= 0 || cfg->lists > 7) return fail(RBL_E_ARG, "list mask must be in 1..7");
    if (cfg->lanes != 0 && cfg->lanes != 1 && cfg->lanes != 2 && cfg->lanes != 4)
        return fail(RBL_E_ARG, "lanes must be 0, 1, 2 or 4");
    if (cfg->persistent < 0 || cfg->persistent > 2) return fail(RBL_E_ARG, "persistent must be 0, 1 or 2");
    if (!(cfg->skin >= 0.0) || !std::isfinite(cfg->skin)) return fail(RBL_E_ARG, "skin must be >= 0");
    if (!(cfg->capacity_factor > 0.0) || !std::isfinite(cfg->capacity_factor))
        return fail(RBL_E_ARG, "capacity_factor must be > 0");
    if (cfg->pair == RBL_PAIR_LJ_ERFC && !(cfg->alpha > 0.0)) return fail(RBL_E_ARG, "alpha must be > 0");
    if (cfg->shell_source != RBL_SHELL_LIST && cfg->shell_source != RBL_SHELL_STENCIL &&
        cfg->shell_source != RBL_SHELL_PAPER)
        return fail(RBL_E_ARG, "shell_source must be RBL_SHELL_LIST, RBL_SHELL_STENCIL or RBL_SHELL_PAPER");
    if (cfg->core_filter < 0 || cfg->core_filter > 2) return fail(RBL_E_ARG, "core_filter must be 0, 1 or 2");
    if (cfg->n_types < 0 || cfg->n_types > kMaxTypes)
        return fail(RBL_E_ARG, "n_types must be in 0 .. " + std::to_string(kMaxTypes));
    if (cfg->n_types == 0 && (cfg->types || cfg->pair_coeffs))
        return fail(RBL_E_ARG, "types and pair_coeffs need n_types >= 1");
    if (cfg->n_types > 0) {
        const int T = cfg->n_types;
        if (!cfg->types || !cfg->pair_coeffs) return fail(RBL_E_ARG, "n_types >= 1 needs types and pair_coeffs");
        if (cfg->pair != RBL_PAIR_LJ || cfg->charges)
            return fail(RBL_E_ARG, "particle types take the LJ pair only (no charges)");
        if (cfg->shell_source != RBL_SHELL_LIST)
            return fail(RBL_E_ARG, "particle types take shell_source RBL_SHELL_LIST");
        for (int a = 0; a < T; ++a)
            for (int b = 0; b < T; ++b) {
                const double e = cfg->pair_coeffs[(a * T + b) * 2], g = cfg->pair_coeffs[(a * T + b) * 2 + 1];
                if (!(e >= 0.0) || !(g > 0.0) || !std::isfinite(e) || !std::isfinite(g))
                    return fail(RBL_E_ARG, "pair_coeffs: epsilon must be >= 0 and sigma > 0, finite");
                if (e != cfg->pair_coeffs[(b * T + a) * 2] || g != cfg->pair_coeffs[(b * T + a) * 2 + 1])
                    return fail(RBL_E_ARG, "pair_coeffs must be symmetric");
            }
        for (int64_t i = 0; i < cfg->n; ++i)
            if (cfg->types[i] < 0 || cfg->types[i] >= T)
                return fail(RBL_E_ARG, "particle " + std::to_string(i) + " has a type outside 0 .. n_types-1");
    }
    std::vector<int64_t> off(cfg->n_replicas + 1);
    if (cfg->n_replicas == 1) {
        off[0] = 0;
        off[1] = cfg->n;
    } else {
        for (int r = 0; r <= cfg->n_replicas; ++r) off[r] = cfg->replica_offsets[r];
        if (off[0] != 0 || off[cfg->n_replicas] != cfg->n)
            return fail(RBL_E_ARG, "replica_offsets must run from 0 to n");
        for (int r = 0; r < cfg->n_replicas; ++r)
            if (off[r + 1] <= off[r]) return fail(RBL_E_ARG, "every replica needs >= 1 particle");
    }
    rbl_ctx* c = new rbl_ctx();
    c->cfg = *cfg;
    c->cfg.replica_offsets = nullptr;
    c->cfg.types = nullptr;
    c->cfg.pair_coeffs = nullptr;
    if (cfg->n_types > 0) {
        const int T = cfg->n_types;
        c->typed = true;
        // explicit rows: a type's stencil may exceed the fused build's
        c->fused_ok = false;
        c->eps_sig.assign(cfg->pair_coeffs, cfg->pair_coeffs + 2 * T * T);
        c->sig_min = c->sig_max = cfg->pair_coeffs[1];
        for (int k = 0; k < T * T; ++k) {
            c->sig_min = std::min(c->sig_min, cfg->pair_coeffs[2 * k + 1]);
            c->sig_max = std::max(c->sig_max, cfg->pair_coeffs[2 * k + 1]);
        }
    }
    c->stream = (hipStream_t)hip_stream;
    c->ls = c->stream;
    c->R = cfg->n_replicas;
    c->n = cfg->n;
    if (cfg->lanes > 0) c->lpp_rbl = c->lpp_full = cfg->lanes;
    c->persist[0] = c->persist[1] = cfg->persistent == 2;
    c->stencil = cfg->shell_source != RBL_SHELL_LIST;
    c->paper = cfg->shell_source == RBL_SHELL_PAPER;
    c->kT.assign(c->R, 1.0);
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            c->n_cu = ncu;
        c->device = dev;
        // the allocation-free force call's array on this device
        (void)scratch_setup(dev);
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess &&
            lds > 0)
            c->lds_per_cu = lds;
    }
    int64_t slot = 0;
    for (int r = 0; r < c->R; ++r) {
        c->id_base.push_back(off[r]);
        c->rep_n.push_back(off[r + 1] - off[r]);
        c->slot_base.push_back(slot);
        slot += (off[r + 1] - off[r] + 63) / 64 * 64;
    }
    c->n_slots = slot;
    c->n_slices = slot / 64;

    auto bail = [&](rbl_status s) {
        std::string keep = g_err;
        rbl_destroy(c);
        g_err = keep;
        return s;
    };
#define CR(expr)                             \
    do {                                     \
        rbl_status s_ = (expr);              \
        if (s_ < 0) return bail(s_);         \
    } while (0)
    CR(dalloc(&c->d_rep, c->R));
    CR(dalloc(&c->d_id_rep, c->n));
    CR(dalloc(&c->d_slice_rep, c->n_slices));
    CR(dalloc(&c->d_cell_of_src, c->n_slots));
    CR(dalloc(&c->d_rank_of_src, c->n_slots));
    CR(dalloc(&c->d_src_of_slot, c->n_slots));
    CR(dalloc(&c->d_perm[0], c->n_slots));
    CR(dalloc(&c->d_perm[1], c->n_slots));
    CR(dalloc(&c->d_slot_of_id, c->n));
    CR(dalloc(&c->d_xs[0], c->n_slots));
    CR(dalloc(&c->d_xs[1], c->n_slots));
    if (c->typed) {
        CR(dalloc(&c->d_tcol, c->n));
        std::vector<double> tv(cfg->types, cfg->types + cfg->n);
        if (hipMemcpy(c->d_tcol, tv.data(), sizeof(double) * c->n, hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(RBL_E_HIP, "upload of particle types failed"));
    }
    if (cfg->precision == RBL_PREC_MIXED) CR(dalloc(&c->d_xq, c->n_slots));
    if (c->paper) {
        CR(dalloc(&c->d_pgrid, c->R));
        CR(dalloc(&c->d_pcell_of_slot, c->n_slots));
        CR(dalloc(&c->d_prank, c->n_slots));
        CR(dalloc(&c->d_pmember, c->n_slots));
    }
    CR(dalloc(&c->d_vs[0], 3 * c->n_slots));
    CR(dalloc(&c->d_vs[1], 3 * c->n_slots));
    CR(dalloc(&c->d_xb, 3 * c->n_slots));
    CR(dalloc(&c->d_f, 3 * c->n_slots));
    CR(dalloc(&c->d_partial, 5 * 4 * c->n_slices));
    {
        int64_t mx = 1;
        for (int r = 0; r < c->R; ++r) mx = std::max<int64_t>(mx, 4 * ((c->rep_n[r] + 63) / 64));
        c->red_blocks = (int)((mx + kReduceSlicesPerBlock - 1) / kReduceSlicesPerBlock);
    }
    CR(dalloc(&c->d_part2, (size_t)5 * c->red_blocks * c->R));
    CR(dalloc(&c->d_rep_sum, 8 * c->R));
    CR(dalloc(&c->d_flags, kNumFlags));
    CR(dalloc(&c->d_step, 8));
    if (hipStreamCreateWithFlags(&c->gs, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess)
        return bail(fail(RBL_E_HIP, "could not create the internal stream"));
    {
        std::vector<int> id_rep(c->n), slice_rep(c->n_slices);
        for (int r = 0; r < c->R; ++r) {
            std::fill(id_rep.begin() + off[r], id_rep.begin() + off[r + 1], r);
            const int64_t s0 = c->slot_base[r] / 64;
            const int64_t ns = (c->rep_n[r] + 63) / 64;
            std::fill(slice_rep.begin() + s0, slice_rep.begin() + s0 + ns, r);
        }
        if (hipMemcpy(c->d_id_rep, id_rep.data(), sizeof(int) * c->n, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(c->d_slice_rep, slice_rep.data(), sizeof(int) * c->n_slices,
                      hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(RBL_E_HIP, "upload of replica tables failed"));
    }
    CR(fill_i32(c, c->d_perm[0], c->n_slots, -1));
    CR(fill_i32(c, c->d_perm[1], c->n_slots, -1));
    CR(fill_i32(c, c->d_flags, kNumFlags, 0));
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(fail(RBL_E_HIP, "stream sync failed"));
#undef CR
    *out = c;
    return RBL_OK;
}

rbl_status rbl_build(rbl_ctx* c, const double* pos, const double* box, double r_s, double r_c)
{
    if (!c || !pos || !box) return fail(RBL_E_ARG, "NULL argument");
    if (!(r_s > 0.0) || !(r_c > r_s) || !std::isfinite(r_c))
        return fail(RBL_E_ARG, "radii must satisfy 0 < r_s < r_c");
    RBL_TRY(setup_geometry(c, box, r_s, r_c));
    c->run.valid = false;
    c->pop_valid = false;
    set_draw(c, 0, 0, 0);
    c->built = false;
    c->shell_counts = false;
    RBL_TRY(clear_flags(c));
    RBL_TRY(bin_particles<kSrcCaller>(c, pos, nullptr, false));
    if (c->paper) paper_bin(c, nullptr);
    RBL_TRY(build_lists(c, c->cfg.lists));
    c->built = true;
    return RBL_OK;
}

}  // extern "C"

namespace {

rbl_status forces_check(rbl_ctx* c, int P, const double* pos, const double* force)
{
    if (!c || !pos || !force) return fail(RBL_E_ARG, "NULL argument");
    RBL_TRY(check_p(P));
    if (!c->built) return fail(RBL_E_STATE, "rbl_forces needs a list build first");
    const int need = c->stencil ? RBL_LIST_CORE : (RBL_LIST_CORE | RBL_LIST_SHELL);
    if ((c->built_mask & need) != need)
        return fail(RBL_E_STATE, c->stencil ? "the last build has no core list"
                                            : "the last build has no core and shell lists");
    return RBL_OK;
}

// The RBL force of rbl_forces (arguments checked).  `record`: the batches
// drawn here are the context's stored ones (rbl_export_drawn_batches).
rbl_status forces_call(rbl_ctx* c, int P, uint64_t seed, uint64_t step, const double* pos, double* force,
                       double* ev, bool record)
{
    c->run.valid = false;
    if (c->stencil) {
        // batches from the stencil cells of the build's binning
        RBL_TRY(ensure_batch(c, 1, P));
        if (!c->d_nI) RBL_TRY(dalloc(&c->d_nI, c->n_slots));
        RBL_TRY(launch_fused(c, P, seed, step, 1, nullptr, true));
        if (record) set_draw(c, (int64_t)step, 1, P);
    }
    IoArgs io = io_args(c, c->cfg.momentum_fix != 0);
    io.pos_in = pos;
    k_load_positions<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(io);
    HIP_TRY(hipGetLastError());
    if (c->stencil) {
        RBL_TRY(rbl_force_sorted(c, P, seed, step, 0, ev != nullptr));
    } else if (P <= 32) {
        RBL_TRY(rbl_force_sorted(c, P, seed, step, -1, ev != nullptr));
    } else {
        RBL_TRY(predraw(c, P, seed, step, 1));
        if (record) set_draw(c, (int64_t)step, 1, P);
        RBL_TRY(rbl_force_sorted(c, P, seed, step, 0, ev != nullptr));
    }
    io.f_out = force;
    k_scatter_out<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(io);
    HIP_TRY(hipGetLastError());
    return emit_ev(c, ev);
}

}  // namespace

extern "C" {

rbl_status rbl_forces(rbl_ctx* c, int P, uint64_t seed, uint64_t step, const double* pos,
                      double* force, double* ev)
{
    RBL_TRY(forces_check(c, P, pos, force));
    return forces_call(c, P, seed, step, pos, force, ev, true);
}

rbl_status rbl_forces_noalloc(rbl_ctx* c, int P, uint64_t seed, uint64_t step, const double* pos,
                              double* force, double* ev)
{
    RBL_TRY(forces_check(c, P, pos, force));
    unsigned char* const base = static_cast<unsigned char*>(scratch_dev[c->device]);
    if (!base) return fail(RBL_E_STATE, "the scratch array's device address is unavailable on this device");
    // carve the call's buffers out of the array, 256-byte aligned
    const bool draws = c->stencil || P > 32;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t o_partial = carve(sizeof(double) * 5 * 4 * (size_t)c->n_slices);
    const size_t o_part2 = carve(sizeof(double) * 5 * (size_t)c->red_blocks * c->R);
    const size_t o_rep = carve(sizeof(double) * 8 * (size_t)c->R);
    const size_t o_batch = draws ? carve(sizeof(int) * (size_t)P * c->n_slots) : 0;
    const size_t o_ni = c->stencil ? carve(sizeof(int) * (size_t)c->n_slots) : 0;
    if (off > kScratchBytes)
        return fail(RBL_E_CAPACITY, "rbl_forces_noalloc needs " + std::to_string(off) + " bytes of scratch for " +
                                        std::to_string(c->n_slots) + " slots at P = " + std::to_string(P) +
                                        ", above its " + std::to_string(kScratchBytes) + "-byte array");
    // the context's own buffers stand aside for the call
    struct Swap {
        rbl_ctx* c;
        double *partial, *part2, *rep_sum;
        int *batch, *nI;
        size_t batch_alloc;
        ~Swap()
        {
            c->d_partial = partial;
            c->d_part2 = part2;
            c->d_rep_sum = rep_sum;
            c->d_batch = batch;
            c->d_nI = nI;
            c->batch_alloc = batch_alloc;
        }
    } swap{c, c->d_partial, c->d_part2, c->d_rep_sum, c->d_batch, c->d_nI, c->batch_alloc};
    c->d_partial = reinterpret_cast<double*>(base + o_partial);
    c->d_part2 = reinterpret_cast<double*>(base + o_part2);
    c->d_rep_sum = reinterpret_cast<double*>(base + o_rep);
    c->d_batch = draws ? reinterpret_cast<int*>(base + o_batch) : nullptr;
    c->batch_alloc = draws ? (size_t)P * c->n_slots : 0;
    c->d_nI = c->stencil ? reinterpret_cast<int*>(base + o_ni) : nullptr;
    return forces_call(c, P, seed, step, pos, force, ev, false);
}

rbl_status rbl_full_forces(rbl_ctx* c, const double* pos, double* force, double* ev)
{
    if (!c || !pos || !force) return fail(RBL_E_ARG, "NULL argument");
    if (!c->built) return fail(RBL_E_STATE, "rbl_full_forces needs a list build first");
    if (!(c->built_mask & RBL_LIST_FULL)) return fail(RBL_E_STATE, "the last build has no full list");
    c->run.valid = false;
    IoArgs io = io_args(c, false);
    io.pos_in = pos;
    k_load_positions<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(io);
    HIP_TRY(hipGetLastError());
    RBL_TRY(full_force_sorted(c, ev != nullptr));
    io.f_out = force;
    k_scatter_out<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(io);
    HIP_TRY(hipGetLastError());
    return emit_ev(c, ev);
}

rbl_status rbl_step(rbl_ctx* c, double* pos, double* vel, double* force, int64_t nsteps, double dt,
                    int P, uint64_t seed, int64_t step0, int rebuild_every, int use_full, double* ev)
{
    if (!c || !pos || !vel) return fail(RBL_E_ARG, "NULL argument");
    if (nsteps < 0 || step0 < 0) return fail(RBL_E_ARG, "nsteps and step0 must be >= 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RBL_E_ARG, "dt must be > 0");
    if (rebuild_every < 1) return fail(RBL_E_ARG, "rebuild_every must be >= 1");
    if (!use_full) RBL_TRY(check_p(P));
    if (c->r_c <= 0.0) return fail(RBL_E_STATE, "rbl_step needs box and radii from rbl_build");
    const bool full = use_full != 0;
    // A run whose rows outgrew their capacity is repeated from the caller's
    // arrays (written only at the end) with rows sized to what it saw.
    for (int attempt = 0; attempt < 3; ++attempt) {
        bool overflow = false;
        c->run.attempts = attempt + 1;
        const rbl_status st = md_run(c, pos, vel, pos, vel, force, nsteps, dt, P, seed, step0, rebuild_every,
                                     full, ev, false, overflow);
        if (st < 0 || !overflow) return st;
        RBL_TRY(grow_after_overflow(c, full));
    }
    return fail(RBL_E_CAPACITY, "neighbour rows kept overflowing their capacity");
}

rbl_status rbl_continue(rbl_ctx* c, double* pos, double* vel, double* force, int64_t nsteps, double* ev)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    if (nsteps < 1) return fail(RBL_E_ARG, "nsteps must be >= 1");
    if (!c->run.valid)
        return fail(RBL_E_STATE, "rbl_continue needs a completed rbl_step or rbl_continue on this context "
                                 "and no call since that loaded positions or drew batches");
    const RbRun r{c->run.P, c->run.seed, c->run.K, c->run.dt, c->run.full, c->run.end_step};
    // the starting state in caller order, for a repeat after an overflow
    if (!c->d_ckpt) RBL_TRY(dalloc(&c->d_ckpt, 6 * (size_t)c->n));
    {
        IoArgs io = io_args(c, false);
        io.pos_out = c->d_ckpt;
        io.vel_out = c->d_ckpt + 3 * c->n;
        k_scatter_out<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(io);
        HIP_TRY(hipGetLastError());
    }
    for (int attempt = 0; attempt < 3; ++attempt) {
        bool overflow = false;
        c->run.attempts = attempt + 1;
        // the repeat rebuilds at its first step from the checkpoint
        const rbl_status st = md_run(c, c->d_ckpt, c->d_ckpt + 3 * c->n, pos, vel, force, nsteps, r.dt, r.P,
                                     r.seed, r.step0, r.K, r.full, ev, attempt == 0, overflow);
        if (st < 0 || !overflow) return st;
        RBL_TRY(grow_after_overflow(c, r.full));
    }
    return fail(RBL_E_CAPACITY, "neighbour rows kept overflowing their capacity");
}

rbl_status rbl_last_run(rbl_ctx* c, int32_t* attempts, int64_t* end_step, int32_t* resumable, int64_t* builds,
                        int64_t* build_step)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    if (attempts) *attempts = c->run.attempts;
    if (end_step) *end_step = c->run.end_step;
    if (resumable) *resumable = c->run.valid ? 1 : 0;
    if (builds) *builds = c->run.builds;
    if (build_step) *build_step = c->run.build_step;
    return RBL_OK;
}

rbl_status rbl_row_counts(rbl_ctx* c, int64_t nrows, const int64_t* rows, int64_t* counts)
{
    if (!c || !counts || nrows < 0) return fail(RBL_E_ARG, "bad argument");
    if (!c->built) return fail(RBL_E_STATE, "no list build");
    std::vector<int64_t> h_rows;
    if (!rows) {
        nrows = c->n;
        h_rows.resize(c->n);
        for (int64_t i = 0; i < c->n; ++i) h_rows[i] = i;
    } else {
        h_rows.assign(rows, rows + nrows);
        for (auto r : h_rows)
            if (r < 0 || r >= c->n) return fail(RBL_E_ARG, "row ID out of range");
    }
    if (nrows == 0) return RBL_OK;
    int64_t* d_rows = nullptr;
    int64_t* d_cnt = nullptr;
    RBL_TRY(dalloc(&d_rows, nrows));
    rbl_status st = dalloc(&d_cnt, nrows);
    if (st < 0) {
        dfree(d_rows);
        return st;
    }
    (void)hipMemcpyAsync(d_rows, h_rows.data(), sizeof(int64_t) * nrows, hipMemcpyHostToDevice, c->ls);
    for (int q = 0; q < 3; ++q) {
        const bool valid = q == 1 ? c->shell_counts : ((c->built_mask >> q) & 1) != 0;
        const int* len = valid ? c->d_len[q] : (q == 1 && c->stencil && c->pop_valid ? c->d_nI : nullptr);
        k_row_counts<<<grid_for(nrows), kBlock, 0, c->ls>>>(d_rows, nrows, c->d_slot_of_id, len, d_cnt);
        (void)hipMemcpyAsync(counts + q * nrows, d_cnt, sizeof(int64_t) * nrows, hipMemcpyDeviceToHost,
                             c->ls);
    }
    hipError_t e = hipStreamSynchronize(c->ls);
    dfree(d_rows);
    dfree(d_cnt);
    if (e != hipSuccess) return fail(RBL_E_HIP, hipGetErrorString(e));
    return RBL_OK;
}

rbl_status rbl_export_lists(rbl_ctx* c, int64_t nrows, const int64_t* rows, const int64_t* core_off,
                            int32_t* core_idx, const int64_t* shell_off, int32_t* shell_idx,
                            const int64_t* full_off, int32_t* full_idx)
{
    if (!c || nrows < 0) return fail(RBL_E_ARG, "bad argument");
    if (!c->built) return fail(RBL_E_STATE, "no list build");
    std::vector<int64_t> h_rows;
    if (!rows) {
        nrows = c->n;
        h_rows.resize(c->n);
        for (int64_t i = 0; i < c->n; ++i) h_rows[i] = i;
    } else {
        h_rows.assign(rows, rows + nrows);
        for (auto r : h_rows)
            if (r < 0 || r >= c->n) return fail(RBL_E_ARG, "row ID out of range");
    }
    if (nrows == 0) return RBL_OK;
    const int64_t* offs[3] = {core_off, shell_off, full_off};
    int32_t* outs[3] = {core_idx, shell_idx, full_idx};
    int64_t* d_rows = nullptr;
    RBL_TRY(dalloc(&d_rows, nrows));
    (void)hipMemcpyAsync(d_rows, h_rows.data(), sizeof(int64_t) * nrows, hipMemcpyHostToDevice, c->ls);
    rbl_status st = RBL_OK;
    for (int q = 0; q < 3 && st == RBL_OK; ++q) {
        if (!outs[q]) continue;
        if (!offs[q]) {
            st = fail(RBL_E_ARG, "offsets missing for a requested list");
            break;
        }
        if (!((c->built_mask >> q) & 1)) {
            st = fail(RBL_E_STATE, "list was not built");
            break;
        }
        const int64_t total = offs[q][nrows];
        int64_t* d_off = nullptr;
        int* d_out = nullptr;
        st = dalloc(&d_off, nrows + 1);
        if (st < 0) break;
        st = dalloc(&d_out, std::max<int64_t>(total, 1));
        if (st < 0) {
            dfree(d_off);
            break;
        }
        (void)hipMemcpyAsync(d_off, offs[q], sizeof(int64_t) * (nrows + 1), hipMemcpyHostToDevice, c->ls);
        k_export_rows<<<grid_for(nrows), kBlock, 0, c->ls>>>(d_rows, nrows, c->d_slot_of_id,
                                                                 c->cur_perm(), c->d_list[q], c->d_len[q],
                                                                 c->cap[q], d_off, d_out);
        if (total > 0)
            (void)hipMemcpyAsync(outs[q], d_out, sizeof(int) * total, hipMemcpyDeviceToHost, c->ls);
        hipError_t e = hipStreamSynchronize(c->ls);
        dfree(d_off);
        dfree(d_out);
        if (e != hipSuccess) st = fail(RBL_E_HIP, hipGetErrorString(e));
    }
    dfree(d_rows);
    return st;
}

rbl_status rbl_export_batches(rbl_ctx* c, int P, uint64_t seed, uint64_t step, int64_t nrows,
                              const int64_t* rows, int32_t* batch, int32_t* count)
{
    if (!c || !batch || !count || nrows < 0) return fail(RBL_E_ARG, "bad argument");
    RBL_TRY(check_p(P));
    if (!c->built) return fail(RBL_E_STATE, "no list build");
    if (!c->stencil && !(c->built_mask & RBL_LIST_SHELL)) return fail(RBL_E_STATE, "no shell list built");
    for (int64_t k = 0; k < nrows; ++k)
        if (!rows || rows[k] < 0 || rows[k] >= c->n) return fail(RBL_E_ARG, "row ID out of range");
    c->run.valid = false;
    if (c->stencil) {
        RBL_TRY(ensure_batch(c, 1, P));
        if (!c->d_nI) RBL_TRY(dalloc(&c->d_nI, c->n_slots));
        RBL_TRY(launch_fused(c, P, seed, step, 1, nullptr, true));
    } else {
        RBL_TRY(predraw(c, P, seed, step, 1));
    }
    set_draw(c, (int64_t)step, 1, P);
    std::vector<int> h_batch((size_t)P * c->n_slots), h_perm(c->n_slots), h_slot(c->n), h_len(c->n_slots);
    HIP_TRY(hipMemcpyAsync(h_batch.data(), c->d_batch, sizeof(int) * h_batch.size(), hipMemcpyDeviceToHost,
                           c->ls));
    HIP_TRY(hipMemcpyAsync(h_perm.data(), c->cur_perm(), sizeof(int) * c->n_slots, hipMemcpyDeviceToHost,
                           c->ls));
    HIP_TRY(hipMemcpyAsync(h_slot.data(), c->d_slot_of_id, sizeof(int) * c->n, hipMemcpyDeviceToHost,
                           c->ls));
    HIP_TRY(hipMemcpyAsync(h_len.data(), c->stencil ? c->d_nI : c->d_len[1], sizeof(int) * c->n_slots,
                           hipMemcpyDeviceToHost, c->ls));
    HIP_TRY(hipStreamSynchronize(c->ls));
    for (int64_t k = 0; k < nrows; ++k) {
        const int slot = h_slot[rows[k]];
        const int cnt = std::min(h_len[slot], P);
        count[k] = cnt;
        for (int m = 0; m < P; ++m)
            batch[k * P + m] = m < cnt ? h_perm[h_batch[(size_t)slot * P + m]] : -1;
    }
    return RBL_OK;
}

rbl_status rbl_export_drawn_batches(rbl_ctx* c, int64_t nrows, const int64_t* rows, int32_t* batch,
                                    int32_t* count, int32_t* nsteps, int32_t* P_out, int64_t* step0)
{
    if (!c || nrows < 0 || (nrows > 0 && !rows)) return fail(RBL_E_ARG, "bad argument");
    if (nsteps) *nsteps = c->draw_steps;
    if (P_out) *P_out = c->draw_P;
    if (step0) *step0 = c->draw_step0;
    if (!batch && !count) return RBL_OK;
    if (!c->built || c->draw_steps == 0) return fail(RBL_E_STATE, "no stored batches (last build drew none)");
    if (!batch || !count) return fail(RBL_E_ARG, "batch and count are both required");
    for (int64_t k = 0; k < nrows; ++k)
        if (rows[k] < 0 || rows[k] >= c->n) return fail(RBL_E_ARG, "row ID out of range");
    const int P = c->draw_P, K = c->draw_steps;
    std::vector<int> h_batch((size_t)K * P * c->n_slots), h_perm(c->n_slots), h_slot(c->n), h_len(c->n_slots);
    HIP_TRY(hipMemcpyAsync(h_batch.data(), c->d_batch, sizeof(int) * h_batch.size(), hipMemcpyDeviceToHost,
                           c->ls));
    HIP_TRY(hipMemcpyAsync(h_perm.data(), c->cur_perm(), sizeof(int) * c->n_slots, hipMemcpyDeviceToHost,
                           c->ls));
    HIP_TRY(hipMemcpyAsync(h_slot.data(), c->d_slot_of_id, sizeof(int) * c->n, hipMemcpyDeviceToHost,
                           c->ls));
    HIP_TRY(hipMemcpyAsync(h_len.data(), c->stencil ? c->d_nI : c->d_len[1], sizeof(int) * c->n_slots,
                           hipMemcpyDeviceToHost, c->ls));
    HIP_TRY(hipStreamSynchronize(c->ls));
    for (int64_t k = 0; k < nrows; ++k) {
        const int slot = h_slot[rows[k]];
        const int cnt = std::min(h_len[slot], P);
        count[k] = cnt;
        for (int r = 0; r < K; ++r)
            for (int m = 0; m < P; ++m) {
                const int e = h_batch[((size_t)r * c->n_slots + slot) * P + m];
                batch[((size_t)r * nrows + k) * P + m] = m < cnt ? h_perm[e] : -1;
            }
    }
    return RBL_OK;
}

rbl_status rbl_export_binning(rbl_ctx* c, int32_t* ncell, int64_t* slot_of_id, int32_t* cell_count)
{
    if (!c || !ncell || !slot_of_id) return fail(RBL_E_ARG, "NULL argument");
    if (!c->built) return fail(RBL_E_STATE, "no list build");
    std::vector<int> h_slot(c->n);
    HIP_TRY(hipMemcpyAsync(h_slot.data(), c->d_slot_of_id, sizeof(int) * c->n, hipMemcpyDeviceToHost,
                           c->ls));
    if (cell_count)
        HIP_TRY(hipMemcpyAsync(cell_count, c->d_cell_count, sizeof(int) * c->n_cells, hipMemcpyDeviceToHost,
                               c->ls));
    HIP_TRY(hipStreamSynchronize(c->ls));
    for (int r = 0; r < c->R; ++r) {
        for (int a = 0; a < 3; ++a) ncell[3 * r + a] = c->h_rep[r].nc[a];
        for (int64_t i = c->id_base[r]; i < c->id_base[r] + c->rep_n[r]; ++i)
            slot_of_id[i] = h_slot[i] - c->slot_base[r];
    }
    return RBL_OK;
}

rbl_status rbl_sync(rbl_ctx* c)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    RBL_TRY(read_flags(c));
    const int nonfinite = c->h_flags[kFlagNonfinite];
    const int skin = c->h_flags[kFlagSkin];
    RBL_TRY(clear_flags(c));
    HIP_TRY(hipStreamSynchronize(c->ls));
    if (nonfinite) return fail(RBL_E_NONFINITE, "non-finite particle position");
    if (skin) {
        g_err = "a particle moved more than skin/2 within one list lifetime";
        return RBL_W_SKIN;
    }
    return RBL_OK;
}

rbl_status rbl_set_profiling(rbl_ctx* c, int on)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    RBL_TRY(resolve_events(c));
    c->profiling = on != 0;
    for (int k = 0; k < kKinds; ++k) {
        c->stat_launches[k] = 0;
        c->stat_ms[k] = 0.0;
    }
    return RBL_OK;
}

rbl_status rbl_kernel_stats(rbl_ctx* c, int kind, int64_t* launches, double* total_ms)
{
    if (!c || kind < 0 || kind >= kKinds || !launches || !total_ms) return fail(RBL_E_ARG, "bad argument");
    RBL_TRY(resolve_events(c));
    *launches = c->stat_launches[kind];
    *total_ms = c->stat_ms[kind];
    return RBL_OK;
}

rbl_status rbl_tuning(rbl_ctx* c, int32_t* lpp_rbl, int32_t* lpp_full, double* force_us)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    if (lpp_rbl) *lpp_rbl = c->lpp_rbl;
    if (lpp_full) *lpp_full = c->lpp_full;
    if (force_us)
        for (int k = 0; k < 2; ++k)
            for (int q = 0; q < 3; ++q) force_us[3 * k + q] = c->tune_us[k][q];
    return RBL_OK;
}

rbl_status rbl_core_filter(rbl_ctx* c, int32_t* used, double* force_us, double* mean_kept)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    if (used) *used = c->filt_last ? 1 : 0;
    if (force_us)
        for (int q = 0; q < 3; ++q) force_us[q] = c->filt_us[q];
    if (mean_kept) {
        *mean_kept = 0.0;
        if (c->filt_last && c->d_fcore_len) {
            std::vector<int> len((size_t)c->n_slots), perm((size_t)c->n_slots);
            HIP_TRY(hipMemcpyAsync(len.data(), c->d_fcore_len, sizeof(int) * c->n_slots, hipMemcpyDeviceToHost,
                                   c->stream));
            HIP_TRY(hipMemcpyAsync(perm.data(), c->cur_perm(), sizeof(int) * c->n_slots, hipMemcpyDeviceToHost,
                                   c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
            double sum = 0.0;
            int64_t cnt = 0;
            for (int64_t s = 0; s < c->n_slots; ++s)
                if (perm[s] >= 0) {
                    sum += len[s];
                    ++cnt;
                }
            *mean_kept = cnt ? sum / (double)cnt : 0.0;
        }
    }
    return RBL_OK;
}

rbl_status rbl_launch_modes(rbl_ctx* c, int32_t* persistent_rbl, int32_t* persistent_full, double* force_us)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    if (persistent_rbl) *persistent_rbl = c->persist[0] ? 1 : 0;
    if (persistent_full) *persistent_full = c->persist[1] ? 1 : 0;
    if (force_us)
        for (int k = 0; k < 2; ++k)
            for (int q = 0; q < 2; ++q) force_us[2 * k + q] = c->persist_us[k][q];
    return RBL_OK;
}

rbl_status rbl_info(rbl_ctx* c, int64_t* n_slots, int32_t* cap_core, int32_t* cap_shell, int32_t* cap_full)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    if (n_slots) *n_slots = c->n_slots;
    if (cap_core) *cap_core = c->cap[0];
    if (cap_shell) *cap_shell = c->cap[1];
    if (cap_full) *cap_full = c->cap[2];
    return RBL_OK;
}

// ---- thermostat and observables (Sec. II Langevin dynamics, Sec. III) ----

rbl_status rbl_set_thermostat(rbl_ctx* c, double gamma, const double* kT)
{
    if (!c) return fail(RBL_E_ARG, "NULL context");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(RBL_E_ARG, "gamma must be finite and >= 0");
    if (gamma > 0.0 && !kT) return fail(RBL_E_ARG, "kT is required when gamma > 0");
    if (kT)
        for (int r = 0; r < c->R; ++r)
            if (!(kT[r] >= 0.0) || !std::isfinite(kT[r])) return fail(RBL_E_ARG, "kT must be finite and >= 0");
    c->gamma = gamma;
    if (kT) c->kT.assign(kT, kT + c->R);
    return RBL_OK;
}

rbl_status rbl_unwrap(rbl_ctx* c, const double* pos, double* out)
{
    if (!c || !pos || !out) return fail(RBL_E_ARG, "NULL argument");
    if (c->r_c <= 0.0) return fail(RBL_E_STATE, "rbl_unwrap needs the boxes of an rbl_build");
    k_unwrap<<<grid_for(c->n), kBlock, 0, c->ls>>>(c->d_rep, c->d_id_rep, pos, c->d_img, c->n, out);
    HIP_TRY(hipGetLastError());
    return RBL_OK;
}


rbl_status rbl_msd(rbl_ctx* c, const double* a, const double* b, double* out)
{
    if (!c || !a || !b || !out) return fail(RBL_E_ARG, "NULL argument");
    if (c->r_c <= 0.0) return fail(RBL_E_STATE, "rbl_msd needs the replica table of an rbl_build");
    return mean_sq(c, a, b, out);
}

rbl_status rbl_rdf(rbl_ctx* c, const double* pos, double r_max, int nbins, uint64_t* counts)
{
    if (!c || !pos || !counts) return fail(RBL_E_ARG, "NULL argument");
    if (!c->built) return fail(RBL_E_STATE, "rbl_rdf needs a list build first");
    // the histogram walks +-2 cells of the build grid: up to the smallest
    // pair cut-off with particle types
    if (!(r_max > 0.0) || !(r_max <= c->r_c * c->sig_min))
        return fail(RBL_E_ARG, c->typed ? "r_max must be in (0, r_c sigma_min]" : "r_max must be in (0, r_c]");
    if (nbins < 1 || nbins > (1 << 20)) return fail(RBL_E_ARG, "nbins must be in 1 .. 2^20");
    c->run.valid = false;
    IoArgs io = io_args(c, false);
    io.pos_in = pos;
    k_load_positions<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(io);
    HIP_TRY(hipGetLastError());
    RdfArgs a;
    a.rep = c->d_rep;
    a.slice_rep = c->d_slice_rep;
    a.perm = c->cur_perm();
    a.xs = c->cur_xs();
    a.xb = c->d_xb;
    a.cell_start = c->d_cell_start;
    a.cell_count = c->d_cell_count;
    a.n_slots = c->n_slots;
    a.n_slices = c->n_slices;
    a.dr = r_max / (double)nbins;
    {
        const double e = (double)nbins * a.dr;
        a.top2 = e * e;
    }
    a.nbins = nbins;
    a.counts = reinterpret_cast<unsigned long long*>(counts);
    k_rdf<<<grid_for(c->n_slots), kBlock, 0, c->ls>>>(a);
    HIP_TRY(hipGetLastError());
    return RBL_OK;
}

rbl_status rbl_thermo(rbl_ctx* c, const double* vel, const double* ev, double* out)
{
    if (!c || !ev || !out) return fail(RBL_E_ARG, "NULL argument");
    if (c->r_c <= 0.0) return fail(RBL_E_STATE, "rbl_thermo needs the boxes of an rbl_build");
    if (c->cfg.shift || c->cfg.pair != RBL_PAIR_LJ)
        return fail(RBL_E_STATE, "rbl_thermo needs the unshifted LJ pair (cfg.shift = 0, RBL_PAIR_LJ)");
    std::vector<double> h_ev(2 * (size_t)c->R), h_msq(c->R, 0.0);
    double* d_msq = nullptr;
    if (vel) {
        RBL_TRY(dalloc(&d_msq, (size_t)c->R));
        const rbl_status st = mean_sq(c, vel, nullptr, d_msq);
        if (st < 0) {
            dfree(d_msq);
            return st;
        }
        (void)hipMemcpyAsync(h_msq.data(), d_msq, sizeof(double) * c->R, hipMemcpyDeviceToHost, c->ls);
    }
    (void)hipMemcpyAsync(h_ev.data(), ev, sizeof(double) * 2 * c->R, hipMemcpyDeviceToHost, c->ls);
    const hipError_t e = hipStreamSynchronize(c->ls);
    dfree(d_msq);
    if (e != hipSuccess) return fail(RBL_E_HIP, hipGetErrorString(e));
    // mean-field tails beyond r_c (sigma = epsilon = 1):
    //   u_tail = (8/3) pi rho (r_c^-9 / 3 - r_c^-3),
    //   p_tail = (16/3) pi rho^2 (2 r_c^-9 / 3 - r_c^-3)
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double c3 = 1.0 / (c->r_c * c->r_c * c->r_c);
    const double c9 = c3 * c3 * c3;
    for (int r = 0; r < c->R; ++r) {
        const DevReplica& R = c->h_rep[r];
        const double V = R.L[0] * R.L[1] * R.L[2];
        const double nr = (double)c->rep_n[r];
        const double rho = nr / V;
        const double ut = 8.0 / 3.0 * M_PI * rho * (c9 / 3.0 - c3);
        const double pt = 16.0 / 3.0 * M_PI * rho * rho * (2.0 * c9 / 3.0 - c3);
        const double pw = h_ev[2 * r + 1] / (3.0 * V);
        const double tk = (vel && c->rep_n[r] > 1) ? h_msq[r] * nr / (3.0 * nr - 3.0) : nan;
        out[4 * r + 0] = h_ev[2 * r] / nr + ut;
        out[4 * r + 1] = c->gamma > 0.0 ? rho * c->kT[r] + pw + pt : nan;
        out[4 * r + 2] = tk;
        out[4 * r + 3] = rho * tk + pw + pt;
    }
    return RBL_OK;
}

}  // extern "C"
