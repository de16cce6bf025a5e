// HIP kernels of the RBL force path (gfx950, wave64).
//
// Data layout in HBM (n_slots = particles padded per replica to 64):
//   xs        double4[n_slots]   cell-sorted positions (x, y, z, charge)
//   vs, f     double[3][n_slots] cell-sorted velocities / raw forces (SoA)
//   perm      int[n_slots]       slot -> caller ID (-1 = padding slot)
//   lists     int[n_slices][cap][64] sliced ELL, partner slots in row order
//   len       int[n_slots]       row lengths
//   batch     int[K][n_slots][P] pre-drawn shell partners (slots)
//   partial   double[5][n_slices] per-wavefront sums (Fx, Fy, Fz, U, W)
#pragma once

#include "device.h"

namespace rbl {

enum { kSrcCaller = 0, kSrcSorted = 1 };
enum { kShellNone = 0, kShellInline = 1, kShellPredraw = 2 };
enum { kIntFirst = 0, kIntMid = 1, kIntLast = 2 };
enum { kFlagOverflow = 0, kFlagMaxCore = 1, kFlagMaxShell = 2, kFlagMaxFull = 3,
       kFlagNonfinite = 4, kFlagSkin = 5, kFlagBadSlot = 6, kFlagStencil = 7, kNumFlags = 8 };
// pair term of the force kernels: LJ of eq. (1); LJ plus the erfc term of
// charges; LJ with per-type parameters and radii
enum { kPairLJ = 0, kPairErfc = 1, kPairTyped = 2 };
// radius zone a force sum tests its partners against
enum { kZoneCore = 0, kZoneShell = 1, kZoneFull = 2 };

// Particle types (Sec. II: systems whose interaction lengths differ).  A
// particle's type travels in the w word of its position record (xs: as a
// double, xq: as FP32 bits).  Pair (a, b) has its own LJ constants, its core
// radius r_s sigma_ab and cut-off r_c sigma_ab; the cell grid is sized by the
// smallest cut-off and a centre of type a searches the cells within h[a] of
// its own.
constexpr int kMaxTypes = 4;

struct TypePair {
    double eps24, eps4, sig2;          // 24 eps_ab, 4 eps_ab, sigma_ab^2
    double rs2, rc2, uc;               // (r_s sigma_ab)^2, (r_c sigma_ab)^2, energy at the cut-off
    double thr_core, thr_in, thr_out;  // list thresholds: squared radii with the skin
    double filt2;                      // core-row filter: (r_s sigma_ab + skin/2)^2
};

struct TypeTable {
    TypePair p[kMaxTypes * kMaxTypes];  // pair (a, b) at a * kMaxTypes + b
    int h[kMaxTypes];                   // stencil half-width in cells of centre type a
    int n_types;
    int pad;
};

// type of a particle from the w word of its record (masked into the table)
__device__ __forceinline__ int type_of(double w) { return (int)w & (kMaxTypes - 1); }

// Block -> work-tile map.  Blocks are dispatched to the 8 XCDs round-robin
// (block b to XCD b % 8); this map hands every XCD chunks of kXcdChunk
// consecutive tiles, the chunks dealt round-robin too, so that an XCD's L2
// sees neighbouring tiles while the load stays balanced when the work is
// concentrated in one part of the tile range (a liquid slab, one dense
// replica).  Tiles past the last whole round map to themselves.
constexpr int64_t kXcdChunk = 16;

__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb)
{
    const int64_t full = nb / (8 * kXcdChunk) * (8 * kXcdChunk);
    if (b >= full) return b;
    const int64_t x = b & 7;   // XCD of block b
    const int64_t r = b >> 3;  // its rank among that XCD's blocks
    return ((r / kXcdChunk) * 8 + x) * kXcdChunk + r % kXcdChunk;
}

// Raises *p to v.  Every wavefront reports its longest row here, and atomics
// on one address serialise in L2, so the atomic is issued only when v
// exceeds the value already stored (a relaxed read; the maximum grows a few
// times per launch).
__device__ __forceinline__ void raise_max(int* p, int v)
{
    if (v > __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(p, v);
}

// Sets *p to 1 unless it is already set (same reasoning as raise_max).
__device__ __forceinline__ void raise_flag(int* p)
{
    if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) atomicOr(p, 1);
}

__global__ void k_fill_i32(int* p, int64_t n, int v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Rebuilds decided on the device.  When lists are rebuilt on displacement,
// every step queues the binning and list-build kernels with the address of
// a gate word that the step's integrator sets when a rebuild is due; they
// return at once while it is 0.  A null gate means "always run".
__device__ __forceinline__ bool gated_off(const uint64_t* gate)
{
    return gate != nullptr && *gate == 0;
}

__global__ void k_clear_counts(int* p, int64_t n, const uint64_t* gate)
{
    if (gated_off(gate)) return;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------------------
// Binning: cell index of every particle (positions wrapped into the box),
// counting-sort histogram.  Source is either the caller's SoA arrays (one
// thread per ID) or the current cell-sorted state (one thread per slot).
struct BinArgs {
    const DevReplica* rep;
    const int* id_rep;
    const int* slice_rep;
    const double* pos;     // caller SoA [3][n]
    const double4* xs;     // sorted source
    const int* perm_old;   // sorted source: slot -> ID
    const double* xb;      // sorted source: positions at the previous build [3][n_slots]
    double half_skin2;     // (skin/2)^2
    int64_t n;
    int64_t n_src;
    int* cell_of_src;
    int* rank_of_src;
    int* cell_count;
    int* flags;
    const uint64_t* gate;  // rebuild gate (null: always run)
    // gated rebuilds of the sorted state keep one buffer set: the counting
    // pass saves every slot's position, velocity and ID here first, the
    // scatter and the gather read them back (null: no save)
    double4* xs_save;
    const double* vs_src;  // [3][n_src]
    double* vs_save;
    int* perm_save;
};

// Cell of every source particle and its rank within the cell (a unique
// index; the in-cell order is fixed later by k_cell_sort).  A cell-sorted
// source has runs of equal cells along the wavefront, so there one lane per
// distinct cell adds the run's size to the histogram and the others take
// consecutive ranks after it: a handful of atomics per wavefront instead of
// one per particle.
template <int SRC>
__global__ __launch_bounds__(256) void k_bin_count(BinArgs a)
{
    if (gated_off(a.gate)) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool live = s < a.n_src;
    int cell = -1;
    if (live) {
        int r;
        double x[3];
        if (SRC == kSrcCaller) {
            r = a.id_rep[s];
            x[0] = a.pos[s];
            x[1] = a.pos[a.n + s];
            x[2] = a.pos[2 * a.n + s];
        } else {
            live = a.perm_old[s] >= 0;
            r = a.slice_rep[s >> 6];
            const double4 p = a.xs[s];
            x[0] = p.x;
            x[1] = p.y;
            x[2] = p.z;
            if (a.xs_save) {
                a.xs_save[s] = p;
                a.perm_save[s] = a.perm_old[s];
                a.vs_save[s] = a.vs_src[s];
                a.vs_save[a.n_src + s] = a.vs_src[a.n_src + s];
                a.vs_save[2 * a.n_src + s] = a.vs_src[2 * a.n_src + s];
            }
            if (live) {
                // skin monitor: displacement over the list lifetime that ends here
                const double dx = p.x - a.xb[s];
                const double dy = p.y - a.xb[a.n_src + s];
                const double dz = p.z - a.xb[2 * a.n_src + s];
                if (dx * dx + dy * dy + dz * dz > a.half_skin2) raise_flag(&a.flags[kFlagSkin]);
            }
        }
        if (live) {
            const DevReplica& R = a.rep[r];
            int c[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (!isfinite(x[d])) {
                    raise_flag(&a.flags[kFlagNonfinite]);
                    x[d] = 0.0;
                }
                const double w = wrap_coord(x[d], R.L[d], R.inv[d]);
                int k = (int)floor(w * R.cscale[d]);
                k = k < 0 ? 0 : (k > R.nc[d] - 1 ? R.nc[d] - 1 : k);
                c[d] = k;
            }
            cell = (int)(R.cell_base + ((int64_t)c[2] * R.nc[1] + c[1]) * R.nc[0] + c[0]);
        }
        a.cell_of_src[s] = cell;
    }
    if (SRC == kSrcCaller) {
        if (live) a.rank_of_src[s] = atomicAdd(&a.cell_count[cell], 1);
        return;
    }
    const int lane = threadIdx.x & 63;
    uint64_t todo = __ballot(live);
    int rank = 0;
    while (todo) {  // one pass per distinct cell of the wavefront
        const int lead = (int)__builtin_ctzll(todo);
        const int lc = __builtin_amdgcn_readlane(cell, lead);
        const uint64_t same = __ballot(cell == lc) & todo;
        int base = 0;
        if (lane == lead) base = atomicAdd(&a.cell_count[lc], (int)__popcll(same));
        base = __builtin_amdgcn_readlane(base, lead);
        if ((same >> lane) & 1ull) rank = base + (int)mbcnt(same);
        todo &= ~same;
    }
    if (live) a.rank_of_src[s] = rank;
}

// Exclusive scan of the cell histogram (three passes, 2048 cells per block),
// then shifted by each replica's slot offset so that replica r starts at its
// 64-aligned slot base.
constexpr int kScanPerThread = 8;
constexpr int kScanBlock = 256;
constexpr int kScanTile = kScanBlock * kScanPerThread;

__device__ __forceinline__ int block_excl_scan(int v, int* lds_waves, int& total)
{
    const int incl = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    if (lane == 63) lds_waves[w] = incl;
    __syncthreads();
    int off = 0, tot = 0;
    for (int q = 0; q < nw; ++q) {
        const int t = lds_waves[q];
        if (q < w) off += t;
        tot += t;
    }
    __syncthreads();
    total = tot;
    return incl - v + off;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const int* cnt, int64_t n, int* tile_sum,
                                                           const uint64_t* gate)
{
    if (gated_off(gate)) return;
    __shared__ int lds[16];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k)
        if (base + k < n) s += cnt[base + k];
    int total;
    block_excl_scan(s, lds, total);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

// One block of 1024 threads scans up to 1024*8 tile sums (exclusive, in place).
__global__ __launch_bounds__(1024) void k_scan_tile_sums(int* tile_sum, int ntiles, const uint64_t* gate)
{
    if (gated_off(gate)) return;
    __shared__ int lds[16];
    const int base = threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = base + k < ntiles ? tile_sum[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_excl_scan(s, lds, total);
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        if (base + k < ntiles) tile_sum[base + k] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final(const int* cnt, int64_t n,
                                                           const int* tile_sum, const int* cell_rep,
                                                           const DevReplica* rep, int* start,
                                                           const uint64_t* gate)
{
    if (gated_off(gate)) return;
    __shared__ int lds[16];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPerThread;
    int v[kScanPerThread];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        v[k] = base + k < n ? cnt[base + k] : 0;
        s += v[k];
    }
    int total;
    int run = block_excl_scan(s, lds, total) + tile_sum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanPerThread; ++k) {
        const int64_t c = base + k;
        if (c < n) {
            // replica r starts at its slot base (no shift without a table)
            start[c] = cell_rep ? run + (int)(rep[cell_rep[c]].slot_base - rep[cell_rep[c]].id_base) : run;
        }
        run += v[k];
    }
}

template <int SRC>
__global__ __launch_bounds__(256) void k_bin_scatter(BinArgs a, const int* cell_start,
                                                     int* perm_new, int* src_of_slot,
                                                     int64_t n_slots)
{
    if (gated_off(a.gate)) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_src) return;
    const int cell = a.cell_of_src[s];
    if (cell < 0) return;
    const int id = SRC == kSrcCaller ? (int)s : a.perm_old[s];
    const int64_t slot = (int64_t)cell_start[cell] + a.rank_of_src[s];
    if (slot < 0 || slot >= n_slots) {
        atomicOr(&a.flags[kFlagBadSlot], 1);
        return;
    }
    perm_new[slot] = id;
    src_of_slot[slot] = (int)s;
}

// Within each cell, order particles by ID (insertion sort; cells hold a
// handful of particles).  Makes the slot order independent of atomic order.
__global__ __launch_bounds__(256) void k_cell_sort(const int* cell_start, const int* cell_count,
                                                   int64_t n_cells, int64_t n_slots, int* perm,
                                                   int* src_of_slot, int* flags, const uint64_t* gate)
{
    if (gated_off(gate)) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int b = cell_start[c];
    const int m = cell_count[c];
    if (b < 0 || (int64_t)b + m > n_slots) {
        atomicOr(&flags[kFlagBadSlot], 4);
        return;
    }
    for (int i = 1; i < m; ++i) {
        const int key = perm[b + i];
        const int val = src_of_slot[b + i];
        int j = i - 1;
        while (j >= 0 && perm[b + j] > key) {
            perm[b + j + 1] = perm[b + j];
            src_of_slot[b + j + 1] = src_of_slot[b + j];
            --j;
        }
        perm[b + j + 1] = key;
        src_of_slot[b + j + 1] = val;
    }
}

struct GatherArgs {
    const DevReplica* rep;
    const int* slice_rep;
    const int* perm;          // new slot -> ID
    const int* src_of_slot;
    const double* pos;        // caller SoA
    const double* vel;        // caller SoA (may be null)
    const double* charges;    // caller order (may be null)
    const double4* xs_old;
    const double* vs_old;
    int64_t n;
    int64_t n_src;
    int64_t n_slots;
    int* flags;
    double4* xs;
    double* vs;               // may be null
    double* xb;               // positions at the build, [3][n_slots] (skin monitor)
    int* slot_of_id;
    int* img_delta;           // may be null: [3][n] box lengths taken off by the wrap
    const uint64_t* gate;     // rebuild gate (null: always run)
    int4* xq;                 // may be null: fixed-point copy of xs (mixed-precision forces)
};

// Fixed-point coordinate for the mixed-precision force kernels: x / L mod 1
// in units of 2^-32 (one rounding, at most half a unit, i.e. L 2^-33).  The
// difference of two such words taken as a signed 32-bit integer is the
// minimum-image displacement in the same units, so a neighbour costs one
// 16-byte load (three words and the charge as FP32 bits) and no image
// arithmetic, while the displacement error stays L 2^-32 whatever the box.
__device__ __forceinline__ int fixq(double x, double inv)
{
    const double t = x * inv;
    const double f = t - floor(t);  // [0, 1]; 1 wraps to 0 below
    return (int)(uint32_t)(uint64_t)rint(f * 4294967296.0);
}

__device__ __forceinline__ int4 fixq4(double x, double y, double z, double q, const DevReplica& R)
{
    return make_int4(fixq(x, R.inv[0]), fixq(y, R.inv[1]), fixq(z, R.inv[2]), __float_as_int((float)q));
}

template <int SRC, bool VEL>
__global__ __launch_bounds__(256) void k_gather(GatherArgs a)
{
    if (gated_off(a.gate)) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_slots) return;
    const int id = a.perm[s];
    if (id < 0) {
        a.xs[s] = make_double4(0.0, 0.0, 0.0, 0.0);
        if (a.xq) a.xq[s] = make_int4(0, 0, 0, 0);
        if (VEL) {
            a.vs[s] = 0.0;
            a.vs[a.n_slots + s] = 0.0;
            a.vs[2 * a.n_slots + s] = 0.0;
        }
        return;
    }
    const DevReplica& R = a.rep[a.slice_rep[s >> 6]];
    const int src = a.src_of_slot[s];
    if (src < 0 || src >= a.n_src) {
        atomicOr(&a.flags[kFlagBadSlot], 8);
        return;
    }
    double x[3];
    double q;
    if (SRC == kSrcCaller) {
        x[0] = a.pos[src];
        x[1] = a.pos[a.n + src];
        x[2] = a.pos[2 * a.n + src];
        q = a.charges ? a.charges[id] : 0.0;
    } else {
        const double4 p = a.xs_old[src];
        x[0] = p.x;
        x[1] = p.y;
        x[2] = p.z;
        q = p.w;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (isfinite(x[d])) {
            // the wrap of wrap_coord, keeping its box count for the
            // continuous trajectory
            const double k = floor(x[d] * R.inv[d]);
            x[d] = fma(-k, R.L[d], x[d]);
            if (a.img_delta && k != 0.0) a.img_delta[d * a.n + id] += (int)k;
        } else {
            x[d] = 0.0;
        }
        a.xb[d * a.n_slots + s] = x[d];
    }
    a.xs[s] = make_double4(x[0], x[1], x[2], q);
    if (a.xq) a.xq[s] = fixq4(x[0], x[1], x[2], q, R);
    if (VEL) {
        if (SRC == kSrcCaller) {
            a.vs[s] = a.vel[src];
            a.vs[a.n_slots + s] = a.vel[a.n + src];
            a.vs[2 * a.n_slots + s] = a.vel[2 * a.n + src];
        } else {
            a.vs[s] = a.vs_old[src];
            a.vs[a.n_slots + s] = a.vs_old[a.n_slots + src];
            a.vs[2 * a.n_slots + s] = a.vs_old[2 * a.n_slots + src];
        }
    }
    a.slot_of_id[id] = (int)s;
}

// ---------------------------------------------------------------------------
// Core / shell / full list build.  One wavefront per centre cell: the lanes
// walk the candidates of the 5x5x5 cell stencil (up to 50 runs of
// consecutive slots, in increasing slot order) 64 at a time, and every
// candidate is tested against each particle of the centre cell, whose
// position is broadcast from a lane with readlane.  Ballot + mbcnt compaction
// appends the accepted candidates to each row in candidate order, so rows
// come out in slot order with no sort.
struct BuildArgs {
    const DevReplica* rep;
    const int* cell_rep;
    const int* cell_start;
    const int* cell_count;
    const double4* xs;
    int64_t n_cells;
    int64_t n_slots;
    double thr_core, thr_shell_in, thr_out;  // squared distances
    int cap_core, cap_shell, cap_full;
    int* core;
    int* shell;
    int* full;
    int* core_len;
    int* shell_len;
    int* full_len;
    int* flags;
    const uint64_t* gate;      // rebuild gate (null: always run)
    const TypeTable* types;    // particle types (k_build_typed), else null
    // the MD loop's builds record themselves: mark[0] = step of the build,
    // mark[1] += 1 (null: not recorded); the step is *mark_step_dev +
    // mark_step, or mark_step alone without a device counter
    uint64_t* mark;
    uint64_t mark_step;
    const uint64_t* mark_step_dev;
};

__device__ __forceinline__ void record_build(const BuildArgs& a)
{
    if (a.mark && blockIdx.x == 0 && threadIdx.x == 0) {
        a.mark[0] = a.mark_step_dev ? *a.mark_step_dev + a.mark_step : a.mark_step;
        a.mark[1] += 1;
    }
}

// Along one axis of nc cells, the stencil of cells within +-2 of c, sorted
// by wrapped coordinate, as at most two runs [p0, p0+l0) and [p1, p1+l1).
struct AxisRuns {
    int p0, l0, p1, l1;
};

__device__ __forceinline__ AxisRuns axis_runs(int c, int nc, int h = 2)
{
    AxisRuns a;
    if (nc <= 2 * h + 1) {
        a.p0 = 0;
        a.l0 = nc;
        a.p1 = 0;
        a.l1 = 0;
        return a;
    }
    const int lo = c - h, hi = c + h;
    if (lo >= 0 && hi <= nc - 1) {
        a.p0 = lo;
        a.l0 = 2 * h + 1;
        a.p1 = 0;
        a.l1 = 0;
    } else if (lo < 0) {
        a.p0 = 0;
        a.l0 = hi + 1;
        a.p1 = lo + nc;
        a.l1 = nc - (lo + nc);
    } else {
        a.p0 = 0;
        a.l0 = hi - nc + 1;
        a.p1 = lo;
        a.l1 = nc - lo;
    }
    return a;
}

__device__ __forceinline__ int axis_cell(const AxisRuns& a, int k)
{
    return k < a.l0 ? a.p0 + k : a.p1 + (k - a.l0);
}

struct AxisRunsS {
    int p0, l0, p1, l1;
    int s0, s1;  // image shift (in box lengths, added to x_i - x_j) of run 0 / run 1
};

__device__ __forceinline__ AxisRunsS axis_runs_s(int c, int nc, int h = 2)
{
    AxisRunsS a;
    const AxisRuns b = axis_runs(c, nc, h);
    a.p0 = b.p0;
    a.l0 = b.l0;
    a.p1 = b.p1;
    a.l1 = b.l1;
    a.s0 = 0;
    a.s1 = 0;
    if (nc > 2 * h + 1) {
        const int lo = c - h, hi = c + h;
        if (lo < 0) {
            a.s1 = 1;   // cells lo+nc..nc-1 are images one box below
        } else if (hi > nc - 1) {
            a.s0 = -1;  // cells 0..hi-nc are images one box above
        }
    }
    return a;
}

__device__ __forceinline__ int axis_shift(const AxisRunsS& a, int k)
{
    return k < a.l0 ? a.s0 : a.s1;
}

// Wave masks of per-lane FP64 compares (llvm.amdgcn.fcmp; an ordered
// predicate, so a NaN compares false).
__device__ __forceinline__ uint64_t cmp_lt_mask(double x, double t)
{
    return __builtin_amdgcn_fcmp(x, t, 4);  // FCMP_OLT
}

__device__ __forceinline__ uint64_t cmp_ge_mask(double x, double t)
{
    return __builtin_amdgcn_fcmp(x, t, 3);  // FCMP_OGE
}

constexpr int kNoShift = 1 | (1 << 2) | (1 << 4);  // image-shift code of no shift

__device__ __forceinline__ double bcast(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int shfl_i32(int v, int src_lane)
{
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}

// Ordering of one wavefront's LDS accesses across its lanes: earlier reads
// done before the writes, the writes visible before the reads after them.
__device__ __forceinline__ void lds_fence_before_write()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void lds_fence_after_write()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool COUNT_ONLY, bool WC, bool WS, bool WF>
__global__ __launch_bounds__(256) void k_build(BuildArgs a)
{
    __shared__ double4 s_ctr[4][64];  // the group's centre positions, per wavefront
    if (gated_off(a.gate)) return;
    if (!COUNT_ONLY) record_build(a);
    const int lane = threadIdx.x & 63;
    const int64_t cell = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (cell >= a.n_cells) return;
    const int m = a.cell_count[cell];
    if (m == 0) return;
    const int i0 = a.cell_start[cell];
    if (i0 < 0 || (int64_t)i0 + m > a.n_slots) {
        if ((threadIdx.x & 63) == 0) atomicOr(&a.flags[kFlagBadSlot], 2);
        return;
    }
    const DevReplica& R = a.rep[a.cell_rep[cell]];
    const int64_t lc = cell - R.cell_base;
    const int cx = (int)(lc % R.nc[0]);
    const int cy = (int)((lc / R.nc[0]) % R.nc[1]);
    const int cz = (int)(lc / ((int64_t)R.nc[0] * R.nc[1]));
    const AxisRunsS ax = axis_runs_s(cx, R.nc[0]);
    const AxisRunsS ay = axis_runs_s(cy, R.nc[1]);
    const AxisRunsS az = axis_runs_s(cz, R.nc[2]);
    const int ny_s = ay.l0 + ay.l1;
    const int nz_s = az.l0 + az.l1;
    // with at least 7 cells per axis the periodic image of every run is
    // known, and x_i - x_j plus that image's shift (0 or -+L) is exactly
    // the minimum-image displacement (as in the fused build)
    const bool SHIFT = R.nc[0] >= 7 && R.nc[1] >= 7 && R.nc[2] >= 7;

    // lane q describes run q = ((z * ny_s) + y) * 2 + xrun of the stencil:
    // slot start, length and image-shift code
    int rstart = 0, rlen = 0, rshift = kNoShift;
    {
        const int q = lane;
        const int zi = q / (2 * ny_s);
        const int yi = (q >> 1) % ny_s;
        const int xr = q & 1;
        if (zi < nz_s) {
            const int zc = axis_cell(AxisRuns{az.p0, az.l0, az.p1, az.l1}, zi);
            const int yc = axis_cell(AxisRuns{ay.p0, ay.l0, ay.p1, ay.l1}, yi);
            const int px = xr == 0 ? ax.p0 : ax.p1;
            const int lx = xr == 0 ? ax.l0 : ax.l1;
            if (lx > 0) {
                const int64_t row = R.cell_base + ((int64_t)zc * R.nc[1] + yc) * R.nc[0];
                const int64_t c0 = row + px;
                const int64_t c1 = row + px + lx - 1;
                rstart = a.cell_start[c0];
                rlen = a.cell_start[c1] + a.cell_count[c1] - rstart;
            }
            const int sx = xr == 0 ? ax.s0 : ax.s1;
            rshift = (sx + 1) | ((axis_shift(ay, yi) + 1) << 2) | ((axis_shift(az, zi) + 1) << 4);
        }
    }
    // exclusive prefix of the run lengths: non-decreasing over the lanes, so
    // the largest lane with rpre <= f owns candidate f (empty runs share the
    // prefix of the next non-empty run and lose the search to it)
    const int incl = wave_incl_scan(rlen);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const int rpre = incl - rlen;

    double4* const ctr = s_ctr[threadIdx.x >> 6];
    for (int g0 = 0; g0 < m; g0 += 64) {
        const int mg = min(64, m - g0);
        double4 xc = make_double4(0.0, 0.0, 0.0, 0.0);
        if (lane < mg) xc = a.xs[i0 + g0 + lane];
        // centre positions for the tests: one LDS read (the same address in
        // every lane) per test instead of six lane reads
        lds_fence_before_write();
        ctr[lane] = xc;
        lds_fence_after_write();
        int cnt_c = 0, cnt_s = 0, cnt_f = 0;
        for (int base = 0; base < total; base += 64) {
            const int f = base + lane;
            // largest run q with rpre[q] <= f
            int q = 0;
#pragma unroll
            for (int step = 32; step > 0; step >>= 1) {
                const int t = shfl_i32(rpre, q + step);
                if (t <= f) q += step;
            }
            const int qs = shfl_i32(rstart, q);
            const int qp = shfl_i32(rpre, q);
            const int j = qs + (f - qp);
            const bool valid = f < total && j >= 0 && (int64_t)j < a.n_slots;
            // (the lane read runs in every lane: a lane permute from a lane
            // that is switched off reads zero)
            const int code_q = shfl_i32(rshift, q);
            const int code = valid ? code_q : kNoShift;
            double4 xj = make_double4(0.0, 0.0, 0.0, 0.0);
            if (valid) xj = a.xs[j];
            const uint64_t vmask = __builtin_amdgcn_ballot_w64(valid);
            // the tests of centre ii against the chunk, each classification
            // one compare that writes its wave mask
            auto test = [&](int ii, double dx, double dy, double dz) {
                const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                const int islot = i0 + g0 + ii;
                const uint64_t ok = vmask & __builtin_amdgcn_ballot_w64(j != islot);
                if (WC) {
                    const uint64_t mk = ok & cmp_lt_mask(r2, a.thr_core);
                    const int b0 = __builtin_amdgcn_readlane(cnt_c, ii);
                    if (!COUNT_ONLY && __builtin_amdgcn_inverse_ballot_w64(mk)) {
                        const int p = b0 + (int)mbcnt(mk);
                        if (p < a.cap_core) a.core[ell(islot, p, a.cap_core)] = j;
                    }
                    if (lane == ii) cnt_c += __popcll(mk);
                }
                if (WS) {
                    const uint64_t mk = ok & cmp_ge_mask(r2, a.thr_shell_in) & cmp_lt_mask(r2, a.thr_out);
                    const int b0 = __builtin_amdgcn_readlane(cnt_s, ii);
                    if (!COUNT_ONLY && __builtin_amdgcn_inverse_ballot_w64(mk)) {
                        const int p = b0 + (int)mbcnt(mk);
                        if (p < a.cap_shell) a.shell[ell(islot, p, a.cap_shell)] = j;
                    }
                    if (lane == ii) cnt_s += __popcll(mk);
                }
                if (WF) {
                    const uint64_t mk = ok & cmp_lt_mask(r2, a.thr_out);
                    const int b0 = __builtin_amdgcn_readlane(cnt_f, ii);
                    if (!COUNT_ONLY && __builtin_amdgcn_inverse_ballot_w64(mk)) {
                        const int p = b0 + (int)mbcnt(mk);
                        if (p < a.cap_full) a.full[ell(islot, p, a.cap_full)] = j;
                    }
                    if (lane == ii) cnt_f += __popcll(mk);
                }
            };
            if (SHIFT && __ballot(code != kNoShift) == 0) {
                // no periodic image in the chunk: (x_i - x_j) + 0 is x_i - x_j
                for (int ii = 0; ii < mg; ++ii) {
                    const double4 xi = ctr[ii];
                    test(ii, xi.x - xj.x, xi.y - xj.y, xi.z - xj.z);
                }
            } else if (SHIFT) {
                const double shx = (double)((code & 3) - 1) * R.L[0];
                const double shy = (double)(((code >> 2) & 3) - 1) * R.L[1];
                const double shz = (double)(((code >> 4) & 3) - 1) * R.L[2];
                for (int ii = 0; ii < mg; ++ii) {
                    const double4 xi = ctr[ii];
                    test(ii, (xi.x - xj.x) + shx, (xi.y - xj.y) + shy, (xi.z - xj.z) + shz);
                }
            } else {
                for (int ii = 0; ii < mg; ++ii) {
                    const double4 xi = ctr[ii];
                    test(ii, min_image(xi.x - xj.x, R.L[0], R.inv[0]), min_image(xi.y - xj.y, R.L[1], R.inv[1]),
                         min_image(xi.z - xj.z, R.L[2], R.inv[2]));
                }
            }
        }
        const bool mine = lane < mg;
        const int islot = i0 + g0 + lane;
        if (WC) {
            if (mine && !COUNT_ONLY) a.core_len[islot] = min(cnt_c, a.cap_core);
            const int mx = wave_max(mine ? cnt_c : 0);
            if (lane == 0) {
                raise_max(&a.flags[kFlagMaxCore], mx);
                if (!COUNT_ONLY && mx > a.cap_core) raise_flag(&a.flags[kFlagOverflow]);
            }
        }
        if (WS) {
            if (mine && !COUNT_ONLY) a.shell_len[islot] = min(cnt_s, a.cap_shell);
            const int mx = wave_max(mine ? cnt_s : 0);
            if (lane == 0) {
                raise_max(&a.flags[kFlagMaxShell], mx);
                if (!COUNT_ONLY && mx > a.cap_shell) raise_flag(&a.flags[kFlagOverflow]);
            }
        }
        if (WF) {
            if (mine && !COUNT_ONLY) a.full_len[islot] = min(cnt_f, a.cap_full);
            const int mx = wave_max(mine ? cnt_f : 0);
            if (lane == 0) {
                raise_max(&a.flags[kFlagMaxFull], mx);
                if (!COUNT_ONLY && mx > a.cap_full) raise_flag(&a.flags[kFlagOverflow]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Core / shell / full list build for particle types (Sec. II).  The cells
// are sized by the smallest pair cut-off; the centres of one type at a time
// walk the stencil of that type's half-width h (every cell within h of the
// centre cell along each axis, each cell once), one z-slab after the other.
// In a slab, lane q describes run q = (y-row q / 2, x-part q % 2) as k_build
// does for its whole stencil, so candidates come in ascending slot order and
// rows need no sort.  Each candidate is tested with the thresholds of its
// pair of types.  2 (2h + 1) <= 64 runs per slab (the host keeps h <= 15).
template <bool COUNT_ONLY, bool WC, bool WS, bool WF>
__global__ __launch_bounds__(256) void k_build_typed(BuildArgs a)
{
    __shared__ double s_thr[3][kMaxTypes * kMaxTypes];  // core, shell inner, outer thresholds per pair
    __shared__ double4 s_ctr[4][64];                     // the group's centre positions, per wavefront
    if (gated_off(a.gate)) return;
    if (!COUNT_ONLY) record_build(a);
    for (int k = threadIdx.x; k < kMaxTypes * kMaxTypes; k += blockDim.x) {
        s_thr[0][k] = a.types->p[k].thr_core;
        s_thr[1][k] = a.types->p[k].thr_in;
        s_thr[2][k] = a.types->p[k].thr_out;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t cell = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (cell >= a.n_cells) return;
    const int m = a.cell_count[cell];
    if (m == 0) return;
    const int i0 = a.cell_start[cell];
    if (i0 < 0 || (int64_t)i0 + m > a.n_slots) {
        if (lane == 0) atomicOr(&a.flags[kFlagBadSlot], 2);
        return;
    }
    const DevReplica& R = a.rep[a.cell_rep[cell]];
    const int64_t lc = cell - R.cell_base;
    const int cx = (int)(lc % R.nc[0]);
    const int cy = (int)((lc / R.nc[0]) % R.nc[1]);
    const int cz = (int)(lc / ((int64_t)R.nc[0] * R.nc[1]));
    const int ntypes = a.types->n_types;
    double4* const ctr = s_ctr[threadIdx.x >> 6];

    for (int g0 = 0; g0 < m; g0 += 64) {
        const int mg = min(64, m - g0);
        double4 xc = make_double4(0.0, 0.0, 0.0, 0.0);
        if (lane < mg) xc = a.xs[i0 + g0 + lane];
        const int tc = lane < mg ? type_of(xc.w) : -1;
        // centre positions for the tests: one LDS read (the same address in
        // every lane) per test instead of six lane reads
        lds_fence_before_write();
        ctr[lane] = xc;
        lds_fence_after_write();
        int cnt_c = 0, cnt_s = 0, cnt_f = 0;
        for (int t = 0; t < ntypes; ++t) {
            const uint64_t centres = __ballot(tc == t);
            if (centres == 0) continue;
            const int h = a.types->h[t];
            const AxisRuns ax = axis_runs(cx, R.nc[0], h);
            const AxisRuns ay = axis_runs(cy, R.nc[1], h);
            const AxisRuns az = axis_runs(cz, R.nc[2], h);
            const int ny_s = ay.l0 + ay.l1;
            const int nz_s = az.l0 + az.l1;
            for (int zi = 0; zi < nz_s; ++zi) {
                const int zc = axis_cell(az, zi);
                int rstart = 0, rlen = 0;
                {
                    const int yi = lane >> 1;
                    const int xr = lane & 1;
                    const int px = xr == 0 ? ax.p0 : ax.p1;
                    const int lx = xr == 0 ? ax.l0 : ax.l1;
                    if (yi < ny_s && lx > 0) {
                        const int yc = axis_cell(ay, yi);
                        const int64_t row = R.cell_base + ((int64_t)zc * R.nc[1] + yc) * R.nc[0];
                        rstart = a.cell_start[row + px];
                        rlen = a.cell_start[row + px + lx - 1] + a.cell_count[row + px + lx - 1] - rstart;
                    }
                }
                const int incl = wave_incl_scan(rlen);
                const int total = __builtin_amdgcn_readlane(incl, 63);
                const int rpre = incl - rlen;
                for (int base = 0; base < total; base += 64) {
                    const int f = base + lane;
                    int q = 0;
#pragma unroll
                    for (int step = 32; step > 0; step >>= 1) {
                        const int tq = shfl_i32(rpre, q + step);
                        if (tq <= f) q += step;
                    }
                    const int j = shfl_i32(rstart, q) + (f - shfl_i32(rpre, q));
                    const bool valid = f < total && j >= 0 && (int64_t)j < a.n_slots;
                    double4 xj = make_double4(0.0, 0.0, 0.0, 0.0);
                    if (valid) xj = a.xs[j];
                    const int pe = t * kMaxTypes + type_of(xj.w);
                    const double thr_core = s_thr[0][pe];
                    const double thr_in = s_thr[1][pe];
                    const double thr_out = s_thr[2][pe];
                    for (uint64_t rest = centres; rest; rest &= rest - 1) {
                        const int ii = (int)__builtin_ctzll(rest);
                        const int islot = i0 + g0 + ii;
                        const double4 xi = ctr[ii];
                        const Delta d = delta(xi, xj, R);
                        const bool ok = valid && j != islot;
                        if (WC) {
                            const bool in = ok && d.r2 < thr_core;
                            const uint64_t mk = __ballot(in);
                            const int b0 = __builtin_amdgcn_readlane(cnt_c, ii);
                            if (!COUNT_ONLY && in) {
                                const int p = b0 + (int)mbcnt(mk);
                                if (p < a.cap_core) a.core[ell(islot, p, a.cap_core)] = j;
                            }
                            if (lane == ii) cnt_c += __popcll(mk);
                        }
                        if (WS) {
                            const bool in = ok && d.r2 >= thr_in && d.r2 < thr_out;
                            const uint64_t mk = __ballot(in);
                            const int b0 = __builtin_amdgcn_readlane(cnt_s, ii);
                            if (!COUNT_ONLY && in) {
                                const int p = b0 + (int)mbcnt(mk);
                                if (p < a.cap_shell) a.shell[ell(islot, p, a.cap_shell)] = j;
                            }
                            if (lane == ii) cnt_s += __popcll(mk);
                        }
                        if (WF) {
                            const bool in = ok && d.r2 < thr_out;
                            const uint64_t mk = __ballot(in);
                            const int b0 = __builtin_amdgcn_readlane(cnt_f, ii);
                            if (!COUNT_ONLY && in) {
                                const int p = b0 + (int)mbcnt(mk);
                                if (p < a.cap_full) a.full[ell(islot, p, a.cap_full)] = j;
                            }
                            if (lane == ii) cnt_f += __popcll(mk);
                        }
                    }
                }
            }
        }
        const bool mine = lane < mg;
        const int islot = i0 + g0 + lane;
        if (WC) {
            if (mine && !COUNT_ONLY) a.core_len[islot] = min(cnt_c, a.cap_core);
            const int mx = wave_max(mine ? cnt_c : 0);
            if (lane == 0) {
                raise_max(&a.flags[kFlagMaxCore], mx);
                if (!COUNT_ONLY && mx > a.cap_core) raise_flag(&a.flags[kFlagOverflow]);
            }
        }
        if (WS) {
            if (mine && !COUNT_ONLY) a.shell_len[islot] = min(cnt_s, a.cap_shell);
            const int mx = wave_max(mine ? cnt_s : 0);
            if (lane == 0) {
                raise_max(&a.flags[kFlagMaxShell], mx);
                if (!COUNT_ONLY && mx > a.cap_shell) raise_flag(&a.flags[kFlagOverflow]);
            }
        }
        if (WF) {
            if (mine && !COUNT_ONLY) a.full_len[islot] = min(cnt_f, a.cap_full);
            const int mx = wave_max(mine ? cnt_f : 0);
            if (lane == 0) {
                raise_max(&a.flags[kFlagMaxFull], mx);
                if (!COUNT_ONLY && mx > a.cap_full) raise_flag(&a.flags[kFlagOverflow]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Batches in HBM: batch[(rr * n_slots + slot) * P + m] is the m-th partner
// (slot) of the particle in `slot` for the rr-th force evaluation after the
// build; a particle's P partners are contiguous, and so are the batches of
// the particles of one cell.
__device__ __forceinline__ int64_t batch_index(int rr, int64_t slot, int m, int64_t n_slots, int P)
{
    return ((int64_t)rr * n_slots + slot) * P + m;
}

struct FusedArgs {
    BuildArgs b;
    const int* perm;
    int* batch;        // [K][n_slots][P]
    uint64_t seed;
    uint64_t step0;
    const uint64_t* step_dev;  // if set, the draw's first step is *step_dev + step0
    int K;
    int P;
    int cap_list;              // LDS shell-list room per centre particle (<= 0: all candidates)
    int list_budget;           // LDS list entries per wavefront (dynamic LDS of the launch)
    // stencil draw population only:
    double core_reach;         // r_s + skin: 3 x 3 x 3 cells hold the core when it fits a cell
    int draw_only;             // 1: batches and population sizes only, core rows untouched
};

__device__ __forceinline__ void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Fused list build + batch draw (the molecular-dynamics loop path).  As in
// k_build, one wavefront per centre cell walks the 5x5x5 stencil, but only
// the core rows go to HBM.  Each centre particle's shell candidates are
// appended, in stencil order, to a list of 16-bit (run, offset-in-run)
// entries in LDS; its length is n_i, and the batches of the next K force
// evaluations are drawn right away, one lane per (particle, step) pair, the
// k-th shell candidate being one LDS read away.  Bit-identical to k_build +
// k_predraw, without writing or re-reading the shell rows.  Details:
//  - the stencil's cells merge into x-runs of contiguous slots (at most 50);
//    the runs with particles sit in LDS (start, prefix count, image shift),
//    and a lane finds the run of its candidate from two ballots over the
//    prefix counts (runs starting before its chunk, and the few starting
//    inside it), with no per-lane search;
//  - lanes past the end of the candidates carry a `live` flag instead of a
//    poisoned position, so no per-chunk initialisation is needed;
//  - the periodic image of every candidate run is known from the stencil
//    geometry when every axis has >= 7 cells, so dx = (x_i - x_j) + s with
//    s in {-L, 0, L} exactly equals the canonical fma(-rint(d/L), L, d)
//    (decided per wavefront: each cell belongs to one replica); smaller
//    grids use the canonical formula per pair;
//  - every cell-level quantity is made wave-uniform with readfirstlane, so
//    it lives in SGPRs;
//  - each chunk is first tested against the bounding box of the group's
//    centre particles (widened by a margin far above rounding): a
//    candidate farther than r_c + skin from the box is farther from every
//    centre and is dropped; the rest (about half of the stencil at liquid
//    density) pass through an LDS ring, in stencil order, and are tested
//    64 at a time, each batch loaded one chunk ahead of its tests;
//  - per centre particle and batch, a non-empty core ballot sends its
//    candidates straight into the particle's sliced-ELL row at the row's
//    count + mbcnt (the count held in lane ii), so rows keep candidate
//    order; the shell ballot is compacted into the particle's LDS list the
//    same way;
//  - a centre particle's list has room for every stencil candidate, so the
//    centre particles go in groups of (LDS list budget) / (room) at most,
//    the budget being set by the host from the shell counts it has seen
//    (dynamic LDS); a room beyond the budget (or a run beyond 1023) raises
//    kFlagStencil and the host redoes the run on explicit lists;
//  - centre cells are mapped to blocks by xcd_tile, so that each XCD works
//    on runs of neighbouring cells (its L2 keeps the neighbourhood).
// STENCIL = true draws from the paper's own population instead (Sec. II):
// all N_I particles of the stencil cells, the centre particle included,
// scaled by N_I/P in eq. (4), with the pair term zero outside the shell
// zone.  N_I is the same for every particle of a cell, so no shell list is
// kept: the k-th stencil particle is found by a binary search over the run
// prefix counts.  The core test then walks only the 3 x 3 x 3 cells around
// the centre cell when r_s + skin fits one cell edge (else the 5 x 5 x 5
// stencil), and with draw_only set the kernel writes just the batches and
// N_I (the batch export and single force evaluations of a build).
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ double rfl(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ int64_t rfl(int64_t v)
{
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// v_writelane_b32 through its LLVM intrinsic, so that the compiler itself
// places the lane select (in M0 when the data operand is an SGPR).
extern "C" __device__ int rbl_writelane(int value, int lane, int old) __asm("llvm.amdgcn.writelane");


// s_waitcnt immediate with vmcnt = 0 and the expcnt / lgkmcnt fields at
// their maximum (no wait on them)
constexpr int kWaitVmcnt0 = 0x0F70;
// Per lane: a where the lane's bit of the wave-uniform mask is set, else b.
// A plain v_cndmask_b32 on the mask; written out so that the compiler keeps
// it a select instead of branching around the computation of a.
__device__ __forceinline__ int select_lanes(uint64_t mask, int a, int b)
{
    int r;
    asm volatile("v_cndmask_b32 %0, %2, %1, %3" : "=v"(r) : "v"(a), "v"(b), "s"(mask));
    return r;
}

constexpr int kCtrMax = 16;        // centre particles per group
constexpr int kListBudgetMax = 6912;  // 16-bit shell-list entries per wavefront, at most
                                      // (the block's LDS stays within 64 KB)
constexpr int kFusedWavesPerEu = 7;   // occupancy the fused build is compiled for (P <= 32):
                                      // as many blocks of 4 wavefronts per CU
constexpr int kRunOffBits = 10;    // list entry = run << 10 | offset in the run
constexpr int kRing = 128;         // ring of kept candidates per wavefront (two chunks)

template <int PMAX, bool STENCIL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PMAX <= 32 ? kFusedWavesPerEu : 2))) void k_build_draw(FusedArgs fa)
{
    __shared__ double4 s_ctr[4][kCtrMax];
    __shared__ int s_rstart[4][64];
    __shared__ int s_rpre[4][64];
    __shared__ unsigned char s_rshift[4][64];
    __shared__ int s_ncnt[4][kCtrMax];
    // kept candidates' list entries on their way to the tests (shell-list form)
    __shared__ unsigned short s_ring[STENCIL ? 1 : 4][STENCIL ? 1 : kRing];
    // STENCIL: run table of the core test (3 x 3 x 3 cells when they reach)
    __shared__ int s_crstart[STENCIL ? 4 : 1][64];
    __shared__ int s_crpre[STENCIL ? 4 : 1][64];
    __shared__ unsigned char s_crshift[STENCIL ? 4 : 1][64];
    // per wavefront: list_budget entries + a write-off word per lane
    extern __shared__ unsigned short s_dyn[];
    const BuildArgs& a = fa.b;
    if (gated_off(a.gate)) return;
    if (!fa.draw_only) record_build(a);
    const int lane = threadIdx.x & 63;
    const int w = rfl((int)(threadIdx.x >> 6));
    const int budget = fa.list_budget;
    unsigned short* const s_lst = s_dyn + w * (budget + 64);
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t cell = tile * 4 + w;
    if (cell >= a.n_cells) return;
    const int m = rfl(a.cell_count[cell]);
    if (m == 0) return;
    const int i0 = rfl(a.cell_start[cell]);
    if (i0 < 0 || (int64_t)i0 + m > a.n_slots) {
        if (lane == 0) atomicOr(&a.flags[kFlagBadSlot], 2);
        return;
    }
    const int rep_id = rfl(a.cell_rep[cell]);
    const DevReplica* Rp = a.rep + rep_id;
    const double L0 = rfl(Rp->L[0]), L1 = rfl(Rp->L[1]), L2 = rfl(Rp->L[2]);
    const double iL0 = rfl(Rp->inv[0]), iL1 = rfl(Rp->inv[1]), iL2 = rfl(Rp->inv[2]);
    const int nc0 = rfl(Rp->nc[0]), nc1 = rfl(Rp->nc[1]), nc2 = rfl(Rp->nc[2]);
    const int64_t cell_base = rfl(Rp->cell_base);
    const int64_t id_base = rfl(Rp->id_base);
    const int64_t lc = cell - cell_base;
    const int cx = (int)(lc % nc0);
    const int cy = (int)((lc / nc0) % nc1);
    const int cz = (int)(lc / ((int64_t)nc0 * nc1));
    const bool SHIFT = nc0 >= 7 && nc1 >= 7 && nc2 >= 7;  // image of every run known
    // runs of the stencil of half-width h around the cell: lane q holds run
    // q (z-row, y-row, x-part) as slot start, length and image-shift code
    auto run_table = [&](int h, int& rstart, int& rlen, int& rshift) {
        const AxisRunsS ax = axis_runs_s(cx, nc0, h);
        const AxisRunsS ay = axis_runs_s(cy, nc1, h);
        const AxisRunsS az = axis_runs_s(cz, nc2, h);
        const int ny_s = ay.l0 + ay.l1;
        const int nz_s = az.l0 + az.l1;
        rstart = 0;
        rlen = 0;
        rshift = 0;
        const int q = lane;
        const int zi = q / (2 * ny_s);
        const int yi = (q >> 1) % ny_s;
        const int xr = q & 1;
        if (zi < nz_s) {
            const int zc = axis_cell(AxisRuns{az.p0, az.l0, az.p1, az.l1}, zi);
            const int yc = axis_cell(AxisRuns{ay.p0, ay.l0, ay.p1, ay.l1}, yi);
            const int px = xr == 0 ? ax.p0 : ax.p1;
            const int lx = xr == 0 ? ax.l0 : ax.l1;
            if (lx > 0) {
                const int64_t row = cell_base + ((int64_t)zc * nc1 + yc) * nc0;
                const int64_t c0 = row + px;
                const int64_t c1 = row + px + lx - 1;
                rstart = a.cell_start[c0];
                rlen = a.cell_start[c1] + a.cell_count[c1] - rstart;
            }
            const int sx = xr == 0 ? ax.s0 : ax.s1;
            const int sy = axis_shift(ay, yi);
            const int sz = axis_shift(az, zi);
            rshift = (sx + 1) | ((sy + 1) << 2) | ((sz + 1) << 4);
        }
    };
    // The run tables in LDS: entry q is the q-th run with particles, in
    // stencil order (slot start, prefix count, image-shift code); runs
    // without particles are dropped, so a chunk of 64 consecutive
    // candidates crosses few run starts.  Entries past the last run hold
    // the total (the stencil draw's binary search relies on it).  A run
    // outside the slot range stops the cell, so every candidate slot taken
    // from a run is valid.
    auto compact_runs = [&](int rs, int rl, int rsh, int* t_st, int* t_pr, unsigned char* t_sh, int& tot,
                            int& nr) -> bool {
        const uint64_t nz = __ballot(rl > 0);
        const int incl = wave_incl_scan(rl);
        tot = rfl(__builtin_amdgcn_readlane(incl, 63));
        nr = (int)__popcll(nz);
        const int qc = (int)mbcnt(nz);
        if (rl > 0) {
            t_st[qc] = rs;
            t_pr[qc] = incl - rl;
            t_sh[qc] = (unsigned char)rsh;
        }
        if (lane >= nr) {
            t_st[lane] = 0;
            t_pr[lane] = tot;
            t_sh[lane] = (unsigned char)kNoShift;
        }
        return __ballot(rl > 0 && (rs < 0 || (int64_t)rs + rl > a.n_slots)) == 0;
    };
    int rstart, rlen, rshift;
    run_table(2, rstart, rlen, rshift);
    int total, nruns;
    bool runs_ok = compact_runs(rstart, rlen, rshift, s_rstart[w], s_rpre[w], s_rshift[w], total, nruns);
    // the table the core test walks: the stencil's own, or (STENCIL, when
    // r_s + skin fits one cell edge with the cell grid's margin) the
    // 3 x 3 x 3 cells around the centre cell
    int ctotal = total, cnruns = nruns;
    if constexpr (STENCIL) {
        const double edge = fmin(L0 / nc0, fmin(L1 / nc1, L2 / nc2));
        const int hc = fa.core_reach * (1.0 + 1e-6) <= edge ? 1 : 2;
        int cs, cl, csh;
        run_table(hc, cs, cl, csh);
        runs_ok = compact_runs(cs, cl, csh, s_crstart[w], s_crpre[w], s_crshift[w], ctotal, cnruns) && runs_ok;
    }
    if (!runs_ok) {
        if (lane == 0) atomicOr(&a.flags[kFlagBadSlot], 64);
        return;
    }
    auto t_start = [&](int q) { if constexpr (STENCIL) return s_crstart[w][q]; else return s_rstart[w][q]; };
    auto t_pre = [&](int q) { if constexpr (STENCIL) return s_crpre[w][q]; else return s_rpre[w][q]; };
    auto t_shift = [&](int q) { if constexpr (STENCIL) return s_crshift[w][q]; else return s_rshift[w][q]; };
    // list room per centre particle: the host's bound on shell counts (a
    // particle beyond it raises the overflow flag), never above the stencil
    const int cap = (fa.cap_list > 0 && fa.cap_list < total) ? fa.cap_list : max(total, 1);
    if (!STENCIL && (cap > budget || wave_max(rlen) >= (1 << kRunOffBits))) {
        // the host repeats the run on explicit rows; until it does, this
        // cell's particles have empty rows, so no force kernel of the run
        // reads a batch entry or core row that was never written
        for (int t = lane; t < m; t += 64) {
            a.core_len[i0 + t] = 0;
            a.shell_len[i0 + t] = 0;
        }
        if (lane == 0) {
            raise_flag(&a.flags[kFlagStencil]);
            raise_flag(&a.flags[kFlagOverflow]);
        }
        return;
    }
    const int nch = (ctotal + 63) >> 6;  // >= 1: the cell itself is in the table
    const int gmax = STENCIL ? kCtrMax : min(kCtrMax, budget / cap);  // >= 1
    const int P = fa.P;
    const bool do_core = !STENCIL || !fa.draw_only;
    wave_lds_fence();

    // Candidate f0 + lane of the core test's table: `live` (false past the
    // table's end), slot (the centre cell's first slot when not live),
    // position, image-shift code and list entry.  The lane's run is the
    // last one whose prefix count is <= its index: the runs starting at or
    // before f0, plus one per run start inside the chunk (wave-uniform,
    // few as the runs are dense).
    const int tpre_v = t_pre(lane);
    const int tnr = STENCIL ? cnruns : nruns;
    auto candidate = [&](int f0, int& j, double4& xj, int& code, int& ent, bool& live) {
        const uint64_t below = __ballot(lane < tnr && tpre_v <= f0);
        uint64_t inside = __ballot(lane < tnr && tpre_v > f0 && tpre_v < f0 + 64);
        int q = (int)__popcll(below) - 1;
        while (inside) {
            const int b = (int)__builtin_ctzll(inside);
            inside &= inside - 1;
            q += lane >= __builtin_amdgcn_readlane(tpre_v, b) - f0 ? 1 : 0;
        }
        const int f = f0 + lane;
        const int off = f - t_pre(q);
        live = f < ctotal;
        j = live ? t_start(q) + off : i0;
        code = live ? (int)t_shift(q) : kNoShift;
        ent = (q << kRunOffBits) | off;
        xj = a.xs[j];
    };

    for (int g0 = 0; g0 < m; g0 += gmax) {
        const int mg = rfl(min(gmax, m - g0));
        const int my_slot = i0 + g0 + lane;
        uint32_t nshell = 0;  // lane ii: shell candidates of centre ii so far
        if (do_core) {
            if (lane < mg) s_ctr[w][lane] = a.xs[i0 + g0 + lane];
            wave_lds_fence();
            uint32_t ncore = 0;  // lane ii: core partners of centre ii so far
            // the tests of the group's centres against 64 candidates (slot
            // jc, position xc, image-shift code, list entry ent, in the
            // lanes where `live`): core partners written to the centre's
            // row, shell candidates appended to its LDS list
            auto test_chunk = [&](int jc, const double4& xc, int code, int ent, bool live) {
                const uint64_t lmask = __builtin_amdgcn_ballot_w64(live);
                auto test = [&](int ii, double dx, double dy, double dz) {
                    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    const int slot_ii = i0 + g0 + ii;
                    // the classifications as wave masks, each compare a
                    // single v_cmp (a ballot of a combined bool would first
                    // turn it into 0/1 in a VGPR and compare that again)
                    const uint64_t other = lmask & __builtin_amdgcn_ballot_w64(jc != slot_ii);
                    const uint64_t mc = other & cmp_lt_mask(r2, a.thr_core);
                    if (mc) {
                        const bool is_core = __builtin_amdgcn_inverse_ballot_w64(mc);
                        // straight into row ii (sliced ELL) in candidate order;
                        // entries past the row's room are counted, not written
                        const int basec = rfl((int)__builtin_amdgcn_readlane((int)ncore, ii));
                        const int k = basec + (int)mbcnt(mc);
                        // row start, wave-uniform: slice (slot / 64) of cap_core
                        // columns of 64, lane slot % 64 (slot < 2^31)
                        const uint32_t su = (uint32_t)slot_ii;
                        int* const row = a.core + ((uint64_t)(su >> 6) * (uint32_t)(a.cap_core * 64) + (su & 63u));
                        if (is_core && k < a.cap_core) row[(uint32_t)k * 64u] = jc;
                        ncore = (uint32_t)rbl_writelane(basec + (int)__popcll(mc), ii, (int)ncore);
                    }
                    if constexpr (STENCIL) return;
                    const uint64_t ms = other & cmp_ge_mask(r2, a.thr_shell_in) & cmp_lt_mask(r2, a.thr_out);
                    const int base = rfl((int)__builtin_amdgcn_readlane((int)nshell, ii));
                    // every lane writes (no branch): a selected lane to its list
                    // position (clamped into the room; an overflowing run is
                    // repeated by the host), the others to their write-off word
                    const int pos = ii * cap + min(base + (int)mbcnt(ms), cap - 1);
                    s_lst[select_lanes(ms, pos, budget + lane)] = (unsigned short)ent;
                    nshell = (uint32_t)rbl_writelane(base + (int)__popcll(ms), ii, (int)nshell);
                };
                if (SHIFT && __ballot(code != kNoShift) == 0) {
                    // no periodic image in the chunk: (x_i - x_j) + 0 is x_i - x_j
                    for (int ii = 0; ii < mg; ++ii) {
                        const double4 xi = s_ctr[w][ii];
                        test(ii, xi.x - xc.x, xi.y - xc.y, xi.z - xc.z);
                    }
                } else if (SHIFT) {
                    const double shx = (double)((code & 3) - 1) * L0;
                    const double shy = (double)(((code >> 2) & 3) - 1) * L1;
                    const double shz = (double)(((code >> 4) & 3) - 1) * L2;
                    for (int ii = 0; ii < mg; ++ii) {
                        const double4 xi = s_ctr[w][ii];
                        test(ii, (xi.x - xc.x) + shx, (xi.y - xc.y) + shy, (xi.z - xc.z) + shz);
                    }
                } else {
                    for (int ii = 0; ii < mg; ++ii) {
                        const double4 xi = s_ctr[w][ii];
                        test(ii, min_image(xi.x - xc.x, L0, iL0), min_image(xi.y - xc.y, L1, iL1),
                             min_image(xi.z - xc.z, L2, iL2));
                    }
                }
            };
            int jn, coden, entn;
            double4 xn;
            bool liven;
            candidate(0, jn, xn, coden, entn, liven);
            // the first chunk's candidates are complete before the chunk loop:
            // with nothing of this load pending at the loop head, the inner loop
            // waits on no vector-memory counter, and each chunk's prefetch of the
            // next one overlaps with the work on the current one
            __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            if constexpr (STENCIL) {
                for (int ch = 0; ch < nch; ++ch) {
                    const int jc = jn;
                    const double4 xc = xn;
                    const int code = coden;
                    const int ent = entn;
                    const bool live = liven;
                    if (ch + 1 < nch) candidate((ch + 1) * 64, jn, xn, coden, entn, liven);
                    test_chunk(jc, xc, code, ent, live);
                }
            } else {
                // The group's bounding box, widened by a margin far above the
                // rounding of the coordinates: a candidate farther than the
                // outer radius from the box is farther from every centre of
                // the group, and skips their tests.  The list entries of the
                // kept candidates pass through a ring in LDS, in stencil
                // order, and are tested 64 at a time; each such batch is
                // loaded one chunk before its tests.
                double lo0 = 1.0e300, lo1 = 1.0e300, lo2 = 1.0e300;
                double hi0 = -1.0e300, hi1 = -1.0e300, hi2 = -1.0e300;
                for (int ii = 0; ii < mg; ++ii) {
                    const double4 xi = s_ctr[w][ii];
                    lo0 = fmin(lo0, xi.x);
                    hi0 = fmax(hi0, xi.x);
                    lo1 = fmin(lo1, xi.y);
                    hi1 = fmax(hi1, xi.y);
                    lo2 = fmin(lo2, xi.z);
                    hi2 = fmax(hi2, xi.z);
                }
                const double margin = 1.0e-9 * (1.0 + L0 + L1 + L2);
                const double bc0 = rfl(0.5 * (lo0 + hi0)), be0 = rfl(0.5 * (hi0 - lo0) + margin);
                const double bc1 = rfl(0.5 * (lo1 + hi1)), be1 = rfl(0.5 * (hi1 - lo1) + margin);
                const double bc2 = rfl(0.5 * (lo2 + hi2)), be2 = rfl(0.5 * (hi2 - lo2) + margin);
                const double keep_thr = fmax(a.thr_core, a.thr_out);
                int head = 0, tail = 0;  // ring positions (wave-uniform)
                bool have = false;       // a batch is loaded and waits for its tests
                int jb = i0, codeb = kNoShift, entb = 0;
                bool liveb = false;
                double4 xb = make_double4(0.0, 0.0, 0.0, 0.0);
                for (int ch = 0;; ++ch) {
                    if (ch < nch) {
                        const int jc = jn;
                        const double4 xc = xn;
                        const int code = coden;
                        const int ent = entn;
                        const bool live = liven;
                        if (ch + 1 < nch) candidate((ch + 1) * 64, jn, xn, coden, entn, liven);
                        double dx, dy, dz;
                        if (SHIFT && __ballot(code != kNoShift) == 0) {
                            dx = bc0 - xc.x;
                            dy = bc1 - xc.y;
                            dz = bc2 - xc.z;
                        } else if (SHIFT) {
                            dx = (bc0 - xc.x) + (double)((code & 3) - 1) * L0;
                            dy = (bc1 - xc.y) + (double)(((code >> 2) & 3) - 1) * L1;
                            dz = (bc2 - xc.z) + (double)(((code >> 4) & 3) - 1) * L2;
                        } else {
                            dx = min_image(bc0 - xc.x, L0, iL0);
                            dy = min_image(bc1 - xc.y, L1, iL1);
                            dz = min_image(bc2 - xc.z, L2, iL2);
                        }
                        const double gx = fmax(fabs(dx) - be0, 0.0);
                        const double gy = fmax(fabs(dy) - be1, 0.0);
                        const double gz = fmax(fabs(dz) - be2, 0.0);
                        const bool keep = live && fma(gz, gz, fma(gy, gy, gx * gx)) < keep_thr;
                        const uint64_t mk = __ballot(keep);
                        // after the reads of the previous batch
                        wave_lds_fence();
                        if (keep) s_ring[w][(tail + (int)mbcnt(mk)) & (kRing - 1)] = (unsigned short)ent;
                        tail += (int)__popcll(mk);
                    }
                    if (have) test_chunk(jb, xb, codeb, entb, liveb);
                    const bool drained = ch + 1 >= nch;
                    have = tail - head >= 64 || (drained && tail > head);
                    if (!have && drained) break;
                    if (have) {
                        wave_lds_fence();
                        const int nb = min(64, tail - head);
                        // lanes past the batch read a stale ring entry (still
                        // a run of the table) and take the centre cell's
                        // first slot
                        liveb = lane < nb;
                        entb = s_ring[w][(head + lane) & (kRing - 1)];
                        const int q = entb >> kRunOffBits;
                        jb = liveb ? s_rstart[w][q] + (entb & ((1 << kRunOffBits) - 1)) : i0;
                        codeb = liveb ? (int)s_rshift[w][q] : kNoShift;
                        xb = a.xs[jb];
                        head += nb;
                    }
                }
            }
            const int cnt_core = (int)ncore;
            if (lane < mg) a.core_len[my_slot] = min(cnt_core, a.cap_core);
            const int mxc = wave_max(lane < mg ? cnt_core : 0);
            const int mxs = STENCIL ? 0 : wave_max(lane < mg ? (int)nshell : 0);
            if (lane == 0) {
                raise_max(&a.flags[kFlagMaxCore], mxc);
                if (!STENCIL) raise_max(&a.flags[kFlagMaxShell], mxs);
                if (mxc > a.cap_core || mxs > cap) raise_flag(&a.flags[kFlagOverflow]);
            }
        }
        // the draw population: the particle's shell list, or N_I
        const int ns = STENCIL ? total : (lane < mg ? (int)nshell : 0);
        if (lane < mg) {
            a.shell_len[my_slot] = ns;
            if (!STENCIL) s_ncnt[w][lane] = ns;
        }
        wave_lds_fence();
        // batches: one lane per (particle, step) pair; the k-th shell
        // candidate of centre ii is entry k of its list.  Loop bounds are
        // wave-uniform; a lane whose shell is small (n <= P) takes positions
        // 0..n-1, and entries it does not own (never read by the force
        // kernels) hold the particle itself
        const int pairs = mg * fa.K;
        const uint64_t s0 = fa.step_dev ? *fa.step_dev + fa.step0 : fa.step0;
        for (int pb = 0; pb < pairs; pb += 64) {
            const int pr = pb + lane;
            if (pr < pairs) {
                const int ii = pr / fa.K;
                const int rr = pr - ii * fa.K;
                const int islot = i0 + g0 + ii;
                const int n = STENCIL ? total : s_ncnt[w][ii];
                const bool small = n <= P;
                const unsigned short* lst = &s_lst[ii * cap];
                int* out = fa.batch + batch_index(rr, islot, 0, a.n_slots, P);
                uint32_t S[PMAX];
                const uint32_t pid = (uint32_t)(fa.perm[islot] - id_base);
                floyd_draw<PMAX>(S, fa.seed, pid, (uint32_t)(s0 + rr), (uint32_t)rep_id, P, small ? P + 1 : n);
                bool bad = false;
                int val[PMAX];
#pragma unroll
                for (int qq = 0; qq < PMAX; ++qq) {
                    val[qq] = islot;
                    if (qq < P) {
                        const uint32_t k = small ? (uint32_t)qq : S[qq];
                        const bool own = (int)k < n;
                        int j;
                        if constexpr (STENCIL) {
                            // run holding stencil particle k: the last run whose
                            // prefix count is <= k (prefix counts never decrease)
                            int q = 0;
#pragma unroll
                            for (int st = 32; st > 0; st >>= 1)
                                if (s_rpre[w][q + st] <= (int)k) q += st;
                            j = s_rstart[w][q] + (int)k - s_rpre[w][q];
                        } else {
                            // past the list room (an overflowing run, repeated
                            // by the host) the entry is read from within the room
                            const int e = lst[min(k, (uint32_t)(cap - 1))];
                            j = s_rstart[w][e >> kRunOffBits] + (e & ((1 << kRunOffBits) - 1));
                        }
                        const bool ok = j >= 0 && (int64_t)j < a.n_slots;
                        bad |= own && !ok;
                        val[qq] = (own && ok) ? j : islot;
                    }
                }
                // the particle's P entries are contiguous: for even P (rows
                // 8-byte aligned, PMAX is even) in pairs
                if ((P & 1) == 0) {
#pragma unroll
                    for (int qq = 0; qq < PMAX; qq += 2)
                        if (qq < P) *reinterpret_cast<int2*>(out + qq) = make_int2(val[qq], val[qq + 1]);
                } else {
#pragma unroll
                    for (int qq = 0; qq < PMAX; ++qq)
                        if (qq < P) out[qq] = val[qq];
                }
                if (bad) atomicOr(&a.flags[kFlagBadSlot], 32);
            }
        }
        wave_lds_fence();
    }
}

// ---------------------------------------------------------------------------
// The draw population on the paper's own cell grid (Sec. II, Fig. 1): cells
// of edge w >= r_s + skin, and around particle i's cell the (2h+1)^3 cells
// with h = floor((r_c + skin)/w) + 1 (an axis of at most 2h+1 cells taken
// whole, each cell once).  The population is every particle of those cells,
// i included, N_I of them, listed cell by cell in ascending z, y, x cell
// index and by particle ID within a cell; the batch is drawn from it as
// from a shell row, and eq. (4) scales it by N_I/P with the pair term zero
// outside the shell zone.  The grid is binned at every list build (count,
// scan, scatter, in-cell sort by ID), and its members are kept for the
// draws of the list lifetime.
struct PaperGrid {
    double scale[3];    // cells per unit length: nc / L
    int nc[3];
    int h;              // stencil half-width in cells
    int64_t cell_base;  // first global cell of the replica
};

struct PaperArgs {
    const PaperGrid* grid;  // per replica
    const DevReplica* rep;
    const int* slice_rep;
    const int* cell_rep;    // paper cell -> replica
    const double4* xs;
    const int* perm;        // slot -> ID (< 0: padding)
    int64_t n_slots;
    int64_t n_cells;
    int* cell_of_slot;      // [n_slots] (-1: padding)
    int* rank;              // [n_slots]: arrival rank in the cell
    int* count;             // [n_cells]
    int* start;             // [n_cells]: first member position of the cell
    int* member;            // [n_slots]: member position -> slot
    int* flags;
    const uint64_t* gate;
};

// Paper-grid cell of every slot (positions as wrapped at the build, the
// cell coordinate floor(x nc / L) clamped into the grid) and arrival ranks.
__global__ __launch_bounds__(256) void k_paper_count(PaperArgs a)
{
    if (gated_off(a.gate)) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_slots) return;
    if (a.perm[s] < 0) {
        a.cell_of_slot[s] = -1;
        return;
    }
    const PaperGrid& G = a.grid[a.slice_rep[s >> 6]];
    const double4 x = a.xs[s];
    const double xv[3] = {x.x, x.y, x.z};
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double f = floor(xv[d] * G.scale[d]);
        c[d] = f < 0.0 ? 0 : (f > (double)(G.nc[d] - 1) ? G.nc[d] - 1 : (int)f);
    }
    const int64_t cell = G.cell_base + ((int64_t)c[2] * G.nc[1] + c[1]) * G.nc[0] + c[0];
    a.cell_of_slot[s] = (int)cell;
    a.rank[s] = atomicAdd(&a.count[cell], 1);
}

__global__ __launch_bounds__(256) void k_paper_scatter(PaperArgs a)
{
    if (gated_off(a.gate)) return;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_slots) return;
    const int cell = a.cell_of_slot[s];
    if (cell < 0) return;
    const int64_t q = (int64_t)a.start[cell] + a.rank[s];
    if (q < 0 || q >= a.n_slots) {
        atomicOr(&a.flags[kFlagBadSlot], 16);
        return;
    }
    a.member[q] = (int)s;
}

// Within each paper cell, members by ID (insertion sort; cells hold a
// handful of particles), so that the order does not depend on atomics.
__global__ __launch_bounds__(256) void k_paper_sort(PaperArgs a)
{
    if (gated_off(a.gate)) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_cells) return;
    const int b = a.start[c];
    const int m = a.count[c];
    if (b < 0 || (int64_t)b + m > a.n_slots) {
        atomicOr(&a.flags[kFlagBadSlot], 16);
        return;
    }
    for (int i = 0; i < m; ++i)
        if ((uint64_t)(uint32_t)a.member[b + i] >= (uint64_t)a.n_slots) {
            atomicOr(&a.flags[kFlagBadSlot], 16);
            return;
        }
    for (int i = 1; i < m; ++i) {
        const int sv = a.member[b + i];
        const int key = a.perm[sv];
        int j = i - 1;
        while (j >= 0 && a.perm[a.member[b + j]] > key) {
            a.member[b + j + 1] = a.member[b + j];
            --j;
        }
        a.member[b + j + 1] = sv;
    }
}

struct PaperDrawArgs {
    PaperArgs p;
    int* batch;                // [K][n_slots][P]
    int* n_pop;                // [n_slots]: N_I
    uint64_t seed;
    uint64_t step0;
    const uint64_t* step_dev;  // if set, the draw's first step is *step_dev + step0
    int K;
    int P;
};

constexpr int kPaperRuns = 256;  // x-runs of a stencil: 2 (2h+1)^2 <= 256, h <= 5

// The members of a stencil axis around cell c, ascending: cells p0..p0+l0-1
// then p1..p1+l1-1 (l1 = 0 without a periodic wrap).
__device__ __forceinline__ void paper_axis(int c, int nc, int h, int& p0, int& l0, int& p1, int& l1)
{
    p1 = 0;
    l1 = 0;
    if (2 * h + 1 >= nc) {
        p0 = 0;
        l0 = nc;
        return;
    }
    const int lo = c - h, hi = c + h;
    if (lo < 0) {
        p0 = 0;
        l0 = hi + 1;
        p1 = lo + nc;
        l1 = -lo;
    } else if (hi > nc - 1) {
        p0 = 0;
        l0 = hi - nc + 1;
        p1 = lo;
        l1 = nc - lo;
    } else {
        p0 = lo;
        l0 = 2 * h + 1;
    }
}

// One wavefront per paper cell: the stencil's x-runs (contiguous member
// positions) with their prefix counts in LDS, N_I = their total; then one
// lane per (particle, step) pair draws P positions k in [0, N_I) (Floyd on
// the same Philox stream as the shell draw) and maps each to its member by
// a binary search over the prefix counts.
template <int PMAX>
__global__ __launch_bounds__(256) void k_paper_draw(PaperDrawArgs d)
{
    __shared__ int s_start[4][kPaperRuns];
    __shared__ int s_pre[4][kPaperRuns];
    const PaperArgs& a = d.p;
    if (gated_off(a.gate)) return;
    const int lane = threadIdx.x & 63;
    const int w = rfl((int)(threadIdx.x >> 6));
    const int64_t cell = xcd_tile(blockIdx.x, gridDim.x) * 4 + w;
    if (cell >= a.n_cells) return;
    const int m = rfl(a.count[cell]);
    if (m == 0) return;
    const int b = rfl(a.start[cell]);
    const int r = rfl(a.cell_rep[cell]);
    const PaperGrid* G = a.grid + r;
    const int nc0 = rfl(G->nc[0]), nc1 = rfl(G->nc[1]), nc2 = rfl(G->nc[2]);
    const int h = rfl(G->h);
    const int64_t base = rfl(G->cell_base);
    const int64_t lc = cell - base;
    const int cx = (int)(lc % nc0);
    const int cy = (int)((lc / nc0) % nc1);
    const int cz = (int)(lc / ((int64_t)nc0 * nc1));
    int px0, lx0, px1, lx1, py0, ly0, py1, ly1, pz0, lz0, pz1, lz1;
    paper_axis(cx, nc0, h, px0, lx0, px1, lx1);
    paper_axis(cy, nc1, h, py0, ly0, py1, ly1);
    paper_axis(cz, nc2, h, pz0, lz0, pz1, lz1);
    const int nxr = lx1 > 0 ? 2 : 1;
    const int ny = ly0 + ly1;
    const int nruns = (lz0 + lz1) * ny * nxr;
    if (nruns > kPaperRuns || b < 0 || (int64_t)b + m > a.n_slots) {
        if (lane == 0) atomicOr(&a.flags[kFlagBadSlot], 16);
        return;
    }
    // run q = (z index, y index, x part); entries past the last run hold
    // the total, which the binary search relies on
    int carry = 0;
    bool bad = false;
#pragma unroll
    for (int k = 0; k < kPaperRuns / 64; ++k) {
        const int q = k * 64 + lane;
        int st = 0, len = 0;
        if (q < nruns) {
            const int xr = q % nxr;
            const int yz = q / nxr;
            const int yi = yz % ny;
            const int zi = yz / ny;
            const int zc = zi < lz0 ? pz0 + zi : pz1 + (zi - lz0);
            const int yc = yi < ly0 ? py0 + yi : py1 + (yi - ly0);
            const int px = xr == 0 ? px0 : px1;
            const int lx = xr == 0 ? lx0 : lx1;
            const int64_t row = base + ((int64_t)zc * nc1 + yc) * nc0;
            st = a.start[row + px];
            len = a.start[row + px + lx - 1] + a.count[row + px + lx - 1] - st;
            bad |= st < 0 || len < 0 || (int64_t)st + len > a.n_slots;
        }
        const int incl = wave_incl_scan(len);
        s_start[w][q] = st;
        s_pre[w][q] = carry + incl - len;
        carry += __builtin_amdgcn_readlane(incl, 63);
    }
    for (int t = lane; t < m; t += 64) bad |= (uint64_t)(uint32_t)a.member[b + t] >= (uint64_t)a.n_slots;
    if (__ballot(bad)) {
        if (lane == 0) atomicOr(&a.flags[kFlagBadSlot], 16);
        return;
    }
    const int NI = rfl(carry);
    for (int t = lane; t < m; t += 64) d.n_pop[a.member[b + t]] = NI;
    wave_lds_fence();
    const uint64_t s0 = d.step_dev ? *d.step_dev + d.step0 : d.step0;
    const int P = d.P;
    const bool small = NI <= P;
    const int64_t id_base = rfl(a.rep[r].id_base);
    const int pairs = m * d.K;
    for (int pb = 0; pb < pairs; pb += 64) {
        const int pr = pb + lane;
        if (pr >= pairs) continue;
        const int ii = pr / d.K;
        const int rr = pr - ii * d.K;
        const int si = a.member[b + ii];
        const uint32_t pid = (uint32_t)(a.perm[si] - id_base);
        uint32_t S[PMAX];
        floyd_draw<PMAX>(S, d.seed, pid, (uint32_t)(s0 + rr), (uint32_t)r, P, small ? P + 1 : NI);
        int* out = d.batch + batch_index(rr, si, 0, a.n_slots, P);
        int val[PMAX];
#pragma unroll
        for (int qq = 0; qq < PMAX; ++qq) {
            val[qq] = si;
            if (qq < P) {
                const uint32_t k = small ? (uint32_t)qq : S[qq];
                if ((int)k < NI) {
                    int q = 0;
#pragma unroll
                    for (int st = kPaperRuns / 2; st > 0; st >>= 1)
                        if (s_pre[w][q + st] <= (int)k) q += st;
                    const int j = a.member[s_start[w][q] + (int)k - s_pre[w][q]];
                    val[qq] = (uint64_t)(uint32_t)j < (uint64_t)a.n_slots ? j : si;
                }
            }
        }
        if ((P & 1) == 0) {
#pragma unroll
            for (int qq = 0; qq < PMAX; qq += 2)
                if (qq < P) *reinterpret_cast<int2*>(out + qq) = make_int2(val[qq], val[qq + 1]);
        } else {
#pragma unroll
            for (int qq = 0; qq < PMAX; ++qq)
                if (qq < P) out[qq] = val[qq];
        }
    }
}

// ---------------------------------------------------------------------------
// Batch pre-draw: for steps step0 .. step0+K-1 the partners of every
// particle's batch, gathered from its shell row (bit-identical to the draw
// the inline force kernel makes).
struct DrawArgs {
    const DevReplica* rep;
    const int* slice_rep;
    const int* perm;
    const int* shell;
    const int* shell_len;
    int cap_shell;
    int64_t n_slots;
    int64_t n_slices;
    uint64_t seed;
    uint64_t step0;
    int K;
    int P;
    int* batch;  // [K][n_slots][P]
};

template <int PMAX>
__global__ __launch_bounds__(256) void k_predraw(DrawArgs a)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((slot >> 6) >= a.n_slices) return;
    const int rep_id = a.slice_rep[slot >> 6];
    const DevReplica& R = a.rep[rep_id];
    if (slot - R.slot_base >= R.n) return;
    const int n = a.shell_len[slot];
    const uint32_t pid = (uint32_t)(a.perm[slot] - R.id_base);
    const int P = a.P;
    for (int rr = 0; rr < a.K; ++rr) {
        if (n <= P) {
            for (int q = 0; q < n; ++q)
                a.batch[batch_index(rr, slot, q, a.n_slots, P)] = a.shell[ell(slot, q, a.cap_shell)];
        } else {
            uint32_t S[PMAX];
            floyd_draw<PMAX>(S, a.seed, pid, (uint32_t)(a.step0 + rr), (uint32_t)rep_id, P, n);
#pragma unroll
            for (int q = 0; q < PMAX; ++q)
                if (q < P) a.batch[batch_index(rr, slot, q, a.n_slots, P)] = a.shell[ell(slot, (int)S[q], a.cap_shell)];
        }
    }
}

// ---------------------------------------------------------------------------
// Force kernel.  One lane per particle slot, one wavefront per slice of 64
// cell-sorted particles.  Core rows are summed exactly (r < r_s); the shell
// batch (drawn inline with Philox + Floyd, or pre-drawn) is summed over
// r_s <= r < r_c and scaled by n_i/P.  Each wavefront also leaves its sums
// of F, U and W for the per-replica reduction.
struct ForceArgs {
    const DevReplica* rep;
    const int* slice_rep;
    const int* perm;
    const double4* xs;
    const int* core;
    const int* core_len;
    int cap_core;
    const int* shell;      // shell list (inline) or full list (full mode)
    const int* shell_len;
    int cap_shell;
    const int* batch;      // pre-drawn: [n_slots][P] for this step, or with bstep the
                           // [K][n_slots][P] batches drawn from step *bstep on
    int64_t n_slots;
    int64_t n_slices;
    double rs2, rc2, uc;   // core radius^2, cut-off^2, LJ energy at the cut-off
    double uce;            // erfc(alpha r_c)/r_c (energy shift per unit charge product)
    double alpha;
    uint64_t seed;
    uint64_t step;
    const uint64_t* step_dev;  // if set, the step counter is *step_dev + step
    int P;
    double* f;             // [3][n_slots]
    double* partial;       // [5][n_slices]
    int64_t vblocks;       // work tiles of 256 lanes; a launch of fewer blocks (a
                           // persistent grid) walks them in steps of its size
    const uint64_t* bstep; // step of the build whose batches `batch` holds (null: this step's)
    uint64_t* gate_clear;  // rebuild gate to reset for the next step (null: none)
    // mixed precision: fixed-point copy of the positions (fixq), one 16-byte
    // load per neighbour; a pair whose r^2 lies within `guard` of a bound it
    // is tested against is classified from the FP64 positions
    const int4* xq;
    double guard;
    const TypeTable* types;  // pair constants of particle types (kPairTyped)
    // Filtered core rows (one lane per particle, rows of at most 64
    // entries, runs with rebuilds on displacement; null fgate: off).  With
    // *fgate set, the launch reads the built rows, writes the partners with
    // r^2 < filt2 = (r_s + d_f)^2 (with types the pair's (r_s sigma_ab +
    // d_f)^2 from the table) to fcore / fcore_len in row order and the
    // positions to xf; otherwise it reads fcore.  The integrator raises
    // *fgate at every rebuild and when a particle has moved more than d_f/2
    // (less a rounding margin) from xf, so a dropped partner stays at
    // r >= r_s, whose term is an exact zero: the sums are those of the
    // built rows bit for bit.
    const uint64_t* fgate;
    int* fcore;
    int* fcore_len;
    float* xf;             // [3][n_slots]
    double filt2;
};

// This step's pre-drawn batches (the force evaluation's step relative to
// the build that drew them, when the build step is known on the device
// only), and the reset of the rebuild gate by the first thread of the launch.
__device__ __forceinline__ const int* step_batches(const ForceArgs& a)
{
    if (!a.bstep) return a.batch;
    const uint64_t st = a.step_dev ? *a.step_dev + a.step : a.step;
    return a.batch + (int64_t)(st - *a.bstep) * a.P * a.n_slots;
}

__device__ __forceinline__ void force_prologue(const ForceArgs& a)
{
    if (a.gate_clear && blockIdx.x == 0 && threadIdx.x == 0) *a.gate_clear = 0;
}

template <int PREC, bool ERFC>
__device__ __forceinline__ void pair_term(double r2, double qq, double alpha, double& fm, double& u)
{
    LJ<PREC>::eval(r2, fm, u);
    if (ERFC) {
        double fe, ue;
        Erfc<PREC>::eval(r2, qq, alpha, fe, ue);
        fm += fe;
        u += ue;
    }
}

// Accumulates the pair terms of U partners whose indices and positions were
// fetched together (all gathers in flight before any arithmetic).  A partner
// counts when `live` and lo2 <= r^2 < hi2; masked partners take r^2 = 1 so
// that no infinities are formed, and contribute exact zeros.
struct Acc {
    double fx, fy, fz, e, w;
};

// Typed pairs (PAIR == kPairTyped) take lo2 / hi2 from the pair's radii by
// `zone` (core [0, r_s^2), shell [r_s^2, r_c^2), full [0, r_c^2)) and its
// LJ constants from `tp` (the type table in LDS).

__device__ __forceinline__ void zone_bounds(const TypePair& pp, int zone, double& lo2, double& hi2)
{
    lo2 = zone == kZoneShell ? pp.rs2 : -1.0;
    hi2 = zone == kZoneCore ? pp.rs2 : pp.rc2;
}

template <int PREC, bool ENERGY, int PAIR, int U>
__device__ __forceinline__ void accumulate(const double4& xi, const double4 (&xj)[U], const bool (&live)[U],
                                           double lo2, double hi2, const DevReplica& R,
                                           const ForceArgs& a, Acc& acc, const TypePair* tp, int zone,
                                           double keep2, uint32_t& keep)
{
    constexpr bool ERFC = PAIR == kPairErfc;
    if constexpr (PAIR == kPairTyped) {
        const TypePair* row = tp + type_of(xi.w) * kMaxTypes;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const Delta d = delta(xi, xj[u], R);
            const TypePair& pp = row[type_of(xj[u].w)];
            // the filter threshold is the pair's own (keep2 > 0: filtering)
            keep |= (live[u] && d.r2 < (keep2 > 0.0 ? pp.filt2 : -1.0) ? 1u : 0u) << u;
            double lo, hi;
            zone_bounds(pp, zone, lo, hi);
            const bool in = live[u] && d.r2 >= lo && d.r2 < hi;
            const double r2 = in ? d.r2 : 1.0;
            double fm, en;
            LJt<PREC>::eval(r2, pp.eps24, pp.eps4, pp.sig2, fm, en);
            fm = in ? fm : 0.0;
            acc.fx += fm * d.x;
            acc.fy += fm * d.y;
            acc.fz += fm * d.z;
            if (ENERGY) {
                acc.e += in ? en - pp.uc : 0.0;
                acc.w += fm * r2;
            }
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const Delta d = delta(xi, xj[u], R);
        keep |= (live[u] && d.r2 < keep2 ? 1u : 0u) << u;
        const bool in = live[u] && d.r2 >= lo2 && d.r2 < hi2;
        const double r2 = in ? d.r2 : 1.0;
        double fm, en;
        pair_term<PREC, ERFC>(r2, xi.w * xj[u].w, a.alpha, fm, en);
        fm = in ? fm : 0.0;
        acc.fx += fm * d.x;
        acc.fy += fm * d.y;
        acc.fz += fm * d.z;
        if (ENERGY) {
            const double shift = ERFC ? a.uc + xi.w * xj[u].w * a.uce : a.uc;
            acc.e += in ? en - shift : 0.0;
            acc.w += fm * r2;
        }
    }
}

// Mixed precision: the displacement from the fixed-point copy (an exact
// integer difference, scaled by L 2^-32 in FP64), the pair term in FP32 and
// the force accumulated in FP64.  Classification stays that of the FP64
// positions: |r^2 - r^2_FP64| <= guard (host bound from the two roundings),
// so a pair farther than the guard from both bounds falls on the same side,
// and one within it is decided from the FP64 positions.
template <bool ENERGY, int PAIR, int U>
__device__ __forceinline__ void accumulate_mixed(const double4& xi, const int4& qi, const int4 (&xj)[U],
                                                 const int (&j)[U], const bool (&live)[U], double lo2,
                                                 double hi2, const DevReplica& R, const ForceArgs& a, Acc& acc,
                                                 const TypePair* tp, int zone, double keep2, uint32_t& keep)
{
    constexpr bool ERFC = PAIR == kPairErfc;
    constexpr double k2m32 = 2.3283064365386962890625e-10;  // 2^-32
    const double s0 = R.L[0] * k2m32, s1 = R.L[1] * k2m32, s2 = R.L[2] * k2m32;
    if constexpr (PAIR == kPairTyped) {
        const TypePair* row = tp + type_of((double)__int_as_float(qi.w)) * kMaxTypes;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double dx = (double)(int)((uint32_t)qi.x - (uint32_t)xj[u].x) * s0;
            const double dy = (double)(int)((uint32_t)qi.y - (uint32_t)xj[u].y) * s1;
            const double dz = (double)(int)((uint32_t)qi.z - (uint32_t)xj[u].z) * s2;
            const double r2q = fma(dz, dz, fma(dy, dy, dx * dx));
            const TypePair& pp = row[type_of((double)__int_as_float(xj[u].w))];
            keep |= (live[u] && r2q < (keep2 > 0.0 ? pp.filt2 : -1.0) ? 1u : 0u) << u;
            double lo, hi;
            zone_bounds(pp, zone, lo, hi);
            bool in = live[u] && r2q >= lo && r2q < hi;
            if (live[u] && (fabs(r2q - lo) <= a.guard || fabs(r2q - hi) <= a.guard)) {
                const Delta d = delta(xi, a.xs[j[u]], R);
                in = d.r2 >= lo && d.r2 < hi;
            }
            const double r2 = in ? r2q : 1.0;
            double fm, en;
            LJt<kMixed>::eval(r2, pp.eps24, pp.eps4, pp.sig2, fm, en);
            fm = in ? fm : 0.0;
            acc.fx += fm * dx;
            acc.fy += fm * dy;
            acc.fz += fm * dz;
            if (ENERGY) {
                acc.e += in ? en - pp.uc : 0.0;
                acc.w += fm * r2;
            }
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const double dx = (double)(int)((uint32_t)qi.x - (uint32_t)xj[u].x) * s0;
        const double dy = (double)(int)((uint32_t)qi.y - (uint32_t)xj[u].y) * s1;
        const double dz = (double)(int)((uint32_t)qi.z - (uint32_t)xj[u].z) * s2;
        const double r2q = fma(dz, dz, fma(dy, dy, dx * dx));
        keep |= (live[u] && r2q < keep2 ? 1u : 0u) << u;
        bool in = live[u] && r2q >= lo2 && r2q < hi2;
        if (live[u] && (fabs(r2q - lo2) <= a.guard || fabs(r2q - hi2) <= a.guard)) {
            const Delta d = delta(xi, a.xs[j[u]], R);
            in = d.r2 >= lo2 && d.r2 < hi2;
        }
        const double r2 = in ? r2q : 1.0;
        const double qq = ERFC ? (double)__int_as_float(qi.w) * (double)__int_as_float(xj[u].w) : 0.0;
        double fm, en;
        pair_term<kMixed, ERFC>(r2, qq, a.alpha, fm, en);
        fm = in ? fm : 0.0;
        acc.fx += fm * dx;
        acc.fy += fm * dy;
        acc.fz += fm * dz;
        if (ENERGY) {
            const double shift = ERFC ? a.uc + qq * a.uce : a.uc;
            acc.e += in ? en - shift : 0.0;
            acc.w += fm * r2;
        }
    }
}

// Gathers the positions of U partners (all loads in flight first) and
// accumulates their pair terms: FP64 positions, or the fixed-point copy
// (mixed).  Bit u of `keep` is set for a live partner with r^2 < keep2 (as
// classified).
template <int PREC, bool ENERGY, int PAIR, int U>
__device__ __forceinline__ void gather_accumulate(const ForceArgs& a, const double4& xi, const int4& qi,
                                                  const int (&j)[U], const bool (&live)[U], double lo2,
                                                  double hi2, const DevReplica& R, Acc& acc,
                                                  const TypePair* tp, int zone, double keep2, uint32_t& keep)
{
    if constexpr (PREC == kMixed) {
        int4 xj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xj[u] = a.xq[j[u]];
        accumulate_mixed<ENERGY, PAIR, U>(xi, qi, xj, j, live, lo2, hi2, R, a, acc, tp, zone, keep2, keep);
    } else {
        double4 xj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xj[u] = a.xs[j[u]];
        accumulate<PREC, ENERGY, PAIR, U>(xi, xj, live, lo2, hi2, R, a, acc, tp, zone, keep2, keep);
    }
}

template <int PREC, bool ENERGY, int PAIR, int U>
__device__ __forceinline__ void gather_accumulate(const ForceArgs& a, const double4& xi, const int4& qi,
                                                  const int (&j)[U], const bool (&live)[U], double lo2,
                                                  double hi2, const DevReplica& R, Acc& acc,
                                                  const TypePair* tp, int zone)
{
    uint32_t keep = 0;
    gather_accumulate<PREC, ENERGY, PAIR, U>(a, xi, qi, j, live, lo2, hi2, R, acc, tp, zone, -1.0, keep);
}

// The type table of a force launch, copied into LDS by the block.
__device__ __forceinline__ void load_type_table(const ForceArgs& a, TypePair* s_tp)
{
    constexpr int words = (int)(sizeof(TypePair) * kMaxTypes * kMaxTypes / 8);
    const double* src = reinterpret_cast<const double*>(a.types->p);
    double* dst = reinterpret_cast<double*>(s_tp);
    for (int k = threadIdx.x; k < words; k += blockDim.x) dst[k] = src[k];
    __syncthreads();
}

// neighbours per lane in flight at one lane per particle: 6 for the
// 16-byte fixed-point records (106 against 109 µs at 4 on the N = 10^6
// fluid; 8 costs occupancy), 4 for the FP64 double4 records
template <int PREC>
constexpr int kGatherBatch = PREC == kMixed ? 6 : 4;

// LDS entries per lane of the filtering instance (its dynamic LDS holds
// min(cap_core, kKeepLds) of them)
constexpr int kKeepLds = 32;

template <int PREC, int MODE, bool ENERGY, int PAIR, int PMAX, bool FILT>
__device__ __forceinline__ void force_tile(const ForceArgs& a, int64_t tile, uint32_t* s_pos, const TypePair* tp,
                                           int* s_keep)
{
    // the filtering instance keeps at most 5 neighbours in flight, which
    // holds it to 4 waves per SIMD with its staging
    constexpr int U = FILT && kGatherBatch<PREC> > 5 ? 5 : kGatherBatch<PREC>;
    const int64_t slot = tile * blockDim.x + threadIdx.x;
    const int64_t slice = slot >> 6;
    if (slice >= a.n_slices) return;
    const int rep_id = a.slice_rep[slice];
    const DevReplica& R = a.rep[rep_id];
    const bool real = slot - R.slot_base < R.n;
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0, w = 0.0;
    if (real) {
        const double4 xi = a.xs[slot];
        const int4 qi = PREC == kMixed ? a.xq[slot] : make_int4(0, 0, 0, 0);
        // pre-drawn batches: the shell size and the first group's batch
        // entries are loaded with the core rows, so that the shell sum
        // starts with its indices at hand
        int bn[U];
        int nb = 0;
        const int* brow = nullptr;
        if constexpr (MODE == kShellPredraw) {
            nb = min(a.shell_len[slot], a.P);
            brow = step_batches(a) + slot * a.P;
#pragma unroll
            for (int u = 0; u < U; ++u) bn[u] = u < nb ? brow[u] : (int)slot;
        }
        // core rows (or the full list in direct-truncation mode): r < cut
        Acc c = {0.0, 0.0, 0.0, 0.0, 0.0};
        {
            const double cut = MODE == kShellNone ? a.rc2 : a.rs2;
            // filtered core rows (see ForceArgs): FILT reads the built rows
            // and writes the filtered ones, the other instance reads those
            constexpr bool filt = FILT && MODE != kShellNone;
            const bool use_f = !FILT && MODE != kShellNone && a.fgate != nullptr;
            const int len = use_f ? a.fcore_len[slot] : a.core_len[slot];
            const int* row = (use_f ? a.fcore : a.core) + ell(slot, 0, a.cap_core);
            int nf = 0;
            // the row entries of the next group are loaded before this
            // group's gathers, so their latency overlaps the gathers'
            int jn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) jn[u] = u < len ? row[(int64_t)u * 64] : (int)slot;
            for (int k = 0; k < len; k += U) {
                int j[U];
                bool live[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    live[u] = k + u < len;
                    j[u] = jn[u];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) jn[u] = k + U + u < len ? row[(int64_t)(k + U + u) * 64] : (int)slot;
                uint32_t keep = 0;
                gather_accumulate<PREC, ENERGY, PAIR, U>(a, xi, qi, j, live, -1.0, cut, R, c, tp,
                                                         MODE == kShellNone ? kZoneFull : kZoneCore,
                                                         filt ? a.filt2 : -1.0, keep);
                if constexpr (filt) {
                    // the first kKeepLds kept partners go to this lane's
                    // column of LDS (entry q at q * blockDim + lane: no bank
                    // conflicts), any further ones straight to the row
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if ((keep >> u) & 1u) {
                            if (nf < kKeepLds) s_keep[nf * (int)blockDim.x + (int)threadIdx.x] = j[u];
                            else a.fcore[ell(slot, nf, a.cap_core)] = j[u];
                            ++nf;
                        }
                    }
                }
            }
            if constexpr (filt) {
                // entry q of every lane's filtered row in one store: whole
                // cache lines of the sliced rows
                int* frow = a.fcore + ell(slot, 0, a.cap_core);
                const int nl = nf < kKeepLds ? nf : kKeepLds;
                for (int q = 0; q < nl; ++q) frow[(int64_t)q * 64] = s_keep[q * (int)blockDim.x + (int)threadIdx.x];
                a.fcore_len[slot] = nf;
                a.xf[slot] = (float)xi.x;
                a.xf[a.n_slots + slot] = (float)xi.y;
                a.xf[2 * a.n_slots + slot] = (float)xi.z;
            }
        }
        if (MODE != kShellNone) {
            const int n = a.shell_len[slot];
            const int P = a.P;
            const int cnt = n < P ? n : P;
            const double scale = n > P ? (double)n / (double)P : 1.0;
            if (MODE == kShellInline && n > P) {
                uint32_t S[PMAX];
                const uint32_t pid = (uint32_t)(a.perm[slot] - R.id_base);
                const uint64_t st = a.step_dev ? *a.step_dev + a.step : a.step;
                floyd_draw<PMAX>(S, a.seed, pid, (uint32_t)st, (uint32_t)rep_id, P, n);
#pragma unroll
                for (int q = 0; q < PMAX; ++q) s_pos[q * 256 + threadIdx.x] = S[q];
            }
            Acc sh = {0.0, 0.0, 0.0, 0.0, 0.0};
            const int* srow = a.shell + ell(slot, 0, a.cap_shell);
            for (int m = 0; m < cnt; m += U) {
                int j[U];
                bool live[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    live[u] = m + u < cnt;
                    int jj = (int)slot;
                    if constexpr (MODE == kShellInline) {
                        if (live[u]) {
                            const int kq = n > P ? (int)s_pos[(m + u) * 256 + threadIdx.x] : m + u;
                            jj = srow[(int64_t)kq * 64];
                        }
                    } else {
                        // a batch entry outside the slots (never written)
                        // reads the particle itself, whose pair term is zero
                        jj = bn[u];
                        if ((uint64_t)(uint32_t)jj >= (uint64_t)a.n_slots) jj = (int)slot;
                    }
                    j[u] = jj;
                }
                if constexpr (MODE == kShellPredraw) {
#pragma unroll
                    for (int u = 0; u < U; ++u) bn[u] = m + U + u < nb ? brow[m + U + u] : (int)slot;
                }
                gather_accumulate<PREC, ENERGY, PAIR, U>(a, xi, qi, j, live, a.rs2, a.rc2, R, sh, tp, kZoneShell);
            }
            fx = c.fx + scale * sh.fx;
            fy = c.fy + scale * sh.fy;
            fz = c.fz + scale * sh.fz;
            if (ENERGY) {
                e = 0.5 * (c.e + scale * sh.e);
                w = 0.5 * (c.w + scale * sh.w);
            }
        } else {
            fx = c.fx;
            fy = c.fy;
            fz = c.fz;
            if (ENERGY) {
                e = 0.5 * c.e;
                w = 0.5 * c.w;
            }
        }
    }
    a.f[slot] = fx;
    a.f[a.n_slots + slot] = fy;
    a.f[2 * a.n_slots + slot] = fz;
    const double tx = wave_sum(fx);
    const double ty = wave_sum(fy);
    const double tz = wave_sum(fz);
    double te = 0.0, tw = 0.0;
    if (ENERGY) {
        te = wave_sum(e);
        tw = wave_sum(w);
    }
    if ((threadIdx.x & 63) == 0) {
        a.partial[slice] = tx;
        a.partial[a.n_slices + slice] = ty;
        a.partial[2 * a.n_slices + slice] = tz;
        a.partial[3 * a.n_slices + slice] = te;
        a.partial[4 * a.n_slices + slice] = tw;
    }
}

// Force kernel with LPP lanes per particle (LPP = 2 or 4; pre-drawn
// batches or the full list).  A wavefront covers 64/LPP consecutive slots;
// lane l of a particle takes row entries l, l+LPP, ...  The core and shell
// sums are reduced over the particle's lanes with DPP quad permutations, in
// a fixed order, and combined as F = F_core + scale * F_shell by lane 0.
// More, shorter wavefronts keep more gathers in flight than one lane per
// particle.
// One tile per block, or (persistent grid) tiles b, b + gridDim.x, ... in
// turn; the grid is a multiple of 8 blocks, so a block keeps to its XCD's
// tiles of the XCD map.
// With filtered core rows (a.fgate set) two instances are queued per
// step: FILT works when the filter gate is raised (built rows in, filtered
// rows out, staged through cap_core x 256 ints of dynamic LDS), the other
// when it is clear (filtered rows in); each returns at once otherwise.
// Separate instances keep the filtering's registers and LDS out of the
// kernel that runs on most steps.
template <int PREC, int MODE, bool ENERGY, int PAIR, int PMAX, bool FILT = false>
__global__ __launch_bounds__(256) void k_forces(ForceArgs a)
{
    if (a.fgate && (*a.fgate != 0) != FILT) return;
    __shared__ uint32_t s_pos[MODE == kShellInline ? PMAX * 256 : 1];
    __shared__ TypePair s_tp[PAIR == kPairTyped ? kMaxTypes * kMaxTypes : 1];
    extern __shared__ int s_keep[];
    force_prologue(a);
    if constexpr (PAIR == kPairTyped) load_type_table(a, s_tp);
    for (int64_t b = blockIdx.x; b < a.vblocks; b += gridDim.x)
        force_tile<PREC, MODE, ENERGY, PAIR, PMAX, FILT>(a, xcd_tile(b, a.vblocks), s_pos, s_tp, s_keep);
}

template <int CTRL>
__device__ __forceinline__ double dpp_quad_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int LPP>
__device__ __forceinline__ double group_sum(double v)
{
    if (LPP >= 2) v += dpp_quad_f64<0xB1>(v);  // quad_perm [1,0,3,2]
    if (LPP >= 4) v += dpp_quad_f64<0x4E>(v);  // quad_perm [2,3,0,1]
    return v;
}

template <int PREC, int MODE, bool ENERGY, int PAIR, int LPP>
__device__ __forceinline__ void force_tile_lpp(const ForceArgs& a, int64_t tile, const TypePair* tp)
{
    constexpr int U = (LPP == 2 && PAIR == kPairLJ) ? 4 : 2;  // neighbours per lane in flight
    const int64_t g = tile * blockDim.x + threadIdx.x;
    const int64_t slot = g / LPP;
    const int l = (int)(g % LPP);
    const int64_t slice = slot >> 6;
    if (slice >= a.n_slices) return;
    const int rep_id = a.slice_rep[slice];
    const DevReplica& R = a.rep[rep_id];
    const bool real = slot - R.slot_base < R.n;
    Acc c = {0.0, 0.0, 0.0, 0.0, 0.0};
    Acc sh = {0.0, 0.0, 0.0, 0.0, 0.0};
    double scale = 1.0;
    if (real) {
        const double4 xi = a.xs[slot];
        const int4 qi = PREC == kMixed ? a.xq[slot] : make_int4(0, 0, 0, 0);
        {
            const double cut = MODE == kShellNone ? a.rc2 : a.rs2;
            const int len = a.core_len[slot];
            const int* row = a.core + ell(slot, 0, a.cap_core);
            // next group's row entries in flight during this group's gathers
            // (not for FP64 records at 4 lanes, whose two loads per
            // neighbour already fill the memory pipeline: 9% slower there)
            constexpr bool PF = PREC == kMixed || LPP <= 2;
            int jn[U];
#pragma unroll
            for (int u = 0; u < U; ++u) jn[u] = l + u * LPP < len ? row[(int64_t)(l + u * LPP) * 64] : (int)slot;
            for (int k = l; k < len; k += U * LPP) {
                int j[U];
                bool live[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    live[u] = k + u * LPP < len;
                    j[u] = PF ? jn[u] : (live[u] ? row[(int64_t)(k + u * LPP) * 64] : (int)slot);
                }
                if constexpr (PF) {
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int kn = k + U * LPP + u * LPP;
                        jn[u] = kn < len ? row[(int64_t)kn * 64] : (int)slot;
                    }
                }
                gather_accumulate<PREC, ENERGY, PAIR, U>(a, xi, qi, j, live, -1.0, cut, R, c, tp,
                                                         MODE == kShellNone ? kZoneFull : kZoneCore);
            }
        }
        if (MODE != kShellNone) {
            const int n = a.shell_len[slot];
            const int P = a.P;
            const int cnt = n < P ? n : P;
            scale = n > P ? (double)n / (double)P : 1.0;
            const int* brow = step_batches(a) + slot * P;
            for (int m = l; m < cnt; m += U * LPP) {
                int j[U];
                bool live[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    live[u] = m + u * LPP < cnt;
                    j[u] = live[u] ? brow[m + u * LPP] : (int)slot;
                    // a batch entry outside the slots (never written) reads the
                    // particle itself, whose pair term is zero
                    if ((uint64_t)(uint32_t)j[u] >= (uint64_t)a.n_slots) j[u] = (int)slot;
                }
                gather_accumulate<PREC, ENERGY, PAIR, U>(a, xi, qi, j, live, a.rs2, a.rc2, R, sh, tp, kZoneShell);
            }
        }
    }
    c.fx = group_sum<LPP>(c.fx);
    c.fy = group_sum<LPP>(c.fy);
    c.fz = group_sum<LPP>(c.fz);
    if (MODE != kShellNone) {
        sh.fx = group_sum<LPP>(sh.fx);
        sh.fy = group_sum<LPP>(sh.fy);
        sh.fz = group_sum<LPP>(sh.fz);
    }
    double fx = c.fx, fy = c.fy, fz = c.fz, e = 0.0, w = 0.0;
    if (MODE != kShellNone) {
        fx = c.fx + scale * sh.fx;
        fy = c.fy + scale * sh.fy;
        fz = c.fz + scale * sh.fz;
    }
    if (ENERGY) {
        c.e = group_sum<LPP>(c.e);
        c.w = group_sum<LPP>(c.w);
        if (MODE != kShellNone) {
            sh.e = group_sum<LPP>(sh.e);
            sh.w = group_sum<LPP>(sh.w);
            e = 0.5 * (c.e + scale * sh.e);
            w = 0.5 * (c.w + scale * sh.w);
        } else {
            e = 0.5 * c.e;
            w = 0.5 * c.w;
        }
    }
    const bool lead = l == 0;
    if (lead) {
        a.f[slot] = fx;
        a.f[a.n_slots + slot] = fy;
        a.f[2 * a.n_slots + slot] = fz;
    }
    // per-slice partials: one wavefront covers 64/LPP slots, so LPP
    // wavefronts share a slice; each adds its part into the slice's entry in
    // a fixed order via a per-wave slot [slice][sub]
    const double tx = wave_sum(lead ? fx : 0.0);
    const double ty = wave_sum(lead ? fy : 0.0);
    const double tz = wave_sum(lead ? fz : 0.0);
    double te = 0.0, tw = 0.0;
    if (ENERGY) {
        te = wave_sum(lead ? e : 0.0);
        tw = wave_sum(lead ? w : 0.0);
    }
    if ((threadIdx.x & 63) == 0) {
        const int64_t wv = g >> 6;  // wavefront index: LPP per slice
        const int64_t ns = a.n_slices * LPP;
        a.partial[wv] = tx;
        a.partial[ns + wv] = ty;
        a.partial[2 * ns + wv] = tz;
        a.partial[3 * ns + wv] = te;
        a.partial[4 * ns + wv] = tw;
    }
}

template <int PREC, int MODE, bool ENERGY, int PAIR, int LPP>
__global__ __launch_bounds__(256) void k_forces_lpp(ForceArgs a)
{
    __shared__ TypePair s_tp[PAIR == kPairTyped ? kMaxTypes * kMaxTypes : 1];
    force_prologue(a);
    if constexpr (PAIR == kPairTyped) load_type_table(a, s_tp);
    for (int64_t b = blockIdx.x; b < a.vblocks; b += gridDim.x)
        force_tile_lpp<PREC, MODE, ENERGY, PAIR, LPP>(a, xcd_tile(b, a.vblocks), s_tp);
}

// Per-replica sums of the wavefront partials in a fixed order, so the result
// does not depend on scheduling.  Stage 1: block (b, r) sums entries
// b*256 .. of replica r into part2[r][b].  Stage 2: one block per replica
// adds its part2 entries (no atomics: all blocks of stage 1 are done when
// stage 2 starts).  rep_sum[8r + q], q = Fx, Fy, Fz, U, W.
constexpr int kReduceSlicesPerBlock = 256;

__global__ __launch_bounds__(256) void k_reduce(const DevReplica* rep, const double* partial,
                                               int64_t n_slices, int per, int blocks_per_rep,
                                               double* part2, uint64_t* fgate_clear)
{
    __shared__ double lds[5][4];
    const int r = blockIdx.y;
    const int b = blockIdx.x;
    // the filter gate of the force launch before is reset for the next step
    if (fgate_clear && r == 0 && b == 0 && threadIdx.x == 0) *fgate_clear = 0;
    const DevReplica& R = rep[r];
    // `per` partial entries per slice (one per wavefront of the force kernel)
    const int64_t s0 = (R.slot_base >> 6) * per;
    const int64_t ns = ((R.n + 63) >> 6) * per;
    const int64_t stride = n_slices * per;
    const int64_t lo = (int64_t)b * kReduceSlicesPerBlock;
    if (lo >= ns) return;
    const int64_t hi = min(ns, lo + kReduceSlicesPerBlock);
    const int wv = threadIdx.x >> 6;
    for (int q = 0; q < 5; ++q) {
        const int64_t s = lo + threadIdx.x;
        double acc = s < hi ? partial[q * stride + s0 + s] : 0.0;
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) lds[q][wv] = acc;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int q = threadIdx.x;
        part2[((int64_t)r * blocks_per_rep + b) * 5 + q] = ((lds[q][0] + lds[q][1]) + lds[q][2]) + lds[q][3];
    }
}

__global__ __launch_bounds__(256) void k_reduce_final(const DevReplica* rep, int per, int blocks_per_rep,
                                                     const double* part2, double* rep_sum)
{
    __shared__ double lds[5][4];
    const int r = blockIdx.x;
    const DevReplica& R = rep[r];
    const int64_t ns = ((R.n + 63) >> 6) * per;
    const int nb = (int)((ns + kReduceSlicesPerBlock - 1) / kReduceSlicesPerBlock);
    const int wv = threadIdx.x >> 6;
    for (int q = 0; q < 5; ++q) {
        double acc = 0.0;
        for (int k = threadIdx.x; k < nb; k += blockDim.x) acc += part2[((int64_t)r * blocks_per_rep + k) * 5 + q];
        acc = wave_sum(acc);
        if ((threadIdx.x & 63) == 0) lds[q][wv] = acc;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int q = threadIdx.x;
        rep_sum[8 * r + q] = ((lds[q][0] + lds[q][1]) + lds[q][2]) + lds[q][3];
    }
}

// ---------------------------------------------------------------------------
// Velocity Verlet (unit mass) on the sorted state; F' = F - F_cor where
// F_cor = (sum_i F_i)/N_r is the replica's average net force.
//   first: v += h F';           x += dt v
//   mid:   v += h F'; v += h F'; x += dt v   (end of one step + start of next)
//   last:  v += h F'
// A mid step given `pending` takes the closing half-kick only when
// *pending != 0: a captured list lifetime then serves both a state whose
// velocities await that half-kick and one whose velocities are complete.
// The skin monitor flags a particle that moved more than skin/2 since the
// last build: at the end of a run here, at every rebuild in k_bin_count.
struct IntArgs {
    const DevReplica* rep;
    const int* slice_rep;
    const double* rep_sum;
    double4* xs;
    double* vs;
    const double* f;
    const double* xb;
    int64_t n_slots;
    int64_t n_slices;
    double h, dt;
    int momentum_fix;
    double half_skin2;
    int* flags;
    // Langevin thermostat (BAOAB) when `langevin`: v <- oc v + osig[r] xi
    int langevin;
    double oc;
    const double* osig;    // per replica sqrt(kT (1 - oc^2))
    const int* perm;
    uint64_t seed;
    uint64_t step;             // force evaluation the step leads to
    const uint64_t* step_dev;  // if set, the step is *step_dev + step
    const uint64_t* pending;   // mid steps: closing half-kick only if *pending (null: always)
    // rebuild on displacement: after the drift, *gate = 1 if some particle
    // moved more than skin/2 since the last build (xb) or the lifetime since
    // that build (*bstep) reached max_life steps (null: fixed lifetimes)
    uint64_t* gate;
    const uint64_t* bstep;
    int64_t max_life;
    int4* xq;                  // may be null: fixed-point copy of the positions, kept in step
    // filtered core rows (null: off): *fgate = 1 with every rebuild and when
    // a particle is farther than sqrt(fhalf2) from its position xf at the
    // last filtering, compared in FP32
    uint64_t* fgate;
    const float* xf;
    float fhalf2;
};

// The three standard normal numbers of the Ornstein-Uhlenbeck step of
// particle pid (replica-local ID) before force evaluation `step`: the
// Philox block with counter (pid, step mod 2^32, replica, 2^31) -- batch
// draws use the blocks below 2^31 -- and Box-Muller (1958) on its two word
// pairs, each word w taken as the uniform (w + 1/2) 2^-32 in (0, 1).
constexpr uint32_t kNoiseBlock = 0x80000000u;

__device__ __forceinline__ void langevin_noise(uint64_t seed, uint32_t pid, uint32_t step, uint32_t replica,
                                               double g[3])
{
    uint32_t w0 = pid, w1 = step, w2 = replica, w3 = kNoiseBlock;
    philox4x32_10(w0, w1, w2, w3, (uint32_t)seed, (uint32_t)(seed >> 32));
    constexpr double kTwoM32 = 2.3283064365386962890625e-10;  // 2^-32
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const double u0 = ((double)w0 + 0.5) * kTwoM32;
    const double u1 = ((double)w1 + 0.5) * kTwoM32;
    const double u2 = ((double)w2 + 0.5) * kTwoM32;
    const double u3 = ((double)w3 + 0.5) * kTwoM32;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    g[0] = r0 * cos(kTwoPi * u1);
    g[1] = r0 * sin(kTwoPi * u1);
    g[2] = r1 * cos(kTwoPi * u3);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_integrate(IntArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (MODE != kIntLast && a.gate && s == 0) {
        // the longest list lifetime is reached
        const uint64_t st = a.step_dev ? *a.step_dev + a.step : a.step;
        if ((int64_t)(st - *a.bstep) >= a.max_life) {
            *a.gate = 1;
            if (a.fgate) *a.fgate = 1;
        }
    }
    if ((s >> 6) >= a.n_slices) return;
    const int r = a.slice_rep[s >> 6];
    const DevReplica& R = a.rep[r];
    if (s - R.slot_base >= R.n) return;
    double fc[3] = {0.0, 0.0, 0.0};
    if (a.momentum_fix) {
        const double nr = (double)R.n;
        fc[0] = a.rep_sum[8 * r] / nr;
        fc[1] = a.rep_sum[8 * r + 1] / nr;
        fc[2] = a.rep_sum[8 * r + 2] / nr;
    }
    const bool close = MODE == kIntMid && (a.pending == nullptr || *a.pending != 0);
    double v[3], F[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v[d] = a.vs[d * a.n_slots + s];
        F[d] = a.f[d * a.n_slots + s] - fc[d];
        v[d] = v[d] + a.h * F[d];
        if (close) v[d] = v[d] + a.h * F[d];
    }
    if (MODE != kIntLast && a.langevin) {
        // A (half drift), O (exact Ornstein-Uhlenbeck step), A
        double g[3];
        const uint64_t step = a.step_dev ? *a.step_dev + a.step : a.step;
        langevin_noise(a.seed, (uint32_t)(a.perm[s] - R.id_base), (uint32_t)step, (uint32_t)r, g);
        const double sig = a.osig[r];
        double4 x = a.xs[s];
        x.x = x.x + a.h * v[0];
        x.y = x.y + a.h * v[1];
        x.z = x.z + a.h * v[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) v[d] = a.oc * v[d] + sig * g[d];
        x.x = x.x + a.h * v[0];
        x.y = x.y + a.h * v[1];
        x.z = x.z + a.h * v[2];
        a.xs[s] = x;
        if (a.xq) a.xq[s] = fixq4(x.x, x.y, x.z, x.w, R);
    } else if (MODE != kIntLast) {
        double4 x = a.xs[s];
        x.x = x.x + a.dt * v[0];
        x.y = x.y + a.dt * v[1];
        x.z = x.z + a.dt * v[2];
        a.xs[s] = x;
        if (a.xq) a.xq[s] = fixq4(x.x, x.y, x.z, x.w, R);
    }
    if (MODE != kIntLast && a.gate) {
        // displacement since the last build past skin/2: rebuild at this step
        const double4 x = a.xs[s];
        const double dx = x.x - a.xb[s];
        const double dy = x.y - a.xb[a.n_slots + s];
        const double dz = x.z - a.xb[2 * a.n_slots + s];
        if (dx * dx + dy * dy + dz * dz > a.half_skin2) {
            *a.gate = 1;
            if (a.fgate) *a.fgate = 1;
        }
        if (a.fgate) {
            const float ex = (float)x.x - a.xf[s];
            const float ey = (float)x.y - a.xf[a.n_slots + s];
            const float ez = (float)x.z - a.xf[2 * a.n_slots + s];
            if (ex * ex + ey * ey + ez * ez > a.fhalf2) *a.fgate = 1;
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) a.vs[d * a.n_slots + s] = v[d];
    if (MODE == kIntLast) {
        // displacement since the last build (the rebuilds check their own
        // list lifetimes while binning)
        const double4 x = a.xs[s];
        const double dx = x.x - a.xb[s];
        const double dy = x.y - a.xb[a.n_slots + s];
        const double dz = x.z - a.xb[2 * a.n_slots + s];
        if (dx * dx + dy * dy + dz * dz > a.half_skin2) raise_flag(&a.flags[kFlagSkin]);
    }
}

// ---------------------------------------------------------------------------
// Caller-order I/O.
struct IoArgs {
    const DevReplica* rep;
    const int* slice_rep;
    const int* perm;
    const double* rep_sum;
    const double* charges;
    int64_t n;
    int64_t n_slots;
    int64_t n_slices;
    int momentum_fix;
    double4* xs;
    const double* vs;
    const double* f;
    const double* pos_in;
    double* pos_out;
    double* vel_out;
    double* f_out;
    const int* img_delta;  // if set, added into img ([3][n], caller order)
    int* img;
    int4* xq;              // may be null: fixed-point copy of xs
};

// xs[slot] <- caller positions as given (no wrapping), for a force call.
__global__ __launch_bounds__(256) void k_load_positions(IoArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.n_slots) return;
    const int id = a.perm[s];
    if (id < 0) return;
    const double q = a.charges ? a.charges[id] : 0.0;
    a.xs[s] = make_double4(a.pos_in[id], a.pos_in[a.n + id], a.pos_in[2 * a.n + id], q);
    if (a.xq) a.xq[s] = fixq4(a.pos_in[id], a.pos_in[a.n + id], a.pos_in[2 * a.n + id], q,
                              a.rep[a.slice_rep[s >> 6]]);
}

__global__ __launch_bounds__(256) void k_scatter_out(IoArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((s >> 6) >= a.n_slices) return;
    const int id = a.perm[s];
    if (id < 0) return;
    const int r = a.slice_rep[s >> 6];
    if (a.pos_out) {
        const double4 x = a.xs[s];
        a.pos_out[id] = x.x;
        a.pos_out[a.n + id] = x.y;
        a.pos_out[2 * a.n + id] = x.z;
    }
    if (a.vel_out) {
        a.vel_out[id] = a.vs[s];
        a.vel_out[a.n + id] = a.vs[a.n_slots + s];
        a.vel_out[2 * a.n + id] = a.vs[2 * a.n_slots + s];
    }
    if (a.f_out) {
        const double nr = (double)a.rep[r].n;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double fc = a.momentum_fix ? a.rep_sum[8 * r + d] / nr : 0.0;
            a.f_out[d * a.n + id] = a.f[d * a.n_slots + s] - fc;
        }
    }
    if (a.img_delta) {
#pragma unroll
        for (int d = 0; d < 3; ++d) a.img[d * a.n + id] += a.img_delta[d * a.n + id];
    }
}

// ---------------------------------------------------------------------------
// Observables of Sec. III: continuous trajectory (for the mean-squared
// displacement), per-replica sums of squares, and the pair-distance
// histogram behind the radial distribution function.

// out = pos + img L (caller order): the positions without the wraps the
// list builds applied since the counters were set up.
__global__ __launch_bounds__(256) void k_unwrap(const DevReplica* rep, const int* id_rep, const double* pos,
                                                const int* img, int64_t n, double* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DevReplica& R = rep[id_rep[i]];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double k = img ? (double)img[d * n + i] : 0.0;
        out[d * n + i] = fma(k, R.L[d], pos[d * n + i]);
    }
}

// Per replica r and chunk b (grid (nb, R)): partial[r * nb + b] = sum over
// the replica's particles i = id_base + b*256*kSqIter ... of |a_i - b_i|^2
// (b may be null), in a fixed order: deterministic.
constexpr int kSqIter = 16;

__global__ __launch_bounds__(256) void k_sumsq(const DevReplica* rep, const double* x, const double* y, int64_t n,
                                               int nb, double* partial)
{
    __shared__ double s_red[256];
    const int r = blockIdx.y;
    const int64_t base = rep[r].id_base;
    const int64_t nr = rep[r].n;
    double acc = 0.0;
    for (int it = 0; it < kSqIter; ++it) {
        const int64_t k = ((int64_t)blockIdx.x * kSqIter + it) * blockDim.x + threadIdx.x;
        if (k < nr) {
            const int64_t i = base + k;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double v = y ? x[d * n + i] - y[d * n + i] : x[d * n + i];
                acc = fma(v, v, acc);
            }
        }
    }
    s_red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s_red[threadIdx.x] += s_red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)r * nb + blockIdx.x] = s_red[0];
}

// out[r] = scale_r * sum_b partial[r * nb + b], scale_r = 1 / (n_r * div)
__global__ void k_sumsq_final(const DevReplica* rep, const double* partial, int nb, int R, double div, double* out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partial[(int64_t)r * nb + b];
    out[r] = t / ((double)rep[r].n * div);
}

// Pair-distance histogram: counts[r * nbins + k] += the ordered pairs (i, j),
// i != j, of replica r with minimum-image distance in [k dr, (k+1) dr),
// r < r_max = nbins dr; the bin decided on r^2 against the squared edges
// (k dr)(k dr).  One lane per particle walks the 5x5x5 stencil of its
// build-time cell (the stencil reaches r_c + skin, so every pair closer
// than r_max <= r_c is found while no particle has moved skin/2).
struct RdfArgs {
    const DevReplica* rep;
    const int* slice_rep;
    const int* perm;
    const double4* xs;
    const double* xb;
    const int* cell_start;
    const int* cell_count;
    int64_t n_slots;
    int64_t n_slices;
    double dr;
    double top2;   // (nbins dr)^2
    int nbins;
    unsigned long long* counts;
};

__device__ __forceinline__ double rdf_edge2(int k, double dr)
{
    const double e = (double)k * dr;
    return e * e;
}

__global__ __launch_bounds__(256) void k_rdf(RdfArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((s >> 6) >= a.n_slices) return;
    const int r = a.slice_rep[s >> 6];
    const DevReplica& R = a.rep[r];
    if (s - R.slot_base >= R.n || a.perm[s] < 0) return;
    int cc[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // the cell the build put the particle in (xb holds the wrapped
        // build-time position the binning used)
        int k = (int)floor(a.xb[d * a.n_slots + s] * R.cscale[d]);
        cc[d] = k < 0 ? 0 : (k > R.nc[d] - 1 ? R.nc[d] - 1 : k);
    }
    const AxisRuns ax = axis_runs(cc[0], R.nc[0]);
    const AxisRuns ay = axis_runs(cc[1], R.nc[1]);
    const AxisRuns az = axis_runs(cc[2], R.nc[2]);
    const double4 xi = a.xs[s];
    unsigned long long* cnt = a.counts + (int64_t)r * a.nbins;
    for (int zi = 0; zi < az.l0 + az.l1; ++zi) {
        const int z = axis_cell(az, zi);
        for (int yi = 0; yi < ay.l0 + ay.l1; ++yi) {
            const int y = axis_cell(ay, yi);
            for (int xi_ = 0; xi_ < ax.l0 + ax.l1; ++xi_) {
                const int x = axis_cell(ax, xi_);
                const int64_t c = R.cell_base + ((int64_t)z * R.nc[1] + y) * R.nc[0] + x;
                const int j0 = a.cell_start[c];
                const int j1 = j0 + a.cell_count[c];
                for (int j = j0; j < j1; ++j) {
                    if (j == s) continue;
                    const double4 xj = a.xs[j];
                    const double dx = min_image(xi.x - xj.x, R.L[0], R.inv[0]);
                    const double dy = min_image(xi.y - xj.y, R.L[1], R.inv[1]);
                    const double dz = min_image(xi.z - xj.z, R.L[2], R.inv[2]);
                    const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
                    if (!(r2 < a.top2)) continue;
                    int k = (int)(sqrt(r2) / a.dr);
                    if (k > a.nbins - 1) k = a.nbins - 1;
                    while (k > 0 && r2 < rdf_edge2(k, a.dr)) --k;
                    while (k < a.nbins - 1 && r2 >= rdf_edge2(k + 1, a.dr)) ++k;
                    atomicAdd(&cnt[k], 1ull);
                }
            }
        }
    }
}

// Last node of a captured block: moves the device step counter to the next
// block.
__global__ void k_advance(uint64_t* step_dev, uint64_t by)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step_dev += by;
}

__global__ void k_ev_out(const double* rep_sum, int nrep, double* ev)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrep) return;
    ev[2 * r] = rep_sum[8 * r + 3];
    ev[2 * r + 1] = rep_sum[8 * r + 4];
}

// Copies requested rows of a sliced-ELL list into CSR, partners as IDs.
__global__ __launch_bounds__(256) void k_export_rows(const int64_t* rows, int64_t nrows,
                                                     const int* slot_of_id, const int* perm,
                                                     const int* list, const int* len, int cap,
                                                     const int64_t* off, int* out)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrows) return;
    const int slot = slot_of_id[rows[k]];
    const int l = len[slot];
    const int64_t o = off[k];
    const int64_t room = off[k + 1] - o;
    for (int q = 0; q < l && q < room; ++q) out[o + q] = perm[list[ell(slot, q, cap)]];
}

__global__ __launch_bounds__(256) void k_row_counts(const int64_t* rows, int64_t nrows,
                                                    const int* slot_of_id, const int* len,
                                                    int64_t* counts)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nrows) return;
    counts[k] = len ? len[slot_of_id[rows[k]]] : 0;
}

}  // namespace rbl
