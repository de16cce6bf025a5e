/*
 * Plain FP64 CPU oracle of the random-batch list (RBL) short-range force path
 * (Liang, Xu & Zhao, "Random-batch list algorithm for short-range molecular
 * dynamics simulations", arXiv:2105.04884).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no code, header, table or constant with the
 * HIP path.
 *
 * It is written to be read against the paper, not to be fast: single
 * threaded, no blocking, loops in the order the definitions give them.
 * Build with -ffp-contract=off so that every multiply-add below is rounded
 * exactly as written (fma() only where it is spelled out).
 *
 * Radius names: the paper calls the core radius r_c and the outer cut-off
 * r_s.  This file uses the names of the public interface instead:
 *   rs = core radius (direct sum, eq. (3)),
 *   rc = outer cut-off (end of the shell zone, eq. (4)).
 *
 * What each function follows:
 *   orc_philox4x32_10   Philox4x32-10 of Salmon, Moraes, Dror & Shaw (SC'11);
 *                       the paper only says "randomly choose", the generator
 *                       is a reading of the batch draw (Sec. II).
 *   orc_floyd_choices   Floyd's sampling without replacement (Bentley &
 *                       Floyd, CACM 1987): the batch B(i) of Sec. II, with the
 *                       without-replacement moments of Appendix A.
 *   orc_lj              LJ 12-6 pair potential eq. (1), truncated at the
 *                       cut-off and shifted to zero there (Sec. II).
 *   orc_lj_typed        the same with the pair's epsilon and sigma, for
 *                       systems of several particle types whose interaction
 *                       lengths differ (Sec. II): pair (a, b) has its own
 *                       epsilon_ab, sigma_ab, core radius rs sigma_ab and
 *                       cut-off rc sigma_ab; the cell grid takes its width
 *                       from the smallest cut-off and each type searches its
 *                       own stencil of cells, wide enough for its largest
 *                       cut-off (orc_sys_new_typed).
 *   orc_erfc_pair       real-space Ewald term q_i q_j erfc(alpha r)/r of a
 *                       pair of charges, added to the LJ pair for charged
 *                       systems (the short-range part that a random-batch
 *                       list would serve beside random-batch Ewald, Sec. IV);
 *                       its form is the standard one, not printed in the
 *                       paper, and is shifted to zero at the cut-off too.
 *   orc_build_*         cell list and core/shell neighbour lists (Sec. II,
 *                       Fig. 1); brute force is the plain definition.
 *   orc_forces_rbl      F_i = F_ic + (n/p) sum_{B(i)} f~_ij, eq. (3) and
 *                       eq. (4); small shells (n <= p) taken whole.
 *   orc_stencil_rows    the paper's own draw population: every particle of
 *                       the stencil cells around i's cell, i included, N_I of
 *                       them (Sec. II, Fig. 1); with these rows in place of
 *                       the shell rows, orc_forces_rbl is eq. (4) with N_I/p
 *                       and f~_ij = 0 outside the shell zone.
 *   orc_paper_stencil_rows  the same population on the paper's own grid:
 *                       cells of edge at least the core radius plus skin,
 *                       (2 floor((rc + skin)/w) + 3)^3 of them around i's
 *                       cell (Sec. II, Fig. 1).
 *   orc_mean_subtract   subtraction of the average net force (Sec. II,
 *                       Algorithm 1, F_cor of Appendix A).
 *   orc_md_run          Algorithm 1 with velocity Verlet (NVE), or with the
 *                       underdamped Langevin thermostat of Sec. II / Sec. III
 *                       (friction gamma, bath temperature kT) integrated by
 *                       the BAOAB splitting of Leimkuhler & Matthews (2013),
 *                       the velocity-Verlet Langevin scheme the paper cites.
 *   orc_langevin_noise  the three standard normal numbers of one particle's
 *                       Ornstein-Uhlenbeck step: Box-Muller (1958) on one
 *                       Philox block.
 *   orc_rdf             pair-distance histogram behind the radial
 *                       distribution function g(r) of Sec. III, by brute
 *                       force over all ordered pairs.
 *   orc_tail            the mean-field tail corrections of the potential
 *                       energy per particle and of the pressure (Sec. III).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, "Parallel random numbers: as easy as
 * 1, 2, 3").  Round multipliers and key (Weyl) increments from that paper. */

#define ORC_PHILOX_MUL0 0xD2511F53u
#define ORC_PHILOX_MUL1 0xCD9E8D57u
#define ORC_PHILOX_WEYL0 0x9E3779B9u
#define ORC_PHILOX_WEYL1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* key schedule: bump before rounds 2..10 */
            k0 += ORC_PHILOX_WEYL0;
            k1 += ORC_PHILOX_WEYL1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_MUL0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_MUL1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Batch draw.  Floyd's algorithm picks p distinct positions out of
 * {0, ..., n-1}: for m = 0..p-1 with J = n-p+m it takes a uniform t in
 * {0..J}; if t was already taken it takes J instead.  Every p-subset comes
 * out with the same probability (simple random sampling without
 * replacement, whose second moment (p-1)/(N-1) Appendix A uses).
 *
 * orc_floyd_choices takes the choices t[m] themselves, so that a test can
 * enumerate them all; the positions are returned sorted ascending. */

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

int orc_floyd_choices(int p, int n, const uint32_t* t, int32_t* out)
{
    if (p <= 0 || n < p) return -1;
    for (int m = 0; m < p; ++m) {
        int32_t J = (int32_t)(n - p + m);
        int32_t pick = (int32_t)t[m];
        if (pick < 0 || pick > J) return -2;
        int taken = 0;
        for (int q = 0; q < m; ++q)
            if (out[q] == pick) taken = 1;
        out[m] = taken ? J : pick;
    }
    qsort(out, (size_t)p, sizeof(int32_t), cmp_i32);
    return p;
}

/* Positions of the batch of particle `pid` at force evaluation `step`.
 * Counter words: (pid, step mod 2^32, replica, block b), key = seed split in
 * two 32-bit halves.  Draw m uses word m mod 4 of block floor(m/4); the
 * uniform word u maps to t = floor(u (J+1) / 2^32).
 * If n <= p the whole shell is the batch (positions 0..n-1).
 * Returns the batch size min(n, p). */
int orc_batch_positions(uint64_t seed, uint32_t pid, uint64_t step, uint32_t replica,
                        int p, int n, int32_t* out)
{
    if (n <= 0) return 0;
    if (n <= p) {
        for (int k = 0; k < n; ++k) out[k] = k;
        return n;
    }
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t* t = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)p);
    uint32_t words[4] = {0, 0, 0, 0};
    for (int m = 0; m < p; ++m) {
        if (m % 4 == 0) {
            uint32_t ctr[4] = {pid, (uint32_t)step, replica, (uint32_t)(m / 4)};
            orc_philox4x32_10(ctr, key, words);
        }
        uint32_t u = words[m % 4];
        uint64_t J = (uint64_t)(n - p + m);
        t[m] = (uint32_t)(((uint64_t)u * (J + 1)) >> 32);
    }
    int r = orc_floyd_choices(p, n, t, out);
    free(t);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Pair term, eq. (1) with epsilon = sigma = 1:
 *   U(r) = 4 (r^-12 - r^-6),
 *   f_ij = -dU/dr * (x_i - x_j)/r = 24 r^-8 (2 r^-6 - 1) (x_i - x_j).
 * fmag is the factor multiplying (x_i - x_j); u is the unshifted energy. */
void orc_lj(double r2, double* fmag, double* u)
{
    double r2i = 1.0 / r2;
    double sr6 = r2i * r2i * r2i;
    *fmag = 24.0 * r2i * sr6 * (2.0 * sr6 - 1.0);
    *u = 4.0 * sr6 * (sr6 - 1.0);
}

/* Pair term of eq. (1) with the pair's own parameters:
 *   U(r) = 4 eps ((sigma/r)^12 - (sigma/r)^6),
 *   fmag = -dU/dr / r = 24 eps r^-2 (sigma/r)^6 (2 (sigma/r)^6 - 1).
 * With eps = sigma = 1 every operation below is that of orc_lj. */
void orc_lj_typed(double r2, double eps, double sig, double* fmag, double* u)
{
    double r2i = 1.0 / r2;
    double s2 = (sig * sig) * r2i;
    double sr6 = s2 * s2 * s2;
    *fmag = (24.0 * eps) * r2i * sr6 * (2.0 * sr6 - 1.0);
    *u = (4.0 * eps) * sr6 * (sr6 - 1.0);
}

/* Real-space Ewald pair of charges with product qq at squared distance r2:
 *   u(r) = qq erfc(alpha r) / r,
 *   -du/dr = qq [erfc(alpha r) / r^2 + (2 alpha / sqrt(pi)) exp(-alpha^2 r^2) / r],
 * and fmag = (-du/dr) / r, the factor of the displacement x_i - x_j. */
void orc_erfc_pair(double r2, double qq, double alpha, double* fmag, double* u)
{
    double r = sqrt(r2);
    double er = erfc(alpha * r);
    double gauss = exp(-(alpha * alpha) * r2);
    double two_over_sqrt_pi = 2.0 / sqrt(3.14159265358979323846);
    *u = qq * er / r;
    *fmag = qq * (er / (r2 * r) + two_over_sqrt_pi * alpha * gauss / r2);
}

/* Pair term of particles i and j: LJ, plus the erfc term when charges are
 * given (q == NULL: LJ only). */
static void pair_term(double r2, const double* q, double alpha, int64_t i, int64_t j,
                      double* fmag, double* u)
{
    orc_lj(r2, fmag, u);
    if (q) {
        double fe, ue;
        orc_erfc_pair(r2, q[i] * q[j], alpha, &fe, &ue);
        *fmag = *fmag + fe;
        *u = *u + ue;
    }
}

/* Energies at the cut-off, for shifting the pair energy to zero there: the
 * LJ part, and the erfc part per unit charge product. */
typedef struct {
    double lj, erfc_per_qq;
} orc_shift;

static orc_shift cutoff_shift(double rc2, int shift, const double* q, double alpha)
{
    orc_shift sh = {0.0, 0.0};
    if (!shift) return sh;
    double fm;
    orc_lj(rc2, &fm, &sh.lj);
    if (q) orc_erfc_pair(rc2, 1.0, alpha, &fm, &sh.erfc_per_qq);
    return sh;
}

static double pair_shift(orc_shift sh, const double* q, int64_t i, int64_t j)
{
    return q ? sh.lj + q[i] * q[j] * sh.erfc_per_qq : sh.lj;
}

/* Minimum-image component of x_i - x_j in a periodic box of side L. */
static double min_image(double d, double L, double invL)
{
    double k = rint(d * invL);
    return fma(-k, L, d);
}

static double dist2(const double* pos, int64_t n, int64_t i, int64_t j,
                    const double box[3], const double inv[3], double d[3])
{
    for (int a = 0; a < 3; ++a)
        d[a] = min_image(pos[a * n + i] - pos[a * n + j], box[a], inv[a]);
    return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
}

/* ------------------------------------------------------------------------ */
/* Particle types (Sec. II, systems with a large disparity in interaction
 * lengths).  nt types, nt <= ORC_MAX_TYPES; type[i] of particle ID i;
 * eps_sig[(a nt + b) 2 + 0 / 1] = epsilon_ab / sigma_ab of pair (a, b),
 * symmetric, positive.  Pair (a, b) interacts by orc_lj_typed with core
 * radius rs sigma_ab and cut-off rc sigma_ab (rs, rc in units of sigma);
 * with `shift` its energy is shifted to zero at its own cut-off.  nt = 0
 * means one type with epsilon = sigma = 1 (eq. (1) as in orc_lj). */

#define ORC_MAX_TYPES 4

typedef struct {
    int nt;
    int32_t* type;                                     /* own copy, per ID */
    double eps[ORC_MAX_TYPES][ORC_MAX_TYPES];
    double sig[ORC_MAX_TYPES][ORC_MAX_TYPES];
    double rs2[ORC_MAX_TYPES][ORC_MAX_TYPES];          /* (rs sigma_ab)^2 */
    double rc2[ORC_MAX_TYPES][ORC_MAX_TYPES];          /* (rc sigma_ab)^2 */
    double ush[ORC_MAX_TYPES][ORC_MAX_TYPES];          /* energy at the cut-off (0: no shift) */
} orc_types;

/* Fills T (T->type is malloc'ed; free with types_free).  Returns 0, or -4
 * for an invalid type count, table or type index. */
static int types_setup(orc_types* T, int64_t n, int nt, const int32_t* type, const double* eps_sig,
                       double rs, double rc, int shift)
{
    memset(T, 0, sizeof(*T));
    if (nt == 0) return 0;
    if (nt < 1 || nt > ORC_MAX_TYPES || !type || !eps_sig) return -4;
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            double e = eps_sig[(a * nt + b) * 2 + 0], g = eps_sig[(a * nt + b) * 2 + 1];
            if (!(e >= 0.0) || !(g > 0.0) || !isfinite(e) || !isfinite(g)) return -4;
            if (e != eps_sig[(b * nt + a) * 2 + 0] || g != eps_sig[(b * nt + a) * 2 + 1]) return -4;
            T->eps[a][b] = e;
            T->sig[a][b] = g;
            double rsab = rs * g, rcab = rc * g;
            T->rs2[a][b] = rsab * rsab;
            T->rc2[a][b] = rcab * rcab;
            T->ush[a][b] = 0.0;
            if (shift) {
                double fm;
                orc_lj_typed(T->rc2[a][b], e, g, &fm, &T->ush[a][b]);
            }
        }
    T->type = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        if (type[i] < 0 || type[i] >= nt) { free(T->type); T->type = NULL; return -4; }
        T->type[i] = type[i];
    }
    T->nt = nt;
    return 0;
}

static void types_free(orc_types* T)
{
    free(T->type);
    T->type = NULL;
}

/* ------------------------------------------------------------------------ */
/* Canonical cell list.  Positions are first wrapped into the box; cells have
 * edge >= (rc + skin)/2, so any pair closer than rc + skin lies within two
 * cells of each other in every direction.  Particles are ordered by cell
 * (z-major linear index) and by ID within a cell; that order ("slot") is the
 * order in which a neighbour row lists its partners, and therefore the order
 * the batch positions of orc_batch_positions index into. */

#define ORC_HALF_STENCIL 2

typedef struct orc_sys {
    int64_t n;
    double box[3], inv[3];
    double rs, rc, skin;
    double *pos;          /* wrapped copy, [3][n] */
    int ncell[3];
    int64_t ncells;
    int64_t *cell_of;     /* per ID */
    int64_t *slot_of;     /* per ID */
    int64_t *id_of;       /* per slot */
    int64_t *cell_start;  /* ncells + 1 */
    orc_types T;          /* particle types (T.nt == 0: one type) */
    int h[ORC_MAX_TYPES][3];  /* typed: stencil half-width per centre type and axis */
} orc_sys;

void orc_wrap(int64_t n, double* pos, const double box[3])
{
    for (int a = 0; a < 3; ++a) {
        double inv = 1.0 / box[a];
        for (int64_t i = 0; i < n; ++i) {
            double x = pos[a * n + i];
            double k = floor(x * inv);
            pos[a * n + i] = fma(-k, box[a], x);
        }
    }
}

int orc_cell_grid(const double box[3], double rc, double skin, int ncell[3])
{
    double w = 0.5 * (rc + skin) * 1.000001;
    for (int a = 0; a < 3; ++a) {
        double c = floor(box[a] / w);
        if (c < 1.0) c = 1.0;
        ncell[a] = (int)c;
    }
    return 0;
}

static int64_t cell_of_pos(const orc_sys* s, int64_t i)
{
    int64_t c[3];
    for (int a = 0; a < 3; ++a) {
        double scale = (double)s->ncell[a] / s->box[a];
        double f = floor(s->pos[a * s->n + i] * scale);
        int64_t k = (int64_t)f;
        if (k < 0) k = 0;
        if (k > s->ncell[a] - 1) k = s->ncell[a] - 1;
        c[a] = k;
    }
    return (c[2] * s->ncell[1] + c[1]) * s->ncell[0] + c[0];
}

/* With particle types (nt > 0) the cells take their width from the
 * smallest pair cut-off, rc times the smallest sigma_ab, and a centre of
 * type a searches the cells within h_a of its own along each axis, h_a the
 * number of cell edges (times 1 + 1e-6) that its largest pair cut-off plus
 * the skin spans: the per-type stencils of Sec. II.  Returns NULL for an
 * invalid type table. */
orc_sys* orc_sys_new_typed(int64_t n, const double* pos, const double box[3],
                           double rs, double rc, double skin,
                           int nt, const int32_t* type, const double* eps_sig)
{
    orc_sys* s = (orc_sys*)calloc(1, sizeof(orc_sys));
    if (types_setup(&s->T, n, nt, type, eps_sig, rs, rc, 0)) {
        free(s);
        return NULL;
    }
    s->n = n;
    for (int a = 0; a < 3; ++a) {
        s->box[a] = box[a];
        s->inv[a] = 1.0 / box[a];
    }
    s->rs = rs; s->rc = rc; s->skin = skin;
    s->pos = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    memcpy(s->pos, pos, sizeof(double) * 3 * (size_t)n);
    orc_wrap(n, s->pos, box);
    if (nt == 0) {
        orc_cell_grid(box, rc, skin, s->ncell);
    } else {
        double smin = s->T.sig[0][0];
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nt; ++b)
                if (s->T.sig[a][b] < smin) smin = s->T.sig[a][b];
        orc_cell_grid(box, rc * smin, skin, s->ncell);
        for (int a = 0; a < nt; ++a) {
            double smax = 0.0;
            for (int b = 0; b < nt; ++b)
                if (s->T.sig[a][b] > smax) smax = s->T.sig[a][b];
            double reach = (rc * smax + skin) * 1.000001;
            for (int ax = 0; ax < 3; ++ax) {
                double edge = box[ax] / (double)s->ncell[ax];
                s->h[a][ax] = (int)ceil(reach / edge);
            }
        }
    }
    s->ncells = (int64_t)s->ncell[0] * s->ncell[1] * s->ncell[2];
    s->cell_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    s->slot_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    s->id_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    s->cell_start = (int64_t*)calloc((size_t)s->ncells + 1, sizeof(int64_t));
    /* counting sort by cell, stable in ID */
    for (int64_t i = 0; i < n; ++i) {
        s->cell_of[i] = cell_of_pos(s, i);
        s->cell_start[s->cell_of[i] + 1] += 1;
    }
    for (int64_t c = 0; c < s->ncells; ++c) s->cell_start[c + 1] += s->cell_start[c];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(s->ncells + 1));
    memcpy(fill, s->cell_start, sizeof(int64_t) * (size_t)(s->ncells + 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t slot = fill[s->cell_of[i]]++;
        s->slot_of[i] = slot;
        s->id_of[slot] = i;
    }
    free(fill);
    return s;
}

orc_sys* orc_sys_new(int64_t n, const double* pos, const double box[3],
                     double rs, double rc, double skin)
{
    return orc_sys_new_typed(n, pos, box, rs, rc, skin, 0, NULL, NULL);
}

void orc_sys_free(orc_sys* s)
{
    if (!s) return;
    free(s->pos); free(s->cell_of); free(s->slot_of); free(s->id_of); free(s->cell_start);
    types_free(&s->T);
    free(s);
}

/* Stencil half-widths of a typed system for centre type a (h[3]); returns
 * -1 for an untyped system or a bad type. */
int orc_sys_stencil(const orc_sys* s, int a, int32_t h[3])
{
    if (s->T.nt == 0 || a < 0 || a >= s->T.nt) return -1;
    for (int ax = 0; ax < 3; ++ax) h[ax] = s->h[a][ax];
    return 0;
}

int64_t orc_sys_ncells(const orc_sys* s) { return s->ncells; }

void orc_sys_info(const orc_sys* s, int32_t ncell[3], double* wrapped_pos,
                  int64_t* slot_of_id, int64_t* cell_start)
{
    for (int a = 0; a < 3; ++a) ncell[a] = s->ncell[a];
    if (wrapped_pos) memcpy(wrapped_pos, s->pos, sizeof(double) * 3 * (size_t)s->n);
    if (slot_of_id) memcpy(slot_of_id, s->slot_of, sizeof(int64_t) * (size_t)s->n);
    if (cell_start) memcpy(cell_start, s->cell_start, sizeof(int64_t) * (size_t)(s->ncells + 1));
}

/* Neighbour-list thresholds, squared distances (skin on both sides of the
 * core radius and outside the cut-off):
 *   core  C_i = { j : r^2 <  (rs+skin)^2 }
 *   shell S_i = { j : max(rs-skin,0)^2 <= r^2 < (rc+skin)^2 }
 *   full  V_i = { j : r^2 <  (rc+skin)^2 }            (direct truncation) */
typedef struct { double core, shell_in, out; } orc_thr;

static orc_thr thresholds(double rs, double rc, double skin)
{
    orc_thr t;
    double a = rs + skin;
    double b = rs - skin;
    if (b < 0.0) b = 0.0;
    double c = rc + skin;
    t.core = a * a;
    t.shell_in = b * b;
    t.out = c * c;
    return t;
}

/* Candidates of row i, collected either from the 5x5x5 cell stencil around
 * i's cell (method 0; the paper's stenciled cells) or from all particles
 * (method 1, brute force).  `emit` receives every candidate j != i with its
 * squared distance.  Rows are put into slot order afterwards. */
typedef struct {
    int64_t* core; int64_t nc;
    int64_t* shell; int64_t ns;
    int64_t* full; int64_t nf;
    int64_t cap;
} orc_row;

static void row_push(int64_t** arr, int64_t* len, int64_t* cap, int64_t v)
{
    if (*len == *cap) {
        *cap = (*cap) * 2 + 16;
        *arr = (int64_t*)realloc(*arr, sizeof(int64_t) * (size_t)(*cap));
    }
    (*arr)[(*len)++] = v;
}

typedef struct { int64_t ccap, scap, fcap; } orc_rowcap;

static void classify(const orc_sys* s, orc_thr th, int64_t i, int64_t j,
                     orc_row* row, orc_rowcap* cap)
{
    double d[3];
    double r2 = dist2(s->pos, s->n, i, j, s->box, s->inv, d);
    if (s->T.nt) {
        /* the pair's own radii: core rs sigma_ab, cut-off rc sigma_ab */
        double g = s->T.sig[s->T.type[i]][s->T.type[j]];
        th = thresholds(s->rs * g, s->rc * g, s->skin);
    }
    if (r2 < th.core) row_push(&row->core, &row->nc, &cap->ccap, j);
    if (r2 >= th.shell_in && r2 < th.out) row_push(&row->shell, &row->ns, &cap->scap, j);
    if (r2 < th.out) row_push(&row->full, &row->nf, &cap->fcap, j);
}

/* unique wrapped cell coordinates within +-h of c along an axis of nc
 * cells (out holds min(2h + 1, nc) entries) */
static int stencil_axis(int c, int nc, int h, int* out)
{
    int k = 0;
    if (nc <= 2 * h + 1) {
        for (int q = 0; q < nc; ++q) out[k++] = q;
        return k;
    }
    for (int d = -h; d <= h; ++d)
        out[k++] = ((c + d) % nc + nc) % nc;
    return k;
}

static const orc_sys* g_sort_sys;
static int cmp_slot(const void* a, const void* b)
{
    int64_t x = g_sort_sys->slot_of[*(const int64_t*)a];
    int64_t y = g_sort_sys->slot_of[*(const int64_t*)b];
    return (x > y) - (x < y);
}

static void build_row(const orc_sys* s, orc_thr th, int method, int64_t i,
                      orc_row* row, orc_rowcap* cap)
{
    row->nc = row->ns = row->nf = 0;
    if (method == 1) {
        for (int64_t j = 0; j < s->n; ++j)
            if (j != i) classify(s, th, i, j, row, cap);
    } else {
        int64_t ci = s->cell_of[i];
        int cx = (int)(ci % s->ncell[0]);
        int cy = (int)((ci / s->ncell[0]) % s->ncell[1]);
        int cz = (int)(ci / ((int64_t)s->ncell[0] * s->ncell[1]));
        /* the stencil: +-2 cells, or a typed centre's own half-widths */
        int hx = ORC_HALF_STENCIL, hy = ORC_HALF_STENCIL, hz = ORC_HALF_STENCIL;
        if (s->T.nt) {
            int t = s->T.type[i];
            hx = s->h[t][0]; hy = s->h[t][1]; hz = s->h[t][2];
        }
        int* sx = (int*)malloc(sizeof(int) * (size_t)(2 * hx + 1));
        int* sy = (int*)malloc(sizeof(int) * (size_t)(2 * hy + 1));
        int* sz = (int*)malloc(sizeof(int) * (size_t)(2 * hz + 1));
        int nx = stencil_axis(cx, s->ncell[0], hx, sx);
        int ny = stencil_axis(cy, s->ncell[1], hy, sy);
        int nz = stencil_axis(cz, s->ncell[2], hz, sz);
        for (int a = 0; a < nz; ++a)
            for (int b = 0; b < ny; ++b)
                for (int c = 0; c < nx; ++c) {
                    int64_t cell = ((int64_t)sz[a] * s->ncell[1] + sy[b]) * s->ncell[0] + sx[c];
                    for (int64_t q = s->cell_start[cell]; q < s->cell_start[cell + 1]; ++q) {
                        int64_t j = s->id_of[q];
                        if (j != i) classify(s, th, i, j, row, cap);
                    }
                }
        free(sx); free(sy); free(sz);
    }
    g_sort_sys = s;
    qsort(row->core, (size_t)row->nc, sizeof(int64_t), cmp_slot);
    qsort(row->shell, (size_t)row->ns, sizeof(int64_t), cmp_slot);
    qsort(row->full, (size_t)row->nf, sizeof(int64_t), cmp_slot);
}

/* Row lengths for the requested rows (all rows when rows == NULL):
 * counts[0*nrows+k] core, counts[1*nrows+k] shell, counts[2*nrows+k] full. */
int orc_list_counts(const orc_sys* s, int method, int64_t nrows, const int64_t* rows,
                    int64_t* counts)
{
    orc_thr th = thresholds(s->rs, s->rc, s->skin);
    orc_row row = {0};
    orc_rowcap cap = {0, 0, 0};
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        if (i < 0 || i >= s->n) return -1;
        build_row(s, th, method, i, &row, &cap);
        counts[k] = row.nc;
        counts[nrows + k] = row.ns;
        counts[2 * nrows + k] = row.nf;
    }
    free(row.core); free(row.shell); free(row.full);
    return 0;
}

/* CSR fill; offsets are exclusive prefix sums of the counts (length nrows+1).
 * Any of the index arrays may be NULL to skip that list. */
int orc_list_fill(const orc_sys* s, int method, int64_t nrows, const int64_t* rows,
                  const int64_t* core_off, int32_t* core_idx,
                  const int64_t* shell_off, int32_t* shell_idx,
                  const int64_t* full_off, int32_t* full_idx)
{
    orc_thr th = thresholds(s->rs, s->rc, s->skin);
    orc_row row = {0};
    orc_rowcap cap = {0, 0, 0};
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        if (i < 0 || i >= s->n) return -1;
        build_row(s, th, method, i, &row, &cap);
        if (core_idx) {
            if (core_off[k + 1] - core_off[k] != row.nc) return -2;
            for (int64_t q = 0; q < row.nc; ++q) core_idx[core_off[k] + q] = (int32_t)row.core[q];
        }
        if (shell_idx) {
            if (shell_off[k + 1] - shell_off[k] != row.ns) return -2;
            for (int64_t q = 0; q < row.ns; ++q) shell_idx[shell_off[k] + q] = (int32_t)row.shell[q];
        }
        if (full_idx) {
            if (full_off[k + 1] - full_off[k] != row.nf) return -2;
            for (int64_t q = 0; q < row.nf; ++q) full_idx[full_off[k] + q] = (int32_t)row.full[q];
        }
    }
    free(row.core); free(row.shell); free(row.full);
    return 0;
}

/* Stencil rows: for each requested row (all when rows == NULL) the IDs of
 * all particles in the stencil cells of its cell (the 5 x 5 x 5 block, each
 * cell once when an axis has fewer than 5 cells), the particle itself
 * included, in ascending slot order.  With idx == NULL only the counts are
 * written to off[k] (length nrows); otherwise off holds the nrows + 1 CSR
 * offsets and idx is filled. */
int orc_stencil_rows(const orc_sys* s, int64_t nrows, const int64_t* rows, int64_t* off,
                     int32_t* idx)
{
    if (s->T.nt) return -4;  /* the stencil population is a one-type form */
    int64_t cap = 64;
    int64_t* buf = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        if (i < 0 || i >= s->n) { free(buf); return -1; }
        int64_t ci = s->cell_of[i];
        int cx = (int)(ci % s->ncell[0]);
        int cy = (int)((ci / s->ncell[0]) % s->ncell[1]);
        int cz = (int)(ci / ((int64_t)s->ncell[0] * s->ncell[1]));
        int sx[5], sy[5], sz[5];
        int nx = stencil_axis(cx, s->ncell[0], ORC_HALF_STENCIL, sx);
        int ny = stencil_axis(cy, s->ncell[1], ORC_HALF_STENCIL, sy);
        int nz = stencil_axis(cz, s->ncell[2], ORC_HALF_STENCIL, sz);
        int64_t m = 0;
        for (int a = 0; a < nz; ++a)
            for (int b = 0; b < ny; ++b)
                for (int c = 0; c < nx; ++c) {
                    int64_t cell = ((int64_t)sz[a] * s->ncell[1] + sy[b]) * s->ncell[0] + sx[c];
                    for (int64_t q = s->cell_start[cell]; q < s->cell_start[cell + 1]; ++q) {
                        if (m == cap) {
                            cap *= 2;
                            buf = (int64_t*)realloc(buf, sizeof(int64_t) * (size_t)cap);
                        }
                        buf[m++] = s->id_of[q];
                    }
                }
        if (!idx) {
            off[k] = m;
            continue;
        }
        if (off[k + 1] - off[k] != m) { free(buf); return -2; }
        g_sort_sys = s;
        qsort(buf, (size_t)m, sizeof(int64_t), cmp_slot);
        for (int64_t q = 0; q < m; ++q) idx[off[k] + q] = (int32_t)buf[q];
    }
    free(buf);
    return 0;
}

/* The stencil population on the grid the paper describes (Sec. II): cells of
 * edge w at least the core radius (here rs + skin, times 1 + 1e-6, so that the
 * 27 nearest cells hold every core candidate), and around particle i's cell
 * the (2h+1)^3 cells with h = floor((rc + skin)/w) + 1 -- the paper's
 * (2 floor(r/w) + 3)^3 with the outer radius widened by the skin, which the
 * list lifetime needs (every particle within rc + skin of i is in these
 * cells).  An axis of fewer than 2h+1 cells contributes every cell once.
 * Members, i included, are listed in the slot order of that grid (cell by
 * z-major index, then ID).  off/idx as orc_stencil_rows (idx NULL: counts
 * into off[k]); ncell and h (may be NULL) receive the grid and half-width. */
int orc_paper_stencil_rows(int64_t n, const double* pos, const double box[3], double rs, double rc,
                           double skin, int64_t nrows, const int64_t* rows, int64_t* off, int32_t* idx,
                           int32_t* ncell_out, int32_t* h_out)
{
    double w = (rs + skin) * 1.000001;
    int nc[3];
    for (int a = 0; a < 3; ++a) {
        double c = floor(box[a] / w);
        nc[a] = c < 1.0 ? 1 : (int)c;
    }
    int h = (int)floor((rc + skin) / w) + 1;
    if (ncell_out) for (int a = 0; a < 3; ++a) ncell_out[a] = nc[a];
    if (h_out) *h_out = h;
    double* wp = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    memcpy(wp, pos, sizeof(double) * 3 * (size_t)n);
    orc_wrap(n, wp, box);
    int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t* cell_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t* start = (int64_t*)calloc((size_t)ncells + 1, sizeof(int64_t));
    int64_t* id_of = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t c[3];
        for (int a = 0; a < 3; ++a) {
            double f = floor(wp[a * n + i] * ((double)nc[a] / box[a]));
            int64_t k = (int64_t)f;
            if (k < 0) k = 0;
            if (k > nc[a] - 1) k = nc[a] - 1;
            c[a] = k;
        }
        cell_of[i] = (c[2] * nc[1] + c[1]) * nc[0] + c[0];
        start[cell_of[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncells; ++c) start[c + 1] += start[c];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncells + 1));
    memcpy(fill, start, sizeof(int64_t) * (size_t)(ncells + 1));
    for (int64_t i = 0; i < n; ++i) id_of[fill[cell_of[i]]++] = i;  /* IDs ascending within a cell */
    int rcode = 0;
    for (int64_t k = 0; k < nrows && !rcode; ++k) {
        int64_t i = rows ? rows[k] : k;
        if (i < 0 || i >= n) { rcode = -1; break; }
        int64_t ci = cell_of[i];
        int ctr[3] = {(int)(ci % nc[0]), (int)((ci / nc[0]) % nc[1]), (int)(ci / ((int64_t)nc[0] * nc[1]))};
        /* the member cells per axis, ascending */
        int ax[3][64], na[3];
        for (int a = 0; a < 3; ++a) {
            char on[4096] = {0};
            if (nc[a] > 4096 || 2 * h + 1 > 64) { rcode = -3; break; }
            if (2 * h + 1 >= nc[a]) {
                for (int q = 0; q < nc[a]; ++q) on[q] = 1;
            } else {
                for (int d = -h; d <= h; ++d) on[((ctr[a] + d) % nc[a] + nc[a]) % nc[a]] = 1;
            }
            na[a] = 0;
            for (int q = 0; q < nc[a]; ++q)
                if (on[q]) ax[a][na[a]++] = q;
        }
        if (rcode) break;
        int64_t m = 0;
        for (int zz = 0; zz < na[2]; ++zz)
            for (int yy = 0; yy < na[1]; ++yy)
                for (int xx = 0; xx < na[0]; ++xx) {
                    int64_t cell = ((int64_t)ax[2][zz] * nc[1] + ax[1][yy]) * nc[0] + ax[0][xx];
                    for (int64_t q = start[cell]; q < start[cell + 1]; ++q) {
                        if (idx) {
                            if (off[k] + m >= off[k + 1]) { rcode = -2; break; }
                            idx[off[k] + m] = (int32_t)id_of[q];
                        }
                        m += 1;
                    }
                }
        if (!idx) off[k] = m;
        else if (!rcode && off[k] + m != off[k + 1]) rcode = -2;
    }
    free(wp); free(cell_of); free(start); free(id_of); free(fill);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* Pair (i, j) at squared distance r2: the factor of x_i - x_j and the energy
 * shifted by the cut-off value (one type: LJ plus the erfc term of charges;
 * typed: the pair's own LJ), and the pair's squared radii. */
static void pair_eval(const orc_types* T, orc_shift sh, const double* q, double alpha,
                      int64_t i, int64_t j, double r2, double* fmag, double* ushifted)
{
    double u;
    if (T->nt) {
        int a = T->type[i], b = T->type[j];
        orc_lj_typed(r2, T->eps[a][b], T->sig[a][b], fmag, &u);
        *ushifted = u - T->ush[a][b];
        return;
    }
    pair_term(r2, q, alpha, i, j, fmag, &u);
    *ushifted = u - pair_shift(sh, q, i, j);
}

static double pair_rs2(const orc_types* T, double rs2, int64_t i, int64_t j)
{
    return T->nt ? T->rs2[T->type[i]][T->type[j]] : rs2;
}

static double pair_rc2(const orc_types* T, double rc2, int64_t i, int64_t j)
{
    return T->nt ? T->rc2[T->type[i]][T->type[j]] : rc2;
}

/* ------------------------------------------------------------------------ */
/* Forces.  Positions `pos` ([3][n]) are the current ones (not necessarily
 * the ones the lists were built at); every pair is classified by its current
 * squared distance.  Row k of the CSR lists belongs to particle rows[k]
 * (rows == NULL: row k is particle k).  Outputs per row: f ([3][nrows]),
 * e (pair energy, half per particle), w (virial sum of r.f, half per
 * particle).  No mean-force subtraction here.  nt, type, eps_sig: particle
 * types as in orc_sys_new_typed (nt = 0: one type; not with charges);
 * returns -4 for an invalid type table. */

int orc_forces_rbl(int64_t n, const double* pos, const double box[3],
                   double rs, double rc, int shift,
                   int64_t nrows, const int64_t* rows,
                   const int64_t* core_off, const int32_t* core_idx,
                   const int64_t* shell_off, const int32_t* shell_idx,
                   int p, uint64_t seed, uint64_t step, uint32_t replica,
                   const int64_t* pid, const double* charge, double alpha,
                   double* f, double* e, double* w,
                   int nt, const int32_t* type, const double* eps_sig)
{
    double inv[3] = {1.0 / box[0], 1.0 / box[1], 1.0 / box[2]};
    double rs2 = rs * rs, rc2 = rc * rc;
    orc_shift sh = cutoff_shift(rc2, shift, charge, alpha);
    orc_types T;
    if ((nt && charge) || types_setup(&T, n, nt, type, eps_sig, rs, rc, shift)) return -4;
    int32_t* K = (int32_t*)malloc(sizeof(int32_t) * (size_t)(p > 0 ? p : 1));
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        double d[3], fm, u;
        /* core: exact sum over r < rs, eq. (3) */
        double Fc[3] = {0, 0, 0}, ec = 0.0, wc = 0.0;
        for (int64_t q = core_off[k]; q < core_off[k + 1]; ++q) {
            int64_t j = core_idx[q];
            double r2 = dist2(pos, n, i, j, box, inv, d);
            if (r2 < pair_rs2(&T, rs2, i, j)) {
                pair_eval(&T, sh, charge, alpha, i, j, r2, &fm, &u);
                for (int a = 0; a < 3; ++a) Fc[a] += fm * d[a];
                ec += u;
                wc += fm * r2;
            }
        }
        /* shell: batch of p candidates, scaled by n_i/p, eq. (4); only
         * candidates whose current distance lies in [rs, rc) contribute. */
        int ns = (int)(shell_off[k + 1] - shell_off[k]);
        uint32_t id_for_rng = (uint32_t)(pid ? pid[k] : i);
        int cnt = orc_batch_positions(seed, id_for_rng, step, replica, p, ns, K);
        double scale = ns > p ? (double)ns / (double)p : 1.0;
        double Fs[3] = {0, 0, 0}, es = 0.0, ws = 0.0;
        for (int m = 0; m < cnt; ++m) {
            int64_t j = shell_idx[shell_off[k] + K[m]];
            double r2 = dist2(pos, n, i, j, box, inv, d);
            if (r2 >= pair_rs2(&T, rs2, i, j) && r2 < pair_rc2(&T, rc2, i, j)) {
                pair_eval(&T, sh, charge, alpha, i, j, r2, &fm, &u);
                for (int a = 0; a < 3; ++a) Fs[a] += fm * d[a];
                es += u;
                ws += fm * r2;
            }
        }
        for (int a = 0; a < 3; ++a) f[a * nrows + k] = Fc[a] + scale * Fs[a];
        if (e) e[k] = 0.5 * (ec + scale * es);
        if (w) w[k] = 0.5 * (wc + scale * ws);
    }
    free(K);
    types_free(&T);
    return 0;
}

int orc_forces_full(int64_t n, const double* pos, const double box[3],
                    double rc, int shift, int64_t nrows, const int64_t* rows,
                    const int64_t* full_off, const int32_t* full_idx,
                    const double* charge, double alpha, double* f, double* e, double* w,
                    int nt, const int32_t* type, const double* eps_sig)
{
    double inv[3] = {1.0 / box[0], 1.0 / box[1], 1.0 / box[2]};
    double rc2 = rc * rc;
    orc_shift sh = cutoff_shift(rc2, shift, charge, alpha);
    orc_types T;
    /* the core radius does not enter the full list: 0 for the table */
    if ((nt && charge) || types_setup(&T, n, nt, type, eps_sig, 0.0, rc, shift)) return -4;
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        double d[3], fm, u;
        double F[3] = {0, 0, 0}, ei = 0.0, wi = 0.0;
        for (int64_t q = full_off[k]; q < full_off[k + 1]; ++q) {
            int64_t j = full_idx[q];
            double r2 = dist2(pos, n, i, j, box, inv, d);
            if (r2 < pair_rc2(&T, rc2, i, j)) {
                pair_eval(&T, sh, charge, alpha, i, j, r2, &fm, &u);
                for (int a = 0; a < 3; ++a) F[a] += fm * d[a];
                ei += u;
                wi += fm * r2;
            }
        }
        for (int a = 0; a < 3; ++a) f[a * nrows + k] = F[a];
        if (e) e[k] = 0.5 * ei;
        if (w) w[k] = 0.5 * wi;
    }
    types_free(&T);
    return 0;
}

/* Average net force (F_cor of Appendix A) subtracted from every particle, so
 * that the total force, and with it the total momentum, is conserved. */
void orc_mean_subtract(int64_t n, double* f, double out_mean[3])
{
    for (int a = 0; a < 3; ++a) {
        double sum = 0.0;
        for (int64_t i = 0; i < n; ++i) sum += f[a * n + i];
        double mean = sum / (double)n;
        for (int64_t i = 0; i < n; ++i) f[a * n + i] = f[a * n + i] - mean;
        if (out_mean) out_mean[a] = mean;
    }
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 for NVE velocity Verlet (unit mass).  Lists are built at the
 * first force evaluation and rebuilt whenever the index of the next force
 * evaluation is a multiple of K; positions are wrapped into the box at every
 * build.  Force evaluation s draws its batches with step counter s.
 *   v += (dt/2) F;  x += dt v;  [rebuild];  F = force(s+1);  v += (dt/2) F
 * ev_out (may be NULL) receives, per force evaluation (nsteps+1 of them),
 * the potential energy and the virial. */

typedef struct {
    int64_t *core_off, *shell_off, *full_off;
    int32_t *core_idx, *shell_idx, *full_idx;
} orc_lists;

static void free_lists(orc_lists* L)
{
    free(L->core_off); free(L->shell_off); free(L->full_off);
    free(L->core_idx); free(L->shell_idx); free(L->full_idx);
    memset(L, 0, sizeof(*L));
}

static int build_all(int64_t n, double* pos, const double box[3], double rs, double rc,
                     double skin, int use_full, int stencil, orc_lists* L,
                     int nt, const int32_t* type, const double* eps_sig)
{
    free_lists(L);
    if (nt && stencil) return -4;
    orc_wrap(n, pos, box);
    orc_sys* s = orc_sys_new_typed(n, pos, box, rs, rc, skin, nt, type, eps_sig);
    if (!s) return -4;
    int64_t* counts = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)n);
    orc_list_counts(s, 0, n, NULL, counts);
    L->core_off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    L->shell_off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    L->full_off = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) {
        L->core_off[i + 1] = L->core_off[i] + counts[i];
        L->shell_off[i + 1] = L->shell_off[i] + counts[n + i];
        L->full_off[i + 1] = L->full_off[i] + counts[2 * n + i];
    }
    free(counts);
    if (use_full) {
        L->full_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->full_off[n] + 1));
    } else {
        L->core_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->core_off[n] + 1));
        L->shell_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->shell_off[n] + 1));
    }
    int rcode = orc_list_fill(s, 0, n, NULL, L->core_off, L->core_idx,
                              stencil ? NULL : L->shell_off, stencil ? NULL : L->shell_idx,
                              L->full_off, L->full_idx);
    if (!rcode && stencil && !use_full) {
        /* the draw population is the stencil cells (the paper's own form):
         * on the 5x5x5 search grid (stencil 1) or on the grid Sec. II
         * describes (stencil 2, orc_paper_stencil_rows) */
        int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
        if (stencil == 2) rcode = orc_paper_stencil_rows(n, pos, box, rs, rc, skin, n, NULL, cnt, NULL, NULL, NULL);
        else orc_stencil_rows(s, n, NULL, cnt, NULL);
        if (!rcode) {
            L->shell_off[0] = 0;
            for (int64_t i = 0; i < n; ++i) L->shell_off[i + 1] = L->shell_off[i] + cnt[i];
            free(L->shell_idx);
            L->shell_idx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(L->shell_off[n] + 1));
            rcode = stencil == 2 ? orc_paper_stencil_rows(n, pos, box, rs, rc, skin, n, NULL, L->shell_off,
                                                          L->shell_idx, NULL, NULL)
                                 : orc_stencil_rows(s, n, NULL, L->shell_off, L->shell_idx);
        }
        free(cnt);
    }
    orc_sys_free(s);
    return rcode;
}

/* ------------------------------------------------------------------------ */
/* Langevin thermostat (Sec. II, m dv = (F - gamma v) dt + sqrt(2 gamma kT)
 * dW; Sec. III: velocity Verlet with underdamped Langevin, gamma = 1).
 * The Ornstein-Uhlenbeck part over a step dt is solved exactly:
 *   v <- c v + sqrt(kT (1 - c^2)) xi,   c = exp(-gamma dt),  xi ~ N(0, 1).
 * The normal numbers of particle pid at step s come from the Philox block
 * with counter (pid, s mod 2^32, replica, 2^31), key (seed mod 2^32,
 * seed >> 32): the batch draws use blocks below 2^31 of the same counters,
 * so the two streams never share a block.  Each word w gives the uniform
 * u = (w + 1/2) 2^-32 in (0, 1); the pairs (u0, u1) and (u2, u3) go through
 * the Box-Muller transform sqrt(-2 ln u) (cos 2 pi u', sin 2 pi u'), and the
 * first three of the four numbers are used. */

#define ORC_NOISE_BLOCK 0x80000000u

void orc_langevin_noise(uint64_t seed, uint32_t pid, uint64_t step, uint32_t replica, double g[3])
{
    uint32_t ctr[4] = {pid, (uint32_t)step, replica, ORC_NOISE_BLOCK};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)w[k] + 0.5) * 2.3283064365386962890625e-10;
    const double two_pi = 6.283185307179586476925286766559;
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    g[0] = r0 * cos(two_pi * u[1]);
    g[1] = r0 * sin(two_pi * u[1]);
    g[2] = r1 * cos(two_pi * u[3]);
}

/* ------------------------------------------------------------------------ */
/* Radial distribution function (Sec. III): g(r) = (1/(N rho)) sum_i
 * sum_{j != i} <delta(r_ij - r)> / (4 pi r^2).  This is its histogram part:
 * counts[k] += number of ordered pairs (i, j), i != j, whose minimum-image
 * distance r falls in [k dr, (k+1) dr), dr = r_max / nbins, r < r_max.  The
 * bin is decided on r^2 against the squared edges (k dr)(k dr), so that it
 * does not depend on how the square root rounds. */

static double rdf_edge2(int k, double dr)
{
    double e = (double)k * dr;
    return e * e;
}

int orc_rdf(int64_t n, const double* pos, const double box[3], double r_max, int nbins,
            uint64_t* counts)
{
    if (n < 0 || nbins < 1 || !(r_max > 0.0)) return -1;
    double inv[3] = {1.0 / box[0], 1.0 / box[1], 1.0 / box[2]};
    double dr = r_max / (double)nbins;
    double top2 = rdf_edge2(nbins, dr);
    double d[3];
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double r2 = dist2(pos, n, i, j, box, inv, d);
            if (!(r2 < top2)) continue;
            int k = (int)(sqrt(r2) / dr);
            if (k > nbins - 1) k = nbins - 1;
            while (k > 0 && r2 < rdf_edge2(k, dr)) --k;
            while (k < nbins - 1 && r2 >= rdf_edge2(k + 1, dr)) ++k;
            counts[k] += 1;
        }
    return 0;
}

/* Tail corrections for the LJ pairs beyond the cut-off rc (Sec. III, after
 * Frenkel & Smit), with sigma = epsilon = 1 and number density rho:
 *   energy per particle  (8/3) pi rho (1/(3 rc^9) - 1/rc^3),
 *   pressure             (16/3) pi rho^2 (2/(3 rc^9) - 1/rc^3). */
void orc_tail(double rho, double rc, double* u_tail, double* p_tail)
{
    const double pi = 3.141592653589793238462643383279;
    double i3 = 1.0 / (rc * rc * rc);
    double i9 = i3 * i3 * i3;
    *u_tail = (8.0 / 3.0) * pi * rho * (i9 / 3.0 - i3);
    *p_tail = (16.0 / 3.0) * pi * rho * rho * (2.0 * i9 / 3.0 - i3);
}

static void total_ev(int64_t n, const double* e, const double* w, double* out)
{
    double U = 0.0, W = 0.0;
    for (int64_t i = 0; i < n; ++i) { U += e[i]; W += w[i]; }
    out[0] = U;
    out[1] = W;
}

/* Algorithm 1.  gamma == 0: velocity Verlet (NVE), per step
 *   v += (dt/2) F;  x += dt v;  [rebuild];  F = force(s);  v += (dt/2) F.
 * gamma > 0: BAOAB (Leimkuhler & Matthews 2013), per step
 *   v += (dt/2) F;  x += (dt/2) v;  v = c v + sqrt(kT (1 - c^2)) xi(s);
 *   x += (dt/2) v;  [rebuild];  F = force(s);  v += (dt/2) F
 * with c = exp(-gamma dt) and xi(s) the normal numbers of orc_langevin_noise
 * for the force evaluation s that the step leads to.  `unwrapped` (may be
 * NULL) receives the same position increments as pos but is never wrapped
 * into the box: it is the continuous trajectory (for the mean-squared
 * displacement), and must hold the starting positions on entry.  nt, type,
 * eps_sig: particle types as in orc_sys_new_typed (nt = 0: one type). */
int orc_md_run(int64_t n, double* pos, double* vel, const double box[3],
               double rs, double rc, double skin, double dt, int64_t nsteps,
               int p, uint64_t seed, int64_t step0, int K, int use_full,
               int shift, int momentum_fix, uint32_t replica,
               const double* charge, double alpha, int stencil,
               double gamma, double kT, double* unwrapped,
               double* force_out, double* ev_out,
               int check, int64_t* build_steps, int64_t* n_builds,
               int nt, const int32_t* type, const double* eps_sig)
{
    if (K < 1 || n < 1 || !(gamma >= 0.0) || !(kT >= 0.0)) return -1;
    /* Lists rebuilt on displacement (check != 0): the Verlet-list criterion
     * behind the skin of Sec. II -- the lists stay complete as long as no
     * particle has moved more than half the skin since they were built --
     * checked at every step after the drift, and at the latest K steps
     * after the last build.  Otherwise before every evaluation s with
     * s mod K == 0.  Builds are recorded in build_steps (nsteps + 1
     * entries) when given. */
    double half2 = (0.5 * skin) * (0.5 * skin);
    double* xb = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    int64_t last_build = step0, nb = 0;
    double c_ou = exp(-gamma * dt);
    double s_ou = sqrt(kT * (1.0 - c_ou * c_ou));
    orc_lists L = {0};
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    double* e = (double*)malloc(sizeof(double) * (size_t)n);
    double* w = (double*)malloc(sizeof(double) * (size_t)n);
    double h = 0.5 * dt;
    int rcode = 0;
    for (int64_t it = 0; it <= nsteps; ++it) {
        int64_t s = step0 + it;
        if (it > 0 && gamma == 0.0) {
            /* first half of step it-1: kick and drift */
            for (int64_t i = 0; i < 3 * n; ++i) vel[i] = vel[i] + h * F[i];
            for (int64_t i = 0; i < 3 * n; ++i) {
                pos[i] = pos[i] + dt * vel[i];
                if (unwrapped) unwrapped[i] = unwrapped[i] + dt * vel[i];
            }
        } else if (it > 0) {
            /* B, A, O, A of step it-1 */
            for (int64_t i = 0; i < n; ++i) {
                double g[3];
                orc_langevin_noise(seed, (uint32_t)i, (uint64_t)s, replica, g);
                for (int a = 0; a < 3; ++a) {
                    int64_t q = a * n + i;
                    vel[q] = vel[q] + h * F[q];
                    pos[q] = pos[q] + h * vel[q];
                    if (unwrapped) unwrapped[q] = unwrapped[q] + h * vel[q];
                    vel[q] = c_ou * vel[q] + s_ou * g[a];
                    pos[q] = pos[q] + h * vel[q];
                    if (unwrapped) unwrapped[q] = unwrapped[q] + h * vel[q];
                }
            }
        }
        int rebuild = it == 0;
        if (it > 0 && !check) rebuild = s % K == 0;
        if (it > 0 && check) {
            rebuild = s - last_build >= K;
            for (int64_t i = 0; i < n && !rebuild; ++i) {
                double dx = pos[i] - xb[i];
                double dy = pos[n + i] - xb[n + i];
                double dz = pos[2 * n + i] - xb[2 * n + i];
                if (dx * dx + dy * dy + dz * dz > half2) rebuild = 1;
            }
        }
        if (rebuild) {
            rcode = build_all(n, pos, box, rs, rc, skin, use_full, stencil, &L, nt, type, eps_sig);
            if (rcode) break;
            memcpy(xb, pos, sizeof(double) * 3 * (size_t)n);  /* positions as wrapped by the build */
            last_build = s;
            if (build_steps) build_steps[nb] = s;
            nb += 1;
        }
        if (use_full) {
            rcode = orc_forces_full(n, pos, box, rc, shift, n, NULL, L.full_off, L.full_idx, charge, alpha,
                                    F, e, w, nt, type, eps_sig);
        } else {
            rcode = orc_forces_rbl(n, pos, box, rs, rc, shift, n, NULL, L.core_off, L.core_idx,
                                   L.shell_off, L.shell_idx, p, seed, (uint64_t)s, replica, NULL,
                                   charge, alpha, F, e, w, nt, type, eps_sig);
            if (momentum_fix) orc_mean_subtract(n, F, NULL);
        }
        if (rcode) break;
        if (ev_out) total_ev(n, e, w, ev_out + 2 * it);
        if (it > 0) {
            /* second half of step it-1: kick with the new force */
            for (int64_t i = 0; i < 3 * n; ++i) vel[i] = vel[i] + h * F[i];
        }
    }
    if (force_out) memcpy(force_out, F, sizeof(double) * 3 * (size_t)n);
    if (n_builds) *n_builds = nb;
    free(F); free(e); free(w); free(xb);
    free_lists(&L);
    return rcode;
}
