// Device-side building blocks for gfx950 (wave64): Philox4x32-10, Floyd's
// sampler in registers, the canonical minimum image, the LJ pair term in
// FP64 and mixed precision, and DPP wavefront scans/reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rbl {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Replica table entry (one per independent system).
struct DevReplica {
    double L[3];       // box edges
    double inv[3];     // 1 / L
    double cscale[3];  // cells per unit length: ncell / L
    int nc[3];         // cells per axis
    int pad0;
    int64_t id_base;   // first caller ID
    int64_t n;         // particles
    int64_t slot_base; // first slot (multiple of 64)
    int64_t cell_base; // first global cell index
};

// Index of entry k of the row of `slot` in a sliced-ELL array: slices of 64
// consecutive slots, each stored column-major with `cap` columns, so that the
// 64 lanes of a wavefront reading column k touch one contiguous 256-byte run.
__device__ __forceinline__ int64_t ell(int64_t slot, int k, int cap)
{
    return ((slot >> 6) * (int64_t)cap + k) * 64 + (slot & 63);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product per multiplier gives both halves
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x0 = y0;
        x1 = (uint32_t)p1;
        x2 = y2;
        x3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Floyd's sampling without replacement of P positions out of {0..n-1}
// (n > P), kept sorted ascending in S[0..P) (S[P..PMAX) = 0xFFFFFFFF).
// Random words: Philox block b = m/4 at counter (pid, step, replica, b),
// word m % 4; choice t = floor(u (J+1) / 2^32) with J = n - P + m.
// Insertion into the sorted array uses only static indices, so S stays in
// VGPRs: new S[q] = min(S[q], max(S[q-1], v)).  Up to PMAX = 32 the loop
// over m is unrolled, so that step m compares and inserts against the m
// filled entries only (the unfilled ones hold 0xFFFFFFFF, which no choice
// equals and which the insertion leaves in place).
template <int PMAX>
__device__ __forceinline__ void floyd_draw(uint32_t (&S)[PMAX], uint64_t seed, uint32_t pid,
                                           uint32_t step, uint32_t replica, int P, int n)
{
#pragma unroll
    for (int q = 0; q < PMAX; ++q) S[q] = 0xFFFFFFFFu;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if constexpr (PMAX <= 32) {
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int m = 0; m < PMAX; ++m) {
            if (m >= P) continue;  // P is uniform across the wavefront
            if ((m & 3) == 0) {
                w[0] = pid;
                w[1] = step;
                w[2] = replica;
                w[3] = (uint32_t)(m >> 2);
                // the key schedule is advanced round by round in SGPRs
                // instead of being precomputed for all blocks (20 values that
                // would be spilled); the empty asm marks the key as changed
                uint32_t kk0 = k0, kk1 = k1;
                asm volatile("" : "+s"(kk0), "+s"(kk1));
                philox4x32_10(w[0], w[1], w[2], w[3], kk0, kk1);
            }
            const uint32_t u = w[m & 3];
            const uint32_t J = (uint32_t)(n - P + m);
            const uint32_t t = (uint32_t)(((uint64_t)u * (uint64_t)(J + 1u)) >> 32);
            bool taken = false;
#pragma unroll
            for (int q = 0; q < m; ++q) taken |= (S[q] == t);
            const uint32_t v = taken ? J : t;
#pragma unroll
            for (int q = m; q > 0; --q) S[q] = min(S[q], max(S[q - 1], v));
            S[0] = min(S[0], v);
        }
    } else {
        uint32_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
        for (int m = 0; m < P; ++m) {
            const int sub = m & 3;
            if (sub == 0) {
                w0 = pid;
                w1 = step;
                w2 = replica;
                w3 = (uint32_t)(m >> 2);
                philox4x32_10(w0, w1, w2, w3, k0, k1);
            }
            const uint32_t u = sub == 0 ? w0 : sub == 1 ? w1 : sub == 2 ? w2 : w3;
            const uint32_t J = (uint32_t)(n - P + m);
            const uint32_t t = __umulhi(u, J + 1u);
            bool taken = false;
#pragma unroll
            for (int q = 0; q < PMAX; ++q) taken |= (S[q] == t);
            const uint32_t v = taken ? J : t;
#pragma unroll
            for (int q = PMAX - 1; q > 0; --q) S[q] = min(S[q], max(S[q - 1], v));
            S[0] = min(S[0], v);
        }
    }
}

// ---------------------------------------------------------------------------
// Canonical geometry (bit-identical to the CPU reference: explicit fma,
// round-to-nearest-even, no contraction).
__device__ __forceinline__ double min_image(double d, double L, double inv)
{
    const double k = rint(d * inv);
    return fma(-k, L, d);
}

__device__ __forceinline__ double wrap_coord(double x, double L, double inv)
{
    const double k = floor(x * inv);
    return fma(-k, L, x);
}

struct Delta {
    double x, y, z, r2;
};

__device__ __forceinline__ Delta delta(const double4& a, const double4& b, const DevReplica& R)
{
    Delta d;
    d.x = min_image(a.x - b.x, R.L[0], R.inv[0]);
    d.y = min_image(a.y - b.y, R.L[1], R.inv[1]);
    d.z = min_image(a.z - b.z, R.L[2], R.inv[2]);
    d.r2 = fma(d.z, d.z, fma(d.y, d.y, d.x * d.x));
    return d;
}

// ---------------------------------------------------------------------------
// LJ 12-6 pair term, eq. (1), epsilon = sigma = 1.  fmag multiplies
// (x_i - x_j); u is unshifted.
enum { kFP64 = 0, kMixed = 1 };

template <int PREC>
struct LJ;

template <>
struct LJ<kFP64> {
    __device__ __forceinline__ static void eval(double r2, double& fmag, double& u)
    {
        const double r2i = 1.0 / r2;
        const double sr6 = r2i * r2i * r2i;
        fmag = 24.0 * r2i * sr6 * (2.0 * sr6 - 1.0);
        u = 4.0 * sr6 * (sr6 - 1.0);
    }
};

template <>
struct LJ<kMixed> {
    __device__ __forceinline__ static void eval(double r2, double& fmag, double& u)
    {
        const float r2f = (float)r2;
        const float r2i = __builtin_amdgcn_rcpf(r2f);
        const float sr6 = r2i * r2i * r2i;
        fmag = (double)(24.0f * r2i * sr6 * (2.0f * sr6 - 1.0f));
        u = (double)(4.0f * sr6 * (sr6 - 1.0f));
    }
};

// LJ pair of particle types a, b with their own parameters, eq. (1) with
// epsilon_ab and sigma_ab: the constants come precomputed per pair (24 eps,
// 4 eps, sigma^2), so that eps = sigma = 1 repeats LJ<PREC> operation for
// operation.
template <int PREC>
struct LJt;

template <>
struct LJt<kFP64> {
    __device__ __forceinline__ static void eval(double r2, double eps24, double eps4, double sig2, double& fmag,
                                                double& u)
    {
        const double r2i = 1.0 / r2;
        const double s2 = sig2 * r2i;
        const double sr6 = s2 * s2 * s2;
        fmag = eps24 * r2i * sr6 * (2.0 * sr6 - 1.0);
        u = eps4 * sr6 * (sr6 - 1.0);
    }
};

template <>
struct LJt<kMixed> {
    __device__ __forceinline__ static void eval(double r2, double eps24, double eps4, double sig2, double& fmag,
                                                double& u)
    {
        const float r2f = (float)r2;
        const float r2i = __builtin_amdgcn_rcpf(r2f);
        const float s2 = (float)sig2 * r2i;
        const float sr6 = s2 * s2 * s2;
        fmag = (double)((float)eps24 * r2i * sr6 * (2.0f * sr6 - 1.0f));
        u = (double)((float)eps4 * sr6 * (sr6 - 1.0f));
    }
};

// Real-space Ewald term q_i q_j erfc(alpha r)/r added to the LJ pair.
template <int PREC>
struct Erfc;

template <>
struct Erfc<kFP64> {
    __device__ __forceinline__ static void eval(double r2, double qq, double alpha,
                                                double& fmag, double& u)
    {
        const double r = sqrt(r2);
        const double e = erfc(alpha * r);
        const double g = exp(-alpha * alpha * r2);
        const double two_over_sqrt_pi = 1.1283791670955126;
        const double ir = 1.0 / r;
        u = qq * e * ir;
        fmag = qq * (e * ir + two_over_sqrt_pi * alpha * g) * ir * ir;
    }
};

template <>
struct Erfc<kMixed> {
    __device__ __forceinline__ static void eval(double r2, double qq, double alpha,
                                                double& fmag, double& u)
    {
        const float r2f = (float)r2;
        const float r = sqrtf(r2f);
        const float af = (float)alpha;
        const float e = erfcf(af * r);
        const float g = expf(-af * af * r2f);
        const float ir = __builtin_amdgcn_rcpf(r);
        u = (double)((float)qq * e * ir);
        fmag = (double)((float)qq * (e * ir + 1.12837917f * af * g) * ir * ir);
    }
};

// ---------------------------------------------------------------------------
// DPP wavefront primitives (GFX9 DPP: row_shr, row_bcast:15/31).
// update_dpp(old, src, ctrl, row_mask, bank_mask, bound_ctrl): lanes whose
// row is masked off keep `old` (0 here), so each step adds zero there.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xF, true);
}

// Inclusive prefix sum over the 64 lanes.
__device__ __forceinline__ int wave_incl_scan(int v)
{
    v += dpp_i32<0x111, 0xF>(v);  // row_shr:1
    v += dpp_i32<0x112, 0xF>(v);  // row_shr:2
    v += dpp_i32<0x114, 0xF>(v);  // row_shr:4
    v += dpp_i32<0x118, 0xF>(v);  // row_shr:8
    v += dpp_i32<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_i32<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __double2loint(v);
    const int hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xF, true);
    const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xF, true);
    return __hiloint2double(hi2, lo2);
}

// Sum over the 64 lanes; the result is returned in every lane.  The FP64
// halves travel through 32-bit DPP moves; the order of additions is fixed.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0x111, 0xF>(v);
    v += dpp_f64<0x112, 0xF>(v);
    v += dpp_f64<0x114, 0xF>(v);
    v += dpp_f64<0x118, 0xF>(v);
    v += dpp_f64<0x142, 0xA>(v);
    v += dpp_f64<0x143, 0xC>(v);
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

// Maximum over the 64 lanes (non-negative ints), returned in every lane.
__device__ __forceinline__ int wave_max(int v)
{
    v = max(v, dpp_i32<0x111, 0xF>(v));
    v = max(v, dpp_i32<0x112, 0xF>(v));
    v = max(v, dpp_i32<0x114, 0xF>(v));
    v = max(v, dpp_i32<0x118, 0xF>(v));
    v = max(v, dpp_i32<0x142, 0xA>(v));
    v = max(v, dpp_i32<0x143, 0xC>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

}  // namespace rbl
