// device_math.hpp -- per-pair arithmetic of the super-droplet coalescence step
// on gfx950: counter-based random numbers, collection kernels, the collision
// probability of eq. (P_ij) (Sect. 5.1.4), the collision count with the gamma
// cap, the multiplicity/radius update and a correctly rounded cube root.
//
// Every floating-point expression is evaluated as written, one IEEE binary64
// operation at a time (the file is compiled with -ffp-contract=off and the
// pragma below), so that results are a function of the inputs only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace sdm {

// binary64 nearest to pi, and (4 pi)/3 rounded once per operation
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kFourThirdsPi = (4.0 * kPi) / 3.0;

enum : uint32_t { kGolovin = 0, kGeometric = 1 };

// Kernel parameters in the order of sdm_kernel_params.
struct KernelParams {
    double golovin_b, k1, k2, k3, r1, r2, eff;
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products; the two key words advance by fixed Weyl increments each round.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w[4];
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
    // each 32x32 -> 64-bit product is one v_mad_u64_u32 (high and low halves)
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = static_cast<uint32_t>(pb);
        c2 = n2;
        c3 = static_cast<uint32_t>(pa);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words4 r;
    r.w[0] = c0;
    r.w[1] = c1;
    r.w[2] = c2;
    r.w[3] = c3;
    return r;
}

// Stream tags of the fourth counter word.
enum : uint32_t { kTagShuffle = 0, kTagUniform = 1 };

// Uniform deviate on (0,1) from two 32-bit words (hi, lo): the top 52 bits k
// of hi:lo give (2k+1) 2^-53, exactly representable, never 0 or 1.
__device__ __forceinline__ double uniform_open01(uint32_t hi, uint32_t lo)
{
    const uint64_t k = ((static_cast<uint64_t>(hi) << 32) | lo) >> 12;
    return static_cast<double>((k << 1) | 1u) * 0x1p-53;
}

// Uniform deviate of pair m in cell `cell` at step `step`.
__device__ __forceinline__ double pair_uniform(uint32_t m, uint32_t cell, uint32_t step,
                                               uint32_t k0, uint32_t k1)
{
    const Words4 w = philox4x32_10(m >> 1, cell, step, kTagUniform, k0, k1);
    return (m & 1u) ? uniform_open01(w.w[2], w.w[3]) : uniform_open01(w.w[0], w.w[1]);
}

// ---------------------------------------------------------------------------
// Correctly rounded cube root for positive finite arguments.
// The candidate y = Y 2^e is the rounded cube root iff the exact cubes of the
// midpoints to its neighbours bracket x; cubes are formed on 64-bit limbs.
// ---------------------------------------------------------------------------
struct U192 {
    uint64_t w0, w1, w2;  // little-endian words
};

__device__ __forceinline__ int bit_length(const U192& v)
{
    if (v.w2) return 192 - __clzll(v.w2);
    if (v.w1) return 128 - __clzll(v.w1);
    if (v.w0) return 64 - __clzll(v.w0);
    return 0;
}

__device__ __forceinline__ U192 cube_u64(uint64_t m)
{
    // m^2 = (s1:s0), then (s1:s0) * m = (w2:w1:w0)
    const uint64_t s0 = m * m;
    const uint64_t s1 = __umul64hi(m, m);
    U192 c;
    c.w0 = s0 * m;
    const uint64_t t = __umul64hi(s0, m);
    const uint64_t u = s1 * m;
    c.w1 = u + t;
    c.w2 = __umul64hi(s1, m) + (c.w1 < t ? 1u : 0u);
    return c;
}

__device__ __forceinline__ U192 shl_u64_to_192(uint64_t x, int d)
{
    U192 r{0, 0, 0};
    const int word = d >> 6, bit = d & 63;
    const uint64_t lo = x << bit;
    const uint64_t hi = bit ? (x >> (64 - bit)) : 0u;
    if (word == 0) { r.w0 = lo; r.w1 = hi; }
    else if (word == 1) { r.w1 = lo; r.w2 = hi; }
    else if (word == 2) { r.w2 = lo; }
    return r;
}

// sign of (m 2^em)^3 - (x 2^ex) with 2^52 <= m < 2^56 and 0 < x < 2^53
__device__ __forceinline__ int cube_vs(uint64_t m, int em, uint64_t x, int ex)
{
    const U192 c = cube_u64(m);
    const int top_c = bit_length(c) + 3 * em;
    const int top_x = (64 - __clzll(x)) + ex;
    if (top_c != top_x) return top_c > top_x ? 1 : -1;
    // equal leading-bit positions: x 2^(ex - 3em) is an integer of the same
    // length as the cube (at most 168 bits)
    const U192 xs = shl_u64_to_192(x, ex - 3 * em);
    if (c.w2 != xs.w2) return c.w2 > xs.w2 ? 1 : -1;
    if (c.w1 != xs.w1) return c.w1 > xs.w1 ? 1 : -1;
    if (c.w0 != xs.w0) return c.w0 > xs.w0 ? 1 : -1;
    return 0;
}

__device__ inline double cbrt_rn(double x)
{
    if (!(x > 0.0) || x == __builtin_inf()) return cbrt(x);  // NaN, 0, negative, inf: not used by the step
    const uint64_t xb = static_cast<uint64_t>(__double_as_longlong(x));
    const int xexp = static_cast<int>((xb >> 52) & 0x7ffu);
    uint64_t X = xb & 0xFFFFFFFFFFFFFull;
    int ex;
    if (xexp == 0) {
        ex = -1074;                    // subnormal: no implicit bit
    } else {
        X |= 1ull << 52;
        ex = xexp - 1075;
    }
    double y = cbrt(x);                // faithful approximation, corrected below
    for (int it = 0; it < 8; ++it) {
        const uint64_t yb = static_cast<uint64_t>(__double_as_longlong(y));
        const int yexp = static_cast<int>((yb >> 52) & 0x7ffu);
        const uint64_t Y = (yb & 0xFFFFFFFFFFFFFull) | (1ull << 52);
        const int e = yexp - 1075;
        // upper midpoint (2Y+1) 2^(e-1)
        if (cube_vs(2u * Y + 1u, e - 1, X, ex) < 0) {
            y = __longlong_as_double(static_cast<long long>(yb + 1u));
            continue;
        }
        // lower midpoint: (2Y-1) 2^(e-1), or (4Y-1) 2^(e-2) at the bottom of a binade
        const bool binade_bottom = (Y == (1ull << 52)) && yexp > 1;
        const int low_vs = binade_bottom ? cube_vs(4u * Y - 1u, e - 2, X, ex)
                                         : cube_vs(2u * Y - 1u, e - 1, X, ex);
        if (low_vs > 0) {
            y = __longlong_as_double(static_cast<long long>(yb - 1u));
            continue;
        }
        break;
    }
    return y;
}

// Remap the hardware workgroup id so that each XCD (workgroups are dealt to
// the 8 XCDs round-robin) works on one contiguous range of logical blocks;
// neighbouring cells then share cache lines in the same L2.
__device__ __forceinline__ uint32_t xcd_contiguous_block(uint32_t bid, uint32_t nblk)
{
    constexpr uint32_t kXcds = 8;
    const uint32_t xcd = bid % kXcds;
    const uint32_t idx = bid / kXcds;
    const uint32_t per = nblk / kXcds;
    const uint32_t extra = nblk % kXcds;
    return xcd * per + (xcd < extra ? xcd : extra) + idx;
}

// ---------------------------------------------------------------------------
// Collection kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ double terminal_velocity(const KernelParams& kp, double r)
{
    if (r < kp.r1) return kp.k1 * (r * r);
    if (r <= kp.r2) return kp.k2 * r;
    return kp.k3 * sqrt(r);
}

// K(r_a, r_b) for the two members of a pair, in pair order.
__device__ __forceinline__ double collection_kernel(uint32_t kind, const KernelParams& kp,
                                                    double ra, double rb)
{
    if (kind == kGolovin) {
        const double va = kFourThirdsPi * ((ra * ra) * ra);
        const double vb = kFourThirdsPi * ((rb * rb) * rb);
        return kp.golovin_b * (va + vb);
    }
    const double s = ra + rb;
    const double cross = kPi * (s * s);
    const double dv = fabs(terminal_velocity(kp, ra) - terminal_velocity(kp, rb));
    return (kp.eff * cross) * dv;
}

// n(n-1)/2 candidate pairs over floor(n/2) examined ones (n >= 2), eq. (P_ij)
__device__ __forceinline__ double upscale_factor(uint32_t n)
{
    const uint64_t nn = n;
    return static_cast<double>((nn * (nn - 1u)) >> 1) / static_cast<double>(nn >> 1);
}

// The same factor for 2 <= n < 2^26, where n(n-1)/2 is exact in binary64 and
// the quotient is the integer n - 1 (n even) or n (n odd): formed directly, it
// equals the rounded quotient bit for bit.
__device__ __forceinline__ double upscale_factor_small(uint32_t n)
{
    return static_cast<double>((n & 1u) ? n : n - 1u);
}

// eq. (P_ij) in the fixed order ((xi_max K) dt / dV) scale
__device__ __forceinline__ double collision_probability(uint64_t xi_max, double K, double dt,
                                                        double dV, double scale)
{
    double p = static_cast<double>(xi_max) * K;
    p = p * dt;
    p = p / dV;
    return p * scale;
}

// gamma = floor(p) + [u < frac(p)], capped at floor(xi_j / xi_k) (xi_j >= xi_k >= 1).
// The 64-bit division is only needed once p >= 1.
__device__ __forceinline__ uint64_t collision_count(double p, double u, uint64_t xj, uint64_t xk)
{
    const double whole = floor(p);
    const double frac = p - whole;
    if (whole < 1.0) return (u < frac) ? 1u : 0u;
    const uint64_t cap = xj / xk;
    if (whole >= static_cast<double>(cap)) return cap;
    const uint64_t g = static_cast<uint64_t>(whole) + ((u < frac) ? 1u : 0u);
    return g < cap ? g : cap;
}

// The release rule of Sect. 5.1.4: one event when u < p, never more.
__device__ __forceinline__ uint64_t collision_count_release(double p, double u)
{
    return (u < p) ? 1u : 0u;
}

// Dry attributes of the droplets formed by g events between j and k
// (Sect. 5.1.4: extensive parameters such as r_d^3 are summed, intensive ones
// such as kappa averaged): each merged droplet holds g droplets of j and one of
// k, so r_d^3 = g r_d,j^3 + r_d,k^3 and kappa is the r_d^3-weighted mean.
__device__ __forceinline__ void merge_dry(uint64_t g, double rd3_j, double kappa_j, double rd3_k,
                                          double kappa_k, double& rd3_new, double& kappa_new)
{
    const double from_j = static_cast<double>(g) * rd3_j;
    const double sum = from_j + rd3_k;
    double weighted = from_j * kappa_j;
    const double weighted_k = rd3_k * kappa_k;
    weighted = weighted + weighted_k;
    rd3_new = sum;
    kappa_new = weighted / sum;
}

// Outcome of g > 0 events between j (xi_j >= xi_k) and k.
struct PairState {
    uint64_t xj, xk;
    double rj, rk;
    bool j_changed_r;   // equal-split case: both radii (and both xi) change
};

// release = true: equal multiplicities leave j with zero multiplicity (and its
// radius) instead of splitting xi_k between both.
__device__ __forceinline__ void apply_collisions(uint64_t g, PairState& s, bool release = false)
{
    const double rj3 = (s.rj * s.rj) * s.rj;
    const double rk3 = (s.rk * s.rk) * s.rk;
    double v = static_cast<double>(g) * rj3;
    v = v + rk3;
    const double rn = cbrt_rn(v);
    const uint64_t moved = g * s.xk;
    if (s.xj > moved) {
        s.xj -= moved;
        s.rk = rn;
        s.j_changed_r = false;
    } else {
        // equal split, or under the release rule j left empty (half = 0)
        const uint64_t half = release ? 0u : (s.xk >> 1);
        s.xj = half;
        s.xk = s.xk - half;
        s.rj = rn;
        s.rk = rn;
        s.j_changed_r = !release;
    }
}

}  // namespace sdm
