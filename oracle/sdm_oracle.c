/*
 * sdm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of one Monte-Carlo
 * coalescence step of the Super-Droplet Method (SDM), as the particle-based
 * scheme of libcloudph++ 0.2 (Arabas, Jaruga, Pawlowska, Grabowski) states it
 * in Sect. 5.1.4 "Coalescence", eq. (P_ij), extended by multiple coalescence
 * with the gamma-capping rule (see oracle_collide_pair), plus the gridded
 * diagnostics of the particle-based scheme (super-droplet concentration and
 * radius moments per cell) and a probe of the largest collision probability a
 * step would meet.
 *
 * It exists to check the HIP library.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the HIP library and includes nothing from it.
 *
 * Build: gcc -O2 -ffp-contract=off (no fast-math) so that every floating-point
 * operation below is one IEEE-754 binary64 operation in the written order.
 *
 * Readings of the paper taken here (the paper is silent or differs):
 *   - n in eq. (P_ij) = number of super-droplets with multiplicity > 0 in the
 *     cell at the start of the step;
 *   - random grouping into non-overlapping pairs = sort the live storage slots
 *     by (32-bit Philox key, slot) and pair neighbours (2m, 2m+1);
 *   - "larger multiplicity" on a tie = the first member of the pair;
 *   - the super-droplet with the smaller multiplicity keeps it and takes the
 *     merged radius, the larger one keeps its radius and loses gamma*xi_k
 *     (the mass-conserving reading of the outcome described in Sect. 5.1.4);
 *   - equal multiplicities after the collision split xi_k in two halves
 *     (instead of leaving a zero-multiplicity particle for recycling);
 *   - random numbers from counter-based Philox4x32-10 instead of the
 *     Mersenne Twister the paper's release uses (Sect. 5.3);
 *   - the release rules (ORACLE_RULE_FIDELITY) keep the same pairing, P_ij
 *     and mass-conserving outcome, with one event when u < P_ij and a zero
 *     multiplicity left on the first pair member when multiplicities are
 *     equal; recycling (ORACLE_RULE_RECYCLE) runs within each cell at the
 *     start of every step, before the pairing, as in oracle_recycle_cell;
 *   - transport: both directions use the Courant numbers of the cell the
 *     particle is in at time level n (dimension-split, not sequential), the
 *     sedimentation fall is applied after the advection, x wraps once per step,
 *     a particle leaving [0, nz dz) gets multiplicity 0 and is clamped into
 *     the boundary row, and the storage is re-sorted by cell keeping the old
 *     storage order within a cell;
 *   - optional dry attributes (r_d^3 and kappa, oracle_dry_merge): the
 *     merged droplets of a collision sum r_d^3 over their constituents and
 *     take the dry-volume-weighted mean of their kappa (the paper names the
 *     two kinds, summed and averaged, without the weight); super-droplets
 *     that keep their radius keep their dry attributes, recycled slots take
 *     the donor's;
 *   - moments count live super-droplets only, the radius range is closed at
 *     both ends, and rho_d defaults to 1 (moments per unit volume) when no
 *     dry-air density is given; the summation order is fixed (see
 *     oracle_moment_cell) so that any implementation can match it bit for bit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* binary64 nearest to pi */
static const double ORACLE_PI = 3.141592653589793238462643383279502884;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications,     */
/* with the key incremented by two Weyl constants between rounds.            */
/* ------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ x1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ x3 ^ k1;
        uint32_t n3 = lo0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Philox over a counter range (test support): element i takes the counter
 * (c0 + lo32(i), c1 + hi32(i), c2, c3), each word modulo 2^32, and the key
 * (k0, k1); out[4i..4i+3] are its four words.  [first, first + n) of the
 * range, so that threads can share one range. */
void oracle_philox_range(uint64_t first, uint64_t n, const uint32_t ctr[4], const uint32_t key[2],
                         uint32_t *out)
{
    for (uint64_t j = 0; j < n; ++j) {
        uint64_t i = first + j;
        uint32_t c[4] = {ctr[0] + (uint32_t)i, ctr[1] + (uint32_t)(i >> 32), ctr[2], ctr[3]};
        oracle_philox4x32_10(c, key, out + 4u * j);
    }
}

/* Shuffle key of storage slot s of cell c at step t: word (s mod 4) of
 * Philox(counter = (s div 4, c, t, 0), key = (seed low, seed high)). */
uint32_t oracle_shuffle_key(uint64_t seed, uint32_t cell, uint32_t step, uint32_t slot)
{
    uint32_t ctr[4] = {slot / 4u, cell, step, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    return w[slot % 4u];
}

/* Uniform deviate on the open interval (0,1) for pair m of cell c at step t:
 * two words of Philox(counter = (m div 2, c, t, 1)) give a 64-bit integer
 * (first word high); its top 52 bits k give u = (2k+1)/2^53, which is exact
 * in binary64 and never 0 or 1. */
double oracle_pair_uniform(uint64_t seed, uint32_t cell, uint32_t step, uint32_t m)
{
    uint32_t ctr[4] = {m / 2u, cell, step, 1u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    uint32_t hi = w[2u * (m % 2u)];
    uint32_t lo = w[2u * (m % 2u) + 1u];
    uint64_t word = ((uint64_t)hi << 32) | (uint64_t)lo;
    uint64_t k = word >> 12;
    return (double)(2u * k + 1u) * 0x1p-53;
}

/* ------------------------------------------------------------------------ */
/* Correctly rounded cube root.  y is the cube root of x rounded to nearest  */
/* iff the exact cubes of the two midpoints around y bracket x.  The test is  */
/* done exactly with 32-bit-limb integers.                                   */
/* ------------------------------------------------------------------------ */
#define BIG_LIMBS 16
typedef struct { uint32_t d[BIG_LIMBS]; } big_t; /* little-endian limbs */

static void big_from_u64(big_t *a, uint64_t v)
{
    memset(a, 0, sizeof(*a));
    a->d[0] = (uint32_t)v;
    a->d[1] = (uint32_t)(v >> 32);
}

static void big_mul_u64(big_t *a, uint64_t v)
{
    /* a <- a * v, schoolbook on 32-bit limbs */
    uint32_t v0 = (uint32_t)v, v1 = (uint32_t)(v >> 32);
    big_t r;
    memset(&r, 0, sizeof(r));
    for (int i = 0; i < BIG_LIMBS; ++i) {
        uint64_t carry = 0;
        for (int j = 0; j < 2; ++j) {
            uint32_t vj = j == 0 ? v0 : v1;
            if (i + j >= BIG_LIMBS) break;
            uint64_t t = (uint64_t)a->d[i] * vj + r.d[i + j] + carry;
            r.d[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
        /* propagate the remaining carry */
        for (int k = i + 2; carry != 0 && k < BIG_LIMBS; ++k) {
            uint64_t t = (uint64_t)r.d[k] + carry;
            r.d[k] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    *a = r;
}

static void big_shl(big_t *a, int bits)
{
    big_t r;
    memset(&r, 0, sizeof(r));
    int limbs = bits / 32, rem = bits % 32;
    for (int i = BIG_LIMBS - 1; i >= 0; --i) {
        int src = i - limbs;
        if (src < 0) continue;
        uint64_t v = (uint64_t)a->d[src] << rem;
        if (rem != 0 && src - 1 >= 0) v |= (uint64_t)a->d[src - 1] >> (32 - rem);
        r.d[i] = (uint32_t)v;
    }
    *a = r;
}

static int big_cmp(const big_t *a, const big_t *b)
{
    for (int i = BIG_LIMBS - 1; i >= 0; --i) {
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    }
    return 0;
}

static int bitlen_u64(uint64_t v)
{
    int n = 0;
    while (v) { ++n; v >>= 1; }
    return n;
}

/* Sign of (M * 2^em)^3 - X * 2^ex for M, X > 0 (M < 2^56, X < 2^54). */
static int cube_cmp(uint64_t M, int em, uint64_t X, int ex)
{
    big_t c, x;
    big_from_u64(&c, M);
    big_mul_u64(&c, M);
    big_mul_u64(&c, M);
    big_from_u64(&x, X);
    int ec = 3 * em;
    /* bit lengths of both values as exponents of 2 */
    int lc = 0;
    for (int i = BIG_LIMBS - 1; i >= 0; --i) {
        if (c.d[i]) { lc = 32 * i + bitlen_u64(c.d[i]); break; }
    }
    int lx = bitlen_u64(X);
    if (lc + ec != lx + ex) return (lc + ec > lx + ex) ? 1 : -1;
    /* same magnitude: align the exponents (the shift is below 3*56 bits) */
    if (ec > ex) big_shl(&c, ec - ex);
    else if (ex > ec) big_shl(&x, ex - ec);
    return big_cmp(&c, &x);
}

/* positive finite normal double -> (Y, e) with d = Y * 2^e, 2^52 <= Y < 2^53 */
static void split_normal(double d, uint64_t *Y, int *e)
{
    int ex;
    double f = frexp(d, &ex);          /* d = f * 2^ex, 0.5 <= f < 1 */
    *Y = (uint64_t)ldexp(f, 53);
    *e = ex - 53;
}

/* positive finite double (normal or subnormal) -> (X, e) with d = X * 2^e */
static void split_any(double d, uint64_t *X, int *e)
{
    int ex;
    double f = frexp(d, &ex);
    *X = (uint64_t)ldexp(f, 53);
    *e = ex - 53;
}

/* midpoint between two adjacent positive normal doubles a < b, as M * 2^em */
static void midpoint(double a, double b, uint64_t *M, int *em)
{
    uint64_t A, B;
    int ea, eb;
    split_normal(a, &A, &ea);
    split_normal(b, &B, &eb);
    int e = ea < eb ? ea : eb;
    uint64_t s = (A << (ea - e)) + (B << (eb - e)); /* both below 2^55 */
    *M = s;
    *em = e - 1;
}

double oracle_cbrt_rn(double x)
{
    if (x != x || x == 0.0 || isinf(x)) return x;
    if (x < 0.0) return -oracle_cbrt_rn(-x);
    uint64_t X;
    int ex;
    split_any(x, &X, &ex);
    double y = cbrt(x);                /* within a few ulp; corrected below */
    for (int guard = 0; guard < 64; ++guard) {
        double up = nextafter(y, INFINITY);
        double dn = nextafter(y, 0.0);
        uint64_t M;
        int em;
        midpoint(y, up, &M, &em);
        if (cube_cmp(M, em, X, ex) < 0) { y = up; continue; }   /* cbrt(x) above the upper midpoint */
        midpoint(dn, y, &M, &em);
        if (cube_cmp(M, em, X, ex) > 0) { y = dn; continue; }   /* below the lower midpoint */
        return y;
    }
    return y; /* not reached for finite positive x */
}

/* ------------------------------------------------------------------------ */
/* Collection kernels                                                        */
/* ------------------------------------------------------------------------ */
enum { ORACLE_GOLOVIN = 0, ORACLE_GEOMETRIC = 1 };

/* params: [0] Golovin b (s^-1), [1] k1 (m^-1 s^-1), [2] k2 (s^-1),
 *         [3] k3 (m^1/2 s^-1), [4] r1 (m), [5] r2 (m), [6] efficiency E */

/* piecewise terminal velocity: Stokes k1 r^2 below r1, k2 r up to and
 * including r2, k3 sqrt(r) above r2 */
double oracle_terminal_velocity(const double *params, double r)
{
    if (r < params[4]) return params[1] * (r * r);
    if (r <= params[5]) return params[2] * r;
    return params[3] * sqrt(r);
}

/* Golovin kernel K = b (v_a + v_b) with v = (4 pi / 3) r^3 (droplet volume). */
static double golovin_kernel(const double *params, double ra, double rb)
{
    const double four_pi_over_3 = (4.0 * ORACLE_PI) / 3.0;
    double va = four_pi_over_3 * ((ra * ra) * ra);
    double vb = four_pi_over_3 * ((rb * rb) * rb);
    return params[0] * (va + vb);
}

/* Geometric kernel of Sect. 5.1.4: K = E pi (r_a + r_b)^2 |v_a - v_b|. */
static double geometric_kernel(const double *params, double ra, double rb)
{
    double sum = ra + rb;
    double area = ORACLE_PI * (sum * sum);
    double dv = fabs(oracle_terminal_velocity(params, ra) - oracle_terminal_velocity(params, rb));
    return (params[6] * area) * dv;
}

double oracle_kernel(int kind, const double *params, double ra, double rb)
{
    return kind == ORACLE_GOLOVIN ? golovin_kernel(params, ra, rb) : geometric_kernel(params, ra, rb);
}

/* Upscaling factor of eq. (P_ij): n(n-1)/2 candidate pairs over floor(n/2) examined ones. */
double oracle_upscale(uint32_t n)
{
    uint64_t all_pairs = (uint64_t)n * (uint64_t)(n - 1u) / 2u;
    uint64_t examined = (uint64_t)(n / 2u);
    return (double)all_pairs / (double)examined;
}

/* eq. (P_ij): p = max(xi_a, xi_b) K dt / dV * scale, evaluated in this order. */
double oracle_probability(uint64_t xi_max, double K, double dt, double dV, double scale)
{
    double p = (double)xi_max * K;
    p = p * dt;
    p = p / dV;
    p = p * scale;
    return p;
}

/* Number of collision events gamma for one pair: floor(p) plus a Bernoulli
 * draw of the fractional part against u, capped at floor(xi_j / xi_k) so the
 * larger super-droplet can supply all of them.  With p < 1 and no binding
 * cap this is the paper's rule "collide iff p > u". */
uint64_t oracle_gamma(double p, double u, uint64_t xi_j, uint64_t xi_k)
{
    uint64_t cap = xi_j / xi_k;
    double fl = floor(p);
    double frac = p - fl;
    if (fl >= (double)cap) return cap;
    uint64_t g = (uint64_t)fl + (u < frac ? 1u : 0u);
    return g < cap ? g : cap;
}

/* Apply gamma collision events between super-droplets j (larger or equal
 * multiplicity) and k.  gamma * xi_k droplets of j merge with the xi_k
 * droplets of k, gamma at a time, so k keeps xi_k and takes the merged radius
 * while j keeps its radius and loses gamma * xi_k.  If that would leave j
 * empty, the xi_k merged droplets are split between both super-droplets. */
void oracle_collide_pair(uint64_t g, uint64_t *xi_j, double *r_j, uint64_t *xi_k, double *r_k)
{
    if (g == 0) return;
    double rj3 = (*r_j * *r_j) * *r_j;
    double rk3 = (*r_k * *r_k) * *r_k;
    double vol = (double)g * rj3;
    vol = vol + rk3;
    double r_new = oracle_cbrt_rn(vol);
    uint64_t removed = g * *xi_k;
    if (*xi_j > removed) {
        *xi_j = *xi_j - removed;
        *r_k = r_new;
    } else {
        uint64_t half = *xi_k / 2u;
        *xi_j = half;
        *xi_k = *xi_k - half;
        *r_j = r_new;
        *r_k = r_new;
    }
}

/* The outcome rules of the paper's own release (Sect. 5.1.4), selected by
 * ORACLE_RULE_FIDELITY: a collision is triggered when the uniform deviate is
 * below P_ij, and then exactly one event happens (no multiple coalescence);
 * equal multiplicities collide by the same scheme, which leaves the larger
 * (first) super-droplet with multiplicity zero. */
#define ORACLE_RULE_FIDELITY 1u
/* Recycling of zero-multiplicity super-droplets at the start of every step. */
#define ORACLE_RULE_RECYCLE 2u

uint64_t oracle_gamma_fidelity(double p, double u)
{
    return u < p ? 1u : 0u;
}

void oracle_collide_pair_fidelity(uint64_t g, uint64_t *xi_j, double *r_j, uint64_t *xi_k,
                                  double *r_k)
{
    (void)r_j;
    if (g == 0) return;
    double rj3 = (*r_j * *r_j) * *r_j;
    double rk3 = (*r_k * *r_k) * *r_k;
    double vol = rj3 + rk3;
    *r_k = oracle_cbrt_rn(vol);
    *xi_j = *xi_j - *xi_k;   /* zero when the multiplicities are equal */
}

/* Dry attributes of the droplets formed by g collision events between j and
 * k (Sect. 5.1.4: extensive parameters such as r_d^3 are summed, intensive
 * ones such as kappa averaged).  Each merged droplet holds g droplets of j and
 * one of k: its r_d^3 is g r_d,j^3 + r_d,k^3 and its kappa the mean of the
 * constituents' kappa weighted by their r_d^3. */
void oracle_dry_merge(uint64_t g, double rd3_j, double kappa_j, double rd3_k, double kappa_k,
                      double *rd3_new, double *kappa_new)
{
    double from_j = (double)g * rd3_j;
    double sum = from_j + rd3_k;
    double weighted = from_j * kappa_j;
    double weighted_k = rd3_k * kappa_k;
    weighted = weighted + weighted_k;
    *rd3_new = sum;
    *kappa_new = weighted / sum;
}

/* Recycling in one cell (the zero-multiplicity rule of Sect. 5.1.4, applied
 * within the cell).  Let z be the number of dead slots (xi = 0) and L the
 * number of live ones.  The donors are the min(z, L) live slots ranked first
 * by multiplicity, largest first, ties broken by the lower slot; those with
 * xi >= 2 can be split.  Taken in ascending slot order, the k-th splittable
 * donor d hands its radius and floor(xi_d / 2) of its multiplicity to the
 * k-th dead slot (ascending slot order) and keeps the rest.  Returns the
 * number of recycled slots. */
typedef struct { uint64_t xi; uint32_t slot; } ranked_slot;

static int cmp_ranked_slot(const void *pa, const void *pb)
{
    const ranked_slot *a = (const ranked_slot *)pa, *b = (const ranked_slot *)pb;
    if (a->xi != b->xi) return a->xi > b->xi ? -1 : 1;   /* larger multiplicity first */
    if (a->slot != b->slot) return a->slot < b->slot ? -1 : 1;
    return 0;
}

static int cmp_u32(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* The recycling procedure over one range of slots (a cell, or the whole
 * domain).  x, z (nullable): positions, copied from the donor with its other
 * properties (location is one of the particle attributes of Sect. 5.1). */
static uint32_t recycle_range(uint32_t n_slots, uint64_t *xi, double *r, double *rd3,
                              double *kappa, double *x, double *z)
{
    uint32_t n = n_slots ? n_slots : 1u;
    uint32_t *dead = (uint32_t *)malloc(sizeof(uint32_t) * n);
    uint32_t *donor = (uint32_t *)malloc(sizeof(uint32_t) * n);
    ranked_slot *live = (ranked_slot *)malloc(sizeof(ranked_slot) * n);
    uint32_t z_dead = 0, L = 0;
    for (uint32_t s = 0; s < n_slots; ++s) {
        if (xi[s] == 0) {
            dead[z_dead++] = s;
        } else {
            live[L].xi = xi[s];
            live[L].slot = s;
            ++L;
        }
    }
    uint32_t nd = 0;
    if (z_dead > 0 && L > 0) {
        qsort(live, L, sizeof(ranked_slot), cmp_ranked_slot);
        uint32_t take = z_dead < L ? z_dead : L;
        for (uint32_t i = 0; i < take; ++i)
            if (live[i].xi >= 2u) donor[nd++] = live[i].slot;
        qsort(donor, nd, sizeof(uint32_t), cmp_u32);
        for (uint32_t i = 0; i < nd; ++i) {
            uint32_t d = donor[i], t = dead[i];
            uint64_t half = xi[d] / 2u;
            xi[t] = half;
            r[t] = r[d];
            if (rd3) {
                rd3[t] = rd3[d];
                kappa[t] = kappa[d];
            }
            if (x) {
                x[t] = x[d];
                z[t] = z[d];
            }
            xi[d] = xi[d] - half;
        }
    }
    free(dead);
    free(donor);
    free(live);
    return nd;
}

uint32_t oracle_recycle_cell_dry(uint32_t n_slots, uint64_t *xi, double *r, double *rd3,
                                 double *kappa)
{
    return recycle_range(n_slots, xi, r, rd3, kappa, NULL, NULL);
}

/* Recycling over the whole domain (the same procedure, with no restriction to
 * a cell): dead and live slots are taken over all n storage slots, the donors
 * are the min(z, L) live slots of the domain ranked first by multiplicity
 * (largest first, ties to the lower storage slot), and each recycled slot takes
 * all of its donor's properties: radius, dry attributes, and its location (the
 * positions x, z when given).  The caller re-sorts the storage by the cells of
 * the new locations.  Returns the number of recycled slots. */
uint32_t oracle_recycle_domain(uint32_t n, uint64_t *xi, double *r, double *rd3, double *kappa,
                               double *x, double *z)
{
    return recycle_range(n, xi, r, rd3, kappa, x, z);
}

uint32_t oracle_recycle_cell(uint32_t n_slots, uint64_t *xi, double *r)
{
    return oracle_recycle_cell_dry(n_slots, xi, r, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Random grouping into non-overlapping pairs                                */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key; uint32_t slot; } keyed_slot;

static int cmp_keyed_slot(const void *pa, const void *pb)
{
    const keyed_slot *a = (const keyed_slot *)pa, *b = (const keyed_slot *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->slot != b->slot) return a->slot < b->slot ? -1 : 1;
    return 0;
}

/* Order of the live slots (xi > 0) of one cell for step t: ascending by
 * (shuffle key, slot).  Returns the number n of live slots; order[0..n). */
uint32_t oracle_cell_order(uint32_t n_slots, const uint64_t *xi, uint64_t seed,
                           uint32_t cell, uint32_t step, uint32_t *order)
{
    keyed_slot *buf = (keyed_slot *)malloc(sizeof(keyed_slot) * (n_slots ? n_slots : 1));
    uint32_t n = 0;
    for (uint32_t s = 0; s < n_slots; ++s) {
        if (xi[s] == 0) continue;
        buf[n].key = oracle_shuffle_key(seed, cell, step, s);
        buf[n].slot = s;
        ++n;
    }
    qsort(buf, n, sizeof(keyed_slot), cmp_keyed_slot);
    for (uint32_t i = 0; i < n; ++i) order[i] = buf[i].slot;
    free(buf);
    return n;
}

/* ------------------------------------------------------------------------ */
/* One coalescence step                                                      */
/* ------------------------------------------------------------------------ */

/* One step over cells [0, n_cells) stored slot-contiguously: cell c owns
 * slots [offsets[c], offsets[c+1]).  The RNG cell index of cell c is
 * cell_index_base + c.  stats[0] += pair tests, stats[1] += collisions.
 * rd3 and kappa (both NULL, or both per slot) are the optional dry attributes. */
int oracle_step_dry(uint32_t n_cells, const uint64_t *offsets, const double *dV,
                    uint64_t *xi, double *r, double dt, int kernel, const double *params,
                    uint64_t seed, uint32_t step, uint32_t cell_index_base, uint64_t *stats,
                    uint32_t rules, double *rd3, double *kappa)
{
    uint32_t max_slots = 0;
    for (uint32_t c = 0; c < n_cells; ++c) {
        uint64_t cnt = offsets[c + 1] - offsets[c];
        if (cnt > max_slots) max_slots = (uint32_t)cnt;
    }
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (max_slots ? max_slots : 1));
    for (uint32_t c = 0; c < n_cells; ++c) {
        uint64_t base = offsets[c];
        uint32_t n_slots = (uint32_t)(offsets[c + 1] - base);
        uint32_t cell = cell_index_base + c;
        if (rules & ORACLE_RULE_RECYCLE)
            oracle_recycle_cell_dry(n_slots, xi + base, r + base, rd3 ? rd3 + base : NULL,
                                    kappa ? kappa + base : NULL);
        uint32_t n = oracle_cell_order(n_slots, xi + base, seed, cell, step, order);
        if (n < 2) continue;
        double scale = oracle_upscale(n);
        for (uint32_t m = 0; m < n / 2u; ++m) {
            uint64_t a = base + order[2u * m];
            uint64_t b = base + order[2u * m + 1u];
            uint64_t j = xi[a] >= xi[b] ? a : b;   /* tie: first member is j */
            uint64_t k = j == a ? b : a;
            double K = oracle_kernel(kernel, params, r[a], r[b]);
            double p = oracle_probability(xi[j], K, dt, dV[c], scale);
            double u = oracle_pair_uniform(seed, cell, step, m);
            uint64_t g;
            int both_merged = 0;   /* the equal split: j takes the merged droplets too */
            if (rules & ORACLE_RULE_FIDELITY) {
                g = oracle_gamma_fidelity(p, u);
            } else {
                g = oracle_gamma(p, u, xi[j], xi[k]);
                both_merged = g > 0 && xi[j] <= g * xi[k];
            }
            if (g > 0) {
                stats[1] += 1;
                if (rd3) {
                    double rd3_new, kappa_new;
                    oracle_dry_merge(g, rd3[j], kappa[j], rd3[k], kappa[k], &rd3_new, &kappa_new);
                    rd3[k] = rd3_new;
                    kappa[k] = kappa_new;
                    if (both_merged) {
                        rd3[j] = rd3_new;
                        kappa[j] = kappa_new;
                    }
                }
            }
            if (rules & ORACLE_RULE_FIDELITY)
                oracle_collide_pair_fidelity(g, &xi[j], &r[j], &xi[k], &r[k]);
            else
                oracle_collide_pair(g, &xi[j], &r[j], &xi[k], &r[k]);
        }
        stats[0] += n / 2u;
    }
    free(order);
    return 0;
}

int oracle_step_rules(uint32_t n_cells, const uint64_t *offsets, const double *dV,
                      uint64_t *xi, double *r, double dt, int kernel, const double *params,
                      uint64_t seed, uint32_t step, uint32_t cell_index_base, uint64_t *stats,
                      uint32_t rules)
{
    return oracle_step_dry(n_cells, offsets, dV, xi, r, dt, kernel, params, seed, step,
                           cell_index_base, stats, rules, NULL, NULL);
}

/* Dry radii from r_d^3 (correctly rounded cube roots), for the dry moments. */
void oracle_dry_radii(uint64_t n, const double *rd3, double *rd)
{
    for (uint64_t i = 0; i < n; ++i) rd[i] = oracle_cbrt_rn(rd3[i]);
}

int oracle_step(uint32_t n_cells, const uint64_t *offsets, const double *dV,
                uint64_t *xi, double *r, double dt, int kernel, const double *params,
                uint64_t seed, uint32_t step, uint32_t cell_index_base, uint64_t *stats)
{
    return oracle_step_rules(n_cells, offsets, dV, xi, r, dt, kernel, params, seed, step,
                             cell_index_base, stats, 0u);
}

/* Stable sort of super-droplets by cell (ties in input order).  Writes the
 * slot offsets (n_cells + 1) and id[slot] = input index.  Returns -1 if a
 * cell index is out of range. */
int oracle_sort_by_cell(uint64_t n_sd, const uint32_t *cell, uint32_t n_cells,
                        uint64_t *offsets, uint64_t *id)
{
    for (uint64_t i = 0; i < n_sd; ++i)
        if (cell[i] >= n_cells) return -1;
    uint64_t *fill = (uint64_t *)calloc((size_t)n_cells + 1u, sizeof(uint64_t));
    memset(offsets, 0, sizeof(uint64_t) * ((size_t)n_cells + 1u));
    for (uint64_t i = 0; i < n_sd; ++i) offsets[cell[i] + 1u] += 1u;
    for (uint32_t c = 0; c < n_cells; ++c) offsets[c + 1u] += offsets[c];
    for (uint64_t i = 0; i < n_sd; ++i) {
        uint32_t c = cell[i];
        id[offsets[c] + fill[c]] = i;
        fill[c] += 1u;
    }
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Gridded diagnostics (the particle-based scheme's diag_sd_conc and        */
/* diag_wet_mom of Sect. 5.2): per cell, the number of live super-droplets   */
/* and the k-th moment  M = (rho_d dV)^-1 sum_{r_i in [r_min, r_max]} N_i r_i^k */
/* over live super-droplets.                                                */
/* The sum is the plain one of the definition, taken term by term in         */
/* ascending slot order; r^k is the product of k factors r, left to right.  */
/* ------------------------------------------------------------------------ */
double oracle_moment_cell(uint32_t n_slots, const uint64_t *xi, const double *r, int k,
                          double r_min, double r_max, double rho_d, double dV)
{
    double sum = 0.0;
    for (uint32_t s = 0; s < n_slots; ++s) {
        if (xi[s] == 0 || !(r[s] >= r_min && r[s] <= r_max)) continue;
        double rk = 1.0;
        for (int i = 0; i < k; ++i) rk = rk * r[s];
        sum = sum + (double)xi[s] * rk;
    }
    return sum / (rho_d * dV);
}

void oracle_moments(uint32_t n_cells, const uint64_t *offsets, const double *dV,
                    const uint64_t *xi, const double *r, int k, double r_min, double r_max,
                    const double *rho_d, double *out)
{
    for (uint32_t c = 0; c < n_cells; ++c) {
        uint64_t b = offsets[c];
        out[c] = oracle_moment_cell((uint32_t)(offsets[c + 1] - b), xi + b, r + b, k, r_min,
                                    r_max, rho_d ? rho_d[c] : 1.0, dV[c]);
    }
}

void oracle_sd_conc(uint32_t n_cells, const uint64_t *offsets, const uint64_t *xi, uint32_t *out)
{
    for (uint32_t c = 0; c < n_cells; ++c) {
        uint32_t n = 0;
        for (uint64_t s = offsets[c]; s < offsets[c + 1]; ++s) n += xi[s] != 0;
        out[c] = n;
    }
}

/* Largest collision probability over the pairs one step would test (the
 * quantity an adaptive sub-step would be chosen from); the state is not
 * changed.  cell_max (optional) receives the largest value of each cell, 0 for
 * a cell with fewer than two live super-droplets. */
double oracle_max_probability(uint32_t n_cells, const uint64_t *offsets, const double *dV,
                              const uint64_t *xi, const double *r, double dt, int kernel,
                              const double *params, uint64_t seed, uint32_t step,
                              uint32_t cell_index_base, double *cell_max)
{
    double pmax = 0.0;
    uint32_t max_slots = 0;
    for (uint32_t c = 0; c < n_cells; ++c) {
        uint64_t cnt = offsets[c + 1] - offsets[c];
        if (cnt > max_slots) max_slots = (uint32_t)cnt;
    }
    uint32_t *order = (uint32_t *)malloc(sizeof(uint32_t) * (max_slots ? max_slots : 1));
    for (uint32_t c = 0; c < n_cells; ++c) {
        uint64_t base = offsets[c];
        uint32_t n = oracle_cell_order((uint32_t)(offsets[c + 1] - base), xi + base, seed,
                                       cell_index_base + c, step, order);
        double cmax = 0.0;
        if (n >= 2) {
            double scale = oracle_upscale(n);
            for (uint32_t m = 0; m < n / 2u; ++m) {
                uint64_t a = base + order[2u * m], b = base + order[2u * m + 1u];
                uint64_t xj = xi[a] >= xi[b] ? xi[a] : xi[b];
                double K = oracle_kernel(kernel, params, r[a], r[b]);
                double p = oracle_probability(xj, K, dt, dV[c], scale);
                if (p > cmax) cmax = p;
            }
        }
        if (cell_max) cell_max[c] = cmax;
        if (cmax > pmax) pmax = cmax;
    }
    free(order);
    return pmax;
}

/* ------------------------------------------------------------------------ */
/* Transport (Sect. 5.1: advection and sedimentation of the particles)       */
/* ------------------------------------------------------------------------ */
/* A 2D domain of nx x nz cells of size dx x dz, periodic in x, cell index    */
/* c = i + nx k with i = floor(x / dx), k = floor(z / dz) (clamped to the     */
/* grid).  Courant numbers on an Arakawa-C grid: cx[k nx + i] on the left     */
/* edge of cell (i, k) (edge nx of a row is edge 0), cz[k nx + i] on the      */
/* bottom edge of cell (i, k), k = 0 .. nz.                                   */
static uint32_t oracle_column(double x, double dx, uint32_t nx)
{
    double f = floor(x / dx);
    if (f < 0.0) return 0u;
    if (f >= (double)nx) return nx - 1u;
    return (uint32_t)f;
}

/* Backward-Euler advection in one dimension with the linear interpolation of
 * the Courant number between the edges of the particle's cell at time level
 * n, solved analytically: x' = (x + d (C_l - i dC)) / (1 - dC), dC = C_r - C_l. */
double oracle_advect_1d(double x, double d, uint32_t i, double c_l, double c_r)
{
    double dC = c_r - c_l;
    double num = x + d * (c_l - (double)i * dC);
    return num / (1.0 - dC);
}

/* Move every super-droplet (storage order): advection by the Courant fields
 * (either may be NULL for no flow in that direction), then, if sediment is set,
 * the fall by v_t(r) dt (explicit Euler).  x wraps periodically (a position
 * that rounds to the domain width becomes 0).  A super-droplet whose z leaves
 * [0, nz dz) gets multiplicity 0 and z clamped to 0 (below) or to the bottom
 * edge of the top row (above).  cell_out receives the new cell index. */
void oracle_transport(uint64_t n, uint32_t nx, uint32_t nz, double dx, double dz,
                      const double *cx, const double *cz, double dt, int sediment,
                      const double *params, double *x, double *z, uint64_t *xi,
                      const double *r, uint32_t *cell_out)
{
    double Lx = (double)nx * dx;
    double Lz = (double)nz * dz;
    for (uint64_t s = 0; s < n; ++s) {
        uint32_t i = oracle_column(x[s], dx, nx);
        uint32_t k = oracle_column(z[s], dz, nz);
        double xn = x[s], zn = z[s];
        if (cx) {
            double cl = cx[(uint64_t)k * nx + i];
            double cr = cx[(uint64_t)k * nx + (i + 1u == nx ? 0u : i + 1u)];
            xn = oracle_advect_1d(x[s], dx, i, cl, cr);
        }
        if (cz) {
            double cb = cz[(uint64_t)k * nx + i];
            double ct = cz[(uint64_t)(k + 1u) * nx + i];
            zn = oracle_advect_1d(z[s], dz, k, cb, ct);
        }
        if (sediment) zn = zn - oracle_terminal_velocity(params, r[s]) * dt;
        if (xn < 0.0) {
            xn = xn + Lx;
            if (xn >= Lx) xn = 0.0;
        } else if (xn >= Lx) {
            xn = xn - Lx;
        }
        if (zn < 0.0) {
            xi[s] = 0;
            zn = 0.0;
        } else if (zn >= Lz) {
            xi[s] = 0;
            zn = (double)(nz - 1u) * dz;
        }
        x[s] = xn;
        z[s] = zn;
        cell_out[s] = oracle_column(xn, dx, nx) + nx * oracle_column(zn, dz, nz);
    }
}

/* Stable counting sort of the storage slots by cell: order[j] = the old slot
 * that moves to new slot j; offsets (n_cells + 1) of the new layout. */
void oracle_resort(uint64_t n, const uint32_t *cell, uint32_t n_cells, uint64_t *offsets,
                   uint64_t *order)
{
    uint64_t *fill = (uint64_t *)calloc((size_t)n_cells + 1u, sizeof(uint64_t));
    memset(offsets, 0, sizeof(uint64_t) * ((size_t)n_cells + 1u));
    for (uint64_t s = 0; s < n; ++s) offsets[cell[s] + 1u] += 1u;
    for (uint32_t c = 0; c < n_cells; ++c) offsets[c + 1u] += offsets[c];
    for (uint64_t s = 0; s < n; ++s) {
        uint32_t c = cell[s];
        order[offsets[c] + fill[c]] = s;
        fill[c] += 1u;
    }
    free(fill);
}
