// transport.hip -- particle transport between cells (Sect. 5.1: advection by
// the Eulerian Courant field with the backward-Euler scheme and its analytic
// solution on an Arakawa-C grid, periodic in x; sedimentation by explicit
// Euler; particles leaving the domain flagged with zero multiplicity),
// followed by the stable re-sort of the storage by cell.
#include "context.hpp"

#include <cmath>
#include <cstring>
#include <vector>

using namespace sdm;

#pragma clang fp contract(off)

namespace {

constexpr unsigned int kErrCourant = 1u;
constexpr unsigned int kErrPosition = 2u;

// floor(v / d) clamped to [0, n - 1]
__device__ __forceinline__ uint32_t column_of(double v, double d, uint32_t n)
{
    const double f = floor(v / d);
    if (f < 0.0) return 0u;
    if (f >= static_cast<double>(n)) return n - 1u;
    return static_cast<uint32_t>(f);
}

// x' = (x + d (C_l - i dC)) / (1 - dC), dC = C_r - C_l: backward Euler with the
// Courant number interpolated linearly between the edges of the cell of time level n.
__device__ __forceinline__ double advect_1d(double x, double d, uint32_t i, double c_l, double c_r)
{
    const double dC = c_r - c_l;
    const double num = x + d * (c_l - static_cast<double>(i) * dC);
    return num / (1.0 - dC);
}

__global__ void k_validate_courant(uint32_t nx, uint32_t nz, const double* cx, const double* cz,
                                   unsigned int* err)
{
    const uint64_t n = static_cast<uint64_t>(nx) * nz;
    for (uint64_t c = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; c < n;
         c += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t i = static_cast<uint32_t>(c % nx), k = static_cast<uint32_t>(c / nx);
        bool bad = false;
        if (cx) {
            const double l = cx[static_cast<uint64_t>(k) * nx + i];
            const double r = cx[static_cast<uint64_t>(k) * nx + (i + 1u == nx ? 0u : i + 1u)];
            bad |= !isfinite(l) || !isfinite(r) || !(1.0 - (r - l) > 0.0);
        }
        if (cz) {
            const double b = cz[static_cast<uint64_t>(k) * nx + i];
            const double t = cz[static_cast<uint64_t>(k + 1u) * nx + i];
            bad |= !isfinite(b) || !isfinite(t) || !(1.0 - (t - b) > 0.0);
        }
        if (bad) atomicOr(err, kErrCourant);
    }
}

// Positions from input order to storage order, checked to lie in the domain.
__global__ void k_positions_in(uint64_t n, const uint32_t* id, const double* x_in,
                               const double* z_in, double* x, double* z, double Lx, double Lz,
                               unsigned int* err)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const double xv = x_in[id[s]], zv = z_in[id[s]];
        if (!(xv >= 0.0 && xv < Lx && zv >= 0.0 && zv < Lz)) atomicOr(err, kErrPosition);
        x[s] = xv;
        z[s] = zv;
    }
}

__global__ void k_cells_of(uint64_t n, const double* x, const double* z, uint32_t nx, uint32_t nz,
                           double dx, double dz, uint32_t* cell)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        cell[s] = column_of(x[s], dx, nx) + nx * column_of(z[s], dz, nz);
}

// Slots are handled in tiles of kTileSlots consecutive slots, one workgroup of
// kTileThreads threads per tile (grid-stride over tiles), each thread taking
// kTileK slots of the tile (slot k * kTileThreads + thread), so that per-tile
// mover counts and in-tile prefixes need no per-slot prefix array and every
// thread has kTileK independent loads in flight.
constexpr uint32_t kTileThreads = 256;
constexpr uint32_t kTileK = 4;
constexpr uint32_t kTileSlots = kTileThreads * kTileK;
constexpr uint32_t kTileWaves = kTileThreads / 64u;

// One workgroup per tile up to 2^20 tiles (grid-stride beyond): independent
// workgroups overlap their load, scan and store phases better than a few
// thousand workgroups walking many tiles each (the transport step of 134 M
// particles took 4.5 ms with 8192 workgroups, 4.1 ms with one per tile).
inline uint32_t tile_blocks(uint64_t ntiles)
{
    return static_cast<uint32_t>(ntiles < (1u << 20) ? ntiles : (1u << 20));
}
constexpr uint32_t kMovedBit = 0x80000000u;   // in the cell word: the particle changed cell

// Exclusive prefix of flag[k] over the tile in slot order, and in *total its sum.
// Every thread of the workgroup must call it.
__device__ __forceinline__ void tile_prefix(const bool (&flag)[kTileK], uint32_t (&pre)[kTileK],
                                            uint32_t* s_w, uint32_t* total)
{
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    const unsigned long long lanes_lt = (1ull << lane) - 1ull;
    uint32_t in_wave[kTileK];
#pragma unroll
    for (uint32_t k = 0; k < kTileK; ++k) {
        const unsigned long long b = __ballot(flag[k]);
        in_wave[k] = static_cast<uint32_t>(__popcll(b & lanes_lt));
        if (lane == 0) s_w[k * kTileWaves + wv] = static_cast<uint32_t>(__popcll(b));
    }
    __syncthreads();
    uint32_t run = 0;
#pragma unroll
    for (uint32_t k = 0; k < kTileK; ++k) {
        uint32_t before = 0, sub = 0;
#pragma unroll
        for (uint32_t w = 0; w < kTileWaves; ++w) {
            const uint32_t v = s_w[k * kTileWaves + w];
            before += w < wv ? v : 0u;
            sub += v;
        }
        pre[k] = run + before + in_wave[k];
        run += sub;
    }
    __syncthreads();
    *total = run;
}

__device__ __forceinline__ uint64_t tile_slot(uint64_t t, uint32_t k)
{
    return t * kTileSlots + k * kTileThreads + threadIdx.x;
}

// The flow of one transport step.
struct Flow {
    uint32_t nx, nz;
    double dx, dz, dt, Lx, Lz;
    const double* cx;   // Courant numbers on the x edges (nz * nx), or null
    const double* cz;   // on the z edges ((nz + 1) * nx), or null
    int sediment;
    KernelParams kp;
};

// The Courant numbers a particle's advection reads: those of the left and
// right x edges and of the bottom and top z edges of its time-level-n cell
// (column i, row k).  Requested apart from their use, so that a thread can
// have those of all its particles in flight together.
struct EdgeCourant {
    uint32_t i, k;
    double l, rr, b, tp;
};
__device__ __forceinline__ EdgeCourant load_courant(const Flow& f, double x0, double z0)
{
    EdgeCourant e;
    e.i = column_of(x0, f.dx, f.nx);
    e.k = column_of(z0, f.dz, f.nz);
    e.l = e.rr = e.b = e.tp = 0.0;
    if (f.cx) {
        e.l = f.cx[static_cast<uint64_t>(e.k) * f.nx + e.i];
        e.rr = f.cx[static_cast<uint64_t>(e.k) * f.nx + (e.i + 1u == f.nx ? 0u : e.i + 1u)];
    }
    if (f.cz) {
        e.b = f.cz[static_cast<uint64_t>(e.k) * f.nx + e.i];
        e.tp = f.cz[static_cast<uint64_t>(e.k + 1u) * f.nx + e.i];
    }
    return e;
}

// New position of the particle at (x0, z0) with radius r: advection from the
// Courant numbers e of its time-level-n cell, then the fall, the periodic wrap
// in x, and a clamp into the boundary row for a particle that left through the
// bottom or the top (*left).  *cell_old is that time-level-n cell.
__device__ __forceinline__ void move_particle(const Flow& f, double x0, double z0, double r,
                                              const EdgeCourant& e, double& xn, double& zn,
                                              bool& left, uint32_t& cell_old)
{
    xn = x0;
    zn = z0;
    if (f.cx) xn = advect_1d(x0, f.dx, e.i, e.l, e.rr);
    if (f.cz) zn = advect_1d(z0, f.dz, e.k, e.b, e.tp);
    if (f.sediment) zn = zn - terminal_velocity(f.kp, r) * f.dt;
    if (xn < 0.0) {
        xn = xn + f.Lx;
        if (xn >= f.Lx) xn = 0.0;
    } else if (xn >= f.Lx) {
        xn = xn - f.Lx;
    }
    left = false;
    if (zn < 0.0) {
        left = true;
        zn = 0.0;
    } else if (zn >= f.Lz) {
        left = true;
        zn = static_cast<double>(f.nz - 1u) * f.dz;
    }
    cell_old = e.i + f.nx * e.k;
}

// One transport step of every super-droplet (storage order): leavers get xi = 0,
// cellm[s] the new cell, with kMovedBit set if it differs from the old one, and
// tcnt[t] the number of such movers in tile t.  The new positions are not stored
// here: the re-sort scatter computes them again as it writes every particle out.
__global__ __launch_bounds__(kTileThreads) void k_transport(
    uint64_t n, Flow f, const double* __restrict__ x, const double* __restrict__ z,
    uint64_t* __restrict__ xi, const double* __restrict__ r, uint32_t* __restrict__ cellm,
    uint32_t* __restrict__ tcnt)
{
    __shared__ uint32_t s_w[kTileK * kTileWaves];
    const uint64_t ntiles = (n + kTileSlots - 1) / kTileSlots;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        // branch-free loads (slots past the end read the last one and are
        // not used), so that all of them are in flight together
        double x0[kTileK], z0[kTileK], rv[kTileK];
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) {
            const uint64_t s = tile_slot(t, k);
            const uint64_t sc = s < n ? s : n - 1u;
            x0[k] = x[sc];
            z0[k] = z[sc];
            rv[k] = f.sediment ? r[sc] : 0.0;
        }
        EdgeCourant ec[kTileK];
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) ec[k] = load_courant(f, x0[k], z0[k]);
        bool moved[kTileK];
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) {
            const uint64_t s = tile_slot(t, k);
            moved[k] = false;
            if (s >= n) continue;
            double xn, zn;
            bool left;
            uint32_t c_old;
            move_particle(f, x0[k], z0[k], rv[k], ec[k], xn, zn, left, c_old);
            if (left) xi[s] = 0;
            const uint32_t c_new = column_of(xn, f.dx, f.nx) + f.nx * column_of(zn, f.dz, f.nz);
            moved[k] = c_new != c_old;
            cellm[s] = c_new | (moved[k] ? kMovedBit : 0u);
        }
        uint32_t pre[kTileK], tot = 0;
        tile_prefix(moved, pre, s_w, &tot);
        if (threadIdx.x == 0) tcnt[t] = tot;
    }
}

// The new positions in place (a step in which no particle changed cell).
__global__ void k_apply_positions(uint64_t n, Flow f, double* __restrict__ x,
                                  double* __restrict__ z, const double* __restrict__ r)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        double xn, zn;
        bool left;
        uint32_t c_old;
        const double xs = x[s], zs = z[s];
        move_particle(f, xs, zs, f.sediment ? r[s] : 0.0, load_courant(f, xs, zs), xn, zn, left,
                      c_old);
        x[s] = xn;
        z[s] = zn;
    }
}

// ---------------------------------------------------------------------------
// Re-sort after a transport step.  Only the particles that changed cell
// ("movers") are sorted; the others keep their relative order.  In the stable
// order by (new cell, old slot), cell c holds first the movers that come from
// lower cells (old slot below c's old range), then its stayers, then the movers
// from higher cells, each in old-slot order.  tpre is the exclusive prefix of
// the per-tile mover counts; the movers before slot s are tpre[tile] plus the
// movers before s in its tile.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTileThreads) void k_compact_movers(uint64_t n,
                                                                  const uint32_t* __restrict__ cellm,
                                                                  const uint32_t* __restrict__ tpre,
                                                                  uint32_t* __restrict__ mk,
                                                                  uint32_t* __restrict__ mv)
{
    __shared__ uint32_t s_w[kTileK * kTileWaves];
    const uint64_t ntiles = (n + kTileSlots - 1) / kTileSlots;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t base = tpre[t];
        uint32_t v[kTileK];
        bool moved[kTileK];
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) {
            const uint64_t s = tile_slot(t, k);
            v[k] = s < n ? cellm[s] : 0u;
            moved[k] = (v[k] & kMovedBit) != 0;
        }
        uint32_t pre[kTileK], tot = 0;
        tile_prefix(moved, pre, s_w, &tot);
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) {
            if (!moved[k]) continue;
            const uint32_t m = base + pre[k];
            mk[m] = v[k] & ~kMovedBit;
            mv[m] = static_cast<uint32_t>(tile_slot(t, k));
        }
    }
}

// first index in mv[0, m) (ascending) whose value is >= key
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ mv, uint32_t lo,
                                                    uint32_t hi, uint32_t key)
{
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (mv[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// New per-cell counts (old - outgoing + incoming), the incoming movers from lower
// cells, and mlo[c] = movers with an old slot below the cell's old range (the
// compacted movers are in old-slot order).  count has n_cells + 1 entries (last 0).
__global__ void k_new_counts(uint32_t n_cells, const uint32_t* __restrict__ old_off, uint32_t m_tot,
                             const uint32_t* __restrict__ inc_off,
                             const uint32_t* __restrict__ order, const uint32_t* __restrict__ mv,
                             uint32_t* __restrict__ count, uint32_t* __restrict__ in_low,
                             uint32_t* __restrict__ mlo)
{
    for (uint64_t c = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; c <= n_cells;
         c += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        if (c == n_cells) {
            count[c] = 0;
            continue;
        }
        const uint32_t ob = old_off[c], oe = old_off[c + 1];
        const uint32_t lo = lower_bound_u32(mv, 0, m_tot, ob);
        const uint32_t out = lower_bound_u32(mv, lo, m_tot, oe) - lo;
        mlo[c] = lo;
        const uint32_t ib = inc_off[c], ie = inc_off[c + 1];
        count[c] = (oe - ob) - out + (ie - ib);
        // incoming movers are in old-slot order: count those below the cell's old range
        uint32_t a = ib, b = ie;
        while (a < b) {
            const uint32_t mid = a + (b - a) / 2;
            if (mv[order[mid]] < ob) a = mid + 1;
            else b = mid;
        }
        in_low[c] = a - ib;
    }
}

// inv[order[q]] = q: sorted position of every compacted mover
__global__ void k_invert_order(uint32_t m_tot, const uint32_t* __restrict__ order,
                               uint32_t* __restrict__ inv)
{
    for (uint64_t q = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; q < m_tot;
         q += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        inv[order[q]] = static_cast<uint32_t>(q);
}

// Every particle to its new slot, reading the old storage in order, with its
// new position.  A stayer goes after the cell's incoming movers from lower
// cells, at its rank among the cell's stayers; a mover (compacted index e,
// sorted position inv[e]) to its rank among the new cell's incoming movers,
// after the stayers if it comes from a higher cell.
__global__ __launch_bounds__(kTileThreads) void k_scatter_resort(
    uint64_t n, Flow f, const uint32_t* __restrict__ cellm, const uint32_t* __restrict__ tpre,
    const uint32_t* __restrict__ old_off, const uint32_t* __restrict__ new_off,
    const uint32_t* __restrict__ in_low, const uint32_t* __restrict__ mlo,
    const uint32_t* __restrict__ inv, const uint32_t* __restrict__ inc_off,
    const uint32_t* __restrict__ count, const uint64_t* __restrict__ xi,
    const double* __restrict__ r, const uint32_t* __restrict__ id, const double* __restrict__ x,
    const double* __restrict__ z, uint64_t* __restrict__ xi_o, double* __restrict__ r_o,
    uint32_t* __restrict__ id_o, double* __restrict__ x_o, double* __restrict__ z_o,
    const double* __restrict__ rd3, const double* __restrict__ kappa, double* __restrict__ rd3_o,
    double* __restrict__ kappa_o)
{
    __shared__ uint32_t s_w[kTileK * kTileWaves];
    const uint64_t ntiles = (n + kTileSlots - 1) / kTileSlots;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t base = tpre[t];
        // the slots' own loads first, all independent
        uint32_t v[kTileK], iv[kTileK];
        uint64_t xv[kTileK];
        double rv[kTileK], xs[kTileK], zs[kTileK];
        bool moved[kTileK];
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) {
            // branch-free (slots past the end read the last one; they are not
            // movers and are not written)
            const uint64_t s = tile_slot(t, k);
            const uint64_t sc = s < n ? s : n - 1u;
            v[k] = cellm[sc];
            xv[k] = xi[sc];
            rv[k] = r[sc];
            xs[k] = x[sc];
            zs[k] = z[sc];
            iv[k] = id[sc];
            moved[k] = s < n && (v[k] & kMovedBit) != 0;
        }
        uint32_t pre[kTileK], tot = 0;
        tile_prefix(moved, pre, s_w, &tot);
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) {
            const uint64_t s = tile_slot(t, k);
            if (s >= n) continue;
            const uint32_t mp = base + pre[k];   // movers before s
            const uint32_t c = v[k] & ~kMovedBit;
            uint64_t j;
            if (!moved[k]) {
                j = static_cast<uint64_t>(new_off[c]) + in_low[c] +
                    (static_cast<uint32_t>(s) - old_off[c]) - (mp - mlo[c]);
            } else {
                const uint32_t ib = inc_off[c];
                const uint32_t rank = inv[mp] - ib;
                const uint32_t stayers = count[c] - (inc_off[c + 1] - ib);
                j = static_cast<uint64_t>(new_off[c]) + rank + (rank >= in_low[c] ? stayers : 0u);
            }
            double xn, zn;
            bool left;
            uint32_t c_old;
            move_particle(f, xs[k], zs[k], rv[k], load_courant(f, xs[k], zs[k]), xn, zn, left, c_old);
            xi_o[j] = xv[k];
            r_o[j] = rv[k];
            id_o[j] = iv[k];
            x_o[j] = xn;
            z_o[j] = zn;
            if (rd3) {
                rd3_o[j] = rd3[s];
                kappa_o[j] = kappa[s];
            }
        }
    }
}

__global__ void k_gather_sd(uint64_t n, const uint32_t* __restrict__ order,
                            const uint64_t* __restrict__ xi, const double* __restrict__ r,
                            const uint32_t* __restrict__ id, const double* __restrict__ x,
                            const double* __restrict__ z, uint64_t* __restrict__ xi_o,
                            double* __restrict__ r_o, uint32_t* __restrict__ id_o,
                            double* __restrict__ x_o, double* __restrict__ z_o,
                            const double* __restrict__ rd3, const double* __restrict__ kappa,
                            double* __restrict__ rd3_o, double* __restrict__ kappa_o)
{
    for (uint64_t j = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; j < n;
         j += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t s = order[j];
        xi_o[j] = xi[s];
        r_o[j] = r[s];
        id_o[j] = id[s];
        x_o[j] = x[s];
        z_o[j] = z[s];
        if (rd3) {
            rd3_o[j] = rd3[s];
            kappa_o[j] = kappa[s];
        }
    }
}

__global__ void k_positions_out(uint64_t n, const uint32_t* id, const double* x, const double* z,
                                double* x_out, double* z_out)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        if (x_out) x_out[id[s]] = x[s];
        if (z_out) z_out[id[s]] = z[s];
    }
}


// ---------------------------------------------------------------------------
// Recycling over the whole domain: the recycling procedure of Sect. 5.1.4 with
// no restriction to a cell (Sect. 5.1.5 sends the particles that leave the
// domain through the same procedure).  With z dead and L live slots over the
// whole storage and take = min(z, L), the donors are the `take` live slots
// ranked first by multiplicity (largest first, ties to the lower storage
// slot); those with xi >= 2 are split, and in ascending slot order the i-th
// split donor gives floor(xi / 2), its radius, its dry attributes and its
// position (location is one of the particle attributes of Sect. 5.1) to the
// i-th dead slot.  The threshold T, the take-th largest multiplicity, comes
// from a radix selection on xi (12 bits per pass from the top significant
// bit); the donors are the slots above T and the rem lowest-slot ones equal to
// T.  Exclusive scans number the donors and the dead slots in slot order.  A
// recycled slot whose donor lies in another cell has changed cell: the
// storage is re-sorted with the movers' re-sort of the transport step.
// ---------------------------------------------------------------------------
constexpr uint32_t kRdDead = 0, kRdLive = 1, kRdMax = 2, kRdDonors = 4, kRdHist = 16;

__global__ void k_rd_stats(uint64_t n, const uint64_t* __restrict__ xi, uint32_t* __restrict__ small)
{
    uint32_t dead = 0, live = 0;
    unsigned long long mx = 0;
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t v = xi[s];
        if (v == 0) {
            ++dead;
        } else {
            ++live;
            mx = v > mx ? v : mx;
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        dead += __shfl_xor(dead, d, 64);
        live += __shfl_xor(live, d, 64);
        const unsigned long long o = __shfl_xor(mx, d, 64);
        mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63u) == 0) {
        if (dead) atomicAdd(&small[kRdDead], dead);
        if (live) atomicAdd(&small[kRdLive], live);
        if (mx) atomicMax(reinterpret_cast<unsigned long long*>(small + kRdMax), mx);
    }
}

// Histogram of bits [pos_new, pos) of the live multiplicities whose bits from
// pos up equal `prefix` (all of them when pos is 64).
__global__ __launch_bounds__(256) void k_rd_hist(uint64_t n, const uint64_t* __restrict__ xi,
                                                 uint32_t pos, uint32_t pos_new, uint64_t prefix,
                                                 uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[1u << kRecycleDomainDigit];
    const uint32_t nb = 1u << (pos - pos_new);
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t v = xi[s];
        if (v != 0 && (pos >= 64 || (v >> pos) == prefix))
            atomicAdd(&h[static_cast<uint32_t>(v >> pos_new) & (nb - 1u)], 1u);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

__device__ __forceinline__ bool rd_donor(uint64_t v, uint64_t T, uint32_t eq_before, uint32_t rem)
{
    return v >= 2u && (v > T || (v == T && eq_before < rem));
}

__global__ void k_rd_eq(uint64_t n, const uint64_t* __restrict__ xi, uint64_t T,
                        uint32_t* __restrict__ eq)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        eq[s] = xi[s] == T ? 1u : 0u;
}

// eq: the slots equal to T before each slot (exclusive scan of k_rd_eq)
__global__ void k_rd_flags(uint64_t n, const uint64_t* __restrict__ xi, uint64_t T, uint32_t rem,
                           const uint32_t* __restrict__ eq, uint32_t* __restrict__ dflag,
                           uint32_t* __restrict__ tflag)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t v = xi[s];
        dflag[s] = rd_donor(v, T, eq[s], rem) ? 1u : 0u;
        tflag[s] = v == 0 ? 1u : 0u;
    }
}

// the number of donors: the exclusive prefix at the last slot plus its own flag
__global__ void k_rd_total(uint64_t n, const uint64_t* __restrict__ xi, uint64_t T, uint32_t rem,
                           const uint32_t* __restrict__ eq, const uint32_t* __restrict__ dpos,
                           uint32_t* __restrict__ small)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        small[kRdDonors] = dpos[n - 1] + (rd_donor(xi[n - 1], T, eq[n - 1], rem) ? 1u : 0u);
}

__global__ void k_rd_lists(uint64_t n, const uint64_t* __restrict__ xi, uint64_t T, uint32_t rem,
                           const uint32_t* __restrict__ eq, const uint32_t* __restrict__ dpos,
                           const uint32_t* __restrict__ tpos, uint32_t nd,
                           uint32_t* __restrict__ dlist, uint32_t* __restrict__ tlist)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t v = xi[s];
        if (rd_donor(v, T, eq[s], rem)) dlist[dpos[s]] = static_cast<uint32_t>(s);
        else if (v == 0 && tpos[s] < nd) tlist[tpos[s]] = static_cast<uint32_t>(s);
    }
}

// cell of every slot from its position (the cells the storage is sorted by)
__global__ void k_rd_cells(uint64_t n, uint32_t nx, uint32_t nz, double dx, double dz,
                           const double* __restrict__ x, const double* __restrict__ z,
                           uint32_t* __restrict__ cellm)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        cellm[s] = column_of(x[s], dx, nx) + nx * column_of(z[s], dz, nz);
}

// the i-th split donor to the i-th dead slot; a recycled slot in another cell
// than its donor is marked as a mover to the donor's cell
__global__ void k_rd_apply(uint32_t nd, const uint32_t* __restrict__ dlist,
                           const uint32_t* __restrict__ tlist, uint64_t* __restrict__ xi,
                           double* __restrict__ r, double* __restrict__ rd3,
                           double* __restrict__ kappa, double* __restrict__ px,
                           double* __restrict__ pz, uint32_t* __restrict__ cellm,
                           unsigned long long* __restrict__ recycled)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x) {
        const uint32_t d = dlist[i], t = tlist[i];
        const uint64_t v = xi[d];
        const uint64_t half = v >> 1;
        xi[t] = half;
        xi[d] = v - half;
        r[t] = r[d];
        if (rd3) {
            rd3[t] = rd3[d];
            kappa[t] = kappa[d];
        }
        if (px) {
            px[t] = px[d];
            pz[t] = pz[d];
            const uint32_t cd = cellm[d];
            cellm[t] = cd | (cd != cellm[t] ? kMovedBit : 0u);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(recycled, static_cast<unsigned long long>(nd));
}

// movers per tile (the recycled slots that changed cell)
__global__ __launch_bounds__(kTileThreads) void k_rd_tcnt(uint64_t n, const uint32_t* __restrict__ cellm,
                                                          uint32_t* __restrict__ tcnt)
{
    __shared__ uint32_t s_w[kTileK * kTileWaves];
    const uint64_t ntiles = (n + kTileSlots - 1) / kTileSlots;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        bool moved[kTileK];
#pragma unroll
        for (uint32_t k = 0; k < kTileK; ++k) {
            const uint64_t s = tile_slot(t, k);
            moved[k] = s < n && (cellm[s] & kMovedBit) != 0;
        }
        uint32_t pre[kTileK], tot = 0;
        tile_prefix(moved, pre, s_w, &tot);
        if (threadIdx.x == 0) tcnt[t] = tot;
    }
}

struct TransportLayout {
    double *x, *z, *x_alt, *z_alt, *r_alt;
    uint64_t* xi_alt;
    uint32_t *id_alt, *cell, *tcnt, *mk, *mv, *mlo;
    uint32_t *off_alt, *inc_off, *in_low, *count, *tile_sums;
    DevicePlanArrays plan;
    size_t bytes;
};

TransportLayout transport_layout(void* ws, size_t ws_bytes, uint64_t n, uint32_t nc)
{
    Carver cv(ws, ws_bytes);
    TransportLayout L{};
    L.x = cv.take<double>(n);
    L.z = cv.take<double>(n);
    L.x_alt = cv.take<double>(n);
    L.z_alt = cv.take<double>(n);
    L.xi_alt = cv.take<uint64_t>(n);
    L.r_alt = cv.take<double>(n);
    L.id_alt = cv.take<uint32_t>(n);
    L.cell = cv.take<uint32_t>(n);
    L.tcnt = cv.take<uint32_t>((n + kTileSlots - 1) / kTileSlots + 1);
    L.mk = cv.take<uint32_t>(n);
    L.mv = cv.take<uint32_t>(n);
    L.mlo = cv.take<uint32_t>(uint64_t(nc) + 1);
    L.off_alt = cv.take<uint32_t>(uint64_t(nc) + 1);
    L.inc_off = cv.take<uint32_t>(uint64_t(nc) + 1);
    L.in_low = cv.take<uint32_t>(nc);
    L.count = cv.take<uint32_t>(uint64_t(nc) + 1);
    const uint64_t longest = (n + 1) > (uint64_t(nc) + 1) ? (n + 1) : (uint64_t(nc) + 1);
    L.tile_sums = cv.take<uint32_t>((longest + kScanTile - 1) / kScanTile + 2);
    carve_device_plan(cv, nc, &L.plan);
    L.bytes = cv.used();
    return L;
}

sdm_status read_error(sdm_ctx* x, unsigned int* out)
{
    SDM_HIP(hipMemcpyAsync(out, x->err, sizeof(unsigned int), hipMemcpyDeviceToHost, x->stream));
    SDM_HIP(hipStreamSynchronize(x->stream));
    return SDM_OK;
}

sdm_status clear_error(sdm_ctx* x)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, x->stream,
                       reinterpret_cast<uint32_t*>(x->err), uint64_t(1), 0u);
    SDM_LAUNCHED();
    return SDM_OK;
}

void swap_state(sdm_ctx* x)
{
    TransportState& T = *x->transport;
    std::swap(x->xi, T.xi_alt);
    std::swap(x->r, T.r_alt);
    std::swap(x->id, T.id_alt);
    std::swap(T.x, T.x_alt);
    std::swap(T.z, T.z_alt);
    std::swap(x->rd3, x->rd3_alt);
    std::swap(x->kappa, x->kappa_alt);
}

sdm_status refresh_plan(sdm_ctx* x);

// Stable re-sort of the whole storage by T.cell, then a new launch plan.
sdm_status resort(sdm_ctx* x)
{
    TransportState& T = *x->transport;
    const uint64_t n = x->n_sd;
    const uint32_t* order = nullptr;
    SDM_TRY(radix_sort_by_cell(x->stream, n, T.cell, x->n_cells, x->sort, x->offsets, &order));
    if (n > 0) {
        hipLaunchKernelGGL(k_gather_sd, dim3(grid_for(n, 256, 8192)), dim3(256), 0, x->stream, n,
                           order, x->xi, x->r, x->id, T.x, T.z, T.xi_alt, T.r_alt, T.id_alt,
                           T.x_alt, T.z_alt, x->rd3, x->kappa, x->rd3_alt, x->kappa_alt);
        SDM_LAUNCHED();
        swap_state(x);
    }
    return refresh_plan(x);
}

// The same order after a transport step, sorting only the movers; the
// particles are written out with their new positions.
sdm_status resort_moved(sdm_ctx* x, const Flow& f)
{
    TransportState& T = *x->transport;
    const uint64_t n = x->n_sd;
    const uint32_t nc = x->n_cells;
    hipStream_t st = x->stream;
    const uint64_t ntiles = (n + kTileSlots - 1) / kTileSlots;
    const dim3 tile_grid(tile_blocks(ntiles));
    const dim3 tile_block(kTileThreads);
    // tile counts -> exclusive tile prefix; the entry past the last tile ends in the total
    SDM_TRY(scan_exclusive(st, T.tcnt, T.tcnt, ntiles + 1, T.tile_sums));
    uint32_t m_tot = 0;
    SDM_HIP(hipMemcpyAsync(&m_tot, T.tcnt + ntiles, sizeof(m_tot), hipMemcpyDeviceToHost, st));
    SDM_HIP(hipStreamSynchronize(st));
    if (m_tot == 0) {
        // nobody changed cell: storage, offsets and plan stay; positions move in place
        hipLaunchKernelGGL(k_apply_positions, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, n, f,
                           T.x, T.z, x->r);
        SDM_LAUNCHED();
        return SDM_OK;
    }
    hipLaunchKernelGGL(k_compact_movers, tile_grid, tile_block, 0, st, n, T.cell, T.tcnt,
                       T.mk, T.mv);
    SDM_LAUNCHED();
    const uint32_t* order = nullptr;
    SDM_TRY(radix_sort_by_cell(st, m_tot, T.mk, nc, x->sort, T.inc_off, &order));
    hipLaunchKernelGGL(k_new_counts, dim3(grid_for(uint64_t(nc) + 1, 256, 8192)), dim3(256), 0, st,
                       nc, x->offsets, m_tot, T.inc_off, order, T.mv, T.count, T.in_low, T.mlo);
    SDM_LAUNCHED();
    SDM_TRY(scan_exclusive(st, T.count, T.off_alt, uint64_t(nc) + 1, T.tile_sums));
    // the sort read its keys from mk: that array now takes the inverse order
    uint32_t* inv = T.mk;
    hipLaunchKernelGGL(k_invert_order, dim3(grid_for(m_tot, 256, 8192)), dim3(256), 0, st, m_tot,
                       order, inv);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_scatter_resort, tile_grid, tile_block, 0, st, n, f, T.cell, T.tcnt,
                       x->offsets, T.off_alt, T.in_low, T.mlo, inv, T.inc_off, T.count, x->xi,
                       x->r, x->id, T.x, T.z, T.xi_alt, T.r_alt, T.id_alt, T.x_alt, T.z_alt,
                       x->rd3, x->kappa, x->rd3_alt, x->kappa_alt);
    SDM_LAUNCHED();
    swap_state(x);
    std::swap(x->offsets, T.off_alt);
    return refresh_plan(x);
}

// Launch plan from the new offsets: on the device when no cell exceeds the
// wavefront tier (the usual case after transport), else on the host.
sdm_status refresh_plan(sdm_ctx* x)
{
    TransportState& T = *x->transport;
    const uint32_t nc = x->n_cells;
    hipStream_t st = x->stream;
    const uint32_t cap = x->shape.group_slots;
    if (nc > 0) {
        uint32_t n_groups = 0;
        bool usable = false, big = false;
        SDM_TRY(device_plan(st, nc, x->offsets, cap, T.plan, x->group_begin, x->group_end,
                            &n_groups, &usable, &big));
        if (usable) {
            Plan empty;
            SDM_TRY(upload_grid(st, empty, &x->grid));
            x->n_groups = n_groups;
            x->n_wave_cells = nc;
            x->sizes_stale = true;
            return SDM_OK;
        }
    }
    x->sizes_stale = true;   // the host plan downloads the offsets first
    return ctx_replan(x);
}

sdm_status check_attached(const sdm_ctx* x)
{
    if (!x) {
        set_error("context is NULL");
        return SDM_EINVAL;
    }
    if (!x->transport) {
        set_error("no transport attached (sdm_transport_attach)");
        return SDM_ESTATE;
    }
    return SDM_OK;
}

}  // namespace

extern "C" size_t sdm_transport_workspace_bytes(uint64_t n_sd, uint32_t n_cells)
{
    return transport_layout(nullptr, 0, n_sd, n_cells).bytes;
}

extern "C" sdm_status sdm_transport_attach(sdm_ctx* x, void* workspace, size_t ws_bytes,
                                           uint32_t nx, uint32_t nz, double dx, double dz,
                                           const double* x_in, const double* z_in)
{
    if (!x) {
        set_error("context is NULL");
        return SDM_EINVAL;
    }
    if (x->transport) {
        set_error("transport is already attached");
        return SDM_ESTATE;
    }
    if (nx == 0 || nz == 0 || static_cast<uint64_t>(nx) * nz != x->n_cells) {
        set_error("the grid (%u x %u) must have exactly n_cells = %u cells", nx, nz, x->n_cells);
        return SDM_EINVAL;
    }
    if (x->n_cells > ~kMovedBit) {
        set_error("transport supports at most 2^31 - 1 cells");
        return SDM_EINVAL;
    }
    if (!(dx > 0.0) || !(dz > 0.0) || !std::isfinite(dx) || !std::isfinite(dz)) {
        set_error("dx and dz must be finite and > 0");
        return SDM_EINVAL;
    }
    if (x->n_sd > 0 && (!x_in || !z_in)) {
        set_error("positions must be non-NULL");
        return SDM_EINVAL;
    }
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
        set_error("workspace must be non-NULL and 256-byte aligned");
        return SDM_EINVAL;
    }
    const TransportLayout L = transport_layout(workspace, ws_bytes, x->n_sd, x->n_cells);
    if (L.bytes > ws_bytes) {
        set_error("transport workspace has %zu bytes, %zu needed", ws_bytes, L.bytes);
        return SDM_ENOMEM;
    }
    const uint64_t n = x->n_sd;
    const double Lx = static_cast<double>(nx) * dx, Lz = static_cast<double>(nz) * dz;
    SDM_TRY(clear_error(x));
    if (n > 0) {
        hipLaunchKernelGGL(k_positions_in, dim3(grid_for(n, 256, 8192)), dim3(256), 0, x->stream,
                           n, x->id, x_in, z_in, L.x, L.z, Lx, Lz, x->err);
        SDM_LAUNCHED();
    }
    unsigned int err = 0;
    SDM_TRY(read_error(x, &err));
    if (err & kErrPosition) {
        set_error("positions must be finite and inside [0, nx dx) x [0, nz dz)");
        return SDM_EINVAL;
    }
    auto T = std::make_unique<TransportState>();
    T->nx = nx;
    T->nz = nz;
    T->dx = dx;
    T->dz = dz;
    T->x = L.x;
    T->z = L.z;
    T->x_alt = L.x_alt;
    T->z_alt = L.z_alt;
    T->xi_alt = L.xi_alt;
    T->r_alt = L.r_alt;
    T->id_alt = L.id_alt;
    T->cell = L.cell;
    T->tcnt = L.tcnt;
    T->mk = L.mk;
    T->mv = L.mv;
    T->mlo = L.mlo;
    T->off_alt = L.off_alt;
    T->inc_off = L.inc_off;
    T->in_low = L.in_low;
    T->count = L.count;
    T->tile_sums = L.tile_sums;
    T->plan = L.plan;
    x->transport = std::move(T);
    if (n > 0) {
        hipLaunchKernelGGL(k_cells_of, dim3(grid_for(n, 256, 8192)), dim3(256), 0, x->stream, n,
                           L.x, L.z, nx, nz, dx, dz, L.cell);
        SDM_LAUNCHED();
    }
    return resort(x);
}

extern "C" sdm_status sdm_transport_step(sdm_ctx* x, const double* cx, const double* cz, double dt,
                                         int sediment)
{
    SDM_TRY(check_attached(x));
    if (!(dt > 0.0) || !std::isfinite(dt)) {
        set_error("dt must be finite and > 0");
        return SDM_EINVAL;
    }
    TransportState& T = *x->transport;
    if (cx || cz) {
        SDM_TRY(clear_error(x));
        hipLaunchKernelGGL(k_validate_courant, dim3(grid_for(x->n_cells, 256, 4096)), dim3(256), 0,
                           x->stream, T.nx, T.nz, cx, cz, x->err);
        SDM_LAUNCHED();
        unsigned int err = 0;
        SDM_TRY(read_error(x, &err));
        if (err & kErrCourant) {
            set_error("Courant numbers must be finite with C_right - C_left < 1 in every cell");
            return SDM_EINVAL;
        }
    }
    const uint64_t n = x->n_sd;
    Flow f;
    f.nx = T.nx;
    f.nz = T.nz;
    f.dx = T.dx;
    f.dz = T.dz;
    f.dt = dt;
    f.Lx = static_cast<double>(T.nx) * T.dx;
    f.Lz = static_cast<double>(T.nz) * T.dz;
    f.cx = cx;
    f.cz = cz;
    f.sediment = sediment ? 1 : 0;
    f.kp = to_kp(x->params);
    if (n > 0) {
        const uint64_t ntiles = (n + kTileSlots - 1) / kTileSlots;
        hipLaunchKernelGGL(k_transport, dim3(tile_blocks(ntiles)),
                           dim3(kTileThreads), 0, x->stream, n, f, T.x, T.z, x->xi, x->r, T.cell,
                           T.tcnt);
        SDM_LAUNCHED();
    }
    return resort_moved(x, f);
}

extern "C" sdm_status sdm_transport_get_positions(sdm_ctx* x, double* x_out, double* z_out)
{
    SDM_TRY(check_attached(x));
    const uint64_t n = x->n_sd;
    if (n > 0 && (x_out || z_out)) {
        hipLaunchKernelGGL(k_positions_out, dim3(grid_for(n, 256, 8192)), dim3(256), 0, x->stream,
                           n, x->id, x->transport->x, x->transport->z, x_out, z_out);
        SDM_LAUNCHED();
    }
    SDM_HIP(hipStreamSynchronize(x->stream));
    return SDM_OK;
}

namespace sdm {

sdm_status recycle_domain(sdm_ctx* x)
{
    if (x->n_cells > 1 && !x->transport) {
        set_error("domain-wide recycling of several cells needs positions (sdm_transport_attach)");
        return SDM_ESTATE;
    }
    const uint64_t n = x->n_sd;
    if (n < 2) return SDM_OK;   // a dead and a live slot are needed
    if (n > 0xFFFFFFFFull) {
        set_error("domain-wide recycling takes fewer than 2^32 slots");
        return SDM_EINVAL;
    }
    hipStream_t st = x->stream;
    uint32_t* small = x->rd_small;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, small, uint64_t(kRdHist), 0u);
    SDM_LAUNCHED();
    const dim3 grid(grid_for(n, 256, 4096)), block(256);
    hipLaunchKernelGGL(k_rd_stats, grid, block, 0, st, n, x->xi, small);
    SDM_LAUNCHED();
    uint32_t head[4] = {0, 0, 0, 0};
    SDM_HIP(hipMemcpyAsync(head, small, sizeof(head), hipMemcpyDeviceToHost, st));
    SDM_HIP(hipStreamSynchronize(st));
    const uint64_t dead = head[kRdDead], live = head[kRdLive];
    uint64_t vmax = 0;
    std::memcpy(&vmax, head + kRdMax, sizeof(vmax));
    if (dead == 0 || live == 0) return SDM_OK;
    const uint64_t take = dead < live ? dead : live;

    // the take-th largest multiplicity T, and how many of the slots equal to T
    // (the lowest ones) are taken
    uint32_t pos = 64u - static_cast<uint32_t>(__builtin_clzll(vmax));
    uint64_t prefix = 0, remaining = take;
    std::vector<uint32_t> h(1u << kRecycleDomainDigit);
    uint32_t* hist = small + kRdHist;
    while (pos > 0) {
        const uint32_t pos_new = pos > kRecycleDomainDigit ? pos - kRecycleDomainDigit : 0u;
        const uint32_t nb = 1u << (pos - pos_new);
        hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(nb, 256, 64)), dim3(256), 0, st, hist,
                           uint64_t(nb), 0u);
        SDM_LAUNCHED();
        hipLaunchKernelGGL(k_rd_hist, dim3(grid_for(n, 256, 2048)), dim3(256), 0, st, n, x->xi, pos,
                           pos_new, prefix, hist);
        SDM_LAUNCHED();
        SDM_HIP(hipMemcpyAsync(h.data(), hist, nb * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        SDM_HIP(hipStreamSynchronize(st));
        uint32_t d = nb - 1u;
        while (h[d] < remaining) {
            remaining -= h[d];
            if (d == 0) {
                set_error("domain-wide recycling: the multiplicity histogram lost slots");
                return SDM_EDEVICE;
            }
            --d;
        }
        prefix = (prefix << (pos - pos_new)) | d;
        pos = pos_new;
    }
    const uint64_t T = prefix;
    const uint32_t rem = static_cast<uint32_t>(remaining);

    // number the donors and the dead slots in slot order (step scratch)
    uint32_t* eq = x->scr_cnt;
    uint32_t* dpos = reinterpret_cast<uint32_t*>(x->scr_kv);
    uint32_t* tpos = dpos + n;
    uint32_t* dlist = reinterpret_cast<uint32_t*>(x->scr_tmp);
    uint32_t* tlist = dlist + n;
    uint32_t* tiles = x->probe_order;
    hipLaunchKernelGGL(k_rd_eq, grid, block, 0, st, n, x->xi, T, eq);
    SDM_LAUNCHED();
    SDM_TRY(scan_exclusive(st, eq, eq, n, tiles));
    hipLaunchKernelGGL(k_rd_flags, grid, block, 0, st, n, x->xi, T, rem, eq, dpos, tpos);
    SDM_LAUNCHED();
    SDM_TRY(scan_exclusive(st, dpos, dpos, n, tiles));
    SDM_TRY(scan_exclusive(st, tpos, tpos, n, tiles));
    hipLaunchKernelGGL(k_rd_total, dim3(1), dim3(64), 0, st, n, x->xi, T, rem, eq, dpos, small);
    SDM_LAUNCHED();
    uint32_t nd = 0;
    SDM_HIP(hipMemcpyAsync(&nd, small + kRdDonors, sizeof(nd), hipMemcpyDeviceToHost, st));
    SDM_HIP(hipStreamSynchronize(st));
    if (nd == 0) return SDM_OK;
    if (nd > take) {
        set_error("domain-wide recycling: more donors than dead slots");
        return SDM_EDEVICE;
    }
    hipLaunchKernelGGL(k_rd_lists, grid, block, 0, st, n, x->xi, T, rem, eq, dpos, tpos, nd, dlist,
                       tlist);
    SDM_LAUNCHED();
    TransportState* T_ = x->transport.get();
    if (T_) {
        hipLaunchKernelGGL(k_rd_cells, grid, block, 0, st, n, T_->nx, T_->nz, T_->dx, T_->dz, T_->x,
                           T_->z, T_->cell);
        SDM_LAUNCHED();
    }
    hipLaunchKernelGGL(k_rd_apply, dim3(grid_for(nd, 256, 4096)), block, 0, st, nd, dlist, tlist,
                       x->xi, x->r, x->rd3, x->kappa, T_ ? T_->x : nullptr, T_ ? T_->z : nullptr,
                       T_ ? T_->cell : nullptr, x->stats + kRecycledStat);
    SDM_LAUNCHED();
    if (!T_ || x->n_cells < 2) return SDM_OK;
    // the recycled slots that joined their donor's cell move there
    const uint64_t ntiles = (n + kTileSlots - 1) / kTileSlots;
    hipLaunchKernelGGL(k_rd_tcnt, dim3(tile_blocks(ntiles)), dim3(kTileThreads), 0, st, n, T_->cell,
                       T_->tcnt);
    SDM_LAUNCHED();
    Flow still;   // positions stay where they are
    still.nx = T_->nx;
    still.nz = T_->nz;
    still.dx = T_->dx;
    still.dz = T_->dz;
    still.dt = 0.0;
    still.Lx = static_cast<double>(T_->nx) * T_->dx;
    still.Lz = static_cast<double>(T_->nz) * T_->dz;
    still.cx = nullptr;
    still.cz = nullptr;
    still.sediment = 0;
    still.kp = to_kp(x->params);
    return resort_moved(x, still);
}

}  // namespace sdm

extern "C" sdm_status sdm_recycle_domain(sdm_ctx* x)
{
    if (!x) {
        set_error("context is NULL");
        return SDM_EINVAL;
    }
    return recycle_domain(x);
}
