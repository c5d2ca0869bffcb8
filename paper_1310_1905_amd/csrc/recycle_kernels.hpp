// recycle_kernels.hpp -- recycling of zero-multiplicity super-droplets
// (Sect. 5.1.4: particles left with zero multiplicity take the attributes of
// the particles with the highest multiplicities, halving those), applied within
// each cell at the start of a step.
//
// Per cell, with z dead and L live slots and take = min(z, L): the donors are
// the `take` live slots ranked first by multiplicity (largest first, ties to
// the lower slot); those with xi >= 2 are split.  In ascending slot order the
// k-th split donor d gives its radius and floor(xi_d / 2) to the k-th dead slot
// and keeps xi_d - floor(xi_d / 2).
//
// One wavefront per cell.  The threshold T (the take-th largest multiplicity)
// is the largest v with #{xi >= v} >= take, always one of the multiplicities
// present: the search walks down the distinct values from the largest, which
// ends in a step or two when many slots share a multiplicity (as after merges of
// equal-multiplicity pairs), and after kRecycleDescent values falls back to
// setting bits from the top.  Counts and maxima of the first 256 slots of a cell
// come from registers (ballots), any further ones from memory.  The donors are
// then every slot above T plus the lowest-slot ones equal to T.
// Cells of up to 256 slots exchange through LDS: each split donor writes its
// half and its slot under its rank, then each dead slot of the same rank takes
// the half and lists the (dead, donor) pair; a second, thread-per-cell kernel
// copies the radii of the listed pairs, so that no wavefront waits on a
// dependent load per cell.  Larger cells list dead and donor slots in slot
// order in a per-cell scratch range and apply the list pairs last, so no slot
// is classified after it has been written.
#pragma once

#include "step_kernels.hpp"

namespace sdm {
namespace {

constexpr int kRecycleBlock = 256;
constexpr uint32_t kRecycleCellsPerBlock = kRecycleBlock / 64;
constexpr int kRecycleRegs = 4;   // slots per lane held in registers (256 per cell)
constexpr int kRecycleDescent = 4;   // distinct values tried before the bit search

__device__ __forceinline__ uint32_t wave_total(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(v, d, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Slots of [b, b+n) whose multiplicity is >= v (v >= 1): the first
// 64 * kRecycleRegs from the registers xr, the rest from memory.
__device__ __forceinline__ uint32_t count_at_least(const uint64_t* __restrict__ xi, uint32_t b,
                                                   uint32_t n, const uint64_t (&xr)[kRecycleRegs],
                                                   uint64_t v, uint32_t lane)
{
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < kRecycleRegs; ++k)
        c += static_cast<uint32_t>(__popcll(__ballot(xr[k] >= v)));
    if (n > 64u * kRecycleRegs) {
        uint32_t t = 0;
        for (uint32_t i = 64u * kRecycleRegs + lane; i < n; i += 64u) t += xi[b + i] >= v ? 1u : 0u;
        c += wave_total(t);
    }
    return c;
}

// Largest multiplicity below v in [b, b+n) (0 if none), registers then memory.
__device__ __forceinline__ uint64_t max_below(const uint64_t* __restrict__ xi, uint32_t b,
                                              uint32_t n, const uint64_t (&xr)[kRecycleRegs],
                                              uint64_t v, uint32_t lane)
{
    uint64_t m = 0;
#pragma unroll
    for (int k = 0; k < kRecycleRegs; ++k)
        if (xr[k] < v && xr[k] > m) m = xr[k];
    for (uint32_t i = 64u * kRecycleRegs + lane; i < n; i += 64u) {
        const uint64_t x = xi[b + i];
        if (x < v && x > m) m = x;
    }
    return wave_max_u64(m);
}

// The take-th largest multiplicity of [b, b+n) (1 <= take <= live slots):
// the largest v with #{xi >= v} >= take.
__device__ __forceinline__ uint64_t recycle_threshold(const uint64_t* __restrict__ xi, uint32_t b,
                                                      uint32_t n,
                                                      const uint64_t (&xr)[kRecycleRegs],
                                                      uint64_t xmax, uint32_t take, uint32_t lane)
{
    if (take == 1) return xmax;
    uint64_t T = xmax;
    uint32_t c = count_at_least(xi, b, n, xr, T, lane);
    for (int s = 0; s < kRecycleDescent && c < take; ++s) {
        T = max_below(xi, b, n, xr, T, lane);   // >= 1: fewer than take <= live are >= T
        c = count_at_least(xi, b, n, xr, T, lane);
    }
    if (c >= take) return T;
    // the answer is below T: bits from T's top bit down
    uint64_t v = 0;
    for (int bit = 63 - __clzll(static_cast<long long>(T)); bit >= 0; --bit) {
        const uint64_t cand = v | (1ull << bit);
        if (count_at_least(xi, b, n, xr, cand, lane) >= take) v = cand;
    }
    return v;
}

// list: uint32[n_sd] scratch, cell c uses [off[c], off[c+1]).
// pairs: uint32[n_cells], zero on entry; cells of up to 256 slots with recycled
// slots get their pair count, their pairs (dead | donor << 16, cell-local) in
// list, and their multiplicities; k_recycle_copy then copies the radii.
// stats (nullable): the recycled-slot counts go to word kRecycledStat of the
// kStatSlots counter slots (one per workgroup, spread so that the workgroups'
// atomics do not serialise on one address).
// rd3, kappa: optional dry attributes (nullable), copied with the radius.
__global__ __launch_bounds__(kRecycleBlock) void k_recycle(const uint32_t* __restrict__ off,
                                                           uint64_t* __restrict__ xi,
                                                           double* __restrict__ r,
                                                           uint32_t n_cells,
                                                           uint32_t* __restrict__ list,
                                                           uint32_t* __restrict__ pairs,
                                                           unsigned long long* stats,
                                                           double* __restrict__ rd3,
                                                           double* __restrict__ kappa)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lanes_lt = (1ull << lane) - 1ull;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kRecycleCellsPerBlock;
    // per-wavefront exchange area of the cells of up to 256 slots
    __shared__ uint64_t s_half[kRecycleCellsPerBlock][64 * kRecycleRegs];
    __shared__ uint32_t s_slot[kRecycleCellsPerBlock][64 * kRecycleRegs];
    uint64_t* xch_half = s_half[threadIdx.x / 64u];
    uint32_t* xch_slot = s_slot[threadIdx.x / 64u];
    uint32_t done = 0;
    for (uint64_t c = static_cast<uint64_t>(blockIdx.x) * kRecycleCellsPerBlock + threadIdx.x / 64u;
         c < n_cells; c += stride) {
        const uint32_t b = off[c], n = off[c + 1] - b;
        // the first 256 slots into registers (independent loads), then the counts of
        // dead and live slots and the largest multiplicity
        uint64_t xr[kRecycleRegs];
#pragma unroll
        for (int k = 0; k < kRecycleRegs; ++k) {
            const uint32_t i = lane + 64u * k;
            xr[k] = i < n ? xi[b + i] : 0u;
        }
        uint32_t z = 0, L = 0;
        uint64_t xmax = 0;
#pragma unroll
        for (int k = 0; k < kRecycleRegs; ++k) {
            const uint32_t i = lane + 64u * k;
            z += static_cast<uint32_t>(__popcll(__ballot(i < n && xr[k] == 0)));
            L += static_cast<uint32_t>(__popcll(__ballot(xr[k] != 0)));
            xmax = xr[k] > xmax ? xr[k] : xmax;
        }
        for (uint32_t base = 64u * kRecycleRegs; base < n; base += 64u) {
            const uint32_t i = base + lane;
            const uint64_t x = i < n ? xi[b + i] : 0u;
            z += static_cast<uint32_t>(__popcll(__ballot(i < n && x == 0)));
            L += static_cast<uint32_t>(__popcll(__ballot(x != 0)));
            xmax = x > xmax ? x : xmax;
        }
        if (z == 0 || L == 0) continue;   // uniform across the wavefront
        xmax = wave_max_u64(xmax);
        const uint32_t take = z < L ? z : L;
        const uint64_t T = recycle_threshold(xi, b, n, xr, xmax, take, lane);
        const uint32_t above = count_at_least(xi, b, n, xr, T + 1u, lane);
        const uint32_t need_eq = take - above;
        if (n <= 64u * kRecycleRegs) {
            // split donors: half and slot into the exchange area under their rank
            uint32_t eq_seen = 0, nd = 0;
#pragma unroll
            for (int k = 0; k < kRecycleRegs; ++k) {
                const uint32_t i = lane + 64u * k;
                const uint64_t x = xr[k];
                const uint64_t eq_mask = __ballot(x == T);   // T >= 1: no padding lane
                const uint32_t eq_rank = eq_seen + static_cast<uint32_t>(__popcll(eq_mask & lanes_lt));
                const bool donor = x >= 2u && (x > T || (x == T && eq_rank < need_eq));
                const uint64_t don_mask = __ballot(donor);
                if (donor) {
                    const uint32_t rank = nd + static_cast<uint32_t>(__popcll(don_mask & lanes_lt));
                    const uint64_t half = x >> 1;
                    xch_half[rank] = half;
                    xch_slot[rank] = i;
                    xi[b + i] = x - half;
                }
                eq_seen += static_cast<uint32_t>(__popcll(eq_mask));
                nd += static_cast<uint32_t>(__popcll(don_mask));
            }
            wave_sync();
            // dead slots (xi still 0 in the registers) take the donor of their rank
            uint32_t dead_seen = 0;
#pragma unroll
            for (int k = 0; k < kRecycleRegs; ++k) {
                const uint32_t i = lane + 64u * k;
                const bool dead = i < n && xr[k] == 0;
                const uint64_t dead_mask = __ballot(dead);
                const uint32_t rank = dead_seen + static_cast<uint32_t>(__popcll(dead_mask & lanes_lt));
                if (dead && rank < nd) {
                    xi[b + i] = xch_half[rank];
                    list[b + rank] = i | (xch_slot[rank] << 16);   // rank < nd <= n
                }
                dead_seen += static_cast<uint32_t>(__popcll(dead_mask));
            }
            if (lane == 0) pairs[c] = nd;
            wave_sync();   // the exchange area is reused by the wavefront's next cell
            done += nd;
            continue;
        }
        // dead slots to list[b, b+z), split donors to list[b+z, b+z+nd), slot order
        uint32_t dead_seen = 0, eq_seen = 0, don_seen = 0;
        for (uint32_t base = 0; base < n; base += 64u) {
            const uint32_t i = base + lane;
            const uint64_t x = i < n ? xi[b + i] : 0u;
            const bool dead = i < n && x == 0;
            const bool eq = x == T;   // T >= 1, so never a padding lane
            const uint64_t eq_mask = __ballot(eq);
            const uint32_t eq_rank = eq_seen + static_cast<uint32_t>(__popcll(eq_mask & lanes_lt));
            const bool donor = x >= 2u && (x > T || (eq && eq_rank < need_eq));
            const uint64_t dead_mask = __ballot(dead);
            const uint64_t don_mask = __ballot(donor);
            if (dead) list[b + dead_seen + static_cast<uint32_t>(__popcll(dead_mask & lanes_lt))] = i;
            if (donor)
                list[b + z + don_seen + static_cast<uint32_t>(__popcll(don_mask & lanes_lt))] = i;
            dead_seen += static_cast<uint32_t>(__popcll(dead_mask));
            eq_seen += static_cast<uint32_t>(__popcll(eq_mask));
            don_seen += static_cast<uint32_t>(__popcll(don_mask));
        }
        wave_sync();   // list entries written by other lanes are read below
        const uint32_t nd = don_seen;   // <= take <= z, and z + nd <= n
        for (uint32_t k = lane; k < nd; k += 64u) {
            const uint32_t d = b + list[b + z + k];
            const uint32_t t = b + list[b + k];
            const uint64_t x = xi[d];
            const uint64_t half = x >> 1;
            xi[t] = half;
            r[t] = r[d];
            if (rd3) {
                rd3[t] = rd3[d];
                kappa[t] = kappa[d];
            }
            xi[d] = x - half;
        }
        done += nd;
    }
    // one atomic per workgroup
    __shared__ uint32_t s_done[kRecycleCellsPerBlock];
    if (lane == 0) s_done[threadIdx.x / 64u] = done;
    __syncthreads();
    if (threadIdx.x == 0 && stats) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < kRecycleCellsPerBlock; ++w) t += s_done[w];
        if (t)
            atomicAdd(stats + (blockIdx.x % kStatSlots) * kStatStride + kRecycledStat,
                      static_cast<unsigned long long>(t));
    }
}

// Second pass of recycling: for the pairs k_recycle listed, the radius (and the
// dry attributes, when present) of the donor to its dead slot.  One thread per
// cell; donors are never targets, so the copies are independent.
__global__ __launch_bounds__(256) void k_recycle_copy(const uint32_t* __restrict__ off,
                                                      const uint32_t* __restrict__ pairs,
                                                      const uint32_t* __restrict__ list,
                                                      uint32_t n_cells, double* __restrict__ r,
                                                      double* __restrict__ rd3,
                                                      double* __restrict__ kappa)
{
    for (uint64_t c = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; c < n_cells;
         c += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t np = pairs[c];
        if (np == 0) continue;
        const uint32_t b = off[c];
        for (uint32_t k = 0; k < np; ++k) {
            const uint32_t e = list[b + k];
            const uint32_t t = b + (e & 0xffffu), d = b + (e >> 16);
            r[t] = r[d];
            if (rd3) {
                rd3[t] = rd3[d];
                kappa[t] = kappa[d];
            }
        }
    }
}

}  // namespace
}  // namespace sdm
