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
// is the largest multiplicity when take = 1, else found bit by bit from the top
// as the largest v with #{xi >= v} >= take (the first 256 slots of the cell are
// counted from registers with ballots, any further ones from memory); the
// donors are then every slot above T plus the lowest-slot ones equal to T.
// Dead and donor slots are listed in slot order (ballot prefix counts) in a
// per-cell scratch range, and the list pairs are applied last, so no slot is
// classified after it has been written.
#pragma once

#include "step_kernels.hpp"

namespace sdm {
namespace {

constexpr int kRecycleBlock = 256;
constexpr uint32_t kRecycleCellsPerBlock = kRecycleBlock / 64;
constexpr int kRecycleRegs = 4;   // slots per lane held in registers (256 per cell)

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

// list: uint32[n_sd] scratch, cell c uses [off[c], off[c+1]).
// recycled: counter (nullable) incremented by the number of recycled slots.
// rd3, kappa: optional dry attributes (nullable), copied with the radius.
__global__ __launch_bounds__(kRecycleBlock) void k_recycle(const uint32_t* __restrict__ off,
                                                           uint64_t* __restrict__ xi,
                                                           double* __restrict__ r,
                                                           uint32_t n_cells,
                                                           uint32_t* __restrict__ list,
                                                           unsigned long long* recycled,
                                                           double* __restrict__ rd3,
                                                           double* __restrict__ kappa)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lanes_lt = (1ull << lane) - 1ull;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kRecycleCellsPerBlock;
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
        // threshold: the take-th largest multiplicity
        uint64_t T = xmax;
        if (take > 1) {
            T = 0;
            for (int bit = 63 - __clzll(static_cast<long long>(xmax)); bit >= 0; --bit) {
                const uint64_t cand = T | (1ull << bit);
                if (count_at_least(xi, b, n, xr, cand, lane) >= take) T = cand;
            }
        }
        const uint32_t above = count_at_least(xi, b, n, xr, T + 1u, lane);
        const uint32_t need_eq = take - above;
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
    if (threadIdx.x == 0 && recycled) {
        uint32_t t = 0;
        for (uint32_t w = 0; w < kRecycleCellsPerBlock; ++w) t += s_done[w];
        if (t) atomicAdd(recycled, static_cast<unsigned long long>(t));
    }
}

}  // namespace
}  // namespace sdm
