// plan_kernels.hpp -- the launch plan of the wavefront tier built on the
// device from the slot offsets, so that no offset has to travel to the host.
#pragma once

#include "init_kernels.hpp"

namespace sdm {

namespace {

// ---------------------------------------------------------------------------
// Launch plan on the device.  The host plan packs consecutive cells greedily
// into wavefront groups (at most group_slots slots and kGroupMaxCells cells);
// cells above group_slots go to other tiers.  Seen as a walk, each small cell c
// that opens a group jumps to the first cell after the group, each large cell to
// the next cell, and the group starts are the small cells on the walk from cell
// 0.  Jumps are at most kGroupMaxCells long, so the walk is cut into chunks of
// kPlanChunk cells: every chunk is walked from each of its first
// kGroupMaxCells cells at once (one lane per entry, the jumps in LDS), giving
// a 64-entry exit table per chunk.  The tables are chained in two levels:
// each run of kPlanSuper chunks composes its tables into one, one thread
// chains those, and each run then hands the entries down to its chunks.  The
// real walk of every chunk then marks its group starts.
// ---------------------------------------------------------------------------
constexpr uint32_t kPlanChunk = 1024;
constexpr uint32_t kPlanSuper = 64;   // chunks per run of the chaining
constexpr uint8_t kPlanBig = 0x80;

// jump[c] = cells in the greedy group that cell c would open (1..64), or
// kPlanBig | 1 for a cell above group_slots.
__global__ void k_plan_jump(uint32_t nc, const uint32_t* __restrict__ off, uint32_t cap,
                            uint8_t* __restrict__ jump, unsigned int* __restrict__ big_flag)
{
    for (uint64_t c = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; c < nc;
         c += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t n = off[c + 1] - off[c];
        if (n > cap) {
            jump[c] = kPlanBig | 1u;
            atomicOr(big_flag, 1u);
            continue;
        }
        uint32_t e = static_cast<uint32_t>(c) + 1u, slots = n;
        while (e < nc && e - c < static_cast<uint32_t>(kGroupMaxCells)) {
            const uint32_t m = off[e + 1] - off[e];
            if (m > cap || slots + m > cap) break;
            slots += m;
            ++e;
        }
        jump[c] = static_cast<uint8_t>(e - c);
    }
}

// exits[j * 64 + e]: where the walk entering chunk j at cell e leaves it
// (offset into chunk j + 1).
__global__ __launch_bounds__(kGroupMaxCells) void k_plan_chunks(uint32_t nc,
                                                               const uint8_t* __restrict__ jump,
                                                               uint8_t* __restrict__ exits)
{
    __shared__ uint8_t s_jump[kPlanChunk];
    const uint32_t c0 = blockIdx.x * kPlanChunk;
    const uint32_t len = nc - c0 < kPlanChunk ? nc - c0 : kPlanChunk;
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) s_jump[i] = jump[c0 + i] & 0x7Fu;
    __syncthreads();
    uint32_t p = threadIdx.x;
    while (p < len) p += s_jump[p];
    exits[static_cast<uint64_t>(blockIdx.x) * kGroupMaxCells + threadIdx.x] =
        static_cast<uint8_t>(p - len);
}

// super_exits[S * 64 + e]: where the walk entering the first chunk of run S at
// cell e leaves the run (offset into the chunk after it).
__global__ __launch_bounds__(kGroupMaxCells) void k_plan_super(uint32_t n_chunks,
                                                              const uint8_t* __restrict__ exits,
                                                              uint8_t* __restrict__ super_exits)
{
    __shared__ uint8_t s_ex[kPlanSuper * kGroupMaxCells];
    const uint32_t j0 = blockIdx.x * kPlanSuper;
    const uint32_t nj = n_chunks - j0 < kPlanSuper ? n_chunks - j0 : kPlanSuper;
    for (uint32_t i = threadIdx.x; i < nj * kGroupMaxCells; i += blockDim.x)
        s_ex[i] = exits[static_cast<uint64_t>(j0) * kGroupMaxCells + i];
    __syncthreads();
    uint32_t e = threadIdx.x;
    for (uint32_t j = 0; j < nj; ++j) e = s_ex[j * kGroupMaxCells + e];
    super_exits[static_cast<uint64_t>(blockIdx.x) * kGroupMaxCells + threadIdx.x] =
        static_cast<uint8_t>(e);
}

// one thread: the entry of every run (the walk starts at cell 0)
__global__ void k_plan_stitch(uint32_t n_super, const uint8_t* __restrict__ super_exits,
                              uint8_t* __restrict__ super_entries)
{
    uint32_t e = 0;
    for (uint32_t S = 0; S < n_super; ++S) {
        super_entries[S] = static_cast<uint8_t>(e);
        e = super_exits[static_cast<uint64_t>(S) * kGroupMaxCells + e];
    }
}

// the entry of every chunk of run S, from the run's entry
__global__ __launch_bounds__(kGroupMaxCells) void k_plan_entries(
    uint32_t n_chunks, const uint8_t* __restrict__ exits, const uint8_t* __restrict__ super_entries,
    uint8_t* __restrict__ entries)
{
    __shared__ uint8_t s_ex[kPlanSuper * kGroupMaxCells];
    const uint32_t j0 = blockIdx.x * kPlanSuper;
    const uint32_t nj = n_chunks - j0 < kPlanSuper ? n_chunks - j0 : kPlanSuper;
    for (uint32_t i = threadIdx.x; i < nj * kGroupMaxCells; i += blockDim.x)
        s_ex[i] = exits[static_cast<uint64_t>(j0) * kGroupMaxCells + i];
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t e = super_entries[blockIdx.x];
        for (uint32_t j = 0; j < nj; ++j) {
            entries[j0 + j] = static_cast<uint8_t>(e);
            e = s_ex[j * kGroupMaxCells + e];
        }
    }
}

// start[c] = 1 for the group starts of chunk j (small cells on the walk), else 0;
// the walk marks in LDS, the flags are written out by the whole workgroup.
__global__ __launch_bounds__(256) void k_plan_mark(uint32_t nc, const uint8_t* __restrict__ jump,
                                                   const uint8_t* __restrict__ entries,
                                                   uint32_t* __restrict__ start)
{
    __shared__ uint8_t s_jump[kPlanChunk];
    __shared__ uint8_t s_mark[kPlanChunk];
    const uint32_t c0 = blockIdx.x * kPlanChunk;
    const uint32_t len = nc - c0 < kPlanChunk ? nc - c0 : kPlanChunk;
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
        s_jump[i] = jump[c0 + i];
        s_mark[i] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t p = entries[blockIdx.x];
        while (p < len) {
            const uint8_t j = s_jump[p];
            if (!(j & kPlanBig)) s_mark[p] = 1;
            p += j & 0x7Fu;
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) start[c0 + i] = s_mark[i];
}

__global__ void k_plan_emit(uint32_t nc, const uint32_t* __restrict__ prefix,
                            const uint8_t* __restrict__ jump, uint32_t* __restrict__ group_begin,
                            uint32_t* __restrict__ group_end)
{
    for (uint64_t c = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; c < nc;
         c += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t g = prefix[c];
        if (prefix[c + 1] != g) {
            group_begin[g] = static_cast<uint32_t>(c);
            group_end[g] = static_cast<uint32_t>(c) + (jump[c] & 0x7Fu);
        }
    }
}

// The device plan must tile [0, nc) with groups of 1..kGroupMaxCells cells and at
// most cap slots; anything else sets bit 0 of *bad and the host plan is used.
__global__ void k_plan_check(uint32_t n_groups, uint32_t nc, const uint32_t* __restrict__ gb,
                             const uint32_t* __restrict__ ge, const uint32_t* __restrict__ off,
                             uint32_t cap, unsigned int* __restrict__ bad)
{
    for (uint64_t g = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; g < n_groups;
         g += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t b = gb[g], e = ge[g];
        bool ok = e > b && e - b <= static_cast<uint32_t>(kGroupMaxCells) && e <= nc &&
                  off[e] - off[b] <= cap;
        ok = ok && (g == 0 ? b == 0u : gb[g] == ge[g - 1]);
        ok = ok && (g + 1 == n_groups ? e == nc : true);
        if (!ok) atomicOr(bad, 1u);
    }
}

}  // namespace

}  // namespace sdm
