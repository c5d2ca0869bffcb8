// init_kernels.hpp -- admission of super-droplets into storage order:
// validation, a stable least-significant-digit radix sort of (cell, input
// index) pairs, the per-cell histogram and exclusive scan that give the slot
// offsets, and the gather/scatter between input order and storage order.
#pragma once

#include "step_kernels.hpp"

namespace sdm {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr uint32_t kScanTile = kScanBlock * kScanItems;   // elements per scan workgroup
constexpr int kRadixBits = 8;
constexpr uint32_t kRadixDigits = 1u << kRadixBits;
constexpr uint32_t kRadixTile = 1024;                     // elements per radix workgroup (one wave)

// Kernels below have internal linkage: every translation unit that launches
// one gets its own copy.
namespace {

enum : uint32_t {
    kErrCell = 1u,      // cell index out of range
    kErrRadius = 2u,    // radius not finite and positive
    kErrVolume = 4u     // cell volume not finite and positive
};

__global__ void k_validate_sds(uint64_t n, const uint32_t* cell, const double* r, uint32_t n_cells,
                               unsigned int* err)
{
    uint32_t bad = 0;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        if (cell[i] >= n_cells) bad |= kErrCell;
        const double v = r[i];
        if (!(v > 0.0) || !(v < __builtin_inf())) bad |= kErrRadius;
    }
    if (bad) atomicOr(err, bad);
}

__global__ void k_validate_volumes(uint32_t n, const double* dV, unsigned int* err)
{
    uint32_t bad = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double v = dV[i];
        if (!(v > 0.0) || !(v < __builtin_inf())) bad |= kErrVolume;
    }
    if (bad) atomicOr(err, bad);
}

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, unsigned long long v)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

// keys = cell + key_add, vals = iota + val_add
__global__ void k_keys_iota(uint64_t n, const uint32_t* cell, uint32_t key_add, uint32_t* keys,
                            uint32_t* vals, uint32_t val_add)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        keys[i] = cell[i] + key_add;
        vals[i] = static_cast<uint32_t>(i) + val_add;
    }
}

// Slot offsets from the cell indices sorted ascending: offsets[c] = first j with
// keys[j] >= c, for c = 0..n_cells (so offsets[n_cells] = n).  Element j writes
// the offsets of the cells that start at j, so every entry is written once and
// no atomics are needed.
__global__ void k_offsets_from_sorted(uint64_t n, const uint32_t* keys, uint32_t n_cells,
                                      uint32_t* offsets)
{
    for (uint64_t j = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; j <= n;
         j += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t lo = j == 0 ? 0u : static_cast<uint64_t>(keys[j - 1]) + 1u;
        const uint64_t hi = j == n ? static_cast<uint64_t>(n_cells) : keys[j];
        for (uint64_t c = lo; c <= hi; ++c) offsets[c] = static_cast<uint32_t>(j);
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of a uint32 array (three launches: tile sums, scan of the
// tile sums by one workgroup, tile scans with their offsets).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_scan_incl_256(uint32_t v, uint32_t* s_w, uint32_t* total)
{
    constexpr int W = kScanBlock / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint32_t incl = wave_inclusive_sum(v, lane);
    if (lane == kWave - 1) s_w[wv] = incl;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const uint32_t t = s_w[w];
        before += (static_cast<uint32_t>(w) < wv) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return before + incl;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tile_sums(const uint32_t* in, uint64_t n,
                                                              uint32_t* tile_sums)
{
    __shared__ uint32_t s_w[kScanBlock / kWave];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile;
    uint32_t s = 0;
    for (uint32_t t = 0; t < kScanItems; ++t) {
        const uint64_t i = base + t * kScanBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t total;
    block_scan_incl_256(s, s_w, &total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tile_offsets(uint32_t* tile_sums, uint32_t n_tiles)
{
    __shared__ uint32_t s_w[kScanBlock / kWave];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < n_tiles; base += kScanBlock) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < n_tiles ? tile_sums[i] : 0u;
        uint32_t total;
        const uint32_t incl = block_scan_incl_256(v, s_w, &total);
        if (i < n_tiles) tile_sums[i] = carry + incl - v;
        carry += total;
    }
}

// out may alias in
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const uint32_t* in, uint32_t* out,
                                                          uint64_t n, const uint32_t* tile_offsets)
{
    __shared__ uint32_t s_w[kScanBlock / kWave];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile;
    uint32_t carry = tile_offsets[blockIdx.x];
    for (uint32_t t = 0; t < kScanItems; ++t) {
        const uint64_t i = base + t * kScanBlock + threadIdx.x;
        const uint32_t v = i < n ? in[i] : 0u;
        uint32_t total;
        const uint32_t incl = block_scan_incl_256(v, s_w, &total);
        if (i < n) out[i] = carry + incl - v;
        carry += total;
    }
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 8-bit digits.
// Per digit pass: per-tile digit counts -> exclusive scan over (digit, tile)
// -> stable scatter, where a wavefront ranks equal digits by lane order with
// ballots and walks its tile chunk by chunk.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWave) void k_radix_count(const uint32_t* keys, uint64_t n,
                                                       uint32_t shift, uint32_t* counts,
                                                       uint32_t n_tiles)
{
    __shared__ uint32_t hist[kRadixDigits];
    const uint32_t lane = threadIdx.x;
    for (uint32_t d = lane; d < kRadixDigits; d += kWave) hist[d] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kRadixTile;
    // all of the lane's keys first (independent loads), then the histogram
    constexpr uint32_t kPer = kRadixTile / kWave;
    uint32_t kk[kPer];
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
        const uint64_t i = base + t * kWave + lane;
        kk[t] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t)
        if (base + t * kWave + lane < n) atomicAdd(&hist[(kk[t] >> shift) & (kRadixDigits - 1)], 1u);
    __syncthreads();
    for (uint32_t d = lane; d < kRadixDigits; d += kWave)
        counts[static_cast<uint64_t>(d) * n_tiles + blockIdx.x] = hist[d];
}

__global__ __launch_bounds__(kWave) void k_radix_scatter(const uint32_t* keys_in,
                                                         const uint32_t* vals_in,
                                                         uint32_t* keys_out, uint32_t* vals_out,
                                                         uint64_t n, uint32_t shift,
                                                         const uint32_t* offsets,
                                                         uint32_t n_tiles)
{
    __shared__ uint32_t run[kRadixDigits];
    const uint32_t lane = threadIdx.x;
    for (uint32_t d = lane; d < kRadixDigits; d += kWave)
        run[d] = offsets[static_cast<uint64_t>(d) * n_tiles + blockIdx.x];
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kRadixTile;
    // all of the lane's keys and values first (independent loads), then the
    // chunks in order
    constexpr uint32_t kPer = kRadixTile / kWave;
    uint32_t kk[kPer], vv[kPer];
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
        const uint64_t i = base + t * kWave + lane;
        kk[t] = i < n ? keys_in[i] : 0u;
        vv[t] = i < n ? vals_in[i] : 0u;
    }
#pragma unroll
    for (uint32_t t = 0; t < kPer; ++t) {
        const uint64_t i = base + t * kWave + lane;
        const bool valid = i < n;
        const uint32_t k = kk[t];
        const uint32_t v = vv[t];
        const uint32_t d = (k >> shift) & (kRadixDigits - 1);
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const unsigned long long ones = __ballot(valid && ((d >> b) & 1u));
            same &= ((d >> b) & 1u) ? ones : ~ones;
        }
        const uint32_t rank = static_cast<uint32_t>(__popcll(same & lt));
        const uint32_t pos = valid ? run[d] + rank : 0u;
        __syncthreads();
        if (valid) {
            keys_out[pos] = k;
            vals_out[pos] = v;
            // the highest lane of each digit group advances the digit's cursor
            if ((same >> lane) == 1ull) run[d] += static_cast<uint32_t>(__popcll(same));
        }
        __syncthreads();
    }
}

// storage order <- input order
__global__ void k_gather_state(uint64_t n, const uint32_t* idx, const uint64_t* xi_in,
                               const double* r_in, uint64_t* xi, double* r, uint32_t idx_sub)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t src = idx[i] - idx_sub;
        xi[i] = xi_in[src];
        r[i] = r_in[src];
    }
}

// input order <- storage order
__global__ void k_scatter_state(uint64_t n, const uint32_t* idx, const uint64_t* xi,
                                const double* r, uint64_t* xi_out, double* r_out,
                                uint32_t idx_sub)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint32_t dst = idx[i] - idx_sub;
        if (xi_out) xi_out[dst] = xi[i];
        if (r_out) r_out[dst] = r[i];
    }
}

__global__ void k_copy_u64(uint64_t n, const uint64_t* src, uint64_t* dst)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

}  // namespace
}  // namespace sdm
