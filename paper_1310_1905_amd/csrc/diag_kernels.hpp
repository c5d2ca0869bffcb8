// diag_kernels.hpp -- gridded diagnostics of the particle-based scheme
// (Sect. 5.2: super-droplet concentration and radius moments per cell), as
// segmented reductions over the cell-sorted storage, and the final maximum of
// the collision-probability probe (whose per-cell maxima the probe mode of the
// step kernels writes).
//
// One wavefront per cell.  Lane l accumulates the cell's local slots
// l, l+64, l+128, ... in ascending order; the 64 partial sums are then folded
// pairwise, partial[l] += partial[l+d] for d = 32, 16, ..., 1.  This order is
// part of the definition of the result, so moments are reproducible bit for bit
// whatever the launch shape.
#pragma once

#include "device_math.hpp"

#pragma clang fp contract(off)

namespace sdm {
namespace {

constexpr int kDiagBlock = 256;
constexpr uint32_t kMaxMomentOrder = 16;
constexpr uint32_t kDiagCellsPerBlock = kDiagBlock / 64;
// grid cap of the per-cell kernels: a few cells per wavefront (grid-stride)
// rather than one wavefront launched per cell
constexpr uint32_t kDiagMaxBlocks = 1u << 16;

__device__ __forceinline__ double wave_fold_sum(double v, uint32_t lane)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const double o = __shfl_down(v, d, 64);
        if (lane < static_cast<uint32_t>(d)) v = v + o;
    }
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    return v;
}

// out[c] = (rho_d[c] dV[c])^-1 sum_{live i in c, r_min <= r_i <= r_max} xi_i r_i^k;
// with DRY, r holds r_d^3 and r_i is its correctly rounded cube root.
template <bool DRY>
__global__ __launch_bounds__(kDiagBlock) void k_moments(const uint32_t* __restrict__ off,
                                                        const double* __restrict__ dV,
                                                        const uint64_t* __restrict__ xi,
                                                        const double* __restrict__ r,
                                                        uint32_t n_cells, uint32_t k, double r_min,
                                                        double r_max,
                                                        const double* __restrict__ rho_d,
                                                        double* __restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kDiagCellsPerBlock;
    const uint32_t blk = xcd_contiguous_block(blockIdx.x, gridDim.x);   // out lines per XCD
    for (uint64_t c = static_cast<uint64_t>(blk) * kDiagCellsPerBlock + threadIdx.x / 64u;
         c < n_cells; c += stride) {
        const uint32_t b = off[c], n = off[c + 1] - b;
        double acc = 0.0;
        // slots lane, lane + 64, ... in ascending order; four rows of loads in flight
        for (uint32_t base = 0; base < n; base += 4u * 64u) {
            uint64_t xv[4];
            double rv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t i = base + lane + 64u * t;
                xv[t] = i < n ? xi[b + i] : 0u;
                rv[t] = i < n ? r[b + i] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (xv[t] == 0) continue;
                const double rad = DRY ? cbrt_rn(rv[t]) : rv[t];
                if (rad >= r_min && rad <= r_max) {
                    double rk = 1.0;
                    for (uint32_t e = 0; e < k; ++e) rk = rk * rad;
                    acc = acc + static_cast<double>(xv[t]) * rk;
                }
            }
        }
        acc = wave_fold_sum(acc, lane);
        if (lane == 0) out[c] = acc / ((rho_d ? rho_d[c] : 1.0) * dV[c]);
    }
}

// out[c] = number of live super-droplets of cell c
__global__ __launch_bounds__(kDiagBlock) void k_sd_conc(const uint32_t* __restrict__ off,
                                                        const uint64_t* __restrict__ xi,
                                                        uint32_t n_cells, uint32_t* __restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * kDiagCellsPerBlock;
    const uint32_t blk = xcd_contiguous_block(blockIdx.x, gridDim.x);   // out lines per XCD
    for (uint64_t c = static_cast<uint64_t>(blk) * kDiagCellsPerBlock + threadIdx.x / 64u;
         c < n_cells; c += stride) {
        const uint32_t b = off[c], n = off[c + 1] - b;
        uint32_t cnt = 0;
        for (uint32_t base = 0; base < n; base += 4u * 64u) {
            uint64_t xv[4];
            // branch-free loads (the index clamped to the cell's last slot, n > 0
            // here), so that all four are in flight together
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t i = base + lane + 64u * t;
                const uint64_t v = xi[b + (i < n ? i : n - 1u)];
                xv[t] = i < n ? v : 0u;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) cnt += static_cast<uint32_t>(__popcll(__ballot(xv[t] != 0)));
        }
        if (lane == 0) out[c] = cnt;
    }
}

// Slots of the running maximum of k_max_reduce, kMaxStride words apart (one
// 128-byte line each, so that the workgroups' atomics spread over lines).
constexpr uint32_t kMaxSlots = 16;
constexpr uint32_t kMaxStride = 16;

// max over the slots gmax[s * kMaxStride] = max(those, max of v[0, n)) for
// non-negative doubles, as the bit pattern (which orders like the value); one
// atomic per workgroup, on slot blockIdx % kMaxSlots.
__global__ __launch_bounds__(kDiagBlock) void k_max_reduce(const double* __restrict__ v, uint32_t n,
                                                          unsigned long long* __restrict__ gmax)
{
    const uint32_t lane = threadIdx.x & 63u;
    double best = 0.0;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * kDiagBlock + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kDiagBlock)
        best = fmax(best, v[i]);
    best = wave_max(best);
    __shared__ double s_best[kDiagCellsPerBlock];
    if (lane == 0) s_best[threadIdx.x / 64u] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = s_best[0];
        for (uint32_t w = 1; w < kDiagCellsPerBlock; ++w) b = fmax(b, s_best[w]);
        if (b > 0.0)
            atomicMax(gmax + (blockIdx.x % kMaxSlots) * kMaxStride,
                      static_cast<unsigned long long>(__double_as_longlong(b)));
    }
}

}  // namespace
}  // namespace sdm
