// runtime.hpp -- host-side helpers shared by the single-run context and the
// batch: error reporting, workspace carving, launch helpers for the scan and
// the sort-by-cell used at admission, and the launch of the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/sdm.h"
#include "init_kernels.hpp"

namespace sdm {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);

#define SDM_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::sdm::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                             __FILE__, __LINE__);                                       \
            return SDM_EDEVICE;                                                         \
        }                                                                               \
    } while (0)

#define SDM_LAUNCHED()                                                                  \
    do {                                                                                \
        hipError_t e_ = hipGetLastError();                                              \
        if (e_ != hipSuccess) {                                                         \
            ::sdm::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_),   \
                             __FILE__, __LINE__);                                       \
            return SDM_EDEVICE;                                                         \
        }                                                                               \
    } while (0)

#define SDM_TRY(...)                                                                    \
    do {                                                                                \
        sdm_status s_ = (__VA_ARGS__);                                                         \
        if (s_ != SDM_OK) return s_;                                                    \
    } while (0)

// --------------------------------------------------------------- workspace
struct Carver {
    uintptr_t base = 0, cur = 0, end = 0;
    bool measuring = true;
    explicit Carver(void* ws = nullptr, size_t bytes = 0)
    {
        base = cur = reinterpret_cast<uintptr_t>(ws);
        end = base + bytes;
        measuring = (ws == nullptr);
    }
    template <class T>
    T* take(uint64_t count)
    {
        cur = (cur + 255u) & ~static_cast<uintptr_t>(255u);
        T* p = reinterpret_cast<T*>(cur);
        cur += static_cast<uintptr_t>(count * sizeof(T));
        return p;
    }
    size_t used() const { return static_cast<size_t>(cur - base) + 256u; }
};

inline uint32_t grid_for(uint64_t n, uint32_t block, uint32_t cap = 1u << 16)
{
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<uint32_t>(g);
}

inline KernelParams to_kp(const sdm_kernel_params& p)
{
    KernelParams k;
    k.golovin_b = p.golovin_b;
    k.k1 = p.vt_k1;
    k.k2 = p.vt_k2;
    k.k3 = p.vt_k3;
    k.r1 = p.vt_r1;
    k.r2 = p.vt_r2;
    k.eff = p.efficiency;
    return k;
}

bool params_valid(const sdm_kernel_params& p);

// Scratch a sort-by-cell of n SDs needs (bytes), and its launch sequence.
struct SortScratch {
    uint32_t* keys_a;
    uint32_t* vals_a;
    uint32_t* keys_b;
    uint32_t* vals_b;
    uint32_t* radix_counts;   // kRadixDigits * tiles
    uint32_t* tile_sums;      // scan tile sums
};
void carve_sort_scratch(Carver& c, uint64_t n_sd, uint32_t n_cells, SortScratch* s);

// exclusive scan of n uint32 (in may equal out)
sdm_status scan_exclusive(hipStream_t s, const uint32_t* in, uint32_t* out, uint64_t n,
                          uint32_t* tile_sums);

// Validate and stable-sort n SDs by cell.  On success: *order (one of the
// scratch arrays) holds the input index of each storage slot, and
// offsets[0..n_cells] (dev) the slot offsets.  Synchronises the stream.
sdm_status sort_by_cell(hipStream_t s, uint64_t n, const uint32_t* cell, const double* r,
                        uint32_t n_cells, const double* dV, SortScratch& scr,
                        uint32_t* offsets, unsigned int* err_dev, const uint32_t** order);

// The sort alone (no validation, no synchronisation): *order (a scratch array)
// holds, for each new slot, the index of the element that moves there (stable),
// offsets[0..n_cells] the slot offsets.  Cell indices must be < n_cells.
sdm_status radix_sort_by_cell(hipStream_t s, uint64_t n, const uint32_t* cell, uint32_t n_cells,
                              SortScratch& scr, uint32_t* offsets, const uint32_t** order);

// Launch shape of the step kernels (none of it changes a result).
struct LaunchShape {
    uint32_t group_slots = 512;      // storage slots per wave-tier group (64, 128, 256 or 512)
    uint32_t groups_per_wave = 2;
    uint32_t waves_per_block = 1;
    uint32_t xcd_remap = 0;
    uint32_t block_slots = kBlockLarge;   // largest cell of the workgroup tier (0: none)
    uint32_t block_split = 0;   // single runs: 2^block_split workgroups per workgroup-tier cell
};

// Work lists of one step: wave-tier groups of consecutive cells and the
// grid-tier cells with their chunk, table-tile and bucket lists.
struct Plan {
    std::vector<uint32_t> group_begin, group_end;
    uint32_t wave_cells = 0;
    // grid tier
    std::vector<GridCell> grid;
    std::vector<uint32_t> grid_sizes;
    // workgroup tier: cells and their slot counts (ordered by plan_finish)
    std::vector<uint32_t> block, block_sizes;
    uint32_t block_big = 0;
    std::vector<uint2> gtile;
    std::vector<uint4> gchunk, gbucket;
};

// Device arrays of the grid tier (inside a workspace) and their capacities.
struct GridArrays {
    GridCell* gcell = nullptr;
    uint4* gchunk = nullptr;
    uint2* gtile = nullptr;
    uint4* gbucket = nullptr;
    uint32_t* gtilesum = nullptr;
    uint32_t* blist = nullptr;      // workgroup-tier cells
    uint32_t* split_arrive = nullptr;   // split tier: arrival counters of those cells
    uint32_t split_epoch = 0;       // split-tier steps since the counters were cleared
    uint64_t cap_cells = 0, cap_chunks = 0, cap_tiles = 0, cap_buckets = 0;
    uint64_t cap_block = 0;
    uint32_t n_grid = 0, n_gchunk = 0, n_gtile = 0, n_gbucket = 0;
    uint32_t n_block = 0, n_block_big = 0;
    uint32_t dmax = 0;              // largest 2^cb of the grid cells
};
void carve_grid(Carver& c, uint64_t n_sd, uint32_t n_cells, GridArrays* g);
sdm_status upload_grid(hipStream_t s, const Plan& plan, GridArrays* g);
void grid_args(const GridArrays& g, StepArgs* a);

// Append to `plan` the cells [c_begin, c_begin + n_cells) whose storage-slot
// counts are sizes[0..): cells above block_slots go to the grid tier, cells
// above group_slots (and up to block_slots) to the workgroup tier, the rest are
// packed greedily into groups of at most group_slots slots and kGroupMaxCells
// cells.
void plan_cells(Plan& plan, uint32_t c_begin, const uint32_t* sizes, uint32_t n_cells,
                uint32_t group_slots, uint32_t block_slots);
// Per-cell parameters and work lists of the grid tier; the workgroup-tier cells
// in descending order of slots (ties by cell index).
void plan_finish(Plan& plan);

// Enqueue the wave-tier and grid-tier kernels for one step (base carries the
// grid-tier arrays, see grid_args).
// probe: instead of the collisions, the largest P_ij of every cell goes to
// base.cell_max (single runs only; grid-tier entries must start at 0).
// *split_enqueued (nullable) becomes true once a split-tier kernel is enqueued.
// fork (nullable): a side stream and two events; when the grid tier and another
// tier both have cells, the wavefront and workgroup tiers run on the side stream,
// concurrently with the grid tier's chain of launches, and s waits for them
// before this returns (their cells are disjoint, and the counters they share
// are integer atomics, so the results do not depend on the interleaving).
struct StreamFork {
    hipStream_t side = nullptr;
    hipEvent_t begin = nullptr, end = nullptr;
};
sdm_status launch_step(hipStream_t s, const StepArgs& base, const uint32_t* group_begin,
                       const uint32_t* group_end, uint32_t n_groups, const LaunchShape& shape,
                       bool batched, bool perm, bool probe = false,
                       bool* split_enqueued = nullptr, const StreamFork* fork = nullptr);

bool shape_valid(const LaunchShape& sh);

// Arrays of the launch plan built on the device (inside a workspace).
struct DevicePlanArrays {
    uint8_t* jump = nullptr;          // cells of the greedy group a cell would open
    uint8_t* exits = nullptr;         // chunk walk exits per entry
    uint8_t* entries = nullptr;       // chunk walk entries
    uint8_t* super_exits = nullptr;   // exits of runs of chunk tables, per entry
    uint8_t* super_entries = nullptr;
    uint32_t* start = nullptr;        // group-start flags, then their prefix (n_cells + 1)
    uint32_t* info = nullptr;         // [0] large-cell flag, [1] plan check flag
    uint32_t* tile_sums = nullptr;    // scan scratch
};
void carve_device_plan(Carver& c, uint32_t n_cells, DevicePlanArrays* p);

// Greedy wavefront-tier groups of the cells [0, nc) (at most cap slots and
// kGroupMaxCells cells each), built on the device from the slot offsets
// (dev, nc + 1 entries) into group_begin / group_end (dev, nc entries each).
// *usable = every cell holds at most cap slots and the groups passed their
// check; then *n_groups is their number.  *big = some cell holds more than cap
// slots.  Synchronises the stream (to read the group count).
sdm_status device_plan(hipStream_t s, uint32_t nc, const uint32_t* offsets, uint32_t cap,
                       const DevicePlanArrays& p, uint32_t* group_begin, uint32_t* group_end,
                       uint32_t* n_groups, bool* usable, bool* big);

}  // namespace sdm
