// runtime.hip -- shared host runtime: errors, scan/sort launches and the
// dispatch of the step kernels over launch shapes.
#include "runtime.hpp"
#include "plan_kernels.hpp"

#include <algorithm>
#include <cmath>

namespace sdm {

static thread_local char g_last_error[768] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

bool params_valid(const sdm_kernel_params& p)
{
    const double v[7] = {p.golovin_b, p.vt_k1, p.vt_k2, p.vt_k3, p.vt_r1, p.vt_r2, p.efficiency};
    for (double x : v)
        if (!std::isfinite(x) || x < 0.0) return false;
    return p.vt_r1 <= p.vt_r2;
}

void carve_sort_scratch(Carver& c, uint64_t n_sd, uint32_t n_cells, SortScratch* s)
{
    const uint64_t tiles = (n_sd + kRadixTile - 1) / kRadixTile;
    const uint64_t radix_entries = tiles * kRadixDigits;
    uint64_t longest = radix_entries > static_cast<uint64_t>(n_cells) + 1 ? radix_entries
                                                                           : static_cast<uint64_t>(n_cells) + 1;
    s->keys_a = c.take<uint32_t>(n_sd);
    s->vals_a = c.take<uint32_t>(n_sd);
    s->keys_b = c.take<uint32_t>(n_sd);
    s->vals_b = c.take<uint32_t>(n_sd);
    s->radix_counts = c.take<uint32_t>(radix_entries);
    s->tile_sums = c.take<uint32_t>((longest + kScanTile - 1) / kScanTile + 1);
}

sdm_status scan_exclusive(hipStream_t s, const uint32_t* in, uint32_t* out, uint64_t n,
                          uint32_t* tile_sums)
{
    if (n == 0) return SDM_OK;
    const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles > 0xFFFFFFFFull) {
        set_error("scan of %llu elements is too long", static_cast<unsigned long long>(n));
        return SDM_EINVAL;
    }
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(static_cast<uint32_t>(tiles)), dim3(kScanBlock), 0,
                       s, in, n, tile_sums);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_scan_tile_offsets, dim3(1), dim3(kScanBlock), 0, s, tile_sums,
                       static_cast<uint32_t>(tiles));
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_scan_tiles, dim3(static_cast<uint32_t>(tiles)), dim3(kScanBlock), 0, s,
                       in, out, n, tile_sums);
    SDM_LAUNCHED();
    return SDM_OK;
}

sdm_status sort_by_cell(hipStream_t s, uint64_t n, const uint32_t* cell, const double* r,
                        uint32_t n_cells, const double* dV, SortScratch& scr,
                        uint32_t* offsets, unsigned int* err_dev, const uint32_t** order)
{
    // validation
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(err_dev),
                       uint64_t(1), 0u);
    SDM_LAUNCHED();
    if (n > 0) {
        hipLaunchKernelGGL(k_validate_sds, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, n, cell,
                           r, n_cells, err_dev);
        SDM_LAUNCHED();
    }
    if (n_cells > 0) {
        hipLaunchKernelGGL(k_validate_volumes, dim3(grid_for(n_cells, 256, 4096)), dim3(256), 0, s,
                           n_cells, dV, err_dev);
        SDM_LAUNCHED();
    }
    unsigned int err_host = 0;
    SDM_HIP(hipMemcpyAsync(&err_host, err_dev, sizeof(err_host), hipMemcpyDeviceToHost, s));
    SDM_HIP(hipStreamSynchronize(s));
    if (err_host) {
        set_error("invalid input:%s%s%s", (err_host & kErrCell) ? " cell index >= n_cells" : "",
                  (err_host & kErrRadius) ? " radius not finite and > 0" : "",
                  (err_host & kErrVolume) ? " cell volume not finite and > 0" : "");
        return SDM_EINVAL;
    }

    return radix_sort_by_cell(s, n, cell, n_cells, scr, offsets, order);
}

sdm_status radix_sort_by_cell(hipStream_t s, uint64_t n, const uint32_t* cell, uint32_t n_cells,
                              SortScratch& scr, uint32_t* offsets, const uint32_t** order)
{
    // stable LSD radix sort of (cell, input index)
    uint32_t* ka = scr.keys_a;
    uint32_t* va = scr.vals_a;
    uint32_t* kb = scr.keys_b;
    uint32_t* vb = scr.vals_b;
    if (n > 0) {
        hipLaunchKernelGGL(k_keys_iota, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, cell, 0u,
                           ka, va, 0u);
        SDM_LAUNCHED();
        const uint32_t bits = n_cells > 1 ? 32u - static_cast<uint32_t>(__builtin_clz(n_cells - 1u)) : 0u;
        const uint64_t tiles = (n + kRadixTile - 1) / kRadixTile;
        for (uint32_t shift = 0; shift < bits; shift += kRadixBits) {
            hipLaunchKernelGGL(k_radix_count, dim3(static_cast<uint32_t>(tiles)), dim3(kWave), 0, s,
                               ka, n, shift, scr.radix_counts, static_cast<uint32_t>(tiles));
            SDM_LAUNCHED();
            SDM_TRY(scan_exclusive(s, scr.radix_counts, scr.radix_counts, tiles * kRadixDigits,
                                   scr.tile_sums));
            hipLaunchKernelGGL(k_radix_scatter, dim3(static_cast<uint32_t>(tiles)), dim3(kWave), 0,
                               s, ka, va, kb, vb, n, shift, scr.radix_counts,
                               static_cast<uint32_t>(tiles));
            SDM_LAUNCHED();
            uint32_t* t = ka; ka = kb; kb = t;
            t = va; va = vb; vb = t;
        }
    }
    *order = va;

    // slot offsets from the sorted cell indices (ka)
    hipLaunchKernelGGL(k_offsets_from_sorted, dim3(grid_for(n + 1, 256, 8192)), dim3(256), 0, s, n,
                       ka, n_cells, offsets);
    SDM_LAUNCHED();
    return SDM_OK;
}

// ------------------------------------------------------------ step plan
void plan_cells(Plan& plan, uint32_t c_begin, const uint32_t* sizes, uint32_t n_cells,
                uint32_t group_slots, uint32_t block_slots)
{
    uint32_t g_start = 0, g_slots = 0;
    bool open = false;
    for (uint32_t i = 0; i < n_cells; ++i) {
        const uint32_t c = c_begin + i;
        const uint32_t n = sizes[i];
        if (n > group_slots) {
            if (open) {
                plan.group_begin.push_back(g_start);
                plan.group_end.push_back(c);
                open = false;
            }
            if (n <= block_slots) {
                plan.block.push_back(c);
                plan.block_sizes.push_back(n);
            } else {
                plan.grid.push_back(GridCell{c, 0, 0, 0, 0, 0, 0, 0});
                plan.grid_sizes.push_back(n);
            }
            continue;
        }
        if (open && (g_slots + n > group_slots || c - g_start >= static_cast<uint32_t>(kGroupMaxCells))) {
            plan.group_begin.push_back(g_start);
            plan.group_end.push_back(c);
            open = false;
        }
        if (!open) {
            g_start = c;
            g_slots = 0;
            open = true;
        }
        g_slots += n;
        ++plan.wave_cells;
    }
    if (open) {
        plan.group_begin.push_back(g_start);
        plan.group_end.push_back(c_begin + n_cells);
    }
}

void plan_finish(Plan& plan)
{
    // workgroup tier: largest cells first
    {
        std::vector<uint32_t> idx(plan.block.size());
        for (uint32_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) {
            return plan.block_sizes[x] > plan.block_sizes[y];
        });
        std::vector<uint32_t> cells(idx.size()), sizes(idx.size());
        plan.block_big = 0;
        for (uint32_t i = 0; i < idx.size(); ++i) {
            cells[i] = plan.block[idx[i]];
            sizes[i] = plan.block_sizes[idx[i]];
            if (sizes[i] > kBlockSmall) ++plan.block_big;
        }
        plan.block.swap(cells);
        plan.block_sizes.swap(sizes);
    }
    // grid tier: digit bits cb = ceil(log2 N) - kGridBucketLg (at most
    // kGridMaxDigitBits) and slot chunks of 2^lgc slots, lgc = max(11, lgN - 9),
    // keep the count table 2^cb * ncol below N, so that it and its sentinel fit
    // the cell's scr_cnt range
    uint32_t tile = 0;
    for (uint32_t i = 0; i < plan.grid.size(); ++i) {
        const uint32_t n = plan.grid_sizes[i];
        const uint32_t lgn = 32u - static_cast<uint32_t>(__builtin_clz(n - 1u));
        GridCell& gc = plan.grid[i];
        gc.lgc = std::max(kGridChunkLg, lgn > 9u ? lgn - 9u : 0u);
        gc.ncol = static_cast<uint32_t>((static_cast<uint64_t>(n) + (1u << gc.lgc) - 1u) >> gc.lgc);
        gc.cb = std::min(lgn > kGridBucketLg ? lgn - kGridBucketLg : 0u, kGridMaxDigitBits);
        while (gc.cb > 0 && (static_cast<uint64_t>(gc.ncol) << gc.cb) + 1u > n) --gc.cb;
        gc.nb = gc.ncol << gc.cb;
        gc.tile0 = tile;
        gc.ntiles = (gc.nb + kGridTile - 1) / kGridTile;
        gc.live = 0;
        for (uint32_t t = 0; t < gc.ntiles; ++t) plan.gtile.push_back(make_uint2(i, t * kGridTile));
        tile += gc.ntiles;
        for (uint64_t s0 = 0; s0 < n; s0 += 1u << gc.lgc)
            plan.gchunk.push_back(make_uint4(i, static_cast<uint32_t>(s0), gc.cell, 0u));
        for (uint32_t d = 0; d < (1u << gc.cb); ++d) plan.gbucket.push_back(make_uint4(i, d, gc.cell, 0u));
    }
}

bool shape_valid(const LaunchShape& c)
{
    const bool waves_ok = c.waves_per_block == 1 || c.waves_per_block == 2 || c.waves_per_block == 4;
    const bool slots_ok = c.group_slots == 64 || c.group_slots == 128 || c.group_slots == 256 ||
                          c.group_slots == 512;
    // groups under 256 slots need the workgroup tier: the grid tier's tables are
    // sized for cells of more than 256 slots
    const bool block_ok = (c.block_slots == 0 && c.group_slots >= 256) ||
                          c.block_slots == kBlockSmall || c.block_slots == kBlockLarge;
    const bool split_ok = c.block_split <= kSplitMaxLg && (c.block_split == 0 || c.block_slots > 0);
    return waves_ok && slots_ok && block_ok && split_ok && c.groups_per_wave >= 1 &&
           c.groups_per_wave <= 64 && c.xcd_remap <= 1;
}

void carve_grid(Carver& c, uint64_t n_sd, uint32_t n_cells, GridArrays* g)
{
    // a grid cell has more slots than the smallest group (256)
    g->cap_cells = n_sd / 257 + 1;
    g->cap_chunks = n_sd / kGridChunk + g->cap_cells;
    g->cap_tiles = n_sd / kGridTile + g->cap_cells;
    // 2^cb <= 2^(ceil(log2 N) - 10) < N / 512
    g->cap_buckets = n_sd / (1u << (kGridBucketLg - 1)) + g->cap_cells;
    g->gcell = c.take<GridCell>(g->cap_cells);
    g->gchunk = c.take<uint4>(g->cap_chunks);
    g->gtile = c.take<uint2>(g->cap_tiles);
    g->gbucket = c.take<uint4>(g->cap_buckets);
    g->gtilesum = c.take<uint32_t>(g->cap_tiles);
    // a workgroup-tier cell has more slots than the smallest group (64)
    g->cap_block = std::min<uint64_t>(n_cells, n_sd / 65 + 1);
    g->blist = c.take<uint32_t>(g->cap_block);
    g->split_arrive = c.take<uint32_t>(g->cap_block);
}

sdm_status upload_grid(hipStream_t s, const Plan& plan, GridArrays* g)
{
    if (plan.grid.size() > g->cap_cells || plan.gchunk.size() > g->cap_chunks ||
        plan.gtile.size() > g->cap_tiles || plan.gbucket.size() > g->cap_buckets ||
        plan.block.size() > g->cap_block) {
        set_error("grid-tier tables exceed their capacity");
        return SDM_ENOMEM;
    }
    if (!plan.grid.empty()) {
        SDM_HIP(hipMemcpyAsync(g->gcell, plan.grid.data(), plan.grid.size() * sizeof(GridCell),
                               hipMemcpyHostToDevice, s));
        SDM_HIP(hipMemcpyAsync(g->gchunk, plan.gchunk.data(), plan.gchunk.size() * sizeof(uint4),
                               hipMemcpyHostToDevice, s));
        SDM_HIP(hipMemcpyAsync(g->gtile, plan.gtile.data(), plan.gtile.size() * sizeof(uint2),
                               hipMemcpyHostToDevice, s));
        SDM_HIP(hipMemcpyAsync(g->gbucket, plan.gbucket.data(), plan.gbucket.size() * sizeof(uint4),
                               hipMemcpyHostToDevice, s));
    }
    if (!plan.block.empty()) {
        SDM_HIP(hipMemcpyAsync(g->blist, plan.block.data(), plan.block.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, s));
        SDM_HIP(hipMemsetAsync(g->split_arrive, 0, plan.block.size() * sizeof(uint32_t), s));
    }
    g->split_epoch = 0;
    g->n_block = static_cast<uint32_t>(plan.block.size());
    g->n_block_big = plan.block_big;
    g->n_grid = static_cast<uint32_t>(plan.grid.size());
    g->n_gchunk = static_cast<uint32_t>(plan.gchunk.size());
    g->n_gtile = static_cast<uint32_t>(plan.gtile.size());
    g->n_gbucket = static_cast<uint32_t>(plan.gbucket.size());
    g->dmax = 0;
    for (const GridCell& gc : plan.grid) g->dmax = std::max(g->dmax, 1u << gc.cb);
    return SDM_OK;
}

void grid_args(const GridArrays& g, StepArgs* a)
{
    a->gcell = g.gcell;
    a->n_grid = g.n_grid;
    a->gchunk = g.gchunk;
    a->n_gchunk = g.n_gchunk;
    a->gtile = g.gtile;
    a->n_gtile = g.n_gtile;
    a->gbucket = g.gbucket;
    a->n_gbucket = g.n_gbucket;
    a->gtilesum = g.gtilesum;
    // even, so that the staged words after the counters and cursors are 8-byte aligned
    a->grid_dcap = std::max(2u, std::min(g.dmax, kGridStagedDigits));
    a->grid_dmax = g.dmax;
    a->blist = g.blist;
    a->split_arrive = g.split_arrive;
    a->split_epoch = g.split_epoch;
    a->n_block = g.n_block;
    a->n_block_big = g.n_block_big;
}

// Workgroup tier: 1024-thread workgroups for the cells above kBlockSmall slots
// (the head of the list), 256-thread ones for the rest.  In single runs with
// split_lg > 0 every such cell takes 2^split_lg workgroups of the split tier
// instead (a step launch needs a.split_epoch set by the caller: the number of
// split-tier step launches since the plan was uploaded, this one included; the
// caller counts the launch when *split_enqueued comes back true).
template <bool BATCHED, bool PERM, bool PROBE>
static sdm_status launch_block(hipStream_t s, const StepArgs& a, uint32_t split_lg,
                               bool* split_enqueued)
{
    if (!BATCHED && split_lg > 0) {
        if (split_lg > kSplitMaxLg || (static_cast<uint64_t>(a.n_block) << split_lg) > 0x7FFFFFFFull) {
            set_error("too many split-tier workgroups for one launch");
            return SDM_EINVAL;
        }
        const dim3 grid(a.n_block << split_lg);
        hipLaunchKernelGGL((k_split_cells<kBlockLarge, 1024, PERM, PROBE>), grid, dim3(1024), 0, s,
                           a, a.blist, split_lg);
        SDM_LAUNCHED();
        if (split_enqueued) *split_enqueued = true;
        return SDM_OK;
    }
    if (a.n_block_big > 0) {
        hipLaunchKernelGGL((k_block_cells<kBlockLarge, 1024, BATCHED, PERM, PROBE>),
                           dim3(a.n_block_big), dim3(1024), 0, s, a, a.blist);
        SDM_LAUNCHED();
    }
    if (a.n_block > a.n_block_big) {
        hipLaunchKernelGGL((k_block_cells<kBlockSmall, 256, BATCHED, PERM, PROBE>),
                           dim3(a.n_block - a.n_block_big), dim3(256), 0, s, a,
                           a.blist + a.n_block_big);
        SDM_LAUNCHED();
    }
    return SDM_OK;
}

template <bool BATCHED, bool PERM, bool PROBE>
static sdm_status launch_grid(hipStream_t s, const StepArgs& a)
{
    const dim3 blk(kGridBlock);
    hipLaunchKernelGGL((k_grid_digits<BATCHED, false>), dim3(a.n_gchunk), blk,
                       grid_digits_lds(false, a.grid_dmax, a.grid_dcap), s, a);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_grid_tile_sums, dim3(a.n_gtile), blk, 0, s, a);
    SDM_LAUNCHED();
    if (PERM || PROBE) {
        StepArgs b = a;
        b.stats = nullptr;   // no counters from a permutation query or a probe
        hipLaunchKernelGGL((k_grid_tile_offsets<false>), dim3((a.n_grid + kGridBlock - 1) / kGridBlock),
                           blk, 0, s, b);
    } else {
        hipLaunchKernelGGL((k_grid_tile_offsets<BATCHED>),
                           dim3((a.n_grid + kGridBlock - 1) / kGridBlock), blk, 0, s, a);
    }
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_grid_tile_scan, dim3(a.n_gtile), blk, 0, s, a);
    SDM_LAUNCHED();
    hipLaunchKernelGGL((k_grid_digits<BATCHED, true>), dim3(a.n_gchunk), blk,
                       grid_digits_lds(true, a.grid_dmax, a.grid_dcap), s, a);
    SDM_LAUNCHED();
    hipLaunchKernelGGL((k_grid_bucket_pairs<BATCHED, PERM, PROBE>), dim3(a.n_gbucket), blk, 0, s, a);
    SDM_LAUNCHED();
    if (!PERM) {
        hipLaunchKernelGGL((k_grid_boundary<BATCHED, PROBE>),
                           dim3((a.n_gbucket + kGridBlock - 1) / kGridBlock), blk, 0, s, a);
        SDM_LAUNCHED();
    }
    return SDM_OK;
}

// ------------------------------------------------------------ step launch
template <int CAP, bool BATCHED, bool PERM, bool DRY, bool PROBE = false>
static sdm_status launch_wave(hipStream_t s, const StepArgs& a, uint32_t n_groups,
                              const LaunchShape& sh)
{
    const uint64_t per_block = static_cast<uint64_t>(sh.groups_per_wave) * sh.waves_per_block;
    const uint64_t blocks = (n_groups + per_block - 1) / per_block;
    if (blocks > 0x7FFFFFFFull) {
        set_error("too many groups for one launch");
        return SDM_EINVAL;
    }
    const dim3 grid(static_cast<uint32_t>(blocks));
    switch (sh.waves_per_block) {
    case 1: hipLaunchKernelGGL((k_wave_groups<CAP, 1, BATCHED, PERM, DRY, PROBE>), grid, dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_wave_groups<CAP, 2, BATCHED, PERM, DRY, PROBE>), grid, dim3(128), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_wave_groups<CAP, 4, BATCHED, PERM, DRY, PROBE>), grid, dim3(256), 0, s, a); break;
    default: set_error("waves_per_block must be 1, 2 or 4"); return SDM_EINVAL;
    }
    SDM_LAUNCHED();
    return SDM_OK;
}

template <bool BATCHED, bool PERM>
static sdm_status launch_wave_any(hipStream_t s, const StepArgs& a, uint32_t n_groups,
                                  const LaunchShape& sh)
{
    // the dry attributes exist in single runs only, and a permutation query changes nothing
    if constexpr (!BATCHED && !PERM) {
        if (a.rd3) {
            if (sh.group_slots == 64) return launch_wave<64, false, false, true>(s, a, n_groups, sh);
            if (sh.group_slots == 128) return launch_wave<128, false, false, true>(s, a, n_groups, sh);
            if (sh.group_slots == 256) return launch_wave<256, false, false, true>(s, a, n_groups, sh);
            if (sh.group_slots == 512) return launch_wave<512, false, false, true>(s, a, n_groups, sh);
        }
    }
    if (sh.group_slots == 64) return launch_wave<64, BATCHED, PERM, false>(s, a, n_groups, sh);
    if (sh.group_slots == 128) return launch_wave<128, BATCHED, PERM, false>(s, a, n_groups, sh);
    if (sh.group_slots == 256) return launch_wave<256, BATCHED, PERM, false>(s, a, n_groups, sh);
    if (sh.group_slots == 512) return launch_wave<512, BATCHED, PERM, false>(s, a, n_groups, sh);
    set_error("group_slots must be 64, 128, 256 or 512");
    return SDM_EINVAL;
}

// The probe of a single run (largest P_ij per cell into base.cell_max).
static sdm_status launch_wave_probe(hipStream_t s, const StepArgs& a, uint32_t n_groups,
                                    const LaunchShape& sh)
{
    if (sh.group_slots == 64) return launch_wave<64, false, false, false, true>(s, a, n_groups, sh);
    if (sh.group_slots == 128) return launch_wave<128, false, false, false, true>(s, a, n_groups, sh);
    if (sh.group_slots == 256) return launch_wave<256, false, false, false, true>(s, a, n_groups, sh);
    if (sh.group_slots == 512) return launch_wave<512, false, false, false, true>(s, a, n_groups, sh);
    set_error("group_slots must be 64, 128, 256 or 512");
    return SDM_EINVAL;
}

sdm_status launch_step(hipStream_t s, const StepArgs& base, const uint32_t* group_begin,
                       const uint32_t* group_end, uint32_t n_groups, const LaunchShape& shape,
                       bool batched, bool perm, bool probe, bool* split_enqueued,
                       const StreamFork* fork)
{
    if (probe) {
        if (batched || perm) {
            set_error("a probe is a single-run launch");
            return SDM_EINVAL;
        }
        if (n_groups > 0) {
            StepArgs a = base;
            a.group_begin = group_begin;
            a.group_end = group_end;
            a.n_groups = n_groups;
            a.groups_per_wave = shape.groups_per_wave;
            a.xcd_remap = shape.xcd_remap;
            SDM_TRY(launch_wave_probe(s, a, n_groups, shape));
        }
        if (base.n_block > 0) SDM_TRY((launch_block<false, false, true>(s, base, shape.block_split, split_enqueued)));
        if (base.n_grid > 0) SDM_TRY((launch_grid<false, false, true>(s, base)));
        return SDM_OK;
    }
    const bool forked = fork && fork->side && fork->begin && fork->end && base.n_grid > 0 &&
                        (n_groups > 0 || base.n_block > 0);
    hipStream_t s_small = s;
    if (forked) {
        SDM_HIP(hipEventRecord(fork->begin, s));
        SDM_HIP(hipStreamWaitEvent(fork->side, fork->begin, 0));
        s_small = fork->side;
    }
    // the wavefront and workgroup tiers (on the side stream when forked; it is
    // joined back even when one of these launches fails)
    sdm_status st = SDM_OK;
    if (n_groups > 0) {
        StepArgs a = base;
        a.group_begin = group_begin;
        a.group_end = group_end;
        a.n_groups = n_groups;
        a.groups_per_wave = shape.groups_per_wave;
        a.xcd_remap = shape.xcd_remap;
        if (batched) st = perm ? launch_wave_any<true, true>(s_small, a, n_groups, shape)
                               : launch_wave_any<true, false>(s_small, a, n_groups, shape);
        else st = perm ? launch_wave_any<false, true>(s_small, a, n_groups, shape)
                       : launch_wave_any<false, false>(s_small, a, n_groups, shape);
    }
    if (st == SDM_OK && base.n_block > 0) {
        if (batched)
            st = perm ? launch_block<true, true, false>(s_small, base, 0, nullptr)
                      : launch_block<true, false, false>(s_small, base, 0, nullptr);
        else
            st = perm ? launch_block<false, true, false>(s_small, base, shape.block_split, split_enqueued)
                      : launch_block<false, false, false>(s_small, base, shape.block_split, split_enqueued);
    }
    if (forked) SDM_HIP(hipEventRecord(fork->end, fork->side));
    // the grid tier on s, then s waits for the side stream
    sdm_status gst = SDM_OK;
    if (st == SDM_OK && base.n_grid > 0) {
        if (batched)
            gst = perm ? launch_grid<true, true, false>(s, base) : launch_grid<true, false, false>(s, base);
        else
            gst = perm ? launch_grid<false, true, false>(s, base) : launch_grid<false, false, false>(s, base);
    }
    if (forked) SDM_HIP(hipStreamWaitEvent(s, fork->end, 0));
    return st != SDM_OK ? st : gst;
}

void carve_device_plan(Carver& c, uint32_t nc, DevicePlanArrays* p)
{
    const uint64_t chunks = (uint64_t(nc) + kPlanChunk - 1) / kPlanChunk + 1;
    const uint64_t supers = (chunks + kPlanSuper - 1) / kPlanSuper;
    p->jump = c.take<uint8_t>(uint64_t(nc) + 1);
    p->exits = c.take<uint8_t>(chunks * kGroupMaxCells);
    p->entries = c.take<uint8_t>(chunks);
    p->super_exits = c.take<uint8_t>(supers * kGroupMaxCells);
    p->super_entries = c.take<uint8_t>(supers);
    p->start = c.take<uint32_t>(uint64_t(nc) + 1);
    p->info = c.take<uint32_t>(64);
    p->tile_sums = c.take<uint32_t>((uint64_t(nc) + 1 + kScanTile - 1) / kScanTile + 2);
}

sdm_status device_plan(hipStream_t st, uint32_t nc, const uint32_t* offsets, uint32_t cap,
                       const DevicePlanArrays& P, uint32_t* group_begin, uint32_t* group_end,
                       uint32_t* n_groups, bool* usable, bool* big)
{
    *usable = false;
    *big = false;
    *n_groups = 0;
    if (nc == 0) {
        *usable = true;
        return SDM_OK;
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, P.info, uint64_t(4), 0u);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_plan_jump, dim3(grid_for(nc, 256, 8192)), dim3(256), 0, st, nc, offsets,
                       cap, P.jump, P.info);
    SDM_LAUNCHED();
    const uint32_t chunks = (nc + kPlanChunk - 1) / kPlanChunk;
    hipLaunchKernelGGL(k_plan_chunks, dim3(chunks), dim3(kGroupMaxCells), 0, st, nc, P.jump,
                       P.exits);
    SDM_LAUNCHED();
    const uint32_t supers = (chunks + kPlanSuper - 1) / kPlanSuper;
    hipLaunchKernelGGL(k_plan_super, dim3(supers), dim3(kGroupMaxCells), 0, st, chunks, P.exits,
                       P.super_exits);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_plan_stitch, dim3(1), dim3(1), 0, st, supers, P.super_exits,
                       P.super_entries);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_plan_entries, dim3(supers), dim3(kGroupMaxCells), 0, st, chunks, P.exits,
                       P.super_entries, P.entries);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_plan_mark, dim3(chunks), dim3(256), 0, st, nc, P.jump, P.entries, P.start);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, P.start + nc, uint64_t(1), 0u);
    SDM_LAUNCHED();
    SDM_TRY(scan_exclusive(st, P.start, P.start, uint64_t(nc) + 1, P.tile_sums));
    hipLaunchKernelGGL(k_plan_emit, dim3(grid_for(nc, 256, 8192)), dim3(256), 0, st, nc, P.start,
                       P.jump, group_begin, group_end);
    SDM_LAUNCHED();
    uint32_t info[2] = {0, 0};   // large-cell flag, group count
    SDM_HIP(hipMemcpyAsync(&info[0], P.info, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SDM_HIP(hipMemcpyAsync(&info[1], P.start + nc, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SDM_HIP(hipStreamSynchronize(st));
    if (info[0] != 0) {
        *big = true;
        return SDM_OK;
    }
    hipLaunchKernelGGL(k_plan_check, dim3(grid_for(info[1], 256, 4096)), dim3(256), 0, st, info[1],
                       nc, group_begin, group_end, offsets, cap, P.info + 1);
    SDM_LAUNCHED();
    uint32_t bad = 0;
    SDM_HIP(hipMemcpyAsync(&bad, P.info + 1, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    SDM_HIP(hipStreamSynchronize(st));
    if (bad) return SDM_OK;
    *usable = true;
    *n_groups = info[1];
    return SDM_OK;
}

}  // namespace sdm

extern "C" const char* sdm_last_error(void) { return sdm::g_last_error; }

extern "C" const char* sdm_strerror(sdm_status s)
{
    switch (s) {
    case SDM_OK: return "ok";
    case SDM_EINVAL: return "invalid argument";
    case SDM_ENOMEM: return "workspace too small";
    case SDM_EDEVICE: return "HIP runtime error";
    case SDM_ESTATE: return "invalid state";
    case SDM_EBUDGET: return "batch capacity exhausted";
    }
    return "unknown status";
}

extern "C" void sdm_default_params(sdm_kernel_params* p)
{
    if (!p) return;
    p->golovin_b = 1500.0;
    p->vt_k1 = 1.19e8;
    p->vt_k2 = 8.0e3;
    p->vt_k3 = 201.0;
    p->vt_r1 = 40e-6;
    p->vt_r2 = 600e-6;
    p->efficiency = 1.0;
}
