// context.hip -- the single-run C ABI: sdm_init / sdm_coalesce_step and the
// state, counter, layout, plan and permutation queries of a context.
#include "context.hpp"
#include "diag_kernels.hpp"
#include "recycle_kernels.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

using namespace sdm;

namespace {

struct CtxLayout {
    uint64_t* xi;
    double* r;
    uint32_t* id;
    uint32_t* offsets;
    double* dV;
    uint32_t* group_begin;
    uint32_t* group_end;
    GridArrays grid;
    unsigned long long* stats;
    unsigned int* err;
    // probe: pairing order, live counts and the running maximum of P_ij
    uint32_t* probe_order;
    double* probe_cell;
    unsigned long long* probe_max;
    uint32_t* rd_small;   // domain-wide recycling: counters and a digit histogram
    // scratch (grid-tier sort arrays during steps; sort-by-cell arrays during init)
    uint64_t* scr_kv;
    uint64_t* scr_tmp;
    uint32_t* scr_pos;
    uint32_t* scr_cnt;
    SortScratch sort;
    size_t bytes;
};

CtxLayout layout(void* ws, size_t ws_bytes, uint64_t n, uint32_t c)
{
    Carver cv(ws, ws_bytes);
    CtxLayout L{};
    L.xi = cv.take<uint64_t>(n);
    L.r = cv.take<double>(n);
    L.id = cv.take<uint32_t>(n);
    L.offsets = cv.take<uint32_t>(uint64_t(c) + 1);
    L.dV = cv.take<double>(c);
    L.group_begin = cv.take<uint32_t>(c);
    L.group_end = cv.take<uint32_t>(c);
    carve_grid(cv, n, c, &L.grid);
    L.stats = cv.take<unsigned long long>(uint64_t(kStatSlots) * kStatStride);
    L.err = cv.take<unsigned int>(64);
    L.probe_order = cv.take<uint32_t>(n);
    L.probe_cell = cv.take<double>(c);
    L.probe_max = cv.take<unsigned long long>(uint64_t(kMaxSlots) * kMaxStride);
    L.rd_small = cv.take<uint32_t>(kRecycleDomainSmall);
    // the scratch region is shared by the step scratch and the init sort
    const uintptr_t scratch_begin = cv.cur;
    L.scr_kv = cv.take<uint64_t>(n);
    L.scr_tmp = cv.take<uint64_t>(n);
    L.scr_pos = cv.take<uint32_t>(n);
    L.scr_cnt = cv.take<uint32_t>(n + 1);
    const uintptr_t step_end = cv.cur;
    cv.cur = scratch_begin;
    carve_sort_scratch(cv, n, c, &L.sort);
    if (cv.cur < step_end) cv.cur = step_end;
    L.bytes = cv.used();
    return L;
}

StepArgs base_args(const sdm_ctx* x)
{
    StepArgs a{};
    a.xi = x->xi;
    a.r = x->r;
    a.n_sd = x->n_sd;
    a.off_begin = x->offsets;
    a.off_end = x->offsets + 1;
    a.dV = x->dV;
    a.split_spin_limit = x->split_spin_limit;
    a.kp = to_kp(x->params);
    a.rules = x->rules;
    a.rd3 = x->rd3;
    a.kappa = x->kappa;
    a.stats = x->stats;
    a.scr_kv = x->scr_kv;
    a.scr_tmp = x->scr_tmp;
    a.scr_pos = x->scr_pos;
    a.scr_cnt = x->scr_cnt;
    grid_args(x->grid, &a);
    return a;
}

sdm_status check_ctx(const sdm_ctx* x)
{
    if (!x) {
        set_error("context is NULL");
        return SDM_EINVAL;
    }
    return SDM_OK;
}

// Build the work lists for the current launch shape and upload them.
sdm_status upload_plan(sdm_ctx* x)
{
    if (x->sizes_stale) {
        // the storage was re-sorted on the device since the host last saw the offsets
        std::vector<uint32_t> off(uint64_t(x->n_cells) + 1);
        SDM_HIP(hipMemcpyAsync(off.data(), x->offsets, off.size() * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, x->stream));
        SDM_HIP(hipStreamSynchronize(x->stream));
        for (uint32_t c = 0; c < x->n_cells; ++c) x->sizes[c] = off[c + 1] - off[c];
        x->sizes_stale = false;
    }
    Plan plan;
    plan_cells(plan, 0, x->sizes.data(), x->n_cells, x->shape.group_slots,
               x->shape.block_slots);
    plan_finish(plan);
    const size_t ng = plan.group_begin.size();
    if (ng) {
        SDM_HIP(hipMemcpyAsync(x->group_begin, plan.group_begin.data(), ng * 4,
                               hipMemcpyHostToDevice, x->stream));
        SDM_HIP(hipMemcpyAsync(x->group_end, plan.group_end.data(), ng * 4, hipMemcpyHostToDevice,
                               x->stream));
    }
    SDM_TRY(upload_grid(x->stream, plan, &x->grid));
    SDM_HIP(hipStreamSynchronize(x->stream));
    x->n_groups = static_cast<uint32_t>(ng);
    x->n_wave_cells = plan.wave_cells;
    return SDM_OK;
}

}  // namespace

namespace sdm {
sdm_status ctx_replan(sdm_ctx* x)
{
    return upload_plan(x);
}
}  // namespace sdm

extern "C" size_t sdm_workspace_bytes(uint64_t n_sd, uint32_t n_cells)
{
    return layout(nullptr, 0, n_sd, n_cells).bytes;
}

extern "C" sdm_status sdm_init(sdm_ctx** out, void* stream, void* workspace, size_t ws_bytes,
                               uint64_t n_sd, const uint32_t* cell, const uint64_t* xi,
                               const double* r, uint32_t n_cells, const double* dV,
                               const sdm_kernel_params* params)
{
    if (!out) {
        set_error("out is NULL");
        return SDM_EINVAL;
    }
    *out = nullptr;
    if (n_sd >= (1ull << 32)) {
        set_error("n_sd must be below 2^32");
        return SDM_EINVAL;
    }
    if (n_sd > 0 && (n_cells == 0 || !cell || !xi || !r)) {
        set_error("SD arrays must be non-NULL and n_cells >= 1 when n_sd > 0");
        return SDM_EINVAL;
    }
    if (n_cells > 0 && !dV) {
        set_error("dV is NULL");
        return SDM_EINVAL;
    }
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
        set_error("workspace must be non-NULL and 256-byte aligned");
        return SDM_EINVAL;
    }
    sdm_kernel_params kp;
    sdm_default_params(&kp);
    if (params) kp = *params;
    if (!params_valid(kp)) {
        set_error("kernel parameters must be finite, non-negative, with vt_r1 <= vt_r2");
        return SDM_EINVAL;
    }
    const CtxLayout L = layout(workspace, ws_bytes, n_sd, n_cells);
    if (L.bytes > ws_bytes) {
        set_error("workspace has %zu bytes, %zu needed", ws_bytes, L.bytes);
        return SDM_ENOMEM;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);

    const uint32_t* order = nullptr;
    SortScratch scr = L.sort;
    SDM_TRY(sort_by_cell(s, n_sd, cell, r, n_cells, dV, scr, L.offsets, L.err, &order));
    if (n_sd > 0) {
        hipLaunchKernelGGL(k_gather_state, dim3(grid_for(n_sd, 256, 8192)), dim3(256), 0, s, n_sd,
                           order, xi, r, L.xi, L.r, 0u);
        SDM_LAUNCHED();
        SDM_HIP(hipMemcpyAsync(L.id, order, n_sd * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    if (n_cells > 0)
        SDM_HIP(hipMemcpyAsync(L.dV, dV, n_cells * sizeof(double), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_fill_u64, dim3(4), dim3(256), 0, s, L.stats,
                       uint64_t(kStatSlots) * kStatStride, 0ull);
    SDM_LAUNCHED();

    std::vector<uint32_t> off(uint64_t(n_cells) + 1);
    SDM_HIP(hipMemcpyAsync(off.data(), L.offsets, off.size() * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    SDM_HIP(hipStreamSynchronize(s));

    auto* x = new sdm_ctx();
    x->stream = s;
    x->n_sd = n_sd;
    x->n_cells = n_cells;
    x->params = kp;
    x->xi = L.xi;
    x->r = L.r;
    x->id = L.id;
    x->offsets = L.offsets;
    x->dV = L.dV;
    x->group_begin = L.group_begin;
    x->group_end = L.group_end;
    x->grid = L.grid;
    x->stats = L.stats;
    x->err = L.err;
    x->probe_order = L.probe_order;
    x->probe_cell = L.probe_cell;
    x->probe_max = L.probe_max;
    x->rd_small = L.rd_small;
    x->scr_kv = L.scr_kv;
    x->scr_tmp = L.scr_tmp;
    x->scr_pos = L.scr_pos;
    x->scr_cnt = L.scr_cnt;
    x->sort = L.sort;
    x->sizes.resize(n_cells);
    for (uint32_t c = 0; c < n_cells; ++c) x->sizes[c] = off[c + 1] - off[c];
    const sdm_status st = upload_plan(x);
    if (st != SDM_OK) {
        delete x;
        return st;
    }
    *out = x;
    return SDM_OK;
}

static sdm_status step_args(sdm_ctx* x, double dt, sdm_kernel kernel, uint64_t seed,
                            uint64_t step, StepArgs* a)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) {
        set_error("dt must be finite and > 0");
        return SDM_EINVAL;
    }
    if (kernel != SDM_KERNEL_GOLOVIN && kernel != SDM_KERNEL_GEOMETRIC) {
        set_error("unknown kernel %d", static_cast<int>(kernel));
        return SDM_EINVAL;
    }
    if (step >= (1ull << 32)) {
        set_error("step must be below 2^32");
        return SDM_EINVAL;
    }
    *a = base_args(x);
    a->seed = seed;
    a->step = static_cast<uint32_t>(step);
    a->kernel = static_cast<uint32_t>(kernel);
    a->dt = dt;
    return SDM_OK;
}

static sdm_status enqueue_recycle(sdm_ctx* x)
{
    if (x->n_cells == 0) return SDM_OK;
    // the per-cell pair counts borrow the probe's per-cell scratch (8 bytes a cell)
    uint32_t* pairs = reinterpret_cast<uint32_t*>(x->probe_cell);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(x->n_cells, 256, 8192)), dim3(256), 0, x->stream,
                       pairs, uint64_t(x->n_cells), 0u);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_recycle, dim3(grid_for(x->n_cells, kRecycleCellsPerBlock, 1u << 16)),
                       dim3(kRecycleBlock), 0, x->stream, x->offsets, x->xi, x->r, x->n_cells,
                       x->probe_order, pairs, x->stats, x->rd3, x->kappa);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_recycle_copy, dim3(grid_for(x->n_cells, 256, 8192)), dim3(256), 0,
                       x->stream, x->offsets, pairs, x->probe_order, x->n_cells, x->r, x->rd3,
                       x->kappa);
    SDM_LAUNCHED();
    return SDM_OK;
}

static sdm_status launch(sdm_ctx* x, const StepArgs& a, bool perm)
{
    // a split-tier step counts itself in once its kernel is enqueued: the
    // device counters then grow by 2^block_split per cell
    StepArgs b = a;
    const bool split = !perm && x->shape.block_split > 0 && x->grid.n_block > 0;
    if (split) b.split_epoch = x->grid.split_epoch + 1;
    bool enqueued = false;
    const sdm_status st = launch_step(x->stream, b, x->group_begin, x->group_end, x->n_groups,
                                      x->shape, false, perm, false, &enqueued);
    if (split && enqueued) x->grid.split_epoch = b.split_epoch;
    return st;
}

extern "C" sdm_status sdm_coalesce_step(sdm_ctx* x, double dt, sdm_kernel kernel, uint64_t seed,
                                        uint64_t step)
{
    SDM_TRY(check_ctx(x));
    StepArgs a;
    SDM_TRY(step_args(x, dt, kernel, seed, step, &a));
    if (x->rules & kRuleRecycle) SDM_TRY(enqueue_recycle(x));
    if (x->rules & kRuleRecycleDomain) {
        // the re-sort moves the storage: take the arguments again
        SDM_TRY(recycle_domain(x));
        SDM_TRY(step_args(x, dt, kernel, seed, step, &a));
    }
    return launch(x, a, false);
}

extern "C" sdm_status sdm_debug_split_wait(sdm_ctx* x, uint32_t spin_limit, uint32_t epoch_skew)
{
    SDM_TRY(check_ctx(x));
    x->split_spin_limit = spin_limit;
    x->grid.split_epoch += epoch_skew;
    return SDM_OK;
}

extern "C" sdm_status sdm_debug_permutation(sdm_ctx* x, uint64_t seed, uint64_t step,
                                            uint32_t* order_out, uint32_t* n_live_out)
{
    SDM_TRY(check_ctx(x));
    if ((x->n_sd > 0 && !order_out) || (x->n_cells > 0 && !n_live_out)) {
        set_error("output arrays must be non-NULL");
        return SDM_EINVAL;
    }
    StepArgs a;
    SDM_TRY(step_args(x, 1.0, SDM_KERNEL_GOLOVIN, seed, step, &a));
    a.perm_out = order_out;
    a.nlive_out = n_live_out;
    SDM_TRY(launch(x, a, true));
    SDM_HIP(hipStreamSynchronize(x->stream));
    return SDM_OK;
}

// ---------------------------------------------------------------------------
// Diagnostics, probability probe and sub-stepping
// ---------------------------------------------------------------------------
// Number of equal sub-steps that brings the probed largest P_ij down to
// p_limit: ceil(pmax / p_limit), at least 1 and at most max_substeps.
static uint32_t substep_count(double pmax, double p_limit, uint32_t max_substeps)
{
    if (!(pmax > p_limit)) return 1;
    const double q = std::ceil(pmax / p_limit);
    return q >= static_cast<double>(max_substeps) ? max_substeps : static_cast<uint32_t>(q);
}

// One wavefront per cell, as many as there are cells (up to 2^20 workgroups),
// so that every cell's loads are in flight at once.
static uint32_t diag_grid(uint32_t n_cells)
{
    return grid_for(n_cells, kDiagCellsPerBlock, kDiagMaxBlocks);
}

extern "C" sdm_status sdm_diag_sd_conc(sdm_ctx* x, uint32_t* out)
{
    SDM_TRY(check_ctx(x));
    if (x->n_cells == 0) return SDM_OK;
    if (!out) {
        set_error("out must be non-NULL");
        return SDM_EINVAL;
    }
    hipLaunchKernelGGL(k_sd_conc, dim3(diag_grid(x->n_cells)), dim3(kDiagBlock), 0, x->stream,
                       x->offsets, x->xi, x->n_cells, out);
    SDM_LAUNCHED();
    return SDM_OK;
}

extern "C" sdm_status sdm_diag_moments(sdm_ctx* x, uint32_t k, double r_min, double r_max,
                                       const double* rho_d, double* out)
{
    SDM_TRY(check_ctx(x));
    if (k > kMaxMomentOrder) {
        set_error("moment order %u above %u", k, kMaxMomentOrder);
        return SDM_EINVAL;
    }
    if (std::isnan(r_min) || std::isnan(r_max)) {
        set_error("radius range bounds must not be NaN");
        return SDM_EINVAL;
    }
    if (x->n_cells == 0) return SDM_OK;
    if (!out) {
        set_error("out must be non-NULL");
        return SDM_EINVAL;
    }
    hipLaunchKernelGGL(k_moments<false>, dim3(diag_grid(x->n_cells)), dim3(kDiagBlock), 0, x->stream,
                       x->offsets, x->dV, x->xi, x->r, x->n_cells, k, r_min, r_max, rho_d, out);
    SDM_LAUNCHED();
    return SDM_OK;
}

// Enqueue the probe of step `step`: the probe mode of the step kernels writes the
// largest P_ij of every cell (into cell_max, or the context's scratch), then one
// reduction puts the overall maximum into x->probe_max.
static sdm_status enqueue_probe(sdm_ctx* x, double dt, sdm_kernel kernel, uint64_t seed,
                                uint64_t step, double* cell_max)
{
    StepArgs a;
    SDM_TRY(step_args(x, dt, kernel, seed, step, &a));
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, x->stream, x->probe_max,
                       uint64_t(kMaxSlots) * kMaxStride, 0ull);
    SDM_LAUNCHED();
    if (x->n_cells == 0) return SDM_OK;
    double* cm = cell_max ? cell_max : x->probe_cell;
    // grid-tier cells take atomic maxima: every entry starts at +0.0
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(x->n_cells, 256, 4096)), dim3(256), 0,
                       x->stream, reinterpret_cast<unsigned long long*>(cm),
                       uint64_t(x->n_cells), 0ull);
    SDM_LAUNCHED();
    a.cell_max = cm;
    a.stats = nullptr;
    SDM_TRY(launch_step(x->stream, a, x->group_begin, x->group_end, x->n_groups, x->shape, false,
                        false, true));
    hipLaunchKernelGGL(k_max_reduce, dim3(grid_for(x->n_cells, kDiagBlock, 1024)),
                       dim3(kDiagBlock), 0, x->stream, cm, x->n_cells, x->probe_max);
    SDM_LAUNCHED();
    return SDM_OK;
}

static sdm_status read_probe_max(sdm_ctx* x, double* out)
{
    unsigned long long h[kMaxSlots * kMaxStride];
    SDM_HIP(hipMemcpyAsync(h, x->probe_max, sizeof(h), hipMemcpyDeviceToHost, x->stream));
    SDM_HIP(hipStreamSynchronize(x->stream));
    unsigned long long bits = 0;   // bit patterns of non-negative doubles order like the values
    for (uint32_t i = 0; i < kMaxSlots; ++i) bits = std::max(bits, h[i * kMaxStride]);
    double v;
    std::memcpy(&v, &bits, sizeof(v));
    *out = v;
    return SDM_OK;
}

extern "C" sdm_status sdm_probe_probability(sdm_ctx* x, double dt, sdm_kernel kernel,
                                            uint64_t seed, uint64_t step, double* cell_max,
                                            double* max_out)
{
    SDM_TRY(check_ctx(x));
    SDM_TRY(enqueue_probe(x, dt, kernel, seed, step, cell_max));
    if (max_out) SDM_TRY(read_probe_max(x, max_out));
    return SDM_OK;
}

// n sub-steps of dt / n; the first one recycles only if recycle_first is set
// (the adaptive path has recycled already, before probing).
static sdm_status run_substeps(sdm_ctx* x, double dt, uint32_t n_substeps, sdm_kernel kernel,
                               uint64_t seed, uint64_t first_step, bool recycle_first)
{
    if (n_substeps == 0) {
        set_error("n_substeps must be >= 1");
        return SDM_EINVAL;
    }
    if (first_step >= (1ull << 32) || first_step + n_substeps > (1ull << 32)) {
        set_error("step counters must stay below 2^32");
        return SDM_EINVAL;
    }
    const double h = dt / static_cast<double>(n_substeps);
    StepArgs a;
    SDM_TRY(step_args(x, h, kernel, seed, first_step, &a));   // validates before any launch
    for (uint32_t i = 0; i < n_substeps; ++i) {
        if (i > 0 || recycle_first) {
            if (x->rules & kRuleRecycle) SDM_TRY(enqueue_recycle(x));
            if (x->rules & kRuleRecycleDomain) SDM_TRY(recycle_domain(x));
        }
        SDM_TRY(step_args(x, h, kernel, seed, first_step + i, &a));
        SDM_TRY(launch(x, a, false));
    }
    return SDM_OK;
}

extern "C" sdm_status sdm_coalesce_substeps(sdm_ctx* x, double dt, uint32_t n_substeps,
                                            sdm_kernel kernel, uint64_t seed, uint64_t first_step)
{
    SDM_TRY(check_ctx(x));
    return run_substeps(x, dt, n_substeps, kernel, seed, first_step, true);
}

extern "C" sdm_status sdm_coalesce_adaptive(sdm_ctx* x, double dt, double p_limit,
                                            uint32_t max_substeps, sdm_kernel kernel,
                                            uint64_t seed, uint64_t first_step,
                                            uint32_t* substeps_out)
{
    SDM_TRY(check_ctx(x));
    if (!(p_limit > 0.0) || !std::isfinite(p_limit) || max_substeps == 0) {
        set_error("p_limit must be finite and > 0 and max_substeps >= 1");
        return SDM_EINVAL;
    }
    if (first_step >= (1ull << 32) || first_step + max_substeps > (1ull << 32)) {
        set_error("step counters must stay below 2^32");
        return SDM_EINVAL;
    }
    StepArgs a;
    SDM_TRY(step_args(x, dt, kernel, seed, first_step, &a));   // validates before any launch
    // recycle first, so that the probed pairing is the one the first sub-step uses
    if (x->rules & kRuleRecycle) SDM_TRY(enqueue_recycle(x));
    if (x->rules & kRuleRecycleDomain) SDM_TRY(recycle_domain(x));
    double pmax = 0.0;
    SDM_TRY(enqueue_probe(x, dt, kernel, seed, first_step, nullptr));
    SDM_TRY(read_probe_max(x, &pmax));
    const uint32_t n = substep_count(pmax, p_limit, max_substeps);
    SDM_TRY(run_substeps(x, dt, n, kernel, seed, first_step, false));
    if (substeps_out) *substeps_out = n;
    return SDM_OK;
}

extern "C" sdm_status sdm_set_rules(sdm_ctx* x, uint32_t rules)
{
    SDM_TRY(check_ctx(x));
    if (rules & ~static_cast<uint32_t>(SDM_RULE_RELEASE | SDM_RULE_RECYCLE |
                                       SDM_RULE_RECYCLE_DOMAIN)) {
        set_error("unknown rule flags 0x%x", rules);
        return SDM_EINVAL;
    }
    if ((rules & SDM_RULE_RECYCLE) && (rules & SDM_RULE_RECYCLE_DOMAIN)) {
        set_error("recycling runs within cells or over the domain, not both");
        return SDM_EINVAL;
    }
    if ((rules & SDM_RULE_RECYCLE_DOMAIN) && x->n_cells > 1 && !x->transport) {
        set_error("domain-wide recycling of several cells needs positions (sdm_transport_attach)");
        return SDM_ESTATE;
    }
    x->rules = rules;
    return SDM_OK;
}

extern "C" sdm_status sdm_get_rules(sdm_ctx* x, uint32_t* rules)
{
    SDM_TRY(check_ctx(x));
    if (!rules) {
        set_error("rules is NULL");
        return SDM_EINVAL;
    }
    *rules = x->rules;
    return SDM_OK;
}

extern "C" sdm_status sdm_recycle(sdm_ctx* x)
{
    SDM_TRY(check_ctx(x));
    return enqueue_recycle(x);
}

extern "C" sdm_status sdm_get_recycled(sdm_ctx* x, uint64_t* total)
{
    SDM_TRY(check_ctx(x));
    if (!total) {
        set_error("total is NULL");
        return SDM_EINVAL;
    }
    // the recycled-slot word of every counter slot
    std::vector<unsigned long long> h(uint64_t(kStatSlots) * kStatStride);
    SDM_HIP(hipMemcpyAsync(h.data(), x->stats, h.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, x->stream));
    SDM_HIP(hipStreamSynchronize(x->stream));
    uint64_t v = 0;
    for (int i = 0; i < kStatSlots; ++i) v += h[uint64_t(i) * kStatStride + kRecycledStat];
    *total = v;
    return SDM_OK;
}

extern "C" sdm_status sdm_get_state(sdm_ctx* x, uint64_t* xi_out, double* r_out)
{
    SDM_TRY(check_ctx(x));
    if (x->n_sd > 0 && (xi_out || r_out)) {
        hipLaunchKernelGGL(k_scatter_state, dim3(grid_for(x->n_sd, 256, 8192)), dim3(256), 0,
                           x->stream, x->n_sd, x->id, x->xi, x->r, xi_out, r_out, 0u);
        SDM_LAUNCHED();
    }
    SDM_HIP(hipStreamSynchronize(x->stream));
    return SDM_OK;
}

extern "C" sdm_status sdm_get_stats(sdm_ctx* x, uint64_t* pair_tests, uint64_t* collisions)
{
    SDM_TRY(check_ctx(x));
    std::vector<unsigned long long> h(uint64_t(kStatSlots) * kStatStride);
    SDM_HIP(hipMemcpyAsync(h.data(), x->stats, h.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, x->stream));
    SDM_HIP(hipStreamSynchronize(x->stream));
    uint64_t p = 0, c = 0;
    for (int i = 0; i < kStatSlots; ++i) {
        p += h[uint64_t(i) * kStatStride];
        c += h[uint64_t(i) * kStatStride + 1];
    }
    if (pair_tests) *pair_tests = p;
    if (collisions) *collisions = c;
    if (h[kSplitTimeoutStat] != 0) {
        set_error("%llu split-tier steps timed out waiting for their cell's workgroups; "
                  "their results are not reliable", h[kSplitTimeoutStat]);
        return SDM_EDEVICE;
    }
    return SDM_OK;
}

extern "C" sdm_status sdm_get_layout(sdm_ctx* x, const uint32_t** offsets,
                                     const uint32_t** input_index)
{
    SDM_TRY(check_ctx(x));
    if (offsets) *offsets = x->offsets;
    if (input_index) *input_index = x->id;
    return SDM_OK;
}

extern "C" sdm_status sdm_get_plan(sdm_ctx* x, uint32_t* groups, uint32_t* wave_cells,
                                   uint32_t* block_cells, uint32_t* grid_cells)
{
    SDM_TRY(check_ctx(x));
    if (groups) *groups = x->n_groups;
    if (wave_cells) *wave_cells = x->n_wave_cells;
    if (block_cells) *block_cells = x->grid.n_block;
    if (grid_cells) *grid_cells = x->grid.n_grid;
    return SDM_OK;
}

static LaunchShape from_cfg(const sdm_launch_config& c)
{
    LaunchShape s;
    s.group_slots = c.group_slots;
    s.groups_per_wave = c.groups_per_wave;
    s.waves_per_block = c.waves_per_block;
    s.xcd_remap = c.xcd_remap;
    s.block_slots = c.block_slots;
    s.block_split = c.block_split;
    return s;
}

static void to_cfg(const LaunchShape& s, sdm_launch_config* c)
{
    c->group_slots = s.group_slots;
    c->groups_per_wave = s.groups_per_wave;
    c->waves_per_block = s.waves_per_block;
    c->xcd_remap = s.xcd_remap;
    c->block_slots = s.block_slots;
    c->block_split = s.block_split;
}

static sdm_status apply_shape(sdm_ctx* x, const LaunchShape& sh)
{
    const bool replan =
        sh.group_slots != x->shape.group_slots || sh.block_slots != x->shape.block_slots;
    x->shape = sh;
    return replan ? upload_plan(x) : SDM_OK;
}

extern "C" sdm_status sdm_get_launch_config(sdm_ctx* x, sdm_launch_config* cfg)
{
    SDM_TRY(check_ctx(x));
    if (!cfg) {
        set_error("cfg is NULL");
        return SDM_EINVAL;
    }
    to_cfg(x->shape, cfg);
    return SDM_OK;
}

extern "C" sdm_status sdm_set_launch_config(sdm_ctx* x, const sdm_launch_config* cfg)
{
    SDM_TRY(check_ctx(x));
    if (!cfg || !shape_valid(from_cfg(*cfg))) {
        set_error("launch config out of range");
        return SDM_EINVAL;
    }
    return apply_shape(x, from_cfg(*cfg));
}

// ---------------------------------------------------------------- autotune
extern "C" size_t sdm_autotune_workspace_bytes(sdm_ctx* x)
{
    if (!x) return 0;
    Carver cv;
    cv.take<uint64_t>(x->n_sd);
    cv.take<double>(x->n_sd);
    cv.take<unsigned long long>(uint64_t(kStatSlots) * kStatStride);
    if (x->rd3) {   // the dry attributes change in the candidate steps as well
        cv.take<double>(x->n_sd);
        cv.take<double>(x->n_sd);
    }
    return cv.used();
}

extern "C" sdm_status sdm_autotune(sdm_ctx* x, void* scratch, size_t scratch_bytes, double dt,
                                   sdm_kernel kernel, uint64_t seed, uint32_t reps,
                                   sdm_launch_config* best_out)
{
    SDM_TRY(check_ctx(x));
    if (!scratch || scratch_bytes < sdm_autotune_workspace_bytes(x) ||
        (reinterpret_cast<uintptr_t>(scratch) & 255u)) {
        set_error("autotune scratch must be 256-byte aligned and hold %zu bytes",
                  sdm_autotune_workspace_bytes(x));
        return SDM_ENOMEM;
    }
    if (reps == 0) reps = 3;
    StepArgs probe;
    SDM_TRY(step_args(x, dt, kernel, seed, 0, &probe));
    Carver cv(scratch, scratch_bytes);
    uint64_t* xi_save = cv.take<uint64_t>(x->n_sd);
    double* r_save = cv.take<double>(x->n_sd);
    unsigned long long* st_save = cv.take<unsigned long long>(uint64_t(kStatSlots) * kStatStride);
    double* rd3_save = x->rd3 ? cv.take<double>(x->n_sd) : nullptr;
    double* kappa_save = x->rd3 ? cv.take<double>(x->n_sd) : nullptr;
    hipStream_t s = x->stream;
    SDM_HIP(hipMemcpyAsync(xi_save, x->xi, x->n_sd * 8, hipMemcpyDeviceToDevice, s));
    SDM_HIP(hipMemcpyAsync(r_save, x->r, x->n_sd * 8, hipMemcpyDeviceToDevice, s));
    if (x->rd3) {
        SDM_HIP(hipMemcpyAsync(rd3_save, x->rd3, x->n_sd * 8, hipMemcpyDeviceToDevice, s));
        SDM_HIP(hipMemcpyAsync(kappa_save, x->kappa, x->n_sd * 8, hipMemcpyDeviceToDevice, s));
    }
    SDM_HIP(hipMemcpyAsync(st_save, x->stats, uint64_t(kStatSlots) * kStatStride * 8,
                           hipMemcpyDeviceToDevice, s));

    // the candidates step without domain-wide recycling: it would re-sort the
    // storage, which the saved state does not restore
    const uint32_t rules_saved = x->rules;
    x->rules &= ~static_cast<uint32_t>(kRuleRecycleDomain);
    const LaunchShape original = x->shape;
    std::vector<LaunchShape> cands;
    for (uint32_t slots : {64u, 128u, 256u, 512u})
        for (uint32_t gpw : {1u, 2u, 4u, 8u, 12u, 16u})
            for (uint32_t wpb : {1u, 2u, 4u})
                for (uint32_t xr : {0u, 1u}) {
                    LaunchShape c = original;
                    c.group_slots = slots;
                    c.groups_per_wave = gpw;
                    c.waves_per_block = wpb;
                    c.xcd_remap = xr;
                    if (shape_valid(c)) cands.push_back(c);
                }
    // the wavefront-tier shapes first; then the workgroup-tier limit on the best
    // of them, then the split of its cells over several workgroups
    const size_t n_wave_cands = cands.size();
    size_t n_block_cands = 0;
    hipEvent_t e0, e1;
    SDM_HIP(hipEventCreate(&e0));
    SDM_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    LaunchShape best = original;
    sdm_status st = SDM_OK;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        if (ci == n_wave_cands) {
            for (uint32_t bs : {0u, kBlockSmall, kBlockLarge}) {
                if (bs == best.block_slots) continue;
                LaunchShape c = best;
                c.block_slots = bs;
                c.block_split = 0;
                if (shape_valid(c)) cands.push_back(c);
            }
            n_block_cands = cands.size();
            if (ci == cands.size()) break;
        }
        if (ci == n_block_cands && x->grid.n_block > 0) {
            for (uint32_t lg = 0; lg <= kSplitMaxLg; ++lg) {
                if (lg == best.block_split) continue;
                LaunchShape c = best;
                c.block_split = lg;
                if (shape_valid(c)) cands.push_back(c);
            }
            if (ci == cands.size()) break;
        }
        const LaunchShape c = cands[ci];
        if ((st = apply_shape(x, c)) != SDM_OK) break;
        // one untimed step, then reps timed ones
        if ((st = sdm_coalesce_step(x, dt, kernel, seed, 0)) != SDM_OK) break;
        hipEventRecord(e0, s);
        for (uint32_t i = 0; i < reps && st == SDM_OK; ++i)
            st = sdm_coalesce_step(x, dt, kernel, seed, 1u + i);
        if (st != SDM_OK) break;
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        // the state must be what it was before the candidate ran
        hipMemcpyAsync(x->xi, xi_save, x->n_sd * 8, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(x->r, r_save, x->n_sd * 8, hipMemcpyDeviceToDevice, s);
        if (x->rd3) {
            hipMemcpyAsync(x->rd3, rd3_save, x->n_sd * 8, hipMemcpyDeviceToDevice, s);
            hipMemcpyAsync(x->kappa, kappa_save, x->n_sd * 8, hipMemcpyDeviceToDevice, s);
        }
    }
    hipMemcpyAsync(x->stats, st_save, uint64_t(kStatSlots) * kStatStride * 8,
                   hipMemcpyDeviceToDevice, s);
    hipStreamSynchronize(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    x->rules = rules_saved;
    const sdm_status st2 = apply_shape(x, st == SDM_OK ? best : original);
    if (st != SDM_OK) return st;
    if (st2 != SDM_OK) return st2;
    if (best_out) to_cfg(best, best_out);
    return SDM_OK;
}

extern "C" void sdm_destroy(sdm_ctx* x) { delete x; }
