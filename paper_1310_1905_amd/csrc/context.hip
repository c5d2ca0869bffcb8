// context.hip -- the single-run C ABI: sdm_init / sdm_coalesce_step and the
// state, counter, layout and permutation queries of a context.
#include "runtime.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>

using namespace sdm;

struct sdm_ctx {
    hipStream_t stream = nullptr;
    uint64_t n_sd = 0;
    uint32_t n_cells = 0;
    sdm_kernel_params params{};
    // device arrays (inside the caller's workspace)
    uint64_t* xi = nullptr;
    double* r = nullptr;
    uint32_t* id = nullptr;
    uint32_t* offsets = nullptr;
    double* dV = nullptr;
    uint32_t* wave_items = nullptr;
    uint32_t* block_items = nullptr;
    unsigned long long* stats = nullptr;
    unsigned int* err = nullptr;
    uint64_t* scr_kv = nullptr;
    uint64_t* scr_tmp = nullptr;
    uint32_t* scr_pos = nullptr;
    uint32_t* scr_cnt = nullptr;
    // plan
    uint32_t n_wave = 0, n_block = 0;
    bool wave_identity = false;
    LaunchShape shape;
};

namespace {

struct CtxLayout {
    uint64_t* xi;
    double* r;
    uint32_t* id;
    uint32_t* offsets;
    double* dV;
    uint32_t* wave_items;
    uint32_t* block_items;
    unsigned long long* stats;
    unsigned int* err;
    // scratch (block-tier sort arrays during steps; sort-by-cell arrays during init)
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
    L.wave_items = cv.take<uint32_t>(c);
    L.block_items = cv.take<uint32_t>(c);
    L.stats = cv.take<unsigned long long>(uint64_t(kStatSlots) * kStatStride);
    L.err = cv.take<unsigned int>(64);
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
    a.off_begin = x->offsets;
    a.off_end = x->offsets + 1;
    a.dV = x->dV;
    a.kp = to_kp(x->params);
    a.stats = x->stats;
    a.scr_kv = x->scr_kv;
    a.scr_tmp = x->scr_tmp;
    a.scr_pos = x->scr_pos;
    a.scr_cnt = x->scr_cnt;
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

}  // namespace

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

    // plan: cells up to kWaveMaxSlots slots go to the wave tier, larger ones
    // to the workgroup tier
    std::vector<uint32_t> off(uint64_t(n_cells) + 1);
    SDM_HIP(hipMemcpyAsync(off.data(), L.offsets, off.size() * sizeof(uint32_t),
                           hipMemcpyDeviceToHost, s));
    SDM_HIP(hipStreamSynchronize(s));
    std::vector<uint32_t> wave, block;
    for (uint32_t c = 0; c < n_cells; ++c) {
        const uint32_t cnt = off[c + 1] - off[c];
        if (cnt <= static_cast<uint32_t>(kWaveMaxSlots)) wave.push_back(c);
        else block.push_back(c);
    }
    // larger cells first
    std::stable_sort(block.begin(), block.end(), [&](uint32_t a, uint32_t b) {
        return off[a + 1] - off[a] > off[b + 1] - off[b];
    });
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
    x->wave_items = L.wave_items;
    x->block_items = L.block_items;
    x->stats = L.stats;
    x->err = L.err;
    x->scr_kv = L.scr_kv;
    x->scr_tmp = L.scr_tmp;
    x->scr_pos = L.scr_pos;
    x->scr_cnt = L.scr_cnt;
    x->n_wave = static_cast<uint32_t>(wave.size());
    x->n_block = static_cast<uint32_t>(block.size());
    x->wave_identity = (wave.size() == n_cells);
    if (!x->wave_identity && !wave.empty()) {
        hipError_t e = hipMemcpyAsync(L.wave_items, wave.data(), wave.size() * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            delete x;
            set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
            return SDM_EDEVICE;
        }
    }
    if (!block.empty()) {
        hipError_t e = hipMemcpyAsync(L.block_items, block.data(), block.size() * sizeof(uint32_t),
                                      hipMemcpyHostToDevice, s);
        if (e != hipSuccess) {
            delete x;
            set_error("hipMemcpyAsync: %s", hipGetErrorString(e));
            return SDM_EDEVICE;
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete x;
        set_error("hipStreamSynchronize: %s", hipGetErrorString(e));
        return SDM_EDEVICE;
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

extern "C" sdm_status sdm_coalesce_step(sdm_ctx* x, double dt, sdm_kernel kernel, uint64_t seed,
                                        uint64_t step)
{
    SDM_TRY(check_ctx(x));
    StepArgs a;
    SDM_TRY(step_args(x, dt, kernel, seed, step, &a));
    return launch_step(x->stream, a, x->wave_identity ? nullptr : x->wave_items, x->n_wave,
                       x->block_items, x->n_block, x->shape, false, false);
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
    SDM_TRY(launch_step(x->stream, a, x->wave_identity ? nullptr : x->wave_items, x->n_wave,
                        x->block_items, x->n_block, x->shape, false, true));
    SDM_HIP(hipStreamSynchronize(x->stream));
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

extern "C" sdm_status sdm_get_plan(sdm_ctx* x, uint32_t* wave_cells, uint32_t* block_cells)
{
    SDM_TRY(check_ctx(x));
    if (wave_cells) *wave_cells = x->n_wave;
    if (block_cells) *block_cells = x->n_block;
    return SDM_OK;
}

static bool shape_valid(const sdm_launch_config& c)
{
    const bool waves_ok = c.waves_per_block == 1 || c.waves_per_block == 2 ||
                          c.waves_per_block == 4 || c.waves_per_block == 8;
    const bool block_ok = c.block_threads == 256 || c.block_threads == 1024;
    return waves_ok && block_ok && c.cells_per_wave >= 1 && c.cells_per_wave <= 64 &&
           c.xcd_remap <= 1;
}

extern "C" sdm_status sdm_get_launch_config(sdm_ctx* x, sdm_launch_config* cfg)
{
    SDM_TRY(check_ctx(x));
    if (!cfg) {
        set_error("cfg is NULL");
        return SDM_EINVAL;
    }
    cfg->cells_per_wave = x->shape.cells_per_wave;
    cfg->waves_per_block = x->shape.waves_per_block;
    cfg->block_threads = x->shape.block_threads;
    cfg->xcd_remap = x->shape.xcd_remap;
    return SDM_OK;
}

extern "C" sdm_status sdm_set_launch_config(sdm_ctx* x, const sdm_launch_config* cfg)
{
    SDM_TRY(check_ctx(x));
    if (!cfg || !shape_valid(*cfg)) {
        set_error("launch config out of range");
        return SDM_EINVAL;
    }
    x->shape.cells_per_wave = cfg->cells_per_wave;
    x->shape.waves_per_block = cfg->waves_per_block;
    x->shape.block_threads = cfg->block_threads;
    x->shape.xcd_remap = cfg->xcd_remap;
    return SDM_OK;
}

// ---------------------------------------------------------------- autotune
extern "C" size_t sdm_autotune_workspace_bytes(sdm_ctx* x)
{
    if (!x) return 0;
    Carver cv;
    cv.take<uint64_t>(x->n_sd);
    cv.take<double>(x->n_sd);
    cv.take<unsigned long long>(uint64_t(kStatSlots) * kStatStride);
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
    hipStream_t s = x->stream;
    SDM_HIP(hipMemcpyAsync(xi_save, x->xi, x->n_sd * 8, hipMemcpyDeviceToDevice, s));
    SDM_HIP(hipMemcpyAsync(r_save, x->r, x->n_sd * 8, hipMemcpyDeviceToDevice, s));
    SDM_HIP(hipMemcpyAsync(st_save, x->stats, uint64_t(kStatSlots) * kStatStride * 8,
                           hipMemcpyDeviceToDevice, s));

    const LaunchShape original = x->shape;
    std::vector<LaunchShape> cands;
    for (uint32_t cpw : {1u, 2u, 4u, 8u, 16u})
        for (uint32_t wpb : {1u, 2u, 4u, 8u})
            for (uint32_t xr : {0u, 1u}) {
                LaunchShape c = original;
                c.cells_per_wave = cpw;
                c.waves_per_block = wpb;
                c.xcd_remap = xr;
                cands.push_back(c);
            }
    if (x->n_block > 0)
        for (uint32_t bt : {256u, 1024u}) {
            LaunchShape c = original;
            c.block_threads = bt;
            cands.push_back(c);
        }
    hipEvent_t e0, e1;
    SDM_HIP(hipEventCreate(&e0));
    SDM_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    LaunchShape best = original;
    sdm_status st = SDM_OK;
    for (const LaunchShape& c : cands) {
        x->shape = c;
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
    }
    hipMemcpyAsync(x->stats, st_save, uint64_t(kStatSlots) * kStatStride * 8,
                   hipMemcpyDeviceToDevice, s);
    hipStreamSynchronize(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    x->shape = (st == SDM_OK) ? best : original;
    if (st != SDM_OK) return st;
    if (best_out) {
        best_out->cells_per_wave = best.cells_per_wave;
        best_out->waves_per_block = best.waves_per_block;
        best_out->block_threads = best.block_threads;
        best_out->xcd_remap = best.xcd_remap;
    }
    return SDM_OK;
}

extern "C" void sdm_destroy(sdm_ctx* x) { delete x; }
