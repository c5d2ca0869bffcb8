// batch.hip -- many independent coalescence runs ("instances") advanced by a
// single step call.  Instances are admitted into fixed-capacity pools of
// super-droplets, cells and instance records inside the caller's workspace;
// every step launches the wave-tier and workgroup-tier kernels once over the
// cells of all admitted instances (workgroup-tier cells largest first), then
// advances every instance's step counter on the device.  The launch sequence
// is captured once as a HIP graph and replayed until the set of instances
// changes.
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <map>

using namespace sdm;

namespace {

// First-fit range allocator over [0, capacity).
class RangePool {
public:
    explicit RangePool(uint64_t cap = 0) { if (cap) free_[0] = cap; }
    bool alloc(uint64_t n, uint64_t* begin)
    {
        if (n == 0) { *begin = 0; return true; }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *begin = it->first;
                const uint64_t rest = it->second - n, nb = it->first + n;
                free_.erase(it);
                if (rest) free_[nb] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t begin, uint64_t n)
    {
        if (n == 0) return;
        auto it = free_.emplace(begin, n).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t free_total() const
    {
        uint64_t t = 0;
        for (auto& kv : free_) t += kv.second;
        return t;
    }
private:
    std::map<uint64_t, uint64_t> free_;
};

struct HostInstance {
    bool live = false;
    uint64_t sd_begin = 0, n_sd = 0;
    uint64_t cell_begin = 0;
    uint32_t n_cells = 0;
    uint64_t next_step = 0;
    std::vector<uint32_t> cell_sizes;
};

__global__ void k_fill_cells(uint32_t n_cells, const uint32_t* local_off, uint32_t sd_begin,
                             uint32_t cell_begin, uint32_t inst, const double* dV_in,
                             uint32_t* cell_off, uint32_t* cell_end, double* dV, uint32_t* cell_inst,
                             uint32_t* cell_local)
{
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n_cells; c += gridDim.x * blockDim.x) {
        cell_off[cell_begin + c] = sd_begin + local_off[c];
        cell_end[cell_begin + c] = sd_begin + local_off[c + 1];
        dV[cell_begin + c] = dV_in[c];
        cell_inst[cell_begin + c] = inst;
        cell_local[cell_begin + c] = c;
    }
}

__global__ void k_advance_instances(InstanceRec* inst, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (inst[i].active) {
            inst[i].step += 1u;
            inst[i].steps_done += 1u;
        }
    }
}

struct BatchLayout {
    uint64_t* xi;
    double* r;
    uint32_t* id;
    uint32_t* cell_off;
    uint32_t* cell_end;
    double* dV;
    uint32_t* cell_inst;
    uint32_t* cell_local;
    InstanceRec* inst;
    uint32_t* group_begin;
    uint32_t* group_end;
    GridArrays grid;
    unsigned int* err;
    uint32_t* local_off;     // admission: offsets of the instance being added
    uint64_t* scr_kv;
    uint64_t* scr_tmp;
    uint32_t* scr_pos;
    uint32_t* scr_cnt;
    SortScratch sort;
    size_t bytes;
};

BatchLayout batch_layout(void* ws, size_t bytes, uint64_t max_sd, uint32_t max_cells,
                         uint32_t max_inst)
{
    Carver cv(ws, bytes);
    BatchLayout L{};
    L.xi = cv.take<uint64_t>(max_sd);
    L.r = cv.take<double>(max_sd);
    L.id = cv.take<uint32_t>(max_sd);
    L.cell_off = cv.take<uint32_t>(max_cells);
    L.cell_end = cv.take<uint32_t>(max_cells);
    L.dV = cv.take<double>(max_cells);
    L.cell_inst = cv.take<uint32_t>(max_cells);
    L.cell_local = cv.take<uint32_t>(max_cells);
    L.inst = cv.take<InstanceRec>(max_inst);
    L.group_begin = cv.take<uint32_t>(max_cells);
    L.group_end = cv.take<uint32_t>(max_cells);
    carve_grid(cv, max_sd, max_cells, &L.grid);
    L.err = cv.take<unsigned int>(64);
    L.local_off = cv.take<uint32_t>(uint64_t(max_cells) + 1);
    // step scratch and admission sort scratch share one region (admission
    // happens between steps, on the same stream)
    const uintptr_t begin = cv.cur;
    L.scr_kv = cv.take<uint64_t>(max_sd);
    L.scr_tmp = cv.take<uint64_t>(max_sd);
    L.scr_pos = cv.take<uint32_t>(max_sd);
    L.scr_cnt = cv.take<uint32_t>(max_sd + 1);
    const uintptr_t step_end = cv.cur;
    cv.cur = begin;
    carve_sort_scratch(cv, max_sd, max_cells, &L.sort);
    if (cv.cur < step_end) cv.cur = step_end;
    L.bytes = cv.used();
    return L;
}

}  // namespace

struct sdm_batch {
    hipStream_t stream = nullptr;
    uint64_t max_sd = 0;
    uint32_t max_cells = 0, max_inst = 0;
    BatchLayout L{};
    RangePool sd_pool, cell_pool;
    std::vector<HostInstance> inst;
    uint32_t n_groups = 0;
    bool dirty = true;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    LaunchShape shape;
    StreamFork fork;   // side stream of the small-instance tiers
};

static sdm_status rebuild_lists(sdm_batch* b)
{
    // groups never span two instances: each instance's cells are planned on their own
    Plan plan;
    for (const HostInstance& h : b->inst) {
        if (!h.live || h.n_cells == 0) continue;
        plan_cells(plan, static_cast<uint32_t>(h.cell_begin), h.cell_sizes.data(), h.n_cells,
                   b->shape.group_slots, b->shape.block_slots);
    }
    plan_finish(plan);
    const size_t ng = plan.group_begin.size();
    if (ng) {
        SDM_HIP(hipMemcpyAsync(b->L.group_begin, plan.group_begin.data(), ng * 4,
                               hipMemcpyHostToDevice, b->stream));
        SDM_HIP(hipMemcpyAsync(b->L.group_end, plan.group_end.data(), ng * 4, hipMemcpyHostToDevice,
                               b->stream));
    }
    SDM_TRY(upload_grid(b->stream, plan, &b->L.grid));
    SDM_HIP(hipStreamSynchronize(b->stream));
    b->n_groups = static_cast<uint32_t>(ng);
    b->dirty = true;
    return SDM_OK;
}

static sdm_status enqueue_step(sdm_batch* b)
{
    StepArgs a{};
    a.xi = b->L.xi;
    a.r = b->L.r;
    a.n_sd = b->max_sd;
    a.off_begin = b->L.cell_off;
    a.off_end = b->L.cell_end;
    a.dV = b->L.dV;
    a.cell_inst = b->L.cell_inst;
    a.cell_local = b->L.cell_local;
    a.inst = b->L.inst;
    a.scr_kv = b->L.scr_kv;
    a.scr_tmp = b->L.scr_tmp;
    a.scr_pos = b->L.scr_pos;
    a.scr_cnt = b->L.scr_cnt;
    grid_args(b->L.grid, &a);
    SDM_TRY(launch_step(b->stream, a, b->L.group_begin, b->L.group_end, b->n_groups, b->shape,
                        true, false, false, nullptr, &b->fork));
    hipLaunchKernelGGL(k_advance_instances, dim3(grid_for(b->max_inst, 256, 1024)), dim3(256), 0,
                       b->stream, b->L.inst, b->max_inst);
    SDM_LAUNCHED();
    return SDM_OK;
}

static void destroy_fork(StreamFork& f)
{
    if (f.begin) hipEventDestroy(f.begin);
    if (f.end) hipEventDestroy(f.end);
    if (f.side) {
        hipStreamSynchronize(f.side);
        hipStreamDestroy(f.side);
    }
    f = StreamFork{};
}

static void drop_graph(sdm_batch* b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

extern "C" size_t sdm_batch_workspace_bytes(uint64_t max_sd, uint32_t max_cells, uint32_t max_instances)
{
    return batch_layout(nullptr, 0, max_sd, max_cells, max_instances).bytes;
}

extern "C" sdm_status sdm_batch_create(sdm_batch** out, void* stream, void* workspace, size_t ws_bytes,
                                       uint64_t max_sd, uint32_t max_cells, uint32_t max_instances)
{
    if (!out) {
        set_error("out is NULL");
        return SDM_EINVAL;
    }
    *out = nullptr;
    if (max_sd >= (1ull << 32) || max_cells == 0 || max_instances == 0) {
        set_error("capacities: max_sd < 2^32, max_cells >= 1, max_instances >= 1");
        return SDM_EINVAL;
    }
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
        set_error("workspace must be non-NULL and 256-byte aligned");
        return SDM_EINVAL;
    }
    BatchLayout L = batch_layout(workspace, ws_bytes, max_sd, max_cells, max_instances);
    if (L.bytes > ws_bytes) {
        set_error("workspace has %zu bytes, %zu needed", ws_bytes, L.bytes);
        return SDM_ENOMEM;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // all instance records inactive
    const uint64_t words = uint64_t(max_instances) * sizeof(InstanceRec) / 8;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(words, 256, 4096)), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(L.inst), words, 0ull);
    SDM_LAUNCHED();
    SDM_HIP(hipStreamSynchronize(s));
    StreamFork fork;
    if (hipStreamCreateWithFlags(&fork.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&fork.begin, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&fork.end, hipEventDisableTiming) != hipSuccess) {
        set_error("side stream or events of the batch: %s", hipGetErrorString(hipGetLastError()));
        destroy_fork(fork);
        return SDM_EDEVICE;
    }
    auto* b = new sdm_batch();
    b->fork = fork;
    b->stream = s;
    b->max_sd = max_sd;
    b->max_cells = max_cells;
    b->max_inst = max_instances;
    b->L = L;
    b->sd_pool = RangePool(max_sd);
    b->cell_pool = RangePool(max_cells);
    b->inst.resize(max_instances);
    *out = b;
    return SDM_OK;
}

extern "C" sdm_status sdm_batch_add(sdm_batch* b, const sdm_instance_desc* d, int32_t* handle_out)
{
    if (!b || !d || !handle_out) {
        set_error("NULL argument");
        return SDM_EINVAL;
    }
    if (d->n_sd > 0 && (!d->cell || !d->xi || !d->r || d->n_cells == 0)) {
        set_error("SD arrays must be non-NULL and n_cells >= 1 when n_sd > 0");
        return SDM_EINVAL;
    }
    if (d->n_cells > 0 && !d->dV) {
        set_error("dV is NULL");
        return SDM_EINVAL;
    }
    if (d->kernel != SDM_KERNEL_GOLOVIN && d->kernel != SDM_KERNEL_GEOMETRIC) {
        set_error("unknown kernel");
        return SDM_EINVAL;
    }
    if (!(d->dt > 0.0) || !std::isfinite(d->dt) || !params_valid(d->params)) {
        set_error("dt must be finite and > 0; kernel parameters finite and non-negative");
        return SDM_EINVAL;
    }
    if (d->first_step >= (1ull << 32)) {
        set_error("first_step must be below 2^32");
        return SDM_EINVAL;
    }
    if (d->n_sd > b->max_sd || d->n_cells > b->max_cells) {
        set_error("instance larger than the batch capacity");
        return SDM_EBUDGET;
    }
    int32_t slot = -1;
    for (uint32_t i = 0; i < b->max_inst; ++i)
        if (!b->inst[i].live) { slot = static_cast<int32_t>(i); break; }
    if (slot < 0) {
        set_error("no free instance slot");
        return SDM_EBUDGET;
    }
    uint64_t sd_begin = 0, cell_begin = 0;
    if (!b->sd_pool.alloc(d->n_sd, &sd_begin)) {
        set_error("not enough free super-droplet capacity");
        return SDM_EBUDGET;
    }
    if (!b->cell_pool.alloc(d->n_cells, &cell_begin)) {
        b->sd_pool.release(sd_begin, d->n_sd);
        set_error("not enough free cell capacity");
        return SDM_EBUDGET;
    }
    hipStream_t s = b->stream;
    auto fail = [&](sdm_status st) {
        b->sd_pool.release(sd_begin, d->n_sd);
        b->cell_pool.release(cell_begin, d->n_cells);
        return st;
    };
    // stable sort by cell into the instance's pool range
    const uint32_t* order = nullptr;
    SortScratch scr = b->L.sort;
    sdm_status st = sort_by_cell(s, d->n_sd, d->cell, d->r, d->n_cells, d->dV, scr, b->L.local_off,
                                 b->L.err, &order);
    if (st != SDM_OK) return fail(st);
    if (d->n_sd > 0) {
        hipLaunchKernelGGL(k_gather_state, dim3(grid_for(d->n_sd, 256, 8192)), dim3(256), 0, s,
                           d->n_sd, order, d->xi, d->r, b->L.xi + sd_begin, b->L.r + sd_begin, 0u);
        if (hipGetLastError() != hipSuccess) return fail(SDM_EDEVICE);
        if (hipMemcpyAsync(b->L.id + sd_begin, order, d->n_sd * 4, hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
            return fail(SDM_EDEVICE);
    }
    if (d->n_cells > 0) {
        hipLaunchKernelGGL(k_fill_cells, dim3(grid_for(d->n_cells, 256, 4096)), dim3(256), 0, s,
                           d->n_cells, b->L.local_off, static_cast<uint32_t>(sd_begin),
                           static_cast<uint32_t>(cell_begin), static_cast<uint32_t>(slot), d->dV,
                           b->L.cell_off, b->L.cell_end, b->L.dV, b->L.cell_inst, b->L.cell_local);
        if (hipGetLastError() != hipSuccess) return fail(SDM_EDEVICE);
    }
    std::vector<uint32_t> off(uint64_t(d->n_cells) + 1);
    if (hipMemcpyAsync(off.data(), b->L.local_off, off.size() * 4, hipMemcpyDeviceToHost, s) !=
        hipSuccess)
        return fail(SDM_EDEVICE);
    InstanceRec rec{};
    rec.seed = d->seed;
    rec.step = d->first_step;
    rec.dt = d->dt;
    rec.kernel = static_cast<uint32_t>(d->kernel);
    rec.active = 1;
    rec.kp = to_kp(d->params);
    if (hipMemcpyAsync(b->L.inst + slot, &rec, sizeof(rec), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(SDM_EDEVICE);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(SDM_EDEVICE);

    HostInstance& h = b->inst[slot];
    h.live = true;
    h.sd_begin = sd_begin;
    h.n_sd = d->n_sd;
    h.cell_begin = cell_begin;
    h.n_cells = d->n_cells;
    h.next_step = d->first_step;
    h.cell_sizes.resize(d->n_cells);
    for (uint32_t c = 0; c < d->n_cells; ++c) h.cell_sizes[c] = off[c + 1] - off[c];
    st = rebuild_lists(b);
    if (st != SDM_OK) {
        // roll the admission back: the instance leaves no record, no pool range
        // and no work-list entry behind, and the lists are those of before
        h = HostInstance();
        InstanceRec off{};
        hipMemcpyAsync(b->L.inst + slot, &off, sizeof(off), hipMemcpyHostToDevice, s);
        fail(st);
        const sdm_status again = rebuild_lists(b);
        return again != SDM_OK ? again : st;
    }
    *handle_out = slot;
    return SDM_OK;
}

extern "C" sdm_status sdm_batch_step(sdm_batch* b, int use_graph)
{
    if (!b) {
        set_error("batch is NULL");
        return SDM_EINVAL;
    }
    for (const HostInstance& h : b->inst)
        if (h.live && h.next_step >= (1ull << 32)) {
            set_error("an instance's step number reached 2^32");
            return SDM_ESTATE;
        }
    if (use_graph) {
        if (b->dirty || !b->exec) {
            drop_graph(b);
            SDM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            sdm_status st = enqueue_step(b);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(b->stream, &g);
            if (st != SDM_OK) {
                if (g) hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess) {
                set_error("hipStreamEndCapture: %s", hipGetErrorString(e));
                return SDM_EDEVICE;
            }
            b->graph = g;
            SDM_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
            b->dirty = false;
        }
        SDM_HIP(hipGraphLaunch(b->exec, b->stream));
    } else {
        SDM_TRY(enqueue_step(b));
    }
    for (HostInstance& h : b->inst)
        if (h.live) ++h.next_step;
    return SDM_OK;
}

extern "C" sdm_status sdm_batch_get(sdm_batch* b, int32_t handle, uint64_t* xi_out, double* r_out,
                                    uint64_t* steps_done, uint64_t* pair_tests, uint64_t* collisions)
{
    if (!b || handle < 0 || static_cast<uint32_t>(handle) >= b->max_inst || !b->inst[handle].live) {
        set_error("invalid batch or handle");
        return SDM_EINVAL;
    }
    const HostInstance& h = b->inst[handle];
    hipStream_t s = b->stream;
    if (h.n_sd > 0 && (xi_out || r_out)) {
        hipLaunchKernelGGL(k_scatter_state, dim3(grid_for(h.n_sd, 256, 8192)), dim3(256), 0, s, h.n_sd,
                           b->L.id + h.sd_begin, b->L.xi + h.sd_begin, b->L.r + h.sd_begin, xi_out,
                           r_out, 0u);
        SDM_LAUNCHED();
    }
    InstanceRec rec{};
    SDM_HIP(hipMemcpyAsync(&rec, b->L.inst + handle, sizeof(rec), hipMemcpyDeviceToHost, s));
    SDM_HIP(hipStreamSynchronize(s));
    if (steps_done) *steps_done = rec.steps_done;
    if (pair_tests) *pair_tests = rec.pair_tests;
    if (collisions) *collisions = rec.collisions;
    return SDM_OK;
}

extern "C" sdm_status sdm_batch_remove(sdm_batch* b, int32_t handle, uint64_t* xi_out, double* r_out)
{
    SDM_TRY(sdm_batch_get(b, handle, xi_out, r_out, nullptr, nullptr, nullptr));
    HostInstance& h = b->inst[handle];
    InstanceRec rec{};
    SDM_HIP(hipMemcpyAsync(b->L.inst + handle, &rec, sizeof(rec), hipMemcpyHostToDevice, b->stream));
    SDM_HIP(hipStreamSynchronize(b->stream));
    b->sd_pool.release(h.sd_begin, h.n_sd);
    b->cell_pool.release(h.cell_begin, h.n_cells);
    h = HostInstance();
    return rebuild_lists(b);
}

extern "C" sdm_status sdm_batch_info(sdm_batch* b, uint32_t* n_instances, uint64_t* free_sd,
                                     uint32_t* free_cells)
{
    if (!b) {
        set_error("batch is NULL");
        return SDM_EINVAL;
    }
    uint32_t n = 0;
    for (const HostInstance& h : b->inst) n += h.live ? 1u : 0u;
    if (n_instances) *n_instances = n;
    if (free_sd) *free_sd = b->sd_pool.free_total();
    if (free_cells) *free_cells = static_cast<uint32_t>(b->cell_pool.free_total());
    return SDM_OK;
}

extern "C" sdm_status sdm_batch_get_launch_config(sdm_batch* b, sdm_launch_config* cfg)
{
    if (!b || !cfg) {
        set_error("NULL argument");
        return SDM_EINVAL;
    }
    cfg->group_slots = b->shape.group_slots;
    cfg->groups_per_wave = b->shape.groups_per_wave;
    cfg->waves_per_block = b->shape.waves_per_block;
    cfg->xcd_remap = b->shape.xcd_remap;
    cfg->block_slots = b->shape.block_slots;
    cfg->block_split = 0;
    return SDM_OK;
}

static sdm_status batch_apply_shape(sdm_batch* b, const LaunchShape& sh)
{
    const bool replan =
        sh.group_slots != b->shape.group_slots || sh.block_slots != b->shape.block_slots;
    b->shape = sh;
    b->dirty = true;   // the captured graph holds the old launches
    return replan ? rebuild_lists(b) : SDM_OK;
}

extern "C" sdm_status sdm_batch_set_launch_config(sdm_batch* b, const sdm_launch_config* cfg)
{
    if (!b || !cfg) {
        set_error("NULL argument");
        return SDM_EINVAL;
    }
    LaunchShape sh;
    sh.group_slots = cfg->group_slots;
    sh.groups_per_wave = cfg->groups_per_wave;
    sh.waves_per_block = cfg->waves_per_block;
    sh.xcd_remap = cfg->xcd_remap;
    sh.block_slots = cfg->block_slots;
    if (!shape_valid(sh) || cfg->block_split != 0) {
        set_error("launch config out of range (block_split is for single runs)");
        return SDM_EINVAL;
    }
    return batch_apply_shape(b, sh);
}

extern "C" size_t sdm_batch_autotune_workspace_bytes(sdm_batch* b)
{
    if (!b) return 0;
    Carver cv;
    cv.take<uint64_t>(b->max_sd);
    cv.take<double>(b->max_sd);
    cv.take<InstanceRec>(b->max_inst);
    return cv.used();
}

extern "C" sdm_status sdm_batch_autotune(sdm_batch* b, void* scratch, size_t scratch_bytes,
                                         uint32_t reps, sdm_launch_config* best_out)
{
    if (!b) {
        set_error("batch is NULL");
        return SDM_EINVAL;
    }
    if (!scratch || scratch_bytes < sdm_batch_autotune_workspace_bytes(b) ||
        (reinterpret_cast<uintptr_t>(scratch) & 255u)) {
        set_error("autotune scratch must be 256-byte aligned and hold %zu bytes",
                  sdm_batch_autotune_workspace_bytes(b));
        return SDM_ENOMEM;
    }
    if (reps == 0) reps = 3;
    hipStream_t s = b->stream;
    Carver cv(scratch, scratch_bytes);
    uint64_t* xi_save = cv.take<uint64_t>(b->max_sd);
    double* r_save = cv.take<double>(b->max_sd);
    InstanceRec* inst_save = cv.take<InstanceRec>(b->max_inst);
    SDM_HIP(hipMemcpyAsync(xi_save, b->L.xi, b->max_sd * 8, hipMemcpyDeviceToDevice, s));
    SDM_HIP(hipMemcpyAsync(r_save, b->L.r, b->max_sd * 8, hipMemcpyDeviceToDevice, s));
    SDM_HIP(hipMemcpyAsync(inst_save, b->L.inst, b->max_inst * sizeof(InstanceRec),
                           hipMemcpyDeviceToDevice, s));
    const LaunchShape original = b->shape;
    std::vector<LaunchShape> cands;
    for (uint32_t slots : {64u, 128u, 256u, 512u})
        for (uint32_t gpw : {1u, 2u, 4u, 8u, 16u})
            for (uint32_t wpb : {1u, 2u, 4u})
                for (uint32_t xr : {0u, 1u}) {
                    LaunchShape c = original;
                    c.group_slots = slots;
                    c.groups_per_wave = gpw;
                    c.waves_per_block = wpb;
                    c.xcd_remap = xr;
                    if (shape_valid(c)) cands.push_back(c);
                }
    const size_t n_wave_cands = cands.size();
    hipEvent_t e0, e1;
    SDM_HIP(hipEventCreate(&e0));
    SDM_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    LaunchShape best = original;
    sdm_status st = SDM_OK;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        if (ci == n_wave_cands) {   // then the workgroup-tier limit on the best of them
            for (uint32_t bs : {0u, kBlockSmall, kBlockLarge}) {
                if (bs == best.block_slots) continue;
                LaunchShape c = best;
                c.block_slots = bs;
                if (shape_valid(c)) cands.push_back(c);
            }
            if (ci == cands.size()) break;
        }
        const LaunchShape c = cands[ci];
        if ((st = batch_apply_shape(b, c)) != SDM_OK) break;
        if ((st = enqueue_step(b)) != SDM_OK) break;   // untimed
        hipEventRecord(e0, s);
        for (uint32_t i = 0; i < reps && st == SDM_OK; ++i) st = enqueue_step(b);
        if (st != SDM_OK) break;
        hipEventRecord(e1, s);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
        // every instance as it was before the candidate ran
        hipMemcpyAsync(b->L.xi, xi_save, b->max_sd * 8, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(b->L.r, r_save, b->max_sd * 8, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(b->L.inst, inst_save, b->max_inst * sizeof(InstanceRec),
                       hipMemcpyDeviceToDevice, s);
    }
    hipMemcpyAsync(b->L.xi, xi_save, b->max_sd * 8, hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(b->L.r, r_save, b->max_sd * 8, hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(b->L.inst, inst_save, b->max_inst * sizeof(InstanceRec),
                   hipMemcpyDeviceToDevice, s);
    hipStreamSynchronize(s);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    const sdm_status st2 = batch_apply_shape(b, st == SDM_OK ? best : original);
    if (st != SDM_OK) return st;
    if (st2 != SDM_OK) return st2;
    if (best_out) SDM_TRY(sdm_batch_get_launch_config(b, best_out));
    return SDM_OK;
}

extern "C" void sdm_batch_destroy(sdm_batch* b)
{
    if (!b) return;
    drop_graph(b);
    destroy_fork(b->fork);
    delete b;
}
