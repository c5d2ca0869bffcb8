// static_step.hip -- one coalescence step over super-droplets the caller keeps
// sorted by cell, with every piece of scratch (launch plan, counters, flags)
// in a fixed-size device array of the library: no device memory is allocated
// or freed, and no workspace is passed in.
#include "runtime.hpp"

#include <cmath>
#include <mutex>

using namespace sdm;

namespace {

constexpr size_t kStaticScratchBytes = size_t(16) << 20;
constexpr uint32_t kStaticMaxCells = 1u << 20;
constexpr int kMaxDevices = 64;

// One copy per device the library runs on, held until the process ends.  In
// host code this name is only a stand-in: kernels get the address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
sdm_status scratch_address(void** out)
{
    int dev = -1;
    SDM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d is beyond the %d devices the static scratch tracks", dev, kMaxDevices);
        return SDM_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SDM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned NULL for the static scratch");
            return SDM_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SDM_OK;
}

struct StaticLayout {
    uint32_t* group_begin;
    uint32_t* group_end;
    DevicePlanArrays plan;
    unsigned long long* stats;   // kStatSlots x kStatStride counters
    unsigned long long* totals;  // their sums: pair tests, collisions
    unsigned int* err;
    size_t bytes;
};

StaticLayout static_layout(void* base, uint32_t nc)
{
    Carver cv(base, kStaticScratchBytes);
    StaticLayout L{};
    L.group_begin = cv.take<uint32_t>(nc);
    L.group_end = cv.take<uint32_t>(nc);
    carve_device_plan(cv, nc, &L.plan);
    L.stats = cv.take<unsigned long long>(uint64_t(kStatSlots) * kStatStride);
    L.totals = cv.take<unsigned long long>(2);
    L.err = cv.take<unsigned int>(64);
    L.bytes = cv.used();
    return L;
}

constexpr unsigned int kStaticBadOffsets = 1u;
constexpr unsigned int kStaticBadVolume = 2u;

// offsets[0] = 0, offsets[nc] = n_sd, non-decreasing; every dV finite and > 0.
__global__ void k_static_check(uint32_t nc, uint64_t n_sd, const uint32_t* __restrict__ off,
                               const double* __restrict__ dV, unsigned int* __restrict__ err)
{
    unsigned int bad = 0;
    for (uint64_t c = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; c < nc;
         c += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        if (off[c + 1] < off[c]) bad |= kStaticBadOffsets;
        if (c == 0 && off[0] != 0u) bad |= kStaticBadOffsets;
        if (c + 1 == nc && static_cast<uint64_t>(off[nc]) != n_sd) bad |= kStaticBadOffsets;
        const double v = dV[c];
        if (!(v > 0.0) || !(v < __builtin_inf())) bad |= kStaticBadVolume;
    }
    if (bad) atomicOr(err, bad);
}

// totals[0..1] = sums of the spread counters
__global__ void k_static_totals(const unsigned long long* __restrict__ stats,
                                unsigned long long* __restrict__ totals)
{
    const uint32_t lane = threadIdx.x;   // one wavefront, one counter slot per lane
    unsigned long long p = stats[uint64_t(lane) * kStatStride];
    unsigned long long c = stats[uint64_t(lane) * kStatStride + 1];
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        p += __shfl_xor(p, d, kWave);
        c += __shfl_xor(c, d, kWave);
    }
    if (lane == 0) {
        totals[0] = p;
        totals[1] = c;
    }
}

}  // namespace

extern "C" size_t sdm_static_scratch_bytes(void) { return kStaticScratchBytes; }

extern "C" sdm_status sdm_coalesce_sorted_static(void* stream, uint64_t n_sd, uint32_t n_cells,
                                                 const uint32_t* offsets, uint64_t* xi, double* r,
                                                 const double* dV, double dt, sdm_kernel kernel,
                                                 const sdm_kernel_params* params, uint64_t seed,
                                                 uint64_t step, uint64_t* pair_tests,
                                                 uint64_t* collisions)
{
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n_cells > kStaticMaxCells) {
        set_error("%u cells: the static scratch holds the plan of at most %u cells", n_cells,
                  kStaticMaxCells);
        return SDM_EINVAL;
    }
    if (n_sd > 0xFFFFFFFFull) {
        set_error("n_sd must be below 2^32");
        return SDM_EINVAL;
    }
    if (n_sd > 0 && n_cells == 0) {
        set_error("SDs without cells");
        return SDM_EINVAL;
    }
    if ((n_cells > 0 && (!offsets || !dV)) || (n_sd > 0 && (!xi || !r))) {
        set_error("NULL array");
        return SDM_EINVAL;
    }
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
    sdm_kernel_params kp;
    sdm_default_params(&kp);
    if (params) {
        if (!params_valid(*params)) {
            set_error("kernel parameters must be finite and >= 0, with vt_r1 <= vt_r2");
            return SDM_EINVAL;
        }
        kp = *params;
    }
    if (static_layout(nullptr, n_cells).bytes > kStaticScratchBytes) {
        set_error("%u cells do not fit the static scratch", n_cells);
        return SDM_EINVAL;
    }
    void* base = nullptr;
    SDM_TRY(scratch_address(&base));
    const StaticLayout L = static_layout(base, n_cells);

    // the flags and counters this call reads start at zero (the array keeps
    // whatever the previous call on this device left)
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(L.err),
                       uint64_t(1), 0u);
    SDM_LAUNCHED();
    hipLaunchKernelGGL(k_fill_u64, dim3(4), dim3(256), 0, st, L.stats,
                       uint64_t(kStatSlots) * kStatStride, 0ull);
    SDM_LAUNCHED();
    if (n_cells > 0) {
        hipLaunchKernelGGL(k_static_check, dim3(grid_for(n_cells, 256, 4096)), dim3(256), 0, st,
                           n_cells, n_sd, offsets, dV, L.err);
        SDM_LAUNCHED();
    }
    // launch plan: 256-slot groups when every cell fits, else 512-slot groups
    LaunchShape shape;
    shape.group_slots = 256;
    shape.groups_per_wave = 16;
    shape.waves_per_block = 1;
    shape.xcd_remap = 1;
    uint32_t n_groups = 0;
    bool usable = false, big = false;
    SDM_TRY(device_plan(st, n_cells, offsets, shape.group_slots, L.plan, L.group_begin,
                        L.group_end, &n_groups, &usable, &big));
    if (big) {
        shape.group_slots = 512;
        shape.groups_per_wave = 8;
        SDM_TRY(device_plan(st, n_cells, offsets, shape.group_slots, L.plan, L.group_begin,
                            L.group_end, &n_groups, &usable, &big));
    }
    unsigned int err = 0;
    SDM_HIP(hipMemcpyAsync(&err, L.err, sizeof(err), hipMemcpyDeviceToHost, st));
    SDM_HIP(hipStreamSynchronize(st));
    if (err & kStaticBadOffsets) {
        set_error("offsets must start at 0, not decrease, and end at n_sd");
        return SDM_EINVAL;
    }
    if (err & kStaticBadVolume) {
        set_error("cell volumes must be finite and > 0");
        return SDM_EINVAL;
    }
    if (big) {
        set_error("a cell holds more than 512 slots: use a context (sdm_init)");
        return SDM_EINVAL;
    }
    if (!usable) {
        set_error("the device launch plan failed its check");
        return SDM_EDEVICE;
    }

    StepArgs a{};
    a.xi = xi;
    a.r = r;
    a.n_sd = n_sd;
    a.off_begin = offsets;
    a.off_end = offsets + 1;
    a.dV = dV;
    a.kp = to_kp(kp);
    a.rules = 0;
    a.stats = L.stats;
    a.seed = seed;
    a.step = static_cast<uint32_t>(step);
    a.kernel = static_cast<uint32_t>(kernel);
    a.dt = dt;
    SDM_TRY(launch_step(st, a, L.group_begin, L.group_end, n_groups, shape, false, false));
    if (pair_tests || collisions) {
        hipLaunchKernelGGL(k_static_totals, dim3(1), dim3(kWave), 0, st, L.stats, L.totals);
        SDM_LAUNCHED();
        unsigned long long h[2] = {0, 0};
        SDM_HIP(hipMemcpyAsync(h, L.totals, sizeof(h), hipMemcpyDeviceToHost, st));
        SDM_HIP(hipStreamSynchronize(st));
        if (pair_tests) *pair_tests = h[0];
        if (collisions) *collisions = h[1];
    }
    return SDM_OK;
}
