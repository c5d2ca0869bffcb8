// context.hpp -- the state of a single-run context, shared by the files that
// implement its C ABI (context.hip: steps and queries; transport.hip: particle
// transport between cells; dry.hip: the optional dry attributes).
#pragma once

#include "runtime.hpp"

#include <memory>

namespace sdm {

// Positions and grid of a context with transport attached; every array is in
// storage order and lives in the caller's transport workspace.
struct TransportState {
    uint32_t nx = 0, nz = 0;
    double dx = 0.0, dz = 0.0;
    double* x = nullptr;        // positions
    double* z = nullptr;
    double* x_alt = nullptr;    // gather targets of the re-sort (swapped with the live arrays)
    double* z_alt = nullptr;
    uint64_t* xi_alt = nullptr;
    double* r_alt = nullptr;
    uint32_t* id_alt = nullptr;
    uint32_t* cell = nullptr;   // new cell of every slot, top bit set if it changed
    // re-sort of the particles that changed cell
    uint32_t* tcnt = nullptr;       // movers per 256-slot tile, then their exclusive prefix
    uint32_t* mk = nullptr;         // movers: new cell, in old-slot order (then the inverse order)
    uint32_t* mv = nullptr;         // movers: old slot
    uint32_t* mlo = nullptr;        // per cell: movers with an old slot below the cell
    uint32_t* off_alt = nullptr;    // new slot offsets (swapped with the live offsets)
    uint32_t* inc_off = nullptr;    // offsets of the incoming movers per new cell
    uint32_t* in_low = nullptr;     // incoming movers from lower cells, per cell
    uint32_t* count = nullptr;      // new slots per cell (n_cells + 1, last 0)
    uint32_t* tile_sums = nullptr;  // scan scratch
    DevicePlanArrays plan;          // launch plan on the device
};

}  // namespace sdm

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
    uint32_t* group_begin = nullptr;
    uint32_t* group_end = nullptr;
    uint32_t split_spin_limit = 0;       // split-tier poll limit (0: the default)
    sdm::GridArrays grid;
    unsigned long long* stats = nullptr;
    unsigned int* err = nullptr;
    uint32_t* probe_order = nullptr;
    double* probe_cell = nullptr;       // probe: largest P_ij per cell (when the caller keeps none)
    unsigned long long* probe_max = nullptr;
    uint32_t* rd_small = nullptr;       // domain-wide recycling: counters and a digit histogram
    uint64_t* scr_kv = nullptr;
    uint64_t* scr_tmp = nullptr;
    uint32_t* scr_pos = nullptr;
    uint32_t* scr_cnt = nullptr;
    // plan
    std::vector<uint32_t> sizes;   // storage slots per cell (host copy)
    bool sizes_stale = false;      // sizes behind the device offsets (device-planned)
    uint32_t n_groups = 0, n_wave_cells = 0;
    sdm::LaunchShape shape;
    uint32_t rules = 0;   // sdm_rule flags applied by every step
    // admission sort scratch (shares the step scratch region; reused by transport)
    sdm::SortScratch sort{};
    // particle positions and the transport buffers, once attached
    std::unique_ptr<sdm::TransportState> transport;
    // optional dry attributes (r_d^3, kappa) in storage order and their re-sort
    // targets, once attached (caller's dry workspace)
    double* rd3 = nullptr;
    double* kappa = nullptr;
    double* rd3_alt = nullptr;
    double* kappa_alt = nullptr;
};

namespace sdm {
// Rebuild the launch plan from x->sizes and upload it (synchronises).
sdm_status ctx_replan(sdm_ctx* x);
// Recycling over the whole domain (synchronises; re-sorts by cell when
// positions are attached).
sdm_status recycle_domain(sdm_ctx* x);
}  // namespace sdm
