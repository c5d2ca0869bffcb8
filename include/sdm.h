/*
 * sdm.h -- C ABI of the MI355X (gfx950) super-droplet coalescence library.
 *
 * The library advances the Monte-Carlo coalescence of super-droplets within
 * grid cells, one time step per call, as the particle-based scheme of
 * libcloudph++ 0.2 (Arabas et al.) describes it in Sect. 5.1.4 (Coalescence):
 *
 *   - per cell and step, the super-droplets (SDs) with multiplicity xi > 0 are
 *     grouped at random into floor(n/2) non-overlapping pairs;
 *   - each pair (a, b) collides with the probability of eq. (P_ij)
 *         p = max(xi_a, xi_b) K(r_a, r_b) dt / dV  *  n(n-1)/2 / floor(n/2),
 *     where n is the number of live SDs in the cell and K the collection
 *     kernel (geometric kernel of Sect. 5.1.4, or Golovin's kernel);
 *   - the number of collision events is gamma = floor(p) + [u < p - floor(p)]
 *     for a uniform deviate u on (0,1), capped at floor(xi_j / xi_k) where j
 *     is the SD with the larger multiplicity (the first one on a tie);
 *   - gamma*xi_k droplets of j merge with the xi_k droplets of k: k keeps xi_k
 *     and takes r_k' = cbrt(gamma r_j^3 + r_k^3) (rounded to nearest), j keeps
 *     r_j and loses gamma*xi_k; when that would empty j, both SDs take the
 *     merged radius and share xi_k as floor(xi_k/2) (j) and the rest (k).
 *     (sdm_set_rules selects the paper's own rules instead: one event when
 *     u < p, a zero multiplicity on equal xi, and recycling; sdm_dry_attach
 *     adds the optional dry attributes r_d^3 and kappa, summed and averaged
 *     into the merged droplets.)
 *
 * Randomness is counter-based Philox4x32-10 keyed by (seed, step, cell, slot)
 * (the paper's release uses Mersenne Twister, Sect. 5.3): the shuffle key of
 * storage slot s of cell c at step t is word (s mod 4) of
 * Philox(counter = (s/4, c, t, 0), key = (seed & 0xffffffff, seed >> 32));
 * the live slots are ordered by (key, slot) and paired as (2m, 2m+1); pair m
 * draws u = (2k+1) 2^-53 with k the top 52 bits of the 64-bit integer formed
 * by words 2(m mod 2) (high) and 2(m mod 2)+1 (low) of
 * Philox(counter = (m/2, c, t, 1), same key).
 *
 * Storage order: at initialisation the SDs are stable-sorted by cell (ties in
 * input order); cell c then owns a range of storage slots, local slot
 * s = 0..N_c-1, which only a transport step changes (it re-sorts by the new
 * cells, stable in the old storage order).  Results are therefore a function
 * of (inputs, seed, step numbers) only: independent of launch shape, batching
 * and mix.
 *
 * Conventions for every call:
 *   - "dev" pointers are device (HBM) pointers on the current HIP device;
 *     "host" pointers are host memory.  The caller owns every buffer it
 *     passes, including the workspace; the library never allocates device
 *     memory and frees none.
 *   - stream arguments are hipStream_t values passed as void* (NULL = the
 *     default stream).  All kernels of a context run on its stream.
 *   - every call returns an sdm_status; no exception crosses the ABI.
 *   - a context or batch is used by one host thread at a time; separate
 *     contexts on separate streams are independent.
 */
#ifndef SDM_H_
#define SDM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SDM_OK = 0,
    SDM_EINVAL = -1,   /* invalid argument or input data */
    SDM_ENOMEM = -2,   /* workspace too small / capacity exhausted */
    SDM_EDEVICE = -3,  /* a HIP runtime call failed */
    SDM_ESTATE = -4,   /* call not valid in the object's current state */
    SDM_EBUDGET = -5   /* batch capacity (SDs, cells or instances) exhausted */
} sdm_status;

typedef enum {
    SDM_KERNEL_GOLOVIN = 0,    /* K = b (v_a + v_b), v = (4 pi / 3) r^3 */
    SDM_KERNEL_GEOMETRIC = 1   /* K = E pi (r_a + r_b)^2 |v_t(r_a) - v_t(r_b)|, Sect. 5.1.4 */
} sdm_kernel;

/* Collection-kernel parameters (SI units).  NULL wherever a pointer to this
 * struct is accepted means the defaults given here. */
typedef struct {
    double golovin_b;   /* Golovin constant b, default 1500 s^-1 */
    double vt_k1;       /* v_t = k1 r^2 for r < vt_r1, default 1.19e8 m^-1 s^-1 */
    double vt_k2;       /* v_t = k2 r for vt_r1 <= r <= vt_r2, default 8.0e3 s^-1 */
    double vt_k3;       /* v_t = k3 sqrt(r) for r > vt_r2, default 201.0 m^1/2 s^-1 */
    double vt_r1;       /* default 40e-6 m */
    double vt_r2;       /* default 600e-6 m */
    double efficiency;  /* collection efficiency E, default 1 */
} sdm_kernel_params;

/* Fill *p with the defaults listed above. */
void sdm_default_params(sdm_kernel_params *p);

/* Text for a status code (static storage). */
const char *sdm_strerror(sdm_status s);

/* Message of the last failure on the calling thread (static thread-local storage). */
const char *sdm_last_error(void);

/* ------------------------------------------------------------------------ */
/* Single run: one set of cells advanced by sdm_coalesce_step.               */
/* ------------------------------------------------------------------------ */
typedef struct sdm_ctx sdm_ctx;

/* Bytes of device workspace sdm_init needs for n_sd SDs in n_cells cells. */
size_t sdm_workspace_bytes(uint64_t n_sd, uint32_t n_cells);

/* Create a context and copy the SDs into workspace-resident state.  The
 * attributes taken are those of a computational particle in Sect. 5.1 that
 * coalescence reads and changes (multiplicity N, here xi; the wet radius; the
 * location, here the index of the grid cell that holds it), plus the volume dV
 * of every grid cell that eq. (P_ij) divides by: the state the particle-based
 * scheme's initialisation (particles_t::init, Sect. 5.2) sets up before the
 * first step.
 *   stream     : hipStream_t (as void*) all work of the context runs on.
 *   workspace  : dev, >= sdm_workspace_bytes(n_sd, n_cells) bytes, 256-byte
 *                aligned; owned by the caller, must outlive the context.
 *   n_sd       : number of SDs, < 2^32.
 *   cell       : dev uint32[n_sd], cell index of each SD, < n_cells.
 *   xi         : dev uint64[n_sd], multiplicity (0 = dead SD, never paired).
 *   r          : dev double[n_sd], radius in metres, finite and > 0.
 *   n_cells    : number of cells (>= 1 when n_sd > 0).
 *   dV         : dev double[n_cells], cell volume in m^3, finite and > 0.
 *   params     : host, nullable (defaults).
 * The inputs may be freed after the call returns.  Synchronises the stream.
 * Errors: SDM_EINVAL for a bad pointer/size, a cell index out of range, a
 * radius or volume that is not finite and positive; SDM_ENOMEM if ws_bytes is
 * too small; SDM_EDEVICE for a HIP failure.  *out is NULL on error. */
sdm_status sdm_init(sdm_ctx **out, void *stream, void *workspace, size_t ws_bytes,
                    uint64_t n_sd, const uint32_t *cell, const uint64_t *xi,
                    const double *r, uint32_t n_cells, const double *dV,
                    const sdm_kernel_params *params);

/* Enqueue one coalescence step (Sect. 5.1.4) of every cell on the context's
 * stream and return without waiting.  dt > 0 is the (sub)step length in s;
 * step < 2^32 is the caller's step number, used only as the RNG counter (the
 * same (seed, step) twice applies the same random draws twice).
 * Errors: SDM_EINVAL (dt not finite and positive, unknown kernel,
 * step >= 2^32), SDM_EDEVICE (launch failure). */
sdm_status sdm_coalesce_step(sdm_ctx *ctx, double dt, sdm_kernel kernel, uint64_t seed,
                             uint64_t step);

/* Copy the current state back in input order: xi_out (dev uint64[n_sd]) and
 * r_out (dev double[n_sd]), either may be NULL: the multiplicity and radius of
 * every computational particle (Sect. 5.1 attribute list) after the steps so
 * far.  A particle the outcome rules of Sect. 5.1.4 left empty reads xi = 0.
 * Synchronises the stream.  Errors: SDM_EINVAL (ctx NULL), SDM_EDEVICE. */
sdm_status sdm_get_state(sdm_ctx *ctx, uint64_t *xi_out, double *r_out);

/* Totals since sdm_init: pair tests, i.e. the floor(n/2) pairs examined per
 * cell and step of which eq. (P_ij) speaks (n live particles), summed over
 * cells and steps; and collisions, the examined pairs with at least one
 * collision event (Sect. 5.1.4).  host outputs, nullable.
 * Synchronises the stream.  Errors: SDM_EINVAL (ctx NULL), SDM_EDEVICE (also
 * when a split-tier step, launch knob block_split, timed out waiting for the
 * other workgroups of a cell: the outputs are filled, but the state of those
 * steps is not reliable). */
sdm_status sdm_get_stats(sdm_ctx *ctx, uint64_t *pair_tests, uint64_t *collisions);

/* Storage-order views for diagnostics: slot offsets (dev uint32[n_cells+1])
 * and slot->input-index map (dev uint32[n_sd]).  Pointers into the workspace,
 * valid while the context lives and until the next transport step. */
sdm_status sdm_get_layout(sdm_ctx *ctx, const uint32_t **offsets, const uint32_t **input_index);

/* Compute, without changing the state, the pairing order step `step` would
 * use: the random grouping into non-overlapping pairs of Sect. 5.1.4
 * (consecutive entries 2m, 2m+1 form pair m).  For each cell c, order_out[offsets[c] + i] (dev uint32[n_sd]) = local
 * slot of the i-th live SD after the shuffle, i < n_live_out[c]
 * (dev uint32[n_cells]).  Slots of order_out past n_live are left unchanged.
 * Synchronises the stream. */
sdm_status sdm_debug_permutation(sdm_ctx *ctx, uint64_t seed, uint64_t step,
                                 uint32_t *order_out, uint32_t *n_live_out);

/* ------------------------------------------------------------------------ */
/* Outcome rules (Sect. 5.1.4).  By default a step applies multiple          */
/* coalescence: gamma = floor(P_ij) + [u < frac(P_ij)] events, capped at     */
/* floor(xi_j / xi_k), and equal multiplicities afterwards split xi_k        */
/* between both particles.  The flags select the paper's own release rules.  */
/* ------------------------------------------------------------------------ */
typedef enum {
    /* one event when u < P_ij, never more; equal multiplicities leave the
     * larger (first in pair order) particle with multiplicity 0 and its radius */
    SDM_RULE_RELEASE = 1,
    /* recycle zero-multiplicity particles at the start of every step, within
     * each cell (see sdm_recycle) */
    SDM_RULE_RECYCLE = 2,
    /* recycle them at the start of every step over the whole domain (see
     * sdm_recycle_domain); excludes SDM_RULE_RECYCLE */
    SDM_RULE_RECYCLE_DOMAIN = 4
} sdm_rule;

/* Set / read the rule flags every later step of the context applies (steps,
 * sub-steps, adaptive sub-steps).  Errors: SDM_EINVAL (unknown flag, or both
 * recycling flags), SDM_ESTATE (SDM_RULE_RECYCLE_DOMAIN on several cells
 * without positions attached). */
sdm_status sdm_set_rules(sdm_ctx *ctx, uint32_t rules);
sdm_status sdm_get_rules(sdm_ctx *ctx, uint32_t *rules);

/* Recycle now, within each cell (the zero-multiplicity rule of Sect. 5.1.4):
 * with z dead (xi = 0) and L live slots, the min(z, L) live slots ranked first
 * by multiplicity (largest first, ties to the lower slot) are the donors; in
 * ascending slot order the k-th donor with xi >= 2 gives its radius and
 * floor(xi / 2) of its multiplicity to the k-th dead slot (ascending slot
 * order) and keeps the rest.  Enqueued on the context stream; uses the
 * context's probe scratch. */
sdm_status sdm_recycle(sdm_ctx *ctx);

/* Recycle now, over the whole domain: the recycling procedure of Sect. 5.1.4
 * with no restriction to a cell (Sect. 5.1.5 sends the particles that left the
 * domain through it too).  With z dead and L live slots in the whole storage,
 * the min(z, L) live slots ranked first by multiplicity (largest first, ties
 * to the lower storage slot) are the donors; in ascending slot order the k-th
 * donor with xi >= 2 gives floor(xi / 2), its radius, its dry attributes and
 * its position to the k-th dead slot (ascending slot order) and keeps the
 * rest.  A recycled particle placed in another cell than its slot's joins
 * that cell: the storage is re-sorted by cell, stable in the old storage order
 * (layout pointers change).  Synchronises.  Errors: SDM_ESTATE (several cells
 * and no positions attached), SDM_EDEVICE. */
sdm_status sdm_recycle_domain(sdm_ctx *ctx);

/* Total number of recycled slots since sdm_init (host out).  Synchronises. */
sdm_status sdm_get_recycled(sdm_ctx *ctx, uint64_t *total);

/* ------------------------------------------------------------------------ */
/* Gridded diagnostics (Sect. 5.2, the particle-based scheme's diagnostics:  */
/* super-droplet concentration and k-th radius moment per cell).  Both are   */
/* enqueued on the context stream and do not synchronise it.                 */
/* ------------------------------------------------------------------------ */

/* out[c] (dev uint32[n_cells]) = number of super-droplets with xi > 0 in c.
 * Errors: SDM_EINVAL (out NULL while n_cells > 0), SDM_EDEVICE. */
sdm_status sdm_diag_sd_conc(sdm_ctx *ctx, uint32_t *out);

/* out[c] (dev double[n_cells]) = (rho_d[c] dV[c])^-1 * sum of xi_i r_i^k over
 * the super-droplets of cell c with xi_i > 0 and r_min <= r_i <= r_max
 * (a closed range; r_min > r_max gives zeros).  rho_d (dev double[n_cells])
 * is the dry-air density; NULL means 1, i.e. moments per unit volume.
 * r_i^k is the product of k factors r_i taken left to right (k <= 16).
 * The terms are added in a fixed wavefront-parallel order (64 strided partial
 * sums folded pairwise), so a result is reproducible bit for bit; against the
 * plain sum of the definition it differs by rounding only, at most
 * (2n + 4) 2^-53 relative for a cell of n slots (all terms are >= 0).
 * Errors: SDM_EINVAL (k > 16, NaN bound, out NULL), SDM_EDEVICE. */
sdm_status sdm_diag_moments(sdm_ctx *ctx, uint32_t k, double r_min, double r_max,
                            const double *rho_d, double *out);

/* ------------------------------------------------------------------------ */
/* Collision-probability probe and sub-stepping (the coalescence sub-steps   */
/* of Sect. 5.1.4, with P_ij driving their number as the paper proposes).   */
/* ------------------------------------------------------------------------ */

/* Evaluate eq. (P_ij) for every pair that sdm_coalesce_step(ctx, dt, kernel,
 * seed, step) would test, without changing the state: cell_max (dev
 * double[n_cells], nullable) gets each cell's largest P_ij (0 for a cell with
 * fewer than two live super-droplets), *max_out (host, nullable) the largest
 * over all cells, in which case the stream is synchronised.
 * Errors: as sdm_coalesce_step. */
sdm_status sdm_probe_probability(sdm_ctx *ctx, double dt, sdm_kernel kernel, uint64_t seed,
                                 uint64_t step, double *cell_max, double *max_out);

/* n_substeps coalescence steps of length dt / n_substeps (dt divided once, in
 * binary64), with step counters first_step .. first_step + n_substeps - 1.
 * Identical to calling sdm_coalesce_step that many times.
 * Errors: SDM_EINVAL (n_substeps == 0, a counter >= 2^32, or as
 * sdm_coalesce_step). */
sdm_status sdm_coalesce_substeps(sdm_ctx *ctx, double dt, uint32_t n_substeps, sdm_kernel kernel,
                                 uint64_t seed, uint64_t first_step);

/* Adaptive sub-stepping: probe step first_step with the full dt, take
 * n = ceil(pmax / p_limit) sub-steps (1 if pmax <= p_limit, at most
 * max_substeps) and run sdm_coalesce_substeps(ctx, dt, n, kernel, seed,
 * first_step).  The first sub-step uses the probed pairing, so its largest
 * P_ij is pmax / n up to rounding; later sub-steps draw new pairings.  With
 * SDM_RULE_RECYCLE the recycling runs before the probe, and the first
 * sub-step does not recycle again.
 * *substeps_out (host, nullable) = n; the caller advances its step counter by
 * n.  Synchronises the stream once (to read pmax).
 * Errors: SDM_EINVAL (p_limit not finite and > 0, max_substeps == 0, or as
 * sdm_coalesce_substeps). */
sdm_status sdm_coalesce_adaptive(sdm_ctx *ctx, double dt, double p_limit, uint32_t max_substeps,
                                 sdm_kernel kernel, uint64_t seed, uint64_t first_step,
                                 uint32_t *substeps_out);

/* ------------------------------------------------------------------------ */
/* Particle transport (Sect. 5.1, advection and sedimentation).  A context   */
/* whose cells form an nx x nz grid (cell = i + nx k) can carry positions:   */
/* each transport step moves every super-droplet and re-sorts the storage by */
/* cell, so the next coalescence step pairs particles in their new cells.    */
/* ------------------------------------------------------------------------ */

/* Bytes of the caller-owned device workspace sdm_transport_attach needs
 * (about 64 B per super-droplet and 25 B per cell: positions, re-sort targets
 * of positions, xi, r and the input index, and the re-sort of the particles
 * that change cell). */
size_t sdm_transport_workspace_bytes(uint64_t n_sd, uint32_t n_cells);

/* Attach positions: x_in, z_in (dev double[n_sd], input order) inside
 * [0, nx dx) x [0, nz dz); nx * nz must equal n_cells.  From here on a
 * super-droplet's cell is i + nx k with i = floor(x / dx), k = floor(z / dz)
 * (clamped to the grid), and the storage is re-sorted by those cells at once
 * (stable in the present storage order), which also rebuilds the launch plan.
 * The workspace (256-byte aligned) must stay allocated while the context lives.
 * Synchronises.  Errors: SDM_EINVAL (grid, more than 2^31 - 1 cells, spacing,
 * NULL or out-of-domain positions, workspace), SDM_ENOMEM (workspace too
 * small), SDM_ESTATE (already attached). */
sdm_status sdm_transport_attach(sdm_ctx *ctx, void *workspace, size_t ws_bytes, uint32_t nx,
                                uint32_t nz, double dx, double dz, const double *x_in,
                                const double *z_in);

/* One transport step of length dt.  cx (dev double[nz * nx]) holds the Courant
 * numbers u dt / dx on the left edge of every cell (the right edge of cell nx-1
 * of a row is edge 0: periodic in x), cz (dev double[(nz + 1) * nx]) the
 * numbers w dt / dz on the bottom edge of every cell (row nz is the top
 * boundary); either may be NULL (no flow in that direction).  Each particle
 * uses the edges of its cell at the start of the step in both directions:
 * x' = (x + dx (C_l - i dC)) / (1 - dC), dC = C_r - C_l (backward Euler with
 * the linearly interpolated Courant number, solved analytically), likewise in
 * z.  With sediment != 0 it then falls by v_t(r) dt (the kernel parameters'
 * terminal velocity, explicit Euler).  x wraps periodically; a particle whose z
 * leaves [0, nz dz) gets xi = 0 and is clamped into the boundary row.  The
 * storage is then re-sorted by cell, stable in the old storage order (only the
 * particles that changed cell are sorted), and the plan rebuilt; pointers from
 * sdm_get_layout change.  Synchronises.  Errors: SDM_ESTATE (no transport
 * attached), SDM_EINVAL (dt, or Courant numbers not finite or with
 * C_r - C_l >= 1 in some cell). */
sdm_status sdm_transport_step(sdm_ctx *ctx, const double *cx, const double *cz, double dt,
                              int sediment);

/* Positions in input order: x_out, z_out (dev double[n_sd]), either may be
 * NULL.  Synchronises.  Errors: SDM_ESTATE (no transport attached). */
sdm_status sdm_transport_get_positions(sdm_ctx *ctx, double *x_out, double *z_out);

/* ------------------------------------------------------------------------ */
/* Optional dry attributes (Sect. 5.1.4: on coalescence, extensive particle  */
/* parameters such as the dry radius cubed are summed and intensive ones     */
/* such as the hygroscopicity kappa averaged).  Each droplet formed by g     */
/* events between j (larger multiplicity) and k holds g droplets of j and    */
/* one of k: its r_d^3 is g r_d,j^3 + r_d,k^3 and its kappa the r_d^3-       */
/* weighted mean of theirs, evaluated as ((g r_d,j^3) kappa_j +             */
/* r_d,k^3 kappa_k) / (g r_d,j^3 + r_d,k^3).  The particle that takes the    */
/* merged radius takes these values (in the equal split, both do); recycled  */
/* slots copy the donor's; transport keeps them with their particles.        */
/* Single-run contexts only.                                                  */
/* ------------------------------------------------------------------------ */

/* Bytes of the caller-owned device workspace sdm_dry_attach needs (32 B per
 * super-droplet: both attributes and their re-sort targets). */
size_t sdm_dry_workspace_bytes(uint64_t n_sd);

/* Attach rd3_in (r_d^3, m^3) and kappa_in (dimensionless), dev double[n_sd]
 * in input order; they are copied into the workspace (256-byte aligned,
 * allocated while the context lives).  Synchronises.  Errors: SDM_EINVAL
 * (NULL arrays while n_sd > 0, an r_d^3 not finite and > 0 or a kappa not
 * finite and >= 0, workspace NULL or misaligned), SDM_ENOMEM (workspace too
 * small), SDM_ESTATE (already attached). */
sdm_status sdm_dry_attach(sdm_ctx *ctx, void *workspace, size_t ws_bytes, const double *rd3_in,
                          const double *kappa_in);

/* r_d^3 and kappa in input order (dev double[n_sd]; either output may be
 * NULL).  Synchronises.  Errors: SDM_ESTATE (nothing attached). */
sdm_status sdm_dry_get(sdm_ctx *ctx, double *rd3_out, double *kappa_out);

/* As sdm_diag_moments for the dry radius r_d, the correctly rounded cube root
 * of r_d^3, with the closed range [rd_min, rd_max].  Errors: as
 * sdm_diag_moments, SDM_ESTATE (nothing attached). */
sdm_status sdm_diag_dry_moments(sdm_ctx *ctx, uint32_t k, double rd_min, double rd_max,
                                const double *rho_d, double *out);

/* Launch plan of a context: number of wave-tier groups (runs of consecutive
 * cells processed by one wavefront), cells in them, cells of the workgroup
 * tier (more storage slots than a group holds, up to block_slots: one
 * workgroup each, the sort in LDS) and cells of the grid tier (larger, each
 * spread over many workgroups).  host outputs, nullable. */
sdm_status sdm_get_plan(sdm_ctx *ctx, uint32_t *groups, uint32_t *wave_cells,
                        uint32_t *block_cells, uint32_t *grid_cells);

/* Launch-shape knobs; none of them changes any result.
 *   group_slots    : storage slots one wavefront handles per group (64, 128,
 *                    256 or 512); cells with more slots go to the other tiers;
 *   groups_per_wave: groups each wavefront takes in sequence (1..64);
 *   waves_per_block: wavefronts per workgroup of the wave tier (1, 2, 4);
 *   xcd_remap      : 1 = give each of the 8 XCDs a contiguous range of groups;
 *   block_slots    : largest cell of the workgroup tier (0, 2048 or 8192,
 *                    default 8192; 0 sends every cell above group_slots to
 *                    the grid tier);
 *   block_split    : single runs only (a batch takes 0): every workgroup-tier
 *                    cell is spread over 2^block_split workgroups (0..5,
 *                    default 0), each taking the SDs of one top-key-bits
 *                    digit, for runs with too few such cells to fill the
 *                    GPU one workgroup each; needs block_slots > 0. */
typedef struct {
    uint32_t group_slots;
    uint32_t groups_per_wave;
    uint32_t waves_per_block;
    uint32_t xcd_remap;
    uint32_t block_slots;
    uint32_t block_split;
} sdm_launch_config;
sdm_status sdm_get_launch_config(sdm_ctx *ctx, sdm_launch_config *cfg);
sdm_status sdm_set_launch_config(sdm_ctx *ctx, const sdm_launch_config *cfg);

/* Time every launch configuration of a small candidate set on this context
 * (each candidate runs `reps` steps under the context's rules), keep the
 * fastest, and restore the state exactly as it was: multiplicities, radii, the
 * dry attributes when attached, and the counters.  Needs
 * sdm_autotune_workspace_bytes() bytes of device scratch (caller-owned, 256-byte
 * aligned; 16 B per SD, 32 B per SD with dry attributes attached, so attach
 * them before asking for the size).  best_out (host, nullable) gets the choice.
 * Synchronises.  Errors: SDM_ENOMEM (scratch too small or misaligned), and as
 * sdm_coalesce_step. */
size_t sdm_autotune_workspace_bytes(sdm_ctx *ctx);
sdm_status sdm_autotune(sdm_ctx *ctx, void *scratch, size_t scratch_bytes, double dt,
                        sdm_kernel kernel, uint64_t seed, uint32_t reps,
                        sdm_launch_config *best_out);

/* Release host-side resources.  Device memory stays with the caller. */
void sdm_destroy(sdm_ctx *ctx);

/* ------------------------------------------------------------------------ */
/* Batched / served instances: many independent runs advanced by one step    */
/* call.  Each instance has its own cells, kernel, parameters, dt, seed and  */
/* step counter; its RNG counters use its own cell indices, so its results   */
/* are bit-identical alone (sdm_init + sdm_coalesce_step) and in any batch.  */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint64_t n_sd;
    uint32_t n_cells;
    const uint32_t *cell;     /* dev, instance-local cell index < n_cells */
    const uint64_t *xi;       /* dev */
    const double *r;          /* dev */
    const double *dV;         /* dev, n_cells */
    sdm_kernel kernel;
    sdm_kernel_params params;
    double dt;                /* step length, s */
    uint64_t seed;
    uint64_t first_step;      /* step number of the instance's first batch step */
} sdm_instance_desc;

typedef struct sdm_batch sdm_batch;

/* Device workspace for a batch holding at most max_sd SDs, max_cells cells
 * and max_instances instances at a time. */
size_t sdm_batch_workspace_bytes(uint64_t max_sd, uint32_t max_cells, uint32_t max_instances);

/* Create an empty batch over caller-owned workspace (dev, 256-byte aligned). */
sdm_status sdm_batch_create(sdm_batch **out, void *stream, void *workspace, size_t ws_bytes,
                            uint64_t max_sd, uint32_t max_cells, uint32_t max_instances);

/* Admit an instance: validate and copy its SDs into the batch (stable sort by
 * cell, as sdm_init).  Inputs may be freed afterwards.  Synchronises the
 * stream.  Errors: SDM_EINVAL (bad data), SDM_EBUDGET (not enough free SDs,
 * cells or instance slots: nothing is changed and the caller may retry after
 * removing instances). */
sdm_status sdm_batch_add(sdm_batch *b, const sdm_instance_desc *desc, int32_t *handle_out);

/* Enqueue one step of every admitted instance: instance i uses step number
 * first_step_i + (number of batch steps since it was admitted).  Returns
 * without waiting.  use_graph = 1 replays a captured HIP graph of the step
 * (captured again only after the instance set changed). */
sdm_status sdm_batch_step(sdm_batch *b, int use_graph);

/* Copy an instance's state in its input order (dev outputs, nullable) and its
 * counters (host outputs, nullable).  Synchronises the stream. */
sdm_status sdm_batch_get(sdm_batch *b, int32_t handle, uint64_t *xi_out, double *r_out,
                         uint64_t *steps_done, uint64_t *pair_tests, uint64_t *collisions);

/* Remove an instance (after copying its state out as sdm_batch_get when the
 * output pointers are not NULL) and free its SDs, cells and slot. */
sdm_status sdm_batch_remove(sdm_batch *b, int32_t handle, uint64_t *xi_out, double *r_out);

/* Number of admitted instances, and free capacity. */
sdm_status sdm_batch_info(sdm_batch *b, uint32_t *n_instances, uint64_t *free_sd,
                          uint32_t *free_cells);

/* Launch shape of a batch's steps (as sdm_set_launch_config; results do not
 * depend on it).  Setting it re-plans the work lists and re-captures the graph
 * at the next step.  Errors: SDM_EINVAL (NULL, out of range). */
sdm_status sdm_batch_get_launch_config(sdm_batch *b, sdm_launch_config *cfg);
sdm_status sdm_batch_set_launch_config(sdm_batch *b, const sdm_launch_config *cfg);

/* Time every launch shape of a candidate set on the admitted instances (each
 * candidate runs reps steps of all of them), keep the fastest, and restore every
 * instance exactly as it was (multiplicities, radii, step counters, counters).
 * Needs sdm_batch_autotune_workspace_bytes() bytes of device scratch
 * (caller-owned, 256-byte aligned: 16 B per SD of capacity and one record per
 * instance slot).  best_out (host, nullable) gets the choice.  Synchronises.
 * Errors: SDM_EINVAL (NULL batch), SDM_ENOMEM (scratch too small or
 * misaligned), SDM_EDEVICE. */
size_t sdm_batch_autotune_workspace_bytes(sdm_batch *b);
sdm_status sdm_batch_autotune(sdm_batch *b, void *scratch, size_t scratch_bytes, uint32_t reps,
                              sdm_launch_config *best_out);

void sdm_batch_destroy(sdm_batch *b);

/* ------------------------------------------------------------------------ */
/* A step that allocates nothing, for callers that cannot allocate device    */
/* memory or pass a workspace (code under stream capture set-up, serving     */
/* loops with a fixed footprint).                                            */
/* ------------------------------------------------------------------------ */

/* Size in bytes of the library's static device scratch (16 MiB; one copy per
 * device, held until the process ends). */
size_t sdm_static_scratch_bytes(void);

/* One coalescence step, as sdm_coalesce_step with the default rules, of SDs
 * that the caller already keeps sorted by cell: cell c owns the storage slots
 * [offsets[c], offsets[c+1]) of xi and r, and the results are those of a
 * context created by sdm_init from these arrays (cell index = the cell whose
 * range holds the slot) after sdm_coalesce_step(ctx, dt, kernel, seed, step),
 * bit for bit.  The launch plan, the counters and the flags live in the static
 * scratch; the call allocates and frees no device memory.
 *   stream   : hipStream_t (as void*) of the current device.
 *   n_sd     : number of SDs, < 2^32; n_cells <= 2^20 cells, every cell with at
 *              most 512 slots (larger cells need a context).
 *   offsets  : dev uint32[n_cells + 1], offsets[0] = 0, non-decreasing,
 *              offsets[n_cells] = n_sd.
 *   xi, r    : dev uint64[n_sd], double[n_sd], updated in place (xi = 0 is a
 *              dead SD; radii must be finite and > 0: they are not checked).
 *   dV       : dev double[n_cells], finite and > 0.
 *   params   : host, nullable (defaults).
 *   pair_tests, collisions : host, nullable; this step's totals.
 * Synchronises the stream (to read the launch plan's size, and the totals).
 * Every call on a device shares that device's scratch, so calls that overlap
 * on one device (other host threads, other streams) race: serialise them.
 * Errors: SDM_EINVAL (more than 2^20 cells, a cell above 512 slots, bad
 * offsets or volumes, dt, kernel, step >= 2^32, NULL arrays; nothing is
 * changed), SDM_EDEVICE (a HIP failure). */
sdm_status sdm_coalesce_sorted_static(void *stream, uint64_t n_sd, uint32_t n_cells,
                                      const uint32_t *offsets, uint64_t *xi, double *r,
                                      const double *dV, double dt, sdm_kernel kernel,
                                      const sdm_kernel_params *params, uint64_t seed,
                                      uint64_t step, uint64_t *pair_tests, uint64_t *collisions);

/* ------------------------------------------------------------------------ */
/* Element-wise checks of the device arithmetic (used by the parity tests).  */
/* All arrays are dev, length n; the call synchronises the stream.           */
/* ------------------------------------------------------------------------ */

/* out[4i..4i+3] = Philox4x32-10(counter = ctr[4i..4i+3], key = key[2i..2i+1]). */
sdm_status sdm_debug_philox(void *stream, uint64_t n, const uint32_t *ctr, const uint32_t *key,
                            uint32_t *out);

/* The bounded wait of the split tier (launch knob block_split), for tests of its
 * time-out path: spin_limit sets how many polls a wait makes before it gives up
 * (0 restores the default, about a second), and epoch_skew is added to the
 * context's count of split-tier steps, so that the following steps wait for
 * arrivals that never come; each of their zero-multiplicity writes then gives up
 * after spin_limit polls, writes anyway and is counted, and sdm_get_stats
 * returns SDM_EDEVICE.  A later re-plan (a launch config with other
 * group_slots or block_slots) clears the skew.  Errors: SDM_EINVAL (ctx NULL). */
sdm_status sdm_debug_split_wait(sdm_ctx *ctx, uint32_t spin_limit, uint32_t epoch_skew);

/* Philox4x32-10 over a counter range: out[4i..4i+3] (dev uint32[4n]) =
 * Philox(counter = (counter[0] + lo32(i), counter[1] + hi32(i), counter[2],
 * counter[3]), key = (key[0], key[1])), words modulo 2^32; counter and key are
 * host arrays. */
sdm_status sdm_debug_philox_range(void *stream, uint64_t n, const uint32_t *counter,
                                  const uint32_t *key, uint32_t *out);

/* The step's square root and division: sqrt_out[i] = sqrt(a[i]) as the
 * terminal velocity above vt_r2 forms it (k3 = 1), div_out[i] = a[i] / b[i] as
 * eq. (P_ij) forms it (xi = dt = scale = 1, K = a[i], dV = b[i]).  Either
 * output may be NULL (not both); b may be NULL without div_out. */
sdm_status sdm_debug_sqrt_div(void *stream, uint64_t n, const double *a, const double *b,
                              double *sqrt_out, double *div_out);

/* y[i] = cube root of x[i] rounded to nearest (the rounding the collision
 * update uses). */
sdm_status sdm_debug_cbrt(void *stream, uint64_t n, const double *x, double *y);

/* One collision test per element, exactly as inside the step: pair
 * (xi_a, r_a) first and (xi_b, r_b) second in a cell of n_live live SDs and
 * volume dV, uniform deviate u.  Outputs: K, p, gamma, and the updated
 * (xi_a, r_a, xi_b, r_b) written back in place. */
sdm_status sdm_debug_collide(void *stream, uint64_t n, sdm_kernel kernel,
                             const sdm_kernel_params *params, double dt,
                             const uint32_t *n_live, const double *dV, const double *u,
                             uint64_t *xi_a, double *r_a, uint64_t *xi_b, double *r_b,
                             double *K_out, double *p_out, uint64_t *gamma_out);

#ifdef __cplusplus
}
#endif

#endif /* SDM_H_ */
