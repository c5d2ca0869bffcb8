// step_kernels.hpp -- the per-step coalescence kernels (Sect. 5.1.4).
//
// One step of a cell = (1) count the live super-droplets n (multiplicity > 0),
// (2) draw a 32-bit Philox key per live storage slot and order the live slots
// by (key, slot), (3) pair neighbours (2m, 2m+1) of that order and run the
// collision test of eq. (P_ij) on each pair, (4) write back the super-droplets
// a collision changed.
//
// The ordering is an exact sort done as one most-significant-digit radix pass
// on the top lg bits of the key (2^lg buckets, lg ~ log2 n): a counting pass
// with LDS/global atomics, an exclusive scan of the bucket counts, a scatter
// by (bucket start + arrival index), and a rank inside each bucket by a full
// (key, slot) comparison.  Because the keys are uniform, a bucket holds O(1)
// entries on average, so the sort is O(n) and its result is independent of
// the atomic arrival order.
//
// Four tiers cover all cell sizes with identical results:
//   k_wave_groups -- one 64-lane wavefront per group of consecutive cells
//                    (at most CAP storage slots in all), everything in LDS;
//   k_block_cells -- one workgroup per cell of up to kBlockLarge slots, the
//                    whole cell in LDS;
//   k_split_cells -- such a cell spread over 2^lgG workgroups, one digit of
//                    the top key bits each (single runs with few such cells);
//   grid tier     -- larger cells, each spread over many workgroups, with the
//                    sort arrays in a global scratch area that is indexed like
//                    the super-droplet arrays (a two-level digit sort, see below).
#pragma once

#include "device_math.hpp"

namespace sdm {

constexpr int kWave = 64;
constexpr int kStatSlots = 64;                     // spread of the global counters
constexpr int kStatStride = 16;                    // 128 bytes between counter pairs

// Outcome rules of a step (bit flags, as the public rule flags).
enum : uint32_t { kRuleRelease = 1u, kRuleRecycle = 2u, kRuleRecycleDomain = 4u };
// Device scratch of the domain-wide recycling: 16 counter words, then a
// 2^kRecycleDomainDigit-entry digit histogram.
constexpr uint32_t kRecycleDomainDigit = 12;
constexpr uint32_t kRecycleDomainSmall = 16 + (1u << kRecycleDomainDigit);
// Index of the recycled-slot counter within each slot of the single-run counter
// array (a free word of every counter slot; the total is their sum).
constexpr int kRecycledStat = 2;

// Per-instance record of a batch (device table).
struct InstanceRec {
    uint64_t seed;
    uint64_t step;            // step number the next batch step uses
    double dt;
    uint32_t kernel;
    uint32_t active;
    KernelParams kp;
    unsigned long long pair_tests;
    unsigned long long collisions;
    unsigned long long steps_done;
    unsigned long long pad;
};

struct StepArgs {
    uint64_t* xi;                 // storage-order multiplicities
    double* r;                    // storage-order radii
    double* rd3;                  // optional dry attributes (null, or both per slot)
    double* kappa;
    uint64_t n_sd;                // length of xi and r
    const uint32_t* group_begin;  // wave tier: first cell of each group
    const uint32_t* group_end;    // one past the last cell
    uint32_t n_groups;
    uint32_t groups_per_wave;
    const uint32_t* off_begin;    // first storage slot of each cell
    const uint32_t* off_end;      // one past the last storage slot
    const double* dV;             // cell volume
    const uint32_t* cell_inst;    // batched: instance of each cell
    const uint32_t* cell_local;   // batched: instance-local cell index (RNG counter)
    InstanceRec* inst;            // batched: instance table
    // single-run parameters
    uint64_t seed;
    uint32_t step;
    uint32_t kernel;
    double dt;
    KernelParams kp;
    uint32_t rules;               // kRuleRelease: one event when u < P_ij, zero on equal xi
    unsigned long long* stats;    // single run: kStatSlots x {pair tests, collisions}
    // workgroup-tier scratch, indexed by storage slot
    uint64_t* scr_kv;
    uint64_t* scr_tmp;
    uint32_t* scr_pos;
    uint32_t* scr_cnt;
    // permutation-only mode outputs
    uint32_t* perm_out;
    uint32_t* nlive_out;
    // probe mode output: largest P_ij per cell (grid-tier cells by atomic max on
    // the bit pattern, so they must start at 0)
    double* cell_max;
    uint32_t xcd_remap;
    // grid tier (cells spread over many workgroups)
    struct GridCell* gcell;
    uint32_t n_grid;
    // (grid cell, first slot, cell) per slot chunk: the cell is there so that its
    // offset and job load beside the grid cell instead of after it
    const uint4* gchunk;
    uint32_t n_gchunk;
    const uint2* gtile;           // (grid cell, first entry) per count-table tile
    uint32_t n_gtile;
    const uint4* gbucket;         // (grid cell, digit, cell) per digit bucket
    uint32_t n_gbucket;
    // workgroup tier: cells in descending order of storage slots; the first
    // n_block_big hold more than kBlockSmall slots
    const uint32_t* blist;
    uint32_t n_block;
    uint32_t n_block_big;
    // split tier: per workgroup-tier cell, workgroups that have read its
    // multiplicities (grows by 2^block_split a step), and the step's number
    uint32_t* split_arrive;
    uint32_t split_epoch;
    uint32_t split_spin_limit;    // polls before a wait gives up (0: kSplitSpinLimit)
    uint32_t* gtilesum;
    // digit counters the placement stages through LDS: the largest 2^cb of the
    // grid cells, at most kGridStagedDigits (sizes the kernels' dynamic LDS)
    uint32_t grid_dcap;
    uint32_t grid_dmax;           // largest 2^cb of the grid cells
};

// One cell of the grid tier.  Everything but `live` depends on the storage-slot
// count only (any digit width gives the same order); live is written during the
// step.  The count table lives in the cell's scr_cnt range: entry d * ncol + c
// counts the live slots of chunk c whose key has digit d, and entry nb is the
// sentinel (the live count) after the scan.
struct GridCell {
    uint32_t cell;     // cell-table index
    uint32_t cb;       // digit bits: a digit is the top cb bits of a key
    uint32_t lgc;      // a slot chunk (one table column) is 2^lgc slots
    uint32_t ncol;     // slot chunks
    uint32_t nb;       // table entries, 2^cb * ncol (< storage slots)
    uint32_t tile0;    // first table tile
    uint32_t ntiles;
    uint32_t live;     // live SDs this step
};

// Resolved per-cell parameters.
struct CellJob {
    uint32_t off, n_slots, rng_cell, step;
    uint32_t k0, k1, kernel, inst;
    double dt, dV;
    KernelParams kp;
};

template <bool BATCHED>
__device__ __forceinline__ CellJob resolve_cell(const StepArgs& a, uint32_t c)
{
    CellJob j;
    j.off = a.off_begin[c];
    j.n_slots = a.off_end[c] - j.off;
    j.dV = a.dV[c];
    if constexpr (BATCHED) {
        const uint32_t i = a.cell_inst[c];
        const InstanceRec& rec = a.inst[i];
        j.inst = i;
        j.rng_cell = a.cell_local[c];
        j.step = static_cast<uint32_t>(rec.step);
        j.k0 = static_cast<uint32_t>(rec.seed);
        j.k1 = static_cast<uint32_t>(rec.seed >> 32);
        j.kernel = rec.kernel;
        j.dt = rec.dt;
        j.kp = rec.kp;
    } else {
        j.inst = 0;
        j.rng_cell = c;
        j.step = a.step;
        j.k0 = static_cast<uint32_t>(a.seed);
        j.k1 = static_cast<uint32_t>(a.seed >> 32);
        j.kernel = a.kernel;
        j.dt = a.dt;
        j.kp = a.kp;
    }
    return j;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, kWave);
        if (lane >= static_cast<uint32_t>(d)) v += t;
    }
    return v;
}

__device__ __forceinline__ uint32_t ceil_log2(uint32_t n)   // n >= 2
{
    return 32u - static_cast<uint32_t>(__clz(static_cast<int>(n - 1u)));
}

// top `lg` bits of the key (lg in 0..32)
__device__ __forceinline__ uint32_t bucket_of(uint32_t key, uint32_t lg)
{
    return static_cast<uint32_t>(static_cast<uint64_t>(key) >> (32u - lg));
}

__device__ __forceinline__ void add_counts(const StepArgs& a, bool batched, uint32_t inst,
                                           uint32_t slot, unsigned long long pairs,
                                           unsigned long long coll)
{
    if (batched) {
        if (pairs) atomicAdd(&a.inst[inst].pair_tests, pairs);
        if (coll) atomicAdd(&a.inst[inst].collisions, coll);
    } else {
        unsigned long long* s = a.stats + (slot % kStatSlots) * kStatStride;
        if (pairs) atomicAdd(s, pairs);
        if (coll) atomicAdd(s + 1, coll);
    }
}

// Dry attributes after g events: k (and j too in the equal split) takes the
// merged droplets' r_d^3 and kappa.
__device__ __forceinline__ void update_dry(const StepArgs& a, uint64_t g, uint64_t gj, uint64_t gk,
                                           bool both)
{
    if (!a.rd3) return;
    double rd3_new, kappa_new;
    merge_dry(g, a.rd3[gj], a.kappa[gj], a.rd3[gk], a.kappa[gk], rd3_new, kappa_new);
    a.rd3[gk] = rd3_new;
    a.kappa[gk] = kappa_new;
    if (both) {
        a.rd3[gj] = rd3_new;
        a.kappa[gj] = kappa_new;
    }
}

// Pair test + update of one pair (a first, b second in shuffle order).
// Writes changed super-droplets to global memory; returns whether gamma > 0.
__device__ __forceinline__ bool collide_pair_global(const StepArgs& a, const CellJob& j,
                                                    double scale, double u, uint32_t sa,
                                                    uint32_t sb, uint64_t xa, uint64_t xb,
                                                    double ra, double rb)
{
    const double K = collection_kernel(j.kernel, j.kp, ra, rb);
    const bool a_is_j = xa >= xb;
    PairState s;
    s.xj = a_is_j ? xa : xb;
    s.xk = a_is_j ? xb : xa;
    s.rj = a_is_j ? ra : rb;
    s.rk = a_is_j ? rb : ra;
    const double p = collision_probability(s.xj, K, j.dt, j.dV, scale);
    const bool release = (a.rules & kRuleRelease) != 0;
    const uint64_t g = release ? collision_count_release(p, u) : collision_count(p, u, s.xj, s.xk);
    if (g == 0) return false;
    apply_collisions(g, s, release);
    const uint32_t slot_j = a_is_j ? sa : sb;
    const uint32_t slot_k = a_is_j ? sb : sa;
    const uint64_t gj = static_cast<uint64_t>(j.off) + slot_j;
    const uint64_t gk = static_cast<uint64_t>(j.off) + slot_k;
    a.xi[gj] = s.xj;
    a.r[gk] = s.rk;
    if (s.j_changed_r) {
        a.xi[gk] = s.xk;
        a.r[gj] = s.rj;
    }
    update_dry(a, g, gj, gk, s.j_changed_r);
    return true;
}

// ---------------------------------------------------------------------------
// Wave tier: one wavefront per group of consecutive cells holding at most CAP
// storage slots (and at most kGroupMaxCells cells), everything staged in LDS.
// Packing several cells into one wavefront keeps all 64 lanes busy in every
// phase; per-slot and per-pair lookups go through small LDS tables so that
// each phase needs one or two dependent LDS round trips.  Collisions are
// queued in LDS and applied 64 at a time, so the cube-root path runs with
// full lanes.  The next group's loads are issued before the current group's
// pair tests, to overlap HBM latency with them.
// ---------------------------------------------------------------------------
constexpr int kGroupMaxCells = 64;
constexpr int kQueueCap = 128;

struct CollEntry {
    uint32_t gj, gk;   // storage slots of j (larger multiplicity) and k
    uint64_t g;        // number of collision events
};

template <int CAP>
struct alignas(16) GroupLds {
    static_assert(CAP % kWave == 0 && CAP <= 512, "group capacity");
    double dV[kGroupMaxCells];
    double scale[kGroupMaxCells];           // upscaling factor of eq. (P_ij)
    uint32_t eqn[kGroupMaxCells];           // first sorted position E | pair base Q << 10 | n << 20
    uint32_t ucb[kGroupMaxCells];           // first uniform call of the cell
    CollEntry queue[kQueueCap];             // pending collisions (ring)
    union {
        // entry CAP of kv / xi / r / slot, CAP/2 of pairinfo and the last
        // ucall entry are write-only dummies that dead slots are sent to
        struct {
            uint64_t kv[CAP + 2];           // (key << 32 | slot) grouped by bucket
            uint32_t start[CAP + 4];        // bucket counts, then bucket starts
            uint32_t keys[CAP];             // shuffle key of every group slot
            uint32_t slotinfo[CAP];         // cell | bucket base << 8 | lg << 24 (base < 2048)
            uint32_t call[CAP / 4 + kGroupMaxCells];   // key call: slot base | cell << 9 | q << 15 | (words-1) << 22
        } sort;
        struct {
            uint64_t xi[CAP + 2];           // live SDs in sorted order
            double r[CAP + 2];
            double u[CAP / 2];              // uniform deviate of every pair
            uint16_t slot[CAP + 2];
            uint16_t pairinfo[CAP / 2 + 2]; // sorted position of the first member | cell << 10
            uint32_t ucall[CAP / 4 + kGroupMaxCells + 1];   // first pair | cell << 9 | h << 15 | 2nd valid << 23
        } pairs;
    };
};

struct GroupJob {
    uint32_t rng_base, step, k0, k1, kernel, inst;
    double dt;
    KernelParams kp;
};

template <bool BATCHED>
__device__ __forceinline__ GroupJob resolve_group(const StepArgs& a, uint32_t c0)
{
    GroupJob j;
    if constexpr (BATCHED) {
        const uint32_t i = a.cell_inst[c0];
        const InstanceRec& rec = a.inst[i];
        j.inst = i;
        j.rng_base = a.cell_local[c0];
        j.step = static_cast<uint32_t>(rec.step);
        j.k0 = static_cast<uint32_t>(rec.seed);
        j.k1 = static_cast<uint32_t>(rec.seed >> 32);
        j.kernel = rec.kernel;
        j.dt = rec.dt;
        j.kp = rec.kp;
    } else {
        j.inst = 0;
        j.rng_base = c0;
        j.step = a.step;
        j.k0 = static_cast<uint32_t>(a.seed);
        j.k1 = static_cast<uint32_t>(a.seed >> 32);
        j.kernel = a.kernel;
        j.dt = a.dt;
        j.kp = a.kp;
    }
    return j;
}

// Apply `count` queued collisions (one per lane) starting at ring index head.
// The pair's multiplicities and radii are re-read from global memory: nothing
// else writes those slots during the step.  DRY: also the dry attributes (a
// separate instantiation, so that the kernel without them keeps its registers).
template <bool DRY>
__device__ __forceinline__ void flush_collisions(const StepArgs& a, const CollEntry* queue,
                                                 uint32_t head, uint32_t count, uint32_t lane)
{
    if (lane < count) {
        const CollEntry e = queue[(head + lane) % kQueueCap];
        if (e.gj < a.n_sd && e.gk < a.n_sd) {
            PairState s;
            s.xj = a.xi[e.gj];
            s.xk = a.xi[e.gk];
            s.rj = a.r[e.gj];
            s.rk = a.r[e.gk];
            apply_collisions(e.g, s, (a.rules & kRuleRelease) != 0);
            a.xi[e.gj] = s.xj;
            a.r[e.gk] = s.rk;
            if (s.j_changed_r) {
                a.xi[e.gk] = s.xk;
                a.r[e.gj] = s.rj;
            }
            if constexpr (DRY) update_dry(a, e.g, e.gj, e.gk, s.j_changed_r);
        }
    }
}

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, uint32_t lane)
{
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), static_cast<int>(lane)));
}

// Inclusive sum over the 64 lanes with DPP row shifts and row broadcasts (no LDS).
__device__ __forceinline__ uint32_t wave_inclusive_sum_dpp(uint32_t v)
{
    int x = static_cast<int>(v);
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return static_cast<uint32_t>(x);
}

// Where a group's slots are: its cells [c0, c1), the first slot of cell
// c0 + lane (lanes < c1 - c0) and one past the group's last slot.
struct GroupHead {
    uint32_t c0, c1, o, end;
};

// A read of a table the step kernels never write, through the constant
// address space: with a wave-uniform index it becomes a scalar load.
__device__ __forceinline__ uint32_t load_const_u32(const uint32_t* p, uint64_t i)
{
    typedef const __attribute__((address_space(4))) uint32_t const_u32;
    return ((const_u32*)p)[i];
}

__device__ __forceinline__ void fetch_head(const StepArgs& a, uint64_t gi, uint32_t lane,
                                           GroupHead& H)
{
    H.c0 = load_const_u32(a.group_begin, gi);
    H.c1 = load_const_u32(a.group_end, gi);
    const uint32_t ncell = H.c1 - H.c0;
    H.o = lane < ncell ? a.off_begin[H.c0 + lane] : 0u;
    H.end = load_const_u32(a.off_end, H.c1 - 1);
}

// The slots of one group in registers, and where they came from.
template <int K>
struct GroupRegs {
    uint32_t c0, c1, g_first, G, o;   // o: first slot of cell c0 + lane (lanes < ncell)
    double dv;                        // volume of cell c0 + lane (lanes < ncell)
    uint64_t xv[K];
    double rv[K];
};

template <int K, bool PERM>
__device__ __forceinline__ void fetch_group(const StepArgs& a, const GroupHead& H, uint32_t lane,
                                            GroupRegs<K>& R)
{
    R.c0 = H.c0;
    R.c1 = H.c1;
    R.o = H.o;
    const uint32_t ncell = R.c1 - R.c0;
    R.g_first = readlane_u32(R.o, 0);
    R.G = H.end - R.g_first;
    R.dv = lane < ncell ? a.dV[R.c0 + lane] : 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t s = lane + k * kWave;
        R.xv[k] = 0;
        R.rv[k] = 0.0;
        if (s < R.G) {
            R.xv[k] = a.xi[R.g_first + s];
            if constexpr (!PERM) R.rv[k] = a.r[R.g_first + s];
        }
    }
}

// The kernel argument of a step kernel in the kernarg segment (it is the
// first argument, at offset 0).
typedef const __attribute__((address_space(4))) StepArgs* KernargPtr;

// PROBE: the same pairing, but instead of the collisions the largest P_ij of
// every cell goes to a.cell_max (no uniforms drawn, nothing written back).
template <int CAP, int WAVES, bool BATCHED, bool PERM, bool DRY = false, bool PROBE = false>
__global__ __launch_bounds__(WAVES * kWave) void k_wave_groups(const StepArgs a)
{
    using Lds = GroupLds<CAP>;
    constexpr int K = CAP / kWave;   // storage slots per lane
    static_assert(!PROBE || (!BATCHED && !PERM && !DRY), "probe of a single run");
    static_assert(sizeof(CollEntry) * kQueueCap >= 8u * kGroupMaxCells, "probe maxima in the queue");
    __shared__ Lds lds_all[WAVES];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    Lds& L = lds_all[wv];
    // probe mode: per-cell maxima (bit patterns of non-negative doubles) in the
    // otherwise unused collision queue
    unsigned long long* pmax = reinterpret_cast<unsigned long long*>(L.queue);
    const unsigned long long lanes_lt = (1ull << lane) - 1ull;

    const uint32_t blk = a.xcd_remap ? xcd_contiguous_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint64_t wave_id = static_cast<uint64_t>(blk) * WAVES + wv;
    uint64_t g = wave_id * a.groups_per_wave;
    const uint64_t g_stop = g + a.groups_per_wave;
    const uint64_t g_end = g_stop < a.n_groups ? g_stop : static_cast<uint64_t>(a.n_groups);

    uint32_t q_head = 0, q_count = 0;
    unsigned long long pair_acc = 0, coll_acc = 0;
    // software pipeline: the slot offsets of group g + 2 and the slots of
    // group g + 1 are loaded while group g is processed
    GroupRegs<K> R;
    GroupHead Hn;
    if (g < g_end) {
        fetch_head(a, g, lane, Hn);
        fetch_group<K, PERM>(a, Hn, lane, R);
        if (g + 1 < g_end) fetch_head(a, g + 1, lane, Hn);
    }

    for (; g < g_end; ++g) {
        // the kernel's arguments, re-read from the kernarg segment by scalar loads
        // in every group (the pointer is opaque to the compiler), instead of being
        // held in scalar registers across the loop, which spilled them to VGPR
        // lanes (a spill or reload is a VALU instruction)
        KernargPtr kp_ptr = (KernargPtr)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(kp_ptr));
        const StepArgs& a = *(const StepArgs*)kp_ptr;
        const uint32_t c0 = R.c0;
        const uint32_t ncell = R.c1 - c0;
        const uint32_t g_first = R.g_first;
        const uint32_t G = R.G;
        const GroupJob job = resolve_group<BATCHED>(a, c0);

        // (1) live SDs: per-item ballots; live slots before each cell's first slot
        unsigned long long live[K];
        uint32_t n_tot = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            live[k] = __ballot(R.xv[k] != 0);
            n_tot += static_cast<uint32_t>(__popcll(live[k]));
        }
        const uint32_t first = R.o - g_first;                       // lanes < ncell
        uint32_t before = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t kb = static_cast<uint32_t>(k) * kWave;
            if (first >= kb + kWave) before += static_cast<uint32_t>(__popcll(live[k]));
            else if (first > kb) before += static_cast<uint32_t>(__popcll(live[k] & ((1ull << (first - kb)) - 1ull)));
        }
        const uint32_t before_next = __shfl_down(before, 1, kWave);
        const uint32_t first_next = __shfl_down(first, 1, kWave);
        const bool has_cell = lane < ncell;
        const bool last_cell = lane + 1 == ncell;
        const uint32_t nl = has_cell ? ((last_cell ? n_tot : before_next) - before) : 0u;
        const uint32_t n_slots_l = has_cell ? ((last_cell ? G : first_next) - first) : 0u;
        // 2^floor(log2 n) buckets: at most n per cell, so the bucket table of a
        // group fits in CAP entries (a smaller LDS footprint keeps 16 wavefronts
        // per CU resident)
        const uint32_t lgl = nl ? 31u - static_cast<uint32_t>(__clz(static_cast<int>(nl))) : 0u;
        const uint32_t nbl = nl ? (1u << lgl) : 0u;
        const uint32_t calls_l = (n_slots_l + 3u) >> 2;            // Philox calls for the keys
        // one scan for bucket bases (bits 0..10), pair bases (11..19) and call bases (20..27)
        const uint32_t packed = nbl | ((nl >> 1) << 11) | (calls_l << 20);
        const uint32_t incl = wave_inclusive_sum_dpp(packed);
        const uint32_t excl = incl - packed;
        const uint32_t tot = readlane_u32(incl, kWave - 1);
        const uint32_t nb_tot = tot & 2047u;
        const uint32_t q_tot = (tot >> 11) & 511u;
        const uint32_t p_tot = tot >> 20;
        const uint32_t b_base = excl & 2047u;
        const uint32_t q_base = (excl >> 11) & 511u;
        const uint32_t p_base = excl >> 20;
        // uniform deviates: one Philox call per two pairs of a cell
        const uint32_t ucalls_l = ((nl >> 1) + 1u) >> 1;
        const uint32_t u_incl = wave_inclusive_sum_dpp(ucalls_l);
        const uint32_t u_tot = readlane_u32(u_incl, kWave - 1);
        if (has_cell) {
            L.ucb[lane] = u_incl - ucalls_l;
            L.eqn[lane] = before | (q_base << 10) | (nl << 20);
            L.dV[lane] = R.dv;
            L.scale[lane] = nl >= 2 ? upscale_factor_small(nl) : 0.0;
            if constexpr (PERM) a.nlive_out[c0 + lane] = nl;
            if constexpr (PROBE) pmax[lane] = 0ull;
        }
        if (n_tot == 0 || (!PERM && q_tot == 0)) {
            if constexpr (PROBE) {
                if (has_cell) a.cell_max[c0 + lane] = 0.0;
            }
            wave_sync();
            if (g + 1 < g_end) {
                fetch_group<K, PERM>(a, Hn, lane, R);
                if (g + 2 < g_end) fetch_head(a, g + 2, lane, Hn);
            }
            continue;
        }
        // per-slot info and per-call info, one cell at a time
        const uint32_t info_l = lane | (b_base << 8) | (lgl << 24);
        for (uint32_t c = 0; c < ncell; ++c) {
            const uint32_t sb = readlane_u32(first, c);
            const uint32_t sn = readlane_u32(n_slots_l, c);
            const uint32_t info = readlane_u32(info_l, c);
            const uint32_t pb = readlane_u32(p_base, c);
            const uint32_t pn = readlane_u32(calls_l, c);
            for (uint32_t s = lane; s < sn; s += kWave) L.sort.slotinfo[sb + s] = info;
            for (uint32_t q = lane; q < pn; q += kWave) {
                const uint32_t words = (sn - 4 * q) < 4u ? (sn - 4 * q) : 4u;
                L.sort.call[pb + q] = (sb + 4 * q) | (c << 9) | (q << 15) | ((words - 1u) << 22);
            }
        }
        for (uint32_t i = lane; i <= nb_tot; i += kWave) L.sort.start[i] = 0;
        wave_sync();

        // (2) keys: call i draws the four keys of local slots 4q..4q+3 of its cell
        for (uint32_t i = lane; i < p_tot; i += kWave) {
            const uint32_t ci = L.sort.call[i];
            const uint32_t base = ci & 511u;
            const uint32_t c = (ci >> 9) & 63u;
            const uint32_t q = (ci >> 15) & 127u;
            const uint32_t words = (ci >> 22) + 1u;
            const Words4 w = philox4x32_10(q, job.rng_base + c, job.step, kTagShuffle, job.k0, job.k1);
#pragma unroll
            for (uint32_t t = 0; t < 4; ++t)
                if (t < words) L.sort.keys[base + t] = w.w[t];
        }
        wave_sync();

        // bucket counts
        uint32_t key[K], bkt[K], arr[K], cid[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            key[k] = 0;
            bkt[k] = 0;
            arr[k] = 0;
            cid[k] = 0;
            if (R.xv[k] != 0) {
                const uint32_t s = lane + k * kWave;
                const uint32_t si = L.sort.slotinfo[s];
                key[k] = L.sort.keys[s];
                cid[k] = si & 255u;
                bkt[k] = ((si >> 8) & 2047u) + bucket_of(key[k], si >> 24);
                arr[k] = atomicAdd(&L.sort.start[bkt[k]], 1u);
            }
        }
        wave_sync();

        // exclusive scan of the nb_tot bucket counts; start[nb_tot] = n_tot
        {
            const uint32_t per = (nb_tot + kWave - 1) / kWave;   // <= K
            const uint32_t base = lane * per;
            uint32_t v[K];
            uint32_t sum = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) {
                v[t] = 0;
                if (static_cast<uint32_t>(t) < per && base + t < nb_tot) v[t] = L.sort.start[base + t];
                sum += v[t];
            }
            const uint32_t inc = wave_inclusive_sum_dpp(sum);
            uint32_t run = inc - sum;
#pragma unroll
            for (int t = 0; t < K; ++t) {
                if (static_cast<uint32_t>(t) < per && base + t < nb_tot) L.sort.start[base + t] = run;
                run += v[t];
            }
            if (lane == kWave - 1) L.sort.start[nb_tot] = inc;
        }
        wave_sync();

        // scatter (key, slot) to bucket start + arrival
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (R.xv[k] != 0)
                L.sort.kv[L.sort.start[bkt[k]] + arr[k]] =
                    (static_cast<uint64_t>(key[k]) << 32) | (lane + k * kWave);
        wave_sync();

        // rank inside the bucket by full (key, slot) comparison
        uint32_t pos[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            pos[k] = static_cast<uint32_t>(CAP);
            if (R.xv[k] != 0) {
                const uint32_t lo = L.sort.start[bkt[k]];
                const uint32_t hi = L.sort.start[bkt[k] + 1];
                const uint64_t me = (static_cast<uint64_t>(key[k]) << 32) | (lane + k * kWave);
                uint32_t rank = 0;
                for (uint32_t e = lo; e < hi; ++e) rank += (L.sort.kv[e] < me) ? 1u : 0u;
                pos[k] = lo + rank;
            }
        }
        wave_sync();   // the sort arrays are overwritten below

        // (3) place the live SDs in sorted order; note the first member of each pair
        if constexpr (!PERM) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (R.xv[k] != 0) {
                    const uint32_t s = lane + k * kWave;
                    const uint32_t p = pos[k];
                    const uint32_t eqn = L.eqn[cid[k]];
                    const uint32_t loc = p - (eqn & 1023u);
                    const uint32_t n_c = eqn >> 20;
                    L.pairs.xi[p] = R.xv[k];
                    L.pairs.r[p] = R.rv[k];
                    L.pairs.slot[p] = static_cast<uint16_t>(s);
                    if (!(loc & 1u) && loc + 1 < n_c) {
                        const uint32_t q = ((eqn >> 10) & 1023u) + (loc >> 1);
                        L.pairs.pairinfo[q] = static_cast<uint16_t>(p | (cid[k] << 10));
                        if (!(loc & 3u))   // first pair of a uniform call
                            L.pairs.ucall[L.ucb[cid[k]] + (loc >> 2)] =
                                q | (cid[k] << 9) | ((loc >> 2) << 15) | ((loc + 3 < n_c ? 1u : 0u) << 23);
                    }
                }
            }
        }
        if constexpr (PERM) {
            // local slot of the SD at sorted position loc of its cell
#pragma unroll
            for (int k = 0; k < K; ++k) {
                // the shuffle runs with every lane active (an inactive source lane reads as 0)
                const uint32_t cell_first = __shfl(first, cid[k], kWave);
                if (R.xv[k] != 0) {
                    const uint32_t s = lane + k * kWave;
                    const uint32_t eqn = L.eqn[cid[k]];
                    const uint32_t loc = pos[k] - (eqn & 1023u);
                    a.perm_out[g_first + cell_first + loc] = s - cell_first;
                }
            }
        }
        wave_sync();
        // the registers of this group are free: start loading the next one
        if (g + 1 < g_end) {
            fetch_group<K, PERM>(a, Hn, lane, R);
            if (g + 2 < g_end) fetch_head(a, g + 2, lane, Hn);
        }
        if constexpr (PERM) continue;

        // (4) uniform deviates, two pairs per Philox call
        for (uint32_t i = lane; !PROBE && i < u_tot; i += kWave) {
            const uint32_t uc = L.pairs.ucall[i];
            const uint32_t q = uc & 511u;
            const uint32_t c = (uc >> 9) & 63u;
            const uint32_t h = (uc >> 15) & 255u;
            const Words4 w = philox4x32_10(h, job.rng_base + c, job.step, kTagUniform, job.k0, job.k1);
            L.pairs.u[q] = uniform_open01(w.w[0], w.w[1]);
            if (uc >> 23) L.pairs.u[q + 1] = uniform_open01(w.w[2], w.w[3]);
        }
        wave_sync();

        if constexpr (PROBE) {
            // (5') P_ij of every pair; the largest per cell
            for (uint32_t q = lane; q < q_tot; q += kWave) {
                const uint32_t pi = L.pairs.pairinfo[q];
                const uint32_t p = pi & 1023u;
                const uint32_t c = pi >> 10;
                const uint64_t xa = L.pairs.xi[p], xb = L.pairs.xi[p + 1];
                const double Kab = collection_kernel(job.kernel, job.kp, L.pairs.r[p], L.pairs.r[p + 1]);
                const double prob =
                    collision_probability(xa >= xb ? xa : xb, Kab, job.dt, L.dV[c], L.scale[c]);
                atomicMax(&pmax[c], static_cast<unsigned long long>(__double_as_longlong(prob)));
            }
            wave_sync();
            if (has_cell) a.cell_max[c0 + lane] = __longlong_as_double(static_cast<long long>(pmax[lane]));
            wave_sync();   // the maxima are read before the next group clears them
            continue;
        }

        // (5) pair tests; colliding pairs go to the queue
        uint32_t coll = 0;
        for (uint32_t qb = 0; qb < q_tot; qb += kWave) {
            const uint32_t q = qb + lane;
            uint64_t gam = 0;
            uint32_t gj = 0, gk = 0;
            if (q < q_tot) {
                const uint32_t pi = L.pairs.pairinfo[q];
                const uint32_t p = pi & 1023u;
                const uint32_t c = pi >> 10;
                const uint32_t sa = L.pairs.slot[p], sb = L.pairs.slot[p + 1];
                const uint64_t xa = L.pairs.xi[p], xb = L.pairs.xi[p + 1];
                const double ra = L.pairs.r[p], rb = L.pairs.r[p + 1];
                const double u = L.pairs.u[q];
                const double Kab = collection_kernel(job.kernel, job.kp, ra, rb);
                const bool a_is_j = xa >= xb;
                const uint64_t xj = a_is_j ? xa : xb;
                const uint64_t xk = a_is_j ? xb : xa;
                const double prob = collision_probability(xj, Kab, job.dt, L.dV[c], L.scale[c]);
                // the release rule is the capped count of min(P_ij, 1)
                gam = collision_count((a.rules & kRuleRelease) ? fmin(prob, 1.0) : prob, u, xj, xk);
                gj = g_first + (a_is_j ? sa : sb);
                gk = g_first + (a_is_j ? sb : sa);
            }
            const unsigned long long hit = __ballot(gam != 0);
            if (gam != 0) {
                const uint32_t idx =
                    (q_head + q_count + static_cast<uint32_t>(__popcll(hit & lanes_lt))) % kQueueCap;
                L.queue[idx].gj = gj;
                L.queue[idx].gk = gk;
                L.queue[idx].g = gam;
            }
            const uint32_t nh = static_cast<uint32_t>(__popcll(hit));
            q_count += nh;
            coll += nh;
            if (q_count >= static_cast<uint32_t>(kWave)) {
                wave_sync();
                flush_collisions<DRY>(a, L.queue, q_head, kWave, lane);
                q_head = (q_head + kWave) % kQueueCap;
                q_count -= kWave;
                wave_sync();
            }
        }
        wave_sync();   // pair reads done before the next group reuses the LDS
        if constexpr (BATCHED) {
            if (lane == 0) add_counts(a, true, job.inst, 0, q_tot, coll);
        } else {
            pair_acc += q_tot;
            coll_acc += coll;
        }
    }
    if constexpr (!PERM && !PROBE) {
        if (q_count > 0) {
            wave_sync();
            flush_collisions<DRY>(a, L.queue, q_head, q_count, lane);
        }
    }
    if constexpr (!BATCHED && !PERM && !PROBE) {
        if (lane == 0 && (pair_acc || coll_acc))
            add_counts(a, false, 0, static_cast<uint32_t>(wave_id), pair_acc, coll_acc);
    }
}

// Sum of v over a workgroup of BLOCK threads (every thread gets it).
template <int BLOCK>
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* s_red)
{
    constexpr int W = BLOCK / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane == 0) s_red[wv] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) t += s_red[w];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// Grid tier: every cell with more storage slots than a wave-tier group holds,
// each spread over many workgroups.  The order by (key, slot) is found in two
// levels:
//   coarse: each slot chunk counts the digits (top cb key bits) of its live
//     slots in LDS into its column of a digit-major count table; after an
//     exclusive scan of the table every (digit, chunk) run has its place, and
//     each chunk writes its (key, slot) words there, so that every digit bucket
//     (about 512 to 1024 entries) is contiguous and the buckets are in order;
//   fine: one workgroup per bucket splits it by the next key bits into
//     sub-buckets of one or two entries on average, in LDS, ranks each entry
//     within its sub-bucket, and tests the pairs that lie inside the bucket
//     (their multiplicities and radii gathered from the state by slot).
// A pair that straddles two buckets (an odd first sorted position) is left to
// a last launch, one thread per bucket, from the two slots the bucket
// workgroups leave at those positions.  The launches cover all grid cells at
// once: digit counts -> table tile sums -> per-cell scan of the tile sums ->
// table tile scans -> placement -> bucket sorts with their pair tests ->
// straddling pairs.  Same order and results as the other tiers.
// ---------------------------------------------------------------------------
constexpr int kGridBlock = 256;
constexpr uint32_t kGridChunkLg = 11;     // smallest slot chunk, 2048 slots
constexpr uint32_t kGridChunk = 1u << kGridChunkLg;
constexpr uint32_t kGridBucketLg = 10;    // cb = ceil(log2 N) - 10: <= 1024 per bucket on average
constexpr uint32_t kGridMaxDigitBits = 12;
constexpr uint32_t kGridMaxDigits = 1u << kGridMaxDigitBits;
constexpr uint32_t kGridTile = 4096;      // table entries per tile
constexpr uint32_t kGridSortCap = 2048;   // larger buckets are ordered through scr_tmp
constexpr uint32_t kGridSubLg = 10;       // at most 2^10 sub-buckets per bucket
// placement through LDS: chunks of kGridChunk slots with at most this many digits
// (cells of up to 2^20 slots have at most 2^10)
constexpr uint32_t kGridStagedDigits = 1024;

// Digit counts (PLACE = false) or placement (PLACE = true) of one slot chunk.
// The order within a (digit, chunk) run is arrival order and does not matter:
// the bucket sort orders it exactly.  A chunk of at most kGridChunk slots is
// placed through LDS: its words are first grouped by digit there (local runs at
// the exclusive scan of the chunk's digit counts) and then copied out, so that
// consecutive threads write consecutive words of a run instead of each word
// being a memory request of its own.  Larger chunks place every word straight
// at its digit's cursor.
// The slots go in rounds of kGridQuads quads of four per thread (one round for
// a chunk of kGridChunk slots).  The first round's multiplicities are requested
// as soon as the cell's offset is known; its keys are drawn and the LDS
// counters set up while they are in flight.
constexpr uint32_t kGridQuads = kGridChunk / (4 * kGridBlock);

// LDS bytes of k_grid_digits for grid cells of at most dmax digits: the D
// counters of a chunk, and when placing also its local cursors and its staged
// words (past grid_dcap counters and cursors), over the same bytes.
inline uint32_t grid_digits_lds(bool place, uint32_t dmax, uint32_t dcap)
{
    const uint32_t direct = dmax * 4u;
    const uint32_t staged = place ? dcap * 8u + kGridChunk * 8u : 0u;
    return direct > staged ? direct : staged;
}

template <bool BATCHED, bool PLACE>
__global__ __launch_bounds__(kGridBlock) void k_grid_digits(const StepArgs a)
{
    static_assert(kGridQuads * 4 * kGridBlock == kGridChunk, "one round per smallest chunk");
    extern __shared__ uint64_t s_raw[];   // grid_digits_lds(PLACE, ...) bytes
    __shared__ uint32_t s_red[kGridBlock / kWave];
    const uint4 ch = a.gchunk[blockIdx.x];
    const uint32_t off = a.off_begin[ch.z];
    const uint32_t n_slots = a.off_end[ch.z] - off;
    const GridCell& gc = a.gcell[ch.x];
    const uint32_t s_end = min(ch.y + (1u << gc.lgc), n_slots);
    const uint32_t q_end = (s_end + 3u) / 4u;
    const uint32_t q_first = ch.y / 4u + threadIdx.x;
    const uint64_t* xi = a.xi + off;
    uint64_t xv[kGridQuads][4];
    const auto load_round = [&](uint32_t q0) {
#pragma unroll
        for (uint32_t i = 0; i < kGridQuads; ++i) {
            const uint32_t q = q0 + i * kGridBlock;
#pragma unroll
            for (uint32_t t = 0; t < 4; ++t) {
                // branch-free: every load in flight together (the index is
                // clamped to the chunk's last slot; s_end > ch.y)
                const uint32_t sl = 4 * q + t;
                const uint64_t v = xi[sl < s_end ? sl : s_end - 1u];
                xv[i][t] = sl < s_end ? v : 0u;
            }
        }
    };
    load_round(q_first);

    const CellJob j = resolve_cell<BATCHED>(a, ch.z);
    const uint32_t cb = gc.cb, D = 1u << cb, ncol = gc.ncol, col = ch.y >> gc.lgc;
    Words4 kw[kGridQuads];
    const auto draw_round = [&](uint32_t q0) {
#pragma unroll
        for (uint32_t i = 0; i < kGridQuads; ++i)
            kw[i] = philox4x32_10(q0 + i * kGridBlock, j.rng_cell, j.step, kTagShuffle, j.k0, j.k1);
    };
    draw_round(q_first);

    uint32_t* tbl = a.scr_cnt + j.off;
    // uniform over the workgroup
    const bool staged = PLACE && gc.lgc == kGridChunkLg && D <= a.grid_dcap;
    uint32_t* s_cnt = reinterpret_cast<uint32_t*>(s_raw);
    uint32_t* s_loc = s_cnt + a.grid_dcap;   // staged only
    uint64_t* s_stage = s_raw + a.grid_dcap;  // staged only (past both counter arrays)
    uint32_t m_chunk = 0;                                   // staged: the chunk's live words
    if (staged) {
        // run (d, col) starts at tbl[i] and holds tbl[i + 1] - tbl[i] words,
        // i = d ncol + col (entry nb is the sentinel); thread t scans a run of
        // `per` digits, then the waves' totals
        constexpr int W = kGridBlock / kWave;
        const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
        const uint32_t per = (D + kGridBlock - 1) / kGridBlock;
        const uint32_t d0 = min(threadIdx.x * per, D), d1 = min(d0 + per, D);
        uint32_t run = 0;
        for (uint32_t d = d0; d < d1; ++d) {
            const uint32_t i = d * ncol + col;
            const uint32_t g = tbl[i];
            const uint32_t c = tbl[i + 1] - g;
            s_cnt[d] = g;
            s_loc[d] = c;
            run += c;
        }
        const uint32_t incl = wave_inclusive_sum(run, lane);
        if (lane == kWave - 1) s_red[wv] = incl;
        __syncthreads();
        uint32_t before = incl - run;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            before += static_cast<uint32_t>(w) < wv ? s_red[w] : 0u;
            m_chunk += s_red[w];
        }
        // s_loc: local cursor from the run's local start; s_cnt: global start
        // minus local start, so that local index + s_cnt is the global place
        for (uint32_t d = d0; d < d1; ++d) {
            const uint32_t c = s_loc[d];
            s_loc[d] = before;
            s_cnt[d] -= before;
            before += c;
        }
    } else {
        for (uint32_t d = threadIdx.x; d < D; d += kGridBlock) s_cnt[d] = PLACE ? tbl[d * ncol + col] : 0u;
    }
    __syncthreads();
    for (uint32_t q0 = q_first; q0 < q_end; q0 += kGridQuads * kGridBlock) {
        if (q0 != q_first) {
            load_round(q0);
            draw_round(q0);
        }
#pragma unroll
        for (uint32_t i = 0; i < kGridQuads; ++i) {
            const uint32_t q = q0 + i * kGridBlock;
#pragma unroll
            for (uint32_t t = 0; t < 4; ++t) {
                if (xv[i][t] == 0u) continue;   // dead, or past the chunk (read as 0)
                const uint32_t d = bucket_of(kw[i].w[t], cb);
                if constexpr (PLACE) {
                    const uint64_t word = (static_cast<uint64_t>(kw[i].w[t]) << 32) | (4 * q + t);
                    if (staged) {
                        s_stage[atomicAdd(&s_loc[d], 1u)] = word;   // < m_chunk <= kGridChunk
                    } else {
                        const uint32_t p = atomicAdd(&s_cnt[d], 1u);
                        a.scr_kv[j.off + p] = word;
                    }
                } else {
                    atomicAdd(&s_cnt[d], 1u);
                }
            }
        }
    }
    if constexpr (PLACE) {
        if (staged) {
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < m_chunk; i += kGridBlock) {
                const uint64_t v = s_stage[i];
                a.scr_kv[j.off + s_cnt[bucket_of(static_cast<uint32_t>(v >> 32), cb)] + i] = v;
            }
        }
    } else {
        __syncthreads();
        for (uint32_t d = threadIdx.x; d < D; d += kGridBlock) tbl[d * ncol + col] = s_cnt[d];
    }
}

static __global__ __launch_bounds__(kGridBlock) void k_grid_tile_sums(const StepArgs a)
{
    __shared__ uint32_t s_red[kGridBlock / kWave];
    const uint2 t = a.gtile[blockIdx.x];
    const GridCell& gc = a.gcell[t.x];
    const uint32_t off = a.off_begin[gc.cell];
    const uint32_t end = min(t.y + kGridTile, gc.nb);
    uint32_t sum = 0;
    for (uint32_t b = t.y + threadIdx.x; b < end; b += kGridBlock) sum += a.scr_cnt[off + b];
    const uint32_t tot = block_sum<kGridBlock>(sum, s_red);
    if (threadIdx.x == 0) a.gtilesum[blockIdx.x] = tot;
}

// one thread per grid cell: exclusive scan of its tile sums; sentinel = live count
template <bool BATCHED>
__global__ __launch_bounds__(kGridBlock) void k_grid_tile_offsets(const StepArgs a)
{
    for (uint32_t i = blockIdx.x * kGridBlock + threadIdx.x; i < a.n_grid; i += gridDim.x * kGridBlock) {
        GridCell& gc = a.gcell[i];
        uint32_t run = 0;
        for (uint32_t t = 0; t < gc.ntiles; ++t) {
            const uint32_t v = a.gtilesum[gc.tile0 + t];
            a.gtilesum[gc.tile0 + t] = run;
            run += v;
        }
        a.scr_cnt[a.off_begin[gc.cell] + gc.nb] = run;
        gc.live = run;
        const unsigned long long pairs = run >> 1;
        if constexpr (BATCHED) {
            if (pairs) atomicAdd(&a.inst[a.cell_inst[gc.cell]].pair_tests, pairs);
        } else {
            if (pairs && a.stats) atomicAdd(a.stats + (i % kStatSlots) * kStatStride, pairs);
        }
    }
}

static __global__ __launch_bounds__(kGridBlock) void k_grid_tile_scan(const StepArgs a)
{
    __shared__ uint32_t s_red[kGridBlock / kWave];
    constexpr int W = kGridBlock / kWave;
    const uint2 t = a.gtile[blockIdx.x];
    const GridCell& gc = a.gcell[t.x];
    const uint32_t off = a.off_begin[gc.cell];
    const uint32_t end = min(t.y + kGridTile, gc.nb);
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint32_t carry = a.gtilesum[blockIdx.x];
    for (uint32_t base = t.y; base < end; base += kGridBlock) {
        const uint32_t b = base + threadIdx.x;
        const uint32_t v = b < end ? a.scr_cnt[off + b] : 0u;
        const uint32_t incl_w = wave_inclusive_sum(v, lane);
        if (lane == kWave - 1) s_red[wv] = incl_w;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t x = s_red[w];
            before += (static_cast<uint32_t>(w) < wv) ? x : 0u;
            total += x;
        }
        if (b < end) a.scr_cnt[off + b] = carry + before + incl_w - v;
        carry += total;
        __syncthreads();
    }
}

struct GridFuseLds {
    union {                                 // (a smaller footprint: more workgroups per CU)
        uint64_t kv[kGridSortCap];          // (key << 32 | slot) grouped by sub-bucket
        uint32_t slot[kGridSortCap];        // then the storage slot at each sorted position
    };
    uint32_t sub[(1u << kGridSubLg) + 1];   // sub-bucket counts, then starts; [S] = M
    uint32_t red[kGridBlock / kWave];
    double dmax[kGridBlock / kWave];
};

// Pair test of the sorted positions (2m, 2m + 1) of a grid cell whose slots are
// sa, sb: the state is read by slot (no pair of this step has changed them).
template <bool PROBE>
__device__ __forceinline__ bool grid_pair(const StepArgs& a, const CellJob& j, double scale,
                                          uint32_t m, uint32_t sa, uint32_t sb, double& best)
{
    const uint64_t xa = a.xi[j.off + sa], xb = a.xi[j.off + sb];
    const double ra = a.r[j.off + sa], rb = a.r[j.off + sb];
    if constexpr (PROBE) {
        const double K = collection_kernel(j.kernel, j.kp, ra, rb);
        best = fmax(best, collision_probability(xa >= xb ? xa : xb, K, j.dt, j.dV, scale));
        return false;
    } else {
        const Words4 w = philox4x32_10(m >> 1, j.rng_cell, j.step, kTagUniform, j.k0, j.k1);
        const double u = (m & 1u) ? uniform_open01(w.w[2], w.w[3]) : uniform_open01(w.w[0], w.w[1]);
        return collide_pair_global(a, j, scale, u, sa, sb, xa, xb, ra, rb);
    }
}

// One workgroup per digit bucket: the exact order of its entries, then the
// pair tests of the pairs with both members in it.  Up to kGridSortCap entries
// are ordered in LDS; a larger bucket (cells of more than about 2^22 slots) is
// ordered through its scr_tmp range and its order written to scr_pos.  The
// bucket's first entry when its sorted position is odd, and its last when that
// position is even and has a successor, leave their slot at their position in
// scr_pos for k_grid_boundary.  Buckets of one cell are consecutive in the
// list and go to one XCD, so that the gathers of a cell share its L2.
template <bool BATCHED, bool PERM, bool PROBE = false>
__global__ __launch_bounds__(kGridBlock) void k_grid_bucket_pairs(const StepArgs a)
{
    constexpr int T = kGridBlock;
    constexpr int K = kGridSortCap / T;
    constexpr int W = T / kWave;
    __shared__ GridFuseLds L;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const uint4 gb = a.gbucket[xcd_contiguous_block(blockIdx.x, gridDim.x)];
    const GridCell& gc = a.gcell[gb.x];
    const CellJob j = resolve_cell<BATCHED>(a, gb.z);
    const uint64_t off = j.off;
    const uint32_t lo = a.scr_cnt[off + gb.y * gc.ncol];
    const uint32_t M = a.scr_cnt[off + (gb.y + 1) * gc.ncol] - lo;   // entry nb is the sentinel
    const uint32_t n = gc.live;
    if constexpr (PERM) {
        if (gb.y == 0 && tid == 0) a.nlive_out[gc.cell] = n;
    }
    if (M == 0) return;
    const uint32_t cb = gc.cb;
    const uint32_t sb = M >= 2 ? min(ceil_log2(M) - 1u, kGridSubLg) : 0u;
    const uint32_t S = 1u << sb;
    const auto sub_of = [cb, sb](uint64_t v) {
        return bucket_of(static_cast<uint32_t>(v >> 32) << cb, sb);
    };
    const bool in_lds = M <= kGridSortCap;
    const uint64_t* src = a.scr_kv + off + lo;
    uint32_t* pos_g = a.scr_pos + off;   // indexed by sorted position within the cell
    for (uint32_t b = tid; b <= S; b += T) L.sub[b] = 0;

    uint64_t kv[K];
    uint32_t arr[K];
    if (in_lds) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t i = tid + static_cast<uint32_t>(k) * T;
            kv[k] = i < M ? src[i] : 0u;
        }
    }
    __syncthreads();
    if (in_lds) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t i = tid + static_cast<uint32_t>(k) * T;
            arr[k] = i < M ? atomicAdd(&L.sub[sub_of(kv[k])], 1u) : 0u;
        }
    } else {
        for (uint32_t i = tid; i < M; i += T) atomicAdd(&L.sub[sub_of(src[i])], 1u);
    }
    __syncthreads();
    // exclusive scan of L.sub[0, S): thread t owns a run of `per` entries
    {
        const uint32_t per = (S + T - 1) / T;
        const uint32_t b0 = min(tid * per, S), b1 = min(b0 + per, S);
        uint32_t run = 0;
        for (uint32_t b = b0; b < b1; ++b) run += L.sub[b];
        const uint32_t incl = wave_inclusive_sum_dpp(run);
        if (lane == kWave - 1) L.red[wv] = incl;
        __syncthreads();
        uint32_t before = incl - run;
#pragma unroll
        for (int w = 0; w < W; ++w) before += static_cast<uint32_t>(w) < wv ? L.red[w] : 0u;
        for (uint32_t b = b0; b < b1; ++b) {
            const uint32_t c = L.sub[b];
            L.sub[b] = before;
            before += c;
        }
        if (tid == 0) L.sub[S] = M;
        __syncthreads();
    }

    if (in_lds) {
        // scatter by sub-bucket start + arrival, then the rank in the sub-bucket
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (tid + static_cast<uint32_t>(k) * T < M) L.kv[L.sub[sub_of(kv[k])] + arr[k]] = kv[k];
        __syncthreads();
        uint32_t pk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            pk[k] = 0;
            if (tid + static_cast<uint32_t>(k) * T >= M) continue;
            const uint32_t b = sub_of(kv[k]);
            const uint32_t e0 = L.sub[b], e1 = L.sub[b + 1];
            uint32_t rank = 0;
            for (uint32_t e = e0; e < e1; ++e) rank += L.kv[e] < kv[k] ? 1u : 0u;
            pk[k] = e0 + rank;
        }
        __syncthreads();   // the slots overwrite the sort array
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (tid + static_cast<uint32_t>(k) * T >= M) continue;
            const uint32_t p = pk[k];
            const uint32_t slot = static_cast<uint32_t>(kv[k]);
            if constexpr (PERM) {
                a.perm_out[off + lo + p] = slot;
            } else {
                L.slot[p] = slot;
                const uint32_t P = lo + p;
                if ((p == 0 && (P & 1u)) || (p == M - 1 && !(P & 1u) && P + 1 < n)) pos_g[P] = slot;
            }
        }
        if constexpr (PERM) return;
    } else {
        // through global memory: place by sub-bucket into scr_tmp, rank, and
        // write the slot of every sorted position to scr_pos
        uint64_t* dst = a.scr_tmp + off + lo;
        for (uint32_t i = tid; i < M; i += T) {
            const uint64_t v = src[i];
            dst[atomicAdd(&L.sub[sub_of(v)], 1u)] = v;
        }
        __syncthreads();   // L.sub[b] now ends sub-bucket b
        for (uint32_t i = tid; i < M; i += T) {
            const uint64_t v = dst[i];
            const uint32_t b = sub_of(v);
            const uint32_t e0 = b ? L.sub[b - 1] : 0u, e1 = L.sub[b];
            uint32_t rank = 0;
            for (uint32_t e = e0; e < e1; ++e) rank += dst[e] < v ? 1u : 0u;
            pos_g[lo + e0 + rank] = static_cast<uint32_t>(v);
        }
        __syncthreads();
        if constexpr (PERM) {
            for (uint32_t i = tid; i < M; i += T) a.perm_out[off + lo + i] = pos_g[lo + i];
            return;
        }
    }
    __syncthreads();

    // pairs (2m, 2m + 1) with both members in the bucket: m in [m_a, m_b)
    const uint32_t m_a = (lo + 1u) >> 1, m_b = (lo + M) >> 1;
    const double scale = n >= 2 ? upscale_factor(n) : 0.0;
    uint32_t coll = 0;
    double best = 0.0;
    // slots[p - first] is the slot at sorted position p of the cell; the branch
    // on in_lds is uniform, so that the LDS case reads the slots as LDS (a
    // pointer that may be either is a flat access, whose wait also covers the
    // stores)
    const auto run_pairs = [&](const uint32_t* slots, uint32_t first) {
        for (uint32_t m = m_a + tid; m < m_b; m += T)
            if (grid_pair<PROBE>(a, j, scale, m, slots[2 * m - first], slots[2 * m + 1 - first], best))
                ++coll;
    };
    if (in_lds) run_pairs(L.slot, lo);
    else run_pairs(pos_g, 0u);
    if constexpr (PROBE) {
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) best = fmax(best, __shfl_xor(best, d, kWave));
        if (lane == 0) L.dmax[wv] = best;
        __syncthreads();
        if (tid == 0) {
            double b = L.dmax[0];
            for (int w = 1; w < W; ++w) b = fmax(b, L.dmax[w]);
            if (b > 0.0)
                atomicMax(reinterpret_cast<unsigned long long*>(a.cell_max + gc.cell),
                          static_cast<unsigned long long>(__double_as_longlong(b)));
        }
        return;
    }
    const uint32_t tot = block_sum<T>(coll, L.red);
    if (tid == 0 && tot) {
        if constexpr (BATCHED) atomicAdd(&a.inst[j.inst].collisions, static_cast<unsigned long long>(tot));
        else atomicAdd(a.stats + (blockIdx.x % kStatSlots) * kStatStride + 1, static_cast<unsigned long long>(tot));
    }
}

// The pairs that straddle two digit buckets: one thread per bucket whose first
// sorted position lo is odd tests the pair (lo - 1, lo) from the slots the
// bucket workgroups left in scr_pos.
template <bool BATCHED, bool PROBE = false>
__global__ __launch_bounds__(kGridBlock) void k_grid_boundary(const StepArgs a)
{
    __shared__ uint32_t s_red[kGridBlock / kWave];
    const uint32_t i = blockIdx.x * kGridBlock + threadIdx.x;
    uint32_t coll = 0;
    if (i < a.n_gbucket) {
        const uint4 gb = a.gbucket[i];
        const GridCell& gc = a.gcell[gb.x];
        const uint64_t off = a.off_begin[gb.z];
        const uint32_t lo = a.scr_cnt[off + gb.y * gc.ncol];
        const uint32_t hi = a.scr_cnt[off + (gb.y + 1) * gc.ncol];
        if (hi > lo && (lo & 1u)) {
            const CellJob j = resolve_cell<BATCHED>(a, gc.cell);
            const double scale = upscale_factor(gc.live);
            const uint32_t sa = a.scr_pos[off + lo - 1], sb = a.scr_pos[off + lo];
            double best = 0.0;
            if (grid_pair<PROBE>(a, j, scale, (lo - 1u) >> 1, sa, sb, best)) {
                if constexpr (BATCHED) atomicAdd(&a.inst[j.inst].collisions, 1ull);
                else ++coll;
            }
            if constexpr (PROBE) {
                if (best > 0.0)
                    atomicMax(reinterpret_cast<unsigned long long*>(a.cell_max + gc.cell),
                              static_cast<unsigned long long>(__double_as_longlong(best)));
            }
        }
    }
    if constexpr (!BATCHED && !PROBE) {
        const uint32_t tot = block_sum<kGridBlock>(coll, s_red);
        if (threadIdx.x == 0 && tot)
            atomicAdd(a.stats + (blockIdx.x % kStatSlots) * kStatStride + 1, static_cast<unsigned long long>(tot));
    }
}

// ---------------------------------------------------------------------------
// Workgroup tier: one workgroup per cell of up to CAPB storage slots (more than
// a wavefront group takes), the whole order by (key, slot) in LDS, then the
// pair tests, in one launch over all such cells.  The sort is the wavefront
// tier's: one most-significant-digit pass over 2^floor(log2 n) buckets with
// LDS atomics, an exclusive scan, a scatter by (bucket start + arrival) and a
// rank inside each bucket by full (key, slot) comparison.  The cells come
// largest first, so that the long ones start early (longest-processing-time
// order); each workgroup reads its cell's xi once, coalesced, and gathers
// xi and r of the pair members from L2.
// ---------------------------------------------------------------------------
constexpr uint32_t kBlockSmall = 2048;   // cells up to here take 256-thread workgroups
constexpr uint32_t kBlockLarge = 8192;   // and up to here 1024-thread ones

template <int CAPB, int T>
struct BlockLds {
    static_assert(CAPB <= 65536, "slots are 16-bit");
    union {
        struct {
            uint64_t kv[CAPB];          // (key << 32 | slot) grouped by bucket
            uint32_t start[CAPB + 1];   // bucket counts, then bucket starts; start[nb] = n
            uint32_t keys[CAPB];        // shuffle key of every slot
        } sort;
        struct {
            uint64_t xi[CAPB];          // live SDs in sorted order
            double r[CAPB];
        } pairs;
    };
    uint16_t slot[CAPB];                // storage slot at each sorted position
    uint32_t red[T / kWave];
    double dmax[T / kWave];
};

template <int CAPB, int T, bool BATCHED, bool PERM, bool PROBE = false>
__global__ __launch_bounds__(T) void k_block_cells(const StepArgs a, const uint32_t* list)
{
    constexpr int K = CAPB / T;   // storage slots per thread
    constexpr int W = T / kWave;
    static_assert(CAPB % T == 0 && T % kWave == 0, "block shape");
    static_assert(!PROBE || (!BATCHED && !PERM), "probe of a single run");
    __shared__ BlockLds<CAPB, T> L;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const uint32_t c = load_const_u32(list, blockIdx.x);
    const CellJob j = resolve_cell<BATCHED>(a, c);
    const uint32_t M = j.n_slots;   // <= CAPB

    // (1) xi and r (coalesced), the live count, and the shuffle keys of all
    // slots (four per Philox call)
    uint64_t xv[K];
    double rv[K];
    uint32_t live_cnt = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t s = tid + static_cast<uint32_t>(k) * T;
        xv[k] = 0u;
        rv[k] = 0.0;
        if (s < M) {
            xv[k] = a.xi[j.off + s];
            if constexpr (!PERM) rv[k] = a.r[j.off + s];
        }
        live_cnt += xv[k] != 0u ? 1u : 0u;
    }
    for (uint32_t q = tid; 4 * q < M; q += T) {
        const Words4 w = philox4x32_10(q, j.rng_cell, j.step, kTagShuffle, j.k0, j.k1);
#pragma unroll
        for (uint32_t t = 0; t < 4; ++t)
            if (4 * q + t < M) L.sort.keys[4 * q + t] = w.w[t];
    }
    const uint32_t n = block_sum<T>(live_cnt, L.red);   // also orders the key writes
    if (n == 0) {
        if (tid == 0) {
            if constexpr (PERM) a.nlive_out[c] = 0;
            if constexpr (PROBE) a.cell_max[c] = 0.0;
        }
        return;
    }
    const uint32_t lg = 31u - static_cast<uint32_t>(__clz(static_cast<int>(n)));
    const uint32_t nb = 1u << lg;
    for (uint32_t i = tid; i <= nb; i += T) L.sort.start[i] = 0;
    __syncthreads();

    // (2) bucket counts on the top lg key bits
    uint32_t key[K], bkt[K], arr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        key[k] = 0;
        bkt[k] = 0;
        arr[k] = 0;
        if (xv[k] != 0u) {
            const uint32_t s = tid + static_cast<uint32_t>(k) * T;
            key[k] = L.sort.keys[s];
            bkt[k] = bucket_of(key[k], lg);
            arr[k] = atomicAdd(&L.sort.start[bkt[k]], 1u);
        }
    }
    __syncthreads();

    // (3) exclusive scan of the nb counts (thread t owns a run of `per`); start[nb] = n
    {
        const uint32_t per = (nb + T - 1) / T;
        const uint32_t b0 = tid * per;
        const uint32_t b1 = b0 + per < nb ? b0 + per : nb;
        uint32_t run = 0;
        for (uint32_t b = b0; b < b1; ++b) run += L.sort.start[b];
        const uint32_t incl = wave_inclusive_sum_dpp(run);
        if (lane == kWave - 1) L.red[wv] = incl;
        __syncthreads();
        uint32_t before = incl - run;
#pragma unroll
        for (int w = 0; w < W; ++w) before += static_cast<uint32_t>(w) < wv ? L.red[w] : 0u;
        for (uint32_t b = b0; b < b1; ++b) {
            const uint32_t cnt = L.sort.start[b];
            L.sort.start[b] = before;
            before += cnt;
        }
        if (tid == 0) L.sort.start[nb] = n;
    }
    __syncthreads();

    // (4) scatter (key, slot) to bucket start + arrival
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (xv[k] != 0u)
            L.sort.kv[L.sort.start[bkt[k]] + arr[k]] =
                (static_cast<uint64_t>(key[k]) << 32) | (tid + static_cast<uint32_t>(k) * T);
    __syncthreads();

    // (5) rank inside the bucket: the sorted position of every live slot
    uint32_t pos[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        pos[k] = 0;
        if (xv[k] != 0u) {
            const uint32_t s = tid + static_cast<uint32_t>(k) * T;
            const uint32_t lo = L.sort.start[bkt[k]];
            const uint32_t hi = L.sort.start[bkt[k] + 1];
            const uint64_t me = (static_cast<uint64_t>(key[k]) << 32) | s;
            uint32_t rank = 0;
            for (uint32_t e = lo; e < hi; ++e) rank += (L.sort.kv[e] < me) ? 1u : 0u;
            pos[k] = lo + rank;
        }
    }
    if constexpr (PERM) {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (xv[k] != 0u) a.perm_out[j.off + pos[k]] = tid + static_cast<uint32_t>(k) * T;
        if (tid == 0) a.nlive_out[c] = n;
        return;
    }
    __syncthreads();   // the sort arrays are overwritten below

    // (6) the live SDs in sorted order
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (xv[k] != 0u) {
            L.pairs.xi[pos[k]] = xv[k];
            L.pairs.r[pos[k]] = rv[k];
            L.slot[pos[k]] = static_cast<uint16_t>(tid + static_cast<uint32_t>(k) * T);
        }
    }
    __syncthreads();

    const uint32_t npairs = n >> 1;
    const double scale = npairs ? upscale_factor_small(n) : 0.0;
    if constexpr (PROBE) {
        double best = 0.0;
        for (uint32_t m = tid; m < npairs; m += T) {
            const uint64_t xa = L.pairs.xi[2 * m], xb = L.pairs.xi[2 * m + 1];
            const double Kab = collection_kernel(j.kernel, j.kp, L.pairs.r[2 * m], L.pairs.r[2 * m + 1]);
            best = fmax(best, collision_probability(xa >= xb ? xa : xb, Kab, j.dt, j.dV, scale));
        }
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) best = fmax(best, __shfl_xor(best, d, kWave));
        if (lane == 0) L.dmax[wv] = best;
        __syncthreads();
        if (tid == 0) {
            double b = L.dmax[0];
            for (int w = 1; w < W; ++w) b = fmax(b, L.dmax[w]);
            a.cell_max[c] = b;
        }
        return;
    }

    // (7) pair tests: each thread takes the two pairs of one uniform call;
    // colliding pairs are written to their storage slots at once
    uint32_t coll = 0;
    const uint32_t h_end = (npairs + 1u) >> 1;
    for (uint32_t h = tid; h < h_end; h += T) {
        const Words4 w = philox4x32_10(h, j.rng_cell, j.step, kTagUniform, j.k0, j.k1);
#pragma unroll
        for (uint32_t t = 0; t < 2; ++t) {
            const uint32_t m = 2 * h + t;
            if (m >= npairs) break;
            const double u = t ? uniform_open01(w.w[2], w.w[3]) : uniform_open01(w.w[0], w.w[1]);
            const uint32_t sa = L.slot[2 * m], sb = L.slot[2 * m + 1];
            const uint64_t xa = L.pairs.xi[2 * m], xb = L.pairs.xi[2 * m + 1];
            const double ra = L.pairs.r[2 * m], rb = L.pairs.r[2 * m + 1];
            if (collide_pair_global(a, j, scale, u, sa, sb, xa, xb, ra, rb)) ++coll;
        }
    }
    const uint32_t tot = block_sum<T>(coll, L.red);
    if (tid == 0) add_counts(a, BATCHED, j.inst, blockIdx.x, npairs, tot);
}

// ---------------------------------------------------------------------------
// Split tier: a workgroup-tier cell spread over G = 2^lgG workgroups, for runs
// with too few such cells to fill the chip one workgroup each.  Workgroup g
// takes the live SDs whose key has g as its top lgG bits.  The order is by key
// first, so these hold the consecutive sorted positions [P0, P0 + M), where P0
// counts the live SDs of smaller digit.  Each workgroup draws all keys of its
// cell (a quarter Philox call per slot) to find P0, its own M SDs and the
// smallest (key, slot) above its digit: the partner of its last SD when that
// one opens a pair.  It orders its own SDs exactly in LDS (one bucket pass on
// the next key bits, scan, scatter, in-bucket rank, as the workgroup tier)
// and tests the pairs whose first member it holds, writing changed SDs at once.
// Every workgroup reads the multiplicities of the whole cell to tell live from
// dead, and another workgroup's collisions only change that when a multiplicity
// drops to zero: such writes wait until every workgroup of the cell has counted
// itself in after reading (a per-cell counter that grows by G each step; the
// wait is bounded, and a time-out is counted and reported by sdm_get_stats).
// Same order and results as the other tiers.
// ---------------------------------------------------------------------------
constexpr uint32_t kSplitMaxLg = 5;   // at most 32 workgroups per cell
constexpr uint32_t kSplitSpinLimit = 1u << 20;   // about a second of polling
// Index of the split-tier time-out counter within the first counter slot.
constexpr int kSplitTimeoutStat = 3;

template <int CAPB, int T>
struct SplitLds {
    static_assert(CAPB <= 65536, "slots are 16-bit");
    union {
        struct {
            uint64_t kv[CAPB + 1];      // own (key << 32 | slot) grouped by sub-bucket; [CAPB] a dummy
            uint32_t start[CAPB + 1];   // sub-bucket counts, then starts; start[nb] = M
        } sort;
        struct {
            uint64_t xi[CAPB + 1];      // own SDs in sorted order, then the last one's partner
            double r[CAPB + 1];
        } pairs;
    };
    uint16_t slot[CAPB + 1];
    uint32_t red[3 * (T / kWave)];
    uint64_t low[T / kWave];
    double dmax[T / kWave];
    uint64_t partner_xi;                // the partner's multiplicity and radius
    double partner_r;
    uint16_t zero[CAPB / 2 + 1];        // slots whose multiplicity drops to zero
    uint32_t ncoll;
    uint32_t nzero;
};

template <int CAPB, int T, bool PERM, bool PROBE = false>
__global__ __launch_bounds__(T) void k_split_cells(const StepArgs a, const uint32_t* list,
                                                   uint32_t lgG)
{
    constexpr int Q = CAPB / (4 * T);   // key calls per thread, four slots each
    constexpr int S = 4 * Q;
    constexpr int W = T / kWave;
    static_assert(CAPB % (4 * T) == 0 && T % kWave == 0, "split shape");
    static_assert(!(PERM && PROBE), "one mode");
    __shared__ SplitLds<CAPB, T> L;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    const uint32_t wv = __builtin_amdgcn_readfirstlane(tid / kWave);
    const uint32_t part = blockIdx.x & ((1u << lgG) - 1u);
    const uint32_t c = load_const_u32(list, blockIdx.x >> lgG);
    const CellJob j = resolve_cell<false>(a, c);
    const uint32_t n = j.n_slots;   // <= CAPB, > 2^(lgG + 1)
    const uint32_t item = blockIdx.x >> lgG;
    if (tid == 0) {
        L.ncoll = 0;
        L.nzero = 0;
    }

    // (1) the keys, multiplicities and radii of all slots of the cell (thread t
    // holds the four slots of calls t, t + T, ...)
    uint32_t key[S];
    uint64_t xv[S];
    double rv[S];
    bool own[S];
    uint32_t below = 0, mine = 0, above = 0;
    uint64_t low = ~0ull;   // smallest (key, slot) above the own digit
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const uint32_t q = tid + static_cast<uint32_t>(i) * T;
        Words4 w = {{0u, 0u, 0u, 0u}};
        if (4 * q < n) w = philox4x32_10(q, j.rng_cell, j.step, kTagShuffle, j.k0, j.k1);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * i + t;
            const uint32_t s = 4 * q + static_cast<uint32_t>(t);
            // branch-free: the index is clamped to the cell's last slot
            const uint32_t sc = s < n ? s : n - 1u;
            const uint64_t xq = a.xi[j.off + sc];
            xv[k] = s < n ? xq : 0u;
            rv[k] = 0.0;
            if constexpr (!PERM) {
                const double rq = a.r[j.off + sc];
                rv[k] = s < n ? rq : 0.0;
            }
            key[k] = w.w[t];
            const uint32_t d = bucket_of(key[k], lgG);
            const bool live = xv[k] != 0u;
            own[k] = live && d == part;
            below += (live && d < part) ? 1u : 0u;
            mine += own[k] ? 1u : 0u;
            if (live && d > part) {
                ++above;
                const uint64_t v = (static_cast<uint64_t>(key[k]) << 32) | s;
                low = v < low ? v : low;
            }
        }
    }
    // (2) block totals: P0, M, the live SDs above, and the partner candidate
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) {
        below += __shfl_xor(below, d, kWave);
        mine += __shfl_xor(mine, d, kWave);
        above += __shfl_xor(above, d, kWave);
        const uint64_t o = __shfl_xor(low, d, kWave);
        low = o < low ? o : low;
    }
    if (lane == 0) {
        L.red[wv] = below;
        L.red[W + wv] = mine;
        L.red[2 * W + wv] = above;
        L.low[wv] = low;
    }
    __syncthreads();
    uint32_t P0 = 0, M = 0, A = 0;
    uint64_t partner = ~0ull;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        P0 += L.red[w];
        M += L.red[W + w];
        A += L.red[2 * W + w];
        partner = L.low[w] < partner ? L.low[w] : partner;
    }
    const uint32_t n_live = P0 + M + A;
    const uint32_t npairs = n_live >> 1;
    // every thread's reads of the cell's multiplicities are complete here
    if constexpr (!PERM && !PROBE) {
        if (tid == 0) __hip_atomic_fetch_add(a.split_arrive + item, 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    }
    if constexpr (!PERM) {
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const uint32_t s = 4 * (tid + static_cast<uint32_t>(k / 4) * T) + static_cast<uint32_t>(k % 4);
            if (A > 0 && xv[k] != 0u && ((static_cast<uint64_t>(key[k]) << 32) | s) == partner) {
                L.partner_xi = xv[k];
                L.partner_r = rv[k];
            }
        }
    }
    // pairs m with 2m in [P0, P0 + M) and 2m + 1 < n_live
    const uint32_t m_lo = (P0 + 1u) >> 1;
    const uint32_t m_end = min((P0 + M + 1u) >> 1, npairs);
    if (M == 0) {
        if constexpr (PERM) {
            if (tid == 0 && part == 0) a.nlive_out[c] = n_live;
        } else if constexpr (!PROBE) {
            if (tid == 0 && part == 0) add_counts(a, false, 0, blockIdx.x, npairs, 0);
        }
        return;
    }
    const uint32_t lg = 31u - static_cast<uint32_t>(__clz(static_cast<int>(M)));
    const uint32_t nb = 1u << lg;
    for (uint32_t i = tid; i <= nb; i += T) L.sort.start[i] = 0;
    __syncthreads();

    // (3) sub-bucket counts on the lg key bits after the digit
    uint32_t bkt[S], arr[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        bkt[k] = 0;
        arr[k] = 0;
        if (own[k]) {
            bkt[k] = bucket_of(key[k] << lgG, lg);
            arr[k] = atomicAdd(&L.sort.start[bkt[k]], 1u);
        }
    }
    __syncthreads();
    {
        const uint32_t per = (nb + T - 1) / T;
        const uint32_t b0 = tid * per;
        const uint32_t b1 = b0 + per < nb ? b0 + per : nb;
        uint32_t run = 0;
        for (uint32_t b = b0; b < b1; ++b) run += L.sort.start[b];
        const uint32_t incl = wave_inclusive_sum_dpp(run);
        if (lane == kWave - 1) L.red[wv] = incl;
        __syncthreads();
        uint32_t before = incl - run;
#pragma unroll
        for (int w = 0; w < W; ++w) before += static_cast<uint32_t>(w) < wv ? L.red[w] : 0u;
        for (uint32_t b = b0; b < b1; ++b) {
            const uint32_t cnt = L.sort.start[b];
            L.sort.start[b] = before;
            before += cnt;
        }
        if (tid == 0) L.sort.start[nb] = M;
    }
    __syncthreads();

    // (4) scatter, then the rank inside each sub-bucket: own sorted positions.
    // Branch-free over the thread's slots (others go to the dummy entry), so
    // that the LDS accesses of all of them are in flight together.
    uint64_t me[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const uint32_t s = 4 * (tid + static_cast<uint32_t>(k / 4) * T) + static_cast<uint32_t>(k % 4);
        me[k] = (static_cast<uint64_t>(key[k]) << 32) | s;
    }
    {
        uint32_t dst[S];
#pragma unroll
        for (int k = 0; k < S; ++k) {
            const uint32_t b = L.sort.start[bkt[k]];
            dst[k] = own[k] ? b + arr[k] : static_cast<uint32_t>(CAPB);
        }
#pragma unroll
        for (int k = 0; k < S; ++k) L.sort.kv[dst[k]] = me[k];
    }
    __syncthreads();
    uint32_t pos[S];
    {
        uint32_t len[S], rank[S];
        uint32_t longest = 0;
#pragma unroll
        for (int k = 0; k < S; ++k) {
            pos[k] = L.sort.start[bkt[k]];
            const uint32_t hi = L.sort.start[bkt[k] + 1];
            len[k] = own[k] ? hi - pos[k] : 0u;
            longest = len[k] > longest ? len[k] : longest;
            rank[k] = 0;
        }
        for (uint32_t t = 0; t < longest; ++t) {
#pragma unroll
            for (int k = 0; k < S; ++k) {
                const bool in = t < len[k];
                const uint64_t v = L.sort.kv[in ? pos[k] + t : static_cast<uint32_t>(CAPB)];
                rank[k] += (in && v < me[k]) ? 1u : 0u;
            }
        }
#pragma unroll
        for (int k = 0; k < S; ++k) pos[k] += rank[k];
    }
    if constexpr (PERM) {
#pragma unroll
        for (int k = 0; k < S; ++k) {
            if (own[k]) {
                const uint32_t s = 4 * (tid + static_cast<uint32_t>(k / 4) * T) + static_cast<uint32_t>(k % 4);
                a.perm_out[j.off + P0 + pos[k]] = s;
            }
        }
        if (tid == 0 && part == 0) a.nlive_out[c] = n_live;
        return;
    }
    __syncthreads();   // the sort arrays are overwritten below

    // (5) own SDs in sorted order, and at M the partner of the last one
#pragma unroll
    for (int k = 0; k < S; ++k) {
        if (own[k]) {
            const uint32_t s = 4 * (tid + static_cast<uint32_t>(k / 4) * T) + static_cast<uint32_t>(k % 4);
            L.pairs.xi[pos[k]] = xv[k];
            L.pairs.r[pos[k]] = rv[k];
            L.slot[pos[k]] = static_cast<uint16_t>(s);
        }
    }
    if (tid == 0 && A > 0) {
        L.pairs.xi[M] = L.partner_xi;
        L.pairs.r[M] = L.partner_r;
        L.slot[M] = static_cast<uint16_t>(partner);
    }
    __syncthreads();

    // (6) pair tests, one thread per own pair (the two pairs of a uniform call
    // draw it twice: a workgroup's pairs are few, and this halves each thread's
    // chain); changed SDs are written at once, zero multiplicities later
    const double scale = npairs ? upscale_factor_small(n_live) : 0.0;
    double best = 0.0;
    for (uint32_t m = m_lo + tid; m < m_end; m += T) {
        const Words4 w = philox4x32_10(m >> 1, j.rng_cell, j.step, kTagUniform, j.k0, j.k1);
        const uint32_t ia = 2 * m - P0, ib = ia + 1;   // ib <= M
        const uint64_t xa = L.pairs.xi[ia], xb = L.pairs.xi[ib];
        const double ra = L.pairs.r[ia], rb = L.pairs.r[ib];
        const double K = collection_kernel(j.kernel, j.kp, ra, rb);
        const bool a_is_j = xa >= xb;
        PairState st;
        st.xj = a_is_j ? xa : xb;
        st.xk = a_is_j ? xb : xa;
        st.rj = a_is_j ? ra : rb;
        st.rk = a_is_j ? rb : ra;
        const double p = collision_probability(st.xj, K, j.dt, j.dV, scale);
        if constexpr (PROBE) {
            best = fmax(best, p);
            continue;
        }
        const double u = (m & 1u) ? uniform_open01(w.w[2], w.w[3]) : uniform_open01(w.w[0], w.w[1]);
        const bool release = (a.rules & kRuleRelease) != 0;
        const uint64_t g = release ? collision_count_release(p, u) : collision_count(p, u, st.xj, st.xk);
        if (g == 0) continue;
        apply_collisions(g, st, release);
        const uint32_t sa = L.slot[ia], sb = L.slot[ib];
        const uint64_t gj = static_cast<uint64_t>(j.off) + (a_is_j ? sa : sb);
        const uint64_t gk = static_cast<uint64_t>(j.off) + (a_is_j ? sb : sa);
        if (st.xj != 0u) a.xi[gj] = st.xj;
        else L.zero[atomicAdd(&L.nzero, 1u)] = static_cast<uint16_t>(a_is_j ? sa : sb);
        a.r[gk] = st.rk;
        if (st.j_changed_r) {
            a.xi[gk] = st.xk;
            a.r[gj] = st.rj;
        }
        update_dry(a, g, gj, gk, st.j_changed_r);
        atomicAdd(&L.ncoll, 1u);
    }
    if constexpr (PROBE) {
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) best = fmax(best, __shfl_xor(best, d, kWave));
        if (lane == 0) L.dmax[wv] = best;
        __syncthreads();
        if (tid == 0) {
            double b = L.dmax[0];
            for (int w = 1; w < W; ++w) b = fmax(b, L.dmax[w]);
            if (b > 0.0)
                atomicMax(reinterpret_cast<unsigned long long*>(a.cell_max + c),
                          static_cast<unsigned long long>(__double_as_longlong(b)));
        }
        return;
    }
    __syncthreads();
    if (L.nzero > 0) {
        // every workgroup of the cell has read the multiplicities once the
        // counter reaches G times the number of this cell's split steps so far
        if (tid == 0) {
            const uint32_t target = a.split_epoch << lgG;
            const uint32_t limit = a.split_spin_limit ? a.split_spin_limit : kSplitSpinLimit;
            uint32_t spins = 0;
            while (static_cast<int32_t>(__hip_atomic_load(a.split_arrive + item, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
                if (++spins >= limit) {
                    atomicAdd(a.stats + kSplitTimeoutStat, 1ull);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __syncthreads();
        for (uint32_t i = tid; i < L.nzero; i += T) a.xi[static_cast<uint64_t>(j.off) + L.zero[i]] = 0u;
    }
    if (tid == 0) add_counts(a, false, 0, blockIdx.x, part == 0 ? npairs : 0u, L.ncoll);
}

}  // namespace sdm
