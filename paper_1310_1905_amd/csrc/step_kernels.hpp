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
// Two kernels cover all cell sizes with identical results:
//   k_wave_cells  -- one 64-lane wavefront per cell, everything in LDS,
//                    cells of at most kWaveMaxSlots storage slots;
//   k_block_cells -- one workgroup per cell for larger cells, with the sort
//                    arrays in a global scratch area (L2-resident) that is
//                    indexed like the super-droplet arrays.
#pragma once

#include "device_math.hpp"

namespace sdm {

constexpr int kWave = 64;
constexpr int kWaveMaxSlots = 256;                 // storage slots per wave-tier cell
constexpr int kWaveItems = kWaveMaxSlots / kWave;  // slots per lane
constexpr int kStatSlots = 64;                     // spread of the global counters
constexpr int kStatStride = 16;                    // 128 bytes between counter pairs

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
    const uint32_t* items;        // work list of cell-table indices (nullptr: item i = cell i)
    uint32_t n_items;
    uint32_t cells_per_wave;
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
    unsigned long long* stats;    // single run: kStatSlots x {pair tests, collisions}
    // workgroup-tier scratch, indexed by storage slot
    uint64_t* scr_kv;
    uint64_t* scr_tmp;
    uint32_t* scr_pos;
    uint32_t* scr_cnt;
    // permutation-only mode outputs
    uint32_t* perm_out;
    uint32_t* nlive_out;
    uint32_t xcd_remap;
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

// Remap the hardware workgroup id so that each XCD (workgroups are dealt to
// the 8 XCDs round-robin) works on one contiguous range of logical blocks;
// neighbouring cells then share cache lines in the same L2.
__device__ __forceinline__ uint32_t xcd_contiguous_block(uint32_t bid, uint32_t nblk)
{
    constexpr uint32_t kXcds = 8;
    const uint32_t xcd = bid % kXcds;
    const uint32_t idx = bid / kXcds;
    const uint32_t per = nblk / kXcds;
    const uint32_t extra = nblk % kXcds;
    return xcd * per + (xcd < extra ? xcd : extra) + idx;
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
    const uint64_t g = collision_count(p, u, s.xj, s.xk);
    if (g == 0) return false;
    apply_collisions(g, s);
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
    return true;
}

// ---------------------------------------------------------------------------
// Wave tier: one wavefront per cell, at most kWaveMaxSlots storage slots.
// ---------------------------------------------------------------------------
struct alignas(16) WaveLds {
    union {
        struct {
            uint64_t kv[kWaveMaxSlots];            // (key << 32 | slot) grouped by bucket
            uint32_t keys[kWaveMaxSlots];          // Philox key of every storage slot
            uint32_t start[kWaveMaxSlots + 4];     // bucket counts, then bucket starts
        } sort;
        struct {
            uint64_t xi[kWaveMaxSlots];            // live SDs in shuffle order
            double r[kWaveMaxSlots];
            uint32_t slot[kWaveMaxSlots];
        } pairs;
    };
};

template <int WAVES, bool BATCHED, bool PERM>
__global__ __launch_bounds__(WAVES * kWave) void k_wave_cells(const StepArgs a)
{
    __shared__ WaveLds lds_all[WAVES];
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = threadIdx.x / kWave;
    WaveLds& L = lds_all[wv];

    const uint32_t blk = a.xcd_remap ? xcd_contiguous_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint64_t wave_id = static_cast<uint64_t>(blk) * WAVES + wv;
    uint64_t it = wave_id * a.cells_per_wave;
    const uint64_t it_stop = it + a.cells_per_wave;
    const uint64_t it_end = it_stop < a.n_items ? it_stop : static_cast<uint64_t>(a.n_items);

    unsigned long long pair_acc = 0, coll_acc = 0;

    for (; it < it_end; ++it) {
        const uint32_t c = a.items ? a.items[it] : static_cast<uint32_t>(it);
        const CellJob j = resolve_cell<BATCHED>(a, c);
        const uint32_t N = j.n_slots;
        if (N > static_cast<uint32_t>(kWaveMaxSlots)) continue;   // never planned here

        // (1) load the cell and count the live super-droplets
        uint64_t xv[kWaveItems];
        double rv[kWaveItems];
        uint32_t n = 0;
#pragma unroll
        for (int k = 0; k < kWaveItems; ++k) {
            const uint32_t s = lane + k * kWave;
            xv[k] = 0;
            rv[k] = 0.0;
            if (s < N) {
                xv[k] = a.xi[j.off + s];
                if constexpr (!PERM) rv[k] = a.r[j.off + s];
            }
            n += static_cast<uint32_t>(__popcll(__ballot(xv[k] != 0)));
        }
        if (n < 2) {
            if constexpr (PERM) {
                if (lane == 0) a.nlive_out[c] = n;
#pragma unroll
                for (int k = 0; k < kWaveItems; ++k)
                    if (xv[k] != 0) a.perm_out[j.off] = lane + k * kWave;
            }
            continue;
        }
        const uint32_t lg = ceil_log2(n);
        const uint32_t nb = 1u << lg;

        // (2) keys: lane q draws the four keys of slots 4q..4q+3
        for (uint32_t i = lane; i <= nb; i += kWave) L.sort.start[i] = 0;
        for (uint32_t q = lane; 4 * q < N; q += kWave) {
            const Words4 w = philox4x32_10(q, j.rng_cell, j.step, kTagShuffle, j.k0, j.k1);
            uint4 v;
            v.x = w.w[0];
            v.y = w.w[1];
            v.z = w.w[2];
            v.w = w.w[3];
            *reinterpret_cast<uint4*>(&L.sort.keys[4 * q]) = v;
        }
        wave_sync();

        // bucket counts (atomic arrival index kept for the scatter)
        uint32_t key[kWaveItems], arrival[kWaveItems];
#pragma unroll
        for (int k = 0; k < kWaveItems; ++k) {
            const uint32_t s = lane + k * kWave;
            key[k] = 0;
            arrival[k] = 0;
            if (xv[k] != 0) {
                key[k] = L.sort.keys[s];
                arrival[k] = atomicAdd(&L.sort.start[bucket_of(key[k], lg)], 1u);
            }
        }
        wave_sync();

        // exclusive scan of the nb bucket counts; start[nb] = n
        {
            const uint32_t per = (nb + kWave - 1) / kWave;   // 1..4
            const uint32_t base = lane * per;
            uint32_t v[kWaveItems];
            uint32_t sum = 0;
#pragma unroll
            for (int t = 0; t < kWaveItems; ++t) {
                v[t] = 0;
                if (static_cast<uint32_t>(t) < per && base + t < nb) v[t] = L.sort.start[base + t];
                sum += v[t];
            }
            const uint32_t incl = wave_inclusive_sum(sum, lane);
            uint32_t run = incl - sum;
#pragma unroll
            for (int t = 0; t < kWaveItems; ++t) {
                if (static_cast<uint32_t>(t) < per && base + t < nb) L.sort.start[base + t] = run;
                run += v[t];
            }
            if (lane == kWave - 1) L.sort.start[nb] = incl;
        }
        wave_sync();

        // scatter (key, slot) to bucket start + arrival
#pragma unroll
        for (int k = 0; k < kWaveItems; ++k) {
            if (xv[k] != 0) {
                const uint32_t s = lane + k * kWave;
                const uint32_t pos = L.sort.start[bucket_of(key[k], lg)] + arrival[k];
                L.sort.kv[pos] = (static_cast<uint64_t>(key[k]) << 32) | s;
            }
        }
        wave_sync();

        // rank inside the bucket by full (key, slot) comparison
        uint32_t final_pos[kWaveItems];
#pragma unroll
        for (int k = 0; k < kWaveItems; ++k) {
            final_pos[k] = 0;
            if (xv[k] != 0) {
                const uint32_t s = lane + k * kWave;
                const uint32_t b = bucket_of(key[k], lg);
                const uint32_t lo = L.sort.start[b];
                const uint32_t hi = L.sort.start[b + 1];
                const uint64_t me = (static_cast<uint64_t>(key[k]) << 32) | s;
                uint32_t rank = 0;
                for (uint32_t e = lo; e < hi; ++e) rank += (L.sort.kv[e] < me) ? 1u : 0u;
                final_pos[k] = lo + rank;
            }
        }
        wave_sync();   // every read of the sort arrays is done before they are overwritten

#pragma unroll
        for (int k = 0; k < kWaveItems; ++k) {
            if (xv[k] != 0) {
                const uint32_t p = final_pos[k];
                L.pairs.xi[p] = xv[k];
                L.pairs.r[p] = rv[k];
                L.pairs.slot[p] = lane + k * kWave;
            }
        }
        wave_sync();

        if constexpr (PERM) {
            for (uint32_t i = lane; i < n; i += kWave) a.perm_out[j.off + i] = L.pairs.slot[i];
            if (lane == 0) a.nlive_out[c] = n;
            wave_sync();
            continue;
        }

        // (3) pairs (2m, 2m+1)
        const uint32_t npairs = n >> 1;
        const double scale = upscale_factor(n);
        uint32_t coll = 0;
        for (uint32_t m = lane; m < npairs; m += kWave) {
            const double u = pair_uniform(m, j.rng_cell, j.step, j.k0, j.k1);
            const ulonglong2 x2 = *reinterpret_cast<const ulonglong2*>(&L.pairs.xi[2 * m]);
            const double2 r2 = *reinterpret_cast<const double2*>(&L.pairs.r[2 * m]);
            const uint2 s2 = *reinterpret_cast<const uint2*>(&L.pairs.slot[2 * m]);
            if (collide_pair_global(a, j, scale, u, s2.x, s2.y, x2.x, x2.y, r2.x, r2.y)) ++coll;
        }
        wave_sync();   // pair reads done before the next cell reuses the LDS

        // counters
        unsigned long long cell_coll = 0;
        {
            // wave total of per-lane collision counts
            uint32_t v = coll;
#pragma unroll
            for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
            cell_coll = v;
        }
        if constexpr (BATCHED) {
            if (lane == 0) add_counts(a, true, j.inst, 0, npairs, cell_coll);
        } else {
            pair_acc += npairs;
            coll_acc += cell_coll;
        }
    }
    if constexpr (!BATCHED && !PERM) {
        if (lane == 0 && (pair_acc || coll_acc))
            add_counts(a, false, 0, static_cast<uint32_t>(wave_id), pair_acc, coll_acc);
    }
}

// ---------------------------------------------------------------------------
// Workgroup tier: one workgroup per cell, any number of storage slots.
// ---------------------------------------------------------------------------
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

// In-place exclusive scan of arr[0..nb) (global), arr[nb] = total.
template <int BLOCK>
__device__ void block_exclusive_scan(uint32_t* arr, uint32_t nb, uint32_t* s_red)
{
    constexpr int W = BLOCK / kWave;
    const uint32_t lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += BLOCK) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? arr[i] : 0u;
        const uint32_t incl_w = wave_inclusive_sum(v, lane);
        if (lane == kWave - 1) s_red[wv] = incl_w;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t t = s_red[w];
            before += (static_cast<uint32_t>(w) < wv) ? t : 0u;
            total += t;
        }
        if (i < nb) arr[i] = carry + before + incl_w - v;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) arr[nb] = carry;
}

template <int BLOCK, bool BATCHED, bool PERM>
__global__ __launch_bounds__(BLOCK) void k_block_cells(const StepArgs a)
{
    __shared__ uint32_t s_red[BLOCK / kWave];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & (kWave - 1);
    unsigned long long pair_acc = 0, coll_acc = 0;

    for (uint64_t it = blockIdx.x; it < a.n_items; it += gridDim.x) {
        const uint32_t c = a.items ? a.items[it] : static_cast<uint32_t>(it);
        const CellJob j = resolve_cell<BATCHED>(a, c);
        const uint32_t N = j.n_slots;
        const uint64_t* xi = a.xi + j.off;

        // (1) live count
        uint32_t cnt = 0;
        for (uint32_t s = tid; s < N; s += BLOCK) cnt += xi[s] != 0 ? 1u : 0u;
        const uint32_t n = block_sum<BLOCK>(cnt, s_red);
        if (n < 2) {
            if constexpr (PERM) {
                if (tid == 0) a.nlive_out[c] = n;
                for (uint32_t s = tid; s < N; s += BLOCK)
                    if (xi[s] != 0) a.perm_out[j.off] = s;
            }
            continue;
        }
        // about two keys per bucket; the bucket array fits in n entries
        const uint32_t lg = ceil_log2(n) - 1u;
        const uint32_t nb = 1u << lg;
        uint32_t* cntp = a.scr_cnt + j.off;
        uint64_t* kv = a.scr_kv + j.off;
        uint64_t* tmp = a.scr_tmp + j.off;
        uint32_t* pos = a.scr_pos + j.off;

        for (uint32_t i = tid; i <= nb; i += BLOCK) cntp[i] = 0;
        __syncthreads();

        // (2) keys and bucket counts
        for (uint32_t q = tid; 4 * q < N; q += BLOCK) {
            const Words4 w = philox4x32_10(q, j.rng_cell, j.step, kTagShuffle, j.k0, j.k1);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t s = 4 * q + t;
                if (s < N && xi[s] != 0) {
                    const uint32_t arr = atomicAdd(&cntp[bucket_of(w.w[t], lg)], 1u);
                    tmp[s] = (static_cast<uint64_t>(w.w[t]) << 32) | arr;
                }
            }
        }
        __syncthreads();
        block_exclusive_scan<BLOCK>(cntp, nb, s_red);
        __syncthreads();

        // scatter
        for (uint32_t s = tid; s < N; s += BLOCK) {
            if (xi[s] != 0) {
                const uint64_t t = tmp[s];
                const uint32_t key = static_cast<uint32_t>(t >> 32);
                const uint32_t p = cntp[bucket_of(key, lg)] + static_cast<uint32_t>(t);
                kv[p] = (static_cast<uint64_t>(key) << 32) | s;
            }
        }
        __syncthreads();

        // rank inside buckets
        for (uint32_t s = tid; s < N; s += BLOCK) {
            if (xi[s] != 0) {
                const uint32_t key = static_cast<uint32_t>(tmp[s] >> 32);
                const uint32_t b = bucket_of(key, lg);
                const uint32_t lo = cntp[b], hi = cntp[b + 1];
                const uint64_t me = (static_cast<uint64_t>(key) << 32) | s;
                uint32_t rank = 0;
                for (uint32_t e = lo; e < hi; ++e) rank += (kv[e] < me) ? 1u : 0u;
                pos[lo + rank] = s;
            }
        }
        __syncthreads();

        if constexpr (PERM) {
            for (uint32_t i = tid; i < n; i += BLOCK) a.perm_out[j.off + i] = pos[i];
            if (tid == 0) a.nlive_out[c] = n;
            __syncthreads();
            continue;
        }

        // (3) pairs
        const uint32_t npairs = n >> 1;
        const double scale = upscale_factor(n);
        uint32_t coll = 0;
        for (uint32_t m = tid; m < npairs; m += BLOCK) {
            const double u = pair_uniform(m, j.rng_cell, j.step, j.k0, j.k1);
            const uint32_t sa = pos[2 * m], sb = pos[2 * m + 1];
            const uint64_t xa = xi[sa], xb = xi[sb];
            const double ra = a.r[j.off + sa], rb = a.r[j.off + sb];
            if (collide_pair_global(a, j, scale, u, sa, sb, xa, xb, ra, rb)) ++coll;
        }
        const uint32_t cell_coll = block_sum<BLOCK>(coll, s_red);
        if constexpr (BATCHED) {
            if (tid == 0) add_counts(a, true, j.inst, 0, npairs, cell_coll);
        } else {
            pair_acc += npairs;
            coll_acc += cell_coll;
        }
        (void)lane;
    }
    if constexpr (!BATCHED && !PERM) {
        if (tid == 0 && (pair_acc || coll_acc))
            add_counts(a, false, 0, blockIdx.x, pair_acc, coll_acc);
    }
}

}  // namespace sdm
