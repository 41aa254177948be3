// Persistent batched APE smearing: many independent lattices of any extents,
// n_steps APE steps each in one persistent launch, then the final plaquettes.
//
// The persistent launch walks through phases, one per APE step.  Within a
// phase the work items are runs of 64-site groups of one lattice.  A
// lattice's groups form a (column, t-row) grid, a column being one brick (or
// run of 64 sites) of one z plane; its columns are split into 8 contiguous
// ranges, one per XCD, and XCD x's queue (ticket counter) walks its range
// t-row by t-row, so a group's x, y and z neighbours are queued a few items
// away and its t neighbours one range further, all on the XCD whose L2 holds
// them (the slab walk of the single-lattice step, per lattice).  A block
// reads its XCD from the XCC_ID hardware register, drains its own queue first
// and then takes items from the other queues, so the load still balances;
// which queue a block uses only affects speed.
//
// When a block finds every queue of the phase empty it publishes how many
// items it finished (one release) and waits until the phase's completion
// counter reaches the item count (one acquire).  Every item it waits for
// was already taken by a running block, so the wait always ends and no
// co-residency assumption is needed.  Fencing once per block and phase, not
// per item, matters on the multi-XCD MI355X: an agent-scope acquire
// invalidates the XCD's L2.  Every wait is bounded; on timeout the block
// records the failure in the status word and leaves, so the grid drains.
//
// The plaquettes of the outputs follow as two ordinary launches (the traces
// of every group of every lattice, then one reducing block per lattice) with
// exactly the arithmetic and partial layout of the standalone plaquette
// pass, in FP64 for every link precision.  Keeping them out of the
// persistent kernel keeps its register budget that of the step alone.
#include "ape_device.hpp"
#include "qdpx_impl.hpp"
#include "reduce_device.hpp"

namespace qdpx {

// LDS tile of the FP32 steps, a level of the single-lattice step's: 3, the
// own and backward links and the plane products (levels 2 and 4 measured the
// same for 12-real links and slower for 18-real ones).
constexpr int kBatchedLds = 3;

// Largest number of stage-A values a lattice's plaquette reduction may need
// (held in LDS): 3*ngroups <= kBatchMaxStage * kFinPerBlock (bounded with 4
// partials per group).
constexpr int kBatchMaxStage = 64;

__global__ void __launch_bounds__(256) k_batched_init(unsigned *__restrict__ counters, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) counters[i] = 0u;
}

// XCD this block runs on (XCC_ID hardware register, bits 3:0).
__device__ __forceinline__ int xcd_id() {
    return (int)(__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (kXcds - 1));
}

// Take the next ticket of counter (thread 0) and broadcast it to the block.
__device__ __forceinline__ unsigned take_ticket(unsigned *counter, unsigned *s_ticket) {
    if (threadIdx.x == 0) *s_ticket = atomicAdd(counter, 1u);
    __syncthreads();
    const unsigned r = __builtin_amdgcn_readfirstlane(*s_ticket);
    __syncthreads();  // s_ticket is rewritten by the next call
    return r;
}

// Lattice whose entry base(q) is the last one <= r (bases ascending).
template <typename F> __device__ __forceinline__ int find_lattice(int n_lat, int r, F base) {
    int lo = 0, hi = n_lat - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base(mid) <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The lattice table comes as its own const __restrict__ argument: the compiler
// may then read it (at wave-uniform indices) with scalar loads, as the
// single-lattice kernels read their geometry from the kernel arguments.
// GPB 64-site groups are processed at once per block (4 waves each).  FP32:
// at most 128 registers, four waves per SIMD, what the LDS tile (36 KB per
// group) leaves room for.
template <typename R, int NR, int GPB>
__global__ void __launch_bounds__(256 * GPB) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_ape_batched(BatchArgs a, const BatchLat *__restrict__ lats) {
    __shared__ unsigned s_ticket;
    __shared__ int s_ok;
    // FP32: the LDS tile of the single-lattice step at level kBatchedLds,
    // each group's own links, backward links and plane-product slots
    __shared__ nv4_t<R> own[GPB][sizeof(R) == 4 ? 4 * 3 * 64 : 1];
    __shared__ nv4_t<R> back[GPB][sizeof(R) == 4 && ape_lds_back(kBatchedLds) ? kApeTileF4 : 1];
    __shared__ nv4_t<R> slots[GPB][sizeof(R) == 4 && ape_lds_slots(kBatchedLds) ? 4 * kApeSlotF4 : 1];
    __shared__ double2 back64[sizeof(R) == 8 ? 4 * GPB * kF64BackPerWave : 1];  // FP64: backward links
    // mu is wave-uniform; readfirstlane lets the compiler keep it in an SGPR
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int mu = w & 3, half = w >> 2;
    const int xid = __builtin_amdgcn_readfirstlane(xcd_id());
    const int nph = a.n_steps;
    unsigned *status = a.counters + 1;
    unsigned *tickets = a.counters + 2;             // [nph][kXcds]
    unsigned *done = a.counters + 2 + nph * kXcds;  // [nph]
    const int per_ticket = a.group_chunk;           // groups per ticket
    for (int phase = 0; phase < nph; ++phase) {
        unsigned mine = 0;
        // step p reads the output of step p-1: step k writes to U_out when
        // n_steps-1-k is even, else to the lattice's scratch links
        const int src_odd = (a.n_steps - phase) & 1, dst_odd = (a.n_steps - 1 - phase) & 1;
        for (int k = 0; k < kXcds; ++k) {
            const int q = (xid + k) & (kXcds - 1);  // own queue first, then the others
            for (;;) {
                const unsigned r = take_ticket(tickets + phase * kXcds + q, &s_ticket);
                if (r >= (unsigned)a.xtotal[q]) break;
                ++mine;
                const BatchLat &L =
                    lats[find_lattice(a.n_lat, (int)r, [&](int i) { return lats[i].xbase[q]; })];  // read in place
                const int ncols = L.xcol1[q] - L.xcol0[q];
                const int j0 = ((int)r - L.xbase[q]) * per_ticket;
                const int j1 = min(j0 + per_ticket, ncols * L.nrow);
                const void *src = (phase == 0) ? L.in : (src_odd == 0 ? L.out : L.tmp);
                void *dst = dst_odd == 0 ? L.out : L.tmp;
                const LinksRO<R, NR> U{(const vec2_t<R> *)src, L.g.S};
                const LinksWO<R, NR> O{(vec2_t<R> *)dst, L.g.S};
                // GPB groups at a time, half h of the block taking j0 + h, ...
                // (no early exit: every wave meets every barrier)
#pragma unroll 1
                for (int jj = j0; jj < j1; jj += GPB) {
                    const int j = jj + half;
                    const bool valid = j < j1;
                    int grp = 0;
                    if (valid) {
                        const int row = L.dcols[q].div(j);
                        grp = (L.xcol0[q] + (j - row * ncols)) + L.ncol * row;
                    }
                    if constexpr (sizeof(R) == 4) {  // links staged in LDS, as the single-lattice step
                        nv4_t<R> *bk = ape_lds_back(kBatchedLds) ? back[half] : nullptr;
                        if (jj > j0) __syncthreads();  // take_ticket's barriers separate items
                        if (valid) {
                            stage_own_link(L.g, U, grp, mu, lane, own[half]);
                            if constexpr (ape_lds_back(kBatchedLds)) stage_back_link(L.g, U, grp, mu, lane, bk);
                        }
                        __syncthreads();
                        if constexpr (ape_lds_slots(kBatchedLds))  // block barriers inside: every wave takes part
                            ape_group_shared<R, NR>(L.g, U, O, a.c1, a.c2, 0xFu, grp, valid, mu, lane, own[half], bk,
                                                    slots[half]);
                        else if (valid)
                            ape_group<R, NR, kApe>(L.g, U, O, a.c1, a.c2, 0xFu, nullptr, grp, mu, lane, own[half],
                                                   nullptr, bk);
                    } else {
                        if (valid)
                            ape_group<R, NR, kApe>(L.g, U, O, a.c1, a.c2, 0xFu, nullptr, grp, mu, lane, nullptr,
                                                   back64 + w * kF64BackPerWave);
                    }
                }
            }
        }
        if (phase + 1 == nph) break;
        const unsigned nitems = (unsigned)a.items_per_phase;
        __syncthreads();  // every wave of the block has issued its stores
        if (threadIdx.x == 0) {
            __threadfence();  // release this block's links of the phase device-wide
            atomicAdd(done + phase, mine);
            unsigned spins = 0;
            int ok = 1;
            while (__hip_atomic_load(done + phase, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < nitems) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > a.spin_limit) {
                    ok = 0;
                    break;
                }
            }
            if (!ok) atomicOr(status, 1u);
            s_ok = ok;
        }
        __syncthreads();
        if (!s_ok) return;  // block-uniform
        __threadfence();    // acquire the phase's results
    }
}

// Plaquette traces of every lattice's output links into its partials: one
// 64-site group per block, the single-lattice plaquette pass's arithmetic
// and partial layout (plaquette_wave), so each lattice's plaquette is the
// one qdpx_plaquette gives for its links, bit for bit.
template <typename R, int NR>
__global__ void __launch_bounds__(64 * kPlaqWavesPerGroup) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_batched_plaq(BatchArgs a, const BatchLat *__restrict__ lats) {
    const int b = blockIdx.x;
    const BatchLat &L = lats[find_lattice(a.n_lat, b, [&](int i) { return lats[i].pbase; })];
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    plaquette_wave(L.g, LinksRO<R, NR>{(const vec2_t<R> *)L.out, L.g.S}, b - L.pbase, w, lane, L.partials);
}

// One block per lattice: its partials reduced exactly as the two
// finalisation kernels of the single-lattice path do.
__global__ void __launch_bounds__(kReduceBlock) k_batched_fin(const BatchLat *__restrict__ lats, int per_group,
                                                             double *__restrict__ plaq) {
    __shared__ double lds[kReduceBlock / 64];
    __shared__ double stage[2][kBatchMaxStage];
    const BatchLat &L = lats[blockIdx.x];
    const int n = per_group * L.ngroups;
    const int nb = (n + kFinPerBlock - 1) / kFinPerBlock;
    double res[2];
    for (int comp = 0; comp < 2; ++comp) {
        for (int b = 0; b < nb; ++b) {
            const double v = fin_stage_a(L.partials + (int64_t)comp * n, n, b, lds);
            if (threadIdx.x == 0) stage[comp][b] = v;
        }
        __syncthreads();
        res[comp] = fin_stage_b(stage[comp], nb, lds);
    }
    if (threadIdx.x == 0) fin_write(res, 1, (double)L.g.V, plaq + 3 * blockIdx.x);
}

int batched_max_stage_groups() { return kBatchMaxStage * kFinPerBlock / 4; }

int batched_plaq_blocks(int, int ngroups) { return ngroups; }

template <typename R, int NR> static hipError_t resident(int gpb, int *per_cu) {
    if (gpb == 2) return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_ape_batched<R, NR, 2>, 512, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_ape_batched<R, NR, 1>, 256, 0);
}

int batched_resident_blocks(int prec, int nrows, int block) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const int gpb = block / 256;
    hipError_t e;
    if (prec == 0) e = resident<double, 3>(gpb, &per_cu);
    else if (nrows == 3) e = resident<float, 3>(gpb, &per_cu);
    else e = resident<float, 2>(gpb, &per_cu);
    // (the occupancy does not depend on the kernel's arguments)
    if (e != hipSuccess) return 0;
    return cus * std::max(per_cu, 1);
}

int batched_counter_words(int max_phases) { return 2 + (kXcds + 1) * (max_phases + 1); }

template <typename R, int NR>
static void launch_all(const BatchArgs &a, int block, int grid, hipStream_t st) {
    if (block == 512) k_ape_batched<R, NR, 2><<<grid, 512, 0, st>>>(a, a.lats);
    else k_ape_batched<R, NR, 1><<<grid, 256, 0, st>>>(a, a.lats);
    if (a.plaq) {
        k_batched_plaq<R, NR><<<a.plaq_blocks, 64 * kPlaqWavesPerGroup, 0, st>>>(a, a.lats);
        k_batched_fin<<<a.n_lat, kReduceBlock, 0, st>>>(a.lats, kPlaqWavesPerGroup, a.plaq);
    }
}

hipError_t launch_ape_batched(const BatchArgs &a, int prec, int nrows, int block, int grid, hipStream_t st) {
    const int ncount = batched_counter_words(a.n_steps);
    k_batched_init<<<std::min((ncount + 255) / 256, 1024), 256, 0, st>>>(a.counters, ncount);
    if (prec == 0) launch_all<double, 3>(a, block, grid, st);
    else if (nrows == 3) launch_all<float, 3>(a, block, grid, st);
    else launch_all<float, 2>(a, block, grid, st);
    return hipGetLastError();
}

}  // namespace qdpx
