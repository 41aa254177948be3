// Persistent batched APE smearing: many independent lattices of any extents,
// n_steps APE steps each and the final plaquettes, in one launch.
//
// The launch walks through phases: the n APE steps, then (with plaquettes)
// the plaquette traces of the outputs and the per-lattice finalisation.
// Within a phase the work items are (lattice, column, run of t-rows): a
// column is one brick of one z plane, so one item walks a column through t
// and reuses each t neighbour from L1/L2 right after loading it.  Each XCD
// has its own queue (ticket counter) holding the columns c with c % 8 equal
// to its id, read from the XCC_ID hardware register; a block drains its own
// XCD's queue first and then takes items from the other queues, so the load
// still balances.  Which queue a block uses only affects speed.
//
// When a block finds every queue of the phase empty it publishes how many
// items it finished (one release) and waits until the phase's completion
// counter reaches the item count (one acquire).  Every item it waits for
// was already taken by a running block, so the wait always ends and no
// co-residency assumption is needed.  Fencing once per block and phase, not
// per item, matters on the multi-XCD MI355X: an agent-scope acquire
// invalidates the XCD's L2.  Every wait is bounded; on timeout the block
// records the failure in the status word and leaves, so the grid drains.
#include "ape_device.hpp"
#include "qdpx_impl.hpp"
#include "reduce_device.hpp"

namespace qdpx {

// Largest number of stage-A values a lattice's plaquette reduction may need
// (held in LDS): 4*ngroups <= kBatchMaxStage * kFinPerBlock.
constexpr int kBatchMaxStage = 64;

__global__ void __launch_bounds__(256) k_batched_init(unsigned *__restrict__ counters, int n) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) counters[i] = 0u;
}

// Reduce lattice L's plaquette partials exactly as the two finalisation
// kernels of the single-lattice path do.
__device__ void batched_finalize(const BatchLat &L, double *out, double *lds, double (*stage)[kBatchMaxStage]) {
    const int n = 4 * L.ngroups;
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
    if (threadIdx.x == 0) fin_write(res, 1, (double)L.g.V, out);
}

// XCD this block runs on (XCC_ID hardware register, bits 3:0).
__device__ __forceinline__ int xcd_id() {
    return (int)(__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (kXcds - 1));
}

// Take the next ticket of queue q (thread 0), broadcast it to the block.
__device__ __forceinline__ unsigned take_ticket(unsigned *counter, unsigned *s_ticket) {
    if (threadIdx.x == 0) *s_ticket = atomicAdd(counter, 1u);
    __syncthreads();
    const unsigned r = __builtin_amdgcn_readfirstlane(*s_ticket);
    __syncthreads();  // s_ticket is rewritten by the next call
    return r;
}

// The lattice table comes as its own const __restrict__ argument: the compiler
// may then read it (at wave-uniform indices) with scalar loads, as the
// single-lattice kernels read their geometry from the kernel arguments.
template <typename R, int NR>
__global__ void __launch_bounds__(256) k_ape_batched(BatchArgs a, const BatchLat *__restrict__ lats) {
    __shared__ unsigned s_ticket;
    __shared__ int s_ok;
    __shared__ double lds[kReduceBlock / 64];
    __shared__ double stage[2][kBatchMaxStage];
    __shared__ nv4_t<R> own[sizeof(R) == 4 ? 4 * 3 * 64 : 1];  // the group's own links (FP32)
    // mu is wave-uniform; readfirstlane lets the compiler keep it in an SGPR
    const int mu = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int xid = __builtin_amdgcn_readfirstlane(xcd_id());
    const int nph = a.n_phases + (a.plaq ? 1 : 0);  // steps, plaquette traces, finalisation
    unsigned *status = a.counters + 1;
    unsigned *tickets = a.counters + 2;             // [nph][kXcds]
    unsigned *done = a.counters + 2 + nph * kXcds;  // [nph]
    for (int phase = 0; phase < nph; ++phase) {
        const bool fin = a.plaq && phase == nph - 1;
        unsigned mine = 0;
        if (fin) {
            for (;;) {
                const unsigned r = take_ticket(tickets + phase * kXcds, &s_ticket);
                if (r >= (unsigned)a.n_lat) break;
                ++mine;
                batched_finalize(lats[r], a.plaq + 3 * r, lds, stage);
            }
        } else {
            // step p reads the output of step p-1: step k writes to U_out when
            // n_steps-1-k is even, else to the lattice's scratch links
            const bool ape = phase < a.n_steps;
            const int src_odd = (a.n_steps - phase) & 1, dst_odd = (a.n_steps - 1 - phase) & 1;
            for (int k = 0; k < kXcds; ++k) {
                const int q = (xid + k) & (kXcds - 1);  // own queue first, then the others
                for (;;) {
                    const unsigned r = take_ticket(tickets + phase * kXcds + q, &s_ticket);
                    if (r >= (unsigned)a.xtotal[q]) break;
                    ++mine;
                    int lo = 0, hi = a.n_lat - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (lats[mid].xbase[q] <= (int)r) lo = mid;
                        else hi = mid - 1;
                    }
                    const BatchLat &L = lats[lo];  // read in place: a private copy would live in scratch
                    const int rr = (int)r - L.xbase[q];
                    const int col = q + kXcds * (rr / L.nchunk);
                    const int row0 = (rr % L.nchunk) * a.group_chunk;
                    const int row1 = min(row0 + a.group_chunk, L.nrow);
                    const void *src = (phase == 0) ? L.in : (src_odd == 0 ? L.out : L.tmp);
                    void *dst = ape ? (dst_odd == 0 ? L.out : L.tmp) : nullptr;
                    const LinksRO<R, NR> U{(const vec2_t<R> *)src, L.g.S};
                    const LinksWO<R, NR> O{(vec2_t<R> *)dst, L.g.S};
                    if (ape) {
#pragma unroll 1
                        for (int row = row0; row < row1; ++row) {
                            const int grp = col + L.ncol * row;
                            if constexpr (sizeof(R) == 4) {  // own links staged in LDS, as the single-lattice step
                                // (take_ticket's barriers separate items; rows of one item need their own)
                                if (row > row0) __syncthreads();
                                stage_own_link(L.g, U, grp, mu, lane, own);
                                __syncthreads();
                                ape_group<R, NR, kApe>(L.g, U, O, a.c1, a.c2, 0xFu, nullptr, grp, mu, lane, own);
                            } else {
                                ape_group<R, NR, kApe>(L.g, U, O, a.c1, a.c2, 0xFu, nullptr, grp, mu, lane);
                            }
                        }
                    } else {
#pragma unroll 1
                        for (int row = row0; row < row1; ++row)
                            ape_group<R, NR, kPlaqOnly>(L.g, U, O, a.c1, a.c2, 0xFu, L.partials, col + L.ncol * row, mu,
                                                        lane);
                    }
                }
            }
        }
        if (phase + 1 == nph) break;
        const unsigned nitems = (unsigned)a.items_per_phase;
        __syncthreads();  // every wave of the block has issued its stores
        if (threadIdx.x == 0) {
            __threadfence();  // release this block's links / partials of the phase device-wide
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

int batched_max_stage_groups() { return kBatchMaxStage * kFinPerBlock / 4; }

int batched_resident_blocks(int prec, int nrows) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e;
    if (prec == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ape_batched<double, 3>, 256, 0);
    else if (nrows == 3) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ape_batched<float, 3>, 256, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ape_batched<float, 2>, 256, 0);
    // (the occupancy does not depend on the kernel's arguments)
    if (e != hipSuccess) return 0;
    return cus * std::max(per_cu, 1);
}

int batched_counter_words(int max_phases) { return 2 + (kXcds + 1) * (max_phases + 1); }

hipError_t launch_ape_batched(const BatchArgs &a, int prec, int nrows, int grid, hipStream_t st) {
    const int ncount = batched_counter_words(a.n_phases);
    k_batched_init<<<std::min((ncount + 255) / 256, 1024), 256, 0, st>>>(a.counters, ncount);
    if (prec == 0) k_ape_batched<double, 3><<<grid, 256, 0, st>>>(a, a.lats);
    else if (nrows == 3) k_ape_batched<float, 3><<<grid, 256, 0, st>>>(a, a.lats);
    else k_ape_batched<float, 2><<<grid, 256, 0, st>>>(a, a.lats);
    return hipGetLastError();
}

}  // namespace qdpx
