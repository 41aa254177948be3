// Single-lattice kernels: one APE step (for FP64 links optionally with the
// plaquette of its input) and the plaquette pass (FP64 products for every
// link precision).
#include "qdpx_impl.hpp"
#include "ape_device.hpp"

namespace qdpx {

// One APE step (for FP64 links in kApePlaq mode with the plaquette of its
// input).  Thread mapping: a block of 256*k threads (k = 1 or 2) holds k
// groups of 64 consecutive sites per iteration; for FP32 links wave w
// handles direction mu = w % 4 of group w / 4, so the four links of a site
// are updated by four waves of the same block, which share the neighbour
// loads in L1/L2; for FP64 links wave w % 4 of group w / 4 takes the four
// directions of 16 of its sites (ape_group_f64).
template <typename R, int NR, int NS, int MODE, int PROJ = 0, int LDS = 0>
__global__ void __launch_bounds__(512) k_ape_step(Geo g, LinksRO<R, NR> U, LinksWO<R, NR> out, double c1,
                                                  double c2, unsigned mask, double *__restrict__ partials, int xcd,
                                                  int tw) {
    const int tile = xcd == 1 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int mu = w & 3;
    const int gpb = blockDim.x >> 8;
    const int ngroups = (g.V + 63) >> 6;
    // The LDS tile of FP32 steps (LDS = 1): each group's four own links (rows
    // 0 and 1) staged once, since the upper staple of direction nu starts from
    // U_nu(x), the own link of wave nu (24 KB per 512-thread block); LDS = 2
    // adds each site's four backward links U_mu(x-mu) (columns 0 and 1), which
    // the lower staples of the three other directions all read (another
    // 24 KB); LDS = 3 adds four slots per group through which the producer of
    // each plane passes its upper product to the consumer (staple_sum_rows01_shared,
    // another 12 KB); LDS = 4 has the own links and the slots but loads the
    // backward links (24 KB in all).  Staged values are the ones the loads
    // would give and every level does the same arithmetic: all levels yield
    // the same bits.
    static_assert(MODE == kApe || sizeof(R) == 8, "FP32 steps take their plaquettes from k_plaquette");
    static_assert(LDS == 0 || (sizeof(R) == 4 && PROJ == 0), "LDS tiles belong to the FP32 row projection");
    // Dynamic LDS, sized at launch: kF64BackPerWave double2 per wave (FP64), or
    // per group ape_lds_f4_per_group(LDS) FP32 pairs: the own links, then
    // (LDS 2 and 3) the backward links, then (LDS 3 and 4) the four product
    // slots.
    extern __shared__ double2 lds_dyn[];
    if constexpr (LDS > 0) {
        nv4_t<R> *tiles = reinterpret_cast<nv4_t<R> *>(lds_dyn);
        nv4_t<R> *mine = tiles + (w >> 2) * ape_lds_f4_per_group(LDS);
        nv4_t<R> *mine_back = ape_lds_back(LDS) ? mine + kApeTileF4 : nullptr;
        nv4_t<R> *mine_slots = ape_lds_slots(LDS) ? mine + (ape_lds_back(LDS) ? 2 : 1) * kApeTileF4 : nullptr;
#pragma unroll 1
        for (int j = 0; j < NS; ++j) {  // no early exit: every wave meets every barrier
            const int i = (tile * NS + j) * gpb + (w >> 2);
            const bool valid = i < ngroups;
            const int grp = !valid ? 0 : xcd == 2 ? slabwalk(g, i, gpb * NS) : traverse(g, i, tw);
            if (j > 0) __syncthreads();  // the previous group's copies have been read
            if (valid) {
                stage_own_link(g, U, grp, mu, lane, mine);
                if constexpr (ape_lds_back(LDS)) stage_back_link(g, U, grp, mu, lane, mine_back);
            }
            // the copies are read after this barrier; at level 4 the first
            // barrier of the staple sum comes before any read of the own
            // links (its phases read them after their barrier), so it serves
            if constexpr (LDS != 4) __syncthreads();
            if constexpr (ape_lds_slots(LDS))  // block barriers inside: every wave takes part
                ape_group_shared<R, NR>(g, U, out, c1, c2, mask, grp, valid, mu, lane, mine, mine_back, mine_slots);
            else if (valid)
                ape_group<R, NR, MODE, PROJ>(g, U, out, c1, c2, mask, partials, grp, mu, lane, mine, nullptr,
                                             mine_back);
        }
        return;
    }
    // FP64 steps exchange each lane's backward link through LDS (one
    // kF64BackPerWave region per wave); FP32 steps without an LDS tile load
    // every link
#pragma unroll 1
    for (int j = 0; j < NS; ++j) {
        const int i = (tile * NS + j) * gpb + (w >> 2);
        if (i >= ngroups) return;
        const int grp = xcd == 2 ? slabwalk(g, i, gpb * NS) : traverse(g, i, tw);
        ape_group<R, NR, MODE, PROJ>(g, U, out, c1, c2, mask, partials, grp, mu, lane, nullptr,
                                     sizeof(R) == 8 ? lds_dyn + w * kF64BackPerWave : nullptr);
    }
}

int ape_num_partials(const Geo &g) { return 4 * ((g.V + 63) / 64); }

hipError_t launch_ape_step(const Geo &g, int prec, int nrows, const void *Uin, void *Uout, double c1, double c2,
                           unsigned mask, double *partials, int mode, const LaunchCfg &cfg, hipStream_t st,
                           int proj) {
    if (mode != kApe && mode != kApePlaq) return hipErrorInvalidValue;
    if (mode == kApePlaq && mask != 0xFu) return hipErrorInvalidValue;  // owned planes need every staple
    if (proj && mode != kApe) return hipErrorInvalidValue;             // polar: plaquettes in their own pass
    if (prec != 0 && mode != kApe) return hipErrorInvalidValue;        // FP32: plaquettes from k_plaquette
    const int groups = (g.V + 63) / 64;
    const int gpb = cfg.block / 256;
    const int per_block = gpb * cfg.nsite;
    const dim3 grid((groups + per_block - 1) / per_block);
    const int xcd = launch_order(g, cfg, per_block);
    const int lds_level = (prec != 0 && !proj) ? cfg.lds : 0;
    const size_t lds64 = (prec == 0 && !proj) ? sizeof(double2) * kF64BackPerWave * (cfg.block / 64)
                                              : (size_t)16 * ape_lds_f4_per_group(lds_level) * gpb;
#define QDPX_APE_LAUNCH(R, NR, NS, M, P, T)                                                                      \
    k_ape_step<R, NR, NS, M, P, T><<<grid, cfg.block, lds64, st>>>(g, LinksRO<R, NR>{(const vec2_t<R> *)Uin, g.S}, \
                                                                LinksWO<R, NR>{(vec2_t<R> *)Uout, g.S}, c1, c2,   \
                                                                mask, partials, xcd, cfg.tw)
#define QDPX_APE_M64(NS)                                                         \
    if (proj) QDPX_APE_LAUNCH(double, 3, NS, kApe, 1, 0);                      \
    else if (mode == kApePlaq) QDPX_APE_LAUNCH(double, 3, NS, kApePlaq, 0, 0); \
    else QDPX_APE_LAUNCH(double, 3, NS, kApe, 0, 0);
#define QDPX_APE_M32(NR, NS)                                           \
    if (proj) QDPX_APE_LAUNCH(float, NR, NS, kApe, 1, 0);              \
    else if (lds_level == 4) QDPX_APE_LAUNCH(float, NR, NS, kApe, 0, 4); \
    else if (lds_level == 3) QDPX_APE_LAUNCH(float, NR, NS, kApe, 0, 3); \
    else if (lds_level == 2) QDPX_APE_LAUNCH(float, NR, NS, kApe, 0, 2); \
    else if (lds_level == 1) QDPX_APE_LAUNCH(float, NR, NS, kApe, 0, 1); \
    else QDPX_APE_LAUNCH(float, NR, NS, kApe, 0, 0);
#define QDPX_APE_NS(M)                             \
    switch (cfg.nsite) {                           \
    case 2: M(2) break;                            \
    case 4: M(4) break;                            \
    default: M(1) break;                           \
    }
#define QDPX_APE_F32_3(NS) QDPX_APE_M32(3, NS)
#define QDPX_APE_F32_2(NS) QDPX_APE_M32(2, NS)
    if (prec == 0) {
        QDPX_APE_NS(QDPX_APE_M64)
    } else if (nrows == 3) {
        QDPX_APE_NS(QDPX_APE_F32_3)
    } else {
        QDPX_APE_NS(QDPX_APE_F32_2)
    }
#undef QDPX_APE_F32_2
#undef QDPX_APE_F32_3
#undef QDPX_APE_M32
#undef QDPX_APE_M64
#undef QDPX_APE_NS
#undef QDPX_APE_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------- plaquette
// One 64-site group per 192-thread block, wave w taking its two planes
// (plaquette_wave).  FP32 links: at most 128 registers, four waves per SIMD
// (without the bound the compiler takes 130 for three).
template <typename R, int NR>
__global__ void __launch_bounds__(64 * kPlaqWavesPerGroup) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 4 : 1)))
k_plaquette(Geo g, LinksRO<R, NR> U, double *__restrict__ partials) {
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    plaquette_wave(g, U, (int)blockIdx.x, w, (int)(threadIdx.x & 63), partials);
}

int plaquette_num_partials(const Geo &g) { return kPlaqWavesPerGroup * ((g.V + 63) / 64); }

hipError_t launch_plaquette(const Geo &g, int prec, int nrows, const void *U, double *partials, hipStream_t st) {
    const dim3 grid((g.V + 63) / 64), block(64 * kPlaqWavesPerGroup);
    if (prec == 0)
        k_plaquette<double, 3><<<grid, block, 0, st>>>(g, LinksRO<double, 3>{(const double2 *)U, g.S}, partials);
    else if (nrows == 3)
        k_plaquette<float, 3><<<grid, block, 0, st>>>(g, LinksRO<float, 3>{(const float2 *)U, g.S}, partials);
    else
        k_plaquette<float, 2><<<grid, block, 0, st>>>(g, LinksRO<float, 2>{(const float2 *)U, g.S}, partials);
    return hipGetLastError();
}

}  // namespace qdpx
