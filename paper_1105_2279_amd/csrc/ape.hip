// Single-lattice kernels: one APE step (optionally with the plaquette of its
// input), the plaquette-only pass, and the standalone FP64 plaquette.
#include "qdpx_impl.hpp"
#include "ape_device.hpp"

namespace qdpx {

// One APE step (or, in kPlaqOnly mode, only the plaquette of the input).
// Thread mapping: a block of 256*k threads (k = 1 or 2) holds k groups of 64
// consecutive sites per iteration; wave w handles direction mu = w % 4 of
// group w / 4, so the four links of a site are updated by four waves of the
// same block, which share the neighbour loads in L1/L2.
template <typename R, int NR, int NS, int MODE, int PROJ = 0>
__global__ void __launch_bounds__(512) k_ape_step(Geo g, LinksRO<R, NR> U, LinksWO<R, NR> out, double c1,
                                                  double c2, unsigned mask, double *__restrict__ partials, int xcd,
                                                  int tw) {
    const int tile = xcd == 1 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
    const int mu = w & 3;
    const int gpb = blockDim.x >> 8;
    const int ngroups = (g.V + 63) >> 6;
    // FP32 steps stage each group's four own links (rows 0 and 1) in LDS: the
    // upper staple of direction nu starts from U_nu(x), the own link of wave
    // nu, so each site loads it once instead of four times (a sixth fewer
    // vector-memory instructions; 24 KB of LDS per 512-thread block).
    constexpr bool kShare = sizeof(R) == 4 && PROJ == 0 && MODE != kPlaqOnly;
    if constexpr (kShare) {
        // the four own links of each group, rows 0 and 1 as three pairs
        __shared__ nv4_t<R> own[2][4 * 3 * 64];
        nv4_t<R> *mine = own[w >> 2];
#pragma unroll 1
        for (int j = 0; j < NS; ++j) {  // no early exit: every wave meets every barrier
            const int i = (tile * NS + j) * gpb + (w >> 2);
            const bool valid = i < ngroups;
            const int grp = !valid ? 0 : xcd == 2 ? slabwalk(g, i, gpb * NS) : traverse(g, i, tw);
            if (j > 0) __syncthreads();  // the previous group's copies have been read
            if (valid) stage_own_link(g, U, grp, mu, lane, mine);
            __syncthreads();
            if (valid) ape_group<R, NR, MODE, PROJ>(g, U, out, c1, c2, mask, partials, grp, mu, lane, mine);
        }
        return;
    }
#pragma unroll 1
    for (int j = 0; j < NS; ++j) {
        const int i = (tile * NS + j) * gpb + (w >> 2);
        if (i >= ngroups) return;
        const int grp = xcd == 2 ? slabwalk(g, i, gpb * NS) : traverse(g, i, tw);
        ape_group<R, NR, MODE, PROJ>(g, U, out, c1, c2, mask, partials, grp, mu, lane);
    }
}

int ape_num_partials(const Geo &g) { return 4 * ((g.V + 63) / 64); }

hipError_t launch_ape_step(const Geo &g, int prec, int nrows, const void *Uin, void *Uout, double c1, double c2,
                           unsigned mask, double *partials, int mode, const LaunchCfg &cfg, hipStream_t st,
                           int proj) {
    if (mode == kApePlaq && mask != 0xFu) return hipErrorInvalidValue;  // owned planes need every staple
    if (proj && mode != kApe) return hipErrorInvalidValue;             // polar: plaquettes in their own pass
    const int groups = (g.V + 63) / 64;
    const int gpb = cfg.block / 256;
    const int per_block = gpb * cfg.nsite;
    const dim3 grid((groups + per_block - 1) / per_block);
    const int xcd = launch_order(g, cfg, per_block);
#define QDPX_APE_LAUNCH(R, NR, NS, M, P)                                                                       \
    k_ape_step<R, NR, NS, M, P><<<grid, cfg.block, 0, st>>>(g, LinksRO<R, NR>{(const vec2_t<R> *)Uin, g.S},     \
                                                         LinksWO<R, NR>{(vec2_t<R> *)Uout, g.S}, c1, c2, mask,  \
                                                         partials, xcd, cfg.tw)
#define QDPX_APE_M(R, NR, NS)                                         \
    if (proj) QDPX_APE_LAUNCH(R, NR, NS, kApe, 1);                    \
    else if (mode == kPlaqOnly) QDPX_APE_LAUNCH(R, NR, NS, kPlaqOnly, 0); \
    else if (mode == kApePlaq) QDPX_APE_LAUNCH(R, NR, NS, kApePlaq, 0);   \
    else QDPX_APE_LAUNCH(R, NR, NS, kApe, 0);
#define QDPX_APE_NS(R, NR)                         \
    switch (cfg.nsite) {                           \
    case 2: QDPX_APE_M(R, NR, 2) break;            \
    case 4: QDPX_APE_M(R, NR, 4) break;            \
    default: QDPX_APE_M(R, NR, 1) break;           \
    }
    if (prec == 0) {
        QDPX_APE_NS(double, 3)
    } else if (nrows == 3) {
        QDPX_APE_NS(float, 3)
    } else {
        QDPX_APE_NS(float, 2)
    }
#undef QDPX_APE_NS
#undef QDPX_APE_M
#undef QDPX_APE_LAUNCH
    return hipGetLastError();
}

// ---------------------------------------------------------------- plaquette
// One site per lane, block of 256 threads; the spatial and temporal sums of
// each 64-site group go to partials[grp] and partials[n + grp].
template <typename R, int NR>
__global__ void __launch_bounds__(256) k_plaquette(Geo g, LinksRO<R, NR> U, double *__restrict__ partials) {
    const int lane = threadIdx.x & 63;
    const int grp = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int n = (g.V + 63) >> 6;
    if (grp >= n) return;
    const int s = grp * 64 + lane;
    double sp = 0.0, tp = 0.0;
    if (s < g.V) {
        Site x;
        x.init(g, s);
#pragma unroll 1
        for (int mu = 0; mu < 3; ++mu) {
            M3<double> a;
            load_f64(U, mu, s, a);
            const int s_mu = hop_fwd(g, s, coord(x, mu), mu);
#pragma unroll 1
            for (int nu = mu + 1; nu < 4; ++nu) {
                M3<double> b, c, d;
                load_f64(U, nu, s_mu, b);                                // U_nu(x+mu)
                load_f64(U, mu, hop_fwd(g, s, coord(x, nu), nu), c);          // U_mu(x+nu)
                load_f64(U, nu, s, d);                                   // U_nu(x)
                // Re Tr[(a b)(d c)^dag]
                double p = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        Cx<double> xab{0.0, 0.0}, xdc{0.0, 0.0};
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            cmac(xab, a.e[i][k], b.e[k][j]);
                            cmac(xdc, d.e[i][k], c.e[k][j]);
                        }
                        p = fma(xab.re, xdc.re, fma(xab.im, xdc.im, p));
                    }
                if (nu == 3) tp += p;
                else sp += p;
            }
        }
    }
    sp = wave_sum(sp);
    tp = wave_sum(tp);
    if (lane == 0) {
        partials[grp] = sp;
        partials[n + grp] = tp;
    }
}

int plaquette_num_partials(const Geo &g) { return (g.V + 63) / 64; }

hipError_t launch_plaquette(const Geo &g, int prec, int nrows, const void *U, double *partials, hipStream_t st) {
    const int groups = (g.V + 63) / 64;
    const dim3 grid((groups + 3) / 4);
    if (prec == 0)
        k_plaquette<double, 3><<<grid, 256, 0, st>>>(g, LinksRO<double, 3>{(const double2 *)U, g.S}, partials);
    else if (nrows == 3)
        k_plaquette<float, 3><<<grid, 256, 0, st>>>(g, LinksRO<float, 3>{(const float2 *)U, g.S}, partials);
    else
        k_plaquette<float, 2><<<grid, 256, 0, st>>>(g, LinksRO<float, 2>{(const float2 *)U, g.S}, partials);
    return hipGetLastError();
}

}  // namespace qdpx
