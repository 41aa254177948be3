// Layout conversion (host canonical AoS <-> library SoA), the shift
// expression chi = sum_mu U_mu(x) psi(x+mu) + a phi(x) with its fused FP64
// norm, the chain update psi - c chi, and the deterministic finalisation of
// FP64 partial sums.
#include "qdpx_impl.hpp"
#include "reduce_device.hpp"

namespace qdpx {

Geo make_geo(const int32_t L[4]) {
    Geo g;
    for (int d = 0; d < 4; ++d) g.L[d] = L[d];
    g.st[0] = 1;
    g.st[1] = L[0];
    g.st[2] = L[0] * L[1];
    g.st[3] = L[0] * L[1] * L[2];
    g.V = g.st[3] * L[3];
    g.S = ((int64_t)g.V + 255) / 256 * 256;
    g.bwl = g.P = g.pbx = g.ncol = 0;
    if (L[0] % 16 == 0 && L[1] % 4 == 0) {
        g.bwl = 4;
        g.pbx = L[0] / 16;
        g.P = g.pbx * (L[1] / 4);
    } else if (L[0] % 8 == 0 && L[1] % 8 == 0) {
        g.bwl = 3;
        g.pbx = L[0] / 8;
        g.P = g.pbx * (L[1] / 8);
    }
    if (g.bwl || g.st[3] % 64 == 0) g.ncol = g.st[3] / 64;
    g.dL0 = FastDiv::make(L[0]);
    g.dL1 = FastDiv::make(L[1]);
    g.dL2 = FastDiv::make(L[2]);
    g.dP = FastDiv::make(g.P ? g.P : 1);
    g.dpbx = FastDiv::make(g.pbx ? g.pbx : 1);
    g.dplane = FastDiv::make(g.P ? g.P * L[2] : 1);
    g.dslab = FastDiv::make(g.ncol >= 8 ? g.ncol >> 3 : 1);
    return g;
}

// The block order a launch uses: the XCD slab walk (mode 2) only where its
// preconditions hold, else the identity order.
int launch_order(const Geo &g, const LaunchCfg &cfg, int groups_per_block) {
    if (cfg.xcd != 2) return cfg.xcd;
    const int groups = (g.V + 63) / 64;
    if (g.ncol && g.ncol % 8 == 0 && groups % (8 * groups_per_block) == 0) return 2;
    return 0;
}

// ------------------------------------------------------------ pack / unpack
// AoS double[V][4][3][3][2] -> the SoA link layout (LinkLayout).
// One thread per (stored element, site); the element is blockIdx.y so the
// SoA writes of a wave are contiguous (every other slot for paired FP32).
template <typename R, int NR>
__global__ void __launch_bounds__(256) k_pack_links(Geo g, const double2 *__restrict__ aos,
                                                    vec2_t<R> *__restrict__ soa) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int comp = blockIdx.y;  // enumerates (mu, a, b) as (mu*NR + a)*3 + b
    if (s >= g.V) return;
    const int b = comp % 3, a = (comp / 3) % NR, mu = comp / (3 * NR);
    const double2 v = aos[((int64_t)s * 4 + mu) * 9 + a * 3 + b];
    vec2_t<R> o;
    o.x = (R)v.x;  // FP64 -> FP32 conversion rounds to nearest even
    o.y = (R)v.y;
    soa[LinkLayout<R, NR>::slot(mu, a * 3 + b, g.S, s)] = o;
}

// SoA -> AoS; one thread per (mu, site), row 2 rebuilt in FP64 for NR == 2.
template <typename R, int NR>
__global__ void __launch_bounds__(256) k_unpack_links(Geo g, const vec2_t<R> *__restrict__ soa,
                                                      double2 *__restrict__ aos) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int mu = blockIdx.y;
    if (s >= g.V) return;
    M3<double> m;
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const vec2_t<R> v = soa[LinkLayout<R, NR>::slot(mu, a * 3 + b, g.S, s)];
            m.e[a][b] = Cx<double>{(double)v.x, (double)v.y};
        }
    if constexpr (NR == 2) rebuild_row2(m);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) aos[((int64_t)s * 4 + mu) * 9 + a * 3 + b] = double2{m.e[a][b].re, m.e[a][b].im};
}

// Index, in complex elements, of component comp of site s in the library's
// Dirac-field layout (FermLayout: FP32 components paired in 16-byte entries).
template <typename R> __device__ __forceinline__ int64_t fermion_index(int comp, int s, int64_t S) {
    if constexpr (FermLayout<R>::kPaired) return ((int64_t)(comp >> 1) * S + s) * 2 + (comp & 1);
    else return (int64_t)comp * S + s;
}

template <typename R>
__global__ void __launch_bounds__(256) k_pack_fermion(Geo g, const double2 *__restrict__ aos,
                                                      vec2_t<R> *__restrict__ soa) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int comp = blockIdx.y;  // spin*3 + colour
    if (s >= g.V) return;
    const double2 v = aos[(int64_t)s * 12 + comp];
    vec2_t<R> o;
    o.x = (R)v.x;
    o.y = (R)v.y;
    soa[fermion_index<R>(comp, s, g.S)] = o;
}

template <typename R>
__global__ void __launch_bounds__(256) k_unpack_fermion(Geo g, const vec2_t<R> *__restrict__ soa,
                                                        double2 *__restrict__ aos) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    const int comp = blockIdx.y;
    if (s >= g.V) return;
    const vec2_t<R> v = soa[fermion_index<R>(comp, s, g.S)];
    aos[(int64_t)s * 12 + comp] = double2{(double)v.x, (double)v.y};
}

static dim3 site_grid(const Geo &g, int comps) { return dim3((g.V + 255) / 256, comps, 1); }

hipError_t launch_pack_links(const Geo &g, int prec, int nrows, const double *aos, void *soa, hipStream_t st) {
    const dim3 grid = site_grid(g, 4 * nrows * 3);
    const double2 *in = reinterpret_cast<const double2 *>(aos);
    if (prec == 0) {
        k_pack_links<double, 3><<<grid, 256, 0, st>>>(g, in, (double2 *)soa);
    } else if (nrows == 3) {
        k_pack_links<float, 3><<<grid, 256, 0, st>>>(g, in, (float2 *)soa);
    } else {
        k_pack_links<float, 2><<<grid, 256, 0, st>>>(g, in, (float2 *)soa);
    }
    return hipGetLastError();
}

hipError_t launch_unpack_links(const Geo &g, int prec, int nrows, const void *soa, double *aos, hipStream_t st) {
    const dim3 grid = site_grid(g, 4);
    double2 *out = reinterpret_cast<double2 *>(aos);
    if (prec == 0) {
        k_unpack_links<double, 3><<<grid, 256, 0, st>>>(g, (const double2 *)soa, out);
    } else if (nrows == 3) {
        k_unpack_links<float, 3><<<grid, 256, 0, st>>>(g, (const float2 *)soa, out);
    } else {
        k_unpack_links<float, 2><<<grid, 256, 0, st>>>(g, (const float2 *)soa, out);
    }
    return hipGetLastError();
}

hipError_t launch_pack_fermion(const Geo &g, int prec, const double *aos, void *soa, hipStream_t st) {
    const dim3 grid = site_grid(g, 12);
    const double2 *in = reinterpret_cast<const double2 *>(aos);
    if (prec == 0) k_pack_fermion<double><<<grid, 256, 0, st>>>(g, in, (double2 *)soa);
    else k_pack_fermion<float><<<grid, 256, 0, st>>>(g, in, (float2 *)soa);
    return hipGetLastError();
}

hipError_t launch_unpack_fermion(const Geo &g, int prec, const void *soa, double *aos, hipStream_t st) {
    const dim3 grid = site_grid(g, 12);
    double2 *out = reinterpret_cast<double2 *>(aos);
    if (prec == 0) k_unpack_fermion<double><<<grid, 256, 0, st>>>(g, (const double2 *)soa, out);
    else k_unpack_fermion<float><<<grid, 256, 0, st>>>(g, (const float2 *)soa, out);
    return hipGetLastError();
}

// ------------------------------------------------------- shift expression
// chi(x) = sum_{mu in mask} h_mu(x) + a phi(x), with the forward hop
// h_mu = U_mu(x) psi(x+mu) or (bwd) the backward hop
// h_mu = U_mu(x-mu)^dag psi(x-mu); MODE 1 (one chain step) stores
// psi(x) - c chi(x) instead of chi.  A block of 256 threads holds one
// 64-site group per iteration and wave w computes direction mu = w for all 12
// spinor components, so the four directions' loads are in flight together.
// Either hop reads each link once per launch, so links are streamed.
// The four partial products meet in LDS; after a barrier wave w adds them in
// direction order for the components it owns (FermLayout), adds a phi, forms
// the FP64 |chi|^2 of those components and stores them.  The four waves'
// norms are added in wave
// order and reduced by a wave butterfly into one partial per group, so
// every sum has a fixed order and nothing depends on the launch geometry.
template <typename R, int NR, int MODE, int NS>
__global__ void __launch_bounds__(256) k_shift(Geo g, LinksRO<R, NR> U, FermRO<R> psi, FermRO<R> phi, R a, R c,
                                                unsigned mask, int bwd, FermWO<R> out, double *__restrict__ partials,
                                                int xcd, int tw) {
    __shared__ vec2_t<R> part[4][12][64];  // [direction][component][lane]
    __shared__ double nrm[4][64];          // [wave][lane]
    const int tile = xcd == 1 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int mu = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ngroups = num_groups(g);
#pragma unroll 1
    for (int j = 0; j < NS; ++j) {
        const int i = tile * NS + j;  // the same for the four waves
        if (i >= ngroups) return;
        const int grp = xcd == 2 ? slabwalk(g, i, NS) : traverse(g, i, tw);
        Site x;
        const bool live = group_site(g, grp, lane, x);
        const int s = x.s;
        const int cmu = coord(x, mu);
        // phi and (MODE 1) psi of the components this wave stores are
        // fetched now so that their latency overlaps the products and the
        // exchange
        constexpr int NO = FermLayout<R>::kOwn;
        Cx<R> f0[NO], p0[NO];
#pragma unroll
        for (int t = 0; t < NO; ++t) f0[t] = p0[t] = Cx<R>{(R)0, (R)0};
        if (live && phi.p) phi.ld_owned(mu, s, f0);
        if constexpr (MODE == 1) {
            if (live) psi.ld_owned(mu, s, p0);
        }
        Cx<R> acc[4][3];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[sp][cc] = Cx<R>{(R)0, (R)0};
        if (live && ((mask >> mu) & 1u)) {  // wave-uniform
            const int f = bwd ? hop_bwd(g, s, cmu, mu) : hop_fwd(g, s, cmu, mu);
            M3<R> u;
            U.template su3<true>(mu, bwd ? f : s, u);  // each link is read once
            if (bwd) {  // U^dag: transpose and conjugate in registers
#pragma unroll
                for (int ca = 0; ca < 3; ++ca) {
                    u.e[ca][ca].im = -u.e[ca][ca].im;
#pragma unroll
                    for (int cb = ca + 1; cb < 3; ++cb) {
                        const Cx<R> t = u.e[ca][cb];
                        u.e[ca][cb] = Cx<R>{u.e[cb][ca].re, -u.e[cb][ca].im};
                        u.e[cb][ca] = Cx<R>{t.re, -t.im};
                    }
                }
            }
            Cx<R> pf[4][3];
            psi.ld_all(f, pf);
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the arithmetic
#pragma unroll
            for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                for (int ca = 0; ca < 3; ++ca)
#pragma unroll
                    for (int cb = 0; cb < 3; ++cb) cmac(acc[sp][ca], u.e[ca][cb], pf[sp][cb]);
        }
        if (j > 0) __syncthreads();  // the previous group's partials have been read
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                vec2_t<R> v;
                v.x = acc[sp][cc].re;
                v.y = acc[sp][cc].im;
                part[mu][3 * sp + cc][lane] = v;
            }
        __syncthreads();
        double n2 = 0.0;
        if (live) {
            Cx<R> o[NO];
#pragma unroll
            for (int t = 0; t < NO; ++t) {
                Cx<R> v{(R)0, (R)0};
                const int q = FermLayout<R>::owned(mu, t);
                if (q >= 0) {  // wave-uniform
#pragma unroll
                    for (int w = 0; w < 4; ++w) {  // directions in order
                        const vec2_t<R> e = part[w][q][lane];
                        v.re += e.x;
                        v.im += e.y;
                    }
                    if (phi.p) {
                        v.re = fma(a, f0[t].re, v.re);
                        v.im = fma(a, f0[t].im, v.im);
                    }
                    n2 = fma((double)v.re, (double)v.re, fma((double)v.im, (double)v.im, n2));
                    if constexpr (MODE == 1) {
                        v.re = fma(-c, v.re, p0[t].re);
                        v.im = fma(-c, v.im, p0[t].im);
                    }
                }
                o[t] = v;
            }
            out.st_owned(mu, s, o);
        }
        if (partials) {
            nrm[mu][lane] = n2;
            __syncthreads();
            if (mu == 0) {
                const double t = ((nrm[0][lane] + nrm[1][lane]) + nrm[2][lane]) + nrm[3][lane];
                const double w = wave_sum(t);
                if (lane == 0) partials[grp] = w;
            }
        }
    }
}

int shift_num_partials(const Geo &g) { return (g.V + 63) / 64; }

template <typename R, int NR, int MODE>
static void shift_dispatch_ns(const Geo &g, const void *U, const void *psi, const void *phi, double a, double c,
                              unsigned mask, int bwd, void *out, double *partials, const LaunchCfg &cfg,
                              hipStream_t st) {
    using V = vec2_t<R>;
    LinksRO<R, NR> u{(const V *)U, g.S};
    FermRO<R> p{(const V *)psi, g.S}, f{(const V *)phi, g.S};
    FermWO<R> o{(V *)out, g.S};
    const int groups = (g.V + 63) / 64;
    const int per_block = cfg.nsite;  // one 64-site group per iteration, four waves
    const dim3 grid((groups + per_block - 1) / per_block);
    const int xcd = launch_order(g, cfg, per_block);
    switch (cfg.nsite) {
    case 2: k_shift<R, NR, MODE, 2><<<grid, 256, 0, st>>>(g, u, p, f, (R)a, (R)c, mask, bwd, o, partials, xcd, cfg.tw); break;
    case 4: k_shift<R, NR, MODE, 4><<<grid, 256, 0, st>>>(g, u, p, f, (R)a, (R)c, mask, bwd, o, partials, xcd, cfg.tw); break;
    case 8: k_shift<R, NR, MODE, 8><<<grid, 256, 0, st>>>(g, u, p, f, (R)a, (R)c, mask, bwd, o, partials, xcd, cfg.tw); break;
    default: k_shift<R, NR, MODE, 1><<<grid, 256, 0, st>>>(g, u, p, f, (R)a, (R)c, mask, bwd, o, partials, xcd, cfg.tw); break;
    }
}

template <int MODE>
static void shift_dispatch(const Geo &g, int prec, int nrows, const void *U, const void *psi, const void *phi,
                           double a, double c, unsigned mask, int bwd, void *out, double *partials,
                           const LaunchCfg &cfg, hipStream_t st) {
    if (prec == 0) shift_dispatch_ns<double, 3, MODE>(g, U, psi, phi, a, c, mask, bwd, out, partials, cfg, st);
    else if (nrows == 3) shift_dispatch_ns<float, 3, MODE>(g, U, psi, phi, a, c, mask, bwd, out, partials, cfg, st);
    else shift_dispatch_ns<float, 2, MODE>(g, U, psi, phi, a, c, mask, bwd, out, partials, cfg, st);
}

hipError_t launch_shift(const Geo &g, int prec, int nrows, const void *U, const void *psi, const void *phi,
                        double a, int mode, double c, void *out, double *partials, const LaunchCfg &cfg,
                        hipStream_t st, unsigned mask, int bwd) {
    if (mode == 0) shift_dispatch<0>(g, prec, nrows, U, psi, phi, a, c, mask, bwd, out, partials, cfg, st);
    else shift_dispatch<1>(g, prec, nrows, U, psi, phi, a, c, mask, bwd, out, partials, cfg, st);
    return hipGetLastError();
}

// ------------------------------------------------------------ Jacobi hop
// out(x) = [s0(x) + kappa * (H psi)(x)] / norm, with
// (H psi)(x) = sum_{mu in mask} [U_mu(x) psi(x+mu) + U_mu(x-mu)^dag psi(x-mu)],
// the hopping term of the smearing operator K.  s0 may be absent (then
// out = kappa H psi / norm); DIV selects the division by norm.
//
// A block of 256 threads holds one 64-site group per iteration and wave w
// computes direction mu = w: its forward and backward hop for all 12 spinor
// components, so the four directions' loads are in flight at once rather
// than one direction after another.  The four partial sums meet in LDS:
// every wave writes its twelve components and, after a barrier, wave w adds
// the four partials of the components it owns (FermLayout) in direction
// order, applies s0, kappa and norm, and stores them.  The order of every
// sum is fixed,
// so each site's result does not depend on the launch geometry.
template <typename R, int NR, int NS, bool DIV>
__global__ void __launch_bounds__(256) k_hop(Geo g, LinksRO<R, NR> U, FermRO<R> psi, FermRO<R> s0, R kappa, R norm,
                                              unsigned mask, FermWO<R> out, int xcd, int tw) {
    __shared__ vec2_t<R> part[4][12][64];  // [direction][component][lane]
    const int tile = xcd == 1 ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int mu = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int ngroups = num_groups(g);
#pragma unroll 1
    for (int j = 0; j < NS; ++j) {
        const int i = tile * NS + j;  // the same for the four waves
        if (i >= ngroups) return;
        const int grp = xcd == 2 ? slabwalk(g, i, NS) : traverse(g, i, tw);
        Site x;
        const bool live = group_site(g, grp, lane, x);
        const int s = x.s;
        Cx<R> acc[4][3];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) acc[sp][cc] = Cx<R>{(R)0, (R)0};
        const int cmu = coord(x, mu);
        // s0 of the components this wave stores is fetched now so that its
        // latency overlaps the hops and the exchange
        constexpr int NO = FermLayout<R>::kOwn;
        Cx<R> z[NO];
#pragma unroll
        for (int t = 0; t < NO; ++t) z[t] = Cx<R>{(R)0, (R)0};
        if (live && s0.p) s0.ld_owned(mu, s, z);
        if (live && ((mask >> mu) & 1u)) {
            // every load of this direction first, then the arithmetic: one
            // memory round trip per group
            const int f = hop_fwd(g, s, cmu, mu), bk = hop_bwd(g, s, cmu, mu);
            M3<R> uf, ub;
            U.template su3<false>(mu, s, uf);   // U_mu(x), also the backward link of x+mu
            U.template su3<false>(mu, bk, ub);  // U_mu(x-mu)
            Cx<R> pf[4][3], pb[4][3];
            psi.ld_all(f, pf);
            psi.ld_all(bk, pb);
            __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of the arithmetic
#pragma unroll
            for (int sp = 0; sp < 4; ++sp) {
#pragma unroll
                for (int ca = 0; ca < 3; ++ca)
#pragma unroll
                    for (int cb = 0; cb < 3; ++cb) cmac(acc[sp][ca], uf.e[ca][cb], pf[sp][cb]);
                // (U^dag p)_a = sum_b conj(U_ba) p_b
#pragma unroll
                for (int ca = 0; ca < 3; ++ca)
#pragma unroll
                    for (int cb = 0; cb < 3; ++cb) cmac_ca(acc[sp][ca], ub.e[cb][ca], pb[sp][cb]);
            }
        }
        if (j > 0) __syncthreads();  // the previous group's partials have been read
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                vec2_t<R> v;
                v.x = acc[sp][cc].re;
                v.y = acc[sp][cc].im;
                part[mu][3 * sp + cc][lane] = v;
            }
        __syncthreads();
        if (live) {
            Cx<R> o[NO];
#pragma unroll
            for (int t = 0; t < NO; ++t) {
                Cx<R> v{(R)0, (R)0};
                const int q = FermLayout<R>::owned(mu, t);
                if (q >= 0) {  // wave-uniform
#pragma unroll
                    for (int w = 0; w < 4; ++w) {  // directions in order
                        const vec2_t<R> e = part[w][q][lane];
                        v.re += e.x;
                        v.im += e.y;
                    }
                    if (s0.p) {
                        v.re = fma(kappa, v.re, z[t].re);
                        v.im = fma(kappa, v.im, z[t].im);
                    } else {
                        v.re *= kappa;
                        v.im *= kappa;
                    }
                    if constexpr (DIV) {
                        v.re = v.re / norm;
                        v.im = v.im / norm;
                    }
                }
                o[t] = v;
            }
            out.st_owned(mu, s, o);
        }
    }
}

template <typename R, int NR, bool DIV>
static void hop_dispatch_ns(const Geo &g, const void *U, const void *psi, const void *s0, double kappa, double norm,
                            unsigned mask, void *out, const LaunchCfg &cfg, hipStream_t st) {
    using V = vec2_t<R>;
    LinksRO<R, NR> u{(const V *)U, g.S};
    FermRO<R> p{(const V *)psi, g.S}, z{(const V *)s0, g.S};
    FermWO<R> o{(V *)out, g.S};
    const int groups = (g.V + 63) / 64;
    const int per_block = cfg.nsite;  // one 64-site group per iteration, four waves
    const dim3 grid((groups + per_block - 1) / per_block);
    const int xcd = launch_order(g, cfg, per_block);
    switch (cfg.nsite) {
    case 2: k_hop<R, NR, 2, DIV><<<grid, 256, 0, st>>>(g, u, p, z, (R)kappa, (R)norm, mask, o, xcd, cfg.tw); break;
    case 4: k_hop<R, NR, 4, DIV><<<grid, 256, 0, st>>>(g, u, p, z, (R)kappa, (R)norm, mask, o, xcd, cfg.tw); break;
    case 8: k_hop<R, NR, 8, DIV><<<grid, 256, 0, st>>>(g, u, p, z, (R)kappa, (R)norm, mask, o, xcd, cfg.tw); break;
    default: k_hop<R, NR, 1, DIV><<<grid, 256, 0, st>>>(g, u, p, z, (R)kappa, (R)norm, mask, o, xcd, cfg.tw); break;
    }
}

template <bool DIV>
static void hop_dispatch(const Geo &g, int prec, int nrows, const void *U, const void *psi, const void *s0,
                         double kappa, double norm, unsigned mask, void *out, const LaunchCfg &cfg, hipStream_t st) {
    if (prec == 0) hop_dispatch_ns<double, 3, DIV>(g, U, psi, s0, kappa, norm, mask, out, cfg, st);
    else if (nrows == 3) hop_dispatch_ns<float, 3, DIV>(g, U, psi, s0, kappa, norm, mask, out, cfg, st);
    else hop_dispatch_ns<float, 2, DIV>(g, U, psi, s0, kappa, norm, mask, out, cfg, st);
}

hipError_t launch_hop(const Geo &g, int prec, int nrows, const void *U, const void *psi, const void *s0, double kappa,
                      double norm, bool divide, unsigned mask, void *out, const LaunchCfg &cfg, hipStream_t st) {
    if (divide) hop_dispatch<true>(g, prec, nrows, U, psi, s0, kappa, norm, mask, out, cfg, st);
    else hop_dispatch<false>(g, prec, nrows, U, psi, s0, kappa, norm, mask, out, cfg, st);
    return hipGetLastError();
}

template <typename V>
__global__ void __launch_bounds__(256) k_copy_fermion(Geo g, const V *__restrict__ src, V *__restrict__ dst) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= g.V) return;
    const int64_t o = (int64_t)blockIdx.y * g.S + s;
    dst[o] = src[o];
}

// One 16-byte entry per (array, site): 12 arrays of double2 (FP64) or the
// six paired arrays of FP32 fields.
hipError_t launch_copy_fermion(const Geo &g, int prec, const void *src, void *dst, hipStream_t st) {
    if (prec == 0)
        k_copy_fermion<double2><<<site_grid(g, 12), 256, 0, st>>>(g, (const double2 *)src, (double2 *)dst);
    else
        k_copy_fermion<float4><<<site_grid(g, 6), 256, 0, st>>>(g, (const float4 *)src, (float4 *)dst);
    return hipGetLastError();
}

// ------------------------------------------------------------ finalisation
// Stage A: block b sums partials [b*4096, (b+1)*4096) of each component;
// stage B: one block sums the stage-A values and applies the mode.  The
// arithmetic lives in reduce_device.hpp so the batched kernel can repeat it
// bit for bit inside one block.
__global__ void __launch_bounds__(kReduceBlock) k_finalize_a(const double *__restrict__ in, int n, int ncomp,
                                                            double *__restrict__ out) {
    __shared__ double lds[kReduceBlock / 64];
    const int nb = gridDim.x;
    for (int comp = 0; comp < ncomp; ++comp) {
        const double v = fin_stage_a(in + (int64_t)comp * n, n, blockIdx.x, lds);
        if (threadIdx.x == 0) out[comp * nb + blockIdx.x] = v;
    }
}

__global__ void __launch_bounds__(kReduceBlock) k_finalize_b(const double *__restrict__ in, int n, int mode,
                                                            double volume, double *__restrict__ out) {
    __shared__ double lds[kReduceBlock / 64];
    const int ncomp = (mode == 1) ? 2 : 1;
    double r[2] = {0.0, 0.0};
    for (int comp = 0; comp < ncomp; ++comp) r[comp] = fin_stage_b(in + comp * n, n, lds);
    if (threadIdx.x == 0) fin_write(r, mode, volume, out);
}

int finalize_stage_a_blocks(int n) { return (n + kFinPerBlock - 1) / kFinPerBlock; }

hipError_t launch_finalize(const double *partials, int n, int mode, double volume, double *out, hipStream_t st) {
    // The stage-A results are stored right after the partials (the workspace
    // reserves room for them: finalize_stage_a_blocks(n) per component).
    const int ncomp = (mode == 1) ? 2 : 1;
    const int nb = finalize_stage_a_blocks(n);
    double *stage = const_cast<double *>(partials) + (int64_t)ncomp * n;
    k_finalize_a<<<nb, kReduceBlock, 0, st>>>(partials, n, ncomp, stage);
    k_finalize_b<<<1, kReduceBlock, 0, st>>>(stage, nb, mode, volume, out);
    return hipGetLastError();
}

}  // namespace qdpx
