// Device-side APE smearing work shared by the single-lattice kernels and
// the persistent batched kernel: staple sums restricted to rows 0 and 1,
// the owned-plane plaquette traces and the per-64-site-group step.
//
// APE step, per link (x, mu), all from the unsmeared field U:
//   S = sum_{nu != mu} [ U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag + U_nu(x-nu)^dag U_mu(x-nu) U_nu(x-nu+mu) ]
//   W = (1-alpha) U_mu(x) + (alpha/6) S,   V = rowwise Gram-Schmidt of W (FP64)
// The projection reads only rows 0 and 1 of W (row 2 of V is conj(row0 x
// row1)), so only rows 0 and 1 of every staple are formed: each staple is
// (2x3) = (2x3)(3x3) then (2x3)(3x3), two thirds of the full products.
#pragma once

#include "su3_device.hpp"

namespace qdpx {

// T = A(rows 0,1) * B
template <typename R> __device__ __forceinline__ void mul_23_33(const M23<R> &A, const M3<R> &B, M23<R> &T) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<R> t{(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(t, A.e[i][k], B.e[k][j]);
            T.e[i][j] = t;
        }
}
// T = (A^dag)(rows 0,1) * B, i.e. T_ij = sum_k conj(A_ki) B_kj
template <typename R> __device__ __forceinline__ void mul_dag23_33(const M3<R> &A, const M3<R> &B, M23<R> &T) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<R> t{(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_ca(t, A.e[k][i], B.e[k][j]);
            T.e[i][j] = t;
        }
}
// S += T * C
template <typename R> __device__ __forceinline__ void acc_23_33(M23<R> &S, const M23<R> &T, const M3<R> &C) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(S.e[i][j], T.e[i][k], C.e[k][j]);
}
// S += T * C^dag
template <typename R> __device__ __forceinline__ void acc_23_33dag(M23<R> &S, const M23<R> &T, const M3<R> &C) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_cb(S.e[i][j], T.e[i][k], C.e[j][k]);
}

// Full 3x3 products (the polar projection, which reads all of W, and the
// FP64 plaquette).
// T = A * B
template <typename R> __device__ __forceinline__ void mul_33_33(const M3<R> &A, const M3<R> &B, M3<R> &T) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<R> t{(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(t, A.e[i][k], B.e[k][j]);
            T.e[i][j] = t;
        }
}
// T = A^dag * B
template <typename R> __device__ __forceinline__ void mul_dag33_33(const M3<R> &A, const M3<R> &B, M3<R> &T) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<R> t{(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_ca(t, A.e[k][i], B.e[k][j]);
            T.e[i][j] = t;
        }
}
// S += T * C
template <typename R> __device__ __forceinline__ void acc_33_33(M3<R> &S, const M3<R> &T, const M3<R> &C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(S.e[i][j], T.e[i][k], C.e[k][j]);
}
// S += T * C^dag
template <typename R> __device__ __forceinline__ void acc_33_33dag(M3<R> &S, const M3<R> &T, const M3<R> &C) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_cb(S.e[i][j], T.e[i][k], C.e[j][k]);
}

// Full link in FP64: stored rows widened, row 2 rebuilt in FP64 for LINK12.
template <typename R, int NR>
__device__ __forceinline__ void load_f64(const LinksRO<R, NR> &U, int mu, int s, M3<double> &m) {
    Cx<R> r[3][3];
    U.template load_rows<false, NR>(mu, s, r);
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) m.e[a][b] = Cx<double>{(double)r[a][b].re, (double)r[a][b].im};
    if constexpr (NR == 2) rebuild_row2(m);
}

// Row i of link (mu, s) in FP64: a stored row widened, or (LINK12, i = 2)
// rebuilt in FP64 from the widened rows 0 and 1, as load_f64 forms it.
template <typename R, int NR, int I>
__device__ __forceinline__ void row_f64(const LinksRO<R, NR> &U, int mu, int s, Cx<double> (&r)[3]) {
    if constexpr (I < 2 || NR == 3) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const Cx<R> z = U.ld(mu, I, b, s);
            r[b] = Cx<double>{(double)z.re, (double)z.im};
        }
    } else {
        M3<double> m;
        Cx<R> e[2][3];
        U.template load_rows<false, 2>(mu, s, e);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) m.e[a][b] = Cx<double>{(double)e[a][b].re, (double)e[a][b].im};
        rebuild_row2(m);
#pragma unroll
        for (int b = 0; b < 3; ++b) r[b] = m.e[2][b];
    }
}

// Re Tr P_{mu nu}(x) = Re Tr[(U_mu(x) U_nu(x+mu)) (U_nu(x) U_mu(x+nu))^dag] of
// the stored links widened to FP64 (row 2 rebuilt in FP64 for LINK12), every
// product and sum in FP64: the plaquette of the standalone pass, of the FP32
// steps' per-step plaquettes and of the batched FP32 plaquettes, one
// function so that they agree bit for bit.  s_mu = x+mu, s_nu = x+nu.  Rows of
// U_mu(x) and U_nu(x) are loaded as they are needed, so that only the two
// neighbour links and one product are held in FP64 at a time.
template <typename R, int NR>
__device__ __forceinline__ double plaquette_plane(const LinksRO<R, NR> &U, int mu, int nu, int s, int s_mu,
                                                  int s_nu) {
    M3<double> m;  // U_mu(x) U_nu(x+mu)
    {
        M3<double> b;
        load_f64(U, nu, s_mu, b);
        Cx<double> a[3];
#define QDPX_PLAQ_ROW_M(I)                                                           \
        row_f64<R, NR, I>(U, mu, s, a);                                              \
        for (int j = 0; j < 3; ++j) {                                                \
            Cx<double> t{0.0, 0.0};                                                  \
            for (int k = 0; k < 3; ++k) cmac(t, a[k], b.e[k][j]);                     \
            m.e[I][j] = t;                                                           \
        }
        QDPX_PLAQ_ROW_M(0)
        QDPX_PLAQ_ROW_M(1)
        QDPX_PLAQ_ROW_M(2)
#undef QDPX_PLAQ_ROW_M
    }
    M3<double> c;  // U_mu(x+nu)
    load_f64(U, mu, s_nu, c);
    double p = 0.0;
    Cx<double> d[3];
#define QDPX_PLAQ_ROW_N(I)                                                               \
    row_f64<R, NR, I>(U, nu, s, d);                                                      \
    for (int j = 0; j < 3; ++j) {                                                        \
        Cx<double> n{0.0, 0.0};                                                          \
        for (int k = 0; k < 3; ++k) cmac(n, d[k], c.e[k][j]);                            \
        p = fma(m.e[I][j].re, n.re, fma(m.e[I][j].im, n.im, p));                          \
    }
    QDPX_PLAQ_ROW_N(0)
    QDPX_PLAQ_ROW_N(1)
    QDPX_PLAQ_ROW_N(2)
#undef QDPX_PLAQ_ROW_N
    return p;
}

// Spatial (nu < 3) and temporal (nu = 3) plaquette sums of site x over the
// six planes, planes (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) added in that order.
template <typename R, int NR>
__device__ __forceinline__ void plaquette_site(const Geo &g, const LinksRO<R, NR> &U, const Site &x, double &sp,
                                               double &tp) {
    sp = tp = 0.0;
#pragma unroll 1
    for (int mu = 0; mu < 3; ++mu) {
        const int s_mu = hop_fwd(g, x.s, coord(x, mu), mu);
#pragma unroll 1
        for (int nu = mu + 1; nu < 4; ++nu) {
            const double p = plaquette_plane(U, mu, nu, x.s, s_mu, hop_fwd(g, x.s, coord(x, nu), nu));
            if (nu == 3) tp += p;
            else sp += p;
        }
    }
}

// Plaquette planes are shared out over the four direction waves so that each
// of the six planes is counted once and each wave's planes are all spatial or
// all temporal: wave 0 owns (0,1), (0,2); wave 1 owns (1,2); wave 2 owns
// (2,3); wave 3 owns (3,0), (3,1).  Ownership is wave-uniform.
__device__ __forceinline__ bool owns_plane(int mu, int nu) {
    return (mu == 0 && (nu == 1 || nu == 2)) || (mu == 1 && nu == 2) || (mu == 2 && nu == 3) ||
           (mu == 3 && nu < 2);
}

// Re Tr[U X^dag] for U, X in SU(3) from their rows 0 and 1 alone.  With
// p_ab = <X_a, U_b> = sum_j conj(X_aj) U_bj and row 2 of each matrix equal to
// conj(row0 x row1), the Binet-Cauchy identity <a x b, c x d> =
// <a, c><b, d> - <a, d><b, c> gives <X_2, U_2> = conj(p00 p11 - p01 p10), so
// Re Tr[U X^dag] = Re p00 + Re p11 + Re(p00 p11 - p01 p10): four 3-term inner
// products (link precision) and one 2x2 determinant (FP64) instead of the
// third row of X.  Exact for SU(3) arguments; stored links and their
// products are SU(3) to the rounding of the link precision.
template <typename R> __device__ __forceinline__ double retrace_rows01(const M23<R> &u, const M23<R> &X) {
    Cx<R> p[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            p[a][b] = Cx<R>{(R)0, (R)0};
#pragma unroll
            for (int j = 0; j < 3; ++j) cmac_ca(p[a][b], X.e[a][j], u.e[b][j]);
        }
    const double p00r = p[0][0].re, p00i = p[0][0].im, p11r = p[1][1].re, p11i = p[1][1].im;
    const double p01r = p[0][1].re, p01i = p[0][1].im, p10r = p[1][0].re, p10i = p[1][0].im;
    const double d = fma(p00r, p11r, -(p00i * p11i)) - fma(p01r, p10r, -(p01i * p10i));
    return (p00r + p11r) + d;
}

// Coordinate mu of x for a run-time, wave-uniform mu.  The FP32 steps read it
// through selects: with their LDS staging, indexing the array made the
// batched kernel keep the coordinates in scratch.  The FP64 steps index the
// array, which the compiler keeps in registers, and the selects would cost
// them a wave of occupancy.
template <typename R> __device__ __forceinline__ int site_coord(const Site &x, int mu) {
    if constexpr (sizeof(R) == 4) return coord(x, mu);
    else return x.c[mu];
}

// Rows 0 and 1 of U_nu(x) from the LDS copy the block stages for its group:
// own[(nu*3 + k)*64 + lane] holds elements 2k and 2k+1 (FP32 only).
template <typename R>
__device__ __forceinline__ void own_rows01(const nv4_t<R> *own, int nu, M23<R> &A) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const nv4_t<R> v = own[(nu * 3 + k) * 64 + lane];
        A.e[(2 * k) / 3][(2 * k) % 3] = Cx<R>{v.x, v.y};
        A.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = Cx<R>{v.z, v.w};
    }
}

// Stage rows 0 and 1 of this wave's own link U_mu(x) for the sites of group
// grp into own[(mu*3 + k)*64 + lane] (FP32 pairs), where own_rows01 of the
// block's other direction waves reads them after a barrier.
template <typename R, int NR>
__device__ __forceinline__ void stage_own_link(const Geo &g, const LinksRO<R, NR> &U, int grp, int mu, int lane,
                                               nv4_t<R> *own) {
    Site x;
    if (!group_site(g, grp, lane, x)) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Cx<R> e0, e1;
        U.template ld_pair<false>(mu, k, x.s, e0, e1);
        nv4_t<R> v;
        v.x = e0.re;
        v.y = e0.im;
        v.z = e1.re;
        v.w = e1.im;
        own[(mu * 3 + k) * 64 + lane] = v;
    }
}

// Staple sum (rows 0 and 1) of link (s, mu) over the planes (mu, nu) with nu
// in mask (bits 0..3; all four for the fused plaquette).  With PLQ, plq
// receives the sum over the planes this wave owns of Re Tr[U_mu(x) X^dag],
// X the plane's upper staple, which is the trace of the plaquette
// P_{mu nu}(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag; u0 holds
// rows 0 and 1 of U_mu(x).
template <typename R, int NR, bool PLQ>
__device__ __forceinline__ void staple_sum_rows01(const Geo &g, const LinksRO<R, NR> &U, const Site &x, int mu,
                                                  unsigned mask, M23<R> &S, const M23<R> &u0, double &plq,
                                                  const nv4_t<R> *own = nullptr) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S.e[i][j] = Cx<R>{(R)0, (R)0};
    plq = 0.0;
    const int s = x.s;
    const int s_mu = hop_fwd(g, s, site_coord<R>(x, mu), mu);
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const int nu = k + (k >= mu);
        if (!((mask >> nu) & 1u)) continue;  // wave-uniform
        // upper: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
        {
            M23<R> A;
            if (own) own_rows01(own, nu, A);  // wave nu's own link, staged in LDS
            else U.rows01(nu, s, A);
            M3<R> B;
            U.full(mu, hop_fwd(g, s, site_coord<R>(x, nu), nu), B);
            M23<R> T;
            mul_23_33(A, B, T);
            M3<R> C;
            U.full(nu, s_mu, C);
            if (owns_plane(mu, nu)) {
                // Owned planes are formed on their own and then added, with or
                // without the plaquette, so the staple sum S (and hence the
                // smeared link) is bit-identical whether or not PLQ is set.
                M23<R> X;
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) X.e[i][j] = Cx<R>{(R)0, (R)0};
                acc_23_33dag(X, T, C);
                if constexpr (PLQ) plq += retrace_rows01(u0, X);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        S.e[i][j].re += X.e[i][j].re;
                        S.e[i][j].im += X.e[i][j].im;
                    }
            } else {
                acc_23_33dag(S, T, C);
            }
        }
        // lower: U_nu(y)^dag U_mu(y) U_nu(y+mu), y = x - nu
        {
            const int y = hop_bwd(g, s, site_coord<R>(x, nu), nu);
            M3<R> A;
            U.full(nu, y, A);
            M3<R> B;
            U.full(mu, y, B);
            M23<R> T;
            mul_dag23_33(A, B, T);
            M3<R> C;
            U.full(nu, hop_fwd(g, y, site_coord<R>(x, mu), mu), C);  // y has the same mu-coordinate as x
            acc_23_33(S, T, C);
        }
    }
}

// Full staple sum (all three rows) of link (s, mu) over nu in mask, the same
// staples in the same order as staple_sum_rows01.
template <typename R, int NR>
__device__ __forceinline__ void staple_sum_full(const Geo &g, const LinksRO<R, NR> &U, const Site &x, int mu,
                                                unsigned mask, M3<R> &S) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S.e[i][j] = Cx<R>{(R)0, (R)0};
    const int s = x.s;
    const int s_mu = hop_fwd(g, s, x.c[mu], mu);
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const int nu = k + (k >= mu);
        if (!((mask >> nu) & 1u)) continue;  // wave-uniform
        {  // upper: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag
            M3<R> A, B, T, C;
            U.full(nu, s, A);
            U.full(mu, hop_fwd(g, s, x.c[nu], nu), B);
            mul_33_33(A, B, T);
            U.full(nu, s_mu, C);
            acc_33_33dag(S, T, C);
        }
        {  // lower: U_nu(y)^dag U_mu(y) U_nu(y+mu), y = x - nu
            const int y = hop_bwd(g, s, x.c[nu], nu);
            M3<R> A, B, T, C;
            U.full(nu, y, A);
            U.full(mu, y, B);
            mul_dag33_33(A, B, T);
            U.full(nu, hop_fwd(g, y, x.c[mu], mu), C);
            acc_33_33(S, T, C);
        }
    }
}

// Store the FP64 link v in link precision (round to nearest).
template <typename R, int NR>
__device__ __forceinline__ void store_narrowed(const LinksWO<R, NR> &out, int mu, int s, const Cx<double> (&v)[3][3]) {
    Cx<R> o[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) o[a][b] = Cx<R>{(R)v[a][b].re, (R)v[a][b].im};
    out.store(mu, s, o);
}

// What one (64-site group, direction) wave computes.
enum ApeMode { kApe = 0, kApePlaq = 1, kPlaqOnly = 2 };

// The owned planes' plaquette traces only: the same arithmetic as the PLQ
// branch of staple_sum_rows01, so both give the same value bit for bit.
template <typename R, int NR>
__device__ __forceinline__ double owned_plaquettes(const Geo &g, const LinksRO<R, NR> &U, const Site &x, int mu,
                                                   const M23<R> &u0) {
    double plq = 0.0;
    const int s = x.s;
    const int s_mu = hop_fwd(g, s, site_coord<R>(x, mu), mu);
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const int nu = k + (k >= mu);
        if (!owns_plane(mu, nu)) continue;
        M23<R> A;
        U.rows01(nu, s, A);
        M3<R> B;
        U.full(mu, hop_fwd(g, s, site_coord<R>(x, nu), nu), B);
        M23<R> T;
        mul_23_33(A, B, T);
        M3<R> C;
        U.full(nu, s_mu, C);
        M23<R> X;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) X.e[i][j] = Cx<R>{(R)0, (R)0};
        acc_23_33dag(X, T, C);
        plq += retrace_rows01(u0, X);
    }
    return plq;
}

// ------------------------------------------------------------- FP64 step
// The FP64 step puts the four directions of 16 sites in one wave: lane L of
// the group's wave w handles site 16 w + (L & 15) of the group (group_site's
// lane index) and direction mu = L >> 4.  In phase p = 0, 1, 2 the lane forms
// the two staples of plane nu = mu ^ (p + 1) while its partner lane
// L ^ 16 (p + 1) (same site, direction nu) forms those of plane mu.  The two
// upper staples U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag and U_mu(x) U_nu(x+mu)
// U_mu(x+nu)^dag are made of the same four links, so each lane loads one
// neighbour link, U_mu(x+nu), and takes U_nu(x+mu) and rows 0 and 1 of
// U_nu(x) from its partner by cross-lane exchange; the lower staple's
// U_nu(x-nu) is the partner's backward link, which every lane loads once
// and shares through LDS.  A link update then issues 96 vector loads of 16
// bytes instead of 151: the vector-memory pipeline, not the arithmetic,
// bounds the FP64 step.  The fused plaquette takes each plane once, in the
// lane of its lower direction.  Direction-dependent addresses differ
// between lanes here, so they are formed in 64 bits per lane.

constexpr int kF64BackPerWave = 9 * 64;  // double2 per wave: one backward link per lane

__device__ __forceinline__ int sel4(int i, int a, int b, int c, int d) {
    return i == 0 ? a : i == 1 ? b : i == 2 ? c : d;
}
// x +- mu for a per-lane mu (selects instead of indexing the geometry)
__device__ __forceinline__ int hop_fwd_v(const Geo &g, int s, int cmu, int mu) {
    const int L = sel4(mu, g.L[0], g.L[1], g.L[2], g.L[3]), st = sel4(mu, g.st[0], g.st[1], g.st[2], g.st[3]);
    return (cmu == L - 1) ? s - (L - 1) * st : s + st;
}
__device__ __forceinline__ int hop_bwd_v(const Geo &g, int s, int cmu, int mu) {
    const int L = sel4(mu, g.L[0], g.L[1], g.L[2], g.L[3]), st = sel4(mu, g.st[0], g.st[1], g.st[2], g.st[3]);
    return (cmu == 0) ? s + (L - 1) * st : s - st;
}

// Element c of the FP64 link at site s of a direction whose array starts at
// the per-lane pointer dir (U.p + mu * 9 * S): the element offset c * S is
// wave-uniform, the site offset per lane.
__device__ __forceinline__ Cx<double> ld_lane(const double2 *dir, int64_t S, int c, int s) {
    const nv2_t<double> v = *gptr<nv2_t<double>>(dir + (c * S + s));
    return Cx<double>{v.x, v.y};
}
__device__ __forceinline__ void st_lane(double2 *dir, int64_t S, int c, int s, const Cx<double> &z) {
    store_stream<double>((void *)(dir + (c * S + s)), z.re, z.im);
}
__device__ __forceinline__ Cx<double> xchg(const Cx<double> &z, int m) {
    return Cx<double>{__shfl_xor(z.re, m, 64), __shfl_xor(z.im, m, 64)};
}

// One wave's share of an FP64 step (modes as ape_group): the four directions
// of 16 sites of group grp.  back: this wave's kF64BackPerWave LDS entries.
// Partials (plaquette modes): partials[grp*4 + w] (spatial planes) and
// partials[4*ngroups + grp*4 + w] (temporal planes) of the INPUT links.
template <int MODE>
__device__ __forceinline__ void ape_group_f64(const Geo &g, const LinksRO<double, 3> &U, const LinksWO<double, 3> &out,
                                              double c1, double c2, unsigned mask, double *__restrict__ partials,
                                              int grp, int w, int lane, double2 *back) {
    const int ngroups = num_groups(g);
    const int mu = lane >> 4;
    Site x;
    const bool live = group_site(g, grp, 16 * w + (lane & 15), x);
    if (!live) x.init(g, 0);  // padding lanes load from site 0 and store nothing
    const int s = x.s;
    const int cmu = coord(x, mu);
    const bool smear = MODE == kPlaqOnly || ((mask >> mu) & 1u);
    const int64_t S9 = 9 * U.S;
    const double2 *dmu = U.p + mu * S9;  // this lane's direction
    if constexpr (MODE != kPlaqOnly) {
        // the backward link U_mu(x-mu), read by the lanes of the other directions
        const int sb = hop_bwd_v(g, s, cmu, mu);
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            const Cx<double> z = ld_lane(dmu, U.S, c, sb);
            back[c * 64 + lane] = double2{z.re, z.im};
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    Cx<double> S[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i][j] = Cx<double>{0.0, 0.0};
    double sp = 0.0, tp = 0.0;
#pragma unroll 1
    for (int p = 0; p < 3; ++p) {
        const int xm = 16 * (p + 1);
        const int nu = mu ^ (p + 1);
        // plane (mu, nu) is smeared for this lane exactly when it is for the
        // partner (both directions in the mask)
        const bool act = smear && (MODE == kPlaqOnly || ((mask >> nu) & 1u));
        const bool own_plane = mu < nu;  // the plaquette of the plane is taken here
        const int cnu = coord(x, nu);
        // upper: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag.  B = U_mu(x+nu) is loaded by
        // every lane (the partner needs it); rows of U_nu(x) (the partner's
        // own rows) and of U_nu(x+mu) (the partner's B) are exchanged one at
        // a time as the products consume them.
        M3<double> B;
        const int s_nu = hop_fwd_v(g, s, cnu, nu);
#pragma unroll
        for (int c = 0; c < 9; ++c) B.e[c / 3][c % 3] = ld_lane(dmu, U.S, c, s_nu);
        const double2 *dnu = U.p + nu * S9;
        Cx<double> T[2][3];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            Cx<double> a[3];  // row i of U_nu(x)
#pragma unroll
            for (int k = 0; k < 3; ++k) a[k] = ld_lane(dnu, U.S, 3 * i + k, s);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                Cx<double> t{0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 3; ++k) cmac(t, a[k], B.e[k][j]);
                T[i][j] = t;
            }
        }
        // X = T U_nu(x+mu)^dag: X_ij = sum_k T_ik conj(C_jk), C row j from the
        // partner; every upper staple is formed on its own and then added, so
        // the smeared link does not depend on whether the plaquette is taken.
        Cx<double> X[2][3];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) X[i][j] = Cx<double>{0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<double> cj[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) cj[k] = xchg(B.e[j][k], xm);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) cmac_cb(X[i][j], T[i][k], cj[k]);
        }
        if (act) {
            if constexpr (MODE != kApe) {
                if (own_plane) {
                    M23<double> uu, xx;  // rows 0 and 1 of U_mu(x) and of X
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            uu.e[i][j] = ld_lane(dmu, U.S, 3 * i + j, s);
                            xx.e[i][j] = X[i][j];
                        }
                    const double pl = retrace_rows01(uu, xx);
                    if (nu == 3) tp += pl;
                    else sp += pl;
                }
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    S[i][j].re += X[i][j].re;
                    S[i][j].im += X[i][j].im;
                }
        }
        if constexpr (MODE != kPlaqOnly) {
            // lower: U_nu(y)^dag U_mu(y) U_nu(y+mu), y = x - nu, by rows k:
            // T2_ij = sum_k conj(LA_ki) LB_kj with LA = U_nu(x-nu), the
            // partner's backward link (columns 0 and 1 from LDS), then
            // S_ij += sum_k T2_ik LC_kj
            __builtin_amdgcn_sched_barrier(0);  // the lower staple's loads stay below the upper one
            if (act) {
                const int sy = hop_bwd_v(g, s, cnu, nu);
                const int syf = hop_fwd_v(g, sy, cmu, mu);  // y has the same mu-coordinate as x
                Cx<double> T2[2][3];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) T2[i][j] = Cx<double>{0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Cx<double> la[2], lb[3];
#pragma unroll
                    for (int i = 0; i < 2; ++i) {
                        const double2 v = back[(3 * k + i) * 64 + (lane ^ xm)];
                        la[i] = Cx<double>{v.x, v.y};
                    }
#pragma unroll
                    for (int j = 0; j < 3; ++j) lb[j] = ld_lane(dmu, U.S, 3 * k + j, sy);
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) cmac_ca(T2[i][j], la[i], lb[j]);
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Cx<double> lc[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) lc[j] = ld_lane(dnu, U.S, 3 * k + j, syf);
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) cmac(S[i][j], T2[i][k], lc[j]);
                }
            }
        }
    }
    if constexpr (MODE != kPlaqOnly) {
        // the next group's backward links overwrite these: every lane has read
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (live) {
            double2 *omu = out.p + mu * S9;
            Cx<double> u0[2][3];  // rows 0 and 1 of U_mu(x)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) u0[a][b] = ld_lane(dmu, U.S, 3 * a + b, s);
            if (!smear) {  // a direction outside the mask is copied
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) st_lane(omu, out.S, 3 * a + b, s, u0[a][b]);
#pragma unroll
                for (int b = 0; b < 3; ++b) st_lane(omu, out.S, 6 + b, s, ld_lane(dmu, U.S, 6 + b, s));
            } else {
                Cx<double> wm[2][3], v[3][3];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        wm[i][j].re = fma(c2, S[i][j].re, c1 * u0[i][j].re);
                        wm[i][j].im = fma(c2, S[i][j].im, c1 * u0[i][j].im);
                    }
                reunitarise(wm, v);
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) st_lane(omu, out.S, 3 * a + b, s, v[a][b]);
            }
        }
    }
    if constexpr (MODE != kApe) {
        if (!live) sp = tp = 0.0;
        sp = wave_sum(sp);
        tp = wave_sum(tp);
        if (lane == 0) {
            partials[grp * 4 + w] = sp;
            partials[4 * ngroups + grp * 4 + w] = tp;
        }
    }
}

// One wave's share of a step: direction mu of the 64 sites of group grp
// (FP64 with the row projection: ape_group_f64, wave mu of the group).
// Writes the smeared links (modes kApe, kApePlaq; a direction outside mask
// is copied unchanged, mask is 0xF in kApePlaq) and, in the plaquette
// modes, the owned planes' trace sum of the INPUT links for (grp, mu):
// partials[grp*4 + mu] (spatial planes, waves 0 and 1) and
// partials[4*ngroups + grp*4 + mu] (temporal planes, waves 2 and 3).
// Depends only on (grp, mu), never on the launch geometry.
template <typename R, int NR, int MODE, int PROJ = 0>
__device__ __forceinline__ void ape_group(const Geo &g, const LinksRO<R, NR> &U, const LinksWO<R, NR> &out, double c1,
                                          double c2, unsigned mask, double *__restrict__ partials, int grp, int mu,
                                          int lane, const nv4_t<R> *own = nullptr, double2 *back64 = nullptr) {
    static_assert(PROJ == 0 || MODE == kApe, "the polar projection runs without the fused plaquette");
    if constexpr (sizeof(R) == 8 && PROJ == 0) {
        // FP64 with the row projection: four directions per wave (mu is
        // then the wave's index within the group)
        ape_group_f64<MODE>(g, U, out, c1, c2, mask, partials, grp, mu, lane, back64);
        return;
    }
    const int ngroups = num_groups(g);
    double p = 0.0;
    Site x;
    if (group_site(g, grp, lane, x)) {
        const int s = x.s;
        if constexpr (MODE == kPlaqOnly) {
            M23<R> u0;
            U.rows01(mu, s, u0);
            p = owned_plaquettes(g, U, x, mu, u0);
        } else if (!((mask >> mu) & 1u)) {  // wave-uniform: not smeared
            M3<R> u;
            U.full(mu, s, u);
            out.store(mu, s, u.e);
        } else if constexpr (PROJ == 1) {
            M3<R> S, u;
            staple_sum_full(g, U, x, mu, mask, S);
            U.full(mu, s, u);
            Cx<double> w[3][3], v[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    w[i][jj].re = fma(c2, (double)S.e[i][jj].re, c1 * (double)u.e[i][jj].re);
                    w[i][jj].im = fma(c2, (double)S.e[i][jj].im, c1 * (double)u.e[i][jj].im);
                }
            polar_project(w, v);
            store_narrowed(out, mu, s, v);
        } else {
            M23<R> S, u0;
            if constexpr (MODE == kApePlaq) {  // the plaquette needs u0 in the staple loop
                if (own) own_rows01(own, mu, u0);
                else U.rows01(mu, s, u0);
                staple_sum_rows01<R, NR, true>(g, U, x, mu, mask, S, u0, p, own);
            } else {
                double unused;
                staple_sum_rows01<R, NR, false>(g, U, x, mu, mask, S, u0, unused, own);
                if (own) own_rows01(own, mu, u0);
                else U.rows01(mu, s, u0);
            }
            Cx<double> wm[2][3], v[3][3];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    wm[i][jj].re = fma(c2, (double)S.e[i][jj].re, c1 * (double)u0.e[i][jj].re);
                    wm[i][jj].im = fma(c2, (double)S.e[i][jj].im, c1 * (double)u0.e[i][jj].im);
                }
            reunitarise(wm, v);
            store_narrowed(out, mu, s, v);
        }
    }
    if constexpr (MODE != kApe) {
        p = wave_sum(p);
        if (lane == 0) {
            const bool temporal = mu >= 2;
            partials[grp * 4 + mu] = temporal ? 0.0 : p;
            partials[4 * ngroups + grp * 4 + mu] = temporal ? p : 0.0;
        }
    }
}

}  // namespace qdpx
