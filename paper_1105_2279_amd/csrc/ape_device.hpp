// Device-side APE smearing work shared by the single-lattice kernels and
// the persistent batched kernel: staple sums restricted to rows 0 and 1,
// the per-64-site-group step (with the FP64 step's fused plaquette traces)
// and the plaquette pass.
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

// Full link in FP64: stored rows widened, row 2 rebuilt in FP64 for LINK12
// and, as the FP64 step takes it, for FP64 links (rows 0 and 1 read, a third
// fewer loads; the 18-real FP32 format is read whole).
template <typename R, int NR>
__device__ __forceinline__ void load_f64(const LinksRO<R, NR> &U, int mu, int s, M3<double> &m) {
    constexpr int kRows = (NR == 2 || sizeof(R) == 8) ? 2 : 3;
    Cx<R> r[3][3];
    U.template load_rows<false, kRows>(mu, s, r);
#pragma unroll
    for (int a = 0; a < kRows; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) m.e[a][b] = Cx<double>{(double)r[a][b].re, (double)r[a][b].im};
    if constexpr (kRows == 2) rebuild_row2(m);
}

// Re Tr P_{mu nu}(x) = Re Tr[(U_mu(x) U_nu(x+mu)) (U_nu(x) U_mu(x+nu))^dag] of
// the stored links widened to FP64 (row 2 rebuilt in FP64, load_f64), every
// product and sum in FP64: the plaquette pass behind every plaquette of
// FP32 links (standalone, per step, batched) and of FP64 links outside the
// fused step.  s_mu = x+mu, s_nu = x+nu.  Each link is loaded once, whole.
template <typename R, int NR>
__device__ __forceinline__ double plaquette_plane(const LinksRO<R, NR> &U, int mu, int nu, int s, int s_mu,
                                                  int s_nu) {
    M3<double> m;  // U_mu(x) U_nu(x+mu)
    {
        M3<double> a, b;
        load_f64(U, mu, s, a);
        load_f64(U, nu, s_mu, b);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                Cx<double> t{0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 3; ++k) cmac(t, a.e[i][k], b.e[k][j]);
                m.e[i][j] = t;
            }
    }
    M3<double> c, d;  // U_mu(x+nu), U_nu(x)
    load_f64(U, mu, s_nu, c);
    load_f64(U, nu, s, d);
    double p = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<double> n{0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac(n, d.e[i][k], c.e[k][j]);
            p = fma(m.e[i][j].re, n.re, fma(m.e[i][j].im, n.im, p));
        }
    return p;
}

template <typename R, int NR, int MU, int NU>
__device__ __forceinline__ double plaquette_at(const Geo &g, const LinksRO<R, NR> &U, const Site &x) {
    return plaquette_plane(U, MU, NU, x.s, hop_fwd(g, x.s, x.c[MU], MU), hop_fwd(g, x.s, x.c[NU], NU));
}

// The plaquette pass: three waves per 64-site group, each lane taking one
// spatial and one temporal plane of its site, wave 0 planes (0,1) and (2,3),
// wave 1 (0,2) and (1,3), wave 2 (1,2) and (0,3) (directions known at
// compile time, three times the waves of a site-per-lane loop over six
// planes).  Wave w of group grp writes its spatial sum to partials[3 grp + w]
// and its temporal sum to partials[3 ngroups + 3 grp + w]; every launch that
// reports a plaquette of stored links goes through here, so they all agree
// bit for bit.
constexpr int kPlaqWavesPerGroup = 3;

template <typename R, int NR>
__device__ __forceinline__ void plaquette_wave(const Geo &g, const LinksRO<R, NR> &U, int grp, int w, int lane,
                                               double *__restrict__ partials) {
    double sp = 0.0, tp = 0.0;
    Site x;
    if (group_site(g, grp, lane, x)) {
        if (w == 0) {
            sp = plaquette_at<R, NR, 0, 1>(g, U, x);
            tp = plaquette_at<R, NR, 2, 3>(g, U, x);
        } else if (w == 1) {
            sp = plaquette_at<R, NR, 0, 2>(g, U, x);
            tp = plaquette_at<R, NR, 1, 3>(g, U, x);
        } else {
            sp = plaquette_at<R, NR, 1, 2>(g, U, x);
            tp = plaquette_at<R, NR, 0, 3>(g, U, x);
        }
    }
    sp = wave_sum(sp);
    tp = wave_sum(tp);
    if (lane == 0) {
        const int n3 = kPlaqWavesPerGroup * num_groups(g);
        partials[kPlaqWavesPerGroup * grp + w] = sp;
        partials[n3 + kPlaqWavesPerGroup * grp + w] = tp;
    }
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

// Columns 0 and 1 of the backward link U_mu(x-mu) of group grp's sites (row
// 2 rebuilt for LINK12), all the lower staples of the other three
// directions read of it, into back[(mu*3 + k)*64 + lane] as (U_k0, U_k1)
// pairs; back_cols01 of the block's other direction waves reads them after a
// barrier.  The same loads and rebuild as U.full in the lower staple, so the
// staged values are the ones it would form.
template <typename R, int NR>
__device__ __forceinline__ void stage_back_link(const Geo &g, const LinksRO<R, NR> &U, int grp, int mu, int lane,
                                                nv4_t<R> *back) {
    Site x;
    if (!group_site(g, grp, lane, x)) return;
    M3<R> A;
    U.full(mu, hop_bwd(g, x.s, coord(x, mu), mu), A);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        nv4_t<R> v;
        v.x = A.e[k][0].re;
        v.y = A.e[k][0].im;
        v.z = A.e[k][1].re;
        v.w = A.e[k][1].im;
        back[(mu * 3 + k) * 64 + lane] = v;
    }
}

// Columns 0 and 1 of U_nu(x-nu) from the block's LDS copy (column 2 unset:
// the lower staple's (A^dag)(rows 0,1) reads only these).
template <typename R> __device__ __forceinline__ void back_cols01(const nv4_t<R> *back, int nu, M3<R> &A) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const nv4_t<R> v = back[(nu * 3 + k) * 64 + lane];
        A.e[k][0] = Cx<R>{v.x, v.y};
        A.e[k][1] = Cx<R>{v.z, v.w};
    }
}

// ------------------------------------------------ FP32 staple sum by plane
// The upper staples of U_mu(x) and U_nu(x) share one product: with
// P = U_mu(x+nu) U_nu(x+mu)^dag the upper staple of U_mu(x) is U_nu(x) P and
// that of U_nu(x) is U_mu(x) P^dag.  In each plane of a site one of the two
// directions, the producer d, forms P_d = U_d(x+c) U_c(x+d)^dag (c the other
// direction, the consumer): rows 0 and 1 as rows 0 and 1 of U_d(x+c) times
// U_c(x+d)^dag, row 2 rebuilt as conj(row0 x row1), P being SU(3) to
// rounding.  d is the lower direction in even groups and the higher one in
// odd groups, so two neighbouring groups form equally many products per
// direction.  The staple sum of U_mu(x) takes the planes nu = mu^1, mu^2,
// mu^3 in that order; in each the lower staple is added to the sum and then
// the upper one, formed on its own: U_c(x) P_d for the producer,
// U_d(x) P_d^dag for the consumer.  Whether each wave forms the products it
// needs (staple_sum_rows01) or a plane's product is formed once and passed
// to the consumer through LDS (staple_sum_rows01_shared), the arithmetic
// and its order are the same, so every path gives the same bits.
__device__ __forceinline__ bool plane_producer(int mu, int nu, int grp) { return (mu < nu) != ((grp & 1) != 0); }

// P = U_d(x+c) U_c(x+d)^dag, rows 0 and 1 formed, row 2 rebuilt.
template <typename R, int NR>
__device__ __forceinline__ void plane_product(const Geo &g, const LinksRO<R, NR> &U, const Site &x, int d, int c,
                                              M3<R> &P) {
    M23<R> B;
    U.rows01(d, hop_fwd(g, x.s, site_coord<R>(x, c), c), B);
    M3<R> C;
    U.full(c, hop_fwd(g, x.s, site_coord<R>(x, d), d), C);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Cx<R> t{(R)0, (R)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) cmac_cb(t, B.e[i][k], C.e[j][k]);
            P.e[i][j] = t;
        }
    rebuild_row2(P);
}

// X = rows 0 and 1 of the upper staple from the plane's product: A P_d for
// the producer, A P_d^dag for the consumer (A = rows 0 and 1 of U_nu(x)).
template <typename R>
__device__ __forceinline__ void upper_staple(const M23<R> &A, const M3<R> &P, bool prod, M23<R> &X) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) X.e[i][j] = Cx<R>{(R)0, (R)0};
    if (prod) acc_23_33(X, A, P);  // wave-uniform
    else acc_23_33dag(X, A, P);
}
// S += X
template <typename R> __device__ __forceinline__ void add_23(M23<R> &S, const M23<R> &X) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            S.e[i][j].re += X.e[i][j].re;
            S.e[i][j].im += X.e[i][j].im;
        }
}

// S += rows 0 and 1 of the lower staple U_nu(y)^dag U_mu(y) U_nu(y+mu),
// y = x - nu.  back: the group's backward links staged in LDS (FP32), or
// nullptr to load U_nu(y).
template <typename R, int NR>
__device__ __forceinline__ void add_lower_staple(const Geo &g, const LinksRO<R, NR> &U, const Site &x, int mu, int nu,
                                                 M23<R> &S, const nv4_t<R> *back) {
    const int y = hop_bwd(g, x.s, site_coord<R>(x, nu), nu);
    M3<R> A;
    if (back) back_cols01(back, nu, A);  // wave nu's backward link, staged in LDS
    else U.full(nu, y, A);
    M3<R> B;
    U.full(mu, y, B);
    M23<R> T;
    mul_dag23_33(A, B, T);
    M3<R> C;
    U.full(nu, hop_fwd(g, y, site_coord<R>(x, mu), mu), C);  // y has the same mu-coordinate as x
    acc_23_33(S, T, C);
}

// Staple sum (rows 0 and 1) of link (x, mu) of group grp over the planes
// (mu, nu) with nu in mask (bits 0..3), every product formed by this wave.
// own / back: the group's own links and backward links staged in LDS (FP32),
// or nullptr to load them.
template <typename R, int NR>
__device__ __forceinline__ void staple_sum_rows01(const Geo &g, const LinksRO<R, NR> &U, const Site &x, int mu,
                                                  int grp, unsigned mask, M23<R> &S, const nv4_t<R> *own = nullptr,
                                                  const nv4_t<R> *back = nullptr) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S.e[i][j] = Cx<R>{(R)0, (R)0};
#pragma unroll 1
    for (int p = 0; p < 3; ++p) {
        const int nu = mu ^ (p + 1);
        if (!((mask >> nu) & 1u)) continue;  // wave-uniform
        const bool prod = plane_producer(mu, nu, grp);
        // the upper staple X is formed on its own, the lower one added to S,
        // then X: in this order the compiler keeps 77 registers (LDS tile 2,
        // FP32-12) instead of 105 with the lower staple first
        M3<R> P;
        plane_product(g, U, x, prod ? mu : nu, prod ? nu : mu, P);
        M23<R> A;                         // rows 0 and 1 of U_nu(x)
        if (own) own_rows01(own, nu, A);  // wave nu's own link, staged in LDS
        else U.rows01(nu, x.s, A);
        M23<R> X;
        upper_staple(A, P, prod, X);
        add_lower_staple(g, U, x, mu, nu, S, back);
        add_23(S, X);
    }
}

// The FP32 step's LDS tile levels: 1 own links, 2 own and backward links,
// 3 own and backward links and four slots (two per phase, even and odd
// phases apart) for the products the producers of a phase pass to their
// consumers, 4 own links and the slots (backward links loaded).  A slot
// holds 3 entries per lane: rows 0 and 1 of P in pairs; the reader
// rebuilds row 2 from them exactly as plane_product did.
constexpr int kApeTileF4 = 4 * 3 * 64;
constexpr int kApeSlotF4 = 3 * 64;
__host__ __device__ constexpr bool ape_lds_back(int level) { return level == 2 || level == 3; }
__host__ __device__ constexpr bool ape_lds_slots(int level) { return level >= 3; }
// float4 entries per 64-site group: own links, backward links, slots in
// that order
__host__ __device__ constexpr int ape_lds_f4_per_group(int level) {
    return (level >= 1 ? kApeTileF4 : 0) + (ape_lds_back(level) ? kApeTileF4 : 0) +
           (ape_lds_slots(level) ? 4 * kApeSlotF4 : 0);
}

// staple_sum_rows01 with each plane's product formed once: in phase p the
// four waves of the group take the planes (mu, mu ^ (p + 1)); the two
// producers store rows 0 and 1 of P_d in the plane's LDS slot (slots of
// even and odd phases apart, so each slot is rewritten only two phases
// later, after a barrier its readers have passed), both add their lower
// staples, and after one block barrier the consumers read P_d.  Contains
// block barriers: every wave of the block calls it, with work false where
// its group is past the end or its direction is not smeared (it then only
// meets the barriers).
template <typename R, int NR>
__device__ __forceinline__ void staple_sum_rows01_shared(const Geo &g, const LinksRO<R, NR> &U, const Site &x,
                                                         int mu, int grp, bool work, unsigned mask, M23<R> &S,
                                                         const nv4_t<R> *own, const nv4_t<R> *back,
                                                         nv4_t<R> *slots) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S.e[i][j] = Cx<R>{(R)0, (R)0};
#pragma unroll 1
    for (int p = 0; p < 3; ++p) {
        const int nu = mu ^ (p + 1);
        const bool act = work && ((mask >> nu) & 1u);  // wave-uniform; the same for both waves of the plane
        const bool prod = plane_producer(mu, nu, grp);
        const int lo = mu < nu ? mu : nu;
        nv4_t<R> *slot = slots + (2 * (p & 1) + (p == 0 ? lo >> 1 : lo)) * kApeSlotF4;  // the phase's two planes
        if (act) {
            if (prod) {
                M3<R> P;
                plane_product(g, U, x, mu, nu, P);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const Cx<R> &z0 = P.e[(2 * k) / 3][(2 * k) % 3], &z1 = P.e[(2 * k + 1) / 3][(2 * k + 1) % 3];
                    nv4_t<R> v;
                    v.x = z0.re;
                    v.y = z0.im;
                    v.z = z1.re;
                    v.w = z1.im;
                    slot[k * 64 + lane] = v;
                }
            }
            add_lower_staple(g, U, x, mu, nu, S, back);
        }
        __syncthreads();  // this phase's products are in LDS
        if (act) {
            M3<R> P;  // P_d, re-read by the producer too: the same bits it stored
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const nv4_t<R> v = slot[k * 64 + lane];
                P.e[(2 * k) / 3][(2 * k) % 3] = Cx<R>{v.x, v.y};
                P.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = Cx<R>{v.z, v.w};
            }
            rebuild_row2(P);
            M23<R> A;  // rows 0 and 1 of U_nu(x)
            own_rows01(own, nu, A);
            M23<R> X;
            upper_staple(A, P, prod, X);
            add_23(S, X);
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

// W = c1 U_mu(x) + c2 S (rows 0 and 1, in FP64), projected by rows in FP64
// and stored in link precision.  own: the group's own links in LDS, or
// nullptr to load U_mu(x).
template <typename R, int NR>
__device__ __forceinline__ void finish_rows01(const LinksRO<R, NR> &U, const LinksWO<R, NR> &out, double c1,
                                              double c2, int mu, int s, const M23<R> &S, const nv4_t<R> *own) {
    M23<R> u0;
    if (own) own_rows01(own, mu, u0);
    else U.rows01(mu, s, u0);
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

// What one (64-site group, direction) wave computes.
enum ApeMode { kApe = 0, kApePlaq = 1 };

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
// and shares through LDS.  Every link is read as its rows 0 and 1, row 2
// rebuilt in FP64.  A link update then issues 84 vector loads of 16 bytes
// instead of 151: the memory pipeline, not the arithmetic, bounds the FP64
// step.  The fused plaquette takes each plane once, in the
// lane of its lower direction.  Direction-dependent addresses differ
// between lanes here, so they are formed in 64 bits per lane.

constexpr int kF64BackPerWave = 6 * 64;  // double2 per wave: columns 0 and 1 of one backward link per lane

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
// FP64 link at site s: rows 0 and 1 loaded, row 2 rebuilt as conj(row0 x row1)
// (exact for SU(3) links; a smeared link's stored row 2 is that by
// construction), so each neighbour link moves 96 bytes instead of 144.
__device__ __forceinline__ void ld_lane_rows01(const double2 *dir, int64_t S, int s, M3<double> &m) {
#pragma unroll
    for (int c = 0; c < 6; ++c) m.e[c / 3][c % 3] = ld_lane(dir, S, c, s);
    rebuild_row2(m);
}

// One wave's share of an FP64 step: the four directions of 16 sites of
// group grp.  back: this wave's kF64BackPerWave LDS entries.  In kApePlaq
// mode also the plaquette traces of the INPUT links: partials[grp*4 + w]
// (spatial planes) and partials[4*ngroups + grp*4 + w] (temporal planes).
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
    const bool smear = (mask >> mu) & 1u;
    const int64_t S9 = 9 * U.S;
    const double2 *dmu = U.p + mu * S9;  // this lane's direction
    {
        // columns 0 and 1 of the backward link U_mu(x-mu) (all the lower
        // staple reads), for the lanes of the other directions: entry
        // 2k + i holds element (k, i)
        const int sb = hop_bwd_v(g, s, cmu, mu);
        M3<double> bl;
        ld_lane_rows01(dmu, U.S, sb, bl);
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 2; ++i) back[(2 * k + i) * 64 + lane] = double2{bl.e[k][i].re, bl.e[k][i].im};
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
        const bool act = smear && ((mask >> nu) & 1u);
        const bool own_plane = mu < nu;  // the plaquette of the plane is taken here
        const int cnu = coord(x, nu);
        // upper: U_nu(x) U_mu(x+nu) U_nu(x+mu)^dag.  B = U_mu(x+nu) is loaded by
        // every lane (the partner needs it); rows of U_nu(x) (the partner's
        // own rows) and of U_nu(x+mu) (the partner's B) are exchanged one at
        // a time as the products consume them.
        M3<double> B;
        const int s_nu = hop_fwd_v(g, s, cnu, nu);
        ld_lane_rows01(dmu, U.S, s_nu, B);
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
        {
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
                        const double2 v = back[(2 * k + i) * 64 + (lane ^ xm)];
                        la[i] = Cx<double>{v.x, v.y};
                    }
                    if (k < 2) {
#pragma unroll
                        for (int j = 0; j < 3; ++j) lb[j] = ld_lane(dmu, U.S, 3 * k + j, sy);
                    } else {  // row 2 of U_mu(y), rebuilt from its rows 0 and 1
                        M3<double> m;
                        ld_lane_rows01(dmu, U.S, sy, m);
#pragma unroll
                        for (int j = 0; j < 3; ++j) lb[j] = m.e[2][j];
                    }
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) cmac_ca(T2[i][j], la[i], lb[j]);
                }
                M3<double> LC;
                ld_lane_rows01(dnu, U.S, syf, LC);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    Cx<double> lc[3];
#pragma unroll
                    for (int j = 0; j < 3; ++j) lc[j] = LC.e[k][j];
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) cmac(S[i][j], T2[i][k], lc[j]);
                }
            }
        }
    }
    {
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

// One wave's share of a step: direction mu of the 64 sites of group grp,
// the smeared links written (a direction outside mask is copied unchanged).
// FP64 links with the row projection go to ape_group_f64 (mu is then the
// wave's index within the group), which also has the plaquette modes.
// Depends only on (grp, mu), never on the launch geometry.
template <typename R, int NR, int MODE, int PROJ = 0>
__device__ __forceinline__ void ape_group(const Geo &g, const LinksRO<R, NR> &U, const LinksWO<R, NR> &out, double c1,
                                          double c2, unsigned mask, double *__restrict__ partials, int grp, int mu,
                                          int lane, const nv4_t<R> *own = nullptr, double2 *back64 = nullptr,
                                          const nv4_t<R> *back = nullptr) {
    static_assert(PROJ == 0 || MODE == kApe, "the polar projection runs without the fused plaquette");
    if constexpr (sizeof(R) == 8 && PROJ == 0) {
        // FP64 with the row projection: four directions per wave (mu is
        // then the wave's index within the group)
        ape_group_f64<MODE>(g, U, out, c1, c2, mask, partials, grp, mu, lane, back64);
        return;
    }
    static_assert(MODE == kApe || (sizeof(R) == 8 && PROJ == 0),
                  "plaquettes of FP32 links come from the plaquette pass");
    Site x;
    if (group_site(g, grp, lane, x)) {
        const int s = x.s;
        if (!((mask >> mu) & 1u)) {  // wave-uniform: not smeared
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
            M23<R> S;
            staple_sum_rows01<R, NR>(g, U, x, mu, grp, mask, S, own, back);
            finish_rows01<R, NR>(U, out, c1, c2, mu, s, S, own);
        }
    }
}

// ape_group for the FP32 step at LDS tile level 3 (each plane's upper
// product formed once and passed through LDS).  Contains block barriers:
// every wave of the block calls it; valid is false for a group past the end.
template <typename R, int NR>
__device__ __forceinline__ void ape_group_shared(const Geo &g, const LinksRO<R, NR> &U, const LinksWO<R, NR> &out,
                                                 double c1, double c2, unsigned mask, int grp, bool valid, int mu,
                                                 int lane, const nv4_t<R> *own, const nv4_t<R> *back,
                                                 nv4_t<R> *slots) {
    Site x;
    const bool live = valid && group_site(g, grp, lane, x);
    if (!live) x.init(g, 0);  // padding lanes and groups past the end compute on site 0 and store nothing
    const bool smear = (mask >> mu) & 1u;
    M23<R> S;
    staple_sum_rows01_shared<R, NR>(g, U, x, mu, grp, valid && smear, mask, S, own, back, slots);
    if (live) {
        if (!smear) {  // wave-uniform: not smeared
            M3<R> u;
            U.full(mu, x.s, u);
            out.store(mu, x.s, u.e);
        } else {
            finish_rows01<R, NR>(U, out, c1, c2, mu, x.s, S, own);
        }
    }
}

}  // namespace qdpx
