// Device-side building blocks: complex numbers, SoA field access, SU(3)
// products restricted to the rows that are actually needed, periodic
// neighbour addressing, the FP64 row Gram-Schmidt projection and
// deterministic wave/block reductions.  gfx950, wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qdpx {

// ------------------------------------------------------ integer division
// Quotient of a non-negative int n < 2^31 by a fixed divisor d >= 1 as one
// multiply-high, an add and a shift: with l = ceil(log2 d) and
// m = floor(2^32 (2^l - d) / d) + 1, n / d = (mulhi(m, n) + n) >> l (the
// round-up method of Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994; n < 2^31 keeps the sum in 32 bits).
// The constants are made on the host.  gfx950 has no scalar floating point,
// so a plain division, even of a wave-uniform value, is a long emulated
// sequence on the vector ALU; this form stays on the scalar unit for
// wave-uniform operands and is three instructions per lane otherwise.
struct FastDiv {
    uint32_t d, m, l;
    static FastDiv make(uint32_t d) {
        FastDiv f;
        f.d = d;
        f.l = 0;
        while ((1ull << f.l) < d) ++f.l;
        f.m = (uint32_t)(((1ull << 32) * ((1ull << f.l) - d)) / d + 1);
        return f;
    }
    __host__ __device__ __forceinline__ int div(int n) const {
        return (int)(((uint32_t)(((uint64_t)m * (uint32_t)n) >> 32) + (uint32_t)n) >> l);
    }
};

// ---------------------------------------------------------------- geometry
// Extents, per-direction site strides, the padded SoA stride and the
// mapping of 64-site groups (one group per wave) to sites.
//
// Brick mapping (bwl = 4 or 3): when Lx is a multiple of bw = 2^bwl and Ly a
// multiple of 64/bw, group g is a bw x (64/bw) brick of one (z, t) plane:
// g = p + P*(z + Lz*t) with p the brick within the xy plane (P bricks per
// plane, pbx along x); lane l sits at x = xb*bw + l % bw, y = yb*(64/bw) + l / bw.
// A wave then touches 64/bw rows of bw consecutive sites (whole cache lines),
// and the groups of one xy plane are numbered consecutively, so a window of
// t planes can be walked together (see traverse()).  Otherwise (bwl = 0)
// group g is the 64 consecutive sites [64 g, 64 g + 64).  The mapping depends
// only on the extents, so per-group partial sums never depend on the launch.
struct Geo {
    int L[4];
    int st[4];  // 1, Lx, Lx*Ly, Lx*Ly*Lz
    int V;
    int bwl;    // log2 of the brick width, 0 for the linear mapping
    int P;      // bricks per xy plane
    int pbx;    // bricks along x
    int ncol;   // groups per t plane when every group lies in one t plane, else 0
    int64_t S;  // padded site count: V rounded up to 256
    // divisors of the site decoding: Lx, Ly, Lz, P, pbx, P*Lz, ncol/8
    FastDiv dL0, dL1, dL2, dP, dpbx, dplane, dslab;
};

// Neighbour addressing for one site: coordinates are decoded once, every hop
// is a stride add with a wrap test (no division in the hot loop).
struct Site {
    int s;
    int c[4];
    __device__ __forceinline__ void init(const Geo &g, int site) {
        s = site;
        const int q0 = g.dL0.div(site), q1 = g.dL1.div(q0), q2 = g.dL2.div(q1);
        c[0] = site - q0 * g.L[0];
        c[1] = q0 - q1 * g.L[1];
        c[2] = q1 - q2 * g.L[2];
        c[3] = q2;
    }
};

__device__ __forceinline__ int num_groups(const Geo &g) { return (g.V + 63) >> 6; }

// Site of lane `lane` of group `grp` (grp is wave-uniform, so the divisions
// run on the scalar unit).  Returns false for the padding lanes of the last
// linear group.
__device__ __forceinline__ bool group_site(const Geo &g, int grp, int lane, Site &x) {
    if (g.bwl) {
        const int r = g.dP.div(grp), p = grp - r * g.P;
        const int t = g.dL2.div(r), z = r - t * g.L[2];
        const int yb = g.dpbx.div(p), xb = p - yb * g.pbx;
        const int bw = 1 << g.bwl;
        x.c[0] = xb * bw + (lane & (bw - 1));
        x.c[1] = yb * (64 >> g.bwl) + (lane >> g.bwl);
        x.c[2] = z;
        x.c[3] = t;
        x.s = x.c[0] + g.L[0] * (x.c[1] + g.L[1] * (z + g.L[2] * t));
        return true;
    }
    const int s = grp * 64 + lane;
    if (s >= g.V) return false;
    x.init(g, s);
    return true;
}

// Launch order -> group.  With the brick mapping and a window of tw t planes
// (tw divides Lt), consecutive logical indices walk the tw planes of one
// (brick, z) column before moving on, so the blocks in flight on one XCD hold
// each other's t neighbours in L2.  tw = 1 (or the linear mapping) is the
// identity.  A bijection on [0, num_groups).
// tw is a power of two (checked on the host).
__device__ __forceinline__ int traverse(const Geo &g, int i, int tw) {
    if (!g.bwl || tw <= 1) return i;
    const int tin = i & (tw - 1), rest = i >> __builtin_ctz(tw);
    const int plane = g.P * g.L[2];
    const int tc = g.dplane.div(rest), pz = rest - tc * plane;
    return pz + plane * (tc * tw + tin);
}

// Launch order -> group, XCD slab walk.  Blocks are dispatched to the 8
// XCDs round-robin (block b runs on XCD b % 8).  The ncol groups of a t plane
// (column index c = brick + P z) are split into 8 contiguous ranges of
// ncol / 8 columns, a slab of z planes, and XCD x takes range x in every t
// plane, walking its slab t plane by t plane.  A group's x, y and z
// neighbours then lie in the same slab a few groups away, and its t
// neighbours ncol / 8 groups away, all handled on the same XCD close together
// in time, so they are served from that XCD's L2.  Requires ncol % 8 == 0 and
// num_groups % (8 m) == 0 for m groups per block (checked on the host).
// A bijection.
// m is a power of two (groups per block times groups per wave).
__device__ __forceinline__ int slabwalk(const Geo &g, int i, int m) {
    const int blk = i >> __builtin_ctz(m), within = i & (m - 1);
    const int x = blk & 7, jj = (blk >> 3) * m + within;
    const int cx = g.ncol >> 3;
    const int t = g.dslab.div(jj), k = jj - t * cx;
    return (x * cx + k) + g.ncol * t;
}

// x.c[mu] for a wave-uniform but run-time mu, by selects: indexing the
// per-lane array directly would place it in scratch memory.
__device__ __forceinline__ int coord(const Site &x, int mu) {
    return mu == 0 ? x.c[0] : mu == 1 ? x.c[1] : mu == 2 ? x.c[2] : x.c[3];
}

__device__ __forceinline__ int hop_fwd(const Geo &g, int s, int cmu, int mu) {
    return (cmu == g.L[mu] - 1) ? s - (g.L[mu] - 1) * g.st[mu] : s + g.st[mu];
}
__device__ __forceinline__ int hop_bwd(const Geo &g, int s, int cmu, int mu) {
    return (cmu == 0) ? s + (g.L[mu] - 1) * g.st[mu] : s - g.st[mu];
}

// ------------------------------------------------------------------ complex
template <typename R> struct V2;
template <> struct V2<double> { using T = double2; };
template <> struct V2<float> { using T = float2; };
template <typename R> using vec2_t = typename V2<R>::T;

template <typename R> struct Cx { R re, im; };


// Every field lives in global memory.  Pointers that come out of a device
// table are generic; converting them to the global address space lets the
// compiler emit global (not flat) loads and stores.
template <typename T> __device__ __forceinline__ const __attribute__((address_space(1))) T *gptr(const void *p) {
    return (const __attribute__((address_space(1))) T *)p;
}
template <typename T> __device__ __forceinline__ __attribute__((address_space(1))) T *gptr_w(void *p) {
    return (__attribute__((address_space(1))) T *)p;
}

// Component bases are wave-uniform.  Passing one through an empty asm with an
// SGPR constraint makes it an opaque scalar value, so the compiler keeps
// base + 32-bit site offset as one SGPR-base / VGPR-offset global access
// instead of re-associating the sum into 64-bit per-lane address arithmetic.
template <typename T> __device__ __forceinline__ T *sbase(T *p) {
    asm("" : "+s"(p));
    return p;
}
// The per-lane byte offset likewise stays an opaque 32-bit value, so it is
// never widened into a 64-bit multiply before the address is formed.
__device__ __forceinline__ uint32_t voff(uint32_t o) {
    asm("" : "+v"(o));
    return o;
}

// Streaming (non-temporal) access to one complex element: the builtins need a
// native two-wide vector type.
template <typename R> using nv2_t = R __attribute__((ext_vector_type(2)));
template <typename R> __device__ __forceinline__ void store_stream(void *addr, R re, R im) {
    nv2_t<R> v;
    v.x = re;
    v.y = im;
    __builtin_nontemporal_store(v, gptr_w<nv2_t<R>>(addr));
}

// acc += a * b
template <typename R> __device__ __forceinline__ void cmac(Cx<R> &acc, const Cx<R> &a, const Cx<R> &b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
}
// acc += a * conj(b)
template <typename R> __device__ __forceinline__ void cmac_cb(Cx<R> &acc, const Cx<R> &a, const Cx<R> &b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.im, b.re, acc.im);
    acc.im = fma(-a.re, b.im, acc.im);
}
// acc += conj(a) * b
template <typename R> __device__ __forceinline__ void cmac_ca(Cx<R> &acc, const Cx<R> &a, const Cx<R> &b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
}
// conj(a*d - b*c): one entry of the conjugated cross product
template <typename R>
__device__ __forceinline__ Cx<R> conj_cross(const Cx<R> &a, const Cx<R> &d, const Cx<R> &b, const Cx<R> &c) {
    R re = a.re * d.re;
    re = fma(-a.im, d.im, re);
    re = fma(-b.re, c.re, re);
    re = fma(b.im, c.im, re);
    R im = a.re * d.im;
    im = fma(a.im, d.re, im);
    im = fma(-b.re, c.im, im);
    im = fma(-b.im, c.re, im);
    return Cx<R>{re, -im};
}

template <typename R> struct M3 { Cx<R> e[3][3]; };   // full 3x3
template <typename R> struct M23 { Cx<R> e[2][3]; };  // rows 0 and 1

// row 2 = conj(row0 x row1)
template <typename R> __device__ __forceinline__ void rebuild_row2(M3<R> &m) {
    m.e[2][0] = conj_cross(m.e[0][1], m.e[1][2], m.e[0][2], m.e[1][1]);
    m.e[2][1] = conj_cross(m.e[0][2], m.e[1][0], m.e[0][0], m.e[1][2]);
    m.e[2][2] = conj_cross(m.e[0][0], m.e[1][1], m.e[0][1], m.e[1][0]);
}

// ----------------------------------------------------------- SoA link field
// NR = stored rows (3: LINK18, 2: LINK12).  Stored element c = 3a + b (row
// a < NR, column b) of direction mu at site s.  Direction mu occupies the
// 3*NR*S complex slots from slot mu*3*NR*S on:
//   FP64  one array of S double2 per element: slot c*S + s;
//   FP32  elements 2k and 2k+1 share the 16-byte entry s of array k (S
//         float4 entries, element 2k in the low half): slot 2kS + 2s + (c&1);
//         with NR = 3 the ninth element (c = 8) has an array of S float2 of
//         its own after the four pair arrays: slot 8S + s.
// A FP32 link is then three (LINK12) or five (LINK18) 16-byte loads per lane,
// which halves the vector-memory instructions the APE staples issue.
template <typename R, int NR> struct LinkLayout {
    static constexpr bool kPaired = sizeof(R) == 4;
    // first slot of the array that holds element c (odd elements start one
    // slot into their pair array)
    __host__ __device__ static constexpr int64_t array(int mu, int c, int64_t S) {
        return (int64_t)mu * 3 * NR * S +
               (kPaired ? (c < 8 ? (int64_t)(c >> 1) * 2 * S + (c & 1) : 8 * S) : (int64_t)c * S);
    }
    // slots between consecutive sites of element c
    __host__ __device__ static constexpr int stride(int c) { return kPaired && c < 8 ? 2 : 1; }
    __host__ __device__ static constexpr int64_t slot(int mu, int c, int64_t S, int64_t s) {
        return array(mu, c, S) + s * stride(c);
    }
};

template <typename R> using nv4_t = R __attribute__((ext_vector_type(4)));

template <typename R, int NR> struct LinksRO {
    using Lay = LinkLayout<R, NR>;
    const vec2_t<R> *__restrict__ p;
    int64_t S;
    // The array base is uniform across the wave (mu is wave-uniform, the
    // element index a constant) and the site offset fits 32 bits (V < 2^28),
    // so every load is one SGPR base + one 32-bit VGPR offset.
    template <bool NT = false> __device__ __forceinline__ Cx<R> ld(int mu, int a, int b, int s) const {
        const int c = a * 3 + b;
        const char *addr = (const char *)sbase(p + Lay::array(mu, c, S)) +
                           voff((uint32_t)s * (uint32_t)(Lay::stride(c) * sizeof(vec2_t<R>)));
        const nv2_t<R> v = NT ? __builtin_nontemporal_load(gptr<nv2_t<R>>(addr)) : *gptr<nv2_t<R>>(addr);
        return Cx<R>{v.x, v.y};
    }
    // FP32: elements 2k and 2k+1 in one 16-byte load
    template <bool NT> __device__ __forceinline__ void ld_pair(int mu, int k, int s, Cx<R> &e0, Cx<R> &e1) const {
        const char *addr = (const char *)sbase(p + Lay::array(mu, 2 * k, S)) + voff((uint32_t)s * 16u);
        const nv4_t<R> v = NT ? __builtin_nontemporal_load(gptr<nv4_t<R>>(addr)) : *gptr<nv4_t<R>>(addr);
        e0 = Cx<R>{v.x, v.y};
        e1 = Cx<R>{v.z, v.w};
    }
    // stored rows 0 .. ROWS-1 of link (mu, s) into e
    template <bool NT, int ROWS, int N> __device__ __forceinline__ void load_rows(int mu, int s, Cx<R> (&e)[N][3]) const {
        static_assert(ROWS <= NR && ROWS <= N, "rows beyond the stored ones");
        if constexpr (Lay::kPaired) {
#pragma unroll
            for (int k = 0; k < (3 * ROWS) / 2; ++k)
                ld_pair<NT>(mu, k, s, e[(2 * k) / 3][(2 * k) % 3], e[(2 * k + 1) / 3][(2 * k + 1) % 3]);
            if constexpr (ROWS == 3) e[2][2] = ld<NT>(mu, 2, 2, s);
        } else {
#pragma unroll
            for (int a = 0; a < ROWS; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) e[a][b] = ld<NT>(mu, a, b, s);
        }
    }
    // The link as the shift and hop kernels read it: every stored row of
    // FP32 18-real links, else rows 0 and 1 with row 2 rebuilt (12-real
    // links; FP64 links, whose stored row 2 is conj(row0 x row1) to rounding
    // for SU(3) links: a third fewer bytes for kernels bound by them).
    template <bool NT> __device__ __forceinline__ void su3(int mu, int s, M3<R> &m) const {
        constexpr int kRows = (NR == 3 && sizeof(R) == 4) ? 3 : 2;
        load_rows<NT, kRows>(mu, s, m.e);
        if constexpr (kRows == 2) rebuild_row2(m);
    }
    __device__ __forceinline__ void rows01(int mu, int s, M23<R> &m) const { load_rows<false, 2>(mu, s, m.e); }
    __device__ __forceinline__ void full(int mu, int s, M3<R> &m) const {
        load_rows<false, NR>(mu, s, m.e);
        if constexpr (NR == 2) rebuild_row2(m);
    }
};

template <typename R, int NR> struct LinksWO {
    using Lay = LinkLayout<R, NR>;
    vec2_t<R> *__restrict__ p;
    int64_t S;
    // Outputs are never re-read by the kernel that writes them: stream them
    // past the caches so L2 keeps the neighbour links.
    __device__ __forceinline__ void st(int mu, int c, int s, const Cx<R> &z) const {
        store_stream<R>((char *)sbase(p + Lay::array(mu, c, S)) +
                            voff((uint32_t)s * (uint32_t)(Lay::stride(c) * sizeof(vec2_t<R>))),
                        z.re, z.im);
    }
    // the NR stored rows of link (mu, s); FP32 as 16-byte pair stores
    __device__ __forceinline__ void store(int mu, int s, const Cx<R> (&e)[3][3]) const {
        if constexpr (Lay::kPaired) {
#pragma unroll
            for (int k = 0; k < (3 * NR) / 2; ++k) {
                const Cx<R> &z0 = e[(2 * k) / 3][(2 * k) % 3], &z1 = e[(2 * k + 1) / 3][(2 * k + 1) % 3];
                nv4_t<R> v;
                v.x = z0.re;
                v.y = z0.im;
                v.z = z1.re;
                v.w = z1.im;
                __builtin_nontemporal_store(
                    v, gptr_w<nv4_t<R>>((char *)sbase(p + Lay::array(mu, 2 * k, S)) + voff((uint32_t)s * 16u)));
            }
            if constexpr (NR == 3) st(mu, 8, s, e[2][2]);
        } else {
#pragma unroll
            for (int a = 0; a < NR; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) st(mu, 3 * a + b, s, e[a][b]);
        }
    }
};

// --------------------------------------------------------- SoA Dirac field
// Component q = 3*spin + colour of site s.  FP64: its own array of S double2,
// p[q*S + s].  FP32: components 2k and 2k+1 share the 16-byte entry s of
// array k (k = 0..5; q even in the low half), so a whole spinor is six
// 16-byte loads.
//
// The hop kernels split a site group's epilogue over four waves; wave w
// finalises and stores the components it owns.  FP64: spin w, components
// 3w + t (t < 3).  FP32: the whole pairs k = w and, for w < 2, k = w + 4
// (slot t is component 2k + (t & 1) of pair k = w + 4 (t >> 1)), so no
// 16-byte entry is ever written in halves by two waves.
template <typename R> struct FermLayout {
    static constexpr bool kPaired = sizeof(R) == 4;
    static constexpr int kOwn = kPaired ? 4 : 3;  // component slots per wave
    // component in slot t of wave w, or -1 where the slot is empty
    __device__ __forceinline__ static int owned(int w, int t) {
        if constexpr (kPaired) {
            const int k = w + 4 * (t >> 1);
            return k < 6 ? 2 * k + (t & 1) : -1;
        } else {
            return 3 * w + t;
        }
    }
};

template <typename R> struct FermRO {
    const vec2_t<R> *__restrict__ p;
    int64_t S;
    using Lay = FermLayout<R>;
    // the whole spinor of site s
    __device__ __forceinline__ void ld_all(int s, Cx<R> (&e)[4][3]) const {
        if constexpr (Lay::kPaired) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const char *b = (const char *)sbase((const char *)p + (int64_t)k * S * 16);
                const nv4_t<R> v = *gptr<nv4_t<R>>(b + voff((uint32_t)s * 16u));
                e[(2 * k) / 3][(2 * k) % 3] = Cx<R>{v.x, v.y};
                e[(2 * k + 1) / 3][(2 * k + 1) % 3] = Cx<R>{v.z, v.w};
            }
        } else {
#pragma unroll
            for (int q = 0; q < 12; ++q) {
                const char *b = (const char *)sbase(p + (int64_t)q * S);
                const nv2_t<R> v = *gptr<nv2_t<R>>(b + voff((uint32_t)s * (uint32_t)sizeof(vec2_t<R>)));
                e[q / 3][q % 3] = Cx<R>{v.x, v.y};
            }
        }
    }
    // the components wave w owns at site s; empty slots are left untouched
    __device__ __forceinline__ void ld_owned(int w, int s, Cx<R> (&z)[Lay::kOwn]) const {
        if constexpr (Lay::kPaired) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = w + 4 * h;
                if (k < 6) {  // wave-uniform
                    const char *b = (const char *)sbase((const char *)p + (int64_t)k * S * 16);
                    const nv4_t<R> v = *gptr<nv4_t<R>>(b + voff((uint32_t)s * 16u));
                    z[2 * h] = Cx<R>{v.x, v.y};
                    z[2 * h + 1] = Cx<R>{v.z, v.w};
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const char *b = (const char *)sbase(p + (int64_t)(3 * w + t) * S);
                const nv2_t<R> v = *gptr<nv2_t<R>>(b + voff((uint32_t)s * (uint32_t)sizeof(vec2_t<R>)));
                z[t] = Cx<R>{v.x, v.y};
            }
        }
    }
};
template <typename R> struct FermWO {
    vec2_t<R> *__restrict__ p;
    int64_t S;
    using Lay = FermLayout<R>;
    // the components wave w owns at site s, streamed past the caches
    __device__ __forceinline__ void st_owned(int w, int s, const Cx<R> (&z)[Lay::kOwn]) const {
        if constexpr (Lay::kPaired) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int k = w + 4 * h;
                if (k < 6) {  // wave-uniform
                    nv4_t<R> v;
                    v.x = z[2 * h].re;
                    v.y = z[2 * h].im;
                    v.z = z[2 * h + 1].re;
                    v.w = z[2 * h + 1].im;
                    char *b = (char *)sbase((char *)p + (int64_t)k * S * 16);
                    __builtin_nontemporal_store(v, gptr_w<nv4_t<R>>(b + voff((uint32_t)s * 16u)));
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < 3; ++t)
                store_stream<R>((char *)sbase(p + (int64_t)(3 * w + t) * S) +
                                    voff((uint32_t)s * (uint32_t)sizeof(vec2_t<R>)),
                                z[t].re, z[t].im);
        }
    }
};

// ------------------------------------------------------------ projection
// 1/sqrt(n) for a finite n > 0: the hardware reciprocal square root refined
// by two Newton steps y <- y + y (1 - n y^2) / 2 (quadratic convergence: from
// an estimate good to 2^-14 relative the result is within a few ulp), nine
// instructions where the correctly rounded square root and division take
// about thirty.
__device__ __forceinline__ double rsqrt_nr(double n) {
    double y = __builtin_amdgcn_rsq(n);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-(n * y), y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// Row Gram-Schmidt in FP64: u = w0/|w0|; v = w1 - (u^dag w1) u, v /= |v|;
// row 2 = conj(u x v).  A vanishing norm gives NaN.
__device__ __forceinline__ void reunitarise(const Cx<double> w[2][3], Cx<double> v[3][3]) {
    double n0 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n0 = fma(w[0][j].re, w[0][j].re, fma(w[0][j].im, w[0][j].im, n0));
    double r0 = rsqrt_nr(n0);
    Cx<double> u[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) u[j] = Cx<double>{w[0][j].re * r0, w[0][j].im * r0};
    Cx<double> d{0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 3; ++j) cmac_ca(d, u[j], w[1][j]);
    Cx<double> q[3];
    double n1 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        // q = w1 - d*u
        q[j].re = w[1][j].re - (d.re * u[j].re - d.im * u[j].im);
        q[j].im = w[1][j].im - (d.re * u[j].im + d.im * u[j].re);
        n1 = fma(q[j].re, q[j].re, fma(q[j].im, q[j].im, n1));
    }
    double r1 = rsqrt_nr(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) q[j] = Cx<double>{q[j].re * r1, q[j].im * r1};
    if (!(n0 > 0.0) || !(n1 > 0.0)) {
        const double nan = __builtin_nan("");
#pragma unroll
        for (int j = 0; j < 3; ++j) { u[j] = Cx<double>{nan, nan}; q[j] = u[j]; }
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) { v[0][j] = u[j]; v[1][j] = q[j]; }
    v[2][0] = conj_cross(u[1], q[2], u[2], q[1]);
    v[2][1] = conj_cross(u[2], q[0], u[0], q[2]);
    v[2][2] = conj_cross(u[0], q[1], u[1], q[0]);
}

// ------------------------------------------------------- polar projection
// Bi-covariant projection in FP64: V = W (W^dag W)^(-1/2), the unitary factor
// of the polar decomposition, by the scaled Newton iteration
//   X <- (z X + X^(-dag) / z) / 2,   z = (||X^-1||_F / ||X||_F)^(1/2)
// from X = W, then the phase of det V removed on the principal branch
// (V exp(-i arg(det V) / 3)).  For a 3x3 matrix with rows x0, x1, x2 the
// cofactor matrix has rows x1 x x2, x2 x x0, x0 x x1 (plain cross products)
// and det X = x0 . (x1 x x2), so X^(-dag) = conj(cofactors) / conj(det).
// kPolarIters iterations reach FP64 rounding for the condition numbers that
// APE combinations have (below about 1e3).  A singular W gives NaN.
constexpr int kPolarIters = 9;

__device__ __forceinline__ Cx<double> cmul(const Cx<double> &a, const Cx<double> &b) {
    return Cx<double>{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
// (a x b)_k without conjugation: cyclic a_i b_j - a_j b_i
__device__ __forceinline__ void cross3(const Cx<double> a[3], const Cx<double> b[3], Cx<double> c[3]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = (k + 1) % 3, j = (k + 2) % 3;
        const Cx<double> t1 = cmul(a[i], b[j]), t2 = cmul(a[j], b[i]);
        c[k] = Cx<double>{t1.re - t2.re, t1.im - t2.im};
    }
}

__device__ __forceinline__ void polar_project(Cx<double> x[3][3], Cx<double> v[3][3]) {
#pragma unroll 1
    for (int it = 0; it < kPolarIters; ++it) {
        Cx<double> c[3][3];
        cross3(x[1], x[2], c[0]);
        cross3(x[2], x[0], c[1]);
        cross3(x[0], x[1], c[2]);
        Cx<double> d{0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const Cx<double> t = cmul(x[0][k], c[0][k]);
            d.re += t.re;
            d.im += t.im;
        }
        double nx = 0.0, nc = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                nx = fma(x[i][j].re, x[i][j].re, fma(x[i][j].im, x[i][j].im, nx));
                nc = fma(c[i][j].re, c[i][j].re, fma(c[i][j].im, c[i][j].im, nc));
            }
        const double dd = fma(d.re, d.re, d.im * d.im);  // |det|^2
        // z^4 = ||X^-1||_F^2 / ||X||_F^2 = (nc / dd) / nx
        const double z = sqrt(sqrt(nc / (dd * nx)));
        const double hz = 0.5 * z, hiz = 0.5 / z;
        const double rdd = 1.0 / dd;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                // conj(c_ij) / conj(d) = conj(c_ij conj(d)) / |d|^2
                const Cx<double> cd{fma(c[i][j].re, d.re, c[i][j].im * d.im), fma(c[i][j].im, d.re, -c[i][j].re * d.im)};
                const Cx<double> y{cd.re * rdd, -cd.im * rdd};
                x[i][j] = Cx<double>{fma(hz, x[i][j].re, hiz * y.re), fma(hz, x[i][j].im, hiz * y.im)};
            }
    }
    Cx<double> c0[3];
    cross3(x[1], x[2], c0);
    Cx<double> d{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const Cx<double> t = cmul(x[0][k], c0[k]);
        d.re += t.re;
        d.im += t.im;
    }
    double sn, cs;
    sincos(-atan2(d.im, d.re) / 3.0, &sn, &cs);
    const Cx<double> ph{cs, sn};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) v[i][j] = cmul(x[i][j], ph);
}

// ------------------------------------------------------------- reductions
// Fixed-shape butterfly over the 64 lanes of a wave: every lane ends with the
// same sum and the order of additions never changes.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of `v` over a block of NW waves, deterministic; result valid in thread 0.
template <int NW> __device__ __forceinline__ double block_sum(double v, double *lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NW; ++i) r += lds[i];
    }
    __syncthreads();
    return r;
}

// Physical block -> logical tile so that each of the 8 XCDs (which receive
// blocks round-robin) works on one contiguous range of tiles and its L2
// sees the neighbouring tiles.  A bijection on [0, nb).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

}  // namespace qdpx
