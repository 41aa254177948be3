// Run-time compiled expression kernels (section 5.1 of the paper: a lattice
// expression becomes one kernel, generated from its tree, compiled at run
// time and kept for reuse).  Here the tree is a small S-expression language
// over Dirac fields, the link field and scalars:
//
//   fK                  field argument K
//   (shift E + mu)      E evaluated at x + mu;  (shift E - mu): at x - mu
//   (umul mu E)         U_mu(x) E(x);  (uadj mu E): U_mu(x)^dagger E(x)
//   (add E F) (sub E F) (scale sK E)      sK: scalar argument K
//   (sum MASK E)        sum over the directions in MASK (hex) of E, the
//                       direction variable m standing for each in turn
//
// The generator writes one HIP kernel per expression (one site per lane,
// blocks of 256 sites, in FP32 taken so that each XCD walks one contiguous
// range; each node becomes straight-line code on a 12-component spinor, a shift
// moves the site index and coordinates, a sum becomes a loop over its
// directions that is not unrolled), compiles it with
// hipRTC for the device's architecture with packed FP32 disabled, and keeps
// the code object in an on-disk cache keyed by a hash of the source and
// options, so a later process loads it without compiling (the paper's
// kernel cache, made persistent).  The |out|^2 reduction, when asked for,
// uses the library's fixed-order finalisation.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>
#include <vector>

#include "../../include/qdpx.h"
#include "qdpx_impl.hpp"

namespace qdpx {
int set_error(int code, const char *msg);  // api.cpp
int device_ok(const qdpx_ctx *ctx, const char *fn);  // api.cpp
bool geom_valid(const qdpx_geom *g, const char *fn);
int workspace_reduce_bytes(const qdpx_geom *g);
}  // namespace qdpx

using namespace qdpx;

namespace {

constexpr int kMaxFields = 8;
constexpr int kMaxScalars = 8;

// ------------------------------------------------------------------ parser
struct Node {
    enum Kind { Field, Shift, Umul, Uadj, Add, Sub, Scale, Sum } kind = Field;
    int idx = 0;         // field or scalar index
    int sign = 0;        // shift: +1 / -1
    int dir = 0;         // 0..3, or -1 for the sum's variable m
    unsigned mask = 0;   // sum
    std::vector<std::unique_ptr<Node>> kids;
};

struct Parser {
    std::vector<std::string> tok;
    size_t pos = 0;
    int n_fields, n_scalars;
    std::string err;

    Parser(const char *text, int nf, int ns) : n_fields(nf), n_scalars(ns) {
        std::string cur;
        for (const char *p = text; *p; ++p) {
            const char ch = *p;
            if (ch == '(' || ch == ')' || ch == ' ' || ch == '\t' || ch == '\n' || ch == '\r') {
                if (!cur.empty()) tok.push_back(cur), cur.clear();
                if (ch == '(' || ch == ')') tok.push_back(std::string(1, ch));
            } else {
                cur += ch;
            }
        }
        if (!cur.empty()) tok.push_back(cur);
    }
    bool fail(const std::string &m) {
        if (err.empty()) err = m;
        return false;
    }
    bool next(std::string &t) {
        if (pos >= tok.size()) return fail("unexpected end of expression");
        t = tok[pos++];
        return true;
    }
    bool index(const std::string &t, char lead, int limit, int &out) {
        if (t.size() < 2 || t[0] != lead) return fail("expected " + std::string(1, lead) + "K, got '" + t + "'");
        char *end = nullptr;
        const long v = std::strtol(t.c_str() + 1, &end, 10);
        if (*end || v < 0 || v >= limit) return fail("index out of range in '" + t + "'");
        out = (int)v;
        return true;
    }
    bool direction(const std::string &t, bool in_sum, int &out) {
        if (t == "m") {
            if (!in_sum) return fail("direction variable m outside a sum");
            out = -1;
            return true;
        }
        if (t.size() != 1 || t[0] < '0' || t[0] > '3') return fail("bad direction '" + t + "'");
        out = t[0] - '0';
        return true;
    }
    bool close() {
        std::string t;
        if (!next(t)) return false;
        return t == ")" || fail("expected ')', got '" + t + "'");
    }
    bool expr(std::unique_ptr<Node> &n, bool in_sum) {
        std::string t;
        if (!next(t)) return false;
        n.reset(new Node);
        if (t != "(") {
            n->kind = Node::Field;
            return index(t, 'f', n_fields, n->idx);
        }
        std::string op;
        if (!next(op)) return false;
        if (op == "shift") {
            n->kind = Node::Shift;
            n->kids.resize(1);
            if (!expr(n->kids[0], in_sum)) return false;
            std::string s, d;
            if (!next(s) || !next(d)) return false;
            if (s != "+" && s != "-") return fail("shift sign must be + or -");
            n->sign = (s == "+") ? 1 : -1;
            return direction(d, in_sum, n->dir) && close();
        }
        if (op == "umul" || op == "uadj") {
            n->kind = (op == "umul") ? Node::Umul : Node::Uadj;
            std::string d;
            if (!next(d) || !direction(d, in_sum, n->dir)) return false;
            n->kids.resize(1);
            return expr(n->kids[0], in_sum) && close();
        }
        if (op == "add" || op == "sub") {
            n->kind = (op == "add") ? Node::Add : Node::Sub;
            n->kids.resize(2);
            return expr(n->kids[0], in_sum) && expr(n->kids[1], in_sum) && close();
        }
        if (op == "scale") {
            n->kind = Node::Scale;
            std::string s;
            if (!next(s) || !index(s, 's', n_scalars, n->idx)) return false;
            n->kids.resize(1);
            return expr(n->kids[0], in_sum) && close();
        }
        if (op == "sum") {
            if (in_sum) return fail("nested sums are not supported");
            n->kind = Node::Sum;
            std::string m;
            if (!next(m)) return false;
            char *end = nullptr;
            const unsigned long v = std::strtoul(m.c_str(), &end, 16);
            if (*end || v == 0 || v > 0xF) return fail("sum mask must be a hex value in [0x1, 0xF]");
            n->mask = (unsigned)v;
            n->kids.resize(1);
            return expr(n->kids[0], true) && close();
        }
        return fail("unknown operation '" + op + "'");
    }
};

// --------------------------------------------------------------- generator
struct Gen {
    std::ostringstream body;
    int next_id = 0;

    std::string fresh(const char *p) { return std::string(p) + std::to_string(next_id++); }

    // Emits code for n evaluated at site `s` with coordinates c[0..3].  A
    // direction of -1 is the sum's loop variable m (a run-time value: sums
    // become loops that are not unrolled, so one direction's operands are
    // live at a time).  Returns the name of the spinor variable.
    std::string emit(const Node &n, const std::string &s, const std::string c[4]) {
        const bool var = (n.dir < 0);
        const std::string D = var ? std::string("m") : std::to_string(n.dir);
        switch (n.kind) {
        case Node::Field: {
            const std::string v = fresh("v");
            body << "    spinor " << v << "; ldspinor(f" << n.idx << ", S, " << s << ", " << v << ");\n";
            return v;
        }
        case Node::Shift: {
            const std::string t = fresh("s"), moved = fresh("c");
            const std::string L = var ? "lsel(m, L0, L1, L2, L3)" : "L" + D;
            const std::string st = var ? "lsel(m, st0, st1, st2, st3)" : "st" + D;
            const std::string cur = var ? "lsel(m, " + c[0] + ", " + c[1] + ", " + c[2] + ", " + c[3] + ")" : c[n.dir];
            body << "    int " << t << " = " << s << ", " << moved << " = " << cur << ";\n";
            if (n.sign > 0)
                body << "    if (" << moved << " == " << L << " - 1) { " << moved << " = 0; " << t << " -= (" << L
                     << " - 1) * " << st << "; } else { ++" << moved << "; " << t << " += " << st << "; }\n";
            else
                body << "    if (" << moved << " == 0) { " << moved << " = " << L << " - 1; " << t << " += (" << L
                     << " - 1) * " << st << "; } else { --" << moved << "; " << t << " -= " << st << "; }\n";
            std::string cc[4];
            for (int d = 0; d < 4; ++d) {
                if (!var) {
                    cc[d] = (d == n.dir) ? moved : c[d];
                } else {
                    cc[d] = fresh("c");
                    body << "    const int " << cc[d] << " = (m == " << d << ") ? " << moved << " : " << c[d] << ";\n";
                }
            }
            return emit(*n.kids[0], t, cc);
        }
        case Node::Umul:
        case Node::Uadj: {
            const std::string a = emit(*n.kids[0], s, c);
            const std::string u = fresh("u"), v = fresh("v");
            body << "    link " << u << "; ldlink(U, S, " << D << ", " << s << ", " << u << ");\n";
            body << "    spinor " << v << "; " << (n.kind == Node::Umul ? "umul" : "uadj") << "(" << u << ", " << a
                 << ", " << v << ");\n";
            return v;
        }
        case Node::Add:
        case Node::Sub: {
            const std::string a = emit(*n.kids[0], s, c), b = emit(*n.kids[1], s, c);
            const std::string v = fresh("v");
            body << "    spinor " << v << "; " << (n.kind == Node::Add ? "sadd" : "ssub") << "(" << a << ", " << b
                 << ", " << v << ");\n";
            return v;
        }
        case Node::Scale: {
            const std::string a = emit(*n.kids[0], s, c), v = fresh("v");
            body << "    spinor " << v << "; sscale(scal" << n.idx << ", " << a << ", " << v << ");\n";
            return v;
        }
        case Node::Sum: {
            const std::string v = fresh("v");
            body << "    spinor " << v << "; szero(" << v << ");\n";
            // Two directions per trip keep two sets of neighbour loads in
            // flight; a full unroll needs every register (occupancy 1).
            body << "#pragma unroll 2\n    for (int m = 0; m < 4; ++m) {\n";
            body << "    if (!((" << n.mask << "u >> m) & 1u)) continue;\n";
            const std::string a = emit(*n.kids[0], s, c);
            body << "    sadd(" << v << ", " << a << ", " << v << ");\n    }\n";
            return v;
        }
        }
        return "";
    }
};

// hipRTC provides the device built-ins itself; the source includes no
// header, so it does not depend on where the HIP headers are installed.
const char *kPrelude = R"HIP(
typedef REAL real;
typedef real real2 __attribute__((ext_vector_type(2)));
struct cx { real re, im; };
struct spinor { cx c[4][3]; };
struct link { cx e[3][3]; };
// the value for direction m of four per-direction values (m run-time, wave-uniform)
__device__ __forceinline__ int lsel(int m, int a, int b, int c, int d) { return m == 0 ? a : m == 1 ? b : m == 2 ? c : d; }
typedef real real4 __attribute__((ext_vector_type(4)));
// element (component comp, site s) of a structure-of-arrays array set with stride S
__device__ __forceinline__ cx ldc(const real2 *__restrict__ p, long long S, int comp, int s) {
    const real2 v = p[(long long)comp * S + s];
    return cx{v.x, v.y};
}
// Dirac fields: component q = 3 spin + colour.  Double: array q of S
// entries.  Float (PAIRED): components 2k and 2k+1 share the 16-byte entry s
// of array k, so a spinor is six 16-byte loads.
__device__ __forceinline__ void ldspinor(const real2 *__restrict__ f, long long S, int s, spinor &r) {
#if PAIRED
    const real4 *P = (const real4 *)f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const real4 v = P[(long long)k * S + s];
        r.c[(2 * k) / 3][(2 * k) % 3] = cx{v.x, v.y};
        r.c[(2 * k + 1) / 3][(2 * k + 1) % 3] = cx{v.z, v.w};
    }
#else
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) r.c[sp][a] = ldc(f, S, sp * 3 + a, s);
#endif
}
__device__ __forceinline__ void stspinor(real2 *__restrict__ f, long long S, int s, const spinor &r) {
#if PAIRED
    real4 *P = (real4 *)f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cx a = r.c[(2 * k) / 3][(2 * k) % 3], b = r.c[(2 * k + 1) / 3][(2 * k + 1) % 3];
        P[(long long)k * S + s] = real4{a.re, a.im, b.re, b.im};
    }
#else
#pragma unroll
    for (int q = 0; q < 12; ++q) f[(long long)q * S + s] = real2{r.c[q / 3][q % 3].re, r.c[q / 3][q % 3].im};
#endif
}
// Link (mu, s): direction mu holds 3*NROWS*S complex slots from slot
// mu*3*NROWS*S on.  Double: one array of S entries per stored element c = 3a+b.
// Float (PAIRED): elements 2k, 2k+1 share the 16-byte entry s of array k;
// the ninth element of a three-row link has an array of its own after the
// four pair arrays.  With NROWS = 2, and for double links (whose stored row 2
// is that row to rounding for SU(3) links; rows 0 and 1 read, as the
// hand-written FP64 kernels read them), the third row is conj(row0 x row1).
__device__ __forceinline__ void ldlink(const real2 *__restrict__ U, long long S, int mu, int s, link &u) {
    const real2 *d = U + (long long)mu * 3 * NROWS * S;
#if PAIRED
    const real4 *P = (const real4 *)d;
#pragma unroll
    for (int k = 0; k < (3 * NROWS) / 2; ++k) {
        const real4 v = P[(long long)k * S + s];
        u.e[(2 * k) / 3][(2 * k) % 3] = cx{v.x, v.y};
        u.e[(2 * k + 1) / 3][(2 * k + 1) % 3] = cx{v.z, v.w};
    }
    if (NROWS == 3) u.e[2][2] = ldc(d + 8 * S, 0, 0, s);
#else
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) u.e[a][b] = ldc(d, S, a * 3 + b, s);
#endif
    if (NROWS == 2 || !PAIRED) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int i = (b + 1) % 3, j = (b + 2) % 3;
            const cx p = u.e[0][i], q = u.e[1][j], r = u.e[0][j], t = u.e[1][i];
            // conj(p q - r t)
            u.e[2][b].re = (p.re * q.re - p.im * q.im) - (r.re * t.re - r.im * t.im);
            u.e[2][b].im = -((p.re * q.im + p.im * q.re) - (r.re * t.im + r.im * t.re));
        }
    }
}
__device__ __forceinline__ void umul(const link &u, const spinor &a, spinor &r) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cx z{(real)0, (real)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                z.re = fma(u.e[i][k].re, a.c[sp][k].re, z.re);
                z.re = fma(-u.e[i][k].im, a.c[sp][k].im, z.re);
                z.im = fma(u.e[i][k].re, a.c[sp][k].im, z.im);
                z.im = fma(u.e[i][k].im, a.c[sp][k].re, z.im);
            }
            r.c[sp][i] = z;
        }
}
__device__ __forceinline__ void uadj(const link &u, const spinor &a, spinor &r) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            cx z{(real)0, (real)0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {  // conj(u_ki) a_k
                z.re = fma(u.e[k][i].re, a.c[sp][k].re, z.re);
                z.re = fma(u.e[k][i].im, a.c[sp][k].im, z.re);
                z.im = fma(u.e[k][i].re, a.c[sp][k].im, z.im);
                z.im = fma(-u.e[k][i].im, a.c[sp][k].re, z.im);
            }
            r.c[sp][i] = z;
        }
}
__device__ __forceinline__ void szero(spinor &r) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) r.c[sp][i] = cx{(real)0, (real)0};
}
__device__ __forceinline__ void sadd(const spinor &a, const spinor &b, spinor &r) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) r.c[sp][i] = cx{a.c[sp][i].re + b.c[sp][i].re, a.c[sp][i].im + b.c[sp][i].im};
}
__device__ __forceinline__ void ssub(const spinor &a, const spinor &b, spinor &r) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) r.c[sp][i] = cx{a.c[sp][i].re - b.c[sp][i].re, a.c[sp][i].im - b.c[sp][i].im};
}
__device__ __forceinline__ void sscale(real k, const spinor &a, spinor &r) {
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int i = 0; i < 3; ++i) r.c[sp][i] = cx{k * a.c[sp][i].re, k * a.c[sp][i].im};
}
)HIP";

std::string generate(const Node &root, int prec, int nrows, int n_fields, int n_scalars) {
    std::ostringstream src;
    std::string pre = kPrelude;
    const std::string real = prec == QDPX_F64 ? "double" : "float";
    src << "#define REAL " << real << "\n#define NROWS " << nrows << "\n#define PAIRED " << (prec == QDPX_F32 ? 1 : 0)
        << "\n" << pre;
    src << "extern \"C\" __global__ void __launch_bounds__(256) qdpx_jit_kernel(int L0, int L1, int L2, int L3, "
           "long long S, const real2 *__restrict__ U";
    for (int i = 0; i < n_fields; ++i) src << ", const real2 *__restrict__ f" << i;
    src << ", real2 *__restrict__ out";
    // scalar K is the parameter scalK: generated locals are named by fresh()
    // as one of v, u, s, c followed by a number, so sK would clash with a site
    for (int i = 0; i < n_scalars; ++i) src << ", real scal" << i;
    src << ", double *__restrict__ partials) {\n";
    src << "    const int V = L0 * L1 * L2 * L3;\n"
           "    const int st0 = 1, st1 = L0, st2 = L0 * L1, st3 = L0 * L1 * L2;\n"
           "    (void)st0;\n";
    if (prec == QDPX_F32) {
        // Blocks reach the 8 XCDs round-robin: block b takes tile
        // (b mod 8) q + min(b mod 8, r) + b div 8 (nb = 8q + r blocks), a
        // bijection that gives each XCD one contiguous range of sites, so the
        // z and t neighbours a block reads were mostly fetched into its own
        // XCD's L2 by the blocks before it (the FP32 hop 3 % faster at
        // 32^3x64; the FP64 one, with twice the bytes per site, 12 % slower,
        // so FP64 kernels keep the plain order).
        src << "    const int nblk = (int)gridDim.x, blk = (int)blockIdx.x;\n"
               "    const int xcq = nblk >> 3, xcr = nblk & 7, xcb = blk & 7;\n"
               "    const int site = (xcb * xcq + min(xcb, xcr) + (blk >> 3)) * 256 + (int)threadIdx.x;\n";
    } else {
        src << "    const int site = blockIdx.x * 256 + threadIdx.x;\n";
    }
    src << "    double n2 = 0.0;\n"
           "    if (site < V) {\n"
           "    int r = site;\n"
           "    int x0 = r % L0; r /= L0;\n"
           "    int x1 = r % L1; r /= L1;\n"
           "    int x2 = r % L2;\n"
           "    int x3 = r / L2;\n";
    Gen g;
    const std::string c[4] = {"x0", "x1", "x2", "x3"};
    const std::string res = g.emit(root, "site", c);
    src << g.body.str();
    src << "    stspinor(out, S, site, " << res << ");\n"
        << "#pragma unroll\n    for (int sp = 0; sp < 4; ++sp)\n#pragma unroll\n"
           "        for (int a = 0; a < 3; ++a) {\n"
           "            const cx z = "
        << res
        << ".c[sp][a];\n"
           "            n2 = fma((double)z.re, (double)z.re, fma((double)z.im, (double)z.im, n2));\n"
           "        }\n"
           "    }\n"
           // a wave whose first site is past the end has no partial (there
           // are ceil(V / 64))
           "    if (partials) {  // |out|^2 of each 64-site group, fixed butterfly\n"
           "#pragma unroll\n"
           "        for (int off = 32; off >= 1; off >>= 1) n2 += __shfl_xor(n2, off, 64);\n"
           "        if ((threadIdx.x & 63) == 0 && site < V) partials[site >> 6] = n2;\n"
           "    }\n"
           "}\n";
    return src.str();
}

// ------------------------------------------------------------------- cache
uint64_t fnv1a(const std::string &s, uint64_t h = 1469598103934665603ull) {
    for (unsigned char ch : s) {
        h ^= ch;
        h *= 1099511628211ull;
    }
    return h;
}

// Directory of the on-disk cache: $QDPX_JIT_CACHE, else $HOME/.cache/qdpx-jit;
// "" (no disk cache) if neither is set.
std::string cache_dir() {
    if (const char *d = std::getenv("QDPX_JIT_CACHE")) return d;
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/qdpx-jit";
    return "";
}

// A file or directory the cache may trust: owned by this user, not a
// symbolic link, and writable by nobody else.
bool private_entry(const struct stat &st) {
    return st.st_uid == geteuid() && (st.st_mode & (S_IWGRP | S_IWOTH)) == 0;
}

// Creates the cache directory (and missing parents) private to this user and
// checks that it is a directory only this user can write; false: do not use
// the disk cache.
bool private_dir(const std::string &path) {
    std::string cur;
    for (size_t i = 0; i < path.size(); ++i) {
        cur += path[i];
        if (path[i] == '/' && cur.size() > 1) mkdir(cur.c_str(), 0700);
    }
    mkdir(path.c_str(), 0700);
    struct stat st;
    return lstat(path.c_str(), &st) == 0 && S_ISDIR(st.st_mode) && private_entry(st);
}

// A cache entry is a header line, the generator's key text (source, options
// and architecture) and the code object.  It is used only if it is a private
// regular file whose stored key equals this kernel's key exactly, so neither
// a hash collision nor a file left by someone else is ever loaded.
const char kEntryMagic[] = "qdpx-jit-entry 1\n";

bool read_entry(const std::string &p, const std::string &key, std::vector<char> &code) {
    const int fd = open(p.c_str(), O_RDONLY | O_NOFOLLOW | O_CLOEXEC);
    if (fd < 0) return false;
    struct stat st;
    std::vector<char> all;
    bool ok = fstat(fd, &st) == 0 && S_ISREG(st.st_mode) && private_entry(st) && st.st_size > 0 &&
              st.st_size < (1 << 28);
    if (ok) {
        all.resize((size_t)st.st_size);
        size_t got = 0;
        while (got < all.size()) {
            const ssize_t n = read(fd, all.data() + got, all.size() - got);
            if (n <= 0) break;
            got += (size_t)n;
        }
        ok = got == all.size();
    }
    close(fd);
    const size_t hm = sizeof kEntryMagic - 1;
    if (!ok || all.size() < hm + 20 + key.size() || std::memcmp(all.data(), kEntryMagic, hm) != 0) return false;
    char lenbuf[21];
    std::memcpy(lenbuf, all.data() + hm, 20);
    lenbuf[20] = '\0';
    const unsigned long long klen = std::strtoull(lenbuf, nullptr, 10);
    if (klen != key.size() || std::memcmp(all.data() + hm + 20, key.data(), key.size()) != 0) return false;
    const size_t off = hm + 20 + key.size();
    if (off >= all.size()) return false;
    code.assign(all.begin() + (std::ptrdiff_t)off, all.end());
    return true;
}

void write_entry_atomic(const std::string &p, const std::string &key, const std::vector<char> &code) {
    const std::string tmp = p + ".tmp" + std::to_string((long)getpid());
    const int fd = open(tmp.c_str(), O_WRONLY | O_CREAT | O_EXCL | O_NOFOLLOW | O_CLOEXEC, 0600);
    if (fd < 0) return;  // the cache is an optimisation: a failed write only costs a later recompile
    char lenbuf[21];
    std::snprintf(lenbuf, sizeof lenbuf, "%019zu\n", key.size());
    std::string head = std::string(kEntryMagic) + lenbuf + key;
    bool ok = true;
    for (const auto &part : {std::make_pair((const char *)head.data(), head.size()),
                             std::make_pair((const char *)code.data(), code.size())}) {
        size_t put = 0;
        while (ok && put < part.second) {
            const ssize_t n = write(fd, part.first + put, part.second - put);
            if (n <= 0) ok = false;
            else put += (size_t)n;
        }
    }
    ok = (close(fd) == 0) && ok;
    if (ok) std::rename(tmp.c_str(), p.c_str());
    else std::remove(tmp.c_str());
}

struct JitKernel {
    std::string source;
    hipModule_t module = nullptr;
    hipFunction_t fn = nullptr;
    int prec = 0, nrows = 3, n_fields = 0, n_scalars = 0;
    bool from_cache = false;
};

std::mutex g_mutex;
std::map<const qdpx_ctx *, std::vector<JitKernel>> g_kernels;

const char *kOptions[] = {"-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
constexpr int kNumOptions = sizeof(kOptions) / sizeof(kOptions[0]);

int parse_and_generate(const char *expr, qdpx_prec prec, qdpx_linkfmt fmt, int n_fields, int n_scalars,
                       std::string &source, const char *fn) {
    char msg[512];
    if (!expr) return set_error(QDPX_EINVAL, (std::string(fn) + ": expression is NULL").c_str());
    if ((prec != QDPX_F64 && prec != QDPX_F32) || (fmt != QDPX_LINK18 && fmt != QDPX_LINK12) ||
        (prec == QDPX_F64 && fmt == QDPX_LINK12)) {
        std::snprintf(msg, sizeof msg, "%s: unsupported precision/link format %d/%d", fn, (int)prec, (int)fmt);
        return set_error(QDPX_EUNSUPPORTED, msg);
    }
    if (n_fields < 1 || n_fields > kMaxFields || n_scalars < 0 || n_scalars > kMaxScalars) {
        std::snprintf(msg, sizeof msg, "%s: %d fields / %d scalars outside [1, %d] / [0, %d]", fn, n_fields,
                      n_scalars, kMaxFields, kMaxScalars);
        return set_error(QDPX_EINVAL, msg);
    }
    Parser p(expr, n_fields, n_scalars);
    std::unique_ptr<Node> root;
    if (!p.expr(root, false) || (p.pos != p.tok.size() && !p.fail("trailing tokens after the expression"))) {
        std::snprintf(msg, sizeof msg, "%s: %s", fn, p.err.c_str());
        return set_error(QDPX_EINVAL, msg);
    }
    source = generate(*root, prec, fmt == QDPX_LINK12 ? 2 : 3, n_fields, n_scalars);
    return QDPX_OK;
}

}  // namespace

namespace qdpx {
void jit_release(const qdpx_ctx *ctx) {
    std::lock_guard<std::mutex> lock(g_mutex);
    auto it = g_kernels.find(ctx);
    if (it == g_kernels.end()) return;
    for (JitKernel &k : it->second)
        if (k.module) (void)hipModuleUnload(k.module);
    g_kernels.erase(it);
}
}  // namespace qdpx

extern "C" int qdpx_jit_generate(const char *expr, qdpx_prec prec, qdpx_linkfmt fmt, int32_t n_fields,
                                 int32_t n_scalars, char *buf, size_t buf_bytes, size_t *needed) {
    std::string src;
    if (int r = parse_and_generate(expr, prec, fmt, n_fields, n_scalars, src, "qdpx_jit_generate")) return r;
    if (needed) *needed = src.size() + 1;
    if (buf && buf_bytes) {
        const size_t n = std::min(buf_bytes - 1, src.size());
        std::memcpy(buf, src.data(), n);
        buf[n] = '\0';
        if (n < src.size()) return set_error(QDPX_ENOMEM, "qdpx_jit_generate: buffer too small");
    }
    return QDPX_OK;
}

extern "C" int qdpx_jit_compile(qdpx_ctx *ctx, const char *expr, qdpx_prec prec, qdpx_linkfmt fmt, int32_t n_fields,
                                int32_t n_scalars, int32_t *kernel) {
    const char *fn = "qdpx_jit_compile";
    if (!ctx || !kernel) return set_error(QDPX_EINVAL, "qdpx_jit_compile: ctx or kernel is NULL");
    if (int r = device_ok(ctx, fn)) return r;
    JitKernel k;
    if (int r = parse_and_generate(expr, prec, fmt, n_fields, n_scalars, k.source, fn)) return r;
    k.prec = prec;
    k.nrows = (fmt == QDPX_LINK12) ? 2 : 3;
    k.n_fields = n_fields;
    k.n_scalars = n_scalars;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return set_error(QDPX_EHIP, "qdpx_jit_compile: no device");
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    const std::string arch_opt = "--offload-arch=" + arch;
    std::string key_text = k.source + "\n" + arch_opt;
    for (int i = 0; i < kNumOptions; ++i) key_text += std::string(" ") + kOptions[i];
    char hex[32];
    std::snprintf(hex, sizeof hex, "%016llx", (unsigned long long)fnv1a(key_text));
    const std::string dir = cache_dir();
    const bool use_disk = !dir.empty() && private_dir(dir);
    const std::string path = dir + "/" + hex + ".co";
    std::vector<char> code;
    if (use_disk) {
        struct stat st;
        const bool present = lstat(path.c_str(), &st) == 0;
        // an entry that is not this kernel's, or no longer loads (a truncated
        // or foreign file), is dropped and rebuilt; a failed load's error is
        // cleared so that the next launch check does not report it
        if (read_entry(path, key_text, code) && hipModuleLoadData(&k.module, code.data()) == hipSuccess) {
            k.from_cache = true;
        } else {
            (void)hipGetLastError();
            if (present) std::remove(path.c_str());
        }
    }
    if (!k.from_cache) {
        hiprtcProgram prog;
        if (hiprtcCreateProgram(&prog, k.source.c_str(), "qdpx_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
            return set_error(QDPX_EHIP, "qdpx_jit_compile: hiprtcCreateProgram failed");
        std::vector<const char *> opts(kOptions, kOptions + kNumOptions);
        opts.push_back(arch_opt.c_str());
        const hiprtcResult cr = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
        if (cr != HIPRTC_SUCCESS) {
            size_t ln = 0;
            hiprtcGetProgramLogSize(prog, &ln);
            std::string log(ln, '\0');
            if (ln) hiprtcGetProgramLog(prog, &log[0]);
            hiprtcDestroyProgram(&prog);
            return set_error(QDPX_EHIP, ("qdpx_jit_compile: hipRTC: " + log.substr(0, 400)).c_str());
        }
        size_t n = 0;
        hiprtcGetCodeSize(prog, &n);
        code.resize(n);
        hiprtcGetCode(prog, code.data());
        hiprtcDestroyProgram(&prog);
        if (use_disk) write_entry_atomic(path, key_text, code);
    }
    hipError_t e = hipSuccess;
    if (!k.from_cache && (e = hipModuleLoadData(&k.module, code.data())) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(QDPX_EHIP, "qdpx_jit_compile: hipModuleLoadData failed");
    }
    e = hipModuleGetFunction(&k.fn, k.module, "qdpx_jit_kernel");
    if (e != hipSuccess) {
        (void)hipGetLastError();
        (void)hipModuleUnload(k.module);
        return set_error(QDPX_EHIP, "qdpx_jit_compile: kernel not found in the code object");
    }
    std::lock_guard<std::mutex> lock(g_mutex);
    std::vector<JitKernel> &v = g_kernels[ctx];
    *kernel = (int32_t)v.size();
    v.push_back(std::move(k));
    return QDPX_OK;
}

extern "C" int qdpx_jit_info(qdpx_ctx *ctx, int32_t kernel, int32_t *from_cache, char *buf, size_t buf_bytes) {
    std::lock_guard<std::mutex> lock(g_mutex);
    auto it = g_kernels.find(ctx);
    if (!ctx || it == g_kernels.end() || kernel < 0 || kernel >= (int32_t)it->second.size())
        return set_error(QDPX_EINVAL, "qdpx_jit_info: unknown kernel");
    const JitKernel &k = it->second[kernel];
    if (from_cache) *from_cache = k.from_cache ? 1 : 0;
    if (buf && buf_bytes) {
        const size_t n = std::min(buf_bytes - 1, k.source.size());
        std::memcpy(buf, k.source.data(), n);
        buf[n] = '\0';
    }
    return QDPX_OK;
}

extern "C" int qdpx_jit_eval(qdpx_ctx *ctx, int32_t kernel, const qdpx_geom *geom, const void *U,
                             const void *const *fields, const double *scalars, void *out, double *norm2, void *work,
                             size_t work_bytes, void *stream) {
    const char *fn = "qdpx_jit_eval";
    if (!ctx) return set_error(QDPX_EINVAL, "qdpx_jit_eval: ctx is NULL");
    if (int r = device_ok(ctx, fn)) return r;
    if (!geom_valid(geom, fn)) return QDPX_EINVAL;
    JitKernel k;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        auto it = g_kernels.find(ctx);
        if (it == g_kernels.end() || kernel < 0 || kernel >= (int32_t)it->second.size())
            return set_error(QDPX_EINVAL, "qdpx_jit_eval: unknown kernel");
        const JitKernel &src = it->second[kernel];
        k.fn = src.fn;
        k.prec = src.prec;
        k.nrows = src.nrows;
        k.n_fields = src.n_fields;
        k.n_scalars = src.n_scalars;
    }
    if (!U || !out || !fields) return set_error(QDPX_EINVAL, "qdpx_jit_eval: NULL pointer");
    if ((uintptr_t)U & 15u) return set_error(QDPX_EINVAL, "qdpx_jit_eval: link field not 16-byte aligned");
    const qdpx_linkfmt fmt = k.nrows == 2 ? QDPX_LINK12 : QDPX_LINK18;
    const size_t fb = qdpx_fermion_bytes(geom, (qdpx_prec)k.prec), lb = qdpx_links_bytes(geom, (qdpx_prec)k.prec, fmt);
    auto overlaps = [](const void *a, size_t na, const void *b, size_t nb) {
        const char *x = (const char *)a, *y = (const char *)b;
        return x < y + nb && y < x + na;
    };
    if (overlaps(out, fb, U, lb)) return set_error(QDPX_EALIAS, "qdpx_jit_eval: out overlaps U");
    const uintptr_t elem = 16;  // fields are read 16 bytes at a time (FP32 components in pairs)
    if ((uintptr_t)out % elem) return set_error(QDPX_EINVAL, "qdpx_jit_eval: out not 16-byte aligned");
    if (norm2 && ((uintptr_t)work & 15u)) return set_error(QDPX_EINVAL, "qdpx_jit_eval: workspace not 16-byte aligned");
    for (int i = 0; i < k.n_fields; ++i) {
        if (!fields[i]) return set_error(QDPX_EINVAL, "qdpx_jit_eval: NULL field");
        if ((uintptr_t)fields[i] % elem)
            return set_error(QDPX_EINVAL, "qdpx_jit_eval: field not 16-byte aligned");
        if (overlaps(out, fb, fields[i], fb)) return set_error(QDPX_EALIAS, "qdpx_jit_eval: out overlaps a field");
    }
    if (k.n_scalars && !scalars) return set_error(QDPX_EINVAL, "qdpx_jit_eval: scalars is NULL");
    const size_t need = (size_t)workspace_reduce_bytes(geom);
    if (norm2 && (!work || work_bytes < need)) return set_error(QDPX_ENOMEM, "qdpx_jit_eval: workspace too small");
    const Geo g = make_geo(geom->L);
    long long S = (long long)g.S;
    int L0 = geom->L[0], L1 = geom->L[1], L2 = geom->L[2], L3 = geom->L[3];
    double *partials = norm2 ? (double *)work : nullptr;
    // kernel arguments in declaration order
    std::vector<void *> args;
    const void *fptr[kMaxFields];
    float sf[kMaxScalars];
    double sd[kMaxScalars];
    args.push_back(&L0);
    args.push_back(&L1);
    args.push_back(&L2);
    args.push_back(&L3);
    args.push_back(&S);
    args.push_back(&U);
    for (int i = 0; i < k.n_fields; ++i) {
        fptr[i] = fields[i];
        args.push_back(&fptr[i]);
    }
    args.push_back(&out);
    for (int i = 0; i < k.n_scalars; ++i) {
        sd[i] = scalars[i];
        sf[i] = (float)scalars[i];
        args.push_back(k.prec == QDPX_F64 ? (void *)&sd[i] : (void *)&sf[i]);
    }
    args.push_back(&partials);
    const unsigned grid = (unsigned)((g.V + 255) / 256);
    hipError_t e = hipModuleLaunchKernel(k.fn, grid, 1, 1, 256, 1, 1, 0, (hipStream_t)stream, args.data(), nullptr);
    if (e != hipSuccess) return set_error(QDPX_EHIP, "qdpx_jit_eval: launch failed");
    if (norm2) {
        e = launch_finalize(partials, shift_num_partials(g), 0, (double)g.V, norm2, (hipStream_t)stream);
        if (e != hipSuccess) return set_error(QDPX_EHIP, "qdpx_jit_eval: finalisation failed");
    }
    return QDPX_OK;
}
