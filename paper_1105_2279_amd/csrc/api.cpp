// C ABI of the library: argument validation, workspace layout, launch
// sequencing of the kernels and the launch-geometry tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/qdpx.h"
#include "qdpx_impl.hpp"
#include "su3_device.hpp"

namespace qdpx {
int finalize_stage_a_blocks(int n);
}  // namespace qdpx

using namespace qdpx;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

static int hip_fail(hipError_t e, const char *what) {
    return fail(QDPX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define QDPX_TRY_HIP(expr, what)               \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

extern "C" const char *qdpx_last_error(void) { return g_err.c_str(); }

namespace qdpx {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
void jit_release(const qdpx_ctx *ctx);
int device_ok(const qdpx_ctx *ctx, const char *fn);
}  // namespace qdpx
extern "C" const char *qdpx_version(void) { return "qdpx 0.1 (gfx950)"; }

// ------------------------------------------------------------------ context
struct TuneKey {
    int op, prec, fmt, L[4];
    bool operator<(const TuneKey &o) const {
        return std::tie(op, prec, fmt, L[0], L[1], L[2], L[3]) <
               std::tie(o.op, o.prec, o.fmt, o.L[0], o.L[1], o.L[2], o.L[3]);
    }
};

struct BatchKey {
    std::vector<uint64_t> v;
    bool operator<(const BatchKey &o) const { return v < o.v; }
};

// Where a remembered geometry came from (qdpx_tune_get's source).
enum { kSrcDefault = 0, kSrcTable = 1, kSrcTuned = 2, kSrcSet = 3 };

struct Tuned {
    LaunchCfg cfg;
    int source = kSrcDefault;
};

struct qdpx_ctx {
    int device = 0;
    std::string arch;        // gcnArchName of the device
    std::string cache_path;  // launch-table file ("" = none)
    double *scratch = nullptr;  // this device's copy of `scratch` (no-allocation entry point)
    std::map<TuneKey, Tuned> tuned;
    std::map<BatchKey, void *> batch_tables;  // device tables of batched calls
};

// QDPX_LOG set to anything but "" or "0": one line on stderr per launch-table
// read or write and per tuning decision.
static bool log_on() {
    const char *e = getenv("QDPX_LOG");
    return e && *e && strcmp(e, "0") != 0;
}

static const char *op_name(int op) {
    static const char *const n[] = {"SHIFT", "CHAIN", "APE", "PLAQ", "BATCHED", "JACOBI"};
    return (op >= 0 && op < 6) ? n[op] : "?";
}

static void log_cfg(const char *what, const TuneKey &k, const LaunchCfg &c) {
    if (!log_on()) return;
    fprintf(stderr,
            "qdpx: %s %s prec %d fmt %d L %dx%dx%dx%d: block %d, groups/wave %d, xcd map %d, t window %d, "
            "LDS tile %d\n",
            what, op_name(k.op), k.prec, k.fmt, k.L[0], k.L[1], k.L[2], k.L[3], c.block, c.nsite, c.xcd, c.tw, c.lds);
}

// LDS tile of the FP32 APE step when nothing chose one: the group's own
// links and the plane products staged.  Every other case has no LDS tile
// level.
static const int kDefaultApeLds = 4;
static int default_lds(int op, int prec) { return (op == QDPX_OP_APE && prec == QDPX_F32) ? kDefaultApeLds : 0; }

static bool cfg_valid(qdpx_op op, qdpx_prec prec, const LaunchCfg &c);

// Scratch memory of qdpx_eval_shift_mul_axpy_noalloc: the per-group |chi|^2
// partials and the finalisation's stage-A sums of a lattice of at most
// kNoAllocMaxSites sites (4 MiB).  Each device holds its own copy for the
// life of the process; host code reaches it only through the device address
// hipGetSymbolAddress gives (qdpx_create keeps it in the context), never
// through the array's name.
static const int kNoAllocMaxSites = 1 << 25;
static const int kNoAllocDoubles = (kNoAllocMaxSites / 64) + (kNoAllocMaxSites / 64 + 4095) / 4096;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

extern "C" int qdpx_create(qdpx_ctx **out, int device, const char *tune_cache_path) {
    if (!out) return fail(QDPX_EINVAL, "qdpx_create: out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(QDPX_EINVAL, "qdpx_create: device %d not in [0, %d)", device, n);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, device);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    std::string path;
    if (tune_cache_path) {
        path = tune_cache_path;
    } else {
        const char *env = getenv("QDPX_TUNE_CACHE");
        if (env) path = env;
    }
    std::vector<TuneEntry> entries;
    if (!path.empty()) {
        std::string err;
        const int r = tune_table_read(path.c_str(), prop.gcnArchName, entries, err);
        if (r < 0) return fail(QDPX_EINVAL, "qdpx_create: launch table %s", err.c_str());
        if (log_on())
            fprintf(stderr, "qdpx: launch table %s: %s\n", path.c_str(),
                    r == 1 ? "no such file yet" : r == 2 ? "recorded on another architecture, ignored" : "read");
        for (TuneEntry &t : entries) {
            if (t.cfg.lds < 0) t.cfg.lds = default_lds(t.op, t.prec);  // written before the LDS tile field
            bool extents_ok = true;
            for (int d = 0; d < 4; ++d) extents_ok = extents_ok && t.L[d] >= 2 && t.L[d] <= 4096;
            if (!extents_ok || !cfg_valid((qdpx_op)t.op, (qdpx_prec)t.prec, t.cfg) || t.L[3] % t.cfg.tw != 0)
                return fail(QDPX_EINVAL, "qdpx_create: launch table %s holds an invalid geometry for op %s",
                            path.c_str(), op_name(t.op));
        }
    }
    // this device's address of the scratch array, looked up with the device current
    int prev = 0;
    e = hipGetDevice(&prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    void *sp = nullptr;
    e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    const hipError_t e2 = hipSetDevice(prev);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (e2 != hipSuccess) return hip_fail(e2, "hipSetDevice");
    if (!sp) return fail(QDPX_EHIP, "qdpx_create: no device address for the scratch array");
    qdpx_ctx *c = new qdpx_ctx;
    c->device = device;
    c->arch = prop.gcnArchName;
    c->cache_path = path;
    c->scratch = (double *)sp;
    for (const TuneEntry &t : entries) {
        const TuneKey k{t.op, t.prec, t.fmt, {t.L[0], t.L[1], t.L[2], t.L[3]}};
        c->tuned[k] = Tuned{t.cfg, kSrcTable};
        log_cfg("table", k, t.cfg);
    }
    *out = c;
    return QDPX_OK;
}

// Merge the context's table and tuned geometries into the file at `path`
// (entries already in the file for other shapes are kept).
static int save_table(qdpx_ctx *ctx, const std::string &path, const char *fn) {
    std::vector<TuneEntry> merged;
    std::string err;
    const int r = tune_table_read(path.c_str(), ctx->arch.c_str(), merged, err);
    if (r < 0) return fail(QDPX_EINVAL, "%s: launch table %s", fn, err.c_str());
    std::map<TuneKey, LaunchCfg> all;
    for (const TuneEntry &t : merged) all[TuneKey{t.op, t.prec, t.fmt, {t.L[0], t.L[1], t.L[2], t.L[3]}}] = t.cfg;
    for (const auto &kv : ctx->tuned)
        if (kv.second.source != kSrcDefault) all[kv.first] = kv.second.cfg;
    std::vector<TuneEntry> rows;
    for (const auto &kv : all) {
        TuneEntry t;
        t.op = kv.first.op;
        t.prec = kv.first.prec;
        t.fmt = kv.first.fmt;
        for (int d = 0; d < 4; ++d) t.L[d] = kv.first.L[d];
        t.cfg = kv.second;
        rows.push_back(t);
    }
    if (tune_table_write(path.c_str(), ctx->arch.c_str(), rows, err) != 0)
        return fail(QDPX_EINVAL, "%s: %s", fn, err.c_str());
    if (log_on()) fprintf(stderr, "qdpx: launch table %s: wrote %zu entries\n", path.c_str(), rows.size());
    return QDPX_OK;
}

extern "C" int qdpx_tune_save(qdpx_ctx *ctx, const char *path) {
    const char *fn = "qdpx_tune_save";
    if (!ctx) return fail(QDPX_EINVAL, "%s: ctx is NULL", fn);
    const std::string p = path ? std::string(path) : ctx->cache_path;
    if (p.empty()) return fail(QDPX_EINVAL, "%s: no path and the context has no launch table", fn);
    return save_table(ctx, p, fn);
}

// Kernels go to the caller's stream on the current device, and the
// context's launch tables and cached device tables belong to its own device:
// a call made while another device is current is refused.
int qdpx::device_ok(const qdpx_ctx *ctx, const char *fn) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, fn);
    if (cur != ctx->device)
        return fail(QDPX_EINVAL, "%s: current device %d is not the context's device %d", fn, cur, ctx->device);
    return QDPX_OK;
}

extern "C" int qdpx_destroy(qdpx_ctx *ctx) {
    if (ctx) qdpx_free_all(ctx);
    delete ctx;
    return QDPX_OK;
}

static void batch_cache_free(qdpx_ctx *ctx);

extern "C" int qdpx_free_all(qdpx_ctx *ctx) {
    if (!ctx) return fail(QDPX_EINVAL, "qdpx_free_all: ctx is NULL");
    batch_cache_free(ctx);
    jit_release(ctx);
    return QDPX_OK;
}

// --------------------------------------------------------------- validation
static bool geom_ok(const qdpx_geom *g, const char *fn) {
    if (!g) {
        fail(QDPX_EINVAL, "%s: geom is NULL", fn);
        return false;
    }
    int64_t v = 1;
    for (int d = 0; d < 4; ++d) {
        if (g->L[d] < 2 || g->L[d] > 4096) {
            fail(QDPX_EINVAL, "%s: extent L[%d] = %d outside [2, 4096]", fn, d, g->L[d]);
            return false;
        }
        v *= g->L[d];
    }
    if (v >= (1LL << 28)) {  // keeps every per-component byte offset within 32 bits
        fail(QDPX_EINVAL, "%s: volume %lld not below 2^28", fn, (long long)v);
        return false;
    }
    return true;
}

static int check_format(qdpx_prec prec, qdpx_linkfmt fmt, const char *fn) {
    if (prec != QDPX_F64 && prec != QDPX_F32) return fail(QDPX_EINVAL, "%s: unknown precision %d", fn, (int)prec);
    if (fmt != QDPX_LINK18 && fmt != QDPX_LINK12) return fail(QDPX_EINVAL, "%s: unknown link format %d", fn, (int)fmt);
    if (prec == QDPX_F64 && fmt == QDPX_LINK12)
        return fail(QDPX_EUNSUPPORTED, "%s: LINK12 is provided with QDPX_F32 only", fn);
    return QDPX_OK;
}

static int nrows_of(qdpx_linkfmt f) { return f == QDPX_LINK12 ? 2 : 3; }
static size_t cplx_bytes(qdpx_prec p) { return p == QDPX_F64 ? 16 : 8; }

static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    if (!a || !b || !na || !nb) return false;
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + nb && pb < pa + na;
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Link and Dirac fields are read with 16-byte accesses (FP32 Dirac-field
// components in pairs); workspaces that hold fields are 16-byte aligned.
static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
static bool field_aligned(const void *p, qdpx_prec) { return aligned16(p); }

extern "C" int64_t qdpx_site_stride(const qdpx_geom *geom) {
    if (!geom_ok(geom, "qdpx_site_stride")) return -1;
    return make_geo(geom->L).S;
}

extern "C" size_t qdpx_links_bytes(const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt) {
    if (!geom_ok(geom, "qdpx_links_bytes") || check_format(prec, fmt, "qdpx_links_bytes") != QDPX_OK) return 0;
    const Geo g = make_geo(geom->L);
    return (size_t)g.S * 4 * nrows_of(fmt) * 3 * cplx_bytes(prec);
}

extern "C" size_t qdpx_fermion_bytes(const qdpx_geom *geom, qdpx_prec prec) {
    if (!geom_ok(geom, "qdpx_fermion_bytes") || check_format(prec, QDPX_LINK18, "qdpx_fermion_bytes") != QDPX_OK)
        return 0;
    const Geo g = make_geo(geom->L);
    return (size_t)g.S * 12 * cplx_bytes(prec);
}

// doubles needed to reduce n partials of ncomp components (partials + stage A)
static size_t reduce_bytes(int n, int ncomp) {
    return round256(sizeof(double) * (size_t)ncomp * ((size_t)n + (size_t)finalize_stage_a_blocks(n)));
}

namespace qdpx {
bool geom_valid(const qdpx_geom *g, const char *fn) { return geom_ok(g, fn); }
int workspace_reduce_bytes(const qdpx_geom *g) { return (int)reduce_bytes(shift_num_partials(make_geo(g->L)), 1); }
}  // namespace qdpx

// Batched tables are defined further below.
static size_t batched_ws_bytes(int n_lat, const qdpx_geom *geoms, qdpx_prec prec, qdpx_linkfmt fmt, int n_steps);

extern "C" size_t qdpx_workspace_bytes(qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt, int n) {
    if (op == QDPX_OP_BATCHED) return batched_ws_bytes(n, geom, prec, fmt, 1 << 20);
    if (!geom_ok(geom, "qdpx_workspace_bytes") || check_format(prec, fmt, "qdpx_workspace_bytes") != QDPX_OK) return 0;
    const Geo g = make_geo(geom->L);
    switch (op) {
    case QDPX_OP_SHIFT:
        return reduce_bytes(shift_num_partials(g), 1);
    case QDPX_OP_CHAIN:
        return round256(qdpx_fermion_bytes(geom, prec)) + reduce_bytes(shift_num_partials(g), 1);
    case QDPX_OP_APE:
        return (n >= 2 ? round256(qdpx_links_bytes(geom, prec, fmt)) : 0) +
               reduce_bytes(std::max(ape_num_partials(g), plaquette_num_partials(g)), 2);
    case QDPX_OP_PLAQ:
        return reduce_bytes(plaquette_num_partials(g), 2);
    case QDPX_OP_JACOBI:
        return 2 * round256(qdpx_fermion_bytes(geom, prec));
    default:
        fail(QDPX_EINVAL, "qdpx_workspace_bytes: unknown op %d", (int)op);
        return 0;
    }
}

static bool stream_capturing(hipStream_t st) {
    hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &s) != hipSuccess) return false;
    return s == hipStreamCaptureStatusActive;
}

static LaunchCfg cfg_for(qdpx_ctx *ctx, qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt) {
    LaunchCfg c;
    if (op == QDPX_OP_BATCHED) c.nsite = 1;  // groups per ticket
    c.lds = default_lds(op, prec);
    if (ctx) {
        TuneKey k{(int)op, (int)prec, (int)fmt, {geom->L[0], geom->L[1], geom->L[2], geom->L[3]}};
        auto it = ctx->tuned.find(k);
        if (it != ctx->tuned.end()) c = it->second.cfg;
    }
    return c;
}

#define QDPX_CHECK_CTX(fn)                                         \
    do {                                                           \
        if (!ctx) return fail(QDPX_EINVAL, "%s: ctx is NULL", fn); \
        if (int r_ = qdpx::device_ok(ctx, fn)) return r_;          \
    } while (0)

// ------------------------------------------------------------ pack / unpack
extern "C" int qdpx_pack_links(qdpx_ctx *ctx, const qdpx_geom *geom, const double *aos, qdpx_prec prec,
                               qdpx_linkfmt fmt, void *soa, void *stream) {
    const char *fn = "qdpx_pack_links";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!aos || !soa) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!aligned16(soa)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    const Geo g = make_geo(geom->L);
    if (overlap(aos, (size_t)g.V * 4 * 18 * 8, soa, qdpx_links_bytes(geom, prec, fmt)))
        return fail(QDPX_EALIAS, "%s: soa overlaps aos", fn);
    QDPX_TRY_HIP(launch_pack_links(g, prec, nrows_of(fmt), aos, soa, (hipStream_t)stream), fn);
    return QDPX_OK;
}

extern "C" int qdpx_unpack_links(qdpx_ctx *ctx, const qdpx_geom *geom, const void *soa, qdpx_prec prec,
                                 qdpx_linkfmt fmt, double *aos, void *stream) {
    const char *fn = "qdpx_unpack_links";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!aos || !soa) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!aligned16(soa)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    const Geo g = make_geo(geom->L);
    if (overlap(aos, (size_t)g.V * 4 * 18 * 8, soa, qdpx_links_bytes(geom, prec, fmt)))
        return fail(QDPX_EALIAS, "%s: aos overlaps soa", fn);
    QDPX_TRY_HIP(launch_unpack_links(g, prec, nrows_of(fmt), soa, aos, (hipStream_t)stream), fn);
    return QDPX_OK;
}

extern "C" int qdpx_pack_fermion(qdpx_ctx *ctx, const qdpx_geom *geom, const double *aos, qdpx_prec prec,
                                 void *soa, void *stream) {
    const char *fn = "qdpx_pack_fermion";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, QDPX_LINK18, fn)) return r;
    if (!aos || !soa) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!field_aligned(soa, prec)) return fail(QDPX_EINVAL, "%s: field not 16-byte aligned", fn);
    const Geo g = make_geo(geom->L);
    if (overlap(aos, (size_t)g.V * 24 * 8, soa, qdpx_fermion_bytes(geom, prec)))
        return fail(QDPX_EALIAS, "%s: soa overlaps aos", fn);
    QDPX_TRY_HIP(launch_pack_fermion(g, prec, aos, soa, (hipStream_t)stream), fn);
    return QDPX_OK;
}

extern "C" int qdpx_unpack_fermion(qdpx_ctx *ctx, const qdpx_geom *geom, const void *soa, qdpx_prec prec,
                                   double *aos, void *stream) {
    const char *fn = "qdpx_unpack_fermion";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, QDPX_LINK18, fn)) return r;
    if (!aos || !soa) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!field_aligned(soa, prec)) return fail(QDPX_EINVAL, "%s: field not 16-byte aligned", fn);
    const Geo g = make_geo(geom->L);
    if (overlap(aos, (size_t)g.V * 24 * 8, soa, qdpx_fermion_bytes(geom, prec)))
        return fail(QDPX_EALIAS, "%s: aos overlaps soa", fn);
    QDPX_TRY_HIP(launch_unpack_fermion(g, prec, soa, aos, (hipStream_t)stream), fn);
    return QDPX_OK;
}

// ------------------------------------------------------------ shift / chain
extern "C" int qdpx_eval_shift_mul_axpy(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                                        const void *U, const void *psi, const void *phi, double a,
                                        uint32_t dir_mask, int sign, void *chi, double *norm2, void *work,
                                        size_t work_bytes, void *stream) {
    const char *fn = "qdpx_eval_shift_mul_axpy";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (dir_mask & ~0xFu) return fail(QDPX_EINVAL, "%s: dir_mask 0x%x has bits beyond the 4 directions", fn, dir_mask);
    if (sign != 1 && sign != -1) return fail(QDPX_EINVAL, "%s: sign %d is neither +1 nor -1", fn, sign);
    if (!U || !psi || !chi) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!aligned16(U)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    if (!field_aligned(psi, prec) || !field_aligned(phi, prec) || !field_aligned(chi, prec))
        return fail(QDPX_EINVAL, "%s: field not 16-byte aligned", fn);
    if (norm2 && !aligned16(work)) return fail(QDPX_EINVAL, "%s: workspace not 16-byte aligned", fn);
    const size_t need = qdpx_workspace_bytes(QDPX_OP_SHIFT, geom, prec, fmt, 0);
    if (norm2 && (!work || work_bytes < need))
        return fail(QDPX_ENOMEM, "%s: workspace of %zu bytes < %zu", fn, work_bytes, need);
    const size_t fb = qdpx_fermion_bytes(geom, prec), lb = qdpx_links_bytes(geom, prec, fmt);
    if (overlap(chi, fb, psi, fb) || overlap(chi, fb, phi, fb) || overlap(chi, fb, U, lb))
        return fail(QDPX_EALIAS, "%s: chi overlaps an input", fn);
    if (norm2 && (overlap(work, need, chi, fb) || overlap(work, need, psi, fb) || overlap(work, need, phi, fb) ||
                  overlap(work, need, U, lb)))
        return fail(QDPX_EALIAS, "%s: workspace overlaps a field", fn);
    const Geo g = make_geo(geom->L);
    const LaunchCfg cfg = cfg_for(ctx, QDPX_OP_SHIFT, geom, prec, fmt);
    hipStream_t st = (hipStream_t)stream;
    double *part = norm2 ? (double *)work : nullptr;
    QDPX_TRY_HIP(launch_shift(g, prec, nrows_of(fmt), U, psi, phi, a, 0, 0.0, chi, part, cfg, st, dir_mask,
                              sign < 0 ? 1 : 0),
                 fn);
    if (norm2) QDPX_TRY_HIP(launch_finalize(part, shift_num_partials(g), 0, (double)g.V, norm2, st), fn);
    return QDPX_OK;
}

// The shift expression without a caller workspace: the |chi|^2 partials go
// to this device's scratch array (every partial and stage-A value is
// rewritten by each call, so nothing needs clearing).
extern "C" int qdpx_eval_shift_mul_axpy_noalloc(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec,
                                                qdpx_linkfmt fmt, const void *U, const void *psi, const void *phi,
                                                double a, uint32_t dir_mask, int sign, void *chi, double *norm2,
                                                void *stream) {
    const char *fn = "qdpx_eval_shift_mul_axpy_noalloc";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    const Geo g = make_geo(geom->L);
    if (g.V > kNoAllocMaxSites)
        return fail(QDPX_EINVAL, "%s: %d sites exceed the %d sites its fixed scratch memory holds", fn, g.V,
                    kNoAllocMaxSites);
    if (dir_mask & ~0xFu) return fail(QDPX_EINVAL, "%s: dir_mask 0x%x has bits beyond the 4 directions", fn, dir_mask);
    if (sign != 1 && sign != -1) return fail(QDPX_EINVAL, "%s: sign %d is neither +1 nor -1", fn, sign);
    if (!U || !psi || !chi) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!aligned16(U)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    if (!field_aligned(psi, prec) || !field_aligned(phi, prec) || !field_aligned(chi, prec))
        return fail(QDPX_EINVAL, "%s: field not 16-byte aligned", fn);
    const size_t fb = qdpx_fermion_bytes(geom, prec), lb = qdpx_links_bytes(geom, prec, fmt);
    if (overlap(chi, fb, psi, fb) || overlap(chi, fb, phi, fb) || overlap(chi, fb, U, lb))
        return fail(QDPX_EALIAS, "%s: chi overlaps an input", fn);
    const int np = shift_num_partials(g);
    if ((size_t)np + (size_t)finalize_stage_a_blocks(np) > (size_t)kNoAllocDoubles)
        return fail(QDPX_EINVAL, "%s: scratch memory too small for %d partials", fn, np);
    const LaunchCfg cfg = cfg_for(ctx, QDPX_OP_SHIFT, geom, prec, fmt);
    hipStream_t st = (hipStream_t)stream;
    double *part = norm2 ? ctx->scratch : nullptr;
    QDPX_TRY_HIP(launch_shift(g, prec, nrows_of(fmt), U, psi, phi, a, 0, 0.0, chi, part, cfg, st, dir_mask,
                              sign < 0 ? 1 : 0),
                 fn);
    if (norm2) QDPX_TRY_HIP(launch_finalize(part, np, 0, (double)g.V, norm2, st), fn);
    return QDPX_OK;
}

extern "C" int qdpx_shift_chain(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                                const void *U, void *psi, const void *phi, double a, double c, int n_iter,
                                double *norms, void *work, size_t work_bytes, void *stream) {
    const char *fn = "qdpx_shift_chain";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!U || !psi) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!aligned16(U)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    if (!field_aligned(psi, prec) || !field_aligned(phi, prec))
        return fail(QDPX_EINVAL, "%s: field not 16-byte aligned", fn);
    if (!aligned16(work)) return fail(QDPX_EINVAL, "%s: workspace not 16-byte aligned", fn);
    if (n_iter < 1) return fail(QDPX_EINVAL, "%s: n_iter = %d < 1", fn, n_iter);
    const size_t need = qdpx_workspace_bytes(QDPX_OP_CHAIN, geom, prec, fmt, n_iter);
    if (!work || work_bytes < need) return fail(QDPX_ENOMEM, "%s: workspace of %zu bytes < %zu", fn, work_bytes, need);
    const size_t fb = qdpx_fermion_bytes(geom, prec), lb = qdpx_links_bytes(geom, prec, fmt);
    if (overlap(psi, fb, phi, fb) || overlap(psi, fb, U, lb)) return fail(QDPX_EALIAS, "%s: psi overlaps an input", fn);
    if (overlap(work, need, psi, fb) || overlap(work, need, phi, fb) || overlap(work, need, U, lb))
        return fail(QDPX_EALIAS, "%s: workspace overlaps a field", fn);
    const Geo g = make_geo(geom->L);
    const LaunchCfg cfg = cfg_for(ctx, QDPX_OP_CHAIN, geom, prec, fmt);
    hipStream_t st = (hipStream_t)stream;
    void *tmp = work;
    double *part = (double *)((char *)work + round256(fb));
    void *buf[2] = {psi, tmp};
    for (int k = 0; k < n_iter; ++k) {
        void *src = buf[k & 1], *dst = buf[(k + 1) & 1];
        QDPX_TRY_HIP(launch_shift(g, prec, nrows_of(fmt), U, src, phi, a, 1, c, dst, norms ? part : nullptr, cfg, st),
                     fn);
        if (norms) QDPX_TRY_HIP(launch_finalize(part, shift_num_partials(g), 0, (double)g.V, norms + k, st), fn);
    }
    if (n_iter & 1) QDPX_TRY_HIP(launch_copy_fermion(g, prec, tmp, psi, st), fn);
    return QDPX_OK;
}

// ------------------------------------------------------------------ Jacobi
extern "C" int qdpx_eval_hop(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt, const void *U,
                             const void *psi, void *out, uint32_t dir_mask, void *stream) {
    const char *fn = "qdpx_eval_hop";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!U || !psi || !out) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!aligned16(U)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    if (!field_aligned(psi, prec) || !field_aligned(out, prec))
        return fail(QDPX_EINVAL, "%s: field not 16-byte aligned", fn);
    if (dir_mask & ~0xFu) return fail(QDPX_EINVAL, "%s: dir_mask 0x%x has bits beyond the 4 directions", fn, dir_mask);
    const size_t fb = qdpx_fermion_bytes(geom, prec), lb = qdpx_links_bytes(geom, prec, fmt);
    if (overlap(out, fb, psi, fb) || overlap(out, fb, U, lb)) return fail(QDPX_EALIAS, "%s: out overlaps an input", fn);
    const Geo g = make_geo(geom->L);
    const LaunchCfg cfg = cfg_for(ctx, QDPX_OP_JACOBI, geom, prec, fmt);
    QDPX_TRY_HIP(launch_hop(g, prec, nrows_of(fmt), U, psi, nullptr, 1.0, 1.0, false, dir_mask, out, cfg,
                            (hipStream_t)stream),
                 fn);
    return QDPX_OK;
}

extern "C" int qdpx_jacobi_smear(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt, const void *U,
                                 void *chi, double kappa, int n_iter, double norm, uint32_t dir_mask, void *work,
                                 size_t work_bytes, void *stream) {
    const char *fn = "qdpx_jacobi_smear";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!U || !chi) return fail(QDPX_EINVAL, "%s: NULL field pointer", fn);
    if (!aligned16(U)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    if (!field_aligned(chi, prec)) return fail(QDPX_EINVAL, "%s: field not 16-byte aligned", fn);
    if (!aligned16(work)) return fail(QDPX_EINVAL, "%s: workspace not 16-byte aligned", fn);
    if (n_iter < 1) return fail(QDPX_EINVAL, "%s: n_iter = %d < 1", fn, n_iter);
    if (norm == 0.0) return fail(QDPX_EINVAL, "%s: norm is 0", fn);
    if (dir_mask & ~0xFu) return fail(QDPX_EINVAL, "%s: dir_mask 0x%x has bits beyond the 4 directions", fn, dir_mask);
    const size_t fb = qdpx_fermion_bytes(geom, prec), lb = qdpx_links_bytes(geom, prec, fmt);
    const size_t need = qdpx_workspace_bytes(QDPX_OP_JACOBI, geom, prec, fmt, n_iter);
    if (!work || work_bytes < need) return fail(QDPX_ENOMEM, "%s: workspace of %zu bytes < %zu", fn, work_bytes, need);
    if (overlap(chi, fb, U, lb)) return fail(QDPX_EALIAS, "%s: chi overlaps U", fn);
    if (overlap(work, need, chi, fb) || overlap(work, need, U, lb))
        return fail(QDPX_EALIAS, "%s: workspace overlaps a field", fn);
    const Geo g = make_geo(geom->L);
    const LaunchCfg cfg = cfg_for(ctx, QDPX_OP_JACOBI, geom, prec, fmt);
    hipStream_t st = (hipStream_t)stream;
    void *s0 = work;
    void *tmp = (char *)work + round256(fb);
    // E_0: s0 = chi.  Iteration k reads the previous iterate (s0 for k = 0)
    // and the last one lands in chi.
    QDPX_TRY_HIP(launch_copy_fermion(g, prec, chi, s0, st), fn);
    const void *src = s0;
    for (int k = 0; k < n_iter; ++k) {
        void *dst = (((n_iter - 1 - k) & 1) == 0) ? chi : tmp;
        const bool last = (k == n_iter - 1);
        QDPX_TRY_HIP(launch_hop(g, prec, nrows_of(fmt), U, src, s0, kappa, norm, last, dir_mask, dst, cfg, st), fn);
        src = dst;
    }
    return QDPX_OK;
}

// ---------------------------------------------------------- APE / plaquette
static int plaquette_into(const Geo &g, qdpx_prec prec, qdpx_linkfmt fmt, const void *U, double *plaq,
                          double *part, hipStream_t st, const char *fn) {
    QDPX_TRY_HIP(launch_plaquette(g, prec, nrows_of(fmt), U, part, st), fn);
    QDPX_TRY_HIP(launch_finalize(part, plaquette_num_partials(g), 1, (double)g.V, plaq, st), fn);
    return QDPX_OK;
}

extern "C" int qdpx_plaquette(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt, const void *U,
                              double *plaq, void *work, size_t work_bytes, void *stream) {
    const char *fn = "qdpx_plaquette";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!U || !plaq) return fail(QDPX_EINVAL, "%s: NULL pointer", fn);
    if (!aligned16(U)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    const size_t need = qdpx_workspace_bytes(QDPX_OP_PLAQ, geom, prec, fmt, 0);
    if (!work || work_bytes < need) return fail(QDPX_ENOMEM, "%s: workspace of %zu bytes < %zu", fn, work_bytes, need);
    if (!aligned16(work)) return fail(QDPX_EINVAL, "%s: workspace not 16-byte aligned", fn);
    if (overlap(work, need, U, qdpx_links_bytes(geom, prec, fmt)))
        return fail(QDPX_EALIAS, "%s: workspace overlaps U", fn);
    return plaquette_into(make_geo(geom->L), prec, fmt, U, plaq, (double *)work, (hipStream_t)stream, fn);
}

extern "C" int qdpx_ape_smear(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                              const void *U_in, void *U_out, double alpha, int n_steps, uint32_t smear_mask,
                              qdpx_proj projection, double *plaq, void *work, size_t work_bytes, void *stream) {
    const char *fn = "qdpx_ape_smear";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!U_in || !U_out) return fail(QDPX_EINVAL, "%s: NULL link pointer", fn);
    if (!aligned16(U_in) || !aligned16(U_out)) return fail(QDPX_EINVAL, "%s: link field not 16-byte aligned", fn);
    if (n_steps < 1) return fail(QDPX_EINVAL, "%s: n_steps = %d < 1", fn, n_steps);
    if (smear_mask & ~0xFu)
        return fail(QDPX_EINVAL, "%s: smear_mask 0x%x has bits beyond the 4 directions", fn, smear_mask);
    if (projection != QDPX_PROJ_GRAM_SCHMIDT && projection != QDPX_PROJ_POLAR)
        return fail(QDPX_EINVAL, "%s: projection %d unknown", fn, (int)projection);
    const int polar = (projection == QDPX_PROJ_POLAR);
    const size_t lb = qdpx_links_bytes(geom, prec, fmt);
    const size_t need = qdpx_workspace_bytes(QDPX_OP_APE, geom, prec, fmt, n_steps);
    const bool need_work = (n_steps >= 2) || plaq;
    if (need_work && (!work || work_bytes < need))
        return fail(QDPX_ENOMEM, "%s: workspace of %zu bytes < %zu", fn, work_bytes, need);
    if (need_work && !aligned16(work))  // intermediate links, plaquette partials
        return fail(QDPX_EINVAL, "%s: workspace not 16-byte aligned", fn);
    if (overlap(U_in, lb, U_out, lb)) return fail(QDPX_EALIAS, "%s: U_out overlaps U_in", fn);
    if (need_work && (overlap(work, need, U_in, lb) || overlap(work, need, U_out, lb)))
        return fail(QDPX_EALIAS, "%s: workspace overlaps the links", fn);
    const Geo g = make_geo(geom->L);
    const LaunchCfg cfg = cfg_for(ctx, QDPX_OP_APE, geom, prec, fmt);
    hipStream_t st = (hipStream_t)stream;
    void *tmp = (n_steps >= 2) ? work : nullptr;
    double *part = (double *)((char *)work + (n_steps >= 2 ? round256(lb) : 0));
    // A smeared link mixes in alpha times the mean of its 2 (d - 1) staples,
    // d = number of smeared directions (alpha/6 for all four).
    const int d = __builtin_popcount(smear_mask);
    const double c1 = 1.0 - alpha, c2 = d > 1 ? alpha / (2.0 * (d - 1)) : 0.0;
    // Plaquettes: the standalone plaquette pass (FP64 products of the
    // widened links), so each value is the one qdpx_plaquette gives on those
    // links, on the input and on every step's output; except that FP64 steps
    // with every direction smeared and the Gram-Schmidt projection reduce the
    // plaquette of their own input inside the APE kernel (the same value to
    // the rounding of FP64), so only the last output needs the pass.
    const bool f32 = (prec == QDPX_F32);
    const bool fused = !f32 && (smear_mask == 0xFu) && !polar;
    const void *src = U_in;
    for (int k = 0; k < n_steps; ++k) {
        // the last step always lands in U_out
        void *dst = (((n_steps - 1 - k) & 1) == 0) ? U_out : tmp;
        if (plaq && !fused)
            if (int r = plaquette_into(g, prec, fmt, src, plaq + 3 * k, part, st, fn)) return r;
        QDPX_TRY_HIP(launch_ape_step(g, prec, nrows_of(fmt), src, dst, c1, c2, smear_mask,
                                     (plaq && fused) ? part : nullptr, (plaq && fused) ? 1 : 0, cfg, st, polar),
                     fn);
        if (plaq && fused)
            QDPX_TRY_HIP(launch_finalize(part, ape_num_partials(g), 1, (double)g.V, plaq + 3 * k, st), fn);
        src = dst;
    }
    if (plaq)
        if (int r = plaquette_into(g, prec, fmt, U_out, plaq + 3 * n_steps, part, st, fn)) return r;
    return QDPX_OK;
}

// ------------------------------------------------------------------ batched
// Workspace: [counters for up to kBatchMaxSteps + 1 phases, 256-aligned]
// then per lattice [ping-pong links][plaquette partials], each 256-aligned.
static const int kBatchMaxSteps = 1024;
static const int kBatchMaxLattices = 4096;

static size_t batched_counter_bytes(int n_lat) {
    (void)n_lat;
    return round256(sizeof(unsigned) * (size_t)batched_counter_words(kBatchMaxSteps + 1));
}

static size_t batched_lattice_bytes(const qdpx_geom *g, qdpx_prec prec, qdpx_linkfmt fmt) {
    const Geo geo = make_geo(g->L);
    const size_t groups = ((size_t)geo.V + 63) / 64;
    return round256(qdpx_links_bytes(g, prec, fmt)) + round256(sizeof(double) * 2 * 4 * groups);
}

static int batched_check_geoms(int n_lat, const qdpx_geom *geoms, const char *fn) {
    if (n_lat < 1 || n_lat > kBatchMaxLattices)
        return fail(QDPX_EINVAL, "%s: n_lat = %d outside [1, %d]", fn, n_lat, kBatchMaxLattices);
    if (!geoms) return fail(QDPX_EINVAL, "%s: geoms is NULL", fn);
    for (int i = 0; i < n_lat; ++i) {
        if (!geom_ok(&geoms[i], fn)) return QDPX_EINVAL;
        const Geo g = make_geo(geoms[i].L);
        if ((g.V + 63) / 64 > batched_max_stage_groups())
            return fail(QDPX_EUNSUPPORTED, "%s: lattice %d has %d sites; batched lattices are limited to %d", fn, i,
                        g.V, batched_max_stage_groups() * 64);
    }
    return QDPX_OK;
}

static size_t batched_ws_bytes(int n_lat, const qdpx_geom *geoms, qdpx_prec prec, qdpx_linkfmt fmt, int n_steps) {
    (void)n_steps;
    const char *fn = "qdpx_workspace_bytes";
    if (batched_check_geoms(n_lat, geoms, fn) != QDPX_OK) return 0;
    if (check_format(prec, fmt, fn) != QDPX_OK) return 0;
    size_t b = batched_counter_bytes(n_lat);
    for (int i = 0; i < n_lat; ++i) b += batched_lattice_bytes(&geoms[i], prec, fmt);
    return b;
}

// The per-lattice device table is built on the first call with a given set
// of arguments and kept by the context (like the paper's device storage for
// shift tables, section 5.2); later calls, and graph replays, reuse it.
static void batch_cache_free(qdpx_ctx *ctx) {
    for (auto &kv : ctx->batch_tables) (void)hipFree(kv.second);
    ctx->batch_tables.clear();
}

static unsigned spin_limit_from_env() {
    const char *e = getenv("QDPX_SPIN_LIMIT");
    if (!e || !*e) return 1u << 24;
    return (unsigned)strtoul(e, nullptr, 10);
}

extern "C" int qdpx_ape_smear_batched(qdpx_ctx *ctx, int n_lat, const qdpx_geom *geoms, qdpx_prec prec,
                                      qdpx_linkfmt fmt, const void *const *U_in, void *const *U_out, double alpha,
                                      int n_steps, double *plaq, void *work, size_t work_bytes, void *stream) {
    const char *fn = "qdpx_ape_smear_batched";
    QDPX_CHECK_CTX(fn);
    if (int r = batched_check_geoms(n_lat, geoms, fn)) return r;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (!U_in || !U_out) return fail(QDPX_EINVAL, "%s: NULL pointer array", fn);
    if (n_steps < 1 || n_steps > kBatchMaxSteps)
        return fail(QDPX_EINVAL, "%s: n_steps = %d outside [1, %d]", fn, n_steps, kBatchMaxSteps);
    const size_t need = batched_ws_bytes(n_lat, geoms, prec, fmt, n_steps);
    if (!work || work_bytes < need) return fail(QDPX_ENOMEM, "%s: workspace of %zu bytes < %zu", fn, work_bytes, need);
    if (!aligned16(work)) return fail(QDPX_EINVAL, "%s: workspace not 16-byte aligned", fn);  // intermediate links
    std::vector<size_t> lb(n_lat);
    for (int i = 0; i < n_lat; ++i) {
        if (!U_in[i] || !U_out[i]) return fail(QDPX_EINVAL, "%s: NULL links for lattice %d", fn, i);
        if (!aligned16(U_in[i]) || !aligned16(U_out[i]))
            return fail(QDPX_EINVAL, "%s: links of lattice %d not 16-byte aligned", fn, i);
        lb[i] = qdpx_links_bytes(&geoms[i], prec, fmt);
    }
    for (int i = 0; i < n_lat; ++i) {
        if (overlap(U_out[i], lb[i], work, need)) return fail(QDPX_EALIAS, "%s: U_out[%d] overlaps the workspace", fn, i);
        if (overlap(U_in[i], lb[i], work, need)) return fail(QDPX_EALIAS, "%s: U_in[%d] overlaps the workspace", fn, i);
        for (int j = 0; j < n_lat; ++j) {
            if (overlap(U_out[i], lb[i], U_in[j], lb[j]))
                return fail(QDPX_EALIAS, "%s: U_out[%d] overlaps U_in[%d]", fn, i, j);
            if (j != i && overlap(U_out[i], lb[i], U_out[j], lb[j]))
                return fail(QDPX_EALIAS, "%s: U_out[%d] overlaps U_out[%d]", fn, i, j);
        }
    }
    if (plaq && overlap(plaq, sizeof(double) * 3 * n_lat, work, need))
        return fail(QDPX_EALIAS, "%s: plaq overlaps the workspace", fn);

    // launch geometry: threads per block (256 or 512: one or two groups at a
    // time) and groups per ticket, tuned per (first lattice's extents,
    // precision, format)
    const LaunchCfg bcfg = cfg_for(ctx, QDPX_OP_BATCHED, &geoms[0], prec, fmt);
    const int block = bcfg.block == 512 ? 512 : 256;
    const int group_chunk = std::max(1, bcfg.nsite);
    // host table: each lattice's groups as a (column, t-row) grid, its
    // columns split into 8 contiguous ranges (one per XCD queue) walked
    // t-row by t-row, in tickets of group_chunk groups
    std::vector<BatchLat> tab(n_lat);
    char *base = (char *)work + batched_counter_bytes(n_lat);
    int64_t xtotal[kXcds] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t pblocks = 0;
    for (int i = 0; i < n_lat; ++i) {
        BatchLat &L = tab[i];
        memset(&L, 0, sizeof L);
        L.g = make_geo(geoms[i].L);
        L.in = U_in[i];
        L.out = U_out[i];
        L.tmp = base;
        L.partials = (double *)(base + round256(lb[i]));
        base += batched_lattice_bytes(&geoms[i], prec, fmt);
        L.ngroups = (L.g.V + 63) / 64;
        const int per_t = L.g.L[0] * L.g.L[1] * L.g.L[2];
        if (L.g.bwl || per_t % 64 == 0) {
            L.ncol = per_t / 64;  // bricks (or runs of 64 sites) of one t plane
            L.nrow = L.g.L[3];
        } else {
            L.ncol = L.ngroups;
            L.nrow = 1;
        }
        for (int x = 0; x < kXcds; ++x) {
            L.xcol0[x] = (int)((int64_t)x * L.ncol / kXcds);
            L.xcol1[x] = (int)((int64_t)(x + 1) * L.ncol / kXcds);
            const int cols = L.xcol1[x] - L.xcol0[x];
            L.dcols[x] = FastDiv::make((uint32_t)std::max(cols, 1));
            L.xbase[x] = (int)xtotal[x];
            xtotal[x] += ((int64_t)cols * L.nrow + group_chunk - 1) / group_chunk;
        }
        L.pbase = (int)pblocks;
        pblocks += batched_plaq_blocks((int)prec, L.ngroups);
    }
    int64_t items = 0;
    for (int x = 0; x < kXcds; ++x) items += xtotal[x];
    if (items >= (int64_t)1 << 31 || pblocks >= (int64_t)1 << 31)
        return fail(QDPX_EUNSUPPORTED, "%s: too many work items", fn);

    BatchKey key;
    key.v = {(uint64_t)n_lat, (uint64_t)prec, (uint64_t)fmt, (uint64_t)(uintptr_t)work, (uint64_t)group_chunk};
    for (int i = 0; i < n_lat; ++i) {
        for (int d = 0; d < 4; ++d) key.v.push_back((uint64_t)geoms[i].L[d]);
        key.v.push_back((uint64_t)(uintptr_t)U_in[i]);
        key.v.push_back((uint64_t)(uintptr_t)U_out[i]);
    }
    hipStream_t st = (hipStream_t)stream;
    void *dtab = nullptr;
    auto it = ctx->batch_tables.find(key);
    if (it != ctx->batch_tables.end()) {
        dtab = it->second;
    } else {
        if (stream_capturing(st))
            return fail(QDPX_ECAPTURE, "%s: the first call with these lattices must not be captured", fn);
        QDPX_TRY_HIP(hipMalloc(&dtab, sizeof(BatchLat) * n_lat), fn);
        hipError_t e = hipMemcpy(dtab, tab.data(), sizeof(BatchLat) * n_lat, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(dtab);
            return hip_fail(e, fn);
        }
        ctx->batch_tables[key] = dtab;
    }
    BatchArgs a;
    memset(&a, 0, sizeof a);
    a.lats = (const BatchLat *)dtab;
    a.counters = (unsigned *)work;
    a.plaq = plaq;
    a.c1 = 1.0 - alpha;
    a.c2 = alpha / 6.0;
    a.n_lat = n_lat;
    a.n_steps = n_steps;
    a.items_per_phase = (int)items;
    for (int x = 0; x < kXcds; ++x) a.xtotal[x] = (int)xtotal[x];
    a.group_chunk = group_chunk;
    a.plaq_blocks = (int)pblocks;
    a.spin_limit = spin_limit_from_env();
    const int resident = batched_resident_blocks(prec, nrows_of(fmt), block);
    if (resident <= 0) return fail(QDPX_EHIP, "%s: occupancy query failed", fn);
    const int grid = (int)std::min<int64_t>(resident, std::max<int64_t>(items, 1));
    QDPX_TRY_HIP(launch_ape_batched(a, prec, nrows_of(fmt), block, grid, st), fn);
    return QDPX_OK;
}

// ------------------------------------------------------------------- tuner
static bool cfg_valid(qdpx_op op, qdpx_prec prec, const LaunchCfg &c) {
    if (c.block < 64 || c.block > 1024 || (c.block % 64)) return false;
    if (c.xcd < 0 || c.xcd > 2) return false;
    if (c.tw != 1 && c.tw != 2 && c.tw != 4 && c.tw != 8 && c.tw != 16) return false;
    // LDS tile: 0..4 for the FP32 APE step, none (0) elsewhere
    if (op == QDPX_OP_APE && prec == QDPX_F32 ? (c.lds < 0 || c.lds > 4) : c.lds != 0) return false;
    if (op == QDPX_OP_APE) return (c.block == 256 || c.block == 512) && (c.nsite == 1 || c.nsite == 2 || c.nsite == 4);
    if (op == QDPX_OP_SHIFT || op == QDPX_OP_CHAIN || op == QDPX_OP_JACOBI)  // four waves per group, one per direction
        return c.block == 256 && (c.nsite == 1 || c.nsite == 2 || c.nsite == 4 || c.nsite == 8);
    if (op == QDPX_OP_BATCHED)  // nsite = groups per ticket; xcd_map and t_window unused
        return (c.block == 256 || c.block == 512) && c.nsite >= 1 && c.nsite <= 1024;
    return false;
}

extern "C" int qdpx_tune_get(qdpx_ctx *ctx, qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                             int32_t *block, int32_t *sites_per_thread, int32_t *xcd_map, int32_t *t_window,
                             int32_t *lds_tile, int32_t *source) {
    const char *fn = "qdpx_tune_get";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    const LaunchCfg c = cfg_for(ctx, op, geom, prec, fmt);
    if (block) *block = c.block;
    if (sites_per_thread) *sites_per_thread = c.nsite;
    if (xcd_map) *xcd_map = c.xcd;
    if (t_window) *t_window = c.tw;
    if (lds_tile) *lds_tile = c.lds;
    if (source) {
        auto it = ctx->tuned.find(TuneKey{(int)op, (int)prec, (int)fmt, {geom->L[0], geom->L[1], geom->L[2], geom->L[3]}});
        *source = it == ctx->tuned.end() ? kSrcDefault : it->second.source;
    }
    return QDPX_OK;
}

extern "C" int qdpx_tune_set(qdpx_ctx *ctx, qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                             int32_t block, int32_t sites_per_thread, int32_t xcd_map, int32_t t_window,
                             int32_t lds_tile) {
    const char *fn = "qdpx_tune_set";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    LaunchCfg c;
    c.block = block;
    c.nsite = sites_per_thread;
    c.xcd = xcd_map;
    c.tw = t_window;
    c.lds = lds_tile;
    if (!cfg_valid(op, prec, c) || geom->L[3] % c.tw != 0)
        return fail(QDPX_EINVAL,
                    "%s: geometry (block %d, sites %d, xcd %d, t window %d, LDS tile %d) not valid for op %d", fn,
                    block, sites_per_thread, xcd_map, t_window, lds_tile, (int)op);
    ctx->tuned[TuneKey{(int)op, (int)prec, (int)fmt, {geom->L[0], geom->L[1], geom->L[2], geom->L[3]}}] =
        Tuned{c, kSrcSet};
    return QDPX_OK;
}

// Times every candidate on temporary buffers filled with a constant byte
// pattern (the kernels' cost does not depend on the values) and keeps the
// fastest in the context.
extern "C" int qdpx_tune(qdpx_ctx *ctx, qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                         void *stream) {
    const char *fn = "qdpx_tune";
    QDPX_CHECK_CTX(fn);
    if (!geom_ok(geom, fn)) return QDPX_EINVAL;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (op != QDPX_OP_APE && op != QDPX_OP_SHIFT && op != QDPX_OP_CHAIN && op != QDPX_OP_JACOBI)
        return fail(QDPX_EUNSUPPORTED, "%s: op %d is not tuned here (QDPX_OP_BATCHED: qdpx_tune_batched)", fn,
                    (int)op);
    hipStream_t st = (hipStream_t)stream;
    if (stream_capturing(st)) return fail(QDPX_ECAPTURE, "%s: stream is capturing", fn);
    const Geo g = make_geo(geom->L);
    const size_t lb = qdpx_links_bytes(geom, prec, fmt), fb = qdpx_fermion_bytes(geom, prec);
    std::vector<void *> bufs;
    auto alloc = [&](size_t n) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, n) != hipSuccess) return nullptr;
        bufs.push_back(p);
        // finite values in both precisions; a buffer that cannot be filled is
        // reported as not allocated
        if (hipMemsetAsync(p, 0x3c, n, st) != hipSuccess) return nullptr;
        return p;
    };
    auto release = [&]() {
        (void)hipStreamSynchronize(st);
        for (void *p : bufs) (void)hipFree(p);
    };
    void *U = alloc(lb), *A = nullptr, *B = nullptr, *C = nullptr, *part = nullptr;
    if (op == QDPX_OP_APE) {
        A = alloc(lb);
    } else {
        A = alloc(fb);
        B = alloc(fb);
        C = alloc(fb);
        part = alloc(reduce_bytes(shift_num_partials(g), 1));
    }
    if (!U || !A || (op != QDPX_OP_APE && (!B || !C || !part))) {
        release();
        return fail(QDPX_ENOMEM, "%s: could not allocate tuning buffers", fn);
    }
    std::vector<LaunchCfg> cands;
    const int blocks_ape[] = {256, 512};
    const int ns_ape[] = {1, 2, 4};
    const int ns_shift[] = {1, 2, 4, 8};
    const int tws[] = {1, 2, 4, 8, 16};
    for (int x = 0; x < 3; ++x)
        for (int tw : tws) {
            if (geom->L[3] % tw || (tw > 1 && (g.bwl == 0 || x == 2))) continue;
            if (op == QDPX_OP_APE) {
                for (int b : blocks_ape)
                    for (int n : ns_ape)
                        for (int t = 0; t <= (prec == QDPX_F32 ? 4 : 0); ++t) cands.push_back(LaunchCfg{b, n, x, tw, t});
            } else {
                for (int n : ns_shift) cands.push_back(LaunchCfg{256, n, x, tw});
            }
        }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        release();
        return fail(QDPX_EHIP, "%s: could not create timing events", fn);
    }
    const int nrows = nrows_of(fmt);
    auto run = [&](const LaunchCfg &c) -> hipError_t {
        if (op == QDPX_OP_APE) return launch_ape_step(g, prec, nrows, U, A, 0.5, 0.5 / 6.0, 0xFu, nullptr, 0, c, st);
        if (op == QDPX_OP_JACOBI) return launch_hop(g, prec, nrows, U, A, B, 0.1, 1.0, false, 0xFu, C, c, st);
        return launch_shift(g, prec, nrows, U, A, B, 0.3, op == QDPX_OP_CHAIN ? 1 : 0, 0.1, C, (double *)part, c, st);
    };
    // milliseconds per launch over `reps` back-to-back launches (1e30 if
    // anything failed, so a failing geometry is never chosen)
    auto time_cfg = [&](const LaunchCfg &c, int reps) -> float {
        bool ok = hipEventRecord(e0, st) == hipSuccess;
        for (int r = 0; r < reps; ++r) ok = run(c) == hipSuccess && ok;
        ok = hipEventRecord(e1, st) == hipSuccess && ok;
        ok = hipEventSynchronize(e1) == hipSuccess && ok;
        float ms = 0.f;
        ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ok;
        return ok ? ms / reps : 1e30f;
    };
    // Warm-up: about 30 launches of the default geometry, so that the first
    // candidates are not timed at idle clocks.  First pass: every candidate
    // once (after one warm-up launch), ten launches.  Second pass: the
    // sixteen fastest again, interleaved over nine passes, keeping each one's
    // best pass, so that neither a single slow or fast sample nor the clock
    // drifting during the first pass decides (candidates within a few per
    // cent of each other are common).
    for (int r = 0; r < 30; ++r) (void)run(LaunchCfg{});
    std::vector<std::pair<float, int>> r1;
    for (size_t i = 0; i < cands.size(); ++i) {
        if (run(cands[i]) != hipSuccess) continue;
        r1.push_back({time_cfg(cands[i], 10), (int)i});
    }
    std::sort(r1.begin(), r1.end());
    const size_t keep = std::min<size_t>(16, r1.size());
    std::vector<float> best_ms(keep, 1e30f);
    for (int pass = 0; pass < 9; ++pass)
        for (size_t k = 0; k < keep; ++k) best_ms[k] = std::min(best_ms[k], time_cfg(cands[r1[k].second], 10));
    LaunchCfg best_cfg;
    float best = 1e30f;
    for (size_t k = 0; k < keep; ++k)
        if (best_ms[k] < best) {
            best = best_ms[k];
            best_cfg = cands[r1[k].second];
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    release();
    if (best >= 1e30f) return fail(QDPX_EHIP, "%s: no candidate geometry ran", fn);
    const TuneKey key{(int)op, (int)prec, (int)fmt, {geom->L[0], geom->L[1], geom->L[2], geom->L[3]}};
    ctx->tuned[key] = Tuned{best_cfg, kSrcTuned};
    log_cfg("tuned", key, best_cfg);
    // a context with a launch table keeps what it tuned for later processes
    if (!ctx->cache_path.empty()) return save_table(ctx, ctx->cache_path, fn);
    return QDPX_OK;
}

// Times the batched call on the caller's batch of extents with temporary
// links filled with a constant byte pattern (the cost does not depend on the
// values): 256- or 512-thread blocks and 1 to 8 groups per ticket; keeps the
// fastest under the first lattice's extents.
extern "C" int qdpx_tune_batched(qdpx_ctx *ctx, int n_lat, const qdpx_geom *geoms, qdpx_prec prec, qdpx_linkfmt fmt,
                                 int n_steps, void *stream) {
    const char *fn = "qdpx_tune_batched";
    QDPX_CHECK_CTX(fn);
    if (int r = batched_check_geoms(n_lat, geoms, fn)) return r;
    if (int r = check_format(prec, fmt, fn)) return r;
    if (n_steps < 1 || n_steps > kBatchMaxSteps)
        return fail(QDPX_EINVAL, "%s: n_steps = %d outside [1, %d]", fn, n_steps, kBatchMaxSteps);
    hipStream_t st = (hipStream_t)stream;
    if (stream_capturing(st)) return fail(QDPX_ECAPTURE, "%s: stream is capturing", fn);
    std::vector<void *> bufs;
    auto alloc = [&](size_t n) -> void * {
        void *p = nullptr;
        if (hipMalloc(&p, n) != hipSuccess) return nullptr;
        bufs.push_back(p);
        if (hipMemsetAsync(p, 0x3c, n, st) != hipSuccess) return nullptr;
        return p;
    };
    std::vector<const void *> in(n_lat);
    std::vector<void *> out(n_lat);
    const size_t wb = batched_ws_bytes(n_lat, geoms, prec, fmt, n_steps);
    void *work = alloc(wb);
    void *plaq = alloc(sizeof(double) * 3 * (size_t)n_lat);
    bool ok = work && plaq;
    for (int i = 0; i < n_lat && ok; ++i) {
        const size_t lb = qdpx_links_bytes(&geoms[i], prec, fmt);
        in[i] = alloc(lb);
        out[i] = alloc(lb);
        ok = in[i] && out[i];
    }
    const TuneKey key{(int)QDPX_OP_BATCHED, (int)prec, (int)fmt, {geoms[0].L[0], geoms[0].L[1], geoms[0].L[2], geoms[0].L[3]}};
    const auto saved = ctx->tuned.find(key) == ctx->tuned.end() ? Tuned{} : ctx->tuned[key];
    const bool had = ctx->tuned.count(key) != 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ok = ok && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        // the device tables built for the temporary buffers
        for (auto it = ctx->batch_tables.begin(); it != ctx->batch_tables.end();) {
            if (it->first.v.size() > 3 && it->first.v[3] == (uint64_t)(uintptr_t)work) {
                (void)hipFree(it->second);
                it = ctx->batch_tables.erase(it);
            } else {
                ++it;
            }
        }
        for (void *p : bufs) (void)hipFree(p);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (had) ctx->tuned[key] = saved;
        else ctx->tuned.erase(key);
    };
    if (!ok) {
        cleanup();
        return fail(QDPX_ENOMEM, "%s: could not allocate tuning buffers", fn);
    }
    auto run = [&](const LaunchCfg &c) -> bool {
        ctx->tuned[key] = Tuned{c, kSrcSet};
        return qdpx_ape_smear_batched(ctx, n_lat, geoms, prec, fmt, in.data(), out.data(), 0.5, n_steps,
                                      (double *)plaq, work, wb, stream) == QDPX_OK;
    };
    std::vector<LaunchCfg> cands;
    for (int b : {256, 512})
        for (int n : {1, 2, 4, 8}) cands.push_back(LaunchCfg{b, n, 1, 1});
    std::vector<float> best_ms(cands.size(), 1e30f);
    for (int pass = 0; pass < 3; ++pass)
        for (size_t i = 0; i < cands.size(); ++i) {
            if (!run(cands[i])) continue;  // warm-up (builds the table on the first pass)
            bool good = hipEventRecord(e0, st) == hipSuccess;
            for (int r = 0; r < 3; ++r) good = run(cands[i]) && good;
            good = hipEventRecord(e1, st) == hipSuccess && good;
            good = hipEventSynchronize(e1) == hipSuccess && good;
            float ms = 0.f;
            good = hipEventElapsedTime(&ms, e0, e1) == hipSuccess && good;
            if (good) best_ms[i] = std::min(best_ms[i], ms / 3);
        }
    size_t bi = 0;
    for (size_t i = 1; i < cands.size(); ++i)
        if (best_ms[i] < best_ms[bi]) bi = i;
    const float best = best_ms[bi];
    cleanup();
    if (best >= 1e30f) return fail(QDPX_EHIP, "%s: no candidate geometry ran", fn);
    ctx->tuned[key] = Tuned{cands[bi], kSrcTuned};
    log_cfg("tuned", key, cands[bi]);
    if (!ctx->cache_path.empty()) return save_table(ctx, ctx->cache_path, fn);
    return QDPX_OK;
}
