// Host-side internal interface between the C ABI layer (api.cpp) and the
// translation units that own the kernels.  Not installed, not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "su3_device.hpp"

namespace qdpx {

// Launch geometry of one operation (chosen by the tuner or defaulted).
struct LaunchCfg {
    int block = 256;  // threads per block, multiple of 64
    int nsite = 1;    // consecutive 64-site groups handled per wave
    int xcd = 1;      // 0: identity, 1: XCD-contiguous tile ranges, 2: XCD slab walk
    int tw = 1;       // t planes walked together (brick mapping only; must divide Lt)
    int lds = 0;      // LDS tile of the FP32 APE step: 0 none, 1 own links, 2 also backward links,
                      // 3 also the plane products, 4 own links and plane products
};

// Threads per block of the fixed-shape reduction kernels (plaquette,
// finalisation).  Kept fixed so that reduced values are bit-identical for
// every tuned geometry of the other kernels.
constexpr int kReduceBlock = 256;

// One stored launch geometry (launch-table file, tunecache.cpp).  op, prec
// and fmt are the qdpx_op, qdpx_prec and qdpx_linkfmt values.
struct TuneEntry {
    int op = 0, prec = 0, fmt = 0;
    int L[4] = {0, 0, 0, 0};
    LaunchCfg cfg;
};
// 0: read; 1: no such file; 2: the file was recorded on another
// architecture (out stays empty); -1: unreadable or malformed (err set).
int tune_table_read(const char *path, const char *arch, std::vector<TuneEntry> &out, std::string &err);
// Writes the table atomically (temporary file + rename); 0 or -1 (err set).
int tune_table_write(const char *path, const char *arch, const std::vector<TuneEntry> &in, std::string &err);

Geo make_geo(const int32_t L[4]);
int launch_order(const Geo &g, const LaunchCfg &cfg, int groups_per_block);

// ---- fields.hip
hipError_t launch_pack_links(const Geo &g, int prec, int nrows, const double *aos, void *soa, hipStream_t st);
hipError_t launch_unpack_links(const Geo &g, int prec, int nrows, const void *soa, double *aos, hipStream_t st);
hipError_t launch_pack_fermion(const Geo &g, int prec, const double *aos, void *soa, hipStream_t st);
hipError_t launch_unpack_fermion(const Geo &g, int prec, const void *soa, double *aos, hipStream_t st);

// Shift expression chi = sum_{mu in mask} hop_mu(psi) + a*phi, forward hops
// (bwd = 0) or backward hops (bwd = 1).  mode 0: out = chi; mode 1:
// out = psi - c*chi.  partials (nullable): one FP64 partial of |chi|^2 per
// 64-site group, shift_num_partials(g) entries.
int shift_num_partials(const Geo &g);
hipError_t launch_shift(const Geo &g, int prec, int nrows, const void *U, const void *psi, const void *phi,
                        double a, int mode, double c, void *out, double *partials, const LaunchCfg &cfg,
                        hipStream_t st, unsigned mask = 0xFu, int bwd = 0);
hipError_t launch_copy_fermion(const Geo &g, int prec, const void *src, void *dst, hipStream_t st);

// Jacobi hop: out = [s0 + kappa * H psi] / norm (s0 nullable; division only
// if `divide`), H summed over the directions in mask, both hop directions.
hipError_t launch_hop(const Geo &g, int prec, int nrows, const void *U, const void *psi, const void *s0, double kappa,
                      double norm, bool divide, unsigned mask, void *out, const LaunchCfg &cfg, hipStream_t st);

// Deterministic finalisation.  mode 0: out[0] = sum of partials[0..n).
// mode 1 (plaquette): partials hold n spatial then n temporal sums;
// out = {(sp+tp)/(18V), sp/(9V), tp/(9V)}.
hipError_t launch_finalize(const double *partials, int n, int mode, double volume, double *out, hipStream_t st);

// ---- ape.hip
// One APE step.  mode 0: links only; mode 1 (FP64 links, Gram-Schmidt
// projection, every direction smeared): also the plaquette traces of the
// INPUT links into partials.
// partials hold ape_num_partials(g) values per component (spatial,
// temporal), reduced by launch_finalize(partials, ape_num_partials(g), 1, V, out).
int ape_num_partials(const Geo &g);
hipError_t launch_ape_step(const Geo &g, int prec, int nrows, const void *Uin, void *Uout, double c1, double c2,
                           unsigned mask, double *partials, int mode, const LaunchCfg &cfg, hipStream_t st,
                           int proj = 0);  // proj 1: polar projection (mode 0 only)
int plaquette_num_partials(const Geo &g);  // per component (2 components)
hipError_t launch_plaquette(const Geo &g, int prec, int nrows, const void *U, double *partials, hipStream_t st);

// ---- batched.hip
// Number of XCDs of the MI355X: each has its own L2 and its own work queue.
constexpr int kXcds = 8;

// One lattice of a batch (device table entry).  Its 64-site groups form a
// (column, t-row) grid, group = col + ncol * row, where a column is one
// brick (or run of groups) of one z plane and rows step in t.  The columns
// are split into 8 contiguous ranges [xcol0[x], xcol1[x]), one per XCD
// queue; queue x walks its range t-row by t-row (group j of the queue is
// row j / cols, column xcol0 + j % cols), in tickets of group_chunk groups.
struct BatchLat {
    Geo g;
    const void *in;    // caller's input links
    void *out;         // caller's output links
    void *tmp;         // ping-pong links in the workspace (n_steps >= 2)
    double *partials;  // 2 * 4 * ngroups plaquette partials in the workspace
    int ngroups;       // 64-site groups
    int ncol, nrow;    // group grid
    int xcol0[kXcds], xcol1[kXcds];  // each XCD queue's column range
    FastDiv dcols[kXcds];            // division by the range's width
    int xbase[kXcds];  // first ticket of this lattice in each XCD's queue
    int pbase;         // first block of this lattice in the plaquette launch
};

struct BatchArgs {
    const BatchLat *lats;  // device table [n_lat]
    unsigned *counters;    // [1] status, then per phase 8 ticket counters and a completion counter
    double *plaq;          // nullable, [n_lat][3]
    double c1, c2;
    int n_lat, n_steps, group_chunk;
    int xtotal[kXcds];     // tickets in each XCD's queue per phase
    int items_per_phase;   // sum of xtotal
    int plaq_blocks;       // blocks of the plaquette launch
    unsigned spin_limit;
};

int batched_max_stage_groups();
int batched_counter_words(int max_phases);
int batched_plaq_blocks(int prec, int ngroups);
// resident blocks of the persistent kernel with `block` (256 or 512) threads
int batched_resident_blocks(int prec, int nrows, int block);
hipError_t launch_ape_batched(const BatchArgs &a, int prec, int nrows, int block, int grid, hipStream_t st);

}  // namespace qdpx
