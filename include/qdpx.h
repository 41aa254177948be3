/*
 * qdpx — site-parallel lattice field expressions and APE link smearing on
 * AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Background.  The method evaluates lattice-wide expressions of a quantum
 * field theory code site by site on the GPU (paper: "Accelerating QDP++ using
 * GPUs", sections 5 and 7).  Its central expression is the nearest-neighbour
 * hop U_mu(x) psi(x+mu) summed over directions plus an axpy term, the
 * building block of the Jacobi smearing operator (section 7, equation for K,
 * and the listing's expressions E_1, E_2, E_3).  This library provides that
 * expression, an iterated chain of it, one or many APE link-smearing steps
 * with an SU(3) projection, and the average plaquette.
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice: extents L[0..3] = (Lx, Ly, Lz, Lt), 2 <= L[d] <= 4096,
 *   V = Lx*Ly*Lz*Lt < 2^28 (so every per-component byte offset fits 32
 *   bits; 2^28 sites of FP64 links are 154 GB); direction mu = 0..3 is x, y, z, t; all
 *   directions periodic; site = x + Lx*(y + Ly*(z + Lz*t)).
 * Matrices: U_mu(x) is a 3x3 complex matrix acting on colour,
 *   (U psi)_a = sum_b U_ab psi_b, identity in spin.  "Row" = first index.
 * Host canonical layout ("AoS"), FP64, used by the pack/unpack calls:
 *   links    double[V][4][3][3][2]   (site, mu, row, column, re/im)
 *   fermions double[V][4][3][2]      (site, spin, colour, re/im)
 * Library layout ("SoA", opaque to callers, sized by qdpx_links_bytes /
 *   qdpx_fermion_bytes): the site index innermost, padded to a stride
 *   S = qdpx_site_stride(geom).  Links store rows 0..2 (LINK18) or rows 0..1
 *   (LINK12; row 2 is rebuilt as conj(row0 x row1) on every load, exact for
 *   SU(3)); stored element c = 3*row + col of direction mu:
 *     QDPX_F64  one array of S double2 per element, [mu][c][S];
 *     QDPX_F32  elements 2k and 2k+1 share one 16-byte entry (float4) of
 *               array k, [mu][k][S]; the ninth LINK18 element has an array
 *               of S float2 of its own after the four pair arrays.
 *   Either way a direction takes 3*rows*S complex slots.  Fermions, with
 *   component q = 3*spin + colour: QDPX_F64 one array of S double2 per
 *   component, [q][S]; QDPX_F32 components 2k and 2k+1 share one 16-byte
 *   entry (float4, q even in the low half) of array k, [k][S], k = 0..5.
 *   Link fields, Dirac fields and workspaces must be 16-byte aligned; other
 *   pointers are refused with QDPX_EINVAL before anything is launched.
 *
 * Memory and streams.  Every pointer argument named *_dev, and every field
 *   argument (U, psi, phi, chi, ...), is a DEVICE pointer owned by the caller.
 *   The library never allocates, frees or keeps caller memory.  Scratch space
 *   is a caller-provided device workspace of at least qdpx_workspace_bytes()
 *   bytes.  Every compute call only enqueues work on `stream` (a hipStream_t
 *   passed as void*, NULL = the null stream), never synchronises, never
 *   allocates and issues no memset, so it may be recorded into a HIP graph
 *   (the one exception, the first batched call for a new batch, is described
 *   at qdpx_ape_smear_batched).
 *   Scalar results (norms, plaquettes) are written to caller DEVICE buffers
 *   of doubles.
 *
 * Errors.  Every call returns QDPX_OK (0) or a negative qdpx_status.  On a
 *   validation error nothing is enqueued and no output is written; the
 *   message is available from qdpx_last_error() (thread-local).  Launch
 *   errors map to QDPX_EHIP; faults during execution surface at the caller's
 *   next synchronisation.
 *
 * Threading.  A context may be used by one host thread at a time.  Calls
 *   that overlap on one device must not share a workspace.
 */
#ifndef QDPX_H
#define QDPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QDPX_OK = 0,
    QDPX_EINVAL = -1,       /* bad extents, sizes, null pointer, n < 1, ... */
    QDPX_EALIAS = -2,       /* an output overlaps an input it must not overlap */
    QDPX_ENOMEM = -3,       /* workspace smaller than qdpx_workspace_bytes() */
    QDPX_EHIP = -4,         /* a HIP runtime call or kernel launch failed */
    QDPX_EUNSUPPORTED = -5, /* precision / link format combination not provided */
    QDPX_ECAPTURE = -6      /* call not allowed while the stream is being captured */
} qdpx_status;

typedef enum { QDPX_F64 = 0, QDPX_F32 = 1 } qdpx_prec;

/* LINK18 stores all 9 complex entries; LINK12 stores rows 0 and 1 only and
 * is accepted with QDPX_F32 only.  Links are taken to be SU(3): FP64 LINK18
 * links are read as rows 0 and 1 with row 2 rebuilt as conj(row0 x row1)
 * in FP64 by the shift, chain, hop, Jacobi, plaquette and run-time compiled
 * kernels and by the Gram-Schmidt APE step (the stored row 2 equals it to
 * rounding for SU(3) links; a third fewer bytes); FP32 LINK18 links are read
 * whole, and the polar APE step and the pack/unpack calls read every stored
 * element. */
typedef enum { QDPX_LINK18 = 0, QDPX_LINK12 = 1 } qdpx_linkfmt;

/* SU(3) projection of the APE combination W (qdpx_ape_smear). */
typedef enum {
    QDPX_PROJ_GRAM_SCHMIDT = 0, /* row Gram-Schmidt, rows 0 and 1 of W only */
    QDPX_PROJ_POLAR = 1         /* W (W^dag W)^(-1/2) with the det phase removed: bi-covariant */
} qdpx_proj;

typedef struct { int32_t L[4]; } qdpx_geom;

/* Operation ids for qdpx_workspace_bytes() and qdpx_tune(). */
typedef enum {
    QDPX_OP_SHIFT = 0,    /* qdpx_eval_shift_mul_axpy */
    QDPX_OP_CHAIN = 1,    /* qdpx_shift_chain */
    QDPX_OP_APE = 2,      /* qdpx_ape_smear */
    QDPX_OP_PLAQ = 3,     /* qdpx_plaquette */
    QDPX_OP_BATCHED = 4,  /* qdpx_ape_smear_batched (n = number of lattices) */
    QDPX_OP_JACOBI = 5    /* qdpx_jacobi_smear and qdpx_eval_hop */
} qdpx_op;

typedef struct qdpx_ctx qdpx_ctx;

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `device`.  The context plays the role
 * of the paper's device storage container (section 5.2): it caches
 * tuned launch geometries and the per-lattice tables of batched calls.
 * Every later call that takes the context and launches, tunes or compiles
 * must be made while `device` is the current HIP device; otherwise it
 * returns QDPX_EINVAL and does nothing.
 * tune_cache_path (nullable): a launch-table file that keeps tuned thread
 *   geometries for later runs, as the paper's auto-tuning proposal does
 *   (sections 5.4 and 9).  NULL takes the path from the environment variable
 *   QDPX_TUNE_CACHE, if set; otherwise the context has no table and every
 *   operation starts from the default geometry.  The file is read here
 *   (a missing file is an empty table; entries recorded for another GPU
 *   architecture are ignored) and rewritten, merged, by every qdpx_tune on
 *   this context and by qdpx_tune_save.  Format: JSON
 *   {"device": "<gcnArchName>", "entries": [{"op": "APE", "prec": "F32",
 *   "fmt": "LINK12", "L": [Lx, Ly, Lz, Lt], "launch": [block,
 *   groups_per_wave, xcd_map, t_window, lds_tile]}, ...]}, op one of SHIFT
 *   CHAIN APE PLAQ BATCHED JACOBI, prec F64 or F32, fmt LINK18 or LINK12
 *   (a four-element "launch" is read with the default lds_tile).
 *   With the environment variable QDPX_LOG set (not "" or "0") the library
 *   prints one line on stderr per table read or write and per tuned geometry.
 * Returns QDPX_EINVAL for a null `out`, a device that does not exist, or a
 * table file that cannot be read or holds malformed or invalid entries. */
int qdpx_create(qdpx_ctx **out, int device, const char *tune_cache_path);

/* Destroy a context (NULL is accepted).  Frees what the context cached. */
int qdpx_destroy(qdpx_ctx *ctx);

/* Release every device table cached by the context (the paper's
 * freeAll of section 6); the context stays usable. */
int qdpx_free_all(qdpx_ctx *ctx);

/* Message describing the last error on the calling thread ("" if none). */
const char *qdpx_last_error(void);

/* Library version string. */
const char *qdpx_version(void);

/* ------------------------------------------------------------------ sizes */

/* Padded site stride S used by the SoA layout (V rounded up to 256), or -1
 * for invalid extents. */
int64_t qdpx_site_stride(const qdpx_geom *geom);

/* Bytes of one SoA link field (all 4 directions) / one SoA Dirac field, or 0
 * for invalid arguments. */
size_t qdpx_links_bytes(const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt);
size_t qdpx_fermion_bytes(const qdpx_geom *geom, qdpx_prec prec);

/* Workspace bytes needed by operation `op` (n = n_steps for APE, n_iter for
 * the chain, number of lattices for the batched call with `geom` pointing to
 * that many extents; ignored otherwise).  0 for invalid arguments. */
size_t qdpx_workspace_bytes(qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt, int n);

/* ------------------------------------------------------------ pack / unpack
 * Conversions between the host canonical AoS layout (already on the device)
 * and the library SoA layout; the analogue of the paper's push/pop of
 * lattice objects between memory domains (sections 5.3 and 6).  FP64 -> FP32
 * rounds to nearest even.  Unpacking LINK12 rebuilds row 2 in FP64. */
int qdpx_pack_links(qdpx_ctx *ctx, const qdpx_geom *geom, const double *aos, qdpx_prec prec,
                    qdpx_linkfmt fmt, void *soa, void *stream);
int qdpx_unpack_links(qdpx_ctx *ctx, const qdpx_geom *geom, const void *soa, qdpx_prec prec,
                      qdpx_linkfmt fmt, double *aos, void *stream);
int qdpx_pack_fermion(qdpx_ctx *ctx, const qdpx_geom *geom, const double *aos, qdpx_prec prec,
                      void *soa, void *stream);
int qdpx_unpack_fermion(qdpx_ctx *ctx, const qdpx_geom *geom, const void *soa, qdpx_prec prec,
                        double *aos, void *stream);

/* ------------------------------------------------------- shift expression
 * chi(x) = sum_{mu in dir_mask} h_mu(x) + a * phi(x), with
 *   sign = +1:  h_mu(x) = U_mu(x) psi(x+mu)          (forward hop)
 *   sign = -1:  h_mu(x) = U_mu(x-mu)^dagger psi(x-mu) (backward hop)
 * The forward term is shift(psi, FORWARD, mu) multiplied by the link, the
 * backward term the shift(adj(U) psi, BACKWARD, mu) of the other hopping
 * term of K, summed over the directions in dir_mask, plus an axpy term added
 * once (paper section 7: the smearing operator K and the listing's
 * expressions E_1, E_2 and E_3).  With dir_mask 0xF and sign +1 this is the
 * 16^3 x 32 shift-expression workload (a = 0.3, four forward hops, FP64 norm).
 *   U: SoA links (prec, fmt); psi, phi: SoA fermions (prec); phi may be NULL
 *   (then `a` is ignored); chi: SoA fermion output, must not overlap psi, phi
 *   or U.  dir_mask: bit mu selects direction mu (0 leaves only a * phi);
 *   bits above 3 are refused.  sign: +1 or -1, anything else is refused.
 *   Both hops of qdpx_eval_hop together are sign +1 plus sign -1.
 *   norm2 (nullable, device double*) receives sum_x |chi(x)|^2
 *   accumulated in FP64 for both precisions.  work: workspace of
 *   work_bytes >= qdpx_workspace_bytes(QDPX_OP_SHIFT, ...). */
int qdpx_eval_shift_mul_axpy(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                             const void *U, const void *psi, const void *phi, double a, uint32_t dir_mask,
                             int sign, void *chi, double *norm2, void *work, size_t work_bytes, void *stream);

/* The shift expression above for callers that cannot allocate or pass a
 * workspace (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels, with the |chi|^2 partials in a
 * scratch array of fixed size that the library keeps in every device's
 * memory for the life of the process (4 MiB per device).  Arguments as for
 * qdpx_eval_shift_mul_axpy without work/work_bytes.  Lattices of more than
 * 2^25 sites are refused with QDPX_EINVAL.  Allocates nothing and issues no
 * memset.  Every call on one device shares that device's array: calls that
 * may overlap on one device (other streams, other host threads) race and
 * must be serialised by the caller. */
int qdpx_eval_shift_mul_axpy_noalloc(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                                     const void *U, const void *psi, const void *phi, double a, uint32_t dir_mask,
                                     int sign, void *chi, double *norm2, void *stream);

/* ------------------------------------------------------- expression chain
 * n_iter repetitions of  chi_k = sum_mu U_mu(x) psi_{k-1}(x+mu) + a*phi(x);
 *                        psi_k = psi_{k-1} - c * chi_k
 * with U and phi fixed (the iteration structure of the paper's smearing
 * listing; as a workload, 8 iterations with a = 0.3 and c = 0.1 on 48^3 x 96
 * after 20 APE steps).  psi is updated in place; chi is not stored.  norms (nullable,
 * device double[n_iter]) receives |chi_k|^2 in FP64.  phi may be NULL.
 * n_iter >= 1.  work: >= qdpx_workspace_bytes(QDPX_OP_CHAIN, ..., n_iter). */
int qdpx_shift_chain(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                     const void *U, void *psi, const void *phi, double a, double c, int n_iter,
                     double *norms, void *work, size_t work_bytes, void *stream);

/* --------------------------------------------------------- Jacobi smearing
 * The paper's application (section 7): the hopping term of the smearing
 * operator K = delta - kappa sum_mu [U_mu(x) delta_{x',x+mu} + U_mu(x-mu)^dag
 * delta_{x',x-mu}] and the iteration of its listing that sums the power series
 * of K^{-1} up to n_iter terms.
 *
 * qdpx_eval_hop: out(x) = sum_{mu in dir_mask} [U_mu(x) psi(x+mu)
 *   + U_mu(x-mu)^dag psi(x-mu)]  (the listing's expressions E_1/E_2 summed over
 *   mu).  dir_mask bit mu selects direction mu (0xF: all four, as the
 *   listing's loop over Nd; 0x7: the three spatial ones).  out must not
 *   overlap psi or U.
 * qdpx_jacobi_smear: chi <- (1/norm) sum_{n=0}^{n_iter} (kappa H)^n chi, the
 *   power series of K^{-1} = (1 - kappa H)^{-1} truncated after n_iter hops
 *   and applied to the source held in chi (H summed over dir_mask), updated
 *   in place; n_iter >= 1, norm != 0.  It is evaluated in Horner form, each
 *   partial sum p_k = s0 + kappa H p_{k-1} (p_0 = s0) one fused kernel with
 *   the division by norm folded into the last one; this is the expression
 *   sequence E_0 .. E_4 of the listing.
 *   work: >= qdpx_workspace_bytes(QDPX_OP_JACOBI, ...) (two fermion fields). */
int qdpx_eval_hop(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt, const void *U,
                  const void *psi, void *out, uint32_t dir_mask, void *stream);
int qdpx_jacobi_smear(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt, const void *U,
                      void *chi, double kappa, int n_iter, double norm, uint32_t dir_mask, void *work,
                      size_t work_bytes, void *stream);

/* ----------------------------------------------------------- APE smearing
 * n_steps >= 1 APE steps.  The step is defined by the workload, not by the
 * paper (whose application is the Jacobi smearing above): one step of
 * alpha = 0.5 on a 4^4 periodic lattice of Haar-random links in FP64 with
 * the row Gram-Schmidt projection and the FP64 plaquette, and 10 iterated
 * steps on 32^3 x 64 with FP32 staples on 12-real links and the projection
 * and plaquette in FP64.  One step, for every site x and every direction
 * mu in smear_mask, from the unsmeared links of that step:
 *   W_mu(x) = (1-alpha) U_mu(x) + alpha/(2(d-1)) sum_{nu in mask, nu != mu} [
 *               U_nu(x) U_mu(x+nu) U_nu(x+mu)^dagger
 *             + U_nu(x-nu)^dagger U_mu(x-nu) U_nu(x-nu+mu) ]
 *   V_mu(x) = rows (u, v, conj(u x v)) with u = w0/|w0|,
 *             v = (w1 - (u^dagger w1) u) / |...|   (w0, w1 = rows 0, 1 of W),
 * d = number of directions in smear_mask, so alpha weighs the mean of the
 * link's staples (alpha/6 with all four directions, alpha/4 with the three
 * spatial ones).  Links of directions outside smear_mask are copied
 * unchanged.  smear_mask: bit mu = direction mu; 0xF smears all four, 0x7
 * leaves the time direction alone (the role of the no-smear direction
 * argument of the smearing routine of section 7).  The projection is always
 * FP64.  With QDPX_F32 the staple products are evaluated in FP32.  FP64
 * steps with the Gram-Schmidt projection read rows 0 and 1 of every input
 * link and take row 2 as conj(row0 x row1), rebuilt in FP64 (exact for SU(3)
 * links; every smeared link's stored row 2 is that by construction); the
 * other steps use the stored row 2 (LINK18) or rebuild it (LINK12).  U_in is
 * not modified; U_out must not overlap U_in.
 * projection: QDPX_PROJ_GRAM_SCHMIDT (the rows above; only rows 0 and 1 of
 * the staples are formed) or QDPX_PROJ_POLAR: V = W (W^dag W)^(-1/2)
 * exp(-i arg(det)/3), the unitary polar factor with the phase of its
 * determinant removed (principal branch), by nine scaled Newton iterations in
 * FP64 on the full staple sum.  The polar projection commutes with
 * W -> g W h^dag for any g, h in SU(3), so the whole step commutes with a
 * gauge transformation U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag; row Gram-Schmidt
 * does so only for diagonal g.
 * plaq (nullable, device double[3*(n_steps+1)]) receives the plaquette
 * triple (total, spatial, temporal; normalised as in qdpx_plaquette; all six
 * planes whatever the mask) of the input and of every step's output, every
 * product and sum in FP64: qdpx_plaquette's pass on those links (FP32
 * entries widened to FP64), bit for bit; except that FP64 links with
 * smear_mask 0xF and the Gram-Schmidt projection fuse the traces of a
 * step's input into that step's kernel (each plaquette from rows 0 and 1 of
 * its two halves, exact for SU(3) links), which agree with qdpx_plaquette
 * to FP64 rounding (the last output's triple is the pass).  The smeared
 * links do not depend on whether plaq is requested.
 * A W whose row 0 or projected row 1 vanishes gives NaN entries.
 * work: >= qdpx_workspace_bytes(QDPX_OP_APE, ..., n_steps). */
int qdpx_ape_smear(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                   const void *U_in, void *U_out, double alpha, int n_steps, uint32_t smear_mask,
                   qdpx_proj projection, double *plaq, void *work, size_t work_bytes, void *stream);

/* -------------------------------------------------------------- plaquette
 * The average plaquette the APE workloads report in FP64 (one step on 4^4,
 * 10 steps on 32^3 x 64); the normalisation, which the workload leaves
 * open, makes unit links give 1:
 * plaq[0] = (1/(18V)) sum_x sum_{mu<nu} Re Tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag]
 * plaq[1] = the same over the three spatial planes (nu < 3), / (9V)
 * plaq[2] = the same over the three planes with nu = t,      / (9V)
 * Products and sums in FP64 for both precisions (FP32 links are widened).
 * plaq: device double[3].  work: >= qdpx_workspace_bytes(QDPX_OP_PLAQ, ...). */
int qdpx_plaquette(qdpx_ctx *ctx, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                   const void *U, double *plaq, void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------------ batched APE smearing
 * The batched workload: 64 independent lattices with extents drawn from
 * 8^4, 12^3 x 24, 16^3 x 32 and 24^3 x 48, 5 APE steps each and the final
 * plaquettes, enqueued as one group of kernels that a HIP graph may capture.
 * n_lat independent lattices of any extents (each at most 4194304 sites),
 * each smeared n_steps times (1 <= n_steps <= 1024) as in qdpx_ape_smear
 * with smear_mask 0xF, followed by each lattice's output plaquette triple.
 * All n_steps steps of all lattices run in ONE persistent kernel launch: it
 * runs in phases (step 1 .. n_steps); within a phase the work items of every
 * lattice are shared by all blocks through per-XCD ticket queues, and a phase
 * starts once every block has finished the previous one, so a batch of small
 * and large lattices fills the GPU as one job.  Around it: a small kernel
 * that clears the counters before, and (plaq non-NULL) two kernels after it
 * that form and reduce the plaquettes of every lattice.
 *   geoms: host array [n_lat]; U_in, U_out: host arrays [n_lat] of device
 *   pointers (SoA, prec, fmt; U_out[i] must not overlap any U_in[j] or
 *   another U_out[j]); plaq (nullable): device double[n_lat][3].
 *   work: >= qdpx_workspace_bytes(QDPX_OP_BATCHED, geoms, prec, fmt, n_lat)
 *   bytes; it holds the counters, ping-pong links and plaquette partials.
 *   Bytes [4, 8) of work receive a uint32 status when the kernel ends: 0, or
 *   1 if a wait for a previous step exceeded its spin limit (outputs are then
 *   incomplete; the limit may be lowered with the environment variable
 *   QDPX_SPIN_LIMIT, read at every call, to exercise this path).
 * The first call with a given (lattices, pointers, workspace, groups per
 * ticket) set copies a small per-lattice table to the device and keeps it in
 * the context (freed by qdpx_free_all / qdpx_destroy); that first call
 * synchronises and returns QDPX_ECAPTURE on a capturing stream.  Later calls,
 * and replays of a graph that captured one, reuse the table and only enqueue
 * the kernels.  Links and plaquettes are identical, bit for bit, to
 * qdpx_ape_smear on each lattice with plaquettes requested.  Work items are
 * runs of 64-site groups of one lattice: each lattice's columns (one brick of
 * one z plane each) are split into 8 contiguous ranges, one per XCD queue,
 * walked t-row by t-row.  Threads per block (256 or 512) and groups per
 * ticket come from qdpx_tune_batched, or qdpx_tune_set(ctx, QDPX_OP_BATCHED,
 * &geoms[0], prec, fmt, block, groups, 1, 1, 0) (default 256 and 1).  The
 * final plaquettes are qdpx_plaquette's pass on each lattice's output. */
int qdpx_ape_smear_batched(qdpx_ctx *ctx, int n_lat, const qdpx_geom *geoms, qdpx_prec prec,
                           qdpx_linkfmt fmt, const void *const *U_in, void *const *U_out,
                           double alpha, int n_steps, double *plaq, void *work, size_t work_bytes,
                           void *stream);

/* ---------------------------------------------- run-time compiled expressions
 * The paper evaluates each lattice expression with a kernel generated from
 * its expression tree, compiled at run time and kept for reuse (section 5.1).
 * Expressions here are S-expressions over Dirac fields (spinor x colour
 * vectors) and the link field:
 *   fK                 field argument K (0 <= K < n_fields <= 8)
 *   (shift E + mu)     E evaluated at x + mu;  (shift E - mu): at x - mu
 *   (umul mu E)        U_mu(x) E(x);  (uadj mu E): U_mu(x)^dagger E(x)
 *   (add E F)  (sub E F)  (scale sK E)   sK: scalar argument K (< n_scalars <= 8)
 *   (sum MASK E)       sum over the directions in MASK (hex, 0x1..0xF) of E
 *                      with the direction variable m standing for each one
 * A direction mu is a digit 0..3 (x, y, z, t) or m inside a sum; sums do not
 * nest.  The listing's hopping term E_1 + E_2 is
 *   (sum 0xF (add (umul m (shift f0 + m)) (shift (uadj m f0) - m)))
 * and a smearing iteration E_3 is (add f1 (scale s0 <that>)).
 *
 * qdpx_jit_generate: the HIP source of the kernel for an expression (no
 *   device needed); *needed receives the size including the terminator; with
 *   buf non-NULL the source is copied (QDPX_ENOMEM if it does not fit).
 * qdpx_jit_compile: generates the kernel, compiles it with hipRTC for the
 *   current device (packed FP32 disabled) or loads the code object from the
 *   on-disk cache (directory $QDPX_JIT_CACHE, else $HOME/.cache/qdpx-jit,
 *   created private to the user; neither variable set, or a directory that
 *   others can write: no disk cache; file name a hash of source, options and
 *   architecture; an entry is loaded only if it is a private regular file
 *   holding this kernel's exact source, options and architecture), and returns a
 *   kernel handle valid for the context (released by qdpx_free_all /
 *   qdpx_destroy).  Not for a capturing stream (it may compile and loads a
 *   module).  EINVAL with the reason for a malformed expression.
 * qdpx_jit_info: whether the kernel came from the cache, and its source.
 * qdpx_jit_eval: out(x) = the expression at every site, fields and links in
 *   the layout of qdpx_pack_* (prec/fmt of the compile call); fields: host
 *   array of n_fields device pointers; scalars: host array of n_scalars
 *   doubles (passed in the field precision).  out must not overlap U or any
 *   field.  norm2 (nullable, device double) receives |out|^2 in FP64 (fixed
 *   order; then work >= qdpx_workspace_bytes(QDPX_OP_SHIFT, ...)).  One site
 *   per thread, 256 threads per block; enqueues only, so it can be captured. */
int qdpx_jit_generate(const char *expr, qdpx_prec prec, qdpx_linkfmt fmt, int32_t n_fields, int32_t n_scalars,
                      char *buf, size_t buf_bytes, size_t *needed);
int qdpx_jit_compile(qdpx_ctx *ctx, const char *expr, qdpx_prec prec, qdpx_linkfmt fmt, int32_t n_fields,
                     int32_t n_scalars, int32_t *kernel);
int qdpx_jit_info(qdpx_ctx *ctx, int32_t kernel, int32_t *from_cache, char *buf, size_t buf_bytes);
int qdpx_jit_eval(qdpx_ctx *ctx, int32_t kernel, const qdpx_geom *geom, const void *U, const void *const *fields,
                  const double *scalars, void *out, double *norm2, void *work, size_t work_bytes, void *stream);

/* -------------------------------------------------------------- autotuner
 * Time the candidate launch geometries of operation `op` (QDPX_OP_APE,
 * QDPX_OP_SHIFT, QDPX_OP_CHAIN or QDPX_OP_JACOBI) on `geom` and remember the
 * fastest in the context: threads per block, consecutive 64-site groups per
 * wave, the block order over the 8 XCDs (xcd_map 0: dispatch order; 1: each
 * XCD a contiguous range of groups; 2: each XCD a slab of z planes walked t
 * plane by t plane, used where the groups of a t plane split evenly over the
 * XCDs, else order 0), the number of t planes walked together, and the LDS
 * tile of the FP32 APE step with the Gram-Schmidt projection (lds_tile 0:
 * every link loaded through the caches; 1: each 64-site group's own links,
 * rows 0 and 1, staged in LDS once for the four direction waves; 2: also
 * every site's backward links U_mu(x-mu), columns 0 and 1, which the lower
 * staples of the other three directions read; 3: also the plane products
 * U_mu(x+nu) U_nu(x+mu)^dag, which the upper staples of U_mu(x) and U_nu(x)
 * share, formed by one of the two direction waves and passed to the other
 * through LDS; 4: the own links and the plane products, the backward links
 * loaded; 0 in every other case: the FP64 step always exchanges backward
 * links through LDS, and the shift, hop and chain kernels meet their
 * per-direction partial sums there).
 * This is the auto-tuning of the thread geometry the paper proposes
 * (sections 5.4 and 9).  Allocates and frees temporary device buffers and
 * synchronises the device, so it returns QDPX_ECAPTURE on a capturing
 * stream.  Every candidate produces bit-identical results.
 * A context created with a launch table writes the tuned geometry to it.
 * qdpx_tune_get / qdpx_tune_set read and write the remembered choice
 * (every output pointer of qdpx_tune_get is nullable; *source receives 0
 * for the default geometry, 1 for one read from the launch table, 2 for one
 * qdpx_tune found, 3 for one qdpx_tune_set gave; a launch table written
 * without lds_tile gives the default, 4 for the FP32 APE step, else 0);
 * t_window must divide Lt and only matters when Lx is a multiple of 8 and Ly
 * of 8 (or Lx of 16 and Ly of 4).  For QDPX_OP_BATCHED (tuned by
 * qdpx_tune_batched, which qdpx_tune refuses with QDPX_EUNSUPPORTED) block is
 * 256 or 512 and sites_per_thread is the number of 64-site groups per work
 * ticket, keyed by the first lattice's extents. */
int qdpx_tune(qdpx_ctx *ctx, qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
              void *stream);
int qdpx_tune_get(qdpx_ctx *ctx, qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                  int32_t *block, int32_t *sites_per_thread, int32_t *xcd_map, int32_t *t_window,
                  int32_t *lds_tile, int32_t *source);
int qdpx_tune_set(qdpx_ctx *ctx, qdpx_op op, const qdpx_geom *geom, qdpx_prec prec, qdpx_linkfmt fmt,
                  int32_t block, int32_t sites_per_thread, int32_t xcd_map, int32_t t_window, int32_t lds_tile);
/* The autotuner of the batched call: times it on this batch of extents
 * (n_lat lattices, n_steps steps, temporary links) with 256- and 512-thread
 * blocks (one or two 64-site groups at a time) and 1, 2, 4 or 8 groups per
 * work ticket, and remembers the fastest for QDPX_OP_BATCHED under the first
 * lattice's extents (written to the context's launch table, if any).
 * Allocates, synchronises, and returns QDPX_ECAPTURE on a capturing stream. */
int qdpx_tune_batched(qdpx_ctx *ctx, int n_lat, const qdpx_geom *geoms, qdpx_prec prec, qdpx_linkfmt fmt,
                      int n_steps, void *stream);

/* Write every geometry the context read, tuned or was given into the
 * launch-table file `path` (NULL: the context's own table), merged with the
 * entries the file already holds for other shapes; the file is replaced
 * atomically.  Host only, no device work.  QDPX_EINVAL if there is no path or
 * the file cannot be read or written. */
int qdpx_tune_save(qdpx_ctx *ctx, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* QDPX_H */
