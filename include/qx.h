/*
 * qx.h -- C ABI of libqx.so: the staggered Dirac operator (Dslash), the
 * even-odd preconditioned conjugate-gradient solve of (m^2 - D_eo D_oe) x = b
 * and the fermion force, on AMD Instinct MI355X (gfx950).
 *
 * The paper (Sec. 4) describes a lattice framework whose hot path is a
 * staggered Dirac operator on SU(N) links (Sec. 1: a 4-D grid with one SU(3)
 * matrix per link) inside single- and double-precision conjugate-gradient
 * solvers, and hybrid Monte Carlo (which needs the fermion force).  The paper
 * gives no formulas; this library implements the textbook Kogut-Susskind
 * operator
 *
 *   (D chi)(x) = 1/2 sum_mu eta_mu(x) [ bc_mu(x) U_mu(x) chi(x+mu)
 *                                      - bc_mu(x-mu) U_mu(x-mu)^dag chi(x-mu) ]
 *   eta_mu(x)  = (-1)^(x_0 + ... + x_{mu-1}),  mu = 0..3 = x, y, z, t,
 *   bc_mu(x)   = -1 for mu = 3, x_3 = L_3 - 1 if QX_BC_T_ANTIPERIODIC, else +1,
 *
 * periodic in all directions, and the Hermitian positive-definite even-site
 * operator A = m^2 - D_eo D_oe (= M^dag M on even sites for M = m + D).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Status: every call returns QX_OK (0) or a QX_E* code; the message of the
 *    last failure on the calling thread is returned by qx_last_error().  No
 *    C++ exception crosses this boundary.
 *  - Memory: the caller owns every device buffer (gauge fields, packed fields,
 *    workspaces, outputs) and passes plain device pointers; the sizes come
 *    from the qx_*_bytes queries.  The library owns only small host handles
 *    and, for solver/batch handles, a few hundred bytes of device metadata
 *    that it frees in the matching destroy call.  Handles are not safe for
 *    concurrent use from several threads.
 *  - Streams: all device work is enqueued on the hipStream_t passed in
 *    (0 = the legacy default stream).  Calls that return host results (solver
 *    statistics, the action, the unitarity check) synchronise that stream
 *    before they return; all others are asynchronous.
 *  - Lattice: dims[4] = (L_x, L_y, L_z, L_t), every extent even and >= 2,
 *    V = L_x L_y L_z L_t < 2^31.  Lexicographic site order
 *    lex = x + L_x (y + L_y (z + L_z t)); parity = (x+y+z+t) mod 2;
 *    checkerboard index cb = lex >> 1; even-odd index eo = parity*V/2 + cb.
 *  - Canonical (caller-facing) layouts, complex = two IEEE doubles (re, im):
 *      gauge field   complex128 [4][V][3][3]   (mu, lex, row, column)
 *      half field    complex128 [nrhs][V/2][3] (source, cb, colour), one parity
 *      link gradient complex128 [4][V][3][3]
 *  - Packed (internal, device) layouts are opaque byte buffers produced by the
 *    pack calls; their sizes come from qx_gauge_bytes / qx_field_bytes.
 *  - Device buffers (packed, canonical, workspaces) are read and written with
 *    16-byte accesses: pass 16-byte aligned pointers (hipMalloc and PyTorch
 *    allocations are 256-byte aligned).
 */
#ifndef QX_H
#define QX_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QX_VERSION 1

/* status codes */
enum {
  QX_OK = 0,
  QX_EINVAL = 1,        /* bad argument (shape, pointer, enum, odd extent) */
  QX_ENOMEM = 2,        /* caller workspace too small, or host allocation failed */
  QX_EHIP = 3,          /* a HIP runtime call failed (message in qx_last_error) */
  QX_ENOTUNITARY = 4,   /* 12-real link compression asked for non-SU(3) links */
  QX_ENOTCONVERGED = 5, /* max_iter reached before the tolerance */
  QX_EBREAKDOWN = 6,    /* <p, A p> <= 0 or non-finite (e.g. NaN/Inf in the input) */
  QX_ENOLIB = 7         /* no usable gfx950 device */
};

/* lattice flags */
enum { QX_BC_T_ANTIPERIODIC = 1 };

/* Storage precision of packed fields.  QX_PREC_F16 (storage below the
   single and double precision the paper measures, Sec. 4): links as IEEE
   binary16 pairs (each part its FP64 value rounded once to nearest, ties to
   even); colour vectors as binary16 pairs scaled per site by one
   FP32 number, the largest |re| or |im| of the site's three colours (16 bytes
   per site and source); every arithmetic step in FP32.  F16 handles and
   fields serve qx_field_pack / qx_field_unpack, qx_dslash, qx_apply_A and the
   launch-shape calls; an F16 gauge handle also serves as the inner handle
   (glo) of a mixed solve, force, molecular-dynamics or meson call, whose
   inner vectors stay FP32.  The FP64 handle of those calls rejects it. */
enum { QX_PREC_F64 = 0, QX_PREC_F32 = 1, QX_PREC_F16 = 2 };

/* link storage: 18 reals, or 12 reals (rows 0-1, row 2 rebuilt in-kernel as
   sign * conj(row0 x row1); exact for SU(3) links) */
/* Link storage.  QX_RECON_NAIK: the improved operator of the paper's
   benchmark "with the Naik term" (Sec. 4): the one-hop term scaled by 9/8 plus
   the three-hop term  -1/24 [N_mu(x) chi(x+3mu) - N_mu(x-3mu)^dag chi(x-3mu)],
   N_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu) with eta and the boundary signs,
   thin links in both terms; 18 reals for each of the two link sets (1146
   flops per output site per half-Dslash).  Every operator and solver call
   takes it; the fermion-force calls reject it. */
enum { QX_RECON_18 = 18, QX_RECON_12 = 12, QX_RECON_NAIK = 36 };

/* solver modes */
enum {
  QX_CG_FP64 = 0,      /* all vectors, links and dot products in FP64 */
  QX_CG_MIXED_F32 = 1  /* FP32 inner iteration, FP64 reliable updates, solution and dots */
};

typedef struct qx_lattice qx_lattice_t;
typedef struct qx_gauge qx_gauge_t;
typedef struct qx_batch qx_batch_t;

/* engines of the CG iteration */
enum {
  QX_ENGINE_AUTO = 0,       /* when every system of the batch has at most 1024 stencil blocks
                               (V/2 <= 65536): QX_ENGINE_FUSED2 if also every system has at
                               most 3 sources and 4 * sources * blocks <= 4096, else
                               QX_ENGINE_FUSED; otherwise QX_ENGINE_LAUNCH */
  QX_ENGINE_LAUNCH = 1,     /* six kernel launches per iteration, five per reliable update
                               (graph-captured in chunks) */
  QX_ENGINE_PERSISTENT = 2, /* one cooperative launch runs many iterations with grid barriers;
                               slower on MI355X, where every barrier costs each block an
                               agent-scope release (L2 writeback) */
  QX_ENGINE_FUSED = 3,      /* three launches per iteration, three per reliable update: the
                               reductions are finished redundantly by every block of the
                               next pass (cheap while partials per source are few) */
  QX_ENGINE_FUSED2 = 4      /* as QX_ENGINE_FUSED with two launches per iteration: the D_eo
                               pass also sums Re<r, Ap>, |Ap|^2 and |r|^2, so the next D_oe
                               pass takes the alpha step, updates x and r and gets the new
                               |r|^2 as |r|^2 - 2 alpha Re<r, Ap> + alpha^2 |Ap|^2 without a
                               pass of its own; a reliable update inside a chunk is two
                               launches, its last step taken by the next D_oe pass; same
                               mathematics, different rounding */
  /* LAUNCH, PERSISTENT and FUSED give the same results bit for bit */
};

/* Solver parameters.  tol: relative residual |b - A x| / |b| to reach, measured
   in FP64 on the returned x.  max_iter: cap on inner iterations per source.
   delta: reliable-update trigger, an update happens when |r| < delta * max|r|
   since the last update (ignored by QX_CG_FP64, which updates only to confirm
   convergence).  use_x0: x holds an initial guess on entry.  chunk: inner
   iterations enqueued between host convergence checks (0 = default).
   engine: QX_ENGINE_*. */
typedef struct {
  double tol;
  int max_iter;
  int mode;
  double delta;
  int use_x0;
  int chunk;
  int engine;
} qx_cg_params_t;

/* Per-source solver statistics. */
typedef struct {
  int status;               /* QX_OK, QX_ENOTCONVERGED or QX_EBREAKDOWN */
  int iters;                /* inner iterations */
  int reliable_updates;     /* FP64 residual recomputations, including the final one */
  double true_rel_residual; /* FP64 |b - A x| / |b| of the returned x, as computed on the GPU */
  double seconds;           /* wall time of the whole call */
} qx_cg_stats_t;

/* ------------------------------------------------------------------ misc */

int qx_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* qx_last_error(void);

/* ------------------------------------------------------------- lattice */

/* Create a lattice description (host only): the 4-D grid of sites with one
   SU(3) matrix per link (Sec. 1).  flags: QX_BC_T_ANTIPERIODIC or 0.
   QX_EINVAL for an odd extent, an extent < 2 or V >= 2^31. */
int qx_lattice_create(const int32_t dims[4], uint32_t flags, qx_lattice_t** out);
int qx_lattice_destroy(qx_lattice_t* lat);
/* Number of sites V, or -1 for a NULL handle. */
int64_t qx_lattice_volume(const qx_lattice_t* lat);

/* Geometry of the 4-D grid (Sec. 1; the even-odd split is this library's
   reading).  Copy the even-odd index maps computed by the device geometry code into
   device buffers: lex_of_eo[V] (int32) and nbr_eo[V][8] (int32; entry k < 4
   is the eo index of x + mu_k, entry 4 + k that of x - mu_k, periodic wrap).
   Exists so that tests can check the on-the-fly neighbour arithmetic of the
   Dslash kernels bit for bit. */
int qx_debug_index_maps(const qx_lattice_t* lat, int32_t* lex_of_eo, int32_t* nbr_eo,
                        hipStream_t stream);

/* ---------------------------------------------------------- gauge field */

/* Bytes of a packed gauge field of the given precision and link storage. */
int qx_gauge_bytes(const qx_lattice_t* lat, int prec, int recon, size_t* bytes);

/* SU(N) gauge field, N = 3 (Sec. 4; one matrix per link, Sec. 1).
   Pack the canonical complex128 [4][V][3][3] gauge field U_canon (device) into
   `packed` (device, qx_gauge_bytes long, owned by the caller and borrowed by
   the handle, which must not outlive it).  The staggered phase eta and the
   boundary sign are folded into the packed links.  With QX_RECON_12 the call
   synchronises the stream and checks that every link is in SU(3): rows 0 and
   1 orthonormal and row2 = conj(row0 x row1), each to 1e-10, every element
   finite (returns QX_ENOTUNITARY otherwise). */
int qx_gauge_load(const qx_lattice_t* lat, const void* U_canon, int prec, int recon, void* packed,
                  hipStream_t stream, qx_gauge_t** out);
int qx_gauge_destroy(qx_gauge_t* g);

/* ------------------------------------------------------------ fields */

/* Bytes of a packed half-lattice field holding nrhs sources. */
int qx_field_bytes(const qx_lattice_t* lat, int nrhs, int prec, size_t* bytes);

/* canonical complex128 [nrhs][V/2][3] <-> packed (device buffers). */
int qx_field_pack(const qx_lattice_t* lat, int nrhs, int prec, const void* canon, void* packed,
                  hipStream_t stream);
int qx_field_unpack(const qx_lattice_t* lat, int nrhs, int prec, const void* packed, void* canon,
                    hipStream_t stream);

/* ---------------------------------------------------------- operators */

/* The staggered Dirac operator on SU(N) links (Sec. 4), half of it: the
   hops from one parity to the other.
   out = D in, from parity 1 - out_parity to parity out_parity, with the factor
   1/2, for nrhs sources at once (each link is loaded once per site and applied
   to every source).  in/out are packed fields of the gauge handle's precision;
   they must not alias. */
int qx_dslash(const qx_gauge_t* g, int out_parity, int nrhs, const void* in, void* out,
              hipStream_t stream);

/* The even-site operator of the conjugate-gradient solver of the staggered
   Dirac matrix (Sec. 4): A = m^2 - D_eo D_oe, Hermitian positive definite.
   out = (m_s^2 - D_eo D_oe) in for each source s on even sites; masses is a
   host array of nrhs values; tmp_odd is a packed odd field of nrhs sources
   used as scratch.  Buffers must not alias. */
int qx_apply_A(const qx_gauge_t* g, int nrhs, const double* masses, const void* in, void* out,
               void* tmp_odd, hipStream_t stream);

/* qx_apply_A without the tmp_odd workspace, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc): the odd intermediate lives in a device array of the
   library (32 MiB, one per GPU, held until the process ends), so the call
   allocates nothing.  It needs nrhs * qx_field_bytes(lat, 1, prec) <= 32 MiB
   (else QX_EINVAL; e.g. FP64 16^4: 20 sources, FP32 32^4: 2 sources).  Same
   kernels and results as qx_apply_A.  Calls on one GPU share the array: calls
   that overlap in time on one GPU (other streams or threads) race. */
int qx_apply_A_noalloc(const qx_gauge_t* g, int nrhs, const double* masses, const void* in,
                       void* out, hipStream_t stream);

/* ------------------------------------------------------------- solver */

/* Workspace bytes for qx_cg_solve with nrhs sources. */
int qx_cg_workspace_bytes(const qx_lattice_t* lat, const qx_cg_params_t* params, int nrhs,
                          size_t* bytes);

/* The conjugate-gradient solve of the staggered Dirac matrix in single and
   double precision (Sec. 4): plain FP64 CG, or FP32 inner iterations with
   FP64 reliable updates (this library's reading of the single-precision
   solver at a double-precision residual).
   Solve (m_s^2 - D_eo D_oe) x_s = b_s for s < nrhs, every source with its own
   CG recurrence (no block Krylov).  g64: FP64 gauge handle (reliable updates
   and the final residual); glo: the inner-precision handle for
   QX_CG_MIXED_F32 (FP32 links, 18 or 12 reals, or FP16 links: the inner
   iterations then load binary16 links and keep FP32 vectors and arithmetic)
   or NULL for QX_CG_FP64.
   b, x: canonical complex128 [nrhs][V/2][3] device buffers (x holds the
   initial guess on entry if params->use_x0).  ws: device workspace of at
   least qx_cg_workspace_bytes.  stats: host array of nrhs entries.
   Synchronises the stream.  Returns QX_OK if every source converged, else the
   first failing source's status (the others are still solved and reported). */
int qx_cg_solve(const qx_gauge_t* g64, const qx_gauge_t* glo, const qx_cg_params_t* params,
                int nrhs, const double* masses, const void* b, void* x, void* ws,
                size_t ws_bytes, qx_cg_stats_t* stats, hipStream_t stream);

/* ------------------------------------------------------------- batches */

/* One system of a batch: a lattice with its gauge handles (g64 FP64, glo the
   inner precision or NULL for QX_CG_FP64), nrhs sources with their masses
   (host array, copied at create), and canonical b / x device buffers. */
typedef struct {
  const qx_gauge_t* g64;
  const qx_gauge_t* glo;
  int nrhs;
  const double* masses;
  const void* b;
  void* x;
} qx_system_t;

/* Workspace bytes for a batch of systems. */
int qx_batch_workspace_bytes(int nsys, const qx_system_t* systems, const qx_cg_params_t* params,
                             size_t* bytes);

/* Many solves of the conjugate-gradient solver (Sec. 4) at once (this
   library's batching of systems and sources; the paper measures one right-hand
   side).  Plan a batch: every system (any mix of lattice sizes) is solved by one set
   of launches per CG step that covers all systems, converged sources are
   masked out, and the launch sequence of a chunk of iterations is captured
   once into a HIP graph that qx_batch_solve replays.  ws must stay valid and
   unchanged in size for the life of the batch. */
int qx_batch_create(int nsys, const qx_system_t* systems, const qx_cg_params_t* params, void* ws,
                    size_t ws_bytes, hipStream_t stream, qx_batch_t** out);

/* Solve every system of the batch; stats: host array with one entry per
   source, systems in order.  Synchronises the stream. */
int qx_batch_solve(qx_batch_t* batch, qx_cg_stats_t* stats, hipStream_t stream);

/* Launch-shape tuner of a batch: times `nchunks` (1..64) chunks of its solve
   (after one untimed chunk) under every launch shape (sources per thread,
   wavefronts per site, block order) the batch admits, and keeps the fastest
   for every later solve of the batch; writes it to *nbt, *lps, *order (each
   may be NULL).  The Dslash tuner times the stencil kernel alone; the
   solver's passes read what the previous pass wrote, so their best shape can
   differ.  A solve's result depends on the shape only through the rounding
   order of the hop sums.  Under the launch-per-pass engine it then times the
   D_eo pass under other (sources per thread, wavefronts per site) beside the
   best shape and keeps one that makes the chunks faster
   (qx_batch_get_launch reports it).  Uses the batch's workspace, never writes
   the systems' x, synchronises the stream.  QX_EINVAL for a NULL batch,
   nchunks outside 1..64 or the persistent engine. */
int qx_batch_tune(qx_batch_t* batch, int nchunks, int* nbt, int* lps, int* order,
                  hipStream_t stream);

/* Set the launch shape of a batch's solver kernels (as qx_batch_tune would
   after finding it), e.g. to repeat a tuned solve or a measurement under the
   same shape.  Synchronises the stream.  QX_EINVAL for a shape the batch
   cannot launch or the persistent engine. */
int qx_batch_set_launch(qx_batch_t* batch, int nbt, int lps, int order, hipStream_t stream);

/* The launch shape a batch's solver runs under: *nbt, *lps, *order for every
   stencil pass, and *deo_nbt, *deo_lps for the launch-per-pass engine's D_eo
   pass (equal to *nbt, *lps unless qx_batch_tune or qx_batch_set_deo_launch
   chose otherwise; the other engines ignore them).  Any pointer may be NULL.
   QX_EINVAL for a NULL batch. */
int qx_batch_get_launch(qx_batch_t* batch, int* nbt, int* lps, int* order, int* deo_nbt,
                        int* deo_lps);

/* Run the launch-per-pass engine's D_eo pass with deo_nbt sources per thread
   and deo_lps wavefronts per site (the block order stays the batch's), e.g.
   to repeat a tuned solve; qx_batch_set_launch resets it.  Results depend on
   it only through the rounding order of the hop sums.  Synchronises the
   stream.  QX_EINVAL for a shape the batch cannot launch or an engine other
   than the launch-per-pass one. */
int qx_batch_set_deo_launch(qx_batch_t* batch, int deo_nbt, int deo_lps, hipStream_t stream);

/* Pass kinds of the solver's launches (qx_batch_profile): the p update
   p = r + beta p, the half-Dslash D_oe (t = D_oe p, with whatever the engine
   fuses into it), the half-Dslash D_eo with the A epilogue and the <p, A p>
   partial sums, the x/r update with the |r|^2 partial sums, the finalize
   kernels of alpha and beta, and every launch of a reliable update. */
enum {
  QX_PASS_P = 0,
  QX_PASS_DOE = 1,
  QX_PASS_DEO = 2,
  QX_PASS_XR = 3,
  QX_PASS_FINALIZE = 4,
  QX_PASS_UPDATE = 5,
  QX_NPASS = 6
};

/* Event timing of one pass kind: launches, those that had work (the host saw
   at least one source in the pass's phase when it enqueued them), the sum over
   those of the number of such sources, and the summed event-to-event
   durations (ms) of all and of the working launches. */
typedef struct {
  int launches;
  int active_launches;
  long long source_launches;
  double ms;
  double active_ms;
} qx_pass_stats_t;

/* Measurement of a batch's solve, pass by pass (for benchmarks and
   profilers): runs the start of the solve and `nchunks` (1..64) chunks of its
   inner iterations with the launch sequence qx_batch_solve replays, but
   enqueued eagerly, with a HIP event recorded on the stream before and after
   every launch, and the host reading the source states before each iteration
   and each reliable-update slot to count the sources it serves.  passes: host
   array of QX_NPASS entries (indexed by QX_PASS_*); stats (nullable): the
   states after the last chunk (seconds = 0).  The systems' x are not written;
   synchronises the stream.  QX_EINVAL for the persistent engine or a bad
   argument. */
int qx_batch_profile(qx_batch_t* batch, int nchunks, qx_pass_stats_t* passes,
                     qx_cg_stats_t* stats, hipStream_t stream);

/* As qx_batch_solve without any host synchronisation (for callers that keep
   enqueueing dependent work): enqueues the start of the solve, exactly
   `nchunks` (>= 1) chunks of inner-iteration slots with their reliable-update
   checks (qx_batch_info gives the chunk length; slots after a source has
   finished do no work for it, so nchunks is an upper bound chosen by the
   caller), the unpacking of every x, and the per-source statistics into
   d_stats, a device array of one qx_cg_stats_t per source (seconds = 0).  A
   source still running after the last chunk reports QX_ENOTCONVERGED and its
   x is the solution of its last reliable update.  Returns QX_OK once the work
   is enqueued; results are valid when the stream reaches its end.  The work
   of two calls on one batch must not overlap (they share the workspace). */
int qx_batch_solve_async(qx_batch_t* batch, int nchunks, qx_cg_stats_t* d_stats,
                         hipStream_t stream);

/* Number of sources (over all systems) and inner-iteration slots per chunk
   (with QX_ENGINE_PERSISTENT a chunk also ends at the first reliable update
   that any source asks for). */
int qx_batch_info(const qx_batch_t* batch, int* nsources, int* chunk);
int qx_batch_destroy(qx_batch_t* batch);

/* -------------------------------------------------------------- force */

/* Fermion force for hybrid Monte Carlo (Sec. 4): the backward of the solve.
   Link gradient of a real function L of the solution x = A^{-1} b, in the
   PyTorch convention for complex tensors (G = dL/dRe U + i dL/dIm U):
   given x and lam = A^{-1} (dL/dRe x + i dL/dIm x) (packed FP64 even fields,
   nrhs sources, summed over sources), with y = D_oe x, nu = D_oe lam,
   W1 = (lam on even, y on odd), W2 = (x on even, nu on odd):
     G_mu(z) = 1/2 eps(z) eta_mu(z) bc_mu(z) sum_s [W1 W1(z+mu)^dag + W2 W2(z+mu)^dag](z)
   with eps = +1 (-1) on even (odd) z.  g64 must be an FP64 handle; tmp_odd
   is scratch for two packed FP64 odd fields of nrhs sources
   (2 * qx_field_bytes).  grad_U: canonical complex128 [4][V][3][3]. */
int qx_force_from_fields(const qx_gauge_t* g64, int nrhs, const void* x_packed,
                         const void* lam_packed, void* tmp_odd, void* grad_U, hipStream_t stream);

/* Workspace bytes for qx_force. */
int qx_force_workspace_bytes(const qx_lattice_t* lat, const qx_cg_params_t* params, int nrhs,
                             size_t* bytes);

/* Fermion force for hybrid Monte Carlo (Sec. 4): the pseudofermion action
   and its link gradient.
   Action S = sum_s phi_s^dag A^{-1} phi_s and its link gradient G (as in
   qx_force_from_fields with lam = x): one solve (params as for qx_cg_solve,
   mass shared by all sources), one extra half-Dslash and one outer-product
   pass.  phi: canonical [nrhs][V/2][3]; x_out (nullable): canonical solution.
   Synchronises the stream. */
int qx_force(const qx_gauge_t* g64, const qx_gauge_t* glo, const qx_cg_params_t* params,
             int nrhs, double mass, const void* phi, void* grad_U, double* S_out, void* x_out,
             void* ws, size_t ws_bytes, qx_cg_stats_t* stats, hipStream_t stream);

/* Backward of the action S = sum_s phi_s^dag A^{-1} phi_s (fermion force, HMC,
   Sec. 4) for a real upstream gradient gS = dL/dS: grad_U = gS * G with G the
   link gradient qx_force returned (grad_U_S), and
   grad_phi = dL/dRe phi + i dL/dIm phi = 2 gS x (A is Hermitian, so
   dS/dphi = 2 A^{-1} phi = 2 x with x the solution qx_force returned).
   Either output may be NULL (its input is then not read); an output may alias
   its input.  Layouts: G, grad_U canonical complex128 [4][V][3][3]; x, grad_phi
   canonical [nrhs][V/2][3] (device).  Asynchronous on the stream; QX_EINVAL
   for a NULL input an output needs or nrhs < 1. */
int qx_action_backward(const qx_lattice_t* lat, int nrhs, double gS, const void* grad_U_S,
                       const void* x, void* grad_U, void* grad_phi, hipStream_t stream);

/* su(3) force along the generators T_a = lambda_a / 2 (Gell-Mann matrices)
   for the left variation U -> exp(i e T_a) U: F^a = Re[i tr(T_a U G^dag)].
   U, G: canonical complex128 [4][V][3][3]; F: double [4][V][8] (device). */
int qx_force_su3(const qx_lattice_t* lat, const void* U_canon, const void* grad_U, double* F,
                 hipStream_t stream);

/* -------------------------------------------------- molecular dynamics */

/* Hybrid Monte Carlo (the paper reports HMC gauge generation as in progress,
   Sec. 4): Wilson plaquette action, pseudofermion action phi^dag A^-1 phi,
   momenta p^a_mu(x) (a = 1..8, P = sum_a p^a lambda_a / 2), Hamiltonian
   H = 1/2 sum p^2 + S_g + S_f, leapfrog integration of
   U <- exp(i eps P) U,  p^a <- p^a - eps F^a,  F^a = d/dw S(exp(i w T_a) U)|_0.
   Layouts (device, FP64): U canonical complex128 [4][V][3][3], p double
   [4][V][8], phi canonical [V/2][3].  ws for the reductions: at least
   qx_md_workspace_bytes (any params) or 8448 bytes. */

/* S_g = beta sum_{x, mu<nu} (1 - Re tr P_munu(x) / 3), written to *S (host).
   Synchronises the stream. */
int qx_gauge_action(const qx_lattice_t* lat, const void* U, double beta, void* ws,
                    size_t ws_bytes, double* S, hipStream_t stream);
/* Link gradient of S_g in the convention of qx_force: G = -(beta/3) A^dag,
   A_mu(x) = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                            + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)].
   accumulate != 0 adds it to G (e.g. to the pseudofermion gradient). */
int qx_gauge_force(const qx_lattice_t* lat, const void* U, double beta, void* G, int accumulate,
                   hipStream_t stream);
/* p^a -= eps F^a, F^a = Re[i tr(T_a U G^dag)] for a link gradient G. */
int qx_md_update_momenta(const qx_lattice_t* lat, const void* U, const void* G, double eps,
                         double* p, hipStream_t stream);
/* U <- exp(i eps sum_a p^a T_a) U (scaling and squaring of a 16-term series). */
int qx_md_update_links(const qx_lattice_t* lat, const double* p, double eps, void* U,
                       hipStream_t stream);
/* K = 1/2 sum p^2 (host).  Synchronises the stream. */
int qx_md_kinetic(const qx_lattice_t* lat, const double* p, void* ws, size_t ws_bytes, double* K,
                  hipStream_t stream);

typedef struct {
  double beta;        /* gauge coupling */
  double mass;        /* staggered mass of the pseudofermion action */
  double eps;         /* step size */
  int nsteps;         /* leapfrog steps (>= 1) */
  qx_cg_params_t cg;  /* solver of the pseudofermion force */
} qx_md_params_t;

int qx_md_workspace_bytes(const qx_lattice_t* lat, const qx_md_params_t* params, size_t* bytes);

/* One leapfrog trajectory of nsteps steps: U and p are advanced in place; the
   gauge handles g64 (FP64) and glo (the inner precision of a mixed solve, or
   NULL; FP32 or FP16 links) must be loaded from U's lattice and are repacked
   from U after every link update.  phi NULL: pure gauge.  Returns H at the start and the end and
   the total CG iterations of the force solves.  One-hop operator only
   (QX_EINVAL for the Naik link storage).  Synchronises the stream. */
int qx_md_trajectory(qx_gauge_t* g64, qx_gauge_t* glo, const qx_md_params_t* params, void* U,
                     double* p, const void* phi, void* ws, size_t ws_bytes, double* H_start,
                     double* H_end, int* cg_iters, hipStream_t stream);

/* -------------------------------------------------------------- mesons */

/* Staggered meson correlators from a point source at the even site src[4]
   (x, y, z, t): per source colour the propagator G = M^-1 delta, M = m + D,
   is m A^-1 b on even sites and -D_oe A^-1 b on odd sites (the three colour
   sources solved together, params as for qx_cg_solve, one mass); then
     C_k(t) = sum_{x with x_t = src_t + t (mod L_t)} s_k(x) sum_{a,c} |G_ac(x)|^2,
     s_k(x) = (-1)^(sum of x_mu over the directions mu set in masks[k] (bit mu)),
   mask 0 being the Goldstone pion.  The paper lists spectrum measurements
   among the framework's uses (Sec. 4).  C: host [nmask][L_t], 1 <= nmask <= 16;
   stats: host array of 3.  QX_EINVAL for an odd source site.  Synchronises. */
int qx_meson_workspace_bytes(const qx_lattice_t* lat, const qx_cg_params_t* params,
                             size_t* bytes);
int qx_meson_correlators(const qx_gauge_t* g64, const qx_gauge_t* glo, const qx_cg_params_t* params,
                         double mass, const int src[4], int nmask, const int* masks, double* C,
                         void* ws, size_t ws_bytes, qx_cg_stats_t* stats, hipStream_t stream);

/* ------------------------------------------------------------- tuning */

/* Pick the launch shape of the stencil kernels for this gauge handle and nrhs
   sources by timing every candidate (20 launches replayed from a HIP graph on
   a private stream that waits for `stream`).  A stencil block covers 64
   sites with lps * groups wavefronts: lps (1, 2, 4, 8) wavefronts share the
   eight hops of each site (more loads in flight on small lattices), and each
   of the groups = ceil(nrhs / nbt) takes nbt (1, 2, 4; 6 and 12 for FP32
   one-hop links) sources, every link applied to all of the wavefront's
   sources.  With one wavefront per site and two or more groups the groups
   share the tile's link loads through LDS (FP32 and FP64 handles with up to
   64 KB of one-hop links per tile: not FP64 18-real links, not the improved
   operator, not F16 handles); otherwise each wavefront loads its links.  xcd_order
   is the block order: 0 as dispatched, 1 gives each of the eight XCDs a
   contiguous range of sites, 2 and 3 do the same and walk the (z, t) planes
   in tiles of 2 x 8 and 4 x 4 planes (when Lh * L1 is a multiple of 64),
   which keeps the colour vectors of many sources in L2 between their uses;
   4 and 5 give each XCD a slab of z or t planes, walked plane by plane, with
   non-temporal output stores.  scratch: two
   packed fields of nrhs sources of the handle's precision
   (2 * qx_field_bytes).  The result is used by every later call with this
   handle and nrhs (Dslash, A and the solvers) and cached per (lattice,
   precision, link storage, nrhs) in the process and in the JSON file named by
   QX_TUNE_CACHE if set.  Synchronises the stream. */
int qx_tune_dslash(const qx_gauge_t* g, int nrhs, void* scratch, hipStream_t stream);

/* The process-wide launch-shape cache that qx_tune_dslash fills (keys: device,
   lattice extents, precision, link storage, source count; values: nbt, lps,
   xcd_order), as the flat JSON object {"key": [nbt, lps, xcd_order], ...}.
   qx_tune_cache_load merges the entries of the file at `path` into it (an
   entry replaces the one of the same key; malformed entries and shapes that
   are not compiled are skipped; QX_EINVAL if the file cannot be read);
   qx_tune_cache_save writes the whole cache to `path` (QX_EINVAL if it cannot
   be written).  Handles use a cached shape for every (handle, nrhs) that has
   not been tuned or set on the handle itself.  Host only, no device work. */
int qx_tune_cache_load(const char* path);
int qx_tune_cache_save(const char* path);

/* Average device time, in ms, of one half-Dslash launch (as qx_dslash, with
   the handle's launch shape for nrhs): `reps` (1..10000) launches are captured
   into a HIP graph on a private stream that first waits for `stream`; the graph
   is replayed once untimed and once between two HIP events on that stream, so
   the figure holds kernel time and the dispatch gaps between dependent
   kernels, not the host's launch rate.  Writes `out`; synchronises. */
int qx_time_dslash(const qx_gauge_t* g, int out_parity, int nrhs, const void* in, void* out,
                   int reps, double* avg_ms, hipStream_t stream);

/* Launch shape currently used for (handle, nrhs). */
int qx_get_launch(const qx_gauge_t* g, int nrhs, int* nbt, int* lps, int* xcd_order);
/* Force a launch shape; QX_EINVAL if it is not one of the compiled shapes or
   does not fit one block. */
int qx_set_launch(const qx_gauge_t* g, int nrhs, int nbt, int lps, int xcd_order);

/* ------------------------------------------------------------- probe */

/* dst = src (device buffers, bytes a multiple of 16) with a plain streaming
   kernel: the measured-bandwidth reference for the roofline figures and the
   calibration kernel for hardware memory counters.  Asynchronous. */
int qx_probe_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

/* Read `bytes` (a multiple of 16) of src once with a plain streaming kernel:
   the measured read bandwidth, the reference for read-dominated kernels such
   as the Dslash.  scratch: 32 KiB of device memory.  Asynchronous. */
int qx_probe_read(const void* src, size_t bytes, void* scratch, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* QX_H */
