/*
 * mspcg.h -- C ABI of the MI355X library for the multi-splitting
 * preconditioned conjugate gradient (MSPCG) solve of the even-odd
 * preconditioned Mobius domain-wall normal equations (arxiv 2104.05615).
 *
 * The library solves  D^dag D x = b  on the even checkerboard, with
 *   D = 1 - M5^-1 M4_eo M5^-1 M4_oe,   M4 = D^w M_phi          (Sec. 2.2)
 * by preconditioned CG (Alg. 1, Sec. 2.4) with Polak-Ribiere beta and
 * reliable updates (Sec. 3.2), preconditioned by a fixed number of CG
 * iterations on the local operator A_s of every subdomain, Dirichlet
 * boundary on the whole four-hop operator so that snake terms are kept
 * (Sec. 2.3-2.5).  Subdomains are virtual: they tile one GPU.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Every call returns an mspcg_status; 0 is success.  Nothing aborts or
 *   throws across the ABI.  mspcg_last_error() gives a message for the last
 *   non-OK status returned on the calling thread.
 * - Host layouts (FP64, complex interleaved re, im):
 *     gauge field   U[T][Z][Y][X][mu][3][3], mu = 0..3 for x, y, z, t;
 *                   U[x][mu] is the SU(3) link from x to x + mu_hat.
 *     5D field      psi[Ls][V/2][4][3] on the sites of one parity, ordered
 *                   by lex/2 with lex = x + X*(y + Y*(z + Z*t)); spins in the
 *                   chiral basis gamma_5 = diag(1, 1, -1, -1); P+ = spins 0,1.
 *   Boundary conditions are periodic in all four directions.
 * - Ownership: the handle owns every device copy and workspace it allocates.
 *   The caller owns every buffer it passes in; the library never keeps a
 *   caller pointer after a call returns.  Device pointers passed to the
 *   *_device entry points are used in stream order on the given HIP stream
 *   (NULL = the handle's own stream); the call returns after the work is
 *   enqueued unless noted.
 * - State: set_mobius, load_gauge and set_subdomains invalidate derived state
 *   (tables, workspaces).  Calls that need state that is missing return
 *   MSPCG_ERR_NO_GAUGE / MSPCG_ERR_NO_PARAMS / MSPCG_ERR_BAD_TILING.
 * - A handle is not thread safe: one handle per thread or an external lock.
 */
#ifndef MSPCG_H
#define MSPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mspcg_ctx* mspcg_t;

typedef enum {
  MSPCG_OK = 0,
  MSPCG_NOT_CONVERGED = 1,     /* result and stats are filled in */
  MSPCG_BUSY = 2,              /* mspcg_cb_submit: every slot is taken (nothing was queued) */
  MSPCG_ERR_INVALID_ARG = -1,
  MSPCG_ERR_BAD_TILING = -2,
  MSPCG_ERR_NO_GAUGE = -3,
  MSPCG_ERR_NO_PARAMS = -4,
  MSPCG_ERR_OOM = -5,
  MSPCG_ERR_HIP = -6,
  MSPCG_ERR_BREAKDOWN = -7     /* NaN/Inf or a non-positive curvature in a reduction */
} mspcg_status;

/* Storage precisions.  FP16, BF16 and INT8 store the 24 reals of each 5D
 * site (one colour-spinor) with one FP32 scale per site, the scaled storage
 * of Sec. 3.2 (value = stored number / limit x scale):
 *   FP16, BF16  the reals divided by their largest magnitude m, rounded to
 *               nearest-even in the 16-bit float format; scale m;
 *   INT8        the integers q = round-half-even(v x (127 / m)) in
 *               [-127, 127], the product formed in FP32; scale m / 127.
 * A site of zeros stores zeros with scale 0.  Arithmetic is FP32. */
typedef enum { MSPCG_FP64 = 0, MSPCG_FP32 = 1, MSPCG_FP16 = 2, MSPCG_BF16 = 3, MSPCG_INT8 = 4 } mspcg_prec;

/* Operators exposed by mspcg_apply (each runs the same kernels the solver runs). */
typedef enum {
  MSPCG_OP_DSLASH_EO = 0,     /* D^w from odd to even sites (Sec. 2.2, def. of D^w)            */
  MSPCG_OP_DSLASH_OE = 1,     /* D^w from even to odd sites                                     */
  MSPCG_OP_DSLASH_DAG_EO = 2, /* (D^w)^dag from odd to even                                      */
  MSPCG_OP_DSLASH_DAG_OE = 3, /* (D^w)^dag from even to odd                                      */
  MSPCG_OP_M5 = 4,            /* M5 = (b(4-M5)+1) + (c(4-M5)-1) P~, diagonal in 4D              */
  MSPCG_OP_M5INV = 5,         /* M5^-1                                                          */
  MSPCG_OP_MPHI = 6,          /* M_phi = -(b + c P~)/2, so that M4 = D^w M_phi                  */
  MSPCG_OP_D = 7,             /* D = 1 - M5^-1 M4_eo M5^-1 M4_oe (eq. dirac_equation), even      */
  MSPCG_OP_DDAG = 8,          /* D^dag, even                                                     */
  MSPCG_OP_A = 9,             /* A = D^dag D (eq. normal_equation), even                         */
  MSPCG_OP_A_SUB = 10,        /* (+)_s A_s, A_s = R_s A R_s^T with snake terms (eq. diri), even   */
  MSPCG_OP_PRECOND = 11,      /* z = (+)_s CG_k(A_s, r_s), k = inner_iters (Sec. 2.4-2.5), even, or the
                                 reduced-Ls z = (T^dag Mhat^-1 T + mu) r when one is set (Sec. 3.3)  */
  MSPCG_OP_STORE = 12         /* the input stored in the given precision and read back (Sec. 3.2) */
} mspcg_op;

typedef struct {
  double tol;             /* stop at ||b - A x|| / ||b|| <= tol (true residual, FP64)            */
  int32_t maxiter;        /* outer iterations                                                     */
  int32_t inner_iters;    /* k: fixed inner CG iterations per preconditioner application          */
  mspcg_prec inner_prec;  /* storage of the inner CG: FP64, FP32, FP16, BF16 or INT8 (FP32 arithmetic) */
  mspcg_prec outer_prec;  /* outer PCG: FP64 or FP32 (FP32 uses FP64 reliable updates)            */
  double reliable_delta;  /* reliable update when ||r|| < delta * max ||r|| since the last one     */
  int32_t beta_rule;      /* 0 = Polak-Ribiere (Sec. 3.2), 1 = Fletcher-Reeves (Alg. 1)            */
  int32_t use_precond;    /* 0 = plain CG (M = 1), 1 = MSPCG                                       */
} mspcg_solver_params;

typedef struct {
  int32_t outer_iters;
  int32_t inner_iters_total;
  int32_t reliable_updates;
  double true_rel_resid;  /* ||b - A x|| / ||b|| in FP64 at exit                                   */
  double iter_rel_resid;  /* iterated residual at exit                                             */
  double ms_total;        /* wall clock of the solve on the device stream                          */
  double ms_precond;      /* part spent in the preconditioner (only when profiling is on)          */
  int32_t status;         /* mspcg_status of this right-hand side                                  */
} mspcg_stats;

/* Create a handle for an X*Y*Z*T lattice on HIP device `device`.  No HIP call
 * is made here; the device is touched by the first call that needs it.
 * Errors: INVALID_ARG if out is NULL, an extent is < 2 or odd, device < 0,
 * the volume is 2^31 sites or more, or the FP64 gauge records (V * 640
 * bytes) reach 4 GiB (see the size limits under mspcg_set_mobius). */
mspcg_status mspcg_create(mspcg_t* out, const int32_t dims[4], int32_t device);

/* Free the handle and everything it owns.  NULL is accepted. */
mspcg_status mspcg_destroy(mspcg_t h);

/* Copy the gauge field (host FP64, layout above; links SU(3), Sec. 2.2) to the
 * device and convert it to the library's FP64 and FP32 link layouts.
 * Errors: INVALID_ARG (NULL), HIP/OOM from the device. */
mspcg_status mspcg_load_gauge(mspcg_t h, const double* U);

/* Mobius parameters of M5 and M_phi (Sec. 2.2 with the Mobius construction the
 * paper cites): fifth-dimension extent Ls >= 2, b, c, domain-wall height M5,
 * quark mass mf.  Errors: INVALID_ARG for Ls < 2 or Ls > 32, a singular M5,
 * or an FP64 5D field (V/2 * Ls * 192 bytes) of 4 GiB or more.
 *
 * Size limits (32-bit addressing of the kernels: buffer ranges and per-lane
 * byte offsets are 32-bit): every array of one right-hand side must stay
 * below 4 GiB -- the FP64 gauge record array (V * 640 bytes, checked by
 * mspcg_create together with V < 2^31), an FP64 5D field (checked here) and
 * the largest subdomain region field, nsub * |N2| * Ls * (192, 96, 48 or 24
 * bytes for FP64, FP32, FP16/BF16, INT8 inner storage; checked by
 * set_subdomains, set_solver and every solve, and by an apply of A_SUB or
 * PRECOND for the precision it names; the other operators use no region
 * field).  A batch of right-hand sides may exceed 4 GiB in total. */
mspcg_status mspcg_set_mobius(mspcg_t h, int32_t Ls, double b, double c, double M5, double mf);

/* Subdomain extents (X, Y, Z, T) of the virtual block decomposition used by the
 * preconditioner (Sec. 2.1, 2.4).  Every extent must be even and divide the
 * lattice extent, and in every partitioned direction (sub < lattice) the
 * lattice must extend at least 4 sites past the subdomain, so that the zero
 * pad of two sites (Sec. 3.1.2) evaluates R_s A R_s^T exactly.
 * Errors: BAD_TILING otherwise. */
mspcg_status mspcg_set_subdomains(mspcg_t h, const int32_t sub[4]);

/* Solver parameters (copied).  Errors: INVALID_ARG for tol <= 0, maxiter < 1,
 * inner_iters < 0, outer_prec not FP64/FP32, an unknown precision or beta rule,
 * or an inner precision whose subdomain region field would reach 4 GiB with
 * the tiling and Ls already set. */
mspcg_status mspcg_set_solver(mspcg_t h, const mspcg_solver_params* p);

/* Solve A x = b (A = D^dag D, eq. normal_equation) for one right-hand side.
 * b, x: host FP64 even fields [Ls][V/2][4][3]; x0 (nullable) is the starting
 * guess (r0 = b - A x0), else 0.  Synchronous.  st (nullable) gets the stats.
 * Returns OK, NOT_CONVERGED (maxiter reached; x is the last iterate),
 * BREAKDOWN (NaN/Inf or <p, A p> <= 0: x is the last iterate whose values are
 * finite -- with FP32 outer precision the solution of the last reliable
 * update when the breaking step is not finite -- and st->true_rel_resid its
 * true residual), NO_GAUGE, NO_PARAMS, BAD_TILING (MSPCG without a tiling).
 * INVALID_ARG when a field would exceed the 32-bit addressing limits (see
 * mspcg_set_mobius). */
mspcg_status mspcg_solve(mspcg_t h, const double* b, double* x, const double* x0, mspcg_stats* st);

/* As mspcg_solve with device FP64 buffers b, x (layout above), x0 nullable.
 * Runs on `hip_stream` (NULL = the handle's stream) and synchronizes it
 * before returning (the convergence test reads the residual on the host). */
mspcg_status mspcg_solve_device(mspcg_t h, const double* b, double* x, const double* x0, void* hip_stream,
                                mspcg_stats* st);

/* Solve the full five-dimensional system M psi = phi on both parities,
 * M = [[M5, M4_eo], [M4_oe, M5]] with M4 = D^w M_phi (Sec. 2.2), through the
 * even-odd Schur complement (eq. dirac_equation): phi^_e = M5^-1 phi_e -
 * M5^-1 M4_eo M5^-1 phi_o; D^dag D psi_e = D^dag phi^_e by the configured
 * solver (as mspcg_solve_device); psi_o = M5^-1 (phi_o - M4_oe psi_e).  The
 * steps outside the solve run in FP64.
 *   phi, psi: device FP64, the even field then the odd field, each of the
 *             layout above (odd sites ordered by lex/2 like even ones).
 *   st: nullable, stats of the even solve; full_rel_resid: nullable, gets
 *   || phi - M psi || / || phi || computed in FP64.
 * Runs on hip_stream (NULL = the handle's stream); returns when done.
 * Returns as mspcg_solve_device. */
mspcg_status mspcg_solve_full_device(mspcg_t h, const double* phi, double* psi, void* hip_stream, mspcg_stats* st,
                                     double* full_rel_resid);

/* Solve A x_r = b_r for nrhs right-hand sides on the loaded gauge field, each
 * by the same PCG as mspcg_solve_device (Alg. 1 with the reliable updates and
 * Polak-Ribiere beta of Sec. 3.2, preconditioner of Sec. 2.4-2.5).  Every
 * kernel of an iteration runs once for all right-hand sides (a hop launch
 * covers every site block of every RHS); the iteration's convergence,
 * reliable-update and breakdown decisions are taken on the device per RHS,
 * a RHS that has stopped drops out of every launch, and two iterations are
 * captured in a HIP graph and replayed without a host round trip (eagerly
 * when profiling is on).  Each RHS gets the result and iteration count the
 * single-RHS solve gives it: same kernels, partitions and reduction orders.
 *   b, x:  device FP64, nrhs fields of the layout above one after another
 *          (RHS r at offset r * Ls * V/2 * 24 doubles);  x0: nullable, same.
 *   st:    nullable, else an array of nrhs stats (status per RHS).
 * Runs on hip_stream (NULL = the handle's stream); returns when done.
 * A RHS that breaks down returns the solution of its last reliable update
 * (its FP32 progress after that is dropped) and its iterated residual at the
 * breakdown as true_rel_resid.
 * Returns BREAKDOWN if any RHS broke down, else NOT_CONVERGED if any did not
 * converge, else OK; INVALID_ARG for nrhs outside [1, 1024] or NULL buffers;
 * NO_GAUGE, NO_PARAMS, BAD_TILING as mspcg_solve. */
mspcg_status mspcg_solve_batch_device(mspcg_t h, int32_t nrhs, const double* b, double* x, const double* x0,
                                      void* hip_stream, mspcg_stats* st);

/* Choose the workgroup schedule of the hop kernels for nrhs right-hand sides
 * by timing the candidates on this handle's lattice, Ls and precisions.  A
 * hop launch runs one workgroup per (site block, RHS); the candidates are
 * the RHS order (RHS outermost, or the RHS of one site block adjacent so that
 * they read its links from one L2) and the XCD mapping (contiguous site-block
 * ranges per XCD, or the hardware's round robin) and, for the full-lattice
 * hops, the order of the site blocks: lexicographic, or time slices swept
 * chunk by chunk (a chunk of a few z-planes and rows, run through every t
 * before the next, so that the +-t neighbour spinors of the blocks in flight
 * are still in the XCD's L2), four chunk sizes.  Kinds: 0 = full-lattice
 * hops in the outer precision, 1 = FP64 hops, 2 = subdomain hops (needs a
 * tiling).  No schedule changes a result: partial sums are indexed by
 * (RHS, site block), not by workgroup.  The choice is kept in the handle
 * until set_mobius / set_subdomains.
 * Errors: INVALID_ARG (nrhs outside [1, 1024]), NO_GAUGE, NO_PARAMS. */
mspcg_status mspcg_autotune(mspcg_t h, int32_t nrhs);

/* The schedule in use for (kind, nrhs): RHS order (0 = RHS outermost, 1 = RHS
 * of a site block adjacent), XCD mapping (1 = contiguous ranges per XCD) and
 * the tuned time of the kind's four hops in microseconds (0 when untuned).
 * Errors: INVALID_ARG for NULL or an unknown kind. */
mspcg_status mspcg_get_schedule(mspcg_t h, int32_t kind, int32_t nrhs, int32_t* order, int32_t* xcd, double* us);

/* Pin the schedule of (kind, nrhs) (extension: lets a caller reuse a tuned
 * schedule or compare schedules): order and xcd as above, tchunk = 0 for the
 * lexicographic block order of the full-lattice hops or 1..4 for the chunked
 * sweep with chunks of about (80 << tchunk) KB of input spinors (falls back
 * to lexicographic when site blocks do not tile whole z-planes; ignored by
 * kind 2).  Results do not depend on it.  Kept until set_mobius /
 * set_subdomains.  mspcg_get_tchunk returns the block order in use (untuned:
 * 3 for the full-lattice kinds, 0 for kind 2).
 * Errors: INVALID_ARG (unknown kind, nrhs outside [1, 1024], order, xcd or
 * tchunk out of range, NULL). */
mspcg_status mspcg_set_schedule(mspcg_t h, int32_t kind, int32_t nrhs, int32_t order, int32_t xcd, int32_t tchunk);
mspcg_status mspcg_get_tchunk(mspcg_t h, int32_t kind, int32_t nrhs, int32_t* tchunk);

/* Apply one operator (mspcg_op) in precision `prec` to a host FP64 field and
 * return the result as host FP64: the input is converted to the storage of
 * `prec`, the operator runs with that storage, the output is converted back.
 * Synchronous.  Errors: INVALID_ARG (op/prec/NULL), NO_GAUGE, NO_PARAMS,
 * BAD_TILING (A_SUB/PRECOND without a tiling). */
mspcg_status mspcg_apply(mspcg_t h, int32_t op, mspcg_prec prec, const double* in, double* out);

/* As mspcg_apply with device FP64 buffers, stream ordered on hip_stream
 * (NULL = the handle's stream); returns once the work is enqueued. */
mspcg_status mspcg_apply_device(mspcg_t h, int32_t op, mspcg_prec prec, const double* in, double* out,
                                void* hip_stream);

/* As mspcg_apply_device, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the call makes no hipMalloc, hipFree or other allocation.
 * Every workspace of the operator (the converted input and output, scratch
 * fields, subdomain region fields, partial sums) is carved from a static
 * device array of 128 MiB that the library holds on each device it runs on
 * until the process ends.  The caller still passes the device FP64 input
 * and output.  All calls on one device share that array and it keeps the
 * last call's contents: calls that overlap in time on one device (on any
 * streams or handles) race and must be serialised by the caller.  The
 * handle must have its gauge field and Mobius parameters set (those calls
 * allocate the handle's own state); profiling is not done inside this call.
 * Errors: as mspcg_apply_device; INVALID_ARG also when the operator's
 * workspace exceeds the static array (e.g. an FP32 A needs about 5 fields of
 * 96 Ls V/2 bytes) or for PRECOND with a reduced-Ls preconditioner set. */
mspcg_status mspcg_apply_device_noalloc(mspcg_t h, int32_t op, mspcg_prec prec, const double* in, double* out,
                                        void* hip_stream);

/* Residual history of the last single-RHS solve on this handle
 * (mspcg_solve / mspcg_solve_device, Alg. 1): out[k] = |r_k| / |b| for
 * k = 0 .. min(max, count) - 1, r_k the iterated residual after k outer
 * iterations (r_0 = b - A x0; before a reliable update replaces it), the
 * quantity the paper plots against the outer iteration (Fig. residual-rbc,
 * Fig. residual-cal).  pap (nullable, max entries): pap[k] = <p_k, A p_k> /
 * |b|^2 of outer iteration k + 1 (0 past the last one); with out they give
 * the CG coefficients alpha_k = |r_k|^2 / <p_k, A p_k> and beta_k =
 * |r_k+1|^2 / |r_k|^2 of a plain CG solve, whose Lanczos matrix estimates
 * the extreme eigenvalues of A.  *count = the number of residuals the solve
 * recorded (outer iterations + 1; 0 for a zero source).  Errors:
 * INVALID_ARG (NULL handle or count, NULL out with max > 0, max < 0). */
mspcg_status mspcg_get_history(mspcg_t h, double* out, double* pap, int32_t max, int32_t* count);

/* Continuous batching (serving extension; the paper's solver is unchanged).
 * A session is a batched solve over `slots` right-hand-side slots of this
 * handle that right-hand sides enter and leave while others iterate: every
 * kernel of an outer iteration runs once for all slots (one launch per
 * operator, masked per slot on the device, the iteration pair captured once
 * in a HIP graph and replayed), and a submitted source starts at the next
 * step with the start-up sequence of Alg. 1 run for the joining slots only.
 * Each slot's arithmetic is independent of the other slots, so its solution
 * and statistics are the same as those of mspcg_solve_batch_device for that
 * source alone.  The solver parameters are those set when the session
 * opens.  While a session is open every other call that uses or changes this
 * handle's state (set_*, solve*, apply*, autotune, ...) returns INVALID_ARG,
 * and mspcg_set_mfma fails for the process.  A handle is not thread-safe:
 * one thread drives its session.
 *
 * mspcg_cb_open   sizes the workspace for `slots` RHS (device memory as
 *                 mspcg_footprint(h, slots)); stream NULL = the handle's.
 * mspcg_cb_submit queues one source: b and x are device FP64 fields of the
 *                 canonical layout; b must stay valid until the slot has
 *                 started (the next step) and x until mspcg_cb_poll reports
 *                 the slot done.  Returns the slot, or MSPCG_BUSY when every
 *                 slot is taken.
 * mspcg_cb_step   starts the pending slots, runs one pair of outer
 *                 iterations for all running slots, and writes x of every
 *                 slot that has finished (converged, breakdown, or the
 *                 iteration limit); returns when that is done, with the
 *                 number of slots still running and still pending.
 * mspcg_cb_poll   done = 1 and the slot's statistics (ms_total: from its
 *                 start to the step that finished it) once it has finished;
 *                 the slot is free again after that call.
 * mspcg_cb_close  ends the session (running slots are abandoned).
 * Errors: INVALID_ARG (no session / one already open / slot out of range /
 * NULL), the errors of mspcg_solve_batch_device. */
mspcg_status mspcg_cb_open(mspcg_t h, int32_t slots, void* hip_stream);
mspcg_status mspcg_cb_submit(mspcg_t h, const double* b, double* x, int32_t* slot);
mspcg_status mspcg_cb_step(mspcg_t h, int32_t* running, int32_t* pending);
mspcg_status mspcg_cb_poll(mspcg_t h, int32_t slot, int32_t* done, mspcg_stats* st);
mspcg_status mspcg_cb_close(mspcg_t h);

/* Kernel timing.  With profiling on, the library brackets every launch of its
 * hop kernels with HIP events on the stream they run on; mspcg_get_kernel_time
 * returns the number of timed launches and their summed duration in ms for a
 * kernel class: 0 = full-lattice hop kernels in FP32/FP16/BF16, 1 = subdomain
 * (inner) hop kernels, 2 = whole preconditioner applications, 3 = full-lattice
 * hop kernels in FP64 (true residuals); or one hop stage of A: 21..24 (full
 * lattice, FP32/16-bit), 31..34 (full lattice, FP64), 11..14 (subdomain hops
 * h1..h4: N1<-C, N2<-N1, N1<-N2, C<-N1).  Counters are reset by set_profiling.
 * on = 1 times every launch; on = N > 1 times one launch in N of each hop
 * stage (every preconditioner application still), so that the average
 * launch time comes from a sample at 1/N of the events' cost; launches then
 * counts the timed ones.  INVALID_ARG for on < 0. */
mspcg_status mspcg_set_profiling(mspcg_t h, int32_t on);
mspcg_status mspcg_get_kernel_time(mspcg_t h, int32_t kind, int64_t* launches, double* ms);

/* Use the device gauge field of `src` in `h` (same lattice extents and
 * device) instead of a copy of its own: the field stays alive while any
 * handle uses it.  For many solver contexts on one resident field.
 * Errors: INVALID_ARG (NULL, extents or device differ), NO_GAUGE (src has
 * none). */
mspcg_status mspcg_share_gauge(mspcg_t h, mspcg_t src);

/* ---- reduced-Ls preconditioner (Sec. 3.3) ----
 * z = (T^dag Mhat^-1 T + mu 1) r replaces the preconditioner z = M^-1 r in
 * every solve and in MSPCG_OP_PRECOND.  Mhat^-1 is the same k-step inner CG
 * (inner_iters, inner_prec) on the local operator (+)_s Ahat_s of the Mobius
 * operator with Lhat slices and parameters b_hat, c_hat (M5 and mf as set by
 * mspcg_set_mobius).  T: host, complex interleaved, [Lhat][4][Ls][4]: row
 * (s, spin) of the reduced field, column (t, spin) of the full one; the
 * identity in colour and on the 4D sites; copied.  Lhat = 0 switches back to
 * the full-Ls preconditioner (T may then be null).  A later mspcg_set_mobius
 * with another Ls switches it off.  Errors: NO_PARAMS, INVALID_ARG (Lhat
 * outside [1, Ls], a non-finite value); a singular reduced operator is
 * reported by the first solve or apply. */
mspcg_status mspcg_set_reduced(mspcg_t h, int32_t Lhat, double b_hat, double c_hat, double mu, const double* T);

/* The current Lhat (0: off) and, if T is not null and Lhat > 0, a copy of T
 * (host, complex interleaved, [Lhat][4][Ls][4]). */
mspcg_status mspcg_get_reduced(mspcg_t h, int32_t* Lhat, double* T);

/* Training loss of Sec. 3.3 over nvec device FP64 fields v (even
 * checkerboard, one after another):
 *   chi2 = sum_i |M (T^dag Mhat^-1 T + mu) v_i - v_i|^2,  M = (+)_s A_s,
 * and, when grad (host, complex interleaved, [Lhat][4][Ls][4]) is not null,
 * d chi2 / d Re T + i d chi2 / d Im T with Mhat^-1 taken as a linear map.
 * Arithmetic in outer_prec (FP64 accumulation of sums), the inner solves in
 * inner_prec.  Errors: INVALID_ARG (no reduced preconditioner, nvec < 1),
 * NO_GAUGE, NO_PARAMS, BAD_TILING. */
mspcg_status mspcg_reduced_loss(mspcg_t h, int32_t nvec, const double* v, double* chi2, double* grad);

/* Trains T in place (Sec. 3.3: line search, momentum): iters steps of
 * d = -grad + momentum d_prev, T += eta d, eta the minimiser over eta >= 0
 * of chi2(T + eta d), a quartic in eta when Mhat^-1 is taken as linear (as
 * for the gradient), whose five coefficients are formed exactly from
 * Mhat^-1 T v_i and Mhat^-1 d v_i.  history (host, iters + 1 entries,
 * nullable): chi2 before the first step and after each.  Errors as
 * mspcg_reduced_loss, and INVALID_ARG for iters < 0. */
mspcg_status mspcg_train_reduced(mspcg_t h, int32_t nvec, const double* v, int32_t iters, double momentum,
                                 double* history);

/* Engine of the fifth-dimension epilogue of the FP32 and 16-bit site kernels
 * with Ls <= 16, for every handle of the process: 1 = MFMA (the default),
 * 0 = vector ALUs.  It waits until no solve, apply, autotune or reduced-Ls
 * training call of any handle is running (those hold the engine for their
 * duration), so a call never sees the engine change under it; work that an
 * apply_device call has enqueued keeps the engine it was launched with.
 * Partial-sum buffers grow on the next call that needs them.  Never fails. */
mspcg_status mspcg_set_mfma(int32_t on);

/* Progress of long solves: one line on stderr every `every` outer
 * iterations (the iterated relative residual; for batched solves the RHS
 * still active), 0 = none (the default).  Errors: INVALID_ARG. */
mspcg_status mspcg_set_log(mspcg_t h, int32_t every);

/* Graph replay of batched solves on (1, the default) or off (0: every
 * iteration is launched eagerly; results are the same either way).  While
 * a solve captures its graph (once per call, before the replays), device-wide
 * synchronization from other threads of the process fails with a capture
 * error; turn graphs off where other threads may synchronize the device.
 * Errors: INVALID_ARG (NULL). */
mspcg_status mspcg_set_graphs(mspcg_t h, int32_t on);

/* Device memory of a handle: `estimate` = bytes a batched solve of nrhs
 * right-hand sides allocates with the current parameters (workspaces,
 * matrices, tables; not the gauge field), `allocated` = bytes the handle
 * holds now.  Errors: INVALID_ARG, NO_PARAMS. */
mspcg_status mspcg_footprint(mspcg_t h, int32_t nrhs, int64_t* estimate, int64_t* allocated);

/* ---------------------------------------------------------------------------
 * Serving: a request loop on one device over resident gauge fields.
 *
 * Requests (a batched solve: field, Mobius parameters, tiling, solver
 * parameters, nrhs device sources and solutions) are admitted in arrival
 * order while their device footprint fits the HBM budget.  By default they
 * are continuously batched (mspcg_server_set_mode): the right-hand sides of
 * requests of one shape share the slots of one running batched solve and
 * enter it as earlier ones finish, and solves of different shapes run
 * concurrently on their own threads and streams.  Solver state stays
 * resident between requests and is evicted least recently used when the
 * budget needs its memory.  A request's result does not depend on what runs
 * beside it.
 * ------------------------------------------------------------------------- */
typedef struct mspcg_server* mspcg_server_t;

typedef struct {
  int32_t field;                /* from mspcg_server_add_field                       */
  int32_t Ls;
  double b, c, M5, mf;          /* Mobius parameters (as mspcg_set_mobius)            */
  int32_t sub[4];               /* subdomain extents (as mspcg_set_subdomains)        */
  mspcg_solver_params solver;
  int32_t nrhs;                 /* 1..1024                                            */
  const double* src;            /* device FP64, nrhs fields one after another; ready  */
  double* x;                    /*   before submit, untouched by the caller until wait */
} mspcg_request;

typedef struct {
  int64_t budget;               /* HBM budget in bytes                                */
  int64_t bytes_in_use;         /* gauge fields + resident contexts + reservations   */
  int64_t bytes_peak;
  int32_t inflight, waiting, peak_inflight, contexts;
  int64_t completed, evictions;
} mspcg_server_stats;

/* Start a server on `device` with an HBM budget (bytes) and at most
 * max_inflight concurrent requests (1..64).  Errors: INVALID_ARG. */
mspcg_status mspcg_server_create(mspcg_server_t* out, int32_t device, int64_t hbm_budget, int32_t max_inflight);

/* Finish the requests in flight and waiting, then free everything. */
mspcg_status mspcg_server_destroy(mspcg_server_t s);

/* Load a gauge field (host FP64, layout above) onto the device; it stays
 * resident until the server is destroyed.  *field gets its id.
 * Errors: INVALID_ARG, OOM (the field does not fit the budget), HIP. */
mspcg_status mspcg_server_add_field(mspcg_server_t s, const int32_t dims[4], const double* U, int32_t* field);

/* Queue a request; *ticket identifies it.  Returns at once.
 * Errors: INVALID_ARG (NULL, unknown field, nrhs outside [1, 1024]). */
mspcg_status mspcg_server_submit(mspcg_server_t s, const mspcg_request* r, int64_t* ticket);

/* *done = 1 when the request has finished.  Errors: INVALID_ARG (ticket). */
mspcg_status mspcg_server_poll(mspcg_server_t s, int64_t ticket, int32_t* done);

/* Wait for a request, fill st[nrhs] (nullable) and *latency_ms (nullable:
 * submit to completion, host wall clock) and release the ticket.  Returns
 * the request's status (as mspcg_solve_batch_device; OOM when it cannot fit
 * the budget even alone; BAD_TILING or INVALID_ARG for bad parameters). */
mspcg_status mspcg_server_wait(mspcg_server_t s, int64_t ticket, mspcg_stats* st, double* latency_ms);

/* Graph replay on or off for every context of the server (as
 * mspcg_set_graphs; off by default, since the caller's threads may
 * synchronize the device at any time).  Errors: INVALID_ARG (NULL). */
mspcg_status mspcg_server_set_graphs(mspcg_server_t s, int32_t on);

/* How the server runs admitted requests (only while none is in flight):
 * mode 1 (default) continuous batching -- one engine per request shape
 * (field, Mobius parameters, tiling and solver parameters), an open
 * mspcg_cb_* session of `slots` right-hand-side slots driven by a thread and
 * stream of its own; a request's right-hand sides queue at its shape's
 * engine and enter slots as earlier ones finish, while the others keep
 * iterating; at most max_inflight engines are busy at once, and an engine
 * opens with as many of the `slots` as the budget holds then (at least one;
 * it holds mspcg_footprint of that many bytes); mode 0 -- one resident
 * context per shape and a worker thread and stream per admitted request,
 * which runs the request as one batched solve (at most max_inflight at
 * once).  In both modes a right-hand side's solution does not depend on what
 * runs beside it.  Errors: INVALID_ARG (mode, slots outside [1, 1024],
 * requests in flight). */
mspcg_status mspcg_server_set_mode(mspcg_server_t s, int32_t mode, int32_t slots);

/* Counters of the server. */
mspcg_status mspcg_server_info(mspcg_server_t s, mspcg_server_stats* info);

/* Message for the last non-OK status returned on the calling thread. */
const char* mspcg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MSPCG_H */
