/*
 * gabp.h -- C ABI of the MI355X (gfx950) flood Gaussian-belief-propagation solver.
 *
 * Solves A x = b for a square, invertible, possibly nonsymmetric sparse A with a nonzero
 * diagonal (arXiv 1904.04093, Sec. 1, eq. linear_problem; the convergence theorem of
 * Sec. 2.3 assumes A_ii != 0) by the reparametrised GaBP of Sec. 2.3
 * (eq. nonsymmetric_GaBP_rules, Algorithm 1) run in the flood ("parallel") schedule of
 * Sec. 2.2: every message of sweep n+1 is computed from the messages of sweep n.
 *
 * Graph and messages. The directed edge j -> i exists iff A_ij != 0 (Sec. 2.3). Every edge
 * carries (Lt_ji, m_ji) with Lt = Lambda / A_ji, m = mu * Lambda
 * (eq. nonsymmetric_GaBP_messages). One sweep, for every node j:
 *     Sigma_j = A_jj + sum_k Lt_kj A_kj,   M_j = b_j + sum_k m_kj,   x_j = M_j / Sigma_j,
 * and for every edge j -> i:
 *     Lt_ji = -A_ij / (Sigma_j - Lt_ij A_ij),   m_ji = Lt_ji (M_j - m_ij).
 * A sweep reads off x from the messages it receives and then updates them, so the s-th
 * read-off uses s-1 updates (one sweep applies h^2/4 to the 5-point Laplacian, two apply
 * h^2/12 [1; 1 4 1; 1], Sec. 4.1). Messages start at zero.
 *
 * Conventions for every entry point:
 *  - Return value: a GABP_* status below. Nothing aborts the process; after a non-zero
 *    return gabp_last_error() describes the failure (thread-local string).
 *  - "device" pointers are HIP device allocations (e.g. torch tensors on cuda:0) on the
 *    device the context was created on; "host" pointers are ordinary CPU memory.
 *  - Every device-side operation is enqueued on the caller's `stream` (0 = null stream).
 *    Calls that report convergence block the host on small (<= 64-byte) readbacks.
 *  - Contexts are not thread-safe: calls on one context must not overlap.
 *  - int32 row/column indices; the internal slot count (twice the number of off-diagonal
 *    pairs of the symmetrised pattern, padded) must stay below 2^31 - 1.
 */
#ifndef GABP_H
#define GABP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------------------- */
#define GABP_OK 0          /* converged (or the requested fixed work was done)            */
#define GABP_MAXSWEEPS 1   /* tolerance not reached; outputs hold the last iterate         */
#define GABP_EINVAL -1     /* bad argument: CSR structure, rev index, sizes, NULL pointer  */
#define GABP_ENOMEM -2     /* device or host allocation failed                              */
#define GABP_EZERODIAG -3  /* a diagonal entry A_ii is missing or zero                      */
#define GABP_ENUMERIC -4   /* non-finite read-off or residual (zero cavity precision, ...) */
#define GABP_EDEVICE -5    /* a HIP runtime call failed                                     */
#define GABP_ENOTSUPP -6   /* valid request the library does not support                     */

/* ---- options ------------------------------------------------------------------------- */
#define GABP_MODE_JOINT 0    /* Algorithm 1 literally: Lt and m updated every sweep        */
#define GABP_MODE_PRECOMP 1  /* Lt iterated alone to convergence first, then frozen and
                                shared by every right-hand side and smoother call
                                (Sec. 2.3 remark on decoupling; Sec. 4.2)                    */
#define GABP_MODE_PRECOMP_SEQ 2 /* the Lt of the first sweeps after a message reset, one set
                                per sweep, computed once from zero messages and kept: the
                                precision messages every smoother call needs (Sec. 4.2;
                                they do not depend on the residual), so gabp_smooth and
                                gabp_sweeps give the iterates of JOINT at the cost of mean-
                                only sweeps. Point schedules only (ENOTSUPP at set-up for
                                line schedules and batches); gabp_solve and
                                gabp_solve_transposed return ENOTSUPP                      */
#define GABP_F64 0           /* all message arithmetic in FP64                              */
#define GABP_F32_IR 1        /* FP32 mean messages (precomputed Lt rounded to FP32) inside
                                FP64 iterative refinement: r = b - A x and x += d are the
                                only FP64 steps                                             */
#define GABP_SCHED_FLOOD 0   /* all nodes send every sweep (Sec. 2.2)                       */
#define GABP_SCHED_REDBLACK 1/* coloured schedule: the nodes of colour 0 send, then those of
                                colour 1, ..., each from the newest messages (the paper's
                                red-black GaBP with two colours, its 4-colour GaBP with four,
                                Sec. 5); needs node colours                                 */
#define GABP_SCHED_LINES 2   /* line GaBP: the two-layer region iteration of Algorithm 2 whose
                                large regions are the grid's rows and columns and whose small
                                regions are the nodes (Fig. two_layers_network), every line
                                from the previous messages; needs grid_nx, grid_ny          */
#define GABP_SCHED_LINES_ALT 3 /* line GaBP with all rows updated first, then all columns from
                                the new row messages (one chain of the flood iteration)     */

typedef struct {
  int32_t mode;              /* GABP_MODE_*                      default GABP_MODE_JOINT   */
  int32_t precision;         /* GABP_F64 | GABP_F32_IR           default GABP_F64          */
  int32_t check_every;       /* sweeps between residual checks   default 16               */
  double tol_lambda;         /* Lt converged when max|dLt| <= tol_lambda * max|Lt|
                                (0: run exactly max_lambda_sweeps)  default 1e-14          */
  int32_t max_lambda_sweeps; /* cap on the Lt phase               default 100000           */
  double ir_inner_tol;       /* IR: inner solve ends when ||r_new|| <= ir_inner_tol*||r||
                                                                  default 1e-4             */
  int32_t ir_max_inner;      /* IR: cap on inner sweeps per outer step  default 1000000   */
  int32_t schedule;          /* GABP_SCHED_*                      default FLOOD            */
  int32_t use_graphs;        /* record each check block (sweeps + residual + readback) as a
                                hipGraph once and replay it       default 1                */
  int32_t grid_nx, grid_ny;  /* line schedules: node (x, y) is row y*grid_nx + x, and A may
                                couple a node only with its horizontal and vertical
                                neighbours (5-point pattern); lines of at most 4096 nodes
                                                                  default 0, 0             */
  int32_t tiles;             /* 1: temporal blocking of the flood schedule -- the rows are
                                laid out in tiles of 13 grid rows (26 with GABP_F32_IR)
                                x 64 columns and one
                                launch does two sweeps per tile, keeping the messages of
                                the first in LDS (the tile's neighbour rows are swept once
                                more to supply them); needs grid_nx, grid_ny (node (x, y) is
                                row y * grid_nx + x), the flood schedule and rows of at most
                                4 off-diagonal neighbours. Same iterates as 0.  default 0 */
  int32_t block;             /* threads per workgroup of the single-system sweep kernels:
                                64, 128 or 256 (gabp_autotune picks one by measurement)
                                                                  default 256              */
  double progress_s;         /* > 0: gabp_solve / gabp_solve_transposed print one line to
                                stderr (sweeps done, relative residual, seconds) at the
                                first check after every progress_s seconds     default 0 */
  int32_t stream_hints;      /* cache hints of the single-system sweep kernels' per-slot
                                streams: -1 by the footprint (non-temporal once a sweep's
                                bytes exceed the last-level cache; gabp_autotune measures
                                instead), 0 plain, 1 non-temporal loads and stores, 2
                                non-temporal stores with plain loads (tiled layouts only:
                                a tile's halo reads its neighbours' lines, which plain loads
                                keep in L2)                                  default -1 */
} gabp_options;

typedef struct {
  int32_t status;        /* GABP_OK or GABP_MAXSWEEPS (or a negative error)                */
  int32_t sweeps;        /* mean/joint sweeps done (all IR inner sweeps summed)            */
  int32_t lambda_sweeps; /* sweeps of the Lt phase (PRECOMP), 0 when reused or JOINT       */
  int32_t outer_iters;   /* IR outer steps (0 for plain solves)                            */
  double rel_res2;       /* ||b - A x||_2 / ||b||_2 of the returned x                      */
  double res_inf;        /* ||b - A x||_inf of the returned x                              */
} gabp_info;

typedef struct gabp_ctx gabp_ctx;
typedef struct mg_ctx mg_ctx;

void gabp_default_options(gabp_options* opt);
const char* gabp_strerror(int status);
const char* gabp_last_error(void);

/* Check a CSR matrix on the host. rowptr[n+1], col[nnz], val[nnz]: host pointers; columns
 * strictly increasing within each row, every diagonal present, finite and nonzero.
 * rev[nnz] (host, may be NULL): rev[e] is the index of the transposed entry (j,i) of entry
 * e = (i,j), or -1 when A has no stored (j,i); a diagonal entry may give itself or -1.
 * Returns GABP_OK, GABP_EINVAL or GABP_EZERODIAG. Needs no GPU. */
int gabp_validate_csr(int32_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                      const double* val, const int32_t* rev);

/* Build a solver context for A (Sec. 2.3: graph of A plus reverse-edge pairing). rowptr,
 * col, val, rev: HOST pointers as in gabp_validate_csr (rev NULL: built here). The CSR is
 * read on the host on purpose: the symmetrised pattern, the reverse index and the slice
 * layout are built there once, so a device-resident CSR is copied to the host by the
 * caller first (later value changes go through gabp_update_values, which takes device
 * values). The matrix
 * is copied into context-owned device memory in slice-of-64-rows, column-major order over
 * the symmetrised pattern; the caller may free its arrays on return. opt NULL = defaults.
 * `colour` (host, may be NULL): one byte per row, the row's colour class 0..7 (red-black:
 * 0 = red, 1 = black); required by GABP_SCHED_REDBLACK, and no edge may join two nodes of
 * one colour (EINVAL otherwise).
 * The context belongs to the current HIP device. */
int gabp_setup(gabp_ctx** out, int32_t n, int64_t nnz, const int32_t* rowptr,
               const int32_t* col, const double* val, const int32_t* rev,
               const uint8_t* colour, const gabp_options* opt, hipStream_t stream);

/* Replace the values of A, same pattern as at setup. val: DEVICE pointer, nnz doubles in
 * the setup CSR order. Precomputed Lt (if any) is invalidated and rebuilt on next use.
 * The new diagonal is checked on the device (one flag read back, so the call waits for
 * the stream): EZERODIAG if any A_ii is zero or not finite. The values are installed
 * either way, so after EZERODIAG the context must get valid values before it solves.
 * Off-diagonal values are not checked (a non-finite one ends a later solve with
 * ENUMERIC). */
int gabp_update_values(gabp_ctx* ctx, const double* val, hipStream_t stream);

void gabp_destroy(gabp_ctx* ctx);

/* Algorithm 1: solve A x = b (b, x: DEVICE, n doubles) from zero messages until
 * ||b - A x||_2 / ||b||_2 <= tol, checked every opt.check_every sweeps (so the sweep count
 * is a multiple of it, or max_sweeps), or max_sweeps. Mode and precision from the options:
 * JOINT/F64 runs the joint sweep; PRECOMP/F64 computes (or reuses) Lt then runs mean-only
 * sweeps; F32_IR runs FP32 mean-only sweeps inside FP64 iterative refinement (max_sweeps
 * then caps the total inner sweeps). info may be NULL. */
int gabp_solve(gabp_ctx* ctx, const double* b, double* x, double tol, int32_t max_sweeps,
               gabp_info* info, hipStream_t stream);

/* Same as gabp_solve for A^T lambda = g (adjoint solves): GaBP on the transposed graph,
 * i.e. with A_ij and A_ji exchanged in every rule. g, lambda: DEVICE, n doubles. */
int gabp_solve_transposed(gabp_ctx* ctx, const double* g, double* lambda, double tol,
                          int32_t max_sweeps, gabp_info* info, hipStream_t stream);

/* Exactly `sweeps` sweeps of the configured mode/schedule with no residual check.
 * reset != 0 starts from zero messages (PRECOMP: with the precomputed Lt, computed first if
 * needed); reset == 0 continues from the context's current messages. x (DEVICE) receives
 * the read-off of the last sweep. Precision GABP_F32_IR runs FP32 mean-only sweeps on
 * fp32(b) and widens the FP32 read-off into x. For parity checks, checkpoints and timing. */
int gabp_sweeps(gabp_ctx* ctx, const double* b, double* x, int32_t sweeps, int32_t reset,
                int32_t transposed, hipStream_t stream);

/* Lt phase only (Sec. 2.3: Lt does not depend on b): iterate Lt from zero until
 * opt.tol_lambda / opt.max_lambda_sweeps, keep Lt*, 1/Sigma* (FP64 and FP32 copies).
 * sweeps_out (host, may be NULL) receives the number of Lt updates. */
int gabp_precompute_lambda(gabp_ctx* ctx, int32_t transposed, int32_t* sweeps_out,
                           hipStream_t stream);

/* Algorithm 3 (error-correction smoother): r = b - A x; mu sweeps on A e = r with the
 * context's mode/schedule/precision, messages restarted from zero (Algorithm 3 applies
 * Algorithm 1 to the error equation); x += e^mu (the mu-th read-off).
 * b: DEVICE const, x: DEVICE in/out, n doubles. */
int gabp_smooth(gabp_ctx* ctx, const double* b, double* x, int32_t mu, hipStream_t stream);

/* r = b - A x (transposed != 0: b - A^T x) and its norms. b, x, r: DEVICE (r may be NULL).
 * norms (host, may be NULL): [||r||_2, ||r||_inf, ||b||_2]. Deterministic reduction order. */
int gabp_residual(gabp_ctx* ctx, const double* b, const double* x, double* r,
                  int32_t transposed, double* norms, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): gabp_residual with the norms written
 * to DEVICE memory and its per-block partial sums kept in a fixed 2 MiB device array that
 * the library holds on each GPU until the process ends, so the call allocates nothing,
 * never waits for the stream and can be captured. b, x, r: DEVICE as in gabp_residual
 * (r may be NULL); norms (DEVICE, may be NULL): [||r||_2, ||r||_inf, ||b||_2], the same
 * values gabp_residual returns (same kernels, same reduction order). Contexts of more than
 * 22,369,280 rows (lanes) are rejected with GABP_EINVAL. Every call on one GPU shares that
 * array: calls that overlap on one GPU (other streams or threads) race; calls in order on
 * one stream do not. */
int gabp_residual_noalloc(gabp_ctx* ctx, const double* b, const double* x, double* r,
                          int32_t transposed, double* norms, hipStream_t stream);

/* Adjoint scatter for L(x(A)) with A x = b: G_e = dL/dA_e = -lambda_row(e) x_col(e) for
 * every stored entry e in setup CSR order (lambda solves A^T lambda = dL/dx). lambda, x:
 * DEVICE n doubles; G: DEVICE nnz doubles (may be NULL). If jptr != NULL the entry
 * gradient is also reduced onto nparam parameters through a parameter-major sparse
 * Jacobian: dtheta_p = sum_{k in jptr[p]..jptr[p+1]} jw[k] * G[jnnz[k]] (jptr, jnnz, jw,
 * dtheta: DEVICE). Each parameter is reduced by one thread in index order (deterministic).
 * The caller guarantees jptr[0] = 0, jptr non-decreasing, and 0 <= jnnz[k] < nnz: the
 * arrays are read on the device without a check (indices outside that range read outside
 * the context's entry arrays). */
int gabp_adjoint_scatter(gabp_ctx* ctx, const double* lambda, const double* x, double* G,
                         int32_t nparam, const int32_t* jptr, const int32_t* jnnz,
                         const double* jw, double* dtheta, hipStream_t stream);

/* Checkpoint: the complete iteration state (messages, precomputed Lt, sweep parity; for
 * line schedules the messages of both orientations and both layouts, the FP32 messages and
 * the frozen multipliers and read-off factors). gabp_get_state with dst == NULL stores the
 * needed size in *bytes; otherwise dst (host) must hold *bytes. gabp_set_state restores a
 * state taken from a context with the same matrix pattern and options (EINVAL for a blob
 * of another layout or schedule family, or a truncated one). */
int gabp_get_state(gabp_ctx* ctx, void* dst, size_t* bytes, hipStream_t stream);
int gabp_set_state(gabp_ctx* ctx, const void* src, size_t bytes, hipStream_t stream);

/* Message state in the matrix's own order, for parity checks of the messages of
 * eq. nonsymmetric_GaBP_rules: for every stored off-diagonal entry e = (i, j) of the setup
 * CSR, lam[e] = Lt_ji and msg[e] = m_ji, the messages j -> i that row i receives now (after
 * the sweeps since the last reset; zero right after a reset). Diagonal entries get 0.
 * PRECOMP: lam is the frozen Lt*; PRECOMP_SEQ: the Lt of the last sweep done; F32_IR
 * precision: msg is the FP32 mean-message state widened. lam, msg: DEVICE, nnz doubles each
 * (either may be NULL). Line schedules and batches: ENOTSUPP. */
int gabp_get_messages(gabp_ctx* ctx, double* lam, double* msg, hipStream_t stream);

/* Residual history of the context's last gabp_solve / gabp_solve_transposed: the
 * ||b - A x||_2 / ||b||_2 read at every check (FP32 refinement: of every trial x + s d),
 * in order. *count (host) receives the number of checks; out (host, may be NULL) receives
 * the first min(cap, count) values. Fault injection for tests of the failure path: when the
 * environment variable GABP_FAULT_INJECT reads nan@sweep:<k> at gabp_setup, the first
 * single-system solve check block that starts at or after sweep k begins with every
 * incoming mean message set to NaN (once), so the check reports GABP_ENUMERIC; with
 * poison-outputs every ping-pong sweep (flood and line schedules) first fills the message
 * arrays it writes with NaN, and every message reset fills the arrays the next sweep reads
 * (not cleared, read as zero) with NaN, so results equal the unpoisoned ones only if every
 * slot that is read was written; gabp_setup returns GABP_EINVAL for any other value of the variable. */
int gabp_residual_history(const gabp_ctx* ctx, double* out, int32_t cap, int32_t* count);

/* Sizes of the internal layout (host outputs, any may be NULL): number of rows, stored
 * nonzeros, directed message slots (2 x off-diagonal pairs), padded slot count, and the
 * bytes per slot of the reverse index the single-system sweeps read (2 when every slot's
 * reverse lies within +-32767 positions, as for grid matrices, else 4). */
int gabp_layout_info(const gabp_ctx* ctx, int32_t* n, int64_t* nnz, int64_t* slots,
                     int64_t* padded_slots, int32_t* rev_bytes);

/* Autotuner. Times the context's own sweep kernel (for its mode, precision and batch
 * shape) with and without non-temporal hints on the per-slot streams and, for single
 * systems, at workgroup sizes of 64, 128 and 256 threads (1, 2 or 4 slices of 64 rows per
 * workgroup), keeps the fastest pair, then sets opt.check_every to the smallest power of
 * two in [8, 256] for which one residual check (kernel, reduction, readback, host wait)
 * costs at most 2% of the sweeps between checks. A tiled context (opt.tiles) is timed with
 * its two-sweep kernels (one workgroup per tile: hints only). Results are cached per
 * (architecture, sizes, mode, schedule, layout) in memory and, when the environment
 * variable GABP_AUTOTUNE_CACHE names a file, in that JSON-lines file. Runs sweeps on a
 * zero right-hand side, so the context's message state is reset; computes the
 * precomputed Lt first when the mode needs it. The measured hint setting and workgroup
 * size replace those given at set-up (opt.stream_hints, opt.block). Outputs (host, may be
 * NULL): the chosen check interval, hint setting (0/1, and 2 for a tiled context: the
 * values of opt.stream_hints) and workgroup size. Because it changes check_every, later
 * solves may stop at a different (rounded-up) sweep count than untuned ones. Sweeps give
 * the same bits under every hint setting and workgroup size (hints change only how the
 * caches treat the streams). Line schedules have no hint or workgroup variants: only
 * the check interval is tuned (from one line sweep), hints_out is 0 and block_out 256;
 * batches keep 256-thread workgroups. */
int gabp_autotune(gabp_ctx* ctx, int32_t* check_every_out, int32_t* hints_out,
                  int32_t* block_out, hipStream_t stream);

/* ---- batches of independent systems ------------------------------------------------- */
/* Build one context for nsys independent systems given as a block-diagonal CSR matrix
 * (HOST arrays, n rows in total; system s owns rows sys_row_off[s] .. sys_row_off[s+1]-1
 * (int32 row offsets, nsys + 1 of them; a system's entries are found through rowptr, so no
 * separate entry offsets are taken)
 * and no entry may couple two systems), each with nrhs right-hand sides (1, 2 or 4).
 * Every system is laid out from a 64-row slice boundary so that a wavefront never mixes
 * two systems. The precision messages Lt* (b-independent, Sec. 2.3) are computed once per
 * system and shared by its right-hand sides. opt as for gabp_setup (red-black schedules
 * are not supported for batches). */
int gabp_setup_batched(gabp_ctx** out, int32_t nsys, const int32_t* sys_row_off, int32_t n,
                       int64_t nnz, const int32_t* rowptr, const int32_t* col,
                       const double* val, int32_t nrhs, const gabp_options* opt,
                       hipStream_t stream);

/* Solve every system for every right-hand side. B, X: DEVICE, [nrhs][n] doubles (rhs-major,
 * rows in the setup numbering). Each (system, rhs) pair stops on its own at
 * ||b - A x||_2 / ||b||_2 <= tol (checked every opt.check_every sweeps), a finished
 * system's wavefronts stop sweeping, and max_sweeps caps the sweeps of the whole batch.
 * F64 precision: flood sweeps (joint or precomputed Lt), each pair keeping the read-off it
 * converged with -- identical, for the same options, to a single-system gabp_solve.
 * F32_IR precision: FP32 mean messages inside FP64 iterative refinement with the rules of
 * gabp_solve applied per pair. infos (HOST, may be NULL): nsys * nrhs entries, pair
 * (s, q) at s * nrhs + q. Returns the worst pair status (OK < MAXSWEEPS < ENUMERIC). */
int gabp_solve_batched(gabp_ctx* ctx, const double* B, double* X, double tol,
                       int32_t max_sweeps, gabp_info* infos, hipStream_t stream);

/* ---- geometric multigrid (Sec. 4: GaBP as a multigrid smoother) ---------------------- */
/* Build a V-cycle over `levels` contexts, finest first (level_ctx[l] owns the operator of
 * level l: a rediscretisation on a vertex-centred side[l] x side[l] interior grid, rows x
 * fastest, with side[l] = 2 side[l+1] + 1; the coarsest side must be <= 63). Grids are
 * square, so one side per level is taken (not separate x and y sizes). Transfers:
 * full-weighting restriction and bilinear interpolation. The coarsest system is solved
 * directly (its inverse is formed once here, by Gauss-Jordan with partial pivoting).
 * smoother 0: GaBP as the error-correction smoother of Algorithm 3, run by each level's
 * context with its own mode, schedule and precision, messages restarted from zero at every
 * call (GABP_MODE_PRECOMP_SEQ keeps the per-sweep Lt between calls); smoother 1: red-black
 * Gauss-Seidel (colour (ix + iy) mod 2, red first). nu1 / nu2: pre- / post-smoothing
 * steps (GaBP: sweeps per smoother call; RB-GS: red+black sweeps). The contexts are
 * borrowed and must outlive the multigrid context; their message state is used by the
 * smoother. Operators must have the 5-point pattern (the RB-GS update is in place).
 * When every level context has opt.use_graphs set, each cycle after the first (which runs
 * eagerly, so that all precomputed-Lt phases and buffers exist) is recorded once as a
 * hipGraph -- the whole V-cycle plus the finest residual's norms -- and replayed. */
int mg_setup(mg_ctx** out, int32_t levels, gabp_ctx* const* level_ctx, const int32_t* side,
             int32_t smoother, int32_t nu1, int32_t nu2, hipStream_t stream);

/* One V(nu1, nu2) cycle on the finest level: x (DEVICE, in/out) is improved for A_0 x = b
 * (b DEVICE). rel_res_out (host, may be NULL): ||b - A_0 x||_2 / ||b||_2 afterwards. */
int mg_vcycle(mg_ctx* m, const double* b, double* x, double* rel_res_out, hipStream_t stream);

/* x = 0, then V-cycles until ||b - A_0 x||_2 / ||b||_2 <= tol or max_cycles. Returns
 * GABP_OK, GABP_MAXSWEEPS (cycle cap) or GABP_ENUMERIC (divergence to non-finite values).
 * cycles_out / rel_res_out: host, may be NULL. Each cycle after the first starts its
 * finest GaBP pre-smoothing from the residual the previous cycle's check formed (x has not
 * changed in between), so the iterates equal those of repeated mg_vcycle calls bit for bit;
 * the finest context's residual buffer holds that residual between cycles. */
int mg_solve(mg_ctx* m, const double* b, double* x, double tol, int32_t max_cycles,
             int32_t* cycles_out, double* rel_res_out, hipStream_t stream);

void mg_destroy(mg_ctx* m);

/* Measurement helper: a plain streaming copy of `bytes` (a multiple of 16) from src to dst
 * (DEVICE, non-overlapping) with 16-byte vector loads and stores. Used to measure the
 * attainable HBM bandwidth and to calibrate the profiler's byte counters against a kernel
 * whose traffic is known exactly (2 x bytes). */
int gabp_copy_probe(const void* src, void* dst, int64_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* GABP_H */
