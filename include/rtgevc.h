/*
 * rtgevc -- robust right generalized eigenvectors of a real Schur pencil on MI355X.
 *
 * C ABI of librtgevc.so.  Every pointer argument named "device" must point to
 * device memory of the current HIP device; sizes are element counts; matrices are
 * column-major with a leading dimension >= max(1, m).  No HIP or torch types
 * appear in the signatures: a stream is passed as `void *` holding a hipStream_t
 * (NULL = the default stream).
 *
 * The problem (Kjelgaard Mikkelsen & Myllykoski, "Parallel Robust Computation of
 * Generalized Eigenvectors of Matrix Pencils"):
 *   - Section 2: S is quasi-upper-triangular with 1x1 and 2x2 diagonal blocks, T is
 *     upper triangular, both of order m (a generalized real Schur form).  A 1x1
 *     block carries a real eigenvalue, a 2x2 block a complex-conjugate pair, and
 *     all eigenvalues are distinct.  Eigenvalues are pairs (alpha, beta), beta >= 0.
 *   - Section 2.1/2.2: with D = diag(beta_j) and B block diagonal holding a_j (1x1)
 *     or [[a_j, b_j], [-b_j, a_j]] (2x2), the eigenvectors V solve S V D - T V B = 0.
 *   - Section 3, Algorithm 1: the blocked solver over an M x M tile grid that never
 *     splits a 2x2 block; Section 4: overflow protection with augmented matrices
 *     (a mantissa tile plus one power-of-two scale factor per eigenvector column),
 *     ProtectDivision and ProtectUpdate, Algorithms 2 and 3; Section 5: pre-
 *     processing (tile norms), solve, update and post-processing (consistent
 *     scaling) tasks, integer scale exponents, selection closed under conjugation.
 *
 * Output layout: Z is m x m.  Column c of a real eigenvalue holds its eigenvector;
 * for a complex pair in columns (p, p+1), column p holds x and column p+1 holds y
 * where z = x + i y is the eigenvector of the eigenvalue with positive imaginary
 * part (the lemma of Section 2.1).  The phase is fixed by the tip convention: a real
 * eigenvector has z_p = 1 at its own row p; a complex one has z_{p+1} = 1.  Rows
 * below an eigenvector's diagonal block are zero.  Unselected columns are zero.
 *
 * Errors: a negative return is a synchronous error (nothing was enqueued):
 *   -i          argument i (1-based) is invalid;
 *   -1000 - e   a HIP call failed with hipError_t e.
 * Numerical conditions never abort: they are reported as bits of the device int32
 * *info, readable after the stream has been synchronised (RTGEVC_INFO_*).
 * All calls are asynchronous with respect to the host and allocate nothing: the
 * caller provides a device workspace of at least rtgevc_workspace_size() bytes.
 * Calls sharing one workspace must be ordered (same stream, or synchronised).
 */
#ifndef RTGEVC_H
#define RTGEVC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* info bits */
#define RTGEVC_INFO_NONFINITE      1   /* NaN or Inf in S or T (back-transformation: V, Z)  */
#define RTGEVC_INFO_BAD_STRUCTURE  2   /* two consecutive non-zero sub-diagonal entries      */
#define RTGEVC_INFO_REAL_PAIR      4   /* a 2x2 block with real eigenvalues (assumption 2)   */
#define RTGEVC_INFO_INDEFINITE     8   /* alpha = beta = 0 in a 1x1 block: e_p returned      */
#define RTGEVC_INFO_PERTURBED     16   /* a pivot below smin was replaced (assumption 3)     */
#define RTGEVC_INFO_SELECT_CLOSED 32   /* select was closed under complex conjugation        */
#define RTGEVC_INFO_REFINE        64   /* mixed precision: a column's backward-error estimate
                                          is above the threshold after the last sweep         */
#define RTGEVC_INFO_WATCHDOG     128   /* a dependency wait gave up (results invalid)        */
#define RTGEVC_INFO_PRESCALED    256   /* S and T were scaled by a common power of two       */

/* Tuning options.  Pass NULL for the defaults. */
typedef struct rtgevc_opts {
  int32_t mb;         /* tile size: 0 = automatic; else 32, 64 or 128.  Tiles are mb or
                         mb - 1 rows (a boundary moves up one row rather than split a
                         2x2 block).                                                   */
  int32_t normalize;  /* 1 (default when opts is NULL): divide each eigenvector by
                         max_i(|x_i| + |y_i|) and return scales = 0;
                         0: return the mantissa in Z and the exponent in scales, so the
                         eigenvector is 2^scales[c] * Z[:, c].                          */
  int32_t band;       /* tile rows per update band: 0 = automatic, else 1..8.  After the
                         rows of a band are solved (with small updates inside the band),
                         one contraction applies all of them to every tile above it.   */
  int32_t schedule;   /* how the task graph of Algorithm 1 is walked:
                         0 or 1: band wavefront (one launch per band step for all tile
                             columns, look-ahead on a second stream);
                         2: persistent walker (one launch; workgroups take tile tasks in
                             a fixed priority order and wait on device-side dependency
                             counters; one source row per update, so band is ignored;
                             needs a larger workspace: W of every tile).
                         Both give the same eigenvectors (schedule 2 equals schedule 1
                         with band = 1 bit for bit).                                    */
  int32_t watchdog;   /* schedule 2: bound on each dependency wait in polling rounds
                         (0 = default, about two seconds).  A wait that runs out sets
                         RTGEVC_INFO_WATCHDOG and the results are invalid.              */
  int32_t precision;  /* 0 (default): tile updates on the FP64 matrix cores.
                         1: mixed precision: the tile-update contraction is emulated on
                            the int8 matrix cores from operands split into a power-of-two
                            scale and 7 signed 7-bit slices (products of slices are exact,
                            summed exactly in int32 per level and folded in FP64; error
                            about 2 K 2^-49 of max|row| max|column| per product, K <= 256
                            per source).  Solves, bounds, scale factors and consolidation
                            stay FP64.  Needs more workspace (slices of every tile pair).
                            Not with schedule 2.                                          */
  int32_t max_refine; /* mixed precision only: at most this many refinement sweeps against
                         an FP64 residual (0 = default, 1; -1 = none; else 1..3).  A sweep
                         estimates for every column still under refinement the componentwise
                         backward error ||r||_1 / ||beta |S||z| + |alpha||T||z| ||_1 of
                         r = (beta S - alpha T) z (Section 2) with a 16-row Cauchy sketch
                         (O(m^2) work), flags the columns above the threshold, forms r in
                         FP64 for them, solves (beta S - alpha T) d = r with the blocked robust
                         solver (d = 0 at the tip) and replaces z by z - d.  The sweeps run
                         before the consolidation, on the tile segments with their own
                         exponents, so eigenvectors spanning more than the double range
                         are refined at full precision; columns whose entries underflow
                         inside a tile (overflow-stress pencils) are not refined.
                         A last estimate sets RTGEVC_INFO_REFINE for columns still above the
                         threshold.  Needs 8 m^2 more bytes of workspace.                 */
  int32_t refine_bits;/* threshold of the flag: 2^-refine_bits (1..100); 0 = the residual
                         bound 64 m 2^-53.                                              */
  int32_t split;      /* band wavefront: the update that applies a solved band to every tile
                         row above it is issued in launches of about this many tiles
                         (whole tile rows, from the bottom); 0 = automatic (from the tuning
                         table when mb and band are the table's as well, else one launch),
                         -1 = one launch.  Performance only: each tile's update is the same
                         computation in any launch, so every value gives the same
                         eigenvectors bit for bit.  The launch boundaries give the chain of
                         tile solves, which runs beside these updates on the caller's
                         stream, a share of the GPU.  rtgevc_batched: tiles per launch
                         summed over a group's pencils (0 or -1: one launch per step). */
  int32_t grid;       /* schedule 2: workgroups of the persistent walker; 0 = automatic (as
                         many as are resident on the GPU at once), else at most that many.
                         Performance only: every count gives the same eigenvectors bit for
                         bit (tasks are taken in one fixed order by running workgroups).
                         Must be >= 0.                                                   */
} rtgevc_opts;

/* Bytes of device workspace rtgevc() needs for order m with these options
 * (0 for m < 0). */
size_t rtgevc_workspace_size(int64_t m, const rtgevc_opts *opts);

/* All selected right eigenvectors of the pencil (S, T).
 *   m        order (m >= 0; m = 0 is a no-op).
 *   S, lds   device, column-major, read-only: upper triangle and first sub-diagonal
 *            are read, the rest is ignored.
 *   T, ldt   device, column-major, read-only: upper triangle is read.
 *   select   device int32[m] or NULL (all).  select[c] != 0 selects eigenvalue c;
 *            either column of a 2x2 block selects both (info bit 32 when applied).
 *   Z, ldz   device, column-major m x m output (written in full).
 *   scales   device int32[m] output or NULL: 0 when normalised, else the exponent.
 *   info     device int32 output or NULL: OR of RTGEVC_INFO_* bits.
 *   work     device workspace of work_bytes >= rtgevc_workspace_size(m, opts),
 *            256-byte aligned; its contents on entry are irrelevant.
 *   opts     NULL or options (see above).
 *   stream   hipStream_t as void *, NULL = default stream.
 * S, T, select must not overlap Z, scales, info or work.  Returns 0 when enqueued. */
int rtgevc(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
           const int32_t *select, double *Z, int64_t ldz, int32_t *scales, int32_t *info,
           void *work, size_t work_bytes, const rtgevc_opts *opts, void *stream);

/* Allocation-free variant of rtgevc(), for callers that cannot allocate device memory or
 * pass a workspace (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  The same computation and results as rtgevc() with the same options (the
 * band schedule runs on the caller's stream alone, without the look-ahead side stream; the
 * persistent walker as in rtgevc), but the workspace is a fixed device array inside the
 * library of RTGEVC_NOALLOC_SCRATCH_BYTES bytes, one per GPU the library runs on, held until
 * the process ends.  The call allocates and frees nothing, creates no stream or event and
 * never synchronises; on its first call on a device it looks up that device's address of
 * the array (with tiles of 128 and bands of more than one row it also raises, once per device,
 * the band-chain kernel's dynamic shared-memory limit; that kernel's four spilled registers
 * use the per-lane private memory the HIP runtime provides with the queue).
 *   Arguments as for rtgevc() (argument numbers: 11 = opts, 12 = stream).
 *   Returns RTGEVC_ERR_SCRATCH, with nothing enqueued, when rtgevc_workspace_size(m, opts)
 *   exceeds RTGEVC_NOALLOC_SCRATCH_BYTES (with default options FP64 fits up to m = 9212).
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (different
 * streams, or host threads, without ordering between them) race and give wrong results;
 * order them on one stream.  The array keeps the last call's contents; everything that must
 * start at zero is cleared by the call's own pre-processing kernels. */
#define RTGEVC_NOALLOC_SCRATCH_BYTES (64u << 20)
#define RTGEVC_ERR_SCRATCH (-2000)
int rtgevc_noalloc(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                   const int32_t *select, double *Z, int64_t ldz, int32_t *scales, int32_t *info,
                   const rtgevc_opts *opts, void *stream);

/* Normalised eigenvalues of (S, T) (Section 2): for each column c, alpha = alpha_re[c]
 * + i alpha_im[c] and beta[c] >= 0, scaled by a power of two so that
 * max(beta, |Re alpha| + |Im alpha|) lies in (1/2, 1]; a complex pair in (p, p+1) has
 * alpha_im[p] > 0 and alpha_im[p+1] = -alpha_im[p].  alpha_re, alpha_im, beta are
 * device double[m]; info as above.  work as for rtgevc with the same m and opts. */
int rtgevc_eigvals(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                   double *alpha_re, double *alpha_im, double *beta, int32_t *info,
                   void *work, size_t work_bytes, const rtgevc_opts *opts, void *stream);

/* Left eigenvectors of the Schur pencil: u^H (beta S - alpha T) = 0 for every selected
 * eigenvalue, with the same robustness (power-of-two scale exponents, no overflow).  They are
 * the right eigenvectors of the flipped transposed pencil (J S^T J, J T^T J), J the exchange
 * matrix, reversed and conjugated, so the library forms that pencil in the workspace and
 * runs the right-eigenvector path on it; its bounds are then the 1-norm bounds of a left
 * solve on (S, T).  Arguments, options, select, info and return codes as for rtgevc();
 * the output Y, ldy takes the place of Z, ldz:
 *   Y      column c is the left eigenvector of eigenvalue c (2^scales[c] Y[:, c]); for a
 *          complex pair (p, p+1), u = Y[:, p] + i Y[:, p+1] is the left eigenvector for
 *          alpha_im[p] > 0.  With normalisation, max_i |u_i| (|Re| + |Im| for a pair) = 1.
 *   work   at least rtgevc_left_workspace_size(m, opts) bytes: rtgevc's workspace plus
 *          16 m^2 + 4 m bytes for the flipped pencil. */
size_t rtgevc_left_workspace_size(int64_t m, const rtgevc_opts *opts);
int rtgevc_left(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                const int32_t *select, double *Y, int64_t ldy, int32_t *scales, int32_t *info,
                void *work, size_t work_bytes, const rtgevc_opts *opts, void *stream);

/* Complex-arithmetic pencils (the conclusion's extension of the method, Section 7): S and T
 * complex upper triangular of order m (no 2x2 blocks), stored column-major with the real and
 * imaginary parts of each entry interleaved (C99 double complex / std::complex<double>);
 * lds, ldt, ldz count complex entries.  For every selected eigenvalue k (lambda = s_kk / t_kk)
 * column k of Z receives the eigenvector z, (beta S - alpha T) z = 0, with z_k = 1 before
 * normalisation (the phase), rows below k zero; with normalisation max_i |Re z_i| + |Im z_i| = 1
 * and scales 0, else z = 2^scales[k] Z[:, k].  select: device int32[m] or NULL (all).
 * The call scales each row of (S, T) by conj(t_ii) 2^-e (right eigenvectors unchanged, the
 * diagonal of T becomes real) and solves the real form of order 2m, each complex entry
 * x + i y as the block [[x, -y], [y, x]], with the real path (its tile size, band, schedule and
 * precision options apply to order 2m; the mixed mode's refinement too); a complex eigenvalue
 * is then a 2x2 block of the real form, an exactly real one two 1x1 blocks, and the complex
 * eigenvector is read back from the real one.  Robustness, info bits and return codes as for
 * rtgevc() (-11/-12: workspace NULL, misaligned or below
 * rtgevc_complex_workspace_size(m, opts): rtgevc's workspace for order 2m plus 96 m^2 + 16 m
 * bytes for the real form and its eigenvectors). */
size_t rtgevc_complex_workspace_size(int64_t m, const rtgevc_opts *opts);
int rtgevc_complex(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                   const int32_t *select, double *Z, int64_t ldz, int32_t *scales, int32_t *info,
                   void *work, size_t work_bytes, const rtgevc_opts *opts, void *stream);

/* Back-transformation to the eigenvectors of the original pencil (the step after the
 * path).  With the real Schur decomposition S = U^T A V, T = U^T B V of Section 1 (U, V
 * orthogonal, (S, T) the real Schur pencil given to rtgevc), S z = lambda T z gives
 * A (V z) = lambda B (V z): the eigenvectors of (A, B) are X = V Z (Section 1 writes U z;
 * V z is the vector that satisfies the equation).  For every column c:
 *     2^xscales[c] X[:, c] = V (2^scales[c] Z[:, c]),
 * with Z, scales the output of rtgevc() (Z upper quasi-triangular: the entries below its
 * first sub-diagonal, and the sub-diagonal entries of columns that do not start a complex
 * pair, are not read).  A complex pair (p, p+1) keeps its real form: X[:, p] + i X[:, p+1]
 * is the eigenvector for alpha_im[p] > 0, and both columns share one exponent.  When
 * m max|V| max|Z_c| could exceed Omega = 2^1020, Z_c is scaled down by a power of two
 * before the product (exact, entries below the smallest normal number may flush to zero)
 * and the exponent added to xscales[c], so nothing overflows.
 *   S         device double, column-major, leading dimension lds >= max(1, m): only its
 *             sub-diagonal is read (the 2x2 block structure).
 *   V         device double, column-major m x m, leading dimension ldv >= max(1, m).
 *   Z, ldz    as returned by rtgevc(); scales: device int32[m] or NULL (all zero).
 *   X, ldx    device double output, column-major m x m.  X may be Z itself (with
 *             ldx == ldz: the result overwrites the input); X must not overlap V.
 *   xscales   device int32[m] output.
 *   info      device int32 output or NULL: RTGEVC_INFO_NONFINITE if V or Z holds a NaN or
 *             an infinity (the result is then not meaningful).
 *   opts      NULL or options: mb (64 or 128; 0 or 32: 128 from m = 2048, else 64) is
 *             the tile of the contraction; normalize (default 1): each eigenvector is
 *             divided by max_i |x_i| (real) or max_i |x_i| + |y_i| (pair) and xscales = 0.
 *             The other fields are not used.
 *   work      device workspace of at least rtgevc_backtransform_workspace_size(m, opts)
 *             bytes, 256-byte aligned (about 4 m^2 bytes: Z in the matrix-core operand order).
 * Asynchronous on stream, no allocation or synchronisation: capturable in a HIP graph.
 * Returns 0 when enqueued, -i for invalid argument i (-9: X overlaps V; -10: X is Z with
 * ldx != ldz; -13/-14: workspace NULL, misaligned or too small), or -1000 - hipError. */
size_t rtgevc_backtransform_workspace_size(int64_t m, const rtgevc_opts *opts);
int rtgevc_backtransform(int64_t m, const double *S, int64_t lds, const double *V, int64_t ldv,
                         const double *Z, int64_t ldz, const int32_t *scales, double *X, int64_t ldx,
                         int32_t *xscales, int32_t *info, void *work, size_t work_bytes,
                         const rtgevc_opts *opts, void *stream);

/* Benchmark variant of rtgevc(): the same work on the same stream, with a HIP event
 * recorded before and after every kernel launch (on the stream the launch runs on).
 * Unlike rtgevc() it synchronises the stream (after pre-processing and at the end) and
 * creates events on first use (kept per device until the process ends), so it is not
 * for graph capture.  On success stats (host double[nstats], nstats >=
 * RTGEVC_TIMED_NSTATS) holds:
 *   [0] total device time, ms (first to last event)
 *   [1..4] summed device time of the pre-processing, diagonal-solve (a band's chain launch,
 *          its solves with the in-band updates, counts here), tile-update and
 *          consolidation launches, ms
 *   [5..8] number of launches of each of those four classes
 *   [9] algorithmic flops of the tile-update launches: over their target rows k, sources r
 *          and columns j >= r, the sum of 4 h_k h_r h_j (the persistent walker: of all tile
 *          updates, sum over k < r <= j)
 *   [10] number of tiles M;  [11] tile size mb
 *   [12] device time of the refinement sweeps (mixed precision), ms;  [13] sweeps
 *   [14..16] the tile-update launches of the side stream alone (the band schedule's updates
 *          of the rows above the next band): summed device time, ms; their algorithmic
 *          flops (the same sum over their target rows, sources and columns); their number
 * Returns 0, a negative argument code as rtgevc() (-15: stats), or -1000 - hipError. */
#define RTGEVC_TIMED_NSTATS 17
int rtgevc_timed(int64_t m, const double *S, int64_t lds, const double *T, int64_t ldt,
                 const int32_t *select, double *Z, int64_t ldz, int32_t *scales, int32_t *info,
                 void *work, size_t work_bytes, const rtgevc_opts *opts, void *stream,
                 double *stats, int nstats);

/* Batches of independent pencils (the workload of many small and medium eigenvector
 * problems; Section 5's selection and output conventions per pencil).
 *
 * count pencils; pencil i has order m[i] >= 0 (m[i] = 0: skipped, info[i] untouched).
 * m, lds, ldt, ldz are HOST arrays of count entries; S, T, select, Z, scales are HOST
 * arrays of count DEVICE pointers (select and scales may be NULL as a whole or per
 * pencil); info is a DEVICE int32[count] (or NULL) receiving each pencil's bits.  Every
 * pencil's arguments obey the rules of rtgevc().  work: device workspace, 256-byte
 * aligned, of at least rtgevc_batched_workspace_size(count, m, opts) bytes.  opts as
 * for rtgevc(); its mb and band, when non-zero, apply to every pencil (band 0: 3); split
 * (> 0) issues the update of the rows above the next band in launches of about that many
 * tiles summed over a group's pencils (0 or -1: one launch per step); its schedule and
 * precision are not used (the batch runs FP64 tile updates in lock-step).
 *
 * Pencils are grouped by tile size (automatic per order unless opts->mb is set); each
 * group runs in lock-step over bands of R tile rows: step t solves the rows of band
 * b = B_p - 1 - t of every pencil p of the group, bottom-up with the updates inside the
 * band, applies the band to the next band's rows, and then, on a second stream of the
 * library (created on the first call on a device, at default priority, kept until the
 * process ends), to every row above those while step t + 1 proceeds on the caller's
 * stream (the look-ahead of rtgevc()'s band schedule, one launch per part of a step and
 * kernel for the whole group; events order the two streams, and the second stream is
 * joined back before the call's last kernel).  The eigenvectors equal those of rtgevc()
 * with the same tile size and band.  The call enqueues kernels and event records and
 * waits only: no allocation, no copy, no synchronisation, so it can be captured in a HIP
 * graph and replayed (the host arrays are read during the call; the device pointers they
 * hold must stay valid for every replay); make the first call on a device outside
 * capture.  Calls from several host threads are serialised while they enqueue.
 * Returns 0 when enqueued; -i for argument i (1-based; per-pencil violations report
 * the argument that holds them); -1000 - hipError on a launch failure. */
size_t rtgevc_batched_workspace_size(int32_t count, const int64_t *m, const rtgevc_opts *opts);

int rtgevc_batched(int32_t count, const int64_t *m, const double *const *S, const int64_t *lds,
                   const double *const *T, const int64_t *ldt, const int32_t *const *select,
                   double *const *Z, const int64_t *ldz, int32_t *const *scales, int32_t *info,
                   void *work, size_t work_bytes, const rtgevc_opts *opts, void *stream);

/* The tile size and band a call with these options would use for order m (batched != 0:
 * as a pencil of rtgevc_batched: its band is opts->band, or 3 when that is 0).  The automatic choices come
 * from a table compiled into the library, written by an autotuning sweep on the GPU
 * (performance parameters only: every choice computes the same eigenvectors).
 * out receives mb, band, schedule, normalize, precision, the refinement sweeps in max_refine
 * (-1 when none run), refine_bits as given, split (tiles per launch; -1: one launch) and grid
 * as given.  Returns 0, -1 (m < 0),
 * -3 (invalid opts) or -4 (out is NULL).  Host only; touches no GPU. */
int rtgevc_resolve_opts(int64_t m, int32_t batched, const rtgevc_opts *opts, rtgevc_opts *out);

/* Human-readable text for a negative return code. */
const char *rtgevc_strerror(int code);

/* Library version, e.g. "0.1.0". */
const char *rtgevc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RTGEVC_H */
