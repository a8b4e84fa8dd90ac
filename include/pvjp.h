/*
 * pvjp.h -- C ABI of libpvjp.so: primal and reverse-mode (VJP) kernels for
 * bulk-parallel operators on AMD Instinct MI355X (gfx950).
 *
 * The rules follow Schenck, Roenning, Henriksen, Oancea, "AD for an Array
 * Language with Nested Parallelism" (arXiv 2202.10297).  A VJP entry point
 * computes x_bar = y_bar . J(x) for the operator at the point x (Sec. 2.0.2,
 * the definition of vjp), recomputing the primal values it needs per tile
 * instead of reading a tape (Sec. 4.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers named for arrays are DEVICE pointers, owned by the caller; the
 *    library never allocates, frees or retains them.  Scalars travel by value
 *    or, where a kernel produces or consumes them, as device pointers.
 *  - Arrays are contiguous, element-aligned, structure-of-arrays.  Indices are
 *    int32; element counts are int64.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Every call is
 *    asynchronous on that stream; a returned PVJP_OK means the launch was
 *    accepted, not that the kernels have finished.
 *  - `accumulate` != 0 selects the paper's adjoint update x_bar += contribution
 *    (Sec. 2.0.2, eq. rewrite-adj); 0 overwrites x_bar with the contribution.
 *  - Outputs must not alias inputs, except where an entry point says it works
 *    in place.
 *  - Workspaces: entry points that take (ws, ws_bytes) need device scratch of
 *    at least the size the matching *_ws_bytes() query returns.  A workspace
 *    must be zero-filled before its first use (pvjp_ws_clear, or any zeroing
 *    allocation); every call leaves it ready for the next call.  Two calls
 *    that may run concurrently must not share a workspace.
 *  - Errors: host-side validation (NULL pointers where data is needed,
 *    negative sizes, unknown op/dtype, workspace too small, index range
 *    limits) returns a non-zero status before any launch; launch failures
 *    return PVJP_EDEVICE.  pvjp_last_error() then describes the failure (text
 *    is per calling thread).  No C++ exception crosses this interface.
 *    Out-of-range indices in reduce_by_index and scatter are not errors: the
 *    element is ignored (its adjoint is zero).
 *  - FP32 entry points compute in FP32 except where stated (FP64 for sums and
 *    products of reductions); FP64 entry points compute in FP64.
 */
#ifndef PVJP_H
#define PVJP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int pvjp_status;
#define PVJP_OK 0
#define PVJP_EINVAL 1      /* bad argument (see pvjp_last_error) */
#define PVJP_ENOMEM 2      /* workspace too small */
#define PVJP_EDEVICE 3     /* HIP launch or runtime error */
#define PVJP_EUNSUPPORTED 4 /* valid but unsupported combination */

typedef enum { PVJP_F32 = 0, PVJP_F64 = 1 } pvjp_dtype;

/* Reduction operators of Sec. 5.1.1 and their neutral elements:
 * ADD 0, MUL 1, MIN +inf, MAX -inf. */
typedef enum { PVJP_ADD = 0, PVJP_MUL = 1, PVJP_MIN = 2, PVJP_MAX = 3 } pvjp_op;

/* Elementwise functions offered by the map entry points (Sec. 5.4). */
typedef enum {
    PVJP_FN_SQUARE = 0, /* x*x, the lambda of Sec. 4.1's example */
    PVJP_FN_EXP = 1,
    PVJP_FN_LOG = 2,
    PVJP_FN_SIN = 3,
    PVJP_FN_TANH = 4
} pvjp_fn;

/* Associative operators for reduce by the general rule of Sec. 5.1.1.  An
 * element has K components, each stored in its own array:
 *  LOGADDEXP (K=1): a (.) b = log(exp(a) + exp(b)), neutral -inf;
 *  LINREC    (K=2, a then b): (a1,b1) (.) (a2,b2) = (a2*a1, a2*b1 + b2),
 *            neutral (1, 0) (the operator of the scan of Sec. 5.2);
 *  MAT2      (K=4, row-major m00 m01 m10 m11): 2x2 matrix product in index
 *            order, y = x_0 x_1 ... x_{n-1}, neutral the identity. */
typedef enum { PVJP_GOP_LOGADDEXP = 0, PVJP_GOP_LINREC = 1, PVJP_GOP_MAT2 = 2 } pvjp_gop;

/* ------------------------------------------------------------------------ */
/* Library                                                                    */
/* ------------------------------------------------------------------------ */

/* Text of the last failure on the calling thread ("" if none). */
const char* pvjp_last_error(void);
/* Version string, e.g. "pvjp 0.1.0 gfx950". */
const char* pvjp_version(void);
/* Zero-fills ws_bytes of device memory at ws on `stream` (a kernel, not a
 * memset node, so it may be captured in a HIP graph). */
pvjp_status pvjp_ws_clear(void* ws, size_t ws_bytes, void* stream);

/* Synchronises `stream`, then reports whether a lookback kernel found the
 * workspace `ws` in a state the protocol never leaves it in (a ticket outside
 * its grid, or a predecessor tile that never published: both mean the
 * workspace was not zero-filled, or was shared by overlapping calls).  Such a
 * launch finishes without hanging but its results are invalid.  Returns
 * PVJP_OK if no error is recorded, PVJP_EDEVICE otherwise (pvjp_last_error()
 * names the condition); clear != 0 resets the recorded error. */
pvjp_status pvjp_ws_check(void* ws, int clear, void* stream);

/* ------------------------------------------------------------------------ */
/* Checked mode: device-side counts of inputs the method leaves undefined    */
/* ------------------------------------------------------------------------ */

/* Slots of the caller's counter block: int64 [PVJP_DIAG_N] in device memory,
 * 8-byte aligned, zeroed by the caller.  Each call ADDS its counts to the
 * block (one atomic add per launched block), so the block collects the
 * counts of many calls until the caller reads and clears it.  None of these
 * calls traps, changes its inputs or is needed by the operators: they are the
 * checks a caller runs beside the operators when it wants them. */
#define PVJP_DIAG_OOB 0 /* index outside [0, m) (reduce_by_index, Sec. 5.1.2; scatter targets outside [0, n)) */
#define PVJP_DIAG_DUP 1 /* scatter target that repeats (Sec. 5.3 assumes unique targets); each extra occurrence once */
#define PVJP_DIAG_NAN 2 /* NaN values */
#define PVJP_DIAG_INF 3 /* +-inf values */
#define PVJP_DIAG_N 4

/* counters[PVJP_DIAG_OOB] += #{i < n : inds[i] < 0 or inds[i] >= m}.
 * inds [n] int32 device. */
pvjp_status pvjp_diag_indices(const int32_t* inds, int64_t n, int64_t m, int64_t* counters, void* stream);
/* Bytes of the bitmap workspace of pvjp_diag_scatter: one bit per target. */
size_t pvjp_diag_scatter_ws_bytes(int64_t n);
/* For the m targets is [m] int32 into an array of n elements (n < 2^31):
 * counters[PVJP_DIAG_OOB] += targets outside [0, n);
 * counters[PVJP_DIAG_DUP] += occurrences of a target after its first.
 * ws: device scratch of pvjp_diag_scatter_ws_bytes(n) bytes, 4-byte aligned;
 * the call clears it itself (with a kernel, so it may be graph-captured). */
pvjp_status pvjp_diag_scatter(const int32_t* is, int64_t m, int64_t n, int64_t* counters, void* ws,
                              size_t ws_bytes, void* stream);
/* counters[PVJP_DIAG_NAN] += NaN elements of x [n] dtype;
 * counters[PVJP_DIAG_INF] += infinite elements. */
pvjp_status pvjp_diag_nonfinite(pvjp_dtype dtype, const void* x, int64_t n, int64_t* counters, void* stream);

/* ------------------------------------------------------------------------ */
/* Inclusive scan of the first-order linear recurrence (Sec. 5.2)             */
/*                                                                            */
/* Operator (a1,b1) (+) (a2,b2) = (a2*a1, a2*b1 + b2), neutral (1, 0):        */
/*   A[0] = a[0], B[0] = b[0]; A[i] = a[i]*A[i-1], B[i] = a[i]*B[i-1] + b[i]. */
/* Single-pass decoupled-lookback scan.                                       */
/* ------------------------------------------------------------------------ */

/* Elements per checkpoint: ckpt[c] holds the scan state before element
 * c * PVJP_LINREC_CKPT_INTERVAL, i.e. the exclusive prefix (A, B). */
#define PVJP_LINREC_CKPT_INTERVAL 1024
/* Number of checkpoint pairs for n elements: ceil(n / interval). */
int64_t pvjp_linrec_ckpt_len(int64_t n);

size_t pvjp_linrec_scan_ws_bytes(pvjp_dtype dtype, int64_t n);
/* a, b: input arrays [n] of dtype.  A, B: outputs [n] of dtype.
 * ckpt (nullable): output, 2 * pvjp_linrec_ckpt_len(n) elements of dtype laid
 * out as pairs (A, B).  A and B may be NULL together to compute only ckpt. */
pvjp_status pvjp_linrec_scan(pvjp_dtype dtype, const void* a, const void* b, int64_t n,
                             void* A, void* B, void* ckpt, void* ws, size_t ws_bytes,
                             void* stream);

size_t pvjp_linrec_scan_vjp_ws_bytes(pvjp_dtype dtype, int64_t n);
/* Reverse sweep of Sec. 5.2: c_i = a_{i+1} (the Jacobian of the operator in
 * its left argument is a_{i+1} * I), a reversed scan with
 * lin_o((d1,c1),(d2,c2)) = (d2 + c2*d1, c2*c1) giving
 * r_bar_i = y_bar_i + a_{i+1} * r_bar_{i+1}, then the map
 * a_bar_i = A_{i-1}*rA_bar_i + B_{i-1}*rB_bar_i, b_bar_i = rB_bar_i with
 * (A_{-1}, B_{-1}) = (1, 0).  The primal prefixes (A_{i-1}, B_{i-1}) are
 * recomputed per tile from `ckpt` (as written by pvjp_linrec_scan for the same
 * a, b, n); with ckpt == NULL a checkpoint-only primal pass into the
 * workspace runs first.  yA_bar, yB_bar: output adjoints [n]; a_bar, b_bar:
 * input adjoints [n]. */
pvjp_status pvjp_linrec_scan_vjp(pvjp_dtype dtype, const void* a, const void* b,
                                 const void* yA_bar, const void* yB_bar, int64_t n,
                                 const void* ckpt, void* a_bar, void* b_bar, int accumulate,
                                 void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * return sweep as pvjp_linrec_scan_vjp, with the same arguments except the
 * workspace, which is a fixed array inside the library (one per GPU, held
 * until the process ends, at most pvjp_linrec_scan_vjp_noalloc_max_bytes():
 * 8 MiB, enough for n up to 2^26 in FP64 and 2^27 in FP32).  Larger n
 * returns PVJP_ENOMEM before any launch.  No call allocates or frees memory.
 * Every call on one GPU shares that GPU's array: calls that may overlap on
 * one GPU (two streams, two threads) race and must be serialised by the
 * caller.  The stream's device is the one whose array is used. */
size_t pvjp_linrec_scan_vjp_noalloc_max_bytes(void);
pvjp_status pvjp_linrec_scan_vjp_noalloc(pvjp_dtype dtype, const void* a, const void* b,
                                         const void* yA_bar, const void* yB_bar, int64_t n,
                                         const void* ckpt, void* a_bar, void* b_bar, int accumulate,
                                         void* stream);

/* ------------------------------------------------------------------------ */
/* reduce (Sec. 5.1, special operators Sec. 5.1.1)                            */
/* ------------------------------------------------------------------------ */

size_t pvjp_reduce_ws_bytes(pvjp_op op, pvjp_dtype dtype, int64_t n);
/* y (device, 1 element of dtype) = x[0] op ... op x[n-1] (neutral if n == 0).
 *  MIN/MAX: arg (device int64, required) = lowest index attaining y, -1 if
 *           n == 0.
 *  MUL:     p (device, 1 element of dtype, required) = product of the non-zero
 *           elements, z (device int64, required) = number of zeros (-0.0
 *           counts); y = p if z == 0 else 0.  The product is formed in FP64.
 *  ADD:     the sum is formed in FP64.
 * Deterministic: the same input gives the same bits. */
pvjp_status pvjp_reduce(pvjp_op op, pvjp_dtype dtype, const void* x, int64_t n, void* y,
                        int64_t* arg, void* p, int64_t* z, void* ws, size_t ws_bytes,
                        void* stream);
/* x_bar (+)= contribution, with y_bar a device scalar of dtype:
 *  ADD: y_bar everywhere;
 *  MUL: z == 0: p / x_i * y_bar;  z == 1: p * y_bar at the zero, 0 elsewhere;
 *       z >= 2: 0  (p, z from pvjp_reduce);
 *  MIN/MAX: y_bar at arg, 0 elsewhere (with accumulate only x_bar[arg] is
 *       touched). */
pvjp_status pvjp_reduce_vjp(pvjp_op op, pvjp_dtype dtype, const void* x, int64_t n,
                            const int64_t* arg, const void* p, const int64_t* z,
                            const void* y_bar, void* x_bar, int accumulate, void* stream);

/* ------------------------------------------------------------------------ */
/* reduce_by_index / histogram (Sec. 5.1.2)                                   */
/* hs = replicate m e; for i: hs[inds[i]] op= vs[i]   (inds outside [0,m)      */
/* are skipped).                                                              */
/* ------------------------------------------------------------------------ */

/* Workspace bytes for pvjp_hist (device memory, zero-initialised once by the
 * caller, owned by the caller, reusable across calls on one stream).  Small
 * m (the bins fit one block's LDS): per-block partial histograms, O(m) with
 * a few hundred rows.  FP32 + / min / max with m beyond that and at most
 * 2^22 bins: the bucket-partitioned path, which sorts every tile of 8192
 * elements by bucket and stores per element the value (4 bytes) and its bin
 * in the bucket (+: 2 bytes; min/max: 4 bytes with the position in the
 * tile): about 8n bytes plus per-tile bucket offsets and per-item partials. */
size_t pvjp_hist_ws_bytes(pvjp_op op, pvjp_dtype dtype, int64_t n, int64_t m);
/* Which path pvjp_hist takes for (op, dtype, n, m, counts != 0), for tests
 * and tuning: info[0] = PVJP_HIST_PATH_*; for the partitioned path info[1] =
 * bins per bucket, info[2] = most records one work item of a bucket takes
 * (a bucket with more is split into several items, merged afterwards), info[3]
 * = number of buckets; 0 otherwise.  info: int64 [4] host memory. */
#define PVJP_HIST_PATH_LDS 0       /* every bin in each block's LDS, per-block partials merged */
#define PVJP_HIST_PATH_CACHE 1     /* LDS cache of bins in front of device-memory atomics */
#define PVJP_HIST_PATH_PARTITION 2 /* records sorted into buckets of bins, each bucket accumulated in LDS */
pvjp_status pvjp_hist_plan_info(pvjp_op op, pvjp_dtype dtype, int64_t n, int64_t m, int counts, int64_t* info);
/* inds [n] int32, vs [n] dtype, 1 <= m <= 2^30, n < 2^31.
 * hs [m] dtype (required).
 * winner [m] int32 (MIN/MAX, required): lowest i with inds[i] == k and
 *        vs[i] == hs[k]; -1 for an empty bin.  hs[k] is vs[winner[k]] bit for
 *        bit (so a -0.0 extreme keeps its sign).
 * p [m] dtype and z [m] int32 (MUL, required): product of the non-zero values
 *        of the bin (formed in FP64) and their zero count; hs = p or 0.
 * count [m] int32 (nullable, any op): elements per bin.
 * ADD sums are accumulated in FP64. */
pvjp_status pvjp_hist(pvjp_op op, pvjp_dtype dtype, const int32_t* inds, const void* vs,
                      int64_t n, int64_t m, void* hs, int32_t* winner, void* p, int32_t* z,
                      int32_t* count, void* ws, size_t ws_bytes, void* stream);
/* vs_bar (+)= contribution of hs_bar [m]:
 *  ADD: hs_bar[inds[i]] (a gather);
 *  MIN/MAX: hs_bar[k] at i == winner[k], 0 elsewhere (with accumulate only
 *       the m winners are touched; without, vs_bar is zero-filled first);
 *  MUL: per bin, the three cases of reduce(MUL) with y_bar = hs_bar[k];
 *       needs vs, p and z.
 *  vs may be NULL for ADD/MIN/MAX; winner is needed for MIN/MAX only. */
pvjp_status pvjp_hist_vjp(pvjp_op op, pvjp_dtype dtype, const int32_t* inds, const void* vs,
                          int64_t n, int64_t m, const int32_t* winner, const void* p,
                          const int32_t* z, const void* hs_bar, void* vs_bar, int accumulate,
                          void* stream);

/* ------------------------------------------------------------------------ */
/* scatter (Sec. 5.3)                                                         */
/* ------------------------------------------------------------------------ */

/* In place on xs [n]: xs_saved[j] = xs[is[j]]; then xs[is[j]] = vs[j], for
 * j < m.  `is` must hold no duplicates (duplicates race; the result is then
 * unspecified); entries outside [0,n) are skipped (xs_saved[j] = 0).
 * xs_saved [m] dtype (nullable if the caller will not restore). */
pvjp_status pvjp_scatter(pvjp_dtype dtype, void* xs, int64_t n, const int32_t* is,
                         const void* vs, int64_t m, void* xs_saved, void* stream);
/* Return sweep, in place on ys_bar [n], fused into one kernel:
 *  vs_bar[j] (+)= ys_bar[is[j]]    (a gather),
 *  ys_bar[is[j]] = 0               (ys_bar becomes xs_bar),
 *  if ys != NULL: ys[is[j]] = xs_saved[j]  (restores xs in place). */
pvjp_status pvjp_scatter_vjp(pvjp_dtype dtype, void* ys_bar, int64_t n, const int32_t* is,
                             int64_t m, void* vs_bar, int accumulate, void* ys,
                             const void* xs_saved, void* stream);

/* Scatter over a target-ordered plan (Sec. 5.3; the forward sweep returns an
 * auxiliary result besides the scattered array).  Same semantics as
 * pvjp_scatter / pvjp_scatter_vjp, different memory behaviour: the forward
 * sweep groups the m updates by window of 32 KiB of the target array (a
 * two-pass bucket sort) and writes that grouping, together with the
 * overwritten values, into `plan`; both sweeps then move the target arrays
 * only as whole windows staged in LDS instead of one random access per
 * update.  The return sweep reads the plan instead of `is`.
 *
 * plan: caller-owned device memory of pvjp_scatter_plan_bytes(dtype, n, m)
 *   bytes, 256-byte aligned; written by pvjp_scatter_planned, read by
 *   pvjp_scatter_planned_vjp for the same (dtype, n, m) and unchanged `is`.
 *   It needs no clearing.  Sizes: n, m < 2^31; n <= 2^31 - 1 for FP32 and
 *   n <= 2^30 for FP64 (pvjp_scatter_plan_bytes returns 0 outside).
 * Targets must be unique (repeats race, as for pvjp_scatter); targets
 * outside [0, n) are dropped: they change nothing and their adjoint is 0. */
size_t pvjp_scatter_plan_bytes(pvjp_dtype dtype, int64_t n, int64_t m);
/* In place on xs [n]: xs[is[j]] = vs[j] for j < m; the overwritten values
 * are kept in the plan. */
pvjp_status pvjp_scatter_planned(pvjp_dtype dtype, void* xs, int64_t n, const int32_t* is,
                                 const void* vs, int64_t m, void* plan, size_t plan_bytes,
                                 void* stream);
/* Return sweep, in place on ys_bar [n]:
 *  vs_bar[j] (+)= ys_bar[is[j]], then ys_bar[is[j]] = 0 (ys_bar becomes
 *  xs_bar); if ys != NULL also ys[is[j]] = the value the forward sweep
 *  overwrote (restores xs in place).  vs_bar [m]. */
pvjp_status pvjp_scatter_planned_vjp(pvjp_dtype dtype, void* ys_bar, int64_t n, int64_t m,
                                     void* vs_bar, int accumulate, void* ys, const void* plan,
                                     size_t plan_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* map (Sec. 5.4): y_i = f(x_i); the VJP recomputes f's intermediates inside  */
/* the lambda instead of reading them from memory (Sec. 4.1).                  */
/* ------------------------------------------------------------------------ */

pvjp_status pvjp_map(pvjp_fn fn, pvjp_dtype dtype, const void* x, int64_t n, void* y,
                     void* stream);
/* x_bar (+)= f'(x_i) * y_bar_i. */
pvjp_status pvjp_map_vjp(pvjp_fn fn, pvjp_dtype dtype, const void* x, const void* y_bar,
                         int64_t n, void* x_bar, int accumulate, void* stream);
/* The program of Fig. 1 mapped over n pairs: (y0, y1) = (x1*sin(x0), x0*x1). */
pvjp_status pvjp_fig1(pvjp_dtype dtype, const void* x0, const void* x1, int64_t n, void* y0,
                      void* y1, void* stream);
/* Its adjoint, Fig. 1(c): x0_bar (+)= x1*y1_bar + cos(x0)*x1*y0_bar,
 * x1_bar (+)= x0*y1_bar + sin(x0)*y0_bar. */
pvjp_status pvjp_fig1_vjp(pvjp_dtype dtype, const void* x0, const void* x1, const void* y0_bar,
                          const void* y1_bar, int64_t n, void* x0_bar, void* x1_bar,
                          int accumulate, void* stream);

/* ------------------------------------------------------------------------ */
/* reduce with a general associative operator (Sec. 5.1.1, general rule):     */
/* y = x_0 (.) ... (.) x_{n-1}.  Its VJP maps                                  */
/*   x_bar_i (+)= (d(ls_i (.) x_i (.) rs_i)/dx_i)^T y_bar                      */
/* over the exclusive prefix folds ls and exclusive suffix folds rs, which     */
/* are recomputed from x (no tape).  Element i is (x[0][i], .., x[K-1][i]).   */
/* ------------------------------------------------------------------------ */

/* K of an operator (1, 2 or 4); 0 for an unknown operator. */
int pvjp_gop_components(pvjp_gop op);
/* Workspace bytes for both entry points (device memory owned by the caller,
 * 256-byte aligned, no initialisation needed): 96 bytes per tile of 2048
 * (FP32) or 1024 (FP64) elements and per group of 64 tiles. */
size_t pvjp_reduce_generic_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n);
/* Bytes of the optional per-tile checkpoint: 32 per tile (the tile folds). */
size_t pvjp_reduce_generic_ckpt_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n);
/* x: host array of K device pointers to n elements each (unused if n == 0).
 * y: host array of K device pointers to one element of dtype each; receives
 * the fold (the neutral element if n == 0).  ckpt (device, nullable, 16-byte
 * aligned, pvjp_reduce_generic_ckpt_bytes): receives the fold of every tile,
 * which lets the VJP skip its first pass over x.  Deterministic: fixed tiles and
 * a fixed combination tree.  LOGADDEXP inputs must be finite or -inf.  With
 * FP32 data the LINREC and MAT2 folds are formed in FP64 (LOGADDEXP in FP32). */
pvjp_status pvjp_reduce_generic(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                void* const* y, void* ckpt, void* ws, size_t ws_bytes, void* stream);
/* ckpt: NULL (the tile folds are recomputed from x) or the checkpoint that
 * pvjp_reduce_generic wrote for this x, op, dtype and n (then x is read once).
 * y_bar: host array of K device pointers to one element each; x_bar: host
 * array of K device pointers to n elements each, overwritten (accumulate = 0)
 * or added to.  LOGADDEXP: x_bar_i = y_bar * exp(x_i - (ls_i (.) x_i (.)
 * rs_i)), and 0 where x_i = -inf.  LINREC, with ls_i = (Al, Bl) and
 * rs_i = (Ar, Br): a_bar_i = Ar*(y_bar_A*Al + y_bar_B*Bl), b_bar_i =
 * Ar*y_bar_B.  MAT2: A_bar_i = ls_i^T Y_bar rs_i^T.  Passes: tile folds
 * (skipped with a checkpoint), group folds, one block scanning the groups
 * both ways, per-tile prefixes and suffixes, then per tile the in-tile folds
 * and f (x read once with a checkpoint, twice without; x_bar written once). */
pvjp_status pvjp_reduce_generic_vjp(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                    const void* ckpt, const void* const* y_bar, void* const* x_bar,
                                    int accumulate, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Inclusive scan with a general associative operator (Sec. 5.2 and its      */
/* Jacobian generalisation): y_i = x_0 (.) ... (.) x_i, same operators and    */
/* layout as the general reduce.  The VJP is the reversed scan of lin_o over  */
/* (d-vector, d x d matrix) pairs (y_bar_i, J_left(i)^T), with                */
/* J_left(i) = d(y_i (.) x_{i+1})/dy_i, followed by x_bar_i (+)=              */
/* J_right(i)^T r_i with J_right(i) = d(y_{i-1} (.) x_i)/dx_i; d = K and the  */
/* Jacobians are formed as explicit d x d matrices.  Primal values are        */
/* recomputed per tile from the checkpoint, never read back.                  */
/* ------------------------------------------------------------------------ */

/* Workspace bytes (device memory owned by the caller, 256-byte aligned, no
 * initialisation needed): per tile (2048 FP32 / 1024 FP64 elements for
 * LOGADDEXP, 1024 for LINREC, 512 for MAT2) two 32-byte states and two
 * 160-byte lin_o states, and as much again per group of 64 tiles. */
size_t pvjp_scan_generic_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n);
/* Bytes of the per-tile checkpoint: 32 per tile (the fold of everything
 * before the tile). */
size_t pvjp_scan_generic_ckpt_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n);
/* x, y: host arrays of K device pointers to n elements each.  ckpt (device,
 * nullable, 16-byte aligned): receives the per-tile checkpoint.  FP32 LINREC
 * and MAT2 scans are formed in FP64 and rounded once per output. */
pvjp_status pvjp_scan_generic(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                              void* const* y, void* ckpt, void* ws, size_t ws_bytes, void* stream);
/* y_bar, x_bar: host arrays of K device pointers to n elements each; x_bar
 * is overwritten (accumulate = 0) or added to.  ckpt: NULL (the tile
 * prefixes are recomputed from x first) or the checkpoint pvjp_scan_generic
 * wrote for this x, op, dtype and n.  Passes: lin_o tile folds (x and y_bar
 * read), group folds, one block scanning the groups backwards, per-tile
 * suffixes, then per tile the adjoints (x and y_bar read, x_bar written).
 * LOGADDEXP: elements equal to -inf get adjoint 0. */
pvjp_status pvjp_scan_generic_vjp(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t n,
                                  const void* ckpt, const void* const* y_bar, void* const* x_bar,
                                  int accumulate, void* ws, size_t ws_bytes, void* stream);

/* Regular segmented scan (Sec. 5.2, the vectorised-operator rule): B
 * independent inclusive scans of L elements each with the same operator,
 * segment b at offset b L of every component array (so x[c] and y[c] are [B x
 * L] row-major, one scan per row).  A scan whose operator is applied
 * componentwise to vectors of w elements, over n such vectors stored [n x w],
 * is this call on the transposed [w x n] arrays (B = w, L = n), which is the
 * paper's rewrite of such a scan into transpose, a map of scans, transpose.
 * The primal and the VJP are those of pvjp_scan_generic(_vjp) per row, in one
 * launch sequence for all rows (rows ride on the grid's second dimension);
 * the VJP's reversed lin_o scan starts afresh at each row's last element.
 * 1 <= B <= 65535; the checkpoint holds B times the single-scan tile
 * prefixes.  The 16-byte vector path is taken when every row starts 16-byte
 * aligned (L * element size a multiple of 16 and 16-byte aligned arrays). */
size_t pvjp_scan_generic_batched_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t B, int64_t L);
size_t pvjp_scan_generic_batched_ckpt_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t B, int64_t L);
pvjp_status pvjp_scan_generic_batched(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t B, int64_t L,
                                      void* const* y, void* ckpt, void* ws, size_t ws_bytes, void* stream);
pvjp_status pvjp_scan_generic_batched_vjp(pvjp_gop op, pvjp_dtype dtype, const void* const* x, int64_t B,
                                          int64_t L, const void* ckpt, const void* const* y_bar,
                                          void* const* x_bar, int accumulate, void* ws, size_t ws_bytes,
                                          void* stream);

/* ------------------------------------------------------------------------ */
/* Forward mode (Sec. 3): Jacobian-vector products.  Each primal is bundled   */
/* with its tangent and the operator runs on the pairs (the dual-number form  */
/* of the tangent rewrite rule).  Tangents (x_dot, ...) have the primal's     */
/* layout and dtype; outputs are overwritten.                                 */
/* ------------------------------------------------------------------------ */

/* y_dot_i = f'(x_i) x_dot_i (the elementwise Jacobian is diagonal: this is
 * the VJP kernel with x_dot in place of y_bar). */
pvjp_status pvjp_map_jvp(pvjp_fn fn, pvjp_dtype dtype, const void* x, const void* x_dot, int64_t n,
                         void* y_dot, void* stream);
/* y_dot (device, 1 element) of y = reduce(op) x, with the auxiliary outputs
 * of pvjp_reduce on the same x:
 *  ADD: sum of x_dot (FP64 accumulation, ws as for pvjp_reduce);
 *  MUL: p * sum x_dot_i / x_i (z == 0), p * x_dot at the zero (z == 1), 0
 *       (z >= 2); needs x, p, z and ws as for pvjp_reduce;
 *  MIN/MAX: x_dot[arg] (0 if n == 0); ws unused. */
pvjp_status pvjp_reduce_jvp(pvjp_op op, pvjp_dtype dtype, const void* x, const void* x_dot, int64_t n,
                            const int64_t* arg, const void* p, const int64_t* z, void* y_dot, void* ws,
                            size_t ws_bytes, void* stream);
/* Workspace bytes of pvjp_hist_jvp (ADD only: that of pvjp_hist(ADD)). */
size_t pvjp_hist_jvp_ws_bytes(pvjp_op op, pvjp_dtype dtype, int64_t n, int64_t m);
/* hs_dot [m] of hs = reduce_by_index(op):
 *  ADD: reduce_by_index(+) of vs_dot over the same inds (ws as pvjp_hist);
 *  MIN/MAX: vs_dot[winner[k]], 0 for an empty bin (winner from pvjp_hist);
 *  MUL: PVJP_EUNSUPPORTED. */
pvjp_status pvjp_hist_jvp(pvjp_op op, pvjp_dtype dtype, const int32_t* inds, const void* vs_dot,
                          int64_t n, int64_t m, const int32_t* winner, void* hs_dot, void* ws,
                          size_t ws_bytes, void* stream);
/* In place on ys_dot [n] (x_dot on entry): ys_dot[is[j]] = vs_dot[j] (the
 * primal scatter of the tangents; same index rules as pvjp_scatter). */
pvjp_status pvjp_scatter_jvp(pvjp_dtype dtype, void* ys_dot, int64_t n, const int32_t* is,
                             const void* vs_dot, int64_t m, void* stream);
/* Reduce / inclusive scan with a general operator on (x, x_dot) pairs: the
 * primal y and its tangent y_dot in one pass (K components each; for the scan
 * K arrays of n).  log-add-exp carries (max, scaled sum, scaled tangent sum);
 * the linear recurrence (A, B, A_dot, B_dot); the 2x2 product (X, X_dot) with
 * X_dot Y + X Y_dot.  Workspaces: the queries below (no initialisation). */
size_t pvjp_reduce_generic_jvp_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n);
size_t pvjp_scan_generic_jvp_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n);
pvjp_status pvjp_reduce_generic_jvp(pvjp_gop op, pvjp_dtype dtype, const void* const* x,
                                    const void* const* x_dot, int64_t n, void* const* y,
                                    void* const* y_dot, void* ws, size_t ws_bytes, void* stream);
pvjp_status pvjp_scan_generic_jvp(pvjp_gop op, pvjp_dtype dtype, const void* const* x,
                                  const void* const* x_dot, int64_t n, void* const* y,
                                  void* const* y_dot, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Segmented batches: many instances of uneven length stored back to back     */
/* (segment s = elements [offsets[s], offsets[s+1])), each processed as one   */
/* segmented operation per launch.  This generalises the rule of Sec. 5.2     */
/* that turns a vectorised scan into a regular-segmented scan to irregular    */
/* segments.  Segments must be non-empty.                                     */
/* ------------------------------------------------------------------------ */

/* Workspace for `total` elements in `nseg` segments with tiles of
 * tile_elems (1024, 2048 or 4096 elements per tile). */
size_t pvjp_seg_ws_bytes(int64_t total, int64_t nseg, int tile_elems);
/* Validates the HOST offsets [nseg+1] (offsets[0] = 0, strictly increasing)
 * and uploads the segment tables into ws (synchronises `stream`).  Later calls
 * with this ws must pass the same total (= offsets[nseg]), nseg and
 * tile_elems.  The lookback header in ws is left as pvjp_ws_clear leaves it
 * only if ws was zero-filled before. */
pvjp_status pvjp_seg_prepare(const int64_t* host_offsets, int64_t nseg, int tile_elems, void* ws,
                             size_t ws_bytes, void* stream);
/* Every segment's linear-recurrence scan (Sec. 5.2) in one decoupled-lookback
 * launch with the segmented operator; A, B (nullable together) and ckpt
 * (nullable; 2 * pvjp_linrec_ckpt_len(total) elements: the state before each
 * global multiple of the checkpoint interval) as for pvjp_linrec_scan. */
pvjp_status pvjp_seg_linrec_scan(pvjp_dtype dtype, const void* a, const void* b, int64_t total,
                                 int64_t nseg, int tile_elems, void* A, void* B, void* ckpt, void* ws,
                                 size_t ws_bytes, void* stream);
/* One persistent launch of `grid_blocks` workgroups that pulls work from a
 * queue: the reverse sweep of every segment's scan (as pvjp_linrec_scan_vjp,
 * needs the segmented ckpt) and, when sum_ybar is given, the adjoint of a
 * sum-reduce per segment, sum_xbar[i] (+)= sum_ybar[segment of i]
 * (Sec. 5.1.1).  Either part may be omitted (a == NULL, or sum_ybar ==
 * sum_xbar == NULL).  Safe to capture in a HIP graph and replay. */
pvjp_status pvjp_seg_batch_vjp(pvjp_dtype dtype, const void* a, const void* b, const void* yA_bar,
                               const void* yB_bar, int64_t total, int64_t nseg, int tile_elems,
                               const void* ckpt, void* a_bar, void* b_bar, const void* sum_ybar,
                               void* sum_xbar, int accumulate, int grid_blocks, void* ws,
                               size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* Gaussian-mixture log-likelihood and its gradient (the workload of          */
/* Sec. 7.6; accumulators turned into contractions as in Sec. 6.1)            */
/*                                                                            */
/* The paper measures this objective without stating it; the definition here  */
/* is the textbook mixture with a precision-Cholesky parametrisation:         */
/*   Q_k = diag(exp(q_k)) + L_k, L_k strictly lower with entry (r, c), r > c,  */
/*         at l[k*D(D-1)/2 + r(r-1)/2 + c];                                    */
/*   s_ik = alpha_k + sum_d q_kd - 0.5 * |Q_k (x_i - mu_k)|^2;                 */
/*   loglik = sum_i LSE_k(s_ik) - N*LSE(alpha) - (N*D/2)*log(2*pi).            */
/* X: N x D row-major FP32 (16-byte aligned); alpha [K]; mu, q: K x D; l:      */
/* K x D(D-1)/2; all FP32.  D must be 32 or 64 (PVJP_EUNSUPPORTED otherwise).  */
/* The contraction Q_k (x_i - mu_k) runs on FP32 MFMA; |z|^2, the log-sum-exp  */
/* and all cross-tile sums are FP64.                                           */
/* ------------------------------------------------------------------------ */

size_t pvjp_gmm_ws_bytes(int64_t N, int D, int K);
/* loglik: device double (output).  lse: device double[N] (nullable output):
 * the per-point LSE_k(s_ik), the checkpoint the reverse sweep reads.
 * s: device double[K x N] (nullable output, component-major: s[k*N + i]):
 * every s_ik, an optional second checkpoint (8 N K bytes) that halves the
 * reverse sweep's contraction work. */
pvjp_status pvjp_gmm_objective(const float* X, int64_t N, int D, int K, const float* alpha,
                               const float* mu, const float* q, const float* l, double* loglik,
                               double* lse, double* s, void* ws, size_t ws_bytes, void* stream);
/* Reverse sweep with output adjoint ell_bar: alpha_bar [K], mu_bar and q_bar
 * [K x D], l_bar [K x D(D-1)/2] (FP32 outputs, (+)=).  lse: the checkpoint
 * written by pvjp_gmm_objective for the same inputs (nullable: the forward
 * sweep then runs first into the workspace).  s (nullable; needs lse): the
 * s_ik checkpoint of the same call.  Without s the weights w_ik = ell_bar *
 * exp(s_ik - LSE_i) are recomputed with z_ik = Q_k (x_i - mu_k) and the
 * sweep contracts G_k = sum_i w_ik z_ik (x_i - mu_k)^T; with s it contracts
 * S_k = sum_i w_ik (x_i - mu_k)(x_i - mu_k)^T and forms G_k = Q_k S_k. */
pvjp_status pvjp_gmm_vjp(const float* X, int64_t N, int D, int K, const float* alpha,
                         const float* mu, const float* q, const float* l, double ell_bar,
                         const double* lse, const double* s, float* alpha_bar, float* mu_bar,
                         float* q_bar, float* l_bar, int accumulate, void* ws, size_t ws_bytes,
                         void* stream);

/* ------------------------------------------------------------------------ */
/* Dense k-means (Sec. 7.4): f(C) = sum_i min_k |x_i - c_k|^2 (squared        */
/* distance), X [N x D] and C [K x D] row-major FP32, 1 <= D <= 1024.         */
/* Distances are the FP64 chain acc = fma(x_d - c_d, x_d - c_d, acc) over     */
/* d = 0..D-1; the nearest centre is the lowest k among equal distances.      */
/* ------------------------------------------------------------------------ */

/* Workspace bytes for both entry points (device, caller-owned, 256-byte
 * aligned, no initialisation needed). */
size_t pvjp_kmeans_ws_bytes(int64_t N, int D, int K);
/* assign [N] int32 (output, the primal's auxiliary result: each point's
 * nearest centre); f: device double (output), summed in a fixed order. */
pvjp_status pvjp_kmeans_objective(const float* X, int64_t N, int D, const float* C, int K,
                                  int32_t* assign, double* f, void* ws, size_t ws_bytes, void* stream);
/* Reverse sweep with output adjoint f_bar and the assignments of
 * pvjp_kmeans_objective (the search is not repeated):
 *   C_bar_k (+)= 2 f_bar (n_k c_k - S_k),  S_k = sum_{a_i = k} x_i, n_k the
 *   number of points of centre k (accumulated in FP64, fixed order).
 * Forward over reverse (nullable pair): with C_dot [K x D], hvp (+)= the jvp
 * of this VJP in direction C_dot, 2 f_bar n_k C_dot_k (the Hessian is
 * diagonal: C_dot = 1 gives its diagonal, and C - C_bar / diagonal is the
 * Newton step). */
pvjp_status pvjp_kmeans_vjp(const float* X, int64_t N, int D, const float* C, int K,
                            const int32_t* assign, double f_bar, float* C_bar, const float* C_dot,
                            float* hvp, int accumulate, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* map over a free array (Sec. 5.4; accumulators lowered as in Sec. 6)        */
/* ------------------------------------------------------------------------ */

typedef enum { PVJP_GMAP_GATHER = 0, PVJP_GMAP_MUL = 1, PVJP_GMAP_SQDIFF = 2 } pvjp_gmap_op;

/* ys[i] = f(as[is[i]], vs[i]) for i < m, the body of a map that reads the
 * free array as [n] at computed indices: GATHER f = a (vs unused, may be
 * NULL), MUL f = a v, SQDIFF f = (a - v)^2.  An index outside [0, n) reads 0.
 * as, vs, ys: dtype; is: int32 [m].  No workspace. */
pvjp_status pvjp_gather_map(int op, pvjp_dtype dtype, const void* as, int64_t n, const int32_t* is,
                            const void* vs, int64_t m, void* ys, void* stream);
/* Bytes of workspace for pvjp_gather_map_vjp (device memory, zero-initialised
 * once by the caller, owned by the caller, reusable across calls on one
 * stream). */
size_t pvjp_gather_map_ws_bytes(pvjp_dtype dtype, int64_t n, int64_t m);
/* Return sweep.  The reads of the free array become an accumulator (Sec.
 * 5.4): as_bar[is[i]] (+)= sum over i of (df/da)(as[is[i]], vs[i]) ys_bar[i];
 * per element vs_bar[i] (+)= (df/dv) ys_bar[i] (not written for GATHER,
 * where vs_bar may be NULL).  accumulate != 0 adds into as_bar and vs_bar,
 * else overwrites them (as_bar is written for every k < n, 0 where nothing
 * was read).  Indices outside [0, n) update nothing.  The partials are
 * summed in FP64: in LDS bins per block when n <= 16384, the blocks' bins
 * then added in a fixed order; otherwise each element's partial (rounded to
 * dtype) goes through the reduce_by_index(+) path (pvjp_hist), whose bin
 * caches and bucket partitioning keep hot indices off contended atomics.
 * Atomic order varies, so as_bar may differ between calls in the last bits.
 * ws: 256-byte aligned, ws_bytes >= pvjp_gather_map_ws_bytes(dtype, n, m),
 * else PVJP_ENOMEM. */
pvjp_status pvjp_gather_map_vjp(int op, pvjp_dtype dtype, const void* as, int64_t n, const int32_t* is,
                                const void* vs, int64_t m, const void* ys_bar, void* as_bar, void* vs_bar,
                                int accumulate, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* sparse k-means (Sec. 7.5)                                                  */
/* ------------------------------------------------------------------------ */

/* f = sum_i min_k |x_i - c_k|^2 for points in CSR (rowptr [N+1] int64 from 0
 * to nnz, non-decreasing; col [nnz] int32 in [0, D); val [nnz] FP32) and
 * dense centres C [K x D] FP32 row-major, 1 <= K <= 64, K D <= 2^30.
 * Distances are the FP64 chain acc = |c_k|^2 (1024-dimension fma-chain
 * blocks added in order), then acc = fma(x, x - 2 c_kj, acc) over the row's
 * stored entries in order; ties go to the lowest k, so the assignments match
 * any implementation of that chain bit for bit.  assign [N] int32 (output);
 * f: one double.  Entries outside [0, nnz) and columns outside [0, D) are
 * skipped rather than read.  ws: 256-byte aligned, ws_bytes >=
 * pvjp_sparse_kmeans_ws_bytes(N, D, K, nnz), else PVJP_ENOMEM. */
size_t pvjp_sparse_kmeans_ws_bytes(int64_t N, int64_t D, int K, int64_t nnz);
pvjp_status pvjp_sparse_kmeans_objective(const int64_t* rowptr, const int32_t* col, const float* val, int64_t N,
                                         int64_t D, int64_t nnz, const float* C, int K, int32_t* assign, double* f,
                                         void* ws, size_t ws_bytes, void* stream);
/* VJP at the objective's assignments: C_bar (+)= 2 f_bar (n_k c_k - S_k),
 * S_k the sum of the rows assigned to k (every stored entry accumulated into
 * bin (a_i, j) on the reduce_by_index(+) path, FP64 sums); with C_dot, also
 * the jvp of the VJP hvp (+)= 2 f_bar n_k C_dot_k (C_dot = 1: the Hessian
 * diagonal).  C_dot and hvp are both NULL or both set. */
pvjp_status pvjp_sparse_kmeans_vjp(const int64_t* rowptr, const int32_t* col, const float* val, int64_t N,
                                   int64_t D, int64_t nnz, const float* C, int K, const int32_t* assign,
                                   double f_bar, float* C_bar, const float* C_dot, float* hvp, int accumulate,
                                   void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------ */
/* reduce_by_index with the log-add-exp operator (Sec. 5.1.2 with the general  */
/* rule of Sec. 5.1.1 inside each bin)                                        */
/* ------------------------------------------------------------------------ */

/* hs[b] = log sum over i with inds[i] = b of e^(x[i]); -inf for an empty bin
 * or one of -inf elements only; inds outside [0, m) skipped.  x, hs: dtype;
 * inds [n] int32; 1 <= m <= 2^30.  Runs the reduce_by_index max and +
 * paths (FP64 sums of the shifted exponentials).  ws: 256-byte aligned,
 * ws_bytes >= pvjp_hist_lae_ws_bytes(dtype, n, m), else PVJP_ENOMEM. */
size_t pvjp_hist_lae_ws_bytes(pvjp_dtype dtype, int64_t n, int64_t m);
pvjp_status pvjp_hist_lae(pvjp_dtype dtype, const int32_t* inds, const void* x, int64_t n, int64_t m, void* hs,
                          void* ws, size_t ws_bytes, void* stream);
/* x_bar[i] (+)= hs_bar[b] e^(x[i] - hs[b]) for b = inds[i] (the operator
 * commutes, so the general rule's ls (.) x (.) rs is the bin's total); 0 for
 * a -inf element or an index out of range.  hs: the primal's output. */
pvjp_status pvjp_hist_lae_vjp(pvjp_dtype dtype, const int32_t* inds, const void* x, int64_t n, int64_t m,
                              const void* hs, const void* hs_bar, void* x_bar, int accumulate, void* stream);

/* ------------------------------------------------------------------------ */
/* reduce_by_index with a general associative operator (Sec. 5.1.2 with the   */
/* general rule of Sec. 5.1.1 inside each bin); the operator need not commute */
/* ------------------------------------------------------------------------ */

/* hs[b] = x_{i_1} (.) x_{i_2} (.) ... over the elements with inds[i] = b in
 * increasing index order i_1 < i_2 < ...; the neutral element for an empty
 * bin; indices outside [0, m) are skipped.  Operators and the component
 * layout are those of pvjp_reduce_generic (x, hs: host arrays of K device
 * pointers, to n and m elements of dtype); inds [n] int32; 1 <= m <= 2^24,
 * n < 2^31.  The elements are stably sorted by bin, each bin is folded by a
 * segmented scan; folds in FP64 for both dtypes.  ws: device memory owned by
 * the caller, 256-byte aligned, no initialisation needed, at least
 * pvjp_hist_generic_ws_bytes bytes (else PVJP_ENOMEM): about 2 (r + 4) n
 * bytes, r = 8 + K s rounded up to a multiple of 16 for elements of s bytes
 * (two buffers of sort records -- bin, element index and the element's
 * components -- and two of their keys alone), plus per-chunk digit counts
 * and per-tile states.  Deterministic. */
size_t pvjp_hist_generic_ws_bytes(pvjp_gop op, pvjp_dtype dtype, int64_t n, int64_t m);
pvjp_status pvjp_hist_generic(pvjp_gop op, pvjp_dtype dtype, const int32_t* inds, const void* const* x, int64_t n,
                              int64_t m, void* const* hs, void* ws, size_t ws_bytes, void* stream);
/* x_bar_i (+)= (d(ls_i (.) x_i (.) rs_i)/dx_i)^T hs_bar[b] for b = inds[i],
 * with ls_i and rs_i the folds of the bin's elements before and after i (the
 * reduce rule inside each bin, y_bar = the bin's hs_bar); 0 for an index out
 * of range.  hs_bar: K device pointers to m elements; x_bar: K device
 * pointers to n elements, overwritten (accumulate = 0) or added to. */
pvjp_status pvjp_hist_generic_vjp(pvjp_gop op, pvjp_dtype dtype, const int32_t* inds, const void* const* x,
                                  int64_t n, int64_t m, const void* const* hs_bar, void* const* x_bar,
                                  int accumulate, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PVJP_H */
