/*
 * nnca.h -- C ABI of the MI355X (gfx950) library for the NNCA-based H2
 * matrix-vector product of Gujjula & Ambikasaran, "A new Nested Cross
 * Approximation".
 *
 * The operator is A_ij = K(p_i, p_j) over one point set P = Q in 2D or 3D
 * (Sec. 1; the symmetric case of Sec. 5), or A_ij = K(p_i, q_j) between
 * targets P and sources Q (nnca_build_general, Sec. 2.1-2.3).  nnca_build runs the single
 * bottom-up traversal of Sec. 2.3.2 on the GPU (tree of Sec. 2.1, lists of
 * Sec. 2.2 / Table 1, one partially pivoted ACA per cell, Sec. 2.2.1, with the
 * transfer operators taken from the ACA by-products, Remark in Sec. 2.3.2).
 * nnca_matvec applies the H2 representation of Sec. 3 with the passes of
 * Sec. 4 (upward, transverse, downward, near field).
 *
 * Conventions shared by every entry point
 *   - Every function returns nnca_status.  Nothing aborts or throws across
 *     the ABI; on error nnca_last_error() holds a message (thread-local) and
 *     output arguments are left untouched.
 *   - Device pointers are HIP device memory on the current device.  Host
 *     pointers are ordinary process memory.  The library never takes
 *     ownership of caller memory.
 *   - Vectors are column-major N x nrhs in the caller's original point order,
 *     with leading dimension ld >= N.
 *   - `stream` is a hipStream_t (NULL = the default stream).  nnca_build and
 *     the export/query functions are blocking; nnca_matvec,
 *     nnca_matvec_adjoint and nnca_direct are asynchronous on `stream`.
 *     Successive calls on one handle are ordered even when they name
 *     different streams (each call waits for the handle's previous one).
 *   - A handle may be used from one thread at a time.
 *   - Device memory of a handle comes from the allocator given at build time
 *     (default: hipMalloc / hipFree).  nnca_matvec and nnca_matvec_adjoint
 *     allocate nothing: their workspace is sized at build time.
 */
#ifndef NNCA_H
#define NNCA_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnca_h2 *nnca_handle;

typedef enum {
    NNCA_OK = 0,
    NNCA_ERR_INVALID_ARG = 1,   /* a bad size, pointer, tolerance or point    */
    NNCA_ERR_OUT_OF_MEMORY = 2, /* a device or host allocation failed         */
    NNCA_ERR_HIP = 3,           /* a HIP runtime call or a kernel launch failed */
    NNCA_ERR_NOT_SUPPORTED = 4, /* valid but unsupported combination          */
    NNCA_ERR_NUMERICAL = 5,     /* a zero pivot in a transfer-operator solve  */
    NNCA_ERR_INTERNAL = 6
} nnca_status;

/* Kernel functions K(x, y) = K(r), r = |x - y| (Sec. 5, Exp. 1-6).
 * log r and 1/r are zero at r = 0; the Gaussian exp(-r^2/h^2) is 1 there.
 * The regularised kernels of Exp. 1-4 take a = length_scale > 0:
 *   NNCA_K_LOG_REG: r (log r - 1) / (a (log a - 1)) for r < a,
 *                   log r / log a for r >= a (2D only; 0 at r = 0);
 *   NNCA_K_INV_REG: r / a for r < a, a / r for r >= a (0 at r = 0).      */
typedef enum {
    NNCA_K_LOG_R = 1,   /* log r, 2D only                                 */
    NNCA_K_INV_R = 2,   /* 1/r                                            */
    NNCA_K_GAUSS = 3,   /* exp(-r^2 / h^2), h = length_scale > 0          */
    NNCA_K_LOG_REG = 4, /* regularised log r, a = length_scale, 2D only   */
    NNCA_K_INV_REG = 5, /* regularised 1/r, a = length_scale              */
    NNCA_K_EXP_R = 6    /* exp(-r / h), h = length_scale > 0 (the "Matern"
                           kernel of Exp. 6); 1 at r = 0                  */
} nnca_kernel_kind;

/* Arithmetic of a matvec.
 *   NNCA_PREC_FP64:  every pass in FP64.
 *   NNCA_PREC_MIXED: every pass in FP32 with FP32 accumulation on cell-local
 *     coordinates; the input is split x = x_hi + x_lo (x_hi = fl32(x),
 *     x_lo = fl32(x - x_hi)), the near field is applied to both parts and
 *     the three partial results are combined in FP64.  Pivots and transfer
 *     operators always come from the FP64 build.                           */
typedef enum { NNCA_PREC_FP64 = 0, NNCA_PREC_MIXED = 1 } nnca_precision;

/* Element type of the caller's X and Y.  The arithmetic is set by the
 * precision alone: FP32 vectors are widened on input and rounded on
 * output.                                                                 */
typedef enum { NNCA_F32 = 0, NNCA_F64 = 1 } nnca_dtype;

/* Caller-supplied device allocator: alloc returns `bytes` of device memory on
 * the current device (NULL on failure), free releases a pointer alloc
 * returned.  Both receive `ctx`.  The library frees only after the device
 * work that uses the memory has finished (it synchronizes the device first).
 * Every device buffer of the handle, at build and later, comes from it.    */
typedef void *(*nnca_alloc_fn)(size_t bytes, void *ctx);
typedef void (*nnca_free_fn)(void *ptr, void *ctx);

typedef struct {
    uint32_t struct_size;    /* sizeof(nnca_build_options)                    */
    int32_t eta2_num;        /* admissibility eta^2 = eta2_num / eta2_den;     */
    int32_t eta2_den;        /*   0/0 selects eta^2 = dim (adjacent cells)    */
    int32_t exhausted_policy;/* 1 (default): a cell whose far-field candidate
                                set has fewer columns than rows keeps all its
                                rows (identity operator); 0: plain ACA        */
    int64_t workspace_bytes; /* cap on the ACA panel workspace; 0 = automatic */
    int32_t rank_reserve;    /* panel rows reserved per non-leaf cell before a
                                cell that needs more is re-run with min(m, n);
                                0 = 256.  Affects memory and speed only.      */
    int32_t reserved;
    /* fields below: struct_size >= their end (older callers get defaults)  */
    int32_t max_rhs;         /* columns of the many-column workspace sized at
                                build time: 0 = 16, 1 = none (matvecs with
                                several columns run one column at a time),
                                else rounded up to a multiple of 16, at most
                                64; wider X run in blocks of that width       */
    int32_t reserved2;
    nnca_alloc_fn alloc;     /* NULL: hipMalloc / hipFree                     */
    nnca_free_fn free;       /*   (both or neither)                           */
    void *alloc_ctx;
} nnca_build_options;

/* Build the H2 representation (Sec. 3 steps 1; steps 2-3 are evaluated on
 * the fly by nnca_matvec).
 *   points: dim x n coordinates, structure of arrays: coordinate q of point i
 *           at points[q * ld + i]; host memory if points_on_device == 0, else
 *           device memory.  Copied; the caller may free it on return.
 *   n >= 1, dim in {2, 3}, ld >= n, leaf_size >= 1 (the nu of Sec. 2.1),
 *   tol >= 0 (epsilon_NCA of Sec. 2.3.2, the same at every level).
 *   opts may be NULL (defaults).  On success *out receives a new handle.
 * Errors: INVALID_ARG for bad sizes, NULL pointers, tol < 0 or NaN,
 * non-finite coordinates, length_scale <= 0 with the Gaussian;
 * NOT_SUPPORTED for the log kernel outside 2D; OUT_OF_MEMORY; HIP.          */
nnca_status nnca_build(const double *points, int64_t n, int32_t dim, int64_t ld,
                       int32_t points_on_device, int32_t kernel_kind, double length_scale,
                       double tol, int32_t leaf_size, const nnca_build_options *opts,
                       void *stream, nnca_handle *out);

/* The general case P != Q (Sec. 2.1, 2.3): A_ij = K(p_i, q_j) with targets
 * P (np points) and sources Q (nq points), for rectangular sets such as the
 * evaluation of a kernel expansion at new points.
 *   targets: dim x np, SoA with stride ldp; sources: dim x nq, stride ldq;
 *   both host memory if points_on_device == 0, else device memory; copied.
 * One uniform tree covers P and Q; it stops at the first level where no
 * cell holds more than leaf_size points of P or more than leaf_size of Q.
 * Every cell runs two ACAs of the bottom-up traversal (Sec. 2.3.2): the
 * incoming one on A(t~^{B,i}, s~^{B,i}) gives t^{B,i}, s^{B,i} and U_B (or
 * the C_{B_c B}); the outgoing one gives t^{B,o}, s^{B,o} and V_B (or the
 * T_{B B_c}).  The outgoing ACA runs on the transposed block, its first
 * pivot among the cell's own sources, so that with P = Q it picks the
 * incoming pivots of the symmetric case (Sec. 5).
 * On such a handle nnca_matvec takes X with nq rows (Q's original order) and
 * writes Y with np rows (P's original order); nnca_matvec_adjoint maps np
 * rows to nq.  Both precisions and dtypes are supported; the transverse pass
 * and the near field evaluate every ordered pair of cells (there is no
 * symmetric form).  nnca_matvec_noalloc, nnca_matvec_backward,
 * nnca_batch_create, nnca_gmres and nnca_svm_train return NOT_SUPPORTED for
 * it.
 * Other arguments and errors as nnca_build; INVALID_ARG also for np or nq
 * < 1 or np + nq > 2^30.                                                  */
nnca_status nnca_build_general(const double *targets, int64_t np, int64_t ldp, const double *sources,
                               int64_t nq, int64_t ldq, int32_t dim, int32_t points_on_device,
                               int32_t kernel_kind, double length_scale, double tol, int32_t leaf_size,
                               const nnca_build_options *opts, void *stream, nnca_handle *out);

/* Rows (|P|) and columns (|Q|; n and n when P = Q) of the operator, and
 * whether the handle is of the general case (host pointers, may be NULL).  */
nnca_status nnca_query_shape(nnca_handle h, int64_t *rows, int64_t *cols, int32_t *general);

/* Y = A~ X (Sec. 4) for nrhs columns.  X, Y: device memory of element type
 * dtype (an nnca_dtype), original point order, column-major with leading
 * dimensions ldx, ldy >= n (elements); X and Y must not overlap.  precision
 * is an nnca_precision.  Asynchronous on `stream`; allocates nothing.
 * Errors: INVALID_ARG (NULL handle or vectors, nrhs < 1, leading dimension
 * < n, unknown dtype or precision, X and Y overlapping); HIP.              */
nnca_status nnca_matvec(nnca_handle h, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                        int32_t dtype, int32_t precision, void *stream);

/* Y = A~^T X.  In the symmetric case of Sec. 5 (P = Q, K(x, y) = K(y, x))
 * V_B = U_B and T_{B B_c} = C_{B_c B}^T, so the transposed passes (P2M <->
 * L2P, M2M <-> L2L, S_{B,B'}^T = S_{B',B}, near blocks likewise) are the
 * forward ones and A~^T = A~; this entry point runs the forward passes.  On
 * a handle of nnca_build_general it runs the transposed passes (up with U_B^T
 * and C_{B_c B}^T over P, across with the transposed blocks, down with V_B
 * and T_{B B_c}^T over Q); X has np rows, Y nq.  Arguments and errors as
 * nnca_matvec.                                                           */
nnca_status nnca_matvec_adjoint(nnca_handle h, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                                int32_t dtype, int32_t precision, void *stream);

/* Y = A~ X like nnca_matvec, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Every per-call buffer of the one-column passes (input in tree
 * order and its FP32 split, multipole and local vectors, column slots, split
 * partial vectors, near- and far-field sums) lives in one static device
 * array of NNCA_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from
 * its first use on that GPU until the process ends; nothing is allocated,
 * on the device or the host.  nrhs > 1 runs the columns one at a time.
 * The handle's own workspace is not touched.  Results equal nnca_matvec's
 * with nrhs = 1 bit for bit.  Every call on one GPU, from any handle, uses
 * the same array and leaves its contents behind: calls that can overlap on
 * one GPU (different streams, different threads) race and must be ordered
 * by the caller.  Arguments as nnca_matvec.
 * Errors: as nnca_matvec; NOT_SUPPORTED when the handle's per-call buffers
 * exceed the array (the message states both sizes; use nnca_matvec); HIP
 * when the array's device address cannot be obtained.                     */
#define NNCA_NOALLOC_SCRATCH_BYTES (64u << 20)
nnca_status nnca_matvec_noalloc(nnca_handle h, const void *X, void *Y, int64_t nrhs, int64_t ldx, int64_t ldy,
                                int32_t dtype, int32_t precision, void *stream);

/* Backward of Y = A~ X for a scalar loss L with G = dL/dY (device FP64,
 * column-major, original point order, like X):
 *   DX    = A~^T G  (the gradient with respect to X; Sec. 5's symmetric case
 *           makes it the forward passes applied to G), if DX != NULL;
 *   *dLdh = sum over the columns c of G_c^T (dA~/dh) X_c, the derivative of
 *           L with respect to the Gaussian length scale h with every pivot
 *           set t^{B,i}, s^{B,i} of the build held fixed, if dLdh != NULL.
 *           With the pivots fixed the transfer operators are
 *           C_B = K(t~, J) K(I, J)^{-1} (Remark in Sec. 2.3.2) and
 *           dC_B = (dK(t~, J) - C_B dK(I, J)) K(I, J)^{-1}, dK/dh =
 *           (2 r^2 / h^3) K; every block of Sec. 4 is differentiated.
 * dLdh is a device pointer to one double.  precision (nnca_precision) sets
 * the arithmetic of the passes; the transfer-operator terms and the FP64
 * factors L U = K(I, J) are FP64 in both.  The first call with dLdh factors
 * K(I, J) of every ACA cell (blocking, allocates sum k_B^2 doubles, kept
 * with the handle); later calls are asynchronous on `stream`.
 * Errors: INVALID_ARG (NULL G, neither output requested, X NULL with dLdh,
 * leading dimensions < n, DX overlapping X, G or dLdh); NOT_SUPPORTED (dLdh
 * with a kernel other than the Gaussian, or a rank above 1024);
 * NUMERICAL (a zero pivot in K(I, J)); OUT_OF_MEMORY; HIP.                */
nnca_status nnca_matvec_backward(nnca_handle h, const double *X, const double *G, int64_t nrhs, int64_t ldx,
                                 int64_t ldg, int32_t precision, double *DX, int64_t lddx, double *dLdh,
                                 void *stream);

/* Apply options of a handle, for the matvecs issued after the call.
 *   NNCA_APPLY_NO_SYMMETRIC: both forms evaluate the transverse blocks, and
 *     the mixed form the near-field blocks, for every ordered pair of cells.
 *     By default (flags = 0) they use the symmetric case of Sec. 5:
 *     K(x, y) = K(y, x) and B' in IL(B) <=> B in IL(B') (likewise for N(B))
 *     make the block of (B', B) the transpose of that of (B, B'), so each
 *     unordered pair is evaluated once and used for both directions (the
 *     transverse pass of every level whose ranks are at most 256; the mixed
 *     near field only where near pairs exceed 1/12 of the transverse
 *     interactions).  Either choice gives the product to the accuracy of its
 *     form; summation orders differ.
 * Errors: INVALID_ARG (NULL handle, unknown bits).                        */
enum { NNCA_APPLY_NO_SYMMETRIC = 1 };
nnca_status nnca_set_apply_flags(nnca_handle h, int32_t flags);

/* Dense FP64 direct sum Y = A X with A_ij = K(p_i, p_j) (the plain
 * definition; used for error reports).  points: device, dim x n SoA with
 * stride ld; X, Y: device FP64 column-major.  Asynchronous on `stream`.    */
nnca_status nnca_direct(const double *points, int64_t n, int32_t dim, int64_t ld,
                        int32_t kernel_kind, double length_scale, const double *X, double *Y,
                        int64_t nrhs, int64_t ldx, int64_t ldy, void *stream);

/* Uneven batches (many independent problems, one set of launches).
 * nnca_batch_create merges the apply data of `count` built handles (same
 * dim, kernel kind and length scale; each with a far field, i.e. kappa >=
 * lmin) into one forest whose tree levels are aligned by their distance from
 * the leaves; each pass of Sec. 4 then runs one launch per aligned level over
 * the cells of every problem, the transverse pass and the near field as
 * before.  The result is the block-diagonal product Y_b = A~_b X_b.  The
 * batch copies what it needs: the handles may be destroyed afterwards.
 * Blocking.  flags:
 *   NNCA_BATCH_GRAPH     the first nnca_batch_matvec with a given (X, Y,
 *                        nrhs, ldx, ldy, precision) runs eagerly, then
 *                        captures the whole matvec into a HIP graph on the
 *                        batch's own stream; later calls with the same
 *                        arguments replay it (other arguments re-capture);
 *   NNCA_BATCH_AUTOTUNE  the first call for a column-block width and
 *                        precision times split factors 1, 2, 4, ..., 64 of
 *                        every level's transverse-pass launch and, on the
 *                        FP32 levels, two tile shapes (sources per LDS tile)
 *                        on the live data and keeps the fastest (many-column
 *                        path).  If the environment variable NNCA_TUNE_CACHE
 *                        names a file, choices are read from it first and
 *                        new ones appended to it (one text line per level
 *                        shape: device architecture, pass, form, column-block
 *                        width and log2 buckets of the level's cell count,
 *                        sources per cell and rank), so later processes skip
 *                        the timing.
 * Errors: INVALID_ARG (NULL, count < 1, unknown flags, mismatched handles),
 * NOT_SUPPORTED (a problem without a far field, more than 2^30 rows),
 * OUT_OF_MEMORY, HIP.                                                     */
typedef struct nnca_batch *nnca_batch_handle;
enum { NNCA_BATCH_GRAPH = 1, NNCA_BATCH_AUTOTUNE = 2 };
nnca_status nnca_batch_create(const nnca_handle *handles, int32_t count, int32_t flags, nnca_batch_handle *out);

/* count, total rows and the count + 1 row offsets of the problems (host;
 * any pointer may be NULL).  Problem b owns rows [offsets[b], offsets[b+1])
 * of the batched vectors, in its own original point order.               */
nnca_status nnca_batch_query(nnca_batch_handle b, int32_t *count, int64_t *rows, int64_t *offsets);

/* Y = diag(A~_1, ..., A~_B) X for nrhs columns; X, Y: device FP64,
 * column-major, rows as given by nnca_batch_query, leading dimensions >= the
 * total rows; X and Y must not overlap.  Ordered after earlier work on
 * `stream` and before later work on it (the batch runs on its own stream).
 * A handle's batch may be used from one thread at a time.                  */
nnca_status nnca_batch_matvec(nnca_batch_handle b, const double *X, double *Y, int64_t nrhs, int64_t ldx,
                              int64_t ldy, int32_t precision, void *stream);
nnca_status nnca_batch_destroy(nnca_batch_handle b);

#define NNCA_MAX_LEVELS 64
typedef struct {
    int64_t n;
    int32_t dim, kappa, lmin, leaf_size;
    int32_t kernel_kind;
    double length_scale, tol;
    double lo[3], side;                   /* the root cell: lo + [0, side]^dim */
    int64_t ncell[NNCA_MAX_LEVELS];       /* non-empty cells per level         */
    int64_t npiv[NNCA_MAX_LEVELS];        /* sum of ranks per level            */
    int64_t nlist[NNCA_MAX_LEVELS][2];    /* total entries of N and IL lists   */
    int32_t max_rank[NNCA_MAX_LEVELS];
    int64_t m2l_level[NNCA_MAX_LEVELS];   /* M2L interactions per level        */
    int64_t transfer_entries;             /* stored non-identity entries of all C */
    int64_t m2l_interactions;             /* sum over IL pairs of k_B k_B'      */
    int64_t p2p_interactions;             /* sum over near pairs |t^B| |t^B'|   */
    double build_seconds;
    int32_t mixed_fp32_levels;            /* NNCA_PREC_MIXED: the finest levels whose
                                             transverse pass runs in FP32 (2 for
                                             1/r, 1 for the other kernels; the
                                             coarser ones in refined FP64)      */
    int32_t mixed_near_symmetric;         /* 1: the mixed near field evaluates each
                                             pair of neighbouring leaves once  */
} nnca_info;

/* Structure and statistics of a handle (blocking). */
nnca_status nnca_query(nnca_handle h, nnca_info *info);

/* Timing of the build (host pointer out, the first `count` of, at most 3):
 *   out[0]  seconds of the whole build (nnca_build / nnca_build_general);
 *   out[1]  seconds of its pivot traversal (the ACAs of Sec. 2.3.2 and the
 *           transfer operators);
 *   out[2]  the traversal's algorithmic panel reads in bytes: step k of a
 *           cell's ACA reads the k previous rows of its n-column panel twice
 *           (row residual, norm update), sum over ACA cells of k (k - 1) n 8.
 * Errors: INVALID_ARG (NULL handle or out, count < 1).                    */
nnca_status nnca_query_build(nnca_handle h, double *out, int32_t count);

/* Parity exports (blocking; all output buffers are host memory sized by the
 * caller from nnca_query).
 *   order[n]: original index of each tree-order position.
 *   cells of level l: key (Morton prefix), first/count (tree-order range).
 *   lists of level l (which = 0: N(B), 1: IL(B)): ptr[ncell+1], idx[total].
 *   pivots of level l: ptr[ncell+1], rows[npiv] (t^{B,i}, original indices,
 *     ACA selection order), cols[npiv] (s^{B,i}, original indices; -1 for
 *     cells kept whole).
 *   operator of cell b at level l: m x k row-major dense C_B into C
 *     (capacity `cap` doubles), *m and *k receive its shape.               */
nnca_status nnca_export_order(nnca_handle h, int64_t *order);
nnca_status nnca_export_cells(nnca_handle h, int32_t level, uint64_t *key, int64_t *first,
                              int64_t *count);
nnca_status nnca_export_lists(nnca_handle h, int32_t level, int32_t which, int64_t *ptr,
                              int64_t *idx);
nnca_status nnca_export_pivots(nnca_handle h, int32_t level, int64_t *ptr, int64_t *rows,
                               int64_t *cols);
nnca_status nnca_export_operator(nnca_handle h, int32_t level, int64_t cell, double *C,
                                 int64_t cap, int64_t *m, int64_t *k);
/* The same per half of a cell (half 0: incoming, half 1: outgoing; both are
 * the one ACA when P = Q).  Half 0: rows = t^{B,i} (indices into P), cols =
 * s^{B,i} (into Q), C = U_B or the stacked C_{B_c B}.  Half 1: rows = s^{B,o}
 * (into Q), cols = t^{B,o} (into P), C = V_B (|s^B| x k) or the stacked
 * T_{B B_c}^T.  For a handle of nnca_build, P = Q and the export of either
 * half equals nnca_export_pivots / nnca_export_operator.  In the general
 * case nnca_export_cells' first/count are P's ranges in P's tree order and
 * nnca_export_order gives P's order.                                      */
nnca_status nnca_export_half(nnca_handle h, int32_t level, int32_t half, int64_t *ptr, int64_t *rows,
                             int64_t *cols);
nnca_status nnca_export_half_operator(nnca_handle h, int32_t level, int32_t half, int64_t cell, double *C,
                                      int64_t cap, int64_t *m, int64_t *k);

/* Evaluate the method's FP64 kernel on the device for `count` pairs
 * (a[i], b[i]); a, b: host, dim x count SoA; out: host, count values.
 * Used to check that the device evaluates K bit for bit as specified.     */
nnca_status nnca_debug_kernel_eval(int32_t kernel_kind, double length_scale, int32_t dim,
                                   const double *a, const double *b, int64_t count, double *out);

/* Per-launch timing of the single-column matvec passes with HIP events
 * recorded on the matvec stream.  nnca_profile_enable(h, mask) clears earlier
 * records and records the launches of every pass p whose bit (1 << p) is set
 * in mask (-1: all, 0: stop).  Passes: 0 gather/split, 1 P2M/M2M, 2 M2L
 * (for the symmetric form, its kernel alone), 3 L2L/L2P, 4 near field +
 * combine, 5 M2L combine (ordered sum of split parts, the partners' column
 * slots).  nnca_profile_read (blocking) copies up to `cap` records -- pass,
 * tree level (-1 for none) and milliseconds -- into host arrays, stores the
 * number of records in *count and clears them.                             */
nnca_status nnca_profile_enable(nnca_handle h, int32_t enable);
nnca_status nnca_profile_read(nnca_handle h, int64_t *count, int32_t *pass, int32_t *level, double *ms,
                              int64_t cap);

/* Solve (alpha I + beta A~) X = F by restarted GMRES(restart) with the H2
 * matvec of the given precision (the integral-equation solve of Exp. 5 in
 * Sec. 5: a Nystrom discretisation of sigma + int K sigma = f gives alpha =
 * 1 and beta = the quadrature weight).  F, X: device FP64 vectors of n
 * entries in original point order; X holds the initial guess on entry and
 * the solution on return.  Stops when the relative residual
 * ||F - (alpha I + beta A~) X|| / ||F|| is at most tol (checked with the
 * Arnoldi recurrence, then recomputed for the final X) or after max_iter
 * matvecs.  *iters receives the matvec count, *relres the final relative
 * residual (host pointers, may be NULL).  Arnoldi uses classical
 * Gram-Schmidt applied twice; inner products are fixed-shape device
 * reductions (deterministic).  Blocking; allocates n (restart + 2) doubles
 * of workspace for the call.
 * Errors: INVALID_ARG (NULL pointers, F and X overlapping, tol < 0, alpha or
 * beta not finite, max_iter < 0, restart outside 1..1000, bad precision);
 * OUT_OF_MEMORY; HIP.                                                     */
nnca_status nnca_gmres(nnca_handle h, double alpha, double beta, const double *F, double *X, double tol,
                       int32_t max_iter, int32_t restart, int32_t precision, int32_t *iters, double *relres,
                       void *stream);

/* Kernel SVM training of Exp. 6 (Sec. 5) on a handle of nnca_build over the
 * N training points: gradient ascent on the penalised dual
 *   L(a) = sum a_i - 1/2 sum_ij K(x_i, x_j) y_i y_j a_i a_j - beta/2 (sum_j a_j y_j)^2,
 * whose gradient is 1 - y .* (K~ v) - beta sum(v) y with v = y .* a and K~ the
 * H2 operator of the handle (one nnca_matvec per step).  Each step is
 *   a <- min(max(a + eta grad, 0), lambda)
 * (the box 0 <= a <= lambda of the dual enforced by projection).
 * y: device, N labels in the original point order (+1 / -1; other values
 * are taken as given).  alpha: device, N entries, the initial iterate on
 * entry (usually zeros), the last iterate on return; must not overlap y.
 * lambda > 0 (the box bound), beta >= 0 (the penalty of the equality
 * constraint sum a_i y_i = 0).  eta > 0 is the step; eta <= 0 picks
 * 1 / (||K~||_2 + beta N) with ||K~||_2 from 30 power steps on K~ started
 * at the normalised all-ones vector (a step no longer than 1 / Lipschitz
 * constant of the gradient, so each step does not decrease L).  The loop
 * stops after max_iter steps or at the first step with
 * ||a_new - a||_2 <= tol ||a_new||_2 (||a_new|| read as 1 when it is 0).
 * Host outputs (may be NULL): *iters = steps taken, *eta_used = the step,
 * *bias = the mean of y_i - (K~ v)_i over the free support vectors
 * (0 < a_i < lambda) of the final iterate, 0 if there are none.  The
 * precision (an nnca_precision) is that of every matvec.  Reductions have
 * a fixed shape, so the iterates repeat bit for bit run to run.  The
 * stopping rule is evaluated on the device and read by the host every 16
 * steps (steps launched after it has fired change nothing).  Blocks until
 * done; allocates device scratch of 2N + 2050 doubles.
 * Errors: INVALID_ARG (NULL handle or vectors, overlap, lambda not > 0,
 * beta < 0, non-finite eta, tol < 0, max_iter < 0, bad precision);
 * NOT_SUPPORTED (a handle of nnca_build_general); NUMERICAL (power steps
 * with ||K~ u|| = 0); OUT_OF_MEMORY; HIP.                                 */
nnca_status nnca_svm_train(nnca_handle h, const double *y, double *alpha, double lambda, double beta, double eta,
                           double tol, int32_t max_iter, int32_t precision, int32_t *iters, double *bias,
                           double *eta_used, void *stream);

/* The SVM decision function of Exp. 6, f(x) = sum_i a_i y_i K(x_i, x) + bias,
 * at the rows of the handle: on a handle of nnca_build_general(targets =
 * the new points, sources = the training points) y and alpha have nq
 * entries and f has np; on a handle of nnca_build f is taken at the
 * training points (n entries each).  Device vectors in the original point
 * order; f must not overlap y or alpha.  The label is sgn f.  Blocks until
 * done; allocates nq doubles of scratch.
 * Errors: INVALID_ARG (NULL handle or vectors, overlap, non-finite bias,
 * bad precision); OUT_OF_MEMORY; HIP.                                     */
nnca_status nnca_svm_decision(nnca_handle h, const double *y, const double *alpha, double bias, double *f,
                              int32_t precision, void *stream);

/* Attainable rates on the current device, for the rooflines of the apply
 * passes (blocking; allocates and frees 512 MiB of workspace):
 *   out[0]  bytes/s of a device-to-device copy (read + write, 2 x 256 MiB);
 *   out[1]  FP32 FMA lane-operations/s (independent chains, no packed FP32);
 *   out[2]  v_rsq_f32 lane-operations/s;
 *   out[3]  pairs/s of the inner loop of the FP32 symmetric transverse pass
 *           of Sec. 4 with its operands in registers (r^2 = |t|^2 + |s|^2
 *           - 2 t.s by one addition and three FMAs, 1/sqrt, the row and the
 *           column FMA);
 *   out[4]  the same loop with r^2 of 16 x 16 pairs from one
 *           v_mfma_f32_16x16x4f32.
 * Only the first `count` (at most 5) are written.
 * Errors: INVALID_ARG (NULL out, count < 1); OUT_OF_MEMORY; HIP.           */
nnca_status nnca_probe_rates(double *out, int32_t count, void *stream);

nnca_status nnca_destroy(nnca_handle h);
const char *nnca_status_string(nnca_status s);
const char *nnca_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
