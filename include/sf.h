/*
 * sf.h — C ABI of the MI355X fused sparse executor (libsparsefusion.so).
 *
 * The library runs two sparse kernels, at least one of which carries loop
 * dependences, as one schedule over their joint dependence DAG (Cheshmi,
 * Strout, Mehri Dehnavi, "Composing Loop-carried Dependence with Other
 * Loops", arXiv 2111.12238):
 *   - SpTRSV -> SpMV:  x = L^{-1} b, then y = A x       (Sec. 1, Fig. 2;
 *                                                        Table 2, comb. 4)
 *   - SpIC0 -> SpTRSV: L L^T ~= A (zero fill), then x = L^{-1} b
 *                                                       (Table 2, comb. 5)
 * plus the adjoint of y = A L^{-1} b, batched right-hand sides and FP32
 * solves with FP64 residual refinement.
 *
 * Following the paper's inspector-executor driver (Sec. 2, Fig. 3b): the
 * inspector runs once on the host from the sparsity patterns and builds a
 * schedule (dependence levels, the joint claim order, work items); the
 * executor calls then run that schedule on the GPU as many times as needed.
 *
 * Conventions shared by every call:
 *   - Every function returns sf_status; nothing throws across the ABI.
 *   - Sparse matrices are CSR with int32 row pointers and column indices,
 *     columns strictly ascending inside a row (no duplicates).
 *   - Patterns passed to sf_inspect are HOST pointers, read during the call
 *     only; the schedule keeps its own copies.
 *   - Values and vectors passed to the executor calls are DEVICE pointers
 *     owned by the caller, laid out in the CSR order of the inspected
 *     pattern.  Dense blocks of right-hand sides are column-major
 *     (element (i, c) at ptr[i + c * ld]).
 *   - Executor calls are asynchronous and stream-ordered on the hipStream_t
 *     given (cast to void*; NULL = the default stream).  Launch and HIP
 *     errors are returned synchronously as SF_ERR_HIP.  Numerical
 *     breakdown of SpIC0 is reported through a device word (see
 *     sf_exec_ic0_trsv); a spin watchdog that fires is reported by
 *     sf_sync_status.
 *   - A schedule is immutable after sf_inspect except for the small device
 *     state it owns (claim counters, workspaces); executions of one
 *     schedule must therefore not overlap (issue them on one stream, or
 *     synchronise between streams).
 *   - NaN and Inf in values propagate and are not checked.  A diagonal
 *     entry whose value is exactly 0.0 gives Inf/NaN in the solution.
 */
#ifndef SF_H_
#define SF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SF_OK = 0,
  SF_ERR_ARG = 1,          /* NULL pointer, bad size, bad option value */
  SF_ERR_CSR = 2,          /* rowptr not monotone, column out of range, unsorted or duplicate */
  SF_ERR_NOT_LOWER = 3,    /* L has an entry above the diagonal */
  SF_ERR_ZERO_DIAG = 4,    /* a row of L has no stored diagonal entry */
  SF_ERR_SHAPE = 5,        /* dimensions of L, A, B, X, Y do not agree */
  SF_ERR_NOT_SPD = 6,      /* reserved: SpIC0 breakdown is reported through d_info */
  SF_ERR_HIP = 7,          /* a HIP runtime call or kernel launch failed */
  SF_ERR_OOM = 8,          /* device or host allocation failed */
  SF_ERR_TIMEOUT = 9,      /* the executor's spin watchdog fired (a dependence never became ready) */
  SF_ERR_UNSUPPORTED = 10  /* valid request this build does not implement */
} sf_status;

typedef enum { SF_F64 = 0, SF_F32 = 1 } sf_dtype;

typedef enum {
  SF_TRSV_SPMV = 0, /* L and A given: x = L^{-1} b, y = A x */
  SF_IC0_TRSV = 1,  /* lower(A) given as L: L L^T ~= A, x = L^{-1} b */
  SF_ILU0_TRSV = 2  /* the whole square A given as L: L U ~= A, y = L^{-1} x (unit L) */
} sf_kind;

/* A sparsity pattern on the host: nrows x ncols, rowptr[nrows + 1],
 * colind[rowptr[nrows]]. */
typedef struct {
  int32_t nrows;
  int32_t ncols;
  const int32_t* rowptr;
  const int32_t* colind;
} sf_csr_pattern;

/* Opaque, library-owned schedule. */
typedef struct sf_schedule_s* sf_schedule;

/* Inspector options; 0 in any field selects the default. */
typedef struct {
  int32_t kind;           /* sf_kind */
  int32_t rows_per_item;  /* maximum rows in one work item (default 64; SpIC0 items hold
                             one batch of 64 / lanes_per_row rows) */
  int32_t max_item_nnz;   /* cost budget of one work item, summing the paper's vertex
                             cost c(v) (Sec. 3.1) = max(1, off-diagonals of the row);
                             default 512 */
  int32_t rhs_block;      /* right-hand sides walked together per DAG pass: 0 (the default:
                             the smallest power of two >= nrhs, at most 64) or a power of
                             two 2..64 */
  int32_t lanes_per_row;  /* lanes of a 64-wide wavefront per SpIC0 row, one per stored
                             entry (4..64, a power of two; default: the longest row) */
  int32_t want_backward;  /* 1: also build the transposed (upper-solve) schedule for sf_backward */
  int32_t validate;       /* 1: check the built schedule against every DAG edge before returning */
  int32_t no_fusion;      /* 1: executor calls run the unfused two-phase baseline instead (the
                             paper's fusion = False switch, Sec. 2.3) */
  int32_t coarsen;        /* work items of the one-right-hand-side fused SpTRSV -> SpMV
                             executor (and of sf_backward's transposed solve): 0 = choose by
                             the inspector's critical-path estimates, 1 = one wavefront per
                             item, 2 = coarsened items spanning several wavefronts (the
                             paper's w-partitions of an s-partition, Sec. 3.2), 3 = regions of
                             up to "region_rows" rows on a block of a computing and a polling
                             wavefront, the region's data in LDS */
} sf_inspect_opts;

/* Summary of a schedule (host values). */
typedef struct {
  int64_t n;               /* rows of L */
  int64_t m;               /* rows of A (SpMV iterations); 0 for SF_IC0_TRSV */
  int64_t nnz_l;
  int64_t nnz_a;
  int32_t depth;           /* number of wavefronts (levels) of the SpTRSV DAG */
  int32_t joint_depth;     /* number of wavefronts of the joint DAG */
  int32_t back_depth;      /* levels of the transposed solve (0 if not built) */
  int32_t n_items;         /* work items of the fused forward schedule */
  int32_t n_back_items;    /* work items of the backward schedule */
  int32_t max_level_width; /* widest SpTRSV wavefront */
  int32_t lanes_per_row;   /* lanes per SpTRSV row in effect */
  int32_t lanes_per_spmv;  /* lanes per SpMV row in effect */
  double reuse_ratio;      /* Sec. 2.2: common / max(per-kernel) accesses */
  double inspect_seconds;  /* host time spent in sf_inspect */
  int32_t coarsened;       /* 1: the one-right-hand-side fused executor runs coarsened items */
  int32_t chunk_items;     /* SpTRSV items of the coarsened plan (0 if none was built) */
  int32_t chunk_chain;     /* longest chain of dependent coarsened items */
  int32_t max_local_depth; /* most wavefronts spanned by one coarsened item */
  double est_level_us;     /* critical-path estimates (microseconds) the inspector compares: */
  double est_chunk_us;     /*   one wavefront per item vs coarsened items */
  int32_t back_coarsened;  /* the same choice for the backward (transposed) solve */
  int32_t back_chunk_chain;
  double est_back_level_us;
  double est_back_chunk_us;
} sf_schedule_stats;

/*
 * sf_inspect — build a schedule from sparsity patterns (host only; does not
 * touch the GPU).
 *   L: n x n lower-triangular pattern, every row holding its diagonal
 *      (for SF_IC0_TRSV: the lower triangle of A, diagonal included).
 *   A: m x n pattern of the SpMV operand (SF_TRSV_SPMV), NULL for
 *      SF_IC0_TRSV.
 * Dependence DAGs (Sec. 2.2): each stored L_ij, j < i, is an edge j -> i
 * (structural: stored zeros count); F = pattern(A) for a CSR SpMV, so SpMV
 * row r depends on every x_j it reads; for SpIC0 -> SpTRSV, F = I.
 * Levels, the joint order (joint level, SpTRSV before SpMV, row) and the
 * work items (runs of one level and one kind, at most rows_per_item rows
 * and max_item_nnz cost) are computed here, and for SF_TRSV_SPMV also the
 * coarsened plan (opts.coarsen): SpTRSV items that span several wavefronts,
 * cut from one topological order so the item graph stays acyclic.
 * Errors: SF_ERR_ARG, SF_ERR_CSR, SF_ERR_NOT_LOWER, SF_ERR_ZERO_DIAG,
 * SF_ERR_SHAPE, SF_ERR_OOM.  On error *out is set to NULL.
 */
sf_status sf_inspect(const sf_csr_pattern* L, const sf_csr_pattern* A,
                     const sf_inspect_opts* opts, sf_schedule* out);

/* Release a schedule and every host and device buffer it owns.  Waits for
 * the work of the last executor call made with it (an event recorded on
 * that call's stream), not for the whole device.  Call it before the HIP
 * runtime is torn down (e.g. not from a static destructor).  NULL is
 * accepted. */
sf_status sf_schedule_free(sf_schedule s);

/* Fill *st with the schedule's summary. */
sf_status sf_schedule_info(sf_schedule s, sf_schedule_stats* st);

/*
 * Copy the schedule to host arrays (for validation against the DAG).  The
 * plan exported is the one the one-right-hand-side fused executor runs
 * (coarsened items when sf_schedule_stats.coarsened is 1):
 *   level[n]       wavefront of each SpTRSV row;
 *   order[n + m]   iteration ids in claim order.  SF_TRSV_SPMV: SpTRSV row i
 *                  is id i, SpMV row r is id n + r.  SF_IC0_TRSV: SpIC0 row
 *                  i is id i and SpTRSV row i is id n + i (n + n ids);
 *   item_ptr[n_items + 1]  item t holds order[item_ptr[t] .. item_ptr[t+1]).
 * Any pointer may be NULL to skip that array.
 */
sf_status sf_schedule_export(sf_schedule s, int32_t* level, int32_t* order, int32_t* item_ptr);

/*
 * Item-local structure of the exported plan (Sec. 3.2: a w-partition runs
 * its vertices in dependence order on one worker):
 *   local_level[n + m]  wavefront of each claim position inside its item
 *                       (2n positions for SF_IC0_TRSV); all 0 when items
 *                       hold one wavefront;
 *   entry_slot[nnz(L)]  per stored L entry (i, j), j < i: the position of
 *                       row j inside row i's item when both share an item,
 *                       else 0xFF (also for the diagonal).
 * Rows of an item are sorted by local_level.  NULL skips an array.
 */
sf_status sf_schedule_export_local(sf_schedule s, uint8_t* local_level, uint8_t* entry_slot);

/* Backward (transposed-solve) schedule: rlevel[n], order[n] (rows),
 * item_ptr[n_back_items + 1] of the plan sf_backward runs (coarsened items
 * when sf_schedule_stats.back_coarsened is 1).  SF_ERR_ARG if it was not
 * built. */
sf_status sf_schedule_export_backward(sf_schedule s, int32_t* rlevel, int32_t* order,
                                      int32_t* item_ptr);

/* Item-local structure of the backward plan, as sf_schedule_export_local:
 * local_level[n] per claim position, entry_slot[nnz(L)] per stored entry of
 * L^T in its CSR order (the diagonal first in each row; 0xFF outside). */
sf_status sf_schedule_export_backward_local(sf_schedule s, uint8_t* local_level, uint8_t* entry_slot);

/*
 * sf_exec_trsv_spmv — fused SpTRSV -> SpMV (Sec. 1; Table 2, comb. 4, with a
 * CSR SpMV).  For each right-hand side c < nrhs:
 *     X[:, c] = L^{-1} B[:, c],    Y[:, c] = A X[:, c]
 * in one persistent kernel launch: wavefronts claim work items in the joint
 * order, wait on per-row readiness flags of the rows they read, and start
 * each SpMV row as soon as the x entries it reads are final.
 *   dtype:  SF_F64 or SF_F32 (values, vectors and accumulation).
 *   L_val:  device, nnz(L) values in the inspected order.
 *   A_val:  device, nnz(A) values; may be NULL when Y is NULL or A stores
 *           no entries.
 *   B:      device n x nrhs, leading dimension ldb >= n.
 *   X:      device n x nrhs output, ldx >= n.  Must not alias B.
 *   Y:      device m x nrhs output, ldy >= m; NULL runs the solve only.
 *   nrhs:   1..64.
 * Several right-hand sides run one of two ways ("multi_path"):
 *   - in blocks of rhs_block columns: B is packed into a library-owned
 *     device workspace (kept with the schedule, grown on demand, freed with
 *     it) in which each row of a block holds its columns contiguously, the
 *     solve and the product run there, and X and Y are unpacked at the end;
 *   - as one chain of the single-RHS work items per column, directly on
 *     the caller's columns (by default for a few right-hand sides on deep,
 *     narrow DAGs with the coarsened plan).
 * Either way only rows < n of X and < m of Y are written.
 * n = 0: B, X and L_val are not used (may be NULL) and every column of Y is
 * set to zero (A has no columns, so y = A x = 0).
 * Several right-hand sides need n * rhs_block < 2^31 (else SF_ERR_UNSUPPORTED).
 * Errors: SF_ERR_ARG, SF_ERR_SHAPE, SF_ERR_UNSUPPORTED, SF_ERR_HIP, SF_ERR_OOM.
 */
sf_status sf_exec_trsv_spmv(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val,
                            const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx,
                            void* Y, int32_t ldy, void* stream);

/*
 * The unfused two-phase baseline on the same GPU (the paper's unfused
 * comparison, Sec. 4): a level-set SpTRSV that takes one grid-wide barrier
 * per wavefront (one persistent cooperative launch), then a separate CSR
 * SpMV launch.  Same arguments and results as sf_exec_trsv_spmv.
 */
sf_status sf_exec_unfused_trsv_spmv(sf_schedule s, sf_dtype dtype, const void* L_val,
                                    const void* A_val, const void* B, int32_t ldb, int32_t nrhs,
                                    void* X, int32_t ldx, void* Y, int32_t ldy, void* stream);

/*
 * Static schedules of the SpTRSV -> SpMV pair, measured beside the
 * dynamic executor.
 *   SF_STATIC_MSP: the paper's fused partitioning (Sec. 3.2, Algorithm 1)
 *     with G1 = the SpTRSV DAG as head and forward pairing:
 *     - consecutive wavefronts grouped into s-partitions, each s-partition's
 *       connected components into at most msp_parts cost-balanced
 *       w-partitions;
 *     - the SpMV rows paired with the w-partition holding all their inputs;
 *     - zero-slack pairs merged;
 *     - slack SpMV rows dispersed to balance the w-partitions;
 *     - separated packing (Table 2: reuse ratio below one).
 *   SF_STATIC_WAVEFRONT: the paper's "fused wavefront" comparison (Sec. 4):
 *     one s-partition per wavefront of the joint DAG.
 * The plan is built on the host at first use (no device needed for the
 * info and export calls) and kept with the schedule.  Execution: one
 * cooperative launch, with a grid barrier between s-partitions; each
 * w-partition runs on one wavefront, its rows in order.
 */
typedef enum { SF_STATIC_MSP = 0, SF_STATIC_WAVEFRONT = 1 } sf_static_plan;

/* Sizes of a static plan: s-partitions, w-partitions, executor batches, and
 * (MSP) the pair partitions merged and the slack rows placed by balancing.
 * Any output pointer may be NULL.  Errors: SF_ERR_ARG (not SF_TRSV_SPMV, bad
 * plan), SF_ERR_OOM. */
sf_status sf_schedule_static_info(sf_schedule s, int32_t plan, int32_t* n_spart, int32_t* n_wpart,
                                  int32_t* n_batches, int32_t* merged, int32_t* slack_moved);

/* Host copies of a static plan: s_ptr[n_spart + 1] indexes w-partitions,
 * w_ptr[n_wpart + 1] indexes order, order[n + m] lists iteration ids (id
 * i < n: SpTRSV row i; id n + r: SpMV row r) in execution order within each
 * w-partition.  NULL outputs are skipped.  Errors as sf_schedule_static_info. */
sf_status sf_schedule_export_static(sf_schedule s, int32_t plan, int32_t* s_ptr, int32_t* w_ptr,
                                    int32_t* order);

/* x = L^{-1} b and y = A x (one right-hand side, FP64 or FP32) under a
 * static plan.  B, X (length n) and Y (length m; may be NULL when m = 0)
 * are device vectors; X must not alias B.  A_val may be NULL when A stores
 * no entries.  n = 0: Y is set to zero and nothing else is used.  Results equal sf_exec_trsv_spmv's bit for bit (same per-row
 * arithmetic).  Errors: SF_ERR_ARG, SF_ERR_OOM, SF_ERR_HIP. */
sf_status sf_exec_static_trsv_spmv(sf_schedule s, int32_t plan, sf_dtype dtype, const void* L_val,
                                   const void* A_val, const void* B, void* X, void* Y, void* stream);

/*
 * sf_exec_spmv_trsv — fused SpMV -> SpTRSV (Table 2, comb. 2):
 *   y = A x, then z = L^{-1} y.
 * The SpMV's row i feeds only the solve's row i (F = I), so the work item of
 * SpTRSV row i computes y_i first (interleaved packing, Sec. 3.2 step 3).
 * Uses a SF_TRSV_SPMV schedule whose A is square (m = n, else SF_ERR_SHAPE);
 * its SpTRSV plan (level or coarsened items) orders the rows.  One
 * right-hand side.  Device vectors: X (n, read), Y (n, written; NULL skips
 * storing y), Z (n, written; must not alias X or Y).  FP64 results equal
 * the sequential definitions' bit for bit (every sum in ascending order).
 * Errors: SF_ERR_ARG (null pointers, aliasing, wrong kind or dtype),
 * SF_ERR_SHAPE, SF_ERR_HIP.
 */
sf_status sf_exec_spmv_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, const void* L_val,
                            const void* X, void* Y, void* Z, void* stream);

/* Unfused baseline of sf_exec_spmv_trsv: the whole SpMV, then the level-set
 * solve (Y must not be NULL: it carries y between the two launches). */
sf_status sf_exec_unfused_spmv_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, const void* L_val,
                                    const void* X, void* Y, void* Z, void* stream);

/*
 * sf_exec_trsv_trsv — fused SpTRSV -> SpTRSV with one L (Table 2, comb. 1):
 *   x = L^{-1} b, then z = L^{-1} x.
 * Row i of the second solve needs x_i and earlier z_j only, so one work item
 * solves both for its rows and reads L once (reuse ratio >= 1: interleaved
 * packing).  Uses the SpTRSV plan of a SF_TRSV_SPMV schedule (A unused).
 * Device vectors: B (n, read), X (n, written), Z (n, written), pairwise
 * distinct.  FP64 results equal two sequential forward substitutions bit
 * for bit.  Errors as sf_exec_spmv_trsv.
 */
sf_status sf_exec_trsv_trsv(sf_schedule s, sf_dtype dtype, const void* L_val, const void* B, void* X, void* Z,
                            void* stream);

/*
 * sf_exec_ic_apply — the incomplete-Cholesky preconditioner apply of a PCG
 * iteration (Table 2's solve pairs with the transposed factor):
 *   w = L^{-1} r, then z = L^{-T} w,
 * in one launch: the SpTRSV plan's items, then the transposed solve's items
 * (reversed wavefronts of L^T, Sec. 2.2 DAGs), each backward row reading
 * its own w_i as soon as it is final (F = I).  When the schedule has region
 * plans for both solves, both run on them (a transposed region stages the
 * w_i of its rows); "precond_regions" = 0 keeps items.  Needs a SF_TRSV_SPMV schedule
 * inspected with want_backward = 1 (else SF_ERR_ARG); L is the factor (for
 * instance from sf_exec_ic0_trsv) in the inspected pattern.  One
 * right-hand side; R, W, Z are distinct device vectors of length n.  FP64
 * results equal forward then backward substitution done row by row, bit for
 * bit.  Errors: SF_ERR_ARG, SF_ERR_HIP.
 */
sf_status sf_exec_ic_apply(sf_schedule s, sf_dtype dtype, const void* L_val, const void* R, void* W, void* Z,
                           void* stream);

/* Unfused baseline of sf_exec_ic_apply: the forward solve, then the
 * transposed solve, as two launches. */
sf_status sf_exec_unfused_ic_apply(sf_schedule s, sf_dtype dtype, const void* L_val, const void* R, void* W,
                                   void* Z, void* stream);

/* Unfused baseline of sf_exec_trsv_trsv: two level-set solves. */
sf_status sf_exec_unfused_trsv_trsv(sf_schedule s, sf_dtype dtype, const void* L_val, const void* B, void* X,
                                    void* Z, void* stream);

/*
 * sf_exec_ilu0_trsv — fused SpILU0 -> SpTRSV (Table 2, comb. 6), FP64:
 *   L U ~= A with zero fill-in (L unit lower, U upper, both on pattern(A)),
 *   then y = L^{-1} x.
 * The schedule must be of kind SF_ILU0_TRSV, inspected from the whole
 * square pattern of A (sorted columns, every diagonal stored; A need not
 * be symmetric).  Row i of the factors is row-wise elimination restricted
 * to the pattern, each sum in ascending column order; row i of the solve
 * runs in the same work item (F = I).  Device arrays: A_val (nnz, read),
 * LU_val (nnz, written: L strictly below the diagonal, U on and above it,
 * in A's CSR positions), X and Y (n; X = NULL skips the solve).  d_info
 * (device int32, may be NULL) receives -1, or the smallest row whose pivot
 * u_ii is zero or NaN; the launch completes either way.  FP64 results equal
 * the sequential definition bit for bit.  Rows with more stored entries
 * than lanes_per_row (at most 64) give SF_ERR_UNSUPPORTED.
 */
sf_status sf_exec_ilu0_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, void* LU_val, const void* X,
                            void* Y, int32_t* d_info, void* stream);

/* Unfused baseline of sf_exec_ilu0_trsv: a level-set factorisation (one
 * grid barrier per level), then a level-set solve reading the factor. */
sf_status sf_exec_unfused_ilu0_trsv(sf_schedule s, sf_dtype dtype, const void* A_val, void* LU_val,
                                    const void* X, void* Y, int32_t* d_info, void* stream);

/*
 * sf_exec_ic0_trsv — fused SpIC0 -> SpTRSV (Table 2, comb. 5), FP64.
 * The schedule must be of kind SF_IC0_TRSV.  Computes the zero fill-in
 * incomplete Cholesky factor L of A (pattern = lower(A)) by the up-looking
 * row recurrence
 *     L_ij = (A_ij - sum_{k<j, k in P_i and P_j} L_ik L_jk) / L_jj,
 *     L_ii = sqrt(A_ii - sum_{k<i} L_ik^2),
 * and in the same work item x_i = (b_i - sum_{j<i} L_ij x_j) / L_ii (the
 * interleaved packing of Sec. 3.2, step 3: reuse ratio >= 1).
 *   A_lower_val: device, values of lower(A) in the inspected pattern.
 *   L_val:       device output, same pattern.
 *   B, X:        device n x nrhs (nrhs == 1 in this build).
 *   d_info:      device int32 written at the end of the launch: -1 if every
 *                pivot was > 0, else the smallest row whose pivot was <= 0
 *                or NaN (its dependents still run; values are then NaN).
 */
sf_status sf_exec_ic0_trsv(sf_schedule s, sf_dtype dtype, const void* A_lower_val, void* L_val,
                           const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx,
                           int32_t* d_info, void* stream);

/* Unfused baseline for SpIC0 -> SpTRSV: a level-set SpIC0 with a grid
 * barrier per wavefront, then a level-set SpTRSV.  Same arguments. */
sf_status sf_exec_unfused_ic0_trsv(sf_schedule s, sf_dtype dtype, const void* A_lower_val,
                                   void* L_val, const void* B, int32_t ldb, int32_t nrhs, void* X,
                                   int32_t ldx, int32_t* d_info, void* stream);

/*
 * sf_backward — adjoint of y = A L^{-1} b (not in the paper).  Given
 * G = dloss/dy (m values), computes with one persistent launch over the
 * transposed schedule (needs want_backward at inspection):
 *     c = A^T G,  lambda = L^{-T} c   (upper solve, reversed levels),
 *     grad_B = lambda,  grad_L_val[p] = -lambda_i x_j  for stored p = (i, j).
 * X holds x = L^{-1} B from the forward pass; if X is NULL it is recomputed
 * from B into the caller's workspace (activation recomputation instead of
 * storage).  workspace may be NULL when X is given; otherwise it must hold
 * sf_backward_workspace_bytes(s, dtype, 1) bytes.  Single right-hand side.
 */
sf_status sf_backward(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val,
                      const void* X, const void* B, const void* G, void* grad_B, void* grad_L_val,
                      void* workspace, size_t ws_bytes, void* stream);

size_t sf_backward_workspace_bytes(sf_schedule s, sf_dtype dtype, int32_t nrhs);

/*
 * sf_backward_noalloc — sf_backward for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc.  Same arguments and results as
 * sf_backward without the workspace: when X is NULL the recomputed x is kept
 * in a fixed device scratch of the library (64 MiB per GPU, held from the
 * library's load until the process ends), so n * sizeof(value) must be at
 * most 64 MiB (8M FP64 or 16M FP32 rows), else SF_ERR_UNSUPPORTED, checked
 * before anything else.  The call allocates nothing: the schedule's device
 * arrays must already be resident on the current device, made by an earlier
 * executor call with this schedule (typically the forward pass); otherwise
 * SF_ERR_ARG.  The timing mode is ignored.  Every call on one GPU shares that
 * GPU's scratch: calls that overlap on one GPU (different streams, or
 * different threads without ordering) race and must be serialised by the
 * caller.  Enqueues only; stream-ordered like sf_backward.
 */
sf_status sf_backward_noalloc(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val,
                              const void* X, const void* B, const void* G, void* grad_B,
                              void* grad_L_val, void* stream);

/*
 * sf_refine_trsv_spmv — FP32 solves with FP64 residual refinement (not in
 * the paper; its stages compose the way the paper's kernels do: each stage
 * reads, per row, only rows the previous stages have already produced).
 *   1. x0 = the FP32 substitution of (L32, fl32(b)), FP32 accumulation;
 *   2. n_corrections times: r = b - L64 x in FP64, d = the FP32
 *      substitution of (L32, fl32(r)), x += d in FP64;
 *   3. y = A64 x with FP64 values and accumulation, and the final relative
 *      residual max_i |b - L64 x|_i / max_i |b_i| per column.
 *   In each FP32 substitution a row sums its off-diagonal products first
 *   (ascending column, from 0) and subtracts the sum from its rounded
 *   right-hand side.  Default (sf_set_param "refine_path" 0, n_corrections
 *   <= 3): every stage runs in ONE fused launch over the SpTRSV -> SpMV
 *   schedule's level items -- each row gathers one tuple of all stage values
 *   of each row it reads -- and the results are bit-identical to that staged
 *   definition.  "refine_path" 1, n_corrections > 3, or one right-hand side
 *   on a coarsened plan: one launch per pass, with the executor's FP32
 *   solves (their own summation order).
 *   L32/L64: device values of L in FP32 and FP64 (same pattern); A64:
 *   device FP64 values of A.  B, X (n x nrhs, ld), Y (m x nrhs, ldy): FP64.
 *   out_relres: HOST array of nrhs doubles, filled after a stream sync
 *   (this call synchronises the stream when out_relres is not NULL).
 *   n_corrections: 0..8 (2 is the usual choice; 0..3 fused).
 *   workspace: device scratch of sf_refine_workspace_bytes(s, nrhs) bytes.
 */
sf_status sf_refine_trsv_spmv(sf_schedule s, const float* L32, const double* L64,
                              const double* A64, const double* B, int32_t ldb, int32_t nrhs,
                              double* X, int32_t ldx, double* Y, int32_t ldy,
                              int32_t n_corrections, double* out_relres, void* workspace,
                              size_t ws_bytes, void* stream);

size_t sf_refine_workspace_bytes(sf_schedule s, int32_t nrhs);

/*
 * Tuning knobs of the executor (defaults are set by sf_inspect):
 *   "lanes_trsv"                lanes per SpIC0 row (SF_IC0_TRSV, 4..64, a
 *                               power of two; re-cuts the items);
 *   "lanes_spmv"                kept for compatibility: SpTRSV and SpMV rows
 *                               deal their entries over all 64 lanes, so
 *                               lanes per row no longer select a kernel;
 *   "rhs_block"                 right-hand sides per DAG pass (0 = by nrhs,
 *                               else a power of two 2..64);
 *   "waves_per_cu"              persistent-grid residency target (4..32); default 8,
 *                               and for SF_IC0_TRSV / SF_ILU0_TRSV schedules, chosen at
 *                               inspection, the smallest power of two >= 4 that holds the
 *                               mean work items of one wavefront per CU (256 CUs);
 *   "levelset_waves_per_cu"     residency of the executors synchronised by
 *                               grid-wide barriers: the level-set baselines
 *                               (SpTRSV with any number of right-hand sides,
 *                               SpIC0, SpILU0) and the static plans (4..32,
 *                               default 4: a barrier costs more as the grid grows);
 *   "multi_waves_per_cu"        residency target of the fused executor for
 *                               several right-hand sides (4..32, or 0, the
 *                               default: 8, 16 or 32 by the units per level);
 *   "multi_path"                several right-hand sides: 1 = interleaved
 *                               blocks over the level units, 2 = one chain of
 *                               the single-RHS items per column (on the
 *                               caller's columns), 0 (default) = 2 for at most
 *                               8 right-hand sides on a coarsened plan of a
 *                               DAG whose mean wavefront is under 2048 rows,
 *                               else 1;
 *   "msp_parts"                 w-partitions per s-partition of the MSP plan
 *                               (its r; 1..2^20, default 1024; rebuilds it);
 *   "spin_limit"                watchdog: polls before SF_ERR_TIMEOUT;
 *   "claim_streams"             work-claim counters (1..32);
 *   "rows_per_item", "max_item_nnz"  re-cut the work items (rows <= 64);
 *   "spmv_delay"                place each SpMV row this many wavefronts after
 *                               the one where its inputs are final (0 = the
 *                               canonical joint order; any value keeps the
 *                               order topological); with coarsened items the
 *                               unit is one step of the item chain; -1
 *                               (default): 0 with level items, after every
 *                               SpTRSV item with coarsened ones (Sec. 3.2's
 *                               slack placement);
 *   "coarsen"                   0 auto, 1 level items, 2 coarsened items,
 *                               3 regions (re-cuts; "coarsened", "regioned",
 *                               "back_coarsened", "back_regioned" read the
 *                               plans in effect, "region_chain" and
 *                               "back_region_chain" the longest chains of
 *                               dependent regions);
 *   "region_rows"               rows per region (64..16384, default 512; halved
 *                               at inspection until a region's LDS fits 64 KB);
 *   "region_poll"               region poller: lanes watching inputs (bits 0-7,
 *                               1..64, default 64), back-off rounds after an
 *                               idle round (bits 8-15, default 0) and lanes
 *                               reading until the region's first input is
 *                               stored (bits 16-23, 0..64, 0 = all; default 2);
 *   "cached_reads"              fused executor: bit 0 = SpMV rows, bit 1 =
 *                               SpTRSV level items read x through the caches
 *                               first (default 0);
 *   "spmv_prefix"               prefix fusion on level items (default 1): SpMV
 *                               row r's entries up to its diagonal, when their
 *                               columns are exactly L's row r, are folded by
 *                               SpTRSV row r's item and the SpMV row continues
 *                               the fold (bit-identical); "prefix_rows" and
 *                               "prefix_entries" (read only) count the rows
 *                               and entries that qualify;
 *   "ic0_cached"                fused SpIC0: values read through the caches
 *                               first (default 0);
 *   "spmv_item_scale"           level items: an SpMV item takes up to this
 *                               many times rows_per_item rows (at most 64)
 *                               and max_item_nnz (1..8, default 4): they are
 *                               off the critical path, and fewer, longer
 *                               items stream faster;
 *   "precond_regions"           sf_exec_ic_apply runs both solves on their
 *                               region plans when the schedule has both
 *                               ("regioned" and "back_regioned"; default 1);
 *   "no_fusion", "timing", "trace"   switches (0/1; "trace" 2: items only).
 */
sf_status sf_set_param(sf_schedule s, const char* key, int64_t value);
sf_status sf_get_param(sf_schedule s, const char* key, int64_t* value);

/*
 * sf_autotune — time executor variants on the device with the caller's
 * data and keep the fastest: a coordinate search over the plan (level
 * items, coarsened items or regions), the several-RHS path and block width,
 * the SpMV slack delay, rows per item, the item cost budget, the residency
 * (waves per CU of the single- and multi-RHS executors), the SpMV items'
 * size on level items and prefix fusion.
 * A candidate replaces the current choice only when it is at least 2%
 * faster.  Cached-first reads are not searched: they measured no different.  The work done once per
 * matrix is amortised over many executions (the paper's inspector-executor
 * split, Sec. 2 and its NER metric, Sec. 4).  The chosen parameters are left
 * set on the schedule (sf_get_param reads them) and cached for the process,
 * keyed by the patterns' fingerprint (sizes, depth and a hash of both CSR
 * patterns), dtype, nrhs and whether Y is given: a later call with an equal
 * key -- on this or another schedule -- applies them without timing and sets
 * the read-only parameter "tuned_from_cache" to 1.  sf_set_param(s,
 * "autotune_cache", 0) makes this schedule tune afresh.  Runs the executor
 * on B, X, Y (their contents are overwritten) and synchronises the stream.
 *   out_best_ms: HOST, the best time per execution (may be NULL).
 */
sf_status sf_autotune(sf_schedule s, sf_dtype dtype, const void* L_val, const void* A_val,
                      const void* B, int32_t ldb, int32_t nrhs, void* X, int32_t ldx, void* Y,
                      int32_t ldy, void* stream, double* out_best_ms);

/* Synchronise the stream and report a watchdog timeout of an earlier
 * execution on this schedule (SF_ERR_TIMEOUT), clearing the report; SF_OK
 * else.  A timeout makes only the launch it happened in drain early: later
 * launches wait normally, whether or not this call was made in between. */
sf_status sf_sync_status(sf_schedule s, void* stream);

/* Trace mode (sf_set_param(s, "trace", 1)): the fused single-RHS
 * SpTRSV -> SpMV executor (and the fused SpIC0 -> SpTRSV executor, whose
 * items also stamp words 5 and 6: the end of the sweep and of the pivot
 * fold; on the region plan a region stamps word 1 when staged, 5 when its
 * first input from another region is stored and 6 when its first batch is
 * published) records a debug execution trace that shows every
 * iteration ran exactly once and after its inputs (the validity of a fused
 * schedule, Sec. 3.1: each DAG edge respected, each iteration executed once).
 * out (HOST) receives, for work item t (export order), 8 words at out[8t]:
 * stamps of the device's 100 MHz real-time counter at processing start,
 * indices and values loaded, every input ready (after the item's last wait)
 * and end, then the number of times the item ran, 3 zero words; then, at
 * out[8 n_items + 2 g] for iteration id g (SpTRSV row i: g = i, SpMV row r:
 * g = n + r), the stamp taken just before its value was published and the
 * number of times it was published.  count must be >= 8 n_items + 2 (n + m);
 * otherwise SF_ERR_SHAPE.  Waits for the last executor call on the schedule.
 * Each traced launch starts from zeroed counts.  Tracing adds stores and
 * atomics to every item: a debugging aid, not a timed mode.  With "trace"
 * set to 2 only the items are stamped (iteration words stay 0), which
 * slows the launch far less. */
sf_status sf_trace_export(sf_schedule s, unsigned long long* out, int64_t count);

/* Time of the last kernel launched by an executor call, measured with HIP
 * events on the executor's stream when enabled with
 * sf_set_param(s, "timing", 1); *ms is filled after a stream sync. */
sf_status sf_last_kernel_ms(sf_schedule s, double* ms);

/* Device probes: the machine constants that bound the executors, measured
 * on the current device.  They calibrate the two bounds of a fused pass:
 * bytes over the copy ceiling, and (for schedules whose x reads have no
 * locality) gathers over the gather rate, beside the critical path of
 * dependent hops times the hop latency.
 *   what: bit mask of SF_PROBE_COPY (stream copy of 1 GiB into 1 GiB, read +
 *         write bytes per second), SF_PROBE_HOP (one-way latency of a value
 *         published with the executors' protocol, between two workgroups on
 *         one XCD and across XCDs), SF_PROBE_GATHER (uniformly random
 *         single-value FP64 gathers from a 2^20-entry vector, 5e7 per pass,
 *         with coalesced column and value streams); 0 = all.
 *   out:  HOST; fields not probed, and a hop pair that could not be placed,
 *         are set to -1.
 *   stream: the probes run on it and the call synchronises it.
 * The probes allocate their own device buffers (up to 2 GiB, freed before
 * return) and are not meant for graph capture.  Errors: SF_ERR_ARG (out is
 * NULL or what has unknown bits), SF_ERR_OOM, SF_ERR_HIP. */
#define SF_PROBE_COPY 1
#define SF_PROBE_HOP 2
#define SF_PROBE_GATHER 4
typedef struct {
  double copy_GBps;         /* GB/s, read + write bytes */
  double hop_us_same_xcd;   /* microseconds per one-way hop */
  double hop_us_cross_xcd;
  double gathers_per_s;     /* single-value gathers per second */
} sf_probe_result;
sf_status sf_device_probe(int32_t what, sf_probe_result* out, void* stream);

const char* sf_status_str(sf_status st);

/* Library version string. */
const char* sf_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SF_H_ */
