/*
 * ccproj.h -- C ABI of the MI355X (gfx950) solver for the regularised
 * metric-constrained LP relaxation of correlation clustering.
 *
 * Problem (paper, Sec. II-A, problem (mn1)): for a signed weighted complete
 * graph on n nodes with a label d_p in {0,1} (1 = negative pair) and a weight
 * w_p > 0 per pair p = (i,j), i < j,
 *     min sum_p w_p f_p   s.t.  x_ij <= x_ik + x_jk  (every triplet, every
 *                               orientation),  |x_p - d_p| <= f_p.
 * Regularisation (Sec. II-B, problem (qp)): min c'v + (eps/2) v'Wv over
 * v = (x, f), c = (0, w), W = diag(w) on x and on f, gamma = 1/eps.
 * Method (Sec. II-B, Algorithm 1): Dykstra's = Hildreth's cyclic projection
 * with one dual per constraint, run on the conflict-free tiled schedule of
 * Sec. III (rounds = block anti-diagonals of the (i,k) grid; the tiles of a
 * round run concurrently without locks).
 *
 * Conventions for every entry point
 *   - Return value: CC_OK (0) on success, CC_ENOTCONV (1) when a solve hit
 *     its sweep limit, a negative CC_E* code on error.  After an error,
 *     cc_last_error() returns a message (thread-local; valid until the next
 *     call on the same thread).  Nothing aborts or throws across the ABI.
 *   - Device pointers are raw device addresses owned by the caller; the
 *     library never frees, resizes or copies them to the host (except where
 *     a function says it reads a result back).  Host pointers are marked
 *     "host".
 *   - Element type of the state arrays x, f, g, y, y_pair is the context's
 *     precision: double for CC_F64, float for CC_F32.  w is always double.
 *   - Layouts.  Pairs: packed upper-triangular column-major order,
 *     p(i,j) = j(j-1)/2 + i for 0-based i < j, N_p = n(n-1)/2 entries.
 *     Pair duals: y_pair[2p + c], c = 0 for x - f <= d, c = 1 for
 *     -x - f <= -d.  Metric duals: schedule order (see cc_dual_slots); use
 *     cc_duals_to_lex for the colex order y_lex[3t + o],
 *     t = C(k,3) + C(j,2) + i, o = 0: x_ij <= x_ik + x_jk,
 *     o = 1: x_ik <= x_ij + x_jk, o = 2: x_jk <= x_ij + x_ik.
 *   - All work of a context is enqueued on the stream given at creation;
 *     functions that return numbers to the host synchronise that stream.
 *     A context is not thread-safe; distinct contexts are independent.
 *   - Indices are 64-bit throughout (3 C(n,3) exceeds 2^31 for n > 1000).
 */
#ifndef CCPROJ_H
#define CCPROJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    CC_OK = 0,
    CC_ENOTCONV = 1,      /* sweep limit reached before the tolerance      */
    CC_EINVAL = -1,       /* bad argument (sizes, weights, gamma, b, ...)  */
    CC_ENOMEM = -2,       /* device or host allocation failed              */
    CC_EHIP = -3,         /* a HIP runtime call or kernel launch failed    */
    CC_ENONFINITE = -4    /* NaN or Inf found in the state                 */
};

enum { CC_F64 = 0, CC_F32 = 1 };                         /* context precision */
enum { CC_MODE_F64 = 0, CC_MODE_F32 = 1, CC_MODE_F32_POLISH = 2 };
enum { CC_MODE_SPARSE = 16 };  /* flag, or-ed into a mode: sparse dual access */
enum { CC_WARM_NONE = 0, CC_WARM_MLP = 1 };
enum { CC_EXEC_ROUNDS = 0, CC_EXEC_DATAFLOW = 1 };       /* sweep executors   */

typedef struct cc_ctx cc_ctx;

/* Convergence measures, all evaluated in FP64 (Sec. IV-D stops on how well
 * the rows hold and on the primal-dual gap).  Fields a solve cannot fill are NaN. */
typedef struct {
    double max_viol_metric;  /* max over metric rows of (x_L - x_S1 - x_S2)^+ */
    double max_viol_pair;    /* max over pairs of (|x - d| - f)^+             */
    double primal_qp;        /* sum w f + (1/(2 gamma)) sum w (x^2 + f^2)     */
    double dual_qp;          /* -b'y - (gamma/2) (c+A'y)' W^{-1} (c+A'y)      */
    double gap;              /* primal_qp - dual_qp                           */
    double lp_cost;          /* sum w |x - d|: the LP objective at x          */
    double cs_max;           /* max over rows of |y (b - a'v)|                */
    double stat_resid;       /* max |v - v(y)|, v(y) = -gamma W^{-1}(c + A'y) */
} cc_resid;

typedef struct {
    int32_t sweeps;          /* sweeps run (all phases)                       */
    int32_t sweeps_f32;      /* of which in FP32                              */
    int32_t warm_accepted;   /* 1 if the learned warm start was kept          */
    int32_t warm_sampled;    /* 1 if the sampled gate rejected it (no full
                                inference ran; see cc_set_gate_sample)       */
    double wall_s;           /* wall time of the whole call                   */
    cc_resid resid;          /* final residuals                               */
} cc_info;

/* Residual selection for cc_residuals. */
enum {
    CC_RESID_VIOL = 1,       /* max violations, primal, LP cost (reads x, f)  */
    CC_RESID_CS = 2,         /* + complementary slackness (reads y)           */
    CC_RESID_DUAL = 4,       /* + dual objective, gap, stationarity (A'y pass)*/
    CC_RESID_ALL = 7
};

/* Message for the last error on this thread ("" if none). */
const char *cc_last_error(void);

/* 3 C(n,3): number of metric constraints (rows x_ij <= x_ik + x_jk). */
int64_t cc_num_metric_duals(int64_t n);

/* Create a context for n nodes, tile size b (1..32; the schedule's b of
 * Sec. III-C), precision CC_F64 or CC_F32, and HIP stream `stream`
 * (hipStream_t; NULL = the null stream).  Builds the schedule tables on the
 * device; owns only those tables and small scratch buffers.
 * Errors: CC_EINVAL (n < 3, b outside 1..32, bad prec), CC_ENOMEM, CC_EHIP. */
int cc_create(cc_ctx **out, int64_t n, int32_t b, int32_t prec, void *stream);

/* Release a context and its device tables.  NULL is accepted. */
int cc_destroy(cc_ctx *ctx);

/* Length (elements) of the schedule-ordered metric dual array y.  Each tile
 * (P,Q) of the schedule owns a contiguous segment, laid out as
 * [tile step m][sub-step t][orientation o][lane il*b + kl]; step m visits
 * middle block J = Q - m in the rounds of the first loop of Fig. 2
 * (P + Q < nb) and J = P + m in the others.  Every sub-step reads and writes
 * 3 contiguous vectors of b*b elements.  Slots of index combinations that
 * are not triplets i<j<k<n are padding: zero after cc_init_cold, and a sweep
 * writes back the value it read.  The count is 3 b^3 nb(nb+1)(nb+2)/6 with
 * nb = ceil(n/b), at least 3 C(n,3). */
int64_t cc_dual_slots(const cc_ctx *ctx);

/* Number of rounds of the schedule, 2 ceil(n/b) - 1. */
int32_t cc_num_rounds(const cc_ctx *ctx);

/* g_p = gamma / w_p (= gamma W^{-1} on pair p), written in the context's
 * precision.  w: device double[N_p]; g: device [N_p].  Validates that every
 * w_p is finite and > 0 and gamma > 0 (CC_EINVAL otherwise; synchronises). */
int cc_prepare(cc_ctx *ctx, const double *w, double gamma, void *g);

/* Starting point of Algorithm 1: y = 0 (every slot), y_pair = 0 and
 * v = -(1/eps) W^{-1} c, i.e. x = 0, f = -gamma.  x, f: device [N_p];
 * y: device [cc_dual_slots]; y_pair: device [2 N_p]. */
int cc_init_cold(cc_ctx *ctx, void *x, void *f, void *y, void *y_pair, double gamma);

/* nsweeps full sweeps (Sec. IV-D: one pass over every constraint): all
 * metric rounds in schedule order, then the pair pass.  g from cc_prepare;
 * d: device uint8[N_p].  exec selects the executor (CC_EXEC_ROUNDS: one
 * launch per round; CC_EXEC_DATAFLOW, for b = 8, 16, 24, 32: one persistent
 * launch per sweep whose tile steps wait only for the earlier steps that
 * touch the same blocks of x).  Both executors apply the updates of every
 * variable in the same order and give identical results.  Enqueues only
 * (no host synchronisation).  A dataflow wait longer than 10 s aborts the
 * sweep (the state is then incomplete); no wait can block forever.  Such an
 * abort is reported as CC_EHIP by the next cc_status or cc_residuals call
 * on the context.  The FP64 dataflow sweep (and every sparse sweep)
 * addresses one tile's duals, ceil(n/b) steps of 3 b^3, with 31-bit byte
 * offsets: CC_EINVAL where they do not fit (n above about 87,000 at b = 32
 * in FP64, far beyond what the dual array allows). */
int cc_sweep(cc_ctx *ctx, void *x, void *f, void *y, void *y_pair, const void *g,
             const uint8_t *d, int32_t nsweeps, int32_t exec);

/* One sweep's metric rounds only (no pair pass) with the given executor;
 * enqueues only. */
int cc_sweep_metric(cc_ctx *ctx, void *x, void *y, const void *g, int32_t exec);

/* Sparse dual access (Sec. III-D: most duals are zero, and the paper keeps
 * only the nonzero ones, in visit order, per processor).  The dense
 * schedule-ordered y stays the storage that every other call reads; a mask
 * with one bit per dual slot marks the slots that may hold a nonzero dual.
 * Layout: tile step c (the steps of the tiles in schedule order, each tile's
 * steps in order) owns 3 b^2 words of b bits (uint8 for b = 8, uint16 for
 * 16, uint32 for 24 and 32; at b = 24 the top 8 bits stay clear); bit t of
 * word [c][o][il*b + kl] belongs to dual slot
 * [c][t][o][il*b + kl] of y.  Invariant: a clear bit means the slot holds
 * +0.0 (bit pattern).  The sparse sweeps keep it (they store a dual only
 * where its bits changed and rewrite the mask); any other writer of y
 * (cc_init_cold, cc_warm_start_mlp, cc_sweep, copies) breaks it until
 * cc_dual_mask_build is called again.  A stale mask gives wrong results,
 * not a fault: every access stays inside y and the mask.
 *
 * Bytes of the mask: cc_dual_slots / 8 (cc_dual_slots / 6 at b = 24); -1
 * unless b is 8, 16, 24 or 32. */
int64_t cc_dual_mask_bytes(const cc_ctx *ctx);

/* mask = nonzero pattern of y (device, cc_dual_mask_bytes bytes, caller
 * owned).  One read of y.  Enqueues only.  CC_EINVAL unless b = 8, 16, 24, 32. */
int cc_dual_mask_build(cc_ctx *ctx, const void *y, void *mask);

/* nsweeps full sweeps on the dataflow executor (as cc_sweep with
 * CC_EXEC_DATAFLOW), reading only the marked duals and storing only changed
 * ones.  x, f, y, y_pair equal cc_sweep's bit for bit.  Needs b = 8, 16, 24, 32
 * and a mask that satisfies the invariant above.  Enqueues only. */
int cc_sweep_sparse(cc_ctx *ctx, void *x, void *f, void *y, void *y_pair, const void *g,
                    const uint8_t *d, void *mask, int32_t nsweeps);

/* One sparse sweep's metric rounds only (no pair pass). */
int cc_sweep_metric_sparse(cc_ctx *ctx, void *x, void *y, const void *g, void *mask);

/* Compacted dual lists: the memory form of Sec. III-D, which keeps only
 * the nonzero duals, per processor, in visit order.  Here each tile step of
 * the schedule keeps a list of (slot, dual) pairs for its nonzero metric
 * duals, in a pool the context owns; there is no dense dual array, so n is
 * no longer bounded by 3 C(n,3) duals fitting in memory.  b must be 8 or 16
 * (CC_EINVAL otherwise).  A sweep expands each step's list in LDS, runs the
 * step, and writes the new nonzeros to a second pool; when they do not fit,
 * the sweep is repeated from a saved x into a pool grown to fit
 * (CC_ENOMEM if memory runs out).  Results equal cc_sweep's bit for bit.
 *
 * cc_compact_init: (re)allocates both pools with room for `capacity`
 * entries each (they grow on demand) plus per-step tables (12 bytes a step
 * per pool) and a copy of x, and sets every list empty: the duals of the
 * cold start.  Synchronises. */
int cc_compact_init(cc_ctx *ctx, int64_t capacity);

/* nsweeps full sweeps with compacted lists (dataflow executor): metric
 * rounds, then the pair pass.  x, f, y_pair, g, d as for cc_sweep, from
 * cc_init_cold with y = NULL.  Synchronises once per sweep (overflow
 * check). */
int cc_sweep_compact(cc_ctx *ctx, void *x, void *f, void *y_pair, const void *g,
                     const uint8_t *d, int32_t nsweeps);

/* The current lists as a dense schedule-ordered y (device,
 * cc_dual_slots elements), zeros elsewhere.  Enqueues only. */
int cc_compact_to_slots(cc_ctx *ctx, void *y);

/* *count = entries in the current lists; if lex and val (device, room for
 * `capacity` entries) are given and capacity >= *count, they receive each
 * entry's colex row index 3 tidx(i,j,k) + o and its dual (in the context's
 * precision), in pool order.  Synchronises. */
int cc_compact_export(cc_ctx *ctx, int64_t *lex, void *val, int64_t capacity, int64_t *count);

/* Entries after the last sweep, device bytes the lists and their tables
 * hold, and sweeps repeated to grow a pool (any pointer may be NULL). */
int cc_compact_info(cc_ctx *ctx, int64_t *nnz, int64_t *bytes, int32_t *regrows);

/* Frees the lists (cc_destroy also does). */
int cc_compact_release(cc_ctx *ctx);

/* l1 metric nearness (Sec. II-A): min sum_p w_p |x_p - d_p| over metric x,
 * for real dissimilarities d.  It is (mn1) with real d in place of the 0/1
 * d of correlation clustering, so it is solved exactly like the CC LP: the
 * same (qp), cold start (cc_init_cold), metric sweeps, x(y) (cc_x_from_y)
 * and stop tests; only the pair rows |x_p - d_p| <= f_p read a real d.
 * dv: device double[N_p].
 *
 * nsweeps full sweeps (metric rounds, then the pair pass with real d): the
 * dataflow executor for b = 8, 16, 24, 32 (with mask:
 * sparse dual access, see cc_sweep_sparse), else the round executor (mask
 * must be NULL).
 * Enqueues only. */
int cc_l1_sweep(cc_ctx *ctx, void *x, void *f, void *y, void *y_pair, const void *g,
                const double *dv, void *mask, int32_t nsweeps);

/* Residuals as cc_residuals, with real d in the pair terms (lp_cost is the
 * l1 nearness objective sum w |x - d|).  Synchronises. */
int cc_l1_residuals(cc_ctx *ctx, const void *x, const void *f, const void *y, const void *y_pair,
                    const double *w, const double *dv, double gamma, int32_t what, cc_resid *out);

/* Another visiting order: the sum-mod-n colouring.  Triplets that share a
 * pair conflict (the colouring view of the related-work section); colour t
 * holds every triplet i<j<k with i + j + k = t (mod n), and a pair fixes
 * the third index of its colour, so a colour's triplets share no pair.  A
 * sweep visits colours t = 0..n-1 in turn (one launch each; within a colour
 * the order cannot matter), the three orientations of each triplet as in
 * the schedule, then the pair pass.  Sec. IV-E: the order changes the
 * iterates and the number of sweeps to a tolerance, not the limit.  Duals
 * are in colex order (the layout of cc_duals_to_lex), y_lex:
 * cc_num_metric_duals(n) elements in the context's precision; the context's
 * b is not used.  g, d as for cc_sweep.  Enqueues only. */
int cc_sweep_colour(cc_ctx *ctx, void *x, void *f, void *y_lex, void *y_pair, const void *g,
                    const uint8_t *d, int32_t nsweeps);

/* Cold start for cc_sweep_colour: as cc_init_cold, with the metric duals
 * in colex order (cc_num_metric_duals(n) zeros). */
int cc_init_cold_lex(cc_ctx *ctx, void *x, void *f, void *y_lex, void *y_pair, double gamma);

/* The number of workgroups of the context's dataflow sweeps (b = 8, 16,
 * 24, 32): the GPU counterpart of the paper's processor count in its
 * core-count experiment (Fig. 5).  A count from 1 up applies to every
 * dataflow sweep of the context, capped at the workgroups the GPU holds at
 * once and at one per tile.  0 restores the defaults: the schedule's
 * average parallelism, about (nb+1)(nb+2)/24 tiles, capped at what the GPU
 * holds at once, for the sparse and compacted sweeps; the same, capped per
 * compute unit at the counts measured fastest (b = 8: 4; b = 16: 2 in
 * FP32, 1 in FP64; b = 24, 32: 1), for the dense sweep.  Any count gives
 * the same results bit for bit (tile steps wait for the earlier steps on
 * their blocks, and tiles are taken in schedule order).  *effective (may
 * be NULL) receives the dense sweep's count.  Host only; CC_EINVAL for a
 * negative count or a b without a dataflow kernel. */
int cc_set_dataflow_workgroups(cc_ctx *ctx, int32_t workgroups, int32_t *effective);

/* Diagnostic: one dataflow metric sweep (b = 8, 16, 24, 32) with a time
 * breakdown summed over all workgroups, in microseconds: out[0] waiting for
 * the blocks a tile step needs, out[1] loading them into LDS, out[2] the
 * sub-steps, out[3] publishing; out[4] tile steps run, out[5] workgroups.
 * Synchronises. */
int cc_dataflow_breakdown(cc_ctx *ctx, void *x, void *y, const void *g, double *out);

/* Synchronise the context's stream and report a dataflow sweep aborted
 * since the last check (CC_EHIP), else CC_OK. */
int cc_status(cc_ctx *ctx);

/* Allocation-free variant of cc_sweep with the dataflow executor, for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, hosts that forbid hipMalloc): nsweeps full sweeps,
 * the same kernels and the same results bit for bit as cc_sweep(ctx, ...,
 * nsweeps, CC_EXEC_DATAFLOW).  The executor's scratch (a ticket counter, an
 * abort flag and one touch counter per block of x) lives in a static device
 * array of 4 MiB that each GPU holds until the process ends, instead of in
 * the context; every call clears it first.  Limit: ceil(n/b) <= 255
 * (n <= 8160 at b = 32, 4080 at b = 16), else CC_EINVAL before any work.
 * Calls that overlap on one GPU (any context, any stream) share that GPU's
 * array and race: serialise them.  Makes no hipMalloc or hipFree call.
 * Synchronises the context's stream at the end and returns CC_EHIP if a
 * dependency wait timed out (the state is then incomplete).  CC_EINVAL for a
 * b without a dataflow kernel (8, 16, 24, 32) or nsweeps < 0. */
int cc_sweep_noalloc(cc_ctx *ctx, void *x, void *f, void *y, void *y_pair, const void *g,
                     const uint8_t *d, int32_t nsweeps);

/* Metric rounds [first_round, first_round + nrounds) of one sweep, without
 * the pair pass (for checks against a prefix of the serial order). */
int cc_sweep_rounds(cc_ctx *ctx, void *x, void *y, const void *g, int32_t first_round,
                    int32_t nrounds);

/* The metric rows of the first `nrounds` rounds of one sweep (Sec. III-C's
 * round order), run by the dataflow executor in the launch configuration of
 * a full dataflow sweep (b = 8, 16, 24, 32): the tiles of later rounds are
 * not visited.  Equal bit for bit to cc_sweep_rounds(ctx, x, y, g, 0,
 * nrounds).  For checks of the dataflow kernel against a prefix of the
 * serial order at sizes where a whole sweep of the oracle is too slow.
 * Afterwards the executor's touch counters start a new epoch.  Synchronises;
 * CC_EINVAL for nrounds outside [0, cc_num_rounds], CC_EHIP if a wait timed
 * out. */
int cc_sweep_metric_prefix(cc_ctx *ctx, void *x, void *y, const void *g, int32_t nrounds);

/* The pair pass alone. */
int cc_pair_pass(cc_ctx *ctx, void *x, void *f, void *y_pair, const void *g,
                 const uint8_t *d);

/* Residuals selected by `what` (CC_RESID_*), evaluated in FP64 and copied to
 * *out (host).  y may be NULL when CC_RESID_CS/DUAL are not requested.
 * w: device double[N_p].  Returns CC_ENONFINITE (with *out filled) if x or f
 * holds a NaN or Inf.  Synchronises. */
int cc_residuals(cc_ctx *ctx, const void *x, const void *f, const void *y,
                 const void *y_pair, const double *w, const uint8_t *d, double gamma,
                 int32_t what, cc_resid *out);

/* x = -gamma W^{-1} (c + A'y) from the duals (the stationarity condition of
 * (qp)): accumulates A'y in FP64 in schedule order (deterministic, no
 * atomics), writes x_out, f_out in the context's precision. */
int cc_x_from_y(cc_ctx *ctx, const void *y, const void *y_pair, const double *w,
                double gamma, void *x_out, void *f_out);

/* Copy metric duals from schedule order to colex order (device y_lex of
 * length 3 C(n,3), same precision). */
int cc_duals_to_lex(cc_ctx *ctx, const void *y_sched, void *y_lex);

/* Colex index 3t + o of each schedule slot in slots[0..count) (device int64
 * arrays; -1 for padding slots). */
int cc_slots_to_lex(cc_ctx *ctx, const int64_t *slots, int64_t count, int64_t *lex_out);

/* Host only, no GPU: the dependency tables of the CC_EXEC_DATAFLOW executor
 * for (n, b), for verification.  Tiles are in schedule order; tile t has
 * blocks (P,Q) = tile_pq[2t], tile_pq[2t+1], its first step at jsbase[t],
 * and waits for need_c[t] earlier touches of block (P,Q); step s waits for
 * needs[2s] earlier touches of block (P,J) (J != Q) and needs[2s+1] of block
 * (J,Q) (J != P); K[X] counts the touches of block X = B(B+1)/2 + A per
 * sweep.  Pass NULL outputs to query the sizes first. */
int cc_dataflow_tables(int64_t n, int32_t b, int64_t *ntiles, int64_t *nsteps, int64_t *nblocks,
                       int32_t *tile_pq, uint32_t *need_c, int32_t *jsbase, uint32_t *needs,
                       uint32_t *K);

/* Element-wise precision change (device arrays, count elements):
 * float -> double (widen) or double -> float (narrow). */
int cc_widen(const float *src, double *dst, int64_t count, void *stream);
int cc_narrow(const double *src, float *dst, int64_t count, void *stream);

/* ----- l2 metric nearness (Sec. II-A, the metric nearness problem, p = 2) --
 * min (1/2) sum_p w_p (x_p - d_p)^2 over x satisfying every x_ij <= x_ik +
 * x_jk, for real dissimilarities d (device double[N_p], packed pair order).
 * It is (qp) with v = x alone, W = diag(w), eps = 1, c = -W d and only the
 * metric rows, so Algorithm 1 starts at x = d with y = 0 and one sweep is
 * cc_sweep_metric (either executor) with g = 1/w, i.e. cc_prepare with
 * gamma = 1.  Same schedule, kernels, layouts and precisions as above;
 * there are no f, y_pair or pair rows. */

/* Residuals of the nearness problem, in FP64.  Fields a call did not
 * request are NaN. */
typedef struct {
    double max_viol;     /* max over metric rows of (x_L - x_S1 - x_S2)^+     */
    double primal;       /* (1/2) sum w (x - d)^2                             */
    double dual;         /* d'A'y - (1/2) (A'y)' W^{-1} (A'y)   (CC_RESID_DUAL) */
    double gap;          /* primal - dual                       (CC_RESID_DUAL) */
    double cs_max;       /* max over rows of |y (x_S1 + x_S2 - x_L)| (CC_RESID_CS) */
    double stat_resid;   /* max |x - (d - W^{-1} A'y)|          (CC_RESID_DUAL) */
} cc_nresid;

/* Starting point: x = d in the context's precision, every metric dual 0.
 * Enqueues only.  Errors: CC_EINVAL (null pointer). */
int cc_nearness_init(cc_ctx *ctx, const double *d, void *x, void *y);

/* Residuals selected by `what` (CC_RESID_VIOL, CC_RESID_CS, CC_RESID_DUAL;
 * the last runs one A'y pass).  y may be NULL for CC_RESID_VIOL alone.
 * w, d: device double[N_p].  Returns CC_ENONFINITE (with *out filled) if x
 * holds a NaN or Inf.  Synchronises. */
int cc_nearness_residuals(cc_ctx *ctx, const void *x, const void *y, const double *w,
                          const double *d, int32_t what, cc_nresid *out);

/* ----- Learned warm start (a 4-32-32-1 network per metric row) ---------
 * A nonnegative dual predicted for every metric row is a valid start for
 * Algorithm 1, which is dual coordinate ascent: started from any y >= 0 at
 * x = x(y) it converges to the same unique primal optimum.
 * Network: ReLU after every layer, mean squared error; parameters are one
 * flat fp32 vector of cc_mlp_num_params() values: W1[32][4], b1[32],
 * W2[32][32], b2[32], W3[32], b3.  Products take bf16 operands and
 * accumulate in fp32 (the 32x32 layer, its transpose and the weight
 * gradient on MFMA).  Features of the row x_ab <= x_ac + x_bc (long side
 * (a,b)): (s_ab w_ab, s_ac w_ac, s_bc w_bc, (deg_a + deg_b) / (2 mean deg)),
 * s = +1 for a positive pair, -1 for a negative one; deg: device float[n],
 * the degrees of the unsigned source graph.  The network's output is the
 * dual times n - 2 (the number of triplets through a pair), so one network
 * serves every n: graph training scales the targets by n - 2 and the warm
 * start divides the prediction by it. */

/* Number of network parameters (1249). */
int32_t cc_mlp_num_params(void);

/* Bytes of device workspace a training step over `count` samples needs. */
int64_t cc_mlp_workspace_bytes(int64_t count);

/* Host: He-initialised parameters from a seeded generator. */
int cc_mlp_init(float *params_host, uint64_t seed);

/* y[i] = network(phi[4i..4i+3]) for count samples (device arrays). */
int cc_mlp_forward(const float *params, const float *phi, int64_t count, float *y, void *stream);

/* One training step on explicit samples (device arrays): mean squared error
 * over the count samples, its gradient (written to grad_out if not NULL),
 * then, if lr > 0, one Adam step (beta 0.9/0.999, eps 1e-8, bias-corrected
 * with `step` >= 1) on params with moment buffers adam_m, adam_v.
 * workspace: cc_mlp_workspace_bytes(count) bytes; loss_out: device float. */
int cc_mlp_train_step(const float *phi, const float *target, int64_t count, float *params,
                      float *adam_m, float *adam_v, int32_t step, float lr, float *grad_out,
                      void *workspace, float *loss_out, void *stream);

/* One training step on `batch` metric rows drawn (seeded, with
 * replacement) from the schedule slots of the context's instance, with
 * targets y_star (converged duals, schedule order, context precision);
 * padding slots drawn count as zero-weight samples.  Same update and
 * outputs as cc_mlp_train_step. */
int cc_mlp_train_graph(cc_ctx *ctx, const void *y_star, const double *w, const uint8_t *d,
                       const float *deg, int64_t batch, uint64_t seed, float *params, float *adam_m,
                       float *adam_v, int32_t step, float lr, void *workspace, float *loss_out);

/* Features (4 floats, bf16-rounded) of the metric rows at the given
 * schedule slots (zeros for padding). */
int cc_mlp_slot_features(cc_ctx *ctx, const double *w, const uint8_t *d, const float *deg,
                         const int64_t *slots, int64_t count, float *phi_out);

/* Network prediction for every metric row into y (schedule order, context
 * precision, 0 on padding): the dual a warm start would take, i.e. the
 * network output divided by n - 2 (its training targets are duals times
 * n - 2, the number of triplets through a pair).  Enqueues only. */
int cc_mlp_infer(cc_ctx *ctx, const float *params, const float *deg, const double *w,
                 const uint8_t *d, void *y);

/* Warm start: y = network prediction for every metric row (0 on padding),
 * y_pair = 0, (x, f) = v(y), then one pair pass (which gives the pair duals
 * their best values for this y: the two pair rows of a pair are
 * W-orthogonal).  The gate compares the dual objective D of this start,
 * D_warm, with the cold start's after its first pair pass, D_cold, against
 * an upper bound U on the optimum (the objective at the best constant
 * point x = c, f = |c - d|, which satisfies every row): the start is kept
 * only if D_warm - D_cold >= 0.05 (U - D_cold), i.e. if it closes at least
 * 5% of the gap a cold start faces; otherwise the state is reset to the
 * cold start.  *accepted (nullable) tells which; *dual_warm, *dual_cold and
 * *dual_bound (nullable) return D_warm, D_cold and U.  g from cc_prepare.
 * For large n a sampled gate runs first (cc_set_gate_sample): when it
 * rejects the start, no full inference runs and *dual_warm is D_cold plus
 * the sample's estimate of D_warm - D_cold.  Synchronises. */
int cc_warm_start_mlp(cc_ctx *ctx, const float *params, const float *deg, const double *w,
                      const uint8_t *d, double gamma, void *x, void *f, void *y, void *y_pair,
                      const void *g, int32_t *accepted, double *dual_warm, double *dual_cold,
                      double *dual_bound);

/* Terms of the warm-start gate for `count` pairs given by packed index
 * (pairs: device int64[count], 0 <= p < N_p, repeats allowed; an index out
 * of range gives NaN).  aty_out[s] (device double[count]) is the pair's
 * metric part of A'y at the network's predicted duals: the sum, over every
 * third vertex, of the three rows' predictions, +1 for the row whose long
 * side is the pair and -1 for the other two (the predictions cc_mlp_infer
 * writes, summed in FP64).  delta_out[s] (device double[count], nullable)
 * is the pair's term of D_warm - D_cold.  Once the pair rows have had
 * their pass, the dual objective of (qp) is a sum of one term per pair
 * (the metric rows have b = 0 and W is diagonal), so N_p times the mean of
 * delta_out over a uniform sample estimates the gate's gain without the
 * full inference.  Synchronises. */
int cc_warm_gate_terms(cc_ctx *ctx, const float *params, const float *deg, const double *w,
                       const uint8_t *d, double gamma, const void *g, const int64_t *pairs,
                       int64_t count, double *aty_out, double *delta_out);

/* The sampled gate of cc_warm_start_mlp (and of cc_solve_cc_lp's warm
 * start).  Before the full inference, D_warm - D_cold is estimated from
 * part of the pairs (cc_warm_gate_terms), with its standard error: the
 * terms of every positive pair (d = 0; few, and where the largest terms
 * sit) are summed exactly, and those of the negative pairs are estimated
 * from `count` of them drawn uniformly with replacement (splitmix64, a
 * fixed seed).  The start is rejected without the full inference when the
 * estimate plus four standard errors stays below the gate's least gain, 5%
 * of U - D_cold, and the estimate below half of it; every other start goes
 * to the exact gate.  The estimate runs only when its pairs' rows are at
 * most 1/8 of all metric rows: 24 (positive pairs + count) <= N_p.  A gain
 * concentrated on few negative pairs can escape the sample; the cost of
 * such a rejection is sweeps, not the result.  count: 0 turns the estimate
 * off; default 16384. */
int cc_set_gate_sample(cc_ctx *ctx, int64_t count);

/* What the last cc_warm_start_mlp on this context drew (nullable outputs):
 * pairs whose terms were computed (positive pairs plus draws; 0 if the
 * estimate did not run), the estimate of
 * D_warm - D_cold, its standard error, and 1 if the sample rejected the
 * start. */
int cc_last_gate_sample(const cc_ctx *ctx, int64_t *drawn, double *gain, double *std_error,
                        int32_t *rejected);

/* One-shot solve from host arrays (allocates its own device buffers).
 * w_host: double[N_p] > 0; d_host: uint8[N_p]; tol: stop when both max
 * violations are <= tol and, if gap_tol > 0, also the duality gap (Sec.
 * IV-D stops on constraint satisfaction and the gap) |primal - dual| <=
 * gap_tol max(1, |primal|) (evaluated in FP64, with A'y, only once the
 * violations are below tol; gap_tol <= 0: violations only); mode:
 * CC_MODE_F64, CC_MODE_F32 (FP32 sweeps to tol)
 * or CC_MODE_F32_POLISH (FP32 sweeps to max(tol, 1e-5), or, within a
 * factor of 100 of it, until 20 sweeps bring no new least violation, then
 * duals widened,
 * x recomputed from them in FP64 and FP64 sweeps to tol), or-ed with
 * CC_MODE_SPARSE for sparse dual access (b = 8, 16, 24, 32; same results, the
 * mask allocated and built per phase); warm: CC_WARM_NONE
 * or CC_WARM_MLP (then mlp_weights_host must point to cc_mlp_num_params()
 * floats and deg_host to n floats; see cc_warm_start_mlp for the gate;
 * info->warm_accepted tells whether the start was kept, info->warm_sampled
 * whether the gate's estimate rejected it before the full inference).  x_out_host: double[N_p] or NULL;
 * y_lex_out_host: double[3 C(n,3)] or NULL.  Returns CC_OK, CC_ENOTCONV
 * (info filled, outputs written), or an error. */
int cc_solve_cc_lp(int64_t n, const double *w_host, const uint8_t *d_host, double gamma,
                   double tol, double gap_tol, int32_t max_sweeps, int32_t b, int32_t mode,
                   int32_t warm,
                   const float *mlp_weights_host, const float *deg_host,
                   double *x_out_host, double *y_lex_out_host, cc_info *info);

#ifdef __cplusplus
}
#endif

#endif /* CCPROJ_H */
