/*
 * mplpxx — MPLP++ dual block-coordinate ascent on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the solver library (libmplpxx.so).  All device work runs in the
 * library's own HIP kernels.  Paper: Tourani, Shekhovtsov, Rother,
 * Savchynskyy, "MPLP++: Fast, Parallel Dual Block-Coordinate Ascent for
 * Dense Graphical Models", ECCV 2018.
 *
 * Model (Sec. 3, Eq. (1)): an undirected graph with n nodes and m edges,
 * one label set {0..L-1} for all nodes, unary costs theta_u(s) and pairwise
 * costs theta_uv(s, t).  The solver maximizes the dual lower bound of
 * Eq. (3) over reparametrizations phi (Eq. (2)) by the handshake update (H)
 * of Sec. 4, applied to every edge once per iteration, matching by matching
 * (Sec. 6, Alg. 1).
 *
 * Conventions shared by every call:
 *  - Return value: 0 on success, a negative MPLPXX_E* code on failure; the
 *    text of the last failure on the calling thread is mplpxx_last_error().
 *  - Handles are not thread-safe; use one handle per thread.
 *  - "Host pointer" arguments are read or written before the call returns;
 *    the caller keeps ownership.  "Device pointer" arguments must stay valid
 *    for as long as the handle uses them (stated per call).
 *  - Layouts are row-major and dense:
 *      edges    int32  [m][2]   any order; (u, v) and (v, u) name the same
 *                               edge; a table given for (v, u) is transposed
 *                               internally so that rows always belong to the
 *                               lower node index (Sec. 3 "Notation");
 *      unaries  T      [n][L]   theta_u(s);
 *      pairwise T      [m][L][L] theta_uv(s, t), row s = label of edges[e][0];
 *    with T = float (MPLPXX_F32) or double (MPLPXX_F64).
 *  - Solver state, in the order of the given edge list:
 *      U        T      [n][L]   reparametrized unaries theta^phi_u (Eq. 2);
 *      phi      T      [m][2][L] messages of edge e = (u, v), u < v:
 *                               phi[e][0] = phi_{v->u} (into the lower
 *                               node), phi[e][1] = phi_{u->v} (into the
 *                               upper node); theta^phi_uv(s,t) =
 *                               theta_uv(s,t) - phi[e][0][s] - phi[e][1][t].
 *    The state starts at phi = 0, U = theta_u.
 */
#ifndef MPLPXX_H
#define MPLPXX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* scalar types of costs and state */
#define MPLPXX_F32 0
#define MPLPXX_F64 1

/* error codes */
#define MPLPXX_OK 0
#define MPLPXX_EINVAL (-1)   /* invalid argument or model */
#define MPLPXX_ENOMEM (-2)   /* host or device allocation failed */
#define MPLPXX_EDEVICE (-3)  /* a HIP call failed (text in mplpxx_last_error) */
#define MPLPXX_ETIMEOUT (-4) /* a device-side wait exceeded its bound */
#define MPLPXX_ESTATE (-5)   /* call not valid in the handle's current state */

/* largest label count the kernels accept */
#define MPLPXX_MAX_LABELS 128

/* largest cost magnitude an FP32 handle accepts (costs, and states passed to
 * mplpxx_set_state); the FP32 kernels pad tables with 2^126 and need every
 * real value far below it */
#define MPLPXX_F32_MAX_COST 1e18

typedef struct mplpxx_solver mplpxx_solver;

/* ------------------------------------------------------------------------
 * Core calls.
 * --------------------------------------------------------------------- */

/* Creates a solver for one model (Sec. 3, Eq. (1)) from HOST pointers; the
 * library copies everything to device memory.  Builds the edge schedule
 * (Alg. 1, Sec. 6): the round-robin 1-factorization for a complete graph,
 * greedy maximal matchings (remaining edges scanned in ascending (u, v)
 * order) otherwise.  Initial state phi = 0, U = unaries.
 * Errors: MPLPXX_EINVAL for n < 1, L < 1, L > MPLPXX_MAX_LABELS, m < 0,
 * m > n(n-1)/2, an index out of [0, n), a self loop, a duplicate unordered
 * pair, a non-finite cost (FP32: |cost| > MPLPXX_F32_MAX_COST), a NULL
 * pointer (edges/pairwise may be NULL only
 * when m == 0), an unknown dtype, or out == NULL; MPLPXX_ENOMEM;
 * MPLPXX_EDEVICE.  On error *out is set to NULL. */
int mplpxx_create(int32_t n, int32_t L, int64_t m, const int32_t* edges, const void* unaries,
                  const void* pairwise, int32_t dtype, mplpxx_solver** out);

/* Schedule kinds (Alg. 1, Sec. 6, asks for a queue of matchings covering
 * every edge once; the paper leaves the matchings' construction open).
 * A complete graph always gets the round-robin 1-factorization (n - 1
 * rounds for even n, the minimum).  Any other graph gets
 *   MPLPXX_SCHED_AUTO, MPLPXX_SCHED_GREEDY: greedy maximal matchings, each
 *     round scanning the remaining edges in ascending (u, v) order;
 *   MPLPXX_SCHED_COLOR: the colour classes of a proper edge colouring with
 *     at most Delta + 1 colours (Misra and Gries' constructive proof of
 *     Vizing's theorem), one round per colour in colour order, with every
 *     choice fixed (edges coloured in ascending (u, v) with u as the fan's
 *     centre; smallest free colours; the fan extended by the neighbour whose
 *     edge has the smallest colour free on the fan's last node; the path
 *     from u alternating d, c swapped; the first fan node that takes d
 *     rotated in).  Fewer rounds than the greedy matchings on irregular or
 *     dense graphs: a shorter chain of dependent steps per iteration, and a
 *     different (equally valid) order of the updates.
 * Edges inside a round are listed in ascending (u, v). */
#define MPLPXX_SCHED_AUTO 0
#define MPLPXX_SCHED_GREEDY 1
#define MPLPXX_SCHED_COLOR 2

/* mplpxx_create with a schedule kind (above); MPLPXX_EINVAL for an unknown
 * kind, else the same errors. */
int mplpxx_create_sched(int32_t n, int32_t L, int64_t m, const int32_t* edges, const void* unaries,
                        const void* pairwise, int32_t dtype, int32_t schedule, mplpxx_solver** out);

/* A model with Potts pairwise terms theta_uv(s, t) = w_uv [s != t] (Sec. 4
 * notes that message passing then takes O(L)): weights = HOST float [m],
 * one weight per edge in the order of edges (any sign; -0 counts as +0);
 * unaries as for mplpxx_create (FP32).  The handle runs on the persistent
 * mailbox engine, either with one compute wave per workgroup in label order
 * (three passes of a minimum / second-minimum reduction over the lanes
 * instead of the L x L tile; MPLPXX_OPT_THREADS = 64, the default above 32
 * labels) or with the dense engine's four compute waves, each tile formed
 * in registers from the edge's weight instead of loaded
 * (MPLPXX_OPT_THREADS = 256, the default up to 32 labels); either way its
 * results are bitwise those of an FP32 handle created with the expanded
 * tables.  dual_bound, decode, iterate_gap, get/set_state,
 * schedule and step profile work as for dense handles.  Errors: those of
 * mplpxx_create, and MPLPXX_EINVAL for L > 64 or a node degree >= 65536;
 * later, MPLPXX_EINVAL from mplpxx_iterate_trace, mplpxx_adjoint_forward,
 * MPLPXX_OPT_ENGINE = per-matching, MPLPXX_OPT_THREADS other than 0, 64
 * and 256, and MPLPXX_OPT_RULE other than (H). */
int mplpxx_create_potts(int32_t n, int32_t L, int64_t m, const int32_t* edges, const float* unaries,
                        const float* weights, mplpxx_solver** out);

/* Structured pairwise costs (Sec. 4 notes that for Potts, absolute
 * difference and similar costs the message-passing minimization takes
 * O(|Y|) instead of O(|Y|^2)), given by parameters per edge instead of
 * tables:
 *   MPLPXX_COST_POTTS         theta_uv(s, t) = w [s != t]; 1 parameter: w
 *                             (any sign; -0 counts as +0);
 *   MPLPXX_COST_TRUNC_LINEAR  theta_uv(s, t) = fl(w * min(|s - t|, tau)),
 *                             the FP32 product; 2 parameters: w >= 0 and
 *                             tau >= 0, -0 counting as +0 for both (as for
 *                             the next kind; tau >= L - 1: absolute difference
 *                             w |s - t|; tau <= 1: Potts with weight
 *                             fl(w * tau)); symmetric, so the orientation of
 *                             an edge does not matter;
 *   MPLPXX_COST_TRUNC_QUAD    theta_uv(s, t) = fl(w * min((s - t)^2, tau)),
 *                             the FP32 product (the square is exact); 2
 *                             parameters: w >= 0 and tau >= 0 (tau >=
 *                             (L - 1)^2: quadratic w (s - t)^2; tau <= 1:
 *                             Potts with weight fl(w * tau)); symmetric. */
#define MPLPXX_COST_POTTS 1
#define MPLPXX_COST_TRUNC_LINEAR 2
#define MPLPXX_COST_TRUNC_QUAD 3

/* A model with structured pairwise costs of one kind (above): params = HOST
 * float [m][P] in the order of edges, P = 1 (Potts) or 2 (truncated
 * linear, truncated quadratic); unaries as for mplpxx_create (FP32).  Runs on the persistent
 * mailbox engine with one compute wave per workgroup in label order, or on
 * its four compute waves with each tile formed from the edge's parameters
 * (MPLPXX_OPT_THREADS 64 or 256; the default: formed tiles for the
 * truncated kinds and for Potts costs up to 32 labels, with one compute wave
 * instead of four at 16 labels when a matching has more edges than the
 * device has compute units, as for tables).  Formed tiles hold exactly the
 * expanded table's entries, so that engine gives the dense handle's bits for
 * every kind.  In label order:
 * Potts: as mplpxx_create_potts (bitwise the dense handle on
 * the expanded tables).
 * Truncated linear: each pass is a min-plus distance transform in O(L) work
 * and O(log L) steps (prefix and suffix minima of x(t) + w |s - t| by
 * doubling distances within rows of 16 lanes, carried across rows, then the
 * truncation at min_t x(t) + fl(w tau)); the sums are formed in a different
 * order than x(t) + fl(w |s - t|), so results agree with the expanded
 * tables up to FP32 rounding, not bitwise.  Truncated quadratic: no table
 * is stored or read; lane s of the pass evaluates every candidate
 * fl(x(t) + fl(w min((s - t)^2, tau))) from the two parameters (O(L) steps
 * with L lanes), so the results are bitwise those of the dense engine on
 * the expanded table.  dual_bound, decode,
 * iterate_gap, get/set_state and the schedule work as for dense handles
 * (on the expanded costs).  Errors: those of mplpxx_create_potts, and
 * MPLPXX_EINVAL for an unknown kind or, for truncated linear and
 * quadratic, w < 0, tau < 0, a non-finite parameter or a cost above
 * MPLPXX_F32_MAX_COST. */
int mplpxx_create_structured(int32_t n, int32_t L, int64_t m, const int32_t* edges, const float* unaries,
                             int32_t kind, const float* params, mplpxx_solver** out);

/* Same as mplpxx_create, but unaries and pairwise are DEVICE pointers (for
 * example torch tensor storage) in the same layout; edges stay on the host.
 * The library copies the costs into its own layout before returning, so the
 * device buffers may be reused afterwards.  The copy runs on the stream
 * given (NULL = the default stream).  Errors: those of mplpxx_create, and
 * MPLPXX_EINVAL when unaries_dev or pairwise_dev is not device memory of the
 * current device (checked with hipPointerGetAttributes before any kernel
 * reads it). */
int mplpxx_create_device(int32_t n, int32_t L, int64_t m, const int32_t* edges, const void* unaries_dev,
                         const void* pairwise_dev, int32_t dtype, void* hip_stream, mplpxx_solver** out);

/* Runs k >= 0 full BCA-iterations (Sec. 5 "BCA-iteration"): every edge gets
 * one (H) update, matching after matching.  Synchronous unless a stream was
 * set with mplpxx_set_stream, in which case the work is queued on it and the
 * value-returning calls below synchronize that stream.  MPLPXX_ETIMEOUT
 * means a device wait exceeded its bound (the state is then undefined). */
int mplpxx_iterate(mplpxx_solver* h, int32_t k);

/* Dual lower bound D(phi) of Eq. (3) for the current state, recomputed from
 * the input costs and the messages (node terms theta_u + sum of incoming
 * messages, edge terms theta_uv - phi[e][0] - phi[e][1]) with FP64
 * accumulation, written to the HOST pointer out. */
int mplpxx_dual_bound(mplpxx_solver* h, double* out);

/* Sequential primal rounding of Eq. (5) on the reparametrized costs: nodes
 * in ascending index order, each takes the label minimizing its
 * reparametrized unary plus the reparametrized pairwise terms to its
 * already-labelled lower neighbours (sums in FP64, ties to the smallest
 * label).  labels: HOST int32 [n].  energy (HOST, may be NULL): Eq. (1) of
 * that labelling on the original costs, accumulated in FP64. */
int mplpxx_decode(mplpxx_solver* h, int32_t* labels, double* energy);

/* Anytime primal-dual gap: runs k >= 1 iterations and after each one
 * records the certified dual bound of Eq. (3) (as mplpxx_dual_bound) in
 * dual[i] and the Eq. (1) energy of the rounding of Eq. (5) (as
 * mplpxx_decode) in energy[i]; best_labels (may be NULL) receives the
 * labelling of the lowest energy seen (the earliest on ties).  Every
 * energy[i] >= every dual[j] (weak duality), so min energy - max dual is a
 * certified bound on the distance of both to the optimum.  All three are
 * HOST buffers (dual, energy: k doubles; best_labels: n int32).  Costs one
 * dual and one rounding per iteration on top of the iteration itself.
 * Errors: MPLPXX_EINVAL (k < 1, NULL dual or energy), MPLPXX_ENOMEM, and
 * those of mplpxx_iterate. */
int mplpxx_iterate_gap(mplpxx_solver* h, int32_t k, double* dual, double* energy, int32_t* best_labels);

/* Frees the handle and all its device memory; NULL is a no-op.  Waits for
 * queued work on the handle's stream first. */
void mplpxx_destroy(mplpxx_solver* h);

/* Static text for an error code. */
const char* mplpxx_error_string(int code);

/* Text of the last failure on the calling thread ("" if none). */
const char* mplpxx_last_error(void);

/* Measured streaming-read rate of the current device, the ceiling reported
 * beside the published HBM bandwidth for the kernels' bandwidth fractions
 * (each of the three passes of Sec. 4 reads every entry of the edge's
 * read-only table once, so the dense kernels are bounded by read
 * streaming).  Allocates a buffer of `bytes` (a multiple of 16, at least 1
 * MiB), fills it with zeros, and times `reps` (1..1000) launches of a plain
 * read kernel (16-byte nontemporal loads at a grid stride, eight in flight
 * per thread, sixteen 256-thread workgroups per compute unit) after one
 * warm-up launch, each with HIP events on its
 * own stream; writes the median and (if gbs_best is not NULL) the best rate
 * in GB/s (1e9 bytes per second) to the HOST pointers.  Frees everything
 * before returning.  Errors: MPLPXX_EINVAL for a bad size, count or NULL
 * gbs_median; MPLPXX_ENOMEM; MPLPXX_EDEVICE. */
int mplpxx_stream_read_probe(int64_t bytes, int32_t reps, double* gbs_median, double* gbs_best);

/* ------------------------------------------------------------------------
 * Extensions (streams, schedule, state, traces, tuning).
 * --------------------------------------------------------------------- */

/* Sets the HIP stream (a hipStream_t, e.g. torch.cuda.current_stream()
 * .cuda_stream) the handle queues its work on; NULL restores the library's
 * synchronous default. */
int mplpxx_set_stream(mplpxx_solver* h, void* hip_stream);

/* Copies the schedule of Alg. 1 to HOST buffers: step_ptr int32 [S+1] and
 * order int32 [m] (edge indices of the input list, matching by matching,
 * each matching in ascending (u, v) order).  Pass NULL buffers to query S
 * alone through n_steps. */
int mplpxx_get_schedule(mplpxx_solver* h, int32_t* n_steps, int32_t* step_ptr, int32_t* order);

/* Host-only (no device work, usable without a GPU): the schedule that
 * mplpxx_create would build for this graph (Alg. 1, Sec. 6; see
 * mplpxx_create).  edges: HOST int32 [m][2].  step_ptr needs m + 1 entries
 * and order m entries; pass NULL for both to query only n_steps.  Errors:
 * MPLPXX_EINVAL for the graph errors listed under mplpxx_create. */
int mplpxx_schedule(int32_t n, int64_t m, const int32_t* edges, int32_t* n_steps, int32_t* step_ptr,
                    int32_t* order);

/* Host-only: the schedule of the given kind (MPLPXX_SCHED_*), as
 * mplpxx_create_sched would build it; otherwise as mplpxx_schedule. */
int mplpxx_schedule_kind(int32_t n, int64_t m, const int32_t* edges, int32_t schedule, int32_t* n_steps,
                         int32_t* step_ptr, int32_t* order);

/* Copies the state (U [n][L], phi [m][2][L], see above) to / from HOST
 * buffers of the handle's dtype.  Any pointer may be NULL to skip it.
 *
 * FP32 handles keep each reparametrized unary as an unevaluated sum
 * U + U_comp: U in FP32 and U_comp a small correction rounded to bf16 that
 * carries the rounding error of the running sum theta_u + (messages into u)
 * (Sec. 4, (H)), updated with error-free additions, so the sum does not
 * drift with the number of updates.  U_comp: HOST float [n][L].  get_state
 * writes zeros for FP64 handles; set_state takes it only together with U
 * (NULL: zero correction), rounds it to bf16, and rejects it for FP64
 * handles (MPLPXX_EINVAL).  Passing back what get_state returned resumes a
 * run bit for bit. */
int mplpxx_get_state(mplpxx_solver* h, void* U, void* phi, float* U_comp);
int mplpxx_set_state(mplpxx_solver* h, const void* U, const void* phi, const float* U_comp);

/* Same as mplpxx_iterate, and writes to the HOST buffer trace[k] the dual
 * bound of Eq. (3) after every iteration, accumulated in FP64: the node
 * terms sum_u min_s U_u(s) plus, for FP32 handles, the edge terms
 * min_{s,t} [theta_e(s,t) - phi_e[0](s) - phi_e[1](t)] of the state after
 * that iteration, computed exactly from the FP32 values.  (After an edge's
 * (H) update its edge term is zero in exact arithmetic, Sec. 4 after (H);
 * in FP32 it is a rounding-level number, and summed over many edges it is
 * not negligible.)  In FP64 the edge terms are left out. */
int mplpxx_iterate_trace(mplpxx_solver* h, int32_t k, double* trace);

/* Tuning options (never change results: every option gives bitwise the same
 * state, because each entry of a pass is one IEEE add followed by an exact,
 * order-free minimum). */
#define MPLPXX_OPT_ENGINE 1      /* 0 auto, 1 one launch per matching, 2 persistent
                                    (FP32 handles with a node of degree >= 65536
                                    always run one launch per matching) */
#define MPLPXX_OPT_THREADS 2     /* threads per workgroup: 0 auto, 256, 512, 1024; 64 (one compute
                                    wave, FP32 persistent engine) up to 32 labels */
#define MPLPXX_OPT_GRID 3        /* workgroups of the persistent engine (0 auto) */
#define MPLPXX_OPT_SPIN_LIMIT 4  /* device wait bound in polls (0 default) */
#define MPLPXX_OPT_PROFILE 5     /* 1: record per-slot timestamps (persistent FP32 engine) */
#define MPLPXX_OPT_ADJOINT_F64 6 /* FP32 handles: 1 (default) differentiate an FP64 run on the same costs
                                    (exactly widened); 0: differentiate the FP32 run itself */
#define MPLPXX_OPT_PHI 8         /* FP32 persistent engine, where a workgroup keeps the messages of its
                                    slots: 0 auto (LDS when they fit 96 KB and one workgroup runs per
                                    compute unit), 1 the same, 2 global memory */
#define MPLPXX_OPT_PREFETCH 9    /* FP32 persistent engine, dense tables up to 64 labels: steps ahead the
                                    tables are loaded into the register ring, 0 auto (2), 1 or 2
                                    (per-iteration traces always use 2) */
/* The BCA-update applied to every edge (Sec. 4), unlike the options above a
 * change of the method: MPLPXX_RULE_H (default) the MPLP++ handshake (H);
 * MPLPXX_RULE_M the MPLP update (M), both nodes get half of the row and
 * column minima of the aggregated cost; MPLPXX_RULE_U the uniform update
 * (U), both nodes get half of its overall minimum.  Traces under (M) or
 * (U), FP64 handles and MPLPXX_OPT_THREADS other than 0 or 256 run the
 * per-matching engine whatever MPLPXX_OPT_ENGINE says; mplpxx_iterate of
 * an FP32 handle under (M) or (U) runs the persistent mailbox engine (four
 * compute waves; two passes per update for (M), one and a reduction for
 * (U)) unless MPLPXX_OPT_ENGINE asks for the per-matching one, with the
 * same bits; MPLPXX_INFO_ENGINE reports the per-matching engine for (M)
 * and (U).  The adjoint and the batch API take
 * (H) only (mplpxx_adjoint_forward returns MPLPXX_EINVAL under another
 * rule). */
#define MPLPXX_OPT_RULE 7
#define MPLPXX_RULE_H 0
#define MPLPXX_RULE_M 1
#define MPLPXX_RULE_U 2
int mplpxx_set_option(mplpxx_solver* h, int32_t key, int64_t value);

/* Read-only facts about the handle. */
#define MPLPXX_INFO_N 1
#define MPLPXX_INFO_L 2
#define MPLPXX_INFO_M 3
#define MPLPXX_INFO_STEPS 4
#define MPLPXX_INFO_DTYPE 5
#define MPLPXX_INFO_ENGINE 6     /* engine the next iterate call will use */
#define MPLPXX_INFO_GRID 7       /* workgroups of the persistent engine */
#define MPLPXX_INFO_THREADS 8    /* threads per workgroup */
#define MPLPXX_INFO_ITERATIONS 9 /* iterations run since create / set_state */
#define MPLPXX_INFO_WALLCLOCK_KHZ 10 /* device wall-clock rate of the timestamps */
#define MPLPXX_INFO_ADJOINT_BYTES 11 /* device bytes held for the adjoint after mplpxx_adjoint_forward
                                        (checkpoints, argmin records, adjoint buffers; for an FP32 handle
                                        differentiating its FP64 twin, also the twin's costs and state) */
int mplpxx_get_info(mplpxx_solver* h, int32_t key, int64_t* value);

/* Per-slot timestamps of the last iteration of the last iterate call of the
 * persistent FP32 engine with MPLPXX_OPT_PROFILE set: HOST int64 [m][4] in
 * schedule (slot) order = (start of the wait for the lower node, its data
 * seen, upper node's data seen, results stored), in device wall-clock ticks
 * (MPLPXX_INFO_WALLCLOCK_KHZ).  MPLPXX_ESTATE if nothing was recorded. */
int mplpxx_get_step_profile(mplpxx_solver* h, int64_t* stamps);

/* Average duration in milliseconds of the device work of the last iterate
 * call, measured with HIP events on the handle's stream around the launch
 * (0 if none). */
int mplpxx_last_iterate_ms(mplpxx_solver* h, double* ms);

/* ------------------------------------------------------------------------
 * Differentiation: adjoint of K unrolled iterations.
 * --------------------------------------------------------------------- */

/* Resets the state to phi = 0, U = unaries, runs K >= 1 iterations with the
 * handle's engine, keeping a checkpoint of (U, phi) every `every` >= 1
 * iterations, and writes to the HOST pointer `loss` (may be NULL) the dual
 * bound D_K of Eq. (3) of the final state (as mplpxx_dual_bound).  After the
 * last sweep every edge's reparametrized pairwise term has minimum zero
 * (Sec. 4, after (H)), so in exact arithmetic D_K = sum_u min_s U_u(s); the
 * gradient below is that of this sum.
 *
 * FP32 handles with MPLPXX_OPT_ADJOINT_F64 = 1 (the default) differentiate
 * an FP64 run on the same costs (widened exactly, kept in a second, FP64
 * state inside the handle), and `loss` is that run's D_K.  Reason: D_K is
 * piecewise linear with kinks at every scale, and the FP32 run, which
 * rounds at the 1e-7 level, selects a neighbouring linear piece for a few
 * percent of the minimizers; its gradient is exact for the FP32 iterates
 * but differs from the FP64 one by about 1% along a generic direction.  The
 * handle's own FP32 state still ends at its FP32 run of K iterations. */
int mplpxx_adjoint_forward(mplpxx_solver* h, int32_t K, int32_t every, double* loss);

/* Gradient of D_K with respect to the input costs, by reverse sweeps over
 * the recorded minimizers (recomputing each segment from its checkpoint).
 * FP64 runs with L <= 64 (an FP64 handle, or the FP64 run of an FP32
 * handle) use persistent kernels unless MPLPXX_OPT_ENGINE = 1: one launch
 * reverses a segment while it recomputes the previous one, the node values
 * and their adjoints passing between workgroups through tagged mailbox
 * words; otherwise one launch per matching.  Both give the same bits.
 * Output:
 * DEVICE buffers grad_unaries [n][L] and grad_pairwise [m][L][L] in the
 * handle's dtype and in the caller's layout (edge order and orientation of
 * mplpxx_create).  D_K is piecewise linear in the costs; the gradient is the
 * one of the linear piece selected by the recorded minimizers (lowest label
 * on ties).  Either pointer may be NULL.  MPLPXX_ESTATE if no
 * mplpxx_adjoint_forward preceded it or the state was changed since.  The
 * handle's state is left at the end of the forward. */
int mplpxx_adjoint_backward(mplpxx_solver* h, void* grad_unaries, void* grad_pairwise);

/* ------------------------------------------------------------------------
 * Solving without device allocation.
 * --------------------------------------------------------------------- */

/* Working memory of mplpxx_solve_noalloc, in MiB: one static device array
 * per GPU, held by each GPU the library runs on until the process ends. */
#define MPLPXX_NOALLOC_SCRATCH_MB 64

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the work of
 * mplpxx_create_device + mplpxx_iterate(iters) + mplpxx_dual_bound + reading
 * the state, in one call that allocates nothing on the device.  Its working
 * memory (tables packed in schedule order, messages, mailboxes, schedule
 * metadata, reduction buffers) lives in a static device array of
 * MPLPXX_NOALLOC_SCRATCH_MB MiB per GPU; the results are bitwise those of the
 * allocating calls on the same FP32 model (default schedule, engine and
 * launch shape).
 *   edges        HOST int32 [m][2], as for mplpxx_create (any orientation);
 *   unaries_dev  DEVICE float [n][L], pairwise_dev DEVICE float [m][L][L]
 *                (read only; layouts of mplpxx_create);
 *   U_dev        DEVICE float [n][L], out: the reparametrized unaries U after
 *                `iters` >= 0 iterations (as mplpxx_get_state's U);
 *   phi_dev      DEVICE float [m][2][L], out: the messages in edge order (as
 *                mplpxx_get_state's phi);
 *   dual         HOST double, out (may be NULL): Eq. (3) of that state, as
 *                mplpxx_dual_bound;
 *   hip_stream   the stream the work is queued on (NULL = the default
 *                stream); the call returns after it is done.
 * All device buffers must be memory of the current device.  Errors:
 * MPLPXX_EINVAL for the model errors of mplpxx_create, non-device buffers,
 * a node degree >= 65536, or a model whose working memory exceeds the array
 * (the message names the size needed; the pose workload n = 200, L = 64 does
 * not fit, n = 100, L = 32 does); MPLPXX_ETIMEOUT, MPLPXX_EDEVICE.  Calls on
 * one GPU share its array and must not overlap (one at a time per GPU, from
 * any thread or stream); the array keeps the last call's contents and every
 * call clears what it needs cleared. */
int mplpxx_solve_noalloc(int32_t n, int32_t L, int64_t m, const int32_t* edges, const float* unaries_dev,
                         const float* pairwise_dev, int32_t iters, float* U_dev, float* phi_dev, double* dual,
                         void* hip_stream);

/* ------------------------------------------------------------------------
 * Batched solving: many independent FP32 models in one persistent launch.
 * --------------------------------------------------------------------- */

typedef struct mplpxx_batch mplpxx_batch;

/* Creates a batch of `count` independent FP32 models (each as in
 * mplpxx_create: Sec. 3, Eq. (1); own schedule of Alg. 1).  n[i], L[i], m[i]
 * are HOST arrays of sizes; edges[i], unaries[i], pairwise[i] HOST pointers
 * to model i's arrays in the layouts of mplpxx_create (edges[i] and
 * pairwise[i] may be NULL when m[i] == 0).  Everything is copied to device
 * memory; the library plans which workgroups run which model (large models
 * are split over a team of workgroups, small ones packed together).  Errors
 * as mplpxx_create, reported with the model index; also MPLPXX_EINVAL for a
 * node of degree >= 65536 (the mailboxes carry 16-bit update counts). */
int mplpxx_batch_create(int32_t count, const int32_t* n, const int32_t* L, const int64_t* m,
                        const int32_t* const* edges, const float* const* unaries, const float* const* pairwise,
                        mplpxx_batch** out);

/* A batch of Potts models (Sec. 4 notes that the message-passing
 * minimization takes O(L) for such pairwise terms): the pairwise term of
 * edge e is w_e [s != t], given as weights[i] = HOST float [m[i]] (one
 * weight per edge, in the edge order of edges[i]); everything else as
 * mplpxx_batch_create.  The passes then take O(L) per update instead of
 * O(L^2) (minimum and second minimum over the labels) and read 4 bytes of
 * pairwise data instead of 4 L^2; every result is bitwise the one of the
 * dense engine on the table w_e [s != t] (a weight of -0 counts as +0).
 * Runs on the wave engine: L[i] <= 64 (else MPLPXX_EINVAL), and
 * MPLPXX_BOPT_ENGINE = 1 is rejected when the plan is made.  A batch holds
 * either dense models or Potts models. */
int mplpxx_batch_create_potts(int32_t count, const int32_t* n, const int32_t* L, const int64_t* m,
                              const int32_t* const* edges, const float* const* unaries, const float* const* weights,
                              mplpxx_batch** out);

/* A batch of models with structured pairwise costs of one kind
 * (MPLPXX_COST_*, see mplpxx_create_structured): params[i] = HOST float
 * [m[i]][P]; everything else as mplpxx_batch_create_potts (wave engine,
 * L[i] <= 64).  Errors: those of mplpxx_batch_create_potts and the
 * parameter errors of mplpxx_create_structured, with the model index. */
int mplpxx_batch_create_structured(int32_t count, const int32_t* n, const int32_t* L, const int64_t* m,
                                   const int32_t* const* edges, const float* const* unaries, int32_t kind,
                                   const float* const* params, mplpxx_batch** out);

/* Runs k >= 0 BCA-iterations (Sec. 5) of every model of the batch in one
 * persistent launch (by default replayed from a hipGraph captured for this
 * k), and waits for it.  Each model's results are bitwise those of
 * mplpxx_iterate on the same model.  MPLPXX_ETIMEOUT: a device wait exceeded
 * its bound (state undefined). */
int mplpxx_batch_iterate(mplpxx_batch* b, int32_t k);

/* Dual bound of Eq. (3) of every model (HOST double [count]), recomputed in
 * FP64 from costs and messages as in mplpxx_dual_bound. */
int mplpxx_batch_dual_bounds(mplpxx_batch* b, double* out);

/* State of one model (HOST float U [n][L], phi [m][2][L], U_comp [n][L],
 * layouts of mplpxx_get_state; any may be NULL). */
int mplpxx_batch_get_state(mplpxx_batch* b, int32_t model, float* U, float* phi, float* U_comp);

/* Back to phi = 0, U = unaries for every model. */
int mplpxx_batch_reset(mplpxx_batch* b);

/* Planning and execution options (results never depend on them). */
#define MPLPXX_BOPT_GRID 1           /* workgroups of the launch (0: all that fit) */
#define MPLPXX_BOPT_GRAPH 2          /* 1: replay a captured hipGraph (default), 0: plain launches */
#define MPLPXX_BOPT_SPIN_LIMIT 3     /* device wait bound in polls (0 default) */
#define MPLPXX_BOPT_ONE_PER_MODEL 4  /* 1: no teams, every model on one workgroup */
#define MPLPXX_BOPT_HANDOFF_US 5     /* planner: cost of one cross-workgroup handoff */
#define MPLPXX_BOPT_EDGE16_US 6      /* planner: cost of one edge update, L <= 16 */
#define MPLPXX_BOPT_EDGE32_US 7      /*                                   L <= 32 */
#define MPLPXX_BOPT_EDGE64_US 8      /*                                   L <= 64 */
#define MPLPXX_BOPT_EDGE128_US 9     /*                                   L <= 128 */
#define MPLPXX_BOPT_LDS 10           /* 1 (default): a model on one workgroup keeps its unaries in LDS
                                        when they fit; 0: always through the mailboxes */
#define MPLPXX_BOPT_ENGINE 11        /* 0 (default): the wave engine when every L <= 64, else the
                                        workgroup engine; 1: workgroup engine (one update at a time per
                                        workgroup, the single-model engine's kernel code); 2: wave engine
                                        (one update per wavefront, many in flight per workgroup; L <= 64,
                                        else MPLPXX_EINVAL when the plan is made) */
#define MPLPXX_BOPT_WAVE_EDGE16_US 12 /* wave-engine planner: workgroup time per edge update, L <= 16 */
#define MPLPXX_BOPT_WAVE_EDGE32_US 13 /*                                                      L <= 32 */
#define MPLPXX_BOPT_WAVE_EDGE64_US 14 /*                                                      L <= 64 */
#define MPLPXX_BOPT_WAVE_LAT_LDS_US 15 /* wave-engine planner: latency of one update, unaries in LDS */
#define MPLPXX_BOPT_WAVE_LAT_MB_US 16  /* wave-engine planner: latency of one update through mailboxes */
#define MPLPXX_BOPT_QUEUE 17         /* 1 (default): models on one workgroup are taken, longest first,
                                        from a shared queue by whichever workgroup is free; 0: packed
                                        onto workgroups by the planner */
int mplpxx_batch_set_option(mplpxx_batch* b, int32_t key, double value);

#define MPLPXX_BINFO_COUNT 1
#define MPLPXX_BINFO_GRID 2
#define MPLPXX_BINFO_TASKS 3
#define MPLPXX_BINFO_TEAMS 4         /* models split over more than one workgroup */
#define MPLPXX_BINFO_MAX_TEAM 5
#define MPLPXX_BINFO_PLAN_US 6       /* planner's estimate of the makespan per iteration */
#define MPLPXX_BINFO_EDGES 7         /* total edges */
#define MPLPXX_BINFO_LAST_MS 8       /* device time of the last batch_iterate (HIP events) */
#define MPLPXX_BINFO_TABLE_BYTES 9   /* bytes of pairwise tables */
#define MPLPXX_BINFO_LDS_TASKS 10    /* models run with LDS-resident unaries */
#define MPLPXX_BINFO_LDS_BYTES 11    /* dynamic LDS per workgroup of the launch */
#define MPLPXX_BINFO_ENGINE 12       /* engine of the plan: 1 workgroup, 2 wave */
#define MPLPXX_BINFO_WAVES 13        /* wave engine: waves (workers) per workgroup */
#define MPLPXX_BINFO_WG_MAX_US 14    /* last launch: longest start-to-end time of a workgroup (us) */
#define MPLPXX_BINFO_WG_MEAN_US 15   /* last launch: mean start-to-end time of the workgroups (us) */
int mplpxx_batch_get_info(mplpxx_batch* b, int32_t key, double* value);

/* Where the last launch spent its time, per logical workgroup w (0 <= w <
 * MPLPXX_BINFO_GRID): start_end_us[2w], start_end_us[2w+1] = its start and
 * end in microseconds after the earliest start (device clock, 10 ns
 * resolution; caller-owned, 2 * grid doubles); team_model[w] = the model of
 * its own (team) task, -1 if it ran only tasks from the shared queue
 * (caller-owned, grid entries, may be NULL).  Before any launch of the
 * current plan the times are 0.  Errors: MPLPXX_EINVAL for a NULL handle or
 * start_end_us, MPLPXX_EDEVICE if the copy fails. */
int mplpxx_batch_wg_profile(mplpxx_batch* b, double* start_end_us, int32_t* team_model);

/* Frees the batch and its device memory; NULL is a no-op. */
void mplpxx_batch_destroy(mplpxx_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* MPLPXX_H */
