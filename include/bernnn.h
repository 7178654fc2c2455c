/*
 * bernnn.h -- C ABI of the MI355X (gfx950) BERN-NN bound-propagation library.
 *
 * The library computes, for a fully connected ReLU network and an input box
 * I_n(d_lo, d_hi), polynomial upper/lower approximations of every neuron
 * (Problem 1 of the paper, Section 2.2) and the absolute bounds they give
 * (Section 5.3, last paragraph): the pre-activation interval [lo, hi] of each
 * hidden neuron (Step 1 of Section 5.1) and the output interval of each network
 * output (Def. 2 applied to the output polynomials).
 *
 * Polynomials live on the GPU as power-basis coefficients in the
 * box-normalised coordinate t in [0,1]^n (x = d_lo + (d_hi - d_lo) t). A
 * polynomial of per-variable degree D on the path has total degree at most D,
 * so only its C(n+D, n) coefficients of exponent sum <= D are stored (graded
 * order); bounds are read from the full tensor-product Bernstein form of
 * per-variable degree D (Section 4.1, Def. 2), expanded on the fly. The
 * step-level entry points below take dense (D+1)^n tensors, last variable
 * fastest (the layout of Section 4.1, Example 1, in the power basis).
 *
 * Conventions for every entry point below:
 *   - Pointers named "device" are GPU (HBM) pointers on the current HIP device;
 *     "host" pointers are ordinary CPU memory.
 *   - Calls taking a `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream) are asynchronous with respect to the host: they only
 *     enqueue work. Their results are valid once the stream has completed.
 *     Scratch comes from the caller's workspace; the only device memory the
 *     library allocates is owned by handles (the network's weights, and its
 *     index tables of the total-degree layout, built synchronously the first
 *     time a call meets a new degree and freed by bern_net_destroy).
 *   - The caller owns every array it passes. The library owns the handles it
 *     returns and the device copies of the weights made at creation; it keeps
 *     no caller pointer after the call returns (the enqueued work still reads
 *     and writes them until the stream completes).
 *   - No exception crosses this interface. On error nothing is enqueued (or,
 *     for errors detected on the device, the outputs are unspecified), the
 *     status says why and bern_last_error() returns a message for the calling
 *     thread.
 *   - All matrices are row-major.
 */
#ifndef BERNNN_H
#define BERNNN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BERN_OK = 0,
  BERN_E_ARG = -1,       /* null pointer, count < 1, unknown enum value            */
  BERN_E_SHAPE = -2,     /* widths / degree combination the library cannot hold    */
  BERN_E_BOX = -3,       /* d_lo > d_hi or a non-finite box coordinate (host check) */
  BERN_E_DEGREE = -4,    /* L outside 1..8, or a degree code outside its range     */
  BERN_E_TOO_LARGE = -5, /* (D+1)^n overflows, or one box does not fit the workspace */
  BERN_E_OOM = -6,       /* a library-side allocation (handles, weights) failed    */
  BERN_E_WORKSPACE = -7, /* workspace pointer/size unusable (null, misaligned)     */
  BERN_E_DEVICE = -8,    /* a HIP runtime call failed                              */
  BERN_E_NUMERIC = -9    /* non-finite weights or a non-finite intermediate bound  */
} bern_status;

typedef enum {
  BERN_FP64 = 0,        /* every tensor and every operation in FP64                 */
  BERN_FP32_PADDED = 1  /* FP32 tensors, FP64 basis change and scalars; every bound
                           is pushed outward by a rigorous rounding-error radius   */
} bern_precision;

typedef enum {
  BERN_PLAN_PLAIN = 0,   /* the paper's rule: ReLU order L for every unstable neuron,
                            all neurons of hidden layer i stored at degree L*D_i
                            (Section 5.4, elevation to the highest expected degree) */
  BERN_PLAN_GIVEN = 1,   /* caller's int8 code per (box, hidden neuron): k >= 1 = ReLU
                            Bernstein order for that neuron if unstable, k <= 0 =
                            linear fallback; stable neurons keep degree D (active)
                            or 0 (inactive); a box's layer is stored at the largest
                            degree of its neurons. Orders are lowered until the
                            post degree k*D stays within the plain rule's degree
                            at order L (opts.L) for that layer, so no tensor
                            outgrows the plain form's                          */
  BERN_PLAN_LEARNED = 2  /* like GIVEN, with the codes chosen on the device by a
                            degree predictor (bern_pred) from each neuron's interval
                            and coefficient statistics                             */
} bern_plan;

typedef enum {
  BERN_SCHED_PER_BOX = 0, /* one launch sequence per box (the plain form)            */
  BERN_SCHED_BATCHED = 1  /* as many boxes per launch sequence (wave) as the
                             workspace holds; with opts.graph, one graph launch     */
} bern_sched;

typedef struct bern_net bern_net;   /* opaque: network on the device               */
typedef struct bern_pred bern_pred; /* opaque: degree predictor (MLP) on the device */

typedef struct {
  int32_t L;          /* ReLU approximation order of the plain rule, 1..8; for the
                         GIVEN / LEARNED plans the degree cap (see bern_plan)      */
  int32_t precision;  /* bern_precision                                            */
  int32_t plan;       /* bern_plan                                                 */
  int32_t sched;      /* bern_sched                                                */
  const bern_pred *pred; /* predictor for BERN_PLAN_LEARNED, else ignored           */
  float *features;    /* optional device output [n_boxes][sum hidden][8]: the
                         predictor's input features of every hidden neuron
                         (written in every plan mode; for training records)      */
  int32_t max_wave;   /* upper limit on boxes per wave (0 = as many as fit)         */
  int32_t graph;      /* nonzero: the call's launch sequence is captured once per
                         distinct argument set into a HIP graph and replayed as one
                         graph launch. Per-neuron plans (GIVEN, LEARNED) then list
                         their boxes' degree classes on the device: every class the
                         rules can give is launched with its box count read from
                         device memory (no host round trip). When those classes
                         are too many (over 48 (pre, post) degree pairs in all,
                         or over 64 lists in one layer) or their index tables
                         exceed their limits, the call runs eagerly as with
                         graph = 0 (bern_stats.graph tells). The outputs are
                         bit-for-bit those of graph = 0. Zero: eager launches;
                         per-neuron plans read every box's post degree back to
                         the host once per hidden layer                         */
  int32_t lin;        /* periodic linearisation (the Lin parameter of Section 5.4):
                         0 = off (the paper's experiments); k >= 1 = after every k-th
                         hidden layer, each neuron's post polynomials are replaced by
                         affine upper / lower bounds -- the least-squares affine fit of
                         their Bernstein control net at the layer's stored degree plus
                         the largest (upper) or smallest (lower) remainder -- so the
                         next layer starts again at degree 1. The post degrees of
                         the linearised layers must be read off by one block each
                         (BERN_E_TOO_LARGE otherwise)                              */
  int32_t no_raise;   /* BERN_PLAN_LEARNED: 0 = per box and hidden layer, once the
                         predictor has chosen, classes below the layer's top class
                         are raised (to order 2 if some neuron takes order >= 2,
                         fallback to order 1 if the top is order 1); 1 = every
                         neuron keeps the predictor's class                        */
  uint64_t mem_budget_bytes; /* 0 = no limit; else bern_workspace_size, bern_bounds and
                         the calls built on it refuse (BERN_E_TOO_LARGE, the size
                         needed in the message) options whose one-box workspace
                         exceeds this many bytes                                   */
  int64_t *counters;  /* optional device output, BERN_NCOUNTERS int64 values written
                         by the call (see bern_counter), or NULL                   */
} bern_opts;

/* Entries of bern_opts.counters (device, int64), summed over the call's boxes. */
typedef enum {
  BERN_CNT_HIDDEN = 0,   /* hidden neurons bounded                                  */
  BERN_CNT_INACTIVE = 1, /* stable neurons with hi <= 0 (zero polynomial)           */
  BERN_CNT_ACTIVE = 2,   /* stable neurons with lo >= 0 (identity)                  */
  BERN_CNT_FALLBACK = 3, /* unstable neurons on the linear fallback                 */
  BERN_CNT_ORDER1 = 4,   /* unstable neurons with a ReLU approximant of order 1     */
  BERN_CNT_ORDER2 = 5,   /* ... of order 2                                          */
  BERN_CNT_ORDER3UP = 6, /* ... of order 3 or more                                  */
  BERN_CNT_MAXPAD = 7,   /* FP32 mode: the largest rounding radius of an output
                            polynomial (the bits of a non-negative double), 0 in FP64 */
  BERN_NCOUNTERS = 8
} bern_counter;

typedef struct {
  int32_t n_waves;      /* waves the boxes were split into                          */
  int32_t boxes_per_wave;
  int32_t out_degree;   /* largest per-variable degree of an output polynomial      */
  int32_t lin_layers;   /* hidden layers linearised (bern_opts.lin)                 */
  uint64_t workspace_used; /* bytes of the workspace actually used                  */
  double enqueue_ms;    /* host time spent inside the call (the device work it
                           enqueued may still be running when it returns)          */
  int32_t graph;        /* 1: the launches ran as one captured graph (opts.graph) */
  int32_t device_classes; /* 1: a per-neuron plan's degree classes were listed on
                           the device (no host round trip)                         */
  uint64_t reserved[4];
} bern_stats;

/* Fill *opts with defaults: L = 2, FP64, plain plan, per-box schedule. */
void bern_opts_default(bern_opts *opts);

/* Create a network handle (Section 2.1 notation).
 *   H        number of affine layers (H-1 hidden ReLU layers), 1..64
 *   widths   host, H+1 entries: n = h_0 (input dimension, 1..16), h_1, ..., h_H
 *   W        host, all W^(i) (h_i x h_{i-1}, row-major) concatenated, i = 1..H
 *   b        host, all b^(i) (h_i) concatenated
 *   out      receives the handle; free it with bern_net_destroy.
 * The weights are copied to the current HIP device (FP64 and an FP32 copy).
 * Errors: BERN_E_ARG (nulls, bad sizes), BERN_E_NUMERIC (non-finite weights),
 * BERN_E_OOM / BERN_E_DEVICE. */
bern_status bern_net_create(int32_t H, const int32_t *widths, const double *W, const double *b,
                            bern_net **out);
void bern_net_destroy(bern_net *net);

/* Number of network inputs / hidden neurons / outputs of a handle. */
int32_t bern_net_inputs(const bern_net *net);
int32_t bern_net_hidden(const bern_net *net);
int32_t bern_net_outputs(const bern_net *net);

/* Workspace bytes bern_bounds needs to process `n_boxes` boxes in a single
 * wave with these options (the schedule BERN_SCHED_PER_BOX always needs the
 * one-box size). A smaller workspace is accepted by bern_bounds, which then
 * splits the boxes into waves; *one_box receives the smallest usable size.
 * For BERN_PLAN_GIVEN / BERN_PLAN_LEARNED the size covers the largest degree
 * the plan can reach (every unstable neuron at its largest code).
 * Errors: BERN_E_ARG, BERN_E_DEGREE, BERN_E_TOO_LARGE (tensor size overflow). */
bern_status bern_workspace_size(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                                size_t *bytes, size_t *one_box);

/* Bounds of `n_boxes` boxes (Problem 1), enqueued on `stream`. The call is
 * asynchronous (it returns once the work is enqueued) for the plain rule, and
 * for per-neuron plans with opts.graph whose classes the device lists
 * (bern_stats.device_classes). Other per-neuron plan runs synchronise `stream`
 * once per hidden layer and wave (each box's post degree is copied to pinned
 * host memory, the network's own, and the class id lists back), so the call
 * returns only once all but the output layer's work of the last wave is done;
 * two such calls on one network from different threads must be serialised. 
 *   box_lo, box_hi   device, [n_boxes][n] FP64; d_lo <= d_hi required (the
 *                    library checks it on the device; a violation gives NaN
 *                    bounds for that box, never an invalid memory access)
 *   plan             device, [n_boxes][sum of hidden widths] int8 codes for
 *                    BERN_PLAN_GIVEN (1..8 or 0), else NULL
 *   neuron_lo/hi     device, [n_boxes][sum of hidden widths] FP64: the
 *                    pre-activation interval of every hidden neuron, layer by
 *                    layer (Step 1); may be NULL
 *   out_lo/out_hi    device, [n_boxes][h_H] FP64 output bounds
 *   used_plan        device, [n_boxes][sum of hidden widths] int8 or NULL:
 *                    the rule applied per neuron (0 inactive, -1 active,
 *                    -2 linear fallback, k >= 1 ReLU order k)
 *   workspace        device scratch of ws_bytes bytes, 256-byte aligned
 *   stats            host, optional
 * Errors: BERN_E_ARG (also: a per-neuron plan run with host-side classes on
 * a stream under capture), BERN_E_DEGREE, BERN_E_WORKSPACE (too small for
 * one box), BERN_E_TOO_LARGE, BERN_E_DEVICE. */
bern_status bern_bounds(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                        const double *box_lo, const double *box_hi, const int8_t *plan,
                        double *neuron_lo, double *neuron_hi, double *out_lo, double *out_hi,
                        int8_t *used_plan, void *workspace, size_t ws_bytes, void *stream,
                        bern_stats *stats);

/* bern_bounds without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation. It calls no allocating routine (no hipMalloc,
 * hipFree, host pinning, event or graph creation); its scratch is a
 * library-owned device array of BERN_NOALLOC_SCRATCH_BYTES bytes, one per GPU,
 * held until the process ends. Arguments and outputs are bern_bounds' (no
 * degree plan, no workspace); the boxes run in waves that fit the scratch.
 * Limits: the plain rule (BERN_PLAN_PLAIN) or the learned plan
 * (BERN_PLAN_LEARNED, its degree classes listed on the device as under
 * opts.graph; refused when they exceed that path's limits), with or without
 * opts.lin, run eagerly (opts.graph is ignored); the network's index tables
 * for these options must already exist -- one bern_bounds call with the same
 * options on the same network builds them (with opts.graph set, for the
 * learned plan). Results are bit-for-bit those of bern_bounds. Every call on a GPU shares that GPU's array,
 * so calls that overlap in time on one GPU (other streams, other threads)
 * race and must be serialised by the caller; nothing in the array needs to
 * start at zero. Asynchronous on `stream` as bern_bounds.
 * Errors: those of bern_bounds; BERN_E_ARG for given codes, too many degree
 * classes or tables not built yet; BERN_E_TOO_LARGE when one box needs more
 * than the array holds. */
#define BERN_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
bern_status bern_bounds_noalloc(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                                const double *box_lo, const double *box_hi, double *neuron_lo, double *neuron_hi,
                                double *out_lo, double *out_hi, int8_t *used_plan, void *stream,
                                bern_stats *stats);

/* The output polynomials themselves (Problem 1 asks for polynomial bounds;
 * the output intervals follow from them): for every box and output neuron,
 * the upper and lower polynomials U(t) >= f(x(t)) >= L(t) on t in [0,1]^n,
 * x_a = d_lo_a + (d_hi_a - d_lo_a) t_a, as dense power tensors at
 * per-variable degree `degree`:
 *   poly_U, poly_L   device, [n_boxes][h_H][(degree+1)^n] FP64, coefficient
 *                    of t^e at sum_a e_a (degree+1)^(n-1-a); zero where a
 *                    box's own degree is lower. In FP32 mode the stored
 *                    coefficients' radii are folded into the constant
 *                    coefficient (rounded outward), so both stay bounds.
 *   degree           at least every box's output degree (the plain rule:
 *                    L^(H-1); bern_stats.out_degree of a bern_bounds run
 *                    with the same options)
 * The other arguments are bern_bounds' (out_lo/out_hi as there); the hidden
 * layers' outputs are not written. Asynchronous on `stream`; never replayed
 * from a graph.
 * Errors: those of bern_bounds; BERN_E_DEGREE when a box's output degree
 * exceeds `degree`; BERN_E_TOO_LARGE when (degree+1)^n exceeds 2^31. */
bern_status bern_output_polys(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                              const double *box_lo, const double *box_hi, const int8_t *plan, int32_t degree,
                              double *poly_U, double *poly_L, double *out_lo, double *out_hi, void *workspace,
                              size_t ws_bytes, void *stream);

/* Relative volume of the output set (Section 6, evaluation metrics): for
 * every box and output neuron j, the integral over the input box of
 * U_j(x) - L_j(x) divided by the box's volume, i.e. the mean of U_j - L_j
 * over t in [0,1]^n (each power coefficient of t^e weighted by
 * prod_a 1/(e_a+1)).
 *   rel_vol          device, [n_boxes][h_H] FP64, written. In FP32 mode the
 *                    stored coefficients' radii are added: the volume of the
 *                    padded pair, which encloses the network.
 * The other arguments are bern_bounds' (out_lo/out_hi as there); the hidden
 * layers' outputs are not written. Asynchronous on `stream`; never replayed
 * from a graph.
 * Errors: those of bern_bounds; BERN_E_ARG when rel_vol is NULL. */
bern_status bern_rel_volume(const bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                            const double *box_hi, const int8_t *plan, double *rel_vol, double *out_lo,
                            double *out_hi, void *workspace, size_t ws_bytes, void *stream);

/* Branch and bound over input boxes (the batched path's producer of many
 * sub-boxes; not in the paper) for the property "output out_index <= threshold
 * on the box". Each round bounds every pending box with bern_bounds (one
 * batch); a box whose out_hi <= threshold is verified, one whose
 * out_lo > threshold violates the property everywhere, and every other box is
 * bisected along its widest input dimension for the next round, while the
 * pending boxes stay within max_boxes and the rounds within max_rounds
 * (after that they count as undecided). The pending boxes, their bounds,
 * the decisions and the bisection stay in device memory across the rounds;
 * each round reads back its open-box count and volume sums (and the round's
 * boxes when a decision log is given). The halves of open box number q (in
 * box order) are pending boxes 2q and 2q + 1 of the next round. Volume
 * fractions are summed in a fixed order, so a call is reproducible
 * bit for bit. box_lo/box_hi are host arrays [n_boxes][n] with
 * d_lo < d_hi in every dimension; the call is synchronous on the null
 * stream and allocates and frees its own device buffers (two box buffers
 * of max_boxes each and a bern_bounds workspace for max_boxes boxes, or
 * the smallest usable one when that does not fit).
 *   res  host: the verified, violated and undecided fractions of the boxes'
 *        total volume (summing to 1 up to rounding), the rounds run, the
 *        number of box bounds computed, and the boxes left undecided.
 * Errors: those of bern_bounds; BERN_E_ARG for a bad out_index, limits or
 * result pointer; BERN_E_BOX for a box with d_lo >= d_hi. */
typedef struct {
  double verified, violated, undecided;  /* fractions of the total input volume */
  int32_t rounds;
  int32_t reserved0;
  int64_t boxes_bounded;
  int64_t undecided_boxes;
  /* optional decision log (host arrays of the caller, NULL to skip): every
   * decided box, round by round: the round's verified (+1) and violated (-1)
   * boxes in box order, then, in the last round, the boxes left undecided
   * (0) -- with its corners and its output
   * bounds, up to log_cap entries; log_count receives the number written */
  int64_t log_cap;
  int64_t log_count;
  double *log_lo, *log_hi;      /* [log_cap][n] */
  double *log_out_lo, *log_out_hi; /* [log_cap]: bounds of output out_index */
  int8_t *log_status;           /* [log_cap] */
} bern_verify_result;
bern_status bern_verify(const bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                        const double *box_hi, int32_t out_index, double threshold, int32_t max_rounds,
                        int64_t max_boxes, bern_verify_result *res);

/* bern_bounds on host memory, synchronous (the same computation, Problem 1):
 * box_lo, box_hi, plan and every output are host arrays with bern_bounds'
 * shapes (plan, neuron_lo/hi and used_plan nullable as there). The library
 * allocates device copies and a workspace for all boxes in one wave (the
 * one-box size, and waves, if that allocation fails), copies the inputs in,
 * runs on the null stream, copies the outputs back and frees everything
 * before returning; the PCIe copies are part of the call. For callers
 * without device buffers of their own.
 * Errors: those of bern_bounds, and BERN_E_DEVICE for a failed allocation
 * or copy (nothing is left allocated). */
bern_status bern_bounds_host(const bern_net *net, const bern_opts *opts, int64_t n_boxes,
                             const double *box_lo, const double *box_hi, const int8_t *plan,
                             double *neuron_lo, double *neuron_hi, double *out_lo, double *out_hi,
                             int8_t *used_plan, bern_stats *stats);

/* Kernel variants and their autotuner (the box-batch scheduler's tile
 * choices; not in the paper). The library has kTune = bern_tune_params()
 * tuning parameters, parameter q having bern_tune_variants(q) variants
 * (0 = the built-in choice): 0 rows per block and inputs per step of the
 * affine kernel for layers wider than 8 neurons, 1 the same for layers of at
 * most 4 neurons, 2 threads of the dense block-per-neuron read-off, 3 the
 * per-neuron read-off: the tree of folds (0), the dense tensor with one wave
 * per neuron up to 1024 coefficients (1), or one block per neuron (2), the
 * tree with one wave per neuron and more variables folded per round (3);
 * degree-1 tensors always take the closed form. The choice is stored in the
 * network handle and used by every
 * later call on it; every variant computes the same bounds up to the order
 * of floating-point sums.
 *   bern_tune_get / bern_tune_set -- read / write `choice` (host,
 *     [bern_tune_params()] ints); set rejects out-of-range variants.
 *   bern_autotune -- takes the arguments of bern_bounds plus `reps`; for
 *     each parameter in turn it times reps runs of bern_bounds under every
 *     variant (the others at their current choice) and keeps the fastest.
 *     Synchronous: it waits for `stream`. On return `choice` (host, nullable)
 *     holds the chosen variants and `best_ms` (host, nullable) the mean time
 *     of one run under them; the outputs hold the last run's results. Not
 *     thread-safe with other calls on the same network. */
int32_t bern_tune_params(void);
int32_t bern_tune_variants(int32_t param);
bern_status bern_tune_get(const bern_net *net, int32_t *choice);
bern_status bern_tune_set(bern_net *net, const int32_t *choice);
bern_status bern_autotune(bern_net *net, const bern_opts *opts, int64_t n_boxes, const double *box_lo,
                          const double *box_hi, const int8_t *plan, double *neuron_lo, double *neuron_hi,
                          double *out_lo, double *out_hi, int8_t *used_plan, void *workspace,
                          size_t ws_bytes, void *stream, int32_t reps, int32_t *choice, float *best_ms);

/* Step-level entry points. Each runs one kernel of the hot path on
 * caller-provided device buffers, asynchronously on `stream`; the tests use
 * them to check every kernel on its own against the oracle.
 *
 * bern_basis_minmax -- power-to-Bernstein basis change at degree D
 * (Def. 1 coefficients, textbook per-variable identity t^j =
 * sum_{k>=j} C(k,j)/C(D,j) Ber_{k,D}) and the range enclosure of Def. 2:
 *   coef     device, [count][(D+1)^n] power coefficients (FP64 if fp64 != 0,
 *            else FP32)
 *   bern     device, [count][(D+1)^n] FP64 Bernstein coefficients out, or NULL
 *   mn, mx   device, [count] FP64: smallest / largest Bernstein coefficient
 *   l1       device, [count] FP64: sum of |power coefficients|, or NULL
 *   scratch  device, >= bern_basis_minmax_scratch(n, D, count) bytes */
size_t bern_basis_minmax_scratch(int32_t n, int32_t D, int64_t count);
bern_status bern_basis_minmax(int32_t n, int32_t D, int64_t count, const void *coef, int32_t fp64,
                              double *bern, double *mn, double *mx, double *l1, void *scratch,
                              size_t scratch_bytes, void *stream);

/* bern_poly_mul -- the product "Prod" of Section 4.2 on power-basis tensors:
 * out_K = sum_{I+J=K} A_I B_J for `count` independent pairs,
 *   A  device [count][(da+1)^n], B device [count][(db+1)^n],
 *   out device [count][(da+db+1)^n]; all FP64 (fp64 != 0) or all FP32.
 * A and B may be the same pointer (a square). */
bern_status bern_poly_mul(int32_t n, int32_t da, int32_t db, int64_t count, const void *A,
                          const void *B, void *out, int32_t fp64, void *stream);

/* bern_relu_poly -- Step 2 for `count` neurons: from [lo, hi] and order L,
 * the power coefficients c[0..L] in u = (y-lo)/(hi-lo) of the Bernstein
 * over-approximant of ReLU (Def. 1, Prop. 1) and its value e at y = 0
 * (Prop. 2). Device arrays: lo, hi [count]; c [count][L+1]; e [count]. */
bern_status bern_relu_poly(int64_t count, int32_t L, const double *lo, const double *hi, double *c,
                           double *e, void *stream);

/* Kernel timing for measurement. While enabled, every kernel the library
 * launches is bracketed by two HIP events recorded on the stream it runs on
 * (process-wide setting; not for use while a stream is being captured).
 * bern_prof_read waits for the recorded events and returns, for one kernel
 * class (0 .. bern_prof_classes()-1, named by bern_prof_name), the number of
 * launches, their summed duration in milliseconds, their summed algorithmic
 * HBM bytes and their summed algorithmic floating-point operations, where the
 * launch shape alone fixes them (else 0; `flops` may be NULL). Algorithmic
 * counts are those of the method on its stored tensors: the basis change
 * counts n (D+1)^n (D+2) flops per tensor (all per-axis triangular sums of
 * the dense degree-D tensor), the affine map 4 h h_in C per box (every
 * input, upper and lower). bern_prof_reset forgets every record. */
bern_status bern_prof_enable(int32_t on);
bern_status bern_prof_reset(void);
int32_t bern_prof_classes(void);
const char *bern_prof_name(int32_t cls);
bern_status bern_prof_read(int32_t cls, int64_t *launches, double *ms, double *bytes, double *flops);

/* Degree predictor (learned plan). A small MLP 8 -> 64 -> 64 -> 4 with ReLU
 * hidden layers maps the features of an unstable neuron to a class: 0 =
 * linear fallback, k = 1..3 = Bernstein ReLU approximant of order k. Any class
 * gives sound bounds (Props. 1-2 for every order, Def. 2 for the fallback),
 * so the predictor only trades tightness for work.
 * Parameters (FP32, bern_pred_params() = 5012 values, in this order):
 *   mean[8], std[8] (feature normalisation), W1[64][8], b1[64], W2[64][64],
 *   b2[64], W3[4][64], b3[4]  (row-major, output index first).
 * Features of a neuron with interval [lo, hi], w = hi - lo, pre degree D in
 * layer i of an H-layer net, downstream sensitivity s (sum over the network's
 * outputs of the products of |W| from this neuron on), affine least-squares
 * fits of its Bernstein control nets (means m_U, m_L, slopes g_U) and their
 * remainder spreads r_U, r_L:
 *   -lo/w, log w, i/(H-1), log(D+1), (m_U - m_L)/w, log(s w), (r_U + r_L)/w,
 *   sum|g_U|/w.
 * Inference inside bern_bounds rounds weights and activations to BF16. */
int32_t bern_pred_params(void);
/* params: host, bern_pred_params() floats; copied to the current device. */
bern_status bern_pred_create(const float *params, int64_t n_params, bern_pred **out);
void bern_pred_destroy(bern_pred *pred);

/* Predictor files and training.
 * bern_pred_load -- a predictor from a file written by bern_pred_train
 *   ("BERNPRED", uint32 version 1, uint32 bern_pred_params(), that many
 *   float32 parameters, uint32 length and bytes of a metadata text; little-
 *   endian). Errors: BERN_E_ARG (missing, foreign or truncated file), those
 *   of bern_pred_create.
 * bern_pred_train -- fit the MLP to N records, synchronously on the current
 *   device with the training kernels below: X host [N][8] features (as
 *   bern_opts.features exports them), y host [N] classes 0..3. The feature
 *   normalisation is the records' mean and standard deviation (+1e-3); the
 *   weights start from a seeded He initialisation (SplitMix64 stream,
 *   Box-Muller normals); each epoch shuffles the records (seeded) and takes
 *   N / batch minibatch Adam steps on the mean softmax cross-entropy, with the
 *   learning rate lr (1 + cos(pi epoch / epochs)) / 2. `path` (nullable)
 *   receives the file, with `meta` (nullable) as its metadata text; `out`
 *   (nullable) a predictor with the trained parameters; opts->loss_out (host,
 *   nullable, [epochs]) each epoch's mean minibatch loss. The library
 *   allocates its device buffers and frees them before returning.
 *   Errors: BERN_E_ARG (bad sizes, labels outside 0..3, an unwritable path),
 *   BERN_E_NUMERIC (a non-finite feature), BERN_E_DEVICE. */
typedef struct {
  int32_t epochs;   /* passes over the records (default 40)                     */
  int32_t batch;    /* records per Adam step (default 8192; at most N)          */
  float lr;         /* peak learning rate (default 3e-3)                        */
  float beta1, beta2, eps;  /* Adam (defaults 0.9, 0.999, 1e-8)                 */
  uint64_t seed;    /* initialisation and shuffling stream (default 0)          */
  float *loss_out;  /* host, optional, [epochs]                                 */
  int32_t reserved[4];
} bern_train_opts;
void bern_train_opts_default(bern_train_opts *opts);
bern_status bern_pred_load(const char *path, bern_pred **out);
bern_status bern_pred_train(const float *X, const int8_t *y, int64_t N, const bern_train_opts *opts,
                            const char *path, const char *meta, bern_pred **out);

/* Training and evaluation kernels of the predictor (FP32, deterministic),
 * asynchronous on `stream`, all pointers device pointers:
 *   bern_mlp_forward   logits [N][4] of features X [N][8] (bf16 != 0: the
 *                      BF16 inference arithmetic of the pipeline)
 *   bern_mlp_backward  mean softmax cross-entropy over labels y [N] (0..3):
 *                      gradient G [5012] (zero on the normalisation entries)
 *                      and the loss in loss[0]; scratch of
 *                      bern_mlp_backward_scratch(N) bytes
 *   bern_mlp_adam      one Adam step (bias-corrected, step >= 1) of P with G,
 *                      moments m, v [5012] (normalisation entries untouched)
 *   bern_mlp_classify  argmax classes [N] (int8) and logits [N][4] */
size_t bern_mlp_backward_scratch(int64_t N);
bern_status bern_mlp_forward(const float *P, int64_t N, const float *X, float *logits, int32_t bf16,
                             void *stream);
bern_status bern_mlp_backward(const float *P, int64_t N, const float *X, const int8_t *y, float *G,
                              float *loss, void *scratch, void *stream);
bern_status bern_mlp_adam(float *P, const float *G, float *m, float *v, int64_t step, float lr,
                          float beta1, float beta2, float eps, void *stream);
bern_status bern_mlp_classify(const float *P, int64_t N, const float *X, float *logits, int8_t *cls,
                              int32_t bf16, void *stream);

/* Status name and the calling thread's last error message. */
const char *bern_status_str(int32_t status);
const char *bern_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BERNNN_H */
