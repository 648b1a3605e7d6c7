/*
 * qtn.h - C ABI of libqtn: sliced tensor-network contraction of QAOA
 * single amplitudes on one MI355X (gfx950).
 *
 * Method (Zhao et al., "Simulation of Quantum Computing on Classical
 * Supercomputers"): the circuit becomes an undirected-graph tensor network
 * (Sec. II A, Fig. 1); a set of index variables is cut, i.e. fixed to each of
 * its values, which yields identical-structure sub-networks whose contraction
 * results sum to the uncut result (Sec. III A, Eq. (2), Fig. 3); each
 * sub-network ("slice") is contracted by pairwise contractions (Eq. (1)) along
 * an elimination order of small width (Sec. II B); the cut set is searched
 * with the genetic algorithm of Sec. III B (Algorithm 1).
 *
 * Index variables here are binary: the ZZ phases are diagonal, so qubit i
 * keeps one variable v(i,l) = l*n + i through the ZZ gates of layer l.  A
 * density-matrix edge of the paper (four values) corresponds to two binary
 * variables.  Circuit: H^n on |0^n>, then for l = 0..p-1 exp(-i gamma_l Z_i Z_j)
 * on every edge and RX(2 beta_l) = exp(-i beta_l X) on every qubit; result
 * <x|U|0^n> for bitstring x (byte i = qubit i).
 *
 * Conventions for every entry point:
 *   - return 0 (QTN_OK) or a negative QTN_E* code; no exception crosses the
 *     ABI; qtn_last_error() gives a thread-local message for the last failure;
 *   - all validation happens before any device work;
 *   - host pointers are only read during the call (the plan copies them);
 *   - device memory for bulk intermediates belongs to the caller and is
 *     bound with qtn_plan_bind_workspace; the library allocates only small
 *     constant buffers (leaf factors, step descriptors, index tables).
 */
#ifndef QTN_H
#define QTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  QTN_OK = 0,
  QTN_EINVAL = -1, /* malformed graph/angles/bitstrings/options           */
  QTN_ERANGE = -2, /* slice range outside [0, 2^k) or lo > hi            */
  QTN_ERANK = -3,  /* no cut set of size <= k_max meets max_rank          */
  QTN_ENOMEM = -4, /* workspace missing or too small; host allocation     */
  QTN_EHIP = -5,   /* HIP runtime error (message names the call)         */
  QTN_ESTATE = -6, /* call not valid in the plan's current state         */
  QTN_ETIMEOUT = -7 /* qtn_contract's wait exceeded QTN_SYNC_TIMEOUT_S      */
};

/*
 * Precision forms.  QTN_FP64: every tensor complex128, FP64 arithmetic, no
 * rescaling.  QTN_FP32 (mixed): the large slice tensors, which carry the HBM
 * traffic, are stored in eight bytes per element, as many as complex64: one
 * 8-bit exponent shared by the real and imaginary parts and two 28-bit
 * two's-complement mantissas (absolute error at most 2^-28 |z| per part,
 * against 2^-24 of each part for complex64), with a per-instance power-of-two
 * exponent (rescaled after every grid-wide step, or not at all in
 * synchronous calls whose values stay in range: qtn_plan_range_state); small
 * tensors (under 3% of the bytes), LDS-resident program tensors and the gate
 * factors stay complex128; all products and sums run in FP64 registers.  The
 * slice sum is always FP64.
 */
enum { QTN_FP64 = 0, QTN_FP32 = 1, QTN_3XBF16 = 2 };

typedef struct qtn_plan_s qtn_plan_t; /* opaque, owned by the library */
typedef struct qtn_mlp_s qtn_mlp_t;   /* learned cut-set cost model (below) */

/* Compensated FP64 sum of slice results: value = (re + re_comp, im + im_comp). */
typedef struct {
  double re, im, re_comp, im_comp;
} qtn_partial;

/* Simple undirected graph: m edges as 2*m vertex ids in [0, n). */
typedef struct {
  uint32_t n;
  uint32_t m;
  const uint32_t *edges;
} qtn_graph;

typedef struct {
  int32_t k;                 /* cut size; -1: smallest k whose searched cut meets max_rank */
  int32_t max_rank;          /* cap on the rank of any slice tensor; 0 = no cap           */
  int32_t k_max;             /* largest k tried when k = -1                               */
  const uint32_t *cut_vars;  /* k explicit cut variable ids, or NULL to search            */
  uint64_t seed;             /* seed of the search's SplitMix64 stream                    */
  int32_t ga_pop;            /* N of Algorithm 1 (default 11)                              */
  int32_t ga_iters;          /* T of Algorithm 1 (default 4)                               */
  int32_t precision;         /* QTN_FP64, QTN_FP32 or QTN_3XBF16                           */
  int32_t fuse_chains;       /* 1: sum chains of trivial buckets in one step (default 1)   */
  int32_t exec_mode;         /* -1 auto (= 0), 0 grid-wide steps, 1 one workgroup per instance */
  int32_t use_cost_model;    /* 1: the cut search ranks its offspring with cost_model and     */
                             /*    scores only the best N-1 exactly (see qtn_cut_search)       */
  int32_t offspring_factor;  /* offspring per kept individual with use_cost_model (16)      */
  qtn_mlp_t *cost_model;     /* trained model (qtn_mlp_create, QTN_COST_FEATURES inputs)     */
  int32_t density_matrix;    /* 1: the density-matrix network of Sec. II A (Markov-Shi
                                tensors over 4-valued edges, each edge the pair of a ket
                                variable v and its bra copy v + n p); the result is
                                |amplitude|^2 (real part of the partials); k and
                                cut_vars count 4-valued edges (ket ids), each cut gives
                                4 slices, so 4^k in all; qtn_plan_cut lists the 2 k
                                binary variables, ket ids first                          */
} qtn_plan_opts;

typedef struct {
  uint32_t n, p, n_vars, n_bitstrings;
  int32_t k;                 /* number of cut variables */
  int32_t width;             /* largest rank of a slice tensor the schedule materialises  */
  int32_t n_steps;           /* contraction steps per slice                               */
  int32_t n_tensors;
  double log2_flops;         /* real flops per slice-contraction (all bitstrings), the
                                slice-invariant steps' share amortised over the 2^k slices */
  double bytes_per_slice;    /* algorithmic HBM bytes per slice (all bitstrings), same   */
  double flops_hoisted;      /* flops of the slice-invariant steps; qtn_contract runs them
                                once per wave of slices, so a range of w waves executes
                                w * flops_hoisted beyond the per-slice work              */
  double work;               /* sum over buckets of 2^(|N+(v)|+1), one slice, one bitstring */
  double prefactor;          /* 2^{-n/2} times the factor normalisations                 */
  double search_seconds;     /* time spent in the cut search                              */
  int32_t precision;
  int32_t f64_below_rank;    /* intermediates of smaller rank are stored as complex128    */
  int32_t n_programs_wide;   /* workgroup programs (trees of small steps), grid-wide mode */
  int32_t n_launches_wide;   /* kernel launches per wave, grid-wide mode                  */
  uint32_t slice_lds_bytes;  /* LDS per workgroup, one-workgroup-per-instance mode        */
  double slice_scratch_bytes;/* global scratch per workgroup, same mode                   */
  int32_t mf_width;          /* width of the min-fill order on G - C, Sec. II B (largest bag
                                minus one; the cut search's fitness); width <= mf_width + 1 */
  int32_t rescaled;          /* bit 0 (grid-wide mode), bit 1 (one-workgroup-per-instance
                                mode): the mixed form keeps some intermediate in the 64-bit
                                form outside LDS and runs the rescaling kernels; when clear,
                                every stored tensor is complex128 and the FP64 kernels run
                                (always for FP64 plans)                                   */
} qtn_plan_info;

/* Fills defaults: k = -1, max_rank = 0, k_max = 24, cut_vars = NULL, seed = 0,
 * ga_pop = 11, ga_iters = 4 (Sec. IV A), precision = QTN_FP64, fuse_chains = 1,
 * exec_mode = -1, use_cost_model = 0, offspring_factor = 16, cost_model = NULL,
 * density_matrix = 0. */
void qtn_plan_opts_default(qtn_plan_opts *opts);

/*
 * Build a host-side plan.  Sec. II A (network), Sec. II B (elimination order),
 * Sec. III A (cut and slice), Sec. III B (cut search, Algorithm 1).  No device
 * call is made, except that with use_cost_model the model ranks candidates on
 * the current device (the model's own buffers; nothing else is allocated).
 *   graph        simple undirected graph (no self-loops or repeated edges)
 *   p            QAOA depth, >= 1
 *   gamma, beta  p angles each, finite
 *   bitstrings   n_bitstrings * n bytes, each 0 or 1, row-major
 *   opts         NULL for defaults
 *   out          receives the plan; free with qtn_plan_destroy
 * Cut variables are sorted ascending; slice s fixes cut[b] to bit b of s.
 */
int qtn_plan(const qtn_graph *graph, uint32_t p, const double *gamma,
             const double *beta, const uint8_t *bitstrings,
             uint32_t n_bitstrings, const qtn_plan_opts *opts,
             qtn_plan_t **out);

/*
 * General circuits (gates that are not diagonal, as in the random circuits of
 * Sec. IV B): a plan for the amplitudes <x|U_m ... U_1|0^n> of n_bitstrings
 * bitstrings.  Each gate acts on 1 or 2 qubits with matrix[out][in]
 * (row-major re/im, 2x2 or 4x4; for two qubits q[0] is the more significant
 * bit of both indices).  The network (Sec. II A, Fig. 1) has one binary
 * variable per wire segment: a diagonal gate keeps its wires' variables (its
 * factor holds the diagonal), any other gate starts new ones; inputs are |0>
 * and the final variables carry the measured bits.  Cut search, order,
 * schedule and contraction are those of qtn_plan (k counts wire variables,
 * slice s fixes cut[b] to bit b of s); density_matrix and use_cost_model are
 * not available here (QTN_EINVAL).  qtn_plan_info.p is 0.
 */
typedef struct {
  uint32_t nq;        /* 1 or 2                                          */
  uint32_t q[2];      /* qubits, distinct, < n                           */
  double re[16];      /* matrix entries, row-major, first 4 or 16 used   */
  double im[16];
} qtn_gate;
int qtn_plan_circuit(uint32_t n, const qtn_gate *gates, uint32_t n_gates, const uint8_t *bitstrings,
                     uint32_t n_bitstrings, const qtn_plan_opts *opts, qtn_plan_t **out);

/* Frees the plan and the constant device buffers it uploaded (leaf factors,
 * program descriptors, pinned partials); the bound workspace stays the
 * caller's.  NULL is ignored. */
void qtn_plan_destroy(qtn_plan_t *plan);

/* Plan summary: cut size k, width (Sec. II B: largest bag minus one = largest
 * slice tensor rank), algorithmic flops and bytes per slice of the schedule
 * (Eq. (1) steps), and the execution structure.  Host only. */
int qtn_plan_query(const qtn_plan_t *plan, qtn_plan_info *info);

/* Copies the k cut variable ids (ascending) into cut[0..k): the index
 * variables fixed per slice (Sec. III A, Fig. 3).  QTN_EINVAL if capacity < k. */
int qtn_plan_cut(const qtn_plan_t *plan, uint32_t *cut, uint32_t capacity);

/* Copies the elimination order of the free variables (n_vars - k ids), the
 * min-fill order on G - C that fixes the contraction order (Sec. II B). */
int qtn_plan_order(const qtn_plan_t *plan, uint32_t *order, uint32_t capacity);

/*
 * Exports the contraction schedule for inspection: the chain of contractions
 * of Eq. (1), C[out] = sum over kappa of the product of the inputs, one per
 * bucket of the elimination order (Sec. II B), shared by every slice
 * (Sec. III A: the sub-networks have identical structure).  For step t:
 *   rec[0] = output tensor id, rec[1] = number of inputs, rec[2] = |kappa|,
 *   rec[3] = output rank, rec[4] = class (0 E, 1 G), rec[5..5+8) = input ids
 *   (-1 unused), rec[13..13+8) = input bit masks over the step index
 *   (kappa bits above the output bits), rec[21] = flags (1 bitstring-dependent,
 *   2 slice-dependent).
 * Tensor t: trec[0] = rank, trec[1] = kind (0 leaf, 1 intermediate),
 *   trec[2] = flags (1 bitstring-dependent, 2 slice-dependent, 4 stored as
 *   complex128), trec[3] = slice-bit mask selecting leaf variants,
 *   trec[4..4+rank) = variables, most significant bit first.
 * Records are QTN_STEP_REC and QTN_TENSOR_REC int32 wide.
 */
#define QTN_STEP_REC 24
#define QTN_TENSOR_REC 40
int qtn_plan_export(const qtn_plan_t *plan, int32_t *steps, uint32_t step_cap,
                    int32_t *tensors, uint32_t tensor_cap);

/* Summed variables of step `step` (most significant first) into kappa[0..nk):
 * the index j of Eq. (1) (several at once in a fused step). */
int qtn_plan_kappa(const qtn_plan_t *plan, int32_t step, int32_t *kappa, uint32_t capacity);

/*
 * Integer index tables of input `input` of step `step` (the index maps of the
 * Eq. (1) contraction, in the form the device derives them in):  table[0..256) = pext(c & 255, cmask & 255), table[256..272) =
 * pext(u << 8, cmask) for u < 16, table[272] = cmask >> 12, table[273] =
 * popcount(cmask & 4095), table[274..274+2^nk) = pext(kappa, kmask) <<
 * popcount(cmask), where cmask / kmask are the input's mask bits over the
 * output / summed part of the step index.  `count` receives the length; with
 * table == NULL only the length is returned.
 */
int qtn_plan_index_table(const qtn_plan_t *plan, int32_t step, int32_t input,
                         uint32_t *table, uint32_t capacity, uint32_t *count);

/* Leaf values (FP64) of tensor `tensor`: [bitstring or 1][variant][2^rank]
 * complex, interleaved re/im; `count` receives the number of complex values.
 * The gate tensors of Sec. II A (Fig. 1), merged per bucket; a variant is one
 * assignment of the cut variables it holds (the restricted tensors of Fig. 3). */
int qtn_plan_leaf_values(const qtn_plan_t *plan, int32_t tensor, double *values,
                         uint64_t capacity, uint64_t *count);

/*
 * Device workspace needed to contract `slices_per_wave` slices of every
 * bitstring at once (intermediates with liveness reuse, scale exponents,
 * per-slice results).  Pure host computation.  The slices of one wave are
 * the identical-structure sub-networks of Sec. III A processed together, the
 * paper's rounds of subgraphs per core count; slices_per_wave is clamped to
 * [1, 2^k].  QTN_EINVAL for 0 or above 2^24.
 */
int qtn_plan_workspace_bytes(const qtn_plan_t *plan, uint64_t slices_per_wave,
                             uint64_t *bytes);

/*
 * Binds caller-owned device memory (e.g. a torch tensor) of `bytes` bytes,
 * 256-byte aligned, to the plan, with `slices_per_wave` slices per wave, and
 * uploads the plan's constants (gate tensors of Sec. II A, step descriptors
 * of the Eq. (1) schedule) to the current device.  The memory must stay valid
 * until the plan is destroyed or rebound.  QTN_ENOMEM if `bytes` is below
 * qtn_plan_workspace_bytes, QTN_EINVAL for misalignment.
 */
int qtn_plan_bind_workspace(qtn_plan_t *plan, void *device_ptr, uint64_t bytes,
                            uint64_t slices_per_wave);

/*
 * Contracts slices [slice_lo, slice_hi) of every bitstring on `stream`
 * (a hipStream_t; NULL = default stream) and writes one compensated partial
 * sum per bitstring to out[0..n_bitstrings).  Eq. (2): summing the partials of
 * disjoint ranges that cover [0, 2^k) gives the amplitude.  The call waits for
 * the stream before returning.  lo == hi gives exact zeros.  With the
 * environment variable QTN_SYNC_TIMEOUT_S set to a positive number of seconds
 * (read once per process), that wait gives up after so long with QTN_ETIMEOUT
 * and leaves the work in flight; by default it waits without limit.
 */
int qtn_contract(qtn_plan_t *plan, uint64_t slice_lo, uint64_t slice_hi,
                 void *stream, qtn_partial *out);

/*
 * As qtn_contract, but returns once the work is enqueued: the contraction and
 * a copy of the partials to `out` are ordered on `stream`, and `out` is valid
 * after the caller synchronises the stream.  Pinned host memory for `out`
 * keeps the copy asynchronous.  Calls on one plan share its workspace: issue
 * them on one stream (they then run one after another) or synchronise in
 * between.  lo == hi writes exact zeros to `out` at once.  Not with timing on
 * (QTN_ESTATE).  For serving loops that pipeline many contractions.
 */
int qtn_contract_async(qtn_plan_t *plan, uint64_t slice_lo, uint64_t slice_hi, void *stream,
                       qtn_partial *out);

/*
 * Enables (1, the default after binding) or disables (0) replay of captured
 * HIP graphs.  With graphs, the launch sequence of a slice range is captured
 * on the first qtn_contract for that range (on a library stream, so nothing
 * runs during capture) and replayed on `stream` by that and later calls with
 * the same range; the sequence contains no memset nodes.  With graphs off,
 * kernels are launched on `stream` directly, one after another in
 * the plan's enqueue order.  Inside a captured graph, independent launches
 * sit on parallel branches (captured from library side streams joined back
 * before the capture ends).  Requires a bound workspace.
 */
int qtn_plan_set_graphs(qtn_plan_t *plan, int enable);

/*
 * Autotuner of the launch configuration: for every grid-wide streaming step
 * of the bound plan it times (HIP events on `stream`, 5 launches each) the
 * block count over the chip (256, 512, 1024, 2048, 4096) and, where the
 * LDS-staged kernel applies, that kernel against the direct one and (for
 * steps that allow it) the row-paired staged one, and takes the fastest.  Steps run alone there but share launches in a contraction,
 * so, starting from the defaults, each step's choice (largest gain first)
 * is kept for later contractions only if a whole contraction of the first
 * wave (5 direct-launch runs) is then at least 1% faster.  Last, the
 * launch mode (qtn_plan_set_graphs) is set to whichever of graph replay and
 * direct launches runs a synchronous qtn_contract of the first wave faster
 * (10 calls each); a later qtn_plan_set_graphs overrides it.
 * cache_path (or NULL): a text file of known choices,
 * one line per step signature ("<hex signature> <blocks> <variant> <us>"); steps
 * found there are not measured, new choices are appended.  Runs one
 * contraction of the first wave first (its results are discarded) and leaves
 * the workspace ready for the next call; drops the captured graph.  Not while
 * timing is on (QTN_ESTATE).  The choices change the block partition only,
 * not the arithmetic of any output element; a step that folds the closing
 * chain groups its partial sums by block, so the amplitude may change in its
 * last bits.
 */
typedef struct {
  uint32_t steps;      /* streaming steps of the plan                      */
  uint32_t measured;   /* configurations timed                             */
  uint32_t cached;     /* steps whose choice came from the cache           */
  double default_us;   /* summed time of the measured steps, default config */
  double tuned_us;     /* the same steps with the chosen configuration     */
  double whole_default_us; /* one contraction of the first wave, defaults   */
  double whole_tuned_us;   /* the same with the choices kept                */
  uint32_t kept;       /* steps whose measured choice is kept               */
  double graph_us;     /* synchronous contraction of the first wave, graph  */
  double direct_us;    /* the same, kernels launched directly               */
  uint32_t graphs;     /* the launch mode kept: 1 graph replay, 0 direct    */
} qtn_tune_stats;
int qtn_plan_autotune(qtn_plan_t *plan, void *stream, const char *cache_path, qtn_tune_stats *stats);

/* Accumulated timing of the streaming step kernels (grid-wide steps whose
 * output holds at least 2^8 elements per instance: step_stream and
 * step_tiled), measured with HIP events recorded on the launch's stream
 * around each launch.  While timing is on, every launch runs on the caller's
 * stream in schedule order, so that the events bracket one kernel each. */
typedef struct {
  uint64_t launches;
  double total_ms;   /* summed launch durations                              */
  double alg_bytes;  /* algorithmic bytes: every input read once, output once */
  double alg_flops;  /* real flops: per step index point, 6 per complex product
                        of the varying operands and the kappa coefficient,
                        plus 2 for the accumulation                          */
  uint64_t dropped;  /* launches whose event pair could not be read           */
  int32_t last_error;/* HIP error of the last unreadable pair (0 if none)     */
} qtn_kernel_timing;

/* Enables (1) or disables (0) the timing above and resets its counters.
 * Requires a bound workspace. */
int qtn_plan_set_timing(qtn_plan_t *plan, int enable);

/* Reads the counters accumulated by qtn_contract calls since the last reset. */
int qtn_plan_timing(const qtn_plan_t *plan, qtn_kernel_timing *out);

/* The same counters restricted to schedule step `step` (zero if the step
 * was not timed).  step = -1 gives the launches of workgroup programs
 * (trees of small steps, one workgroup per instance), timed the same way and
 * not part of the totals above; their algorithmic bytes are the gate factors,
 * workspace and scratch tensors each item reads or writes outside LDS, once
 * each, and their flops those of every step in the program. */
int qtn_plan_step_timing(const qtn_plan_t *plan, int32_t step, qtn_kernel_timing *out);

/* Name of the kernel instance that runs grid-wide step `step` under the
 * bound workspace, e.g. "step_tiled<true, 4, 3, 3>" (rescaled, 4 summed
 * variables, 3 varying operands of which 3 complex64); "" for steps run
 * inside workgroup programs.  NUL-terminated, truncated to `capacity`. */
int qtn_plan_step_kernel(const qtn_plan_t *plan, int32_t step, char *name, uint32_t capacity);

/* Launch configuration in use for grid-wide step `step` (qtn_plan_autotune's
 * kept choice, else the default): *blocks = the block count over the chip it
 * targets (1024 by default); *variant = 0 for the default kernel, 1 when the
 * direct kernel runs a step that could stage its operands in LDS, 2 for the
 * row-paired staged kernel (each thread sums two rows that share the staged
 * runs of operand 0).  Host-side; no device work. */
int qtn_plan_step_tune(const qtn_plan_t *plan, int32_t step, uint32_t *blocks, int32_t *variant);

/* Rescaling of the mixed form (QTN_FP32, above; not part of the paper's
 * method, which does not fix a precision).  For callers that want to know
 * which kernels ran; no caller has to act on it.  A plan that
 * stores tensors in the 64-bit form runs synchronous qtn_contract calls
 * without per-instance rescaling while the values stay inside the form's
 * exponent range: every encoder that would flush a non-zero value below
 * 2^-127 or clamp one at 2^128 sets a word of the plan's workspace, the
 * call's last kernel hands it to the host, and a call that set it is
 * repeated with rescaling
 * (the returned partials are those of the rescaled run).  After two such
 * calls in a row, or with QTN_RESCALE=1 in the environment at bind time,
 * every call rescales.  Asynchronous calls, qtn_contract_noalloc and
 * qtn_batch_contract always rescale.  *unscaled = 1 while synchronous calls
 * run without the rescaling kernels (always for plans that store nothing in
 * the 64-bit form); *reruns = calls repeated so far.  Errors:
 * QTN_ESTATE (no workspace). */
int qtn_plan_range_state(const qtn_plan_t *plan, int32_t *unscaled, uint64_t *reruns);

/* Sets the launch configuration of grid-wide step `step` by hand (the same
 * fields qtn_plan_autotune chooses; a later autotune overrides them):
 * `blocks` in [1, 2^20] targeted over the chip, `variant` 0 default kernel,
 * 1 direct kernel, 2 row-paired staged kernel.  A variant the step does not
 * allow runs the default kernel; the arithmetic of every output element is
 * unchanged (a step with the folded closing chain groups its partials by
 * block).  Drops the captured graph.  Errors: QTN_ESTATE (no workspace),
 * QTN_ERANGE (step), QTN_EINVAL (blocks or variant). */
int qtn_plan_set_step_tune(qtn_plan_t *plan, int32_t step, uint32_t blocks, int32_t variant);

/* ---------------------------------------------------------------------------
 * Learned cut-set cost model.  Not part of the paper: it ranks candidate cut
 * sets for the search of Sec. III B by predicted log2 cost and peak rank;
 * every returned cut set is scored by the exact evaluator.
 * ------------------------------------------------------------------------- */
#define QTN_COST_FEATURES 32

/* Features of n_sets candidate cut sets of size k (row-major n_sets x k
 * variable ids) into features[n_sets x QTN_COST_FEATURES]: mean, max, min
 * and sum over the set of six per-variable statistics of the uncut min-fill
 * elimination (degree, position, bag size, fill-in, bags holding it, layer),
 * then n, p, k, uncut width, uncut log2 work, and three set statistics. */
int qtn_cost_features(const qtn_graph *graph, uint32_t p, const uint32_t *cut_sets,
                      uint32_t n_sets, uint32_t k, float *features);

/* Exact cost of each cut set (labels and fallback): width of the min-fill
 * order on G - C (= largest slice tensor rank) and log2(work * 2^k) with
 * work = sum over eliminated variables of 2^(|N+(v)|+1).  threads >= 1. */
int qtn_cost_exact(const qtn_graph *graph, uint32_t p, const uint32_t *cut_sets,
                   uint32_t n_sets, uint32_t k, int32_t *width, double *log2_cost,
                   int32_t threads);

/* Multilayer perceptron in_dim -> hidden (x n_hidden, ReLU) -> out_dim on the
 * current device, FP32, He-initialised from `seed`.  Dense layers run on FP32
 * matrix cores.  The library owns its parameters and activations (sized for
 * max_batch rows). */
int qtn_mlp_create(uint32_t in_dim, uint32_t hidden, uint32_t n_hidden, uint32_t out_dim,
                   uint32_t max_batch, uint64_t seed, qtn_mlp_t **out);
void qtn_mlp_destroy(qtn_mlp_t *mlp);

/* Parameter vector: for each layer, W [fan_in x fan_out] row-major then b. */
int qtn_mlp_num_params(const qtn_mlp_t *mlp, uint64_t *count);
int qtn_mlp_get_params(const qtn_mlp_t *mlp, float *host, uint64_t capacity);
int qtn_mlp_set_params(qtn_mlp_t *mlp, const float *host, uint64_t count);
/* Gradients of the last qtn_mlp_train_step, same layout as the parameters. */
int qtn_mlp_get_grads(const qtn_mlp_t *mlp, float *host, uint64_t capacity);

/* Feature and label standardisation used by the guided search. */
int qtn_mlp_set_normalization(qtn_mlp_t *mlp, const float *x_mean, const float *x_std,
                              const float *y_mean, const float *y_std);

/* y_dev[batch x out_dim] = MLP(x_dev[batch x in_dim]) on `stream` (device pointers). */
int qtn_mlp_forward(qtn_mlp_t *mlp, const float *x_dev, uint32_t batch, float *y_dev,
                    void *stream);

/* One step of mean-squared-error training with Adam (lr = 0: gradients only).
 * loss (host, may be NULL) receives the batch loss; the call then waits. */
int qtn_mlp_train_step(qtn_mlp_t *mlp, const float *x_dev, const float *t_dev, uint32_t batch,
                       float lr, void *stream, float *loss);

typedef struct {
  double seconds;        /* wall time, model inference included */
  uint64_t exact_evals;  /* distinct cut sets scored exactly    */
  uint64_t model_evals;  /* candidates ranked by the model      */
  int32_t width;         /* exact width of the returned cut set */
  double log2_cost;      /* exact log2(work * 2^k)             */
} qtn_search_stats;

/*
 * Cut search of size k.  model == NULL: each generation replaces the N-1
 * non-best individuals by crossover/mutation offspring (Sec. III B) scored
 * exactly.  model != NULL: offspring_factor x (N-1) offspring per generation
 * are ranked by the model and only the best N-1 distinct ones are scored
 * exactly.  Returns the best exactly-scored cut set (ascending) in cut_out.
 */
int qtn_cut_search(const qtn_graph *graph, uint32_t p, uint32_t k, int32_t pop, int32_t iters,
                   uint64_t seed, qtn_mlp_t *model, int32_t offspring_factor,
                   uint32_t *cut_out, qtn_search_stats *stats);

/*
 * Several circuits (plans of different graphs, depths, cut sets and bitstring
 * counts) in one persistent launch: the whole-schedule workgroup programs of
 * all plans run in one kernel whose workgroups take (plan, bitstring, slice)
 * items from all of them, as the paper's cores take subgraphs (Sec. III A),
 * then each plan's slice sum follows; the call waits for `stream`.  Every
 * plan must be bound (qtn_plan_bind_workspace) in one-workgroup-per-instance
 * mode (exec_mode = 1), on the current device, with slice_hi[i] - slice_lo[i]
 * at most its slices per wave, and all plans in the same precision form;
 * a plan may appear once.  out receives the partials of plan 0's bitstrings,
 * then plan 1's, and so on (n_bitstrings of each); an empty range gives
 * zeros.  At most 32 plans.  The result of each plan equals its own
 * qtn_contract over the same range bit for bit.
 */
int qtn_batch_contract(qtn_plan_t *const *plans, uint32_t n_plans, const uint64_t *slice_lo,
                       const uint64_t *slice_hi, void *stream, qtn_partial *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * qtn_contract_async, but the workspace, the gate factors and the program
 * descriptors live in a file-scope device array of QTN_NOALLOC_BYTES per
 * GPU that the library holds from load until the process ends, and the
 * partials go to device memory.  No workspace binding is needed and the call
 * allocates nothing: it uploads the plan's constants into that array from
 * host copies kept with the plan (hipMemcpyAsync on `stream`, so the plan
 * must outlive any graph that captures the call), clears the exponent words
 * with a kernel, and enqueues the contraction of slices [slice_lo, slice_hi)
 * with `slices_per_wave` slices per wave on `stream`, one launch after
 * another.  out_dev: n_bitstrings qtn_partial in device memory, written by
 * the last kernel; valid after the stream is synchronised.  QTN_ENOMEM (with
 * the bytes needed) when the plan's constants and workspace exceed the
 * array.  Every call on one GPU uses the same array: calls that overlap on
 * one GPU (other streams, other threads) race and must be serialised by the
 * caller.  Results equal qtn_contract's for the same slices per wave.
 */
#define QTN_NOALLOC_BYTES (64ull << 20)
int qtn_contract_noalloc(qtn_plan_t *plan, uint64_t slice_lo, uint64_t slice_hi,
                         uint64_t slices_per_wave, void *stream, qtn_partial *out_dev);

/* ---------------------------------------------------------------------------
 * Range-partitioned contraction with recovery.  The slices are independent
 * and the master sums one value per slice (Sec. III A); missing slices are
 * recovered by contracting them again (Sec. V).
 * ------------------------------------------------------------------------- */
typedef struct {
  uint64_t ranges;      /* ranges of [0, 2^k)                                   */
  uint64_t contracted;  /* ranges contracted by this call                       */
  uint64_t resumed;     /* ranges read from the checkpoint                      */
  uint64_t retried;     /* failed range calls that were issued again            */
} qtn_range_stats;

/*
 * Contracts [0, 2^k) as ranges [j R, min((j+1) R, 2^k)) with R = range_slices,
 * one qtn_contract call per range on `stream`, and writes the amplitude
 * partial of every bitstring to out[0..n_bitstrings).  A range whose call
 * fails is issued again after the pass, up to max_retries more passes
 * (QTN_ETIMEOUT stops at once, its work may be in flight).  The range partials
 * are combined with qtn_partial_combine in ascending range order, so the
 * result is bit-identical whichever ranges were re-issued or resumed.
 * checkpoint: NULL, or a file path.  Its first line identifies the plan
 * (qtn_plan_fingerprint), the range size, n_bitstrings and k; every further
 * line is one completed range as JSON, {"lo": L, "hi": H, "p": [...]}, with
 * the four doubles of each bitstring's partial in C99 hexadecimal notation
 * (exact).  Ranges already in the file are not contracted again; every
 * completed range is appended and flushed to disk at once.  A torn last line
 * is dropped.  A file of another plan or range size gives QTN_EINVAL.  When
 * ranges are still missing after the retries, the call returns the last
 * range's error and leaves `out` unwritten; the checkpoint keeps the rest.
 */
int qtn_contract_ranges(qtn_plan_t *plan, uint64_t range_slices, int32_t max_retries,
                        const char *checkpoint, void *stream, qtn_partial *out,
                        qtn_range_stats *stats);

/* 64-bit FNV-1a fingerprint of what fixes a plan's slices and amplitudes
 * (graph, p, angles, bitstrings, cut set, precision form); the checkpoint
 * header carries it.  Host only. */
int qtn_plan_fingerprint(const qtn_plan_t *plan, uint64_t *fingerprint);

/* Test hook: the next `count` range calls of qtn_contract_ranges that start
 * at slice `slice_lo` fail with QTN_EHIP without any device work (a lost range
 * forced from the host).  count = 0 clears it.  Host only. */
int qtn_plan_inject_faults(qtn_plan_t *plan, uint64_t slice_lo, int32_t count);

/* Error-free combination of two partials (TwoSum on each component): the
 * sum of the contraction results of two disjoint slice ranges, Eq. (2) and
 * the master-side sum of Sec. III A.  Combining range partials in ascending
 * order of their first slice gives a bit-reproducible amplitude.  Host only;
 * out may alias a or b. */
int qtn_partial_combine(const qtn_partial *a, const qtn_partial *b,
                        qtn_partial *out);

/* Thread-local message describing the last failure ("" if none). */
const char *qtn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QTN_H */
