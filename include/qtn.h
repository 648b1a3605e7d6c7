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
 * traffic, are stored as complex64 with a per-instance power-of-two exponent
 * (rescaled after every grid-wide step); small tensors (under 3% of the
 * bytes), LDS-resident program tensors and the gate factors stay complex128;
 * all products and sums run in FP64 registers.  The slice sum is always FP64.
 * QTN_3XBF16 (split-BF16 matrix-core products) is reserved: the schedules
 * built here sum at most 4 variables per step (Eq. (1) with |kappa| <= 4),
 * an arithmetic intensity far below the matrix-core ridge, so no step is
 * dense enough for it; qtn_plan rejects it with QTN_EINVAL.
 */
enum { QTN_FP64 = 0, QTN_FP32 = 1, QTN_3XBF16 = 2 };

typedef struct qtn_plan_s qtn_plan_t; /* opaque, owned by the library */

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
} qtn_plan_opts;

typedef struct {
  uint32_t n, p, n_vars, n_bitstrings;
  int32_t k;                 /* number of cut variables */
  int32_t width;             /* largest rank of a slice tensor (min-fill width of G - C)  */
  int32_t n_steps;           /* contraction steps per slice                               */
  int32_t n_tensors;
  double log2_flops;         /* real flops per slice-contraction (all bitstrings)          */
  double bytes_per_slice;    /* algorithmic HBM bytes per slice (all bitstrings)          */
  double flops_hoisted;      /* flops of slice-invariant steps, once per wave             */
  double work;               /* sum over buckets of 2^(|N+(v)|+1), one slice, one bitstring */
  double prefactor;          /* 2^{-n/2} times the factor normalisations                 */
  double search_seconds;     /* time spent in the cut search                              */
  int32_t precision;
  int32_t f64_below_rank;    /* intermediates of smaller rank are stored as complex128    */
  int32_t n_programs_wide;   /* workgroup programs (trees of small steps), grid-wide mode */
  int32_t n_launches_wide;   /* kernel launches per wave, grid-wide mode                  */
  uint32_t slice_lds_bytes;  /* LDS per workgroup, one-workgroup-per-instance mode        */
  double slice_scratch_bytes;/* global scratch per workgroup, same mode                   */
} qtn_plan_info;

/* Fills defaults: k = -1, max_rank = 0, k_max = 24, cut_vars = NULL, seed = 0,
 * ga_pop = 11, ga_iters = 4 (Sec. IV A), precision = QTN_FP64, fuse_chains = 1,
 * exec_mode = -1. */
void qtn_plan_opts_default(qtn_plan_opts *opts);

/*
 * Build a host-side plan (no device calls).  Sec. II A (network), Sec. II B
 * (elimination order), Sec. III A (cut and slice), Sec. III B (cut search).
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

void qtn_plan_destroy(qtn_plan_t *plan);

int qtn_plan_query(const qtn_plan_t *plan, qtn_plan_info *info);

/* Copies the k cut variable ids (ascending) into cut[0..k). */
int qtn_plan_cut(const qtn_plan_t *plan, uint32_t *cut, uint32_t capacity);

/* Copies the elimination order of the free variables (n_vars - k ids). */
int qtn_plan_order(const qtn_plan_t *plan, uint32_t *order, uint32_t capacity);

/*
 * Exports the contraction schedule for inspection.  For step t:
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

/* Summed variables of step `step` (most significant first) into kappa[0..nk). */
int qtn_plan_kappa(const qtn_plan_t *plan, int32_t step, int32_t *kappa, uint32_t capacity);

/*
 * Integer index tables of input `input` of step `step`, as uploaded to the
 * device: table[0..256) = pext(c & 255, cmask & 255), table[256..272) =
 * pext(u << 8, cmask) for u < 16, table[272] = cmask >> 12, table[273] =
 * popcount(cmask & 4095), table[274..274+2^nk) = pext(kappa, kmask) <<
 * popcount(cmask), where cmask / kmask are the input's mask bits over the
 * output / summed part of the step index.  `count` receives the length; with
 * table == NULL only the length is returned.
 */
int qtn_plan_index_table(const qtn_plan_t *plan, int32_t step, int32_t input,
                         uint32_t *table, uint32_t capacity, uint32_t *count);

/* Leaf values (FP64) of tensor `tensor`: [bitstring or 1][variant][2^rank]
 * complex, interleaved re/im; `count` receives the number of complex values. */
int qtn_plan_leaf_values(const qtn_plan_t *plan, int32_t tensor, double *values,
                         uint64_t capacity, uint64_t *count);

/*
 * Device workspace needed to contract `slices_per_wave` slices of every
 * bitstring at once (intermediates with liveness reuse, scale exponents,
 * per-slice results).  Pure host computation.
 */
int qtn_plan_workspace_bytes(const qtn_plan_t *plan, uint64_t slices_per_wave,
                             uint64_t *bytes);

/*
 * Binds caller-owned device memory (e.g. a torch tensor) of `bytes` bytes,
 * 256-byte aligned, to the plan, with `slices_per_wave` slices per wave, and
 * uploads the plan's constants to the current device.  The memory must stay
 * valid until the plan is destroyed or rebound.
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
 * was not timed). */
int qtn_plan_step_timing(const qtn_plan_t *plan, int32_t step, qtn_kernel_timing *out);

/* Name of the kernel instance that runs grid-wide step `step` under the
 * bound workspace, e.g. "step_tiled<true, 4, 3, 3>" (rescaled, 4 summed
 * variables, 3 varying operands of which 3 complex64); "" for steps run
 * inside workgroup programs.  NUL-terminated, truncated to `capacity`. */
int qtn_plan_step_kernel(const qtn_plan_t *plan, int32_t step, char *name, uint32_t capacity);

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

typedef struct qtn_mlp_s qtn_mlp_t;

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

/* Error-free combination of two partials (TwoSum on each component). */
int qtn_partial_combine(const qtn_partial *a, const qtn_partial *b,
                        qtn_partial *out);

/* Thread-local message describing the last failure ("" if none). */
const char *qtn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QTN_H */
