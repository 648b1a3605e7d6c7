// Host planner of the sliced QAOA contraction: network construction, line
// graph, min-fill elimination order, cut search (Algorithm 1) and the batched
// contraction schedule shared by every slice.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace qtn {

using cd = std::complex<double>;

constexpr int kMaxIn = 8;        // inputs of one fused contraction step
// Inputs of a step small enough for a workgroup program (output rank below
// kSmallRank): the program kernel holds registers for this many operands
// (with 8 it needs 130-148 registers, spills, and runs 3 waves per SIMD;
// with 4, 102 and 4 waves)
constexpr int kMaxProgIn = 4;
constexpr int kLeafMaxRank = 12; // largest merged leaf group
constexpr int kAlwaysF64Rank = 8; // intermediates below this rank stay complex128
constexpr int kSmallRank = 11;    // steps with fewer output bits run inside one workgroup
constexpr int kMaxStreamKappa = 4; // summed variables per streaming pass
// Each rescaled workspace tensor keeps, per instance, its exponent and the
// maximum magnitude of its entries spread over kMaxSlots words, so that the
// many blocks writing one instance do not all update one address.
constexpr int kMaxSlots = 32;

// One gate factor of the merged binary network (Sec. II A, Fig. 1).  In the
// density-matrix form a factor spans the ket variables and their bra copies.
struct Factor {
  int nv;      // 1 to 4 variables
  int v[4];    // variable ids, axis order of the values (first = most significant)
  int kind;    // 0 ZZ, 1 RX between layers, 2 measured RX (depends on x)
  int layer;
  int qubit;   // RX / OUT qubit
};

struct Network {
  uint32_t n = 0, p = 0, nv = 0;
  // Density-matrix form (Sec. II A): every variable v < n p has a bra copy
  // v + n p; each gate's factor is the Markov-Shi tensor over both, the ket
  // factor times the conjugate of its copy, and the result is |amplitude|^2.
  bool dm = false;
  std::vector<std::pair<uint32_t, uint32_t>> edges;
  std::vector<double> gamma, beta;
  std::vector<uint8_t> bits;  // [B][n]
  uint32_t B = 0;
  std::vector<Factor> factors;
  double prefactor = 1.0;     // 2^{-n/2} times the normalisations below
  // normalised factor values; OUT factors hold one value pair per bitstring
  std::vector<std::vector<cd>> values;  // [factor][B or 1][2^nv]
};

// Build factors, values and the normalisation prefactor.
void build_network(Network &net);

// A gate of a general circuit: matrix[out][in] (row-major), 2x2 or 4x4; for
// two qubits q[0] is the more significant bit of both indices.
struct GateSpec {
  int nq;
  int q[2];
  std::vector<cd> m;
};

// Network of a general circuit on |0^n> measured in bitstrings net.bits
// (net.n qubits, net.B bitstrings): one binary variable per wire segment;
// a diagonal gate keeps its wires' variables (its factor holds the diagonal),
// any other gate starts new ones.  Factors: |0> on every input variable, the
// gate tensors, and the measured value of every final variable.
void build_circuit_network(Network &net, const std::vector<GateSpec> &gates);

// Line graph (variable interaction graph), Sec. II B; adjacency lists sorted.
std::vector<std::vector<int>> line_graph(const Network &net);

struct EliminationResult {
  std::vector<int> order;                 // free variables in elimination order
  std::vector<std::vector<int>> nplus;    // neighbours at elimination, ascending
  int width = 0;                          // max |N+(v)|
  uint64_t work = 0;                      // sum 2^(|N+(v)|+1)
};

// Greedy min-fill on the line graph minus `removed`; ties (fill, degree, id).
EliminationResult min_fill(const std::vector<std::vector<int>> &adj,
                           const std::vector<int> &removed);

// Counter-based SplitMix64 stream (Steele, Lea, Flood 2014).
struct SplitMix64 {
  uint64_t seed, counter = 0;
  explicit SplitMix64(uint64_t s) : seed(s) {}
  uint64_t next();
  uint64_t below(uint64_t m) { return next() % m; }
};

struct CutResult {
  std::vector<int> cut;  // ascending
  int width = 0;
  uint64_t work = 0;
  uint64_t evals = 0;    // distinct cut sets scored exactly
};

// Algorithm 1 (Sec. III B) with exact min-fill fitness.
CutResult ga_cut_search(const std::vector<std::vector<int>> &adj, int M, int N,
                        int T, uint64_t seed);

// ---------------------------------------------------------------------------
// Schedule
// ---------------------------------------------------------------------------

struct Tensor {
  std::vector<int> vars;   // ascending elimination position = MSB first
  int rank() const { return (int)vars.size(); }
  bool leaf = false;
  bool bdep = false;       // depends on the bitstring
  bool sdep = false;       // depends on the slice
  bool f64 = true;         // intermediates: stored as complex128 (else the 64-bit shared-exponent form of the runtime)
  uint32_t selmask = 0;    // leaves: slice bits selecting the variant
  std::vector<cd> values;  // leaves: [B or 1][2^popcount(selmask)][2^rank]
  int producer = -1, last_use = -1;
  // workspace placement (intermediates), set by layout()
  uint64_t data_off = 0;   // byte offset of the data block
  uint64_t exp_off = 0;    // byte offset of the exponent block
  // leaves: element offset in the leaf buffer
  uint64_t leaf_off = 0;
};

struct Step {
  int out = -1;
  std::vector<int> in;
  std::vector<int> kappa;  // summed variables, MSB first
  int rC = 0, nk = 0;
  std::vector<uint32_t> mask;  // per input, over the nk + rC step-index bits
  bool bdep = false, sdep = false;
  int cls = 0;             // 0 E (streaming), 1 G (dense)
};

struct Schedule {
  std::vector<Tensor> tensors;
  std::vector<Step> steps;
  int result = -1;         // rank-0 tensor holding each slice's value
  int width = 0;           // largest intermediate rank
};

struct PlanOpts {
  int precision = 0;
  bool fuse_chains = true;
};

Schedule build_schedule(const Network &net, const std::vector<int> &cut,
                        const std::vector<int> &order, const PlanOpts &o);

// Host index tables of one step input (bit-exact integer maps).
struct InputTables {
  uint32_t lo[256];   // pext(c & 255, cmask & 255)
  uint32_t mid[16];   // pext(((c >> 8) & 15) << 8, cmask)
  uint32_t hi_mask;   // cmask >> 12
  uint32_t hi_shift;  // popcount(cmask & 4095)
  std::vector<uint32_t> kap;  // pext(kappa, kmask) << popcount(cmask)
};
uint32_t pext32(uint32_t x, uint32_t mask);
InputTables input_tables(uint32_t mask, int rC, int nk);

// ---------------------------------------------------------------------------
// Execution plan: which steps run inside one workgroup and where every tensor
// lives.
// ---------------------------------------------------------------------------
enum Loc : int { LOC_LDS = 0, LOC_SCRATCH = 1, LOC_GLOBAL = 2, LOC_LEAF = 3 };
enum ExecMode : int { MODE_WIDE = 0, MODE_SLICE = 1 };

// A tree of steps executed in order by one workgroup per instance.
struct Program {
  std::vector<int> steps;       // schedule step indices, ascending
  int root = -1;                // output tensor of the last step
  bool bdep = false, sdep = false;
  uint32_t lds_bytes = 0;       // LDS tensors (complex128)
  uint64_t scratch_bytes = 0;   // per-workgroup global scratch
  int nslots = 0;               // program-local exponent slots
  std::vector<int> staged;      // gate factors copied to LDS at program start
  // workspace tensors made outside the program that it copies to LDS
  // (complex128) at its start: tensor id, LDS byte offset, exponent slot
  struct StagedGlobal {
    int tensor;
    uint64_t off;
    int slot;
  };
  std::vector<StagedGlobal> staged_global;
};

struct LaunchGroup {
  int kind = 0;                 // 0 workgroup programs, 1 one grid-wide step
  std::vector<int> programs;
  int step = -1;
};

struct ExecPlan {
  int mode = MODE_WIDE;
  std::vector<Program> programs;
  std::vector<LaunchGroup> launches;
  std::vector<int> loc;         // per tensor
  std::vector<uint64_t> off;    // LDS or scratch byte offset
  std::vector<int> slot;        // exponent slot of LDS / scratch tensors
  uint32_t lds_bytes = 0;       // largest program LDS footprint
  uint64_t scratch_per_wg = 0;
  // Closing chain folded into a grid-wide step (grid-wide mode): when every
  // step after `dot_step` only sums variables of its output T against gate
  // factors over T's variables, the rank-0 result is sum_c T[c] W(c) with W
  // the product of those factors.  dot_step then reduces its outputs against
  // W instead of storing T, and the closing steps are not launched.
  int dot_step = -1;
  int dot_tensor = -1;              // T
  std::vector<int> dot_leaves;      // the closing chain's gate factors
  std::vector<uint32_t> dot_masks;  // their variables as bits of T's index
};

constexpr int kMaxDotLeaves = 32;   // gate factors of a folded closing chain
constexpr int kMaxDotMixed = 8;     // of those, with variables on both sides of bit 8
constexpr int kMaxDotValues = 256;  // their values together (complex)

// MODE_WIDE: trees of small steps become workgroup programs, the rest run as
// grid-wide steps.  MODE_SLICE: the whole schedule is one program per
// (bitstring, slice) instance.
ExecPlan build_exec(const Schedule &s, int mode, uint32_t lds_budget);

struct Layout {
  uint64_t S = 1;                // slices per wave
  uint64_t data_bytes = 0;       // intermediates region
  uint64_t exp_bytes = 0;        // exponents region
  uint64_t total_bytes = 0;
  uint64_t partial_off = 0;      // running per-bitstring partials
  uint64_t flag_off = 0;         // range word of the 64-bit form (after the partials)
  uint64_t scratch_off = 0;      // per-workgroup scratch region
  uint64_t wg_slots = 0;
  uint64_t dot_off = 0;          // block partials of a folded closing chain
  uint64_t dot_slots = 0;        // per instance of T
};

// Instance count of a tensor inside a wave.
inline uint64_t instances(const Tensor &t, uint64_t B, uint64_t S) {
  return (t.bdep ? B : 1) * (t.sdep ? S : 1);
}

// Storage precision of every intermediate.  FP64 plans store everything as
// complex128.  Mixed plans store the large tensors, which carry the HBM
// traffic, in 8 bytes per element (a shared 8-bit exponent and two 28-bit
// mantissas) and keep the small ones (at most `small_share` of the 8-byte
// bytes) as complex128.  Returns the rank below which tensors stay
// complex128.
int assign_storage(Schedule &s, int precision, double small_share = 0.03);

inline int elem_bytes(const Tensor &t) { return t.f64 ? 16 : 8; }

// Workspace: GLOBAL tensors (first-fit with liveness), their exponents,
// per-workgroup scratch for `wg_slots` workgroups, partial sums.
Layout layout(Schedule &s, const ExecPlan &x, uint64_t B, uint64_t S, uint64_t wg_slots);

// Launch units of one wave: 0 clears the exponent region, 1..n are the
// launch groups of the execution plan, n+1 is the slice sum.  A unit depends
// on every earlier unit whose workspace bytes it reads or writes while the
// other writes them (or reads what it writes); units that do not depend on
// each other may run on different streams.
struct LaunchGraph {
  std::vector<std::vector<int>> deps;  // direct predecessors, transitively reduced
  std::vector<int> stream;             // stream of each unit (0 = the caller's)
  std::vector<char> record;            // another stream waits for this unit
  std::vector<int> order;              // enqueue order: a topological order, longest remaining path first
  int nstreams = 1;
  // longest dependency path from a unit without dependencies: units of one
  // level never depend on each other and may run in one launch
  std::vector<int> level;
  int nlevels = 0;
};
LaunchGraph launch_graph(const Schedule &s, const ExecPlan &x, const Layout &L, uint64_t B,
                         uint64_t S, bool scaled, int max_streams);

struct Costs {
  double flops_per_slice = 0;    // all bitstrings
  double bytes_per_slice = 0;
  double flops_hoisted = 0;      // slice-invariant steps, once per wave
  double bytes_hoisted = 0;
};
Costs schedule_costs(const Schedule &s, uint64_t B, uint64_t S);

}  // namespace qtn
