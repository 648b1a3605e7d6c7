// Device side of libqtn for gfx950: plan upload, the contraction kernels
// (Eq. (1) generalised to several operands and summed indices) and the
// compensated FP64 slice sum (Eq. (2); the master-side sum of Sec. III A).
//
// Two kinds of launches execute a wave of (bitstring, slice) instances:
//   * workgroup programs: one workgroup runs a tree of steps for one instance,
//     its intermediates in LDS (complex128) or per-workgroup scratch;
//   * grid-wide steps: one large step over all instances and output elements.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/qtn.h"
#include "plan_state.h"

namespace qtn {

// ---------------------------------------------------------------------------
// Descriptors
// ---------------------------------------------------------------------------
// Operand of a step.  Every index map follows from `mask`, the operand's bits
// over the step index kappa:c (kappa above the rC output bits): the operand
// index of step index x is pext(x, mask).
struct OpDesc {
  const void *base;       // GLOBAL: workspace tensor; LEAF: leaf block
  uint64_t bstride;       // elements between bitstrings
  uint64_t sstride;       // elements between slice-local instances
  int *E;                 // GLOBAL scaled tensors: exponent per instance
  uint32_t *M;            // GLOBAL scaled tensors: kMaxSlots max-exponent words each
  uint32_t ebstride, esstride;
  // the last 16 bytes are what a workgroup program step reads first
  uint32_t mask;          // operand bits over the step index kappa:c
  uint32_t off;           // LDS / scratch byte offset
  int16_t slot;           // LDS / scratch: exponent slot, -1 for none
  uint8_t loc;            // Loc
  uint8_t f64;            // stored as complex128 (else the 64-bit shared-exponent form)
  uint32_t selmask;       // leaves: slice bits that pick the variant
};
static_assert(sizeof(OpDesc) == 64, "OpDesc layout");

struct PStep {
  OpDesc in[kMaxIn];      // operands varying with the output element first
  OpDesc out;
  int nin, rC, nk;
  int nvary;              // in[0..nvary) vary with the output element
  int nf32;               // of those, in[0..nf32) are stored in the 64-bit form
  uint32_t tiled_lds;     // > 0: run as step_tiled with this much LDS
  uint32_t wg_flags;      // in a workgroup program: 1 = every operand in LDS
  int tiled_fold;         // step_tiled: operand staged as complex128 times the
                          // kappa coefficient, or -1
  uint32_t tiled_pair;    // > 0: step_tiled_pair may run it with this much more LDS
  uint32_t dot;           // 1: reduce the outputs against the closing chain's
                          //    gate factors (DotArgs) instead of storing them
  uint32_t dot_lds;       // dynamic LDS bytes of that epilogue
  const void *dotp;       // DotArgs in device memory (set at launch)
  uint32_t *range_flag;   // the workspace's range word (enc_c64e)
};
static_assert(sizeof(PStep) % 16 == 0, "PStep layout");

// Gate factors of a closing chain folded into a grid-wide step: the step
// adds acc(c) W(c) over its outputs c, W(c) = prod_l leaf_l[pext(c, mask_l)],
// one partial per block and instance.  Leaves are ordered: variables only in
// the low 8 bits of c (fixed per lane), only above them (fixed per row), both.
struct DotLeaf {
  const double *base;     // complex128 values, interleaved re/im
  uint64_t bstride;       // complex values between bitstrings (0: shared)
  uint32_t selmask;       // slice bits selecting the variant
  uint32_t mask;          // variables as bits of the step's output index
  uint32_t rank;          // 2^rank values per variant
  uint32_t off;           // position of its values in the staged table
};
static_assert(sizeof(DotLeaf) == 32, "DotLeaf layout");
constexpr uint32_t kDotValues = kMaxDotValues;   // staged leaf values per instance
struct DotArgs {
  uint32_t nleaf, nlo, nhi, nmix;
  uint32_t nvals;         // staged values (<= kDotValues)
  uint32_t slots;         // partial slots per instance
  double2 *part;          // [instance][slots] block partials
  DotLeaf leaf[kMaxDotLeaves];
  uint8_t owner[kDotValues];  // leaf of each staged value
};
static_assert(sizeof(DotArgs) % 16 == 0, "DotArgs layout");

// One tensor a program stages in LDS at its start (as complex128):
//  * a gate factor: the variant of instance (b, s) is
//    base + b * bstride + pext(s, selmask) * count, count complex128 values;
//  * a workspace tensor made by an earlier launch: base + b * bstride +
//    sl * sstride, 64-bit form or complex128; in the rescaled form its
//    exponent E[b * ebstride + sl * esstride] goes to the program's slot.
struct LeafStage {
  const void *base;
  uint64_t bstride, sstride;
  const int *E;
  uint32_t selmask, count, lds_off;
  uint32_t ebstride, esstride;
  int16_t slot;
  uint8_t f64, global;
  uint32_t pad[2];
};
static_assert(sizeof(LeafStage) == 64, "LeafStage layout");

// A program in device memory is one blob: its LeafStage records, then its
// PStep descriptors.  A launch of workgroup programs names up to
// kMaxGroupProgs of them in its arguments, so that a workgroup finds its
// program without a memory round trip.  The programs of one launch may come
// from different plans (several circuits in one persistent launch): each
// carries its own blob, slice range and per-workgroup scratch.
constexpr int kMaxGroupProgs = 32;
constexpr int kDescChunk = 8;          // program steps resident in LDS at a time
struct GroupArgs {
  uint32_t nprog;
  uint32_t item_end[kMaxGroupProgs];   // cumulative item counts
  uint16_t nsteps[kMaxGroupProgs];
  uint16_t nstage[kMaxGroupProgs];
  uint8_t bdep[kMaxGroupProgs];
  uint8_t sdep[kMaxGroupProgs];
  uint32_t ns[kMaxGroupProgs];         // slices of the program's wave
  const char *blob[kMaxGroupProgs];    // the program's blob
  char *scratch[kMaxGroupProgs];       // its plan's per-workgroup scratch region
  uint64_t scratch_stride[kMaxGroupProgs];
  uint64_t s_lo[kMaxGroupProgs];       // first slice of the program's wave
};

// Launch configuration of a grid-wide streaming step.
struct StepTune {
  uint32_t target = 1024;   // blocks over the chip
  bool stream_only = false; // run step_stream even where step_tiled applies
  bool pair = false;        // run step_tiled_pair where it applies
};

struct DeviceState {
  int device = -1;
  int mode = MODE_WIDE;
  void *leafbuf = nullptr;        // complex128 gate factors
  char *blobbuf = nullptr;        // program blobs
  qtn_partial *host_partials = nullptr;      // pinned host memory, B partials
  qtn_partial *host_partials_dev = nullptr;  // its device address
  std::vector<uint64_t> blob_off; // per program
  std::vector<uint64_t> leaf_elem_off;
  std::vector<PStep> steps;       // one descriptor per schedule step (host copy)
  char *ws = nullptr;
  uint64_t ws_bytes = 0;
  Layout L;
  uint32_t lds_bytes = 0, lds_total = 0;
  uint32_t desc_bytes = 0;        // program descriptor region of the LDS
  int max_slots = 0;
  // optional per-launch timing of the streaming step kernel
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  std::vector<double> ev_bytes, ev_flops;
  std::vector<int> ev_step;
  double t_ms = 0, t_bytes = 0, t_flops = 0;
  struct StepTiming {
    uint64_t launches = 0;
    double ms = 0, bytes = 0, flops = 0;
  };
  std::vector<StepTiming> t_step;  // per schedule step
  StepTiming t_prog;               // launches of workgroup programs
  uint64_t t_launches = 0, t_failed = 0;
  int t_last_error = 0;
  std::vector<double> step_bytes, step_flops;  // per instance of each step
  // per item of each workgroup program: bytes of the tensors it reads or
  // writes outside LDS (gate factors, workspace, scratch) and flops of its steps
  std::vector<double> prog_bytes, prog_flops;
  uint64_t dot_args_off = 0;      // DotArgs of a folded closing chain in the blob
  std::vector<StepTune> tune;     // launch configuration per step (qtn_plan_autotune)
  // independent launch units run on side streams (default priority),
  // ordered by events after their dependencies
  LaunchGraph lg;
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
  std::vector<hipEvent_t> unit_ev;
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kSide] = {nullptr, nullptr, nullptr};
  int max_streams = 1 + kSide;
  // launch units level by level, independent steps of a level in one
  // step_multi launch (QTN_LEVELS=0: side streams under graph capture)
  bool levels = true;
  // captured launch sequence of one slice range, replayed while it matches
  bool use_graphs = true;
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  uint64_t g_lo = 0, g_hi = 0;
  bool g_timing = false;
  bool g_scaled = false;
  // plans that store tensors in the 64-bit form: synchronous contractions
  // run without per-instance rescaling (the values are checked against the
  // form's exponent range by the range word) until one leaves the range;
  // from then on, and for asynchronous calls, they rescale
  bool unscaled = true;
  bool force_scaled = false;      // the re-run of a contraction that left the range
  int range_misses = 0;           // consecutive such contractions
  uint64_t range_reruns = 0;      // contractions repeated with rescaling
  uint32_t *flag_dev = nullptr;   // device address of the range word (host_partials slot B)
  size_t g_ev_used = 0;
  std::vector<double> g_ev_bytes, g_ev_flops;
  std::vector<int> g_ev_step;
};

static void drop_graph(DeviceState *d) {
  if (d->gexec) (void)hipGraphExecDestroy(d->gexec);
  d->gexec = nullptr;
}

void device_state_free(DeviceState *d) {
  if (!d) return;
  drop_graph(d);
  if (d->gstream) (void)hipStreamDestroy(d->gstream);
  for (auto e : d->unit_ev) (void)hipEventDestroy(e);
  if (d->fork_ev) (void)hipEventDestroy(d->fork_ev);
  for (int k = 0; k < DeviceState::kSide; ++k) {
    if (d->join_ev[k]) (void)hipEventDestroy(d->join_ev[k]);
    if (d->side[k]) (void)hipStreamDestroy(d->side[k]);
  }
  for (auto e : d->ev) (void)hipEventDestroy(e);
  for (void *p : {(void *)d->leafbuf, (void *)d->blobbuf})
    if (p) (void)hipFree(p);
  if (d->host_partials) (void)hipHostFree(d->host_partials);
  delete d;
}

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t dpext(uint32_t x, uint32_t m) {
  uint32_t r = 0;
  uint32_t k = 0;
  while (m) {
    uint32_t low = m & (0u - m);
    r |= ((x & low) ? 1u : 0u) << k;
    ++k;
    m &= m - 1;
  }
  return r;
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  double2 r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// c + a b with four fused multiply-adds
__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {
  c.x = fma(a.x, b.x, c.x);
  c.x = fma(-a.y, b.y, c.x);
  c.y = fma(a.x, b.y, c.y);
  c.y = fma(a.y, b.x, c.y);
  return c;
}

// 64-bit complex storage of the rescaled (mixed) form: one biased exponent
// shared by both parts and two 28-bit two's-complement mantissas,
//   word = E << 56 | (re & 0xFFFFFFF) << 28 | (im & 0xFFFFFFF),
//   value = (re + i im) * 2^(E - 154);  E = 0 only in the zero word.
// With m = max(|re|, |im|) in [2^(e-1), 2^e), E = e + 127 and the parts are
// rounded to the nearest multiple of 2^(e-27): an absolute error of at most
// 2^-28 |z| per part (complex64 rounds each part to 2^-24 of itself).  The
// same eight bytes as complex64.
// The range word `flag` (one per plan workspace) is set when enc_c64e
// flushes a non-zero value or clamps one: in a run without per-instance
// rescaling that means the values left the 64-bit form's exponent range and
// the contraction is repeated with rescaling.  Read and cleared by the last
// slice_sum of each contraction.
__device__ __forceinline__ uint64_t enc_c64e(double2 v, uint32_t *flag) {
  const double m = fmax(fabs(v.x), fabs(v.y));
  if (!(m > 0.0)) return 0ull;
  int e;
  (void)frexp(m, &e);
  const int E = e + 127;
  // one atomic per wave and store, from its lowest lane that left the range
  const bool out = E < 1 || E > 255;
  const uint64_t outs = __ballot(out);
  if (out && flag && __lane_id() == (uint32_t)(__ffsll((unsigned long long)outs) - 1)) atomicOr(flag, 1u);
  if (E < 1) return 0ull;   // below 2^-127 of the instance scale: flushed
  const double lim = 134217727.0;  // 2^27 - 1
  const int sh = 27 - min(e, 128);
  const int mr = (int)fmin(fmax(rint(ldexp(v.x, sh)), -lim), lim);
  const int mi = (int)fmin(fmax(rint(ldexp(v.y, sh)), -lim), lim);
  return ((uint64_t)min(E, 255) << 56) | ((uint64_t)((uint32_t)mr & 0xFFFFFFFu) << 28) |
         (uint64_t)((uint32_t)mi & 0xFFFFFFFu);
}

// The rescaled store of a grid-wide step: v * 2^-sh stored in the tensor's
// form.  For the 64-bit form the shift only changes the stored exponent (the
// mantissas are those of v), so no scaling pass over the values is needed.
// Returns the float exponent field of the stored value's larger part (the
// per-instance maximum that consumers shift by).
__device__ __forceinline__ uint32_t store_scaled(void *base, uint32_t f64, uint64_t i, double2 v, int sh) {
  if (f64) {
    v.x = ldexp(v.x, -sh);
    v.y = ldexp(v.y, -sh);
    ((double2 *)base)[i] = v;
    const float ax = (float)fabs(v.x), ay = (float)fabs(v.y);
    return max(__float_as_uint(ax), __float_as_uint(ay)) & 0x7F800000u;
  }
  const double m = fmax(fabs(v.x), fabs(v.y));
  uint64_t w = 0ull;
  uint32_t mb = 0u;
  if (m > 0.0) {
    // frexp exponent of m from its bits (m is normal: |v| of the steps is far
    // above 2^-1022)
    const int e = (int)((__double_as_longlong(m) >> 52) & 0x7ff) - 1022;
    const int es = e - sh;   // exponent of the stored value
    const int E = es + 127;
    if (E >= 1) {
      const int lim = 134217727;  // 2^27 - 1
      const int mr = min(max(__double2int_rn(ldexp(v.x, 27 - e)), -lim), lim);
      const int mi = min(max(__double2int_rn(ldexp(v.y, 27 - e)), -lim), lim);
      w = ((uint64_t)min(E, 255) << 56) | ((uint64_t)((uint32_t)mr & 0xFFFFFFFu) << 28) |
          (uint64_t)((uint32_t)mi & 0xFFFFFFFu);
      mb = (uint32_t)min(max(es + 126, 0), 255) << 23;
    }
  }
  ((uint64_t *)base)[i] = w;
  return mb;
}

__device__ __forceinline__ double2 dec_c64e(uint64_t w) {
  const int re = ((int)((uint32_t)(w >> 28) << 4)) >> 4;
  const int im = ((int)((uint32_t)w << 4)) >> 4;
  const int sc = (int)(uint32_t)(w >> 56) - 154;
  return make_double2(ldexp((double)re, sc), ldexp((double)im, sc));
}

__device__ __forceinline__ double2 load_g(const void *base, uint32_t f64, uint64_t i) {
  if (f64) return ((const double2 *)base)[i];
  return dec_c64e(((const uint64_t *)base)[i]);
}

__device__ __forceinline__ void store_g(void *base, uint32_t f64, uint64_t i, double2 v, uint32_t *flag) {
  if (f64)
    ((double2 *)base)[i] = v;
  else
    ((uint64_t *)base)[i] = enc_c64e(v, flag);
}

// Exponent e with 2^(e-1) <= x < 2^e for the positive float with bits `b`
// (0 for zero or subnormal): frexp's convention.
__device__ __forceinline__ int exp_of_bits(uint32_t b) {
  int be = (int)((b >> 23) & 255u);
  return be == 0 ? 0 : be - 126;
}

// Float exponent field of the larger component magnitude, rounded to float
// (an upper bound on the stored value's binade in either storage form).
__device__ __forceinline__ uint32_t max_bits(double2 v, uint32_t f64) {
  (void)f64;
  const float ax = (float)fabs(v.x);
  const float ay = (float)fabs(v.y);
  return max(__float_as_uint(ax), __float_as_uint(ay)) & 0x7F800000u;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t m) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o, 64));
  return m;
}

// Block-wide max over 256 threads; every thread must call it.
template <typename P>
__device__ __forceinline__ uint32_t block_max(uint32_t m, P red4) {
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red4[threadIdx.x >> 6] = m;
  __syncthreads();
  const uint32_t r = max(max(red4[0], red4[1]), max(red4[2], red4[3]));
  __syncthreads();
  return r;
}

// Raise the instance maximum (a no-return atomic; zero never raises it).
__device__ __forceinline__ void raise_max(uint32_t *slot, uint32_t m) {
  if (m) atomicMax(slot, m);
}

// Maximum over the kMaxSlots words of one instance (any thread, serial).
__device__ __forceinline__ uint32_t slots_max(const uint32_t *M) {
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < kMaxSlots; ++k) m = max(m, M[k]);
  return m;
}

// Offset of the operand's block for instance (bitstring b, slice-local sl,
// slice s); a leaf's variant holds 2^popcount(mask) values.
template <typename D>
__device__ __forceinline__ uint64_t inst_off(const D &o, uint32_t b, uint32_t sl, uint32_t s) {
  uint64_t r = (uint64_t)b * o.bstride + (uint64_t)sl * o.sstride;
  if (o.selmask) r += (uint64_t)dpext(s, o.selmask) << __popc(o.mask);
  return r;
}

__device__ __forceinline__ uint32_t out_bits(int rC) { return rC >= 32 ? ~0u : ((1u << rC) - 1u); }

// Operand index contributed by output element c and by summed value kappa.
__device__ __forceinline__ uint32_t cpart(const OpDesc &o, uint32_t c, int rC) {
  return dpext(c, o.mask & out_bits(rC));
}
__device__ __forceinline__ uint32_t kpart(const OpDesc &o, uint32_t kap, int rC) {
  return rC >= 32 ? 0u : (dpext(kap, o.mask >> rC) << __popc(o.mask & out_bits(rC)));
}

// ---------------------------------------------------------------------------
// Folded closing chain: the epilogue of a grid-wide step that adds acc(c) W(c)
// over its outputs c instead of storing them (see DotArgs).  LDS (dynamic,
// after the step's own): staged factor values | 32 row products | 4 sums.
// ---------------------------------------------------------------------------
struct DotState {
  double2 wl;                 // product of the lane-only factors at this lane
  uint32_t li[kMaxDotMixed];  // lane part of each mixed factor's index
  double2 acc;                // this thread's sum of acc(c) W(c)
};

// Copies the DotArgs record into LDS (once per block); every thread calls it.
__device__ void dot_args_to_lds(const DotArgs *src, DotArgs *dst) {
  const uint32_t *s = (const uint32_t *)src;
  uint32_t *d = (uint32_t *)dst;
  for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(DotArgs) / 4); i += blockDim.x) d[i] = s[i];
  __syncthreads();
}

// Stages the factor values of instance (b, s) and sets this lane's parts.
// A is the LDS copy of the record.  Every thread of the block calls it.
__device__ void dot_begin(const DotArgs *A, uint32_t b, uint32_t s, double2 *sv, DotState &D) {
  const uint32_t t = threadIdx.x;
  const uint32_t nvals = A->nvals, nlo = A->nlo, nmix = A->nmix;
  __syncthreads();  // the previous instance is done with the table
  if (t < nvals) {
    const DotLeaf &L = A->leaf[A->owner[t]];
    const uint64_t o = (uint64_t)b * L.bstride + ((uint64_t)dpext(s, L.selmask) << L.rank) + (t - L.off);
    sv[t] = make_double2(L.base[2 * o], L.base[2 * o + 1]);
  }
  __syncthreads();
  D.wl = make_double2(1.0, 0.0);
  for (uint32_t l = 0; l < nlo; ++l) D.wl = cmul(D.wl, sv[A->leaf[l].off + dpext(t, A->leaf[l].mask)]);
#pragma unroll
  for (uint32_t j = 0; j < (uint32_t)kMaxDotMixed; ++j)
    D.li[j] = j < nmix ? dpext(t, A->leaf[nlo + A->nhi + j].mask & 255u) : 0u;
  D.acc = make_double2(0.0, 0.0);
}

// Products of the row-only factors for rows row0 .. row0 + n - 1 (n <= 32).
// Every thread of the block calls it.
__device__ void dot_rows(const DotArgs *A, const double2 *sv, uint32_t row0, uint32_t n, double2 *sw) {
  __syncthreads();  // readers of the previous rows' products are done
  const uint32_t t = threadIdx.x;
  if (t < n) {
    const uint32_t row = row0 + t;
    double2 w = make_double2(1.0, 0.0);
    for (uint32_t l = A->nlo; l < A->nlo + A->nhi; ++l) w = cmul(w, sv[A->leaf[l].off + dpext(row, A->leaf[l].mask >> 8)]);
    sw[t] = w;
  }
  __syncthreads();
}

// Adds v W(c) / wl for the output c = row:lane, wrow being the row's
// product: the lane-only factor wl is applied once, in dot_end.
__device__ __forceinline__ void dot_add(const DotArgs *A, const double2 *sv, DotState &D, double2 wrow,
                                        uint32_t row, double2 v) {
  const uint32_t nmix = A->nmix, m0 = A->nlo + A->nhi;
  double2 w = wrow;
#pragma unroll
  for (uint32_t j = 0; j < (uint32_t)kMaxDotMixed; ++j)
    if (j < nmix) {
      const DotLeaf &L = A->leaf[m0 + j];
      w = cmul(w, sv[L.off + (D.li[j] | (dpext(row, L.mask >> 8) << __popc(L.mask & 255u)))]);
    }
  D.acc = cfma(v, w, D.acc);
}

// Block sum in a fixed order to part[qo * slots + slot].  Every thread calls it.
__device__ void dot_end(const DotArgs *A, DotState &D, uint64_t qo, uint32_t slot, double2 *red) {
  double2 v = cmul(D.acc, D.wl);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  if ((threadIdx.x & 63u) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 r = red[0];
    for (int w = 1; w < 4; ++w) {
      r.x += red[w].x;
      r.y += red[w].y;
    }
    A->part[qo * A->slots + slot] = r;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Workgroup programs
// ---------------------------------------------------------------------------
// Dynamic LDS of the program kernel: tensors | 256 partial sums | exponent
// slots | 4 reduction words.
extern __shared__ __align__(16) char wg_smem[];

// LDS-qualified pointee types, so that every access compiles to an LDS
// instruction rather than a generic (flat) one.
#define QTN_LDS __attribute__((address_space(3)))

// complex128 in LDS as one 16-byte vector (a single ds_read_b128/ds_write_b128)
typedef double lds_c128 __attribute__((ext_vector_type(2)));

// complex128 values in LDS as (re, im) pairs of doubles
__device__ __forceinline__ double2 lds_ld(const QTN_LDS double *p, uint32_t i) {
  return make_double2(p[2 * i], p[2 * i + 1]);
}
__device__ __forceinline__ void lds_st(QTN_LDS double *p, uint32_t i, double2 v) {
  p[2 * i] = v.x;
  p[2 * i + 1] = v.y;
}

struct WgCtx {
  QTN_LDS double *lds;    // program tensors (complex128)
  QTN_LDS double *red;    // 256 partial sums (complex128)
  QTN_LDS int *sE;        // exponent slots
  QTN_LDS uint32_t *sM;
  QTN_LDS uint32_t *red4;
  char *scratch;          // this workgroup's global scratch
};

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// pext of the low 8 bits of x under an 8-bit mask m that is the same in
// every lane, unrolled over the 8 mask bits: no loop and no branch (the bit
// loop of dpext costs a scalar branch and a few scalar instructions per set
// bit, and every wave of the workgroup runs it for every operand and step)
__device__ __forceinline__ uint32_t pext8_uniform(uint32_t x, uint32_t m) {
  uint32_t r = 0, k = 0;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint32_t mb = (m >> b) & 1u;
    r |= ((x >> b) & mb) << k;
    k += mb;
  }
  return r;
}

// One step of a workgroup program.  Complex128 tensors in LDS are not
// rescaled: they carry their power-of-two exponent in sE[slot] and FP64 has
// range to spare.  Outputs stored in global memory or scratch keep the
// rescaled form of the grid steps (values times 2^-sh, maximum tracked).
// Specialised on the operand count NIN and on LDSONLY (every operand is an
// LDS tensor or a staged gate factor), so that the operand loop is straight
// code whose LDS reads issue together.
template <bool SCALE, int NIN, bool LDSONLY>
__device__ void wg_step_n(const QTN_LDS PStep &st, uint32_t b, uint32_t sl, uint32_t s, const WgCtx &W) {
  constexpr int kMaxIn = NIN;   // the loops below cover exactly the operands
  const uint32_t t = threadIdx.x;
  const int nin = NIN, rC = (int)uni((uint32_t)st.rC), nk = (int)uni((uint32_t)st.nk);
  // operand keys, read in one batch
  uint32_t mk[kMaxIn], ok[kMaxIn], mt[kMaxIn];
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i) {
    mk[i] = st.in[i].mask;
    ok[i] = st.in[i].off;
    mt[i] = *(const QTN_LDS uint32_t *)&st.in[i].slot;   // slot | loc << 16 | f64 << 24
  }
  const uint32_t omt = *(const QTN_LDS uint32_t *)&st.out.slot;
  const uint32_t ooff = uni(st.out.off);
  const bool all_lds = LDSONLY;
  uint32_t lo[kMaxIn], loff[kMaxIn], hm[kMaxIn], hs[kMaxIn];
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i) {
    const bool used = i < nin;
    const uint32_t m = used ? uni(mk[i]) : 0u;
    mk[i] = m;
    mt[i] = uni(mt[i]);
    lo[i] = pext8_uniform(t, m & 255u);
    hm[i] = m >> 8;
    hs[i] = __popc(m & 255u);
    loff[i] = used ? uni(ok[i]) / 16 : 0u;
  }
  const bool wide_idx = rC + nk > 8;   // else every step index fits in the low 8 bits
  // operands outside the LDS
  const char *gptr[kMaxIn];
  uint32_t gf64[kMaxIn];
  int sh = 0, esum = 0;
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i) {
    gptr[i] = nullptr;
    gf64[i] = 1;
    if (i >= nin) continue;
    if (LDSONLY && !SCALE) continue;   // nothing outside LDS, no exponents
    const uint32_t loc = (mt[i] >> 16) & 255u;
    const int slot = (int16_t)(mt[i] & 0xffffu);
    if (loc == LOC_SCRATCH) {
      gptr[i] = W.scratch + uni(ok[i]);
      gf64[i] = mt[i] >> 24;
    } else if (loc == LOC_GLOBAL || loc == LOC_LEAF) {
      const QTN_LDS OpDesc &o = st.in[i];
      const uint64_t es = (loc == LOC_LEAF || (mt[i] >> 24)) ? 16 : 8;
      gptr[i] = (const char *)o.base + inst_off(o, b, sl, s) * es;
      gf64[i] = loc == LOC_LEAF ? 1u : (mt[i] >> 24);
    }
    if (SCALE) {
      if (loc == LOC_LDS && slot >= 0) {
        esum += W.sE[slot];
      } else if (loc == LOC_SCRATCH && slot >= 0) {
        const int e = exp_of_bits(W.sM[slot]);
        sh += e;
        esum += W.sE[slot] + e;
      } else if (loc == LOC_GLOBAL) {
        const QTN_LDS OpDesc &o = st.in[i];
        const uint32_t qi = b * o.ebstride + sl * o.esstride;
        const int e = exp_of_bits(slots_max(o.M + (uint64_t)qi * kMaxSlots));
        sh += e;
        esum += o.E[qi] + e;
      }
    }
  }
  // product of the operands at the step index whose low 8 bits are this
  // thread's and whose bits above are `hi`
  auto point = [&](uint32_t hi) -> double2 {
    double2 v[kMaxIn];
#pragma unroll
    for (int i = 0; i < kMaxIn; ++i) {
      const uint32_t idx = lo[i] + (wide_idx ? (dpext(hi, hm[i]) << hs[i]) : 0u);
      if (all_lds || ((mt[i] >> 16) & 255u) == LOC_LDS || i >= nin)
        v[i] = lds_ld(W.lds, loff[i] + idx);
      else
        v[i] = load_g(gptr[i], gf64[i], idx);
    }
    double2 prod = v[0];
#pragma unroll
    for (int i = 1; i < kMaxIn; ++i)
      if (i < nin) prod = cmul(prod, v[i]);
    return prod;
  };
  const uint32_t oloc = (omt >> 16) & 255u, of64 = oloc == LOC_LDS ? 1u : (omt >> 24);
  const int oslot = (int16_t)(omt & 0xffffu);
  const bool scale_out = SCALE && oloc != LOC_LDS;
  const int shift = scale_out ? sh : 0;
  if (!scale_out) esum -= sh;  // LDS outputs keep the unscaled products
  char *optr = nullptr;
  if (oloc == LOC_SCRATCH) {
    optr = W.scratch + ooff;
  } else if (oloc == LOC_GLOBAL) {
    const QTN_LDS OpDesc &out = st.out;
    optr = (char *)out.base + ((uint64_t)b * out.bstride + (uint64_t)sl * out.sstride) * (of64 ? 16 : 8);
  }
  auto put = [&](uint32_t c, double2 v) {
    if (oloc == LOC_LDS)
      lds_st(W.lds, ooff / 16 + c, v);
    else
      store_g(optr, of64, c, v, st.range_flag);
  };
  const uint32_t nC = 1u << rC;
  uint32_t mx = 0;
  if (rC >= 8) {
    const uint32_t nkap = 1u << nk;
    const uint32_t rows = nC >> 8;
    for (uint32_t j = 0; j < rows; ++j) {
      const uint32_t c = (j << 8) | t;
      double2 acc = make_double2(0.0, 0.0);
      for (uint32_t k = 0; k < nkap; ++k) {
        const double2 p = point((k << (rC - 8)) | j);
        acc.x += p.x;
        acc.y += p.y;
      }
      if (scale_out) {
        acc.x = ldexp(acc.x, -shift);
        acc.y = ldexp(acc.y, -shift);
        mx = max(mx, max_bits(acc, of64));
      }
      put(c, acc);
    }
  } else {
    // Threads cover the low 8 bits of the index kappa:c; the kappa bits
    // among them are summed by a fixed-order tree through LDS.
    const int kb = min(nk, 8 - rC);
    const uint32_t c = t & (nC - 1u);
    const uint32_t kl = t >> rC;
    double2 acc = make_double2(0.0, 0.0);
    if (kl < (1u << kb)) {
      const uint32_t nkh = 1u << (nk - kb);
      for (uint32_t kh = 0; kh < nkh; ++kh) {
        const double2 p = point(kh);
        acc.x += p.x;
        acc.y += p.y;
      }
    }
    if (kb > 0) {
      lds_st(W.red, t, acc);
      __syncthreads();
      for (uint32_t h = (1u << kb) >> 1; h >= 1; h >>= 1) {
        if (kl < h) {
          const double2 o = lds_ld(W.red, t + (h << rC));
          const double2 m = lds_ld(W.red, t);
          lds_st(W.red, t, make_double2(m.x + o.x, m.y + o.y));
        }
        __syncthreads();
      }
      if (t < nC) acc = lds_ld(W.red, t);
    }
    if (t < nC) {
      if (scale_out) {
        acc.x = ldexp(acc.x, -shift);
        acc.y = ldexp(acc.y, -shift);
        mx = max_bits(acc, of64);
      }
      put(c, acc);
    }
  }
  if (SCALE) {
    if (scale_out) mx = block_max(mx, W.red4);
    if (t == 0) {
      if (oloc == LOC_GLOBAL) {
        const QTN_LDS OpDesc &out = st.out;
        const uint32_t qo = b * out.ebstride + sl * out.esstride;
        out.E[qo] = esum;
        out.M[(uint64_t)qo * kMaxSlots] = mx;
      } else {
        W.sE[oslot] = esum;
        if (scale_out) W.sM[oslot] = mx;
      }
    }
  }
  __syncthreads();
}

// MAXNIN: the largest operand count among the launch's steps (4 or 8); the
// kernel's registers are those of its largest case.
template <bool SCALE, int MAXNIN>
__device__ void wg_step(const QTN_LDS PStep &st, uint32_t b, uint32_t sl, uint32_t s, const WgCtx &W) {
  const uint32_t nin = uni((uint32_t)st.nin);
  const bool lds_only = (uni((uint32_t)st.wg_flags) & 1u) != 0;
#define QTN_WG(N)                                      \
  case N:                                              \
    if (lds_only)                                      \
      wg_step_n<SCALE, N, true>(st, b, sl, s, W);     \
    else                                               \
      wg_step_n<SCALE, N, false>(st, b, sl, s, W);    \
    break;
  if constexpr (MAXNIN <= 4) {
    switch (nin) {
      QTN_WG(1) QTN_WG(2) QTN_WG(3) QTN_WG(4)
      default: break;
    }
  } else {
    switch (nin) {
      QTN_WG(1) QTN_WG(2) QTN_WG(3) QTN_WG(4) QTN_WG(5) QTN_WG(6) QTN_WG(7) QTN_WG(8)
      default: break;
    }
  }
#undef QTN_WG
}

// Source of element i of a staging record for instance (b, sl, s).
__device__ __forceinline__ double2 stage_load(const QTN_LDS LeafStage &L, uint32_t b, uint32_t sl,
                                              uint32_t s, uint32_t i) {
  if (L.global) {
    const uint64_t o = (uint64_t)b * L.bstride + (uint64_t)sl * L.sstride + i;
    if (L.f64) return ((const double2 *)L.base)[o];
    return dec_c64e(((const uint64_t *)L.base)[o]);
  }
  return ((const double2 *)L.base)[b * L.bstride + (uint64_t)dpext(s, L.selmask) * L.count + i];
}

// Copies the staged tensors of a program into LDS for instance (b, sl, s).
// Records of at most 64 values: wave w takes records w, w+4, ..., eight
// loads in flight before any store.  Larger records: the whole workgroup,
// eight loads in flight per thread.
__device__ void stage_leaves(const QTN_LDS LeafStage *ls, uint32_t n, uint32_t b, uint32_t sl,
                             uint32_t s, QTN_LDS double *lds, QTN_LDS int *sE) {
  constexpr int G = 8;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (uint32_t j0 = w * G; j0 < n; j0 += 4 * G) {
    double2 v[G];
    uint32_t dst[G];
#pragma unroll
    for (int r = 0; r < G; ++r) {
      dst[r] = ~0u;
      const uint32_t j = j0 + r;
      if (j < n) {
        const QTN_LDS LeafStage &L = ls[j];
        const uint32_t count = L.count;
        if (count <= 64 && lane < count) {
          v[r] = stage_load(L, b, sl, s, lane);
          dst[r] = L.lds_off + lane;
        }
        if (lane == 0 && L.global && L.E) sE[L.slot] = L.E[b * L.ebstride + sl * L.esstride];
      }
    }
#pragma unroll
    for (int r = 0; r < G; ++r)
      if (dst[r] != ~0u) lds_st(lds, dst[r], v[r]);
  }
  for (uint32_t j = 0; j < n; ++j) {
    const QTN_LDS LeafStage &L = ls[j];
    const uint32_t count = L.count;
    if (count <= 64) continue;
    for (uint32_t i0 = 0; i0 < count; i0 += G * 256) {
      double2 v[G];
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const uint32_t i = i0 + r * 256 + threadIdx.x;
        if (i < count) v[r] = stage_load(L, b, sl, s, i);
      }
#pragma unroll
      for (int r = 0; r < G; ++r) {
        const uint32_t i = i0 + r * 256 + threadIdx.x;
        if (i < count) lds_st(lds, L.lds_off + i, v[r]);
      }
    }
  }
}

// Copies n bytes (a multiple of 16) from global memory to LDS, four 16-byte
// loads per thread in flight at a time.
__device__ __forceinline__ void copy_to_lds(QTN_LDS char *dst, const char *__restrict__ src, uint32_t n) {
  typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
  const uint32_t n16 = n >> 4;
  for (uint32_t i0 = 0; i0 < n16; i0 += 4 * 256) {
    u64x2 v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = i0 + r * 256 + threadIdx.x;
      if (i < n16) v[r] = ((const u64x2 *)src)[i];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = i0 + r * 256 + threadIdx.x;
      if (i < n16) ((QTN_LDS u64x2 *)dst)[i] = v[r];
    }
  }
}

// Persistent workgroups walk the items of one launch: the items of program
// j are its instances, (bitstring, slice) or fewer when the program's root
// does not depend on them.  Per item the workgroup copies the program's
// staging records and first steps into LDS, stages the gate factors, then
// runs the steps, kDescChunk descriptors at a time.  Items never wait on
// each other.
template <bool SCALE, int MAXNIN>
__global__ __launch_bounds__(256) void wg_programs(const GroupArgs ga, uint32_t total, uint32_t lds_bytes,
                                                   int max_slots, uint32_t desc_off) {
  char *smem = wg_smem;
  WgCtx W;
  QTN_LDS char *sm = (QTN_LDS char *)smem;
  W.lds = (QTN_LDS double *)sm;
  W.red = (QTN_LDS double *)(sm + lds_bytes);
  W.sE = (QTN_LDS int *)(sm + lds_bytes + 256 * 16);
  W.sM = (QTN_LDS uint32_t *)(W.sE + max_slots);
  W.red4 = W.sM + max_slots;
  QTN_LDS char *desc = sm + desc_off;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    uint32_t j = 0;
    while (j + 1 < ga.nprog && item >= ga.item_end[j]) ++j;
    const uint32_t q = item - (j ? ga.item_end[j - 1] : 0u);
    const uint32_t ns = ga.sdep[j] ? ga.ns[j] : 1u;
    const uint32_t b = q / ns;
    const uint32_t sl = q - b * ns;
    const uint32_t s = (uint32_t)(ga.s_lo[j] + sl);
    W.scratch = ga.scratch[j] + (uint64_t)blockIdx.x * ga.scratch_stride[j];
    const char *blob = ga.blob[j];
    const uint32_t nst = ga.nsteps[j], nstg = ga.nstage[j];
    const uint32_t lsb = nstg * (uint32_t)sizeof(LeafStage);
    __syncthreads();  // the previous item is done with the LDS
    copy_to_lds(desc, blob, lsb + min(nst, (uint32_t)kDescChunk) * (uint32_t)sizeof(PStep));
    __syncthreads();
    if (nstg) {
      stage_leaves((const QTN_LDS LeafStage *)desc, nstg, b, sl, s, W.lds, W.sE);
      __syncthreads();
    }
    const QTN_LDS PStep *ps = (const QTN_LDS PStep *)(desc + lsb);
    for (uint32_t k = 0; k < nst; ++k) {
      if (k && k % kDescChunk == 0) {
        // the previous step ended with a barrier
        copy_to_lds(desc + lsb, blob + lsb + k * (uint32_t)sizeof(PStep),
                    min(nst - k, (uint32_t)kDescChunk) * (uint32_t)sizeof(PStep));
        __syncthreads();
      }
      wg_step<SCALE, MAXNIN>(ps[k % kDescChunk], b, sl, s, W);
    }
  }
}

// ---------------------------------------------------------------------------
// Grid-wide steps (operands in the workspace or leaves)
// ---------------------------------------------------------------------------
struct InstanceSetup {
  uint64_t off[kMaxIn];
  int sh, esum;
  uint32_t qo;
  uint64_t obase;
};

// The same set-up done by a whole block.  setup_begin issues every load at
// once: thread t reads slot word t % 32 of input t / 32 (and the exponent
// word of that input), the 32 slot words of an input are reduced within the
// wave, so that all rescaled inputs cost one memory round trip instead of
// one each.  After a barrier, setup_end adds the shifts from LDS.  The block
// must not rewrite S before every thread has passed setup_end.
struct SetupLds {
  uint32_t m[kMaxIn];   // slot maximum of each input (0: not rescaled)
  int e[kMaxIn];        // exponent word of each input
};
template <bool SCALE>
__device__ __forceinline__ void setup_begin(const PStep &d, uint32_t ns, uint64_t q, uint64_t s_lo,
                                            InstanceSetup &I, SetupLds &S) {
  const uint32_t b = (uint32_t)(q / ns);
  const uint32_t sl = (uint32_t)(q - (uint64_t)b * ns);
  const uint32_t s = (uint32_t)(s_lo + sl);
  I.sh = 0;
  I.esum = 0;
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i)
    if (i < d.nin) I.off[i] = inst_off(d.in[i], b, sl, s);
  I.qo = b * d.out.ebstride + sl * d.out.esstride;
  I.obase = (uint64_t)b * d.out.bstride + (uint64_t)sl * d.out.sstride;
  if (SCALE) {
    static_assert(kMaxIn * kMaxSlots <= 256, "one thread per slot word");
    const uint32_t t = threadIdx.x, i = t / kMaxSlots, k = t % kMaxSlots;
    uint32_t w = 0;
    int e = 0;
    if (i < (uint32_t)d.nin && d.in[i].loc == LOC_GLOBAL) {
      const OpDesc &in = d.in[i];
      const uint32_t qi = b * in.ebstride + sl * in.esstride;
      w = in.M[(uint64_t)qi * kMaxSlots + k];
      if (k == 0) e = in.E[qi];
    }
#pragma unroll
    for (int o = kMaxSlots / 2; o > 0; o >>= 1) w = max(w, (uint32_t)__shfl_xor((int)w, o, kMaxSlots));
    if (k == 0 && i < (uint32_t)kMaxIn) {
      S.m[i] = w;
      S.e[i] = e;
    }
  }
}
template <bool SCALE>
__device__ __forceinline__ void setup_end(const PStep &d, InstanceSetup &I, const SetupLds &S) {
  if (SCALE) {
#pragma unroll
    for (int i = 0; i < kMaxIn; ++i)
      if (i < d.nin) {
        const int x = exp_of_bits(S.m[i]);   // 0 for inputs that are not rescaled
        I.sh += x;
        I.esum += S.e[i] + x;
      }
  }
}

template <bool SCALE>
__device__ __forceinline__ void setup_instance(const PStep &d, uint32_t ns, uint64_t q,
                                               uint64_t s_lo, InstanceSetup &I) {
  const uint32_t b = (uint32_t)(q / ns);
  const uint32_t sl = (uint32_t)(q - (uint64_t)b * ns);
  const uint32_t s = (uint32_t)(s_lo + sl);
  I.sh = 0;
  I.esum = 0;
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i) {
    if (i < d.nin) {
      const OpDesc &in = d.in[i];
      I.off[i] = inst_off(in, b, sl, s);
      if (SCALE && in.loc == LOC_GLOBAL) {
        const uint32_t qi = b * in.ebstride + sl * in.esstride;
        const int e = exp_of_bits(slots_max(in.M + (uint64_t)qi * kMaxSlots));
        I.sh += e;
        I.esum += in.E[qi] + e;
      }
    }
  }
  I.qo = b * d.out.ebstride + sl * d.out.esstride;
  I.obase = (uint64_t)b * d.out.bstride + (uint64_t)sl * d.out.sstride;
}

__device__ __forceinline__ double2 grid_point(const PStep &d, const uint64_t *cidx, uint32_t nkap) {
  double2 acc = make_double2(0.0, 0.0);
  for (uint32_t kk = 0; kk < nkap; ++kk) {
    double2 prod = load_g(d.in[0].base, d.in[0].f64, cidx[0] + kpart(d.in[0], kk, d.rC));
#pragma unroll
    for (int i = 1; i < kMaxIn; ++i)
      if (i < d.nin) prod = cmul(prod, load_g(d.in[i].base, d.in[i].f64, cidx[i] + kpart(d.in[i], kk, d.rC)));
    acc.x += prod.x;
    acc.y += prod.y;
  }
  return acc;
}

// Streaming steps (output of >= 2^kStreamMinRank elements per instance).
// The block's y coordinate walks the instances; each x-block owns chunks of 4096
// consecutive output elements.  Thread t always handles elements with low
// bits t, so its per-lane index part is fixed; the mid/high parts and the
// kappa offsets are block-uniform and come from LDS.  Operands that do not
// depend on the output element (gate factors on summed variables) are folded
// into one coefficient per kappa value, computed once per instance.
template <bool SCALE, int NK, int NV, int NF>
__device__ __forceinline__ void stream_body(const PStep &d, uint32_t nb, uint32_t ns, uint64_t s_lo,
                                            uint32_t jspan, uint32_t bx, uint32_t by, uint32_t gx,
                                            uint32_t gy) {
  constexpr uint32_t NKAP = 1u << NK;
  __shared__ uint32_t s_mid[NV][16];
  __shared__ uint32_t s_kap[NV][NKAP];
  __shared__ double2 s_coef[NKAP];
  __shared__ uint32_t red4[4];
  const uint32_t t = threadIdx.x;
  const uint32_t cb = out_bits(d.rC);
  if (t < NV * 16) s_mid[t >> 4][t & 15] = dpext((t & 15) << 8, d.in[t >> 4].mask & cb);
  if (t < NV * NKAP) s_kap[t / NKAP][t % NKAP] = kpart(d.in[t / NKAP], t % NKAP, d.rC);
  uint32_t lo[NV], hmask[NV], hshift[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const uint32_t cm = d.in[v].mask & cb;
    lo[v] = dpext(t, cm & 255u);
    hmask[v] = cm >> 12;
    hshift[v] = __popc(cm & 4095u);
  }
  const uint64_t Q = (uint64_t)nb * ns;
  const uint32_t nC = 1u << d.rC;
  // work units of the instance: jspan x 256 consecutive elements
  const uint32_t units = (nC >> 8) / jspan;
  extern __shared__ __align__(16) char dsm[];
  const bool dot = d.dot != 0;
  DotArgs *DA = (DotArgs *)dsm;
  double2 *dsv = (double2 *)(dsm + sizeof(DotArgs));
  if (dot) dot_args_to_lds((const DotArgs *)d.dotp, DA);
  double2 *dsw = dot ? dsv + DA->nvals : nullptr;
  DotState DS;
  __shared__ SetupLds SL;
  for (uint64_t q = by; q < Q; q += gy) {
    InstanceSetup I;
    setup_begin<SCALE>(d, ns, q, s_lo, I, SL);
    if (dot) {
      const uint32_t b = (uint32_t)(q / ns);
      dot_begin(DA, b, (uint32_t)(s_lo + (q - (uint64_t)b * ns)), dsv, DS);
    }
    if (t < NKAP) {
      double2 c = make_double2(1.0, 0.0);
#pragma unroll
      for (int i = NV; i < kMaxIn; ++i)
        if (i < d.nin) c = cmul(c, load_g(d.in[i].base, d.in[i].f64, I.off[i] + kpart(d.in[i], t, d.rC)));
      s_coef[t] = c;
    }
    __syncthreads();
    setup_end<SCALE>(d, I, SL);
    // per-lane operand pointers for this instance; in[0..NF) are in the 64-bit form
    const char *vp[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
      vp[v] = (const char *)d.in[v].base + (I.off[v] + lo[v]) * (v < NF ? 8u : 16u);
    char *op = (char *)d.out.base + I.obase * (d.out.f64 ? 16u : 8u);
    const uint32_t of = d.out.f64;
    const int sh = I.sh;
    uint32_t wmax = 0;
    for (uint32_t u = bx; u < units; u += gx) {
      const uint32_t j0 = u * jspan;            // in units of 256 elements
      if (dot) dot_rows(DA, dsv, j0, jspan, dsw);
      uint32_t hoff[NV];
#pragma unroll 1
      for (uint32_t jj = 0; jj < jspan; ++jj) {
        const uint32_t j = (j0 + jj) & 15u;
        const uint32_t c = ((j0 + jj) << 8) | t;
        if (jj == 0 || j == 0) {
          // a unit may span several chunks of 16 rows: the high part of
          // each operand index changes at every chunk boundary
          const uint32_t ch = (j0 + jj) >> 4;
#pragma unroll
          for (int v = 0; v < NV; ++v) hoff[v] = dpext(ch, hmask[v]) << hshift[v];
        }
        double2 acc = make_double2(0.0, 0.0);
        // all loads of a group of kappa values are issued before any product:
        // up to 16 loads in flight per thread (every kappa value at once
        // when the step has few varying operands)
        constexpr uint32_t KU = NKAP * NV <= 16 ? NKAP : (NKAP > 4 ? 4 : NKAP);
#pragma unroll 1
        for (uint32_t kb = 0; kb < NKAP; kb += KU) {
          uint64_t xf[KU][NF > 0 ? NF : 1];
          double2 xd[KU][NV - NF > 0 ? NV - NF : 1];
#pragma unroll
          for (uint32_t kk = 0; kk < KU; ++kk) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const uint32_t idx = hoff[v] + s_mid[v][j] + s_kap[v][kb + kk];
              if (v < NF)
                xf[kk][v < NF ? v : 0] = ((const uint64_t *)vp[v])[idx];
              else
                xd[kk][v >= NF ? v - NF : 0] = ((const double2 *)vp[v])[idx];
            }
          }
          // keep the loads above together so they are in flight at once
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (uint32_t kk = 0; kk < KU; ++kk) {
            double2 prod = s_coef[kb + kk];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              const double2 x = v < NF ? dec_c64e(xf[kk][v < NF ? v : 0]) : xd[kk][v >= NF ? v - NF : 0];
              prod = cmul(prod, x);
            }
            acc.x += prod.x;
            acc.y += prod.y;
          }
        }
        if (dot) {
          if (SCALE) {
            acc.x = ldexp(acc.x, -sh);
            acc.y = ldexp(acc.y, -sh);
          }
          dot_add(DA, dsv, DS, dsw[jj], j0 + jj, acc);
        } else if (SCALE) {
          wmax = max(wmax, store_scaled(op, of, c, acc, sh));
        } else {
          store_g(op, of, c, acc, d.range_flag);
        }
      }
    }
    if (dot) {
      dot_end(DA, DS, I.qo, bx, dsw + 32);
      if (SCALE && t == 0 && bx == 0) d.out.E[I.qo] = I.esum;
    } else if (SCALE) {
      // every thread of the block ran the same trips
      const uint32_t m = block_max(wmax, red4);
      if (t == 0) {
        raise_max(d.out.M + (uint64_t)I.qo * kMaxSlots + (bx % kMaxSlots), m);
        if (bx == 0) d.out.E[I.qo] = I.esum;
      }
    }
    __syncthreads();  // s_coef and SL are rewritten for the next instance
  }
}

template <bool SCALE, int NK, int NV, int NF>
__global__ __launch_bounds__(256) void step_stream(const PStep d, uint32_t nb, uint32_t ns,
                                                   uint64_t s_lo, uint32_t jspan) {
  stream_body<SCALE, NK, NV, NF>(d, nb, ns, s_lo, jspan, blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
}

// Visiting order of the four low row bits of a 16-row chunk of step_tiled,
// 2 bits per position (innermost first): bits that large operands lack come
// first, so that their staged runs serve consecutive rows; the weight of a
// bit is the number of staged elements of the operands that lack it (ties:
// lower bit first).  The host uses it to decide row pairing.
__host__ __device__ inline uint32_t tiled_row_order(const PStep &d) {
  const uint32_t cb = d.rC >= 32 ? ~0u : ((1u << d.rC) - 1u);
  uint32_t wbit[4] = {0u, 0u, 0u, 0u};
  for (int v = 0; v < d.nvary && v < 4; ++v) {
    const uint32_t cm = d.in[v].mask & cb;
    const uint32_t rdep = cm >> 8;
    const uint32_t n = 1u << (__builtin_popcount(d.in[v].mask >> d.rC) + __builtin_popcount(cm & 255u));
    for (int b = 0; b < 4; ++b)
      if (!((rdep >> b) & 1u)) wbit[b] += n;
  }
  uint32_t rord = 0;
  for (int i = 0; i < 4; ++i) {
    uint32_t rank = 0;
    for (int b = 0; b < 4; ++b) rank += (wbit[b] > wbit[i] || (wbit[b] == wbit[i] && b < i)) ? 1u : 0u;
    rord |= (uint32_t)i << (2u * rank);
  }
  return rord;
}

// Streaming steps whose varying operands are re-read many times per row.
// For a row of 256 consecutive output elements, operand v is touched at
// base_v(row) + pext(c & 255, mask) + (pext(kappa, kmask) << pc): 2^nkv runs
// of 2^nlo contiguous elements (pext keeps the summed bits on top and the
// low output bits at the bottom of the operand index).  The block stages
// those runs in LDS once per row and sums over kappa from LDS, so each
// operand element is fetched once per row instead of once per use.
template <bool SCALE, int NK, int NV, int NF, bool FOLD, bool PAIR = false>
__device__ __forceinline__ void tiled_body(const PStep &d, uint32_t nb, uint32_t ns, uint64_t s_lo,
                                           uint32_t jspan, uint32_t bx, uint32_t by, uint32_t gx,
                                           uint32_t gy) {
  // PAIR (FOLD steps, jspan >= 16): each thread sums two rows that differ in
  // the innermost row bit of the visiting order, which operand 0 lacks and
  // every other operand has; operand 0's staged runs and LDS reads serve
  // both rows, the others are staged twice (second regions after the first).
  constexpr uint32_t NKAP = 1u << NK;
  extern __shared__ __align__(16) char stage[];
  __shared__ uint32_t s_mid[NV][16];
  __shared__ uint32_t s_kap[NV][NKAP];
  __shared__ double2 s_coef[NKAP];   // by kappa
  __shared__ double2 s_coefl[NKAP];  // by position in the sum (unfolded steps)
  __shared__ uint32_t red4[4];
  const uint32_t t = threadIdx.x;
  const uint32_t cb = out_bits(d.rC);
  // The kappa sum runs in a permuted order: when the last operand does not
  // depend on some summed bit b, bits 0 and b trade places, so that the
  // positions 2j and 2j+1 share that operand's element and the products of
  // the other operands are summed before it multiplies them once (the same
  // sum, regrouped by distributivity).  The swap is its own inverse.
  const uint32_t missing = NV > 1 ? ~(d.in[NV - 1].mask >> d.rC) & (NKAP - 1u) : 0u;
  const bool fact = missing != 0;
  const uint32_t bsw = fact ? (uint32_t)__builtin_ctz(missing) : 0u;
  auto perm = [&](uint32_t k) {
    const uint32_t x = (k ^ (k >> bsw)) & 1u;  // bits 0 and bsw differ
    return k ^ (x | (x << bsw));
  };
  if (t < NV * 16) s_mid[t >> 4][t & 15] = dpext((t & 15) << 8, d.in[t >> 4].mask & cb);
  if (t < NV * NKAP) {
    const OpDesc &in = d.in[t / NKAP];
    s_kap[t / NKAP][t % NKAP] = dpext(perm(t % NKAP), in.mask >> d.rC) << __popc(in.mask & cb & 255u);
  }
  uint32_t lo[NV], soff[NV], nlo[NV], nkv[NV], pc[NV], hmask[NV], hshift[NV];
  uint32_t bytes = 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const uint32_t cm = d.in[v].mask & cb;
    lo[v] = dpext(t, cm & 255u);
    nlo[v] = __popc(cm & 255u);
    nkv[v] = __popc(d.in[v].mask >> d.rC);
    pc[v] = __popc(cm);
    hmask[v] = cm >> 12;
    hshift[v] = __popc(cm & 4095u);
    soff[v] = bytes;
    bytes += (1u << (nkv[v] + nlo[v])) * 16u;   // staged as complex128
  }
  uint32_t soff2[NV];   // PAIR: the second row's runs of operands 1..NV-1
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    soff2[v] = soff[v];
    if (PAIR && v > 0) {
      soff2[v] = bytes;
      bytes += (1u << (nkv[v] + nlo[v])) * 16u;
    }
  }
  // row bits each operand depends on, and the visiting order of the four
  // low row bits (2 bits per position: the row bit visited there)
  uint32_t rdep[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) rdep[v] = (d.in[v].mask & cb) >> 8;
  const uint32_t rord = tiled_row_order(d);
  constexpr int fold = FOLD ? 0 : -1;
  const uint64_t Q = (uint64_t)nb * ns;
  const uint32_t rows = (1u << d.rC) >> 8;
  const uint32_t units = rows / jspan;
  const bool dot = d.dot != 0;
  DotArgs *DA = (DotArgs *)(stage + d.tiled_lds);
  double2 *dsv = (double2 *)(stage + d.tiled_lds + sizeof(DotArgs));
  if (dot) dot_args_to_lds((const DotArgs *)d.dotp, DA);
  double2 *dsw = dot ? dsv + DA->nvals : nullptr;
  DotState DS;
  __shared__ SetupLds SL;
  for (uint64_t q = by; q < Q; q += gy) {
    InstanceSetup I;
    setup_begin<SCALE>(d, ns, q, s_lo, I, SL);
    if (dot) {
      const uint32_t b = (uint32_t)(q / ns);
      dot_begin(DA, b, (uint32_t)(s_lo + (q - (uint64_t)b * ns)), dsv, DS);
    }
    if (t < NKAP) {
      double2 c = make_double2(1.0, 0.0);
#pragma unroll
      for (int i = NV; i < kMaxIn; ++i)
        if (i < d.nin) c = cmul(c, load_g(d.in[i].base, d.in[i].f64, I.off[i] + kpart(d.in[i], t, d.rC)));
      s_coef[t] = c;
      s_coefl[perm(t)] = c;
    }
    __syncthreads();
    setup_end<SCALE>(d, I, SL);
    char *op = (char *)d.out.base + I.obase * (d.out.f64 ? 16u : 8u);
    const uint32_t of = d.out.f64;
    const int sh = I.sh;
    uint32_t wmax = 0;
    // operand v at position k of the sum, as complex128
    auto opnd = [&](int v, uint32_t k) __attribute__((always_inline)) {
      const uint32_t idx = s_kap[v][k] + lo[v];
      const lds_c128 c = ((const QTN_LDS lds_c128 *)(stage + soff[v]))[idx];
      return make_double2(c.x, c.y);
    };
    // PAIR: operand v (v >= 1) for the second row
    auto opnd2 = [&](int v, uint32_t k) __attribute__((always_inline)) {
      const uint32_t idx = s_kap[v][k] + lo[v];
      const lds_c128 c = ((const QTN_LDS lds_c128 *)(stage + soff2[v]))[idx];
      return make_double2(c.x, c.y);
    };
    // coefficient x operands 0 .. upto-1 at position k (the folded operand
    // carries the coefficient)
    auto head = [&](uint32_t k, int upto) __attribute__((always_inline)) {
      double2 prod = fold < 0 ? s_coefl[k] : make_double2(1.0, 0.0);
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (v < upto) {
          const double2 x = opnd(v, k);
          prod = (v == 0 && fold >= 0) ? x : cmul(prod, x);
        }
      return prod;
    };
    // acc + head(k, v) x operand v at position k
    auto mac = [&](uint32_t k, int v, double2 acc) __attribute__((always_inline)) {
      if (v == 0 && fold >= 0) {
        const double2 x = opnd(0, k);
        return make_double2(acc.x + x.x, acc.y + x.y);
      }
      return cfma(head(k, v), opnd(v, k), acc);
    };
    for (uint32_t u = bx; u < units; u += gx) {
      if (dot) dot_rows(DA, dsv, u * jspan, jspan, dsw);
      // operand bases of the current chunk of 16 rows: instance offset plus
      // the index part of the row bits above the lowest four
      const char *cbase[NV];
      uint32_t key[NV];
      if constexpr (PAIR) {
        // the two rows' outputs: stored, or reduced against the closing chain
        auto finish = [&](uint32_t row, double2 acc) __attribute__((always_inline)) {
          if (dot) {
            if (SCALE) {
              acc.x = ldexp(acc.x, -sh);
              acc.y = ldexp(acc.y, -sh);
            }
            dot_add(DA, dsv, DS, dsw[row - u * jspan], row, acc);
          } else if (SCALE) {
            wmax = max(wmax, store_scaled(op, of, ((uint64_t)row << 8) | t, acc, sh));
          } else {
            store_g(op, of, ((uint64_t)row << 8) | t, acc, d.range_flag);
          }
        };
        // operand v's runs for `row`, as complex128, at byte `off` of the stage
        auto stage_op = [&](int v, uint32_t row, uint32_t off) __attribute__((always_inline)) {
          constexpr uint32_t esz_f = 8u, esz_d = 16u;
          const uint32_t esz = v < NF ? esz_f : esz_d;
          const char *rb = cbase[v] + (uint64_t)__builtin_amdgcn_readfirstlane(s_mid[v][row & 15u]) * esz;
          const uint32_t n = 1u << (nkv[v] + nlo[v]);
          const uint32_t lmask = (1u << nlo[v]) - 1u;
          QTN_LDS lds_c128 *dst = (QTN_LDS lds_c128 *)(stage + off);
          for (uint32_t e = t; e < n; e += 512) {
            const bool two = e + 256 < n;
            const uint32_t g0 = (((e >> nlo[v]) << pc[v]) + (e & lmask)) * esz;
            const uint32_t e1 = e + 256;
            const uint32_t g1 = (((e1 >> nlo[v]) << pc[v]) + (e1 & lmask)) * esz;
            double2 x0, x1 = make_double2(0.0, 0.0);
            if (v < NF) {
              const uint64_t w0 = *(const uint64_t *)(rb + g0);
              uint64_t w1 = 0ull;
              if (two) w1 = *(const uint64_t *)(rb + g1);
              x0 = dec_c64e(w0);
              x1 = dec_c64e(w1);
            } else {
              x0 = *(const double2 *)(rb + g0);
              if (two) x1 = *(const double2 *)(rb + g1);
            }
            if (v == 0) x0 = cmul(x0, s_coef[e >> nlo[v]]);
            lds_c128 c;
            c.x = x0.x;
            c.y = x0.y;
            dst[e] = c;
            if (two) {
              if (v == 0) x1 = cmul(x1, s_coef[e1 >> nlo[v]]);
              c.x = x1.x;
              c.y = x1.y;
              dst[e1] = c;
            }
          }
        };
        auto rowmap = [&](uint32_t jj) __attribute__((always_inline)) {
          const uint32_t lo4 = jj & 15u;
          return u * jspan + ((jj & ~15u) | (((lo4 >> 0) & 1u) << (rord & 3u)) |
                              (((lo4 >> 1) & 1u) << ((rord >> 2) & 3u)) |
                              (((lo4 >> 2) & 1u) << ((rord >> 4) & 3u)) |
                              (((lo4 >> 3) & 1u) << ((rord >> 6) & 3u)));
        };
#pragma unroll 1
        for (uint32_t jj = 0; jj < jspan; jj += 2) {
          // rows 2i and 2i+1 of the visiting order differ in row bit rord & 3
          const uint32_t row0 = rowmap(jj), row1 = rowmap(jj + 1);
          if ((jj & 15u) == 0) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
              cbase[v] = (const char *)d.in[v].base +
                         (I.off[v] + ((uint64_t)dpext(row0 >> 4, hmask[v]) << hshift[v])) * (v < NF ? 8u : 16u);
          }
          __syncthreads();  // the previous rows' readers are done
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const uint32_t kv = row0 & rdep[v];
            if (jj > 0 && kv == key[v]) continue;
            key[v] = kv;
            stage_op(v, row0, soff[v]);
            if (v > 0) stage_op(v, row1, soff2[v]);
          }
          __syncthreads();
          double2 acc0 = make_double2(0.0, 0.0), acc1 = make_double2(0.0, 0.0);
          if (NV > 1 && fact) {
            // positions 2j and 2j+1 share the last operand's element
#pragma unroll 2
            for (uint32_t k = 0; k < NKAP; k += 2) {
              const double2 a0 = opnd(0, k), a1 = opnd(0, k + 1);
              double2 h0 = a0, g0 = a1, h1 = a0, g1 = a1;
#pragma unroll
              for (int v = 1; v < NV - 1; ++v) {
                h0 = cmul(h0, opnd(v, k));
                g0 = cmul(g0, opnd(v, k + 1));
                h1 = cmul(h1, opnd2(v, k));
                g1 = cmul(g1, opnd2(v, k + 1));
              }
              acc0 = cfma(make_double2(h0.x + g0.x, h0.y + g0.y), opnd(NV - 1, k), acc0);
              acc1 = cfma(make_double2(h1.x + g1.x, h1.y + g1.y), opnd2(NV - 1, k), acc1);
            }
          } else {
#pragma unroll 2
            for (uint32_t k = 0; k < NKAP; ++k) {
              const double2 a = opnd(0, k);
              double2 p0 = a, p1 = a;
#pragma unroll
              for (int v = 1; v < NV; ++v) {
                p0 = cmul(p0, opnd(v, k));
                p1 = cmul(p1, opnd2(v, k));
              }
              acc0 = make_double2(acc0.x + p0.x, acc0.y + p0.y);
              acc1 = make_double2(acc1.x + p1.x, acc1.y + p1.y);
            }
          }
          finish(row0, acc0);
          finish(row1, acc1);
        }
        continue;
      }
#pragma unroll 1
      for (uint32_t jj = 0; jj < jspan; ++jj) {
        // rows of a 16-row chunk in the order rord (innermost bits first)
        const uint32_t lo4 = jj & 15u;
        const uint32_t row = u * jspan + (jspan >= 16u
                                             ? (jj & ~15u) | (((lo4 >> 0) & 1u) << (rord & 3u)) |
                                                   (((lo4 >> 1) & 1u) << ((rord >> 2) & 3u)) |
                                                   (((lo4 >> 2) & 1u) << ((rord >> 4) & 3u)) |
                                                   (((lo4 >> 3) & 1u) << ((rord >> 6) & 3u))
                                             : jj);
        if (jj == 0 || lo4 == 0) {
#pragma unroll
          for (int v = 0; v < NV; ++v)
            cbase[v] = (const char *)d.in[v].base +
                       (I.off[v] + ((uint64_t)dpext(row >> 4, hmask[v]) << hshift[v])) * (v < NF ? 8u : 16u);
        }
        __syncthreads();  // the previous row's readers are done
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          // the staged runs of v depend only on its row bits: when those are
          // the previous row's, the runs in LDS are this row's too
          const uint32_t kv = row & rdep[v];
          if (jj > 0 && kv == key[v]) continue;
          key[v] = kv;
          constexpr uint32_t esz_f = 8u, esz_d = 16u;
          const uint32_t esz = v < NF ? esz_f : esz_d;
          // the table entry is the same for every lane
          const char *rb = cbase[v] + (uint64_t)__builtin_amdgcn_readfirstlane(s_mid[v][row & 15u]) * esz;
          const uint32_t n = 1u << (nkv[v] + nlo[v]);
          const uint32_t lmask = (1u << nlo[v]) - 1u;
          // every operand is staged as complex128 (the 64-bit stored form is
          // decoded here, once per element and row, not in the kappa loop);
          // the folded operand is multiplied by the kappa coefficient of its
          // run.  Two elements per trip, both loads issued before either write.
          QTN_LDS lds_c128 *dst = (QTN_LDS lds_c128 *)(stage + soff[v]);
          for (uint32_t e = t; e < n; e += 512) {
            const bool two = e + 256 < n;
            // byte offsets within the operand: below 2^31 (checked by the host)
            const uint32_t g0 = (((e >> nlo[v]) << pc[v]) + (e & lmask)) * esz;
            const uint32_t e1 = e + 256;
            const uint32_t g1 = (((e1 >> nlo[v]) << pc[v]) + (e1 & lmask)) * esz;
            double2 x0, x1 = make_double2(0.0, 0.0);
            if (v < NF) {
              const uint64_t w0 = *(const uint64_t *)(rb + g0);
              uint64_t w1 = 0ull;
              if (two) w1 = *(const uint64_t *)(rb + g1);
              x0 = dec_c64e(w0);
              x1 = dec_c64e(w1);
            } else {
              x0 = *(const double2 *)(rb + g0);
              if (two) x1 = *(const double2 *)(rb + g1);
            }
            if (v == fold) x0 = cmul(x0, s_coef[e >> nlo[v]]);
            lds_c128 c;
            c.x = x0.x;
            c.y = x0.y;
            dst[e] = c;
            if (two) {
              if (v == fold) x1 = cmul(x1, s_coef[e1 >> nlo[v]]);
              c.x = x1.x;
              c.y = x1.y;
              dst[e1] = c;
            }
          }
        }
        __syncthreads();
        double2 acc = make_double2(0.0, 0.0);
        if (NV > 1 && fact) {
          // positions 2j and 2j+1 share the last operand's element
#pragma unroll 2
          for (uint32_t k = 0; k < NKAP; k += 2) {
            const double2 inner = mac(k + 1, NV - 2, head(k, NV - 1));
            acc = cfma(inner, opnd(NV - 1, k), acc);
          }
        } else {
#pragma unroll 4
          for (uint32_t k = 0; k < NKAP; ++k) acc = mac(k, NV - 1, acc);
        }
        if (dot) {
          if (SCALE) {
            acc.x = ldexp(acc.x, -sh);
            acc.y = ldexp(acc.y, -sh);
          }
          dot_add(DA, dsv, DS, dsw[row - u * jspan], row, acc);
        } else if (SCALE) {
          wmax = max(wmax, store_scaled(op, of, ((uint64_t)row << 8) | t, acc, sh));
        } else {
          store_g(op, of, ((uint64_t)row << 8) | t, acc, d.range_flag);
        }
      }
    }
    if (dot) {
      dot_end(DA, DS, I.qo, bx, dsw + 32);
      if (SCALE && t == 0 && bx == 0) d.out.E[I.qo] = I.esum;
    } else if (SCALE) {
      const uint32_t m = block_max(wmax, red4);
      if (t == 0) {
        raise_max(d.out.M + (uint64_t)I.qo * kMaxSlots + (bx % kMaxSlots), m);
        if (bx == 0) d.out.E[I.qo] = I.esum;
      }
    }
    __syncthreads();  // s_coef and the stage are rewritten for the next instance
  }
}

template <bool SCALE, int NK, int NV, int NF, bool FOLD>
__global__ __launch_bounds__(256) void step_tiled(const PStep d, uint32_t nb, uint32_t ns,
                                                  uint64_t s_lo, uint32_t jspan) {
  tiled_body<SCALE, NK, NV, NF, FOLD>(d, nb, ns, s_lo, jspan, blockIdx.x, blockIdx.y, gridDim.x, gridDim.y);
}

// Row-paired form (operand 0 carries the coefficient; d.tiled_lds includes
// the second rows' regions; jspan >= 16).
template <bool SCALE, int NK, int NV, int NF>
__global__ __launch_bounds__(256) void step_tiled_pair(const PStep d, uint32_t nb, uint32_t ns,
                                                       uint64_t s_lo, uint32_t jspan) {
  tiled_body<SCALE, NK, NV, NF, true, true>(d, nb, ns, s_lo, jspan, blockIdx.x, blockIdx.y, gridDim.x,
                                            gridDim.y);
}

// Several independent streaming steps in one launch.  The steps of one
// level of the launch graph (no path between any two of them) are often
// each too small to fill the chip; run back to back they leave it idle
// between launches, and on separate streams each join costs a few
// microseconds.  Here each member owns a contiguous range of the launch's
// blocks and runs as its own kernel would, with its block coordinates
// taken from that range.  The member kernels are the common shapes of the
// mid-size steps (LDS-staged: 1 or 2 summed variables and 2 or 3 varying
// operands; direct: 1 summed variable and 2 varying operands; at most one
// operand in the 64-bit form); other steps launch on their own.
constexpr int kMaxMulti = 4;
struct MultiArgs {
  PStep step[kMaxMulti];
  uint32_t n;
  uint32_t vid[kMaxMulti];       // member shape (multi_shape)
  uint32_t blk_end[kMaxMulti];   // cumulative block counts
  uint32_t gx[kMaxMulti];        // the member's x extent (y = blocks / gx)
  uint32_t nb[kMaxMulti], ns[kMaxMulti], jspan[kMaxMulti];
  uint64_t s_lo;
};

// id = ((tiled * 2 + NK - 1) * 2 + NV - 2) * 2 + NF.  The kernel needs the
// registers of its largest member; the streaming shapes with more loads in
// flight (2 summed variables or 3 varying operands) would lower the
// occupancy of all the others and launch on their own.
#define QTN_MULTI_SHAPES(X)                                                                        \
  X(0, 1, 2, 0) X(0, 1, 2, 1) X(1, 1, 2, 0) X(1, 1, 2, 1) X(1, 1, 3, 0) X(1, 1, 3, 1) X(1, 2, 2, 0) \
  X(1, 2, 2, 1) X(1, 2, 3, 0) X(1, 2, 3, 1)

template <bool SCALE>
__global__ __launch_bounds__(256) void step_multi(const MultiArgs args) {
  // the arguments are read in place (the first kernel argument starts the
  // kernel-argument segment): indexing the by-value copy with the member
  // number would make a private copy of all of it
  const MultiArgs &a = *(const MultiArgs *)__builtin_amdgcn_kernarg_segment_ptr();
  (void)args;
  const uint32_t blk = blockIdx.x;
  uint32_t m = 0;
  while (m + 1 < a.n && blk >= a.blk_end[m]) ++m;
  const uint32_t local = blk - (m ? a.blk_end[m - 1] : 0u);
  const uint32_t gx = a.gx[m];
  const uint32_t gy = (a.blk_end[m] - (m ? a.blk_end[m - 1] : 0u)) / gx;
  const uint32_t bx = local % gx, by = local / gx;
  const PStep &d = a.step[m];
  switch (a.vid[m]) {
#define QTN_MULTI_CASE(T, K, V, F)                                                                 \
  case ((T * 2 + K - 1) * 2 + V - 2) * 2 + F:                                                      \
    if constexpr (true) {                                                               \
      if constexpr (T)                                                                             \
        tiled_body<SCALE, K, V, F, true>(d, a.nb[m], a.ns[m], a.s_lo, a.jspan[m], bx, by, gx, gy); \
      else                                                                                         \
        stream_body<SCALE, K, V, F>(d, a.nb[m], a.ns[m], a.s_lo, a.jspan[m], bx, by, gx, gy);      \
    }                                                                                              \
    break;
    QTN_MULTI_SHAPES(QTN_MULTI_CASE)
#undef QTN_MULTI_CASE
    default: break;
  }
}

// Other grid-wide steps: one flat index over (instance, output element).
template <bool SCALE>
__global__ __launch_bounds__(256) void step_small(const PStep d, uint32_t nb, uint32_t ns,
                                                  uint64_t s_lo) {
  const int rC = d.rC;
  const uint64_t total = ((uint64_t)nb * ns) << rC;
  const uint32_t cmask = (1u << rC) - 1u;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t nkap = 1u << d.nk;
  for (uint64_t G = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; G < total; G += stride) {
    const uint64_t q = G >> rC;
    const uint32_t c = (uint32_t)G & cmask;
    InstanceSetup I;
    setup_instance<SCALE>(d, ns, q, s_lo, I);
    uint64_t cidx[kMaxIn];
#pragma unroll
    for (int i = 0; i < kMaxIn; ++i)
      if (i < d.nin) cidx[i] = I.off[i] + cpart(d.in[i], c, rC);
    double2 acc = grid_point(d, cidx, nkap);
    if (SCALE) {
      acc.x = ldexp(acc.x, -I.sh);
      acc.y = ldexp(acc.y, -I.sh);
      uint32_t mb = max_bits(acc, d.out.f64);
      if (rC >= 6) {
        // the 64 lanes of a wave hold one instance (total is a multiple of 64)
        mb = wave_max(mb);
        if ((threadIdx.x & 63) == 0)
          raise_max(d.out.M + (uint64_t)I.qo * kMaxSlots + ((G >> 6) % kMaxSlots), mb);
      } else {
        raise_max(d.out.M + (uint64_t)I.qo * kMaxSlots, mb);
      }
      if (c == 0) d.out.E[I.qo] = I.esum;
    }
    store_g((void *)d.out.base, d.out.f64, I.obase + c, acc, d.range_flag);
  }
}
constexpr int kStreamMinRank = 8;

// ---------------------------------------------------------------------------
// Compensated FP64 slice sum: one block per bitstring, fixed reduction order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <bool SCALE>
__global__ __launch_bounds__(256) void slice_sum(const void *res, uint32_t res64, const int *E,
                                                 uint64_t bstride, uint64_t sstride,
                                                 uint32_t count, double pref,
                                                 qtn_partial *partials, int init,
                                                 qtn_partial *host_out, uint32_t *clear,
                                                 uint64_t nclear, uint64_t keep_lo, uint64_t keep_hi,
                                                 const double2 *dotp, uint64_t dstride, uint32_t dslots,
                                                 uint32_t *flag, uint32_t *flag_out) {
  __shared__ double sre[256], cre[256], sim[256], cim[256];
  const uint32_t b = blockIdx.x;
  const uint32_t t = threadIdx.x;
  double ar = 0, cr = 0, ai = 0, ci = 0;
  auto accumulate = [&](double2 v, uint64_t at) {
    double vr = v.x, vi = v.y;
    if (SCALE) {
      const int e = E[at];
      vr = ldexp(vr, e);
      vi = ldexp(vi, e);
    }
    vr *= pref;
    vi *= pref;
    double s, e2;
    two_sum(ar, vr, s, e2);
    ar = s;
    cr += e2;
    two_sum(ai, vi, s, e2);
    ai = s;
    ci += e2;
  };
  if (dotp && dslots > 16) {
    // many block partials per instance (few instances): the block sums each
    // instance's partials together, in a fixed tree order
    for (uint32_t sl = 0; sl < count; ++sl) {
      const uint64_t at = (uint64_t)b * bstride + (uint64_t)sl * sstride;
      double2 v = make_double2(0.0, 0.0);
      for (uint32_t j = t; j < dslots; j += 256) {
        const double2 w = dotp[at * dstride + j];
        v.x += w.x;
        v.y += w.y;
      }
      sre[t] = v.x;
      sim[t] = v.y;
      __syncthreads();
      for (uint32_t h = 128; h > 0; h >>= 1) {
        if (t < h) {
          sre[t] += sre[t + h];
          sim[t] += sim[t + h];
        }
        __syncthreads();
      }
      if (t == 0) accumulate(make_double2(sre[0], sim[0]), at);
      __syncthreads();
    }
  } else {
    for (uint32_t sl = t; sl < count; sl += 256) {
      const uint64_t at = (uint64_t)b * bstride + (uint64_t)sl * sstride;
      double2 v;
      if (dotp) {
        // block partials of a folded closing chain, summed in slot order
        v = make_double2(0.0, 0.0);
        for (uint32_t j = 0; j < dslots; ++j) {
          const double2 w = dotp[at * dstride + j];
          v.x += w.x;
          v.y += w.y;
        }
      } else {
        v = load_g(res, res64, at);
      }
      accumulate(v, at);
    }
  }
  sre[t] = ar;
  cre[t] = cr;
  sim[t] = ai;
  cim[t] = ci;
  __syncthreads();
  for (uint32_t h = 128; h > 0; h >>= 1) {
    if (t < h) {
      double s, e2;
      two_sum(sre[t], sre[t + h], s, e2);
      sre[t] = s;
      cre[t] = cre[t] + cre[t + h] + e2;
      two_sum(sim[t], sim[t + h], s, e2);
      sim[t] = s;
      cim[t] = cim[t] + cim[t + h] + e2;
    }
    __syncthreads();
  }
  if (t == 0) {
    qtn_partial w;
    w.re = sre[0];
    w.re_comp = cre[0];
    w.im = sim[0];
    w.im_comp = cim[0];
    if (init) {
      partials[b] = w;
    } else {
      qtn_partial a = partials[b];
      double s, e2;
      two_sum(a.re, w.re, s, e2);
      a.re_comp += w.re_comp + e2;
      a.re = s;
      two_sum(a.im, w.im, s, e2);
      a.im_comp += w.im_comp + e2;
      a.im = s;
      partials[b] = a;
      w = a;
    }
    // the last wave also writes the result straight to its destination;
    // block 0 takes the range flag of the whole contraction (to flag_out when
    // given) and clears it for the next one (every earlier kernel has ended)
    if (host_out) {
      host_out[b] = w;
      if (b == 0) {
        const uint32_t f = atomicExch(flag, 0u);
        if (flag_out) *flag_out = f;
      }
    }
  }
  // Clear the exponent words for the next wave, except the result's
  // exponents [keep_lo, keep_hi) that this kernel reads; every other word
  // has been read by its consumer, all of which ran before this launch.
  if (clear)
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + t; i < nclear; i += (uint64_t)gridDim.x * blockDim.x)
      if (i < keep_lo || i >= keep_hi) clear[i] = 0u;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return QTN_EHIP;
}

#define HIP_TRY(call)                                 \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return hip_fail(_e, #call); \
  } while (0)

// Waits for `stream` to drain.  With QTN_SYNC_TIMEOUT_S set to a positive
// number of seconds (read once), the wait polls the stream and gives up with
// QTN_ETIMEOUT after that long, so that work that never completes becomes an
// error naming the call instead of a process that blocks for ever; the work
// itself is left in flight.  Unset or 0: hipStreamSynchronize.
static int wait_stream(hipStream_t stream, const char *what) {
  static const double limit = [] {
    const char *e = std::getenv("QTN_SYNC_TIMEOUT_S");
    return e ? std::atof(e) : 0.0;
  }();
  if (!(limit > 0)) {
    const hipError_t e = hipStreamSynchronize(stream);
    return e == hipSuccess ? QTN_OK : hip_fail(e, what);
  }
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t i = 1;; ++i) {
    const hipError_t q = hipStreamQuery(stream);
    if (q == hipSuccess) return QTN_OK;
    if (q != hipErrorNotReady) return hip_fail(q, what);
    if ((i & 63u) == 0) {
      const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (el > limit) {
        set_error(std::string(what) + ": stream work unfinished after " + std::to_string(limit) +
                  " s (QTN_SYNC_TIMEOUT_S)");
        return QTN_ETIMEOUT;
      }
      std::this_thread::yield();
    }
  }
}

template <typename T>
static int upload(T **dst, const std::vector<T> &src, const char *what) {
  if (*dst) (void)hipFree(*dst);
  *dst = nullptr;
  hipError_t e = hipMalloc((void **)dst, std::max<size_t>(src.size(), 1) * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, what);
  if (!src.empty()) HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return QTN_OK;
}

}  // namespace qtn

using namespace qtn;

static uint32_t tiled_lds_bytes(const PStep &d);
static uint32_t tiled_pair_bytes(const PStep &d);

// Layout and LDS sizes of a binding with S slices per wave (host only).
struct BindShape {
  uint64_t S = 1;
  int mode = MODE_WIDE;
  Layout L;
  int max_slots = 1;
  uint32_t lds_bytes = 0, desc_off = 0, lds_total = 0;
};

static int bind_shape(qtn_plan_t *P, uint64_t S, BindShape &B_) {
  if (S == 0 || S > (1ull << 24)) {
    set_error("slices_per_wave must be in [1, 2^24]");
    return QTN_EINVAL;
  }
  const uint64_t maxS = P->cut.empty() ? 1 : (1ull << P->cut.size());
  if (S > maxS) S = maxS;
  Schedule &sch = P->sched;
  const int mode = choose_mode(P, S);
  const ExecPlan &X = P->exec[mode];
  try {
    B_.L = layout(sch, X, P->net.B, S, wg_slots_for(P, mode, S));
  } catch (const std::exception &e) {
    set_error(e.what());
    return QTN_ESTATE;
  }
  if (!P->cut.empty() && !sch.tensors[sch.result].sdep) {
    set_error("internal: sliced result does not depend on the slice");
    return QTN_ESTATE;
  }
  // LDS of the program kernel: tensors | 256 partial sums | exponent slots | 4 words
  int max_slots = 1;
  for (const Program &pr : X.programs) max_slots = std::max(max_slots, pr.nslots);
  const uint32_t lds_bytes = (X.lds_bytes + 15) & ~15u;
  // ... | program descriptors (LeafStage records, kDescChunk steps)
  uint32_t max_stage = 0;
  for (const Program &pr : X.programs)
    max_stage = std::max<uint32_t>(max_stage, (uint32_t)(pr.staged.size() + pr.staged_global.size()));
  const uint32_t desc_off = (lds_bytes + 256 * 16 + (uint32_t)(2 * max_slots + 4) * 4 + 15) & ~15u;
  const uint32_t desc_bytes = max_stage * (uint32_t)sizeof(LeafStage) + kDescChunk * (uint32_t)sizeof(PStep);
  const uint32_t lds_total = desc_off + desc_bytes;
  if (lds_total > 160 * 1024) {
    set_error("program LDS footprint too large");
    return QTN_ESTATE;
  }
  B_.S = S;
  B_.mode = mode;
  B_.max_slots = max_slots;
  B_.lds_bytes = lds_bytes;
  B_.desc_off = desc_off;
  B_.lds_total = lds_total;
  return QTN_OK;
}

// Gate factors (complex128 in every precision form) as one interleaved
// re/im array, and the element offset of each leaf tensor in it.
static std::vector<double> leaf_host(const qtn_plan_t *P, std::vector<uint64_t> &leaf_elem_off) {
  const Schedule &sch = P->sched;
  leaf_elem_off.assign(sch.tensors.size(), 0);
  uint64_t nleaf = 0;
  for (size_t t = 0; t < sch.tensors.size(); ++t)
    if (sch.tensors[t].leaf) {
      leaf_elem_off[t] = nleaf;
      nleaf += sch.tensors[t].values.size();
    }
  std::vector<double> host(std::max<uint64_t>(nleaf, 1) * 2, 0.0);
  for (size_t t = 0; t < sch.tensors.size(); ++t) {
    const Tensor &T = sch.tensors[t];
    if (!T.leaf) continue;
    for (size_t i = 0; i < T.values.size(); ++i) {
      const uint64_t k = leaf_elem_off[t] + i;
      host[2 * k] = T.values[i].real();
      host[2 * k + 1] = T.values[i].imag();
    }
  }
  return host;
}

static int set_program_lds(uint32_t lds_total) {
  if (lds_total > 64 * 1024) {
    HIP_TRY(hipFuncSetAttribute((const void *)wg_programs<true, 4>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_total));
    HIP_TRY(hipFuncSetAttribute((const void *)wg_programs<false, 4>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_total));
    HIP_TRY(hipFuncSetAttribute((const void *)wg_programs<true, 8>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_total));
    HIP_TRY(hipFuncSetAttribute((const void *)wg_programs<false, 8>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_total));
  }
  return QTN_OK;
}

// Largest operand count among the steps of some programs: the program kernel
// with registers for 4 operands runs them when it is at most 4.
static int programs_max_nin(const Schedule &sch, const ExecPlan &X, const int *progs, size_t n) {
  size_t m = 0;
  for (size_t k = 0; k < n; ++k)
    for (int st : X.programs[progs[k]].steps) m = std::max(m, sch.steps[st].in.size());
  return (int)m;
}

template <bool SCALE>
static void launch_programs(int max_nin, dim3 grid, uint32_t lds_total, hipStream_t stream, const GroupArgs &ga,
                            uint32_t total, uint32_t lds_bytes, int max_slots, uint32_t desc_off) {
  if (max_nin <= 4)
    hipLaunchKernelGGL((wg_programs<SCALE, 4>), grid, dim3(256), lds_total, stream, ga, total, lds_bytes,
                       max_slots, desc_off);
  else
    hipLaunchKernelGGL((wg_programs<SCALE, 8>), grid, dim3(256), lds_total, stream, ga, total, lds_bytes,
                       max_slots, desc_off);
}

static void fill_tables(qtn_plan_t *P, DeviceState *D, const ExecPlan &X, std::vector<char> &blob);

// Per-step costs, operand descriptors and program blobs of a binding whose
// workspace (D->ws), leaf buffer (D->leafbuf) and layout (D->L) are set.
static void fill_tables(qtn_plan_t *P, DeviceState *D, const ExecPlan &X, std::vector<char> &blob) {
  const Schedule &sch = P->sched;
  const uint64_t S = D->L.S;
  const uint64_t B = P->net.B;
  // exponent words exist for every mixed-form plan (a plan whose tensors are
  // all complex128 runs the rescaling kernels when batched with one that is not)
  const bool scaled = P->precision != QTN_FP64;
  // algorithmic bytes and flops of each step, per instance
  D->step_bytes.assign(sch.steps.size(), 0.0);
  D->step_flops.assign(sch.steps.size(), 0.0);
  for (size_t st = 0; st < sch.steps.size(); ++st) {
    const Step &S_ = sch.steps[st];
    double by = std::ldexp((double)elem_bytes(sch.tensors[S_.out]), S_.rC);
    for (int i : S_.in) by += std::ldexp((double)elem_bytes(sch.tensors[i]), sch.tensors[i].rank());
    D->step_bytes[st] = by;
    // complex products per step index point: the varying operands, and one
    // with the kappa coefficient of the uniform operands when there are any
    const uint32_t cbits = S_.rC >= 32 ? ~0u : ((1u << S_.rC) - 1u);
    int nvary = 0;
    for (size_t i = 0; i < S_.in.size(); ++i) nvary += (S_.mask[i] & cbits) ? 1 : 0;
    const int nuni = (int)S_.in.size() - nvary;
    const int nprod = std::max(0, nvary - 1) + (nuni > 0 && nvary > 0 ? 1 : 0);
    D->step_flops[st] = std::ldexp(1.0, S_.nk + S_.rC) * (6.0 * nprod + (S_.nk > 0 ? 2.0 : 0.0));
  }
  if (X.dot_step >= 0) {
    // the folding step reads its operands and writes no output tensor
    const Step &H = sch.steps[X.dot_step];
    D->step_bytes[X.dot_step] -= std::ldexp((double)elem_bytes(sch.tensors[H.out]), H.rC);
    D->step_flops[X.dot_step] += std::ldexp(8.0, H.rC);
  }
  D->prog_bytes.assign(X.programs.size(), 0.0);
  D->prog_flops.assign(X.programs.size(), 0.0);
  for (size_t pi = 0; pi < X.programs.size(); ++pi) {
    std::vector<char> seen(sch.tensors.size(), 0);
    for (int st : X.programs[pi].steps) {
      const Step &S_ = sch.steps[st];
      D->prog_flops[pi] += D->step_flops[st];
      std::vector<int> touched(S_.in.begin(), S_.in.end());
      touched.push_back(S_.out);
      for (int tid : touched) {
        if (seen[tid] || (X.loc[tid] == LOC_LDS && !sch.tensors[tid].leaf)) continue;
        seen[tid] = 1;
        D->prog_bytes[pi] += std::ldexp((double)elem_bytes(sch.tensors[tid]), sch.tensors[tid].rank());
      }
    }
  }
  // operand descriptors
  auto describe = [&](int tid, OpDesc &o) {
    const Tensor &T = sch.tensors[tid];
    std::memset(&o, 0, sizeof(o));
    o.loc = (uint32_t)X.loc[tid];
    o.f64 = T.f64 ? 1u : 0u;
    o.off = (uint32_t)X.off[tid];
    o.slot = X.slot[tid];
    const uint64_t size = 1ull << T.rank();
    if (T.leaf) {
      // staged factors are read from the program's LDS; the source fields
      // stay for the staging list
      o.loc = X.loc[tid] == LOC_LDS ? LOC_LDS : LOC_LEAF;
      o.slot = -1;
      o.f64 = 1;
      o.base = (const double *)D->leafbuf + 2 * D->leaf_elem_off[tid];
      o.selmask = T.selmask;
      o.bstride = T.bdep ? (size << __builtin_popcount(T.selmask)) : 0;
    } else if (o.loc == LOC_GLOBAL) {
      o.base = D->ws + T.data_off;
      o.bstride = T.bdep ? (T.sdep ? S : 1) * size : 0;
      o.sstride = T.sdep ? size : 0;
      if (scaled) {
        o.E = (int *)(D->ws + T.exp_off);
        o.M = (uint32_t *)(D->ws + T.exp_off) + instances(T, B, S);  // kMaxSlots words each
      }
      o.ebstride = T.bdep ? (uint32_t)(T.sdep ? S : 1) : 0;
      o.esstride = T.sdep ? 1 : 0;
    }
  };
  D->steps.assign(sch.steps.size(), PStep{});
  for (size_t st = 0; st < sch.steps.size(); ++st) {
    const Step &S_ = sch.steps[st];
    PStep &d = D->steps[st];
    std::memset(&d, 0, sizeof(d));
    d.range_flag = (uint32_t *)(D->ws + D->L.flag_off);
    d.nin = (int)S_.in.size();
    d.rC = S_.rC;
    d.nk = S_.nk;
    // operands whose index depends on the output element come first
    const uint32_t cbits = (S_.rC >= 32) ? 0xffffffffu : ((1u << S_.rC) - 1u);
    // order: varying 64-bit, varying complex128, then the rest
    std::vector<size_t> ord;
    auto vary = [&](size_t i) { return (S_.mask[i] & cbits) != 0; };
    auto is32 = [&](size_t i) { return !sch.tensors[S_.in[i]].leaf && !sch.tensors[S_.in[i]].f64; };
    for (size_t i = 0; i < S_.in.size(); ++i)
      if (vary(i) && is32(i)) ord.push_back(i);
    d.nf32 = (int)ord.size();
    for (size_t i = 0; i < S_.in.size(); ++i)
      if (vary(i) && !is32(i)) ord.push_back(i);
    for (size_t i = 0; i < S_.in.size(); ++i)
      if (!vary(i)) ord.push_back(i);
    d.nvary = 0;
    for (size_t j = 0; j < ord.size(); ++j) {
      const size_t i = ord[j];
      describe(S_.in[i], d.in[j]);
      d.in[j].mask = S_.mask[i];
      d.nvary += (S_.mask[i] & cbits) ? 1 : 0;
    }
    describe(S_.out, d.out);
    // the first varying operand carrying every summed bit takes the
    // coefficient of the uniform operands (only operand 0, so that the
    // product chain starts from it)
    d.tiled_fold = (d.nk > 0 && d.nin > d.nvary &&
                    __builtin_popcount(S_.rC >= 32 ? 0u : (d.in[0].mask >> S_.rC)) == d.nk) ? 0 : -1;
    d.tiled_lds = tiled_lds_bytes(d);
    d.tiled_pair = tiled_pair_bytes(d);
  }
  // program blobs: LeafStage records, then PStep descriptors
  blob.clear();
  D->blob_off.assign(X.programs.size(), 0);
  for (size_t pi = 0; pi < X.programs.size(); ++pi) {
    const Program &pr = X.programs[pi];
    D->blob_off[pi] = blob.size();
    for (int tid : pr.staged) {
      const Tensor &T = sch.tensors[tid];
      OpDesc o;
      describe(tid, o);
      LeafStage ls;
      std::memset(&ls, 0, sizeof(ls));
      ls.base = o.base;
      ls.bstride = o.bstride;
      ls.selmask = o.selmask;
      ls.count = 1u << T.rank();
      ls.lds_off = (uint32_t)(X.off[tid] / 16);
      ls.slot = -1;
      ls.f64 = 1;
      const char *pb = (const char *)&ls;
      blob.insert(blob.end(), pb, pb + sizeof(ls));
    }
    for (const Program::StagedGlobal &g : pr.staged_global) {
      const Tensor &T = sch.tensors[g.tensor];
      OpDesc o;
      describe(g.tensor, o);
      LeafStage ls;
      std::memset(&ls, 0, sizeof(ls));
      ls.base = o.base;
      ls.bstride = o.bstride;
      ls.sstride = o.sstride;
      ls.E = o.E;
      ls.ebstride = o.ebstride;
      ls.esstride = o.esstride;
      ls.count = 1u << T.rank();
      ls.lds_off = (uint32_t)(g.off / 16);
      ls.slot = (int16_t)g.slot;
      ls.f64 = o.f64;
      ls.global = 1;
      const char *pb = (const char *)&ls;
      blob.insert(blob.end(), pb, pb + sizeof(ls));
    }
    for (int st : pr.steps) {
      PStep ps = D->steps[st];
      // operands staged from the workspace are read from the program's LDS
      for (int i = 0; i < ps.nin; ++i)
        for (const Program::StagedGlobal &g : pr.staged_global)
          if (ps.in[i].loc == LOC_GLOBAL &&
              ps.in[i].base == (const void *)(D->ws + sch.tensors[g.tensor].data_off)) {
            ps.in[i].loc = LOC_LDS;
            ps.in[i].off = (uint32_t)g.off;
            ps.in[i].slot = (int16_t)g.slot;
            ps.in[i].f64 = 1;
          }
      bool lds_only = true;
      for (int i = 0; i < ps.nin; ++i) lds_only = lds_only && ps.in[i].loc == LOC_LDS;
      ps.wg_flags = lds_only ? 1u : 0u;
      const char *pb = (const char *)&ps;
      blob.insert(blob.end(), pb, pb + sizeof(PStep));
    }
  }
  // the folded closing chain: its gate factors, lane-only first, then
  // row-only, then mixed, and the block partials' place in the workspace
  D->dot_args_off = 0;
  if (X.dot_step >= 0) {
    DotArgs A;
    std::memset(&A, 0, sizeof(A));
    std::vector<size_t> ord;
    for (int cls = 0; cls < 3; ++cls)
      for (size_t j = 0; j < X.dot_leaves.size(); ++j) {
        const uint32_t m = X.dot_masks[j];
        const int c = (m >> 8) == 0 ? 0 : ((m & 255u) == 0 ? 1 : 2);
        if (c == cls) ord.push_back(j);
      }
    uint32_t off = 0;
    for (size_t j : ord) {
      const uint32_t m = X.dot_masks[j];
      const Tensor &T = sch.tensors[X.dot_leaves[j]];
      for (uint32_t v = 0; v < (1u << T.rank()) && off + v < kDotValues; ++v) A.owner[off + v] = (uint8_t)A.nleaf;
      DotLeaf &L = A.leaf[A.nleaf++];
      L.base = (const double *)D->leafbuf + 2 * D->leaf_elem_off[X.dot_leaves[j]];
      L.rank = (uint32_t)T.rank();
      L.bstride = T.bdep ? ((uint64_t)1 << (T.rank() + __builtin_popcount(T.selmask))) : 0;
      L.selmask = T.selmask;
      L.mask = m;
      L.off = off;
      off += 1u << T.rank();
      if ((m >> 8) == 0)
        ++A.nlo;
      else if ((m & 255u) == 0)
        ++A.nhi;
      else
        ++A.nmix;
    }
    A.nvals = off;
    A.slots = (uint32_t)D->L.dot_slots;
    A.part = (double2 *)(D->ws + D->L.dot_off);
    if (A.nvals > kDotValues) throw std::runtime_error("folded closing chain: too many factor values");
    while (blob.size() % 256) blob.push_back(0);
    D->dot_args_off = blob.size();
    const char *pa = (const char *)&A;
    blob.insert(blob.end(), pa, pa + sizeof(A));
    PStep &h = D->steps[X.dot_step];
    h.dot = 1;
    h.dot_lds = (uint32_t)sizeof(DotArgs) + (A.nvals + 32 + 4) * 16u;
  }
}

extern "C" int qtn_plan_bind_workspace(qtn_plan_t *P, void *dev_ptr, uint64_t bytes,
                                       uint64_t S_req) {
  set_error("");
  if (!P || !dev_ptr) {
    set_error("NULL argument");
    return QTN_EINVAL;
  }
  if (((uintptr_t)dev_ptr) & 255u) {
    set_error("workspace must be 256-byte aligned");
    return QTN_EINVAL;
  }
  BindShape shape;
  if (int rc = bind_shape(P, S_req, shape)) return rc;
  const int mode = shape.mode;
  const Layout &L = shape.L;
  const ExecPlan &X = P->exec[mode];
  Schedule &sch = P->sched;
  if (bytes < L.total_bytes) {
    set_error("workspace too small: need " + std::to_string(L.total_bytes) + " bytes");
    return QTN_ENOMEM;
  }
  const int max_slots = shape.max_slots;
  const uint32_t lds_bytes = shape.lds_bytes, desc_off = shape.desc_off, lds_total = shape.lds_total;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceState *D = P->dev;
  if (!D || D->device != dev) {
    device_state_free(D);
    D = new DeviceState();
    P->dev = D;
    D->device = dev;
    // gate factors stay complex128 in every precision form
    const std::vector<double> host = leaf_host(P, D->leaf_elem_off);
    double *lb = nullptr;
    if (int rc = upload(&lb, host, "hipMalloc(leaves)")) return rc;
    D->leafbuf = lb;
    // pinned host memory the slice sum writes the final partials to
    HIP_TRY(hipHostMalloc((void **)&D->host_partials, (P->net.B + 1) * sizeof(qtn_partial),
                          hipHostMallocMapped));
    HIP_TRY(hipHostGetDevicePointer((void **)&D->host_partials_dev, D->host_partials, 0));
    D->flag_dev = (uint32_t *)(D->host_partials_dev + P->net.B);
    static const bool rescale_always = [] {
      const char *e = std::getenv("QTN_RESCALE");  // tuning switch: 1 rescales every contraction
      return e && e[0] == '1';
    }();
    D->unscaled = !rescale_always;
  }
  if (int rc = set_program_lds(lds_total)) return rc;
  LaunchGraph lg;
  try {
    static const int env_streams = [] {
      const char *e = std::getenv("QTN_STREAMS");  // tuning switch: 1 serialises every launch
      return e ? std::max(1, std::min(1 + DeviceState::kSide, std::atoi(e))) : 1 + DeviceState::kSide;
    }();
    lg = launch_graph(sch, X, L, P->net.B, L.S, P->precision != QTN_FP64, env_streams);
  } catch (const std::exception &e) {
    set_error(e.what());
    return QTN_ESTATE;
  }
  for (int k = 0; k + 1 < lg.nstreams; ++k) {
    if (!D->side[k]) HIP_TRY(hipStreamCreateWithFlags(&D->side[k], hipStreamNonBlocking));
    if (!D->join_ev[k]) HIP_TRY(hipEventCreateWithFlags(&D->join_ev[k], hipEventDisableTiming));
  }
  if (!D->fork_ev) HIP_TRY(hipEventCreateWithFlags(&D->fork_ev, hipEventDisableTiming));
  while (D->unit_ev.size() < lg.deps.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    D->unit_ev.push_back(e);
  }
  static const bool env_levels = [] {
    const char *e = std::getenv("QTN_LEVELS");  // tuning switch: 0 uses side streams
    return !(e && e[0] == '0');
  }();
  drop_graph(D);
  D->lg = lg;
  D->levels = env_levels;
  D->mode = mode;
  D->ws = (char *)dev_ptr;
  D->ws_bytes = bytes;
  // the exponent words start cleared; the slice sum clears them after each wave
  if (P->precision != QTN_FP64 && L.exp_bytes) HIP_TRY(hipMemset(D->ws + L.data_bytes, 0, L.exp_bytes));
  HIP_TRY(hipMemset(D->ws + L.flag_off, 0, 4));   // the range word
  D->L = L;
  D->max_slots = max_slots;
  D->lds_bytes = lds_bytes;
  D->lds_total = lds_total;
  D->desc_bytes = desc_off;
  std::vector<char> blob;
  fill_tables(P, D, X, blob);
  if (blob.size() > 0xffffffffull) {
    set_error("program descriptors too large");
    return QTN_ESTATE;
  }
  if (int rc = upload(&D->blobbuf, blob, "hipMalloc(program descriptors)")) return rc;
  return QTN_OK;
}

// LDS bytes of step_tiled for this step, or 0 when staging does not pay:
// the rows must be whole, every varying operand in global memory, the staged
// runs at most a third of the direct loads and small enough for several
// blocks per compute unit.
static uint32_t tiled_lds_bytes(const PStep &d) {
  static const bool enabled = [] {
    const char *e = std::getenv("QTN_TILED");  // tuning switch: 0 keeps step_stream
    return !(e && e[0] == '0');
  }();
  if (!enabled || d.rC < 8 || d.nk > 4 || d.nvary < 1 || d.nvary > 4) return 0;
  uint64_t staged = 0, bytes = 0;
  for (int v = 0; v < d.nvary; ++v) {
    const OpDesc &in = d.in[v];
    if (in.loc != LOC_GLOBAL && in.loc != LOC_LEAF) return 0;
    const uint32_t cb = d.rC >= 32 ? ~0u : ((1u << d.rC) - 1u);
    const uint64_t n = 1ull << (__builtin_popcount(d.rC >= 32 ? 0u : (in.mask >> d.rC)) +
                                __builtin_popcount(in.mask & cb & 255u));
    // byte offsets within one operand instance are computed in 32 bits
    if ((uint64_t)(v < d.nf32 ? 8u : 16u) << __builtin_popcount(in.mask) >= (1ull << 31)) return 0;
    staged += n;
    bytes += n * 16u;   // staged as complex128
  }
  const uint64_t direct = (uint64_t)d.nvary * 256u << d.nk;
  if (3 * staged > direct || bytes > 48 * 1024) return 0;
  return (uint32_t)bytes;
}

// Extra LDS bytes of the row-paired form of a staged step (the second row's
// runs of operands 1..nvary-1), or 0 when it does not apply: the step must
// fold the coefficient into operand 0, sum at least 3 variables (the kappa
// loop dominates) over at least two varying operands, and operand 0 must
// lack the innermost row bit of the visiting order, so that the two rows
// share its runs.  QTN_PAIR=0 switches it off.
static uint32_t tiled_pair_bytes(const PStep &d) {
  static const bool enabled = [] {
    const char *e = std::getenv("QTN_PAIR");  // tuning switch
    return !(e && e[0] == '0');
  }();
  if (!enabled || !d.tiled_lds || d.tiled_fold != 0 || d.nk < 3 || d.nvary < 2) return 0;
  const uint32_t cb = d.rC >= 32 ? ~0u : ((1u << d.rC) - 1u);
  const uint32_t pb = tiled_row_order(d) & 3u;
  if ((((d.in[0].mask & cb) >> 8) >> pb) & 1u) return 0;
  uint32_t extra = 0;
  for (int v = 1; v < d.nvary; ++v) {
    const OpDesc &in = d.in[v];
    extra += (1u << (__builtin_popcount(in.mask >> d.rC) + __builtin_popcount(in.mask & cb & 255u))) * 16u;
  }
  if (d.tiled_lds + extra > 64 * 1024) return 0;
  return extra;
}

template <bool SCALE, int NK, int NV>
static void launch_stream_nv(const PStep &d, dim3 grid, hipStream_t stream, uint32_t nb, uint32_t ns,
                             uint64_t s_lo, uint32_t jspan) {
  // the row-paired form of staged steps that allow it (rows in 16-row chunks)
  if constexpr (NK >= 3 && NV >= 2) {
    if (d.tiled_lds && d.tiled_pair && d.tiled_fold == 0 && jspan >= 16) {
      PStep dp = d;
      dp.tiled_lds = d.tiled_lds + d.tiled_pair;
      switch (d.nf32) {
#define QTN_NFP(F)                                                                                 \
  case F:                                                                                          \
    if constexpr (F <= NV) {                                                  \
      hipLaunchKernelGGL((step_tiled_pair<SCALE, NK, NV, (F <= NV ? F : 0)>), grid, dim3(256),     \
                         dp.tiled_lds + dp.dot_lds, stream, dp, nb, ns, s_lo, jspan);              \
      return;                                                                                      \
    }                                                                                              \
    break;
        QTN_NFP(0) QTN_NFP(1) QTN_NFP(2) QTN_NFP(3) QTN_NFP(4)
#undef QTN_NFP
        default: break;
      }
    }
  }
  // NF = number of 64-bit-form operands among the NV varying ones
  switch (d.nf32) {
#define QTN_NF(F)                                                                                  \
  case F:                                                                                          \
    if constexpr (F <= NV)        \
    {                                                                                              \
      if (d.tiled_lds && d.tiled_fold == 0)                                                        \
        hipLaunchKernelGGL((step_tiled<SCALE, NK, NV, (F <= NV ? F : 0), true>), grid, dim3(256),  \
                           d.tiled_lds + d.dot_lds, stream, d, nb, ns, s_lo, jspan);               \
      else if (d.tiled_lds)                                                                        \
        hipLaunchKernelGGL((step_tiled<SCALE, NK, NV, (F <= NV ? F : 0), false>), grid, dim3(256), \
                           d.tiled_lds + d.dot_lds, stream, d, nb, ns, s_lo, jspan);               \
      else                                                                                         \
        hipLaunchKernelGGL((step_stream<SCALE, NK, NV, (F <= NV ? F : 0)>), grid, dim3(256),       \
                           d.dot_lds, stream, d, nb, ns, s_lo, jspan);                             \
    }                                                                                              \
    break;
    QTN_NF(0) QTN_NF(1) QTN_NF(2) QTN_NF(3) QTN_NF(4)
#undef QTN_NF
    default: break;
  }
}

template <bool SCALE, int NK>
static void launch_stream_nk(const PStep &d, dim3 grid, hipStream_t stream, uint32_t nb, uint32_t ns,
                             uint64_t s_lo, uint32_t jspan) {
  switch (d.nvary) {
    case 1: launch_stream_nv<SCALE, NK, 1>(d, grid, stream, nb, ns, s_lo, jspan); break;
    case 2: launch_stream_nv<SCALE, NK, 2>(d, grid, stream, nb, ns, s_lo, jspan); break;
    case 3: launch_stream_nv<SCALE, NK, 3>(d, grid, stream, nb, ns, s_lo, jspan); break;
    default: launch_stream_nv<SCALE, NK, 4>(d, grid, stream, nb, ns, s_lo, jspan); break;
  }
}

template <bool SCALE>
static void launch_stream(const PStep &d, dim3 grid, hipStream_t stream, uint32_t nb, uint32_t ns,
                          uint64_t s_lo, uint32_t jspan) {
  switch (d.nk) {
    case 0: launch_stream_nk<SCALE, 0>(d, grid, stream, nb, ns, s_lo, jspan); break;
    case 1: launch_stream_nk<SCALE, 1>(d, grid, stream, nb, ns, s_lo, jspan); break;
    case 2: launch_stream_nk<SCALE, 2>(d, grid, stream, nb, ns, s_lo, jspan); break;
    case 3: launch_stream_nk<SCALE, 3>(d, grid, stream, nb, ns, s_lo, jspan); break;
    default: launch_stream_nk<SCALE, 4>(d, grid, stream, nb, ns, s_lo, jspan); break;
  }
}

// Grid of a streaming step over Q instances: units of jspan rows of 256
// elements (jspan <= 32), about `target` blocks in all.
static dim3 stream_grid(const PStep &d, uint64_t Q, uint64_t target, uint32_t *jspan_out) {
  const uint32_t rows = (1u << d.rC) >> 8;
  uint32_t jspan = 32;
  while (jspan > 1 && (uint64_t)(rows / jspan) * Q < target) jspan >>= 1;
  const uint64_t units = rows / jspan;
  const uint64_t want = std::max<uint64_t>(1, 2 * target / std::max<uint64_t>(Q, 1));
  *jspan_out = jspan;
  return dim3((unsigned)std::min<uint64_t>(units, want), (unsigned)std::min<uint64_t>(Q, 65535));
}

// Shape id of a step that step_multi can run (QTN_MULTI_SHAPES), or -1.
static int multi_shape(const PStep &d, bool scale, bool stream_only) {
  const bool streaming = d.rC >= kStreamMinRank && d.nk <= 4 && d.nvary >= 1 && d.nvary <= 4;
  if (!streaming || d.dot) return -1;
  const bool tiled = d.tiled_lds != 0 && !stream_only;
  if (tiled && d.tiled_fold != 0) return -1;
  if (d.nk < 1 || d.nk > 2 || d.nvary < 2 || d.nvary > 3 || d.nf32 > 1) return -1;
  if (!tiled && (d.nk != 1 || d.nvary != 2)) return -1;
  return (((tiled ? 1 : 0) * 2 + d.nk - 1) * 2 + d.nvary - 2) * 2 + d.nf32;
}

// Blocks per member of a shared launch: QTN_MULTI_TARGET, else half the
// step's own target (on the n=120 levels of 2 to 4 steps: 512 per member
// 0.244 ms per contraction, 1024 0.254, 256 0.260, 2048 0.283).
static uint64_t multi_target(const StepTune &tu) {
  static const long env = [] {
    const char *e = std::getenv("QTN_MULTI_TARGET");  // tuning switch
    return e ? std::atol(e) : 0L;
  }();
  return env > 0 ? (uint64_t)env : std::max<uint64_t>(64, tu.target / 2);
}

// One step_multi launch of the launch units units[0..n) (grid-wide steps of
// one level, each with a multi_shape).
template <bool SCALE>
static int launch_multi(const qtn_plan_t *P, const DeviceState *D, const int *units, size_t n,
                        hipStream_t stream, uint64_t s_lo, uint64_t cnt) {
  const ExecPlan &X = P->exec[D->mode];
  const Schedule &sch = P->sched;
  MultiArgs a;
  std::memset(&a, 0, sizeof a);
  a.n = (uint32_t)n;
  a.s_lo = s_lo;
  uint64_t blocks = 0;
  uint32_t lds = 0;
  for (size_t i = 0; i < n; ++i) {
    const int st = X.launches[(size_t)(units[i] - 1)].step;
    const StepTune tu = D->tune.empty() ? StepTune() : D->tune[st];
    PStep d = D->steps[st];
    if (tu.stream_only) d.tiled_lds = 0;
    const int vid = multi_shape(d, SCALE, false);
    if (vid < 0) {
      set_error("internal: step without a shared-launch shape");
      return QTN_ESTATE;
    }
    const uint32_t nb = sch.steps[st].bdep ? (uint32_t)P->net.B : 1;
    const uint32_t ns = sch.steps[st].sdep ? (uint32_t)cnt : 1;
    uint32_t jspan = 1;
    const dim3 g = stream_grid(d, (uint64_t)nb * ns, multi_target(tu), &jspan);
    a.step[i] = d;
    a.vid[i] = (uint32_t)vid;
    a.gx[i] = g.x;
    a.nb[i] = nb;
    a.ns[i] = ns;
    a.jspan[i] = jspan;
    blocks += (uint64_t)g.x * g.y;
    a.blk_end[i] = (uint32_t)blocks;
    lds = std::max(lds, d.tiled_lds);
  }
  if (blocks == 0 || blocks > 0x7fffffffull) {
    set_error("internal: shared launch size");
    return QTN_ESTATE;
  }
  hipLaunchKernelGGL((step_multi<SCALE>), dim3((unsigned)blocks), dim3(256), lds, stream, a);
  return QTN_OK;
}

// Launches grid-wide step `st` for the wave of `cnt` slices starting at
// s_lo.  Streaming steps: units of jspan x 256 elements, about tu.target
// blocks over the chip, each walking up to 32 rows, so that the per-block
// set-up (index tables, instance offsets and kappa coefficients, a chain of
// dependent loads) is paid once per up to 8192 outputs; the default of 1024
// (4 per compute unit) was measured best on the n=120 steps (2048 to 8192 up
// to 3x slower for the direct kernels, 256 slower, 512 about even), and
// qtn_plan_autotune measures the alternatives per step.  A folding step
// reports its grid.x (the partial slots the slice sum reads) in *dot_gx.
template <bool SCALE>
static int launch_grid_step(const qtn_plan_t *P, const DeviceState *D, int st, hipStream_t stream, uint64_t s_lo,
                            uint64_t cnt, const StepTune &tu, uint32_t *dot_gx) {
  const Schedule &sch = P->sched;
  const uint64_t B = P->net.B;
  PStep d = D->steps[st];
  if (d.dot) d.dotp = D->blobbuf + D->dot_args_off;
  if (tu.stream_only) d.tiled_lds = 0;
  if (!tu.pair) d.tiled_pair = 0;   // the row-paired form only where tuned in
  const uint32_t nb = sch.steps[st].bdep ? (uint32_t)B : 1;
  const uint32_t ns = sch.steps[st].sdep ? (uint32_t)cnt : 1;
  const uint64_t Q = (uint64_t)nb * ns;
  const bool streaming = d.rC >= kStreamMinRank && d.nk <= 4 && d.nvary >= 1 && d.nvary <= 4;
  if (d.dot && !streaming) {
    set_error("internal: the folded closing chain sits on a step that does not stream");
    return QTN_ESTATE;
  }
  if (streaming) {
    uint32_t jspan = 1;
    const dim3 grid = stream_grid(d, Q, tu.target, &jspan);
    if (d.dot && dot_gx) *dot_gx = grid.x;
    launch_stream<SCALE>(d, grid, stream, nb, ns, s_lo, jspan);
  } else {
    const uint64_t total = Q << d.rC;
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((total + 255) / 256, 16384));
    hipLaunchKernelGGL((step_small<SCALE>), dim3(blocks), dim3(256), 0, stream, d, nb, ns, s_lo);
  }
  return QTN_OK;
}

template <bool SCALE>
static int run_waves(qtn_plan_t *P, DeviceState *D, uint64_t lo, uint64_t hi, hipStream_t stream,
                     bool concurrent) {
  const Schedule &sch = P->sched;
  const ExecPlan &X = P->exec[D->mode];
  const uint64_t S = D->L.S;
  const uint64_t B = P->net.B;
  qtn_partial *partials = (qtn_partial *)(D->ws + D->L.partial_off);
  // the slice sum reads the result tensor, or with a folded closing chain the
  // block partials and exponents of the folding step's output
  const bool folded = X.dot_step >= 0;
  const Tensor &res = sch.tensors[folded ? X.dot_tensor : sch.result];
  uint32_t dot_gx = 0;
  const uint64_t scratch_stride = (X.scratch_per_wg + 255) & ~uint64_t(255);
  bool first = true;
  const LaunchGraph &lg = D->lg;
  // Without timing, the launch units run level by level on `stream`, the
  // eligible steps of one level in shared launches (step_multi).  With
  // QTN_LEVELS=0, side streams are used instead while a graph is being
  // captured (the graph then holds the launch graph's edges).  Any launch
  // sequence with timing on runs on `stream` in the enqueue order.
  const bool levels = D->levels && !D->timing && lg.nlevels > 0;
  const bool multi = !levels && concurrent && lg.nstreams > 1 && !D->timing;
  auto unit_stream = [&](int u) {
    return (!multi || lg.stream[u] == 0) ? stream : D->side[lg.stream[u] - 1];
  };
  for (uint64_t s_lo = lo; s_lo < hi; s_lo += S) {
    const uint64_t cnt = std::min<uint64_t>(S, hi - s_lo);
    const int U = (int)lg.deps.size();
    auto launch_unit = [&](int u, hipStream_t stream) -> int {
      if (u == 0) {
        // exponents were cleared at bind time or by the previous slice sum
      } else if (u == U - 1) {
        const uint64_t rb = res.bdep ? (res.sdep ? S : 1) : 0, rs = res.sdep ? 1 : 0;
        hipLaunchKernelGGL((slice_sum<SCALE>), dim3((unsigned)B), dim3(256), 0, stream,
                           (const void *)(D->ws + res.data_off), res.f64 ? 1u : 0u,
                           (const int *)(D->ws + res.exp_off), rb, rs, (uint32_t)cnt,
                           P->net.prefactor, partials, first ? 1 : 0,
                           s_lo + S >= hi ? D->host_partials_dev : (qtn_partial *)nullptr,
                           (SCALE && D->L.exp_bytes) ? (uint32_t *)(D->ws + D->L.data_bytes) : (uint32_t *)nullptr,
                           D->L.exp_bytes / 4, SCALE ? (res.exp_off - D->L.data_bytes) / 4 : 0,
                           SCALE ? (res.exp_off - D->L.data_bytes) / 4 + instances(res, B, S) : 0,
                           folded ? (const double2 *)(D->ws + D->L.dot_off) : (const double2 *)nullptr,
                           (uint64_t)D->L.dot_slots, dot_gx, (uint32_t *)(D->ws + D->L.flag_off),
                           s_lo + S >= hi ? D->flag_dev : (uint32_t *)nullptr);
        first = false;
      } else {
        const size_t g = (size_t)(u - 1);
        const LaunchGroup &G = X.launches[g];
        if (G.kind == 0) {
          const bool timed = D->timing;
          double tb = 0, tf = 0;
          if (timed) {
            if (D->ev_used + 2 > D->ev.size()) {
              for (int j = 0; j < 64; ++j) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                D->ev.push_back(e);
              }
            }
            HIP_TRY(hipEventRecord(D->ev[D->ev_used], stream));
          }
          // at most kMaxGroupProgs programs per launch
          for (size_t p0 = 0; p0 < G.programs.size(); p0 += kMaxGroupProgs) {
            GroupArgs ga;
            std::memset(&ga, 0, sizeof(ga));
            uint64_t total = 0;
            for (size_t k = p0; k < G.programs.size() && k < p0 + kMaxGroupProgs; ++k) {
              const Program &pr = X.programs[G.programs[k]];
              const uint32_t j = ga.nprog++;
              const uint64_t items = (pr.bdep ? B : 1) * (pr.sdep ? cnt : 1);
              total += items;
              tb += (double)items * D->prog_bytes[G.programs[k]];
              tf += (double)items * D->prog_flops[G.programs[k]];
              ga.item_end[j] = (uint32_t)total;
              ga.nsteps[j] = (uint16_t)pr.steps.size();
              ga.nstage[j] = (uint16_t)(pr.staged.size() + pr.staged_global.size());
              ga.bdep[j] = pr.bdep ? 1 : 0;
              ga.sdep[j] = pr.sdep ? 1 : 0;
              ga.ns[j] = (uint32_t)cnt;
              ga.blob[j] = D->blobbuf + D->blob_off[G.programs[k]];
              ga.scratch[j] = D->ws + D->L.scratch_off;
              ga.scratch_stride[j] = scratch_stride;
              ga.s_lo[j] = s_lo;
            }
            const uint64_t cap = D->mode == MODE_SLICE ? D->L.wg_slots : 2048;
            const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(total, cap));
            const size_t np = std::min<size_t>(G.programs.size() - p0, (size_t)kMaxGroupProgs);
            launch_programs<SCALE>(programs_max_nin(sch, X, G.programs.data() + p0, np), dim3((unsigned)grid),
                                   D->lds_total, stream, ga, (uint32_t)total, D->lds_bytes, D->max_slots,
                                   D->desc_bytes);
          }
          if (timed) {
            HIP_TRY(hipEventRecord(D->ev[D->ev_used + 1], stream));
            D->ev_used += 2;
            D->ev_bytes.push_back(tb);
            D->ev_flops.push_back(tf);
            D->ev_step.push_back(-1);
          }
        } else {
          const int st = G.step;
          const uint32_t nb = sch.steps[st].bdep ? (uint32_t)B : 1;
          const uint32_t ns = sch.steps[st].sdep ? (uint32_t)cnt : 1;
          const uint64_t Q = (uint64_t)nb * ns;
          const PStep &d0 = D->steps[st];
          const bool streaming = d0.rC >= kStreamMinRank && d0.nk <= 4 && d0.nvary >= 1 && d0.nvary <= 4;
          const bool timed = D->timing && streaming;
          if (timed) {
            if (D->ev_used + 2 > D->ev.size()) {
              for (int j = 0; j < 64; ++j) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                D->ev.push_back(e);
              }
            }
            HIP_TRY(hipEventRecord(D->ev[D->ev_used], stream));
          }
          const StepTune tu = D->tune.empty() ? StepTune() : D->tune[st];
          if (int rc = launch_grid_step<SCALE>(P, D, st, stream, s_lo, cnt, tu, &dot_gx)) return rc;
          if (timed) {
            HIP_TRY(hipEventRecord(D->ev[D->ev_used + 1], stream));
            D->ev_used += 2;
            D->ev_bytes.push_back((double)Q * D->step_bytes[st]);
            D->ev_flops.push_back((double)Q * D->step_flops[st]);
            D->ev_step.push_back(st);
          }
        }
      }
      return QTN_OK;
    };
    if (levels) {
      std::vector<int> grp;
      for (int lv = 0; lv < lg.nlevels; ++lv) {
        grp.clear();
        for (int u = 1; u + 1 < U; ++u) {
          if (lg.level[u] != lv) continue;
          const LaunchGroup &G = X.launches[(size_t)(u - 1)];
          const StepTune tu = (G.kind == 1 && !D->tune.empty()) ? D->tune[G.step] : StepTune();
          if (G.kind == 1 && multi_shape(D->steps[G.step], SCALE, tu.stream_only) >= 0)
            grp.push_back(u);
          else if (int rc = launch_unit(u, stream))
            return rc;
        }
        for (size_t i = 0; i < grp.size(); i += kMaxMulti) {
          const size_t n = std::min<size_t>(grp.size() - i, kMaxMulti);
          if (n == 1) {
            if (int rc = launch_unit(grp[i], stream)) return rc;
          } else if (int rc = launch_multi<SCALE>(P, D, &grp[i], n, stream, s_lo, cnt)) {
            return rc;
          }
        }
      }
      if (int rc = launch_unit(U - 1, stream)) return rc;   // the slice sum
      continue;
    }
    if (multi) {
      // side streams start after everything before this wave
      HIP_TRY(hipEventRecord(D->fork_ev, stream));
      for (int k = 0; k + 1 < lg.nstreams; ++k) HIP_TRY(hipStreamWaitEvent(D->side[k], D->fork_ev, 0));
    }
    for (int ui = 0; ui < U; ++ui) {
      // timing keeps the schedule order on one stream
      const int u = multi ? lg.order[ui] : ui;
      const hipStream_t ustream = unit_stream(u);
      if (multi)
        for (int d : lg.deps[u])
          if (lg.stream[d] != lg.stream[u]) HIP_TRY(hipStreamWaitEvent(ustream, D->unit_ev[d], 0));
      if (int rc = launch_unit(u, ustream)) return rc;
      if (multi && lg.record[u]) HIP_TRY(hipEventRecord(D->unit_ev[u], ustream));
    }
    if (multi) {
      for (int k = 0; k + 1 < lg.nstreams; ++k) {
        HIP_TRY(hipEventRecord(D->join_ev[k], D->side[k]));
        HIP_TRY(hipStreamWaitEvent(stream, D->join_ev[k], 0));
      }
    }
  }
  HIP_TRY(hipGetLastError());
  return QTN_OK;
}

// Whether a contraction of this plan runs the rescaling kernels: plans that
// store tensors in the 64-bit form rescale in asynchronous calls (whose
// results cannot be checked before they are used), in the re-run of a
// synchronous call that left the form's exponent range, and once that has
// happened twice in a row; otherwise synchronous calls run without
// rescaling (the workspace's range word guards them).
static bool scaled_run(const qtn_plan_t *P, const DeviceState *D, bool async) {
  return P->scaled[D->mode] && (async || !D->unscaled || D->force_scaled);
}

static int contract_impl(qtn_plan_t *P, uint64_t lo, uint64_t hi, void *stream_v,
                         qtn_partial *out, bool async) {
  set_error("");
  if (!P || !out) {
    set_error("NULL argument");
    return QTN_EINVAL;
  }
  const uint64_t nslices = 1ull << P->cut.size();
  if (lo > hi || hi > nslices) {
    set_error("slice range outside [0, 2^k)");
    return QTN_ERANGE;
  }
  const uint64_t B = P->net.B;
  if (lo == hi) {
    for (uint64_t b = 0; b < B; ++b) out[b] = qtn_partial{0.0, 0.0, 0.0, 0.0};
    return QTN_OK;
  }
  if (!P->dev || !P->dev->ws) {
    set_error("no workspace bound");
    return QTN_ENOMEM;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != P->dev->device) {
    set_error("plan bound on another device");
    return QTN_ESTATE;
  }
  hipStream_t stream = (hipStream_t)stream_v;
  DeviceState *D = P->dev;
  if (async && D->timing) {
    set_error("timing reads its events when the call returns; use qtn_contract");
    return QTN_ESTATE;
  }
  if (D->timing) {
    // events are created before any capture begins: two per timed launch
    const ExecPlan &X = P->exec[D->mode];
    const uint64_t waves = (hi - lo + D->L.S - 1) / D->L.S;
    const size_t need = (size_t)(2 * waves * X.launches.size());
    while (D->ev.size() < need) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      // an event is recorded once outside any capture; events whose first
      // record is a graph node cannot be read back afterwards
      HIP_TRY(hipEventRecord(e, stream));
      D->ev.push_back(e);
    }
  }
  const bool sc = scaled_run(P, D, async);
  auto enqueue = [&](hipStream_t st, bool concurrent) {
    return !sc ? run_waves<false>(P, D, lo, hi, st, concurrent) : run_waves<true>(P, D, lo, hi, st, concurrent);
  };
  if (D->use_graphs) {
    // The launch sequence of [lo, hi) is captured once on an internal stream
    // and replayed on the caller's stream while it matches.
    if (!D->gstream) {
      HIP_TRY(hipStreamCreateWithFlags(&D->gstream, hipStreamNonBlocking));
    }
    if (!D->gexec || D->g_lo != lo || D->g_hi != hi || D->g_timing != D->timing || D->g_scaled != sc) {
      drop_graph(D);
      D->ev_used = 0;
      D->ev_bytes.clear();
      D->ev_flops.clear();
      D->ev_step.clear();
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(D->gstream, hipStreamCaptureModeThreadLocal));
      int rc = enqueue(D->gstream, true);
      hipError_t ce = hipStreamEndCapture(D->gstream, &graph);
      if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
      }
      if (ce != hipSuccess) return hip_fail(ce, "hipStreamEndCapture");
      hipError_t ie = hipGraphInstantiate(&D->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        D->gexec = nullptr;
        return hip_fail(ie, "hipGraphInstantiate");
      }
      D->g_lo = lo;
      D->g_hi = hi;
      D->g_timing = D->timing;
      D->g_scaled = sc;
      D->g_ev_used = D->ev_used;
      D->g_ev_bytes = D->ev_bytes;
      D->g_ev_flops = D->ev_flops;
      D->g_ev_step = D->ev_step;
    }
    // the replay is ordered on the caller's stream itself
    HIP_TRY(hipGraphLaunch(D->gexec, stream));
    if (async) {
      HIP_TRY(hipMemcpyAsync(out, D->ws + D->L.partial_off, B * sizeof(qtn_partial),
                             hipMemcpyDeviceToHost, stream));
    } else {
      if (int rc = wait_stream(stream, "qtn_contract")) return rc;
      std::memcpy(out, D->host_partials, B * sizeof(qtn_partial));
    }
    D->ev_used = D->g_ev_used;
    D->ev_bytes = D->g_ev_bytes;
    D->ev_flops = D->g_ev_flops;
    D->ev_step = D->g_ev_step;
  } else {
    int rc = enqueue(stream, false);
    if (rc) return rc;
    if (async) {
      HIP_TRY(hipMemcpyAsync(out, D->ws + D->L.partial_off, B * sizeof(qtn_partial),
                             hipMemcpyDeviceToHost, stream));
    } else {
      if (int rc = wait_stream(stream, "qtn_contract")) return rc;
      std::memcpy(out, D->host_partials, B * sizeof(qtn_partial));
    }
  }
  if (D->timing) {
    for (size_t j = 0; j + 1 < D->ev_used; j += 2) {
      float ms = 0.f;
      const hipError_t te = hipEventElapsedTime(&ms, D->ev[j], D->ev[j + 1]);
      if (te != hipSuccess) {
        (void)hipGetLastError();
        ++D->t_failed;
        D->t_last_error = (int)te;
        continue;  // a sample that cannot be read is dropped, not an error
      }
      const int st = D->ev_step[j / 2];
      if (st < 0) {
        // workgroup programs: counted apart from the streaming steps
        D->t_prog.launches += 1;
        D->t_prog.ms += ms;
        D->t_prog.bytes += D->ev_bytes[j / 2];
        D->t_prog.flops += D->ev_flops[j / 2];
        continue;
      }
      D->t_ms += ms;
      D->t_bytes += D->ev_bytes[j / 2];
      D->t_flops += D->ev_flops[j / 2];
      if (st >= 0 && (size_t)st < D->t_step.size()) {
        D->t_step[st].launches += 1;
        D->t_step[st].ms += ms;
        D->t_step[st].bytes += D->ev_bytes[j / 2];
        D->t_step[st].flops += D->ev_flops[j / 2];
      }
      D->t_launches += 1;
    }
  }
  D->ev_used = 0;
  D->ev_bytes.clear();
  D->ev_flops.clear();
  D->ev_step.clear();
  if (!async && P->scaled[D->mode] && !sc) {
    // a run without rescaling: repeat it with rescaling if any value left
    // the 64-bit form's exponent range (QTN_RANGE_TEST=1, a test hook, makes
    // every such run count as one that did)
    const char *tf = std::getenv("QTN_RANGE_TEST");
    const bool miss = *(volatile uint32_t *)(D->host_partials + B) != 0u || (tf && tf[0] == '1');
    if (miss) {
      if (++D->range_misses >= 2) D->unscaled = false;
      ++D->range_reruns;
      D->force_scaled = true;
      const int rc = contract_impl(P, lo, hi, stream_v, out, false);
      D->force_scaled = false;
      return rc;
    }
    D->range_misses = 0;
  }
  return QTN_OK;
}

extern "C" int qtn_plan_range_state(const qtn_plan_t *P, int32_t *unscaled, uint64_t *reruns) {
  if (!P || !P->dev || !unscaled || !reruns) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  *unscaled = scaled_run(P, P->dev, false) ? 0 : 1;
  *reruns = P->dev->range_reruns;
  return QTN_OK;
}

extern "C" int qtn_contract(qtn_plan_t *P, uint64_t lo, uint64_t hi, void *stream,
                            qtn_partial *out) {
  return contract_impl(P, lo, hi, stream, out, false);
}

extern "C" int qtn_contract_async(qtn_plan_t *P, uint64_t lo, uint64_t hi, void *stream,
                                  qtn_partial *out) {
  return contract_impl(P, lo, hi, stream, out, true);
}

// ---------------------------------------------------------------------------
// Autotuner: launch configuration of each grid-wide streaming step, measured.
// ---------------------------------------------------------------------------
static uint64_t step_signature(const PStep &d, uint64_t Q) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 255u;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)d.rC | (uint64_t)d.nk << 8 | (uint64_t)d.nvary << 16 | (uint64_t)d.nf32 << 24 |
      (uint64_t)d.nin << 32 | (uint64_t)d.dot << 40 | (uint64_t)(d.tiled_fold + 1) << 48);
  mix(d.tiled_lds);
  mix(Q);
  for (int i = 0; i < d.nin; ++i) mix((uint64_t)d.in[i].mask | (uint64_t)d.in[i].f64 << 32 | (uint64_t)d.in[i].loc << 40);
  return h;
}

template <bool SCALE>
static int autotune_impl(qtn_plan_t *P, hipStream_t stream, const char *cache_path, qtn_tune_stats *st) {
  DeviceState *D = P->dev;
  const Schedule &sch = P->sched;
  const ExecPlan &X = P->exec[D->mode];
  const uint64_t nsl = 1ull << P->cut.size();
  const uint64_t cnt = std::min<uint64_t>(D->L.S, nsl);
  // cache: one line per signature, "<hex signature> <target> <variant> <us>"
  // (variant 0 the default kernel, 1 the direct kernel, 2 the row-paired one)
  std::map<uint64_t, StepTune> cache;
  if (cache_path && cache_path[0])
    if (FILE *f = std::fopen(cache_path, "r")) {
      unsigned long long sig;
      unsigned target;
      int so;
      double us;
      while (std::fscanf(f, "%llx %u %d %lf", &sig, &target, &so, &us) == 4) {
        StepTune t;
        t.target = target;
        t.stream_only = so == 1;
        t.pair = so == 2;
        cache[(uint64_t)sig] = t;
      }
      std::fclose(f);
    }
  D->tune.assign(sch.steps.size(), StepTune());
  drop_graph(D);
  // the inputs of every step exist after one contraction of the first wave
  if (int rc = run_waves<SCALE>(P, D, 0, cnt, stream, false)) return rc;
  if (int rc = wait_stream(stream, "qtn_plan_autotune")) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::vector<std::pair<uint64_t, std::pair<StepTune, double>>> learned;
  std::vector<std::pair<double, int>> gain;   // (time saved alone, step)
  int rc = QTN_OK;
  for (const LaunchGroup &G : X.launches) {
    if (G.kind != 1) continue;
    const int s_ = G.step;
    const PStep &d = D->steps[s_];
    const bool streaming = d.rC >= kStreamMinRank && d.nk <= 4 && d.nvary >= 1 && d.nvary <= 4;
    if (!streaming) continue;
    const uint64_t Q = (uint64_t)(sch.steps[s_].bdep ? P->net.B : 1) * (sch.steps[s_].sdep ? cnt : 1);
    const uint64_t sig = step_signature(d, Q);
    ++st->steps;
    auto hit = cache.find(sig);
    if (hit != cache.end()) {
      D->tune[s_] = hit->second;
      ++st->cached;
      gain.push_back({0.0, s_});
      continue;
    }
    // (timing of garbage inputs: every launch reads only its own operands'
    // memory, which later tensors may have reused; the timing is unchanged and
    // the state is rebuilt by the next contraction)
    double best_us = 0, default_us = 0;
    StepTune best;
    // variants: the staged kernel (or the direct one where nothing is
    // staged), the direct kernel, the row-paired staged kernel
    for (uint32_t target : {256u, 512u, 1024u, 2048u, 4096u})
      for (int so = 0; so < (d.tiled_lds ? (d.tiled_pair ? 3 : 2) : 1); ++so) {
        StepTune t;
        t.target = target;
        t.stream_only = so == 1;
        t.pair = so == 2;
        uint32_t gx = 0;
        if ((rc = launch_grid_step<SCALE>(P, D, s_, stream, 0, cnt, t, &gx))) break;
        constexpr int R = 5;
        if (hipEventRecord(e0, stream) != hipSuccess) break;
        for (int r = 0; r < R && !rc; ++r) rc = launch_grid_step<SCALE>(P, D, s_, stream, 0, cnt, t, &gx);
        if (rc || hipEventRecord(e1, stream) != hipSuccess) break;
        if ((rc = wait_stream(stream, "qtn_plan_autotune"))) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          rc = hip_fail(hipGetLastError(), "hipEventElapsedTime");
          break;
        }
        const double us = 1e3 * ms / R;
        ++st->measured;
        if (target == 1024 && so == 0) default_us = us;
        if (best_us == 0 || us < best_us) {
          best_us = us;
          best = t;
        }
      }
    if (rc) break;
    D->tune[s_] = best;
    st->default_us += default_us;
    st->tuned_us += best_us;
    learned.push_back({sig, {best, best_us}});
    gain.push_back({default_us - best_us, s_});
  }
  // The steps were timed alone; in a contraction the steps of one launch
  // level share a launch and run together, so a choice that is faster alone
  // can be slower there.  Starting from the defaults, each step's choice
  // (largest gain alone first) stays only if a whole contraction of the
  // first wave is then at least 1% faster.
  const std::vector<StepTune> chosen = D->tune;
  if (!rc) {
    auto whole = [&](double *us) -> int {
      if (int r = run_waves<SCALE>(P, D, 0, cnt, stream, false)) return r;  // warm-up
      constexpr int R = 5;
      if (hipEventRecord(e0, stream) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventRecord");
      for (int r = 0; r < R; ++r)
        if (int w = run_waves<SCALE>(P, D, 0, cnt, stream, false)) return w;
      if (hipEventRecord(e1, stream) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventRecord");
      if (int w = wait_stream(stream, "qtn_plan_autotune")) return w;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return hip_fail(hipGetLastError(), "hipEventElapsedTime");
      *us = 1e3 * ms / R;
      return QTN_OK;
    };
    std::vector<StepTune> cur(sch.steps.size(), StepTune());
    D->tune = cur;
    double cur_us = 0;
    rc = whole(&cur_us);
    st->whole_default_us = cur_us;
    std::stable_sort(gain.begin(), gain.end(),
                     [](const std::pair<double, int> &a, const std::pair<double, int> &b) { return a.first > b.first; });
    for (const auto &g : gain) {
      if (rc) break;
      const StepTune &c = chosen[g.second];
      if (c.target == StepTune().target && !c.stream_only && !c.pair) continue;
      D->tune = cur;
      D->tune[g.second] = c;
      double us = 0;
      if ((rc = whole(&us))) break;
      if (us < 0.99 * cur_us) {
        cur = D->tune;
        cur_us = us;
        ++st->kept;
      }
    }
    D->tune = cur;
    st->whole_tuned_us = cur_us;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  // Launch mode: the whole contraction of the first wave through the public
  // call (synchronous, partials to host memory), replayed from a captured
  // graph against launched directly; the faster mode stays.
  {
    std::vector<qtn_partial> part(P->net.B);
    auto whole_call = [&](bool graphs, double *us) -> int {
      D->use_graphs = graphs;
      drop_graph(D);
      for (int r = 0; r < 2; ++r)   // capture (with graphs) and warm-up
        if (int w = contract_impl(P, 0, cnt, stream, part.data(), false)) return w;
      constexpr int R = 10;
      const auto t0 = std::chrono::steady_clock::now();
      for (int r = 0; r < R; ++r)
        if (int w = contract_impl(P, 0, cnt, stream, part.data(), false)) return w;
      *us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count() / R;
      return QTN_OK;
    };
    if (int w = whole_call(true, &st->graph_us)) return w;
    if (int w = whole_call(false, &st->direct_us)) return w;
    D->use_graphs = st->graph_us <= st->direct_us;
    drop_graph(D);
    st->graphs = D->use_graphs ? 1u : 0u;
  }
  // the measurements raised exponent words: start the next contraction clean
  if (SCALE && D->L.exp_bytes) HIP_TRY(hipMemsetAsync(D->ws + D->L.data_bytes, 0, D->L.exp_bytes, stream));
  if (int w = wait_stream(stream, "qtn_plan_autotune")) return w;
  if (cache_path && cache_path[0] && !learned.empty()) {
    FILE *f = std::fopen(cache_path, "a");
    if (!f) {
      set_error(std::string("cannot append to autotune cache ") + cache_path);
      return QTN_EINVAL;
    }
    for (const auto &l : learned)
      std::fprintf(f, "%016llx %u %d %.3f\n", (unsigned long long)l.first, l.second.first.target,
                   l.second.first.pair ? 2 : l.second.first.stream_only ? 1 : 0, l.second.second);
    std::fclose(f);
  }
  return QTN_OK;
}

extern "C" int qtn_plan_autotune(qtn_plan_t *P, void *stream_v, const char *cache_path, qtn_tune_stats *stats) {
  set_error("");
  if (!P || !stats) {
    set_error("NULL argument");
    return QTN_EINVAL;
  }
  if (!P->dev || !P->dev->ws) {
    set_error("no workspace bound");
    return QTN_ENOMEM;
  }
  if (P->dev->timing) {
    set_error("turn timing off before tuning");
    return QTN_ESTATE;
  }
  std::memset(stats, 0, sizeof(*stats));
  const hipStream_t stream = (hipStream_t)stream_v;
  return !scaled_run(P, P->dev, false) ? autotune_impl<false>(P, stream, cache_path, stats)
                                       : autotune_impl<true>(P, stream, cache_path, stats);
}

// ---------------------------------------------------------------------------
// Several circuits in one persistent launch: the whole-schedule programs of
// plans bound in one-workgroup-per-instance mode share one wg_programs
// launch, whose workgroups take (plan, bitstring, slice) items from all of
// them; each plan's slice sum follows.
// ---------------------------------------------------------------------------
template <bool SCALE>
static int batch_enqueue(qtn_plan_t *const *plans, uint32_t n, const uint64_t *lo, const uint64_t *hi,
                         hipStream_t stream) {
  GroupArgs ga;
  std::memset(&ga, 0, sizeof(ga));
  uint64_t total = 0, cap = ~0ull;
  uint32_t lds_bytes = 0, desc_bytes = 0;
  int max_slots = 1;
  for (uint32_t i = 0; i < n; ++i) {
    qtn_plan_t *P = plans[i];
    DeviceState *D = P->dev;
    if (lo[i] == hi[i]) continue;
    const Program &pr = P->exec[MODE_SLICE].programs[0];
    const uint64_t cnt = hi[i] - lo[i];
    const uint32_t j = ga.nprog++;
    total += (pr.bdep ? P->net.B : 1) * (pr.sdep ? cnt : 1);
    ga.item_end[j] = (uint32_t)total;
    ga.nsteps[j] = (uint16_t)pr.steps.size();
    ga.nstage[j] = (uint16_t)(pr.staged.size() + pr.staged_global.size());
    ga.bdep[j] = pr.bdep ? 1 : 0;
    ga.sdep[j] = pr.sdep ? 1 : 0;
    ga.ns[j] = (uint32_t)cnt;
    ga.blob[j] = D->blobbuf + D->blob_off[0];
    ga.scratch[j] = D->ws + D->L.scratch_off;
    ga.scratch_stride[j] = (P->exec[MODE_SLICE].scratch_per_wg + 255) & ~uint64_t(255);
    ga.s_lo[j] = lo[i];
    cap = std::min<uint64_t>(cap, std::max<uint64_t>(1, D->L.wg_slots));
    lds_bytes = std::max(lds_bytes, D->lds_bytes);
    max_slots = std::max(max_slots, D->max_slots);
    desc_bytes = std::max(desc_bytes, D->lds_total - D->desc_bytes);
  }
  if (ga.nprog) {
    // one LDS layout that holds every program: the largest tensor region,
    // slot count and descriptor region
    const uint32_t desc_off = (lds_bytes + 256 * 16 + (uint32_t)(2 * max_slots + 4) * 4 + 15) & ~15u;
    const uint32_t lds_total = desc_off + desc_bytes;
    if (lds_total > 160 * 1024) {
      set_error("the programs of the batch do not fit one LDS layout");
      return QTN_ESTATE;
    }
    if (int rc = set_program_lds(lds_total)) return rc;
    const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(total, cap));
    int max_nin = 0;
    for (uint32_t i = 0; i < n; ++i)
      if (lo[i] != hi[i]) {
        const int zero = 0;
        max_nin = std::max(max_nin, programs_max_nin(plans[i]->sched, plans[i]->exec[MODE_SLICE], &zero, 1));
      }
    launch_programs<SCALE>(max_nin, dim3((unsigned)grid), lds_total, stream, ga, (uint32_t)total, lds_bytes,
                           max_slots, desc_off);
  }
  for (uint32_t i = 0; i < n; ++i) {
    qtn_plan_t *P = plans[i];
    if (lo[i] == hi[i]) continue;
    DeviceState *D = P->dev;
    const Schedule &sch = P->sched;
    const Tensor &res = sch.tensors[sch.result];
    const uint64_t S = D->L.S, B = P->net.B;
    const uint64_t rb = res.bdep ? (res.sdep ? S : 1) : 0, rs = res.sdep ? 1 : 0;
    hipLaunchKernelGGL((slice_sum<SCALE>), dim3((unsigned)B), dim3(256), 0, stream,
                       (const void *)(D->ws + res.data_off), res.f64 ? 1u : 0u,
                       (const int *)(D->ws + res.exp_off), rb, rs, (uint32_t)(hi[i] - lo[i]),
                       P->net.prefactor, (qtn_partial *)(D->ws + D->L.partial_off), 1,
                       D->host_partials_dev,
                       (SCALE && D->L.exp_bytes) ? (uint32_t *)(D->ws + D->L.data_bytes) : (uint32_t *)nullptr,
                       D->L.exp_bytes / 4, SCALE ? (res.exp_off - D->L.data_bytes) / 4 : 0,
                       SCALE ? (res.exp_off - D->L.data_bytes) / 4 + instances(res, B, S) : 0,
                       (const double2 *)nullptr, (uint64_t)0, 0u, (uint32_t *)(D->ws + D->L.flag_off),
                       (uint32_t *)nullptr);
  }
  HIP_TRY(hipGetLastError());
  return QTN_OK;
}

extern "C" int qtn_batch_contract(qtn_plan_t *const *plans, uint32_t n_plans, const uint64_t *slice_lo,
                                  const uint64_t *slice_hi, void *stream_v, qtn_partial *out) {
  set_error("");
  if (!plans || !slice_lo || !slice_hi || !out || n_plans == 0) {
    set_error("NULL argument or no plans");
    return QTN_EINVAL;
  }
  if (n_plans > (uint32_t)kMaxGroupProgs) {
    set_error("at most " + std::to_string(kMaxGroupProgs) + " plans per batch");
    return QTN_EINVAL;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  const int prec = plans[0] ? plans[0]->precision : 0;
  // one kernel form for the launch: the rescaling one if any plan needs it
  // (a mixed-form plan whose tensors are all complex128 runs it correctly)
  bool scaled0 = false;
  for (uint32_t i = 0; i < n_plans; ++i) scaled0 = scaled0 || (plans[i] && plans[i]->scaled[MODE_SLICE]);
  uint64_t total = 0;
  for (uint32_t i = 0; i < n_plans; ++i) {
    qtn_plan_t *P = plans[i];
    if (!P || !P->dev || !P->dev->ws) {
      set_error("plan " + std::to_string(i) + " has no bound workspace");
      return QTN_ENOMEM;
    }
    if (P->dev->device != dev) {
      set_error("plan " + std::to_string(i) + " is bound on another device");
      return QTN_ESTATE;
    }
    if (P->dev->mode != MODE_SLICE) {
      set_error("plan " + std::to_string(i) + " is not bound in one-workgroup-per-instance mode (exec_mode 1)");
      return QTN_ESTATE;
    }
    if ((P->precision == QTN_FP64) != (prec == QTN_FP64)) {
      set_error("the plans of a batch share one precision form");
      return QTN_EINVAL;
    }
    const uint64_t nsl = 1ull << P->cut.size();
    if (slice_lo[i] > slice_hi[i] || slice_hi[i] > nsl) {
      set_error("plan " + std::to_string(i) + ": slice range outside [0, 2^k)");
      return QTN_ERANGE;
    }
    if (slice_hi[i] - slice_lo[i] > P->dev->L.S) {
      set_error("plan " + std::to_string(i) + ": the range exceeds its slices per wave (one wave per plan)");
      return QTN_ERANGE;
    }
    for (uint32_t j = 0; j < i; ++j)
      if (plans[j] == P) {
        set_error("a plan appears twice in the batch (its workspace would be shared)");
        return QTN_EINVAL;
      }
    total += P->net.B;
  }
  hipStream_t stream = (hipStream_t)stream_v;
  const int rc = !scaled0 ? batch_enqueue<false>(plans, n_plans, slice_lo, slice_hi, stream)
                                  : batch_enqueue<true>(plans, n_plans, slice_lo, slice_hi, stream);
  if (rc) return rc;
  if (int w = wait_stream(stream, "qtn_batch_contract")) return w;
  uint64_t at = 0;
  for (uint32_t i = 0; i < n_plans; ++i) {
    qtn_plan_t *P = plans[i];
    for (uint64_t b = 0; b < P->net.B; ++b)
      out[at + b] = slice_lo[i] == slice_hi[i] ? qtn_partial{0.0, 0.0, 0.0, 0.0} : P->dev->host_partials[b];
    at += P->net.B;
  }
  (void)total;
  return QTN_OK;
}

// ---------------------------------------------------------------------------
// Contraction without any allocation: the workspace, the gate factors and the
// program descriptors live in one file-scope device array.
// ---------------------------------------------------------------------------
constexpr uint64_t kNoAllocBytes = QTN_NOALLOC_BYTES;
static __device__ __align__(256) char scratch[kNoAllocBytes];

// Device address of `scratch` on each device, taken once per device with
// that device current.  In host code the array's name is not a device
// address; only these pointers are ever handed to kernels or copies.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices] = {};

static int scratch_address(int dev, char **out) {
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device ordinal out of range");
    return QTN_ESTATE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p || ((uintptr_t)p & 255u)) {
      set_error("scratch array has no aligned device address");
      return QTN_EHIP;
    }
    g_scratch_ptr[dev] = (char *)p;
  }
  *out = g_scratch_ptr[dev];
  return QTN_OK;
}

__global__ __launch_bounds__(256) void zero_words(uint32_t *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

namespace qtn {
// Host tables of a plan laid out in the scratch of one device: built on the
// first call for (device, slices per wave) and kept with the plan.
struct NoAllocState {
  int device = -1;
  uint64_t S = 0;
  char *base = nullptr;
  DeviceState D;              // its device pointers point into the scratch
  std::vector<double> leaves; // uploaded by every call (the scratch is shared)
  std::vector<char> blob;
  uint64_t leaf_off = 0, blob_off = 0, ws_off = 0, total = 0;
};

void noalloc_state_free(NoAllocState *n) { delete n; }
}  // namespace qtn

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

extern "C" int qtn_contract_noalloc(qtn_plan_t *P, uint64_t lo, uint64_t hi, uint64_t slices_per_wave,
                                    void *stream_v, qtn_partial *out_dev) {
  set_error("");
  if (!P || !out_dev) {
    set_error("NULL argument");
    return QTN_EINVAL;
  }
  const uint64_t nslices = 1ull << P->cut.size();
  if (lo > hi || hi > nslices) {
    set_error("slice range outside [0, 2^k)");
    return QTN_ERANGE;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  char *base = nullptr;
  if (int rc = scratch_address(dev, &base)) return rc;
  hipStream_t stream = (hipStream_t)stream_v;
  const uint64_t B = P->net.B;
  NoAllocState *N = P->na;
  if (!N || N->device != dev || N->S != std::min(slices_per_wave, nslices)) {
    BindShape shape;
    if (int rc = bind_shape(P, slices_per_wave, shape)) return rc;
    std::unique_ptr<NoAllocState> fresh(new NoAllocState());
    N = fresh.get();
    N->device = dev;
    N->S = shape.S;
    N->base = base;
    DeviceState &D = N->D;
    D.device = dev;
    D.mode = shape.mode;
    D.L = shape.L;
    D.max_slots = shape.max_slots;
    D.lds_bytes = shape.lds_bytes;
    D.lds_total = shape.lds_total;
    D.desc_bytes = shape.desc_off;
    D.use_graphs = false;
    try {
      // launch units in schedule order on the caller's stream
      D.lg = launch_graph(P->sched, P->exec[D.mode], D.L, P->net.B, D.L.S, P->precision != QTN_FP64, 1);
    } catch (const std::exception &e) {
      set_error(e.what());
      return QTN_ESTATE;
    }
    N->leaves = leaf_host(P, D.leaf_elem_off);
    // scratch: gate factors | program descriptors | workspace
    N->leaf_off = 0;
    D.leafbuf = base + N->leaf_off;
    N->blob_off = align256(N->leaf_off + N->leaves.size() * sizeof(double));
    // the descriptor blob's size does not depend on the addresses it holds
    D.ws = base;
    fill_tables(P, &D, P->exec[D.mode], N->blob);
    N->ws_off = align256(N->blob_off + N->blob.size());
    N->total = N->ws_off + D.L.total_bytes;
    if (N->total > kNoAllocBytes) {
      set_error("qtn_contract_noalloc: this plan needs " + std::to_string(N->total) +
                " bytes of scratch (gate factors, descriptors, workspace) at " +
                std::to_string(shape.S) + " slices per wave; the scratch holds " +
                std::to_string(kNoAllocBytes));
      return QTN_ENOMEM;
    }
    D.ws = base + N->ws_off;
    D.ws_bytes = D.L.total_bytes;
    fill_tables(P, &D, P->exec[D.mode], N->blob);
    delete P->na;
    P->na = fresh.release();
  }
  if (lo == hi) {
    // exact zeros, written on the stream like every other result
    hipLaunchKernelGGL(zero_words, dim3(1), dim3(256), 0, stream, (uint32_t *)out_dev,
                       (uint64_t)(B * sizeof(qtn_partial) / 4));
    HIP_TRY(hipGetLastError());
    return QTN_OK;
  }
  DeviceState &D = N->D;
  if (int rc = set_program_lds(D.lds_total)) return rc;
  // the scratch is shared by every plan on this device: upload this plan's
  // constants and clear its exponent words on the stream, before its kernels
  HIP_TRY(hipMemcpyAsync(base + N->leaf_off, N->leaves.data(), N->leaves.size() * sizeof(double),
                         hipMemcpyHostToDevice, stream));
  if (!N->blob.empty())
    HIP_TRY(hipMemcpyAsync(base + N->blob_off, N->blob.data(), N->blob.size(), hipMemcpyHostToDevice, stream));
  D.blobbuf = base + N->blob_off;
  const bool scaled = P->scaled[D.mode];
  if (scaled && D.L.exp_bytes) {
    const uint64_t words = D.L.exp_bytes / 4;
    const unsigned blocks = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((words + 255) / 256, 1024));
    hipLaunchKernelGGL(zero_words, dim3(blocks), dim3(256), 0, stream, (uint32_t *)(D.ws + D.L.data_bytes), words);
  }
  D.host_partials_dev = out_dev;   // the last wave's slice sum writes the result here
  return scaled ? run_waves<true>(P, &D, lo, hi, stream, false) : run_waves<false>(P, &D, lo, hi, stream, false);
}

extern "C" int qtn_plan_set_graphs(qtn_plan_t *P, int enable) {
  if (!P || !P->dev) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  P->dev->use_graphs = enable != 0;
  drop_graph(P->dev);
  return QTN_OK;
}

extern "C" int qtn_plan_set_timing(qtn_plan_t *P, int enable) {
  if (!P || !P->dev) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  DeviceState *D = P->dev;
  D->timing = enable != 0;
  D->t_ms = D->t_bytes = D->t_flops = 0;
  D->t_launches = D->t_failed = 0;
  D->t_last_error = 0;
  D->t_step.assign(P->sched.steps.size(), DeviceState::StepTiming());
  D->t_prog = DeviceState::StepTiming();
  return QTN_OK;
}

extern "C" int qtn_plan_timing(const qtn_plan_t *P, qtn_kernel_timing *out) {
  if (!P || !out || !P->dev) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  const DeviceState *D = P->dev;
  out->launches = D->t_launches;
  out->total_ms = D->t_ms;
  out->alg_bytes = D->t_bytes;
  out->alg_flops = D->t_flops;
  out->dropped = D->t_failed;
  out->last_error = D->t_last_error;
  return QTN_OK;
}

extern "C" int qtn_plan_step_timing(const qtn_plan_t *P, int32_t step, qtn_kernel_timing *out) {
  if (!P || !out || !P->dev) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  if (step < -1 || step >= (int32_t)P->sched.steps.size()) {
    set_error("step out of range");
    return QTN_ERANGE;
  }
  const DeviceState *D = P->dev;
  std::memset(out, 0, sizeof(*out));
  if (step == -1) {
    out->launches = D->t_prog.launches;
    out->total_ms = D->t_prog.ms;
    out->alg_bytes = D->t_prog.bytes;
    out->alg_flops = D->t_prog.flops;
  } else if ((size_t)step < D->t_step.size()) {
    const DeviceState::StepTiming &T = D->t_step[step];
    out->launches = T.launches;
    out->total_ms = T.ms;
    out->alg_bytes = T.bytes;
    out->alg_flops = T.flops;
  }
  return QTN_OK;
}

extern "C" int qtn_plan_step_tune(const qtn_plan_t *P, int32_t step, uint32_t *blocks, int32_t *variant) {
  if (!P || !P->dev || !blocks || !variant) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  if (step < 0 || (size_t)step >= P->sched.steps.size()) {
    set_error("step out of range");
    return QTN_ERANGE;
  }
  const StepTune t = P->dev->tune.empty() ? StepTune() : P->dev->tune[step];
  *blocks = t.target;
  *variant = t.pair ? 2 : t.stream_only ? 1 : 0;
  return QTN_OK;
}

extern "C" int qtn_plan_set_step_tune(qtn_plan_t *P, int32_t step, uint32_t blocks, int32_t variant) {
  if (!P || !P->dev) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  if (step < 0 || (size_t)step >= P->sched.steps.size()) {
    set_error("step out of range");
    return QTN_ERANGE;
  }
  if (blocks < 1 || blocks > (1u << 20) || variant < 0 || variant > 2) {
    set_error("blocks must be in [1, 2^20] and variant in {0, 1, 2}");
    return QTN_EINVAL;
  }
  DeviceState *D = P->dev;
  if (D->tune.empty()) D->tune.assign(P->sched.steps.size(), StepTune());
  StepTune &t = D->tune[step];
  t.target = blocks;
  t.stream_only = variant == 1;
  t.pair = variant == 2;
  drop_graph(D);
  return QTN_OK;
}

extern "C" int qtn_plan_step_kernel(const qtn_plan_t *P, int32_t step, char *name, uint32_t capacity) {
  if (!P || !P->dev || !name || capacity == 0) {
    set_error("bind a workspace first");
    return QTN_ESTATE;
  }
  if (step < 0 || (size_t)step >= P->sched.steps.size()) {
    set_error("step out of range");
    return QTN_ERANGE;
  }
  const DeviceState *D = P->dev;
  const ExecPlan &X = P->exec[D->mode];
  std::string k;
  for (const LaunchGroup &G : X.launches)
    if (G.kind == 1 && G.step == step) {
      const PStep &d = D->steps[step];
      const bool sc = scaled_run(P, D, false);   // the kernels a synchronous call runs
      const bool streaming = d.rC >= kStreamMinRank && d.nk <= 4 && d.nvary >= 1 && d.nvary <= 4;
      const std::string tf = sc ? "true" : "false";
      // the autotuner may have chosen the direct kernel for a staged step
      const StepTune tu = D->tune.empty() ? StepTune() : D->tune[step];
      const bool tiled = d.tiled_lds && !tu.stream_only;
      // the row-paired form runs where the step's rows come in 16-row chunks
      uint32_t jspan = 1;
      const uint64_t Q = (uint64_t)(P->sched.steps[step].bdep ? P->net.B : 1) *
                         (P->sched.steps[step].sdep ? std::min<uint64_t>(D->L.S, 1ull << P->cut.size()) : 1);
      if (streaming) (void)stream_grid(d, Q, tu.target, &jspan);
      const bool pair = tiled && tu.pair && d.tiled_pair && d.tiled_fold == 0 && d.nk >= 3 && jspan >= 16;
      if (!streaming)
        k = "step_small<" + tf + ">";
      else
        k = std::string(pair ? "step_tiled_pair<" : tiled ? "step_tiled<" : "step_stream<") + tf + ", " +
            std::to_string(d.nk) + ", " + std::to_string(d.nvary) + ", " +
            std::to_string(d.nf32 <= d.nvary ? d.nf32 : 0) +
            (pair ? ">" : tiled ? (d.tiled_fold == 0 ? ", true>" : ", false>") : ">") +
            (d.dot ? " + closing-chain reduction" : "");
    }
  std::strncpy(name, k.c_str(), capacity - 1);
  name[capacity - 1] = 0;
  return QTN_OK;
}
