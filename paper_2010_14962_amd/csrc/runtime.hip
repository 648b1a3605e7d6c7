// Device side of libqtn for gfx950: plan upload, the fused contraction step
// kernel (Eq. (1) generalised to several operands and summed indices) and the
// compensated FP64 slice sum (Eq. (2); the master-side sum of Sec. III A).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qtn.h"
#include "plan_state.h"

namespace qtn {

// ---------------------------------------------------------------------------
// Descriptors passed by value to the step kernels.
// ---------------------------------------------------------------------------
struct InDesc {
  const void *base;       // element 0 of the tensor (leaf block or workspace)
  uint64_t bstride;       // elements between bitstrings
  uint64_t sstride;       // elements between slice-local instances
  uint64_t vsize;         // leaves: elements per slice variant
  const uint32_t *tab;    // lo[256] | mid[16] | kap[2^nk]
  const int *E;           // scaled intermediates: accumulated exponent per instance
  const uint32_t *M;      // scaled intermediates: max |component| (float bits)
  uint32_t ebstride, esstride;
  uint32_t selmask;       // leaves: slice bits that pick the variant
  uint32_t hi_mask, hi_shift;
  uint32_t f64;           // stored as complex128 (else complex64)
};

struct StepDesc {
  InDesc in[kMaxIn];
  void *out;
  int *oE;
  uint32_t *oM;
  uint64_t obstride, osstride;
  uint32_t oebstride, oesstride;
  int nin, rC, nk;
  uint32_t nb, ns;        // instance grid of the launch
  uint64_t s_lo;          // global slice index of slice-local 0
};

struct DeviceState {
  int device = -1;
  void *leafbuf = nullptr;                        // complex128 gate factors
  uint32_t *tabbuf = nullptr;
  std::vector<uint64_t> leaf_elem_off;            // per tensor
  std::vector<std::vector<uint64_t>> tab_off;     // per step, per input (uint32 units)
  char *ws = nullptr;
  uint64_t ws_bytes = 0;
  Layout L;
  std::vector<StepDesc> descs;
  // optional per-launch timing of the streaming step kernel
  bool timing = false;
  std::vector<hipEvent_t> ev;      // start/stop pairs
  size_t ev_used = 0;
  std::vector<double> ev_bytes;    // algorithmic bytes of each timed launch
  std::vector<double> ev_flops;
  double t_ms = 0, t_bytes = 0, t_flops = 0;
  uint64_t t_launches = 0;
  std::vector<double> step_bytes, step_flops;  // per instance of each step
};

void device_state_free(DeviceState *d) {
  if (!d) return;
  for (auto e : d->ev) (void)hipEventDestroy(e);
  if (d->leafbuf) (void)hipFree(d->leafbuf);
  if (d->tabbuf) (void)hipFree(d->tabbuf);
  delete d;
}

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

__device__ __forceinline__ double2 load_c(const InDesc &in, uint64_t i) {
  if (in.f64) return ((const double2 *)in.base)[i];
  const float2 f = ((const float2 *)in.base)[i];
  return make_double2((double)f.x, (double)f.y);
}

// Exponent e with 2^(e-1) <= x < 2^e for the positive float with bits `b`
// (0 for zero or subnormal): frexp's convention.
__device__ __forceinline__ int exp_of_bits(uint32_t b) {
  int be = (int)((b >> 23) & 255u);
  return be == 0 ? 0 : be - 126;
}

// Per-instance part of every operand offset, and the exponent bookkeeping of
// the scaled form: inputs are read as mantissa * 2^E; the product is scaled by
// 2^-(sum of input max-exponents) so the stored result stays near 1.
struct InstanceSetup {
  uint64_t off[kMaxIn];
  int sh, esum;
  uint32_t qo;
  uint64_t obase;
};

template <bool SCALE>
__device__ __forceinline__ void setup_instance(const StepDesc &d, uint64_t q, InstanceSetup &I) {
  const uint32_t b = (uint32_t)(q / d.ns);
  const uint32_t sl = (uint32_t)(q - (uint64_t)b * d.ns);
  const uint32_t s = (uint32_t)(d.s_lo + sl);
  I.sh = 0;
  I.esum = 0;
#pragma unroll
  for (int i = 0; i < kMaxIn; ++i) {
    if (i < d.nin) {
      const InDesc &in = d.in[i];
      uint64_t o = (uint64_t)b * in.bstride + (uint64_t)sl * in.sstride;
      if (in.selmask) o += (uint64_t)dpext(s, in.selmask) * in.vsize;
      I.off[i] = o;
      if (SCALE && in.E) {
        const uint32_t qi = b * in.ebstride + sl * in.esstride;
        const int e = exp_of_bits(in.M[qi]);
        I.sh += e;
        I.esum += in.E[qi] + e;
      }
    }
  }
  I.qo = b * d.oebstride + sl * d.oesstride;
  I.obase = (uint64_t)b * d.obstride + (uint64_t)sl * d.osstride;
}

// Sum over kappa of the operand product at output element c (FP64 registers).
__device__ __forceinline__ double2 contract_point(const StepDesc &d, const uint64_t *cidx,
                                                  uint32_t nkap) {
  double2 acc = make_double2(0.0, 0.0);
  for (uint32_t kk = 0; kk < nkap; ++kk) {
    double2 prod = load_c(d.in[0], cidx[0] + d.in[0].tab[272 + kk]);
#pragma unroll
    for (int i = 1; i < kMaxIn; ++i)
      if (i < d.nin) prod = cmul(prod, load_c(d.in[i], cidx[i] + d.in[i].tab[272 + kk]));
    acc.x += prod.x;
    acc.y += prod.y;
  }
  return acc;
}

template <bool OUT64>
__device__ __forceinline__ void store_c(void *base, uint64_t i, double2 v) {
  if (OUT64)
    ((double2 *)base)[i] = v;
  else
    ((float2 *)base)[i] = make_float2((float)v.x, (float)v.y);
}

template <bool OUT64>
__device__ __forceinline__ uint32_t max_bits(double2 v) {
  // magnitude of the stored value, as non-negative float bits (order-preserving)
  const float ax = OUT64 ? (float)fabs(v.x) : fabsf((float)v.x);
  const float ay = OUT64 ? (float)fabs(v.y) : fabsf((float)v.y);
  return max(__float_as_uint(ax), __float_as_uint(ay));
}

// Streaming steps (output of >= 2^12 elements per instance): blockIdx.y walks
// the (bitstring, slice) instances, x-blocks stream the output elements.  All
// per-instance offsets and exponents are block-uniform.
template <bool SCALE, bool OUT64>
__global__ __launch_bounds__(256) void step_stream(const StepDesc d) {
  const uint64_t Q = (uint64_t)d.nb * d.ns;
  const uint32_t nC = 1u << d.rC;
  const uint32_t nkap = 1u << d.nk;
  for (uint64_t q = blockIdx.y; q < Q; q += gridDim.y) {
    InstanceSetup I;
    setup_instance<SCALE>(d, q, I);
    uint32_t wmax = 0;
    for (uint32_t c = blockIdx.x * 256u + threadIdx.x; c < nC; c += gridDim.x * 256u) {
      uint64_t cidx[kMaxIn];
#pragma unroll
      for (int i = 0; i < kMaxIn; ++i) {
        if (i < d.nin) {
          const InDesc &in = d.in[i];
          uint64_t o = I.off[i] + in.tab[c & 255u] + in.tab[256 + ((c >> 8) & 15u)];
          if (in.hi_mask) o += (uint64_t)dpext(c >> 12, in.hi_mask) << in.hi_shift;
          cidx[i] = o;
        }
      }
      double2 acc = contract_point(d, cidx, nkap);
      if (SCALE) {
        acc.x = ldexp(acc.x, -I.sh);
        acc.y = ldexp(acc.y, -I.sh);
        wmax = max(wmax, max_bits<OUT64>(acc));
      }
      store_c<OUT64>(d.out, I.obase + c, acc);
    }
    if (SCALE) {
      // nC is a multiple of 256: every lane of the block ran the same trips
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, (uint32_t)__shfl_xor((int)wmax, o, 64));
      if ((threadIdx.x & 63) == 0 && wmax) atomicMax(d.oM + I.qo, wmax);
      if (blockIdx.x == 0 && threadIdx.x == 0) d.oE[I.qo] = I.esum;
    }
  }
}

// Small steps: one flat index over (instance, output element).
template <bool SCALE, bool OUT64>
__global__ __launch_bounds__(256) void step_small(const StepDesc d) {
  const int rC = d.rC;
  const uint64_t total = ((uint64_t)d.nb * d.ns) << rC;
  const uint32_t cmask = (1u << rC) - 1u;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint32_t nkap = 1u << d.nk;
  for (uint64_t G = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; G < total; G += stride) {
    const uint64_t q = G >> rC;
    const uint32_t c = (uint32_t)G & cmask;
    InstanceSetup I;
    setup_instance<SCALE>(d, q, I);
    uint64_t cidx[kMaxIn];
#pragma unroll
    for (int i = 0; i < kMaxIn; ++i) {
      if (i < d.nin) {
        const InDesc &in = d.in[i];
        uint64_t o = I.off[i] + in.tab[c & 255u] + in.tab[256 + ((c >> 8) & 15u)];
        if (in.hi_mask) o += (uint64_t)dpext(c >> 12, in.hi_mask) << in.hi_shift;
        cidx[i] = o;
      }
    }
    double2 acc = contract_point(d, cidx, nkap);
    if (SCALE) {
      acc.x = ldexp(acc.x, -I.sh);
      acc.y = ldexp(acc.y, -I.sh);
      const uint32_t mb = max_bits<OUT64>(acc);
      if (mb) atomicMax(d.oM + I.qo, mb);
      if (c == 0) d.oE[I.qo] = I.esum;
    }
    store_c<OUT64>(d.out, I.obase + c, acc);
  }
}
constexpr int kStreamMinRank = 12;

// ---------------------------------------------------------------------------
// Compensated FP64 slice sum: one block per bitstring, fixed reduction order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

template <bool RES64, bool SCALE>
__global__ __launch_bounds__(256) void slice_sum(const void *res, const int *E, uint64_t bstride,
                                                 uint64_t sstride, uint32_t ebstride,
                                                 uint32_t esstride, uint32_t count, double pref,
                                                 qtn_partial *partials, int init) {
  __shared__ double sre[256], cre[256], sim[256], cim[256];
  const uint32_t b = blockIdx.x;
  const uint32_t t = threadIdx.x;
  double ar = 0, cr = 0, ai = 0, ci = 0;
  for (uint32_t sl = t; sl < count; sl += 256) {
    const uint64_t at = (uint64_t)b * bstride + (uint64_t)sl * sstride;
    double vr, vi;
    if (RES64) {
      const double2 v = ((const double2 *)res)[at];
      vr = v.x;
      vi = v.y;
    } else {
      const float2 v = ((const float2 *)res)[at];
      vr = (double)v.x;
      vi = (double)v.y;
    }
    if (SCALE) {
      int e = E[b * ebstride + sl * esstride];
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
    }
  }
}

__global__ void zero_words(uint32_t *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
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


}  // namespace qtn

using namespace qtn;

extern "C" int qtn_plan_bind_workspace(qtn_plan_t *P, void *dev_ptr, uint64_t bytes,
                                       uint64_t S) {
  set_error("");
  if (!P || !dev_ptr) {
    set_error("NULL argument");
    return QTN_EINVAL;
  }
  if (S == 0 || S > (1ull << 24)) {
    set_error("slices_per_wave must be in [1, 2^24]");
    return QTN_EINVAL;
  }
  if (((uintptr_t)dev_ptr) & 255u) {
    set_error("workspace must be 256-byte aligned");
    return QTN_EINVAL;
  }
  const uint64_t maxS = P->cut.empty() ? 1 : (1ull << P->cut.size());
  if (S > maxS) S = maxS;
  Schedule &sch = P->sched;
  Layout L = layout(sch, P->net.B, S);
  if (bytes < L.total_bytes) {
    set_error("workspace too small: need " + std::to_string(L.total_bytes) + " bytes");
    return QTN_ENOMEM;
  }
  if (!P->cut.empty() && !sch.tensors[sch.result].sdep) {
    set_error("internal: sliced result does not depend on the slice");
    return QTN_ESTATE;
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  DeviceState *D = P->dev;
  if (!D || D->device != dev) {
    device_state_free(D);
    D = new DeviceState();
    P->dev = D;
    D->device = dev;
    // gate factors stay complex128 in every precision form
    D->leaf_elem_off.assign(sch.tensors.size(), 0);
    uint64_t nleaf = 0;
    for (size_t t = 0; t < sch.tensors.size(); ++t)
      if (sch.tensors[t].leaf) {
        D->leaf_elem_off[t] = nleaf;
        nleaf += sch.tensors[t].values.size();
      }
    std::vector<double> host(std::max<uint64_t>(nleaf, 1) * 2, 0.0);
    for (size_t t = 0; t < sch.tensors.size(); ++t) {
      const Tensor &T = sch.tensors[t];
      if (!T.leaf) continue;
      for (size_t i = 0; i < T.values.size(); ++i) {
        uint64_t k = D->leaf_elem_off[t] + i;
        host[2 * k] = T.values[i].real();
        host[2 * k + 1] = T.values[i].imag();
      }
    }
    hipError_t e = hipMalloc(&D->leafbuf, host.size() * sizeof(double));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(leaves)");
    HIP_TRY(hipMemcpy(D->leafbuf, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice));
    // index tables
    std::vector<uint32_t> tabs;
    D->tab_off.assign(sch.steps.size(), {});
    for (size_t st = 0; st < sch.steps.size(); ++st) {
      const Step &S_ = sch.steps[st];
      for (size_t i = 0; i < S_.in.size(); ++i) {
        InputTables it = input_tables(S_.mask[i], S_.rC, S_.nk);
        D->tab_off[st].push_back(tabs.size());
        tabs.insert(tabs.end(), it.lo, it.lo + 256);
        tabs.insert(tabs.end(), it.mid, it.mid + 16);
        tabs.insert(tabs.end(), it.kap.begin(), it.kap.end());
        while (tabs.size() & 63) tabs.push_back(0);
      }
    }
    e = hipMalloc((void **)&D->tabbuf, std::max<size_t>(tabs.size(), 1) * 4);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(tables)");
    HIP_TRY(hipMemcpy(D->tabbuf, tabs.data(), tabs.size() * 4, hipMemcpyHostToDevice));
  }
  // algorithmic bytes and flops of each step, per instance
  D->step_bytes.assign(sch.steps.size(), 0.0);
  D->step_flops.assign(sch.steps.size(), 0.0);
  for (size_t st = 0; st < sch.steps.size(); ++st) {
    const Step &S_ = sch.steps[st];
    const Tensor &O = sch.tensors[S_.out];
    double by = std::ldexp((double)elem_bytes(O), S_.rC);
    for (int i : S_.in) by += std::ldexp((double)elem_bytes(sch.tensors[i]), sch.tensors[i].rank());
    D->step_bytes[st] = by;
    D->step_flops[st] = std::ldexp(1.0, S_.nk + S_.rC) *
                        (6.0 * (double)(S_.in.size() - 1) + (S_.nk > 0 ? 2.0 : 0.0));
  }
  D->ws = (char *)dev_ptr;
  D->ws_bytes = bytes;
  D->L = L;
  // descriptors with workspace addresses
  const uint64_t B = P->net.B;
  const bool scaled = P->precision != QTN_FP64;
  D->descs.assign(sch.steps.size(), StepDesc{});
  for (size_t st = 0; st < sch.steps.size(); ++st) {
    const Step &S_ = sch.steps[st];
    StepDesc &d = D->descs[st];
    std::memset(&d, 0, sizeof(d));
    d.nin = (int)S_.in.size();
    d.rC = S_.rC;
    d.nk = S_.nk;
    for (size_t i = 0; i < S_.in.size(); ++i) {
      const Tensor &T = sch.tensors[S_.in[i]];
      InDesc &in = d.in[i];
      InputTables it = input_tables(S_.mask[i], S_.rC, S_.nk);
      in.tab = D->tabbuf + D->tab_off[st][i];
      in.hi_mask = it.hi_mask;
      in.hi_shift = it.hi_shift;
      in.f64 = T.f64 ? 1u : 0u;
      const uint64_t size = 1ull << T.rank();
      if (T.leaf) {
        in.base = (const double *)D->leafbuf + 2 * D->leaf_elem_off[S_.in[i]];
        in.vsize = size;
        in.selmask = T.selmask;
        in.bstride = T.bdep ? (size << __builtin_popcount(T.selmask)) : 0;
        in.sstride = 0;
      } else {
        in.base = D->ws + T.data_off;
        in.bstride = T.bdep ? (T.sdep ? S : 1) * size : 0;
        in.sstride = T.sdep ? size : 0;
        if (scaled) {
          in.E = (const int *)(D->ws + T.exp_off);
          in.M = (const uint32_t *)(D->ws + T.exp_off) + instances(T, B, S);
        }
        in.ebstride = T.bdep ? (uint32_t)(T.sdep ? S : 1) : 0;
        in.esstride = T.sdep ? 1 : 0;
      }
    }
    const Tensor &O = sch.tensors[S_.out];
    const uint64_t osize = 1ull << O.rank();
    d.out = D->ws + O.data_off;
    d.obstride = O.bdep ? (O.sdep ? S : 1) * osize : 0;
    d.osstride = O.sdep ? osize : 0;
    d.oE = (int *)(D->ws + O.exp_off);
    d.oM = (uint32_t *)(D->ws + O.exp_off) + instances(O, B, S);
    d.oebstride = O.bdep ? (uint32_t)(O.sdep ? S : 1) : 0;
    d.oesstride = O.sdep ? 1 : 0;
    d.nb = O.bdep ? (uint32_t)B : 1;
  }
  return QTN_OK;
}

template <bool SCALE, bool OUT64>
static void launch_step(DeviceState *D, const StepDesc &d, hipStream_t stream) {
  if (d.rC >= kStreamMinRank) {
    const uint64_t Q = (uint64_t)d.nb * d.ns;
    const uint32_t per_inst = (1u << d.rC) / 256u;
    // about 8 waves of blocks over the chip, at least one block per instance
    const uint64_t want = std::max<uint64_t>(1, 8192 / std::max<uint64_t>(Q, 1));
    const unsigned gx = (unsigned)std::min<uint64_t>(per_inst, std::max<uint64_t>(want, 1));
    const unsigned gy = (unsigned)std::min<uint64_t>(Q, 65535);
    hipLaunchKernelGGL((step_stream<SCALE, OUT64>), dim3(gx, gy), dim3(256), 0, stream, d);
  } else {
    const uint64_t total = ((uint64_t)d.nb * d.ns) << d.rC;
    const unsigned blocks =
        (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((total + 255) / 256, 16384));
    hipLaunchKernelGGL((step_small<SCALE, OUT64>), dim3(blocks), dim3(256), 0, stream, d);
  }
  (void)D;
}

template <bool SCALE>
static int run_waves(qtn_plan_t *P, uint64_t lo, uint64_t hi, hipStream_t stream) {
  DeviceState *D = P->dev;
  const Schedule &sch = P->sched;
  const uint64_t S = D->L.S;
  const uint64_t B = P->net.B;
  qtn_partial *partials = (qtn_partial *)(D->ws + D->L.partial_off);
  const Tensor &res = sch.tensors[sch.result];
  bool first = true;
  for (uint64_t s_lo = lo; s_lo < hi; s_lo += S) {
    const uint64_t cnt = std::min<uint64_t>(S, hi - s_lo);
    if (SCALE) {
      const uint64_t words = D->L.exp_bytes / 4;
      hipLaunchKernelGGL(zero_words, dim3((unsigned)std::min<uint64_t>((words + 255) / 256, 4096)),
                         dim3(256), 0, stream, (uint32_t *)(D->ws + D->L.data_bytes), words);
    }
    for (size_t st = 0; st < sch.steps.size(); ++st) {
      StepDesc d = D->descs[st];
      d.s_lo = s_lo;
      d.ns = sch.steps[st].sdep ? (uint32_t)cnt : 1;
      const bool out64 = sch.tensors[sch.steps[st].out].f64;
      const bool timed = D->timing && d.rC >= kStreamMinRank;
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
      if (out64)
        launch_step<SCALE, true>(D, d, stream);
      else
        launch_step<SCALE, false>(D, d, stream);
      if (timed) {
        HIP_TRY(hipEventRecord(D->ev[D->ev_used + 1], stream));
        D->ev_used += 2;
        const double q = (double)d.nb * d.ns;
        D->ev_bytes.push_back(q * D->step_bytes[st]);
        D->ev_flops.push_back(q * D->step_flops[st]);
      }
    }
    const uint64_t rb = res.bdep ? (res.sdep ? S : 1) : 0, rs = res.sdep ? 1 : 0;
    const void *rp = (const void *)(D->ws + res.data_off);
    const int *re = (const int *)(D->ws + res.exp_off);
    if (res.f64)
      hipLaunchKernelGGL((slice_sum<true, SCALE>), dim3((unsigned)B), dim3(256), 0, stream, rp, re,
                         rb, rs, (uint32_t)rb, (uint32_t)rs, (uint32_t)cnt, P->net.prefactor,
                         partials, first ? 1 : 0);
    else
      hipLaunchKernelGGL((slice_sum<false, SCALE>), dim3((unsigned)B), dim3(256), 0, stream, rp, re,
                         rb, rs, (uint32_t)rb, (uint32_t)rs, (uint32_t)cnt, P->net.prefactor,
                         partials, first ? 1 : 0);
    first = false;
  }
  HIP_TRY(hipGetLastError());
  return QTN_OK;
}

extern "C" int qtn_contract(qtn_plan_t *P, uint64_t lo, uint64_t hi, void *stream_v,
                            qtn_partial *out) {
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
  int rc;
  if (P->precision == QTN_FP64)
    rc = run_waves<false>(P, lo, hi, stream);
  else
    rc = run_waves<true>(P, lo, hi, stream);
  if (rc) return rc;
  HIP_TRY(hipMemcpyAsync(out, P->dev->ws + P->dev->L.partial_off, B * sizeof(qtn_partial),
                         hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  DeviceState *D = P->dev;
  if (D->timing) {
    for (size_t j = 0; j + 1 < D->ev_used; j += 2) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, D->ev[j], D->ev[j + 1]));
      D->t_ms += ms;
      D->t_bytes += D->ev_bytes[j / 2];
      D->t_flops += D->ev_flops[j / 2];
      D->t_launches += 1;
    }
  }
  D->ev_used = 0;
  D->ev_bytes.clear();
  D->ev_flops.clear();
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
  D->t_launches = 0;
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
  return QTN_OK;
}
