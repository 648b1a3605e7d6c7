// Learned cut-set cost model on gfx950: a ReLU multilayer perceptron whose
// dense layers run on FP32 matrix cores (v_mfma_f32_16x16x4f32), trained with
// MSE and Adam by hand-written kernels, and the model-guided cut search that
// uses it to rank candidates before exact evaluation.  The model is not part
// of the paper; it only speeds up the search of Sec. III B, and every cut set
// it helps choose is scored exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/qtn.h"
#include "costmodel.h"
#include "plan_state.h"

namespace qtn {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// C(m, n) = sum_k A(m, k) B(k, n) with A(m, k) = A[m*a_m + k*a_k] and
// B(k, n) = B[k*b_k + n*b_n].  One wave computes one 16x16 tile with the
// 16x16x4 FP32 matrix instruction: lane l holds A(l%16, k0 + l/16) and
// B(k0 + l/16, l%16), and receives D rows 4*(l/16) .. 4*(l/16)+3 of column
// l%16.  Epilogue: + bias[n], times (mask(m, n) > 0), ReLU copy.
__global__ __launch_bounds__(64) void gemm_f32_mfma(const float *__restrict__ A, int a_m, int a_k,
                                                    const float *__restrict__ B, int b_k, int b_n,
                                                    int M, int N, int K,
                                                    const float *__restrict__ bias,
                                                    const float *__restrict__ mask, int ld_mask,
                                                    float *__restrict__ Z, int ldz,
                                                    float *__restrict__ H) {
  const int lane = threadIdx.x;
  const int m0 = blockIdx.y * 16, n0 = blockIdx.x * 16;
  const int ar = m0 + (lane & 15);
  const int bc = n0 + (lane & 15);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int kk = k0 + (lane >> 4);
    const float a = (ar < M && kk < K) ? A[(long)ar * a_m + (long)kk * a_k] : 0.f;
    const float b = (bc < N && kk < K) ? B[(long)kk * b_k + (long)bc * b_n] : 0.f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = m0 + 4 * (lane >> 4) + i;
    const int c = n0 + (lane & 15);
    if (r < M && c < N) {
      float z = acc[i];
      if (bias) z += bias[c];
      if (mask) z = mask[(long)r * ld_mask + c] > 0.f ? z : 0.f;
      Z[(long)r * ldz + c] = z;
      if (H) H[(long)r * ldz + c] = z > 0.f ? z : 0.f;
    }
  }
}

// Column sums in a fixed order: out[n] = sum_m X[m*ld + n].
__global__ void colsum(const float *X, int M, int N, int ld, float *out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += X[(long)m * ld + n];
  out[n] = s;
}

// Mean squared error over batch x outputs and its gradient (one block, fixed order).
__global__ __launch_bounds__(256) void mse_loss(const float *Y, const float *T, int count,
                                                float *dY, float *loss) {
  __shared__ float red[256];
  float s = 0.f;
  const float scale = 2.0f / (float)count;
  for (int i = threadIdx.x; i < count; i += 256) {
    const float d = Y[i] - T[i];
    s += d * d;
    dY[i] = scale * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] / (float)count;
}

// Adam (Kingma and Ba, 2015) with bias-corrected moments.
__global__ void adam_step(float *w, const float *g, float *m, float *v, long n, float lr, float b1,
                          float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace qtn

using namespace qtn;

struct qtn_mlp_s {
  int in_dim = 0, hidden = 0, nh = 0, out_dim = 0, max_batch = 0;
  std::vector<int> dims;             // layer widths: in, hidden x nh, out
  std::vector<long> woff, boff;      // parameter offsets per layer
  long nparams = 0;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  float *acts = nullptr;             // per layer l: Z_l then H_l (max_batch x dims[l+1] each)
  std::vector<long> zoff, hoff;
  float *dz[2] = {nullptr, nullptr}; // ping-pong gradient buffers
  float *dy = nullptr, *loss = nullptr, *xin = nullptr, *tin = nullptr;
  long t = 0;
  std::vector<float> x_mean, x_std, y_mean, y_std;
  int device = 0;
};

static int mlp_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return QTN_EHIP;
}
#define MLP_TRY(call)                                 \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return mlp_fail(_e, #call); \
  } while (0)

static void mlp_free(qtn_mlp_t *M) {
  for (void *p : {(void *)M->params, (void *)M->grads, (void *)M->m, (void *)M->v, (void *)M->acts,
                  (void *)M->dz[0], (void *)M->dz[1], (void *)M->dy, (void *)M->loss,
                  (void *)M->xin, (void *)M->tin})
    if (p) (void)hipFree(p);
}

extern "C" int qtn_mlp_create(uint32_t in_dim, uint32_t hidden, uint32_t n_hidden, uint32_t out_dim,
                              uint32_t max_batch, uint64_t seed, qtn_mlp_t **out) {
  set_error("");
  if (!out || !in_dim || !hidden || !out_dim || !max_batch || n_hidden > 16 || in_dim > 4096 ||
      hidden > 4096 || out_dim > 4096 || max_batch > (1u << 18)) {
    set_error("invalid MLP shape");
    return QTN_EINVAL;
  }
  qtn_mlp_t *M = new qtn_mlp_t();
  M->in_dim = (int)in_dim;
  M->hidden = (int)hidden;
  M->nh = (int)n_hidden;
  M->out_dim = (int)out_dim;
  M->max_batch = (int)max_batch;
  M->dims.push_back((int)in_dim);
  for (uint32_t i = 0; i < n_hidden; ++i) M->dims.push_back((int)hidden);
  M->dims.push_back((int)out_dim);
  const int L = (int)M->dims.size() - 1;
  long off = 0, aoff = 0;
  int widest = 0;
  for (int l = 0; l < L; ++l) {
    M->woff.push_back(off);
    off += (long)M->dims[l] * M->dims[l + 1];
    M->boff.push_back(off);
    off += M->dims[l + 1];
    M->zoff.push_back(aoff);
    aoff += (long)max_batch * M->dims[l + 1];
    M->hoff.push_back(aoff);
    aoff += (long)max_batch * M->dims[l + 1];
    widest = std::max(widest, M->dims[l + 1]);
  }
  M->nparams = off;
  // He initialisation from SplitMix64 through a Box-Muller pair
  std::vector<float> host(off, 0.f);
  SplitMix64 rng(seed);
  auto uni = [&]() { return ((double)(rng.next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  for (int l = 0; l < L; ++l) {
    const double sd = std::sqrt(2.0 / M->dims[l]);
    for (long i = 0; i < (long)M->dims[l] * M->dims[l + 1]; ++i) {
      const double u1 = uni(), u2 = uni();
      host[M->woff[l] + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  }
  M->x_mean.assign(in_dim, 0.f);
  M->x_std.assign(in_dim, 1.f);
  M->y_mean.assign(out_dim, 0.f);
  M->y_std.assign(out_dim, 1.f);
  hipError_t e = hipGetDevice(&M->device);
  auto alloc = [&](float **p, long n) {
    if (e == hipSuccess) e = hipMalloc((void **)p, std::max<long>(n, 1) * sizeof(float));
    if (e == hipSuccess) e = hipMemset(*p, 0, std::max<long>(n, 1) * sizeof(float));
  };
  alloc(&M->params, off);
  alloc(&M->grads, off);
  alloc(&M->m, off);
  alloc(&M->v, off);
  alloc(&M->acts, aoff);
  alloc(&M->dz[0], (long)max_batch * std::max(widest, (int)in_dim));
  alloc(&M->dz[1], (long)max_batch * std::max(widest, (int)in_dim));
  alloc(&M->dy, (long)max_batch * out_dim);
  alloc(&M->loss, 1);
  alloc(&M->xin, (long)max_batch * in_dim);
  alloc(&M->tin, (long)max_batch * out_dim);
  if (e == hipSuccess) e = hipMemcpy(M->params, host.data(), off * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    mlp_free(M);
    delete M;
    return mlp_fail(e, "MLP allocation");
  }
  *out = M;
  return QTN_OK;
}

extern "C" void qtn_mlp_destroy(qtn_mlp_t *M) {
  if (!M) return;
  mlp_free(M);
  delete M;
}

extern "C" int qtn_mlp_num_params(const qtn_mlp_t *M, uint64_t *count) {
  if (!M || !count) return QTN_EINVAL;
  *count = (uint64_t)M->nparams;
  return QTN_OK;
}

static int copy_params(const qtn_mlp_t *M, const float *src, float *host, uint64_t cap) {
  if (!M || !host || cap < (uint64_t)M->nparams) {
    set_error("capacity too small");
    return QTN_EINVAL;
  }
  MLP_TRY(hipMemcpy(host, src, M->nparams * sizeof(float), hipMemcpyDeviceToHost));
  return QTN_OK;
}

extern "C" int qtn_mlp_get_params(const qtn_mlp_t *M, float *host, uint64_t cap) {
  return copy_params(M, M ? M->params : nullptr, host, cap);
}

extern "C" int qtn_mlp_get_grads(const qtn_mlp_t *M, float *host, uint64_t cap) {
  return copy_params(M, M ? M->grads : nullptr, host, cap);
}

extern "C" int qtn_mlp_set_params(qtn_mlp_t *M, const float *host, uint64_t count) {
  if (!M || !host || count != (uint64_t)M->nparams) {
    set_error("parameter count mismatch");
    return QTN_EINVAL;
  }
  MLP_TRY(hipMemcpy(M->params, host, count * sizeof(float), hipMemcpyHostToDevice));
  MLP_TRY(hipMemset(M->m, 0, count * sizeof(float)));
  MLP_TRY(hipMemset(M->v, 0, count * sizeof(float)));
  M->t = 0;
  return QTN_OK;
}

extern "C" int qtn_mlp_set_normalization(qtn_mlp_t *M, const float *x_mean, const float *x_std,
                                         const float *y_mean, const float *y_std) {
  if (!M || !x_mean || !x_std || !y_mean || !y_std) return QTN_EINVAL;
  M->x_mean.assign(x_mean, x_mean + M->in_dim);
  M->x_std.assign(x_std, x_std + M->in_dim);
  M->y_mean.assign(y_mean, y_mean + M->out_dim);
  M->y_std.assign(y_std, y_std + M->out_dim);
  return QTN_OK;
}

static void gemm(const float *A, int a_m, int a_k, const float *B, int b_k, int b_n, int Mr, int N,
                 int K, const float *bias, const float *mask, int ld_mask, float *Z, int ldz, float *H,
                 hipStream_t s) {
  dim3 grid((N + 15) / 16, (Mr + 15) / 16);
  hipLaunchKernelGGL(gemm_f32_mfma, grid, dim3(64), 0, s, A, a_m, a_k, B, b_k, b_n, Mr, N, K, bias,
                     mask, ld_mask, Z, ldz, H);
}

// Forward pass on device input x (batch x in_dim); the output layer is linear.
static void forward(qtn_mlp_t *M, const float *x, int batch, hipStream_t s) {
  const int L = (int)M->dims.size() - 1;
  const float *h = x;
  for (int l = 0; l < L; ++l) {
    const int din = M->dims[l], dout = M->dims[l + 1];
    float *Z = M->acts + M->zoff[l];
    float *H = (l + 1 < L) ? M->acts + M->hoff[l] : nullptr;
    gemm(h, din, 1, M->params + M->woff[l], dout, 1, batch, dout, din, M->params + M->boff[l],
         nullptr, 0, Z, dout, H, s);
    h = H;
  }
}

extern "C" int qtn_mlp_forward(qtn_mlp_t *M, const float *x_dev, uint32_t batch, float *y_dev,
                               void *stream) {
  if (!M || !x_dev || !y_dev || batch == 0 || (int)batch > M->max_batch) {
    set_error("invalid forward arguments");
    return QTN_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  forward(M, x_dev, (int)batch, s);
  const int L = (int)M->dims.size() - 1;
  MLP_TRY(hipMemcpyAsync(y_dev, M->acts + M->zoff[L - 1], (size_t)batch * M->out_dim * sizeof(float),
                         hipMemcpyDeviceToDevice, s));
  MLP_TRY(hipGetLastError());
  return QTN_OK;
}

extern "C" int qtn_mlp_train_step(qtn_mlp_t *M, const float *x_dev, const float *t_dev,
                                  uint32_t batch, float lr, void *stream, float *loss_out) {
  if (!M || !x_dev || !t_dev || batch == 0 || (int)batch > M->max_batch) {
    set_error("invalid training arguments");
    return QTN_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int B = (int)batch;
  const int L = (int)M->dims.size() - 1;
  forward(M, x_dev, B, s);
  const float *Y = M->acts + M->zoff[L - 1];
  hipLaunchKernelGGL(mse_loss, dim3(1), dim3(256), 0, s, Y, t_dev, B * M->out_dim, M->dy, M->loss);
  // backward: dZ of layer l lives in `cur`
  const float *cur = M->dy;
  int pp = 0;
  for (int l = L - 1; l >= 0; --l) {
    const int din = M->dims[l], dout = M->dims[l + 1];
    const float *Hin = (l == 0) ? x_dev : M->acts + M->hoff[l - 1];
    // dW_l = H_in^T dZ  (din x dout, summed over the batch)
    gemm(Hin, 1, din, cur, dout, 1, din, dout, B, nullptr, nullptr, 0, M->grads + M->woff[l], dout,
         nullptr, s);
    hipLaunchKernelGGL(colsum, dim3((dout + 255) / 256), dim3(256), 0, s, cur, B, dout, dout,
                       M->grads + M->boff[l]);
    if (l > 0) {
      // dZ_{l-1} = (dZ W_l^T) * (Z_{l-1} > 0)
      float *nxt = M->dz[pp];
      gemm(cur, dout, 1, M->params + M->woff[l], 1, dout, B, din, dout, nullptr,
           M->acts + M->zoff[l - 1], din, nxt, din, nullptr, s);
      cur = nxt;
      pp ^= 1;
    }
  }
  M->t += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)M->t), c2 = 1.f - std::pow(b2, (float)M->t);
  if (lr > 0.f)
    hipLaunchKernelGGL(adam_step, dim3(256), dim3(256), 0, s, M->params, M->grads, M->m, M->v,
                       M->nparams, lr, b1, b2, 1e-8f, c1, c2);
  MLP_TRY(hipGetLastError());
  if (loss_out) {
    MLP_TRY(hipMemcpyAsync(loss_out, M->loss, sizeof(float), hipMemcpyDeviceToHost, s));
    MLP_TRY(hipStreamSynchronize(s));
  }
  return QTN_OK;
}

// Host-side prediction for the guided search: normalise, run, denormalise.
static int predict_host(qtn_mlp_t *M, const std::vector<float> &feat, int n, std::vector<float> &out) {
  out.assign((size_t)n * M->out_dim, 0.f);
  std::vector<float> x((size_t)M->max_batch * M->in_dim);
  for (int b0 = 0; b0 < n; b0 += M->max_batch) {
    const int bn = std::min(M->max_batch, n - b0);
    for (int i = 0; i < bn; ++i)
      for (int j = 0; j < M->in_dim; ++j)
        x[(size_t)i * M->in_dim + j] =
            (feat[(size_t)(b0 + i) * M->in_dim + j] - M->x_mean[j]) / M->x_std[j];
    MLP_TRY(hipMemcpy(M->xin, x.data(), (size_t)bn * M->in_dim * sizeof(float), hipMemcpyHostToDevice));
    forward(M, M->xin, bn, nullptr);
    const int L = (int)M->dims.size() - 1;
    std::vector<float> y((size_t)bn * M->out_dim);
    MLP_TRY(hipMemcpy(y.data(), M->acts + M->zoff[L - 1], y.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int i = 0; i < bn; ++i)
      for (int j = 0; j < M->out_dim; ++j)
        out[(size_t)(b0 + i) * M->out_dim + j] = y[(size_t)i * M->out_dim + j] * M->y_std[j] + M->y_mean[j];
  }
  return QTN_OK;
}

extern "C" int qtn_cut_search(const qtn_graph *graph, uint32_t p, uint32_t k, int32_t pop,
                              int32_t iters, uint64_t seed, qtn_mlp_t *model,
                              int32_t offspring_factor, uint32_t *cut_out, qtn_search_stats *stats) {
  set_error("");
  if (!cut_out && k) {
    set_error("NULL output");
    return QTN_EINVAL;
  }
  CostContext *ctx = cost_context_new(graph, p);
  if (!ctx) {
    set_error("invalid graph");
    return QTN_EINVAL;
  }
  const int V = cost_context_vars(ctx);
  if ((int)k >= V || pop < 2 || iters < 0) {
    cost_context_free(ctx);
    set_error("need k < n*p and population >= 2");
    return QTN_EINVAL;
  }
  if (model && model->in_dim != QTN_COST_FEATURES) {
    cost_context_free(ctx);
    set_error("model input width differs from the feature count");
    return QTN_EINVAL;
  }
  const auto t0 = std::chrono::steady_clock::now();
  if (!model) {
    // Algorithm 1 itself, as the planner runs it
    CutResult r = ga_cut_search(cost_context_adj(ctx), (int)k, pop, iters, seed);
    for (uint32_t i = 0; i < k; ++i) cut_out[i] = (uint32_t)r.cut[i];
    if (stats) {
      stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      stats->exact_evals = r.evals;
      stats->model_evals = 0;
      stats->width = r.width;
      stats->log2_cost = std::log2((double)r.work) + (double)k;
    }
    cost_context_free(ctx);
    return QTN_OK;
  }
  const int N = pop, T = iters, M = (int)k;
  SplitMix64 rng(seed);
  std::map<std::vector<uint32_t>, std::pair<int32_t, double>> cache;
  uint64_t model_evals = 0;
  auto exact = [&](const std::vector<uint32_t> &ind) {
    std::vector<uint32_t> s(ind);
    std::sort(s.begin(), s.end());
    auto it = cache.find(s);
    if (it != cache.end()) return it->second;
    std::pair<int32_t, double> r;
    cost_exact(ctx, s.data(), (uint32_t)s.size(), r.first, r.second);
    cache.emplace(s, r);
    return r;
  };
  auto less = [&](const std::vector<uint32_t> &a, const std::vector<uint32_t> &b) {
    auto fa = exact(a), fb = exact(b);
    if (fa.first != fb.first) return fa.first < fb.first;
    if (fa.second != fb.second) return fa.second < fb.second;
    std::vector<uint32_t> sa(a), sb(b);
    std::sort(sa.begin(), sa.end());
    std::sort(sb.begin(), sb.end());
    return sa < sb;
  };
  auto contains = [](const std::vector<uint32_t> &v, uint32_t u) {
    return std::find(v.begin(), v.end(), u) != v.end();
  };
  auto nonmember = [&](const std::vector<uint32_t> &ind) {
    for (;;) {
      const uint32_t u = (uint32_t)rng.below((uint64_t)V);
      if (!contains(ind, u)) return u;
    }
  };
  std::vector<std::vector<uint32_t>> P;
  for (int i = 0; i < N; ++i) {
    std::vector<uint32_t> ind;
    while ((int)ind.size() < M) {
      const uint32_t u = (uint32_t)rng.below((uint64_t)V);
      if (!contains(ind, u)) ind.push_back(u);
    }
    P.push_back(ind);
  }
  int rc = QTN_OK;
  const int h = M / 2;
  const int F = std::max(1, offspring_factor);
  auto sorted_of = [](const std::vector<uint32_t> &v) {
    std::vector<uint32_t> s(v);
    std::sort(s.begin(), s.end());
    return s;
  };
  for (int t = 0; t <= T && rc == QTN_OK && M > 0; ++t) {
    std::stable_sort(P.begin(), P.end(), less);
    // F x (N-1) offspring: tail crossover of two members (the operator of
    // Algorithm 1, Step 2, on random pairs) and, for half of them, a mutation
    std::vector<std::vector<uint32_t>> cand;
    while ((int)cand.size() < F * (N - 1)) {
      const int a = (int)rng.below((uint64_t)N), b = (int)rng.below((uint64_t)N);
      std::vector<uint32_t> child(P[a]);
      for (int q = M - h; q < M; ++q) child[q] = P[b][q];
      for (int q = 0; q < M; ++q)
        if (std::find(child.begin(), child.begin() + q, child[q]) != child.begin() + q)
          child[q] = nonmember(child);
      if (rng.below(2)) child[rng.below((uint64_t)M)] = nonmember(child);
      cand.push_back(child);
    }
    std::vector<float> feat((size_t)cand.size() * QTN_COST_FEATURES), pred;
    for (size_t i = 0; i < cand.size(); ++i)
      cost_features(ctx, cand[i].data(), (uint32_t)M, feat.data() + i * QTN_COST_FEATURES);
    rc = predict_host(model, feat, (int)cand.size(), pred);
    model_evals += cand.size();
    std::vector<int> idx(cand.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
    const int od = model->out_dim;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
      // predicted peak rank (rounded) first, then predicted log2 cost
      const float rx = std::round(pred[(size_t)x * od]), ry = std::round(pred[(size_t)y * od]);
      if (rx != ry) return rx < ry;
      return pred[(size_t)x * od + 1] < pred[(size_t)y * od + 1];
    });
    // the N best-predicted sets not yet in the population are scored exactly;
    // the population keeps the N best of old and new (exact fitness)
    std::vector<std::vector<uint32_t>> seen;
    for (const auto &ind : P) seen.push_back(sorted_of(ind));
    int taken = 0;
    for (int i : idx) {
      std::vector<uint32_t> sv = sorted_of(cand[i]);
      if (std::find(seen.begin(), seen.end(), sv) != seen.end()) continue;
      seen.push_back(sv);
      (void)exact(cand[i]);
      P.push_back(cand[i]);
      if (++taken == N) break;
    }
    std::stable_sort(P.begin(), P.end(), less);
    P.resize(N);
  }
  std::stable_sort(P.begin(), P.end(), less);
  std::vector<uint32_t> best(P[0]);
  std::sort(best.begin(), best.end());
  for (int i = 0; i < M; ++i) cut_out[i] = best[i];
  if (stats) {
    auto f = exact(best);
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->exact_evals = cache.size();
    stats->model_evals = model_evals;
    stats->width = f.first;
    stats->log2_cost = f.second;
  }
  cost_context_free(ctx);
  return rc;
}
