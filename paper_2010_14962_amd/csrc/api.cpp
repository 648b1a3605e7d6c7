// C ABI: host-side entry points (plan construction, queries, partial sums).
#include <chrono>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <new>
#include <set>
#include <stdexcept>
#include <string>

#include "../../include/qtn.h"
#include "plan_state.h"

namespace qtn {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace qtn

using namespace qtn;

extern "C" const char *qtn_last_error(void) { return g_err.c_str(); }

extern "C" void qtn_plan_opts_default(qtn_plan_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->k = -1;
  o->max_rank = 0;
  o->k_max = 24;
  o->cut_vars = nullptr;
  o->seed = 0;
  o->ga_pop = 11;   // Sec. IV A: population size 11
  o->ga_iters = 4;  // Sec. IV A: 4 iterations
  o->precision = QTN_FP64;
  o->fuse_chains = 1;
  o->exec_mode = -1;
  o->use_cost_model = 0;
  o->offspring_factor = 16;
  o->cost_model = nullptr;
  o->density_matrix = 0;
}

static int fail(int code, const std::string &msg) {
  set_error(msg);
  return code;
}

// Everything after the network: line graph, cut search (Algorithm 1, or the
// model-guided search with use_cost_model; for the density-matrix form on
// the graph of (ket, bra) pairs), min-fill order, schedule, storage and
// execution plans.  graph and p describe a QAOA network for the cost model
// (graph NULL for general circuits).  On failure P is freed and the error
// code returned.
static int plan_rest(qtn_plan_t *P, const qtn_plan_opts &opts, const qtn_graph *graph, uint32_t p) {
  try {
    Network &net = P->net;
    auto adj = line_graph(net);
    const int V = (int)net.nv;
    auto t0 = std::chrono::steady_clock::now();
    if (opts.cut_vars) {
      if (opts.k < 0 || opts.k > V) {
        delete P;
        return fail(QTN_EINVAL, "explicit cut needs 0 <= k <= n*p");
      }
      std::set<int> cs;
      for (int i = 0; i < opts.k; ++i) {
        if (opts.cut_vars[i] >= (uint32_t)V) {
          delete P;
          return fail(QTN_EINVAL, "cut variable out of range");
        }
        cs.insert((int)opts.cut_vars[i]);
      }
      if ((int)cs.size() != opts.k) {
        delete P;
        return fail(QTN_EINVAL, "repeated cut variable");
      }
      P->cut.assign(cs.begin(), cs.end());
    } else {
      // Cut search of size k: Algorithm 1 (Sec. III B) with exact fitness, or
      // with use_cost_model the same operators with offspring ranked by the
      // learned model and only the best ones scored exactly; either way the
      // returned set carries its exact (width, work) from min-fill on G - C.
      int search_rc = QTN_OK;
      auto search = [&](int k) {
        CutResult r;
        if (!opts.use_cost_model || k == 0) return ga_cut_search(adj, k, opts.ga_pop, opts.ga_iters, opts.seed);
        std::vector<uint32_t> c(k);
        qtn_search_stats st;
        search_rc = qtn_cut_search(graph, p, (uint32_t)k, opts.ga_pop, opts.ga_iters, opts.seed,
                                   opts.cost_model, opts.offspring_factor, c.data(), &st);
        if (search_rc != QTN_OK) return r;
        r.cut.assign(c.begin(), c.end());
        std::sort(r.cut.begin(), r.cut.end());
        const EliminationResult e = min_fill(adj, r.cut);  // exact re-score
        r.width = e.width;
        r.work = e.work;
        r.evals = st.exact_evals;
        return r;
      };
      if (opts.use_cost_model && !opts.cost_model) {
        delete P;
        return fail(QTN_EINVAL, "use_cost_model needs a cost_model");
      }
      if (opts.use_cost_model && opts.offspring_factor < 1) {
        delete P;
        return fail(QTN_EINVAL, "offspring_factor must be >= 1");
      }
      bool found = false;
      if (opts.k >= 0) {
        if (opts.k > V || (opts.use_cost_model && opts.k == V)) {
          delete P;
          return fail(QTN_EINVAL, opts.k > V ? "k > n*p" : "use_cost_model needs k < n*p");
        }
        P->cut = search(opts.k).cut;
        found = true;
      } else {
        for (int k = 0; k <= std::min(opts.k_max, opts.use_cost_model ? V - 1 : V); ++k) {
          CutResult r = search(k);
          if (search_rc != QTN_OK) break;
          // density-matrix form: a pair width w means binary ranks up to 2 w
          const int rank = opts.density_matrix ? 2 * r.width : r.width;
          if (opts.max_rank <= 0 || rank <= opts.max_rank) {
            P->cut = r.cut;
            found = true;
            break;
          }
        }
      }
      if (search_rc != QTN_OK) {
        const std::string m = g_err;
        delete P;
        return fail(search_rc, "cut search: " + m);
      }
      if (!found) {
        delete P;
        return fail(QTN_ERANK, "no cut set of size <= k_max meets max_rank");
      }
    }
    P->search_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (P->cut.size() > 30) {
      delete P;
      return fail(QTN_EINVAL, "at most 30 cut variables");
    }
    EliminationResult er = min_fill(adj, P->cut);
    P->order = er.order;
    P->mf_width = er.width;
    P->work = er.work;
    if (opts.density_matrix) {
      // Sec. II A, Sec. III A: every 4-valued edge of the density-matrix
      // network is the pair (v, v + n p) of a ket variable and its bra copy.
      // The search and the order above ran on the graph of those pairs; a
      // cut edge fixes both variables of its pair (4 slices per cut) and the
      // two variables of a pair are eliminated one after the other.
      if (2 * P->cut.size() > 30) {
        delete P;
        return fail(QTN_EINVAL, "at most 15 density-matrix cuts");
      }
      net.dm = true;
      build_network(net);
      std::vector<int> cut2(P->cut);
      for (int c : P->cut) cut2.push_back(c + V);
      P->cut = cut2;
      std::vector<int> ord;
      for (int v : er.order) {
        ord.push_back(v);
        ord.push_back(v + V);
      }
      P->order = ord;
    }
    P->precision = opts.precision;
    P->popts.precision = opts.precision;
    P->popts.fuse_chains = opts.fuse_chains != 0;
    P->sched = build_schedule(net, P->cut, P->order, P->popts);
    P->f64_below_rank = assign_storage(P->sched, P->precision);
    P->exec_mode = opts.exec_mode;
    P->exec[MODE_WIDE] = build_exec(P->sched, MODE_WIDE, kLdsBudget);
    P->exec[MODE_SLICE] = build_exec(P->sched, MODE_SLICE, kLdsBudget);
    for (int m = 0; m < 2; ++m) {
      P->scaled[m] = false;
      if (P->precision == QTN_FP64) continue;
      for (size_t t = 0; t < P->sched.tensors.size(); ++t) {
        const Tensor &T = P->sched.tensors[t];
        const int loc = P->exec[m].loc[t];
        if (!T.leaf && !T.f64 && (loc == LOC_GLOBAL || loc == LOC_SCRATCH)) P->scaled[m] = true;
      }
    }
    if (const char *e = std::getenv("QTN_PLAN_REPORT"); e && e[0] == '1') {
      // launch structure of both execution modes, for tuning
      for (int m = 0; m < 2; ++m) {
        const ExecPlan &X = P->exec[m];
        std::fprintf(stderr, "qtn plan: mode %d, %zu programs, %zu launches, program LDS %u B\n", m,
                     X.programs.size(), X.launches.size(), X.lds_bytes);
        for (size_t i = 0; i < X.programs.size(); ++i) {
          const Program &pr = X.programs[i];
          int nleaf = 0;
          for (int st : pr.steps)
            for (int in : P->sched.steps[st].in) nleaf += P->sched.tensors[in].leaf ? 1 : 0;
          std::fprintf(stderr, "  program %zu: %zu steps, %zu of %d factors and %zu workspace tensors staged, LDS %u B\n",
                       i, pr.steps.size(), pr.staged.size(), nleaf, pr.staged_global.size(), pr.lds_bytes);
        }
      }
    }
    if (opts.max_rank > 0 && P->sched.width > opts.max_rank) {
      delete P;
      return fail(QTN_ERANK, "cut set does not meet max_rank");
    }
  } catch (const std::bad_alloc &) {
    delete P;
    return fail(QTN_ENOMEM, "host allocation");
  } catch (const std::exception &e) {
    delete P;
    return fail(QTN_EINVAL, e.what());
  }
  return QTN_OK;
}

extern "C" int qtn_plan(const qtn_graph *graph, uint32_t p, const double *gamma,
                        const double *beta, const uint8_t *bitstrings,
                        uint32_t n_bitstrings, const qtn_plan_opts *opts_in,
                        qtn_plan_t **out) {
  set_error("");
  if (!out) return fail(QTN_EINVAL, "out is NULL");
  *out = nullptr;
  qtn_plan_opts opts;
  if (opts_in)
    opts = *opts_in;
  else
    qtn_plan_opts_default(&opts);
  if (!graph || !gamma || !beta || !bitstrings)
    return fail(QTN_EINVAL, "NULL argument");
  if (graph->n == 0 || (graph->m > 0 && !graph->edges))
    return fail(QTN_EINVAL, "empty graph");
  if (p == 0 || p > 64) return fail(QTN_EINVAL, "p must be in [1, 64]");
  if (n_bitstrings == 0) return fail(QTN_EINVAL, "no bitstrings");
  if ((uint64_t)graph->n * p > 4096) return fail(QTN_EINVAL, "too many variables");
  if (opts.precision == QTN_3XBF16)
    return fail(QTN_EINVAL, "split-BF16 products need dense steps; no step of these schedules is dense");
  if (opts.precision < QTN_FP64 || opts.precision > QTN_3XBF16)
    return fail(QTN_EINVAL, "unknown precision");
  for (uint32_t l = 0; l < p; ++l)
    if (!std::isfinite(gamma[l]) || !std::isfinite(beta[l]))
      return fail(QTN_EINVAL, "non-finite angle");
  std::set<std::pair<uint32_t, uint32_t>> seen;
  for (uint32_t e = 0; e < graph->m; ++e) {
    uint32_t a = graph->edges[2 * e], b = graph->edges[2 * e + 1];
    if (a >= graph->n || b >= graph->n) return fail(QTN_EINVAL, "edge vertex out of range");
    if (a == b) return fail(QTN_EINVAL, "self-loop");
    if (a > b) std::swap(a, b);
    if (!seen.insert({a, b}).second) return fail(QTN_EINVAL, "repeated edge");
  }
  for (uint64_t i = 0; i < (uint64_t)n_bitstrings * graph->n; ++i)
    if (bitstrings[i] > 1) return fail(QTN_EINVAL, "bitstring byte not 0/1");

  qtn_plan_t *P = new (std::nothrow) qtn_plan_t();
  if (!P) return fail(QTN_ENOMEM, "host allocation");
  try {
    Network &net = P->net;
    net.n = graph->n;
    net.p = p;
    net.edges.assign(seen.begin(), seen.end());
    net.gamma.assign(gamma, gamma + p);
    net.beta.assign(beta, beta + p);
    net.B = n_bitstrings;
    net.bits.assign(bitstrings, bitstrings + (size_t)n_bitstrings * graph->n);
    build_network(net);
    if (int rc = plan_rest(P, opts, graph, p)) return rc;   // frees P on failure
  } catch (const std::bad_alloc &) {
    delete P;
    return fail(QTN_ENOMEM, "host allocation");
  } catch (const std::exception &e) {
    delete P;
    return fail(QTN_EINVAL, e.what());
  }
  *out = P;
  return QTN_OK;
}

extern "C" int qtn_plan_circuit(uint32_t n, const qtn_gate *gates, uint32_t n_gates,
                                const uint8_t *bitstrings, uint32_t n_bitstrings,
                                const qtn_plan_opts *opts_in, qtn_plan_t **out) {
  set_error("");
  if (!out) return fail(QTN_EINVAL, "out is NULL");
  *out = nullptr;
  qtn_plan_opts opts;
  if (opts_in)
    opts = *opts_in;
  else
    qtn_plan_opts_default(&opts);
  if (n == 0 || n > 4096 || !bitstrings || (n_gates && !gates)) return fail(QTN_EINVAL, "NULL argument or no qubits");
  if (n_bitstrings == 0) return fail(QTN_EINVAL, "no bitstrings");
  if (opts.precision == QTN_3XBF16)
    return fail(QTN_EINVAL, "split-BF16 products need dense steps; no step of these schedules is dense");
  if (opts.precision < QTN_FP64 || opts.precision > QTN_3XBF16) return fail(QTN_EINVAL, "unknown precision");
  if (opts.density_matrix) return fail(QTN_EINVAL, "the density-matrix form is built for QAOA plans only");
  if (opts.use_cost_model) return fail(QTN_EINVAL, "the cost model is trained on QAOA networks only");
  std::vector<GateSpec> gs(n_gates);
  for (uint32_t g = 0; g < n_gates; ++g) {
    const qtn_gate &G = gates[g];
    if (G.nq < 1 || G.nq > 2) return fail(QTN_EINVAL, "gate " + std::to_string(g) + ": 1 or 2 qubits");
    for (uint32_t j = 0; j < G.nq; ++j)
      if (G.q[j] >= n) return fail(QTN_EINVAL, "gate " + std::to_string(g) + ": qubit out of range");
    if (G.nq == 2 && G.q[0] == G.q[1]) return fail(QTN_EINVAL, "gate " + std::to_string(g) + ": repeated qubit");
    const int d = 1 << G.nq;
    gs[g].nq = (int)G.nq;
    gs[g].q[0] = (int)G.q[0];
    gs[g].q[1] = G.nq > 1 ? (int)G.q[1] : -1;
    gs[g].m.resize((size_t)d * d);
    for (int i = 0; i < d * d; ++i) {
      if (!std::isfinite(G.re[i]) || !std::isfinite(G.im[i]))
        return fail(QTN_EINVAL, "gate " + std::to_string(g) + ": non-finite matrix entry");
      gs[g].m[i] = cd(G.re[i], G.im[i]);
    }
  }
  for (uint64_t i = 0; i < (uint64_t)n_bitstrings * n; ++i)
    if (bitstrings[i] > 1) return fail(QTN_EINVAL, "bitstring byte not 0/1");
  qtn_plan_t *P = new (std::nothrow) qtn_plan_t();
  if (!P) return fail(QTN_ENOMEM, "host allocation");
  try {
    Network &net = P->net;
    net.n = n;
    net.p = 0;
    net.B = n_bitstrings;
    net.bits.assign(bitstrings, bitstrings + (size_t)n_bitstrings * n);
    build_circuit_network(net, gs);
    if (net.nv > 4096) {
      delete P;
      return fail(QTN_EINVAL, "too many wire variables");
    }
  } catch (const std::bad_alloc &) {
    delete P;
    return fail(QTN_ENOMEM, "host allocation");
  }
  if (int rc = plan_rest(P, opts, nullptr, 0)) return rc;   // frees P on failure
  *out = P;
  return QTN_OK;
}

extern "C" void qtn_plan_destroy(qtn_plan_t *plan) {
  if (!plan) return;
  device_state_free(plan->dev);
  noalloc_state_free(plan->na);
  delete plan;
}

extern "C" int qtn_plan_query(const qtn_plan_t *P, qtn_plan_info *info) {
  if (!P || !info) return fail(QTN_EINVAL, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n = P->net.n;
  info->p = P->net.p;
  info->n_vars = P->net.nv;
  info->n_bitstrings = P->net.B;
  info->k = (int32_t)P->cut.size();
  info->width = P->sched.width;
  info->n_steps = (int32_t)P->sched.steps.size();
  info->n_tensors = (int32_t)P->sched.tensors.size();
  Costs c = schedule_costs(P->sched, P->net.B, 1);
  // slice-invariant work is shared by the 2^k slices of an amplitude
  const double nsl = std::ldexp(1.0, (int)P->cut.size());
  info->log2_flops = std::log2(std::max(1.0, c.flops_per_slice + c.flops_hoisted / nsl));
  info->bytes_per_slice = c.bytes_per_slice + c.bytes_hoisted / nsl;
  info->flops_hoisted = c.flops_hoisted;
  info->work = (double)P->work;
  info->prefactor = P->net.prefactor;
  info->search_seconds = P->search_seconds;
  info->precision = P->precision;
  info->f64_below_rank = P->f64_below_rank;
  info->n_programs_wide = (int32_t)P->exec[MODE_WIDE].programs.size();
  info->n_launches_wide = (int32_t)P->exec[MODE_WIDE].launches.size();
  info->slice_lds_bytes = P->exec[MODE_SLICE].lds_bytes;
  info->slice_scratch_bytes = (double)P->exec[MODE_SLICE].scratch_per_wg;
  info->mf_width = P->mf_width;
  info->rescaled = (P->scaled[MODE_WIDE] ? 1 : 0) | (P->scaled[MODE_SLICE] ? 2 : 0);
  return QTN_OK;
}

extern "C" int qtn_plan_cut(const qtn_plan_t *P, uint32_t *cut, uint32_t cap) {
  if (!P || (!cut && !P->cut.empty())) return fail(QTN_EINVAL, "NULL argument");
  if (cap < P->cut.size()) return fail(QTN_EINVAL, "capacity too small");
  for (size_t i = 0; i < P->cut.size(); ++i) cut[i] = (uint32_t)P->cut[i];
  return QTN_OK;
}

extern "C" int qtn_plan_order(const qtn_plan_t *P, uint32_t *order, uint32_t cap) {
  if (!P || !order) return fail(QTN_EINVAL, "NULL argument");
  if (cap < P->order.size()) return fail(QTN_EINVAL, "capacity too small");
  for (size_t i = 0; i < P->order.size(); ++i) order[i] = (uint32_t)P->order[i];
  return QTN_OK;
}

extern "C" int qtn_plan_export(const qtn_plan_t *P, int32_t *steps, uint32_t step_cap,
                               int32_t *tensors, uint32_t tensor_cap) {
  if (!P) return fail(QTN_EINVAL, "NULL plan");
  const Schedule &S = P->sched;
  if (steps) {
    if (step_cap < S.steps.size()) return fail(QTN_EINVAL, "step capacity too small");
    for (size_t t = 0; t < S.steps.size(); ++t) {
      const Step &st = S.steps[t];
      int32_t *r = steps + t * QTN_STEP_REC;
      for (int j = 0; j < QTN_STEP_REC; ++j) r[j] = -1;
      r[0] = st.out;
      r[1] = (int32_t)st.in.size();
      r[2] = st.nk;
      r[3] = st.rC;
      r[4] = st.cls;
      for (size_t i = 0; i < st.in.size(); ++i) {
        r[5 + i] = st.in[i];
        r[13 + i] = (int32_t)st.mask[i];
      }
      r[21] = (st.bdep ? 1 : 0) | (st.sdep ? 2 : 0);
      r[22] = st.nk > 0 ? st.kappa[0] : -1;
    }
  }
  if (tensors) {
    if (tensor_cap < S.tensors.size()) return fail(QTN_EINVAL, "tensor capacity too small");
    for (size_t t = 0; t < S.tensors.size(); ++t) {
      const Tensor &T = S.tensors[t];
      int32_t *r = tensors + t * QTN_TENSOR_REC;
      for (int j = 0; j < QTN_TENSOR_REC; ++j) r[j] = -1;
      if (T.rank() > QTN_TENSOR_REC - 4) return fail(QTN_EINVAL, "tensor rank too large to export");
      r[0] = T.rank();
      r[1] = T.leaf ? 0 : 1;
      r[2] = (T.bdep ? 1 : 0) | (T.sdep ? 2 : 0) | (T.f64 ? 4 : 0);
      r[3] = (int32_t)T.selmask;
      for (int j = 0; j < T.rank(); ++j) r[4 + j] = T.vars[j];
    }
  }
  return QTN_OK;
}

extern "C" int qtn_plan_kappa(const qtn_plan_t *P, int32_t step, int32_t *kappa, uint32_t cap) {
  if (!P || !kappa || step < 0 || step >= (int32_t)P->sched.steps.size())
    return fail(QTN_EINVAL, "bad argument");
  const Step &st = P->sched.steps[step];
  if (cap < st.kappa.size()) return fail(QTN_EINVAL, "capacity too small");
  for (size_t i = 0; i < st.kappa.size(); ++i) kappa[i] = st.kappa[i];
  return QTN_OK;
}

extern "C" int qtn_plan_index_table(const qtn_plan_t *P, int32_t step, int32_t input,
                                    uint32_t *table, uint32_t cap, uint32_t *count) {
  if (!P || step < 0 || step >= (int32_t)P->sched.steps.size())
    return fail(QTN_EINVAL, "bad step");
  const Step &st = P->sched.steps[step];
  if (input < 0 || input >= (int32_t)st.in.size()) return fail(QTN_EINVAL, "bad input");
  InputTables t = input_tables(st.mask[input], st.rC, st.nk);
  uint32_t need = 256 + 16 + 2 + (uint32_t)t.kap.size();
  if (count) *count = need;
  if (!table) return QTN_OK;
  if (cap < need) return fail(QTN_EINVAL, "capacity too small");
  std::memcpy(table, t.lo, 256 * 4);
  std::memcpy(table + 256, t.mid, 16 * 4);
  table[272] = t.hi_mask;
  table[273] = t.hi_shift;
  for (size_t k = 0; k < t.kap.size(); ++k) table[274 + k] = t.kap[k];
  return QTN_OK;
}

extern "C" int qtn_plan_leaf_values(const qtn_plan_t *P, int32_t tensor, double *values,
                                    uint64_t cap, uint64_t *count) {
  if (!P || tensor < 0 || tensor >= (int32_t)P->sched.tensors.size())
    return fail(QTN_EINVAL, "bad tensor");
  const Tensor &T = P->sched.tensors[tensor];
  if (!T.leaf) return fail(QTN_EINVAL, "not a leaf");
  if (count) *count = T.values.size();
  if (!values) return QTN_OK;
  if (cap < T.values.size()) return fail(QTN_EINVAL, "capacity too small");
  for (size_t i = 0; i < T.values.size(); ++i) {
    values[2 * i] = T.values[i].real();
    values[2 * i + 1] = T.values[i].imag();
  }
  return QTN_OK;
}

namespace qtn {
uint64_t wg_slots_for(const qtn_plan_t *P, int mode, uint64_t S) {
  if (mode != MODE_SLICE) return 0;
  const Program &pr = P->exec[MODE_SLICE].programs[0];
  const uint64_t items = (pr.bdep ? P->net.B : 1) * (pr.sdep ? S : 1);
  return std::min<uint64_t>(items, kMaxWorkgroups);
}

// Automatic choice: wide mode.  Measured on MI355X it beats slice mode on
// every workload here, also where a whole slice fits in LDS (n=40, p=2,
// 32 bitstrings x 256 slices: 1.7 ms against 2.1 ms per contraction; n=80,
// p=2, 65,536 slices: 0.72 s against 4.4 s), because its grid-wide steps
// batch thousands of instances per launch.  Slice mode stays selectable.
int choose_mode(const qtn_plan_t *P, uint64_t S) {
  (void)S;
  if (P->exec_mode == MODE_WIDE || P->exec_mode == MODE_SLICE) return P->exec_mode;
  return MODE_WIDE;
}
}  // namespace qtn

static uint64_t clamp_S(const qtn_plan_t *P, uint64_t S) {
  const uint64_t maxS = P->cut.empty() ? 1 : (1ull << P->cut.size());
  return std::min(S, maxS);
}

extern "C" int qtn_plan_workspace_bytes(const qtn_plan_t *P, uint64_t S, uint64_t *bytes) {
  if (!P || !bytes) return fail(QTN_EINVAL, "NULL argument");
  if (S == 0) return fail(QTN_EINVAL, "slices_per_wave must be >= 1");
  S = clamp_S(P, S);
  const int mode = choose_mode(P, S);
  Schedule copy = P->sched;
  try {
    Layout L = layout(copy, P->exec[mode], P->net.B, S, wg_slots_for(P, mode, S));
    // the stream assignment of the launches checks itself as well
    LaunchGraph lg = launch_graph(copy, P->exec[mode], L, P->net.B, S, P->precision != QTN_FP64, 4);
    if (const char *e = std::getenv("QTN_PLAN_REPORT"); e && e[0] == '1') {
      const ExecPlan &X = P->exec[mode];
      std::fprintf(stderr, "qtn launch graph (S=%llu): %d streams\n", (unsigned long long)S, lg.nstreams);
      for (size_t ui = 0; ui < lg.deps.size(); ++ui) {
        const size_t u = (size_t)lg.order[ui];
        std::string what = u == 0 ? "clear exponents"
                           : u + 1 == lg.deps.size() ? "slice sum"
                           : X.launches[u - 1].kind == 0
                               ? "programs x" + std::to_string(X.launches[u - 1].programs.size())
                               : "step " + std::to_string(X.launches[u - 1].step);
        std::string deps;
        for (int d : lg.deps[u]) deps += " " + std::to_string(d);
        std::fprintf(stderr, "  unit %2zu stream %d %-16s after:%s\n", u, lg.stream[u], what.c_str(),
                     deps.c_str());
      }
    }
    *bytes = L.total_bytes;
  } catch (const std::exception &e) {
    return fail(QTN_ESTATE, e.what());
  }
  return QTN_OK;
}

static inline void two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

extern "C" int qtn_partial_combine(const qtn_partial *a, const qtn_partial *b,
                                   qtn_partial *out) {
  if (!a || !b || !out) return fail(QTN_EINVAL, "NULL argument");
  double s, e;
  qtn_partial r;
  two_sum(a->re, b->re, s, e);
  r.re = s;
  r.re_comp = a->re_comp + b->re_comp + e;
  two_sum(a->im, b->im, s, e);
  r.im = s;
  r.im_comp = a->im_comp + b->im_comp + e;
  *out = r;
  return QTN_OK;
}
