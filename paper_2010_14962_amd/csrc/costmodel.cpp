// Host side of the learned cut-set cost model: features of candidate cut sets
// and their exact costs (the labels and the fallback), plus the model-guided
// variant of the cut search.  The model only ranks candidates; every cut set
// that is returned is scored by the exact evaluator.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <set>
#include <thread>
#include <vector>

#include "../../include/qtn.h"
#include "costmodel.h"
#include "plan_state.h"

namespace qtn {

// Per-network statistics of the uncut min-fill elimination.
struct BaseStats {
  int V = 0, n = 0, p = 0;
  std::vector<std::vector<int>> adj;
  std::vector<double> deg, pos, bag, fill, nbags, layer;
  int width = 0;
  double log2work = 0;
  std::vector<char> in_max_bag;
};

static BaseStats base_stats(const Network &net) {
  BaseStats b;
  b.adj = line_graph(net);
  b.V = (int)net.nv;
  b.n = (int)net.n;
  b.p = (int)net.p;
  const int V = b.V;
  EliminationResult er = min_fill(b.adj, {});
  b.width = er.width;
  b.log2work = std::log2((double)er.work);
  b.deg.assign(V, 0);
  b.pos.assign(V, 0);
  b.bag.assign(V, 0);
  b.fill.assign(V, 0);
  b.nbags.assign(V, 1);
  b.layer.assign(V, 0);
  b.in_max_bag.assign(V, 0);
  for (int v = 0; v < V; ++v) {
    b.deg[v] = (double)b.adj[v].size();
    b.layer[v] = (double)(v / b.n) / (double)std::max(1, b.p);
  }
  // replay the elimination to count fill edges
  std::vector<std::set<int>> g(V);
  for (int v = 0; v < V; ++v) g[v].insert(b.adj[v].begin(), b.adj[v].end());
  bool marked = false;
  for (size_t i = 0; i < er.order.size(); ++i) {
    const int v = er.order[i];
    const auto &nb = er.nplus[i];
    b.pos[v] = (double)i / (double)V;
    b.bag[v] = (double)nb.size();
    int fill = 0;
    for (size_t a = 0; a < nb.size(); ++a)
      for (size_t c = a + 1; c < nb.size(); ++c)
        if (!g[nb[a]].count(nb[c])) {
          ++fill;
          g[nb[a]].insert(nb[c]);
          g[nb[c]].insert(nb[a]);
        }
    b.fill[v] = (double)fill;
    for (int u : nb) {
      b.nbags[u] += 1;
      g[u].erase(v);
    }
    if (!marked && (int)nb.size() == er.width) {
      marked = true;
      b.in_max_bag[v] = 1;
      for (int u : nb) b.in_max_bag[u] = 1;
    }
  }
  return b;
}

constexpr int kPerVar = 6;

static void features_of(const BaseStats &b, const uint32_t *cut, uint32_t k, float *f) {
  const std::vector<double> *cols[kPerVar] = {&b.deg, &b.pos, &b.bag, &b.fill, &b.nbags, &b.layer};
  int o = 0;
  for (int c = 0; c < kPerVar; ++c) {
    double mn = 1e300, mx = -1e300, sum = 0;
    for (uint32_t i = 0; i < k; ++i) {
      const double x = (*cols[c])[cut[i]];
      mn = std::min(mn, x);
      mx = std::max(mx, x);
      sum += x;
    }
    if (k == 0) mn = mx = 0;
    f[o++] = (float)(k ? sum / k : 0.0);
    f[o++] = (float)mx;
    f[o++] = (float)mn;
    f[o++] = (float)sum;
  }
  int inner = 0, inmax = 0, near = 0;
  for (uint32_t i = 0; i < k; ++i) {
    const int v = (int)cut[i];
    for (uint32_t j = i + 1; j < k; ++j)
      if (std::binary_search(b.adj[v].begin(), b.adj[v].end(), (int)cut[j])) ++inner;
    inmax += b.in_max_bag[v];
    near += b.bag[v] >= b.width - 2 ? 1 : 0;
  }
  f[o++] = (float)b.n;
  f[o++] = (float)b.p;
  f[o++] = (float)k;
  f[o++] = (float)b.width;
  f[o++] = (float)b.log2work;
  f[o++] = (float)(k ? (double)inner / k : 0.0);
  f[o++] = (float)(k ? (double)inmax / k : 0.0);
  f[o++] = (float)(k ? (double)near / k : 0.0);
}

static int build_net(const qtn_graph *graph, uint32_t p, Network &net) {
  if (!graph || graph->n == 0 || p == 0 || (graph->m && !graph->edges)) return QTN_EINVAL;
  net.n = graph->n;
  net.p = p;
  std::set<std::pair<uint32_t, uint32_t>> seen;
  for (uint32_t e = 0; e < graph->m; ++e) {
    uint32_t a = graph->edges[2 * e], c = graph->edges[2 * e + 1];
    if (a >= graph->n || c >= graph->n || a == c) return QTN_EINVAL;
    if (a > c) std::swap(a, c);
    seen.insert({a, c});
  }
  net.edges.assign(seen.begin(), seen.end());
  net.gamma.assign(p, 0.0);
  net.beta.assign(p, 0.0);
  net.B = 1;
  net.bits.assign(graph->n, 0);
  build_network(net);
  return QTN_OK;
}

static int check_sets(const uint32_t *sets, uint32_t n_sets, uint32_t k, int V) {
  if (n_sets && k && !sets) return QTN_EINVAL;
  for (uint64_t i = 0; i < (uint64_t)n_sets * k; ++i)
    if (sets[i] >= (uint32_t)V) return QTN_EINVAL;
  return QTN_OK;
}

// Exact cost of a cut set: width of G - C and log2 of (work * 2^k).
static void exact_cost(const std::vector<std::vector<int>> &adj, const uint32_t *cut, uint32_t k,
                       int32_t &width, double &log2cost) {
  std::vector<int> c(cut, cut + k);
  EliminationResult r = min_fill(adj, c);
  width = r.width;
  log2cost = std::log2((double)r.work) + (double)k;
}

struct CostContext {
  Network net;
  BaseStats base;
};

CostContext *cost_context_new(const qtn_graph *graph, uint32_t p) {
  CostContext *c = new CostContext();
  if (build_net(graph, p, c->net) != QTN_OK) {
    delete c;
    return nullptr;
  }
  c->base = base_stats(c->net);
  return c;
}

void cost_context_free(CostContext *c) { delete c; }

int cost_context_vars(const CostContext *c) { return (int)c->net.nv; }

const std::vector<std::vector<int>> &cost_context_adj(const CostContext *c) { return c->base.adj; }

void cost_features(const CostContext *c, const uint32_t *cut, uint32_t k, float *f) {
  features_of(c->base, cut, k, f);
}

void cost_exact(const CostContext *c, const uint32_t *cut, uint32_t k, int32_t &width,
                double &log2cost) {
  exact_cost(c->base.adj, cut, k, width, log2cost);
}

template <typename F>
static void parallel_for(uint32_t n, int threads, F f) {
  threads = std::max(1, std::min<int>(threads, (int)n));
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&, t]() {
      for (uint32_t i = t; i < n; i += threads) f(i);
    });
  for (auto &th : pool) th.join();
}

}  // namespace qtn

using namespace qtn;

extern "C" int qtn_cost_features(const qtn_graph *graph, uint32_t p, const uint32_t *cut_sets,
                                 uint32_t n_sets, uint32_t k, float *features) {
  Network net;
  if (build_net(graph, p, net) != QTN_OK || (!features && n_sets)) {
    set_error("invalid graph or arguments");
    return QTN_EINVAL;
  }
  if (check_sets(cut_sets, n_sets, k, (int)net.nv) != QTN_OK) {
    set_error("cut variable out of range");
    return QTN_EINVAL;
  }
  BaseStats b = base_stats(net);
  for (uint32_t i = 0; i < n_sets; ++i)
    features_of(b, cut_sets + (uint64_t)i * k, k, features + (uint64_t)i * QTN_COST_FEATURES);
  return QTN_OK;
}

extern "C" int qtn_cost_exact(const qtn_graph *graph, uint32_t p, const uint32_t *cut_sets,
                              uint32_t n_sets, uint32_t k, int32_t *width, double *log2_cost,
                              int32_t threads) {
  Network net;
  if (build_net(graph, p, net) != QTN_OK || (n_sets && (!width || !log2_cost))) {
    set_error("invalid graph or arguments");
    return QTN_EINVAL;
  }
  if (check_sets(cut_sets, n_sets, k, (int)net.nv) != QTN_OK) {
    set_error("cut variable out of range");
    return QTN_EINVAL;
  }
  auto adj = line_graph(net);
  parallel_for(n_sets, threads <= 0 ? 1 : threads, [&](uint32_t i) {
    exact_cost(adj, cut_sets + (uint64_t)i * k, k, width[i], log2_cost[i]);
  });
  return QTN_OK;
}
