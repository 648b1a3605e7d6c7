// Host planner: network (Sec. II A), line graph and min-fill order (Sec. II B),
// cut search (Sec. III B, Algorithm 1) and the slice-invariant contraction
// schedule (Sec. III A: every slice has the same structure, Eq. (2)).
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <map>
#include <set>
#include <numeric>
#include <stdexcept>

namespace qtn {

// ---------------------------------------------------------------------------
// Network: gates of the QAOA circuit as factors over binary index variables.
// ---------------------------------------------------------------------------
void build_network(Network &net) {
  const uint32_t n = net.n, p = net.p;
  net.nv = n * p;
  net.factors.clear();
  net.values.clear();
  double pref = std::pow(2.0, -0.5 * (double)n);  // H^n |0^n> = 2^{-n/2} sum |v>
  auto var = [n](uint32_t q, uint32_t l) { return (int)(l * n + q); };
  for (uint32_t l = 0; l < p; ++l) {
    for (auto &e : net.edges) {
      Factor f{2, {var(e.first, l), var(e.second, l), -1, -1}, 0, (int)l, -1};
      std::vector<cd> v(4);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          double zz = (a == b) ? 1.0 : -1.0;  // eigenvalue of Z_i Z_j
          v[a * 2 + b] = cd(std::cos(net.gamma[l] * zz), -std::sin(net.gamma[l] * zz));
        }
      net.factors.push_back(f);
      net.values.push_back(v);
    }
  }
  auto rx = [](double beta, int a, int b) {
    return a == b ? cd(std::cos(beta), 0.0) : cd(0.0, -std::sin(beta));
  };
  for (uint32_t l = 0; l + 1 < p; ++l) {
    double m = std::max(std::fabs(std::cos(net.beta[l])), std::fabs(std::sin(net.beta[l])));
    for (uint32_t q = 0; q < n; ++q) {
      Factor f{2, {var(q, l + 1), var(q, l), -1, -1}, 1, (int)l, (int)q};
      std::vector<cd> v(4);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) v[a * 2 + b] = rx(net.beta[l], a, b) / m;
      pref *= m;
      net.factors.push_back(f);
      net.values.push_back(v);
    }
  }
  {
    const uint32_t l = p - 1;
    double m = std::max(std::fabs(std::cos(net.beta[l])), std::fabs(std::sin(net.beta[l])));
    for (uint32_t q = 0; q < n; ++q) {
      Factor f{1, {var(q, l), -1, -1, -1}, 2, (int)l, (int)q};
      std::vector<cd> v(2 * net.B);
      for (uint32_t b = 0; b < net.B; ++b) {
        int x = net.bits[(size_t)b * n + q];
        for (int a = 0; a < 2; ++a) v[b * 2 + a] = rx(net.beta[l], x, a) / m;
      }
      pref *= m;
      net.factors.push_back(f);
      net.values.push_back(v);
    }
  }
  net.prefactor = pref;
  if (net.dm) {
    // Markov-Shi tensors: the factor over (ket vars, bra vars) is the ket
    // factor times the conjugate of the same factor on the bra copies, so
    // that the contraction is amplitude times conjugate amplitude.
    const int V = (int)net.nv;
    for (size_t f = 0; f < net.factors.size(); ++f) {
      Factor &F = net.factors[f];
      const int k = F.nv;
      const std::vector<cd> ket = net.values[f];
      const uint32_t nbv = F.kind == 2 ? net.B : 1;
      std::vector<cd> v((size_t)nbv << (2 * k));
      for (uint32_t b = 0; b < nbv; ++b)
        for (int a = 0; a < (1 << k); ++a)
          for (int c = 0; c < (1 << k); ++c)
            v[((size_t)b << (2 * k)) + ((size_t)a << k) + c] = ket[(size_t)b * (1u << k) + a] *
                                                              std::conj(ket[(size_t)b * (1u << k) + c]);
      for (int j = 0; j < k; ++j) F.v[k + j] = F.v[j] + V;
      F.nv = 2 * k;
      net.values[f] = v;
    }
    net.nv = 2 * V;
    net.prefactor = pref * pref;
  }
}

void build_circuit_network(Network &net, const std::vector<GateSpec> &gates) {
  const uint32_t n = net.n;
  net.factors.clear();
  net.values.clear();
  std::vector<int> wire(n);
  int nv = 0;
  for (uint32_t q = 0; q < n; ++q) {
    wire[q] = nv++;
    net.factors.push_back(Factor{1, {wire[q], -1, -1, -1}, 0, 0, (int)q});
    net.values.push_back({cd(1.0, 0.0), cd(0.0, 0.0)});   // |0>
  }
  for (size_t g = 0; g < gates.size(); ++g) {
    const GateSpec &G = gates[g];
    const int d = 1 << G.nq;
    bool diag = true;
    for (int r = 0; r < d; ++r)
      for (int c = 0; c < d; ++c)
        if (r != c && G.m[(size_t)r * d + c] != cd(0.0, 0.0)) diag = false;
    if (diag) {
      // a diagonal gate leaves the wire values unchanged: one factor on the
      // current variables holding the diagonal
      Factor f{G.nq, {wire[G.q[0]], G.nq > 1 ? wire[G.q[1]] : -1, -1, -1}, 0, (int)g, G.q[0]};
      std::vector<cd> v(d);
      for (int r = 0; r < d; ++r) v[r] = G.m[(size_t)r * d + r];
      net.factors.push_back(f);
      net.values.push_back(v);
    } else {
      Factor f{2 * G.nq, {-1, -1, -1, -1}, 0, (int)g, G.q[0]};
      for (int j = 0; j < G.nq; ++j) f.v[G.nq + j] = wire[G.q[j]];   // inputs
      for (int j = 0; j < G.nq; ++j) {
        wire[G.q[j]] = nv++;
        f.v[j] = wire[G.q[j]];                                          // outputs
      }
      // index bits: outputs (first qubit most significant), then inputs
      net.factors.push_back(f);
      net.values.push_back(G.m);
    }
  }
  for (uint32_t q = 0; q < n; ++q) {
    Factor f{1, {wire[q], -1, -1, -1}, 2, 0, (int)q};
    std::vector<cd> v(2 * net.B);
    for (uint32_t b = 0; b < net.B; ++b) {
      const int x = net.bits[(size_t)b * n + q];
      v[b * 2 + 0] = cd(x == 0 ? 1.0 : 0.0, 0.0);
      v[b * 2 + 1] = cd(x == 1 ? 1.0 : 0.0, 0.0);
    }
    net.factors.push_back(f);
    net.values.push_back(v);
  }
  net.nv = (uint32_t)nv;
  net.prefactor = 1.0;
}

std::vector<std::vector<int>> line_graph(const Network &net) {
  std::vector<std::vector<int>> adj(net.nv);
  for (auto &f : net.factors)
    for (int a = 0; a < f.nv; ++a)
      for (int b = 0; b < f.nv; ++b)
        if (a != b) adj[f.v[a]].push_back(f.v[b]);
  for (auto &a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  return adj;
}

// ---------------------------------------------------------------------------
// Min-fill elimination order on bitset adjacency.
// ---------------------------------------------------------------------------
EliminationResult min_fill(const std::vector<std::vector<int>> &adj,
                           const std::vector<int> &removed) {
  const int V = (int)adj.size();
  const int W = (V + 63) / 64;
  std::vector<uint64_t> nb((size_t)V * W, 0);
  std::vector<char> alive(V, 1);
  for (int r : removed) alive[r] = 0;
  int remaining = 0;
  for (int u = 0; u < V; ++u) {
    if (!alive[u]) continue;
    ++remaining;
    for (int w : adj[u])
      if (alive[w]) nb[(size_t)u * W + (w >> 6)] |= 1ull << (w & 63);
  }
  auto row = [&](int u) { return &nb[(size_t)u * W]; };
  EliminationResult res;
  std::vector<int> members;
  while (remaining > 0) {
    int best = -1;
    long long bf = 0, bd = 0;
    for (int u = 0; u < V; ++u) {
      if (!alive[u]) continue;
      const uint64_t *ru = row(u);
      long long deg = 0;
      for (int w = 0; w < W; ++w) deg += __builtin_popcountll(ru[w]);
      long long pairs = 0;
      for (int w = 0; w < W; ++w) {
        uint64_t bits = ru[w];
        while (bits) {
          int a = (w << 6) + __builtin_ctzll(bits);
          bits &= bits - 1;
          const uint64_t *ra = row(a);
          for (int x = 0; x < W; ++x) pairs += __builtin_popcountll(ra[x] & ru[x]);
        }
      }
      long long fill = deg * (deg - 1) / 2 - pairs / 2;
      if (best < 0 || fill < bf || (fill == bf && deg < bd)) {
        best = u;
        bf = fill;
        bd = deg;
      }
    }
    members.clear();
    uint64_t *rb = row(best);
    for (int w = 0; w < W; ++w) {
      uint64_t bits = rb[w];
      while (bits) {
        members.push_back((w << 6) + __builtin_ctzll(bits));
        bits &= bits - 1;
      }
    }
    for (int a : members) {
      uint64_t *ra = row(a);
      for (int w = 0; w < W; ++w) ra[w] |= rb[w];
      ra[a >> 6] &= ~(1ull << (a & 63));
      ra[best >> 6] &= ~(1ull << (best & 63));
    }
    for (int w = 0; w < W; ++w) rb[w] = 0;
    alive[best] = 0;
    --remaining;
    res.order.push_back(best);
    res.nplus.push_back(members);
    res.width = std::max(res.width, (int)members.size());
    res.work += 1ull << (members.size() + 1);
  }
  return res;
}

// ---------------------------------------------------------------------------
// SplitMix64 and Algorithm 1.
// ---------------------------------------------------------------------------
uint64_t SplitMix64::next() {
  uint64_t z = seed + (counter + 1) * 0x9E3779B97F4A7C15ull;
  ++counter;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

namespace {
struct Fit {
  int width;
  uint64_t work;
  std::vector<int> sorted;
  bool operator<(const Fit &o) const {
    if (width != o.width) return width < o.width;
    if (work != o.work) return work < o.work;
    return sorted < o.sorted;
  }
};
}  // namespace

CutResult ga_cut_search(const std::vector<std::vector<int>> &adj, int M, int N,
                        int T, uint64_t seed) {
  const int V = (int)adj.size();
  std::map<std::vector<int>, Fit> cache;
  auto fitness = [&](const std::vector<int> &ind) -> const Fit & {
    std::vector<int> s(ind);
    std::sort(s.begin(), s.end());
    auto it = cache.find(s);
    if (it != cache.end()) return it->second;
    EliminationResult r = min_fill(adj, s);
    Fit f{r.width, r.work, s};
    return cache.emplace(s, f).first->second;
  };
  CutResult out;
  if (M <= 0 || M >= V) {
    std::vector<int> all;
    if (M >= V)
      for (int v = 0; v < V; ++v) all.push_back(v);
    const Fit &f = fitness(all);
    out.cut = f.sorted;
    out.width = f.width;
    out.work = f.work;
    return out;
  }
  SplitMix64 rng(seed);
  auto contains = [](const std::vector<int> &ind, int u) {
    return std::find(ind.begin(), ind.end(), u) != ind.end();
  };
  auto nonmember = [&](const std::vector<int> &ind) {
    for (;;) {
      int u = (int)rng.below((uint64_t)V);
      if (!contains(ind, u)) return u;
    }
  };
  std::vector<std::vector<int>> pop;
  for (int i = 0; i < N; ++i) {
    std::vector<int> ind;
    while ((int)ind.size() < M) {
      int u = (int)rng.below((uint64_t)V);
      if (!contains(ind, u)) ind.push_back(u);
    }
    pop.push_back(ind);
  }
  auto by_fitness = [&](const std::vector<int> &a, const std::vector<int> &b) {
    return fitness(a) < fitness(b);
  };
  const int h = M / 2;
  int t = 0;
  for (;;) {
    std::stable_sort(pop.begin(), pop.end(), by_fitness);          // Step 1
    for (int i = 1; i + 1 < N; i += 2) {                          // Step 2
      auto &a = pop[i], &b = pop[i + 1];
      for (int q = M - h; q < M; ++q) std::swap(a[q], b[q]);
      for (auto *ind : {&a, &b})
        for (int q = 0; q < M; ++q)
          if (std::find(ind->begin(), ind->begin() + q, (*ind)[q]) != ind->begin() + q)
            (*ind)[q] = nonmember(*ind);
    }
    if (N > 1) {                                                  // Step 3
      int j = 1 + (int)rng.below((uint64_t)(N - 1));
      int q = (int)rng.below((uint64_t)M);
      pop[j][q] = nonmember(pop[j]);
    }
    ++t;                                                          // Step 4
    if (t > T) break;
  }
  std::stable_sort(pop.begin(), pop.end(), by_fitness);            // Step 5
  const Fit &f = fitness(pop[0]);
  out.cut = f.sorted;
  out.width = f.width;
  out.work = f.work;
  out.evals = cache.size();
  return out;
}

// ---------------------------------------------------------------------------
// Schedule: bucket elimination with fused multi-input steps.
// ---------------------------------------------------------------------------
uint32_t pext32(uint32_t x, uint32_t mask) {
  uint32_t r = 0;
  int k = 0;
  for (int b = 0; b < 32; ++b)
    if ((mask >> b) & 1u) r |= ((x >> b) & 1u) << k++;
  return r;
}

InputTables input_tables(uint32_t mask, int rC, int nk) {
  InputTables t;
  uint32_t cm = rC >= 32 ? mask : (mask & ((1u << rC) - 1u));
  uint32_t km = rC >= 32 ? 0 : (mask >> rC);
  for (uint32_t c = 0; c < 256; ++c) t.lo[c] = pext32(c, cm & 255u);
  for (uint32_t u = 0; u < 16; ++u) t.mid[u] = pext32(u << 8, cm);
  t.hi_mask = cm >> 12;
  t.hi_shift = (uint32_t)__builtin_popcount(cm & 4095u);
  uint32_t sh = (uint32_t)__builtin_popcount(cm);
  t.kap.resize((size_t)1 << nk);
  for (uint32_t k = 0; k < (1u << nk); ++k) t.kap[k] = pext32(k, km) << sh;
  return t;
}

Schedule build_schedule(const Network &net, const std::vector<int> &cut,
                        const std::vector<int> &order, const PlanOpts &o) {
  const int V = (int)net.nv;
  Schedule s;
  std::vector<int> pos(V, -1), cutbit(V, -1);
  for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int)i;
  for (size_t b = 0; b < cut.size(); ++b) cutbit[cut[b]] = (int)b;
  for (int v = 0; v < V; ++v)
    if ((pos[v] < 0) == (cutbit[v] < 0))
      throw std::runtime_error("order and cut must partition the variables");
  auto by_pos = [&](int a, int b) { return pos[a] < pos[b]; };

  // Group every factor with the earliest-eliminated of its free variables.
  std::vector<std::vector<int>> group(V);
  std::vector<int> scalar_group;
  for (size_t f = 0; f < net.factors.size(); ++f) {
    const Factor &F = net.factors[f];
    int first = -1;
    for (int j = 0; j < F.nv; ++j)
      if (pos[F.v[j]] >= 0 && (first < 0 || pos[F.v[j]] < pos[first])) first = F.v[j];
    if (first < 0)
      scalar_group.push_back((int)f);
    else
      group[first].push_back((int)f);
  }
  auto add_tensor = [&](Tensor t) {
    s.tensors.push_back(std::move(t));
    return (int)s.tensors.size() - 1;
  };
  // Merge a group of factors into one leaf: values for every bitstring and
  // every assignment of the cut variables it holds (Fig. 3: the cut edge
  // carries its fixed value into the factors on both sides).
  auto make_leaf = [&](const std::vector<int> &fs) {
    Tensor t;
    t.leaf = true;
    std::vector<int> fv;
    uint32_t sel = 0;
    for (int f : fs) {
      const Factor &F = net.factors[f];
      for (int j = 0; j < F.nv; ++j) {
        int v = F.v[j];
        if (pos[v] >= 0) {
          if (std::find(fv.begin(), fv.end(), v) == fv.end()) fv.push_back(v);
        } else {
          sel |= 1u << cutbit[v];
        }
      }
      if (F.kind == 2) t.bdep = true;
    }
    std::sort(fv.begin(), fv.end(), by_pos);
    if ((int)fv.size() > kLeafMaxRank) throw std::runtime_error("leaf group too large");
    t.vars = fv;
    t.selmask = sel;
    t.sdep = sel != 0;
    const int r = (int)fv.size();
    const int ns = __builtin_popcount(sel);
    const uint32_t nb = t.bdep ? net.B : 1;
    t.values.assign((size_t)nb << (ns + r), cd(1.0, 0.0));
    std::vector<int> selbits;
    for (int b = 0; b < 32; ++b)
      if ((sel >> b) & 1u) selbits.push_back(b);
    for (uint32_t bi = 0; bi < nb; ++bi)
      for (uint32_t sv = 0; sv < (1u << ns); ++sv)
        for (uint32_t e = 0; e < (1u << r); ++e) {
          cd prod(1.0, 0.0);
          for (int f : fs) {
            const Factor &F = net.factors[f];
            int idx = 0;
            for (int j = 0; j < F.nv; ++j) {
              int v = F.v[j], bit;
              if (pos[v] >= 0) {
                int k = (int)(std::find(fv.begin(), fv.end(), v) - fv.begin());
                bit = (e >> (r - 1 - k)) & 1;
              } else {
                int k = (int)(std::find(selbits.begin(), selbits.end(), cutbit[v]) - selbits.begin());
                bit = (sv >> k) & 1;
              }
              idx = idx * 2 + bit;
            }
            const auto &vals = net.values[f];
            prod *= (F.kind == 2) ? vals[((size_t)bi << F.nv) + idx] : vals[idx];
          }
          t.values[(((size_t)bi << ns) + sv) * ((size_t)1 << r) + e] = prod;
        }
    return add_tensor(std::move(t));
  };

  std::vector<int> leaf_of(V, -1);
  for (int v : order)
    if (!group[v].empty()) leaf_of[v] = make_leaf(group[v]);
  int scalar_leaf = scalar_group.empty() ? -1 : make_leaf(scalar_group);

  auto has = [](const Tensor &t, int v) {
    return std::find(t.vars.begin(), t.vars.end(), v) != t.vars.end();
  };
  std::vector<int> pool, finals;
  std::vector<char> done(V, 0);

  auto emit = [&](std::vector<int> inputs, std::vector<int> kappa,
                  std::vector<int> out) {
    Step st;
    std::sort(out.begin(), out.end(), by_pos);
    Tensor c;
    c.vars = out;
    for (int i : inputs) {
      c.bdep |= s.tensors[i].bdep;
      c.sdep |= s.tensors[i].sdep;
    }
    const int stepno = (int)s.steps.size();
    c.producer = stepno;
    int cid = add_tensor(std::move(c));
    st.out = cid;
    st.in = inputs;
    st.kappa = kappa;
    st.rC = (int)out.size();
    st.nk = (int)kappa.size();
    st.bdep = s.tensors[cid].bdep;
    st.sdep = s.tensors[cid].sdep;
    std::vector<int> ivars(kappa);
    ivars.insert(ivars.end(), out.begin(), out.end());
    const int rI = (int)ivars.size();
    if (rI > 31) throw std::runtime_error("step index space too large");
    for (int i : inputs) {
      const Tensor &t = s.tensors[i];
      uint32_t m = 0;
      size_t k = 0;
      for (int j = 0; j < rI; ++j) {
        if (has(t, ivars[j])) {
          if (k >= t.vars.size() || t.vars[k] != ivars[j])
            throw std::runtime_error("input layout is not a subsequence");
          m |= 1u << (rI - 1 - j);
          ++k;
        }
      }
      if (k != t.vars.size()) throw std::runtime_error("input variable outside step");
      st.mask.push_back(m);
      s.tensors[i].last_use = stepno;
    }
    s.width = std::max(s.width, st.rC);
    s.steps.push_back(st);
    return cid;
  };

  auto union_vars = [&](const std::vector<int> &ins) {
    std::vector<int> u;
    for (int i : ins)
      for (int v : s.tensors[i].vars)
        if (std::find(u.begin(), u.end(), v) == u.end()) u.push_back(v);
    std::sort(u.begin(), u.end(), by_pos);
    return u;
  };

  for (size_t idx = 0; idx < order.size(); ++idx) {
    const int v = order[idx];
    if (done[v]) continue;
    std::vector<int> inputs;
    if (leaf_of[v] >= 0) inputs.push_back(leaf_of[v]);
    std::vector<int> keep;
    for (int t : pool) (has(s.tensors[t], v) ? inputs : keep).push_back(t);
    pool.swap(keep);
    done[v] = 1;
    std::vector<int> U = union_vars(inputs);
    std::vector<int> kappa{v};
    std::vector<int> out;
    for (int u : U)
      if (u != v) out.push_back(u);
    // Too many operands (kMaxIn, or kMaxProgIn for a step that will run in
    // a workgroup program): multiply the two smallest first (v stays open;
    // the union, and so the step's index space, does not change).
    const int limit = (int)out.size() < kSmallRank ? kMaxProgIn : kMaxIn;
    while ((int)inputs.size() > limit) {
      std::stable_sort(inputs.begin(), inputs.end(), [&](int a, int b) {
        return s.tensors[a].rank() < s.tensors[b].rank();
      });
      std::vector<int> two{inputs[0], inputs[1]};
      int pid = emit(two, {}, union_vars(two));
      inputs.erase(inputs.begin(), inputs.begin() + 2);
      inputs.push_back(pid);
    }
    // Chain fusion: a following bucket that holds this result, a leaf and
    // other tensors whose variables all lie in this step's outputs is summed
    // in the same pass over the same index space (the index space does not
    // grow; the intermediate of the first bucket is never stored).  Without
    // the other tensors this is the plain chain of one result and its leaf;
    // with them it also removes an expansion followed by a contraction, as
    // at the end of the n = 80, depth-2 orders (QTN_ABSORB=0 keeps the plain
    // chains only).
    static const bool absorb = [] {
      const char *e = std::getenv("QTN_ABSORB");  // tuning switch
      return !(e && e[0] == '0');
    }();
    auto inside_out = [&](int t) {
      for (int u : s.tensors[t].vars)
        if (std::find(out.begin(), out.end(), u) == out.end()) return false;
      return true;
    };
    if (o.fuse_chains) {
      const int rI = (int)U.size();
      while (idx + 1 < order.size()) {
        const int w = order[idx + 1];
        if (std::find(out.begin(), out.end(), w) == out.end()) break;
        std::vector<int> others;
        bool outside = false;
        for (int t : pool)
          if (has(s.tensors[t], w)) {
            others.push_back(t);
            outside |= !inside_out(t);
          }
        if (!others.empty() && (!absorb || outside)) break;
        const int lw = leaf_of[w];
        const int rC_next = (int)out.size() - 1;
        const int limit = rC_next < kSmallRank ? kMaxProgIn : kMaxIn;
        if ((int)(inputs.size() + others.size()) + (lw >= 0 ? 1 : 0) > limit) break;
        if (lw >= 0 && !inside_out(lw)) break;
        // Small index spaces are summed in one workgroup and may fuse freely;
        // streaming steps keep enough outputs to fill the chip and sum at
        // most kMaxStreamKappa variables per pass.
        const int rC_after = (int)out.size() - 1;
        if (rI <= kSmallRank) {
          if ((int)kappa.size() >= 12) break;
        } else {
          if (rC_after < kSmallRank || (int)kappa.size() >= kMaxStreamKappa) break;
        }
        kappa.push_back(w);
        out.erase(std::find(out.begin(), out.end(), w));
        if (lw >= 0) inputs.push_back(lw);
        for (int t : others) {
          inputs.push_back(t);
          pool.erase(std::find(pool.begin(), pool.end(), t));
        }
        done[w] = 1;
        ++idx;
      }
    }
    int cid = emit(inputs, kappa, out);
    if (s.tensors[cid].rank() == 0)
      finals.push_back(cid);
    else
      pool.push_back(cid);
  }
  if (!pool.empty()) throw std::runtime_error("unfinished tensors after elimination");
  if (scalar_leaf >= 0) finals.push_back(scalar_leaf);
  if (finals.empty()) throw std::runtime_error("empty network");
  while (finals.size() > 1 || s.tensors[finals[0]].leaf) {
    std::vector<int> take(finals.begin(),
                          finals.begin() + std::min<size_t>(finals.size(), kMaxProgIn));
    std::vector<int> rest(finals.begin() + take.size(), finals.end());
    int cid = emit(take, {}, {});
    rest.insert(rest.begin(), cid);
    finals.swap(rest);
  }
  s.result = finals[0];
  s.tensors[s.result].last_use = (int)s.steps.size();  // read by the slice sum
  return s;
}

// ---------------------------------------------------------------------------
// Workspace layout: first-fit with liveness, per wave of S slices.
// ---------------------------------------------------------------------------

int assign_storage(Schedule &s, int precision, double small_share) {
  if (precision == 0) {
    for (auto &t : s.tensors) t.f64 = true;
    return 64;
  }
  // bytes moved per instance by tensors of each rank, stored in 8 bytes
  std::vector<double> by_rank(64, 0.0);
  double total = 0.0;
  for (const Step &st : s.steps) {
    auto add = [&](int r) {
      by_rank[r] += std::ldexp(8.0, r);
      total += std::ldexp(8.0, r);
    };
    add(st.rC);
    for (int i : st.in)
      if (!s.tensors[i].leaf) add(s.tensors[i].rank());
  }
  int R = 0;
  double acc = 0.0;
  while (R < 63 && acc + by_rank[R] <= small_share * total) acc += by_rank[R++];
  R = std::max(R, kAlwaysF64Rank);
  static const int env_rank = [] {
    const char *e = std::getenv("QTN_F64_RANK");  // tuning switch: tensors below this rank stay complex128
    return e ? std::atoi(e) : 0;
  }();
  R = std::max(R, env_rank);
  for (auto &t : s.tensors) t.f64 = t.leaf || t.rank() < R;
  return R;
}

static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

namespace {
// First-fit interval allocator over a linear address space.
struct FirstFit {
  std::vector<std::pair<uint64_t, uint64_t>> freel;  // (offset, size), sorted
  uint64_t top = 0, peak = 0;
  uint64_t limit = ~uint64_t(0);
  bool alloc(uint64_t size, uint64_t &off) {
    for (size_t i = 0; i < freel.size(); ++i) {
      if (freel[i].second >= size) {
        off = freel[i].first;
        freel[i].first += size;
        freel[i].second -= size;
        if (freel[i].second == 0) freel.erase(freel.begin() + i);
        return true;
      }
    }
    if (top + size > limit) return false;
    off = top;
    top += size;
    peak = std::max(peak, top);
    return true;
  }
  void release(uint64_t off, uint64_t size) {
    auto it = std::lower_bound(freel.begin(), freel.end(), std::make_pair(off, uint64_t(0)));
    it = freel.insert(it, {off, size});
    size_t i = it - freel.begin();
    if (i + 1 < freel.size() && freel[i].first + freel[i].second == freel[i + 1].first) {
      freel[i].second += freel[i + 1].second;
      freel.erase(freel.begin() + i + 1);
    }
    if (i > 0 && freel[i - 1].first + freel[i - 1].second == freel[i].first) {
      freel[i - 1].second += freel[i].second;
      freel.erase(freel.begin() + i);
    }
    if (!freel.empty() && freel.back().first + freel.back().second == top) {
      top = freel.back().first;
      freel.pop_back();
    }
  }
};
}  // namespace

// The closing chain of a schedule: the last steps each take the previous
// step's output and gate factors only, down to the rank-0 result.  Their
// whole effect is sum_c T[c] W(c), T the chain's first input and W the
// product of its gate factors (each a function of some of T's variables).
// The earliest grid-wide streaming step whose output can serve as T takes
// the reduction as its epilogue; the chain's launches are dropped.
static void fold_closing_chain(const Schedule &s, ExecPlan &x, const std::vector<int> &consumer) {
  static const bool enabled = [] {
    const char *e = std::getenv("QTN_DOT");  // tuning switch: 0 keeps the closing steps
    return !(e && e[0] == '0');
  }();
  if (!enabled || s.steps.empty() || s.result < 0) return;
  std::vector<char> in_launch(s.steps.size(), 0);
  for (const LaunchGroup &G : x.launches)
    if (G.kind == 1) in_launch[G.step] = 1;
  int cur = (int)s.steps.size() - 1;
  if (s.steps[cur].out != s.result) return;
  std::vector<int> chain{cur};
  int best = -1;
  size_t best_len = 0;
  for (;;) {
    int prev = -1, n_nonleaf = 0;
    for (int i : s.steps[cur].in)
      if (!s.tensors[i].leaf) {
        ++n_nonleaf;
        prev = i;
      }
    if (n_nonleaf != 1 || consumer[prev] != cur) break;
    const int p = s.tensors[prev].producer;
    if (p < 0) break;
    const Step &H = s.steps[p];
    // the head must be a grid-wide streaming step (output of at least 2^8
    // elements per instance, at most 4 summed and 4 varying operands)
    int nvary = 0;
    const uint32_t cbits = H.rC >= 32 ? ~0u : ((1u << H.rC) - 1u);
    for (size_t i = 0; i < H.in.size(); ++i) nvary += (H.mask[i] & cbits) ? 1 : 0;
    const bool streaming = in_launch[p] && H.rC >= 8 && H.nk <= 4 && nvary >= 1 && nvary <= 4 &&
                           x.loc[prev] == LOC_GLOBAL;
    if (streaming) {
      best = p;
      best_len = chain.size();
    }
    chain.push_back(p);
    cur = p;
  }
  if (best < 0) return;
  const int T = s.steps[best].out;
  const Tensor &TT = s.tensors[T];
  const Tensor &R = s.tensors[s.result];
  if (TT.bdep != R.bdep || TT.sdep != R.sdep) return;
  std::vector<int> tail(chain.begin(), chain.begin() + best_len);
  std::vector<char> is_tail(s.steps.size(), 0);
  for (int st : tail) is_tail[st] = 1;
  // gate factors of the chain, as bits of T's index (first variable = top bit)
  std::vector<int> leaves;
  std::vector<uint32_t> masks;
  int nmixed = 0;
  for (int st : tail)
    for (int i : s.steps[st].in) {
      if (!s.tensors[i].leaf) continue;
      uint32_t m = 0;
      for (int v : s.tensors[i].vars) {
        auto it = std::find(TT.vars.begin(), TT.vars.end(), v);
        if (it == TT.vars.end()) return;   // a variable T does not carry
        m |= 1u << (TT.rank() - 1 - (int)(it - TT.vars.begin()));
      }
      if ((m & 255u) && (m >> 8)) ++nmixed;
      if (s.tensors[i].rank() > 4) return;
      leaves.push_back(i);
      masks.push_back(m);
    }
  if ((int)leaves.size() > kMaxDotLeaves || nmixed > kMaxDotMixed) return;
  int nvals = 0;
  for (int i : leaves) nvals += 1 << s.tensors[i].rank();
  if (nvals > kMaxDotValues) return;
  // every program of the chain must hold chain steps only
  for (LaunchGroup &G : x.launches) {
    if (G.kind != 0) continue;
    for (int p : G.programs) {
      int nt = 0;
      for (int st : x.programs[p].steps) nt += is_tail[st];
      if (nt && nt != (int)x.programs[p].steps.size()) return;
    }
  }
  std::vector<LaunchGroup> kept;
  for (LaunchGroup &G : x.launches) {
    if (G.kind == 1) {
      if (!is_tail[G.step]) kept.push_back(G);
      continue;
    }
    LaunchGroup g = G;
    g.programs.clear();
    for (int p : G.programs)
      if (!is_tail[x.programs[p].steps[0]]) g.programs.push_back(p);
    if (!g.programs.empty()) kept.push_back(g);
  }
  x.launches = kept;
  x.dot_step = best;
  x.dot_tensor = T;
  x.dot_leaves = leaves;
  x.dot_masks = masks;
}

ExecPlan build_exec(const Schedule &s, int mode, uint32_t lds_budget) {
  const int nst = (int)s.steps.size();
  const int nt = (int)s.tensors.size();
  ExecPlan x;
  x.mode = mode;
  x.loc.assign(nt, LOC_GLOBAL);
  x.off.assign(nt, 0);
  x.slot.assign(nt, -1);
  std::vector<int> consumer(nt, -1);
  for (int st = 0; st < nst; ++st)
    for (int i : s.steps[st].in) consumer[i] = st;
  for (int t = 0; t < nt; ++t)
    if (s.tensors[t].leaf) x.loc[t] = LOC_LEAF;

  // Pack the tensors of one program: LDS first (complex128), else scratch
  // (or the workspace in wide mode).  Returns false if nothing could be placed.
  auto pack = [&](Program &P, bool scratch_ok) {
    FirstFit lds, scr;
    lds.limit = lds_budget;
    std::vector<char> mine(nt, 0);
    for (int st : P.steps) mine[s.steps[st].out] = 1;
    // LDS intervals of the intermediates: bytes [off, off+size) during the
    // steps at positions t0..t1 of the program
    struct Iv {
      uint64_t off, size;
      int t0, t1;
    };
    std::vector<Iv> ivs;
    std::vector<int> iv_of(nt, -1);
    int slots = 0;
    for (size_t si = 0; si < P.steps.size(); ++si) {
      const int st = P.steps[si];
      const int o = s.steps[st].out;
      if (o != P.root) {
        const uint64_t lbytes = (uint64_t)16 << s.tensors[o].rank();
        uint64_t off;
        if (lds.alloc((lbytes + 15) & ~uint64_t(15), off)) {
          x.loc[o] = LOC_LDS;
          x.off[o] = off;
          iv_of[o] = (int)ivs.size();
          ivs.push_back({off, (lbytes + 15) & ~uint64_t(15), (int)si, (int)si});
        } else if (scratch_ok) {
          const uint64_t sb = (((uint64_t)elem_bytes(s.tensors[o]) << s.tensors[o].rank()) + 255) & ~uint64_t(255);
          scr.alloc(sb, off);
          x.loc[o] = LOC_SCRATCH;
          x.off[o] = off;
        } else {
          x.loc[o] = LOC_GLOBAL;
        }
        if (x.loc[o] != LOC_GLOBAL) x.slot[o] = slots++;
      }
      for (int i : s.steps[st].in) {
        if (!mine[i] || consumer[i] != st) continue;
        const Tensor &t = s.tensors[i];
        if (x.loc[i] == LOC_LDS) {
          lds.release(x.off[i], (((uint64_t)16 << t.rank()) + 15) & ~uint64_t(15));
          ivs[iv_of[i]].t1 = (int)si;
        } else if (x.loc[i] == LOC_SCRATCH) {
          scr.release(x.off[i], (((uint64_t)elem_bytes(t) << t.rank()) + 255) & ~uint64_t(255));
        }
      }
    }
    // Gate factors and workspace tensors made by earlier launches are staged
    // in LDS at the program's start where they fit: each is live from the
    // start to its consuming step.
    uint64_t top = lds.peak;
    for (size_t si = 0; si < P.steps.size(); ++si)
      for (int i : s.steps[P.steps[si]].in) {
        const bool outside = !s.tensors[i].leaf && !mine[i] && x.loc[i] == LOC_GLOBAL;
        if (!s.tensors[i].leaf && !outside) continue;
        const uint64_t size = (uint64_t)16 << s.tensors[i].rank();
        std::vector<uint64_t> cand{0};
        for (const Iv &v : ivs)
          if (v.t0 <= (int)si) cand.push_back(v.off + v.size);
        std::sort(cand.begin(), cand.end());
        for (uint64_t c : cand) {
          if (c + size > lds_budget) break;
          bool ok = true;
          for (const Iv &v : ivs)
            if (v.t0 <= (int)si && c < v.off + v.size && v.off < c + size) {
              ok = false;
              break;
            }
          if (!ok) continue;
          ivs.push_back({c, size, -1, (int)si});
          if (outside) {
            // the tensor stays in the workspace for its producer; only this
            // program reads its LDS copy
            P.staged_global.push_back({i, c, slots++});
          } else {
            x.loc[i] = LOC_LDS;
            x.off[i] = c;
            P.staged.push_back(i);
          }
          top = std::max(top, c + size);
          break;
        }
      }
    P.lds_bytes = (uint32_t)top;
    P.scratch_bytes = scr.peak;
    P.nslots = slots;
  };

  if (mode == MODE_SLICE) {
    Program P;
    for (int st = 0; st < nst; ++st) P.steps.push_back(st);
    P.root = s.result;
    P.bdep = s.tensors[s.result].bdep;
    P.sdep = s.tensors[s.result].sdep;
    pack(P, true);
    x.programs.push_back(P);
    LaunchGroup g;
    g.kind = 0;
    g.programs.push_back(0);
    x.launches.push_back(g);
  } else {
    std::vector<char> small(nst, 0);
    for (int st = 0; st < nst; ++st) {
      const Step &S_ = s.steps[st];
      small[st] = S_.rC < kSmallRank && S_.rC + S_.nk <= kSmallRank + 4;
    }
    // components of small steps joined through small -> small edges
    std::vector<int> parent(nst);
    std::iota(parent.begin(), parent.end(), 0);
    std::function<int(int)> find = [&](int a) { return parent[a] == a ? a : parent[a] = find(parent[a]); };
    for (int st = 0; st < nst; ++st) {
      if (!small[st]) continue;
      for (int i : s.steps[st].in) {
        const int pr = s.tensors[i].producer;
        if (!s.tensors[i].leaf && pr >= 0 && small[pr]) parent[find(pr)] = find(st);
      }
    }
    std::map<int, int> comp_of_rep;
    std::vector<int> comp(nst, -1);
    for (int st = 0; st < nst; ++st) {
      if (!small[st]) continue;
      int r = find(st);
      auto it = comp_of_rep.find(r);
      if (it == comp_of_rep.end()) {
        it = comp_of_rep.emplace(r, (int)x.programs.size()).first;
        x.programs.emplace_back();
      }
      comp[st] = it->second;
      x.programs[it->second].steps.push_back(st);
    }
    for (auto &P : x.programs) {
      // the root is the one step whose output leaves the component
      int roots = 0;
      for (int st : P.steps) {
        const int o = s.steps[st].out;
        const int c = consumer[o];
        if (c < 0 || !small[c]) {
          P.root = o;
          ++roots;
        }
      }
      if (roots != 1) throw std::runtime_error("small-step component is not a tree");
      P.bdep = s.tensors[P.root].bdep;
      P.sdep = s.tensors[P.root].sdep;
      pack(P, false);
    }
    // launch sequence: every component without grid-step inputs first, then
    // grid steps in order, each preceded by the components it consumes
    std::vector<char> needs_grid(x.programs.size(), 0), launched(x.programs.size(), 0);
    for (size_t c = 0; c < x.programs.size(); ++c)
      for (int st : x.programs[c].steps)
        for (int i : s.steps[st].in) {
          const int pr = s.tensors[i].producer;
          if (!s.tensors[i].leaf && pr >= 0 && !small[pr]) needs_grid[c] = 1;
        }
    LaunchGroup g0;
    for (size_t c = 0; c < x.programs.size(); ++c)
      if (!needs_grid[c]) {
        g0.programs.push_back((int)c);
        launched[c] = 1;
      }
    if (!g0.programs.empty()) x.launches.push_back(g0);
    for (int st = 0; st < nst; ++st) {
      if (small[st]) continue;
      LaunchGroup pre;
      for (int i : s.steps[st].in) {
        const int pr = s.tensors[i].producer;
        if (s.tensors[i].leaf || pr < 0 || !small[pr]) continue;
        const int c = comp[pr];
        if (!launched[c]) {
          pre.programs.push_back(c);
          launched[c] = 1;
        }
      }
      if (!pre.programs.empty()) x.launches.push_back(pre);
      LaunchGroup g;
      g.kind = 1;
      g.step = st;
      x.launches.push_back(g);
    }
    LaunchGroup tail;
    for (size_t c = 0; c < x.programs.size(); ++c)
      if (!launched[c]) tail.programs.push_back((int)c);
    if (!tail.programs.empty()) x.launches.push_back(tail);
  }
  if (mode == MODE_WIDE) fold_closing_chain(s, x, consumer);
  for (auto &P : x.programs) {
    x.lds_bytes = std::max(x.lds_bytes, P.lds_bytes);
    x.scratch_per_wg = std::max(x.scratch_per_wg, P.scratch_bytes);
  }
  return x;
}

Layout layout(Schedule &s, const ExecPlan &x, uint64_t B, uint64_t S, uint64_t wg_slots) {
  Layout L;
  L.S = S;
  FirstFit ff;
  auto bytes_of = [&](const Tensor &t) {
    return align256(instances(t, B, S) * ((uint64_t)1 << t.rank()) * (uint64_t)elem_bytes(t));
  };
  auto global = [&](int t) { return !s.tensors[t].leaf && x.loc[t] == LOC_GLOBAL; };
  // Liveness follows the launch sequence: the steps of one launch run
  // concurrently, so everything a launch writes is placed before anything it
  // reads last is released.
  const size_t nl = x.launches.size();
  std::vector<std::vector<int>> lsteps(nl);
  for (size_t g = 0; g < nl; ++g) {
    const LaunchGroup &G = x.launches[g];
    if (G.kind == 1)
      lsteps[g].push_back(G.step);
    else
      for (int p : G.programs)
        for (int st : x.programs[p].steps) lsteps[g].push_back(st);
  }
  std::vector<int> last_launch(s.tensors.size(), -1);
  for (size_t g = 0; g < nl; ++g)
    for (int st : lsteps[g])
      for (int i : s.steps[st].in) last_launch[i] = std::max(last_launch[i], (int)g);
  last_launch[x.dot_step >= 0 ? x.dot_tensor : s.result] = (int)nl;  // read by the slice sum
  for (size_t g = 0; g < nl; ++g) {
    for (int st : lsteps[g]) {
      const int o = s.steps[st].out;
      if (!global(o)) continue;
      uint64_t off;
      ff.alloc(bytes_of(s.tensors[o]), off);
      s.tensors[o].data_off = off;
    }
    std::vector<int> done;
    for (int st : lsteps[g])
      for (int i : s.steps[st].in)
        if (global(i) && last_launch[i] == (int)g && std::find(done.begin(), done.end(), i) == done.end()) {
          ff.release(s.tensors[i].data_off, bytes_of(s.tensors[i]));
          done.push_back(i);
        }
  }
  // self-check: tensors whose launch intervals overlap never share memory
  {
    std::vector<int> first_launch(s.tensors.size(), -1);
    for (size_t g = 0; g < nl; ++g)
      for (int st : lsteps[g]) first_launch[s.steps[st].out] = (int)g;
    std::vector<int> gl;
    for (size_t t = 0; t < s.tensors.size(); ++t)
      if (global((int)t) && first_launch[t] >= 0) gl.push_back((int)t);
    for (size_t a = 0; a < gl.size(); ++a)
      for (size_t b = a + 1; b < gl.size(); ++b) {
        const int u = gl[a], v = gl[b];
        const bool live = first_launch[u] <= last_launch[v] && first_launch[v] <= last_launch[u];
        const uint64_t u0 = s.tensors[u].data_off, u1 = u0 + bytes_of(s.tensors[u]);
        const uint64_t v0 = s.tensors[v].data_off, v1 = v0 + bytes_of(s.tensors[v]);
        if (live && u0 < v1 && v0 < u1) throw std::runtime_error("workspace layout overlap");
      }
  }
  L.data_bytes = align256(ff.peak);
  uint64_t eo = L.data_bytes;
  for (size_t t = 0; t < s.tensors.size(); ++t) {
    if (!global((int)t)) continue;
    s.tensors[t].exp_off = eo;
    eo += align256(instances(s.tensors[t], B, S) * 4 * (1 + kMaxSlots));
  }
  L.exp_bytes = eo - L.data_bytes;
  L.partial_off = eo;
  L.flag_off = eo + B * 32;
  uint64_t po = align256(eo + B * 32 + 4);
  if (x.dot_step >= 0) {
    const Tensor &T = s.tensors[x.dot_tensor];
    L.dot_slots = (uint64_t)1 << std::max(0, s.steps[x.dot_step].rC - 8);
    L.dot_off = po;
    po = align256(po + instances(T, B, S) * L.dot_slots * 16);
  }
  L.scratch_off = po;
  L.wg_slots = wg_slots;
  L.total_bytes = align256(L.scratch_off + wg_slots * align256(x.scratch_per_wg));
  return L;
}

LaunchGraph launch_graph(const Schedule &s, const ExecPlan &x, const Layout &L, uint64_t B,
                         uint64_t S, bool scaled, int max_streams) {
  struct Range {
    uint64_t lo, hi;
    bool write;
  };
  const size_t nl = x.launches.size();
  const size_t U = nl + 2;
  std::vector<std::vector<Range>> rng(U);
  auto global = [&](int t) { return !s.tensors[t].leaf && x.loc[t] == LOC_GLOBAL; };
  auto data = [&](int t, bool w, std::vector<Range> &r) {
    const Tensor &T = s.tensors[t];
    const uint64_t n = align256(instances(T, B, S) * ((uint64_t)1 << T.rank()) * (uint64_t)elem_bytes(T));
    r.push_back({T.data_off, T.data_off + n, w});
    if (scaled) {
      const uint64_t e = align256(instances(T, B, S) * 4 * (1 + kMaxSlots));
      r.push_back({T.exp_off, T.exp_off + e, w});
    }
  };
  // Unit 0 launches nothing: the exponent region is cleared once when the
  // workspace is bound and then by the slice sum at the end of every wave,
  // for the next one (its words are read by nobody after the slice sum).
  for (size_t g = 0; g < nl; ++g) {
    const LaunchGroup &G = x.launches[g];
    std::vector<int> sts;
    if (G.kind == 1) {
      sts.push_back(G.step);
    } else {
      for (int p : G.programs)
        for (int st : x.programs[p].steps) sts.push_back(st);
      if (x.scratch_per_wg) rng[g + 1].push_back({L.scratch_off, L.total_bytes, true});
    }
    std::set<int> made;
    for (int st : sts) made.insert(s.steps[st].out);
    for (int st : sts) {
      for (int i : s.steps[st].in)
        if (global(i) && !made.count(i)) data(i, false, rng[g + 1]);
      if (global(s.steps[st].out)) data(s.steps[st].out, true, rng[g + 1]);
      if (st == x.dot_step)
        rng[g + 1].push_back({L.dot_off, L.dot_off + instances(s.tensors[x.dot_tensor], B, S) * L.dot_slots * 16,
                              true});
    }
  }
  if (x.dot_step >= 0) {
    data(x.dot_tensor, false, rng[nl + 1]);
    rng[nl + 1].push_back({L.dot_off, L.dot_off + instances(s.tensors[x.dot_tensor], B, S) * L.dot_slots * 16,
                           false});
  } else {
    data(s.result, false, rng[nl + 1]);
  }
  rng[nl + 1].push_back({L.partial_off, L.partial_off + B * 32, true});
  if (scaled && L.exp_bytes) rng[nl + 1].push_back({L.data_bytes, L.data_bytes + L.exp_bytes, true});

  auto conflict = [&](size_t a, size_t b) {
    for (const Range &p : rng[a])
      for (const Range &q : rng[b])
        if ((p.write || q.write) && p.lo < q.hi && q.lo < p.hi) return true;
    return false;
  };
  LaunchGraph G;
  G.deps.assign(U, {});
  std::vector<std::vector<char>> anc(U, std::vector<char>(U, 0));  // anc[v][u]: u before v
  for (size_t v = 0; v < U; ++v) {
    std::vector<int> direct;
    for (size_t u = v; u-- > 0;)
      if (conflict(u, v)) direct.push_back((int)u);
    // transitive reduction: drop u when a later kept dependency already follows it
    for (int u : direct) {  // descending
      bool implied = false;
      for (int w : G.deps[v])
        if (anc[w][u]) {
          implied = true;
          break;
        }
      if (!implied) G.deps[v].push_back(u);
    }
    for (int u : G.deps[v]) {
      anc[v][u] = 1;
      for (size_t a = 0; a < U; ++a)
        if (anc[u][a]) anc[v][a] = 1;
    }
  }
  G.level.assign(U, 0);
  for (size_t v = 0; v < U; ++v) {
    for (int u : G.deps[v]) G.level[v] = std::max(G.level[v], G.level[u] + 1);
    G.nlevels = std::max(G.nlevels, G.level[v] + 1);
  }
  // enqueue order: among ready units, the one with the longest remaining
  // path first, a unit weighing a fixed launch latency plus its bytes
  std::vector<double> w(U, 0.0), bottom(U, 0.0);
  for (size_t u = 0; u < U; ++u) {
    double by = 0;
    for (const Range &r : rng[u]) by += (double)(r.hi - r.lo);
    w[u] = 4.0e7 + by;
  }
  std::vector<std::vector<int>> succ(U);
  for (size_t v = 0; v < U; ++v)
    for (int u : G.deps[v]) succ[u].push_back((int)v);
  for (size_t v = U; v-- > 0;) {
    double m = 0;
    for (int x : succ[v]) m = std::max(m, bottom[x]);
    bottom[v] = w[v] + m;
  }
  {
    std::vector<int> indeg(U, 0);
    for (size_t v = 0; v < U; ++v) indeg[v] = (int)G.deps[v].size();
    std::vector<int> ready;
    for (size_t v = 0; v < U; ++v)
      if (!indeg[v]) ready.push_back((int)v);
    while (!ready.empty()) {
      size_t bi = 0;
      for (size_t i = 1; i < ready.size(); ++i)
        if (bottom[ready[i]] > bottom[ready[bi]] ||
            (bottom[ready[i]] == bottom[ready[bi]] && ready[i] < ready[bi]))
          bi = i;
      const int v = ready[bi];
      ready.erase(ready.begin() + bi);
      G.order.push_back(v);
      for (int x : succ[v])
        if (--indeg[x] == 0) ready.push_back(x);
    }
  }
  // streams, in enqueue order: follow a dependency's stream when that
  // dependency is the stream's last unit, else take a stream whose last unit
  // is already an ancestor, else the one whose last unit came earliest
  const int ns = std::max(1, max_streams);
  G.stream.assign(U, 0);
  G.record.assign(U, 0);
  std::vector<int> tail(ns, -1);
  std::vector<int> pos(U, 0);
  for (size_t i = 0; i < U; ++i) pos[G.order[i]] = (int)i;
  for (int v : G.order) {
    int pick = -1;
    for (int u : G.deps[v])
      if (tail[G.stream[u]] == u && (pick < 0 || pos[u] > pos[tail[pick]])) pick = G.stream[u];
    if (pick < 0) {
      // a stream whose last unit is already an ancestor adds no ordering
      for (int k = 0; k < ns && pick < 0; ++k)
        if (tail[k] < 0 || anc[v][tail[k]]) pick = k;
    }
    if (pick < 0) {
      pick = 0;
      for (int k = 1; k < ns; ++k)
        if (pos[tail[k]] < pos[tail[pick]]) pick = k;
    }
    G.stream[v] = pick;
    tail[pick] = v;
    for (int u : G.deps[v])
      if (G.stream[u] != pick) G.record[u] = 1;
    G.nstreams = std::max(G.nstreams, pick + 1);
  }
  // self-check: units left unordered never touch conflicting bytes, and a
  // stream never holds a unit before one it depends on
  for (size_t v = 0; v < U; ++v)
    for (size_t u = 0; u < v; ++u) {
      bool ordered = anc[v][u] != 0;
      if (!ordered && G.stream[u] == G.stream[v]) ordered = true;  // same stream: FIFO
      if (!ordered && conflict(u, v)) throw std::runtime_error("launch graph misses a dependency");
    }
  for (size_t v = 0; v < U; ++v)
    for (int u : G.deps[v])
      if (pos[u] >= pos[v]) throw std::runtime_error("launch order breaks a dependency");
  return G;
}

Costs schedule_costs(const Schedule &s, uint64_t B, uint64_t S) {
  // Per wave of S slices; slice-invariant steps are reported apart and
  // amortised by the caller over the slices of one amplitude.
  Costs c;
  for (const Step &st : s.steps) {
    const Tensor &o = s.tensors[st.out];
    double q = (double)instances(o, B, S);
    double pts = q * std::ldexp(1.0, st.nk + st.rC);
    double fl = pts * (6.0 * (double)(st.in.size() - 1) + (st.nk > 0 ? 2.0 : 0.0));
    double by = q * std::ldexp(1.0, st.rC) * elem_bytes(o);
    for (int i : st.in) {
      const Tensor &t = s.tensors[i];
      double qi = t.leaf ? (double)((t.bdep ? B : 1) *
                                    std::min<uint64_t>(S, (uint64_t)1 << __builtin_popcount(t.selmask)))
                         : (double)instances(t, B, S);
      by += qi * std::ldexp(1.0, t.rank()) * elem_bytes(t);
    }
    if (st.sdep) {
      c.flops_per_slice += fl / (double)S;
      c.bytes_per_slice += by / (double)S;
    } else {
      c.flops_hoisted += fl;
      c.bytes_hoisted += by;
    }
  }
  return c;
}

}  // namespace qtn
