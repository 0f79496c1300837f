// Planner (Section "The variable elimination ordering" and Section
// "Parallelization by fixing the values of variables").
//
// * Cost of an ordering: eliminating v creates a tensor of size 2^deg(v) in
//   the graph at that moment; the cost of an ordering is the sum over steps.
// * Ordering: greedy min-fill (the branching heuristic the paper runs its
//   anytime search with), with randomised tie-breaking restarts kept when
//   they lower the cost.
// * Slicing: vertices are removed greedily, each time the one that most
//   lowers the cost under one fixed ordering; the ordering is recomputed
//   after the removals.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <random>

#include "host.h"

namespace qgm {

void Graph::init(int n_) {
  n = n_;
  words = (n + 63) / 64;
  if (words == 0) words = 1;
  adj.assign((size_t)n * words, 0);
}

void Graph::add_edge(int a, int b) {
  if (a == b) return;
  row(a)[b >> 6] |= 1ull << (b & 63);
  row(b)[a >> 6] |= 1ull << (a & 63);
}

Graph model_graph(const Network& net, std::vector<int>& vertex_of_var) {
  vertex_of_var.assign(net.vars.size(), -1);
  for (size_t i = 0; i < net.free_vars.size(); ++i) vertex_of_var[net.free_vars[i]] = (int)i;
  Graph g;
  g.init((int)net.free_vars.size());
  // two variables are adjacent when a factor holds both (a clique per factor)
  for (const Factor& f : net.factors)
    for (int i = 0; i < f.nv; ++i)
      for (int j = i + 1; j < f.nv; ++j) {
        int a = vertex_of_var[f.var[i]], b = vertex_of_var[f.var[j]];
        if (a >= 0 && b >= 0) g.add_edge(a, b);
      }
  return g;
}

static inline int popcount_row(const uint64_t* r, int words) {
  int c = 0;
  for (int w = 0; w < words; ++w) c += __builtin_popcountll(r[w]);
  return c;
}

// Eliminate v in place: connect its neighbours, then drop v.
static int eliminate(Graph& g, int v) {
  uint64_t* rv = g.row(v);
  int deg = popcount_row(rv, g.words);
  std::vector<uint64_t> nb(rv, rv + g.words);
  for (int w = 0; w < g.words; ++w) {
    uint64_t bits = nb[w];
    while (bits) {
      int u = w * 64 + __builtin_ctzll(bits);
      bits &= bits - 1;
      uint64_t* ru = g.row(u);
      for (int x = 0; x < g.words; ++x) ru[x] |= nb[x];
      ru[u >> 6] &= ~(1ull << (u & 63));
      ru[v >> 6] &= ~(1ull << (v & 63));
    }
  }
  std::memset(rv, 0, sizeof(uint64_t) * g.words);
  return deg;
}

static void drop(Graph& g, int v) {
  uint64_t* rv = g.row(v);
  for (int w = 0; w < g.words; ++w) {
    uint64_t bits = rv[w];
    while (bits) {
      int u = w * 64 + __builtin_ctzll(bits);
      bits &= bits - 1;
      g.row(u)[v >> 6] &= ~(1ull << (v & 63));
    }
    rv[w] = 0;
  }
}

OrderCost order_cost(const Graph& g0, const std::vector<int>& order, const std::vector<char>& removed) {
  Graph g = g0;
  for (int v = 0; v < g.n; ++v)
    if (removed[v]) drop(g, v);
  OrderCost c{0.0, 0};
  for (int v : order) {
    if (removed[v]) continue;
    int d = eliminate(g, v);
    c.cost += std::ldexp(1.0, d);
    c.width = std::max(c.width, d);
  }
  return c;
}

static int fill_in(const Graph& g, int v) {
  const uint64_t* rv = g.row(v);
  int missing = 0;
  for (int w = 0; w < g.words; ++w) {
    uint64_t bits = rv[w];
    while (bits) {
      int u = w * 64 + __builtin_ctzll(bits);
      bits &= bits - 1;
      // neighbours of v that are not neighbours of u (excluding u), counted once per pair
      const uint64_t* ru = g.row(u);
      for (int x = 0; x < g.words; ++x) {
        uint64_t m = rv[x] & ~ru[x];
        if (x == (u >> 6)) m &= ~(1ull << (u & 63));
        missing += __builtin_popcountll(m);
      }
    }
  }
  return missing / 2;
}

std::vector<int> min_fill_order(const Graph& g0, const std::vector<char>& removed, uint64_t seed, int randomize) {
  Graph g = g0;
  std::vector<char> alive(g.n, 1);
  int left = 0;
  for (int v = 0; v < g.n; ++v) {
    if (removed[v]) {
      drop(g, v);
      alive[v] = 0;
    } else {
      ++left;
    }
  }
  std::mt19937_64 rng(seed);
  std::vector<int> order;
  order.reserve(left);
  std::vector<int> fill(g.n, 0);
  std::vector<char> dirty(g.n, 1);
  while (left > 0) {
    int best = -1;
    long best_key = 0;
    std::vector<int> ties;
    for (int v = 0; v < g.n; ++v) {
      if (!alive[v]) continue;
      if (dirty[v]) {
        fill[v] = fill_in(g, v);
        dirty[v] = 0;
      }
      long key = (long)fill[v] * 4096 + popcount_row(g.row(v), g.words);
      if (best < 0 || key < best_key) {
        best = v;
        best_key = key;
        ties.clear();
        ties.push_back(v);
      } else if (key == best_key) {
        ties.push_back(v);
      }
    }
    if (randomize && ties.size() > 1) best = ties[rng() % ties.size()];
    // fill counts change for the neighbours of `best` and their neighbours
    const uint64_t* rb = g.row(best);
    for (int w = 0; w < g.words; ++w) {
      uint64_t bits = rb[w];
      while (bits) {
        int u = w * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        dirty[u] = 1;
        const uint64_t* ru = g.row(u);
        for (int x = 0; x < g.words; ++x) {
          uint64_t b2 = ru[x];
          while (b2) {
            dirty[x * 64 + __builtin_ctzll(b2)] = 1;
            b2 &= b2 - 1;
          }
        }
      }
    }
    eliminate(g, best);
    alive[best] = 0;
    order.push_back(best);
    --left;
  }
  return order;
}

// Minor-min-width of the graph on the `alive` vertices: repeatedly contract
// a vertex of minimum degree into its minimum-degree neighbour (dropping it
// when isolated); the largest minimum degree met bounds the width of every
// elimination ordering from below (a minor's treewidth never exceeds the
// graph's, and every graph's treewidth is at least its minimum degree).
static int minor_min_width(Graph g, std::vector<char> alive) {
  int lb = 0;
  for (;;) {
    int v = -1, dv = 1 << 30;
    for (int u = 0; u < g.n; ++u) {
      if (!alive[u]) continue;
      const int d = popcount_row(g.row(u), g.words);
      if (d < dv) v = u, dv = d;
    }
    if (v < 0) break;
    lb = std::max(lb, dv);
    if (dv == 0) {
      alive[v] = 0;
      continue;
    }
    // neighbour of minimum degree; v's edges move to it
    int w = -1, dw = 1 << 30;
    const uint64_t* rv = g.row(v);
    for (int x = 0; x < g.words; ++x) {
      uint64_t bits = rv[x];
      while (bits) {
        const int u = x * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        const int d = popcount_row(g.row(u), g.words);
        if (d < dw) w = u, dw = d;
      }
    }
    std::vector<uint64_t> nb(rv, rv + g.words);
    for (int x = 0; x < g.words; ++x) {
      uint64_t bits = nb[x];
      while (bits) {
        const int u = x * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        if (u != w) g.add_edge(u, w);
      }
    }
    drop(g, v);
    alive[v] = 0;
  }
  return lb;
}

// Branch and bound over elimination orderings, the QuickBB scheme the paper
// uses (Section "The variable elimination ordering"): depth-first over the
// next vertex to eliminate, children in min-fill order, a node pruned when
// the minor-min-width of what is left shows it cannot beat the incumbent.
// Objective: (width, cost) compared lexicographically, width = max deg(v)
// and cost = sum 2^deg(v) at elimination.  Anytime: the incumbent starts as
// `init` and the search stops after max_nodes nodes; beam > 0 tries only
// that many children per node (all otherwise, which makes the search exact
// when it completes).
BnbResult bnb_order(const Graph& g0, const std::vector<char>& removed, const std::vector<int>& init,
                    long max_nodes, int beam) {
  BnbResult res;
  res.order = init;
  res.cost = order_cost(g0, init, removed);
  Graph g = g0;
  std::vector<char> alive(g.n, 0);
  int left = 0;
  for (int v = 0; v < g.n; ++v) {
    if (removed[v]) {
      drop(g, v);
    } else {
      alive[v] = 1;
      ++left;
    }
  }
  auto better = [](int w, double c, const OrderCost& b) { return w < b.width || (w == b.width && c < b.cost); };
  std::vector<int> path;
  path.reserve(left);
  long nodes = 0;
  bool stopped = false;
  std::function<void(Graph&, int, double, int)> dfs = [&](Graph& cur, int width, double cost, int remaining) {
    if (stopped) return;
    if (++nodes > max_nodes) {
      stopped = true;
      return;
    }
    if (remaining == 0) {
      if (better(width, cost, res.cost)) {
        res.cost = OrderCost{cost, width};
        res.order = path;
      }
      return;
    }
    const int lbw = std::max(width, minor_min_width(cur, alive));
    // every remaining step costs at least 2^0, one of them at least 2^lbw
    const double lbc = cost + std::max((double)remaining, std::ldexp(1.0, lbw) + remaining - 1);
    if (!better(lbw, lbc, res.cost)) return;
    std::vector<std::pair<long, int>> kids;
    for (int v = 0; v < cur.n; ++v)
      if (alive[v]) kids.push_back({(long)fill_in(cur, v) * 4096 + popcount_row(cur.row(v), cur.words), v});
    std::sort(kids.begin(), kids.end());
    if (beam > 0 && (int)kids.size() > beam) kids.resize(beam);
    for (auto& kv : kids) {
      const int v = kv.second;
      Graph next = cur;
      const int d = eliminate(next, v);
      alive[v] = 0;
      path.push_back(v);
      if (better(std::max(width, d), cost + std::ldexp(1.0, d), res.cost)) dfs(next, std::max(width, d),
                                                                                 cost + std::ldexp(1.0, d),
                                                                                 remaining - 1);
      path.pop_back();
      alive[v] = 1;
      if (stopped) return;
    }
  };
  dfs(g, 0, 0.0, left);
  res.nodes = std::min(nodes, max_nodes);
  res.complete = !stopped;
  return res;
}

}  // namespace qgm

namespace qgm {

// Work of the compiled program for a plan, without building it: tensors are
// bitsets over graph vertices; eliminating v fuses T_v into one step that
// also sums every variable occurring only in T_v (as the compiler does).
// Returns bytes (inputs + output of every step, 8 B per element), flops and
// the critical path: the largest flop count along a chain of dependent
// steps, the time of one item when its steps run on unboundedly many
// wavefronts.
struct SimCost {
  double bytes = 0, flops = 0, cp = 0;
};

static SimCost simulate(const Network& net, const std::vector<int>& vov, int n, const std::vector<char>& removed,
                        const std::vector<int>& order) {
  const int words = (n + 63) / 64 + 1;
  std::vector<std::vector<uint64_t>> tens;
  for (const Factor& f : net.factors) {
    std::vector<uint64_t> b(words, 0);
    int cnt = 0;
    for (int j = 0; j < f.nv; ++j) {
      int v = vov[f.var[j]];
      if (v >= 0 && !removed[v]) {
        b[v >> 6] |= 1ull << (v & 63);
        ++cnt;
      }
    }
    if (cnt) tens.push_back(b);
  }
  std::vector<double> fin(tens.size(), 0.0);  // flops along the longest chain ending at each tensor
  std::vector<char> alive(tens.size(), 1);
  std::vector<int> count(n, 0);
  for (auto& b : tens)
    for (int v = 0; v < n; ++v)
      if ((b[v >> 6] >> (v & 63)) & 1) count[v]++;
  std::vector<char> done(n, 0);
  SimCost c;
  auto pc = [&](const std::vector<uint64_t>& b) {
    int k = 0;
    for (uint64_t w : b) k += __builtin_popcountll(w);
    return k;
  };
  for (int v : order) {
    if (removed[v] || done[v]) continue;
    std::vector<int> tv;
    std::vector<uint64_t> un(words, 0);
    for (size_t i = 0; i < tens.size(); ++i)
      if (alive[i] && ((tens[i][v >> 6] >> (v & 63)) & 1)) {
        tv.push_back((int)i);
        for (int w = 0; w < words; ++w) un[w] |= tens[i][w];
      }
    if (tv.empty()) {
      done[v] = 1;
      continue;
    }
    std::vector<int> cin;
    std::vector<uint64_t> out = un, sum(words, 0);
    double in_elems = 0;
    for (int i : tv) in_elems += std::ldexp(1.0, pc(tens[i]));
    for (int w = 0; w < words; ++w) {
      uint64_t bits = un[w];
      while (bits) {
        int u = w * 64 + __builtin_ctzll(bits);
        bits &= bits - 1;
        int inside = 0;
        for (int i : tv) inside += (tens[i][u >> 6] >> (u & 63)) & 1;
        if (u == v || inside == count[u]) {
          sum[u >> 6] |= 1ull << (u & 63);
          out[u >> 6] &= ~(1ull << (u & 63));
        }
      }
    }
    const int r = pc(out), ns = pc(sum), m = (int)tv.size();
    const double f = std::ldexp(1.0, r + ns) * (6.0 * (m - 1) + 2.0);
    c.flops += f;
    double f0 = 0;
    for (int i : tv) f0 = std::max(f0, fin[i]);
    fin.push_back(f0 + f);
    c.cp = std::max(c.cp, fin.back());
    c.bytes += 8.0 * (in_elems + std::ldexp(1.0, r));
    for (int i : tv) {
      alive[i] = 0;
      for (int u = 0; u < n; ++u)
        if ((tens[i][u >> 6] >> (u & 63)) & 1) count[u]--;
    }
    for (int u = 0; u < n; ++u) {
      if ((sum[u >> 6] >> (u & 63)) & 1) done[u] = 1;
      if ((out[u >> 6] >> (u & 63)) & 1) count[u]++;
    }
    tens.push_back(out);
    alive.push_back(1);
  }
  return c;
}

// Best of several min-fill orderings (deterministic first, then randomised
// tie-breaking) until the time budget is spent.  Objectives: OBJ_COST, the
// sum of 2^deg(v); OBJ_BYTES, the compiled program's memory traffic (which
// sets the run time of large plans); OBJ_LATENCY, max(4 x critical path,
// flops), the time of one item on four wavefronts (for batches too small to
// fill the GPU), ties broken by flops.
enum { OBJ_COST = 0, OBJ_BYTES = 1, OBJ_LATENCY = 2 };
// With `det` the budget is a work count instead of a deadline:
// kRestartsPerSecond restarts per second of budget, whatever the host's
// speed, so every host returns the same ordering.
constexpr double kRestartsPerSecond = 320.0;
static std::vector<int> best_order(const Graph& g, const std::vector<char>& removed, uint64_t seed, double budget_s,
                                   OrderCost* out_cost, int objective = OBJ_COST, const Network* net = nullptr,
                                   const std::vector<int>* vov = nullptr, bool det = false) {
  auto t0 = std::chrono::steady_clock::now();
  std::vector<int> best = min_fill_order(g, removed, seed, 0);
  OrderCost bc = order_cost(g, best, removed);
  auto score = [&](const std::vector<int>& o) -> std::pair<double, double> {
    if (objective == OBJ_COST) return {0.0, 0.0};
    const SimCost sc = simulate(*net, *vov, g.n, removed, o);
    if (objective == OBJ_BYTES) return {sc.bytes, 0.0};
    return {std::max(4.0 * sc.cp, sc.flops), sc.flops};
  };
  std::pair<double, double> best_score = score(best);
  // At most kMaxRestarts restarts, so small graphs give the same ordering on
  // every run; large graphs may stop earlier on the time budget.
  const int kMaxRestarts = 128;
  const int n_restarts = det ? (int)std::min<double>(kMaxRestarts, std::floor(budget_s * kRestartsPerSecond + 0.5))
                             : kMaxRestarts;
  for (int it = 1; it <= n_restarts; ++it) {
    double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (!det && el >= budget_s) break;
    std::vector<int> o = min_fill_order(g, removed, seed + 0x9e3779b97f4a7c15ull * it, 1);
    OrderCost c = order_cost(g, o, removed);
    if (objective != OBJ_COST) {
      const std::pair<double, double> sc = score(o);
      if (sc < best_score) {
        best.swap(o);
        bc = c;
        best_score = sc;
      }
    } else if (c.cost < bc.cost || (c.cost == bc.cost && c.width < bc.width)) {
      best.swap(o);
      bc = c;
    }
  }
  if (out_cost) *out_cost = bc;
  return best;
}

// Greedy key-vertex removal: at each round remove the vertex whose removal
// gives the lowest cost under the fixed ordering `order0` (ties: lower width,
// then lower vertex id).  Candidates are the `n_cand` highest-degree
// vertices of the graph with the previous picks removed.
static bool plan_once(const Network& net, int k_req, int target_rank, double time_budget_s, uint64_t seed,
                      std::vector<int>& sliced_vars, std::vector<int>& order_vars, int flags, double* score,
                      double* item_elems = nullptr) {
  const bool reorder_each = (flags & 1) != 0;
  const bool det = (flags & 64) != 0;
  std::vector<int> vov;
  Graph g = model_graph(net, vov);
  std::vector<char> removed(g.n, 0);
  double b0 = k_req == 0 ? time_budget_s : time_budget_s * 0.4;
  OrderCost c0;
  std::vector<int> order0 = best_order(g, removed, seed, b0, &c0, OBJ_COST, nullptr, nullptr, det);
  std::vector<int> picks;
  const int n_cand = 64;
  int kmax = k_req >= 0 ? k_req : 40;
  OrderCost cur = c0;
  while ((int)picks.size() < kmax && (int)picks.size() < g.n) {
    if (k_req < 0 && cur.width <= target_rank) break;
    // current graph degrees (with picks removed)
    Graph gr = g;
    for (int p : picks) drop(gr, p);
    std::vector<std::pair<int, int>> cand;
    for (int v = 0; v < g.n; ++v)
      if (!removed[v]) cand.push_back({-popcount_row(gr.row(v), gr.words), v});
    std::sort(cand.begin(), cand.end());
    if ((int)cand.size() > n_cand) cand.resize(n_cand);
    int best_v = -1;
    OrderCost best_c{0, 0};
    for (auto& cv : cand) {
      int v = cv.second;
      removed[v] = 1;
      OrderCost c = order_cost(g, order0, removed);
      removed[v] = 0;
      if (best_v < 0 || c.cost < best_c.cost || (c.cost == best_c.cost && (c.width < best_c.width ||
                                                                           (c.width == best_c.width && v < best_v)))) {
        best_v = v;
        best_c = c;
      }
    }
    if (best_v < 0) break;
    removed[best_v] = 1;
    picks.push_back(best_v);
    cur = best_c;
    if (reorder_each) {
      // a fresh ordering of the reduced graph guides the next removal
      const double per_pick = time_budget_s * 0.4 / std::max(1, kmax);
      OrderCost c1;
      std::vector<int> o1 = best_order(g, removed, seed + 31 * picks.size(), per_pick, &c1, OBJ_COST, nullptr, nullptr,
                                       det);
      if (c1.cost < cur.cost || (c1.cost == cur.cost && c1.width < cur.width)) {
        order0 = o1;
        cur = c1;
      }
    }
  }
  double b1 = k_req == 0 ? 0.0 : time_budget_s * 0.6;
  const int objective = (flags & 4) ? OBJ_LATENCY : (flags & 2) ? OBJ_BYTES : OBJ_COST;
  const bool bnb = (flags & 128) != 0 && objective == OBJ_COST;
  if (bnb && k_req == 0) b1 = time_budget_s;  // the whole budget goes to the final ordering
  std::vector<int> order1 = best_order(g, removed, seed + 17, bnb ? b1 / 2 : b1, nullptr, objective, &net, &vov, det);
  if (bnb) {
    // QGM_PLAN_BNB: branch and bound from the best min-fill ordering, a
    // node count in proportion to the other half of the budget (so the
    // same on every host); beam of 3 children per node on large graphs
    constexpr double kBnbNodesPerSecond = 200.0;
    int left = 0;
    for (int v = 0; v < g.n; ++v) left += !removed[v];
    const long nodes = std::max(1L, (long)(b1 / 2 * kBnbNodesPerSecond));
    BnbResult r = bnb_order(g, removed, order1, nodes, left <= 20 ? 0 : 3);
    order1 = r.order;
  }
  sliced_vars.clear();
  for (int p : picks) sliced_vars.push_back(net.free_vars[p]);
  order_vars.clear();
  for (int v : order1) order_vars.push_back(net.free_vars[v]);
  if (score) {
    if (flags & 16) {
      // the compiled program of the wide engine (with its regroupings):
      // estimated seconds per slice at the rates those kernels reach
      Program prog;
      std::string err;
      int code = 0;
      if (!compile_program(net, sliced_vars, order_vars, prog, err, code, false, true)) return false;
      // seconds per slice at the rates the wide engine reaches on one
      // MI355X: matrix-core contractions ~65 TFLOP/s, other steps ~30
      // TFLOP/s, streaming ~5 TB/s; with group sharing, in passes of G
      // groups (what 96 GiB holds in complex64, at most 4 and 2^(k - 6)),
      // a step independent of the sliced variables at the varying group
      // bits counts 1 / G
      const int k = (int)sliced_vars.size();
      int G = 1;
      const double group_bytes = (double)prog.item_elems * 64.0 * 8.0;
      while (G < 4 && G < (1 << std::max(0, k - 6)) && (G + 1) * group_bytes <= 96.0 * (1ull << 30)) ++G;
      uint64_t vary = 0;
      if (G > 1) {
        const std::vector<int> pos = group_bit_positions(prog, k);
        for (int y = 1; y < G; ++y)
          for (int t = 0; t < 2 && t < (int)pos.size(); ++t)
            if ((y >> t) & 1) vary |= 1ull << pos[t];
      }
      double sc = 0.0;
      for (const Step& st : prog.steps) {
        if (st.is_const || st.kind == ST_LEAF) continue;
        double elems = std::ldexp(1.0, st.r);
        for (const Operand& o : st.opnd) elems += std::ldexp(1.0, (int)o.vars.size());
        const double t = st.flops / (matrix_core_shape(st) ? 65e12 : 30e12) + 8.0 * elems / 5e12;
        sc += (G > 1 && (st.fix_mask & vary) == 0) ? t / G : t;
      }
      *score = sc;
      if (item_elems) *item_elems = prog.item_elems;
    } else if (objective == OBJ_COST) {
      *score = order_cost(g, order1, removed).cost;
    } else {
      const SimCost sc = simulate(net, vov, g.n, removed, order1);
      *score = objective == OBJ_BYTES ? sc.bytes : std::max(4.0 * sc.cp, sc.flops);
    }
  }
  return true;
}

// QGM_PLAN_SEARCH: whole plans from different seeds, alternately keeping the
// first ordering and re-ordering after each removal, while the time budget
// lasts (each attempt with an eighth of it, at most kAttempts); the plan
// with the best final score is kept.  Seeds vary widely in quality (the
// estimated time per slice of 8x8x40 plans spans 10x), so more attempts
// pay on large circuits.
// The SEARCH loop for one k: the best-scoring plan of the attempts that fit
// in the budget, its score and (WIDE_TIME) its item memory.
static bool search(const Network& net, int k_req, int target_rank, double time_budget_s, uint64_t seed,
                   std::vector<int>& sliced_vars, std::vector<int>& order_vars, int flags, double* best_score,
                   double* best_elems) {
  constexpr int kAttempts = 64;
  const bool det = (flags & 64) != 0;  // deterministic: exactly 8 attempts of budget / 8 each
  const auto t0 = std::chrono::steady_clock::now();
  const double per = time_budget_s / 8;
  bool found = false;
  double best = 0;
  for (int a = 0; a < (det ? 8 : kAttempts); ++a) {
    if (!det && a > 0 &&
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() >= time_budget_s)
      break;
    const int f = (flags & ~1) | (((flags & 1) ^ (a & 1)) ? 1 : 0);
    std::vector<int> sv, ov;
    double score = 0, elems = 0;
    if (!plan_once(net, k_req, target_rank, per, seed + 0x51ed27ull * (a / 2), sv, ov, f, &score, &elems)) continue;
    if (!found || score < best) {
      found = true;
      best = score;
      sliced_vars = sv;
      order_vars = ov;
      if (best_elems) *best_elems = elems;
    }
  }
  if (best_score) *best_score = best;
  return found;
}

bool plan_slices(const Network& net, int k_req, int target_rank, double time_budget_s, uint64_t seed,
                 std::vector<int>& sliced_vars, std::vector<int>& order_vars, int flags) {
  if (!(flags & 8)) return plan_once(net, k_req, target_rank, time_budget_s, seed, sliced_vars, order_vars, flags,
                                     nullptr);
  if (!(flags & 32) || !(flags & 16) || k_req < 0)
    return search(net, k_req, target_rank, time_budget_s, seed, sliced_vars, order_vars, flags, nullptr, nullptr);
  // QGM_PLAN_CHOOSE_K: k_req is the largest k tried.  Each k from k_req down
  // to k_req - 6 gets an equal share of the budget; the plan with the least
  // predicted time for the whole amplitude, 2^k times the per-slice score,
  // wins among those whose item memory fits one 64-item group in 96 GiB.
  constexpr double kMaxGroupBytes = 96.0 * (1ull << 30);
  const int k_lo = std::max(0, k_req - 6);
  const double per_k = time_budget_s / (k_req - k_lo + 1);
  bool found = false;
  double best = 0;
  for (int k = k_req; k >= k_lo; --k) {
    std::vector<int> sv, ov;
    double score = 0, elems = 0;
    if (!search(net, k, 0, per_k, seed, sv, ov, flags & ~32, &score, &elems)) continue;
    if (elems * 64.0 * 16.0 > kMaxGroupBytes) continue;  // complex128 bytes of one group
    const double total = std::ldexp(score, k);
    if (!found || total < best) {
      found = true;
      best = total;
      sliced_vars = sv;
      order_vars = ov;
    }
  }
  return found;
}

}  // namespace qgm
