// Circuit text parser and graphical-model builder (Section "Undirected
// Graphical Model"; gate gadgets of Fig. "tensornodes").
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <sstream>

#include "host.h"

namespace qgm {

namespace {

bool gate_kind(const std::string& s, GateKind& k) {
  if (s == "H") k = G_H;
  else if (s == "SX") k = G_SX;
  else if (s == "SY") k = G_SY;
  else if (s == "T") k = G_T;
  else if (s == "RZ") k = G_RZ;
  else if (s == "I") k = G_I;
  else if (s == "CZ") k = G_CZ;
  else if (s == "CX") k = G_CX;
  else if (s == "ISWAP") k = G_ISWAP;
  else if (s == "SQISW") k = G_SQISW;
  else return false;
  return true;
}

bool to_int(const std::string& s, int& v) {
  if (s.empty()) return false;
  char* end = nullptr;
  long x = std::strtol(s.c_str(), &end, 10);
  if (*end != '\0' || x < -2147483647L || x > 2147483647L) return false;
  v = (int)x;
  return true;
}

// Non-diagonal one-qubit gate matrices U[out][in], (re, im).
//   H  = (1/sqrt 2)[[1, 1], [1, -1]]
//   SX = principal square root of X = 1/2 [[1+i, 1-i], [1-i, 1+i]]
//   SY = principal square root of Y = 1/2 [[1+i, -1-i], [1+i, 1+i]]
void nondiag_matrix(GateKind k, double u[2][2][2]) {
  const double h = 0.70710678118654752440;
  if (k == G_H) {
    double m[2][2][2] = {{{h, 0}, {h, 0}}, {{h, 0}, {-h, 0}}};
    std::memcpy(u, m, sizeof(m));
  } else if (k == G_SX) {
    double m[2][2][2] = {{{0.5, 0.5}, {0.5, -0.5}}, {{0.5, -0.5}, {0.5, 0.5}}};
    std::memcpy(u, m, sizeof(m));
  } else {
    double m[2][2][2] = {{{0.5, 0.5}, {-0.5, -0.5}}, {{0.5, 0.5}, {0.5, 0.5}}};
    std::memcpy(u, m, sizeof(m));
  }
}

bool two_qubit(GateKind k) { return k == G_CZ || k == G_CX || k == G_ISWAP || k == G_SQISW; }

// Non-diagonal two-qubit gate matrices U[out][in], (re, im), over the index
// bit(q0) + 2 bit(q1):
//   CX: control q0, target q1, |c t> -> |c, t xor c>
//   ISWAP: |01> -> i|10>, |10> -> i|01>, |00> and |11> unchanged
//   SQISW: the square root of ISWAP, (1/sqrt 2)[[1, i], [i, 1]] on {|01>, |10>}
void nondiag2_matrix(GateKind k, double u[4][4][2]) {
  std::memset(u, 0, sizeof(double) * 32);
  if (k == G_CX) {
    for (int c = 0; c < 2; ++c)
      for (int t = 0; t < 2; ++t) u[c + 2 * (t ^ c)][c + 2 * t][0] = 1.0;
    return;
  }
  const double h = 0.70710678118654752440;
  u[0][0][0] = u[3][3][0] = 1.0;
  if (k == G_ISWAP) {
    u[2][1][1] = u[1][2][1] = 1.0;
  } else {
    u[1][1][0] = u[2][2][0] = h;
    u[2][1][1] = u[1][2][1] = h;
  }
}

}  // namespace

bool parse_circuit(const char* text, size_t len, Network& net, std::string& err) {
  net = Network();
  std::string s(text, len);
  std::istringstream in(s);
  std::string raw;
  int lineno = 0;
  int nq = -1;
  while (std::getline(in, raw)) {
    ++lineno;
    size_t hash = raw.find('#');
    if (hash != std::string::npos) raw.resize(hash);
    std::istringstream ls(raw);
    std::vector<std::string> tok;
    std::string t;
    while (ls >> t) tok.push_back(t);
    if (tok.empty()) continue;
    auto fail = [&](const std::string& why) {
      err = "line " + std::to_string(lineno) + ": " + why;
      return false;
    };
    if (tok[0] == "qubits") {
      int v;
      if (tok.size() != 2 || !to_int(tok[1], v) || v < 0 || v > 64) return fail("bad 'qubits' header (0..64)");
      nq = v;
      continue;
    }
    if (tok[0] == "grid") continue;
    if (nq < 0) return fail("gate before 'qubits' header");
    Gate g{};
    g.line = lineno;
    g.q1 = -1;
    g.param = -1;
    if (!to_int(tok[0], g.cycle) || g.cycle < 0) return fail("bad cycle");
    if (tok.size() < 2 || !gate_kind(tok[1], g.kind)) return fail("unknown gate");
    size_t want = (two_qubit(g.kind) || g.kind == G_RZ) ? 4 : 3;
    if (tok.size() != want) return fail("wrong number of fields for " + tok[1]);
    if (!to_int(tok[2], g.q0) || g.q0 < 0 || g.q0 >= nq) return fail("qubit out of range");
    if (two_qubit(g.kind)) {
      if (!to_int(tok[3], g.q1) || g.q1 < 0 || g.q1 >= nq) return fail("qubit out of range");
      if (g.q1 == g.q0) return fail(tok[1] + " on a single qubit");
    } else if (g.kind == G_RZ) {
      if (!to_int(tok[3], g.param) || g.param < 0 || g.param > (1 << 24)) return fail("bad parameter index");
      net.n_params = std::max(net.n_params, g.param + 1);
    }
    net.gates.push_back(g);
  }
  if (nq < 0) {
    err = "missing 'qubits N' header";
    return false;
  }
  net.n_qubits = nq;
  // gates of one cycle must act on distinct qubits
  std::vector<Gate> sorted = net.gates;
  std::stable_sort(sorted.begin(), sorted.end(), [](const Gate& a, const Gate& b) { return a.cycle < b.cycle; });
  std::vector<int> last_cycle(nq, -1);
  for (const Gate& g : sorted) {
    int qs[2] = {g.q0, g.q1};
    for (int q : qs) {
      if (q < 0) continue;
      if (last_cycle[q] == g.cycle) {
        err = "line " + std::to_string(g.line) + ": two gates on qubit " + std::to_string(q) + " in cycle " +
              std::to_string(g.cycle);
        return false;
      }
      last_cycle[q] = g.cycle;
    }
  }
  net.gates = sorted;
  return true;
}

// Variables are created by non-diagonal one-qubit gates, taken by ascending
// cycle and, inside a cycle, ascending (lowest) qubit.  The input index i_0 is
// the constant 0 (marker -1); a factor touching it is indexed at 0 here.
void build_network(Network& net) {
  std::vector<Gate> gs = net.gates;
  std::stable_sort(gs.begin(), gs.end(), [](const Gate& a, const Gate& b) {
    if (a.cycle != b.cycle) return a.cycle < b.cycle;
    int qa = a.q1 >= 0 ? std::min(a.q0, a.q1) : a.q0;
    int qb = b.q1 >= 0 ? std::min(b.q0, b.q1) : b.q0;
    return qa < qb;
  });
  std::vector<int> cur(net.n_qubits, -1);
  net.vars.clear();
  net.factors.clear();
  for (const Gate& g : gs) {
    Factor f{};
    f.param = -1;
    if (g.kind == G_CZ) {
      int u = cur[g.q0], w = cur[g.q1];
      if (u < 0 || w < 0) continue;  // CZ with |0> on one side is the identity
      f.nv = 2;
      f.var[0] = u;
      f.var[1] = w;
      for (int b = 0; b < 4; ++b) {
        f.tab[2 * b] = (b == 3) ? -1.0 : 1.0;
        f.tab[2 * b + 1] = 0.0;
      }
      net.factors.push_back(f);
    } else if (g.kind == G_CX || g.kind == G_ISWAP || g.kind == G_SQISW) {
      // Not diagonal: a new variable on each qubit (the lower qubit's
      // first) and one factor over the new and the old variables, U[new
      // a, new b][old a, old b] (the K4 gadget of Fig. "tensornodes").  An
      // old index that is still the input constant 0 is fixed at 0.
      double m[4][4][2];
      nondiag2_matrix(g.kind, m);
      const int a = g.q0, b = g.q1;
      int nv[2];
      for (int q : {std::min(a, b), std::max(a, b)}) {
        const int v = (int)net.vars.size();
        net.vars.push_back(Var{v, q, g.cycle, 0});
        nv[q == a ? 0 : 1] = v;
      }
      const int old[2] = {cur[a], cur[b]};
      f.nv = 0;
      f.var[f.nv++] = nv[0];
      f.var[f.nv++] = nv[1];
      int old_bit[2] = {-1, -1};  // position of the old variable in f.var, or -1 (fixed at 0)
      for (int j = 0; j < 2; ++j)
        if (old[j] >= 0) {
          old_bit[j] = f.nv;
          f.var[f.nv++] = old[j];
        }
      for (int e = 0; e < (1 << f.nv); ++e) {
        const int out = (e & 1) + 2 * ((e >> 1) & 1);
        int in = 0;
        for (int j = 0; j < 2; ++j)
          if (old_bit[j] >= 0) in |= ((e >> old_bit[j]) & 1) << j;
        f.tab[2 * e] = m[out][in][0];
        f.tab[2 * e + 1] = m[out][in][1];
      }
      net.factors.push_back(f);
      cur[a] = nv[0];
      cur[b] = nv[1];
    } else if (g.kind == G_I) {
      continue;  // identity: no factor
    } else if (g.kind == G_T || g.kind == G_RZ) {
      int u = cur[g.q0];
      if (g.kind == G_T) {
        // T = diag(1, e^{i pi/4})
        const double c = 0.70710678118654752440;
        double d[4] = {1.0, 0.0, c, c};
        if (u < 0) continue;  // T on |0> multiplies by 1
        f.nv = 1;
        f.var[0] = u;
        std::memcpy(f.tab, d, sizeof(d));
      } else {
        f.param = g.param;
        if (u < 0) {
          f.nv = 0;  // RZ on |0>: scalar e^{-i theta/2}, made on the device
        } else {
          f.nv = 1;
          f.var[0] = u;
        }
      }
      net.factors.push_back(f);
    } else {
      double m[2][2][2];
      nondiag_matrix(g.kind, m);
      int v = (int)net.vars.size();
      net.vars.push_back(Var{v, g.q0, g.cycle, 0});
      int old = cur[g.q0];
      if (old < 0) {
        f.nv = 1;
        f.var[0] = v;
        for (int b = 0; b < 2; ++b) {
          f.tab[2 * b] = m[b][0][0];
          f.tab[2 * b + 1] = m[b][0][1];
        }
      } else {
        f.nv = 2;
        f.var[0] = v;
        f.var[1] = old;
        for (int bo = 0; bo < 2; ++bo)
          for (int bn = 0; bn < 2; ++bn) {
            int e = bn + 2 * bo;
            f.tab[2 * e] = m[bn][bo][0];
            f.tab[2 * e + 1] = m[bn][bo][1];
          }
      }
      net.factors.push_back(f);
      cur[g.q0] = v;
    }
  }
  net.output_var = cur;
  for (int q = 0; q < net.n_qubits; ++q)
    if (cur[q] >= 0) net.vars[cur[q]].is_output = 1;
  net.free_vars.clear();
  for (const Var& v : net.vars)
    if (!v.is_output) net.free_vars.push_back(v.id);
}

}  // namespace qgm
