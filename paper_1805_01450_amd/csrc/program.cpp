// Compiler from (network, sliced variables, elimination order) to the
// per-item contraction program run by the device interpreter.
//
// Variable elimination (Section "Variable elimination"): to eliminate v,
// take T_v (the tensors containing v) and V_v (their variables), multiply
// the tensors of T_v and sum over v.  Here one step does both at once,
// sigma'(V_v \ S) = sum_{S} prod_{tau in T_v} tau, with S = {v} plus every
// other variable that occurs in no tensor outside T_v (summing such a
// variable now equals eliminating it right after v, at lower cost).
//
// Fixing variables (Section "Parallelization by fixing the values of
// variables"): output variables are fixed to x and the k sliced variables
// to the bits of the slice index s; a factor touching a fixed variable
// becomes a leaf whose table is read at the fixed values, per work item.
// Tensors that depend on no fixed variable are the same for every item and
// are computed once per call ("constant" steps).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace qgm {

namespace {

struct Tn {
  std::vector<int> vars;  // bit j of the element index = value of vars[j]
  int is_const;
  int storage;  // element offset: constant area, or item memory (-1: leaf not yet materialised)
  int leaf;     // leaf index or -1
  int alive;
};

// Item-memory buffers have static lifetimes [first step, last step]; after
// compilation they are packed offline (largest first, lowest offset that does
// not overlap any time-overlapping buffer already placed).
struct Buf {
  int size, first, last, offset;
};

int pack_buffers(std::vector<Buf>& bufs) {
  std::vector<int> idx(bufs.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (bufs[a].size != bufs[b].size) return bufs[a].size > bufs[b].size;
    return bufs[a].first < bufs[b].first;
  });
  std::vector<int> placed;
  int peak = 0;
  std::vector<std::pair<int, int>> busy;
  for (int i : idx) {
    Buf& b = bufs[i];
    busy.clear();
    for (int j : placed) {
      const Buf& o = bufs[j];
      if (o.first <= b.last && b.first <= o.last) busy.push_back({o.offset, o.offset + o.size});
    }
    std::sort(busy.begin(), busy.end());
    int at = 0;
    for (auto& r : busy) {
      if (r.first >= at + b.size) break;
      at = std::max(at, r.second);
    }
    b.offset = at;
    peak = std::max(peak, at + b.size);
    placed.push_back(i);
  }
  return peak;
}

constexpr int kMaxStepBits = 16;
constexpr size_t kMaxOptab = (size_t)1 << 26;

}  // namespace

bool validate_plan(const Network& net, const std::vector<int>& sliced, const std::vector<int>& order,
                   std::string& err, int& code) {
  const int nvars = (int)net.vars.size();
  if (sliced.size() > 40) {
    err = "at most 40 sliced variables";
    code = -4;
    return false;
  }
  std::vector<int> fixed_src(nvars, -1), fixed_bit(nvars, -1);
  for (int q = 0; q < net.n_qubits; ++q) {
    int v = net.output_var[q];
    if (v >= 0) {
      fixed_src[v] = 0;
      fixed_bit[v] = q;
    }
  }
  for (size_t j = 0; j < sliced.size(); ++j) {
    int v = sliced[j];
    if (v < 0 || v >= nvars || net.vars[v].is_output) {
      err = "sliced variable " + std::to_string(v) + " is not a free variable";
      code = -4;
      return false;
    }
    if (fixed_src[v] >= 0) {
      err = "sliced variable " + std::to_string(v) + " listed twice";
      code = -4;
      return false;
    }
    fixed_src[v] = 1;
    fixed_bit[v] = (int)j;
  }
  std::vector<int> pos(nvars, -1);
  for (size_t i = 0; i < order.size(); ++i) {
    int v = order[i];
    if (v < 0 || v >= nvars || fixed_src[v] >= 0 || pos[v] >= 0) {
      err = "order entry " + std::to_string(v) + " is not a free, non-sliced variable or is repeated";
      code = -3;
      return false;
    }
    pos[v] = (int)i;
  }
  for (int v : net.free_vars) {
    if (fixed_src[v] < 0 && pos[v] < 0) {
      err = "order misses free variable " + std::to_string(v);
      code = -3;
      return false;
    }
  }
  return true;
}

bool compile_program(const Network& net, const std::vector<int>& sliced, const std::vector<int>& order,
                     Program& prog, std::string& err, int& code) {
  prog = Program();
  if (!validate_plan(net, sliced, order, err, code)) return false;
  const int nvars = (int)net.vars.size();
  std::vector<int> fixed_src(nvars, -1), fixed_bit(nvars, -1);
  for (int q = 0; q < net.n_qubits; ++q) {
    int v = net.output_var[q];
    if (v >= 0) {
      fixed_src[v] = 0;
      fixed_bit[v] = q;
    }
  }
  for (size_t j = 0; j < sliced.size(); ++j) {
    fixed_src[sliced[j]] = 1;
    fixed_bit[sliced[j]] = (int)j;
  }
  std::vector<int> pos(nvars, -1);
  for (size_t i = 0; i < order.size(); ++i) pos[order[i]] = (int)i;

  // ---- raw tables (constant area prefix)
  std::vector<int> raw_off(net.factors.size(), -1);
  auto push_raw = [&](double re, double im, int param, int bit) {
    prog.raw.push_back(re);
    prog.raw.push_back(im);
    prog.raw_param.push_back(param);
    prog.raw_bit.push_back(bit);
    return prog.n_raw++;
  };
  for (size_t f = 0; f < net.factors.size(); ++f) {
    const Factor& fa = net.factors[f];
    int n = 1 << fa.nv;
    raw_off[f] = prog.n_raw;
    for (int e = 0; e < n; ++e) {
      if (fa.param >= 0)
        push_raw(0.0, 0.0, fa.param, fa.nv == 0 ? 0 : (e & 1));
      else
        push_raw(fa.tab[2 * e], fa.tab[2 * e + 1], -1, 0);
    }
  }
  int delta_tab = push_raw(1.0, 0.0, -1, 0);
  push_raw(0.0, 0.0, -1, 0);
  int two_tab = push_raw(2.0, 0.0, -1, 0);

  // ---- leaves and initial tensors
  std::vector<Tn> T;
  for (size_t f = 0; f < net.factors.size(); ++f) {
    const Factor& fa = net.factors[f];
    Leaf L{};
    L.factor = (int)f;
    L.table = raw_off[f];
    std::vector<int> fv;
    for (int j = 0; j < fa.nv; ++j) {
      int v = fa.var[j];
      if (fixed_src[v] >= 0) {
        L.dep_src[L.ndep] = fixed_src[v];
        L.dep_bit[L.ndep] = fixed_bit[v];
        L.dep_stride[L.ndep] = 1 << j;
        L.ndep++;
      } else {
        L.free_var[L.nfree] = v;
        L.free_stride[L.nfree] = 1 << j;
        L.nfree++;
        fv.push_back(v);
      }
    }
    Tn t;
    t.vars = fv;
    t.alive = 1;
    if (L.ndep == 0) {
      // constant: the raw table itself, element index = factor's own layout
      t.is_const = 1;
      t.storage = raw_off[f];
      t.leaf = -1;
    } else {
      t.is_const = 0;
      t.storage = -1;
      t.leaf = (int)prog.leaves.size();
      prog.leaves.push_back(L);
    }
    T.push_back(t);
  }
  for (int q = 0; q < net.n_qubits; ++q) {
    if (net.output_var[q] >= 0) continue;
    Leaf L{};
    L.factor = -1;
    L.table = delta_tab;
    L.ndep = 1;
    L.dep_src[0] = 0;
    L.dep_bit[0] = q;
    L.dep_stride[0] = 1;
    Tn t;
    t.is_const = 0;
    t.storage = -1;
    t.leaf = (int)prog.leaves.size();
    t.alive = 1;
    prog.leaves.push_back(L);
    T.push_back(t);
  }

  std::vector<int> count(nvars, 0);
  for (auto& t : T)
    for (int v : t.vars) count[v]++;

  std::vector<Buf> bufs;        // item-memory buffers (Tn::storage holds the buffer id)
  std::vector<int> op_buf;       // per optab entry: buffer id or -1 (constant)
  std::vector<int> step_buf;     // per step: output buffer id or -1
  auto new_buf = [&](int size) {
    bufs.push_back(Buf{size, (int)prog.steps.size(), (int)prog.steps.size(), 0});
    return (int)bufs.size() - 1;
  };
  int const_top = prog.n_raw;
  std::vector<char> done(nvars, 0);
  int n_two = 0;

  auto materialise = [&](Tn& t) {
    if (t.is_const || t.storage >= 0) return;
    int n = 1 << t.vars.size();
    t.storage = new_buf(n);
    Step st{};
    st.kind = ST_LEAF;
    st.out = 0;
    st.r = (int)t.vars.size();
    st.leaf = t.leaf;
    prog.steps.push_back(st);
    step_buf.push_back(t.storage);
  };
  // Constant operands get their final offset now; item operands are patched
  // after buffer packing.  Reading a buffer extends its lifetime to this step.
  auto operand_entry = [&](const Tn& t, int off) -> uint32_t {
    if (t.is_const) {
      op_buf.push_back(-1);
      return OP_CONST | (uint32_t)(t.storage + off);
    }
    op_buf.push_back(t.storage);
    bufs[t.storage].last = (int)prog.steps.size();
    return (uint32_t)off;
  };

  for (int v : order) {
    if (done[v]) continue;
    std::vector<int> tv;
    for (size_t i = 0; i < T.size(); ++i)
      if (T[i].alive && std::find(T[i].vars.begin(), T[i].vars.end(), v) != T[i].vars.end()) tv.push_back((int)i);
    if (tv.empty()) {
      done[v] = 1;
      n_two++;
      continue;
    }
    std::vector<int> vv;
    std::vector<int> cnt_in(nvars, 0);
    for (int i : tv)
      for (int u : T[i].vars) {
        if (cnt_in[u] == 0) vv.push_back(u);
        cnt_in[u]++;
      }
    std::vector<int> S{v}, out;
    for (int u : vv) {
      if (u == v) continue;
      if (cnt_in[u] == count[u]) S.push_back(u);
      else out.push_back(u);
    }
    std::sort(out.begin(), out.end(), [&](int a, int b) { return pos[a] < pos[b]; });
    std::sort(S.begin(), S.end(), [&](int a, int b) { return pos[a] < pos[b]; });
    int r = (int)out.size(), ns = (int)S.size(), m = (int)tv.size();
    bool all_const = true;
    for (int i : tv) {
      materialise(T[i]);
      all_const = all_const && T[i].is_const;
    }
    Tn nt;
    nt.vars = out;
    nt.is_const = all_const ? 1 : 0;
    nt.leaf = -1;
    nt.alive = 1;
    if (all_const) {
      nt.storage = const_top;
      const_top += 1 << r;
    } else {
      nt.storage = new_buf(1 << r);
    }
    Step st{};
    st.kind = ST_ELIM;
    st.is_const = nt.is_const;
    st.out = nt.storage;
    st.r = r;
    st.ns = ns;
    st.m = m;
    st.ops = (int)prog.optab.size();
    // value of each variable of V_v at (c, s)
    std::vector<int> bitpos(nvars, -1), from_s(nvars, 0);
    for (int j = 0; j < r; ++j) bitpos[out[j]] = j;
    for (int j = 0; j < ns; ++j) {
      bitpos[S[j]] = j;
      from_s[S[j]] = 1;
    }
    if (r + ns > kMaxStepBits || prog.optab.size() + ((size_t)m << (r + ns)) > kMaxOptab) {
      err = "plan has a step of rank " + std::to_string(r) + " summing " + std::to_string(ns) +
            " variables; the per-item program supports rank + summed <= " + std::to_string(kMaxStepBits);
      code = -7;
      return false;
    }
    for (int c = 0; c < (1 << r); ++c)
      for (int s = 0; s < (1 << ns); ++s)
        for (int i : tv) {
          int off = 0;
          const Tn& t = T[i];
          for (size_t j = 0; j < t.vars.size(); ++j) {
            int u = t.vars[j];
            int val = from_s[u] ? (s >> bitpos[u]) & 1 : (c >> bitpos[u]) & 1;
            off |= val << j;
          }
          prog.optab.push_back(operand_entry(t, off));
        }
    st.flops = std::ldexp(1.0, r + ns) * (6.0 * (m - 1) + 2.0);
    prog.steps.push_back(st);
    step_buf.push_back(all_const ? -1 : nt.storage);
    prog.max_rank = std::max(prog.max_rank, r);
    if (all_const) {
      prog.flops_const += st.flops;
      prog.n_const_steps++;
    } else {
      prog.flops_item += st.flops;
      double in_elems = 0;
      for (int i : tv) in_elems += std::ldexp(1.0, (int)T[i].vars.size());
      prog.bytes_item += 8.0 * (in_elems + std::ldexp(1.0, r));
    }
    for (int i : tv) {
      for (int u : T[i].vars) count[u]--;
      T[i].alive = 0;
    }
    for (int u : S) done[u] = 1;
    for (int u : out) count[u]++;
    T.push_back(nt);
  }

  // ---- final product of the remaining scalars
  std::vector<int> rest;
  for (size_t i = 0; i < T.size(); ++i) {
    if (!T[i].alive) continue;
    if (!T[i].vars.empty()) {
      err = "internal: variable left after elimination";
      code = -3;
      return false;
    }
    rest.push_back((int)i);
  }
  for (int i : rest) materialise(T[i]);
  Step fin{};
  fin.kind = ST_FINAL;
  fin.m = (int)rest.size() + n_two;
  fin.ops = (int)prog.optab.size();
  for (int i : rest) prog.optab.push_back(operand_entry(T[i], 0));
  for (int i = 0; i < n_two; ++i) {
    prog.optab.push_back(OP_CONST | (uint32_t)two_tab);
    op_buf.push_back(-1);
  }
  fin.flops = 6.0 * std::max(0, fin.m - 1);
  prog.flops_item += fin.flops;
  prog.steps.push_back(fin);
  step_buf.push_back(-1);
  prog.n_const = const_top;
  prog.item_elems = std::max(1, pack_buffers(bufs));
  for (size_t i = 0; i < prog.optab.size(); ++i)
    if (op_buf[i] >= 0) prog.optab[i] += (uint32_t)bufs[op_buf[i]].offset;
  for (size_t i = 0; i < prog.steps.size(); ++i)
    if (step_buf[i] >= 0) prog.steps[i].out = bufs[step_buf[i]].offset;
  // constant steps must come first in execution; they only read constants, so
  // a stable partition keeps every dependency satisfied.
  std::stable_partition(prog.steps.begin(), prog.steps.end(), [](const Step& s) { return s.is_const; });
  return true;
}

}  // namespace qgm
