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
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <cmath>
#include <cstring>

#include "host.h"

namespace qgm {

namespace {


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

namespace {

// Compile-time tensor.
struct Tn {
  std::vector<int> vars;  // bit j of the element index = value of vars[j]
  int is_const = 0;
  int storage = -1;       // constant: element offset; item: buffer id (-1: leaf not materialised)
  int leaf = -1;          // leaf index or -1
  int alive = 1;
  int grad = 0;           // depends on an RZ angle (gradient programs)
  int rz_factor = -1;     // tensor is the table/leaf of this RZ factor
  int producer = -1;      // forward step that produced it
  int id = -1;            // index in the tensor list
  std::vector<int> inputs;  // tensors consumed by the producing step
  uint64_t fix_mask = 0;    // fixed variables it depends on (as Step::fix_mask)
};

int popc_bits(int x) { return __builtin_popcount((unsigned)x); }

}  // namespace

bool matrix_core_shape(const Step& st) {
  if (st.kind != ST_ELIM || st.is_const || st.opnd.size() < 2 || st.opnd.size() > 3 || st.ns < 1) return false;
  const Operand& a = st.opnd[0];
  const Operand& b = st.opnd[1];
  if (a.is_const || b.is_const) return false;
  auto has = [](const Operand& o, int v) { return std::find(o.vars.begin(), o.vars.end(), v) != o.vars.end(); };
  if (st.opnd.size() == 3) {
    // a constant scale of the output, applied to the results
    const Operand& c = st.opnd[2];
    if (!c.is_const) return false;
    for (int v : c.vars)
      if (std::find(st.out_vars.begin(), st.out_vars.end(), v) == st.out_vars.end()) return false;
  }
  int rows = 0, cols = 0;
  for (int v : st.out_vars) {
    const bool ia = has(a, v), ib = has(b, v);
    if (ia && !ib) ++rows;
    if (ib && !ia) ++cols;
    if (!ia && !ib) return false;
  }
  for (int v : st.sum_vars)
    if (!has(a, v) || !has(b, v)) return false;
  return rows >= 4 && cols >= 4;
}

bool compile_program(const Network& net, const std::vector<int>& sliced, const std::vector<int>& order,
                     Program& prog, std::string& err, int& code, bool gradient, bool combine_consts,
                     int checkpoint_every, const std::vector<int>& open_qubits) {
  prog = Program();
  if (!validate_plan(net, sliced, order, err, code)) return false;
  const int nvars = (int)net.vars.size();
  // Open outputs: the output variables of these qubits are neither fixed
  // nor summed; the final product keeps them, bit i of its element index
  // being the output of open_qubits[i] (2^j amplitudes per contraction).
  std::vector<char> is_open(nvars, 0);
  std::vector<int> open_vars;
  for (int q : open_qubits) {
    if (q < 0 || q >= net.n_qubits || net.output_var[q] < 0 || is_open[net.output_var[q]]) {
      err = "open qubit " + std::to_string(q) + " is out of range, repeated, or has no variable of its own";
      code = -1;
      return false;
    }
    is_open[net.output_var[q]] = 1;
    open_vars.push_back(net.output_var[q]);
  }
  if (!open_vars.empty() && gradient) {
    err = "open outputs and gradients cannot be combined";
    code = -7;
    return false;
  }
  prog.n_open = (int)open_vars.size();
  std::vector<int> fixed_src(nvars, -1), fixed_bit(nvars, -1);
  for (int q = 0; q < net.n_qubits; ++q) {
    int v = net.output_var[q];
    if (v >= 0 && !is_open[v]) {
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

  // ---- raw tables (constant-area prefix)
  auto push_raw = [&](double re, double im, int param, int bit, int deriv) {
    prog.raw.push_back(re);
    prog.raw.push_back(im);
    prog.raw_param.push_back(param);
    prog.raw_bit.push_back(bit);
    prog.raw_deriv.push_back(deriv);
    return prog.n_raw++;
  };
  std::vector<int> raw_off(net.factors.size(), -1), deriv_off(net.factors.size(), -1);
  for (size_t f = 0; f < net.factors.size(); ++f) {
    const Factor& fa = net.factors[f];
    int n = 1 << fa.nv;
    raw_off[f] = prog.n_raw;
    for (int e = 0; e < n; ++e) {
      if (fa.param >= 0)
        push_raw(0.0, 0.0, fa.param, fa.nv == 0 ? 0 : (e & 1), 0);
      else
        push_raw(fa.tab[2 * e], fa.tab[2 * e + 1], -1, 0, 0);
    }
    if (gradient && fa.param >= 0) {
      deriv_off[f] = prog.n_raw;
      for (int e = 0; e < n; ++e) push_raw(0.0, 0.0, fa.param, fa.nv == 0 ? 0 : (e & 1), 1);
    }
  }
  const int delta_tab = push_raw(1.0, 0.0, -1, 0, 0);
  push_raw(0.0, 0.0, -1, 0, 0);
  const int two_tab = push_raw(2.0, 0.0, -1, 0, 0);
  const int one_tab = push_raw(1.0, 0.0, -1, 0, 0);

  // ---- leaves and initial tensors
  std::vector<Tn> T;
  auto make_leaf = [&](int f, int table) {
    const Factor& fa = net.factors[f];
    Leaf L{};
    L.factor = f;
    L.table = table;
    std::vector<int> fv;
    uint64_t fm = 0;
    for (int j = 0; j < fa.nv; ++j) {
      int v = fa.var[j];
      if (fixed_src[v] >= 0) {
        fm |= fixed_src[v] == 1 ? 1ull << fixed_bit[v] : 1ull << 63;
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
    t.id = (int)T.size();
    t.fix_mask = fm;
    if (L.ndep == 0) {
      t.is_const = 1;
      t.storage = table;
    } else {
      t.leaf = (int)prog.leaves.size();
      prog.leaves.push_back(L);
    }
    return t;
  };
  for (size_t f = 0; f < net.factors.size(); ++f) {
    Tn t = make_leaf((int)f, raw_off[f]);
    if (gradient && net.factors[f].param >= 0) {
      t.grad = 1;
      t.rz_factor = (int)f;
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
    t.leaf = (int)prog.leaves.size();
    t.id = (int)T.size();
    t.fix_mask = 1ull << 63;
    prog.leaves.push_back(L);
    T.push_back(t);
  }

  std::vector<int> count(nvars, 0);
  for (auto& t : T)
    for (int v : t.vars) count[v]++;

  std::vector<Buf> bufs;
  std::vector<int> step_buf;  // per step: output buffer id or -1
  int const_top = prog.n_raw;
  auto new_buf = [&](int size) {
    bufs.push_back(Buf{size, (int)prog.steps.size(), (int)prog.steps.size(), 0});
    return (int)bufs.size() - 1;
  };
  auto materialise = [&](Tn& t) {
    if (t.is_const || t.storage >= 0) return;
    t.storage = new_buf(1 << t.vars.size());
    Step st;
    st.kind = ST_LEAF;
    st.r = (int)t.vars.size();
    st.leaf = t.leaf;
    st.out_tid = t.id;
    st.fix_mask = t.fix_mask;
    prog.steps.push_back(st);
    step_buf.push_back(t.storage);
  };
  auto as_operand = [&](const Tn& t) {
    Operand o;
    o.is_const = t.is_const;
    o.storage = t.storage;
    o.vars = t.vars;
    o.tid = t.id;
    o.fix_mask = t.fix_mask;
    if (!t.is_const) bufs[t.storage].last = (int)prog.steps.size();
    return o;
  };
  // Append a product-sum step; returns the index of the new tensor (or -1
  // for FINAL / GRAD steps, which write outside item memory).
  std::vector<int> elim_created;  // every tensor made by an ELIM step, in creation order
  auto emit_one = [&](int kind, const std::vector<int>& in, const std::vector<int>& out_vars,
                      const std::vector<int>& sum_vars, bool make_const, int grad_slot, int extra_const,
                      int n_extra) -> int {
    Step st;
    st.kind = kind;
    st.out_vars = out_vars;
    st.sum_vars = sum_vars;
    st.r = (int)out_vars.size();
    st.ns = (int)sum_vars.size();
    st.grad_slot = grad_slot;
    // leaves first: a leaf step pushed between two operand reads would end the
    // earlier operand's lifetime before this step
    for (int i : in) materialise(T[i]);
    for (int i : in) st.opnd.push_back(as_operand(T[i]));
    for (int e = 0; e < n_extra; ++e) st.opnd.push_back(Operand{1, extra_const, {}});
    st.m = (int)st.opnd.size();
    // item steps multiply the operands that carry no summed variable into
    // each sum once (the wide kernels do; plans of the other engines have
    // no such operand); constant steps multiply every operand in the loop
    int m_in = st.m, m_out = 0;
    if (!make_const) {
      m_in = 0;
      for (const Operand& o : st.opnd) {
        bool summed = false;
        for (int u : o.vars) summed = summed || std::find(sum_vars.begin(), sum_vars.end(), u) != sum_vars.end();
        (summed ? m_in : m_out)++;
      }
    }
    st.flops = step_flops(st.r, st.ns, m_in, m_out);
    for (int i : in) st.fix_mask |= T[i].fix_mask;
    if (kind != ST_ELIM) st.fix_mask = ~0ull;  // per-item results: every item writes its own
    int id = -1, buf = -1;
    if (kind == ST_ELIM) {
      Tn nt;
      nt.vars = out_vars;
      nt.is_const = make_const ? 1 : 0;
      if (make_const) {
        nt.storage = const_top;
        const_top += 1 << st.r;
      } else {
        nt.storage = buf = new_buf(1 << st.r);
      }
      st.is_const = nt.is_const;
      st.out = nt.storage;
      nt.producer = (int)prog.steps.size();
      nt.inputs = in;
      nt.id = (int)T.size();
      st.out_tid = nt.id;
      for (int i : in) nt.grad |= T[i].grad;
      nt.fix_mask = st.fix_mask;
      T.push_back(nt);
      id = (int)T.size() - 1;
      elim_created.push_back(id);
    }
    // the output buffer is placed after inputs are read: a step's inputs and
    // output never share memory because their lifetimes overlap at the step
    // (first == last == this step for the output start)
    prog.steps.push_back(st);
    step_buf.push_back(buf);
    prog.max_rank = std::max(prog.max_rank, st.r);
    if (st.is_const) {
      prog.flops_const += st.flops;
      prog.n_const_steps++;
    } else {
      prog.flops_item += st.flops;
      double in_elems = 0;
      for (const Operand& o : prog.steps.back().opnd) in_elems += std::ldexp(1.0, (int)o.vars.size());
      const double bytes = 8.0 * (in_elems + std::ldexp(1.0, st.r));
      prog.bytes_item += bytes;
      prog.roof_s_item += std::max(st.flops / 157.3e12, bytes / 8e12);
      if (matrix_core_shape(prog.steps.back())) prog.flops_mc_item += st.flops;
    }
    return id;
  };

  // A step that sums many variables into a small output has little
  // parallelism across output elements; it is split into a partial-sum step
  // that keeps some summed variables as outputs and a plain sum over them
  // (repeated while the remaining sum is still large).
  constexpr int kSplitSum = 8, kKeepSum = 6, kSplitRank = 14;
  constexpr int kMaxCombinedRank = 20;  // largest constant tensor made by combining constant factors
  // (the lists are taken by value: callers pass the variables of a tensor in
  // T, and emit_one appends to T, which may move its elements)
  std::function<int(int, std::vector<int>, std::vector<int>, std::vector<int>, bool, int, int, int)> emit;
  emit = [&](int kind, std::vector<int> in, std::vector<int> out_vars, std::vector<int> sum_vars, bool make_const,
             int grad_slot, int extra_const, int n_extra) -> int {
    const int ns = (int)sum_vars.size(), r = (int)out_vars.size();
    if (ns <= kSplitSum || in.empty()) return emit_one(kind, in, out_vars, sum_vars, make_const, grad_slot,
                                                       extra_const, n_extra);
    const int h = std::max(1, std::min(ns - kKeepSum, std::max(1, kSplitRank - r)));
    std::vector<int> keep(sum_vars.end() - h, sum_vars.end());
    std::vector<int> inner(sum_vars.begin(), sum_vars.end() - h);
    std::vector<int> part_out = out_vars;
    part_out.insert(part_out.end(), keep.begin(), keep.end());
    int part = emit_one(ST_ELIM, in, part_out, inner, make_const, -1, 0, 0);
    int id = emit(kind, {part}, out_vars, keep, make_const, grad_slot, extra_const, n_extra);
    T[part].alive = 0;  // consumed by the sum step just emitted
    return id;
  };

  // ---- forward: variable elimination along the order
  std::vector<char> done(nvars, 0);
  int n_two = 0;

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
    // summed: variables all of whose tensors are in tv (v among them)
    std::vector<int> S, out;
    auto split_vars = [&]() {
      std::vector<int> vv;
      std::vector<int> cnt_in(nvars, 0);
      for (int i : tv)
        for (int u : T[i].vars) {
          if (cnt_in[u] == 0) vv.push_back(u);
          cnt_in[u]++;
        }
      S.clear();
      out.clear();
      for (int u : vv) (cnt_in[u] == count[u] && !is_open[u] ? S : out).push_back(u);
      std::sort(out.begin(), out.end(), [&](int a, int b) { return pos[a] < pos[b]; });
      std::sort(S.begin(), S.end(), [&](int a, int b) { return pos[a] < pos[b]; });
    };
    split_vars();
    if (combine_consts && !gradient) {
      // A large step also takes over the eliminations that follow it in the
      // order while each touches its output and, besides, only small tensors
      // (constants, leaves, or at most 2^10 elements) over variables the
      // step already spans plus new ones: those variables are summed here,
      // and the large intermediates between the steps are never written (the
      // sums are regrouped; the pairwise pre-contraction below then folds
      // such a factor into the operand it shares variables with).  Each
      // absorbed variable may bring one variable new to the step (it is
      // summed itself, so the output rank stays); a factor that brings two
      // is taken when the next absorption brings none, and the step falls
      // back to the last state where the count balances.
      constexpr int kFuseMinSpan = 16, kFuseMaxSum = 8, kFuseSmallRank = 10;
      std::vector<int> tv_ok = tv;
      int n_absorbed = 0, n_fresh = 0;
      for (size_t oi = (size_t)pos[v] + 1; oi < order.size(); ++oi) {
        const int u = order[oi];
        if (done[u] || std::find(S.begin(), S.end(), u) != S.end()) continue;
        if ((int)(out.size() + S.size()) < kFuseMinSpan || (int)S.size() >= kFuseMaxSum) break;
        if (std::find(out.begin(), out.end(), u) == out.end()) break;
        std::vector<int> tu, fresh;
        bool ok = true;
        for (size_t i = 0; i < T.size() && ok; ++i) {
          if (!T[i].alive || std::find(tv.begin(), tv.end(), (int)i) != tv.end()) continue;
          if (std::find(T[i].vars.begin(), T[i].vars.end(), u) == T[i].vars.end()) continue;
          ok = T[i].is_const || T[i].leaf >= 0 || (int)T[i].vars.size() <= kFuseSmallRank;
          for (int w : T[i].vars)
            if (std::find(out.begin(), out.end(), w) == out.end() && std::find(S.begin(), S.end(), w) == S.end() &&
                std::find(fresh.begin(), fresh.end(), w) == fresh.end())
              fresh.push_back(w);
          tu.push_back((int)i);
        }
        ok = ok && n_fresh + (int)fresh.size() <= n_absorbed + 2;
        if (!ok) break;
        n_absorbed++;
        n_fresh += (int)fresh.size();
        tv.insert(tv.end(), tu.begin(), tu.end());
        split_vars();
        if (n_fresh <= n_absorbed) tv_ok = tv;
      }
      if (tv_ok.size() != tv.size()) {
        tv = tv_ok;
        split_vars();
      }
    }
    bool all_const = !gradient;
    for (int i : tv) all_const = all_const && T[i].is_const;
    if (combine_consts && !gradient && !all_const) {
      // Constant factors of the step (gate tables and constant
      // intermediates) are first multiplied into one constant tensor, summing
      // the variables that occur only in them, by a constant step that runs
      // once per call; the item step then multiplies by one constant operand
      // instead of several (the same product, grouped differently).
      std::vector<int> ct, rest_tv;
      for (int i : tv) (T[i].is_const && T[i].leaf < 0 ? ct : rest_tv).push_back(i);
      if (ct.size() >= 2) {
        std::vector<char> in_rest(nvars, 0), in_ct(nvars, 0);
        for (int i : rest_tv)
          for (int u : T[i].vars) in_rest[u] = 1;
        std::vector<int> c_out, c_sum;
        for (int i : ct)
          for (int u : T[i].vars) {
            if (in_ct[u]) continue;
            in_ct[u] = 1;
            const bool summed = std::find(S.begin(), S.end(), u) != S.end();
            (summed && !in_rest[u] ? c_sum : c_out).push_back(u);
          }
        if ((int)c_out.size() <= kMaxCombinedRank) {
          std::sort(c_out.begin(), c_out.end(), [&](int a, int b) { return pos[a] < pos[b]; });
          std::sort(c_sum.begin(), c_sum.end(), [&](int a, int b) { return pos[a] < pos[b]; });
          const int k = emit(ST_ELIM, ct, c_out, c_sum, true, -1, 0, 0);
          for (int i : ct) {
            for (int u : T[i].vars) count[u]--;
            T[i].alive = 0;
          }
          for (int u : c_out) count[u]++;
          for (int u : c_sum) done[u] = 1;
          std::vector<int> S2;
          for (int u : S)
            if (std::find(c_sum.begin(), c_sum.end(), u) == c_sum.end()) S2.push_back(u);
          S.swap(S2);
          rest_tv.push_back(k);
          tv.swap(rest_tv);
        }
      }
      // A small constant factor whose variables all belong to a large item
      // operand made by an earlier item step is multiplied in by that step
      // (one more operand of it, a scale of its output; the same product,
      // grouped differently): no pass over a large tensor is spent on it,
      // which the pairwise pre-contraction below would spend when it pairs
      // the factor with the other operand and adds a variable to it.
      if ((int)(out.size() + S.size()) >= 16 && tv.size() > 2) {
        for (size_t x = 0; x < tv.size();) {
          const Tn& C = T[tv[x]];
          int host = -1;
          if (C.is_const && C.leaf < 0 && (int)C.vars.size() <= 10)
            for (int y : tv) {
              const Tn& Y = T[y];
              if (y == tv[x] || Y.is_const || Y.leaf >= 0 || Y.producer < 0 || (int)Y.vars.size() < 16) continue;
              const Step& ps = prog.steps[Y.producer];
              if (ps.kind != ST_ELIM || ps.is_const || ps.out_tid != Y.id) continue;
              bool sub = true;
              for (int u : C.vars) sub = sub && std::find(Y.vars.begin(), Y.vars.end(), u) != Y.vars.end();
              if (!sub) continue;
              // one scale per step, and only on a product of two operands
              if (ps.opnd.size() != 2) continue;
              host = y;
              break;
            }
          if (host < 0) {
            ++x;
            continue;
          }
          Step& ps = prog.steps[T[host].producer];
          const double old_bytes = 8.0 * [&] {
            double e = std::ldexp(1.0, ps.r);
            for (const Operand& o : ps.opnd) e += std::ldexp(1.0, (int)o.vars.size());
            return e;
          }();
          const double old_t = std::max(ps.flops / 157.3e12, old_bytes / 8e12);
          const bool old_mc = matrix_core_shape(ps);
          ps.opnd.push_back(as_operand(C));
          ps.m = (int)ps.opnd.size();
          const double old_flops = ps.flops;
          ps.flops = step_flops(ps.r, ps.ns, 2, 1);  // the scale multiplies each sum once
          const double new_bytes = old_bytes + 8.0 * std::ldexp(1.0, (int)C.vars.size());
          prog.flops_item += ps.flops - old_flops;
          prog.bytes_item += new_bytes - old_bytes;
          prog.roof_s_item += std::max(ps.flops / 157.3e12, new_bytes / 8e12) - old_t;
          if (old_mc) prog.flops_mc_item -= old_flops;
          if (matrix_core_shape(ps)) prog.flops_mc_item += ps.flops;
          for (int u : C.vars) count[u]--;
          T[tv[x]].alive = 0;
          tv.erase(tv.begin() + x);
          split_vars();
        }
      }
      // Pairwise pre-contraction of a large step: while it has more than
      // two operands, the pair whose variables together span the fewest
      // (two or more fewer than the step) is multiplied first, summing the
      // variables only the two carry; each factor taken out this way costs
      // the size of the pair's span instead of the step's full span.
      const int full = (int)(out.size() + S.size());
      while (full >= 16 && tv.size() > 2) {
        int ba = -1, bb = -1, bspan = 1 << 30;
        for (size_t x = 0; x < tv.size(); ++x)
          for (size_t y = x + 1; y < tv.size(); ++y) {
            std::vector<int> un = T[tv[x]].vars;
            for (int w : T[tv[y]].vars)
              if (std::find(un.begin(), un.end(), w) == un.end()) un.push_back(w);
            if ((int)un.size() < bspan) {
              bspan = (int)un.size();
              ba = tv[x];
              bb = tv[y];
            }
          }
        if (bspan > full - 2) break;
        std::vector<int> p_out, p_sum;
        std::vector<int> un = T[ba].vars;
        for (int w : T[bb].vars)
          if (std::find(un.begin(), un.end(), w) == un.end()) un.push_back(w);
        for (int w : un) {
          const int c_in = (int)(std::find(T[ba].vars.begin(), T[ba].vars.end(), w) != T[ba].vars.end()) +
                           (int)(std::find(T[bb].vars.begin(), T[bb].vars.end(), w) != T[bb].vars.end());
          (c_in == count[w] && !is_open[w] ? p_sum : p_out).push_back(w);
        }
        std::sort(p_out.begin(), p_out.end(), [&](int x, int y) { return pos[x] < pos[y]; });
        std::sort(p_sum.begin(), p_sum.end(), [&](int x, int y) { return pos[x] < pos[y]; });
        const bool pc = T[ba].is_const && T[bb].is_const && T[ba].leaf < 0 && T[bb].leaf < 0;
        const int c = emit(ST_ELIM, {ba, bb}, p_out, p_sum, pc, -1, 0, 0);
        for (int i : {ba, bb}) {
          for (int w : T[i].vars) count[w]--;
          T[i].alive = 0;
        }
        for (int w : p_out) count[w]++;
        for (int w : p_sum) done[w] = 1;
        std::vector<int> tv2{c};
        for (int i : tv)
          if (i != ba && i != bb) tv2.push_back(i);
        tv.swap(tv2);
        split_vars();
      }
    }
    emit(ST_ELIM, tv, out, S, all_const, -1, 0, 0);
    for (int i : tv) {
      for (int u : T[i].vars) count[u]--;
      T[i].alive = 0;
    }
    for (int u : S) done[u] = 1;
    for (int u : out) count[u]++;
  }

  // ---- final product of the remaining scalars
  std::vector<int> rest;
  for (size_t i = 0; i < T.size(); ++i) {
    if (!T[i].alive) continue;
    bool only_open = true;
    for (int u : T[i].vars) only_open = only_open && is_open[u];
    if (!only_open) {
      err = "internal: variable left after elimination";
      code = -3;
      return false;
    }
    rest.push_back((int)i);
  }
  emit(ST_FINAL, rest, open_vars, {}, false, -1, two_tab, n_two);
  const std::vector<int> fwd_steps = elim_created;  // forward tensors, creation order

  // ---- reverse mode (gradient programs)
  if (gradient) {
    // Checkpointing: with checkpoint_every = n > 0 the forward elimination
    // outputs are cut into segments of n in creation order.  A forward
    // output stays in item memory for the reverse pass only when its
    // consumer lies in another segment (or it is an operand of the final
    // product): a checkpoint.  Any other forward value the reverse pass
    // needs is recomputed from checkpoints and values of its own segment,
    // once, by the same step as in the forward pass (same operands in the
    // same order, so the same values); its memory is free between its last
    // forward use and the reverse pass over its segment.  Every forward
    // tensor has one consumer, so the recomputation costs at most one more
    // forward pass.
    std::vector<int> fwd_pos(T.size(), -1), consumer_pos(T.size(), -1);
    for (size_t k = 0; k < fwd_steps.size(); ++k) fwd_pos[fwd_steps[k]] = (int)k;
    for (size_t k = 0; k < fwd_steps.size(); ++k)
      for (int x : T[fwd_steps[k]].inputs) consumer_pos[x] = (int)k;
    std::vector<char> in_rest(T.size(), 0);
    for (int t : rest) in_rest[t] = 1;
    auto kept = [&](int t) {
      if (checkpoint_every <= 0 || t >= (int)fwd_pos.size() || fwd_pos[t] < 0 || in_rest[t] || consumer_pos[t] < 0)
        return true;
      return fwd_pos[t] / checkpoint_every != consumer_pos[t] / checkpoint_every;
    };
    std::map<int, int> recomputed;
    std::function<int(int)> value = [&](int t) -> int {
      if (kept(t)) return t;
      auto it = recomputed.find(t);
      if (it != recomputed.end()) return it->second;
      const Step st = prog.steps[T[t].producer];
      std::vector<int> in;
      for (int x : T[t].inputs) in.push_back(value(x));
      const int id = emit_one(ST_ELIM, in, st.out_vars, st.sum_vars, false, -1, 0, 0);
      recomputed[t] = id;
      return id;
    };
    std::vector<int> adj(T.size(), -1);
    auto grad_out = [&](int t) {
      // d alpha / d theta contribution of RZ factor f: sum_u adj(u) * D_f(u)
      const int f = T[t].rz_factor;
      const int slot = prog.n_grad_slots++;
      prog.grad_param.push_back(net.factors[f].param);
      Tn d = make_leaf(f, deriv_off[f]);  // derivative table, same fixed bits as the gate
      T.push_back(d);
      const int di = (int)T.size() - 1;
      std::vector<int> sv = T[t].vars;
      emit(ST_GRAD, {adj[t], di}, {}, sv, false, slot, 0, 0);
    };
    // adjoints of the FINAL operands
    for (size_t a = 0; a < rest.size(); ++a) {
      int t = rest[a];
      if (!T[t].grad) continue;
      std::vector<int> others;
      for (size_t b = 0; b < rest.size(); ++b)
        if (b != a) others.push_back(rest[b]);
      adj[t] = emit(ST_ELIM, others, {}, {}, false, -1, others.empty() ? one_tab : two_tab,
                    others.empty() ? 1 : n_two);
      if (adj.size() < T.size()) adj.resize(T.size(), -1);
    }
    // reverse over the forward eliminations
    for (int k = (int)fwd_steps.size() - 1; k >= 0; --k) {
      const int o = fwd_steps[k];
      if (o < 0 || adj[o] < 0) continue;
      const Step st = prog.steps[T[o].producer];
      std::vector<int> full = st.out_vars;
      full.insert(full.end(), st.sum_vars.begin(), st.sum_vars.end());
      const std::vector<int> ins = T[o].inputs;
      for (size_t a = 0; a < ins.size(); ++a) {
        int t = ins[a];
        if (!T[t].grad) continue;
        std::vector<int> ops{adj[o]};
        for (size_t b = 0; b < ins.size(); ++b)
          if (b != a) ops.push_back(value(ins[b]));
        std::vector<int> sum;
        for (int u : full)
          if (std::find(T[t].vars.begin(), T[t].vars.end(), u) == T[t].vars.end()) sum.push_back(u);
        int id = emit(ST_ELIM, ops, T[t].vars, sum, false, -1, 0, 0);
        if (adj.size() < T.size()) adj.resize(T.size(), -1);
        adj[t] = id;
      }
    }
    for (size_t t = 0; t < T.size(); ++t)
      if (T[t].rz_factor >= 0 && t < adj.size() && adj[t] >= 0) grad_out((int)t);
  }

  // ---- place item memory, then patch operand and output offsets
  prog.n_const = const_top;
  prog.item_elems = std::max(1, pack_buffers(bufs));
  for (size_t i = 0; i < prog.steps.size(); ++i) {
    Step& st = prog.steps[i];
    if (step_buf[i] >= 0) st.out = bufs[step_buf[i]].offset;
    for (Operand& o : st.opnd)
      if (!o.is_const) o.storage = bufs[o.storage].offset;
  }
  // constant steps first; they read constants only, so their order among
  // themselves and the item steps' order are unchanged
  std::stable_partition(prog.steps.begin(), prog.steps.end(), [](const Step& s) { return s.is_const; });

  // ---- check: replay the item steps on an ownership map of item memory;
  // every operand must find its own tensor in place when it is read
  {
    std::vector<int> owner((size_t)prog.item_elems, -1);
    for (size_t i = 0; i < prog.steps.size(); ++i) {
      const Step& st = prog.steps[i];
      if (st.is_const) continue;
      for (const Operand& o : st.opnd) {
        if (o.is_const) continue;
        const int n = 1 << o.vars.size();
        for (int e = 0; e < n; ++e)
          if (o.storage + e >= prog.item_elems || owner[o.storage + e] != o.tid) {
            err = "internal: item memory check failed at step " + std::to_string(i);
            code = -1;
            return false;
          }
      }
      if (st.kind == ST_LEAF || st.kind == ST_ELIM) {
        const int n = 1 << st.r;
        if (st.out + n > prog.item_elems) {
          err = "internal: item memory overflow at step " + std::to_string(i);
          code = -1;
          return false;
        }
        for (int e = 0; e < n; ++e) owner[st.out + e] = st.out_tid;
      }
    }
  }

  // ---- per-element operand table for the small-rank engines
  constexpr int kMaxStepBits = 16;
  constexpr size_t kMaxOptab = (size_t)1 << 26;
  size_t need = 0;
  bool fits = true;
  for (const Step& st : prog.steps) {
    if (st.kind == ST_LEAF) continue;
    if (st.r + st.ns > kMaxStepBits) fits = false;
    else need += (size_t)st.m << (st.r + st.ns);
  }
  fits = fits && need <= kMaxOptab;
  if (fits) {
    prog.optab.reserve(need);
    std::vector<int> bitpos(nvars, -1), from_s(nvars, 0);
    for (Step& st : prog.steps) {
      if (st.kind == ST_LEAF) continue;
      st.ops = (int)prog.optab.size();
      for (int j = 0; j < st.r; ++j) {
        bitpos[st.out_vars[j]] = j;
        from_s[st.out_vars[j]] = 0;
      }
      for (int j = 0; j < st.ns; ++j) {
        bitpos[st.sum_vars[j]] = j;
        from_s[st.sum_vars[j]] = 1;
      }
      for (int c = 0; c < (1 << st.r); ++c)
        for (int s2 = 0; s2 < (1 << st.ns); ++s2)
          for (const Operand& o : st.opnd) {
            int off = 0;
            for (size_t j = 0; j < o.vars.size(); ++j) {
              int u = o.vars[j];
              int val = from_s[u] ? (s2 >> bitpos[u]) & 1 : (c >> bitpos[u]) & 1;
              off |= val << j;
            }
            prog.optab.push_back((o.is_const ? OP_CONST : 0u) | (uint32_t)(o.storage + off));
          }
    }
    prog.has_optab = true;
  }
  (void)popc_bits;
  return true;
}

std::vector<int> group_bit_positions(const Program& prog, int k, double* shared_frac) {
  if (shared_frac) *shared_frac = 0.0;
  std::vector<int> pos_at;  // sliced positions chosen for bits 6, 7, ...
  if (k <= 6) return pos_at;
  // per item step: roofline time (as Program::roof_s_item) and the sliced
  // positions it depends on
  std::vector<std::pair<double, uint64_t>> work;
  double total = 0.0;
  for (const Step& st : prog.steps) {
    if (st.is_const || st.kind == ST_LEAF) continue;
    double elems = std::ldexp(1.0, st.r);
    for (const Operand& o : st.opnd) elems += std::ldexp(1.0, (int)o.vars.size());
    const double t = std::max(st.flops / 157.3e12, 8.0 * elems / 8e12);
    work.push_back({t, st.fix_mask});
    total += t;
  }
  uint64_t chosen = 0;
  for (int b = 6; b < k; ++b) {
    int best = -1;
    double best_w = -1.0;
    for (int j = 0; j < k; ++j) {
      if ((chosen >> j) & 1) continue;
      const uint64_t m = chosen | (1ull << j);
      double w = 0.0;
      for (auto& x : work)
        if ((x.second & m) == 0) w += x.first;
      if (w > best_w) {
        best_w = w;
        best = j;
      }
    }
    chosen |= 1ull << best;
    pos_at.push_back(best);
    if (b == std::min(k - 1, 7) && shared_frac && total > 0.0) *shared_frac = best_w / total;
  }
  return pos_at;
}

std::vector<int> sliced_order_for_groups(const Network& net, const std::vector<int>& sliced,
                                         const std::vector<int>& order, double* shared_frac) {
  if (shared_frac) *shared_frac = 0.0;
  const int k = (int)sliced.size();
  if (k <= 6) return sliced;
  Program prog;
  std::string err;
  int code = 0;
  if (!compile_program(net, sliced, order, prog, err, code, false, true)) return sliced;
  const std::vector<int> pos_at = group_bit_positions(prog, k, shared_frac);
  uint64_t chosen = 0;
  for (int j : pos_at) chosen |= 1ull << j;
  std::vector<int> out;
  for (int j = 0; j < k; ++j)
    if (!((chosen >> j) & 1)) out.push_back(sliced[j]);
  for (int j : pos_at) out.push_back(sliced[j]);
  return out;
}

}  // namespace qgm
