// extern "C" entry points declared in include/qgm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/qgm.h"
#include "exec.h"
#include "host.h"

using namespace qgm;

struct qgm_circuit {
  Network net;
};

struct qgm_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct qgm_plan {
  Network net;
  std::vector<int> sliced, order;
  Program prog;
  DevProgram dev;
  int engine = QGM_ENGINE_INTERPRETER;  // engine in use
  std::vector<char> code;                // generated kernel code object (engine GENERATED)
  WideProgram wide;                      // descriptors (engine WIDE)
  std::vector<char> wide_code;           // generated per-step kernels (engine WIDE)
  std::vector<WideKernel> wide_kernels;
  double compile_s = 0;
  qgm_plan_opts opts;
  double cost = 0;
  std::mutex mu;
  std::vector<std::array<hipEvent_t, 4>> runs;  // profiling events, one set per run
  std::vector<std::vector<hipEvent_t>> level_runs;  // WIDE profiling: events around each level launch
  std::vector<uint64_t> level_items;                 // items of the pass those events cover
  std::vector<uint64_t> level_vary;                  // that pass's group_vary_mask
  TileTable tiles;                                   // WIDE: matrix-core tile table (opts.tile_table_path)
  std::string tile_table_path;
  ~qgm_plan() {
    for (auto& r : runs)
      for (hipEvent_t e : r) (void)hipEventDestroy(e);
    for (auto& r : level_runs)
      for (hipEvent_t e : r) (void)hipEventDestroy(e);
  }
};

namespace {

thread_local std::string g_err;

qgm_status fail(qgm_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define GUARD_BEGIN try {
#define GUARD_END                                              \
  }                                                            \
  catch (const std::bad_alloc&) {                              \
    return fail(QGM_E_ARG, "out of host memory");              \
  }                                                            \
  catch (const std::exception& e) {                            \
    return fail(QGM_E_ARG, std::string("internal: ") + e.what()); \
  }                                                            \
  catch (...) {                                                \
    return fail(QGM_E_ARG, "internal error");                  \
  }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Staging {
  size_t bits, params, partial, gpartial, total;
};

Staging staging(const WsLayout& ws, int n_bs, int n_qubits, int n_params, bool grads, int n_open = 0) {
  Staging st;
  size_t off = ws.total;
  st.bits = off;
  off = align256(off + (size_t)std::max(1, n_bs) * std::max(1, n_qubits));
  st.params = off;
  off = align256(off + (size_t)std::max(1, n_params) * sizeof(double));
  st.partial = off;
  off = align256(off + ((size_t)std::max(1, n_bs) << n_open) * 4 * sizeof(double));
  st.gpartial = off;
  if (grads) off = align256(off + (size_t)std::max(1, n_bs) * std::max(1, n_params) * 4 * sizeof(double));
  st.total = off;
  return st;
}

qgm_status ensure_device(qgm_plan* p) {
  std::string err;
  int rc = dev_upload(p->prog, p->code, p->engine == QGM_ENGINE_WIDE ? &p->wide : nullptr, p->dev, err,
                      &p->wide_code, &p->wide_kernels);
  if (rc) return fail((qgm_status)rc, err);
  // constants of plans without angles: contracted once, here, not per run
  // (the generated kernels fold them at compile time)
  if (p->net.n_params == 0 && p->engine != QGM_ENGINE_GENERATED && !p->dev.cst_cached &&
      !std::getenv("QGM_NO_CONST_CACHE")) {
    rc = dev_cache_constants(p->prog, p->dev, p->opts.prec, p->engine == QGM_ENGINE_WIDE, err);
    if (rc) return fail((qgm_status)rc, err);
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->dev.device)
    return fail(QGM_E_ARG, "plan was uploaded to device " + std::to_string(p->dev.device) +
                               " but the current device is " + std::to_string(dev));
  return QGM_OK;
}

qgm_status layout_for(qgm_plan* p, int n_bs, uint64_t n_s, WsLayout& ws, LaunchCfg& cfg) {
  cfg.prec = p->opts.prec;
  cfg.generated = p->engine == QGM_ENGINE_GENERATED ? 1 : 0;
  cfg.wide = p->engine == QGM_ENGINE_WIDE ? 1 : 0;
  cfg.wide_budget = p->opts.workspace_cap ? p->opts.workspace_cap : ((size_t)96 << 30);
  cfg.n_qubits = p->net.n_qubits;
  cfg.n_bs = n_bs;
  cfg.s_begin = 0;
  cfg.n_s = n_s;
  cfg.n_params = p->net.n_params;
  std::string err;
  int rc = dev_layout(p->prog, p->dev, cfg, ws, err);
  if (rc) return fail((qgm_status)rc, err);
  return QGM_OK;
}

qgm_status check_range(const qgm_plan* p, uint64_t s_begin, uint64_t s_end) {
  const uint64_t ns = 1ull << p->sliced.size();
  if (s_begin > s_end || s_end > ns) return fail(QGM_E_ARG, "slice range outside [0, 2^k)");
  return QGM_OK;
}

qgm_status validate_plan_inputs(const Network& net, const int32_t* sliced, int32_t k, const int32_t* order,
                                int32_t n_order, std::vector<int>& sv, std::vector<int>& ov) {
  if (k < 0 || (k > 0 && !sliced)) return fail(QGM_E_SLICE, "bad sliced_vars / k");
  if (k > 40) return fail(QGM_E_SLICE, "at most 40 sliced variables");
  if (n_order < 0 || (n_order > 0 && !order)) return fail(QGM_E_ORDER, "bad order / n_order");
  sv.assign(sliced, sliced + k);
  ov.assign(order, order + n_order);
  (void)net;
  return QGM_OK;
}

}  // namespace

extern "C" {

const char* qgm_last_error(void) { return g_err.c_str(); }

qgm_status qgm_circuit_parse(const char* text, size_t len, qgm_circuit** out) {
  GUARD_BEGIN
  if (!out || (!text && len)) return fail(QGM_E_ARG, "null argument");
  *out = nullptr;
  auto* c = new qgm_circuit();
  std::string err;
  if (!parse_circuit(text ? text : "", len, c->net, err)) {
    delete c;
    return fail(QGM_E_PARSE, err);
  }
  build_network(c->net);
  *out = c;
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_circuit_info(const qgm_circuit* c, int32_t* n_qubits, int32_t* n_vars, int32_t* n_params) {
  if (!c) return fail(QGM_E_ARG, "null circuit");
  if (n_qubits) *n_qubits = c->net.n_qubits;
  if (n_vars) *n_vars = (int32_t)c->net.vars.size();
  if (n_params) *n_params = c->net.n_params;
  return QGM_OK;
}

qgm_status qgm_circuit_vars(const qgm_circuit* c, qgm_var_info* buf, int32_t cap) {
  if (!c || (cap > 0 && !buf) || cap < 0) return fail(QGM_E_ARG, "null argument");
  int n = std::min<int>(cap, (int)c->net.vars.size());
  for (int i = 0; i < n; ++i) {
    const Var& v = c->net.vars[i];
    buf[i] = qgm_var_info{v.id, v.qubit, v.cycle, v.is_output};
  }
  return QGM_OK;
}

qgm_status qgm_circuit_graph(const qgm_circuit* c, int32_t* edges, int32_t cap, int32_t* n_edges) {
  GUARD_BEGIN
  if (!c || cap < 0 || (cap > 0 && !edges) || !n_edges) return fail(QGM_E_ARG, "null argument");
  std::vector<int> vov;
  Graph g = model_graph(c->net, vov);
  int cnt = 0;
  for (int a = 0; a < g.n; ++a)
    for (int b = a + 1; b < g.n; ++b)
      if (g.has(a, b)) {
        if (cnt < cap) {
          edges[2 * cnt] = c->net.free_vars[a];
          edges[2 * cnt + 1] = c->net.free_vars[b];
        }
        ++cnt;
      }
  *n_edges = cnt;
  return QGM_OK;
  GUARD_END
}

void qgm_circuit_free(qgm_circuit* c) { delete c; }

qgm_status qgm_plan_slices(const qgm_circuit* c, int32_t k_req, int32_t target_rank, double time_budget_s,
                           uint64_t seed, int32_t* sliced_out, int32_t* k_out, int32_t* order_out,
                           int32_t* n_order_out) {
  return qgm_plan_slices_ex(c, k_req, target_rank, time_budget_s, seed, 0, sliced_out, k_out, order_out,
                            n_order_out);
}

qgm_status qgm_plan_slices_ex(const qgm_circuit* c, int32_t k_req, int32_t target_rank, double time_budget_s,
                              uint64_t seed, int32_t flags, int32_t* sliced_out, int32_t* k_out, int32_t* order_out,
                              int32_t* n_order_out) {
  GUARD_BEGIN
  if (!c || !sliced_out || !k_out || !order_out || !n_order_out) return fail(QGM_E_ARG, "null argument");
  if (k_req > 40) return fail(QGM_E_ARG, "k_req > 40");
  if (!(time_budget_s >= 0)) return fail(QGM_E_ARG, "negative time budget");
  std::vector<int> sl, ord;
  if (!plan_slices(c->net, k_req, target_rank, time_budget_s, seed, sl, ord, flags))
    return fail((flags & QGM_PLAN_CHOOSE_K) ? QGM_E_WORKSPACE : QGM_E_SLICE,
                "no plan found (QGM_PLAN_CHOOSE_K: no k fits a 64-item group in 96 GiB)");
  sl = sliced_order_for_groups(c->net, sl, ord);
  for (size_t i = 0; i < sl.size(); ++i) sliced_out[i] = sl[i];
  *k_out = (int32_t)sl.size();
  for (size_t i = 0; i < ord.size(); ++i) order_out[i] = ord[i];
  *n_order_out = (int32_t)ord.size();
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_sliced_order_for_groups(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k,
                                       const int32_t* order, int32_t n_order, int32_t* sliced_out,
                                       double* shared_frac) {
  GUARD_BEGIN
  if (!c || !sliced_out) return fail(QGM_E_ARG, "null argument");
  std::vector<int> sv, ov;
  qgm_status s = validate_plan_inputs(c->net, sliced_vars, k, order, n_order, sv, ov);
  if (s) return s;
  std::string err;
  int code = 0;
  if (!validate_plan(c->net, sv, ov, err, code)) return fail((qgm_status)code, err);
  double frac = 0.0;
  const std::vector<int> out = sliced_order_for_groups(c->net, sv, ov, &frac);
  for (size_t i = 0; i < out.size(); ++i) sliced_out[i] = out[i];
  if (shared_frac) *shared_frac = frac;
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_order_cost(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k, const int32_t* order,
                          int32_t n_order, double* cost, int32_t* width) {
  GUARD_BEGIN
  if (!c || !cost || !width) return fail(QGM_E_ARG, "null argument");
  std::vector<int> sv, ov;
  qgm_status s = validate_plan_inputs(c->net, sliced_vars, k, order, n_order, sv, ov);
  if (s) return s;
  std::string err;
  int code = 0;
  if (!validate_plan(c->net, sv, ov, err, code)) return fail((qgm_status)code, err);
  std::vector<int> vov;
  Graph g = model_graph(c->net, vov);
  std::vector<char> removed(g.n, 0);
  for (int v : sv) removed[vov[v]] = 1;
  std::vector<int> o;
  for (int v : ov) o.push_back(vov[v]);
  OrderCost oc = order_cost(g, o, removed);
  *cost = oc.cost;
  *width = oc.width;
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_order_search(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k, const int32_t* init_order,
                            int32_t n_order, int64_t max_nodes, int32_t beam, int32_t* order_out, double* cost,
                            int32_t* width, int32_t* complete) {
  GUARD_BEGIN
  if (!c || !order_out || !cost || !width || !complete || max_nodes < 1) return fail(QGM_E_ARG, "bad argument");
  std::vector<int> sv, ov;
  qgm_status s = validate_plan_inputs(c->net, sliced_vars, k, init_order, n_order, sv, ov);
  if (s) return s;
  std::string err;
  int code = 0;
  if (!validate_plan(c->net, sv, ov, err, code)) return fail((qgm_status)code, err);
  std::vector<int> vov;
  Graph g = model_graph(c->net, vov);
  std::vector<char> removed(g.n, 0);
  for (int v : sv) removed[vov[v]] = 1;
  std::vector<int> o;
  for (int v : ov) o.push_back(vov[v]);
  BnbResult r = bnb_order(g, removed, o, (long)max_nodes, beam);
  for (size_t i = 0; i < r.order.size(); ++i) order_out[i] = c->net.free_vars[r.order[i]];
  *cost = r.cost.cost;
  *width = r.cost.width;
  *complete = r.complete ? 1 : 0;
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_plan_create(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k, const int32_t* order,
                           int32_t n_order, const qgm_plan_opts* opts, qgm_plan** out) {
  GUARD_BEGIN
  if (!c || !out) return fail(QGM_E_ARG, "null argument");
  *out = nullptr;
  std::vector<int> sv, ov;
  qgm_status s = validate_plan_inputs(c->net, sliced_vars, k, order, n_order, sv, ov);
  if (s) return s;
  qgm_plan_opts o{};
  o.prec = QGM_C128;
  if (opts) o = *opts;
  if (o.prec != QGM_C128 && o.prec != QGM_C64 && o.prec != QGM_BF16X3)
    return fail(QGM_E_UNSUPPORTED, "unknown precision");
  if (o.engine < QGM_ENGINE_AUTO || o.engine > QGM_ENGINE_WIDE) return fail(QGM_E_ARG, "unknown engine");
  if (o.waves != 0 && o.waves != 1 && o.waves != 2 && o.waves != 4 && o.waves != 8)
    return fail(QGM_E_ARG, "waves must be 0, 1, 2, 4 or 8");
  if (o.vector_only != 0 && o.vector_only != 1) return fail(QGM_E_ARG, "vector_only must be 0 or 1");
  if (o.persistent != 0 && o.persistent != 1) return fail(QGM_E_ARG, "persistent must be 0 or 1");
  if (o.deterministic != 0 && o.deterministic != 1) return fail(QGM_E_ARG, "deterministic must be 0 or 1");
  if (o.n_open < 0 || o.n_open > 10 || (o.n_open > 0 && !o.open_qubits))
    return fail(QGM_E_ARG, "n_open must be 0..10 with open_qubits given");
  std::vector<int> open_q(o.open_qubits, o.open_qubits + o.n_open);
  o.open_qubits = nullptr;  // the caller's array is not kept
  if (o.checkpoint_every < 0) return fail(QGM_E_ARG, "checkpoint_every must be >= 0");
  if (o.checkpoint_every > 0 && !o.gradient) return fail(QGM_E_ARG, "checkpoint_every needs a gradient plan");
  TileTable tiles;
  std::string tile_path;
  if (o.tile_table_path) {
    tile_path = o.tile_table_path;
    std::string terr;
    if (!read_tile_table(tile_path, tiles, terr)) return fail(QGM_E_ARG, terr);
    o.tile_table_path = nullptr;  // the caller's string is not kept
  }
  auto* p = new qgm_plan();
  p->net = c->net;
  p->sliced = sv;
  p->order = ov;
  p->opts = o;
  p->tiles = std::move(tiles);
  p->tile_table_path = tile_path;
  std::string err;
  int code = 0;
  if (!compile_program(p->net, sv, ov, p->prog, err, code, o.gradient != 0, false, o.checkpoint_every, open_q)) {
    delete p;
    return fail((qgm_status)code, err);
  }
  if (!p->prog.has_optab && (o.engine == QGM_ENGINE_INTERPRETER || o.engine == QGM_ENGINE_GENERATED)) {
    delete p;
    return fail(QGM_E_UNSUPPORTED, "plan has a step of rank + summed variables > 16: only the WIDE engine runs it");
  }
  std::vector<int> vov;
  Graph g = model_graph(p->net, vov);
  std::vector<char> removed(g.n, 0);
  for (int v : sv) removed[vov[v]] = 1;
  std::vector<int> og;
  for (int v : ov) og.push_back(vov[v]);
  p->cost = order_cost(g, og, removed).cost;
  // Engine: the generated kernel keeps item tensors in registers, so it is
  // chosen automatically only when the live item memory is small; plans
  // with large steps run on the wide engine.
  const int reg_limit = o.prec == QGM_C128 ? 320 : 512;
  bool want_gen = o.engine == QGM_ENGINE_GENERATED ||
                  (o.engine == QGM_ENGINE_AUTO && p->prog.has_optab && p->prog.item_elems <= reg_limit);
  bool want_wide = o.engine == QGM_ENGINE_WIDE || (o.engine == QGM_ENGINE_AUTO && !p->prog.has_optab);
  p->engine = QGM_ENGINE_INTERPRETER;
  if (want_wide && !o.gradient) {
    // the wide engine loads constants from memory: their factors are
    // combined per step first (a different grouping of the same products)
    Program combined;
    if (compile_program(p->net, sv, ov, combined, err, code, false, true, 0, open_q)) p->prog = std::move(combined);
  }
  // the cap applies to the program that runs (after the wide engine's
  // regrouping, which changes its item memory)
  if (o.workspace_cap) {
    const size_t el = o.prec == QGM_C128 ? 16 : 8;
    size_t need = (size_t)p->prog.item_elems * 64 * el + (size_t)p->prog.n_const * el;
    if (need > o.workspace_cap) {
      delete p;
      return fail(QGM_E_WORKSPACE, "plan needs " + std::to_string(need) + " bytes per wavefront, over the cap");
    }
  }
  if (const char* dir = std::getenv("QGM_DUMP_DIR")) {
    // debugging aid: the compiled step list, one step per line
    if (FILE* f = std::fopen((std::string(dir) + "/qgm_program_" + std::to_string((uintptr_t)p) + ".txt").c_str(), "w")) {
      for (size_t i = 0; i < p->prog.steps.size(); ++i) {
        const Step& st = p->prog.steps[i];
        std::fprintf(f, "%zu kind %d const %d r %d ns %d m %d out_tid %d fix %llx |", i, st.kind, st.is_const, st.r,
                     st.ns, st.m, st.out_tid, (unsigned long long)st.fix_mask);
        for (int v : st.out_vars) std::fprintf(f, " o%d", v);
        for (int v : st.sum_vars) std::fprintf(f, " s%d", v);
        for (const Operand& op : st.opnd) {
          std::fprintf(f, " | %s%d:", op.is_const ? "c" : "t", op.tid);
          for (int v : op.vars) std::fprintf(f, " %d", v);
        }
        std::fprintf(f, "\n");
      }
      std::fclose(f);
    }
  }
  if (want_wide) {
    std::string werr;
    if (!encode_wide(p->prog, p->wide, werr)) {
      delete p;
      return fail(QGM_E_UNSUPPORTED, werr);
    }
    p->engine = QGM_ENGINE_WIDE;
    want_gen = false;
    // per-step generated kernels; the prebuilt step kernel stays the fallback
    if (!std::getenv("QGM_WIDE_PREBUILT")) {
      auto t0 = std::chrono::steady_clock::now();
      std::string src = generate_wide_source(p->prog, p->wide, o.prec, p->wide_kernels, !o.vector_only,
                                             p->tiles.empty() ? nullptr : &p->tiles);
      if (const char* dir = std::getenv("QGM_DUMP_DIR")) {
        // debugging aid: keep the generated source
        if (FILE* f = std::fopen((std::string(dir) + "/qgm_wide_" + std::to_string((uintptr_t)p) + ".hip").c_str(), "w")) {
          std::fwrite(src.data(), 1, src.size(), f);
          std::fclose(f);
        }
      }
      std::string jerr;
      if (!jit_compile(src, "qgm_wide.hip", p->wide_code, jerr)) {
        p->wide_code.clear();
        p->wide_kernels.clear();
      }
      p->compile_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  }
  if (want_gen) {
    auto t0 = std::chrono::steady_clock::now();
    std::string src = generate_chain_source(p->prog, o.prec, p->net.n_qubits, &p->dev.chain_waves, o.waves,
                                            o.persistent != 0);
    p->dev.chain_persistent = o.persistent;
    std::string jerr;
    bool ok = jit_compile(src, "qgm_chain.hip", p->code, jerr);
    if (const char* dir = std::getenv("QGM_DUMP_DIR")) {
      // debugging aid: keep the generated source and code object
      std::string base = std::string(dir) + "/qgm_chain_" + std::to_string((uintptr_t)p);
      if (FILE* f = std::fopen((base + ".hip").c_str(), "w")) {
        std::fwrite(src.data(), 1, src.size(), f);
        std::fclose(f);
      }
      if (ok)
        if (FILE* f = std::fopen((base + ".co").c_str(), "wb")) {
          std::fwrite(p->code.data(), 1, p->code.size(), f);
          std::fclose(f);
        }
    }
    if (ok) {
      p->engine = QGM_ENGINE_GENERATED;
    } else if (o.engine == QGM_ENGINE_GENERATED) {
      delete p;
      return fail(QGM_E_UNSUPPORTED, "generated kernel did not compile: " + jerr);
    }
    p->compile_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  *out = p;
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_plan_stats(const qgm_plan* p, qgm_stats* out) {
  if (!p || !out) return fail(QGM_E_ARG, "null argument");
  qgm_stats s{};
  s.n_steps = (int32_t)p->prog.steps.size();
  s.n_const_steps = p->prog.n_const_steps;
  s.max_rank = p->prog.max_rank;
  s.item_elems = p->prog.item_elems;
  s.n_leaves = (int32_t)p->prog.leaves.size();
  s.k = (int32_t)p->sliced.size();
  s.flops_item = p->prog.flops_item;
  s.flops_const = p->prog.flops_const;
  s.bytes_item = p->prog.bytes_item;
  s.roof_s_item = p->prog.roof_s_item;
  s.n_open = p->prog.n_open;
  s.cost = p->cost;
  s.engine = p->engine;
  s.compile_s = p->compile_s;
  s.waves = p->dev.chain_waves;
  s.launches = 1;
  if (p->engine == QGM_ENGINE_WIDE) {
    int lv = 0, item_steps = 0;
    for (const WideKernel& k : p->wide_kernels) {
      lv += k.kind == 0;
      s.mfma_steps += k.mfma_steps;
      s.flops_mfma += k.mfma_flops;
    }
    for (int si = 0; si < p->wide.n_steps; ++si) item_steps += !p->wide.steps[8 * si + 7];
    s.launches = lv > 0 ? lv : item_steps;
  }
  *out = s;
  return QGM_OK;
}

qgm_status qgm_workspace_size(const qgm_plan* pc, int32_t n_bs, uint64_t n_slices, size_t* bytes) {
  GUARD_BEGIN
  auto* p = const_cast<qgm_plan*>(pc);
  if (!p || !bytes || n_bs < 0) return fail(QGM_E_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(p->mu);
  qgm_status s = ensure_device(p);
  if (s) return s;
  WsLayout ws;
  LaunchCfg cfg;
  if ((s = layout_for(p, n_bs, n_slices, ws, cfg))) return s;
  *bytes = staging(ws, n_bs, p->net.n_qubits, p->net.n_params, p->prog.n_grad_slots > 0, p->prog.n_open).total;
  return QGM_OK;
  GUARD_END
}

}  // extern "C"

namespace {

// Queue one run on `stream`; the caller holds p->mu.
// no_alloc: nothing is allocated on the device or registered with the
// runtime: the plan's tables must already be on the current device (they
// are uploaded by the first ordinary run or qgm_workspace_size) and no
// profiling events are recorded.
qgm_status enqueue_run(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs, const double* d_params, uint64_t s_begin,
                       uint64_t s_end, void* d_ws, size_t ws_bytes, void* stream, double* d_partial,
                       bool capturing = false, double* d_grad_partial = nullptr, bool no_alloc = false) {
  if (!p || n_bs < 0 || (n_bs > 0 && (!d_bits || !d_partial)) || !d_ws) return fail(QGM_E_ARG, "bad argument");
  if (p->net.n_params > 0 && !d_params) return fail(QGM_E_ARG, "circuit has RZ gates but params is NULL");
  qgm_status s = check_range(p, s_begin, s_end);
  if (s) return s;
  if (no_alloc) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(QGM_E_HIP, "hipGetDevice failed");
    if (!p->dev.steps || p->dev.device != dev)
      return fail(QGM_E_ARG, "plan tables are not on the current device yet (call qgm_workspace_size first)");
    capturing = true;  // no profiling events
  } else if ((s = ensure_device(p))) {
    return s;
  }
  WsLayout ws;
  LaunchCfg cfg;
  if ((s = layout_for(p, n_bs, s_end - s_begin, ws, cfg))) return s;
  if (ws_bytes < ws.total) return fail(QGM_E_WORKSPACE, "workspace holds " + std::to_string(ws_bytes) +
                                                             " bytes, run needs " + std::to_string(ws.total));
  cfg.s_begin = s_begin;
  if (n_bs == 0) return QGM_OK;
  std::string err;
  void* ev[4] = {nullptr, nullptr, nullptr, nullptr};
  const bool profile = p->opts.profile && !capturing;
  if (profile) {
    std::array<hipEvent_t, 4> r{};
    for (auto& e : r)
      if (hipEventCreate(&e) != hipSuccess) return fail(QGM_E_HIP, "hipEventCreate failed");
    p->runs.push_back(r);
    for (int i = 0; i < 4; ++i) ev[i] = r[i];
    if (p->engine == QGM_ENGINE_WIDE && !p->dev.wide.levels.empty()) {
      std::vector<hipEvent_t> le(p->dev.wide.levels.size() + 1);
      for (auto& e : le)
        if (hipEventCreate(&e) != hipSuccess) return fail(QGM_E_HIP, "hipEventCreate failed");
      p->level_runs.push_back(le);
      p->level_items.push_back(std::min<uint64_t>((uint64_t)n_bs * (s_end - s_begin), (uint64_t)ws.wide_groups * 64));
      p->level_vary.push_back(group_vary_mask(0, (int)((p->level_items.back() + 63) / 64), s_begin, s_end - s_begin));
      p->dev.wide.level_events = (void* const*)p->level_runs.back().data();
    }
  }
  int rc = dev_run(p->prog, p->dev, cfg, ws, d_bits, d_params, d_ws, stream, d_partial, d_grad_partial,
                   profile ? ev : nullptr, err);
  p->dev.wide.level_events = nullptr;
  if (rc) return fail((qgm_status)rc, err);
  return QGM_OK;
}

}  // namespace

namespace qgm {
// The run of qgm_amplitudes_device on a workspace the allocation-free entry
// point supplies (its fixed device array); see enqueue_run's no_alloc.
qgm_status run_on_fixed_workspace(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs, const double* d_params,
                                  uint64_t s_begin, uint64_t s_end, void* d_ws, size_t ws_bytes, void* stream,
                                  double* d_partial) {
  GUARD_BEGIN
  if (!p) return fail(QGM_E_ARG, "null plan");
  std::lock_guard<std::mutex> lk(p->mu);
  return enqueue_run(p, d_bits, n_bs, d_params, s_begin, s_end, d_ws, ws_bytes, stream, d_partial, false, nullptr,
                     true);
  GUARD_END
}
qgm_status fail_status(qgm_status s, const char* msg) { return fail(s, msg); }
}  // namespace qgm

extern "C" {

qgm_status qgm_amplitudes_device(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs, const double* d_params,
                                 uint64_t s_begin, uint64_t s_end, void* d_ws, size_t ws_bytes, void* stream,
                                 double* d_partial) {
  GUARD_BEGIN
  if (!p) return fail(QGM_E_ARG, "null plan");
  std::lock_guard<std::mutex> lk(p->mu);
  return enqueue_run(p, d_bits, n_bs, d_params, s_begin, s_end, d_ws, ws_bytes, stream, d_partial);
  GUARD_END
}

qgm_status qgm_graph_create(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs, const double* d_params,
                            uint64_t s_begin, uint64_t s_end, void* d_ws, size_t ws_bytes, double* d_partial,
                            int32_t repeat, qgm_graph** out) {
  GUARD_BEGIN
  if (!p || !out || repeat < 1) return fail(QGM_E_ARG, "bad argument");
  *out = nullptr;
  std::lock_guard<std::mutex> lk(p->mu);
  qgm_status s = ensure_device(p);
  if (s) return s;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return fail(QGM_E_HIP, "hipStreamCreateWithFlags failed");
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(QGM_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  for (int r = 0; r < repeat && !s; ++r)
    s = enqueue_run(p, d_bits, n_bs, d_params, s_begin, s_end, d_ws, ws_bytes, cs, d_partial, true);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (s) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(QGM_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  auto* g = new qgm_graph();
  g->graph = graph;
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return fail(QGM_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  *out = g;
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_graph_launch(qgm_graph* g, void* stream) {
  if (!g) return fail(QGM_E_ARG, "null graph");
  hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(QGM_E_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return QGM_OK;
}

void qgm_graph_free(qgm_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

qgm_status qgm_amplitudes_range(qgm_plan* p, const uint8_t* bits, int32_t n_bs, const double* params,
                                uint64_t s_begin, uint64_t s_end, void* d_ws, size_t ws_bytes, void* stream_,
                                double* partial) {
  GUARD_BEGIN
  if (!p || n_bs < 0 || (n_bs > 0 && (!bits || !partial)) || !d_ws) return fail(QGM_E_ARG, "bad argument");
  const int nq = p->net.n_qubits;
  for (size_t i = 0; i < (size_t)n_bs * nq; ++i)
    if (bits[i] > 1) return fail(QGM_E_ARG, "bitstring entries must be 0 or 1");
  if (p->net.n_params > 0 && !params) return fail(QGM_E_ARG, "circuit has RZ gates but params is NULL");
  qgm_status s = check_range(p, s_begin, s_end);
  if (s) return s;
  hipStream_t stream = (hipStream_t)stream_;
  WsLayout ws;
  LaunchCfg cfg;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if ((s = ensure_device(p))) return s;
    if ((s = layout_for(p, n_bs, s_end - s_begin, ws, cfg))) return s;
  }
  Staging st = staging(ws, n_bs, nq, p->net.n_params, p->prog.n_grad_slots > 0, p->prog.n_open);
  if (ws_bytes < st.total) return fail(QGM_E_WORKSPACE, "workspace holds " + std::to_string(ws_bytes) +
                                                             " bytes, run needs " + std::to_string(st.total));
  char* base = (char*)d_ws;
  if (n_bs == 0) return QGM_OK;
  if (hipMemcpyAsync(base + st.bits, bits, (size_t)n_bs * nq, hipMemcpyHostToDevice, stream) != hipSuccess)
    return fail(QGM_E_HIP, "bitstring upload failed");
  if (p->net.n_params > 0 &&
      hipMemcpyAsync(base + st.params, params, (size_t)p->net.n_params * sizeof(double), hipMemcpyHostToDevice,
                     stream) != hipSuccess)
    return fail(QGM_E_HIP, "parameter upload failed");
  s = qgm_amplitudes_device(p, (const uint8_t*)(base + st.bits), n_bs,
                            p->net.n_params > 0 ? (const double*)(base + st.params) : nullptr, s_begin, s_end, d_ws,
                            ws.total, stream, (double*)(base + st.partial));
  if (s) return s;
  if (hipMemcpyAsync(partial, base + st.partial, ((size_t)n_bs << p->prog.n_open) * 4 * sizeof(double),
                     hipMemcpyDeviceToHost, stream) != hipSuccess)
    return fail(QGM_E_HIP, "result download failed");
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(QGM_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_amplitudes(qgm_plan* p, const uint8_t* bits, int32_t n_bs, const double* params, void* d_ws,
                          size_t ws_bytes, void* stream, double* out) {
  GUARD_BEGIN
  if (!p || n_bs < 0 || (n_bs > 0 && !out)) return fail(QGM_E_ARG, "bad argument");
  std::vector<double> part(((size_t)std::max(1, n_bs) << p->prog.n_open) * 4);
  qgm_status s = qgm_amplitudes_range(p, bits, n_bs, params, 0, 1ull << p->sliced.size(), d_ws, ws_bytes, stream,
                                      part.data());
  if (s) return s;
  for (int b = 0; b < (n_bs << p->prog.n_open); ++b) {
    out[2 * b] = part[4 * b] + part[4 * b + 2];
    out[2 * b + 1] = part[4 * b + 1] + part[4 * b + 3];
  }
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_plan_timing(qgm_plan* p, int32_t reset, double ms[3], int32_t* n_runs) {
  GUARD_BEGIN
  if (!p || !ms || !n_runs) return fail(QGM_E_ARG, "null argument");
  if (!p->opts.profile) return fail(QGM_E_ARG, "plan was not created with opts.profile = 1");
  std::lock_guard<std::mutex> lk(p->mu);
  double acc[3] = {0, 0, 0};
  for (auto& r : p->runs) {
    if (hipEventSynchronize(r[3]) != hipSuccess) return fail(QGM_E_HIP, "hipEventSynchronize failed");
    for (int i = 0; i < 3; ++i) {
      float t = 0;
      if (hipEventElapsedTime(&t, r[i], r[i + 1]) != hipSuccess) return fail(QGM_E_HIP, "hipEventElapsedTime failed");
      acc[i] += t;
    }
  }
  const int n = (int)p->runs.size();
  for (int i = 0; i < 3; ++i) ms[i] = n ? acc[i] / n : 0.0;
  *n_runs = n;
  if (reset) {
    for (auto& r : p->runs)
      for (hipEvent_t e : r) (void)hipEventDestroy(e);
    p->runs.clear();
    for (auto& r : p->level_runs)
      for (hipEvent_t e : r) (void)hipEventDestroy(e);
    p->level_runs.clear();
    p->level_items.clear();
    p->level_vary.clear();
  }
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_plan_level_timing(qgm_plan* p, int32_t reset, double* ms, double* flops_item, double* bytes_item,
                                 int32_t* mfma_steps, int32_t cap, int32_t* n_levels, int32_t* n_runs,
                                 uint64_t* items, double* roof_s_item) {
  GUARD_BEGIN
  if (!p || !n_levels || !n_runs || !items || cap < 0 ||
      (cap > 0 && (!ms || !flops_item || !bytes_item || !mfma_steps)))
    return fail(QGM_E_ARG, "bad argument");
  if (!p->opts.profile) return fail(QGM_E_ARG, "plan was not created with opts.profile = 1");
  std::lock_guard<std::mutex> lk(p->mu);
  std::vector<const WideKernel*> lv;
  for (const WideKernel& k : p->wide_kernels)
    if (k.kind == 0) lv.push_back(&k);
  *n_levels = (int32_t)lv.size();
  *n_runs = (int32_t)p->level_runs.size();
  *items = p->level_items.empty() ? 0 : p->level_items.back();
  // work of the timed pass: a step shared between its G groups is done for
  // one group, 1 / G of it per item of the pass
  const uint64_t vary = p->level_vary.empty() ? ~0ull : p->level_vary.back();
  const double G = (double)std::max<uint64_t>(1, (*items + 63) / 64);
  std::vector<double> eff_f(lv.size(), 0.0), eff_b(lv.size(), 0.0);
  double roof = 0.0;
  for (size_t i = 0; i < lv.size(); ++i)
    for (size_t j = 0; j < lv[i]->step_flops.size(); ++j) {
      const double w = (lv[i]->step_fix[j] & vary) == 0 ? 1.0 / G : 1.0;
      eff_f[i] += w * lv[i]->step_flops[j];
      eff_b[i] += w * lv[i]->step_bytes[j];
      roof += w * std::max(lv[i]->step_flops[j] / 157.3e12, lv[i]->step_bytes[j] / 8e12);
    }
  if (roof_s_item) *roof_s_item = roof;
  for (int i = 0; i < std::min<int>(cap, (int)lv.size()); ++i) {
    double acc = 0;
    for (auto& r : p->level_runs) {
      if (r.size() != lv.size() + 1) return fail(QGM_E_HIP, "level event count mismatch");
      if (hipEventSynchronize(r.back()) != hipSuccess) return fail(QGM_E_HIP, "hipEventSynchronize failed");
      float t = 0;
      if (hipEventElapsedTime(&t, r[i], r[i + 1]) != hipSuccess) return fail(QGM_E_HIP, "hipEventElapsedTime failed");
      acc += t;
    }
    ms[i] = p->level_runs.empty() ? 0.0 : acc / p->level_runs.size();
    flops_item[i] = eff_f[i];
    bytes_item[i] = eff_b[i];
    mfma_steps[i] = lv[i]->mfma_steps;
  }
  if (reset) {
    for (auto& r : p->level_runs)
      for (hipEvent_t e : r) (void)hipEventDestroy(e);
    p->level_runs.clear();
    p->level_items.clear();
    p->level_vary.clear();
  }
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_gradients_device(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs, const double* d_params,
                                uint64_t s_begin, uint64_t s_end, void* d_ws, size_t ws_bytes, void* stream,
                                double* d_partial, double* d_grad_partial) {
  GUARD_BEGIN
  if (!p) return fail(QGM_E_ARG, "null plan");
  if (p->prog.n_grad_slots == 0 && p->net.n_params > 0 && !p->opts.gradient)
    return fail(QGM_E_ARG, "plan was not created with opts.gradient = 1");
  if (n_bs > 0 && p->net.n_params > 0 && !d_grad_partial) return fail(QGM_E_ARG, "null gradient output");
  std::lock_guard<std::mutex> lk(p->mu);
  return enqueue_run(p, d_bits, n_bs, d_params, s_begin, s_end, d_ws, ws_bytes, stream, d_partial, false,
                     d_grad_partial);
  GUARD_END
}

qgm_status qgm_amplitude_grad(qgm_plan* p, const uint8_t* bitstring, const double* params, void* d_ws,
                              size_t ws_bytes, void* stream_, double* amp_out, double* dalpha) {
  GUARD_BEGIN
  if (!p || !bitstring || !amp_out || !d_ws) return fail(QGM_E_ARG, "bad argument");
  const int nq = p->net.n_qubits, np = p->net.n_params;
  if (np > 0 && (!params || !dalpha)) return fail(QGM_E_ARG, "params and dalpha_dtheta are required");
  if (!p->opts.gradient) return fail(QGM_E_ARG, "plan was not created with opts.gradient = 1");
  for (int q = 0; q < nq; ++q)
    if (bitstring[q] > 1) return fail(QGM_E_ARG, "bitstring entries must be 0 or 1");
  hipStream_t stream = (hipStream_t)stream_;
  WsLayout ws;
  LaunchCfg cfg;
  const uint64_t ns = 1ull << p->sliced.size();
  qgm_status s;
  {
    std::lock_guard<std::mutex> lk(p->mu);
    if ((s = ensure_device(p))) return s;
    if ((s = layout_for(p, 1, ns, ws, cfg))) return s;
  }
  Staging st = staging(ws, 1, nq, np, true);
  if (ws_bytes < st.total) return fail(QGM_E_WORKSPACE, "workspace holds " + std::to_string(ws_bytes) +
                                                             " bytes, run needs " + std::to_string(st.total));
  char* base = (char*)d_ws;
  if (hipMemcpyAsync(base + st.bits, bitstring, (size_t)nq, hipMemcpyHostToDevice, stream) != hipSuccess)
    return fail(QGM_E_HIP, "bitstring upload failed");
  if (np > 0 && hipMemcpyAsync(base + st.params, params, (size_t)np * sizeof(double), hipMemcpyHostToDevice,
                               stream) != hipSuccess)
    return fail(QGM_E_HIP, "parameter upload failed");
  s = qgm_gradients_device(p, (const uint8_t*)(base + st.bits), 1, np > 0 ? (const double*)(base + st.params) : nullptr,
                           0, ns, d_ws, ws.total, stream, (double*)(base + st.partial),
                           (double*)(base + st.gpartial));
  if (s) return s;
  std::vector<double> part(4), gpart((size_t)std::max(1, np) * 4);
  if (hipMemcpyAsync(part.data(), base + st.partial, 4 * sizeof(double), hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      (np > 0 && hipMemcpyAsync(gpart.data(), base + st.gpartial, (size_t)np * 4 * sizeof(double),
                                hipMemcpyDeviceToHost, stream) != hipSuccess))
    return fail(QGM_E_HIP, "result download failed");
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(QGM_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  amp_out[0] = part[0] + part[2];
  amp_out[1] = part[1] + part[3];
  for (int j = 0; j < np; ++j) {
    dalpha[2 * j] = gpart[4 * j] + gpart[4 * j + 2];
    dalpha[2 * j + 1] = gpart[4 * j + 1] + gpart[4 * j + 3];
  }
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_plan_autotune(qgm_plan* p, int32_t n_bs, uint64_t n_slices, void* d_ws, size_t ws_bytes,
                             void* stream_, int32_t* waves_out) {
  GUARD_BEGIN
  if (!p || !waves_out || n_bs < 1 || n_slices < 1 || !d_ws) return fail(QGM_E_ARG, "bad argument");
  *waves_out = 1;
  if (p->engine != QGM_ENGINE_GENERATED) return QGM_OK;
  if (n_slices > (1ull << p->sliced.size())) return fail(QGM_E_ARG, "more slices than the plan has");
  hipStream_t stream = (hipStream_t)stream_;
  std::lock_guard<std::mutex> lk(p->mu);
  qgm_status s = ensure_device(p);
  if (s) return s;
  WsLayout ws;
  LaunchCfg cfg;
  if ((s = layout_for(p, n_bs, n_slices, ws, cfg))) return s;
  Staging st = staging(ws, n_bs, p->net.n_qubits, p->net.n_params, p->prog.n_grad_slots > 0, p->prog.n_open);
  if (ws_bytes < st.total) return fail(QGM_E_WORKSPACE, "workspace smaller than qgm_workspace_size");
  char* base = (char*)d_ws;
  if (hipMemsetAsync(base + st.bits, 0, st.partial - st.bits, stream) != hipSuccess)
    return fail(QGM_E_HIP, "hipMemsetAsync failed");
  const uint8_t* d_bits = (const uint8_t*)(base + st.bits);
  const double* d_params = p->net.n_params > 0 ? (const double*)(base + st.params) : nullptr;
  double* d_part = (double*)(base + st.partial);
  double* d_gpart = p->prog.n_grad_slots > 0 ? (double*)(base + st.gpartial) : nullptr;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(QGM_E_HIP, "hipEventCreate failed");
  struct Variant {
    std::vector<char> code;
    hipModule_t mod = nullptr;
    hipFunction_t fn = nullptr;
    int waves = 1;
    float ms = 0;
  };
  // the current kernel is one candidate
  Variant best;
  best.code = p->code;
  best.mod = (hipModule_t)p->dev.module;
  best.fn = (hipFunction_t)p->dev.chain_fn;
  best.waves = p->dev.chain_waves;
  auto time_current = [&](float& ms) -> qgm_status {
    std::string err;
    for (int r = 0; r < 13; ++r) {
      if (r == 3 && hipEventRecord(e0, stream) != hipSuccess) return fail(QGM_E_HIP, "hipEventRecord failed");
      int rc = dev_run(p->prog, p->dev, cfg, ws, d_bits, d_params, d_ws, stream, d_part, d_gpart, nullptr, err);
      if (rc) return fail((qgm_status)rc, err);
    }
    if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return fail(QGM_E_HIP, "event timing failed");
    return QGM_OK;
  };
  if ((s = time_current(best.ms))) return s;
  for (int w : {1, 2, 4, 8}) {
    if (w == best.waves) continue;  // the current kernel
    int got = 0;
    std::string src = generate_chain_source(p->prog, p->opts.prec, p->net.n_qubits, &got, w, p->opts.persistent != 0);
    if (got != w) continue;  // no cut on w wavefronts fits for the plan
    Variant v;
    std::string jerr;
    if (!jit_compile(src, "qgm_chain.hip", v.code, jerr)) continue;
    if (hipModuleLoadData(&v.mod, v.code.data()) != hipSuccess) continue;
    if (hipModuleGetFunction(&v.fn, v.mod, "qgm_chain") != hipSuccess) {
      (void)hipModuleUnload(v.mod);
      continue;
    }
    v.waves = w;
    p->dev.module = v.mod;
    p->dev.chain_fn = v.fn;
    p->dev.chain_waves = w;
    s = time_current(v.ms);
    if (s || v.ms >= best.ms) {
      (void)hipModuleUnload(v.mod);
    } else {
      if (best.mod) (void)hipModuleUnload(best.mod);
      best = v;
    }
    p->dev.module = best.mod;
    p->dev.chain_fn = best.fn;
    p->dev.chain_waves = best.waves;
    if (s) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  p->code = best.code;
  *waves_out = best.waves;
  return s;
  GUARD_END
}

void qgm_plan_free(qgm_plan* p) {
  if (!p) return;
  dev_free(p->dev);
  delete p;
}

qgm_status qgm_amplitude(const char* text, size_t len, const uint8_t* bitstring, const int32_t* sliced, int32_t k,
                         const int32_t* order, int32_t n_order, const double* params, double out[2]) {
  GUARD_BEGIN
  if (!out) return fail(QGM_E_ARG, "null output");
  qgm_circuit* c = nullptr;
  qgm_status s = qgm_circuit_parse(text, len, &c);
  if (s) return s;
  qgm_plan* p = nullptr;
  s = qgm_plan_create(c, sliced, k, order, n_order, nullptr, &p);
  qgm_circuit_free(c);
  if (s) return s;
  size_t bytes = 0;
  s = qgm_workspace_size(p, 1, 1ull << k, &bytes);
  void* ws = nullptr;
  if (!s && hipMalloc(&ws, bytes) != hipSuccess) s = fail(QGM_E_HIP, "hipMalloc of workspace failed");
  if (!s) s = qgm_amplitudes(p, bitstring, 1, params, ws, bytes, nullptr, out);
  if (ws) (void)hipFree(ws);
  qgm_plan_free(p);
  return s;
  GUARD_END
}

}  // extern "C"

// ------------------------------------------------------------------------
// One two-operand contraction step on caller-laid-out item tensors.
struct qgm_contraction {
  int prec = 1, nb = 0, ni = 0, nj = 0, nk = 0;
  uint64_t ea = 0, eb = 0, ec = 0;  // elements per item of A, B, C
  WideKernel kern;
  std::vector<char> code;
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  int device = -1;
  std::mutex mu;
  ~qgm_contraction() {
    if (mod) (void)hipModuleUnload(mod);
  }
};

extern "C" {

qgm_status qgm_contraction_create(int32_t prec, int32_t nb, int32_t ni, int32_t nj, int32_t nk, int32_t flags,
                                  const qgm_tile* tile, qgm_contraction** out) {
  GUARD_BEGIN
  if (!out) return fail(QGM_E_ARG, "null argument");
  if (tile && (tile->per < 1 || tile->per > 16 || (tile->per & (tile->per - 1)) || tile->lds_budget < 1024 ||
               tile->lds_budget > 163840 || tile->jband < 0 || tile->jband > 8 || tile->layout < 0 || tile->layout > 63))
    return fail(QGM_E_ARG, "tile parameters out of range");
  *out = nullptr;
  if (prec != QGM_C128 && prec != QGM_C64 && prec != QGM_BF16X3) return fail(QGM_E_UNSUPPORTED, "unknown precision");
  if (nb < 0 || ni < 0 || nj < 0 || nk < 0 || nb + ni + nj > kWideMaxOut || nk > kWideMaxSum)
    return fail(QGM_E_ARG, "index counts out of range (b + i + j <= 32, k <= 16)");
  if (flags & ~1) return fail(QGM_E_ARG, "unknown flags");
  const uint64_t ea = 1ull << (nb + ni + nk), eb = 1ull << (nb + nk + nj), ec = 1ull << (nb + ni + nj);
  if (ea + eb + ec >= (1ull << 31)) return fail(QGM_E_ARG, "operands exceed 2^31 elements per item");
  if (ec >= (1ull << 40)) return fail(QGM_E_ARG, "output too large");
  auto* c = new qgm_contraction();
  c->prec = prec;
  c->nb = nb;
  c->ni = ni;
  c->nj = nj;
  c->nk = nk;
  c->ea = ea;
  c->eb = eb;
  c->ec = ec;
  // one elimination step: output bits i (0..ni-1), j, b; A = [b][k][i],
  // B = [b][j][k], C = [b][j][i] (first index slowest), item-major rows
  WideProgram w;
  const int r = ni + nj + nb;
  std::vector<int32_t> A(kWideOpInts, 0), B(kWideOpInts, 0);
  A[0] = B[0] = WOP_ITEM;
  A[1] = 0;
  B[1] = (int32_t)ea;
  for (int t = 0; t < ni; ++t) A[16 + t] = 1 << t;
  for (int t = 0; t < nj; ++t) B[16 + ni + t] = 1 << (nk + t);
  for (int t = 0; t < nb; ++t) {
    A[16 + ni + nj + t] = 1 << (ni + nk + t);
    B[16 + ni + nj + t] = 1 << (nk + nj + t);
  }
  for (int t = 0; t < nk; ++t) {
    A[48 + t] = 1 << (ni + t);
    B[48 + t] = 1 << t;
  }
  w.ops.insert(w.ops.end(), A.begin(), A.end());
  w.ops.insert(w.ops.end(), B.begin(), B.end());
  const int32_t srec[8] = {ST_ELIM, (int32_t)(ea + eb), r, nk, 2, -1, 0, 0};
  w.steps.assign(srec, srec + 8);
  w.n_steps = 1;
  std::vector<WideKernel> kernels;
  Program none;
  TileTable one;
  if (tile) one[TileKey{prec, ni, nj, nk}] = MfmaTile{tile->per, tile->lds_budget, tile->jband, tile->layout};
  const std::string src = generate_wide_source(none, w, prec, kernels, (flags & 1) == 0, tile ? &one : nullptr);
  if (const char* dir = std::getenv("QGM_DUMP_DIR")) {
    // debugging aid: keep the generated source
    if (FILE* f = std::fopen((std::string(dir) + "/qgm_contract_" + std::to_string((uintptr_t)c) + ".hip").c_str(), "w")) {
      std::fwrite(src.data(), 1, src.size(), f);
      std::fclose(f);
    }
  }
  std::string jerr;
  if (kernels.size() != 1 || !jit_compile(src, "qgm_contract.hip", c->code, jerr)) {
    delete c;
    return fail(QGM_E_UNSUPPORTED, "contraction kernel did not compile: " + jerr);
  }
  c->kern = kernels[0];
  if (c->kern.blocks == 0 || c->kern.blocks > 0x7fffffffull) {
    delete c;
    return fail(QGM_E_ARG, "contraction grid out of range");
  }
  *out = c;
  return QGM_OK;
  GUARD_END
}

qgm_status qgm_contraction_info(const qgm_contraction* c, int32_t* matrix_cores, uint64_t* elems_per_item,
                                double* flops_per_item) {
  if (!c) return fail(QGM_E_ARG, "null contraction");
  if (matrix_cores) *matrix_cores = c->kern.mfma_steps;
  if (elems_per_item) *elems_per_item = c->ea + c->eb + c->ec;
  if (flops_per_item) *flops_per_item = c->kern.flops;
  return QGM_OK;
}

qgm_status qgm_contraction_run(qgm_contraction* c, void* d_mem, int64_t n_groups, void* stream) {
  GUARD_BEGIN
  if (!c || !d_mem || n_groups < 0) return fail(QGM_E_ARG, "bad argument");
  if (n_groups > 65535) return fail(QGM_E_ARG, "at most 65535 groups of 64 items per call");
  if (n_groups == 0) return QGM_OK;
  std::lock_guard<std::mutex> lk(c->mu);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(QGM_E_HIP, "hipGetDevice failed");
  if (!c->mod) {
    hipError_t e = hipModuleLoadData(&c->mod, c->code.data());
    if (e == hipSuccess) e = hipModuleGetFunction(&c->fn, c->mod, c->kern.name.c_str());
    if (e != hipSuccess) return fail(QGM_E_HIP, std::string("loading the contraction kernel: ") + hipGetErrorString(e));
    c->device = dev;
  } else if (dev != c->device) {
    return fail(QGM_E_ARG, "contraction was loaded on device " + std::to_string(c->device));
  }
  // The level kernel's item bookkeeping: one bitstring (b = item >> 40 = 0)
  // whose packed bits are read from d_mem[0] and never used (no leaves);
  // no constants, results or gradient rows are touched by an item step.
  void* a_mem = d_mem;
  const void* a_cst = d_mem;
  const void* a_packed = d_mem;
  unsigned long long a_ge = c->ea + c->eb + c->ec, a_sb = 0, a_ns = 1ull << 40, a_ni = (unsigned long long)n_groups * 64,
                     a_nbs = 1;
  int a_g0 = 0, a_log2 = 40;
  void* a_res = d_mem;
  void* a_gres = d_mem;
  unsigned long long a_vary = ~0ull;  // one contraction step: nothing shared between groups
  void* args[] = {&a_mem, &a_cst, &a_packed, &a_ge, &a_sb, &a_ns, &a_g0, &a_log2, &a_ni, &a_nbs, &a_res, &a_gres,
                  &a_vary};
  hipError_t e = hipModuleLaunchKernel(c->fn, (unsigned)c->kern.blocks, (unsigned)n_groups, 1, (unsigned)c->kern.threads, 1, 1, 0,
                                       (hipStream_t)stream, args, nullptr);
  if (e != hipSuccess) return fail(QGM_E_HIP, std::string("contraction launch: ") + hipGetErrorString(e));
  return QGM_OK;
  GUARD_END
}

void qgm_contraction_free(qgm_contraction* c) { delete c; }

qgm_status qgm_plan_tune_tiles(qgm_plan* p, const char* table_path, void* stream_, int32_t* n_tuned) {
  GUARD_BEGIN
  if (!p || !table_path || !n_tuned) return fail(QGM_E_ARG, "null argument");
  *n_tuned = 0;
  if (p->engine != QGM_ENGINE_WIDE || (p->opts.prec != QGM_C64 && p->opts.prec != QGM_BF16X3) || p->opts.vector_only)
    return QGM_OK;  // no matrix-core steps
  hipStream_t stream = (hipStream_t)stream_;
  // the plan's matrix-core shapes by their flops per item, largest first
  std::map<TileKey, double> shape_flops;
  std::map<TileKey, int> shape_nb;
  for (int si = 0; si < p->wide.n_steps; ++si) {
    int nb = 0, ni = 0, nj = 0, nk = 0;
    if (!mfma_step_shape(p->wide, si, p->opts.prec, nb, ni, nj, nk)) continue;
    const TileKey key{p->opts.prec, ni, nj, nk};
    shape_flops[key] += std::ldexp(8.0, nb + ni + nj + nk);
    shape_nb[key] = std::max(shape_nb[key], nb);
  }
  std::vector<std::pair<double, TileKey>> order;
  double total = 0;
  for (auto& e : shape_flops) {
    order.push_back({-e.second, e.first});
    total += e.second;
  }
  std::sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  TileTable table;
  {
    std::string terr;
    FILE* f = std::fopen(table_path, "r");
    if (f) {
      std::fclose(f);
      if (!read_tile_table(table_path, table, terr)) return fail(QGM_E_ARG, terr);
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(QGM_E_HIP, "hipEventCreate failed");
  void* mem = nullptr;
  size_t mem_bytes = 0;
  qgm_status st = QGM_OK;
  double covered = 0;
  // Time one candidate on a batch that fills the GPU: nb batch bits chosen
  // so the step has at least 4096 blocks, at most 8 GiB of operands.
  auto time_tile = [&](const TileKey& key, int nb, const qgm_tile& t, float& ms) -> qgm_status {
    qgm_contraction* c = nullptr;
    qgm_status s2 = qgm_contraction_create(key.prec, nb, key.ni, key.nj, key.nk, 0, &t, &c);
    if (s2) return s2;
    const size_t need = (size_t)(c->ea + c->eb + c->ec) * 64 * 8;
    if (need > mem_bytes) {
      if (mem) (void)hipFree(mem);
      mem = nullptr;
      mem_bytes = 0;
      if (hipMalloc(&mem, need) != hipSuccess) {
        qgm_contraction_free(c);
        return fail(QGM_E_HIP, "hipMalloc of tuning operands failed");
      }
      mem_bytes = need;
      if (hipMemsetAsync(mem, 0x3c, need, stream) != hipSuccess) {
        qgm_contraction_free(c);
        return fail(QGM_E_HIP, "hipMemsetAsync failed");
      }
    }
    for (int r = 0; r < 7 && !s2; ++r) {
      if (r == 2 && hipEventRecord(e0, stream) != hipSuccess) s2 = fail(QGM_E_HIP, "hipEventRecord failed");
      if (!s2) s2 = qgm_contraction_run(c, mem, 1, stream);
    }
    if (!s2 && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      s2 = fail(QGM_E_HIP, "event timing failed");
    qgm_contraction_free(c);
    return s2;
  };
  for (auto& oe : order) {
    if (st || covered >= 0.99 * total) break;
    covered += -oe.first;
    const TileKey key = oe.second;
    const int nbi = key.ni >= 5 ? key.ni - 5 : 0, nbj = key.nj >= 5 ? key.nj - 5 : 0;
    int nb = std::max(0, 12 - nbi - nbj);
    while (nb > 0 && std::ldexp(64.0 * 8.0, nb) * (std::ldexp(1.0, key.ni + key.nk) + std::ldexp(1.0, key.nk + key.nj) +
                                                 std::ldexp(1.0, key.ni + key.nj)) > 8.0 * (1ull << 30))
      --nb;
    qgm_tile best{2, 53248, 2, 0};
    float best_ms = 0;
    bool have = false;
    if (key.prec == QGM_BF16X3 && key.nk >= 2) {
      // the per-item form: row / column tile (layouts 0, 4, 5, 6; + 8 for
      // eight items per block) x K steps per stage, and the 16-item forms (7
      // = built-in, 1 to 3); then the ring budget of the winner (the
      // per-item block order has no band)
      for (int layout : {0, 4, 5, 6, 8, 12, 13, 14})
        for (int per : {1, 2}) {
          if (st || 4 * per > (1 << key.nk)) continue;
          qgm_tile t{per, layout & 8 ? 131072 : 65536, 0, layout};
          float ms = 0;
          st = time_tile(key, nb, t, ms);
          if (!st && (!have || ms < best_ms)) best = t, best_ms = ms, have = true;
        }
      for (int layout : {7, 1, 2, 3}) {
        if (st) break;
        qgm_tile t{2, 53248, 2, layout};
        float ms = 0;
        st = time_tile(key, nb, t, ms);
        if (!st && ms < best_ms) best = t, best_ms = ms;
      }
      const bool per_item = (best.layout & 7) == 0 || ((best.layout & 7) >= 4 && (best.layout & 7) <= 6);
      const std::vector<int> budgets = !per_item ? std::vector<int>{81920, 114688}
                                       : best.layout & 8 ? std::vector<int>{65536, 98304, 163840}
                                                         : std::vector<int>{32768, 49152, 98304};
      for (int lds : budgets) {
        if (st) break;
        qgm_tile t{best.per, lds, per_item ? 0 : best.jband, best.layout};
        float ms = 0;
        st = time_tile(key, nb, t, ms);
        if (!st && ms < best_ms) best = t, best_ms = ms;
      }
    } else {
      // stage 1: block layout x k steps per stage; stage 2: ring budget x
      // band.  BF16x3 keeps two k per stage: more pairs per stage hold more
      // split operands live than two waves per SIMD have registers for,
      // which the level kernels of a plan (every step of a level in one
      // kernel) pay for even where a lone contraction does not
      std::vector<int> pers = key.prec == QGM_BF16X3 ? std::vector<int>{2} : std::vector<int>{1, 2, 4};
      for (int layout = 0; layout < 4 && !st; ++layout)
        for (int per : pers) {
          if (per > (1 << key.nk)) continue;
          qgm_tile t{per, 53248, 2, layout};
          float ms = 0;
          st = time_tile(key, nb, t, ms);
          if (st) break;
          if (!have || ms < best_ms) best = t, best_ms = ms, have = true;
        }
      // complex64 also tries its per-item form (FP32 16 x 16 x 4, layouts
      // 16 + the per-item variants, + 8 for eight items per block)
      if (key.prec == QGM_C64 && key.nk >= 2)
        for (int layout : {16, 20, 21, 22, 24, 28, 29, 30})
          for (int per : {1, 2}) {
            if (st || 4 * per > (1 << key.nk)) continue;
            qgm_tile t{per, layout & 8 ? 131072 : 65536, 0, layout};
            float ms = 0;
            st = time_tile(key, nb, t, ms);
            if (!st && ms < best_ms) best = t, best_ms = ms;
          }
      if (best.layout & 16) {
        for (int lds : best.layout & 8 ? std::vector<int>{65536, 98304, 163840} : std::vector<int>{32768, 49152, 98304}) {
          if (st) break;
          qgm_tile t{best.per, lds, 0, best.layout};
          float ms = 0;
          st = time_tile(key, nb, t, ms);
          if (!st && ms < best_ms) best = t, best_ms = ms;
        }
      } else {
        for (int lds : {53248, 81920, 114688})
          for (int jb = 0; jb <= 3 && !st; ++jb) {
            qgm_tile t{best.per, lds, jb, best.layout};
            if (lds == 53248 && jb == 2) continue;  // timed in stage 1
            float ms = 0;
            st = time_tile(key, nb, t, ms);
            if (!st && ms < best_ms) best = t, best_ms = ms;
          }
      }
    }
    if (st) break;
    table[key] = MfmaTile{best.per, best.lds_budget, best.jband, best.layout};
    ++*n_tuned;
  }
  if (mem) (void)hipFree(mem);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  std::string werr;
  if (!write_tile_table(table_path, table, werr)) return fail(QGM_E_ARG, werr);
  return QGM_OK;
  GUARD_END
}

}  // extern "C"
