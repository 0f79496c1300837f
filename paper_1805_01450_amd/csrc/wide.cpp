// Descriptors of the wide engine (large-rank plans).
//
// Operand record (kWideOpInts int32):
//   [0] kind (WOP_ITEM, WOP_CONST, WOP_LEAF)   [1] base element offset
//   [2] number of fixed-bit dependencies (leaves, at most 4)
//   [3..6] dependency source (0 = output bit, 1 = slice bit)
//   [7..10] dependency bit   [11..14] dependency stride in the table
//   [16 .. 16+32) stride per output bit of the step
//   [48 .. 48+16) stride per summed bit of the step
// Element offset of an operand at output index c and summed index s:
//   base + sum_j c_j * out_stride[j] + sum_j s_j * sum_stride[j] (+ deps).
#include <algorithm>
#include <map>

#include "host.h"

namespace qgm {

bool encode_wide(const Program& prog, WideProgram& wide, std::string& err) {
  wide = WideProgram();
  std::map<int, int> leaf_of_tid;  // tensor id of a materialised leaf -> leaf index
  for (const Step& st : prog.steps)
    if (st.kind == ST_LEAF) leaf_of_tid[st.out_tid] = st.leaf;
  for (const Step& st : prog.steps) {
    if (st.kind == ST_LEAF) continue;  // leaves are read in place
    if (st.r > kWideMaxOut || st.ns > kWideMaxSum) {
      err = "step of rank " + std::to_string(st.r) + " summing " + std::to_string(st.ns) + " is beyond the wide engine";
      return false;
    }
    const int op_begin = (int)(wide.ops.size() / kWideOpInts);
    for (const Operand& o : st.opnd) {
      std::vector<int32_t> rec(kWideOpInts, 0);
      std::vector<int> stride_of(o.vars.size());
      auto it = o.is_const ? leaf_of_tid.end() : leaf_of_tid.find(o.tid);
      if (it != leaf_of_tid.end()) {
        const Leaf& L = prog.leaves[it->second];
        rec[0] = WOP_LEAF;
        rec[1] = L.table;
        rec[2] = L.ndep;
        for (int j = 0; j < L.ndep; ++j) {
          rec[3 + j] = L.dep_src[j];
          rec[7 + j] = L.dep_bit[j];
          rec[11 + j] = L.dep_stride[j];
        }
        for (size_t j = 0; j < o.vars.size(); ++j) stride_of[j] = L.free_stride[j];
      } else {
        rec[0] = o.is_const ? WOP_CONST : WOP_ITEM;
        rec[1] = o.storage;
        for (size_t j = 0; j < o.vars.size(); ++j) stride_of[j] = 1 << j;
      }
      for (size_t j = 0; j < o.vars.size(); ++j) {
        const int u = o.vars[j];
        auto po = std::find(st.out_vars.begin(), st.out_vars.end(), u);
        if (po != st.out_vars.end()) {
          rec[16 + (po - st.out_vars.begin())] = stride_of[j];
          continue;
        }
        auto ps = std::find(st.sum_vars.begin(), st.sum_vars.end(), u);
        if (ps == st.sum_vars.end()) {
          err = "internal: operand variable " + std::to_string(u) + " of a step (kind " + std::to_string(st.kind) +
                ", rank " + std::to_string(st.r) + ", summed " + std::to_string(st.ns) + ", operands " +
                std::to_string(st.m) + ") neither kept nor summed";
          for (int v2 : st.out_vars) err += " o" + std::to_string(v2);
          for (int v2 : st.sum_vars) err += " s" + std::to_string(v2);
          for (const Operand& o2 : st.opnd) {
            err += " |";
            for (int v2 : o2.vars) err += " " + std::to_string(v2);
          }
          return false;
        }
        rec[48 + (ps - st.sum_vars.begin())] = stride_of[j];
      }
      wide.ops.insert(wide.ops.end(), rec.begin(), rec.end());
      wide.op_fix.push_back(o.fix_mask);
    }
    const int32_t srec[8] = {st.kind, st.out, st.r, st.ns, st.m, st.grad_slot, op_begin, st.is_const};
    wide.steps.insert(wide.steps.end(), srec, srec + 8);
    wide.step_fix.push_back(st.fix_mask);
    wide.n_steps++;
  }
  return true;
}

}  // namespace qgm
