// Host-side data structures of the qgm library: circuit, graphical model,
// planner and the compiled per-slice contraction program.
#pragma once
#include <cstddef>
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

namespace qgm {

enum GateKind { G_H = 0, G_SX, G_SY, G_T, G_RZ, G_I, G_CZ, G_CX, G_ISWAP, G_SQISW };

struct Gate {
  int cycle;
  GateKind kind;
  int q0, q1;
  int param;
  int line;
};

// One binary variable of the undirected graphical model: a distinct index
// value i_k^(j) of the Feynman sum, Eq. (1).
struct Var {
  int id, qubit, cycle, is_output;
};

// A factor over at most four variables (four: the gadget of a two-qubit
// gate that is not diagonal).  Table entry b = sum_j bit(var_j) << j.
// param >= 0 marks an RZ(theta_param) diagonal whose table is made on the
// device from the angle.
struct Factor {
  int nv;
  int var[4];
  int param;
  double tab[32];  // re, im pairs
};

struct Network {
  int n_qubits = 0, n_params = 0;
  std::vector<Gate> gates;
  std::vector<Var> vars;
  std::vector<Factor> factors;
  std::vector<int> output_var;  // per qubit; -1 = input constant
  std::vector<int> free_vars;   // non-output variables, ascending id
};

bool parse_circuit(const char* text, size_t len, Network& net, std::string& err);
void build_network(Network& net);

// ------------------------------------------------------------------ planner
struct Graph {
  int n = 0, words = 0;
  std::vector<uint64_t> adj;  // n rows of `words` words
  uint64_t* row(int v) { return adj.data() + (size_t)v * words; }
  const uint64_t* row(int v) const { return adj.data() + (size_t)v * words; }
  void init(int n_);
  void add_edge(int a, int b);
  bool has(int a, int b) const { return (row(a)[b >> 6] >> (b & 63)) & 1; }
};

// Graph over the free variables (vertex i = net.free_vars[i]); outputs fixed.
Graph model_graph(const Network& net, std::vector<int>& vertex_of_var);

struct OrderCost {
  double cost;  // sum over steps of 2^deg(v)
  int width;    // max deg(v)
};
OrderCost order_cost(const Graph& g, const std::vector<int>& order, const std::vector<char>& removed);
std::vector<int> min_fill_order(const Graph& g, const std::vector<char>& removed, uint64_t seed, int randomize);
// Branch and bound over elimination orderings of the graph without the
// removed vertices (QuickBB scheme): objective (width, sum 2^deg)
// lexicographic, incumbent `init`, at most max_nodes search nodes, beam
// children per node (<= 0: all; the search is then exact when complete).
struct BnbResult {
  std::vector<int> order;
  OrderCost cost;
  long nodes = 0;
  bool complete = false;
};
BnbResult bnb_order(const Graph& g, const std::vector<char>& removed, const std::vector<int>& init, long max_nodes,
                    int beam);
// flags bit 0: recompute the ordering after every removal (instead of
// keeping the first ordering throughout).
bool plan_slices(const Network& net, int k_req, int target_rank, double time_budget_s, uint64_t seed,
                 std::vector<int>& sliced_vars, std::vector<int>& order_vars, int flags = 0);

// ------------------------------------------------------------------ program
// Operand reference of a fused elimination step.
enum : uint32_t { OP_CONST = 0x80000000u };

struct Leaf {
  int factor;        // index into net.factors, or -1 for a delta(x_q, 0) leaf
  int nfree;         // free variables (0..4)
  int free_var[4];
  int free_stride[4];
  int ndep;          // fixed variables the table is indexed at (0..4)
  int dep_src[4];    // 0 = output bit (qubit), 1 = slice bit
  int dep_bit[4];
  int dep_stride[4];
  int table;         // element offset of the raw table in the constant area
};

// Step kinds of the per-item program.
//   ST_LEAF : materialise a leaf read at the item's fixed bits
//   ST_ELIM : out(out_vars) = sum over sum_vars of the product of the operands
//   ST_FINAL: the item's amplitude alpha_{x,s} (rank-0 product)
//   ST_GRAD : one RZ gate's contribution to d alpha_{x,s} / d theta (rank 0),
//             written to gradient slot `grad_slot`
enum StepKind { ST_LEAF = 0, ST_ELIM = 1, ST_FINAL = 2, ST_GRAD = 3 };

struct Operand {
  int is_const;           // 1: constant area (raw table or constant intermediate)
  int storage;            // element offset (constant area or packed item memory)
  std::vector<int> vars;  // bit j of the element index = value of vars[j]
  int tid = -1;           // compile-time tensor id (for the memory check)
  uint64_t fix_mask = 0;  // fixed variables its values depend on (as Step::fix_mask)
};

struct Step {
  int kind = ST_ELIM;
  int is_const = 0;   // runs once per call in the prologue (all operands constant)
  int out = 0;        // element offset: item memory or constant area
  int r = 0, ns = 0, m = 0;   // output rank, summed variables, operands
  int ops = -1;       // offset into the operand table (2^(r+ns) * m entries), -1 if not encoded
  int leaf = -1;      // ST_LEAF: leaf index
  int grad_slot = -1; // ST_GRAD: gradient slot
  std::vector<int> out_vars, sum_vars;
  std::vector<Operand> opnd;
  int out_tid = -1;   // compile-time tensor id of the output (item memory outputs)
  double flops = 0;   // useful real flops per item
  // fixed variables the output depends on: bit j = sliced variable j (bit j
  // of the slice index), bit 63 = the output bits; all bits set for steps
  // that write per-item results (FINAL, GRAD)
  uint64_t fix_mask = 0;
};

struct Program {
  std::vector<Leaf> leaves;
  std::vector<Step> steps;
  std::vector<uint32_t> optab;   // per-element operand table (small-rank engines)
  bool has_optab = false;
  std::vector<double> raw;       // raw factor tables, complex (re,im), const-area layout
  std::vector<int> raw_param;    // per raw complex entry: RZ parameter index or -1
  std::vector<int> raw_bit;      // per raw complex entry: 0/1 value of the RZ variable
  std::vector<int> raw_deriv;    // per raw entry: 1 = derivative table (i/2)(2u-1) e^{i theta (2u-1)/2}
  int n_raw = 0;                 // complex entries of raw tables
  int n_const = 0;               // total constant-area elements (raw + const intermediates)
  int item_elems = 0;            // peak item-memory elements per item
  int n_const_steps = 0;
  int max_rank = 0;
  int n_grad_slots = 0;          // gradient programs: one slot per RZ gate
  int n_open = 0;                // open outputs: the final step has rank n_open (2^n_open amplitudes per item)
  std::vector<int> grad_param;   // slot -> parameter index
  double flops_item = 0, flops_const = 0;
  double bytes_item = 0;         // algorithmic bytes per item at 8 B per element
  double flops_mc_item = 0;      // flops per item of steps with the matrix-core shape
  double roof_s_item = 0;        // sum over item steps of max(flops / 157.3 TFLOP/s, bytes / 8 TB/s)
};

bool validate_plan(const Network& net, const std::vector<int>& sliced, const std::vector<int>& order,
                   std::string& err, int& code);
// gradient = true appends the reverse-mode steps that give d alpha / d theta
// for every RZ gate (and disables constant hoisting).  encode = true builds
// the per-element operand table when every step is small enough (rank +
// summed variables <= 16); otherwise has_optab stays false.
// combine_consts = true first multiplies the constant factors of each
// elimination step into one constant tensor (constant step, once per call):
// for engines that load constants from memory rather than folding literals.
// A two-operand contraction of item tensors whose operands split the output
// variables into rows (only the first carries them), columns (only the
// second) and a batch (both), with every summed variable in both, at least
// 4 row and 4 column variables and one summed variable: a batch of complex
// GEMMs per item, the shape the wide engine runs on the matrix cores.
bool matrix_core_shape(const Step& st);
// checkpoint_every = n > 0 (gradient programs): the reverse pass keeps every
// n-th forward elimination output and recomputes the others it needs.
// open_qubits: qubits whose output variables stay open (the final step has
// rank open_qubits.size(); bit i of its element index is open_qubits[i]).
bool compile_program(const Network& net, const std::vector<int>& sliced, const std::vector<int>& order,
                     Program& prog, std::string& err, int& code, bool gradient = false, bool combine_consts = false,
                     int checkpoint_every = 0, const std::vector<int>& open_qubits = {});

// The same sliced variables in an order for group sharing (slice-index bits
// 6 and up tell the 64-item groups of a pass apart; an item step that
// depends on none of a pass's varying bits runs once per pass): from bit 6
// up, each position takes the variable that leaves the most item work (the
// program's per-step roofline time) independent of the variables placed
// there so far; bits 0..5 keep the others in their given order.  Returns the
// input unchanged when k <= 6 or the program does not compile.  *shared_frac
// (if not null) gets the fraction of the item work independent of the
// variables at bits 6 and 7.
std::vector<int> sliced_order_for_groups(const Network& net, const std::vector<int>& sliced,
                                         const std::vector<int>& order, double* shared_frac = nullptr);
// The greedy choice behind it on a compiled program (combine_consts) with k
// sliced variables: the sliced positions for bits 6, 7, ..., k - 1.
std::vector<int> group_bit_positions(const Program& prog, int k, double* shared_frac = nullptr);

// ------------------------------------------------------------ wide engine
// Descriptors for plans whose tensors are too large for registers or LDS.
// Item tensors live in HBM as [element][64 items] rows; every step is one
// kernel.  Leaves are read in place from the gate tables.
enum WideOpKind { WOP_ITEM = 0, WOP_CONST = 1, WOP_LEAF = 2 };
constexpr int kWideOpInts = 64;  // per operand: see encode_wide
constexpr int kWideMaxOut = 32, kWideMaxSum = 16;

struct WideProgram {
  std::vector<int32_t> steps;  // 8 ints per step: kind, out, r, ns, m, grad_slot, op_begin, is_const
  std::vector<int32_t> ops;    // kWideOpInts ints per operand
  int n_steps = 0;
  // fixed-variable dependence (Step::fix_mask) per step and per operand;
  // empty: every step depends on all of them
  std::vector<uint64_t> step_fix, op_fix;
};

// Builds the wide descriptors; false (with err) if a step exceeds the limits.
bool encode_wide(const Program& prog, WideProgram& wide, std::string& err);

// Generated wide kernels.  kind 0: one level of mutually independent item
// steps (blocks of 256 threads per 64-item group, each block running four
// wavefront tiles of one step); kind 1: a run of small constant steps in one
// block of 1024 threads; kind 2: one large constant step, `blocks` = its
// output elements (one thread each).
struct WideKernel {
  int kind;
  std::string name;
  unsigned long long blocks;
  int threads = 256;          // threads per block (level kernels: 64 per wavefront)
  std::vector<int> steps;
  int mfma_steps = 0;       // steps of this kernel on the matrix cores
  double mfma_flops = 0.0;  // their flops per item
  double flops = 0.0;       // flops per item of all its steps
  double bytes = 0.0;       // algorithmic bytes per item of all its steps (8 B per element)
  // per item step of a level kernel: flops, bytes and fixed-variable
  // dependence (Step::fix_mask), for the work a pass with group sharing does
  std::vector<double> step_flops, step_bytes;
  std::vector<uint64_t> step_fix;
};

// Useful real flops of one product-sum step per item: 2^(r + ns) products
// of the m_in operands that carry summed variables (6 flops per complex
// multiply, 2 per complex add), then, when something is summed, each of the
// 2^r sums times the m_out operands that carry none (they are the same for
// every summed index, so they multiply the sum once).
inline double step_flops(int r, int ns, int m_in, int m_out) {
  if (ns == 0 || m_in == 0) {
    m_in += m_out;
    m_out = 0;
  }
  return std::ldexp(1.0, r + ns) * (6.0 * std::max(0, m_in - 1) + 2.0) + 6.0 * std::ldexp(1.0, r) * m_out;
}

// Fixed variables that differ between the 64-item groups first_group ..
// first_group + n_groups - 1 of a pass (item i: bitstring i / n_s, slice
// s_begin + i % n_s): slice bits, and bit 63 when the groups span several
// bitstrings.  Lanes of different groups agree on slice bits 0..5 only
// when n_s and s_begin are multiples of 64; otherwise all bits (~0: no step
// is the same in every group).  A step whose fix_mask has none of these
// bits computes the same values in every group of the pass.
inline uint64_t group_vary_mask(uint64_t first_group, int n_groups, uint64_t s_begin, uint64_t n_s) {
  if (n_s % 64 != 0 || s_begin % 64 != 0) return ~0ull;
  const uint64_t i0 = first_group * 64;
  const uint64_t b0 = i0 / n_s, s0 = s_begin + i0 % n_s;
  uint64_t v = 0;
  for (int y = 1; y < n_groups; ++y) {
    const uint64_t iy = i0 + (uint64_t)y * 64;
    if (iy / n_s != b0) v |= 1ull << 63;
    v |= (s_begin + iy % n_s) ^ s0;
  }
  return v;
}
// Tile parameters of a matrix-core step (two-operand contraction with ni
// row, nj column and nk summed bits).  per: k steps per LDS stage (one block
// barrier each); lds_budget: bytes of LDS the operand ring may take (2..8
// stages); jband: log2 of the j blocks that run next to each other on one
// XCD; layout: 0 = built-in (2 x 2 wavefront tiles when both sides have 5
// bits), 1 = four 16-item groups per block, 2 = two i tiles x two item
// groups, 3 = two j tiles x two item groups (2 and 3 need 5 bits on that
// side, else the built-in choice is kept).
struct MfmaTile {
  int per = 2;
  int lds_budget = 53248;
  int jband = 2;
  int layout = 0;
};
struct TileKey {
  int prec, ni, nj, nk;
  bool operator<(const TileKey& o) const {
    return prec != o.prec ? prec < o.prec : ni != o.ni ? ni < o.ni : nj != o.nj ? nj < o.nj : nk < o.nk;
  }
};
using TileTable = std::map<TileKey, MfmaTile>;
// Text form, one entry per line: "prec ni nj nk per lds_budget jband layout";
// '#' starts a comment.  read: false (with err) on a malformed line.
bool read_tile_table(const std::string& path, TileTable& t, std::string& err);
// (nb, ni, nj, nk) of wide step si when it runs on the matrix cores in
// precision prec (1 = complex64, 2 = BF16x3).
bool mfma_step_shape(const WideProgram& wide, int si, int prec, int& nb, int& ni, int& nj, int& nk);
bool write_tile_table(const std::string& path, const TileTable& t, std::string& err);
std::string generate_wide_source(const Program& prog, const WideProgram& wide, int prec,
                                 std::vector<WideKernel>& kernels, bool mfma, const TileTable* tiles = nullptr);

// Straight-line HIP source (kernel "qgm_chain") for the item steps of `prog`;
// prec 0 = complex128, 1 = complex64.
// *waves_out gets the wavefronts per block (the item tree may be cut across
// several wavefronts that run the same 64 items).
// force_waves > 0 requests that many wavefronts (0 = cost model).
// persistent = true: a grid of resident blocks pulls 64-item chunks from a
// device work queue (a counter that must be zero at launch) instead of one
// block per chunk.
std::string generate_chain_source(const Program& prog, int prec, int n_qubits, int* waves_out, int force_waves = 0,
                                  bool persistent = false);
// hiprtc compilation of `src` for gfx950 into a code object.
bool jit_compile(const std::string& src, const char* name, std::vector<char>& code, std::string& err);

}  // namespace qgm
