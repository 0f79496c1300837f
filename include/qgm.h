/* qgm -- single output amplitudes <x|C|0^N> of grid random circuits by
 * sliced variable elimination on the undirected graphical model, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method (Chen, Zhang, Huang, Newman, Shi, "Classical Simulation of
 * Intermediate-Size Quantum Circuits", arXiv:1805.01450):
 *   - the amplitude is the Feynman sum of Eq. (1);
 *   - diagonal gates identify indices, every distinct index is a binary
 *     variable, gates are factors (Section "Undirected Graphical Model",
 *     gadgets of Fig. "tensornodes");
 *   - output variables are fixed to x and k chosen variables are fixed
 *     ("sliced") to the bits of s in [0, 2^k), giving 2^k independent sums
 *     whose total is the amplitude (Section "Parallelization by fixing the
 *     values of variables");
 *   - each slice is evaluated by variable elimination along a fixed order
 *     (Section "Variable elimination"), and the slices are summed.
 *
 * Conventions for every entry point:
 *   - Every function returns a qgm_status; no C++ exception crosses the ABI.
 *     On a non-OK status qgm_last_error() returns a thread-local message
 *     (valid until the next failing call on the same thread).
 *   - The caller owns every array it passes; arrays are read during the call
 *     only.  Opaque handles are owned by the library until their *_free.
 *   - Device workspace and HIP stream belong to the caller.
 *   - Bitstrings are bytes 0/1, row-major (n_bs rows of n_qubits); x[q] is
 *     the value of qubit q.  Amplitudes are FP64 (re, im) pairs.
 *   - Variable ids: variables are created by non-diagonal gates taken by
 *     ascending cycle, then ascending (lowest) qubit, and numbered 0, 1, ...
 *     in that order; a non-diagonal two-qubit gate creates two, the lower
 *     qubit's first; the output variable of a qubit is its last variable.
 *   - Slice s fixes sliced_vars[j] to bit j of s.
 */
#ifndef QGM_H
#define QGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QGM_OK = 0,
  QGM_E_ARG = -1,         /* bad argument (null pointer, size, bitstring value) */
  QGM_E_PARSE = -2,       /* circuit text rejected */
  QGM_E_ORDER = -3,       /* order is not a permutation of the free, non-sliced variables */
  QGM_E_SLICE = -4,       /* sliced variables not distinct free variables, or k > 40 */
  QGM_E_WORKSPACE = -5,   /* workspace too small, or plan exceeds the caller's cap */
  QGM_E_HIP = -6,         /* HIP runtime error (message has hipGetErrorString) */
  QGM_E_UNSUPPORTED = -7  /* option or combination of options not supported by the library */
} qgm_status;

typedef enum {
  QGM_C128 = 0,  /* complex128 contraction */
  QGM_C64 = 1,   /* complex64 contraction, FP32 accumulation */
  QGM_BF16X3 = 2 /* complex64 storage; every real product from bf16 splits x = xh + xl (round to
                    nearest even): xh*yh + xh*yl + xl*yh, accumulated in FP32 */
} qgm_precision;

typedef struct qgm_circuit qgm_circuit;
typedef struct qgm_plan qgm_plan;

typedef struct {
  int32_t id, qubit, cycle_created, is_output;
} qgm_var_info;

typedef struct {
  int32_t prec;          /* qgm_precision */
  int32_t profile;       /* 1 = record HIP events around each kernel of every run (qgm_plan_timing) */
  size_t workspace_cap;  /* bytes; 0 = no cap (WIDE: 96 GiB of item tensors per pass); else the
                            WIDE engine's item memory per pass, and plan_create fails with
                            QGM_E_WORKSPACE when the memory of one 64-item group (one
                            wavefront) of the program that runs cannot fit */
  int32_t engine;        /* QGM_ENGINE_*: how the per-item chain runs on the device */
  int32_t gradient;      /* 1 = also compile the reverse-mode steps for d alpha / d theta */
  int32_t waves;         /* GENERATED: wavefronts per block to cut the item tree across
                            (1, 2, 4 or 8; fewer when the exchange does not fit in LDS or
                            the program is not a tree); 0 = chosen by the cost model */
  int32_t vector_only;   /* WIDE: 1 = run every step on the vector ALUs; 0 = two-operand
                            complex64 and BF16x3 contractions with >= 4 row bits, >= 4
                            column bits and >= 1 summed bit (optionally times a constant
                            scale of the results) run on the matrix cores */
  int32_t checkpoint_every;  /* gradient plans: 0 = every forward tensor stays in item memory
                                until its reverse step; n > 0 = only every n-th forward
                                elimination output is kept (a checkpoint) and the others are
                                recomputed from the checkpoints during the reverse pass */
  int32_t persistent;        /* GENERATED: 1 = a resident grid (as many blocks as fit on the
                                device) pulls 64-item chunks from a device work queue instead
                                of one block per chunk (INTERPRETER always works this way;
                                WIDE launches one kernel per level) */
  int32_t deterministic;     /* 0 or 1.  Every engine already returns bit-identical results for
                                identical inputs (fixed slice-sum order, no atomics in any
                                sum); 1 documents the caller's reliance on it */
  int32_t n_open;            /* open outputs: the number of entries of open_qubits (0..10) */
  const char* tile_table_path; /* WIDE matrix-core steps: a tile table written by
                                qgm_plan_tune_tiles (read at plan creation; the string is
                                not kept); steps whose shape has an entry use the tuned
                                tile parameters; NULL = built-in choice.  An unreadable or
                                malformed table is QGM_E_ARG */
  const int32_t* open_qubits;  /* n_open distinct qubits whose output variables stay open: they
                                are neither fixed to the bitstring nor summed, so one
                                contraction gives 2^n_open amplitudes (the paper's Discussion:
                                a large slice of amplitudes from one evaluation).  Amplitude e
                                of bitstring b is <x|C|0> with x = b except x[open_qubits[i]]
                                = bit i of e; the bitstring's entries at open qubits are
                                ignored.  Every amplitude output (out, partial, d_partial)
                                then holds 2^n_open entries per bitstring, b-major.  Not with
                                gradient = 1 (QGM_E_UNSUPPORTED); a qubit without a variable
                                of its own (no H, SX or SY) cannot be open (QGM_E_ARG).  The
                                array is read during qgm_plan_create only */
} qgm_plan_opts;

/* Per-item chain engines.  AUTO picks GENERATED when the plan's live item
 * memory fits in registers, INTERPRETER when every step is small (rank +
 * summed variables <= 16) and WIDE otherwise.
 * GENERATED: plan_create emits straight-line HIP for the plan (every operand
 *   offset is static) and compiles it for gfx950 with hiprtc; item tensors
 *   live in registers; slice sums are fused into the kernel.
 * INTERPRETER: one prebuilt persistent kernel walks a step table with a
 *   device work queue; item tensors live in LDS (or global scratch).
 * WIDE: one kernel per elimination step; item tensors live in HBM as
 *   [element][64 items] rows (every access a contiguous row); groups of 64
 *   items are processed in passes that fit workspace_cap (default 96 GiB). */
enum { QGM_ENGINE_AUTO = 0, QGM_ENGINE_INTERPRETER = 1, QGM_ENGINE_GENERATED = 2, QGM_ENGINE_WIDE = 3 };

typedef struct {
  int32_t n_steps;        /* elimination + leaf steps of the compiled program */
  int32_t n_const_steps;  /* steps independent of the output bits and the slice */
  int32_t max_rank;       /* largest intermediate tensor rank */
  int32_t item_elems;     /* peak live tensor elements per work item */
  int32_t n_leaves;       /* factors read at fixed (output or sliced) values per item */
  int32_t k;              /* sliced variables */
  double flops_item;      /* useful real flops per slice contraction (6 per complex
                             multiply, 2 per complex add) */
  double flops_const;     /* flops of the constant steps, once per call */
  double bytes_item;      /* bytes read + written per slice if every intermediate made
                             one trip to memory, at 8 B per element */
  double cost;            /* sum over eliminations of 2^deg(v) (Section "Variable elimination") */
  int32_t engine;         /* engine the plan runs with (INTERPRETER, GENERATED or WIDE) */
  int32_t waves;          /* GENERATED: wavefronts per block the item tree is cut across */
  double compile_s;       /* seconds spent generating and compiling the plan's kernel */
  int32_t launches;       /* kernel launches of the item steps per pass: WIDE with
                             generated kernels, one per level of mutually independent
                             steps; otherwise the item steps' kernel count */
  int32_t mfma_steps;     /* WIDE, complex64 and BF16x3: item steps that run on the matrix
                             cores (two-operand contractions with >= 4 row, >= 4 column and
                             >= 1 summed bits, optionally times a constant scale) */
  double flops_mfma;      /* the part of flops_item those steps perform */
  double roof_s_item;     /* chain roofline time per slice contraction: the sum over item
                             steps of max(flops / 157.3 TFLOP/s, bytes / 8 TB/s), MI355X's
                             FP32 and HBM peaks, bytes as in bytes_item */
  int32_t n_open;         /* open outputs: 2^n_open amplitudes per bitstring */
} qgm_stats;

/* Circuit text v1, one gate per line, '#' starts a comment:
 *   qubits N            (N <= 64)
 *   grid R C            (optional)
 *   <cycle> <GATE> <q0> [<q1>] [<param_index>]
 * GATE in {H, CZ, T, SX, SY, RZ, I, CX, ISWAP, SQISW}.  CZ, CX, ISWAP and
 * SQISW take two qubits, RZ one qubit and a parameter index into the params
 * array of the amplitude calls.  Gates of one cycle must act on distinct
 * qubits.  Matrices: H = [[1,1],[1,-1]]/sqrt2, SX and SY the principal square
 * roots of X and Y, T = diag(1, e^{i pi/4}), RZ(t) = diag(e^{-it/2},
 * e^{it/2}), CZ = diag(1,1,1,-1); CX has control q0 and target q1, ISWAP maps
 * |01> to i|10> and |10> to i|01>, SQISW is its principal square root.  The
 * non-diagonal two-qubit gates give one four-variable factor (two new
 * variables, two old ones: the gadget of Fig. "tensornodes").
 * (Clock cycles C_1..C_d of Eq. (1); gates of Fig. 2 and Rule 3.)
 * Errors: QGM_E_ARG (null), QGM_E_PARSE (message names the line). */
qgm_status qgm_circuit_parse(const char* text, size_t len, qgm_circuit** out);
/* Sizes of a parsed circuit: qubits, variables of the graphical model
 * (Section "Undirected Graphical Model"), RZ parameters.  Errors: QGM_E_ARG. */
qgm_status qgm_circuit_info(const qgm_circuit* c, int32_t* n_qubits, int32_t* n_vars, int32_t* n_params);
/* Variable table (Section "Undirected Graphical Model"): writes min(cap, n_vars)
 * entries of buf. */
qgm_status qgm_circuit_vars(const qgm_circuit* c, qgm_var_info* buf, int32_t cap);
/* Edges (u, w), u < w, of the graph over the free (non-output) variables:
 * two variables are adjacent when a gate acts on both (Fig. 3).  Writes up to
 * cap pairs into edges[2*cap]; *n_edges gets the total count. */
qgm_status qgm_circuit_graph(const qgm_circuit* c, int32_t* edges, int32_t cap, int32_t* n_edges);
/* Releases a parsed circuit.  NULL is a no-op. */
void qgm_circuit_free(qgm_circuit* c);

/* Host planner (Section "The variable elimination ordering", Section
 * "Parallelization by fixing the values of variables"): a min-fill ordering
 * (best of randomised restarts within the time budget), then greedy removal of
 * key vertices, each minimising sum 2^deg under that fixed ordering, then a
 * new ordering of the remaining variables.  k_req >= 0 removes exactly k_req
 * vertices; k_req < 0 removes vertices until the width is <= target_rank
 * (at most 40).  sliced_out needs room for 40 ids (or k_req), order_out for
 * n_vars ids.  Errors: QGM_E_ARG. */
qgm_status qgm_plan_slices(const qgm_circuit* c, int32_t k_req, int32_t target_rank, double time_budget_s,
                           uint64_t seed, int32_t* sliced_out, int32_t* k_out, int32_t* order_out,
                           int32_t* n_order_out);
/* As qgm_plan_slices, with flags:
 *   QGM_PLAN_REORDER: recompute the ordering after every removal, as the
 *     paper's Discussion suggests, instead of keeping the first ordering;
 *   QGM_PLAN_BYTES: choose the final ordering among the restarts by the
 *     memory traffic of the compiled program (each step's inputs and output,
 *     fused eliminations as compiled) instead of the sum of 2^deg(v);
 *   QGM_PLAN_LATENCY: choose it by the time of one item on four wavefronts,
 *     max(4 x critical path, total) in flops of the compiled steps, for
 *     batches too small to fill the GPU (takes precedence over BYTES);
 *   QGM_PLAN_SEARCH: plan repeatedly (seeds seed, seed', ...; each seed
 *     once keeping the first ordering and once re-ordering after every
 *     removal; each attempt with budget / 8; at most 64 attempts) while the
 *     time budget lasts, and keep the plan whose final ordering scores best
 *     (sum of 2^deg(v), or the BYTES / LATENCY / WIDE_TIME objective).  The
 *     number of attempts depends on the host's speed, so the same budget can
 *     give different plans on different hosts;
 *   QGM_PLAN_WIDE_TIME: with SEARCH, score each plan by its program as the
 *     WIDE engine compiles it (constant factors combined, small eliminations
 *     absorbed, operand pairs pre-contracted): seconds per slice with the
 *     flops of matrix-core-shaped contractions at 65 TFLOP/s, the other
 *     flops at 30 TFLOP/s and the bytes at 5 TB/s, the rates its kernels
 *     reach on MI355X;
 *   QGM_PLAN_CHOOSE_K: with SEARCH | WIDE_TIME and k_req >= 0, k_req is the
 *     largest k tried: each k from k_req down to k_req - 6 gets an equal
 *     share of the budget, and the plan with the least predicted time for
 *     the whole amplitude (2^k x the per-slice score) wins among those
 *     whose peak item memory fits a 64-item group in 96 GiB (complex128).
 *     *k_out gives the chosen k.  Fails with QGM_E_WORKSPACE when no k
 *     fits;
 *   QGM_PLAN_BNB: after the min-fill restarts (half the final ordering's
 *     budget), a branch-and-bound search over orderings (the QuickBB scheme
 *     of Section "The variable elimination ordering", see qgm_order_search)
 *     from the best of them, 200 search nodes per second of the other half,
 *     3 children per node on graphs of more than 20 vertices; with k_req = 0
 *     the whole budget goes to the ordering.  Sum-of-2^deg objective only;
 *   QGM_PLAN_DETERMINISTIC: the budget counts work instead of wall-clock
 *     time (320 min-fill restarts per second of budget, at most 128 per ordering; SEARCH makes
 *     exactly 8 attempts), so every host returns the same plan for the
 *     same arguments. */
enum {
  QGM_PLAN_REORDER = 1,
  QGM_PLAN_BYTES = 2,
  QGM_PLAN_LATENCY = 4,
  QGM_PLAN_SEARCH = 8,
  QGM_PLAN_WIDE_TIME = 16,
  QGM_PLAN_CHOOSE_K = 32,
  QGM_PLAN_DETERMINISTIC = 64,
  QGM_PLAN_BNB = 128
};
qgm_status qgm_plan_slices_ex(const qgm_circuit* c, int32_t k_req, int32_t target_rank, double time_budget_s,
                              uint64_t seed, int32_t flags, int32_t* sliced_out, int32_t* k_out, int32_t* order_out,
                              int32_t* n_order_out);
/* Branch and bound over elimination orderings (the QuickBB scheme of
 * Section "The variable elimination ordering"): depth-first over the next
 * vertex to eliminate, children in min-fill order, a branch pruned when the
 * minor-min-width of the remaining graph shows it cannot beat the best
 * ordering found so far.  Graph: the free variables with the sliced ones
 * removed.  Objective: (width, cost) compared lexicographically, width =
 * max deg(v) and cost = sum 2^deg(v) at elimination.  init_order (a
 * permutation of the free non-sliced variables) is the first incumbent;
 * the search stops after max_nodes nodes; beam > 0 tries only that many
 * children per node (<= 0: all, and then *complete = 1 means the result is
 * optimal).  order_out gets n_order ids.  Errors: QGM_E_SLICE, QGM_E_ORDER as
 * for qgm_plan_create, QGM_E_ARG. */
qgm_status qgm_order_search(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k, const int32_t* init_order,
                            int32_t n_order, int64_t max_nodes, int32_t beam, int32_t* order_out, double* cost,
                            int32_t* width, int32_t* complete);
/* Not in the paper (a layout choice of this library).  The same sliced
 * variables in an order for group sharing.  Slice s fixes sliced_vars[j] to
 * bit j of s; 64 consecutive slices form one item group, so bits 6 and up
 * tell the groups of a pass apart, and an item step that depends on none of
 * the sliced variables at the bits that vary within a pass (nor on the
 * output bits, when a pass spans several bitstrings) is computed once per
 * pass and read by every group (WIDE engine; only when the call's slice
 * range starts at a multiple of 64 and holds a multiple of 64 slices).
 * From bit 6 up, each position gets the variable that leaves the most item
 * work (the compiled program's per-step roofline time) independent of the
 * variables already placed there; bits 0..5 keep the others in their given
 * order.  The amplitude (the sum over all slices) does not change; which
 * assignment a single slice index denotes does.  qgm_plan_slices and
 * qgm_plan_slices_ex return their sliced variables in this order.
 * sliced_out: k ids (may alias sliced_vars only if the caller copies them
 * first: it is written after the input is read).  *shared_frac (may be
 * NULL): the fraction of the item work independent of the variables at
 * bits 6 and 7.  k <= 6: the input order.  Errors: QGM_E_SLICE,
 * QGM_E_ORDER as for qgm_plan_create, QGM_E_ARG. */
qgm_status qgm_sliced_order_for_groups(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k,
                                       const int32_t* order, int32_t n_order, int32_t* sliced_out,
                                       double* shared_frac);
/* Cost (sum of 2^deg(v)) and width (max deg(v)) of eliminating `order` after
 * removing the sliced vertices (Section "Variable elimination", cost model).
 * Errors: QGM_E_SLICE, QGM_E_ORDER as for qgm_plan_create. */
qgm_status qgm_order_cost(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k, const int32_t* order,
                          int32_t n_order, double* cost, int32_t* width);

/* Compile the per-slice contraction program for (circuit, sliced_vars,
 * order): the variable elimination of Section "Variable elimination"
 * (steps 1-4: for each variable in the order, multiply the tensors that hold
 * it and sum it out) on the network with the outputs and the sliced
 * variables fixed (Section "Parallelization by fixing the values of
 * variables").  Host only; device tables are uploaded at the first run on the
 * then-current device.  opts may be NULL (complex128, no cap).
 * Errors: QGM_E_SLICE (ids not distinct free variables, or k > 40),
 * QGM_E_ORDER (order not a permutation of the free non-sliced variables),
 * QGM_E_WORKSPACE (over opts->workspace_cap), QGM_E_UNSUPPORTED (precision). */
qgm_status qgm_plan_create(const qgm_circuit* c, const int32_t* sliced_vars, int32_t k, const int32_t* order,
                           int32_t n_order, const qgm_plan_opts* opts, qgm_plan** out);
/* Statistics of a compiled plan (cost: the sum of 2^deg(v) of Section
 * "Variable elimination"; flops and bytes: the algorithmic work of the
 * compiled steps).  Errors: QGM_E_ARG (null). */
qgm_status qgm_plan_stats(const qgm_plan* p, qgm_stats* out);
/* Device workspace bytes needed by a run over n_bs bitstrings and n_slices
 * slices, including the staging room that the host-pointer entry points use.
 * (Workspace sizing is this library's; the paper's subtasks each hold one
 * slice's tensors.)  Errors: QGM_E_ARG, QGM_E_HIP (first upload). */
qgm_status qgm_workspace_size(const qgm_plan* p, int32_t n_bs, uint64_t n_slices, size_t* bytes);

/* alpha_x = <x|C|0...0> (Eq. (1)) for n_bs bitstrings, summed over all 2^k
 * slices (Section "Parallelization by fixing the values of variables":
 * the slices are independent and their results are added).  Host inputs
 * (bitstrings n_bs x n_qubits bytes; params n_params doubles, or NULL when
 * the circuit has no RZ), host output out[2*n_bs] = (re, im).  The slice sum
 * is FP64 with Neumaier compensation in ascending s.  Synchronises `stream`
 * (a hipStream_t, NULL = default stream).
 * Errors: QGM_E_ARG (bitstring entry not 0/1, n_bs < 0, missing params),
 * QGM_E_WORKSPACE (ws_bytes < qgm_workspace_size), QGM_E_HIP. */
qgm_status qgm_amplitudes(qgm_plan* p, const uint8_t* bitstrings, int32_t n_bs, const double* params,
                          void* d_workspace, size_t ws_bytes, void* hip_stream, double* out);
/* Slices [s_begin, s_end) only: the paper's subtasks, any contiguous subset
 * of which can run on its own (Section "Parallelization by fixing the values
 * of variables").  partial[4*n_bs] = (sum re, sum im, comp re,
 * comp im) per bitstring: the Neumaier sum and its compensation, so ranges run
 * separately (e.g. after a failure) combine to the full result.
 * Errors: as qgm_amplitudes, plus QGM_E_ARG when the range is not inside
 * [0, 2^k). */
qgm_status qgm_amplitudes_range(qgm_plan* p, const uint8_t* bitstrings, int32_t n_bs, const double* params,
                                uint64_t s_begin, uint64_t s_end, void* d_workspace, size_t ws_bytes,
                                void* hip_stream, double* partial);
/* Same as qgm_amplitudes_range with every array in device memory and no
 * synchronisation: d_bitstrings (n_bs x n_qubits bytes), d_params, and
 * d_partial[4*n_bs] are device pointers; the work is queued on `stream`.
 * Bitstring entries are used as (value & 1).  Errors: QGM_E_ARG,
 * QGM_E_WORKSPACE, QGM_E_HIP. */
qgm_status qgm_amplitudes_device(qgm_plan* p, const uint8_t* d_bitstrings, int32_t n_bs, const double* d_params,
                                 uint64_t s_begin, uint64_t s_end, void* d_workspace, size_t ws_bytes,
                                 void* hip_stream, double* d_partial);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the run of
 * qgm_amplitudes_device with the workspace taken from a fixed array of
 * QGM_NOALLOC_SCRATCH_BYTES (64 MiB) in the library's device image, one copy
 * per GPU, held until the process ends.  No device memory is allocated or
 * freed by the call.  The plan's tables must already be on the current device
 * (any earlier ordinary call on it, e.g. qgm_workspace_size, uploads them);
 * profiling events are not recorded.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (on different streams or
 * threads) race and give wrong results; the run clears what must start at
 * zero itself.  Arguments and results as qgm_amplitudes_device.
 * Errors: QGM_E_ARG (as qgm_amplitudes_device; plan not yet on this device),
 * QGM_E_WORKSPACE (the run needs more than QGM_NOALLOC_SCRATCH_BYTES; the
 * message gives the size), QGM_E_HIP. */
#define QGM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
qgm_status qgm_amplitudes_device_noalloc(qgm_plan* p, const uint8_t* d_bits, int32_t n_bs, const double* d_params,
                                         uint64_t s_begin, uint64_t s_end, void* hip_stream, double* d_partial);
/* Batching (the paper's independent subtasks run together, Section
 * "Parallelization by fixing the values of variables"; the graph itself is
 * this library's launch mechanism):
 * HIP graph of `repeat` back-to-back runs of qgm_amplitudes_device with
 * these arguments (every array a device pointer, read at each replay).  The
 * runs are captured from a private stream; each replay executes them again
 * on the launch stream, so repeated amplitude batches cost one host call.
 * Captured runs record no profiling events (time a replay with events around
 * qgm_graph_launch on the launch stream).  Errors: as qgm_amplitudes_device, QGM_E_ARG (repeat < 1),
 * QGM_E_HIP (capture or instantiation failed). */
typedef struct qgm_graph qgm_graph;
qgm_status qgm_graph_create(qgm_plan* p, const uint8_t* d_bitstrings, int32_t n_bs, const double* d_params,
                            uint64_t s_begin, uint64_t s_end, void* d_workspace, size_t ws_bytes,
                            double* d_partial, int32_t repeat, qgm_graph** out);
qgm_status qgm_graph_launch(qgm_graph* g, void* hip_stream);
void qgm_graph_free(qgm_graph* g);

/* Not in the paper (a launch-shape choice of this library).
 * Autotuner of the GENERATED engine: the item tree of a plan can be cut
 * across 1, 2, 4 or 8 wavefronts of a block (the cut is the launch shape of
 * the generated kernel).  Each feasible variant is generated, compiled,
 * timed on the device for a batch of n_bs bitstrings x n_slices slices (all
 * bits 0, angles 0, 3 warm-up and 10 timed runs with HIP events on `stream`),
 * and the fastest one is kept for the plan.  *waves_out gets the chosen
 * count.  Other engines: no-op, *waves_out = 1.  The workspace must hold
 * qgm_workspace_size(p, n_bs, n_slices) bytes; its contents are overwritten.
 * Errors: QGM_E_ARG, QGM_E_WORKSPACE, QGM_E_HIP. */
qgm_status qgm_plan_autotune(qgm_plan* p, int32_t n_bs, uint64_t n_slices, void* d_workspace, size_t ws_bytes,
                             void* hip_stream, int32_t* waves_out);

/* Measurement (not in the paper, which times whole subtasks on CPU nodes).
 * Kernel durations of the runs made since the last reset by a plan created
 * with opts.profile = 1: ms[0] prologue (tables, constant steps), ms[1]
 * per-item contraction chain, ms[2] slice reduction, each averaged over the
 * runs and measured with HIP events recorded on each run's own stream.
 * Waits for the last recorded run.  reset = 1 forgets the runs afterwards.
 * Errors: QGM_E_ARG (plan not profiling), QGM_E_HIP. */
qgm_status qgm_plan_timing(qgm_plan* p, int32_t reset, double ms[3], int32_t* n_runs);
/* Measurement (not in the paper).
 * WIDE engine, plan created with opts.profile = 1: per level kernel (one
 * launch of mutually independent elimination steps, in launch order) the
 * duration averaged over the runs since the last reset, measured with HIP
 * events recorded on the run's stream around each launch of the first pass
 * of items, plus the kernel's useful flops and algorithmic bytes per slice
 * contraction of that pass (the flops_item / bytes_item conventions of
 * qgm_stats; a step computed once for the G groups of the pass, see
 * qgm_sliced_order_for_groups, counts 1 / G per item) and its number of
 * matrix-core steps.
 * Fills min(cap, *n_levels) entries of the caller's arrays; *n_levels gets
 * the level count, *n_runs the runs averaged, *items the slice contractions
 * that first pass held (the last run's; a run larger than the workspace
 * takes several passes), *roof_s_item (may be NULL) the pass's roofline
 * time per slice contraction (as qgm_stats roof_s_item, shared steps at
 * 1 / G).  Waits for the last recorded run.  reset = 1 forgets the runs
 * afterwards.  Other engines: *n_levels = 0.  Errors: QGM_E_ARG (null or
 * negative arguments, plan not profiling), QGM_E_HIP. */
qgm_status qgm_plan_level_timing(qgm_plan* p, int32_t reset, double* ms, double* flops_item, double* bytes_item,
                                 int32_t* mfma_steps, int32_t cap, int32_t* n_levels, int32_t* n_runs,
                                 uint64_t* items, double* roof_s_item);
/* Not in the paper (which evaluates amplitudes only): reverse-mode
 * differentiation of the elimination of Section "Variable elimination".
 * Amplitudes and their derivatives with respect to every RZ angle, for a
 * plan created with opts.gradient = 1.  Reverse mode over the elimination
 * steps: the adjoint of alpha_{x,s} is 1; a step out = sum_S prod_i op_i
 * gives each operand the adjoint sum over the variables it lacks of
 * adj(out) * prod_{j != i} op_j (no conjugation: alpha is holomorphic in
 * the gate entries); an RZ(theta) table f(u) = e^{i theta (2u-1)/2} then
 * contributes sum_u adj(u) * (i/2)(2u-1) f(u) to d alpha / d theta.  Forward
 * tensors stay in item memory until their reverse step (no recomputation).
 * Slice sums of gradients use the amplitudes' FP64 compensated order.
 * d_grad_partial[4 * (b * n_params + j)] = (sum re, sum im, comp re, comp
 * im) of d alpha_b / d theta_j.  Device pointers, no synchronisation.
 * Errors: as qgm_amplitudes_device; QGM_E_ARG when the plan has no gradient
 * program or d_grad_partial is NULL. */
qgm_status qgm_gradients_device(qgm_plan* p, const uint8_t* d_bitstrings, int32_t n_bs, const double* d_params,
                                uint64_t s_begin, uint64_t s_end, void* d_workspace, size_t ws_bytes,
                                void* hip_stream, double* d_partial, double* d_grad_partial);
/* Host form of qgm_gradients_device (same passages) for one bitstring over
 * all slices: amp_out[2] = alpha,
 * dalpha_dtheta[2 * n_params] = (re, im) of d alpha / d theta_j.  Synchronises
 * `stream`.  Errors: as qgm_gradients_device, QGM_E_WORKSPACE. */
qgm_status qgm_amplitude_grad(qgm_plan* p, const uint8_t* bitstring, const double* params, void* d_workspace,
                              size_t ws_bytes, void* hip_stream, double* amp_out, double* dalpha_dtheta);
/* Releases the plan and its device tables (call with the plan's device
 * current).  NULL is a no-op. */
void qgm_plan_free(qgm_plan* p);
/* Message of the last non-OK status on this thread. */
const char* qgm_last_error(void);

/* One step of the elimination on its own: out[b, j, i] = sum_k A[b, k, i] *
 * B[b, j, k] for every item, the pairwise form of "multiply the tensors that
 * hold the summed variables, then sum them out" (Section "Variable
 * elimination", steps 2-3) with ni row, nj column, nb batch and nk summed
 * binary indices.  The kernel is generated by the same code as the chain's
 * level kernels: on the matrix cores when the shape qualifies (complex64 or
 * BF16x3, nk >= 1, ni >= 4, nj >= 4) unless flags bit 0 (vector ALUs only)
 * is set, else on the vector ALUs.  For tests and tile tuning.
 * Layout (caller-owned device memory, complex elements of the precision:
 * 16 B for QGM_C128, 8 B (float re, im) otherwise): group g of 64 items
 * starts at element g * E * 64 with E = 2^(nb+ni+nk) + 2^(nb+nk+nj) +
 * 2^(nb+ni+nj); inside a group element e of item l is at e * 64 + l.  A is
 * elements [0, 2^(nb+ni+nk)) with index i + 2^ni k + 2^(ni+nk) b, B follows
 * with index k + 2^nk j + 2^(nk+nj) b, then C with index i + 2^ni j +
 * 2^(ni+nj) b.  qgm_contraction_run queues n_groups groups (at most 65535)
 * on `stream`, overwriting C only; no synchronisation.
 * Errors: QGM_E_ARG (counts: nb + ni + nj <= 32, nk <= 16, E < 2^31),
 * QGM_E_UNSUPPORTED (precision, compile failure), QGM_E_HIP. */
typedef struct qgm_contraction qgm_contraction;
/* Tile parameters of a matrix-core step (see qgm_plan_tune_tiles):
 *   per: k steps per LDS stage, one block barrier each (power of two; the
 *     16-item BF16x3 forms use pairs, so at least 2; in the per-item BF16x3
 *     form one step is four complex k, one 16 x 16 x 32 MFMA pair);
 *   lds_budget: bytes of LDS the operand ring may use (2..8 stages);
 *   jband: log2 of the j blocks that run next to each other on one XCD
 *     (16-item forms only);
 *   layout: complex64, and BF16x3 steps that sum fewer than 2 bits: 0 =
 *     built-in (2 x 2 wavefront tiles when both sides have 5 or more bits),
 *     1 = four 16-item groups per block, 2 = two i tiles x two item groups,
 *     3 = two j tiles x two item groups.  BF16x3: 0 = the per-item form
 *     (one item per wavefront, up to 64 x 64 outputs of it), 4, 5, 6 = that
 *     form with at most 32 rows, 32 columns, or both; 1 to 3 = the 16-item
 *     forms above, 7 = their built-in choice; 8 + (0, 4, 5, 6) = the
 *     per-item form with eight items (wavefronts) per block instead of
 *     four.  16 + (0, 4, 5, 6) (+ 8): the per-item form for either
 *     precision; complex64 runs it on v_mfma_f32_16x16x4_f32 (four real
 *     products per tile and K step of four complex k).  In the per-item
 *     form jband 1 stores results straight from registers instead of
 *     through LDS.
 *     complex64 per-item layouts + 32: the three-multiplication complex
 *     product (Cr = sum ar br - sum ai bi, Ci = sum (ar + ai)(br + bi) -
 *     sum ar br - sum ai bi: three FP32 products per tile and K step
 *     instead of four; error bound (3K + 9) 2^-24 sum |a||b| instead of
 *     (2K + 2) 2^-24 for a sum of K terms).
 *   Built in for BF16x3: the per-item form with two K steps per stage and
 *   a 64 KiB ring when the step sums 5 or more bits, else layout 7. */
typedef struct {
  int32_t per, lds_budget, jband, layout;
} qgm_tile;
/* tile: NULL = built-in choice.  Errors also: QGM_E_ARG (tile out of range). */
qgm_status qgm_contraction_create(int32_t prec, int32_t nb, int32_t ni, int32_t nj, int32_t nk, int32_t flags,
                                  const qgm_tile* tile, qgm_contraction** out);
/* *matrix_cores = 1 when the step runs on the matrix cores; *elems_per_item
 * = E; *flops_per_item = useful real flops per item (8 per complex
 * multiply-add). */
qgm_status qgm_contraction_info(const qgm_contraction* c, int32_t* matrix_cores, uint64_t* elems_per_item,
                                double* flops_per_item);
qgm_status qgm_contraction_run(qgm_contraction* c, void* d_mem, int64_t n_groups, void* hip_stream);
void qgm_contraction_free(qgm_contraction* c);

/* Not in the paper (a launch-shape choice of this library).  Tile autotuner
 * for the matrix-core steps of a WIDE complex64 or BF16x3 plan: for each
 * step shape (ni, nj, nk), largest flops first until 99 % of the plan's
 * matrix-core flops are covered, candidate tiles (block layout and k per
 * stage, then ring budget and band) are generated, compiled and timed on the
 * device as single contractions (qgm_contraction_*; a batch of 64 items with
 * enough batch bits to fill the GPU, at most 8 GiB of operands, allocated
 * and freed here; 2 warm-up and 5 timed runs with HIP events on `stream`),
 * and the fastest is written to the text table at table_path (entries of
 * other shapes already there are kept).  Plans created with
 * opts.tile_table_path = table_path then use the tuned tiles.  *n_tuned gets
 * the number of shapes tuned (0 for plans without matrix-core steps).
 * Errors: QGM_E_ARG (null, unreadable or unwritable table), QGM_E_HIP. */
qgm_status qgm_plan_tune_tiles(qgm_plan* p, const char* table_path, void* hip_stream, int32_t* n_tuned);

/* One-shot form plan(circuit, bitstring, sliced_vars, order) -> amplitude,
 * the paper's problem statement (compute one amplitude <x|C|0...0> of a
 * circuit, Section "Our Contributions") with a given slicing and ordering:
 * parse, plan, run one bitstring in complex128 with a library-allocated
 * workspace on the default stream, free.  out[2] = (re, im). */
qgm_status qgm_amplitude(const char* circuit_text, size_t len, const uint8_t* bitstring,
                         const int32_t* sliced_vars, int32_t k, const int32_t* order, int32_t n_order,
                         const double* params, double out[2]);

#ifdef __cplusplus
}
#endif
#endif /* QGM_H */
