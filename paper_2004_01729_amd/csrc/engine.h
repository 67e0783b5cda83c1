// A small tensor-program engine for the FT-CCSD residual.
//
// A Program is a list of tensor contractions written with index letters
//     out[oi] (+)= alpha * A[ai] * B[bi]      (einsum semantics, one or two operands)
// over tensors whose every axis has length n (hole and particle slots both run
// over all orbitals at finite temperature).  An Executor binds the symbolic
// tensors of one Program to device buffers for a list of problems (one
// instance and one imaginary-time node each) and lowers every op once into
// grouped kernel launches: LDS-tiled index permutes, FP64-MFMA GEMMs (split-K
// when M*N is small) and dot reductions.  The launch lists are replayed on
// every sweep.
//
// Reverse mode: every op is linear in each operand, so its vector-Jacobian
// product is a contraction of the same form,
//     dA[ai] += alpha * dOut[oi] * B[bi],   dB[bi] += alpha * A[ai] * dOut[oi],
// and the backward launch list is the forward program reversed.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <initializer_list>
#include <map>
#include <string>
#include <vector>

#include "kernels.h"

namespace ftcc {

enum TensorKind { T_INPUT = 0, T_CONST = 1, T_INTER = 2, T_OUTPUT = 3 };

struct TensorDecl {
  std::string name;
  int rank;
  TensorKind kind;
  bool derived = false;   // computed from constants only (set-up ops)
};

struct SymOp {
  int out;
  std::string oi;
  double alpha;
  int a;
  std::string ai;
  int b;  // -1: single operand
  std::string bi;
  bool accumulate;
  bool setup;
};

class Program {
 public:
  int tensor(const std::string& name, int rank, TensorKind kind);
  int id(const std::string& name) const;
  // out[oi] (+)= alpha * A[ai] (* B[bi]); the first op on `out` must have acc = false
  void op(const std::string& out, const std::string& oi, double alpha, const std::string& a,
          const std::string& ai, const std::string& b, const std::string& bi, bool acc);
  void set(const std::string& out, const std::string& oi, double alpha, const std::string& a,
           const std::string& ai, const std::string& b = "", const std::string& bi = "") {
    op(out, oi, alpha, a, ai, b, bi, false);
  }
  void add(const std::string& out, const std::string& oi, double alpha, const std::string& a,
           const std::string& ai, const std::string& b = "", const std::string& bi = "") {
    op(out, oi, alpha, a, ai, b, bi, true);
  }
  void finalize();
  bool finalized() const { return finalized_; }
  // Conservation law of a tensor: sum over its axes of sign[axis] * k(index) = 0
  // for every nonzero element (k: the orbitals' conserved momentum).  Declared
  // for inputs and constants; the executor infers the laws of the other tensors.
  void set_law(const std::string& name, const std::vector<int>& signs);
  std::vector<TensorDecl> t;
  std::vector<SymOp> ops;
  std::vector<std::vector<int>> law;   // per tensor, empty: not declared

 private:
  bool finalized_ = false;
};

// The spin-restricted FT-CCSD kernels E, S1, S2 as a Program.
Program build_residual_program();
Program build_spin_orbital_program();

struct Launch {
  enum Kind { PERM, GEMM, DOT, FILL, SGEMM, ELEM, DOTB } kind = PERM;
  int n_prob = 0;
  int total = 0;
  int cfg = 0;
  bool ta = false, tb = false;
  int splitk_blocks = 0;
  int min_k = 0;                    // smallest K of the launch's GEMM problems
  void* d_tasks = nullptr;          // SGEMM / ELEM: task list
  int n_tasks = 0;
  void* d_bfirst = nullptr;         // ELEM / DOTB: per 256-element block, the task of its first element
  void* d_red = nullptr;            // SGEMM: reductions of split inner ranges
  int n_red = 0;
  bool zero_fill = false;           // ELEM with alpha = beta = 0 (host copies kept for merging)
  std::vector<ElemProblem> eprobs;
  std::vector<ElemTask> etasks;
  long long n_elem = 0;             // ELEM: allowed elements
  int dot_blocks = 0;
  void* d_desc = nullptr;
  int* d_prefix = nullptr;
  int* d_prefix2 = nullptr;
  double* d_partial = nullptr;
  double flops = 0.0;
  std::vector<double> prob_flops;   // per problem (GEMM), for gated accounting
  std::vector<int> prob_inst;
  float tuned_ms = 0.f;
  std::string tag;
  std::vector<Launch> alts;         // GEMM: other descriptor sets of the same contraction (tile
                                    // size, split-K) for the autotuner; emptied once it has chosen
  // Device byte ranges [lo, hi) the launch reads and writes.  `ranged` false: not
  // recorded, and the launch stays ordered against every other one.
  std::vector<std::pair<uintptr_t, uintptr_t>> rd, wr;
  bool ranged = false;
  // algorithmic bytes: each operand element read once, each result element written
  // once (and read where it accumulates), over the allowed elements when blocked
  double bytes = 0.0;
  // SGEMM: host copies of the descriptors, kept until the launch lists are fused
  std::vector<SgemmProblem> sprobs;
  std::vector<SgemmTask> stasks;
  std::vector<SgemmReduce> sreds;
};

struct ProblemRef {
  int inst;
  int node;
  int n;
};

// Conserved momentum of the orbitals of one instance: orbital p has components
// labels[p * dims + c], compared modulo modulus[c] when modulus[c] > 0.
struct InstMomentum {
  int dims = 0;
  std::vector<int> modulus;
  std::vector<int> labels;
};

// (tensor id, problem index, gradient buffer?, elements the executor addresses)
// -> device pointer.  The count is n^rank, or n^(rank-1) for an intermediate the
// executor stores packed (see Executor::packed).
using Binder = std::function<double*(int tensor, int prob, bool grad, size_t count)>;

// Packed storage of momentum-blocked intermediates: when every orbital of an
// instance has its own momentum label, the last index of an allowed element is
// fixed by the others, so an intermediate is stored as n^(rank-1) doubles indexed
// by all but its last axis.  Labels that repeat (several orbitals per momentum)
// keep dense storage.  FTCC_PACK=0 keeps every intermediate dense (diagnostics).
bool labels_distinct(const struct InstMomentum& m);
bool packing_enabled();

struct Scratch {
  std::vector<double*> a, b, c, part;   // per problem: n^4 doubles each
  double* dot_partial = nullptr;        // >= n_prob * 64 doubles
  double* tail_ws = nullptr;            // partial tiles of split GEMM tails, blocked GEMM chunks, blocked dots
  size_t tail_ws_doubles = 0;           // its size (at most kTailWorkspaceDoubles)
};

// HIP-event timing of the dominant kernel (the FP64-MFMA GEMM with 128x128
// tiles, BK 16 or 32): events are recorded around each such launch on the launch
// stream and harvested at the next host synchronisation.
struct KernelProfiler {
  bool enabled = false;
  std::vector<hipEvent_t> ev;   // pairs
  std::vector<double> pending_flops;
  int used = 0;
  double flops = 0.0, seconds = 0.0;
  long launches = 0;
  void reset();
  void record_begin(hipStream_t s);
  void record_end(hipStream_t s, double flops);
  void harvest();               // call after the stream has been synchronised
  ~KernelProfiler();
};

class Executor {
 public:
  Executor() = default;
  ~Executor();
  Executor(const Executor&) = delete;
  Executor& operator=(const Executor&) = delete;

  // const_alloc(inst, count) returns a persistent per-instance buffer for a
  // permuted copy of a constant.  const_grads lists constants whose gradients
  // the backward list must produce.
  // cache_alloc(count) (may be empty) provides buffers for reused permuted copies of
  // value operands, up to cache_budget bytes in total; it may return nullptr (no
  // room), and the operand is then permuted into scratch at each use instead.
  void build(const Program* prog, const std::vector<ProblemRef>& probs, Binder bind, Scratch* scratch,
             std::function<double*(int inst, size_t count)> const_alloc, bool want_backward,
             const std::vector<int>& const_grads, std::function<double*(size_t)> cache_alloc = nullptr,
             size_t cache_budget = 0);

  // Evaluate the constant combinations (derived tensors) with every forward
  // pass instead of once in the set-up, so that the reverse pass carries
  // gradients through them to the raw constants (for the gradient with respect
  // to the integrals).  Call before build().
  void set_inline_setup(bool on) { inline_setup_ = on; }

  // time the candidate GEMM tile configurations of every large GEMM launch and keep the best
  void autotune(hipStream_t s);
  void run_setup(hipStream_t s) const { run(setup_, s); }
  void run_forward(hipStream_t s) const { run(fwd_, s); }
  void run_backward(hipStream_t s) const { run(bwd_, s); }

  void set_profiler(KernelProfiler* p) { prof_ = p; }
  // Per-instance run flags (device int array indexed by instance, read when the
  // kernels run): forward and backward launches of an instance whose flag is 0
  // return at once.  Set before build(); set-up launches are never gated.
  // h_flags mirrors the device flags on the host (flop accounting of the profiler).
  void set_gate(const int* d_flags, const int* h_flags) {
    gate_ = d_flags;
    gate_host_ = h_flags;
  }
  // Momentum labels per instance (indexed by ProblemRef::inst; every instance
  // needs them).  Set before build(): every two-operand contraction is then
  // evaluated over its momentum-allowed blocks only (laws from the Program).
  void set_momentum(const std::vector<const InstMomentum*>& by_instance) { mom_ = by_instance; }
  double sgemm_flops_forward() const;
  // intermediates stored packed (after build)
  int n_packed() const;
  double gemm_flops_forward() const;
  double gemm_flops_backward() const;
  int n_launches_forward() const { return (int)fwd_.size(); }
  // kernel dispatches of one pass of a launch list, and the algorithmic bytes of the forward list
  long dispatches_forward() const { return dispatches(fwd_); }
  long dispatches_backward() const { return dispatches(bwd_); }
  double bytes_forward() const;
  // device bytes taken by the cached permuted copies of value operands and by the
  // permuted copies of constants
  size_t cache_bytes() const { return cache_bytes_; }
  size_t const_copy_bytes() const { return const_bytes_; }

 private:
  using PerProb = std::vector<double*>;
  void run(const std::vector<Launch>& L, hipStream_t s) const;
  long dispatches(const std::vector<Launch>& L) const;
  void contract(std::vector<Launch>& dst, const PerProb& out, const std::string& oi, double alpha,
                const PerProb& A, const std::string& ai, int a_const, const PerProb* B, const std::string& bi,
                int b_const, bool acc, const std::string& tag, int a_val = -1, int b_val = -1, int t_out = -1,
                int t_a = -1, int t_b = -1);
  PerProb value_permuted(std::vector<Launch>& dst, int tensor, const PerProb& X, const std::string& xi,
                         const std::string& yi, const PerProb& scratch, const std::string& tag);
  void perm(std::vector<Launch>& dst, const PerProb& X, const std::string& xi, const PerProb& Y,
            const std::string& yi, double alpha, double beta, const std::vector<const double*>* scale,
            const std::string& tag);
  void fill(std::vector<Launch>& dst, const PerProb& Y, int rank, const std::string& tag, int t_y = -1);
  // full contraction <A, B> over A's momentum-allowed elements
  bool dot_blocked(std::vector<Launch>& dst, const PerProb& A, const std::string& ai, const PerProb& B,
                   const std::string& bi, const PerProb& out, double alpha, double beta, int t_a, int t_b,
                   const std::string& tag);
  // xp / yp >= 0 override the storage (packed or not) of the X / Y side
  bool elem_blocked(std::vector<Launch>& dst, const PerProb& X, const std::string& xi, const PerProb& Y,
                    const std::string& yi, double alpha, double beta, int t_y, int t_x, const std::string& tag,
                    const std::vector<const double*>* scale = nullptr, int xp = -1, int yp = -1);
  PerProb const_permuted(int tensor, const PerProb& X, const std::string& xi, const std::string& yi);
  void* upload(const void* host, size_t bytes);
  void dump_plan() const;

  const Program* prog_ = nullptr;
  std::vector<ProblemRef> probs_;
  Scratch* scratch_ = nullptr;
  bool inline_setup_ = false;
  // consecutive zero fills write disjoint buffers: one launch serves them all
  void merge_fills(std::vector<Launch>& L);
  // Momentum-blocked lists: every launch moves to the earliest dependency level
  // its byte ranges allow, and the blocked contractions (and the blocked
  // elementwise ops) of one level become one launch each.  Every buffer sees its
  // writes in program order, so results are unchanged.
  void fuse_levels(std::vector<Launch>& L);
  Launch merge_sgemm(const std::vector<Launch*>& parts);
  Launch merge_elem(const std::vector<Launch*>& parts);
  void release(const std::vector<void*>& dev);
  std::function<double*(int, size_t)> const_alloc_;
  std::map<std::pair<int, std::string>, PerProb> const_cache_;
  struct CacheEntry {
    PerProb buf;
    int version;
  };
  std::map<std::pair<int, std::string>, CacheEntry> value_cache_;
  std::vector<int> version_;
  std::function<double*(size_t)> cache_alloc_;
  size_t cache_budget_ = 0, cache_bytes_ = 0, const_bytes_ = 0;
  std::vector<Launch> setup_, fwd_, bwd_;
  std::vector<void*> owned_;
  KernelProfiler* prof_ = nullptr;
  const int* gate_ = nullptr;
  const int* gate_host_ = nullptr;
  // momentum blocking
  std::vector<const InstMomentum*> mom_;
  std::vector<std::vector<int>> law_;      // per tensor (empty: no usable law)
  std::vector<char> law_ok_;
  struct GroupTable {
    void* off1 = nullptr;                  // device: element offsets in the first operand
    void* off2 = nullptr;                  // device: element offsets in the second operand
    std::map<long long, std::pair<int, int>> blocks;   // packed momentum -> (first tuple, count)
  };
  std::map<std::string, GroupTable> group_cache_;
  std::map<std::string, const unsigned*> out_tables_;   // output offset tables of GEMMs (device)
  const unsigned* out_offsets(long n, const std::string& letters, const std::string& oi);
  void infer_laws();
  bool contract_blocked(std::vector<Launch>& dst, const PerProb& out, const std::string& oi, double alpha,
                        const PerProb& A, const std::string& ai, const PerProb& B, const std::string& bi, bool acc,
                        const std::string& tag, int t_out, int t_a, int t_b);
  const GroupTable& group_table(int inst, long n, const std::string& letters, const std::string& xi, bool xp,
                                const std::string& yi, bool yp, const std::vector<int>& signs);
  std::vector<char> packed_;               // per tensor: stored packed (n^(rank-1) doubles)
  bool pack_on_ = false;                   // packing applies to this executor's problems
  void plan_packing(bool want_backward);
  // constants (and derived constants) read through packed copies: no gradient asked
  // for them, and every op that reads them lowers to blocked kernels
  std::vector<int> plan_const_packing(const std::vector<int>& const_grads) const;
  // inputs and outputs of rank >= 2 worked on through packed shadows: gathered from
  // their dense buffers at the start of a pass, scattered back at its end
  std::vector<int> plan_io_packing() const;
  bool is_packed(int t) const { return t >= 0 && t < (int)packed_.size() && packed_[t]; }
  size_t elems(int t, long n, int rank) const { return (size_t)ipow_l(n, is_packed(t) ? rank - 1 : rank); }
  static long ipow_l(long n, int r) {
    long v = 1;
    for (int k = 0; k < r; ++k) v *= n;
    return v;
  }
  void dense_guard(const std::string& tag, std::initializer_list<int> ts) const;
  double run_flops(const Launch& l) const;
  GemmTail tail_of(const Launch& l, int cfg) const {
    return plan_gemm_tail(cfg, l.total, l.min_k, l.splitk_blocks > 0, scratch_ ? scratch_->tail_ws : nullptr,
                          scratch_ ? scratch_->tail_ws_doubles : 0);
  }
  const int* gate_for(const std::vector<Launch>& dst, int p) const {
    return (gate_ && &dst != &setup_) ? gate_ + probs_[p].inst : nullptr;
  }
};

}  // namespace ftcc
