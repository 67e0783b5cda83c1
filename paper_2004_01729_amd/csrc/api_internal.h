// Internal interface of the host code behind the C ABI (not part of the ABI):
// the context and per-instance state, and the helpers shared by ftcc_api.hip
// (context, thermal set-up, the integral-form march, Lambda, response),
// rk_march.hip (the differential form) and density.hip (the two-body response
// density).  Every helper takes the context and enqueues work on its stream.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "engine.h"
#include "ftcc.h"
#include "kernels.h"
#include "tau_kernels.h"
#include "util.h"

namespace ftcc {
namespace host {

struct Fail {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

// names of the 4 one-body and 12 two-body weighted blocks
extern const char* kU[4];
extern const char* kG[12];

}  // namespace host
}  // namespace ftcc

// Included only by the three sources above, which name the kernels, the engine
// and these helpers unqualified (never by a public header).
using namespace ftcc;
using namespace ftcc::host;

// ------------------------------------------------------------------ context
// a cached exponential-sum launch of the Simpson integral form: problems, block
// prefix and terms in one device buffer
struct SpLaunch {
  char* buf = nullptr;
  int n_prob = 0;
  int blocks = 0;
};

struct Instance {
  int n = 0;
  bool has_ham = false;
  double mu = 0.0, beta = 1.0;
  double *h = nullptr, *eri = nullptr, *eps = nullptr;
  std::vector<double> eps_host;
  InstMomentum mom;                // dims == 0: no momentum labels
  unsigned* d_allowed[2] = {nullptr, nullptr};   // momentum-allowed elements of the t1 / t2 segments
  long n_allowed[2] = {0, 0};
  int* d_labels = nullptr;         // device copies for the conservation checks
  int* d_modulus = nullptr;
  double *occ = nullptr, *wo = nullptr, *wv = nullptr, *fock = nullptr;
  double *dn = nullptr, *dwo = nullptr, *dwv = nullptr, *du_raw = nullptr, *u_raw = nullptr;
  std::map<std::string, double*> blk, dblk;
  std::vector<double*> grid, resid, sb, lam, abuf;
  double* mf = nullptr;          // meanfield outputs (5)
  double* acc = nullptr;         // response accumulators: [0] mu, [1] beta, [2] theta, [3] beta grid
  std::vector<double> energies;  // per node
  double omega0 = 0, omega1 = 0, omega_cc = 0;
  int iters = 0, status = 0, lam_iters = 0, lam_status = 0;
  double* ugrad_acc[4] = {nullptr, nullptr, nullptr, nullptr};
  double* rk_tmp[2] = {nullptr, nullptr};   // differential form: reverse-pass temporaries
  double* gacc[12] = {};                    // two-body density: accumulated gradients of the 12 weighted blocks
  double* rk_hbar = nullptr;                // d Omega_CC / d(step) at fixed integrals
  // orbital-energy response (allocated on first request): per-orbital accumulators of
  // the thermal-integral part, dL/dDelta of every amplitude element, the direction
  // du = -e_q e_q^T and the assembled vector
  double *deps_acc = nullptr, *deps_delta = nullptr, *deps_dh = nullptr, *deps_out = nullptr;
};

struct ftcc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  ftcc_options opt;
  int B = 0, m = 4, P = 4;
  PanelRule rule;
  PanelRule* d_rule = nullptr;
  std::vector<Instance> inst;
  std::vector<void*> allocs;
  Program prog;
  std::unique_ptr<Executor> ex_main, ex_d, ex_g;   // ex_g: integral gradients (built on first use)
  std::map<std::pair<int, int>, double*> g_derived, g_cgrad;   // (tensor, problem) buffers of ex_g
  bool built = false, solved = false, have_lambda = false;
  // per node (instance * m + x): amplitudes, residuals, energies, gradients, cotangents
  std::vector<double*> amp, S, e, gr, cot, ebar, dS, de;
  // per executor slot (instance * slots + slot); the same pointers as the node
  // buffers when every node of a panel has its own slot (slots == m)
  int slots = 0;
  std::vector<double*> s_amp, s_S, s_e, s_gr, s_cot, s_ebar, s_dS, s_de;
  std::vector<std::array<double*, 4>> s_ugrad;
  std::map<std::pair<int, int>, double*> inter, inter_grad, dderived;   // (tensor, problem) / (tensor, inst)
  std::map<const double*, long> buf_elems;    // element counts of the buffers above (shared by executors)
  // grouped response accumulation (built on first use): one dot per (instance,
  // node) into resp_vals, the node sums per instance in node order
  DotProblem* d_resp_dots = nullptr;
  double* d_resp_vals = nullptr;
  double* d_resp_w = nullptr;                 // [m] (1/beta) g_x
  const double** d_de_ptrs = nullptr;         // [B m] derivative energies of the nodes
  double** d_acc_ptrs = nullptr;              // [B] response accumulators
  const double** d_ug_src = nullptr;          // [B 4 m] one-body gradients of the nodes
  double** d_ug_dst = nullptr;                // [B 4] their accumulators
  long* d_n2 = nullptr;                       // [B] n^2
  long max_n2 = 0;
  std::map<std::pair<int, int>, double*> derived;
  std::vector<std::array<double*, 4>> ugrad;
  Scratch scratch;
  unsigned long long* d_maxbits = nullptr;    // [B][2]
  double* d_partial = nullptr;                // TAU_BETA partial sums
  std::vector<int> tau_prefix_host;
  int* d_active = nullptr;                    // [B] propagator step flags
  int* d_run = nullptr;                       // [B] residual-program run flags (executor gate)
  std::vector<int> run_host;                  // host copy of d_run
  KernelProfiler prof;
  hipGraphExec_t g_fwd = nullptr, g_bwd = nullptr;
  std::vector<int> beta_part_off;             // first TAU_BETA partial of each instance
  std::vector<int> active_host;               // per-instance "still iterating" flags
  std::map<std::pair<int, int>, std::pair<TauProblem*, int*>> tau_cache;
  std::map<std::pair<int, int>, std::pair<int, int>> tau_shape;   // (n_prob, blocks)
  // DIIS state: per instance `depth` stored iterates X and residuals R (m * len each)
  std::vector<std::vector<double*>> diis_X, diis_R;
  std::vector<int> diis_count, diis_next;
  double* d_gram = nullptr;     // [B][D][D]
  double* d_coef = nullptr;     // [B][D]
  int* d_dcount = nullptr;      // [B]
  int* d_dnewest = nullptr;     // [B]
  long resid_evals = 0, vjp_evals = 0;
  double t_solve = 0.0, t_lambda = 0.0;
  size_t bytes = 0;
  // differential form (propagator >= 2): explicit Runge-Kutta with m = stages,
  // P = n_tau steps; tableau a (row-major m x m, strictly lower) and b
  bool rk = false;
  bool simpson = false;                       // propagator 5: the Simpson integral form (m = 1, P = n_tau)
  std::map<long, SpLaunch> sp_cache;          // its exponential-sum descriptor sets (until the next solve)
  double gdeg = 2.0;                          // electrons per orbital and occupation: 2 restricted, 1 spin orbitals
  std::vector<double> rk_a, rk_b;
  double* d_rkw = nullptr;                    // [P + 1] Simpson weight / beta of each grid point
  int* d_bad = nullptr;                       // flag of the conservation-law checks
  std::map<std::tuple<int, int, int>, std::pair<RKProblem*, int*>> rk_cache;
  std::map<std::tuple<int, int, int>, int> rk_blocks;
  std::map<std::tuple<int, int, int>, DotProblem*> rk_dots;
  ftcc_alloc_fn ualloc = nullptr;   // caller's device memory supplier (or hipMalloc)
  ftcc_free_fn ufree = nullptr;
  void* uuser = nullptr;

  double* dalloc(size_t count) {
    void* p = nullptr;
    // 256-byte granules keep every buffer aligned for 16-byte vector loads
    const size_t nb = (std::max<size_t>(count, 1) * sizeof(double) + 255) / 256 * 256;
    if (opt.mem_cap_bytes && bytes + nb > opt.mem_cap_bytes)
      fail(FTCC_ENOMEM, "allocation of " + std::to_string(nb) + " bytes would exceed mem_cap_bytes (" +
                            std::to_string(bytes) + " bytes already held)");
    if (ualloc) {
      p = ualloc(nb, uuser);
      if (!p) fail(FTCC_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(nb) + " bytes");
    } else if (hipMalloc(&p, nb) != hipSuccess) {
      (void)hipGetLastError();
      fail(FTCC_ENOMEM, "hipMalloc of " + std::to_string(nb) + " bytes failed (" + std::to_string(bytes) +
                            " bytes already held)");
    }
    // every buffer starts zeroed: momentum-blocked contractions write only the
    // allowed blocks of their outputs and rely on the forbidden elements being 0
    if (hipMemset(p, 0, nb) != hipSuccess) fail(FTCC_EDEVICE, "hipMemset of a new buffer failed");
    bytes += nb;
    allocs.push_back(p);
    return (double*)p;
  }

  // device memory this context may still take: free memory, bounded by the cap
  double available() {
    size_t free_b = 0, total_b = 0;
    FTCC_HIP(hipMemGetInfo(&free_b, &total_b));
    double a = (double)free_b;
    if (opt.mem_cap_bytes) a = std::min(a, (double)opt.mem_cap_bytes - (double)bytes);
    return std::max(a, 0.0);
  }
};

namespace ftcc {
namespace host {

// Divergence of the fixed-point sweeps of one panel: the max |change| of an
// instance grew in kDivergeSweeps consecutive sweeps and stands more than
// kDivergeFactor above the smallest change of the panel so far (a converging
// iteration, DIIS-accelerated or not, does not grow that long).
constexpr int kDivergeSweeps = 8;
constexpr double kDivergeFactor = 1e4;
struct DivergenceWatch {
  int grew = 0;
  double prev = INFINITY, low = INFINITY;
  bool diverged(double chg) {
    grew = chg > prev ? grew + 1 : 0;
    prev = chg;
    low = std::min(low, chg);
    return grew >= kDivergeSweeps && chg > kDivergeFactor * low;
  }
};

// one exponential-sum launch of the Simpson integral form, per instance: out =
// x0 * base + (prod ? prod : 1) * sum of terms (X, C, k); see ExpSumProblem
struct ExpSpec {
  int mode = 0;
  const double* base = nullptr;
  double x0 = 0.0;
  const double* prod = nullptr;
  std::vector<std::tuple<const double*, double, double>> terms;
  double* out = nullptr;
  bool track = false;
};

// buffer of node x of an instance (DIIS histories)
using NodeBufs = std::function<double*(int inst, int x)>;

// one Runge-Kutta combination of the differential form: out = x0 * base +
// sum_l coef[l] * (-Delta Y_l + sigma S_l) over the stage buffers Y_l, S_l
struct RKSpec {
  const double* base = nullptr;
  double x0 = 0.0;
  int nst = 0;
  double coef[kMaxStages] = {0.0, 0.0, 0.0, 0.0};
  const double* Y[kMaxStages] = {nullptr, nullptr, nullptr, nullptr};
  const double* S[kMaxStages] = {nullptr, nullptr, nullptr, nullptr};
  double* out = nullptr;
};

// ftcc_api.hip: context, thermal set-up, the integral-form march, DIIS
long ipow(long n, int r);
int run_guarded(const std::function<void()>& f);
bool trace_on();
// the buffer of (t, key) in `store`, allocated with `count` elements on first use;
// a later request for more elements than it holds is an error (executors that
// share intermediates must agree on their storage)
double* shared_buf(ftcc_ctx* c, std::map<std::pair<int, int>, double*>& store, int t, int key, long count);
// FTCC_TRACE=2: a line per sweep as well (the largest change over the batch)
void trace_sweep(const char* phase, int panel, int it, const std::vector<double>& maxbits);
void trace(ftcc_ctx* c, const char* phase, int panel, int n_panels, const std::vector<int>& sweeps,
           std::chrono::steady_clock::time_point t0);
void trace_mem(ftcc_ctx* c, const char* stage);
void trace_executor(ftcc_ctx* c, const char* which, const Executor& ex);
void sync(ftcc_ctx* c);
void thermal_setup(ftcc_ctx* c, int i);
void deriv_setup(ftcc_ctx* c, int i, int which, const double* d_dh, const double* d_deri);
void deriv_setup_eps(ftcc_ctx* c, int i, int q);
long node_len_of(long n);
void check_momentum(ftcc_ctx* c, int i, const double* x, int rank, const char* what);
bool momentum_on(const ftcc_ctx* c);
void allowed_elements(ftcc_ctx* c, int i);
long seg_len(const ftcc_ctx* c, int i, int seg);
void build(ftcc_ctx* c);
long n_running(ftcc_ctx* c);
void run_fwd_slots(ftcc_ctx* c);
void run_bwd_slots(ftcc_ctx* c);
long node_len(ftcc_ctx* c, int i);
void dcopy(ftcc_ctx* c, double* dst, const double* src, long count);
void node_copy(ftcc_ctx* c, int i, double* dst, const double* src);
void forward(ftcc_ctx* c);
void backward(ftcc_ctx* c);
void d_forward(ftcc_ctx* c);
void clear_tau_cache(ftcc_ctx* c);
int tau_problems(ftcc_ctx* c, int mode, int panel, double* partial_base, std::vector<TauProblem>& ps,
                 std::vector<int>& prefix);
void tau_run(ftcc_ctx* c, int mode, int panel);
void set_active(ftcc_ctx* c, const std::vector<bool>& active);
void set_run(ftcc_ctx* c, const std::vector<bool>& run);
void run_all(ftcc_ctx* c);
void reset_maxbits(ftcc_ctx* c);
std::vector<double> read_maxbits(ftcc_ctx* c);
void copy_d(ftcc_ctx* c, double* dst, const double* src, long count);
void zero_d(ftcc_ctx* c, double* dst, long count);
void diis_reset(ftcc_ctx* c);
void diis_before(ftcc_ctx* c, const NodeBufs& it, const std::vector<bool>& active);
void diis_after(ftcc_ctx* c, const NodeBufs& it, const std::vector<bool>& active);
std::vector<int> panel_solve(ftcc_ctx* c, int panel, std::vector<int>& status);
void load_panel(ftcc_ctx* c, int p);

// rk_march.hip: the differential form
void forward_one(ftcc_ctx* c, int x);
void backward_one(ftcc_ctx* c, int x);
void d_forward_one(ftcc_ctx* c, int x);
void rk_combine(ftcc_ctx* c, int kind, int p, int x, double sigma, bool track,
                const std::function<RKSpec(int)>& spec);
void rk_dot(ftcc_ctx* c, int kind, int p, int x, const std::function<std::array<const double*, 3>(int)>& xyz);
double rk_h(const ftcc_ctx* c, int i);
double rk_a(const ftcc_ctx* c, int j, int l);
void rk_stage_state(ftcc_ctx* c, int p, int x);
void rk_recompute_stages(ftcc_ctx* c, int p);
void set_ebar(ftcc_ctx* c, int x, int grid_point);
void rk_solve(ftcc_ctx* c, std::vector<int>& status);
void rk_lambda(ftcc_ctx* c, std::vector<int>& status);

// simpson_march.hip: the implicit integral form generated by Simpson's rule
std::vector<double> simpson_row(int y);
void expsum_run(ftcc_ctx* c, long key, const std::function<ExpSpec(int)>& spec);
void simpson_solve(ftcc_ctx* c, std::vector<int>& status, std::vector<int>& total);
void simpson_lambda(ftcc_ctx* c, std::vector<int>& status, std::vector<int>& total);
void simpson_lamt(ftcc_ctx* c, int x);
void simpson_grid_term(ftcc_ctx* c, int y, int mode, const std::function<double*(int)>& out,
                       const std::function<const double*(int)>& prod);

// noalloc.hip: the fixed device scratch of the allocation-free entry point
void noalloc_setup(int device);

// density.hip: the two-body response density
void build_gamma_executor(ftcc_ctx* c);
void gamma_pass(ftcc_ctx* c);
void gamma_node(ftcc_ctx* c, int x);

}  // namespace host
}  // namespace ftcc
