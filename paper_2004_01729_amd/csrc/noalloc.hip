// Allocation-free variant of the response derivatives dOmega/dmu and dOmega/dbeta
// (ftcc_response_noalloc): every launch descriptor and partial sum of the call
// lives in one fixed device array of this file instead of memory the call would
// allocate, for callers that cannot allocate device memory.
#include <mutex>

#include "api_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;   // 4 MiB per device, held until the process ends

// Device scratch of ftcc_response_noalloc.  Host code never passes this name to a
// kernel or a copy (on the host it only stands in for the symbol): it uses the
// device address that noalloc_setup resolved for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::map<int, unsigned char*> g_scratch;   // device -> address of `scratch` on that device

unsigned char* scratch_on(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_scratch.find(device);
  return it == g_scratch.end() ? nullptr : it->second;
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

namespace ftcc {
namespace host {

// Resolves the scratch array's address on `device` (which must be current);
// once per device, from ftcc_create.
void noalloc_setup(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch.count(device)) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    fail(FTCC_EDEVICE, std::string("hipGetSymbolAddress of the response scratch failed: ") + hipGetErrorString(e));
  }
  g_scratch[device] = (unsigned char*)p;
}

}  // namespace host
}  // namespace ftcc

extern "C" {

int ftcc_response_noalloc(ftcc_ctx* c, double* dO_dmu, double* dO_dbeta) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    if (!c->have_lambda) fail(FTCC_ESTATE, "call ftcc_lambda first");
    if (c->rk || c->simpson)
      fail(FTCC_EINVAL, "ftcc_response_noalloc covers the Gauss-Legendre integral form (propagators 0 and 1)");
    FTCC_HIP(hipSetDevice(c->device));
    unsigned char* base = scratch_on(c->device);
    if (!base) fail(FTCC_ESTATE, "the response scratch of this device was not set up");
    const int B = c->B, m = c->m, P = c->P;
    if (c->opt.checkpoint)   // panels are recomputed through the march's own propagator descriptors
      for (int p = 0; p < P; ++p)
        for (int mode : {TAU_INIT, TAU_STEP, TAU_END})
          if (!c->tau_cache.count(std::make_pair(mode, p)))
            fail(FTCC_ESTATE, "the checkpointed march's propagator descriptors are missing (solve and lambda first)");

    // layout of the scratch: propagator descriptors and their block prefix, the dot
    // descriptors of one accumulation, the dot partial sums, the TAU_BETA partial sums
    std::vector<TauProblem> ps;
    std::vector<int> prefix;
    long beta_blocks = 0;   // TAU_BETA partial sums: one per 1024 elements of every segment
    for (int i = 0; i < B; ++i) beta_blocks += (seg_len(c, i, 0) + 1023) / 1024 + (seg_len(c, i, 1) + 1023) / 1024;
    const size_t n_tau = 2 * (size_t)B;   // two amplitude segments per instance
    const size_t off_tau = 0;
    const size_t off_pre = off_tau + align256(n_tau * sizeof(TauProblem));
    const size_t off_dot = off_pre + align256(n_tau * sizeof(int));
    const size_t off_dpart = off_dot + align256((size_t)B * m * sizeof(DotProblem));
    const size_t off_bpart = off_dpart + align256(64 * sizeof(double));
    const size_t need = off_bpart + align256((size_t)beta_blocks * sizeof(double));
    if (need > kScratchBytes)
      fail(FTCC_EINVAL, "this context needs " + std::to_string(need) + " bytes of response scratch; the fixed array " +
                            "holds " + std::to_string(kScratchBytes) + " (use ftcc_response)");
    double* bpart = (double*)(base + off_bpart);
    double* dpart = (double*)(base + off_dpart);
    TauProblem* d_tau = (TauProblem*)(base + off_tau);
    int* d_pre = (int*)(base + off_pre);
    DotProblem* d_dot = (DotProblem*)(base + off_dot);

    // host sources of the staged copies stay alive until the final synchronisation
    std::vector<std::vector<char>> keep;
    auto stage = [&](void* dst, const void* src, size_t bytes) {
      keep.emplace_back((const char*)src, (const char*)src + bytes);
      FTCC_HIP(hipMemcpyAsync(dst, keep.back().data(), bytes, hipMemcpyHostToDevice, c->stream));
    };
    auto propagate = [&](int mode, int p) {   // one propagator launch with staged descriptors
      const int total = tau_problems(c, mode, p, bpart, ps, prefix);
      stage(d_tau, ps.data(), ps.size() * sizeof(TauProblem));
      stage(d_pre, prefix.data(), prefix.size() * sizeof(int));
      launch_tau(c->d_rule, m, mode, d_tau, d_pre, (int)ps.size(), total, c->stream);
      FTCC_HIP(hipGetLastError());
    };

    for (int i = 0; i < B; ++i) zero_d(c, c->inst[i].acc, 8);
    for (int p = 0; p < P; ++p) {
      load_panel(c, p);
      propagate(TAU_LAMT, p);   // lambda-tilde of the panel into the cotangent slots
      if (dO_dbeta) {           // explicit beta dependence of the propagator weights
        propagate(TAU_BETA, p);
        for (int i = 0; i < B; ++i) {
          const int nb = (int)((seg_len(c, i, 0) + 1023) / 1024 + (seg_len(c, i, 1) + 1023) / 1024);
          launch_sum(bpart + prefix[2 * i], nb, c->inst[i].acc + 4, c->stream);
          launch_axpby(1, 1.0 / P, c->inst[i].acc + 4, 1.0, c->inst[i].acc + 3, c->stream);
        }
      }
      for (int which = 0; which < 2; ++which) {
        if ((which == 0 && !dO_dmu) || (which == 1 && !dO_dbeta)) continue;
        for (int i = 0; i < B; ++i) deriv_setup(c, i, which, nullptr, nullptr);
        c->ex_d->run_setup(c->stream);
        d_forward(c);
        // <lamt_x, dS_x> + (g_x / beta) dE_x into acc[which], one problem at a time
        std::vector<DotProblem> ds;
        for (int i = 0; i < B; ++i)
          for (int x = 0; x < m; ++x) {
            const Instance& I = c->inst[i];
            const long n = I.n;
            DotProblem d{};
            d.X = c->cot[i * m + x];
            d.Y = c->dS[i * m + x];
            d.out = I.acc + which;
            d.len = n * n + n * n * n * n;
            if (I.d_allowed[0]) {
              d.ia = I.d_allowed[0];
              d.na = I.n_allowed[0];
              d.ib = I.d_allowed[1];
              d.nb = I.n_allowed[1];
              d.second = n * n;
            }
            d.alpha = 1.0;
            d.beta = 1.0;
            ds.push_back(d);
          }
        stage(d_dot, ds.data(), ds.size() * sizeof(DotProblem));
        for (size_t k = 0; k < ds.size(); ++k) launch_dot(d_dot + k, 1, 64, dpart, c->stream);
        for (int i = 0; i < B; ++i)
          for (int x = 0; x < m; ++x)
            launch_axpby(1, c->rule.b[x] / P, c->de[i * m + x], 1.0, c->inst[i].acc + which, c->stream);
      }
    }
    run_all(c);
    std::vector<double> accs(8 * (size_t)B), mfv(5 * (size_t)B);
    for (int i = 0; i < B; ++i) {
      FTCC_HIP(hipMemcpyAsync(&mfv[5 * i], c->inst[i].mf, sizeof(double) * 5, hipMemcpyDeviceToHost, c->stream));
      FTCC_HIP(hipMemcpyAsync(&accs[8 * i], c->inst[i].acc, sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
    }
    sync(c);
    for (int i = 0; i < B; ++i) {
      if (dO_dmu) dO_dmu[i] = mfv[5 * i + 2] + accs[8 * i + 0];
      if (dO_dbeta) dO_dbeta[i] = mfv[5 * i + 3] + accs[8 * i + 1] + accs[8 * i + 3];
    }
  });
}

}  // extern "C"
