// C ABI of the FT-CCSD hot path: context, thermal set-up, forward march,
// Lambda adjoint and response derivatives (the differential form's march is in
// rk_march.hip, the two-body response density in density.hip; the shared state
// and helpers in api_internal.h).  All arithmetic runs in the HIP kernels of this
// directory; the host only sequences launches and tests the convergence flags.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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
#include "api_internal.h"

namespace {

thread_local std::string g_err;

// ------------------------------------------------------------------ mean-field kernel
// out[0] Omega_0, out[1] Omega_1, out[2] d(Omega_0+Omega_1)/dmu, out[3] .../dbeta,
// out[4] dOmega_1/dtheta for the direction (dh, deri) at frozen occupations.
// g = electrons per orbital and occupation (2 spatial restricted, 1 spin orbitals):
//   Omega_0 = -(g/beta) sum ln(1 + e^{-beta(eps-mu)}),
//   Omega_1 = g sum (h_pp - eps_p) n_p + (g/2) sum_pq (g <pq|pq> - <pq|qp>) n_p n_q.
__global__ void meanfield_kernel(int n, const double* eps, const double* h, const double* eri, const double* occ,
                                 const double* fock, double mu, double beta, const double* dh, const double* deri,
                                 double g, double* out) {
  __shared__ double red[5][256];
  double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
  const long nn = (long)n * n;
  for (long e = threadIdx.x; e < nn; e += blockDim.x) {
    const int p = (int)(e / n), q = (int)(e % n);
    const double gd = eri[(((long)p * n + q) * n + p) * n + q];   // <pq|pq>
    const double gx = eri[(((long)p * n + q) * n + q) * n + p];   // <pq|qp>
    a1 += 0.5 * g * (g * gd - gx) * occ[p] * occ[q];
    if (deri) {
      const double dd = deri[(((long)p * n + q) * n + p) * n + q];
      const double dx = deri[(((long)p * n + q) * n + q) * n + p];
      a4 += 0.5 * g * (g * dd - dx) * occ[p] * occ[q];
    }
  }
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const double x = beta * (eps[p] - mu);
    const double sp = (x > 0.0) ? log1p(exp(-x)) : (-x + log1p(exp(x)));   // ln(1 + e^-x)
    const double nocc = occ[p], nvir = 1.0 - occ[p];
    a0 += sp;
    a1 += g * (h[(long)p * n + p] - eps[p]) * nocc;
    const double fq = fock[(long)p * n + p] - eps[p];
    const double nn1 = (x > 0.0) ? nocc * (1.0 / (1.0 + exp(-x))) : nocc * (exp(x) / (1.0 + exp(x)));
    (void)nvir;
    // d(Omega_0)/dmu = -g n ; d(Omega_1)/dmu = g (f_qq - eps_q) beta n (1-n)
    a2 += -g * nocc + g * fq * beta * nn1;
    // d(Omega_0)/dbeta = -Omega_0/beta + g (eps - mu) n / beta ; d(Omega_1)/dbeta = g fq (-(eps-mu) n(1-n))
    a3 += g * (eps[p] - mu) * nocc / beta - g * fq * (eps[p] - mu) * nn1;
    if (dh) a4 += g * dh[(long)p * n + p] * nocc;
  }
  red[0][threadIdx.x] = a0;
  red[1][threadIdx.x] = a1;
  red[2][threadIdx.x] = a2;
  red[3][threadIdx.x] = a3;
  red[4][threadIdx.x] = a4;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double om0 = -g * red[0][0] / beta;
    out[0] = om0;
    out[1] = red[1][0];
    out[2] = red[2][0];
    out[3] = red[3][0] - om0 / beta;
    out[4] = red[4][0];
  }
}

// dn/dmu = beta n (1-n), dn/dbeta = -(eps - mu) n (1-n); dw = dn / (2 w) on kept slots
__global__ void occ_deriv_kernel(int n, const double* eps, const double* occ, const double* wo, const double* wv,
                                 double mu, double beta, int which, double* dn, double* dwo, double* dwv) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const double x = beta * (eps[p] - mu);
  const double nvir = (x > 0.0) ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x));
  const double nn1 = occ[p] * nvir;
  const double d = (which == 0) ? beta * nn1 : -(eps[p] - mu) * nn1;
  dn[p] = d;
  dwo[p] = (wo[p] > 0.0) ? d / (2.0 * wo[p]) : 0.0;
  dwv[p] = (wv[p] > 0.0) ? -d / (2.0 * wv[p]) : 0.0;
}

// dO/dh_pq = g n_p delta_pq + sum_XY w^X_p w^Y_q G^XY_pq
__global__ void dh_assemble_kernel(int n, const double* occ, const double* wo, const double* wv, const double* goo,
                                   const double* gov, const double* gvo, const double* gvv, double g, double* out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int p = (int)(e / n), q = (int)(e % n);
  double v = (p == q) ? g * occ[p] : 0.0;
  v += wo[p] * wo[q] * goo[e] + wo[p] * wv[q] * gov[e] + wv[p] * wo[q] * gvo[e] + wv[p] * wv[q] * gvv[e];
  out[e] = v;
}

// Direction of the orbital energy eps_q at a frozen reference: dn_p = dn_p/deps_q =
// -beta n_q (1 - n_q) delta_pq (the weights follow, dw = dn / (2 w) on kept slots),
// and the explicit dependence of u = f - diag(eps): du = -e_q e_q^T (in dh).
__global__ void occ_deriv_eps_kernel(int n, int q, const double* eps, const double* occ, const double* wo,
                                     const double* wv, double mu, double beta, double* dn, double* dwo, double* dwv,
                                     double* dh) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)n * n) dh[e] = (e == (long)q * n + q) ? -1.0 : 0.0;
  if (e >= n) return;
  const int p = (int)e;
  double d = 0.0;
  if (p == q) {
    const double x = beta * (eps[p] - mu);
    const double nvir = (x > 0.0) ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x));
    d = -beta * occ[p] * nvir;
  }
  dn[p] = d;
  dwo[p] = (wo[p] > 0.0) ? d / (2.0 * wo[p]) : 0.0;
  dwv[p] = (wv[p] > 0.0) ? -d / (2.0 * wv[p]) : 0.0;
}

// Mean-field part of dOmega/deps_q: Omega_0 gives g n_q and the explicit -eps_q n_q of
// Omega_1 gives -g n_q (they cancel); what remains is Omega_1 through the occupation,
// g (f_qq - eps_q) dn_q/deps_q = -g (f_qq - eps_q) beta n_q (1 - n_q).
__global__ void deps_meanfield_kernel(int n, const double* eps, const double* occ, const double* fock, double mu,
                                      double beta, double g, double* out) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const double x = beta * (eps[q] - mu);
  const double nvir = (x > 0.0) ? 1.0 / (1.0 + exp(-x)) : exp(x) / (1.0 + exp(x));
  out[q] = -g * (fock[(long)q * n + q] - eps[q]) * beta * occ[q] * nvir;
}

// out[q] += sum over the amplitude elements of D[e] dDelta_e/deps_q (Delta_i^a = eps_a - eps_i
// on t1[i][a], Delta_ij^ab = eps_a + eps_b - eps_i - eps_j on t2[i][j][a][b]); D is one node
// state (t1 block, then t2 block).  One block per orbital, fixed summation order.
__global__ void __launch_bounds__(256) deps_reduce_kernel(int n, const double* __restrict__ D, double* out) {
  const int q = blockIdx.x;
  const long n2 = (long)n * n, n3 = n2 * n;
  const double* t2 = D + n2;
  double acc = 0.0;
  for (long r = threadIdx.x; r < n; r += blockDim.x) acc += D[r * n + q] - D[(long)q * n + r];
  for (long r = threadIdx.x; r < n3; r += blockDim.x) {
    // r enumerates the other three indices of each slot in row-major order
    const long hi = r / n2, mid = (r / n) % n, lo = r % n;
    acc -= t2[(long)q * n3 + r];                                // i = q
    acc -= t2[hi * n3 + (long)q * n2 + mid * n + lo];           // j = q
    acc += t2[hi * n3 + mid * n2 + (long)q * n + lo];           // a = q
    acc += t2[hi * n3 + mid * n2 + lo * n + q];                 // b = q
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[q] += red[0];
}

// y[e] += a[e] * b[e]
__global__ void mul_acc_kernel(long len, const double* a, const double* b, double* y) {
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < len; e += (long)gridDim.x * blockDim.x)
    y[e] += a[e] * b[e];
}

// Elements of a one-body (rank 2, law k_p = k_q) or two-body (rank 4,
// k_p + k_q = k_r + k_s) array that are nonzero although momentum forbids them;
// any such element sets *bad (plain stores of the same value).
__global__ void momentum_check_kernel(int n, int rank, int dims, const int* __restrict__ labels,
                                      const int* __restrict__ modulus, const double* __restrict__ x, int* bad) {
  const long total = rank == 2 ? (long)n * n : (long)n * n * n * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    if (x[e] == 0.0) continue;
    long r = e;
    int idx[4];
    for (int a = rank - 1; a >= 0; --a) {
      idx[a] = (int)(r % n);
      r /= n;
    }
    bool ok = true;
    for (int c = 0; c < dims; ++c) {
      int q = rank == 2 ? labels[idx[0] * dims + c] - labels[idx[1] * dims + c]
                        : labels[idx[0] * dims + c] + labels[idx[1] * dims + c] - labels[idx[2] * dims + c] -
                              labels[idx[3] * dims + c];
      if (modulus[c] > 0) q %= modulus[c];
      ok = ok && q == 0;
    }
    if (!ok) *bad = 1;
  }
}

// One-body gradients of every node added into the instance accumulators, node
// by node in order (the sums of one add per node): block row = (instance, block).
__global__ void ugrad_sum_kernel(int m, const double* const* src, double* const* dst, const long* n2) {
  const int ik = blockIdx.y;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2[ik / 4]) return;
  double v = dst[ik][e];
  for (int x = 0; x < m; ++x) v = src[(size_t)ik * m + x][e] + v;
  dst[ik][e] = v;
}

// acc[i] += the node dots of instance i in node order, then (1/beta) g_x dE_x
// in node order (the sums the per-node dots and adds gave)
__global__ void resp_combine_kernel(int B, int m, const double* vals, const double* const* de, const double* w,
                                    double* const* acc, int slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  double s = acc[i][slot];
  for (int x = 0; x < m; ++x) s = vals[i * m + x] + s;
  for (int x = 0; x < m; ++x) s = w[x] * de[i * m + x][0] + s;
  acc[i][slot] = s;
}

__global__ void zero_u64_kernel(unsigned long long* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0ull;
}

}  // namespace

namespace ftcc {
namespace host {

[[noreturn]] void fail(int code, const std::string& msg) { throw Fail{code, msg}; }

const char* kU[4] = {"u_oo", "u_ov", "u_vo", "u_vv"};
const char* kG[12] = {"g_oooo", "g_ooov", "g_oovo", "g_oovv", "g_ovov", "g_ovvo",
                      "g_ovvv", "g_vovv", "g_vvvv", "g_vvvo", "g_ovoo", "g_vvoo"};

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_m)
void gauss_legendre(int m, double* c, double* b) {
  for (int i = 0; i < m; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= m; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pm = (m == 1) ? x : p1;
      double pm1 = (m == 1) ? 1.0 : p0;
      double dp = m * (x * pm - pm1) / (x * x - 1.0);
      double dx = pm / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= m; ++k) {
      double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pm = (m == 1) ? x : p1, pm1 = (m == 1) ? 1.0 : p0;
    double dp = m * (x * pm - pm1) / (x * x - 1.0);
    c[m - 1 - i] = 0.5 * (x + 1.0);
    b[m - 1 - i] = 1.0 / ((1.0 - x * x) * dp * dp);   // 2/((1-x^2)P'^2) on [-1,1], halved
  }
}

PanelRule make_rule(int m, int lawson) {
  PanelRule R;
  std::memset(&R, 0, sizeof(R));
  R.m = m;
  R.lawson = lawson;
  gauss_legendre(m, R.c, R.b);
  for (int y = 0; y < m; ++y) {
    // l_y(u) = prod_{j != y} (u - c_j) / (c_y - c_j) as monomial coefficients
    double poly[kMaxNodes + 1] = {0};
    poly[0] = 1.0;
    int deg = 0;
    for (int j = 0; j < m; ++j) {
      if (j == y) continue;
      const double den = R.c[y] - R.c[j];
      double nw[kMaxNodes + 1] = {0};
      for (int k = 0; k <= deg; ++k) {
        nw[k + 1] += poly[k] / den;
        nw[k] -= poly[k] * R.c[j] / den;
      }
      ++deg;
      std::memcpy(poly, nw, sizeof(nw));
    }
    for (int k = 0; k < m; ++k) R.lc[y][k] = poly[k];
  }
  for (int x = 0; x < m; ++x)
    for (int y = 0; y < m; ++y) {
      double a = 0.0, p = R.c[x];
      for (int k = 0; k < m; ++k) {
        a += R.lc[y][k] * p / (k + 1);
        p *= R.c[x];
      }
      R.A[x][y] = a;
    }
  for (int x = 0; x <= m; ++x) {
    const double cx = (x < m) ? R.c[x] : 1.0;
    for (int y = 0; y < m; ++y) {
      double p = cx, f = 1.0;   // c_x^(k+1), k!
      for (int k = 0; k < m; ++k) {
        R.gc[x][y][k] = R.lc[y][k] * p * f;
        p *= cx;
        f *= (k + 1);
      }
    }
  }
  return R;
}

long ipow(long n, int r) {
  long v = 1;
  for (int k = 0; k < r; ++k) v *= n;
  return v;
}

int run_guarded(const std::function<void()>& f) {
  try {
    f();
    return FTCC_OK;
  } catch (const Fail& e) {
    g_err = e.msg;
    return e.code;
  } catch (const HipError& e) {
    g_err = e.what();
    return FTCC_EDEVICE;
  } catch (const std::exception& e) {
    g_err = e.what();
    return FTCC_EINVAL;
  }
}

// A device buffer shared by the executors under (kind t, key): allocated on first
// request, checked against the size of every later request.
double* shared_buf(ftcc_ctx* c, std::map<std::pair<int, int>, double*>& store, int t, int key, long count) {
  auto k = std::make_pair(t, key);
  auto it = store.find(k);
  if (it != store.end()) {
    if (c->buf_elems[it->second] < count)
      fail(FTCC_EINVAL, "an executor asked for " + std::to_string(count) + " elements of a shared buffer of " +
                            std::to_string(c->buf_elems[it->second]));
    return it->second;
  }
  double* p = c->dalloc(count);
  store[k] = p;
  c->buf_elems[p] = count;
  return p;
}

// Progress lines on stderr (one per panel of each phase, and one per sweep at
// level 2) when FTCC_TRACE is set: large instances spend minutes per phase.
static int trace_level() {
  static const int lv = [] {
    const char* e = std::getenv("FTCC_TRACE");
    return e ? std::atoi(e) : 0;
  }();
  return lv;
}

bool trace_on() { return trace_level() > 0; }

void trace_sweep(const char* phase, int panel, int it, const std::vector<double>& maxbits) {
  if (trace_level() < 2) return;
  double mx = 0.0;
  for (size_t k = 0; k + 1 < maxbits.size(); k += 2) mx = std::max(mx, maxbits[k]);
  std::fprintf(stderr, "[ftcc] %s panel %d sweep %d: largest change %.3e\n", phase, panel, it, mx);
  std::fflush(stderr);
}

void trace(ftcc_ctx* c, const char* phase, int panel, int n_panels, const std::vector<int>& sweeps,
           std::chrono::steady_clock::time_point t0) {
  if (!trace_on()) return;
  const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int mx = 0;
  for (int v : sweeps) mx = std::max(mx, v);
  std::fprintf(stderr, "[ftcc] %s panel %d/%d: max sweeps %d, %.2f s since phase start, %.2f GiB held\n",
               phase, panel, n_panels, mx, s, c->bytes / 1073741824.0);
  std::fflush(stderr);
}

void trace_mem(ftcc_ctx* c, const char* stage) {
  if (!trace_on()) return;
  std::fprintf(stderr, "[ftcc] device memory held after %s: %.2f GiB\n", stage, c->bytes / 1073741824.0);
  std::fflush(stderr);
}

void trace_executor(ftcc_ctx* c, const char* which, const Executor& ex) {
  if (!trace_on()) return;
  std::fprintf(stderr,
               "[ftcc] %s executor built: %.2f GiB held (cached operand copies %.2f GiB, permuted constants %.2f GiB, "
               "%d packed intermediates, %d slots)\n",
               which, c->bytes / 1073741824.0, ex.cache_bytes() / 1073741824.0, ex.const_copy_bytes() / 1073741824.0,
               ex.n_packed(), c->slots);
  std::fflush(stderr);
}

void sync(ftcc_ctx* c) {
  FTCC_HIP(hipStreamSynchronize(c->stream));
  if (c->prof.enabled) c->prof.harvest();
}

// ------------------------------------------------------------------ thermal set-up
void thermal_setup(ftcc_ctx* c, int i) {
  Instance& I = c->inst[i];
  const int n = I.n;
  ThermalProblem tp;
  tp.n = n;
  tp.eps = I.eps;
  tp.h = I.h;
  tp.eri = I.eri;
  tp.mu = I.mu;
  tp.beta = I.beta;
  tp.thr = c->opt.occ_thresh;
  tp.g = c->gdeg;
  tp.occ = I.occ;
  tp.wo = I.wo;
  tp.wv = I.wv;
  tp.fock = I.fock;
  launch_thermal(tp, c->stream);
  launch_u_from_fock(n, I.fock, I.eps, I.u_raw, c->stream);
  for (int k = 0; k < 4; ++k) {
    BlockSpec b;
    b.n = n;
    b.rank = 2;
    b.pat[0] = kU[k][2];
    b.pat[1] = kU[k][3];
    b.base = I.u_raw;
    b.dbase = I.u_raw;
    b.wo = I.wo;
    b.wv = I.wv;
    b.dwo = b.dwv = nullptr;
    b.out = I.blk[kU[k]];
    launch_block(b, c->stream);
  }
  for (int k = 0; k < 12; ++k) {
    BlockSpec b;
    b.n = n;
    b.rank = 4;
    for (int s = 0; s < 4; ++s) b.pat[s] = kG[k][2 + s];
    b.base = I.eri;
    b.dbase = I.eri;
    b.wo = I.wo;
    b.wv = I.wv;
    b.dwo = b.dwv = nullptr;
    b.out = I.blk[kG[k]];
    b.idx = I.d_allowed[1];   // with momentum labels: the allowed elements (the law of t2)
    b.count = I.n_allowed[1];
    launch_block(b, c->stream);
  }
  hipLaunchKernelGGL(meanfield_kernel, dim3(1), dim3(256), 0, c->stream, n, I.eps, I.h, I.eri, I.occ, I.fock, I.mu,
                     I.beta, nullptr, nullptr, c->gdeg, I.mf);
  FTCC_HIP(hipGetLastError());
}

// derivative blocks for theta: which = 0 (mu), 1 (beta), 2 (direction dh, deri)
void deriv_setup(ftcc_ctx* c, int i, int which, const double* d_dh, const double* d_deri) {
  Instance& I = c->inst[i];
  const int n = I.n;
  if (which < 2) {
    hipLaunchKernelGGL(occ_deriv_kernel, dim3((n + 63) / 64), dim3(64), 0, c->stream, n, I.eps, I.occ, I.wo, I.wv,
                       I.mu, I.beta, which, I.dn, I.dwo, I.dwv);
    launch_fock_deriv(n, I.eri, nullptr, nullptr, I.occ, I.dn, c->gdeg, I.du_raw, c->stream);
  } else {
    launch_fock_deriv(n, I.eri, d_deri, d_dh, I.occ, nullptr, c->gdeg, I.du_raw, c->stream);
  }
  for (int k = 0; k < 4; ++k) {
    BlockSpec b;
    b.n = n;
    b.rank = 2;
    b.pat[0] = kU[k][2];
    b.pat[1] = kU[k][3];
    b.base = I.u_raw;
    b.dbase = I.du_raw;
    b.wo = I.wo;
    b.wv = I.wv;
    b.dwo = (which < 2) ? I.dwo : nullptr;
    b.dwv = (which < 2) ? I.dwv : nullptr;
    b.out = I.dblk[kU[k]];
    launch_block(b, c->stream);
  }
  for (int k = 0; k < 12; ++k) {
    BlockSpec b;
    b.n = n;
    b.rank = 4;
    for (int s = 0; s < 4; ++s) b.pat[s] = kG[k][2 + s];
    b.base = I.eri;
    b.dbase = (which < 2) ? nullptr : d_deri;
    b.wo = I.wo;
    b.wv = I.wv;
    b.dwo = (which < 2) ? I.dwo : nullptr;
    b.dwv = (which < 2) ? I.dwv : nullptr;
    b.out = I.dblk[kG[k]];
    b.idx = I.d_allowed[1];
    b.count = I.n_allowed[1];
    launch_block(b, c->stream);
  }
  FTCC_HIP(hipGetLastError());
}

// derivative blocks along the orbital energy eps_q (occupation and explicit u parts)
void deriv_setup_eps(ftcc_ctx* c, int i, int q) {
  Instance& I = c->inst[i];
  const int n = I.n;
  const long n2 = (long)n * n;
  hipLaunchKernelGGL(occ_deriv_eps_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, c->stream, n, q, I.eps,
                     I.occ, I.wo, I.wv, I.mu, I.beta, I.dn, I.dwo, I.dwv, I.deps_dh);
  launch_fock_deriv(n, I.eri, nullptr, I.deps_dh, I.occ, I.dn, c->gdeg, I.du_raw, c->stream);
  for (int k = 0; k < 4; ++k) {
    BlockSpec b;
    b.n = n;
    b.rank = 2;
    b.pat[0] = kU[k][2];
    b.pat[1] = kU[k][3];
    b.base = I.u_raw;
    b.dbase = I.du_raw;
    b.wo = I.wo;
    b.wv = I.wv;
    b.dwo = I.dwo;
    b.dwv = I.dwv;
    b.out = I.dblk[kU[k]];
    launch_block(b, c->stream);
  }
  for (int k = 0; k < 12; ++k) {
    BlockSpec b;
    b.n = n;
    b.rank = 4;
    for (int s = 0; s < 4; ++s) b.pat[s] = kG[k][2 + s];
    b.base = I.eri;
    b.dbase = nullptr;
    b.wo = I.wo;
    b.wv = I.wv;
    b.dwo = I.dwo;
    b.dwv = I.dwv;
    b.out = I.dblk[kG[k]];
    b.idx = I.d_allowed[1];
    b.count = I.n_allowed[1];
    launch_block(b, c->stream);
  }
  FTCC_HIP(hipGetLastError());
}

long node_len_of(long n) { return n * n + n * n * n * n; }

// Throws FTCC_EINVAL when a rank-2 or rank-4 array of instance i breaks the
// instance's momentum conservation.
void check_momentum(ftcc_ctx* c, int i, const double* x, int rank, const char* what) {
  Instance& I = c->inst[i];
  if (!c->d_bad) c->d_bad = (int*)c->dalloc(1);
  int* d_bad = c->d_bad;
  FTCC_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), c->stream));   // ordinary stream work, never captured
  hipLaunchKernelGGL(momentum_check_kernel, dim3(1024), dim3(256), 0, c->stream, I.n, rank, I.mom.dims, I.d_labels,
                     I.d_modulus, x, d_bad);
  FTCC_HIP(hipGetLastError());
  int bad = 0;
  FTCC_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  FTCC_HIP(hipStreamSynchronize(c->stream));
  if (bad)
    fail(FTCC_EINVAL, std::string(what) + " of instance " + std::to_string(i) +
                          " has nonzero elements that its momentum labels forbid");
}

bool momentum_on(const ftcc_ctx* c) {
  for (const Instance& I : c->inst)
    if (I.mom.dims == 0) return false;
  return !c->inst.empty();
}

// Offsets, in memory order, of the amplitude elements momentum allows:
// t1[i][a] with k_i = k_a and t2[i][j][a][b] with k_i + k_j = k_a + k_b.
void allowed_elements(ftcc_ctx* c, int i) {
  Instance& I = c->inst[i];
  const int n = I.n, D = I.mom.dims;
  auto mom = [&](int p, int q, int sign) {
    std::vector<int> v(D);
    for (int d = 0; d < D; ++d) {
      int x = I.mom.labels[(size_t)p * D + d] + sign * (q >= 0 ? I.mom.labels[(size_t)q * D + d] : 0);
      const int m = I.mom.modulus[d];
      if (m > 0) x = ((x % m) + m) % m;
      v[d] = x;
    }
    return v;
  };
  std::vector<unsigned> l1, l2;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q)
      if (mom(p, -1, 0) == mom(q, -1, 0)) l1.push_back((unsigned)(p * n + q));
  std::map<std::vector<int>, std::vector<unsigned>> pairs;   // pair momentum -> offsets a*n+b (ascending)
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) pairs[mom(a, b, +1)].push_back((unsigned)(a * n + b));
  const unsigned n2 = (unsigned)n * n;
  for (int p = 0; p < n; ++p)
    for (int q = 0; q < n; ++q) {
      auto it = pairs.find(mom(p, q, +1));
      if (it == pairs.end()) continue;
      const unsigned row = (unsigned)(p * n + q) * n2;
      for (unsigned ab : it->second) l2.push_back(row + ab);
    }
  for (int seg = 0; seg < 2; ++seg) {
    const std::vector<unsigned>& l = seg ? l2 : l1;
    I.n_allowed[seg] = (long)l.size();
    I.d_allowed[seg] = (unsigned*)c->dalloc(l.size() / 2 + 1);
    if (!l.empty())
      FTCC_HIP(hipMemcpy(I.d_allowed[seg], l.data(), sizeof(unsigned) * l.size(), hipMemcpyHostToDevice));
  }
}

// elements the propagator visits in segment seg (0: t1, 1: t2) of instance i
long seg_len(const ftcc_ctx* c, int i, int seg) {
  const Instance& I = c->inst[i];
  if (I.d_allowed[seg]) return I.n_allowed[seg];
  const long n2 = (long)I.n * I.n;
  return seg ? n2 * n2 : n2;
}

// ------------------------------------------------------------------ build
void build(ftcc_ctx* c) {
  if (c->built) return;
  for (int i = 0; i < c->B; ++i)
    if (!c->inst[i].has_ham) fail(FTCC_ESTATE, "instance " + std::to_string(i) + " has no Hamiltonian");
  const int m = c->m, P = c->P, B = c->B;
  c->prog = c->opt.spin_orbital ? build_spin_orbital_program() : build_residual_program();
  const bool mom = momentum_on(c);
  if (mom)
    for (int i = 0; i < B; ++i) {
      Instance& I = c->inst[i];
      I.d_labels = (int*)c->dalloc(I.mom.labels.size() / 2 + 1);
      I.d_modulus = (int*)c->dalloc(I.mom.modulus.size() / 2 + 1);
      FTCC_HIP(hipMemcpy(I.d_labels, I.mom.labels.data(), sizeof(int) * I.mom.labels.size(), hipMemcpyHostToDevice));
      FTCC_HIP(
          hipMemcpy(I.d_modulus, I.mom.modulus.data(), sizeof(int) * I.mom.modulus.size(), hipMemcpyHostToDevice));
      check_momentum(c, i, I.h, 2, "h");
      check_momentum(c, i, I.eri, 4, "<pq|rs>");
      allowed_elements(c, i);
    }
  const Program& prog = c->prog;

  for (int i = 0; i < B; ++i) {
    Instance& I = c->inst[i];
    const int n = I.n;
    const long n2 = (long)n * n, n4 = n2 * n2, len = n2 + n4;
    I.occ = c->dalloc(n);
    I.wo = c->dalloc(n);
    I.wv = c->dalloc(n);
    I.dn = c->dalloc(n);
    I.dwo = c->dalloc(n);
    I.dwv = c->dalloc(n);
    I.fock = c->dalloc(n2);
    I.u_raw = c->dalloc(n2);
    I.du_raw = c->dalloc(n2);
    for (int k = 0; k < 4; ++k) {
      I.blk[kU[k]] = c->dalloc(n2);
      I.dblk[kU[k]] = c->dalloc(n2);
    }
    for (int k = 0; k < 12; ++k) {
      I.blk[kG[k]] = c->dalloc(n4);
      I.dblk[kG[k]] = c->dalloc(n4);
    }
    I.mf = c->dalloc(5);
    I.acc = c->dalloc(8);
    for (int k = 0; k < 4; ++k) I.ugrad_acc[k] = c->dalloc(n2);
    I.sb.resize(P + 1);
    for (int p = 0; p <= P; ++p) I.sb[p] = c->dalloc(len);
  }
  // Checkpointing when the stored grid (amplitudes and residuals of every node)
  // would take more than half of the capped memory.
  if (!c->opt.checkpoint && c->opt.mem_cap_bytes) {
    double grid = 0.0;
    for (int i = 0; i < B; ++i) grid += 2.0 * P * m * (double)node_len_of(c->inst[i].n) * sizeof(double);
    if (grid > 0.5 * (double)c->opt.mem_cap_bytes) c->opt.checkpoint = 1;
  }
  for (int i = 0; i < B; ++i) {
    Instance& I = c->inst[i];
    const long len = node_len_of(I.n);
    // Lambda of every node and the panel-boundary adjoint states a_p, allocated up
    // front so that the optional caches below are sized to what is left;
    // lambda-tilde is not stored (recomputed from lambda and a_{p+1} when needed)
    const int nlam = c->simpson ? P + 1 : P * m;
    I.lam.resize(nlam);
    for (int k = 0; k < nlam; ++k) I.lam[k] = c->dalloc(len);
    I.abuf.resize(P + 1);
    for (int p = 0; p <= P; ++p) I.abuf[p] = c->dalloc(len);
    if (!c->opt.checkpoint && !c->rk && !c->simpson) {
      I.grid.resize(P * m);
      I.resid.resize(P * m);
      for (int k = 0; k < P * m; ++k) {
        I.grid[k] = c->dalloc(len);
        I.resid[k] = c->dalloc(len);
      }
    }
    I.energies.assign((c->rk || c->simpson) ? P + 1 : P * m, 0.0);
    if (c->rk || c->simpson) {
      I.rk_tmp[0] = c->dalloc(len);
      I.rk_tmp[1] = c->dalloc(len);
      I.rk_hbar = c->dalloc(1);
    }
  }
  if (c->rk || c->simpson) {
    // (1/beta) g_k of Simpson's rule on the uniform grid: w_k / (3 n_g), w = 1 4 2 ... 4 1
    std::vector<double> w(P + 1);
    for (int k = 0; k <= P; ++k) w[k] = ((k == 0 || k == P) ? 1.0 : (k % 2 ? 4.0 : 2.0)) / (3.0 * P);
    c->d_rkw = c->dalloc(P + 1);
    FTCC_HIP(hipMemcpy(c->d_rkw, w.data(), sizeof(double) * (P + 1), hipMemcpyHostToDevice));
  }
  trace_mem(c, "integrals, panel states and Lambda storage");
  // Executor slots per instance: every node of a panel evaluated in one grouped
  // launch (slots = m) unless the per-slot working set would take more than half
  // of the free device memory; then the nodes go through one slot in turn.  The
  // working set is about 40 n^4 doubles (intermediates, their gradients,
  // scratch), or, when the momentum-blocked intermediates are stored packed
  // (n^3 each), the scratch and the derivative residual of each slot, 5 n^4.
  {
    bool packed = momentum_on(c) && packing_enabled();
    for (const Instance& I : c->inst) packed = packed && labels_distinct(I.mom);
    double need = 0.0;
    for (int i = 0; i < B; ++i)
      need += (packed ? 5.0 : 40.0) * m * std::pow((double)c->inst[i].n, 4) * sizeof(double);
    c->slots = (need > 0.5 * c->available()) ? 1 : m;
    const char* senv = std::getenv("FTCC_NODE_SLOTS");
    if (senv && senv[0] == '1') c->slots = 1;
    if (c->rk || c->simpson) c->slots = 1;   // stages / grid points are evaluated in turn
  }
  const int SL = c->slots;
  const int nn = B * m;
  c->amp.resize(nn);
  c->S.resize(nn);
  c->e.resize(nn);
  c->gr.resize(nn);
  c->cot.resize(nn);
  c->ebar.resize(nn);
  c->dS.resize(nn);
  c->de.resize(nn);
  c->ugrad.resize(nn);
  for (int i = 0; i < B; ++i)
    for (int x = 0; x < m; ++x) {
      const int p = i * m + x;
      const int n = c->inst[i].n;
      const long n2 = (long)n * n, n4 = n2 * n2, len = n2 + n4;
      c->amp[p] = c->dalloc(len);
      c->S[p] = c->dalloc(len);
      c->e[p] = c->dalloc(1);
      c->gr[p] = c->dalloc(len);
      c->cot[p] = c->dalloc(len);
      c->ebar[p] = c->dalloc(1);
      // with one slot the derivative residuals reuse the gradient buffers (never live together)
      c->dS[p] = (SL == m) ? c->dalloc(len) : c->gr[p];
      c->de[p] = c->dalloc(1);
      for (int k = 0; k < 4; ++k) c->ugrad[p][k] = c->dalloc(n2);
      const double eb = c->rule.b[x] / P;   // (1/beta) g_x
      FTCC_HIP(hipMemcpy(c->ebar[p], &eb, sizeof(double), hipMemcpyHostToDevice));
      (void)n4;
    }
  const int np = B * SL;
  c->scratch.a.resize(np);
  c->scratch.b.resize(np);
  c->scratch.c.resize(np);
  c->scratch.part.resize(np);
  c->s_amp.resize(np);
  c->s_S.resize(np);
  c->s_e.resize(np);
  c->s_gr.resize(np);
  c->s_cot.resize(np);
  c->s_ebar.resize(np);
  c->s_dS.resize(np);
  c->s_de.resize(np);
  c->s_ugrad.resize(np);
  std::vector<ProblemRef> probs;
  for (int i = 0; i < B; ++i)
    for (int x = 0; x < SL; ++x) {
      const int q = i * SL + x;
      const int n = c->inst[i].n;
      const long n2 = (long)n * n, n4 = n2 * n2, len = n2 + n4;
      probs.push_back({i, x, n});
      if (SL == m) {
        const int p = i * m + x;
        c->s_amp[q] = c->amp[p];
        c->s_S[q] = c->S[p];
        c->s_e[q] = c->e[p];
        c->s_gr[q] = c->gr[p];
        c->s_cot[q] = c->cot[p];
        c->s_ebar[q] = c->ebar[p];
        c->s_dS[q] = c->dS[p];
        c->s_de[q] = c->de[p];
        c->s_ugrad[q] = c->ugrad[p];
      } else {
        c->s_amp[q] = c->dalloc(len);
        c->s_S[q] = c->dalloc(len);
        c->s_e[q] = c->dalloc(1);
        c->s_gr[q] = c->dalloc(len);
        c->s_cot[q] = c->dalloc(len);
        c->s_ebar[q] = c->dalloc(1);
        c->s_dS[q] = c->s_S[q];       // the derivative executor runs apart from the main one
        c->s_de[q] = c->dalloc(1);
        for (int k = 0; k < 4; ++k) c->s_ugrad[q][k] = c->dalloc(n2);
      }
      c->scratch.a[q] = c->dalloc(n4);
      c->scratch.b[q] = c->dalloc(n4);
      c->scratch.c[q] = c->dalloc(n4);
      c->scratch.part[q] = c->dalloc(n4);
    }
  c->scratch.dot_partial = c->dalloc((size_t)nn * 64 + 64);
  {
    // workspace for partial tiles: 128 MiB, or an eighth of a memory cap below 1 GiB
    size_t ws = kTailWorkspaceDoubles;
    if (c->opt.mem_cap_bytes) ws = std::min(ws, std::max<size_t>(c->opt.mem_cap_bytes / 64, 64 * 256));
    c->scratch.tail_ws = c->dalloc(ws);
    c->scratch.tail_ws_doubles = ws;
  }
  c->d_maxbits = (unsigned long long*)c->dalloc(2 * B);
  c->d_active = (int*)c->dalloc(B);
  c->d_run = (int*)c->dalloc(B);
  c->run_host.assign(B, 1);
  FTCC_HIP(hipMemcpy(c->d_run, c->run_host.data(), sizeof(int) * B, hipMemcpyHostToDevice));
  {
    std::vector<int> ones(2 * B, 1);
    FTCC_HIP(hipMemcpy(c->d_active, ones.data(), sizeof(int) * B, hipMemcpyHostToDevice));
  }
  const int D = c->opt.diis_depth;
  if (D > 0) {
    c->diis_X.assign(B, {});
    c->diis_R.assign(B, {});
    for (int i = 0; i < B; ++i) {
      const long n = c->inst[i].n, len = n * n + n * n * n * n;
      for (int d = 0; d < D; ++d) {
        c->diis_X[i].push_back(c->dalloc((size_t)m * len));
        c->diis_R[i].push_back(c->dalloc((size_t)m * len));
      }
    }
    c->d_gram = c->dalloc((size_t)B * D * D);
    c->d_coef = c->dalloc((size_t)B * D);
    c->d_dcount = (int*)c->dalloc(B);
    c->d_dnewest = (int*)c->dalloc(B);
    c->diis_count.assign(B, 0);
    c->diis_next.assign(B, 0);
  }
  c->d_rule = (PanelRule*)c->dalloc(sizeof(PanelRule) / sizeof(double) + 1);
  FTCC_HIP(hipMemcpy(c->d_rule, &c->rule, sizeof(PanelRule), hipMemcpyHostToDevice));
  {
    size_t blocks = 16;
    c->beta_part_off.assign(B, 0);
    for (int i = 0; i < B; ++i) {
      c->beta_part_off[i] = (int)blocks - 16;
      blocks += (seg_len(c, i, 0) + 1023) / 1024 + (seg_len(c, i, 1) + 1023) / 1024;
    }
    c->d_partial = c->dalloc(blocks);
  }

  trace_mem(c, "node and slot buffers");
  std::vector<int> ugrads;
  for (int k = 0; k < 4; ++k) ugrads.push_back(prog.id(kU[k]));
  const int id_t1 = prog.id("t1"), id_t2 = prog.id("t2"), id_S1 = prog.id("S1"), id_S2 = prog.id("S2"),
            id_E = prog.id("E");

  auto tensor_buf = [c, &probs](std::map<std::pair<int, int>, double*>& store, int t, int key, long count) {
    return shared_buf(c, store, t, key, count);
  };
  // intermediates take the element count the executor addresses (packed or dense)
  auto bind_common = [&, c](int t, int p, bool grad, size_t count) -> double* {
    const TensorDecl& d = prog.t[t];
    const long n = probs[p].n, n2 = n * n;
    const long cnt = (long)count;
    if (t == id_t1) return grad ? c->s_gr[p] : c->s_amp[p];
    if (t == id_t2) return grad ? c->s_gr[p] + n2 : c->s_amp[p] + n2;
    if (grad) {
      if (t == id_S1) return c->s_cot[p];
      if (t == id_S2) return c->s_cot[p] + n2;
      if (t == id_E) return c->s_ebar[p];
      if (d.kind == T_CONST) {
        for (int k = 0; k < 4; ++k)
          if (d.name == kU[k]) return c->s_ugrad[p][k];
        fail(FTCC_EINVAL, "no gradient buffer for " + d.name);
      }
      return tensor_buf(c->inter_grad, t, p, cnt);
    }
    if (d.kind == T_INTER && !d.derived) return tensor_buf(c->inter, t, p, cnt);
    return nullptr;
  };
  Binder bind_main = [&, c](int t, int p, bool grad, size_t count) -> double* {
    const TensorDecl& d = prog.t[t];
    if (double* q = bind_common(t, p, grad, count)) return q;
    const int i = probs[p].inst;
    const long n = probs[p].n, n2 = n * n;
    if (d.kind == T_CONST) return c->inst[i].blk[d.name];
    if (d.derived) return tensor_buf(c->derived, t, i, ipow(n, d.rank));
    if (t == id_S1) return c->s_S[p];
    if (t == id_S2) return c->s_S[p] + n2;
    if (t == id_E) return c->s_e[p];
    fail(FTCC_EINVAL, "unbound tensor " + d.name);
  };
  Binder bind_d = [&, c](int t, int p, bool grad, size_t count) -> double* {
    const TensorDecl& d = prog.t[t];
    if (double* q = bind_common(t, p, grad, count)) return q;
    const int i = probs[p].inst;
    const long n = probs[p].n, n2 = n * n;
    if (d.kind == T_CONST) return c->inst[i].dblk[d.name];
    if (d.derived) return tensor_buf(c->dderived, t, i, ipow(n, d.rank));
    if (t == id_S1) return c->s_dS[p];
    if (t == id_S2) return c->s_dS[p] + n2;
    if (t == id_E) return c->s_de[p];
    fail(FTCC_EINVAL, "unbound tensor " + d.name);
  };
  auto calloc_ = [c](int, size_t count) { return c->dalloc(count); };
  // Reused permuted copies of value operands are optional: one is taken only while
  // it leaves a reserve for what the executors must still allocate (the second
  // executor's intermediates and permuted constants: 16 n^4 doubles per instance,
  // plus 1 GiB), and an allocation that fails leaves the operand uncached.
  double reserve = 1073741824.0;
  for (int i = 0; i < B; ++i) reserve += 16.0 * std::pow((double)c->inst[i].n, 4) * sizeof(double);
  auto vcache = [c, reserve](size_t count) -> double* {
    if (c->available() < reserve + (double)count * sizeof(double)) return nullptr;
    try {
      return c->dalloc(count);
    } catch (const Fail& f) {
      if (f.code != FTCC_ENOMEM) throw;
      return nullptr;
    }
  };
  // reuse budget for permuted operand copies: a quarter of the memory still available
  // (the blocked contractions address their operands in place: no permuted copies)
  const size_t budget = mom ? 0 : (size_t)(c->available() / 4);
  std::vector<const InstMomentum*> by_inst;
  if (mom)
    for (const Instance& I : c->inst) by_inst.push_back(&I.mom);
  c->ex_main.reset(new Executor());
  c->ex_main->set_gate(c->d_run, c->run_host.data());
  if (mom) c->ex_main->set_momentum(by_inst);
  c->ex_main->build(&prog, probs, bind_main, &c->scratch, calloc_, true, ugrads, vcache, budget);
  c->ex_main->set_profiler(&c->prof);
  trace_executor(c, "main", *c->ex_main);
  c->ex_d.reset(new Executor());
  if (mom) c->ex_d->set_momentum(by_inst);
  c->ex_d->build(&prog, probs, bind_d, &c->scratch, calloc_, false, {}, vcache, budget / 2);
  c->ex_d->set_profiler(&c->prof);
  trace_executor(c, "derivative", *c->ex_d);
  trace_mem(c, "executors");
  // no kernel-profiler events inside the autotuner or a graph capture
  const bool prof_on = c->prof.enabled;
  c->prof.enabled = false;
  c->ex_main->autotune(c->stream);
  c->ex_d->autotune(c->stream);
  FTCC_HIP(hipStreamSynchronize(c->stream));
  const char* genv = std::getenv("FTCC_GRAPH");
  if (!(genv && genv[0] == '0')) {
    // the forward and backward launch lists are static: capture each once as a graph
    hipGraph_t g;
    FTCC_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->ex_main->run_forward(c->stream);
    FTCC_HIP(hipStreamEndCapture(c->stream, &g));
    FTCC_HIP(hipGraphInstantiate(&c->g_fwd, g, nullptr, nullptr, 0));
    FTCC_HIP(hipGraphDestroy(g));
    FTCC_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->ex_main->run_backward(c->stream);
    FTCC_HIP(hipStreamEndCapture(c->stream, &g));
    FTCC_HIP(hipGraphInstantiate(&c->g_bwd, g, nullptr, nullptr, 0));
    FTCC_HIP(hipGraphDestroy(g));
  }

  c->prof.enabled = prof_on;
  c->built = true;
}

// number of instances whose residual programs currently run
long n_running(ftcc_ctx* c) {
  long k = 0;
  for (int v : c->run_host) k += v ? 1 : 0;
  return k;
}

// the forward / backward programs: graph replay unless the kernel profiler records events
void run_fwd_slots(ftcc_ctx* c) {
  if (c->g_fwd && !c->prof.enabled) FTCC_HIP(hipGraphLaunch(c->g_fwd, c->stream));
  else c->ex_main->run_forward(c->stream);
}

void run_bwd_slots(ftcc_ctx* c) {
  if (c->g_bwd && !c->prof.enabled) FTCC_HIP(hipGraphLaunch(c->g_bwd, c->stream));
  else c->ex_main->run_backward(c->stream);
}

long node_len(ftcc_ctx* c, int i) {
  const long n = c->inst[i].n;
  return n * n + n * n * n * n;
}

void dcopy(ftcc_ctx* c, double* dst, const double* src, long count) {
  FTCC_HIP(hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyDeviceToDevice, c->stream));
}

// Copy of one node state of instance i (t1 block, then t2 block).  With momentum
// labels only the allowed elements move: every state buffer keeps its forbidden
// elements at zero (buffers start zeroed and no kernel of the blocked path
// writes them), so the rest of the copy would move zeros onto zeros.
void node_copy(ftcc_ctx* c, int i, double* dst, const double* src) {
  const Instance& I = c->inst[i];
  if (!I.d_allowed[0] || !I.d_allowed[1]) {
    dcopy(c, dst, src, node_len(c, i));
    return;
  }
  launch_copy_listed(I.d_allowed[0], I.n_allowed[0], I.d_allowed[1], I.n_allowed[1], (long)I.n * I.n, src, dst,
                     c->stream);
  FTCC_HIP(hipGetLastError());
}

// forward residuals of every node of the panel slots (node amplitudes -> S, E)
void forward(ftcc_ctx* c) {
  if (c->slots == c->m) {
    run_fwd_slots(c);
    return;
  }
  for (int x = 0; x < c->m; ++x) {
    for (int i = 0; i < c->B; ++i)
      if (c->run_host[i]) node_copy(c, i, c->s_amp[i], c->amp[i * c->m + x]);
    run_fwd_slots(c);
    for (int i = 0; i < c->B; ++i) {
      if (!c->run_host[i]) continue;
      node_copy(c, i, c->S[i * c->m + x], c->s_S[i]);
      dcopy(c, c->e[i * c->m + x], c->s_e[i], 1);
    }
  }
}

// reverse pass of every node (cotangents cot, E weights ebar -> gradients gr, ugrad).
// With one slot each node's forward tape is recomputed first.
void backward(ftcc_ctx* c) {
  if (c->slots == c->m) {
    run_bwd_slots(c);
    return;
  }
  for (int x = 0; x < c->m; ++x) {
    for (int i = 0; i < c->B; ++i)
      if (c->run_host[i]) node_copy(c, i, c->s_amp[i], c->amp[i * c->m + x]);
    run_fwd_slots(c);
    c->resid_evals += n_running(c);
    for (int i = 0; i < c->B; ++i) {
      if (!c->run_host[i]) continue;
      const int p = i * c->m + x;
      node_copy(c, i, c->s_cot[i], c->cot[p]);
      dcopy(c, c->s_ebar[i], c->ebar[p], 1);
    }
    run_bwd_slots(c);
    for (int i = 0; i < c->B; ++i) {
      if (!c->run_host[i]) continue;
      const int p = i * c->m + x;
      const long n = c->inst[i].n;
      node_copy(c, i, c->gr[p], c->s_gr[i]);
      for (int k = 0; k < 4; ++k) dcopy(c, c->ugrad[p][k], c->s_ugrad[i][k], n * n);
    }
  }
}

// derivative-integral residuals of every node (-> dS, dE)
void d_forward(ftcc_ctx* c) {
  if (c->slots == c->m) {
    c->ex_d->run_forward(c->stream);
    return;
  }
  for (int x = 0; x < c->m; ++x) {
    for (int i = 0; i < c->B; ++i) node_copy(c, i, c->s_amp[i], c->amp[i * c->m + x]);
    c->ex_d->run_forward(c->stream);
    for (int i = 0; i < c->B; ++i) {
      node_copy(c, i, c->dS[i * c->m + x], c->s_dS[i]);
      dcopy(c, c->de[i * c->m + x], c->s_de[i], 1);
    }
  }
}

void clear_tau_cache(ftcc_ctx* c) {
  for (auto& kv : c->tau_cache) {
    (void)hipFree(kv.second.first);
    (void)hipFree(kv.second.second);
  }
  c->tau_cache.clear();
  c->tau_shape.clear();
  for (auto& kv : c->rk_cache) {
    (void)hipFree(kv.second.first);
    (void)hipFree(kv.second.second);
  }
  c->rk_cache.clear();
  c->rk_blocks.clear();
  for (auto& kv : c->rk_dots) (void)hipFree(kv.second);
  c->rk_dots.clear();
  for (auto& kv : c->sp_cache) (void)hipFree(kv.second.buf);
  c->sp_cache.clear();
}

// Descriptor set for the propagator: per instance two segments (t1, t2).
// `panel` selects per-panel buffers (sb, lambda, a, ...).  Descriptors are built
// once per (mode, panel) and kept until the next solve (beta may change).
// Host descriptors of one propagator launch (mode, panel): per instance the t1 and
// t2 segments; TAU_BETA partial sums go to partial_base (one per 1024 elements).
int tau_problems(ftcc_ctx* c, int mode, int panel, double* partial_base, std::vector<TauProblem>& ps,
                 std::vector<int>& prefix) {
  const int B = c->B, m = c->m;
  int total = 0;
  ps.clear();
  prefix.clear();
    for (int i = 0; i < B; ++i) {
      Instance& I = c->inst[i];
      const long n = I.n, n2 = n * n, n4 = n2 * n2;
      for (int seg = 0; seg < 2; ++seg) {
        TauProblem t;
        std::memset(&t, 0, sizeof(t));
        const long off = seg ? n2 : 0;
        t.eps = I.eps;
        t.n = (int)n;
        t.rank = seg ? 4 : 2;
        t.len = seg_len(c, i, seg);
        t.idx = I.d_allowed[seg];
        t.h = I.beta / c->P;
        t.maxbits = c->d_maxbits + 2 * i;
        t.active = (mode == TAU_STEP || mode == TAU_LSTEP) ? c->d_active + i : nullptr;
        for (int x = 0; x < m; ++x) {
          const int p = i * m + x;
          switch (mode) {
            case TAU_INIT:
            case TAU_STEP:
              t.S[x] = c->S[p] + off;
              t.s[x] = c->amp[p] + off;
              break;
            case TAU_END:
              t.S[x] = c->S[p] + off;
              break;
            case TAU_LAMT:      // S = lambda (node storage), s = lambda-tilde (cotangent slots)
              t.S[x] = I.lam[panel * m + x] + off;
              t.s[x] = c->cot[p] + off;
              break;
            case TAU_LSTEP:     // s = lambda (node storage), R = gradient
              t.s[x] = I.lam[panel * m + x] + off;
              t.R[x] = c->gr[p] + off;
              break;
            case TAU_APREV:
              t.S[x] = I.lam[panel * m + x] + off;
              break;
            case TAU_BETA:      // S = lambda, R = converged residuals
            case TAU_DEPS:
              t.S[x] = I.lam[panel * m + x] + off;
              t.R[x] = c->S[p] + off;
              break;
          }
        }
        if (mode == TAU_INIT || mode == TAU_STEP || mode == TAU_END || mode == TAU_BETA || mode == TAU_DEPS)
          t.sb = I.sb[panel] + off;
        if (mode == TAU_END) t.out = I.sb[panel + 1] + off;
        if (mode == TAU_LAMT || mode == TAU_APREV) t.sb = I.abuf[panel + 1] + off;
        if (mode == TAU_APREV) t.out = I.abuf[panel] + off;
        if (mode == TAU_BETA || mode == TAU_DEPS) t.lam_a = I.abuf[panel + 1] + off;
        if (mode == TAU_DEPS) t.out = I.deps_delta + off;
        const int nb = (int)((t.len + 1023) / 1024);
        t.partial = partial_base + (long)total;
        prefix.push_back(total);
        total += nb;
        ps.push_back(t);
      }
    }
  return total;
}

void tau_run(ftcc_ctx* c, int mode, int panel) {
  const auto key = std::make_pair(mode, panel);
  auto it = c->tau_cache.find(key);
  if (it == c->tau_cache.end()) {
    std::vector<TauProblem> ps;
    std::vector<int> prefix;
    const int total = tau_problems(c, mode, panel, c->d_partial, ps, prefix);
    TauProblem* d_ps = nullptr;
    int* d_pre = nullptr;
    FTCC_HIP(hipMalloc((void**)&d_ps, sizeof(TauProblem) * ps.size()));
    FTCC_HIP(hipMalloc((void**)&d_pre, sizeof(int) * prefix.size()));
    FTCC_HIP(hipMemcpy(d_ps, ps.data(), sizeof(TauProblem) * ps.size(), hipMemcpyHostToDevice));
    FTCC_HIP(hipMemcpy(d_pre, prefix.data(), sizeof(int) * prefix.size(), hipMemcpyHostToDevice));
    it = c->tau_cache.emplace(key, std::make_pair(d_ps, d_pre)).first;
    c->tau_shape[key] = std::make_pair((int)ps.size(), total);
  }
  const auto shp = c->tau_shape[key];
  launch_tau(c->d_rule, c->m, mode, it->second.first, it->second.second, shp.first, shp.second, c->stream);
  FTCC_HIP(hipGetLastError());
}

void set_active(ftcc_ctx* c, const std::vector<bool>& active) {
  // the device flags change only here: no copy when they already hold this set
  bool same = (int)c->active_host.size() == c->B;
  for (int i = 0; same && i < c->B; ++i) same = (c->active_host[i] != 0) == active[i];
  if (same) return;
  c->active_host.assign(c->B, 0);
  for (int i = 0; i < c->B; ++i) c->active_host[i] = active[i] ? 1 : 0;
  FTCC_HIP(hipMemcpyAsync(c->d_active, c->active_host.data(), sizeof(int) * c->B, hipMemcpyHostToDevice,
                          c->stream));
}

// Which instances the forward / backward residual programs evaluate (the
// others' launches return at once).  Outside the fixed-point loops every
// instance runs.
void set_run(ftcc_ctx* c, const std::vector<bool>& run) {
  bool same = true;
  for (int i = 0; i < c->B; ++i) same = same && ((c->run_host[i] != 0) == run[i]);
  if (same) return;
  for (int i = 0; i < c->B; ++i) c->run_host[i] = run[i] ? 1 : 0;
  FTCC_HIP(hipMemcpyAsync(c->d_run, c->run_host.data(), sizeof(int) * c->B, hipMemcpyHostToDevice, c->stream));
  // the host array is reused by the next call: finish this copy first
  FTCC_HIP(hipStreamSynchronize(c->stream));
}

void run_all(ftcc_ctx* c) { set_run(c, std::vector<bool>(c->B, true)); }

void reset_maxbits(ftcc_ctx* c) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(256), 0, c->stream, c->d_maxbits, 2 * c->B);
}

std::vector<double> read_maxbits(ftcc_ctx* c) {
  std::vector<unsigned long long> bits(2 * c->B);
  FTCC_HIP(hipMemcpyAsync(bits.data(), c->d_maxbits, sizeof(unsigned long long) * bits.size(),
                          hipMemcpyDeviceToHost, c->stream));
  sync(c);
  std::vector<double> v(bits.size());
  for (size_t k = 0; k < bits.size(); ++k) std::memcpy(&v[k], &bits[k], sizeof(double));
  return v;
}

void copy_d(ftcc_ctx* c, double* dst, const double* src, long count) {
  FTCC_HIP(hipMemcpyAsync(dst, src, sizeof(double) * count, hipMemcpyDeviceToDevice, c->stream));
}

void zero_d(ftcc_ctx* c, double* dst, long count) { launch_axpby(count, 0.0, dst, 0.0, dst, c->stream); }

// ------------------------------------------------------------------ DIIS (Anderson) acceleration
// The fixed-point map G is one sweep (forward residual + propagator, or one
// adjoint sweep).  Before the sweep the iterate s_k is saved as X_k; after it
// R_k = G(s_k) - s_k, the Gram matrix row <R_k, R_j> is updated by dot
// kernels, the bordered least-squares system is solved on the device and the
// iterate is replaced by sum_j c_j (X_j + R_j).
void diis_reset(ftcc_ctx* c) {
  for (int i = 0; i < c->B; ++i) c->diis_count[i] = c->diis_next[i] = 0;
}


void diis_before(ftcc_ctx* c, const NodeBufs& it, const std::vector<bool>& active) {
  for (int i = 0; i < c->B; ++i) {
    if (!active[i]) continue;
    const long n = c->inst[i].n, len = n * n + n * n * n * n;
    double* X = c->diis_X[i][c->diis_next[i]];
    for (int x = 0; x < c->m; ++x) copy_d(c, X + x * len, it(i, x), len);
  }
}

void diis_after(ftcc_ctx* c, const NodeBufs& it, const std::vector<bool>& active) {
  const int D = c->opt.diis_depth, m = c->m;
  std::vector<int> newest(c->B, 0);
  bool any = false;
  for (int i = 0; i < c->B; ++i) {
    newest[i] = c->diis_next[i];
    if (!active[i]) continue;
    any = true;
    const long n = c->inst[i].n, len = n * n + n * n * n * n;
    const int slot = c->diis_next[i];
    double* X = c->diis_X[i][slot];
    double* R = c->diis_R[i][slot];
    for (int x = 0; x < m; ++x) {
      copy_d(c, R + x * len, it(i, x), len);
      launch_axpby(len, -1.0, X + x * len, 1.0, R + x * len, c->stream);
    }
    c->diis_count[i] = std::min(D, c->diis_count[i] + 1);
    c->diis_next[i] = (slot + 1) % D;
    // Gram entries of the new residual against every stored one
    std::vector<DotProblem> ds;
    for (int t = 0; t < c->diis_count[i]; ++t) {
      for (int tw = 0; tw < 2; ++tw) {
        DotProblem d{};
        d.X = R;
        d.Y = c->diis_R[i][t];
        d.out = c->d_gram + (long)i * D * D + (tw ? t * D + slot : slot * D + t);
        d.len = m * len;
        d.alpha = 1.0;
        d.beta = 0.0;
        ds.push_back(d);
      }
    }
    DotProblem* dd = nullptr;
    FTCC_HIP(hipMallocAsync((void**)&dd, sizeof(DotProblem) * ds.size(), c->stream));
    FTCC_HIP(hipMemcpyAsync(dd, ds.data(), sizeof(DotProblem) * ds.size(), hipMemcpyHostToDevice, c->stream));
    launch_dot(dd, (int)ds.size(), 64, c->scratch.dot_partial, c->stream);
    FTCC_HIP(hipFreeAsync(dd, c->stream));
  }
  if (!any) return;
  FTCC_HIP(hipMemcpyAsync(c->d_dcount, c->diis_count.data(), sizeof(int) * c->B, hipMemcpyHostToDevice, c->stream));
  std::vector<int>* keep = new std::vector<int>(newest);
  FTCC_HIP(hipMemcpyAsync(c->d_dnewest, keep->data(), sizeof(int) * c->B, hipMemcpyHostToDevice, c->stream));
  launch_diis_solve(c->B, c->d_dcount, c->d_dnewest, c->d_gram, D, c->d_coef, c->stream);
  for (int i = 0; i < c->B; ++i) {
    if (!active[i] || c->diis_count[i] < 2) continue;
    const long n = c->inst[i].n, len = n * n + n * n * n * n;
    for (int x = 0; x < m; ++x) {
      DiisTerms t;
      t.k = c->diis_count[i];
      t.coef = c->d_coef + (long)i * D;
      for (int j = 0; j < t.k; ++j) {
        t.X[j] = c->diis_X[i][j] + x * len;
        t.R[j] = c->diis_R[i][j] + x * len;
      }
      launch_diis_combine(len, t, it(i, x), c->stream);
    }
  }
  FTCC_HIP(hipStreamSynchronize(c->stream));
  delete keep;
}


// Converge the Picard iteration of one panel for all instances (amplitudes in
// the slots, residuals at the final amplitudes in S).  Returns per-instance sweeps.
std::vector<int> panel_solve(ftcc_ctx* c, int panel, std::vector<int>& status) {
  const int B = c->B;
  std::vector<int> its(B, 0);
  std::vector<bool> active(B, true);
  for (int i = 0; i < B; ++i)
    if (status[i] != 0) active[i] = false;
  tau_run(c, TAU_INIT, panel);
  const bool diis = c->opt.diis_depth > 0;
  NodeBufs amp_of = [c](int i, int x) { return c->amp[i * c->m + x]; };
  if (diis) diis_reset(c);
  set_run(c, active);   // converged or failed instances stop costing residual evaluations
  std::vector<DivergenceWatch> watch(B);
  for (int it = 1; it <= c->opt.max_iter; ++it) {
    forward(c);
    c->resid_evals += n_running(c) * c->m;
    reset_maxbits(c);
    set_active(c, active);
    if (diis) diis_before(c, amp_of, active);
    tau_run(c, TAU_STEP, panel);
    std::vector<double> mb = read_maxbits(c);
    trace_sweep("forward", panel, it, mb);
    bool any = false;
    for (int i = 0; i < B; ++i) {
      if (!active[i]) continue;
      its[i] = it;
      const double chg = mb[2 * i], val = mb[2 * i + 1];
      if (!std::isfinite(chg) || !std::isfinite(val)) {
        status[i] = FTCC_ENONFINITE;
        active[i] = false;
        continue;
      }
      if (chg <= c->opt.tol * std::max(1.0, val)) {
        active[i] = false;
        continue;
      }
      if (watch[i].diverged(chg)) {
        status[i] = FTCC_EDIVERGE;
        active[i] = false;
        continue;
      }
      any = true;
    }
    if (!any) break;
    set_run(c, active);
    if (diis) diis_after(c, amp_of, active);
    if (it == c->opt.max_iter)
      for (int i = 0; i < B; ++i)
        if (active[i]) status[i] = FTCC_ENOCONV;
  }
  // residuals at the final amplitudes of every instance still in good standing
  std::vector<bool> ok(B);
  for (int i = 0; i < B; ++i) ok[i] = status[i] == 0;
  set_run(c, ok);
  forward(c);
  c->resid_evals += n_running(c) * c->m;
  run_all(c);
  return its;
}

}  // namespace host
}  // namespace ftcc

// ------------------------------------------------------------------ ABI
extern "C" {

void ftcc_default_options(ftcc_options* opt) {
  if (!opt) return;
  opt->n_tau = 16;
  opt->nodes_per_panel = 4;
  opt->propagator = 0;
  opt->occ_thresh = 0.0;
  opt->tol = 1e-12;
  opt->max_iter = 200;
  opt->checkpoint = 0;
  opt->diis_depth = 0;
  opt->mem_cap_bytes = 0;
  opt->spin_orbital = 0;
}

int ftcc_abi_version(void) { return FTCC_ABI_VERSION; }

const char* ftcc_last_error(void) { return g_err.c_str(); }

int ftcc_create(ftcc_ctx** out, int device, int n_instances, const ftcc_options* opt) {
  return run_guarded([&] {
    if (!out || n_instances <= 0) fail(FTCC_EINVAL, "ftcc_create: bad arguments");
    ftcc_options o;
    ftcc_default_options(&o);
    if (opt) o = *opt;
    if (o.propagator < 0 || o.propagator > 5) fail(FTCC_EINVAL, "propagator must be 0..5");
    const bool rk = o.propagator >= 2 && o.propagator <= 4;
    const bool simpson = o.propagator == 5;
    if (rk || simpson) {
      if (o.n_tau < 2 || o.n_tau % 2) fail(FTCC_EINVAL, "the uniform-grid forms need an even n_tau >= 2 (Simpson)");
      if (o.diis_depth != 0) fail(FTCC_EINVAL, "diis_depth applies to the Gauss-Legendre integral form only");
    } else {
      if (o.nodes_per_panel < 1 || o.nodes_per_panel > kMaxNodes)
        fail(FTCC_EINVAL, "nodes_per_panel must be 1..6");
      if (o.n_tau < o.nodes_per_panel || o.n_tau % o.nodes_per_panel)
        fail(FTCC_EINVAL, "n_tau must be a positive multiple of nodes_per_panel");
    }
    if (!(o.tol > 0.0) || o.max_iter < 1) fail(FTCC_EINVAL, "tol must be > 0 and max_iter >= 1");
    if (!(o.occ_thresh >= 0.0)) fail(FTCC_EINVAL, "occ_thresh must be >= 0");
    if (o.spin_orbital != 0 && o.spin_orbital != 1) fail(FTCC_EINVAL, "spin_orbital must be 0 or 1");
    if (o.diis_depth < 0 || o.diis_depth == 1 || o.diis_depth > kMaxDiis)
      fail(FTCC_EINVAL, "diis_depth must be 0 (plain fixed-point sweeps) or 2..8");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) fail(FTCC_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) fail(FTCC_EINVAL, "device index out of range");
    FTCC_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    FTCC_HIP(hipGetDeviceProperties(&prop, device));
    if (std::string(prop.gcnArchName).rfind("gfx950", 0) != 0)
      fail(FTCC_EDEVICE, std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    FTCC_HIP(init_tau_constants());
    noalloc_setup(device);
    std::unique_ptr<ftcc_ctx> c(new ftcc_ctx());
    c->device = device;
    c->opt = o;
    c->gdeg = o.spin_orbital ? 1.0 : 2.0;
    c->B = n_instances;
    if (rk) {
      // Butcher tableaus: forward Euler, explicit trapezoid (Heun), classical RK4
      c->rk = true;
      if (o.propagator == 2) {
        c->rk_b = {1.0};
      } else if (o.propagator == 3) {
        c->rk_b = {0.5, 0.5};
      } else {
        c->rk_b = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
      }
      c->m = (int)c->rk_b.size();
      c->rk_a.assign(c->m * c->m, 0.0);
      if (c->m == 2) c->rk_a[1 * 2 + 0] = 1.0;
      if (c->m == 4) {
        c->rk_a[1 * 4 + 0] = 0.5;
        c->rk_a[2 * 4 + 1] = 0.5;
        c->rk_a[3 * 4 + 2] = 1.0;
      }
      c->P = o.n_tau;
      c->rule = make_rule(c->m, 0);   // unused by the march; keeps the device rule valid
    } else if (simpson) {
      c->simpson = true;
      c->m = 1;
      c->P = o.n_tau;
      c->rule = make_rule(1, 0);      // unused by the march; keeps the device rule valid
    } else {
      c->m = o.nodes_per_panel;
      c->P = o.n_tau / o.nodes_per_panel;
      c->rule = make_rule(c->m, o.propagator);
    }
    c->inst.resize(n_instances);
    FTCC_HIP(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking));
    c->stream = c->own_stream;
    *out = c.release();
  });
}

int ftcc_destroy(ftcc_ctx* c) {
  if (!c) return FTCC_OK;
  return run_guarded([&] {
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    clear_tau_cache(c);
    if (c->g_fwd) (void)hipGraphExecDestroy(c->g_fwd);
    if (c->g_bwd) (void)hipGraphExecDestroy(c->g_bwd);
    c->ex_main.reset();
    c->ex_d.reset();
    c->ex_g.reset();
    for (void* p : c->allocs) {
      if (c->ufree) c->ufree(p, c->uuser);
      else if (!c->ualloc) (void)hipFree(p);
    }
    if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
    delete c;
  });
}

int ftcc_set_stream(ftcc_ctx* c, void* s) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    c->stream = s ? (hipStream_t)s : c->own_stream;
  });
}

int ftcc_set_allocator(ftcc_ctx* c, ftcc_alloc_fn alloc, ftcc_free_fn free_fn, void* user) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    if (!c->allocs.empty()) fail(FTCC_ESTATE, "set the allocator before the first ftcc_set_hamiltonian");
    c->ualloc = alloc;
    c->ufree = alloc ? free_fn : nullptr;
    c->uuser = alloc ? user : nullptr;
  });
}

int ftcc_set_momentum(ftcc_ctx* c, int i, int n, int dims, const int* labels, const int* modulus) {
  return run_guarded([&] {
    if (!c || !labels || !modulus) fail(FTCC_EINVAL, "null argument");
    if (i < 0 || i >= c->B) fail(FTCC_EINVAL, "instance index out of range");
    if (c->built) fail(FTCC_ESTATE, "momentum labels must be set before the first solve");
    if (n < 1 || n > 255) fail(FTCC_EINVAL, "n must be 1..255");
    if (dims < 1 || dims > 3) fail(FTCC_EINVAL, "dims must be 1..3");
    Instance& I = c->inst[i];
    if (I.has_ham && I.n != n) fail(FTCC_EINVAL, "n differs from the instance's Hamiltonian");
    for (int d = 0; d < dims; ++d)
      if (modulus[d] < 0) fail(FTCC_EINVAL, "modulus must be >= 0");
    for (long k = 0; k < (long)n * dims; ++k)
      if (labels[k] <= -(1 << 16) || labels[k] >= (1 << 16)) fail(FTCC_EINVAL, "labels must lie in (-65536, 65536)");
    I.mom.dims = dims;
    I.mom.modulus.assign(modulus, modulus + dims);
    I.mom.labels.assign(labels, labels + (long)n * dims);
    if (!I.has_ham) I.n = n;
  });
}

int ftcc_set_hamiltonian(ftcc_ctx* c, int i, int n, const double* h, const double* eri, const double* eps) {
  return run_guarded([&] {
    if (!c || !h || !eri || !eps) fail(FTCC_EINVAL, "null argument");
    if (i < 0 || i >= c->B) fail(FTCC_EINVAL, "instance index out of range");
    if (n < 1 || n > 256) fail(FTCC_EINVAL, "n must be 1..256");
    FTCC_HIP(hipSetDevice(c->device));
    Instance& I = c->inst[i];
    if (c->built && n != I.n) fail(FTCC_EINVAL, "n cannot change after the first solve");
    const long n2 = (long)n * n, n4 = n2 * n2;
    for (long k = 0; k < n2; ++k)
      if (!std::isfinite(h[k])) fail(FTCC_EINVAL, "h has a non-finite entry");
    for (long k = 0; k < n; ++k)
      if (!std::isfinite(eps[k])) fail(FTCC_EINVAL, "eps has a non-finite entry");
    for (long k = 0; k < n4; ++k)
      if (!std::isfinite(eri[k])) fail(FTCC_EINVAL, "eri has a non-finite entry");
    if (I.mom.dims && (long)I.mom.labels.size() != (long)n * I.mom.dims)
      fail(FTCC_EINVAL, "n differs from the instance's momentum labels");
    if (!I.h) {
      I.n = n;
      I.h = c->dalloc(n2);
      I.eri = c->dalloc(n4);
      I.eps = c->dalloc(n);
    }
    FTCC_HIP(hipMemcpy(I.h, h, sizeof(double) * n2, hipMemcpyHostToDevice));
    FTCC_HIP(hipMemcpy(I.eri, eri, sizeof(double) * n4, hipMemcpyHostToDevice));
    FTCC_HIP(hipMemcpy(I.eps, eps, sizeof(double) * n, hipMemcpyHostToDevice));
    I.eps_host.assign(eps, eps + n);
    if (c->built && momentum_on(c)) {   // a new Hamiltonian must keep the declared conservation law
      check_momentum(c, i, I.h, 2, "h");
      check_momentum(c, i, I.eri, 4, "<pq|rs>");
    }
    I.has_ham = true;
    c->solved = false;
    c->have_lambda = false;
  });
}

int ftcc_solve_amplitudes(ftcc_ctx* c, const double* mu, const double* beta, int* iters_out, int* status_out) {
  int any_fail = 0;
  int rc = run_guarded([&] {
    if (!c || !mu || !beta) fail(FTCC_EINVAL, "null argument");
    FTCC_HIP(hipSetDevice(c->device));
    for (int i = 0; i < c->B; ++i)
      if (!std::isfinite(mu[i]) || !(beta[i] > 0.0) || !std::isfinite(beta[i]))
        fail(FTCC_EINVAL, "mu must be finite and beta positive");
    build(c);
    clear_tau_cache(c);
    const int B = c->B, m = c->m, P = c->P;
    auto lenof = [c](int i) { const long n = c->inst[i].n; return n * n + n * n * n * n; };
    hipEvent_t e0, e1;
    FTCC_HIP(hipEventCreate(&e0));
    FTCC_HIP(hipEventCreate(&e1));
    FTCC_HIP(hipEventRecord(e0, c->stream));
    c->resid_evals = 0;
    for (int i = 0; i < B; ++i) {
      Instance& I = c->inst[i];
      I.mu = mu[i];
      I.beta = beta[i];
      thermal_setup(c, i);
      zero_d(c, I.sb[0], lenof(i));
      I.iters = 0;
      I.status = 0;
    }
    c->ex_main->run_setup(c->stream);
    std::vector<int> status(B, 0), total(B, 0);
    std::vector<double> ebuf(B * m);
    const auto wall0 = std::chrono::steady_clock::now();
    if (c->rk) rk_solve(c, status);
    if (c->simpson) simpson_solve(c, status, total);
    for (int p = 0; p < ((c->rk || c->simpson) ? 0 : P); ++p) {
      std::vector<int> its = panel_solve(c, p, status);
      for (int i = 0; i < B; ++i) total[i] += its[i];
      for (int i = 0; i < B; ++i) {
        Instance& I = c->inst[i];
        for (int x = 0; x < m; ++x) {
          FTCC_HIP(hipMemcpyAsync(&ebuf[i * m + x], c->e[i * m + x], sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream));
          if (!c->opt.checkpoint) {
            copy_d(c, I.grid[p * m + x], c->amp[i * m + x], lenof(i));
            copy_d(c, I.resid[p * m + x], c->S[i * m + x], lenof(i));
          }
        }
      }
      tau_run(c, TAU_END, p);
      sync(c);
      for (int i = 0; i < B; ++i)
        for (int x = 0; x < m; ++x) c->inst[i].energies[p * m + x] = ebuf[i * m + x];
      trace(c, "forward", p + 1, P, its, wall0);
    }
    FTCC_HIP(hipEventRecord(e1, c->stream));
    sync(c);
    float ms = 0.f;
    FTCC_HIP(hipEventElapsedTime(&ms, e0, e1));
    c->t_solve = ms * 1e-3;
    FTCC_HIP(hipEventDestroy(e0));
    FTCC_HIP(hipEventDestroy(e1));
    for (int i = 0; i < B; ++i) {
      Instance& I = c->inst[i];
      double mf[5];
      FTCC_HIP(hipMemcpy(mf, I.mf, sizeof(mf), hipMemcpyDeviceToHost));
      I.omega0 = mf[0];
      I.omega1 = mf[1];
      if (!c->rk && !c->simpson) {
        double occ_cc = 0.0;
        for (int p = 0; p < P; ++p)
          for (int x = 0; x < m; ++x) occ_cc += c->rule.b[x] / P * I.energies[p * m + x];
        // an instance whose march failed has no grand potential
        I.omega_cc = status[i] == 0 ? occ_cc : std::nan("");
        I.iters = total[i];
      }
      I.status = status[i];
      if (iters_out) iters_out[i] = I.iters;
      if (status_out) status_out[i] = status[i];
      if (status[i] != 0) any_fail = status[i];
    }
    c->solved = true;
    c->have_lambda = false;
  });
  if (rc == FTCC_OK && any_fail) {
    g_err = "at least one instance did not converge (see status_out)";
    return any_fail;
  }
  return rc;
}

int ftcc_grand_potential(ftcc_ctx* c, double* omega, double* parts) {
  return run_guarded([&] {
    if (!c || !omega) fail(FTCC_EINVAL, "null argument");
    if (!c->solved) fail(FTCC_ESTATE, "call ftcc_solve_amplitudes first");
    for (int i = 0; i < c->B; ++i) {
      const Instance& I = c->inst[i];
      omega[i] = I.omega0 + I.omega1 + I.omega_cc;
      if (parts) {
        parts[3 * i] = I.omega0;
        parts[3 * i + 1] = I.omega1;
        parts[3 * i + 2] = I.omega_cc;
      }
    }
  });
}

int ftcc_get_amplitudes(ftcc_ctx* c, int i, int k, double* t1, double* t2) {
  return run_guarded([&] {
    if (!c || !t1 || !t2) fail(FTCC_EINVAL, "null argument");
    if (!c->solved) fail(FTCC_ESTATE, "call ftcc_solve_amplitudes first");
    const bool uniform = c->rk || c->simpson;
    if (c->opt.checkpoint && !uniform) fail(FTCC_ESTATE, "amplitudes are not kept with checkpoint = 1");
    // uniform-grid forms: the grid states s(tau_k), k = 0..n_tau
    if (i < 0 || i >= c->B || k < 0 || k >= c->opt.n_tau + (uniform ? 1 : 0)) fail(FTCC_EINVAL, "index out of range");
    const long n = c->inst[i].n, n2 = n * n;
    FTCC_HIP(hipSetDevice(c->device));
    sync(c);
    const double* src = uniform ? c->inst[i].sb[k] : c->inst[i].grid[k];
    FTCC_HIP(hipMemcpy(t1, src, sizeof(double) * n2, hipMemcpyDeviceToHost));
    FTCC_HIP(hipMemcpy(t2, src + n2, sizeof(double) * n2 * n2, hipMemcpyDeviceToHost));
  });
}

}  // extern "C"

namespace ftcc {
namespace host {

// Bring the converged amplitudes of panel p into the slots and evaluate the
// forward program there (tape for the backward, residuals in S).
// Leaves the run flags on the instances whose forward march succeeded.
void load_panel(ftcc_ctx* c, int p) {
  const int B = c->B, m = c->m;
  std::vector<int> st(B);
  std::vector<bool> ok(B);
  for (int i = 0; i < B; ++i) {
    st[i] = c->inst[i].status;
    ok[i] = st[i] == 0;
  }
  if (!c->opt.checkpoint) {
    for (int i = 0; i < B; ++i) {
      const long n = c->inst[i].n, len = n * n + n * n * n * n;
      for (int x = 0; x < m; ++x) copy_d(c, c->amp[i * m + x], c->inst[i].grid[p * m + x], len);
    }
    set_run(c, ok);
    forward(c);
  } else {
    panel_solve(c, p, st);   // deterministic: reproduces the forward sweep
    set_run(c, ok);
  }
}

}  // namespace host
}  // namespace ftcc

extern "C" {

int ftcc_lambda(ftcc_ctx* c, int* iters_out, int* status_out) {
  int any_fail = 0;
  int rc = run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    if (!c->solved) fail(FTCC_ESTATE, "call ftcc_solve_amplitudes first");
    FTCC_HIP(hipSetDevice(c->device));
    const int B = c->B, m = c->m, P = c->P;
    for (int i = 0; i < B && !c->simpson; ++i) {   // a_P = 0 (the Simpson form keeps S[s_P] there)
      Instance& I = c->inst[i];
      const long n = I.n, len = n * n + n * n * n * n;
      zero_d(c, I.abuf[P], len);
    }
    hipEvent_t e0, e1;
    FTCC_HIP(hipEventCreate(&e0));
    FTCC_HIP(hipEventCreate(&e1));
    FTCC_HIP(hipEventRecord(e0, c->stream));
    c->vjp_evals = 0;
    std::vector<int> total(B, 0), status(B, 0);
    for (int i = 0; i < B; ++i) status[i] = c->inst[i].status;   // a failed forward march has no adjoint
    const auto wall0 = std::chrono::steady_clock::now();
    if (c->rk) {
      rk_lambda(c, status);
      for (int i = 0; i < B; ++i) total[i] = P;
    }
    if (c->simpson) simpson_lambda(c, status, total);
    for (int p = ((c->rk || c->simpson) ? -1 : P - 1); p >= 0; --p) {
      const std::vector<int> before = total;
      load_panel(c, p);
      // lambda_x = -(g_x/beta) dE/ds : backward with zero S-cotangent
      for (int q = 0; q < B * m; ++q) {
        const long n = c->inst[q / m].n;
        zero_d(c, c->cot[q], n * n + n * n * n * n);
      }
      backward(c);
      c->vjp_evals += n_running(c) * m;
      reset_maxbits(c);
      std::vector<bool> active(B);
      for (int i = 0; i < B; ++i) active[i] = c->inst[i].status == 0;
      set_active(c, active);
      tau_run(c, TAU_LSTEP, p);
      const bool diis = c->opt.diis_depth > 0;
      NodeBufs lam_of = [c, p](int i, int x) { return c->inst[i].lam[p * c->m + x]; };
      if (diis) diis_reset(c);
      std::vector<DivergenceWatch> watch(B);
      for (int it = 1; it <= c->opt.max_iter; ++it) {
        tau_run(c, TAU_LAMT, p);
        backward(c);
        c->vjp_evals += n_running(c) * m;
        reset_maxbits(c);
        set_active(c, active);
        if (diis) diis_before(c, lam_of, active);
        tau_run(c, TAU_LSTEP, p);
        std::vector<double> mb = read_maxbits(c);
        trace_sweep("lambda", p, it, mb);
        bool any = false;
        for (int i = 0; i < B; ++i) {
          if (!active[i]) continue;
          total[i] += 1;
          const double chg = mb[2 * i], val = mb[2 * i + 1];
          if (!std::isfinite(chg) || !std::isfinite(val)) {
            status[i] = FTCC_ENONFINITE;
            active[i] = false;
            continue;
          }
          if (chg <= c->opt.tol * std::max(val, 1e-30) || chg == 0.0) {
            active[i] = false;
            continue;
          }
          if (watch[i].diverged(chg)) {
            status[i] = FTCC_EDIVERGE;
            active[i] = false;
            continue;
          }
          any = true;
        }
        if (!any) break;
        set_run(c, active);
        if (diis) diis_after(c, lam_of, active);
        if (it == c->opt.max_iter)
          for (int i = 0; i < B; ++i)
            if (active[i]) status[i] = FTCC_ENOCONV;
      }
      run_all(c);
      tau_run(c, TAU_APREV, p);
      if (trace_on()) {
        sync(c);
        std::vector<int> sw(B);
        for (int i = 0; i < B; ++i) sw[i] = total[i] - before[i];
        trace(c, "lambda", P - p, P, sw, wall0);
      }
    }
    FTCC_HIP(hipEventRecord(e1, c->stream));
    sync(c);
    float ms = 0.f;
    FTCC_HIP(hipEventElapsedTime(&ms, e0, e1));
    c->t_lambda = ms * 1e-3;
    FTCC_HIP(hipEventDestroy(e0));
    FTCC_HIP(hipEventDestroy(e1));
    for (int i = 0; i < B; ++i) {
      c->inst[i].lam_iters = total[i];
      c->inst[i].lam_status = status[i];
      if (iters_out) iters_out[i] = total[i];
      if (status_out) status_out[i] = status[i];
      if (status[i]) any_fail = status[i];
    }
    c->have_lambda = true;
  });
  if (rc == FTCC_OK && any_fail) {
    g_err = "at least one instance did not converge in the adjoint (see status_out)";
    return any_fail;
  }
  return rc;
}

int ftcc_get_lambda(ftcc_ctx* c, int i, int k, double* l1, double* l2, double* lt1, double* lt2) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    if (!c->have_lambda) fail(FTCC_ESTATE, "call ftcc_lambda first");
    if (c->simpson) {
      // Simpson integral form: lambda of grid point k, k = 0..n_tau (lambda_0 = 0)
      if (i < 0 || i >= c->B || k < 0 || k > c->opt.n_tau) fail(FTCC_EINVAL, "index out of range");
      const long n = c->inst[i].n, n2 = n * n;
      FTCC_HIP(hipSetDevice(c->device));
      if (lt1 || lt2) {
        run_all(c);
        simpson_lamt(c, k);
      }
      sync(c);
      if (l1) FTCC_HIP(hipMemcpy(l1, c->inst[i].lam[k], sizeof(double) * n2, hipMemcpyDeviceToHost));
      if (l2) FTCC_HIP(hipMemcpy(l2, c->inst[i].lam[k] + n2, sizeof(double) * n2 * n2, hipMemcpyDeviceToHost));
      if (lt1) FTCC_HIP(hipMemcpy(lt1, c->cot[i * c->m], sizeof(double) * n2, hipMemcpyDeviceToHost));
      if (lt2) FTCC_HIP(hipMemcpy(lt2, c->cot[i * c->m] + n2, sizeof(double) * n2 * n2, hipMemcpyDeviceToHost));
      return;
    }
    if (c->rk) {
      // differential form: the cotangent of the grid state s(tau_k), k = 0..n_tau
      if (i < 0 || i >= c->B || k < 0 || k > c->opt.n_tau) fail(FTCC_EINVAL, "index out of range");
      if (lt1 || lt2) fail(FTCC_EINVAL, "the differential form has no lambda-tilde");
      const long n = c->inst[i].n, n2 = n * n;
      FTCC_HIP(hipSetDevice(c->device));
      sync(c);
      if (l1) FTCC_HIP(hipMemcpy(l1, c->inst[i].abuf[k], sizeof(double) * n2, hipMemcpyDeviceToHost));
      if (l2) FTCC_HIP(hipMemcpy(l2, c->inst[i].abuf[k] + n2, sizeof(double) * n2 * n2, hipMemcpyDeviceToHost));
      return;
    }
    if (i < 0 || i >= c->B || k < 0 || k >= c->opt.n_tau) fail(FTCC_EINVAL, "index out of range");
    const long n = c->inst[i].n, n2 = n * n;
    FTCC_HIP(hipSetDevice(c->device));
    sync(c);
    if (l1) FTCC_HIP(hipMemcpy(l1, c->inst[i].lam[k], sizeof(double) * n2, hipMemcpyDeviceToHost));
    if (l2) FTCC_HIP(hipMemcpy(l2, c->inst[i].lam[k] + n2, sizeof(double) * n2 * n2, hipMemcpyDeviceToHost));
    if (lt1 || lt2) {
      tau_run(c, TAU_LAMT, k / c->m);
      sync(c);
      const double* src = c->cot[i * c->m + k % c->m];
      if (lt1) FTCC_HIP(hipMemcpy(lt1, src, sizeof(double) * n2, hipMemcpyDeviceToHost));
      if (lt2) FTCC_HIP(hipMemcpy(lt2, src + n2, sizeof(double) * n2 * n2, hipMemcpyDeviceToHost));
    }
  });
}

// Descriptors of the grouped response accumulation (collocation panels): the
// node buffers are fixed for the context, so they are uploaded once.
static void ensure_resp_groups(ftcc_ctx* c) {
  if (c->d_resp_dots) return;
  const int B = c->B, m = c->m, P = c->P;
  std::vector<DotProblem> ds(B * m);
  std::vector<const double*> de(B * m), ugs((size_t)B * 4 * m);
  std::vector<double*> acc(B), ugd((size_t)B * 4);
  std::vector<long> n2(B);
  std::vector<double> w(m);
  c->d_resp_vals = c->dalloc(B * m);
  for (int x = 0; x < m; ++x) w[x] = c->rule.b[x] / P;
  for (int i = 0; i < B; ++i) {
    const long n = c->inst[i].n;
    n2[i] = n * n;
    c->max_n2 = std::max(c->max_n2, n2[i]);
    acc[i] = c->inst[i].acc;
    for (int k = 0; k < 4; ++k) ugd[i * 4 + k] = c->inst[i].ugrad_acc[k];
    for (int x = 0; x < m; ++x) {
      const int q = i * m + x;
      DotProblem d{};
      d.X = c->cot[q];
      d.Y = c->dS[q];
      d.out = c->d_resp_vals + q;
      d.len = n * n + n * n * n * n;
      if (c->inst[i].d_allowed[0]) {   // momentum labels: the allowed elements only
        d.ia = c->inst[i].d_allowed[0];
        d.na = c->inst[i].n_allowed[0];
        d.ib = c->inst[i].d_allowed[1];
        d.nb = c->inst[i].n_allowed[1];
        d.second = n * n;
      }
      d.alpha = 1.0;
      d.beta = 0.0;
      ds[q] = d;
      de[q] = c->de[q];
      for (int k = 0; k < 4; ++k) ugs[((size_t)i * 4 + k) * m + x] = c->ugrad[q][k];
    }
  }
  auto up = [c](const void* h, size_t bytes) {
    double* d = c->dalloc((bytes + 7) / 8);
    FTCC_HIP(hipMemcpy(d, h, bytes, hipMemcpyHostToDevice));
    return (void*)d;
  };
  c->d_resp_dots = (DotProblem*)up(ds.data(), sizeof(DotProblem) * ds.size());
  c->d_resp_w = (double*)up(w.data(), sizeof(double) * w.size());
  c->d_de_ptrs = (const double**)up(de.data(), sizeof(double*) * de.size());
  c->d_acc_ptrs = (double**)up(acc.data(), sizeof(double*) * acc.size());
  c->d_ug_src = (const double**)up(ugs.data(), sizeof(double*) * ugs.size());
  c->d_ug_dst = (double**)up(ugd.data(), sizeof(double*) * ugd.size());
  c->d_n2 = (long*)up(n2.data(), sizeof(long) * n2.size());
}

int ftcc_response(ftcc_ctx* c, double* dO_dmu, double* dO_dbeta, double* dO_dh, double* dO_deps,
                  const double* const* deri_dtheta, const double* const* dh_dtheta, double* dO_dtheta) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    if (!c->have_lambda) fail(FTCC_ESTATE, "call ftcc_lambda first");
    FTCC_HIP(hipSetDevice(c->device));
    const int B = c->B, m = c->m, P = c->P;
    int nmax = 0;
    for (int i = 0; i < B; ++i) nmax = std::max(nmax, c->inst[i].n);
    if (dO_deps) {
      for (int i = 0; i < B; ++i) {
        Instance& I = c->inst[i];
        const long n = I.n;
        if (!I.deps_acc) {
          I.deps_acc = c->dalloc(n);
          I.deps_out = c->dalloc(n);
          I.deps_dh = c->dalloc(n * n);
          I.deps_delta = c->dalloc(node_len(c, i));
        }
        zero_d(c, I.deps_acc, n);
        zero_d(c, I.deps_delta, node_len(c, i));
      }
    }
    const bool want_theta = dO_dtheta && (deri_dtheta || dh_dtheta);
    // device copies of the theta directions
    std::vector<double*> d_deri(B, nullptr), d_dh(B, nullptr);
    // freed when the call ends, also when it ends with an error
    struct DeviceTemps {
      hipStream_t s;
      std::vector<void*> p;
      void push_back(void* x) { p.push_back(x); }
      ~DeviceTemps() {
        if (p.empty()) return;
        (void)hipStreamSynchronize(s);
        for (void* x : p) (void)hipFree(x);
      }
    } tmp{c->stream, {}};
    if (want_theta) {
      for (int i = 0; i < B; ++i) {
        const long n = c->inst[i].n, n2 = n * n, n4 = n2 * n2;
        if (deri_dtheta && deri_dtheta[i]) {
          FTCC_HIP(hipMalloc((void**)&d_deri[i], sizeof(double) * n4));
          tmp.push_back(d_deri[i]);
          FTCC_HIP(hipMemcpy(d_deri[i], deri_dtheta[i], sizeof(double) * n4, hipMemcpyHostToDevice));
          if (momentum_on(c)) check_momentum(c, i, d_deri[i], 4, "deri_dtheta");
        }
        if (dh_dtheta && dh_dtheta[i]) {
          FTCC_HIP(hipMalloc((void**)&d_dh[i], sizeof(double) * n2));
          tmp.push_back(d_dh[i]);
          FTCC_HIP(hipMemcpy(d_dh[i], dh_dtheta[i], sizeof(double) * n2, hipMemcpyHostToDevice));
          if (momentum_on(c)) check_momentum(c, i, d_dh[i], 2, "dh_dtheta");
        }
      }
    }
    for (int i = 0; i < B; ++i) {
      const long n = c->inst[i].n;
      zero_d(c, c->inst[i].acc, 8);
      for (int k = 0; k < 4; ++k) zero_d(c, c->inst[i].ugrad_acc[k], n * n);
    }
    // dot launches: <lamt_x, dS_x> and (g_x/beta) dE_x accumulated into acc[slot]
    // all (instance, node) dots in one launch, then the node sums per instance
    auto accumulate = [&](int slot) {
      ensure_resp_groups(c);
      launch_dot(c->d_resp_dots, B * m, 64, c->scratch.dot_partial, c->stream);
      hipLaunchKernelGGL(resp_combine_kernel, dim3((B + 63) / 64), dim3(64), 0, c->stream, B, m,
                         (const double*)c->d_resp_vals, c->d_de_ptrs, (const double*)c->d_resp_w, c->d_acc_ptrs, slot);
      FTCC_HIP(hipGetLastError());
    };
    // the same for the orbital-energy direction q: into deps_acc[q] of the
    // instances with more than q orbitals
    auto accumulate_eps = [&](int q) {
      for (int i = 0; i < B; ++i) {
        if (q >= c->inst[i].n) continue;
        const long n = c->inst[i].n;
        for (int x = 0; x < m; ++x) {
          DotProblem d{};
          d.X = c->cot[i * m + x];
          d.Y = c->dS[i * m + x];
          d.out = c->inst[i].deps_acc + q;
          d.len = n * n + n * n * n * n;
          if (c->inst[i].d_allowed[0]) {
            d.ia = c->inst[i].d_allowed[0];
            d.na = c->inst[i].n_allowed[0];
            d.ib = c->inst[i].d_allowed[1];
            d.nb = c->inst[i].n_allowed[1];
            d.second = n * n;
          }
          d.alpha = 1.0;
          d.beta = 1.0;
          DotProblem* dd = nullptr;
          FTCC_HIP(hipMallocAsync((void**)&dd, sizeof(DotProblem), c->stream));
          FTCC_HIP(hipMemcpyAsync(dd, &d, sizeof(DotProblem), hipMemcpyHostToDevice, c->stream));
          launch_dot(dd, 1, 64, c->scratch.dot_partial, c->stream);
          FTCC_HIP(hipFreeAsync(dd, c->stream));
          launch_axpby(1, c->rule.b[x] / P, c->de[i * m + x], 1.0, c->inst[i].deps_acc + q, c->stream);
        }
      }
    };
    const auto wall0 = std::chrono::steady_clock::now();
    if (c->rk) {
      // differential form: every grid point k (energy weight) and every stage of
      // step k (cotangent -kbar of its residual)
      std::vector<bool> ok(B);
      for (int i = 0; i < B; ++i) ok[i] = c->inst[i].status == 0 && c->inst[i].lam_status == 0;
      set_run(c, ok);
      for (int k = 0; k <= P; ++k) {
        const int ns = k < P ? m : 1;
        const double wk = ((k == 0 || k == P) ? 1.0 : (k % 2 ? 4.0 : 2.0)) / (3.0 * P);
        if (k < P) rk_recompute_stages(c, k);
        else rk_stage_state(c, P, 0);
        for (int x = 0; x < ns; ++x) {
          if (k < P) {
            rk_combine(c, 7, k, x, 0.0, false, [c, k, x](int i) {
              RKSpec sp;
              sp.base = c->inst[i].lam[k * c->m + x];
              sp.x0 = -1.0;
              sp.out = c->cot[i * c->m + x];
              return sp;
            });
          } else {
            for (int i = 0; i < B; ++i)
              if (ok[i]) zero_d(c, c->cot[i * m], node_len(c, i));
          }
          set_ebar(c, x, x == 0 ? k : -1);
          if (dO_dh) {
            backward_one(c, x);
            for (int i = 0; i < B; ++i) {
              if (!ok[i]) continue;
              const long n = c->inst[i].n;
              for (int q = 0; q < 4; ++q)
                launch_axpby(n * n, 1.0, c->ugrad[i * m + x][q], 1.0, c->inst[i].ugrad_acc[q], c->stream);
            }
          }
          for (int which = 0; which < 3; ++which) {
            if (which == 0 && !dO_dmu) continue;
            if (which == 1 && !dO_dbeta) continue;
            if (which == 2 && !want_theta) continue;
            for (int i = 0; i < B; ++i) deriv_setup(c, i, which, d_dh[i], d_deri[i]);
            c->ex_d->run_setup(c->stream);
            d_forward_one(c, x);
            rk_dot(c, 2 + which, k, x, [c, x, which](int i) {
              return std::array<const double*, 3>{c->cot[i * c->m + x], c->dS[i * c->m + x],
                                                  c->inst[i].acc + which};
            });
            if (x == 0)
              for (int i = 0; i < B; ++i)
                if (ok[i]) launch_axpby(1, wk, c->de[i * m], 1.0, c->inst[i].acc + which, c->stream);
          }
          if (dO_deps) {
            // the slopes' Delta dependence, d k / d Delta = -Y, weighted by the slope
            // cotangent: cot = -kbar, so dL/dDelta += cot * Y (stage state in amp)
            if (k < P)
              for (int i = 0; i < B; ++i) {
                if (!ok[i]) continue;
                const long len = node_len(c, i);
                hipLaunchKernelGGL(mul_acc_kernel, dim3((unsigned)std::min<long>((len + 255) / 256, 65536)),
                                   dim3(256), 0, c->stream, len, c->cot[i * m + x], c->amp[i * m + x],
                                   c->inst[i].deps_delta);
              }
            for (int q = 0; q < nmax; ++q) {
              for (int i = 0; i < B; ++i)
                if (q < c->inst[i].n) deriv_setup_eps(c, i, q);
              c->ex_d->run_setup(c->stream);
              d_forward_one(c, x);
              for (int i = 0; i < B; ++i) {
                if (!ok[i] || q >= c->inst[i].n) continue;
                const long n = c->inst[i].n;
                DotProblem d{};
                d.X = c->cot[i * m + x];
                d.Y = c->dS[i * m + x];
                d.out = c->inst[i].deps_acc + q;
                d.len = n * n + n * n * n * n;
                d.alpha = 1.0;
                d.beta = 1.0;
                DotProblem* dd = nullptr;
                FTCC_HIP(hipMallocAsync((void**)&dd, sizeof(DotProblem), c->stream));
                FTCC_HIP(hipMemcpyAsync(dd, &d, sizeof(DotProblem), hipMemcpyHostToDevice, c->stream));
                launch_dot(dd, 1, 64, c->scratch.dot_partial, c->stream);
                FTCC_HIP(hipFreeAsync(dd, c->stream));
                if (x == 0) launch_axpby(1, wk, c->de[i * m], 1.0, c->inst[i].deps_acc + q, c->stream);
              }
            }
          }
        }
        if (trace_on()) {
          sync(c);
          trace(c, "response (Runge-Kutta)", k + 1, P + 1, std::vector<int>(1, 0), wall0);
        }
      }
      if (dO_dbeta)
        for (int i = 0; i < B; ++i) launch_axpby(1, 1.0 / P, c->inst[i].rk_hbar, 0.0, c->inst[i].acc + 3, c->stream);
    }
    if (c->simpson) {
      // Simpson integral form: every grid point x (energy weight g_x / beta and
      // cotangent lamt_x of its residual), then the grid terms of beta and Delta
      std::vector<bool> ok(B);
      for (int i = 0; i < B; ++i) ok[i] = c->inst[i].status == 0 && c->inst[i].lam_status == 0;
      set_run(c, ok);
      const std::vector<double> g = simpson_row(P);
      auto dot_into = [&](const double* X, const double* Y, std::function<double*(int)> out) {
        for (int i = 0; i < B; ++i) {
          if (!ok[i]) continue;
          DotProblem d{};
          d.X = X ? X : c->cot[i * m];
          d.Y = Y ? Y : c->dS[i * m];
          d.out = out(i);
          d.len = node_len(c, i);
          d.alpha = 1.0;
          d.beta = 1.0;
          DotProblem* dd = nullptr;
          FTCC_HIP(hipMallocAsync((void**)&dd, sizeof(DotProblem), c->stream));
          FTCC_HIP(hipMemcpyAsync(dd, &d, sizeof(DotProblem), hipMemcpyHostToDevice, c->stream));
          launch_dot(dd, 1, 64, c->scratch.dot_partial, c->stream);
          FTCC_HIP(hipFreeAsync(dd, c->stream));
        }
      };
      for (int x = 0; x <= P; ++x) {
        const double wx = g[x] / P;   // (1/beta) g_x
        simpson_lamt(c, x);
        for (int i = 0; i < B; ++i)
          if (ok[i]) node_copy(c, i, c->amp[i * m], c->inst[i].sb[x]);
        if (dO_dh) {
          set_ebar(c, 0, x);
          forward(c);
          backward(c);
          for (int i = 0; i < B; ++i) {
            if (!ok[i]) continue;
            const long n = c->inst[i].n;
            for (int k = 0; k < 4; ++k)
              launch_axpby(n * n, 1.0, c->ugrad[i * m][k], 1.0, c->inst[i].ugrad_acc[k], c->stream);
          }
        }
        for (int which = 0; which < 3; ++which) {
          if (which == 0 && !dO_dmu) continue;
          if (which == 1 && !dO_dbeta) continue;
          if (which == 2 && !want_theta) continue;
          for (int i = 0; i < B; ++i) deriv_setup(c, i, which, d_dh[i], d_deri[i]);
          c->ex_d->run_setup(c->stream);
          d_forward_one(c, 0);
          dot_into(nullptr, nullptr, [c, which](int i) { return c->inst[i].acc + which; });
          for (int i = 0; i < B; ++i)
            if (ok[i]) launch_axpby(1, wx, c->de[i * m], 1.0, c->inst[i].acc + which, c->stream);
        }
        if (dO_deps) {
          for (int q = 0; q < nmax; ++q) {
            for (int i = 0; i < B; ++i)
              if (q < c->inst[i].n) deriv_setup_eps(c, i, q);
            c->ex_d->run_setup(c->stream);
            d_forward_one(c, 0);
            for (int i = 0; i < B; ++i) {
              if (!ok[i] || q >= c->inst[i].n) continue;
              DotProblem d{};
              d.X = c->cot[i * m];
              d.Y = c->dS[i * m];
              d.out = c->inst[i].deps_acc + q;
              d.len = node_len(c, i);
              d.alpha = 1.0;
              d.beta = 1.0;
              DotProblem* dd = nullptr;
              FTCC_HIP(hipMallocAsync((void**)&dd, sizeof(DotProblem), c->stream));
              FTCC_HIP(hipMemcpyAsync(dd, &d, sizeof(DotProblem), hipMemcpyHostToDevice, c->stream));
              launch_dot(dd, 1, 64, c->scratch.dot_partial, c->stream);
              FTCC_HIP(hipFreeAsync(dd, c->stream));
              launch_axpby(1, wx, c->de[i * m], 1.0, c->inst[i].deps_acc + q, c->stream);
            }
          }
        }
      }
      for (int y = 1; y <= P; ++y) {
        if (dO_dbeta) {   // (1/n_g) sum_y <lam_y, sum_x d/dh[G^y_x e^{-Delta h (y-x)}] S_x>
          if (y == 1)
            for (int i = 0; i < B; ++i) zero_d(c, c->inst[i].rk_hbar, 1);
          simpson_grid_term(c, y, 1, [c](int i) { return c->inst[i].rk_tmp[0]; }, nullptr);
          for (int i = 0; i < B; ++i) {
            if (!ok[i]) continue;
            DotProblem d{};
            d.X = c->inst[i].lam[y];
            d.Y = c->inst[i].rk_tmp[0];
            d.out = c->inst[i].rk_hbar;
            d.len = node_len(c, i);
            d.alpha = 1.0;
            d.beta = 1.0;
            DotProblem* dd = nullptr;
            FTCC_HIP(hipMallocAsync((void**)&dd, sizeof(DotProblem), c->stream));
            FTCC_HIP(hipMemcpyAsync(dd, &d, sizeof(DotProblem), hipMemcpyHostToDevice, c->stream));
            launch_dot(dd, 1, 64, c->scratch.dot_partial, c->stream);
            FTCC_HIP(hipFreeAsync(dd, c->stream));
          }
        }
        if (dO_deps)      // dL/dDelta elementwise: lam_y * sum_x d/dDelta[G^y_x e^{-Delta h (y-x)}] S_x
          simpson_grid_term(c, y, 2, [c](int i) { return c->inst[i].deps_delta; },
                            [c, y](int i) { return (const double*)c->inst[i].lam[y]; });
      }
      if (dO_dbeta)
        for (int i = 0; i < B; ++i) launch_axpby(1, 1.0 / P, c->inst[i].rk_hbar, 0.0, c->inst[i].acc + 3, c->stream);
    }
    for (int p = 0; p < ((c->rk || c->simpson) ? 0 : P); ++p) {
      if (trace_on() && p > 0) {
        sync(c);
        trace(c, "response", p, P, std::vector<int>(1, 0), wall0);
      }
      load_panel(c, p);
      tau_run(c, TAU_LAMT, p);   // lambda-tilde of the panel into the cotangent buffers
      if (dO_dh) {
        backward(c);
        ensure_resp_groups(c);
        hipLaunchKernelGGL(ugrad_sum_kernel, dim3((unsigned)((c->max_n2 + 255) / 256), (unsigned)(4 * B)), dim3(256), 0,
                           c->stream, m, c->d_ug_src, c->d_ug_dst, (const long*)c->d_n2);
        FTCC_HIP(hipGetLastError());
      }
      // beta: explicit dependence of the propagator weights (needs S at converged s)
      if (dO_dbeta) {
        tau_run(c, TAU_BETA, p);
        // partial sums per (instance, segment) -> acc[3]
        for (int i = 0; i < B; ++i) {
          const long n2 = (long)c->inst[i].n * c->inst[i].n;
          const int nb1 = (int)((seg_len(c, i, 0) + 1023) / 1024), nb2 = (int)((seg_len(c, i, 1) + 1023) / 1024);
          launch_sum(c->d_partial + c->beta_part_off[i], nb1 + nb2, c->inst[i].acc + 4, c->stream);
          launch_axpby(1, 1.0 / P, c->inst[i].acc + 4, 1.0, c->inst[i].acc + 3, c->stream);
        }
      }
      for (int which = 0; which < 3; ++which) {
        if (which == 0 && !dO_dmu) continue;
        if (which == 1 && !dO_dbeta) continue;
        if (which == 2 && !want_theta) continue;
        for (int i = 0; i < B; ++i) deriv_setup(c, i, which, d_dh[i], d_deri[i]);
        c->ex_d->run_setup(c->stream);
        d_forward(c);
        accumulate(which);
      }
      if (dO_deps) {
        // the propagator weights' Delta dependence (elementwise), then one
        // derivative-integral evaluation per orbital energy
        tau_run(c, TAU_DEPS, p);
        for (int q = 0; q < nmax; ++q) {
          for (int i = 0; i < B; ++i)
            if (q < c->inst[i].n) deriv_setup_eps(c, i, q);
          c->ex_d->run_setup(c->stream);
          d_forward(c);
          accumulate_eps(q);
        }
      }
    }
    run_all(c);
    // mean-field parts and assembly
    std::vector<double> accs(8 * B), mfv(5 * B);
    for (int i = 0; i < B; ++i) {
      Instance& I = c->inst[i];
      const long n = I.n, n2 = n * n;
      hipLaunchKernelGGL(meanfield_kernel, dim3(1), dim3(256), 0, c->stream, (int)n, I.eps, I.h, I.eri, I.occ,
                         I.fock, I.mu, I.beta, d_dh[i], d_deri[i], c->gdeg, I.mf);
      FTCC_HIP(hipMemcpyAsync(&mfv[5 * i], I.mf, sizeof(double) * 5, hipMemcpyDeviceToHost, c->stream));
      FTCC_HIP(hipMemcpyAsync(&accs[8 * i], I.acc, sizeof(double) * 8, hipMemcpyDeviceToHost, c->stream));
      if (dO_dh) {
        double* dd = nullptr;
        FTCC_HIP(hipMallocAsync((void**)&dd, sizeof(double) * n2, c->stream));
        hipLaunchKernelGGL(dh_assemble_kernel, dim3((n2 + 255) / 256), dim3(256), 0, c->stream, (int)n, I.occ, I.wo,
                           I.wv, I.ugrad_acc[0], I.ugrad_acc[1], I.ugrad_acc[2], I.ugrad_acc[3], c->gdeg, dd);
        long off = 0;
        for (int k = 0; k < i; ++k) off += (long)c->inst[k].n * c->inst[k].n;
        FTCC_HIP(hipMemcpyAsync(dO_dh + off, dd, sizeof(double) * n2, hipMemcpyDeviceToHost, c->stream));
        FTCC_HIP(hipFreeAsync(dd, c->stream));
      }
    }
    if (dO_deps) {
      long off = 0;
      for (int i = 0; i < B; ++i) {
        Instance& I = c->inst[i];
        const int n = I.n;
        hipLaunchKernelGGL(deps_meanfield_kernel, dim3((n + 63) / 64), dim3(64), 0, c->stream, n, I.eps, I.occ,
                           I.fock, I.mu, I.beta, c->gdeg, I.deps_out);
        launch_axpby(n, 1.0, I.deps_acc, 1.0, I.deps_out, c->stream);
        hipLaunchKernelGGL(deps_reduce_kernel, dim3(n), dim3(256), 0, c->stream, n, I.deps_delta, I.deps_out);
        FTCC_HIP(hipGetLastError());
        FTCC_HIP(hipMemcpyAsync(dO_deps + off, I.deps_out, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
        off += n;
      }
    }
    sync(c);
    for (int i = 0; i < B; ++i) {
      if (dO_dmu) dO_dmu[i] = mfv[5 * i + 2] + accs[8 * i + 0];
      if (dO_dbeta) dO_dbeta[i] = mfv[5 * i + 3] + accs[8 * i + 1] + accs[8 * i + 3];
      if (want_theta) dO_dtheta[i] = mfv[5 * i + 4] + accs[8 * i + 2];
    }
  });
}


int ftcc_eval_residual(ftcc_ctx* c, int i, double mu, double beta, const double* t1, const double* t2, double* S1,
                       double* S2, double* E) {
  return run_guarded([&] {
    if (!c || !t1 || !t2) fail(FTCC_EINVAL, "null argument");
    if (i < 0 || i >= c->B) fail(FTCC_EINVAL, "instance index out of range");
    FTCC_HIP(hipSetDevice(c->device));
    build(c);
    Instance& I = c->inst[i];
    const long n = I.n, n2 = n * n, n4 = n2 * n2;
    I.mu = mu;
    I.beta = beta;
    thermal_setup(c, i);
    c->ex_main->run_setup(c->stream);
    for (int x = 0; x < c->m; ++x) {
      FTCC_HIP(hipMemcpyAsync(c->amp[i * c->m + x], t1, sizeof(double) * n2, hipMemcpyHostToDevice, c->stream));
      FTCC_HIP(
          hipMemcpyAsync(c->amp[i * c->m + x] + n2, t2, sizeof(double) * n4, hipMemcpyHostToDevice, c->stream));
    }
    if (I.d_allowed[0]) {   // the blocked path keeps every forbidden element of a state at zero
      check_momentum(c, i, c->amp[i * c->m], 2, "t1");
      check_momentum(c, i, c->amp[i * c->m] + n2, 4, "t2");
    }
    forward(c);
    const int q = i * c->m;
    if (S1) FTCC_HIP(hipMemcpyAsync(S1, c->S[q], sizeof(double) * n2, hipMemcpyDeviceToHost, c->stream));
    if (S2) FTCC_HIP(hipMemcpyAsync(S2, c->S[q] + n2, sizeof(double) * n4, hipMemcpyDeviceToHost, c->stream));
    if (E) FTCC_HIP(hipMemcpyAsync(E, c->e[q], sizeof(double), hipMemcpyDeviceToHost, c->stream));
    sync(c);
    c->solved = false;
    c->have_lambda = false;
  });
}

int ftcc_time_residual(ftcc_ctx* c, int reps, double* seconds_out, double* flops_out) {
  return run_guarded([&] {
    if (!c || reps < 1) fail(FTCC_EINVAL, "bad argument");
    if (!c->built) fail(FTCC_ESTATE, "evaluate a residual or solve first");
    FTCC_HIP(hipSetDevice(c->device));
    hipEvent_t e0, e1;
    FTCC_HIP(hipEventCreate(&e0));
    FTCC_HIP(hipEventCreate(&e1));
    FTCC_HIP(hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps; ++r) forward(c);
    FTCC_HIP(hipEventRecord(e1, c->stream));
    sync(c);
    float ms = 0.f;
    FTCC_HIP(hipEventElapsedTime(&ms, e0, e1));
    FTCC_HIP(hipEventDestroy(e0));
    FTCC_HIP(hipEventDestroy(e1));
    if (seconds_out) *seconds_out = ms * 1e-3;
    // one forward() evaluates every node: m / slots passes of the slot program
    if (flops_out) *flops_out = c->ex_main->gemm_flops_forward() * (c->m / c->slots);
  });
}

int ftcc_plan_info(ftcc_ctx* c, long* disp_fwd, long* disp_bwd, double* bytes_fwd, int* slots_out) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    if (!c->built) fail(FTCC_ESTATE, "evaluate a residual or solve first");
    if (disp_fwd) *disp_fwd = c->ex_main->dispatches_forward();
    if (disp_bwd) *disp_bwd = c->ex_main->dispatches_backward();
    if (bytes_fwd) *bytes_fwd = c->ex_main->bytes_forward();
    if (slots_out) *slots_out = c->slots;
  });
}

int ftcc_kernel_profile(ftcc_ctx* c, int enable, double* flops, double* seconds, long* launches) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    FTCC_HIP(hipSetDevice(c->device));
    sync(c);
    if (flops) *flops = c->prof.flops;
    if (seconds) *seconds = c->prof.seconds;
    if (launches) *launches = c->prof.launches;
    c->prof.reset();
    c->prof.enabled = enable != 0;
  });
}

int ftcc_find_mu(ftcc_ctx* c, const double* n_target, double* mu, const double* beta, double tol, int max_iter,
                 double* n_out, int* iters_out, int* status_out) {
  int any_fail = 0;
  int rc = run_guarded([&] {
    if (!c || !n_target || !mu || !beta) fail(FTCC_EINVAL, "null argument");
    if (!(tol > 0.0) || max_iter < 1) fail(FTCC_EINVAL, "tol must be > 0 and max_iter >= 1");
    const int B = c->B;
    for (int i = 0; i < B; ++i)
      if (!std::isfinite(n_target[i]) || !std::isfinite(mu[i])) fail(FTCC_EINVAL, "non-finite target or start");
    // per-instance root finder on f(mu) = N(mu) - n_target: bracket from the start
    // value in steps set by the mean-field compressibility, then regula falsi
    // with the Illinois modification
    enum { START, BRACKET, FALSI, DONE };
    std::vector<int> phase(B, START), side(B, 0), its(B, 0), st(B, 0);
    std::vector<double> x(mu, mu + B), a(B), fa(B), b(B), fb(B), step(B), nval(B, 0.0);
    auto mf_slope = [&](int i, double m) {
      double s = 0.0;
      for (double e : c->inst[i].eps_host) {
        const double z = beta[i] * (e - m);
        const double nocc = 1.0 / (1.0 + std::exp(z)), nvir = 1.0 / (1.0 + std::exp(-z));
        s += nocc * nvir;
      }
      return std::max(c->gdeg * beta[i] * s, 1e-12);
    };
    std::vector<int> fst(B), lst(B);
    std::vector<double> dmu(B);
    for (int it = 0; it < max_iter; ++it) {
      bool any = false;
      for (int i = 0; i < B; ++i) any = any || phase[i] != DONE;
      if (!any) break;
      int r = ftcc_solve_amplitudes(c, x.data(), beta, nullptr, fst.data());
      if (r != FTCC_OK && r != FTCC_ENOCONV && r != FTCC_ENONFINITE && r != FTCC_EDIVERGE) fail(r, g_err);
      r = ftcc_lambda(c, nullptr, lst.data());
      if (r != FTCC_OK && r != FTCC_ENOCONV && r != FTCC_ENONFINITE && r != FTCC_EDIVERGE) fail(r, g_err);
      r = ftcc_response(c, dmu.data(), nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
      if (r != FTCC_OK) fail(r, g_err);
      for (int i = 0; i < B; ++i) {
        if (phase[i] == DONE) continue;
        if (fst[i] || lst[i]) {
          st[i] = fst[i] ? fst[i] : lst[i];
          phase[i] = DONE;
          continue;
        }
        ++its[i];
        nval[i] = -dmu[i];
        const double f = nval[i] - n_target[i];
        if (std::fabs(f) <= tol * std::max(1.0, std::fabs(n_target[i]))) {
          phase[i] = DONE;
          continue;
        }
        if (phase[i] == START) {
          a[i] = x[i];
          fa[i] = f;
          step[i] = -f / mf_slope(i, x[i]);
          x[i] = a[i] + step[i];
          phase[i] = BRACKET;
        } else if (phase[i] == BRACKET) {
          b[i] = x[i];
          fb[i] = f;
          if (fa[i] * fb[i] < 0.0) {
            phase[i] = FALSI;
            side[i] = 0;
            x[i] = (a[i] * fb[i] - b[i] * fa[i]) / (fb[i] - fa[i]);
          } else {
            a[i] = b[i];
            fa[i] = fb[i];
            step[i] *= 2.0;
            x[i] = a[i] + step[i];
          }
        } else {   // FALSI: x is the new point c
          if (f * fb[i] < 0.0) {
            a[i] = b[i];
            fa[i] = fb[i];
            side[i] = 0;
          } else {
            if (side[i] == -1) fa[i] *= 0.5;
            side[i] = -1;
          }
          b[i] = x[i];
          fb[i] = f;
          x[i] = (a[i] * fb[i] - b[i] * fa[i]) / (fb[i] - fa[i]);
        }
      }
    }
    for (int i = 0; i < B; ++i) {
      if (phase[i] != DONE) st[i] = FTCC_ENOCONV;
      mu[i] = x[i];
      if (n_out) n_out[i] = nval[i];
      if (iters_out) iters_out[i] = its[i];
      if (status_out) status_out[i] = st[i];
      if (st[i]) any_fail = st[i];
    }
  });
  if (rc == FTCC_OK && any_fail) {
    g_err = "at least one instance did not reach its electron number (see status_out)";
    return any_fail;
  }
  return rc;
}

int ftcc_stats(ftcc_ctx* c, long* resid_evals, long* vjp_evals, double* solve_seconds, double* lambda_seconds) {
  return run_guarded([&] {
    if (!c) fail(FTCC_EINVAL, "null context");
    if (resid_evals) *resid_evals = c->resid_evals;
    if (vjp_evals) *vjp_evals = c->vjp_evals;
    if (solve_seconds) *solve_seconds = c->t_solve;
    if (lambda_seconds) *lambda_seconds = c->t_lambda;
  });
}

}  // extern "C"
