// Imaginary-time kernels: thermal blocks and the exponential-collocation propagator.
//
// Propagator weights for one amplitude with orbital-energy difference D and
// panel width h (composite exponential Gauss collocation of the integral
// equation eqn:smu; nodes c_x, Lagrange basis l_y(u) = sum_k lc[y][k] u^k):
//   E_x  = exp(-D h c_x)
//   W_xy = h int_0^{c_x} exp(D h (u - c_x)) l_y(u) du
//        = h sum_k lc[y][k] c_x^(k+1) k! phi_{k+1}(-D h c_x)
//   We_y = h sum_k lc[y][k] k! phi_{k+1}(-D h)
// with phi_k(z) = int_0^1 exp((1-t) z) t^(k-1) / (k-1)! dt.  phi_k is summed by
// its Taylor series for |z| <= 4 and by the recurrence
// phi_{k+1} = (phi_k - 1/k!) / z from phi_1 = expm1(z)/z otherwise (both
// directions are well conditioned there).  The h-derivative used by the beta
// response is d/dh [h phi_{k+1}(a h)] = (z - k) phi_{k+1}(z) + 1/k!; the
// D-derivative used by the orbital-energy response follows from
// phi_k'(z) = phi_k(z) - k phi_{k+1}(z):
// d/dD [h phi_{k+1}(-D h c)] = -h^2 c (phi_{k+1}(z) - (k+1) phi_{k+2}(z)).
#include <hip/hip_runtime.h>
#include <math.h>

#include "gmem.h"
#include "tau_kernels.h"

namespace ftcc {

__constant__ double c_inv_fact[48];

// 1/k! table; must be uploaded on each device before the first propagator launch
hipError_t init_tau_constants() {
  double f[48];
  f[0] = 1.0;
  for (int k = 1; k < 48; ++k) f[k] = f[k - 1] / k;
  return hipMemcpyToSymbol(HIP_SYMBOL(c_inv_fact), f, sizeof(f));
}

// phi[k] = phi_k(z) for k = 1..kmax.  Small |z|: phi_kmax by its Taylor series,
// then downward phi_k = z phi_{k+1} + 1/k! (stable there: |z| <= 4 and every term
// of the series is positive for z > 0).
template <int kmax>
__device__ __forceinline__ void phi_all(double z, double* phi) {
  if (fabs(z) <= 4.0) {
    double acc = c_inv_fact[kmax + 34];
#pragma unroll 4
    for (int j = 33; j >= 0; --j) acc = fma(acc, z, c_inv_fact[j + kmax]);
    phi[kmax] = acc;
    for (int k = kmax - 1; k >= 1; --k) phi[k] = fma(z, phi[k + 1], c_inv_fact[k]);
  } else {
    double p = expm1(z) / z;
    phi[1] = p;
    for (int k = 1; k < kmax; ++k) {
      p = (p - c_inv_fact[k]) / z;
      phi[k + 1] = p;
    }
  }
}

// Weights of one amplitude for a panel of M nodes (M is a compile-time constant,
// so the arrays live in registers).
template <int M>
struct Weights {
  double E[M], W[M][M], We[M], Ee;
};

// need_end: also the panel-end row (Ee, We).  deriv: 0 the weights, 1 their
// h-derivatives at fixed D, 2 their D-derivatives at fixed h.
template <int M>
__device__ void weights(const PanelRule& R, double D, double h, Weights<M>& w, int deriv, bool need_end) {
  // R is the rule in global memory (uniform across the grid: scalar loads)
  constexpr int m = M;
  double phi[M + 2];
  for (int x = 0; x <= m; ++x) {
    if (x == m && !need_end) break;
    const double cx = (x < m) ? R.c[x] : 1.0;
    const double z = -D * h * cx;
    double e = exp(z);
    if (deriv == 1) e = -D * cx * e;            // dE/dh
    else if (deriv == 2) e = -h * cx * e;       // dE/dD
    if (x < m) w.E[x] = e; else w.Ee = e;
    if (R.lawson) {
      for (int y = 0; y < m; ++y) {
        const double arg = D * h * (R.c[y] - cx);
        const double a = (x < m) ? R.A[x][y] : R.b[y];
        const double v = deriv == 1 ? a * exp(arg) * (1.0 + arg)
                                    : (deriv == 2 ? h * a * exp(arg) * h * (R.c[y] - cx) : h * a * exp(arg));
        if (x < m) w.W[x][y] = v; else w.We[y] = v;
      }
      continue;
    }
    if (deriv == 2) phi_all<M + 1>(z, phi);
    else phi_all<M>(z, phi);
    for (int y = 0; y < m; ++y) {
      double acc = 0.0;
      for (int k = 0; k < m; ++k) {
        const double g = R.gc[x][y][k];
        if (deriv == 1) acc += g * ((z - k) * phi[k + 1] + c_inv_fact[k]);
        else if (deriv == 2) acc += g * (phi[k + 1] - (k + 1) * phi[k + 2]);
        else acc += g * phi[k + 1];
      }
      if (deriv == 0) acc *= h;
      else if (deriv == 2) acc *= -h * h * cx;
      if (x < m) w.W[x][y] = acc; else w.We[y] = acc;
    }
  }
}

// orbital-energy difference of element e of a t1 (rank 2, [i][a]) or t2
// (rank 4, [i][j][a][b]) segment
__device__ __forceinline__ double seg_delta(const double* eps_ptr, int n, int rank, long e) {
  const gptr<const double> eps = gview(eps_ptr);
  if (rank == 2) {
    const int a = (int)(e % n), i = (int)(e / n);
    return eps[a] - eps[i];
  }
  const int b = (int)(e % n);
  long r = e / n;
  const int a = (int)(r % n);
  r /= n;
  const int j = (int)(r % n);
  const int i = (int)(r / n);
  return eps[a] + eps[b] - eps[i] - eps[j];
}

__device__ __forceinline__ double delta_of(const TauProblem& P, long e) { return seg_delta(P.eps, P.n, P.rank, e); }

// max that propagates NaN as +infinity (fmax would drop it)
__device__ __forceinline__ double nan_max(double a, double b) {
  if (b != b) return INFINITY;
  return fmax(a, b);
}

__device__ __forceinline__ void atomic_max_pos(unsigned long long* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

template <int M>
__global__ void __launch_bounds__(256) tau_kernel(const PanelRule* __restrict__ rule, int mode,
                                                  const TauProblem* __restrict__ probs,
                                                  const int* __restrict__ prefix, int n_prob) {
  int lo = 0, hi = n_prob - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const TauProblem& P = probs[lo];
  if (P.active && *gview(P.active) == 0) return;   // converged instance of a batch: left unchanged
  const PanelRule& R = *rule;
  constexpr int m = M;
  const long base = (long)(b - prefix[lo]) * 1024;
  double mchg = 0.0, mval = 0.0, acc = 0.0;
  for (int u = 0; u < 4; ++u) {
    const long ei = base + u * 256 + threadIdx.x;
    if (ei >= P.len) break;
    const long e = P.idx ? (long)gview(P.idx)[ei] : ei;   // element offset in the segment
    const double sb = P.sb ? gview(P.sb)[e] : 0.0;
    double Sv[M];
    bool any = (sb != 0.0);
    for (int y = 0; y < m; ++y) {
      Sv[y] = P.S[y] ? gview(P.S[y])[e] : 0.0;
      any = any || (Sv[y] != 0.0);
    }
    if (mode == TAU_LSTEP) {
      for (int x = 0; x < m; ++x) {
        const double nv = -gview(P.R[x])[e];
        mchg = nan_max(mchg, fabs(nv - gview(P.s[x])[e]));
        mval = nan_max(mval, fabs(nv));
        gview(P.s[x])[e] = nv;
      }
      continue;
    }
    if (mode == TAU_BETA || mode == TAU_DEPS) {
      double Rv[M];
      bool anyb = any || (P.lam_a && gview(P.lam_a)[e] != 0.0);
      for (int y = 0; y < m; ++y) {
        Rv[y] = gview(P.R[y])[e];
        anyb = anyb || (Rv[y] != 0.0);
      }
      if (!anyb) continue;
      Weights<M> w;
      weights<M>(R, delta_of(P, e), P.h, w, mode == TAU_BETA ? 1 : 2, P.lam_a != nullptr);
      double val = 0.0;
      for (int x = 0; x < m; ++x) {
        double f = (sb != 0.0) ? -w.E[x] * sb : 0.0;
        for (int y = 0; y < m; ++y)
          if (Rv[y] != 0.0) f += w.W[x][y] * Rv[y];
        val += Sv[x] * f;
      }
      if (P.lam_a) {
        double f = (sb != 0.0) ? -w.Ee * sb : 0.0;
        for (int y = 0; y < m; ++y)
          if (Rv[y] != 0.0) f += w.We[y] * Rv[y];
        val += gview(P.lam_a)[e] * f;
      }
      if (mode == TAU_BETA) acc += val;
      else gview(P.out)[e] += val;
      continue;
    }
    if (!any) {
      // structurally zero (dropped slots, or zero start): outputs stay zero
      if (mode == TAU_INIT || mode == TAU_LAMT) {
        for (int x = 0; x < m; ++x) gview(P.s[x])[e] = 0.0;
      } else if (mode == TAU_STEP) {
        for (int x = 0; x < m; ++x) {
          mchg = nan_max(mchg, fabs(gview(P.s[x])[e]));
          gview(P.s[x])[e] = 0.0;
        }
      } else {
        gview(P.out)[e] = 0.0;
      }
      continue;
    }
    Weights<M> w;
    weights<M>(R, delta_of(P, e), P.h, w, 0, mode != TAU_INIT && mode != TAU_STEP);
    if (mode == TAU_INIT) {
      for (int x = 0; x < m; ++x) gview(P.s[x])[e] = (sb != 0.0) ? w.E[x] * sb : 0.0;
    } else if (mode == TAU_STEP) {
      for (int x = 0; x < m; ++x) {
        double v = (sb != 0.0) ? w.E[x] * sb : 0.0;
        for (int y = 0; y < m; ++y)
          if (Sv[y] != 0.0) v -= w.W[x][y] * Sv[y];
        mchg = nan_max(mchg, fabs(v - gview(P.s[x])[e]));
        mval = nan_max(mval, fabs(v));
        gview(P.s[x])[e] = v;
      }
    } else if (mode == TAU_END) {
      double v = (sb != 0.0) ? w.Ee * sb : 0.0;
      for (int y = 0; y < m; ++y)
        if (Sv[y] != 0.0) v -= w.We[y] * Sv[y];
      gview(P.out)[e] = v;
    } else if (mode == TAU_LAMT) {
      for (int x = 0; x < m; ++x) {
        double v = (sb != 0.0) ? w.We[x] * sb : 0.0;
        for (int y = 0; y < m; ++y)
          if (Sv[y] != 0.0) v += w.W[y][x] * Sv[y];
        gview(P.s[x])[e] = v;
      }
    } else if (mode == TAU_APREV) {
      double v = (sb != 0.0) ? w.Ee * sb : 0.0;
      for (int x = 0; x < m; ++x)
        if (Sv[x] != 0.0) v += w.E[x] * Sv[x];
      gview(P.out)[e] = v;
    }
  }
  // block reductions
  __shared__ double r0[256], r1[256];
  if (mode == TAU_STEP || mode == TAU_LSTEP) {
    r0[threadIdx.x] = mchg;
    r1[threadIdx.x] = mval;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        r0[threadIdx.x] = nan_max(r0[threadIdx.x], r0[threadIdx.x + s]);
        r1[threadIdx.x] = nan_max(r1[threadIdx.x], r1[threadIdx.x + s]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      atomic_max_pos(P.maxbits, r0[0]);
      atomic_max_pos(P.maxbits + 1, r1[0]);
    }
  } else if (mode == TAU_BETA) {
    r0[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) r0[threadIdx.x] += r0[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) gview(P.partial)[b - prefix[lo]] = r0[0];
  }
}

void launch_tau(const PanelRule* d_rule, int m, int mode, const TauProblem* d_probs, const int* d_prefix, int n_prob,
                int total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
#define FTCC_TAU(MM)                                                                                              \
  case MM:                                                                                                        \
    hipLaunchKernelGGL(tau_kernel<MM>, dim3(total_blocks), dim3(256), 0, s, d_rule, mode, d_probs, d_prefix, n_prob); \
    break;
  switch (m) {
    FTCC_TAU(1)
    FTCC_TAU(2)
    FTCC_TAU(3)
    FTCC_TAU(4)
    FTCC_TAU(5)
    FTCC_TAU(6)
  }
#undef FTCC_TAU
}

// Runge-Kutta combinations (differential form, Algorithm alg:diff):
//   out = x0 * base + sum_l coef[l] * (-Delta Y_l + sigma S_l)
// over the (allowed) elements of one segment.  One block covers 1024 elements.
__global__ void __launch_bounds__(256) rk_combine_kernel(const RKProblem* __restrict__ probs,
                                                         const int* __restrict__ prefix, int n_prob) {
  int lo = 0, hi = n_prob - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const RKProblem& P = probs[lo];
  if (P.active && *gview(P.active) == 0) return;   // uniform per block, before the barrier
  const long first = (long)(b - prefix[lo]) * 1024;
  double vmax = 0.0;
  for (int u = 0; u < 4; ++u) {
    const long ei = first + u * 256 + threadIdx.x;
    if (ei >= P.len) break;
    const long e = P.idx ? (long)gview(P.idx)[ei] : ei;
    const double d = seg_delta(P.eps, P.n, P.rank, e);
    double v = P.base ? P.x0 * gview(P.base)[e] : 0.0;
    for (int l = 0; l < P.nst; ++l) {
      const double y = P.Y[l] ? gview(P.Y[l])[e] : 0.0;
      const double sv = P.S[l] ? gview(P.S[l])[e] : 0.0;
      v += P.coef[l] * (-d * y + P.sigma * sv);
    }
    gview(P.out)[e] = v;
    vmax = nan_max(vmax, fabs(v));
  }
  if (!P.maxbits) return;   // uniform per launch problem
  __shared__ double red[256];
  red[threadIdx.x] = vmax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = nan_max(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomic_max_pos(P.maxbits, red[0]);
}

void launch_rk_combine(const RKProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(rk_combine_kernel, dim3(total_blocks), dim3(256), 0, s, d_probs, d_prefix, n_prob);
}

__global__ void __launch_bounds__(256) expsum_kernel(const ExpSumProblem* __restrict__ probs,
                                                     const int* __restrict__ prefix, int n_prob) {
  int lo = 0, hi = n_prob - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const ExpSumProblem& P = probs[lo];
  if (P.active && *gview(P.active) == 0) return;   // uniform per block, before the barrier
  const long first = (long)(b - prefix[lo]) * 1024;
  double vmax = 0.0, cmax = 0.0;
  for (int u = 0; u < 4; ++u) {
    const long ei = first + u * 256 + threadIdx.x;
    if (ei >= P.len) break;
    const long e = P.idx ? (long)gview(P.idx)[ei] : ei;
    const double d = seg_delta(P.eps, P.n, P.rank, e);
    double acc = 0.0;
    for (int l = 0; l < P.nterms; ++l) {
      const ExpTerm t = P.terms[l];
      const double x = gview(t.X)[e];
      if (x == 0.0) continue;
      const double z = d * P.h * t.k;
      const double ex = exp(-z);
      const double f = P.mode == 0 ? P.h * t.C * ex
                                   : (P.mode == 1 ? t.C * ex * (1.0 - z) : -P.h * P.h * t.C * t.k * ex);
      acc += f * x;
    }
    if (P.prod) acc *= gview(P.prod)[e];
    const double v = (P.base ? P.x0 * gview(P.base)[e] : 0.0) + acc;
    if (P.maxbits) cmax = nan_max(cmax, fabs(v - gview(P.out)[e]));
    gview(P.out)[e] = v;
    vmax = nan_max(vmax, fabs(v));
  }
  if (!P.maxbits) return;   // uniform per launch problem
  __shared__ double r0[256], r1[256];
  r0[threadIdx.x] = cmax;
  r1[threadIdx.x] = vmax;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      r0[threadIdx.x] = nan_max(r0[threadIdx.x], r0[threadIdx.x + st]);
      r1[threadIdx.x] = nan_max(r1[threadIdx.x], r1[threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomic_max_pos(P.maxbits, r0[0]);
    atomic_max_pos(P.maxbits + 1, r1[0]);
  }
}

void launch_expsum(const ExpSumProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(expsum_kernel, dim3(total_blocks), dim3(256), 0, s, d_probs, d_prefix, n_prob);
}

__global__ void __launch_bounds__(256) copy_listed_kernel(const unsigned* __restrict__ a, long na,
                                                          const unsigned* __restrict__ b, long nb, long second,
                                                          const double* __restrict__ src, double* __restrict__ dst) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= na + nb) return;
  const long off = e < na ? (long)gview(a)[e] : second + (long)gview(b)[e - na];
  gview(dst)[off] = gview(src)[off];
}

void launch_copy_listed(const unsigned* a, long na, const unsigned* b, long nb, long second, const double* src,
                        double* dst, hipStream_t s) {
  const long total = na + nb;
  if (total <= 0) return;
  hipLaunchKernelGGL(copy_listed_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a, na, b, nb,
                     second, src, dst);
}

// ------------------------------------------------------------------ thermal quantities
__global__ void occ_kernel(ThermalProblem P) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P.n) return;
  const double x = P.beta * (P.eps[p] - P.mu);
  // n = 1 / (1 + e^x), 1 - n = 1 / (1 + e^-x), each without cancellation
  double nocc, nvir;
  if (x > 0.0) {
    const double t = exp(-x);
    nocc = t / (1.0 + t);
    nvir = 1.0 / (1.0 + t);
  } else {
    const double t = exp(x);
    nocc = 1.0 / (1.0 + t);
    nvir = t / (1.0 + t);
  }
  P.occ[p] = nocc;
  P.wo[p] = (nocc > P.thr) ? sqrt(nocc) : 0.0;
  P.wv[p] = (nvir > P.thr) ? sqrt(nvir) : 0.0;
}

// f_pq = h_pq + sum_r (2 <pr|qr> - <pr|rq>) n_r
__global__ void fock_kernel(ThermalProblem P) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  const int n = P.n;
  if (q >= n) return;
  double acc = P.h[(long)p * n + q];
  for (int r = 0; r < n; ++r) {
    const double d = P.eri[(((long)p * n + r) * n + q) * n + r];
    const double x = P.eri[(((long)p * n + r) * n + r) * n + q];
    acc += (P.g * d - x) * P.occ[r];
  }
  P.fock[(long)p * n + q] = acc;
}

void launch_thermal(const ThermalProblem& p, hipStream_t s) {
  hipLaunchKernelGGL(occ_kernel, dim3((p.n + 63) / 64), dim3(64), 0, s, p);
  hipLaunchKernelGGL(fock_kernel, dim3((p.n + 63) / 64, p.n), dim3(64), 0, s, p);
}

// du_pq = dh_pq + sum_r (2 <pr|qr> - <pr|rq>) dn_r + sum_r (2 d<pr|qr> - d<pr|rq>) n_r
__global__ void fock_deriv_kernel(int n, const double* eri, const double* deri, const double* dh,
                                  const double* occ, const double* docc, double g, double* du) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  if (q >= n) return;
  double acc = dh ? dh[(long)p * n + q] : 0.0;
  for (int r = 0; r < n; ++r) {
    const long id = (((long)p * n + r) * n + q) * n + r;
    const long ix = (((long)p * n + r) * n + r) * n + q;
    if (docc) acc += (g * eri[id] - eri[ix]) * docc[r];
    if (deri) acc += (g * deri[id] - deri[ix]) * occ[r];
  }
  du[(long)p * n + q] = acc;
}

void launch_fock_deriv(int n, const double* eri, const double* deri, const double* dh, const double* occ,
                       const double* docc, double g, double* du, hipStream_t s) {
  hipLaunchKernelGGL(fock_deriv_kernel, dim3((n + 63) / 64, n), dim3(64), 0, s, n, eri, deri, dh, occ, docc, g, du);
}

__global__ void u_from_fock_kernel(int n, const double* fock, const double* eps, double* u) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * n) return;
  const int p = (int)(e / n), q = (int)(e % n);
  u[e] = fock[e] - (p == q ? eps[p] : 0.0);
}

void launch_u_from_fock(int n, const double* fock, const double* eps, double* u, hipStream_t s) {
  const long len = (long)n * n;
  hipLaunchKernelGGL(u_from_fock_kernel, dim3((len + 255) / 256), dim3(256), 0, s, n, fock, eps, u);
}

// ------------------------------------------------------------------ weighted blocks
__global__ void block_kernel(BlockSpec B) {
  const long len = (B.rank == 4) ? (long)B.n * B.n * B.n * B.n : (long)B.n * B.n;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (B.idx ? B.count : len)) return;
  const long e = B.idx ? (long)gview(B.idx)[t] : t;
  int idx[4];
  long r = e;
  for (int k = B.rank - 1; k >= 0; --k) {
    idx[k] = (int)(r % B.n);
    r /= B.n;
  }
  double w[4], dw[4];
  for (int k = 0; k < B.rank; ++k) {
    const bool o = (B.pat[k] == 'o');
    w[k] = o ? B.wo[idx[k]] : B.wv[idx[k]];
    const double* dv = o ? B.dwo : B.dwv;
    dw[k] = dv ? dv[idx[k]] : 0.0;
  }
  double prod = 1.0;
  for (int k = 0; k < B.rank; ++k) prod *= w[k];
  double v = B.dbase ? prod * B.dbase[e] : 0.0;
  if (B.dwo || B.dwv) {
    for (int k = 0; k < B.rank; ++k) {
      if (dw[k] == 0.0) continue;
      double pk = dw[k];
      for (int j = 0; j < B.rank; ++j)
        if (j != k) pk *= w[j];
      v += pk * B.base[e];
    }
  }
  B.out[e] = v;
}

void launch_block(const BlockSpec& b, hipStream_t s) {
  const long len = b.idx ? b.count : (b.rank == 4) ? (long)b.n * b.n * b.n * b.n : (long)b.n * b.n;
  if (len <= 0) return;
  hipLaunchKernelGGL(block_kernel, dim3((len + 255) / 256), dim3(256), 0, s, b);
}

// ------------------------------------------------------------------ DIIS (Anderson) extrapolation
// One thread per instance: minimise |sum_j c_j r_j|^2 subject to sum_j c_j = 1 over
// the `count` stored residuals (Gram matrix G, row-major with leading dimension
// ld), by Gaussian elimination with partial pivoting on the bordered system.
// A singular or non-finite system falls back to the newest iterate (plain Picard).
__global__ void diis_solve_kernel(int n_inst, const int* counts, const int* newest, const double* G, int ld,
                                  double* coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  const int k = counts[i];
  const double* g = G + (long)i * ld * ld;
  double* c = coef + (long)i * ld;
  double A[9][10];
  double scale = 0.0;
  for (int a = 0; a < k; ++a) scale = fmax(scale, fabs(g[a * ld + a]));
  bool ok = (k > 1) && scale > 0.0 && isfinite(scale);
  if (ok) {
    for (int a = 0; a < k; ++a) {
      for (int b = 0; b < k; ++b) A[a][b] = g[a * ld + b] / scale;
      A[a][k] = -1.0;
      A[a][k + 1] = 0.0;
    }
    for (int b = 0; b < k; ++b) A[k][b] = -1.0;
    A[k][k] = 0.0;
    A[k][k + 1] = -1.0;
    const int nn = k + 1;
    for (int col = 0; col < nn && ok; ++col) {
      int piv = col;
      for (int r = col + 1; r < nn; ++r)
        if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
      if (!(fabs(A[piv][col]) > 1e-14)) {
        ok = false;
        break;
      }
      if (piv != col)
        for (int q = 0; q <= nn; ++q) {
          const double t = A[col][q];
          A[col][q] = A[piv][q];
          A[piv][q] = t;
        }
      for (int r = 0; r < nn; ++r) {
        if (r == col) continue;
        const double f = A[r][col] / A[col][col];
        for (int q = col; q <= nn; ++q) A[r][q] -= f * A[col][q];
      }
    }
    if (ok)
      for (int a = 0; a < k; ++a) {
        c[a] = A[a][nn] / A[a][a];
        if (!isfinite(c[a])) ok = false;
      }
  }
  if (!ok)
    for (int a = 0; a < ld; ++a) c[a] = (a == newest[i]) ? 1.0 : 0.0;
}

void launch_diis_solve(int n_inst, const int* counts, const int* newest, const double* G, int ld, double* coef,
                       hipStream_t s) {
  hipLaunchKernelGGL(diis_solve_kernel, dim3((n_inst + 63) / 64), dim3(64), 0, s, n_inst, counts, newest, G, ld,
                     coef);
}

// out[e] = sum_j coef[j] * (X_j[e] + R_j[e])
__global__ void diis_combine_kernel(long len, DiisTerms t, double* out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double v = 0.0;
  for (int j = 0; j < t.k; ++j) {
    const double cj = t.coef[j];
    if (cj != 0.0) v += cj * (t.X[j][e] + t.R[j][e]);
  }
  out[e] = v;
}

void launch_diis_combine(long len, const DiisTerms& t, double* out, hipStream_t s) {
  if (len <= 0) return;
  hipLaunchKernelGGL(diis_combine_kernel, dim3((len + 255) / 256), dim3(256), 0, s, len, t, out);
}

// ------------------------------------------------------------------ small utilities
__global__ void sum_kernel(const double* x, int count, double* out) {
  __shared__ double r[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) a += x[i];
  r[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) r[threadIdx.x] += r[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = r[0];
}

void launch_sum(const double* x, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, x, count, out);
}

__global__ void axpby_kernel(long len, double a, const double* x, double b, double* y) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const double xv = (a != 0.0) ? a * x[e] : 0.0;
  y[e] = (b != 0.0) ? xv + b * y[e] : xv;
}

void launch_axpby(long len, double a, const double* x, double b, double* y, hipStream_t s) {
  if (len <= 0) return;
  hipLaunchKernelGGL(axpby_kernel, dim3((len + 255) / 256), dim3(256), 0, s, len, a, x, b, y);
}

}  // namespace ftcc
