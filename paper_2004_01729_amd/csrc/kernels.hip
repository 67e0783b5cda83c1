// Device kernels of the FT-CCSD hot path (gfx950, FP64 throughout).
//
//   gemm_mfma      grouped C = alpha * op(A) op(B) + beta * C on v_mfma_f64_16x16x4f64,
//                  LDS double-buffered 128x128 (or 64x64) tiles, XCD-aware tile order,
//                  optional split-K with a deterministic second-pass reduction
//   permute4       grouped 4-index transpose-accumulate Y[perm] = alpha X + beta Y,
//                  LDS-tiled when the fastest index moves
//   dot            grouped full contractions (two-pass, deterministic)
//
// The imaginary-time kernels (thermal blocks, propagator, adjoint) are in
// tau_kernels.hip.
//
// Every grouped kernel takes a device array of problem descriptors; the block
// index is mapped to (problem, tile) through the exclusive prefix of tile counts.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace ftcc {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int find_problem(const int* prefix, int n_prob, int b) {
  int lo = 0, hi = n_prob - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Bijective remap of the linear block id so that the blocks scheduled on one XCD
// (the hardware assigns block b to XCD b % 8) cover a contiguous range of tiles.
__device__ __forceinline__ int xcd_remap(int b, int total) {
  const int nx = 8;
  int q = total / nx, r = total % nx;
  int x = b % nx, i = b / nx;
  return x * q + (x < r ? x : r) + i;
}

// ------------------------------------------------------------------ GEMM
// Fragment layouts of v_mfma_f64_16x16x4f64 (wave64):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l holds D[4 * r + l / 16][l % 16], r = 0..3
typedef double double4_t __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, bool TA, bool TB>
__global__ void __launch_bounds__(256)
gemm_mfma_kernel(const GemmProblem* __restrict__ probs, const int* __restrict__ prefix,
                 int n_prob, int total_tiles) {
  constexpr int WM = BM / 2, WN = BN / 2;        // 2 x 2 waves
  constexpr int FM = WM / 16, FN = WN / 16;      // MFMA tiles per wave
  constexpr int PA = BM + 1, PB = BN + 1;        // LDS row pitch (doubles)
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  __shared__ double As[2][BK * PA];
  __shared__ double Bs[2][BK * PB];

  const int tile = xcd_remap(blockIdx.x, total_tiles);
  const int pi = find_problem(prefix, n_prob, tile);
  const GemmProblem P = probs[pi];
  int local = tile - prefix[pi];
  const int tiles_mn = P.tiles_m * P.tiles_n;
  const int ks = local / tiles_mn;
  local -= ks * tiles_mn;
  // grouped ordering inside the problem: bands of 8 tile-rows
  const int GM = 8;
  const int band = local / (GM * P.tiles_n);
  const int first_m = band * GM;
  const int band_rows = min(GM, P.tiles_m - first_m);
  const int tm = first_m + (local % (GM * P.tiles_n)) % band_rows;
  const int tn = (local % (GM * P.tiles_n)) / band_rows;

  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = ks * P.kchunk;
  const int kend = min(P.K, kbeg + P.kchunk);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const double* __restrict__ A = P.A;
  const double* __restrict__ B = P.B;
  const long lda = P.lda, ldb = P.ldb;

  double ra[LA], rb[LB];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int j = 0; j < LA; ++j) {
      int e = tid + 256 * j;
      int m, k;
      if (TA) { k = e / BM; m = e % BM; } else { m = e / BK; k = e % BK; }
      int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < P.M && gk < kend) v = TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk];
      ra[j] = v;
    }
#pragma unroll
    for (int j = 0; j < LB; ++j) {
      int e = tid + 256 * j;
      int n, k;
      if (TB) { n = e / BK; k = e % BK; } else { k = e / BN; n = e % BN; }
      int gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < P.N && gk < kend) v = TB ? B[(long)gn * ldb + gk] : B[(long)gk * ldb + gn];
      rb[j] = v;
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int j = 0; j < LA; ++j) {
      int e = tid + 256 * j;
      int m, k;
      if (TA) { k = e / BM; m = e % BM; } else { m = e / BK; k = e % BK; }
      As[buf][k * PA + m] = ra[j];
    }
#pragma unroll
    for (int j = 0; j < LB; ++j) {
      int e = tid + 256 * j;
      int n, k;
      if (TB) { n = e / BK; k = e % BK; } else { k = e / BN; n = e % BN; }
      Bs[buf][k * PB + n] = rb[j];
    }
  };

  double4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  const int nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    load_tiles(kbeg);
    store_tiles(0);
    __syncthreads();
  }
  for (int it = 0; it < nk; ++it) {
    const int cur = it & 1;
    const bool more = (it + 1) < nk;
    if (more) load_tiles(kbeg + (it + 1) * BK);
    const double* as = As[cur];
    const double* bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = as[kr * PA + wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = bs[kr * PB + wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (more) store_tiles(cur ^ 1);
    __syncthreads();
  }

  // epilogue
  double* C;
  long ldc;
  double alpha, beta;
  if (P.ksplit > 1) {
    C = P.partial + (long)ks * P.M * P.N;
    ldc = P.N;
    alpha = 1.0;
    beta = 0.0;
  } else {
    C = P.C;
    ldc = P.ldc;
    alpha = P.alpha;
    beta = P.beta;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int gn = n0 + wn * WN + j * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm * WM + i * 16 + 4 * r + (lane >> 4);
        if (gm < P.M && gn < P.N) {
          double* c = C + (long)gm * ldc + gn;
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v += beta * (*c);
          *c = v;
        }
      }
    }
}

// C = alpha * sum_s partial[s] + beta * C for split-K problems
__global__ void splitk_reduce_kernel(const GemmProblem* __restrict__ probs, const int* __restrict__ prefix,
                                     int n_prob, int total) {
  const int pi = find_problem(prefix, n_prob, blockIdx.x);
  const GemmProblem P = probs[pi];
  if (P.ksplit <= 1) return;
  const long mn = (long)P.M * P.N;
  const long chunk = (long)(blockIdx.x - prefix[pi]) * 256 * 4;
  for (int u = 0; u < 4; ++u) {
    long e = chunk + u * 256 + threadIdx.x;
    if (e >= mn) return;
    double s = 0.0;
    for (int k = 0; k < P.ksplit; ++k) s += P.partial[k * mn + e];
    long gm = e / P.N, gn = e % P.N;
    double* c = P.C + gm * P.ldc + gn;
    double v = P.alpha * s;
    if (P.beta != 0.0) v += P.beta * (*c);
    *c = v;
  }
}

// ------------------------------------------------------------------ permute
// Y[o0,o1,o2,o3] = alpha * X[sum_k o_k * xs[k]] + beta * Y   (Y contiguous, dims d)
// Tiled path: axis `ta` of Y (its fastest, 3) against the Y axis `tb` that is
// X's fastest; a 32x32 LDS tile keeps both the read and the write coalesced.
__global__ void permute4_kernel(const PermProblem* __restrict__ probs, const int* __restrict__ prefix,
                                int n_prob) {
  const int pi = find_problem(prefix, n_prob, blockIdx.x);
  const PermProblem P = probs[pi];
  const long local = blockIdx.x - prefix[pi];
  const double alpha = P.scale ? P.alpha * (*P.scale) : P.alpha;
  __shared__ double tileb[32][33];
  if (P.tb < 0) {
    // contiguous-run path: Y's fastest axis is also X's fastest axis
    const long total = (long)P.d[0] * P.d[1] * P.d[2] * P.d[3];
    for (int u = 0; u < 4; ++u) {
      long e = local * 1024 + u * 256 + threadIdx.x;
      if (e >= total) return;
      long r = e;
      int o3 = r % P.d[3]; r /= P.d[3];
      int o2 = r % P.d[2]; r /= P.d[2];
      int o1 = r % P.d[1]; r /= P.d[1];
      int o0 = (int)r;
      long xo = o0 * P.xs[0] + o1 * P.xs[1] + o2 * P.xs[2] + o3 * P.xs[3];
      double v = (alpha != 0.0) ? alpha * P.X[xo] : 0.0;
      if (P.beta != 0.0) v += P.beta * P.Y[e];
      P.Y[e] = v;
    }
    return;
  }
  // tiled path over Y axes (tb, 3); the other two Y axes (p, q) enumerate tiles
  const int tb = P.tb;
  int oth[2], c = 0;
  for (int k = 0; k < 3; ++k) if (k != tb) oth[c++] = k;
  const int nt3 = (P.d[3] + 31) / 32, ntb = (P.d[tb] + 31) / 32;
  long r = local;
  const int t3 = r % nt3; r /= nt3;
  const int tbb = r % ntb; r /= ntb;
  const int iq = r % P.d[oth[1]]; r /= P.d[oth[1]];
  const int ip = (int)r;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  int o[4];
  o[oth[0]] = ip;
  o[oth[1]] = iq;
  // read: X fastest is Y axis tb -> consecutive tx along tb
  for (int y = ty; y < 32; y += 8) {
    o[tb] = tbb * 32 + tx;
    o[3] = t3 * 32 + y;
    double v = 0.0;
    if (o[tb] < P.d[tb] && o[3] < P.d[3])
      v = P.X[o[0] * P.xs[0] + o[1] * P.xs[1] + o[2] * P.xs[2] + o[3] * P.xs[3]];
    tileb[y][tx] = v;
  }
  __syncthreads();
  for (int y = ty; y < 32; y += 8) {
    o[tb] = tbb * 32 + y;
    o[3] = t3 * 32 + tx;
    if (o[tb] < P.d[tb] && o[3] < P.d[3]) {
      long yo = (((long)o[0] * P.d[1] + o[1]) * P.d[2] + o[2]) * P.d[3] + o[3];
      double v = alpha * tileb[tx][y];
      if (P.beta != 0.0) v += P.beta * P.Y[yo];
      P.Y[yo] = v;
    }
  }
}

// ------------------------------------------------------------------ dot
__global__ void dot_partial_kernel(const DotProblem* __restrict__ probs, int blocks_per, double* partial) {
  const int pi = blockIdx.x / blocks_per;
  const int bi = blockIdx.x % blocks_per;
  const DotProblem P = probs[pi];
  double s = 0.0;
  for (long e = (long)bi * 256 + threadIdx.x; e < P.len; e += (long)blocks_per * 256) s += P.X[e] * P.Y[e];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void dot_final_kernel(const DotProblem* __restrict__ probs, int n_prob, int blocks_per,
                                 const double* partial) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= n_prob) return;
  const DotProblem P = probs[pi];
  double s = 0.0;
  for (int b = 0; b < blocks_per; ++b) s += partial[pi * blocks_per + b];
  double v = P.alpha * s;
  if (P.beta != 0.0) v += P.beta * (*P.out);
  *P.out = v;
}

// ------------------------------------------------------------------ launchers
template <int BM, int BN, bool TA, bool TB>
static void launch_gemm_t(const GemmProblem* d_probs, const int* d_prefix, int n_prob, int total_tiles,
                          hipStream_t s) {
  hipLaunchKernelGGL((gemm_mfma_kernel<BM, BN, 16, TA, TB>), dim3(total_tiles), dim3(256), 0, s,
                     d_probs, d_prefix, n_prob, total_tiles);
}

void launch_gemm(int cfg, bool ta, bool tb, const GemmProblem* d_probs, const int* d_prefix, int n_prob,
                 int total_tiles, hipStream_t s) {
  if (total_tiles <= 0) return;
#define FTCC_G(BM, BN)                                                                        \
  do {                                                                                        \
    if (ta && tb) launch_gemm_t<BM, BN, true, true>(d_probs, d_prefix, n_prob, total_tiles, s);    \
    else if (ta) launch_gemm_t<BM, BN, true, false>(d_probs, d_prefix, n_prob, total_tiles, s);    \
    else if (tb) launch_gemm_t<BM, BN, false, true>(d_probs, d_prefix, n_prob, total_tiles, s);    \
    else launch_gemm_t<BM, BN, false, false>(d_probs, d_prefix, n_prob, total_tiles, s);           \
  } while (0)
  if (cfg == 0) FTCC_G(128, 128);
  else FTCC_G(64, 64);
#undef FTCC_G
}

void launch_splitk_reduce(const GemmProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks,
                          hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(total_blocks), dim3(256), 0, s, d_probs, d_prefix, n_prob,
                     total_blocks);
}

void launch_permute(const PermProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks,
                    hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(permute4_kernel, dim3(total_blocks), dim3(256), 0, s, d_probs, d_prefix, n_prob);
}

void launch_dot(const DotProblem* d_probs, int n_prob, int blocks_per, double* d_partial, hipStream_t s) {
  if (n_prob <= 0) return;
  hipLaunchKernelGGL(dot_partial_kernel, dim3(n_prob * blocks_per), dim3(256), 0, s, d_probs, blocks_per,
                     d_partial);
  hipLaunchKernelGGL(dot_final_kernel, dim3((n_prob + 63) / 64), dim3(64), 0, s, d_probs, n_prob, blocks_per,
                     d_partial);
}

}  // namespace ftcc
