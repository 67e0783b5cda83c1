// Internal kernel interfaces (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

namespace ftcc {

// One GEMM problem of a grouped launch.
//   TA = false: A[m * lda + k]   TA = true: A[k * lda + m]
//   TB = false: B[k * ldb + n]   TB = true: B[n * ldb + k]
//   C[m * ldc + n] = alpha * sum_k A B + beta * C
// With ksplit > 1 the K range is cut into chunks of kchunk; each chunk writes
// its partial product to partial + s * M * N and a second kernel reduces.
struct GemmProblem {
  const double* A;
  const double* B;
  double* C;
  double* partial;
  long lda, ldb, ldc;
  int M, N, K;
  int tiles_m, tiles_n, ksplit, kchunk;
  double alpha, beta;
};

// Y (contiguous, dims d) = alpha * (*scale) * X[o . xs] + beta * Y ; tb = Y axis that is X's
// fastest axis when it differs from Y's fastest axis, else -1.
struct PermProblem {
  const double* X;
  double* Y;
  const double* scale;   // optional device scalar multiplying alpha (nullptr: 1)
  long xs[4];
  int d[4];
  int tb;
  double alpha, beta;
};

// *out = alpha * sum_e X[e] Y[e] + beta * *out
struct DotProblem {
  const double* X;
  const double* Y;
  double* out;
  long len;
  double alpha, beta;
};

void launch_gemm(int cfg, bool ta, bool tb, const GemmProblem* d_probs, const int* d_prefix, int n_prob,
                 int total_tiles, hipStream_t s);
void launch_splitk_reduce(const GemmProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks,
                          hipStream_t s);
void launch_permute(const PermProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks,
                    hipStream_t s);
void launch_dot(const DotProblem* d_probs, int n_prob, int blocks_per, double* d_partial, hipStream_t s);

// tile sizes of the GEMM configurations
inline int gemm_bm(int cfg) { return cfg == 0 ? 128 : 64; }
inline int gemm_bn(int cfg) { return cfg == 0 ? 128 : 64; }

}  // namespace ftcc
