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
  const int* active;     // optional run flag of the problem's instance (0: skip the problem)
  // optional output offset tables: element (m, n) of C goes to C[offM[m] + offN[n]]
  // instead of C[m * ldc + n] (a contraction whose output layout is neither
  // [M][N] nor [N][M]: written in place of a separate permute pass)
  const unsigned* offM;
  const unsigned* offN;
};

// Unsigned 32-bit division by a runtime constant: q = umulhi(x, mul) >> shr
// (Granlund-Montgomery; exact for x < 2^31).
struct FastDiv {
  unsigned int d, mul, shr;
};
FastDiv make_fastdiv(unsigned int d);

// Y (contiguous, dims d) = alpha * (*scale) * X[o . xs] + beta * Y ; tb = Y axis that is X's
// fastest axis when it differs from Y's fastest axis, else -1.  div[k] divide by d[k];
// for the tiled path tdiv[0..1] divide by the tile counts of axes 3 and tb.
struct PermProblem {
  const double* X;
  double* Y;
  const double* scale;   // optional device scalar multiplying alpha (nullptr: 1)
  long xs[4];
  int d[4];
  int tb;
  int oth[2];            // the two Y axes other than 3 and tb (tiled path)
  FastDiv div[4];
  FastDiv tdiv[2];
  double alpha, beta;
  const int* active;     // optional run flag (0: skip)
};

// *out = alpha * sum_e X[e] Y[e] + beta * *out
struct DotProblem {
  const double* X;
  const double* Y;
  double* out;
  long len;
  double alpha, beta;
  const int* active;     // optional run flag (0: skip, *out keeps its value)
  // optional element lists: with ia set the sum runs over the offsets ia[0..na)
  // and second + ib[0..nb) (the other elements are zero in X or Y) instead of [0, len)
  const unsigned* ia;
  long na;
  const unsigned* ib;
  long nb, second;
};

// Tail split of a grouped GEMM launch.  The tiles of a launch run in waves of
// gemm_slots(cfg) resident blocks; when the last wave would be mostly idle, the
// last total - dp_tiles tiles are cut into `splits` K-segments each.  Their
// partial tiles (BM x BN, row-major) go to ws and gemm_tail_reduce adds them in
// segment order (deterministic) and applies alpha / beta.
struct GemmTail {
  int dp_tiles = 0;     // tiles computed whole: blocks [0, dp_tiles)
  int splits = 1;       // 1: no tail split
  double* ws = nullptr;
};
int gemm_slots(int cfg);
// min_k: smallest K of the launch's problems; any_ksplit: a problem already uses split-K
GemmTail plan_gemm_tail(int cfg, int total_tiles, int min_k, bool any_ksplit, double* ws, size_t ws_doubles);
constexpr size_t kTailWorkspaceDoubles = (size_t)1024 * 128 * 128;   // 128 MiB

void launch_gemm(int cfg, bool ta, bool tb, const GemmProblem* d_probs, const int* d_prefix, int n_prob,
                 int total_tiles, const GemmTail& tail, hipStream_t s);
// Momentum-blocked contraction: C[m, n] = alpha * sum_k A[m, k] B[k, n] + beta * C
// restricted to the blocks allowed by a conserved quantity.  Rows, inner indices
// and columns of a block are lists of element offsets into the dense operands
// (the row offset of A plus the inner offset of A addresses A[m, k], and so on),
// so no operand is permuted.  One task is one 16 x 16 output tile of one block.
struct SgemmProblem {
  const double* A;
  const double* B;
  double* C;
  const unsigned* offAM;
  const unsigned* offAK;
  const unsigned* offBK;
  const unsigned* offBN;
  const unsigned* offCM;
  const unsigned* offCN;
  double alpha, beta;
  const int* active;     // optional run flag (0: skip)
};
struct SgemmTask {
  int prob;
  int mb, mlen;          // first row (index into offAM / offCM) and rows
  int kb, klen;          // first inner index (into offAK / offBK) and count
  int nb, nlen;          // first column (into offBN / offCN) and columns
  int part;              // -1: write C; else the 16 x 16 partial tile goes to ws[part * 256 ...]
  int shape;             // 0: one 16 x 16 MFMA tile (rows, columns <= 16); else a lane-mapped tile of
                         // 2^lr rows x 2^lc columns whose inner range is split over 2^ls lanes
                         // (lr | lc << 3 | ls << 6, lr + lc + ls = 6; never split into parts)
};
// shape code of a lane-mapped tile
constexpr int sgemm_thin_shape(int lr, int lc, int ls) { return lr | (lc << 3) | (ls << 6); }
// A tile whose inner range was split into `count` consecutive partial tiles
// ws[first .. first + count - 1]: C = alpha * (their sum, in order) + beta * C.
struct SgemmReduce {
  int prob;
  int mb, mlen;
  int nb, nlen;
  int first, count;
};
// Inner ranges longer than this are split into chunks of kSgemmChunk (or a
// power-of-two multiple of it when the partial tiles would not fit the workspace).
constexpr int kSgemmChunk = 64;
void launch_sgemm(const SgemmProblem* d_probs, const SgemmTask* d_tasks, int n_tasks, double* ws,
                  const SgemmReduce* d_red, int n_red, hipStream_t s);

// Momentum-blocked elementwise op over the allowed elements of Y only:
// Y[oy1[u] + oy2[v]] = alpha * s * X[ox1[u] + ox2[v]] + beta * Y[oy1[u] + oy2[v]] for
// every pair (u, v) of a matched pair of index-group blocks, s = *scale (a device
// scalar) or 1 (alpha = beta = 0: zero fill, nothing read).  Forbidden elements
// are never touched.
struct ElemProblem {
  const double* X;
  double* Y;
  const unsigned* ox1;
  const unsigned* oy1;
  const unsigned* ox2;
  const unsigned* oy2;
  double alpha, beta;
  const int* active;
  const double* scale;   // optional device scalar factor of X
};
struct ElemTask {
  long long first;       // elements of the tasks before this one
  int prob;
  int u0, ulen, v0, vlen;
};
// d_bfirst: per 256-element block the task of its first element, then the last
// task (total / 256 rounded up, plus one entries)
void launch_elem(const ElemProblem* d_probs, const ElemTask* d_tasks, const int* d_bfirst, int n_tasks,
                 long long total, hipStream_t s);

// Momentum-blocked full contraction: out = alpha * sum X[ox1[u] + ox2[v]] * Y[oy1[u] + oy2[v]]
// + beta * out over the allowed elements (task list as for elem_kernel).  Each
// problem's elements start at a 256-element block boundary, so a block belongs
// to one problem; its partial sums are partial[first_block ..
// first_block + n_blocks - 1], added in order by the final kernel.
struct DotbProblem {
  const double* X;
  const double* Y;
  const unsigned* ox1;
  const unsigned* oy1;
  const unsigned* ox2;
  const unsigned* oy2;
  double* out;
  double alpha, beta;
  const int* active;
  int first_block, n_blocks;
};
void launch_dotb(const DotbProblem* d_probs, int n_prob, const ElemTask* d_tasks, const int* d_bfirst, int n_tasks,
                 long long total, double* partial, hipStream_t s);

void launch_splitk_reduce(const GemmProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks,
                          hipStream_t s);
void launch_permute(const PermProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks,
                    hipStream_t s);
void launch_dot(const DotProblem* d_probs, int n_prob, int blocks_per, double* d_partial, hipStream_t s);

// GEMM tile configurations: 0: 128x128 BK 16, 1: 64x64 BK 16, 2: 128x128 BK 32
constexpr int kGemmConfigs = 3;
inline int gemm_bm(int cfg) { return cfg == 1 ? 64 : 128; }
inline int gemm_bn(int cfg) { return cfg == 1 ? 64 : 128; }

}  // namespace ftcc
