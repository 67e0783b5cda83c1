// Device kernels of the FT-CCSD hot path (gfx950, FP64 throughout).
//
//   gemm_mfma      grouped C = alpha * op(A) op(B) + beta * C on v_mfma_f64_16x16x4f64,
//                  LDS double-buffered 128x128 (or 64x64) tiles, XCD-aware tile order,
//                  optional split-K with a deterministic second-pass reduction, C in
//                  GEMM layout or written into a permuted layout through row and
//                  column offset tables
//   permute4       grouped 4-index transpose-accumulate Y[perm] = alpha X + beta Y,
//                  LDS-tiled when the fastest index moves
//   dot            grouped full contractions (two-pass, deterministic)
//   sgemm, elem,   momentum-blocked contractions over element-offset lists (one wave
//   dotb           per 16x16 MFMA tile), unary ops and full contractions over the
//                  momentum-allowed elements
//
// The imaginary-time kernels (thermal blocks, propagator, adjoint) are in
// tau_kernels.hip.
//
// Every grouped kernel takes a device array of problem descriptors; the block
// index is mapped to (problem, tile) through the exclusive prefix of tile counts.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "gmem.h"
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

// Tile (tm, tn) of the local tile index inside a problem: bands of 8 tile-rows,
// column-major inside a band, so that consecutive blocks share B columns and A rows.
__device__ __forceinline__ void tile_coords(int local, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int GM = 8;
  const int band = local / (GM * tiles_n);
  const int first_m = band * GM;
  const int band_rows = min(GM, tiles_m - first_m);
  tm = first_m + (local % (GM * tiles_n)) % band_rows;
  tn = (local % (GM * tiles_n)) / band_rows;
}

// ------------------------------------------------------------------ GEMM
// Fragment layouts of v_mfma_f64_16x16x4f64 (wave64):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l holds D[4 * r + l / 16][l % 16], r = 0..3
typedef double double4_t __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, bool TA, bool TB, int WPE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, 4)))
gemm_mfma_kernel(const GemmProblem* __restrict__ probs, const int* __restrict__ prefix,
                 int n_prob, int dp_tiles, int splits, double* __restrict__ ws) {
  constexpr int WM = BM / 2, WN = BN / 2;        // 2 x 2 waves
  constexpr int FM = WM / 16, FN = WN / 16;      // MFMA tiles per wave
  // LDS tiles keep the global layout of each operand (no transposing stores):
  //   TA: As[k][m] (pitch BM+1)   !TA: As[m][k] (pitch BK+1)
  //   TB: Bs[n][k] (pitch BK+1)   !TB: Bs[k][n] (pitch BN+1)
  constexpr int PA = TA ? BM + 1 : BK + 1;
  constexpr int PB = TB ? BK + 1 : BN + 1;
  constexpr int SA = TA ? BK * PA : BM * PA;
  constexpr int SB = TB ? BN * PB : BK * PB;
  constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
  // thread -> element maps: e = tid + 256 j; rows of the stored layout
  constexpr int RA = TA ? BM : BK;   // contiguous extent of A's stored rows
  constexpr int RB = TB ? BK : BN;
  __shared__ double As[2][SA];
  __shared__ double Bs[2][SB];

  // blocks [0, dp_tiles): whole tiles in XCD-aware order; the rest: K-segments of
  // the tail tiles (unit u = segment u % splits of tile dp_tiles + u / splits)
  const int b = blockIdx.x;
  int tile, kseg = -1;
  if (b < dp_tiles) {
    tile = xcd_remap(b, dp_tiles);
  } else {
    const int u = b - dp_tiles;
    tile = dp_tiles + u / splits;
    kseg = u % splits;
  }
  const int pi = find_problem(prefix, n_prob, tile);
  const GemmProblem& P = probs[pi];
  if (P.active && *gview(P.active) == 0) return;   // the whole block leaves before any barrier
  int local = tile - prefix[pi];
  const int tiles_mn = P.tiles_m * P.tiles_n;
  const int ks = local / tiles_mn;
  local -= ks * tiles_mn;
  int tm, tn;
  tile_coords(local, P.tiles_m, P.tiles_n, tm, tn);

  const int m0 = tm * BM, n0 = tn * BN;
  int kbeg, kend;
  if (kseg < 0) {
    kbeg = ks * P.kchunk;
    kend = min(P.K, kbeg + P.kchunk);
  } else {
    const int kc = ((P.K + splits - 1) / splits + BK - 1) / BK * BK;
    kbeg = kseg * kc;
    kend = min(P.K, kbeg + kc);
  }
  const int M = P.M, N = P.N;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Each thread loads LA elements of A: stored row r = (tid + 256 j) / RA, column c = tid % RA
  // (256 is a multiple of RA), i.e. rows advance by 256 / RA per j.  Offsets are 32-bit:
  // the host guarantees every operand holds fewer than 2^31 elements.
  const int ca = tid % RA, r0a = tid / RA;
  const int cb = tid % RB, r0b = tid / RB;
  constexpr int DRA = 256 / RA, DRB = 256 / RB;
  const gptr<const double> __restrict__ A = gview(P.A);
  const gptr<const double> __restrict__ B = gview(P.B);
  const int lda = (int)P.lda, ldb = (int)P.ldb;

  double ra[LA], rb[LB];
  // Branch-free operand loads of the K step starting at k0: the element index is
  // clamped into the operand (a valid address also past the step's K range) and
  // the elements outside the range are zeroed on their way into LDS, so that a
  // whole K step is one basic block that the scheduler can interleave.
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int j = 0; j < LA; ++j) {
      const int r = r0a + DRA * j;
      const unsigned off = TA ? (unsigned)(min(k0 + r, kend - 1) * lda + min(m0 + ca, M - 1))
                              : (unsigned)(min(m0 + r, M - 1) * lda + min(k0 + ca, kend - 1));
      ra[j] = A[off];
    }
#pragma unroll
    for (int j = 0; j < LB; ++j) {
      const int r = r0b + DRB * j;
      const unsigned off = TB ? (unsigned)(min(n0 + r, N - 1) * ldb + min(k0 + cb, kend - 1))
                              : (unsigned)(min(k0 + r, kend - 1) * ldb + min(n0 + cb, N - 1));
      rb[j] = B[off];
    }
  };
  auto store_tiles = [&](double* as, double* bs, int k0) {
#pragma unroll
    for (int j = 0; j < LA; ++j) {
      const int r = r0a + DRA * j;
      const bool ok = TA ? (k0 + r < kend && m0 + ca < M) : (m0 + r < M && k0 + ca < kend);
      as[r * PA + ca] = ok ? ra[j] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < LB; ++j) {
      const int r = r0b + DRB * j;
      const bool ok = TB ? (n0 + r < N && k0 + cb < kend) : (k0 + r < kend && n0 + cb < N);
      bs[r * PB + cb] = ok ? rb[j] : 0.0;
    }
  };

  double4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};

  const int nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  const int fr = lane & 15, fk = lane >> 4;
  const int abase = TA ? fk * PA + wm * WM + fr : (wm * WM + fr) * PA + fk;
  const int bbase = TB ? (wn * WN + fr) * PB + fk : fk * PB + wn * WN + fr;
  constexpr int ASTEP_I = TA ? 16 : 16 * PA;    // next MFMA tile in M
  constexpr int ASTEP_K = TA ? 4 * PA : 4;      // next k group
  constexpr int BSTEP_J = TB ? 16 * PB : 16;
  constexpr int BSTEP_K = TB ? 4 : 4 * PB;
  constexpr int KG = BK / 4;                    // k groups of one K step
  // One K step on LDS buffer CUR (a compile-time index, so that the compiler sees
  // that the stores into the other buffer never alias this step's fragment reads):
  // the global loads of the next step, the MFMAs of this one, the next step's
  // operands into the other buffer, a barrier.  The two waves that share a SIMD
  // run this same code and would otherwise fall into step: both in their MFMA
  // section together and then both in their loads and stores with the matrix
  // pipe idle.  The scheduling groups below spread the memory instructions
  // between the MFMAs instead.
  auto kstep = [&](auto cur_c, auto live_c, int it) {
    constexpr int CUR = decltype(cur_c)::value;
    const int kn = kbeg + (it + 1) * BK;
    load_tiles(kn);
    if constexpr (!decltype(live_c)::value) {   // a wave with no output in the tile: loads, stores, barrier
      store_tiles(As[CUR ^ 1], Bs[CUR ^ 1], kn);
      __syncthreads();
      return;
    }
    const double* as = As[CUR] + abase;
    const double* bs = Bs[CUR] + bbase;
    double af[2][FM], bf[2][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) af[0][i] = as[i * ASTEP_I];
#pragma unroll
    for (int j = 0; j < FN; ++j) bf[0][j] = bs[j * BSTEP_J];
#pragma unroll
    for (int kq = 0; kq < KG; ++kq) {
      const int c = kq & 1;
      if (kq + 1 < KG) {   // fetch the next k group while this one multiplies
#pragma unroll
        for (int i = 0; i < FM; ++i) af[c ^ 1][i] = as[(kq + 1) * ASTEP_K + i * ASTEP_I];
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[c ^ 1][j] = bs[(kq + 1) * BSTEP_K + j * BSTEP_J];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[c][i], bf[c][j], acc[i][j], 0, 0, 0);
    }
    store_tiles(As[CUR ^ 1], Bs[CUR ^ 1], kn);
    // Instruction order (MFMA slot u = 0 .. T-1): the first k group's fragment
    // reads, then after each MFMA at most one global load of the next step (every
    // other slot of the first 2 (LA + LB) when the step has room for that before
    // its stores, else the first LA + LB slots), one fragment read of the next k
    // group (second half of each group), one LDS store of the next step's operands
    // (last group only, long after their loads were issued).  Masks: 0x008 MFMA,
    // 0x020 VMEM read, 0x100 DS read, 0x200 DS write.
    {
      constexpr int MG = FM * FN, T = MG * KG, NV = LA + LB, NW = LA + LB;
      constexpr bool spread = T >= 2 * NV + NW;
      __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
#pragma unroll
      for (int u = 0; u < T; ++u) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        if (spread ? (u < 2 * NV && (u % 2) == 0) : (u < NV)) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        if (u < T - MG && (u % MG) >= MG - (FM + FN)) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        if (u >= T - NW) __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
      }
    }
    __syncthreads();
  };
  if (nk > 0) {
    load_tiles(kbeg);
    store_tiles(As[0], Bs[0], kbeg);
    __syncthreads();
  }
  // The last step's loads read clamped (valid) addresses and its stores fill the
  // buffer that is no longer read.  A wave whose 64x64 part of the tile lies
  // wholly outside C (edge tiles of a matrix that is not a multiple of the tile)
  // takes its share of the loads, stores and barriers but issues no MFMAs, which
  // leaves the matrix pipe to the other wave on its SIMD.  Both marches pass the
  // same barriers; the flag is made wave-uniform (a scalar branch), so a wave runs
  // exactly one of them.
  const int live = __builtin_amdgcn_readfirstlane((m0 + wm * WM < M && n0 + wn * WN < N) ? 1 : 0);
  auto march = [&](auto live_c) {
    for (int it = 0; it < nk; it += 2) {
      kstep(std::integral_constant<int, 0>{}, live_c, it);
      if (it + 1 < nk) kstep(std::integral_constant<int, 1>{}, live_c, it + 1);
    }
  };
  if (live)
    march(std::true_type{});
  else
    march(std::false_type{});

  // epilogue
  if (kseg >= 0) {   // partial tile of a tail segment, summed by gemm_tail_reduce
    const gptr<double> W = gview(ws) + (long)(b - dp_tiles) * (BM * BN);
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          W[(wm * WM + i * 16 + 4 * r + fk) * BN + wn * WN + j * 16 + fr] = acc[i][j][r];
    return;
  }
  gptr<double> C;
  long ldc;
  double alpha, beta;
  if (P.ksplit > 1) {
    C = gview(P.partial) + (long)ks * M * N;
    ldc = N;
    alpha = 1.0;
    beta = 0.0;
  } else {
    C = gview(P.C);
    ldc = P.ldc;
    alpha = P.alpha;
    beta = P.beta;
  }
  const bool tab = P.ksplit <= 1 && P.offM;   // uniform per block
  // Column offsets once per tile; then per row group of MFMA tiles the element
  // offsets (clamped into C for the elements outside it), all the target loads
  // together, then the stores: one memory latency per group instead of one per
  // element.
  long coff[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int gn = min(n0 + wn * WN + j * 16 + fr, N - 1);
    coff[j] = tab ? (long)gview(P.offN)[gn] : (long)gn;
  }
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    long off[4][FN];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = min(m0 + wm * WM + i * 16 + 4 * r + fk, M - 1);
      const long roff = tab ? (long)gview(P.offM)[gm] : (long)gm * ldc;
#pragma unroll
      for (int j = 0; j < FN; ++j) off[r][j] = roff + coff[j];
    }
    double cv[4][FN];
    if (beta != 0.0) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int j = 0; j < FN; ++j) cv[r][j] = C[off[r][j]];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wm * WM + i * 16 + 4 * r + fk;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const int gn = n0 + wn * WN + j * 16 + fr;
        if (gm < M && gn < N) {
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v += beta * cv[r][j];
          C[off[r][j]] = v;
        }
      }
    }
  }
}

// C = alpha * (sum of the K-segment partials, in segment order) + beta * C for the
// tail tiles of a launch; blockIdx.y = tail tile, 1024 elements per block in x.
template <int BM, int BN>
__global__ void __launch_bounds__(256) gemm_tail_reduce_kernel(const GemmProblem* __restrict__ probs,
                                                               const int* __restrict__ prefix, int n_prob,
                                                               int dp_tiles, int splits,
                                                               const double* __restrict__ ws) {
  const int t = dp_tiles + blockIdx.y;
  const int pi = find_problem(prefix, n_prob, t);
  const GemmProblem& P = probs[pi];
  if (P.active && *gview(P.active) == 0) return;
  int tm, tn;
  tile_coords(t - prefix[pi], P.tiles_m, P.tiles_n, tm, tn);   // tail launches have no split-K problems
  const gptr<const double> W = gview(ws) + (long)blockIdx.y * splits * (BM * BN);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = blockIdx.x * 1024 + u * 256 + threadIdx.x;
    if (e >= BM * BN) break;
    const int gm = tm * BM + e / BN, gn = tn * BN + e % BN;
    if (gm >= P.M || gn >= P.N) continue;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += W[(long)k * (BM * BN) + e];
    const long off = P.offM ? (long)gview(P.offM)[gm] + gview(P.offN)[gn] : (long)gm * P.ldc + gn;
    const gptr<double> c = gview(P.C) + off;
    double v = P.alpha * s;
    if (P.beta != 0.0) v += P.beta * (*c);
    *c = v;
  }
}

// Momentum-blocked tiles: one wave per 16 x 16 output tile, or per chunk of a
// long inner range (its partial tile then goes to the workspace and
// sgemm_reduce_kernel adds the chunks); operands are gathered through the
// block's offset lists straight into MFMA fragments (the blocks are small, so
// nothing is staged in LDS).  No barriers: waves leave independently.
__global__ void __launch_bounds__(256) sgemm_kernel(const SgemmProblem* __restrict__ probs,
                                                    const SgemmTask* __restrict__ tasks, int n_tasks,
                                                    double* __restrict__ ws) {
  const int lane = threadIdx.x & 63;
  // the task index is uniform over the wave: task and problem come in through
  // scalar loads and their pointers stay in scalar registers
  const int ti = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (ti >= n_tasks) return;
  const SgemmTask T = tasks[ti];
  const SgemmProblem& P = probs[T.prob];
  if (P.active && *gview(P.active) == 0) return;
  const gptr<const double> __restrict__ A = gview(P.A);
  const gptr<const double> __restrict__ B = gview(P.B);
  const gptr<const unsigned> __restrict__ offAK = gview(P.offAK) + T.kb;
  const gptr<const unsigned> __restrict__ offBK = gview(P.offBK) + T.kb;
  if (T.shape) {
    // Lane-mapped tile of a thin block (a single row or column, or a long inner
    // range on a few outputs): lane = (row, column, inner slice); each lane adds its
    // slice's products, 8 gathers in flight, then the slices are added by a fixed
    // butterfly over the wave (every lane takes part, so the order is the same on
    // every run).
    const int ls = (T.shape >> 6) & 7, lc = (T.shape >> 3) & 7;
    const int S = 1 << ls;
    const int s = lane & (S - 1);
    const int tc = (lane >> ls) & ((1 << lc) - 1);
    const int tr = lane >> (ls + lc);
    const bool ok = tr < T.mlen && tc < T.nlen;
    double acc = 0.0;
    if (ok) {
      const unsigned am = gview(P.offAM)[T.mb + tr];
      const unsigned bn = gview(P.offBN)[T.nb + tc];
      int k = s;
      for (; k + 7 * S < T.klen; k += 8 * S) {
        unsigned ak[8], bk[8];
        double a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          ak[u] = offAK[k + u * S];
          bk[u] = offBK[k + u * S];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a[u] = A[am + ak[u]];
          b[u] = B[bk[u] + bn];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(a[u], b[u], acc);
      }
      for (; k < T.klen; k += S) acc = fma(A[am + offAK[k]], B[offBK[k] + bn], acc);
    }
    for (int o = S >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (ok && s == 0) {
      const gptr<double> c = gview(P.C) + (size_t)gview(P.offCM)[T.mb + tr] + gview(P.offCN)[T.nb + tc];
      double v = P.alpha * acc;
      if (P.beta != 0.0) v += P.beta * (*c);
      *c = v;
    }
    return;
  }
  const int r = lane & 15, q = lane >> 4;
  const bool row_ok = r < T.mlen, col_ok = r < T.nlen;
  const unsigned am = row_ok ? gview(P.offAM)[T.mb + r] : 0u;
  const unsigned bn = col_ok ? gview(P.offBN)[T.nb + r] : 0u;
  double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
  // G groups of 4 inner indices per step: the offset loads of all groups are
  // issued together, then all operand gathers, then the MFMAs, so one step
  // waits for two memory latencies instead of two per group.  Loads past the
  // end of the range read the range's first entry (in bounds) and are zeroed.
  constexpr int G = 8;
  for (int k0 = 0; k0 < T.klen; k0 += 4 * G) {
    unsigned ak[G], bk[G];
    double a[G], b[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int k = k0 + 4 * u + q;
      const int kk = k < T.klen ? k : 0;
      ak[u] = offAK[kk];
      bk[u] = offBK[kk];
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const bool ok = k0 + 4 * u + q < T.klen;
      const double va = A[am + ak[u]];     // A fragment: row r, inner q
      const double vb = B[bk[u] + bn];     // B fragment: inner q, column r
      a[u] = (ok && row_ok) ? va : 0.0;
      b[u] = (ok && col_ok) ? vb : 0.0;
    }
#pragma unroll
    for (int u = 0; u < G; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
  if (T.part >= 0) {   // one chunk of a split inner range: the whole tile, lane-major
    const gptr<double> w = gview(ws) + (size_t)T.part * 256;
#pragma unroll
    for (int i = 0; i < 4; ++i) w[i * 64 + lane] = acc[i];
    return;
  }
  // the offsets of the lane's four elements (clamped into the tile), then the
  // target loads together, then the stores: one memory latency per stage
  // instead of a chain per element
  const size_t cn = gview(P.offCN)[T.nb + max(min(r, T.nlen - 1), 0)];
  size_t cm[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cm[i] = gview(P.offCM)[T.mb + max(min(4 * i + q, T.mlen - 1), 0)];
  const gptr<double> C = gview(P.C);
  double cv[4] = {0.0, 0.0, 0.0, 0.0};
  if (P.beta != 0.0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) cv[i] = C[cm[i] + cn];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (4 * i + q < T.mlen && r < T.nlen) C[cm[i] + cn] = P.alpha * acc[i] + P.beta * cv[i];
}

// Sum of the partial tiles of a split inner range, in chunk order (deterministic).
__global__ void __launch_bounds__(256) sgemm_reduce_kernel(const SgemmProblem* __restrict__ probs,
                                                           const SgemmReduce* __restrict__ red, int n_red,
                                                           const double* __restrict__ ws) {
  const int lane = threadIdx.x & 63;
  const int ti = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (ti >= n_red) return;
  const SgemmReduce R = red[ti];
  const SgemmProblem& P = probs[R.prob];
  if (P.active && *gview(P.active) == 0) return;
  const int r = lane & 15, q = lane >> 4;
  // chunk partials added in chunk order per element (deterministic); offsets,
  // target loads and stores batched over the lane's four elements
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < R.count; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += gview(ws)[(size_t)(R.first + c) * 256 + i * 64 + lane];
  const size_t cn = gview(P.offCN)[R.nb + max(min(r, R.nlen - 1), 0)];
  size_t cm[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) cm[i] = gview(P.offCM)[R.mb + max(min(4 * i + q, R.mlen - 1), 0)];
  const gptr<double> C = gview(P.C);
  double cv[4] = {0.0, 0.0, 0.0, 0.0};
  if (P.beta != 0.0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) cv[i] = C[cm[i] + cn];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (4 * i + q < R.mlen && r < R.nlen) C[cm[i] + cn] = P.alpha * acc[i] + P.beta * cv[i];
}

// One thread per allowed element; the task is found by binary search over the
// element prefix, between the tasks of this block's first element and of the
// next block's (a few steps instead of a search of the whole list).
__global__ void __launch_bounds__(256) elem_kernel(const ElemProblem* __restrict__ probs,
                                                   const ElemTask* __restrict__ tasks,
                                                   const int* __restrict__ bfirst, long long total) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  int lo = gview(bfirst)[blockIdx.x], hi = gview(bfirst)[blockIdx.x + 1];
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].first <= e) lo = mid; else hi = mid - 1;
  }
  const ElemTask& T = tasks[lo];
  const ElemProblem& P = probs[T.prob];
  if (P.active && *gview(P.active) == 0) return;
  const int r = (int)(e - T.first);
  const int u = T.u0 + r / T.vlen, v = T.v0 + r % T.vlen;
  const gptr<double> y = gview(P.Y) + gview(P.oy1)[u] + gview(P.oy2)[v];
  double val = 0.0;
  if (P.alpha != 0.0) {
    const double a = P.scale ? P.alpha * *gview(P.scale) : P.alpha;
    val = a * gview(P.X)[gview(P.ox1)[u] + gview(P.ox2)[v]];
  }
  if (P.beta != 0.0) val += P.beta * (*y);
  *y = val;
}

// Blocked dot: one thread per allowed element (padding threads add 0), then a
// block sum per 256 elements; every thread reaches the barrier.
__global__ void __launch_bounds__(256) dotb_partial_kernel(const DotbProblem* __restrict__ probs,
                                                           const ElemTask* __restrict__ tasks,
                                                           const int* __restrict__ bfirst, long long total,
                                                           double* __restrict__ partial) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (e < total) {
    int lo = gview(bfirst)[blockIdx.x], hi = gview(bfirst)[blockIdx.x + 1];
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].first <= e) lo = mid; else hi = mid - 1;
    }
    const ElemTask& T = tasks[lo];
    const DotbProblem& P = probs[T.prob];
    const long long r = e - T.first;
    if (r >= 0 && r < (long long)T.ulen * T.vlen) {
      const int u = T.u0 + (int)(r / T.vlen), w = T.v0 + (int)(r % T.vlen);
      v = gview(P.X)[gview(P.ox1)[u] + gview(P.ox2)[w]] * gview(P.Y)[gview(P.oy1)[u] + gview(P.oy2)[w]];
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// One block per problem: strided sums of its block partials, then a tree in LDS
// (a fixed order: deterministic).
__global__ void __launch_bounds__(256) dotb_final_kernel(const DotbProblem* __restrict__ probs, int n_prob,
                                                         const double* partial) {
  const DotbProblem& P = probs[blockIdx.x];
  if (P.active && *gview(P.active) == 0) return;   // uniform per block, before the barriers
  double s = 0.0;
  for (int b = threadIdx.x; b < P.n_blocks; b += 256) s += gview(partial)[P.first_block + b];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  double v = P.alpha * red[0];
  const gptr<double> out = gview(P.out);
  if (P.beta != 0.0) v += P.beta * (*out);
  *out = v;
}

// C = alpha * sum_s partial[s] + beta * C for split-K problems
__global__ void splitk_reduce_kernel(const GemmProblem* __restrict__ probs, const int* __restrict__ prefix,
                                     int n_prob, int total) {
  const int pi = find_problem(prefix, n_prob, blockIdx.x);
  const GemmProblem P = probs[pi];
  if (P.ksplit <= 1 || (P.active && *gview(P.active) == 0)) return;
  const long mn = (long)P.M * P.N;
  const long chunk = (long)(blockIdx.x - prefix[pi]) * 256 * 4;
  for (int u = 0; u < 4; ++u) {
    long e = chunk + u * 256 + threadIdx.x;
    if (e >= mn) return;
    double s = 0.0;
    for (int k = 0; k < P.ksplit; ++k) s += gview(P.partial)[k * mn + e];
    long gm = e / P.N, gn = e % P.N;
    const long off = P.offM ? (long)gview(P.offM)[gm] + gview(P.offN)[gn] : gm * P.ldc + gn;
    const gptr<double> c = gview(P.C) + off;
    double v = P.alpha * s;
    if (P.beta != 0.0) v += P.beta * (*c);
    *c = v;
  }
}

// ------------------------------------------------------------------ permute
FastDiv make_fastdiv(unsigned int d) {
  FastDiv f;
  f.d = d;
  unsigned int l = 0;
  while ((1u << l) < d) ++l;     // l = ceil(log2 d)
  // mul = floor(2^32 (2^l - d) / d) + 1, valid for numerators < 2^31
  f.mul = (unsigned int)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  f.shr = l;
  return f;
}

__device__ __forceinline__ unsigned int fdiv(unsigned int x, const FastDiv& f) {
  const unsigned int t = __umulhi(x, f.mul);
  return (t + ((x - t) >> 1)) >> (f.shr > 0 ? f.shr - 1 : 0);
}

__device__ __forceinline__ void fdivmod(unsigned int x, const FastDiv& f, unsigned int& q, unsigned int& r) {
  q = (f.d == 1) ? x : fdiv(x, f);
  r = x - q * f.d;
}

// Y[o0,o1,o2,o3] = alpha * X[sum_k o_k * xs[k]] + beta * Y   (Y contiguous, dims d)
// Row path (X fastest = Y fastest): 1024 consecutive Y elements per block.
// Tiled path: a 32x32 LDS tile over Y axes (tb, 3) keeps reads and writes coalesced.
__global__ void __launch_bounds__(256) permute4_kernel(const PermProblem* __restrict__ probs,
                                                       const int* __restrict__ prefix, int n_prob) {
  const int pi = find_problem(prefix, n_prob, blockIdx.x);
  const PermProblem& P = probs[pi];
  if (P.active && *gview(P.active) == 0) return;   // uniform per block, before the barrier
  const unsigned int local = blockIdx.x - prefix[pi];
  const double alpha = P.scale ? P.alpha * (*gview(P.scale)) : P.alpha;
  const double beta = P.beta;
  const gptr<const double> __restrict__ X = gview(P.X);
  const gptr<double> __restrict__ Y = gview(P.Y);
  __shared__ double tileb[32][33];
  if (P.tb < 0) {
    const unsigned int total = (unsigned int)P.d[0] * P.d[1] * P.d[2] * P.d[3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned int e = local * 1024u + u * 256u + threadIdx.x;
      if (e >= total) break;
      unsigned int r = e, o3, o2, o1, o0;
      fdivmod(r, P.div[3], r, o3);
      fdivmod(r, P.div[2], r, o2);
      fdivmod(r, P.div[1], o0, o1);
      const long xo = o0 * P.xs[0] + o1 * P.xs[1] + o2 * P.xs[2] + (long)o3 * P.xs[3];
      double v = (alpha != 0.0) ? alpha * X[xo] : 0.0;
      if (beta != 0.0) v += beta * Y[e];
      Y[e] = v;
    }
    return;
  }
  const int tb = P.tb;
  unsigned int r = local, t3, tbb, iq, ip;
  fdivmod(r, P.tdiv[0], r, t3);
  fdivmod(r, P.tdiv[1], r, tbb);
  fdivmod(r, P.div[P.oth[1]], ip, iq);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const long base = (long)ip * P.xs[P.oth[0]] + (long)iq * P.xs[P.oth[1]];
  const int b0 = tbb * 32, c0 = t3 * 32;
  const int db = P.d[tb], d3 = P.d[3];
  const long xsb = P.xs[tb], xs3 = P.xs[3];
#pragma unroll
  for (int y = ty; y < 32; y += 8) {
    const int ob = b0 + tx, o3 = c0 + y;
    tileb[y][tx] = (ob < db && o3 < d3 && alpha != 0.0) ? X[base + ob * xsb + o3 * xs3] : 0.0;
  }
  __syncthreads();
  // Y strides of the four axes
  long ys[4];
  ys[3] = 1;
  ys[2] = d3;
  ys[1] = ys[2] * P.d[2];
  ys[0] = ys[1] * P.d[1];
  const long ybase = (long)ip * ys[P.oth[0]] + (long)iq * ys[P.oth[1]];
#pragma unroll
  for (int y = ty; y < 32; y += 8) {
    const int ob = b0 + y, o3 = c0 + tx;
    if (ob < db && o3 < d3) {
      const long yo = ybase + ob * ys[tb] + o3;
      double v = alpha * tileb[tx][y];
      if (beta != 0.0) v += beta * Y[yo];
      Y[yo] = v;
    }
  }
}

// ------------------------------------------------------------------ dot
__global__ void dot_partial_kernel(const DotProblem* __restrict__ probs, int blocks_per, double* partial) {
  const int pi = blockIdx.x / blocks_per;
  const int bi = blockIdx.x % blocks_per;
  const DotProblem P = probs[pi];
  if (P.active && *gview(P.active) == 0) return;
  double s = 0.0;
  if (P.ia) {
    const long cnt = P.na + P.nb;
    for (long t = (long)bi * 256 + threadIdx.x; t < cnt; t += (long)blocks_per * 256) {
      const long e = t < P.na ? (long)gview(P.ia)[t] : P.second + (long)gview(P.ib)[t - P.na];
      s += gview(P.X)[e] * gview(P.Y)[e];
    }
  } else {
    for (long e = (long)bi * 256 + threadIdx.x; e < P.len; e += (long)blocks_per * 256)
      s += gview(P.X)[e] * gview(P.Y)[e];
  }
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
  if (P.active && *gview(P.active) == 0) return;
  double s = 0.0;
  for (int b = 0; b < blocks_per; ++b) s += partial[pi * blocks_per + b];
  double v = P.alpha * s;
  const gptr<double> out = gview(P.out);
  if (P.beta != 0.0) v += P.beta * (*out);
  *out = v;
}

// ------------------------------------------------------------------ launchers
template <int BM, int BN, int BK, bool TA, bool TB>
static void launch_gemm_t(const GemmProblem* d_probs, const int* d_prefix, int n_prob, int total_tiles,
                          const GemmTail& tail, hipStream_t s) {
  constexpr int WPE = (BK == 16) ? 2 : 1;
  const bool split = tail.splits > 1 && tail.dp_tiles < total_tiles;
  const int dp = split ? tail.dp_tiles : total_tiles;
  const int blocks = dp + (split ? (total_tiles - dp) * tail.splits : 0);
  hipLaunchKernelGGL((gemm_mfma_kernel<BM, BN, BK, TA, TB, WPE>), dim3(blocks), dim3(256), 0, s, d_probs, d_prefix,
                     n_prob, dp, split ? tail.splits : 1, tail.ws);
  if (split)
    hipLaunchKernelGGL((gemm_tail_reduce_kernel<BM, BN>), dim3((BM * BN + 1023) / 1024, total_tiles - dp),
                       dim3(256), 0, s, d_probs, d_prefix, n_prob, dp, tail.splits, (const double*)tail.ws);
}

void launch_gemm(int cfg, bool ta, bool tb, const GemmProblem* d_probs, const int* d_prefix, int n_prob,
                 int total_tiles, const GemmTail& tail, hipStream_t s) {
  if (total_tiles <= 0) return;
#define FTCC_G(BM, BN, BK)                                                                              \
  do {                                                                                                  \
    if (ta && tb) launch_gemm_t<BM, BN, BK, true, true>(d_probs, d_prefix, n_prob, total_tiles, tail, s);    \
    else if (ta) launch_gemm_t<BM, BN, BK, true, false>(d_probs, d_prefix, n_prob, total_tiles, tail, s);    \
    else if (tb) launch_gemm_t<BM, BN, BK, false, true>(d_probs, d_prefix, n_prob, total_tiles, tail, s);    \
    else launch_gemm_t<BM, BN, BK, false, false>(d_probs, d_prefix, n_prob, total_tiles, tail, s);           \
  } while (0)
  if (cfg == 0) FTCC_G(128, 128, 16);
  else if (cfg == 1) FTCC_G(64, 64, 16);
  else FTCC_G(128, 128, 32);
#undef FTCC_G
}

// Resident blocks of one configuration on the current device (occupancy x CUs).
int gemm_slots(int cfg) {
  static int cache[kGemmConfigs] = {0, 0, 0};
  if (cfg < 0 || cfg >= kGemmConfigs) return 0;
  if (cache[cfg] > 0) return cache[cfg];
  int dev = 0, per_cu = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  hipError_t e;
  if (cfg == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_mfma_kernel<128, 128, 16, false, false, 2>, 256, 0);
  else if (cfg == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_mfma_kernel<64, 64, 16, false, false, 2>, 256, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gemm_mfma_kernel<128, 128, 32, false, false, 1>, 256, 0);
  if (e != hipSuccess || per_cu <= 0) return 0;
  cache[cfg] = per_cu * prop.multiProcessorCount;
  return cache[cfg];
}

// Choose the tail split: waves of `slots` blocks; the r = total mod slots tiles of
// the last wave are cut into s segments when ceil(r s / slots) / s waves of
// segment work beat the one wave they would otherwise take.
GemmTail plan_gemm_tail(int cfg, int total_tiles, int min_k, bool any_ksplit, double* ws, size_t ws_doubles) {
  GemmTail t;
  t.dp_tiles = total_tiles;
  const int slots = gemm_slots(cfg);
  if (!ws || any_ksplit || slots <= 0 || total_tiles < slots) return t;
  const int r = total_tiles % slots;
  if (r == 0) return t;
  const int bm = gemm_bm(cfg), bn = gemm_bn(cfg), bk = (cfg == 2) ? 32 : 16;
  double best = 1.0;
  int best_s = 1;
  for (int s = 2; s <= 8; ++s) {
    if (min_k / s < 4 * bk) break;
    if ((size_t)r * s * bm * bn > ws_doubles) break;
    const double waves = (double)((r * s + slots - 1) / slots) / s + 0.02 * s;   // + segment reduce
    if (waves < best) {
      best = waves;
      best_s = s;
    }
  }
  if (best_s > 1) {
    t.dp_tiles = total_tiles - r;
    t.splits = best_s;
    t.ws = ws;
  }
  return t;
}

void launch_splitk_reduce(const GemmProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks,
                          hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(splitk_reduce_kernel, dim3(total_blocks), dim3(256), 0, s, d_probs, d_prefix, n_prob,
                     total_blocks);
}

void launch_sgemm(const SgemmProblem* d_probs, const SgemmTask* d_tasks, int n_tasks, double* ws,
                  const SgemmReduce* d_red, int n_red, hipStream_t s) {
  if (n_tasks <= 0) return;
  hipLaunchKernelGGL(sgemm_kernel, dim3((n_tasks + 3) / 4), dim3(256), 0, s, d_probs, d_tasks, n_tasks, ws);
  if (n_red > 0)
    hipLaunchKernelGGL(sgemm_reduce_kernel, dim3((n_red + 3) / 4), dim3(256), 0, s, d_probs, d_red, n_red,
                       (const double*)ws);
}

void launch_elem(const ElemProblem* d_probs, const ElemTask* d_tasks, const int* d_bfirst, int n_tasks,
                 long long total, hipStream_t s) {
  if (n_tasks <= 0 || total <= 0) return;
  hipLaunchKernelGGL(elem_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, d_probs, d_tasks, d_bfirst,
                     total);
}

void launch_dotb(const DotbProblem* d_probs, int n_prob, const ElemTask* d_tasks, const int* d_bfirst, int n_tasks,
                 long long total, double* partial, hipStream_t s) {
  if (n_prob <= 0) return;
  const long long blocks = (total + 255) / 256;
  if (blocks > 0 && n_tasks > 0)
    hipLaunchKernelGGL(dotb_partial_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d_probs, d_tasks, d_bfirst,
                       total, partial);
  hipLaunchKernelGGL(dotb_final_kernel, dim3(n_prob), dim3(256), 0, s, d_probs, n_prob, (const double*)partial);
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
