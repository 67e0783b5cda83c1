// Tensor-program engine: lowering of contractions to grouped kernel launches.
#include "engine.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <stdexcept>

#include "util.h"

namespace ftcc {

// ------------------------------------------------------------------ Program
int Program::tensor(const std::string& name, int rank, TensorKind kind) {
  for (size_t i = 0; i < t.size(); ++i)
    if (t[i].name == name) throw std::runtime_error("duplicate tensor " + name);
  t.push_back({name, rank, kind, false});
  return (int)t.size() - 1;
}

int Program::id(const std::string& name) const {
  for (size_t i = 0; i < t.size(); ++i)
    if (t[i].name == name) return (int)i;
  throw std::runtime_error("unknown tensor " + name);
}

void Program::op(const std::string& out, const std::string& oi, double alpha, const std::string& a,
                 const std::string& ai, const std::string& b, const std::string& bi, bool acc) {
  SymOp o;
  o.out = id(out);
  o.oi = oi;
  o.alpha = alpha;
  o.a = id(a);
  o.ai = ai;
  o.b = b.empty() ? -1 : id(b);
  o.bi = bi;
  o.accumulate = acc;
  if ((int)oi.size() != t[o.out].rank || (int)ai.size() != t[o.a].rank ||
      (o.b >= 0 && (int)bi.size() != t[o.b].rank))
    throw std::runtime_error("rank mismatch in op on " + out);
  o.setup = false;
  ops.push_back(o);
}

// An intermediate is derived (a constant combination) when every op writing it
// reads only constants or derived tensors; those ops form the set-up list.
void Program::set_law(const std::string& name, const std::vector<int>& signs) {
  const int k = id(name);
  if ((int)signs.size() != t[k].rank) throw std::runtime_error("law rank mismatch: " + name);
  if ((int)law.size() < (int)t.size()) law.resize(t.size());
  law[k] = signs;
}

void Program::finalize() {
  law.resize(t.size());
  for (auto& d : t) d.derived = false;
  bool changed = true;
  while (changed) {
    changed = false;
    for (size_t k = 0; k < t.size(); ++k) {
      if (t[k].kind != T_INTER || t[k].derived) continue;
      bool any = false, all_const = true;
      for (const SymOp& o : ops) {
        if (o.out != (int)k) continue;
        any = true;
        auto c = [&](int x) { return x < 0 || t[x].kind == T_CONST || t[x].derived; };
        if (!c(o.a) || !c(o.b)) all_const = false;
      }
      if (any && all_const) {
        t[k].derived = true;
        changed = true;
      }
    }
  }
  for (SymOp& o : ops) o.setup = t[o.out].derived;
  finalized_ = true;
}

// ------------------------------------------------------------------ helpers
static long ipow(long n, int r) {
  long v = 1;
  for (int k = 0; k < r; ++k) v *= n;
  return v;
}

static bool has(const std::string& s, char c) { return s.find(c) != std::string::npos; }

static std::string filter(const std::string& src, const std::string& a, const std::string& b, bool in_a,
                          bool in_b) {
  std::string out;
  for (char c : src)
    if (has(a, c) == in_a && has(b, c) == in_b) out.push_back(c);
  return out;
}

Executor::~Executor() {
  for (void* p : owned_) (void)hipFree(p);
}

void* Executor::upload(const void* host, size_t bytes) {
  void* d = nullptr;
  FTCC_HIP(hipMalloc(&d, bytes > 0 ? bytes : 8));
  if (bytes) FTCC_HIP(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
  owned_.push_back(d);
  return d;
}

void Executor::release(const std::vector<void*>& dev) {
  if (dev.empty()) return;
  std::vector<void*> keep;
  keep.reserve(owned_.size());
  for (void* p : owned_) {
    if (std::find(dev.begin(), dev.end(), p) != dev.end()) FTCC_HIP(hipFree(p));
    else keep.push_back(p);
  }
  owned_.swap(keep);
}

using Ranges = std::vector<std::pair<uintptr_t, uintptr_t>>;

static void add_range(Ranges& v, const void* p, size_t bytes) {
  if (p && bytes) v.emplace_back((uintptr_t)p, (uintptr_t)p + bytes);
}

// sorted, overlapping and touching ranges joined
static void normalize(Ranges& v) {
  if (v.empty()) return;
  std::sort(v.begin(), v.end());
  size_t w = 0;
  for (size_t k = 1; k < v.size(); ++k) {
    if (v[k].first <= v[w].second) v[w].second = std::max(v[w].second, v[k].second);
    else v[++w] = v[k];
  }
  v.resize(w + 1);
}

static bool overlaps(const Ranges& a, const Ranges& b) {
  size_t i = 0, j = 0;
  while (i < a.size() && j < b.size()) {
    if (a[i].second <= b[j].first) ++i;
    else if (b[j].second <= a[i].first) ++j;
    else return true;
  }
  return false;
}

// must b run after a (a earlier in program order)?
static bool ordered(const Launch& a, const Launch& b) {
  if (!a.ranged || !b.ranged) return true;
  return overlaps(a.wr, b.rd) || overlaps(a.wr, b.wr) || overlaps(a.rd, b.wr);
}

// Task of the first element of every 256-element block of an element-task list
// (the largest task index whose first element is at or before it), and the last
// task after the final block: the kernels search only between two neighbours.
static std::vector<int> block_first_tasks(const std::vector<ElemTask>& tasks, long long total) {
  const long long nb = (total + 255) / 256;
  std::vector<int> bf((size_t)nb + 1);
  int t = 0;
  for (long long b = 0; b < nb; ++b) {
    while (t + 1 < (int)tasks.size() && tasks[t + 1].first <= b * 256) ++t;
    bf[(size_t)b] = t;
  }
  bf[(size_t)nb] = tasks.empty() ? 0 : (int)tasks.size() - 1;
  return bf;
}

// ------------------------------------------------------------------ lowering: permute / fill
void Executor::perm(std::vector<Launch>& dst, const PerProb& X, const std::string& xi, const PerProb& Y,
                    const std::string& yi, double alpha, double beta, const std::vector<const double*>* scale,
                    const std::string& tag) {
  const int np = (int)probs_.size();
  const int r = (int)yi.size();
  if ((int)xi.size() != r) throw std::runtime_error("permute rank mismatch " + xi + "->" + yi);
  std::vector<PermProblem> ps(np);
  std::vector<int> prefix(np);
  Ranges rd, wr;
  int total = 0;
  for (int p = 0; p < np; ++p) {
    const long n = probs_[p].n;
    PermProblem& q = ps[p];
    q.X = X[p];
    q.Y = Y[p];
    q.scale = scale ? (*scale)[p] : nullptr;
    q.alpha = alpha;
    q.beta = beta;
    q.active = gate_for(dst, p);
    // Y axes padded on the left to 4; X strides of each Y axis
    for (int k = 0; k < 4; ++k) {
      q.d[k] = 1;
      q.xs[k] = 0;
    }
    for (int k = 0; k < r; ++k) {
      const int ya = 4 - r + k;
      const size_t pos = xi.find(yi[k]);
      if (pos == std::string::npos) throw std::runtime_error("permute letter mismatch " + xi + "->" + yi);
      q.d[ya] = (int)n;
      q.xs[ya] = ipow(n, r - 1 - (int)pos);
    }
    q.tb = -1;
    if (q.xs[3] != 1 && q.d[3] > 1) {
      for (int k = 0; k < 3; ++k)
        if (q.xs[k] == 1 && q.d[k] > 1) q.tb = k;
    }
    for (int k = 0; k < 4; ++k) q.div[k] = make_fastdiv((unsigned)q.d[k]);
    prefix[p] = total;
    if (alpha != 0.0) add_range(rd, X[p], sizeof(double) * (size_t)ipow(n, r));
    if (q.scale) add_range(rd, q.scale, sizeof(double));
    add_range(wr, Y[p], sizeof(double) * (size_t)ipow(n, r));
    if (q.tb < 0) {
      const long el = (long)q.d[0] * q.d[1] * q.d[2] * q.d[3];
      total += (int)((el + 1023) / 1024);
    } else {
      int c = 0;
      for (int k = 0; k < 3; ++k)
        if (k != q.tb) q.oth[c++] = k;
      const int nt3 = (q.d[3] + 31) / 32, ntb = (q.d[q.tb] + 31) / 32;
      q.tdiv[0] = make_fastdiv((unsigned)nt3);
      q.tdiv[1] = make_fastdiv((unsigned)ntb);
      total += nt3 * ntb * q.d[q.oth[0]] * q.d[q.oth[1]];
    }
  }
  Launch L;
  L.kind = Launch::PERM;
  L.n_prob = np;
  L.total = total;
  L.d_desc = upload(ps.data(), sizeof(PermProblem) * np);
  L.d_prefix = (int*)upload(prefix.data(), sizeof(int) * np);
  L.tag = tag;
  for (int p = 0; p < np; ++p)
    L.bytes += sizeof(double) * (double)ipow(probs_[p].n, r) * ((alpha != 0.0) + (beta != 0.0) + 1);
  L.rd = std::move(rd);
  L.wr = std::move(wr);
  L.ranged = true;
  dst.push_back(L);
}

void Executor::fill(std::vector<Launch>& dst, const PerProb& Y, int rank, const std::string& tag, int t_y) {
  // zero fill: the contiguous permute path with alpha = 0 and beta = 0 reads neither X nor Y;
  // with momentum laws only the allowed elements (the others never leave zero)
  if (rank > 0) {
    std::string idx;
    for (int k = 0; k < rank; ++k) idx.push_back((char)('p' + k));
    if (elem_blocked(dst, Y, idx, Y, idx, 0.0, 0.0, t_y, t_y, tag)) return;
  }
  dense_guard(tag, {t_y});
  const int np = (int)probs_.size();
  std::vector<PermProblem> ps(np);
  std::vector<int> prefix(np);
  int total = 0;
  for (int p = 0; p < np; ++p) {
    const long n = probs_[p].n;
    PermProblem& q = ps[p];
    std::memset(&q, 0, sizeof(q));
    q.X = Y[p];
    q.Y = Y[p];
    q.d[0] = 1;
    q.d[1] = 1;
    q.d[2] = 1;
    q.d[3] = (int)ipow(n, rank);
    q.xs[3] = 1;
    q.tb = -1;
    for (int k = 0; k < 4; ++k) q.div[k] = make_fastdiv((unsigned)q.d[k]);
    q.alpha = 0.0;
    q.beta = 0.0;
    q.active = gate_for(dst, p);
    prefix[p] = total;
    total += (int)((q.d[3] + 1023) / 1024);
  }
  Launch L;
  for (int p = 0; p < np; ++p) {
    add_range(L.wr, Y[p], sizeof(double) * (size_t)ipow(probs_[p].n, rank));
    L.bytes += sizeof(double) * (double)ipow(probs_[p].n, rank);
  }
  L.ranged = true;
  L.kind = Launch::FILL;
  L.n_prob = np;
  L.total = total;
  L.d_desc = upload(ps.data(), sizeof(PermProblem) * np);
  L.d_prefix = (int*)upload(prefix.data(), sizeof(int) * np);
  L.tag = tag;
  dst.push_back(L);
}

// Element offsets, in a tensor of layout `oi` (n per letter), of every index
// tuple of `letters` (first letter most significant): the rows or columns of a
// GEMM written straight into that tensor.  Built once per (n, letters, oi).
const unsigned* Executor::out_offsets(long n, const std::string& letters, const std::string& oi) {
  const std::string key = std::to_string(n) + ":" + letters + ":" + oi;
  auto it = out_tables_.find(key);
  if (it != out_tables_.end()) return it->second;
  const int r = (int)letters.size(), ro = (int)oi.size();
  std::vector<long> stride(r);
  for (int k = 0; k < r; ++k) stride[k] = ipow(n, ro - 1 - (int)oi.find(letters[k]));
  std::vector<unsigned> t((size_t)ipow(n, r));
  for (size_t idx = 0; idx < t.size(); ++idx) {
    long rem = (long)idx, off = 0;
    for (int k = r - 1; k >= 0; --k) {
      off += (rem % n) * stride[k];
      rem /= n;
    }
    t[idx] = (unsigned)off;
  }
  const unsigned* d = (const unsigned*)upload(t.data(), sizeof(unsigned) * std::max<size_t>(t.size(), 1));
  out_tables_[key] = d;
  return d;
}

Executor::PerProb Executor::const_permuted(int tensor, const PerProb& X, const std::string& xi,
                                           const std::string& yi) {
  // canonical key: the permutation as positions
  std::string key;
  for (char c : yi) key.push_back((char)('0' + xi.find(c)));
  auto k = std::make_pair(tensor, key);
  auto it = const_cache_.find(k);
  if (it != const_cache_.end()) return it->second;
  const int np = (int)probs_.size();
  PerProb Y(np);
  std::map<int, double*> per_inst;
  for (int p = 0; p < np; ++p) {
    const int inst = probs_[p].inst;
    if (!per_inst.count(inst)) {
      per_inst[inst] = const_alloc_(inst, (size_t)ipow(probs_[p].n, (int)xi.size()));
      const_bytes_ += sizeof(double) * (size_t)ipow(probs_[p].n, (int)xi.size());
    }
    Y[p] = per_inst[inst];
  }
  // one permute per instance: restrict to the first problem of each instance
  std::vector<ProblemRef> saved = probs_;
  std::vector<ProblemRef> firsts;
  PerProb Xf, Yf;
  std::map<int, bool> seen;
  for (int p = 0; p < np; ++p) {
    if (seen[probs_[p].inst]) continue;
    seen[probs_[p].inst] = true;
    firsts.push_back(probs_[p]);
    Xf.push_back(X[p]);
    Yf.push_back(Y[p]);
  }
  probs_ = firsts;
  perm(setup_, Xf, xi, Yf, yi, 1.0, 0.0, nullptr, "const-permute");
  probs_ = saved;
  const_cache_[k] = Y;
  return Y;
}

// Permuted copy of a non-constant value operand.  Copies are kept and reused by
// later consumers until the tensor is written again (its version changes); the
// operands of the backward program are forward values, fixed during backward.
Executor::PerProb Executor::value_permuted(std::vector<Launch>& dst, int tensor, const PerProb& X,
                                           const std::string& xi, const std::string& yi, const PerProb& scratch,
                                           const std::string& tag) {
  if (tensor < 0 || !cache_alloc_) {
    perm(dst, X, xi, scratch, yi, 1.0, 0.0, nullptr, tag);
    return scratch;
  }
  std::string key;
  for (char c : yi) key.push_back((char)('0' + xi.find(c)));
  auto k = std::make_pair(tensor, key);
  auto it = value_cache_.find(k);
  if (it != value_cache_.end() && it->second.version == version_[tensor]) return it->second.buf;
  const int np = (int)probs_.size();
  PerProb Y;
  if (it != value_cache_.end()) {
    Y = it->second.buf;
  } else {
    size_t bytes = 0;
    for (int p = 0; p < np; ++p) bytes += sizeof(double) * (size_t)ipow(probs_[p].n, (int)xi.size());
    if (cache_bytes_ + bytes > cache_budget_) {
      perm(dst, X, xi, scratch, yi, 1.0, 0.0, nullptr, tag);
      return scratch;
    }
    for (int p = 0; p < np; ++p) {
      double* q = cache_alloc_((size_t)ipow(probs_[p].n, (int)xi.size()));
      if (!q) {   // no room: uncached (buffers taken for earlier problems stay unused)
        perm(dst, X, xi, scratch, yi, 1.0, 0.0, nullptr, tag);
        return scratch;
      }
      cache_bytes_ += sizeof(double) * (size_t)ipow(probs_[p].n, (int)xi.size());
      Y.push_back(q);
    }
  }
  perm(dst, X, xi, Y, yi, 1.0, 0.0, nullptr, tag + "(cached)");
  value_cache_[k] = CacheEntry{Y, version_[tensor]};
  return Y;
}

// ------------------------------------------------------------------ lowering: contraction
void Executor::contract(std::vector<Launch>& dst, const PerProb& out, const std::string& oi, double alpha,
                        const PerProb& A, const std::string& ai, int a_const, const PerProb* B,
                        const std::string& bi, int b_const, bool acc, const std::string& tag, int a_val,
                        int b_val, int t_out, int t_a, int t_b) {
  const double beta = acc ? 1.0 : 0.0;
  const int np = (int)probs_.size();
  if (B && !oi.empty() && !ai.empty() && !bi.empty() && &dst != &setup_ &&
      contract_blocked(dst, out, oi, alpha, A, ai, *B, bi, acc, tag, t_out, t_a, t_b))
    return;
  if (!B) {
    for (char c : ai)
      if (!has(oi, c)) throw std::runtime_error("single-operand reduction unsupported: " + tag);
    if (elem_blocked(dst, A, ai, out, oi, alpha, beta, t_out, t_a, tag)) return;
    dense_guard(tag, {t_out, t_a});
    perm(dst, A, ai, out, oi, alpha, beta, nullptr, tag);
    return;
  }
  // scalar operand: scaled permute with a device scalar (over the allowed elements
  // when the laws are known)
  if (ai.empty() || bi.empty()) {
    const PerProb& S = ai.empty() ? A : *B;
    const PerProb& X = ai.empty() ? *B : A;
    const std::string& xi = ai.empty() ? bi : ai;
    std::vector<const double*> sc(S.begin(), S.end());
    const int t_x = ai.empty() ? t_b : t_a;
    if (&dst != &setup_ && !oi.empty() && elem_blocked(dst, X, xi, out, oi, alpha, beta, t_out, t_x, tag, &sc))
      return;
    dense_guard(tag, {t_out, t_a, t_b});
    perm(dst, X, xi, out, oi, alpha, beta, &sc, tag);
    return;
  }
  for (char c : ai)
    if (!has(bi, c) && !has(oi, c)) throw std::runtime_error("letter summed in one operand only: " + tag);
  for (char c : bi)
    if (!has(ai, c) && !has(oi, c)) throw std::runtime_error("letter summed in one operand only: " + tag);
  for (char c : oi)
    if (has(ai, c) && has(bi, c)) throw std::runtime_error("batch letters unsupported: " + tag);

  // full contraction -> dot
  if (oi.empty()) {
    if (&dst != &setup_ && dot_blocked(dst, A, ai, *B, bi, out, alpha, beta, t_a, t_b, tag)) return;
    dense_guard(tag, {t_a, t_b, t_out});
    PerProb Bp = *B;
    if (bi != ai) {
      if (b_const >= 0) Bp = const_permuted(b_const, *B, bi, ai);
      else Bp = value_permuted(dst, b_val, *B, bi, ai, scratch_->b, tag + ":permB");
    }
    std::vector<DotProblem> ds(np);
    for (int p = 0; p < np; ++p) {
      ds[p].X = A[p];
      ds[p].Y = Bp[p];
      ds[p].out = out[p];
      ds[p].len = ipow(probs_[p].n, (int)ai.size());
      ds[p].alpha = alpha;
      ds[p].beta = beta;
      ds[p].active = gate_for(dst, p);
    }
    Launch L;
    for (int p = 0; p < np; ++p) {
      add_range(L.rd, ds[p].X, sizeof(double) * (size_t)ds[p].len);
      add_range(L.rd, ds[p].Y, sizeof(double) * (size_t)ds[p].len);
      add_range(L.wr, ds[p].out, sizeof(double));
      L.bytes += 2.0 * sizeof(double) * (double)ds[p].len;
    }
    L.ranged = true;
    L.kind = Launch::DOT;
    L.n_prob = np;
    L.dot_blocks = 64;
    L.d_desc = upload(ds.data(), sizeof(DotProblem) * np);
    L.d_partial = scratch_->dot_partial;
    L.tag = tag;
    dst.push_back(L);
    return;
  }

  dense_guard(tag, {t_out, t_a, t_b});
  const std::string M_a = filter(ai, bi, oi, false, true);   // in A and out only
  const std::string K_a = filter(ai, bi, oi, true, false);   // in A and B only
  const std::string N_b = filter(bi, ai, oi, false, true);
  const std::string K_b = filter(bi, ai, oi, true, false);
  const std::string M_o = filter(oi, ai, bi, true, false);
  const std::string N_o = filter(oi, bi, ai, true, false);

  struct Choice {
    std::string M, N, K;
    bool swap;
    double cost;
  };
  Choice best{"", "", "", false, 1e300};
  const long n0 = probs_[0].n;
  auto sz = [&](const std::string& s) { return (double)ipow(n0, (int)s.size()); };
  for (int im = 0; im < 2; ++im)
    for (int in = 0; in < 2; ++in)
      for (int ik = 0; ik < 2; ++ik) {
        std::string M = im ? M_o : M_a, N = in ? N_o : N_b, K = ik ? K_b : K_a;
        double cost = 0.0;
        const bool a_ok = (ai == M + K) || (ai == K + M);
        const bool b_ok = (bi == K + N) || (bi == N + K);
        if (!a_ok && a_const < 0) cost += sz(ai);
        if (!b_ok && b_const < 0) cost += sz(bi);
        bool swap = false;
        if (oi == M + N) {
        } else if (oi == N + M) {
          swap = true;
        } else if (!N.empty() && N.back() == oi.back()) {
          cost += 0.1 * sz(oi);   // written through output offset tables, columns contiguous
        } else if (!M.empty() && M.back() == oi.back()) {
          swap = true;            // the same with C transposed
          cost += 0.1 * sz(oi);
        } else {
          cost += 2.0 * sz(oi);   // GEMM layout, then a permute pass
        }
        if (cost < best.cost) best = {M, N, K, swap, cost};
      }

  // operands in GEMM layout
  auto place = [&](const PerProb& X, const std::string& xi, int xconst, int xval, const std::string& first,
                   const std::string& second, PerProb& scratch, bool& trans, std::string& lay) -> PerProb {
    if (xi == first + second) {
      trans = false;
      lay = xi;
      return X;
    }
    if (xi == second + first) {
      trans = true;
      lay = xi;
      return X;
    }
    trans = false;
    lay = first + second;
    if (xconst >= 0) return const_permuted(xconst, X, xi, lay);
    return value_permuted(dst, xval, X, xi, lay, scratch, tag + ":perm");
  };
  // C[M][N] = A[M][K] B[K][N]; with swap, C^T[N][M] = B^T[N][K] A^T[K][M]
  std::string M = best.M, N = best.N, K = best.K;
  PerProb Ap, Bp;
  bool ta = false, tb = false;
  std::string alay, blay;
  if (!best.swap) {
    Ap = place(A, ai, a_const, a_val, M, K, scratch_->a, ta, alay);     // ta: stored [K][M]
    Bp = place(*B, bi, b_const, b_val, K, N, scratch_->b, tb, blay);    // tb: stored [N][K]
  } else {
    // rows of C = N letters (from B), cols = M letters (from A)
    Ap = place(*B, bi, b_const, b_val, N, K, scratch_->b, ta, alay);
    Bp = place(A, ai, a_const, a_val, K, M, scratch_->a, tb, blay);
    std::swap(M, N);
  }
  const bool c_direct = (oi == M + N);
  // Output in neither [M][N] nor [N][M] but with its fastest letter the GEMM's
  // fastest column letter: the GEMM writes it through row and column offset
  // tables (coalesced along that letter) instead of C plus a permute pass; not
  // when the output aliases an operand, which the GEMM would overwrite while
  // other tiles still read it.
  bool c_table = !c_direct && !N.empty() && N.back() == oi.back();
  for (int p = 0; p < np && c_table; ++p) {
    if (out[p] == A[p] || out[p] == (*B)[p] || out[p] == Ap[p] || out[p] == Bp[p]) c_table = false;
    if (ipow(probs_[p].n, (int)oi.size()) >= (1L << 32)) c_table = false;
  }
  const double galpha = alpha;
  const double gbeta = (c_direct || c_table) ? beta : 0.0;
  const PerProb& Cp = (c_direct || c_table) ? out : scratch_->c;

  int cfg = 0;
  {
    const long m = ipow(n0, (int)M.size()), nn = ipow(n0, (int)N.size()), kk = ipow(n0, (int)K.size());
    cfg = (m >= 128 && nn >= 128) ? (kk >= 512 ? 2 : 0) : 1;
  }
  // descriptors of the grouped launch for one tile configuration; allow_split:
  // split K when the launch would not fill the device
  auto build_gemm = [&](int gcfg, bool allow_split) {
    std::vector<GemmProblem> gs(np);
    std::vector<int> prefix(np), prefix2(np);
    const int BM = gemm_bm(gcfg), BN = gemm_bn(gcfg);
    int total = 0, total2 = 0;
    bool any_split = false;
    double flops = 0.0;
    long tiles_all = 0;
    for (int p = 0; p < np; ++p) {
      const long n = probs_[p].n;
      tiles_all += ((ipow(n, (int)M.size()) + BM - 1) / BM) * ((ipow(n, (int)N.size()) + BN - 1) / BN);
    }
    for (int p = 0; p < np; ++p) {
      const long n = probs_[p].n;
      GemmProblem& g = gs[p];
      g.M = (int)ipow(n, (int)M.size());
      g.N = (int)ipow(n, (int)N.size());
      g.K = (int)ipow(n, (int)K.size());
      g.A = Ap[p];
      g.B = Bp[p];
      g.C = Cp[p];
      g.lda = ta ? g.M : g.K;
      g.ldb = tb ? g.K : g.N;
      g.ldc = g.N;
      g.alpha = galpha;
      g.beta = gbeta;
      g.active = gate_for(dst, p);
      g.tiles_m = (g.M + BM - 1) / BM;
      g.tiles_n = (g.N + BN - 1) / BN;
      if (c_table) {
        g.offM = out_offsets(n, M, oi);
        g.offN = out_offsets(n, N, oi);
      }
      int ks = 1;
      if (allow_split && tiles_all < 512 && g.K >= 512) {
        ks = (int)std::min<long>((512 + tiles_all - 1) / tiles_all, g.K / 256);
        // the partial buffer holds n^4 doubles
        while (ks > 1 && (long)ks * g.M * g.N > ipow(n, 4)) --ks;
        ks = std::max(ks, 1);
      }
      if ((long)g.M * g.K >= (1L << 31) || (long)g.K * g.N >= (1L << 31) || (long)g.M * g.N >= (1L << 31))
        throw std::runtime_error("GEMM operand exceeds 2^31 elements: " + tag);
      g.ksplit = ks;
      g.kchunk = (g.K + ks - 1) / ks;
      g.kchunk = ((g.kchunk + 15) / 16) * 16;
      g.ksplit = (g.K + g.kchunk - 1) / g.kchunk;
      g.partial = scratch_->part[p];
      if (g.ksplit > 1) any_split = true;
      prefix[p] = total;
      total += g.tiles_m * g.tiles_n * g.ksplit;
      prefix2[p] = total2;
      total2 += (int)(((long)g.M * g.N + 1023) / 1024);
      flops += 2.0 * g.M * (double)g.N * g.K;
    }
    std::vector<double> pf(np);
    std::vector<int> pinst(np);
    Launch L;
    for (int p = 0; p < np; ++p) {
      pf[p] = 2.0 * gs[p].M * (double)gs[p].N * gs[p].K;
      pinst[p] = probs_[p].inst;
      L.bytes += sizeof(double) * ((double)gs[p].M * gs[p].K + (double)gs[p].K * gs[p].N +
                                   (double)gs[p].M * gs[p].N * (beta != 0.0 ? 2 : 1));
    }
    L.kind = Launch::GEMM;
    L.n_prob = np;
    L.total = total;
    L.min_k = np > 0 ? gs[0].K : 0;
    for (int p = 1; p < np; ++p) L.min_k = std::min(L.min_k, gs[p].K);
    if (&dst != &setup_) {
      L.prob_flops = pf;
      L.prob_inst = pinst;
    }
    L.cfg = gcfg;
    L.ta = ta;
    L.tb = tb;
    L.d_desc = upload(gs.data(), sizeof(GemmProblem) * np);
    L.d_prefix = (int*)upload(prefix.data(), sizeof(int) * np);
    if (any_split) {
      // problems without a split still need their own reduce pass skipped: mark via ksplit
      L.splitk_blocks = total2;
      L.d_prefix2 = (int*)upload(prefix2.data(), sizeof(int) * np);
    }
    L.flops = flops;
    L.tag = tag;
    return L;
  };
  Launch L = build_gemm(cfg, true);
  if (&dst != &setup_) {
    // candidates for the autotuner: 64 x 64 tiles while the 128 x 128 launch is
    // short of four waves of resident blocks (beyond that its edge waste is small
    // and the larger tile wins), and the launch without split-K
    if (gemm_bm(cfg) == 128 && L.total < 4 * gemm_slots(cfg)) L.alts.push_back(build_gemm(1, true));
    if (L.splitk_blocks > 0) L.alts.push_back(build_gemm(cfg, false));
  }
  dst.push_back(L);
  if (!c_direct && !c_table) perm(dst, scratch_->c, M + N, out, oi, 1.0, beta, nullptr, tag + ":permC");
}


// ------------------------------------------------------------------ momentum blocking
// Laws of the intermediates from the ops, in program order: a unary op copies
// its operand's signs; for out = A * B the contracted letters fix the relative
// orientation s of B's law (sign_A * sign_B, the same for every contracted
// letter), and out gets sign_A on A's free letters and -s * sign_B on B's.
// Every op writing a tensor must give the same law up to an overall sign.
bool packing_enabled() {
  const char* e = std::getenv("FTCC_PACK");
  return !(e && e[0] == '0');
}

bool labels_distinct(const InstMomentum& M) {
  const int D = M.dims;
  if (D <= 0) return false;
  const int n = (int)(M.labels.size() / D);
  std::vector<std::vector<int>> keys(n, std::vector<int>(D));
  for (int p = 0; p < n; ++p)
    for (int c = 0; c < D; ++c) {
      int v = M.labels[(size_t)p * D + c];
      if (M.modulus[c] > 0) v = ((v % M.modulus[c]) + M.modulus[c]) % M.modulus[c];
      keys[p][c] = v;
    }
  std::sort(keys.begin(), keys.end());
  return std::adjacent_find(keys.begin(), keys.end()) == keys.end();
}

void Executor::dense_guard(const std::string& tag, std::initializer_list<int> ts) const {
  for (int t : ts)
    if (is_packed(t)) throw std::runtime_error("packed intermediate on a dense path: " + tag);
}

int Executor::n_packed() const {
  int k = 0;
  for (char v : packed_) k += v ? 1 : 0;
  return k;
}

// Which intermediates are stored packed: rank >= 2, a known momentum law, every
// instance's labels distinct, and every op that touches the tensor (forward, and
// its reverse forms when the backward list is built) has known laws on all of
// its tensors, so that it lowers to blocked kernels, which address elements
// through offset tables only.  Derived constants keep dense storage (their set-up
// ops are dense permutes).
void Executor::plan_packing(bool want_backward) {
  const int nt = (int)prog_->t.size();
  packed_.assign(nt, 0);
  pack_on_ = false;
  if (mom_.empty() || !packing_enabled()) return;
  for (const ProblemRef& p : probs_)
    if (p.inst < 0 || p.inst >= (int)mom_.size() || !mom_[p.inst] || !labels_distinct(*mom_[p.inst])) return;
  pack_on_ = true;
  for (int k = 0; k < nt; ++k) {
    const TensorDecl& d = prog_->t[k];
    packed_[k] = (d.kind == T_INTER && !d.derived && d.rank >= 2 && law_ok_[k]) ? 1 : 0;
  }
  (void)want_backward;   // the reverse forms of an op lower blocked exactly when the forward does
  for (const SymOp& o : prog_->ops) {
    if (o.setup && !inline_setup_) continue;
    const bool ok = law_ok_[o.out] && law_ok_[o.a] && (o.b < 0 || law_ok_[o.b]);
    if (ok) continue;
    packed_[o.out] = 0;
    packed_[o.a] = 0;
    if (o.b >= 0) packed_[o.b] = 0;
  }
}

std::vector<int> Executor::plan_const_packing(const std::vector<int>& const_grads) const {
  std::vector<int> out;
  if (!pack_on_ || inline_setup_) return out;
  const int nt = (int)prog_->t.size();
  for (int k = 0; k < nt; ++k) {
    const TensorDecl& d = prog_->t[k];
    if (!(d.kind == T_CONST || d.derived) || d.rank < 2 || !law_ok_[k]) continue;
    if (std::find(const_grads.begin(), const_grads.end(), k) != const_grads.end()) continue;
    bool ok = true, used = false;
    for (const SymOp& o : prog_->ops) {
      if (o.setup) continue;
      if (o.out != k && o.a != k && o.b != k) continue;
      used = true;
      if (!(law_ok_[o.out] && law_ok_[o.a] && (o.b < 0 || law_ok_[o.b]))) ok = false;
    }
    if (ok && used) out.push_back(k);
  }
  return out;
}

std::vector<int> Executor::plan_io_packing() const {
  std::vector<int> out;
  if (!pack_on_ || inline_setup_) return out;
  const int nt = (int)prog_->t.size();
  for (int k = 0; k < nt; ++k) {
    const TensorDecl& d = prog_->t[k];
    if (!(d.kind == T_INPUT || d.kind == T_OUTPUT) || d.rank < 2 || !law_ok_[k]) continue;
    bool ok = true;
    for (const SymOp& o : prog_->ops) {
      if (o.setup || (o.out != k && o.a != k && o.b != k)) continue;
      if (!(law_ok_[o.out] && law_ok_[o.a] && (o.b < 0 || law_ok_[o.b]))) ok = false;
    }
    if (ok) out.push_back(k);
  }
  return out;
}

void Executor::infer_laws() {
  const int nt = (int)prog_->t.size();
  law_.assign(nt, {});
  law_ok_.assign(nt, 0);
  std::vector<char> bad(nt, 0), known(nt, 0);
  for (int k = 0; k < nt; ++k)
    if ((k < (int)prog_->law.size() && !prog_->law[k].empty()) || prog_->t[k].rank == 0) {
      if (k < (int)prog_->law.size()) law_[k] = prog_->law[k];
      known[k] = 1;
    }
  for (const SymOp& o : prog_->ops) {
    bool ok = known[o.a] && !bad[o.a] && (o.b < 0 || (known[o.b] && !bad[o.b]));
    std::vector<int> lc;
    if (ok) {
      auto sg = [&](int t, const std::string& idx, char c) { return law_[t][idx.find(c)]; };
      int s = -1;
      bool first = true;
      if (o.b >= 0)
        for (char c : o.ai)
          if (has(o.bi, c)) {
            const int r = sg(o.a, o.ai, c) * sg(o.b, o.bi, c);
            if (first) {
              s = r;
              first = false;
            } else if (r != s) {
              ok = false;
            }
          }
      if (ok)
        for (char c : o.oi) lc.push_back(has(o.ai, c) ? sg(o.a, o.ai, c) : -s * sg(o.b, o.bi, c));
    }
    const int k = o.out;
    if (!ok) {
      bad[k] = 1;
    } else if (!known[k]) {
      law_[k] = lc;
      known[k] = 1;
    } else {
      std::vector<int> neg(lc);
      for (int& v : neg) v = -v;
      if (law_[k] != lc && law_[k] != neg) bad[k] = 1;
    }
  }
  for (int k = 0; k < nt; ++k) law_ok_[k] = known[k] && !bad[k];
}

static long long pack_momentum(const std::vector<int>& q) {
  long long key = 0;
  for (size_t c = 0; c < q.size(); ++c) key |= (long long)(q[c] + (1 << 19)) << (21 * c);
  return key;
}

// Tuples of `letters` (each 0..n-1) in momentum-block order, with their element
// offsets in the operands indexed by xi and yi (row-major, every axis n) and
// the packed momentum sum_l signs[l] k(index_l) of each block.
const Executor::GroupTable& Executor::group_table(int inst, long n, const std::string& letters,
                                                  const std::string& xi, bool xp, const std::string& yi,
                                                  bool yp, const std::vector<int>& signs) {
  std::string key = std::to_string(inst) + "|" + letters + "|" + xi + (xp ? "#" : "") + "|" + yi +
                    (yp ? "#" : "") + "|";
  for (int v : signs) key += (v > 0 ? '+' : '-');
  auto it = group_cache_.find(key);
  if (it != group_cache_.end()) return it->second;
  const InstMomentum& M = *mom_[inst];
  const int g = (int)letters.size(), D = M.dims;
  // row-major strides; a packed tensor drops its last axis (stride 0: that index
  // is fixed by the others on every allowed element)
  auto stride = [&](const std::string& idx, bool packed, char c) -> unsigned long {
    const int pos = (int)idx.find(c), len = (int)idx.size();
    if (!packed) return (unsigned long)ipow(n, len - 1 - pos);
    return pos == len - 1 ? 0ul : (unsigned long)ipow(n, len - 2 - pos);
  };
  std::vector<unsigned long> sx(g), sy(g);
  for (int l = 0; l < g; ++l) {
    sx[l] = stride(xi, xp, letters[l]);
    sy[l] = stride(yi, yp, letters[l]);
  }
  const long count = ipow(n, g);
  struct Row {
    long long key;
    unsigned ox, oy;
  };
  std::vector<Row> rows(count);
  std::vector<int> idx(g, 0), q(D);
  for (long t = 0; t < count; ++t) {
    unsigned long ox = 0, oy = 0;
    std::fill(q.begin(), q.end(), 0);
    for (int l = 0; l < g; ++l) {
      ox += idx[l] * sx[l];
      oy += idx[l] * sy[l];
      for (int c = 0; c < D; ++c) q[c] += signs[l] * M.labels[(size_t)idx[l] * D + c];
    }
    for (int c = 0; c < D; ++c)
      if (M.modulus[c] > 0) q[c] = ((q[c] % M.modulus[c]) + M.modulus[c]) % M.modulus[c];
    rows[t] = Row{pack_momentum(q), (unsigned)ox, (unsigned)oy};
    for (int l = g - 1; l >= 0; --l) {   // next tuple, last letter fastest
      if (++idx[l] < n) break;
      idx[l] = 0;
    }
  }
  std::stable_sort(rows.begin(), rows.end(), [](const Row& a, const Row& b) { return a.key < b.key; });
  GroupTable T;
  std::vector<unsigned> o1(count), o2(count);
  for (long t = 0; t < count; ++t) {
    o1[t] = rows[t].ox;
    o2[t] = rows[t].oy;
    auto b = T.blocks.find(rows[t].key);
    if (b == T.blocks.end()) T.blocks[rows[t].key] = std::make_pair((int)t, 1);
    else b->second.second++;
  }
  T.off1 = upload(o1.data(), sizeof(unsigned) * count);
  T.off2 = upload(o2.data(), sizeof(unsigned) * count);
  return group_cache_.emplace(key, std::move(T)).first->second;
}

// Tile shape of one block of a blocked contraction (ml rows, nl columns, kl inner):
// 0 (16 x 16 MFMA tiles) or a lane-mapped shape code, whichever needs fewer wave
// latencies by a simple count: a wave costs 3 dependent memory latencies (task,
// offsets, the store) plus 2 per step of its inner loop; an MFMA step covers 32
// inner indices, a lane-mapped step 8 per lane of the inner slices (at most
// `cap` steps: longer ranges go to MFMA tiles split over several waves).  With
// the operands in cache (packed storage) long lane-mapped chains pay: 1.31 s per
// 123-PW step with a cap of 16 steps against 1.44 s with 2 and 1.79 s without
// lane-mapped tiles; with every operand scattered over dense arrays a cap of 2
// had been the best.
static int sgemm_shape(int ml, int nl, int kl, long cap) {
  auto cdiv = [](long a, long b) { return (a + b - 1) / b; };
  auto steps = [&](long per) { return std::max(1L, cdiv(kl, per)); };
  const long mfma = cdiv(ml, 16) * cdiv(nl, 16) * (3 + 2 * steps(32));
  long best = mfma;
  int shape = 0;
  for (int lr = 0; lr <= 6; ++lr)
    for (int lc = 0; lr + lc <= 6; ++lc) {
      const int ls = 6 - lr - lc;
      if (steps(8L << ls) > cap) continue;   // longer ranges: MFMA tiles split over several waves
      const long c = cdiv(ml, 1L << lr) * cdiv(nl, 1L << lc) * (3 + 2 * steps(8L << ls));
      if (c < best) {
        best = c;
        shape = sgemm_thin_shape(lr, lc, ls);
      }
    }
  return shape;
}

constexpr long kSgemmThinSteps = 16;

// wave latencies of a task by the same count (the order of a merged task list)
static long sgemm_task_cost(const SgemmTask& t) {
  const long per = t.shape ? (8L << ((t.shape >> 6) & 7)) : 32L;
  return 3 + 2 * std::max(1L, (t.klen + per - 1) / per);
}

// C[oi] (+)= alpha A[ai] B[bi] over the momentum-allowed blocks: rows M (letters
// of A and C), inner K (A and B), columns N (B and C).  A row tuple of momentum
// q pairs with inner tuples of A-momentum -q and column tuples of B-momentum s q.
// Returns false (dense lowering) when a law is unknown.
bool Executor::contract_blocked(std::vector<Launch>& dst, const PerProb& out, const std::string& oi, double alpha,
                                const PerProb& A, const std::string& ai, const PerProb& B, const std::string& bi,
                                bool acc, const std::string& tag, int t_out, int t_a, int t_b) {
  if (mom_.empty() || t_out < 0 || t_a < 0 || t_b < 0) return false;
  if (!law_ok_[t_out] || !law_ok_[t_a] || !law_ok_[t_b]) return false;
  const std::vector<int>&la = law_[t_a], &lb = law_[t_b];
  auto sa = [&](char c) { return la[ai.find(c)]; };
  auto sb = [&](char c) { return lb[bi.find(c)]; };
  const std::string M = filter(ai, bi, oi, false, true);   // A and C
  const std::string K = filter(ai, bi, oi, true, false);   // A and B
  const std::string N = filter(bi, ai, oi, false, true);   // B and C
  int s = -1;
  bool first = true;
  for (char c : K) {
    const int r = sa(c) * sb(c);
    if (first) {
      s = r;
      first = false;
    } else if (r != s) {
      return false;
    }
  }
  std::vector<int> sgM, sgK, sgN;
  for (char c : M) sgM.push_back(sa(c));
  for (char c : K) sgK.push_back(sa(c));
  for (char c : N) sgN.push_back(sb(c));
  const int np = (int)probs_.size();
  std::vector<SgemmProblem> ps(np);
  std::vector<SgemmTask> tasks;
  struct Tile {
    int p, m0, ml, k0, kl, n0, nl, shape;
  };
  std::vector<Tile> tiles;
  // FTCC_SGEMM_THIN=0: 16 x 16 MFMA tiles for every block; =N: at most N inner
  // steps per lane-mapped wave (diagnostics)
  double bytes = 0.0;
  const char* thin_env = std::getenv("FTCC_SGEMM_THIN");
  const long thin_cap = thin_env ? std::atol(thin_env) : kSgemmThinSteps;
  const bool thin_ok = thin_cap > 0;
  std::vector<double> pf(np, 0.0);
  std::vector<int> pinst(np);
  double flops = 0.0;
  for (int p = 0; p < np; ++p) {
    const int inst = probs_[p].inst;
    const long n = probs_[p].n;
    if (inst < 0 || inst >= (int)mom_.size() || !mom_[inst]) throw std::runtime_error("momentum labels missing");
    if (ipow(n, (int)std::max(std::max(ai.size(), bi.size()), oi.size())) >= (1L << 32))
      throw std::runtime_error("tensor exceeds 2^32 elements: " + tag);
    const GroupTable& TM = group_table(inst, n, M, ai, is_packed(t_a), oi, is_packed(t_out), sgM);
    const GroupTable& TK = group_table(inst, n, K, ai, is_packed(t_a), bi, is_packed(t_b), sgK);
    const GroupTable& TN = group_table(inst, n, N, bi, is_packed(t_b), oi, is_packed(t_out), sgN);
    SgemmProblem& P = ps[p];
    P.A = A[p];
    P.B = B[p];
    P.C = out[p];
    P.offAM = (const unsigned*)TM.off1;
    P.offCM = (const unsigned*)TM.off2;
    P.offAK = (const unsigned*)TK.off1;
    P.offBK = (const unsigned*)TK.off2;
    P.offBN = (const unsigned*)TN.off1;
    P.offCN = (const unsigned*)TN.off2;
    P.alpha = alpha;
    P.beta = acc ? 1.0 : 0.0;
    P.active = gate_for(dst, p);
    pinst[p] = inst;
    const InstMomentum& Mm = *mom_[inst];
    for (const auto& blk : TM.blocks) {
      std::vector<int> q(Mm.dims), qk(Mm.dims), qn(Mm.dims);
      for (int c = 0; c < Mm.dims; ++c) {
        q[c] = (int)((blk.first >> (21 * c)) & ((1 << 21) - 1)) - (1 << 19);
        qk[c] = -q[c];
        qn[c] = s * q[c];
        if (Mm.modulus[c] > 0) {
          qk[c] = ((qk[c] % Mm.modulus[c]) + Mm.modulus[c]) % Mm.modulus[c];
          qn[c] = ((qn[c] % Mm.modulus[c]) + Mm.modulus[c]) % Mm.modulus[c];
        }
      }
      auto nb = TN.blocks.find(pack_momentum(qn));
      if (nb == TN.blocks.end()) continue;
      auto kb = TK.blocks.find(pack_momentum(qk));
      const int k0 = kb == TK.blocks.end() ? 0 : kb->second.first;
      const int kl = kb == TK.blocks.end() ? 0 : kb->second.second;
      if (kl == 0 && acc) continue;   // nothing to add; a set writes its zeros
      const int m0 = blk.second.first, ml = blk.second.second;
      const int n0 = nb->second.first, nl = nb->second.second;
      const int shape = thin_ok ? sgemm_shape(ml, nl, kl, thin_cap) : 0;
      const int R = shape ? 1 << (shape & 7) : 16, C = shape ? 1 << ((shape >> 3) & 7) : 16;
      for (int r = 0; r < ml; r += R)
        for (int c = 0; c < nl; c += C)
          tiles.push_back(Tile{p, m0 + r, std::min(R, ml - r), k0, kl, n0 + c, std::min(C, nl - c), shape});
      pf[p] += 2.0 * ml * (double)nl * kl;
      bytes += sizeof(double) * ((double)ml * kl + (double)kl * nl + (double)ml * nl * (acc ? 2 : 1));
    }
    flops += pf[p];
  }
  // A tile with a long inner range would be one wave's long serial chain of
  // dependent gathers: its range is cut into chunks whose partial tiles a
  // second kernel adds in order.  The chunk grows (powers of two) until every
  // partial tile fits the workspace.
  const long ws_tiles = scratch_ && scratch_->tail_ws ? (long)(scratch_->tail_ws_doubles / 256) : 0;
  int chunk = kSgemmChunk;
  auto parts_needed = [&](int ch) {
    long n = 0;
    for (const Tile& t : tiles)
      if (!t.shape && t.kl > ch + ch / 2) n += (t.kl + ch - 1) / ch;
    return n;
  };
  while (ws_tiles > 0 && parts_needed(chunk) > ws_tiles) chunk *= 2;
  std::vector<SgemmReduce> reds;
  int parts = 0;
  for (const Tile& t : tiles) {
    if (t.shape || ws_tiles == 0 || t.kl <= chunk + chunk / 2) {
      tasks.push_back(SgemmTask{t.p, t.m0, t.ml, t.k0, t.kl, t.n0, t.nl, -1, t.shape});
      continue;
    }
    const int first = parts;
    for (int k = 0; k < t.kl; k += chunk)
      tasks.push_back(SgemmTask{t.p, t.m0, t.ml, t.k0 + k, std::min(chunk, t.kl - k), t.n0, t.nl, parts++, 0});
    reds.push_back(SgemmReduce{t.p, t.m0, t.ml, t.n0, t.nl, first, parts - first});
  }
  Launch L;
  for (int p = 0; p < np; ++p) {
    const long n = probs_[p].n;
    add_range(L.rd, A[p], sizeof(double) * elems(t_a, n, (int)ai.size()));
    add_range(L.rd, B[p], sizeof(double) * elems(t_b, n, (int)bi.size()));
    add_range(L.wr, out[p], sizeof(double) * elems(t_out, n, (int)oi.size()));
  }
  L.ranged = true;
  L.bytes = bytes;
  if (&dst != &setup_) {
    L.sprobs = ps;
    L.stasks = tasks;
    L.sreds = reds;
  }
  L.kind = Launch::SGEMM;
  L.n_prob = np;
  L.d_desc = upload(ps.data(), sizeof(SgemmProblem) * np);
  L.n_tasks = (int)tasks.size();
  L.d_tasks = upload(tasks.data(), sizeof(SgemmTask) * std::max<size_t>(tasks.size(), 1));
  L.n_red = (int)reds.size();
  if (L.n_red > 0) {
    L.d_red = upload(reds.data(), sizeof(SgemmReduce) * reds.size());
    L.d_partial = scratch_->tail_ws;
  }
  L.total = (L.n_tasks + 3) / 4;
  L.flops = flops;
  if (&dst != &setup_) {
    L.prob_flops = pf;
    L.prob_inst = pinst;
  }
  L.tag = tag + "(blocked)";
  dst.push_back(L);
  return true;
}

// Y[yi] = alpha X[xi] + beta Y over the allowed elements of Y (its law known):
// Y's letters split into two halves whose momentum blocks q and -q pair up.
// Returns false (dense lowering) when a law is unknown.
bool Executor::elem_blocked(std::vector<Launch>& dst, const PerProb& X, const std::string& xi, const PerProb& Y,
                            const std::string& yi, double alpha, double beta, int t_y, int t_x,
                            const std::string& tag, const std::vector<const double*>* scale, int xp, int yp) {
  const bool xpk = xp >= 0 ? xp != 0 : is_packed(t_x), ypk = yp >= 0 ? yp != 0 : is_packed(t_y);
  if (mom_.empty() || t_y < 0 || t_x < 0 || !law_ok_[t_y] || !law_ok_[t_x] || yi.empty()) return false;
  const std::vector<int>& ly = law_[t_y];
  const std::vector<int>& lx = law_[t_x];
  // the operand's law must describe the same allowed set (equal or opposite signs)
  int rel = 0;
  for (size_t a = 0; a < yi.size(); ++a) {
    const int r = ly[a] * lx[xi.find(yi[a])];
    if (rel == 0) rel = r;
    else if (r != rel) return false;
  }
  const std::string G1 = yi.substr(0, yi.size() / 2), G2 = yi.substr(yi.size() / 2);
  std::vector<int> s1, s2;
  for (size_t a = 0; a < G1.size(); ++a) s1.push_back(ly[a]);
  for (size_t a = 0; a < G2.size(); ++a) s2.push_back(ly[G1.size() + a]);
  const int np = (int)probs_.size();
  std::vector<ElemProblem> ps(np);
  std::vector<ElemTask> tasks;
  long long total = 0;
  for (int p = 0; p < np; ++p) {
    const int inst = probs_[p].inst;
    const long n = probs_[p].n;
    if (ipow(n, (int)yi.size()) >= (1L << 32)) throw std::runtime_error("tensor exceeds 2^32 elements: " + tag);
    const GroupTable& T1 = group_table(inst, n, G1, xi, xpk, yi, ypk, s1);
    const GroupTable& T2 = group_table(inst, n, G2, xi, xpk, yi, ypk, s2);
    ElemProblem& P = ps[p];
    P.X = X[p];
    P.Y = Y[p];
    P.ox1 = (const unsigned*)T1.off1;
    P.oy1 = (const unsigned*)T1.off2;
    P.ox2 = (const unsigned*)T2.off1;
    P.oy2 = (const unsigned*)T2.off2;
    P.alpha = alpha;
    P.beta = beta;
    P.active = gate_for(dst, p);
    P.scale = scale ? (*scale)[p] : nullptr;
    const InstMomentum& Mm = *mom_[inst];
    for (const auto& blk : T1.blocks) {
      std::vector<int> q(Mm.dims);
      for (int c = 0; c < Mm.dims; ++c) {
        q[c] = -((int)((blk.first >> (21 * c)) & ((1 << 21) - 1)) - (1 << 19));
        if (Mm.modulus[c] > 0) q[c] = ((q[c] % Mm.modulus[c]) + Mm.modulus[c]) % Mm.modulus[c];
      }
      auto b2 = T2.blocks.find(pack_momentum(q));
      if (b2 == T2.blocks.end()) continue;
      tasks.push_back(ElemTask{total, p, blk.second.first, blk.second.second, b2->second.first, b2->second.second});
      total += (long long)blk.second.second * b2->second.second;
    }
  }
  Launch L;
  for (int p = 0; p < np; ++p) {
    const long n = probs_[p].n;
    if (alpha != 0.0 && scale) add_range(L.rd, (*scale)[p], sizeof(double));
    const size_t ex = (size_t)ipow_l(n, (int)xi.size() - (xpk ? 1 : 0));
    const size_t ey = (size_t)ipow_l(n, (int)yi.size() - (ypk ? 1 : 0));
    if (alpha != 0.0) add_range(L.rd, X[p], sizeof(double) * ex);
    if (beta != 0.0) add_range(L.rd, Y[p], sizeof(double) * ey);
    add_range(L.wr, Y[p], sizeof(double) * ey);
  }
  L.ranged = true;
  L.kind = Launch::ELEM;
  L.n_prob = np;
  L.d_desc = upload(ps.data(), sizeof(ElemProblem) * np);
  L.n_tasks = (int)tasks.size();
  L.d_tasks = upload(tasks.data(), sizeof(ElemTask) * std::max<size_t>(tasks.size(), 1));
  {
    const std::vector<int> bf = block_first_tasks(tasks, total);
    L.d_bfirst = upload(bf.data(), sizeof(int) * bf.size());
  }
  L.n_elem = total;
  L.bytes = sizeof(double) * (double)total * ((alpha != 0.0) + (beta != 0.0) + 1);
  L.zero_fill = alpha == 0.0 && beta == 0.0;
  if (&dst != &setup_) {
    L.eprobs = ps;
    L.etasks = tasks;
  }
  L.total = (int)std::min<long long>((total + 255) / 256, 1 << 30);
  L.tag = tag + "(blocked)";
  dst.push_back(L);
  return true;
}

bool Executor::dot_blocked(std::vector<Launch>& dst, const PerProb& A, const std::string& ai, const PerProb& B,
                           const std::string& bi, const PerProb& out, double alpha, double beta, int t_a, int t_b,
                           const std::string& tag) {
  if (mom_.empty() || t_a < 0 || !law_ok_[t_a] || ai.empty() || !scratch_ || !scratch_->tail_ws) return false;
  const std::vector<int>& la = law_[t_a];
  const std::string G1 = ai.substr(0, ai.size() / 2), G2 = ai.substr(ai.size() / 2);
  const std::vector<int> s1(la.begin(), la.begin() + G1.size()), s2(la.begin() + G1.size(), la.end());
  const int np = (int)probs_.size();
  std::vector<DotbProblem> ps(np);
  std::vector<ElemTask> tasks;
  long long total = 0;
  for (int p = 0; p < np; ++p) {
    const int inst = probs_[p].inst;
    const long n = probs_[p].n;
    if (ipow(n, (int)ai.size()) >= (1L << 32)) throw std::runtime_error("tensor exceeds 2^32 elements: " + tag);
    // A's allowed elements: index groups G1 of momentum q with G2 of momentum -q
    const GroupTable& T1 = group_table(inst, n, G1, ai, is_packed(t_a), bi, is_packed(t_b), s1);
    const GroupTable& T2 = group_table(inst, n, G2, ai, is_packed(t_a), bi, is_packed(t_b), s2);
    DotbProblem& P = ps[p];
    P.X = A[p];
    P.Y = B[p];
    P.ox1 = (const unsigned*)T1.off1;
    P.oy1 = (const unsigned*)T1.off2;
    P.ox2 = (const unsigned*)T2.off1;
    P.oy2 = (const unsigned*)T2.off2;
    P.out = out[p];
    P.alpha = alpha;
    P.beta = beta;
    P.active = gate_for(dst, p);
    total = (total + 255) / 256 * 256;     // every problem starts on a block boundary
    const long long start = total;
    const InstMomentum& Mm = *mom_[inst];
    for (const auto& blk : T1.blocks) {
      std::vector<int> q(Mm.dims);
      for (int c = 0; c < Mm.dims; ++c) {
        q[c] = -((int)((blk.first >> (21 * c)) & ((1 << 21) - 1)) - (1 << 19));
        if (Mm.modulus[c] > 0) q[c] = ((q[c] % Mm.modulus[c]) + Mm.modulus[c]) % Mm.modulus[c];
      }
      auto b2 = T2.blocks.find(pack_momentum(q));
      if (b2 == T2.blocks.end()) continue;
      tasks.push_back(ElemTask{total, p, blk.second.first, blk.second.second, b2->second.first, b2->second.second});
      total += (long long)blk.second.second * b2->second.second;
    }
    P.first_block = (int)(start / 256);
    P.n_blocks = (int)((total - start + 255) / 256);
  }
  if ((total + 255) / 256 > (long long)scratch_->tail_ws_doubles) return false;
  Launch L;
  for (int p = 0; p < np; ++p) {
    const long n = probs_[p].n;
    add_range(L.rd, A[p], sizeof(double) * elems(t_a, n, (int)ai.size()));
    add_range(L.rd, B[p], sizeof(double) * elems(t_b, n, (int)bi.size()));
    add_range(L.wr, out[p], sizeof(double));
  }
  L.ranged = true;
  L.kind = Launch::DOTB;
  L.n_prob = np;
  L.d_desc = upload(ps.data(), sizeof(DotbProblem) * np);
  L.n_tasks = (int)tasks.size();
  L.d_tasks = upload(tasks.data(), sizeof(ElemTask) * std::max<size_t>(tasks.size(), 1));
  {
    const std::vector<int> bf = block_first_tasks(tasks, total);
    L.d_bfirst = upload(bf.data(), sizeof(int) * bf.size());
  }
  L.n_elem = total;
  L.bytes = 2.0 * sizeof(double) * (double)total;
  L.d_partial = scratch_->tail_ws;
  L.tag = tag + "(blocked dot)";
  dst.push_back(L);
  return true;
}

void Executor::merge_fills(std::vector<Launch>& L) {
  std::vector<Launch> out;
  std::vector<bool> merged;
  for (Launch& l : L) {
    if (l.kind == Launch::ELEM && l.zero_fill && !out.empty() && out.back().kind == Launch::ELEM &&
        out.back().zero_fill) {
      Launch& m = out.back();
      const int po = (int)m.eprobs.size();
      m.eprobs.insert(m.eprobs.end(), l.eprobs.begin(), l.eprobs.end());
      for (ElemTask t : l.etasks) {
        t.prob += po;
        t.first += m.n_elem;
        m.etasks.push_back(t);
      }
      m.n_elem += l.n_elem;
      m.bytes += l.bytes;
      m.tag += "+" + l.tag;
      merged.back() = true;
      continue;
    }
    out.push_back(std::move(l));
    merged.push_back(false);
  }
  for (size_t k = 0; k < out.size(); ++k) {
    if (!merged[k]) continue;
    Launch& m = out[k];
    m.n_prob = (int)m.eprobs.size();
    m.d_desc = upload(m.eprobs.data(), sizeof(ElemProblem) * m.eprobs.size());
    m.n_tasks = (int)m.etasks.size();
    m.d_tasks = upload(m.etasks.data(), sizeof(ElemTask) * std::max<size_t>(m.etasks.size(), 1));
    const std::vector<int> bf = block_first_tasks(m.etasks, m.n_elem);
    m.d_bfirst = upload(bf.data(), sizeof(int) * bf.size());
    m.total = (int)std::min<long long>((m.n_elem + 255) / 256, 1 << 30);
  }
  L = std::move(out);
}

double Executor::sgemm_flops_forward() const {
  double f = 0.0;
  for (const Launch& l : fwd_)
    if (l.kind == Launch::SGEMM) f += l.flops;
  return f;
}

Launch Executor::merge_sgemm(const std::vector<Launch*>& parts) {
  Launch M;
  M.kind = Launch::SGEMM;
  M.ranged = true;
  int part_base = 0;
  for (const Launch* l : parts) {
    const int po = (int)M.sprobs.size();
    M.sprobs.insert(M.sprobs.end(), l->sprobs.begin(), l->sprobs.end());
    for (SgemmTask t : l->stasks) {
      t.prob += po;
      if (t.part >= 0) t.part += part_base;
      M.stasks.push_back(t);
    }
    int n_parts = 0;
    for (SgemmReduce r : l->sreds) {
      r.prob += po;
      r.first += part_base;
      n_parts += r.count;
      M.sreds.push_back(r);
    }
    part_base += n_parts;
    M.flops += l->flops;
    M.bytes += l->bytes;
    M.prob_flops.insert(M.prob_flops.end(), l->prob_flops.begin(), l->prob_flops.end());
    M.prob_inst.insert(M.prob_inst.end(), l->prob_inst.begin(), l->prob_inst.end());
    M.rd.insert(M.rd.end(), l->rd.begin(), l->rd.end());
    M.wr.insert(M.wr.end(), l->wr.begin(), l->wr.end());
    M.tag += (M.tag.empty() ? "" : "+") + l->tag;
  }
  // longest tasks first, so that the last wave of the launch holds short ones
  std::stable_sort(M.stasks.begin(), M.stasks.end(),
                   [](const SgemmTask& a, const SgemmTask& b) { return sgemm_task_cost(a) > sgemm_task_cost(b); });
  normalize(M.rd);
  normalize(M.wr);
  M.n_prob = (int)M.sprobs.size();
  M.d_desc = upload(M.sprobs.data(), sizeof(SgemmProblem) * M.sprobs.size());
  M.n_tasks = (int)M.stasks.size();
  M.d_tasks = upload(M.stasks.data(), sizeof(SgemmTask) * std::max<size_t>(M.stasks.size(), 1));
  M.n_red = (int)M.sreds.size();
  if (M.n_red > 0) {
    M.d_red = upload(M.sreds.data(), sizeof(SgemmReduce) * M.sreds.size());
    M.d_partial = scratch_->tail_ws;
  }
  M.total = (M.n_tasks + 3) / 4;
  return M;
}

Launch Executor::merge_elem(const std::vector<Launch*>& parts) {
  Launch M;
  M.kind = Launch::ELEM;
  M.ranged = true;
  M.zero_fill = true;
  for (const Launch* l : parts) {
    const int po = (int)M.eprobs.size();
    M.eprobs.insert(M.eprobs.end(), l->eprobs.begin(), l->eprobs.end());
    for (ElemTask t : l->etasks) {
      t.prob += po;
      t.first += M.n_elem;
      M.etasks.push_back(t);
    }
    M.n_elem += l->n_elem;
    M.bytes += l->bytes;
    M.zero_fill = M.zero_fill && l->zero_fill;
    M.rd.insert(M.rd.end(), l->rd.begin(), l->rd.end());
    M.wr.insert(M.wr.end(), l->wr.begin(), l->wr.end());
    M.tag += (M.tag.empty() ? "" : "+") + l->tag;
  }
  normalize(M.rd);
  normalize(M.wr);
  M.n_prob = (int)M.eprobs.size();
  M.d_desc = upload(M.eprobs.data(), sizeof(ElemProblem) * M.eprobs.size());
  M.n_tasks = (int)M.etasks.size();
  M.d_tasks = upload(M.etasks.data(), sizeof(ElemTask) * std::max<size_t>(M.etasks.size(), 1));
  const std::vector<int> bf = block_first_tasks(M.etasks, M.n_elem);
  M.d_bfirst = upload(bf.data(), sizeof(int) * bf.size());
  M.total = (int)std::min<long long>((M.n_elem + 255) / 256, 1 << 30);
  return M;
}

void Executor::fuse_levels(std::vector<Launch>& L) {
  const int nL = (int)L.size();
  for (Launch& l : L) {
    normalize(l.rd);
    normalize(l.wr);
  }
  // level: one more than the highest level of any earlier launch it must follow
  std::vector<int> level(nL, 0);
  int top = 0;
  for (int i = 0; i < nL; ++i) {
    int lv = 0;
    for (int j = i - 1; j >= 0; --j)
      if (level[j] + 1 > lv && ordered(L[j], L[i])) lv = level[j] + 1;
    level[i] = lv;
    top = std::max(top, lv);
  }
  std::vector<std::vector<int>> at(top + 1);
  for (int i = 0; i < nL; ++i) at[level[i]].push_back(i);
  const long ws_tiles = scratch_ && scratch_->tail_ws ? (long)(scratch_->tail_ws_doubles / 256) : 0;
  std::vector<Launch> out;
  std::vector<void*> freed;
  auto retire = [&](Launch& l) {
    for (void* d : {l.d_desc, l.d_tasks, l.d_red, l.d_bfirst})
      if (d) freed.push_back(d);
  };
  for (const std::vector<int>& lv : at) {
    std::vector<Launch*> sg, el;
    for (int i : lv) {
      Launch& l = L[i];
      if (l.kind == Launch::SGEMM && !l.sprobs.empty()) sg.push_back(&l);
      else if (l.kind == Launch::ELEM && !l.eprobs.empty()) el.push_back(&l);
      else out.push_back(std::move(l));
    }
    if (el.size() == 1) {
      out.push_back(std::move(*el[0]));
    } else if (el.size() > 1) {
      out.push_back(merge_elem(el));
      for (Launch* l : el) retire(*l);
    }
    // blocked contractions: one launch while their partial tiles fit the workspace
    size_t k = 0;
    while (k < sg.size()) {
      std::vector<Launch*> grp;
      long parts = 0;
      for (; k < sg.size(); ++k) {
        long np = 0;
        for (const SgemmReduce& r : sg[k]->sreds) np += r.count;
        if (!grp.empty() && parts + np > ws_tiles) break;
        grp.push_back(sg[k]);
        parts += np;
      }
      if (grp.size() == 1) {
        out.push_back(std::move(*grp[0]));
      } else {
        out.push_back(merge_sgemm(grp));
        for (Launch* l : grp) retire(*l);
      }
    }
  }
  release(freed);
  for (Launch& l : out) {   // host copies no longer needed
    std::vector<SgemmProblem>().swap(l.sprobs);
    std::vector<SgemmTask>().swap(l.stasks);
    std::vector<SgemmReduce>().swap(l.sreds);
    std::vector<ElemProblem>().swap(l.eprobs);
    std::vector<ElemTask>().swap(l.etasks);
  }
  L = std::move(out);
}

// ------------------------------------------------------------------ build
void Executor::build(const Program* prog, const std::vector<ProblemRef>& probs, Binder bind, Scratch* scratch,
                     std::function<double*(int, size_t)> const_alloc, bool want_backward,
                     const std::vector<int>& const_grads, std::function<double*(size_t)> cache_alloc,
                     size_t cache_budget) {
  cache_alloc_ = cache_alloc;
  cache_budget_ = cache_budget;
  if (!prog->finalized()) throw std::runtime_error("Program::finalize() not called");
  prog_ = prog;
  probs_ = probs;
  scratch_ = scratch;
  const_alloc_ = const_alloc;
  if (!mom_.empty()) infer_laws();
  plan_packing(want_backward);
  const int np = (int)probs.size();
  const int nt = (int)prog->t.size();
  std::vector<PerProb> fwd(nt, PerProb(np)), grd(nt, PerProb(np));
  std::vector<bool> need_grad(nt, false);
  for (int k = 0; k < nt; ++k) {
    const TensorDecl& d = prog->t[k];
    for (int p = 0; p < np; ++p) fwd[k][p] = bind(k, p, false, elems(k, probs[p].n, d.rank));
    bool g = (d.kind == T_INPUT || d.kind == T_OUTPUT || (d.kind == T_INTER && (!d.derived || inline_setup_)));
    if (std::find(const_grads.begin(), const_grads.end(), k) != const_grads.end()) g = true;
    need_grad[k] = g && want_backward;
    if (need_grad[k])
      for (int p = 0; p < np; ++p) grd[k][p] = bind(k, p, true, elems(k, probs[p].n, d.rank));
  }
  auto cidx = [&](int k) {
    return (k >= 0 && (prog->t[k].kind == T_CONST || (prog->t[k].derived && !inline_setup_))) ? k : -1;
  };
  // set-up ops first (constants only), once per instance
  if (!inline_setup_) {
    std::vector<ProblemRef> firsts;
    std::vector<int> idx;
    std::vector<bool> seen_inst;
    for (int p = 0; p < np; ++p) {
      const int inst = probs[p].inst;
      if (inst >= (int)seen_inst.size()) seen_inst.resize(inst + 1, false);
      if (seen_inst[inst]) continue;
      seen_inst[inst] = true;
      firsts.push_back(probs[p]);
      idx.push_back(p);
    }
    auto sub = [&](const PerProb& v) {
      PerProb r;
      for (int p : idx) r.push_back(v[p]);
      return r;
    };
    Scratch firsts_scratch;
    firsts_scratch.a = sub(scratch->a);
    firsts_scratch.b = sub(scratch->b);
    firsts_scratch.c = sub(scratch->c);
    firsts_scratch.part = sub(scratch->part);
    firsts_scratch.dot_partial = scratch->dot_partial;
    probs_ = firsts;
    scratch_ = &firsts_scratch;
    for (const SymOp& o : prog->ops) {
      if (!o.setup) continue;
      PerProb ob;
      if (o.b >= 0) ob = sub(fwd[o.b]);
      contract(setup_, sub(fwd[o.out]), o.oi, o.alpha, sub(fwd[o.a]), o.ai, -1, o.b >= 0 ? &ob : nullptr, o.bi,
               -1, o.accumulate, "setup:" + prog->t[o.out].name, -1, -1, o.out, o.a, o.b);
    }
    // Packed copies of the constants the blocked ops read, gathered from the dense
    // blocks (after the derived ones are made) each time the set-up list runs; the
    // program then reads the copies.
    for (int k : plan_const_packing(const_grads)) {
      const TensorDecl& d = prog->t[k];
      std::string ix;
      for (int a = 0; a < d.rank; ++a) ix.push_back((char)('p' + a));
      PerProb pk;
      std::map<int, double*> of_inst;
      for (const ProblemRef& f : firsts) {
        const size_t cnt = (size_t)ipow_l(f.n, d.rank - 1);
        double* q = const_alloc_(f.inst, cnt);
        const_bytes_ += sizeof(double) * cnt;
        of_inst[f.inst] = q;
        pk.push_back(q);
      }
      if (!elem_blocked(setup_, sub(fwd[k]), ix, pk, ix, 1.0, 0.0, k, k, "setup:pack:" + d.name, nullptr, 0, 1))
        throw std::runtime_error("no packed copy of constant " + d.name);
      for (int p = 0; p < np; ++p) fwd[k][p] = of_inst[probs[p].inst];
      packed_[k] = 1;
    }
    probs_ = probs;
    scratch_ = scratch;
  }
  // Packed shadows of the rank >= 2 inputs and outputs (and of their gradients):
  // the ops work on the shadows, the inputs are gathered into them first and the
  // outputs scattered back last (over the allowed elements; the dense buffers'
  // forbidden elements stay zero).
  const std::vector<int> io = plan_io_packing();
  std::vector<PerProb> dense_f(nt), dense_g(nt);
  auto shadows = [&](int k) {
    PerProb s(np);
    for (int p = 0; p < np; ++p) {
      const size_t cnt = (size_t)ipow_l(probs[p].n, prog->t[k].rank - 1);
      s[p] = const_alloc_(probs[p].inst, cnt);
      const_bytes_ += sizeof(double) * cnt;
    }
    return s;
  };
  auto letters = [](int r) {
    std::string ix;
    for (int a = 0; a < r; ++a) ix.push_back((char)('p' + a));
    return ix;
  };
  for (int k : io) {
    dense_f[k] = fwd[k];
    fwd[k] = shadows(k);
    if (need_grad[k]) {
      dense_g[k] = grd[k];
      grd[k] = shadows(k);
    }
    packed_[k] = 1;
  }
  auto move_packed = [&](std::vector<Launch>& dst, const PerProb& X, const PerProb& Y, int k, bool to_packed,
                         const std::string& what) {
    const std::string ix = letters(prog->t[k].rank);
    if (!elem_blocked(dst, X, ix, Y, ix, 1.0, 0.0, k, k, what + prog->t[k].name, nullptr, to_packed ? 0 : 1,
                      to_packed ? 1 : 0))
      throw std::runtime_error("no packed shadow of " + prog->t[k].name);
  };
  for (int k : io)
    if (prog->t[k].kind == T_INPUT) move_packed(fwd_, dense_f[k], fwd[k], k, true, "gather:");
  version_.assign(nt, 0);
  auto vidx = [&](int k) { return (k >= 0 && cidx(k) < 0) ? k : -1; };
  for (const SymOp& o : prog->ops) {
    if (o.setup && !inline_setup_) continue;
    contract(fwd_, fwd[o.out], o.oi, o.alpha, fwd[o.a], o.ai, cidx(o.a), o.b >= 0 ? &fwd[o.b] : nullptr, o.bi,
             cidx(o.b), o.accumulate, prog->t[o.out].name, vidx(o.a), vidx(o.b), o.out, o.a, o.b);
    version_[o.out]++;
  }
  for (int k : io)
    if (prog->t[k].kind == T_OUTPUT) move_packed(fwd_, fwd[k], dense_f[k], k, false, "scatter:");
  if (!want_backward) {
    const char* fz = std::getenv("FTCC_FUSE");
    if (!mom_.empty() && !(fz && fz[0] == '0')) fuse_levels(fwd_);
    dump_plan();
    return;
  }
  // zero every gradient buffer except the cotangents of the outputs
  for (int k = 0; k < nt; ++k)
    if (need_grad[k] && prog->t[k].kind != T_OUTPUT)
      fill(bwd_, grd[k], prog->t[k].rank, "zero:" + prog->t[k].name, k);
  for (int k : io)
    if (need_grad[k] && prog->t[k].kind == T_OUTPUT) move_packed(bwd_, dense_g[k], grd[k], k, true, "gather:d");
  for (int i = (int)prog->ops.size() - 1; i >= 0; --i) {
    const SymOp& o = prog->ops[i];
    if (o.setup && !inline_setup_) continue;
    const std::string tag = "bwd:" + prog->t[o.out].name;
    if (o.b < 0) {
      if (need_grad[o.a])
        contract(bwd_, grd[o.a], o.ai, o.alpha, grd[o.out], o.oi, -1, nullptr, "", -1, true, tag, -1, -1, o.a, o.out,
                 -1);
      continue;
    }
    if (need_grad[o.a])
      contract(bwd_, grd[o.a], o.ai, o.alpha, grd[o.out], o.oi, -1, &fwd[o.b], o.bi, cidx(o.b), true, tag + ":dA",
               -1, vidx(o.b), o.a, o.out, o.b);
    if (need_grad[o.b])
      contract(bwd_, grd[o.b], o.bi, o.alpha, fwd[o.a], o.ai, cidx(o.a), &grd[o.out], o.oi, -1, true, tag + ":dB",
               vidx(o.a), -1, o.b, o.a, o.out);
  }
  for (int k : io)
    if (need_grad[k] && prog->t[k].kind == T_INPUT) move_packed(bwd_, grd[k], dense_g[k], k, false, "scatter:d");
  // FTCC_FUSE=0 keeps the program order, one launch per contraction (diagnostics)
  const char* fz = std::getenv("FTCC_FUSE");
  if (!mom_.empty() && !(fz && fz[0] == '0')) {
    fuse_levels(fwd_);
    fuse_levels(bwd_);
  } else {
    merge_fills(bwd_);
  }
  dump_plan();
}

// Autotuner: every grouped GEMM launch with 128x128 tiles is timed on its own
// descriptors (the real operand pointers and shapes of the program) with each
// candidate tile configuration, and the fastest is kept.  Outputs written while
// timing are overwritten by the first real sweep (every tensor's first op
// overwrites it; gradient buffers are zero-filled before each backward).
void Executor::autotune(hipStream_t s) {
  const char* env = std::getenv("FTCC_AUTOTUNE");
  hipEvent_t e0, e1;
  FTCC_HIP(hipEventCreate(&e0));
  FTCC_HIP(hipEventCreate(&e1));
  // every candidate of a GEMM launch: its own descriptor set (tile size, split-K)
  // with each tile configuration of that size (BK 16 or 32 for 128 x 128 tiles),
  // timed over two launches after a warm-up (split-K reduce included)
  auto time_one = [&](const Launch& v, int cfg) {
    auto go = [&] {
      launch_gemm(cfg, v.ta, v.tb, (const GemmProblem*)v.d_desc, v.d_prefix, v.n_prob, v.total, tail_of(v, cfg), s);
      if (v.splitk_blocks > 0)
        launch_splitk_reduce((const GemmProblem*)v.d_desc, v.d_prefix2, v.n_prob, v.splitk_blocks, s);
    };
    go();
    FTCC_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 2; ++r) go();
    FTCC_HIP(hipEventRecord(e1, s));
    FTCC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FTCC_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms * 0.5f;
  };
  for (std::vector<Launch>* lst : {&fwd_, &bwd_}) {
    for (Launch& l : *lst) {
      if (l.kind != Launch::GEMM) continue;
      if (env && env[0] == '0') {
        l.alts.clear();
        continue;
      }
      int best_v = -1, best_cfg = l.cfg;
      float best_ms = 1e30f;
      for (int v = -1; v < (int)l.alts.size(); ++v) {
        const Launch& cand = v < 0 ? l : l.alts[v];
        const std::vector<int> cfgs = gemm_bm(cand.cfg) == 128 ? std::vector<int>{0, 2} : std::vector<int>{1};
        for (int cfg : cfgs) {
          const float ms = time_one(cand, cfg);
          if (ms < best_ms) {
            best_ms = ms;
            best_v = v;
            best_cfg = cfg;
          }
        }
      }
      if (best_v >= 0) {
        const Launch& w = l.alts[best_v];
        l.d_desc = w.d_desc;
        l.d_prefix = w.d_prefix;
        l.d_prefix2 = w.d_prefix2;
        l.total = w.total;
        l.splitk_blocks = w.splitk_blocks;
        l.min_k = w.min_k;
      }
      l.cfg = best_cfg;
      l.tuned_ms = best_ms;
      l.alts.clear();
    }
  }
  FTCC_HIP(hipEventDestroy(e0));
  FTCC_HIP(hipEventDestroy(e1));
  dump_plan();
}

// FTCC_PLAN_DUMP=1 prints the lowered launch lists (diagnostics only)
void Executor::dump_plan() const {
  const char* env = std::getenv("FTCC_PLAN_DUMP");
  if (!env || env[0] != '1') return;
  const char* kinds[] = {"perm", "gemm", "dot", "fill", "sgemm", "elem", "dotb"};
  const std::pair<const char*, const std::vector<Launch>*> lists[] = {
      {"setup", &setup_}, {"forward", &fwd_}, {"backward", &bwd_}};
  for (const auto& pl : lists) {
    int counts[7] = {0, 0, 0, 0, 0, 0, 0};
    double fl = 0.0;
    for (const Launch& l : *pl.second) {
      counts[l.kind]++;
      fl += l.flops;
      std::fprintf(stderr, "[plan] %-8s %-4s cfg=%d ta=%d tb=%d blocks=%d split=%d gflop=%.3f ms=%.3f %s\n",
                   pl.first, kinds[l.kind], l.cfg, (int)l.ta, (int)l.tb, l.total, l.splitk_blocks > 0,
                   l.flops * 1e-9, l.tuned_ms, l.tag.c_str());
    }
    std::fprintf(stderr,
                 "[plan] %s: %d perm, %d gemm, %d dot, %d fill, %d blocked, %d blocked-elem, %d blocked-dot, "
                 "%.3f GFLOP\n",
                 pl.first, counts[0], counts[1], counts[2], counts[3], counts[4], counts[5], counts[6], fl * 1e-9);
  }
}

// ------------------------------------------------------------------ run
// algorithmic flops of a GEMM launch over the problems whose instance runs
double Executor::run_flops(const Launch& l) const {
  if (!gate_host_ || l.prob_flops.empty()) return l.flops;
  double f = 0.0;
  for (size_t p = 0; p < l.prob_flops.size(); ++p)
    if (gate_host_[l.prob_inst[p]]) f += l.prob_flops[p];
  return f;
}

void Executor::run(const std::vector<Launch>& L, hipStream_t s) const {
  for (const Launch& l : L) {
    switch (l.kind) {
      case Launch::PERM:
      case Launch::FILL:
        launch_permute((const PermProblem*)l.d_desc, l.d_prefix, l.n_prob, l.total, s);
        break;
      case Launch::GEMM: {
        const bool timed = prof_ && prof_->enabled && gemm_bm(l.cfg) == 128;
        if (timed) prof_->record_begin(s);
        launch_gemm(l.cfg, l.ta, l.tb, (const GemmProblem*)l.d_desc, l.d_prefix, l.n_prob, l.total, tail_of(l, l.cfg),
                    s);
        if (timed) prof_->record_end(s, run_flops(l));
      }
        if (l.splitk_blocks > 0)
          launch_splitk_reduce((const GemmProblem*)l.d_desc, l.d_prefix2, l.n_prob, l.splitk_blocks, s);
        break;
      case Launch::DOT:
        launch_dot((const DotProblem*)l.d_desc, l.n_prob, l.dot_blocks, l.d_partial, s);
        break;
      case Launch::SGEMM:
        launch_sgemm((const SgemmProblem*)l.d_desc, (const SgemmTask*)l.d_tasks, l.n_tasks, l.d_partial,
                     (const SgemmReduce*)l.d_red, l.n_red, s);
        break;
      case Launch::DOTB:
        launch_dotb((const DotbProblem*)l.d_desc, l.n_prob, (const ElemTask*)l.d_tasks, (const int*)l.d_bfirst,
                    l.n_tasks, l.n_elem,
                    l.d_partial, s);
        break;
      case Launch::ELEM:
        launch_elem((const ElemProblem*)l.d_desc, (const ElemTask*)l.d_tasks, (const int*)l.d_bfirst, l.n_tasks,
                    l.n_elem, s);
        break;
    }
  }
}

// ------------------------------------------------------------------ profiler
void KernelProfiler::reset() {
  used = 0;
  pending_flops.clear();
  flops = seconds = 0.0;
  launches = 0;
}

void KernelProfiler::record_begin(hipStream_t s) {
  if (used + 2 > (int)ev.size()) {
    // pool full: wait for the stream and harvest before reusing events
    FTCC_HIP(hipStreamSynchronize(s));
    harvest();
    if (ev.size() < 8192) {
      const size_t old = ev.size();
      ev.resize(old ? old * 2 : 512);
      for (size_t k = old; k < ev.size(); ++k) FTCC_HIP(hipEventCreate(&ev[k]));
    }
  }
  FTCC_HIP(hipEventRecord(ev[used], s));
}

void KernelProfiler::record_end(hipStream_t s, double f) {
  FTCC_HIP(hipEventRecord(ev[used + 1], s));
  pending_flops.push_back(f);
  used += 2;
}

void KernelProfiler::harvest() {
  for (size_t k = 0; k < pending_flops.size(); ++k) {
    float ms = 0.f;
    FTCC_HIP(hipEventElapsedTime(&ms, ev[2 * k], ev[2 * k + 1]));
    seconds += ms * 1e-3;
    flops += pending_flops[k];
    ++launches;
  }
  pending_flops.clear();
  used = 0;
}

KernelProfiler::~KernelProfiler() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
}

long Executor::dispatches(const std::vector<Launch>& L) const {
  long k = 0;
  for (const Launch& l : L) {
    switch (l.kind) {
      case Launch::GEMM: {
        const GemmTail t = tail_of(l, l.cfg);
        k += (l.total > 0) + (t.splits > 1 && t.dp_tiles < l.total) + (l.splitk_blocks > 0);
        break;
      }
      case Launch::SGEMM: k += (l.n_tasks > 0) + (l.n_tasks > 0 && l.n_red > 0); break;
      case Launch::DOT: k += 2; break;
      case Launch::DOTB: k += 1 + (l.n_elem > 0 && l.n_tasks > 0); break;
      case Launch::ELEM: k += (l.n_tasks > 0 && l.n_elem > 0); break;
      default: k += (l.total > 0); break;
    }
  }
  return k;
}

double Executor::bytes_forward() const {
  double b = 0.0;
  for (const Launch& l : fwd_) b += l.bytes;
  return b;
}

double Executor::gemm_flops_forward() const {
  double f = 0.0;
  for (const Launch& l : fwd_) f += l.flops;
  return f;
}

double Executor::gemm_flops_backward() const {
  double f = 0.0;
  for (const Launch& l : bwd_) f += l.flops;
  return f;
}

}  // namespace ftcc
