// Two-body response density Gamma_pqrs = dOmega/d<pq|rs> (the response of
// Section II.D at a frozen reference, with respect to every integral): a third
// executor whose reverse pass reaches the raw integral blocks, and the entry
// point ftcc_two_body_density.
#include "api_internal.h"

namespace {

// Two-body response density Gamma_abcd = dOmega/d<ab|cd> at a frozen reference:
//   sum over the 12 weighted blocks of w_a w_b w_c w_d G^XYZW_abcd
//   + g gc_ac n_b delta_bd - gc_ad n_b delta_bc          (through the Fock operator in u)
//   + (g/2) (g delta_ac delta_bd - delta_ad delta_bc) n_a n_b   (Omega_1)
// with gc_pq = sum_XY w^X_p w^Y_q U^XY_pq, projected on the integrals with
// <ab|cd> = <ba|dc> (the average of the element and its exchange partner).
struct GammaBlocks {
  const double* G[12];
  char pat[12][4];
  const double* U[4];
  char upat[4][2];
};
__device__ double gamma_raw(const GammaBlocks& B, int n, const double* occ, const double* wo, const double* wv,
                            double g, int a, int b, int c, int d) {
  const long e = (((long)a * n + b) * n + c) * n + d;
  const int idx[4] = {a, b, c, d};
  double v = 0.0;
  for (int k = 0; k < 12; ++k) {
    double w = 1.0;
    for (int s = 0; s < 4; ++s) w *= (B.pat[k][s] == 'o') ? wo[idx[s]] : wv[idx[s]];
    if (w != 0.0) v += w * B.G[k][e];
  }
  auto gc = [&](int p, int q) {
    double x = 0.0;
    for (int k = 0; k < 4; ++k) {
      const double w = ((B.upat[k][0] == 'o') ? wo[p] : wv[p]) * ((B.upat[k][1] == 'o') ? wo[q] : wv[q]);
      if (w != 0.0) x += w * B.U[k][(long)p * n + q];
    }
    return x;
  };
  if (b == d) v += g * gc(a, c) * occ[b];
  if (b == c) v -= gc(a, d) * occ[b];
  if (a == c && b == d) v += 0.5 * g * g * occ[a] * occ[b];
  if (a == d && b == c) v -= 0.5 * g * occ[a] * occ[b];
  return v;
}
__global__ void gamma_assemble_kernel(GammaBlocks B, int n, const double* occ, const double* wo, const double* wv,
                                      double g, double* out) {
  const long total = (long)n * n * n * n;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int d = (int)(e % n), c = (int)((e / n) % n), b = (int)((e / n / n) % n), a = (int)(e / n / n / n);
    out[e] = 0.5 * (gamma_raw(B, n, occ, wo, wv, g, a, b, c, d) + gamma_raw(B, n, occ, wo, wv, g, b, a, d, c));
  }
}

}  // namespace

namespace ftcc {
namespace host {

// ------------------------------------------------------------------ two-body density
// A third executor of the same program whose reverse pass also yields the
// gradients with respect to every constant block (the u and g blocks): the
// constant combinations are evaluated inside the forward pass so that their
// gradients reach the raw blocks.  Built on first use; its intermediates share
// the main executor's buffers (the two never run interleaved).
void build_gamma_executor(ftcc_ctx* c) {
  if (c->ex_g) return;
  const Program& prog = c->prog;
  const int SL = c->slots;
  std::vector<ProblemRef> probs;
  for (int i = 0; i < c->B; ++i)
    for (int x = 0; x < SL; ++x) probs.push_back({i, x, c->inst[i].n});
  const int id_t1 = prog.id("t1"), id_t2 = prog.id("t2"), id_S1 = prog.id("S1"), id_S2 = prog.id("S2"),
            id_E = prog.id("E");
  auto buf = [c](std::map<std::pair<int, int>, double*>& store, int t, int key, long count) {
    return shared_buf(c, store, t, key, count);
  };
  Binder bind = [&, c](int t, int p, bool grad, size_t count) -> double* {
    const TensorDecl& d = prog.t[t];
    const int i = probs[p].inst;
    const long n = probs[p].n, n2 = n * n, cnt = ipow(n, d.rank);
    if (t == id_t1) return grad ? c->s_gr[p] : c->s_amp[p];
    if (t == id_t2) return grad ? c->s_gr[p] + n2 : c->s_amp[p] + n2;
    if (t == id_S1) return grad ? c->s_cot[p] : c->s_S[p];
    if (t == id_S2) return grad ? c->s_cot[p] + n2 : c->s_S[p] + n2;
    if (t == id_E) return grad ? c->s_ebar[p] : c->s_e[p];
    if (d.kind == T_CONST) return grad ? buf(c->g_cgrad, t, p, cnt) : c->inst[i].blk[d.name];
    if (d.derived) return buf(grad ? c->g_cgrad : c->g_derived, t, p, cnt);
    return buf(grad ? c->inter_grad : c->inter, t, p, (long)count);
  };
  std::vector<int> cgrads;
  for (int k = 0; k < (int)prog.t.size(); ++k)
    if (prog.t[k].kind == T_CONST) cgrads.push_back(k);
  auto calloc_ = [c](int, size_t count) { return c->dalloc(count); };
  auto vcache = [c](size_t count) { return c->dalloc(count); };
  std::unique_ptr<Executor> ex(new Executor());
  ex->set_inline_setup(true);
  ex->set_gate(c->d_run, c->run_host.data());
  if (momentum_on(c)) {
    std::vector<const InstMomentum*> by_inst;
    for (const Instance& I : c->inst) by_inst.push_back(&I.mom);
    ex->set_momentum(by_inst);
  }
  ex->build(&prog, probs, bind, &c->scratch, calloc_, true, cgrads, vcache, 0);
  c->ex_g = std::move(ex);
  for (int i = 0; i < c->B; ++i) {
    Instance& I = c->inst[i];
    const long n2 = (long)I.n * I.n;
    for (int k = 0; k < 12; ++k)
      if (!I.gacc[k]) I.gacc[k] = c->dalloc(n2 * n2);
  }
}

// forward + reverse pass of ex_g over the slots, then add the constant-block
// gradients of every running slot to the instance accumulators (u blocks into
// ugrad_acc, g blocks into gacc)
void gamma_pass(ftcc_ctx* c) {
  const Program& prog = c->prog;
  c->ex_g->run_forward(c->stream);
  c->ex_g->run_backward(c->stream);
  const int SL = c->slots;
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    Instance& I = c->inst[i];
    const long n2 = (long)I.n * I.n;
    for (int x = 0; x < SL; ++x) {
      const int q = i * SL + x;
      for (int k = 0; k < 4; ++k)
        launch_axpby(n2, 1.0, c->g_cgrad.at(std::make_pair(prog.id(kU[k]), q)), 1.0, I.ugrad_acc[k], c->stream);
      for (int k = 0; k < 12; ++k)
        launch_axpby(n2 * n2, 1.0, c->g_cgrad.at(std::make_pair(prog.id(kG[k]), q)), 1.0, I.gacc[k], c->stream);
    }
  }
}

// one node (or RK stage) x through the single slot
void gamma_node(ftcc_ctx* c, int x) {
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    const int q = i * c->m + x;
    node_copy(c, i, c->s_amp[i], c->amp[q]);
    node_copy(c, i, c->s_cot[i], c->cot[q]);
    dcopy(c, c->s_ebar[i], c->ebar[q], 1);
  }
  gamma_pass(c);
}

}  // namespace host
}  // namespace ftcc

extern "C" {

int ftcc_two_body_density(ftcc_ctx* c, double* gamma) {
  return run_guarded([&] {
    if (!c || !gamma) fail(FTCC_EINVAL, "null argument");
    if (!c->have_lambda) fail(FTCC_ESTATE, "call ftcc_lambda first");
    if (c->simpson) fail(FTCC_EINVAL, "the two-body density is built for propagators 0 to 4");
    FTCC_HIP(hipSetDevice(c->device));
    build_gamma_executor(c);
    const int B = c->B, m = c->m, P = c->P;
    std::vector<bool> ok(B);
    for (int i = 0; i < B; ++i) {
      Instance& I = c->inst[i];
      const long n2 = (long)I.n * I.n;
      ok[i] = I.status == 0 && I.lam_status == 0;
      for (int k = 0; k < 4; ++k) zero_d(c, I.ugrad_acc[k], n2);
      for (int k = 0; k < 12; ++k) zero_d(c, I.gacc[k], n2 * n2);
    }
    const auto wall0 = std::chrono::steady_clock::now();
    if (!c->rk) {
      // every node: (g_x/beta) dE/dI + <lambda-tilde_x, dS/dI> through the reverse pass
      for (int p = 0; p < P; ++p) {
        load_panel(c, p);
        set_run(c, ok);
        tau_run(c, TAU_LAMT, p);
        if (c->slots == m) {
          gamma_pass(c);
        } else {
          for (int x = 0; x < m; ++x) gamma_node(c, x);
        }
        trace(c, "two-body density", p + 1, P, std::vector<int>(1, 0), wall0);
      }
    } else {
      // every grid point (energy weight) and every stage (cotangent -kbar of its residual)
      set_run(c, ok);
      for (int k = 0; k <= P; ++k) {
        const int ns = k < P ? m : 1;
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
          gamma_node(c, x);
        }
      }
    }
    run_all(c);
    long off = 0;
    for (int i = 0; i < B; ++i) {
      Instance& I = c->inst[i];
      const long n = I.n, n4 = n * n * n * n;
      if (!ok[i]) {
        for (long e = 0; e < n4; ++e) gamma[off + e] = std::nan("");
        off += n4;
        continue;
      }
      GammaBlocks gb;
      for (int k = 0; k < 12; ++k) {
        gb.G[k] = I.gacc[k];
        std::memcpy(gb.pat[k], kG[k] + 2, 4);
      }
      for (int k = 0; k < 4; ++k) {
        gb.U[k] = I.ugrad_acc[k];
        std::memcpy(gb.upat[k], kU[k] + 2, 2);
      }
      double* d = nullptr;
      FTCC_HIP(hipMallocAsync((void**)&d, sizeof(double) * n4, c->stream));
      hipLaunchKernelGGL(gamma_assemble_kernel, dim3((unsigned)std::min<long>((n4 + 255) / 256, 65536)), dim3(256), 0,
                         c->stream, gb, (int)n, I.occ, I.wo, I.wv, c->gdeg, d);
      FTCC_HIP(hipGetLastError());
      FTCC_HIP(hipMemcpyAsync(gamma + off, d, sizeof(double) * n4, hipMemcpyDeviceToHost, c->stream));
      FTCC_HIP(hipFreeAsync(d, c->stream));
      off += n4;
    }
    sync(c);
  });
}

}  // extern "C"
