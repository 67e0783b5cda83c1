// Differential form of the imaginary-time amplitude equations (Section III):
// explicit Runge-Kutta steps on a uniform tau grid with Simpson's rule for
// Omega_CC, and the reverse pass of the march for Lambda and the response.
#include "api_internal.h"

namespace ftcc {
namespace host {

// ------------------------------------------------------------------ differential form
// Algorithm alg:diff: ds/dtau = -(Delta s + S[s]) (eqn:smud) stepped across the
// uniform grid tau_k = k h, h = beta / n_g, by an explicit Runge-Kutta method
// (Section III: RK1, RK2, RK4 with Simpson's rule for Omega_CC).  The executor
// has one slot per instance; "node" x of the node buffers is stage x of the
// current step: amp[x] its state Y_x, S[x] its residual, gr[x] its reverse-pass
// gradient.  Grid states s_k live in sb[k] (k = 0..n_g), their cotangents in
// abuf[k], and the slope cotangents kbar of step p, stage x in lam[p m + x].

// stage x of every running instance: amp[x] -> S[x], e[x]
void forward_one(ftcc_ctx* c, int x) {
  for (int i = 0; i < c->B; ++i)
    if (c->run_host[i]) node_copy(c, i, c->s_amp[i], c->amp[i * c->m + x]);
  run_fwd_slots(c);
  c->resid_evals += n_running(c);
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    node_copy(c, i, c->S[i * c->m + x], c->s_S[i]);
    dcopy(c, c->e[i * c->m + x], c->s_e[i], 1);
  }
}

// reverse pass of stage x (tape recomputed first): cot[x], ebar[x] -> gr[x], ugrad[x]; also S[x]
void backward_one(ftcc_ctx* c, int x) {
  for (int i = 0; i < c->B; ++i)
    if (c->run_host[i]) node_copy(c, i, c->s_amp[i], c->amp[i * c->m + x]);
  run_fwd_slots(c);
  c->resid_evals += n_running(c);
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    const int q = i * c->m + x;
    node_copy(c, i, c->S[q], c->s_S[i]);
    node_copy(c, i, c->s_cot[i], c->cot[q]);
    dcopy(c, c->s_ebar[i], c->ebar[q], 1);
  }
  run_bwd_slots(c);
  c->vjp_evals += n_running(c);
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    const int q = i * c->m + x;
    const long n = c->inst[i].n;
    node_copy(c, i, c->gr[q], c->s_gr[i]);
    for (int k = 0; k < 4; ++k) dcopy(c, c->ugrad[q][k], c->s_ugrad[i][k], n * n);
  }
}

// derivative-integral residual of stage x: amp[x] -> dS[x], de[x]
void d_forward_one(ftcc_ctx* c, int x) {
  for (int i = 0; i < c->B; ++i)
    if (c->run_host[i]) node_copy(c, i, c->s_amp[i], c->amp[i * c->m + x]);
  c->ex_d->run_forward(c->stream);
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    node_copy(c, i, c->dS[i * c->m + x], c->s_dS[i]);
    dcopy(c, c->de[i * c->m + x], c->s_de[i], 1);
  }
}

// out = x0 base + sum_l coef_l (-Delta Y_l + sigma S_l) for every instance (both
// amplitude segments); descriptors cached under (kind, step, stage) until the
// next solve.  track: max |out| into maxbits[2 i + 1].
void rk_combine(ftcc_ctx* c, int kind, int p, int x, double sigma, bool track,
                const std::function<RKSpec(int)>& spec) {
  const auto key = std::make_tuple(kind, p, x);
  auto it = c->rk_cache.find(key);
  if (it == c->rk_cache.end()) {
    std::vector<RKProblem> ps;
    std::vector<int> prefix;
    int total = 0;
    for (int i = 0; i < c->B; ++i) {
      const RKSpec sp = spec(i);
      const Instance& I = c->inst[i];
      const long n2 = (long)I.n * I.n;
      for (int seg = 0; seg < 2; ++seg) {
        RKProblem r;
        std::memset(&r, 0, sizeof(r));
        const long off = seg ? n2 : 0;
        r.eps = I.eps;
        r.n = I.n;
        r.rank = seg ? 4 : 2;
        r.len = seg_len(c, i, seg);
        r.idx = I.d_allowed[seg];
        r.base = sp.base ? sp.base + off : nullptr;
        r.x0 = sp.x0;
        r.nst = sp.nst;
        for (int l = 0; l < sp.nst; ++l) {
          r.coef[l] = sp.coef[l];
          r.Y[l] = sp.Y[l] ? sp.Y[l] + off : nullptr;
          r.S[l] = sp.S[l] ? sp.S[l] + off : nullptr;
        }
        r.sigma = sigma;
        r.out = sp.out + off;
        r.maxbits = track ? c->d_maxbits + 2 * i + 1 : nullptr;
        r.active = c->d_run + i;
        prefix.push_back(total);
        total += (int)((r.len + 1023) / 1024);
        ps.push_back(r);
      }
    }
    RKProblem* d_ps = nullptr;
    int* d_pre = nullptr;
    FTCC_HIP(hipMalloc((void**)&d_ps, sizeof(RKProblem) * ps.size()));
    FTCC_HIP(hipMalloc((void**)&d_pre, sizeof(int) * prefix.size()));
    FTCC_HIP(hipMemcpy(d_ps, ps.data(), sizeof(RKProblem) * ps.size(), hipMemcpyHostToDevice));
    FTCC_HIP(hipMemcpy(d_pre, prefix.data(), sizeof(int) * prefix.size(), hipMemcpyHostToDevice));
    it = c->rk_cache.emplace(key, std::make_pair(d_ps, d_pre)).first;
    c->rk_blocks[key] = total;
  }
  launch_rk_combine(it->second.first, it->second.second, 2 * c->B, c->rk_blocks[key], c->stream);
  FTCC_HIP(hipGetLastError());
}

// acc_i += <X_i, Y_i> over whole amplitude vectors, one deterministic dot per instance
void rk_dot(ftcc_ctx* c, int kind, int p, int x, const std::function<std::array<const double*, 3>(int)>& xyz) {
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    const auto key = std::make_tuple(kind * 65536 + i, p, x);
    auto it = c->rk_dots.find(key);
    if (it == c->rk_dots.end()) {
      const auto v = xyz(i);
      DotProblem d{};
      d.X = v[0];
      d.Y = v[1];
      d.out = const_cast<double*>(v[2]);
      d.len = node_len(c, i);
      d.alpha = 1.0;
      d.beta = 1.0;
      DotProblem* dd = nullptr;
      FTCC_HIP(hipMalloc((void**)&dd, sizeof(DotProblem)));
      FTCC_HIP(hipMemcpy(dd, &d, sizeof(DotProblem), hipMemcpyHostToDevice));
      it = c->rk_dots.emplace(key, dd).first;
    }
    launch_dot(it->second, 1, 64, c->scratch.dot_partial, c->stream);
  }
}

double rk_h(const ftcc_ctx* c, int i) { return c->inst[i].beta / c->P; }
double rk_a(const ftcc_ctx* c, int j, int l) { return c->rk_a[j * c->m + l]; }

// stage state Y_x of step p: sb[p] + h sum_{l<x} a_xl k_l, k_l = -(Delta Y_l + S_l)
void rk_stage_state(ftcc_ctx* c, int p, int x) {
  if (x == 0) {
    for (int i = 0; i < c->B; ++i)
      if (c->run_host[i]) node_copy(c, i, c->amp[i * c->m], c->inst[i].sb[p]);
    return;
  }
  rk_combine(c, 0, p, x, -1.0, false, [c, p, x](int i) {
    RKSpec sp;
    sp.base = c->inst[i].sb[p];
    sp.x0 = 1.0;
    for (int l = 0; l < x; ++l) {
      sp.coef[sp.nst] = rk_h(c, i) * rk_a(c, x, l);
      sp.Y[sp.nst] = c->amp[i * c->m + l];
      sp.S[sp.nst] = c->S[i * c->m + l];
      ++sp.nst;
    }
    sp.out = c->amp[i * c->m + x];
    return sp;
  });
}

// every stage state of step p with the residuals of stages 0..m-2 (the last
// stage's residual comes from the tape of its reverse pass, or is evaluated by
// the caller)
void rk_recompute_stages(ftcc_ctx* c, int p) {
  for (int x = 0; x < c->m; ++x) {
    rk_stage_state(c, p, x);
    if (x < c->m - 1) forward_one(c, x);
  }
}

void set_ebar(ftcc_ctx* c, int x, int grid_point) {
  for (int i = 0; i < c->B; ++i) {
    if (!c->run_host[i]) continue;
    double* e = c->ebar[i * c->m + x];
    if (grid_point >= 0) dcopy(c, e, c->d_rkw + grid_point, 1);
    else zero_d(c, e, 1);
  }
}

void rk_solve(ftcc_ctx* c, std::vector<int>& status) {
  const int B = c->B, m = c->m, P = c->P;
  std::vector<double> ebuf((size_t)B * (P + 1), 0.0);
  std::vector<bool> ok(B);
  const auto wall0 = std::chrono::steady_clock::now();
  auto energy_to_host = [&](int k) {
    for (int i = 0; i < B; ++i)
      if (c->run_host[i])
        FTCC_HIP(hipMemcpyAsync(&ebuf[(size_t)i * (P + 1) + k], c->e[i * m], sizeof(double), hipMemcpyDeviceToHost,
                                c->stream));
  };
  for (int p = 0; p < P; ++p) {
    for (int i = 0; i < B; ++i) ok[i] = status[i] == 0;
    set_run(c, ok);
    for (int x = 0; x < m; ++x) {
      rk_stage_state(c, p, x);
      forward_one(c, x);
      if (x == 0) energy_to_host(p);     // E at the grid point s_p = Y_0
    }
    reset_maxbits(c);
    rk_combine(c, 1, p, 0, -1.0, true, [c, p](int i) {
      RKSpec sp;
      sp.base = c->inst[i].sb[p];
      sp.x0 = 1.0;
      for (int l = 0; l < c->m; ++l) {
        sp.coef[sp.nst] = rk_h(c, i) * c->rk_b[l];
        sp.Y[sp.nst] = c->amp[i * c->m + l];
        sp.S[sp.nst] = c->S[i * c->m + l];
        ++sp.nst;
      }
      sp.out = c->inst[i].sb[p + 1];
      return sp;
    });
    const std::vector<double> mb = read_maxbits(c);
    for (int i = 0; i < B; ++i)
      if (status[i] == 0 && !std::isfinite(mb[2 * i + 1])) status[i] = FTCC_ENONFINITE;
    trace(c, "forward (Runge-Kutta)", p + 1, P, std::vector<int>(1, m), wall0);
  }
  for (int i = 0; i < B; ++i) ok[i] = status[i] == 0;
  set_run(c, ok);
  rk_stage_state(c, P, 0);
  forward_one(c, 0);
  energy_to_host(P);
  run_all(c);
  sync(c);
  for (int i = 0; i < B; ++i) {
    Instance& I = c->inst[i];
    double om = 0.0;
    for (int k = 0; k <= P; ++k) {
      I.energies[k] = ebuf[(size_t)i * (P + 1) + k];
      om += ((k == 0 || k == P) ? 1.0 : (k % 2 ? 4.0 : 2.0)) / (3.0 * P) * I.energies[k];
    }
    I.omega_cc = status[i] == 0 ? om : std::nan("");
    I.iters = P;
  }
}

// Reverse-mode sweep: sbar_{n_g} = (g/beta) dE/ds(s_{n_g}); per step p (last first)
//   kbar_x = h b_x sbar_{p+1} + h sum_{y>x} a_yx Z_y,  Z_y = -Delta kbar_y + J_S(Y_y)^T (-kbar_y)
//   sbar_p = sbar_{p+1} + sum_x Z_x   (Z_0 carries (g_p/beta) dE/ds(s_p) as well)
// and the explicit step-length term
//   hbar += <sbar_{p+1}, sum_x b_x k_x> + sum_{x>0} <Z_x, sum_{l<x} a_xl k_l>.
void rk_lambda(ftcc_ctx* c, std::vector<int>& status) {
  const int B = c->B, m = c->m, P = c->P;
  std::vector<bool> ok(B);
  for (int i = 0; i < B; ++i) ok[i] = status[i] == 0;
  set_run(c, ok);
  for (int i = 0; i < B; ++i) zero_d(c, c->inst[i].rk_hbar, 1);
  const auto wall0 = std::chrono::steady_clock::now();
  // final grid point: only the energy term
  rk_stage_state(c, P, 0);
  for (int i = 0; i < B; ++i)
    if (ok[i]) zero_d(c, c->cot[i * m], node_len(c, i));
  set_ebar(c, 0, P);
  backward_one(c, 0);
  for (int i = 0; i < B; ++i)
    if (ok[i]) node_copy(c, i, c->inst[i].abuf[P], c->gr[i * m]);
  for (int p = P - 1; p >= 0; --p) {
    rk_recompute_stages(c, p);
    for (int x = m - 1; x >= 0; --x) {
      rk_combine(c, 2, p, x, +1.0, false, [c, p, x](int i) {
        RKSpec sp;
        const Instance& I = c->inst[i];
        const double h = rk_h(c, i);
        sp.base = I.abuf[p + 1];
        sp.x0 = h * c->rk_b[x];
        for (int y = x + 1; y < c->m; ++y) {
          if (rk_a(c, y, x) == 0.0) continue;
          sp.coef[sp.nst] = h * rk_a(c, y, x);
          sp.Y[sp.nst] = I.lam[p * c->m + y];
          sp.S[sp.nst] = c->gr[i * c->m + y];
          ++sp.nst;
        }
        sp.out = I.lam[p * c->m + x];
        return sp;
      });
      rk_combine(c, 7, p, x, 0.0, false, [c, p, x](int i) {   // cotangent of S at the stage: -kbar
        RKSpec sp;
        sp.base = c->inst[i].lam[p * c->m + x];
        sp.x0 = -1.0;
        sp.out = c->cot[i * c->m + x];
        return sp;
      });
      set_ebar(c, x, x == 0 ? p : -1);
      backward_one(c, x);
    }
    rk_combine(c, 3, p, 0, +1.0, false, [c, p](int i) {
      RKSpec sp;
      const Instance& I = c->inst[i];
      sp.base = I.abuf[p + 1];
      sp.x0 = 1.0;
      for (int x = 0; x < c->m; ++x) {
        sp.coef[sp.nst] = 1.0;
        sp.Y[sp.nst] = I.lam[p * c->m + x];
        sp.S[sp.nst] = c->gr[i * c->m + x];
        ++sp.nst;
      }
      sp.out = I.abuf[p];
      return sp;
    });
    // explicit dependence on the step length
    rk_combine(c, 4, p, 0, -1.0, false, [c](int i) {
      RKSpec sp;
      for (int l = 0; l < c->m; ++l) {
        sp.coef[sp.nst] = c->rk_b[l];
        sp.Y[sp.nst] = c->amp[i * c->m + l];
        sp.S[sp.nst] = c->S[i * c->m + l];
        ++sp.nst;
      }
      sp.out = c->inst[i].rk_tmp[0];
      return sp;
    });
    rk_dot(c, 0, p, 0, [c, p](int i) {
      const Instance& I = c->inst[i];
      return std::array<const double*, 3>{I.abuf[p + 1], I.rk_tmp[0], I.rk_hbar};
    });
    for (int x = 1; x < m; ++x) {
      rk_combine(c, 5, p, x, -1.0, false, [c, x](int i) {
        RKSpec sp;
        for (int l = 0; l < x; ++l) {
          if (rk_a(c, x, l) == 0.0) continue;
          sp.coef[sp.nst] = rk_a(c, x, l);
          sp.Y[sp.nst] = c->amp[i * c->m + l];
          sp.S[sp.nst] = c->S[i * c->m + l];
          ++sp.nst;
        }
        sp.out = c->inst[i].rk_tmp[0];
        return sp;
      });
      rk_combine(c, 6, p, x, +1.0, false, [c, p, x](int i) {
        RKSpec sp;
        const Instance& I = c->inst[i];
        sp.nst = 1;
        sp.coef[0] = 1.0;
        sp.Y[0] = I.lam[p * c->m + x];
        sp.S[0] = c->gr[i * c->m + x];
        sp.out = I.rk_tmp[1];
        return sp;
      });
      rk_dot(c, 1, p, x, [c](int i) {
        const Instance& I = c->inst[i];
        return std::array<const double*, 3>{I.rk_tmp[1], I.rk_tmp[0], I.rk_hbar};
      });
    }
    if (trace_on()) {
      sync(c);
      trace(c, "lambda (Runge-Kutta)", P - p, P, std::vector<int>(1, m), wall0);
    }
  }
  // a reverse pass that produced non-finite cotangents
  reset_maxbits(c);
  rk_combine(c, 8, 0, 0, 0.0, true, [c](int i) {
    RKSpec sp;
    sp.base = c->inst[i].abuf[0];
    sp.x0 = 1.0;
    sp.out = c->inst[i].rk_tmp[1];
    return sp;
  });
  const std::vector<double> mb = read_maxbits(c);
  for (int i = 0; i < B; ++i) {
    if (status[i] == 0 && !std::isfinite(mb[2 * i + 1])) status[i] = FTCC_ENONFINITE;
    c->inst[i].lam_iters = P;
  }
  run_all(c);
}

}  // namespace host
}  // namespace ftcc
