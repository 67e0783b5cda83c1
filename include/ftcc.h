/* FT-CCSD hot path on one AMD Instinct MI355X (gfx950): C ABI.
 *
 * Finite-temperature coupled cluster singles and doubles in the formulation of
 * White and Chan (2020): the grand potential
 *     Omega = Omega_0 + Omega_1 + Omega_CC,  Omega_CC = (1/beta) int_0^beta E[s(tau)] dtau   (eqn:Ecc)
 * with amplitudes s(tau) from the imaginary-time integral equation
 *     s_mu(tau) = -int_0^tau exp(Delta_mu (tau' - tau)) S_mu[s(tau')] dtau'                  (eqn:smu)
 * on thermal integrals scaled by sqrt(n_p) and sqrt(1 - n_p) (Section II.A,
 * Appendix A), the Lambda adjoint of the Lagrangian (eqn:Lagrangian, eqn:lmu,
 * eqn:ltilde) and the response derivatives of Section II.D / Appendix B.
 *
 * Discretisation (Section II.C leaves G open for Gauss-Legendre nodes): [0, beta]
 * is cut into n_tau / nodes_per_panel panels of m = nodes_per_panel Gauss-Legendre
 * nodes; inside a panel the integral equation is collocated at the nodes with
 * the source interpolated by the degree-(m-1) Lagrange polynomial and the
 * exponential integrated exactly (propagator 0), or with the whole integrand
 * interpolated (propagator 1, the paper's G^y_x exp(Delta (tau_x - tau_y))).
 * The implicit panel system is solved by fixed-point (Picard) sweeps.
 *
 * Differential form (Algorithm alg:diff; propagators 2, 3, 4): the amplitudes
 * obey ds/dtau = -(Delta s + S[s]) (eqn:smud) from s(0) = 0 and are stepped
 * across the uniform grid tau_k = k beta / n_tau (k = 0..n_tau) by an explicit
 * Runge-Kutta method (2: forward Euler, 3: explicit trapezoid (Heun), 4: the
 * classical fourth-order method); Omega_CC uses Simpson's rule on the same grid
 * (Section III, Table tab:numerr).  Lambda is the reverse-mode adjoint of the
 * explicit march, and the response derivatives are those of the discrete
 * Omega.  No fixed-point iteration is involved (tol, max_iter, diis_depth and
 * checkpoint do not apply; every grid state is kept).
 *
 * The reference is spin-restricted by default: h, <pq|rs> and eps are spatial,
 * amplitudes are closed-shell t1[i][a] = s_{i alpha}^{a alpha} and
 * t2[i][j][a][b] = s_{i alpha, j beta}^{a alpha, b beta}.  With
 * spin_orbital = 1 every array is over spin orbitals and the amplitudes are
 * the paper's spin-orbital s_i^a, s_ij^ab (unrestricted references).
 *
 * Conventions of every entry point
 *   - return 0 on success, a negative FTCC_E* code on failure; the message of
 *     the last failure on the calling thread is ftcc_last_error();
 *   - pointer arguments are HOST memory owned by the caller, read or written
 *     only during the call; the library keeps its own device copies;
 *   - a context owns all device memory it allocates and frees it in ftcc_destroy
 *     (through the caller's allocator when ftcc_set_allocator installed one);
 *   - one context must not be used by two threads at once;
 *   - required order: create -> set_hamiltonian (every instance) ->
 *     solve_amplitudes -> grand_potential -> lambda -> response.
 *     set_hamiltonian invalidates amplitudes and Lambda.
 *   - a GPU that is missing or not gfx950 is an error (FTCC_EDEVICE); there is
 *     no CPU fallback.
 */
#ifndef FTCC_H
#define FTCC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FTCC_ABI_VERSION 4

#define FTCC_OK 0
#define FTCC_EINVAL -1      /* bad argument */
#define FTCC_ESTATE -2      /* wrong call order */
#define FTCC_ENOMEM -3      /* device allocation failed */
#define FTCC_EDEVICE -4     /* HIP runtime error or unsupported device */
#define FTCC_ENOCONV -5     /* an instance hit max_iter (per-instance status) */
#define FTCC_ENONFINITE -6  /* NaN or Inf in the amplitudes (per-instance status) */

typedef struct ftcc_ctx ftcc_ctx;

typedef struct {
  int n_tau;            /* total imaginary-time nodes n_g (multiple of nodes_per_panel); for the
                           differential form the number of steps (even, >= 2) */
  int nodes_per_panel;  /* m, 1..6 (integral form only) */
  int propagator;       /* 0: exponential collocation, 1: integrating factor (Lawson),
                           2 / 3 / 4: differential form with RK1 / RK2 / RK4 and Simpson's rule */
  double occ_thresh;    /* Section III.A: hole slot kept if n_p > thr, particle slot if 1 - n_p > thr */
  double tol;           /* Picard stop: max|change| <= tol * max(1, max|s|) over the panel */
  int max_iter;         /* Picard sweeps per panel */
  int checkpoint;       /* 0: keep every node; 1: keep panel-start states only and
                           recompute each panel in the adjoint (HBM checkpointing) */
  int diis_depth;       /* 0: plain fixed-point sweeps; 2..8: DIIS (Anderson) extrapolation over
                           this many sweeps, forward and adjoint (needs 2 * depth * m * (n^2 + n^4)
                           doubles per instance) */
  size_t mem_cap_bytes; /* 0: no cap.  Otherwise an upper bound on the device memory the context
                           allocates; the schedule is chosen to fit it: checkpointing is switched
                           on when the stored tau grid would take more than half the cap, and the
                           nodes of a panel share one executor slot when the per-node working set
                           would not fit.  An allocation beyond the cap fails with FTCC_ENOMEM. */
  int spin_orbital;     /* 0: spin-restricted spatial orbitals (closed-shell amplitudes);
                           1: general spin orbitals (unrestricted references such as the Neel
                           state or UHF, Section IV.A): h is N x N, <pq|rs> N^4 over spin orbitals
                           (zero between different spins as the Hamiltonian makes them), eps N,
                           amplitudes t1[i][a], t2[i][j][a][b] antisymmetric in (i,j) and (a,b);
                           Omega_0 and Omega_1 count one electron per orbital */
} ftcc_options;

/* Defaults: n_tau 16, m 4, propagator 0, thr 0, tol 1e-12, max_iter 200, checkpoint 0, diis_depth 0,
 * mem_cap_bytes 0, spin_orbital 0. */
void ftcc_default_options(ftcc_options* opt);

/* Create a context for n_instances independent (Hamiltonian, mu, beta) problems
 * on HIP device `device`.  opt may be NULL (defaults).  All instances share the
 * options and are advanced together (one grouped launch per step). */
int ftcc_create(ftcc_ctx** ctx, int device, int n_instances, const ftcc_options* opt);
int ftcc_destroy(ftcc_ctx* ctx);

/* Run all device work on this hipStream_t (NULL: the context's own stream).
 * The stream must stay valid until it is replaced or the context destroyed. */
int ftcc_set_stream(ftcc_ctx* ctx, void* hip_stream);

/* Device memory supplier for the context's bulk buffers (integrals, amplitudes,
 * residuals, intermediates, Lambda), e.g. a framework's caching allocator.
 *   alloc(bytes, user) returns device memory on the context's device, usable
 *   from its stream, or NULL (reported as FTCC_ENOMEM);
 *   free(ptr, user) is called once for every pointer alloc returned, in
 *   ftcc_destroy (free may be NULL when the caller reclaims the memory itself).
 * Must be called before the first ftcc_set_hamiltonian (FTCC_ESTATE otherwise).
 * NULL alloc restores hipMalloc / hipFree.  Launch descriptors (a few KB) are
 * always the library's own hipMalloc. */
typedef void* (*ftcc_alloc_fn)(size_t bytes, void* user);
typedef void (*ftcc_free_fn)(void* ptr, void* user);
int ftcc_set_allocator(ftcc_ctx* ctx, ftcc_alloc_fn alloc, ftcc_free_fn free_fn, void* user);

/* Crystal momentum of the orbitals of instance `inst` (plane waves of the
 * electron gas, Bloch orbitals of a ring): orbital p carries the integer
 * vector labels[p * dims + c], c < dims <= 3, component c compared modulo
 * modulus[c] when modulus[c] > 0 (e.g. k mod L on an L-site ring), |label| <
 * 65536.  When every instance has labels, every two-operand contraction of the
 * residual, of its reverse and of the response runs over its momentum-allowed
 * blocks only: an amplitude s_{ij..}^{ab..} or integral <pq|rs> is nonzero only
 * when k_i + k_j = k_a + k_b (the translation invariance that Section II.D
 * notes for the electron gas), which removes all but 1/36 (6-site ring) to
 * 1/1e5 (123 plane waves) of the dense O(n^6) work.  h, <pq|rs> and any
 * response direction must vanish where the labels forbid (checked on the
 * device when the plan is built or the direction is passed: FTCC_EINVAL).
 * Must be called before the first solve; labels are copied. */
int ftcc_set_momentum(ftcc_ctx* ctx, int inst, int n, int dims, const int* labels, const int* modulus);

/* Instance `inst` (0 <= inst < n_instances) with n spatial orbitals:
 *   h    n*n row-major one-body matrix (reference orbital basis)
 *   eri  n^4 row-major <pq|rs> = int phi_p*(1) phi_q*(2) r12^-1 phi_r(1) phi_s(2);
 *        real, with <pq|rs> = <qp|sr> (plane waves and Bloch waves need not
 *        satisfy the real-orbital symmetry <pq|rs> = <rq|ps>)
 *   eps  n reference orbital energies (H_0 = sum_p eps_p a_p^+ a_p, Section II.B)
 * Instances may have different n; every step is one grouped launch over all of them. */
int ftcc_set_hamiltonian(ftcc_ctx* ctx, int inst, int n, const double* h, const double* eri, const double* eps);

/* Thermal integrals for (mu[i], beta[i]) and the forward imaginary-time march
 * (Algorithm alg:int in panels).  iters_out[i]: total Picard sweeps of instance
 * i; status_out[i]: 0, FTCC_ENOCONV or FTCC_ENONFINITE.  Either output may be
 * NULL.  Returns FTCC_ENOCONV / FTCC_ENONFINITE if any instance failed. */
int ftcc_solve_amplitudes(ftcc_ctx* ctx, const double* mu, const double* beta, int* iters_out, int* status_out);

/* omega[i] = Omega; parts (optional, [n_instances][3]) = Omega_0, Omega_1, Omega_CC. */
int ftcc_grand_potential(ftcc_ctx* ctx, double* omega, double* parts);

/* Converged amplitudes of node k (0 <= k < n_tau) of one instance: t1 n*n, t2 n^4.
 * Needs checkpoint == 0.  Differential form: the grid state s(tau_k), 0 <= k <= n_tau. */
int ftcc_get_amplitudes(ftcc_ctx* ctx, int inst, int node, double* t1, double* t2);

/* The Lambda adjoint, swept backward in tau panel by panel (stationarity of the
 * discrete Lagrangian; lambda_x = -L[s(tau_x), lambda-tilde(tau_x)] with
 * lambda-tilde the discrete eqn:ltilde).  Same output conventions as solve. */
int ftcc_lambda(ftcc_ctx* ctx, int* iters_out, int* status_out);

/* Lambda and lambda-tilde of node k of one instance (n*n then n^4 each).
 * Differential form: lam = the cotangent dOmega_CC/ds(tau_k) of the grid state
 * (0 <= k <= n_tau) and lamt must be NULL. */
int ftcc_get_lambda(ftcc_ctx* ctx, int inst, int node, double* lam1, double* lam2, double* lamt1, double* lamt2);

/* Derivatives of Omega at a frozen reference (orbitals, eps and the dropped
 * slots fixed; Section II.D types 1, 2, 4, 5, 6 for this discretisation):
 *   dO_dmu[i], dO_dbeta[i]   (either may be NULL)
 *   dO_dh                    dOmega/dh_pq of every instance, n_i*n_i row-major blocks one after
 *                            the other in instance order (sum_i n_i^2 doubles), or NULL
 *   deri_dtheta, dh_dtheta   optional direction of a scalar parameter theta per
 *                            instance (arrays of n_instances host pointers to n^4
 *                            and n*n arrays; an entry may be NULL), e.g.
 *                            deri = eri / U for theta = U; result in dO_dtheta[i]. */
int ftcc_response(ftcc_ctx* ctx, double* dO_dmu, double* dO_dbeta, double* dO_dh,
                  const double* const* deri_dtheta, const double* const* dh_dtheta, double* dO_dtheta);

/* Two-body response density (Section II.D / Appendix B, the response of Omega
 * to the two-electron integrals; the N-particle density Gamma_N): for every
 * instance Gamma_pqrs = dOmega/d<pq|rs> at a frozen reference (orbitals, eps,
 * dropped slots), taken within the integrals that keep <pq|rs> = <qp|sr> (the
 * average of an element and its exchange partner), so that for any direction
 * deri of that kind sum_pqrs Gamma_pqrs deri_pqrs = dOmega/dtheta of
 * ftcc_response.  Includes the mean-field part and the dependence through the
 * Fock operator.  gamma: n_i^4 row-major blocks one after the other in instance
 * order (NaN for an instance whose march or adjoint failed).  Needs
 * ftcc_lambda; builds a third executor on first use (gradient buffers for
 * every integral block per executor slot, 12 n^4 accumulators per instance). */
int ftcc_two_body_density(ftcc_ctx* ctx, double* gamma);

/* Fixed electron number (Section III fixes <N> = 14 for the electron gas this
 * way; the appendix on the UEG basis-set error chooses mu_CC so that the
 * coupled-cluster system holds N electrons): for every instance, the chemical
 * potential at which N = -dOmega/dmu (Section II.D, the mu response at a frozen
 * reference) equals n_target[i] to |N - n_target| <= tol * max(1, |n_target|).
 *   mu_inout  start values in, solutions out;  beta  fixed inverse temperatures
 *   n_out     optional: N at the returned mu
 *   max_iter  evaluations of N per instance; each is a forward march, the
 *             Lambda adjoint and the mu response of the whole batch
 * Bracketing from the start value in steps set by the mean-field
 * compressibility 2 beta sum_p n_p (1 - n_p), then regula falsi (Illinois).
 * status_out[i]: 0, FTCC_ENOCONV (max_iter reached) or the status of a failed
 * march.  On return the context holds the amplitudes and Lambda at the
 * returned mu of every instance with status 0, so grand_potential and
 * response need no new solve. */
int ftcc_find_mu(ftcc_ctx* ctx, const double* n_target, double* mu_inout, const double* beta, double tol,
                 int max_iter, double* n_out, int* iters_out, int* status_out);

/* One evaluation of the kernels E, S1, S2 (eqn:E, eqn:ccS1, eqn:ccS2) of instance
 * `inst` at the given amplitudes and the thermal integrals of (mu, beta):
 * t1, S1 n*n; t2, S2 n^4; E scalar.  With momentum labels, amplitudes with
 * nonzero elements that the labels forbid are rejected (FTCC_EINVAL). */
int ftcc_eval_residual(ftcc_ctx* ctx, int inst, double mu, double beta, const double* t1, const double* t2,
                       double* S1, double* S2, double* E);

/* Timing of the kernels alone: evaluate S for every node slot of every
 * instance `reps` times at the amplitudes currently in the slots (after
 * ftcc_eval_residual or a solve) on device-resident data, between HIP events.
 * seconds_out: elapsed seconds; flops_out: algorithmic GEMM flops per sweep
 * (all slots).  Either may be NULL. */
int ftcc_time_residual(ftcc_ctx* ctx, int reps, double* seconds_out, double* flops_out);

/* HIP-event timing of the dominant kernel (the 128x128 FP64-MFMA GEMM tile
 * configuration, which carries the O(n^6) contractions) on the context's
 * stream.  Returns the algorithmic flops (sum of 2*M*N*K), the summed launch
 * durations and the launch count accumulated since the previous call, then
 * resets the counters and enables (enable != 0) or disables recording. */
int ftcc_kernel_profile(ftcc_ctx* ctx, int enable, double* flops, double* seconds, long* launches);

/* Counters of the last solve / lambda: residual evaluations (instance x node),
 * backward evaluations, and device seconds spent in each phase. */
int ftcc_stats(ftcc_ctx* ctx, long* resid_evals, long* vjp_evals, double* solve_seconds, double* lambda_seconds);

const char* ftcc_last_error(void);
int ftcc_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FTCC_H */
