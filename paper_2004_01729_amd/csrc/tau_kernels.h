// Imaginary-time kernels: thermal integral blocks and the panel propagator.
#pragma once
#include <hip/hip_runtime.h>

namespace ftcc {

constexpr int kMaxNodes = 6;

// Panel quadrature shared by all instances: m Gauss-Legendre nodes c_x on [0,1],
// weights b_x, and the monomial coefficients of the Lagrange basis,
// l_y(u) = sum_k lc[y][k] u^k.
struct PanelRule {
  int m;
  int lawson;               // 0: exponential collocation, 1: integrating factor
  double c[kMaxNodes];
  double b[kMaxNodes];
  double lc[kMaxNodes][kMaxNodes];
  double A[kMaxNodes][kMaxNodes];   // int_0^{c_x} l_y(u) du (Lawson)
  // gc[x][y][k] = lc[y][k] c_x^(k+1) k!  (x = m: the panel end, c = 1), so that
  // W_xy = h sum_k gc[x][y][k] phi_{k+1}(-D h c_x)
  double gc[kMaxNodes + 1][kMaxNodes][kMaxNodes];
};

enum TauMode {
  TAU_INIT = 0,     // s_x = E_x s_b
  TAU_STEP = 1,     // s_x = E_x s_b - sum_y W_xy S_y   (+ max|change|, max|s|)
  TAU_END = 2,      // out = E_e s_b - sum_y We_y S_y
  TAU_LAMT = 3,     // s_x (lambda tilde) = sum_y W_yx S_y (lambda) + We_x s_b (a)
  TAU_APREV = 4,    // out = E_e s_b (a) + sum_x E_x S_x (lambda)
  TAU_BETA = 5,     // partial += sum_x <S_x(lam), -dE_x sb + sum_y dW_xy R_y> + <a, -dEe sb + sum dWe_y R_y>
  TAU_LSTEP = 6,    // s_x (lambda) = -R_x (gradient), with max|change|, max|lambda|
};

// One amplitude segment of one instance (t1: n^2 elements, t2: n^4 elements).
struct TauProblem {
  const double* eps;
  int n;
  int rank;           // 2 or 4
  long len;
  double h;           // panel width beta / P
  const double* sb;   // panel-start state s_b (or adjoint a_{p+1})
  const double* S[kMaxNodes];   // residuals (or lambda)
  const double* R[kMaxNodes];   // residuals for TAU_BETA / gradients for TAU_LSTEP
  double* s[kMaxNodes];         // node amplitudes (or lambda-tilde / lambda)
  double* out;                  // end state / previous adjoint state
  const double* lam_a;          // a_{p+1} for TAU_BETA
  unsigned long long* maxbits;  // [0] max |change|, [1] max |value| (bit patterns of doubles >= 0)
  const int* active;            // STEP / LSTEP: instance still iterating (nullptr: always)
  double* partial;              // TAU_BETA: one partial sum per block
  const unsigned* idx;          // optional: the elements to visit (momentum-allowed ones), len of them;
                                // nullptr: every element 0..len-1
};

// blocks: 1024 elements each, per problem; d_rule is a device copy of the rule
void launch_tau(const PanelRule* d_rule, int m, int mode, const TauProblem* d_probs, const int* d_prefix, int n_prob,
                int total_blocks, hipStream_t s);
hipError_t init_tau_constants();

// Explicit Runge-Kutta march of the differential form (Algorithm alg:diff,
// eqn:smud: ds/dtau = -(Delta s + S[s])) and its reverse: one combination per
// amplitude segment,
//   out = x0 * base + sum_l coef[l] * (-Delta * Y_l + sigma * S_l)
// with Delta the segment's orbital-energy difference.  sigma = -1 makes the
// terms the slopes k_l = -(Delta Y_l + S_l) (stage states, step end);
// sigma = +1 the reverse-mode terms -Delta kbar_l + g_l (g the residual VJP).
// Null base / Y_l / S_l read as zero.  maxbits (optional) receives max |out|.
constexpr int kMaxStages = 4;
struct RKProblem {
  const double* eps;
  int n;
  int rank;                      // 2 or 4
  long len;                      // elements to visit
  const unsigned* idx;           // optional allowed-element list (len entries)
  const double* base;
  double x0;
  int nst;
  double coef[kMaxStages];
  const double* Y[kMaxStages];
  const double* S[kMaxStages];
  double sigma;
  double* out;
  unsigned long long* maxbits;
  const int* active;             // instance runs (nullptr: always)
};
// blocks: 1024 elements each, per problem
void launch_rk_combine(const RKProblem* d_probs, const int* d_prefix, int n_prob, int total_blocks, hipStream_t s);

// dst[o] = src[o] for the element offsets o of a node state listed in a (the t1
// block, na entries) and, shifted by `second`, in b (the t2 block, nb entries):
// the copy of a node state whose other elements are zero in both buffers.
void launch_copy_listed(const unsigned* a, long na, const unsigned* b, long nb, long second, const double* src,
                        double* dst, hipStream_t s);

// Thermal quantities of one instance.
struct ThermalProblem {
  int n;
  const double* eps;
  const double* h;     // n x n
  const double* eri;   // n^4, <pq|rs>
  double mu, beta, thr;
  double g;            // electrons per orbital and occupation: 2 (spatial, restricted), 1 (spin orbitals)
  double* occ;         // n_p
  double* wo;          // sqrt(n_p) or 0 when dropped
  double* wv;          // sqrt(1 - n_p) or 0 when dropped
  double* fock;        // n x n
};
void launch_thermal(const ThermalProblem& p, hipStream_t s);

// out[p,q,r,s] = sum over the product rule of prod_k w_k(slot) * base:
//   out = (prod w) * dbase + sum_k (prod_{j != k} w_j) dw_k * base
// For plain blocks pass dbase = base and dw = nullptr.
struct BlockSpec {
  int n;
  int rank;            // 2 or 4
  char pat[4];         // 'o' or 'v' per slot
  const double* base;  // unweighted tensor
  const double* dbase; // derivative of the unweighted tensor (may equal base)
  const double* wo;
  const double* wv;
  const double* dwo;   // may be nullptr
  const double* dwv;
  double* out;
  // optional list of the elements to compute (the others stay as they are: zero);
  // rank 4 only
  const unsigned* idx = nullptr;
  long count = 0;
};
void launch_block(const BlockSpec& b, hipStream_t s);

// u = f - diag(eps) and its derivative du = dh + J[dn] + dJ[n], with the Fock
// operator f_pq = h_pq + sum_r (g <pr|qr> - <pr|rq>) n_r (g = 2: spin-restricted
// spatial orbitals, g = 1: spin orbitals)
void launch_fock_deriv(int n, const double* eri, const double* deri, const double* dh, const double* occ,
                       const double* docc, double g, double* du, hipStream_t s);
void launch_u_from_fock(int n, const double* fock, const double* eps, double* u, hipStream_t s);

// DIIS: coefficients for every instance from its Gram matrix (ld x ld, count entries
// valid), then the extrapolated iterate sum_j c_j (X_j + R_j) of one buffer.
constexpr int kMaxDiis = 8;
struct DiisTerms {
  int k;
  const double* coef;
  const double* X[kMaxDiis];
  const double* R[kMaxDiis];
};
void launch_diis_solve(int n_inst, const int* counts, const int* newest, const double* G, int ld, double* coef,
                       hipStream_t s);
void launch_diis_combine(long len, const DiisTerms& t, double* out, hipStream_t s);

// sum of `count` doubles into *out (single block, deterministic)
void launch_sum(const double* x, int count, double* out, hipStream_t s);
// element-wise: y = a * x + b * y over len doubles
void launch_axpby(long len, double a, const double* x, double b, double* y, hipStream_t s);

}  // namespace ftcc
