// The spin-restricted FT-CCSD kernels as a tensor Program.
//
// Amplitudes t1[i,a] = s_{i alpha}^{a alpha} and t2[i,j,a,b] = s_{i alpha, j beta}^{a alpha, b beta};
// every index runs over all n spatial orbitals.  Constants are the thermal
// blocks (Appendix A): u_XY[p,q] = w^X_p w^Y_q (<p|f|q> - delta_pq eps_p) and
// g_XYZW[p,q,r,s] = w^X_p w^Y_q w^Z_r w^W_s <pq|rs>, with w^o = sqrt(n) for hole
// slots and w^v = sqrt(1 - n) for particle slots.
//
// The kernels E (eqn:E), S1 (eqn:ccS1) and S2 (eqn:ccS2) are evaluated through
// intermediates in the manner of the Stanton-Gauss scheme that the paper uses
// (Appendix A, last paragraph), spin-adapted for closed-shell amplitudes.  At
// finite temperature the orbital-energy part of the Fock operator is carried by
// the propagator, so u replaces f and no diagonal is removed from the F
// intermediates.  With tau = t2 + t1 t1 and taut = t2 + t1 t1 / 2:
//
//   F_me  = u_me + t_nf L_mnef                       L_mnef = 2 g_mnef - g_mnfe
//   F_ae  = u_ae - u_me t_ma / 2 + t_mf (2 g_mafe - g_maef) - taut_mnaf L_mnef
//   F_mi  = u_mi + t_ie u_me / 2 + t_ne (2 g_mnie - g_mnei) + taut_inef L_mnef
//   W_mnij = g_mnij + t_je g_mnie + t_ie g_mnej + tau_ijef g_mnef
//   W_abef = g_abef - t_mb g_amef - t_ma g_mbef
//   Z_mbef = g_mbef - t_nb g_mnef
//   W1_mbej = g_mbej + t_jf Z_mbef - t_nb g_mnej + t2_njfb L_mnef / 2 - t2_jnfb g_mnef / 2
//   W3_mbej = -g_mbje - t_jf Z_mbfe + t_nb g_mnje + t2_jnfb g_mnfe / 2
//   X_ijab = g_abij / 2 + t2_ijae (F_be - t_mb F_me / 2) - t2_imab (F_mj + t_je F_me / 2)
//          + tau_mnab W_mnij / 2 + tau_ijef W_abef / 2
//          + (2 t2_imae - t2_imea) W1_mbej + t2_imae W3_mbej + t2_mjae W3_mbei
//          + t_ie (g_abej - t_ma g_mbej) - t_je t_ma g_mbie - t_ma g_mbij
//   S2_ijab = X_ijab + X_jiba
//   S1_ia = u_ai + t_ie F_ae - t_ma F_mi + (2 t2_imae - t2_imea) F_me + t_nf (2 g_nafi - g_naif)
//         + (2 t2_imef - t2_imfe) g_mafe - t2_mnae (2 g_mnie - g_mnei)
//   E = 2 u_ia t_ia + L_ijab tau_ijab
//
// (repeated letters are summed; hole letters i..n, particle letters a..f)
#include "engine.h"

namespace ftcc {

Program build_residual_program() {
  Program P;
  P.tensor("t1", 2, T_INPUT);
  P.tensor("t2", 4, T_INPUT);
  for (const char* u : {"u_oo", "u_ov", "u_vo", "u_vv"}) P.tensor(u, 2, T_CONST);
  for (const char* g : {"g_oooo", "g_ooov", "g_oovo", "g_oovv", "g_ovov", "g_ovvo", "g_ovvv", "g_vovv", "g_vvvv",
                        "g_vvvo", "g_ovoo", "g_vvoo"})
    P.tensor(g, 4, T_CONST);
  for (const char* x : {"L", "Lo3", "Lvo", "Lov3", "tt", "tau", "taut", "T2x", "Wmnij", "Wabef", "Z", "W1", "W3",
                        "P1", "Q2", "X"})
    P.tensor(x, 4, T_INTER);
  for (const char* x : {"Fme", "Fae", "Fmi", "Fpbe", "Fpmj"}) P.tensor(x, 2, T_INTER);
  P.tensor("S1", 2, T_OUTPUT);
  P.tensor("S2", 4, T_OUTPUT);
  P.tensor("E", 0, T_OUTPUT);
  // Conservation laws for crystal momentum: an amplitude s_{i..}^{a..} or an
  // integral <pq|rs> is nonzero only when the momenta of its creation slots sum
  // to those of its annihilation slots.
  P.set_law("t1", {+1, -1});
  P.set_law("t2", {+1, +1, -1, -1});
  for (const char* u : {"u_oo", "u_ov", "u_vo", "u_vv"}) P.set_law(u, {+1, -1});
  for (const char* g : {"g_oooo", "g_ooov", "g_oovo", "g_oovv", "g_ovov", "g_ovvo", "g_ovvv", "g_vovv", "g_vvvv",
                        "g_vvvo", "g_ovoo", "g_vvoo"})
    P.set_law(g, {+1, +1, -1, -1});

  // constant combinations (evaluated once per set of thermal integrals)
  P.set("L", "mnef", 2.0, "g_oovv", "mnef");
  P.add("L", "mnef", -1.0, "g_oovv", "mnfe");
  P.set("Lo3", "mnie", 2.0, "g_ooov", "mnie");
  P.add("Lo3", "mnie", -1.0, "g_oovo", "mnei");
  P.set("Lvo", "nafi", 2.0, "g_ovvo", "nafi");
  P.add("Lvo", "nafi", -1.0, "g_ovov", "naif");
  P.set("Lov3", "mafe", 2.0, "g_ovvv", "mafe");
  P.add("Lov3", "mafe", -1.0, "g_ovvv", "maef");

  // amplitude combinations
  P.set("tt", "ijab", 1.0, "t1", "ia", "t1", "jb");
  P.set("tau", "ijab", 1.0, "t2", "ijab");
  P.add("tau", "ijab", 1.0, "tt", "ijab");
  P.set("taut", "ijab", 1.0, "t2", "ijab");
  P.add("taut", "ijab", 0.5, "tt", "ijab");
  P.set("T2x", "imae", 2.0, "t2", "imae");
  P.add("T2x", "imae", -1.0, "t2", "imea");

  // one-body intermediates
  P.set("Fme", "me", 1.0, "u_ov", "me");
  P.add("Fme", "me", 1.0, "t1", "nf", "L", "mnef");
  P.set("Fae", "ae", 1.0, "u_vv", "ae");
  P.add("Fae", "ae", -0.5, "u_ov", "me", "t1", "ma");
  P.add("Fae", "ae", 1.0, "t1", "mf", "Lov3", "mafe");
  P.add("Fae", "ae", -1.0, "taut", "mnaf", "L", "mnef");
  P.set("Fmi", "mi", 1.0, "u_oo", "mi");
  P.add("Fmi", "mi", 0.5, "t1", "ie", "u_ov", "me");
  P.add("Fmi", "mi", 1.0, "t1", "ne", "Lo3", "mnie");
  P.add("Fmi", "mi", 1.0, "taut", "inef", "L", "mnef");
  P.set("Fpbe", "be", 1.0, "Fae", "be");
  P.add("Fpbe", "be", -0.5, "t1", "mb", "Fme", "me");
  P.set("Fpmj", "mj", 1.0, "Fmi", "mj");
  P.add("Fpmj", "mj", 0.5, "t1", "je", "Fme", "me");

  // two-body intermediates
  P.set("Wmnij", "mnij", 1.0, "g_oooo", "mnij");
  P.add("Wmnij", "mnij", 1.0, "t1", "je", "g_ooov", "mnie");
  P.add("Wmnij", "mnij", 1.0, "t1", "ie", "g_oovo", "mnej");
  P.add("Wmnij", "mnij", 1.0, "tau", "ijef", "g_oovv", "mnef");
  P.set("Wabef", "abef", 1.0, "g_vvvv", "abef");
  P.add("Wabef", "abef", -1.0, "t1", "mb", "g_vovv", "amef");
  P.add("Wabef", "abef", -1.0, "t1", "ma", "g_ovvv", "mbef");
  P.set("Z", "mbef", 1.0, "g_ovvv", "mbef");
  P.add("Z", "mbef", -1.0, "t1", "nb", "g_oovv", "mnef");
  P.set("W1", "mbej", 1.0, "g_ovvo", "mbej");
  P.add("W1", "mbej", 1.0, "t1", "jf", "Z", "mbef");
  P.add("W1", "mbej", -1.0, "t1", "nb", "g_oovo", "mnej");
  P.add("W1", "mbej", 0.5, "t2", "njfb", "L", "mnef");
  P.add("W1", "mbej", -0.5, "t2", "jnfb", "g_oovv", "mnef");
  P.set("W3", "mbej", -1.0, "g_ovov", "mbje");
  P.add("W3", "mbej", -1.0, "t1", "jf", "Z", "mbfe");
  P.add("W3", "mbej", 1.0, "t1", "nb", "g_ooov", "mnje");
  P.add("W3", "mbej", 0.5, "t2", "jnfb", "g_oovv", "mnfe");
  P.set("P1", "abej", 1.0, "g_vvvo", "abej");
  P.add("P1", "abej", -1.0, "t1", "ma", "g_ovvo", "mbej");
  P.set("Q2", "abie", 1.0, "t1", "ma", "g_ovov", "mbie");

  // doubles
  P.set("X", "ijab", 0.5, "g_vvoo", "abij");
  P.add("X", "ijab", 1.0, "t2", "ijae", "Fpbe", "be");
  P.add("X", "ijab", -1.0, "t2", "imab", "Fpmj", "mj");
  P.add("X", "ijab", 0.5, "tau", "mnab", "Wmnij", "mnij");
  P.add("X", "ijab", 0.5, "tau", "ijef", "Wabef", "abef");
  P.add("X", "ijab", 1.0, "T2x", "imae", "W1", "mbej");
  P.add("X", "ijab", 1.0, "t2", "imae", "W3", "mbej");
  P.add("X", "ijab", 1.0, "t2", "mjae", "W3", "mbei");
  P.add("X", "ijab", 1.0, "t1", "ie", "P1", "abej");
  P.add("X", "ijab", -1.0, "t1", "je", "Q2", "abie");
  P.add("X", "ijab", -1.0, "t1", "ma", "g_ovoo", "mbij");
  P.set("S2", "ijab", 1.0, "X", "ijab");
  P.add("S2", "ijab", 1.0, "X", "jiba");

  // singles
  P.set("S1", "ia", 1.0, "u_vo", "ai");
  P.add("S1", "ia", 1.0, "t1", "ie", "Fae", "ae");
  P.add("S1", "ia", -1.0, "t1", "ma", "Fmi", "mi");
  P.add("S1", "ia", 1.0, "T2x", "imae", "Fme", "me");
  P.add("S1", "ia", 1.0, "t1", "nf", "Lvo", "nafi");
  P.add("S1", "ia", 1.0, "T2x", "imef", "g_ovvv", "mafe");
  P.add("S1", "ia", -1.0, "t2", "mnae", "Lo3", "mnie");

  // energy
  P.set("E", "", 2.0, "u_ov", "ia", "t1", "ia");
  P.add("E", "", 1.0, "L", "ijab", "tau", "ijab");
  P.finalize();
  return P;
}

// The general spin-orbital FT-CCSD kernels (unrestricted references: Neel
// state, UHF).  Every index runs over all N spin orbitals; t2 is antisymmetric
// in (i, j) and in (a, b).  The weighted raw blocks g_XYZW of <pq|rs> are
// antisymmetrised once per set of thermal integrals,
//   A_XYZW[pqrs] = w_p w_q w_r w_s (<pq|rs> - <pq|sr>)   (Appendix A's <pq||rs>),
// with <ab|je> = <ba|ej> used for the vvvo block.  The kernels E (eqn:E), S1
// (eqn:ccS1) and S2 (eqn:ccS2) through Stanton-Gauss intermediates, u in place
// of f (the orbital-energy part is carried by the propagator); with
// tau = t2 + P(ab) t1 t1 and taut = t2 + P(ab) t1 t1 / 2:
//   F_me  = u_me + t_nf A_mnef
//   F_ae  = u_ae - u_me t_ma / 2 + t_mf A_mafe - taut_mnaf A_mnef / 2
//   F_mi  = u_mi + t_ie u_me / 2 + t_ne A_mnie + taut_inef A_mnef / 2
//   W_mnij = A_mnij + P(ij) t_je A_mnie + tau_ijef A_mnef / 4
//   W_abef = A_abef - P(ab) t_mb A_amef + tau_mnab A_mnef / 4
//   W_mbej = A_mbej + t_jf A_mbef - t_nb A_mnej - (t2_jnfb / 2 + t_jf t_nb) A_mnef
//   S2_ijab = A_abij + P(ab) t2_ijae (F_be - t_mb F_me / 2) - P(ij) t2_imab (F_mj + t_je F_me / 2)
//           + tau_mnab W_mnij / 2 + tau_ijef W_abef / 2
//           + P(ij) P(ab) (t2_imae W_mbej - t_ie t_ma A_mbej) + P(ij) t_ie A_abej - P(ab) t_ma A_mbij
//   S1_ia = u_ai + t_ie F_ae - t_ma F_mi + t2_imae F_me - t_nf A_naif - t2_imef A_maef / 2 - t2_mnae A_nmei / 2
//   E = u_ia t_ia + A_ijab t2_ijab / 4 + A_ijab t_ia t_jb / 2
// where P(pq) X = X - X(p <-> q).
Program build_spin_orbital_program() {
  Program P;
  P.tensor("t1", 2, T_INPUT);
  P.tensor("t2", 4, T_INPUT);
  for (const char* u : {"u_oo", "u_ov", "u_vo", "u_vv"}) P.tensor(u, 2, T_CONST);
  const char* graw[] = {"g_oooo", "g_ooov", "g_oovo", "g_oovv", "g_ovov", "g_ovvo",
                        "g_ovvv", "g_vovv", "g_vvvv", "g_vvvo", "g_ovoo", "g_vvoo"};
  for (const char* g : graw) P.tensor(g, 4, T_CONST);
  for (const char* x : {"A_oooo", "A_ooov", "A_oovo", "A_oovv", "A_ovov", "A_ovvo", "A_ovvv", "A_vovv", "A_vvvv",
                        "A_vvvo", "A_ovoo", "A_vvoo", "tt", "tau", "taut", "Y", "Wmnij", "Wabef", "Wmbej", "K", "Xa",
                        "Xi", "R", "T3", "T4"})
    P.tensor(x, 4, T_INTER);
  for (const char* x : {"Fme", "Fae", "Fmi", "Fpbe", "Fpmj"}) P.tensor(x, 2, T_INTER);
  P.tensor("S1", 2, T_OUTPUT);
  P.tensor("S2", 4, T_OUTPUT);
  P.tensor("E", 0, T_OUTPUT);
  // conservation laws (crystal momentum and/or S_z of the spin orbitals)
  P.set_law("t1", {+1, -1});
  P.set_law("t2", {+1, +1, -1, -1});
  for (const char* u : {"u_oo", "u_ov", "u_vo", "u_vv"}) P.set_law(u, {+1, -1});
  for (const char* g : graw) P.set_law(g, {+1, +1, -1, -1});

  // antisymmetrised integral blocks (constant per set of thermal integrals)
  P.set("A_oooo", "mnij", 1.0, "g_oooo", "mnij");
  P.add("A_oooo", "mnij", -1.0, "g_oooo", "mnji");
  P.set("A_ooov", "mnie", 1.0, "g_ooov", "mnie");
  P.add("A_ooov", "mnie", -1.0, "g_oovo", "mnei");
  P.set("A_oovo", "mnej", 1.0, "g_oovo", "mnej");
  P.add("A_oovo", "mnej", -1.0, "g_ooov", "mnje");
  P.set("A_oovv", "mnef", 1.0, "g_oovv", "mnef");
  P.add("A_oovv", "mnef", -1.0, "g_oovv", "mnfe");
  P.set("A_ovov", "naif", 1.0, "g_ovov", "naif");
  P.add("A_ovov", "naif", -1.0, "g_ovvo", "nafi");
  P.set("A_ovvo", "mbej", 1.0, "g_ovvo", "mbej");
  P.add("A_ovvo", "mbej", -1.0, "g_ovov", "mbje");
  P.set("A_ovvv", "mafe", 1.0, "g_ovvv", "mafe");
  P.add("A_ovvv", "mafe", -1.0, "g_ovvv", "maef");
  P.set("A_vovv", "amef", 1.0, "g_vovv", "amef");
  P.add("A_vovv", "amef", -1.0, "g_vovv", "amfe");
  P.set("A_vvvv", "abef", 1.0, "g_vvvv", "abef");
  P.add("A_vvvv", "abef", -1.0, "g_vvvv", "abfe");
  P.set("A_vvvo", "abej", 1.0, "g_vvvo", "abej");
  P.add("A_vvvo", "abej", -1.0, "g_vvvo", "baej");
  P.set("A_ovoo", "mbij", 1.0, "g_ovoo", "mbij");
  P.add("A_ovoo", "mbij", -1.0, "g_ovoo", "mbji");
  P.set("A_vvoo", "abij", 1.0, "g_vvoo", "abij");
  P.add("A_vvoo", "abij", -1.0, "g_vvoo", "abji");

  // amplitude combinations
  P.set("tt", "ijab", 1.0, "t1", "ia", "t1", "jb");
  P.set("tau", "ijab", 1.0, "t2", "ijab");
  P.add("tau", "ijab", 1.0, "tt", "ijab");
  P.add("tau", "ijab", -1.0, "tt", "ijba");
  P.set("taut", "ijab", 1.0, "t2", "ijab");
  P.add("taut", "ijab", 0.5, "tt", "ijab");
  P.add("taut", "ijab", -0.5, "tt", "ijba");
  P.set("Y", "jnfb", 0.5, "t2", "jnfb");
  P.add("Y", "jnfb", 1.0, "tt", "jnfb");

  // one-body intermediates
  P.set("Fme", "me", 1.0, "u_ov", "me");
  P.add("Fme", "me", 1.0, "t1", "nf", "A_oovv", "mnef");
  P.set("Fae", "ae", 1.0, "u_vv", "ae");
  P.add("Fae", "ae", -0.5, "u_ov", "me", "t1", "ma");
  P.add("Fae", "ae", 1.0, "t1", "mf", "A_ovvv", "mafe");
  P.add("Fae", "ae", -0.5, "taut", "mnaf", "A_oovv", "mnef");
  P.set("Fmi", "mi", 1.0, "u_oo", "mi");
  P.add("Fmi", "mi", 0.5, "t1", "ie", "u_ov", "me");
  P.add("Fmi", "mi", 1.0, "t1", "ne", "A_ooov", "mnie");
  P.add("Fmi", "mi", 0.5, "taut", "inef", "A_oovv", "mnef");
  P.set("Fpbe", "be", 1.0, "Fae", "be");
  P.add("Fpbe", "be", -0.5, "t1", "mb", "Fme", "me");
  P.set("Fpmj", "mj", 1.0, "Fmi", "mj");
  P.add("Fpmj", "mj", 0.5, "t1", "je", "Fme", "me");

  // two-body intermediates
  P.set("Wmnij", "mnij", 1.0, "A_oooo", "mnij");
  P.add("Wmnij", "mnij", 1.0, "t1", "je", "A_ooov", "mnie");
  P.add("Wmnij", "mnij", -1.0, "t1", "ie", "A_ooov", "mnje");
  P.add("Wmnij", "mnij", 0.25, "tau", "ijef", "A_oovv", "mnef");
  P.set("Wabef", "abef", 1.0, "A_vvvv", "abef");
  P.add("Wabef", "abef", -1.0, "t1", "mb", "A_vovv", "amef");
  P.add("Wabef", "abef", 1.0, "t1", "ma", "A_vovv", "bmef");
  P.add("Wabef", "abef", 0.25, "tau", "mnab", "A_oovv", "mnef");
  P.set("Wmbej", "mbej", 1.0, "A_ovvo", "mbej");
  P.add("Wmbej", "mbej", 1.0, "t1", "jf", "A_ovvv", "mbef");
  P.add("Wmbej", "mbej", -1.0, "t1", "nb", "A_oovo", "mnej");
  P.add("Wmbej", "mbej", -1.0, "Y", "jnfb", "A_oovv", "mnef");

  // doubles
  P.set("Xa", "ijab", 1.0, "t2", "ijae", "Fpbe", "be");
  P.set("Xi", "ijab", 1.0, "t2", "imab", "Fpmj", "mj");
  P.set("K", "abej", 1.0, "t1", "ma", "A_ovvo", "mbej");
  P.set("R", "ijab", 1.0, "t2", "imae", "Wmbej", "mbej");
  P.add("R", "ijab", -1.0, "t1", "ie", "K", "abej");
  P.set("T3", "ijab", 1.0, "t1", "ie", "A_vvvo", "abej");
  P.set("T4", "ijab", 1.0, "t1", "ma", "A_ovoo", "mbij");
  P.set("S2", "ijab", 1.0, "A_vvoo", "abij");
  P.add("S2", "ijab", 1.0, "Xa", "ijab");
  P.add("S2", "ijab", -1.0, "Xa", "ijba");
  P.add("S2", "ijab", -1.0, "Xi", "ijab");
  P.add("S2", "ijab", 1.0, "Xi", "jiab");
  P.add("S2", "ijab", 0.5, "tau", "mnab", "Wmnij", "mnij");
  P.add("S2", "ijab", 0.5, "tau", "ijef", "Wabef", "abef");
  P.add("S2", "ijab", 1.0, "R", "ijab");
  P.add("S2", "ijab", -1.0, "R", "jiab");
  P.add("S2", "ijab", -1.0, "R", "ijba");
  P.add("S2", "ijab", 1.0, "R", "jiba");
  P.add("S2", "ijab", 1.0, "T3", "ijab");
  P.add("S2", "ijab", -1.0, "T3", "jiab");
  P.add("S2", "ijab", -1.0, "T4", "ijab");
  P.add("S2", "ijab", 1.0, "T4", "ijba");

  // singles
  P.set("S1", "ia", 1.0, "u_vo", "ai");
  P.add("S1", "ia", 1.0, "t1", "ie", "Fae", "ae");
  P.add("S1", "ia", -1.0, "t1", "ma", "Fmi", "mi");
  P.add("S1", "ia", 1.0, "t2", "imae", "Fme", "me");
  P.add("S1", "ia", -1.0, "t1", "nf", "A_ovov", "naif");
  P.add("S1", "ia", -0.5, "t2", "imef", "A_ovvv", "maef");
  P.add("S1", "ia", -0.5, "t2", "mnae", "A_oovo", "nmei");

  // energy
  P.set("E", "", 1.0, "u_ov", "ia", "t1", "ia");
  P.add("E", "", 0.25, "A_oovv", "ijab", "t2", "ijab");
  P.add("E", "", 0.5, "A_oovv", "ijab", "tt", "ijab");
  P.finalize();
  return P;
}

}  // namespace ftcc
