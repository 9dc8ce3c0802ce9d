// Plain FP64 CPU oracle for one IMEX step of relativistic radiation MHD under
// the gray M1 closure, with PLM reconstruction (MinMod, MC, VanLeer) and the
// Jacobian-free PVM-int face flux (Lopez-Miralles, Marti & Perucho, CPC,
// arXiv 2212.00370).
//
// TEST INFRASTRUCTURE ONLY. This file is the slow, obviously-correct
// reference that the GPU library is checked against. Only the test suite, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the
// product path never calls it. It shares no source with the GPU library.
// Parity unpinned: the zero-mass-flux branch of the CT upwind rule (upwind).
//
// Every function follows the paper's definitions directly (section or
// equation named in its comment). Where the paper leaves a choice open (the
// primitive-recovery algorithm, the RK2 coefficients, the iteration used for
// the stiff source, floors), the reading taken is stated in the comment.
//
// Floating point: IEEE binary64, no contraction (build with
// -ffp-contract=off), no fast-math. The operation order of every expression
// is the one written below, left to right with the parentheses shown.
//
// Build modes:
//   default            : `real` is double.
//   -DORACLE_COUNT_OPS : `real` is a wrapper that counts + - * / and sqrt,
//                        so the same source yields the algorithmic operation
//                        count of the method (results are bitwise unchanged).

#include <cfloat>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORACLE_COUNT_OPS
struct OpCounts { unsigned long long add, mul, div, sqrt; };
static OpCounts g_ops = {0, 0, 0, 0};
struct real {
  double v;
  real() : v(0.0) {}
  real(double x) : v(x) {}
};
static inline real operator+(real a, real b) { g_ops.add++; return real(a.v + b.v); }
static inline real operator-(real a, real b) { g_ops.add++; return real(a.v - b.v); }
static inline real operator*(real a, real b) { g_ops.mul++; return real(a.v * b.v); }
static inline real operator/(real a, real b) { g_ops.div++; return real(a.v / b.v); }
static inline real operator-(real a) { return real(-a.v); }
static inline bool operator<(real a, real b) { return a.v < b.v; }
static inline bool operator>(real a, real b) { return a.v > b.v; }
static inline bool operator<=(real a, real b) { return a.v <= b.v; }
static inline bool operator>=(real a, real b) { return a.v >= b.v; }
static inline bool operator==(real a, real b) { return a.v == b.v; }
static inline bool operator!=(real a, real b) { return a.v != b.v; }
static inline real rsqrt_(real a) { g_ops.sqrt++; return real(std::sqrt(a.v)); }
static inline double dv(real a) { return a.v; }
static inline bool rfinite(real a) { return std::isfinite(a.v); }
// Operations spent in the Newton phase of the implicit solve (a subset of
// g_ops), for the split of the implicit solve's work between its phases.
static OpCounts g_ops_newton = {0, 0, 0, 0};
struct NewtonPhaseOps {
  OpCounts at_start;
  NewtonPhaseOps() : at_start(g_ops) {}
  ~NewtonPhaseOps() {
    g_ops_newton.add += g_ops.add - at_start.add;
    g_ops_newton.mul += g_ops.mul - at_start.mul;
    g_ops_newton.div += g_ops.div - at_start.div;
    g_ops_newton.sqrt += g_ops.sqrt - at_start.sqrt;
  }
};
#define COUNT_NEWTON_PHASE NewtonPhaseOps newton_phase_ops_
#else
typedef double real;
static inline real rsqrt_(real a) { return std::sqrt(a); }
static inline double dv(real a) { return a; }
static inline bool rfinite(real a) { return std::isfinite(a); }
#define COUNT_NEWTON_PHASE
#endif

static inline real rabs(real a) { return (a < real(0.0)) ? -a : a; }
static inline real rmax(real a, real b) { return (a > b) ? a : b; }
static inline real rmin(real a, real b) { return (a < b) ? a : b; }

// Dual number v + d e with e^2 = 0: carrying d through an evaluation gives
// the directional derivative of the result (forward mode). Constants enter
// with d = 0, and every operation is written on (v, d) pairs so that mixed
// constant-dual expressions are evaluated as dual-dual ones.
struct Dual {
  real v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(real a) : v(a), d(0.0) {}
#ifdef ORACLE_COUNT_OPS
  Dual(double a) : v(a), d(0.0) {}
#endif
  Dual(real a, real b) : v(a), d(b) {}
};
static inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
static inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
static inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
static inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.v * b.d + a.d * b.v); }
static inline Dual operator/(Dual a, Dual b) {
  const real q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
static inline Dual rsqrt_(Dual a) {
  const real r = rsqrt_(a.v);
  return Dual(r, a.d / (real(2.0) * r));
}
static inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
static inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
static inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }

// Variable order. Conserved U and primitive V share slots 5..11 (B, E_r, F_r
// are both primitive and conserved; Section 2.1).
enum { NV = 12 };
// U: 0 D, 1..3 S^j, 4 tau_e, 5..7 B^j, 8 E_r, 9..11 F_r^j
// V: 0 rho, 1..3 v^j, 4 p, 5..7 B^j, 8 E_r, 9..11 F_r^j

extern "C" {
// Parameters (a ctypes mirror lives in oracle.py; keep the order).
struct OPar {
  double gamma;      // ideal-gas adiabatic index (eq. eos)
  double a_rad;      // radiation constant a_R, 4*pi*B = a_R T^4
  double t_coeff;    // T = t_coeff * p / rho (code units, mu m_p / k_B folded in)
  double pvm_eps;    // finite-difference step of the Jacobian-free PVM (1e-8)
  double c2p_tol;    // relative Newton step tolerance of primitive recovery
  double imp_tol;    // relative tolerance of the implicit radiation solve
  double rho_floor;  // state used only when recovery fails (counted)
  double p_floor;
  int pvm_k;         // degree index k of the internal polynomial, deg = 2^k
  int beta_mode;     // 0: beta scales all 12 components; 1: radiation rows only; 2: beta = 1
  int recon;         // 0: Godunov (piecewise constant); PLM with 1: MinMod, 2: MC, 3: VanLeer
  int rk_order;      // 2: SSP-RK2 analogue; 3: the paper's IMEX RK3
  int c2p_maxit;
  int imp_maxit;
  int imp_picard_it; // Picard (lagged) iterations before Newton takes over
  int imp_method;    // 0: Picard then Newton; 1: Newton only; 2: Picard only
  double e_floor;    // > 0: a non-positive explicit E_r is raised to this (counted); 0: failure
  int solver;        // 0: PVM-int (Section 3.2); 1: Rad-HLL (Section 3.2, Radiative HLL);
                     // 2: PVM-int with exact Jacobian-vector products
  int ct;            // 0: cell-centred B; 1: constrained transport (staggered normal B on
                     //    the faces, CT-contact edge EMFs); periodic grids, ndim >= 2
};

struct OGrid {
  int ndim;
  int n[3];
  double dx[3];
  int bc_lo[3], bc_hi[3];        // 0 periodic, 1 outflow, 2 inflow (lo side of last axis)
  long long var_stride;          // elements between variable planes of U
  const double* inflow_U;        // [12][transverse cells] conserved inflow state
  const unsigned char* inflow_mask;  // [transverse cells] 1 = inflow, 0 = outflow
};

struct OReport {
  long long c2p_fail, pvm_fallback, imp_fail, nonfinite, e_floor_hits;
  long long first_bad_cell;
  int max_c2p_it, max_imp_it;
};
}

// ---------------------------------------------------------------------------
// Derived constants of the gamma-law EOS (eq. eos): rho*h = rho + g1*p.
struct Consts {
  double g1;    // gamma / (gamma - 1)
  double gm1g;  // (gamma - 1) / gamma
  double gm1;   // gamma - 1
};
static Consts consts_of(const OPar& P) {
  Consts c;
  c.g1 = P.gamma / (P.gamma - 1.0);
  c.gm1g = (P.gamma - 1.0) / P.gamma;
  c.gm1 = P.gamma - 1.0;
  return c;
}

// ---------------------------------------------------------------------------
// Quantities derived from the primitives (Section 2.1, definitions after
// eqs. eqU/eqF): W, b^0 = W (v.B), b^i = B^i/W + v^i b^0,
// |b|^2 = B^2/W^2 + (v.B)^2, total enthalpy density rho h* = rho h + |b|^2
// (the printed h* carries a typo gamma/rho for p/rho), p* = p + |b|^2/2.
// Templated on the scalar T: `real` for the method itself, Dual (below) for
// the forward-mode derivatives of the exact-JVP variant.
template <class T>
struct AuxT {
  T W, iW, l2;     // Lorentz factor, 1/W, 1/W^2 = 1 - v^2
  T b0, b[3], bb;  // magnetic four-vector components and |b|^2
  T wtot;          // rho h* W^2
  T ps;            // total pressure p*
  T D;             // rho W
};
using Aux = AuxT<real>;

// From l2 = 1 - v^2 and iW = 1/W = sqrt(l2) of the state.
template <class T>
static void prim_aux_lw(const T V[NV], T l2, T iW, const Consts& K, AuxT<T>& a) {
  const T vx = V[1], vy = V[2], vz = V[3];
  a.l2 = l2;
  a.iW = iW;
  a.W = T(1.0) / a.iW;
  const T vB = (vx * V[5] + vy * V[6]) + vz * V[7];
  a.b0 = a.W * vB;
  for (int j = 0; j < 3; ++j) a.b[j] = V[5 + j] * a.iW + V[1 + j] * a.b0;
  const T B2 = (V[5] * V[5] + V[6] * V[6]) + V[7] * V[7];
  a.bb = B2 * a.l2 + vB * vB;
  const T rhoh = V[0] + T(K.g1) * V[4];
  a.wtot = (rhoh + a.bb) * (a.W * a.W);
  a.ps = V[4] + T(0.5) * a.bb;
  a.D = V[0] * a.W;
}

static void prim_aux(const real V[NV], const Consts& K, Aux& a) {
  const real v2 = (V[1] * V[1] + V[2] * V[2]) + V[3] * V[3];
  const real l2 = 1.0 - v2;
  prim_aux_lw(V, l2, rsqrt_(l2), K, a);
}

// Primitive -> conserved map, eq. eqU.
static void p2c(const real V[NV], const Aux& a, real U[NV]) {
  U[0] = a.D;
  for (int j = 0; j < 3; ++j) U[1 + j] = a.wtot * V[1 + j] - a.b0 * a.b[j];
  U[4] = ((a.wtot - a.ps) - a.b0 * a.b0) - a.D;
  for (int q = 5; q < NV; ++q) U[q] = V[q];
}

// M1 closure (Section 2.2, eq. xi): row d of P_r = D_r E_r with
// D_r = (1-xi)/2 delta + (3 xi - 1)/2 n n, n = F/|F|, f = |F|/E,
// xi = (3 + 4 f^2) / (5 + 2 sqrt(4 - 3 f^2)). n n is taken as 0 when F = 0,
// and also when |F|^2 is below the smallest normal double (|F| < 1.5e-154):
// there n n = F F / |F|^2 would divide by an underflowed |F|^2, while its
// weight (3 xi - 1)/2 ~ f^2 is negligible.
static const double kMinNormal = DBL_MIN;
template <class T>
static void m1_row(T E, const T F[3], int d, T P[3]) {
  const T FF = (F[0] * F[0] + F[1] * F[1]) + F[2] * F[2];
  const T f2 = FF / (E * E);
  T t = T(4.0) - T(3.0) * f2;
  t = (t > T(0.0)) ? t : T(0.0);
  const T s = rsqrt_(t);
  const T xi = (T(3.0) + T(4.0) * f2) / (T(5.0) + T(2.0) * s);
  const T ca = T(0.5) * (T(1.0) - xi);
  const T cb = T(0.5) * (T(3.0) * xi - T(1.0));
  if (FF >= T(kMinNormal)) {
    const T iFF = T(1.0) / FF;
    for (int j = 0; j < 3; ++j) {
      const T nn = (F[d] * F[j]) * iFF;
      P[j] = (j == d) ? E * (ca + cb * nn) : E * (cb * nn);
    }
  } else {
    for (int j = 0; j < 3; ++j) P[j] = (j == d) ? E * ca : T(0.0);
  }
}

// Physical flux in direction d, eq. eqF.
template <class T>
static void flux(const T V[NV], const AuxT<T>& a, int d, T F[NV]) {
  const T vd = V[1 + d];
  F[0] = a.D * vd;
  const T wv = a.wtot * vd;
  for (int j = 0; j < 3; ++j) {
    if (j == d) F[1 + j] = (wv * V[1 + j] + a.ps) - a.b[d] * a.b[j];
    else        F[1 + j] = wv * V[1 + j] - a.b[d] * a.b[j];
  }
  F[4] = (wv - a.b0 * a.b[d]) - a.D * vd;
  for (int j = 0; j < 3; ++j) F[5 + j] = vd * V[5 + j] - V[5 + d] * V[1 + j];
  F[8] = V[9 + d];
  m1_row(V[8], &V[9], d, &F[9]);
}

// ---------------------------------------------------------------------------
// Conserved -> primitive recovery of the magnetofluid (Section 3.2 step 2 and
// the implicit step; the paper defers the algorithm to its RMHD code).
// Reading taken: Newton-Raphson on Z = rho h W^2 with a maintained bracket,
// using the closed relations implied by eq. eqU
//   S = (Z + B^2) v - (v.B) B,   v.B = (S.B)/Z,
//   v^2(Z) = [S^2 + (S.B/Z)^2 (2Z + B^2)] / (Z + B^2)^2,
//   tau + D = Z + B^2 - p - B^2/(2 W^2) - (S.B)^2/(2 Z^2),
//   p(Z) = (gamma-1)/gamma (Z/W^2 - D/W).
// f(Z) = Z + B^2 - p - B^2/(2W^2) - (S.B)^2/(2Z^2) - (tau + D).
// Bracket: [D, gamma (tau + D)]; states with v^2 >= 1 or p <= 0 lie below the
// root and are treated as f < 0. A Newton iterate that leaves the bracket
// (or a non-positive slope) is replaced by bisection.
struct C2PIn {
  real D, S[3], B[3], Et, B2, S2, SB;
};

struct C2PEval {
  bool ok;
  real l2, iW, rho, p, vB, iZ, iZb, f, df;
};

static C2PEval c2p_eval(real Z, const C2PIn& in, const Consts& K, bool want_df) {
  C2PEval e;
  const real Zb = Z + in.B2;
  // 1/Z and 1/(Z + B^2) from one reciprocal of the product
  const real rZZb = 1.0 / (Z * Zb);
  const real iZ = Zb * rZZb;
  e.iZ = iZ;
  e.iZb = Z * rZZb;
  e.vB = in.SB * iZ;
  const real vB2 = e.vB * e.vB;
  const real v2 = (in.S2 + vB2 * (Z + Zb)) * (e.iZb * e.iZb);
  e.ok = false;
  if (!(v2 < real(1.0))) return e;
  e.l2 = 1.0 - v2;
  e.iW = rsqrt_(e.l2);
  e.rho = in.D * e.iW;
  e.p = K.gm1g * (Z * e.l2 - e.rho);
  if (!(e.p > real(0.0))) return e;
  e.ok = true;
  if (!want_df) return e;
  const real f = (((Z + in.B2) - e.p) - 0.5 * (in.B2 * e.l2)) - (0.5 * vB2 + in.Et);
  // d(v^2)/dZ = -2 [S^2 + (S.B/Z)^2 (3 Z (Z+B^2) + B^4)/Z] / (Z+B^2)^3
  const real dv2 = -2.0 * (in.S2 + (vB2 * (3.0 * (Z * Zb) + in.B2 * in.B2)) * iZ) *
                   ((e.iZb * e.iZb) * e.iZb);
  // f and f' are returned multiplied by 1/W > 0 (same signs, same Newton
  // quotient), which needs no 1/(1/W):
  //   f'/W = 1/W - [(gamma-1)/gamma] (l2/W + dv2 (D/2 - Z/W))
  //          + (B^2/2) dv2 /W + (S.B)^2/Z^3 /W,
  // from dp/dZ = [(gamma-1)/gamma] (l2 + dv2 (D W/2 - Z)).
  e.f = f * e.iW;
  const real dpw = K.gm1g * (e.l2 * e.iW + dv2 * (0.5 * in.D - Z * e.iW));
  e.df = ((e.iW - dpw) + (0.5 * (in.B2 * dv2)) * e.iW) + (vB2 * iZ) * e.iW;
  return e;
}

// Returns 0 on success. Zguess > 0 warm-starts the iteration (used for the
// intermediate states of the PVM chain and inside the implicit solve); the
// cold start is the rest-frame estimate Z0 = gamma (E - B^2/2) - (gamma-1) D,
// exact for a fluid at rest.
// lw (optional): 1 - v^2 and 1/W of the recovered state, as the final
// evaluation at the converged Z forms them.
static int c2p(const real U[NV], const OPar& P, const Consts& K, real Zguess,
               real V[NV], real* Zout, int* nit, real* lw = nullptr) {
  C2PIn in;
  in.D = U[0];
  for (int j = 0; j < 3; ++j) { in.S[j] = U[1 + j]; in.B[j] = U[5 + j]; }
  in.Et = U[4] + U[0];
  in.B2 = (in.B[0] * in.B[0] + in.B[1] * in.B[1]) + in.B[2] * in.B[2];
  in.S2 = (in.S[0] * in.S[0] + in.S[1] * in.S[1]) + in.S[2] * in.S[2];
  in.SB = (in.S[0] * in.B[0] + in.S[1] * in.B[1]) + in.S[2] * in.B[2];
  for (int q = 5; q < NV; ++q) V[q] = U[q];
  *nit = 0;
  if (!(in.D > real(0.0)) || !rfinite(in.Et) || !rfinite(in.S2) || !rfinite(in.B2)) return 1;
  real lo = in.D;
  real hi = P.gamma * in.Et;
  if (!(hi > lo)) return 1;
  real Z;
  if (Zguess > real(0.0) && Zguess > lo && Zguess < hi) {
    Z = Zguess;
  } else {
    Z = P.gamma * (in.Et - 0.5 * in.B2) - K.gm1 * in.D;
    if (!(Z > lo && Z < hi)) Z = 0.5 * (lo + hi);
  }
  bool conv = false;
  int it = 0;
  while (it < P.c2p_maxit) {
    ++it;
    const C2PEval e = c2p_eval(Z, in, K, true);
    real Zn;
    if (!e.ok) {
      lo = Z;
      Zn = 0.5 * (lo + hi);
    } else {
      if (e.f == real(0.0)) { conv = true; break; }
      if (e.f > real(0.0)) hi = Z; else lo = Z;
      Zn = Z - e.f / e.df;
      if (!(e.df > real(0.0)) || !(Zn > lo && Zn < hi)) Zn = 0.5 * (lo + hi);
    }
    const real dZ = rabs(Zn - Z);
    Z = Zn;
    if (dZ <= P.c2p_tol * Z) { conv = true; break; }
  }
  *nit = it;
  if (!conv) return 2;
  const C2PEval e = c2p_eval(Z, in, K, false);
  if (!e.ok) return 3;
  V[0] = e.rho;
  for (int j = 0; j < 3; ++j) V[1 + j] = (in.S[j] + e.vB * in.B[j]) * e.iZb;
  V[4] = e.p;
  *Zout = Z;
  if (lw) { lw[0] = e.l2; lw[1] = e.iW; }
  return 0;
}

// Recovery failure fallback: a finite state at rest (counted, never silent).
static void c2p_fallback(const real U[NV], const OPar& P, real V[NV]) {
  V[0] = (U[0] > real(0.0)) ? U[0] : real(P.rho_floor);
  V[1] = 0.0; V[2] = 0.0; V[3] = 0.0;
  V[4] = P.p_floor;
  for (int q = 5; q < NV; ++q) V[q] = U[q];
}

// ---------------------------------------------------------------------------
// Coefficients of the internal polynomial approximation of |x| (eq. iterat):
// p_0 = 1, p_k = (2 p_{k-1} - p_{k-1}^2 + x^2)/2. p_k is a polynomial in x^2
// of degree M = 2^(k-1); c[m] multiplies x^(2m). All coefficients are dyadic
// rationals, so this expansion is exact in binary64 for k <= 4.
static int internal_poly(int k, double c[17]) {
  double p[17];
  for (int m = 0; m < 17; ++m) p[m] = 0.0;
  p[0] = 1.0;
  int M = 0;  // degree in x^2
  for (int s = 1; s <= k; ++s) {
    double q[17];
    for (int m = 0; m < 17; ++m) q[m] = 0.0;
    // p^2 (degree 2M in x^2)
    for (int a = 0; a <= M; ++a)
      for (int b = 0; b <= M; ++b) q[a + b] -= p[a] * p[b];
    for (int m = 0; m <= M; ++m) q[m] += 2.0 * p[m];
    q[1] += 1.0;
    for (int m = 0; m < 17; ++m) p[m] = 0.5 * q[m];
    M = (M == 0) ? 1 : 2 * M;
  }
  for (int m = 0; m < 17; ++m) c[m] = p[m];
  return M;
}

// ---------------------------------------------------------------------------
// Jacobian-free PVM-int face flux (Section 3.2, PVM algorithm and eq. beta).
// Y(w) = [F(U_m + F(U_m + eps w) - F(U_m)) - F(U_m)] / eps approximates
// A(U_m)^2 w; Horner's scheme over x^2 gives U_{M} ~ p_k(A) U_0 with
// lambda_max = 1, and F^ = (F_L + F_R)/2 - beta U_M / 2,
// beta = min(1/tau_L, 1/tau_R, 1). If any intermediate recovery fails the face
// falls back to p_0 = 1 (Rusanov with lambda = 1), counted.
struct FaceOut { int fallback; int c2p_it; };

// Recovery of an intermediate state U near U_m, warm-started at Z_m. The
// recovery is a function of the fluid part of U only, so when that part equals
// U_m's bit for bit the known V_m is reused (this makes the chain exact for
// U_0 = 0 and for perturbations that leave the fluid untouched).
static bool recover_near(const real U[NV], const real Um[NV], const real Vm[NV], real Zm,
                         const real lwm[2], const OPar& P, const Consts& K, real V[NV], int* nit,
                         real lw[2]) {
  bool same = true;
  for (int q = 0; q < 8; ++q) same = same && (U[q] == Um[q]);
  if (same) {
    for (int q = 0; q < 5; ++q) V[q] = Vm[q];
    for (int q = 5; q < NV; ++q) V[q] = U[q];
    *nit = 0;
    lw[0] = lwm[0];
    lw[1] = lwm[1];
    return true;
  }
  real Z = 0.0;
  return c2p(U, P, K, Zm, V, &Z, nit, lw) == 0;
}

static void pvm_face(const real VL[NV], const real VR[NV], real tauL, real tauR, int d,
                     const OPar& P, const Consts& K, const double* coef, int M,
                     real Fh[NV], FaceOut& fo) {
  Aux aL, aR;
  prim_aux(VL, K, aL);
  prim_aux(VR, K, aR);
  real UL[NV], UR[NV], FL[NV], FR[NV];
  p2c(VL, aL, UL); flux(VL, aL, d, FL);
  p2c(VR, aR, UR); flux(VR, aR, d, FR);
  real U0[NV], Um[NV];
  for (int q = 0; q < NV; ++q) { U0[q] = UR[q] - UL[q]; Um[q] = 0.5 * (UL[q] + UR[q]); }
  const real beta = 1.0 / rmax(rmax(tauL, tauR), real(1.0));
  fo.fallback = 0;
  fo.c2p_it = 0;
  real Uk[NV];
  bool ok = true;
  if (M == 0) {
    for (int q = 0; q < NV; ++q) Uk[q] = U0[q];
  } else {
    // Fluxes of recovered states take 1 - v^2 and 1/W from the recovery.
    real Vm[NV], Zm = 0.0, lwm[2] = {0.0, 0.0};
    int it = 0;
    if (c2p(Um, P, K, real(0.0), Vm, &Zm, &it, lwm) != 0) ok = false;
    fo.c2p_it += it;
    real Fm[NV];
    if (ok) { Aux am; prim_aux_lw(Vm, lwm[0], lwm[1], K, am); flux(Vm, am, d, Fm); }
    const real ieps = 1.0 / P.pvm_eps;
    real w[NV];
    for (int q = 0; q < NV; ++q) w[q] = U0[q];
    for (int l = 0; l < M && ok; ++l) {
      // Y(w)
      real Ue[NV], Ve[NV], Fe[NV], Ut[NV], Vt[NV], Ft[NV], lwe[2], lwt[2];
      for (int q = 0; q < NV; ++q) Ue[q] = Um[q] + P.pvm_eps * w[q];
      if (!recover_near(Ue, Um, Vm, Zm, lwm, P, K, Ve, &it, lwe)) { ok = false; fo.c2p_it += it; break; }
      fo.c2p_it += it;
      { Aux ae; prim_aux_lw(Ve, lwe[0], lwe[1], K, ae); flux(Ve, ae, d, Fe); }
      for (int q = 0; q < NV; ++q) Ut[q] = Um[q] + (Fe[q] - Fm[q]);
      if (!recover_near(Ut, Um, Vm, Zm, lwm, P, K, Vt, &it, lwt)) { ok = false; fo.c2p_it += it; break; }
      fo.c2p_it += it;
      { Aux at; prim_aux_lw(Vt, lwt[0], lwt[1], K, at); flux(Vt, at, d, Ft); }
      const real cnext = coef[M - 1 - l];
      if (l == 0) {
        const real ctop = coef[M];
        for (int q = 0; q < NV; ++q) w[q] = ctop * ((Ft[q] - Fm[q]) * ieps) + cnext * U0[q];
      } else {
        for (int q = 0; q < NV; ++q) w[q] = (Ft[q] - Fm[q]) * ieps + cnext * U0[q];
      }
    }
    if (ok) {
      for (int q = 0; q < NV; ++q) Uk[q] = w[q];
    } else {
      fo.fallback = 1;
      for (int q = 0; q < NV; ++q) Uk[q] = U0[q];
    }
  }
  for (int q = 0; q < NV; ++q) {
    const real bq = (P.beta_mode == 2 || (P.beta_mode == 1 && q < 8)) ? real(1.0) : beta;
    Fh[q] = 0.5 * (FL[q] + FR[q]) - 0.5 * (bq * Uk[q]);
  }
}

// ---------------------------------------------------------------------------
// Exact-JVP variant of the PVM-int flux. The polynomial viscosity p_k(A) U_0
// of eq. utilde is evaluated with the same Horner scheme in A^2, but each
// product A w = (dF/dU)(U_m) w is the exact directional derivative of
// U -> F(V(U)) at U_m, taken in forward mode (Dual), instead of the nested
// finite differences with step eps of eq. iterat. The recovery V(U) is
// differentiated implicitly: at its converged Z, the residual
//   f(Z; U) = (Z + B^2) - p - B^2 (1 - v^2)/2 - (S.B/Z)^2/2 - (tau + D)
// (the closed relations of eq. eqU, as in c2p_eval, not scaled) gives
//   dZ = -(df/dU . w) / (df/dZ),
// and V follows from Z by the same closed relations:
//   v = (S + (S.B/Z) B)/(Z + B^2), 1 - v^2, 1/W = sqrt(1 - v^2),
//   rho = D/W, p = (gamma-1)/gamma (Z (1 - v^2) - rho).
// The radiation rows need no recovery (E_r, F_r are conserved and primitive).
// A recovery failure at U_m drops the face to p_0 = 1, as in pvm_face.
struct C2PInD {
  Dual D, S[3], B[3], Et, B2, S2, SB;
};

static C2PInD c2p_in_dual(const real U[NV], const real w[NV]) {
  C2PInD in;
  in.D = Dual(U[0], w[0]);
  for (int j = 0; j < 3; ++j) {
    in.S[j] = Dual(U[1 + j], w[1 + j]);
    in.B[j] = Dual(U[5 + j], w[5 + j]);
  }
  in.Et = Dual(U[4], w[4]) + in.D;
  in.B2 = (in.B[0] * in.B[0] + in.B[1] * in.B[1]) + in.B[2] * in.B[2];
  in.S2 = (in.S[0] * in.S[0] + in.S[1] * in.S[1]) + in.S[2] * in.S[2];
  in.SB = (in.S[0] * in.B[0] + in.S[1] * in.B[1]) + in.S[2] * in.B[2];
  return in;
}

// V (fluid part, with B), 1 - v^2 and 1/W from Z; and the residual f.
static Dual c2p_closed(Dual Z, const C2PInD& in, const Consts& K, Dual V[NV], Dual& l2, Dual& iW) {
  const Dual vB = in.SB / Z;
  const Dual iZb = Dual(1.0) / (Z + in.B2);
  const Dual v2 = (in.S2 + (vB * vB) * (Z + (Z + in.B2))) * (iZb * iZb);
  l2 = Dual(1.0) - v2;
  iW = rsqrt_(l2);
  const Dual rho = in.D * iW;
  const Dual p = Dual(K.gm1g) * (Z * l2 - rho);
  V[0] = rho;
  for (int j = 0; j < 3; ++j) V[1 + j] = (in.S[j] + vB * in.B[j]) * iZb;
  V[4] = p;
  for (int j = 0; j < 3; ++j) V[5 + j] = in.B[j];
  return (((Z + in.B2) - p) - Dual(0.5) * (in.B2 * l2)) - (Dual(0.5) * (vB * vB) + in.Et);
}

// df/dZ at the converged Z of U_m.
static real c2p_dfdZ(const real Um[NV], real Zm, const Consts& K) {
  real zero[NV];
  for (int q = 0; q < NV; ++q) zero[q] = 0.0;
  const C2PInD in = c2p_in_dual(Um, zero);
  Dual V[NV], l2, iW;
  return c2p_closed(Dual(Zm, real(1.0)), in, K, V, l2, iW).d;
}

// A w at U_m (all 12 rows) in direction d.
static void jvp_flux(const real Um[NV], real Zm, real fZ, const real w[NV], int d, const Consts& K,
                     real Aw[NV]) {
  const C2PInD in = c2p_in_dual(Um, w);
  Dual V[NV], l2, iW;
  const real fU = c2p_closed(Dual(Zm), in, K, V, l2, iW).d;
  const real dZ = -(fU / fZ);
  c2p_closed(Dual(Zm, dZ), in, K, V, l2, iW);
  for (int q = 8; q < NV; ++q) V[q] = Dual(Um[q], w[q]);
  AuxT<Dual> a;
  prim_aux_lw(V, l2, iW, K, a);
  Dual F[NV];
  flux(V, a, d, F);
  for (int q = 0; q < NV; ++q) Aw[q] = F[q].d;
}

static void pvm_face_jvp(const real VL[NV], const real VR[NV], real tauL, real tauR, int d,
                         const OPar& P, const Consts& K, const double* coef, int M,
                         real Fh[NV], FaceOut& fo) {
  Aux aL, aR;
  prim_aux(VL, K, aL);
  prim_aux(VR, K, aR);
  real UL[NV], UR[NV], FL[NV], FR[NV];
  p2c(VL, aL, UL); flux(VL, aL, d, FL);
  p2c(VR, aR, UR); flux(VR, aR, d, FR);
  real U0[NV], Um[NV];
  for (int q = 0; q < NV; ++q) { U0[q] = UR[q] - UL[q]; Um[q] = 0.5 * (UL[q] + UR[q]); }
  const real beta = 1.0 / rmax(rmax(tauL, tauR), real(1.0));
  fo.fallback = 0;
  fo.c2p_it = 0;
  real Uk[NV];
  for (int q = 0; q < NV; ++q) Uk[q] = U0[q];
  if (M > 0) {
    real Vm[NV], Zm = 0.0;
    int it = 0;
    if (c2p(Um, P, K, real(0.0), Vm, &Zm, &it) != 0) {
      fo.fallback = 1;
    } else {
      const real fZ = c2p_dfdZ(Um, Zm, K);
      real w[NV], t1[NV], t2[NV];
      for (int q = 0; q < NV; ++q) w[q] = U0[q];
      for (int l = 0; l < M; ++l) {
        jvp_flux(Um, Zm, fZ, w, d, K, t1);
        jvp_flux(Um, Zm, fZ, t1, d, K, t2);
        const real cnext = coef[M - 1 - l];
        if (l == 0) {
          const real ctop = coef[M];
          for (int q = 0; q < NV; ++q) w[q] = ctop * t2[q] + cnext * U0[q];
        } else {
          for (int q = 0; q < NV; ++q) w[q] = t2[q] + cnext * U0[q];
        }
      }
      for (int q = 0; q < NV; ++q) Uk[q] = w[q];
    }
    fo.c2p_it = it;
  }
  for (int q = 0; q < NV; ++q) {
    const real bq = (P.beta_mode == 2 || (P.beta_mode == 1 && q < 8)) ? real(1.0) : beta;
    Fh[q] = 0.5 * (FL[q] + FR[q]) - 0.5 * (bq * Uk[q]);
  }
}

// ---------------------------------------------------------------------------
// PLM reconstruction (Section 3.2, reconstruction paragraph: MinMod, MC or
// VanLeer slopes). With a = V_i - V_{i-1} and b = V_{i+1} - V_i, every limiter
// gives 0 unless a and b share a sign, and then
//   MinMod   (Roe):        a or b, whichever is smaller in magnitude;
//   MC       (van Leer 77): the smallest in magnitude of 2a, 2b, (a + b)/2;
//   VanLeer  (van Leer 74): the harmonic form 2ab / (a + b).
// A cell whose reconstructed face values give |v|^2 >= 1 falls back to zeroth
// order on both of its faces. After reconstruction the face radiation flux is
// limited to |F_r| <= E_r by rescaling.
static inline bool same_sign(real a, real b) {
  return (a > real(0.0) && b > real(0.0)) || (a < real(0.0) && b < real(0.0));
}

static inline real minmod(real a, real b) {
  if (same_sign(a, b)) return (rabs(a) < rabs(b)) ? a : b;
  return real(0.0);
}

static inline real mc_slope(real a, real b) {
  if (!same_sign(a, b)) return real(0.0);
  const real ta = real(2.0) * a, tb = real(2.0) * b, c = real(0.5) * (a + b);
  const real m = (rabs(ta) < rabs(tb)) ? ta : tb;
  return (rabs(c) < rabs(m)) ? c : m;
}

static inline real vanleer_slope(real a, real b) {
  if (!same_sign(a, b)) return real(0.0);
  return (real(2.0) * (a * b)) / (a + b);
}

static inline real limited_slope(int recon, real a, real b) {
  switch (recon) {
    case 1: return minmod(a, b);
    case 2: return mc_slope(a, b);
    case 3: return vanleer_slope(a, b);
    default: return real(0.0);
  }
}

static void cell_slopes(const real Vm[NV], const real Vc[NV], const real Vp[NV], int recon,
                        real s[NV]) {
  for (int q = 0; q < NV; ++q) s[q] = limited_slope(recon, Vc[q] - Vm[q], Vp[q] - Vc[q]);
  if (recon != 0) {
    real lo[3], hi[3];
    for (int j = 0; j < 3; ++j) { lo[j] = Vc[1 + j] - 0.5 * s[1 + j]; hi[j] = Vc[1 + j] + 0.5 * s[1 + j]; }
    const real v2lo = (lo[0] * lo[0] + lo[1] * lo[1]) + lo[2] * lo[2];
    const real v2hi = (hi[0] * hi[0] + hi[1] * hi[1]) + hi[2] * hi[2];
    if (!(v2lo < real(1.0)) || !(v2hi < real(1.0)))
      for (int q = 0; q < NV; ++q) s[q] = 0.0;
  }
}

static void limit_rad_flux(real V[NV]) {
  const real FF = (V[9] * V[9] + V[10] * V[10]) + V[11] * V[11];
  if (FF > V[8] * V[8]) {
    const real r = V[8] / rsqrt_(FF);
    for (int j = 0; j < 3; ++j) V[9 + j] = V[9 + j] * r;
  }
}

// ---------------------------------------------------------------------------
// 4x4 linear solve by Gaussian elimination with partial pivoting (the paper
// names LU decomposition for the implicit system).
static bool solve4(real A[4][4], real b[4], real x[4]) {
  for (int k = 0; k < 4; ++k) {
    int piv = k;
    real amax = rabs(A[k][k]);
    for (int i = k + 1; i < 4; ++i)
      if (rabs(A[i][k]) > amax) { amax = rabs(A[i][k]); piv = i; }
    if (!(amax > real(0.0))) return false;
    if (piv != k) {
      for (int j = 0; j < 4; ++j) std::swap(A[k][j], A[piv][j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < 4; ++i) {
      const real l = A[i][k] / A[k][k];
      for (int j = k + 1; j < 4; ++j) A[i][j] = A[i][j] - l * A[k][j];
      b[i] = b[i] - l * b[k];
    }
  }
  for (int i = 3; i >= 0; --i) {
    real s = b[i];
    for (int j = i + 1; j < 4; ++j) s = s - A[i][j] * x[j];
    x[i] = s / A[i][i];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Implicit radiation-matter step (Section 3.3, eqs. timeadv, totale, totalm,
// g0, gi). Unknown X = (E_r, F_r); the fluid follows from recovery of
// (D, S_t - F_r, tau_t - E_r, B). With h the implicit step, the backward-Euler
// system X = X* + h S_r(X), S_r = (-G^0, -G^i), is C(X) X = b(X) with
//   C11 = 1 - h rho W [-kappa + sigma (W^2 - 1 + u.D.u)]
//   C1j = -h rho u_j [kappa - sigma (2 W^2 - 1)]
//   Ci1 = -h rho [(kappa + sigma) (D.u)_i + sigma u_i (W^2 + u.D.u)]
//   Cij = delta_ij + h rho W [(kappa + sigma) delta_ij + 2 sigma u_i u_j]
//   b   = (E* + h rho W kappa a_R T^4,  F*_i + h rho u_i kappa a_R T^4).
// Cij carries a plus sign: expanding eq. gi gives +, while the printed matrix
// shows a minus (which would anti-damp F_r in a static medium).
struct ImpSys {
  real C[4][4];
  real b[4];
  real Z;
};

static bool imp_build(const real X[4], const real Us[NV], real Et, const real St[3], real h,
                      real kap, real sig, const OPar& P, const Consts& K, real Zg,
                      ImpSys& sy, int* c2p_it) {
  real Uf[NV], Vf[NV];
  Uf[0] = Us[0];
  for (int j = 0; j < 3; ++j) Uf[1 + j] = St[j] - X[1 + j];
  Uf[4] = Et - X[0];
  for (int j = 0; j < 3; ++j) Uf[5 + j] = Us[5 + j];
  Uf[8] = X[0];
  for (int j = 0; j < 3; ++j) Uf[9 + j] = X[1 + j];
  int it = 0;
  real Z = 0.0, lw[2];
  if (c2p(Uf, P, K, Zg, Vf, &Z, &it, lw) != 0) { *c2p_it += it; return false; }
  *c2p_it += it;
  sy.Z = Z;
  const real rho = Vf[0], p = Vf[4];
  // 1/W of the fluid state as the recovery formed it
  const real iW = lw[1];
  const real W = 1.0 / iW;
  real u[3];
  for (int j = 0; j < 3; ++j) u[j] = W * Vf[1 + j];
  const real T = (P.t_coeff * p) / rho;
  const real T2 = T * T;
  const real aT4 = P.a_rad * (T2 * T2);
  // Eddington tensor at the current radiation iterate (eq. xi).
  const real E = X[0];
  const real F[3] = {X[1], X[2], X[3]};
  const real FF = (F[0] * F[0] + F[1] * F[1]) + F[2] * F[2];
  const real f2 = FF / (E * E);
  real t = 4.0 - 3.0 * f2;
  t = (t > real(0.0)) ? t : real(0.0);
  const real xi = (3.0 + 4.0 * f2) / (5.0 + 2.0 * rsqrt_(t));
  const real ca = 0.5 * (1.0 - xi);
  const real cb = 0.5 * (3.0 * xi - 1.0);
  real Dm[3][3];
  if (FF >= real(kMinNormal)) {  // as in m1_row
    const real iFF = 1.0 / FF;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const real nn = (F[i] * F[j]) * iFF;
        Dm[i][j] = (i == j) ? ca + cb * nn : cb * nn;
      }
  } else {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Dm[i][j] = (i == j) ? ca : real(0.0);
  }
  real Du[3];
  for (int i = 0; i < 3; ++i) Du[i] = (Dm[i][0] * u[0] + Dm[i][1] * u[1]) + Dm[i][2] * u[2];
  const real uDu = (u[0] * Du[0] + u[1] * Du[1]) + u[2] * Du[2];
  const real W2 = W * W;
  const real hr = h * rho;
  const real hrW = hr * W;
  const real ks = kap + sig;
  sy.C[0][0] = 1.0 - hrW * (sig * ((W2 - 1.0) + uDu) - kap);
  const real c1 = kap - sig * (2.0 * W2 - 1.0);
  for (int j = 0; j < 3; ++j) sy.C[0][1 + j] = -((hr * u[j]) * c1);
  const real c2 = sig * (W2 + uDu);
  for (int i = 0; i < 3; ++i) sy.C[1 + i][0] = -(hr * (ks * Du[i] + c2 * u[i]));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const real g = 2.0 * ((sig * u[i]) * u[j]);
      sy.C[1 + i][1 + j] = (i == j) ? 1.0 + hrW * (ks + g) : hrW * g;
    }
  const real em = (hr * kap) * aT4;
  sy.b[0] = Us[8] + W * em;
  for (int i = 0; i < 3; ++i) sy.b[1 + i] = Us[9 + i] + u[i] * em;
  return true;
}

static void imp_residual(const ImpSys& sy, const real X[4], real R[4]) {
  for (int i = 0; i < 4; ++i)
    R[i] = (((sy.C[i][0] * X[0] + sy.C[i][1] * X[1]) + sy.C[i][2] * X[2]) + sy.C[i][3] * X[3]) - sy.b[i];
}

static real xscale(const real X[4]) {
  return rmax(rmax(rabs(X[0]), rabs(X[1])), rmax(rabs(X[2]), rabs(X[3])));
}

static real vmaxabs4(const real a[4]) {
  return rmax(rmax(rabs(a[0]), rabs(a[1])), rmax(rabs(a[2]), rabs(a[3])));
}

// Returns 0 on success and writes the new state; on failure Un = Us.
// Picard (the paper's lagged iteration): X^{m+1} = C(X^m)^{-1} b(X^m), started
// at X^0 = X*, accepted when max|X^{m+1} - X^m| <= tol * max|X| and the
// recovery at X^{m+1} succeeds. If it has not converged after imp_picard_it
// iterations (it diverges where the radiation heat capacity exceeds the
// gas's), Newton on R(X) = C(X) X - b(X) with a forward-difference Jacobian
// and step halving finishes from the last admissible iterate. Both reach the
// same root of the backward-Euler system.
// Zg0: recovery Z of the stage's cell state (warm start of the first
// recovery at X*; 0 for a cold start).
static int implicit_cell(const real Us[NV], real h, real kap, real sig, const OPar& P,
                         const Consts& K, real Un[NV], int* iters, int* c2p_it, int* floored, real Zg0) {
  const real Et = Us[4] + Us[8];
  real St[3];
  for (int j = 0; j < 3; ++j) St[j] = Us[1 + j] + Us[9 + j];
  // The upper limit |F_r| <= E_r (Section 3.2) is applied to the explicit
  // radiation state before the solve, keeping the totals tau + E_r and
  // S + F_r: the solve starts from, and its right-hand side uses, the
  // limited state. A non-positive E_r cannot be repaired and fails.
  real Ul[NV];
  for (int q = 0; q < NV; ++q) Ul[q] = Us[q];
  *floored = 0;
  if (!(Ul[8] > real(0.0))) {
    // Optional floor: the totals tau + E_r and S + F_r are kept, so the gas
    // pays for the raised radiation energy (conservative; counted).
    if (P.e_floor > 0.0 && rfinite(Ul[8])) {
      Ul[8] = P.e_floor;
      *floored = 1;
    } else {
      for (int q = 0; q < NV; ++q) Un[q] = Us[q];
      *iters = 0;
      *c2p_it = 0;
      return 1;
    }
  }
  {
    const real FF = (Ul[9] * Ul[9] + Ul[10] * Ul[10]) + Ul[11] * Ul[11];
    if (FF > Ul[8] * Ul[8]) {
      const real r = Ul[8] / rsqrt_(FF);
      for (int j = 0; j < 3; ++j) Ul[9 + j] = Ul[9 + j] * r;
    }
  }
  real X[4] = {Ul[8], Ul[9], Ul[10], Ul[11]};
  ImpSys sy;
  real Zg = Zg0;
  int it = 0;
  bool conv = false;
  bool have = false;
  *c2p_it = 0;
  const int npic = (P.imp_method == 1) ? 0 : ((P.imp_method == 2) ? P.imp_maxit : P.imp_picard_it);
  // Picard phase; it stops early once its update grows. If Picard is still
  // contracting when it reaches its iteration cap, Newton continues from its
  // last (admissible) iterate; otherwise Newton restarts from X*.
  const real Xg[4] = {X[0], X[1], X[2], X[3]};
  real dlast = 0.0, dprev = 0.0;
  bool built = false, capped = false;
  for (int m = 0; m <= npic; ++m) {
    built = imp_build(X, Ul, Et, St, h, kap, sig, P, K, Zg, sy, c2p_it);
    if (!built) break;
    Zg = sy.Z;
    if (m == 0) have = true;
    if (m == npic) { capped = true; break; }
    if (m > 1 && P.imp_method == 0 && dlast > dprev) break;
    real A[4][4], bb[4], Xn[4];
    for (int i = 0; i < 4; ++i) { bb[i] = sy.b[i]; for (int j = 0; j < 4; ++j) A[i][j] = sy.C[i][j]; }
    if (!solve4(A, bb, Xn)) break;
    ++it;
    if (!(Xn[0] > real(0.0)) || !rfinite(Xn[0]) || !rfinite(Xn[1]) || !rfinite(Xn[2]) || !rfinite(Xn[3])) break;
    real dd[4];
    for (int i = 0; i < 4; ++i) { dd[i] = Xn[i] - X[i]; X[i] = Xn[i]; }
    dprev = dlast;
    dlast = vmaxabs4(dd);
    // converged once the update is below tolerance; the system is not built
    // again at the accepted iterate
    if (dlast <= P.imp_tol * xscale(X)) { conv = true; break; }
  }
  if (!conv && have && P.imp_method != 2) {
    COUNT_NEWTON_PHASE;
    // Newton phase (its system is rebuilt at the start point).
    const bool from_picard = built && capped && npic > 1 && dlast < dprev;
    if (!from_picard) {
      for (int i = 0; i < 4; ++i) X[i] = Xg[i];
      Zg = Zg0;
    }
    real R[4];
    if (imp_build(X, Ul, Et, St, h, kap, sig, P, K, Zg, sy, c2p_it)) {
      Zg = sy.Z;
      imp_residual(sy, X, R);
      real sprev = 0.0;
      for (int n = 0; n < P.imp_maxit; ++n) {
        ++it;
        // difference step: relative to the iterate and to the scale of the
        // solution of the current linear system, ~ b_i / C_ii
        real bd[4];
        for (int i = 0; i < 4; ++i) bd[i] = sy.b[i] / sy.C[i][i];
        const real sc = rmax(xscale(X), vmaxabs4(bd));
        const real del = 1e-8 * sc;
        real J[4][4];
        bool okj = true;
        for (int j = 0; j < 4; ++j) {
          real Xp[4] = {X[0], X[1], X[2], X[3]};
          Xp[j] = Xp[j] + del;
          ImpSys sp;
          if (!imp_build(Xp, Ul, Et, St, h, kap, sig, P, K, Zg, sp, c2p_it)) { okj = false; break; }
          real Rp[4];
          imp_residual(sp, Xp, Rp);
          for (int i = 0; i < 4; ++i) J[i][j] = (Rp[i] - R[i]) / del;
        }
        if (!okj) break;
        real nR[4] = {-R[0], -R[1], -R[2], -R[3]}, dX[4];
        if (!solve4(J, nR, dX)) break;
        const real rn = vmaxabs4(R);
        const real dn = vmaxabs4(dX);
        real lam = 1.0;
        bool acc = false;
        real Xt[4], Rt[4];
        ImpSys st;
        for (int ls = 0; ls < 12; ++ls) {
          for (int i = 0; i < 4; ++i) Xt[i] = X[i] + lam * dX[i];
          if (Xt[0] > real(0.0) && imp_build(Xt, Ul, Et, St, h, kap, sig, P, K, Zg, st, c2p_it)) {
            imp_residual(st, Xt, Rt);
            if (vmaxabs4(Rt) < rn || lam * dn <= 1e-10 * sc) { acc = true; break; }
          }
          lam = 0.5 * lam;
        }
        if (!acc) break;
        real stp[4];
        for (int i = 0; i < 4; ++i) { stp[i] = Xt[i] - X[i]; X[i] = Xt[i]; R[i] = Rt[i]; }
        sy = st;
        Zg = st.Z;
        const real sn = vmaxabs4(stp);
        if (sn <= P.imp_tol * xscale(X)) { conv = true; break; }
        // at the rounding floor: a tiny step that no longer shrinks
        if (n > 0 && sn <= 1e-9 * sc && sn >= sprev) { conv = true; break; }
        sprev = sn;
      }
    }
  }
  *iters = it;
  if (!conv) {
    for (int q = 0; q < NV; ++q) Un[q] = Us[q];
    return 1;
  }
  // |F_r| <= E_r after the solve, by a rescale that keeps S + F_r fixed.
  const real FF = (X[1] * X[1] + X[2] * X[2]) + X[3] * X[3];
  if (FF > X[0] * X[0]) {
    const real r = X[0] / rsqrt_(FF);
    for (int j = 0; j < 3; ++j) X[1 + j] = X[1 + j] * r;
  }
  Un[0] = Us[0];
  for (int j = 0; j < 3; ++j) Un[1 + j] = St[j] - X[1 + j];
  Un[4] = Et - X[0];
  for (int j = 0; j < 3; ++j) Un[5 + j] = Us[5 + j];
  Un[8] = X[0];
  for (int j = 0; j < 3; ++j) Un[9 + j] = X[1 + j];
  return 0;
}

// ---------------------------------------------------------------------------
// The outer M1 eigenvalues lambda_r1 <= lambda_r3 of a radiation state in
// direction d (eqs. lam1, lam2, lam3): f = |F|/E (capped at 1), theta the
// angle between F and e_d (cos(theta) = 0 when F = 0).
static void rad_speeds(const real V[NV], int d, real& l1, real& l3) {
  const real E = V[8];
  const real FF = (V[9] * V[9] + V[10] * V[10]) + V[11] * V[11];
  real f = 0.0, cth = 0.0;
  if (FF > real(0.0)) {
    const real Fn = rsqrt_(FF);
    f = rmin(Fn / E, real(1.0));
    cth = V[9 + d] / Fn;
  }
  const real f2 = f * f;
  const real r43 = 4.0 - 3.0 * f2;
  const real sr = rsqrt_(r43);
  real zz = (2.0 / 3.0) * (r43 - sr) + (2.0 * (cth * cth)) * ((2.0 - f2) - sr);
  zz = (zz > real(0.0)) ? zz : real(0.0);
  const real zeta = rsqrt_(zz);
  l1 = (f * cth - zeta) / sr;
  l3 = (f * cth + zeta) / sr;
}

// ---------------------------------------------------------------------------
// Signal speed bound of one cell in direction d (for the CFL condition).
// Fluid: the relativistic fast-speed bound with a^2 = cs^2 + ca^2 - cs^2 ca^2,
//   lambda = [v_d (1 - a^2) +- sqrt(a^2 (1 - v^2)(1 - v^2 a^2 - v_d^2 (1 - a^2)))]
//            / (1 - v^2 a^2).
// Radiation: the M1 eigenvalues lambda_r1, lambda_r3 (eqs. lam1, lam2, lam3)
// with cos(theta) = F_d/|F| (0 when F = 0).
static real cell_speed(const real V[NV], int d, const OPar& P, const Consts& K) {
  Aux a;
  prim_aux(V, K, a);
  const real rho = V[0], p = V[4];
  const real rhoh = rho + K.g1 * p;
  const real cs2 = (P.gamma * p) / rhoh;
  const real ca2 = a.bb / (rhoh + a.bb);
  const real a2 = (cs2 + ca2) - cs2 * ca2;
  const real v2 = 1.0 - a.l2;
  const real vd = V[1 + d];
  const real den = 1.0 - v2 * a2;
  real disc = (a2 * a.l2) * (den - (vd * vd) * (1.0 - a2));
  disc = (disc > real(0.0)) ? disc : real(0.0);
  const real sq = rsqrt_(disc);
  const real lp = (vd * (1.0 - a2) + sq) / den;
  const real lm = (vd * (1.0 - a2) - sq) / den;
  real s = rmax(rabs(lp), rabs(lm));
  real l1, l3;
  rad_speeds(V, d, l1, l3);
  s = rmax(s, rmax(rabs(l1), rabs(l3)));
  return s;
}

// ---------------------------------------------------------------------------
// Rad-HLL face flux (Section 3.2, Radiative HLL). The magnetofluid rows 0..7
// and the radiation rows 8..11 each take the HLL flux with speeds of their own
// block of the Jacobian (eq. jacobian):
//   F^ = F_L                                          if lambda_L > 0,
//        F_R                                          if lambda_R < 0,
//        (lambda_R F_L - lambda_L F_R + lambda_R lambda_L (U_R - U_L))
//          / (lambda_R - lambda_L)                    otherwise,
// and, when lambda_L = lambda_R = 0, (F_L + F_R)/2 (reading: a fan of zero
// width, which the formula leaves undefined).
//
// Magnetofluid speeds: the extreme eigenvalues of the RMHD block, i.e. the
// smallest and the largest root of the quartic of Anile (1989), written as in
// Mignone & Bodo (2006),
//   Q(l) = w (1 - cs^2) a^4 - (1 - l^2) [(w cs^2 + |b|^2) a^2 - cs^2 B~^2],
//   a = W (l - v_d),   B~ = b^d - l b^0,   w = rho h,   cs^2 = gamma p / w.
// Its four roots (the fast and slow magnetosonic speeds) are real and lie in
// (-1, 1), and Q(+-1) > 0. For a polynomial of degree n with only real roots,
// Laguerre's iteration
//   l <- l - n / (G +- sqrt((n - 1)(n H - G^2))),  G = Q'/Q,  H = G^2 - Q''/Q,
// (sign: that of G, which is > 0 right of all roots and < 0 left of them)
// started outside the roots moves monotonically, and cubically near the end,
// to the nearest root: from l = 1 down to the largest, from l = -1 up to the
// smallest (reading: the paper names a root finder without giving it). The
// iteration stops when Q is no longer > 0, when an iterate no longer moves,
// or after kQuartIt steps; an early stop leaves the speed outside the root,
// which only widens the HLL fan. Each state gives (min, max); the face takes
// the min over L and R and the max over L and R.
//
// Radiation speeds: lambda_r1 and lambda_r3 of both states (eqs. lam1..lam3),
// the smaller r1 and the larger r3, limited by eq. limits with the optical
// depth tau = max(tau_L, tau_R) of the two cells next to the face (reading:
// the same cell depths that give beta of the PVM flux).
static const int kQuartIt = 20;

struct QuartIn {
  real w1cs;  // w (1 - cs^2)
  real wcsb;  // w cs^2 + |b|^2
  real cs2, W2, vd, bd, b0;
};

// Q, Q' and Q'' at l, from the factored form: with A = a^2 = W^2 (l - v_d)^2,
// br = (w cs^2 + |b|^2) A - cs^2 B~^2 and om = 1 - l^2, Q = w (1 - cs^2) A^2 - om br.
static void quartic(const QuartIn& q, real l, real& Q, real& dQ, real& d2Q) {
  const real x = l - q.vd;
  const real A = q.W2 * (x * x);
  const real Bt = q.bd - l * q.b0;
  const real om = 1.0 - l * l;
  const real br = q.wcsb * A - q.cs2 * (Bt * Bt);
  Q = q.w1cs * (A * A) - om * br;
  // A' = 2 W^2 (l - v_d), A'' = 2 W^2, B~' = -b^0, om' = -2 l, om'' = -2
  const real dA = 2.0 * (q.W2 * x);
  const real dbr = q.wcsb * dA + 2.0 * (q.cs2 * (q.b0 * Bt));
  const real d2br = q.wcsb * (2.0 * q.W2) - 2.0 * (q.cs2 * (q.b0 * q.b0));
  dQ = ((2.0 * q.w1cs) * (A * dA) + (2.0 * l) * br) - om * dbr;
  d2Q = (((2.0 * q.w1cs) * (dA * dA + A * (2.0 * q.W2)) + 2.0 * br) + (4.0 * l) * dbr) - om * d2br;
}

// One Laguerre step for the quartic (n = 4) from l toward the root below
// (down) or above (!down); returns false when the iteration has ended.
static bool laguerre_step(const QuartIn& q, bool down, real& l) {
  real Q, dQ, d2Q;
  quartic(q, l, Q, dQ, d2Q);
  if (!(Q > real(0.0))) return false;
  const real iQ = 1.0 / Q;
  const real G = dQ * iQ;
  const real H = G * G - d2Q * iQ;
  real t = 3.0 * (4.0 * H - G * G);
  t = (t > real(0.0)) ? t : real(0.0);
  const real sq = rsqrt_(t);
  const real ln = l - 4.0 / (down ? (G + sq) : (G - sq));
  if (!(down ? (ln < l) : (ln > l))) return false;
  l = ln;
  return true;
}

static void fast_speeds(const real V[NV], const Aux& a, int d, const OPar& P, const Consts& K,
                        real& lmin, real& lmax, int* iters) {
  QuartIn q;
  const real w = V[0] + K.g1 * V[4];
  q.cs2 = (P.gamma * V[4]) / w;
  q.w1cs = w * (1.0 - q.cs2);
  q.wcsb = w * q.cs2 + a.bb;
  q.W2 = a.W * a.W;
  q.vd = V[1 + d];
  q.bd = a.b[d];
  q.b0 = a.b0;
  int n = 0;
  real l = 1.0;
  for (int it = 0; it < kQuartIt && laguerre_step(q, true, l); ++it) ++n;
  lmax = l;
  l = -1.0;
  for (int it = 0; it < kQuartIt && laguerre_step(q, false, l); ++it) ++n;
  lmin = l;
  if (iters) *iters = n;
}

static void hll_rows(const real FL[NV], const real FR[NV], const real UL[NV], const real UR[NV],
                     real lL, real lR, int q0, int q1, real Fh[NV]) {
  for (int q = q0; q < q1; ++q) {
    if (lL > real(0.0)) Fh[q] = FL[q];
    else if (lR < real(0.0)) Fh[q] = FR[q];
    else if (lR > lL) Fh[q] = ((lR * FL[q] - lL * FR[q]) + (lR * lL) * (UR[q] - UL[q])) / (lR - lL);
    else Fh[q] = 0.5 * (FL[q] + FR[q]);
  }
}

static void hll_face(const real VL[NV], const real VR[NV], real tauL, real tauR, int d,
                     const OPar& P, const Consts& K, real Fh[NV], FaceOut& fo) {
  Aux aL, aR;
  prim_aux(VL, K, aL);
  prim_aux(VR, K, aR);
  real UL[NV], UR[NV], FL[NV], FR[NV];
  p2c(VL, aL, UL); flux(VL, aL, d, FL);
  p2c(VR, aR, UR); flux(VR, aR, d, FR);
  real mnL, mxL, mnR, mxR;
  int itL = 0, itR = 0;
  fast_speeds(VL, aL, d, P, K, mnL, mxL, &itL);
  fast_speeds(VR, aR, d, P, K, mnR, mxR, &itR);
  hll_rows(FL, FR, UL, UR, rmin(mnL, mnR), rmax(mxL, mxR), 0, 8, Fh);
  real r1L, r3L, r1R, r3R;
  rad_speeds(VL, d, r1L, r3L);
  rad_speeds(VR, d, r1R, r3R);
  const real lim = 4.0 / (3.0 * rmax(tauL, tauR));
  hll_rows(FL, FR, UL, UR, rmax(rmin(r1L, r1R), -lim), rmin(rmax(r3L, r3R), lim), 8, NV, Fh);
  fo.fallback = 0;
  fo.c2p_it = itL + itR;
}

// ---------------------------------------------------------------------------
// Grid helpers. U holds interior cells only, cell (i, j, k) at
// i + n0 (j + n1 k), variable q at offset q * var_stride. Cells outside the
// domain are mapped: periodic wraps, outflow copies the nearest interior cell
// (zero gradient), inflow (lo side of the last axis) takes the prescribed
// state where the mask is set and copies elsewhere.
struct Grid {
  OGrid g;
  long long ncell;
  int n[3];
};

// Returns the interior cell index, or -(t + 1) for an inflow cell with
// transverse index t.
static long long map_cell(const Grid& G, int i, int j, int k, int dir) {
  int c[3] = {i, j, k};
  const int d = dir;
  const int nd = G.n[d];
  if (c[d] < 0) {
    if (G.g.bc_lo[d] == 0) c[d] = ((c[d] % nd) + nd) % nd;
    else if (G.g.bc_lo[d] == 2) {
      const long long t = (d == 0) ? 0 : ((d == 1) ? c[0] : (long long)c[0] + (long long)G.n[0] * c[1]);
      if (G.g.inflow_mask && G.g.inflow_mask[t]) return -(t + 1);
      c[d] = 0;
    } else c[d] = 0;
  } else if (c[d] >= nd) {
    if (G.g.bc_hi[d] == 0) c[d] = c[d] % nd;
    else c[d] = nd - 1;
  }
  return (long long)c[0] + (long long)G.n[0] * ((long long)c[1] + (long long)G.n[1] * c[2]);
}

struct CellPrim {
  std::vector<double> V;      // [12][ncell]
  std::vector<double> taup;   // D (kappa + sigma), optical depth per unit length
  std::vector<double> Z;      // recovered Z = rho h W^2 (0 where recovery failed)
  std::vector<double> inV;    // inflow primitives [12][ntrans]
  std::vector<double> intaup;
};

static void load_U(const double* U, long long vs, long long c, real out[NV]) {
  for (int q = 0; q < NV; ++q) out[q] = U[q * vs + c];
}

static double opac_at(const double* arr, double uni, long long c) { return arr ? arr[c] : uni; }

// Cell recovery for one stage. Returns the number of failures.
static long long stage_prims(const Grid& G, const OPar& P, const Consts& K, const double* U,
                             const double* kap, const double* sig, double kap0, double sig0,
                             CellPrim& cp, long long* first_bad, int* max_it) {
  const long long N = G.ncell;
  const long long vs = G.g.var_stride;
  cp.V.assign((size_t)NV * N, 0.0);
  cp.taup.assign(N, 0.0);
  cp.Z.assign(N, 0.0);
  long long nfail = 0;
  long long fb = -1;
  int mit = 0;
#pragma omp parallel for schedule(static) reduction(+ : nfail) reduction(max : mit)
  for (long long c = 0; c < N; ++c) {
    real Uc[NV], Vc[NV], Z;
    int it = 0;
    load_U(U, vs, c, Uc);
    if (c2p(Uc, P, K, real(0.0), Vc, &Z, &it) != 0) {
      c2p_fallback(Uc, P, Vc);
      Z = 0.0;
      nfail += 1;
#pragma omp critical
      { if (fb < 0 || c < fb) fb = c; }
    }
    cp.Z[c] = dv(Z);
    mit = std::max(mit, it);
    for (int q = 0; q < NV; ++q) cp.V[q * N + c] = dv(Vc[q]);
    cp.taup[c] = dv(Uc[0] * (real(opac_at(kap, kap0, c)) + real(opac_at(sig, sig0, c))));
  }
  // Inflow cells (lo side of the last axis).
  const int dl = G.g.ndim - 1;
  cp.inV.clear();
  cp.intaup.clear();
  if (G.g.bc_lo[dl] == 2 && G.g.inflow_U) {
    long long nt = 1;
    for (int e = 0; e < G.g.ndim; ++e) if (e != dl) nt *= G.n[e];
    cp.inV.assign((size_t)NV * nt, 0.0);
    cp.intaup.assign(nt, 0.0);
    for (long long t = 0; t < nt; ++t) {
      real Uc[NV], Vc[NV], Z;
      int it = 0;
      for (int q = 0; q < NV; ++q) Uc[q] = G.g.inflow_U[q * nt + t];
      if (c2p(Uc, P, K, real(0.0), Vc, &Z, &it) != 0) c2p_fallback(Uc, P, Vc);
      for (int q = 0; q < NV; ++q) cp.inV[q * nt + t] = dv(Vc[q]);
      // Inflow ghosts take the opacity of the adjacent interior cell.
      long long c = (dl == 0) ? 0 : t;
      cp.intaup[t] = dv(Uc[0] * (real(opac_at(kap, kap0, c)) + real(opac_at(sig, sig0, c))));
    }
  }
  if (first_bad && fb >= 0 && (*first_bad < 0 || fb < *first_bad)) *first_bad = fb;
  if (max_it && mit > *max_it) *max_it = mit;
  return nfail;
}

static void get_cell(const Grid& G, const CellPrim& cp, long long m, real V[NV], real* taup) {
  if (m >= 0) {
    for (int q = 0; q < NV; ++q) V[q] = cp.V[q * G.ncell + m];
    *taup = cp.taup[m];
  } else {
    const long long t = -m - 1;
    const long long nt = (long long)cp.intaup.size();
    for (int q = 0; q < NV; ++q) V[q] = cp.inV[q * nt + t];
    *taup = cp.intaup[t];
  }
}

static long long face_count(const Grid& G, int d) {
  long long nf = 1;
  for (int e = 0; e < 3; ++e) nf *= (e == d) ? (G.n[e] + 1) : G.n[e];
  return nf;
}

// Face fluxes of one direction. Face index: along d the face i sits between
// cells i-1 and i (i = 0..n_d); faces are numbered with x fastest over the
// face-grid extents.
// bface (constrained transport): the staggered normal field b_d, one value per
// cell for the face on its lower side along d; both reconstructed states of a
// face take the face's own b_d as their normal field component.
static long long stage_faces(const Grid& G, const OPar& P, const Consts& K, const CellPrim& cp,
                             int d, double* Fh, const double* coef, int M, const double* bface = nullptr) {
  const long long nf = face_count(G, d);
  int fn[3] = {G.n[0], G.n[1], G.n[2]};
  fn[d] += 1;
  long long nfb = 0;
  const double dxd = G.g.dx[d];
#pragma omp parallel for schedule(static) reduction(+ : nfb)
  for (long long f = 0; f < nf; ++f) {
    int c[3];
    c[0] = (int)(f % fn[0]);
    c[1] = (int)((f / fn[0]) % fn[1]);
    c[2] = (int)(f / ((long long)fn[0] * fn[1]));
    real Vs[4][NV];
    real tp[4];
    for (int s = 0; s < 4; ++s) {
      int cc[3] = {c[0], c[1], c[2]};
      cc[d] = c[d] - 2 + s;
      const long long m = map_cell(G, cc[0], cc[1], cc[2], d);
      get_cell(G, cp, m, Vs[s], &tp[s]);
    }
    real sa[NV], sb[NV];
    cell_slopes(Vs[0], Vs[1], Vs[2], P.recon, sa);
    cell_slopes(Vs[1], Vs[2], Vs[3], P.recon, sb);
    real VL[NV], VR[NV];
    for (int q = 0; q < NV; ++q) { VL[q] = Vs[1][q] + 0.5 * sa[q]; VR[q] = Vs[2][q] - 0.5 * sb[q]; }
    limit_rad_flux(VL);
    limit_rad_flux(VR);
    if (bface) {
      int cc[3] = {c[0], c[1], c[2]};
      cc[d] = c[d] % G.n[d];  // face n_d is face 0 (periodic)
      const real bn = bface[(long long)cc[0] + (long long)G.n[0] * ((long long)cc[1] + (long long)G.n[1] * cc[2])];
      VL[5 + d] = bn;
      VR[5 + d] = bn;
    }
    const real tauL = tp[1] * dxd, tauR = tp[2] * dxd;
    real Fq[NV];
    FaceOut fo;
    if (P.solver == 1) hll_face(VL, VR, tauL, tauR, d, P, K, Fq, fo);
    else if (P.solver == 2) pvm_face_jvp(VL, VR, tauL, tauR, d, P, K, coef, M, Fq, fo);
    else pvm_face(VL, VR, tauL, tauR, d, P, K, coef, M, Fq, fo);
    nfb += fo.fallback;
    for (int q = 0; q < NV; ++q) Fh[q * nf + f] = dv(Fq[q]);
  }
  return nfb;
}

// ---------------------------------------------------------------------------
// Constrained transport (Section 4, opening paragraph: div B = 0 is kept with
// CT, the edge electromotive forces averaged by the CT-contact rule of
// Gardiner & Stone 2005). Periodic grids with ndim >= 2.
// Storage: the normal field b_a of the face on the lower side of cell c along
// a; the edge EMF E_k (edge along k, (a, b, k) cyclic) of the edge at the
// lower corner of cell c in the (a, b) plane. Only edges whose plane lies in
// the grid exist (2D: E_z).
// Face EMFs follow from the face fluxes of the induction equation,
// F_a(B_b) = v_a B_b - B_a v_b = -E_k on a-faces and F_b(B_a) = +E_k on
// b-faces; the cell-centre EMF from the cell's primitives,
// E_k = -(v_a B_b - v_b B_a). The corner EMF is the mean of its four face
// EMFs plus, along each plane direction, a quarter of the difference of the
// EMF gradients on the two sides of the corner, each gradient taken from the
// cell upwind of the contact (the sign of the mass flux through the face
// that separates the two candidate cells; their mean when it is zero).

// Periodic cell index of (i, j, k) + shifts.
static long long pcell(const Grid& G, int i, int j, int k) {
  i = ((i % G.n[0]) + G.n[0]) % G.n[0];
  j = ((j % G.n[1]) + G.n[1]) % G.n[1];
  k = ((k % G.n[2]) + G.n[2]) % G.n[2];
  return (long long)i + (long long)G.n[0] * ((long long)j + (long long)G.n[1] * k);
}

// Index of the face on the lower side of cell (i, j, k) along d (face grid
// with n_d + 1 faces along d, x fastest).
static long long lower_face(const Grid& G, int d, int i, int j, int k) {
  int fn[3] = {G.n[0], G.n[1], G.n[2]};
  fn[d] += 1;
  return (long long)i + (long long)fn[0] * ((long long)j + (long long)fn[1] * k);
}

// Upwind choice by the sign of a mass flux: lower-side value when it is
// positive, upper-side when negative, their mean when zero.
// Parity unpinned: the branch for an exactly zero face mass flux (the mean
// of the two sides) has no CPU pin of its own.
static real upwind(real mflux, real lower_side, real upper_side) {
  if (mflux > real(0.0)) return lower_side;
  if (mflux < real(0.0)) return upper_side;
  return 0.5 * (lower_side + upper_side);
}

// Edge EMFs E_k (k = 0..2; empty where the edge's plane is not in the grid)
// from the stage's face fluxes Fh[d] ([12][faces_d]) and cell primitives.
static void ct_edge_emfs(const Grid& G, const CellPrim& cp, const std::vector<std::vector<double>>& Fh,
                         std::vector<double> E[3]) {
  const long long N = G.ncell;
  const int nd = G.g.ndim;
  for (int k = 0; k < 3; ++k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    E[k].clear();
    if (a >= nd || b >= nd) continue;
    E[k].assign(N, 0.0);
    const long long nfa = face_count(G, a), nfb = face_count(G, b);
    const double* Fa = Fh[a].data();
    const double* Fb = Fh[b].data();
#pragma omp parallel for schedule(static)
    for (long long c = 0; c < N; ++c) {
      const int x[3] = {(int)(c % G.n[0]), (int)((c / G.n[0]) % G.n[1]), (int)(c / ((long long)G.n[0] * G.n[1]))};
      // cells around the corner: c, c - e_a, c - e_b, c - e_a - e_b (periodic)
      int ya[3] = {x[0], x[1], x[2]}, yb[3] = {x[0], x[1], x[2]}, yab[3] = {x[0], x[1], x[2]};
      ya[a] -= 1; yb[b] -= 1; yab[a] -= 1; yab[b] -= 1;
      const long long c_a = pcell(G, ya[0], ya[1], ya[2]);
      const long long c_b = pcell(G, yb[0], yb[1], yb[2]);
      const long long c_ab = pcell(G, yab[0], yab[1], yab[2]);
      // lower faces (along a of c and c - e_b; along b of c and c - e_a)
      const long long fa_c = lower_face(G, a, x[0], x[1], x[2]);
      const int xb[3] = {(int)(c_b % G.n[0]), (int)((c_b / G.n[0]) % G.n[1]), (int)(c_b / ((long long)G.n[0] * G.n[1]))};
      const long long fa_cb = lower_face(G, a, xb[0], xb[1], xb[2]);
      const long long fb_c = lower_face(G, b, x[0], x[1], x[2]);
      const int xa[3] = {(int)(c_a % G.n[0]), (int)((c_a / G.n[0]) % G.n[1]), (int)(c_a / ((long long)G.n[0] * G.n[1]))};
      const long long fb_ca = lower_face(G, b, xa[0], xa[1], xa[2]);
      // face EMFs
      const real Ea_c = -real(Fa[(5 + b) * nfa + fa_c]);
      const real Ea_cb = -real(Fa[(5 + b) * nfa + fa_cb]);
      const real Eb_c = real(Fb[(5 + a) * nfb + fb_c]);
      const real Eb_ca = real(Fb[(5 + a) * nfb + fb_ca]);
      // cell-centre EMFs
      auto ecell = [&](long long m) {
        const real va = cp.V[(1 + a) * N + m], vb = cp.V[(1 + b) * N + m];
        const real Ba = cp.V[(5 + a) * N + m], Bb = cp.V[(5 + b) * N + m];
        return -(va * Bb - vb * Ba);
      };
      const real Ec_c = ecell(c), Ec_a = ecell(c_a), Ec_b = ecell(c_b), Ec_ab = ecell(c_ab);
      // mass fluxes through the faces that separate the candidate cells
      const real ma_c = Fa[0 * nfa + fa_c], ma_cb = Fa[0 * nfa + fa_cb];
      const real mb_c = Fb[0 * nfb + fb_c], mb_ca = Fb[0 * nfb + fb_ca];
      // gradients along b on the upper (b) and lower (b - 1) side of the
      // corner, and along a on the upper (a) and lower (a - 1) side, as
      // differences over half a cell
      const real Dbhi = upwind(ma_c, Ec_a - Eb_ca, Ec_c - Eb_c);
      const real Dblo = upwind(ma_cb, Eb_ca - Ec_ab, Eb_c - Ec_b);
      const real Dahi = upwind(mb_c, Ec_b - Ea_cb, Ec_c - Ea_c);
      const real Dalo = upwind(mb_ca, Ea_cb - Ec_ab, Ea_c - Ec_a);
      const real s4 = (Ea_c + Ea_cb) + (Eb_c + Eb_ca);
      const real corr = (Dblo - Dbhi) + (Dalo - Dahi);
      E[k][c] = dv(0.25 * (s4 + corr));
    }
  }
}

// New face fields b_a = a0 b_a^(0) + a1 b_a^(s) - c dt (curl E)_a of a stage,
// (curl E)_a = dE_k/dx_b - dE_b/dx_k for (a, b, k) cyclic (terms whose edges
// exist only).
static void ct_face_update(const Grid& G, const std::vector<double> E[3], const double idx[3], const double* b0,
                           const double* bs, double a0, double a1, real cdt, double* bn) {
  const long long N = G.ncell;
  const int nd = G.g.ndim;
  for (int a = 0; a < nd; ++a) {
    const int b = (a + 1) % 3, k = (a + 2) % 3;
#pragma omp parallel for schedule(static)
    for (long long c = 0; c < N; ++c) {
      const int x[3] = {(int)(c % G.n[0]), (int)((c / G.n[0]) % G.n[1]), (int)(c / ((long long)G.n[0] * G.n[1]))};
      real t1 = 0.0, t2 = 0.0;
      if (!E[k].empty()) {
        int y[3] = {x[0], x[1], x[2]};
        y[b] += 1;
        t1 = (real(E[k][pcell(G, y[0], y[1], y[2])]) - real(E[k][c])) * idx[b];
      }
      if (!E[b].empty()) {
        int y[3] = {x[0], x[1], x[2]};
        y[k] += 1;
        t2 = (real(E[b][pcell(G, y[0], y[1], y[2])]) - real(E[b][c])) * idx[k];
      }
      const real curl = t1 - t2;
      bn[a * N + c] = dv((real(a0) * real(b0[a * N + c]) + real(a1) * real(bs[a * N + c])) - cdt * curl);
    }
  }
}

struct StageCoef { double a0, a1, c; };

static int rk_stages(int order, StageCoef s[3]) {
  if (order == 3) {
    // The paper's IMEX RK3 (Section 3.1, Shu-Osher form).
    s[0] = {1.0, 0.0, 1.0};
    s[1] = {0.75, 0.25, 0.25};
    s[2] = {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0};
    return 3;
  }
  // RK2 analogue of the same pattern (Heun / SSP-RK2), implicit steps dt, dt/2.
  s[0] = {1.0, 0.0, 1.0};
  s[1] = {0.5, 0.5, 0.5};
  return 2;
}

// One IMEX step (eqs. explicit, impliciteq and the RK pattern of Section 3.1).
// Each stage: U* = a0 U^(0) + a1 U^(s) + c dt L(U^(s)) with
// L = -sum_d (F^_{d,+} - F^_{d,-}) / dx_d (unsplit sum over directions), then
// U^(s+1) = implicit solve of U* with h = c dt.
static int step_impl(const OGrid& og, const OPar& P, double* U, const double* kap, const double* sig,
                     double kap0, double sig0, double dt, OReport* rep) {
  Grid G;
  G.g = og;
  for (int e = 0; e < 3; ++e) G.n[e] = (e < og.ndim) ? og.n[e] : 1;
  G.ncell = (long long)G.n[0] * G.n[1] * G.n[2];
  const Consts K = consts_of(P);
  const long long N = G.ncell, vs = og.var_stride;
  double coef[17];
  const int M = internal_poly(P.pvm_k, coef);
  OReport R = {0, 0, 0, 0, 0, -1, 0, 0};
  if (P.ct) {
    // constrained transport is defined here for periodic grids of 2 or 3 dimensions
    bool ok = og.ndim >= 2;
    for (int d = 0; d < og.ndim; ++d) ok = ok && og.bc_lo[d] == 0 && og.bc_hi[d] == 0;
    if (!ok) { if (rep) *rep = R; return 5; }
  }
  // With constrained transport, planes NV .. NV + ndim - 1 hold the staggered
  // normal fields, and the cell-centred B_a (a < ndim) is the mean of the two
  // face values of its cell.
  const int nb = P.ct ? og.ndim : 0;
  const int NT = NV + nb;
  std::vector<double> U0((size_t)NT * N), Us((size_t)NT * N);
  for (int q = 0; q < NT; ++q)
    for (long long c = 0; c < N; ++c) { U0[q * N + c] = U[q * vs + c]; Us[q * N + c] = U[q * vs + c]; }
  std::vector<double> Ek[3], bnew;
  StageCoef sc[3];
  const int ns = rk_stages(P.rk_order, sc);
  std::vector<std::vector<double>> Fh(og.ndim);
  CellPrim cp;
  Grid Gs = G;
  Gs.g.var_stride = N;
  double idx[3];
  for (int d = 0; d < og.ndim; ++d) idx[d] = 1.0 / og.dx[d];
  for (int s = 0; s < ns; ++s) {
    R.c2p_fail += stage_prims(Gs, P, K, Us.data(), kap, sig, kap0, sig0, cp, &R.first_bad_cell, &R.max_c2p_it);
    for (int d = 0; d < og.ndim; ++d) {
      Fh[d].assign((size_t)NV * face_count(G, d), 0.0);
      R.pvm_fallback += stage_faces(G, P, K, cp, d, Fh[d].data(), coef, M,
                                    P.ct ? Us.data() + (size_t)(NV + d) * N : nullptr);
    }
    const real cdt = real(sc[s].c) * real(dt);
    if (P.ct) {
      ct_edge_emfs(G, cp, Fh, Ek);
      bnew.assign((size_t)nb * N, 0.0);
      ct_face_update(G, Ek, idx, U0.data() + (size_t)NV * N, Us.data() + (size_t)NV * N, sc[s].a0, sc[s].a1, cdt,
                     bnew.data());
    }
    std::vector<double> Un((size_t)NT * N);
    long long nimp = 0, nnf = 0, nfl = 0, fb = -1;
    int mit = 0;
#pragma omp parallel for schedule(static) reduction(+ : nimp, nnf, nfl) reduction(max : mit)
    for (long long c = 0; c < N; ++c) {
      const int ci[3] = {(int)(c % G.n[0]), (int)((c / G.n[0]) % G.n[1]), (int)(c / ((long long)G.n[0] * G.n[1]))};
      real Ust[NV];
      for (int q = 0; q < NV; ++q) {
        if (q >= 5 && q < 5 + nb) {
          // constrained transport: the mean of the cell's two new face values
          int y[3] = {ci[0], ci[1], ci[2]};
          y[q - 5] += 1;
          const int a = q - 5;
          Ust[q] = 0.5 * (real(bnew[a * N + c]) + real(bnew[a * N + pcell(G, y[0], y[1], y[2])]));
          continue;
        }
        real div = 0.0;
        for (int d = 0; d < og.ndim; ++d) {
          int fn[3] = {G.n[0], G.n[1], G.n[2]};
          fn[d] += 1;
          const long long fm = (long long)ci[0] + (long long)fn[0] * ((long long)ci[1] + (long long)fn[1] * ci[2]);
          long long stride = 1;
          if (d == 1) stride = fn[0];
          if (d == 2) stride = (long long)fn[0] * fn[1];
          const long long nf = face_count(G, d);
          const real dF = real(Fh[d][q * nf + fm + stride]) - real(Fh[d][q * nf + fm]);
          if (d == 0) div = dF * idx[0];
          else div = div + dF * idx[d];
        }
        Ust[q] = (real(sc[s].a0) * real(U0[q * N + c]) + real(sc[s].a1) * real(Us[q * N + c])) - cdt * div;
      }
      real Unc[NV];
      int iters = 0, cit = 0, fl = 0;
      const int st = implicit_cell(Ust, cdt, real(opac_at(kap, kap0, c)), real(opac_at(sig, sig0, c)), P, K, Unc, &iters, &cit, &fl,
                                   real(cp.Z[c]));
      if (st != 0) nimp += 1;
      nfl += fl;
      mit = std::max(mit, iters);
      bool fin = true;
      for (int q = 0; q < NV; ++q) { Un[q * N + c] = dv(Unc[q]); if (!std::isfinite(dv(Unc[q]))) fin = false; }
      for (int a = 0; a < nb; ++a) Un[(NV + a) * N + c] = bnew[a * N + c];
      if (!fin) nnf += 1;
      if (st != 0 || !fin) {
#pragma omp critical
        { if (fb < 0 || c < fb) fb = c; }
      }
    }
    R.imp_fail += nimp;
    R.nonfinite += nnf;
    R.e_floor_hits += nfl;
    if (fb >= 0 && (R.first_bad_cell < 0 || fb < R.first_bad_cell)) R.first_bad_cell = fb;
    if (mit > R.max_imp_it) R.max_imp_it = mit;
    Us.swap(Un);
  }
  for (int q = 0; q < NT; ++q)
    for (long long c = 0; c < N; ++c) U[q * vs + c] = Us[q * N + c];
  if (rep) *rep = R;
  return (R.c2p_fail || R.imp_fail) ? 1 : ((R.nonfinite) ? 4 : 0);
}

// ===========================================================================
// C entry points used by the tests (ctypes). Arrays are [12][n] with the given
// stride between variable planes.
extern "C" {

int or_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
  return omp_get_max_threads();
#else
  (void)nt;
  return 1;
#endif
}

void or_p2c(long long n, const double* V, long long sv, const OPar* P, double* U, long long su) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real Vc[NV], Uc[NV];
    for (int q = 0; q < NV; ++q) Vc[q] = V[q * sv + c];
    Aux a;
    prim_aux(Vc, K, a);
    p2c(Vc, a, Uc);
    for (int q = 0; q < NV; ++q) U[q * su + c] = dv(Uc[q]);
  }
}

void or_flux(long long n, const double* V, long long sv, int d, const OPar* P, double* F, long long sf) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real Vc[NV], Fc[NV];
    for (int q = 0; q < NV; ++q) Vc[q] = V[q * sv + c];
    Aux a;
    prim_aux(Vc, K, a);
    flux(Vc, a, d, Fc);
    for (int q = 0; q < NV; ++q) F[q * sf + c] = dv(Fc[q]);
  }
}

// Z_in: optional warm-start values (NULL or <= 0: cold). status[c]: 0 ok.
void or_c2p(long long n, const double* U, long long su, const OPar* P, const double* Z_in,
            double* V, long long sv, double* Z_out, int* status, int* iters) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real Uc[NV], Vc[NV], Z = 0.0;
    for (int q = 0; q < NV; ++q) Uc[q] = U[q * su + c];
    int it = 0;
    const real zg = Z_in ? real(Z_in[c]) : real(0.0);
    int st = c2p(Uc, *P, K, zg, Vc, &Z, &it);
    if (st != 0) c2p_fallback(Uc, *P, Vc);
    for (int q = 0; q < NV; ++q) V[q * sv + c] = dv(Vc[q]);
    if (Z_out) Z_out[c] = dv(Z);
    if (status) status[c] = st;
    if (iters) iters[c] = it;
  }
}

// Recovery of each U (cold start) that also returns 1 - v^2 and 1/W as the
// final evaluation at the converged Z forms them: lw[0][c] = 1 - v^2,
// lw[1][c] = 1/W (0 where the recovery failed). For the tests that compare
// this Lorentz factor with the one of the recovered velocity.
void or_c2p_lw(long long n, const double* U, long long su, const OPar* P, double* V, long long sv,
               double* lw, int* status) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real Uc[NV], Vc[NV], Z = 0.0, l[2] = {0.0, 0.0};
    for (int q = 0; q < NV; ++q) Uc[q] = U[q * su + c];
    int it = 0;
    const int st = c2p(Uc, *P, K, real(0.0), Vc, &Z, &it, l);
    if (st != 0) c2p_fallback(Uc, *P, Vc);
    for (int q = 0; q < NV; ++q) V[q * sv + c] = dv(Vc[q]);
    lw[c] = dv(l[0]);
    lw[n + c] = dv(l[1]);
    if (status) status[c] = st;
  }
}

// One evaluation of the recovery's residual at a given Z for each U:
// out[k][c] for k = 0..8 is (ok, 1 - v^2, 1/W, 1/Z, 1/(Z + B^2), f/W, f'/W,
// rho, p), the quantities the Newton iteration on Z uses (f and f' are
// returned scaled by 1/W, as the iteration takes them). For the tests that
// compare them with their plain forms.
void or_c2p_eval(long long n, const double* U, long long su, const double* Z, const OPar* P,
                 double* out) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    C2PIn in;
    in.D = U[0 * su + c];
    for (int j = 0; j < 3; ++j) { in.S[j] = U[(1 + j) * su + c]; in.B[j] = U[(5 + j) * su + c]; }
    in.Et = real(U[4 * su + c]) + in.D;
    in.B2 = (in.B[0] * in.B[0] + in.B[1] * in.B[1]) + in.B[2] * in.B[2];
    in.S2 = (in.S[0] * in.S[0] + in.S[1] * in.S[1]) + in.S[2] * in.S[2];
    in.SB = (in.S[0] * in.B[0] + in.S[1] * in.B[1]) + in.S[2] * in.B[2];
    const C2PEval e = c2p_eval(real(Z[c]), in, K, true);
    // 1/Z and 1/(Z + B^2) are formed before any admissibility test; the rest
    // only for an admissible Z (v^2 < 1, p > 0).
    double r[9] = {e.ok ? 1.0 : 0.0, 0.0, 0.0, dv(e.iZ), dv(e.iZb), 0.0, 0.0, 0.0, 0.0};
    if (e.ok) {
      r[1] = dv(e.l2); r[2] = dv(e.iW); r[5] = dv(e.f); r[6] = dv(e.df); r[7] = dv(e.rho); r[8] = dv(e.p);
    }
    for (int k = 0; k < 9; ++k) out[k * n + c] = r[k];
  }
}

// PVM face flux from given reconstructed states.
void or_pvm_face(long long n, const double* VL, const double* VR, long long sv, const double* tauL,
                 const double* tauR, int d, const OPar* P, double* Fh, long long sf, int* fallback,
                 int* c2p_its) {
  const Consts K = consts_of(*P);
  double coef[17];
  const int M = internal_poly(P->pvm_k, coef);
  for (long long c = 0; c < n; ++c) {
    real L[NV], Rr[NV], Fq[NV];
    for (int q = 0; q < NV; ++q) { L[q] = VL[q * sv + c]; Rr[q] = VR[q * sv + c]; }
    FaceOut fo;
    if (P->solver == 2) pvm_face_jvp(L, Rr, real(tauL[c]), real(tauR[c]), d, *P, K, coef, M, Fq, fo);
    else pvm_face(L, Rr, real(tauL[c]), real(tauR[c]), d, *P, K, coef, M, Fq, fo);
    for (int q = 0; q < NV; ++q) Fh[q * sf + c] = dv(Fq[q]);
    if (fallback) fallback[c] = fo.fallback;
    if (c2p_its) c2p_its[c] = fo.c2p_it;
  }
}

// Rad-HLL face flux from given reconstructed states; iters: Newton steps of
// the four quartic roots.
void or_hll_face(long long n, const double* VL, const double* VR, long long sv, const double* tauL,
                 const double* tauR, int d, const OPar* P, double* Fh, long long sf, int* iters) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real L[NV], Rr[NV], Fq[NV];
    for (int q = 0; q < NV; ++q) { L[q] = VL[q * sv + c]; Rr[q] = VR[q * sv + c]; }
    FaceOut fo;
    hll_face(L, Rr, real(tauL[c]), real(tauR[c]), d, *P, K, Fq, fo);
    for (int q = 0; q < NV; ++q) Fh[q * sf + c] = dv(Fq[q]);
    if (iters) iters[c] = fo.c2p_it;
  }
}

// Smallest and largest magnetofluid characteristic speed of each state in
// direction d (the extreme roots of the RMHD quartic).
void or_fast_speeds(long long n, const double* V, long long sv, int d, const OPar* P, double* lmin,
                    double* lmax, int* iters) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real X[NV];
    for (int q = 0; q < NV; ++q) X[q] = V[q * sv + c];
    Aux a;
    prim_aux(X, K, a);
    real mn, mx;
    int it = 0;
    fast_speeds(X, a, d, *P, K, mn, mx, &it);
    lmin[c] = dv(mn);
    lmax[c] = dv(mx);
    if (iters) iters[c] = it;
  }
}

// A w at the conserved states U (exact JVP through the recovery), direction d;
// status[c] != 0 where the recovery of U fails.
void or_jvp(long long n, const double* U, const double* w, long long su, int d, const OPar* P, double* Aw,
            long long sa, int* status) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real X[NV], W[NV], V[NV], out[NV];
    for (int q = 0; q < NV; ++q) { X[q] = U[q * su + c]; W[q] = w[q * su + c]; }
    real Z = 0.0;
    int it = 0;
    const int st = c2p(X, *P, K, real(0.0), V, &Z, &it);
    if (status) status[c] = st;
    if (st != 0) {
      for (int q = 0; q < NV; ++q) Aw[q * sa + c] = 0.0;
      continue;
    }
    jvp_flux(X, Z, c2p_dfdZ(X, Z, K), W, d, K, out);
    for (int q = 0; q < NV; ++q) Aw[q * sa + c] = dv(out[q]);
  }
}

// Q, Q' and Q'' of the RMHD quartic of each state in direction d at l[c].
void or_quartic(long long n, const double* V, long long sv, int d, const OPar* P, const double* l,
                double* out /* [3][n] */) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real X[NV];
    for (int q = 0; q < NV; ++q) X[q] = V[q * sv + c];
    Aux a;
    prim_aux(X, K, a);
    QuartIn qi;
    const real w = X[0] + K.g1 * X[4];
    qi.cs2 = (P->gamma * X[4]) / w;
    qi.w1cs = w * (1.0 - qi.cs2);
    qi.wcsb = w * qi.cs2 + a.bb;
    qi.W2 = a.W * a.W;
    qi.vd = X[1 + d];
    qi.bd = a.b[d];
    qi.b0 = a.b0;
    real Q, dQ, d2Q;
    quartic(qi, real(l[c]), Q, dQ, d2Q);
    out[c] = dv(Q);
    out[n + c] = dv(dQ);
    out[2 * n + c] = dv(d2Q);
  }
}

// The outer M1 eigenvalues lambda_r1, lambda_r3 of each radiation state.
void or_rad_speeds(long long n, const double* V, long long sv, int d, double* l1, double* l3) {
  for (long long c = 0; c < n; ++c) {
    real X[NV];
    for (int q = 0; q < NV; ++q) X[q] = V[q * sv + c];
    real a, b;
    rad_speeds(X, d, a, b);
    l1[c] = dv(a);
    l3[c] = dv(b);
  }
}

int or_poly_coef(int k, double* c) {
  double cc[17];
  const int M = internal_poly(k, cc);
  for (int m = 0; m <= M; ++m) c[m] = cc[m];
  return M;
}

void or_implicit(long long n, const double* Us, long long su, const double* h, const double* kap,
                 const double* sig, const OPar* P, double* Un, long long sn, int* status, int* iters) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real Uc[NV], Uo[NV];
    for (int q = 0; q < NV; ++q) Uc[q] = Us[q * su + c];
    int it = 0, cit = 0, fl = 0;
    int st = implicit_cell(Uc, real(h[c]), real(kap[c]), real(sig[c]), *P, K, Uo, &it, &cit, &fl, real(0.0));
    for (int q = 0; q < NV; ++q) Un[q * sn + c] = dv(Uo[q]);
    if (status) status[c] = st;
    if (iters) iters[c] = it;
  }
}

// Direct evaluation of the radiation four-force (eqs. g0, gi) from a full
// primitive state: out = (G^0, G^1, G^2, G^3). Used by the tests to check the
// implicit solution against the backward-Euler equations without the matrix.
void or_four_force(long long n, const double* V, long long sv, const double* kap, const double* sig,
                   const OPar* P, double* G, long long sg) {
  for (long long c = 0; c < n; ++c) {
    real Vc[NV];
    for (int q = 0; q < NV; ++q) Vc[q] = V[q * sv + c];
    const real rho = Vc[0], p = Vc[4];
    const real v2 = (Vc[1] * Vc[1] + Vc[2] * Vc[2]) + Vc[3] * Vc[3];
    const real W = 1.0 / rsqrt_(1.0 - v2);
    real u[3];
    for (int j = 0; j < 3; ++j) u[j] = W * Vc[1 + j];
    const real T = (P->t_coeff * p) / rho;
    const real fourpiB = P->a_rad * ((T * T) * (T * T));
    const real E = Vc[8];
    const real F[3] = {Vc[9], Vc[10], Vc[11]};
    real Pr[3][3];
    for (int i = 0; i < 3; ++i) m1_row(E, F, i, Pr[i]);
    const real k = kap[c], s = sig[c];
    real uF = 0.0, uPu = 0.0;
    for (int i = 0; i < 3; ++i) uF = uF + u[i] * F[i];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) uPu = uPu + u[i] * u[j] * Pr[i][j];
    const real G0 = -rho * k * (fourpiB * W - W * E + uF)
                    - rho * s * (W * (W * W - 1.0) * E + W * uPu - (2.0 * W * W - 1.0) * uF);
    G[0 * sg + c] = dv(G0);
    for (int i = 0; i < 3; ++i) {
      real uP = 0.0;
      for (int j = 0; j < 3; ++j) uP = uP + u[j] * Pr[i][j];
      const real Gi = -fourpiB * rho * k * u[i] + rho * (k + s) * (W * F[i] - uP)
                      - rho * s * u[i] * (W * W * E - 2.0 * W * uF + uPu);
      G[(1 + i) * sg + c] = dv(Gi);
    }
  }
}

void or_cell_speed(long long n, const double* V, long long sv, int d, const OPar* P, double* s) {
  const Consts K = consts_of(*P);
  for (long long c = 0; c < n; ++c) {
    real Vc[NV];
    for (int q = 0; q < NV; ++q) Vc[q] = V[q * sv + c];
    s[c] = dv(cell_speed(Vc, d, *P, K));
  }
}

// Global maximum signal speed of U (capped at 1), as used by the CFL rule.
double or_max_speed(const OGrid* og, const OPar* P, const double* U, long long* nfail) {
  Grid G;
  G.g = *og;
  for (int e = 0; e < 3; ++e) G.n[e] = (e < og->ndim) ? og->n[e] : 1;
  G.ncell = (long long)G.n[0] * G.n[1] * G.n[2];
  const Consts K = consts_of(*P);
  const long long vs = og->var_stride;
  double smax = 0.0;
  long long nf = 0;
#pragma omp parallel for schedule(static) reduction(max : smax) reduction(+ : nf)
  for (long long c = 0; c < G.ncell; ++c) {
    real Uc[NV], Vc[NV], Z;
    int it;
    load_U(U, vs, c, Uc);
    if (c2p(Uc, *P, K, real(0.0), Vc, &Z, &it) != 0) { c2p_fallback(Uc, *P, Vc); nf += 1; }
    for (int d = 0; d < og->ndim; ++d) smax = std::max(smax, dv(cell_speed(Vc, d, *P, K)));
  }
  if (nfail) *nfail = nf;
  return std::min(smax, 1.0);
}

int or_step(const OGrid* og, const OPar* P, double* U, const double* kap, const double* sig,
            double kap0, double sig0, double dt, OReport* rep) {
  return step_impl(*og, *P, U, kap, sig, kap0, sig0, dt, rep);
}

// Face fluxes of the first stage only (cell recovery + reconstruction + PVM),
// for per-face comparisons. Fh_d: [12][faces_d] per direction, packed one
// direction after another.
long long or_face_fluxes(const OGrid* og, const OPar* P, const double* U, const double* kap,
                         const double* sig, double kap0, double sig0, double* Fh) {
  Grid G;
  G.g = *og;
  for (int e = 0; e < 3; ++e) G.n[e] = (e < og->ndim) ? og->n[e] : 1;
  G.ncell = (long long)G.n[0] * G.n[1] * G.n[2];
  const Consts K = consts_of(*P);
  double coef[17];
  const int M = internal_poly(P->pvm_k, coef);
  CellPrim cp;
  stage_prims(G, *P, K, U, kap, sig, kap0, sig0, cp, nullptr, nullptr);
  long long off = 0, nfb = 0;
  for (int d = 0; d < og->ndim; ++d) {
    nfb += stage_faces(G, *P, K, cp, d, Fh + off, coef, M,
                       P->ct ? U + (size_t)(NV + d) * og->var_stride : nullptr);
    off += NV * face_count(G, d);
  }
  return nfb;
}

// Explicit part of one stage: Ustar = a0 U0 + a1 Us - c dt sum_d dF^/dx_d,
// with the fluxes computed from Us (no implicit solve). For stage-level tests.
long long or_explicit_stage(const OGrid* og, const OPar* P, const double* U0, const double* Us,
                            const double* kap, const double* sig, double kap0, double sig0,
                            double a0, double a1, double c, double dt, double* Ust) {
  Grid G;
  G.g = *og;
  for (int e = 0; e < 3; ++e) G.n[e] = (e < og->ndim) ? og->n[e] : 1;
  G.ncell = (long long)G.n[0] * G.n[1] * G.n[2];
  const Consts K = consts_of(*P);
  double coef[17];
  const int M = internal_poly(P->pvm_k, coef);
  CellPrim cp;
  long long nbad = stage_prims(G, *P, K, Us, kap, sig, kap0, sig0, cp, nullptr, nullptr);
  std::vector<std::vector<double>> Fh(og->ndim);
  for (int d = 0; d < og->ndim; ++d) {
    Fh[d].assign((size_t)NV * face_count(G, d), 0.0);
    stage_faces(G, *P, K, cp, d, Fh[d].data(), coef, M);
  }
  double idx[3];
  for (int d = 0; d < og->ndim; ++d) idx[d] = 1.0 / og->dx[d];
  const real cdt = real(c) * real(dt);
  const long long N = G.ncell, vs = og->var_stride;
  for (long long cc = 0; cc < N; ++cc) {
    const int ci[3] = {(int)(cc % G.n[0]), (int)((cc / G.n[0]) % G.n[1]), (int)(cc / ((long long)G.n[0] * G.n[1]))};
    for (int q = 0; q < NV; ++q) {
      real div = 0.0;
      for (int d = 0; d < og->ndim; ++d) {
        int fn[3] = {G.n[0], G.n[1], G.n[2]};
        fn[d] += 1;
        const long long fm = (long long)ci[0] + (long long)fn[0] * ((long long)ci[1] + (long long)fn[1] * ci[2]);
        long long stride = 1;
        if (d == 1) stride = fn[0];
        if (d == 2) stride = (long long)fn[0] * fn[1];
        const long long nf = face_count(G, d);
        const real dF = real(Fh[d][q * nf + fm + stride]) - real(Fh[d][q * nf + fm]);
        if (d == 0) div = dF * idx[0];
        else div = div + dF * idx[d];
      }
      Ust[q * vs + cc] = dv((real(a0) * real(U0[q * vs + cc]) + real(a1) * real(Us[q * vs + cc])) - cdt * div);
    }
  }
  return nbad;
}

#ifdef ORACLE_COUNT_OPS
void or_opcount_reset(void) {
  g_ops = {0, 0, 0, 0};
  g_ops_newton = {0, 0, 0, 0};
}
void or_opcount_get(unsigned long long* out) {
  out[0] = g_ops.add; out[1] = g_ops.mul; out[2] = g_ops.div; out[3] = g_ops.sqrt;
}
void or_opcount_get_newton(unsigned long long* out) {
  out[0] = g_ops_newton.add; out[1] = g_ops_newton.mul; out[2] = g_ops_newton.div; out[3] = g_ops_newton.sqrt;
}
#endif

}  // extern "C"
