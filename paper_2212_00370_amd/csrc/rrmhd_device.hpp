// Device physics of the RRMHD + M1 hot path for gfx950 (HIP).
//
// Per-cell and per-face functions of the scheme of Lopez-Miralles, Marti &
// Perucho (CPC, arXiv 2212.00370): primitive/conserved maps (eq. eqU),
// fluxes (eq. eqF), the M1 closure (eq. xi), primitive recovery, PLM MinMod
// reconstruction, the Jacobian-free PVM-int face flux with the opacity factor
// beta (Section 3.2, eq. beta) and the implicit radiation-matter solve
// (Section 3.3, eqs. g0, gi).
//
// Floating point: every expression is evaluated in the order written (the
// library is compiled with -ffp-contract=off, no fast-math). The same fixed
// evaluation order is used by the CPU reference the tests compare against, so
// that the eps = 1e-8 finite-difference chain of the PVM flux, which
// amplifies rounding by 1/eps, yields identical results. Division and sqrt
// are the correctly rounded IEEE operations.
#pragma once

#include <hip/hip_runtime.h>

namespace rr {

constexpr int NV = 12;
constexpr int MAXCOEF = 17;

// Per-run constants, passed by value to every kernel.
struct Phys {
  double gamma, g1, gm1g, gm1;  // gamma, gamma/(gamma-1), (gamma-1)/gamma, gamma-1
  double a_rad, t_coeff;
  double eps, ieps;             // PVM finite-difference step and its reciprocal
  double eps32;                 // relative step of the FP32 chain (mixed precision)
  double c2p_tol, imp_tol;
  double rho_floor, p_floor;
  double e_floor;               // > 0: floor for a non-positive explicit E_r (counted)
  int c2p_maxit, imp_maxit, imp_picard_it, imp_method;
  int beta_mode, recon, M;      // M = 2^(k-1) Horner steps (0 for k = 0)
  double coef[MAXCOEF];         // p_k coefficients of x^(2m)
};

__device__ __forceinline__ double dabs(double a) { return (a < 0.0) ? -a : a; }
__device__ __forceinline__ double dmax(double a, double b) { return (a > b) ? a : b; }
__device__ __forceinline__ double dmin(double a, double b) { return (a < b) ? a : b; }

// Dual number v + d e with e^2 = 0 (forward-mode derivative). Constants enter
// with d = 0 and every operation is written on (v, d) pairs, so the templated
// flux code below evaluates derivatives when instantiated with Dual (binary64)
// or DualF (binary32, the mixed-precision path).
template <typename T>
struct DualT {
  T v, d;
  __device__ __forceinline__ DualT() : v(T(0)), d(T(0)) {}
  __device__ __forceinline__ DualT(T a) : v(a), d(T(0)) {}
  __device__ __forceinline__ DualT(T a, T b) : v(a), d(b) {}
};
using Dual = DualT<double>;
using DualF = DualT<float>;
template <typename T>
__device__ __forceinline__ DualT<T> operator+(DualT<T> a, DualT<T> b) { return DualT<T>(a.v + b.v, a.d + b.d); }
template <typename T>
__device__ __forceinline__ DualT<T> operator-(DualT<T> a, DualT<T> b) { return DualT<T>(a.v - b.v, a.d - b.d); }
template <typename T>
__device__ __forceinline__ DualT<T> operator-(DualT<T> a) { return DualT<T>(-a.v, -a.d); }
template <typename T>
__device__ __forceinline__ DualT<T> operator*(DualT<T> a, DualT<T> b) {
  return DualT<T>(a.v * b.v, a.v * b.d + a.d * b.v);
}
template <typename T>
__device__ __forceinline__ DualT<T> operator/(DualT<T> a, DualT<T> b) {
  const T q = a.v / b.v;
  return DualT<T>(q, (a.d - q * b.d) / b.v);
}
// The global float and double overloads stay visible next to this one.
using ::sqrt;
template <typename T>
__device__ __forceinline__ DualT<T> sqrt(DualT<T> a) {
  const T r = ::sqrt(a.v);
  return DualT<T>(r, a.d / (T(2) * r));
}
template <typename T>
__device__ __forceinline__ bool operator<(DualT<T> a, DualT<T> b) { return a.v < b.v; }
template <typename T>
__device__ __forceinline__ bool operator>(DualT<T> a, DualT<T> b) { return a.v > b.v; }
template <typename T>
__device__ __forceinline__ bool operator>=(DualT<T> a, DualT<T> b) { return a.v >= b.v; }

// Binary32 arithmetic types (float and its dual) take the reduced-flux form of
// the M1 closure.
template <typename R>
struct LowP { static constexpr bool value = false; };
template <>
struct LowP<float> { static constexpr bool value = true; };
template <>
struct LowP<DualF> { static constexpr bool value = true; };

// ---------------------------------------------------------------------------
// Quantities derived from primitives (definitions after eqs. eqU/eqF):
// W, b^0 = W v.B, b^i = B^i/W + v^i b^0, |b|^2 = B^2/W^2 + (v.B)^2,
// rho h* W^2 with rho h* = rho + gamma/(gamma-1) p + |b|^2, p* = p + |b|^2/2.
// Templated on the arithmetic type: double for the FP64 path, float for the
// FP32 flux arithmetic of the mixed-precision path. The double instantiation
// performs exactly the operations written (constants are exact).
template <typename R>
struct AuxT {
  R W, iW, l2, b0, b[3], bb, wtot, ps, D;
};
using Aux = AuxT<double>;

template <typename R>
__device__ __forceinline__ void prim_aux(const R V[NV], R g1, AuxT<R>& a) {
  const R vx = V[1], vy = V[2], vz = V[3];
  const R v2 = (vx * vx + vy * vy) + vz * vz;
  a.l2 = R(1) - v2;
  a.iW = sqrt(a.l2);
  a.W = R(1) / a.iW;
  const R vB = (vx * V[5] + vy * V[6]) + vz * V[7];
  a.b0 = a.W * vB;
#pragma unroll
  for (int j = 0; j < 3; ++j) a.b[j] = V[5 + j] * a.iW + V[1 + j] * a.b0;
  const R B2 = (V[5] * V[5] + V[6] * V[6]) + V[7] * V[7];
  a.bb = B2 * a.l2 + vB * vB;
  const R rhoh = V[0] + g1 * V[4];
  a.wtot = (rhoh + a.bb) * (a.W * a.W);
  a.ps = V[4] + R(0.5) * a.bb;
  a.D = V[0] * a.W;
}

__device__ __forceinline__ void prim_aux(const double V[NV], const Phys& K, Aux& a) { prim_aux<double>(V, K.g1, a); }

// prim_aux of a recovered state, with 1 - v^2 and 1/W as the recovery formed them.
__device__ __forceinline__ void prim_aux_w(const double V[NV], const double lw[2], const Phys& K, Aux& a) {
  const double vx = V[1], vy = V[2], vz = V[3];
  a.l2 = lw[0];
  a.iW = lw[1];
  a.W = 1.0 / a.iW;
  const double vB = (vx * V[5] + vy * V[6]) + vz * V[7];
  a.b0 = a.W * vB;
#pragma unroll
  for (int j = 0; j < 3; ++j) a.b[j] = V[5 + j] * a.iW + V[1 + j] * a.b0;
  const double B2 = (V[5] * V[5] + V[6] * V[6]) + V[7] * V[7];
  a.bb = B2 * a.l2 + vB * vB;
  const double rhoh = V[0] + K.g1 * V[4];
  a.wtot = (rhoh + a.bb) * (a.W * a.W);
  a.ps = V[4] + 0.5 * a.bb;
  a.D = V[0] * a.W;
}

// eq. eqU
template <typename R>
__device__ __forceinline__ void p2c(const R V[NV], const AuxT<R>& a, R U[NV]) {
  U[0] = a.D;
#pragma unroll
  for (int j = 0; j < 3; ++j) U[1 + j] = a.wtot * V[1 + j] - a.b0 * a.b[j];
  U[4] = ((a.wtot - a.ps) - a.b0 * a.b0) - a.D;
#pragma unroll
  for (int q = 5; q < NV; ++q) U[q] = V[q];
}

// Rows 0..7 of eq. eqU.
template <typename R>
__device__ __forceinline__ void p2c8(const R V[8], const AuxT<R>& a, R U[8]) {
  U[0] = a.D;
#pragma unroll
  for (int j = 0; j < 3; ++j) U[1 + j] = a.wtot * V[1 + j] - a.b0 * a.b[j];
  U[4] = ((a.wtot - a.ps) - a.b0 * a.b0) - a.D;
#pragma unroll
  for (int q = 5; q < 8; ++q) U[q] = V[q];
}

// Smallest normal double: |F|^2 below it counts as F = 0 in the closure's n n
// term (F F / |F|^2 would divide by an underflowed |F|^2; the term's weight
// (3 xi - 1)/2 ~ f^2 is negligible there).
constexpr double kMinNormal = 0x1p-1022;

// Row d of the M1 radiation pressure P = D_r E_r (eq. xi); n n := 0 when F = 0
// (or |F|^2 < kMinNormal).
// The FP32 instantiation works with the reduced flux f = F/E_r (|f| <~ 1):
// products of raw F_r components underflow FP32 where E_r ~ 1e-11.
template <int d, typename R>
__device__ __forceinline__ void m1_row(R E, const R F[3], R P[3]) {
  if constexpr (LowP<R>::value) {
    const R iE = R(1) / E;
    const R g[3] = {F[0] * iE, F[1] * iE, F[2] * iE};
    const R f2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
    R t = R(4) - R(3) * f2;
    t = (t > R(0)) ? t : R(0);
    const R s = sqrt(t);
    const R xi = (R(3) + R(4) * f2) / (R(5) + R(2) * s);
    const R ca = R(0.5) * (R(1) - xi);
    const R cb = R(0.5) * (R(3) * xi - R(1));
    if (f2 > R(1e-30)) {
      const R if2 = R(1) / f2;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R nn = (g[d] * g[j]) * if2;
        P[j] = (j == d) ? E * (ca + cb * nn) : E * (cb * nn);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j) P[j] = (j == d) ? E * ca : R(0);
    }
  } else {
    const R FF = (F[0] * F[0] + F[1] * F[1]) + F[2] * F[2];
    const R f2 = FF / (E * E);
    R t = R(4) - R(3) * f2;
    t = (t > R(0)) ? t : R(0);
    const R s = sqrt(t);
    const R xi = (R(3) + R(4) * f2) / (R(5) + R(2) * s);
    const R ca = R(0.5) * (R(1) - xi);
    const R cb = R(0.5) * (R(3) * xi - R(1));
    if (FF >= R(kMinNormal)) {
      const R iFF = R(1) / FF;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const R nn = (F[d] * F[j]) * iFF;
        P[j] = (j == d) ? E * (ca + cb * nn) : E * (cb * nn);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 3; ++j) P[j] = (j == d) ? E * ca : R(0);
    }
  }
}

// Rows 0..7 of eq. eqF (fluid and magnetic field) in direction d.
template <int d, typename R>
__device__ __forceinline__ void flux_mhd(const R V[8], const AuxT<R>& a, R F[8]) {
  const R vd = V[1 + d];
  F[0] = a.D * vd;
  const R wv = a.wtot * vd;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j == d) F[1 + j] = (wv * V[1 + j] + a.ps) - a.b[d] * a.b[j];
    else        F[1 + j] = wv * V[1 + j] - a.b[d] * a.b[j];
  }
  F[4] = (wv - a.b0 * a.b[d]) - a.D * vd;
#pragma unroll
  for (int j = 0; j < 3; ++j) F[5 + j] = vd * V[5 + j] - V[5 + d] * V[1 + j];
}

// Rows 8..11 of eq. eqF from Vr = (E_r, F_r): they involve the radiation
// variables only.
template <int d, typename R>
__device__ __forceinline__ void flux_rad(const R Vr[4], R F[4]) {
  F[0] = Vr[1 + d];
  m1_row<d, R>(Vr[0], &Vr[1], &F[1]);
}

// eq. eqF in direction d.
template <int d, typename R>
__device__ __forceinline__ void flux(const R V[NV], const AuxT<R>& a, R F[NV]) {
  const R vd = V[1 + d];
  F[0] = a.D * vd;
  const R wv = a.wtot * vd;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    if (j == d) F[1 + j] = (wv * V[1 + j] + a.ps) - a.b[d] * a.b[j];
    else        F[1 + j] = wv * V[1 + j] - a.b[d] * a.b[j];
  }
  F[4] = (wv - a.b0 * a.b[d]) - a.D * vd;
#pragma unroll
  for (int j = 0; j < 3; ++j) F[5 + j] = vd * V[5 + j] - V[5 + d] * V[1 + j];
  F[8] = V[9 + d];
  m1_row<d, R>(V[8], &V[9], &F[9]);
}

// ---------------------------------------------------------------------------
// Primitive recovery: bracketed Newton on Z = rho h W^2 (closed relations of
// eq. eqU): v^2(Z) = [S^2 + (S.B/Z)^2 (2Z + B^2)]/(Z + B^2)^2,
// p = (gamma-1)/gamma (Z/W^2 - D/W),
// f(Z) = Z + B^2 - p - B^2/(2W^2) - (S.B)^2/(2Z^2) - (tau + D).
// Bracket [D, gamma (tau + D)]; v^2 >= 1 or p <= 0 counts as f < 0; a Newton
// iterate outside the bracket (or a non-positive slope) is replaced by
// bisection. Converged when |dZ| <= tol Z.
struct C2PIn {
  double D, S[3], B[3], Et, B2, S2, SB;
};

struct C2PEval {
  bool ok;
  double l2, iW, rho, p, vB, iZb, f, df;
};

template <bool WANT_DF>
__device__ __forceinline__ C2PEval c2p_eval(double Z, const C2PIn& in, const Phys& K) {
  C2PEval e;
  const double Zb = Z + in.B2;
  // 1/Z and 1/(Z + B^2) from one reciprocal of the product
  const double rZZb = 1.0 / (Z * Zb);
  const double iZ = Zb * rZZb;
  e.iZb = Z * rZZb;
  e.vB = in.SB * iZ;
  const double vB2 = e.vB * e.vB;
  const double v2 = (in.S2 + vB2 * (Z + Zb)) * (e.iZb * e.iZb);
  // Evaluated without early exits (branch-free in a wave); where the state is
  // inadmissible (v^2 >= 1 or p <= 0) ok is false and the other fields are
  // not used.
  e.l2 = 1.0 - v2;
  e.iW = sqrt(e.l2);
  e.rho = in.D * e.iW;
  e.p = K.gm1g * (Z * e.l2 - e.rho);
  e.ok = (v2 < 1.0) && (e.p > 0.0);
  e.f = 0.0;
  e.df = 0.0;
  if (!WANT_DF) return e;
  const double f = (((Z + in.B2) - e.p) - 0.5 * (in.B2 * e.l2)) - (0.5 * vB2 + in.Et);
  const double dv2 = -2.0 * (in.S2 + (vB2 * (3.0 * (Z * Zb) + in.B2 * in.B2)) * iZ) *
                     ((e.iZb * e.iZb) * e.iZb);
  // f and f' times 1/W > 0: same signs and Newton quotient, no 1/(1/W).
  e.f = f * e.iW;
  const double dpw = K.gm1g * (e.l2 * e.iW + dv2 * (0.5 * in.D - Z * e.iW));
  e.df = ((e.iW - dpw) + (0.5 * (in.B2 * dv2)) * e.iW) + (vB2 * iZ) * e.iW;
  return e;
}

// Returns 0 on success. Zguess > 0 warm-starts; otherwise the rest-frame
// estimate gamma (E - B^2/2) - (gamma - 1) D is used.
// NU = NV: full state; NU = 8: fluid and magnetic field only (the radiation
// variables are not involved in the recovery).
// tol > 0 replaces K.c2p_tol (the binary32 chain of mixed precision needs Z
// only to its own rounding).
template <int NU = NV>
__device__ __forceinline__ int c2p(const double U[NU], const Phys& K, double Zguess, double V[NU],
                                   double& Zout, int& nit, double* lw = nullptr, double tol = -1.0) {
  const double ztol = (tol > 0.0) ? tol : K.c2p_tol;
  C2PIn in;
  in.D = U[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) { in.S[j] = U[1 + j]; in.B[j] = U[5 + j]; }
  in.Et = U[4] + U[0];
  in.B2 = (in.B[0] * in.B[0] + in.B[1] * in.B[1]) + in.B[2] * in.B[2];
  in.S2 = (in.S[0] * in.S[0] + in.S[1] * in.S[1]) + in.S[2] * in.S[2];
  in.SB = (in.S[0] * in.B[0] + in.S[1] * in.B[1]) + in.S[2] * in.B[2];
#pragma unroll
  for (int q = 5; q < NU; ++q) V[q] = U[q];
  nit = 0;
  if (!(in.D > 0.0) || !isfinite(in.Et) || !isfinite(in.S2) || !isfinite(in.B2)) return 1;
  double lo = in.D;
  double hi = K.gamma * in.Et;
  if (!(hi > lo)) return 1;
  double Z;
  if (Zguess > 0.0 && Zguess > lo && Zguess < hi) {
    Z = Zguess;
  } else {
    Z = K.gamma * (in.Et - 0.5 * in.B2) - K.gm1 * in.D;
    if (!(Z > lo && Z < hi)) Z = 0.5 * (lo + hi);
  }
  bool conv = false;
  int it = 0;
  // One straight-line body per iteration (selects instead of branches):
  // an inadmissible Z (ok false) raises lo and bisects; f = 0 stops at Z.
  while (it < K.c2p_maxit) {
    ++it;
    const C2PEval e = c2p_eval<true>(Z, in, K);
    const bool up = e.ok && (e.f > 0.0);
    hi = up ? Z : hi;
    lo = up ? lo : Z;
    const double Zt = Z - e.f / e.df;
    const bool take = e.ok && (e.df > 0.0) && (Zt > lo && Zt < hi);
    const double Zn = take ? Zt : 0.5 * (lo + hi);
    const bool hit = e.ok && (e.f == 0.0);
    const double dZ = dabs(Zn - Z);
    conv = hit || (dZ <= ztol * Zn);
    Z = hit ? Z : Zn;
    if (conv) break;
  }
  nit = it;
  if (!conv) return 2;
  const C2PEval e = c2p_eval<false>(Z, in, K);
  if (!e.ok) return 3;
  V[0] = e.rho;
#pragma unroll
  for (int j = 0; j < 3; ++j) V[1 + j] = (in.S[j] + e.vB * in.B[j]) * e.iZb;
  V[4] = e.p;
  Zout = Z;
  if (lw) { lw[0] = e.l2; lw[1] = e.iW; }
  return 0;
}

__device__ __forceinline__ void c2p_fallback(const double U[NV], const Phys& K, double V[NV]) {
  V[0] = (U[0] > 0.0) ? U[0] : K.rho_floor;
  V[1] = 0.0; V[2] = 0.0; V[3] = 0.0;
  V[4] = K.p_floor;
#pragma unroll
  for (int q = 5; q < NV; ++q) V[q] = U[q];
}

// Recovery of an intermediate PVM state: reuse V_m when the fluid part of U
// equals U_m's bit for bit (recovery depends on it only), else warm-start.
template <int NU = NV>
__device__ __forceinline__ bool recover_near(const double U[NU], const double Um[NU],
                                             const double Vm[NU], double Zm, const Phys& K,
                                             double V[NU], int& nit, const double* lwm = nullptr,
                                             double* lw = nullptr) {
  bool same = true;
#pragma unroll
  for (int q = 0; q < 8; ++q) same = same && (U[q] == Um[q]);
  if (same) {
#pragma unroll
    for (int q = 0; q < 5; ++q) V[q] = Vm[q];
#pragma unroll
    for (int q = 5; q < NU; ++q) V[q] = U[q];
    nit = 0;
    if (lw) { lw[0] = lwm[0]; lw[1] = lwm[1]; }
    return true;
  }
  double Z = 0.0;
  return c2p<NU>(U, K, Zm, V, Z, nit, lw) == 0;
}

// ---------------------------------------------------------------------------
// PLM with the Godunov fallback for |v|^2 >= 1 and the |F_r| <= E_r limit
// (Section 3.2, reconstruction). With a = V_i - V_{i-1}, b = V_{i+1} - V_i
// the slope is 0 unless a and b share a sign, else MinMod: the smaller of a, b
// in magnitude; MC: the smallest of 2a, 2b, (a + b)/2; VanLeer: 2ab/(a + b).
template <typename R>
__device__ __forceinline__ R rabs_(R a) { return a < R(0) ? -a : a; }

// REC >= 0 fixes the limiter at compile time; REC < 0 reads `recon`.
template <typename R, int REC = -1>
__device__ __forceinline__ R limited_slope(int recon, R a, R b) {
  if constexpr (REC >= 0) recon = REC;
  const bool same = (a > R(0) && b > R(0)) || (a < R(0) && b < R(0));
  R s;
  if (recon == 1) {
    s = (rabs_(a) < rabs_(b)) ? a : b;
  } else if (recon == 2) {
    const R ta = R(2) * a, tb = R(2) * b, c = R(0.5) * (a + b);
    const R m = (rabs_(ta) < rabs_(tb)) ? ta : tb;
    s = (rabs_(c) < rabs_(m)) ? c : m;
  } else {
    s = (R(2) * (a * b)) / (a + b);
  }
  return (same && recon != 0) ? s : R(0);
}

template <typename R, int REC = -1>
__device__ __forceinline__ void cell_slopes(const R Vm[NV], const R Vc[NV], const R Vp[NV], int recon, R s[NV]) {
  if constexpr (REC >= 0) recon = REC;
#pragma unroll
  for (int q = 0; q < NV; ++q) s[q] = limited_slope<R, REC>(recon, Vc[q] - Vm[q], Vp[q] - Vc[q]);
  if (recon != 0) {
    R lo[3], hi[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) { lo[j] = Vc[1 + j] - R(0.5) * s[1 + j]; hi[j] = Vc[1 + j] + R(0.5) * s[1 + j]; }
    const R v2lo = (lo[0] * lo[0] + lo[1] * lo[1]) + lo[2] * lo[2];
    const R v2hi = (hi[0] * hi[0] + hi[1] * hi[1]) + hi[2] * hi[2];
    if (!(v2lo < R(1)) || !(v2hi < R(1))) {
#pragma unroll
      for (int q = 0; q < NV; ++q) s[q] = R(0);
    }
  }
}

template <typename R>
__device__ __forceinline__ void limit_rad_flux(R V[NV]) {
  if constexpr (sizeof(R) == sizeof(float)) {
    // reduced flux, as in m1_row
    const R iE = R(1) / V[8];
    const R g[3] = {V[9] * iE, V[10] * iE, V[11] * iE};
    const R f2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
    if (f2 > R(1)) {
      const R r = R(1) / sqrt(f2);
#pragma unroll
      for (int j = 0; j < 3; ++j) V[9 + j] = V[9 + j] * r;
    }
  } else {
    const R FF = (V[9] * V[9] + V[10] * V[10]) + V[11] * V[11];
    if (FF > V[8] * V[8]) {
      const R r = V[8] / sqrt(FF);
#pragma unroll
      for (int j = 0; j < 3; ++j) V[9 + j] = V[9 + j] * r;
    }
  }
}

// ---------------------------------------------------------------------------
// LDS slots per lane for values the FP64 PVM chain keeps from its start to its
// end, so that they occupy no registers during the chain: (F_L + F_R)/2 of
// rows 0..7 (slots 0..7), the two candidate radiation rows (8..15) and U_0 of
// rows 0..7 (16..23). Workgroups of kParkLanes threads; slot k of thread t
// at [k * kParkLanes + t].
constexpr int kParkSlots = 24;
constexpr int kParkLanes = 64;
__device__ __forceinline__ double* park_lane() {
  __shared__ double park[kParkSlots * kParkLanes];
  return park + threadIdx.x;
}

// ---------------------------------------------------------------------------
// Jacobian-free PVM-int face flux (Section 3.2, PVM algorithm; eq. beta).
// Y(w) = [F(U_m + F(U_m + eps w) - F(U_m)) - F(U_m)] / eps ~ A(U_m)^2 w;
// Horner over x^2 gives U_M ~ p_k(A) U_0; F^ = (F_L + F_R)/2 - beta U_M / 2.
// A failed intermediate recovery drops the face to p_0 = 1 (Rusanov).
//
// The flux rows of the radiation variables (8..11) depend on those variables
// only, and rows 0..7 do not depend on them, so A(U) is block diagonal and
// every step of the chain acts on the two blocks separately. The radiation
// block (no recovery) runs first; the fluid/magnetic block follows with
// 8-wide states. Each component sees exactly the operations of the
// 12-wide chain.
template <int d>
__device__ __forceinline__ void pvm_face(const double VL[NV], const double VR[NV], double tauL,
                                         double tauR, const Phys& K, double Fh[NV],
                                         int& fallback, int& c2p_its) {
  const double beta = 1.0 / dmax(dmax(tauL, tauR), 1.0);
  double* sh = park_lane();
  // Radiation rows with the chain's dissipation (slots 8..11) and with
  // p_0 = 1 (slots 12..15).
  {
    double Fa[4], U0[4], Um[4], w[4];
    {
      double FL[4], FR[4];
      flux_rad<d, double>(&VL[8], FL);
      flux_rad<d, double>(&VR[8], FR);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        U0[q] = VR[8 + q] - VL[8 + q];
        Um[q] = 0.5 * (VL[8 + q] + VR[8 + q]);
        Fa[q] = 0.5 * (FL[q] + FR[q]);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) w[q] = U0[q];
    if (K.M > 0) {
      double Fm[4];
      flux_rad<d, double>(Um, Fm);
      for (int l = 0; l < K.M; ++l) {
        double Ue[4], Fe[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) Ue[q] = Um[q] + K.eps * w[q];
        flux_rad<d, double>(Ue, Fe);
#pragma unroll
        for (int q = 0; q < 4; ++q) Ue[q] = Um[q] + (Fe[q] - Fm[q]);
        flux_rad<d, double>(Ue, Fe);
        const double cnext = K.coef[K.M - 1 - l];
        if (l == 0) {
          const double ctop = K.coef[K.M];
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = ctop * ((Fe[q] - Fm[q]) * K.ieps) + cnext * U0[q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = (Fe[q] - Fm[q]) * K.ieps + cnext * U0[q];
        }
      }
    }
    const double bq = (K.beta_mode == 2) ? 1.0 : beta;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sh[(8 + q) * kParkLanes] = Fa[q] - 0.5 * (bq * w[q]);
      sh[(12 + q) * kParkLanes] = Fa[q] - 0.5 * (bq * U0[q]);
    }
  }
  // Fluid and magnetic rows. Only (F_L + F_R)/2, U_0 and U_m are needed past
  // the reconstruction.
  double Um[8], w[8];
  {
    double UL[8], UR[8], FL[8], FR[8];
    {
      Aux aL;
      prim_aux(VL, K, aL);
      p2c8(VL, aL, UL);
      flux_mhd<d, double>(VL, aL, FL);
    }
    {
      Aux aR;
      prim_aux(VR, K, aR);
      p2c8(VR, aR, UR);
      flux_mhd<d, double>(VR, aR, FR);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      w[q] = UR[q] - UL[q];
      sh[(16 + q) * kParkLanes] = w[q];  // U_0
      Um[q] = 0.5 * (UL[q] + UR[q]);
      sh[q * kParkLanes] = 0.5 * (FL[q] + FR[q]);  // (F_L + F_R)/2
    }
  }
  fallback = 0;
  c2p_its = 0;
  bool ok = true;
  if (K.M > 0) {
    double Vm[8], Zm = 0.0, lwm[2] = {0.0, 0.0};
    int it = 0;
    if (c2p<8>(Um, K, 0.0, Vm, Zm, it, lwm) != 0) ok = false;
    c2p_its += it;
    double Fm[8];
    if (ok) {
      Aux am;
      prim_aux_w(Vm, lwm, K, am);
      flux_mhd<d, double>(Vm, am, Fm);
    } else {
#pragma unroll
      for (int q = 0; q < 8; ++q) Fm[q] = 0.0;
    }
    for (int l = 0; l < K.M && ok; ++l) {
      double Ue[8], Ve[8], Fe[8], lw[2];
#pragma unroll
      for (int q = 0; q < 8; ++q) Ue[q] = Um[q] + K.eps * w[q];
      if (!recover_near<8>(Ue, Um, Vm, Zm, K, Ve, it, lwm, lw)) { ok = false; c2p_its += it; break; }
      c2p_its += it;
      {
        Aux ae;
        prim_aux_w(Ve, lw, K, ae);
        flux_mhd<d, double>(Ve, ae, Fe);
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) Ue[q] = Um[q] + (Fe[q] - Fm[q]);
      if (!recover_near<8>(Ue, Um, Vm, Zm, K, Ve, it, lwm, lw)) { ok = false; c2p_its += it; break; }
      c2p_its += it;
      {
        Aux at;
        prim_aux_w(Ve, lw, K, at);
        flux_mhd<d, double>(Ve, at, Fe);
      }
      const double cnext = K.coef[K.M - 1 - l];
      if (l == 0) {
        const double ctop = K.coef[K.M];
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = ctop * ((Fe[q] - Fm[q]) * K.ieps) + cnext * sh[(16 + q) * kParkLanes];
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = (Fe[q] - Fm[q]) * K.ieps + cnext * sh[(16 + q) * kParkLanes];
      }
    }
    if (!ok) {
      fallback = 1;
#pragma unroll
      for (int q = 0; q < 8; ++q) w[q] = sh[(16 + q) * kParkLanes];
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double bq = (K.beta_mode == 1 || K.beta_mode == 2) ? 1.0 : beta;
    Fh[q] = sh[q * kParkLanes] - 0.5 * (bq * w[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) Fh[8 + q] = ok ? sh[(8 + q) * kParkLanes] : sh[(12 + q) * kParkLanes];
}

// ---------------------------------------------------------------------------
// Exact-JVP variant of the PVM-int flux: the Horner scheme in A^2 of eq.
// utilde with every product A w = (dF/dU)(U_m) w formed in forward mode (Dual)
// instead of by the nested eps differences of eq. iterat. The recovery is
// differentiated implicitly at its converged Z: with the residual
// f(Z; U) = (Z + B^2) - p - B^2 (1 - v^2)/2 - (S.B/Z)^2/2 - (tau + D) of the
// closed relations of eq. eqU (not scaled), dZ = -(df/dU . w)/(df/dZ), and V
// follows from Z by v = (S + (S.B/Z) B)/(Z + B^2), 1/W = sqrt(1 - v^2),
// rho = D/W, p = (gamma-1)/gamma (Z (1 - v^2) - rho). One recovery per face
// (of U_m); none inside the chain. A failed recovery of U_m drops the face to
// p_0 = 1, as in pvm_face.
template <typename R>
__device__ __forceinline__ void prim_aux_lw(const R V[NV], R l2, R iW, double g1, AuxT<R>& a) {
  const R vx = V[1], vy = V[2], vz = V[3];
  a.l2 = l2;
  a.iW = iW;
  a.W = R(1.0) / a.iW;
  const R vB = (vx * V[5] + vy * V[6]) + vz * V[7];
  a.b0 = a.W * vB;
#pragma unroll
  for (int j = 0; j < 3; ++j) a.b[j] = V[5 + j] * a.iW + V[1 + j] * a.b0;
  const R B2 = (V[5] * V[5] + V[6] * V[6]) + V[7] * V[7];
  a.bb = B2 * a.l2 + vB * vB;
  const R rhoh = V[0] + R(g1) * V[4];
  a.wtot = (rhoh + a.bb) * (a.W * a.W);
  a.ps = V[4] + R(0.5) * a.bb;
  a.D = V[0] * a.W;
}

struct C2PInD {
  Dual D, S[3], B[3], Et, B2, S2, SB;
};

__device__ __forceinline__ C2PInD c2p_in_dual(const double U[NV], const double w[NV]) {
  C2PInD in;
  in.D = Dual(U[0], w[0]);
#pragma unroll
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

// Fluid V (rows 0..7), 1 - v^2 and 1/W from Z; returns the residual f.
__device__ __forceinline__ Dual c2p_closed(Dual Z, const C2PInD& in, const Phys& K, Dual V[8], Dual& l2, Dual& iW) {
  const Dual vB = in.SB / Z;
  const Dual iZb = Dual(1.0) / (Z + in.B2);
  const Dual v2 = (in.S2 + (vB * vB) * (Z + (Z + in.B2))) * (iZb * iZb);
  l2 = Dual(1.0) - v2;
  iW = sqrt(l2);
  const Dual rho = in.D * iW;
  const Dual p = Dual(K.gm1g) * (Z * l2 - rho);
  V[0] = rho;
#pragma unroll
  for (int j = 0; j < 3; ++j) V[1 + j] = (in.S[j] + vB * in.B[j]) * iZb;
  V[4] = p;
#pragma unroll
  for (int j = 0; j < 3; ++j) V[5 + j] = in.B[j];
  return (((Z + in.B2) - p) - Dual(0.5) * (in.B2 * l2)) - (Dual(0.5) * (vB * vB) + in.Et);
}

__device__ __forceinline__ double c2p_dfdZ(const double Um[NV], double Zm, const Phys& K) {
  double zero[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) zero[q] = 0.0;
  const C2PInD in = c2p_in_dual(Um, zero);
  Dual V[8], l2, iW;
  return c2p_closed(Dual(Zm, 1.0), in, K, V, l2, iW).d;
}

// A w at U_m, magnetofluid rows 0..7 (they depend on w[0..7] only).
template <int d>
__device__ __forceinline__ void jvp_flux_mhd(const double Um[8], double Zm, double fZ, const double w[8],
                                             const Phys& K, double Aw[8]) {
  double U12[NV], w12[NV];
#pragma unroll
  for (int q = 0; q < 8; ++q) { U12[q] = Um[q]; w12[q] = w[q]; }
#pragma unroll
  for (int q = 8; q < NV; ++q) { U12[q] = 0.0; w12[q] = 0.0; }
  const C2PInD in = c2p_in_dual(U12, w12);
  Dual V[8], l2, iW;
  const double fU = c2p_closed(Dual(Zm), in, K, V, l2, iW).d;
  const double dZ = -(fU / fZ);
  c2p_closed(Dual(Zm, dZ), in, K, V, l2, iW);
  Dual V12[NV];
#pragma unroll
  for (int q = 0; q < 8; ++q) V12[q] = V[q];
  AuxT<Dual> a;
  prim_aux_lw<Dual>(V12, l2, iW, K.g1, a);
  Dual F[8];
  flux_mhd<d, Dual>(V12, a, F);
#pragma unroll
  for (int q = 0; q < 8; ++q) Aw[q] = F[q].d;
}

// A w at U_m, radiation rows 8..11 (Ur, w: E_r, F_r).
template <int d>
__device__ __forceinline__ void jvp_flux_rad(const double Ur[4], const double w[4], double Aw[4]) {
  Dual X[4], F[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) X[q] = Dual(Ur[q], w[q]);
  flux_rad<d, Dual>(X, F);
#pragma unroll
  for (int q = 0; q < 4; ++q) Aw[q] = F[q].d;
}

template <int d>
__device__ __forceinline__ void pvm_face_jvp(const double VL[NV], const double VR[NV], double tauL,
                                             double tauR, const Phys& K, double Fh[NV],
                                             int& fallback, int& c2p_its) {
  const double beta = 1.0 / dmax(dmax(tauL, tauR), 1.0);
  double Fa[NV], U0[NV], Um[NV];
  {
    Aux aL, aR;
    prim_aux(VL, K, aL);
    prim_aux(VR, K, aR);
    double UL[NV], UR[NV], FL[NV], FR[NV];
    p2c(VL, aL, UL);
    flux<d>(VL, aL, FL);
    p2c(VR, aR, UR);
    flux<d>(VR, aR, FR);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      U0[q] = UR[q] - UL[q];
      Um[q] = 0.5 * (UL[q] + UR[q]);
      Fa[q] = 0.5 * (FL[q] + FR[q]);
    }
  }
  fallback = 0;
  c2p_its = 0;
  double w[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) w[q] = U0[q];
  if (K.M > 0) {
    double Vm[NV], Zm = 0.0;
    int it = 0;
    if (c2p<NV>(Um, K, 0.0, Vm, Zm, it) != 0) {
      fallback = 1;
    } else {
      // radiation block
      for (int l = 0; l < K.M; ++l) {
        double t1[4], t2[4];
        jvp_flux_rad<d>(&Um[8], &w[8], t1);
        jvp_flux_rad<d>(&Um[8], t1, t2);
        const double cnext = K.coef[K.M - 1 - l];
        const double ctop = (l == 0) ? K.coef[K.M] : 1.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) w[8 + q] = (l == 0) ? ctop * t2[q] + cnext * U0[8 + q] : t2[q] + cnext * U0[8 + q];
      }
      // magnetofluid block
      const double fZ = c2p_dfdZ(Um, Zm, K);
      for (int l = 0; l < K.M; ++l) {
        double t1[8], t2[8];
        jvp_flux_mhd<d>(Um, Zm, fZ, w, K, t1);
        jvp_flux_mhd<d>(Um, Zm, fZ, t1, K, t2);
        const double cnext = K.coef[K.M - 1 - l];
        const double ctop = (l == 0) ? K.coef[K.M] : 1.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = (l == 0) ? ctop * t2[q] + cnext * U0[q] : t2[q] + cnext * U0[q];
      }
    }
    c2p_its = it;
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double bq = (K.beta_mode == 2 || (K.beta_mode == 1 && q < 8)) ? 1.0 : beta;
    Fh[q] = Fa[q] - 0.5 * (bq * w[q]);
  }
}

// ---------------------------------------------------------------------------
// Mixed-precision PVM-int face flux: reconstruction, p2c, fluxes and the
// Horner/finite-difference arithmetic in FP32; every primitive recovery
// (U_m and the intermediate states) in FP64. eps = 1e-8 is below FP32
// rounding (U_m + eps w == U_m), so the chain keeps the paper's form
// U_m + eps w with eps = eps32 = 2^-12, about the square root of the FP32
// unit roundoff, which balances truncation and rounding error.
// recover_near for the FP32 chain's fluid block (8-wide): the recovery
// itself in FP64.
// Relative tolerance on Z of the recoveries inside the binary32 chain: below
// binary32's half unit (2^-24), so the rounded primitives are those of the
// converged root, and about one Newton step short of the binary64 tolerance
// from the chain's 2^-12 perturbations.
constexpr double kMixedC2PTol = 0x1p-26;

__device__ __forceinline__ bool recover_near_mixed(const float U[8], const float Um[8], const float Vm[8],
                                                   double Zm, const Phys& K, float V[8], int& nit) {
  bool same = true;
#pragma unroll
  for (int q = 0; q < 8; ++q) same = same && (U[q] == Um[q]);
  if (same) {
#pragma unroll
    for (int q = 0; q < 5; ++q) V[q] = Vm[q];
#pragma unroll
    for (int q = 5; q < 8; ++q) V[q] = U[q];
    nit = 0;
    return true;
  }
  double Ud[8], Vd[8], Z = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) Ud[q] = (double)U[q];
  if (c2p<8>(Ud, K, Zm, Vd, Z, nit, nullptr, kMixedC2PTol) != 0) return false;
#pragma unroll
  for (int q = 0; q < 5; ++q) V[q] = (float)Vd[q];
#pragma unroll
  for (int q = 5; q < 8; ++q) V[q] = U[q];
  return true;
}

// LDS slots of the FP32 chain (as park_lane for the FP64 chain): (F_L + F_R)/2
// and U_0 of rows 0..7 (slots 0..7, 16..23), the two candidate radiation rows
// (8..15).
__device__ __forceinline__ float* park_lane_f() {
  __shared__ float park[kParkSlots * kParkLanes];
  return park + threadIdx.x;
}

// Difference step of the binary32 chain, normalised to the direction w: the
// perturbation s w has max-norm h max|U_m| (h = 2^-12 ~ sqrt of the binary32
// unit), so A w = (F(U_m + s w) - F(U_m)) / s keeps about half of the
// binary32 digits however small w is against U_m (an absolute step h w
// rounds away once |w| < 2^-12 |U_m|). Returns false when w is zero or too
// small for any binary32 step (its image is then below the flux's rounding).
template <int N>
__device__ __forceinline__ bool dir_step(const float w[N], const float Um[N], float h, float& s, float& is) {
  float wn = 0.0f, un = 0.0f;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    wn = fmaxf(wn, fabsf(w[q]));
    un = fmaxf(un, fabsf(Um[q]));
  }
  if (!(wn > 0.0f)) return false;
  s = (h * ((un > 0.0f) ? un : 1.0f)) / wn;
  if (!(s < 1e30f)) return false;
  is = 1.0f / s;
  return true;
}

// The same block-diagonal split as pvm_face: radiation rows first, then the
// fluid and magnetic rows with 8-wide states.
template <int d>
__device__ __forceinline__ void pvm_face_mixed(const float VL[NV], const float VR[NV], float tauL, float tauR,
                                               const Phys& K, float Fh[NV], int& fallback, int& c2p_its) {
  const float g1 = (float)K.g1;
  const float beta = 1.0f / fmaxf(fmaxf(tauL, tauR), 1.0f);
  const float h = (float)K.eps32;
  float* sh = park_lane_f();
  {
    float Fa[4], U0[4], Um[4], w[4];
    {
      float FL[4], FR[4];
      flux_rad<d, float>(&VL[8], FL);
      flux_rad<d, float>(&VR[8], FR);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        U0[q] = VR[8 + q] - VL[8 + q];
        Um[q] = 0.5f * (VL[8 + q] + VR[8 + q]);
        Fa[q] = 0.5f * (FL[q] + FR[q]);
        w[q] = U0[q];
      }
    }
    if (K.M > 0) {
      float Fm[4];
      flux_rad<d, float>(Um, Fm);
      for (int l = 0; l < K.M; ++l) {
        float Ue[4], Fe[4], Y[4];
        float s, is;
        if (dir_step<4>(w, Um, h, s, is)) {
#pragma unroll
          for (int q = 0; q < 4; ++q) Ue[q] = Um[q] + s * w[q];
          flux_rad<d, float>(Ue, Fe);
#pragma unroll
          for (int q = 0; q < 4; ++q) Ue[q] = Um[q] + (Fe[q] - Fm[q]);
          flux_rad<d, float>(Ue, Fe);
#pragma unroll
          for (int q = 0; q < 4; ++q) Y[q] = (Fe[q] - Fm[q]) * is;
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) Y[q] = 0.0f;
        }
        const float cnext = (float)K.coef[K.M - 1 - l];
        if (l == 0) {
          const float ctop = (float)K.coef[K.M];
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = ctop * Y[q] + cnext * U0[q];
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = Y[q] + cnext * U0[q];
        }
      }
    }
    const float bq = (K.beta_mode == 2) ? 1.0f : beta;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sh[(8 + q) * kParkLanes] = Fa[q] - 0.5f * (bq * w[q]);
      sh[(12 + q) * kParkLanes] = Fa[q] - 0.5f * (bq * U0[q]);
    }
  }
  float Um[8], w[8];
  {
    float UL[8], UR[8], FL[8], FR[8];
    {
      AuxT<float> aL;
      prim_aux<float>(VL, g1, aL);
      p2c8<float>(VL, aL, UL);
      flux_mhd<d, float>(VL, aL, FL);
    }
    {
      AuxT<float> aR;
      prim_aux<float>(VR, g1, aR);
      p2c8<float>(VR, aR, UR);
      flux_mhd<d, float>(VR, aR, FR);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      w[q] = UR[q] - UL[q];
      sh[(16 + q) * kParkLanes] = w[q];  // U_0
      Um[q] = 0.5f * (UL[q] + UR[q]);
      sh[q * kParkLanes] = 0.5f * (FL[q] + FR[q]);
    }
  }
  fallback = 0;
  c2p_its = 0;
  bool ok = true;
  if (K.M > 0) {
    float Vm[8], Fm[8];
    double Zm = 0.0;
    int it = 0;
    {
      double Ud[8], Vd[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) Ud[q] = (double)Um[q];
      if (c2p<8>(Ud, K, 0.0, Vd, Zm, it, nullptr, kMixedC2PTol) != 0) ok = false;
#pragma unroll
      for (int q = 0; q < 5; ++q) Vm[q] = (float)Vd[q];
#pragma unroll
      for (int q = 5; q < 8; ++q) Vm[q] = Um[q];
    }
    c2p_its += it;
    if (ok) {
      AuxT<float> am;
      prim_aux<float>(Vm, g1, am);
      flux_mhd<d, float>(Vm, am, Fm);
    }
    for (int l = 0; l < K.M && ok; ++l) {
      float Y[8];
      float s, is;
      if (!dir_step<8>(w, Um, h, s, is)) {
#pragma unroll
        for (int q = 0; q < 8; ++q) Y[q] = 0.0f;
      } else {
        float Ue[8], Ve[8], Fe[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) Ue[q] = Um[q] + s * w[q];
        if (!recover_near_mixed(Ue, Um, Vm, Zm, K, Ve, it)) { ok = false; c2p_its += it; break; }
        c2p_its += it;
        {
          AuxT<float> ae;
          prim_aux<float>(Ve, g1, ae);
          flux_mhd<d, float>(Ve, ae, Fe);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) Ue[q] = Um[q] + (Fe[q] - Fm[q]);
        if (!recover_near_mixed(Ue, Um, Vm, Zm, K, Ve, it)) { ok = false; c2p_its += it; break; }
        c2p_its += it;
        {
          AuxT<float> at;
          prim_aux<float>(Ve, g1, at);
          flux_mhd<d, float>(Ve, at, Fe);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) Y[q] = (Fe[q] - Fm[q]) * is;
      }
      const float cnext = (float)K.coef[K.M - 1 - l];
      if (l == 0) {
        const float ctop = (float)K.coef[K.M];
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = ctop * Y[q] + cnext * sh[(16 + q) * kParkLanes];
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = Y[q] + cnext * sh[(16 + q) * kParkLanes];
      }
    }
    if (!ok) {
      fallback = 1;
#pragma unroll
      for (int q = 0; q < 8; ++q) w[q] = sh[(16 + q) * kParkLanes];
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float bq = (K.beta_mode == 1 || K.beta_mode == 2) ? 1.0f : beta;
    Fh[q] = sh[q * kParkLanes] - 0.5f * (bq * w[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) Fh[8 + q] = ok ? sh[(8 + q) * kParkLanes] : sh[(12 + q) * kParkLanes];
}

// Mixed-precision form of the exact-JVP flux: reconstruction, fluxes and the
// forward-mode products of eq. eqF in binary32 (DualF); the recovery of U_m,
// its implicit derivative dZ and the derivative of V in binary64 (the parts
// that need the digits), rounded to binary32 where the flux takes over.
template <int d>
__device__ __forceinline__ void jvp_flux_mhd_mixed(const double Umd[NV], double Zm, double fZ, const float w[8],
                                                   const Phys& K, float Aw[8]) {
  double w12[NV];
#pragma unroll
  for (int q = 0; q < 8; ++q) w12[q] = (double)w[q];
#pragma unroll
  for (int q = 8; q < NV; ++q) w12[q] = 0.0;
  const C2PInD in = c2p_in_dual(Umd, w12);
  Dual V[8], l2, iW;
  const double fU = c2p_closed(Dual(Zm), in, K, V, l2, iW).d;
  const double dZ = -(fU / fZ);
  c2p_closed(Dual(Zm, dZ), in, K, V, l2, iW);
  DualF Vf[NV];
#pragma unroll
  for (int q = 0; q < 8; ++q) Vf[q] = DualF((float)V[q].v, (float)V[q].d);
  AuxT<DualF> a;
  prim_aux_lw<DualF>(Vf, DualF((float)l2.v, (float)l2.d), DualF((float)iW.v, (float)iW.d), K.g1, a);
  DualF F[8];
  flux_mhd<d, DualF>(Vf, a, F);
#pragma unroll
  for (int q = 0; q < 8; ++q) Aw[q] = F[q].d;
}

template <int d>
__device__ __forceinline__ void jvp_flux_rad_f(const float Ur[4], const float w[4], float Aw[4]) {
  DualF X[4], F[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) X[q] = DualF(Ur[q], w[q]);
  flux_rad<d, DualF>(X, F);
#pragma unroll
  for (int q = 0; q < 4; ++q) Aw[q] = F[q].d;
}

template <int d>
__device__ __forceinline__ void pvm_face_jvp_mixed(const float VL[NV], const float VR[NV], float tauL, float tauR,
                                                   const Phys& K, float Fh[NV], int& fallback, int& c2p_its) {
  const float g1 = (float)K.g1;
  const float beta = 1.0f / fmaxf(fmaxf(tauL, tauR), 1.0f);
  float Fa[NV], U0[NV], Um[NV];
  {
    AuxT<float> aL, aR;
    prim_aux<float>(VL, g1, aL);
    prim_aux<float>(VR, g1, aR);
    float UL[NV], UR[NV], FL[NV], FR[NV];
    p2c<float>(VL, aL, UL);
    flux<d, float>(VL, aL, FL);
    p2c<float>(VR, aR, UR);
    flux<d, float>(VR, aR, FR);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      U0[q] = UR[q] - UL[q];
      Um[q] = 0.5f * (UL[q] + UR[q]);
      Fa[q] = 0.5f * (FL[q] + FR[q]);
    }
  }
  fallback = 0;
  c2p_its = 0;
  float w[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) w[q] = U0[q];
  if (K.M > 0) {
    double Umd[NV], Vmd[NV], Zm = 0.0;
#pragma unroll
    for (int q = 0; q < NV; ++q) Umd[q] = (double)Um[q];
    int it = 0;
    if (c2p<NV>(Umd, K, 0.0, Vmd, Zm, it) != 0) {
      fallback = 1;
    } else {
      for (int l = 0; l < K.M; ++l) {
        float t1[4], t2[4];
        jvp_flux_rad_f<d>(&Um[8], &w[8], t1);
        jvp_flux_rad_f<d>(&Um[8], t1, t2);
        const float cnext = (float)K.coef[K.M - 1 - l];
        const float ctop = (l == 0) ? (float)K.coef[K.M] : 1.0f;
#pragma unroll
        for (int q = 0; q < 4; ++q) w[8 + q] = ctop * t2[q] + cnext * U0[8 + q];
      }
      const double fZ = c2p_dfdZ(Umd, Zm, K);
      for (int l = 0; l < K.M; ++l) {
        float t1[8], t2[8];
        jvp_flux_mhd_mixed<d>(Umd, Zm, fZ, w, K, t1);
        jvp_flux_mhd_mixed<d>(Umd, Zm, fZ, t1, K, t2);
        const float cnext = (float)K.coef[K.M - 1 - l];
        const float ctop = (l == 0) ? (float)K.coef[K.M] : 1.0f;
#pragma unroll
        for (int q = 0; q < 8; ++q) w[q] = ctop * t2[q] + cnext * U0[q];
      }
    }
    c2p_its = it;
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const float bq = (K.beta_mode == 2 || (K.beta_mode == 1 && q < 8)) ? 1.0f : beta;
    Fh[q] = Fa[q] - 0.5f * (bq * w[q]);
  }
}

// ---------------------------------------------------------------------------
// 4x4 Gaussian elimination with partial pivoting (first maximum wins), all
// indices static so the matrix stays in registers.
__device__ __forceinline__ bool solve4(double A[4][4], double b[4], double x[4]) {
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int piv = k;
    double amax = dabs(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < 4; ++i)
      if (dabs(A[i][k]) > amax) { amax = dabs(A[i][k]); piv = i; }
    if (!(amax > 0.0)) return false;
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      if (piv == i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) { const double t = A[k][j]; A[k][j] = A[i][j]; A[i][j] = t; }
        const double t = b[k]; b[k] = b[i]; b[i] = t;
      }
    }
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      const double l = A[i][k] / A[k][k];
#pragma unroll
      for (int j = k + 1; j < 4; ++j) A[i][j] = A[i][j] - l * A[k][j];
      b[i] = b[i] - l * b[k];
    }
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    double s = b[i];
#pragma unroll
    for (int j = i + 1; j < 4; ++j) s = s - A[i][j] * x[j];
    x[i] = s / A[i][i];
  }
  return true;
}

// ---------------------------------------------------------------------------
// Implicit radiation-matter step (Section 3.3). X = (E_r, F_r); the fluid
// follows from recovery of (D, S_t - F_r, tau_t - E_r, B). The backward-Euler
// system from eqs. g0/gi reads C(X) X = b(X) with
//   C11 = 1 - h rho W [-kappa + sigma (W^2 - 1 + u.D.u)]
//   C1j = -h rho u_j [kappa - sigma (2W^2 - 1)]
//   Ci1 = -h rho [(kappa + sigma)(D.u)_i + sigma u_i (W^2 + u.D.u)]
//   Cij = delta_ij + h rho W [(kappa + sigma) delta_ij + 2 sigma u_i u_j]
//   b   = (E* + h rho W kappa a T^4, F*_i + h rho u_i kappa a T^4)
// (Cij with the sign that follows from eq. gi).
struct ImpSys {
  double C[4][4];
  double b[4];
  double Z;
};

__device__ __forceinline__ bool imp_build(const double X[4], const double Ul[NV], double Et,
                                          const double St[3], double h, double kap, double sig,
                                          const Phys& K, double Zg, ImpSys& sy, int& c2p_it) {
  double Uf[NV], Vf[NV];
  Uf[0] = Ul[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) Uf[1 + j] = St[j] - X[1 + j];
  Uf[4] = Et - X[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) Uf[5 + j] = Ul[5 + j];
  Uf[8] = X[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) Uf[9 + j] = X[1 + j];
  int it = 0;
  double Z = 0.0, lw[2];
  if (c2p(Uf, K, Zg, Vf, Z, it, lw) != 0) { c2p_it += it; return false; }
  c2p_it += it;
  sy.Z = Z;
  const double rho = Vf[0], p = Vf[4];
  const double iW = lw[1];
  const double W = 1.0 / iW;
  double u[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) u[j] = W * Vf[1 + j];
  const double T = (K.t_coeff * p) / rho;
  const double T2 = T * T;
  const double aT4 = K.a_rad * (T2 * T2);
  const double E = X[0];
  const double F[3] = {X[1], X[2], X[3]};
  const double FF = (F[0] * F[0] + F[1] * F[1]) + F[2] * F[2];
  const double f2 = FF / (E * E);
  double t = 4.0 - 3.0 * f2;
  t = (t > 0.0) ? t : 0.0;
  const double xi = (3.0 + 4.0 * f2) / (5.0 + 2.0 * sqrt(t));
  const double ca = 0.5 * (1.0 - xi);
  const double cb = 0.5 * (3.0 * xi - 1.0);
  double Dm[3][3];
  if (FF >= kMinNormal) {
    const double iFF = 1.0 / FF;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double nn = (F[i] * F[j]) * iFF;
        Dm[i][j] = (i == j) ? ca + cb * nn : cb * nn;
      }
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Dm[i][j] = (i == j) ? ca : 0.0;
  }
  double Du[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Du[i] = (Dm[i][0] * u[0] + Dm[i][1] * u[1]) + Dm[i][2] * u[2];
  const double uDu = (u[0] * Du[0] + u[1] * Du[1]) + u[2] * Du[2];
  const double W2 = W * W;
  const double hr = h * rho;
  const double hrW = hr * W;
  const double ks = kap + sig;
  sy.C[0][0] = 1.0 - hrW * (sig * ((W2 - 1.0) + uDu) - kap);
  const double c1 = kap - sig * (2.0 * W2 - 1.0);
#pragma unroll
  for (int j = 0; j < 3; ++j) sy.C[0][1 + j] = -((hr * u[j]) * c1);
  const double c2 = sig * (W2 + uDu);
#pragma unroll
  for (int i = 0; i < 3; ++i) sy.C[1 + i][0] = -(hr * (ks * Du[i] + c2 * u[i]));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double g = 2.0 * ((sig * u[i]) * u[j]);
      sy.C[1 + i][1 + j] = (i == j) ? 1.0 + hrW * (ks + g) : hrW * g;
    }
  const double em = (hr * kap) * aT4;
  sy.b[0] = Ul[8] + W * em;
#pragma unroll
  for (int i = 0; i < 3; ++i) sy.b[1 + i] = Ul[9 + i] + u[i] * em;
  return true;
}

__device__ __forceinline__ void imp_residual(const ImpSys& sy, const double X[4], double R[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
    R[i] = (((sy.C[i][0] * X[0] + sy.C[i][1] * X[1]) + sy.C[i][2] * X[2]) + sy.C[i][3] * X[3]) - sy.b[i];
}

__device__ __forceinline__ double vmaxabs4(const double a[4]) {
  return dmax(dmax(dabs(a[0]), dabs(a[1])), dmax(dabs(a[2]), dabs(a[3])));
}

// The implicit solve runs in two phases that together give one cell's result.
// Phase 1 is the paper's Picard iteration X^{m+1} = C(X^m)^{-1} b(X^m) from
// the explicit state X*, stopped once its update grows; phase 2 is Newton on
// C(X) X - b(X) (forward-difference Jacobian, step halving) from X*, for the
// cells phase 1 did not converge. The |F_r| <= E_r limit is applied to the
// explicit radiation state first (keeping S + F_r), and to the result.
struct ImpIn {
  double Ul[NV];  // explicit state with the radiation flux limited
  double Et, St[3];
};

// A non-positive explicit E_r fails the cell, or, with e_floor > 0, is raised
// to e_floor keeping tau + E_r and S + F_r (the gas pays; `floored` is set).
__device__ __forceinline__ bool imp_prepare(const double Us[NV], const Phys& K, ImpIn& in, bool& floored) {
  in.Et = Us[4] + Us[8];
#pragma unroll
  for (int j = 0; j < 3; ++j) in.St[j] = Us[1 + j] + Us[9 + j];
#pragma unroll
  for (int q = 0; q < NV; ++q) in.Ul[q] = Us[q];
  floored = false;
  if (!(in.Ul[8] > 0.0)) {
    if (K.e_floor > 0.0 && isfinite(in.Ul[8])) {
      in.Ul[8] = K.e_floor;
      floored = true;
    } else {
      return false;
    }
  }
  const double FF = (in.Ul[9] * in.Ul[9] + in.Ul[10] * in.Ul[10]) + in.Ul[11] * in.Ul[11];
  if (FF > in.Ul[8] * in.Ul[8]) {
    const double r = in.Ul[8] / sqrt(FF);
#pragma unroll
    for (int j = 0; j < 3; ++j) in.Ul[9 + j] = in.Ul[9 + j] * r;
  }
  return true;
}

__device__ __forceinline__ void imp_finish(double X[4], const double Us[NV], const ImpIn& in, double Un[NV]) {
  const double FF = (X[1] * X[1] + X[2] * X[2]) + X[3] * X[3];
  if (FF > X[0] * X[0]) {
    const double r = X[0] / sqrt(FF);
#pragma unroll
    for (int j = 0; j < 3; ++j) X[1 + j] = X[1 + j] * r;
  }
  Un[0] = Us[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) Un[1 + j] = in.St[j] - X[1 + j];
  Un[4] = in.Et - X[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) Un[5 + j] = Us[5 + j];
  Un[8] = X[0];
#pragma unroll
  for (int j = 0; j < 3; ++j) Un[9 + j] = X[1 + j];
}

enum { IMP_DONE = 0, IMP_FAILED = 1, IMP_NEED_NEWTON = 2 };

// Phase 1, the paper's Picard iteration from X* (recovery warm start Zg0,
// the stage cell's Z). IMP_DONE: Un holds the result; IMP_FAILED: Un = Us;
// IMP_NEED_NEWTON: phase 2 must finish the cell from X0 (recovery warm start
// Z0): the last Picard iterate if Picard was still contracting at its cap,
// else X* with Zg0. its: Picard solves done.
__device__ __forceinline__ int picard_run(const double Us[NV], const ImpIn& in, double h, double kap, double sig,
                                          const Phys& K, double Zg0, double Un[NV], double X0[4], double& Z0,
                                          int& its) {
  ImpSys sy;
  int c2p_it = 0;
  double X[4] = {in.Ul[8], in.Ul[9], in.Ul[10], in.Ul[11]};
  double Zg = Zg0, dlast = 0.0, dprev = 0.0;
  bool conv = false, built = false, capped = false, have = false;
  its = 0;
  const int npic = (K.imp_method == 1) ? 0 : ((K.imp_method == 2) ? K.imp_maxit : K.imp_picard_it);
  for (int m = 0; m <= npic; ++m) {
    built = imp_build(X, in.Ul, in.Et, in.St, h, kap, sig, K, Zg, sy, c2p_it);
    if (!built) break;
    Zg = sy.Z;
    if (m == 0) have = true;
    if (m == npic) { capped = true; break; }
    if (m > 1 && K.imp_method == 0 && dlast > dprev) break;
    double A[4][4], bb[4], Xn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      bb[i] = sy.b[i];
#pragma unroll
      for (int j = 0; j < 4; ++j) A[i][j] = sy.C[i][j];
    }
    if (!solve4(A, bb, Xn)) break;
    ++its;
    if (!(Xn[0] > 0.0) || !isfinite(Xn[0]) || !isfinite(Xn[1]) || !isfinite(Xn[2]) || !isfinite(Xn[3])) break;
    double dd[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { dd[i] = Xn[i] - X[i]; X[i] = Xn[i]; }
    dprev = dlast;
    dlast = vmaxabs4(dd);
    // converged once the update is below tolerance; the system is not built
    // again at the accepted iterate
    if (dlast <= K.imp_tol * vmaxabs4(X)) { conv = true; break; }
  }
  if (conv) {
    imp_finish(X, Us, in, Un);
    return IMP_DONE;
  }
  if (have && K.imp_method != 2) {
    const bool from_picard = built && capped && npic > 1 && dlast < dprev;
#pragma unroll
    for (int i = 0; i < 4; ++i) X0[i] = from_picard ? X[i] : in.Ul[8 + i];
    Z0 = from_picard ? Zg : Zg0;
    return IMP_NEED_NEWTON;
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) Un[q] = Us[q];
  return IMP_FAILED;
}

// Phase 2, Newton on C(X) X - b(X) from X0 (warm start Z0), on a quad of 4
// lanes (lanes 4k..4k+3 of a wave, all on the same cell and all active
// together). Each Newton iteration is a column round, where lane j evaluates
// the system at X + del e_j for Jacobian column j (forward difference, step
// 1e-8 max(|X|, |b_i/C_ii|)), followed by line-search rounds, where lane j
// evaluates it at X + 2^-(j + 4r) dX in round r; the quad then shares the
// results. The selections are those of one lane doing it all in order
// (columns 0..3, stopping at the first that fails; the first acceptable step
// of 1, 1/2, 1/4, ...), so the result is the same bit for bit. Every round
// evaluates one point per lane through the same code (one recovery and
// system build), which keeps the register footprint of a single evaluation.
// Returns true on convergence with the root in X (before imp_finish).
__device__ __forceinline__ double quad_get(double v, int base, int k) { return __shfl(v, base + k, 64); }

__device__ __forceinline__ bool implicit_newton_quad(const ImpIn& in, double h, double kap, double sig,
                                                     const Phys& K, double X[4], double Z0, int& iters) {
  const int lane = threadIdx.x & 63;
  const int j = lane & 3;
  const int base = lane & ~3;
  enum { kInit = 0, kColumns = 1, kSearch = 2 };
  int phase = kInit, round = 0, n = 0, it = 0;
  double R[4] = {0.0, 0.0, 0.0, 0.0}, bd[4] = {0.0, 0.0, 0.0, 0.0}, dX[4] = {0.0, 0.0, 0.0, 0.0};
  double Zg = Z0, sc = 0.0, del = 0.0, lam0 = 1.0, rn = 0.0, dn = 0.0, sprev = 0.0;
  bool conv = false;
  // every round advances `round` (at most 3 per iteration) or `n` (at most
  // imp_maxit), so the loop ends
  while (true) {
    // this lane's evaluation point
    double Xe[4] = {X[0], X[1], X[2], X[3]};
    double lam = lam0;
    bool valid = true;
    if (phase == kColumns) {
#pragma unroll
      for (int k = 0; k < 4; ++k) Xe[k] = (k == j) ? X[k] + del : X[k];
    } else if (phase == kSearch) {
      for (int k = 0; k < j; ++k) lam = 0.5 * lam;
#pragma unroll
      for (int i = 0; i < 4; ++i) Xe[i] = X[i] + lam * dX[i];
      valid = Xe[0] > 0.0;
    }
    double Re[4] = {0.0, 0.0, 0.0, 0.0}, be[4] = {0.0, 0.0, 0.0, 0.0}, Ze = 0.0;
    bool ok = false;
    if (valid) {
      ImpSys sy;
      int c2p_it = 0;
      ok = imp_build(Xe, in.Ul, in.Et, in.St, h, kap, sig, K, Zg, sy, c2p_it);
      if (ok) {
        imp_residual(sy, Xe, Re);
        if (phase != kColumns) {
#pragma unroll
          for (int i = 0; i < 4; ++i) be[i] = sy.b[i] / sy.C[i][i];
          Ze = sy.Z;
        }
      }
    }
    bool start = false;
    if (phase == kInit) {
      // all four lanes evaluated X0
      if (!ok) break;
#pragma unroll
      for (int i = 0; i < 4; ++i) { R[i] = Re[i]; bd[i] = be[i]; }
      Zg = Ze;
      start = true;
    } else if (phase == kColumns) {
      double col[4] = {0.0, 0.0, 0.0, 0.0};
      if (ok) {
#pragma unroll
        for (int i = 0; i < 4; ++i) col[i] = (Re[i] - R[i]) / del;
      }
      const double okc = ok ? 1.0 : 0.0;
      // the sequential rule stops at the first failing column: any failure breaks
      const double okall = quad_get(okc, base, 0) * quad_get(okc, base, 1) * quad_get(okc, base, 2) *
                           quad_get(okc, base, 3);
      if (okall == 0.0) break;
      double J[4][4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) J[i][k] = quad_get(col[i], base, k);
      double nR[4] = {-R[0], -R[1], -R[2], -R[3]};
      if (!solve4(J, nR, dX)) break;
      rn = vmaxabs4(R);
      dn = vmaxabs4(dX);
      lam0 = 1.0;
      round = 0;
      phase = kSearch;
    } else {
      const double good = (ok && (vmaxabs4(Re) < rn || lam * dn <= 1e-10 * sc)) ? 1.0 : 0.0;
      // first acceptable lane in order 0..3
      int pick = -1;
#pragma unroll
      for (int k = 3; k >= 0; --k)
        if (quad_get(good, base, k) != 0.0) pick = k;
      if (pick < 0) {
        if (++round == 3) break;
        lam0 = 0.5 * (0.5 * (0.5 * (0.5 * lam0)));
      } else {
        double stp[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double xt = quad_get(Xe[i], base, pick);
          stp[i] = xt - X[i];
          X[i] = xt;
          R[i] = quad_get(Re[i], base, pick);
          bd[i] = quad_get(be[i], base, pick);
        }
        Zg = quad_get(Ze, base, pick);
        const double sn = vmaxabs4(stp);
        if (sn <= K.imp_tol * vmaxabs4(X)) { conv = true; break; }
        if (n > 0 && sn <= 1e-9 * sc && sn >= sprev) { conv = true; break; }
        sprev = sn;
        ++n;
        start = true;
      }
    }
    if (start) {
      // next Newton iteration: its difference step
      if (n >= K.imp_maxit) break;
      ++it;
      sc = dmax(vmaxabs4(X), vmaxabs4(bd));
      del = 1e-8 * sc;
      phase = kColumns;
    }
  }
  iters = it;
  return conv;
}

// ---------------------------------------------------------------------------
// The outer M1 eigenvalues lambda_r1 <= lambda_r3 in direction d (eqs.
// lam1-lam3): f = |F|/E capped at 1, cos(theta) = F_d/|F| (0 when F = 0).
template <int d, typename R = double>
__device__ __forceinline__ void rad_speeds(const R V[NV], R& l1, R& l3) {
  const R E = V[8];
  const R FF = (V[9] * V[9] + V[10] * V[10]) + V[11] * V[11];
  R f = R(0), cth = R(0);
  if (FF > R(0)) {
    const R Fn = sqrt(FF);
    const R fe = Fn / E;
    f = (fe < R(1)) ? fe : R(1);
    cth = V[9 + d] / Fn;
  }
  const R f2 = f * f;
  const R r43 = R(4) - R(3) * f2;
  const R sr = sqrt(r43);
  R zz = (R(2) / R(3)) * (r43 - sr) + (R(2) * (cth * cth)) * ((R(2) - f2) - sr);
  zz = (zz > R(0)) ? zz : R(0);
  const R zeta = sqrt(zz);
  l1 = (f * cth - zeta) / sr;
  l3 = (f * cth + zeta) / sr;
}

// ---------------------------------------------------------------------------
// Signal speed bound of a cell in direction d: relativistic fast-speed bound
// with a^2 = cs^2 + ca^2 - cs^2 ca^2 for the fluid, M1 eigenvalues
// lambda_r1, lambda_r3 (eqs. lam1-lam3) for the radiation.
template <int d>
__device__ __forceinline__ double cell_speed(const double V[NV], const Aux& a, const Phys& K) {
  const double rho = V[0], p = V[4];
  const double rhoh = rho + K.g1 * p;
  const double cs2 = (K.gamma * p) / rhoh;
  const double ca2 = a.bb / (rhoh + a.bb);
  const double a2 = (cs2 + ca2) - cs2 * ca2;
  const double v2 = 1.0 - a.l2;
  const double vd = V[1 + d];
  const double den = 1.0 - v2 * a2;
  double disc = (a2 * a.l2) * (den - (vd * vd) * (1.0 - a2));
  disc = (disc > 0.0) ? disc : 0.0;
  const double sq = sqrt(disc);
  const double lp = (vd * (1.0 - a2) + sq) / den;
  const double lm = (vd * (1.0 - a2) - sq) / den;
  double s = dmax(dabs(lp), dabs(lm));
  double l1, l3;
  rad_speeds<d>(V, l1, l3);
  s = dmax(s, dmax(dabs(l1), dabs(l3)));
  return s;
}

// ---------------------------------------------------------------------------
// Rad-HLL face flux (Section 3.2, Radiative HLL): the HLL flux of eq.
// F^hll, applied to the magnetofluid rows 0..7 and to the radiation rows
// 8..11 with the signal speeds of each block of the Jacobian (eq. jacobian).
//
// Magnetofluid speeds: the smallest and largest roots of the RMHD quartic
// (Anile 1989), Q(l) = w (1 - cs^2) a^4 - (1 - l^2)[(w cs^2 + |b|^2) a^2 -
// cs^2 B~^2] with a = W (l - v_d), B~ = b^d - l b^0, w = rho h. All roots are
// real and inside (-1, 1), so Laguerre's iteration for degree 4,
// l <- l - 4/(G +- sqrt(3 (4H - G^2))), G = Q'/Q, H = G^2 - Q''/Q, moves
// monotonically from l = +1 (l = -1) down (up) to the largest (smallest) root,
// cubically near it; it stops when Q is no longer > 0, when an iterate stalls,
// or after kQuartIt steps, and an early stop only widens the fan. The four
// roots of a face (min and max of the L and R states) advance together in one
// straight-line loop, each frozen once its own test stops it: the values are
// those of four separate loops, with four independent dependency chains for
// the FP64 pipeline.
//
// Radiation speeds: lambda_r1 and lambda_r3 (eqs. lam1-lam3) of both states,
// limited to |lambda| <= 4/(3 tau) (eq. limits) with tau the larger optical
// depth of the two cells next to the face. A fan of zero width takes the mean
// of F_L and F_R.
constexpr int kQuartIt = 20;

template <typename R>
struct QuartIn {
  R w1cs, wcsb, cs2, W2, vd, bd, b0;
};

// Q, Q', Q'' at l from the factored form (A = a^2, br = (w cs^2 + |b|^2) A -
// cs^2 B~^2, om = 1 - l^2, Q = w (1 - cs^2) A^2 - om br).
template <typename R>
__device__ __forceinline__ void quartic(const QuartIn<R>& q, R l, R& Q, R& dQ, R& d2Q) {
  const R x = l - q.vd;
  const R A = q.W2 * (x * x);
  const R Bt = q.bd - l * q.b0;
  const R om = R(1) - l * l;
  const R br = q.wcsb * A - q.cs2 * (Bt * Bt);
  Q = q.w1cs * (A * A) - om * br;
  const R dA = R(2) * (q.W2 * x);
  const R dbr = q.wcsb * dA + R(2) * (q.cs2 * (q.b0 * Bt));
  const R d2br = q.wcsb * (R(2) * q.W2) - R(2) * (q.cs2 * (q.b0 * q.b0));
  dQ = ((R(2) * q.w1cs) * (A * dA) + (R(2) * l) * br) - om * dbr;
  d2Q = (((R(2) * q.w1cs) * (dA * dA + A * (R(2) * q.W2)) + R(2) * br) + (R(4) * l) * dbr) - om * d2br;
}

template <int d, typename R>
__device__ __forceinline__ QuartIn<R> quartic_in(const R V[NV], const AuxT<R>& a, R gamma, R g1) {
  QuartIn<R> q;
  const R w = V[0] + g1 * V[4];
  q.cs2 = (gamma * V[4]) / w;
  q.w1cs = w * (R(1) - q.cs2);
  q.wcsb = w * q.cs2 + a.bb;
  q.W2 = a.W * a.W;
  q.vd = V[1 + d];
  q.bd = a.b[d];
  q.b0 = a.b0;
  return q;
}

// lam[0], lam[1]: min and max of state L; lam[2], lam[3]: of state R.
template <typename R>
__device__ __forceinline__ void fast_speeds2(const QuartIn<R>& qL, const QuartIn<R>& qR, R lam[4]) {
  bool run[4] = {true, true, true, true};
  lam[0] = R(-1); lam[1] = R(1); lam[2] = R(-1); lam[3] = R(1);
  for (int it = 0; it < kQuartIt; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const bool down = (r & 1) != 0;  // the largest root is approached from above
      R Q, dQ, d2Q;
      quartic<R>((r < 2) ? qL : qR, lam[r], Q, dQ, d2Q);
      const R iQ = R(1) / Q;
      const R G = dQ * iQ;
      const R H = G * G - d2Q * iQ;
      R t = R(3) * (R(4) * H - G * G);
      t = (t > R(0)) ? t : R(0);
      const R sq = sqrt(t);
      const R ln = lam[r] - R(4) / (down ? (G + sq) : (G - sq));
      run[r] = run[r] && (Q > R(0)) && (down ? (ln < lam[r]) : (ln > lam[r]));
      lam[r] = run[r] ? ln : lam[r];
    }
    if (!(run[0] || run[1] || run[2] || run[3])) break;
  }
}

template <typename R>
__device__ __forceinline__ void hll_rows(const R* FL, const R* FR, const R* UL, const R* UR, R lL, R lR, int n,
                                         R* Fh) {
#pragma unroll
  for (int q = 0; q < n; ++q) {
    const R h = ((lR * FL[q] - lL * FR[q]) + (lR * lL) * (UR[q] - UL[q])) / (lR - lL);
    const R m = R(0.5) * (FL[q] + FR[q]);
    Fh[q] = (lL > R(0)) ? FL[q] : ((lR < R(0)) ? FR[q] : ((lR > lL) ? h : m));
  }
}

template <int d, typename R = double>
__device__ __forceinline__ void hll_face(const R VL[NV], const R VR[NV], R tauL, R tauR, const Phys& K, R Fh[NV]) {
  const R g1 = R(K.g1), gam = R(K.gamma);
  // radiation block: its variables are both primitive and conserved
  {
    R r1L, r3L, r1R, r3R;
    rad_speeds<d, R>(VL, r1L, r3L);
    rad_speeds<d, R>(VR, r1R, r3R);
    const R tm = (tauL > tauR) ? tauL : tauR;
    const R lim = R(4) / (R(3) * tm);
    R FL[4], FR[4];
    flux_rad<d, R>(VL + 8, FL);
    flux_rad<d, R>(VR + 8, FR);
    const R mn = (r1L < r1R) ? r1L : r1R, mx = (r3L > r3R) ? r3L : r3R;
    const R nlim = -lim;
    hll_rows<R>(FL, FR, VL + 8, VR + 8, (mn > nlim) ? mn : nlim, (mx < lim) ? mx : lim, 4, Fh + 8);
  }
  // magnetofluid block
  AuxT<R> aL, aR;
  prim_aux<R>(VL, g1, aL);
  prim_aux<R>(VR, g1, aR);
  R lam[4];
  fast_speeds2<R>(quartic_in<d, R>(VL, aL, gam, g1), quartic_in<d, R>(VR, aR, gam, g1), lam);
  R UL[8], UR[8], FL[8], FR[8];
  p2c8<R>(VL, aL, UL);
  flux_mhd<d, R>(VL, aL, FL);
  p2c8<R>(VR, aR, UR);
  flux_mhd<d, R>(VR, aR, FR);
  const R lo = (lam[0] < lam[2]) ? lam[0] : lam[2], hi = (lam[1] > lam[3]) ? lam[1] : lam[3];
  hll_rows<R>(FL, FR, UL, UR, lo, hi, 8, Fh);
}

}  // namespace rr
