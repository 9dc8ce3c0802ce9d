// Host driver, kernels and C ABI of the RRMHD + M1 hot path on gfx950.
//
// One IMEX step (Section 3.1 of Lopez-Miralles, Marti & Perucho, CPC,
// arXiv 2212.00370) is, per Runge-Kutta stage:
//   k_prims   : cell primitive recovery of the stage state -> V, D(kappa+sigma)
//   k_faces   : per face of every direction, PLM + PVM-int (eps differences or
//               exact JVP) or Rad-HLL flux (Section 3.2) -> F^_d
//   k_update  : U* = a0 U^(0) + a1 U^(s) - c dt sum_d dF^_d/dx_d (eq. explicit)
//               followed by the per-cell implicit source solve (Section 3.3)
// All kernels read and write structure-of-arrays float64 planes in HBM; one
// thread owns one face or one cell, so the step is race-free and needs no
// floating-point atomics. The CFL speed uses a per-block maximum in LDS and a
// second single-block pass (deterministic, no memset); in rrmhd_advance that
// pass is block 0 of the step's first face launch.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "rrmhd.h"
#include "rrmhd_device.hpp"

using rr::NV;
using rr::Phys;

namespace {

// One wave per workgroup: waves of the face and cell kernels take very
// different times (iteration counts vary per cell), and a wave that finishes
// frees its slot at once instead of waiting for the rest of a larger group.
#ifndef RRMHD_BLOCK
#define RRMHD_BLOCK 64
#endif
constexpr int kBlock = RRMHD_BLOCK;
static_assert(kBlock == rr::kParkLanes, "the PVM chain's LDS slots assume one-wave workgroups");
// Workgroup size of the single-block reductions over per-block partials.
constexpr int kRedBlock = 1024;
constexpr int kWave = 64;
// Minimum waves per SIMD the register allocation of the face and update
// kernels targets (a hint to the compiler). Faces: three, with the PVM
// chain's start-to-end values in LDS (FP64: 168 VGPRs and 12.5 KB LDS per
// one-wave block; mixed precision: 136 VGPRs, 6.5 KB). Update pass: two (no
// spills; its 4096 one-wave blocks at 512^2 cells fill two rounds of 2048
// slots). Newton pass: two (256 VGPRs, 8 of them spilled; at one wave per
// SIMD its work list needed two rounds of the 1024 slots late in a blast).
#ifndef RRMHD_NEWTON_WAVES
#define RRMHD_NEWTON_WAVES 2
#endif
#ifndef RRMHD_FACES_WAVES
#define RRMHD_FACES_WAVES 3
#endif
#ifndef RRMHD_FACES_WAVES_MIXED
#define RRMHD_FACES_WAVES_MIXED 3
#endif
#ifndef RRMHD_FACES_WAVES_HLL
#define RRMHD_FACES_WAVES_HLL 3
#endif
#ifndef RRMHD_FACES_WAVES_JVP
#define RRMHD_FACES_WAVES_JVP 2
#endif
#ifndef RRMHD_FACES_WAVES_JVP_MIXED
#define RRMHD_FACES_WAVES_JVP_MIXED 3
#endif
#ifndef RRMHD_UPDATE_WAVES
#define RRMHD_UPDATE_WAVES 2
#endif
// Size of the per-device scratch array of rrmhd_advance_noalloc (64 MiB: the
// workspace of grids up to about 140 000 cells, e.g. 360^2 or 1D runs).
#ifndef RRMHD_NOALLOC_SCRATCH_BYTES
#define RRMHD_NOALLOC_SCRATCH_BYTES (64ull << 20)
#endif

struct DevReport {
  unsigned long long c2p_fail, pvm_fallback, imp_fail, nonfinite, e_floor_hits;
  unsigned long long first_bad;
  unsigned int max_c2p_it, max_imp_it;
  unsigned int pad[2];
};

// Grid description used on the device.
struct GridDev {
  int ndim;
  int n[3];
  int bc_lo[3], bc_hi[3];
  long long N;              // interior cells
  long long nt;             // transverse cells of the inflow face (0 if none)
  const unsigned char* mask;
};

struct Opac {
  const double* kappa;
  const double* sigma;
  double kappa0, sigma0;
};

__device__ __forceinline__ double opac_at(const double* a, double uni, long long c) {
  return a ? a[c] : uni;
}

__device__ __forceinline__ unsigned int wave_max_u32(unsigned int v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned int w = __shfl_xor(v, o, kWave);
    v = (w > v) ? w : v;
  }
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o, kWave);
    v = (w < v) ? w : v;
  }
  return v;
}

// Accumulate per-thread failure flags into the device report. Failures are
// rare: one atomic per wave and field, only when the wave saw one. Iteration
// maxima are not updated atomically (a same-address atomic per wave
// serializes thousands of waves): each block keeps a running maximum in its
// own slot of `blkmax` (one writer per slot, launches ordered on the stream),
// folded into the report by rrmhd_report_sync.
__device__ __forceinline__ void report_add(DevReport* rep, unsigned int* blkmax, long long slot_block,
                                           unsigned long long f_c2p,
                                           unsigned long long f_pvm, unsigned long long f_imp,
                                           unsigned long long f_nf, unsigned long long bad_cell,
                                           unsigned int c2p_it, unsigned int imp_it,
                                           unsigned long long f_floor = 0, bool shared_slot = false) {
  __shared__ unsigned int red_it[2][kBlock / kWave];
  const unsigned long long s_c2p = wave_sum_u64(f_c2p);
  const unsigned long long s_pvm = wave_sum_u64(f_pvm);
  const unsigned long long s_imp = wave_sum_u64(f_imp);
  const unsigned long long s_nf = wave_sum_u64(f_nf);
  const unsigned long long s_fl = wave_sum_u64(f_floor);
  const unsigned long long s_bad = wave_min_u64(bad_cell);
  const unsigned int m_c2p = wave_max_u32(c2p_it);
  const unsigned int m_imp = wave_max_u32(imp_it);
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  if (lane == 0) {
    if (s_c2p) atomicAdd(&rep->c2p_fail, s_c2p);
    if (s_pvm) atomicAdd(&rep->pvm_fallback, s_pvm);
    if (s_imp) atomicAdd(&rep->imp_fail, s_imp);
    if (s_nf) atomicAdd(&rep->nonfinite, s_nf);
    if (s_fl) atomicAdd(&rep->e_floor_hits, s_fl);
    if (s_bad != ULLONG_MAX) atomicMin(&rep->first_bad, s_bad);
    red_it[0][wid] = m_c2p;
    red_it[1][wid] = m_imp;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int a = red_it[0][0], b = red_it[1][0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) {
      a = (red_it[0][w] > a) ? red_it[0][w] : a;
      b = (red_it[1][w] > b) ? red_it[1][w] : b;
    }
    unsigned int* slot = blkmax + 2 * (size_t)slot_block;
    if (shared_slot) {
      // a slot that another block may update at the same time
      if (a) atomicMax(&slot[0], a);
      if (b) atomicMax(&slot[1], b);
    } else {
      if (a > slot[0]) slot[0] = a;
      if (b > slot[1]) slot[1] = b;
    }
  }
}

// Map cell coordinates (c[d] possibly outside [0, n_d)) to an index into the
// stage primitives: interior cells 0..N-1, inflow cells N + t.
__device__ __forceinline__ long long map_cell(const GridDev& G, int c0, int c1, int c2, int d) {
  int c[3] = {c0, c1, c2};
  const int nd = G.n[d];
  int cd = c[d];
  if (cd < 0) {
    const int bc = G.bc_lo[d];
    if (bc == RRMHD_BC_PERIODIC) {
      cd = ((cd % nd) + nd) % nd;
    } else if (bc == RRMHD_BC_INFLOW) {
      const long long t = (d == 0) ? 0 : ((d == 1) ? (long long)c[0] : (long long)c[0] + (long long)G.n[0] * c[1]);
      if (G.mask && G.mask[t]) return G.N + t;
      cd = 0;
    } else {
      cd = 0;
    }
  } else if (cd >= nd) {
    cd = (G.bc_hi[d] == RRMHD_BC_PERIODIC) ? (cd % nd) : (nd - 1);
  }
  c[d] = cd;
  return (long long)c[0] + (long long)G.n[0] * ((long long)c[1] + (long long)G.n[1] * c[2]);
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_p2c(long long n, const double* __restrict__ V, long long sv,
                                                double* __restrict__ U, long long su, Phys K) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double v[NV], u[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = V[q * sv + c];
  rr::Aux a;
  rr::prim_aux(v, K, a);
  rr::p2c(v, a, u);
#pragma unroll
  for (int q = 0; q < NV; ++q) U[q * su + c] = u[q];
}

__global__ void __launch_bounds__(kBlock) k_c2p(long long n, const double* __restrict__ U, long long su,
                                                double* __restrict__ V, long long sv, Phys K, DevReport* rep, unsigned int* blkmax) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long fail = 0, bad = ULLONG_MAX;
  unsigned int its = 0;
  if (c < n) {
    double u[NV], v[NV], Z = 0.0;
    int it = 0;
#pragma unroll
    for (int q = 0; q < NV; ++q) u[q] = U[q * su + c];
    if (rr::c2p(u, K, 0.0, v, Z, it) != 0) {
      rr::c2p_fallback(u, K, v);
      fail = 1;
      bad = (unsigned long long)c;
    }
    its = (unsigned int)it;
#pragma unroll
    for (int q = 0; q < NV; ++q) V[q * sv + c] = v[q];
  }
  report_add(rep, blkmax, blockIdx.x, fail, 0, 0, 0, bad, its, 0);
}

// Block maximum of per-thread signal speeds s -> partial[lb] (wave butterfly,
// then the waves in order).
__device__ __forceinline__ void block_max_to(double s, double* __restrict__ partial, long long lb) {
  __shared__ double red[kBlock / kWave];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s = rr::dmax(s, __shfl_xor(s, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) m = rr::dmax(m, red[w]);
    partial[lb] = m;
  }
}

// The block's maximum of s >= 0 (or NaN) folded into *slot by an atomic
// maximum of the bit patterns (their order is that of the values for
// non-negative doubles); *slot starts at +0.
__device__ __forceinline__ void block_max_atomic(double s, double* slot) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s = rr::dmax(s, __shfl_xor(s, o, kWave));
  static_assert(kBlock == kWave, "one wave per block");
  if (threadIdx.x == 0) {
    const double w = (s == 0.0) ? 0.0 : s;  // -0 as +0
    atomicMax((unsigned long long*)slot, (unsigned long long)__double_as_longlong(w));
  }
}

// Largest signal speed of one cell with primitives v over the active directions.
__device__ __forceinline__ double cell_signal_speed(const GridDev& G, const double v[NV], const Phys& K) {
  rr::Aux a;
  rr::prim_aux(v, K, a);
  double s = rr::dmax(0.0, rr::cell_speed<0>(v, a, K));
  if (G.ndim > 1) s = rr::dmax(s, rr::cell_speed<1>(v, a, K));
  if (G.ndim > 2) s = rr::dmax(s, rr::cell_speed<2>(v, a, K));
  return s;
}

// Stage primitives: interior cells (c < N) from U, inflow cells from inflow_U.
// Vp: [12][Np], taup: [Np] = D (kappa + sigma). lb: block index within the
// simulation. Cell 0 also clears the Newton work-list counter wcount (if set).
// With a non-null `partial`, the block also writes the maximum signal speed of
// its interior cells to partial[lb] (lb < blocks over the N interior cells);
// the recovered primitives are those a separate signal-speed pass computes.
__device__ __forceinline__ void prims_block(long long lb, const GridDev& G, const double* __restrict__ U,
                                            long long su, const double* __restrict__ inU, const Opac& op,
                                            double* __restrict__ Vp, double* __restrict__ taup, long long np,
                                            const Phys& K, DevReport* rep, unsigned int* blkmax,
                                            unsigned long long* wcount, double* __restrict__ Zc,
                                            double* __restrict__ partial = nullptr) {
  const long long c = lb * kBlock + threadIdx.x;
  if (c == 0 && wcount) *wcount = 0;
  unsigned long long fail = 0, bad = ULLONG_MAX;
  unsigned int its = 0;
  double s = 0.0;
  if (c < G.N + G.nt) {
    double u[NV], v[NV], Z = 0.0;
    int it = 0;
    long long oc;  // cell whose opacity applies
    if (c < G.N) {
#pragma unroll
      for (int q = 0; q < NV; ++q) u[q] = U[q * su + c];
      oc = c;
    } else {
      const long long t = c - G.N;
#pragma unroll
      for (int q = 0; q < NV; ++q) u[q] = inU[q * G.nt + t];
      oc = (G.ndim == 1) ? 0 : t;
    }
    if (rr::c2p(u, K, 0.0, v, Z, it) != 0) {
      rr::c2p_fallback(u, K, v);
      Z = 0.0;
      if (c < G.N) { fail = 1; bad = (unsigned long long)c; }
    }
    if (c < G.N) {
      its = (unsigned int)it;
      Zc[c] = Z;
      if (partial) s = cell_signal_speed(G, v, K);
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) Vp[q * np + c] = v[q];
    taup[c] = u[0] * (opac_at(op.kappa, op.kappa0, oc) + opac_at(op.sigma, op.sigma0, oc));
  }
  report_add(rep, blkmax, lb, fail, 0, 0, 0, bad, its, 0);
  if (partial && lb * kBlock < G.N) block_max_to(s, partial, lb);
}

__global__ void __launch_bounds__(kBlock) k_prims(GridDev G, const double* __restrict__ U, long long su,
                                                  const double* __restrict__ inU, Opac op,
                                                  double* __restrict__ Vp, double* __restrict__ taup,
                                                  long long np, Phys K, DevReport* rep, unsigned int* blkmax,
                                                  unsigned long long* wcount, double* Zc) {
  prims_block(blockIdx.x, G, U, su, inU, op, Vp, taup, np, K, rep, blkmax, wcount, Zc);
}

// Stage primitives of the first stage and the signal-speed block maxima in one
// pass (the step's time step is then formed on the device).
__global__ void __launch_bounds__(kBlock) k_prims_speed(GridDev G, const double* __restrict__ U, long long su,
                                                        const double* __restrict__ inU, Opac op,
                                                        double* __restrict__ Vp, double* __restrict__ taup,
                                                        long long np, Phys K, DevReport* rep, unsigned int* blkmax,
                                                        unsigned long long* wcount, double* Zc,
                                                        double* __restrict__ partial) {
  prims_block(blockIdx.x, G, U, su, inU, op, Vp, taup, np, K, rep, blkmax, wcount, Zc, partial);
}

struct FaceArgs {
  const double* Vp;
  const double* taup;
  long long np;
  double* Fh[3];
  long long nf[3];
  long long nb[3];   // blocks per direction
  double dx[3];
  // Constrained transport: plane d of bface (stride bs) holds the normal
  // field of the face on the lower side of each cell along d; nullptr: none.
  const double* bface;
  long long bs;
};

// Constrained transport: both states of a d-face take the face's own normal
// field (face n_d is face 0 of the periodic grid).
template <int d, typename T>
__device__ __forceinline__ void face_normal_field(const GridDev& G, const FaceArgs& A, const int c[3], T VL[NV],
                                                  T VR[NV]) {
  int cc[3] = {c[0], c[1], c[2]};
  if (cc[d] == G.n[d]) cc[d] = 0;
  const double bn = A.bface[d * A.bs + ((long long)cc[0] + (long long)G.n[0] * ((long long)cc[1] + (long long)G.n[1] * cc[2]))];
  VL[5 + d] = (T)bn;
  VR[5 + d] = (T)bn;
}

// One face of direction d: PLM on the 4-cell stencil, |F_r| <= E_r,
// then the PVM-int flux with beta from the two adjacent cells. REC >= 0 fixes
// the limiter at compile time (the launch picks the MinMod copy when K.recon
// is MinMod); REC < 0 reads K.recon.
template <int d, int REC, int SOLVER>
__device__ __forceinline__ void face_body(const GridDev& G, const FaceArgs& A, long long f, const Phys& K,
                                          unsigned long long& fb, unsigned int& its) {
  int fn0 = G.n[0], fn1 = G.n[1];
  if (d == 0) fn0 += 1;
  if (d == 1) fn1 += 1;
  int c[3];
  {
    // 32-bit index arithmetic: face counts stay below 2^32 (grid_valid)
    const unsigned int fu = (unsigned int)f, u0 = (unsigned int)fn0, u1 = (unsigned int)fn1;
    const unsigned int q0 = fu / u0;
    c[0] = (int)(fu - q0 * u0);
    const unsigned int q1 = q0 / u1;
    c[1] = (int)(q0 - q1 * u1);
    c[2] = (int)q1;
  }
  double Vs[4][NV];
  double tp[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[d] = c[d] - 2 + s;
    const long long m = map_cell(G, cc[0], cc[1], cc[2], d);
#pragma unroll
    for (int q = 0; q < NV; ++q) Vs[s][q] = A.Vp[q * A.np + m];
    tp[s] = A.taup[m];
  }
  double sa[NV], sb[NV];
  rr::cell_slopes<double, REC>(Vs[0], Vs[1], Vs[2], K.recon, sa);
  rr::cell_slopes<double, REC>(Vs[1], Vs[2], Vs[3], K.recon, sb);
  double VL[NV], VR[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) { VL[q] = Vs[1][q] + 0.5 * sa[q]; VR[q] = Vs[2][q] - 0.5 * sb[q]; }
  rr::limit_rad_flux(VL);
  rr::limit_rad_flux(VR);
  if (A.bface) face_normal_field<d>(G, A, c, VL, VR);
  const double tauL = tp[1] * A.dx[d], tauR = tp[2] * A.dx[d];
  double Fq[NV];
  int fallback = 0, cit = 0;
  if constexpr (SOLVER == RRMHD_SOLVER_HLL) rr::hll_face<d>(VL, VR, tauL, tauR, K, Fq);
  else if constexpr (SOLVER == RRMHD_SOLVER_PVM_JVP) rr::pvm_face_jvp<d>(VL, VR, tauL, tauR, K, Fq, fallback, cit);
  else rr::pvm_face<d>(VL, VR, tauL, tauR, K, Fq, fallback, cit);
  double* out = A.Fh[d];
  const long long nf = A.nf[d];
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q * nf + f] = Fq[q];
  fb = (unsigned long long)fallback;
  its = (unsigned int)cit;
}

// Mixed precision: the same stencil in FP32 (FP64 recoveries inside), FP32
// fluxes out.
template <int d, int REC, int SOLVER>
__device__ __forceinline__ void face_body_mixed(const GridDev& G, const FaceArgs& A, long long f, const Phys& K,
                                                unsigned long long& fb, unsigned int& its) {
  int fn0 = G.n[0], fn1 = G.n[1];
  if (d == 0) fn0 += 1;
  if (d == 1) fn1 += 1;
  int c[3];
  {
    // 32-bit index arithmetic: face counts stay below 2^32 (grid_valid)
    const unsigned int fu = (unsigned int)f, u0 = (unsigned int)fn0, u1 = (unsigned int)fn1;
    const unsigned int q0 = fu / u0;
    c[0] = (int)(fu - q0 * u0);
    const unsigned int q1 = q0 / u1;
    c[1] = (int)(q0 - q1 * u1);
    c[2] = (int)q1;
  }
  float Vs[4][NV];
  float tp[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int cc[3] = {c[0], c[1], c[2]};
    cc[d] = c[d] - 2 + s;
    const long long m = map_cell(G, cc[0], cc[1], cc[2], d);
#pragma unroll
    for (int q = 0; q < NV; ++q) Vs[s][q] = (float)A.Vp[q * A.np + m];
    tp[s] = (float)A.taup[m];
  }
  float sa[NV], sb[NV];
  rr::cell_slopes<float, REC>(Vs[0], Vs[1], Vs[2], K.recon, sa);
  rr::cell_slopes<float, REC>(Vs[1], Vs[2], Vs[3], K.recon, sb);
  float VL[NV], VR[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) { VL[q] = Vs[1][q] + 0.5f * sa[q]; VR[q] = Vs[2][q] - 0.5f * sb[q]; }
  rr::limit_rad_flux<float>(VL);
  rr::limit_rad_flux<float>(VR);
  if (A.bface) face_normal_field<d>(G, A, c, VL, VR);
  const float dxd = (float)A.dx[d];
  float Fq[NV];
  int fallback = 0, cit = 0;
  if constexpr (SOLVER == RRMHD_SOLVER_PVM_JVP)
    rr::pvm_face_jvp_mixed<d>(VL, VR, tp[1] * dxd, tp[2] * dxd, K, Fq, fallback, cit);
  else if constexpr (SOLVER == RRMHD_SOLVER_HLL)
    rr::hll_face<d, float>(VL, VR, tp[1] * dxd, tp[2] * dxd, K, Fq);
  else
    rr::pvm_face_mixed<d>(VL, VR, tp[1] * dxd, tp[2] * dxd, K, Fq, fallback, cit);
  float* out = (float*)A.Fh[d];
  const long long nf = A.nf[d];
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q * nf + f] = Fq[q];
  fb = (unsigned long long)fallback;
  its = (unsigned int)cit;
}

// Face fluxes of all directions in one launch: blocks [0, nb0) take x faces,
// the next nb1 blocks y faces, then z. The direction is uniform per block.
// MIXED selects the mixed-precision stencil (FP32 fluxes out).
template <bool MIXED, int REC, int SOLVER = RRMHD_SOLVER_PVM>
__device__ __forceinline__ void faces_block(long long lb, const GridDev& G, const FaceArgs& A, const Phys& K,
                                            DevReport* rep, unsigned int* blkmax) {
  long long b = lb;
  int d = 0;
  if (b >= A.nb[0]) {
    b -= A.nb[0];
    d = 1;
    if (b >= A.nb[1]) { b -= A.nb[1]; d = 2; }
  }
  const long long f = b * kBlock + threadIdx.x;
  unsigned long long fb = 0;
  unsigned int its = 0;
  if (f < A.nf[d]) {
    if constexpr (!MIXED) {
      if (d == 0) face_body<0, REC, SOLVER>(G, A, f, K, fb, its);
      else if (d == 1) face_body<1, REC, SOLVER>(G, A, f, K, fb, its);
      else face_body<2, REC, SOLVER>(G, A, f, K, fb, its);
    } else {
      if (d == 0) face_body_mixed<0, REC, SOLVER>(G, A, f, K, fb, its);
      else if (d == 1) face_body_mixed<1, REC, SOLVER>(G, A, f, K, fb, its);
      else face_body_mixed<2, REC, SOLVER>(G, A, f, K, fb, its);
    }
  }
  report_add(rep, blkmax, lb, 0, fb, 0, 0, ULLONG_MAX, its, 0);
}

// The step's time step from the signal-speed block maxima of the previous
// pass: s_max = min(max partial, 1), dt = (cfl dx_min) / s_max into sd[1]
// (and dt_out[k] when given); a dt that is not finite and >= 0 becomes 0 and
// is counted as non-finite. partial == nullptr: nothing to do.
struct DtReduce {
  const double* partial;
  long long n;
  double* sd;
  double cfl_dx;
  double* dt_out;
  int k;
};

__device__ __forceinline__ void dt_block(const DtReduce& R, DevReport* rep) {
  double s = 0.0;
#pragma unroll 16
  for (long long i = threadIdx.x; i < R.n; i += kBlock) s = rr::dmax(s, R.partial[i]);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s = rr::dmax(s, __shfl_xor(s, o, kWave));
  if (threadIdx.x == 0) {
    const double m = rr::dmin(s, 1.0);
    R.sd[0] = m;
    double dt = R.cfl_dx / m;
    if (!(dt >= 0.0) || !(dt < 1e300)) {
      dt = 0.0;
      atomicAdd(&rep->nonfinite, 1ull);
    }
    R.sd[1] = dt;
    if (R.dt_out) R.dt_out[R.k] = dt;
  }
}

// Dispatch order of the next update pass: its nb cell blocks sorted by
// decreasing cost (the Picard solves of each block's slowest cell in the
// previous update pass), so that the slow blocks start in the first round of
// waves and the partial last round holds fast ones. Counting sort in one
// block; the order within a cost class is arbitrary (blocks are independent,
// so results do not depend on it). cost == nullptr: nothing to do.
struct BlockOrder {
  const unsigned int* cost;
  unsigned int* perm;
  long long nb;
};

constexpr int kCostClasses = 32;

__device__ __forceinline__ void order_block(const BlockOrder& O) {
  __shared__ unsigned int cnt[kCostClasses];
  if (threadIdx.x < kCostClasses) cnt[threadIdx.x] = 0;
  __syncthreads();
  for (long long i = threadIdx.x; i < O.nb; i += kBlock) {
    const unsigned int k = O.cost[i];
    atomicAdd(&cnt[(k < kCostClasses) ? k : kCostClasses - 1], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned int s = 0;
    for (int k = kCostClasses - 1; k >= 0; --k) {
      const unsigned int n = cnt[k];
      cnt[k] = s;
      s += n;
    }
  }
  __syncthreads();
  for (long long i = threadIdx.x; i < O.nb; i += kBlock) {
    const unsigned int k = O.cost[i];
    const unsigned int pos = atomicAdd(&cnt[(k < kCostClasses) ? k : kCostClasses - 1], 1u);
    O.perm[pos] = (unsigned int)i;
  }
}

// More waves per SIMD hide more of the FP64 and transcendental latency (three
// with 18 spilled registers beat two with none by 7 %).
// FT = double: FP64 path; FT = float: mixed-precision path. The first
// blocks do the step's time step (dt_block, with R.partial set) and the next
// update pass's block order (order_block, with O.cost set); the rest take the
// faces. The update pass, which reads both, runs after this launch.
template <typename FT, int REC, int SOLVER>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(SOLVER == RRMHD_SOLVER_HLL ? RRMHD_FACES_WAVES_HLL
                                   : SOLVER == RRMHD_SOLVER_PVM_JVP
                                       ? (sizeof(FT) == sizeof(double) ? RRMHD_FACES_WAVES_JVP
                                                                       : RRMHD_FACES_WAVES_JVP_MIXED)
                                       : (sizeof(FT) == sizeof(double) ? RRMHD_FACES_WAVES : RRMHD_FACES_WAVES_MIXED))))
k_faces(GridDev G, FaceArgs A, Phys K, DevReport* rep, unsigned int* blkmax, unsigned long long* wreset,
        DtReduce R, BlockOrder O) {
  // the work-list counter of the update pass that follows (not read here)
  if (wreset && blockIdx.x == 0 && threadIdx.x == 0) *wreset = 0;
  long long b = blockIdx.x;
  if (R.partial) {
    if (b == 0) {
      dt_block(R, rep);
      return;
    }
    b -= 1;
  }
  if (O.cost) {
    if (b == 0) {
      order_block(O);
      return;
    }
    b -= 1;
  }
  faces_block<sizeof(FT) == sizeof(float), REC, SOLVER>(b, G, A, K, rep, blkmax);
}

// Periodic cell index of cell (x) shifted by +1 along axis e.
__device__ __forceinline__ long long cell_plus(const GridDev& G, const int x[3], int e) {
  int y[3] = {x[0], x[1], x[2]};
  y[e] += 1;
  if (y[e] == G.n[e]) y[e] = 0;
  return (long long)y[0] + (long long)G.n[0] * ((long long)y[1] + (long long)G.n[1] * y[2]);
}

__device__ __forceinline__ void cell_coords(const GridDev& G, long long c, int x[3]) {
  // 32-bit index arithmetic: fewer than 2^31 cells (grid_valid)
  const unsigned int cu = (unsigned int)c, u0 = (unsigned int)G.n[0], u1 = (unsigned int)G.n[1];
  const unsigned int q0 = cu / u0;
  x[0] = (int)(cu - q0 * u0);
  const unsigned int q1 = q0 / u1;
  x[1] = (int)(q0 - q1 * u1);
  x[2] = (int)q1;
}

// ---------------------------------------------------------------------------
// Constrained transport (Section 4: div B kept by CT with CT-contact averaged
// EMFs, after Gardiner & Stone 2005). Periodic grids. The normal field b_a is
// held per cell for the face on its lower side along a; the edge EMF E_k
// (edge along k, (a, b, k) cyclic) per cell for the edge at its lower corner
// in the (a, b) plane. Face EMFs come from the face fluxes of the induction
// equation (F_a(B_b) = -E_k on a-faces, F_b(B_a) = +E_k on b-faces), the
// cell-centre EMF from the stage primitives, E_k = -(v_a B_b - v_b B_a). The
// edge value is the mean of its four face EMFs plus a quarter of the
// difference of the half-cell EMF gradients on both sides of the edge along
// each plane direction, each taken from the cell upwind of the contact (sign
// of the mass flux through the face between the two candidate cells; their
// mean for zero).
struct CTArgs {
  const void* Fh[3];    // stage face fluxes (double, or float in mixed precision)
  long long nf[3];
  const double* Vp;     // stage primitives, stride np
  long long np;
  double* E;            // edge EMFs [3][N] (planes of edges in the grid only)
  double* bnew;         // new face fields [ndim][N]
  const double* b0;     // face fields of U^(0) (stride s0) and U^(s) (stride ss)
  long long s0;
  const double* bs;
  long long ss;
  double idx[3];
  double a0, a1, cdt, cc;
  const double* dtp;    // device time step (rrmhd_advance), or nullptr
};

__device__ __forceinline__ double ct_upwind(double mflux, double lower_side, double upper_side) {
  if (mflux > 0.0) return lower_side;
  if (mflux < 0.0) return upper_side;
  return 0.5 * (lower_side + upper_side);
}

// Index of the face on the lower side of cell x along d.
__device__ __forceinline__ long long lower_face_index(const GridDev& G, int d, const int x[3]) {
  int fn0 = G.n[0], fn1 = G.n[1];
  if (d == 0) fn0 += 1;
  if (d == 1) fn1 += 1;
  return (long long)x[0] + (long long)fn0 * ((long long)x[1] + (long long)fn1 * x[2]);
}

template <typename FT>
__global__ void __launch_bounds__(kBlock) k_ct_emf(GridDev G, CTArgs A) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= G.N) return;
  int x[3];
  cell_coords(G, c, x);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int a = (k + 1) % 3, b = (k + 2) % 3;
    if (a >= G.ndim || b >= G.ndim) continue;
    const FT* Fa = (const FT*)A.Fh[a];
    const FT* Fb = (const FT*)A.Fh[b];
    const long long nfa = A.nf[a], nfb = A.nf[b];
    // cells around the edge: x, x - e_a, x - e_b, x - e_a - e_b (periodic)
    int xa[3] = {x[0], x[1], x[2]}, xb[3] = {x[0], x[1], x[2]}, xab[3] = {x[0], x[1], x[2]};
    xa[a] = (x[a] == 0) ? G.n[a] - 1 : x[a] - 1;
    xb[b] = (x[b] == 0) ? G.n[b] - 1 : x[b] - 1;
    xab[a] = xa[a];
    xab[b] = xb[b];
    const long long c_a = (long long)xa[0] + (long long)G.n[0] * ((long long)xa[1] + (long long)G.n[1] * xa[2]);
    const long long c_b = (long long)xb[0] + (long long)G.n[0] * ((long long)xb[1] + (long long)G.n[1] * xb[2]);
    const long long c_ab = (long long)xab[0] + (long long)G.n[0] * ((long long)xab[1] + (long long)G.n[1] * xab[2]);
    const long long fa_c = lower_face_index(G, a, x), fa_cb = lower_face_index(G, a, xb);
    const long long fb_c = lower_face_index(G, b, x), fb_ca = lower_face_index(G, b, xa);
    const double Ea_c = -(double)Fa[(5 + b) * nfa + fa_c];
    const double Ea_cb = -(double)Fa[(5 + b) * nfa + fa_cb];
    const double Eb_c = (double)Fb[(5 + a) * nfb + fb_c];
    const double Eb_ca = (double)Fb[(5 + a) * nfb + fb_ca];
    const double* V = A.Vp;
    const long long np = A.np;
    const double Ec_c = -(V[(1 + a) * np + c] * V[(5 + b) * np + c] - V[(1 + b) * np + c] * V[(5 + a) * np + c]);
    const double Ec_a = -(V[(1 + a) * np + c_a] * V[(5 + b) * np + c_a] - V[(1 + b) * np + c_a] * V[(5 + a) * np + c_a]);
    const double Ec_b = -(V[(1 + a) * np + c_b] * V[(5 + b) * np + c_b] - V[(1 + b) * np + c_b] * V[(5 + a) * np + c_b]);
    const double Ec_ab =
        -(V[(1 + a) * np + c_ab] * V[(5 + b) * np + c_ab] - V[(1 + b) * np + c_ab] * V[(5 + a) * np + c_ab]);
    const double ma_c = (double)Fa[fa_c], ma_cb = (double)Fa[fa_cb];
    const double mb_c = (double)Fb[fb_c], mb_ca = (double)Fb[fb_ca];
    const double Dbhi = ct_upwind(ma_c, Ec_a - Eb_ca, Ec_c - Eb_c);
    const double Dblo = ct_upwind(ma_cb, Eb_ca - Ec_ab, Eb_c - Ec_b);
    const double Dahi = ct_upwind(mb_c, Ec_b - Ea_cb, Ec_c - Ea_c);
    const double Dalo = ct_upwind(mb_ca, Ea_cb - Ec_ab, Ea_c - Ec_a);
    const double s4 = (Ea_c + Ea_cb) + (Eb_c + Eb_ca);
    const double corr = (Dblo - Dbhi) + (Dalo - Dahi);
    A.E[k * G.N + c] = 0.25 * (s4 + corr);
  }
}

// New face fields of a stage: b_a = a0 b_a^(0) + a1 b_a^(s) - c dt (curl E)_a
// with (curl E)_a = dE_k/dx_b - dE_b/dx_k, (a, b, k) cyclic (edges in the
// grid only).
__global__ void __launch_bounds__(kBlock) k_ct_face(GridDev G, CTArgs A) {
  const long long c = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (c >= G.N) return;
  int x[3];
  cell_coords(G, c, x);
  const double cdt = A.dtp ? A.cc * A.dtp[0] : A.cdt;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= G.ndim) continue;
    const int b = (a + 1) % 3, k = (a + 2) % 3;
    double t1 = 0.0, t2 = 0.0;
    if (b < G.ndim) t1 = (A.E[k * G.N + cell_plus(G, x, b)] - A.E[k * G.N + c]) * A.idx[b];
    if (k < G.ndim) t2 = (A.E[b * G.N + cell_plus(G, x, k)] - A.E[b * G.N + c]) * A.idx[k];
    const double curl = t1 - t2;
    A.bnew[a * G.N + c] = (A.a0 * A.b0[a * A.s0 + c] + A.a1 * A.bs[a * A.ss + c]) - cdt * curl;
  }
}

struct StageArgs {
  const double* U0;
  long long s0;
  const double* Us;
  long long ss;
  double* Uo;
  long long so;
  const void* Fh[3];   // double (FP64 path) or float (mixed path)
  double* Zc;          // recovery Z of the stage state per cell (warm start)
  long long nf[3];
  double idx[3];
  double a0, a1, cdt;
  // Time step held on the device: when dtp is set, the stage uses
  // cdt = cc * dtp[0] instead of cdt.
  const double* dtp;
  double cc;
  // Next stage's primitives: with nextp set, each cell's recovery from its
  // output state is done where the cell finishes (Vp, taup, Zc of the next
  // stage); with speed also set, the signal-speed block maxima go to
  // partial[update block] and partial[npart + work-list block].
  int nextp, speed;
  double* Vp;
  double* taup;
  long long np;
  double* partial;
  long long npart;
  // Dispatch order of the cell blocks (perm[blockIdx] = block; nullptr:
  // identity) and each block's cost, written for the next ordering.
  const unsigned int* perm;
  unsigned int* cost;
  // Constrained transport: the stage's new face fields ([ndim][N], from
  // k_ct_face); the cell-centred B_a is their mean over the cell's two faces
  // and they go to the output's planes 12 + a. nullptr: none.
  const double* bnew;
};

__device__ __forceinline__ double stage_cdt(const StageArgs& A) { return A.dtp ? A.cc * A.dtp[0] : A.cdt; }

// Stage primitives of interior cell c from its new state Un (as prims_block
// computes them); returns the cell's signal speed when A.speed is set.
__device__ __forceinline__ double next_prims(const GridDev& G, const StageArgs& A, const Opac& op, const Phys& K,
                                             long long c, const double Un[NV], unsigned long long& fail,
                                             unsigned long long& bad, unsigned int& c2p_its) {
  double v[NV], Z = 0.0;
  int it = 0;
  if (rr::c2p(Un, K, 0.0, v, Z, it) != 0) {
    rr::c2p_fallback(Un, K, v);
    Z = 0.0;
    fail += 1;
    if ((unsigned long long)c < bad) bad = (unsigned long long)c;
  }
  c2p_its = ((unsigned int)it > c2p_its) ? (unsigned int)it : c2p_its;
  A.Zc[c] = Z;
#pragma unroll
  for (int q = 0; q < NV; ++q) A.Vp[q * A.np + c] = v[q];
  A.taup[c] = Un[0] * (opac_at(op.kappa, op.kappa0, c) + opac_at(op.sigma, op.sigma0, c));
  return A.speed ? cell_signal_speed(G, v, K) : 0.0;
}

// Work-list entry of a cell handed to the second pass, planes of `xs`:
// 0-3 the Newton start point X0, 4 its recovery warm start Z0, 5 the Picard
// solves done.
constexpr int kWorkPlanes = 6;

// Flux divergence and stage combination, then phase 1 of the implicit solve
// (Picard). Cells that need phase 2 (Newton) get their explicit state U*
// written to the output and are appended to `worklist` (one atomic per wave)
// with their Newton start point.
// FT: storage type of the face fluxes; the divergence is accumulated in FP64
// either way (differences of stored values are exact in FP64 for FP32 data).
template <typename FT>
__device__ __forceinline__ void update_block(long long lb, const GridDev& G, const StageArgs& A, const Opac& op,
                                             const Phys& K, DevReport* rep, unsigned int* blkmax,
                                             long long* worklist, unsigned long long* wcount) {
  const FT* F0 = (const FT*)A.Fh[0];
  const FT* F1 = (const FT*)A.Fh[1];
  const FT* F2 = (const FT*)A.Fh[2];
  const double cdt = stage_cdt(A);
  const long long c = lb * kBlock + threadIdx.x;
  unsigned long long fimp = 0, fnf = 0, ffl = 0, fc2p = 0, bad = ULLONG_MAX;
  unsigned int its = 0, cits = 0;
  double spd = 0.0;
  bool newton = false;
  double X0[4] = {0.0, 0.0, 0.0, 0.0}, Z0 = 0.0;
  int pits = 0;
  if (c < G.N) {
    int ci[3];
    {
      // 32-bit index arithmetic: fewer than 2^31 cells (grid_valid)
      const unsigned int cu = (unsigned int)c, u0 = (unsigned int)G.n[0], u1 = (unsigned int)G.n[1];
      const unsigned int q0 = cu / u0;
      ci[0] = (int)(cu - q0 * u0);
      const unsigned int q1 = q0 / u1;
      ci[1] = (int)(q0 - q1 * u1);
      ci[2] = (int)q1;
    }
    long long fm[3], fs[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int fn0 = G.n[0], fn1 = G.n[1];
      if (d == 0) fn0 += 1;
      if (d == 1) fn1 += 1;
      fm[d] = (long long)ci[0] + (long long)fn0 * ((long long)ci[1] + (long long)fn1 * ci[2]);
      fs[d] = (d == 0) ? 1 : ((d == 1) ? (long long)fn0 : (long long)fn0 * fn1);
    }
    // The x and y face loads and the two states are issued together (one
    // round of memory latency instead of one per variable). In 1D the y
    // addresses stay inside the x buffer and the values are not used.
    FT fp[2][NV], fq[2][NV];
    double u0[NV], us[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      fp[0][q] = F0[q * A.nf[0] + fm[0] + fs[0]];
      fq[0][q] = F0[q * A.nf[0] + fm[0]];
      fp[1][q] = F1[q * A.nf[1] + fm[1] + fs[1]];
      fq[1][q] = F1[q * A.nf[1] + fm[1]];
      u0[q] = A.U0[q * A.s0 + c];
      us[q] = A.Us[q * A.ss + c];
    }
    double div[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      div[q] = ((double)fp[0][q] - (double)fq[0][q]) * A.idx[0];
      if (G.ndim > 1) div[q] = div[q] + ((double)fp[1][q] - (double)fq[1][q]) * A.idx[1];
    }
    if (G.ndim > 2) {
#pragma unroll
      for (int q = 0; q < NV; ++q)
        div[q] = div[q] + ((double)F2[q * A.nf[2] + fm[2] + fs[2]] - (double)F2[q * A.nf[2] + fm[2]]) * A.idx[2];
    }
    double Ust[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) Ust[q] = (A.a0 * u0[q] + A.a1 * us[q]) - cdt * div[q];
    if (A.bnew) {
      // constrained transport: B_a of the cell is the mean of its two new
      // face values, which also become the output's face planes (unrolled:
      // constant register indices)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (a < G.ndim) {
          const double blo = A.bnew[a * G.N + c];
          Ust[5 + a] = 0.5 * (blo + A.bnew[a * G.N + cell_plus(G, ci, a)]);
          A.Uo[(NV + a) * A.so + c] = blo;
        }
      }
    }
    double Un[NV];
    bool floored = false;
    rr::ImpIn in;
    int st;
    const double Zg0 = A.Zc[c];
    if (!rr::imp_prepare(Ust, K, in, floored)) {
#pragma unroll
      for (int q = 0; q < NV; ++q) Un[q] = Ust[q];
      st = rr::IMP_FAILED;
    } else {
      st = rr::picard_run(Ust, in, cdt, opac_at(op.kappa, op.kappa0, c), opac_at(op.sigma, op.sigma0, c), K, Zg0,
                          Un, X0, Z0, pits);
    }
    its = (unsigned int)pits;
    ffl = floored ? 1 : 0;
    if (st == rr::IMP_NEED_NEWTON) {
      newton = true;
#pragma unroll
      for (int q = 0; q < NV; ++q) A.Uo[q * A.so + c] = Ust[q];
    } else {
      bool fin = true;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        A.Uo[q * A.so + c] = Un[q];
        fin = fin && isfinite(Un[q]);
      }
      if (st != rr::IMP_DONE) fimp = 1;
      if (!fin) fnf = 1;
      if (st != rr::IMP_DONE || !fin) bad = (unsigned long long)c;
      if (A.nextp) spd = next_prims(G, A, op, K, c, Un, fc2p, bad, cits);
    }
  }
  // Append the cells that need phase 2.
  const unsigned long long mask = __ballot(newton);
  if (mask) {
    const int lane = threadIdx.x & (kWave - 1);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(wcount, (unsigned long long)__popcll(mask));
    base = __shfl(base, 0, kWave);
    if (newton) {
      const unsigned int below = __builtin_amdgcn_mbcnt_hi((unsigned int)(mask >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((unsigned int)mask, 0u));
      const unsigned long long slot = base + below;
      worklist[slot] = c;
      double* xs = (double*)(worklist + G.N);
      xs[0 * G.N + slot] = X0[0];
      xs[1 * G.N + slot] = X0[1];
      xs[2 * G.N + slot] = X0[2];
      xs[3 * G.N + slot] = X0[3];
      xs[4 * G.N + slot] = Z0;
      xs[5 * G.N + slot] = (double)pits;
    }
  }
  report_add(rep, blkmax, lb, fc2p, 0, fimp, fnf, bad, cits, its, ffl);
  if (A.cost) {
    // the block's cost: Picard solves of its slowest cell (one wave per block)
    const unsigned int wm = wave_max_u32(its);
    if (threadIdx.x == 0) A.cost[lb] = wm;
  }
  if (A.speed) block_max_to(spd, A.partial, lb);
}

template <typename FT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RRMHD_UPDATE_WAVES)))
k_update(GridDev G, StageArgs A, Opac op, Phys K, DevReport* rep, unsigned int* blkmax,
         long long* worklist, unsigned long long* wcount) {
  const long long lb = A.perm ? (long long)A.perm[blockIdx.x] : (long long)blockIdx.x;
  update_block<FT>(lb, G, A, op, K, rep, blkmax, worklist, wcount);
}

// Second pass of the implicit solve for the cells in `worklist`: Newton from
// the start point the update pass left; the explicit state U* is in the
// output. Each cell is handled by a quad of 4 lanes (see
// implicit_newton_quad); grid-stride over the list with blocks bi = 0..nb-1
// (16 cells per block).
__device__ __forceinline__ void newton_blocks(long long bi, long long nb, const GridDev& G, const StageArgs& A,
                                              const Opac& op, const Phys& K, DevReport* rep, unsigned int* blkmax,
                                              const long long* __restrict__ worklist,
                                              const unsigned long long* wcount, long long slot,
                                              bool shared_slot = false) {
  const long long ncell = G.N;
  const double* xs = (const double*)(worklist + ncell);
  const unsigned long long n = *wcount;
  const double cdt = stage_cdt(A);
  unsigned long long fimp = 0, fnf = 0, fc2p = 0, bad = ULLONG_MAX;
  unsigned int its = 0, cits = 0;
  double spd = 0.0;
  constexpr int kCellsPerBlock = kBlock / 4;
  const unsigned long long quad = threadIdx.x >> 2;
  const bool lead = (threadIdx.x & 3) == 0;
  // trip count is uniform over the quad (same i for its 4 lanes)
  for (unsigned long long i = (unsigned long long)bi * kCellsPerBlock + quad; i < n;
       i += (unsigned long long)nb * kCellsPerBlock) {
    const long long c = worklist[i];
    double Un[NV];
    bool conv = false;
    int it = 0;
    {
      rr::ImpIn in;
      {
        double Ust[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) Ust[q] = A.Uo[q * A.so + c];
        bool floored = false;
        rr::imp_prepare(Ust, K, in, floored);  // succeeded in the update pass
      }
      const double kap = opac_at(op.kappa, op.kappa0, c), sig = opac_at(op.sigma, op.sigma0, c);
      double X[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) X[k] = xs[k * ncell + i];
      const double Z0 = xs[4 * ncell + i];
      it = (int)xs[5 * ncell + i];
      int nit = 0;
      conv = rr::implicit_newton_quad(in, cdt, kap, sig, K, X, Z0, nit);
      it += nit;
      if (conv) {
        // D and B of the prepared state are those of U*
        rr::imp_finish(X, in.Ul, in, Un);
      } else {
        // U* again, from the output (not kept in registers through the solve)
        const volatile double* uo = A.Uo;
#pragma unroll
        for (int q = 0; q < NV; ++q) Un[q] = uo[q * A.so + c];
      }
    }
    if (lead) {
      bool fin = true;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        A.Uo[q * A.so + c] = Un[q];
        fin = fin && isfinite(Un[q]);
      }
      if (!conv) fimp += 1;
      if (!fin) fnf += 1;
      if ((!conv || !fin) && (unsigned long long)c < bad) bad = (unsigned long long)c;
      its = ((unsigned int)it > its) ? (unsigned int)it : its;
      if (A.nextp) spd = rr::dmax(spd, next_prims(G, A, op, K, c, Un, fc2p, bad, cits));
    }
  }
  report_add(rep, blkmax, slot, fc2p, 0, fimp, fnf, bad, cits, its, 0, shared_slot);
  if (A.speed) {
    if (shared_slot) block_max_atomic(spd, A.partial + A.npart + bi % A.npart);
    else block_max_to(spd, A.partial, A.npart + bi);
  }
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RRMHD_NEWTON_WAVES)))
k_newton(GridDev G, StageArgs A, Opac op, Phys K, DevReport* rep, unsigned int* blkmax,
         const long long* __restrict__ worklist, const unsigned long long* wcount) {
  newton_blocks(blockIdx.x, gridDim.x, G, A, op, K, rep, blkmax, worklist, wcount, blockIdx.x);
}

// Per-block maximum of the cell signal speeds -> partial[lb].
__device__ __forceinline__ void speed_block(long long lb, const GridDev& G, const double* __restrict__ U,
                                            long long su, const Phys& K, double* __restrict__ partial,
                                            DevReport* rep, unsigned int* blkmax) {
  const long long c = lb * kBlock + threadIdx.x;
  double s = 0.0;
  unsigned long long fail = 0, bad = ULLONG_MAX;
  if (c < G.N) {
    double u[NV], v[NV], Z = 0.0;
    int it = 0;
#pragma unroll
    for (int q = 0; q < NV; ++q) u[q] = U[q * su + c];
    if (rr::c2p(u, K, 0.0, v, Z, it) != 0) {
      rr::c2p_fallback(u, K, v);
      fail = 1;
      bad = (unsigned long long)c;
    }
    s = cell_signal_speed(G, v, K);
  }
  report_add(rep, blkmax, lb, fail, 0, 0, 0, bad, 0, 0);
  block_max_to(s, partial, lb);
}

__global__ void __launch_bounds__(kBlock) k_speed(GridDev G, const double* __restrict__ U, long long su,
                                                  Phys K, double* __restrict__ partial, DevReport* rep,
                                                  unsigned int* blkmax) {
  speed_block(blockIdx.x, G, U, su, K, partial, rep, blkmax);
}

__device__ __forceinline__ void reduce_max_block(const double* __restrict__ partial, long long n,
                                                 double* __restrict__ out) {
  __shared__ double red[kRedBlock / kWave];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += kRedBlock) s = rr::dmax(s, partial[i]);
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s = rr::dmax(s, __shfl_xor(s, o, kWave));
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
#pragma unroll
    for (int w = 1; w < kRedBlock / kWave; ++w) m = rr::dmax(m, red[w]);
    out[0] = rr::dmin(m, 1.0);
  }
}

__global__ void __launch_bounds__(kRedBlock) k_reduce_max(const double* __restrict__ partial, long long n,
                                                       double* __restrict__ out) {
  reduce_max_block(partial, n, out);
}

// ---------------------------------------------------------------------------
// Batched kernels: one launch covers every simulation of a batch. Each block
// finds its simulation by binary search in a block-offset table and works on
// that simulation's data exactly as the single-simulation kernels do, so a
// simulation's result does not depend on what else is in the batch.
struct SimDesc {
  GridDev G;
  Phys K;
  Opac op;
  FaceArgs FA;
  double* Vp;
  double* taup;
  double idx[3];
  double* U;
  long long vs;
  double* Us;
  long long ns;
  const double* inflow_U;
  long long* work;
  unsigned long long* wcount;
  double* Zc;
  DevReport* rep;
  unsigned int* blkmax;
  double* partial;
  long long npartial;
  long long nblkmax;  // report slots of the simulation's per-block maxima
  double dt;
  int mixed;
  int solver;  // RRMHD_SOLVER_*: which face-kernel launch of a tick takes this simulation
};

enum { OFF_PRIMS = 0, OFF_FACES = 1, OFF_CELLS = 2, OFF_NEWTON = 3, OFF_KINDS = 4 };

__device__ __forceinline__ int find_sim(const long long* __restrict__ off, int nsim, long long b) {
  int lo = 0, hi = nsim;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// Per-simulation clock of the batched advance (rrmhd_advance_batch), [nsim]
// arrays on the device. t == nullptr: no clock (the per-call entry points).
struct BatchClock {
  double* t;              // time reached
  long long* n;           // steps taken
  const double* tend;     // end time (+inf for a step-count request)
  const long long* nmax;  // steps to take (< 0: an end-time request)
  const double* cfl_dx;   // CFL number times the smallest cell width
};

// Simulation s has reached its end: n >= nmax for a step-count request,
// t >= t_end (1 - 1e-14) otherwise (the same test as the serving loop's).
__device__ __forceinline__ bool clock_at_end(const BatchClock& C, int s) {
  return (C.nmax[s] >= 0) ? (C.n[s] >= C.nmax[s]) : (C.t[s] >= C.tend[s] * (1.0 - 1e-14));
}

// Blocks of a step launch skip a simulation whose time step in `gate` is 0
// (one at its end in rrmhd_advance_batch); gate == nullptr: none skipped.
__device__ __forceinline__ bool step_gated(const double* gate, int s) { return gate && !(gate[s] > 0.0); }

// after: the last stage also recovers the primitives of its result (the next
// step's first stage) and the signal-speed maxima of the next step's time
// step: update blocks into partial[0, npartial), Newton blocks into
// partial[npartial, 2 npartial) (atomic maxima, cleared by the update pass).
__device__ __forceinline__ StageArgs stage_args(const SimDesc& D, double dt, int stage, int last, double a0,
                                                double a1, double c, int after = 0) {
  StageArgs A;
  A.U0 = D.U; A.s0 = D.vs;
  A.Us = (stage == 0) ? D.U : D.Us;
  A.ss = (stage == 0) ? D.vs : D.ns;
  A.Uo = last ? D.U : D.Us;
  A.so = last ? D.vs : D.ns;
  for (int d = 0; d < 3; ++d) {
    A.Fh[d] = (d < D.G.ndim) ? (const void*)D.FA.Fh[d] : (const void*)D.FA.Fh[0];
    A.nf[d] = D.FA.nf[d];
    A.idx[d] = D.idx[d];
  }
  A.a0 = a0;
  A.a1 = a1;
  A.cdt = c * dt;
  A.dtp = nullptr;
  A.cc = c;
  A.Zc = D.Zc;
  // the next stage's primitives where each cell finishes (after the last
  // stage only when the step is followed by another in the same launch run)
  A.nextp = (last && !after) ? 0 : 1;
  A.speed = (last && after) ? 1 : 0;
  A.Vp = D.Vp;
  A.taup = D.taup;
  A.np = D.FA.np;
  A.partial = A.speed ? D.partial : nullptr;
  A.npart = A.speed ? D.npartial : 0;
  A.perm = nullptr;
  A.cost = nullptr;
  A.bnew = nullptr;
  return A;
}

__global__ void __launch_bounds__(kBlock) k_prims_b(const SimDesc* __restrict__ T, const long long* __restrict__ off,
                                                    int nsim, int stage, const double* gate) {
  const long long* o = off + OFF_PRIMS * (nsim + 1);
  const int s = find_sim(o, nsim, blockIdx.x);
  if (step_gated(gate, s)) return;
  const SimDesc& D = T[s];
  const double* Us = (stage == 0) ? D.U : D.Us;
  const long long ss = (stage == 0) ? D.vs : D.ns;
  prims_block(blockIdx.x - o[s], D.G, Us, ss, D.inflow_U, D.op, D.Vp, D.taup, D.FA.np, D.K, D.rep, D.blkmax,
              D.wcount, D.Zc);
}

// One launch per face flux present in the batch (each its own kernel copy, so
// the PVM copy keeps its register budget); a block of a simulation with
// another flux returns at once.
template <int SOLVER>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_faces_b(const SimDesc* __restrict__ T, const long long* __restrict__ off, int nsim, const double* gate) {
  const long long* o = off + OFF_FACES * (nsim + 1);
  const int s = find_sim(o, nsim, blockIdx.x);
  if (step_gated(gate, s)) return;
  const SimDesc& D = T[s];
  if (D.solver != SOLVER) return;
  // the work-list counter of this simulation's update pass that follows
  if (blockIdx.x == o[s] && threadIdx.x == 0) *D.wcount = 0;
  if (D.mixed) faces_block<true, -1, SOLVER>(blockIdx.x - o[s], D.G, D.FA, D.K, D.rep, D.blkmax);
  else faces_block<false, -1, SOLVER>(blockIdx.x - o[s], D.G, D.FA, D.K, D.rep, D.blkmax);
}

__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
k_update_b(const SimDesc* __restrict__ T, const long long* __restrict__ off, const double* __restrict__ dts, int nsim,
           int stage, int last, double a0, double a1, double c, const double* gate, int after) {
  const long long* o = off + OFF_CELLS * (nsim + 1);
  const int s = find_sim(o, nsim, blockIdx.x);
  if (step_gated(gate, s)) return;
  const SimDesc& D = T[s];
  const StageArgs A = stage_args(D, dts[s], stage, last, a0, a1, c, after);
  // the Newton pass's speed slot of this block, folded into atomically
  if (A.speed && threadIdx.x == 0) A.partial[A.npart + (blockIdx.x - o[s])] = 0.0;
  if (D.mixed) update_block<float>(blockIdx.x - o[s], D.G, A, D.op, D.K, D.rep, D.blkmax, D.work, D.wcount);
  else update_block<double>(blockIdx.x - o[s], D.G, A, D.op, D.K, D.rep, D.blkmax, D.work, D.wcount);
}

// Work-list blocks of a batch's Newton pass: simulation s has
// ceil(wcount_s / (kBlock/4)) of them (none when gated); vprefix[s] is the
// number before s, vprefix[nsim] the total. One block.
__global__ void __launch_bounds__(kRedBlock) k_wprefix_b(const SimDesc* __restrict__ T, int nsim,
                                                      long long* __restrict__ vprefix, const double* gate) {
  __shared__ long long wsum[kRedBlock / kWave];
  __shared__ long long carry;
  constexpr long long kq = kBlock / 4;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nsim; base += kRedBlock) {
    const int s = base + (int)threadIdx.x;
    long long v = 0;
    if (s < nsim && !step_gated(gate, s)) v = ((long long)*T[s].wcount + kq - 1) / kq;
    // inclusive scan within the wave, then across the waves
    long long x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const long long y = __shfl_up(x, o, kWave);
      if ((int)(threadIdx.x & (kWave - 1)) >= o) x += y;
    }
    if ((threadIdx.x & (kWave - 1)) == kWave - 1) wsum[threadIdx.x / kWave] = x;
    __syncthreads();
    long long before = carry;
    for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) before += wsum[w];
    if (s < nsim) vprefix[s] = before + x - v;
    __syncthreads();
    if (threadIdx.x == kRedBlock - 1) carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) vprefix[nsim] = carry;
}

// The batch's Newton pass, balanced over the batch: the grid walks the
// work-list blocks of all simulations (vprefix), each taking kBlock/4 entries
// of one simulation, so a simulation with a long list gets as many blocks as
// it needs whatever its size. Report maxima go to slot vb mod nblkmax of the
// simulation (atomic: several blocks may share a slot).
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RRMHD_NEWTON_WAVES)))
k_newton_b(const SimDesc* __restrict__ T, const long long* __restrict__ vprefix, const double* __restrict__ dts,
           int nsim, int stage, int last, double a0, double a1, double c, int after) {
  const long long total = vprefix[nsim];
  for (long long v = blockIdx.x; v < total; v += gridDim.x) {
    int lo = 0, hi = nsim;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (vprefix[mid] <= v) lo = mid; else hi = mid;
    }
    const SimDesc& D = T[lo];
    const StageArgs A = stage_args(D, dts[lo], stage, last, a0, a1, c, after);
    const long long vb = v - vprefix[lo];
    newton_blocks(vb, vprefix[lo + 1] - vprefix[lo], D.G, A, D.op, D.K, D.rep, D.blkmax, D.work, D.wcount,
                  vb % D.nblkmax, true);
  }
}

__global__ void __launch_bounds__(kBlock) k_speed_b(const SimDesc* __restrict__ T, const long long* __restrict__ off,
                                                    int nsim, BatchClock C) {
  const long long* o = off + OFF_CELLS * (nsim + 1);
  const int s = find_sim(o, nsim, blockIdx.x);
  if (C.t && clock_at_end(C, s)) return;
  const SimDesc& D = T[s];
  // the Newton pass's slot of this block (read with the cell blocks' after a
  // step that leaves the next step's speeds, and until then 0)
  if (threadIdx.x == 0) D.partial[D.npartial + (blockIdx.x - o[s])] = 0.0;
  speed_block(blockIdx.x - o[s], D.G, D.U, D.vs, D.K, D.partial, D.rep, D.blkmax);
}

// slots: 1 after k_speed_b (cell blocks), 2 after a last stage with `after`
// set (cell blocks, then the Newton pass's slots).
__global__ void __launch_bounds__(kRedBlock) k_reduce_max_b(const SimDesc* __restrict__ T, double* __restrict__ smax,
                                                         BatchClock C, int slots) {
  if (C.t && clock_at_end(C, (int)blockIdx.x)) return;
  const SimDesc& D = T[blockIdx.x];
  reduce_max_block(D.partial, slots * D.npartial, smax + blockIdx.x);
}

// Each simulation's time step of a batched advance: for one not at its end,
// dt = min(cfl_dx / s_max, t_end - t) (the serving loop's rule), then t += dt,
// n += 1; dts[s] = 0 for one at its end, which the step launches then skip.
// A time step that is not finite and >= 0 is counted as non-finite and sets
// t = +inf (an end-time request then ends; a step-count request stops
// advancing).
__global__ void __launch_bounds__(kRedBlock) k_dt_b(const SimDesc* __restrict__ T, const double* __restrict__ smax,
                                                 double* __restrict__ dts, int nsim, BatchClock C) {
  for (int s = threadIdx.x; s < nsim; s += kRedBlock) {
    if (clock_at_end(C, s)) {
      dts[s] = 0.0;
      continue;
    }
    const double a = C.cfl_dx[s] / smax[s];
    const double b = C.tend[s] - C.t[s];
    const double dt = (b < a) ? b : a;
    if (!(dt >= 0.0) || !(dt < 1e300)) {
      dts[s] = 0.0;
      C.t[s] = HUGE_VAL;
      atomicAdd(&T[s].rep->nonfinite, 1ull);
      continue;
    }
    dts[s] = dt;
    C.t[s] = C.t[s] + dt;
    C.n[s] = C.n[s] + 1;
  }
}

// Clear the counters and the per-block iteration maxima.
__global__ void __launch_bounds__(kBlock) k_report_reset(DevReport* rep, unsigned int* blkmax, long long nslots) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    rep->c2p_fail = 0; rep->pvm_fallback = 0; rep->imp_fail = 0; rep->nonfinite = 0; rep->e_floor_hits = 0;
    rep->first_bad = ULLONG_MAX;
    rep->max_c2p_it = 0; rep->max_imp_it = 0;
  }
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nslots; i += (long long)gridDim.x * blockDim.x)
    blkmax[i] = 0;
}

__global__ void __launch_bounds__(kBlock) k_zero_u32(unsigned int* p, long long n) {
  for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) p[i] = 0u;
}

// Fold the per-block iteration maxima into the report (single block).
__device__ __forceinline__ void k_report_fold_body(DevReport* rep, const unsigned int* blkmax, long long nblk) {
  __shared__ unsigned int red[2][kRedBlock / kWave];
  unsigned int a = 0, b = 0;
  for (long long i = threadIdx.x; i < nblk; i += blockDim.x) {
    a = (blkmax[2 * i] > a) ? blkmax[2 * i] : a;
    b = (blkmax[2 * i + 1] > b) ? blkmax[2 * i + 1] : b;
  }
  a = wave_max_u32(a);
  b = wave_max_u32(b);
  if ((threadIdx.x & (kWave - 1)) == 0) { red[0][threadIdx.x / kWave] = a; red[1][threadIdx.x / kWave] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRedBlock / kWave; ++w) {
      a = (red[0][w] > a) ? red[0][w] : a;
      b = (red[1][w] > b) ? red[1][w] : b;
    }
    a = (red[0][0] > a) ? red[0][0] : a;
    b = (red[1][0] > b) ? red[1][0] : b;
    rep->max_c2p_it = (a > rep->max_c2p_it) ? a : rep->max_c2p_it;
    rep->max_imp_it = (b > rep->max_imp_it) ? b : rep->max_imp_it;
  }
}

__global__ void __launch_bounds__(kRedBlock) k_report_fold(DevReport* rep, const unsigned int* blkmax, long long nblk) {
  k_report_fold_body(rep, blkmax, nblk);
}

// Fold the per-block iteration maxima and write the counters as the public
// report struct to caller-owned device memory (single block).
__global__ void __launch_bounds__(kRedBlock) k_report_out(DevReport* rep, const unsigned int* blkmax, long long nblk,
                                                          rrmhd_report* out) {
  k_report_fold_body(rep, blkmax, nblk);
  if (threadIdx.x == 0) {
    out->c2p_fail = (long long)rep->c2p_fail;
    out->pvm_fallback = (long long)rep->pvm_fallback;
    out->imp_fail = (long long)rep->imp_fail;
    out->nonfinite = (long long)rep->nonfinite;
    out->e_floor_hits = (long long)rep->e_floor_hits;
    out->first_bad_cell = (rep->first_bad == ULLONG_MAX) ? -1 : (long long)rep->first_bad;
    out->max_c2p_it = (int)rep->max_c2p_it;
    out->max_imp_it = (int)rep->max_imp_it;
  }
}

// ---------------------------------------------------------------------------
// Host side.
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

long long grid_cells(const rrmhd_grid* g) {
  return (long long)g->n[0] * g->n[1] * g->n[2];
}

long long transverse_cells(const rrmhd_grid* g) {
  const int dl = g->ndim - 1;
  long long nt = 1;
  for (int e = 0; e < g->ndim; ++e)
    if (e != dl) nt *= g->n[e];
  return nt;
}

bool grid_valid(const rrmhd_grid* g) {
  if (!g || g->ndim < 1 || g->ndim > 3) return false;
  for (int e = 0; e < 3; ++e) {
    if (g->n[e] < 1) return false;
    if (e >= g->ndim && g->n[e] != 1) return false;
    if (e < g->ndim) {
      if (!(g->dx[e] > 0.0)) return false;
      for (int bc : {g->bc_lo[e], g->bc_hi[e]})
        if (bc < RRMHD_BC_PERIODIC || bc > RRMHD_BC_INFLOW) return false;
      if (g->bc_hi[e] == RRMHD_BC_INFLOW) return false;
      if (g->bc_lo[e] == RRMHD_BC_INFLOW && e != g->ndim - 1) return false;
      if ((g->bc_lo[e] == RRMHD_BC_PERIODIC) != (g->bc_hi[e] == RRMHD_BC_PERIODIC)) return false;
    }
  }
  const long long N = grid_cells(g);
  // fewer than 2^31 cells: cell and face indices (at most 2N faces per
  // direction) then fit the kernels' 32-bit index arithmetic
  if (N >= (1LL << 31)) return false;
  if (g->var_stride < N) return false;
  if (g->bc_lo[g->ndim - 1] == RRMHD_BC_INFLOW && (!g->inflow_U || !g->inflow_mask)) return false;
  return true;
}

bool params_valid(const rrmhd_params* p) {
  if (!p) return false;
  if (!(p->gamma > 1.0 && p->gamma <= 2.0)) return false;
  if (!(p->a_rad >= 0.0) || !(p->t_coeff > 0.0)) return false;
  if (!(p->pvm_eps > 0.0)) return false;
  if (p->pvm_k < 0 || p->pvm_k > 4) return false;
  if (p->beta_mode < 0 || p->beta_mode > 2) return false;
  if (p->recon < 0 || p->recon > 3) return false;
  if (p->rk_order != 2 && p->rk_order != 3) return false;
  if (p->c2p_maxit < 1 || p->imp_maxit < 1 || p->imp_picard_it < 0) return false;
  if (p->imp_method < 0 || p->imp_method > 2) return false;
  if (!(p->c2p_tol > 0.0) || !(p->imp_tol > 0.0)) return false;
  if (!(p->e_floor >= 0.0)) return false;
  if (p->precision != RRMHD_FP64 && p->precision != RRMHD_MIXED) return false;
  if (!(p->pvm_eps_mixed > 0.0 && p->pvm_eps_mixed < 0.5)) return false;
  if (p->solver != RRMHD_SOLVER_PVM && p->solver != RRMHD_SOLVER_HLL && p->solver != RRMHD_SOLVER_PVM_JVP)
    return false;
  if (p->ct != 0 && p->ct != 1) return false;
  return true;
}

// Constrained transport is defined for periodic grids of 2 or 3 dimensions.
bool ct_grid_ok(const rrmhd_grid* g, const rrmhd_params* p) {
  if (!p->ct) return true;
  if (g->ndim < 2) return false;
  for (int e = 0; e < g->ndim; ++e)
    if (g->bc_lo[e] != RRMHD_BC_PERIODIC || g->bc_hi[e] != RRMHD_BC_PERIODIC) return false;
  return true;
}

// Coefficients of the internal polynomial approximation of |x| (eq. iterat):
// q_0(y) = 1, q_k(y) = q_{k-1}(y) - q_{k-1}(y)^2 / 2 + y / 2 with y = x^2.
// Dyadic rationals: exact in binary64 for k <= 4.
int internal_coefficients(int k, double out[rr::MAXCOEF]) {
  double q[rr::MAXCOEF] = {1.0};
  for (int m = 1; m < rr::MAXCOEF; ++m) q[m] = 0.0;
  int deg = 0;
  for (int step = 0; step < k; ++step) {
    double sq[rr::MAXCOEF];
    for (int m = 0; m < rr::MAXCOEF; ++m) sq[m] = 0.0;
    for (int a = 0; a <= deg; ++a)
      for (int b = 0; b <= deg; ++b) sq[a + b] += q[a] * q[b];
    const int ndeg = (deg == 0) ? 1 : 2 * deg;
    for (int m = 0; m <= ndeg; ++m) q[m] = q[m] - 0.5 * sq[m];
    q[1] += 0.5;
    deg = ndeg;
  }
  for (int m = 0; m < rr::MAXCOEF; ++m) out[m] = q[m];
  return (k == 0) ? 0 : deg;
}

Phys make_phys(const rrmhd_params* p) {
  Phys K;
  std::memset(&K, 0, sizeof(K));
  K.gamma = p->gamma;
  K.g1 = p->gamma / (p->gamma - 1.0);
  K.gm1g = (p->gamma - 1.0) / p->gamma;
  K.gm1 = p->gamma - 1.0;
  K.a_rad = p->a_rad;
  K.t_coeff = p->t_coeff;
  K.eps = p->pvm_eps;
  K.ieps = 1.0 / p->pvm_eps;
  K.eps32 = p->pvm_eps_mixed;
  K.c2p_tol = p->c2p_tol;
  K.imp_tol = p->imp_tol;
  K.rho_floor = p->rho_floor;
  K.e_floor = p->e_floor;
  K.p_floor = p->p_floor;
  K.c2p_maxit = p->c2p_maxit;
  K.imp_maxit = p->imp_maxit;
  K.imp_picard_it = p->imp_picard_it;
  K.imp_method = p->imp_method;
  K.beta_mode = p->beta_mode;
  K.recon = p->recon;
  K.M = internal_coefficients(p->pvm_k, K.coef);
  return K;
}

struct Layout {
  long long N, nt, Np, Ns;
  long long nf[3];
  long long npartial;
  long long nb_faces[3];
  long long nblkmax;  // block slots for the iteration maxima
  int nb;             // face-field planes of the state (constrained transport: ndim)
  size_t off_Vp, off_taup, off_Us, off_Fh[3], off_partial, off_smax, off_rep, off_blkmax, off_work, off_wcount, off_Zc,
      off_cost, off_perm, off_ctE, off_ctb, total;
};

Layout make_layout(const rrmhd_grid* g, const rrmhd_params* p) {
  Layout L;
  std::memset(&L, 0, sizeof(L));
  L.N = grid_cells(g);
  L.nt = (g->bc_lo[g->ndim - 1] == RRMHD_BC_INFLOW) ? transverse_cells(g) : 0;
  L.Np = (L.N + L.nt + 31) / 32 * 32;
  L.Ns = (L.N + 31) / 32 * 32;
  for (int d = 0; d < 3; ++d) {
    if (d < g->ndim) {
      long long nf = 1;
      for (int e = 0; e < 3; ++e) nf *= (e == d) ? (g->n[e] + 1) : g->n[e];
      L.nf[d] = nf;
    }
  }
  L.npartial = (L.N + kBlock - 1) / kBlock;
  long long nbf = 0;
  for (int d = 0; d < 3; ++d) { L.nb_faces[d] = (L.nf[d] + kBlock - 1) / kBlock; nbf += L.nb_faces[d]; }
  const long long nbc = (L.N + L.nt + kBlock - 1) / kBlock;
  L.nblkmax = (nbf > nbc) ? nbf : nbc;
  size_t o = 0;
  L.nb = (p && p->ct) ? g->ndim : 0;
  L.off_Vp = o; o = align256(o + sizeof(double) * NV * L.Np);
  L.off_taup = o; o = align256(o + sizeof(double) * L.Np);
  L.off_Us = o; o = align256(o + sizeof(double) * (NV + L.nb) * L.Ns);
  for (int d = 0; d < 3; ++d) { L.off_Fh[d] = o; o = align256(o + sizeof(double) * NV * L.nf[d]); }
  // signal-speed block maxima: cell blocks, then work-list blocks (<= cell blocks)
  L.off_partial = o; o = align256(o + sizeof(double) * 2 * L.npartial);
  L.off_smax = o; o = align256(o + 2 * sizeof(double));
  L.off_rep = o; o = align256(o + sizeof(DevReport));
  L.off_blkmax = o; o = align256(o + sizeof(unsigned int) * 2 * L.nblkmax);
  L.off_work = o; o = align256(o + sizeof(long long) * L.N + sizeof(double) * kWorkPlanes * L.N);  // cells + state
  L.off_wcount = o; o = align256(o + 2 * sizeof(unsigned long long));  // one per stage parity
  L.off_Zc = o; o = align256(o + sizeof(double) * L.N);
  // update-pass block costs and dispatch order (cell blocks)
  L.off_cost = o; o = align256(o + sizeof(unsigned int) * L.npartial);
  L.off_perm = o; o = align256(o + sizeof(unsigned int) * L.npartial);
  // constrained transport: edge EMFs [3][N] and the stage's new face fields [ndim][N]
  L.off_ctE = o; o = align256(o + (L.nb ? sizeof(double) * 3 * L.N : 0));
  L.off_ctb = o; o = align256(o + sizeof(double) * L.nb * L.N);
  L.total = o;
  return L;
}

GridDev make_griddev(const rrmhd_grid* g, const Layout& L) {
  GridDev G;
  G.ndim = g->ndim;
  for (int e = 0; e < 3; ++e) { G.n[e] = g->n[e]; G.bc_lo[e] = g->bc_lo[e]; G.bc_hi[e] = g->bc_hi[e]; }
  G.N = L.N;
  G.nt = L.nt;
  G.mask = g->inflow_mask;
  return G;
}

unsigned int nblocks(long long n) { return (unsigned int)((n + kBlock - 1) / kBlock); }

}  // namespace

struct rrmhd_ctx {
  rrmhd_grid grid;
  rrmhd_params par;
  Phys K;
  Layout L;
  char* ws;
  double* Vp;
  double* taup;
  double* Us;
  double* Fh[3];
  double* partial;
  double* smax;
  DevReport* rep;
  unsigned int* blkmax;
  long long* work;              // cells left to the Newton phase of the implicit solve
  unsigned long long* wcount;   // two counters, alternating between stages
  unsigned long long stage_ctr;
  double* Zc;                   // recovery Z of the stage state per cell
  unsigned int* cost;           // per cell block: cost in the last update pass
  unsigned int* perm;           // dispatch order of the next update pass
  double* ctE;                  // constrained transport: edge EMFs [3][N]
  double* ctb;                  // ... and the stage's new face fields [ndim][N]
  hipStream_t stream;
  unsigned int newton_blocks;
  void* host;  // pinned: DevReport + one double
  // Diagnostic timing (rrmhd_profile_*).
  int prof;                     // bit k: launches of kernel class k are timed
  int prof_stride;              // ... every prof_stride-th launch of the class
  long long prof_seen[RRMHD_K_COUNT];
  std::vector<hipEvent_t> ev;   // pairs: start, stop
  std::vector<int> ev_kind;
  std::vector<long long> ev_units;
  int ev_used;
  unsigned long long serial;    // distinct per context created in this process (batch descriptor cache)
};

namespace {

constexpr int kMaxTimed = 8192;

// Record the start event of a timed launch; returns the pair index or -1.
int prof_begin(rrmhd_ctx* c, int kind, long long units) {
  if (!((c->prof >> kind) & 1) || c->ev_used >= kMaxTimed) return -1;
  if ((c->prof_seen[kind]++) % c->prof_stride != 0) return -1;
  const int i = c->ev_used;
  if (hipEventRecord(c->ev[2 * i], c->stream) != hipSuccess) return -1;  // launch left untimed
  c->ev_used = i + 1;
  c->ev_kind[i] = kind;
  c->ev_units[i] = units;
  return i;
}

void prof_end(rrmhd_ctx* c, int i) {
  // a pair whose stop event could not be recorded is left out of the totals
  if (i >= 0 && hipEventRecord(c->ev[2 * i + 1], c->stream) != hipSuccess) c->ev_kind[i] = -1;
}

rrmhd_status launch_ok() {
  return (hipGetLastError() == hipSuccess) ? RRMHD_OK : RRMHD_E_DEVICE;
}

bool same_shape(const rrmhd_ctx* c, const rrmhd_grid* g) {
  if (!g) return false;
  if (g->ndim != c->grid.ndim) return false;
  for (int e = 0; e < 3; ++e) if (g->n[e] != c->grid.n[e]) return false;
  return true;
}

Opac make_opac(const rrmhd_opacities* o) {
  Opac op;
  op.kappa = o ? o->kappa : nullptr;
  op.sigma = o ? o->sigma : nullptr;
  op.kappa0 = o ? o->kappa0 : 0.0;
  op.sigma0 = o ? o->sigma0 : 0.0;
  return op;
}

// Stage primitives and face fluxes of state Us (stride ss) into `out[d]`.
// have_prims: the stage primitives of Us are already in the workspace.
// wreset: work-list counter of the following update pass, cleared here.
rrmhd_status stage_fluxes(rrmhd_ctx* c, const rrmhd_grid* g, const double* Us, long long ss,
                          const Opac& op, double* const out[3], bool have_prims = false,
                          unsigned long long* wreset = nullptr, const DtReduce* red = nullptr) {
  const Layout& L = c->L;
  const GridDev G = make_griddev(g, L);
  int pe;
  if (!have_prims) {
    pe = prof_begin(c, RRMHD_K_PRIMS, L.N + L.nt);
    k_prims<<<nblocks(L.N + L.nt), kBlock, 0, c->stream>>>(G, Us, ss, g->inflow_U, op, c->Vp, c->taup,
                                                             L.Np, c->K, c->rep, c->blkmax, nullptr, c->Zc);
    prof_end(c, pe);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  }
  FaceArgs A;
  A.Vp = c->Vp;
  A.taup = c->taup;
  A.np = L.Np;
  A.bface = L.nb ? Us + NV * ss : nullptr;
  A.bs = ss;
  long long nbt = 0;
  for (int d = 0; d < 3; ++d) {
    const bool on = d < g->ndim;
    A.Fh[d] = on ? out[d] : nullptr;
    A.nf[d] = on ? L.nf[d] : 0;
    A.nb[d] = on ? L.nb_faces[d] : 0;
    A.dx[d] = on ? g->dx[d] : 1.0;
    nbt += A.nb[d];
  }
  DtReduce R{};
  if (red) R = *red;
  BlockOrder O;
  O.cost = c->cost;
  O.perm = c->perm;
  O.nb = L.npartial;
  const unsigned int nlaunch = (unsigned int)(nbt + (R.partial ? 1 : 0) + 1);
  pe = prof_begin(c, RRMHD_K_FACES, A.nf[0] + A.nf[1] + A.nf[2]);
  const bool mm = c->K.recon == RRMHD_RECON_MINMOD;
  constexpr int PVM = RRMHD_SOLVER_PVM, HLL = RRMHD_SOLVER_HLL, JVP = RRMHD_SOLVER_PVM_JVP;
  if (c->par.solver == HLL) {
    if (c->par.precision == RRMHD_MIXED)
      k_faces<float, -1, HLL><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
    else
      k_faces<double, -1, HLL><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
  } else if (c->par.solver == JVP) {
    if (c->par.precision == RRMHD_MIXED)
      k_faces<float, -1, JVP><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
    else
      k_faces<double, -1, JVP><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
  } else if (c->par.precision == RRMHD_MIXED) {
    if (mm) k_faces<float, 1, PVM><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
    else k_faces<float, -1, PVM><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
  } else {
    if (mm) k_faces<double, 1, PVM><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
    else k_faces<double, -1, PVM><<<nlaunch, kBlock, 0, c->stream>>>(G, A, c->K, c->rep, c->blkmax, wreset, R, O);
  }
  prof_end(c, pe);
  if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  return RRMHD_OK;
}

SimDesc make_desc(rrmhd_ctx* c, double* U, const rrmhd_opacities* opac) {
  SimDesc D;
  std::memset(&D, 0, sizeof(D));
  const Layout& L = c->L;
  const rrmhd_grid* g = &c->grid;
  D.G = make_griddev(g, L);
  D.K = c->K;
  D.op = make_opac(opac);
  D.Vp = c->Vp;
  D.taup = c->taup;
  D.FA.Vp = c->Vp;
  D.FA.taup = c->taup;
  D.FA.np = L.Np;
  for (int d = 0; d < 3; ++d) {
    const bool on = d < g->ndim;
    D.FA.Fh[d] = on ? c->Fh[d] : nullptr;
    D.FA.nf[d] = on ? L.nf[d] : 0;
    D.FA.nb[d] = on ? L.nb_faces[d] : 0;
    D.FA.dx[d] = on ? g->dx[d] : 1.0;
    D.idx[d] = on ? 1.0 / g->dx[d] : 0.0;
  }
  D.U = U;
  D.vs = g->var_stride;
  D.Us = c->Us;
  D.ns = L.Ns;
  D.inflow_U = g->inflow_U;
  D.work = c->work;
  D.wcount = c->wcount;
  D.Zc = c->Zc;
  D.rep = c->rep;
  D.blkmax = c->blkmax;
  D.partial = c->partial;
  D.npartial = L.npartial;
  D.nblkmax = L.nblkmax;
  D.mixed = (c->par.precision == RRMHD_MIXED) ? 1 : 0;
  D.solver = c->par.solver;
  return D;
}

}  // namespace

struct rrmhd_batch {
  int max_sims;
  hipStream_t stream;
  SimDesc* table;       // device
  long long* off;       // device [OFF_KINDS][max_sims + 1]
  double* smax;         // device [max_sims]
  double* dts;          // device [max_sims]: each simulation's time step
  long long* vprefix;   // device [max_sims + 1]: work-list blocks before each simulation
  // device [max_sims] each: the clock of rrmhd_advance_batch (t, n, t_end,
  // step count, cfl * dx_min)
  double* ct;
  long long* cn;
  double* ctend;
  long long* cnmax;
  double* ccfl;
  void* host[2];        // pinned staging: table + offsets + time steps + clock
  hipEvent_t ev[2];
  int cur;
  double* hsmax;        // pinned [max_sims]
  double* hclock;       // pinned [2][max_sims]: (t, n) after the last advance
  hipEvent_t ev_clock;  // recorded after the last advance's clock copy
  int clock_n;          // simulations of the last advance (0: none yet)
  unsigned int newton_cap;
  // The descriptor table on the device describes these simulations (same
  // contexts, states and, when built by a step, opacities): a call with the
  // same list reuses it and uploads only its time steps. A table built by a
  // signal-speed pass (no opacities) serves only signal-speed passes.
  int cached_n;
  bool cached_with_opac;
  std::vector<unsigned long long> cached_serial;
  std::vector<const double*> cached_U;
  std::vector<rrmhd_opacities> cached_op;
  std::vector<char> cached_has_op;
  long long cached_tot[4];
};

namespace {

size_t batch_table_bytes(int m) { return align256(sizeof(SimDesc) * (size_t)m); }
size_t batch_off_bytes(int m) { return align256(sizeof(long long) * OFF_KINDS * (size_t)(m + 1)); }
size_t batch_dt_bytes(int m) { return align256(sizeof(double) * (size_t)m); }
// clock planes: t, n, t_end, step count, cfl * dx_min
constexpr int kClockPlanes = 5;
size_t batch_staging_bytes(int m) {
  return batch_table_bytes(m) + batch_off_bytes(m) + (1 + kClockPlanes) * batch_dt_bytes(m);
}

// Host values of a batched advance's clock, uploaded with the table.
struct ClockIn {
  const double* t;
  const long long* n;
  const double* tend;
  const long long* nmax;
  const double* cfl_dx;
};

bool same_opac(const rrmhd_opacities* a, const rrmhd_opacities& b) {
  return a->kappa == b.kappa && a->sigma == b.sigma && a->kappa0 == b.kappa0 && a->sigma0 == b.sigma0;
}

// Fill a staging buffer with the batch's descriptors and block offsets and
// copy it to the device (enqueued). Returns total blocks per kind in tot[].
rrmhd_status batch_upload(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, double* const* U,
                          const double* dt, const rrmhd_opacities* const* opac, long long tot[OFF_KINDS],
                          const ClockIn* clock = nullptr) {
  // Is the device table already that of this list?
  bool same = b->cached_n == nsim && (opac == nullptr || b->cached_with_opac);
  for (int s = 0; s < nsim && same; ++s) {
    same = ctx[s]->serial == b->cached_serial[s] && U[s] == b->cached_U[s];
    if (same && opac) {
      const rrmhd_opacities* o = opac[s];
      same = (o != nullptr) == (b->cached_has_op[s] != 0) && (o == nullptr || same_opac(o, b->cached_op[s]));
    }
  }
  const int k = b->cur;
  b->cur ^= 1;
  if (hipEventSynchronize(b->ev[k]) != hipSuccess) return RRMHD_E_DEVICE;
  char* hk = (char*)b->host[k];
  if (!same) {
    b->cached_n = 0;  // until the new table is complete
    SimDesc* T = (SimDesc*)hk;
    long long* off = (long long*)(hk + batch_table_bytes(b->max_sims));
    for (int i = 0; i < OFF_KINDS; ++i) { off[i * (nsim + 1)] = 0; tot[i] = 0; }
    for (int s = 0; s < nsim; ++s) {
      rrmhd_ctx* c = ctx[s];
      T[s] = make_desc(c, U[s], opac ? opac[s] : nullptr);
      const Layout& L = c->L;
      const long long nbc = nblocks(L.N);
      const long long nb[OFF_KINDS] = {(long long)nblocks(L.N + L.nt), L.nb_faces[0] + L.nb_faces[1] + L.nb_faces[2],
                                       nbc, (L.N + kBlock / 4 - 1) / (kBlock / 4)};
      for (int i = 0; i < OFF_KINDS; ++i) {
        tot[i] += nb[i];
        off[i * (nsim + 1) + s + 1] = tot[i];
      }
    }
    if (hipMemcpyAsync(b->table, T, sizeof(SimDesc) * nsim, hipMemcpyHostToDevice, b->stream) != hipSuccess)
      return RRMHD_E_DEVICE;
    if (hipMemcpyAsync(b->off, off, sizeof(long long) * OFF_KINDS * (nsim + 1), hipMemcpyHostToDevice, b->stream) !=
        hipSuccess)
      return RRMHD_E_DEVICE;
    b->cached_n = nsim;
    b->cached_with_opac = opac != nullptr;
    for (int s = 0; s < nsim; ++s) {
      b->cached_serial[s] = ctx[s]->serial;
      b->cached_U[s] = U[s];
      const rrmhd_opacities* o = opac ? opac[s] : nullptr;
      b->cached_has_op[s] = o ? 1 : 0;
      if (o) b->cached_op[s] = *o;
    }
    // the Newton launch: a grid walking every simulation's work-list blocks
    if (tot[OFF_NEWTON] > (long long)b->newton_cap) tot[OFF_NEWTON] = b->newton_cap;
    for (int i = 0; i < OFF_KINDS; ++i) b->cached_tot[i] = tot[i];
  } else {
    for (int i = 0; i < OFF_KINDS; ++i) tot[i] = b->cached_tot[i];
  }
  if (dt) {
    double* hd = (double*)(hk + batch_table_bytes(b->max_sims) + batch_off_bytes(b->max_sims));
    std::memcpy(hd, dt, sizeof(double) * nsim);
    if (hipMemcpyAsync(b->dts, hd, sizeof(double) * nsim, hipMemcpyHostToDevice, b->stream) != hipSuccess)
      return RRMHD_E_DEVICE;
  }
  if (clock) {
    char* hc = hk + batch_table_bytes(b->max_sims) + batch_off_bytes(b->max_sims) + batch_dt_bytes(b->max_sims);
    const size_t pb = batch_dt_bytes(b->max_sims);
    const void* src[kClockPlanes] = {clock->t, clock->n, clock->tend, clock->nmax, clock->cfl_dx};
    void* dst[kClockPlanes] = {b->ct, b->cn, b->ctend, b->cnmax, b->ccfl};
    for (int i = 0; i < kClockPlanes; ++i) {
      std::memcpy(hc + i * pb, src[i], 8 * (size_t)nsim);
      if (hipMemcpyAsync(dst[i], hc + i * pb, 8 * (size_t)nsim, hipMemcpyHostToDevice, b->stream) != hipSuccess)
        return RRMHD_E_DEVICE;
    }
  }
  if (hipEventRecord(b->ev[k], b->stream) != hipSuccess) return RRMHD_E_DEVICE;
  return RRMHD_OK;
}

rrmhd_status batch_check(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, const void* const* U) {
  if (!b || nsim < 1 || nsim > b->max_sims || !ctx || !U) return RRMHD_E_INVALID;
  for (int s = 0; s < nsim; ++s) {
    if (!ctx[s] || !U[s]) return RRMHD_E_INVALID;
    if (ctx[s]->par.rk_order != ctx[0]->par.rk_order) return RRMHD_E_INVALID;
    if (ctx[s]->par.ct) return RRMHD_E_INVALID;  // constrained transport: single-simulation entry points only
    for (int t = 0; t < s; ++t)
      if (ctx[t] == ctx[s]) return RRMHD_E_INVALID;  // each context's workspace is used once per launch
  }
  return RRMHD_OK;
}


// Signal-speed passes of a batch into b->smax (simulations at the end of
// their clock skipped when C.t is set).
rrmhd_status batch_speed_launches(rrmhd_batch* b, int nsim, const long long tot[OFF_KINDS], const BatchClock& C) {
  k_speed_b<<<(unsigned int)tot[OFF_CELLS], kBlock, 0, b->stream>>>(b->table, b->off, nsim, C);
  if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  k_reduce_max_b<<<(unsigned int)nsim, kRedBlock, 0, b->stream>>>(b->table, b->smax, C, 1);
  return launch_ok();
}

// The stages of one IMEX step of a batch with the time steps in b->dts
// (simulations whose gate entry is 0 skipped when gate is set). prims0: the
// first stage's primitives are in the workspaces (left by the previous step
// with `after`). after: the last stage also leaves the next step's
// primitives and signal-speed maxima (stage_args).
rrmhd_status batch_step_launches(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, const long long tot[OFF_KINDS],
                                 const double* gate, bool prims0 = false, bool after = false) {
  double co[3][3];
  int ns;
  if (ctx[0]->par.rk_order == 3) {
    const double t[3][3] = {{1.0, 0.0, 1.0}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};
    std::memcpy(co, t, sizeof(t));
    ns = 3;
  } else {
    const double t[3][3] = {{1.0, 0.0, 1.0}, {0.5, 0.5, 0.5}, {0.0, 0.0, 0.0}};
    std::memcpy(co, t, sizeof(t));
    ns = 2;
  }
  for (int s = 0; s < ns; ++s) {
    const int last = (s == ns - 1) ? 1 : 0;
    // later stages get their primitives from the passes that finish each cell
    if (s == 0 && !prims0) {
      k_prims_b<<<(unsigned int)tot[OFF_PRIMS], kBlock, 0, b->stream>>>(b->table, b->off, nsim, s, gate);
      if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    }
    bool has[3] = {false, false, false};
    for (int t = 0; t < nsim; ++t) has[ctx[t]->par.solver] = true;
    if (has[RRMHD_SOLVER_PVM])
      k_faces_b<RRMHD_SOLVER_PVM><<<(unsigned int)tot[OFF_FACES], kBlock, 0, b->stream>>>(b->table, b->off, nsim,
                                                                                     gate);
    if (has[RRMHD_SOLVER_HLL])
      k_faces_b<RRMHD_SOLVER_HLL><<<(unsigned int)tot[OFF_FACES], kBlock, 0, b->stream>>>(b->table, b->off, nsim,
                                                                                     gate);
    if (has[RRMHD_SOLVER_PVM_JVP])
      k_faces_b<RRMHD_SOLVER_PVM_JVP><<<(unsigned int)tot[OFF_FACES], kBlock, 0, b->stream>>>(b->table, b->off,
                                                                                         nsim, gate);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    const int aft = (last && after) ? 1 : 0;
    k_update_b<<<(unsigned int)tot[OFF_CELLS], kBlock, 0, b->stream>>>(b->table, b->off, b->dts, nsim, s, last,
                                                                       co[s][0], co[s][1], co[s][2], gate, aft);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    k_wprefix_b<<<1, kRedBlock, 0, b->stream>>>(b->table, nsim, b->vprefix, gate);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    k_newton_b<<<(unsigned int)tot[OFF_NEWTON], kBlock, 0, b->stream>>>(b->table, b->vprefix, b->dts, nsim, s, last,
                                                                        co[s][0], co[s][1], co[s][2], aft);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  }
  return RRMHD_OK;
}

// Point a context at its workspace (no allocation).
void ctx_bind(rrmhd_ctx* c, const rrmhd_grid* g, const rrmhd_params* p, const Layout& L, char* ws,
              void* hip_stream) {
  c->grid = *g;
  c->par = *p;
  c->K = make_phys(p);
  c->L = L;
  c->ws = ws;
  c->Vp = (double*)(c->ws + L.off_Vp);
  c->taup = (double*)(c->ws + L.off_taup);
  c->Us = (double*)(c->ws + L.off_Us);
  for (int d = 0; d < 3; ++d) c->Fh[d] = (double*)(c->ws + L.off_Fh[d]);
  c->partial = (double*)(c->ws + L.off_partial);
  c->smax = (double*)(c->ws + L.off_smax);
  c->rep = (DevReport*)(c->ws + L.off_rep);
  c->blkmax = (unsigned int*)(c->ws + L.off_blkmax);
  c->work = (long long*)(c->ws + L.off_work);
  c->wcount = (unsigned long long*)(c->ws + L.off_wcount);
  c->stage_ctr = 0;
  c->Zc = (double*)(c->ws + L.off_Zc);
  c->cost = (unsigned int*)(c->ws + L.off_cost);
  c->perm = (unsigned int*)(c->ws + L.off_perm);
  c->ctE = L.nb ? (double*)(c->ws + L.off_ctE) : nullptr;
  c->ctb = L.nb ? (double*)(c->ws + L.off_ctb) : nullptr;
  c->stream = (hipStream_t)hip_stream;
  c->host = nullptr;
  c->prof = 0;
  c->prof_stride = 1;
  for (int k = 0; k < RRMHD_K_COUNT; ++k) c->prof_seen[k] = 0;
  c->ev_used = 0;
  static std::atomic<unsigned long long> next_serial{1};
  c->serial = next_serial.fetch_add(1);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
    ncu = 256;
  c->newton_blocks = (unsigned int)(4 * ncu * (256 / kBlock));  // kBlock/4 cells (4 lanes each) per block
}

// Clear what the kernels expect to start at zero: the failure counters, the
// per-block iteration maxima and the update blocks' costs (enqueued kernels,
// no memset, so a captured graph replays them as well).
rrmhd_status ctx_clear(rrmhd_ctx* c) {
  k_report_reset<<<64, kBlock, 0, c->stream>>>(c->rep, c->blkmax, 2 * c->L.nblkmax);
  if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  k_zero_u32<<<64, kBlock, 0, c->stream>>>(c->cost, c->L.npartial);
  return launch_ok();
}

}  // namespace

extern "C" {

void rrmhd_default_params(rrmhd_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->gamma = 5.0 / 3.0;
  p->a_rad = 1.0;
  p->t_coeff = 1.0;
  p->pvm_eps = 1e-8;
  p->c2p_tol = 1e-12;
  p->imp_tol = 1e-13;
  p->rho_floor = 1e-12;
  p->p_floor = 1e-12;
  p->pvm_k = 3;
  p->beta_mode = RRMHD_BETA_RAD_ONLY;
  p->recon = RRMHD_RECON_MINMOD;
  p->rk_order = 2;
  p->c2p_maxit = 100;
  p->imp_maxit = 50;
  p->imp_picard_it = 8;
  p->imp_method = RRMHD_IMP_PICARD_NEWTON;
  p->precision = RRMHD_FP64;
  p->pvm_eps_mixed = 1.0 / 4096.0;
}

size_t rrmhd_workspace_bytes(const rrmhd_grid* g, const rrmhd_params* p) {
  if (!grid_valid(g) || !params_valid(p) || !ct_grid_ok(g, p)) return 0;
  return make_layout(g, p).total;
}

rrmhd_status rrmhd_init(rrmhd_ctx** out, const rrmhd_grid* g, const rrmhd_params* p, void* workspace,
                        size_t ws_bytes, void* hip_stream) {
  if (!out) return RRMHD_E_INVALID;
  *out = nullptr;
  if (!grid_valid(g) || !params_valid(p) || !ct_grid_ok(g, p)) return RRMHD_E_INVALID;
  const Layout L = make_layout(g, p);
  if (!workspace || ws_bytes < L.total || ((uintptr_t)workspace & 255u) != 0) return RRMHD_E_WORKSPACE;
  rrmhd_ctx* c = new (std::nothrow) rrmhd_ctx;
  if (!c) return RRMHD_E_DEVICE;
  ctx_bind(c, g, p, L, (char*)workspace, hip_stream);
  if (hipHostMalloc(&c->host, sizeof(DevReport) + sizeof(double), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return RRMHD_E_DEVICE;
  }
  if (ctx_clear(c) != RRMHD_OK) {
    (void)hipHostFree(c->host);
    delete c;
    return RRMHD_E_DEVICE;
  }
  *out = c;
  return RRMHD_OK;
}

rrmhd_status rrmhd_prim_to_cons(rrmhd_ctx* c, const double* V, double* U) {
  if (!c || !V || !U) return RRMHD_E_INVALID;
  const long long N = c->L.N, s = c->grid.var_stride;
  if (N == 0) return RRMHD_OK;
  k_p2c<<<nblocks(N), kBlock, 0, c->stream>>>(N, V, s, U, s, c->K);
  return launch_ok();
}

rrmhd_status rrmhd_cons_to_prim(rrmhd_ctx* c, const double* U, double* V) {
  if (!c || !V || !U) return RRMHD_E_INVALID;
  const long long N = c->L.N, s = c->grid.var_stride;
  if (N == 0) return RRMHD_OK;
  k_c2p<<<nblocks(N), kBlock, 0, c->stream>>>(N, U, s, V, s, c->K, c->rep, c->blkmax);
  return launch_ok();
}

rrmhd_status rrmhd_face_fluxes(rrmhd_ctx* c, const double* U, const rrmhd_opacities* opac, double* Fh) {
  if (!c || !U || !Fh) return RRMHD_E_INVALID;
  double* out[3] = {Fh, nullptr, nullptr};
  for (int d = 1; d < c->grid.ndim; ++d) out[d] = out[d - 1] + NV * c->L.nf[d - 1];
  return stage_fluxes(c, &c->grid, U, c->grid.var_stride, make_opac(opac), out);
}

namespace {

// Blocks of the single-simulation work-list pass: a few per CU, at most one
// per cell block.
unsigned int worklist_blocks(const rrmhd_ctx* c) {
  const long long nb = nblocks(c->L.N);
  return (unsigned int)((nb < c->newton_blocks) ? nb : c->newton_blocks);
}

// The stages of one IMEX step. dt_dev: when set, the time step is read on the
// device from dt_dev[0] (dt unused). prims0: the first stage's primitives are
// already in the workspace. prims_after: also recover the primitives of the
// step's result (the next step's first stage) and the signal-speed block
// maxima, cell blocks then work-list blocks, into `partial`.
rrmhd_status step_stages(rrmhd_ctx* c, double* U, const rrmhd_grid* g, double dt, const double* dt_dev,
                         const Opac& op, bool prims0, bool prims_after, const DtReduce* red = nullptr) {
  const Layout& L = c->L;
  const GridDev G = make_griddev(g, L);
  const long long vs = g->var_stride;
  // Stage coefficients (a0, a1, c) of U* = a0 U^(0) + a1 U^(s) + c dt L(U^(s)).
  double co[3][3];
  int ns;
  if (c->par.rk_order == 3) {
    const double t[3][3] = {{1.0, 0.0, 1.0}, {0.75, 0.25, 0.25}, {1.0 / 3.0, 2.0 / 3.0, 2.0 / 3.0}};
    std::memcpy(co, t, sizeof(t));
    ns = 3;
  } else {
    const double t[3][3] = {{1.0, 0.0, 1.0}, {0.5, 0.5, 0.5}, {0.0, 0.0, 0.0}};
    std::memcpy(co, t, sizeof(t));
    ns = 2;
  }
  double* const fl[3] = {c->Fh[0], c->Fh[1], c->Fh[2]};
  const unsigned int nbn = worklist_blocks(c);
  for (int s = 0; s < ns; ++s) {
    // work-list counters alternate between stages
    unsigned long long* wc = c->wcount + (c->stage_ctr & 1);
    c->stage_ctr += 1;
    const double* Us = (s == 0) ? U : c->Us;
    const long long ss = (s == 0) ? vs : L.Ns;
    const rrmhd_status st = stage_fluxes(c, g, Us, ss, op, fl, (s == 0) ? prims0 : true, wc,
                                         (s == 0) ? red : nullptr);
    if (st != RRMHD_OK) return st;
    StageArgs A;
    A.U0 = U; A.s0 = vs;
    A.Us = Us; A.ss = ss;
    const bool last = (s == ns - 1);
    A.Uo = last ? U : c->Us;
    A.so = last ? vs : L.Ns;
    for (int d = 0; d < 3; ++d) {
      A.Fh[d] = (d < g->ndim) ? c->Fh[d] : c->Fh[0];
      A.nf[d] = (d < g->ndim) ? L.nf[d] : 0;
      A.idx[d] = (d < g->ndim) ? 1.0 / g->dx[d] : 0.0;
    }
    A.a0 = co[s][0];
    A.a1 = co[s][1];
    A.cdt = co[s][2] * dt;
    A.dtp = dt_dev;
    A.cc = co[s][2];
    A.Zc = c->Zc;
    A.nextp = (!last || prims_after) ? 1 : 0;
    A.speed = (last && prims_after) ? 1 : 0;
    A.Vp = c->Vp;
    A.taup = c->taup;
    A.np = L.Np;
    A.partial = c->partial;
    A.npart = L.npartial;
    A.perm = c->perm;
    A.cost = c->cost;
    A.bnew = nullptr;
    if (L.nb) {
      // constrained transport: edge EMFs, then the new face fields
      CTArgs T;
      for (int d = 0; d < 3; ++d) {
        T.Fh[d] = (d < g->ndim) ? (const void*)c->Fh[d] : (const void*)c->Fh[0];
        T.nf[d] = (d < g->ndim) ? L.nf[d] : 0;
        T.idx[d] = A.idx[d];
      }
      T.Vp = c->Vp;
      T.np = L.Np;
      T.E = c->ctE;
      T.bnew = c->ctb;
      T.b0 = U + NV * vs;
      T.s0 = vs;
      T.bs = Us + NV * ss;
      T.ss = ss;
      T.a0 = A.a0;
      T.a1 = A.a1;
      T.cdt = A.cdt;
      T.cc = A.cc;
      T.dtp = A.dtp;
      if (c->par.precision == RRMHD_MIXED)
        k_ct_emf<float><<<nblocks(L.N), kBlock, 0, c->stream>>>(G, T);
      else
        k_ct_emf<double><<<nblocks(L.N), kBlock, 0, c->stream>>>(G, T);
      if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
      k_ct_face<<<nblocks(L.N), kBlock, 0, c->stream>>>(G, T);
      if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
      A.bnew = c->ctb;
    }
    int pe = prof_begin(c, RRMHD_K_UPDATE, L.N);
    if (c->par.precision == RRMHD_MIXED)
      k_update<float><<<nblocks(L.N), kBlock, 0, c->stream>>>(G, A, op, c->K, c->rep, c->blkmax, c->work, wc);
    else
      k_update<double><<<nblocks(L.N), kBlock, 0, c->stream>>>(G, A, op, c->K, c->rep, c->blkmax, c->work, wc);
    prof_end(c, pe);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    pe = prof_begin(c, RRMHD_K_NEWTON, L.N);
    k_newton<<<nbn, kBlock, 0, c->stream>>>(G, A, op, c->K, c->rep, c->blkmax, c->work, wc);
    prof_end(c, pe);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  }
  return RRMHD_OK;
}

}  // namespace

rrmhd_status rrmhd_step(rrmhd_ctx* c, double* U, const rrmhd_grid* g, double dt, const rrmhd_opacities* opac) {
  if (!c || !U || !same_shape(c, g) || !grid_valid(g)) return RRMHD_E_INVALID;
  if (!(dt >= 0.0) || !(dt < 1e300)) return RRMHD_E_INVALID;
  return step_stages(c, U, g, dt, nullptr, make_opac(opac), false, false);
}

rrmhd_status rrmhd_advance(rrmhd_ctx* c, double* U, const rrmhd_grid* g, double cfl, int nsteps,
                           const rrmhd_opacities* opac, double* dt_out) {
  if (!c || !U || !same_shape(c, g) || !grid_valid(g)) return RRMHD_E_INVALID;
  if (!(cfl > 0.0) || !(cfl < 1e300) || nsteps < 0) return RRMHD_E_INVALID;
  const Layout& L = c->L;
  const GridDev G = make_griddev(g, L);
  const Opac op = make_opac(opac);
  double dxmin = g->dx[0];
  for (int d = 1; d < g->ndim; ++d) dxmin = (g->dx[d] < dxmin) ? g->dx[d] : dxmin;
  const double cfl_dx = cfl * dxmin;
  const long long nred = L.npartial + worklist_blocks(c);
  for (int k = 0; k < nsteps; ++k) {
    if (k == 0) {
      // later steps get their primitives and speeds from the previous step
      int pe = prof_begin(c, RRMHD_K_PRIMS, L.N + L.nt);
      k_prims_speed<<<nblocks(L.N + L.nt), kBlock, 0, c->stream>>>(G, U, g->var_stride, g->inflow_U, op, c->Vp,
                                                                    c->taup, L.Np, c->K, c->rep, c->blkmax,
                                                                    nullptr, c->Zc, c->partial);
      prof_end(c, pe);
      if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    }
    // the step's dt is formed by block 0 of the first face launch
    DtReduce red;
    red.partial = c->partial;
    red.n = (k == 0) ? L.npartial : nred;
    red.sd = c->smax;
    red.cfl_dx = cfl_dx;
    red.dt_out = dt_out;
    red.k = k;
    const rrmhd_status st = step_stages(c, U, g, 0.0, c->smax + 1, op, true, k + 1 < nsteps, &red);
    if (st != RRMHD_OK) return st;
  }
  return RRMHD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free variant of rrmhd_advance. Its workspace is this array: one
// copy per device, allocated when the code object is loaded and held until
// the process ends. Host code never passes `scratch` itself to a kernel (on
// the host it is only a stand-in for the symbol); it uses the device address
// that hipGetSymbolAddress returns for the current device.
static constexpr size_t kScratchBytes = (size_t)RRMHD_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current and kept.
rrmhd_status scratch_for_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RRMHD_E_DEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RRMHD_E_DEVICE;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RRMHD_OK;
}

}  // namespace

extern "C" {

rrmhd_status rrmhd_advance_noalloc(const rrmhd_grid* g, const rrmhd_params* p, double* U, double cfl, int nsteps,
                                   const rrmhd_opacities* opac, double* dt_out, rrmhd_report* report_dev,
                                   void* hip_stream) {
  if (!U || !grid_valid(g) || !params_valid(p) || !ct_grid_ok(g, p)) return RRMHD_E_INVALID;
  if (!(cfl > 0.0) || !(cfl < 1e300) || nsteps < 0) return RRMHD_E_INVALID;
  const Layout L = make_layout(g, p);
  if (L.total > kScratchBytes) return RRMHD_E_WORKSPACE;
  void* ws = nullptr;
  const rrmhd_status sst = scratch_for_current_device(&ws);
  if (sst != RRMHD_OK) return sst;
  // A context on the stack (its profiling vectors stay empty: no host
  // allocation), pointed at the device's scratch array.
  rrmhd_ctx c;
  ctx_bind(&c, g, p, L, (char*)ws, hip_stream);
  if (ctx_clear(&c) != RRMHD_OK) return RRMHD_E_DEVICE;
  const rrmhd_status st = rrmhd_advance(&c, U, g, cfl, nsteps, opac, dt_out);
  if (st != RRMHD_OK) return st;
  if (report_dev) {
    k_report_out<<<1, kRedBlock, 0, c.stream>>>(c.rep, c.blkmax, L.nblkmax, report_dev);
    return launch_ok();
  }
  return RRMHD_OK;
}

rrmhd_status rrmhd_max_speed(rrmhd_ctx* c, const double* U, const rrmhd_grid* g, double* smax_host) {
  if (!c || !U || !smax_host || !same_shape(c, g)) return RRMHD_E_INVALID;
  const Layout& L = c->L;
  const GridDev G = make_griddev(g, L);
  const int pe = prof_begin(c, RRMHD_K_SPEED, L.N);
  k_speed<<<nblocks(L.N), kBlock, 0, c->stream>>>(G, U, g->var_stride, c->K, c->partial, c->rep, c->blkmax);
  prof_end(c, pe);
  if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  k_reduce_max<<<1, kRedBlock, 0, c->stream>>>(c->partial, L.npartial, c->smax);
  if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  double* h = (double*)((char*)c->host + sizeof(DevReport));
  if (hipMemcpyAsync(h, c->smax, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return RRMHD_E_DEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return RRMHD_E_DEVICE;
  *smax_host = *h;
  return RRMHD_OK;
}

rrmhd_status rrmhd_report_sync(rrmhd_ctx* c, rrmhd_report* out) {
  if (!c || !out) return RRMHD_E_INVALID;
  DevReport* h = (DevReport*)c->host;
  k_report_fold<<<1, kRedBlock, 0, c->stream>>>(c->rep, c->blkmax, c->L.nblkmax);
  if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
  if (hipMemcpyAsync(h, c->rep, sizeof(DevReport), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return RRMHD_E_DEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return RRMHD_E_DEVICE;
  out->c2p_fail = (long long)h->c2p_fail;
  out->pvm_fallback = (long long)h->pvm_fallback;
  out->imp_fail = (long long)h->imp_fail;
  out->nonfinite = (long long)h->nonfinite;
  out->e_floor_hits = (long long)h->e_floor_hits;
  out->first_bad_cell = (h->first_bad == ULLONG_MAX) ? -1 : (long long)h->first_bad;
  out->max_c2p_it = (int)h->max_c2p_it;
  out->max_imp_it = (int)h->max_imp_it;
  k_report_reset<<<64, kBlock, 0, c->stream>>>(c->rep, c->blkmax, 2 * c->L.nblkmax);
  return launch_ok();
}

rrmhd_status rrmhd_profile_enable(rrmhd_ctx* c, int enable) {
  if (!c || enable < 0 || enable >= (1 << RRMHD_K_COUNT)) return RRMHD_E_INVALID;
  if (enable && c->ev.empty()) {
    // all events or none: a partial set would be taken as created next time
    std::vector<hipEvent_t> ev(2 * kMaxTimed, nullptr);
    for (size_t n = 0; n < ev.size(); ++n) {
      if (hipEventCreate(&ev[n]) != hipSuccess) {
        for (size_t m = 0; m < n; ++m) (void)hipEventDestroy(ev[m]);
        return RRMHD_E_DEVICE;
      }
    }
    c->ev.swap(ev);
    c->ev_kind.assign(kMaxTimed, -1);
    c->ev_units.assign(kMaxTimed, 0);
  }
  c->prof = enable;
  if (enable) {
    c->ev_used = 0;
    for (int k = 0; k < RRMHD_K_COUNT; ++k) c->prof_seen[k] = 0;
  }
  return RRMHD_OK;
}

rrmhd_status rrmhd_profile_stride(rrmhd_ctx* c, int stride) {
  if (!c || stride < 1) return RRMHD_E_INVALID;
  c->prof_stride = stride;
  return RRMHD_OK;
}

rrmhd_status rrmhd_profile_read(rrmhd_ctx* c, int k, double* total_ms, long long* launches, long long* units) {
  if (!c || !total_ms || !launches || !units || k < 0 || k >= RRMHD_K_COUNT) return RRMHD_E_INVALID;
  *total_ms = 0.0;
  *launches = 0;
  *units = 0;
  if (c->ev_used == 0) return RRMHD_OK;
  if (hipEventSynchronize(c->ev[2 * (c->ev_used - 1) + 1]) != hipSuccess) return RRMHD_E_DEVICE;
  for (int i = 0; i < c->ev_used; ++i) {
    if (c->ev_kind[i] != k) continue;
    if (hipEventSynchronize(c->ev[2 * i + 1]) != hipSuccess) return RRMHD_E_DEVICE;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) != hipSuccess) return RRMHD_E_DEVICE;
    *total_ms += ms;
    *launches += 1;
    *units += c->ev_units[i];
  }
  return RRMHD_OK;
}

void rrmhd_destroy(rrmhd_ctx* c) {
  if (!c) return;
  // teardown: nothing to report an error to; release what can be released
  (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->ev) (void)hipEventDestroy(e);
  if (c->host) (void)hipHostFree(c->host);
  delete c;
}

size_t rrmhd_batch_workspace_bytes(int max_sims) {
  if (max_sims < 1 || max_sims > 65536) return 0;
  return batch_table_bytes(max_sims) + batch_off_bytes(max_sims) + (2 + kClockPlanes) * batch_dt_bytes(max_sims) +
         batch_dt_bytes(max_sims + 1);
}

rrmhd_status rrmhd_batch_init(rrmhd_batch** out, int max_sims, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out) return RRMHD_E_INVALID;
  *out = nullptr;
  const size_t need = rrmhd_batch_workspace_bytes(max_sims);
  if (need == 0) return RRMHD_E_INVALID;
  if (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255u) != 0) return RRMHD_E_WORKSPACE;
  rrmhd_batch* b = new (std::nothrow) rrmhd_batch();
  if (!b) return RRMHD_E_DEVICE;
  b->max_sims = max_sims;
  b->stream = (hipStream_t)hip_stream;
  char* w = (char*)workspace;
  b->table = (SimDesc*)w;
  b->off = (long long*)(w + batch_table_bytes(max_sims));
  b->smax = (double*)(w + batch_table_bytes(max_sims) + batch_off_bytes(max_sims));
  b->dts = (double*)(w + batch_table_bytes(max_sims) + batch_off_bytes(max_sims) + batch_dt_bytes(max_sims));
  {
    char* cw = w + batch_table_bytes(max_sims) + batch_off_bytes(max_sims) + 2 * batch_dt_bytes(max_sims);
    const size_t pb = batch_dt_bytes(max_sims);
    b->ct = (double*)cw;
    b->cn = (long long*)(cw + pb);
    b->ctend = (double*)(cw + 2 * pb);
    b->cnmax = (long long*)(cw + 3 * pb);
    b->ccfl = (double*)(cw + 4 * pb);
    b->vprefix = (long long*)(cw + 5 * pb);
  }
  b->clock_n = 0;
  const size_t hb = batch_staging_bytes(max_sims);
  bool ok = true;
  try {
    b->cached_serial.assign(max_sims, 0);
    b->cached_U.assign(max_sims, nullptr);
    b->cached_op.assign(max_sims, rrmhd_opacities{});
    b->cached_has_op.assign(max_sims, 0);
  } catch (...) {
    ok = false;
  }
  for (int k = 0; k < 2 && ok; ++k) {
    ok = hipHostMalloc(&b->host[k], hb, hipHostMallocDefault) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&b->ev[k], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipHostMalloc((void**)&b->hsmax, sizeof(double) * max_sims, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&b->hclock, 2 * sizeof(double) * max_sims, hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&b->ev_clock, hipEventDisableTiming) == hipSuccess;
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
    ncu = 256;
  b->newton_cap = (unsigned int)(4 * ncu * (256 / kBlock));
  if (!ok) {
    rrmhd_batch_destroy(b);
    return RRMHD_E_DEVICE;
  }
  *out = b;
  return RRMHD_OK;
}

rrmhd_status rrmhd_max_speed_batch(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, const double* const* U,
                                   double* smax_host) {
  rrmhd_status st = batch_check(b, nsim, ctx, (const void* const*)U);
  if (st != RRMHD_OK) return st;
  if (!smax_host) return RRMHD_E_INVALID;
  long long tot[OFF_KINDS];
  st = batch_upload(b, nsim, ctx, (double* const*)U, nullptr, nullptr, tot);
  if (st != RRMHD_OK) return st;
  st = batch_speed_launches(b, nsim, tot, BatchClock{});
  if (st != RRMHD_OK) return st;
  if (hipMemcpyAsync(b->hsmax, b->smax, sizeof(double) * nsim, hipMemcpyDeviceToHost, b->stream) != hipSuccess)
    return RRMHD_E_DEVICE;
  if (hipStreamSynchronize(b->stream) != hipSuccess) return RRMHD_E_DEVICE;
  std::memcpy(smax_host, b->hsmax, sizeof(double) * nsim);
  return RRMHD_OK;
}

rrmhd_status rrmhd_step_batch(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, double* const* U,
                              const double* dt_host, const rrmhd_opacities* const* opac) {
  rrmhd_status st = batch_check(b, nsim, ctx, (const void* const*)U);
  if (st != RRMHD_OK) return st;
  if (!dt_host) return RRMHD_E_INVALID;
  for (int s = 0; s < nsim; ++s)
    if (!(dt_host[s] >= 0.0) || !(dt_host[s] < 1e300)) return RRMHD_E_INVALID;
  long long tot[OFF_KINDS];
  st = batch_upload(b, nsim, ctx, U, dt_host, opac, tot);
  if (st != RRMHD_OK) return st;
  return batch_step_launches(b, nsim, ctx, tot, nullptr);
}

rrmhd_status rrmhd_advance_batch(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, double* const* U,
                                 const rrmhd_opacities* const* opac, const double* cfl_dx, const double* t_end,
                                 const long long* max_steps, const double* t, const long long* n, int nsteps) {
  rrmhd_status st = batch_check(b, nsim, ctx, (const void* const*)U);
  if (st != RRMHD_OK) return st;
  if (!cfl_dx || !t_end || !max_steps || !t || !n || nsteps < 0) return RRMHD_E_INVALID;
  for (int s = 0; s < nsim; ++s) {
    if (!(cfl_dx[s] > 0.0) || !(cfl_dx[s] < 1e300)) return RRMHD_E_INVALID;
    if (!(t_end[s] >= 0.0) || !(t[s] >= 0.0) || !(t[s] < 1e300) || n[s] < 0) return RRMHD_E_INVALID;
    if (max_steps[s] < 0 && !(t_end[s] < 1e300)) return RRMHD_E_INVALID;  // neither end given
  }
  long long tot[OFF_KINDS];
  const ClockIn ci = {t, n, t_end, max_steps, cfl_dx};
  st = batch_upload(b, nsim, ctx, U, nullptr, opac, tot, &ci);
  if (st != RRMHD_OK) return st;
  const BatchClock C = {b->ct, b->cn, b->ctend, b->cnmax, b->ccfl};
  for (int k = 0; k < nsteps; ++k) {
    // later steps take their primitives and speed maxima from the last stage
    // of the step before
    if (k == 0) {
      st = batch_speed_launches(b, nsim, tot, C);
      if (st != RRMHD_OK) return st;
    } else {
      k_reduce_max_b<<<(unsigned int)nsim, kRedBlock, 0, b->stream>>>(b->table, b->smax, C, 2);
      if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    }
    k_dt_b<<<1, kRedBlock, 0, b->stream>>>(b->table, b->smax, b->dts, nsim, C);
    if (launch_ok() != RRMHD_OK) return RRMHD_E_DEVICE;
    st = batch_step_launches(b, nsim, ctx, tot, b->dts, k > 0, k + 1 < nsteps);
    if (st != RRMHD_OK) return st;
  }
  if (hipMemcpyAsync(b->hclock, b->ct, sizeof(double) * nsim, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
      hipMemcpyAsync(b->hclock + b->max_sims, b->cn, sizeof(long long) * nsim, hipMemcpyDeviceToHost, b->stream) !=
          hipSuccess ||
      hipEventRecord(b->ev_clock, b->stream) != hipSuccess)
    return RRMHD_E_DEVICE;
  b->clock_n = nsim;
  return RRMHD_OK;
}

rrmhd_status rrmhd_batch_clock(rrmhd_batch* b, int nsim, double* t, long long* n) {
  if (!b || !t || !n || nsim < 1 || nsim != b->clock_n) return RRMHD_E_INVALID;
  if (hipEventSynchronize(b->ev_clock) != hipSuccess) return RRMHD_E_DEVICE;
  std::memcpy(t, b->hclock, sizeof(double) * nsim);
  std::memcpy(n, b->hclock + b->max_sims, sizeof(long long) * nsim);
  return RRMHD_OK;
}

void rrmhd_batch_destroy(rrmhd_batch* b) {
  if (!b) return;
  // teardown: nothing to report an error to; release what can be released
  (void)hipStreamSynchronize(b->stream);
  for (int k = 0; k < 2; ++k) {
    if (b->host[k]) (void)hipHostFree(b->host[k]);
    if (b->ev[k]) (void)hipEventDestroy(b->ev[k]);
  }
  if (b->hsmax) (void)hipHostFree(b->hsmax);
  if (b->hclock) (void)hipHostFree(b->hclock);
  if (b->ev_clock) (void)hipEventDestroy(b->ev_clock);
  delete b;
}

const char* rrmhd_strerror(rrmhd_status s) {
  switch (s) {
    case RRMHD_OK: return "ok";
    case RRMHD_E_INVALID: return "invalid argument";
    case RRMHD_E_C2P: return "primitive recovery failed";
    case RRMHD_E_IMPLICIT: return "implicit source solve failed";
    case RRMHD_E_NONFINITE: return "non-finite value";
    case RRMHD_E_DEVICE: return "HIP device error";
    case RRMHD_E_WORKSPACE: return "workspace missing, too small or misaligned";
  }
  return "unknown status";
}

}  // extern "C"
