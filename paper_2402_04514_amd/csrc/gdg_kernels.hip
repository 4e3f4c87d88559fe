// gdg_kernels.hip -- the per-stage sweeps of the graph-based DG scheme on
// gfx950 (FP64, and the mixed-precision variant of sweeps 1 and 2).  One
// thread owns one row i of the stencil; a workgroup (one wavefront) owns
// whole cells (R rows), so the cell-local consistent-mass solve runs in LDS.
//
// Sweeps of one forward-Euler stage Phi(U; tau):
//   k_prim    per node: velocity, pressure, sound speed, p^-alpha, Harten
//             entropy f(s), rescaled entropy s~ (Sec. 2.2, Sec. 5.2, 5.4),
//             with the state, as the node record the sweeps gather; with the
//             limiter, the last limiter pass writes the stage output's
//             records, and k_prim runs only at the start of a host-driven step
//   k_sweep1  d^L_ij, d_i^{d,k} (eq. dij_low_order, dij_low_order_modified),
//             min_i m_i/(2|d_ii|) (eq. MaxCFLdt), the entropy-viscosity ratio
//             N_i (Sec. 5.2) and ring-1 partial bounds over bar states
//             (eq. UsualBarState)
//   k_sweep2  tau, U^L (eq. cijdijschememodified), the relaxed bounds
//             (eq. local_bounds), d^H (eq. HighOrderViscosity, ViscMin), the
//             high-order residual and the cell solve (eq. HighScheme)
//   k_limit   one limiter pass (eq. ConvexScheme, Lemma ConsInvariants) on
//             the antidiffusive fluxes A_ij (eq. HighLowOrderIdentity); run
//             twice (Sec. 6.1), the second pass on the remaining (1 - l) A
// Every grid-wide dependency (tau, neighbours' N_j and bound partials, their
// U^L_j / B_j / dU^H_j, the symmetric l_ij) is a kernel boundary.  The kb_*
// kernels run the same per-block bodies for every request resident in the
// request server, from a work list in device memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gdg_internal.h"

// Occupancy targets (waves per SIMD) chosen by measurement: sweep 2 gains
// from a third wave; sweep 1 keeps its neighbour prefetch in registers at
// two; the limiter loses more to spills than it would gain.
#ifndef GDG_WPE_LIMIT
#define GDG_WPE_LIMIT 1
#endif
#ifndef GDG_WPE_SWEEP
#define GDG_WPE_SWEEP 3
#endif
#ifndef GDG_WPE_SWEEP1
#define GDG_WPE_SWEEP1 2
#endif

namespace gdg {

__device__ __forceinline__ double ipow_d(double x, int n) {
  double r = 1.0, b = x;
  while (n > 0) {
    if (n & 1) r *= b;
    b *= b;
    n >>= 1;
  }
  return r;
}

// Two-rarefaction upper bound of the maximum wave speed of the projected
// Riemann problem (Guermond & Popov 2016), valid for 1 < gamma <= 5/3.
// Left state (rl, ul, pl, al, pal = pl^-alpha), right state likewise; ul, ur
// are the velocities projected on the unit normal.
// ipl, ipr are 1/p of the two states.
__device__ __forceinline__ double lambda_plus(const KArgs &A, double ul, double pl, double al, double pal,
                                              double ipl, double ur, double pr, double ar, double par,
                                              double ipr) {
  const double g = A.gamma;
  double num = al + ar - 0.5 * (g - 1.0) * (ur - ul);
  double pstar = 0.0;
  if (num > 0.0) {
    double x = num / (al * pal + ar * par);
    pstar = A.ipow > 0 ? ipow_d(x, A.ipow) : pow(x, A.inv_alpha);
  }
  double kf = (g + 1.0) / (2.0 * g);
  double l1 = ul - al * sqrt(1.0 + kf * fmax(pstar - pl, 0.0) * ipl);
  double l3 = ur + ar * sqrt(1.0 + kf * fmax(pstar - pr, 0.0) * ipr);
  return fmax(fmax(-l1, l3), 0.0);
}

// f(U) c for the Euler flux of eq. euler_flux, from conserved U and the
// velocity u and pressure p of the node.
// Contraction stays off here: f(U_j) c - f(U_i) c must be exactly zero for
// equal states (x*y - x*y under a fused multiply-add leaves the rounding
// error of x*y), so constant states give R_i = D_i = 0 and no flux.
template <int D, typename T>
__device__ __forceinline__ void flux_dot(const T *U, const T *u, T p, const T *c, T *out) {
#pragma clang fp contract(off)
  T uc = 0;
  for (int e = 0; e < D; ++e) uc += u[e] * c[e];
  out[0] = U[0] * uc;
  for (int e = 0; e < D; ++e) out[1 + e] = U[1 + e] * uc + p * c[e];
  out[D + 1] = (U[D + 1] + p) * uc;
}

template <int D>
__device__ __forceinline__ double eps_of(const double *V) {
  double m2 = 0.0;
  for (int e = 0; e < D; ++e) m2 += V[1 + e] * V[1 + e];
  return V[D + 1] - 0.5 * m2 / V[0];
}

// Accumulator type of the flux and entropy-viscosity sums: FP32 in the mixed
// precision variant, FP64 otherwise.
template <bool MX>
struct AccT { using type = double; };
template <>
struct AccT<true> { using type = float; };

// c_ij of slot s, widened to FP64 (FP32 storage in the mixed variant)
template <int D, bool MX>
__device__ __forceinline__ void load_c(const KArgs &A, int64_t s, double *c) {
  for (int e = 0; e < D; ++e) c[e] = MX ? (double)A.cf[e * A.nslots + s] : A.c[e * A.nslots + s];
}

// ---------------------------------------------------------------------------
// Rescaled entropy tests.  For gamma = 7/5 the comparison
//   eps >= s rho^(7/5)   <=>   (rho eps)^5 >= s^5 rho^12     (eps, s, rho > 0)
// needs multiplies only; the power function is left to the rare cases.
__device__ __forceinline__ double pow5(double x) {
  double x2 = x * x;
  return x2 * x2 * x;
}

// s~^5 = (rho eps)^5 / rho^12 for gamma = 7/5 (monotone in s~), else s~
// itself; reps = rho eps = rho E - |m|^2/2.
__device__ __forceinline__ double stilde_key(const KArgs &A, double reps, double rho) {
  if (A.g75) {
    const double r3 = rho * rho * rho, r6 = r3 * r3;
    return pow5(reps) / (r6 * r6);
  }
  return reps / rho * pow(rho, -A.gamma);
}

// Line search of Sec. 5.4: the largest l in [0, 1] with U + l P in B_i,
// P = sc * Av.  Density part in closed form; rescaled-entropy part on the
// concave psi(l) = eps(U + l P) - s_min rho(U + l P)^gamma by a bracket
// narrowed with a secant step (feasible side) and a tangent step at the
// infeasible end, until the bracket is 1e-14 wide; the feasible end is
// returned.
template <int D>
__device__ double ls_psi(double g, const double *U, const double *P, double smin, double l,
                         double *dpsi) {
  double V[D + 2];
  for (int c = 0; c < D + 2; ++c) V[c] = U[c] + l * P[c];
  double eps = eps_of<D>(V);
  double rg = pow(V[0], g);
  if (dpsi) {
    double u2 = 0.0, dot = 0.0;
    for (int e = 0; e < D; ++e) {
      double u = V[1 + e] / V[0];
      u2 += u * u;
      dot -= u * P[1 + e];
    }
    dot += 0.5 * u2 * P[0] + P[D + 1];
    *dpsi = dot - smin * g * rg / V[0] * P[0];
  }
  return eps - smin * rg;
}

// Common path of the line search, branch free: the density limit
// l_rho and whether the rescaled-entropy bound holds there.  When it holds,
// LS = l_rho; otherwise ls_slow() brackets the root.
template <int D>
__device__ __forceinline__ bool ls_fast(const KArgs &A, const double *U, const double *P, double rmin,
                                        double rmax, double smin, double smin5, double *lhi_out) {
  const double r = U[0], pr = P[0], rp = r + pr;
  // only one of the two limits can be active: rho + P_rho > rho_max needs P_rho > 0
  const double lim = (rp > rmax ? rmax : rmin) - r;
  const double t = lim / pr;
  double lhi = (rp > rmax || rp < rmin) ? t : 1.0;
  lhi = lhi > 0.0 ? lhi : 0.0;  // also maps NaN to 0
  lhi = lhi < 1.0 ? lhi : 1.0;
  *lhi_out = lhi;
  double V[D + 2];
  for (int c = 0; c < D + 2; ++c) V[c] = U[c] + lhi * P[c];
  if (A.g75) {
    double m2 = 0.0;
    for (int e = 0; e < D; ++e) m2 += V[1 + e] * V[1 + e];
    const double re = V[0] * V[D + 1] - 0.5 * m2;  // rho eps
    const double r3 = V[0] * V[0] * V[0], r6 = r3 * r3;
    const double lhs = pow5(re), rhs = smin5 * (r6 * r6);
    // inside the range where the integer powers are exact enough to decide
    const bool decided = isfinite(lhs) && isfinite(rhs) && rhs > 1e-290 && smin5 > 0.0;
    return decided && re > 0.0 && lhs >= rhs;
  }
  return eps_of<D>(V) - smin * pow(V[0], A.gamma) >= 0.0;
}

template <int D>
__device__ __forceinline__ double ls_slow(double g, const double *U, const double *P, double smin, double lhi) {
  double ph = ls_psi<D>(g, U, P, smin, lhi, nullptr);
  if (ph >= 0.0) return lhi;
  double p0 = ls_psi<D>(g, U, P, smin, 0.0, nullptr);
  if (p0 <= 0.0) return 0.0;
  double l = 0.0, rr = lhi, pl = p0, prr = ph;
  for (int it = 0; it < 60; ++it) {
    if (rr - l <= 1e-14) break;
    double x = l + pl * (rr - l) / (pl - prr);
    if (!(x > l && x < rr)) x = 0.5 * (l + rr);
    double px = ls_psi<D>(g, U, P, smin, x, nullptr);
    if (px >= 0.0) { l = x; pl = px; } else { rr = x; prr = px; }
    if (rr - l <= 1e-14) break;
    double dr;
    ls_psi<D>(g, U, P, smin, rr, &dr);
    x = dr < 0.0 ? rr - prr / dr : 0.5 * (l + rr);
    if (!(x > l && x < rr)) x = 0.5 * (l + rr);
    px = ls_psi<D>(g, U, P, smin, x, nullptr);
    if (px >= 0.0) { l = x; pl = px; } else { rr = x; prr = px; }
  }
  return l;
}

// For gamma = 7/5 the bracket is narrowed on
//   phi(l) = (rho eps)^5 - s^5 rho^12,   rho eps = rho E - |m|^2 / 2,
// at V = U + l P, which has the sign of psi wherever rho > 0 (both sides of
// eps >= s rho^(7/5) multiplied by rho and raised to the fifth power), so the
// same feasible interval [0, l*] is found with multiplies instead of the
// power function.  phi is not concave, so the steps are those of the Illinois
// variant of regula falsi (the end kept twice in a row has its value halved),
// with a bisection whenever two steps did not halve the bracket; the bracket
// is kept by sign down to a width of 1e-14 and its feasible end returned.
// Returns false when the powers leave the range where they decide the sign
// reliably; the caller then uses psi.
template <int D>
__device__ __forceinline__ double ls_phi75(const double *U, const double *P, double s5, double l) {
  double V[D + 2];
  for (int c = 0; c < D + 2; ++c) V[c] = U[c] + l * P[c];
  double m2 = 0.0;
  for (int e = 0; e < D; ++e) m2 += V[1 + e] * V[1 + e];
  const double re = V[0] * V[D + 1] - 0.5 * m2;
  const double r3 = V[0] * V[0] * V[0], r6 = r3 * r3;
  return pow5(re) - s5 * (r6 * r6);
}

template <int D>
__device__ __forceinline__ bool ls_slow75(const double *U, const double *P, double s5, double lhi, double *out) {
  double pr = ls_phi75<D>(U, P, s5, lhi);
  double pl = ls_phi75<D>(U, P, s5, 0.0);
  // both ends must be decided: finite, and s^5 rho^12 at both ends well above the underflow range
  const double rl = U[0], rh = U[0] + lhi * P[0];
  const double rm = rl < rh ? rl : rh;
  const double rm3 = rm * rm * rm, rm6 = rm3 * rm3;
  if (!(isfinite(pr) && isfinite(pl)) || !(s5 * rm6 * rm6 > 1e-290)) return false;
  if (pr >= 0.0) { *out = lhi; return true; }
  if (pl <= 0.0) { *out = 0.0; return true; }
  double l = 0.0, r = lhi, w2 = lhi;
  int side = 0;
  for (int it = 0; it < 100; ++it) {
    const double w = r - l;
    if (w <= 1e-14) break;
    double x;
    if ((it & 1) == 0 && it > 0 && w > 0.5 * w2) {
      x = 0.5 * (l + r);  // two steps without halving the bracket
    } else {
      x = (l * pr - r * pl) / (pr - pl);
      if (!(x > l && x < r)) x = 0.5 * (l + r);
    }
    if ((it & 1) == 0) w2 = w;
    const double px = ls_phi75<D>(U, P, s5, x);
    if (px >= 0.0) {
      l = x;
      pl = px;
      if (side == 1) pr *= 0.5;
      side = 1;
    } else {
      r = x;
      pr = px;
      if (side == -1) pl *= 0.5;
      side = -1;
    }
  }
  *out = l;
  return true;
}

// Bracketing part of the line search after ls_fast found the density limit
// lhi infeasible for the entropy bound.
template <int D>
__device__ __forceinline__ double ls_root(const KArgs &A, const double *U, const double *P, double smin, double smin5,
                                          double lhi) {
  double l;
  if (A.g75 && smin5 > 0.0 && ls_slow75<D>(U, P, smin5, lhi, &l)) return l;
  return ls_slow<D>(A.gamma, U, P, smin, lhi);
}

// Line search of Sec. 5.4: the largest l in [0, 1] with U + l P in B, P = sc Av.
template <int D>
__device__ __forceinline__ double line_search(const KArgs &A, const double *U, const double *Av, double sc,
                                              double rmin, double rmax, double smin, double smin5) {
  double P[D + 2], lhi;
  for (int c = 0; c < D + 2; ++c) P[c] = sc * Av[c];
  if (ls_fast<D>(A, U, P, rmin, rmax, smin, smin5, &lhi)) return lhi;
  return ls_root<D>(A, U, P, smin, smin5, lhi);
}

// Workgroups are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2.  Remapping the hardware block id so that every XCD sweeps
// one contiguous range of row blocks keeps a block's face neighbours (the
// blocks one cell row earlier) in the same L2.  A bijection of [0, nblocks).
__device__ __forceinline__ int64_t xcd_position(int64_t hw, int64_t nblocks) {
  constexpr int64_t kX = 8;
  const int64_t q = nblocks / kX, r = nblocks % kX;
  const int64_t x = hw % kX, k = hw / kX;
  return x * q + (x < r ? x : r) + k;
}

// Row block at position L of the sweep order (a bijection of [0, nblocks)):
// the block order itself, or for a tiled 3D mesh (KArgs::tiled) the order
// tile by tile (tiles of t_tx row blocks in x by t_ty cell rows in y, through
// every z-plane), inside a tile z-plane by z-plane, y-row by y-row, x-block
// by x-block.
__device__ __forceinline__ int64_t sweep_block(const KArgs &A, int64_t L) {
  if (!A.tiled) return L;
  const int64_t plane = A.t_tx * A.t_ty;  // blocks of one tile in one z-plane
  const int64_t tile = L / (plane * A.t_nz), rem = L % (plane * A.t_nz);
  const int64_t z = rem / plane, rem2 = rem % plane;
  const int64_t ntx = A.t_nbx / A.t_tx;
  const int64_t y = (tile / ntx) * A.t_ty + rem2 / A.t_tx;
  const int64_t bx = (tile % ntx) * A.t_tx + rem2 % A.t_tx;
  return bx + A.t_nbx * (y + A.t_ny * z);
}

__device__ __forceinline__ int64_t xcd_block(const KArgs &A, int64_t hw) {
  return sweep_block(A, xcd_position(hw, A.nblocks));
}

// ---------------------------------------------------------------------------
// Setup: expand the cell-class tables into the row-blocked ELL stencil.
template <int D, int DEG>
__global__ __launch_bounds__(kBlockThreads) void k_fill(KArgs A) {
  constexpr int NB = DEG + 1;
  constexpr int NLOC = D == 1 ? NB : (D == 2 ? NB * NB : NB * NB * NB);
  constexpr int NFACE = NLOC / NB;
  const int lane = threadIdx.x;
  if (lane >= A.R || A.ustruct) return;
  const int64_t blk = xcd_block(A, blockIdx.x);
  const int64_t i = blk * A.R + lane;
  const RefTables *T = A.ref;
  int t = 0;
  auto put = [&](int32_t col, const double *c, uint8_t meta) {
    int64_t s = (blk * A.W + t) * A.R + lane;
    A.col[s] = col;
    for (int e = 0; e < D; ++e) {
      if (A.mixed) A.cf[e * A.nslots + s] = c ? (float)c[e] : 0.0f;
      else A.c[e * A.nslots + s] = c ? c[e] : 0.0;
    }
    A.meta[s] = meta;
    ++t;
  };
  int graph = 0;
  if (i < A.N) {
    const int64_t K = i / NLOC;
    const int a = (int)(i % NLOC);
    int64_t ki[3] = {0, 0, 0};
    int64_t r = K;
    for (int e = 0; e < D; ++e) { ki[e] = r % A.cells[e]; r /= A.cells[e]; }
    for (int b = 0; b < NLOC; ++b) {
      put((int32_t)(K * NLOC + b), &T->cin[(a * NLOC + b) * kMaxD], (uint8_t)(SK_CELL | (b << 3)));
      ++graph;
    }
    for (int f = 0; f < 2 * D; ++f) {
      if (!T->onface[f * kMaxNloc + a]) continue;
      const int e = f / 2, side = f % 2;
      int64_t kn[3] = {ki[0], ki[1], ki[2]};
      kn[e] += side ? 1 : -1;
      bool bnd = false;
      if (kn[e] < 0 || kn[e] >= A.cells[e]) {
        if (A.bc[f] == 0) kn[e] = (kn[e] + A.cells[e]) % A.cells[e];
        else bnd = true;
      }
      if (bnd) {
        // the part's kind: its own (boundary parts), else the box face's
        int kind = A.bc[f];
        if (A.bcc) {
          int64_t idx = 0, st = 1;
          for (int g = 0; g < D; ++g) {
            if (g == e) continue;
            idx += ki[g] * st;
            st *= A.cells[g];
          }
          kind = A.bcc[A.bcc_off[f] + idx];
        }
        put((int32_t)i, &T->cghost[(f * kMaxNloc + a) * kMaxD], (uint8_t)(SK_GHOST | (bclass(f, kind) << 3)));
        continue;
      }
      int64_t Kn = 0, stride = 1;
      for (int e2 = 0; e2 < D; ++e2) { Kn += kn[e2] * stride; stride *= A.cells[e2]; }
      for (int tt = 0; tt < NFACE; ++tt) {
        int b = T->bface[f * 9 + tt];
        int co = T->colloc[(f * kMaxNloc + a) * 9 + tt];
        put((int32_t)(Kn * NLOC + b), &T->cface[((f * kMaxNloc + a) * 9 + tt) * kMaxD],
            (uint8_t)(co ? SK_FACE_COLLOC : SK_FACE));
        ++graph;
      }
    }
    A.kscale[i] = (double)(graph + 1) / T->mlump[a];  // 1 / (kappa_i m_i), kappa_i = 1/(card I(i) + 1)
  }
  while (t < A.W) put((int32_t)(i < A.N ? i : 0), nullptr, SK_PAD);
}

// First kernel of a step.  Host-driven: the host passes the cap and a fixed
// tau and has cleared the flags' causes.  Device-driven (graphs): the cap is
// t_final - t, and a finished run, a step limit or a flag left by an earlier
// step of the graph halts the step.
__device__ __forceinline__ void begin_step(Ctl *ctl, double dt_cap, double tau_fixed, int device_driven) {
  if (device_driven) {
    if (ctl->cfl_flag || ctl->bad_flag || ctl->halt || !(ctl->t < ctl->t_final) ||
        ctl->steps >= ctl->step_limit) {
      ctl->halt = 1;
      return;
    }
    dt_cap = ctl->t_final - ctl->t;
    tau_fixed = 0.0;
  } else {
    ctl->t_final = dt_cap > 0.0 ? ctl->t + dt_cap : 0.0;
  }
  for (int s = 0; s < kMaxStages; ++s) ctl->taumin_bits[s] = 0x7ff0000000000000ull;  // +inf
  ctl->cfl_flag = 0;
  ctl->bad_flag = 0;
  ctl->halt = 0;
  ctl->viol_stage = -1;
  ctl->dt_cap = dt_cap;
  ctl->tau_fixed = tau_fixed;
}

__global__ void k_begin(Ctl *ctl, double dt_cap, double tau_fixed, int device_driven) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  begin_step(ctl, dt_cap, tau_fixed, device_driven);
}

// Last kernel of a step: advance t (exactly to the cap's end on a capped step).
__device__ __forceinline__ void end_step(Ctl *ctl) {
  if (ctl->halt || ctl->cfl_flag || ctl->bad_flag) return;
  const bool capped = ctl->dt_cap > 0.0 && ctl->tau == ctl->dt_cap;
  ctl->t = capped ? ctl->t + ctl->dt_cap : ctl->t + ctl->tau;
  if (capped && ctl->t_final > 0.0 && ctl->t_final - ctl->t < 1e-14 * ctl->t_final) ctl->t = ctl->t_final;
  ctl->steps += 1;
}

__global__ void k_end(Ctl *ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  end_step(ctl);
}

// Between two device-driven steps of a graph: the end of one and the start of
// the next in one launch.
__global__ void k_end_begin(Ctl *ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  end_step(ctl);
  begin_step(ctl, 0.0, 0.0, 1);
}

// ---------------------------------------------------------------------------
// Node-cache fields of a state V: velocity (D), p, a, p^-alpha, f(s), s~,
// 1/p.  Returns whether V lies in A.
template <int D>
__device__ __forceinline__ bool node_fields(const KArgs &A, const double *V, double *W) {
  // no contraction: every kernel that builds node fields (the node cache, the
  // boundary data) rounds them alike, so equal states give equal fields
#pragma clang fp contract(off)
  const double g = A.gamma;
  double rho = V[0];
  double m2 = 0.0;
  for (int e = 0; e < D; ++e) m2 += V[1 + e] * V[1 + e];
  double eps = V[D + 1] - 0.5 * m2 / rho;
  double p = (g - 1.0) * eps;
  double rg = pow(rho, -g);
  for (int e = 0; e < D; ++e) W[e] = V[1 + e] / rho;
  W[D + 0] = p;
  W[D + 1] = sqrt(g * p / rho);
  W[D + 2] = pow(p, -A.alpha);
  W[D + 3] = exp(log(rg * p) / (g + 1.0));  // Harten entropy f(s) = e^{s/(gamma+1)}
  W[D + 4] = rg * eps;                      // s~ = rho^-gamma eps
  W[D + 5] = 1.0 / p;
  return rho > 0.0 && eps > 0.0;
}

// Node record of the stage input (buffer 0 or 1 by the parity of
// nst * steps + stage: each stage reads one buffer and its last sweep writes
// the other, which the next stage reads).
__device__ __forceinline__ double *node_buffer(const KArgs &A, int stage) {
  const long long k = (long long)A.nst * A.ctl->steps + stage;
  return A.Nd + (size_t)(k & 1) * (size_t)A.N * kNodeStride;
}

// Node record of row i from its state V (and the admissibility flag).
// Record writes of a row block through LDS.  A lane's record would otherwise
// go out as stores 128 (or 64, 32) bytes apart from its neighbour lane's, one
// cache line per lane and instruction; staged in LDS, the block's records
// (consecutive rows, so one contiguous range) leave as whole 16-byte chunks
// of consecutive addresses.  The staging rows are padded by one double so
// that the lanes' LDS writes spread over the banks.
template <int S>
constexpr int kStage = kBlockThreads * (S + 1);
constexpr int kStageDoubles = kStage<kNodeStride>;

template <int S>
__device__ __forceinline__ double *stage_row(double *stage, int lane) {
  return stage + lane * (S + 1);
}

// Stores the staged records of rows row0 .. row0 + nrows - 1 (S doubles each,
// the pad values included) to dst.  Every lane of the wavefront must call it.
template <int S>
__device__ __forceinline__ void stage_flush(double *stage, double *dst, int64_t row0, int nrows) {
  __syncthreads();  // the lanes' LDS writes before the block's reads
  double2 *out = reinterpret_cast<double2 *>(dst + (size_t)row0 * S);
  const int chunks = nrows * S / 2;
  for (int c = threadIdx.x; c < chunks; c += kBlockThreads) {
    const int r = (2 * c) / S, col = (2 * c) % S;
    const double *v = stage + r * (S + 1) + col;
    out[c] = make_double2(v[0], v[1]);
  }
  __syncthreads();  // the staging area may be reused
}

// The node record of state V into a staging row (and the admissibility flag).
template <int D>
__device__ __forceinline__ void stage_node(const KArgs &A, double *row, const double *V) {
  double W[D + 6];
  if (!node_fields<D>(A, V, W)) atomicOr(&A.ctl->bad_flag, 1);
  for (int c = 0; c < D + 2; ++c) row[c] = V[c];
  for (int k = 0; k < D + 6; ++k) row[D + 2 + k] = W[k];
}

// Set-up: the node fields of each face's Dirichlet data, computed by the same
// code as the node cache, so that data equal to a node's state gives that
// node's fields bit for bit.
template <int D>
__global__ void k_bnodes(KArgs A, RefTables *T) {
  const int f = threadIdx.x;
  if (f >= 2 * D || A.vortex_data || A.old_data) return;  // data that vary: evaluated where used
  if (!((A.bcdata >> f) & 1)) return;        // no part of the face takes data
  double V[D + 2], W[D + 6];
  for (int q = 0; q < D + 2; ++q) V[q] = T->bstate[f][q];
  if (!node_fields<D>(A, V, W)) atomicOr(&A.ctl->bad_flag, 1);
  for (int q = 0; q < D + 2; ++q) T->bnode[f][q] = V[q];
  for (int k = 0; k < D + 6; ++k) T->bnode[f][D + 2 + k] = W[k];
}

// Node records of rows row0 .. row0 + nrows - 1 from the SoA state U; every
// lane of the wavefront calls it.
template <int D>
__device__ __forceinline__ void prim_rows(const KArgs &A, const double *__restrict__ U, int64_t row0, int nrows,
                                          double *nd) {
  __shared__ double stage[kStageDoubles];
  const int lane = threadIdx.x;
  if (lane < nrows) {
    const int64_t i = row0 + lane;
    double V[D + 2];
    for (int c = 0; c < D + 2; ++c) V[c] = U[c * A.N + i];
    stage_node<D>(A, stage_row<kNodeStride>(stage, lane), V);
  }
  stage_flush<kNodeStride>(stage, nd, row0, nrows);
}

template <int D>
__global__ __launch_bounds__(kBlockThreads) void k_prim(KArgs A, const double *__restrict__ U, int stage) {
  const int64_t row0 = (int64_t)blockIdx.x * kBlockThreads;
  const int nrows = (int)(A.N - row0 < kBlockThreads ? A.N - row0 : kBlockThreads);
  prim_rows<D>(A, U, row0, nrows, node_buffer(A, stage));
}

// Node records of U^n for step-start boundary data, from the first stage's
// input (U^n itself), in a buffer of their own that the step's later stages
// do not write.
template <int D>
__global__ __launch_bounds__(kBlockThreads) void k_start_records(KArgs A, const double *__restrict__ U) {
  const int64_t row0 = (int64_t)blockIdx.x * kBlockThreads;
  const int nrows = (int)(A.N - row0 < kBlockThreads ? A.N - row0 : kBlockThreads);
  prim_rows<D>(A, U, row0, nrows, A.Nold);
}

template <int D>
struct Node {
  double U[D + 2];
  double u[D];
  double p, a, pal, fs, st, ip;
};

// The whole node record of dof j: D + 4 loads of 16 bytes from one 128-byte line.
template <int D>
__device__ __forceinline__ void load_node(const double *__restrict__ nd, int64_t j, Node<D> &n) {
  using R = Rec<D>;
  const double2 *r = reinterpret_cast<const double2 *>(nd + (size_t)j * kNodeStride);
  double v[2 * (D + 4)];
  for (int k = 0; k < D + 4; ++k) {
    const double2 t = r[k];
    v[2 * k] = t.x;
    v[2 * k + 1] = t.y;
  }
  for (int c = 0; c < D + 2; ++c) n.U[c] = v[R::U + c];
  for (int e = 0; e < D; ++e) n.u[e] = v[R::u + e];
  n.p = v[R::p];
  n.a = v[R::a];
  n.pal = v[R::pal];
  n.fs = v[R::fs];
  n.st = v[R::st];
  n.ip = v[R::ip];
}

// The first n doubles of a record (n even or odd), by 16-byte loads.
template <int NV>
__device__ __forceinline__ void load_rec(const double *__restrict__ rec, double *out) {
  const double2 *r = reinterpret_cast<const double2 *>(rec);
  for (int k = 0; k < NV / 2; ++k) {
    const double2 t = r[k];
    out[2 * k] = t.x;
    out[2 * k + 1] = t.y;
  }
  if (NV % 2) out[NV - 1] = rec[NV - 1];
}

// Time of a stage's boundary data: t + c_k tau, c_k the stage's abscissa
// (SSP-RK3: t, t + tau, t + tau / 2; tau is fixed in stage 1, whose data are
// at t).
__device__ __forceinline__ double stage_time(const KArgs &A, int stage) {
  const double t = A.ctl->t;
  return stage == 0 ? t : t + A.tfrac[stage] * A.ctl->tau;
}

// The isentropic vortex of Sec. 6.2 at dof i and time t (free space): with
// xb = x_i - x0 - t u_inf, rho = (1 - (gamma-1) beta^2 / (8 gamma pi^2)
// e^{1-r^2})^{1/(gamma-1)}, p = rho^gamma and
// u = u_inf + beta / (2 pi) e^{(1-r^2)/2} (-xb_2, xb_1).  2D.
template <int D, int DEG>
__device__ __forceinline__ void vortex_state(const KArgs &A, int64_t i, double t, double *V) {
#pragma clang fp contract(off)
  constexpr int NB = DEG + 1;
  constexpr int NLOC = D == 1 ? NB : (D == 2 ? NB * NB : NB * NB * NB);
  const int64_t K = i / NLOC;
  const int a = (int)(i % NLOC);
  const double x0 = A.lo[0] + ((double)(K % A.cells[0]) + A.ref->xg[a % NB]) * A.hx[0];
  const double x1 = A.lo[1] + ((double)(K / A.cells[0]) + A.ref->xg[a / NB]) * A.hx[1];
  const double beta = A.vx[0], g = A.vx[5];
  const double xb0 = x0 - A.vx[1] - t * A.vx[3], xb1 = x1 - A.vx[2] - t * A.vx[4];
  const double r2 = xb0 * xb0 + xb1 * xb1;
  const double pi = 3.14159265358979323846;
  const double T = 1.0 - (g - 1.0) * beta * beta / (8.0 * g * pi * pi) * exp(1.0 - r2);
  const double rho = pow(T, 1.0 / (g - 1.0)), p = pow(rho, g);
  const double fac = beta / (2.0 * pi) * exp(0.5 * (1.0 - r2));
  const double u0 = A.vx[3] - fac * xb1, u1 = A.vx[4] + fac * xb0;
  V[0] = rho;
  V[1] = rho * u0;
  V[2] = rho * u1;
  V[D + 1] = p / (g - 1.0) + 0.5 * rho * (u0 * u0 + u1 * u1);
}

template <int D>
__device__ __forceinline__ void node_from_state(const KArgs &A, const double *V, Node<D> &n);

// Data U^d of face f at dof i and time t, as a node (state and fields): the
// face's constant data (fields computed at set-up), the vortex, or the
// node's state at the start of the step (its record, kept for the step).
template <int D, int DEG>
__device__ __forceinline__ void data_node(const KArgs &A, int f, int64_t i, double t, Node<D> &d) {
  if (D == 2 && A.vortex_data) {
    double V[D + 2];
    vortex_state<D, DEG>(A, i, t, V);
    node_from_state<D>(A, V, d);
    return;
  }
  // a step-start record has the layout of bnode
  const double *b = A.old_data ? A.Nold + (size_t)i * kNodeStride : A.ref->bnode[f];
  for (int q = 0; q < D + 2; ++q) d.U[q] = b[q];
  for (int e = 0; e < D; ++e) d.u[e] = b[D + 2 + e];
  d.p = b[2 * D + 2];
  d.a = b[2 * D + 3];
  d.pal = b[2 * D + 4];
  d.fs = b[2 * D + 5];
  d.st = b[2 * D + 6];
  d.ip = b[2 * D + 7];
}

template <int D>
__device__ __forceinline__ void node_from_state(const KArgs &A, const double *V, Node<D> &n) {
  double W[D + 6];
  if (!node_fields<D>(A, V, W)) atomicOr(&A.ctl->bad_flag, 1);
  for (int q = 0; q < D + 2; ++q) n.U[q] = V[q];
  for (int e = 0; e < D; ++e) n.u[e] = W[e];
  n.p = W[D];
  n.a = W[D + 1];
  n.pal = W[D + 2];
  n.fs = W[D + 3];
  n.st = W[D + 4];
  n.ip = W[D + 5];
}

// Sub- and supersonic in/outflow in the subsonic range: the state whose
// characteristic variables (eq. characteristics) R1 = v_n - 2a/(gamma-1),
// R2 = p/rho^gamma, R3 = v - v_n n, R4 = v_n + 2a/(gamma-1) are the data's
// for the incoming characteristics and U_i's for the others (R1 always
// incoming, R4 outgoing, R2 and R3 incoming where v_n <= 0); rebuilt from
// v_n = (R1 + R4)/2, a = (gamma-1)(R4 - R1)/4, rho = (a^2/(gamma R2))^{1/(gamma-1)},
// p = R2 rho^gamma.  Returns false if a <= 0.
template <int D>
__device__ __forceinline__ bool characteristic_state(const KArgs &A, const Node<D> &ni, const Node<D> &nd,
                                                     const double *n, double vni, double *V) {
  const double g = A.gamma;
  double vnd = 0.0;
  for (int e = 0; e < D; ++e) vnd += nd.u[e] * n[e];
  const bool in23 = vni <= 0.0;
  const double R1 = vnd - 2.0 * nd.a / (g - 1.0);
  const double R4 = vni + 2.0 * ni.a / (g - 1.0);
  const Node<D> &s = in23 ? nd : ni;
  const double vns = in23 ? vnd : vni;
  const double R2 = s.p / pow(s.U[0], g);
  const double vn = 0.5 * (R1 + R4), a = 0.25 * (g - 1.0) * (R4 - R1);
  if (!(a > 0.0)) return false;
  const double rho = pow(a * a / (g * R2), 1.0 / (g - 1.0)), p = R2 * pow(rho, g);
  double u2 = 0.0;
  V[0] = rho;
  for (int e = 0; e < D; ++e) {
    const double v = (s.u[e] - vns * n[e]) + vn * n[e];
    V[1 + e] = rho * v;
    u2 += v * v;
  }
  V[D + 1] = p / (g - 1.0) + 0.5 * rho * u2;
  return true;
}

// Boundary data of Sec. 4.1 for a boundary part of row i on box face f, with
// outward unit normal n, at time t: outflow keeps U_i; slip reflects the
// normal momentum (eq. slip_boundary; pressure, sound speed and entropy stay
// those of U_i); Dirichlet takes the face's data; supersonic in/outflow
// (eq. supersonic_inoutflow) takes the data where u_i.n < -a_i and U_i where
// u_i.n >= a_i, and flags the subsonic range between (bit 2 of bad_flag: the
// step fails); sub- and supersonic in/outflow builds the subsonic state from
// the characteristic variables (bit 2 if it has no positive sound speed).
// BD = false: the mesh has no face with data (the caller knows), and that
// code is left out.
template <int D, int DEG, bool BD = true>
__device__ __forceinline__ void ghost_node(const KArgs &A, const Node<D> &ni, int cls, const double *n, int64_t i,
                                           double t, Node<D> &gh) {
  // cls: the part's boundary class (its data face and its kind)
  const int f = bclass_face(cls), kind = bclass_kind(cls);
  gh = ni;
  if (kind == GDG_BC_SLIP) {
    double mn = 0.0, un = 0.0;
    for (int e = 0; e < D; ++e) {
      mn += ni.U[1 + e] * n[e];
      un += ni.u[e] * n[e];
    }
    for (int e = 0; e < D; ++e) {
      gh.U[1 + e] = ni.U[1 + e] - 2.0 * mn * n[e];
      gh.u[e] = ni.u[e] - 2.0 * un * n[e];
    }
  }
  if constexpr (BD) {
    if (kind == GDG_BC_DIRICHLET || kind == GDG_BC_SUPERSONIC || kind == GDG_BC_INOUTFLOW) {
      double un = 0.0;
      for (int e = 0; e < D; ++e) un += ni.u[e] * n[e];
      const bool data = kind == GDG_BC_DIRICHLET || un < -ni.a;
      const bool keep = kind != GDG_BC_DIRICHLET && un >= ni.a;
      if (data) {
        data_node<D, DEG>(A, f, i, t, gh);
      } else if (!keep) {
        if (kind == GDG_BC_SUPERSONIC) {
          atomicOr(&A.ctl->bad_flag, 2);
        } else {
          Node<D> nd;
          data_node<D, DEG>(A, f, i, t, nd);
          double V[D + 2];
          if (characteristic_state<D>(A, ni, nd, n, un, V)) node_from_state<D>(A, V, gh);
          else atomicOr(&A.ctl->bad_flag, 2);
        }
      }
    }
  }
}

__device__ __forceinline__ double block_min_atomic(double v, unsigned long long *dst) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) {
    // the minimum only falls, so a value not below what the address holds
    // (even an older copy of it) changes nothing: most wavefronts skip the
    // atomic, which all of them would otherwise queue on one address
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b < *(volatile unsigned long long *)dst) atomicMin(dst, b);
  }
  return v;
}

__device__ __forceinline__ unsigned long long *cnt_slot(const KArgs &A, int kind) {
  return A.cnt + ((size_t)kind * kCntSlots + blockIdx.x % kCntSlots) * kCntStride;
}

// Adds the counts v (0 .. 127) of the wave's active lanes to *dst: the sum is
// assembled bit by bit from ballots, and the first active lane issues one
// atomic (none if the sum is zero).
__device__ __forceinline__ void wave_count_add(unsigned long long *dst, unsigned v) {
  const unsigned long long act = __ballot(1);
  unsigned long long tot = 0;
  for (int b = 0; b < 7; ++b) tot += (unsigned long long)__popcll(__ballot((v >> b) & 1u)) << b;
  if (tot != 0 && (int)__lane_id() == __ffsll((long long)act) - 1) atomicAdd(dst, tot);
}

// ---------------------------------------------------------------------------
template <int D, int DEG, bool MX, bool BD = true>
__device__ __forceinline__ void sweep1_body(const KArgs &A, const double *__restrict__ U, int stage,
                                            int64_t blk) {
  using Acc = typename AccT<MX>::type;
  constexpr int M = D + 2;
  constexpr int NB = DEG + 1;
  constexpr int NLOC = D == 1 ? NB : (D == 2 ? NB * NB : NB * NB * NB);
  if (A.ctl->halt || A.ctl->cfl_flag) return;  // set by an earlier kernel or never
  const int lane = threadIdx.x;
  const int64_t i = blk * A.R + lane;
  const bool active = lane < A.R && i < A.N;
  const double *__restrict__ nd = node_buffer(A, stage);
  double tau_i = INFINITY;
  if (active) {
    const double g = A.gamma;
    const double tstage = stage_time(A, stage);
    Node<D> ni;
    load_node<D>(nd, i, ni);
    // gradient of the shifted Harten entropy at U_i, rho_i f'(s_i) grad s(U_i)
    double grad[M];
    {
      double u2 = 0.0;
      for (int e = 0; e < D; ++e) u2 += ni.u[e] * ni.u[e];
      double gp = (g - 1.0) / ni.p;
      grad[0] = gp * 0.5 * u2 - g / ni.U[0];
      for (int e = 0; e < D; ++e) grad[1 + e] = -gp * ni.u[e];
      grad[M - 1] = gp;
      double sc = ni.U[0] * ni.fs / (g + 1.0);
      for (int c = 0; c < M; ++c) grad[c] *= sc;
    }
    // entropy-residual sums (Sec. 5.2): FP32 with FP32 accumulation in the
    // mixed variant; the flux differences come from the FP64 evaluation that
    // the bar states need
    Acc T = 0, S[M];
    for (int c = 0; c < M; ++c) S[c] = 0;
    double dsum = 0.0;
    double rmin = INFINITY, rmax = -INFINITY, smin = INFINITY;
    // bar state with the smallest rescaled entropy, ranked by stilde_key
    double kbar = INFINITY, ebar = 0.0, rbar = 1.0;
    // software pipeline over the slots: the kind and column two slots ahead,
    // the coefficients and the neighbour's node data one slot ahead, so that
    // the gathers overlap the arithmetic of the current slot (pad and ghost
    // slots name a valid row, so their prefetch is harmless)
    const int64_t s0 = blk * A.W * A.R + lane;
    uint8_t meta_n = A.meta[s0];
    int32_t col_n = A.col[s0];
    double c_n[D];
    load_c<D, MX>(A, s0, c_n);
    Node<D> nj_n;
    load_node<D>(nd, col_n, nj_n);
    uint8_t meta_nn = 0;
    int32_t col_nn = 0;
    if (A.W > 1) {
      meta_nn = A.meta[s0 + A.R];
      col_nn = A.col[s0 + A.R];
    }
    for (int t = 0; t < A.W; ++t) {
      const int64_t s = s0 + (int64_t)t * A.R;
      const uint8_t meta = meta_n;
      const int32_t colv = col_n;
      double c[D];
      for (int e = 0; e < D; ++e) c[e] = c_n[e];
      const Node<D> nj = nj_n;
      if (t + 1 < A.W) {
        meta_n = meta_nn;
        col_n = col_nn;
        load_c<D, MX>(A, s + A.R, c_n);
        load_node<D>(nd, col_n, nj_n);
        if (t + 2 < A.W) {
          meta_nn = A.meta[s + 2 * A.R];
          col_nn = A.col[s + 2 * A.R];
        }
      }
      // One path for every slot kind, so that the loads of the next slot stay
      // in flight across it: pad and diagonal slots have c = 0 (no flux, d = 0)
      // and name row i (harmless in the extrema); a ghost slot's right state
      // is the boundary state of Sec. 4.1.
      const int kind = meta & 7;
      const bool ghost = kind == SK_GHOST;
      const int64_t j = colv;
      double nc2 = 0.0;
      for (int e = 0; e < D; ++e) nc2 += c[e] * c[e];
      const double nc = sqrt(nc2);
      const bool graph = kind != SK_PAD && !ghost && j != i && nc2 > 0.0;
      const bool pair = graph || (ghost && nc2 > 0.0);
      rmin = fmin(rmin, nj.U[0]);
      rmax = fmax(rmax, nj.U[0]);
      smin = fmin(smin, nj.st);
      const double inv = nc2 > 0.0 ? 1.0 / nc : 0.0;
      Node<D> nr = nj;
      if (ghost) {
        double n[D];
        for (int e = 0; e < D; ++e) n[e] = c[e] * inv;
        ghost_node<D, DEG, BD>(A, ni, meta >> 3, n, i, tstage, nr);
      }
      // d^L_ij from the lower index for a graph pair, so d_ij = d_ji bitwise;
      // the inside state on the left for a boundary part
      const bool lo = ghost || i < j;
      const Node<D> &na = lo ? ni : nr;
      const Node<D> &nb = lo ? nr : ni;
      const double inc = lo ? inv : -inv;
      double ua = 0.0, ub = 0.0;
      for (int e = 0; e < D; ++e) {
        double ne = c[e] * inc;
        ua += na.u[e] * ne;
        ub += nb.u[e] * ne;
      }
      const double lam = lambda_plus(A, ua, na.p, na.a, na.pal, na.ip, ub, nb.p, nb.a, nb.pal, nb.ip);
      const double d = pair ? nc * lam : 0.0;
      A.dL[s] = d;
      dsum += d;
      double fj[M], fi[M];
      flux_dot<D>(nr.U, nr.u, nr.p, c, fj);
      flux_dot<D>(ni.U, ni.u, ni.p, c, fi);
      Acc mc = 0;
      for (int e = 0; e < D; ++e) mc += (Acc)nr.U[1 + e] * (Acc)c[e];
      T += mc * (Acc)(nr.fs - ni.fs);
      double bar[M];
      const double h2d = graph ? 0.5 / d : 0.0;
      for (int q = 0; q < M; ++q) {
        double df = fj[q] - fi[q];
        S[q] += (Acc)df;
        bar[q] = 0.5 * (ni.U[q] + nr.U[q]) - df * h2d;
      }
      if (graph) {
        rmin = fmin(rmin, bar[0]);
        rmax = fmax(rmax, bar[0]);
      }
      double m2 = 0.0;
      for (int e = 0; e < D; ++e) m2 += bar[1 + e] * bar[1 + e];
      const double rb = bar[0] * bar[M - 1] - 0.5 * m2;  // rho eps of the bar state
      const double kb = graph ? stilde_key(A, rb, bar[0]) : INFINITY;
      if (kb < kbar) { kbar = kb; ebar = rb; rbar = bar[0]; }
    }
    if (kbar < INFINITY) smin = fmin(smin, ebar / rbar * pow(rbar, -g));
    Acc R = T, Dn = fabs(T);
    for (int q = 0; q < M; ++q) {
      const Acc gq = (Acc)grad[q];
      R -= gq * S[q];
      Dn += fabs(gq) * fabs(S[q]);
    }
    const double Nval = Dn > 0 ? (double)(R / Dn) : 0.0;
    // the flux sum of the row (graph and boundary parts, difference form) is
    // the one the low- and high-order updates of sweep 2 need
    for (int q = 0; q < M; ++q) A.fsum[q * A.N + i] = (double)S[q];
    double2 *qr = reinterpret_cast<double2 *>(A.Qd + (size_t)i * kQStride);
    qr[0] = make_double2(rmin, rmax);
    qr[1] = make_double2(smin, Nval);
    const double mi = A.general ? A.mrow[i] : A.ref->mlump[i % NLOC];
    tau_i = mi / (2.0 * dsum);
  }
  block_min_atomic(tau_i, &A.ctl->taumin_bits[stage]);
}

template <int D, int DEG, bool MX, bool BD>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(GDG_WPE_SWEEP1))) void k_sweep1(
    KArgs A, const double *__restrict__ U, int stage) {
  sweep1_body<D, DEG, MX, BD>(A, U, stage, xcd_block(A, blockIdx.x));
}

// high-order viscosity of eq. HighOrderViscosity / ViscMin for a graph pair;
// hpk = c_k hhat_i^{p_k} of row i (the constant c_k is already in it)
__device__ __forceinline__ double visc_high(const KArgs &A, double d, double Ni, double Nj, int kind,
                                           double hpk) {
  double dev = d * fmin(A.c_ev * fmax(fabs(Ni), fabs(Nj)), 1.0);
  double dmin = kind == SK_FACE_COLLOC ? hpk * d : 0.0;
  return fmax(dmin, dev);
}

// c_k hhat^{p_k} of the pair (i, j) for eq. ViscMin: on general cells a
// collocated pair takes hhat_ij = ((m_i + m_j) / (2 |Omega|))^{1/d}, the mean
// of the two rows' masses (on a uniform mesh both rows have the same m and
// this is hpk_i); odd degrees have p_k = 0 and need no power
__device__ __forceinline__ double pair_hpk(const KArgs &A, double hpk_i, double mi, int64_t j, int kind) {
  if (!A.general || kind != SK_FACE_COLLOC || A.pk == 0.0) return hpk_i;
  return A.c_k * pow(pow(0.5 * (mi + A.mrow[j]) / A.vol, 1.0 / A.dim), A.pk);
}

// ---------------------------------------------------------------------------
// Resolves the step's tau (stage 0 picks it) and this stage's Euler step
// tstep[stage] * tau; returns false (uniformly) if the stage must stop.
__device__ __forceinline__ bool stage_tau(const KArgs &A, int stage, double *tau, double *tau_e) {
  if (A.ctl->halt || A.ctl->cfl_flag) return false;
  const double tm = __longlong_as_double((long long)A.ctl->taumin_bits[stage]);
  if (stage == 0) {
    double t = A.ctl->tau_fixed > 0.0 ? A.ctl->tau_fixed : A.cfl * tm / A.tstep_max;
    if (A.ctl->dt_cap > 0.0 && t > A.ctl->dt_cap) t = A.ctl->dt_cap;
    *tau = t;
    *tau_e = A.tstep[0] * t;
    return true;
  }
  *tau = A.ctl->tau;
  *tau_e = A.tstep[stage] * *tau;
  return !(*tau_e > tm);
}

template <int D, int DEG, bool MX>
__device__ __forceinline__ void sweep2_body(const KArgs &A, const StageBufs &sb, int stage, int64_t blk) {
  constexpr int M = D + 2;
  constexpr int NB = DEG + 1;
  constexpr int NLOC = D == 1 ? NB : (D == 2 ? NB * NB : NB * NB * NB);

  __shared__ int qs[kBlockThreads];
  // The limiter records go out staged in LDS (whole lines of consecutive
  // rows); the residual r^H of the cell solve lives in their dU^H slots until
  // dU^H overwrites it.
  __shared__ double stage_lds[kStage<kLimStride>];
  auto rs = [&](int q, int row) -> double & { return stage_lds[row * (kLimStride + 1) + Rec<D>::dUH + q]; };
  double tau_step, tau;
  if (!stage_tau(A, stage, &tau_step, &tau)) {
    if (stage > 0 && blk == 0 && threadIdx.x == 0 && A.ctl->cfl_flag == 0 && A.ctl->halt == 0) {
      A.ctl->viol_stage = stage;
      atomicOr(&A.ctl->cfl_flag, 1);
    }
    return;
  }
  if (stage == 0 && blk == 0 && threadIdx.x == 0) A.ctl->tau = tau_step;
  using R = Rec<D>;
  const double *__restrict__ nd = node_buffer(A, stage);
  const int lane = threadIdx.x;
  const int64_t i = blk * A.R + lane;
  const bool active = lane < A.R && i < A.N;
  const int64_t N = A.N;
  const double g = A.gamma;
  // this row's limiter record, staged
  double *lr = stage_row<kLimStride>(stage_lds, lane);
  Node<D> ni;
  int a = 0;
  if (active) {
    a = (int)(i % NLOC);
    load_node<D>(nd, i, ni);
    const double Ni = A.Qd[(size_t)i * kQStride + 3];
    const double hpk = A.general ? A.hprow[i] : A.ref->hpk[a];
    const double mi = A.general ? A.mrow[i] : A.ref->mlump[a];
    // accL / accH: the viscous terms sum_j d_ij (U_j - U_i) of the low- and
    // high-order updates (with their boundary parts); the flux sum comes from
    // sweep 1
    double accL[M], accH[M];
    for (int c = 0; c < M; ++c) accL[c] = accH[c] = 0.0;
    double rmin = INFINITY, rmax = -INFINITY, smin = INFINITY;
    // dev = sum of |U_j - U_i| over the neighbours and boundary states: zero
    // exactly when all of them equal U_i bit for bit (the row is quiet); a
    // NaN keeps it nonzero
    double dev = 0.0;
    // the next slot's kind and column are loaded one slot ahead, so that the
    // dependent gather of the neighbour does not wait for them
    const int64_t s0 = blk * A.W * A.R + lane;
    uint8_t meta_n = A.meta[s0];
    int32_t col_n = A.col[s0];
    for (int t = 0; t < A.W; ++t) {
      const int64_t s = s0 + (int64_t)t * A.R;
      const uint8_t meta = meta_n;
      const int32_t colv = col_n;
      if (t + 1 < A.W) {
        meta_n = A.meta[s + A.R];
        col_n = A.col[s + A.R];
      }
      const int kind = meta & 7;
      if (kind == SK_PAD) continue;
      const double d = A.dL[s];
      if (kind == SK_GHOST) {
        double c[D];
        load_c<D, MX>(A, s, c);
        double nc2 = 0.0;
        for (int e = 0; e < D; ++e) nc2 += c[e] * c[e];
        const double nc = sqrt(nc2);
        double n[D];
        const double inc = 1.0 / nc;
        for (int e = 0; e < D; ++e) n[e] = c[e] * inc;
        Node<D> gh;
        ghost_node<D, DEG>(A, ni, meta >> 3, n, i, stage_time(A, stage), gh);
        double fj[M], fi[M];
        flux_dot<D>(gh.U, gh.u, gh.p, c, fj);
        flux_dot<D>(ni.U, ni.u, ni.p, c, fi);
        // boundary analogue of eq. HighOrderViscosity: the ghost is collocated
        const double dH = fmax(hpk * d, d * fmin(A.c_ev * fabs(Ni), 1.0));
        double bar[M];
        for (int q = 0; q < M; ++q) {
          double df = fj[q] - fi[q];
          double du = gh.U[q] - ni.U[q];
          dev += fabs(du);
          accL[q] -= d * du;
          accH[q] -= dH * du;
          bar[q] = 0.5 * (gh.U[q] + ni.U[q]) - df / (2.0 * d);  // eq. BoundaryBarState
        }
        rmin = fmin(rmin, bar[0]);
        rmax = fmax(rmax, bar[0]);
        smin = fmin(smin, pow(bar[0], -g) * eps_of<D>(bar));
        continue;
      }
      const int64_t j = colv;
      double qj[4];
      load_rec<4>(A.Qd + (size_t)j * kQStride, qj);
      rmin = fmin(rmin, qj[0]);
      rmax = fmax(rmax, qj[1]);
      smin = fmin(smin, qj[2]);
      if (j == i) continue;
      const double dH = visc_high(A, d, Ni, qj[3], kind, pair_hpk(A, hpk, mi, j, kind));
      // U_j from the neighbour's node record
      double Uj[M];
      load_rec<M>(nd + (size_t)j * kNodeStride, Uj);
      for (int q = 0; q < M; ++q) {
        const double du = Uj[q] - ni.U[q];
        dev += fabs(du);
        accL[q] -= d * du;
        accH[q] -= dH * du;
      }
    }
    qs[lane] = dev == 0.0 ? 1 : 0;
    for (int q = 0; q < M; ++q) {
      const double f = A.fsum[q * N + i];
      accL[q] += f;
      accH[q] += f;
    }
    // eq. cijdijschememodified in the difference form
    double UL[M];
    for (int q = 0; q < M; ++q) {
      UL[q] = ni.U[q] - tau / mi * accL[q];
      lr[R::UL + q] = UL[q];
    }
    // eq. local_bounds with r^-+ = 1 -+ c_r hhat_i^{p_r}
    const double rel = A.general ? A.relrow[i] : A.ref->relax[a];
    lr[R::B] = (1.0 - rel) * rmin;
    lr[R::B + 1] = (1.0 + rel) * rmax;
    lr[R::B + 2] = (1.0 - rel) * smin;
    lr[R::ks] = A.kscale[i];
    lr[R::N] = Ni;
    for (int q = 0; q < M; ++q) lr[R::LU + q] = ni.U[q];
    for (int q = 0; q < M; ++q) rs(q, lane) = -accH[q];
    if (A.scheme == 0 || (A.scheme == 2 && A.passes == 0)) {
      for (int q = 0; q < M; ++q) {
        sb.out[q * N + i] = sb.ca == 0.0 ? UL[q] : sb.ca * sb.Un[q * N + i] + sb.cb * UL[q];
        if (sb.out2) sb.out2[q * N + i] = sb.cx * sb.X2[q * N + i] + sb.cy * UL[q];
      }
      if (!(UL[0] > 0.0) || !(eps_of<D>(UL) > 0.0)) atomicOr(&A.ctl->bad_flag, 1);
    }
  }
  __syncthreads();
  double du[M];
  for (int q = 0; q < M; ++q) du[q] = 0.0;
  // continuous elements run the low-order scheme only: no cell solve (their
  // rows are nodes, not whole cells)
  if (active && !A.cg) {
  // eq. HighScheme: M_K dU^H_K = tau r^H_K for the cell of row i, from LDS
  const int cellbase = lane - a;
  // A cell whose rows are all quiet has a zero residual and dU^H = 0 in every
  // row, so every antidiffusive flux of its rows (eq. HighLowOrderIdentity)
  // is exactly zero: the limiter's first pass accepts the row as it stands
  // without visiting its pairs.
  {
    int cq = A.no_quiet ? 0 : 1;
    for (int b = 0; b < NLOC; ++b) cq &= qs[cellbase + b];
    A.accepted[i] = (uint8_t)cq;
    wave_count_add(cnt_slot(A, kCntQuiet), (unsigned)cq);
  }
  const double *minv = (A.general ? A.cminv + (i / NLOC) * (NLOC * NLOC) : A.ref->minv) + a * NLOC;
  for (int q = 0; q < M; ++q) {
    double s = 0.0;
    for (int b = 0; b < NLOC; ++b) s += minv[b] * rs(q, cellbase + b);
    du[q] = tau * s;
  }
  if (A.scheme == 1) {
    double V[M];
    for (int q = 0; q < M; ++q) V[q] = ni.U[q] + du[q];
    for (int q = 0; q < M; ++q) {
      sb.out[q * N + i] = sb.ca == 0.0 ? V[q] : sb.ca * sb.Un[q * N + i] + sb.cb * V[q];
      if (sb.out2) sb.out2[q * N + i] = sb.cx * sb.X2[q * N + i] + sb.cy * V[q];
    }
    if (!(V[0] > 0.0) || !(eps_of<D>(V) > 0.0)) atomicOr(&A.ctl->bad_flag, 1);
  }
  }
  // the cell's residuals are read: dU^H may take their place
  __syncthreads();
  if (active)
    for (int q = 0; q < M; ++q) lr[R::dUH + q] = du[q];
  const int64_t row0 = blk * A.R;
  stage_flush<kLimStride>(stage_lds, A.Ld, row0, (int)(N - row0 < A.R ? N - row0 : A.R));
}

template <int D, int DEG, bool MX>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(GDG_WPE_SWEEP))) void k_sweep2(
    KArgs A, StageBufs sb, int stage) {
  sweep2_body<D, DEG, MX>(A, sb, stage, xcd_block(A, blockIdx.x));
}

// ---------------------------------------------------------------------------
// Antidiffusive flux of eq. HighLowOrderIdentity for a graph pair:
//   A_ij = tau (d^H_ij - d^L_ij)(U_j - U_i) - m_ij (dU^H_j - dU^H_i).
// d^L, d^H and m_ij are symmetric, so row j computes exactly -A_ij.
// mblk_a: row a (of row i) of the cell's consistent mass block; hpk: c_k
// hhat^{p_k} of the pair.
template <int D>
__device__ __forceinline__ void pair_flux(const KArgs &A, const double *Uj, const double *dUj, double Nj, uint8_t meta,
                                          const double *mblk_a, const double *Ui, const double *dUi, double Ni,
                                          double hpk, double tau, double d, double *Aij) {
  const int kind = meta & 7;
  const double dH = visc_high(A, d, Ni, Nj, kind, hpk);
  const double mij = kind == SK_CELL ? mblk_a[meta >> 3] : 0.0;
  const double td = tau * (dH - d);
  for (int q = 0; q < D + 2; ++q) Aij[q] = td * (Uj[q] - Ui[q]) - mij * (dUj[q] - dUi[q]);
}

// Boundary part of A_i^d for one ghost slot: tau (d^{d,H} - d^{d,L})(U^d - U_i),
// with U^d built from the node of row i as in the sweeps.
template <int D, int DEG>
__device__ __forceinline__ void ghost_flux(const KArgs &A, const double *__restrict__ nd, int64_t i, int64_t s,
                                           uint8_t meta, const double *Ui, double Ni, double hpk, double tau,
                                           double d, double t, double *Ab) {
  double c[D], nc2 = 0.0;
  for (int e = 0; e < D; ++e) {
    c[e] = A.mixed ? (double)A.cf[e * A.nslots + s] : A.c[e * A.nslots + s];
    nc2 += c[e] * c[e];
  }
  const double inc = 1.0 / sqrt(nc2);
  double n[D];
  for (int e = 0; e < D; ++e) n[e] = c[e] * inc;
  const int cls = meta >> 3;
  const int kind = bclass_kind(cls);
  double Ug[D + 2];
  if (kind == GDG_BC_DIRICHLET || kind == GDG_BC_SUPERSONIC || kind == GDG_BC_INOUTFLOW) {
    // the data kinds decide from the node of row i, as the sweeps do
    Node<D> ni, gh;
    load_node<D>(nd, i, ni);
    ghost_node<D, DEG>(A, ni, cls, n, i, t, gh);
    for (int q = 0; q < D + 2; ++q) Ug[q] = gh.U[q];
  } else {
    // outflow and slip need U_i alone (the same arithmetic as ghost_node)
    for (int q = 0; q < D + 2; ++q) Ug[q] = Ui[q];
    if (kind == GDG_BC_SLIP) {
      double mn = 0.0;
      for (int e = 0; e < D; ++e) mn += Ui[1 + e] * n[e];
      for (int e = 0; e < D; ++e) Ug[1 + e] = Ui[1 + e] - 2.0 * mn * n[e];
    }
  }
  const double dH = fmax(hpk * d, d * fmin(A.c_ev * fabs(Ni), 1.0));
  for (int q = 0; q < D + 2; ++q) Ab[q] += tau * (dH - d) * (Ug[q] - Ui[q]);
}

// One limiter pass (eq. ConvexScheme, Lemma ConsInvariants).  Row i runs both
// line searches of each pair, l^i_ij = LS(base_i, A_ij/(kappa_i m_i), B_i) and
// l^j_ji = LS(base_j, -A_ij/(kappa_j m_j), B_j), so l_ij = min(l^i_ij, l^j_ji)
// is symmetric bit for bit without a grid-wide exchange; l_i^d comes from the
// boundary part alone.  pass 0: base U^L, fluxes A, writes l per slot and
// U^(1).  pass 1: base U^(1), fluxes (1 - l^(1)) A.  The final pass writes the
// SSP combination.
template <int D, int DEG>
__device__ __forceinline__ void limit_body(const KArgs &A, const StageBufs &sb, int stage, int pass, int final_pass,
                                           int64_t blk) {
  constexpr int M = D + 2;
  constexpr int NB = DEG + 1;
  constexpr int NLOC = D == 1 ? NB : (D == 2 ? NB * NB : NB * NB * NB);
  constexpr int NL = Rec<D>::nlim;  // limiter record: dU^H, U^L, bounds, 1/(kappa m), N, U
  using R = Rec<D>;
  if (A.ctl->halt || A.ctl->cfl_flag) return;  // the same for every block
  __shared__ double stage_lds[kStageDoubles];  // the block's output records
  const int lane = threadIdx.x;
  const int64_t i = blk * A.R + lane;
  const int64_t N = A.N;
  const int64_t row0 = blk * A.R;
  const int nrows = (int)(N - row0 < A.R ? N - row0 : A.R);
  const double *__restrict__ nd = node_buffer(A, stage);
  // every lane reaches the record writes at the end (they are staged in LDS
  // and stored by the whole wavefront); rows outside the block compute nothing
  double V[M];
  if (lane < nrows) {
  const double tau = A.tstep[stage] * A.ctl->tau;
  const int a = (int)(i % NLOC);
  if (pass == 1 && final_pass && A.accepted[i]) {
    // pass 1 accepted every pair and the boundary part of this row whole:
    // nothing is left to limit (every remaining flux is 0 A), and the result
    // is U^(1) itself
    load_rec<M>(A.U1d + (size_t)i * kU1Stride, V);
  } else {
  const double mi = A.general ? A.mrow[i] : A.ref->mlump[a];
  const double hpk = A.general ? A.hprow[i] : A.ref->hpk[a];
  const double *mblk_a = (A.general ? A.cmblk + (i / NLOC) * (NLOC * NLOC) : A.ref->mblk) + a * NLOC;
  double Ui[M], Li[M], dUi[M], lri[NL];
  load_rec<NL>(A.Ld + (size_t)i * kLimStride, lri);
  for (int q = 0; q < M; ++q) {
    Ui[q] = lri[R::LU + q];
    dUi[q] = lri[R::dUH + q];
  }
  if (pass == 0) {
    for (int q = 0; q < M; ++q) Li[q] = lri[R::UL + q];
  } else {
    load_rec<M>(A.U1d + (size_t)i * kU1Stride, Li);
  }
  const double rmin = lri[R::B], rmax = lri[R::B + 1], smin = lri[R::B + 2];
  const double sci = lri[R::ks];  // 1 / (kappa_i m_i)
  const double Ni = lri[R::N];
  const double smin5 = A.g75 ? pow5(smin) : 0.0;
  double acc[M], Ab[M];
  for (int q = 0; q < M; ++q) acc[q] = Ab[q] = 0.0;
  int64_t gslot = -1;
  bool allone = true;  // every l of the row is 1
  unsigned ncut = 0;   // pairs of the row with l < 1
  // pass 0 of a row that sweep 2 found quiet (all its fluxes are exactly
  // zero): no pair to visit; its l are never read, since pass 1 returns U^(1)
  // for an accepted row
  const bool quiet = pass == 0 && A.accepted[i];
  const int64_t s0 = blk * A.W * A.R + lane;
  uint8_t meta_n = A.meta[s0];
  int32_t col_n = A.col[s0];
  for (int t = 0; t < (quiet ? 0 : A.W); ++t) {
    const int64_t s = s0 + (int64_t)t * A.R;
    const uint8_t meta = meta_n;
    const int32_t colv = col_n;
    if (t + 1 < A.W) {
      meta_n = A.meta[s + A.R];
      col_n = A.col[s + A.R];
    }
    const int kind = meta & 7;
    if (kind == SK_PAD) continue;
    const double d = A.dL[s];
    if (kind == SK_GHOST) {
      ghost_flux<D, DEG>(A, nd, i, s, meta, Ui, Ni, hpk, tau, d, stage_time(A, stage), Ab);
      if (gslot < 0) gslot = s;
      continue;
    }
    const int64_t j = colv;
    if (j == i) continue;  // A_ii = 0
    // A pair whose flux is exactly zero adds l * 0 whatever l is: pass 1
    // records l = 1 for it and skips its searches, pass 2 skips every pair
    // that pass 1 accepted whole (nothing of it remains).
    double rest = 1.0;
    if (pass == 1) {
      rest = 1.0 - A.l1[s];
      if (rest == 0.0) continue;
    }
    // the neighbour's limiter record, its state included
    double lrj[NL];
    load_rec<NL>(A.Ld + (size_t)j * kLimStride, lrj);
    double Aij[M];
    pair_flux<D>(A, lrj + R::LU, lrj + R::dUH, lrj[R::N], meta, mblk_a, Ui, dUi, Ni,
                 pair_hpk(A, hpk, mi, j, meta & 7), tau, d, Aij);
    bool zero = true;
    for (int q = 0; q < M; ++q) zero = zero && Aij[q] == 0.0;
    if (zero) {
      if (pass == 0) A.l1[s] = 1.0;
      continue;
    }
    if (pass == 1)
      for (int q = 0; q < M; ++q) Aij[q] = rest * Aij[q];
    double Lj[M], Pi[M], Pj[M];
    const double scj = lrj[R::ks];
    if (pass == 0) {
      for (int q = 0; q < M; ++q) Lj[q] = lrj[R::UL + q];
    } else {
      load_rec<M>(A.U1d + (size_t)j * kU1Stride, Lj);
    }
    for (int q = 0; q < M; ++q) {
      Pi[q] = sci * Aij[q];
      Pj[q] = -(scj * Aij[q]);
    }
    const double rminj = lrj[R::B], rmaxj = lrj[R::B + 1], sj = lrj[R::B + 2];
    double li, lj;
    const bool oki = ls_fast<D>(A, Li, Pi, rmin, rmax, smin, smin5, &li);
    const bool okj = ls_fast<D>(A, Lj, Pj, rminj, rmaxj, sj, A.g75 ? pow5(sj) : 0.0, &lj);
    if (!oki) li = ls_root<D>(A, Li, Pi, smin, smin5, li);
    if (!okj) lj = ls_root<D>(A, Lj, Pj, sj, A.g75 ? pow5(sj) : 0.0, lj);
    const double l = fmin(li, lj);
    for (int q = 0; q < M; ++q) acc[q] += l * Aij[q];
    if (pass == 0) A.l1[s] = l;
    allone = allone && l == 1.0;
    ncut += l < 1.0 ? 1u : 0u;
  }
  bool bzero = true;
  for (int q = 0; q < M; ++q) bzero = bzero && Ab[q] == 0.0;
  if (gslot >= 0 && bzero && pass == 0) A.l1[gslot] = 1.0;
  if (gslot >= 0 && !bzero) {
    if (pass == 1) {
      const double rest = 1.0 - A.l1[gslot];
      for (int q = 0; q < M; ++q) Ab[q] = rest * Ab[q];
    }
    const double lb = line_search<D>(A, Li, Ab, sci, rmin, rmax, smin, smin5);
    for (int q = 0; q < M; ++q) acc[q] += lb * Ab[q];
    if (pass == 0) A.l1[gslot] = lb;
    allone = allone && lb == 1.0;
  }
  for (int q = 0; q < M; ++q) V[q] = Li[q] + acc[q] / mi;
  if (pass == 0) {
    double *u1 = stage_row<kU1Stride>(stage_lds, lane);
    for (int q = 0; q < M; ++q) u1[q] = V[q];
    A.accepted[i] = allone ? 1 : 0;
    wave_count_add(cnt_slot(A, kCntLimited), ncut);
  }
  // Lemma ConsInvariants: the pass's output lies in B_i.  Counted with the
  // tolerances of rounding (1e-12 relative on rho, 1e-11 on s~), so that a
  // nonzero count means a defect, not the last bits of the line search.  Rows
  // that the last pass returns as U^(1) were counted in pass 0.
  {
    bool in = V[0] >= rmin * (1.0 - 1e-12) && V[0] <= rmax * (1.0 + 1e-12);
    double m2 = 0.0;
    for (int e = 0; e < D; ++e) m2 += V[1 + e] * V[1 + e];
    const double re = V[0] * V[M - 1] - 0.5 * m2;  // rho eps
    if (A.g75) {
      const double r3 = V[0] * V[0] * V[0], r6 = r3 * r3;
      in = in && re > 0.0 && pow5(re) >= smin5 * (1.0 - 5e-11) * (r6 * r6);
    } else {
      in = in && re > 0.0 && re / V[0] * pow(V[0], -A.gamma) >= smin * (1.0 - 1e-11);
    }
    wave_count_add(cnt_slot(A, kCntViolations), in ? 0u : 1u);
  }
  }  // rows through the pair loop
  }  // rows of the block
  if (pass == 0) stage_flush<kU1Stride>(stage_lds, A.U1d, row0, nrows);
  if (final_pass) {
    // the stage output, and its node record for the next stage (the other
    // buffer: this pass still reads the stage input's records)
    if (lane < nrows) {
      double O[M];
      for (int q = 0; q < M; ++q) {
        O[q] = sb.ca == 0.0 ? V[q] : sb.ca * sb.Un[q * N + i] + sb.cb * V[q];
        sb.out[q * N + i] = O[q];
        if (sb.out2) sb.out2[q * N + i] = sb.cx * sb.X2[q * N + i] + sb.cy * V[q];
      }
      if (!(V[0] > 0.0) || !(eps_of<D>(V) > 0.0)) atomicOr(&A.ctl->bad_flag, 1);
      stage_node<D>(A, stage_row<kNodeStride>(stage_lds, lane), O);
    }
    stage_flush<kNodeStride>(stage_lds, node_buffer(A, stage + 1), row0, nrows);
  }
}

template <int D, int DEG>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(GDG_WPE_LIMIT))) void k_limit(
    KArgs A, StageBufs sb, int stage, int pass, int final_pass) {
  limit_body<D, DEG>(A, sb, stage, pass, final_pass, xcd_block(A, blockIdx.x));
}

// ---------------------------------------------------------------------------
// Batched steps of the request server.  One persistent grid walks the row
// blocks of all resident requests listed in device memory; each XCD takes one
// contiguous range of the concatenated blocks (as xcd_position does for one
// mesh).  Every row block runs the same body as the single-mesh kernels, with
// that request's arguments, so a request's arithmetic does not depend on what
// else is resident.
__device__ __forceinline__ int find_req(const BatchList *L, int64_t tile) {
  int lo = 0, hi = L->nreq - 1;  // the entry with tile_begin[r] <= tile < tile_begin[r + 1]
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (L->tile_begin[mid] <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename F>
__device__ __forceinline__ void for_tiles(const BatchList *L, F &&f) {
  constexpr int64_t kX = 8;
  const int64_t nt = L->ntiles;
  const int64_t per = gridDim.x / kX;
  const int64_t x = blockIdx.x % kX, k = blockIdx.x / kX;
  const int64_t lo = nt * x / kX, hi = nt * (x + 1) / kX;
  for (int64_t t = lo + k; t < hi; t += per) {
    const int r = find_req(L, t);
    f(L->e[r], sweep_block(L->e[r].A, t - L->tile_begin[r]));
  }
}

template <int D>
__global__ __launch_bounds__(kBlockThreads) void kb_prim(const BatchList *L, int stage) {
  for_tiles(L, [&](const BatchEntry &E, int64_t blk) {
    if (E.A.ctl->halt || E.A.ctl->cfl_flag) return;
    if (E.A.scheme == 2 && E.A.passes > 0) return;  // cache written by the last limiter pass
    const int64_t row0 = blk * E.A.R;
    const int nrows = (int)(E.A.N - row0 < E.A.R ? E.A.N - row0 : E.A.R);
    prim_rows<D>(E.A, E.sb[stage].in, row0, nrows, node_buffer(E.A, stage));
  });
}

template <int D, int DEG, bool MX>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(GDG_WPE_SWEEP1))) void kb_sweep1(
    const BatchList *L, int stage) {
  for_tiles(L, [&](const BatchEntry &E, int64_t blk) { sweep1_body<D, DEG, MX>(E.A, E.sb[stage].in, stage, blk); });
}

template <int D, int DEG, bool MX>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(GDG_WPE_SWEEP))) void kb_sweep2(
    const BatchList *L, int stage) {
  for_tiles(L, [&](const BatchEntry &E, int64_t blk) {
    __syncthreads();  // the previous block's cell solve has read its LDS rows
    sweep2_body<D, DEG, MX>(E.A, E.sb[stage], stage, blk);
  });
}

template <int D, int DEG>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(GDG_WPE_LIMIT))) void kb_limit(
    const BatchList *L, int stage, int pass) {
  for_tiles(L, [&](const BatchEntry &E, int64_t blk) {
    if (E.A.scheme != 2 || pass >= E.A.passes) return;
    limit_body<D, DEG>(E.A, E.sb[stage], stage, pass, pass + 1 == E.A.passes ? 1 : 0, blk);
  });
}

__global__ void kb_begin(const BatchList *L) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < L->nreq) begin_step(L->e[r].A.ctl, 0.0, 0.0, 1);
}

__global__ void kb_end(const BatchList *L) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < L->nreq) end_step(L->e[r].A.ctl);
}

__global__ void kb_end_begin(const BatchList *L) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < L->nreq) {
    end_step(L->e[r].A.ctl);
    begin_step(L->e[r].A.ctl, 0.0, 0.0, 1);
  }
}

__global__ void kb_status(const BatchList *L, Ctl *status) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < L->nreq) status[r] = *L->e[r].A.ctl;
}

// ---------------------------------------------------------------------------
// Statistics of a state: min rho, min eps = min (E - |m|^2 / (2 rho)), and the
// conserved totals sum_i m_i U_i (Sec. 3, the quantities the scheme keeps),
// as kRedBlocks per-block partials (grid-stride rows, a fixed tree in LDS)
// combined by one block in a fixed order: the same state gives the same bits.
template <int D>
__global__ __launch_bounds__(kRedThreads) void k_state_stats1(KArgs A, const double *__restrict__ U) {
  constexpr int M = D + 2, F = 2 + M;
  __shared__ double sh[F][kRedThreads];
  double v[F];
  v[0] = INFINITY;
  v[1] = INFINITY;
  for (int c = 0; c < M; ++c) v[2 + c] = 0.0;
  const int64_t N = A.N;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < N; i += (int64_t)kRedBlocks * kRedThreads) {
    double V[M];
    for (int c = 0; c < M; ++c) V[c] = U[c * N + i];
    v[0] = fmin(v[0], V[0]);
    v[1] = fmin(v[1], eps_of<D>(V));
    const double mi = A.general ? A.mrow[i] : A.ref->mlump[i % A.nloc];
    for (int c = 0; c < M; ++c) v[2 + c] += mi * V[c];
  }
  for (int f = 0; f < F; ++f) sh[f][threadIdx.x] = v[f];
  __syncthreads();
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
      sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
      for (int f = 2; f < F; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int f = 0; f < F; ++f) A.red[blockIdx.x * kRedFields + f] = sh[f][0];
}

template <int D>
__global__ __launch_bounds__(kRedBlocks) void k_state_stats2(KArgs A) {
  constexpr int M = D + 2, F = 2 + M;
  __shared__ double sh[F][kRedBlocks];
  for (int f = 0; f < F; ++f) sh[f][threadIdx.x] = A.red[threadIdx.x * kRedFields + f];
  __syncthreads();
  for (int w = kRedBlocks / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] = fmin(sh[0][threadIdx.x], sh[0][threadIdx.x + w]);
      sh[1][threadIdx.x] = fmin(sh[1][threadIdx.x], sh[1][threadIdx.x + w]);
      for (int f = 2; f < F; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int f = 0; f < F; ++f) A.red[kRedBlocks * kRedFields + f] = sh[f][0];
  // the spread counters' totals into the control block
  __shared__ unsigned long long cs[kCntKinds][kCntSlots];
  if ((int)threadIdx.x < kCntSlots)
    for (int c = 0; c < kCntKinds; ++c) cs[c][threadIdx.x] = A.cnt[((size_t)c * kCntSlots + threadIdx.x) * kCntStride];
  __syncthreads();
  for (int w = kCntSlots / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < kCntKinds; ++c) cs[c][threadIdx.x] += cs[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    A.ctl->bound_violations = cs[kCntViolations][0];
    A.ctl->limited_pairs = cs[kCntLimited][0];
    A.ctl->quiet_rows = cs[kCntQuiet][0];
  }
}

__global__ void k_zero_counts(unsigned long long *cnt, int n) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) cnt[k] = 0;
}

// ---------------------------------------------------------------------------
// host launchers
static inline hipStream_t S(void *s) { return (hipStream_t)s; }

static inline void prof_mark(Prof *p, int kid, int end, void *stream) {
  if (!p || p->n >= p->cap) return;
  (void)hipEventRecord((hipEvent_t)p->ev[2 * p->n + end], S(stream));
  if (end) {
    p->kid[p->n] = kid;
    ++p->n;
  }
}

// Errors left in the thread's HIP error state by other code (for instance a
// "not ready" stream query) must not be mistaken for a failed launch.
static inline void clear_stale() { (void)hipGetLastError(); }

template <int D, int DEG, bool MX>
static int stage_impl(const KArgs &A, const StageBufs &b, int stage, void *stream, Prof *prof, int need_prim) {
  clear_stale();
  const dim3 grid((unsigned)A.nblocks), blk(kBlockThreads);
  const unsigned gp = (unsigned)((A.N + kBlockThreads - 1) / kBlockThreads);
  // with the limiter's last pass the node cache of a stage's output is written
  // there; otherwise it is computed at the start of the next stage
  if (need_prim || !(A.scheme == 2 && A.passes > 0)) {
    prof_mark(prof, KID_PRIM, 0, stream);
    hipLaunchKernelGGL(k_prim<D>, dim3(gp), blk, 0, S(stream), A, b.in, stage);
    prof_mark(prof, KID_PRIM, 1, stream);
  }
  if (A.old_data && stage == 0) hipLaunchKernelGGL(k_start_records<D>, dim3(gp), blk, 0, S(stream), A, b.in);
  // sweep 1 without the boundary-data code where no face has data: its
  // registers set the occupancy of the hottest kernel
  const bool bd = A.bcdata != 0;
  prof_mark(prof, KID_SWEEP1, 0, stream);
  if (bd)
    hipLaunchKernelGGL((k_sweep1<D, DEG, MX, true>), grid, blk, 0, S(stream), A, b.in, stage);
  else
    hipLaunchKernelGGL((k_sweep1<D, DEG, MX, false>), grid, blk, 0, S(stream), A, b.in, stage);
  prof_mark(prof, KID_SWEEP1, 1, stream);
  prof_mark(prof, KID_SWEEP2, 0, stream);
  hipLaunchKernelGGL((k_sweep2<D, DEG, MX>), grid, blk, 0, S(stream), A, b, stage);
  prof_mark(prof, KID_SWEEP2, 1, stream);
  for (int pass = 0; pass < (A.scheme == 2 ? A.passes : 0); ++pass) {
    prof_mark(prof, KID_LIMIT1 + pass, 0, stream);
    hipLaunchKernelGGL((k_limit<D, DEG>), grid, blk, 0, S(stream), A, b, stage, pass, pass + 1 == A.passes ? 1 : 0);
    prof_mark(prof, KID_LIMIT1 + pass, 1, stream);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int D, int DEG>
static int fill_impl(const KArgs &A, void *stream) {
  clear_stale();
  hipLaunchKernelGGL((k_fill<D, DEG>), dim3((unsigned)A.nblocks), dim3(kBlockThreads), 0, S(stream), A);
  hipLaunchKernelGGL(k_bnodes<D>, dim3(1), dim3(kBlockThreads), 0, S(stream), A, const_cast<RefTables *>(A.ref));
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

#define GDG_DISPATCH(FN, ...)                                   \
  switch (A.dim * 10 + A.deg) {                                 \
    case 11: return FN<1, 1>(__VA_ARGS__);                      \
    case 12: return FN<1, 2>(__VA_ARGS__);                      \
    case 13: return FN<1, 3>(__VA_ARGS__);                      \
    case 21: return FN<2, 1>(__VA_ARGS__);                      \
    case 22: return FN<2, 2>(__VA_ARGS__);                      \
    case 23: return FN<2, 3>(__VA_ARGS__);                      \
    case 31: return FN<3, 1>(__VA_ARGS__);                      \
    case 32: return FN<3, 2>(__VA_ARGS__);                      \
    default: return -2;                                         \
  }

int launch_stage(const KArgs &A, const StageBufs &b, int stage, void *stream, Prof *prof, int need_prim) {
  if (A.mixed) {
#define GDG_STAGE_MX(D_, K_) stage_impl<D_, K_, true>
    switch (A.dim * 10 + A.deg) {
      case 11: return GDG_STAGE_MX(1, 1)(A, b, stage, stream, prof, need_prim);
      case 12: return GDG_STAGE_MX(1, 2)(A, b, stage, stream, prof, need_prim);
      case 13: return GDG_STAGE_MX(1, 3)(A, b, stage, stream, prof, need_prim);
      case 21: return GDG_STAGE_MX(2, 1)(A, b, stage, stream, prof, need_prim);
      case 22: return GDG_STAGE_MX(2, 2)(A, b, stage, stream, prof, need_prim);
      case 23: return GDG_STAGE_MX(2, 3)(A, b, stage, stream, prof, need_prim);
      case 31: return GDG_STAGE_MX(3, 1)(A, b, stage, stream, prof, need_prim);
      case 32: return GDG_STAGE_MX(3, 2)(A, b, stage, stream, prof, need_prim);
      default: return -2;
    }
#undef GDG_STAGE_MX
  }
#define GDG_STAGE_64(D_, K_) stage_impl<D_, K_, false>
  switch (A.dim * 10 + A.deg) {
    case 11: return GDG_STAGE_64(1, 1)(A, b, stage, stream, prof, need_prim);
    case 12: return GDG_STAGE_64(1, 2)(A, b, stage, stream, prof, need_prim);
    case 13: return GDG_STAGE_64(1, 3)(A, b, stage, stream, prof, need_prim);
    case 21: return GDG_STAGE_64(2, 1)(A, b, stage, stream, prof, need_prim);
    case 22: return GDG_STAGE_64(2, 2)(A, b, stage, stream, prof, need_prim);
    case 23: return GDG_STAGE_64(2, 3)(A, b, stage, stream, prof, need_prim);
    case 31: return GDG_STAGE_64(3, 1)(A, b, stage, stream, prof, need_prim);
    case 32: return GDG_STAGE_64(3, 2)(A, b, stage, stream, prof, need_prim);
    default: return -2;
  }
#undef GDG_STAGE_64
}

int launch_fill(const KArgs &A, void *stream) { GDG_DISPATCH(fill_impl, A, stream) }

template <int D, int DEG, bool MX>
static int batch_impl(const BatchList *L, Ctl *status, int ksteps, int grid, void *stream) {
  clear_stale();
  const dim3 g((unsigned)grid), b(kBlockThreads), gr((kMaxBatch + 63) / 64), br(64);
  hipLaunchKernelGGL(kb_begin, gr, br, 0, S(stream), L);
  for (int k = 0; k < ksteps; ++k) {
    for (int stage = 0; stage < 3; ++stage) {
      hipLaunchKernelGGL(kb_prim<D>, g, b, 0, S(stream), L, stage);
      hipLaunchKernelGGL((kb_sweep1<D, DEG, MX>), g, b, 0, S(stream), L, stage);
      hipLaunchKernelGGL((kb_sweep2<D, DEG, MX>), g, b, 0, S(stream), L, stage);
      for (int pass = 0; pass < 2; ++pass) hipLaunchKernelGGL((kb_limit<D, DEG>), g, b, 0, S(stream), L, stage, pass);
    }
    if (k + 1 < ksteps)
      hipLaunchKernelGGL(kb_end_begin, gr, br, 0, S(stream), L);
    else
      hipLaunchKernelGGL(kb_end, gr, br, 0, S(stream), L);
  }
  hipLaunchKernelGGL(kb_status, gr, br, 0, S(stream), L, status);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_batch_steps(int dim, int deg, int mixed, const BatchList *L, Ctl *status, int ksteps, int grid,
                       void *stream) {
  if (grid <= 0 || grid % 8 != 0) return -2;
  switch (dim * 100 + deg * 10 + (mixed ? 1 : 0)) {
    case 110: return batch_impl<1, 1, false>(L, status, ksteps, grid, stream);
    case 111: return batch_impl<1, 1, true>(L, status, ksteps, grid, stream);
    case 120: return batch_impl<1, 2, false>(L, status, ksteps, grid, stream);
    case 121: return batch_impl<1, 2, true>(L, status, ksteps, grid, stream);
    case 130: return batch_impl<1, 3, false>(L, status, ksteps, grid, stream);
    case 131: return batch_impl<1, 3, true>(L, status, ksteps, grid, stream);
    case 210: return batch_impl<2, 1, false>(L, status, ksteps, grid, stream);
    case 211: return batch_impl<2, 1, true>(L, status, ksteps, grid, stream);
    case 220: return batch_impl<2, 2, false>(L, status, ksteps, grid, stream);
    case 221: return batch_impl<2, 2, true>(L, status, ksteps, grid, stream);
    case 230: return batch_impl<2, 3, false>(L, status, ksteps, grid, stream);
    case 231: return batch_impl<2, 3, true>(L, status, ksteps, grid, stream);
    case 310: return batch_impl<3, 1, false>(L, status, ksteps, grid, stream);
    case 311: return batch_impl<3, 1, true>(L, status, ksteps, grid, stream);
    case 320: return batch_impl<3, 2, false>(L, status, ksteps, grid, stream);
    case 321: return batch_impl<3, 2, true>(L, status, ksteps, grid, stream);
    default: return -2;
  }
}

int launch_begin(const KArgs &A, double dt_cap, double tau_fixed, int device_driven, void *stream) {
  clear_stale();
  hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, S(stream), A.ctl, dt_cap, tau_fixed, device_driven);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Start of a device-driven run: end time, step limit, cleared flags.
__global__ void k_set_run(Ctl *ctl, double t_final, long long step_limit) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  ctl->t_final = t_final;
  ctl->step_limit = step_limit;
  ctl->halt = 0;
  ctl->cfl_flag = 0;
  ctl->bad_flag = 0;
}

int launch_set_run(const KArgs &A, double t_final, long long step_limit, void *stream) {
  clear_stale();
  hipLaunchKernelGGL(k_set_run, dim3(1), dim3(64), 0, S(stream), A.ctl, t_final, step_limit);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_end(const KArgs &A, void *stream) {
  clear_stale();
  hipLaunchKernelGGL(k_end, dim3(1), dim3(64), 0, S(stream), A.ctl);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_end_begin(const KArgs &A, void *stream) {
  clear_stale();
  hipLaunchKernelGGL(k_end_begin, dim3(1), dim3(64), 0, S(stream), A.ctl);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int D>
static int stats_impl(const KArgs &A, const double *U, void *stream) {
  hipLaunchKernelGGL(k_state_stats1<D>, dim3(kRedBlocks), dim3(kRedThreads), 0, S(stream), A, U);
  hipLaunchKernelGGL(k_state_stats2<D>, dim3(1), dim3(kRedBlocks), 0, S(stream), A);
  return 0;
}

int launch_state_stats(const KArgs &A, const double *U, void *stream) {
  clear_stale();
  switch (A.dim) {
    case 1: stats_impl<1>(A, U, stream); break;
    case 2: stats_impl<2>(A, U, stream); break;
    case 3: stats_impl<3>(A, U, stream); break;
    default: return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_zero_counts(const KArgs &A, void *stream) {
  clear_stale();
  const int n = kCntKinds * kCntSlots * kCntStride;
  hipLaunchKernelGGL(k_zero_counts, dim3((n + 255) / 256), dim3(256), 0, S(stream), A.cnt, n);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_prim(const KArgs &A, const double *U, int stage, void *stream) {
  clear_stale();
  const unsigned gp = (unsigned)((A.N + kBlockThreads - 1) / kBlockThreads);
  switch (A.dim) {
    case 1: hipLaunchKernelGGL(k_prim<1>, dim3(gp), dim3(kBlockThreads), 0, S(stream), A, U, stage); break;
    case 2: hipLaunchKernelGGL(k_prim<2>, dim3(gp), dim3(kBlockThreads), 0, S(stream), A, U, stage); break;
    case 3: hipLaunchKernelGGL(k_prim<3>, dim3(gp), dim3(kBlockThreads), 0, S(stream), A, U, stage); break;
    default: return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace gdg
