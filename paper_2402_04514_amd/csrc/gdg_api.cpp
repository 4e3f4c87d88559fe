// gdg_api.cpp -- the C-ABI of include/gdg.h: validation, workspace layout,
// SSP-RK3 and SSPRK(5,4) driver with CFL restarts, state transfer.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gdg.h"
#include "gdg_internal.h"

using namespace gdg;

struct gdg_ctx {
  gdg_mesh_desc mesh;
  gdg_params prm;
  KArgs A;
  hipStream_t stream;
  double *U[3];   // three state buffers; U[cur] holds the state
  int cur;
  RefTables *dref;
  std::string err;
  Ctl hctl;
  double t;
  int64_t steps, restarts;
  double last_dt;
  int M;
  // kernel timing (gdg_profile)
  bool prof_on;
  std::vector<void *> prof_ev;   // events of the host-driven path
  std::vector<int> prof_kid;
  Prof prof;
  double prof_ms[KID_COUNT];
  int64_t prof_launches[KID_COUNT];
  // device-driven runs: a captured graph of kGraphSteps steps
  hipStream_t cap_stream;
  hipGraphExec_t graph_exec;
  // general cells: the caller's vertices (mesh.vertices points here); boundary
  // parts: their kinds (mesh.bc_cells points here)
  std::vector<double> vx;
  std::vector<int8_t> bcc;
  // unstructured meshes: the cells' point ids and the boundary faces' kinds
  std::vector<int64_t> ucp;
  std::vector<int8_t> ufb;
};

namespace {

// message of the last failed gdg_create on this thread (no context exists)
thread_local std::string g_create_err;

struct Layout {
  int nloc, nb1, R, cpb, W, M;
  int64_t N, ncells, nblocks, nslots;
  size_t off_ref, off_ctl, off_col, off_c, off_meta, off_kscale, off_U[3], off_Nd, off_Nold, off_Qd, off_Ld, off_U1d,
      off_dL, off_l1, off_acc, off_fsum, off_red, off_cnt, off_mrow, off_hprow, off_relrow, off_cmblk, off_cminv,
      off_bcc, total;
  int64_t bcc_off[6], nbcc;  // boundary parts: first entry of each face, and the count
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool is_data_kind(int k) { return k == GDG_BC_DIRICHLET || k == GDG_BC_SUPERSONIC || k == GDG_BC_INOUTFLOW; }

// Entries of the boundary parts before face f and on it (bc_cells layout).
void part_offsets(const gdg_mesh_desc *m, int64_t *off, int64_t *total) {
  int64_t n = 0;
  for (int f = 0; f < 6; ++f) {
    off[f] = n;
    if (f >= 2 * m->dim || m->bc[f] == GDG_BC_PERIODIC) continue;
    int64_t cnt = 1;
    for (int g = 0; g < m->dim; ++g)
      if (g != f / 2) cnt *= m->cells[g];
    n += cnt;
  }
  *total = n;
}

// Whether some part of face f takes the face's data.
bool face_has_data(const gdg_mesh_desc *m, int f) {
  if (m->ucells > 0) {
    // unstructured: some boundary face names a data kind with data slot f
    for (int64_t q = 0; q < m->ucells * 2 * m->dim; ++q) {
      const int8_t u = m->uface_bc[q];
      if (u > 0 && is_data_kind(u & 7) && (u >> 3) == f) return true;
    }
    return false;
  }
  if (m->bc[f] == GDG_BC_PERIODIC) return false;
  if (!m->bc_cells) return is_data_kind(m->bc[f]);
  int64_t off[6], n;
  part_offsets(m, off, &n);
  const int64_t end = f + 1 < 6 ? off[f + 1] : n;
  for (int64_t q = off[f]; q < end; ++q)
    if (is_data_kind(m->bc_cells[q])) return true;
  return false;
}

bool validate(const gdg_mesh_desc *m, const gdg_params *p, std::string *err) {
  if (!m || !p) { *err = "null argument"; return false; }
  if (m->dim < 1 || m->dim > 3) { *err = "dim must be 1, 2 or 3"; return false; }
  if (m->degree < 1 || m->degree > 3) { *err = "degree must be 1, 2 or 3"; return false; }
  if (m->degree == 3 && m->dim == 3) { *err = "degree 3 is built for dim 1 and 2"; return false; }
  int64_t ncells = 1;
  if (m->ucells < 0) { *err = "ucells must be >= 0"; return false; }
  if (m->ucells > 0) {
    // unstructured: points, cells' point lists and boundary faces
    if (m->dim < 2) { *err = "unstructured meshes are built for dim 2 and 3"; return false; }
    if (!m->vertices || !m->ucell_points || !m->uface_bc || m->npoints < 1) {
      *err = "an unstructured mesh needs vertices, npoints, ucell_points and uface_bc";
      return false;
    }
    if (m->bc_cells) { *err = "bc_cells is for lattice meshes (unstructured: uface_bc)"; return false; }
    if (m->data_kind == GDG_DATA_VORTEX) { *err = "vortex data are built for the uniform box"; return false; }
    const int g = m->map_degree == 2 ? 2 : 1;
    int np = 1;
    for (int e = 0; e < m->dim; ++e) np *= g + 1;
    for (int64_t q = 0; q < m->ucells * np; ++q)
      if (m->ucell_points[q] < 0 || m->ucell_points[q] >= m->npoints) {
        *err = "a cell names a point outside vertices";
        return false;
      }
    ncells = m->ucells;
  }
  for (int e = 0; e < m->dim && m->ucells == 0; ++e) {
    if (m->cells[e] < 1) { *err = "cells must be >= 1"; return false; }
    if (!m->vertices && !(m->hi[e] > m->lo[e])) { *err = "hi must exceed lo"; return false; }
    int b0 = m->bc[2 * e], b1 = m->bc[2 * e + 1];
    for (int b : {b0, b1})
      if (b < GDG_BC_PERIODIC || b > GDG_BC_INOUTFLOW) { *err = "unknown boundary kind"; return false; }
    if ((b0 == GDG_BC_PERIODIC) != (b1 == GDG_BC_PERIODIC)) {
      *err = "periodic must be set on both faces of an axis";
      return false;
    }
    if (b0 == GDG_BC_PERIODIC && m->cells[e] < 2) {
      *err = "a periodic axis needs at least 2 cells";
      return false;
    }
    ncells *= m->cells[e];
  }
  // boundary parts and the data of the faces, once every axis is checked
  for (int e = 0; e < m->dim; ++e) {
    if (m->ucells > 0) {
      for (int side = 0; side < 2; ++side) {
        const int f = 2 * e + side;
        if (!face_has_data(m, f) || m->data_kind != GDG_DATA_CONSTANT) continue;
        const double *V = m->bc_state[f];
        double m2 = 0.0;
        for (int k = 0; k < m->dim; ++k) m2 += V[1 + k] * V[1 + k];
        const double rho = V[0], eps = V[m->dim + 1] - 0.5 * m2 / rho;
        if (!(rho > 0.0) || !(eps > 0.0) || !std::isfinite(rho) || !std::isfinite(V[m->dim + 1])) {
          *err = "Dirichlet data of a face is not admissible (rho <= 0, eps <= 0 or not finite)";
          return false;
        }
      }
      continue;
    }
    if (m->bc_cells) {
      // the parts' own kinds: no periodic or unknown kind
      int64_t off[6], n;
      part_offsets(m, off, &n);
      for (int side = 0; side < 2; ++side) {
        const int f = 2 * e + side;
        const int64_t end = f + 1 < 6 ? off[f + 1] : n;
        for (int64_t q = off[f]; q < end; ++q)
          if (m->bc_cells[q] <= GDG_BC_PERIODIC || m->bc_cells[q] > GDG_BC_INOUTFLOW) {
            *err = "a boundary part has a periodic or unknown kind";
            return false;
          }
      }
    }
    for (int side = 0; side < 2; ++side) {
      const int f = 2 * e + side;
      if (!face_has_data(m, f)) continue;
      if (m->data_kind != GDG_DATA_CONSTANT) continue;  // vortex: checked below; step start: U^n
      // the face's data must lie in A (eq. AddSet)
      const double *V = m->bc_state[f];
      double m2 = 0.0;
      for (int k = 0; k < m->dim; ++k) m2 += V[1 + k] * V[1 + k];
      const double rho = V[0], eps = V[m->dim + 1] - 0.5 * m2 / rho;
      if (!(rho > 0.0) || !(eps > 0.0) || !std::isfinite(rho) || !std::isfinite(V[m->dim + 1])) {
        *err = "Dirichlet data of a face is not admissible (rho <= 0, eps <= 0 or not finite)";
        return false;
      }
    }
  }
  if (m->data_kind != GDG_DATA_CONSTANT && m->data_kind != GDG_DATA_VORTEX && m->data_kind != GDG_DATA_STEP_START) {
    *err = "unknown boundary data kind";
    return false;
  }
  if (m->continuous != 0 && m->continuous != 1) { *err = "continuous must be 0 or 1"; return false; }
  if (m->continuous) {
    if (m->bc_cells || m->ucells > 0 || m->data_kind != GDG_DATA_CONSTANT) {
      *err = "continuous elements are built for lattices of cells (no bc_cells, unstructured cells, vortex or "
             "step-start data)";
      return false;
    }
    if (p->scheme != GDG_LOW_ORDER) {
      *err = "continuous elements take the low-order scheme (their high-order update needs a global mass "
             "solve)";
      return false;
    }
    for (int e = 0; e < m->dim; ++e)
      if (m->bc[2 * e] == GDG_BC_PERIODIC && m->degree * m->cells[e] < 2 * m->degree + 1) {
        *err = "a periodic axis of continuous elements needs at least 2 degree + 1 nodes";
        return false;
      }
  }
  if (m->map_degree < 0 || m->map_degree > 2 || (m->map_degree == 2 && !m->vertices)) {
    *err = "map_degree must be 0 or 1 (multilinear), or 2 (quadratic, with vertices)";
    return false;
  }
  if (m->vertices && m->data_kind == GDG_DATA_VORTEX) {
    *err = "vortex boundary data are built for the uniform box (vertices must be NULL)";
    return false;
  }
  if (m->data_kind == GDG_DATA_VORTEX) {
    // the vortex of Sec. 6.2: beta, x0, u_inf, gamma; its density is positive
    // where 1 - (gamma-1) beta^2 e / (8 gamma pi^2) > 0 (the core, r = 0)
    const double *v = m->vortex;
    const double pi = 3.14159265358979323846;
    bool ok = m->dim == 2;
    for (int k = 0; k < 6; ++k) ok = ok && std::isfinite(v[k]);
    ok = ok && v[0] >= 0.0 && v[5] > 1.0 && v[5] <= 5.0 / 3.0 + 1e-12;
    ok = ok && 1.0 - (v[5] - 1.0) * v[0] * v[0] * std::exp(1.0) / (8.0 * v[5] * pi * pi) > 0.0;
    if (!ok) {
      *err = "vortex boundary data need a 2D mesh, finite parameters, beta >= 0, gamma in (1, 5/3] and a "
             "positive core density";
      return false;
    }
  }
  int nloc = 1;
  for (int e = 0; e < m->dim; ++e) nloc *= m->degree + 1;
  if (ncells * nloc >= (int64_t(1) << 31)) { *err = "too many dofs for 32-bit column indices"; return false; }
  {
    int nface = 1;
    for (int e = 0; e < m->dim - 1; ++e) nface *= m->degree + 1;
    const int cpb = kBlockThreads / nloc;
    const int64_t nblocks = (ncells + cpb - 1) / cpb;
    if (nblocks * (nloc + m->dim * nface) * (cpb * nloc) >= (int64_t(1) << 31)) {
      *err = "too many stencil slots for 32-bit slot indices";
      return false;
    }
  }
  // the two-rarefaction bound is an upper bound for 1 < gamma <= 5/3
  if (!(p->gamma > 1.0 && p->gamma <= 5.0 / 3.0 + 1e-12)) { *err = "gamma must lie in (1, 5/3]"; return false; }
  if (!(p->cfl > 0.0 && p->cfl <= 1.0)) { *err = "cfl must lie in (0, 1]"; return false; }
  if (!(p->c_ev >= 0.0) || !(p->c_k >= 0.0) || !(p->c_r >= 0.0) || !(p->p_r >= 0.0)) {
    *err = "scheme constants must be non-negative";
    return false;
  }
  if (p->limiter_passes < 0 || p->limiter_passes > 2) { *err = "limiter_passes must be 0, 1 or 2"; return false; }
  if (p->flags & ~GDG_FLAG_NO_QUIET_ROWS) { *err = "unknown flags"; return false; }
  if (p->scheme < 0 || p->scheme > 2) { *err = "unknown scheme"; return false; }
  if (p->precision != GDG_FP64 && p->precision != GDG_MIXED) { *err = "unknown precision"; return false; }
  if (p->integrator != GDG_SSPRK3 && p->integrator != GDG_SSPRK54) { *err = "unknown integrator"; return false; }
  return true;
}

Layout layout(const gdg_mesh_desc *m, const gdg_params *p) {
  Layout L;
  L.nb1 = m->degree + 1;
  L.nloc = 1;
  int nface = 1;
  for (int e = 0; e < m->dim; ++e) L.nloc *= L.nb1;
  for (int e = 0; e < m->dim - 1; ++e) nface *= L.nb1;
  L.M = m->dim + 2;
  L.cpb = kBlockThreads / L.nloc;
  L.R = L.cpb * L.nloc;
  L.W = L.nloc + m->dim * nface;
  L.ncells = 1;
  for (int e = 0; e < m->dim; ++e) L.ncells *= m->cells[e];
  if (m->ucells > 0) L.ncells = m->ucells;
  L.N = L.ncells * L.nloc;
  L.nblocks = (L.ncells + L.cpb - 1) / L.cpb;
  if (m->continuous) {
    // one row per node of the continuous space, full wavefronts of rows; a
    // row holds the (2k+1)^d nodes around it and a part per box face
    int64_t gn[3];
    cg_nodes(m, gn);
    L.N = gn[0] * gn[1] * gn[2];
    L.R = kBlockThreads;
    int span = 1;
    for (int e = 0; e < m->dim; ++e) span *= 2 * m->degree + 1;
    L.W = span + m->dim;
    L.nblocks = (L.N + L.R - 1) / L.R;
  }
  L.nslots = L.nblocks * L.W * L.R;
  const size_t N = (size_t)L.N, S = (size_t)L.nslots, d = (size_t)m->dim, M = (size_t)L.M;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  L.off_ref = take(sizeof(RefTables));
  L.off_ctl = take(sizeof(Ctl));
  L.off_col = take(S * 4);
  L.off_c = take(S * d * (p->precision == GDG_MIXED ? 4 : 8));
  const bool host_tables = m->vertices || m->continuous;
  L.off_meta = take(S);
  L.off_kscale = take(N * 8);
  for (int k = 0; k < 3; ++k) L.off_U[k] = take(M * N * 8);
  L.off_Nd = take(2 * N * kNodeStride * 8);
  L.off_Nold = m->data_kind == GDG_DATA_STEP_START ? take(N * kNodeStride * 8) : 0;
  L.off_Qd = take(N * kQStride * 8);
  L.off_Ld = take(N * kLimStride * 8);
  L.off_U1d = take(N * kU1Stride * 8);
  L.off_dL = take(S * 8);
  L.off_l1 = take(S * 8);
  L.off_acc = take(N);
  L.off_fsum = take(M * N * 8);
  L.off_red = take((size_t)(kRedBlocks + 1) * kRedFields * 8);
  L.off_cnt = take((size_t)kCntKinds * kCntSlots * kCntStride * 8);
  L.off_mrow = L.off_hprow = L.off_relrow = L.off_cmblk = L.off_cminv = L.off_bcc = 0;
  for (int f = 0; f < 6; ++f) L.bcc_off[f] = 0;
  L.nbcc = 0;
  if (m->bc_cells) part_offsets(m, L.bcc_off, &L.nbcc);
  if (m->bc_cells) L.off_bcc = take((size_t)L.nbcc);
  if (host_tables) {
    const size_t blk = m->continuous ? 0 : (size_t)L.ncells * L.nloc * L.nloc * 8;
    L.off_mrow = take(N * 8);
    L.off_hprow = take(N * 8);
    L.off_relrow = take(N * 8);
    L.off_cmblk = take(blk);
    L.off_cminv = take(blk);
  }
  L.total = o;
  return L;
}

#define HIPCHK(ctx, call)                                                     \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);         \
      return GDG_E_DEVICE;                                                    \
    }                                                                         \
  } while (0)

gdg_status launched(gdg_ctx *ctx, int rc, const char *what) {
  if (rc == 0) return GDG_OK;
  ctx->err = std::string("kernel launch failed: ") + what;
  return GDG_E_DEVICE;
}

gdg_status read_ctl(gdg_ctx *ctx) {
  HIPCHK(ctx, hipMemcpyAsync(&ctx->hctl, ctx->A.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return GDG_OK;
}

// Folds the bracketed launches of a synchronized stream into the sums.
gdg_status harvest_prof(gdg_ctx *ctx, const Prof &p) {
  for (int k = 0; k < p.n; ++k) {
    float ms = 0.0f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, (hipEvent_t)p.ev[2 * k], (hipEvent_t)p.ev[2 * k + 1]));
    ctx->prof_ms[p.kid[k]] += ms;
    ctx->prof_launches[p.kid[k]] += 1;
  }
  return GDG_OK;
}

gdg_status harvest(gdg_ctx *ctx) {
  if (!ctx->prof_on) return GDG_OK;
  gdg_status s = harvest_prof(ctx, ctx->prof);
  ctx->prof.n = 0;
  return s;
}

Prof *prof_of(gdg_ctx *ctx) { return ctx->prof_on ? &ctx->prof : nullptr; }

gdg_status make_events(gdg_ctx *ctx, std::vector<void *> &ev, std::vector<int> &kid, int launches, Prof &p) {
  ev.resize(2 * (size_t)launches);
  kid.resize((size_t)launches);
  for (auto &e : ev) {
    hipEvent_t h;
    HIPCHK(ctx, hipEventCreate(&h));
    e = (void *)h;
  }
  p.ev = ev.data();
  p.kid = kid.data();
  p.cap = launches;
  p.n = 0;
  return GDG_OK;
}

void free_events(std::vector<void *> &ev) {
  for (void *e : ev) (void)hipEventDestroy((hipEvent_t)e);
  ev.clear();
}

void drop_graph(gdg_ctx *ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  ctx->graph_exec = nullptr;
}

// SSPRK(5,4) of Spiteri and Ruuth, Shu-Osher form
//   u(i) = sum_k alpha_ik u(k) + tau beta_ik L(u(k)),  u(0) = U^n, u(5) = U^{n+1},
// with the coefficients as published (15 digits).  Each stage i > 0 reads at
// most two earlier states besides its Euler step, which the buffers below
// exploit.
constexpr double kA10 = 1.0;
constexpr double kB10 = 0.391752226571890;
constexpr double kA20 = 0.444370493651235, kA21 = 0.555629506348765, kB21 = 0.368410593050371;
constexpr double kA30 = 0.620101851488403, kA32 = 0.379898148511597, kB32 = 0.251891774271694;
constexpr double kA40 = 0.178079954393132, kA43 = 0.821920045606868, kB43 = 0.544974750228521;
constexpr double kA52 = 0.517231671970585, kA53 = 0.096059710526147;  // beta_53 = 0.063692468666290
constexpr double kA54 = 0.386708617503269, kB54 = 0.226007483236906;

// Stage k of a step as a forward-Euler stage of size tstep[k] tau at time
// t + tfrac[k] tau.  SSP-RK3: three stages of size tau at t, t + tau,
// t + tau / 2.  SSPRK(5,4): r_k = beta_{k+1,k} / alpha_{k+1,k}; tfrac[k] is
// the stage's abscissa c_k, the row sum of the method's Butcher matrix
// (c_0 = 0, c_1 = b10, c_2 = a21 b10 + b21, c_3 = a32 c_2 + b32,
// c_4 = a43 c_3 + b43).  The term beta_53 tau L(u(3)) of the last stage
// reuses the Euler step of u(3): beta_53 / alpha_53 equals r_3 to the
// published digits (they differ by 1.2e-15 relative).
void set_integrator(KArgs &A, int integrator) {
  if (integrator == GDG_SSPRK54) {
    A.nst = 5;
    const double c1 = kB10, c2 = kA21 * kB10 + kB21, c3 = kA32 * c2 + kB32, c4 = kA43 * c3 + kB43;
    const double r[5] = {kB10 / kA10, kB21 / kA21, kB32 / kA32, kB43 / kA43, kB54 / kA54};
    const double c[5] = {0.0, c1, c2, c3, c4};
    A.tstep_max = 0.0;
    for (int k = 0; k < 5; ++k) {
      A.tstep[k] = r[k];
      A.tfrac[k] = c[k];
      A.tstep_max = r[k] > A.tstep_max ? r[k] : A.tstep_max;
    }
    return;
  }
  A.nst = 3;
  const double c[5] = {0.0, 1.0, 0.5, 0.0, 0.0};
  for (int k = 0; k < kMaxStages; ++k) {
    A.tstep[k] = k < 3 ? 1.0 : 0.0;
    A.tfrac[k] = c[k];
  }
  A.tstep_max = 1.0;
}

// One step on a stream: begin, the integrator's stages, end.
// first / last: whether this step opens / closes a sequence of device-driven
// steps (inside a sequence, one launch ends a step and starts the next).
int enqueue_step(gdg_ctx *ctx, hipStream_t st, int device_driven, double dt_cap, double tau_fixed, Prof *prof,
                 bool first = true, bool last = true) {
  const KArgs &A = ctx->A;
  const int c0 = ctx->cur, c1 = (c0 + 1) % 3, c2 = (c0 + 2) % 3;
  double *B0 = ctx->U[c0], *B1 = ctx->U[c1], *B2 = ctx->U[c2];
  StageBufs b[kMaxStages];
  if (A.nst == 5) {
    // U^n stays whole in B0 until the last stage has passed its CFL check
    // (a restart starts again from it).  A stage reads its input state in
    // its first sweep only (later sweeps read the node records), so stage 3
    // may write u(4) over its input u(3).  u(2) turns into the partial sum
    // alpha_52 u(2) + beta_53 tau L(u(3)) in place.
    b[0] = {B0, B1, B0, 0.0, 1.0};                        // u1 = Phi_0(u0)
    b[1] = {B1, B2, B0, kA20, kA21};                      // u2
    b[2] = {B2, B1, B0, kA30, kA32};                      // u3 over u1
    b[3] = {B1, B1, B0, kA40, kA43, B2, B2, kA52, kA53};  // u4 over u3, partial sum over u2
    b[4] = {B1, B0, B2, 1.0, kA54};                       // u5 = partial sum + alpha_54 Phi_4(u4)
  } else {
    b[0] = {B0, B1, B0, 0.0, 1.0};
    b[1] = {B1, B2, B0, 0.75, 0.25};
    b[2] = {B2, B0, B0, 1.0 / 3.0, 2.0 / 3.0};
  }
  int rc = first ? launch_begin(A, dt_cap, tau_fixed, device_driven, st) : 0;
  // host-driven steps recompute the node cache of U^n: after a restart it
  // holds the state of an abandoned stage; device-driven steps follow a
  // completed step (or the upload, or a host-driven step) whose last stage
  // wrote it
  for (int k = 0; k < A.nst; ++k) rc |= launch_stage(A, b[k], k, st, prof, k == 0 && !device_driven ? 1 : 0);
  rc |= last ? launch_end(A, st) : launch_end_begin(A, st);
  return rc;
}

constexpr int kGraphSteps = 8;

// Captures kGraphSteps device-driven steps into a graph (once per context
// and profiling mode).  Capture runs on a private stream; launches go to the
// context's stream.
gdg_status ensure_graph(gdg_ctx *ctx) {
  if (ctx->graph_exec) return GDG_OK;
  if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  Prof *pp = nullptr;
  HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = 0;
  for (int k = 0; k < kGraphSteps; ++k)
    rc |= enqueue_step(ctx, ctx->cap_stream, 1, 0.0, 0.0, pp, k == 0, k + 1 == kGraphSteps);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
  if (rc != 0 || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    ctx->err = std::string("graph capture failed: ") + hipGetErrorString(e);
    return GDG_E_DEVICE;
  }
  e = hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ctx->graph_exec = nullptr;
    ctx->err = std::string("graph instantiation failed: ") + hipGetErrorString(e);
    return GDG_E_DEVICE;
  }
  return GDG_OK;
}

void sync_time(gdg_ctx *ctx) {
  ctx->t = ctx->hctl.t;
  ctx->steps = ctx->hctl.steps;
}

double bits_to_double(unsigned long long b) {
  double d;
  std::memcpy(&d, &b, sizeof d);
  return d;
}

}  // namespace

extern "C" {

gdg_status gdg_default_params(int32_t degree, gdg_params *out) {
  if (!out || degree < 1 || degree > 3) return GDG_E_INVALID;
  std::memset(out, 0, sizeof *out);
  out->gamma = 1.4;
  out->cfl = 0.5;
  out->c_ev = degree == 1 ? 1.0 : (degree == 2 ? 0.5 : 0.25);
  out->c_k = 1.0;
  out->c_r = 4.0;
  out->p_r = 1.5;
  out->limiter_passes = 2;
  out->scheme = GDG_LIMITED;
  out->precision = GDG_FP64;
  return GDG_OK;
}

gdg_status gdg_workspace_bytes(const gdg_mesh_desc *mesh, const gdg_params *prm, size_t *bytes) {
  std::string err;
  if (!bytes || !validate(mesh, prm, &err)) return GDG_E_INVALID;
  *bytes = layout(mesh, prm).total;
  return GDG_OK;
}

gdg_status gdg_create(const gdg_mesh_desc *mesh, const gdg_params *prm, void *dev_workspace,
                      size_t ws_bytes, void *hip_stream, gdg_ctx **out) {
  g_create_err.clear();
  if (!out) { g_create_err = "null output pointer"; return GDG_E_INVALID; }
  *out = nullptr;
  std::string err;
  if (!validate(mesh, prm, &err)) { g_create_err = err; return GDG_E_INVALID; }
  Layout L = layout(mesh, prm);
  if (!dev_workspace || ws_bytes < L.total) {
    g_create_err = "workspace smaller than gdg_workspace_bytes()";
    return GDG_E_NOMEM;
  }
  if (((uintptr_t)dev_workspace & 255) != 0) {
    g_create_err = "workspace not 256-byte aligned";
    return GDG_E_INVALID;
  }
  gdg_ctx *ctx = new gdg_ctx();
  ctx->mesh = *mesh;
  if (mesh->vertices) {
    size_t npts = 1;
    for (int e = 0; e < mesh->dim; ++e) npts *= (size_t)(map_degree(mesh) * mesh->cells[e] + 1);
    if (mesh->ucells > 0) npts = (size_t)mesh->npoints;
    ctx->vx.assign(mesh->vertices, mesh->vertices + npts * mesh->dim);
    ctx->mesh.vertices = ctx->vx.data();
  }
  if (mesh->ucells > 0) {
    int np = 1;
    for (int e = 0; e < mesh->dim; ++e) np *= map_degree(mesh) + 1;
    ctx->ucp.assign(mesh->ucell_points, mesh->ucell_points + mesh->ucells * np);
    ctx->ufb.assign(mesh->uface_bc, mesh->uface_bc + mesh->ucells * 2 * mesh->dim);
    ctx->mesh.ucell_points = ctx->ucp.data();
    ctx->mesh.uface_bc = ctx->ufb.data();
  }
  if (mesh->bc_cells) {
    ctx->bcc.assign(mesh->bc_cells, mesh->bc_cells + L.nbcc);
    ctx->mesh.bc_cells = ctx->bcc.data();
  }
  ctx->prm = *prm;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->M = L.M;
  char *ws = (char *)dev_workspace;
  KArgs &A = ctx->A;
  std::memset(&A, 0, sizeof A);
  A.N = L.N;
  A.nblocks = L.nblocks;
  A.ncells = L.ncells;
  A.R = L.R;
  A.W = L.W;
  A.nloc = L.nloc;
  A.nb1 = L.nb1;
  A.deg = mesh->degree;
  A.dim = mesh->dim;
  A.cpb = L.cpb;
  A.tiled = 0;
  A.t_nbx = A.t_ny = A.t_nz = A.t_tx = A.t_ty = 1;
  if (mesh->dim == 3 && mesh->ucells == 0 && !mesh->continuous && mesh->cells[0] % L.cpb == 0) {
    // tiles one row block wide in x and ty cell rows in y, ty the largest
    // divisor of ny up to kTileRows (measured on the 128^3 blast: 1 x 32 and
    // 1 x 64 beat the 16 x 8 tiles by 5 %)
    const int64_t nbx = mesh->cells[0] / L.cpb, ny = mesh->cells[1];
    const int64_t tx = 1;
    int64_t ty = 1;
    for (int64_t b = 1; b <= ny && b <= kTileRows; ++b)
      if (ny % b == 0) ty = b;
    A.tiled = 1;
    A.t_nbx = nbx;
    A.t_ny = ny;
    A.t_nz = mesh->cells[2];
    A.t_tx = tx;
    A.t_ty = ty;
  }
  double h[3] = {1, 1, 1}, vol = 1.0;
  for (int e = 0; e < 3; ++e) A.cells[e] = e < mesh->dim ? mesh->cells[e] : 1;
  if (mesh->ucells > 0) A.cells[0] = mesh->ucells, A.cells[1] = A.cells[2] = 1;
  for (int e = 0; e < mesh->dim && !mesh->vertices; ++e) {
    h[e] = (mesh->hi[e] - mesh->lo[e]) / (double)mesh->cells[e];
    vol *= mesh->hi[e] - mesh->lo[e];
  }
  A.bcdata = 0;
  for (int f = 0; f < 6; ++f) {
    A.bc[f] = f < 2 * mesh->dim && mesh->ucells == 0 ? mesh->bc[f] : GDG_BC_OUTFLOW;
    if (f < 2 * mesh->dim && face_has_data(mesh, f)) A.bcdata |= 1 << f;
    A.bcc_off[f] = L.bcc_off[f];
  }
  A.bcc = mesh->bc_cells ? (const int8_t *)(ws + L.off_bcc) : nullptr;
  A.gamma = prm->gamma;
  A.cfl = prm->cfl;
  A.c_ev = prm->c_ev;
  A.c_k = prm->c_k;
  A.pk = mesh->degree % 2 == 0 ? 0.5 : 0.0;
  A.c_r = prm->c_r;
  A.p_r = prm->p_r;
  A.vol = vol;
  A.alpha = (prm->gamma - 1.0) / (2.0 * prm->gamma);
  A.inv_alpha = 1.0 / A.alpha;
  double ri = std::round(A.inv_alpha);
  A.ipow = (std::fabs(A.inv_alpha - ri) < 1e-9 && ri >= 1 && ri <= 32) ? (int)ri : 0;
  A.g75 = std::fabs(prm->gamma - 1.4) < 1e-15 ? 1 : 0;
  A.scheme = prm->scheme;
  A.passes = prm->limiter_passes;
  set_integrator(A, prm->integrator);
  A.no_quiet = (prm->flags & GDG_FLAG_NO_QUIET_ROWS) ? 1 : 0;
  A.nslots = L.nslots;
  A.ref = (const RefTables *)(ws + L.off_ref);
  ctx->dref = (RefTables *)(ws + L.off_ref);
  A.ctl = (Ctl *)(ws + L.off_ctl);
  A.col = (int32_t *)(ws + L.off_col);
  A.mixed = prm->precision == GDG_MIXED ? 1 : 0;
  A.c = A.mixed ? nullptr : (double *)(ws + L.off_c);
  A.cf = A.mixed ? (float *)(ws + L.off_c) : nullptr;
  A.meta = (uint8_t *)(ws + L.off_meta);
  A.kscale = (double *)(ws + L.off_kscale);
  for (int k = 0; k < 3; ++k) ctx->U[k] = (double *)(ws + L.off_U[k]);
  ctx->cur = 0;

  A.Nd = (double *)(ws + L.off_Nd);
  A.Nold = mesh->data_kind == GDG_DATA_STEP_START ? (double *)(ws + L.off_Nold) : nullptr;
  A.Qd = (double *)(ws + L.off_Qd);
  A.Ld = (double *)(ws + L.off_Ld);
  A.U1d = (double *)(ws + L.off_U1d);
  A.dL = (double *)(ws + L.off_dL);
  A.l1 = (double *)(ws + L.off_l1);
  A.accepted = (uint8_t *)(ws + L.off_acc);
  A.fsum = (double *)(ws + L.off_fsum);
  A.red = (double *)(ws + L.off_red);
  A.cnt = (unsigned long long *)(ws + L.off_cnt);
  A.general = mesh->vertices || mesh->continuous ? 1 : 0;
  A.ustruct = mesh->ucells > 0 || mesh->continuous ? 1 : 0;
  A.cg = mesh->continuous ? 1 : 0;
  if (A.general) {
    A.mrow = (const double *)(ws + L.off_mrow);
    A.hprow = (const double *)(ws + L.off_hprow);
    A.relrow = (const double *)(ws + L.off_relrow);
    A.cmblk = (const double *)(ws + L.off_cmblk);
    A.cminv = (const double *)(ws + L.off_cminv);
  }

  RefTables *T = new RefTables();
  if (!build_ref_tables(mesh->dim, mesh->degree, h, T, &err)) {
    g_create_err = err;
    delete T;
    delete ctx;
    return GDG_E_INVALID;
  }
  // general cells: per-row and per-cell tables from the map, and the stencil
  // coefficients that replace those of the fill kernel
  MappedSetup G;
  if (A.cg) {
    if (!build_cg(&ctx->mesh, prm, L.R, L.W, L.nslots, &G, &err)) {
      g_create_err = err;
      delete T;
      delete ctx;
      return GDG_E_INVALID;
    }
    A.vol = vol = G.vol;
  } else if (A.general) {
    if (!build_mapped(&ctx->mesh, prm, ctx->vx.data(), *T, L.R, L.W, L.nslots, &G, &err)) {
      g_create_err = err;
      delete T;
      delete ctx;
      return GDG_E_INVALID;
    }
    A.vol = vol = G.vol;
  }
  for (int a = 0; a < L.nloc && !A.general; ++a) {
    double hh = std::pow(T->mlump[a] / vol, 1.0 / mesh->dim);
    T->hpk[a] = prm->c_k * std::pow(hh, A.pk);
    T->relax[a] = prm->c_r * std::pow(hh, prm->p_r);
    if (!(T->relax[a] < 1.0)) {
      g_create_err = "relaxation c_r h^p_r >= 1: the lower bounds would not be positive";
      delete T;
      delete ctx;
      return GDG_E_INVALID;
    }
  }
  const bool data_faces = mesh->data_kind == GDG_DATA_CONSTANT;
  for (int f = 0; f < 2 * mesh->dim; ++f)
    if (data_faces &&
        ((A.bcdata >> f) & 1))
      for (int q = 0; q < L.M; ++q) T->bstate[f][q] = mesh->bc_state[f][q];
  {
    // Gauss-Lobatto nodes on [0, 1], as in gdg_node_coords
    const double r5 = 0.5 / std::sqrt(5.0);
    const double x1[4] = {0.0, 1.0, 0.0, 0.0}, x2[4] = {0.0, 0.5, 1.0, 0.0}, x3[4] = {0.0, 0.5 - r5, 0.5 + r5, 1.0};
    const double *xg = mesh->degree == 1 ? x1 : (mesh->degree == 2 ? x2 : x3);
    for (int k = 0; k < 4; ++k) T->xg[k] = xg[k];
  }
  A.vortex_data = mesh->data_kind == GDG_DATA_VORTEX ? 1 : 0;
  A.old_data = mesh->data_kind == GDG_DATA_STEP_START ? 1 : 0;
  for (int k = 0; k < 6; ++k) A.vx[k] = mesh->vortex[k];
  for (int e = 0; e < 3; ++e) {
    A.lo[e] = e < mesh->dim ? mesh->lo[e] : 0.0;
    A.hx[e] = h[e];
  }
  std::memset(&ctx->hctl, 0, sizeof(Ctl));
  hipError_t e1 = hipMemcpyAsync(ctx->dref, T, sizeof(RefTables), hipMemcpyHostToDevice, ctx->stream);
  hipError_t e2 = hipMemcpyAsync(A.ctl, &ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream);
  if (e2 == hipSuccess && A.bcc)
    e2 = hipMemcpyAsync((void *)A.bcc, ctx->bcc.data(), (size_t)L.nbcc, hipMemcpyHostToDevice, ctx->stream);
  int rc = (e1 == hipSuccess && e2 == hipSuccess) ? launch_fill(A, ctx->stream) : -1;
  if (rc == 0 && A.general) {
    // after the fill kernel on the same stream: its c and kappa entries are
    // those of the uniform cell and are overwritten here
    std::vector<float> cf;
    const void *csrc = G.c.data();
    size_t cbytes = G.c.size() * sizeof(double);
    if (A.mixed) {
      cf.assign(G.c.begin(), G.c.end());
      csrc = cf.data();
      cbytes = cf.size() * sizeof(float);
    }
    const size_t nb = (size_t)A.N * 8, bb = G.cmblk.size() * 8;
    hipError_t e = hipSuccess;
    auto cp = [&](const void *dst, const void *src, size_t bytes) {
      if (e == hipSuccess) e = hipMemcpyAsync((void *)dst, src, bytes, hipMemcpyHostToDevice, ctx->stream);
    };
    cp(A.mixed ? (const void *)A.cf : (const void *)A.c, csrc, cbytes);
    cp(A.kscale, G.kscale.data(), nb);
    cp(A.mrow, G.mrow.data(), nb);
    cp(A.hprow, G.hprow.data(), nb);
    cp(A.relrow, G.relrow.data(), nb);
    cp(A.cmblk, G.cmblk.data(), bb);
    cp(A.cminv, G.cminv.data(), bb);
    if (A.ustruct) {
      // the whole stencil: the fill kernel leaves unstructured meshes alone
      cp(A.col, G.col.data(), G.col.size() * sizeof(int32_t));
      cp(A.meta, G.meta.data(), G.meta.size());
    }
    // the host vectors must outlive the copies
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      g_create_err = std::string("copy of the general-cell tables failed: ") + hipGetErrorString(e);
      delete T;
      delete ctx;
      return GDG_E_DEVICE;
    }
  }
  if (rc == 0) rc = launch_zero_counts(A, ctx->stream);
  hipError_t e4 = rc == 0 ? hipSuccess : hipGetLastError();
  hipError_t e3 = hipStreamSynchronize(ctx->stream);
  Ctl chk;
  std::memset(&chk, 0, sizeof chk);
  if (rc == 0 && e3 == hipSuccess) e3 = hipMemcpy(&chk, A.ctl, sizeof(Ctl), hipMemcpyDeviceToHost);
  delete T;
  if (rc == 0 && e3 == hipSuccess && chk.bad_flag) {
    g_create_err = "internal error: the stencil is not symmetric";
    delete ctx;
    return GDG_E_DEVICE;
  }
  if (rc != 0 || e3 != hipSuccess) {
    hipError_t e = e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : (e4 != hipSuccess ? e4 : e3));
    g_create_err = std::string(e1 != hipSuccess || e2 != hipSuccess ? "copy of the setup tables"
                                                                     : (rc ? "stencil fill launch" : "stream sync")) +
                   " failed: " + hipGetErrorString(e);
    delete ctx;
    return GDG_E_DEVICE;
  }
  *out = ctx;
  return GDG_OK;
}

void gdg_destroy(gdg_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  drop_graph(ctx);
  free_events(ctx->prof_ev);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  delete ctx;
}

int64_t gdg_num_dofs(const gdg_ctx *ctx) { return ctx ? ctx->A.N : -1; }

gdg_status gdg_node_coords(const gdg_ctx *ctx, double *xyz) {
  if (!ctx || !xyz) return GDG_E_INVALID;
  const gdg_mesh_desc &m = ctx->mesh;
  const int d = m.dim, nb = m.degree + 1, nloc = ctx->A.nloc;
  const double r5 = 0.5 / std::sqrt(5.0);
  const double xg2[3] = {0.0, 0.5, 1.0}, xg1[2] = {0.0, 1.0}, xg3[4] = {0.0, 0.5 - r5, 0.5 + r5, 1.0};
  const double *xg = m.degree == 1 ? xg1 : (m.degree == 2 ? xg2 : xg3);
  if (m.continuous) {
    // node (I_0, I_1, I_2): cell I_e / k (the last node: the last cell's end), local node I_e % k
    int64_t gn[3];
    cg_nodes(&m, gn);
    for (int64_t i = 0; i < ctx->A.N; ++i) {
      int64_t r = i, Kc = 0, stc = 1;
      double xi[3] = {0, 0, 0};
      for (int e = 0; e < d; ++e) {
        const int64_t I = r % gn[e];
        r /= gn[e];
        int64_t K = I / m.degree;
        int a = (int)(I % m.degree);
        if (K == m.cells[e]) K -= 1, a = m.degree;
        const double h = (m.hi[e] - m.lo[e]) / (double)m.cells[e];
        xyz[i * d + e] = m.lo[e] + ((double)K + xg[a]) * h;
        xi[e] = xg[a];
        Kc += K * stc;
        stc *= m.cells[e];
      }
      if (m.vertices) {
        // general cells: the node's cell's map at its reference point
        double X[27][3];
        mapped_cell_points(&m, m.vertices, Kc, X);
        mapped_point(d, map_degree(&m), X, xi, &xyz[i * d]);
      }
    }
    return GDG_OK;
  }
  if (m.vertices) {
    // x_i = F_K(xi_a): the cell's map at the node's reference point
    for (int64_t K = 0; K < ctx->A.ncells; ++K) {
      double X[27][3];
      mapped_cell_points(&m, m.vertices, K, X);
      for (int a = 0; a < nloc; ++a) {
        double xi[3] = {0, 0, 0};
        for (int e = 0, r = a; e < d; ++e, r /= nb) xi[e] = xg[r % nb];
        mapped_point(d, map_degree(&m), X, xi, &xyz[(K * nloc + a) * d]);
      }
    }
    return GDG_OK;
  }
  for (int64_t i = 0; i < ctx->A.N; ++i) {
    int64_t K = i / nloc;
    int a = (int)(i % nloc);
    for (int e = 0; e < d; ++e) {
      int64_t ke = K % m.cells[e];
      K /= m.cells[e];
      int ae = a % nb;
      a /= nb;
      double h = (m.hi[e] - m.lo[e]) / (double)m.cells[e];
      xyz[i * d + e] = m.lo[e] + ((double)ke + xg[ae]) * h;
    }
  }
  return GDG_OK;
}

gdg_status gdg_upload_state(gdg_ctx *ctx, const double *U, int32_t is_device_ptr) {
  if (!ctx || !U) return GDG_E_INVALID;
  (void)is_device_ptr;
  const size_t bytes = (size_t)ctx->M * ctx->A.N * sizeof(double);
  HIPCHK(ctx, hipMemcpyAsync(ctx->U[ctx->cur], U, bytes, hipMemcpyDefault, ctx->stream));
  std::memset(&ctx->hctl, 0, sizeof(Ctl));
  HIPCHK(ctx, hipMemcpyAsync(ctx->A.ctl, &ctx->hctl, sizeof(Ctl), hipMemcpyHostToDevice, ctx->stream));
  if (gdg_status s = launched(ctx, launch_zero_counts(ctx->A, ctx->stream), "zero counters")) return s;
  if (gdg_status s = launched(ctx, launch_begin(ctx->A, 0.0, 0.0, 0, ctx->stream), "begin")) return s;
  if (gdg_status s = launched(ctx, launch_prim(ctx->A, ctx->U[ctx->cur], 0, ctx->stream), "prim")) return s;
  if (gdg_status s = read_ctl(ctx)) return s;
  ctx->t = 0.0;
  ctx->steps = ctx->restarts = 0;
  ctx->last_dt = 0.0;
  if (ctx->hctl.bad_flag) {
    ctx->err = "uploaded state is not admissible (rho <= 0, eps <= 0 or NaN)";
    return GDG_E_INADMISSIBLE;
  }
  ctx->err.clear();
  return GDG_OK;
}

gdg_status gdg_download_state(gdg_ctx *ctx, double *U, int32_t is_device_ptr) {
  if (!ctx || !U) return GDG_E_INVALID;
  (void)is_device_ptr;
  const size_t bytes = (size_t)ctx->M * ctx->A.N * sizeof(double);
  HIPCHK(ctx, hipMemcpyAsync(U, ctx->U[ctx->cur], bytes, hipMemcpyDefault, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return GDG_OK;
}

}  // extern "C"

namespace {
constexpr int kMaxRestarts = 8;

// tau of a restarted step: stage vs found its Euler step tstep[vs] tau above
// its bound tau_max(u_vs); the new tau gives it Cr tau_max(u_vs).
double restart_tau(const gdg_ctx *ctx, const Ctl &h) {
  const int vs = h.viol_stage < 1 ? 1 : (h.viol_stage >= ctx->A.nst ? ctx->A.nst - 1 : h.viol_stage);
  return ctx->prm.cfl * bits_to_double(h.taumin_bits[vs]) / ctx->A.tstep[vs];
}

// One step of the integrator with the restart rule; `used` restarts of this step were
// already spent (a device-driven attempt that halted on a violation).
gdg_status step_impl(gdg_ctx *ctx, double dt_cap, double dt_fixed, double *dt_taken, int used) {
  double tau_fixed = dt_fixed > 0.0 ? dt_fixed : 0.0;
  for (int attempt = used; attempt <= kMaxRestarts; ++attempt) {
    if (gdg_status s = launched(ctx, enqueue_step(ctx, ctx->stream, 0, dt_cap, tau_fixed, prof_of(ctx)), "step"))
      return s;
    if (gdg_status s = read_ctl(ctx)) return s;
    if (gdg_status s = harvest(ctx)) return s;
    const Ctl &h = ctx->hctl;
    if (h.cfl_flag) {
      tau_fixed = restart_tau(ctx, h);
      ++ctx->restarts;
      continue;
    }
    if (h.bad_flag) return gdg::flag_status(ctx, h.bad_flag, "a stage output left the admissible set");
    ctx->last_dt = h.tau;
    sync_time(ctx);
    if (dt_taken) *dt_taken = h.tau;
    return GDG_OK;
  }
  ctx->err = "CFL condition violated after 8 restarts";
  return GDG_E_CFL;
}
}  // namespace

extern "C" {

gdg_status gdg_step(gdg_ctx *ctx, double dt_cap, double dt_fixed, double *dt_taken) {
  if (!ctx) return GDG_E_INVALID;
  return step_impl(ctx, dt_cap, dt_fixed, dt_taken, 0);
}

}  // extern "C"

namespace gdg {

// Device-driven time loop: kGraphSteps steps per round (a captured graph, or
// with use_graph = false the same launches enqueued directly), one host
// synchronization per round.  A CFL violation halts the rest of that round;
// the step is then redone on the host-driven path with its restart rule.
gdg_status run_loop(gdg_ctx *ctx, double t_final, int64_t max_steps, gdg_stats *stats, bool use_graph) {
  if (!ctx) return GDG_E_INVALID;
  if (max_steps <= 0 || !(ctx->t < t_final)) return gdg_get_stats(ctx, stats);
  const int64_t limit = ctx->steps + (max_steps > (int64_t(1) << 60) ? (int64_t(1) << 60) : max_steps);
  if (ctx->prof_on) {
    // HIP events recorded inside a graph carry no timestamps: with kernel
    // timing on, the same steps run host-driven.
    while (ctx->steps < limit && ctx->t < t_final) {
      double dt = 0.0;
      if (gdg_status s = gdg_step(ctx, t_final - ctx->t, 0.0, &dt)) return s;
    }
    return gdg_get_stats(ctx, stats);
  }
  if (use_graph)
    if (gdg_status s = ensure_graph(ctx)) return s;
  if (gdg_status s = launched(ctx, launch_set_run(ctx->A, t_final, limit, ctx->stream), "set run")) return s;
  for (;;) {
    if (use_graph) {
      HIPCHK(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
    } else {
      int rc = 0;
      for (int k = 0; k < kGraphSteps; ++k)
        rc |= enqueue_step(ctx, ctx->stream, 1, 0.0, 0.0, nullptr, k == 0, k + 1 == kGraphSteps);
      if (gdg_status s = launched(ctx, rc, "device-driven steps")) return s;
    }
    if (gdg_status s = read_ctl(ctx)) return s;
    const Ctl h = ctx->hctl;
    if (h.bad_flag) return gdg::flag_status(ctx, h.bad_flag, "a stage output left the admissible set");
    ctx->last_dt = h.tau;
    sync_time(ctx);
    if (h.cfl_flag) {
      const double tau = restart_tau(ctx, h);
      ++ctx->restarts;
      double dt = 0.0;
      if (gdg_status s = step_impl(ctx, t_final - ctx->t, tau, &dt, 1)) return s;
      if (ctx->steps >= limit || !(ctx->t < t_final)) break;
      if (gdg_status s = launched(ctx, launch_set_run(ctx->A, t_final, limit, ctx->stream), "set run")) return s;
      continue;
    }
    if (h.halt || ctx->steps >= limit || !(ctx->t < t_final)) break;
  }
  return gdg_get_stats(ctx, stats);
}

}  // namespace gdg

extern "C" {

gdg_status gdg_run_to(gdg_ctx *ctx, double t_final, int64_t max_steps, gdg_stats *stats) {
  return gdg::run_loop(ctx, t_final, max_steps, stats, true);
}

}  // extern "C"

namespace gdg {

const KArgs &ctx_kargs(const gdg_ctx *ctx) { return ctx->A; }

void ctx_stage_bufs(const gdg_ctx *ctx, StageBufs sb[3]) {
  const int c0 = ctx->cur, c1 = (c0 + 1) % 3, c2 = (c0 + 2) % 3;
  sb[0] = {ctx->U[c0], ctx->U[c1], ctx->U[c0], 0.0, 1.0};
  sb[1] = {ctx->U[c1], ctx->U[c2], ctx->U[c0], 0.75, 0.25};
  sb[2] = {ctx->U[c2], ctx->U[c0], ctx->U[c0], 1.0 / 3.0, 2.0 / 3.0};
}

int ctx_arm(gdg_ctx *ctx, double t_final) {
  return launch_set_run(ctx->A, t_final, (long long)(int64_t(1) << 60), ctx->stream);
}

void ctx_sync(gdg_ctx *ctx, const Ctl &c) {
  ctx->hctl = c;
  ctx->last_dt = c.tau;
  sync_time(ctx);
}

gdg_status ctx_restart(gdg_ctx *ctx, const Ctl &c, double t_final) {
  ctx_sync(ctx, c);
  const double tau = restart_tau(ctx, c);
  ++ctx->restarts;
  double dt = 0.0;
  if (gdg_status s = step_impl(ctx, t_final - ctx->t, tau, &dt, 1)) return s;
  return launched(ctx, ctx_arm(ctx, t_final), "set run");
}

const char *ctx_error(const gdg_ctx *ctx) { return ctx->err.c_str(); }

int ctx_launch_steps(gdg_ctx *ctx, void *stream) {
  if (ensure_graph(ctx) != GDG_OK) return -1;
  return hipGraphLaunch(ctx->graph_exec, (hipStream_t)stream) == hipSuccess ? 0 : -1;
}

const Ctl *ctx_dev_ctl(const gdg_ctx *ctx) { return ctx->A.ctl; }

void set_create_error(const std::string &msg) { g_create_err = msg; }

void ctx_counts(const gdg_ctx *ctx, double *t, int64_t *steps, int64_t *restarts) {
  *t = ctx->t;
  *steps = ctx->steps;
  *restarts = ctx->restarts;
}

gdg_status flag_status(gdg_ctx *ctx, int flag, const char *what) {
  if (flag & 2) {
    ctx->err = "subsonic normal flow at a node of a supersonic in/outflow face";
    return GDG_E_BOUNDARY;
  }
  ctx->err = what;
  return GDG_E_INADMISSIBLE;
}

}  // namespace gdg

extern "C" {

gdg_status gdg_stage(gdg_ctx *ctx, double tau, double *tau_used) {
  if (!ctx) return GDG_E_INVALID;
  const int c0 = ctx->cur, c1 = (c0 + 1) % 3;
  if (gdg_status s = launched(ctx, launch_begin(ctx->A, 0.0, tau > 0.0 ? tau : 0.0, 0, ctx->stream), "begin"))
    return s;
  StageBufs b = {ctx->U[c0], ctx->U[c1], ctx->U[c0], 0.0, 1.0};
  // one forward-Euler stage of size tau = Cr tau_max (or the given tau),
  // whatever the context's integrator
  KArgs A1 = ctx->A;
  set_integrator(A1, GDG_SSPRK3);
  if (gdg_status s = launched(ctx, launch_stage(A1, b, 0, ctx->stream, prof_of(ctx), 1), "stage")) return s;
  if (gdg_status s = read_ctl(ctx)) return s;
  if (gdg_status s = harvest(ctx)) return s;
  if (ctx->hctl.bad_flag) return gdg::flag_status(ctx, ctx->hctl.bad_flag, "the stage output left the admissible set");
  ctx->cur = c1;
  drop_graph(ctx);  // the captured graph names the old buffer roles
  // the node records of the next stage input: the step counter did not move,
  // so the next step reads the buffer this stage read
  if (gdg_status s = launched(ctx, launch_prim(ctx->A, ctx->U[ctx->cur], 0, ctx->stream), "prim")) return s;
  if (tau_used) *tau_used = ctx->hctl.tau;
  return GDG_OK;
}

gdg_status gdg_read_field(gdg_ctx *ctx, int32_t field, double *dst, int32_t is_device_ptr) {
  if (!ctx || !dst) return GDG_E_INVALID;
  (void)is_device_ptr;
  const size_t N = (size_t)ctx->A.N, M = (size_t)ctx->M;
  if (field == GDG_FIELD_STATE) {
    HIPCHK(ctx, hipMemcpyAsync(dst, ctx->U[ctx->cur], M * N * sizeof(double), hipMemcpyDefault, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return GDG_OK;
  }
  // the other fields sit in per-dof records: plane k is the column at
  // `first + k` of records of `stride` doubles
  const double *rec = nullptr;
  size_t planes = 0, first = 0, stride = 0;
  switch (field) {
    case GDG_FIELD_EV_N: rec = ctx->A.Qd; stride = kQStride; first = 3; planes = 1; break;
    case GDG_FIELD_BOUNDS: rec = ctx->A.Ld; stride = kLimStride; first = 2 * M; planes = 3; break;
    case GDG_FIELD_UL: rec = ctx->A.Ld; stride = kLimStride; first = M; planes = M; break;
    case GDG_FIELD_DUH: rec = ctx->A.Ld; stride = kLimStride; first = 0; planes = M; break;
    case GDG_FIELD_U1: rec = ctx->A.U1d; stride = kU1Stride; first = 0; planes = M; break;
    default: ctx->err = "unknown field"; return GDG_E_INVALID;
  }
  for (size_t k = 0; k < planes; ++k)
    HIPCHK(ctx, hipMemcpy2DAsync(dst + k * N, sizeof(double), rec + first + k, stride * sizeof(double),
                                 sizeof(double), N, hipMemcpyDefault, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return GDG_OK;
}

gdg_status gdg_get_stats(gdg_ctx *ctx, gdg_stats *stats) {
  if (!ctx) return GDG_E_INVALID;
  if (!stats) return GDG_OK;
  std::memset(stats, 0, sizeof *stats);
  stats->t = ctx->t;
  stats->steps = ctx->steps;
  stats->restarts = ctx->restarts;
  stats->last_dt = ctx->last_dt;
  double r[kRedFields];
  if (gdg_status s = launched(ctx, launch_state_stats(ctx->A, ctx->U[ctx->cur], ctx->stream), "state statistics"))
    return s;
  HIPCHK(ctx, hipMemcpyAsync(r, ctx->A.red + (size_t)kRedBlocks * kRedFields, sizeof r, hipMemcpyDeviceToHost,
                             ctx->stream));
  if (gdg_status s = read_ctl(ctx)) return s;  // also waits for the copy above
  stats->min_rho = r[0];
  stats->min_eps = r[1];
  for (int c = 0; c < ctx->M; ++c) stats->total[c] = r[2 + c];
  stats->bound_violations = (int64_t)ctx->hctl.bound_violations;
  stats->limited_pairs = (int64_t)ctx->hctl.limited_pairs;
  stats->quiet_rows = (int64_t)ctx->hctl.quiet_rows;
  return GDG_OK;
}

gdg_status gdg_profile(gdg_ctx *ctx, int32_t enable) {
  if (!ctx) return GDG_E_INVALID;
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (enable && !ctx->prof_on) {
    if (gdg_status s = make_events(ctx, ctx->prof_ev, ctx->prof_kid, 32, ctx->prof)) return s;
    ctx->prof_on = true;
  } else if (!enable && ctx->prof_on) {
    free_events(ctx->prof_ev);
    ctx->prof_on = false;
  }
  for (int k = 0; k < KID_COUNT; ++k) {
    ctx->prof_ms[k] = 0.0;
    ctx->prof_launches[k] = 0;
  }
  return GDG_OK;
}

gdg_status gdg_profile_read(const gdg_ctx *ctx, double *ms_total, int64_t *launches) {
  if (!ctx || !ms_total || !launches) return GDG_E_INVALID;
  for (int k = 0; k < KID_COUNT; ++k) {
    ms_total[k] = ctx->prof_ms[k];
    launches[k] = ctx->prof_launches[k];
  }
  return GDG_OK;
}

const char *gdg_last_error(const gdg_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

}  // extern "C"
