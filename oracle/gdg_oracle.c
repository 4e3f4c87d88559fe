/*
 * gdg_oracle.c -- plain CPU FP64 oracle for the graph-based DG scheme of
 * Kronbichler, Maier & Tomas, "Graph-based methods for hyperbolic systems of
 * conservation laws using discontinuous space discretizations" (arXiv 2402.04514).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, literal reference that the
 * GPU library is checked against.  Only the tests, the smoke check and the
 * bench's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * Everything is double precision and written in the order the paper states
 * the method: setup (Sec. 2.3), low-order update (Sec. 3, eq. cijdijscheme,
 * dij_low_order), boundary data (Sec. 4), high-order update with entropy
 * viscosity (Sec. 5.1-5.2), algebraic reformulation (Sec. 5.3) and convex
 * limiting (Sec. 5.4), inside SSP-RK3 or SSPRK(5,4) (Sec. 6.2).  Sums over a stencil run in
 * stored CSR order.  Where the paper is silent or garbled the reading used is
 * named in a comment ("reading R<n>"); the list of readings is kept with the
 * design notes of the repository.
 *
 * Parity of the limited scheme's absolute values (N_i, d^H, l_ij, U^{n+1}) is
 * unpinned by any printed example: the paper prints none.  Those values are
 * pinned only through the invariants tested in tests/ (conservation, bounds,
 * identities, limits l=0 / l=1, exact solutions).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXD 3
#define OR_MAXM 5
#define OR_PI 3.14159265358979323846

enum { OR_BC_PERIODIC = 0, OR_BC_OUTFLOW = 1, OR_BC_SLIP = 2, OR_BC_DIRICHLET = 3, OR_BC_SUPERSONIC = 4,
       OR_BC_INOUTFLOW = 5 };
enum { OR_LOW_ORDER = 0, OR_HIGH_ORDER = 1, OR_LIMITED = 2 };
enum { OR_KIND_CELL = 0, OR_KIND_FACE_COLLOC = 1, OR_KIND_FACE = 2 };

typedef struct {
  double gamma;   /* ratio of specific heats */
  double cfl;     /* Cr of eq. MaxCFLdt */
  double c_ev;    /* entropy-viscosity constant (Sec. 5.2) */
  double c_k;     /* minimal-viscosity constant (eq. ViscMin) */
  double c_r;     /* relaxation constant (eq. ViscMinConst2) */
  double p_r;     /* relaxation power (eq. ViscMinConst2) */
  int passes;     /* limiter passes (Sec. 6.1: two) */
  int scheme;     /* OR_LOW_ORDER / OR_HIGH_ORDER / OR_LIMITED */
  int integrator; /* 0: SSP-RK3; 1: SSPRK(5,4) (Sec. 6.2's fourth-order runs) */
} or_params;

typedef struct {
  int dim, deg, nb1, nloc, m;
  long n[3];
  double lo[3], hi[3], h[3];
  int bc[6];
  double bstate[6][OR_MAXM];  /* Dirichlet data U^d per box face (Sec. 4.1) */
  /* Dirichlet data from the isentropic vortex of Sec. 6.2 instead (2D):
   * beta, x0 (2), u_inf (2), gamma of the data; evaluated at the node and the
   * stage time */
  int vortex_data;
  /* strategy (d) of Sec. 6.3: the data of every Dirichlet-type face are the
   * node's own state at the start of the step, U^n_i, kept here by the step
   * (and by a single stage: its input) */
  int step_start_data;
  double *un;
  double vortex[6];
  double t0;                  /* time at the start of the step (boundary data) */
  long ncells, ndofs;
  double vol;
  /* CSR of the stencil I(i), diagonal included (reading R4) */
  long *rowptr;
  long *col;
  double *c;     /* nnz * dim */
  double *mij;   /* nnz; zero outside the cell */
  int *kind;     /* OR_KIND_* */
  double *mi;    /* lumped mass, eq. mass_matrices */
  /* boundary parts per row (Sec. 4.2): face id, c_i^{d,k}, boundary kind */
  long *bptr;
  int *bface;
  int *bkind;    /* boundary kind of each boundary part: bc[bface], or the
                    part's own kind (or_set_boundary_kinds) */
  double *bc_c;  /* nbnd * dim */
  /* reference tables */
  double xg[4];  /* Gauss-Lobatto nodes on [0,1] */
  int nq;
  double xq[8], wq[8]; /* Gauss-Legendre rule on [0,1] */
  /* general (non-affine) cells: the vertices of the cell lattice,
   * (n_0+1)(n_1+1)(n_2+1) points of dim coordinates, x fastest; every cell is
   * the multilinear image of the reference cell through its 2^dim corners.
   * NULL: the uniform box lo .. hi. */
  double *vx;
  int mapdeg;    /* general cells: degree g of the cell map (1 multilinear, 2 quadratic) */
  /* continuous elements (App. B): one dof per lattice node of the box, gn[e]
   * nodes per axis, their coordinates */
  int cg;
  long gn[3];
  double *cgx;
  /* unstructured meshes: the (mapdeg+1)^dim point ids of each cell, the
   * neighbour across each local face (-1: boundary) and its local face, and
   * per boundary face its kind | data face << 3 */
  long *ucp, *unb;
  int *unf;
  signed char *ubc;
} or_setup;

/* ------------------------------------------------------------------------ */
/* 1D reference element: Lagrange basis on Gauss-Lobatto nodes (Sec. 2.3).   */
/* ------------------------------------------------------------------------ */

static double lag(const or_setup *S, int a, double x) {
  double v = 1.0;
  for (int b = 0; b < S->nb1; ++b)
    if (b != a) v *= (x - S->xg[b]) / (S->xg[a] - S->xg[b]);
  return v;
}

static double dlag(const or_setup *S, int a, double x) {
  double s = 0.0;
  for (int c = 0; c < S->nb1; ++c) {
    if (c == a) continue;
    double t = 1.0 / (S->xg[a] - S->xg[c]);
    for (int b = 0; b < S->nb1; ++b)
      if (b != a && b != c) t *= (x - S->xg[b]) / (S->xg[a] - S->xg[b]);
    s += t;
  }
  return s;
}

static void local_multi(const or_setup *S, int a, int *ai) {
  for (int e = 0; e < 3; ++e) { ai[e] = a % S->nb1; a /= S->nb1; }
}

static void cell_multi(const or_setup *S, long K, long *ki) {
  for (int e = 0; e < 3; ++e) {
    long ne = e < S->dim ? S->n[e] : 1;
    ki[e] = K % ne;
    K /= ne;
  }
}

static long cell_index(const or_setup *S, const long *ki) {
  long K = 0, stride = 1;
  for (int e = 0; e < S->dim; ++e) { K += ki[e] * stride; stride *= S->n[e]; }
  return K;
}

/* Neighbour of cell K across face f = 2e+side; -1 on a non-periodic boundary. */
static long neighbour(const or_setup *S, long K, int f) {
  if (S->ucp) return S->unb[K * 2 * S->dim + f];
  int e = f / 2, side = f % 2;
  long ki[3];
  cell_multi(S, K, ki);
  ki[e] += side ? 1 : -1;
  if (ki[e] < 0 || ki[e] >= S->n[e]) {
    if (S->bc[f] != OR_BC_PERIODIC) return -1;
    ki[e] = (ki[e] + S->n[e]) % S->n[e];
  }
  return cell_index(S, ki);
}

/* ------------------------------------------------------------------------ */
/* General cells: the multilinear map of cell K and the integrals of Sec. 2.3 */
/* written with its Jacobian (change of variables x = F_K(xi)).               */
/* ------------------------------------------------------------------------ */

/* Quadratic Lagrange basis on the points 0, 1/2, 1 of [0, 1]: value and
 * derivative of the one at point q. */
static double lag2(int q, double t) {
  return q == 0 ? 2.0 * (t - 0.5) * (t - 1.0) : (q == 1 ? -4.0 * t * (t - 1.0) : 2.0 * t * (t - 0.5));
}
static double lag2d(int q, double t) { return q == 0 ? 4.0 * t - 3.0 : (q == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0); }

/* Point q (q_e in 0 .. mapdeg per axis) of cell K's map: from the cell's own
 * list on unstructured meshes, else from the point lattice of mapdeg n_e + 1
 * points per axis. */
static const double *map_point(const or_setup *S, long K, const int *q) {
  const int g = S->mapdeg, dim = S->dim;
  if (S->ucp) {
    long v = 0, st = 1;
    for (int e = 0; e < dim; ++e) { v += q[e] * st; st *= g + 1; }
    return S->vx + S->ucp[K * st + v] * dim;
  }
  long ki[3];
  cell_multi(S, K, ki);
  long vi = 0, stride = 1;
  for (int e = 0; e < dim; ++e) { vi += (g * ki[e] + q[e]) * stride; stride *= g * S->n[e] + 1; }
  return S->vx + vi * dim;
}

/* x = F_K(xi) and J[r][c] = dx_r / dxi_c.  Degree 1: the multilinear map,
 * sum over the corners v of X_v prod_e (xi_e if bit e of v else 1 - xi_e).
 * Degree 2: the tensor-product quadratic map through the 3^d points of the
 * cell on the point lattice of 2 n_e + 1 points per axis (corners, edge and
 * face midpoints, centre), each weighted by prod_e lag2(q_e, xi_e). */
static void cell_map(const or_setup *S, long K, const double *xi, double *x, double J[3][3]) {
  const int dim = S->dim;
  for (int r = 0; r < 3; ++r) {
    x[r] = 0.0;
    for (int c = 0; c < 3; ++c) J[r][c] = 0.0;
  }
  if (S->mapdeg == 2) {
    int npt = 1;
    for (int e = 0; e < dim; ++e) npt *= 3;
    for (int v = 0; v < npt; ++v) {
      int q[3] = {0, 0, 0}, r = v;
      for (int e = 0; e < dim; ++e) { q[e] = r % 3; r /= 3; }
      double w = 1.0, dw[3];
      for (int e = 0; e < dim; ++e) w *= lag2(q[e], xi[e]);
      for (int c = 0; c < dim; ++c) {
        dw[c] = 1.0;
        for (int e = 0; e < dim; ++e) dw[c] *= e == c ? lag2d(q[e], xi[e]) : lag2(q[e], xi[e]);
      }
      const double *X = map_point(S, K, q);
      for (int rr = 0; rr < dim; ++rr) {
        x[rr] += w * X[rr];
        for (int c = 0; c < dim; ++c) J[rr][c] += dw[c] * X[rr];
      }
    }
    return;
  }
  for (int v = 0; v < (1 << dim); ++v) {
    int q[3] = {0, 0, 0};
    double w = 1.0, dw[3];
    for (int e = 0; e < dim; ++e) {
      int bit = (v >> e) & 1;
      q[e] = bit;
      w *= bit ? xi[e] : 1.0 - xi[e];
    }
    for (int c = 0; c < dim; ++c) {
      dw[c] = 1.0;
      for (int e = 0; e < dim; ++e) {
        int bit = (v >> e) & 1;
        if (e == c) dw[c] *= bit ? 1.0 : -1.0;
        else dw[c] *= bit ? xi[e] : 1.0 - xi[e];
      }
    }
    const double *X = map_point(S, K, q);
    for (int r = 0; r < dim; ++r) {
      x[r] += w * X[r];
      for (int c = 0; c < dim; ++c) J[r][c] += dw[c] * X[r];
    }
  }
}

/* det J and Ji = J^{-1} (dim 1, 2 or 3). */
static double inverse(int dim, double J[3][3], double Ji[3][3]) {
  double det;
  if (dim == 1) {
    det = J[0][0];
    Ji[0][0] = 1.0 / det;
    return det;
  }
  if (dim == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
    return det;
  }
  det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      /* the cofactor of J[c][r] over det */
      int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
      Ji[r][c] = (J[r1][c1] * J[r2][c2] - J[r1][c2] * J[r2][c1]) / det;
    }
  return det;
}

static double phi(const or_setup *S, int a, const double *xi);

/* Reference gradient d phi_a / d xi. */
static void grad_ref(const or_setup *S, int a, const double *xi, double *g) {
  int ai[3];
  local_multi(S, a, ai);
  for (int c = 0; c < S->dim; ++c) {
    double v = 1.0;
    for (int e = 0; e < S->dim; ++e) v *= (e == c) ? dlag(S, ai[e], xi[e]) : lag(S, ai[e], xi[e]);
    g[c] = v;
  }
}

/* Over general cell K, by the tensor Gauss rule: kind 0 m_ab = int phi_a
 * phi_b, kind 1 int phi_a grad phi_b (out[0 .. dim)), kind 2 int phi_a; with
 * grad phi = J^{-T} grad_xi phi and dx = det J dxi. */
static void cell_integral_mapped(const or_setup *S, long K, int kind, int a, int b, double *out) {
  const int dim = S->dim, nq = S->nq;
  int tot = 1;
  for (int e = 0; e < dim; ++e) tot *= nq;
  for (int e = 0; e < 3; ++e) out[e] = 0.0;
  for (int q = 0; q < tot; ++q) {
    double xi[3] = {0, 0, 0}, w = 1.0;
    int r = q;
    for (int e = 0; e < dim; ++e) { xi[e] = S->xq[r % nq]; w *= S->wq[r % nq]; r /= nq; }
    double x[3], J[3][3], Ji[3][3];
    cell_map(S, K, xi, x, J);
    const double det = inverse(dim, J, Ji);
    const double pa = phi(S, a, xi);
    if (kind == 0) out[0] += w * pa * phi(S, b, xi) * det;
    else if (kind == 2) out[0] += w * pa * det;
    else {
      double g[3];
      grad_ref(S, b, xi, g);
      for (int e = 0; e < dim; ++e) {
        double ge = 0.0;
        for (int c = 0; c < dim; ++c) ge += Ji[c][e] * g[c];
        out[e] += w * pa * ge * det;
      }
    }
  }
}

/* Over face f = 2e + side of general cell K: int_F phi_a phi_b n ds (out[0 ..
 * dim)), n the outward unit normal of K; phi_b of the same cell or of the
 * neighbour across f (its reference coordinate e is 1 - side), b < 0 meaning 1.
 * n ds = (outward sign) det J J^{-T} e_e dxi over the face (Nanson's formula). */
/* The reference point eta of cell K with F_K(eta) = x, by Newton's method
 * from the cell's centre (used for points on the cell's boundary). */
static void map_inverse(const or_setup *S, long K, const double *x, double *eta) {
  const int dim = S->dim;
  for (int e = 0; e < 3; ++e) eta[e] = e < dim ? 0.5 : 0.0;
  for (int it = 0; it < 60; ++it) {
    double y[3], J[3][3], Ji[3][3], dmax = 0.0;
    cell_map(S, K, eta, y, J);
    inverse(dim, J, Ji);
    double d[3] = {0, 0, 0};
    for (int r = 0; r < dim; ++r)
      for (int c = 0; c < dim; ++c) d[r] += Ji[r][c] * (x[c] - y[c]);
    for (int r = 0; r < dim; ++r) { eta[r] += d[r]; dmax = fmax(dmax, fabs(d[r])); }
    if (dmax < 1e-15) break;
  }
}

/* Whether local node b of cell Kn lies on the face that Kn shares with cell
 * K across K's face f (lattice: the opposite face; unstructured: the
 * neighbour's own local face). */
static int on_shared_face(const or_setup *S, long K, int f, int b) {
  int bi[3];
  local_multi(S, b, bi);
  if (S->ucp) {
    int fn = S->unf[K * 2 * S->dim + f];
    return bi[fn / 2] == (fn % 2) * S->deg;
  }
  return bi[f / 2] == (1 - f % 2) * S->deg;
}

static void face_integral_mapped(const or_setup *S, long K, int f, int a, int b, int same_cell, double *out) {
  const int dim = S->dim, nq = S->nq, e = f / 2, side = f % 2;
  int tot = 1;
  for (int d = 0; d < dim - 1; ++d) tot *= nq;
  for (int d = 0; d < 3; ++d) out[d] = 0.0;
  for (int q = 0; q < tot; ++q) {
    double xi[3] = {0, 0, 0}, w = 1.0;
    int r = q;
    for (int d = 0; d < dim; ++d) {
      if (d == e) { xi[d] = side ? 1.0 : 0.0; continue; }
      xi[d] = S->xq[r % nq]; w *= S->wq[r % nq]; r /= nq;
    }
    double x[3], J[3][3], Ji[3][3];
    cell_map(S, K, xi, x, J);
    const double det = inverse(dim, J, Ji);
    double va = phi(S, a, xi), vb = 1.0;
    if (b >= 0) {
      double xb[3] = {xi[0], xi[1], xi[2]};
      if (!same_cell && S->ucp) {
        /* b belongs to the neighbour: its reference point of x, on its face */
        const long Kn = S->unb[K * 2 * dim + f];
        const int fn = S->unf[K * 2 * dim + f];
        map_inverse(S, Kn, x, xb);
        xb[fn / 2] = (fn % 2) ? 1.0 : 0.0;
      } else if (!same_cell) {
        xb[e] = 1.0 - xi[e];
      }
      vb = phi(S, b, xb);
    }
    const double sgn = side ? 1.0 : -1.0;
    for (int d = 0; d < dim; ++d) out[d] += w * va * vb * sgn * det * Ji[e][d];
  }
}

/* Tensor-product basis value / gradient at reference point xi of the cell. */
static double phi(const or_setup *S, int a, const double *xi) {
  int ai[3];
  local_multi(S, a, ai);
  double v = 1.0;
  for (int e = 0; e < S->dim; ++e) v *= lag(S, ai[e], xi[e]);
  return v;
}

static double dphi(const or_setup *S, int a, int dir, const double *xi) {
  int ai[3];
  local_multi(S, a, ai);
  double v = 1.0;
  for (int e = 0; e < S->dim; ++e)
    v *= (e == dir) ? dlag(S, ai[e], xi[e]) / S->h[e] : lag(S, ai[e], xi[e]);
  return v;
}

/* Cell quadrature: calls fn at every tensor Gauss point with weight w*|K|. */
typedef struct { int a, b, dir; } pair_arg;

static double cell_integral(const or_setup *S, int kind, pair_arg p) {
  /* kind 0: m_ab = int phi_a phi_b ; kind 1: int d_dir phi_b phi_a ; kind 2: int phi_a */
  double jac = 1.0;
  for (int e = 0; e < S->dim; ++e) jac *= S->h[e];
  int nq = S->nq, tot = 1;
  for (int e = 0; e < S->dim; ++e) tot *= nq;
  double sum = 0.0;
  for (int q = 0; q < tot; ++q) {
    double xi[3] = {0, 0, 0}, w = 1.0;
    int r = q;
    for (int e = 0; e < S->dim; ++e) { xi[e] = S->xq[r % nq]; w *= S->wq[r % nq]; r /= nq; }
    double g;
    if (kind == 0) g = phi(S, p.a, xi) * phi(S, p.b, xi);
    else if (kind == 1) g = dphi(S, p.b, p.dir, xi) * phi(S, p.a, xi);
    else g = phi(S, p.a, xi);
    sum += w * g;
  }
  return sum * jac;
}

/* Face integral over face f of a cell: int_F phi_a^(A) phi_b^(B) ds where
 * phi_b is either a basis function of the same cell (same_cell = 1) or of the
 * neighbour across f (conforming uniform cells: the neighbour's reference
 * coordinate normal to the face is 1 - side).  b < 0 means "phi_b = 1". */
static double face_integral(const or_setup *S, int f, int a, int b, int same_cell) {
  int e = f / 2, side = f % 2;
  double area = 1.0;
  for (int d = 0; d < S->dim; ++d) if (d != e) area *= S->h[d];
  int nq = S->nq, tot = 1;
  for (int d = 0; d < S->dim - 1; ++d) tot *= nq;
  double sum = 0.0;
  for (int q = 0; q < tot; ++q) {
    double xi[3] = {0, 0, 0}, w = 1.0;
    int r = q;
    for (int d = 0; d < S->dim; ++d) {
      if (d == e) { xi[d] = side ? 1.0 : 0.0; continue; }
      xi[d] = S->xq[r % nq]; w *= S->wq[r % nq]; r /= nq;
    }
    double va = phi(S, a, xi), vb = 1.0;
    if (b >= 0) {
      double xb[3] = {xi[0], xi[1], xi[2]};
      if (!same_cell) xb[e] = 1.0 - xi[e];
      vb = phi(S, b, xb);
    }
    sum += w * va * vb;
  }
  return sum * area;
}

/* c_ij written out from eq. cij_def1 / cij_def2 for one ordered pair. */
static void literal_cij(const or_setup *S, long i, long j, double *out) {
  long Ki = i / S->nloc, Kj = j / S->nloc;
  int a = (int)(i % S->nloc), b = (int)(j % S->nloc);
  int ai[3], bi[3];
  local_multi(S, a, ai);
  local_multi(S, b, bi);
  for (int e = 0; e < S->dim; ++e) out[e] = 0.0;
  if (S->vx) {
    /* general cells: the same definitions with vector-valued face normals */
    double t[3];
    if (Ki == Kj) {
      cell_integral_mapped(S, Ki, 1, a, b, out);
      for (int f = 0; f < 2 * S->dim; ++f) {
        face_integral_mapped(S, Ki, f, a, b, 1, t);
        for (int e = 0; e < S->dim; ++e) out[e] -= 0.5 * t[e];
      }
      return;
    }
    for (int f = 0; f < 2 * S->dim; ++f) {
      int e = f / 2, side = f % 2;
      if (ai[e] != side * S->deg) continue;
      if (neighbour(S, Ki, f) != Kj) continue;
      if (!on_shared_face(S, Ki, f, b)) continue;
      face_integral_mapped(S, Ki, f, a, b, 0, t);
      for (int d = 0; d < S->dim; ++d) out[d] = 0.5 * t[d];
      return;
    }
    return;
  }
  if (Ki == Kj) {
    for (int e = 0; e < S->dim; ++e) {
      pair_arg p = {a, b, e};
      double cK = cell_integral(S, 1, p);
      /* c^{dK}: half the boundary integral over all faces of K, outward n */
      double cdK = 0.0;
      for (int side = 0; side < 2; ++side) {
        int f = 2 * e + side;
        double n = side ? 1.0 : -1.0;
        cdK += 0.5 * n * face_integral(S, f, a, b, 1);
      }
      out[e] = cK - cdK;
    }
    return;
  }
  /* different cells: the face of K_i shared with K_j that carries both nodes */
  for (int f = 0; f < 2 * S->dim; ++f) {
    int e = f / 2, side = f % 2;
    if (ai[e] != side * S->deg) continue;
    if (bi[e] != (1 - side) * S->deg) continue;
    if (neighbour(S, Ki, f) != Kj) continue;
    double n = side ? 1.0 : -1.0;
    out[e] = 0.5 * n * face_integral(S, f, a, b, 0);
    return;
  }
}

/* Reading R3: c_ji is stored as exactly -c_ij, the pair evaluated from the
 * lower index; c_ii = 0 (Lemma PropSkew). */
static void canonical_cij(const or_setup *S, long i, long j, double *out) {
  if (i == j) { for (int e = 0; e < S->dim; ++e) out[e] = 0.0; return; }
  if (i < j) { literal_cij(S, i, j, out); return; }
  literal_cij(S, j, i, out);
  for (int e = 0; e < S->dim; ++e) out[e] = -out[e];
}

void or_destroy(or_setup *S) {
  if (!S) return;
  free(S->rowptr); free(S->col); free(S->c); free(S->mij); free(S->kind); free(S->mi);
  free(S->bptr); free(S->bface); free(S->bkind); free(S->bc_c); free(S->vx);
  free(S->ucp); free(S->unb); free(S->unf); free(S->ubc); free(S->cgx); free(S->un);
  free(S);
}

/* Gauss-Legendre rule of n points on [0, 1]: the roots of the Legendre
 * polynomial P_n by Newton's method from the Chebyshev guesses, P_n and its
 * derivative by the three-term recurrence; weights 2 / ((1 - x^2) P_n'(x)^2)
 * on [-1, 1], halved on [0, 1]. */
static void gauss_rule(int n, double *x01, double *w01) {
  for (int k = 0; k < n; ++k) {
    double x = cos(OR_PI * (k + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = x;
      for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * x * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0);
    }
    x01[n - 1 - k] = 0.5 * (1.0 + x);
    w01[n - 1 - k] = 1.0 / ((1.0 - x * x) * dp * dp);
  }
}

static or_setup *setup_init(int dim, int deg, const long *cells, const double *lo, const double *hi, const int *bc);
static void setup_build(or_setup *S);
static void node_x(const or_setup *S, long i, double *x);

/* Setup: GL nodes, cell-major numbering, m_ij, m_i, c_ij, c_i^{d,k} (Sec. 2.3,
 * Sec. 4.2).  Exact Gauss-Legendre integration with k+1 points (reading R5). */
or_setup *or_create(int dim, int deg, const long *cells, const double *lo, const double *hi,
                    const int *bc) {
  or_setup *S = setup_init(dim, deg, cells, lo, hi, bc);
  if (S) setup_build(S);
  return S;
}

/* The same on general cells: vx holds the (n_0+1)(n_1+1)(n_2+1) vertices of
 * the cell lattice (dim coordinates each, x fastest; on a periodic axis the
 * last layer is the first one shifted by the period).  The integrals use the
 * Gauss rule of k + 2 points (exact for the multilinear maps' polynomial
 * integrands); |Omega| is the sum of the cells' volumes.  NULL if a cell's
 * Jacobian determinant is not positive at a node or a Gauss point. */
/* General cells with a cell map of degree mapdeg (1: the lattice of
 * n_e + 1 points per axis, multilinear cells; 2: 2 n_e + 1 points per axis,
 * quadratic (curved) cells). */
static or_setup *finish_general(or_setup *S);
void or_destroy(or_setup *S);

or_setup *or_create_curved(int dim, int deg, const long *cells, const double *vx, const int *bc, int mapdeg) {
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  if (mapdeg != 1 && mapdeg != 2) return NULL;
  or_setup *S = setup_init(dim, deg, cells, lo, hi, bc);
  if (!S) return NULL;
  S->mapdeg = mapdeg;
  long nv = 1;
  for (int e = 0; e < dim; ++e) nv *= mapdeg * S->n[e] + 1;
  S->vx = (double *)malloc(nv * dim * sizeof(double));
  memcpy(S->vx, vx, nv * dim * sizeof(double));
  return finish_general(S);
}

/* The quadrature, the admissibility of every cell (det J > 0 at the nodes
 * and quadrature points), |Omega| and the stencil of general cells. */
static or_setup *finish_general(or_setup *S) {
  const int dim = S->dim, deg = S->deg, mapdeg = S->mapdeg;
  /* a rule exact for the integrands: products of the basis with det J or
   * with the cofactors, of degree at most 2 deg + 3 mapdeg - 1 per direction */
  S->nq = deg + 2 + (mapdeg == 2 ? 2 : 0);
  gauss_rule(S->nq, S->xq, S->wq);
  /* admissible cells, and the volume */
  double vol = 0.0;
  for (long K = 0; K < S->ncells; ++K) {
    double t[3];
    cell_integral_mapped(S, K, 2, 0, 0, t);
    for (int a = 0; a < S->nloc; ++a) {
      int ai[3];
      local_multi(S, a, ai);
      double xi[3] = {0, 0, 0}, x[3], J[3][3], Ji[3][3];
      for (int e = 0; e < dim; ++e) xi[e] = S->xg[ai[e]];
      cell_map(S, K, xi, x, J);
      if (!(inverse(dim, J, Ji) > 0.0)) { or_destroy(S); return NULL; }
    }
    int tot = 1;
    for (int e = 0; e < dim; ++e) tot *= S->nq;
    for (int q = 0; q < tot; ++q) {
      double xi[3] = {0, 0, 0}, w = 1.0, x[3], J[3][3], Ji[3][3];
      int r = q;
      for (int e = 0; e < dim; ++e) { xi[e] = S->xq[r % S->nq]; w *= S->wq[r % S->nq]; r /= S->nq; }
      cell_map(S, K, xi, x, J);
      const double det = inverse(dim, J, Ji);
      if (!(det > 0.0)) { or_destroy(S); return NULL; }
      vol += w * det;
    }
  }
  S->vol = vol;
  setup_build(S);
  return S;
}

or_setup *or_create_mapped(int dim, int deg, const long *cells, const double *vx, const int *bc) {
  return or_create_curved(dim, deg, cells, vx, bc, 1);
}

/* Unstructured meshes: ncells cells, cell K the image of the reference cell
 * under the map of degree mapdeg through the points pts[cell_pts[K (g+1)^dim
 * + v]] (v: digits q_e in base g + 1, the first axis lowest).  Two cells are
 * neighbours across the faces whose corner points are the same set; a face
 * without a neighbour is a boundary part with kind ubc[K 2 dim + f] & 7 and
 * the data of face ubc >> 3.  NULL for a face shared by more than two cells,
 * bad kinds or a non-positive Jacobian. */
typedef struct { long key[4]; long K; int f; } or_facekey;
static int facekey_cmp(const void *pa, const void *pb) {
  const or_facekey *a = (const or_facekey *)pa, *b = (const or_facekey *)pb;
  for (int k = 0; k < 4; ++k)
    if (a->key[k] != b->key[k]) return a->key[k] < b->key[k] ? -1 : 1;
  return 0;
}
static int long_cmp(const void *pa, const void *pb) {
  long a = *(const long *)pa, b = *(const long *)pb;
  return a < b ? -1 : (a > b);
}

or_setup *or_create_unstructured(int dim, int deg, long ncells, const long *cell_pts, long npts, const double *pts,
                                 int mapdeg, const signed char *ubc) {
  if ((mapdeg != 1 && mapdeg != 2) || ncells < 1 || dim < 2) return NULL;
  long cells[3] = {ncells, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  int bc[6] = {1, 1, 1, 1, 1, 1};
  or_setup *S = setup_init(dim, deg, cells, lo, hi, bc);
  if (!S) return NULL;
  S->mapdeg = mapdeg;
  int np = 1;
  for (int e = 0; e < dim; ++e) np *= mapdeg + 1;
  S->ucp = (long *)malloc(ncells * np * sizeof(long));
  memcpy(S->ucp, cell_pts, ncells * np * sizeof(long));
  S->vx = (double *)malloc(npts * dim * sizeof(double));
  memcpy(S->vx, pts, npts * dim * sizeof(double));
  S->ubc = (signed char *)malloc(ncells * 2 * dim);
  memcpy(S->ubc, ubc, ncells * 2 * dim);
  S->unb = (long *)malloc(ncells * 2 * dim * sizeof(long));
  S->unf = (int *)malloc(ncells * 2 * dim * sizeof(int));
  for (long q = 0; q < ncells * np; ++q)
    if (S->ucp[q] < 0 || S->ucp[q] >= npts) { or_destroy(S); return NULL; }
  /* faces keyed by their sorted corner point ids */
  const long nf = ncells * 2 * dim;
  or_facekey *fk = (or_facekey *)malloc(nf * sizeof(or_facekey));
  for (long K = 0; K < ncells; ++K)
    for (int f = 0; f < 2 * dim; ++f) {
      or_facekey *k = &fk[K * 2 * dim + f];
      int nc = 0;
      for (int v = 0; v < (1 << dim); ++v) {
        if (((v >> (f / 2)) & 1) != f % 2) continue;
        long idx = 0, st = 1;
        for (int e = 0; e < dim; ++e) { idx += ((v >> e) & 1) * mapdeg * st; st *= mapdeg + 1; }
        k->key[nc++] = S->ucp[K * np + idx];
      }
      for (int c = nc; c < 4; ++c) k->key[c] = -1;
      qsort(k->key, nc, sizeof(long), long_cmp);
      k->K = K;
      k->f = f;
      S->unb[K * 2 * dim + f] = -1;
      S->unf[K * 2 * dim + f] = -1;
    }
  qsort(fk, nf, sizeof(or_facekey), facekey_cmp);
  int bad = 0;
  for (long q = 0; q < nf;) {
    long r = q + 1;
    while (r < nf && facekey_cmp(&fk[q], &fk[r]) == 0) ++r;
    if (r - q == 2) {
      S->unb[fk[q].K * 2 * dim + fk[q].f] = fk[q + 1].K;
      S->unf[fk[q].K * 2 * dim + fk[q].f] = fk[q + 1].f;
      S->unb[fk[q + 1].K * 2 * dim + fk[q + 1].f] = fk[q].K;
      S->unf[fk[q + 1].K * 2 * dim + fk[q + 1].f] = fk[q].f;
    } else if (r - q == 1) {
      const signed char u = S->ubc[fk[q].K * 2 * dim + fk[q].f];
      if (u < 0 || (u & 7) < OR_BC_OUTFLOW || (u & 7) > OR_BC_INOUTFLOW || (u >> 3) > 5) bad = 1;
    } else {
      bad = 1;
    }
    q = r;
  }
  free(fk);
  if (bad) { or_destroy(S); return NULL; }
  return finish_general(S);
}

/* ------------------------------------------------------------------------ */
/* Continuous elements (App. B): the same graph scheme on the dofs of a       */
/* continuous Q_k space, with c_ij and c_i^d of eq. cijcidefCg.               */
/* ------------------------------------------------------------------------ */

/* Global node of local node a of cell K: index k K_e + a_e per axis (modulo
 * the axis's node count on a periodic axis), x fastest. */
static long cg_node(const or_setup *S, long K, int a) {
  long ki[3];
  int ai[3];
  cell_multi(S, K, ki);
  local_multi(S, a, ai);
  long g = 0, st = 1;
  for (int e = 0; e < S->dim; ++e) {
    long ge = S->deg * ki[e] + ai[e];
    if (ge >= S->gn[e]) ge -= S->gn[e];  /* periodic wrap */
    g += ge * st;
    st *= S->gn[e];
  }
  return g;
}

/* c_ij of eq. cijcidefCg from its definition: the volume integrals over
 * every cell that holds both nodes, minus half the boundary integral of
 * phi_j phi_i n over the box faces (not periodic) that hold both. */
static void literal_cij_cg(const or_setup *S, long i, long j, double *out) {
  const int dim = S->dim, nloc = S->nloc;
  for (int e = 0; e < dim; ++e) out[e] = 0.0;
  for (long K = 0; K < S->ncells; ++K) {
    int a = -1, b = -1;
    for (int q = 0; q < nloc; ++q) {
      long g = cg_node(S, K, q);
      if (g == i) a = q;
      if (g == j) b = q;
    }
    if (a < 0 || b < 0) continue;
    if (S->vx) {
      double t[3];
      cell_integral_mapped(S, K, 1, a, b, t);
      for (int e = 0; e < dim; ++e) out[e] += t[e];
    } else {
      for (int e = 0; e < dim; ++e) {
        pair_arg pr = {a, b, e};
        out[e] += cell_integral(S, 1, pr);
      }
    }
    long ki[3];
    int ai[3], bi[3];
    cell_multi(S, K, ki);
    local_multi(S, a, ai);
    local_multi(S, b, bi);
    for (int f = 0; f < 2 * dim; ++f) {
      int e = f / 2, side = f % 2;
      if (S->bc[f] == OR_BC_PERIODIC) continue;
      if (ki[e] != (side ? S->n[e] - 1 : 0)) continue;       /* a cell face on box face f */
      if (ai[e] != side * S->deg || bi[e] != side * S->deg) continue;
      if (S->vx) {
        double t[3];
        face_integral_mapped(S, K, f, a, b, 1, t);
        for (int d = 0; d < dim; ++d) out[d] -= 0.5 * t[d];
      } else {
        out[e] -= 0.5 * (side ? 1.0 : -1.0) * face_integral(S, f, a, b, 1);
      }
    }
  }
}

static or_setup *cg_structure(or_setup *S);

or_setup *or_create_cg(int dim, int deg, const long *cells, const double *lo, const double *hi, const int *bc) {
  or_setup *S = setup_init(dim, deg, cells, lo, hi, bc);
  if (!S) return NULL;
  return cg_structure(S);
}

/* Continuous elements on general (mapdeg 1) or curved (mapdeg 2) cells of
 * the lattice: the integrals of eq. cijcidefCg through each cell's map. */
or_setup *or_create_cg_curved(int dim, int deg, const long *cells, const double *vx, const int *bc, int mapdeg) {
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  if (mapdeg != 1 && mapdeg != 2) return NULL;
  or_setup *S = setup_init(dim, deg, cells, lo, hi, bc);
  if (!S) return NULL;
  S->mapdeg = mapdeg;
  long nv = 1;
  for (int e = 0; e < dim; ++e) nv *= mapdeg * S->n[e] + 1;
  S->vx = (double *)malloc(nv * dim * sizeof(double));
  memcpy(S->vx, vx, nv * dim * sizeof(double));
  S->nq = deg + 2 + (mapdeg == 2 ? 2 : 0);
  gauss_rule(S->nq, S->xq, S->wq);
  double vol = 0.0;
  for (long K = 0; K < S->ncells; ++K) {
    double t[3];
    for (int a = 0; a < S->nloc; ++a) {
      cell_integral_mapped(S, K, 2, a, 0, t);
      vol += t[0];
    }
    int tot = 1;
    for (int e = 0; e < dim; ++e) tot *= S->nq;
    for (int q = 0; q < tot; ++q) {
      double xi[3] = {0, 0, 0}, x[3], J[3][3], Ji[3][3];
      int r = q;
      for (int e = 0; e < dim; ++e) { xi[e] = S->xq[r % S->nq]; r /= S->nq; }
      cell_map(S, K, xi, x, J);
      if (!(inverse(dim, J, Ji) > 0.0)) { or_destroy(S); return NULL; }
    }
  }
  S->vol = vol;
  return cg_structure(S);
}

static or_setup *cg_structure(or_setup *S) {
  const int dim = S->dim, deg = S->deg;
  S->cg = 1;
  long N = 1;
  for (int e = 0; e < 3; ++e) {
    S->gn[e] = e < dim ? deg * S->n[e] + (S->bc[2 * e] == OR_BC_PERIODIC ? 0 : 1) : 1;
    /* a periodic axis needs 2k + 1 distinct nodes for a node's neighbours */
    if (e < dim && S->bc[2 * e] == OR_BC_PERIODIC && S->gn[e] < 2 * deg + 1) { free(S); return NULL; }
    N *= S->gn[e];
  }
  S->ndofs = N;
  const int nloc = S->nloc, W = 1;
  (void)W;
  /* the stencil of node i: the nodes of every cell that holds i, found by
   * offsets -k .. k per axis (dense per row), then compacted */
  int span = 1;
  for (int e = 0; e < dim; ++e) span *= 2 * deg + 1;
  double *cc = (double *)calloc((size_t)N * span * dim, sizeof(double));
  double *mm = (double *)calloc((size_t)N * span, sizeof(double));
  char *used = (char *)calloc((size_t)N * span, 1);
  double *cb = (double *)calloc((size_t)N * 2 * dim * dim, sizeof(double));
  char *onb = (char *)calloc((size_t)N * 2 * dim, 1);
  S->mi = (double *)calloc(N, sizeof(double));
  S->cgx = (double *)malloc(N * dim * sizeof(double));
  for (long K = 0; K < S->ncells; ++K) {
    long ki[3];
    cell_multi(S, K, ki);
    for (int a = 0; a < nloc; ++a) {
      const long i = cg_node(S, K, a);
      int ai[3];
      local_multi(S, a, ai);
      pair_arg pa = {a, 0, 0};
      double tm[3];
      if (S->vx) cell_integral_mapped(S, K, 2, a, 0, tm);
      S->mi[i] += S->vx ? tm[0] : cell_integral(S, 2, pa);
      int wrapped = 0;  /* the last node of a periodic axis is the first: keep the first's position */
      for (int e = 0; e < dim; ++e) wrapped |= deg * ki[e] + ai[e] >= S->gn[e];
      if (!wrapped && S->vx) {
        double xi[3] = {0, 0, 0}, J[3][3];
        for (int e = 0; e < dim; ++e) xi[e] = S->xg[ai[e]];
        cell_map(S, K, xi, S->cgx + i * dim, J);
      }
      for (int e = 0; e < dim && !wrapped && !S->vx; ++e)
        S->cgx[i * dim + e] = S->lo[e] + (ki[e] + S->xg[ai[e]]) * S->h[e];
      for (int b = 0; b < nloc; ++b) {
        int bi[3], off = 0, st = 1;
        local_multi(S, b, bi);
        for (int e = 0; e < dim; ++e) { off += (bi[e] - ai[e] + deg) * st; st *= 2 * deg + 1; }
        used[(size_t)i * span + off] = 1;
        if (S->vx) {
          double t[3];
          cell_integral_mapped(S, K, 1, a, b, t);
          for (int e = 0; e < dim; ++e) cc[((size_t)i * span + off) * dim + e] += t[e];
          cell_integral_mapped(S, K, 0, a, b, t);
          mm[(size_t)i * span + off] += t[0];
        } else {
          for (int e = 0; e < dim; ++e) {
            pair_arg pr = {a, b, e};
            cc[((size_t)i * span + off) * dim + e] += cell_integral(S, 1, pr);
          }
          pair_arg pm = {a, b, 0};
          mm[(size_t)i * span + off] += cell_integral(S, 0, pm);
        }
      }
      /* boundary terms of the cell faces on box faces (App. B) */
      for (int f = 0; f < 2 * dim; ++f) {
        int e = f / 2, side = f % 2;
        if (S->bc[f] == OR_BC_PERIODIC) continue;
        if (ki[e] != (side ? S->n[e] - 1 : 0) || ai[e] != side * deg) continue;
        const double n = side ? 1.0 : -1.0;
        onb[(size_t)i * 2 * dim + f] = 1;
        if (S->vx) {
          double t[3];
          face_integral_mapped(S, K, f, a, -1, 1, t);
          for (int d = 0; d < dim; ++d) cb[((size_t)i * 2 * dim + f) * dim + d] += 0.5 * t[d];
        } else {
          cb[((size_t)i * 2 * dim + f) * dim + e] += 0.5 * n * face_integral(S, f, a, -1, 1);
        }
        for (int b = 0; b < nloc; ++b) {
          int bi[3], off = 0, st = 1;
          local_multi(S, b, bi);
          if (bi[e] != side * deg) continue;
          for (int d = 0; d < dim; ++d) { off += (bi[d] - ai[d] + deg) * st; st *= 2 * deg + 1; }
          if (S->vx) {
            double t[3];
            face_integral_mapped(S, K, f, a, b, 1, t);
            for (int d = 0; d < dim; ++d) cc[((size_t)i * span + off) * dim + d] -= 0.5 * t[d];
          } else {
            cc[((size_t)i * span + off) * dim + e] -= 0.5 * n * face_integral(S, f, a, b, 1);
          }
        }
      }
    }
  }
  /* CSR: the used offsets in offset order; boundary parts per box face */
  S->rowptr = (long *)calloc(N + 1, sizeof(long));
  S->bptr = (long *)calloc(N + 1, sizeof(long));
  for (long i = 0; i < N; ++i) {
    long g = 0, nb = 0;
    for (int o = 0; o < span; ++o) g += used[(size_t)i * span + o];
    for (int f = 0; f < 2 * dim; ++f) nb += onb[(size_t)i * 2 * dim + f];
    S->rowptr[i + 1] = S->rowptr[i] + g;
    S->bptr[i + 1] = S->bptr[i] + nb;
  }
  long nnz = S->rowptr[N], nbt = S->bptr[N];
  S->col = (long *)malloc(nnz * sizeof(long));
  S->c = (double *)malloc(nnz * dim * sizeof(double));
  S->mij = (double *)malloc(nnz * sizeof(double));
  S->kind = (int *)malloc(nnz * sizeof(int));
  S->bface = (int *)malloc((nbt + 1) * sizeof(int));
  S->bkind = (int *)malloc((nbt + 1) * sizeof(int));
  S->bc_c = (double *)malloc((nbt + 1) * dim * sizeof(double));
  for (long i = 0; i < N; ++i) {
    long gi[3], r = i;
    for (int e = 0; e < dim; ++e) { gi[e] = r % S->gn[e]; r /= S->gn[e]; }
    long q = S->rowptr[i];
    for (int o = 0; o < span; ++o) {
      if (!used[(size_t)i * span + o]) continue;
      long j = 0, st = 1;
      int rr = o;
      for (int e = 0; e < dim; ++e) {
        long ge = gi[e] + rr % (2 * deg + 1) - deg;
        rr /= 2 * deg + 1;
        if (ge < 0) ge += S->gn[e];
        if (ge >= S->gn[e]) ge -= S->gn[e];
        j += ge * st;
        st *= S->gn[e];
      }
      S->col[q] = j;
      for (int e = 0; e < dim; ++e) S->c[q * dim + e] = cc[((size_t)i * span + o) * dim + e];
      S->mij[q] = mm[(size_t)i * span + o];
      S->kind[q] = OR_KIND_CELL;
      ++q;
    }
    long b = S->bptr[i];
    for (int f = 0; f < 2 * dim; ++f) {
      if (!onb[(size_t)i * 2 * dim + f]) continue;
      for (int e = 0; e < dim; ++e) S->bc_c[b * dim + e] = cb[((size_t)i * 2 * dim + f) * dim + e];
      S->bface[b] = f;
      S->bkind[b] = S->bc[f];
      ++b;
    }
  }
  /* reading R3: c_ji is stored as exactly -c_ij, from the lower index */
  for (long i = 0; i < N; ++i)
    for (long q = S->rowptr[i]; q < S->rowptr[i + 1]; ++q) {
      const long j = S->col[q];
      if (j == i) { for (int e = 0; e < dim; ++e) S->c[q * dim + e] = 0.0; continue; }
      if (j > i) continue;
      for (long p = S->rowptr[j]; p < S->rowptr[j + 1]; ++p)
        if (S->col[p] == i)
          for (int e = 0; e < dim; ++e) S->c[q * dim + e] = -S->c[p * dim + e];
    }
  free(cc); free(mm); free(used); free(cb); free(onb);
  return S;
}

static or_setup *setup_init(int dim, int deg, const long *cells, const double *lo, const double *hi, const int *bc) {
  if (dim < 1 || dim > 3 || deg < 1 || deg > 3) return NULL;
  or_setup *S = (or_setup *)calloc(1, sizeof(or_setup));
  S->dim = dim; S->deg = deg; S->nb1 = deg + 1; S->m = dim + 2;
  S->nloc = 1;
  for (int e = 0; e < dim; ++e) S->nloc *= S->nb1;
  S->ncells = 1; S->vol = 1.0;
  for (int e = 0; e < 3; ++e) {
    S->n[e] = e < dim ? cells[e] : 1;
    S->lo[e] = e < dim ? lo[e] : 0.0;
    S->hi[e] = e < dim ? hi[e] : 1.0;
    S->h[e] = (S->hi[e] - S->lo[e]) / (double)S->n[e];
    if (e < dim) { S->ncells *= S->n[e]; S->vol *= S->hi[e] - S->lo[e]; }
  }
  for (int f = 0; f < 6; ++f) S->bc[f] = f < 2 * dim ? bc[f] : OR_BC_OUTFLOW;
  for (int f = 0; f < 2 * dim; ++f)
    if (S->bc[f] < OR_BC_PERIODIC || S->bc[f] > OR_BC_INOUTFLOW) { free(S); return NULL; }
  for (int e = 0; e < dim; ++e) {
    int p0 = S->bc[2 * e] == OR_BC_PERIODIC, p1 = S->bc[2 * e + 1] == OR_BC_PERIODIC;
    if (p0 != p1 || (p0 && S->n[e] < 2) || S->n[e] < 1) { free(S); return NULL; }
  }
  S->ndofs = S->ncells * S->nloc;
  /* Gauss-Lobatto nodes on [0, 1]: the end points and, for k = 2, 3, the
   * roots of the derivative of the Legendre polynomial of degree k */
  if (deg == 1) { S->xg[0] = 0.0; S->xg[1] = 1.0; }
  else if (deg == 2) { S->xg[0] = 0.0; S->xg[1] = 0.5; S->xg[2] = 1.0; }
  else {
    double r = 0.5 / sqrt(5.0);
    S->xg[0] = 0.0; S->xg[1] = 0.5 - r; S->xg[2] = 0.5 + r; S->xg[3] = 1.0;
  }
  /* Gauss-Legendre rule with k + 1 points on [0, 1] (exact to degree 2k + 1) */
  S->nq = deg + 1;
  if (deg == 1) {
    double r = 0.5 / sqrt(3.0);
    S->xq[0] = 0.5 - r; S->xq[1] = 0.5 + r; S->wq[0] = S->wq[1] = 0.5;
  } else if (deg == 2) {
    double r = 0.5 * sqrt(0.6);
    S->xq[0] = 0.5 - r; S->xq[1] = 0.5; S->xq[2] = 0.5 + r;
    S->wq[0] = S->wq[2] = 5.0 / 18.0; S->wq[1] = 8.0 / 18.0;
  } else {
    /* on [-1, 1]: x = +-sqrt(3/7 -+ (2/7) sqrt(6/5)), w = (18 +- sqrt(30)) / 36 */
    double xi = sqrt(3.0 / 7.0 - 2.0 / 7.0 * sqrt(1.2)), xo = sqrt(3.0 / 7.0 + 2.0 / 7.0 * sqrt(1.2));
    double wi = (18.0 + sqrt(30.0)) / 36.0, wo = (18.0 - sqrt(30.0)) / 36.0;
    S->xq[0] = 0.5 * (1.0 - xo); S->xq[1] = 0.5 * (1.0 - xi);
    S->xq[2] = 0.5 * (1.0 + xi); S->xq[3] = 0.5 * (1.0 + xo);
    S->wq[0] = S->wq[3] = 0.5 * wo; S->wq[1] = S->wq[2] = 0.5 * wi;
  }
  return S;
}

static void setup_build(or_setup *S) {
  const int dim = S->dim, deg = S->deg;
  long N = S->ndofs;
  int nloc = S->nloc;
  /* stencil rows: all in-cell dofs, then face neighbours on each face i lies on */
  S->rowptr = (long *)calloc(N + 1, sizeof(long));
  S->bptr = (long *)calloc(N + 1, sizeof(long));
  long cap = N * (nloc + 2 * dim * nloc), bcap = N * dim + 1;
  S->col = (long *)malloc(cap * sizeof(long));
  S->c = (double *)malloc(cap * dim * sizeof(double));
  S->mij = (double *)malloc(cap * sizeof(double));
  S->kind = (int *)malloc(cap * sizeof(int));
  S->mi = (double *)malloc(N * sizeof(double));
  S->bface = (int *)malloc(bcap * sizeof(int));
  S->bkind = (int *)malloc(bcap * sizeof(int));
  S->bc_c = (double *)malloc(bcap * dim * sizeof(double));

  /* reference cell quantities (identical for every uniform cell, but computed
   * per row so the code reads as the definition) */
  double *Mloc = (double *)malloc(nloc * nloc * sizeof(double));
  double *mloc = (double *)malloc(nloc * sizeof(double));
  for (int a = 0; a < nloc; ++a) {
    pair_arg p = {a, 0, 0};
    mloc[a] = cell_integral(S, 2, p);
    for (int b = 0; b < nloc; ++b) {
      pair_arg q = {a, b, 0};
      Mloc[a * nloc + b] = cell_integral(S, 0, q);
    }
  }

  /* row lengths first, so that the rows can be filled independently */
  for (long i = 0; i < N; ++i) {
    long K = i / nloc;
    int a = (int)(i % nloc), ai[3];
    local_multi(S, a, ai);
    long g = nloc, bnd = 0;
    for (int f = 0; f < 2 * dim; ++f) {
      int e = f / 2, side = f % 2;
      if (ai[e] != side * deg) continue;
      if (neighbour(S, K, f) >= 0) g += nloc / S->nb1;
      else ++bnd;
    }
    S->rowptr[i + 1] = S->rowptr[i] + g;
    S->bptr[i + 1] = S->bptr[i] + bnd;
  }
#pragma omp parallel for schedule(dynamic, 4096)
  for (long i = 0; i < N; ++i) {
    long K = i / nloc;
    int a = (int)(i % nloc), ai[3];
    local_multi(S, a, ai);
    long nnz = S->rowptr[i], nb = S->bptr[i];
    double t[3];
    if (S->vx) cell_integral_mapped(S, K, 2, a, 0, t);
    S->mi[i] = S->vx ? t[0] : mloc[a];
    for (int b = 0; b < nloc; ++b) {
      long j = K * nloc + b;
      S->col[nnz] = j;
      canonical_cij(S, i, j, S->c + nnz * dim);
      if (S->vx) cell_integral_mapped(S, K, 0, a, b, t);
      S->mij[nnz] = S->vx ? t[0] : Mloc[a * nloc + b];
      S->kind[nnz] = OR_KIND_CELL;
      ++nnz;
    }
    for (int f = 0; f < 2 * dim; ++f) {
      int e = f / 2, side = f % 2;
      if (ai[e] != side * deg) continue;
      long Kn = neighbour(S, K, f);
      if (Kn >= 0) {
        for (int b = 0; b < nloc; ++b) {
          int bi[3];
          local_multi(S, b, bi);
          if (!on_shared_face(S, K, f, b)) continue;
          long j = Kn * nloc + b;
          int colloc = 1;
          if (S->ucp) {
            /* collocated: the same point (reading R12 on unstructured cells) */
            double xa[3], xb[3], dd = 0.0, hs = 0.0;
            node_x(S, i, xa);
            node_x(S, j, xb);
            for (int d = 0; d < dim; ++d) { dd = fmax(dd, fabs(xa[d] - xb[d])); hs = fmax(hs, fabs(xa[d])); }
            colloc = dd <= 1e-12 * (1.0 + hs);
          } else {
            for (int d = 0; d < dim; ++d) if (d != e && bi[d] != ai[d]) colloc = 0;
          }
          S->col[nnz] = j;
          canonical_cij(S, i, j, S->c + nnz * dim);
          S->mij[nnz] = 0.0;
          S->kind[nnz] = colloc ? OR_KIND_FACE_COLLOC : OR_KIND_FACE;
          ++nnz;
        }
      } else {
        /* boundary part k = face f: c_i^{d,k} = 1/2 int_{dK cap dOmega_k} phi_i n */
        double n = side ? 1.0 : -1.0;
        for (int d = 0; d < dim; ++d) S->bc_c[nb * dim + d] = 0.0;
        if (S->vx) {
          face_integral_mapped(S, K, f, a, -1, 1, t);
          for (int d = 0; d < dim; ++d) S->bc_c[nb * dim + d] = 0.5 * t[d];
        } else {
          S->bc_c[nb * dim + e] = 0.5 * n * face_integral(S, f, a, -1, 1);
        }
        S->bface[nb] = f;
        S->bkind[nb] = S->bc[f];
        if (S->ucp) {
          const signed char u = S->ubc[K * 2 * dim + f];
          S->bface[nb] = u >> 3;
          S->bkind[nb] = u & 7;
        }
        ++nb;
      }
    }
  }
  free(Mloc);
  free(mloc);
}

/* threads the row loops use (OpenMP) */
int or_num_threads(void) { return omp_get_max_threads(); }

/* The entropy-viscosity constant c_ev of Sec. 5.2 for degree k (the paper's
 * choice: 1, 0.5, 0.25 for k = 1, 2, 3); 0 for a degree it gives none. */
double or_default_cev(int degree) {
  switch (degree) {
    case 1: return 1.0;
    case 2: return 0.5;
    case 3: return 0.25;
    default: return 0.0;
  }
}

/* sets the threads of the row loops (timing on one core and on all) */
void or_set_num_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

long or_num_dofs(const or_setup *S) { return S->ndofs; }
long or_nnz(const or_setup *S) { return S->rowptr[S->ndofs]; }
long or_nbnd(const or_setup *S) { return S->bptr[S->ndofs]; }
double or_volume(const or_setup *S) { return S->vol; }

/* The volume |Omega| that the mesh-size measure hhat_i = (m_i / |Omega|)^(1/d)
 * of eq. ViscMin and eq. ViscMinConst2 refers to.  By default the box itself;
 * a sub-box cut out of a larger domain passes that domain's volume, so that
 * its rows get the constants of the full problem. */
void or_set_reference_volume(or_setup *S, double vol) {
  if (vol > 0.0) S->vol = vol;
}

/* Boundary kinds per boundary cell face instead of one per box face (Sec. 4.1
 * applies its conditions part by part of the boundary): for each box face f
 * that is not periodic, in order of f, one kind per cell face on it, the
 * cells of that face taken lexicographically over the other axes with the
 * lowest axis fastest.  Data kinds take the data of box face f.  Returns 0,
 * or -1 (nothing changed) for a periodic kind or an unknown one. */
int or_set_boundary_kinds(or_setup *S, const signed char *kinds) {
  const int dim = S->dim;
  long off[6], n = 0;
  for (int f = 0; f < 2 * dim; ++f) {
    off[f] = n;
    if (S->bc[f] == OR_BC_PERIODIC) continue;
    long cnt = 1;
    for (int g = 0; g < dim; ++g)
      if (g != f / 2) cnt *= S->n[g];
    n += cnt;
  }
  for (long q = 0; q < n; ++q)
    if (kinds[q] <= OR_BC_PERIODIC || kinds[q] > OR_BC_INOUTFLOW) return -1;
  for (long i = 0; i < S->ndofs; ++i) {
    long ki[3];
    cell_multi(S, i / S->nloc, ki);
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
      const int f = S->bface[b], e = f / 2;
      long idx = 0, stride = 1;
      for (int g = 0; g < dim; ++g) {
        if (g == e) continue;
        idx += ki[g] * stride;
        stride *= S->n[g];
      }
      S->bkind[b] = kinds[off[f] + idx];
    }
  }
  return 0;
}

void or_csr(const or_setup *S, long *rowptr, long *col, double *c, double *mij, int *kind) {
  long N = S->ndofs, nnz = S->rowptr[N];
  memcpy(rowptr, S->rowptr, (N + 1) * sizeof(long));
  memcpy(col, S->col, nnz * sizeof(long));
  memcpy(c, S->c, nnz * S->dim * sizeof(double));
  memcpy(mij, S->mij, nnz * sizeof(double));
  memcpy(kind, S->kind, nnz * sizeof(int));
}

void or_lumped(const or_setup *S, double *mi) { memcpy(mi, S->mi, S->ndofs * sizeof(double)); }

void or_boundary(const or_setup *S, long *bptr, int *bface, double *bc_c) {
  long N = S->ndofs, nb = S->bptr[N];
  memcpy(bptr, S->bptr, (N + 1) * sizeof(long));
  memcpy(bface, S->bface, nb * sizeof(int));
  memcpy(bc_c, S->bc_c, nb * S->dim * sizeof(double));
}

/* Collocation points x_i. */
static void node_x(const or_setup *S, long i, double *x);

void or_node_coords(const or_setup *S, double *xyz) {
  for (long i = 0; i < S->ndofs; ++i) node_x(S, i, xyz + i * S->dim);
}

/* literal c_ij for both orders (pins Lemma PropSkew without the R3 reading) */
static void literal_cij_cg(const or_setup *S, long i, long j, double *out);
void or_literal_cij(const or_setup *S, long i, long j, double *out) {
  if (S->cg) literal_cij_cg(S, i, j, out);
  else literal_cij(S, i, j, out);
}

/* ------------------------------------------------------------------------ */
/* Euler physics (Sec. 2.2)                                                   */
/* ------------------------------------------------------------------------ */

/* internal energy per volume eps = E - |m|^2/(2 rho), eq. PressurEuler */
static double eps_of(int dim, const double *U) {
  double m2 = 0.0;
  for (int e = 0; e < dim; ++e) m2 += U[1 + e] * U[1 + e];
  return U[dim + 1] - 0.5 * m2 / U[0];
}

static double pres_of(double g, int dim, const double *U) { return (g - 1.0) * eps_of(dim, U); }

/* specific entropy s = log(rho^-gamma p), eq. EntropyEuler */
static double spec_entropy(double g, int dim, const double *U) {
  return log(pow(U[0], -g) * pres_of(g, dim, U));
}

/* rescaled entropy s~ = rho^-gamma eps (Sec. 5.4) */
static double stilde(double g, int dim, const double *U) {
  return pow(U[0], -g) * eps_of(dim, U);
}

/* f(U) c, the flux of eq. euler_flux applied to a vector c */
static void flux_dot(double g, int dim, const double *U, const double *c, double *out) {
  double rho = U[0], E = U[dim + 1], p = pres_of(g, dim, U);
  double mc = 0.0;
  for (int e = 0; e < dim; ++e) mc += U[1 + e] * c[e];
  out[0] = mc;
  for (int e = 0; e < dim; ++e) out[1 + e] = U[1 + e] * mc / rho + p * c[e];
  out[dim + 1] = (E + p) * mc / rho;
}

/* Reading R1: lambda^+ is the two-rarefaction upper bound of Guermond & Popov
 * (2016) for 1 < gamma <= 5/3, evaluated without Newton refinement; a
 * non-positive numerator means vacuum, p* = 0. */
double or_lambda_max(double g, int dim, const double *UL, const double *UR, const double *n) {
  double rl = UL[0], rr = UR[0];
  double ul = 0.0, ur = 0.0;
  for (int e = 0; e < dim; ++e) { ul += UL[1 + e] * n[e]; ur += UR[1 + e] * n[e]; }
  ul /= rl; ur /= rr;
  double pl = pres_of(g, dim, UL), pr = pres_of(g, dim, UR);
  double al = sqrt(g * pl / rl), ar = sqrt(g * pr / rr);
  double alpha = (g - 1.0) / (2.0 * g);
  double num = al + ar - 0.5 * (g - 1.0) * (ur - ul);
  double den = al * pow(pl, -alpha) + ar * pow(pr, -alpha);
  double pstar = num > 0.0 ? pow(num / den, 1.0 / alpha) : 0.0;
  double kfac = (g + 1.0) / (2.0 * g);
  double lam1 = ul - al * sqrt(1.0 + kfac * fmax(pstar - pl, 0.0) / pl);
  double lam3 = ur + ar * sqrt(1.0 + kfac * fmax(pstar - pr, 0.0) / pr);
  double lm = fmax(-lam1, lam3);
  return fmax(lm, 0.0);
}

/* Exact 1D Riemann solver (textbook: Toro 2009, Ch. 4).  Test support only:
 * the reference solution for the shock tube and the brute-force check of
 * the wave-speed bound.  Returns 0, or 1 when a vacuum forms. */
static double toro_f(double g, double p, double rk, double pk, double ak, double *df) {
  if (p > pk) {
    double A = 2.0 / ((g + 1.0) * rk), B = (g - 1.0) / (g + 1.0) * pk;
    double q = sqrt(A / (p + B));
    *df = q * (1.0 - 0.5 * (p - pk) / (p + B));
    return (p - pk) * q;
  }
  double ex = (g - 1.0) / (2.0 * g);
  *df = 1.0 / (rk * ak) * pow(p / pk, -(g + 1.0) / (2.0 * g));
  return 2.0 * ak / (g - 1.0) * (pow(p / pk, ex) - 1.0);
}

int or_exact_riemann(double g, double rl, double ul, double pl, double rr, double ur, double pr,
                     double *pstar, double *ustar) {
  double al = sqrt(g * pl / rl), ar = sqrt(g * pr / rr);
  double d0, d1;
  double phi0 = toro_f(g, 0.0, rl, pl, al, &d0) + toro_f(g, 0.0, rr, pr, ar, &d1) + ur - ul;
  if (phi0 >= 0.0) { *pstar = 0.0; *ustar = 0.5 * (ul + ur); return 1; }
  /* bracket [0, hi] with phi(hi) > 0, then bisect to full precision */
  double lo = 0.0, hi = fmax(pl, pr);
  for (int it = 0; it < 200; ++it) {
    double v = toro_f(g, hi, rl, pl, al, &d0) + toro_f(g, hi, rr, pr, ar, &d1) + ur - ul;
    if (v > 0.0) break;
    lo = hi;
    hi *= 2.0;
  }
  for (int it = 0; it < 2000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double v = toro_f(g, mid, rl, pl, al, &d0) + toro_f(g, mid, rr, pr, ar, &d1) + ur - ul;
    if (v > 0.0) hi = mid; else lo = mid;
  }
  double p = 0.5 * (lo + hi);
  double fl = toro_f(g, p, rl, pl, al, &d0), fr = toro_f(g, p, rr, pr, ar, &d1);
  *pstar = p;
  *ustar = 0.5 * (ul + ur) + 0.5 * (fr - fl);
  return 0;
}

/* Largest wave speed of the exact solution: the same wave-speed formulas as
 * the bound, evaluated at the exact p*. */
double or_exact_lambda(double g, double rl, double ul, double pl, double rr, double ur, double pr) {
  double ps, us;
  or_exact_riemann(g, rl, ul, pl, rr, ur, pr, &ps, &us);
  double al = sqrt(g * pl / rl), ar = sqrt(g * pr / rr);
  double kfac = (g + 1.0) / (2.0 * g);
  double lam1 = ul - al * sqrt(1.0 + kfac * fmax(ps - pl, 0.0) / pl);
  double lam3 = ur + ar * sqrt(1.0 + kfac * fmax(ps - pr, 0.0) / pr);
  return fmax(fmax(-lam1, lam3), 0.0);
}

/* Sample the exact self-similar solution at xi = x/t. */
void or_riemann_sample(double g, double rl, double ul, double pl, double rr, double ur, double pr,
                       double xi, double *out /* rho, u, p */) {
  double ps, us;
  or_exact_riemann(g, rl, ul, pl, rr, ur, pr, &ps, &us);
  double al = sqrt(g * pl / rl), ar = sqrt(g * pr / rr);
  double gm = (g - 1.0) / (g + 1.0);
  double r, u, p;
  if (xi <= us) {
    if (ps > pl) { /* left shock */
      double sl = ul - al * sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g));
      if (xi <= sl) { r = rl; u = ul; p = pl; }
      else { r = rl * (ps / pl + gm) / (gm * ps / pl + 1.0); u = us; p = ps; }
    } else { /* left rarefaction */
      double head = ul - al, ast = al * pow(ps / pl, (g - 1.0) / (2.0 * g)), tail = us - ast;
      if (xi <= head) { r = rl; u = ul; p = pl; }
      else if (xi >= tail) { r = rl * pow(ps / pl, 1.0 / g); u = us; p = ps; }
      else {
        u = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * ul + xi);
        double c = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * (ul - xi));
        r = rl * pow(c / al, 2.0 / (g - 1.0));
        p = pl * pow(c / al, 2.0 * g / (g - 1.0));
      }
    }
  } else {
    if (ps > pr) { /* right shock */
      double sr = ur + ar * sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g));
      if (xi >= sr) { r = rr; u = ur; p = pr; }
      else { r = rr * (ps / pr + gm) / (gm * ps / pr + 1.0); u = us; p = ps; }
    } else { /* right rarefaction */
      double head = ur + ar, ast = ar * pow(ps / pr, (g - 1.0) / (2.0 * g)), tail = us + ast;
      if (xi >= head) { r = rr; u = ur; p = pr; }
      else if (xi <= tail) { r = rr * pow(ps / pr, 1.0 / g); u = us; p = ps; }
      else {
        u = 2.0 / (g + 1.0) * (-ar + 0.5 * (g - 1.0) * ur + xi);
        double c = 2.0 / (g + 1.0) * (ar - 0.5 * (g - 1.0) * (ur - xi));
        r = rr * pow(c / ar, 2.0 / (g - 1.0));
        p = pr * pow(c / ar, 2.0 * g / (g - 1.0));
      }
    }
  }
  out[0] = r; out[1] = u; out[2] = p;
}

/* ------------------------------------------------------------------------ */
/* Boundary data (Sec. 4.1)                                                   */
/* ------------------------------------------------------------------------ */

/* Ghost state U^{d,k} for the boundary part on box face f of row i, with
 * n = c_i^{d,k}/|c_i^{d,k}|:
 *  - outflow: the supersonic-outflow branch U^d := U_i (reading R28);
 *  - slip: the normal momentum reflected, eq. slip_boundary;
 *  - Dirichlet: the face's data U^d;
 *  - supersonic in/outflow, eq. supersonic_inoutflow: U^d if u_i.n < -a_i
 *    (inflow), U_i if u_i.n >= a_i (outflow).  The subsonic range between
 *    needs the characteristic construction, which is not built: there the
 *    function returns -4 (and U_i as the ghost).
 * Returns 0 or -4. */
/* Node coordinates x_i. */
static void node_x(const or_setup *S, long i, double *x) {
  if (S->cg) {
    for (int e = 0; e < S->dim; ++e) x[e] = S->cgx[i * S->dim + e];
    return;
  }
  long ki[3];
  int ai[3];
  cell_multi(S, i / S->nloc, ki);
  local_multi(S, (int)(i % S->nloc), ai);
  if (S->vx) {
    double xi[3] = {0, 0, 0}, J[3][3];
    for (int e = 0; e < S->dim; ++e) xi[e] = S->xg[ai[e]];
    cell_map(S, i / S->nloc, xi, x, J);
    return;
  }
  for (int e = 0; e < S->dim; ++e) x[e] = S->lo[e] + (ki[e] + S->xg[ai[e]]) * S->h[e];
}

/* The isentropic vortex of Sec. 6.2 at point x and time t (free space, no
 * periodic images): with xb = x - x0 - t u_inf, r = |xb|,
 * rho = (1 - (gamma-1) beta^2 / (8 gamma pi^2) e^{1-r^2})^{1/(gamma-1)},
 * p = rho^gamma, u = u_inf + beta / (2 pi) e^{(1-r^2)/2} (-xb_2, xb_1)
 * (the velocity factor with the exponent halved: reading R23, the form in
 * radial balance). */
static void vortex_at(const double *vp, const double *x, double t, double *U) {
  const double beta = vp[0], g = vp[5];
  const double xb0 = x[0] - vp[1] - t * vp[3], xb1 = x[1] - vp[2] - t * vp[4];
  const double r2 = xb0 * xb0 + xb1 * xb1;
  const double T = 1.0 - (g - 1.0) * beta * beta / (8.0 * g * OR_PI * OR_PI) * exp(1.0 - r2);
  const double rho = pow(T, 1.0 / (g - 1.0)), p = pow(rho, g);
  const double fac = beta / (2.0 * OR_PI) * exp(0.5 * (1.0 - r2));
  const double u0 = vp[3] - fac * xb1, u1 = vp[4] + fac * xb0;
  U[0] = rho;
  U[1] = rho * u0;
  U[2] = rho * u1;
  U[3] = p / (g - 1.0) + 0.5 * rho * (u0 * u0 + u1 * u1);
}

/* Dirichlet data U^d of box face f at node i and time t (Sec. 4.1: the data
 * at position x_i for time t). */
static void data_state(const or_setup *S, int f, long i, double t, double *Ud) {
  if (S->step_start_data) {
    for (int c = 0; c < S->m; ++c) Ud[c] = S->un[(long)c * S->ndofs + i];
    return;
  }
  if (S->vortex_data) {
    double x[3];
    node_x(S, i, x);
    vortex_at(S->vortex, x, t, Ud);
    return;
  }
  for (int c = 0; c < S->m; ++c) Ud[c] = S->bstate[f][c];
}

/* Sub- and supersonic in/outflow (Sec. 4.1): eq. supersonic_inoutflow where
 * |u_i.n| >= a_i, and in the subsonic range the state whose characteristic
 * variables of eq. characteristics equal those of the data U^d for the
 * incoming characteristics (speed lambda_k(U_i, n) <= 0) and those of U_i for
 * the others.  The state follows from its four variables
 * R1 = v_n - 2a/(gamma-1), R2 = p / rho^gamma, R3 = v - v_n n,
 * R4 = v_n + 2a/(gamma-1):  v_n = (R1 + R4)/2, a = (gamma-1)(R4 - R1)/4,
 * rho = (a^2 / (gamma R2))^{1/(gamma-1)}, p = R2 rho^gamma (reading R35).
 * Returns -4 if that state has no positive sound speed. */
static int inoutflow_state(int dim, double g, const double *Ui, const double *Ud, const double *n, double *Ug) {
  double vi[3], vd[3], vni = 0.0, vnd = 0.0;
  for (int e = 0; e < dim; ++e) {
    vi[e] = Ui[1 + e] / Ui[0];
    vd[e] = Ud[1 + e] / Ud[0];
    vni += vi[e] * n[e];
    vnd += vd[e] * n[e];
  }
  const double pi = (g - 1.0) * eps_of(dim, Ui), pd = (g - 1.0) * eps_of(dim, Ud);
  const double ai = sqrt(g * pi / Ui[0]), ad = sqrt(g * pd / Ud[0]);
  if (vni < -ai) {
    for (int c = 0; c < dim + 2; ++c) Ug[c] = Ud[c];
    return 0;
  }
  if (vni >= ai) {
    for (int c = 0; c < dim + 2; ++c) Ug[c] = Ui[c];
    return 0;
  }
  /* characteristic speeds at U_i: v_n - a < 0, v_n, v_n, v_n + a > 0 */
  const int in23 = vni <= 0.0;
  const double R1 = vnd - 2.0 * ad / (g - 1.0);
  const double R4 = vni + 2.0 * ai / (g - 1.0);
  const double R2 = in23 ? pd / pow(Ud[0], g) : pi / pow(Ui[0], g);
  double R3[3];
  for (int e = 0; e < dim; ++e) R3[e] = in23 ? vd[e] - vnd * n[e] : vi[e] - vni * n[e];
  const double vn = 0.5 * (R1 + R4), a = 0.25 * (g - 1.0) * (R4 - R1);
  if (!(a > 0.0)) {
    for (int c = 0; c < dim + 2; ++c) Ug[c] = Ui[c];
    return -4;
  }
  const double rho = pow(a * a / (g * R2), 1.0 / (g - 1.0)), p = R2 * pow(rho, g);
  double u2 = 0.0;
  Ug[0] = rho;
  for (int e = 0; e < dim; ++e) {
    const double v = R3[e] + vn * n[e];
    Ug[1 + e] = rho * v;
    u2 += v * v;
  }
  Ug[dim + 1] = p / (g - 1.0) + 0.5 * rho * u2;
  return 0;
}

/* Boundary state U^d of one boundary part (Sec. 4.1) of node i, face f,
 * c_i^{d,f} = cb, at time t:
 *  - outflow: U_i (the supersonic-outflow branch of eq. supersonic_inoutflow);
 *  - slip: eq. slip_boundary;
 *  - Dirichlet: the data U^d;
 *  - supersonic in/outflow, eq. supersonic_inoutflow: U^d if u_i.n < -a_i
 *    (inflow), U_i if u_i.n >= a_i (outflow); the subsonic range between
 *    returns -4 (and U_i as the ghost);
 *  - sub- and supersonic in/outflow: inoutflow_state().
 * Returns 0 or -4. */
static int ghost_state(const or_setup *S, double gamma, int f, int bkind, long i, double t, const double *Ui,
                       const double *cb, double *Ug) {
  int dim = S->dim;
  double nn = 0.0;
  for (int e = 0; e < dim; ++e) nn += cb[e] * cb[e];
  nn = sqrt(nn);
  for (int c = 0; c < S->m; ++c) Ug[c] = Ui[c];
  if (bkind == OR_BC_SLIP) {
    double mn = 0.0;
    for (int e = 0; e < dim; ++e) mn += Ui[1 + e] * cb[e] / nn;
    for (int e = 0; e < dim; ++e) Ug[1 + e] = Ui[1 + e] - 2.0 * mn * cb[e] / nn;
  } else if (bkind == OR_BC_DIRICHLET) {
    data_state(S, f, i, t, Ug);
  } else if (bkind == OR_BC_SUPERSONIC) {
    double un = 0.0;
    for (int e = 0; e < dim; ++e) un += (Ui[1 + e] / Ui[0]) * cb[e] / nn;
    double a = sqrt(gamma * (gamma - 1.0) * eps_of(dim, Ui) / Ui[0]);
    if (un < -a) {
      data_state(S, f, i, t, Ug);
    } else if (!(un >= a)) {
      return -4;
    }
  } else if (bkind == OR_BC_INOUTFLOW) {
    double Ud[OR_MAXM], n[3];
    data_state(S, f, i, t, Ud);
    for (int e = 0; e < dim; ++e) n[e] = cb[e] / nn;
    return inoutflow_state(dim, gamma, Ui, Ud, n, Ug);
  }
  return 0;
}

/* inoutflow_state() for the pins of eq. characteristics. */
int or_inoutflow_state(int dim, double gamma, const double *Ui, const double *Ud, const double *n, double *Ug) {
  return inoutflow_state(dim, gamma, Ui, Ud, n, Ug);
}

/* Time of the boundary data at the start of the next step. */
void or_set_time(or_setup *S, double t) { S->t0 = t; }

/* Boundary data of every Dirichlet-type face from the isentropic vortex
 * (beta, x0[2], u_inf[2], gamma) instead of the constant face states; 2D
 * meshes only.  Returns 0, or -1 for another dimension. */
int or_set_vortex_data(or_setup *S, const double *params) {
  if (S->dim != 2) return -1;
  S->vortex_data = 1;
  for (int k = 0; k < 6; ++k) S->vortex[k] = params[k];
  return 0;
}

/* Boundary data of every Dirichlet-type face from the step's start state at
 * the node (strategy (d) of Sec. 6.3). */
void or_set_step_start_data(or_setup *S) {
  S->step_start_data = 1;
  if (!S->un) S->un = (double *)calloc((size_t)S->m * S->ndofs, sizeof(double));
}

/* Keeps U^n for step-start data. */
static void keep_step_start(const or_setup *S, const double *U) {
  if (S->step_start_data) memcpy(S->un, U, (size_t)S->m * S->ndofs * sizeof(double));
}

/* Dirichlet data U^d (conserved, m components) of box face f, used by the
 * Dirichlet and supersonic kinds. */
void or_set_boundary_state(or_setup *S, int f, const double *U) {
  for (int c = 0; c < S->m; ++c) S->bstate[f][c] = U[c];
}

/* ------------------------------------------------------------------------ */
/* One forward-Euler stage of the scheme                                      */
/* ------------------------------------------------------------------------ */

typedef struct {
  double tau_max;   /* min_i -m_i/(2 d_ii) of the input state, eq. MaxCFLdt */
  double *N;        /* N entropy-viscosity ratio per row (may be NULL) */
  double *rho_min, *rho_max, *s_min; /* relaxed bounds, eq. local_bounds */
  double *UL;       /* low-order update, m*N SoA */
  double *dUH;      /* high-order increment U^H - U, m*N SoA */
  double *U1;       /* after limiter pass 1, m*N SoA */
  double *dij;      /* d^L per CSR entry */
  double *lij;      /* l_ij of pass 1 per CSR entry */
  double *lbd;      /* l_i^d of pass 1 per row */
  double *Aij;      /* A_ij per CSR entry, m per entry */
  double *Abd;      /* A_i^d per row, m per row */
  double *Ncond;    /* sum of |terms| of R_i and D_i over D_i: N_i's sensitivity to rounding */
} or_diag;

static void get_state(const or_setup *S, const double *U, long i, double *out) {
  for (int c = 0; c < S->m; ++c) out[c] = U[c * S->ndofs + i];
}

static double norm_c(int dim, const double *c) {
  double s = 0.0;
  for (int e = 0; e < dim; ++e) s += c[e] * c[e];
  return sqrt(s);
}

/* d^L_ij = |c_ij| lambda^+(U_i, U_j, n_ij) evaluated from the lower index
 * (reading R3), so that d_ij = d_ji holds exactly. */
static double dij_low(const or_setup *S, double g, const double *U, long i, long j, const double *cij) {
  int dim = S->dim;
  double nc = norm_c(dim, cij);
  if (nc == 0.0) return 0.0;
  double Ua[OR_MAXM], Ub[OR_MAXM], n[3];
  long a = i < j ? i : j, b = i < j ? j : i;
  double sgn = i < j ? 1.0 : -1.0;
  get_state(S, U, a, Ua);
  get_state(S, U, b, Ub);
  for (int e = 0; e < dim; ++e) n[e] = sgn * cij[e] / nc;
  return nc * or_lambda_max(g, dim, Ua, Ub, n);
}

/* Line search on the density bounds: largest l in [0, 1] with
 * rho_min <= rho(U + l P) <= rho_max. */
static double ls_rho(double r, double pr, double rmin, double rmax) {
  double l = 1.0;
  if (r + pr > rmax) l = (rmax - r) / pr;
  if (r + pr < rmin) l = (rmin - r) / pr;
  if (!(l > 0.0)) l = 0.0;
  if (l > 1.0) l = 1.0;
  return l;
}

/* psi(l) = eps(U + l P) - s_min rho(U + l P)^gamma, concave in l. */
static double ls_psi(double g, int dim, const double *U, const double *P, double smin, double l,
                     double *dpsi) {
  double V[OR_MAXM];
  for (int c = 0; c < dim + 2; ++c) V[c] = U[c] + l * P[c];
  double eps = eps_of(dim, V);
  double rg = pow(V[0], g);
  if (dpsi) {
    double u2 = 0.0, dot = 0.0;
    for (int e = 0; e < dim; ++e) {
      double u = V[1 + e] / V[0];
      u2 += u * u;
      dot -= u * P[1 + e];
    }
    dot += 0.5 * u2 * P[0] + P[dim + 1];
    *dpsi = dot - smin * g * rg / V[0] * P[0];
  }
  return eps - smin * rg;
}

#define OR_LS_TOL 1e-14
#define OR_LS_MAXIT 60

/* Reading R16: line search for the rescaled-entropy bound.  Largest l in
 * [0, lhi] with s~(U + l P) >= s_min, found on the concave psi by a bracket
 * [l, r] (psi(l) >= 0 > psi(r)) narrowed with a secant step (lands on the
 * feasible side) and a tangent step at r (lands on the infeasible side) until
 * r - l <= 1e-14; the feasible end is returned. */
static double ls_entropy(double g, int dim, const double *U, const double *P, double smin, double lhi) {
  double ph = ls_psi(g, dim, U, P, smin, lhi, NULL);
  if (ph >= 0.0) return lhi;
  double p0 = ls_psi(g, dim, U, P, smin, 0.0, NULL);
  if (p0 <= 0.0) return 0.0;
  double l = 0.0, r = lhi, pl = p0, pr = ph;
  for (int it = 0; it < OR_LS_MAXIT; ++it) {
    if (r - l <= OR_LS_TOL) break;
    /* secant */
    double x = l + pl * (r - l) / (pl - pr);
    if (!(x > l && x < r)) x = 0.5 * (l + r);
    double px = ls_psi(g, dim, U, P, smin, x, NULL);
    if (px >= 0.0) { l = x; pl = px; } else { r = x; pr = px; }
    if (r - l <= OR_LS_TOL) break;
    /* tangent at the infeasible end */
    double dr;
    ls_psi(g, dim, U, P, smin, r, &dr);
    x = dr < 0.0 ? r - pr / dr : 0.5 * (l + r);
    if (!(x > l && x < r)) x = 0.5 * (l + r);
    px = ls_psi(g, dim, U, P, smin, x, NULL);
    if (px >= 0.0) { l = x; pl = px; } else { r = x; pr = px; }
  }
  return l;
}

/* Line search LS(U, P, B): the density part, then the entropy part on
 * [0, l_rho] (Sec. 5.4, Lemma ConsInvariants). */
static double line_search(double g, int dim, const double *U, const double *P, double rmin,
                          double rmax, double smin) {
  double lr = ls_rho(U[0], P[0], rmin, rmax);
  return ls_entropy(g, dim, U, P, smin, lr);
}

/* Dense LU solve (partial pivoting) of the n x n cell mass block, reading R6. */
static void dense_solve(int n, double *A, double *b) {
  int piv[64];
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r) if (fabs(A[r * n + k]) > fabs(A[p * n + k])) p = r;
    piv[k] = p;
    if (p != k) {
      for (int c = 0; c < n; ++c) { double t = A[k * n + c]; A[k * n + c] = A[p * n + c]; A[p * n + c] = t; }
      double t = b[k]; b[k] = b[p]; b[p] = t;
    }
    for (int r = k + 1; r < n; ++r) {
      double f = A[r * n + k] / A[k * n + k];
      for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
      b[r] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * b[c];
    b[k] = s / A[k * n + k];
  }
  (void)piv;
}

static double *dalloc(long n) { return (double *)calloc(n > 0 ? n : 1, sizeof(double)); }

/* Phi(U; tau): one forward-Euler step of the scheme selected by P->scheme.
 * tau <= 0 selects tau = Cr * tau_max of this state (eq. MaxCFLdt).
 * Returns 0 on success, -2 if the output leaves the admissible set, -4 if a
 * node of a supersonic in/outflow face sees subsonic normal flow. */
static int stage_at(const or_setup *S, const or_params *P, const double *U, double tau, double t, double *Uout,
                    or_diag *dg);

/* One stage at the time of the step's start (or_set_time). */
int or_stage(const or_setup *S, const or_params *P, const double *U, double tau, double *Uout,
             or_diag *dg) {
  keep_step_start(S, U);
  return stage_at(S, P, U, tau, S->t0, Uout, dg);
}

/* The stage with boundary data at time t. */
static int stage_at(const or_setup *S, const or_params *P, const double *U, double tau, double t, double *Uout,
                    or_diag *dg) {
  const int dim = S->dim, m = S->m;
  const long N = S->ndofs, nnz = S->rowptr[N];
  const double g = P->gamma;
  double *dij = dalloc(nnz), *dbd = dalloc(S->bptr[N]), *dii = dalloc(N);
  double *UL = dalloc(m * N), *Nr = dalloc(N), *dH = dalloc(nnz), *dbH = dalloc(S->bptr[N]);
  double *dUH = dalloc(m * N), *A = dalloc(nnz * m), *Ab = dalloc(N * m);
  double *qrmin = dalloc(N), *qrmax = dalloc(N), *qsmin = dalloc(N);
  double *Brmin = dalloc(N), *Brmax = dalloc(N), *Bsmin = dalloc(N);
  double *l1 = dalloc(nnz), *lb1 = dalloc(N), *U1 = dalloc(m * N);
  double *Ug = dalloc((S->bptr[N] + 1) * m);
  double *Ncd = (dg && dg->Ncond) ? dg->Ncond : NULL;
  int status = 0;

  /* Sec. 4.1: boundary data per boundary part */
  int subsonic = 0;
  for (long i = 0; i < N; ++i) {
    double Ui[OR_MAXM];
    get_state(S, U, i, Ui);
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b)
      if (ghost_state(S, g, S->bface[b], S->bkind[b], i, t, Ui, S->bc_c + b * dim, Ug + b * m)) subsonic = 1;
  }

  /* eq. dij_low_order, dij_low_order_modified (reading R2: inside state on
   * the left, outward normal), eq. dij_low_order_supplement */
  double tmax = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : tmax)
  for (long i = 0; i < N; ++i) {
    double s = 0.0;
    for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
      long j = S->col[k];
      dij[k] = (j == i) ? 0.0 : dij_low(S, g, U, i, j, S->c + k * dim);
      if (j != i) s += dij[k];
    }
    double Ui[OR_MAXM];
    get_state(S, U, i, Ui);
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
      const double *cb = S->bc_c + b * dim;
      double nc = norm_c(dim, cb), n[3];
      for (int e = 0; e < dim; ++e) n[e] = cb[e] / nc;
      dbd[b] = nc * or_lambda_max(g, dim, Ui, Ug + b * m, n);
      s += dbd[b];
    }
    dii[i] = -s;
    double t = -S->mi[i] / (2.0 * dii[i]);
    if (t < tmax) tmax = t;
  }
  if (tau <= 0.0) tau = P->cfl * tmax;

  /* eq. cijdijscheme / cijdijschememodified: low-order update, with the
   * flux sums in the difference form sum_j (f(U_j) - f(U_i)) c_ij that the
   * proof of Lemma ConveRef derives from Lemma LemPart (reading R30) */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double Ui[OR_MAXM], Uj[OR_MAXM], acc[OR_MAXM] = {0}, fc[OR_MAXM], fi[OR_MAXM];
    get_state(S, U, i, Ui);
    for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
      long j = S->col[k];
      get_state(S, U, j, Uj);
      flux_dot(g, dim, Uj, S->c + k * dim, fc);
      flux_dot(g, dim, Ui, S->c + k * dim, fi);
      for (int c = 0; c < m; ++c) acc[c] += (fc[c] - fi[c]) - dij[k] * (Uj[c] - Ui[c]);
    }
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
      const double *Ub = Ug + b * m;
      flux_dot(g, dim, Ub, S->bc_c + b * dim, fc);
      flux_dot(g, dim, Ui, S->bc_c + b * dim, fi);
      for (int c = 0; c < m; ++c) acc[c] += (fc[c] - fi[c]) - dbd[b] * (Ub[c] - Ui[c]);
    }
    for (int c = 0; c < m; ++c) UL[c * N + i] = Ui[c] - tau / S->mi[i] * acc[c];
  }

  if (P->scheme == OR_LOW_ORDER) {
    memcpy(Uout, UL, m * N * sizeof(double));
    goto finish;
  }

  /* eq. UsualBarState: ring-1 partial bounds over k in I(j) (reading R18:
   * the diagonal contributes U_j itself, no bar state; reading R19: pairs
   * with c = 0 have no bar state) */
#pragma omp parallel for schedule(static)
  for (long j = 0; j < N; ++j) {
    double Uj[OR_MAXM], Uk[OR_MAXM], fj[OR_MAXM], fk[OR_MAXM], Ub[OR_MAXM];
    get_state(S, U, j, Uj);
    double rmin = INFINITY, rmax = -INFINITY, smin = INFINITY;
    for (long k = S->rowptr[j]; k < S->rowptr[j + 1]; ++k) {
      long kk = S->col[k];
      get_state(S, U, kk, Uk);
      rmin = fmin(rmin, Uk[0]);
      rmax = fmax(rmax, Uk[0]);
      smin = fmin(smin, stilde(g, dim, Uk));
      if (kk == j || dij[k] == 0.0) continue;
      const double *c = S->c + k * dim;
      flux_dot(g, dim, Uj, c, fj);
      flux_dot(g, dim, Uk, c, fk);
      for (int q = 0; q < m; ++q) Ub[q] = 0.5 * (Uj[q] + Uk[q]) - (fk[q] - fj[q]) / (2.0 * dij[k]);
      rmin = fmin(rmin, Ub[0]);
      rmax = fmax(rmax, Ub[0]);
      smin = fmin(smin, stilde(g, dim, Ub));
    }
    qrmin[j] = rmin; qrmax[j] = rmax; qsmin[j] = smin;
  }

  /* Sec. 5.2 entropy viscosity: Harten entropy f(s) = exp(s/(gamma+1))
   * (reading R8), gradient of the shifted entropy at U_i (reading R9), D_i as
   * the sum of absolute parts so |N_i| <= 1 (reading R10), the boundary part
   * included as a ghost neighbour (reading R11), flux sums in the difference
   * form (reading R30) so a constant state gives R_i = D_i = 0 exactly. */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double Ui[OR_MAXM], Uj[OR_MAXM], fc[OR_MAXM], fi[OR_MAXM], grad[OR_MAXM], Sk[OR_MAXM] = {0};
    get_state(S, U, i, Ui);
    double si = spec_entropy(g, dim, Ui);
    double fsi = exp(si / (g + 1.0)), dfsi = fsi / (g + 1.0);
    double rho = Ui[0], p = pres_of(g, dim, Ui), u2 = 0.0;
    for (int e = 0; e < dim; ++e) u2 += (Ui[1 + e] / rho) * (Ui[1 + e] / rho);
    /* grad s = (gamma-1)/p (|u|^2/2, -u, 1) - (gamma/rho, 0, 0) */
    grad[0] = (g - 1.0) / p * 0.5 * u2 - g / rho;
    for (int e = 0; e < dim; ++e) grad[1 + e] = -(g - 1.0) / p * (Ui[1 + e] / rho);
    grad[dim + 1] = (g - 1.0) / p;
    for (int c = 0; c < m; ++c) grad[c] *= rho * dfsi;
    double T = 0.0;
    for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
      long j = S->col[k];
      get_state(S, U, j, Uj);
      const double *c = S->c + k * dim;
      double fsj = exp(spec_entropy(g, dim, Uj) / (g + 1.0));
      double mc = 0.0;
      for (int e = 0; e < dim; ++e) mc += Uj[1 + e] * c[e];
      T += mc * (fsj - fsi);
      flux_dot(g, dim, Uj, c, fc);
      flux_dot(g, dim, Ui, c, fi);
      for (int q = 0; q < m; ++q) Sk[q] += fc[q] - fi[q];
    }
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
      const double *Ub = Ug + b * m, *c = S->bc_c + b * dim;
      double fsb = exp(spec_entropy(g, dim, Ub) / (g + 1.0));
      double mc = 0.0;
      for (int e = 0; e < dim; ++e) mc += Ub[1 + e] * c[e];
      T += mc * (fsb - fsi);
      flux_dot(g, dim, Ub, c, fc);
      flux_dot(g, dim, Ui, c, fi);
      for (int q = 0; q < m; ++q) Sk[q] += fc[q] - fi[q];
    }
    double R = T, D = fabs(T);
    for (int q = 0; q < m; ++q) { R -= grad[q] * Sk[q]; D += fabs(grad[q]) * fabs(Sk[q]); }
    Nr[i] = D > 0.0 ? R / D : 0.0;
    if (Ncd) {
      /* magnitude of the summed terms (before cancellation) over D_i */
      double mag = 0.0, Sabs[OR_MAXM] = {0};
      for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
        get_state(S, U, S->col[k], Uj);
        const double *c = S->c + k * dim;
        double fsj = exp(spec_entropy(g, dim, Uj) / (g + 1.0)), mc = 0.0;
        for (int e = 0; e < dim; ++e) mc += Uj[1 + e] * c[e];
        mag += fabs(mc) * (fabs(fsj) + fabs(fsi));
        flux_dot(g, dim, Uj, c, fc);
        flux_dot(g, dim, Ui, c, fi);
        for (int q = 0; q < m; ++q) Sabs[q] += fabs(fc[q]) + fabs(fi[q]);
      }
      for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
        const double *Ub = Ug + b * m, *c = S->bc_c + b * dim;
        double fsb = exp(spec_entropy(g, dim, Ub) / (g + 1.0)), mc = 0.0;
        for (int e = 0; e < dim; ++e) mc += Ub[1 + e] * c[e];
        mag += fabs(mc) * (fabs(fsb) + fabs(fsi));
        flux_dot(g, dim, Ub, c, fc);
        flux_dot(g, dim, Ui, c, fi);
        for (int q = 0; q < m; ++q) Sabs[q] += fabs(fc[q]) + fabs(fi[q]);
      }
      for (int q = 0; q < m; ++q) mag += fabs(grad[q]) * Sabs[q];
      Ncd[i] = D > 0.0 ? mag / D : (mag > 0.0 ? INFINITY : 0.0);
    }
  }

  /* eq. HighOrderViscosity with eq. ViscMin (reading R12: collocation is
   * topological) and the boundary analogue of reading R7 */
  {
    const double pk = (S->deg % 2 == 0) ? 0.5 : 0.0;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
      for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
        long j = S->col[k];
        if (j == i) { dH[k] = 0.0; continue; }
        double dev = dij[k] * fmin(P->c_ev * fmax(fabs(Nr[i]), fabs(Nr[j])), 1.0);
        double dmin = 0.0;
        if (S->kind[k] == OR_KIND_FACE_COLLOC) {
          double hh = pow(0.5 * (S->mi[i] + S->mi[j]) / S->vol, 1.0 / dim);
          dmin = P->c_k * pow(hh, pk) * dij[k];
        }
        dH[k] = fmax(dmin, dev);
      }
      for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
        double hh = pow(S->mi[i] / S->vol, 1.0 / dim);
        double dmin = P->c_k * pow(hh, pk) * dbd[b];
        double dev = dbd[b] * fmin(P->c_ev * fabs(Nr[i]), 1.0);
        dbH[b] = fmax(dmin, dev);
      }
    }
  }

  /* eq. HighScheme: cell-local consistent-mass solve (reading R6) */
  {
    int nloc = S->nloc;
#pragma omp parallel for schedule(static)
    for (long K = 0; K < S->ncells; ++K) {
      double Mk[64 * 64], rhs[OR_MAXM][64];
      for (int a = 0; a < nloc; ++a) {
        long i = K * nloc + a;
        double Ui[OR_MAXM], Uj[OR_MAXM], fc[OR_MAXM], fi[OR_MAXM], acc[OR_MAXM] = {0};
        get_state(S, U, i, Ui);
        for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
          long j = S->col[k];
          get_state(S, U, j, Uj);
          flux_dot(g, dim, Uj, S->c + k * dim, fc);
          flux_dot(g, dim, Ui, S->c + k * dim, fi);
          for (int c = 0; c < m; ++c) acc[c] += (fc[c] - fi[c]) - dH[k] * (Uj[c] - Ui[c]);
        }
        for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
          const double *Ub = Ug + b * m;
          flux_dot(g, dim, Ub, S->bc_c + b * dim, fc);
          flux_dot(g, dim, Ui, S->bc_c + b * dim, fi);
          for (int c = 0; c < m; ++c) acc[c] += (fc[c] - fi[c]) - dbH[b] * (Ub[c] - Ui[c]);
        }
        for (int c = 0; c < m; ++c) rhs[c][a] = -tau * acc[c];
      }
      for (int c = 0; c < m; ++c) {
        /* m_ij of the cell, taken from the in-cell CSR entries */
        for (int a = 0; a < nloc; ++a) {
          long i = K * nloc + a;
          for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k)
            if (S->kind[k] == OR_KIND_CELL) Mk[a * nloc + (S->col[k] - K * nloc)] = S->mij[k];
        }
        dense_solve(nloc, Mk, rhs[c]);
        for (int a = 0; a < nloc; ++a) dUH[c * N + K * nloc + a] = rhs[c][a];
      }
    }
  }

  if (P->scheme == OR_HIGH_ORDER) {
    for (long q = 0; q < m * N; ++q) Uout[q] = U[q] + dUH[q];
    goto finish;
  }

  /* eq. HighLowOrderIdentity: A_ij = tau (d^H - d^L)(U_j - U_i)
   *   - (m_ij - delta_ij m_i)(dU^H_j - dU^H_i),  A_i^d = tau (d^dH - d^dL)(U^d - U_i) */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double Ui[OR_MAXM], Uj[OR_MAXM];
    get_state(S, U, i, Ui);
    for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
      long j = S->col[k];
      get_state(S, U, j, Uj);
      double mm = S->mij[k] - (j == i ? S->mi[i] : 0.0);
      for (int c = 0; c < m; ++c)
        A[k * m + c] = tau * (dH[k] - dij[k]) * (Uj[c] - Ui[c]) - mm * (dUH[c * N + j] - dUH[c * N + i]);
    }
    for (int c = 0; c < m; ++c) Ab[i * m + c] = 0.0;
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b)
      for (int c = 0; c < m; ++c) Ab[i * m + c] += tau * (dbH[b] - dbd[b]) * (Ug[b * m + c] - Ui[c]);
  }

  /* eq. local_bounds with relaxation r_h^{+-} = 1 +- c_r h_i^{p_r} */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double rmin = INFINITY, rmax = -INFINITY, smin = INFINITY;
    double Ui[OR_MAXM], fi[OR_MAXM], fb[OR_MAXM], Ub[OR_MAXM];
    get_state(S, U, i, Ui);
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
      /* eq. BoundaryBarState */
      const double *Ug_ = Ug + b * m, *c = S->bc_c + b * dim;
      flux_dot(g, dim, Ui, c, fi);
      flux_dot(g, dim, Ug_, c, fb);
      for (int q = 0; q < m; ++q) Ub[q] = 0.5 * (Ug_[q] + Ui[q]) - (fb[q] - fi[q]) / (2.0 * dbd[b]);
      rmin = fmin(rmin, Ub[0]);
      rmax = fmax(rmax, Ub[0]);
      smin = fmin(smin, stilde(g, dim, Ub));
    }
    for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
      long j = S->col[k];
      rmin = fmin(rmin, qrmin[j]);
      rmax = fmax(rmax, qrmax[j]);
      smin = fmin(smin, qsmin[j]);
    }
    double hh = pow(S->mi[i] / S->vol, 1.0 / dim);
    double rel = P->c_r * pow(hh, P->p_r);
    Brmin[i] = (1.0 - rel) * rmin;
    Brmax[i] = (1.0 + rel) * rmax;
    Bsmin[i] = (1.0 - rel) * smin;
  }

  /* eq. ConvexScheme and Lemma ConsInvariants: kappa_i = 1/(card I(i) + 1)
   * with I(i) the stored row (reading R4); l_ij = min(l^i_ij, l^j_ji)
   * (reading R15); the boundary parts share one A_i^d (reading R27).  The
   * second pass limits the remaining (1 - l) A from U^(1) against the same
   * bounds (reading R14). */
  {
    const double *Ubase = UL;
    double *Acur = A, *Abcur = Ab;
    double *A2 = NULL, *Ab2 = NULL;
    double *Unext = U1;
    for (int pass = 0; pass < P->passes; ++pass) {
      if (pass == 1) {
        A2 = dalloc(nnz * m); Ab2 = dalloc(N * m);
        for (long k = 0; k < nnz; ++k) for (int c = 0; c < m; ++c) A2[k * m + c] = (1.0 - l1[k]) * A[k * m + c];
        for (long i = 0; i < N; ++i) for (int c = 0; c < m; ++c) Ab2[i * m + c] = (1.0 - lb1[i]) * Ab[i * m + c];
        Acur = A2; Abcur = Ab2; Ubase = U1;
        Unext = Uout;
      }
      double *lp = pass == 0 ? l1 : dalloc(nnz);
      double *lbp = pass == 0 ? lb1 : dalloc(N);
#pragma omp parallel for schedule(static)
      for (long i = 0; i < N; ++i) {
        double Li[OR_MAXM], Lj[OR_MAXM], Pv[OR_MAXM];
        long leni = S->rowptr[i + 1] - S->rowptr[i];
        double kap_i = 1.0 / (double)(leni + 1);
        get_state(S, Ubase, i, Li);
        double acc[OR_MAXM] = {0};
        for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
          long j = S->col[k];
          double li, lj;
          for (int c = 0; c < m; ++c) Pv[c] = Acur[k * m + c] / (kap_i * S->mi[i]);
          li = line_search(g, dim, Li, Pv, Brmin[i], Brmax[i], Bsmin[i]);
          long lenj = S->rowptr[j + 1] - S->rowptr[j];
          double kap_j = 1.0 / (double)(lenj + 1);
          get_state(S, Ubase, j, Lj);
          for (int c = 0; c < m; ++c) Pv[c] = -Acur[k * m + c] / (kap_j * S->mi[j]);
          lj = line_search(g, dim, Lj, Pv, Brmin[j], Brmax[j], Bsmin[j]);
          lp[k] = fmin(li, lj);
          for (int c = 0; c < m; ++c) acc[c] += lp[k] * Acur[k * m + c];
        }
        for (int c = 0; c < m; ++c) Pv[c] = Abcur[i * m + c] / (kap_i * S->mi[i]);
        lbp[i] = line_search(g, dim, Li, Pv, Brmin[i], Brmax[i], Bsmin[i]);
        for (int c = 0; c < m; ++c) acc[c] += lbp[i] * Abcur[i * m + c];
        for (int c = 0; c < m; ++c) Unext[c * N + i] = Li[c] + acc[c] / S->mi[i];
      }
      if (pass == 1) { free(lp); free(lbp); }
    }
    if (P->passes == 1) memcpy(Uout, U1, m * N * sizeof(double));
    if (P->passes <= 0) memcpy(Uout, UL, m * N * sizeof(double));
    free(A2); free(Ab2);
  }

finish:
  for (long i = 0; i < N; ++i) {
    double V[OR_MAXM];
    get_state(S, Uout, i, V);
    if (!(V[0] > 0.0) || !(eps_of(dim, V) > 0.0)) status = -2;
  }
  if (dg) {
    dg->tau_max = tmax;
    if (dg->N) memcpy(dg->N, Nr, N * sizeof(double));
    if (dg->rho_min) memcpy(dg->rho_min, Brmin, N * sizeof(double));
    if (dg->rho_max) memcpy(dg->rho_max, Brmax, N * sizeof(double));
    if (dg->s_min) memcpy(dg->s_min, Bsmin, N * sizeof(double));
    if (dg->UL) memcpy(dg->UL, UL, m * N * sizeof(double));
    if (dg->dUH) memcpy(dg->dUH, dUH, m * N * sizeof(double));
    if (dg->U1) memcpy(dg->U1, U1, m * N * sizeof(double));
    if (dg->dij) memcpy(dg->dij, dij, nnz * sizeof(double));
    if (dg->lij) memcpy(dg->lij, l1, nnz * sizeof(double));
    if (dg->lbd) memcpy(dg->lbd, lb1, N * sizeof(double));
    if (dg->Aij) memcpy(dg->Aij, A, nnz * m * sizeof(double));
    if (dg->Abd) memcpy(dg->Abd, Ab, N * m * sizeof(double));
  }
  free(dij); free(dbd); free(dii); free(UL); free(Nr); free(dH); free(dbH); free(dUH);
  free(A); free(Ab); free(qrmin); free(qrmax); free(qsmin); free(Brmin); free(Brmax); free(Bsmin);
  free(l1); free(lb1); free(U1); free(Ug);
  return subsonic ? -4 : status;
}

/* Per-row CFL quantity -m_i/(2 d_ii), eq. CFLcond; the global minimum is
 * tau_max of eq. MaxCFLdt. */
void or_tau_rows(const or_setup *S, const or_params *P, const double *U, double *out) {
  const int dim = S->dim, m = S->m;
  const long N = S->ndofs;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double s = 0.0, Ui[OR_MAXM], Ug[OR_MAXM];
    for (long k = S->rowptr[i]; k < S->rowptr[i + 1]; ++k) {
      long j = S->col[k];
      if (j != i) s += dij_low(S, P->gamma, U, i, j, S->c + k * dim);
    }
    get_state(S, U, i, Ui);
    for (long b = S->bptr[i]; b < S->bptr[i + 1]; ++b) {
      const double *cb = S->bc_c + b * dim;
      double nc = norm_c(dim, cb), n[3];
      ghost_state(S, P->gamma, S->bface[b], S->bkind[b], i, S->t0, Ui, cb, Ug);
      for (int e = 0; e < dim; ++e) n[e] = cb[e] / nc;
      s += nc * or_lambda_max(P->gamma, dim, Ui, Ug, n);
    }
    out[i] = S->mi[i] / (2.0 * s);
  }
  (void)m;
}

/* SSP-RK3 in Shu-Osher form (Sec. 6.2).  tau is fixed in stage 1 from the
 * CFL rule and capped by dt_cap (reading R21); stages 2 and 3 re-check the
 * CFL condition of their own state and, on violation, the step restarts from
 * U^n with tau = Cr * tau_max of the violating stage (reading R20).
 * dt_fixed > 0 replaces the CFL rule for stage 1.
 * Returns 0, -2 (inadmissible output), -3 (CFL restarts exhausted) or -4
 * (subsonic normal flow at a supersonic in/outflow face). */
/* SSPRK(5,4) of Spiteri and Ruuth in Shu-Osher form,
 *   u(i) = sum_k alpha_ik u(k) + beta_ik tau L(u(k)),  u(0) = U^n, u(5) = U^{n+1},
 * the coefficients as that work prints them (15 digits).  Every stage is a
 * convex combination of forward-Euler steps of size (beta/alpha) tau. */
static const double rk54_a[6][5] = {
    {0, 0, 0, 0, 0},
    {1.0, 0, 0, 0, 0},
    {0.444370493651235, 0.555629506348765, 0, 0, 0},
    {0.620101851488403, 0, 0.379898148511597, 0, 0},
    {0.178079954393132, 0, 0, 0.821920045606868, 0},
    {0, 0, 0.517231671970585, 0.096059710526147, 0.386708617503269}};
static const double rk54_b[6][5] = {
    {0, 0, 0, 0, 0},
    {0.391752226571890, 0, 0, 0, 0},
    {0, 0.368410593050371, 0, 0, 0},
    {0, 0, 0.251891774271694, 0, 0},
    {0, 0, 0, 0.544974750228521, 0},
    {0, 0, 0, 0.063692468666290, 0.226007483236906}};

/* The Shu-Osher table for the pins (order conditions, SSP coefficient). */
void or_ssprk54_table(double *alpha, double *beta) {
  for (int i = 0; i < 6; ++i)
    for (int k = 0; k < 5; ++k) {
      alpha[i * 5 + k] = rk54_a[i][k];
      beta[i * 5 + k] = rk54_b[i][k];
    }
}

/* One SSPRK(5,4) step (reading R45).  Stage k takes the forward-Euler step
 * Phi of size r_k tau, r_k = beta_{k+1,k} / alpha_{k+1,k}, at its own state
 * u(k) and time t + c_k tau (c_k: the stage's abscissa, the row sums of the
 * Butcher table of the same method); the last stage also reuses the step of
 * u(3) for the term beta_53 tau L(u(3)) (its ratio beta/alpha equals r_3 to
 * the printed digits).  tau = Cr tau_max(U^n) / max_k r_k, so that every
 * Euler step is within Cr of the CFL bound of U^n; stage k re-checks
 * r_k tau <= tau_max(u(k)) and on violation the step restarts with
 * tau = Cr tau_max(u(k)) / r_k. */
static int step_rk54(const or_setup *S, const or_params *P, double *U, double dt_cap, double dt_fixed,
                     double *dt_taken, int *restarts) {
  const long M = (long)S->m * S->ndofs;
  double *u[5], *Ph = dalloc(M), *acc = dalloc(M);
  for (int k = 0; k < 5; ++k) u[k] = dalloc(M);
  double r[5], c[5], A[6][5];
  memset(A, 0, sizeof A);
  for (int i = 1; i < 6; ++i)
    for (int k = 0; k < i; ++k) {
      for (int j = 0; j < 5; ++j) A[i][j] += rk54_a[i][k] * A[k][j];
      A[i][k] += rk54_b[i][k];
    }
  double rmax = 0.0;
  for (int k = 0; k < 5; ++k) {
    r[k] = rk54_b[k + 1][k] / rk54_a[k + 1][k];
    rmax = fmax(rmax, r[k]);
    c[k] = 0.0;
    for (int j = 0; j < 5; ++j) c[k] += A[k][j];
  }
  or_diag dg;
  memset(&dg, 0, sizeof(dg));
  int st = 0, nres = 0;
  double tau;
  if (dt_fixed > 0.0) {
    tau = dt_fixed;
  } else {
    double *tr = dalloc(S->ndofs);
    or_tau_rows(S, P, U, tr);
    double tm = INFINITY;
    for (long i = 0; i < S->ndofs; ++i) tm = fmin(tm, tr[i]);
    free(tr);
    tau = P->cfl * tm / rmax;
  }
  if (dt_cap > 0.0 && tau > dt_cap) tau = dt_cap;
  for (;;) {
    memcpy(u[0], U, M * sizeof(double));
    int restart = 0;
    for (int k = 0; k < 5 && !st && !restart; ++k) {
      st = stage_at(S, P, u[k], r[k] * tau, S->t0 + c[k] * tau, Ph, &dg);
      if (k > 0 && r[k] * tau > dg.tau_max) {
        if (++nres > 8) { st = -3; break; }
        tau = P->cfl * dg.tau_max / r[k];
        restart = 1;
        st = 0;
        break;
      }
      if (st) break;
      if (k == 3)  /* the last stage's terms in u(2) and L(u(3)) */
        for (long q = 0; q < M; ++q) acc[q] = rk54_a[5][2] * u[2][q] + rk54_a[5][3] * Ph[q];
      if (k < 4) {
        for (long q = 0; q < M; ++q) u[k + 1][q] = rk54_a[k + 1][k] * Ph[q] + (k ? rk54_a[k + 1][0] * u[0][q] : 0.0);
      } else {
        for (long q = 0; q < M; ++q) U[q] = acc[q] + rk54_a[5][4] * Ph[q];
      }
    }
    if (restart) continue;
    break;
  }
  *dt_taken = tau;
  if (restarts) *restarts = nres;
  for (int k = 0; k < 5; ++k) free(u[k]);
  free(Ph); free(acc);
  return st;
}

int or_step(const or_setup *S, const or_params *P, double *U, double dt_cap, double dt_fixed,
            double *dt_taken, int *restarts) {
  keep_step_start(S, U);
  if (P->integrator == 1) return step_rk54(S, P, U, dt_cap, dt_fixed, dt_taken, restarts);
  const long M = (long)S->m * S->ndofs;
  double *Ua = dalloc(M), *Ub = dalloc(M), *Ph = dalloc(M);
  or_diag dg;
  memset(&dg, 0, sizeof(dg));
  int st = 0, nres = 0;
  double tau;
  if (dt_fixed > 0.0) {
    tau = dt_fixed;
  } else {
    double *tr = dalloc(S->ndofs);
    or_tau_rows(S, P, U, tr);
    double tm = INFINITY;
    for (long i = 0; i < S->ndofs; ++i) tm = fmin(tm, tr[i]);
    free(tr);
    tau = P->cfl * tm;
  }
  if (dt_cap > 0.0 && tau > dt_cap) tau = dt_cap;
  /* stage times of the Shu-Osher form: t0, t0 + tau, t0 + tau / 2 (the
   * boundary data of each stage at its own time, reading R29) */
  for (;;) {
    st = stage_at(S, P, U, tau, S->t0, Ua, &dg);
    if (st) break;
    st = stage_at(S, P, Ua, tau, S->t0 + tau, Ph, &dg);
    if (tau > dg.tau_max) {
      if (++nres > 8) { st = -3; break; }
      tau = P->cfl * dg.tau_max;
      continue;
    }
    if (st) break;
    for (long q = 0; q < M; ++q) Ub[q] = 0.75 * U[q] + 0.25 * Ph[q];
    st = stage_at(S, P, Ub, tau, S->t0 + 0.5 * tau, Ph, &dg);
    if (tau > dg.tau_max) {
      if (++nres > 8) { st = -3; break; }
      tau = P->cfl * dg.tau_max;
      continue;
    }
    if (st) break;
    for (long q = 0; q < M; ++q) U[q] = (1.0 / 3.0) * U[q] + (2.0 / 3.0) * Ph[q];
    break;
  }
  *dt_taken = tau;
  if (restarts) *restarts = nres;
  free(Ua); free(Ub); free(Ph);
  return st;
}
