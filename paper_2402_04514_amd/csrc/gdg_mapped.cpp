// Stencil coefficients of general quadrilateral / hexahedral cells (Sec. 2.3,
// eq. mass_matrices, cij_def1, cij_def2, with Sec. 4.2's boundary parts):
// every cell is the multilinear image x = F_K(xi) of the reference cell
// through its 2^d corners, and the integrals are taken on the reference cell
// with the change of variables.  With cof(J) = det(J) J^{-T} (the cofactor
// matrix of the Jacobian, a polynomial in xi for a multilinear map):
//   m_ab      = int phi_a phi_b det J dxi,
//   c^K_ab    = int phi_a cof(J) grad_xi phi_b dxi,
//   n ds      = +-cof(J) e_e dxi on the face xi_e = 0 or 1 (outward sign),
// so every integrand is a polynomial and a Gauss rule of k + 2 points per
// direction integrates it exactly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "gdg.h"
#include "gdg_internal.h"

namespace gdg {

namespace {

// Gauss-Legendre rule of n = 2 .. 5 points on [0, 1], from the closed forms of
// the roots of the Legendre polynomials on [-1, 1].
void gauss01(int n, double *x, double *w) {
  double r[5], q[5];
  if (n == 2) {
    r[0] = -1.0 / std::sqrt(3.0), r[1] = -r[0];
    q[0] = q[1] = 1.0;
  } else if (n == 3) {
    r[0] = -std::sqrt(0.6), r[1] = 0.0, r[2] = -r[0];
    q[0] = q[2] = 5.0 / 9.0, q[1] = 8.0 / 9.0;
  } else if (n == 4) {
    const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2)), b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
    r[0] = -b, r[1] = -a, r[2] = a, r[3] = b;
    q[1] = q[2] = (18.0 + std::sqrt(30.0)) / 36.0, q[0] = q[3] = (18.0 - std::sqrt(30.0)) / 36.0;
  } else {
    const double a = std::sqrt(5.0 - 2.0 * std::sqrt(10.0 / 7.0)) / 3.0,
                 b = std::sqrt(5.0 + 2.0 * std::sqrt(10.0 / 7.0)) / 3.0;
    r[0] = -b, r[1] = -a, r[2] = 0.0, r[3] = a, r[4] = b;
    q[0] = q[4] = (322.0 - 13.0 * std::sqrt(70.0)) / 900.0;
    q[1] = q[3] = (322.0 + 13.0 * std::sqrt(70.0)) / 900.0;
    q[2] = 128.0 / 225.0;
  }
  for (int k = 0; k < n; ++k) {
    x[k] = 0.5 * (1.0 + r[k]);
    w[k] = 0.5 * q[k];
  }
}

// 1D Lagrange basis on the Gauss-Lobatto nodes of degree k.
struct Lag1D {
  int nb;
  double xg[4];
  double val(int a, double t) const {
    double v = 1.0;
    for (int b = 0; b < nb; ++b)
      if (b != a) v *= (t - xg[b]) / (xg[a] - xg[b]);
    return v;
  }
  double der(int a, double t) const {
    double s = 0.0;
    for (int c = 0; c < nb; ++c) {
      if (c == a) continue;
      double p = 1.0 / (xg[a] - xg[c]);
      for (int b = 0; b < nb; ++b)
        if (b != a && b != c) p *= (t - xg[b]) / (xg[a] - xg[b]);
      s += p;
    }
    return s;
  }
};

Lag1D lag1d(int deg) {
  Lag1D L;
  L.nb = deg + 1;
  const double r5 = 0.5 / std::sqrt(5.0);
  const double x1[4] = {0.0, 1.0, 0, 0}, x2[4] = {0.0, 0.5, 1.0, 0}, x3[4] = {0.0, 0.5 - r5, 0.5 + r5, 1.0};
  const double *x = deg == 1 ? x1 : (deg == 2 ? x2 : x3);
  for (int k = 0; k < 4; ++k) L.xg[k] = x[k];
  return L;
}

void split(int a, int nb, int *ai) {
  for (int e = 0; e < 3; ++e) {
    ai[e] = a % nb;
    a /= nb;
  }
}

// 1D shape functions of a cell map of degree g (1: the end points; 2: the
// points 0, 1/2, 1 of [0, 1]) and their derivatives.
double shape(int g, int q, double t) {
  if (g == 1) return q ? t : 1.0 - t;
  return q == 0 ? (1.0 - t) * (1.0 - 2.0 * t) : (q == 1 ? 4.0 * t * (1.0 - t) : t * (2.0 * t - 1.0));
}
double dshape(int g, int q, double t) {
  if (g == 1) return q ? 1.0 : -1.0;
  return q == 0 ? 4.0 * t - 3.0 : (q == 1 ? 4.0 - 8.0 * t : 4.0 * t - 1.0);
}

// Jacobian J[r][c] = dx_r/dxi_c at xi of the degree-g map through the cell's
// (g+1)^d points X (point v: digits q_e of v in base g + 1, the first axis
// lowest); its cofactor matrix cof = det(J) J^{-T}; returns det J.
double jacobian(int d, int g, const double (*X)[3], const double *xi, double cof[3][3]) {
  double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  int np = 1;
  for (int e = 0; e < d; ++e) np *= g + 1;
  for (int v = 0; v < np; ++v)
    for (int c = 0; c < d; ++c) {
      double w = 1.0;
      for (int e = 0, r = v; e < d; ++e, r /= g + 1)
        w *= e == c ? dshape(g, r % (g + 1), xi[e]) : shape(g, r % (g + 1), xi[e]);
      for (int r = 0; r < d; ++r) J[r][c] += w * X[v][r];
    }
  if (d == 1) {
    cof[0][0] = 1.0;
    return J[0][0];
  }
  if (d == 2) {
    cof[0][0] = J[1][1], cof[0][1] = -J[1][0];
    cof[1][0] = -J[0][1], cof[1][1] = J[0][0];
    return J[0][0] * J[1][1] - J[0][1] * J[1][0];
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      // the (r, c) cofactor: the 2 x 2 minor without row r and column c, signed
      const int r1 = (r + 1) % 3, r2 = (r + 2) % 3, c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      cof[r][c] = J[r1][c1] * J[r2][c2] - J[r1][c2] * J[r2][c1];
    }
  return J[0][0] * cof[0][0] + J[0][1] * cof[0][1] + J[0][2] * cof[0][2];
}

// Gauss-Jordan inverse with partial pivoting of an n x n matrix.
bool invert_n(int n, const double *A, double *Ai) {
  std::vector<double> M((size_t)n * 2 * n);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) M[r * 2 * n + c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(M[r * 2 * n + k]) > std::fabs(M[p * 2 * n + k])) p = r;
    if (M[p * 2 * n + k] == 0.0) return false;
    if (p != k)
      for (int c = 0; c < 2 * n; ++c) std::swap(M[k * 2 * n + c], M[p * 2 * n + c]);
    const double piv = M[k * 2 * n + k];
    for (int c = 0; c < 2 * n; ++c) M[k * 2 * n + c] /= piv;
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      const double f = M[r * 2 * n + k];
      if (f == 0.0) continue;
      for (int c = 0; c < 2 * n; ++c) M[r * 2 * n + c] -= f * M[k * 2 * n + c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Ai[r * n + c] = M[r * 2 * n + c + n];
  return true;
}

// body(begin, end) over [0, n) in contiguous ranges on up to 16 host threads
// (every index is computed by the same arithmetic whatever the split).
template <class F>
void parallel_ranges(int64_t n, F body) {
  int nt = (int)std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency()));
  if (n < 4096) nt = 1;
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(body, n * t / nt, n * (t + 1) / nt);
  body(0, n / nt);
  for (auto &x : th) x.join();
}

}  // namespace

int map_degree(const gdg_mesh_desc *m) { return m->map_degree == 2 ? 2 : 1; }

void gauss_rule01(int n, double *x, double *w) { gauss01(n, x, w); }

double map_jacobian(int d, int g, const double (*X)[3], const double *xi, double cof[3][3]) {
  return jacobian(d, g, X, xi, cof);
}

void mapped_cell_points(const gdg_mesh_desc *m, const double *vx, int64_t K, double (*X)[3]) {
  const int d = m->dim, g = map_degree(m);
  if (m->ucells > 0) {
    // unstructured: the cell's own point list
    int np = 1;
    for (int e = 0; e < d; ++e) np *= g + 1;
    for (int v = 0; v < np; ++v) {
      const int64_t id = m->ucell_points[K * np + v];
      for (int c = 0; c < 3; ++c) X[v][c] = c < d ? vx[id * d + c] : 0.0;
    }
    return;
  }
  int64_t ki[3] = {0, 0, 0}, r = K;
  for (int e = 0; e < d; ++e) {
    ki[e] = r % m->cells[e];
    r /= m->cells[e];
  }
  int np = 1;
  for (int e = 0; e < d; ++e) np *= g + 1;
  for (int v = 0; v < np; ++v) {
    int64_t idx = 0, stride = 1;
    for (int e = 0, q = v; e < d; ++e, q /= g + 1) {
      idx += (g * ki[e] + q % (g + 1)) * stride;
      stride *= g * m->cells[e] + 1;
    }
    for (int c = 0; c < 3; ++c) X[v][c] = c < d ? vx[idx * d + c] : 0.0;
  }
}

void mapped_point(int d, int g, const double (*X)[3], const double *xi, double *x) {
  for (int c = 0; c < d; ++c) x[c] = 0.0;
  int np = 1;
  for (int e = 0; e < d; ++e) np *= g + 1;
  for (int v = 0; v < np; ++v) {
    double w = 1.0;
    for (int e = 0, q = v; e < d; ++e, q /= g + 1) w *= shape(g, q % (g + 1), xi[e]);
    for (int c = 0; c < d; ++c) x[c] += w * X[v][c];
  }
}

namespace {

// A face of an unstructured mesh keyed by its sorted corner point ids.
struct FaceKey {
  int64_t id[4];
  int64_t K;
  int f;
  bool operator<(const FaceKey &o) const {
    for (int k = 0; k < 4; ++k)
      if (id[k] != o.id[k]) return id[k] < o.id[k];
    return K != o.K ? K < o.K : f < o.f;
  }
  bool same_face(const FaceKey &o) const { return std::equal(id, id + 4, o.id); }
};

// Point id of cell K at map position q (0 .. g per axis).
int64_t upoint(const gdg_mesh_desc *m, int64_t K, const int *q) {
  const int g = map_degree(m), d = m->dim;
  int np = 1, v = 0, st = 1;
  for (int e = 0; e < d; ++e) np *= g + 1;
  for (int e = 0; e < d; ++e) {
    v += q[e] * st;
    st *= g + 1;
  }
  return m->ucell_points[K * np + v];
}

// Map position of face f's point at in-face position t (0 .. g on the face's
// axes, the lower axis first): q_e = side * g on the face's own axis.
void face_point(int d, int g, int f, const int *t, int *q) {
  const int e = f / 2, side = f % 2;
  for (int a = 0, j = 0; a < d; ++a) q[a] = a == e ? side * g : t[j++];
}

}  // namespace

// Stencil of an unstructured mesh in the ELL layout: per row the in-cell
// nodes, then per local face the row lies on its neighbour's face nodes (by
// the position of each on this cell's face) or its boundary part; c_ij from
// the cell of the lower index, negated in the other row (reading R3).  The
// neighbour's face parametrization is this cell's turned by the symmetry
// that matches the two cells' face corners.
bool assemble_unstructured(const gdg_mesh_desc *m, const RefTables &T, int R, int W, int64_t nslots, int nloc,
                           int nface, const std::vector<int> &fnode, const std::vector<double> &cin,
                           const std::vector<double> &cfc, const std::vector<double> &cgh, MappedSetup *out,
                           std::string *err) {
  const int d = m->dim, deg = m->degree, g = map_degree(m), nb = deg + 1;
  const int64_t ncells = m->ucells, N = ncells * nloc;
  const int nfc = 1 << (d - 1);  // corners per face
  // 1. neighbours: faces with the same corner set
  std::vector<FaceKey> keys((size_t)ncells * 2 * d);
  for (int64_t K = 0; K < ncells; ++K)
    for (int f = 0; f < 2 * d; ++f) {
      FaceKey &k = keys[(size_t)K * 2 * d + f];
      for (int c = 0; c < 4; ++c) k.id[c] = -1;
      for (int c = 0; c < nfc; ++c) {
        int t[2] = {(c & 1) * g, ((c >> 1) & 1) * g}, q[3];
        face_point(d, g, f, t, q);
        k.id[c] = upoint(m, K, q);
      }
      std::sort(k.id, k.id + nfc);
      k.K = K;
      k.f = f;
    }
  std::vector<FaceKey> sorted = keys;
  std::sort(sorted.begin(), sorted.end());
  std::vector<int64_t> nbr((size_t)ncells * 2 * d, -1);
  std::vector<int> nbf((size_t)ncells * 2 * d, -1);
  for (size_t q = 0; q < sorted.size();) {
    size_t r = q + 1;
    while (r < sorted.size() && sorted[r].same_face(sorted[q])) ++r;
    if (r - q > 2) {
      *err = "a face is shared by more than two cells";
      return false;
    }
    if (r - q == 2) {
      const FaceKey &a = sorted[q], &b = sorted[q + 1];
      nbr[(size_t)a.K * 2 * d + a.f] = b.K, nbf[(size_t)a.K * 2 * d + a.f] = b.f;
      nbr[(size_t)b.K * 2 * d + b.f] = a.K, nbf[(size_t)b.K * 2 * d + b.f] = a.f;
    }
    q = r;
  }
  // 2. the symmetry between the two face parametrizations: corner c of this
  // face (bits on the face's axes) sits at corner c' of the neighbour's;
  // position t maps to o k + t_0 u + t_1 v, per face of each cell
  struct Orient { int o[2], u[2], v[2]; };
  std::vector<Orient> orient((size_t)ncells * 2 * d);
  for (int64_t K = 0; K < ncells; ++K)
    for (int f = 0; f < 2 * d; ++f) {
      const int64_t Kn = nbr[(size_t)K * 2 * d + f];
      if (Kn < 0) {
        const int8_t u = m->uface_bc[K * 2 * d + f];
        const int kind = u & 7, df = u >> 3;
        if (u < 0 || kind < GDG_BC_OUTFLOW || kind > GDG_BC_INOUTFLOW || df >= 2 * d) {
          *err = "a boundary face has no valid kind and data face in uface_bc";
          return false;
        }
        continue;
      }
      const int fn = nbf[(size_t)K * 2 * d + f];
      int cc[4][2];  // neighbour corner bits of each of this face's corners
      for (int c = 0; c < nfc; ++c) {
        int t[2] = {(c & 1) * g, ((c >> 1) & 1) * g}, q[3];
        face_point(d, g, f, t, q);
        const int64_t id = upoint(m, K, q);
        int found = -1;
        for (int c2 = 0; c2 < nfc && found < 0; ++c2) {
          int t2[2] = {(c2 & 1) * g, ((c2 >> 1) & 1) * g}, q2[3];
          face_point(d, g, fn, t2, q2);
          if (upoint(m, Kn, q2) == id) found = c2;
        }
        cc[c][0] = found & 1, cc[c][1] = (found >> 1) & 1;
      }
      Orient &o = orient[(size_t)K * 2 * d + f];
      for (int j = 0; j < 2; ++j) {
        o.o[j] = cc[0][j];
        o.u[j] = nfc > 1 ? cc[1][j] - cc[0][j] : 0;
        o.v[j] = nfc > 2 ? cc[2][j] - cc[0][j] : 0;
      }
      // every point of the face must agree (edge midpoints of curved faces)
      for (int t0 = 0; t0 <= g; ++t0)
        for (int t1 = 0; t1 <= (d == 3 ? g : 0); ++t1) {
          int t[2] = {t0, t1}, tn[2], q[3], qn[3];
          for (int j = 0; j < 2; ++j) tn[j] = o.o[j] * g + o.u[j] * t0 + o.v[j] * t1;
          face_point(d, g, f, t, q);
          face_point(d, g, fn, tn, qn);
          if (upoint(m, K, q) != upoint(m, Kn, qn)) {
            *err = "a face's points differ between its two cells";
            return false;
          }
        }
    }
  // position (t_0, t_1) on a face <-> index (first axis fastest), 0 .. nface-1
  auto pos_of = [&](int tb, int *t) { t[0] = tb % nb, t[1] = tb / nb; };
  auto index_of = [&](const int *t) { return t[0] + (d == 3 ? nb * t[1] : 0); };
  auto map_pos = [&](const Orient &o, const int *t, int *tn) {
    for (int j = 0; j < 2; ++j) tn[j] = o.o[j] * deg + o.u[j] * t[0] + o.v[j] * t[1];
  };
  // 3. rows
  out->col.assign((size_t)nslots, 0);
  out->meta.assign((size_t)nslots, (uint8_t)SK_PAD);
  out->kscale.assign(N, 0.0);
  const int64_t nblocks = nslots / ((int64_t)W * R);
  for (int64_t i = 0; i < nblocks * R; ++i) {
    const int64_t blk = i / R, lane = i % R;
    int t = 0;
    auto put = [&](int32_t col, const double *c, double sgn, uint8_t meta) {
      const int64_t s = (blk * W + t) * R + lane;
      out->col[s] = col;
      out->meta[s] = meta;
      for (int e = 0; e < d; ++e) out->c[(size_t)e * nslots + s] = c ? sgn * c[e] : 0.0;
      ++t;
    };
    if (i < N) {
      const int64_t K = i / nloc;
      const int a = (int)(i % nloc);
      int graph = 0;
      for (int b = 0; b < nloc; ++b) {
        put((int32_t)(K * nloc + b), &cin[((size_t)K * nloc * nloc + a * nloc + b) * d], 1.0,
            (uint8_t)(SK_CELL | (b << 3)));
        ++graph;
      }
      for (int f = 0; f < 2 * d; ++f) {
        if (!T.onface[f * kMaxNloc + a]) continue;
        int ta = 0;
        while (fnode[f * nface + ta] != a) ++ta;
        const int64_t Kn = nbr[(size_t)K * 2 * d + f];
        if (Kn < 0) {
          const int8_t u = m->uface_bc[K * 2 * d + f];
          put((int32_t)i, &cgh[(((size_t)K * 2 * d + f) * nloc + a) * d], 1.0,
              (uint8_t)(SK_GHOST | (bclass(u >> 3, u & 7) << 3)));
          continue;
        }
        const int fn = nbf[(size_t)K * 2 * d + f];
        const Orient &o = orient[(size_t)K * 2 * d + f];
        int tA[2], tAn[2];
        pos_of(ta, tA);
        map_pos(o, tA, tAn);
        const int tan_ = index_of(tAn);
        for (int tb = 0; tb < nface; ++tb) {
          int tB[2], tBn[2];
          pos_of(tb, tB);
          map_pos(o, tB, tBn);
          const int tbn = index_of(tBn);
          const int bn = fnode[fn * nface + tbn];  // the neighbour's node at this position
          const uint8_t kind = tb == ta ? SK_FACE_COLLOC : SK_FACE;
          if (K < Kn)
            put((int32_t)(Kn * nloc + bn), &cfc[((((size_t)K * 2 * d + f) * nface + ta) * nface + tb) * d], 1.0,
                kind);
          else
            put((int32_t)(Kn * nloc + bn), &cfc[((((size_t)Kn * 2 * d + fn) * nface + tbn) * nface + tan_) * d],
                -1.0, kind);
          ++graph;
        }
      }
      out->kscale[i] = (double)(graph + 1) / out->mrow[i];
    }
    while (t < W) put((int32_t)(i < N ? i : 0), nullptr, 0.0, (uint8_t)SK_PAD);
  }
  return true;
}

bool build_mapped(const gdg_mesh_desc *m, const gdg_params *p, const double *vx, const RefTables &T, int R, int W,
                  int64_t nslots, MappedSetup *out, std::string *err) {
  const int d = m->dim, deg = m->degree, nb = deg + 1;
  int nloc = 1;
  for (int e = 0; e < d; ++e) nloc *= nb;
  const int nface = nloc / nb;
  int64_t ncells = 1;
  for (int e = 0; e < d; ++e) ncells *= m->cells[e];
  if (m->ucells > 0) ncells = m->ucells;
  const int64_t N = ncells * nloc;
  const Lag1D L = lag1d(deg);
  // Gauss points per direction, exact for every integrand: with a map of
  // degree gm, det J has degree d gm - 1 per direction and the cofactors
  // (d - 1) gm, so the masses need deg + 2 points in 2D and deg + 3 in 3D
  // with quadratic maps, the stencil coefficients deg + 2
  const int gm = map_degree(m);
  const int nq = deg + 2 + (d == 3 && gm == 2 ? 1 : 0);
  double xq[5], wq[5];
  gauss01(nq, xq, wq);
  int nvol = 1, nsurf = 1;
  for (int e = 0; e < d; ++e) nvol *= nq;
  for (int e = 0; e + 1 < d; ++e) nsurf *= nq;

  out->mrow.assign(N, 0.0);
  out->cmblk.assign((size_t)ncells * nloc * nloc, 0.0);
  out->cminv.assign((size_t)ncells * nloc * nloc, 0.0);
  // per cell: in-cell c (nloc x nloc x d), each face's pair integrals from
  // this cell's side (2d faces x face node x neighbour face node x d), and the
  // boundary parts (2d faces x node x d)
  std::vector<double> cin((size_t)ncells * nloc * nloc * d), cfc((size_t)ncells * 2 * d * nface * nface * d),
      cgh((size_t)ncells * 2 * d * nloc * d);
  // face nodes of each face, in the order of T.bface for the neighbour side
  std::vector<int> fnode(2 * d * nface);
  for (int f = 0; f < 2 * d; ++f) {
    const int e = f / 2, side = f % 2;
    int t = 0;
    for (int a = 0; a < nloc; ++a) {
      int ai[3];
      split(a, nb, ai);
      if (ai[e] == side * deg) fnode[f * nface + t++] = a;
    }
  }
  std::vector<double> cvol(ncells, 0.0);  // |K|, summed in cell order below
  std::atomic<bool> ok{true};
  parallel_ranges(ncells, [&](int64_t K0, int64_t K1) {
  for (int64_t K = K0; K < K1; ++K) {
    double X[27][3];
    mapped_cell_points(m, vx, K, X);
    double *Mk = &out->cmblk[(size_t)K * nloc * nloc];
    double *Ck = &cin[(size_t)K * nloc * nloc * d];
    std::vector<double> Craw((size_t)nloc * nloc * d, 0.0);
    for (int q = 0; q < nvol; ++q) {
      double xi[3] = {0, 0, 0}, w = 1.0;
      int r = q;
      for (int e = 0; e < d; ++e) {
        xi[e] = xq[r % nq];
        w *= wq[r % nq];
        r /= nq;
      }
      double cof[3][3];
      const double det = jacobian(d, gm, X, xi, cof);
      if (!(det > 0.0)) ok = false;
      cvol[K] += w * det;
      double phv[64], gr[64][3];
      for (int a = 0; a < nloc; ++a) {
        int ai[3];
        split(a, nb, ai);
        double v = 1.0;
        for (int e = 0; e < d; ++e) v *= L.val(ai[e], xi[e]);
        phv[a] = v;
        for (int c = 0; c < d; ++c) {
          double g = 1.0;
          for (int e = 0; e < d; ++e) g *= e == c ? L.der(ai[e], xi[e]) : L.val(ai[e], xi[e]);
          gr[a][c] = g;
        }
      }
      for (int a = 0; a < nloc; ++a) {
        out->mrow[K * nloc + a] += w * phv[a] * det;
        for (int b = 0; b < nloc; ++b) {
          Mk[a * nloc + b] += w * phv[a] * phv[b] * det;
          for (int e = 0; e < d; ++e) {
            double gx = 0.0;
            for (int c = 0; c < d; ++c) gx += cof[e][c] * gr[b][c];
            Craw[(a * nloc + b) * d + e] += w * phv[a] * gx;
          }
        }
      }
    }
    // the cell's faces: n ds = sign cof(J) e_e dxi, column e of the cofactor matrix
    for (int f = 0; f < 2 * d; ++f) {
      const int e = f / 2, side = f % 2;
      const double sgn = side ? 1.0 : -1.0;
      for (int q = 0; q < nsurf; ++q) {
        double xi[3] = {0, 0, 0}, w = 1.0;
        int r = q;
        for (int g = 0; g < d; ++g) {
          if (g == e) {
            xi[g] = side ? 1.0 : 0.0;
            continue;
          }
          xi[g] = xq[r % nq];
          w *= wq[r % nq];
          r /= nq;
        }
        double cof[3][3];
        jacobian(d, gm, X, xi, cof);
        double ns[3];
        for (int c = 0; c < d; ++c) ns[c] = sgn * cof[c][e];
        for (int ta = 0; ta < nface; ++ta) {
          const int a = fnode[f * nface + ta];
          int ai[3];
          split(a, nb, ai);
          double va = 1.0;
          for (int g = 0; g < d; ++g)
            if (g != e) va *= L.val(ai[g], xi[g]);
          for (int c = 0; c < d; ++c) cgh[(((size_t)K * 2 * d + f) * nloc + a) * d + c] += 0.5 * w * va * ns[c];
          for (int tb = 0; tb < nface; ++tb) {
            // the same cell's node b on this face (c^{dK} of the in-cell pair)
            const int b = fnode[f * nface + tb];
            int bi[3];
            split(b, nb, bi);
            double vb = 1.0;
            for (int g = 0; g < d; ++g)
              if (g != e) vb *= L.val(bi[g], xi[g]);
            for (int c = 0; c < d; ++c) Craw[(a * nloc + b) * d + c] -= 0.5 * w * va * vb * ns[c];
            // the neighbour's node T.bface[f][tb] across this face: its trace
            // on the face is the same tensor of the other directions' values
            const int bn = T.bface[f * 9 + tb];
            int bni[3];
            split(bn, nb, bni);
            double vbn = 1.0;
            for (int g = 0; g < d; ++g)
              if (g != e) vbn *= L.val(bni[g], xi[g]);
            for (int c = 0; c < d; ++c)
              cfc[((((size_t)K * 2 * d + f) * nface + ta) * nface + tb) * d + c] += 0.5 * w * va * vbn * ns[c];
          }
        }
      }
    }
    // Lemma PropSkew as stored (reading R3): c_aa = 0, c_ba = -c_ab from a < b
    for (int a = 0; a < nloc; ++a)
      for (int b = 0; b < nloc; ++b)
        for (int e = 0; e < d; ++e)
          Ck[(a * nloc + b) * d + e] =
              a == b ? 0.0 : (a < b ? Craw[(a * nloc + b) * d + e] : -Craw[(b * nloc + a) * d + e]);
    if (!invert_n(nloc, Mk, &out->cminv[(size_t)K * nloc * nloc])) ok = false;
  }
  });
  if (!ok) {
    *err = "a mapped cell has a non-positive Jacobian determinant (inverted or degenerate corners)";
    return false;
  }
  double vol = 0.0;
  for (int64_t K = 0; K < ncells; ++K) vol += cvol[K];
  out->vol = vol;
  // per-row constants and the stencil in the ELL layout of k_fill: in-cell
  // nodes b = 0 .. nloc-1, then per face the node lies on either its boundary
  // part or the neighbour's face nodes in the order of T.bface, then pads
  const double pk = deg % 2 == 0 ? 0.5 : 0.0;
  out->relrow.resize(N);
  out->hprow.resize(N);
  out->kscale.resize(N);
  out->c.assign((size_t)d * nslots, 0.0);
  if (m->ucells > 0) {
    for (int64_t i = 0; i < N; ++i) {
      const double hh = std::pow(out->mrow[i] / vol, 1.0 / d);
      out->hprow[i] = p->c_k * std::pow(hh, pk);
      out->relrow[i] = p->c_r * std::pow(hh, p->p_r);
      if (!(out->relrow[i] < 1.0)) {
        *err = "relaxation c_r h^p_r >= 1: the lower bounds would not be positive";
        return false;
      }
    }
    return assemble_unstructured(m, T, R, W, nslots, nloc, nface, fnode, cin, cfc, cgh, out, err);
  }
  std::atomic<bool> relax_ok{true};
  parallel_ranges(N, [&](int64_t i0, int64_t i1) {
  for (int64_t i = i0; i < i1; ++i) {
    const int64_t K = i / nloc;
    const int a = (int)(i % nloc);
    const double hh = std::pow(out->mrow[i] / vol, 1.0 / d);
    out->hprow[i] = p->c_k * std::pow(hh, pk);
    out->relrow[i] = p->c_r * std::pow(hh, p->p_r);
    if (!(out->relrow[i] < 1.0)) {
      relax_ok = false;
      continue;
    }
    const int64_t blk = i / R, lane = i % R;
    int t = 0, graph = 0;
    auto put = [&](const double *c, double sgn) {
      const int64_t s = (blk * W + t) * R + lane;
      for (int e = 0; e < d; ++e) out->c[(size_t)e * nslots + s] = sgn * c[e];
      ++t;
    };
    for (int b = 0; b < nloc; ++b) {
      put(&cin[((size_t)K * nloc * nloc + a * nloc + b) * d], 1.0);
      ++graph;
    }
    int64_t ki[3] = {0, 0, 0}, r = K;
    for (int e = 0; e < d; ++e) {
      ki[e] = r % m->cells[e];
      r /= m->cells[e];
    }
    for (int f = 0; f < 2 * d; ++f) {
      if (!T.onface[f * kMaxNloc + a]) continue;
      const int e = f / 2, side = f % 2;
      int64_t kn[3] = {ki[0], ki[1], ki[2]};
      kn[e] += side ? 1 : -1;
      if (kn[e] < 0 || kn[e] >= m->cells[e]) {
        if (m->bc[f] != GDG_BC_PERIODIC) {
          put(&cgh[(((size_t)K * 2 * d + f) * nloc + a) * d], 1.0);
          continue;
        }
        kn[e] = (kn[e] + m->cells[e]) % m->cells[e];
      }
      int64_t Kn = 0, stride = 1;
      for (int g = 0; g < d; ++g) {
        Kn += kn[g] * stride;
        stride *= m->cells[g];
      }
      int ta = 0;
      while (fnode[f * nface + ta] != a) ++ta;
      for (int tb = 0; tb < nface; ++tb) {
        // the pair from the cell of the lower index (reading R3): from this
        // side if K < Kn, else minus the neighbour's integral over its face
        // f^1 (a cell that meets itself across a periodic axis: from side 1)
        if (K < Kn || (K == Kn && side == 1)) {
          put(&cfc[((((size_t)K * 2 * d + f) * nface + ta) * nface + tb) * d], 1.0);
        } else {
          const int bn = T.bface[f * 9 + tb];
          int tbn = 0;
          while (fnode[(f ^ 1) * nface + tbn] != bn) ++tbn;
          // in the neighbour's face list, node a of this cell is T.bface[f^1][.]
          int tan = 0;
          while (T.bface[(f ^ 1) * 9 + tan] != a) ++tan;
          put(&cfc[((((size_t)Kn * 2 * d + (f ^ 1)) * nface + tbn) * nface + tan) * d], -1.0);
        }
        ++graph;
      }
    }
    out->kscale[i] = (double)(graph + 1) / out->mrow[i];
  }
  });
  if (!relax_ok) {
    *err = "relaxation c_r h^p_r >= 1: the lower bounds would not be positive";
    return false;
  }
  return true;
}

}  // namespace gdg
