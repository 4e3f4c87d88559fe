// Continuous Q_k elements on a Cartesian box (App. B, eq. cijcidefCg):
//   c_ij   = int_Omega phi_i grad phi_j - 1/2 int_{dOmega} phi_i phi_j n,
//   c_i^d  = 1/2 int_{dOmega} phi_i n           (one part per box face),
//   m_i    = int_Omega phi_i.
// On the box every cell is the same scaled reference cell, so the integrals
// are tensor products of 1D integrals of the Gauss-Lobatto Lagrange basis
// (exact Gauss rules); general and curved cells (vertices, map_degree) take
// them through each cell's map (cofactors, Nanson's formula on faces, the
// exact Gauss rules of the discontinuous general cells).  Each cell's values
// are scattered to the global nodes it holds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "gdg.h"
#include "gdg_internal.h"

namespace gdg {

namespace {

// Gauss-Legendre points and weights on [0, 1] for n = 2 .. 4 (exact to degree
// 2n - 1: the products of two 1D basis functions of degree <= 3).
void gauss_n(int n, double *x, double *w) {
  if (n == 2) {
    const double r = 0.5 / std::sqrt(3.0);
    x[0] = 0.5 - r, x[1] = 0.5 + r, w[0] = w[1] = 0.5;
  } else if (n == 3) {
    const double r = 0.5 * std::sqrt(0.6);
    x[0] = 0.5 - r, x[1] = 0.5, x[2] = 0.5 + r;
    w[0] = w[2] = 5.0 / 18.0, w[1] = 8.0 / 18.0;
  } else {
    const double a = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2)), b = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
    x[0] = 0.5 - 0.5 * b, x[1] = 0.5 - 0.5 * a, x[2] = 0.5 + 0.5 * a, x[3] = 0.5 + 0.5 * b;
    w[1] = w[2] = 0.25 * (18.0 + std::sqrt(30.0)) / 18.0, w[0] = w[3] = 0.25 * (18.0 - std::sqrt(30.0)) / 18.0;
  }
}

struct Basis1D {
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

}  // namespace

void cg_nodes(const gdg_mesh_desc *m, int64_t *gn) {
  for (int e = 0; e < 3; ++e)
    gn[e] = e < m->dim ? m->degree * m->cells[e] + (m->bc[2 * e] == GDG_BC_PERIODIC ? 0 : 1) : 1;
}

bool build_cg(const gdg_mesh_desc *m, const gdg_params *p, int R, int W, int64_t nslots, MappedSetup *out,
              std::string *err) {
  const int d = m->dim, k = m->degree, nb = k + 1;
  int nloc = 1, span = 1;
  for (int e = 0; e < d; ++e) nloc *= nb, span *= 2 * k + 1;
  int64_t gn[3];
  cg_nodes(m, gn);
  const int64_t N = gn[0] * gn[1] * gn[2];
  double h[3] = {1, 1, 1}, vol = 1.0;
  for (int e = 0; e < d; ++e) {
    h[e] = (m->hi[e] - m->lo[e]) / (double)m->cells[e];
    vol *= m->hi[e] - m->lo[e];
  }
  // 1D reference integrals: M_ab = int L_a L_b, G_ab = int L_a L_b', w_a = int L_a
  Basis1D B;
  B.nb = nb;
  const double r5 = 0.5 / std::sqrt(5.0);
  const double x1[4] = {0.0, 1.0, 0, 0}, x2[4] = {0.0, 0.5, 1.0, 0}, x3[4] = {0.0, 0.5 - r5, 0.5 + r5, 1.0};
  const double *xg = k == 1 ? x1 : (k == 2 ? x2 : x3);
  for (int q = 0; q < 4; ++q) B.xg[q] = xg[q];
  double xq[4], wq[4];
  const int nq = k + 1;
  gauss_n(nq, xq, wq);
  double M1[4][4] = {}, G1[4][4] = {}, w1[4] = {};
  for (int q = 0; q < nq; ++q)
    for (int a = 0; a < nb; ++a) {
      w1[a] += wq[q] * B.val(a, xq[q]);
      for (int b = 0; b < nb; ++b) {
        M1[a][b] += wq[q] * B.val(a, xq[q]) * B.val(b, xq[q]);
        G1[a][b] += wq[q] * B.val(a, xq[q]) * B.der(b, xq[q]);
      }
    }
  // per row: c over the (2k+1)^d offsets, the boundary parts per box face
  std::vector<double> cc((size_t)N * span * d, 0.0), cb((size_t)N * 2 * d * d, 0.0);
  std::vector<uint8_t> used((size_t)N * span, 0), onb((size_t)N * 2 * d, 0);
  out->mrow.assign(N, 0.0);
  int64_t ncells = 1;
  for (int e = 0; e < d; ++e) ncells *= m->cells[e];
  // general cells: per cell, int phi_a cof(J) grad phi_b, int phi_a det J,
  // and on each face int phi_a phi_b n ds and int phi_a n ds
  const int gm = map_degree(m);
  const int nqm = k + 2 + (d == 3 && gm == 2 ? 1 : 0);
  double xqm[5], wqm[5];
  if (m->vertices) gauss_rule01(nqm, xqm, wqm);
  std::vector<double> gv(nloc * nloc * d), gmass(nloc), gfp(2 * d * nloc * nloc * d), gfs(2 * d * nloc * d);
  double gvol = 0.0;
  auto general_cell = [&](int64_t K) -> bool {
    double X[27][3];
    mapped_cell_points(m, m->vertices, K, X);
    std::fill(gv.begin(), gv.end(), 0.0);
    std::fill(gmass.begin(), gmass.end(), 0.0);
    std::fill(gfp.begin(), gfp.end(), 0.0);
    std::fill(gfs.begin(), gfs.end(), 0.0);
    int nvol = 1;
    for (int e = 0; e < d; ++e) nvol *= nqm;
    double phv[64], gr[64][3];
    auto basis = [&](const double *xi) {
      for (int a = 0; a < nloc; ++a) {
        int ai[3] = {0, 0, 0};
        for (int e = 0, q = a; e < d; ++e, q /= nb) ai[e] = q % nb;
        double v = 1.0;
        for (int e = 0; e < d; ++e) v *= B.val(ai[e], xi[e]);
        phv[a] = v;
        for (int c = 0; c < d; ++c) {
          double g = 1.0;
          for (int e = 0; e < d; ++e) g *= e == c ? B.der(ai[e], xi[e]) : B.val(ai[e], xi[e]);
          gr[a][c] = g;
        }
      }
    };
    for (int q = 0; q < nvol; ++q) {
      double xi[3] = {0, 0, 0}, w = 1.0, cof[3][3];
      for (int e = 0, r = q; e < d; ++e, r /= nqm) xi[e] = xqm[r % nqm], w *= wqm[r % nqm];
      const double det = map_jacobian(d, gm, X, xi, cof);
      if (!(det > 0.0)) return false;
      gvol += w * det;
      basis(xi);
      for (int a = 0; a < nloc; ++a) {
        gmass[a] += w * phv[a] * det;
        for (int b = 0; b < nloc; ++b)
          for (int e = 0; e < d; ++e) {
            double gx = 0.0;
            for (int c = 0; c < d; ++c) gx += cof[e][c] * gr[b][c];
            gv[(a * nloc + b) * d + e] += w * phv[a] * gx;
          }
      }
    }
    int nsurf = 1;
    for (int e = 0; e + 1 < d; ++e) nsurf *= nqm;
    for (int f = 0; f < 2 * d; ++f) {
      const int e = f / 2, side = f % 2;
      for (int q = 0; q < nsurf; ++q) {
        double xi[3] = {0, 0, 0}, w = 1.0, cof[3][3];
        for (int g = 0, r = q; g < d; ++g) {
          if (g == e) {
            xi[g] = side ? 1.0 : 0.0;
            continue;
          }
          xi[g] = xqm[r % nqm], w *= wqm[r % nqm], r /= nqm;
        }
        map_jacobian(d, gm, X, xi, cof);
        basis(xi);
        for (int a = 0; a < nloc; ++a) {
          for (int c = 0; c < d; ++c) gfs[(f * nloc + a) * d + c] += w * phv[a] * (side ? 1.0 : -1.0) * cof[c][e];
          for (int b = 0; b < nloc; ++b)
            for (int c = 0; c < d; ++c)
              gfp[((f * nloc + a) * nloc + b) * d + c] += w * phv[a] * phv[b] * (side ? 1.0 : -1.0) * cof[c][e];
        }
      }
    }
    return true;
  };
  for (int64_t K = 0; K < ncells; ++K) {
    int64_t ki[3] = {0, 0, 0}, r = K;
    for (int e = 0; e < d; ++e) ki[e] = r % m->cells[e], r /= m->cells[e];
    if (m->vertices && !general_cell(K)) {
      *err = "a mapped cell has a non-positive Jacobian determinant (inverted or degenerate corners)";
      return false;
    }
    for (int a = 0; a < nloc; ++a) {
      int ai[3] = {0, 0, 0};
      for (int e = 0, q = a; e < d; ++e, q /= nb) ai[e] = q % nb;
      int64_t i = 0, st = 1;
      for (int e = 0; e < d; ++e) {
        int64_t ge = k * ki[e] + ai[e];
        if (ge == gn[e]) ge = 0;  // periodic axis: the last node is the first
        i += ge * st;
        st *= gn[e];
      }
      double ma = 1.0;
      for (int e = 0; e < d; ++e) ma *= h[e] * w1[ai[e]];
      out->mrow[i] += m->vertices ? gmass[a] : ma;
      for (int b = 0; b < nloc; ++b) {
        int bi[3] = {0, 0, 0};
        for (int e = 0, q = b; e < d; ++e, q /= nb) bi[e] = q % nb;
        int off = 0;
        for (int e = 0, st2 = 1; e < d; ++e, st2 *= 2 * k + 1) off += (bi[e] - ai[e] + k) * st2;
        used[(size_t)i * span + off] = 1;
        for (int e = 0; e < d; ++e) {
          // int_K phi_a d_e phi_b: G in direction e (the 1/h_e of the
          // derivative cancels the h_e of the measure), M h elsewhere
          double v = G1[ai[e]][bi[e]];
          for (int g = 0; g < d; ++g)
            if (g != e) v *= h[g] * M1[ai[g]][bi[g]];
          cc[((size_t)i * span + off) * d + e] += m->vertices ? gv[(a * nloc + b) * d + e] : v;
        }
      }
      // the cell's faces on box faces (not periodic)
      for (int f = 0; f < 2 * d; ++f) {
        const int e = f / 2, side = f % 2;
        if (m->bc[f] == GDG_BC_PERIODIC) continue;
        if (ki[e] != (side ? m->cells[e] - 1 : 0) || ai[e] != side * k) continue;
        const double n = side ? 1.0 : -1.0;
        onb[(size_t)i * 2 * d + f] = 1;
        double wa = 1.0;
        for (int g = 0; g < d; ++g)
          if (g != e) wa *= h[g] * w1[ai[g]];
        if (m->vertices)
          for (int c = 0; c < d; ++c) cb[((size_t)i * 2 * d + f) * d + c] += 0.5 * gfs[(f * nloc + a) * d + c];
        else
          cb[((size_t)i * 2 * d + f) * d + e] += 0.5 * n * wa;
        for (int b = 0; b < nloc; ++b) {
          int bi[3] = {0, 0, 0};
          for (int g = 0, q = b; g < d; ++g, q /= nb) bi[g] = q % nb;
          if (bi[e] != side * k) continue;
          int off = 0;
          for (int g = 0, st2 = 1; g < d; ++g, st2 *= 2 * k + 1) off += (bi[g] - ai[g] + k) * st2;
          double v = 1.0;
          for (int g = 0; g < d; ++g)
            if (g != e) v *= h[g] * M1[ai[g]][bi[g]];
          if (m->vertices)
            for (int c = 0; c < d; ++c)
              cc[((size_t)i * span + off) * d + c] -= 0.5 * gfp[((f * nloc + a) * nloc + b) * d + c];
          else
            cc[((size_t)i * span + off) * d + e] -= 0.5 * n * v;
        }
      }
    }
  }
  // node of row i at offset o (periodic wrap), or -1 outside the box
  auto neighbour = [&](int64_t i, int o) -> int64_t {
    int64_t gi[3] = {0, 0, 0}, r = i, j = 0, st = 1;
    for (int e = 0; e < d; ++e) gi[e] = r % gn[e], r /= gn[e];
    for (int e = 0; e < d; ++e, o /= 2 * k + 1) {
      int64_t ge = gi[e] + o % (2 * k + 1) - k;
      if (m->bc[2 * e] == GDG_BC_PERIODIC) ge = (ge + gn[e]) % gn[e];
      if (ge < 0 || ge >= gn[e]) return -1;
      j += ge * st;
      st *= gn[e];
    }
    return j;
  };
  if (m->vertices) vol = gvol;
  out->vol = vol;
  const double pk = k % 2 == 0 ? 0.5 : 0.0;
  out->hprow.resize(N);
  out->relrow.resize(N);
  out->kscale.assign(N, 0.0);
  out->c.assign((size_t)d * nslots, 0.0);
  out->col.assign((size_t)nslots, 0);
  out->meta.assign((size_t)nslots, (uint8_t)SK_PAD);
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
      const double hh = std::pow(out->mrow[i] / vol, 1.0 / d);
      out->hprow[i] = p->c_k * std::pow(hh, pk);
      out->relrow[i] = p->c_r * std::pow(hh, p->p_r);
      int graph = 0;
      const double zero[3] = {0, 0, 0};
      for (int o = 0; o < span; ++o) {
        if (!used[(size_t)i * span + o]) continue;
        const int64_t j = neighbour(i, o);
        ++graph;
        if (j == i) {
          put((int32_t)j, zero, 1.0, (uint8_t)SK_FACE);  // c_ii = 0 (reading R3)
          continue;
        }
        // reading R3: from the lower index; the other row stores -c_ji
        if (i < j) {
          put((int32_t)j, &cc[((size_t)i * span + o) * d], 1.0, (uint8_t)SK_FACE);
        } else {
          const int oj = span - 1 - o;  // the opposite offset, j -> i
          put((int32_t)j, &cc[((size_t)j * span + oj) * d], -1.0, (uint8_t)SK_FACE);
        }
      }
      for (int f = 0; f < 2 * d; ++f)
        if (onb[(size_t)i * 2 * d + f])
          put((int32_t)i, &cb[((size_t)i * 2 * d + f) * d], 1.0,
              (uint8_t)(SK_GHOST | (bclass(f, m->bc[f]) << 3)));
      out->kscale[i] = (double)(graph + 1) / out->mrow[i];
      if (!(out->relrow[i] < 1.0)) {
        *err = "relaxation c_r h^p_r >= 1: the lower bounds would not be positive";
        return false;
      }
    }
    if (t > W) {
      *err = "internal: continuous stencil wider than its rows";
      return false;
    }
    while (t < W) put((int32_t)(i < N ? i : 0), nullptr, 0.0, (uint8_t)SK_PAD);
  }
  return true;
}

}  // namespace gdg
