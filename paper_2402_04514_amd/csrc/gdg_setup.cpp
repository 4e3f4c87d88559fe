// gdg_setup.cpp -- host side of the stencil setup of libgdg (Sec. 2.3).
//
// The matrices of eq. mass_matrices, cij_def1 and cij_def2 on a uniform
// Cartesian mesh are tensor products of 1D reference quantities on [0, 1]:
//   M1[a][b] = int phi_a phi_b,  w1[a] = int phi_a,  C1[a][b] = int phi_b' phi_a
// with phi_a the Lagrange polynomials on the Gauss-Lobatto nodes.  They are
// integrated exactly here from the polynomial coefficients.  Integration by
// parts gives C1 + C1^T = [phi_a phi_b]_0^1, so the in-cell coefficient
// c^K - c^dK reduces per axis to the skew part (C1 - C1^T)/2 times the mass
// factors of the other axes; across a face c_ij = (1/2) n times the face mass;
// on the boundary c_i^{d,f} = (1/2) n times the face-lumped mass.  Skew
// symmetry (Lemma PropSkew) therefore holds exactly in floating point.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "gdg_internal.h"

namespace gdg {

namespace {

struct Poly {
  double c[4] = {0, 0, 0, 0};  // coefficients of 1, x, x^2, x^3
};

Poly mul_linear(const Poly &p, double root, double scale) {
  Poly r;
  for (int i = 0; i < 3; ++i) {
    r.c[i + 1] += p.c[i] * scale;
    r.c[i] -= p.c[i] * root * scale;
  }
  return r;
}

double integrate01(const Poly &a, const Poly &b, bool deriv_b) {
  double s = 0.0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double bj = b.c[j];
      int pj = j;
      if (deriv_b) {
        if (j == 0) continue;
        bj = j * b.c[j];
        pj = j - 1;
      }
      s += a.c[i] * bj / double(i + pj + 1);
    }
  return s;
}

double integrate01(const Poly &a) {
  double s = 0.0;
  for (int i = 0; i < 4; ++i) s += a.c[i] / double(i + 1);
  return s;
}

void invert(int n, const double *A, double *Ai) {
  double M[4][8];
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < 2 * n; ++c) M[r][c] = c < n ? A[r * n + c] : (c - n == r ? 1.0 : 0.0);
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(M[r][k]) > std::fabs(M[p][k])) p = r;
    if (p != k)
      for (int c = 0; c < 2 * n; ++c) std::swap(M[k][c], M[p][c]);
    double d = M[k][k];
    for (int c = 0; c < 2 * n; ++c) M[k][c] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == k) continue;
      double f = M[r][k];
      for (int c = 0; c < 2 * n; ++c) M[r][c] -= f * M[k][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Ai[r * n + c] = M[r][c + n];
}

struct Ref1D {
  int nb;
  double M[4][4], Minv[4][4], Cs[4][4], w[4];
};

Ref1D make_ref1d(int deg) {
  Ref1D R;
  R.nb = deg + 1;
  // Gauss-Lobatto nodes on [0, 1]
  double xg[4] = {0.0, 0.5, 1.0, 1.0};
  if (deg == 1) xg[1] = 1.0;
  if (deg == 3) {
    const double r = 0.5 / std::sqrt(5.0);
    xg[1] = 0.5 - r;
    xg[2] = 0.5 + r;
    xg[3] = 1.0;
  }
  Poly phi[4];
  for (int a = 0; a < R.nb; ++a) {
    Poly p;
    p.c[0] = 1.0;
    for (int b = 0; b < R.nb; ++b)
      if (b != a) p = mul_linear(p, xg[b], 1.0 / (xg[a] - xg[b]));
    phi[a] = p;
  }
  double C1[4][4];
  for (int a = 0; a < R.nb; ++a) {
    R.w[a] = integrate01(phi[a]);
    for (int b = 0; b < R.nb; ++b) {
      R.M[a][b] = integrate01(phi[a], phi[b], false);
      C1[a][b] = integrate01(phi[a], phi[b], true);
    }
  }
  for (int a = 0; a < R.nb; ++a)
    for (int b = 0; b < R.nb; ++b) R.Cs[a][b] = 0.5 * (C1[a][b] - C1[b][a]);
  double Mf[16], Mi[16];
  for (int a = 0; a < R.nb; ++a)
    for (int b = 0; b < R.nb; ++b) Mf[a * R.nb + b] = R.M[a][b];
  invert(R.nb, Mf, Mi);
  for (int a = 0; a < R.nb; ++a)
    for (int b = 0; b < R.nb; ++b) R.Minv[a][b] = Mi[a * R.nb + b];
  return R;
}

void multi(int a, int nb, int *ai) {
  for (int e = 0; e < 3; ++e) {
    ai[e] = a % nb;
    a /= nb;
  }
}

}  // namespace

// Fills the reference tables of a uniform mesh with cell sizes h[0..dim-1].
bool build_ref_tables(int dim, int deg, const double *h, RefTables *T, std::string *err) {
  if (dim < 1 || dim > 3 || deg < 1 || deg > 3 || (deg == 3 && dim == 3)) {
    *err = "dim must be 1..3 and degree 1..3 (degree 3 in 1D and 2D)";
    return false;
  }
  std::memset(T, 0, sizeof(RefTables));
  Ref1D R = make_ref1d(deg);
  const int nb = R.nb;
  int nloc = 1;
  for (int e = 0; e < dim; ++e) nloc *= nb;
  for (int a = 0; a < nloc; ++a) {
    int ai[3];
    multi(a, nb, ai);
    double ml = 1.0;
    for (int e = 0; e < dim; ++e) ml *= h[e] * R.w[ai[e]];
    T->mlump[a] = ml;
    for (int b = 0; b < nloc; ++b) {
      int bi[3];
      multi(b, nb, bi);
      double mm = 1.0, mi = 1.0;
      for (int e = 0; e < dim; ++e) {
        mm *= h[e] * R.M[ai[e]][bi[e]];
        mi *= R.Minv[ai[e]][bi[e]] / h[e];
      }
      T->mblk[a * nloc + b] = mm;
      T->minv[a * nloc + b] = mi;
      for (int e = 0; e < dim; ++e) {
        double v = R.Cs[ai[e]][bi[e]];
        for (int f = 0; f < dim; ++f)
          if (f != e) v *= h[f] * R.M[ai[f]][bi[f]];
        T->cin[(a * nloc + b) * kMaxD + e] = (a == b) ? 0.0 : v;
      }
    }
  }
  for (int f = 0; f < 2 * dim; ++f) {
    const int e = f / 2, side = f % 2;
    const double n = side ? 1.0 : -1.0;
    // nodes b of the neighbour on its touching face (b_e = (1 - side) k), lexicographic
    int t = 0;
    for (int b = 0; b < nloc; ++b) {
      int bi[3];
      multi(b, nb, bi);
      if (bi[e] != (1 - side) * deg) continue;
      T->bface[f * 9 + t] = b;
      ++t;
    }
    const int nface = t;
    for (int a = 0; a < nloc; ++a) {
      int ai[3];
      multi(a, nb, ai);
      if (ai[e] != side * deg) continue;
      T->onface[f * kMaxNloc + a] = 1;
      double gl = 0.5 * n;
      for (int g = 0; g < dim; ++g)
        if (g != e) gl *= h[g] * R.w[ai[g]];
      T->cghost[(f * kMaxNloc + a) * kMaxD + e] = gl;
      for (int tt = 0; tt < nface; ++tt) {
        int b = T->bface[f * 9 + tt], bi[3];
        multi(b, nb, bi);
        double v = 0.5 * n;
        int co = 1;
        for (int g = 0; g < dim; ++g)
          if (g != e) {
            v *= h[g] * R.M[ai[g]][bi[g]];
            if (ai[g] != bi[g]) co = 0;
          }
        T->cface[((f * kMaxNloc + a) * 9 + tt) * kMaxD + e] = v;
        T->colloc[(f * kMaxNloc + a) * 9 + tt] = co;
      }
    }
  }
  return true;
}

}  // namespace gdg
