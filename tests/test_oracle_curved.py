"""Pins of the oracle on curved cells: each cell the image of the reference
cell under the tensor-product quadratic map through its 3^d points (corners,
edge and face midpoints, centre), the stencil of Sec. 2.3 integrated through
that map.

* Quadratic points placed by multilinear interpolation of a multilinear
  mesh's corners give that mesh's c_ij, m_ij, c_i^d and node coordinates.
* The area of an O-grid annulus with its points on circles converges to
  pi (r1^2 - r0^2) at fourth order (quadratic cells) against second order
  (bilinear cells through the same corners).
* Lemma LemPart, Lemma PropSkew (c_ij against c_ji integrated separately) and
  sum_j m_ij = m_i row by row on curved 2D and 3D cells; the boundary parts
  along each closed circle of the annulus sum to zero.
* Limited Q2 converges at third order on the vortex over curved periodic
  cells.
"""
import math

import numpy as np
import pytest

from paper_2402_04514_amd import workloads as W

from test_oracle_scheme import _l1


def _shell(ntheta, nr, nz, r0=0.5, r1=1.0):
    """3D: the curved annulus O-grid extruded over z in [0, 0.5], quadratic
    points (x fastest: around, then outwards, then z)."""
    P = W.annulus_ogrid(ntheta, nr, r0, r1, map_degree=2)
    z = 0.5 * np.arange(2 * nz + 1) / (2 * nz)
    return np.concatenate([np.column_stack([P, np.full(len(P), zz)]) for zz in z])


def _curved_periodic(n, lo, hi, amp):
    """Quadratic points of the uniform box moved by the smooth periodic field
    amp h sin(2 pi xi_1) sin(2 pi xi_2) (+ on x, - on y): curved cells."""
    cells = (n, n)
    V = W.refine_points(W.lattice(cells, lo, hi), cells)
    h = (hi[0] - lo[0]) / n
    xi = (V - np.array(lo)) / (np.array(hi) - np.array(lo))
    s = np.prod(np.sin(2 * np.pi * xi), axis=1)
    V[:, 0] += amp * h * s
    V[:, 1] -= amp * h * s
    return V


MULTI = {
    "2d_q1": (2, 1, (5, 4)), "2d_q2": (2, 2, (4, 3)), "2d_q3": (2, 3, (3, 3)),
    "3d_q1": (3, 1, (3, 3, 2)), "3d_q2": (3, 2, (2, 2, 2)),
}


@pytest.mark.parametrize("name", sorted(MULTI))
def test_quadratic_points_of_multilinear_cells_give_the_multilinear_mesh(oracle, name):
    dim, k, cells = MULTI[name]
    lo, hi = (0.0,) * dim, (1.0,) * dim
    bc = (1,) * (2 * dim)
    V = W.perturbed_lattice(cells, lo, hi, amp=0.25, seed=11)
    A = oracle.Mesh(dim, k, cells, lo, hi, bc, vertices=V)
    B = oracle.Mesh(dim, k, cells, lo, hi, bc, vertices=W.refine_points(V, cells), map_degree=2)
    ra, ca, cca, ma, _ = A.csr()
    rb, cb, ccb, mb, _ = B.csr()
    assert np.array_equal(ca, cb)
    assert np.abs(cca - ccb).max() < 1e-14 and np.abs(ma - mb).max() < 1e-14
    assert np.abs(A.boundary()[2] - B.boundary()[2]).max() < 1e-14
    assert np.abs(A.coords() - B.coords()).max() < 1e-14
    assert B.volume == pytest.approx(A.volume, rel=1e-13)


def test_annulus_area_converges_at_fourth_order(oracle):
    exact = math.pi * (1.0 - 0.25)
    err = {1: [], 2: []}
    for n in (8, 16, 32):
        for md in (1, 2):
            V = W.annulus_ogrid(n, n // 4, map_degree=md)
            M = oracle.Mesh(2, 1, (n, n // 4), (0, 0), (1, 1), (0, 0, 2, 2), vertices=V, map_degree=md)
            err[md].append(abs(M.volume - exact))
    r1 = [err[1][i] / err[1][i + 1] for i in range(2)]
    r2 = [err[2][i] / err[2][i + 1] for i in range(2)]
    assert all(3.5 < r < 4.5 for r in r1), (err, r1)
    assert all(r > 14.0 for r in r2), (err, r2)


CURVED = {
    "annulus_q1": (2, 1, (12, 3)), "annulus_q2": (2, 2, (10, 3)), "annulus_q3": (2, 3, (8, 2)),
    "shell_q1": (3, 1, (8, 2, 2)), "shell_q2": (3, 2, (6, 2, 1)),
}


@pytest.mark.parametrize("name", sorted(CURVED))
def test_identities_on_curved_cells(oracle, name):
    dim, k, cells = CURVED[name]
    if dim == 2:
        V = W.annulus_ogrid(*cells, map_degree=2)
        bc = (0, 0, 2, 2)
    else:
        V = _shell(*cells)
        bc = (0, 0, 2, 2, 2, 2)
    M = oracle.Mesh(dim, k, cells, (0.0,) * dim, (1.0,) * dim, bc, vertices=V, map_degree=2)
    rp, col, cc, mij, _ = M.csr()
    bp, bf, bcc = M.boundary()
    mi = M.lumped()
    N = M.ndofs
    rows = np.repeat(np.arange(N), np.diff(rp))
    part = np.zeros((N, dim))
    np.add.at(part, rows, cc)
    brow = np.repeat(np.arange(N), np.diff(bp))
    np.add.at(part, brow, bcc)
    scale = np.abs(cc).max()
    assert np.abs(part).max() < 1e-13 * scale, "Lemma LemPart"
    msum = np.zeros(N)
    np.add.at(msum, rows, mij)
    assert np.abs(msum - mi).max() < 1e-13 * mi.max()
    # Lemma PropSkew with both orders integrated, on a sample of pairs
    rng = np.random.default_rng(2)
    for q in rng.choice(len(col), size=min(300, len(col)), replace=False):
        i, j = rows[q], col[q]
        assert np.abs(M.literal_cij(i, j) + M.literal_cij(j, i)).max() < 1e-13 * scale
    # each closed circle (inner face 2, outer face 3) has boundary parts summing to 0
    for f in (2, 3):
        assert np.abs(bcc[bf == f].sum(axis=0)).max() < 1e-13 * scale


def test_vortex_converges_at_third_order_on_curved_cells(oracle):
    """Limited Q2 on the vortex (periodic [-5, 5]^2, the quadratic points moved
    by a smooth periodic field of a quarter cell, so every cell is curved) to
    t = 0.5: rates 2.57 then 3.11 between 8^2, 16^2 and 32^2 cells."""
    lo, hi = (-5.0, -5.0), (5.0, 5.0)
    errs = []
    for n in (8, 16, 32):
        M = oracle.Mesh(2, 2, (n, n), lo, hi, (0,) * 4, vertices=_curved_periodic(n, lo, hi, 0.25), map_degree=2)
        U0 = W.vortex_exact(M.coords(), 0.0)
        U, _, _ = M.run_to(oracle.params(degree=2), U0, 0.5)
        errs.append(_l1(M, U, W.vortex_exact(M.coords(), 0.5)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[0] > 2.3 and rates[1] > 2.8, (errs, rates)
