"""Pins of the oracle's discretization setup (Sec. 2.3, Lemmas LemPart and
PropSkew) against hand-derived closed forms and the paper's identities."""
import json
import math
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "stencil_pins.json")))

MESHES = [
    # dim, k, cells, lo, hi, bc
    (1, 1, (6,), (0.0,), (1.0,), (1, 1)),
    (1, 2, (5,), (0.0,), (2.0,), (0, 0)),
    (2, 1, (4, 3), (0.0, -1.0), (1.0, 2.0), (1, 1, 2, 2)),
    (2, 1, (4, 4), (-5.0, -5.0), (5.0, 5.0), (0, 0, 0, 0)),
    (2, 2, (3, 4), (0.0, 0.0), (1.0, 1.0), (1, 1, 1, 1)),
    (2, 2, (3, 3), (0.0, 0.0), (1.0, 1.0), (0, 0, 1, 1)),
    (3, 1, (3, 2, 3), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (2, 2, 2, 2, 2, 2)),
    (3, 1, (2, 2, 2), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (0, 0, 1, 1, 2, 2)),
    (1, 3, (5,), (0.0,), (1.5,), (1, 1)),
    (2, 3, (3, 2), (0.0, 0.0), (1.0, 2.0), (1, 1, 2, 2)),
    (2, 3, (2, 3), (-1.0, -1.0), (1.0, 1.0), (0, 0, 0, 0)),
]


def _mesh(O, spec):
    return O.Mesh(*spec)


@pytest.mark.parametrize("spec", MESHES)
def test_partition_of_unity(oracle, spec):
    """Lemma LemPart: sum_j c_ij + c_i^d = 0 for every row."""
    M = _mesh(oracle, spec)
    rp, col, c, mij, kind = M.csr()
    bptr, bface, bcc = M.boundary()
    scale = np.abs(c).max()
    for i in range(M.ndofs):
        s = c[rp[i]:rp[i + 1]].sum(0) + bcc[bptr[i]:bptr[i + 1]].sum(0)
        assert np.all(np.abs(s) <= 1e-14 * scale), (i, s)


@pytest.mark.parametrize("spec", MESHES)
def test_skew_symmetry_literal(oracle, spec):
    """Lemma PropSkew on the literal integrals (both orders computed), and the
    stored matrix exactly skew with c_ii = 0."""
    M = _mesh(oracle, spec)
    rp, col, c, mij, kind = M.csr()
    scale = np.abs(c).max()
    lut = {}
    for i in range(M.ndofs):
        for k in range(rp[i], rp[i + 1]):
            lut[(i, int(col[k]))] = k
    for (i, j), k in lut.items():
        assert (j, i) in lut, "stencil not symmetric"
        if i == j:
            assert np.all(c[k] == 0.0)
            continue
        assert np.array_equal(c[k], -c[lut[(j, i)]])
        a, b = M.literal_cij(i, j), M.literal_cij(j, i)
        assert np.all(np.abs(a + b) <= 1e-14 * scale)
        assert np.all(np.abs(a - c[k]) <= 1e-15 * scale)


@pytest.mark.parametrize("spec", MESHES)
def test_mass_identities(oracle, spec):
    """sum_j m_ij = m_i (Sec. 5.3) and sum_i m_i = |Omega|; m_ij symmetric."""
    M = _mesh(oracle, spec)
    rp, col, c, mij, kind = M.csr()
    mi = M.lumped()
    for i in range(M.ndofs):
        assert abs(mij[rp[i]:rp[i + 1]].sum() - mi[i]) <= 1e-15 * mi[i] * 10
    assert abs(mi.sum() - M.volume) <= 1e-12 * M.volume
    assert np.all(mi > 0)


def test_q1_1d_closed_form(oracle):
    g = GOLD["q1_1d"]
    h = 0.25
    M = oracle.Mesh(1, 1, (4,), (0.0,), (1.0,), (1, 1))
    rp, col, c, mij, kind = M.csr()
    mi = M.lumped()
    bptr, bface, bcc = M.boundary()
    assert np.allclose(mi / h, g["m_i_over_h"][0], rtol=0, atol=1e-15)
    # node 2 = cell 1, left node; node 3 = cell 1, right node
    row = {int(col[k]): c[k, 0] for k in range(rp[2], rp[3])}
    assert row == pytest.approx({2: 0.0, 3: g["incell_c"][0][1],
                                 1: g["face_c_left_node_to_prev_cell_right_node"]}, abs=1e-15)
    row = {int(col[k]): c[k, 0] for k in range(rp[3], rp[4])}
    assert row == pytest.approx({2: g["incell_c"][1][0], 3: 0.0,
                                 4: g["face_c_right_node_to_next_cell_left_node"]}, abs=1e-15)
    assert bcc[bptr[0]:bptr[1], 0] == pytest.approx([g["boundary_c_left_end"]])
    assert bcc[bptr[7]:bptr[8], 0] == pytest.approx([g["boundary_c_right_end"]])
    assert bptr[1] - bptr[0] == 1 and bptr[7] - bptr[6] == 0


def test_q2_1d_closed_form(oracle):
    g = GOLD["q2_1d"]
    h = 0.5
    M = oracle.Mesh(1, 2, (4,), (0.0,), (2.0,), (0, 0))
    rp, col, c, mij, kind = M.csr()
    mi = M.lumped()
    K = 2
    for a in range(3):
        i = 3 * K + a
        assert mi[i] / h == pytest.approx(g["m_i_over_h"][a], abs=1e-15)
        got = {int(col[k]): (c[k, 0], mij[k]) for k in range(rp[i], rp[i + 1])}
        for b in range(3):
            cc, mm = got[3 * K + b]
            assert cc == pytest.approx(g["incell_c"][a][b], abs=1e-14)
            assert mm / h == pytest.approx(g["mij_over_h"][a][b], abs=1e-15)
    # end nodes couple to the neighbouring cell across the face with +-1/2
    i = 3 * K
    got = {int(col[k]): c[k, 0] for k in range(rp[i], rp[i + 1])}
    assert got[3 * (K - 1) + 2] == pytest.approx(-0.5, abs=1e-15)
    assert len(got) == 4


def test_q3_1d_closed_form(oracle):
    """1D Q3 on Gauss-Lobatto nodes {0, 1/2 -+ 1/(2 sqrt 5), 1}: the lumped
    masses are h times the four-point Gauss-Lobatto weights 1/12, 5/12, 5/12,
    1/12; m_ab and the in-cell c_ab = int phi_b' phi_a - (1/2)[phi_a phi_b n]
    over the cell's ends come from the Lagrange polynomials integrated exactly
    with an eight-point Gauss-Legendre rule from numpy (exact to degree 15,
    where these integrands have degree 6), independent of the oracle's
    four-point rule."""
    r = 0.5 / math.sqrt(5.0)
    x = [0.0, 0.5 - r, 0.5 + r, 1.0]
    gx, gw = np.polynomial.legendre.leggauss(8)
    gx, gw = 0.5 * (gx + 1.0), 0.5 * gw

    def val(a, t):
        v = np.ones_like(t)
        for b in range(4):
            if b != a:
                v = v * (t - x[b]) / (x[a] - x[b])
        return v

    def der(a, t):
        v = np.zeros_like(t)
        for c in range(4):
            if c == a:
                continue
            w = np.full_like(t, 1.0 / (x[a] - x[c]))
            for b in range(4):
                if b != a and b != c:
                    w = w * (t - x[b]) / (x[a] - x[b])
            v = v + w
        return v

    one, zero = np.array([1.0]), np.array([0.0])
    mass = lambda a, b: float(np.sum(gw * val(a, gx) * val(b, gx)))
    grad = lambda a, b: float(np.sum(gw * val(a, gx) * der(b, gx)))   # int phi_b' phi_a
    lump = lambda a: float(np.sum(gw * val(a, gx)))
    ends = lambda a, b: float(val(a, one)[0] * val(b, one)[0] - val(a, zero)[0] * val(b, zero)[0])
    h = 0.3
    M = oracle.Mesh(1, 3, (5,), (0.0,), (1.5,), (1, 1))
    rp, col, c, mij, kind = M.csr()
    mi = M.lumped()
    K = 2
    for a in range(4):
        i = 4 * K + a
        assert mi[i] / h == pytest.approx([1 / 12, 5 / 12, 5 / 12, 1 / 12][a], abs=1e-15)
        assert mi[i] / h == pytest.approx(lump(a), abs=1e-15)
        got = {int(col[k]): (c[k, 0], mij[k]) for k in range(rp[i], rp[i + 1])}
        for b in range(4):
            cc, mm = got[4 * K + b]
            assert cc == pytest.approx(grad(a, b) - 0.5 * ends(a, b), abs=5e-15)
            assert mm / h == pytest.approx(mass(a, b), abs=2e-15)
    # the end nodes couple across the faces with -+1/2 (phi_a = 1 there)
    got = {int(col[k]): c[k, 0] for k in range(rp[4 * K], rp[4 * K + 1])}
    assert got[4 * (K - 1) + 3] == pytest.approx(-0.5, abs=1e-15) and len(got) == 5
    got = {int(col[k]): c[k, 0] for k in range(rp[4 * K + 3], rp[4 * K + 4])}
    assert got[4 * (K + 1)] == pytest.approx(0.5, abs=1e-15) and len(got) == 5


def test_q1_2d_corner(oracle):
    g = GOLD["q1_2d_corner"]
    h = 0.25
    M = oracle.Mesh(2, 1, (4, 4), (0.0, 0.0), (1.0, 1.0), (1, 1, 1, 1))
    rp, col, c, mij, kind = M.csr()
    mi = M.lumped()
    K = 1 + 4 * 1  # interior cell (1, 1)
    i = 4 * K + 0
    row = {int(col[k]): (c[k] / h, kind[k]) for k in range(rp[i], rp[i + 1])}
    assert row[4 * K + 1][0] == pytest.approx(g["incell_x1"], abs=1e-15)
    assert row[4 * K + 2][0] == pytest.approx(g["incell_y1"], abs=1e-15)
    assert row[4 * K + 3][0] == pytest.approx(g["incell_xy"], abs=1e-15)
    Kx = K - 1  # x-low neighbour; its right nodes are local 1 (y=0) and 3 (y=1)
    assert row[4 * Kx + 1][0] == pytest.approx(g["face_x_colloc"], abs=1e-15)
    assert row[4 * Kx + 1][1] == oracle.KIND_FACE_COLLOC
    assert row[4 * Kx + 3][0] == pytest.approx(g["face_x_other"], abs=1e-15)
    assert row[4 * Kx + 3][1] == oracle.KIND_FACE
    Ky = K - 4
    assert row[4 * Ky + 2][0] == pytest.approx(g["face_y_colloc"], abs=1e-15)
    assert row[4 * Ky + 3][0] == pytest.approx(g["face_y_other"], abs=1e-15)
    assert len(row) == 8
    assert mi[i] / h ** 2 == pytest.approx(g["m_i_over_h2"], abs=1e-15)
    s = sum(np.linalg.norm(v[0]) for v in row.values())
    assert s == pytest.approx(g["sum_abs_c_over_h"], rel=1e-12)


def test_q1_3d_corner(oracle):
    g = GOLD["q1_3d_corner"]
    h = 1.0 / 3.0
    M = oracle.Mesh(3, 1, (3, 3, 3), (0.0,) * 3, (1.0,) * 3, (2,) * 6)
    rp, col, c, mij, kind = M.csr()
    mi = M.lumped()
    K = 1 + 3 * (1 + 3 * 1)  # centre cell
    i = 8 * K
    row = {int(col[k]): c[k] / h ** 2 for k in range(rp[i], rp[i + 1])}
    assert len(row) == 20
    assert row[8 * K + 1] == pytest.approx([g["incell_one_step"], 0, 0], abs=1e-15)
    assert row[8 * K + 3] == pytest.approx([g["incell_two_steps"]] * 2 + [0], abs=1e-15)
    assert row[8 * K + 7] == pytest.approx([g["incell_three_steps"]] * 3, abs=1e-15)
    Kx = K - 1  # local nodes with ax = 1: 1, 3, 5, 7
    assert row[8 * Kx + 1] == pytest.approx([g["face_colloc"], 0, 0], abs=1e-15)
    assert row[8 * Kx + 3] == pytest.approx([g["face_one_off"], 0, 0], abs=1e-15)
    assert row[8 * Kx + 7] == pytest.approx([g["face_two_off"], 0, 0], abs=1e-15)
    assert mi[i] / h ** 3 == pytest.approx(g["m_i_over_h3"], abs=1e-15)


def test_boundary_parts_multivalued(oracle):
    """Sec. 4.2: a corner dof of a box carries one boundary part per face,
    with c_i^{d,k} = (1/2) int phi_i n over that face only."""
    h = 0.5
    M = oracle.Mesh(3, 1, (2, 2, 2), (0.0,) * 3, (1.0,) * 3, (2,) * 6)
    bptr, bface, bcc = M.boundary()
    i = 0  # corner (0,0,0)
    assert list(bface[bptr[i]:bptr[i + 1]]) == [0, 2, 4]
    for t, f in enumerate([0, 2, 4]):
        v = np.zeros(3)
        v[f // 2] = -0.5 * h * h / 4.0
        assert bcc[bptr[i] + t] == pytest.approx(v, abs=1e-16)
    # stencil widths: corner 8 in-cell + 3 faces x 4 minus boundary faces
    rp = M.csr()[0]
    assert rp[1] - rp[0] == 8 + 3 * 4 - 3 * 4


def test_node_coords(oracle):
    M = oracle.Mesh(2, 2, (2, 3), (0.0, 1.0), (1.0, 4.0), (1, 1, 1, 1))
    x = M.coords()
    # dof 9 + 4 = local (1,1) of cell 1 (cx=1, cy=0): centre of [0.5,1]x[1,2]
    assert x[9 + 4] == pytest.approx([0.75, 1.5])
    assert x[0] == pytest.approx([0.0, 1.0])
    assert x[-1] == pytest.approx([1.0, 4.0])


def test_invalid_mesh_rejected(oracle):
    with pytest.raises(ValueError):
        oracle.Mesh(2, 1, (1, 4), (0, 0), (1, 1), (0, 0, 1, 1))  # periodic axis with 1 cell
    with pytest.raises(ValueError):
        oracle.Mesh(2, 1, (4, 4), (0, 0), (1, 1), (0, 1, 1, 1))  # half-periodic axis
