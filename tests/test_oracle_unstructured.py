"""Pins of the oracle on unstructured meshes: cells given by their own point
lists, neighbours found by shared face corners, the neighbour's basis
evaluated through the inverse of its map (so any relative orientation of two
cells is handled), collocated partners found by position.

* A lattice mesh written as an unstructured one, with the cells shuffled and
  each cell's local axes turned by a random rotation of the reference cell,
  gives the lattice mesh's masses and c_ij pair by pair, and its stage and
  steps dof by dof (2D Q1-Q3, 3D Q1-Q2, curved 2D Q2; walls only, since
  cells connect through shared points only).
* A triangle cut into three quadrilateral blocks (a point with three cells):
  Lemma LemPart, Lemma PropSkew and the mass row sums row by row, the area,
  one collocated partner per face node, and mass and energy kept to rounding
  over ten steps inside slip walls (Lemma TotBalLemma).
* A face on three cells and boundary parts without a kind are refused.
"""
import numpy as np
import pytest

from paper_2402_04514_amd import workloads as W


def _smooth(x, dim, seed=3):
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, size=(4, dim))
    f = lambda r: np.sum(np.sin(2 * np.pi * x + ph[r]), axis=1) / dim
    vel = np.stack([0.3 * f(1 + (e % 2)) for e in range(dim)])
    return W.to_conserved(1.0 + 0.3 * f(0), vel, 1.0 + 0.4 * f(3))


def _dof_map(A, B, perm, nloc):
    """mp[i]: the dof of B at the same point of the same cell as dof i of A."""
    xa, xb = A.coords(), B.coords()
    mp = np.zeros(A.ndofs, dtype=np.int64)
    for i in range(A.ndofs):
        Kb = perm[i // nloc]
        d = np.abs(xb[Kb * nloc:(Kb + 1) * nloc] - xa[i]).max(axis=1)
        assert d.min() < 1e-12
        mp[i] = Kb * nloc + int(np.argmin(d))
    assert len(set(mp.tolist())) == A.ndofs
    return mp


CASES = {
    "2d_q1_walls": (2, 1, (6, 5), (1, 2, 2, 1), 1),
    "2d_q2_walls": (2, 2, (5, 4), (2, 2, 2, 1), 1),
    "2d_q3": (2, 3, (3, 3), (2, 1, 1, 2), 1),
    "3d_q1_walls": (3, 1, (4, 3, 3), (1, 2, 2, 1, 2, 1), 1),
    "3d_q2": (3, 2, (2, 2, 2), (2, 1, 1, 2, 2, 1), 1),
    "2d_q2_curved": (2, 2, (4, 4), (1, 2, 2, 1), 2),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_renumbered_lattice_gives_the_lattice_result(oracle, name):
    dim, k, cells, bc, g = CASES[name]
    lo, hi = (0.0,) * dim, (1.0,) * dim
    V = W.perturbed_lattice(cells, lo, hi, amp=0.2, seed=7)
    if g == 2:
        V = W.refine_points(V, cells)
        V[:, 0] += 0.01 * np.sin(3 * np.pi * V[:, 0]) * np.sin(np.pi * V[:, 1])  # curved cells
    A = oracle.Mesh(dim, k, cells, lo, hi, bc, vertices=V, map_degree=g)
    cp, P, fb, perm, rot = W.unstructured_from_lattice(cells, V, bc, map_degree=g, seed=5)
    B = oracle.Mesh.unstructured(dim, k, cp, P, fb, map_degree=g)
    nloc = (k + 1) ** dim
    mp = _dof_map(A, B, perm, nloc)
    assert np.abs(A.lumped() - B.lumped()[mp]).max() < 1e-15
    ra, ca, cca, ma, ka = A.csr()
    rb, cb, ccb, mb, kb = B.csr()
    for i in range(A.ndofs):
        ib = mp[i]
        pairs_b = {int(cb[q]): (ccb[q], mb[q], kb[q]) for q in range(rb[ib], rb[ib + 1])}
        assert rb[ib + 1] - rb[ib] == ra[i + 1] - ra[i]
        for q in range(ra[i], ra[i + 1]):
            cbq, mbq, kbq = pairs_b[int(mp[ca[q]])]
            assert np.abs(cbq - cca[q]).max() < 1e-15 and abs(mbq - ma[q]) < 1e-15 and kbq == ka[q]
    ba, bb = A.boundary(), B.boundary()
    assert len(ba[1]) == len(bb[1])
    U = _smooth(A.coords(), dim)
    Ub = np.zeros_like(U)
    Ub[:, mp] = U
    op = oracle.params(degree=k)
    oa, _ = A.stage(op, U, diag=True)
    ob, _ = B.stage(op, Ub, diag=True)
    scale = np.abs(oa).max(axis=1, keepdims=True)
    assert (np.abs(ob[:, mp] - oa) / scale).max() < 1e-12
    Ua, ta, na = A.run_to(op, U, 1.0, max_steps=3)
    Ubb, tb, nb = B.run_to(op, Ub, 1.0, max_steps=3)
    assert na == nb == 3 and tb == pytest.approx(ta, rel=1e-13)
    assert (np.abs(Ubb[:, mp] - Ua) / scale).max() < 1e-11


def _triangle(oracle, k, n=4, g=1, kind=2):
    cp, P, fb = W.triangle_three_blocks(n, map_degree=g)
    # boundary kinds on the faces without a neighbour (corner pairs that
    # appear once)
    keys = {}
    for K in range(len(cp)):
        for f in range(4):
            e, side = f // 2, f % 2
            vs = []
            for v in range(4):
                if ((v >> e) & 1) != side:
                    continue
                qi, qj = (v & 1) * g, ((v >> 1) & 1) * g
                vs.append(int(cp[K, qj * (g + 1) + qi]))
            keys.setdefault(tuple(sorted(vs)), []).append((K, f))
    for lst in keys.values():
        if len(lst) == 1:
            K, f = lst[0]
            fb[K, f] = kind
    return oracle.Mesh.unstructured(2, k, cp, P, fb, map_degree=g), cp


@pytest.mark.parametrize("k", [1, 2, 3])
def test_three_block_triangle(oracle, k):
    M, cp = _triangle(oracle, k)
    area = 0.5 * abs(1.0 * 0.9 - 0.0 * 0.3)
    assert M.volume == pytest.approx(area, rel=1e-13)
    rp, col, cc, mij, kind = M.csr()
    bp, bf, bcc = M.boundary()
    N = M.ndofs
    rows = np.repeat(np.arange(N), np.diff(rp))
    part = np.zeros((N, 2))
    np.add.at(part, rows, cc)
    np.add.at(part, np.repeat(np.arange(N), np.diff(bp)), bcc)
    scale = np.abs(cc).max()
    assert np.abs(part).max() < 1e-13 * scale, "Lemma LemPart"
    msum = np.zeros(N)
    np.add.at(msum, rows, mij)
    assert np.abs(msum - M.lumped()).max() < 1e-13 * M.lumped().max()
    rng = np.random.default_rng(4)
    for q in rng.choice(len(col), size=min(300, len(col)), replace=False):
        i, j = rows[q], col[q]
        assert np.abs(M.literal_cij(i, j) + M.literal_cij(j, i)).max() < 1e-13 * scale
    # collocated pairs (kind 1) join nodes at the same point, and every node
    # on a face shared with another cell has one such partner per shared face
    x = M.coords()
    colloc = kind == 1
    assert np.abs(x[rows[colloc]] - x[col[colloc]]).max() < 1e-12
    cross = col // ((k + 1) ** 2) != rows // ((k + 1) ** 2)
    same_point = np.abs(x[rows] - x[col]).max(axis=1) < 1e-12
    assert np.array_equal(colloc, cross & same_point)
    # mass and energy inside slip walls
    U = _smooth(x, 2)
    op = oracle.params(degree=k)
    Un, _, n = M.run_to(op, U, 1.0, max_steps=10)
    mi = M.lumped()
    for c in (0, 3):
        t0, t1 = (U[c] * mi).sum(), (Un[c] * mi).sum()
        assert abs(t1 - t0) <= 1e-13 * abs(t0)


def test_curved_three_block_triangle_has_the_same_area(oracle):
    M, _ = _triangle(oracle, 2, n=3, g=2)
    assert M.volume == pytest.approx(0.45, rel=1e-13)


def test_refused_meshes(oracle):
    cp, P, fb = W.triangle_three_blocks(2)
    with pytest.raises(ValueError):  # boundary faces without a kind
        oracle.Mesh.unstructured(2, 1, cp, P, fb)
    M, cp1 = _triangle(oracle, 1, n=2)
    # a fourth cell on an existing interior face: three cells on one face
    extra = cp1[:1].copy()
    cp2 = np.concatenate([cp1, extra])
    fb2 = np.full((len(cp2), 4), 2, dtype=np.int8)
    with pytest.raises(ValueError):
        oracle.Mesh.unstructured(2, 1, cp2, W.triangle_three_blocks(2)[1], fb2)
