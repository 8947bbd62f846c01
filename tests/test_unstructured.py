"""Unstructured meshes (triangles, tetrahedra) as inputs of the method
(the blunt-wedge and truncated-plate cases of Sec. 4 run on unstructured
physical meshes).  CPU only: the generators' geometric invariants, and the
oracle's least-squares gradient and free-stream behaviour on them against
closed forms."""
import numpy as np
import pytest

from oracle import avs_oracle as O
from workloads import fields as F
from workloads import meshes as MM

WALLS2 = dict(left=0, right=0, bottom=0, top=0)


def meshes():
    return {
        'tri_box': MM.tri_box(9, 7, 11, lx=1.5, ly=1.0, sides=WALLS2, bcs=[(MM.WALL, (1, 0, 0, 1))]),
        'tet_box': MM.tet_box(4, 3, 3, 12, l=(1.0, 0.8, 0.6)),
        'wedge': MM.blunt_wedge(h_wall=0.2, growth=1.15, box=(-3.0, 10.0, -5.0, 5.0)),
    }


MESHES = meshes()


def per_cell_closure(m):
    acc = np.zeros((m['ncells'], m['dim']))
    lr = m['face_lr']
    An = m['face_area'][:, None] * m['face_nrm']
    np.add.at(acc, lr[:, 0], An)
    inner = lr[:, 1] >= 0
    np.add.at(acc, lr[inner, 1], -An[inner])
    return acc


@pytest.mark.parametrize("name", list(MESHES))
def test_cells_are_closed_and_faces_oriented(name):
    """Divergence theorem: sum_f sigma_if A_f n_f = 0 for every closed
    cell; the normal of an interior face points from L's centroid side to
    R's; unit normals; faces per cell within a simplex's count."""
    m = MESHES[name]
    D = m['dim']
    assert np.abs(per_cell_closure(m)).max() < 1e-13 * max(1.0, m['face_area'].max())
    np.testing.assert_allclose(np.linalg.norm(m['face_nrm'], axis=1), 1.0, rtol=0, atol=1e-14)
    lr = m['face_lr']
    inner = lr[:, 1] >= 0
    d = m['cell_ctr'][lr[inner, 1]] - m['cell_ctr'][lr[inner, 0]]
    assert np.all(np.sum(d * m['face_nrm'][inner], axis=1) > 0)
    # boundary normals point out of their cell
    b = ~inner
    out = m['face_ctr'][b] - m['cell_ctr'][lr[b, 0]]
    assert np.all(np.sum(out * m['face_nrm'][b], axis=1) > 0)
    cnt = np.bincount(np.concatenate([lr[:, 0], lr[inner, 1]]), minlength=m['ncells'])
    assert np.all(cnt == D + 1)
    assert np.all(lr[inner, 0] < lr[inner, 1])


def test_box_meshes_tile_their_box():
    t = MESHES['tri_box']
    assert t['ncells'] == 2 * 9 * 7 and abs(t['cell_vol'].sum() - 1.5) < 1e-13
    q = MESHES['tet_box']
    assert q['ncells'] == 6 * 4 * 3 * 3 and abs(q['cell_vol'].sum() - 0.48) < 1e-13
    # the boundary faces cover the box surface
    b = q['face_lr'][:, 1] < 0
    assert abs(q['face_area'][b].sum() - 2 * (0.8 + 0.48 + 0.6)) < 1e-13


def test_wedge_geometry():
    """The wedge mesh fills the rectangle minus the body: its wall is a
    polygon through outline points (Delaunay may skip an outline point
    where three consecutive ones form a triangle inside the body), so the
    fluid area and the wall length agree with the outline's to its chord
    error; the flanks keep the 10 degree half angle and the base the
    3.736 nose-radius height."""
    m = MESHES['wedge']
    body, xb = MM.wedge_outline(h=0.2)
    area_body, _ = MM._polygon(body)
    rect = 13.0 * 10.0
    assert abs(m['cell_vol'].sum() + area_body - rect) < 2e-3 * area_body
    wall = m['face_lr'][:, 1] == -1
    per = np.sum(np.hypot(*np.diff(np.vstack([body, body[:1]]), axis=0).T))
    assert abs(m['face_area'][wall].sum() - per) < 2e-3 * per
    # exact outline: tip at the origin, base height and flank slope
    assert abs(body[:, 0].min()) < 1e-12 and abs(body[:, 1].max() - 0.5 * 3.736) < 1e-12
    flank = body[(body[:, 1] > 1.0) & (body[:, 0] < xb - 1e-9)]
    slope = np.diff(flank[:, 1]) / np.diff(flank[:, 0])
    np.testing.assert_allclose(np.abs(slope), np.tan(np.radians(10.0)), rtol=1e-12)
    # every far-field face lies on the rectangle
    far = m['face_lr'][:, 1] == -2
    fc = m['face_ctr'][far]
    on = np.minimum.reduce([abs(fc[:, 0] + 3), abs(fc[:, 0] - 10), abs(fc[:, 1] + 5), abs(fc[:, 1] - 5)])
    assert far.any() and np.all(on < 1e-9)


def test_wedge_workload_size():
    """At its default resolution the wedge mesh has the cell count of the
    paper's unstructured blunt-wedge mesh within 1 % (Sec. 4.3 quotes
    11 905 cells)."""
    m = MM.blunt_wedge()
    assert abs(m['ncells'] - 11905) < 0.01 * 11905


@pytest.mark.parametrize("name", ['tri_box', 'tet_box'])
def test_lsq_gradient_on_simplices(name):
    """The least-squares gradient of a linear field is the field's slope
    projected onto the span of the cell's neighbour offsets (the full slope
    where they span the space, Sec. 2.3.3 with the pseudo-inverse for the
    rank-deficient corner cells)."""
    desc = MESHES[name]
    D = desc['dim']
    mesh = O.Mesh(desc)
    a = np.array([0.7, -1.3, 0.4][:D])
    lin = desc['cell_ctr'] @ a
    deficient = 0
    for i in range(mesh.nc):
        dx = np.array([desc['cell_ctr'][s.nbr] - desc['cell_ctr'][i] for s in mesh.slots[i] if s.nbr >= 0])
        g = sum(c * (lin[s.nbr] - lin[i]) for s, c in zip(mesh.slots[i], mesh.lsq[i]) if s.nbr >= 0)
        # projector onto the span of the offsets, from an orthonormal basis
        u, sv, _ = np.linalg.svd(dx.T, full_matrices=False)
        basis = u[:, sv > 1e-9 * sv[0]]
        deficient += basis.shape[1] < D
        np.testing.assert_allclose(g, basis @ (basis.T @ a), rtol=1e-10, atol=1e-10)
    if name == 'tet_box':
        assert deficient > 0          # the corner cells take the pseudo-inverse path


def rings(desc, k):
    """Cells at least ``k`` face-neighbour rings away from any boundary face."""
    lr = desc['face_lr']
    near = set(int(L) for L, R in lr if R < 0)
    front = set(near)
    nbrs = [[] for _ in range(desc['ncells'])]
    for L, R in lr:
        if R >= 0:
            nbrs[L].append(R)
            nbrs[R].append(L)
    for _ in range(k - 1):
        front = {n for c in front for n in nbrs[c]} - near
        near |= front
    return np.array(sorted(set(range(desc['ncells'])) - near))


@pytest.mark.parametrize("name", ['tri_box', 'tet_box'])
def test_uniform_state_is_kept_away_from_walls(name):
    """A uniform state on closed cells has no net transport (the face
    fluxes of a cell sum to (xi . sum_f A_f n_f) phi = 0): W is unchanged
    and the VDF stays the same in every cell beyond the two rings that the
    walls reach in one step."""
    desc = MESHES[name]
    D = desc['dim']
    vs = dict(dim=D, lo=(-5.0,) * D, hi=(5.0,) * D, base=(8,) * D if D == 2 else (4,) * D, max_level=1)
    gas = dict(R=1.0, Pr=2 / 3, omega=0.5, mu_ref=0.05, T_ref=1.0, model=1)
    prim = F.uniform(desc['ncells'], 1.1, (0.3, -0.2, 0.1)[:D], 1.2)
    o = O.Solver(desc, vs, gas, 2e-3, 1.0, prim)
    W0 = o.W.copy()
    o.step(1)
    far = rings(desc, 3)
    assert len(far) > 0
    np.testing.assert_allclose(o.W[far], W0[far], rtol=1e-13, atol=1e-14)
    spread = np.abs(o.phi[:, far] - o.phi[:, far[:1]]).max()
    assert spread < 1e-13 * np.abs(o.phi).max()
