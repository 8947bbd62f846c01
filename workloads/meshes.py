"""Seeded/synthetic physical meshes (geometry only).

Every generator returns a plain dict of NumPy arrays describing a finite-volume
mesh: cell volumes and centres, and a face list with the two adjacent cells,
area, unit normal (pointing from the first cell to the second), midpoint and
a periodic shift.  Nothing here knows about distribution functions, moments
or the kinetic scheme: this module is the common *input* of the CPU oracle and
of the GPU library, and it carries none of the method's arithmetic.

Conventions
-----------
* ``face_lr[f] = (L, R)``.  For a boundary face ``R = -1 - bc_id`` and the
  normal points out of the domain (out of ``L``).
* ``face_shift[f]`` is the vector to add to the centre of ``R`` so that it
  sits next to ``L`` (non-zero only across a periodic seam of a box).
* ``bc_kind``: 0 = isothermal diffuse wall, 1 = far field.
* ``bc_state[b] = (rho, U_1..U_D, T)``; for a wall ``rho`` is ignored.
* Faces of zero area (poles of a spherical grid) are omitted.
"""
from __future__ import annotations

import math

import numpy as np

WALL = 0
FARFIELD = 1


def _finish(dim, vol, ctr, faces, bcs, shape):
    lr = np.array([f[0] for f in faces], dtype=np.int64).reshape(-1, 2)
    area = np.array([f[1] for f in faces], dtype=np.float64)
    nrm = np.array([f[2] for f in faces], dtype=np.float64).reshape(-1, dim)
    fctr = np.array([f[3] for f in faces], dtype=np.float64).reshape(-1, dim)
    shift = np.array([f[4] for f in faces], dtype=np.float64).reshape(-1, dim)
    kinds = np.array([b[0] for b in bcs], dtype=np.int32)
    state = np.array([b[1] for b in bcs], dtype=np.float64).reshape(len(bcs), dim + 2)
    return dict(dim=dim, ncells=len(vol), nfaces=len(lr),
                cell_vol=np.asarray(vol, np.float64), cell_ctr=np.asarray(ctr, np.float64).reshape(-1, dim),
                face_lr=lr, face_area=area, face_nrm=nrm, face_ctr=fctr, face_shift=shift,
                nbc=len(bcs), bc_kind=kinds, bc_state=state, shape=tuple(shape))


def box2d(nx, ny, lx=1.0, ly=1.0, periodic=(False, False), sides=None, bcs=None):
    """Uniform Cartesian ``nx x ny`` grid on ``[0,lx] x [0,ly]``.

    ``sides`` maps 'left','right','bottom','top' to a bc id (ignored on a
    periodic axis); ``bcs`` is the list of ``(kind, state)``.
    Cells are numbered ``iy*nx + ix`` (x fastest).
    """
    dx, dy = lx / nx, ly / ny
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny))
    ctr = np.stack([(ix.ravel() + 0.5) * dx, (iy.ravel() + 0.5) * dy], 1)
    vol = np.full(nx * ny, dx * dy)
    sides = sides or {}
    bcs = bcs or []
    faces = []
    cid = lambda i, j: j * nx + i
    # x-normal faces
    for j in range(ny):
        for i in range(nx + 1):
            fc = (i * dx, (j + 0.5) * dy)
            if 0 < i < nx:
                faces.append(((cid(i - 1, j), cid(i, j)), dy, (1.0, 0.0), fc, (0.0, 0.0)))
            elif i == nx:
                if periodic[0]:
                    faces.append(((cid(nx - 1, j), cid(0, j)), dy, (1.0, 0.0), fc, (lx, 0.0)))
                else:
                    faces.append(((cid(nx - 1, j), -1 - sides['right']), dy, (1.0, 0.0), fc, (0.0, 0.0)))
            elif not periodic[0]:
                faces.append(((cid(0, j), -1 - sides['left']), dy, (-1.0, 0.0), fc, (0.0, 0.0)))
    # y-normal faces
    for j in range(ny + 1):
        for i in range(nx):
            fc = ((i + 0.5) * dx, j * dy)
            if 0 < j < ny:
                faces.append(((cid(i, j - 1), cid(i, j)), dx, (0.0, 1.0), fc, (0.0, 0.0)))
            elif j == ny:
                if periodic[1]:
                    faces.append(((cid(i, ny - 1), cid(i, 0)), dx, (0.0, 1.0), fc, (0.0, ly)))
                else:
                    faces.append(((cid(i, ny - 1), -1 - sides['top']), dx, (0.0, 1.0), fc, (0.0, 0.0)))
            elif not periodic[1]:
                faces.append(((cid(i, 0), -1 - sides['bottom']), dx, (0.0, -1.0), fc, (0.0, 0.0)))
    return _finish(2, vol, ctr, faces, bcs, (ny, nx))


def box3d(nx, ny, nz, l=(1.0, 1.0, 1.0), periodic=(True, True, True), bc=None):
    """Uniform Cartesian 3-D grid; non-periodic sides all use bc id 0."""
    d = [l[0] / nx, l[1] / ny, l[2] / nz]
    n = (nx, ny, nz)
    cid = lambda i, j, k: (k * ny + j) * nx + i
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing='ij')
    order = np.argsort(cid(I, J, K).ravel())
    ctr = np.stack([(I.ravel() + 0.5) * d[0], (J.ravel() + 0.5) * d[1], (K.ravel() + 0.5) * d[2]], 1)[order]
    vol = np.full(nx * ny * nz, d[0] * d[1] * d[2])
    faces = []
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        area = d[o1] * d[o2]
        nrm = [0.0, 0.0, 0.0]
        nrm[ax] = 1.0
        for a in range(n[o1]):
            for b in range(n[o2]):
                for c in range(n[ax] + 1):
                    idx = [0, 0, 0]
                    idx[o1], idx[o2] = a, b
                    fc = [0.0, 0.0, 0.0]
                    fc[o1], fc[o2], fc[ax] = (a + 0.5) * d[o1], (b + 0.5) * d[o2], c * d[ax]
                    def cell(cc):
                        t = list(idx)
                        t[ax] = cc
                        return cid(*t)
                    if 0 < c < n[ax]:
                        faces.append(((cell(c - 1), cell(c)), area, tuple(nrm), tuple(fc), (0.0, 0.0, 0.0)))
                    elif periodic[ax]:
                        if c == n[ax]:
                            sh = [0.0, 0.0, 0.0]
                            sh[ax] = l[ax]
                            faces.append(((cell(n[ax] - 1), cell(0)), area, tuple(nrm), tuple(fc), tuple(sh)))
                    else:
                        if c == n[ax]:
                            faces.append(((cell(n[ax] - 1), -1), area, tuple(nrm), tuple(fc), (0.0, 0.0, 0.0)))
                        else:
                            m = [0.0, 0.0, 0.0]
                            m[ax] = -1.0
                            faces.append(((cell(0), -1), area, tuple(m), tuple(fc), (0.0, 0.0, 0.0)))
    bcs = [bc] if bc is not None else ([] if all(periodic) else [(WALL, (1.0, 0.0, 0.0, 0.0, 1.0))])
    return _finish(3, vol, ctr, faces, bcs, (nz, ny, nx))


def _polygon(pts):
    """Area and centroid of a simple polygon (counter-clockwise vertices)."""
    x, y = pts[:, 0], pts[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    a = 0.5 * cr.sum()
    cx = ((x + xn) * cr).sum() / (6 * a)
    cy = ((y + yn) * cr).sum() / (6 * a)
    return a, np.array([cx, cy])


def geometric_radii(n, r0, r1, first):
    """``n+1`` radii from r0 to r1 with first spacing ``first`` and constant growth."""
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        q = 0.5 * (lo + hi)
        s = first * (q ** n - 1.0) / (q - 1.0)
        if s > r1 - r0:
            hi = q
        else:
            lo = q
    q = 0.5 * (lo + hi)
    r = r0 + first * (q ** np.arange(n + 1) - 1.0) / (q - 1.0)
    r[-1] = r1
    return r


def ogrid(nr, nth, r0=0.5, r1=15.0, first=0.01, wall_bc=(WALL, None), far_bc=(FARFIELD, None)):
    """Body-fitted O-grid around a circle of radius ``r0`` (straight-edged quads).

    Cells are numbered ``ir*nth + it`` (circumferential index fastest); the
    grid closes on itself in theta, so the seam needs no shift.  bc 0 is the
    body (wall), bc 1 the outer far-field circle.
    """
    r = geometric_radii(nr, r0, r1, first)
    th = np.linspace(0.0, 2 * np.pi, nth + 1)
    P = lambda i, j: np.array([r[i] * np.cos(th[j % nth]), r[i] * np.sin(th[j % nth])])
    vol = np.empty(nr * nth)
    ctr = np.empty((nr * nth, 2))
    for i in range(nr):
        for j in range(nth):
            a, c = _polygon(np.stack([P(i, j), P(i + 1, j), P(i + 1, j + 1), P(i, j + 1)]))
            vol[i * nth + j], ctr[i * nth + j] = a, c
    faces = []
    cid = lambda i, j: i * nth + (j % nth)

    def seg(p, q):
        t = q - p
        L = np.hypot(t[0], t[1])
        return L, (t[1] / L, -t[0] / L), tuple(0.5 * (p + q))
    # radial-direction faces (constant r): between ir-1 and ir; normal +r
    for i in range(nr + 1):
        for j in range(nth):
            p, q = P(i, j), P(i, j + 1)    # oriented so that (dy,-dx) points outward (+r)
            L, n, fc = seg(p, q)
            if 0 < i < nr:
                faces.append(((cid(i - 1, j), cid(i, j)), L, n, fc, (0.0, 0.0)))
            elif i == nr:
                faces.append(((cid(nr - 1, j), -1 - 1), L, n, fc, (0.0, 0.0)))
            else:
                faces.append(((cid(0, j), -1 - 0), L, (-n[0], -n[1]), fc, (0.0, 0.0)))
    # circumferential faces (constant theta): between it-1 and it; normal +theta
    for i in range(nr):
        for j in range(nth):
            p, q = P(i, j), P(i + 1, j)    # (dy,-dx) of an outward ray points to -theta
            L, n, fc = seg(p, q)
            faces.append(((cid(i, j - 1), cid(i, j)), L, (-n[0], -n[1]), fc, (0.0, 0.0)))
    bcs = [(WALL, wall_bc[1] if wall_bc[1] is not None else (1.0, 0.0, 0.0, 1.0)),
           (FARFIELD, far_bc[1] if far_bc[1] is not None else (1.0, 0.0, 0.0, 1.0))]
    m = _finish(2, vol, ctr, faces, bcs, (nr, nth))
    m['radii'] = r
    return m


def _quad_area_vec(p0, p1, p2, p3):
    """Area vector (|a| = area, direction = right-hand normal) of a planar quad."""
    return 0.5 * np.cross(p2 - p0, p3 - p1)


def sphere_grid(nr, nth, nph, r0=0.5, r1=8.0, first=0.02, wall_state=None, far_state=None):
    """Body-fitted spherical grid around a sphere of radius ``r0``.

    Polar angle theta in [0, pi] (``nth`` cells), azimuth phi in [0, 2 pi)
    (``nph`` cells, closed), radius geometric.  All faces are planar quads;
    the zero-area faces on the polar axis are omitted.  Cells are numbered
    ``(ir*nth + ith)*nph + iph``.  bc 0 = body wall, bc 1 = far field.
    """
    r = geometric_radii(nr, r0, r1, first)
    th = np.linspace(0.0, np.pi, nth + 1)
    ph = np.linspace(0.0, 2 * np.pi, nph + 1)

    def P(i, j, k):
        return r[i] * np.array([np.sin(th[j]) * np.cos(ph[k % nph]), np.sin(th[j]) * np.sin(ph[k % nph]), np.cos(th[j])])
    cid = lambda i, j, k: (i * nth + j) * nph + (k % nph)
    N = nr * nth * nph
    vol = np.zeros(N)
    ctr = np.zeros((N, 3))
    faces = []
    # per cell corner sets (for volume/centroid): accumulate from faces
    acc_v = np.zeros(N)
    acc_c = np.zeros((N, 3))

    def add_face(cl, cr, quad, shift=(0.0, 0.0, 0.0)):
        av = _quad_area_vec(*quad)
        a = np.linalg.norm(av)
        fc = np.mean(quad, axis=0)
        if a <= 1e-14 * r1 * r1:
            return
        n = av / a
        faces.append(((cl, cr), a, tuple(n), tuple(fc), shift))
        # divergence theorem: V = 1/3 sum x_f . A_f n_f (signed per side)
        acc_v[cl] += np.dot(fc, av) / 3.0
        if cr >= 0:
            acc_v[cr] -= np.dot(fc, av) / 3.0
    # r-faces (normal +r): quad ordered so area vector points outward
    for i in range(nr + 1):
        for j in range(nth):
            for k in range(nph):
                q = [P(i, j, k), P(i, j + 1, k), P(i, j + 1, k + 1), P(i, j, k + 1)]
                if 0 < i < nr:
                    add_face(cid(i - 1, j, k), cid(i, j, k), q)
                elif i == nr:
                    add_face(cid(nr - 1, j, k), -1 - 1, q)
                else:
                    add_face(cid(0, j, k), -1 - 0, q[::-1])
    # theta-faces (normal +theta), interior only (poles have zero area)
    for i in range(nr):
        for j in range(1, nth):
            for k in range(nph):
                q = [P(i, j, k), P(i, j, k + 1), P(i + 1, j, k + 1), P(i + 1, j, k)]
                add_face(cid(i, j - 1, k), cid(i, j, k), q)
    # phi-faces (normal +phi), closed ring
    for i in range(nr):
        for j in range(nth):
            for k in range(nph):
                q = [P(i, j, k), P(i + 1, j, k), P(i + 1, j + 1, k), P(i, j + 1, k)]
                add_face(cid(i, j, k - 1), cid(i, j, k), q)
    # fix orientation: make every interior normal point from L to R (by centre test)
    vol[:] = acc_v
    # centroid approximated by the mean of the 8 corners
    for i in range(nr):
        for j in range(nth):
            for k in range(nph):
                pts = [P(a, b, c) for a in (i, i + 1) for b in (j, j + 1) for c in (k, k + 1)]
                ctr[cid(i, j, k)] = np.mean(pts, axis=0)
    ws = wall_state if wall_state is not None else (1.0, 0.0, 0.0, 0.0, 1.0)
    fs = far_state if far_state is not None else (1.0, 0.0, 0.0, 0.0, 1.0)
    m = _finish(3, vol, ctr, faces, [(WALL, ws), (FARFIELD, fs)], (nr, nth, nph))
    m['radii'] = r
    return m


def submesh(desc, cells, halo=2):
    """The cells within ``halo`` face-neighbour rings of ``cells``, as a mesh.

    Faces between two kept cells and boundary faces of kept cells are kept;
    faces to dropped cells are dropped, so only the outermost ring has an
    incomplete face list.  Returns ``(sub, keep)`` with ``keep`` the global
    ids of the kept cells (sub cell j is global cell keep[j]).
    """
    lr = np.asarray(desc['face_lr'])
    nbrs = [[] for _ in range(desc['ncells'])]
    for L, R in lr:
        if R >= 0:
            nbrs[L].append(R)
            nbrs[R].append(L)
    keep = set(int(c) for c in cells)
    ring = set(keep)
    for _ in range(halo):
        ring = {n for c in ring for n in nbrs[c]} - keep
        keep |= ring
    keep = np.array(sorted(keep), dtype=np.int64)
    loc = {int(g): j for j, g in enumerate(keep)}
    fsel = [f for f, (L, R) in enumerate(lr) if L in loc and (R < 0 or R in loc)]
    fsel = np.array(fsel, dtype=np.int64)
    sub_lr = lr[fsel].copy()
    sub_lr[:, 0] = [loc[int(L)] for L in sub_lr[:, 0]]
    sub_lr[:, 1] = [loc[int(R)] if R >= 0 else int(R) for R in sub_lr[:, 1]]
    sub = dict(desc)
    sub.update(ncells=len(keep), nfaces=len(fsel), cell_vol=desc['cell_vol'][keep], cell_ctr=desc['cell_ctr'][keep],
               face_lr=sub_lr, face_area=desc['face_area'][fsel], face_nrm=desc['face_nrm'][fsel],
               face_ctr=desc['face_ctr'][fsel], face_shift=desc['face_shift'][fsel])
    return sub, keep


# ------------------------------------------------------------- simplices ---

def simplicial(points, simplices, classify, bcs, shape=None):
    """Finite-volume mesh of triangles (2-D) or tetrahedra (3-D).

    ``points`` (nv, D), ``simplices`` (nc, D+1) vertex ids.  A face shared
    by two cells runs from the lower cell id (L) to the other; a face with
    one cell is a boundary face whose bc id is ``classify(face_centre)``
    and whose normal points out of the cell.  Cell centres are centroids.
    """
    P = np.asarray(points, np.float64)
    S = np.asarray(simplices, np.int64)
    D = P.shape[1]
    X = P[S]                                   # (nc, D+1, D)
    E = X[:, 1:, :] - X[:, :1, :]
    vol = np.abs(np.linalg.det(E)) / (2.0 if D == 2 else 6.0)
    if not np.all(vol > 0):
        raise ValueError("degenerate simplex")
    ctr = X.mean(axis=1)
    owner = {}
    for c in range(len(S)):
        for k in range(D + 1):
            key = tuple(sorted(int(v) for v in np.delete(S[c], k)))
            owner.setdefault(key, []).append((c, int(S[c, k])))
    faces = []
    for key in sorted(owner):
        cells = sorted(owner[key])
        if len(cells) > 2:
            raise ValueError("non-manifold face")
        V = P[list(key)]
        fc = V.mean(axis=0)
        if D == 2:
            t = V[1] - V[0]
            area = float(np.hypot(t[0], t[1]))
            n = np.array([t[1], -t[0]]) / area
        else:
            cr = np.cross(V[1] - V[0], V[2] - V[0])
            area = 0.5 * float(np.linalg.norm(cr))
            n = cr / (2.0 * area)
        L, opp = cells[0]
        if np.dot(n, fc - P[opp]) < 0:         # away from L's opposite vertex
            n = -n
        if len(cells) == 2:
            faces.append(((L, cells[1][0]), area, tuple(n), tuple(fc), (0.0,) * D))
        else:
            faces.append(((L, -1 - int(classify(fc))), area, tuple(n), tuple(fc), (0.0,) * D))
    return _finish(D, vol, ctr, faces, bcs, shape if shape is not None else (len(S),))


def _side_bc(lo, hi, sides):
    """Boundary classifier of a box: the side whose plane the face centre
    lies on (x- x+ y- y+ z- z+ as 'left','right','bottom','top','front','back')."""
    names = ['left', 'right', 'bottom', 'top', 'front', 'back']
    span = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)

    def classify(fc):
        best, arg = np.inf, None
        for ax in range(len(span)):
            for s, plane in ((0, lo[ax]), (1, hi[ax])):
                d = abs(fc[ax] - plane) / span[ax]
                if d < best:
                    best, arg = d, names[2 * ax + s]
        return sides[arg]
    return classify


def tri_box(nx, ny, seed, lx=1.0, ly=1.0, jitter=0.2, sides=None, bcs=None):
    """Unstructured triangles on ``[0,lx] x [0,ly]``: a lattice of
    ``(nx+1) x (ny+1)`` vertices moved by a seeded jitter of up to
    ``jitter`` of the spacing (boundary vertices slide along their side,
    corners stay), each quad cut along a seeded random diagonal.  2 nx ny
    cells with three faces each."""
    rng = np.random.default_rng(seed)
    hx, hy = lx / nx, ly / ny
    I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing='ij')
    px = I * hx + jitter * hx * rng.uniform(-1, 1, I.shape) * ((I > 0) & (I < nx))
    py = J * hy + jitter * hy * rng.uniform(-1, 1, J.shape) * ((J > 0) & (J < ny))
    pts = np.stack([px.ravel(), py.ravel()], 1)
    vid = lambda i, j: i * (ny + 1) + j
    diag = rng.integers(0, 2, (nx, ny))
    tris = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris += [(a, b, c), (a, c, d)] if diag[i, j] else [(a, b, d), (b, c, d)]
    sides = sides or {}
    return simplicial(pts, tris, _side_bc((0.0, 0.0), (lx, ly), sides), bcs or [])


def tet_box(nx, ny, nz, seed, l=(1.0, 1.0, 1.0), jitter=0.12, sides=None, bcs=None):
    """Unstructured tetrahedra in a box: a jittered vertex lattice (boundary
    vertices stay on their faces), each hexahedron cut into the six
    tetrahedra around its main diagonal (the same cut everywhere, so faces
    match).  6 nx ny nz cells with four faces each."""
    rng = np.random.default_rng(seed)
    n = (nx, ny, nz)
    h = [l[a] / n[a] for a in range(3)]
    G = np.meshgrid(*[np.arange(m + 1) for m in n], indexing='ij')
    pts = np.stack([(G[a] * h[a] + jitter * h[a] * rng.uniform(-1, 1, G[a].shape) * ((G[a] > 0) & (G[a] < n[a])))
                    .ravel() for a in range(3)], 1)
    vid = lambda i, j, k: (i * (ny + 1) + j) * (nz + 1) + k
    # the six monotone paths from corner 000 to 111
    paths = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = []
    for i in range(nx):
        for j in range(ny):
            for k in range(nz):
                for p in paths:
                    c = [0, 0, 0]
                    vs = [vid(i, j, k)]
                    for ax in p:
                        c[ax] = 1
                        vs.append(vid(i + c[0], j + c[1], k + c[2]))
                    tets.append(vs)
    sides = sides or {s: 0 for s in ['left', 'right', 'bottom', 'top', 'front', 'back']}
    return simplicial(pts, tets, _side_bc((0.0, 0.0, 0.0), l, sides), bcs or [(WALL, (1.0, 0.0, 0.0, 0.0, 1.0))])


def wedge_outline(nose=1.0, half_angle_deg=10.0, base_height=3.736, h=0.05):
    """Closed counter-clockwise outline of a 2-D blunt wedge pointing
    upstream (-x): a nose circle of radius ``nose`` centred at (nose, 0)
    joined tangentially to two straight flanks of the given half angle,
    closed by a flat base of height ``base_height``.  Points are spaced
    about ``h`` apart.  Returns (points, base x)."""
    th = math.radians(half_angle_deg)
    cx = nose
    yt = nose * math.cos(th)
    xt = cx - nose * math.sin(th)
    yb = 0.5 * base_height
    xb = xt + (yb - yt) / math.tan(th)
    # the nose arc runs from the lower tangent point through the tip to the upper one
    a0, a1 = -(math.pi / 2 + th), -(3 * math.pi / 2 - th)
    out = []

    def seg(p, q):
        n = max(1, int(math.ceil(math.hypot(q[0] - p[0], q[1] - p[1]) / h)))
        for k in range(n):
            out.append((p[0] + (q[0] - p[0]) * k / n, p[1] + (q[1] - p[1]) * k / n))
    # base (bottom to top), upper flank, nose arc, lower flank
    seg((xb, -yb), (xb, yb))
    seg((xb, yb), (xt, yt))
    na = max(2, int(math.ceil(nose * abs(a1 - a0) / h)))
    for k in range(na):
        a = -a0 + (-a1 + a0) * k / na
        out.append((cx + nose * math.cos(a), nose * math.sin(a)))
    seg((xt, -yt), (xb, -yb))
    return np.array(out), xb


def _convex_offset(poly, d, h):
    """Points about ``h`` apart on the curve at distance ``d`` outside the
    convex polygon ``poly`` (counter-clockwise)."""
    phi = np.linspace(0.0, 2 * np.pi, 4096, endpoint=False)
    nrm = np.stack([np.cos(phi), np.sin(phi)], 1)
    sup = poly[np.argmax(nrm @ poly.T, axis=1)]
    curve = sup + d * nrm
    curve = np.vstack([curve, curve[:1]])
    seg = np.hypot(*(np.diff(curve, axis=0).T))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    n = max(8, int(round(s[-1] / h)))
    t = np.arange(n) * s[-1] / n
    return np.stack([np.interp(t, s, curve[:, 0]), np.interp(t, s, curve[:, 1])], 1)


def _inside_convex(poly, pts):
    """True where a point lies strictly inside the convex polygon (CCW)."""
    e = np.roll(poly, -1, axis=0) - poly
    rel = pts[:, None, :] - poly[None, :, :]
    cross = e[None, :, 0] * rel[:, :, 1] - e[None, :, 1] * rel[:, :, 0]
    return np.all(cross > 0, axis=1)


def blunt_wedge(seed=0, h_wall=0.0538, growth=1.07, box=(-4.0, 16.0, -8.0, 8.0), jitter=0.15,
                nose=1.0, half_angle_deg=10.0, base_height=3.736):
    """Unstructured triangles around a 2-D blunt wedge (lengths in nose radii).

    Layers of points at growing distance from the body (spacing ``h_wall``
    on the wall, times ``growth`` per layer), moved by a seeded jitter of
    up to ``jitter`` of their spacing, the sides of the rectangle ``box`` =
    (x0, x1, y0, y1) sampled at the local spacing, then a Delaunay
    triangulation with the triangles inside the body removed.  bc 0 = the
    body (wall), bc 1 = the rectangle (far field); states are filled by the
    workload.  Cell count grows like 1/h_wall^2 at fixed growth."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    body, xb = wedge_outline(nose, half_angle_deg, base_height, h_wall)
    x0, x1, y0, y1 = box
    pts = [body]
    d, hk = 0.0, h_wall
    far = max(abs(x0), abs(x1 - xb), abs(y0), abs(y1)) + 2 * nose
    while d < far:
        d += 0.866 * hk
        hk *= growth
        lay = _convex_offset(body, d, hk)
        lay = lay + jitter * hk * rng.uniform(-1, 1, lay.shape)
        keep = ((lay[:, 0] > x0 + 0.5 * hk) & (lay[:, 0] < x1 - 0.5 * hk) &
                (lay[:, 1] > y0 + 0.5 * hk) & (lay[:, 1] < y1 - 0.5 * hk))
        pts.append(lay[keep])

    def spacing(p):
        dist = np.sqrt(np.min(np.sum((body - p) ** 2, axis=1)))
        # spacing of the layer at this distance: d_k ~ 0.866 h_wall (g^k - 1) / (g - 1) g
        k = math.log(1.0 + dist * (growth - 1.0) / (0.866 * h_wall * growth)) / math.log(growth)
        return h_wall * growth ** k
    rect = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    for a in range(4):
        p, q = np.array(rect[a]), np.array(rect[(a + 1) % 4])
        L = float(np.hypot(*(q - p)))
        t = 0.0
        while t < L:
            pts.append((p + (q - p) * t / L)[None, :])
            t += spacing(p + (q - p) * t / L)
    P = np.vstack(pts)
    tri = Delaunay(P).simplices
    cen = P[tri].mean(axis=1)
    tri = tri[~_inside_convex(body, cen)]
    # counter-clockwise orientation, drop slivers of zero area
    X = P[tri]
    cr = (X[:, 1, 0] - X[:, 0, 0]) * (X[:, 2, 1] - X[:, 0, 1]) - (X[:, 1, 1] - X[:, 0, 1]) * (X[:, 2, 0] - X[:, 0, 0])
    tri = tri[np.abs(cr) > 1e-12 * h_wall * h_wall]
    used = np.unique(tri)
    remap = -np.ones(len(P), np.int64)
    remap[used] = np.arange(len(used))
    P, tri = P[used], remap[tri]
    eps = 1e-9 * (x1 - x0)

    def classify(fc):
        on_rect = (abs(fc[0] - x0) < eps or abs(fc[0] - x1) < eps or abs(fc[1] - y0) < eps or abs(fc[1] - y1) < eps)
        return 1 if on_rect else 0
    return simplicial(P, tri, classify, [(WALL, (1.0, 0.0, 0.0, 1.0)), (FARFIELD, (1.0, 0.0, 0.0, 1.0))])
