"""Seeded synthetic inputs for the compact third-order gas-kinetic scheme.

This module is shared by the HIP path, the tests and the benchmark.  It holds
none of the scheme's arithmetic: it only builds tetrahedral meshes (a Kuhn
split of a jittered hexahedral grid, periodic or walled), their face
adjacency, and exact cell averages of analytic initial fields (values and
gradients) by a high-order collapsed Gauss rule.  Nothing here computes a
volume, a normal, a reconstruction or a flux.

Array conventions (the library's C-ABI uses the same ones):

* ``xyz``        float64 [n_vert, 3]
* ``tet``        int64   [n_cell, 4]   vertex ids, positively oriented
* ``face_vert``  int64   [n_face, 3]   vertex ids of the face as seen from the owner
* ``face_cell``  int64   [n_face, 2]   (owner, neighbour); neighbour = -1 on a wall
* ``face_tag``   int32   [n_face]      FACE_* below
* ``face_shift`` float64 [n_face, 3]   translation that carries the neighbour's
  geometry into the owner's frame (non-zero only across a periodic seam)
* ``face_wall_u`` float64 [n_face, 3]  velocity of a no-slip wall face (optional)

Cell fields are component-major: ``W[5, n_cell]`` holds (rho, rho u, rho v,
rho w, rho E) and ``gW[15, n_cell]`` holds the cell-averaged gradient, with
component ``c`` and direction ``d`` at row ``3 c + d``.
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import permutations

import numpy as np

FACE_INTERIOR = 0
FACE_PERIODIC = 1
FACE_SLIP = 2
FACE_NOSLIP_ADIABATIC = 3
FACE_NOSLIP_ISOTHERMAL = 4
FACE_FARFIELD = 5


@dataclass
class TetMesh:
    xyz: np.ndarray
    tet: np.ndarray
    face_vert: np.ndarray
    face_cell: np.ndarray
    face_tag: np.ndarray
    face_shift: np.ndarray
    length: float
    n: int
    periodic: bool
    face_wall_u: np.ndarray | None = None  # [n_face, 3] velocity of no-slip wall faces (None: at rest)
    # [n_cell, 6, 3] control points of quadratic elements on the edges QEDGES
    # of each tet (None: straight-sided tetrahedra)
    tet_mid: np.ndarray | None = None

    @property
    def n_cell(self) -> int:
        return int(self.tet.shape[0])

    @property
    def n_face(self) -> int:
        return int(self.face_vert.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])


# edges of a tetrahedron in the order of the quadratic element's shape
# functions (Sec. 4.1): (0,1), (1,2), (0,2), (0,3), (1,3), (2,3)
QEDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def straight_edge_points(mesh: TetMesh) -> np.ndarray:
    """[n_cell, 6, 3] midpoints of every tet's edges in QEDGES order: the
    control points that make a quadratic element straight-sided."""
    x = mesh.xyz[mesh.tet]
    return np.ascontiguousarray(np.stack([0.5 * (x[:, a] + x[:, b]) for a, b in QEDGES], axis=1))


def _kuhn_local_tets():
    """Six tetrahedra of the unit cube sharing the (0,0,0)-(1,1,1) diagonal,
    one per axis permutation, as corner offsets, all positively oriented."""
    out = []
    for perm in permutations(range(3)):
        c = [np.zeros(3, dtype=np.int64)]
        for ax in perm:
            nxt = c[-1].copy()
            nxt[ax] += 1
            c.append(nxt)
        c = np.array(c)
        det = np.linalg.det((c[1:] - c[0]).astype(float))
        if det < 0:
            c[[1, 2]] = c[[2, 1]]
        out.append(c)
    return np.array(out)  # [6, 4, 3]


def kuhn_cube_mesh(n: int, length: float = 1.0, jitter: float = 0.1, seed: int = 0,
                   periodic: bool = True, curve: float = 0.0) -> TetMesh:
    """Cube [0, length]^3 split into n^3 hexahedra, each into 6 Kuhn tetrahedra.

    Vertices are displaced by iid U(-jitter h, jitter h) per axis (numpy
    ``default_rng(seed)``, PCG64), h = length / n.  On a periodic mesh every
    vertex is jittered and periodic images share one displacement.  On a
    walled mesh, boundary vertices only slide tangentially.

    curve > 0 makes the elements quadratic (``tet_mid``): the control point of
    every edge moves from the edge midpoint by iid U(-curve h, curve h) per
    axis, drawn after the jitter from the same generator, one draw per edge
    (periodic images of an edge share it); on a walled mesh the edges that
    lie in a boundary plane stay straight.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    h = length / n
    rng = np.random.default_rng(seed)
    g = np.arange(n + 1)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    grid = np.stack([I, J, K], axis=-1).reshape(-1, 3)  # vertex id -> grid index
    if periodic:
        disp = rng.uniform(-jitter * h, jitter * h, size=(n, n, n, 3))
        wrapped = grid % n
        d = disp[wrapped[:, 0], wrapped[:, 1], wrapped[:, 2]]
    else:
        disp = rng.uniform(-jitter * h, jitter * h, size=(n + 1, n + 1, n + 1, 3))
        d = disp.reshape(-1, 3).copy()
        on_wall = (grid == 0) | (grid == n)
        d[on_wall] = 0.0
    xyz = (grid * length) / n + d

    def vid(ijk):
        return (ijk[..., 0] * (n + 1) + ijk[..., 1]) * (n + 1) + ijk[..., 2]

    local = _kuhn_local_tets()  # [6,4,3]
    hexes = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"),
                     axis=-1).reshape(-1, 3)
    corners = hexes[:, None, None, :] + local[None, :, :, :]  # [n^3, 6, 4, 3]
    tet = vid(corners).reshape(-1, 4).astype(np.int64)
    nc = tet.shape[0]

    # all cell faces: face opposite local vertex a
    opp = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    cf = tet[:, opp].reshape(-1, 3)  # [4 nc, 3] unwrapped vertex ids
    g3 = grid[cf]  # [4 nc, 3 vertices, 3 axes] grid coordinates
    if periodic:
        # canonical lattice translate: per axis, bring the face's smallest
        # coordinate into [0, n); equal faces have equal translated vertex sets
        lat = (g3.min(axis=1) // n) * n  # [4 nc, 3]
    else:
        lat = np.zeros((g3.shape[0], 3), dtype=np.int64)
    gt = g3 - lat[:, None, :]
    base = np.int64(2 * n + 3)
    vkey = (gt[..., 0] * base + gt[..., 1]) * base + gt[..., 2]  # [4 nc, 3]
    vkey = np.sort(vkey, axis=1)
    B3 = base ** 3
    key = (vkey[:, 0] * B3 + vkey[:, 1]) * B3 + vkey[:, 2]
    owner_cell = np.repeat(np.arange(nc, dtype=np.int64), 4)
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same_next = np.zeros(ks.shape[0], dtype=bool)
    same_next[:-1] = ks[:-1] == ks[1:]
    if np.any(same_next[:-1] & same_next[1:]):
        raise RuntimeError("a face is shared by more than two cells")
    pair_first = np.nonzero(same_next)[0]
    paired = np.zeros(ks.shape[0], dtype=bool)
    paired[pair_first] = True
    paired[pair_first + 1] = True
    single = np.nonzero(~paired)[0]
    if periodic and single.size:
        raise RuntimeError("unmatched face on a periodic mesh")

    a_idx = order[pair_first]
    b_idx = order[pair_first + 1]
    ca, cb = owner_cell[a_idx], owner_cell[b_idx]
    if np.any(ca == cb):
        raise RuntimeError("a cell is its own neighbour; use a finer mesh")
    swap = ca > cb
    own_idx = np.where(swap, b_idx, a_idx)
    nb_idx = np.where(swap, a_idx, b_idx)
    own = owner_cell[own_idx]
    nb = owner_cell[nb_idx]
    fv_own = cf[own_idx]
    # periodic shift carrying the neighbour's copy of the face onto the owner's
    dg = lat[own_idx] - lat[nb_idx]
    shift = (dg // n).astype(np.float64) * length
    tag = np.where(np.any(dg != 0, axis=1), FACE_PERIODIC, FACE_INTERIOR).astype(np.int32)

    face_vert = fv_own
    face_cell = np.stack([own, nb], axis=1)
    face_shift = shift
    face_tag = tag
    if single.size:
        s_idx = order[single]
        face_vert = np.concatenate([face_vert, cf[s_idx]])
        face_cell = np.concatenate(
            [face_cell, np.stack([owner_cell[s_idx], -np.ones(s_idx.size, np.int64)], axis=1)])
        face_shift = np.concatenate([face_shift, np.zeros((s_idx.size, 3))])
        face_tag = np.concatenate([face_tag, np.full(s_idx.size, FACE_SLIP, np.int32)])

    # faces ordered by owner, then neighbour: a locality-friendly default order
    fo = np.lexsort((face_cell[:, 1], face_cell[:, 0]))
    mesh = TetMesh(xyz=np.ascontiguousarray(xyz), tet=np.ascontiguousarray(tet),
                   face_vert=np.ascontiguousarray(face_vert[fo]),
                   face_cell=np.ascontiguousarray(face_cell[fo]),
                   face_tag=np.ascontiguousarray(face_tag[fo]),
                   face_shift=np.ascontiguousarray(face_shift[fo]),
                   length=float(length), n=int(n), periodic=bool(periodic))
    if curve > 0.0:
        # each edge by its lattice end points, translated so that the smaller
        # coordinate per axis lies in [0, n) on a periodic mesh
        ga = grid[tet[:, [a for a, _ in QEDGES]]]          # [nc, 6, 3]
        gb = grid[tet[:, [b for _, b in QEDGES]]]
        if periodic:
            lat_e = (np.minimum(ga, gb) // n) * n
            ga, gb = ga - lat_e, gb - lat_e
        base = np.int64(2 * n + 3)
        ka = (ga[..., 0] * base + ga[..., 1]) * base + ga[..., 2]
        kb = (gb[..., 0] * base + gb[..., 1]) * base + gb[..., 2]
        ekey = np.minimum(ka, kb) * base ** 3 + np.maximum(ka, kb)
        uniq, inv = np.unique(ekey.ravel(), return_inverse=True)
        delta = rng.uniform(-curve * h, curve * h, size=(uniq.size, 3))[inv].reshape(ekey.shape + (3,))
        if not periodic:
            flat = np.any((ga == gb) & ((ga == 0) | (ga == n)), axis=-1)
            delta[flat] = 0.0
        mesh.tet_mid = np.ascontiguousarray(straight_edge_points(mesh) + delta)
    return mesh


def _match_faces(tet: np.ndarray):
    """All faces of the tetrahedra matched by their sorted vertex triples:
    (face_vert as seen from the owner, face_cell with -1 for a boundary face)."""
    local = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    fv = tet[:, local].reshape(-1, 3)
    owner = np.repeat(np.arange(tet.shape[0]), 4)
    key = np.sort(fv, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    if cnt.max() > 2:
        raise ValueError("a face is shared by more than two cells")
    order = np.argsort(inv, kind="stable")
    first = np.ones(inv.size, bool)
    first[1:] = inv[order][1:] != inv[order][:-1]
    own_idx = order[first]                      # first occurrence of every face
    nbr = -np.ones(own_idx.size, np.int64)
    second = order[~first]                      # the second occurrence, if any
    pos = np.searchsorted(inv[own_idx], inv[second])
    nbr[pos] = owner[second]
    return fv[own_idx], np.stack([owner[own_idx], nbr], axis=1)


def cubed_sphere_shell(n: int, layers: int, r_out: float = 20.0, ratio: float = 1.08,
                       curved: bool = False, wall_tag: int = FACE_SLIP) -> TetMesh:
    """Shell 1 <= r <= r_out around the unit sphere: the cube surface cut into
    6 panels of n x n cells (n even), mapped to the sphere equiangularly
    (lattice point p with |p|_inf = n/2 goes to the direction tan(pi/4 p/(n/2))),
    and `layers` radial layers whose thickness grows geometrically by `ratio`.
    Each hexahedron is split into two prisms along the surface diagonal
    through its smallest vertex id, each prism into three tetrahedra by the
    minimum-vertex-id rule, so the split conforms across cells and panel
    seams.  Faces on r = 1 are walls of kind `wall_tag` (slip by default; a
    no-slip tag gives a sphere at rest), on r = r_out far field.

    curved: quadratic elements (``tet_mid``) whose edges on the wall r = 1 are
    arcs: their control point is the edge midpoint moved radially onto the
    sphere (Sec. 2.1); every other edge stays straight."""
    if n < 2 or n % 2:
        raise ValueError("n must be even and >= 2")
    m = n // 2
    g = np.arange(-m, m + 1)
    P = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    on = np.abs(P).max(axis=1) == m
    S = P[on]                                   # the cube-surface lattice, 6 n^2 + 2 points
    lookup = -np.ones((n + 1,) * 3, np.int64)
    lookup[S[:, 0] + m, S[:, 1] + m, S[:, 2] + m] = np.arange(S.shape[0])
    d = np.tan(np.pi / 4 * S / m)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    # radii: r_0 = 1, thicknesses h0 ratio^k summing to r_out - 1
    h0 = (r_out - 1.0) * (ratio - 1.0) / (ratio ** layers - 1.0) if ratio != 1.0 else (r_out - 1.0) / layers
    r = np.concatenate([[1.0], 1.0 + np.cumsum(h0 * ratio ** np.arange(layers))])
    r[-1] = r_out
    ns = S.shape[0]
    xyz = (r[:, None, None] * d[None, :, :]).reshape(-1, 3)
    # surface quads of the six panels, corners in cyclic order
    quads = []
    for axis in range(3):
        for sign in (-1, 1):
            u, v = [a for a in range(3) if a != axis]
            ii, jj = np.meshgrid(np.arange(-m, m), np.arange(-m, m), indexing="ij")
            ii, jj = ii.ravel(), jj.ravel()
            corners = []
            for du, dv in ((0, 0), (1, 0), (1, 1), (0, 1)):
                q = np.zeros((ii.size, 3), np.int64)
                q[:, axis] = sign * m
                q[:, u] = ii + du
                q[:, v] = jj + dv
                corners.append(lookup[q[:, 0] + m, q[:, 1] + m, q[:, 2] + m])
            quads.append(np.stack(corners, axis=1))
    quads = np.concatenate(quads)               # [6 n^2, 4]
    # two triangles per quad along the diagonal through its smallest id
    k0 = np.argmin(quads, axis=1)
    rot = np.stack([quads[np.arange(quads.shape[0]), (k0 + t) % 4] for t in range(4)], axis=1)
    tris = np.concatenate([rot[:, [0, 1, 2]], rot[:, [0, 2, 3]]])
    # prisms of every layer: bottom (a, b, c) at layer k, top at k + 1
    kk = np.arange(layers)
    bot = (tris[None, :, :] + (kk * ns)[:, None, None]).reshape(-1, 3)
    pr = np.concatenate([bot, bot + ns], axis=1)  # [n_prism, 6]: (a, b, c, a', b', c')
    # minimum-vertex-id rule: bring the smallest id to position 0 (reflecting
    # top and bottom if it is on top, then rotating), split the quad opposite it
    imin = np.argmin(pr, axis=1)
    top = imin >= 3
    pr = np.where(top[:, None], pr[:, [3, 4, 5, 0, 1, 2]], pr)
    i0 = imin % 3
    idx = np.stack([(i0 + t) % 3 for t in range(3)], axis=1)
    ar = np.arange(pr.shape[0])[:, None]
    pr = np.concatenate([pr[ar, idx], pr[ar, idx + 3]], axis=1)
    v0, v1, v2, v3, v4, v5 = pr.T
    diag15 = np.minimum(v1, v5) < np.minimum(v2, v4)
    t1 = np.where(diag15[:, None], np.stack([v0, v1, v2, v5], 1), np.stack([v0, v1, v2, v4], 1))
    t2 = np.where(diag15[:, None], np.stack([v0, v1, v5, v4], 1), np.stack([v0, v4, v2, v5], 1))
    t3 = np.stack([v0, v4, v5, v3], 1)
    tet = np.concatenate([t1, t2, t3])
    # positive orientation
    e = xyz[tet[:, 1:]] - xyz[tet[:, :1]]
    neg = np.linalg.det(e) < 0
    tet[neg] = tet[neg][:, [0, 2, 1, 3]]
    face_vert, face_cell = _match_faces(tet)
    wall = face_cell[:, 1] < 0
    rad = np.linalg.norm(xyz[face_vert].mean(axis=1), axis=1)
    tag = np.where(wall, np.where(rad < 0.5 * (1.0 + r_out), wall_tag, FACE_FARFIELD), FACE_INTERIOR)
    fo = np.lexsort((face_cell[:, 1], face_cell[:, 0]))
    mesh = TetMesh(xyz=np.ascontiguousarray(xyz), tet=np.ascontiguousarray(tet),
                   face_vert=np.ascontiguousarray(face_vert[fo]), face_cell=np.ascontiguousarray(face_cell[fo]),
                   face_tag=np.ascontiguousarray(tag[fo].astype(np.int32)),
                   face_shift=np.zeros((face_vert.shape[0], 3)), length=float(r_out), n=int(n), periodic=False)
    if curved:
        mid = straight_edge_points(mesh)
        inner = np.arange(xyz.shape[0]) < ns            # the vertices of layer 0 lie on r = 1
        on = np.stack([inner[tet[:, a]] & inner[tet[:, b]] for a, b in QEDGES], axis=1)
        mid[on] /= np.linalg.norm(mid[on], axis=1, keepdims=True)
        mesh.tet_mid = np.ascontiguousarray(mid)
    return mesh


def uniform_state(mesh: TetMesh, rho: float, U, p: float, gamma: float = 1.4):
    """A uniform state (W, grad W = 0)."""
    U = np.asarray(U, np.float64)
    W = np.empty((5, mesh.n_cell))
    W[0] = rho
    W[1:4] = rho * U[:, None]
    W[4] = p / (gamma - 1.0) + 0.5 * rho * (U @ U)
    return W, np.zeros((15, mesh.n_cell))


def with_walls(mesh: TetMesh, tags: dict, velocity: dict | None = None) -> TetMesh:
    """The walled cube mesh with its six sides retagged: ``tags`` maps a side
    name ("x0", "x1", "y0", "y1", "z0", "z1": the plane x = 0, x = length,
    ...) to a FACE_* wall tag (sides not named stay slip walls); ``velocity``
    maps a side to its wall velocity (3 components; others at rest).  A side
    is found from the mean of its face's vertices."""
    if mesh.periodic:
        raise ValueError("a periodic mesh has no walls")
    wall = mesh.face_cell[:, 1] < 0
    cen = mesh.xyz[mesh.face_vert].mean(axis=1)
    tag = mesh.face_tag.copy()
    wu = np.zeros((mesh.n_face, 3))
    tol = 1e-9 * mesh.length
    for name in set(tags) | set(velocity or {}):
        axis, end = "xyz".index(name[0]), float(name[1]) * mesh.length
        on = wall & (np.abs(cen[:, axis] - end) < tol)
        if name in tags:
            tag[on] = tags[name]
        if velocity and name in velocity:
            wu[on] = np.asarray(velocity[name], np.float64)
    return TetMesh(xyz=mesh.xyz, tet=mesh.tet, face_vert=mesh.face_vert, face_cell=mesh.face_cell,
                   face_tag=np.ascontiguousarray(tag), face_shift=mesh.face_shift, length=mesh.length,
                   n=mesh.n, periodic=False, face_wall_u=np.ascontiguousarray(wu), tet_mid=mesh.tet_mid)


# ----------------------------------------------------------------------------
# collapsed Gauss rule on the reference tetrahedron (Duffy map of a cube rule)
# ----------------------------------------------------------------------------

def tet_rule(npts: int = 6):
    """Barycentric-free reference points (xi, eta, zeta) and weights that sum to 1.

    Gauss-Legendre on [0,1]^3 mapped by xi=a, eta=(1-a)b, zeta=(1-a)(1-b)c with
    Jacobian (1-a)^2 (1-b); exact for polynomials of degree <= 2 npts - 3.
    """
    x, w = np.polynomial.legendre.leggauss(npts)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    A, B, C = np.meshgrid(x, x, x, indexing="ij")
    WA, WB, WC = np.meshgrid(w, w, w, indexing="ij")
    xi = A
    eta = (1 - A) * B
    zeta = (1 - A) * (1 - B) * C
    wt = WA * WB * WC * (1 - A) ** 2 * (1 - B)
    pts = np.stack([xi.ravel(), eta.ravel(), zeta.ravel()], axis=1)
    wt = wt.ravel()
    return pts, wt / wt.sum()


def cell_points(mesh: TetMesh, pts: np.ndarray) -> np.ndarray:
    """Physical points [n_cell, n_pts, 3] of reference points inside every tet."""
    v = mesh.xyz[mesh.tet]  # [nc,4,3]
    e = v[:, 1:, :] - v[:, :1, :]  # [nc,3,3]
    return v[:, None, 0, :] + np.einsum("qk,ckd->cqd", pts, e)


# ----------------------------------------------------------------------------
# analytic fields: each returns (Q[5,...], dQ[5,3,...]) at points X[...,3]
# ----------------------------------------------------------------------------

def sine_wave_field(gamma: float = 1.4, amp: float = 0.2, length: float = 1.0,
                    vel=(1.0, 1.0, 1.0), p: float = 1.0, t: float = 0.0,
                    direction=(1.0, 1.0, 1.0)):
    """Density wave rho = 1 + amp sin(2 pi d.(x - u t) / length), uniform u and p;
    d has integer components so that the wave is periodic on the cube."""
    kk = 2.0 * np.pi / length
    u = np.asarray(vel, dtype=float)
    dv = np.asarray(direction, dtype=float)

    def f(X):
        ph = kk * ((X[..., 0] - u[0] * t) * dv[0] + (X[..., 1] - u[1] * t) * dv[1] +
                   (X[..., 2] - u[2] * t) * dv[2])
        rho = 1.0 + amp * np.sin(ph)
        drho = amp * kk * np.cos(ph)
        Q = np.stack([rho, rho * u[0], rho * u[1], rho * u[2],
                      p / (gamma - 1.0) + 0.5 * rho * (u @ u)])
        dr = np.stack([drho * dv[0], drho * dv[1], drho * dv[2]])  # d rho / dx_j
        dQ = np.stack([dr, dr * u[0], dr * u[1], dr * u[2], 0.5 * (u @ u) * dr])
        return Q, dQ
    return f


def taylor_green_field(gamma: float = 1.4, mach: float = 0.1, u0: float = 1.0,
                       rho0: float = 1.0, ell: float = 1.0):
    """Taylor-Green vortex on [0, 2 pi ell]^3 with an isothermal start (rho = rho0 p / p0)."""
    p0 = rho0 * u0 * u0 / (gamma * mach * mach)

    def f(X):
        x, y, z = X[..., 0] / ell, X[..., 1] / ell, X[..., 2] / ell
        sx, cx, sy, cy, sz, cz = np.sin(x), np.cos(x), np.sin(y), np.cos(y), np.sin(z), np.cos(z)
        u = u0 * sx * cy * cz
        v = -u0 * cx * sy * cz
        w = np.zeros_like(u)
        ux, uy, uz = u0 * cx * cy * cz / ell, -u0 * sx * sy * cz / ell, -u0 * sx * cy * sz / ell
        vx, vy, vz = u0 * sx * sy * cz / ell, -u0 * cx * cy * cz / ell, u0 * cx * sy * sz / ell
        c2x, c2y, c2z = np.cos(2 * x), np.cos(2 * y), np.cos(2 * z)
        k = rho0 * u0 * u0 / 16.0
        p = p0 + k * (c2x + c2y) * (c2z + 2.0)
        px = k * (-2.0 * np.sin(2 * x)) * (c2z + 2.0) / ell
        py = k * (-2.0 * np.sin(2 * y)) * (c2z + 2.0) / ell
        pz = k * (c2x + c2y) * (-2.0 * np.sin(2 * z)) / ell
        rho = rho0 * p / p0
        rx, ry, rz = rho0 * px / p0, rho0 * py / p0, rho0 * pz / p0
        ke = 0.5 * (u * u + v * v)
        kex, key, kez = u * ux + v * vx, u * uy + v * vy, u * uz + v * vz
        Q = np.stack([rho, rho * u, rho * v, rho * w, p / (gamma - 1.0) + rho * ke])
        dQ = np.stack([
            np.stack([rx, ry, rz]),
            np.stack([rx * u + rho * ux, ry * u + rho * uy, rz * u + rho * uz]),
            np.stack([rx * v + rho * vx, ry * v + rho * vy, rz * v + rho * vz]),
            np.stack([np.zeros_like(x)] * 3),
            np.stack([px / (gamma - 1.0) + rx * ke + rho * kex,
                      py / (gamma - 1.0) + ry * ke + rho * key,
                      pz / (gamma - 1.0) + rz * ke + rho * kez]),
        ])
        return Q, dQ
    return f


def bump_stream_field(gamma: float = 1.4, speed: float = 0.3, center=(2.0, 0.0, 0.0), width: float = 0.3):
    """Uniform stream rho = 1, U = (speed, 0, 0), p = 1/gamma with a smooth
    density and pressure bump exp(-|x - c|^2 / width) (rho + 0.1 b, p + 0.05 b)
    around c: a disturbed free stream for flows past the sphere."""
    c = np.asarray(center, np.float64)

    def f(X):
        x, y, z = X[..., 0] - c[0], X[..., 1] - c[1], X[..., 2] - c[2]
        b = np.exp(-(x * x + y * y + z * z) / width)
        db = [-2.0 * r / width * b for r in (x, y, z)]
        rho = 1.0 + 0.1 * b
        p = 1.0 / gamma + 0.05 * b
        u = speed * np.ones_like(x)
        zero = np.zeros_like(x)
        Q = np.stack([rho, rho * u, zero, zero, p / (gamma - 1) + 0.5 * rho * u * u])
        dQ = np.stack([np.stack([0.1 * g for g in db]), np.stack([0.1 * g * speed for g in db]),
                       np.stack([zero] * 3), np.stack([zero] * 3),
                       np.stack([0.05 * g / (gamma - 1) + 0.5 * speed * speed * 0.1 * g for g in db])])
        return Q, dQ
    return f


def _quadratic_map(x: np.ndarray, pts: np.ndarray):
    """Points X [c, q, 3] and |det dX/dxi| [c, q] of ten-node tetrahedra with
    nodes x [c, 10, 3] (vertices, then the points on the edges QEDGES) at
    reference points pts [q, 3]: vertex shape functions l (2l - 1), edge ones
    4 l_a l_b in the barycentric coordinates l."""
    lam = np.concatenate([1.0 - pts.sum(axis=1, keepdims=True), pts], axis=1)       # [q, 4]
    dlam = np.array([[-1.0, -1.0, -1.0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])           # [4, 3]
    N = [lam[:, a] * (2 * lam[:, a] - 1) for a in range(4)]
    dN = [(4 * lam[:, a] - 1)[:, None] * dlam[a] for a in range(4)]
    for a, b in QEDGES:
        N.append(4 * lam[:, a] * lam[:, b])
        dN.append(4 * (lam[:, b][:, None] * dlam[a] + lam[:, a][:, None] * dlam[b]))
    N, dN = np.stack(N, axis=1), np.stack(dN, axis=1)                                # [q, 10], [q, 10, 3]
    c, nq = x.shape[0], N.shape[0]
    xt = np.ascontiguousarray(x.transpose(1, 0, 2)).reshape(10, 3 * c)                 # [l, c d]
    X = (N @ xt).reshape(nq, c, 3).transpose(1, 0, 2)
    # J[c, q, d, j] = sum_l dN[q, l, j] x[c, l, d], one matrix product
    J = (dN.transpose(0, 2, 1).reshape(3 * nq, 10) @ xt).reshape(nq, 3, c, 3)        # [q, j, c, d]
    a = J.transpose(2, 0, 3, 1)                                                         # [c, q, d, j]
    det = (a[..., 0, 0] * (a[..., 1, 1] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 1])
           - a[..., 0, 1] * (a[..., 1, 0] * a[..., 2, 2] - a[..., 1, 2] * a[..., 2, 0])
           + a[..., 0, 2] * (a[..., 1, 0] * a[..., 2, 1] - a[..., 1, 1] * a[..., 2, 0]))
    return np.ascontiguousarray(X), np.abs(det)


def cell_averages(mesh: TetMesh, field, npts: int = 6, chunk: int = 65536, progress=None):
    """Exact (to quadrature) cell averages of a field and of its gradient;
    over a quadratic element (``tet_mid``) through its isoparametric map.
    ``progress(done, total)``, if given, is called after each chunk of cells.

    Returns ``W[5, n_cell]`` and ``gW[15, n_cell]`` (row 3 c + d)."""
    pts, wt = tet_rule(npts)
    nc = mesh.n_cell
    W = np.empty((5, nc))
    gW = np.empty((15, nc))
    v_all = mesh.xyz[mesh.tet]
    for s in range(0, nc, chunk):
        v = v_all[s:s + chunk]
        if mesh.tet_mid is None:
            e = v[:, 1:, :] - v[:, :1, :]
            X = v[:, None, 0, :] + np.einsum("qk,ckd->cqd", pts, e)
            Q, dQ = field(X)  # Q [5, c, q], dQ [5, 3, c, q]
            W[:, s:s + chunk] = Q @ wt
            gW[:, s:s + chunk] = (dQ @ wt).reshape(15, -1)
            if progress:
                progress(min(s + chunk, nc), nc)
            continue
        X, dj = _quadratic_map(np.concatenate([v, mesh.tet_mid[s:s + chunk]], axis=1), pts)
        w = dj * wt
        w = w / w.sum(axis=1, keepdims=True)
        Q, dQ = field(X)
        W[:, s:s + chunk] = np.einsum("pcq,cq->pc", Q, w)
        gW[:, s:s + chunk] = np.einsum("pdcq,cq->pdc", dQ, w).reshape(15, -1)
        if progress:
            progress(min(s + chunk, nc), nc)
    return W, gW


def conservative_to_primitive(W: np.ndarray, gamma: float):
    rho = W[0]
    u = W[1:4] / rho
    p = (gamma - 1.0) * (W[4] - 0.5 * rho * np.sum(u * u, axis=0))
    return rho, u, p


def box_vortex_field(gamma: float = 1.4, amp: float = 0.2, p0: float = 1.0, bump: float = 0.3,
                     length: float = 1.0):
    """A smooth state in the box [0, L]^3 with slip walls: the swirl
    U = amp (sin(pi x/L) cos(pi y/L), -cos(pi x/L) sin(pi y/L), 0), which has no
    normal velocity on the walls, rho = 1 + bump/2 exp(-|x - c|^2 / (0.05 L^2)),
    p = p0 (1 + bump exp(-|x - c|^2 / (0.05 L^2))), c the centre."""
    k = np.pi / length
    s2 = 0.05 * length * length

    def f(X):
        x, y, z = X[..., 0], X[..., 1], X[..., 2]
        dx, dy, dz = x - 0.5 * length, y - 0.5 * length, z - 0.5 * length
        G = np.exp(-(dx * dx + dy * dy + dz * dz) / s2)
        dG = [-2.0 * dx / s2 * G, -2.0 * dy / s2 * G, -2.0 * dz / s2 * G]
        rho = 1.0 + 0.5 * bump * G
        drho = [0.5 * bump * g for g in dG]
        p = p0 * (1.0 + bump * G)
        dp = [p0 * bump * g for g in dG]
        u = amp * np.sin(k * x) * np.cos(k * y)
        v = -amp * np.cos(k * x) * np.sin(k * y)
        w = np.zeros_like(x)
        du = [amp * k * np.cos(k * x) * np.cos(k * y), -amp * k * np.sin(k * x) * np.sin(k * y), 0 * x]
        dv = [amp * k * np.sin(k * x) * np.sin(k * y), -amp * k * np.cos(k * x) * np.cos(k * y), 0 * x]
        dw = [0 * x, 0 * x, 0 * x]
        q = 0.5 * (u * u + v * v + w * w)
        dq = [u * du[d] + v * dv[d] + w * dw[d] for d in range(3)]
        E = p / (gamma - 1.0) + rho * q
        Q = np.stack([rho, rho * u, rho * v, rho * w, E])
        dQ = np.stack([
            np.stack(drho),
            np.stack([drho[d] * u + rho * du[d] for d in range(3)]),
            np.stack([drho[d] * v + rho * dv[d] for d in range(3)]),
            np.stack([drho[d] * w + rho * dw[d] for d in range(3)]),
            np.stack([dp[d] / (gamma - 1.0) + drho[d] * q + rho * dq[d] for d in range(3)]),
        ])
        return Q, dQ

    return f


def _refined_centroids(levels: int) -> np.ndarray:
    """Barycentric coordinates of the centroids of the 8^levels tetrahedra of
    `levels` regular refinements of a tetrahedron (four corner tetrahedra and
    the central octahedron cut along one diagonal into four); the children of
    a regular refinement have equal volumes."""
    tets = [np.eye(4)]
    for _ in range(levels):
        out = []
        for t in tets:
            v = t
            m = {(a, b): 0.5 * (v[a] + v[b]) for a in range(4) for b in range(a + 1, 4)}
            e = lambda a, b: m[(min(a, b), max(a, b))]
            out += [np.stack([v[0], e(0, 1), e(0, 2), e(0, 3)]),
                    np.stack([e(0, 1), v[1], e(1, 2), e(1, 3)]),
                    np.stack([e(0, 2), e(1, 2), v[2], e(2, 3)]),
                    np.stack([e(0, 3), e(1, 3), e(2, 3), v[3]])]
            # octahedron (midpoints of the six edges) cut along e(0,2)-e(1,3)
            a, b = e(0, 2), e(1, 3)
            ring = [e(0, 1), e(1, 2), e(2, 3), e(0, 3)]
            for k in range(4):
                out.append(np.stack([a, b, ring[k], ring[(k + 1) % 4]]))
        tets = out
    return np.stack([t.mean(axis=0) for t in tets])  # [8^levels, 4]


def blast_cell_averages(mesh: TetMesh, gamma: float = 1.4, radius: float = 0.1, center=(0.5, 0.5, 0.5),
                        inside=(1.0, 10.0), outside=(1.0, 0.1), levels: int = 3, chunk: int = 16384):
    """The spherical blast: gas at rest, (rho, p) = inside for |x - c| < radius
    and outside elsewhere.  Cell averages from the volume fraction of each
    cell inside the sphere, counted on its 8^levels equal sub-tetrahedra by
    their centroids; averaged gradients by the divergence theorem, the sum
    over the cell's faces of |Gamma| n times the three-point face rule applied
    to point values of the step.  Returns W[5, n], gW[15, n]."""
    c = np.asarray(center, dtype=np.float64)
    Win = np.array([inside[0], 0.0, 0.0, 0.0, inside[1] / (gamma - 1.0)])
    Wout = np.array([outside[0], 0.0, 0.0, 0.0, outside[1] / (gamma - 1.0)])
    bary = _refined_centroids(levels)
    nc = mesh.n_cell
    frac = np.empty(nc)
    v_all = mesh.xyz[mesh.tet]
    for s in range(0, nc, chunk):
        v = v_all[s:s + chunk]
        X = np.matmul(bary[None], v - c)  # sub-tetrahedron centroids relative to c
        frac[s:s + chunk] = (np.einsum("ckd,ckd->ck", X, X) < radius * radius).mean(axis=1)
    W = np.outer(Win, frac) + np.outer(Wout, 1.0 - frac)
    # divergence theorem with the face rule at (1/6,1/6), (2/3,1/6), (1/6,2/3)
    gp = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
    vol = np.abs(np.linalg.det(v_all[:, 1:] - v_all[:, :1])) / 6.0
    cen = v_all.mean(axis=1)
    acc = np.zeros((nc, 3, 5))
    for a in range(4):
        fv = v_all[:, [b for b in range(4) if b != a]]  # [nc, 3, 3]
        an = 0.5 * np.cross(fv[:, 1] - fv[:, 0], fv[:, 2] - fv[:, 0])  # area * normal
        out = np.sign(np.einsum("cd,cd->c", an, fv[:, 0] - cen))
        an *= out[:, None]
        P = np.matmul(gp[None], fv)  # [nc, 3 points, 3]
        ins = (np.sum((P - c) ** 2, axis=2) < radius * radius).astype(np.float64)
        Wp = ins[:, :, None] * Win + (1.0 - ins[:, :, None]) * Wout  # [nc, 3, 5]
        acc += an[:, :, None] * Wp.mean(axis=1)[:, None, :]
    gW = (acc / vol[:, None, None]).transpose(2, 1, 0).reshape(15, nc)
    return W, gW


def rms_directions(W: np.ndarray, gW: np.ndarray, ndir: int, seed: int):
    """`ndir` seeded Gaussian directions in the space of (W, gW), each row
    scaled by the RMS of that row of the state (gradient rows: plus 1e-3, so
    that a row that vanishes still moves).  Returns dW[ndir][5][n],
    dgW[ndir][15][n]."""
    rng = np.random.default_rng(seed)
    sW = np.sqrt((W ** 2).mean(axis=1, keepdims=True))
    sG = np.sqrt((gW ** 2).mean(axis=1, keepdims=True)) + 1e-3
    dW = np.empty((ndir,) + W.shape)
    dG = np.empty((ndir,) + gW.shape)
    for k in range(ndir):
        dW[k] = rng.standard_normal(W.shape) * sW
        dG[k] = rng.standard_normal(gW.shape) * sG
    return dW, dG
