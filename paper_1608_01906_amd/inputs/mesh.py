"""Seeded synthetic P1 meshes (inputs shared by the oracle and the device path).

The paper samples the populations at the vertices of a linear simplex mesh
(Section 2.2.1, discrete-field equation) but gives its meshes only by element
count (Section 3.1, Table 1), so every workload here runs on a generated
stand-in: a unit-spaced grid whose nodes are jittered uniformly, each square
cell cut into 2 triangles along its (0,0)-(1,1) diagonal, each cube cell cut
into the 6 Kuhn tetrahedra around its (0,0,0)-(1,1,1) diagonal.

This module holds no arithmetic of the method: it only places nodes, lists
elements and flags wall nodes.  Random numbers come from SplitMix64
(Steele, Lea and Flood, OOPSLA 2014), evaluated counter-style so that the
i-th draw of a stream is mix(seed + (i+1) * 0x9E3779B97F4A7C15).

Mesh dictionary (all numpy arrays, caller node order):
  dim        2 or 3
  xyz        float64 [n_nodes, dim]   node coordinates (inside or near the box)
  conn       int32   [n_elems, dim+1] vertex indices, positively oriented
  shift      int8    [n_elems, dim+1, dim] periodic image of each vertex:
             unwrapped position = xyz[conn[e, a]] + shift[e, a] * box
  box        float64 [dim]  period along each axis, 0 where the axis is walled
  wall       uint8   [n_nodes] 1 on wall nodes
  wall_normal float64 [n_nodes, dim] unit normal pointing into the fluid
"""
from __future__ import annotations

import itertools

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Draws start..start+n-1 of the SplitMix64 stream seeded with `seed`."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform01(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of each draw."""
    return (splitmix64(seed, n, start) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _jitter(seed: int, n_nodes: int, dim: int, amp: float) -> np.ndarray:
    if amp == 0.0:
        return np.zeros((n_nodes, dim))
    u = uniform01(seed, n_nodes * dim).reshape(n_nodes, dim)
    return (2.0 * u - 1.0) * amp


def grid_mesh_2d(nx: int, ny: int, *, wall_y: bool = False, jitter: float = 0.2,
                 seed: int = 1608) -> dict:
    """nx x ny node grid, periodic in x; periodic in y unless `wall_y`.

    With walls the node rows j = 0 and j = ny-1 lie on the walls (y exact,
    jittered along x only) and there are ny-1 cell rows; otherwise ny cell
    rows wrap around.
    """
    if nx < 2 or ny < 2:
        raise ValueError("grid needs at least 2 nodes per axis")
    n = nx * ny
    j_idx, i_idx = np.divmod(np.arange(n, dtype=np.int64), nx)
    xyz = np.stack([i_idx, j_idx], axis=1).astype(np.float64)
    jit = _jitter(seed, n, 2, jitter)
    wall = np.zeros(n, np.uint8)
    normal = np.zeros((n, 2))
    if wall_y:
        on_wall = (j_idx == 0) | (j_idx == ny - 1)
        jit[on_wall, 1] = 0.0
        wall[on_wall] = 1
        normal[j_idx == 0, 1] = 1.0
        normal[j_idx == ny - 1, 1] = -1.0
    xyz += jit
    box = np.array([float(nx), 0.0 if wall_y else float(ny)])

    ncy = ny - 1 if wall_y else ny
    cj, ci = np.divmod(np.arange(nx * ncy, dtype=np.int64), nx)

    def corner(di, dj):
        ii, jj = ci + di, cj + dj
        sx, sy = ii // nx, jj // ny
        node = (jj % ny) * nx + (ii % nx)
        return node, np.stack([sx, sy], axis=1)

    c00, s00 = corner(0, 0)
    c10, s10 = corner(1, 0)
    c11, s11 = corner(1, 1)
    c01, s01 = corner(0, 1)
    conn = np.empty((2 * nx * ncy, 3), np.int32)
    shift = np.empty((2 * nx * ncy, 3, 2), np.int8)
    conn[0::2] = np.stack([c00, c10, c11], axis=1)
    conn[1::2] = np.stack([c00, c11, c01], axis=1)
    shift[0::2] = np.stack([s00, s10, s11], axis=1)
    shift[1::2] = np.stack([s00, s11, s01], axis=1)
    return dict(dim=2, xyz=xyz, conn=conn, shift=shift, box=box, wall=wall,
                wall_normal=normal)


def _kuhn_corners():
    """The 6 Kuhn tetrahedra of the unit cube as corner offsets, oriented positively."""
    tets = []
    for perm in itertools.permutations(range(3)):
        v = [np.zeros(3, np.int64)]
        for ax in perm:
            nxt = v[-1].copy()
            nxt[ax] = 1
            v.append(nxt)
        det = np.linalg.det(np.array([v[1] - v[0], v[2] - v[0], v[3] - v[0]], float))
        if det < 0:
            v[1], v[2] = v[2], v[1]
        tets.append(v)
    return tets


def grid_mesh_3d(nx: int, ny: int, nz: int, *, jitter: float = 0.2, seed: int = 1608) -> dict:
    """nx x ny x nz periodic node grid cut into Kuhn tetrahedra."""
    if min(nx, ny, nz) < 2:
        raise ValueError("grid needs at least 2 nodes per axis")
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    k_idx, rem = np.divmod(idx, nx * ny)
    j_idx, i_idx = np.divmod(rem, nx)
    xyz = np.stack([i_idx, j_idx, k_idx], axis=1).astype(np.float64)
    xyz += _jitter(seed, n, 3, jitter)
    box = np.array([float(nx), float(ny), float(nz)])
    dims = np.array([nx, ny, nz])
    cells = np.stack([i_idx, j_idx, k_idx], axis=1)  # one cell per node (periodic)

    conn = np.empty((6 * n, 4), np.int32)
    shift = np.empty((6 * n, 4, 3), np.int8)
    for t, corners in enumerate(_kuhn_corners()):
        for a, off in enumerate(corners):
            p = cells + off
            s = p // dims
            q = p % dims
            conn[t::6, a] = (q[:, 2] * ny + q[:, 1]) * nx + q[:, 0]
            shift[t::6, a] = s
    return dict(dim=3, xyz=xyz, conn=conn, shift=shift, box=box,
                wall=np.zeros(n, np.uint8), wall_normal=np.zeros((n, 3)))


def delaunay_mesh(dims, *, jitter: float = 0.4, seed: int = 1613) -> dict:
    """Periodic unstructured simplex mesh (2-D triangles or 3-D tetrahedra).

    Nodes: a unit grid of shape `dims` jittered by +-jitter per coordinate.
    Elements: the Delaunay triangulation of those nodes together with their
    3^d - 1 periodic copies, keeping the simplices whose centroid lies in the
    base cell [0, n_x) x [0, n_y) (x [0, n_z)), a fundamental domain, so every
    periodic simplex is kept once; a vertex taken from copy c gets the image
    shift c.  Unlike the grid meshes the connectivity is irregular (2-D
    valence up to about 10, 3-D up to about 22).
    """
    from scipy.spatial import Delaunay
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    if dim not in (2, 3) or min(dims) < 3:
        raise ValueError("need 2 or 3 axes of at least 3 nodes")
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx
    for d in dims[:-1]:
        rem, r = np.divmod(rem, d)
        coords.append(r)
    coords.append(rem)
    xyz = np.stack(coords, axis=1).astype(np.float64) + _jitter(seed, n, dim, jitter)
    box = np.array(dims, dtype=np.float64)
    offsets = np.array(list(itertools.product((-1, 0, 1), repeat=dim)), dtype=np.int64)
    pts = (xyz[None, :, :] + offsets[:, None, :] * box).reshape(-1, dim)
    node = np.tile(idx, len(offsets))
    shift = np.repeat(offsets, n, axis=0)
    simp = Delaunay(pts).simplices
    cen = pts[simp].mean(axis=1)
    keep = np.all((cen >= 0.0) & (cen < box), axis=1)
    simp = simp[keep]
    conn = node[simp].astype(np.int32)
    sh = shift[simp].astype(np.int8)
    # positive orientation: swap the first two vertices of negative simplices
    v = pts[simp]
    edges = v[:, 1:, :] - v[:, :1, :]
    vol = np.linalg.det(edges)
    neg = vol < 0
    conn[neg, 0], conn[neg, 1] = conn[neg, 1].copy(), conn[neg, 0].copy()
    sh[neg, 0], sh[neg, 1] = sh[neg, 1].copy(), sh[neg, 0].copy()
    return dict(dim=dim, xyz=xyz, conn=conn, shift=sh, box=box, wall=np.zeros(n, np.uint8),
                wall_normal=np.zeros((n, dim)))


def pipe_mesh_3d(radius: float, nz: int, *, jitter: float = 0.2, seed: int = 1614) -> dict:
    """Circular pipe of the given radius, periodic along z (nz unit layers),
    with a curved no-slip wall: the setting of the concurrent pipe flow of
    Section 3.3.

    Cross-section: a centre node and concentric rings k = 1..K (K = round
    radius) at radius k radius / K, ring k carrying round(2 pi r_k) equally
    spaced nodes rotated by a seeded angle; the interior rings are jittered
    radially by +-jitter/2 and angularly by +-jitter/2 of a spacing.  The
    rings are triangulated by Delaunay (scipy), the triangles extruded
    through the layers and every prism cut into 3 tetrahedra along the
    diagonals that run from the lower-numbered vertex of a side face to the
    higher-numbered one, so the cuts of neighbouring prisms agree.  The
    outer ring is the wall, with the inward radial unit normal.  The pipe
    axis sits at (radius, radius).
    """
    from scipy.spatial import Delaunay
    K = int(round(radius))
    if K < 2 or nz < 2:
        raise ValueError("pipe needs radius >= 2 and at least 2 layers")
    pts, wall2 = [np.zeros((1, 2))], [np.zeros(1, np.uint8)]
    draw = 0
    for k in range(1, K + 1):
        rk = k * radius / K
        m = max(6, int(round(2.0 * np.pi * rk)))
        th0 = 2.0 * np.pi * uniform01(seed, 1, draw)[0]
        draw += 1
        th = th0 + 2.0 * np.pi * np.arange(m) / m
        r = np.full(m, rk)
        if k < K and jitter > 0.0:
            u = uniform01(seed, 2 * m, draw).reshape(m, 2) - 0.5
            draw += 2 * m
            r = r + jitter * u[:, 0]
            th = th + jitter * u[:, 1] * (2.0 * np.pi / m)
        pts.append(np.stack([r * np.cos(th), r * np.sin(th)], axis=1))
        wall2.append(np.full(m, 1 if k == K else 0, np.uint8))
    p2 = np.concatenate(pts)
    w2 = np.concatenate(wall2)
    n2 = p2.shape[0]
    tri = np.sort(Delaunay(p2).simplices, axis=1).astype(np.int64)   # a < b < c
    # 3 tets per prism, vertices as (2-D index, layer offset)
    pattern = [((0, 0), (1, 0), (2, 0), (2, 1)),
               ((0, 0), (1, 0), (1, 1), (2, 1)),
               ((0, 0), (0, 1), (1, 1), (2, 1))]
    layers = np.arange(nz, dtype=np.int64)
    ntri = tri.shape[0]
    conn = np.empty((3 * ntri * nz, 4), np.int64)
    shift = np.zeros((3 * ntri * nz, 4, 3), np.int8)
    L = np.repeat(layers, ntri)
    T = np.tile(tri, (nz, 1))
    for t, verts in enumerate(pattern):
        for a, (v, dl) in enumerate(verts):
            lay = L + dl
            conn[t::3, a] = (lay % nz) * n2 + T[:, v]
            shift[t::3, a, 2] = (lay // nz).astype(np.int8)
    xyz = np.empty((n2 * nz, 3))
    xyz[:, 0] = np.tile(p2[:, 0], nz) + radius
    xyz[:, 1] = np.tile(p2[:, 1], nz) + radius
    xyz[:, 2] = np.repeat(np.arange(nz, dtype=np.float64), n2)
    box = np.array([0.0, 0.0, float(nz)])
    v = xyz[conn] + shift * box
    vol = np.linalg.det(v[:, 1:, :] - v[:, :1, :])
    neg = vol < 0
    conn[neg, 2], conn[neg, 3] = conn[neg, 3].copy(), conn[neg, 2].copy()
    shift[neg, 2], shift[neg, 3] = shift[neg, 3].copy(), shift[neg, 2].copy()
    wall = np.tile(w2, nz)
    normal = np.zeros((n2 * nz, 3))
    on = wall == 1
    rr = np.hypot(xyz[on, 0] - radius, xyz[on, 1] - radius)
    normal[on, 0] = -(xyz[on, 0] - radius) / rr
    normal[on, 1] = -(xyz[on, 1] - radius) / rr
    return dict(dim=3, xyz=xyz, conn=conn.astype(np.int32), shift=shift, box=box, wall=wall,
                wall_normal=normal)


def box_mesh(dims, *, jitter: float = 0.2, seed: int = 1615) -> dict:
    """Closed box with no-slip walls on every side: a unit node grid of shape
    `dims` (2 or 3 axes), interior nodes jittered by +-jitter per coordinate,
    each square cut into 2 triangles or each cube into the 6 Kuhn
    tetrahedra, not periodic.  Wall flags and inward normals come from the
    boundary facets (inputs.mesh_files), as for a mesh read from a file."""
    from .mesh_files import _boundary
    dims = tuple(int(d) for d in dims)
    dim = len(dims)
    if dim not in (2, 3) or min(dims) < 2:
        raise ValueError("need 2 or 3 axes of at least 2 nodes")
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords, rem = [], idx
    for d in dims[:-1]:
        rem, r = np.divmod(rem, d)
        coords.append(r)
    coords.append(rem)
    ijk = np.stack(coords, axis=1)
    xyz = ijk.astype(np.float64)
    interior = np.all((ijk > 0) & (ijk < np.array(dims) - 1), axis=1)
    xyz[interior] += _jitter(seed, n, dim, jitter)[interior]
    cells = ijk[np.all(ijk < np.array(dims) - 1, axis=1)]
    stride = np.cumprod((1,) + dims[:-1])

    def node(c):
        return (c * stride).sum(axis=1)

    if dim == 2:
        corners = [[(0, 0), (1, 0), (1, 1)], [(0, 0), (1, 1), (0, 1)]]
    else:
        corners = [[tuple(v) for v in t] for t in _kuhn_corners()]
    conn = np.concatenate([np.stack([node(cells + np.array(off)) for off in t], axis=1) for t in corners])
    v = xyz[conn]
    vol = np.linalg.det(v[:, 1:, :] - v[:, :1, :])
    neg = vol < 0
    conn[neg, 0], conn[neg, 1] = conn[neg, 1].copy(), conn[neg, 0].copy()
    wall, normal = _boundary(xyz, conn, dim)
    return dict(dim=dim, xyz=xyz, conn=conn.astype(np.int32), shift=np.zeros((conn.shape[0], dim + 1, dim), np.int8),
                box=np.zeros(dim), wall=wall, wall_normal=normal)


def mesh_summary(mesh: dict) -> dict:
    return dict(dim=mesh["dim"], n_nodes=int(mesh["xyz"].shape[0]),
                n_elems=int(mesh["conn"].shape[0]),
                n_wall=int(mesh["wall"].sum()))
