"""External simplex meshes: Gmsh 2.2 ASCII files.

The paper runs on meshes from a mesher (Section 3.1, Table 1); the workloads
here are generated, and this module lets a caller bring a mesh of their own
instead.  `read_gmsh` returns the mesh dictionary of `inputs.mesh`: the
top-dimensional simplices (triangles, element type 2, for a 2-D mesh whose
nodes all have z = 0; tetrahedra, type 4, otherwise) become the elements,
oriented positively; lower-dimensional elements are ignored.  The mesh is
not periodic; every node on a boundary facet (an edge or triangle of one
element only) is a wall node.  Its inward normal is the negated mean of the
unit outward normals of its boundary facets, each triangle weighted by its
angle at the node (the two edges of a 2-D boundary node weigh the same), so
a node on a flat face gets the face normal and a node on an edge or corner
of flat faces the normalised sum of their normals, whatever the
triangulation of the faces.
`write_gmsh` writes a non-periodic mesh dictionary in the same format.

No arithmetic of the method is here.
"""
from __future__ import annotations

import numpy as np

_TRI, _TET = 2, 4


def _sections(text: str) -> dict:
    out, name, body = {}, None, []
    for line in text.splitlines():
        s = line.strip()
        if s.startswith("$End"):
            out[name] = body
            name, body = None, []
        elif s.startswith("$"):
            name = s[1:]
        elif name is not None and s:
            body.append(s)
    return out


def read_gmsh(path: str) -> dict:
    """Reads a Gmsh 2.2 ASCII mesh file (see the module docstring)."""
    with open(path) as f:
        sec = _sections(f.read())
    fmt = sec.get("MeshFormat", ["?"])[0].split()
    if not fmt or not fmt[0].startswith("2") or (len(fmt) > 1 and fmt[1] != "0"):
        raise ValueError(f"{path}: only Gmsh 2.x ASCII meshes are read")
    nodes = sec["Nodes"]
    n = int(nodes[0])
    ids = np.empty(n, np.int64)
    xyz = np.empty((n, 3))
    for i, line in enumerate(nodes[1:n + 1]):
        p = line.split()
        ids[i] = int(p[0])
        xyz[i] = [float(v) for v in p[1:4]]
    index = {int(k): i for i, k in enumerate(ids)}
    elems = {_TRI: [], _TET: []}
    body = sec["Elements"]
    for line in body[1:int(body[0]) + 1]:
        p = [int(v) for v in line.split()]
        etype, ntags = p[1], p[2]
        if etype in elems:
            elems[etype].append([index[k] for k in p[3 + ntags:]])
    if elems[_TET]:
        dim, conn = 3, np.array(elems[_TET], np.int64)
    elif elems[_TRI]:
        if np.any(xyz[:, 2] != 0.0):
            raise ValueError(f"{path}: triangles off the z = 0 plane (a surface mesh, not a 2-D domain)")
        dim, conn = 2, np.array(elems[_TRI], np.int64)
    else:
        raise ValueError(f"{path}: no triangles or tetrahedra")
    used = np.unique(conn)
    if used.size != n:  # drop nodes no element references (geometry points)
        remap = -np.ones(n, np.int64)
        remap[used] = np.arange(used.size)
        conn = remap[conn]
        xyz = xyz[used]
        n = used.size
    xyz = np.ascontiguousarray(xyz[:, :dim])
    # positive orientation
    v = xyz[conn]
    vol = np.linalg.det(v[:, 1:, :] - v[:, :1, :])
    if np.any(vol == 0.0):
        raise ValueError(f"{path}: degenerate element")
    neg = vol < 0
    conn[neg, 0], conn[neg, 1] = conn[neg, 1].copy(), conn[neg, 0].copy()
    wall, normal = _boundary(xyz, conn, dim)
    return dict(dim=dim, xyz=xyz, conn=conn.astype(np.int32), shift=np.zeros((conn.shape[0], dim + 1, dim), np.int8),
                box=np.zeros(dim), wall=wall, wall_normal=normal)


def _boundary(xyz, conn, dim):
    """Wall flags and inward unit normals from the facets of one element."""
    nv = dim + 1
    facets = np.concatenate([conn[:, [j for j in range(nv) if j != skip]] for skip in range(nv)])
    opposite = np.concatenate([conn[:, skip] for skip in range(nv)])
    key = np.sort(facets, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    open_ = cnt[inv.ravel()] == 1
    f, opp = facets[open_], opposite[open_]
    p = xyz[f]
    if dim == 2:
        t = p[:, 1] - p[:, 0]
        nrm = np.stack([t[:, 1], -t[:, 0]], axis=1)
    else:
        nrm = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    # outward: away from the element's opposite vertex
    flip = ((p[:, 0] - xyz[opp]) * nrm).sum(axis=1) < 0
    nrm[flip] *= -1
    n = xyz.shape[0]
    acc = np.zeros((n, dim))
    for j in range(dim):
        if dim == 2:
            wgt = np.ones(len(f))
        else:  # the facet's angle at vertex j
            e1 = p[:, (j + 1) % 3] - p[:, j]
            e2 = p[:, (j + 2) % 3] - p[:, j]
            c = (e1 * e2).sum(axis=1) / (np.linalg.norm(e1, axis=1) * np.linalg.norm(e2, axis=1))
            wgt = np.arccos(np.clip(c, -1.0, 1.0))
        np.add.at(acc, f[:, j], wgt[:, None] * nrm)
    wall = np.zeros(n, np.uint8)
    wall[np.unique(f)] = 1
    normal = np.zeros((n, dim))
    on = wall == 1
    normal[on] = -acc[on] / np.linalg.norm(acc[on], axis=1)[:, None]
    return wall, normal


def write_gmsh(mesh: dict, path: str) -> None:
    """Writes a non-periodic mesh dictionary as a Gmsh 2.2 ASCII file."""
    if np.any(mesh["shift"] != 0):
        raise ValueError("periodic meshes have no Gmsh 2.2 form here")
    xyz, conn, dim = mesh["xyz"], mesh["conn"], mesh["dim"]
    etype = _TET if dim == 3 else _TRI
    with open(path, "w") as f:
        f.write("$MeshFormat\n2.2 0 8\n$EndMeshFormat\n$Nodes\n")
        f.write(f"{xyz.shape[0]}\n")
        for i, p in enumerate(xyz):
            z = float(p[2]) if dim == 3 else 0.0
            f.write(f"{i + 1} {float(p[0])!r} {float(p[1])!r} {z!r}\n")
        f.write("$EndNodes\n$Elements\n")
        f.write(f"{conn.shape[0]}\n")
        for e, c in enumerate(conn):
            f.write(f"{e + 1} {etype} 2 1 1 " + " ".join(str(int(k) + 1) for k in c) + "\n")
        f.write("$EndElements\n")
