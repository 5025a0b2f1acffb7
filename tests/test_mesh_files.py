"""Meshes from files (Gmsh 2.2 ASCII): the reader a caller uses to bring
a mesh of their own, with walls on every boundary facet.

  * round trip: generated closed-box meshes (2-D triangles, 3-D Kuhn
    tetrahedra) written and read back give the same nodes, elements, wall
    flags and normals;
  * a hand-written file with non-contiguous node numbers, lower-dimensional
    elements, a geometry point no element uses and a negatively oriented
    triangle reads as the intended mesh;
  * walls are exactly the nodes on the box surface, normals point inward:
    the face normal on a face, the normalised sum of the face normals on an
    edge or corner;
  * surface meshes and degenerate elements are refused.
"""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import box_droplet, box_mesh, read_gmsh, write_gmsh


@pytest.mark.parametrize("dims", [(9, 7), (5, 4, 6)])
def test_round_trip(tmp_path, dims):
    m = box_mesh(dims)
    path = tmp_path / "box.msh"
    write_gmsh(m, str(path))
    r = read_gmsh(str(path))
    assert r["dim"] == len(dims)
    np.testing.assert_array_equal(r["xyz"], m["xyz"])
    np.testing.assert_array_equal(np.sort(r["conn"], axis=1), np.sort(m["conn"], axis=1))
    np.testing.assert_array_equal(r["wall"], m["wall"])
    np.testing.assert_allclose(r["wall_normal"], m["wall_normal"], atol=1e-15)
    assert not r["shift"].any() and not r["box"].any()


@pytest.mark.parametrize("dims", [(9, 7), (5, 4, 6)])
def test_box_walls_and_normals(dims):
    m = box_mesh(dims)
    dim = len(dims)
    xyz = m["xyz"]
    v = xyz[m["conn"]]
    vol = np.linalg.det(v[:, 1:, :] - v[:, :1, :])
    assert vol.min() > 0
    np.testing.assert_allclose(vol.sum() / (2 if dim == 2 else 6), np.prod(np.array(dims) - 1.0), rtol=1e-12)
    hi = np.array(dims) - 1.0
    lo_side = xyz == 0.0
    hi_side = xyz == hi
    on_surface = np.any(lo_side | hi_side, axis=1)
    np.testing.assert_array_equal(m["wall"].astype(bool), on_surface)
    want = (lo_side.astype(float) - hi_side.astype(float))[on_surface]
    want /= np.linalg.norm(want, axis=1)[:, None]
    np.testing.assert_allclose(m["wall_normal"][on_surface], want, atol=1e-12)


def test_hand_written_file(tmp_path):
    text = """$MeshFormat
2.2 0 8
$EndMeshFormat
$Nodes
6
10 0 0 0
20 1 0 0
30 1 1 0
40 0 1 0
50 0.5 0.5 0
99 7 7 0
$EndNodes
$Elements
8
1 15 2 0 1 99
2 1 2 0 1 10 20
3 1 2 0 1 20 30
4 2 2 0 1 10 20 50
5 2 2 0 1 20 30 50
6 2 2 0 1 30 40 50
7 2 2 0 1 40 10 50
8 2 2 0 1 50 30 40
$EndElements
"""
    path = tmp_path / "square.msh"
    path.write_text(text.replace("8 2 2 0 1 50 30 40\n", "").replace("$Elements\n8", "$Elements\n7"))
    m = read_gmsh(str(path))
    assert m["dim"] == 2 and m["xyz"].shape == (5, 2) and m["conn"].shape == (4, 3)
    np.testing.assert_array_equal(m["xyz"][4], [0.5, 0.5])
    v = m["xyz"][m["conn"]]
    assert np.all(np.linalg.det(v[:, 1:, :] - v[:, :1, :]) > 0)
    np.testing.assert_array_equal(m["wall"], [1, 1, 1, 1, 0])
    s = np.sqrt(0.5)
    np.testing.assert_allclose(m["wall_normal"][:4], [[s, s], [-s, s], [-s, -s], [s, -s]], atol=1e-15)
    # a clockwise triangle is reoriented
    path.write_text(text.replace("6 2 2 0 1 30 40 50\n", "").replace("$Elements\n8", "$Elements\n7")
                    .replace("8 2 2 0 1 50 30 40", "8 2 2 0 1 50 40 30"))
    m2 = read_gmsh(str(path))
    v = m2["xyz"][m2["conn"]]
    assert np.all(np.linalg.det(v[:, 1:, :] - v[:, :1, :]) > 0)
    np.testing.assert_array_equal(m2["wall"], m["wall"])


def test_refused_files(tmp_path):
    surface = """$MeshFormat
2.2 0 8
$EndMeshFormat
$Nodes
3
1 0 0 0
2 1 0 0
3 0 1 1
$EndNodes
$Elements
1
1 2 2 0 1 1 2 3
$EndElements
"""
    p = tmp_path / "s.msh"
    p.write_text(surface)
    with pytest.raises(ValueError, match="surface"):
        read_gmsh(str(p))
    p.write_text(surface.replace("3 0 1 1", "3 2 0 0"))
    with pytest.raises(ValueError, match="degenerate"):
        read_gmsh(str(p))
    p.write_text(surface.replace("2.2 0 8", "4.1 0 8"))
    with pytest.raises(ValueError, match="2.x"):
        read_gmsh(str(p))


def test_oracle_drop_in_a_closed_box_from_a_file(tmp_path, oracle_mod):
    """A drop in a closed 2-D box read from a file: 50 oracle steps keep it
    finite and at rest, its spurious currents those of the same drop in a
    periodic square (5 % and 4.5 % of the Laplace velocity scale
    sqrt(sigma / (rho_l R)) at this early point), and the bounce-back walls
    change the mass only by the populations they replace (3.7e-4 here)."""
    path = tmp_path / "box.msh"
    write_gmsh(box_mesh((24, 24)), str(path))
    w = box_droplet(mesh=read_gmsh(str(path)), xi=4.0)
    inst = w.instances[0]
    o = oracle_mod.Oracle(inst.mesh, w.lattice, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    s0 = o.conserved()
    o.step(50)
    f = o.fields()
    s1 = o.conserved()
    assert np.isfinite(f["rho"]).all()
    scale = np.sqrt(inst.phys.sigma / (inst.phys.rho_l * inst.meta["radius"]))
    assert np.abs(f["u"]).max() < 0.1 * scale
    assert abs(s1[0] / s0[0] - 1.0) < 1e-3
