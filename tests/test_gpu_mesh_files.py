"""Meshes read from files on the device: a drop in a closed box, walls on
every side (corner and edge nodes with diagonal normals), the mesh written
to and read back from a Gmsh 2.2 file, against the oracle over 20 steps:
FP64 within 1e-11, FP32 within 2e-5 on rho, u and C (2-D triangles and 3-D
Kuhn tetrahedra)."""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import box_droplet, box_mesh, read_gmsh, write_gmsh
from tests._parity import U32, U64, compare_fields, max_deviation, velocity_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def felbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_01906_amd import felbm as F
    F.load_library()
    return F


@pytest.mark.parametrize("dims", [(32, 32), (12, 12, 12)], ids=["2d", "3d"])
def test_box_drop_from_file_vs_oracle(felbm, oracle_mod, tmp_path, dims):
    path = tmp_path / "box.msh"
    write_gmsh(box_mesh(dims), str(path))
    w = box_droplet(mesh=read_gmsh(str(path)), xi=4.0)
    inst = w.instances[0]
    dim = len(dims)
    o = oracle_mod.Oracle(inst.mesh, w.lattice, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    d0 = max_deviation(o.get_state(), o.fields(), w.lattice)
    o.step(20)
    ref = o.fields()
    md = max(d0, max_deviation(o.get_state(), ref, w.lattice))
    for precision, tol, eps in (("fp64", 1e-11, U64), ("fp32", 2e-5, U32)):
        ctx = felbm.from_workload(w, precision=precision)
        ctx.step(20)
        ctx.sync()
        e = compare_fields(ctx.read_fields(0), ref, inst)
        ctx.close()
        print("box drop from file", dims, precision, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
        for k in ("rho", "u", "C"):
            assert e[k] < tol, (dims, precision, k, e[k])
        ub = velocity_bound(md, inst.phys.rho_v, float(np.abs(ref["u"]).max()), dim, 20, eps, arith=tol)
        assert e["u_rel"] < ub, (dims, precision, e["u_rel"], ub)
