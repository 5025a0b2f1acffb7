"""Seeded input generators: random stream, mesh validity, workload shapes."""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import (grid_mesh_2d, grid_mesh_3d, splitmix64, uniform01, droplet2d,
                                         channel2d, ensemble2d)
from tests._bruteforce import unwrap


def test_splitmix64_published_values():
    # SplitMix64 seeded with 0: first outputs of the reference generator
    # (Steele, Lea, Flood 2014; also the seeding generator of xoshiro).
    z = splitmix64(0, 3)
    assert int(z[0]) == 0xE220A8397B1DCDAF
    assert int(z[1]) == 0x6E789E6AA1B965F4
    assert int(z[2]) == 0x06C45D188009454F
    # counter form: draws i..j equal the tail of a longer stream
    assert np.array_equal(splitmix64(99, 5, start=7), splitmix64(99, 12)[7:])
    u = uniform01(5, 100000)
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.01


def _signed_volumes(mesh):
    out = []
    for e in range(mesh["conn"].shape[0]):
        X = unwrap(mesh, e)
        J = (X[1:] - X[0]).T
        out.append(np.linalg.det(J))
    return np.array(out)


@pytest.mark.parametrize("wall", [False, True])
def test_mesh2d_valid(wall):
    m = grid_mesh_2d(7, 6, wall_y=wall, seed=3)
    n_cells = 7 * (5 if wall else 6)
    assert m["conn"].shape == (2 * n_cells, 3)
    v = _signed_volumes(m) / 2
    assert v.min() > 0.05
    assert abs(v.sum() - (7 * (5 if wall else 6))) < 1e-9  # tiling covers the box exactly
    jit = m["xyz"] - np.stack(np.divmod(np.arange(42), 7)[::-1], axis=1)
    assert np.abs(jit).max() <= 0.2
    if wall:
        assert m["wall"].sum() == 14
        assert np.all(jit[m["wall"] == 1, 1] == 0.0)
        ys = m["xyz"][:, 1]
        assert np.all(m["wall_normal"][ys == 0][:, 1] == 1.0)


def test_mesh3d_valid():
    m = grid_mesh_3d(3, 4, 5, seed=9)
    assert m["conn"].shape == (6 * 60, 4)
    v = _signed_volumes(m) / 6
    assert v.min() > 0.0
    assert abs(v.sum() - 60.0) < 1e-9


def test_workloads_shapes():
    w = droplet2d()
    assert w.n_nodes == 4096 and w.lattice == 9
    inst = w.instances[0]
    assert inst.rho0.max() <= 1.0 and inst.rho0.min() >= 0.1
    w = channel2d(nx=16, ny=32)
    inst = w.instances[0]
    assert inst.mesh["wall"].sum() == 32
    assert inst.u0[inst.mesh["wall"] == 1].max() < 1e-3
    e = ensemble2d(count=4, side_lo=8, side_hi=16)
    assert len(e.instances) == 4
    assert all(1.05 <= i.meta["ratio"] <= 1000 for i in e.instances)
