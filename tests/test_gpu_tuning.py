"""Population batch of the mass-solve pipelines.

The batch only sets how far ahead a solver kernel issues its loads; every
population's row sum and its tile reduction run in the same order, so every
setting (and the per-kernel choice the library times on the first step)
must give bitwise equal states, and one of them is checked against the
oracle.
"""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import droplet2d, droplet3d
from tests._parity import compare_fields

pytestmark = pytest.mark.gpu

SOLVER = ("cg_init", "cg_a", "cg_b", "cheb")


@pytest.fixture(scope="module")
def felbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_01906_amd import felbm as F
    F.load_library()
    return F


def _workload(dim):
    # 37^2 = 1369 rows (5 full tiles and a ragged one); 11^3 = 1331 rows
    return droplet2d(37, radius=9.0) if dim == 2 else droplet3d(11, radius=3.0, xi=3.0)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("mass_mode", [0, 2])
def test_solver_batch_bitwise_equal(felbm, oracle_mod, dim, precision, mass_mode):
    w = _workload(dim)
    steps = 6
    states = {}
    for nb in (1, 2, 4, 0):
        print("case", dim, precision, mass_mode, nb, flush=True)
        ctx = felbm.from_workload(w, precision=precision, mass_mode=mass_mode, solver_batch=nb)
        ctx.step(steps)
        ctx.sync()
        states[nb] = ctx.get_state(0)
        t = ctx.tuning()
        used = ("cheb",) if mass_mode == 2 else ("cg_init", "cg_a", "cg_b")
        for name in SOLVER:
            if nb:
                assert t[name] == nb
            else:
                assert t[name] in ((1, 2, 4) if name in used else (1,)), (name, t[name])
        assert all(v == 1 for k, v in t.items() if k not in SOLVER)
        if nb == 4:
            inst = w.instances[0]
            o = oracle_mod.Oracle(inst.mesh, w.lattice, inst.phys)
            o.init(inst.rho0, inst.u0, inst.p0)
            o.step(steps)
            e = compare_fields(ctx.read_fields(0), o.fields(), inst)
            tol = 1e-11 if precision == "fp64" else 2e-5
            for k in ("rho", "u", "C"):
                assert e[k] < tol, (k, e[k])
    for nb in (2, 4, 0):
        np.testing.assert_array_equal(states[1], states[nb])


def test_tuning_reads_zero_before_first_step(felbm):
    w = _workload(2)
    ctx = felbm.from_workload(w, precision="fp32")
    t = ctx.tuning()
    assert all(t[k] == 0 for k in SOLVER)
    ctx.step(1)
    ctx.sync()
    t = ctx.tuning()
    assert t["cheb"] == 1 and all(t[k] in (1, 2, 4) for k in ("cg_init", "cg_a", "cg_b"))
