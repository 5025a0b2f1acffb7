"""Schedule of the mass solve: population batch and LDS staging.

The batch only sets how far ahead a solver kernel issues its loads (or how
many populations an LDS pass stages); every population's row sum and its
tile reduction run in the same order, so all batches of one form give
bitwise equal states.  The staged forms (a stage per tile, a stage per
64-row wavefront) read the same neighbour values from LDS instead of
memory; they agree with the direct form to rounding (the forms may contract
multiply-adds differently) and are checked against the oracle.  The
per-wavefront form exists for ELL width 7 (the 2-D grids): forced on a 3-D
layout, or with a batch whose stage does not fit 60 KB of LDS (FP64, batch
4), the first step reports FEL_EINVAL.
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
@pytest.mark.parametrize("node_order", [0, 1])
def test_solver_schedules(felbm, oracle_mod, dim, precision, mass_mode, node_order):
    w = _workload(dim)
    steps = 6
    inst = w.instances[0]
    o = oracle_mod.Oracle(inst.mesh, w.lattice, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    o.step(steps)
    tol = 1e-11 if precision == "fp64" else 2e-5
    used = ("cheb",) if mass_mode == 2 else ("cg_init", "cg_a", "cg_b")
    states = {}
    for sg in (1, 2, 3):
        for nb in (1, 2, 4):
            print("case", dim, precision, mass_mode, node_order, sg, nb, flush=True)
            ctx = felbm.from_workload(w, precision=precision, mass_mode=mass_mode, solver_batch=nb,
                                      lds_staging=sg, node_order=node_order, fused_reductions=1)
            if sg == 3 and (dim == 3 or (precision == "fp64" and nb == 4)):
                with pytest.raises(felbm.FelError) as ei:
                    ctx.step(steps)
                assert ei.value.status == felbm.FEL_EINVAL
                continue
            ctx.step(steps)
            ctx.sync()
            states[sg, nb] = ctx.get_state(0)
            t = ctx.tuning()
            # on 3-D layouts the second CG kernel reads no neighbour values: never staged; the
            # direct FP64 kernels of ELL width 15 stop at batch 2
            for name in SOLVER:
                st = 1 if (name == "cg_b" and dim == 3) else sg
                cap = 2 if (precision == "fp64" and dim == 3 and st == 1) else 4
                assert t[name] == (min(nb, cap), st), (name, t[name])
            # the streaming kernel has a staged form (per tile) for 2-D deviation storage
            assert t["stream"] == (1, min(sg, 2) if (dim == 2 and precision != "fp64") else 1), t["stream"]
            e = compare_fields(ctx.read_fields(0), o.fields(), inst)
            for k in ("rho", "u", "C"):
                assert e[k] < tol, (sg, nb, k, e[k])
        for nb in (2, 4):
            if (sg, nb) in states:
                np.testing.assert_array_equal(states[sg, 1], states[sg, nb])
    # the tuner's choice is one of the candidates, for the kernels in use
    ctx = felbm.from_workload(w, precision=precision, mass_mode=mass_mode, node_order=node_order)
    ctx.step(steps)
    ctx.sync()
    t = ctx.tuning()
    for name in SOLVER:
        b, sg = t[name]
        assert (b in (1, 2, 4) and sg in (1, 2, 3)) if name in used else (b, sg) == (1, 1), (name, t[name])
    e = compare_fields(ctx.read_fields(0), o.fields(), inst)
    for k in ("rho", "u", "C"):
        assert e[k] < tol, ("tuned", k, e[k])


def test_tuning_reads_zero_before_first_step(felbm):
    w = _workload(2)
    ctx = felbm.from_workload(w, precision="fp32")
    t = ctx.tuning()
    assert all(t[k] == (0, 0) for k in SOLVER)
    assert t["stream"] == (1, 0)
    ctx.step(1)
    ctx.sync()
    t = ctx.tuning()
    assert t["cheb"] == (1, 1) and t["fused"] in (1, 2)
    assert t["stream"] in ((1, 1), (1, 2))
    assert all(t[k][0] in (1, 2, 4) and t[k][1] in (1, 2, 3) for k in ("cg_init", "cg_a", "cg_b"))


@pytest.mark.parametrize("node_order", [0, 1])
def test_staged_stream_fp16_storage_vs_oracle(felbm, oracle_mod, node_order):
    """FP16 deviation storage with every kernel LDS-staged (the streaming
    kernel's staged form converts the stored FP16 values as the direct one
    does) and with every kernel direct, against the oracle within the FP16
    storage bound; the two forms agree to rounding."""
    from tests._parity import fp16_storage_bound, max_deviation
    w = _workload(2)
    inst = w.instances[0]
    steps = 6
    o = oracle_mod.Oracle(inst.mesh, w.lattice, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    d0 = max_deviation(o.get_state(), o.fields(), w.lattice)
    o.step(steps)
    ref = o.fields()
    tol = fp16_storage_bound(max(d0, max_deviation(o.get_state(), ref, w.lattice)), inst.phys.rho_l,
                             inst.phys.rho_v, steps)
    got = {}
    for sg in (1, 2, 3):
        ctx = felbm.from_workload(w, precision="fp32_fp16", lds_staging=sg, node_order=node_order,
                                  fused_reductions=1)
        ctx.step(steps)
        ctx.sync()
        assert ctx.tuning()["stream"] == (1, min(sg, 2))
        got[sg] = ctx.read_fields(0)
        e = compare_fields(got[sg], ref, inst)
        print("fp16 storage, staging", sg, {k: f"{v:.2e}" for k, v in e.items()}, "bound", f"{tol:.2e}", flush=True)
        for k in ("rho", "C"):
            assert e[k] < tol, (sg, k, e[k], tol)
    for sg in (2, 3):
        e = compare_fields(got[sg], got[1], inst)
        assert e["rho"] < 1e-5 and e["C"] < 1e-4, (sg, e)


@pytest.mark.parametrize("mass_mode", [0, 2])
def test_partly_fixed_schedules_are_kept(felbm, mass_mode):
    """Options that fix part of the schedule hold through the whole tuning,
    the in-context pass that times whole solves included: a fixed staging
    leaves only batches to choose, a fixed batch only the staging (finalize
    launches forced, so the choice applies to the kernels that run)."""
    w = _workload(2)
    classes = ("cg_init", "cg_a", "cg_b") if mass_mode == 0 else ("cheb",)
    for sg in (1, 2, 3):
        ctx = felbm.from_workload(w, precision="fp32", mass_mode=mass_mode, lds_staging=sg, fused_reductions=1)
        ctx.step(1)
        ctx.sync()
        t = ctx.tuning()
        print("staging fixed", sg, t, flush=True)
        assert all(t[k][1] == sg and t[k][0] in (1, 2, 4) for k in classes)
    for b in (1, 2, 4):
        ctx = felbm.from_workload(w, precision="fp32", mass_mode=mass_mode, solver_batch=b, fused_reductions=1)
        ctx.step(1)
        ctx.sync()
        t = ctx.tuning()
        print("batch fixed", b, t, flush=True)
        assert all(t[k][0] == b and t[k][1] in (1, 2, 3) for k in classes)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_fused_reductions_vs_oracle(felbm, oracle_mod, precision, tol):
    """The fused-reduction CG (no finalize launches) against the oracle, on
    one instance and on three uneven instances in one batch (one of them a
    single partial tile); all fused batches give bitwise equal states.  The
    fused kernels are built only for the batches that fit their 128
    registers per thread (cg_a 1; cg_init 4 / 2 and cg_b 4 / 1 in FP32 /
    FP64): a larger requested batch runs as the largest built."""
    from paper_1608_01906_amd.inputs import Workload, droplet_instance, grid_mesh_2d
    insts = []
    for i, (n, ratio) in enumerate([(11, 10.0), (70, 3.0), (37, 20.0)]):
        mesh = grid_mesh_2d(n, n, seed=700 + i)
        insts.append(droplet_instance(mesh, radius=n / 4, rho_l=1.0, rho_v=1.0 / ratio, sigma=0.01, xi=4.0,
                                      tau_l=0.05, tau_v=0.1, center=np.array([n / 2, n / 2])))
    w = Workload("batch3", 9, insts, 8)
    states = {}
    for nb in (1, 2, 4):
        ctx = felbm.from_workload(w, precision=precision, fused_reductions=2, solver_batch=nb)
        ctx.step(8)
        ctx.sync()
        t = ctx.tuning()
        assert t["fused"] == 2 and t["cg_a"][0] == 1, t
        assert t["cg_init"][0] == min(nb, 4 if precision == "fp32" else 2), t
        assert t["cg_b"][0] == min(nb, 4 if precision == "fp32" else 1), t
        states[nb] = [ctx.get_state(i) for i in range(len(insts))]
        if nb == 2:
            for i, inst in enumerate(insts):
                o = oracle_mod.Oracle(inst.mesh, 9, inst.phys)
                o.init(inst.rho0, inst.u0, inst.p0)
                o.step(8)
                e = compare_fields(ctx.read_fields(i), o.fields(), inst)
                print("fused", precision, "inst", i, e, flush=True)
                for k in ("rho", "u", "C"):
                    assert e[k] < tol, (i, k, e[k])
    for nb in (2, 4):
        for a, b in zip(states[1], states[nb]):
            np.testing.assert_array_equal(a, b)


def test_fused_matches_finalize_path(felbm):
    """Fused and finalize-launch CG solve the same systems: states agree to
    rounding after 20 steps of the 64 x 64 droplet, and the tuner's choice
    is one of the two."""
    w = droplet2d(64)
    a = felbm.from_workload(w, precision="fp64", fused_reductions=1)
    b = felbm.from_workload(w, precision="fp64", fused_reductions=2)
    c = felbm.from_workload(w, precision="fp64")
    for ctx in (a, b, c):
        ctx.step(20)
        ctx.sync()
    assert a.tuning()["fused"] == 1 and b.tuning()["fused"] == 2 and c.tuning()["fused"] in (1, 2)
    np.testing.assert_allclose(b.get_state(0), a.get_state(0), rtol=0, atol=1e-12)


def test_fused_unavailable_cases(felbm):
    """3-D layouts and instances above 1024 tiles cannot take the fused path:
    asking for it with the CG solve is an error at bind, the tuner falls
    back to finalize launches."""
    from paper_1608_01906_amd.inputs import grid_mesh_2d, droplet_instance, Workload
    w3 = droplet3d(11, radius=3.0, xi=3.0)
    with pytest.raises(felbm.FelError):
        felbm.from_workload(w3, fused_reductions=2)
    ctx = felbm.from_workload(w3)
    ctx.step(1)
    ctx.sync()
    assert ctx.tuning()["fused"] == 1
    # the reduction-free Chebyshev solve ignores the option
    ctx = felbm.from_workload(w3, mass_mode=2, fused_reductions=2)
    ctx.step(1)
    ctx.sync()
    assert ctx.tuning()["fused"] == 1
    big = grid_mesh_2d(520, 520, seed=9)          # 270,400 nodes = 1057 tiles
    inst = droplet_instance(big, radius=100.0, rho_l=1.0, rho_v=0.1, sigma=0.01, xi=4.0, tau_l=0.05, tau_v=0.05)
    wb = Workload("big", 9, [inst], 1)
    with pytest.raises(felbm.FelError):
        felbm.from_workload(wb, precision="fp32", fused_reductions=2)
    ctx = felbm.from_workload(wb, precision="fp32")
    ctx.step(1)
    ctx.sync()
    assert ctx.tuning()["fused"] == 1


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
@pytest.mark.parametrize("stage", [2, 3])
def test_staged_forms_uneven_batch_vs_oracle(felbm, oracle_mod, precision, tol, stage):
    """Both LDS stagings (per tile, per 64-row wavefront) on three uneven
    instances in one Z-ordered layout (sides 11, 70, 37: a single partial
    tile, full and ragged tiles, wavefronts that straddle instance padding),
    every population batch, against the oracle on each instance; the
    batches of one form are bitwise equal."""
    from paper_1608_01906_amd.inputs import Workload, droplet_instance, grid_mesh_2d
    insts = []
    for i, (n, ratio) in enumerate([(11, 10.0), (70, 3.0), (37, 20.0)]):
        mesh = grid_mesh_2d(n, n, seed=900 + i)
        insts.append(droplet_instance(mesh, radius=n / 4, rho_l=1.0, rho_v=1.0 / ratio, sigma=0.01, xi=4.0,
                                      tau_l=0.05, tau_v=0.1, center=np.array([n / 2, n / 2])))
    w = Workload("batch3", 9, insts, 6)
    refs = []
    for inst in insts:
        o = oracle_mod.Oracle(inst.mesh, 9, inst.phys)
        o.init(inst.rho0, inst.u0, inst.p0)
        o.step(6)
        refs.append(o.fields())
    states = {}
    for nb in (1, 2) if precision == "fp64" and stage == 3 else (1, 2, 4):
        print("case", precision, stage, nb, flush=True)
        ctx = felbm.from_workload(w, precision=precision, solver_batch=nb, lds_staging=stage, node_order=1,
                                  fused_reductions=1)
        ctx.step(6)
        ctx.sync()
        t = ctx.tuning()
        assert all(t[k] == (nb, stage) for k in ("cg_init", "cg_a", "cg_b")), t
        states[nb] = [ctx.get_state(i) for i in range(len(insts))]
        for i, inst in enumerate(insts):
            e = compare_fields(ctx.read_fields(i), refs[i], inst)
            for k in ("rho", "u", "C"):
                assert e[k] < tol, (nb, i, k, e[k])
    for nb in states:
        for a, b in zip(states[1], states[nb]):
            np.testing.assert_array_equal(a, b)
