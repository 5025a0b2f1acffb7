"""FP32 device path (scaled-deviation population storage, FP32 operators
and collision, FP64 CG dots and sums) against the FP64 oracle.

Bound: 2e-5 max-norm error relative to max(|oracle|, floor) on rho, u and
the composition C.  The pressure is a small difference of large populations
and is held to a looser bound, stated per test.  FP16 deviation storage is
reported and held to the bounds measured for it.
"""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import droplet2d, droplet3d, channel2d, Workload, droplet_instance, grid_mesh_2d
from tests._parity import compare_fields, fp16_storage_bound, max_deviation

pytestmark = pytest.mark.gpu

TOL32 = 2e-5


@pytest.fixture(scope="module")
def felbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_01906_amd import felbm as F
    F.load_library()
    return F


def _oracle(oracle_mod, inst, lattice, steps, **kw):
    o = oracle_mod.Oracle(inst.mesh, lattice, inst.phys, **kw)
    o.init(inst.rho0, inst.u0, inst.p0)
    if steps:
        o.step(steps)
    return o


def _errs(ctx, o, inst, i=0, label=""):
    e = compare_fields(ctx.read_fields(i), o.fields(), inst)
    print(label, {k: f"{v:.2e}" for k, v in e.items()}, flush=True)
    return e


def test_fp32_init_state(felbm, oracle_mod):
    w = droplet2d(24)
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision="fp32")
    o = _oracle(oracle_mod, inst, 9, 0)
    st, ref = ctx.get_state(0), o.get_state()
    assert np.abs(st - ref).max() < 2e-7 * np.abs(ref).max()


def test_fp32_droplet_full_length(felbm, oracle_mod):
    w = droplet2d()
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision="fp32")
    c0 = ctx.conserved_sums(0)
    ctx.step(w.steps)
    ctx.sync()
    o = _oracle(oracle_mod, inst, 9, w.steps)
    e = _errs(ctx, o, inst, label="fp32 droplet 200")
    for k in ("rho", "u", "C"):
        assert e[k] < TOL32, (k, e[k])
    assert e["p"] < 1e-3
    c1 = ctx.conserved_sums(0)
    assert abs(c1[0] - c0[0]) < 1e-6 * c0[0]


def test_fp32_channel(felbm, oracle_mod):
    w = channel2d(nx=20, ny=37)
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision="fp32")
    ctx.step(30)
    ctx.sync()
    o = _oracle(oracle_mod, inst, 9, 30)
    e = _errs(ctx, o, inst, label="fp32 channel 30")
    for k in ("rho", "u", "C"):
        assert e[k] < TOL32, (k, e[k])


def test_fp32_batched(felbm, oracle_mod):
    insts = []
    for i, (n, ratio) in enumerate([(11, 10.0), (40, 3.0), (23, 20.0)]):
        mesh = grid_mesh_2d(n, n, seed=500 + i)
        insts.append(droplet_instance(mesh, radius=n / 4, rho_l=1.0, rho_v=1.0 / ratio, sigma=0.01, xi=4.0,
                                      tau_l=0.05, tau_v=0.1, center=np.array([n / 2, n / 2])))
    w = Workload("batch3", 9, insts, 10)
    ctx = felbm.from_workload(w, precision="fp32")
    ctx.step(20)
    ctx.sync()
    for i, inst in enumerate(insts):
        o = _oracle(oracle_mod, inst, 9, 20)
        e = _errs(ctx, o, inst, i=i, label=f"fp32 batch {i}")
        for k in ("rho", "u", "C"):
            assert e[k] < TOL32, (i, k, e[k])


def test_fp32_3d(felbm, oracle_mod):
    w = droplet3d(10, radius=3.0, xi=3.0)
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision="fp32")
    ctx.step(5)
    ctx.sync()
    o = _oracle(oracle_mod, inst, 19, 5)
    e = _errs(ctx, o, inst, label="fp32 3d 5")
    for k in ("rho", "u", "C"):
        assert e[k] < TOL32, (k, e[k])


def test_fp16_storage_droplet(felbm, oracle_mod):
    """FP16 deviations (x 2^8) against the oracle, within the FP16 rounding
    bound (one rounding of every stored deviation per step, linear
    accumulation) over the largest deviation of the oracle's states."""
    w = droplet2d(32, radius=8.0)
    inst = w.instances[0]
    steps = 50
    ctx = felbm.from_workload(w, precision="fp32_fp16")
    ctx.step(steps)
    ctx.sync()
    o = _oracle(oracle_mod, inst, 9, 0)
    md = max_deviation(o.get_state(), o.fields(), 9)
    o.step(steps)
    md = max(md, max_deviation(o.get_state(), o.fields(), 9))
    tol = fp16_storage_bound(md, inst.phys.rho_l, inst.phys.rho_v, steps)
    e = _errs(ctx, o, inst, label=f"fp16 storage droplet {steps} (bound {tol:.2e})")
    for k in ("rho", "C"):
        assert e[k] < tol, (k, e[k], tol)


def test_fp32_checkpoint_roundtrip(felbm):
    w = droplet2d(32, radius=8.0)
    a = felbm.from_workload(w, precision="fp32")
    a.step(3)
    st = a.get_state(0)
    b = felbm.from_workload(w, precision="fp32")
    b.set_state(0, st)
    st2 = b.get_state(0)
    assert np.abs(st2 - st).max() < 1e-7 * np.abs(st).max()


def test_fp32_full_size_channel_prefix(felbm, oracle_mod):
    w = channel2d()
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision="fp32")
    ctx.step(2)
    ctx.sync()
    o = _oracle(oracle_mod, inst, 9, 2)
    e = _errs(ctx, o, inst, label="fp32 channel full 2")
    for k in ("rho", "u", "C"):
        assert e[k] < TOL32, (k, e[k])


def test_fp32_chebyshev_channel(felbm, oracle_mod):
    w = channel2d(nx=20, ny=37)
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision="fp32", mass_mode=2)
    ctx.step(30)
    ctx.sync()
    o = _oracle(oracle_mod, inst, 9, 30)
    e = _errs(ctx, o, inst, label="fp32 chebyshev channel 30")
    for k in ("rho", "u", "C"):
        assert e[k] < TOL32, (k, e[k])
