"""The other workloads on the device: reduced sizes against the FP64 oracle,
full sizes through properties that hold at any size (Laplace jump,
conservation, finiteness) and FP32 against the oracle-verified FP64 path."""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import rt2d, droplet3d, ensemble2d, channel2d
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


def _oracle(oracle_mod, inst, lattice, steps):
    o = oracle_mod.Oracle(inst.mesh, lattice, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    o.step(steps)
    return o


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp32_fp16"])
def test_rayleigh_taylor_reduced(felbm, oracle_mod, precision):
    """Heavy over light between walls with gravity, 32 x 96 nodes, 40 steps:
    FP64 within 1e-11, FP32 within 2e-5 on rho, u and C; FP16 storage on rho
    and C within its rounding bound over the oracle's largest deviation."""
    w = rt2d(nx=32, ny=96)
    inst = w.instances[0]
    steps = 40
    ctx = felbm.from_workload(w, precision=precision)
    ctx.step(steps)
    ctx.sync()
    o = _oracle(oracle_mod, inst, 9, 0)
    md = max_deviation(o.get_state(), o.fields(), 9)
    o.step(steps)
    md = max(md, max_deviation(o.get_state(), o.fields(), 9))
    e = compare_fields(ctx.read_fields(0), o.fields(), inst)
    print("rt", precision, e, flush=True)
    if precision == "fp32_fp16":
        tol, keys = fp16_storage_bound(md, inst.phys.rho_l, inst.phys.rho_v, steps), ("rho", "C")
    else:
        tol, keys = {"fp64": 1e-11, "fp32": TOL32}[precision], ("rho", "u", "C")
    for k in keys:
        assert e[k] < tol, (k, e[k], tol)


def test_droplet3d_full_size_laplace(felbm):
    """128^3 periodic Kuhn-tet mesh (2.1 M nodes), D3Q19, density ratio 100,
    FP32, 500 steps: stays finite, conserves mass, and holds a pressure jump
    near 2 sigma / R (Section 3.1; the diffuse interface xi/R = 1/4 lowers it)."""
    w = droplet3d()
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision="fp32")
    c0 = ctx.conserved_sums(0)
    ctx.step(w.steps)
    ctx.sync()
    c1 = ctx.conserved_sums(0)
    assert abs(c1[0] - c0[0]) < 1e-5 * c0[0]
    f = ctx.read_fields(0)
    R, xi = inst.meta["radius"], inst.phys.xi
    d = inst.mesh["xyz"] - inst.meta["center"]
    r = np.sqrt((d ** 2).sum(1))
    dp = f["p"][r < R - xi].mean() - f["p"][r > R + xi].mean()
    ratio = dp / inst.meta["dp_laplace"]
    print("3-D Laplace dp / (2 sigma / R) =", ratio, flush=True)
    assert 0.75 < ratio < 1.1


def test_droplet3d_full_size_fp32_vs_fp64(felbm):
    """128^3 droplet (2.1 M nodes, D3Q19) at full size in the bench's launch
    configuration: the FP32 path, tuned (LDS-staged kernels where they win)
    in the mesh's node order and in Z-order, within 2e-5 of the FP64 device
    path (itself checked against the oracle on smaller 3-D meshes) after 20
    steps."""
    import torch
    w = droplet3d()
    inst = w.instances[0]
    steps = 20
    ref = felbm.from_workload(w, precision="fp64")
    ref.step(steps)
    ref.sync()
    fr = ref.read_fields(0)
    del ref
    torch.cuda.empty_cache()
    for order in (0, 1):
        ctx = felbm.from_workload(w, precision="fp32", node_order=order)
        ctx.step(steps)
        ctx.sync()
        e = compare_fields(ctx.read_fields(0), fr, inst)
        print("3-D full size fp32 vs fp64, node order", order, ctx.tuning(), e, flush=True)
        for k in ("rho", "u", "C"):
            assert e[k] < TOL32, (order, k, e[k])
        del ctx
        torch.cuda.empty_cache()


def test_ensemble_full_size_fp32_vs_fp64(felbm):
    """64 independent drops of uneven size (6.6 M nodes) advanced together:
    every instance finite and within 2e-5 of the FP64 device path."""
    w = ensemble2d()
    steps = 100
    a = felbm.from_workload(w, precision="fp32")
    a.step(steps)
    a.sync()
    b = felbm.from_workload(w, precision="fp64")
    b.step(steps)
    b.sync()
    worst = {}
    for i, inst in enumerate(w.instances):
        e = compare_fields(a.read_fields(i), b.read_fields(i), inst)
        for k in ("rho", "u", "C"):
            worst[k] = max(worst.get(k, 0.0), e[k])
    print("ensemble fp32 vs fp64 worst", worst, flush=True)
    for k in ("rho", "u", "C"):
        assert worst[k] < TOL32, (k, worst[k])


def test_ensemble_small_instances_vs_oracle(felbm, oracle_mod):
    """Eight small drops of the same recipe in one batch, FP32, against the
    oracle instance by instance."""
    w = ensemble2d(count=8, side_lo=16, side_hi=40)
    ctx = felbm.from_workload(w, precision="fp32")
    ctx.step(30)
    ctx.sync()
    for i, inst in enumerate(w.instances):
        o = _oracle(oracle_mod, inst, 9, 30)
        e = compare_fields(ctx.read_fields(i), o.fields(), inst)
        print("ensemble inst", i, inst.meta["side"], round(inst.meta["ratio"], 1), e, flush=True)
        for k in ("rho", "u", "C"):
            assert e[k] < TOL32, (i, k, e[k])


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_channel_full_length_keeps_analytic_profile(felbm, precision):
    """The 1024 x 256 layered channel (density ratio 1000) over its full 5000
    steps: the x-averaged velocity of every grid row stays on the analytic
    diffuse-interface Poiseuille profile it starts from, and the heavy-phase
    volume is kept (walls: bounce-back, so not to round-off)."""
    from paper_1608_01906_amd.inputs import channel_profile
    w = channel2d()
    inst = w.instances[0]
    m = inst.meta
    ctx = felbm.from_workload(w, precision=precision)
    s0 = ctx.conserved_sums(0)
    ctx.step(w.steps)
    ctx.sync()
    f = ctx.read_fields(0)
    nx, ny = 1024, 256
    ubar = f["u"][:, 0].reshape(ny, nx).mean(axis=1)
    y = np.arange(ny) - m["yc"]
    ph = inst.phys
    u_an = channel_profile(y, half_width=m["half_width"], core=m["core"], rho_heavy=ph.rho_l, rho_light=ph.rho_v,
                           tau_heavy=ph.tau_l, tau_light=ph.tau_v, xi=ph.xi, g=m["g"], dt=ph.dt)
    umax = u_an.max()
    dev = np.abs(ubar - u_an).max() / umax
    vmax = np.abs(f["u"][:, 1]).max() / umax
    s1 = ctx.conserved_sums(0)
    print("channel", precision, "u_max", umax, "max row deviation / u_max", dev, "max |v| / u_max", vmax,
          "heavy volume drift", s1[1] / s0[1] - 1, flush=True)
    assert dev < 0.03      # measured 1.9 % (FP32)
    assert vmax < 0.03     # spurious currents at the ratio-1000 interface, measured 1.1 %
    assert abs(s1[1] / s0[1] - 1.0) < 1e-3


def test_rayleigh_taylor_full_size_fp16_vs_fp32(felbm):
    """1024 x 4096 Rayleigh-Taylor (4.2 M nodes) over its full 2000 steps with
    FP16 and FP32 deviation storage: both stay finite, keep the heavy-phase
    volume, and the FP16 fields stay within 2e-3 of the FP32 ones.  The
    worst-case FP16 rounding bound grows linearly with the steps (0.04
    here); roundings of independent sign add up as the square root of the
    steps, sqrt(2000) 2^-11 max|delta| / (rho_l - rho_v) = 8.8e-4 at the
    largest deviation 0.027 of this workload's oracle states (0.025 at t = 0,
    0.027 after 40 steps on the 32 x 96 and 64 x 256 meshes), and the 2e-3
    bound allows about twice that."""
    w = rt2d()
    inst = w.instances[0]
    out = {}
    for precision in ("fp32", "fp32_fp16"):
        ctx = felbm.from_workload(w, precision=precision)
        s0 = ctx.conserved_sums(0)
        ctx.step(w.steps)
        ctx.sync()
        s1 = ctx.conserved_sums(0)
        out[precision] = ctx.read_fields(0)
        drift = s1[1] / s0[1] - 1.0
        print("rt", precision, "heavy volume drift", drift, flush=True)
        assert abs(drift) < 1e-4
        del ctx
    e = compare_fields(out["fp32_fp16"], out["fp32"], inst)
    print("rt fp16 vs fp32", e, flush=True)
    for k in ("rho", "u", "C"):
        assert e[k] < 2e-3, (k, e[k])
