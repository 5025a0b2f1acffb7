"""Droplet translation (Section 3.2, in 2-D) on the device: a prefix against
the oracle, and a full round trip against what a Galilean-invariant scheme
must give (drop back at its start, still round, mass and momentum kept)."""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import translate2d
from tests._parity import compare_fields
from tests._translation import drop_shape, min_image

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def felbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_01906_amd import felbm as F
    F.load_library()
    return F


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_translation_prefix_vs_oracle(felbm, oracle_mod, precision, tol):
    w = translate2d(64)
    inst = w.instances[0]
    ctx = felbm.from_workload(w, precision=precision)
    ctx.step(40)
    ctx.sync()
    o = oracle_mod.Oracle(inst.mesh, 9, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    o.step(40)
    e = compare_fields(ctx.read_fields(0), o.fields(), inst)
    print("translation prefix", precision, e, flush=True)
    for k in ("rho", "u", "C"):
        assert e[k] < tol, (k, e[k])


def test_translation_round_trip(felbm):
    """128 x 128, density ratio 100, u0 = 0.02 along x: 32,000 steps (one
    box length), FP32, consistent mass by CG."""
    w = translate2d()
    inst = w.instances[0]
    m = inst.mesh
    ctx = felbm.from_workload(w, precision="fp32")
    c0, e0 = drop_shape(m["xyz"], m["box"], ctx.read_fields(0)["C"])
    s0 = ctx.conserved_sums(0)
    ctx.step(w.steps)
    ctx.sync()
    f = ctx.read_fields(0)
    c, ecc = drop_shape(m["xyz"], m["box"], f["C"])
    s = ctx.conserved_sums(0)
    err = float(np.linalg.norm(min_image(c - c0, m["box"])))
    print("round trip: centre error", err, "eccentricity", e0, "->", ecc, "mass drift", s[0] / s0[0] - 1,
          "momentum", s0[3:5], "->", s[3:5], "rho min", f["rho"].min(), flush=True)
    assert np.isfinite(f["rho"]).all() and f["rho"].min() > 0
    assert err < 0.5                       # lattice units, radius 32 (measured 0.22)
    assert ecc < 0.12                      # from 0.022 (sampling of the circle), measured 0.073
    # FP32 state: exact conservation holds to rounding per step (pinned in
    # FP64); over 32,000 steps it accumulates to ~1e-5 (mass) and ~6e-4
    # (momentum along the stream)
    assert abs(s[0] / s0[0] - 1.0) < 3e-5
    assert abs(s[1] / s0[1] - 1.0) < 3e-4  # heavy-phase volume
    np.testing.assert_allclose(s[3], s0[3], rtol=3e-3)
    assert abs(s[4]) < 1e-4 * abs(s0[3])


def test_translation_diagonal_prefix_vs_oracle(felbm, oracle_mod):
    """The drop carried along the box diagonal: 40 steps against the oracle
    (FP64 within 1e-11, FP32 within 2e-5)."""
    w = translate2d(64, diagonal=True)
    inst = w.instances[0]
    o = oracle_mod.Oracle(inst.mesh, 9, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    o.step(40)
    for precision, tol in (("fp64", 1e-11), ("fp32", 2e-5)):
        ctx = felbm.from_workload(w, precision=precision)
        ctx.step(40)
        ctx.sync()
        e = compare_fields(ctx.read_fields(0), o.fields(), inst)
        print("diagonal translation prefix", precision, e, flush=True)
        for k in ("rho", "u", "C"):
            assert e[k] < tol, (precision, k, e[k])


def test_translation_diagonal_round_trip(felbm):
    """The droplet translation of Section 3.2 along the diagonal: 128 x 128,
    density ratio 100, |u0| = 0.02 at 45 degrees, one round trip of
    sqrt(2) 128 / 0.02 time units (45,255 steps: one box length along each
    axis), FP32, consistent mass by CG.  The drop must come back where it
    started and stay round, with the bounds of the axis-aligned trip; mass
    and both momentum components are kept.  The paper reports eccentricity
    errors of 0.0036 and 0.0030 after four trips on its two finer 3-D
    meshes (context only: other meshes, dimension and contrasts)."""
    w = translate2d(diagonal=True)
    inst = w.instances[0]
    m = inst.mesh
    ctx = felbm.from_workload(w, precision="fp32")
    c0, e0 = drop_shape(m["xyz"], m["box"], ctx.read_fields(0)["C"])
    s0 = ctx.conserved_sums(0)
    ctx.step(w.steps)
    ctx.sync()
    f = ctx.read_fields(0)
    c, ecc = drop_shape(m["xyz"], m["box"], f["C"])
    s = ctx.conserved_sums(0)
    err = float(np.linalg.norm(min_image(c - c0, m["box"])))
    print("diagonal round trip:", w.steps, "steps, centre error", err, "eccentricity", e0, "->", ecc,
          "(paper, 3-D, four trips: 0.0036 / 0.0030)", "mass drift", s[0] / s0[0] - 1, "momentum", s0[3:5],
          "->", s[3:5], "rho min", f["rho"].min(), flush=True)
    assert np.isfinite(f["rho"]).all() and f["rho"].min() > 0
    assert err < 0.5
    assert ecc < 0.12
    # FP32 conservation drifts by rounding step after step: the axis-aligned
    # trip's bounds per step (3e-5 and 3e-4 over its 32,000 steps)
    assert abs(s[0] / s0[0] - 1.0) < 3e-5 / 32000 * w.steps
    assert abs(s[1] / s0[1] - 1.0) < 3e-4 / 32000 * w.steps
    np.testing.assert_allclose(s[3:5], s0[3:5], rtol=3e-3)
