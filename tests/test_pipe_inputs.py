"""Concurrent pipe flow (Section 3.3): the curved-wall pipe mesh, the
steady profile the pipe workloads start from, the relative-permeability
closed forms, and the oracle on a curved wall.

Pins:
  * mesh: positive tetrahedra, every face shared by two of them except the
    wall faces, whose vertices are all wall nodes, inward unit normals, and
    the volume of the inscribed polygon times the length;
  * the diffuse-interface profile tends to the two-parabola profile of
    Section 3.3 as the interface narrows and the densities meet;
  * integrating that two-parabola profile over each phase gives
    k_rw = S_w^2 and k_rnw = (1 - S_w)^2 + 2 M S_w (1 - S_w) (the reading of
    the printed non-wetting formula, which does not return 1 at S_w = 0);
  * the oracle keeps single-phase Poiseuille flow in the pipe: no
    transverse flow beyond rounding, the axial profile within the
    discretisation error of the polygonal wall, mass up to the bounce-back.
"""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs.mesh import pipe_mesh_3d
from paper_1608_01906_amd.inputs.workloads import CS2, pipe_instance, pipe_profile


def _faces(conn):
    f = np.concatenate([np.sort(conn[:, [i for i in range(4) if i != skip]], axis=1) for skip in range(4)])
    uniq, cnt = np.unique(f, axis=0, return_counts=True)
    return uniq, cnt


@pytest.mark.parametrize("radius,nz", [(6.0, 4), (12.0, 3)])
def test_pipe_mesh_is_a_valid_tet_mesh_with_curved_wall(radius, nz):
    m = pipe_mesh_3d(radius, nz)
    xyz, conn, sh, box = m["xyz"], m["conn"], m["shift"], m["box"]
    v = xyz[conn] + sh * box
    vol = np.linalg.det(v[:, 1:, :] - v[:, :1, :]) / 6.0
    assert vol.min() > 0.05
    uniq, cnt = _faces(conn)
    assert set(cnt.tolist()) == {1, 2}
    wall = m["wall"].astype(bool)
    assert wall[uniq[cnt == 1]].all()                  # open faces lie on the wall
    # wall: the outer ring, at the radius, inward unit normals in the cross-section
    r = np.hypot(xyz[:, 0] - radius, xyz[:, 1] - radius)
    np.testing.assert_allclose(r[wall], radius, rtol=1e-12)
    assert r[~wall].max() < radius - 0.5
    n = m["wall_normal"][wall]
    np.testing.assert_allclose(np.linalg.norm(n, axis=1), 1.0, rtol=1e-12)
    assert np.all(n[:, 2] == 0.0)
    outward = np.stack([xyz[wall, 0] - radius, xyz[wall, 1] - radius], axis=1) / radius
    np.testing.assert_allclose((n[:, :2] * outward).sum(axis=1), -1.0, rtol=1e-12)
    # volume = inscribed polygon (the wall ring in angular order) x length
    ring = xyz[wall & (xyz[:, 2] == 0.0)]
    ang = np.arctan2(ring[:, 1] - radius, ring[:, 0] - radius)
    ring = ring[np.argsort(ang)]
    x, y = ring[:, 0], ring[:, 1]
    area = 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))
    np.testing.assert_allclose(vol.sum(), area * nz, rtol=1e-12)
    # the 3-D ELL layout takes up to 24 entries per row (diagonal included)
    valence = np.zeros(xyz.shape[0], int)
    edges = np.unique(np.sort(np.concatenate([conn[:, [a, b]] for a in range(4) for b in range(a + 1, 4)]), axis=1),
                      axis=0)
    np.add.at(valence, edges.ravel(), 1)
    assert valence.max() + 1 <= 24


def _two_parabolas(r, R, a, g, mu_w, mu_nw):
    """The steady profile of Section 3.3 (sharp interface at a, equal densities)."""
    return np.where(r > a, g / (4 * mu_w) * (R ** 2 - r ** 2),
                    g / (4 * mu_w) * (R ** 2 - a ** 2) + g / (4 * mu_nw) * (a ** 2 - r ** 2))


@pytest.mark.parametrize("M", [0.2, 1.0, 5.0])
def test_diffuse_profile_tends_to_the_two_parabolas(M):
    R, s_w, g, dt, tau_w, rho = 10.0, 0.5, 1e-5, 0.05, 1.0, 1.0
    a = R * np.sqrt(1 - s_w)
    tau_nw = tau_w * M
    r = np.linspace(0.0, R, 401)
    want = _two_parabolas(r, R, a, rho * g, rho * CS2 * tau_w * dt, rho * CS2 * tau_nw * dt)
    errs = []
    for xi in (0.4, 0.1, 0.025):
        got = pipe_profile(r, radius=R, a=a, rho_w=rho, rho_nw=rho * (1 - 1e-9), tau_w=tau_w, tau_nw=tau_nw,
                           xi=xi, g=g, dt=dt, sub=4000)
        errs.append(np.abs(got - want).max() / want.max())
    assert errs[-1] < 2e-3, errs
    if M != 1.0:  # equal viscosities: no interface effect to shrink
        assert errs[0] > errs[1] > errs[2], errs


@pytest.mark.parametrize("M", [0.2, 1.0, 5.0])
@pytest.mark.parametrize("s_w", [0.1, 0.25, 0.5, 0.75, 0.9])
def test_relative_permeability_closed_forms(M, s_w):
    R, g, mu_w = 1.0, 1.0, 1.0
    mu_nw = M * mu_w
    a = R * np.sqrt(1 - s_w)
    r = np.linspace(0.0, R, 400001)
    u = _two_parabolas(r, R, a, g, mu_w, mu_nw)
    dA = 2 * np.pi * r
    q_w = np.trapezoid(np.where(r > a, u, 0.0) * dA, r)
    q_nw = np.trapezoid(np.where(r <= a, u, 0.0) * dA, r)
    k_rw = q_w / (np.pi * g * R ** 4 / (8 * mu_w))
    k_rnw = q_nw / (np.pi * g * R ** 4 / (8 * mu_nw))
    assert k_rw == pytest.approx(s_w ** 2, rel=2e-4, abs=1e-6)
    assert k_rnw == pytest.approx((1 - s_w) ** 2 + 2 * M * s_w * (1 - s_w), rel=2e-4)


def test_oracle_keeps_single_phase_pipe_flow(oracle_mod):
    """200 oracle steps of Poiseuille flow through the 6-radius pipe: mass
    moves only through the nodal bounce-back at the wall (which replaces
    populations rather than exchanging them: 3e-9 over these steps), no
    transverse flow appears, and the axial profile
    stays within 3 % of the analytic one (it relaxes towards the steady
    state of the discrete wall over a viscous time, ~190 time units here,
    of which these steps are 10)."""
    m = pipe_mesh_3d(6.0, 4)
    inst = pipe_instance(m, radius=6.0, s_w=1.0, visc_ratio=1.0, phase="w", tau_w=2.0)
    o = oracle_mod.Oracle(inst.mesh, 19, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    s0 = o.conserved()
    o.step(200)
    s1 = o.conserved()
    f = o.fields()
    uz0 = inst.u0[:, 2]
    assert abs(s1[0] / s0[0] - 1.0) < 1e-7
    assert np.abs(f["u"][:, :2]).max() < 1e-4 * uz0.max()
    assert np.abs(f["u"][:, 2] - uz0).max() < 0.03 * uz0.max()
