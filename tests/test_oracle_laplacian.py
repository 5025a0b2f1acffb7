"""Pins of the oracle's weak-form Laplacian (the FEL_LAP_WEAK reading of
Section 2.3, which recovers derivatives but never defines the Laplacian of
the density): lap phi = -m^-1 (sum_r K_rr) phi, with K_rr the second-order
finite-element matrices of Section 2.2.1 and m the lumped mass.

Each pin fixes it by something other than the oracle's own element loop:
  * dense brute-force assembly (Vandermonde shape functions, quadrature
    lumped mass) on the five small meshes of the operator pins;
  * the closed form on unjittered grids: the P1 stiffness of the
    (0,0)-(1,1) triangle split is the 5-point stencil and that of the Kuhn
    6-tet split the 7-point stencil, with lumped mass h^d, so a Fourier mode
    cos(k.x) is an eigenvector with eigenvalue sum_r 2 (cos(k_r h) - 1) / h^2
    (spacing h = 0.5, so a dropped 1/m is off by a factor 4);
  * the energy identity sum_i m_i phi_i lap_i = -int |grad phi_h|^2 on a
    jittered periodic mesh, which tends to -(2 pi / L)^2 L^2 / 2 for
    phi = cos(2 pi x / L) at second order under refinement;
  * constants have zero Laplacian.
A sign flip, a dropped or squared 1/m, or a missing K_rr term fails at
least one of them.
"""
import numpy as np
import pytest

from paper_1608_01906_amd.inputs import grid_mesh_2d, grid_mesh_3d
from tests._bruteforce import dense_operators
from tests.test_oracle_operators import PHYS, _meshes


def _scaled(mesh, h):
    m = dict(mesh)
    m["xyz"] = mesh["xyz"] * h
    m["box"] = mesh["box"] * h
    return m


@pytest.mark.parametrize("name,mesh,Q", _meshes(), ids=[m[0] for m in _meshes()])
def test_weak_laplacian_matches_dense_assembly(oracle_mod, name, mesh, Q):
    o = oracle_mod.Oracle(mesh, Q, PHYS)
    M, G, K = dense_operators(mesh)
    dim = mesh["dim"]
    m = M.sum(axis=1)
    Ksum = sum(K[r, r] for r in range(dim))
    rng = np.random.default_rng(7)
    N = mesh["xyz"].shape[0]
    for _ in range(3):
        phi = rng.standard_normal(N)
        want = -(Ksum @ phi) / m
        got = o.weak_laplacian(phi)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max(), name


@pytest.mark.parametrize("dim", [2, 3])
def test_weak_laplacian_fourier_mode_closed_form(oracle_mod, dim):
    h = 0.5
    if dim == 2:
        n = (12, 10)
        mesh = _scaled(grid_mesh_2d(*n, jitter=0.0), h)
        Q = 9
    else:
        n = (6, 5, 4)
        mesh = _scaled(grid_mesh_3d(*n, jitter=0.0), h)
        Q = 19
    o = oracle_mod.Oracle(mesh, Q, PHYS)
    x = mesh["xyz"]
    # one mode per axis combination, wave numbers fitting the periods
    for modes in ([1] + [0] * (dim - 1), [2, 1] + [1] * (dim - 2), [3] + [2] * (dim - 1)):
        k = np.array([2 * np.pi * modes[r] / (n[r] * h) for r in range(dim)])
        phi = np.cos(x @ k)
        lam = sum(2.0 * (np.cos(k[r] * h) - 1.0) / h ** 2 for r in range(dim))
        got = o.weak_laplacian(phi)
        assert np.abs(got - lam * phi).max() <= 1e-12 * abs(lam), (modes, lam)


def test_weak_laplacian_energy_converges_on_jittered_mesh(oracle_mod):
    errs = []
    for n in (16, 32, 64):
        mesh = grid_mesh_2d(n, n, jitter=0.2, seed=21)
        o = oracle_mod.Oracle(mesh, 9, PHYS)
        m = o.lumped_mass()
        phi = np.cos(2 * np.pi * mesh["xyz"][:, 0] / n)
        energy = -(m * phi * o.weak_laplacian(phi)).sum()
        exact = (2 * np.pi / n) ** 2 * n * n / 2.0
        errs.append(abs(energy / exact - 1.0))
    assert errs[-1] < 2e-3, errs
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


@pytest.mark.parametrize("name,mesh,Q", _meshes()[:3], ids=[m[0] for m in _meshes()[:3]])
def test_weak_laplacian_of_constant_vanishes(oracle_mod, name, mesh, Q):
    o = oracle_mod.Oracle(mesh, Q, PHYS)
    got = o.weak_laplacian(np.full(mesh["xyz"].shape[0], 3.5))
    assert np.abs(got).max() < 1e-13, name
