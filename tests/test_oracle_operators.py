"""Pins of the oracle's finite-element operators (Sections 2.2.1 and 2.3).

Each test checks the oracle against something other than itself: dense
quadrature assembly, textbook element matrices, linear-field patch tests,
the a-priori spectrum of the lumped-preconditioned mass matrix, a dense
direct solve.
"""
import os

import numpy as np
import pytest

from paper_1608_01906_amd.inputs import grid_mesh_2d, grid_mesh_3d
from paper_1608_01906_amd.inputs.mesh import delaunay_mesh
from tests._bruteforce import dense_operators, stream_matrix

D2Q9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
D3Q19_AXES = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, -1, 0], [1, 0, 1],
                       [0, 1, -1]], float)
PHYS = (1.0, 0.1, 0.05, 0.05, 0.01, 4.0, 0.25, 0.0, 0.0, 0.0)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _meshes():
    return [("periodic2d", grid_mesh_2d(6, 5, seed=11), 9),
            ("walled2d", grid_mesh_2d(5, 6, wall_y=True, seed=12), 9),
            ("periodic3d", grid_mesh_3d(3, 3, 4, seed=13), 19),
            # unstructured (Delaunay) periodic meshes: irregular valence
            ("delaunay2d", delaunay_mesh((6, 5), seed=14), 9),
            ("delaunay3d", delaunay_mesh((4, 3, 4), seed=15), 19)]


@pytest.fixture(scope="module", params=_meshes(), ids=lambda m: m[0])
def case(request, oracle_mod):
    name, mesh, Q = request.param
    o = oracle_mod.Oracle(mesh, Q, PHYS)
    M, G, K = dense_operators(mesh)
    return dict(name=name, mesh=mesh, o=o, M=M, G=G, K=K, N=mesh["xyz"].shape[0])


def _columns(fn, N):
    return np.stack([fn(np.eye(N)[j]) for j in range(N)], axis=1)


def test_golden_reference_element_mass():
    """Textbook P1 mass matrices: (|T| / 12)(1 + delta) for a triangle, (|T| / 20)(1 + delta) for a tet."""
    data = {}
    with open(os.path.join(GOLDEN, "p1_reference_mass.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                key, vals = line.split(":")
                data[key.strip()] = np.array([float(v) for v in vals.split()])
    tri = dict(dim=2, xyz=np.array([[0., 0.], [1., 0.], [0., 1.]]), conn=np.array([[0, 1, 2]], np.int32),
               shift=np.zeros((1, 3, 2), np.int8), box=np.zeros(2), wall=np.zeros(3, np.uint8),
               wall_normal=np.zeros((3, 2)))
    tet = dict(dim=3, xyz=np.array([[0., 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]),
               conn=np.array([[0, 1, 2, 3]], np.int32), shift=np.zeros((1, 4, 3), np.int8),
               box=np.zeros(3), wall=np.zeros(4, np.uint8), wall_normal=np.zeros((4, 3)))
    from oracle import oracle as O
    for mesh, Q, key in [(tri, 9, "triangle"), (tet, 19, "tetrahedron")]:
        o = O.Oracle(mesh, Q, PHYS)
        n = mesh["xyz"].shape[0]
        Mo = _columns(o.apply_M, n)
        np.testing.assert_allclose(Mo.ravel(), data[key], rtol=0, atol=1e-15)


def test_mass_matches_quadrature(case):
    Mo = _columns(case["o"].apply_M, case["N"])
    np.testing.assert_allclose(Mo, case["M"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(case["o"].lumped_mass(), case["M"].sum(axis=1), rtol=1e-14)


def test_stream_operator_matches_quadrature(case):
    o, N = case["o"], case["N"]
    dim = case["mesh"]["dim"]
    dirs = D2Q9[1:] if dim == 2 else D3Q19_AXES
    Q = 9 if dim == 2 else 19
    # map each direction to the oracle's index by matching velocity vectors
    lat = _lattice(Q)
    for c in dirs:
        alpha = int(np.where((lat == c).all(axis=1))[0][0])
        Ao = _columns(lambda x: o.apply_A(alpha, x), N)
        Ab = stream_matrix(case["G"], case["K"], c, 0.25)
        np.testing.assert_allclose(Ao, Ab, rtol=0, atol=1e-14)


def _lattice(Q):
    if Q == 9:
        return D2Q9
    ax = [[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
          [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1], [1, 0, -1],
          [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]]
    return np.array(ax, float)


def test_rest_direction_does_not_stream(case):
    x = np.random.default_rng(1).standard_normal(case["N"])
    assert np.abs(case["o"].apply_A(0, x)).max() == 0.0


def test_recovery_equals_lumped_inverse_times_advection(case):
    """Volume-weighted averaging of element gradients (Section 2.3) = m^-1 G."""
    rng = np.random.default_rng(2)
    phi = rng.standard_normal(case["N"])
    m = case["M"].sum(axis=1)
    ref = np.stack([case["G"][r] @ phi / m for r in range(case["mesh"]["dim"])], axis=1)
    np.testing.assert_allclose(case["o"].recover_grad(phi), ref, rtol=0, atol=1e-13)


def test_patch_constants(case):
    """Constants are not streamed: (C + D) 1 = 0 row-wise."""
    o, N = case["o"], case["N"]
    Q = 9 if case["mesh"]["dim"] == 2 else 19
    for alpha in range(1, Q):
        assert np.abs(o.apply_A(alpha, np.ones(N))).max() < 1e-14
    g = o.recover_grad(np.full(N, 3.0))
    assert np.abs(g).max() < 1e-13


def test_periodic_column_sums_vanish(case):
    """On a periodic mesh 1^T C_alpha = 1^T D_alpha = 0: streaming conserves sum m psi."""
    if case["name"] == "walled2d":
        pytest.skip("walled mesh has boundary terms")
    o, N = case["o"], case["N"]
    rng = np.random.default_rng(3)
    x = rng.standard_normal(N)
    Q = 9 if case["mesh"]["dim"] == 2 else 19
    for alpha in range(1, Q):
        assert abs(o.apply_A(alpha, x).sum()) < 1e-13 * np.abs(x).sum()


def test_linear_field_patch_walled():
    """On a mesh periodic in x and walled in y, phi = a y is linear in every element:
    the recovered gradient is (0, a) everywhere and, at interior nodes, the
    lumped streaming increment is exactly -dt c_y a."""
    from oracle import oracle as O
    mesh = grid_mesh_2d(8, 7, wall_y=True, seed=5)
    o = O.Oracle(mesh, 9, PHYS)
    a = 0.37
    phi = a * mesh["xyz"][:, 1]
    g = o.recover_grad(phi)
    np.testing.assert_allclose(g[:, 0], 0.0, atol=1e-13)
    np.testing.assert_allclose(g[:, 1], a, rtol=1e-13)
    m = o.lumped_mass()
    interior = mesh["wall"] == 0
    for alpha in range(1, 9):
        d = -o.apply_A(alpha, phi) / m
        np.testing.assert_allclose(d[interior], -0.25 * D2Q9[alpha, 1] * a, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_lumped_preconditioned_spectrum(dim, oracle_mod):
    """Eigenvalues of m^-1 M lie in [1/(d+2), 1] (element-wise bound for P1 simplices)."""
    mesh = grid_mesh_2d(8, 8, seed=21) if dim == 2 else grid_mesh_3d(4, 4, 4, seed=22)
    o = oracle_mod.Oracle(mesh, 9 if dim == 2 else 19, PHYS)
    N = mesh["xyz"].shape[0]
    M = _columns(o.apply_M, N)
    m = o.lumped_mass()
    ev = np.linalg.eigvals(M / m[:, None]).real
    assert ev.min() >= 1.0 / (dim + 2) - 1e-12
    assert ev.max() <= 1.0 + 1e-12


def test_mass_solve_matches_dense(case):
    o = case["o"]
    rng = np.random.default_rng(4)
    b = rng.standard_normal(case["N"])
    x, it, rel = o.solve_M(b)
    ref = np.linalg.solve(case["M"], b)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    assert rel < 1e-14


def test_streaming_stability_at_run_step(oracle_mod):
    """Spectral radius of the one-direction streaming map I - M^-1 A_alpha:
    <= 1 at the run step and > 1 at dt = 1 on a jittered periodic mesh."""
    mesh = grid_mesh_2d(10, 10, seed=31)
    N = mesh["xyz"].shape[0]
    M, G, K = dense_operators(mesh)
    from paper_1608_01906_amd.inputs import DT_RUN
    for dt, stable in [(DT_RUN, True), (1.0, False)]:
        worst = 0.0
        for c in D2Q9[1:]:
            T = np.eye(N) - np.linalg.solve(M, stream_matrix(G, K, c, dt))
            worst = max(worst, np.abs(np.linalg.eigvals(T)).max())
        assert (worst <= 1.0 + 1e-9) == stable, (dt, worst)
