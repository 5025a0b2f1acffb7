"""Dense brute-force P1 assembly by numerical quadrature (NumPy, tiny meshes).

Independent of the oracle's element formulas: the shape functions come from
solving the Vandermonde system of each element (N_a = c0 + c . x with
N_a(x_b) = delta_ab), volumes from a determinant, and the integrals of
Section 2.2.1 (mass, advection, second-order matrices) from quadrature rules
exact for the integrands (degree 2 for N N^T, degree 1 for N dN^T).
"""
from __future__ import annotations

import numpy as np

# degree-2 exact rules on the reference simplex, barycentric points + weights (sum 1)
_TRI_PTS = np.array([[0.5, 0.5, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5]])
_TRI_W = np.full(3, 1.0 / 3.0)
_a, _b = 0.5854101966249685, 0.1381966011250105
_TET_PTS = np.array([[_a, _b, _b, _b], [_b, _a, _b, _b], [_b, _b, _a, _b], [_b, _b, _b, _a]])
_TET_W = np.full(4, 0.25)


def unwrap(mesh, e):
    dim = mesh["dim"]
    c = mesh["conn"][e]
    return mesh["xyz"][c] + mesh["shift"][e].astype(float) * mesh["box"][None, :dim]


def dense_operators(mesh):
    """Returns M, G[r], K[s][r] as dense (N, N) arrays."""
    dim = mesh["dim"]
    N = mesh["xyz"].shape[0]
    nv = dim + 1
    M = np.zeros((N, N))
    G = np.zeros((dim, N, N))
    K = np.zeros((dim, dim, N, N))
    pts, wts = (_TRI_PTS, _TRI_W) if dim == 2 else (_TET_PTS, _TET_W)
    fact = 2.0 if dim == 2 else 6.0
    for e in range(mesh["conn"].shape[0]):
        X = unwrap(mesh, e)
        V = np.hstack([np.ones((nv, 1)), X])            # rows [1, x, y(, z)]
        coef = np.linalg.solve(V, np.eye(nv))           # column a: coefficients of N_a
        vol = abs(np.linalg.det(V)) / fact
        grads = coef[1:, :].T                           # [a, r]
        c = mesh["conn"][e]
        for q, wq in zip(pts, wts):
            xq = q @ X
            Nq = np.concatenate([[1.0], xq]) @ coef      # N_a at the point
            M[np.ix_(c, c)] += vol * wq * np.outer(Nq, Nq)
            for r in range(dim):
                G[r][np.ix_(c, c)] += vol * wq * np.outer(Nq, grads[:, r])
        for s in range(dim):
            for r in range(dim):
                K[s, r][np.ix_(c, c)] += vol * np.outer(grads[:, s], grads[:, r])
    return M, G, K


def stream_matrix(G, K, c, dt):
    """dt C_alpha + dt^2 D_alpha for lattice velocity c."""
    dim = G.shape[0]
    A = sum(dt * c[r] * G[r] for r in range(dim))
    for s in range(dim):
        for r in range(dim):
            A = A + 0.5 * dt * dt * c[s] * c[r] * K[s, r]
    return A
