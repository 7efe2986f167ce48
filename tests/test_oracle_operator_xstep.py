"""Pins for the oracle's forward operator and x-step (CPU only).

The operator is checked by the adjoint identity and by an explicit sparse
matrix Phi built entry by entry; the x-step by the paper's Woodbury closed form
(end of Sec. III-B) at gamma = 0 and by a global dense solve of the
normal equations with Phi and L (x) I assembled explicitly.
"""
import numpy as np
import pytest

import oracle
from oracle.laplacian import zlaplacian, temporal_energy


def rng(*s):
    return np.random.default_rng([7, *s])


def explicit_phi(masks, N):
    """Phi as an (N*H*W) x (N*R*H*W) matrix, one entry per (shot, slice, pixel)."""
    R, H, W = masks.shape
    P = H * W
    Phi = np.zeros((N * P, N * R * P))
    for j in range(N):
        for r in range(R):
            for p in range(P):
                Phi[j * P + p, (j * R + r) * P + p] = masks[r].reshape(-1)[p]
    return Phi


def laplacian_chain(n, zbc):
    """Laplacian of the z-chain from the list of adjacent pairs (each pair once)."""
    pairs = [(i, i + 1) for i in range(n - 1)]
    if zbc == "periodic" and n >= 2:
        pairs.append((n - 1, 0))
    L = np.zeros((n, n))
    for a, b in pairs:
        e = np.zeros(n)
        e[a] += 1.0
        e[b] -= 1.0
        L += np.outer(e, e)
    return L


@pytest.mark.parametrize("N,R,H,W", [(1, 5, 3, 4), (2, 3, 2, 5), (1, 1, 4, 4), (3, 2, 3, 3)])
def test_forward_matches_explicit_matrix_and_adjoint(N, R, H, W):
    g = rng(N, R, H, W)
    masks = (g.random((R, H, W)) < 0.5).astype(np.uint8)
    x = g.normal(size=(N * R, H, W))
    b = g.normal(size=(N, H, W))
    Phi = explicit_phi(masks, N)
    np.testing.assert_allclose(oracle.forward(x, masks).reshape(-1), Phi @ x.reshape(-1), atol=1e-14)
    np.testing.assert_allclose(oracle.adjoint(b, masks).reshape(-1), Phi.T @ b.reshape(-1), atol=1e-14)
    lhs = np.vdot(oracle.forward(x, masks), b)
    rhs = np.vdot(x, oracle.adjoint(b, masks))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_forward_all_ones_masks_sums_slices():
    g = rng(1)
    x = g.normal(size=(6, 4, 5))
    masks = np.ones((6, 4, 5), np.uint8)
    np.testing.assert_allclose(oracle.forward(x, masks)[0], x.sum(axis=0), atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("zbc", ["periodic", "neumann"])
def test_laplacian_is_sum_over_pairs(n, zbc):
    np.testing.assert_allclose(zlaplacian(n, zbc), laplacian_chain(n, zbc), atol=0)
    v = rng(n).normal(size=(n, 2, 3))
    q = 0.5 * np.einsum("ipq,ij,jpq->", v, zlaplacian(n, zbc), v)
    assert abs(q - temporal_energy(v, zbc)) < 1e-12


def paper_woodbury_vupdate(b, u, d, masks, rho):
    """Final form of eq. (v-update) after Woodbury (Sec. III-B), N = 1:
    v = Phi^T b / (rho + Phi Phi^T) + g - Phi^T (Phi g / (rho + Phi Phi^T)), g = u - d."""
    m = masks.astype(np.float64)
    g = u - d
    c = m.sum(axis=0)  # Phi Phi^T is diagonal with entries sum_r phi_r
    phig = (m * g).sum(axis=0)
    return m * b[0] / (rho + c) + g - m * (phig / (rho + c))


@pytest.mark.parametrize("rho", [1.0, 0.0114, 1e-3, 7.5])
def test_xstep_gamma0_equals_paper_closed_form(rho):
    g = rng(2, int(rho * 1e4))
    R, H, W = 5, 3, 4
    masks = (g.random((R, H, W)) < 0.5).astype(np.uint8)
    masks[:, 0, 0] = 0  # a pixel no mask opens
    masks[:, 1, 1] = 1  # a pixel every mask opens
    b = g.normal(size=(1, H, W))
    u = g.normal(size=(R, H, W))
    d = g.normal(size=(R, H, W))
    x = oracle.xstep(b, u, d, masks, rho, 0.0)
    ref = paper_woodbury_vupdate(b, u, d, masks, rho)
    np.testing.assert_allclose(x, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("zbc", ["periodic", "neumann"])
@pytest.mark.parametrize("N,R,H,W", [(1, 5, 3, 4), (1, 2, 2, 3), (2, 3, 2, 2), (1, 1, 3, 3), (1, 8, 2, 2)])
@pytest.mark.parametrize("rho,gamma", [(1.0, 0.1), (0.01, 0.6), (2.0, 0.0)])
def test_xstep_matches_global_dense_solve(zbc, N, R, H, W, rho, gamma):
    g = rng(3, N, R, H, W, int(gamma * 10))
    masks = (g.random((R, H, W)) < 0.5).astype(np.uint8)
    masks[:, 0, 0] = 0
    b = g.normal(size=(N, H, W))
    u = g.normal(size=(N * R, H, W))
    d = g.normal(size=(N * R, H, W))
    NR, P = N * R, H * W
    Phi = explicit_phi(masks, N)
    A = Phi.T @ Phi + gamma * np.kron(laplacian_chain(NR, zbc), np.eye(P)) + rho * np.eye(NR * P)
    rhs = Phi.T @ b.reshape(-1) + rho * (u - d).reshape(-1)
    ref = np.linalg.solve(A, rhs).reshape(NR, H, W)
    x = oracle.xstep(b, u, d, masks, rho, gamma, zbc)
    np.testing.assert_allclose(x, ref, rtol=1e-11, atol=1e-12)


def test_xstep_is_stationary_point_of_its_objective():
    g = rng(4)
    R, H, W = 6, 3, 3
    masks = (g.random((R, H, W)) < 0.5).astype(np.uint8)
    b = g.normal(size=(1, H, W))
    u = g.normal(size=(R, H, W))
    d = g.normal(size=(R, H, W))
    rho, gamma = 0.7, 0.3

    def J(x):
        r = b - oracle.forward(x, masks)
        return 0.5 * np.sum(r * r) + gamma * temporal_energy(x) + 0.5 * rho * np.sum((x - (u - d)) ** 2)

    x = oracle.xstep(b, u, d, masks, rho, gamma)
    j0 = J(x)
    for k in range(20):
        e = g.normal(size=x.shape) * 1e-3
        assert J(x + e) > j0 - 1e-15
