"""The v-sub-problem (x-step) of the ADMM, solved by its plain definition (oracle).

With the 1/2-scaled data term (the scale under which eq. (v-update) is exact)
and the temporal term carried by the v-block, the x-step minimises

    1/2 ||b - Phi x||^2 + (gamma/2) x^T (L (x) I) x + (rho/2) ||x - (u - d)||^2

(Sec. III-B eq. (v-sub-1) and eq. (v-update); temporal term Sec. III-C).  Its
normal equations decouple over pixels p:

    (M_p^T M_p + gamma L + rho I) x_p = M_p^T b_p + rho (u_p - d_p),

where M_p (N x NR) holds the pixel's mask bits m_p in row j, columns
(j-1)R+1..jR.  This module forms every pixel's NR x NR matrix densely and
calls a dense LU solve; it deliberately does not use the Woodbury/Thomas
structure.  gamma = 0 gives the paper's eq. (v-update) exactly.
"""
import numpy as np

from .laplacian import zlaplacian


def pixel_systems(masks, N, rho, gamma, zbc="periodic"):
    """Dense per-pixel matrices A_p, shape [H*W][NR][NR] (float64 or complex)."""
    m = np.asarray(masks).astype(np.float64)
    R, H, W = m.shape
    NR = N * R
    P = H * W
    mp = m.reshape(R, P).T  # [P][R]
    dt = np.result_type(np.float64, type(rho), type(gamma))
    A = np.zeros((P, NR, NR), dtype=dt)
    for j in range(N):
        blk = slice(j * R, (j + 1) * R)
        A[:, blk, blk] += mp[:, :, None] * mp[:, None, :]
    A += gamma * zlaplacian(NR, zbc)[None, :, :]
    A += rho * np.eye(NR)[None, :, :]
    return A


def xstep(b, u, d, masks, rho, gamma, zbc="periodic", chunk=16384):
    """x = argmin of the x-step objective; b: [N][H][W], u, d: [N*R][H][W] -> x: [N*R][H][W]."""
    b = np.asarray(b)
    u = np.asarray(u)
    d = np.asarray(d)
    m = np.asarray(masks).astype(np.float64)
    R, H, W = m.shape
    N = b.shape[0]
    NR = N * R
    P = H * W
    dt = np.result_type(np.float64, b.dtype, u.dtype, d.dtype, type(rho), type(gamma))
    mp = m.reshape(R, P).T  # [P][R]
    bp = b.reshape(N, P).T  # [P][N]
    g = (u.reshape(NR, P) - d.reshape(NR, P)).T  # [P][NR]
    rhs = rho * g.astype(dt)
    for j in range(N):
        rhs[:, j * R:(j + 1) * R] += mp * bp[:, j:j + 1]
    L = zlaplacian(NR, zbc)
    x = np.empty((P, NR), dtype=dt)
    for s in range(0, P, chunk):
        e = min(P, s + chunk)
        A = np.zeros((e - s, NR, NR), dtype=dt)
        for j in range(N):
            blk = slice(j * R, (j + 1) * R)
            A[:, blk, blk] += mp[s:e, :, None] * mp[s:e, None, :]
        A += gamma * L[None]
        A += rho * np.eye(NR)[None]
        x[s:e] = np.linalg.solve(A, rhs[s:e, :, None])[:, :, 0]
    return x.T.reshape(NR, H, W)
