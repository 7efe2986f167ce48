"""Forward model of the DMD-coded acquisition and its adjoint (oracle).

Sec. III-A and eq. (model-slice): shot j records b_j = sum_{r=1..R} phi_r (.) v_{(j-1)R+r},
where phi_r is the r-th binary mask (a diagonal matrix, shared by all shots)
and (.) the Hadamard product.  The adjoint, which appears as Phi^T b in the
v-update (eq. (v-update)), places phi_r (.) b_j into slice (j-1)R+r.
"""
import numpy as np


def _dtype(*arrays):
    return np.result_type(np.float64, *[a.dtype for a in arrays])


def forward(x, masks):
    """b[j] = sum_r masks[r] * x[j*R + r];  x: [N*R][H][W], masks: [R][H][W] -> b: [N][H][W]."""
    x = np.asarray(x)
    m = np.asarray(masks).astype(np.float64)
    R = m.shape[0]
    NR, H, W = x.shape
    if NR % R:
        raise ValueError("slice count must be a multiple of R")
    N = NR // R
    b = np.zeros((N, H, W), dtype=_dtype(x))
    for j in range(N):
        for r in range(R):
            b[j] += m[r] * x[j * R + r]
    return b


def adjoint(b, masks):
    """x[j*R + r] = masks[r] * b[j];  b: [N][H][W] -> x: [N*R][H][W]."""
    b = np.asarray(b)
    m = np.asarray(masks).astype(np.float64)
    R = m.shape[0]
    N, H, W = b.shape
    x = np.zeros((N * R, H, W), dtype=_dtype(b))
    for j in range(N):
        for r in range(R):
            x[j * R + r] = m[r] * b[j]
    return x
