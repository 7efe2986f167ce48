"""z-direction Laplacian of the temporal-smoothness term (oracle).

Sec. III-C adds (gamma/2) sum_n ||v_n - v_{n-1}||^2 with a periodic wrap
(u_0 = u_{NR}, u_{NR+1} = u_1).  Written as (gamma/2) v^T L v per pixel:

* periodic: every adjacent pair, including the wrap pair (NR, 1), counted once,
  L = 2I - S - S^T with S the cyclic shift (so NR = 2 weights its single pair
  twice and NR = 1 gives L = 0);
* neumann (free ends, an option): L = D^T D with D the (n-1) x n forward difference.
"""
import numpy as np


def zlaplacian(n, zbc="periodic"):
    if n < 1:
        raise ValueError("n must be >= 1")
    if zbc == "periodic":
        S = np.roll(np.eye(n), 1, axis=1)
        return 2.0 * np.eye(n) - S - S.T
    if zbc == "neumann":
        D = np.zeros((n - 1, n))
        for i in range(n - 1):
            D[i, i] = -1.0
            D[i, i + 1] = 1.0
        return D.T @ D
    raise ValueError(f"unknown z boundary {zbc!r}")


def temporal_energy(v, zbc="periodic"):
    """(1/2) sum over adjacent z-pairs of ||v_n - v_{n-1}||^2, pairs as in :func:`zlaplacian`."""
    v = np.asarray(v)
    n = v.shape[0]
    if zbc == "periodic":
        if n == 1:
            return 0.0
        diffs = [v[i] - v[i - 1] for i in range(1, n)] + [v[0] - v[n - 1]]
    else:
        diffs = [v[i] - v[i - 1] for i in range(1, n)]
    return 0.5 * sum(np.sum(dd * dd) for dd in diffs)
