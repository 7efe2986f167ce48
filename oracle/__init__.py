"""FP64 CPU oracle for the PnP-ADMM compressive light-sheet reconstruction.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
leg of the benchmark import this package; the library and its Python binding
never do, and this package imports nothing from them.

Every routine is a plain NumPy transcription of a definition in the paper
(arXiv 2511.03093) or of a cited textbook algorithm, in float64, with no
blocking, fusion or reordering beyond what the definition states.  Routines
are also written so that complex inputs work (complex-step derivatives).

Parity status: every function here is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, brute force, optimality
conditions or an independent derivative; none is "parity unpinned" except the
end-to-end reconstruction quality, which the paper reports on a dataset that
is not available.
"""
from .operator import forward, adjoint
from .laplacian import zlaplacian
from .xstep import xstep, pixel_systems
from .tv import grad2d, div2d, tv_chambolle, tv_value
from .denoise import tikhonov, tv_prox, denoise
from .admm import Params, iterate, solve, iterate_paper, solve_paper, objective

__all__ = [
    "forward", "adjoint", "zlaplacian", "xstep", "pixel_systems", "grad2d", "div2d",
    "tv_chambolle", "tv_value", "tikhonov", "tv_prox", "denoise", "Params", "iterate",
    "solve", "iterate_paper", "solve_paper", "objective",
]
