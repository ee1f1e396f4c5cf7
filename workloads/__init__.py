"""Seeded synthetic inputs for the PB-SpGEMM hot path.

This package is shared by the tests, the benchmark and the CPU oracle's
callers.  It holds matrix generators and format plumbing only: none of the
product's arithmetic (no multiply, merge or reduction of C = A*B) lives here.
"""
from .gen import (  # noqa: F401
    batched_er_sizes,
    Csx,
    amg_problem,
    batched_er_problems,
    csc_to_csr,
    csr_to_csc,
    er_csc,
    er_problem,
    identity,
    random_sparse,
    rmat_symmetric,
)
