"""Float64 CPU oracle for the EMD lower bounds (RWMD, OMR, ACT, ICT, EMD).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library or its binding.
"""
from .emd_oracle import (  # noqa: F401
    METHODS,
    DIRECTIONS,
    Oracle,
    act,
    act_rows,
    cost_matrix,
    emd_lp,
    ict,
    measure,
    omr,
    relaxed_lp,
    rwmd,
    squared_distances,
)
