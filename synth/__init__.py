"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This package only draws random histograms and embeddings; it contains none
of the distance arithmetic of the method.
"""
from .generators import (  # noqa: F401
    CSR,
    Workload,
    make_workload,
    WORKLOADS,
    arrival_trace,
    zipf_histograms,
    blob_histograms,
    gaussian_embeddings,
    grid_embeddings,
)
