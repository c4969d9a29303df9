"""Seeded synthetic inputs for the least-squares workloads.

This package draws problem data only (A, b, x_true, request streams).  It
holds none of the sketch-and-solve arithmetic and imports neither the oracle
nor the product library, so both sides can consume the same inputs.
"""
from .gen import (CONFIGS, Dense, Sparse, dense_ill_conditioned, dense_gaussian,  # noqa: F401
                  dense_scaled_columns, paper_benchmark, paper_benchmark_device, request_window,
                  serving_pool,
                  serving_requests, sparse_csr)
