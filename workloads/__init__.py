"""Seeded synthetic inputs for the stencil sweep.

This package only draws and lays out inputs (fields, coefficients) and names the
workloads; it holds none of the sweep's arithmetic.  The tests, the benchmark,
the smoke check and the oracle all take their inputs from here, so the GPU path
and the oracle see identical bytes.
"""
from .grids import (WORKLOADS, Workload, field_and_coefs, padded_shape, to_padded,
                    from_padded, RADIUS, N_COEF_ARRAYS, N_CONST_COEFS, STENCILS)

__all__ = ["WORKLOADS", "Workload", "field_and_coefs", "padded_shape", "to_padded",
           "from_padded", "RADIUS", "N_COEF_ARRAYS", "N_CONST_COEFS", "STENCILS"]
