"""Oracle for exact density-peaks clustering (test infrastructure only).

``dpc_oracle``: numpy, exact int64, O(n^2) (small inputs).
``scan``: the same plain method in C with OpenMP over query points (larger
inputs, and the benchmark's CPU baseline).  Neither imports the product package.
"""
