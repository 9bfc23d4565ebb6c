"""FP64 CPU oracle for the FAS multigrid with Hybrid Smoother 2.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports,
links or executes anything from this package, and this package imports
nothing from the product package.
"""
from .core import (Oracle, OracleParams, box_dense, box_tridiag, build_oracle, hull, line_units, prolong,  # noqa: F401
                   restrict, setup_maps, tridiag_solve, visit_order)
