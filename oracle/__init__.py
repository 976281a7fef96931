"""CPU oracle for block principal pivoting NNLS.  TEST INFRASTRUCTURE ONLY: imported by
the test suite, the package smoke check and the benchmark's CPU-baseline leg, never by
the GPU library."""
from .nnls_oracle import (TAU, P_MAX, BRANCH_BLOCK_IMPROVED, BRANCH_BLOCK_BUDGET,  # noqa: F401
                          BRANCH_SINGLE, Result, TraceRow, bpp_solve, classify, dual,
                          exchange_rule, gram, inverse_onenorm_estimate, kkt_residuals,
                          predicted_rel_error, principal_block, solve_free)
