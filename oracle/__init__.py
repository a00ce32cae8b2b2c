"""FP64 CPU oracle for TC2 purification and its first-order response.

Test infrastructure only: the GPU library never imports, links or runs
anything under this package.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark use it.
"""
from .tc2_oracle import (  # noqa: F401
    bsr_to_dense, gershgorin, tc2_init, block_drop, tc2_step, tc2_solve,
    band_energies, OracleResult, SQUARE, DOUBLE,
)
from .exact import exact_projector, exact_response, exact_alpha  # noqa: F401
