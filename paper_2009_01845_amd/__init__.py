"""MI355X (gfx950) dense state-vector simulator: the hot path of Qibo
(arXiv:2009.01845) as hand-written HIP kernels behind a C ABI (include/qsim.h).

The Python layer marshals arguments only; libqsim.so must be built
(``python -m paper_2009_01845_amd.build``) -- there is no CPU fallback.
"""
from ._lib import QS_C64, QS_C128, QsError, LIB_PATH  # noqa: F401
from .api import (Circuit, DensityCircuit, DensityMatrix, Observable, State, adiabatic_run, adjoint,  # noqa: F401
                  apply, expectation,
                  gate_matrix, norm2, sample)
