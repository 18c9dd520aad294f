"""Plain FP64 CPU oracle for the density-matrix emulation -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library and does not
import it.

* :mod:`oracle.core`     -- ctypes front end of ``dm_oracle.c`` (row-major rho,
  ops applied one at a time as ``M rho M^dagger`` or ``sum_j K_j rho K_j^dagger``).
* :mod:`oracle.channels` -- the oracle's own builders of gate matrices and
  Kraus maps from ``(kind, params)``, written from the paper's definitions.
* :mod:`oracle.emulator` -- runs an op stream and computes the read-outs.
* :mod:`oracle.mlp`      -- FP64 reference of the surrogate network.
* :mod:`oracle.trajectories` -- Monte Carlo state-vector trajectories (one
  Kraus operator drawn per channel per sample), in numpy.

Parity status of each function is stated in its docstring; a function without
an independent pin says "parity unpinned".
"""
from .core import OracleDM  # noqa: F401
from .emulator import emulate, readouts  # noqa: F401
