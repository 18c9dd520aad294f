"""Run an op stream on the oracle and compute its read-outs.  Test infrastructure."""
from __future__ import annotations

from typing import Iterable, Optional

import numpy as np

from . import channels
from .core import OracleDM


def emulate(n: int, ops: Iterable, dm: Optional[OracleDM] = None) -> OracleDM:
    """Apply ``ops`` in order, one at a time, to |0..0><0..0| (or to ``dm``)."""
    if dm is None:
        dm = OracleDM(n)
    for op in ops:
        what, payload = channels.build(op)
        if what == "matrix":
            dm.apply_matrix(op[1], payload)
        else:
            dm.apply_kraus(op[1], payload)
    return dm


def readouts(dm: OracleDM, pairs=None, with_probs: bool = True) -> dict:
    """Trace, <Z_i>, <Z_iZ_j> for ``pairs`` (all pairs when None), purity and
    (optionally) the diagonal probabilities."""
    n = dm.n
    if pairs is None:
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    out = {
        "trace": dm.trace(),
        "expec_z": dm.expec_z(),
        "purity": dm.purity(),
    }
    if pairs:
        out["expec_zz"] = dm.expec_zz(pairs)
    if with_probs:
        out["probs"] = dm.probs()
    return out
