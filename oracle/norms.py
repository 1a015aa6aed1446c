"""Error measures (oracle; test infrastructure only)."""

from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def rel_inf(x, ref) -> float:
    """max |x - ref| / max |ref| (the relative infinity norm used in section 4.2)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def rel_fro(x, ref) -> float:
    """||x - ref||_F / ||ref||_F (the relative Frobenius norm used in section 4.1)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(np.asarray(ref).ravel()))


def observed_orders(errors: Sequence[float], steps: Sequence[int]):
    """Observed order log(e_{k-1}/e_k) / log(m_k/m_{k-1}) between consecutive runs
    with m_k constant steps (the order rows of the tables in section 4.2)."""
    return [math.log(errors[k - 1] / errors[k]) / math.log(steps[k] / steps[k - 1])
            for k in range(1, len(errors))]
