"""Relative errors e_p = ||approx - exact||_p / ||exact||_p (eq. (5.6))."""
from __future__ import annotations

import numpy as np


def rel_err(approx, exact, p=2) -> float:
    a = np.asarray(approx).reshape(-1)
    e = np.asarray(exact).reshape(-1)
    num = np.linalg.norm(a - e, ord=p)
    den = np.linalg.norm(e, ord=p)
    return float(num / den) if den > 0 else float(num)


def rel_err_rows(approx, exact) -> np.ndarray:
    """Per-right-hand-side relative l2 error for (R, n) arrays."""
    a = np.asarray(approx).reshape(approx.shape[0], -1)
    e = np.asarray(exact).reshape(exact.shape[0], -1)
    return np.linalg.norm(a - e, axis=1) / np.linalg.norm(e, axis=1)
