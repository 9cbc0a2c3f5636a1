"""Shared helpers of the test suite (no method arithmetic)."""
import numpy as np


def smooth_at_least(L: int) -> int:
    """Smallest 2^a 3^b >= L (the documented grid-size rule of lc.h)."""
    best = None
    p3 = 1
    while True:
        v = p3
        while v < L:
            v *= 2
        best = v if best is None else min(best, v)
        if p3 > L:
            break
        p3 *= 3
    return best


def expected_grid(M: int) -> int:
    """M_eff = 4 * smooth_at_least(ceil(max(M, 4) / 4)), computed here
    independently of the library."""
    return 4 * smooth_at_least(-(-max(M, 4) // 4))


def rel_err(got, ref) -> float:
    got = np.asarray(got, dtype=float)
    ref = np.asarray(ref, dtype=float)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def banner(msg: str) -> None:
    print(msg, flush=True)
