"""Shared helpers of the test suite (no method arithmetic)."""
import numpy as np


def smooth_at_least(L: int) -> int:
    """Smallest 2^a 3^b 5^c >= L with c <= 1 (the documented grid-size rule of
    lc.h), by counting up from L."""
    n = max(int(L), 1)
    while True:
        m = n
        for p in (2, 3):
            while m % p == 0:
                m //= p
        if m in (1, 5):
            return n
        n += 1


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
