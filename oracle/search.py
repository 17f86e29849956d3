"""Plain oracle of the search for a first collision-free motion (paper Sec. IV-B, Alg. 1).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may use this module.  It shares no code with the HIP library.

The algorithm is run exactly as the paper states it, one motion at a time, in plain
Python: a first loop over the motions in the given order asks the proxy d_hat(X, m)
and runs the exact distance d(X, m) only where d_hat exceeds the margin eps, returning
the first motion whose exact distance exceeds eps; failing that, a second loop visits
the motions the first loop did not check, by d_hat descending, and returns the first
whose exact distance exceeds eps.  Without a proxy (the plain search) every motion is
checked exactly in the given order.

Reading where the paper is silent: motions with equal d_hat keep their given order in
the second loop (a stable sort), and a NaN proxy value sorts last.
"""
from __future__ import annotations

import math


def first_free(d, eps, d_hat=None):
    """Alg. 1 over exact distances d[m] (and proxy values d_hat[m], or None).

    Returns (motion or -1, exact checks made, proxy evaluations made, first-loop motions).
    """
    M = len(d)
    if d_hat is None:
        for m in range(M):
            if d[m] > eps:
                return m, m + 1, 0, 0
        return -1, M, 0, 0
    key = [(-math.inf if math.isnan(v) else float(v)) for v in d_hat]
    done = set()
    n_exact = 0
    n_nn = 0
    for m in range(M):                      # first loop
        n_nn += 1
        if key[m] > eps:
            n_exact += 1
            done.add(m)
            if d[m] > eps:
                return m, n_exact, n_nn, sum(1 for v in key if v > eps)
    rest = sorted((m for m in range(M) if m not in done), key=lambda m: -key[m])   # stable: ties keep order
    for m in rest:                          # second loop
        n_exact += 1
        if d[m] > eps:
            return m, n_exact, n_nn, len(done)
    return -1, n_exact, n_nn, len(done)


def visiting_order(d_hat, eps):
    """The order in which Alg. 1 runs exact checks when no motion is free."""
    M = len(d_hat)
    key = [(-math.inf if math.isnan(v) else float(v)) for v in d_hat]
    first = [m for m in range(M) if key[m] > eps]
    rest = sorted((m for m in range(M) if not key[m] > eps), key=lambda m: -key[m])
    return first + rest
