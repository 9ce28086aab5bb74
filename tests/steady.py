"""Run-to-steady-state helper for the oracle tests (test infrastructure)."""
import numpy as np


def residual(prev, cur, K):
    """R = |m Ut(t) - m Ut(t-K)|_2 / (K |m Ut(t)|_2), summed over interior cells."""
    den = np.linalg.norm(cur)
    return np.linalg.norm(cur - prev) / (K * den) if den > 0 else np.linalg.norm(cur - prev) / K


def run_to_steady(o, tol=1e-11, K=500, max_steps=400000, threads=0):
    prev = None
    done = 0
    R = np.inf
    while done < max_steps:
        o.step(K, threads)
        done += K
        m, U, Ut = o.moments(threads)
        if not np.isfinite(m).all():
            raise FloatingPointError("non-finite state after %d steps" % done)
        cur = m[:, None] * Ut
        if prev is not None:
            R = residual(prev, cur, K)
            if R < tol:
                break
        prev = cur
    return done, R
