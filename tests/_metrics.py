"""Error norms used by the parity tests.

Field error (the field relative-error norm is not fixed by the paper; the two
gated norms are):
  l2       ||E_gpu - E_ref||_2 / ||E_ref||_2 over every particle and component;
  cond_max max_i |E_gpu,i - E_ref,i| / A_i with A_i = k sum_j |w q_j| |r_ij| /
           (|r_ij|^2 + eps^2)^(3/2), the sum of the magnitudes of i's terms
           (a per-particle error relative to what the sum had to cancel).
"""
import numpy as np


def vec(d, keys=("ex", "ey", "ez")):
    return np.stack([np.asarray(d[k]) for k in keys], axis=1)


def l2_rel(got, ref):
    num = np.sqrt(np.sum((got - ref) ** 2))
    den = np.sqrt(np.sum(ref ** 2))
    return num / den if den > 0 else num


def cond_max(got, ref, amag):
    err = np.linalg.norm(got - ref, axis=1)
    ok = amag > 0
    if not np.any(ok):
        return float(np.max(err)) if err.size else 0.0
    return float(np.max(err[ok] / amag[ok]))
