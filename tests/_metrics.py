"""Error norms used by the parity tests.

Field error (the field relative-error norm is not fixed by the paper; the two
gated norms are):
  l2       ||E_gpu - E_ref||_2 / ||E_ref||_2 over every particle and component;
  cond_max max_i |E_gpu,i - E_ref,i| / A_i with A_i = k sum_j |w q_j| |r_ij| /
           (|r_ij|^2 + eps^2)^(3/2), the sum of the magnitudes of i's terms
           (a per-particle error relative to what the sum had to cancel).
Potential error, per particle: max_i |phi_gpu,i - phi_ref,i| / P_i with
P_i = k sum_j |w q_j| / (|r_ij|^2 + eps^2)^(1/2), the sum of the magnitudes of
phi_i's terms (|phi_i| itself when every charge has one sign).
A receiver with A_i = 0 (or P_i = 0) has only zero terms (a bunch of one
particle, or every other charge zero): its exact value is 0 and any nonzero
result counts as an infinite error.
"""
import numpy as np


def vec(d, keys=("ex", "ey", "ez")):
    return np.stack([np.asarray(d[k]) for k in keys], axis=1)


def l2_rel(got, ref):
    num = np.sqrt(np.sum((got - ref) ** 2))
    den = np.sqrt(np.sum(ref ** 2))
    return num / den if den > 0 else num


def _scaled_max(err, scale):
    err = np.asarray(err, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    if err.size == 0:
        return 0.0
    zero = scale == 0
    if np.any(zero & (err != 0)):
        return float("inf")
    ok = ~zero
    return float(np.max(err[ok] / scale[ok])) if np.any(ok) else 0.0


def vnorm(v):
    """Euclidean norm of each row of an (n, 3) array, without the underflow of
    squaring tiny components."""
    v = np.asarray(v, dtype=np.float64)
    return np.hypot(np.hypot(v[:, 0], v[:, 1]), v[:, 2])


def cond_max(got, ref, amag):
    """max_i |dE_i| / A_i (vectors of shape (n, 3)); A_i = 0 demands dE_i = 0."""
    return _scaled_max(vnorm(got - ref), amag)


def phi_cond_max(got, ref, pmag):
    """max_i |dphi_i| / P_i; P_i = 0 demands dphi_i = 0."""
    return _scaled_max(np.abs(np.asarray(got) - np.asarray(ref)), pmag)
