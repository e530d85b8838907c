"""Angle between unit-normal fields, for the normal parity checks.

arccos of a dot product is ill-conditioned near 0: a float32 unit vector whose
norm is off by ~1e-7 already reads as ~4e-4 rad.  Both fields are normalised
in float64 and the angle is taken as atan2(|a x b|, a . b), accurate at every
angle.  Rows where either vector is zero give 0 (the caller masks them)."""
import numpy as np


def angle(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    na = np.linalg.norm(a, axis=1, keepdims=True)
    nb = np.linalg.norm(b, axis=1, keepdims=True)
    a = a / np.where(na > 0, na, 1.0)
    b = b / np.where(nb > 0, nb, 1.0)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))
