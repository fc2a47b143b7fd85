"""Reference for the radial profile diagnostic, written from its definition:
element nodes at distance r < rmax from the line through origin along the
unit axis n fall into nbins equal bins of [0, rmax); per bin the lumped-mass
sums sum wJ (u . n) and sum wJ over those nodes (Sec. 3.5 averages the
streamwise velocity over the pipe's axial and azimuthal directions)."""
import numpy as np


def radial_sums(xyz, wJ, u, origin, axis, rmax, nbins):
    d = xyz.shape[-1]
    n = np.asarray(axis, dtype=np.float64)[:d]
    n = n / np.linalg.norm(n)
    v = xyz.reshape(-1, d) - np.asarray(origin, dtype=np.float64)[:d]
    along = v @ n
    r = np.linalg.norm(v - along[:, None] * n[None, :], axis=1)
    b = np.floor(r / rmax * nbins).astype(np.int64)
    ok = b < nbins
    un = u.reshape(-1, d) @ n
    w = wJ.reshape(-1)
    s_un = np.bincount(b[ok], weights=(w * un)[ok], minlength=nbins)
    s_w = np.bincount(b[ok], weights=w[ok], minlength=nbins)
    return s_un, s_w
