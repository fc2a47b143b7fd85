"""Pins of the radial-profile reference (tests/radial_ref.py) on the oracle's
pipe geometry: a uniform axial velocity U gives U in every bin exactly; a
velocity U + b x (odd in x) averages to U in every bin, since the O-grid is
symmetric under x -> -x; the weights of all bins add up to the volume of the
pipe (pi R^2 L, to quadrature accuracy of the curved wall elements)."""
import math

import numpy as np

from paper_2509_19171_amd import inputs as I
from radial_ref import radial_sums


def test_radial_reference_pins(oracle_mod):
    c = I.case_pipe(N=4, nsq=2, nrad=2, nax=2, L=2.0, pert=0.0, filt=None)
    o = oracle_mod.from_case(c)
    wJ, _, _ = o.geometry()
    x = c.mesh.xyz
    R, L = c.meta["R"], c.meta["L"]
    u = np.zeros_like(x)
    u[..., 2] = 0.03
    s, w = radial_sums(x, wJ, u, (0, 0, 0), (0, 0, 2.0), R * (1 + 1e-12), 8)
    assert np.all(w > 0)
    np.testing.assert_allclose(s / w, 0.03, rtol=1e-13)
    u[..., 2] = 0.03 + 0.01 * x[..., 0]
    s, w = radial_sums(x, wJ, u, (0, 0, 0), (0, 0, 1.0), R * (1 + 1e-12), 8)
    np.testing.assert_allclose(s / w, 0.03, rtol=1e-12)
    assert abs(w.sum() - math.pi * R * R * L) < 1e-6 * math.pi * R * R * L
