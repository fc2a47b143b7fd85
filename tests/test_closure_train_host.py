"""Host-side pieces of the closure training pipeline: the constant-increment
blob against the oracle's network, and the a-posteriori least-squares fit
against cases whose answer is known."""
import numpy as np
import pytest

from paper_2509_19171_amd import closure_train as T


def test_constant_blob_gives_uniform_increment():
    """The oracle's network on the blob returns dtau = tau y for any features
    (output weights zero, output bias softplus^-1(y))."""
    import oracle
    from oracle import closure as C

    oracle._load()
    X = np.random.Generator(np.random.PCG64(5)).normal(0, 3, size=(50, 6))
    for y in (0.05, 1.0, 3.0):
        p = C.unpack(T.constant_blob(y).astype(np.float64))
        d = C.dtau_of(p, X, 0.7)
        np.testing.assert_allclose(d, 0.7 * y, rtol=1e-6)


def _fields(seed, E=5, npn=8, dim=3):
    r = np.random.Generator(np.random.PCG64(seed))
    return (r.normal(size=(E, npn, dim)), r.normal(size=(E, npn, dim)), r.uniform(0.5, 2.0, size=(E, npn)))


def test_posterior_fit_recovers_linear_response():
    """If the reference is reached by moving each element c_e of the way along
    the probe's response, the fit returns y_probe c_e (clipped to [0, y_max])."""
    u0, d, wJ = _fields(1)
    c = np.array([0.0, 0.3, 1.0, 2.5, 40.0])
    u1 = u0 + d
    ur = u0 + c[:, None, None] * d
    y = T.posterior_fit(u0, u1, ur, wJ, 0.5, 10.0)
    assert y.shape == wJ.shape
    np.testing.assert_allclose(y[:, 0], np.minimum(0.5 * c, 10.0), rtol=1e-12, atol=1e-15)
    assert np.all(y == y[:, :1])  # one value per element


def test_posterior_fit_projection_and_clipping():
    """A reference off the response line gives the weighted projection; a
    reference behind the plain run gives 0; a probe that moved nothing gives 0."""
    u0, d, wJ = _fields(2, E=3)
    u1 = u0 + d
    rng = np.random.Generator(np.random.PCG64(3))
    ur = u0 + rng.normal(size=u0.shape)
    y = T.posterior_fit(u0, u1, ur, wJ, 1.0, 1e9)
    for e in range(3):
        num = np.sum(wJ[e][:, None] * (ur[e] - u0[e]) * d[e])
        den = np.sum(wJ[e][:, None] * d[e] * d[e])
        assert y[e, 0] == pytest.approx(max(0.0, num / den), rel=1e-12, abs=1e-15)
    y = T.posterior_fit(u0, u1, u0 - d, wJ, 1.0, 10.0)
    assert np.all(y == 0.0)
    y = T.posterior_fit(u0, u0, ur, wJ, 1.0, 10.0)
    assert np.all(y == 0.0)


def test_posterior_fit_over_selected_components():
    """Restricted to one component, the fit sees only that component's
    residual and response."""
    u0, d, wJ = _fields(4, E=2)
    u1 = u0 + d
    ur = u0.copy()
    ur[..., 2] += 0.7 * d[..., 2]          # the axial component moved 0.7 of the way
    ur[..., 0] -= 5.0 * d[..., 0]          # the others against the probe
    y = T.posterior_fit(u0, u1, ur, wJ, 1.0, 10.0, components=(2,))
    np.testing.assert_allclose(y, 0.7, rtol=1e-12)
