"""Pins of the oracle's tables: GLL nodes and weights, the derivative matrix,
the lattices and the filter (closed forms, exactness, invariants, golden values)."""
import json
import math
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from conftest import ROOT

GOLDEN = os.path.join(ROOT, "tests", "golden")


# ---------------------------------------------------------------- GLL -------
@pytest.mark.parametrize("N,nodes,weights", [
    (2, [-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    (3, [-1.0, -1 / math.sqrt(5), 1 / math.sqrt(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (4, [-1.0, -math.sqrt(3 / 7), 0.0, math.sqrt(3 / 7), 1.0],
     [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_gll_closed_forms(oracle_mod, N, nodes, weights):
    xi, w = oracle_mod.gll(N)
    np.testing.assert_allclose(xi, nodes, atol=1e-15)
    np.testing.assert_allclose(w, weights, rtol=1e-14)


@pytest.mark.parametrize("N", range(1, 16))
def test_gll_against_library_and_quadrature(oracle_mod, N):
    xi, w = oracle_mod.gll(N)
    # interior nodes are the roots of P_N' (library root finder)
    c = np.zeros(N + 1)
    c[N] = 1
    if N >= 2:
        r = np.sort(np.real(npleg.legroots(npleg.legder(c))))
        np.testing.assert_allclose(xi[1:-1], r, atol=1e-13)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    np.testing.assert_allclose(xi, -xi[::-1], atol=1e-15)
    np.testing.assert_allclose(w, w[::-1], rtol=1e-13)
    # GLL quadrature is exact for degree <= 2N - 1
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, (N, k)
    if N >= 1:
        # and not for degree 2N (the GLL rule has precision exactly 2N - 1)
        assert abs(np.dot(w, xi ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-11


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7, 8, 12])
def test_dmat_exact_on_polynomials(oracle_mod, N):
    xi, _ = oracle_mod.gll(N)
    D = oracle_mod.dmat(N, xi)
    for k in range(N + 1):
        d = D @ xi ** k
        exact = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.abs(d - exact).max() < 1e-12 * max(1, N * N), (N, k)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-12)
    # centro-antisymmetry of the GLL derivative
    np.testing.assert_allclose(D[::-1, ::-1], -D, atol=1e-12)
    # corner entries -N(N+1)/4, +N(N+1)/4
    assert abs(D[0, 0] + N * (N + 1) / 4) < 1e-12
    assert abs(D[N, N] - N * (N + 1) / 4) < 1e-12


def test_legendre_against_library(oracle_mod):
    for n in range(0, 12):
        c = np.zeros(n + 1)
        c[n] = 1
        for x in (-1.0, -0.3, 0.2, 0.77, 1.0):
            L, dL = oracle_mod.legendre(n, x)
            assert abs(L - npleg.legval(x, c)) < 1e-13
            assert abs(dL - npleg.legval(x, npleg.legder(c))) < 1e-11


# ------------------------------------------------------------- lattice -------
@pytest.mark.parametrize("dim,Q,w0", [(2, 9, 4 / 9), (3, 19, 1 / 3), (3, 27, 8 / 27)])
def test_lattice_isotropy(oracle_mod, dim, Q, w0):
    e, t, opp = oracle_mod.lattice(dim, Q)
    cs2 = 1 / 3
    assert e.shape == (Q, dim)
    assert abs(t.sum() - 1) < 1e-15
    assert abs(t[0] - w0) < 1e-15 and np.all(e[0] == 0)
    np.testing.assert_allclose(t @ e, 0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("a,ai,aj->ij", t, e, e), cs2 * np.eye(dim), atol=1e-15)
    np.testing.assert_allclose(np.einsum("a,ai,aj,ak->ijk", t, e, e, e), 0, atol=1e-15)
    I = np.eye(dim)
    iso4 = cs2 ** 2 * (np.einsum("ij,kl->ijkl", I, I) + np.einsum("ik,jl->ijkl", I, I) +
                       np.einsum("il,jk->ijkl", I, I))
    np.testing.assert_allclose(np.einsum("a,ai,aj,ak,al->ijkl", t, e, e, e, e), iso4, atol=1e-15)
    # opposite index
    assert np.all(opp[opp] == np.arange(Q))
    np.testing.assert_array_equal(e[opp], -e)
    np.testing.assert_array_equal(t[opp], t)
    # the velocity ordering convention a = a0 + 3 a1 (+ 9 a2), components {0,+1,-1}
    comp = np.array([0, 1, -1])
    full = [(comp[a % 3], comp[(a // 3) % 3], comp[a // 9]) for a in range(3 ** dim)]
    full = [v[:dim] for v in full if sum(x * x for x in v[:dim]) <= (2 if Q == 19 else 3)]
    np.testing.assert_array_equal(e, np.array(full))


# -------------------------------------------------------------- filter -------
def test_filter_sigma_golden(oracle_mod):
    with open(os.path.join(GOLDEN, "filter_sigma.json")) as fh:
        gold = json.load(fh)
    for c in gold["cases"]:
        s = oracle_mod.filter_sigma(c["N"], "quad", c["kc"], c["gamma"])
        exp = np.array(c["sigma_num"], float) / np.array(c["sigma_den"], float)
        np.testing.assert_allclose(s, exp, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N,ftype,kc,amp,order", [
    (7, "quad", 2, 0.1, 2.0), (4, "quad", 2, 0.1, 2.0), (8, "quad", 2, 0.1, 2.0),
    (7, "exp", 4, 36.0, 16.0), (5, "exp", 3, 36.0, 16.0), (7, "quad", 3, 0.3, 2.0)])
def test_filter_properties(oracle_mod, N, ftype, kc, amp, order):
    xi, w = oracle_mod.gll(N)
    F = oracle_mod.filter_matrix(N, ftype, kc, amp, order, xi)
    sigma = oracle_mod.filter_sigma(N, ftype, kc, amp, order)
    # eigenvalues are sigma
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(F).real), np.sort(sigma), atol=1e-12)
    # polynomials of degree <= kc are unchanged
    for k in range(kc + 1):
        np.testing.assert_allclose(F @ xi ** k, xi ** k, atol=1e-13)
    # each basis mode phi_k (nodal values) is scaled by sigma_k
    for k in range(N + 1):
        ck = np.zeros(N + 1)
        ck[k] = 1
        phi = npleg.legval(xi, ck)
        if k >= 2:
            ck2 = np.zeros(N + 1)
            ck2[k - 2] = 1
            phi = phi - npleg.legval(xi, ck2)
        np.testing.assert_allclose(F @ phi, sigma[k] * phi, atol=1e-12)
    # end rows are unit vectors: face values are only filtered tangentially
    np.testing.assert_allclose(F[0], np.eye(N + 1)[0], atol=1e-14)
    np.testing.assert_allclose(F[N], np.eye(N + 1)[N], atol=1e-14)
    # reversal symmetry
    np.testing.assert_allclose(F[::-1, ::-1], F, atol=1e-13)
    # element integral preserved for kc >= 2
    np.testing.assert_allclose(w @ F, w, atol=1e-14)


def test_filter_identity_and_mass_fails_for_kc1(oracle_mod):
    N = 7
    F = oracle_mod.filter_matrix(N, "quad", 2, 0.0)
    np.testing.assert_allclose(F, np.eye(N + 1), atol=1e-13)
    xi, w = oracle_mod.gll(N)
    F1 = oracle_mod.filter_matrix(N, "quad", 1, 0.1, 2.0, xi)
    assert np.abs(w @ F1 - w).max() > 1e-4  # mode 2 has non-zero mean


def test_filter_exponential_values(oracle_mod):
    # exp(-alpha ((k - kc)/(N - kc))^s) with alpha = 36, s = 16, kc = 4, N = 7
    s = oracle_mod.filter_sigma(7, "exp", 4, 36.0, 16.0)
    assert np.all(s[:5] == 1.0)
    assert abs(s[7] - math.exp(-36.0)) < 1e-20
    assert abs(s[6] - math.exp(-36.0 * (2 / 3) ** 16)) < 1e-15
