"""The seeded input generators (shared by the oracle tests and the GPU path):
the spherical-harmonic basis is orthonormal on the sphere, a temperature drawn
with a precomputed basis equals the one drawn without it (to rounding), and the
profile keeps the conductive boundary values."""
import numpy as np

import synthetic
from oracle.mesh import ShellMesh


def test_harmonic_basis_is_orthonormal():
    # Fibonacci points give a quadrature of the sphere accurate enough for l <= 4
    n = 20000
    k = np.arange(n) + 0.5
    z = 1.0 - 2.0 * k / n
    phi = np.pi * (1.0 + 5.0 ** 0.5) * k
    rho = np.sqrt(1.0 - z * z)
    pts = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    B = synthetic.harmonic_basis(pts, 1, 4)
    assert B.shape == (n, sum(2 * l + 1 for l in range(1, 5)))
    G = 4.0 * np.pi * (B.T @ B) / n
    assert np.abs(G - np.eye(G.shape[0])).max() < 2e-3


def test_temperature_with_basis_equals_without():
    om = ShellMesh(8, 8)
    basis = synthetic.harmonic_basis(om.s, 1, 16)
    for seed in (1, 7, 123):
        a = synthetic.temperature(om.s, om.r, seed=seed, lmin=1, lmax=16)
        b = synthetic.temperature(om.s, om.r, seed=seed, lmin=1, lmax=16, basis=basis)
        assert np.allclose(a, b, rtol=0, atol=1e-14)


def test_temperature_boundary_values():
    om = ShellMesh(8, 8)
    T = synthetic.temperature(om.s, om.r, seed=3)
    assert np.allclose(T[:, 0], 1.0, atol=1e-14) and np.allclose(T[:, -1], 0.0, atol=1e-14)
