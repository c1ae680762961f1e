"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds none of the method's arithmetic: it only draws random
numbers and evaluates the initial fields that define the workloads (a
temperature made of a conductive profile plus random spherical harmonics, an
internal-heating field, request streams with Poisson arrivals).  It knows
nothing about meshes, elements or operators; callers pass the points or the
entity counts, in their own order.

All draws use numpy.random.default_rng(seed) in the order documented on each
function.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_operator_inputs", "temperature", "conductive_profile",
    "heating", "serving_requests", "poisson_arrivals", "random_vector",
]


def uniform_operator_inputs(n_wedges: int, n_vel_nodes: int, n_p_nodes: int, seed: int = 0):
    """Operator-apply inputs: eta = 10^U(-1, 1) per wedge, then u ~ U(-1, 1) as
    [n_vel_nodes, 3] (node-major, component fastest), then p ~ U(-1, 1)."""
    rng = np.random.default_rng(seed)
    eta = 10.0 ** rng.uniform(-1.0, 1.0, n_wedges)
    u = rng.uniform(-1.0, 1.0, (n_vel_nodes, 3))
    p = rng.uniform(-1.0, 1.0, n_p_nodes)
    return eta, u, p


def random_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def conductive_profile(r, r_in: float, r_out: float):
    """Steady spherical conduction between T(r_in) = 1 and T(r_out) = 0."""
    r = np.asarray(r, dtype=np.float64)
    return r_in * (r_out - r) / (r * (r_out - r_in))


def _real_sph_harm(l: int, m: int, theta, phi):
    """Real orthonormal spherical harmonic (theta polar, phi azimuth)."""
    from scipy.special import sph_harm_y
    if m == 0:
        return np.real(sph_harm_y(l, 0, theta, phi))
    y = sph_harm_y(l, abs(m), theta, phi)
    return np.sqrt(2.0) * (np.real(y) if m > 0 else np.imag(y))


def harmonic_basis(unit_xyz: np.ndarray, lmin: int, lmax: int) -> np.ndarray:
    """[n_points, n_harmonics] real orthonormal Y_lm, l-major then m = -l..l, for
    reuse by many temperature draws on the same points."""
    unit_xyz = np.asarray(unit_xyz, np.float64)
    x, y, z = unit_xyz[:, 0], unit_xyz[:, 1], unit_xyz[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))
    phi = np.arctan2(y, x)
    cols = [_real_sph_harm(l, m, theta, phi) for l in range(lmin, lmax + 1) for m in range(-l, l + 1)]
    return np.stack(cols, axis=1)


def _harmonic_pattern(unit_xyz: np.ndarray, lmin: int, lmax: int, rng, basis=None) -> np.ndarray:
    if basis is None:
        basis = harmonic_basis(unit_xyz, lmin, lmax)
    c = np.concatenate([rng.standard_normal(2 * l + 1) for l in range(lmin, lmax + 1)])
    a = basis @ c
    return a / np.max(np.abs(a))


def temperature(unit_xyz: np.ndarray, r: np.ndarray, seed: int, r_in: float = 0.55,
                r_out: float = 1.0, lmin: int = 1, lmax: int = 8, amp: float = 0.01, basis=None):
    """Initial temperature on a tensor grid of lateral points x radii.

    T(s, r) = T_cond(r) + amp * A(s) * sin(pi (r - r_in) / (r_out - r_in)), with
    A = sum_{l=lmin..lmax} sum_m c_lm Y_lm (real, orthonormal), c_lm ~ N(0, 1)
    drawn l-major then m = -l..l, and A rescaled so that max |A| = 1 over the
    given lateral points.  Returns [n_lat, n_r].  basis: harmonic_basis(unit_xyz,
    lmin, lmax) of the same points, to skip re-evaluating the harmonics.
    """
    rng = np.random.default_rng(seed)
    A = _harmonic_pattern(np.asarray(unit_xyz, np.float64), lmin, lmax, rng, basis)
    r = np.asarray(r, dtype=np.float64)
    prof = conductive_profile(r, r_in, r_out)
    bump = np.sin(np.pi * (r - r_in) / (r_out - r_in))
    return prof[None, :] + amp * A[:, None] * bump[None, :]


def heating(n: int, seed: int, lo: float = 0.0, hi: float = 10.0):
    """Internal heating H ~ U(lo, hi), one independent value per node."""
    return np.random.default_rng(seed).uniform(lo, hi, n)


def serving_requests(n: int, levels=((16, 16), (32, 32), (64, 64)), base_seed: int = 1000,
                     log10_contrast=(2.0, 6.0)):
    """Request i draws from rng(base_seed + i): the level index (uniform), then
    log10 of the viscosity contrast (uniform); its temperature seed is
    base_seed + i.  Returns a list of dicts."""
    out = []
    for i in range(n):
        rng = np.random.default_rng(base_seed + i)
        li = int(rng.integers(len(levels)))
        lc = float(rng.uniform(*log10_contrast))
        out.append({"id": i, "level": li, "mt": levels[li][0], "nr": levels[li][1],
                    "log10_contrast": lc, "seed": base_seed + i})
    return out


def poisson_arrivals(n: int, rate: float, seed: int):
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    gaps = np.random.default_rng(seed).exponential(1.0 / rate, n)
    return np.cumsum(gaps) - gaps[0]
