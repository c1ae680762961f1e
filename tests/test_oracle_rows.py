"""The row-at-a-time oracle (used for full-size sampled parity) reproduces every
row of the assembled, already pinned StokesOracle at small sizes, for the
velocity rows (interior and Dirichlet) and the pressure rows, and its viscosity
law on a wedge subset equals the whole-mesh law."""
import math

import numpy as np
import pytest

import synthetic
from oracle.mesh import ShellMesh
from oracle.rows import StokesRows, eta_law
from oracle.stokes import StokesOracle, eta_from_temperature


@pytest.mark.parametrize("mt,nr", [(4, 4), (8, 6)])
def test_rows_equal_assembled_operator(mt, nr):
    om = ShellMesh(mt, nr)
    omp = ShellMesh(mt // 2, nr // 2, hierarchy=om.h)
    eta, u, p = synthetic.uniform_operator_inputs(om.n_wedges, om.n_nodes, omp.n_nodes, seed=3)
    orc = StokesOracle(mt, nr, eta, hierarchy=om.h)
    yu, yp = orc.apply(u, p)
    rows = StokesRows(om)
    eta_of = lambda w: eta[w]
    scale_u = np.abs(yu).max()
    for nd in range(om.n_nodes):
        y, s = rows.velocity_row(nd, eta_of, u, p)
        assert np.all(s >= np.abs(y) * (1 - 1e-12))
        assert np.abs(y - yu[nd]).max() <= 1e-13 * scale_u, nd
    scale_p = np.abs(yp).max()
    for q in range(omp.n_nodes):
        y, s = rows.pressure_row(q, eta_of, u)
        assert s >= abs(y) * (1 - 1e-12)
        assert abs(y - yp[q]) <= 1e-13 * scale_p, q


def test_eta_law_on_subset():
    om = ShellMesh(8, 8)
    T = synthetic.temperature(om.s, om.r, seed=1, lmin=1, lmax=8, amp=0.01).ravel()
    full = eta_from_temperature(om, T, math.log(1e3), math.log(10.0))
    w = np.random.default_rng(0).choice(om.n_wedges, 300, replace=False)
    assert np.allclose(eta_law(om, T, w, math.log(1e3), math.log(10.0)), full[w], rtol=1e-15, atol=0)
