"""Pins of the assembled oracle operator (Sec. 3 eq:matfree, Sec. 7 saddle point)."""
import numpy as np
import pytest

import synthetic
from oracle.mesh import ShellMesh
from oracle.stokes import StokesOracle


@pytest.fixture(scope="module")
def op44():
    m = ShellMesh(4, 4)
    eta, _, _ = synthetic.uniform_operator_inputs(m.n_wedges, 1, 1, seed=11)
    return StokesOracle(4, 4, eta)


def _rigid_fields(xyz):
    out = {f"t{c}": np.tile(np.eye(3)[c], (len(xyz), 1)) for c in range(3)}
    for c in range(3):
        out[f"r{c}"] = np.cross(np.eye(3)[c], xyz)
    return out


def test_symmetry(op44):
    """x^T K_D y = y^T K_D x, and the two off-diagonal blocks are transposes."""
    rng = np.random.default_rng(1)
    K = op44.K
    for _ in range(3):
        x, y = rng.standard_normal(K.shape[0]), rng.standard_normal(K.shape[0])
        assert abs(x @ (K @ y) - y @ (K @ x)) < 1e-13 * np.abs(x) @ (abs(K) @ np.abs(y))
    assert abs(op44.BT_D - op44.B_D.T).max() == 0.0


def test_null_spaces_without_dirichlet(op44):
    """A annihilates translations, rotations and the dilation x; B annihilates
    translations and rotations (isoparametric linear fields are exact)."""
    xyz = op44.mesh.node_xyz()
    scale = abs(op44.A).max()
    for name, v in _rigid_fields(xyz).items():
        assert np.abs(op44.A @ v.ravel()).max() < 1e-13 * scale, name
        assert np.abs(op44.B @ v.ravel()).max() < 1e-14, name
    assert np.abs(op44.A @ xyz.ravel()).max() < 1e-13 * scale
    assert np.abs(op44.B @ xyz.ravel()).max() > 1e-3          # div x = 3


def test_patch_test_uniform_layers(op44):
    """With uniform radial spacing sum_e V_e grad phi_j(q_c) = 0 at interior
    nodes, hence B^T 1 = 0 on interior rows and, for constant eta, A (linear
    field) = 0 on interior rows."""
    m = op44.mesh
    interior = ~m.boundary_nodes()
    bt1 = (op44.B.T @ np.ones(op44.n_p)).reshape(-1, 3)
    assert np.abs(bt1[interior]).max() < 1e-15
    assert np.abs(bt1[~interior]).max() > 1e-3
    o1 = StokesOracle(4, 4, np.ones(m.n_wedges))
    G = np.random.default_rng(2).standard_normal((3, 3))
    r = (o1.A @ (m.node_xyz() @ G.T).ravel()).reshape(-1, 3)
    assert np.abs(r[interior]).max() < 1e-14
    assert np.abs(r[~interior]).max() > 1e-3


def test_velocity_block_positive_definite(op44):
    """D A D restricted to interior DoFs is positive definite (Sec. 4: local
    hourglass modes do not persist on the assembled shell)."""
    interior = ~op44.dirichlet
    Ad = op44.A_D.toarray()[np.ix_(interior, interior)]
    ev = np.linalg.eigvalsh(Ad)
    assert ev[0] > 1e-4 * ev[-1]


def test_pressure_null_space_is_constant_only(op44):
    """The only pressure vector with B D^T p = 0 is the constant (inf-sup stable pair)."""
    interior = ~op44.dirichlet
    BD = op44.B.toarray()[:, interior]
    s = np.linalg.svd(BD, compute_uv=False)
    assert s[-1] < 1e-14 * s[0]
    assert s[-2] > 1e-2 * s[0]


def test_dirichlet_rows_are_identity(op44):
    rng = np.random.default_rng(4)
    u = rng.uniform(-1, 1, (op44.mesh.n_nodes, 3))
    p = rng.uniform(-1, 1, op44.n_p)
    yu, _ = op44.apply(u, p)
    bnd = op44.mesh.boundary_nodes()
    assert np.array_equal(yu[bnd], u[bnd])


def test_solve_residual_and_pressure_mean(op44):
    rng = np.random.default_rng(6)
    f = rng.standard_normal((op44.mesh.n_nodes, 3))
    f[op44.mesh.boundary_nodes()] = 0.0
    u, p = op44.solve(f)
    yu, yp = op44.apply(u, p)
    assert np.abs(yu - f).max() < 1e-10 * np.abs(f).max()
    assert np.abs(yp).max() < 1e-10
    assert abs(p.mean()) < 1e-12
