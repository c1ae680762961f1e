"""GPU parity of the buoyancy right-hand side, the SUPG energy operator
and the coupled time step with the FP64 oracle."""
import math

import numpy as np
import pytest

import synthetic
from oracle.energy import EnergyOracle
from oracle.mesh import ShellMesh
from oracle.stokes import buoyancy_rhs, eta_from_temperature
from tests._support import LayoutMap

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2609_21633_amd as t
    return t


@pytest.fixture(scope="module")
def ctx(tng):
    return tng.Context(0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def setup(tng, ctx, mt, levels=2):
    mesh = tng.Mesh(ctx, mt, mt, levels=levels)
    om = ShellMesh(mt, mt)
    lm = LayoutMap(*mesh.coords(0), om)
    return mesh, om, lm


def test_buoyancy_rhs(tng, ctx):
    import torch
    mesh, om, lm = setup(tng, ctx, 8)
    T = synthetic.temperature(om.s, om.r, seed=3).ravel()
    f = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    tng.rhs_buoyancy(ctx, mesh, 0, torch.tensor(lm.to_lib(T), device="cuda"), 1e5, f)
    torch.cuda.synchronize()
    want = buoyancy_rhs(om, T, 1e5)
    want[om.boundary_nodes()] = 0.0
    assert rel(lm.from_lib(f.cpu().numpy(), check_dups=1e-13), want) < 1e-12


@pytest.mark.parametrize("dtype,tol", [("float64", 1e-12), ("float32", 1e-5)])
def test_energy_apply(tng, ctx, dtype, tol):
    import torch
    dt_ = getattr(torch, dtype)
    mesh, om, lm = setup(tng, ctx, 8)
    rng = np.random.default_rng(11)
    u = 30.0 * rng.standard_normal((om.n_nodes, 3))
    T = rng.uniform(0, 1, om.n_nodes)
    dt = 2e-3
    eo = EnergyOracle(om, u, dt)
    y = torch.empty(mesh.shape(0), dtype=dt_, device="cuda")
    ut = torch.tensor(lm.to_lib(u), device="cuda").to(dt_).contiguous()
    tng.energy_apply(ctx, mesh, 0, ut, dt, torch.tensor(lm.to_lib(T), device="cuda").to(dt_), y)
    torch.cuda.synchronize()
    assert rel(lm.from_lib(y.double().cpu().numpy()), eo.apply(T)) < tol


def test_coupled_step_energy_matches_oracle(tng, ctx):
    """One coupled step: the GPU velocity is fed to the oracle's energy
    system with the same dt; T^{n+1} must agree with its direct solve."""
    import torch
    mt = 8
    mesh, om, lm = setup(tng, ctx, mt, levels=3)
    T0 = synthetic.temperature(om.s, om.r, seed=4).ravel()
    H = synthetic.heating(om.n_nodes, seed=5)
    s = tng.StokesSolver(ctx, mesh, mixed=1, rtol=1e-8)
    Tt = torch.tensor(lm.to_lib(T0), device="cuda")
    Ht = torch.tensor(lm.to_lib(H), device="cuda")
    u = torch.empty((3,) + mesh.shape(0), dtype=torch.float64, device="cuda")
    p = torch.empty(mesh.shape(1), dtype=torch.float64, device="cuda")
    info = s.energy_step(Tt, u, p, H=Ht, Ra=1e5, E=math.log(1e3), F=math.log(10.0), courant=1.0,
                         energy_rtol=1e-11)
    print("step", info)
    ug = lm.from_lib(u.cpu().numpy(), check_dups=1e-12)
    eo = EnergyOracle(om, ug, info["dt"])
    want = eo.step(T0, H)
    got = lm.from_lib(Tt.cpu().numpy(), check_dups=1e-12)
    assert rel(got, want) < 1e-9
    assert info["stokes"]["rel_res"] <= 1e-8
    assert np.abs(ug).max() > 0
