"""Writes stokes16_contrast1e6.npz: the oracle's exact discrete Stokes solution
on the (16,16) copy of the contrast-1e6 workload, for the GPU solve parity
test.  Calls only ``oracle/`` (and the seeded input generator ``synthetic``).

Workload (the (128,128) contrast-1e6 configuration at (16,16) resolution):
T = conductive profile + 0.01 x seeded spherical harmonics l = 1..8 (seed 1),
eta_e = exp(-ln(1e6) Tbar_e) per wedge (Tbar_e the mean of its six nodal T),
f = Ra T rhat with Ra = 1e5 (one-point buoyancy of eq:stokes, Boussinesq form),
g = 0, zero velocity on both spheres; pressure with zero mean over unique
nodes.  Solved by the oracle's Schur-complement reduction (exact A_D
factorisation, CG on the Schur system to 1e-13).

The file also holds the lateral unit vectors and radii of the velocity and
pressure nodes in the stored order (unique nodes, radial index fastest).

Run:  python tests/golden/make_stokes16_contrast1e6.py   (about 4 minutes)
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from oracle.mesh import ShellMesh  # noqa: E402
from oracle.saddle import SchurSolver  # noqa: E402
from oracle.stokes import StokesOracle, buoyancy_rhs, eta_from_temperature  # noqa: E402

MT = NR = 16
SEED, LMAX, AMP = 1, 8, 0.01
E, RA = np.log(1e6), 1e5
OUT = os.path.join(HERE, "stokes16_contrast1e6.npz")


def inputs():
    om = ShellMesh(MT, NR)
    T = synthetic.temperature(om.s, om.r, seed=SEED, lmin=1, lmax=LMAX, amp=AMP).ravel()
    eta = eta_from_temperature(om, T, E, 0.0)
    f = buoyancy_rhs(om, T, RA)
    f[om.boundary_nodes()] = 0.0
    return om, T, eta, f


def main():
    t0 = time.time()
    om, T, eta, f = inputs()
    orc = StokesOracle(MT, NR, eta, hierarchy=om.h)
    print(f"assembled in {time.time() - t0:.1f} s; factorising A_D", flush=True)
    sol = SchurSolver(orc, eta)
    print(f"factorised in {time.time() - t0:.1f} s; Schur CG", flush=True)
    u, p, info = sol.solve(f, rtol=1e-13)
    print(f"CG its {info['cg_its']}, relative residual of K_D x = b: {info['rel_res']:.2e}, "
          f"total {time.time() - t0:.1f} s", flush=True)
    omp = ShellMesh(MT // 2, NR // 2, hierarchy=om.h)
    # node coordinates (unit vectors of the lateral nodes, radii) of the velocity and
    # pressure grids, so that a reader can match other layouts to this node order
    np.savez_compressed(OUT, u=u, p=p, T_sum=T.sum(), eta_logsum=np.log(eta).sum(), f_norm=np.linalg.norm(f),
                        cg_its=info["cg_its"], rel_res=info["rel_res"], s_u=om.s, r_u=om.r, s_p=omp.s, r_p=omp.r)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
