"""Exact discrete solution of the Stokes saddle point K_D [u; p] = [f; g]
(Sec. 7) by Schur-complement reduction.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

With velocity Dirichlet rows the viscous block A_D is symmetric positive
definite, so  u = A_D^{-1} (f - B_D^T p)  and the pressure solves the Schur
system

    S p = B_D A_D^{-1} f - g,        S = B_D A_D^{-1} B_D^T,

which is symmetric positive semi-definite with the constant pressures as its
null space (B_D^T 1 = 0 once the sphere rows are Dirichlet rows).  A_D is
factorised once (sparse LU with a symmetric ordering and no pivoting, which
an SPD matrix does not need), and S p = r is solved by conjugate gradients
on mean-zero pressures, preconditioned by the inverse of the row-sum-lumped
inverse-viscosity pressure mass (the Schur approximation of eq:pmass).  Every
CG step applies S exactly (one forward and one backward substitution), so
the result is the exact discrete solution up to the CG tolerance: the same x
as a direct solve of K_D, without the fill-in that pivoting on the zero
pressure block causes in a direct saddle-point factorisation.

The Krylov method here is only a route to that exact x; it is not the
paper's solver (FGMRES with a multigrid-preconditioned block-triangular
preconditioner), and nothing of it is compared with the GPU path except the
solution itself.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .solver_ref import lumped_pressure_mass
from .stokes import StokesOracle


class SchurSolver:
    """Factorises A_D of ``orc`` once; ``solve`` returns (u, p, info)."""

    def __init__(self, orc: StokesOracle, eta_wedge: np.ndarray):
        self.orc = orc
        self.lu = spla.splu(orc.A_D.tocsc(), permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                            options=dict(SymmetricMode=True))
        self.minv = 1.0 / lumped_pressure_mass(orc, eta_wedge)
        self.BT = orc.BT_D.tocsr()
        self.B = orc.B_mass.tocsr()
        # a mass block other than B_D (the reference density of TALA) makes S
        # non-symmetric: GMRES instead of CG
        self.symmetric = orc.B_mass is orc.B_D

    def _schur(self, p: np.ndarray) -> np.ndarray:
        return self.B @ self.lu.solve(self.BT @ p)


    def _gmres(self, r: np.ndarray, rtol: float, maxiter: int):
        """S p = r on mean-zero pressures by right-preconditioned restarted GMRES
        (Saad's algorithm with modified Gram-Schmidt), the same preconditioner."""
        n = len(r)
        m = 60
        p = np.zeros(n)
        r0 = np.linalg.norm(r)
        its = 0
        res = r.copy()
        while its < maxiter:
            beta = np.linalg.norm(res)
            if beta <= rtol * r0:
                break
            V = np.zeros((m + 1, n))
            Z = np.zeros((m, n))
            H = np.zeros((m + 1, m))
            V[0] = res / beta
            k_used = 0
            for k in range(m):
                z = self.minv * V[k]
                z -= z.mean()
                Z[k] = z
                w = self._schur(z)
                w -= w.mean()
                for i in range(k + 1):
                    H[i, k] = w @ V[i]
                    w -= H[i, k] * V[i]
                H[k + 1, k] = np.linalg.norm(w)
                k_used = k + 1
                its += 1
                e1 = np.zeros(k + 2)
                e1[0] = beta
                y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)
                if np.linalg.norm(H[:k + 2, :k + 1] @ y - e1) <= rtol * r0 or H[k + 1, k] == 0.0:
                    break
                V[k + 1] = w / H[k + 1, k]
            e1 = np.zeros(k_used + 1)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k_used + 1, :k_used], e1, rcond=None)
            p += y @ Z[:k_used]
            res = r - self._schur(p)
            res -= res.mean()
        return p, its

    def solve(self, f: np.ndarray, g: np.ndarray | None = None, rtol: float = 1e-13, maxiter: int = 5000):
        """K_D [u; p] = [f; g], f as [n_nodes, 3] (its Dirichlet rows are the
        prescribed boundary velocity).  The pressure is returned with zero mean
        over the unique pressure nodes.  CG stops when the Schur residual is
        below rtol times its initial value."""
        orc = self.orc
        fu = np.asarray(f, np.float64).ravel()
        gp = np.zeros(orc.n_p) if g is None else np.asarray(g, np.float64)
        w = self.lu.solve(fu)
        r = self.B @ w - gp
        r -= r.mean()
        p = np.zeros(orc.n_p)
        r0 = np.linalg.norm(r)
        its = 0
        if r0 > 0.0 and not self.symmetric:
            p, its = self._gmres(r, rtol, maxiter)
        elif r0 > 0.0:
            z = self.minv * r
            z -= z.mean()
            d = z.copy()
            rz = r @ z
            while its < maxiter:
                its += 1
                q = self._schur(d)
                a = rz / (d @ q)
                p += a * d
                r -= a * q
                r -= r.mean()
                if np.linalg.norm(r) <= rtol * r0:
                    break
                z = self.minv * r
                z -= z.mean()
                rz_new = r @ z
                d = z + (rz_new / rz) * d
                rz = rz_new
        p -= p.mean()
        u = self.lu.solve(fu - self.BT @ p)

        x = np.concatenate([u, p])
        b = np.concatenate([fu, gp])
        res = np.linalg.norm(orc.K @ x - b) / max(np.linalg.norm(b), 1e-300)
        return u.reshape(-1, 3), p, {"cg_its": its, "rel_res": float(res)}
