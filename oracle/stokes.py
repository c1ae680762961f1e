"""Oracle Stokes operator: assembled element matrices, SpMV and direct solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The matrix-free product of eq:matfree equals, up to rounding order, the
assembled sparse product  y = sum_e I_e^T A_e I_e x.  This module therefore
forms every element matrix explicitly from eq:elemmat, evaluated with the one
quadrature point q_c = (1/3, 1/3, 0) of weight w_q = 1 (Sec. 4, eq:oneptenergy:
V_e = w_q |det J(q_c)|; the reference wedge has volume 1/2 * 2 = 1), assembles
them with scipy, and multiplies.  It deliberately does NOT use the strain
contraction of eq:epsq / eq:localapply that the GPU kernel uses.

Readings (the same on both sides):
* geometry: isoparametric 6-node map x(xi, eta, zeta) = sum_j N_j x_j, x_j the
  physical node positions (chordal triangle times linear radius);
* pressure: W1 on the coarse grid (level - 1, nr / 2); its value inside a fine
  wedge is the fine-W1 interpolant P p of the coarse nodal values, so that
  B = P^T B_f with B_f the divergence form against fine W1 test functions;
* sign: B is the weak form of -div, (B_f)_{i,(j,c)} = -V_e N_i(q_c) d_c phi_j(q_c);
* Dirichlet: velocity rows on both spheres become identity rows and their
  columns are dropped:  K_D = [[D A D + (I - D), D B^T], [B D, 0]];
* free slip (the setup of the paper's verification runs, Sec. 8): at a node of
  a free-slip sphere the velocity is expressed in the local frame (rhat, two
  tangential directions), rhat = x / |x| the sphere's normal at the node; the
  normal component is a Dirichlet DoF (identity row, column dropped) and the
  two tangential ones are free (zero tangential traction, a natural condition).
  Rotating back to Cartesian components gives, per node, the projection
  P = I - rhat rhat^T onto the tangent plane and N = rhat rhat^T:
  K = [[P A P + N, P B^T], [B P, 0]], which is the no-slip K_D with P = 0,
  N = I on no-slip nodes (and P = I, N = 0 inside);
* compressible mass balance (TALA, eq:mass: div(rhobar u) = 0, rhobar(r) the
  reference density): the mass rows are -(psi_I, div(rhobar u)) with the mass
  flux rhobar u interpolated in the velocity space, i.e. the nodal products
  rhobar(r_j) u_j, so B_rho = B R with R = diag(rhobar at each node's radius).
  This keeps the discrete compatibility 1^T B_rho = 0 of the Dirichlet/free-
  slip spaces (the divergence of a field that vanishes, or is tangential, on
  the spheres sums to zero over the pressure nodes), which the product form
  rhobar div u + u . grad rhobar evaluated at q_c does not; the momentum rows
  keep B^T (eq:stokes);
* per-wedge viscosity: eta(q_c) is the wedge's value; for temperature-driven
  laws it is the law evaluated at the mean of the six nodal temperatures and
  the wedge's mid radius (the value of the W1 interpolant at q_c);
* pressure normalisation: the nodal mean over unique pressure nodes is zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .mesh import ShellMesh, SphereHierarchy, prolongation

QC = (1.0 / 3.0, 1.0 / 3.0, 0.0)   # barycentre of the reference wedge (Sec. 4)
W_Q = 1.0                          # weight of the one-point rule


def ref_basis(xi: float, eta: float, zeta: float):
    """eq:wedgebasis: N_j = N^lat_{j mod 3}(xi, eta) N^rad_{floor(j/3)}(zeta).

    Returns (N[6], dN[6, 3]) with dN[j] = (dN_j/dxi, dN_j/deta, dN_j/dzeta).
    """
    nl = np.array([1.0 - xi - eta, xi, eta])
    dnl = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])   # d/dxi, d/deta of N^lat
    nrad = np.array([0.5 * (1.0 - zeta), 0.5 * (1.0 + zeta)])
    dnrad = np.array([-0.5, 0.5])
    N = np.empty(6)
    dN = np.empty((6, 3))
    for j in range(6):
        a, b = j % 3, j // 3
        N[j] = nl[a] * nrad[b]
        dN[j, 0] = dnl[a, 0] * nrad[b]
        dN[j, 1] = dnl[a, 1] * nrad[b]
        dN[j, 2] = nl[a] * dnrad[b]
    return N, dN


def wedge_geometry(xw: np.ndarray, point=QC):
    """Jacobian, |det J| and physical basis gradients at a reference point.

    xw: [n, 6, 3] physical node positions of n wedges.  J[:, a, m] =
    sum_j x_j[a] dN_j/dxi_m; grad phi_j = J^{-T} dN_j.  Returns (J, V, grads)
    with V = w_q |det J| (eq:oneptenergy) and grads[n, 6, 3].
    """
    _, dN = ref_basis(*point)
    J = np.einsum("wja,jm->wam", xw, dN)
    V = W_Q * np.abs(np.linalg.det(J))
    Jinv = np.linalg.inv(J)
    grads = np.einsum("jm,wma->wja", dN, Jinv)   # row j: dN_j^T J^{-1} = (J^{-T} dN_j)^T
    return J, V, grads


def element_matrices(xw: np.ndarray, eta: np.ndarray):
    """A_e of eq:elemmat with the one-point rule, for n wedges -> [n, 18, 18].

    Local DoF a = 3 j + c is basis function phi_j times unit vector e_c.
    (A_e)_ab = V_e eta_e [2 eps(phi_a) : eps(phi_b) - 2/3 div(phi_a) div(phi_b)].
    """
    _, V, g = wedge_geometry(xw)
    n = len(xw)
    eye = np.eye(3)
    # eps(phi_j e_c) = 1/2 (e_c g_j^T + g_j e_c^T), shape [n, 6, 3(c), 3, 3]
    outer = np.einsum("cm,wjn->wjcmn", eye, g)
    eps = 0.5 * (outer + np.swapaxes(outer, 3, 4))
    eps = eps.reshape(n, 18, 3, 3)
    div = g.reshape(n, 18)                      # div(phi_j e_c) = d_c phi_j
    epseps = np.einsum("wamn,wbmn->wab", eps, eps)
    A = (V * eta)[:, None, None] * (2.0 * epseps - (2.0 / 3.0) * div[:, :, None] * div[:, None, :])
    return A


ZETA2 = 1.0 / np.sqrt(3.0)    # Gauss points of the two-radial-point rule


def element_matrices_2pt(xw: np.ndarray, eta: np.ndarray):
    """A_e of eq:elemmat with the two-radial-point rule (Sec. 4, the second remedy
    beside eq:hgstab): the lateral centroid (1/3, 1/3) times the two-point Gauss
    rule in the radial coordinate, zeta = -+1/sqrt(3), weight 1/2 each (the
    reference wedge has volume 1).  The viscosity is the wedge's value.  -> [n, 18, 18]."""
    n = len(xw)
    A = np.zeros((n, 18, 18))
    eye = np.eye(3)
    for zq in (-ZETA2, ZETA2):
        _, V, g = wedge_geometry(xw, point=(1.0 / 3.0, 1.0 / 3.0, zq))
        outer = np.einsum("cm,wjn->wjcmn", eye, g)
        eps = (0.5 * (outer + np.swapaxes(outer, 3, 4))).reshape(n, 18, 3, 3)
        div = g.reshape(n, 18)
        epseps = np.einsum("wamn,wbmn->wab", eps, eps)
        A += (0.5 * V * eta)[:, None, None] * (2.0 * epseps - (2.0 / 3.0) * div[:, :, None] * div[:, None, :])
    return A


def hourglass_vectors():
    """Nodal values of the three barycentric hourglass modes h_a = (lambda_a - 1/3) zeta,
    a = 0, 1, 2, of the reference wedge (eq:hourglass: w_1 = h_1, w_2 = h_2 and
    h_0 = -h_1 - h_2).  Returns [3, 6] (nodes 0-2 at zeta = -1, 3-5 at zeta = +1)."""
    h = np.empty((3, 6))
    for a in range(3):
        for j in range(6):
            lam = 1.0 if j % 3 == a else 0.0
            zeta = -1.0 if j < 3 else 1.0
            h[a, j] = (lam - 1.0 / 3.0) * zeta
    return h


def element_matrices_hg(xw: np.ndarray, eta: np.ndarray, alpha: float):
    """One-point element matrices with hourglass control (eq:hgstab), [n, 18, 18].

    A_e^stab = A_e + eps_e sum_a sum_d (h_a (x) e_d)(h_a (x) e_d)^T, with eps_e =
    alpha * mean(diag A_e) (a small parameter scaled with the local stiffness).
    The sum runs over all three barycentric hourglass modes h_a, which span the
    same space as w_1, w_2 and make the term independent of which lateral vertex
    a wedge numbers first.
    """
    A = element_matrices(xw, eta)
    if alpha == 0.0:
        return A
    eps = alpha * np.einsum("wii->w", A) / 18.0
    h = hourglass_vectors()
    W = np.zeros((18, 9))                      # columns h_a (x) e_d
    for a in range(3):
        for d in range(3):
            W[d::3, 3 * a + d] = h[a]
    return A + eps[:, None, None] * (W @ W.T)[None, :, :]


def element_divergence(xw: np.ndarray):
    """B_f per wedge, [n, 6, 18]: (B_f)_{i,a} = -V_e N_i(q_c) div(phi_a) at q_c."""
    N, _ = ref_basis(*QC)
    _, V, g = wedge_geometry(xw)
    div = g.reshape(len(xw), 18)
    return -(V[:, None, None] * N[None, :, None] * div[:, None, :])


BC_KINDS = ("noslip", "freeslip", "none")


def boundary_projections(mesh: ShellMesh, bc=("noslip", "noslip")):
    """Sparse block-diagonal P (velocity subspace a node may take) and N = I - P
    on the spheres (0 inside), DoF order 3 node + component.  bc = (inner, outer),
    each "noslip" (P = 0), "freeslip" (P = I - rhat rhat^T) or "none" (P = I, N = 0)."""
    if len(bc) != 2 or any(b not in BC_KINDS for b in bc):
        raise ValueError("bc must be a pair of 'noslip', 'freeslip' or 'none'")
    nn = mesh.n_nodes
    k = np.tile(np.arange(mesh.nr + 1), mesh.n_lat)
    x = mesh.node_xyz()
    rhat = x / np.linalg.norm(x, axis=1)[:, None]
    Pb = np.tile(np.eye(3), (nn, 1, 1))
    Nb = np.zeros((nn, 3, 3))
    for kind, layer in zip(bc, (0, mesh.nr)):
        sel = k == layer
        if kind == "noslip":
            Pb[sel] = 0.0
            Nb[sel] = np.eye(3)
        elif kind == "freeslip":
            nnT = rhat[sel][:, :, None] * rhat[sel][:, None, :]
            Pb[sel] = np.eye(3) - nnT
            Nb[sel] = nnT
    rows = (3 * np.arange(nn)[:, None, None] + np.arange(3)[None, :, None]).repeat(3, axis=2)
    cols = (3 * np.arange(nn)[:, None, None] + np.arange(3)[None, None, :]).repeat(3, axis=1)
    P = sp.csr_matrix((Pb.ravel(), (rows.ravel(), cols.ravel())), shape=(3 * nn, 3 * nn))
    N = sp.csr_matrix((Nb.ravel(), (rows.ravel(), cols.ravel())), shape=(3 * nn, 3 * nn))
    P.eliminate_zeros()
    N.eliminate_zeros()
    return P, N


class StokesOracle:
    """Assembled FP64 Stokes saddle-point operator on the (mt, nr) shell
    (hg_alpha > 0: viscous block with hourglass control, eq:hgstab; quad = "two":
    viscous block with the two-radial-point rule, the divergence blocks keep the
    one-point rule; bc = velocity condition on (inner, outer) sphere, see
    boundary_projections; rho_nodes: TALA reference density)."""

    def __init__(self, mt: int, nr: int, eta_wedge: np.ndarray, r_in: float = 0.55,
                 r_out: float = 1.0, hierarchy: SphereHierarchy | None = None,
                 chunk: int = 200_000, hg_alpha: float = 0.0, bc=("noslip", "noslip"),
                 rho_nodes: np.ndarray | None = None, quad: str = "one"):
        self.mesh = m = ShellMesh(mt, nr, r_in, r_out, hierarchy)
        self.mt, self.nr = mt, nr
        eta_wedge = np.asarray(eta_wedge, dtype=np.float64)
        if eta_wedge.shape != (m.n_wedges,):
            raise ValueError("eta_wedge must have one value per wedge")
        wn = m.wedge_nodes()
        xyz = m.node_xyz()
        nu = 3 * m.n_nodes
        A = sp.csr_matrix((nu, nu))
        Bf = sp.csr_matrix((m.n_nodes, nu))
        for s in range(0, m.n_wedges, chunk):
            w = wn[s:s + chunk]
            xw = xyz[w]
            dof = (w[:, :, None] * 3 + np.arange(3)[None, None, :]).reshape(len(w), 18)
            if quad == "two":
                if hg_alpha != 0.0:
                    raise ValueError("the two-radial-point rule is an alternative to hourglass control")
                Ae = element_matrices_2pt(xw, eta_wedge[s:s + chunk])
            elif quad == "one":
                Ae = element_matrices_hg(xw, eta_wedge[s:s + chunk], hg_alpha)
            else:
                raise ValueError("quad must be 'one' or 'two'")
            rows = np.repeat(dof, 18, axis=1).ravel()
            cols = np.tile(dof, (1, 18)).ravel()
            A = A + sp.csr_matrix((Ae.ravel(), (rows, cols)), shape=(nu, nu))
            Be = element_divergence(xw)
            rows = np.repeat(w, 18, axis=1).ravel()
            cols = np.tile(dof, (1, 6)).ravel()
            Bf = Bf + sp.csr_matrix((Be.ravel(), (rows, cols)), shape=(m.n_nodes, nu))
        self.A = A.tocsr()
        self.Bf = Bf.tocsr()
        self.P = prolongation(m.h, m.L, nr)                 # fine nodes x coarse pressure nodes
        self.B = (self.P.T @ self.Bf).tocsr()               # B = P^T B_f
        self.n_u = nu
        self.n_p = self.P.shape[1]
        self.bc = tuple(bc)
        Pm, Nm = boundary_projections(m, self.bc)
        self.P_bc, self.N_bc = Pm, Nm
        # DoFs with a no-slip (identity) row
        k = np.repeat(np.tile(np.arange(nr + 1), m.n_lat), 3)
        self.dirichlet = ((k == 0) & (self.bc[0] == "noslip")) | ((k == nr) & (self.bc[1] == "noslip"))
        self.A_D = (Pm @ self.A @ Pm + Nm).tocsr()
        self.BT_D = (Pm @ self.B.T).tocsr()
        self.B_D = (self.B @ Pm).tocsr()
        # mass rows: B_D, or B R P with the reference density (TALA)
        self.rho_nodes = None
        self.B_mass = self.B_D
        if rho_nodes is not None:
            rho_nodes = np.asarray(rho_nodes, np.float64)
            if rho_nodes.shape != (nr + 1,):
                raise ValueError("rho_nodes must hold one value per radial node layer")
            self.rho_nodes = rho_nodes
            R = sp.diags(np.repeat(np.tile(rho_nodes, m.n_lat), 3))
            self.B_mass = (self.B @ R @ Pm).tocsr()
        self.K = sp.bmat([[self.A_D, self.BT_D], [self.B_mass, None]], format="csr")

    # -- products -----------------------------------------------------------
    def apply(self, u: np.ndarray, p: np.ndarray):
        """y = K_D [u; p] with u as [n_nodes, 3] and p as [n_p]."""
        x = np.concatenate([np.asarray(u, np.float64).ravel(), np.asarray(p, np.float64)])
        y = self.K @ x
        return y[:self.n_u].reshape(-1, 3), y[self.n_u:]

    def apply_A(self, u: np.ndarray):
        return (self.A_D @ np.asarray(u, np.float64).ravel()).reshape(-1, 3)

    # -- solve --------------------------------------------------------------
    def solve(self, f: np.ndarray, g: np.ndarray | None = None):
        """Exact discrete solution of K_D [u; p] = [f; g] (Sec. 7 saddle point).

        f's Dirichlet rows hold the prescribed boundary velocity.  One pressure
        DoF is pinned to remove the constant-pressure null space, then the
        pressure is projected to zero nodal mean.
        """
        b = np.concatenate([np.asarray(f, np.float64).ravel(),
                            np.zeros(self.n_p) if g is None else np.asarray(g, np.float64)])
        i0 = self.n_u                       # first pressure DoF
        keep = np.ones(self.K.shape[0])
        keep[i0] = 0.0
        Mk = sp.diags(keep)
        K = (Mk @ self.K @ Mk + sp.diags(1.0 - keep)).tocsc()
        b[i0] = 0.0
        x = spla.splu(K).solve(b)
        u = x[:self.n_u].reshape(-1, 3)
        p = x[self.n_u:]
        return u, p - p.mean()

    def solve_gauged(self, f: np.ndarray, g: np.ndarray | None = None):
        """Exact discrete solution with the pressure gauge fixed by a Lagrange
        multiplier c (Sec. 7 saddle point): A_D u + B_D^T p = f, B_D u - c 1 = g,
        1^T p = 0, i.e. the mass rows modulo constants and a zero-mean pressure.

        With no slip 1^T B_D = 0 and B_D^T 1 = 0, so c = 0 and this is the solution
        of solve().  With free slip the node-normal projection P = I - rhat rhat^T
        keeps the constant pressure in the null space only to O(h^2) (the boundary
        flux of a velocity tangential at the nodes does not vanish on the chordal
        facets): K_D is then non-singular with a pressure mean fixed by that
        discretisation residue, and this gauged problem is the reading the solve
        takes (the no-slip gauge kept).  With free slip on both spheres the velocity
        is also taken orthogonal to the rigid rotations.  Returns (u, p, c).
        """
        nk = self.K.shape[0]
        cols = [np.concatenate([np.zeros(self.n_u), -np.ones(self.n_p)])]
        if self.bc == ("freeslip", "freeslip"):
            # the rigid rotations are a null space of A_D too: the velocity is taken
            # orthogonal to them (R^T u = 0, multipliers lambda; f must be orthogonal
            # to them for lambda = 0)
            for w in self.rotations().T:
                cols.append(np.concatenate([w, np.zeros(self.n_p)]))
        C = sp.csr_matrix(np.stack(cols, axis=1))
        Kb = sp.bmat([[self.K, C], [C.T, None]], format="csc")
        b = np.concatenate([np.asarray(f, np.float64).ravel(),
                            np.zeros(self.n_p) if g is None else np.asarray(g, np.float64), np.zeros(len(cols))])
        x = spla.splu(Kb).solve(b)
        self.last_rotation_multipliers = x[nk + 1:]
        return x[:self.n_u].reshape(-1, 3), x[self.n_u:nk], float(x[nk])

    def rotations(self):
        """The rigid rotations e_a x x at the nodes, as three columns over the
        velocity DoFs ([node][component] order)."""
        x = self.mesh.node_xyz()
        return np.stack([np.cross(np.tile(e, (self.mesh.n_nodes, 1)), x).ravel() for e in np.eye(3)], axis=1)

    def diag_A(self):
        return self.A_D.diagonal().reshape(-1, 3)


def eta_from_temperature(mesh: ShellMesh, T_node: np.ndarray, E: float, F: float = 0.0):
    """Per-wedge viscosity eta_e = exp(-E Tbar_e + F (1 - r_m,e)).

    Tbar_e is the W1 interpolant of T at q_c (mean of the six nodal values) and
    r_m,e the radius of q_c; the exponential law family is the Frank-Kamenetskii
    form of Sec. 8 with a depth factor.
    """
    wn = mesh.wedge_nodes()
    Tbar = T_node[wn].mean(axis=1)
    k = np.tile(np.arange(mesh.nr), len(mesh.tris))
    rm = 0.5 * (mesh.r[k] + mesh.r[k + 1])
    return np.exp(-E * Tbar + F * (1.0 - rm))


def buoyancy_rhs_tala(mesh: ShellMesh, T_node: np.ndarray, Ra: float, Tbar_nodes: np.ndarray,
                      rhoalpha_nodes: np.ndarray):
    """TALA buoyancy of eq:stokes, f = Ra rhobar alphabar T' rhat with T' = T - Tbar(r)
    (eq:tsplit; Tbar the radial reference profile): f_(j,c) = sum_e V_e N_j(q_c) Ra
    (rhobar alphabar)(q_c) T'(q_c) rhat_c(q_c), both factors the W1 interpolants of
    their nodal values (Tbar_nodes, rhoalpha_nodes given per radial node layer).
    Returns [n_nodes, 3]."""
    wn = mesh.wedge_nodes()
    xyz = mesh.node_xyz()
    xw = xyz[wn]
    N, _ = ref_basis(*QC)
    _, V, _ = wedge_geometry(xw)
    xq = np.einsum("j,wja->wa", N, xw)
    rhat = xq / np.linalg.norm(xq, axis=1)[:, None]
    k = np.tile(np.arange(mesh.nr + 1), mesh.n_lat)
    Tp = T_node - np.asarray(Tbar_nodes, np.float64)[k]
    ra = np.asarray(rhoalpha_nodes, np.float64)[k]
    Tq = np.einsum("j,wj->w", N, Tp[wn])
    rq = np.einsum("j,wj->w", N, ra[wn])
    f = np.zeros((mesh.n_nodes, 3))
    np.add.at(f, wn, (V * Ra * Tq * rq)[:, None, None] * N[None, :, None] * rhat[:, None, :])
    return f


def buoyancy_rhs(mesh: ShellMesh, T_node: np.ndarray, Ra: float):
    """f_(j,c) = sum_e V_e N_j(q_c) Ra T(q_c) rhat_c(q_c)  (eq:stokes right-hand side,
    Boussinesq form rho = alpha = 1, one-point rule).  Returns [n_nodes, 3]."""
    wn = mesh.wedge_nodes()
    xyz = mesh.node_xyz()
    xw = xyz[wn]
    N, _ = ref_basis(*QC)
    _, V, _ = wedge_geometry(xw)
    xq = np.einsum("j,wja->wa", N, xw)
    rhat = xq / np.linalg.norm(xq, axis=1)[:, None]
    Tq = np.einsum("j,wj->w", N, T_node[wn])
    f = np.zeros((mesh.n_nodes, 3))
    contrib = (V * Tq * Ra)[:, None, None] * N[None, :, None] * rhat[:, None, :]
    np.add.at(f, wn, contrib)
    return f
