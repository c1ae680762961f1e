"""Pins of the oracle's one-point element matrix (Sec. 3 eq:elemmat, Sec. 4)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.mesh import ShellMesh
from oracle.stokes import QC, element_divergence, element_matrices, hourglass_vectors, ref_basis, wedge_geometry

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _mesh_wedges(n=8, mt=4, nr=4, seed=3):
    m = ShellMesh(mt, nr)
    rng = np.random.default_rng(seed)
    pick = rng.choice(m.n_wedges, n, replace=False)
    return m.node_xyz()[m.wedge_nodes()[pick]]


def _hourglass():
    out = {}
    with open(os.path.join(GOLDEN, "hourglass_modes.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, *vals = line.split()
            out[name] = np.array([float(Fraction(v)) for v in vals])
    return out


def test_reference_basis_partition_of_unity_and_nodality():
    """eq:wedgebasis: N_j(node_i) = delta_ij, sum_j N_j = 1, gradients sum to 0."""
    nodes = [(0, 0, -1), (1, 0, -1), (0, 1, -1), (0, 0, 1), (1, 0, 1), (0, 1, 1)]
    for i, p in enumerate(nodes):
        N, _ = ref_basis(*p)
        assert np.allclose(N, np.eye(6)[i])
    N, dN = ref_basis(*QC)
    assert np.allclose(N, 1.0 / 6.0)
    assert np.allclose(dN.sum(axis=0), 0.0)
    # reference gradients at q_c from the product rule
    want = np.array([[-.5, -.5, -1 / 6], [.5, 0, -1 / 6], [0, .5, -1 / 6],
                     [-.5, -.5, 1 / 6], [.5, 0, 1 / 6], [0, .5, 1 / 6]])
    assert np.allclose(dN, want)


def test_rank_and_null_space():
    """Sec. 4: 18x18 one-point matrix has rank 5 -> 13 zero modes
    (3 translations + 6 hourglass + 3 rotations + 1 dilation); A_e is PSD."""
    xw = _mesh_wedges()
    A = element_matrices(xw, np.full(len(xw), 2.5))
    for a in A:
        ev = np.linalg.eigvalsh(a)
        assert ev.min() > -1e-12 * ev.max()
        assert np.sum(ev > 1e-10 * ev.max()) == 5
        assert np.allclose(a, a.T, atol=1e-14 * np.abs(a).max())


def test_hourglass_modes_are_zero_energy():
    """eq:hourglass: w_m (x) e_d lies in the null space for m = 1, 2 and d = 1..3."""
    hg = _hourglass()
    xw = _mesh_wedges()
    A = element_matrices(xw, np.ones(len(xw)))
    for a in A:
        for w in hg.values():
            for d in range(3):
                v = np.zeros(18)
                v[d::3] = w
                assert np.abs(a @ v).max() < 1e-13 * np.abs(a).max()
    # the six modes are independent
    V = np.zeros((18, 6))
    for i, w in enumerate(hg.values()):
        for d in range(3):
            V[d::3, 3 * i + d] = w
    assert np.linalg.matrix_rank(V) == 6


def test_rigid_and_dilation_modes():
    """Translations, rotations and the dilation x have zero one-point energy
    (2 eps:eps - 2/3 (div)^2 = 2 |dev eps|^2)."""
    xw = _mesh_wedges()
    A = element_matrices(xw, np.ones(len(xw)))
    for a, x in zip(A, xw):
        modes = [np.tile(e, 6) for e in np.eye(3)]
        for w in np.eye(3):
            modes.append(np.cross(w, x).ravel())
        modes.append(x.ravel())
        for v in modes:
            assert np.abs(a @ v).max() < 1e-13 * np.abs(a).max() * np.abs(v).max()


def _energy_fd(x6, u6, eta, h=1e-6):
    """Brute-force one-point energy: gradients of the interpolated field and of
    the map by central differences in reference coordinates at q_c."""
    def interp(vals, p):
        N, _ = ref_basis(*p)
        return N @ vals
    Jc = np.zeros((3, 3))
    Gu = np.zeros((3, 3))
    for m in range(3):
        e = np.zeros(3); e[m] = h
        p1, p0 = np.add(QC, e), np.subtract(QC, e)
        Jc[:, m] = (interp(x6, p1) - interp(x6, p0)) / (2 * h)
        Gu[:, m] = (interp(u6, p1) - interp(u6, p0)) / (2 * h)
    L = Gu @ np.linalg.inv(Jc)              # du_c / dx_a
    eps = 0.5 * (L + L.T)
    V = abs(np.linalg.det(Jc))
    return V * eta * (2 * np.sum(eps * eps) - 2.0 / 3.0 * np.trace(L) ** 2)


def test_element_matrix_against_finite_differences():
    """(A_e)_ab by polarisation of the brute-force energy E_e (eq:oneptenergy)."""
    xw = _mesh_wedges(n=2)
    A = element_matrices(xw, np.array([1.3, 0.7]))
    for a, x, eta in zip(A, xw, (1.3, 0.7)):
        E = lambda v: _energy_fd(x, v.reshape(6, 3), eta)
        B = np.zeros((18, 18))
        I = np.eye(18)
        e1 = [E(I[i]) for i in range(18)]
        for i in range(18):
            for j in range(i, 18):
                B[i, j] = B[j, i] = 0.5 * (E(I[i] + I[j]) - e1[i] - e1[j])
        assert np.abs(B - a).max() < 1e-6 * np.abs(a).max()


def _gauss_wedge(n=4):
    """Gauss rule on the reference wedge: collapsed-square triangle rule x Gauss-Legendre."""
    g, w = np.polynomial.legendre.leggauss(n)
    pts, wts = [], []
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            u = 0.5 * (1 + a)
            v = 0.5 * (1 + b) * (1 - u)
            jac = 0.25 * (1 - u)
            for c, wc in zip(g, w):
                pts.append((u, v, c))
                wts.append(wa * wb * wc * jac)
    return np.array(pts), np.array(wts)


def test_one_point_rule_exact_for_linear_fields_on_affine_wedge():
    """Sec. 4: the centroid rule integrates constants and linears exactly.  On an
    affine wedge, linear velocity fields have constant gradients, so
    v^T A_e u equals the exact integral of eta [2 eps(u):eps(v) - 2/3 div u div v]."""
    rng = np.random.default_rng(5)
    base = rng.standard_normal((3, 3))
    top = base + np.array([0.1, 0.2, 1.0])              # translated copy: affine prism
    x6 = np.vstack([base, top])
    A = element_matrices(x6[None], np.array([2.0]))[0]
    pts, wts = _gauss_wedge()
    vol = 0.0
    for p, w in zip(pts, wts):
        _, dN = ref_basis(*p)
        vol += w * abs(np.linalg.det(x6.T @ dN))
    assert vol == pytest.approx(wedge_geometry(x6[None])[1][0], rel=1e-13)
    for _ in range(3):
        Gu, Gv = rng.standard_normal((3, 3)), rng.standard_normal((3, 3))
        u = (x6 @ Gu.T).ravel()
        v = (x6 @ Gv.T).ravel()
        eu, ev = 0.5 * (Gu + Gu.T), 0.5 * (Gv + Gv.T)
        exact = 2.0 * vol * (2 * np.sum(eu * ev) - 2.0 / 3.0 * np.trace(Gu) * np.trace(Gv))
        assert v @ A @ u == pytest.approx(exact, rel=1e-12)


def test_divergence_form_matches_trace_of_gradient():
    """B_f of one wedge applied to a linear field gives -V/6 div u at each node."""
    xw = _mesh_wedges(n=3)
    Bf = element_divergence(xw)
    _, V, _ = wedge_geometry(xw)
    rng = np.random.default_rng(9)
    G = rng.standard_normal((3, 3))
    for b, x, v in zip(Bf, xw, V):
        u = (x @ G.T).ravel()
        assert np.allclose(b @ u, -v / 6.0 * np.trace(G), rtol=1e-12)


def test_two_wedge_hex_symmetric_psd():
    """The two wedges of one hexahedron (8 nodes) assembled into a 24x24 matrix."""
    m = ShellMesh(2, 2)
    xyz = m.node_xyz()
    wn = m.wedge_nodes()
    # wedges sharing a lateral edge and the same layer form a hexahedron
    t = m.tris
    e0 = set(t[0])
    j = next(i for i in range(1, len(t)) if len(e0 & set(t[i])) == 2)
    w0, w1 = 0 * m.nr, j * m.nr
    nodes = np.unique(np.concatenate([wn[w0], wn[w1]]))
    assert len(nodes) == 8
    K = np.zeros((24, 24))
    for w in (w0, w1):
        a = element_matrices(xyz[wn[w]][None], np.ones(1))[0]
        loc = np.searchsorted(nodes, wn[w])
        dof = (loc[:, None] * 3 + np.arange(3)).ravel()
        K[np.ix_(dof, dof)] += a
    ev = np.linalg.eigvalsh(K)
    assert np.allclose(K, K.T)
    assert ev.min() > -1e-12 * ev.max()


# ---- hourglass control (eq:hgstab) ------------------------------------------------

def _hg_vec(h, d):
    v = np.zeros(18)
    v[d::3] = h
    return v


def test_hourglass_vectors_match_eq_hourglass():
    """h_1, h_2 are the nodal values of w_1, w_2 (golden file); h_0 = -h_1 - h_2."""
    from oracle.stokes import hourglass_vectors
    hg = _hourglass()
    h = hourglass_vectors()
    w = list(hg.values())
    assert np.allclose(h[1], w[0]) and np.allclose(h[2], w[1])
    assert np.allclose(h.sum(axis=0), 0.0)


def test_hourglass_control_lifts_exactly_the_hourglass_modes():
    """A_e^stab = A_e + eps H: the six hourglass modes become eigenvectors with
    eigenvalue 2 eps (H h_a = 2 h_a, from h_a . h_b = 2 (delta_ab - 1/3) and
    sum_a h_a = 0), with eps = alpha mean(diag A_e); translations stay in the
    null space.  On a curved wedge (x = r(zeta) s(xi, eta) has xi zeta and
    eta zeta parts) rotations and the dilation carry hourglass components, so
    what stays null is their part orthogonal to the hourglass span: the null
    space keeps dimension 7 and the rank goes from 5 to 11."""
    from oracle.stokes import element_matrices_hg, hourglass_vectors
    xw = _mesh_wedges()
    eta = np.linspace(0.5, 3.0, len(xw))
    alpha = 0.05
    A0 = element_matrices(xw, eta)
    A1 = element_matrices_hg(xw, eta, alpha)
    h = hourglass_vectors()
    for a0, a1, x in zip(A0, A1, xw):
        eps = alpha * np.trace(a0) / 18.0
        for a in range(3):
            for d in range(3):
                v = _hg_vec(h[a], d)
                assert np.abs(a1 @ v - 2 * eps * v).max() < 1e-13 * np.abs(a1).max()
        W = np.stack([_hg_vec(h[a], d) for a in range(3) for d in range(3)], axis=1)
        Q, _ = np.linalg.qr(W)
        Q = Q[:, :6]                                      # orthonormal basis of the hourglass span
        modes = [np.tile(e, 6) for e in np.eye(3)]
        modes += [(v - Q @ (Q.T @ v)) for v in [np.cross(wv, x).ravel() for wv in np.eye(3)] + [x.ravel()]]
        for v in modes:
            assert np.abs(a1 @ v).max() < 1e-12 * np.abs(a1).max() * np.abs(v).max()
        ev = np.linalg.eigvalsh(a1)
        assert ev.min() > -1e-12 * ev.max()
        assert np.sum(ev > 1e-10 * ev.max()) == 11
        assert np.allclose(a1, a1.T, atol=1e-14 * np.abs(a1).max())


def test_hourglass_control_independent_of_vertex_numbering():
    """Renumbering the lateral vertices of a wedge (cyclically or by a swap, the
    same on both faces) permutes A_e^stab accordingly: the term does not depend
    on which vertex a wedge calls 0."""
    from oracle.stokes import element_matrices_hg
    xw = _mesh_wedges(n=4)
    eta = np.full(len(xw), 1.7)
    for perm in ((1, 2, 0), (0, 2, 1), (2, 1, 0)):
        node = list(perm) + [p + 3 for p in perm]
        dof = np.array([3 * j + c for j in node for c in range(3)])
        A = element_matrices_hg(xw, eta, 0.08)
        B = element_matrices_hg(xw[:, node, :], eta, 0.08)
        for a, b in zip(A, B):
            assert np.abs(a[np.ix_(dof, dof)] - b).max() < 1e-13 * np.abs(a).max()


# ---- two-radial-point rule (Sec. 4, the remedy beside eq:hgstab) --------------------------

def _basis_and_map(xs):
    def N(xi, et, ze):
        lat = (1.0 - xi - et, xi, et)
        rad = (0.5 * (1.0 - ze), 0.5 * (1.0 + ze))
        return np.array([lat[j % 3] * rad[j // 3] for j in range(6)])
    return N, (lambda pt: N(*pt) @ xs)


def test_two_point_element_matrix_equals_brute_force_quadrature():
    """A_e = sum over the points (1/3, 1/3, -+1/sqrt 3), weight 1/2, of V(q) eta
    [2 eps:eps - 2/3 div div](q), every quantity from the wedge's own map and basis
    by central differences (exact for the map's quadratic terms), in plain loops."""
    from oracle.stokes import element_matrices_2pt
    m = ShellMesh(2, 2)
    wn = m.wedge_nodes()
    xyz = m.node_xyz()
    for w in (0, 7, 33):
        xs = xyz[wn[w]]
        N, x_of = _basis_and_map(xs)
        A = np.zeros((18, 18))
        h = 1e-3
        for zq in (-1.0 / np.sqrt(3.0), 1.0 / np.sqrt(3.0)):
            q = np.array([1.0 / 3.0, 1.0 / 3.0, zq])
            J = np.empty((3, 3))
            dN = np.empty((6, 3))
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                J[:, a] = (x_of(q + e) - x_of(q - e)) / (2 * h)
                dN[:, a] = (N(*(q + e)) - N(*(q - e))) / (2 * h)
            grads = dN @ np.linalg.inv(J)                   # rows: grad phi_j
            V = 0.5 * abs(np.linalg.det(J))
            for i in range(18):
                for k in range(18):
                    ji, ci, jk, ck = i // 3, i % 3, k // 3, k % 3
                    Gi = np.zeros((3, 3))
                    Gi[ci] = grads[ji]
                    Gk = np.zeros((3, 3))
                    Gk[ck] = grads[jk]
                    ei, ek = 0.5 * (Gi + Gi.T), 0.5 * (Gk + Gk.T)
                    A[i, k] += V * 1.7 * (2.0 * np.sum(ei * ek) - (2.0 / 3.0) * np.trace(Gi) * np.trace(Gk))
        got = element_matrices_2pt(xs[None], np.array([1.7]))[0]
        assert np.abs(got - A).max() < 1e-9 * np.abs(A).max()


def test_two_point_rule_controls_the_hourglass_modes():
    """With two radial points the element energy sees the hourglass modes.  The energy is
    2 |dev eps|^2 at two points: 10 conditions on 18 DoFs, so the null space has dimension
    8 -- the translations, rotations and the dilation, plus one volumetric mode (deviatoric
    strain zero at both points, its volume change left to the divergence block) -- and every
    hourglass mode w_m (x) e_d has energy."""
    from oracle.stokes import element_matrices_2pt
    m = ShellMesh(2, 2)
    xs = m.node_xyz()[m.wedge_nodes()[5]]
    A = element_matrices_2pt(xs[None], np.array([1.0]))[0]
    lam, vec = np.linalg.eigh(A)
    assert np.sum(lam < 1e-10 * lam.max()) == 8 and lam.min() > -1e-12 * lam.max()
    # rigid motions and the dilation x are in the null space
    rigid = [np.tile(e, 6) for e in np.eye(3)]
    rigid += [np.cross(np.tile(w, (6, 1)), xs).ravel() for w in np.eye(3)] + [xs.ravel()]
    for v in rigid:
        assert np.abs(A @ v).max() < 1e-12 * lam.max() * np.abs(v).max()
    h = hourglass_vectors()
    for a in range(3):
        for d in range(3):
            v = np.zeros(18)
            v[d::3] = h[a]
            assert v @ A @ v > 1e-3 * lam.max() * (v @ v)
