// Per-wedge arithmetic of the one-point W1-iso-W2 / W1 Stokes operator.
//
// Sec. 3 (eq:epsq, eq:localapply) contracts the gathered element DoFs into
// the strain at the quadrature point and tests it against every basis
// gradient; Sec. 4 fixes one point q_c = (1/3, 1/3, 0) of weight 1.  With
// the isoparametric map x = r(zeta) s(xi, eta) the Jacobian at q_c factors as
// J = G diag(r_m, r_m, h) with G = [s1 - s0 | s2 - s0 | s_c], so
//   grad phi_j = (g_j1 / r_m) rho1 + (g_j2 / r_m) rho2 + (g_j3 / h) rho3,
// where rho_m are the rows of G^{-1} and g_j the reference gradients
//   g_0 = (-1/2, -1/2, -1/6), g_1 = (1/2, 0, -1/6), g_2 = (0, 1/2, -1/6),
//   g_3 = (-1/2, -1/2, 1/6),  g_4 = (1/2, 0, 1/6),  g_5 = (0, 1/2, 1/6).
// The constants 1/2 and 1/6 and the radial scalings are folded into the rows
// (rho1~ = rho1 / (2 r_m), rho2~ = rho2 / (2 r_m), rho3' = rho3 / (6 h)), so
// that with the nodal differences
//   A_c = u1 + u4 - u0 - u3,  B_c = u2 + u5 - u0 - u3,  C_c = u3 + u4 + u5 - u0 - u1 - u2
// the velocity gradient is  du_c/dx_a = A_c rho1~_a + B_c rho2~_a + C_c rho3'_a.
// The element result y_j = V_e sigma grad phi_j with
//   sigma = 2 eta dev sym(grad u) - pbar I      (eq:stress, the B^T block),
//   V_e   = |det J(q_c)| = r_m^2 h |det G|      (eq:oneptenergy, w_q = 1),
// reduces to y_j = sum_m g'_jm Z_m with Z_m = (V sigma) rho_m (folded rows)
// and g'_j the reference gradients without their 1/2, 1/6 factors.  The band
// kernel of stokes_apply.hip evaluates these formulas in streaming form; this
// header holds the constants it shares with the other kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace tng {

// Iso-W1 pressure weights (Sec. 3: pressure W1 on the coarser grid).  A fine
// cell (i, j, k) lies in coarse cell (i/2, j/2, k/2); its fine nodes are
// coarse nodes or midpoints of coarse edges, so the pressure at q_c of a fine
// wedge is a fixed combination of the coarse cell's 8 corner values:
//   pbar = sum_lc LW[a][b][w][lc] * (RW[c][0] p(lc, K) + RW[c][1] p(lc, K+1)),
// with a = i&1, b = j&1, c = k&1, w the wedge, lc = e_i + 2 e_j the lateral
// corner of the coarse quad.  The same weights test the divergence against
// the coarse pressure basis (B = P^T B_f), making B and B^T transposes.
template <typename T>
struct IsoWeights {
    T lw[2][2][2][4];   // [a][b][w][lateral corner]
    T rw[2][2];         // [c][bottom/top coarse layer]
};

constexpr void iso_lat_node(int x, int y, double w[4]) {
    // fine node at (x, y) in {0,1,2}^2 inside a coarse quad with corners
    // (0,0)->0, (2,0)->1, (0,2)->2, (2,2)->3 in fine units
    for (int q = 0; q < 4; ++q) w[q] = 0.0;
    if (x % 2 == 0 && y % 2 == 0) {
        w[(x / 2) + 2 * (y / 2)] = 1.0;
    } else if (x == 1 && y % 2 == 0) {
        w[0 + 2 * (y / 2)] = 0.5;
        w[1 + 2 * (y / 2)] = 0.5;
    } else if (y == 1 && x % 2 == 0) {
        w[(x / 2) + 0] = 0.5;
        w[(x / 2) + 2] = 0.5;
    } else {  // (1, 1): midpoint of the coarse split diagonal (2,0)-(0,2)
        w[1] = 0.5;
        w[2] = 0.5;
    }
}

template <typename T>
constexpr IsoWeights<T> make_iso_weights() {
    IsoWeights<T> t{};
    // lateral node offsets of wedge 0 and wedge 1 inside the fine cell
    const int off[2][3][2] = {{{0, 0}, {1, 0}, {0, 1}}, {{1, 1}, {0, 1}, {1, 0}}};
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int w = 0; w < 2; ++w) {
                double acc[4] = {0, 0, 0, 0};
                for (int n = 0; n < 3; ++n) {
                    double nw[4] = {0, 0, 0, 0};
                    iso_lat_node(a + off[w][n][0], b + off[w][n][1], nw);
                    for (int q = 0; q < 4; ++q) acc[q] += nw[q] / 3.0;
                }
                for (int q = 0; q < 4; ++q) t.lw[a][b][w][q] = T(acc[q]);
            }
    // radial: fine layers c and c+1 of the coarse interval, mean of the two
    t.rw[0][0] = T(0.75); t.rw[0][1] = T(0.25);
    t.rw[1][0] = T(0.25); t.rw[1][1] = T(0.75);
    return t;
}

}  // namespace tng
