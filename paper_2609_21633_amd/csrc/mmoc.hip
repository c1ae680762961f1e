// Modified method of characteristics for the temperature (Sec. 6:
// eq:characteristic, eq:departure, eq:mmoc): departure points by the explicit
// midpoint rule backwards along the velocity, and the old temperature
// interpolated there (W1).  One thread per node slot, FP64.
//
// Point location.  A wedge is the set {lam s : s in the flat triangle of its
// three lateral unit vectors, lam in [r_k, r_k+1]} (the isoparametric map
// x = r(zeta) s(xi, eta)), so a point x = a s0 + b s1 + c s2 (Cramer's rule)
// lies over the triangle when a, b, c >= 0, with lam = a + b + c and
// (xi, eta) = (b, c) / lam.  The lateral grid is the recursive midpoint
// refinement of the 20 icosahedron faces (two per diamond), and the child
// triangles of a triangle cover exactly its cone (their outer edges lie on
// the parent's great circles), so the triangle is found by testing the 20
// faces and then descending one refinement level at a time into the child
// (of four) with the largest min(a, b, c).  In a diamond's index space a
// triangle of level size S at origin (i0, j0) is
//   type 0: (i0, j0), (i0+S, j0), (i0, j0+S);  type 1: (i0+S, j0+S), (i0, j0+S), (i0+S, j0)
// and the coarse nodes are the fine nodes at multiples of S, so the finest
// level's unit vectors serve every level.
#include <cmath>

#include "mg.hpp"
#include "tng_internal.hpp"

namespace tng {
namespace {

struct LocGeo {
    const double* unit;   // [10][m+1][m+1][3]
    int m, n;
    double r_in, r_out, dr;
};

__device__ __forceinline__ const double* unit_at(const LocGeo& G, int d, int i, int j) {
    return G.unit + (((long long)d * (G.m + 1) + i) * (G.m + 1) + j) * 3;
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// (a, b, c) of x over the triangle (d, i0, j0, S, w); returns min(a, b, c) / lam, or
// -inf when the triangle lies on the far side (lam <= 0: all three coefficients can then
// be negative, and their quotient by lam positive)
__device__ double bary(const LocGeo& G, const double x[3], int d, int i0, int j0, int S, int w, double abc[3]) {
    const double* s0 = w == 0 ? unit_at(G, d, i0, j0) : unit_at(G, d, i0 + S, j0 + S);
    const double* s1 = w == 0 ? unit_at(G, d, i0 + S, j0) : unit_at(G, d, i0, j0 + S);
    const double* s2 = w == 0 ? unit_at(G, d, i0, j0 + S) : unit_at(G, d, i0 + S, j0);
    double c12[3], c20[3], c01[3];
    cross3(s1, s2, c12);
    cross3(s2, s0, c20);
    cross3(s0, s1, c01);
    const double D = s0[0] * c12[0] + s0[1] * c12[1] + s0[2] * c12[2];
    abc[0] = (x[0] * c12[0] + x[1] * c12[1] + x[2] * c12[2]) / D;
    abc[1] = (x[0] * c20[0] + x[1] * c20[1] + x[2] * c20[2]) / D;
    abc[2] = (x[0] * c01[0] + x[1] * c01[1] + x[2] * c01[2]) / D;
    const double lam = abc[0] + abc[1] + abc[2];
    return lam > 0.0 ? fmin(fmin(abc[0], abc[1]), abc[2]) / lam : -1e300;
}

struct Loc {
    int d, ci, cj, w, k;
    double xi, eta, zeta;
};

__device__ Loc locate(const LocGeo& G, const double x[3]) {
    const int m = G.m;
    // the 20 icosahedron faces: the two triangles of each diamond's single coarsest cell
    int bd = 0, bw = 0;
    double best = -1e300, abc[3];
    for (int d = 0; d < 10; ++d)
        for (int w = 0; w < 2; ++w) {
            const double sc = bary(G, x, d, 0, 0, m, w, abc);
            if (sc > best) {
                best = sc;
                bd = d;
                bw = w;
            }
        }
    int i0 = 0, j0 = 0, w = bw;
    for (int S = m; S > 1; S >>= 1) {
        const int h = S >> 1;
        // children (origin offsets in units of h, type)
        int ci[4], cj[4], cw[4];
        if (w == 0) {
            ci[0] = i0;     cj[0] = j0;     cw[0] = 0;
            ci[1] = i0 + h; cj[1] = j0;     cw[1] = 0;
            ci[2] = i0;     cj[2] = j0 + h; cw[2] = 0;
            ci[3] = i0;     cj[3] = j0;     cw[3] = 1;
        } else {
            ci[0] = i0 + h; cj[0] = j0 + h; cw[0] = 1;
            ci[1] = i0;     cj[1] = j0 + h; cw[1] = 1;
            ci[2] = i0 + h; cj[2] = j0;     cw[2] = 1;
            ci[3] = i0 + h; cj[3] = j0 + h; cw[3] = 0;
        }
        double bs = -1e300;
        int bc = 0;
        for (int c = 0; c < 4; ++c) {
            const double sc = bary(G, x, bd, ci[c], cj[c], h, cw[c], abc);
            if (sc > bs) {
                bs = sc;
                bc = c;
            }
        }
        i0 = ci[bc];
        j0 = cj[bc];
        w = cw[bc];
    }
    bary(G, x, bd, i0, j0, 1, w, abc);
    double lam = abc[0] + abc[1] + abc[2];
    Loc L;
    L.d = bd;
    L.ci = i0;
    L.cj = j0;
    L.w = w;
    L.xi = abc[1] / lam;
    L.eta = abc[2] / lam;
    // a point outside the shell is brought back radially onto it
    lam = fmin(fmax(lam, G.r_in), G.r_out);
    int k = (int)floor((lam - G.r_in) / G.dr);
    k = k < 0 ? 0 : (k > G.n - 1 ? G.n - 1 : k);
    L.k = k;
    L.zeta = 2.0 * (lam - (G.r_in + k * G.dr)) / G.dr - 1.0;
    return L;
}

// lateral offsets of the three nodes of a type-0 / type-1 cell triangle
__constant__ int c_mi[2][3] = {{0, 1, 0}, {1, 0, 1}};
__constant__ int c_mj[2][3] = {{0, 0, 1}, {1, 1, 0}};

// W1 interpolant of node field f at a located point
__device__ double interp(const LocGeo& G, const Loc& L, const double* __restrict__ f) {
    const double lat[3] = {1.0 - L.xi - L.eta, L.xi, L.eta};
    const double rad[2] = {0.5 * (1.0 - L.zeta), 0.5 * (1.0 + L.zeta)};
    double v = 0.0;
    for (int a = 0; a < 3; ++a) {
        const long long s = (((long long)L.d * (G.m + 1) + L.ci + c_mi[L.w][a]) * (G.m + 1) + L.cj + c_mj[L.w][a]) *
                            (G.n + 1) + L.k;
        v += lat[a] * (rad[0] * f[s] + rad[1] * f[s + 1]);
    }
    return v;
}

__global__ void mmoc_departure_kernel(LocGeo G, const double* __restrict__ u0, const double* __restrict__ u1,
                                      const double* __restrict__ u2, const double* __restrict__ Tn, double dt,
                                      double* __restrict__ That, long long nslots) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const int n = G.n, m = G.m;
    const int k = (int)(t % (n + 1));
    long long r = t / (n + 1);
    const int j = (int)(r % (m + 1));
    r /= (m + 1);
    const int i = (int)(r % (m + 1));
    const int d = (int)(r / (m + 1));
    const double rk = G.r_in + k * G.dr;
    const double* s = unit_at(G, d, i, j);
    const double x[3] = {rk * s[0], rk * s[1], rk * s[2]};
    // explicit midpoint rule backwards over dt (eq:departure)
    const double xm[3] = {x[0] - 0.5 * dt * u0[t], x[1] - 0.5 * dt * u1[t], x[2] - 0.5 * dt * u2[t]};
    const Loc Lm = locate(G, xm);
    const double um[3] = {interp(G, Lm, u0), interp(G, Lm, u1), interp(G, Lm, u2)};
    const double xh[3] = {x[0] - dt * um[0], x[1] - dt * um[1], x[2] - dt * um[2]};
    That[t] = interp(G, locate(G, xh), Tn);
}

}  // namespace

void mmoc_departure(const tng_ctx* ctx, const Level& L, const double* const u[3], double dt, const double* Tn,
                    double* That) {
    LocGeo G{L.unit64.p, L.m, L.n, L.r_in, L.r_out, L.dr()};
    const long long ns = L.node_slots();
    ScopedKernelTimer timer(ctx, "mmoc_departure");
    mmoc_departure_kernel<<<(unsigned)((ns + 127) / 128), 128, 0, ctx->stream>>>(G, u[0], u[1], u[2], Tn, dt, That,
                                                                                 ns);
    TNG_HIP(hipGetLastError());
    // copies of a duplicate node computed the same value up to rounding of their own
    // coordinates: make them equal
    void* f[1] = {That};
    launch_interface(ctx, L, TNG_F64, 1, 1, f);
}

}  // namespace tng
