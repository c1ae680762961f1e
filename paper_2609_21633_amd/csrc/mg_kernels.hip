// Multigrid and Krylov building blocks (Sec. 7): operator diagonal, lumped
// inverse-viscosity pressure mass, W1 transfer operators, Chebyshev update,
// BLAS-1 with deterministic reductions, precision casts, and the dense
// coarsest-level solve.
//
// All velocity vectors are in the duplicated-diamond layout with equal values
// in every copy of a shared node.  Gathers that run per diamond produce
// partial sums on diamond-edge nodes; the interface kernel then adds the
// copies.  Reductions count every unique node once (owner mask).
#include "batch_dev.hpp"
#include "tng_internal.hpp"
#include "mg.hpp"
#include "wedge.hpp"

namespace tng {
namespace {

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// per-slot vector counts of a batched multi-dot / multi-axpy stay in range
inline void check_counts(const SlotBatch& sb) {
    if (!sb.has_cnt) return;
    for (int z = 0; z < sb.nb; ++z)
        TNG_REQUIRE(sb.cnt[z] >= 1 && sb.cnt[z] <= MAX_MDOT, "per-slot vector count out of range");
}

__constant__ IsoWeights<double> c_isomg = make_iso_weights<double>();

struct NodeIdx {
    int d, i, j, k;
};
__device__ __forceinline__ NodeIdx decode_node(long long t, int m, int n) {
    NodeIdx r;
    r.k = (int)(t % (n + 1));
    t /= (n + 1);
    r.j = (int)(t % (m + 1));
    t /= (m + 1);
    r.i = (int)(t % (m + 1));
    r.d = (int)(t / (m + 1));
    return r;
}

// Gradient of the wedge basis function of local node (lat, top) at q_c, with
// the constants folded as in wedge.hpp: sign pattern of the reference gradient
// times the folded rows of G^{-1}.
__device__ __forceinline__ void basis_grad(const double* g, double s1, int lat, int top, double out[3]) {
    const double a = lat == 0 ? -1.0 : (lat == 1 ? 1.0 : 0.0);
    const double b = lat == 0 ? -1.0 : (lat == 2 ? 1.0 : 0.0);
    const double c = top ? 1.0 : -1.0;
    for (int x = 0; x < 3; ++x) out[x] = a * s1 * g[x] + b * s1 * g[3 + x] + c * g[6 + x];
}

// Two-radial-point rule (Sec. 4): points zeta = -+1/sqrt 3 on the lateral centroid,
// weight 1/2 each.  There the Jacobian is G diag(r_q, r_q, dr/2) with r_q = r_m +
// zeta dr/2, so the lateral part of a basis gradient carries 1/r_q and the radial
// shape factor (1 + zeta) on the top face, (1 - zeta) on the bottom face; the
// radial part is the one of q_c.  s1q = 1/(2 r_q).
constexpr double TWOPT_ZETA = 0.57735026918962576451;
__device__ __forceinline__ void basis_grad_at(const double* g, double s1q, double zq, int lat, int top,
                                              double out[3]) {
    const double a = lat == 0 ? -1.0 : (lat == 1 ? 1.0 : 0.0);
    const double b = lat == 0 ? -1.0 : (lat == 2 ? 1.0 : 0.0);
    const double c = top ? 1.0 : -1.0;
    const double f = top ? 1.0 + zq : 1.0 - zq;
    for (int x = 0; x < 3; ++x) out[x] = f * (a * s1q * g[x] + b * s1q * g[3 + x]) + c * g[6 + x];
}

// Hourglass-control scale of a wedge (eq:hgstab over the three barycentric
// modes): eps_e = alpha mean(diag A_e) = alpha 5/27 eta V sum_j |grad phi_j|^2,
// sum_j |grad phi_j|^2 = 4 (|rho1~|^2 + |rho2~|^2 + rho1~.rho2~) + 6 |rho3'|^2.
__device__ __forceinline__ double hg_eps(const double* g, double s1, double V, double e, double alpha) {
    const double a = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3] + g[4] * g[4] + g[5] * g[5] +
                     g[0] * g[3] + g[1] * g[4] + g[2] * g[5];
    const double b = g[6] * g[6] + g[7] * g[7] + g[8] * g[8];
    return alpha * (5.0 / 27.0) * e * V * (4.0 * s1 * s1 * a + 6.0 * b);
}

// diag(A)_(node,c) = sum over the node's wedges of V eta (|grad phi|^2 + 1/3 (d_c phi)^2),
// the diagonal of eq:elemmat with the one-point rule, plus 2/3 eps_e with hourglass
// control (sum_a h_a[j]^2 = 2/3 for every node); twopt: the same sum over the two
// radial points, each with V_q = r_q^2 |det G| / 2.  On a free-slip sphere (fs bit 0
// inner, bit 1 outer) the row block is P A_jj P + N with P = I - rhat rhat^T: its two
// tangential diagonal entries are replaced by their mean, the same value in all three
// components, so that D^{-1} maps tangential vectors to tangential vectors:
// trace(P A_jj P) / 2 = sum_e V eta (|grad phi|^2 + (|grad phi|^2 - (rhat.grad phi)^2) / 6).
// Per-diamond partial sums.
template <typename T>
__global__ void diag_A_kernel(const T* __restrict__ eta, const double* __restrict__ geo, int m, int n,
                              double r_in, double dr, double hg_alpha, int twopt, int fs,
                              const double* __restrict__ unit, T* d0, T* d1, T* d2, long long nslots) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const NodeIdx q = decode_node(t, m, n);
    const bool proj = ((fs & 1) && q.k == 0) || ((fs & 2) && q.k == n);
    const double* rh = unit + 3 * ((((long long)q.d * (m + 1) + q.i) * (m + 1)) + q.j);
    double acc[3] = {0, 0, 0};
    for (int ci = q.i - 1; ci <= q.i; ++ci) {
        if (ci < 0 || ci >= m) continue;
        for (int cj = q.j - 1; cj <= q.j; ++cj) {
            if (cj < 0 || cj >= m) continue;
            const int di = q.i - ci, dj = q.j - cj;
            const double* gcol = geo + (((long long)q.d * m + ci) * m + cj) * GEO_PER_COL;
            for (int ck = q.k - 1; ck <= q.k; ++ck) {
                if (ck < 0 || ck >= n) continue;
                const int top = q.k - ck;
                const double rm = r_in + (ck + 0.5) * dr;
                const double s1 = 0.5 / rm;
                for (int wd = 0; wd < 2; ++wd) {
                    // local lateral index of the node in this wedge, -1 if not a vertex
                    int lat = -1;
                    if (wd == 0) lat = (di == 0 && dj == 0) ? 0 : (di == 1 && dj == 0) ? 1 : (di == 0 && dj == 1) ? 2 : -1;
                    else lat = (di == 1 && dj == 1) ? 0 : (di == 0 && dj == 1) ? 1 : (di == 1 && dj == 0) ? 2 : -1;
                    if (lat < 0) continue;
                    const double* g = gcol + wd * GEO_PER_TRI;
                    double gr[3];
                    const double e = (double)eta[((((long long)q.d * m + ci) * m + cj) * n + ck) * 2 + wd];
                    if (twopt) {
                        for (int qq = 0; qq < 2; ++qq) {
                            const double zq = qq == 0 ? -TWOPT_ZETA : TWOPT_ZETA;
                            const double rq = rm + zq * (0.5 * dr);
                            basis_grad_at(g, 0.5 / rq, zq, lat, top, gr);
                            const double Vq = 0.5 * rq * rq * g[9];
                            const double nn = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
                            for (int c = 0; c < 3; ++c) acc[c] += Vq * e * (nn + gr[c] * gr[c] / 3.0);
                        }
                        continue;
                    }
                    basis_grad(g, s1, lat, top, gr);
                    const double V = rm * rm * g[9];
                    const double nn = gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2];
                    if (proj) {
                        const double gn = rh[0] * gr[0] + rh[1] * gr[1] + rh[2] * gr[2];
                        const double v = V * e * (nn + (nn - gn * gn) / 6.0);
                        for (int c = 0; c < 3; ++c) acc[c] += v;
                        continue;
                    }
                    const double hg = hg_alpha != 0.0 ? (2.0 / 3.0) * hg_eps(g, s1, V, e, hg_alpha) : 0.0;
                    for (int c = 0; c < 3; ++c) acc[c] += V * e * (nn + gr[c] * gr[c] / 3.0) + hg;
                }
            }
        }
    }
    d0[t] = T(acc[0]);
    d1[t] = T(acc[1]);
    d2[t] = T(acc[2]);
}

// Lumped M_{1/eta} on the pressure level: m_I = sum_e (V_e / eta_e) psi_I(q_c^e)
// (eq:pmass, row-sum lumping, one-point rule), gathered per coarse node.
template <typename T>
__global__ void pmass_kernel(const T* __restrict__ eta, const double* __restrict__ geo, int m, int n,
                             double r_in, double dr, T* __restrict__ out, long long ncslots) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncslots) return;
    const int mc = m / 2, nc = n / 2;
    const NodeIdx q = decode_node(t, mc, nc);
    double acc = 0.0;
    for (int Ic = q.i - 1; Ic <= q.i; ++Ic) {
        if (Ic < 0 || Ic >= mc) continue;
        for (int Jc = q.j - 1; Jc <= q.j; ++Jc) {
            if (Jc < 0 || Jc >= mc) continue;
            const int lc = (q.i - Ic) + 2 * (q.j - Jc);
            for (int Kc = q.k - 1; Kc <= q.k; ++Kc) {
                if (Kc < 0 || Kc >= nc) continue;
                const int rc = q.k - Kc;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        const int ci = 2 * Ic + a, cj = 2 * Jc + b;
                        const double* gcol = geo + (((long long)q.d * m + ci) * m + cj) * GEO_PER_COL;
                        for (int c = 0; c < 2; ++c) {
                            const int ck = 2 * Kc + c;
                            const double rm = r_in + (ck + 0.5) * dr;
                            const double rw = c_isomg.rw[c][rc];
                            for (int wd = 0; wd < 2; ++wd) {
                                const double V = rm * rm * gcol[wd * GEO_PER_TRI + 9];
                                const double e = (double)eta[((((long long)q.d * m + ci) * m + cj) * n + ck) * 2 + wd];
                                acc += V / e * c_isomg.lw[a][b][wd][lc] * rw;
                            }
                        }
                    }
            }
        }
    }
    out[t] = T(acc);
}

// Prolongation (W1 interpolation in index space): a fine node that is a
// coarse node copies it, one on a coarse edge takes the mean of the edge's
// end nodes (edges along i, along j, or the split diagonal), radially odd
// layers take the mean of the two coarse layers.  y += P x (add) or y = P x.
template <typename T>
__global__ void prolong_kernel(int mf, int nf, const T* __restrict__ c0, const T* __restrict__ c1,
                               const T* __restrict__ c2, T* f0, T* f1, T* f2, int add, long long nslots,
                               SlotBatch sb) {
    const long long so = slot_off(sb);
    c0 = at_slot(c0, so);
    c1 = at_slot(c1, so);
    c2 = at_slot(c2, so);
    f0 = at_slot(f0, so);
    f1 = at_slot(f1, so);
    f2 = at_slot(f2, so);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const NodeIdx q = decode_node(t, mf, nf);
    const int mc = mf / 2, nc = nf / 2;
    int li[2], lj[2], nl;
    if ((q.i & 1) == 0 && (q.j & 1) == 0) { li[0] = q.i / 2; lj[0] = q.j / 2; nl = 1; }
    else if ((q.i & 1) && (q.j & 1) == 0) { li[0] = q.i / 2; lj[0] = q.j / 2; li[1] = q.i / 2 + 1; lj[1] = q.j / 2; nl = 2; }
    else if ((q.i & 1) == 0 && (q.j & 1)) { li[0] = q.i / 2; lj[0] = q.j / 2; li[1] = q.i / 2; lj[1] = q.j / 2 + 1; nl = 2; }
    else { li[0] = q.i / 2; lj[0] = q.j / 2 + 1; li[1] = q.i / 2 + 1; lj[1] = q.j / 2; nl = 2; }
    int kr[2], nk;
    if ((q.k & 1) == 0) { kr[0] = q.k / 2; nk = 1; } else { kr[0] = q.k / 2; kr[1] = q.k / 2 + 1; nk = 2; }
    const T wl = nl == 1 ? T(1) : T(0.5), wk = nk == 1 ? T(1) : T(0.5);
    T s[3] = {0, 0, 0};
    const T* cs[3] = {c0, c1, c2};
    for (int a = 0; a < nl; ++a)
        for (int b = 0; b < nk; ++b) {
            const long long ci = (((long long)q.d * (mc + 1) + li[a]) * (mc + 1) + lj[a]) * (nc + 1) + kr[b];
            for (int c = 0; c < 3; ++c) s[c] += cs[c][ci];
        }
    T* fs[3] = {f0, f1, f2};
    for (int c = 0; c < 3; ++c) {
        const T v = s[c] * wl * wk;
        fs[c][t] = add ? fs[c][t] + v : v;
    }
}

// Restriction R = P^T, per diamond: a coarse node gathers the fine nodes it
// interpolates to, each weighted by its interpolation weight and by
// 1/multiplicity of the fine node (so the interface sum over diamond copies
// counts every fine node once).  No-slip layers of the result are zero; the layer of
// a free-slip sphere (fs bit 0 inner, bit 1 outer) is restricted like the interior.
template <typename T>
__global__ void restrict_kernel(int mf, int nf, const T* __restrict__ f0, const T* __restrict__ f1,
                                const T* __restrict__ f2, const T* __restrict__ inv_mult,
                                T* c0, T* c1, T* c2, long long ncslots, int fs, SlotBatch sb) {
    const long long so = slot_off(sb);
    f0 = at_slot(f0, so);
    f1 = at_slot(f1, so);
    f2 = at_slot(f2, so);
    c0 = at_slot(c0, so);
    c1 = at_slot(c1, so);
    c2 = at_slot(c2, so);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncslots) return;
    const int mc = mf / 2, nc = nf / 2;
    const NodeIdx q = decode_node(t, mc, nc);
    T s[3] = {0, 0, 0};
    if ((q.k > 0 || (fs & 1)) && (q.k < nc || (fs & 2))) {
        // lateral fine neighbours that interpolate from this coarse node
        const int di[7] = {0, 1, -1, 0, 0, 1, -1};
        const int dj[7] = {0, 0, 0, 1, -1, -1, 1};
        const T wl[7] = {T(1), T(0.5), T(0.5), T(0.5), T(0.5), T(0.5), T(0.5)};
        const T* fs[3] = {f0, f1, f2};
        for (int l = 0; l < 7; ++l) {
            const int fi = 2 * q.i + di[l], fj = 2 * q.j + dj[l];
            if (fi < 0 || fi > mf || fj < 0 || fj > mf) continue;
            const long long lat = ((long long)q.d * (mf + 1) + fi) * (mf + 1) + fj;
            const T wm = wl[l] * inv_mult[lat];
            for (int dk = -1; dk <= 1; ++dk) {
                const int fk = 2 * q.k + dk;
                if (fk < 0 || fk > nf) continue;
                const T w = dk == 0 ? wm : T(0.5) * wm;
                const long long fidx = lat * (nf + 1) + fk;
                for (int c = 0; c < 3; ++c) s[c] += w * fs[c][fidx];
            }
        }
    }
    c0[t] = s[0];
    c1[t] = s[1];
    c2[t] = s[2];
}

// One Chebyshev step of the smoother on D^{-1} A, fused after y = A x:
//   d <- alpha d + beta D^{-1} (b - y),   x <- x + d,
// with (alpha, beta) = ab[2k], ab[2k + 1] (per slot: they scale with the
// slot's eigenvalue estimate).
constexpr int EW_PER = 4;   // elements per thread of the streaming elementwise kernels

template <typename T>
__global__ void __launch_bounds__(256) cheb_update_kernel(long long n, const double* __restrict__ ab, int k,
                                                          const T* __restrict__ b, const T* __restrict__ y,
                                                          const T* __restrict__ invd, T* d, T* x, SlotBatch sb) {
    const long long so = slot_off(sb);
    ab = at_slot(ab, so);
    b = at_slot(b, so);
    y = at_slot(y, so);
    invd = at_slot(invd, so);
    d = at_slot(d, so);
    x = at_slot(x, so);
    const T alpha = T(ab[2 * k]), beta = T(ab[2 * k + 1]);
    const long long t0 = (long long)blockIdx.x * (256 * EW_PER) + threadIdx.x;
    T bv[EW_PER], yv[EW_PER], iv[EW_PER], dv[EW_PER], xv[EW_PER];
#pragma unroll
    for (int e = 0; e < EW_PER; ++e) {
        const long long t = t0 + e * 256;
        const bool in = t < n;
        bv[e] = in ? b[t] : T(0);
        yv[e] = in ? y[t] : T(0);
        iv[e] = in ? invd[t] : T(0);
        dv[e] = in && alpha != T(0) ? d[t] : T(0);   // d may hold garbage on the first step
        xv[e] = in ? x[t] : T(0);
    }
#pragma unroll
    for (int e = 0; e < EW_PER; ++e) {
        const long long t = t0 + e * 256;
        if (t >= n) break;
        const T r = beta * iv[e] * (bv[e] - yv[e]);
        const T nd = alpha == T(0) ? r : alpha * dv[e] + r;
        d[t] = nd;
        x[t] = xv[e] + nd;
    }
}

// The same update with 16-byte vector accesses (every pointer 16-byte aligned):
// vector i of L = 16 / sizeof(T) values per thread, block 0 also the n % L tail;
// the arithmetic of every value is that of cheb_update_kernel.
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
};
template <>
struct Vec16<double> {
    using type = double2;
};

template <typename T>
__global__ void __launch_bounds__(256) cheb_update_vec_kernel(long long n, const double* __restrict__ ab, int k,
                                                              const T* __restrict__ b, const T* __restrict__ y,
                                                              const T* __restrict__ invd, T* d, T* x, SlotBatch sb) {
    using V = typename Vec16<T>::type;
    constexpr int L = 16 / sizeof(T);
    const long long so = slot_off(sb);
    ab = at_slot(ab, so);
    b = at_slot(b, so);
    y = at_slot(y, so);
    invd = at_slot(invd, so);
    d = at_slot(d, so);
    x = at_slot(x, so);
    const T alpha = T(ab[2 * k]), beta = T(ab[2 * k + 1]);
    const long long nv = n / L;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < nv) {
        V bv = reinterpret_cast<const V*>(b)[i], yv = reinterpret_cast<const V*>(y)[i];
        V iv = reinterpret_cast<const V*>(invd)[i], xv = reinterpret_cast<const V*>(x)[i];
        V dv{};
        if (alpha != T(0)) dv = reinterpret_cast<const V*>(d)[i];   // d may hold garbage on the first step
        const T* pb = reinterpret_cast<const T*>(&bv);
        const T* py = reinterpret_cast<const T*>(&yv);
        const T* pi = reinterpret_cast<const T*>(&iv);
        T* pd = reinterpret_cast<T*>(&dv);
        T* px = reinterpret_cast<T*>(&xv);
#pragma unroll
        for (int c = 0; c < L; ++c) {
            const T r = beta * pi[c] * (pb[c] - py[c]);
            pd[c] = alpha == T(0) ? r : alpha * pd[c] + r;
            px[c] += pd[c];
        }
        reinterpret_cast<V*>(d)[i] = dv;
        reinterpret_cast<V*>(x)[i] = xv;
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * L) {
        const long long t = nv * L + threadIdx.x;
        const T r = beta * invd[t] * (b[t] - y[t]);
        const T dn = alpha == T(0) ? r : alpha * d[t] + r;
        d[t] = dn;
        x[t] += dn;
    }
}

// y <- a x + b y with 16-byte vector accesses (as axpby_kernel)
template <typename T>
__global__ void __launch_bounds__(256) axpby_vec_kernel(long long n, T a, const T* __restrict__ x, T b, T* y,
                                                        SlotBatch sb) {
    using V = typename Vec16<T>::type;
    constexpr int L = 16 / sizeof(T);
    const long long so = slot_off(sb);
    x = at_slot(x, so);
    y = at_slot(y, so);
    const long long nv = n / L;
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < nv) {
        V xv = reinterpret_cast<const V*>(x)[i];
        V yv{};
        if (b != T(0)) yv = reinterpret_cast<const V*>(y)[i];
        const T* px = reinterpret_cast<const T*>(&xv);
        T* py = reinterpret_cast<T*>(&yv);
#pragma unroll
        for (int c = 0; c < L; ++c) py[c] = b == T(0) ? a * px[c] : a * px[c] + b * py[c];
        reinterpret_cast<V*>(y)[i] = yv;
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * L) {
        const long long t = nv * L + threadIdx.x;
        y[t] = b == T(0) ? a * x[t] : a * x[t] + b * y[t];
    }
}

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <typename T>
__global__ void invert_kernel(long long n, T* a) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = T(1) / a[t];
}

// Dirichlet (no-slip) rows of a velocity diagonal are identity rows; fs: free-slip
// spheres (bit 0 inner, bit 1 outer), whose rows keep their diagonal.
template <typename T>
__global__ void diag_dirichlet_kernel(long long ncol, int n, int fs, T* d0, T* d1, T* d2) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * ncol) return;
    if ((t & 1) ? (fs & 2) : (fs & 1)) return;
    const long long idx = (t >> 1) * (n + 1) + ((t & 1) ? n : 0);
    d0[idx] = T(1);
    d1[idx] = T(1);
    d2[idx] = T(1);
}

// Free-slip boundary rows of an iterate: x <- P x + N b = x + (rhat.b - rhat.x) rhat at
// the layers of the free-slip spheres (fs bit 0 inner, bit 1 outer), b == nullptr: b = 0.
// The normal rows of P A P + N are identity rows, so this solves them exactly and leaves
// the tangential part to the smoother.
template <typename T>
__global__ void fs_project_kernel(long long ncol, int n, int fs, const T* __restrict__ unit, T* x0, T* x1, T* x2,
                                  const T* __restrict__ b0, const T* __restrict__ b1, const T* __restrict__ b2) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * ncol) return;
    if (!((t & 1) ? (fs & 2) : (fs & 1))) return;
    const long long col = t >> 1;
    const long long idx = col * (n + 1) + ((t & 1) ? n : 0);
    const T r0 = unit[3 * col], r1 = unit[3 * col + 1], r2 = unit[3 * col + 2];
    const T dx = r0 * x0[idx] + r1 * x1[idx] + r2 * x2[idx];
    const T db = b0 ? r0 * b0[idx] + r1 * b1[idx] + r2 * b2[idx] : T(0);
    x0[idx] += (db - dx) * r0;
    x1[idx] += (db - dx) * r1;
    x2[idx] += (db - dx) * r2;
}

// Rigid rotation e_a x x of the shell's nodes (x = r_k rhat), component c at every
// node slot: a null vector of the viscous block with free slip on both spheres.
template <typename T>
__global__ void rotation_fill_kernel(int m, int n, double r_in, double dr, const double* __restrict__ unit, int a,
                                     T* o0, T* o1, T* o2, long long nslots) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const long long lat = t / (n + 1);
    const double r = r_in + (double)(t % (n + 1)) * dr;
    const double x = r * unit[3 * lat], y = r * unit[3 * lat + 1], z = r * unit[3 * lat + 2];
    const double v0 = a == 0 ? 0.0 : (a == 1 ? z : -y);
    const double v1 = a == 0 ? -z : (a == 1 ? 0.0 : x);
    const double v2 = a == 0 ? y : (a == 1 ? -x : 0.0);
    o0[t] = T(v0);
    o1[t] = T(v1);
    o2[t] = T(v2);
}

// The coarsest matrix with free slip on both spheres is singular (the three rigid
// rotations).  q: the rotations over the coarse DoFs, orthonormalised (Gram-Schmidt in
// DoF order), and sigma the mean diagonal entry; one thread.
__global__ void coarse_rotation_basis_kernel(int nd, const int* __restrict__ dof_slot, int m, int n, double r_in,
                                             double dr, const double* __restrict__ unit,
                                             const double* __restrict__ Ad, double* q) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int a = 0; a < 3; ++a) {
        double* qa = q + (long long)a * nd;
        for (int d = 0; d < nd; ++d) {
            const long long slot = dof_slot[d] >> 2;
            const int c = dof_slot[d] & 3;
            const long long lat = slot / (n + 1);
            const double r = r_in + (double)(slot % (n + 1)) * dr;
            const double x[3] = {r * unit[3 * lat], r * unit[3 * lat + 1], r * unit[3 * lat + 2]};
            // (e_a x x)_c = eps_{c a b} x_b
            const int b = 3 - a - c;
            qa[d] = a == c ? 0.0 : (((a - c + 3) % 3 == 1) ? x[b] : -x[b]);
        }
        for (int b2 = 0; b2 < a; ++b2) {
            const double* qb = q + (long long)b2 * nd;
            double dt = 0.0;
            for (int d = 0; d < nd; ++d) dt += qa[d] * qb[d];
            for (int d = 0; d < nd; ++d) qa[d] -= dt * qb[d];
        }
        double nn = 0.0;
        for (int d = 0; d < nd; ++d) nn += qa[d] * qa[d];
        const double inv = 1.0 / sqrt(nn);
        for (int d = 0; d < nd; ++d) qa[d] *= inv;
    }
    double tr = 0.0;
    for (int d = 0; d < nd; ++d) tr += Ad[(long long)d * nd + d];
    q[3LL * nd] = tr / nd;
}

// A <- A + sigma sum_a q_a q_a^T: the rotations get eigenvalue sigma, the rest of the
// spectrum is unchanged (the q_a span the null space), so for a right-hand side
// orthogonal to them the inverse gives the solution orthogonal to them.
__global__ void coarse_rotation_shift_kernel(int nd, const double* __restrict__ q, double* Ad) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nd) return;
    const double sigma = q[3LL * nd];
    const double c0 = q[col], c1 = q[nd + col], c2 = q[2LL * nd + col];
    for (int r = 0; r < nd; ++r)
        Ad[(long long)col * nd + r] += sigma * (c0 * q[r] + c1 * q[nd + r] + c2 * q[2LL * nd + r]);
}

template <typename TO, typename TI>
__global__ void cast_kernel(long long n, const TI* __restrict__ a, TO* __restrict__ b, SlotBatch sb) {
    const long long so = slot_off(sb);
    a = at_slot(a, so);
    b = at_slot(b, so);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) b[t] = TO(a[t]);
}

// y <- a x + b y  (x may alias nothing; pass b = 0 to overwrite)
template <typename T>
__global__ void __launch_bounds__(256) axpby_kernel(long long n, T a, const T* __restrict__ x, T b, T* y,
                                                    SlotBatch sb) {
    const long long so = slot_off(sb);
    x = at_slot(x, so);
    y = at_slot(y, so);
    const long long t0 = (long long)blockIdx.x * (256 * EW_PER) + threadIdx.x;
    T xv[EW_PER], yv[EW_PER];
#pragma unroll
    for (int e = 0; e < EW_PER; ++e) {
        const long long t = t0 + e * 256;
        xv[e] = t < n ? x[t] : T(0);
        yv[e] = t < n && b != T(0) ? y[t] : T(0);
    }
#pragma unroll
    for (int e = 0; e < EW_PER; ++e) {
        const long long t = t0 + e * 256;
        if (t >= n) break;
        y[t] = b == T(0) ? a * xv[e] : a * xv[e] + b * yv[e];
    }
}

// Multi-dot partials: for every vector v_q (q < nq <= NQ) the block sum of
// mask(slot) x v_q over one grid-stride share; a second kernel adds the block
// sums in a fixed order, so the result does not depend on timing.  Node slot
// t lies in radial column t / n1 (division by a magic multiplier, exact for
// all 32-bit t); the owner mask counts every unique node once.  The vector
// pointers are read once per block into scalar registers, and every load of
// an element is issued before the first use.
constexpr int DOT_BS = 256;

struct MagicDiv {
    unsigned mul;   // ceil(2^(32 + sh) / d) - 2^32
    int sh;         // ceil(log2 d)
};
inline MagicDiv magic_div(unsigned d) {
    MagicDiv m{0u, 0};
    while ((1ull << m.sh) < d) ++m.sh;
    const unsigned long long big = 1ull << (32 + m.sh);
    m.mul = (unsigned)((big + d - 1) / d - (1ull << 32));
    return m;
}
__device__ __forceinline__ unsigned mdiv(unsigned t, MagicDiv m) {
    return (unsigned)((((unsigned long long)__umulhi(t, m.mul)) + t) >> m.sh);
}

// Residual r = b - A_D x from a raw viscous apply y (the closing pass fused as in
// cheb_post_update_kernel: copies summed in group order, identity rows r = b - x).
template <typename T>
__global__ void __launch_bounds__(256) resid_post_kernel(int ns, int n1, MagicDiv dn1, const int* __restrict__ lat_grp,
                                                        const int* __restrict__ gp, const int* __restrict__ gs,
                                                        int ns_in, int ns_out, const T* __restrict__ b,
                                                        const T* __restrict__ x, const T* y, T* r, SlotBatch sb) {
    const long long so = slot_off(sb);
    const unsigned t = blockIdx.x * 256u + threadIdx.x;
    if (t >= (unsigned)ns) return;
    const long long e = (long long)blockIdx.y * ns + t;
    const unsigned lat = mdiv(t, dn1);
    const int kk = (int)(t - lat * (unsigned)n1);
    T yv;
    if ((ns_in && kk == 0) || (ns_out && kk == n1 - 1)) {
        yv = at_slot(x, so)[e];
    } else {
        const int g = lat_grp[lat];
        const T* yy = at_slot(y, so) + (long long)blockIdx.y * ns;
        if (g < 0) {
            yv = yy[t];
        } else {
            const int s0 = gp[g], s1 = gp[g + 1];
            yv = yy[(long long)gs[s0] * n1 + kk];
            for (int q = s0 + 1; q < s1; ++q) yv += yy[(long long)gs[q] * n1 + kk];
        }
    }
    at_slot(r, so)[e] = at_slot(b, so)[e] - yv;
}

// One Chebyshev step of the smoother in its two-term form
//   x_k+1 = x_k + alpha (x_k - x_k-1) + beta D^-1 (b - A_D x_k)
// (the form with the direction d_k = x_k+1 - x_k needs one more vector per step),
// fused with the closing pass of the raw viscous apply before it (y = A_D x_k with
// each diamond's partial sums on duplicated nodes and nothing on the no-slip rows):
// per node, the completed A_D x_k is the sum of the node's copies in group order
// (the interface pass's order), or x_k itself on an identity row.  xo holds x_k-1
// on entry (read when alpha != 0 and not prev_zero; x_k-1 = 0 otherwise) and x_k+1
// on return, element by element in place.  first: the step from x_k = 0
// (y and x_k are not read).  Each thread takes one 16-byte vector of the flat
// [3][node slots] arrays (16-byte aligned; the tail of fewer than one vector is the
// first block's) and locates its elements' node (component, lateral slot, layer)
// incrementally.
template <typename T>
__global__ void __launch_bounds__(256) cheb_post_update_kernel(unsigned ns, int n1, MagicDiv dns, MagicDiv dn1,
                                                              const int* __restrict__ lat_grp,
                                                              const int* __restrict__ gp, const int* __restrict__ gs,
                                                              int ns_in, int ns_out, const double* __restrict__ ab,
                                                              int k, int first, int prev_zero,
                                                              const T* __restrict__ b, const T* __restrict__ y,
                                                              const T* __restrict__ invd, const T* __restrict__ xk,
                                                              T* xo, SlotBatch sb) {
    using V = typename Vec16<T>::type;
    constexpr int L = 16 / sizeof(T);
    const long long so = slot_off(sb);
    ab = at_slot(ab, so);
    b = at_slot(b, so);
    y = at_slot(y, so);
    invd = at_slot(invd, so);
    xk = at_slot(xk, so);
    xo = at_slot(xo, so);
    const T alpha = T(ab[2 * k]), beta = T(ab[2 * k + 1]);
    const bool use_prev = alpha != T(0) && !prev_zero;
    const unsigned n = 3u * ns, nv = n / L;
    const unsigned v = blockIdx.x * 256u + threadIdx.x;
    // completed A_D x_k at element e (component c, lateral slot lat, layer kk)
    auto yat = [&](unsigned c, unsigned lat, int kk, T yraw, T xv) -> T {
        if ((ns_in && kk == 0) || (ns_out && kk == n1 - 1)) return xv;
        const int g = lat_grp[lat];
        if (g < 0) return yraw;
        const T* yy = y + (size_t)c * ns;
        const int s0 = gp[g], s1 = gp[g + 1];
        T acc = yy[(size_t)gs[s0] * n1 + kk];
        for (int q = s0 + 1; q < s1; ++q) acc += yy[(size_t)gs[q] * n1 + kk];
        return acc;
    };
    auto step = [&](T bq, T iq, T yq, T xq, T pq) -> T {
        const T r = beta * iq * (bq - yq);
        return use_prev ? xq + (alpha * (xq - pq) + r) : (alpha == T(0) ? xq + r : xq + (alpha * xq + r));
    };
    if (v < nv) {
        const V bv = reinterpret_cast<const V*>(b)[v], iv = reinterpret_cast<const V*>(invd)[v];
        const T* pb = reinterpret_cast<const T*>(&bv);
        const T* pi = reinterpret_cast<const T*>(&iv);
        V ov{};
        T* po = reinterpret_cast<T*>(&ov);
        if (first) {
#pragma unroll
            for (int q = 0; q < L; ++q) po[q] = beta * pi[q] * (pb[q] - T(0));
        } else {
            const V yv = reinterpret_cast<const V*>(y)[v], xv = reinterpret_cast<const V*>(xk)[v];
            V pv{};
            if (use_prev) pv = reinterpret_cast<const V*>(xo)[v];
            const T* py = reinterpret_cast<const T*>(&yv);
            const T* px = reinterpret_cast<const T*>(&xv);
            const T* pp = reinterpret_cast<const T*>(&pv);
            const unsigned e0 = v * L;
            unsigned c = mdiv(e0, dns);
            unsigned t = e0 - c * ns;
            unsigned lat = mdiv(t, dn1);
            int kk = (int)(t - lat * (unsigned)n1);
#pragma unroll
            for (int q = 0; q < L; ++q) {
                po[q] = step(pb[q], pi[q], yat(c, lat, kk, py[q], px[q]), px[q], pp[q]);
                // next element: the next layer, column or component
                if (++kk == n1) {
                    kk = 0;
                    if (++t == ns) {
                        t = 0;
                        ++c;
                        lat = 0;
                    } else {
                        ++lat;
                    }
                } else {
                    ++t;
                }
            }
        }
        reinterpret_cast<V*>(xo)[v] = ov;
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * L) {
        const unsigned e = nv * L + threadIdx.x;
        if (first) {
            xo[e] = beta * invd[e] * (b[e] - T(0));
        } else {
            const unsigned c = mdiv(e, dns), t = e - c * ns, lat = mdiv(t, dn1);
            const int kk = (int)(t - lat * (unsigned)n1);
            const T xe = xk[e];
            xo[e] = step(b[e], invd[e], yat(c, lat, kk, y[e], xe), xe, use_prev ? xo[e] : T(0));
        }
    }
}

// A pointer read from a table lost its address space; loads through this
// global-memory pointer type are global, not flat, instructions.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
    return (gptr<T>)p;
}

// Block sums of acc[q], q < nq, to part[blockIdx.x][q] (fixed order).
template <int NQ>
__device__ __forceinline__ void block_partials(const double (&acc)[NQ], int nq, double* __restrict__ part) {
    __shared__ double sh[DOT_BS / 64][NQ];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q >= nq) break;
        double v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) sh[wv][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < nq) {
        double v = 0.0;
        for (int w = 0; w < DOT_BS / 64; ++w) v += sh[w][threadIdx.x];
        part[(long long)blockIdx.x * MAX_MDOT + threadIdx.x] = v;
    }
}

// n slots of up to three node-field components of one level (n1 layers per
// column, nlat lateral slots per component).
template <typename T, int NQ>
__global__ void __launch_bounds__(DOT_BS) mdot_partial_kernel(unsigned n, MagicDiv dn1, unsigned nlat,
                                                              const uint8_t* __restrict__ owner,
                                                              const T* __restrict__ x, const T* const* __restrict__ vs,
                                                              int nq, double* __restrict__ part, SlotBatch sb) {
    const long long so = slot_off(sb);
    x = at_slot(x, so);
    vs = at_slot(vs, so);
    part = at_slot(part, so);
    nq = slot_count(sb, nq);
    gptr<T> vp[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) vp[q] = as_global(vs[q < nq ? q : 0]);
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    // two elements per step, every load (mask and data) issued before the first use
    const unsigned stride = gridDim.x * DOT_BS;
    for (unsigned t0 = blockIdx.x * DOT_BS + threadIdx.x; t0 < n; t0 += 2 * stride) {
        T xv[2], v[2][NQ];
        bool own[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned t = t0 + e * stride;
            const bool in = t < n;
            const unsigned tt = in ? t : 0;
            unsigned lat = mdiv(tt, dn1);
            lat = lat >= nlat ? lat - nlat : lat;
            lat = lat >= nlat ? lat - nlat : lat;
            own[e] = in && owner[lat];
            xv[e] = x[tt];
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[e][q] = q < nq ? vp[q][tt] : T(0);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!own[e]) continue;
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += (double)xv[e] * (double)v[e][q];
        }
    }
    block_partials<NQ>(acc, nq, part);
}

// y <- y + sign * sum_q coef[q] v_q (q < nq <= NQ), coefficients read from
// device memory; pointers and coefficients in scalar registers, all loads of
// an element in flight together.
template <typename T, int NQ>
__global__ void __launch_bounds__(256) maxpy_kernel(unsigned n, const double* __restrict__ coef, double sign,
                                                    const T* const* __restrict__ vs, int nq, T* y, SlotBatch sb) {
    const long long so = slot_off(sb);
    coef = at_slot(coef, so);
    vs = at_slot(vs, so);
    y = at_slot(y, so);
    nq = slot_count(sb, nq);
    gptr<T> vp[NQ];
    double cf[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        vp[q] = as_global(vs[q < nq ? q : 0]);
        cf[q] = q < nq ? sign * coef[q] : 0.0;
    }
    const unsigned stride = gridDim.x * blockDim.x;
    for (unsigned t0 = blockIdx.x * blockDim.x + threadIdx.x; t0 < n; t0 += 2 * stride) {
        T v[2][NQ], yv[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned t = t0 + e * stride;
            const unsigned tt = t < n ? t : 0;
            yv[e] = y[tt];
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[e][q] = q < nq ? vp[q][tt] : T(0);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned t = t0 + e * stride;
            if (t >= n) break;
            double acc = (double)yv[e];
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (q < nq) acc += cf[q] * (double)v[e][q];
            y[t] = T(acc);
        }
    }
}

template <typename T>
__global__ void mul_kernel(unsigned n, const T* __restrict__ a, const T* __restrict__ b, T* c) {
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) c[t] = a[t] * b[t];
}

template <typename T>
__global__ void fillv_kernel(unsigned n, T v, T* a, SlotBatch sb) {
    a = at_slot(a, slot_off(sb));
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) a[t] = v;
}

// out[q] = sum of the block partials of vector q: wave w takes q = w, w + 4,
// ..., every lane a fixed strided share of the blocks, then a fixed shuffle
// tree; the order depends only on nblocks.
__global__ void __launch_bounds__(256) mdot_final_kernel(int nblocks, int nq, const double* __restrict__ part,
                                                         double* out, int accumulate, SlotBatch sb) {
    const long long so = slot_off(sb);
    part = at_slot(part, so);
    out = at_slot(out, so);
    nq = slot_count(sb, nq);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int q = wv; q < nq; q += 4) {
        // eight independent partial sums per lane keep eight loads in flight (the loads
        // are a strided gather, latency-bound one by one); combined in a fixed order
        double v8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int b = lane;
        for (; b + 7 * 64 < nblocks; b += 8 * 64)
#pragma unroll
            for (int u = 0; u < 8; ++u) v8[u] += part[(long long)(b + u * 64) * MAX_MDOT + q];
        for (; b < nblocks; b += 64) v8[0] += part[(long long)b * MAX_MDOT + q];
        double v = ((v8[0] + v8[1]) + (v8[2] + v8[3])) + ((v8[4] + v8[5]) + (v8[6] + v8[7]));
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) out[q] = accumulate ? out[q] + v : v;
    }
}

// Dense coarsest level ------------------------------------------------------

// Column `col` of the assembled coarsest operator restricted to unique
// interior DoFs: y = A e_col has been computed in the slot layout; gather the
// owner copies into row-major dense storage (A is symmetric).
template <typename T>
__global__ void coarse_gather_col_kernel(int ndof, const int* __restrict__ dof_slot, const T* __restrict__ y0,
                                         const T* __restrict__ y1, const T* __restrict__ y2, int col,
                                         double* __restrict__ Ad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= ndof) return;
    const int s = dof_slot[r];
    const int c = s & 3;
    const long long slot = s >> 2;
    const T v = c == 0 ? y0[slot] : (c == 1 ? y1[slot] : y2[slot]);
    Ad[(long long)col * ndof + r] = (double)v;
}

// Gauss-Jordan inversion of an SPD matrix in one workgroup (no pivoting is
// needed for SPD matrices).  a: ndof x ndof, overwritten by its inverse.
__global__ void __launch_bounds__(1024) gauss_jordan_kernel(int nd, double* a) {
    __shared__ double prow[MAX_COARSE_DOF];
    __shared__ double pcol[MAX_COARSE_DOF];
    for (int p = 0; p < nd; ++p) {
        __syncthreads();
        const double piv = a[(long long)p * nd + p];
        for (int x = threadIdx.x; x < nd; x += blockDim.x) {
            prow[x] = a[(long long)p * nd + x];
            pcol[x] = a[(long long)x * nd + p];
        }
        __syncthreads();
        const double ip = 1.0 / piv;
        const long long total = (long long)nd * nd;
        for (long long e = threadIdx.x; e < total; e += blockDim.x) {
            const int r = (int)(e / nd), c = (int)(e % nd);
            double v;
            if (r == p && c == p) v = ip;
            else if (r == p) v = prow[c] * ip;
            else if (c == p) v = -pcol[r] * ip;
            else v = a[e] - pcol[r] * prow[c] * ip;
            a[e] = v;
        }
    }
}

// x = A^{-1} b on the coarsest level: gather b at owner slots of interior
// DoFs, dense symmetric matvec, scatter to every copy; other rows set to zero
// (their right-hand side is zero in a V-cycle: Dirichlet rows).
template <typename T>
__global__ void __launch_bounds__(1024) coarse_solve_kernel(int nd, const int* __restrict__ dof_slot,
                                                            const int* __restrict__ slot_dof, long long nslots,
                                                            const double* __restrict__ Ainv,
                                                            const T* __restrict__ b0, const T* __restrict__ b1,
                                                            const T* __restrict__ b2, T* x0, T* x1, T* x2,
                                                            SlotBatch sb) {
    const long long so = slot_off(sb);
    dof_slot = at_slot(dof_slot, so);
    slot_dof = at_slot(slot_dof, so);
    Ainv = at_slot(Ainv, so);
    b0 = at_slot(b0, so);
    b1 = at_slot(b1, so);
    b2 = at_slot(b2, so);
    x0 = at_slot(x0, so);
    x1 = at_slot(x1, so);
    x2 = at_slot(x2, so);
    __shared__ double rhs[MAX_COARSE_DOF];
    __shared__ double sol[MAX_COARSE_DOF];
    for (int r = threadIdx.x; r < nd; r += blockDim.x) {
        const int s = dof_slot[r];
        const int c = s & 3;
        const long long slot = s >> 2;
        rhs[r] = (double)(c == 0 ? b0[slot] : (c == 1 ? b1[slot] : b2[slot]));
    }
    __syncthreads();
    for (int r = threadIdx.x; r < nd; r += blockDim.x) {
        double v = 0.0;
        for (int c = 0; c < nd; ++c) v += Ainv[(long long)c * nd + r] * rhs[c];
        sol[r] = v;
    }
    __syncthreads();
    for (long long t = threadIdx.x; t < 3 * nslots; t += blockDim.x) {
        const int c = (int)(t / nslots);
        const long long slot = t % nslots;
        const int dof = slot_dof[c * nslots + slot];
        const T v = dof >= 0 ? T(sol[dof]) : T(0);
        if (c == 0) x0[slot] = v;
        else if (c == 1) x1[slot] = v;
        else x2[slot] = v;
    }
}

template <typename T>
__global__ void unit_vector_kernel(long long nslots, const int* __restrict__ slot_dof, int col, T* x0, T* x1,
                                   T* x2) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * nslots) return;
    const int c = (int)(t / nslots);
    const long long slot = t % nslots;
    const T v = slot_dof[c * nslots + slot] == col ? T(1) : T(0);
    if (c == 0) x0[slot] = v;
    else if (c == 1) x1[slot] = v;
    else x2[slot] = v;
}

// Pressure: zero nodal mean projection helper  p <- p - mean
template <typename T>
__global__ void shift_kernel(long long n, const double* __restrict__ sum_cnt, T* p, SlotBatch sb) {
    const long long so = slot_off(sb);
    sum_cnt = at_slot(sum_cnt, so);
    p = at_slot(p, so);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] -= T(sum_cnt[0] / sum_cnt[1]);
}

// Schur preconditioner on the pressure: z = -r / m (Sec. 7, eq:pmass)
template <typename T>
__global__ void schur_diag_kernel(long long n, const T* __restrict__ r, const T* __restrict__ mdiag, T* z,
                                  SlotBatch sb) {
    const long long so = slot_off(sb);
    r = at_slot(r, so);
    mdiag = at_slot(mdiag, so);
    z = at_slot(z, so);
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) z[t] = -r[t] / mdiag[t];
}

// Multi-dot over a Stokes vector [u0 u1 u2 p] (velocity slots of one level
// followed by its pressure slots): owner masks of both grids.
template <typename T, int NQ>
__global__ void __launch_bounds__(DOT_BS) smdot_partial_kernel(unsigned ns, MagicDiv dn1u, unsigned nlat_u,
                                                               const uint8_t* __restrict__ ou, unsigned np,
                                                               MagicDiv dn1p, const uint8_t* __restrict__ op,
                                                               const T* __restrict__ x,
                                                               const T* const* __restrict__ vs, int nq,
                                                               double* __restrict__ part, SlotBatch sb) {
    const long long so = slot_off(sb);
    x = at_slot(x, so);
    vs = at_slot(vs, so);
    part = at_slot(part, so);
    nq = slot_count(sb, nq);
    gptr<T> vp[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) vp[q] = as_global(vs[q < nq ? q : 0]);
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const unsigned nu = 3u * ns, n = nu + np;
    // two elements per step, every load (mask and data) issued before the first use
    const unsigned stride = gridDim.x * DOT_BS;
    for (unsigned t0 = blockIdx.x * DOT_BS + threadIdx.x; t0 < n; t0 += 2 * stride) {
        T xv[2], v[2][NQ];
        bool own[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned t = t0 + e * stride;
            const bool in = t < n;
            const unsigned tt = in ? t : 0;
            if (tt < nu) {
                unsigned lat = mdiv(tt, dn1u);
                lat = lat >= nlat_u ? lat - nlat_u : lat;
                lat = lat >= nlat_u ? lat - nlat_u : lat;
                own[e] = in && ou[lat];
            } else {
                own[e] = in && op[mdiv(tt - nu, dn1p)];
            }
            xv[e] = x[tt];
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[e][q] = q < nq ? vp[q][tt] : T(0);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (!own[e]) continue;
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += (double)xv[e] * (double)v[e][q];
        }
    }
    block_partials<NQ>(acc, nq, part);
}

// Gram-Schmidt step fused with the dots that follow it, over a Stokes vector:
//   y <- y - sum_q c_q v_q   (every slot, as maxpy_kernel),
// then, over owned slots, the dots of the new y with the same v_q (NORM false:
// the re-orthogonalisation coefficients) or with itself (NORM true: the
// squared norm), from the stored (rounded) value of y; block partials as in
// smdot_partial_kernel.  One pass instead of a multi-axpy and a multi-dot.
template <typename T, int NQ, bool NORM>
__global__ void __launch_bounds__(DOT_BS) maxpy_dot_kernel(unsigned ns, MagicDiv dn1u, unsigned nlat_u,
                                                           const uint8_t* __restrict__ ou, unsigned np,
                                                           MagicDiv dn1p, const uint8_t* __restrict__ op,
                                                           const double* __restrict__ coef, double sign,
                                                           const T* const* __restrict__ vs, int nq, T* y,
                                                           double* __restrict__ part, SlotBatch sb) {
    const long long so = slot_off(sb);
    coef = at_slot(coef, so);
    vs = at_slot(vs, so);
    y = at_slot(y, so);
    part = at_slot(part, so);
    nq = slot_count(sb, nq);
    gptr<T> vp[NQ];
    double cf[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        vp[q] = as_global(vs[q < nq ? q : 0]);
        cf[q] = q < nq ? sign * coef[q] : 0.0;
    }
    constexpr int NA = NORM ? 1 : NQ;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    const unsigned nu = 3u * ns, n = nu + np;
    const unsigned stride = gridDim.x * DOT_BS;
    for (unsigned t0 = blockIdx.x * DOT_BS + threadIdx.x; t0 < n; t0 += 2 * stride) {
        T yv[2], v[2][NQ];
        bool own[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned t = t0 + e * stride;
            const bool in = t < n;
            const unsigned tt = in ? t : 0;
            if (tt < nu) {
                unsigned lat = mdiv(tt, dn1u);
                lat = lat >= nlat_u ? lat - nlat_u : lat;
                lat = lat >= nlat_u ? lat - nlat_u : lat;
                own[e] = in && ou[lat];
            } else {
                own[e] = in && op[mdiv(tt - nu, dn1p)];
            }
            yv[e] = y[tt];
#pragma unroll
            for (int q = 0; q < NQ; ++q) v[e][q] = q < nq ? vp[q][tt] : T(0);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const unsigned t = t0 + e * stride;
            if (t >= n) break;
            double a = (double)yv[e];
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (q < nq) a += cf[q] * (double)v[e][q];
            const T yn = T(a);
            y[t] = yn;
            if (!own[e]) continue;
            if (NORM) {
                acc[0] += (double)yn * (double)yn;
            } else {
#pragma unroll
                for (int q = 0; q < NA; ++q) acc[q] += (double)v[e][q] * (double)yn;
            }
        }
    }
    block_partials<NA>(acc, NORM ? 1 : nq, part);
}

// 16 bytes of T values as a native vector (it loads out of the global address space
// as one 16-byte access)
template <typename T>
struct Pack16 {
    typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
};

template <typename T>
__device__ __forceinline__ bool stokes_owned(unsigned t, unsigned nu, MagicDiv dn1u, unsigned nlat_u,
                                             const uint8_t* __restrict__ ou, MagicDiv dn1p,
                                             const uint8_t* __restrict__ op) {
    if (t < nu) {
        unsigned lat = mdiv(t, dn1u);
        lat = lat >= nlat_u ? lat - nlat_u : lat;
        lat = lat >= nlat_u ? lat - nlat_u : lat;
        return ou[lat] != 0;
    }
    return op[mdiv(t - nu, dn1p)] != 0;
}

// smdot_partial_kernel and maxpy_dot_kernel with 16-byte accesses, for vectors that are all
// 16-byte aligned (the Krylov basis, also in the slots of a batch): a thread takes
// L = 16 / sizeof(T) consecutive values of every vector per load, block 0 also the n % L
// tail.  Same arithmetic per value (FP64 products and sums); the owner mask of every value.
template <typename T, int NQ>
__global__ void __launch_bounds__(DOT_BS) smdot_vec_kernel(unsigned ns, MagicDiv dn1u, unsigned nlat_u,
                                                           const uint8_t* __restrict__ ou, unsigned np,
                                                           MagicDiv dn1p, const uint8_t* __restrict__ op,
                                                           const T* __restrict__ x,
                                                           const T* const* __restrict__ vs, int nq,
                                                           double* __restrict__ part, SlotBatch sb) {
    using V = typename Pack16<T>::type;
    constexpr int L = 16 / sizeof(T);
    using gvptr = const __attribute__((address_space(1))) V*;
    const long long so = slot_off(sb);
    x = at_slot(x, so);
    vs = at_slot(vs, so);
    part = at_slot(part, so);
    nq = slot_count(sb, nq);
    gvptr vp[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) vp[q] = (gvptr)vs[q < nq ? q : 0];
    const gvptr xp = (gvptr)x;
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    const unsigned nu = 3u * ns, n = nu + np, nv = n / L;
    const unsigned stride = gridDim.x * DOT_BS;
    for (unsigned c = blockIdx.x * DOT_BS + threadIdx.x; c < nv; c += stride) {
        const V xv = xp[c];
        V v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = vp[q < nq ? q : 0][c];
        const V px = xv;
#pragma unroll
        for (int e = 0; e < L; ++e) {
            if (!stokes_owned<T>(c * L + e, nu, dn1u, nlat_u, ou, dn1p, op)) continue;
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[q] += (double)px[e] * (double)v[q][e];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * L) {
        const unsigned t = nv * L + threadIdx.x;
        if (stokes_owned<T>(t, nu, dn1u, nlat_u, ou, dn1p, op)) {
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (q < nq) acc[q] += (double)x[t] * (double)vs[q][t];
        }
    }
    block_partials<NQ>(acc, nq, part);
}

template <typename T, int NQ, bool NORM>
__global__ void __launch_bounds__(DOT_BS) maxpy_dot_vec_kernel(unsigned ns, MagicDiv dn1u, unsigned nlat_u,
                                                               const uint8_t* __restrict__ ou, unsigned np,
                                                               MagicDiv dn1p, const uint8_t* __restrict__ op,
                                                               const double* __restrict__ coef, double sign,
                                                               const T* const* __restrict__ vs, int nq, T* y,
                                                               double* __restrict__ part, SlotBatch sb) {
    using V = typename Pack16<T>::type;
    constexpr int L = 16 / sizeof(T);
    using gvptr = const __attribute__((address_space(1))) V*;
    const long long so = slot_off(sb);
    coef = at_slot(coef, so);
    vs = at_slot(vs, so);
    y = at_slot(y, so);
    part = at_slot(part, so);
    nq = slot_count(sb, nq);
    gvptr vp[NQ];
    double cf[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        vp[q] = (gvptr)vs[q < nq ? q : 0];
        cf[q] = q < nq ? sign * coef[q] : 0.0;
    }
    constexpr int NA = NORM ? 1 : NQ;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    const unsigned nu = 3u * ns, n = nu + np, nv = n / L;
    const unsigned stride = gridDim.x * DOT_BS;
    V* yv = reinterpret_cast<V*>(y);
    for (unsigned c = blockIdx.x * DOT_BS + threadIdx.x; c < nv; c += stride) {
        V w = yv[c];
        V v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) v[q] = vp[q < nq ? q : 0][c];
        #pragma unroll
        for (int e = 0; e < L; ++e) {
            double a2 = (double)w[e];
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                if (q < nq) a2 += cf[q] * (double)v[q][e];
            w[e] = T(a2);
        }
        yv[c] = w;
#pragma unroll
        for (int e = 0; e < L; ++e) {
            if (!stokes_owned<T>(c * L + e, nu, dn1u, nlat_u, ou, dn1p, op)) continue;
            const double yn = (double)w[e];
            if (NORM) {
                acc[0] += yn * yn;
            } else {
#pragma unroll
                for (int q = 0; q < NA; ++q) acc[q] += (double)v[q][e] * yn;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < n - nv * L) {
        const unsigned t = nv * L + threadIdx.x;
        double a2 = (double)y[t];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < nq) a2 += cf[q] * (double)vs[q][t];
        const T yn = T(a2);
        y[t] = yn;
        if (stokes_owned<T>(t, nu, dn1u, nlat_u, ou, dn1p, op)) {
            if (NORM) {
                acc[0] += (double)yn * (double)yn;
            } else {
#pragma unroll
                for (int q = 0; q < NA; ++q)
                    if (q < nq) acc[q] += (double)vs[q][t] * (double)yn;
            }
        }
    }
    block_partials<NA>(acc, NORM ? 1 : nq, part);
}

// Counter-based uniform numbers in [-1, 1) (splitmix64 of seed and index).
template <typename T>
__global__ void rand_kernel(unsigned n, unsigned long long seed, T* a) {
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
        unsigned long long z = seed + 0x9E3779B97F4A7C15ULL * (unsigned long long)(t + 1);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z = z ^ (z >> 31);
        a[t] = T((double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0);
    }
}

// y <- x / sqrt(s[0])  (normalise by a device-side squared norm)
template <typename T>
__global__ void scale_rsqrt_kernel(unsigned n, const double* __restrict__ s, const T* __restrict__ x, T* y,
                                   SlotBatch sb) {
    const long long so = slot_off(sb);
    s = at_slot(s, so);
    x = at_slot(x, so);
    y = at_slot(y, so);
    const double f = 1.0 / sqrt(s[0]);
    for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        y[t] = T(f * (double)x[t]);
}

// y <- f x with x = src or the table entry src_tab[i], y = dst or dst_tab[i]
// (i: the slot's table index), f = 1 / sqrt(sq[0]) when sq is given, else 1.
// Moves vectors in and out of a Krylov basis whose index differs per slot.
template <typename T>
__global__ void tab_copy_kernel(unsigned n, const T* __restrict__ src, const T* const* __restrict__ src_tab,
                                T* dst, T* const* __restrict__ dst_tab, int idx, const double* __restrict__ sq,
                                SlotBatch sb) {
    using gw = __attribute__((address_space(1))) T*;
    const long long so = slot_off(sb);
    const int i = slot_count(sb, idx);
    const gptr<T> x = src_tab ? as_global(at_slot(src_tab, so)[i]) : as_global(at_slot(src, so));
    const gw y = dst_tab ? (gw)at_slot(dst_tab, so)[i] : (gw)at_slot(dst, so);
    if (sq) {
        const double f = 1.0 / sqrt(at_slot(sq, so)[0]);
        for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
            y[t] = T(f * (double)x[t]);
    } else {
        for (unsigned t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) y[t] = x[t];
    }
}

// Short per-slot arrays to and from one shared staging array (row z: slot z).
__global__ void scal_gather_kernel(const double* __restrict__ src, int k, double* __restrict__ dst, SlotBatch sb) {
    src = at_slot(src, slot_off(sb));
    for (int i = threadIdx.x; i < k; i += blockDim.x) dst[(long long)blockIdx.z * k + i] = src[i];
}
__global__ void scal_scatter_kernel(const double* __restrict__ src, int k, double* __restrict__ dst, SlotBatch sb) {
    dst = at_slot(dst, slot_off(sb));
    for (int i = threadIdx.x; i < k; i += blockDim.x) dst[i] = src[(long long)blockIdx.z * k + i];
}

// Column `col` of D A D on the coarsest level, assembled from the one-point
// element matrices (eq:elemmat) of every wedge around every copy of the
// column's node; one thread per column, fixed loop order.
template <typename T>
__global__ void coarse_assemble_kernel(int nd, const int* __restrict__ copy_ptr, const int* __restrict__ copy_slot,
                                       const int* __restrict__ slot_dof, long long nslots, const T* __restrict__ eta,
                                       const double* __restrict__ geo, int m, int n, double r_in, double dr,
                                       double hg_alpha, int twopt, int fs, const double* __restrict__ unit,
                                       double* __restrict__ Ad) {
    const int col = blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= nd) return;
    for (int r = 0; r < nd; ++r) Ad[(long long)col * nd + r] = 0.0;
    auto on_fs = [&](int k) { return ((fs & 1) && k == 0) || ((fs & 2) && k == n); };
    for (int cp = copy_ptr[col]; cp < copy_ptr[col + 1]; ++cp) {
        const int sc = copy_slot[cp];
        const long long slot = sc >> 2;
        const int ccomp = sc & 3;
        const NodeIdx q = decode_node(slot, m, n);
        // free slip: the column is (P A P) e_c, P = I - rhat rhat^T at the column node and
        // at every row node on a free-slip sphere
        const bool pc = on_fs(q.k);
        const double* nc = unit + 3 * ((((long long)q.d * (m + 1) + q.i) * (m + 1)) + q.j);
        for (int ci = q.i - 1; ci <= q.i; ++ci) {
            if (ci < 0 || ci >= m) continue;
            for (int cj = q.j - 1; cj <= q.j; ++cj) {
                if (cj < 0 || cj >= m) continue;
                const int di = q.i - ci, dj = q.j - cj;
                const double* gcol = geo + (((long long)q.d * m + ci) * m + cj) * GEO_PER_COL;
                for (int ck = q.k - 1; ck <= q.k; ++ck) {
                    if (ck < 0 || ck >= n) continue;
                    const int top = q.k - ck;
                    const double rm = r_in + (ck + 0.5) * dr;
                    const double s1 = 0.5 / rm;
                    for (int wd = 0; wd < 2; ++wd) {
                        const int cdi[2][3] = {{0, 1, 0}, {1, 0, 1}};
                        const int cdj[2][3] = {{0, 0, 1}, {1, 1, 0}};
                        int lat = -1;
                        for (int l = 0; l < 3; ++l)
                            if (cdi[wd][l] == di && cdj[wd][l] == dj) lat = l;
                        if (lat < 0) continue;
                        const double* g = gcol + wd * GEO_PER_TRI;
                        const double e = (double)eta[((((long long)q.d * m + ci) * m + cj) * n + ck) * 2 + wd];
                        // quadrature points: q_c (weight 1), or the two radial points
                        const int nq = twopt ? 2 : 1;
                        for (int qq = 0; qq < nq; ++qq) {
                            const double zq = twopt ? (qq == 0 ? -TWOPT_ZETA : TWOPT_ZETA) : 0.0;
                            const double rq = twopt ? rm + zq * (0.5 * dr) : rm;
                            const double V = (twopt ? 0.5 : 1.0) * rq * rq * g[9];
                            double gj[3];
                            if (twopt)
                                basis_grad_at(g, 0.5 / rq, zq, lat, top, gj);
                            else
                                basis_grad(g, s1, lat, top, gj);
                            const double eps = hg_alpha != 0.0 ? hg_eps(g, s1, V, e, hg_alpha) : 0.0;
                            for (int l2 = 0; l2 < 6; ++l2) {
                                const int lat2 = l2 % 3, top2 = l2 / 3;
                                double gl[3];
                                if (twopt)
                                    basis_grad_at(g, 0.5 / rq, zq, lat2, top2, gl);
                                else
                                    basis_grad(g, s1, lat2, top2, gl);
                                const long long s2 = (((long long)q.d * (m + 1) + ci + cdi[wd][lat2]) * (m + 1) +
                                                      cj + cdj[wd][lat2]) * (n + 1) + ck + top2;
                                const double gg = gj[0] * gl[0] + gj[1] * gl[1] + gj[2] * gl[2];
                                // (A_e)_{(j,c),(l,d)} = V eta [delta_cd g_j.g_l + (g_j)_d (g_l)_c
                                //                              - 2/3 (g_j)_c (g_l)_d]
                                // hourglass term: eps delta_cd zeta_j zeta_l (delta_{lat_j, lat_l} - 1/3)
                                auto entry = [&](int d2, int cc) {
                                    double v = V * e * ((cc == d2 ? gg : 0.0) + gj[d2] * gl[cc] -
                                                        (2.0 / 3.0) * gj[cc] * gl[d2]);
                                    if (cc == d2)
                                        v += eps * (top ? 1.0 : -1.0) * (top2 ? 1.0 : -1.0) *
                                             ((lat == lat2 ? 1.0 : 0.0) - 1.0 / 3.0);
                                    return v;
                                };
                                double w[3];
                                for (int d2 = 0; d2 < 3; ++d2) {
                                    if (!pc) {
                                        w[d2] = entry(d2, ccomp);
                                    } else {
                                        w[d2] = 0.0;
                                        for (int cc = 0; cc < 3; ++cc)
                                            w[d2] += entry(d2, cc) * ((cc == ccomp ? 1.0 : 0.0) - nc[cc] * nc[ccomp]);
                                    }
                                }
                                if (on_fs(ck + top2)) {
                                    const double* nr = unit + 3 * ((((long long)q.d * (m + 1) + ci + cdi[wd][lat2]) *
                                                                    (m + 1)) + cj + cdj[wd][lat2]);
                                    const double dw = nr[0] * w[0] + nr[1] * w[1] + nr[2] * w[2];
                                    for (int a2 = 0; a2 < 3; ++a2) w[a2] -= dw * nr[a2];
                                }
                                for (int d2 = 0; d2 < 3; ++d2) {
                                    const int row = slot_dof[d2 * nslots + s2];
                                    if (row < 0) continue;
                                    Ad[(long long)col * nd + row] += w[d2];
                                }
                            }
                        }
                    }
                }
            }
        }
    }
    // the normal row of a free-slip node: + N e_c = rhat rhat_c, once per DoF
    {
        const int sc = copy_slot[copy_ptr[col]];
        const long long slot = sc >> 2;
        const int ccomp = sc & 3;
        const NodeIdx q = decode_node(slot, m, n);
        if (on_fs(q.k)) {
            const double* nc = unit + 3 * ((((long long)q.d * (m + 1) + q.i) * (m + 1)) + q.j);
            for (int a2 = 0; a2 < 3; ++a2) {
                const int row = slot_dof[a2 * nslots + slot];
                if (row >= 0) Ad[(long long)col * nd + row] += nc[a2] * nc[ccomp];
            }
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T>
void mg_diag_A(const tng_ctx* ctx, const Level& L, const T* eta, double hg_alpha, T* const d[3], bool twopt,
               unsigned fs) {
    require_unbatched("mg_diag_A");
    const long long ns = L.node_slots();
    diag_A_kernel<T><<<nblk(ns, 256), 256, 0, ctx->stream>>>(eta, L.geo64.p, L.m, L.n, L.r_in, L.dr(),
                                                             hg_alpha, twopt ? 1 : 0, (int)fs, L.unit64.p,
                                                             d[0], d[1], d[2], ns);
    TNG_HIP(hipGetLastError());
    void* f[3] = {d[0], d[1], d[2]};
    launch_interface(ctx, L, prec_of<T>(), 0, 3, f);
    diag_dirichlet_kernel<T><<<nblk(2 * L.lat_slots(), 256), 256, 0, ctx->stream>>>(L.lat_slots(), L.n, (int)fs,
                                                                                  d[0], d[1], d[2]);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void mg_pmass(const tng_ctx* ctx, const Level& L, const Level& Lp, const T* eta, T* mdiag) {
    require_unbatched("mg_pmass");
    const long long ns = Lp.node_slots();
    pmass_kernel<T><<<nblk(ns, 256), 256, 0, ctx->stream>>>(eta, L.geo64.p, L.m, L.n, L.r_in, L.dr(), mdiag, ns);
    TNG_HIP(hipGetLastError());
    void* f[1] = {mdiag};
    launch_interface(ctx, Lp, prec_of<T>(), 0, 1, f);
}

template <typename T>
void mg_prolong(const tng_ctx* ctx, const Level& Lf, const T* const c[3], T* const f[3], bool add) {
    const long long ns = Lf.node_slots();
    const SlotBatch sb = launch_batch();
    prolong_kernel<T><<<dim3(nblk(ns, 256), 1, sb.nb), 256, 0, ctx->stream>>>(Lf.m, Lf.n, c[0], c[1], c[2], f[0],
                                                                              f[1], f[2], add ? 1 : 0, ns, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void mg_restrict(const tng_ctx* ctx, const Level& Lf, const Level& Lc, const T* const f[3], T* const c[3],
                 unsigned fs) {
    const long long ns = Lc.node_slots();
    const T* im = std::is_same<T, double>::value ? (const T*)Lf.inv_mult64.p : (const T*)Lf.inv_mult32.p;
    const SlotBatch sb = launch_batch();
    restrict_kernel<T><<<dim3(nblk(ns, 256), 1, sb.nb), 256, 0, ctx->stream>>>(Lf.m, Lf.n, f[0], f[1], f[2], im,
                                                                               c[0], c[1], c[2], ns, (int)fs, sb);
    TNG_HIP(hipGetLastError());
    void* g[3] = {c[0], c[1], c[2]};
    launch_interface(ctx, Lc, prec_of<T>(), 0, 3, g);
    if (fs) vec_fs_project<T>(ctx, Lc, fs, c, nullptr);
}

template <typename T>
void vec_fs_project(const tng_ctx* ctx, const Level& L, unsigned fs, T* const x[3], const T* const b[3]) {
    if (!fs) return;
    require_unbatched("vec_fs_project");
    const T* un = std::is_same<T, double>::value ? (const T*)L.unit64.p : (const T*)L.unit32.p;
    fs_project_kernel<T><<<nblk(2 * L.lat_slots(), 256), 256, 0, ctx->stream>>>(
        L.lat_slots(), L.n, (int)fs, un, x[0], x[1], x[2], b ? b[0] : nullptr, b ? b[1] : nullptr,
        b ? b[2] : nullptr);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_cheb_update(const tng_ctx* ctx, long long n, const double* ab_dev, int k, const T* b, const T* y,
                     const T* invd, T* d, T* x) {
    const SlotBatch sb = launch_batch();
    if (aligned16(b) && aligned16(y) && aligned16(invd) && aligned16(d) && aligned16(x)) {
        const long long nv = n / (16 / (long long)sizeof(T));
        cheb_update_vec_kernel<T><<<dim3(std::max(1u, nblk(nv, 256)), 1, sb.nb), 256, 0, ctx->stream>>>(
            n, ab_dev, k, b, y, invd, d, x, sb);
        TNG_HIP(hipGetLastError());
        return;
    }
    cheb_update_kernel<T><<<dim3(nblk(n, 256 * EW_PER), 1, sb.nb), 256, 0, ctx->stream>>>(n, ab_dev, k, b, y, invd, d, x,
                                                                                  sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_cheb_post_update(const tng_ctx* ctx, const Level& L, bool ns_in, bool ns_out, const double* ab_dev, int k,
                          bool first, bool prev_zero, const T* b, const T* y, const T* invd, const T* xk, T* xo) {
    const SlotBatch sb = launch_batch();
    const long long ns = L.node_slots();
    TNG_REQUIRE(3 * ns < (1LL << 32), "smoother update: more than 2^32 values");
    TNG_REQUIRE(aligned16(b) && aligned16(y) && aligned16(invd) && aligned16(xk) && aligned16(xo),
                "smoother update: vectors must be 16-byte aligned");
    const long long nv = 3 * ns / (16 / (long long)sizeof(T));
    cheb_post_update_kernel<T><<<dim3(std::max(1u, nblk(nv, 256)), 1, sb.nb), 256, 0, ctx->stream>>>(
        (unsigned)ns, L.n + 1, magic_div((unsigned)ns), magic_div((unsigned)(L.n + 1)), L.lat_grp.p, L.grp_ptr.p,
        L.grp_slot.p, ns_in ? 1 : 0, ns_out ? 1 : 0, ab_dev, k, first ? 1 : 0, prev_zero ? 1 : 0, b, y, invd, xk, xo,
        sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_resid_post(const tng_ctx* ctx, const Level& L, bool ns_in, bool ns_out, const T* b, const T* x, const T* y,
                    T* r) {
    const SlotBatch sb = launch_batch();
    const long long ns = L.node_slots();
    resid_post_kernel<T><<<dim3(std::max(1u, nblk(ns, 256)), 3, sb.nb), 256, 0, ctx->stream>>>(
        (int)ns, L.n + 1, magic_div((unsigned)(L.n + 1)), L.lat_grp.p, L.grp_ptr.p, L.grp_slot.p, ns_in ? 1 : 0,
        ns_out ? 1 : 0, b, x, y, r, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_invert(const tng_ctx* ctx, long long n, T* a) {
    require_unbatched("vec_invert");
    invert_kernel<T><<<nblk(n, 256), 256, 0, ctx->stream>>>(n, a);
    TNG_HIP(hipGetLastError());
}

template <typename TO, typename TI>
void vec_cast(const tng_ctx* ctx, long long n, const TI* a, TO* b) {
    const SlotBatch sb = launch_batch();
    cast_kernel<TO, TI><<<dim3(nblk(n, 256), 1, sb.nb), 256, 0, ctx->stream>>>(n, a, b, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_axpby(const tng_ctx* ctx, long long n, double a, const T* x, double b, T* y) {
    const SlotBatch sb = launch_batch();
    if (aligned16(x) && aligned16(y)) {
        const long long nv = n / (16 / (long long)sizeof(T));
        axpby_vec_kernel<T><<<dim3(std::max(1u, nblk(nv, 256)), 1, sb.nb), 256, 0, ctx->stream>>>(n, T(a), x, T(b),
                                                                                                 y, sb);
        TNG_HIP(hipGetLastError());
        return;
    }
    axpby_kernel<T><<<dim3(nblk(n, 256 * EW_PER), 1, sb.nb), 256, 0, ctx->stream>>>(n, T(a), x, T(b), y, sb);
    TNG_HIP(hipGetLastError());
}

// smallest compiled vector count >= every slot's count
inline int count_class(const SlotBatch& sb, int nq) {
    int mx = nq;
    if (sb.has_cnt)
        for (int z = 0; z < sb.nb; ++z) mx = std::max(mx, sb.cnt[z]);
    return mx <= 1 ? 1 : mx <= 2 ? 2 : mx <= 4 ? 4 : mx <= 8 ? 8 : mx <= 12 ? 12 : mx <= 16 ? 16 : MAX_MDOT;
}

#define TNG_NQ_DISPATCH(NQV, CALL)                     \
    switch (NQV) {                                     \
        case 1: { constexpr int NQ = 1; CALL; } break;  \
        case 2: { constexpr int NQ = 2; CALL; } break;  \
        case 4: { constexpr int NQ = 4; CALL; } break;  \
        case 8: { constexpr int NQ = 8; CALL; } break;  \
        case 12: { constexpr int NQ = 12; CALL; } break; \
        case 16: { constexpr int NQ = 16; CALL; } break; \
        default: { constexpr int NQ = MAX_MDOT; CALL; } break; \
    }

template <typename T>
void vec_mdot(const tng_ctx* ctx, DotScratch& ds, long long n, int n1, long long nlat, const uint8_t* owner,
              const T* x, const T* const* vs_dev, int nq, double* out_dev, bool accumulate) {
    TNG_REQUIRE(nq >= 1 && nq <= MAX_MDOT, "too many vectors in a multi-dot");
    TNG_REQUIRE(n <= 3LL * nlat * n1 && n < (1LL << 32), "multi-dot length out of range");
    const int nb = (int)std::min<long long>(DOT_BLOCKS, (n + DOT_BS - 1) / DOT_BS);
    const SlotBatch sb = launch_batch();
    check_counts(sb);
    const MagicDiv dn1 = magic_div((unsigned)n1);
    TNG_NQ_DISPATCH(count_class(sb, nq),
                    (mdot_partial_kernel<T, NQ><<<dim3(nb, 1, sb.nb), DOT_BS, 0, ctx->stream>>>(
                        (unsigned)n, dn1, (unsigned)nlat, owner, x, vs_dev, nq, ds.part.p, sb)));
    TNG_HIP(hipGetLastError());
    mdot_final_kernel<<<dim3(1, 1, sb.nb), 256, 0, ctx->stream>>>(nb, nq, ds.part.p, out_dev, accumulate ? 1 : 0, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_maxpy(const tng_ctx* ctx, long long n, const double* coef_dev, double sign, const T* const* vs_dev,
               int nq, T* y) {
    TNG_REQUIRE(nq >= 1 && nq <= MAX_MDOT, "too many vectors in a multi-axpy");
    const unsigned nb = (unsigned)std::min<long long>(nblk(n, 256), 8192);
    const SlotBatch sb = launch_batch();
    check_counts(sb);
    TNG_NQ_DISPATCH(count_class(sb, nq),
                    (maxpy_kernel<T, NQ><<<dim3(nb, 1, sb.nb), 256, 0, ctx->stream>>>((unsigned)n, coef_dev, sign,
                                                                                      vs_dev, nq, y, sb)));
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_smdot(const tng_ctx* ctx, DotScratch& ds, const Level& Lu, const Level& Lp, const T* x,
               const T* const* vs_dev, int nq, double* out_dev, bool accumulate, bool vs_aligned) {
    TNG_REQUIRE(nq >= 1 && nq <= MAX_MDOT, "too many vectors in a multi-dot");
    const long long n = 3 * Lu.node_slots() + Lp.node_slots();
    TNG_REQUIRE(n < (1LL << 32), "multi-dot length out of range");
    const SlotBatch sb = launch_batch();
    check_counts(sb);
    const MagicDiv du = magic_div((unsigned)(Lu.n + 1)), dp = magic_div((unsigned)(Lp.n + 1));
    // 16-byte accesses pay in FP32 (four values per load); the FP64 kernel already streams at
    // about 5.6 TB/s with its two 8-byte loads per vector and step
    if (sizeof(T) == 4 && vs_aligned && aligned16(x)) {
        const long long nv = n / (16 / (long long)sizeof(T));
        const int nb = (int)std::max<long long>(1, std::min<long long>(DOT_BLOCKS, (nv + DOT_BS - 1) / DOT_BS));
        TNG_NQ_DISPATCH(count_class(sb, nq), (smdot_vec_kernel<T, NQ><<<dim3(nb, 1, sb.nb), DOT_BS, 0, ctx->stream>>>(
                                (unsigned)Lu.node_slots(), du, (unsigned)Lu.lat_slots(), Lu.owner.p,
                                (unsigned)Lp.node_slots(), dp, Lp.owner.p, x, vs_dev, nq, ds.part.p, sb)));
        TNG_HIP(hipGetLastError());
        mdot_final_kernel<<<dim3(1, 1, sb.nb), 256, 0, ctx->stream>>>(nb, nq, ds.part.p, out_dev,
                                                                      accumulate ? 1 : 0, sb);
        TNG_HIP(hipGetLastError());
        return;
    }
    const int nb = (int)std::min<long long>(DOT_BLOCKS, (n + DOT_BS - 1) / DOT_BS);
    TNG_NQ_DISPATCH(count_class(sb, nq),
                    (smdot_partial_kernel<T, NQ><<<dim3(nb, 1, sb.nb), DOT_BS, 0, ctx->stream>>>(
                        (unsigned)Lu.node_slots(), du, (unsigned)Lu.lat_slots(), Lu.owner.p,
                        (unsigned)Lp.node_slots(), dp, Lp.owner.p, x, vs_dev, nq, ds.part.p, sb)));
    TNG_HIP(hipGetLastError());
    mdot_final_kernel<<<dim3(1, 1, sb.nb), 256, 0, ctx->stream>>>(nb, nq, ds.part.p, out_dev, accumulate ? 1 : 0, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_maxpy_smdot(const tng_ctx* ctx, DotScratch& ds, const Level& Lu, const Level& Lp, const double* coef_dev,
                     double sign, const T* const* vs_dev, int nq, T* y, double* out_dev, bool norm, bool vs_aligned) {
    TNG_REQUIRE(nq >= 1 && nq <= MAX_MDOT, "too many vectors in a multi-axpy");
    const long long n = 3 * Lu.node_slots() + Lp.node_slots();
    TNG_REQUIRE(n < (1LL << 32), "vector length out of range");
    const SlotBatch sb = launch_batch();
    check_counts(sb);
    const MagicDiv du = magic_div((unsigned)(Lu.n + 1)), dp = magic_div((unsigned)(Lp.n + 1));
    if (sizeof(T) == 4 && vs_aligned && aligned16(y)) {
        const long long nv = n / (16 / (long long)sizeof(T));
        const int nb = (int)std::max<long long>(1, std::min<long long>(DOT_BLOCKS, (nv + DOT_BS - 1) / DOT_BS));
        const dim3 grid(nb, 1, sb.nb);
        if (norm) {
            TNG_NQ_DISPATCH(count_class(sb, nq), (maxpy_dot_vec_kernel<T, NQ, true><<<grid, DOT_BS, 0, ctx->stream>>>(
                                    (unsigned)Lu.node_slots(), du, (unsigned)Lu.lat_slots(), Lu.owner.p,
                                    (unsigned)Lp.node_slots(), dp, Lp.owner.p, coef_dev, sign, vs_dev, nq, y,
                                    ds.part.p, sb)));
        } else {
            TNG_NQ_DISPATCH(count_class(sb, nq), (maxpy_dot_vec_kernel<T, NQ, false><<<grid, DOT_BS, 0, ctx->stream>>>(
                                    (unsigned)Lu.node_slots(), du, (unsigned)Lu.lat_slots(), Lu.owner.p,
                                    (unsigned)Lp.node_slots(), dp, Lp.owner.p, coef_dev, sign, vs_dev, nq, y,
                                    ds.part.p, sb)));
        }
        TNG_HIP(hipGetLastError());
        // the norm has one value for every slot: the per-slot counts do not apply to it
        SlotBatch sf = sb;
        if (norm) sf.has_cnt = 0;
        mdot_final_kernel<<<dim3(1, 1, sf.nb), 256, 0, ctx->stream>>>(nb, norm ? 1 : nq, ds.part.p, out_dev, 0, sf);
        TNG_HIP(hipGetLastError());
        return;
    }
    const int nb = (int)std::min<long long>(DOT_BLOCKS, (n + DOT_BS - 1) / DOT_BS);
    if (norm) {
        TNG_NQ_DISPATCH(count_class(sb, nq),
                        (maxpy_dot_kernel<T, NQ, true><<<dim3(nb, 1, sb.nb), DOT_BS, 0, ctx->stream>>>(
                            (unsigned)Lu.node_slots(), du, (unsigned)Lu.lat_slots(), Lu.owner.p,
                            (unsigned)Lp.node_slots(), dp, Lp.owner.p, coef_dev, sign, vs_dev, nq, y, ds.part.p, sb)));
    } else {
        TNG_NQ_DISPATCH(count_class(sb, nq),
                        (maxpy_dot_kernel<T, NQ, false><<<dim3(nb, 1, sb.nb), DOT_BS, 0, ctx->stream>>>(
                            (unsigned)Lu.node_slots(), du, (unsigned)Lu.lat_slots(), Lu.owner.p,
                            (unsigned)Lp.node_slots(), dp, Lp.owner.p, coef_dev, sign, vs_dev, nq, y, ds.part.p, sb)));
    }
    TNG_HIP(hipGetLastError());
    // the norm has one value for every slot: the per-slot counts do not apply to it
    SlotBatch sf = sb;
    if (norm) sf.has_cnt = 0;
    mdot_final_kernel<<<dim3(1, 1, sf.nb), 256, 0, ctx->stream>>>(nb, norm ? 1 : nq, ds.part.p, out_dev, 0, sf);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_rand(const tng_ctx* ctx, long long n, unsigned long long seed, T* a) {
    require_unbatched("vec_rand");
    const unsigned nb = (unsigned)std::min<long long>(nblk(n, 256), 8192);
    rand_kernel<T><<<nb, 256, 0, ctx->stream>>>((unsigned)n, seed, a);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_scale_rsqrt(const tng_ctx* ctx, long long n, const double* s, const T* x, T* y) {
    const unsigned nb = (unsigned)std::min<long long>(nblk(n, 256), 8192);
    const SlotBatch sb = launch_batch();
    scale_rsqrt_kernel<T><<<dim3(nb, 1, sb.nb), 256, 0, ctx->stream>>>((unsigned)n, s, x, y, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_tab_copy(const tng_ctx* ctx, long long n, const T* src, const T* const* src_tab, T* dst, T* const* dst_tab,
                  int idx, const double* sq) {
    const SlotBatch sb = launch_batch();
    const unsigned nb = (unsigned)std::min<long long>(nblk(n, 256), 8192);
    tab_copy_kernel<T><<<dim3(nb, 1, sb.nb), 256, 0, ctx->stream>>>((unsigned)n, src, src_tab, dst, dst_tab, idx,
                                                                     sq, sb);
    TNG_HIP(hipGetLastError());
}

void scal_gather(const tng_ctx* ctx, const double* src, int k, double* staging) {
    const SlotBatch sb = launch_batch();
    scal_gather_kernel<<<dim3(1, 1, sb.nb), 64, 0, ctx->stream>>>(src, k, staging, sb);
    TNG_HIP(hipGetLastError());
}

void scal_scatter(const tng_ctx* ctx, const double* staging, int k, double* dst) {
    const SlotBatch sb = launch_batch();
    scal_scatter_kernel<<<dim3(1, 1, sb.nb), 64, 0, ctx->stream>>>(staging, k, dst, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void coarse_assemble(const tng_ctx* ctx, const CoarseDense& cd, const Level& L, const T* eta, double hg_alpha,
                     bool twopt, unsigned fs) {
    require_unbatched("coarse_assemble");
    coarse_assemble_kernel<T><<<nblk(cd.ndof, 64), 64, 0, ctx->stream>>>(
        cd.ndof, cd.copy_ptr.p, cd.copy_slot.p, cd.slot_dof.p, cd.nslots, eta, L.geo64.p, L.m, L.n, L.r_in,
        L.dr(), hg_alpha, twopt ? 1 : 0, (int)fs, L.unit64.p, cd.Ainv.p);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_mul(const tng_ctx* ctx, long long n, const T* a, const T* b, T* c) {
    require_unbatched("vec_mul");
    const unsigned nb = (unsigned)std::min<long long>(nblk(n, 256), 8192);
    mul_kernel<T><<<nb, 256, 0, ctx->stream>>>((unsigned)n, a, b, c);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_fill(const tng_ctx* ctx, long long n, T v, T* a) {
    if (n <= 0) return;
    const unsigned nb = (unsigned)std::min<long long>(nblk(n, 256), 8192);
    const SlotBatch sb = launch_batch();
    fillv_kernel<T><<<dim3(nb, 1, sb.nb), 256, 0, ctx->stream>>>((unsigned)n, v, a, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void coarse_unit(const tng_ctx* ctx, const CoarseDense& cd, int col, T* const x[3]) {
    require_unbatched("coarse_unit");
    unit_vector_kernel<T><<<nblk(3 * cd.nslots, 256), 256, 0, ctx->stream>>>(cd.nslots, cd.slot_dof.p, col, x[0],
                                                                             x[1], x[2]);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void coarse_gather(const tng_ctx* ctx, const CoarseDense& cd, int col, const T* const y[3], double* Ad) {
    require_unbatched("coarse_gather");
    coarse_gather_col_kernel<T><<<nblk(cd.ndof, 256), 256, 0, ctx->stream>>>(cd.ndof, cd.dof_slot.p, y[0], y[1],
                                                                              y[2], col, Ad);
    TNG_HIP(hipGetLastError());
}

void coarse_rotation_shift(const tng_ctx* ctx, CoarseDense& cd, const Level& L) {
    require_unbatched("coarse_rotation_shift");
    if (cd.rotq.n != (size_t)(3 * cd.ndof + 1)) cd.rotq.alloc(3 * cd.ndof + 1);
    coarse_rotation_basis_kernel<<<1, 1, 0, ctx->stream>>>(cd.ndof, cd.dof_slot.p, L.m, L.n, L.r_in, L.dr(),
                                                         L.unit64.p, cd.Ainv.p, cd.rotq.p);
    TNG_HIP(hipGetLastError());
    coarse_rotation_shift_kernel<<<nblk(cd.ndof, 64), 64, 0, ctx->stream>>>(cd.ndof, cd.rotq.p, cd.Ainv.p);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_rotation(const tng_ctx* ctx, const Level& L, int a, T* const out[3]) {
    require_unbatched("vec_rotation");
    const long long ns = L.node_slots();
    rotation_fill_kernel<T><<<nblk(ns, 256), 256, 0, ctx->stream>>>(L.m, L.n, L.r_in, L.dr(), L.unit64.p, a, out[0],
                                                                   out[1], out[2], ns);
    TNG_HIP(hipGetLastError());
}

void coarse_invert(const tng_ctx* ctx, CoarseDense& cd) {
    require_unbatched("coarse_invert");
    gauss_jordan_kernel<<<1, 1024, 0, ctx->stream>>>(cd.ndof, cd.Ainv.p);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void coarse_solve(const tng_ctx* ctx, const CoarseDense& cd, const T* const b[3], T* const x[3]) {
    const SlotBatch sb = launch_batch();
    coarse_solve_kernel<T><<<dim3(1, 1, sb.nb), 1024, 0, ctx->stream>>>(
        cd.ndof, cd.dof_slot.p, cd.slot_dof.p, cd.nslots, cd.Ainv.p, b[0], b[1], b[2], x[0], x[1], x[2], sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_shift(const tng_ctx* ctx, long long n, const double* sum_cnt, T* p) {
    const SlotBatch sb = launch_batch();
    shift_kernel<T><<<dim3(nblk(n, 256), 1, sb.nb), 256, 0, ctx->stream>>>(n, sum_cnt, p, sb);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void vec_schur(const tng_ctx* ctx, long long n, const T* r, const T* mdiag, T* z) {
    const SlotBatch sb = launch_batch();
    schur_diag_kernel<T><<<dim3(nblk(n, 256), 1, sb.nb), 256, 0, ctx->stream>>>(n, r, mdiag, z, sb);
    TNG_HIP(hipGetLastError());
}

#define TNG_INST(T)                                                                                        \
    template void mg_diag_A<T>(const tng_ctx*, const Level&, const T*, double, T* const[3], bool, unsigned);      \
    template void vec_fs_project<T>(const tng_ctx*, const Level&, unsigned, T* const[3], const T* const[3]);      \
    template void vec_rotation<T>(const tng_ctx*, const Level&, int, T* const[3]);                                \
    template void mg_pmass<T>(const tng_ctx*, const Level&, const Level&, const T*, T*);                  \
    template void mg_prolong<T>(const tng_ctx*, const Level&, const T* const[3], T* const[3], bool);      \
    template void mg_restrict<T>(const tng_ctx*, const Level&, const Level&, const T* const[3],           \
                                 T* const[3], unsigned);                                                   \
    template void vec_resid_post<T>(const tng_ctx*, const Level&, bool, bool, const T*, const T*, const T*, T*); \
    template void vec_cheb_post_update<T>(const tng_ctx*, const Level&, bool, bool, const double*, int, bool,   \
                                          bool, const T*, const T*, const T*, const T*, T*);                 \
    template void vec_cheb_update<T>(const tng_ctx*, long long, const double*, int, const T*, const T*,   \
                                     const T*, T*, T*);                                                    \
    template void vec_invert<T>(const tng_ctx*, long long, T*);                                           \
    template void vec_axpby<T>(const tng_ctx*, long long, double, const T*, double, T*);                  \
    template void vec_mdot<T>(const tng_ctx*, DotScratch&, long long, int, long long, const uint8_t*,     \
                              const T*, const T* const*, int, double*, bool);                              \
    template void coarse_unit<T>(const tng_ctx*, const CoarseDense&, int, T* const[3]);                   \
    template void coarse_gather<T>(const tng_ctx*, const CoarseDense&, int, const T* const[3], double*);  \
    template void coarse_solve<T>(const tng_ctx*, const CoarseDense&, const T* const[3], T* const[3]);    \
    template void vec_shift<T>(const tng_ctx*, long long, const double*, T*);                             \
    template void vec_schur<T>(const tng_ctx*, long long, const T*, const T*, T*);                       \
    template void vec_maxpy<T>(const tng_ctx*, long long, const double*, double, const T* const*, int, T*); \
    template void vec_fill<T>(const tng_ctx*, long long, T, T*);                                          \
    template void vec_mul<T>(const tng_ctx*, long long, const T*, const T*, T*);                          \
    template void vec_smdot<T>(const tng_ctx*, DotScratch&, const Level&, const Level&, const T*,         \
                               const T* const*, int, double*, bool, bool);                                 \
    template void vec_maxpy_smdot<T>(const tng_ctx*, DotScratch&, const Level&, const Level&, const double*,  \
                                     double, const T* const*, int, T*, double*, bool, bool);                 \
    template void vec_rand<T>(const tng_ctx*, long long, unsigned long long, T*);                         \
    template void vec_scale_rsqrt<T>(const tng_ctx*, long long, const double*, const T*, T*);             \
    template void vec_tab_copy<T>(const tng_ctx*, long long, const T*, const T* const*, T*, T* const*, int, \
                                  const double*);                                                          \
    template void coarse_assemble<T>(const tng_ctx*, const CoarseDense&, const Level&, const T*, double, bool,  \
                                     unsigned);
TNG_INST(double)
TNG_INST(float)
#undef TNG_INST
template void vec_cast<float, double>(const tng_ctx*, long long, const double*, float*);
template void vec_cast<double, float>(const tng_ctx*, long long, const float*, double*);
template void vec_cast<float, float>(const tng_ctx*, long long, const float*, float*);
template void vec_cast<double, double>(const tng_ctx*, long long, const double*, double*);

}  // namespace tng
