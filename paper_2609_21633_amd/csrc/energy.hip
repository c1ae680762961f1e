// Energy equation kernels (Sec. 1 eq:energy in Boussinesq form, Sec. 6 scheme
// list: SUPG-stabilised Galerkin) and the buoyancy right-hand side of
// eq:stokes, all with the one-point rule of Sec. 4.
//
// Per wedge e at q_c: V_e, basis gradients grad phi_j, the mean velocity
// ubar = (1/6) sum_j u_j, and the SUPG parameter
//   tau_e = h_e / (2 |ubar|) (coth Pe - 1/Pe),  Pe = |ubar| h_e / 2,  h_e = V_e^(1/3)
// (unit diffusivity).  The backward-Euler operator on a temperature T is
//   (E T)_i = sum_e V_e [ N_i T_i / dt + grad phi_i . grad T
//                          + N_i ubar . grad T + tau (ubar . grad phi_i)(ubar . grad T) ]
// with N_i(q_c) = 1/6, i.e. lumped mass, diffusion, advection and streamline
// diffusion.  Every kernel gathers over the wedges around a node (no atomics)
// and produces per-diamond partial sums that the interface pass completes.
#include <cstdio>
#include <type_traits>

#include "mg.hpp"
#include "tng_internal.hpp"

namespace tng {
namespace {

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct NodeIdx4 {
    int d, i, j, k;
};
__device__ __forceinline__ NodeIdx4 decode4(long long t, int m, int n) {
    NodeIdx4 r;
    r.k = (int)(t % (n + 1));
    t /= (n + 1);
    r.j = (int)(t % (m + 1));
    t /= (m + 1);
    r.i = (int)(t % (m + 1));
    r.d = (int)(t / (m + 1));
    return r;
}

// lateral offsets of the three nodes of wedge 0 / wedge 1 in a cell
__constant__ int c_cdi[2][3] = {{0, 1, 0}, {1, 0, 1}};
__constant__ int c_cdj[2][3] = {{0, 0, 1}, {1, 1, 0}};

__device__ __forceinline__ void grad_of(const double* g, double s1, int lat, int top, double out[3]) {
    const double a = lat == 0 ? -1.0 : (lat == 1 ? 1.0 : 0.0);
    const double b = lat == 0 ? -1.0 : (lat == 2 ? 1.0 : 0.0);
    const double c = top ? 1.0 : -1.0;
    for (int x = 0; x < 3; ++x) out[x] = a * s1 * g[x] + b * s1 * g[3 + x] + c * g[6 + x];
}

__device__ __forceinline__ double supg_tau(double unorm, double h) {
    const double pe = 0.5 * unorm * h;
    // coth(Pe) - 1/Pe = Pe/3 - Pe^3/45 + ... ; tau = h/(2|u|) (coth Pe - 1/Pe)
    if (pe < 1e-3) return h * h / 12.0 * (1.0 - pe * pe / 15.0);
    return h / (2.0 * unorm) * (1.0 / tanh(pe) - 1.0 / pe);
}

// Wedges around node (q.d, q.i, q.j, q.k): calls f(ci, cj, ck, wd, lat, top)
// for every wedge having the node as local vertex (lat, top).
template <typename F>
__device__ __forceinline__ void for_node_wedges(const NodeIdx4& q, int m, int n, F&& f) {
    for (int ci = q.i - 1; ci <= q.i; ++ci) {
        if (ci < 0 || ci >= m) continue;
        for (int cj = q.j - 1; cj <= q.j; ++cj) {
            if (cj < 0 || cj >= m) continue;
            const int di = q.i - ci, dj = q.j - cj;
            for (int ck = q.k - 1; ck <= q.k; ++ck) {
                if (ck < 0 || ck >= n) continue;
                const int top = q.k - ck;
                for (int wd = 0; wd < 2; ++wd) {
                    int lat = -1;
                    for (int l = 0; l < 3; ++l)
                        if (c_cdi[wd][l] == di && c_cdj[wd][l] == dj) lat = l;
                    if (lat >= 0) f(ci, cj, ck, wd, lat, top);
                }
            }
        }
    }
}

struct EnergyGeo {
    const double* geo;
    int m, n;
    double r_in, dr;
};

template <typename T>
struct WedgeField {
    // gathers the six nodal values of a field for wedge (d, ci, cj, ck, wd)
    __device__ __forceinline__ static void gather(const T* f, int d, int ci, int cj, int ck, int wd, int m, int n,
                                                  double v[6]) {
        for (int l = 0; l < 6; ++l) {
            const int lat = l % 3, top = l / 3;
            const long long s = (((long long)d * (m + 1) + ci + c_cdi[wd][lat]) * (m + 1) + cj + c_cdj[wd][lat]) *
                                    (n + 1) + ck + top;
            v[l] = (double)f[s];
        }
    }
};

// Flow data of every wedge for the SUPG operator, which depends on the velocity
// only: ubar (3 values) and tau at q_c, FP64, [10][m][m][n][2][4].  Computed once
// per velocity field instead of once per node of the wedge in every apply.
constexpr int WF = 4;
template <typename T>
__global__ void wedge_flow_kernel(EnergyGeo G, const T* __restrict__ u0, const T* __restrict__ u1,
                                  const T* __restrict__ u2, double* __restrict__ wf, long long ncells) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncells) return;
    const int m = G.m, n = G.n;
    const int ck = (int)(c % n);
    long long r = c / n;
    const int cj = (int)(r % m);
    r /= m;
    const int ci = (int)(r % m);
    const int d = (int)(r / m);
    const double rm = G.r_in + (ck + 0.5) * G.dr;
    for (int wd = 0; wd < 2; ++wd) {
        const double* g = G.geo + (((long long)d * m + ci) * m + cj) * GEO_PER_COL + wd * GEO_PER_TRI;
        const double V = rm * rm * g[9];
        double uu[3][6];
        WedgeField<T>::gather(u0, d, ci, cj, ck, wd, m, n, uu[0]);
        WedgeField<T>::gather(u1, d, ci, cj, ck, wd, m, n, uu[1]);
        WedgeField<T>::gather(u2, d, ci, cj, ck, wd, m, n, uu[2]);
        double ub[3];
        for (int x = 0; x < 3; ++x)
            ub[x] = (uu[x][0] + uu[x][1] + uu[x][2] + uu[x][3] + uu[x][4] + uu[x][5]) * (1.0 / 6.0);
        const double un = sqrt(ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
        double* w = wf + (c * 2 + wd) * WF;
        w[0] = ub[0];
        w[1] = ub[1];
        w[2] = ub[2];
        w[3] = supg_tau(un, cbrt(V));
    }
}

// y = E T (mode 0), or the diagonal of E (mode 1).  Dirichlet rows handled later.
template <typename T, int MODE>
__global__ void energy_node_kernel(EnergyGeo G, const T* __restrict__ Tin, const double* __restrict__ wf,
                                   double inv_dt, T* __restrict__ y, long long nslots) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const NodeIdx4 q = decode4(t, G.m, G.n);
    const int m = G.m, n = G.n;
    double acc = 0.0;
    for_node_wedges(q, m, n, [&](int ci, int cj, int ck, int wd, int lat, int top) {
        const double* g = G.geo + (((long long)q.d * m + ci) * m + cj) * GEO_PER_COL + wd * GEO_PER_TRI;
        const double rm = G.r_in + (ck + 0.5) * G.dr;
        const double s1 = 0.5 / rm;
        const double V = rm * rm * g[9];
        const double* w = wf + (((((long long)q.d * m + ci) * m + cj) * n + ck) * 2 + wd) * WF;
        const double ub[3] = {w[0], w[1], w[2]};
        const double tau = w[3];
        double gi[3];
        grad_of(g, s1, lat, top, gi);
        const double ugi = ub[0] * gi[0] + ub[1] * gi[1] + ub[2] * gi[2];
        if (MODE == 0) {
            double Tv[6];
            WedgeField<T>::gather(Tin, q.d, ci, cj, ck, wd, m, n, Tv);
            // grad T = A rho1~ + B rho2~ + C rho3' with nodal differences
            const double A = Tv[1] + Tv[4] - Tv[0] - Tv[3];
            const double B = Tv[2] + Tv[5] - Tv[0] - Tv[3];
            const double C = Tv[3] + Tv[4] + Tv[5] - Tv[0] - Tv[1] - Tv[2];
            double gT[3];
            for (int x = 0; x < 3; ++x) gT[x] = A * s1 * g[x] + B * s1 * g[3 + x] + C * g[6 + x];
            const double a = ub[0] * gT[0] + ub[1] * gT[1] + ub[2] * gT[2];
            const double Ti = Tv[lat + 3 * top];
            acc += V * ((1.0 / 6.0) * Ti * inv_dt + gi[0] * gT[0] + gi[1] * gT[1] + gi[2] * gT[2] +
                        (1.0 / 6.0) * a + tau * ugi * a);
        } else {
            // diagonal: T = e_i, grad T = grad phi_i
            acc += V * ((1.0 / 6.0) * inv_dt + gi[0] * gi[0] + gi[1] * gi[1] + gi[2] * gi[2] +
                        (1.0 / 6.0) * ugi + tau * ugi * ugi);
        }
    });
    y[t] = T(acc);
}

// b_i = m_i (T_i / dt + H_i), m_i = sum_e V_e / 6 (lumped mass)
template <typename T>
__global__ void energy_rhs_kernel(EnergyGeo G, const T* __restrict__ Tn, const T* __restrict__ H, double inv_dt,
                                  T* __restrict__ b, long long nslots) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const NodeIdx4 q = decode4(t, G.m, G.n);
    double mass = 0.0;
    for_node_wedges(q, G.m, G.n, [&](int ci, int cj, int ck, int wd, int, int) {
        const double* g = G.geo + (((long long)q.d * G.m + ci) * G.m + cj) * GEO_PER_COL + wd * GEO_PER_TRI;
        const double rm = G.r_in + (ck + 0.5) * G.dr;
        mass += rm * rm * g[9] / 6.0;
    });
    b[t] = T(mass * ((double)Tn[t] * inv_dt + (H ? (double)H[t] : 0.0)));
}

// Buoyancy f_(i,c) = sum_e V_e N_i(q_c) Ra T(q_c) rhat_c(q_c), rhat the
// direction of x(q_c) = r_m s_c (s_c the mean of the triangle's unit vectors).
template <typename T>
__global__ void buoyancy_kernel(EnergyGeo G, const double* __restrict__ unit, const T* __restrict__ Tn, double Ra,
                                T* f0, T* f1, T* f2, long long nslots, const double* __restrict__ tbar,
                                const double* __restrict__ rhoalpha) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const int m = G.m, n = G.n;
    const NodeIdx4 q = decode4(t, m, n);
    double acc[3] = {0, 0, 0};
    for_node_wedges(q, m, n, [&](int ci, int cj, int ck, int wd, int, int) {
        const double* g = G.geo + (((long long)q.d * m + ci) * m + cj) * GEO_PER_COL + wd * GEO_PER_TRI;
        const double rm = G.r_in + (ck + 0.5) * G.dr;
        const double V = rm * rm * g[9];
        double Tv[6];
        WedgeField<T>::gather(Tn, q.d, ci, cj, ck, wd, m, n, Tv);
        double Tq = (Tv[0] + Tv[1] + Tv[2] + Tv[3] + Tv[4] + Tv[5]) * (1.0 / 6.0);
        if (tbar) {
            // compressible form: T' = T - Tbar(r) and rhobar alphabar, W1 in the radius
            Tq = (Tq - 0.5 * (tbar[ck] + tbar[ck + 1])) * (0.5 * (rhoalpha[ck] + rhoalpha[ck + 1]));
        }
        double sc[3] = {0, 0, 0};
        for (int l = 0; l < 3; ++l) {
            const long long lat = ((long long)q.d * (m + 1) + ci + c_cdi[wd][l]) * (m + 1) + cj + c_cdj[wd][l];
            for (int x = 0; x < 3; ++x) sc[x] += unit[lat * 3 + x];
        }
        const double nn = 1.0 / sqrt(sc[0] * sc[0] + sc[1] * sc[1] + sc[2] * sc[2]);
        const double w = V * (1.0 / 6.0) * Ra * Tq * nn;
        for (int x = 0; x < 3; ++x) acc[x] += w * sc[x];
    });
    f0[t] = T(acc[0]);
    f1[t] = T(acc[1]);
    f2[t] = T(acc[2]);
}

// CFL data: per block max of |ubar_e| / h_e over wedges (deterministic max)
template <typename T>
__global__ void cfl_kernel(EnergyGeo G, const T* __restrict__ u0, const T* __restrict__ u1,
                           const T* __restrict__ u2, double* __restrict__ part, long long ncells) {
    __shared__ double sh[256];
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = G.m, n = G.n;
    double best = 0.0;
    if (t < ncells) {
        const int ck = (int)(t % n);
        long long r = t / n;
        const int cj = (int)(r % m);
        r /= m;
        const int ci = (int)(r % m);
        const int d = (int)(r / m);
        const double rm = G.r_in + (ck + 0.5) * G.dr;
        for (int wd = 0; wd < 2; ++wd) {
            const double* g = G.geo + (((long long)d * m + ci) * m + cj) * GEO_PER_COL + wd * GEO_PER_TRI;
            const double V = rm * rm * g[9];
            double uu[3][6];
            WedgeField<T>::gather(u0, d, ci, cj, ck, wd, m, n, uu[0]);
            WedgeField<T>::gather(u1, d, ci, cj, ck, wd, m, n, uu[1]);
            WedgeField<T>::gather(u2, d, ci, cj, ck, wd, m, n, uu[2]);
            double ub[3];
            for (int c = 0; c < 3; ++c)
                ub[c] = (uu[c][0] + uu[c][1] + uu[c][2] + uu[c][3] + uu[c][4] + uu[c][5]) * (1.0 / 6.0);
            const double v = sqrt(ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]) / cbrt(V);
            best = fmax(best, v);
        }
    }
    sh[threadIdx.x] = best;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Dirichlet temperature rows: value v0 on k = 0 (inner sphere), v1 on k = n
template <typename T>
__global__ void set_layers_kernel(long long ncol, int n, T* y, const T* src, double v0, double v1) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * ncol) return;
    const long long idx = (t >> 1) * (n + 1) + ((t & 1) ? n : 0);
    y[idx] = src ? src[idx] : T((t & 1) ? v1 : v0);
}

// velocity Dirichlet rows of a vector field to zero (fs: free-slip spheres, bit 0 inner,
// bit 1 outer, whose layers are left alone)
template <typename T>
__global__ void zero_layers3_kernel(long long ncol, int n, int fs, T* a0, T* a1, T* a2) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * ncol) return;
    if ((t & 1) ? (fs & 2) : (fs & 1)) return;
    const long long idx = (t >> 1) * (n + 1) + ((t & 1) ? n : 0);
    a0[idx] = T(0);
    a1[idx] = T(0);
    a2[idx] = T(0);
}

EnergyGeo make_geo(const Level& L) { return EnergyGeo{L.geo64.p, L.m, L.n, L.r_in, L.dr()}; }

}  // namespace

template <typename T>
void energy_wedge_flow(const tng_ctx* ctx, const Level& L, const T* const u[3], double* wf) {
    require_unbatched("energy_wedge_flow");
    const long long nc = L.cells();
    wedge_flow_kernel<T><<<nblk(nc, 256), 256, 0, ctx->stream>>>(make_geo(L), u[0], u[1], u[2], wf, nc);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void energy_apply_wf(const tng_ctx* ctx, const Level& L, const double* wf, double dt, const T* Tin, T* y) {
    require_unbatched("energy_apply");
    const long long ns = L.node_slots();
    {
        char detail[48] = {0};
        if (ctx->profile)
            std::snprintf(detail, sizeof(detail), "%s/SUPG/%dx%d", std::is_same<T, double>::value ? "f64" : "f32",
                          L.m, L.n);
        ScopedKernelTimer timer(ctx, "energy_apply", detail);
        energy_node_kernel<T, 0><<<nblk(ns, 256), 256, 0, ctx->stream>>>(make_geo(L), Tin, wf, 1.0 / dt, y, ns);
        TNG_HIP(hipGetLastError());
    }
    void* f[1] = {y};
    launch_interface(ctx, L, prec_of<T>(), 0, 1, f);
    set_layers_kernel<T><<<nblk(2 * L.lat_slots(), 256), 256, 0, ctx->stream>>>(L.lat_slots(), L.n, y, Tin, 0, 0);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void energy_apply(const tng_ctx* ctx, const Level& L, const T* const u[3], double dt, const T* Tin, T* y) {
    if (energy_stream_fits(L)) {
        energy_apply_stream<T>(ctx, L, u, dt, Tin, y);
        return;
    }
    DevBuf<double> wf((size_t)L.cells() * 2 * WF);
    energy_wedge_flow<T>(ctx, L, u, wf.p);
    energy_apply_wf<T>(ctx, L, wf.p, dt, Tin, y);
    TNG_HIP(hipStreamSynchronize(ctx->stream));   // wf is freed on return
}

template <typename T>
void energy_diag(const tng_ctx* ctx, const Level& L, const double* wf, double dt, T* diag) {
    require_unbatched("energy_diag");
    const long long ns = L.node_slots();
    energy_node_kernel<T, 1><<<nblk(ns, 256), 256, 0, ctx->stream>>>(make_geo(L), nullptr, wf, 1.0 / dt, diag, ns);
    TNG_HIP(hipGetLastError());
    void* f[1] = {diag};
    launch_interface(ctx, L, prec_of<T>(), 0, 1, f);
    set_layers_kernel<T><<<nblk(2 * L.lat_slots(), 256), 256, 0, ctx->stream>>>(L.lat_slots(), L.n, diag, nullptr,
                                                                               1.0, 1.0);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void energy_rhs(const tng_ctx* ctx, const Level& L, const T* Tn, const T* H, double dt, double T_in,
                double T_out, T* b) {
    const long long ns = L.node_slots();
    energy_rhs_kernel<T><<<nblk(ns, 256), 256, 0, ctx->stream>>>(make_geo(L), Tn, H, 1.0 / dt, b, ns);
    TNG_HIP(hipGetLastError());
    void* f[1] = {b};
    launch_interface(ctx, L, prec_of<T>(), 0, 1, f);
    set_layers_kernel<T><<<nblk(2 * L.lat_slots(), 256), 256, 0, ctx->stream>>>(L.lat_slots(), L.n, b, nullptr,
                                                                               T_in, T_out);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void buoyancy_rhs(const tng_ctx* ctx, const Level& L, const T* Tn, double Ra, T* const f[3], const double* tbar,
                  const double* rhoalpha, unsigned fs) {
    const long long ns = L.node_slots();
    buoyancy_kernel<T><<<nblk(ns, 256), 256, 0, ctx->stream>>>(make_geo(L), L.unit64.p, Tn, Ra, f[0], f[1], f[2],
                                                              ns, tbar, rhoalpha);
    TNG_HIP(hipGetLastError());
    void* g[3] = {f[0], f[1], f[2]};
    launch_interface(ctx, L, prec_of<T>(), 0, 3, g);
    zero_layers3_kernel<T><<<nblk(2 * L.lat_slots(), 256), 256, 0, ctx->stream>>>(L.lat_slots(), L.n, (int)fs,
                                                                                 f[0], f[1], f[2]);
    TNG_HIP(hipGetLastError());
    // an impermeable free-slip sphere: the normal rows prescribe zero normal velocity
    vec_fs_project<T>(ctx, L, fs, f, nullptr);
}

// max over wedges of |ubar| / h into host memory (synchronises)
template <typename T>
double cfl_rate(const tng_ctx* ctx, const Level& L, const T* const u[3], DevBuf<double>& part) {
    const long long nc = L.cells();
    const unsigned nb = nblk(nc, 256);
    if (part.n < nb) part.alloc(nb);
    cfl_kernel<T><<<nb, 256, 0, ctx->stream>>>(make_geo(L), u[0], u[1], u[2], part.p, nc);
    TNG_HIP(hipGetLastError());
    std::vector<double> h(nb);
    TNG_HIP(hipMemcpyAsync(h.data(), part.p, nb * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    TNG_HIP(hipStreamSynchronize(ctx->stream));
    double best = 0.0;
    for (double v : h) best = std::max(best, v);
    return best;
}

#define TNG_EINST(T)                                                                                   \
    template void energy_apply<T>(const tng_ctx*, const Level&, const T* const[3], double, const T*, T*); \
    template void energy_wedge_flow<T>(const tng_ctx*, const Level&, const T* const[3], double*);          \
    template void energy_apply_wf<T>(const tng_ctx*, const Level&, const double*, double, const T*, T*);   \
    template void energy_diag<T>(const tng_ctx*, const Level&, const double*, double, T*);                 \
    template void energy_rhs<T>(const tng_ctx*, const Level&, const T*, const T*, double, double, double, T*); \
    template void buoyancy_rhs<T>(const tng_ctx*, const Level&, const T*, double, T* const[3], const double*,  \
                                  const double*, unsigned);                                                       \
    template double cfl_rate<T>(const tng_ctx*, const Level&, const T* const[3], DevBuf<double>&);
TNG_EINST(double)
TNG_EINST(float)
#undef TNG_EINST

}  // namespace tng
