// Coupled Stokes-energy time step (Sec. 6 and the time-stepping structure of
// Secs. 9-10): viscosity from the current temperature, buoyancy right-hand
// side, Stokes solve, CFL time step, and a backward-Euler SUPG energy solve
// with Jacobi-preconditioned GMRES on the device.
#include <chrono>
#include <cmath>
#include <cstring>

#include "mg.hpp"

namespace tng {

template <typename T>
void energy_wedge_flow(const tng_ctx* ctx, const Level& L, const T* const u[3], double* wf);
template <typename T>
void energy_apply_wf(const tng_ctx* ctx, const Level& L, const double* wf, double dt, const T* Tin, T* y);
template <typename T>
void energy_diag(const tng_ctx* ctx, const Level& L, const double* wf, double dt, T* diag);
template <typename T>
void energy_rhs(const tng_ctx* ctx, const Level& L, const T* Tn, const T* H, double dt, double T_in,
                double T_out, T* b);
template <typename T>
double cfl_rate(const tng_ctx* ctx, const Level& L, const T* const u[3], DevBuf<double>& part);

// Right-preconditioned (Jacobi) GMRES on a scalar node field, FP64.
struct EnergyWS {
    int restart = 0;
    long long ns = 0;
    DevBuf<double> V, Z, w, invd, b, f;
    DevBuf<double> wf;                  // per-wedge flow data (mean velocity, tau) of the current velocity
    DevBuf<const double*> vptr, zptr, wptr;
    DevBuf<double> coef, part;
    DotScratch ds;
    double* host = nullptr;
    double* Vi(int i) { return V.p + (long long)i * ns; }
    double* Zi(int i) { return Z.p + (long long)i * ns; }
    ~EnergyWS() {
        if (host) (void)hipHostFree(host);
    }
};

namespace {

void ews_init(EnergyWS& W, const Level& L, int restart) {
    if (W.restart == restart && W.ns == L.node_slots()) return;
    W.restart = restart;
    W.ns = L.node_slots();
    W.V.alloc((size_t)(restart + 1) * W.ns);
    W.Z.alloc((size_t)restart * W.ns);
    W.w.alloc(W.ns);
    W.invd.alloc(W.ns);
    W.b.alloc(W.ns);
    W.f.alloc(3 * W.ns);
    W.wf.alloc((size_t)L.cells() * 2 * 4);
    W.coef.alloc(4 * MAX_MDOT);
    std::vector<const double*> vp(restart + 1), zp(restart), wp(2);
    for (int i = 0; i <= restart; ++i) vp[i] = W.Vi(i);
    for (int i = 0; i < restart; ++i) zp[i] = W.Zi(i);
    wp[0] = W.b.p;
    wp[1] = W.w.p;
    W.vptr.alloc(vp.size());
    W.zptr.alloc(zp.size());
    W.wptr.alloc(2);
    TNG_HIP(hipMemcpy(W.vptr.p, vp.data(), vp.size() * sizeof(double*), hipMemcpyHostToDevice));
    TNG_HIP(hipMemcpy(W.zptr.p, zp.data(), zp.size() * sizeof(double*), hipMemcpyHostToDevice));
    TNG_HIP(hipMemcpy(W.wptr.p, wp.data(), wp.size() * sizeof(double*), hipMemcpyHostToDevice));
    if (!W.host) TNG_HIP(hipHostMalloc(reinterpret_cast<void**>(&W.host), 128 * sizeof(double), hipHostMallocDefault));
}

double rb(const tng_ctx* ctx, EnergyWS& W, const double* dev, int n) {
    TNG_HIP(hipMemcpyAsync(W.host, dev, n * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    TNG_HIP(hipStreamSynchronize(ctx->stream));
    return W.host[0];
}

// y = E x: the streaming apply with the velocity u (NULL: no flow terms) where it
// fits, else the node-gather apply with the per-wedge flow data of W.wf.
void energy_op(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const* u, double dt, const double* x,
               double* y) {
    if (energy_stream_fits(L))
        energy_apply_stream<double>(ctx, L, u, dt, x, y);
    else
        energy_apply_wf<double>(ctx, L, W.wf.p, dt, x, y);
}

// Solves E x = b (b in W.b); x holds the initial guess on entry.
int energy_gmres(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const* u, double dt, double* x,
                 double rtol, int maxit, int* its_out, double* rel_out) {
    const long long ns = W.ns;
    const int m = W.restart;
    const long long nlat = L.lat_slots();
    double* dsc = W.coef.p;
    auto dot1 = [&](const double* a, const double* const* bptr, double* out) {
        vec_mdot<double>(ctx, W.ds, ns, L.n + 1, nlat, L.owner.p, a, bptr, 1, out, false);
    };
    // ||b||
    dot1(W.b.p, W.wptr.p, dsc);
    const double bn = std::sqrt(std::max(0.0, rb(ctx, W, dsc, 1)));
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    int its = 0;
    double res = 0.0;
    if (!(bn > 0)) {
        vec_fill<double>(ctx, ns, 0.0, x);
        *its_out = 0;
        *rel_out = 0.0;
        return TNG_OK;
    }
    for (;;) {
        // r = b - E x
        energy_op(ctx, L, W, u, dt, x, W.w.p);
        vec_axpby<double>(ctx, ns, 1.0, W.b.p, -1.0, W.w.p);
        dot1(W.w.p, W.wptr.p + 1, dsc);
        const double beta = std::sqrt(std::max(0.0, rb(ctx, W, dsc, 1)));
        res = beta;
        if (!std::isfinite(beta)) return TNG_E_NOTCONV;
        if (beta <= rtol * bn || its >= maxit) break;
        vec_axpby<double>(ctx, ns, 1.0 / beta, W.w.p, 0.0, W.Vi(0));
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jend = -1;
        for (int j = 0; j < m; ++j) {
            vec_mul<double>(ctx, ns, W.invd.p, W.Vi(j), W.Zi(j));
            energy_op(ctx, L, W, u, dt, W.Zi(j), W.w.p);
            vec_mdot<double>(ctx, W.ds, ns, L.n + 1, nlat, L.owner.p, W.w.p, W.vptr.p, j + 1, dsc, false);
            vec_maxpy<double>(ctx, ns, dsc, -1.0, W.vptr.p, j + 1, W.w.p);
            vec_mdot<double>(ctx, W.ds, ns, L.n + 1, nlat, L.owner.p, W.w.p, W.vptr.p, j + 1, dsc + MAX_MDOT, false);
            vec_maxpy<double>(ctx, ns, dsc + MAX_MDOT, -1.0, W.vptr.p, j + 1, W.w.p);
            dot1(W.w.p, W.wptr.p + 1, dsc + 2 * MAX_MDOT);
            vec_scale_rsqrt<double>(ctx, ns, dsc + 2 * MAX_MDOT, W.w.p, W.Vi(j + 1));
            TNG_HIP(hipMemcpyAsync(W.host, dsc, (2 * MAX_MDOT + 1) * sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->stream));
            TNG_HIP(hipStreamSynchronize(ctx->stream));
            double* h = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) h[i] = W.host[i] + W.host[MAX_MDOT + i];
            h[j + 1] = std::sqrt(std::max(0.0, W.host[2 * MAX_MDOT]));
            if (!std::isfinite(h[j + 1])) return TNG_E_NOTCONV;
            for (int i = 0; i < j; ++i) {
                const double t0 = cs[i] * h[i] + sn[i] * h[i + 1];
                h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
                h[i] = t0;
            }
            const double den = std::hypot(h[j], h[j + 1]);
            cs[j] = den > 0 ? h[j] / den : 1.0;
            sn[j] = den > 0 ? h[j + 1] / den : 0.0;
            h[j] = den;
            h[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++its;
            jend = j;
            if (std::fabs(g[j + 1]) <= rtol * bn || its >= maxit || den == 0.0) break;
        }
        for (int i = jend; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k <= jend; ++k) acc -= H[(size_t)k * (m + 1) + i] * y[k];
            y[i] = acc / H[(size_t)i * (m + 1) + i];
        }
        std::memcpy(W.host, y.data(), (jend + 1) * sizeof(double));
        TNG_HIP(hipMemcpyAsync(dsc + 3 * MAX_MDOT, W.host, (jend + 1) * sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream));
        vec_maxpy<double>(ctx, ns, dsc + 3 * MAX_MDOT, 1.0, W.zptr.p, jend + 1, x);
        TNG_HIP(hipStreamSynchronize(ctx->stream));
    }
    *its_out = its;
    *rel_out = res / bn;
    return res <= rtol * bn ? TNG_OK : TNG_E_NOTCONV;
}

}  // namespace

// Owned by the solver; created on the first energy step.
EnergyWS* energy_ws_create() { return new EnergyWS(); }
void energy_ws_destroy(EnergyWS* w) { delete w; }

int energy_solve(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const u[3], const double* H,
                 double dt, double T_in, double T_out, double* T, double rtol, int maxit, int restart, int* its,
                 double* rel) {
    ews_init(W, L, restart);
    energy_rhs<double>(ctx, L, T, H, dt, T_in, T_out, W.b.p);
    energy_wedge_flow<double>(ctx, L, u, W.wf.p);   // the velocity is fixed during the solve
    energy_diag<double>(ctx, L, W.wf.p, dt, W.invd.p);
    vec_invert<double>(ctx, W.ns, W.invd.p);
    // initial guess: T^n with the boundary values imposed
    void* f[1] = {T};
    (void)f;
    return energy_gmres(ctx, L, W, u, dt, T, rtol, maxit, its, rel);
}

// MMOC step (eq:mmoc): That = T^n at the departure points, then the implicit diffusion
// step (M_L / dt + K) T^{n+1} = M_L (That / dt + H) by the same Jacobi-GMRES with the
// flow terms off (zero mean velocity and tau).
int energy_solve_mmoc(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const u[3], const double* H,
                      double dt, double T_in, double T_out, double* T, double rtol, int maxit, int restart, int* its,
                      double* rel) {
    ews_init(W, L, restart);
    double* That = W.f.p;                       // scratch of one node field
    mmoc_departure(ctx, L, u, dt, T, That);
    energy_rhs<double>(ctx, L, That, H, dt, T_in, T_out, W.b.p);
    vec_fill<double>(ctx, (long long)L.cells() * 2 * 4, 0.0, W.wf.p);
    energy_diag<double>(ctx, L, W.wf.p, dt, W.invd.p);
    vec_invert<double>(ctx, W.ns, W.invd.p);
    TNG_HIP(hipMemcpyAsync(T, That, W.ns * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    return energy_gmres(ctx, L, W, nullptr, dt, T, rtol, maxit, its, rel);
}

double energy_cfl_dt(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const u[3], double courant) {
    const double rate = cfl_rate<double>(ctx, L, u, W.part);
    return rate > 0 ? courant / rate : 1e30;
}

void energy_buoyancy(const tng_ctx* ctx, const Level& L, const double* T, double Ra, double* const f[3],
                     unsigned fs) {
    buoyancy_rhs<double>(ctx, L, T, Ra, f, nullptr, nullptr, fs);
}

}  // namespace tng
