// Stokes solver (Sec. 7): FGMRES right-preconditioned by the block-triangular
// Schur preconditioner of eq:block-precond,
//   z_p = S^{-1} r_p = -diag(M_{1/eta})^{-1} r_p       (eq:pmass, lumped),
//   z_u = A^{-1} (r_u - B^T z_p),  A^{-1} ~ one geometric multigrid V-cycle
// with Chebyshev smoothing (degree 2, pre/post steps per level), re-discretised
// coarse operators on averaged viscosity, and an exact solve on the coarsest
// level.  Mixed precision: FP64 iterative refinement around an FP32 inner
// FGMRES whose operator applies, smoothers and Krylov basis are FP32 (the
// coarsest solve stays FP64).
//
// All vectors live on the device in the duplicated-diamond layout; a Stokes
// vector is [u0 | u1 | u2 | p] with the velocity of level 0 and the pressure
// of level 1.  Host work is limited to the small Hessenberg least-squares
// problem; every FGMRES iteration reads back one short array of dots.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>

#include "batch.hpp"
#include "mg.hpp"

namespace tng {

template <typename T>
struct MGLevel {
    const Level* L = nullptr;
    long long ns = 0;
    DevBuf<T> eta;                      // wedge viscosity of this level
    DevBuf<T> invd;                     // 3 ns: inverse diagonal of A
    DevBuf<T> x, b, r, y, d;            // 3 ns scratch
    DevBuf<const T*> xy;                // device pointers {x, y} for reductions
    DevBuf<double> cheb;                // Chebyshev coefficients (alpha_k, beta_k) of this level
    std::vector<double> cheb_h;         //   host copy (kept until the upload has run)
    double lmax = 1.0;                  // largest eigenvalue of D^{-1} A (estimate)
    T* c(DevBuf<T>& v, int k) { return v.p + (long long)k * ns; }
};

template <typename T>
struct KrylovWS {
    int restart = 0;
    long long N = 0;
    DevBuf<T> V, Z, w, t;
    DevBuf<T> zb;                       // preconditioner output of a batch slot (index-free)
    DevBuf<const T*> vptr, zptr, wptr;
    DevBuf<double> coef;                // device dots / coefficients
    long long ld = 0;                   // basis stride: N rounded up to 256 bytes
    T* Vi(int i) { return V.p + (long long)i * ld; }
    T* Zi(int i) { return Z.p + (long long)i * ld; }
};

}  // namespace tng

struct tng_solver {
    tng_ctx* ctx = nullptr;
    tng_mesh* mesh = nullptr;
    tng_solver_opts opts{};
    int nlev = 0;
    std::vector<tng::MGLevel<double>> h64;
    std::vector<tng::MGLevel<float>> h32;
    tng::CoarseDense cd;
    std::unique_ptr<tng::DotScratch> ds;
    tng::KrylovWS<double> k64;
    tng::KrylovWS<float> k32;
    tng::DevBuf<double> pm64;           // lumped M_{1/eta} on the pressure level
    tng::DevBuf<float> pm32;
    tng::DevBuf<double> ones_p;         // pressure-level ones (mean projection)
    tng::DevBuf<float> ones_p32;
    tng::DevBuf<const double*> onesp64; // [ones_p]
    tng::DevBuf<const float*> onesp32;  // [ones_p32]
    // free slip on both spheres: the rigid rotations e_a x x orthonormalised over unique
    // DoFs (three velocity vectors, FP64 and FP32) and device pointers to them
    tng::DevBuf<double> rot64;
    tng::DevBuf<float> rot32;
    tng::DevBuf<const double*> rotptr64;
    tng::DevBuf<const float*> rotptr32;
    tng::DevBuf<double> xo, ro, bo;     // outer FP64 vectors (mixed precision)
    tng::DevBuf<float> r32, d32;
    // mixed precision after a stalled refinement: FP64 inner solves (level scratch,
    // Krylov basis on ro, correction d64), set up on first use; fp64_ops: the FP64
    // level operators are those of the current viscosity
    bool fp64_inner = false, fp64_ops = false;
    tng::DevBuf<double> d64;
    tng::DevBuf<double> scal;           // device scalars
    tng::DevBuf<const double*> dptr;    // [bo, ro, pressure of xo, k64.w]
    double* host = nullptr;             // pinned read-back buffer
    bool ready = false;
    bool batch_slot = false;            // slot of a SolverBatch (extra index-free buffers)
    long long ns0 = 0, np = 0, N = 0;
    tng::EnergyWS* ews = nullptr;       // energy step workspace (created on first use)
    tng::DevBuf<double> eta_step, f_step;
    // preconditioner graphs: z_j = P^{-1} v_j of Krylov index j, captured on a
    // private stream (gctx) at first use and replayed there, ordered with the
    // context's stream by the events
    hipStream_t gstream = nullptr;
    tng_ctx* gctx = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<hipGraphExec_t> pg32, pg64;
    ~tng_solver() {
        if (gstream) (void)hipStreamSynchronize(gstream);
        for (auto g : pg32)
            if (g) (void)hipGraphExecDestroy(g);
        for (auto g : pg64)
            if (g) (void)hipGraphExecDestroy(g);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
        if (gctx) tng_ctx_destroy(gctx);
        if (gstream) (void)hipStreamDestroy(gstream);
        if (host) (void)hipHostFree(host);
        if (ews) tng::energy_ws_destroy(ews);
    }
};

namespace tng {
namespace {

const Level& L0(const tng_solver* s) { return s->mesh->lv[0]; }
const Level& L1(const tng_solver* s) { return s->mesh->lv[1]; }

void sync(const tng_solver* s) { TNG_HIP(hipStreamSynchronize(s->ctx->stream)); }

// read n doubles from device scalars into the pinned host buffer
void readback(tng_solver* s, const double* dev, int n) {
    TNG_HIP(hipMemcpyAsync(s->host, dev, n * sizeof(double), hipMemcpyDeviceToHost, s->ctx->stream));
    sync(s);
}

template <typename T>
std::vector<MGLevel<T>>& hier(tng_solver* s);
template <>
std::vector<MGLevel<double>>& hier<double>(tng_solver* s) { return s->h64; }
template <>
std::vector<MGLevel<float>>& hier<float>(tng_solver* s) { return s->h32; }
template <typename T>
KrylovWS<T>& kws(tng_solver* s);
template <>
KrylovWS<double>& kws<double>(tng_solver* s) { return s->k64; }
template <>
KrylovWS<float>& kws<float>(tng_solver* s) { return s->k32; }
template <typename T>
T* pmass(tng_solver* s);
template <>
double* pmass<double>(tng_solver* s) { return s->pm64.p; }
template <>
float* pmass<float>(tng_solver* s) { return s->pm32.p; }

// ---- operators ------------------------------------------------------------
// the solve's operator options: the two-radial-point rule and free slip reach every
// viscous apply, the compressible mass rows only the outer operator K
unsigned twopt_flag(const tng_solver* s) { return s->opts.op_flags & TNG_OP_TWOPOINT; }
unsigned fs_flag(const tng_solver* s) { return s->opts.op_flags & (TNG_OP_FREESLIP_INNER | TNG_OP_FREESLIP_OUTER); }
// the same as bits 0 (inner) and 1 (outer sphere)
unsigned fs_bits(const tng_solver* s) { return fs_flag(s) >> 4; }

template <typename T>
const T* const* ones_ptr(tng_solver* s);
template <>
const double* const* ones_ptr<double>(tng_solver* s) { return s->onesp64.p; }
template <>
const float* const* ones_ptr<float>(tng_solver* s) { return s->onesp32.p; }

// p <- p - mean(p) over unique pressure nodes
template <typename T>
void project_mean(tng_solver* s, T* p) {
    const Level& P = L1(s);
    vec_mdot<T>(s->ctx, *s->ds, P.node_slots(), P.n + 1, P.lat_slots(), P.owner.p, p, ones_ptr<T>(s), 1,
                s->scal.p + 40, false);
    vec_shift<T>(s->ctx, P.node_slots(), s->scal.p + 40, p);
}

template <typename T>
const T* const* rot_ptr(tng_solver* s);
template <>
const double* const* rot_ptr<double>(tng_solver* s) { return s->rotptr64.p; }
template <>
const float* const* rot_ptr<float>(tng_solver* s) { return s->rotptr32.p; }

// free slip on both spheres: u <- u - Q Q^T u, Q the orthonormalised rigid rotations
// (inner products over unique DoFs; the rotations are a null space of K, so this changes
// no residual and fixes the solution up to them as the pressure is fixed up to its mean)
template <typename T>
void project_rotations(tng_solver* s, T* u) {
    if (fs_bits(s) != 3) return;
    const Level& L = L0(s);
    const long long n3 = 3 * s->ns0;
    vec_mdot<T>(s->ctx, *s->ds, n3, L.n + 1, L.lat_slots(), L.owner.p, u, rot_ptr<T>(s), 3, s->scal.p + 56, false);
    vec_maxpy<T>(s->ctx, n3, s->scal.p + 56, -1.0, rot_ptr<T>(s), 3, u);
}

// With free slip the velocity projection P = I - rhat rhat^T at the nodes does not
// keep the constant pressure in the null space exactly: the boundary flux of a
// velocity that is tangential at the nodes is O(h^2), so B_D^T 1 = P B^T 1 != 0 and
// 1^T B_D != 0 by as much.  The solve keeps the pressure gauge of the no-slip case:
// the mass rows are taken modulo constants and the pressure at zero mean, i.e. the
// operator is diag(I, Pi) K diag(I, Pi), Pi = I - 1 1^T / n, which has the exact null
// space (0, 1) again.  The Krylov vectors' pressures have zero mean (projected in the
// preconditioner), so Pi on the input is implied and K's mass rows are projected here.
template <typename T>
void apply_K(tng_solver* s, const T* eta0, const T* x, T* y) {
    const long long ns = s->ns0;
    const void* u[3] = {x, x + ns, x + 2 * ns};
    void* yu[3] = {y, y + ns, y + 2 * ns};
    launch_stokes_apply(s->ctx, L0(s), &L1(s), prec_of<T>(),
                        TNG_OP_A | TNG_OP_BT | TNG_OP_B | TNG_OP_DIRICHLET | s->opts.op_flags, s->opts.hg_alpha,
                        eta0, u, x + 3 * ns, yu, y + 3 * ns);
    if (fs_flag(s)) project_mean<T>(s, y + 3 * ns);
}

template <typename T>
void apply_A(tng_solver* s, int l, const T* eta, const T* x, T* y) {
    const Level& L = s->mesh->lv[l];
    const long long ns = L.node_slots();
    const void* u[3] = {x, x + ns, x + 2 * ns};
    void* yu[3] = {y, y + ns, y + 2 * ns};
    launch_stokes_apply(s->ctx, L, nullptr, prec_of<T>(), TNG_OP_A | TNG_OP_DIRICHLET | twopt_flag(s) | fs_flag(s),
                        s->opts.hg_alpha, eta, u, nullptr, yu, nullptr);
}

template <typename T>
void apply_BT(tng_solver* s, const T* p, T* yu) {
    const long long ns = s->ns0;
    void* y[3] = {yu, yu + ns, yu + 2 * ns};
    launch_stokes_apply(s->ctx, L0(s), &L1(s), prec_of<T>(), TNG_OP_BT | TNG_OP_DIRICHLET | fs_flag(s), 0.0,
                        nullptr, nullptr, p, y, nullptr);
}

// squared owner-masked norm of a velocity vector of level l into device scalar
template <typename T>
void vel_dot(tng_solver* s, int l, const T* x, const T* const* ydev, double* out) {
    const Level& L = s->mesh->lv[l];
    vec_mdot<T>(s->ctx, *s->ds, 3 * L.node_slots(), L.n + 1, L.lat_slots(), L.owner.p, x, ydev, 1, out, false);
}

// ---- smoother, V-cycle ----------------------------------------------------
}  // namespace

// Chebyshev smoother on D^{-1} A (Saad's three-term recurrence) for the
// eigenvalue interval [lo, hi]: every step is a polynomial of degree `deg`
// (deg operator applies; the first one is skipped when x starts at zero).
// Step k of the recurrence is d <- alpha_k d + beta_k D^{-1}(b - A x), x += d.
std::vector<double> chebyshev_coefficients(int deg, double lo, double hi) {
    std::vector<double> ab(2 * (size_t)std::max(deg, 1));
    chebyshev_coefficients(deg, lo, hi, ab.data());
    return ab;
}

void chebyshev_coefficients(int deg, double lo, double hi, double* ab) {
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    ab[0] = 0.0;
    ab[1] = 1.0 / theta;
    double rho_old = 1.0 / sigma;
    for (int k = 1; k < deg; ++k) {
        const double rho = 1.0 / (2.0 * sigma - rho_old);
        ab[2 * k] = rho * rho_old;
        ab[2 * k + 1] = 2.0 * rho / delta;
        rho_old = rho;
    }
}

template <typename T>
void chebyshev_steps(const tng_ctx* ctx, const Level& L, const T* eta, double hg_alpha, const T* invd, const T* b,
                     T* x, T* y, T* d, const double* ab_dev, int deg, int steps, bool x_zero, bool twopt) {
    const long long ns = L.node_slots();
    const unsigned aflags = TNG_OP_A | TNG_OP_DIRICHLET | (twopt ? TNG_OP_TWOPOINT : 0u);
    // each update: the raw viscous apply, then one pass that completes its duplicated
    // nodes and identity rows and takes the two-term Chebyshev step (the apply's
    // closing pass and the update fused).  x_k alternates between x and d: a step of
    // degree deg starts from x and, for even deg, ends in x
    auto applyA = [&](const T* xin, T* yout) {
        const void* u[3] = {xin, xin + ns, xin + 2 * ns};
        void* yu[3] = {yout, yout + ns, yout + 2 * ns};
        launch_stokes_apply_raw(ctx, L, prec_of<T>(), aflags, hg_alpha, eta, u, yu);
    };
    for (int st = 0; st < steps; ++st) {
        for (int k = 0; k < deg; ++k) {
            const bool first = x_zero && st == 0 && k == 0;
            const bool prev_zero = x_zero && st == 0 && k == 1;   // x_k-1 is the zero start
            T* cur = (k & 1) ? d : x;
            T* out = (k & 1) ? x : d;
            if (!first) applyA(cur, y);
            vec_cheb_post_update<T>(ctx, L, true, true, ab_dev, k, first, prev_zero, b, y, invd, cur, out);
        }
        if (deg & 1) vec_cast<T, T>(ctx, 3 * ns, d, x);
    }
}

namespace {

// The smoother with a free-slip sphere: the whole apply (interface sums and the
// boundary rows P A P + N), the Chebyshev step in direction form, then the normal
// rows solved exactly (x <- P x + N b), so that the iterate stays tangential there
// and D^{-1} (isotropic on those rows) only ever sees tangential residuals.
template <typename T>
void chebyshev_fs(tng_solver* s, int l, const T* b, T* x, bool x_zero, int steps) {
    MGLevel<T>& M = hier<T>(s)[l];
    const long long ns = M.ns, n3 = 3 * ns;
    T* xx[3] = {x, x + ns, x + 2 * ns};
    const T* bb[3] = {b, b + ns, b + 2 * ns};
    if (x_zero && steps > 0) vec_fill<T>(s->ctx, n3, T(0), x);
    const int deg = std::max(1, s->opts.cheb_degree);
    for (int st = 0; st < steps; ++st)
        for (int k = 0; k < deg; ++k) {
            apply_A<T>(s, l, M.eta.p, x, M.y.p);
            vec_cheb_update<T>(s->ctx, n3, M.cheb.p, k, b, M.y.p, M.invd.p, M.d.p, x);
            vec_fs_project<T>(s->ctx, *M.L, fs_bits(s), xx, bb);
        }
}

template <typename T>
void chebyshev(tng_solver* s, int l, const T* b, T* x, bool x_zero, int steps) {
    if (fs_flag(s)) {
        chebyshev_fs<T>(s, l, b, x, x_zero, steps);
        return;
    }
    MGLevel<T>& M = hier<T>(s)[l];
    chebyshev_steps<T>(s->ctx, *M.L, M.eta.p, s->opts.hg_alpha, M.invd.p, b, x, M.y.p, M.d.p, M.cheb.p,
                       std::max(1, s->opts.cheb_degree), steps, x_zero, twopt_flag(s) != 0);
}

template <typename T>
void vcycle(tng_solver* s, int l, const T* b, T* x) {
    auto& H = hier<T>(s);
    MGLevel<T>& M = H[l];
    const long long ns = M.ns;
    if (l == s->nlev - 1) {
        const T* bb[3] = {b, b + ns, b + 2 * ns};
        T* xx[3] = {x, x + ns, x + 2 * ns};
        coarse_solve<T>(s->ctx, s->cd, bb, xx);
        return;
    }
    chebyshev<T>(s, l, b, x, true, s->opts.pre);
    // r = b - A x: the raw apply into the smoother's work vector, then one pass that
    // completes it and forms the residual
    if (fs_flag(s)) {
        // free slip: the whole apply, then r = b - y
        apply_A<T>(s, l, M.eta.p, x, M.y.p);
        vec_cast<T, T>(s->ctx, 3 * ns, b, M.r.p);
        vec_axpby<T>(s->ctx, 3 * ns, -1.0, M.y.p, 1.0, M.r.p);
    } else {
        const Level& L = *M.L;
        const void* u[3] = {x, x + ns, x + 2 * ns};
        void* yu[3] = {M.y.p, M.y.p + ns, M.y.p + 2 * ns};
        launch_stokes_apply_raw(s->ctx, L, prec_of<T>(), TNG_OP_A | TNG_OP_DIRICHLET | twopt_flag(s),
                                s->opts.hg_alpha, M.eta.p, u, yu);
        vec_resid_post<T>(s->ctx, L, true, true, b, x, M.y.p, M.r.p);
    }
    MGLevel<T>& C = H[l + 1];
    const T* rf[3] = {M.r.p, M.r.p + ns, M.r.p + 2 * ns};
    T* bc[3] = {C.b.p, C.b.p + C.ns, C.b.p + 2 * C.ns};
    mg_restrict<T>(s->ctx, *M.L, *C.L, rf, bc, fs_bits(s));
    vcycle<T>(s, l + 1, C.b.p, C.x.p);
    const T* xc[3] = {C.x.p, C.x.p + C.ns, C.x.p + 2 * C.ns};
    T* xf[3] = {x, x + ns, x + 2 * ns};
    mg_prolong<T>(s->ctx, *M.L, xc, xf, true);
    if (fs_flag(s)) {
        const T* bf[3] = {b, b + ns, b + 2 * ns};
        vec_fs_project<T>(s->ctx, *M.L, fs_bits(s), xf, bf);
    }
    chebyshev<T>(s, l, b, x, false, s->opts.post);
}

// block-triangular Schur preconditioner: z = P^{-1} v
template <typename T>
void precond(tng_solver* s, const T* v, T* z) {
    KrylovWS<T>& K = kws<T>(s);
    const long long ns = s->ns0, np = s->np;
    vec_schur<T>(s->ctx, np, v + 3 * ns, pmass<T>(s), z + 3 * ns);
    if (fs_flag(s)) project_mean<T>(s, z + 3 * ns);             // free slip: zero-mean pressures
    apply_BT<T>(s, z + 3 * ns, K.t.p);                           // t = B^T z_p
    vec_axpby<T>(s->ctx, 3 * ns, 1.0, v, -1.0, K.t.p);           // t = v_u - B^T z_p
    vcycle<T>(s, 0, K.t.p, z);                                   // z_u ~ A^{-1} t
    // free slip on both spheres: keep the Krylov directions free of the rigid rotations
    // (the null space of K), so that the iterate's rotation content cannot grow and
    // swamp its other components in finite precision
    project_rotations<T>(s, z);
}

template <typename T>
std::vector<hipGraphExec_t>& pgraphs(tng_solver* s);
template <>
std::vector<hipGraphExec_t>& pgraphs<float>(tng_solver* s) { return s->pg32; }
template <>
std::vector<hipGraphExec_t>& pgraphs<double>(tng_solver* s) { return s->pg64; }

// Z_j = P^{-1} V_j, as a replayed graph when the solver has graphs
template <typename T>
void precond_j(tng_solver* s, int j) {
    KrylovWS<T>& K = kws<T>(s);
    if (!s->gctx) {
        precond<T>(s, K.Vi(j), K.Zi(j));
        return;
    }
    auto& G = pgraphs<T>(s);
    if (G.size() < (size_t)K.restart) G.assign(K.restart, nullptr);
    if (!G[j]) {
        // capture with every launch on the private stream; no timers inside
        tng_ctx* saved = s->ctx;
        hipGraph_t graph = nullptr;
        TNG_HIP(hipStreamBeginCapture(s->gstream, hipStreamCaptureModeThreadLocal));
        s->ctx = s->gctx;
        try {
            precond<T>(s, K.Vi(j), K.Zi(j));
        } catch (...) {
            s->ctx = saved;
            (void)hipStreamEndCapture(s->gstream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        s->ctx = saved;
        TNG_HIP(hipStreamEndCapture(s->gstream, &graph));
        const hipError_t e = hipGraphInstantiate(&G[j], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            G[j] = nullptr;
            throw Error(TNG_E_HIP, std::string("preconditioner graph: ") + hipGetErrorString(e));
        }
    }
    TNG_HIP(hipEventRecord(s->ev_in, s->ctx->stream));
    TNG_HIP(hipStreamWaitEvent(s->gstream, s->ev_in, 0));
    TNG_HIP(hipGraphLaunch(G[j], s->gstream));
    TNG_HIP(hipEventRecord(s->ev_out, s->gstream));
    TNG_HIP(hipStreamWaitEvent(s->ctx->stream, s->ev_out, 0));
}

double host_norm_from_dev(tng_solver* s, const double* dev) {
    readback(s, dev, 1);
    return std::sqrt(std::max(0.0, s->host[0]));
}

// ---- FGMRES ---------------------------------------------------------------
// Solves K x = b to a relative (to ||b||) tolerance; x is overwritten (x0 = 0).
template <typename T>
int fgmres(tng_solver* s, const T* eta0, const T* b, T* x, double rtol, int maxit, int* its_out,
           double* relres_out) {
    KrylovWS<T>& K = kws<T>(s);
    const Level& Lu = L0(s);
    const Level& Lp = L1(s);
    const long long N = s->N;
    const int m = K.restart;
    double* dsc = K.coef.p;               // [0, 2*MAX_MDOT + 2)
    vec_fill<T>(s->ctx, N, T(0), x);
    // beta = ||b||; K.wptr[0] points at b (fixed at creation)
    vec_smdot<T>(s->ctx, *s->ds, Lu, Lp, b, K.wptr.p, 1, dsc, false);
    const double bnorm = host_norm_from_dev(s, dsc);
    int its = 0;
    if (!(bnorm > 0.0)) {
        *its_out = 0;
        *relres_out = 0.0;
        return std::isfinite(bnorm) ? TNG_OK : TNG_E_NOTCONV;
    }
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m);
    double beta = bnorm;
    // V0 = b / beta
    vec_axpby<T>(s->ctx, N, 1.0 / beta, b, 0.0, K.Vi(0));
    double res = beta;
    bool done = false;
    while (!done) {
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < m; ++j) {
            precond_j<T>(s, j);
            apply_K<T>(s, eta0, K.Zi(j), K.w.p);
            // classical Gram-Schmidt, twice: h1 = V^T w; w -= V h1 with h2 = V^T w in the
            // same pass; w -= V h2 with |w|^2 in the same pass
            // (the basis vectors sit at 256-byte strides: 16-byte accesses)
            vec_smdot<T>(s->ctx, *s->ds, Lu, Lp, K.w.p, K.vptr.p, j + 1, dsc, false, true);
            vec_maxpy_smdot<T>(s->ctx, *s->ds, Lu, Lp, dsc, -1.0, K.vptr.p, j + 1, K.w.p, dsc + MAX_MDOT, false,
                               true);
            vec_maxpy_smdot<T>(s->ctx, *s->ds, Lu, Lp, dsc + MAX_MDOT, -1.0, K.vptr.p, j + 1, K.w.p,
                               dsc + 2 * MAX_MDOT, true, true);
            vec_scale_rsqrt<T>(s->ctx, N, dsc + 2 * MAX_MDOT, K.w.p, K.Vi(j + 1));
            readback(s, dsc, 2 * MAX_MDOT + 1);
            double* h = &H[(size_t)j * (m + 1)];
            for (int i = 0; i <= j; ++i) h[i] = s->host[i] + s->host[MAX_MDOT + i];
            h[j + 1] = std::sqrt(std::max(0.0, s->host[2 * MAX_MDOT]));
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
            res = std::fabs(g[j + 1]);
            ++its;
            jend = j;
            if (res <= rtol * bnorm || its >= maxit || h[j] == 0.0) {
                done = true;
                break;
            }
        }
        // y = H^{-1} g (upper triangular), x += Z y
        for (int i = jend; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k <= jend; ++k) acc -= H[(size_t)k * (m + 1) + i] * y[k];
            y[i] = acc / H[(size_t)i * (m + 1) + i];
        }
        std::memcpy(s->host, y.data(), (jend + 1) * sizeof(double));
        TNG_HIP(hipMemcpyAsync(dsc + 3 * MAX_MDOT, s->host, (jend + 1) * sizeof(double), hipMemcpyHostToDevice,
                               s->ctx->stream));
        vec_maxpy<T>(s->ctx, N, dsc + 3 * MAX_MDOT, 1.0, K.zptr.p, jend + 1, x);
        sync(s);   // the pinned buffer is reused below
        if (done) break;
        // restart from the true residual
        apply_K<T>(s, eta0, x, K.w.p);
        vec_axpby<T>(s->ctx, N, 1.0, b, -1.0, K.w.p);
        vec_smdot<T>(s->ctx, *s->ds, Lu, Lp, K.w.p, K.wptr.p + 1, 1, dsc, false);
        beta = host_norm_from_dev(s, dsc);
        res = beta;
        if (beta <= rtol * bnorm) break;
        if (!std::isfinite(beta)) return TNG_E_NOTCONV;
        vec_axpby<T>(s->ctx, N, 1.0 / beta, K.w.p, 0.0, K.Vi(0));
    }
    *its_out = its;
    *relres_out = res / bnorm;
    return std::isfinite(res) ? TNG_OK : TNG_E_NOTCONV;
}

void remove_rotations(tng_solver* s) { project_rotations<double>(s, s->xo.p); }

// p <- p - mean(p) over unique pressure nodes of the outer solution xo
void remove_pressure_mean(tng_solver* s) {
    const Level& P = L1(s);
    double* p = s->xo.p + 3 * s->ns0;
    vec_mdot<double>(s->ctx, *s->ds, P.node_slots(), P.n + 1, P.lat_slots(), P.owner.p, s->ones_p.p,
                     s->dptr.p + 2, 1, s->scal.p + 32, false);
    vec_shift<double>(s->ctx, P.node_slots(), s->scal.p + 32, p);
}

// ---- setup ----------------------------------------------------------------
void build_coarse_maps(tng_solver* s) {
    const Level& C = s->mesh->lv[s->nlev - 1];
    const int m = C.m, n = C.n;
    const long long nl = C.lat_slots(), nsl = C.node_slots();
    // owner slot of every unique lateral id
    std::vector<int> owner_of(C.n_unique_lat, -1);
    for (long long q = 0; q < nl; ++q)
        if (owner_of[C.uid[q]] < 0) owner_of[C.uid[q]] = (int)q;
    // unknowns: interior layers, and the layer of a free-slip sphere
    const int k0 = (fs_bits(s) & 1) ? 0 : 1, k1 = (fs_bits(s) & 2) ? n : n - 1;
    std::vector<int> dof_of_uid_k((size_t)C.n_unique_lat * (n + 1) * 3, -1);
    std::vector<int> dof_slot;
    for (long long q = 0; q < nl; ++q) {
        if (owner_of[C.uid[q]] != q) continue;
        for (int k = k0; k <= k1; ++k)
            for (int c = 0; c < 3; ++c) {
                dof_of_uid_k[((size_t)C.uid[q] * (n + 1) + k) * 3 + c] = (int)dof_slot.size();
                dof_slot.push_back((int)(((q * (n + 1) + k) << 2) | c));
            }
    }
    const int nd = (int)dof_slot.size();
    if (nd > MAX_COARSE_DOF)
        throw Error(TNG_E_INVAL, "coarsest level has " + std::to_string(nd) + " interior DoFs (max " +
                                     std::to_string(MAX_COARSE_DOF) + "); build more levels");
    std::vector<int> slot_dof((size_t)3 * nsl, -1);
    std::vector<std::vector<int>> copies(nd);
    for (long long q = 0; q < nl; ++q)
        for (int k = k0; k <= k1; ++k)
            for (int c = 0; c < 3; ++c) {
                const int dof = dof_of_uid_k[((size_t)C.uid[q] * (n + 1) + k) * 3 + c];
                const long long slot = q * (n + 1) + k;
                slot_dof[(size_t)c * nsl + slot] = dof;
                copies[dof].push_back((int)((slot << 2) | c));
            }
    std::vector<int> cptr(1, 0), cslot;
    for (auto& v : copies) {
        cslot.insert(cslot.end(), v.begin(), v.end());
        cptr.push_back((int)cslot.size());
    }
    s->cd.ndof = nd;
    s->cd.nslots = nsl;
    s->cd.dof_slot.alloc(nd);
    TNG_HIP(hipMemcpy(s->cd.dof_slot.p, dof_slot.data(), nd * sizeof(int), hipMemcpyHostToDevice));
    s->cd.slot_dof.alloc(slot_dof.size());
    TNG_HIP(hipMemcpy(s->cd.slot_dof.p, slot_dof.data(), slot_dof.size() * sizeof(int), hipMemcpyHostToDevice));
    s->cd.copy_ptr.alloc(cptr.size());
    TNG_HIP(hipMemcpy(s->cd.copy_ptr.p, cptr.data(), cptr.size() * sizeof(int), hipMemcpyHostToDevice));
    s->cd.copy_slot.alloc(cslot.size());
    TNG_HIP(hipMemcpy(s->cd.copy_slot.p, cslot.data(), cslot.size() * sizeof(int), hipMemcpyHostToDevice));
    s->cd.Ainv.alloc((size_t)nd * nd);
}

template <typename T>
void alloc_level_scratch(tng_solver* s, MGLevel<T>& M);

template <typename T>
void alloc_hierarchy(tng_solver* s, bool scratch) {
    auto& H = hier<T>(s);
    H.clear();
    H.resize(s->nlev);
    for (int l = 0; l < s->nlev; ++l) {
        MGLevel<T>& M = H[l];
        M.L = &s->mesh->lv[l];
        M.ns = M.L->node_slots();
        M.eta.alloc(2 * M.L->cells());
        if (scratch) alloc_level_scratch<T>(s, M);
    }
}

// smoother, residual and transfer vectors of one level
template <typename T>
void alloc_level_scratch(tng_solver* s, MGLevel<T>& M) {
    const long long n3 = 3 * M.ns;
    M.invd.alloc(n3);
    M.x.alloc(n3);
    M.b.alloc(n3);
    M.r.alloc(n3);
    M.y.alloc(n3);
    M.d.alloc(n3);
    M.cheb.alloc(2 * (size_t)std::max(1, s->opts.cheb_degree));
    const T* xy[2] = {M.x.p, M.y.p};
    M.xy.alloc(2);
    TNG_HIP(hipMemcpy(M.xy.p, xy, sizeof(xy), hipMemcpyHostToDevice));
}

template <typename T>
void alloc_krylov(tng_solver* s, const T* rhs) {
    KrylovWS<T>& K = kws<T>(s);
    const int m = s->opts.restart;
    K.restart = m;
    K.N = s->N;
    // every basis vector starts on a 256-byte boundary (16-byte vector loads)
    K.ld = (s->N + (long long)(256 / sizeof(T)) - 1) / (long long)(256 / sizeof(T)) * (long long)(256 / sizeof(T));
    K.V.alloc((size_t)(m + 1) * K.ld);
    K.Z.alloc((size_t)m * K.ld);
    K.w.alloc(s->N);
    K.t.alloc(3 * s->ns0);
    if (s->batch_slot) K.zb.alloc(s->N);
    K.coef.alloc(4 * MAX_MDOT);
    std::vector<const T*> vp(m + 1), zp(m), wp(2);
    for (int i = 0; i <= m; ++i) vp[i] = K.Vi(i);
    for (int i = 0; i < m; ++i) zp[i] = K.Zi(i);
    wp[0] = rhs;
    wp[1] = K.w.p;
    K.vptr.alloc(m + 1);
    K.zptr.alloc(m);
    K.wptr.alloc(2);
    TNG_HIP(hipMemcpy(K.vptr.p, vp.data(), vp.size() * sizeof(T*), hipMemcpyHostToDevice));
    TNG_HIP(hipMemcpy(K.zptr.p, zp.data(), zp.size() * sizeof(T*), hipMemcpyHostToDevice));
    TNG_HIP(hipMemcpy(K.wptr.p, wp.data(), wp.size() * sizeof(T*), hipMemcpyHostToDevice));
}

// largest eigenvalue of D^{-1} A on level l by seeded power iteration
template <typename T>
double power_lmax(tng_solver* s, int l) {
    MGLevel<T>& M = hier<T>(s)[l];
    const long long n3 = 3 * M.ns;
    vec_rand<T>(s->ctx, n3, 0x5eed0000ULL + (unsigned long long)l, M.x.p);
    {
        void* f[3] = {M.x.p, M.x.p + M.ns, M.x.p + 2 * M.ns};
        launch_interface(s->ctx, *M.L, prec_of<T>(), 1, 3, f);
    }
    // free slip: the normal rows of D^{-1} (P A P + N) have eigenvalue 1 / d, outside
    // the smoother's spectrum; the iteration stays tangential there
    T* xv[3] = {M.x.p, M.x.p + M.ns, M.x.p + 2 * M.ns};
    T* yv[3] = {M.y.p, M.y.p + M.ns, M.y.p + 2 * M.ns};
    vec_fs_project<T>(s->ctx, *M.L, fs_bits(s), xv, nullptr);
    const T* const* xp = M.xy.p;
    const T* const* yp = M.xy.p + 1;
    double lam = 1.0;
    for (int it = 0; it < s->opts.power_its; ++it) {
        apply_A<T>(s, l, M.eta.p, M.x.p, M.y.p);
        vec_mul<T>(s->ctx, n3, M.invd.p, M.y.p, M.y.p);
        vec_fs_project<T>(s->ctx, *M.L, fs_bits(s), yv, nullptr);
        vel_dot<T>(s, l, M.x.p, xp, s->scal.p);
        vel_dot<T>(s, l, M.y.p, yp, s->scal.p + 1);
        readback(s, s->scal.p, 2);
        const double nx = std::sqrt(s->host[0]), ny = std::sqrt(s->host[1]);
        if (!(nx > 0) || !std::isfinite(ny)) throw Error(TNG_E_NOTCONV, "power iteration failed");
        lam = ny / nx;
        vec_axpby<T>(s->ctx, n3, 1.0 / ny, M.y.p, 0.0, M.x.p);
    }
    return lam;
}

template <typename T>
void setup_level_operators(tng_solver* s) {
    auto& H = hier<T>(s);
    for (int l = 0; l < s->nlev - 1; ++l) {
        MGLevel<T>& M = H[l];
        T* d[3] = {M.invd.p, M.invd.p + M.ns, M.invd.p + 2 * M.ns};
        mg_diag_A<T>(s->ctx, *M.L, M.eta.p, s->opts.hg_alpha, d, twopt_flag(s) != 0, fs_bits(s));
        vec_invert<T>(s->ctx, 3 * M.ns, M.invd.p);
        M.lmax = power_lmax<T>(s, l);
        M.cheb_h = chebyshev_coefficients(std::max(1, s->opts.cheb_degree), s->opts.cheb_lo * M.lmax,
                                          s->opts.cheb_hi * M.lmax);
        M.cheb.upload(M.cheb_h.data(), M.cheb_h.size(), s->ctx->stream);
    }
}

void setup_viscosity(tng_solver* s, const double* eta_dev) {
    const bool mixed = s->opts.mixed != 0;
    s->fp64_ops = false;
    auto& H = s->h64;
    TNG_HIP(hipMemcpyAsync(H[0].eta.p, eta_dev, 2 * L0(s).cells() * sizeof(double), hipMemcpyDeviceToDevice,
                           s->ctx->stream));
    for (int l = 0; l + 1 < s->nlev; ++l) launch_eta_coarsen(s->ctx, s->mesh->lv[l + 1], TNG_F64, H[l].eta.p, H[l + 1].eta.p);
    // coarsest level: dense inverse of D A D over its interior DoFs
    coarse_assemble<double>(s->ctx, s->cd, s->mesh->lv[s->nlev - 1], H[s->nlev - 1].eta.p, s->opts.hg_alpha,
                            twopt_flag(s) != 0, fs_bits(s));
    if (fs_bits(s) == 3) coarse_rotation_shift(s->ctx, s->cd, s->mesh->lv[s->nlev - 1]);
    coarse_invert(s->ctx, s->cd);
    mg_pmass<double>(s->ctx, L0(s), L1(s), H[0].eta.p, s->pm64.p);
    if (!mixed) {
        setup_level_operators<double>(s);
    } else {
        for (int l = 0; l < s->nlev; ++l)
            vec_cast<float, double>(s->ctx, 2 * s->mesh->lv[l].cells(), H[l].eta.p, s->h32[l].eta.p);
        vec_cast<float, double>(s->ctx, s->np, s->pm64.p, s->pm32.p);
        setup_level_operators<float>(s);
    }
    sync(s);
    s->ready = true;
}

// Mixed precision: the FP32 inner solves cannot resolve near-null modes whose relative
// eigenvalue is below about the FP32 unit roundoff times the growth of the
// preconditioner (free slip over a 1e6-weaker core: the core turning against the lid),
// and the refinement then stalls.  The solve goes on with FP64 inner solves: level
// scratch, operators and a Krylov basis on ro, allocated and set up here on first use.
void enable_fp64_inner(tng_solver* s) {
    if (!s->fp64_inner) {
        for (auto& M : s->h64) alloc_level_scratch<double>(s, M);
        alloc_krylov<double>(s, s->ro.p);
        s->d64.alloc(s->N);
        s->fp64_inner = true;
    }
    if (!s->fp64_ops) {
        setup_level_operators<double>(s);
        sync(s);
        s->fp64_ops = true;
    }
}

}  // namespace

template void chebyshev_steps<double>(const tng_ctx*, const Level&, const double*, double, const double*,
                                      const double*, double*, double*, double*, const double*, int, int, bool,
                                      bool);
template void chebyshev_steps<float>(const tng_ctx*, const Level&, const float*, double, const float*,
                                     const float*, float*, float*, float*, const double*, int, int, bool, bool);

// ---- lockstep batch of solver slots (serving) --------------------------------
// A slot is a solver built inside its own arena, so the buffers of all slots
// sit at the same offsets and one launch reaches every slot (SlotBatch).  The
// algorithm per slot is the one of tng_stokes_solve: FGMRES(restart) with the
// block preconditioner, FP64 refinement around FP32 inner solves when mixed.
// Slots of a step may be at different Krylov indices j: the basis vectors of
// the step are moved through index-free buffers (w, zb) with per-slot table
// indices, and the multi-dots / multi-axpys take per-slot vector counts.

struct SolverBatch::Slot {
    Arena arena;
    tng_solver* s = nullptr;
    DevBuf<double> eta, f;              // request viscosity and body force (in the arena)
    bool busy = false;
    int rc = TNG_OK;
    tng_solve_info info{};
    std::chrono::steady_clock::time_point t0;
    double* uo[3] = {nullptr, nullptr, nullptr};
    double* po = nullptr;
    // outer (refinement) state
    double bn = 0.0, relres = 0.0;
    int outer = 0, inner_total = 0;
    // Krylov cycle state
    double bnorm = 0.0, res = 0.0;
    int its = 0, j = 0, jend = 0;
    bool cycle_end = false, inner_done = false, failed = false;
    std::vector<double> H, cs, sn, g, y;
    ~Slot() {
        delete s;
        eta.release();
        f.release();
        if (arena.base) (void)hipFree(arena.base);
    }
};

constexpr int BATCH_STG = 4 * MAX_MDOT;   // staging doubles per slot

struct SolverBatch::Staging {
    DevBuf<double> rd, up;              // device staging rows (owned, outside the arenas)
    double* host = nullptr;             // pinned: read-back rows, then upload rows
    bool upload_pending = false;
    ~Staging() {
        if (host) (void)hipHostFree(host);
    }
    double* host_rd() { return host; }
    double* host_up() { return host + (size_t)MAX_BATCH * BATCH_STG; }
};

namespace {

using BSlot = SolverBatch::Slot;
using Group = std::vector<BSlot*>;

SlotBatch batch_of(const Group& g, const std::vector<int>* cnt) {
    TNG_REQUIRE(!g.empty() && (int)g.size() <= MAX_BATCH, "batch of 1..16 slots");
    SlotBatch b;
    b.nb = (int)g.size();
    b.has_cnt = cnt != nullptr ? 1 : 0;
    const char* base = g[0]->arena.base;
    for (int z = 0; z < b.nb; ++z) {
        b.off[z] = (long long)(g[z]->arena.base - base);
        if (cnt) b.cnt[z] = (*cnt)[z];
    }
    return b;
}

// k doubles at the reference slot's device address src, for every slot of g
const double* batch_gather(tng_ctx* ctx, SolverBatch::Staging& st, const Group& g, const double* src, int k) {
    const SlotBatch b = batch_of(g, nullptr);
    {
        BatchScope bs(&b);
        scal_gather(ctx, src, k, st.rd.p);
    }
    TNG_HIP(hipMemcpyAsync(st.host_rd(), st.rd.p, (size_t)b.nb * k * sizeof(double), hipMemcpyDeviceToHost,
                           ctx->stream));
    TNG_HIP(hipStreamSynchronize(ctx->stream));
    st.upload_pending = false;
    return st.host_rd();
}

// rows z * k .. of st.host_up() to the reference slot's device address dst of every slot of g
void batch_scatter(tng_ctx* ctx, SolverBatch::Staging& st, const Group& g, int k, double* dst) {
    const SlotBatch b = batch_of(g, nullptr);
    TNG_HIP(hipMemcpyAsync(st.up.p, st.host_up(), (size_t)b.nb * k * sizeof(double), hipMemcpyHostToDevice,
                           ctx->stream));
    st.upload_pending = true;
    BatchScope bs(&b);
    scal_scatter(ctx, st.up.p, k, dst);
}

double* host_up_rows(tng_ctx* ctx, SolverBatch::Staging& st) {
    if (st.upload_pending) {          // the last upload may still read the pinned rows
        TNG_HIP(hipStreamSynchronize(ctx->stream));
        st.upload_pending = false;
    }
    return st.host_up();
}

template <typename T>
T* inner_x(tng_solver* s);
template <>
float* inner_x<float>(tng_solver* s) { return s->d32.p; }
template <>
double* inner_x<double>(tng_solver* s) { return s->xo.p; }
template <typename T>
const T* inner_b(tng_solver* s);
template <>
const float* inner_b<float>(tng_solver* s) { return s->r32.p; }
template <>
const double* inner_b<double>(tng_solver* s) { return s->bo.p; }

void finish(BSlot* sl, int rc) {
    sl->rc = rc;
    sl->failed = rc != TNG_OK;
    sl->busy = false;
}

// Result of a finished slot to the caller's buffers (asynchronous).
void copy_out(tng_ctx* ctx, BSlot* sl) {
    tng_solver* s = sl->s;
    const long long ns = s->ns0, np = s->np;
    for (int c = 0; c < 3; ++c)
        TNG_HIP(hipMemcpyAsync(sl->uo[c], s->xo.p + c * ns, ns * sizeof(double), hipMemcpyDeviceToDevice,
                               ctx->stream));
    TNG_HIP(hipMemcpyAsync(sl->po, s->xo.p + 3 * ns, np * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
}

// new Krylov cycle of every slot of g from its (device) starting vector v with
// squared norm at the slot's Krylov coefficient 0: V_0 = v / |v|
template <typename T>
void begin_cycle(tng_ctx* ctx, const Group& g, const T* v, const double* host_sq, int stride, bool first) {
    tng_solver* r = g[0]->s;
    KrylovWS<T>& K = kws<T>(r);
    const SlotBatch b = batch_of(g, nullptr);
    {
        BatchScope bs(&b);
        vec_tab_copy<T>(ctx, r->N, v, nullptr, nullptr, (T* const*)K.vptr.p, 0, K.coef.p);
    }
    const int m = K.restart;
    for (size_t z = 0; z < g.size(); ++z) {
        BSlot* sl = g[z];
        const double beta = std::sqrt(std::max(0.0, host_sq[z * stride]));
        if (first) {
            sl->bnorm = beta;
            sl->its = 0;
            sl->H.assign((size_t)(m + 1) * m, 0.0);
            sl->cs.assign(m, 0.0);
            sl->sn.assign(m, 0.0);
            sl->y.assign(m, 0.0);
        }
        sl->g.assign(m + 1, 0.0);
        sl->g[0] = beta;
        sl->res = beta;
        sl->j = 0;
        sl->cycle_end = sl->inner_done = false;
    }
}

}  // namespace

SolverBatch::SolverBatch(tng_ctx* ctx, tng_mesh* mesh, const tng_solver_opts& opts)
    : ctx_(ctx), mesh_(mesh), opts_(opts), st_(std::make_unique<Staging>()) {
    TNG_REQUIRE(ctx != nullptr && mesh != nullptr, "NULL argument");
    TNG_HIP(hipSetDevice(ctx->device));
    // one slot's device bytes: the arena demand of building one
    const long long before = tl_arena_demand;
    {
        std::unique_ptr<tng_solver> probe(create_solver(ctx, mesh, &opts, true));
        const Level& L = mesh->lv[0];
        DevBuf<double> eta(2 * L.cells()), f(3 * L.node_slots());
        slot_bytes_ = tl_arena_demand - before;
    }
    st_->rd.alloc((size_t)MAX_BATCH * BATCH_STG);
    st_->up.alloc((size_t)MAX_BATCH * BATCH_STG);
    TNG_HIP(hipHostMalloc(reinterpret_cast<void**>(&st_->host), 2 * (size_t)MAX_BATCH * BATCH_STG * sizeof(double),
                          hipHostMallocDefault));
}

SolverBatch::~SolverBatch() {
    if (ctx_ && ctx_->stream) (void)hipStreamSynchronize(ctx_->stream);
    slot_.clear();
}

int SolverBatch::running() const {
    int n = 0;
    for (auto& sl : slot_) n += sl->busy ? 1 : 0;
    return n;
}

int SolverBatch::idle_slot() const {
    for (size_t i = 0; i < slot_.size(); ++i)
        if (!slot_[i]->busy) return (int)i;
    return -1;
}

int SolverBatch::add_slot() {
    auto sl = std::make_unique<Slot>();
    if (hipMalloc(reinterpret_cast<void**>(&sl->arena.base), (size_t)slot_bytes_) != hipSuccess) {
        sl->arena.base = nullptr;
        (void)hipGetLastError();
        throw Error(TNG_E_NOMEM, "slot arena of " + std::to_string(slot_bytes_) + " bytes failed");
    }
    sl->arena.cap = (size_t)slot_bytes_;
    {
        ArenaScope as(&sl->arena);
        sl->s = create_solver(ctx_, mesh_, &opts_, true);
        const Level& L = mesh_->lv[0];
        sl->eta.alloc(2 * L.cells());
        sl->f.alloc(3 * L.node_slots());
    }
    TNG_REQUIRE((long long)sl->arena.used == slot_bytes_, "slot layout differs from the measured one");
    slot_.push_back(std::move(sl));
    return (int)slot_.size() - 1;
}

void SolverBatch::remove_slot(int i) {
    TNG_REQUIRE(i >= 0 && i < (int)slot_.size() && !slot_[i]->busy, "only an idle slot can be removed");
    TNG_HIP(hipStreamSynchronize(ctx_->stream));
    slot_.erase(slot_.begin() + i);
}

int SolverBatch::rc(int i) const { return slot_.at(i)->rc; }
tng_solve_info SolverBatch::info(int i) const { return slot_.at(i)->info; }

namespace {

void set_info(BSlot* sl) {
    sl->info.outer_its = sl->outer;
    sl->info.inner_its = sl->inner_total;
    sl->info.fp64_its = sl->s->opts.mixed ? 0 : sl->inner_total;
    sl->info.rel_res = sl->relres;
    sl->info.status = sl->rc;
    sl->info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - sl->t0).count();
}

// inner solve of the slots of g (mixed precision): r32 = ro, d = 0, V_0 = r32 / |r32|
void begin_inner(tng_ctx* ctx, SolverBatch::Staging& st, const Group& g, std::vector<BSlot*>& done) {
    tng_solver* r = g[0]->s;
    KrylovWS<float>& K = r->k32;
    const SlotBatch b = batch_of(g, nullptr);
    {
        BatchScope bs(&b);
        vec_cast<float, double>(ctx, r->N, r->ro.p, r->r32.p);
        vec_fill<float>(ctx, r->N, 0.0f, r->d32.p);
        vec_smdot<float>(ctx, *r->ds, L0(r), L1(r), r->r32.p, K.wptr.p, 1, K.coef.p, false);
    }
    const double* hb = batch_gather(ctx, st, g, K.coef.p, 1);
    Group go;
    std::vector<double> sq;
    for (size_t z = 0; z < g.size(); ++z) {
        if (!(hb[z] > 0.0) || !std::isfinite(hb[z])) {
            finish(g[z], TNG_E_NOTCONV);           // nothing left to reduce, or a non-finite residual
            done.push_back(g[z]);
            continue;
        }
        go.push_back(g[z]);
        sq.push_back(hb[z]);
    }
    if (!go.empty()) begin_cycle<float>(ctx, go, go[0]->s->r32.p, sq.data(), 1, true);
}

// x += dx in FP64 and the true residual of the slots of g; finished slots go to done
template <typename T>
void outer_update(tng_ctx* ctx, SolverBatch::Staging& st, const tng_solver_opts& o, const Group& g,
                  std::vector<BSlot*>& done) {
    tng_solver* r = g[0]->s;
    const long long N = r->N;
    const SlotBatch b = batch_of(g, nullptr);
    {
        BatchScope bs(&b);
        if (std::is_same<T, float>::value) {
            vec_cast<double, float>(ctx, N, r->d32.p, r->ro.p);
            vec_axpby<double>(ctx, N, 1.0, r->ro.p, 1.0, r->xo.p);
        }
        remove_pressure_mean(r);
        apply_K<double>(r, r->h64[0].eta.p, r->xo.p, r->ro.p);
        vec_axpby<double>(ctx, N, 1.0, r->bo.p, -1.0, r->ro.p);
        vec_smdot<double>(ctx, *r->ds, L0(r), L1(r), r->ro.p, r->dptr.p + 1, 1, r->scal.p, false);
    }
    const double* hb = batch_gather(ctx, st, g, r->scal.p, 1);
    Group again;
    for (size_t z = 0; z < g.size(); ++z) {
        BSlot* sl = g[z];
        sl->inner_total += sl->its;
        sl->outer += 1;
        sl->relres = sl->bn > 0 ? std::sqrt(std::max(0.0, hb[z])) / sl->bn : 0.0;
        if (!std::isfinite(sl->relres)) {
            finish(sl, TNG_E_NOTCONV);
        } else if (sl->relres <= o.rtol) {
            finish(sl, TNG_OK);
        } else if (!std::is_same<T, float>::value || sl->outer >= o.max_outer) {
            finish(sl, TNG_E_NOTCONV);
        } else {
            again.push_back(sl);
            continue;
        }
        done.push_back(sl);
    }
    if (!again.empty()) begin_inner(ctx, st, again, done);
}

// one FGMRES iteration of the slots of g, then the work of the cycles that end
template <typename T>
void step_group(tng_ctx* ctx, SolverBatch::Staging& st, const tng_solver_opts& o, const Group& g,
                std::vector<BSlot*>& done) {
    tng_solver* r = g[0]->s;
    KrylovWS<T>& K = kws<T>(r);
    const int m = K.restart;
    const long long N = r->N;
    double* dsc = K.coef.p;
    const T* eta0 = hier<T>(r)[0].eta.p;
    T* const* vtab = (T* const*)K.vptr.p;
    T* const* ztab = (T* const*)K.zptr.p;
    const bool mixed = std::is_same<T, float>::value;
    const double rtol_in = mixed ? o.inner_rtol : o.rtol;
    const int maxit_in = mixed ? o.inner_max_iters : o.max_iters;
    const int nb = (int)g.size();
    std::vector<int> jv(nb), jv1(nb);
    for (int z = 0; z < nb; ++z) {
        jv[z] = g[z]->j;
        jv1[z] = g[z]->j + 1;
    }
    const SlotBatch bj = batch_of(g, &jv), bj1 = batch_of(g, &jv1), b0 = batch_of(g, nullptr);
    {
        BatchScope bs(&bj);
        vec_tab_copy<T>(ctx, N, nullptr, K.vptr.p, K.w.p, nullptr, 0, nullptr);     // w = V_j
    }
    {
        BatchScope bs(&b0);
        precond<T>(r, K.w.p, K.zb.p);                                                // zb = P^{-1} V_j
    }
    {
        BatchScope bs(&bj);
        vec_tab_copy<T>(ctx, N, K.zb.p, nullptr, nullptr, ztab, 0, nullptr);         // Z_j = zb
    }
    {
        BatchScope bs(&b0);
        apply_K<T>(r, eta0, K.zb.p, K.w.p);                                          // w = K Z_j
    }
    {
        BatchScope bs(&bj1);                                                         // CGS2 against V_0..V_j
        // (every slot's basis sits in its arena at 256-byte strides: 16-byte accesses)
        vec_smdot<T>(ctx, *r->ds, L0(r), L1(r), K.w.p, K.vptr.p, 1, dsc, false, true);
        vec_maxpy_smdot<T>(ctx, *r->ds, L0(r), L1(r), dsc, -1.0, K.vptr.p, 1, K.w.p, dsc + MAX_MDOT, false, true);
        vec_maxpy_smdot<T>(ctx, *r->ds, L0(r), L1(r), dsc + MAX_MDOT, -1.0, K.vptr.p, 1, K.w.p,
                           dsc + 2 * MAX_MDOT, true, true);
    }
    {
        BatchScope bs(&bj1);
        vec_tab_copy<T>(ctx, N, K.w.p, nullptr, nullptr, vtab, 0, dsc + 2 * MAX_MDOT);  // V_{j+1} = w / |w|
    }
    const int kr = 2 * MAX_MDOT + 1;
    const double* hb = batch_gather(ctx, st, g, dsc, kr);
    Group ends;
    for (int z = 0; z < nb; ++z) {
        BSlot* sl = g[z];
        const double* row = hb + (size_t)z * kr;
        const int j = sl->j;
        double* h = &sl->H[(size_t)j * (m + 1)];
        for (int i = 0; i <= j; ++i) h[i] = row[i] + row[MAX_MDOT + i];
        h[j + 1] = std::sqrt(std::max(0.0, row[2 * MAX_MDOT]));
        if (!std::isfinite(h[j + 1])) {
            sl->inner_total += sl->its;
            sl->outer += 1;
            finish(sl, TNG_E_NOTCONV);
            done.push_back(sl);
            continue;
        }
        for (int i = 0; i < j; ++i) {
            const double t0 = sl->cs[i] * h[i] + sl->sn[i] * h[i + 1];
            h[i + 1] = -sl->sn[i] * h[i] + sl->cs[i] * h[i + 1];
            h[i] = t0;
        }
        const double den = std::hypot(h[j], h[j + 1]);
        sl->cs[j] = den > 0 ? h[j] / den : 1.0;
        sl->sn[j] = den > 0 ? h[j + 1] / den : 0.0;
        h[j] = den;
        h[j + 1] = 0.0;
        sl->g[j + 1] = -sl->sn[j] * sl->g[j];
        sl->g[j] = sl->cs[j] * sl->g[j];
        sl->res = std::fabs(sl->g[j + 1]);
        sl->its += 1;
        sl->jend = j;
        if (sl->res <= rtol_in * sl->bnorm || sl->its >= maxit_in || h[j] == 0.0) {
            sl->cycle_end = sl->inner_done = true;
        } else if (j == m - 1) {
            sl->cycle_end = true;
        } else {
            sl->j = j + 1;
            continue;
        }
        ends.push_back(sl);
    }
    if (ends.empty()) return;
    // x += Z y with y = H^{-1} g (upper triangular) per slot
    double* up = host_up_rows(ctx, st);
    std::vector<int> cnt(ends.size());
    for (size_t z = 0; z < ends.size(); ++z) {
        BSlot* sl = ends[z];
        const int je = sl->jend;
        double* yrow = up + z * MAX_MDOT;
        for (int i = je; i >= 0; --i) {
            double acc = sl->g[i];
            for (int k = i + 1; k <= je; ++k) acc -= sl->H[(size_t)k * (m + 1) + i] * yrow[k];
            yrow[i] = acc / sl->H[(size_t)i * (m + 1) + i];
        }
        cnt[z] = je + 1;
    }
    // (a sub-group's launches name the buffers of its own first slot)
    tng_solver* re = ends[0]->s;
    KrylovWS<T>& KE = kws<T>(re);
    batch_scatter(ctx, st, ends, MAX_MDOT, KE.coef.p + 3 * MAX_MDOT);
    {
        const SlotBatch be = batch_of(ends, &cnt);
        BatchScope bs(&be);
        vec_maxpy<T>(ctx, N, KE.coef.p + 3 * MAX_MDOT, 1.0, KE.zptr.p, 1, inner_x<T>(re));
    }
    Group restart, fin;
    for (BSlot* sl : ends) (sl->inner_done ? fin : restart).push_back(sl);
    if (!restart.empty()) {
        // restart from the true inner residual w = b - K x
        tng_solver* rr = restart[0]->s;
        KrylovWS<T>& KR = kws<T>(rr);
        const SlotBatch br = batch_of(restart, nullptr);
        {
            BatchScope bs(&br);
            apply_K<T>(rr, hier<T>(rr)[0].eta.p, inner_x<T>(rr), KR.w.p);
            vec_axpby<T>(ctx, N, 1.0, inner_b<T>(rr), -1.0, KR.w.p);
            vec_smdot<T>(ctx, *rr->ds, L0(rr), L1(rr), KR.w.p, KR.wptr.p + 1, 1, KR.coef.p, false);
        }
        const double* hr = batch_gather(ctx, st, restart, KR.coef.p, 1);
        Group cont;
        std::vector<double> sq;
        for (size_t z = 0; z < restart.size(); ++z) {
            BSlot* sl = restart[z];
            const double beta = std::sqrt(std::max(0.0, hr[z]));
            sl->res = beta;
            if (beta <= rtol_in * sl->bnorm) {
                sl->inner_done = true;
                fin.push_back(sl);
            } else if (!std::isfinite(beta)) {
                sl->inner_total += sl->its;
                sl->outer += 1;
                finish(sl, TNG_E_NOTCONV);
                done.push_back(sl);
            } else {
                cont.push_back(sl);
                sq.push_back(hr[z]);
            }
        }
        if (!cont.empty()) {
            // the squared norms are already at each slot's coefficient 0
            begin_cycle<T>(ctx, cont, kws<T>(cont[0]->s).w.p, sq.data(), 1, false);
        }
    }
    if (!fin.empty()) outer_update<T>(ctx, st, o, fin, done);
}

}  // namespace

bool SolverBatch::start(int i, const double* T, double E, double Ra, double* const u_out[3], double* p_out) {
    Slot* sl = slot_.at(i).get();
    TNG_REQUIRE(!sl->busy, "slot is busy");
    TNG_REQUIRE(T != nullptr && u_out != nullptr && p_out != nullptr, "NULL argument");
    tng_solver* s = sl->s;
    const Level& L = mesh_->lv[0];
    const long long ns = s->ns0, np = s->np;
    hipStream_t stm = ctx_->stream;
    sl->t0 = std::chrono::steady_clock::now();
    for (int c = 0; c < 3; ++c) sl->uo[c] = u_out[c];
    sl->po = p_out;
    sl->rc = TNG_OK;
    sl->failed = false;
    sl->outer = sl->inner_total = 0;
    sl->its = 0;
    sl->relres = 0.0;
    sl->info = tng_solve_info{};
    sl->busy = true;
    std::vector<BSlot*> done;
    try {
        vec_fill<double>(ctx_, s->N, 0.0, s->xo.p);     // the result of a request that fails in set-up
        launch_eta_from_T(ctx_, L, TNG_F64, T, sl->eta.p, E, 0.0);
        double* f[3] = {sl->f.p, sl->f.p + ns, sl->f.p + 2 * ns};
        energy_buoyancy(ctx_, L, T, Ra, f);
        setup_viscosity(s, sl->eta.p);
        TNG_HIP(hipMemcpyAsync(s->bo.p, sl->f.p, 3 * ns * sizeof(double), hipMemcpyDeviceToDevice, stm));
        vec_fill<double>(ctx_, np, 0.0, s->bo.p + 3 * ns);
        vec_smdot<double>(ctx_, *s->ds, L0(s), L1(s), s->bo.p, s->dptr.p, 1, s->scal.p + 1, false);
        readback(s, s->scal.p + 1, 1);
        const double bsq = s->host[0];
        sl->bn = std::sqrt(std::max(0.0, bsq));
        if (!std::isfinite(sl->bn)) {
            finish(sl, TNG_E_NOTCONV);
        } else if (!(sl->bn > 0.0)) {
            finish(sl, TNG_OK);                       // b = 0: x = 0
        } else {
            sl->relres = 1.0;
            Group one{sl};
            if (opts_.mixed) {
                TNG_HIP(hipMemcpyAsync(s->ro.p, s->bo.p, s->N * sizeof(double), hipMemcpyDeviceToDevice, stm));
                begin_inner(ctx_, *st_, one, done);
            } else {
                // FP64: FGMRES on b itself, V_0 = b / |b| (|b|^2 at the Krylov coefficient 0)
                TNG_HIP(hipMemcpyAsync(s->k64.coef.p, s->scal.p + 1, sizeof(double), hipMemcpyDeviceToDevice, stm));
                begin_cycle<double>(ctx_, one, s->bo.p, &bsq, 1, true);
            }
        }
    } catch (const Error& e) {
        finish(sl, e.code);
    }
    if (!sl->busy) {
        copy_out(ctx_, sl);
        TNG_HIP(hipStreamSynchronize(stm));
        set_info(sl);
        return false;
    }
    return true;
}

std::vector<int> SolverBatch::step() {
    std::vector<int> run;
    for (size_t i = 0; i < slot_.size(); ++i)
        if (slot_[i]->busy) run.push_back((int)i);
    std::vector<BSlot*> done;
    for (size_t c0 = 0; c0 < run.size(); c0 += MAX_BATCH) {
        Group g;
        for (size_t k = c0; k < std::min(run.size(), c0 + MAX_BATCH); ++k) g.push_back(slot_[run[k]].get());
        try {
            if (opts_.mixed)
                step_group<float>(ctx_, *st_, opts_, g, done);
            else
                step_group<double>(ctx_, *st_, opts_, g, done);
        } catch (const Error& e) {
            // a launch or copy failed: every slot of the group ends with the error
            for (BSlot* sl : g)
                if (sl->busy) {
                    finish(sl, e.code);
                    done.push_back(sl);
                }
        }
    }
    std::vector<int> out;
    if (done.empty()) return out;
    for (BSlot* sl : done) copy_out(ctx_, sl);
    TNG_HIP(hipStreamSynchronize(ctx_->stream));
    for (BSlot* sl : done) {
        set_info(sl);
        for (size_t i = 0; i < slot_.size(); ++i)
            if (slot_[i].get() == sl) out.push_back((int)i);
    }
    return out;
}

}  // namespace tng

using tng::Error;

extern "C" {

int tng_solver_opts_default(tng_solver_opts* o) {
    TNG_API_BEGIN
    TNG_REQUIRE(o != nullptr, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->mixed = 0;
    o->restart = 10;
    o->max_iters = 200;
    o->rtol = 1e-8;
    o->cheb_degree = 2;
    o->pre = 2;
    o->post = 2;
    o->levels = 0;
    o->cheb_lo = 0.1;
    o->cheb_hi = 1.1;
    o->inner_rtol = 1e-4;
    o->inner_max_iters = 30;
    o->max_outer = 20;
    o->power_its = 10;
    o->hg_alpha = 0.0;
    o->graphs = 1;
    o->op_flags = 0;
    TNG_API_END
}

int tng_stokes_solver_create(tng_ctx* ctx, tng_mesh* mesh, const tng_solver_opts* opts, tng_solver** out) {
    TNG_API_BEGIN
    TNG_REQUIRE(out != nullptr, "NULL argument");
    *out = tng::create_solver(ctx, mesh, opts, false);
    TNG_API_END
}

int tng_stokes_solver_destroy(tng_solver* s) {
    TNG_API_BEGIN
    delete s;
    TNG_API_END
}

}  // extern "C"

namespace tng {

tng_solver* create_solver(tng_ctx* ctx, tng_mesh* mesh, const tng_solver_opts* opts, bool batch_slot) {
    TNG_REQUIRE(ctx != nullptr && mesh != nullptr && opts != nullptr, "NULL argument");
    TNG_REQUIRE(mesh->ctx != nullptr, "mesh was built without a context");
    TNG_REQUIRE(mesh->lv.size() >= 2, "the solver needs at least two mesh levels");
    TNG_REQUIRE(opts->restart >= 1 && opts->restart + 1 <= tng::MAX_MDOT, "restart must be in 1..23");
    TNG_REQUIRE(opts->rtol > 0 && opts->max_iters >= 1, "bad tolerance or iteration limit");
    TNG_REQUIRE(opts->cheb_degree >= 1 && opts->pre >= 0 && opts->post >= 0, "bad smoother options");
    TNG_REQUIRE(opts->cheb_lo > 0 && opts->cheb_hi > opts->cheb_lo, "bad Chebyshev interval");
    TNG_REQUIRE(opts->power_its >= 1, "power_its must be >= 1");
    TNG_REQUIRE(opts->hg_alpha >= 0.0 && std::isfinite(opts->hg_alpha), "hg_alpha must be finite and >= 0");
    TNG_REQUIRE(opts->op_flags == 0 || opts->op_flags == TNG_OP_TWOPOINT ||
                    (opts->op_flags & ~(unsigned)(TNG_OP_TALA | TNG_OP_FREESLIP_INNER | TNG_OP_FREESLIP_OUTER)) == 0,
                "op_flags must be 0, TNG_OP_TWOPOINT, or TNG_OP_TALA and/or free-slip bits (TNG_OP_FREESLIP_INNER, "
                "TNG_OP_FREESLIP_OUTER or both)");
    TNG_REQUIRE(!(opts->op_flags & (TNG_OP_FREESLIP_INNER | TNG_OP_FREESLIP_OUTER)) || opts->hg_alpha == 0.0,
                "free slip has no hourglass-controlled form (hg_alpha must be 0)");
    TNG_REQUIRE(!(opts->op_flags & TNG_OP_TWOPOINT) || opts->hg_alpha == 0.0,
                "the two-radial-point rule is an alternative to hourglass control (hg_alpha must be 0)");
    TNG_REQUIRE(!(opts->op_flags & TNG_OP_TALA) || mesh->lv[0].rho64.p != nullptr,
                "op_flags TNG_OP_TALA needs the mesh's reference density (tng_mesh_set_density)");
    TNG_REQUIRE(!batch_slot || opts->op_flags == 0, "the serving batches take the plain operator only (op_flags 0)");
    const int nlev = opts->levels > 0 ? opts->levels : (int)mesh->lv.size();
    TNG_REQUIRE(nlev >= 2 && nlev <= (int)mesh->lv.size(), "levels out of range");
    for (int l = 0; l + 1 < nlev; ++l)
        TNG_REQUIRE(mesh->lv[l].m % 2 == 0 && mesh->lv[l].n % 2 == 0, "every non-coarsest level needs even m, n");
    TNG_HIP(hipSetDevice(ctx->device));
    auto s = std::make_unique<tng_solver>();
    s->ctx = ctx;
    s->mesh = mesh;
    s->opts = *opts;
    s->batch_slot = batch_slot;
    s->nlev = nlev;
    s->ns0 = mesh->lv[0].node_slots();
    s->np = mesh->lv[1].node_slots();
    s->N = 3 * s->ns0 + s->np;
    // the vector kernels take Stokes-vector lengths (with the basis padding) as 32-bit counts
    TNG_REQUIRE(s->N + 64 < (1LL << 32), "mesh too large for the solver: a Stokes vector must have fewer than 2^32 values");
    s->ds = std::make_unique<tng::DotScratch>();
    tng::build_coarse_maps(s.get());
    const bool mixed = opts->mixed != 0;
    tng::alloc_hierarchy<double>(s.get(), !mixed);
    s->pm64.alloc(s->np);
    s->xo.alloc(s->N);
    s->ro.alloc(s->N);
    s->bo.alloc(s->N);
    if (mixed) {
        tng::alloc_hierarchy<float>(s.get(), true);
        s->r32.alloc(s->N);
        s->d32.alloc(s->N);
        tng::alloc_krylov<float>(s.get(), s->r32.p);
        s->pm32.alloc(s->np);
    } else {
        tng::alloc_krylov<double>(s.get(), s->bo.p);
    }
    s->ones_p.alloc(s->np);
    tng::vec_fill<double>(ctx, s->np, 1.0, s->ones_p.p);
    s->ones_p32.alloc(s->np);
    tng::vec_fill<float>(ctx, s->np, 1.0f, s->ones_p32.p);
    {
        const double* o64 = s->ones_p.p;
        const float* o32 = s->ones_p32.p;
        s->onesp64.alloc(1);
        s->onesp32.alloc(1);
        TNG_HIP(hipMemcpy(s->onesp64.p, &o64, sizeof(o64), hipMemcpyHostToDevice));
        TNG_HIP(hipMemcpy(s->onesp32.p, &o32, sizeof(o32), hipMemcpyHostToDevice));
    }
    s->scal.alloc(64);
    {
        const double* dp[4] = {s->bo.p, s->ro.p, s->xo.p + 3 * s->ns0, s->k64.w.p};
        s->dptr.alloc(4);
        TNG_HIP(hipMemcpy(s->dptr.p, dp, sizeof(dp), hipMemcpyHostToDevice));
        // count of unique pressure nodes for the mean projection
        const tng::Level& P = mesh->lv[1];
        const double cnt = (double)P.n_unique_lat * (P.n + 1);
        TNG_HIP(hipMemcpy(s->scal.p + 33, &cnt, sizeof(double), hipMemcpyHostToDevice));
        TNG_HIP(hipMemcpy(s->scal.p + 41, &cnt, sizeof(double), hipMemcpyHostToDevice));
    }
    if (tng::fs_bits(s.get()) == 3) {
        // rigid rotations of the velocity level, orthonormalised over unique DoFs by the
        // Cholesky factor of their Gram matrix (Q = R L^{-T})
        const tng::Level& L = mesh->lv[0];
        const long long n3 = 3 * s->ns0;
        s->rot64.alloc(3 * n3);
        double* r[3];
        const double* rp[3];
        for (int a = 0; a < 3; ++a) {
            r[a] = s->rot64.p + a * n3;
            rp[a] = r[a];
            double* o[3] = {r[a], r[a] + s->ns0, r[a] + 2 * s->ns0};
            tng::vec_rotation<double>(ctx, L, a, o);
        }
        s->rotptr64.alloc(3);
        TNG_HIP(hipMemcpy(s->rotptr64.p, rp, sizeof(rp), hipMemcpyHostToDevice));
        for (int a = 0; a < 3; ++a)
            tng::vec_mdot<double>(ctx, *s->ds, n3, L.n + 1, L.lat_slots(), L.owner.p, rp[a], s->rotptr64.p, 3,
                                  s->scal.p + 48 + 3 * a, false);
        double G[9];
        TNG_HIP(hipMemcpyAsync(G, s->scal.p + 48, sizeof(G), hipMemcpyDeviceToHost, ctx->stream));
        TNG_HIP(hipStreamSynchronize(ctx->stream));
        const double l00 = std::sqrt(G[0]);
        const double l10 = G[3] / l00, l20 = G[6] / l00;
        const double l11 = std::sqrt(G[4] - l10 * l10);
        const double l21 = (G[7] - l20 * l10) / l11;
        const double l22 = std::sqrt(G[8] - l20 * l20 - l21 * l21);
        TNG_REQUIRE(std::isfinite(l22) && l22 > 0.0, "rigid rotations: singular Gram matrix");
        tng::vec_axpby<double>(ctx, n3, 0.0, r[0], 1.0 / l00, r[0]);                       // q0 = r0 / l00
        tng::vec_axpby<double>(ctx, n3, -l10, r[0], 1.0, r[1]);                             // q1
        tng::vec_axpby<double>(ctx, n3, 0.0, r[1], 1.0 / l11, r[1]);
        tng::vec_axpby<double>(ctx, n3, -l20, r[0], 1.0, r[2]);                             // q2
        tng::vec_axpby<double>(ctx, n3, -l21, r[1], 1.0, r[2]);
        tng::vec_axpby<double>(ctx, n3, 0.0, r[2], 1.0 / l22, r[2]);
        s->rot32.alloc(3 * n3);
        tng::vec_cast<float, double>(ctx, 3 * n3, s->rot64.p, s->rot32.p);
        const float* rp32[3] = {s->rot32.p, s->rot32.p + n3, s->rot32.p + 2 * n3};
        s->rotptr32.alloc(3);
        TNG_HIP(hipMemcpy(s->rotptr32.p, rp32, sizeof(rp32), hipMemcpyHostToDevice));
    }
    TNG_HIP(hipHostMalloc(reinterpret_cast<void**>(&s->host), 256 * sizeof(double), hipHostMallocDefault));
    if (opts->graphs && !batch_slot) {
        TNG_HIP(hipStreamCreateWithFlags(&s->gstream, hipStreamNonBlocking));   // default priority
        if (tng_ctx_create(ctx->device, s->gstream, &s->gctx) != TNG_OK)
            throw Error(TNG_E_HIP, "graph context creation failed");
        TNG_HIP(hipEventCreateWithFlags(&s->ev_in, hipEventDisableTiming));
        TNG_HIP(hipEventCreateWithFlags(&s->ev_out, hipEventDisableTiming));
    }
    TNG_HIP(hipStreamSynchronize(ctx->stream));
    return s.release();
}

}  // namespace tng

extern "C" {

int tng_stokes_solver_setup(tng_solver* s, const double* eta_wedge) {
    TNG_API_BEGIN
    TNG_REQUIRE(s != nullptr && eta_wedge != nullptr, "NULL argument");
    tng::require_device(s->ctx, eta_wedge, 2 * tng::L0(s).cells() * sizeof(double), "eta_wedge");
    TNG_HIP(hipSetDevice(s->ctx->device));
    tng::setup_viscosity(s, eta_wedge);
    TNG_API_END
}

int tng_stokes_solve(tng_solver* s, const double* eta_wedge, const double* const f[3], const double* g,
                     double* const u[3], double* p, tng_solve_info* info) {
    TNG_API_BEGIN
    TNG_REQUIRE(s != nullptr && f != nullptr && u != nullptr && p != nullptr, "NULL argument");
    for (int c = 0; c < 3; ++c) TNG_REQUIRE(f[c] != nullptr && u[c] != nullptr, "NULL field pointer");
    {
        const size_t nsb = (size_t)s->ns0 * sizeof(double), npb = (size_t)s->np * sizeof(double);
        if (eta_wedge) tng::require_device(s->ctx, eta_wedge, 2 * tng::L0(s).cells() * sizeof(double), "eta_wedge");
        for (int c = 0; c < 3; ++c) {
            tng::require_device(s->ctx, f[c], nsb, "f");
            tng::require_device(s->ctx, u[c], nsb, "u");
        }
        if (g) tng::require_device(s->ctx, g, npb, "g");
        tng::require_device(s->ctx, p, npb, "p");
    }
    TNG_HIP(hipSetDevice(s->ctx->device));
    auto t0 = std::chrono::steady_clock::now();
    if (eta_wedge) tng::setup_viscosity(s, eta_wedge);
    TNG_REQUIRE(s->ready, "no viscosity: pass eta_wedge or call tng_stokes_solver_setup first");
    const long long ns = s->ns0, np = s->np, N = s->N;
    hipStream_t st = s->ctx->stream;
    const bool mixed = s->opts.mixed != 0;
    double* bvec = s->bo.p;
    double* xo = s->xo.p;
    double* ro = s->ro.p;
    for (int c = 0; c < 3; ++c)
        TNG_HIP(hipMemcpyAsync(bvec + c * ns, f[c], ns * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (g)
        TNG_HIP(hipMemcpyAsync(bvec + 3 * ns, g, np * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
        tng::vec_fill<double>(s->ctx, np, 0.0, bvec + 3 * ns);
    if (tng::fs_flag(s)) tng::project_mean<double>(s, bvec + 3 * ns);   // mass rows modulo constants
    const double* const* bp = s->dptr.p;         // -> bo
    const double* const* rp = s->dptr.p + 1;     // -> ro
    tng::vec_smdot<double>(s->ctx, *s->ds, tng::L0(s), tng::L1(s), bvec, bp, 1, s->scal.p + 1, false);
    tng::readback(s, s->scal.p + 1, 1);
    const double bn = std::sqrt(s->host[0]);
    int status = TNG_OK;
    int inner_total = 0, outer = 0, fp64_total = 0;
    double relres = bn > 0 ? 1.0 : 0.0;
    auto true_residual = [&]() {
        tng::remove_pressure_mean(s);
        tng::remove_rotations(s);
        tng::apply_K<double>(s, s->h64[0].eta.p, xo, ro);
        tng::vec_axpby<double>(s->ctx, N, 1.0, bvec, -1.0, ro);
        tng::vec_smdot<double>(s->ctx, *s->ds, tng::L0(s), tng::L1(s), ro, rp, 1, s->scal.p, false);
        tng::readback(s, s->scal.p, 1);
        return bn > 0 ? std::sqrt(s->host[0]) / bn : 0.0;
    };
    if (!mixed) {
        int its = 0;
        double est = 0.0;
        status = tng::fgmres<double>(s, s->h64[0].eta.p, bvec, xo, s->opts.rtol, s->opts.max_iters, &its, &est);
        inner_total = its;
        outer = 1;
        relres = true_residual();
        if (!std::isfinite(relres)) status = TNG_E_NOTCONV;
    } else {
        tng::vec_fill<double>(s->ctx, N, 0.0, xo);
        TNG_HIP(hipMemcpyAsync(ro, bvec, N * sizeof(double), hipMemcpyDeviceToDevice, st));
        double best = relres;
        int stalled = 0;
        while (relres > s->opts.rtol && outer < s->opts.max_outer) {
            if (stalled >= 2) {
                // two refinement steps in a row left the residual above 0.9 of the best
                // one: FGMRES in FP64 on K d = r to the remaining tolerance
                tng::enable_fp64_inner(s);
                int its = 0;
                double est = 0.0;
                const int left = std::max(1, s->opts.max_iters - fp64_total);
                const int rc = tng::fgmres<double>(s, s->h64[0].eta.p, ro, s->d64.p, s->opts.rtol / relres, left,
                                                   &its, &est);
                inner_total += its;
                fp64_total += its;
                ++outer;
                if (rc != TNG_OK) {
                    status = rc;
                    break;
                }
                tng::vec_axpby<double>(s->ctx, N, 1.0, s->d64.p, 1.0, xo);
                relres = true_residual();
                if (!std::isfinite(relres)) {
                    status = TNG_E_NOTCONV;
                    break;
                }
                if (fp64_total >= s->opts.max_iters) break;
                continue;
            }
            tng::vec_cast<float, double>(s->ctx, N, ro, s->r32.p);
            int its = 0;
            double inner_rel = 0.0;
            const int rc = tng::fgmres<float>(s, s->h32[0].eta.p, s->r32.p, s->d32.p, s->opts.inner_rtol,
                                              s->opts.inner_max_iters, &its, &inner_rel);
            inner_total += its;
            ++outer;
            if (rc != TNG_OK) {
                status = rc;
                break;
            }
            // x += d in FP64, then the FP64 residual r = b - K x
            tng::vec_cast<double, float>(s->ctx, N, s->d32.p, ro);
            tng::vec_axpby<double>(s->ctx, N, 1.0, ro, 1.0, xo);
            relres = true_residual();
            if (!std::isfinite(relres)) {
                status = TNG_E_NOTCONV;
                break;
            }
            stalled = relres > 0.9 * best ? stalled + 1 : 0;
            best = std::min(best, relres);
        }
    }
    if (status == TNG_OK && !(relres <= s->opts.rtol)) status = TNG_E_NOTCONV;
    for (int c = 0; c < 3; ++c)
        TNG_HIP(hipMemcpyAsync(u[c], xo + c * ns, ns * sizeof(double), hipMemcpyDeviceToDevice, st));
    TNG_HIP(hipMemcpyAsync(p, xo + 3 * ns, np * sizeof(double), hipMemcpyDeviceToDevice, st));
    TNG_HIP(hipStreamSynchronize(st));
    if (info) {
        info->outer_its = outer;
        info->inner_its = inner_total;
        info->fp64_its = mixed ? fp64_total : inner_total;
        info->rel_res = relres;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->status = status;
    }
    if (status != TNG_OK) {
        tng::set_last_error("Stokes solve did not reach rtol (rel_res " + std::to_string(relres) + ")");
        return status;
    }
    TNG_API_END
}

int tng_energy_step(tng_solver* s, const tng_step_opts* o, const double* H, double* T, double* const u[3],
                    double* p, tng_step_info* info) {
    TNG_API_BEGIN
    TNG_REQUIRE(s != nullptr && o != nullptr && T != nullptr && u != nullptr && p != nullptr, "NULL argument");
    for (int c = 0; c < 3; ++c) TNG_REQUIRE(u[c] != nullptr, "NULL velocity pointer");
    TNG_REQUIRE(std::isfinite(o->Ra) && std::isfinite(o->E) && std::isfinite(o->F), "non-finite parameter");
    TNG_REQUIRE(o->dt > 0 || o->courant > 0, "need dt > 0 or courant > 0");
    TNG_REQUIRE(o->energy_restart >= 1 && o->energy_restart + 1 <= tng::MAX_MDOT, "energy_restart in 1..23");
    TNG_REQUIRE(o->scheme == 0 || o->scheme == 1, "scheme must be 0 (SUPG) or 1 (MMOC)");
    TNG_REQUIRE(!(s->opts.op_flags & TNG_OP_TALA),
                "the coupled step is of the Boussinesq form: its solver must not take TNG_OP_TALA");
    {
        const size_t nsb = (size_t)s->ns0 * sizeof(double);
        if (H) tng::require_device(s->ctx, H, nsb, "H");
        tng::require_device(s->ctx, T, nsb, "T");
        for (int c = 0; c < 3; ++c) tng::require_device(s->ctx, u[c], nsb, "u");
        tng::require_device(s->ctx, p, (size_t)s->np * sizeof(double), "p");
    }
    TNG_HIP(hipSetDevice(s->ctx->device));
    auto t0 = std::chrono::steady_clock::now();
    const tng::Level& L = tng::L0(s);
    const long long ns = s->ns0;
    if (!s->ews) s->ews = tng::energy_ws_create();
    if (s->eta_step.n == 0) s->eta_step.alloc(2 * L.cells());
    if (s->f_step.n == 0) s->f_step.alloc(3 * ns);
    // viscosity of the current temperature, buoyancy, Stokes solve
    tng::launch_eta_from_T(s->ctx, L, TNG_F64, T, s->eta_step.p, o->E, o->F);
    double* f[3] = {s->f_step.p, s->f_step.p + ns, s->f_step.p + 2 * ns};
    // rows of a free-slip sphere: the tangential part of the buoyancy (zero normal velocity)
    tng::energy_buoyancy(s->ctx, L, T, o->Ra, f, tng::fs_bits(s));
    const double* fc[3] = {f[0], f[1], f[2]};
    tng_solve_info sinfo{};
    const int rc = tng_stokes_solve(s, s->eta_step.p, fc, nullptr, u, p, &sinfo);
    if (rc != TNG_OK && rc != TNG_E_NOTCONV) return rc;
    // time step and energy solve
    const double* uc[3] = {u[0], u[1], u[2]};
    const double dt = o->dt > 0 ? o->dt : tng::energy_cfl_dt(s->ctx, L, *s->ews, uc, o->courant);
    int eits = 0;
    double erel = 0.0;
    const int erc = o->scheme == 1
                        ? tng::energy_solve_mmoc(s->ctx, L, *s->ews, uc, H, dt, o->T_inner, o->T_outer, T,
                                                 o->energy_rtol, o->energy_max_iters, o->energy_restart, &eits, &erel)
                        : tng::energy_solve(s->ctx, L, *s->ews, uc, H, dt, o->T_inner, o->T_outer, T, o->energy_rtol,
                                            o->energy_max_iters, o->energy_restart, &eits, &erel);
    TNG_HIP(hipStreamSynchronize(s->ctx->stream));
    if (info) {
        info->stokes = sinfo;
        info->energy_its = eits;
        info->energy_rel_res = erel;
        info->dt = dt;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (rc != TNG_OK) {
        tng::set_last_error("Stokes solve of the time step did not converge");
        return rc;
    }
    if (erc != TNG_OK) {
        tng::set_last_error("energy solve did not reach energy_rtol");
        return erc;
    }
    TNG_API_END
}

// One V-cycle of the solver's velocity preconditioner on level 0 (x = M^{-1} b),
// in the solver's Krylov precision.  Needs a prior setup.
int tng_stokes_solver_vcycle(tng_solver* s, const void* const b[3], void* const x[3]) {
    TNG_API_BEGIN
    TNG_REQUIRE(s != nullptr && b != nullptr && x != nullptr, "NULL argument");
    TNG_REQUIRE(s->ready, "call tng_stokes_solver_setup first");
    for (int c = 0; c < 3; ++c) {
        const size_t vb = (size_t)s->ns0 * (s->opts.mixed ? sizeof(float) : sizeof(double));
        tng::require_device(s->ctx, b[c], vb, "b");
        tng::require_device(s->ctx, x[c], vb, "x");
    }
    TNG_HIP(hipSetDevice(s->ctx->device));
    const long long ns = s->ns0;
    hipStream_t st = s->ctx->stream;
    if (s->opts.mixed) {
        auto& M = s->h32[0];
        for (int c = 0; c < 3; ++c)
            TNG_HIP(hipMemcpyAsync(M.b.p + c * ns, b[c], ns * sizeof(float), hipMemcpyDeviceToDevice, st));
        tng::vcycle<float>(s, 0, M.b.p, s->k32.t.p);
        for (int c = 0; c < 3; ++c)
            TNG_HIP(hipMemcpyAsync(x[c], s->k32.t.p + c * ns, ns * sizeof(float), hipMemcpyDeviceToDevice, st));
    } else {
        auto& M = s->h64[0];
        for (int c = 0; c < 3; ++c)
            TNG_HIP(hipMemcpyAsync(M.b.p + c * ns, b[c], ns * sizeof(double), hipMemcpyDeviceToDevice, st));
        tng::vcycle<double>(s, 0, M.b.p, s->k64.t.p);
        for (int c = 0; c < 3; ++c)
            TNG_HIP(hipMemcpyAsync(x[c], s->k64.t.p + c * ns, ns * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
    TNG_API_END
}

}  // extern "C"
