// Declarations of the multigrid / Krylov launchers (mg_kernels.hip) and the
// small device-side helper objects they share with the solver.
#pragma once

#include <algorithm>
#include <type_traits>

#include "tng_internal.hpp"

namespace tng {

constexpr int MAX_MDOT = 24;          // vectors in one multi-dot / multi-axpy
constexpr int DOT_BLOCKS = 4096;      // partial sums of a reduction (enough waves to fill HBM)
constexpr int MAX_COARSE_DOF = 1024;  // dense coarsest-level solve

template <typename T>
constexpr tng_prec prec_of() {
    return std::is_same<T, double>::value ? TNG_F64 : TNG_F32;
}

struct DotScratch {
    DevBuf<double> part;   // DOT_BLOCKS x MAX_MDOT
    DotScratch() : part((size_t)DOT_BLOCKS * MAX_MDOT) {}
};

// Dense inverse of the coarsest-level viscous operator over its unique
// interior DoFs.
struct CoarseDense {
    int ndof = 0;
    long long nslots = 0;
    DevBuf<int> dof_slot;   // [ndof]: (owner slot << 2) | component
    DevBuf<int> slot_dof;   // [3][nslots]: DoF of every copy, -1 on Dirichlet rows
    DevBuf<int> copy_ptr;   // [ndof + 1]: copies of each DoF (CSR)
    DevBuf<int> copy_slot;  //   (slot << 2) | component of every copy
    DevBuf<double> Ainv;    // ndof x ndof
    DevBuf<double> rotq;    // [3][ndof] orthonormal rigid rotations + sigma (free slip on both spheres)
};

// free slip on both spheres: A <- A + sigma Q Q^T over the coarsest DoFs, Q the
// orthonormalised rigid rotations, sigma the mean diagonal (before coarse_invert)
void coarse_rotation_shift(const tng_ctx* ctx, CoarseDense& cd, const Level& L);
// rigid rotation e_a x x at every node slot of L, in three component fields
template <typename T>
void vec_rotation(const tng_ctx* ctx, const Level& L, int a, T* const out[3]);

template <typename T>
// twopt: the viscous block with the two-radial-point rule (hg_alpha must then be 0);
// fs: free-slip spheres (bit 0 inner, bit 1 outer, the TNG_OP_FREESLIP_* bits >> 4),
// whose rows get the isotropic projected diagonal trace(P A_jj P) / 2
void mg_diag_A(const tng_ctx* ctx, const Level& L, const T* eta, double hg_alpha, T* const d[3], bool twopt = false,
               unsigned fs = 0);
// x <- P x + N b at the free-slip layers fs (b == nullptr: b = 0)
template <typename T>
void vec_fs_project(const tng_ctx* ctx, const Level& L, unsigned fs, T* const x[3], const T* const b[3]);
template <typename T>
void mg_pmass(const tng_ctx* ctx, const Level& L, const Level& Lp, const T* eta, T* mdiag);
template <typename T>
void mg_prolong(const tng_ctx* ctx, const Level& Lf, const T* const c[3], T* const f[3], bool add);
template <typename T>
// fs: free-slip spheres of the coarse level, whose layers are restricted like the
// interior and then projected (no-slip layers are zero)
void mg_restrict(const tng_ctx* ctx, const Level& Lf, const Level& Lc, const T* const f[3], T* const c[3],
                 unsigned fs = 0);
// x, d <- one Chebyshev step with (alpha, beta) = ab_dev[2k], ab_dev[2k + 1]
template <typename T>
void vec_cheb_update(const tng_ctx* ctx, long long n, const double* ab_dev, int k, const T* b, const T* y,
                     const T* invd, T* d, T* x);
// One step of the two-term Chebyshev recurrence x_k+1 = x_k + alpha (x_k - x_k-1) +
// beta D^-1 (b - A_D x_k) after a raw viscous apply y = A x_k (launch_stokes_apply_raw):
// completes the duplicated nodes (sum of the copies) and the no-slip identity rows on
// the fly.  xo: x_k-1 in (not read when alpha = 0 or prev_zero, then taken as 0),
// x_k+1 out.  first: the step from x_k = 0 (y and xk not read).
template <typename T>
void vec_cheb_post_update(const tng_ctx* ctx, const Level& L, bool ns_in, bool ns_out, const double* ab_dev, int k,
                          bool first, bool prev_zero, const T* b, const T* y, const T* invd, const T* xk, T* xo);
// r = b - A_D x from a raw viscous apply y = A x (closing pass fused, as above)
template <typename T>
void vec_resid_post(const tng_ctx* ctx, const Level& L, bool ns_in, bool ns_out, const T* b, const T* x, const T* y,
                    T* r);
template <typename T>
void vec_invert(const tng_ctx* ctx, long long n, T* a);
template <typename TO, typename TI>
void vec_cast(const tng_ctx* ctx, long long n, const TI* a, TO* b);
template <typename T>
void vec_axpby(const tng_ctx* ctx, long long n, double a, const T* x, double b, T* y);
template <typename T>
void vec_mdot(const tng_ctx* ctx, DotScratch& ds, long long n, int n1, long long nlat, const uint8_t* owner,
              const T* x, const T* const* vs_dev, int nq, double* out_dev, bool accumulate);
template <typename T>
void vec_mul(const tng_ctx* ctx, long long n, const T* a, const T* b, T* c);
template <typename T>
void vec_maxpy(const tng_ctx* ctx, long long n, const double* coef_dev, double sign, const T* const* vs_dev,
               int nq, T* y);
template <typename T>
void coarse_unit(const tng_ctx* ctx, const CoarseDense& cd, int col, T* const x[3]);
template <typename T>
void coarse_gather(const tng_ctx* ctx, const CoarseDense& cd, int col, const T* const y[3], double* Ad);
void coarse_invert(const tng_ctx* ctx, CoarseDense& cd);
template <typename T>
void coarse_solve(const tng_ctx* ctx, const CoarseDense& cd, const T* const b[3], T* const x[3]);
template <typename T>
void vec_shift(const tng_ctx* ctx, long long n, const double* sum_cnt, T* p);
template <typename T>
void vec_schur(const tng_ctx* ctx, long long n, const T* r, const T* mdiag, T* z);
template <typename T>
void vec_fill(const tng_ctx* ctx, long long n, T v, T* a);
template <typename T>
// vs_aligned: every vector of vs_dev (of every slot of a batch) is 16-byte aligned (then, in
// FP32 with x aligned, the kernel takes 16-byte accesses)
void vec_smdot(const tng_ctx* ctx, DotScratch& ds, const Level& Lu, const Level& Lp, const T* x,
               const T* const* vs_dev, int nq, double* out_dev, bool accumulate, bool vs_aligned = false);
// y <- y + sign * sum_q coef[q] v_q over a Stokes vector, then out = the owner-masked
// dots of the new y with v_0..v_{nq-1} (norm false) or its squared norm (norm true)
template <typename T>
void vec_maxpy_smdot(const tng_ctx* ctx, DotScratch& ds, const Level& Lu, const Level& Lp, const double* coef_dev,
                     double sign, const T* const* vs_dev, int nq, T* y, double* out_dev, bool norm,
                     bool vs_aligned = false);
template <typename T>
void vec_rand(const tng_ctx* ctx, long long n, unsigned long long seed, T* a);
template <typename T>
void vec_scale_rsqrt(const tng_ctx* ctx, long long n, const double* s, const T* x, T* y);
// y = f x: x = src or src_tab[idx], y = dst or dst_tab[idx] (idx per slot in a
// batch with counts), f = 1 / sqrt(*sq) or 1 when sq is NULL
template <typename T>
void vec_tab_copy(const tng_ctx* ctx, long long n, const T* src, const T* const* src_tab, T* dst, T* const* dst_tab,
                  int idx, const double* sq);
// staging[z * k + i] = src_z[i] and dst_z[i] = staging[z * k + i] for the slots z of a batch
void scal_gather(const tng_ctx* ctx, const double* src, int k, double* staging);
void scal_scatter(const tng_ctx* ctx, const double* staging, int k, double* dst);
template <typename T>
void coarse_assemble(const tng_ctx* ctx, const CoarseDense& cd, const Level& L, const T* eta, double hg_alpha,
                     bool twopt = false, unsigned fs = 0);

struct EnergyWS;
EnergyWS* energy_ws_create();
void energy_ws_destroy(EnergyWS* w);
int energy_solve(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const u[3], const double* H,
                 double dt, double T_in, double T_out, double* T, double rtol, int maxit, int restart, int* its,
                 double* rel);
double energy_cfl_dt(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const u[3], double courant);
int energy_solve_mmoc(const tng_ctx* ctx, const Level& L, EnergyWS& W, const double* const u[3], const double* H,
                      double dt, double T_in, double T_out, double* T, double rtol, int maxit, int restart, int* its,
                      double* rel);
// That = T^n at the departure points of the nodes (explicit midpoint rule backwards
// over dt along the W1 velocity u), W1-interpolated (eq:departure); FP64 node fields.
void mmoc_departure(const tng_ctx* ctx, const Level& L, const double* const u[3], double dt, const double* Tn,
                    double* That);
// fs: free-slip spheres (bit 0 inner, bit 1 outer): their rows keep the tangential part
void energy_buoyancy(const tng_ctx* ctx, const Level& L, const double* T, double Ra, double* const f[3],
                     unsigned fs = 0);
template <typename T>
void energy_apply(const tng_ctx* ctx, const Level& L, const T* const u[3], double dt, const T* Tin, T* y);
// Streaming energy apply (levels with at most 256 radial layers): y = E(u) T with the
// Dirichlet rows; u == NULL applies the operator without flow (lumped mass and
// diffusion only).
bool energy_stream_fits(const Level& L);
template <typename T>
void energy_apply_stream(const tng_ctx* ctx, const Level& L, const T* const u[3], double dt, const T* Tin, T* y);
// tbar, rhoalpha: device [n+1] profiles of the compressible (TALA) form, or NULL for
// the Boussinesq form (Tbar = 0, rhobar alphabar = 1)
template <typename T>
void buoyancy_rhs(const tng_ctx* ctx, const Level& L, const T* Tn, double Ra, T* const f[3],
                  const double* tbar = nullptr, const double* rhoalpha = nullptr, unsigned fs = 0);

// Coefficients (alpha_k, beta_k), k < deg, of one Chebyshev smoothing step of
// degree deg for the eigenvalue interval [lo, hi].
std::vector<double> chebyshev_coefficients(int deg, double lo, double hi);
// the same into ab[0 .. 2 max(deg, 1))
void chebyshev_coefficients(int deg, double lo, double hi, double* ab);
template <typename T>
void chebyshev_steps(const tng_ctx* ctx, const Level& L, const T* eta, double hg_alpha, const T* invd, const T* b,
                     T* x, T* y, T* d, const double* ab_dev, int deg, int steps, bool x_zero, bool twopt = false);

}  // namespace tng
