/*
 * tng.h -- C ABI of the MI355X-native matrix-free wedge Stokes library.
 *
 * Method: TERRA-NG (arXiv 2609.21633).  The library builds the icosahedral
 * shell mesh of Sec. 2, applies the W1-iso-W2 / W1 wedge Stokes operator of
 * Sec. 3 with the one-point quadrature of Sec. 4, and solves the saddle-point
 * system of Sec. 7 with the block-triangular Schur preconditioner of
 * eq:block-precond whose velocity block is a geometric multigrid V-cycle with
 * Chebyshev smoothing.  A W1 temperature step (Sec. 6 scheme list, SUPG form)
 * and a continuous-batching request server sit on top.
 *
 * Conventions shared by every call
 * --------------------------------
 * Return value: TNG_OK (0) or a negative TNG_E_* code; tng_last_error() then
 *   returns a message for the calling thread.  Arguments are validated before
 *   any kernel is launched; a failed validation launches nothing.
 * Ownership: handles (tng_ctx, tng_mesh, tng_solver, tng_server) are created
 *   and destroyed by the library.  Field pointers are caller-owned memory and
 *   are never freed or retained beyond the call (server submissions excepted,
 *   see tng_server_submit).
 * Memory: "device" pointers must be ordinary (coarse-grained) device memory
 *   of the context's GPU from hipMalloc, e.g. torch CUDA tensors, holding the
 *   whole field; "host" pointers are ordinary host memory.  Every call checks
 *   its device pointers (hipPointerGetAttributes: device memory of the
 *   context's device, not managed; hipMemGetAddressRange: the field fits in
 *   the allocation) and returns TNG_E_INVAL otherwise.  Host, pinned-host and
 *   managed memory are refused: the operator kernels add seam partial sums
 *   with floating-point atomics that are only reliable on coarse-grained
 *   device memory.
 * Streams: applies, smoothers, transfers and field kernels are enqueued on the
 *   context's stream and return without synchronising.  Solves, energy steps
 *   and server polls synchronise that stream.
 * Precision: tng_prec selects the element type of every field pointer of a
 *   call (double for TNG_F64, float for TNG_F32).  Solve inputs and outputs are
 *   always double.
 *
 * Layouts (level l of a mesh has m = mt / 2^l lateral intervals per diamond
 * edge and n = nr / 2^l radial intervals):
 *   node field   [10][m+1][m+1][n+1]  diamond, i, j, radial layer k fastest.
 *                Nodes on diamond edges are stored once per diamond that holds
 *                them ("duplicate group"); inputs must hold equal values in all
 *                copies and outputs are returned with equal values in all
 *                copies.
 *   velocity     three node fields, one per Cartesian component (SoA), passed
 *                as an array of three pointers.
 *   pressure     one node field on level l + 1 (W1 on the coarser grid).
 *   wedge field  [10][m][m][n][2]: hexahedral cell (i, j, k) of diamond d is
 *                split into wedge 0 with lateral nodes (i,j),(i+1,j),(i,j+1)
 *                and wedge 1 with (i+1,j+1),(i,j+1),(i+1,j); the split is
 *                parallel to the diamond's shared diagonal (Sec. 2).
 *   lateral node (i, j) of diamond d is the recursive geodesic-midpoint
 *                refinement of the diamond's corners (0,0), (m,0), (0,m), (m,m):
 *                north diamonds d = 0..4: N, U_d, U_{d+1}, L_d;
 *                south diamonds d = 5..9: U_{d-4}, L_{d-5}, L_{d-4}, S;
 *                with poles N, S on the z axis, upper ring U_k at z = 1/sqrt 5 and
 *                longitude 2 pi k/5, lower ring L_k at z = -1/sqrt 5 and longitude
 *                2 pi k/5 + pi/5 (indices mod 5).  Radii are uniform on [r_in, r_out].
 */
#ifndef TNG_H
#define TNG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tng_ctx tng_ctx;
typedef struct tng_mesh tng_mesh;
typedef struct tng_solver tng_solver;
typedef struct tng_server tng_server;

typedef enum { TNG_F64 = 0, TNG_F32 = 1 } tng_prec;

enum {
    TNG_OK = 0,
    TNG_E_INVAL = -1,    /* bad argument: null pointer, size, level, flag */
    TNG_E_NOMEM = -2,    /* device or host allocation failed */
    TNG_E_HIP = -3,      /* a HIP runtime call failed */
    TNG_E_NOTCONV = -4,  /* solver did not reach its tolerance, or met NaN/Inf */
    TNG_E_BUDGET = -5,   /* request does not fit the server's memory budget */
    TNG_E_STATE = -6     /* call not valid in the object's current state */
};

/* Operator blocks of K = [[A, B^T], [B, 0]] (Sec. 7).  Any non-empty subset. */
enum {
    TNG_OP_A = 1,       /* viscous block A(eta), eq:elemmat with one-point rule */
    TNG_OP_BT = 2,      /* gradient block B^T (pressure -> velocity)           */
    TNG_OP_B = 4,       /* divergence block B (velocity -> pressure)           */
    TNG_OP_DIRICHLET = 8, /* zero-velocity rows on both spheres: identity rows,
                            columns dropped (K_D = [[DAD + I - D, DB^T],[BD, 0]]) */
    /* Free slip (the paper's verification setup, Sec. 8) on the inner / outer
     * sphere instead: a node's velocity is taken in the frame (rhat, two
     * tangents), rhat = the node's unit vector; the normal component is a
     * Dirichlet DoF (identity row, column dropped), the tangential ones are
     * free (zero tangential traction).  In Cartesian components, with
     * P = I - rhat rhat^T and N = rhat rhat^T at the sphere's nodes:
     * y_u = P (A P u + B^T p) + N u there, y_p = B P u.  A sphere with its
     * free-slip bit set is free slip whatever TNG_OP_DIRICHLET says; the other
     * sphere is no slip with TNG_OP_DIRICHLET and unconstrained without it. */
    TNG_OP_FREESLIP_INNER = 16,
    TNG_OP_FREESLIP_OUTER = 32,
    /* Compressible mass balance (TALA, Sec. 1 eq:mass, div(rhobar u) = 0): the
     * divergence rows become -(psi_I, div(rhobar u)) with the mass flux
     * rhobar u interpolated nodally (rhobar(r_j) u_j, rhobar from
     * tng_mesh_set_density), i.e. y_p = B R u with R = diag(rhobar(r_j)); the
     * momentum rows keep B^T (eq:stokes).  With TNG_OP_B, alone or in the full
     * operator, also with free slip (y_p = B R P u); not with hourglass control. */
    TNG_OP_TALA = 64,
    /* The viscous block with the two-radial-point rule (Sec. 4, the remedy
     * beside eq:hgstab): the lateral centroid times the two-point Gauss rule
     * in zeta (-+1/sqrt 3, weight 1/2 each); B and B^T keep the one point.
     * With TNG_OP_A (alone, with B^T, or the full operator); not with
     * hg_alpha > 0, free slip or TNG_OP_TALA. */
    TNG_OP_TWOPOINT = 128
};

/* Message of the last failed call on this thread ("" if none).  Library-owned. */
const char* tng_last_error(void);

/* ---- context ----------------------------------------------------------- */
/* device: HIP device ordinal.  hip_stream: a hipStream_t owned by the caller
 * (may be NULL for the null stream); the library enqueues all work on it. */
int tng_ctx_create(int device, void* hip_stream, tng_ctx** out);
int tng_ctx_set_stream(tng_ctx* ctx, void* hip_stream);
int tng_ctx_destroy(tng_ctx* ctx);
/* Band count of the operator apply (a tuning override, Sec. 3 kernel layout):
 * the apply splits every diamond's cell rows into bands streamed by one
 * workgroup each.  bands = 0 (the default) chooses the count per launch from
 * the chip's resident workgroups; bands > 0 forces that many bands (clamped to
 * [1, m/2] on a level of m rows; unequal bands start on even rows).  Results do
 * not depend on it beyond rounding.  TNG_E_INVAL for bands < 0. */
int tng_ctx_set_apply_bands(tng_ctx* ctx, int bands);
/* Measurement: with enable != 0, every call records a HIP event pair on the
 * context stream around its main kernel, under the name
 * "<kernel>/<precision>/<variant>/<m>x<n>" (kernels "stokes_apply" with
 * variant A, BT, B, A+BT, ... and a "+HG" suffix for hourglass control, then
 * "/b<bands>" and, for serving batches, "/batch"; "energy_apply").  tng_ctx_kernel_stats synchronises on the recorded events
 * and returns the summed elapsed milliseconds and the number of launches
 * since profiling was (re)enabled, over the names equal to `name` or starting
 * with `name` + "/" (so "stokes_apply" sums every variant); none gives 0 and
 * 0.  tng_ctx_kernel_stats_at returns the index-th recorded full name (copied
 * into name, at most name_len bytes with the terminator) and its figures,
 * TNG_E_INVAL past the last one. */
int tng_ctx_profile(tng_ctx* ctx, int enable);
int tng_ctx_kernel_stats(tng_ctx* ctx, const char* name, double* total_ms, long long* launches);
int tng_ctx_kernel_stats_at(tng_ctx* ctx, int index, char* name, int name_len, double* total_ms,
                            long long* launches);

/* Plain streaming copy dst = src of `bytes` device bytes (a multiple of 16,
 * both pointers 16-byte aligned, not overlapping), enqueued on the context's
 * stream and timed as "stream_copy" when profiling is on: the practical HBM
 * roof (2 x bytes moved per launch) that the operator kernels are measured
 * against, and a kernel of known traffic for scaling HBM counters. */
int tng_stream_copy(tng_ctx* ctx, const void* src, void* dst, size_t bytes);
/* Checks that `bytes` bytes at p are device memory that every call of this
 * library accepts (the check every entry point applies to its device
 * pointers): TNG_OK, or TNG_E_INVAL with the reason in tng_last_error(). */
int tng_check_device_buffer(tng_ctx* ctx, const void* p, size_t bytes);

/* ---- mesh (Sec. 2) ------------------------------------------------------ */
/* Builds the shell with mt lateral intervals per diamond edge (power of two)
 * and nr radial intervals on [r_in, r_out], and uploads `levels` levels to the
 * context's device.  ctx may be NULL: then only the host-side description is
 * built (counts, coordinates, duplicate groups) and the mesh cannot be used by
 * device calls, which reject it with TNG_E_INVAL.  Levels:
 * (level l = (mt/2^l, nr/2^l); both must stay integers >= 1).  The pressure of
 * level l lives on level l + 1, so an operator on level l needs l + 1 < levels.
 * Fields are indexed with 32-bit offsets: 10(mt+1)^2(nr+1) < 2^31 and
 * 20 mt^2 nr < 2^32, else TNG_E_INVAL (the (512,512) shell is the largest
 * power-of-two shell that fits; a solver further needs its Stokes vector,
 * 3 node fields plus the pressure, below 2^32 values). */
int tng_mesh_create(tng_ctx* ctx, int mt, int nr, double r_in, double r_out,
                    int levels, tng_mesh** out);
/* out[0..7] = m, n, lateral slots 10(m+1)^2, unique lateral nodes 10 m^2 + 2,
 *             node slots 10(m+1)^2(n+1), unique nodes (10 m^2 + 2)(n+1),
 *             hexahedral cells 10 m^2 n, wedges 20 m^2 n. */
int tng_mesh_counts(const tng_mesh* mesh, int level, long long out[8]);
/* Host copies: unit vectors [10][m+1][m+1][3] and radii [n+1].  Either may be NULL. */
int tng_mesh_coords(const tng_mesh* mesh, int level, double* unit_xyz_host, double* r_host);
/* Host copy [10][m+1][m+1]: unique lateral node id of every lateral slot, ids
 * numbered by first appearance in slot order; equal ids = one duplicate group. */
int tng_mesh_dup_groups(const tng_mesh* mesh, int level, int* unique_id_host);
int tng_mesh_destroy(tng_mesh* mesh);
/* Reference density of the compressible (TALA) terms, Sec. 1: rho_host[k] =
 * rhobar(r_k) at the nr + 1 radial node layers of the finest level (host
 * array, copied; every value finite and > 0).  Level l uses the values of its
 * own layers (every 2^l-th).  The mesh must have been built with a context. */
int tng_mesh_set_density(tng_mesh* mesh, const double* rho_host);

/* ---- operator (Sec. 3 eq:matfree, eq:epsq, eq:localapply) -------------- */
/* y = K(eta) x restricted to the blocks in op_flags, on level `level`.
 * eta_wedge: device wedge field of level `level`.  u[3]: device velocity in;
 * p: device pressure (level + 1) in, may be NULL unless TNG_OP_BT is set.
 * y_u[3]: device velocity out (required if TNG_OP_A or TNG_OP_BT);
 * y_p: device pressure out (required if TNG_OP_B).  Outputs are overwritten
 * (not accumulated) and are assembled: every copy of a duplicate node holds
 * the full sum.  With TNG_OP_DIRICHLET the velocity input is read as zero on
 * both spheres and y_u = u there.  Inputs and outputs must not alias.
 * hg_alpha: hourglass control of the viscous block (Sec. 4, eq:hgstab), 0 for
 *   the plain one-point operator.  With alpha > 0 every wedge adds
 *   eps_e sum_a sum_d (h_a (x) e_d)(h_a (x) e_d)^T to A_e, summed over the three
 *   barycentric hourglass modes h_a = (lambda_a - 1/3) zeta (span of w_1, w_2,
 *   independent of the wedge's vertex numbering), eps_e = alpha mean(diag A_e).
 *   Must be finite and >= 0 (TNG_E_INVAL otherwise). */
int tng_stokes_apply(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec,
                     unsigned op_flags, double hg_alpha, const void* eta_wedge,
                     const void* const u[3], const void* p,
                     void* const y_u[3], void* y_p);

/* Decomposition that tng_stokes_apply uses for these arguments (the kernel
 * layout of Sec. 5 as built here; for tests that target its seams and for
 * measurement).  Launches nothing.  out[0..7] = cell columns per workgroup
 * tile, waves per column (radial split), cells per lane, waves per workgroup,
 * tiles per diamond, bands per diamond (the per-launch choice, or the forced
 * count of tng_ctx_set_apply_bands), radial ranges per column, cells per
 * radial range.  Band b of m rows covers the cell rows
 * [2 floor(b (m/2) / bands), 2 floor((b+1) (m/2) / bands)); tile t covers the
 * cell columns [t tile, (t+1) tile); radial range c covers the cells
 * [c range, (c+1) range) and is split into stretches of 64 x (cells per lane). */
int tng_stokes_apply_layout(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, unsigned op_flags,
                            double hg_alpha, int out[8]);

/* ---- fields ------------------------------------------------------------- */
/* Per-wedge viscosity from nodal temperature: eta_e = exp(-E Tbar_e + F (1 - r_m)),
 * Tbar_e the mean of the wedge's six nodal values (the W1 interpolant at q_c,
 * Sec. 4) and r_m the wedge's mid radius; the Frank-Kamenetskii family of
 * Sec. 8 with a depth factor.  T: device node field of `level`; eta_wedge:
 * device wedge field of `level`. */
int tng_eta_from_temperature(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec,
                             const void* T, double E, double F, void* eta_wedge);
/* Re-discretised coarse viscosity for the multigrid hierarchy (Sec. 7): each
 * wedge of level fine_level + 1 gets the arithmetic mean of the 8 fine wedges
 * it contains (4 lateral children x 2 layers). */
int tng_eta_coarsen(tng_ctx* ctx, const tng_mesh* mesh, int fine_level, tng_prec prec,
                    const void* eta_fine, void* eta_coarse);

/* ---- multigrid pieces (Sec. 7) ------------------------------------------ */
/* Diagonal of K_D's viscous block on `level`: diag_(node,c) = sum over the
 * node's wedges of V eta (|grad phi|^2 + (d_c phi)^2 / 3) (eq:elemmat, one
 * point), plus 2/3 eps_e per wedge with hourglass control (hg_alpha as in
 * tng_stokes_apply), 1 on Dirichlet rows.  diag[3]: device velocity field out. */
int tng_diag_A(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
               double hg_alpha, void* const diag[3]);
/* diag(A) of the viscous block with the two-radial-point rule (Sec. 4; the
 * operator of TNG_OP_TWOPOINT): the sum over the node's wedges and over the
 * two points zeta = -+1/sqrt 3 of (V_q / 2) eta (|grad phi|^2 + 1/3
 * (d_c phi)^2), 1 on Dirichlet rows.  Arguments as in tng_diag_A. */
int tng_diag_A_twopoint(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
                        void* const diag[3]);
/* Row-sum lumped inverse-viscosity pressure mass of eq:pmass on the pressure
 * level of `level` (i.e. level + 1): m_I = sum_e (V_e / eta_e) psi_I(q_c^e).
 * mass: device node field of level + 1 out.  The Schur preconditioner is
 * S^{-1} r = -r / m. */
int tng_pressure_mass(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
                      void* mass);
/* Chebyshev smoother: `steps` applications of x <- x + p(D^{-1} A)(b - A x),
 * p the degree-`degree` Chebyshev polynomial for the eigenvalue interval
 * [lmin, lmax] of D^{-1} A (A with Dirichlet rows and hourglass control
 * hg_alpha, D = diag).  diag: the diagonal as returned by tng_diag_A.  x is
 * updated in place.  Allocates scratch and synchronises. */
int tng_smooth(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
               double hg_alpha, const void* const diag[3], const void* const b[3], void* const x[3], int degree,
               int steps, double lmin, double lmax);
/* tng_smooth without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Arguments, result and stream as in tng_smooth,
 * except: degree <= 16, and the call neither allocates nor synchronises.  Its
 * five work vectors and step coefficients live in one library-owned device
 * array of 48 MiB per GPU (held from the first tng_ctx_create on that GPU
 * until the process ends): a level needs 5 x 3 x node_slots values (rounded
 * up to 256-byte pieces) plus 256 bytes, so levels up to (32,32) fit in FP64
 * and FP32; larger levels return TNG_E_INVAL and launch nothing.  Every call
 * on a GPU uses that GPU's one array: calls enqueued on one stream are ordered,
 * but calls that overlap on one GPU (different streams or contexts) race. */
int tng_smooth_noalloc(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
                       double hg_alpha, const void* const diag[3], const void* const b[3], void* const x[3],
                       int degree, int steps, double lmin, double lmax);
/* W1 transfer between fine_level and fine_level + 1 (index-space
 * interpolation: coarse nodes copied, edge midpoints and odd layers averaged).
 * Restriction c = P^T f with Dirichlet layers of c set to zero; prolongation
 * f = P c (overwrites f).  Velocity fields of the two levels. */
int tng_restrict(tng_ctx* ctx, const tng_mesh* mesh, int fine_level, tng_prec prec, const void* const f[3],
                 void* const c[3]);
int tng_prolong(tng_ctx* ctx, const tng_mesh* mesh, int fine_level, tng_prec prec, const void* const c[3],
                void* const f[3]);

/* ---- Stokes solver (Sec. 7) --------------------------------------------- */
/* Options of the FGMRES / block-preconditioner / multigrid solve.
 * mixed: 0 = everything FP64; 1 = FP64 iterative refinement (outer residual,
 *   correction, pressure-mean projection, coarsest solve in FP64) around an
 *   FP32 inner FGMRES (FP32 applies, smoothers and Krylov basis).
 * restart: FGMRES restart length (paper: 10; 1..23).
 * max_iters: FGMRES iteration limit (FP64 mode, and of the FP64 inner solves
 *   of a mixed solve whose refinement stalled).  rtol: target of
 *   ||b - K x||_2 / ||b||_2 over unique DoFs, both blocks, x0 = 0.
 * cheb_degree, pre, post: Chebyshev smoother of degree cheb_degree on
 *   D^{-1} A, pre/post steps per level (paper: 2, 2, 2), on the interval
 *   [cheb_lo, cheb_hi] * lambda_max(D^{-1} A), lambda_max from power_its
 *   seeded power iterations.  With free slip on a sphere of much weaker
 *   viscosity (contrast 1e6) the largest eigenvalue can belong to a mode
 *   localised there that 10 iterations miss; the stand-alone FP32 V-cycle
 *   then needs about 100; a mixed solve there stalls and finishes with FP64
 *   inner solves (tng_solve_info).
 * levels: multigrid levels used (0 = all levels of the mesh); the coarsest
 *   one is solved exactly and must have at most 1024 interior DoFs.
 * inner_rtol, inner_max_iters, max_outer: mixed-precision inner tolerance and
 *   iteration limit per refinement step, and the refinement step limit.
 * hg_alpha: hourglass control (eq:hgstab, see tng_stokes_apply) of the viscous
 *   block on every level: the solve is then of that stabilised operator.
 * graphs: 1 (default) replays the preconditioner of each Krylov index as a
 *   HIP graph captured at its first use (on a private stream ordered with the
 *   context's stream by events); 0 launches every kernel from the host.
 * op_flags: operator variant of the solve (Sec. 4, eq:stokes), 0 (default) or
 *   one of
 *   TNG_OP_TWOPOINT: the viscous block with the two-radial-point rule on every
 *     level (outer operator, smoother and residual applies, diag(A) and the
 *     coarsest matrix), so that the multigrid works on the operator without
 *     one-point hourglass modes; hg_alpha must be 0;
 *   TNG_OP_TALA (alone or with the free-slip bits): the outer operator's mass
 *     rows -(psi, div(rhobar u)) with the mesh's reference density
 *     (tng_mesh_set_density before the solver is created); the preconditioner
 *     keeps A, B^T and M_{1/eta}.  The right-hand side g must sum to zero over
 *     unique pressure nodes (with no slip 1^T B_rho = 0; with free slip the
 *     mass rows are taken modulo constants, below).
 *   TNG_OP_FREESLIP_INNER and/or TNG_OP_FREESLIP_OUTER: free slip on that sphere
 *     (rows P A P + N, P = I - rhat rhat^T at its nodes, as in tng_stokes_apply),
 *     no slip on a sphere without the bit, on every level: the smoother keeps the iterate
 *     tangential there (normal rows solved exactly, an isotropic diagonal
 *     trace(P A_jj P) / 2), transfers keep the layer, the coarsest matrix
 *     includes it.  The normal component of f at its nodes is the prescribed
 *     normal velocity (0 for an impermeable sphere: tng_rhs_buoyancy_bc; the
 *     coupled step does so).  The node-normal projection keeps the constant
 *     pressure in the null space only to O(h^2) (B_D^T 1 != 0): the solve takes
 *     the mass rows modulo constants with a zero-mean pressure, the gauge of the
 *     no-slip case.  Both bits: free slip on both spheres; the rigid rotations
 *     e_a x x are then a null space too: f must be orthogonal to them (a
 *     buoyancy force is), the coarsest matrix is shifted by sigma Q Q^T on them
 *     (Q orthonormal, sigma its mean diagonal) and the solution is returned
 *     orthogonal to them (inner products over unique DoFs).
 *   Not for the serving batches, which take op_flags 0; hg_alpha must be 0
 *   with every option but TNG_OP_TALA. */
typedef struct {
    int mixed;
    int restart;
    int max_iters;
    double rtol;
    int cheb_degree;
    int pre, post;
    int levels;
    double cheb_lo, cheb_hi;
    double inner_rtol;
    int inner_max_iters;
    int max_outer;
    int power_its;
    double hg_alpha;
    int graphs;
    unsigned op_flags;
} tng_solver_opts;

/* outer_its: refinement steps (1 in FP64 mode); inner_its: FGMRES iterations
 * in total; rel_res: final true FP64 relative residual; seconds: wall time
 * of the call; status: TNG_OK or TNG_E_NOTCONV; fp64_its: the FGMRES
 * iterations made in FP64 (all of them in FP64 mode).  A mixed-precision
 * solve whose refinement stalls (two steps in a row each leaving the residual
 * above 0.9 of the best so far: FP32 cannot resolve modes of K whose relative
 * eigenvalue is near its roundoff, as with free slip over a much weaker core)
 * finishes with FP64 inner FGMRES (at most max_iters iterations), allocating
 * the FP64 multigrid scratch and Krylov basis on first use. */
typedef struct {
    int outer_its, inner_its;
    double rel_res;
    double seconds;
    int status;
    int fp64_its;
} tng_solve_info;

/* Fills the defaults listed above (FP64, restart 10, rtol 1e-8, degree 2, 2+2). */
int tng_solver_opts_default(tng_solver_opts* opts);
/* The solver keeps the multigrid hierarchy, Krylov basis and scratch on the
 * device (library-owned) for the mesh's levels; the mesh must outlive it. */
int tng_stokes_solver_create(tng_ctx* ctx, tng_mesh* mesh, const tng_solver_opts* opts, tng_solver** out);
int tng_stokes_solver_destroy(tng_solver* solver);
/* Viscosity-dependent setup: per-level averaged viscosity, diagonals and
 * Chebyshev intervals, lumped pressure mass, dense coarsest inverse.
 * eta_wedge: device FP64 wedge field of level 0.  Synchronises. */
int tng_stokes_solver_setup(tng_solver* solver, const double* eta_wedge);
/* Solves K_D [u; p] = [f; g] (saddle point of Sec. 7) with x0 = 0.
 * eta_wedge: device FP64 wedge field, or NULL to reuse the last setup.
 * f[3]: device FP64 velocity right-hand side (its Dirichlet rows are the
 * prescribed boundary velocity; zero in all uses here); g: device FP64
 * pressure right-hand side or NULL for zero.  u[3], p: device FP64 outputs;
 * the pressure is returned with zero nodal mean over unique nodes.
 * Synchronises.  Returns TNG_E_NOTCONV (outputs still written) if rtol was
 * not reached within the limits or a NaN/Inf appeared. */
int tng_stokes_solve(tng_solver* solver, const double* eta_wedge, const double* const f[3], const double* g,
                     double* const u[3], double* p, tng_solve_info* info);
/* One V-cycle of the velocity preconditioner on level 0, x = M^{-1} b, in the
 * solver's Krylov precision (FP32 when mixed).  b, x: device velocity fields. */
int tng_stokes_solver_vcycle(tng_solver* solver, const void* const b[3], void* const x[3]);

/* ---- buoyancy and energy (Sec. 6) --------------------------------------- */
/* Buoyancy right-hand side of eq:stokes in Boussinesq form (rho = alpha = 1):
 * f_(i,c) = sum_e V_e N_i(q_c) Ra T(q_c) rhat_c(q_c), one-point rule, T(q_c)
 * the mean of the wedge's nodal temperatures and rhat the direction of x(q_c);
 * Dirichlet rows zero.  T: device node field; f[3]: device velocity out. */
int tng_rhs_buoyancy(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* T, double Ra,
                     void* const f[3]);
/* tng_rhs_buoyancy for free-slip spheres (the setup of Sec. 8): bc_flags holds
 * TNG_OP_FREESLIP_INNER and/or TNG_OP_FREESLIP_OUTER; the rows of such a sphere
 * keep the tangential part of the buoyancy and a zero normal part (zero
 * normal velocity in the free-slip rows of the solve), the rows of the other
 * spheres are zero.  bc_flags 0 is tng_rhs_buoyancy. */
int tng_rhs_buoyancy_bc(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, unsigned bc_flags,
                        const void* T, double Ra, void* const f[3]);
/* Buoyancy of the compressible (TALA) form of eq:stokes, with the split
 * T = Tbar(r) + T' of eq:tsplit: f_(i,c) = sum_e V_e N_i(q_c) Ra
 * (rhobar alphabar)(q_c) T'(q_c) rhat_c(q_c), both factors the W1 interpolants
 * of their nodal values, T'_j = T_j - Tbar(r_j).  Tbar_host, rhoalpha_host:
 * host arrays of the n + 1 radial node layers of `level` (Tbar(r_k) and
 * rhobar(r_k) alphabar(r_k)).  Otherwise as tng_rhs_buoyancy. */
int tng_rhs_buoyancy_tala(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* T, double Ra,
                          const double* Tbar_host, const double* rhoalpha_host, void* const f[3]);
/* Backward-Euler SUPG energy operator (unit diffusivity, Sec. 6 scheme list):
 * y_i = sum_e V_e [ N_i T_i / dt + grad phi_i . grad T + N_i ubar . grad T
 *                   + tau_e (ubar . grad phi_i)(ubar . grad T) ],
 * ubar the wedge's mean velocity, tau_e = h/(2|ubar|)(coth Pe - 1/Pe),
 * Pe = |ubar| h / 2, h = V_e^(1/3); identity rows on both spheres (Dirichlet
 * temperature; columns kept).  u[3], T in, y out: device fields of `level`. */
int tng_energy_apply(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* const u[3],
                     double dt, const void* T, void* y);

/* The advection half of an MMOC step (Sec. 6, eq:departure): T_hat at every
 * node = T at the node's departure point, traced back over dt with the
 * explicit midpoint rule along the velocity u (both W1 fields, linear
 * interpolation in the wedge that contains the point; a point outside the
 * shell is brought back radially onto it).  u[3], T: device FP64 node fields
 * of `level`; T_hat: device FP64 out (equal in all copies of a node). */
int tng_mmoc_advect(tng_ctx* ctx, const tng_mesh* mesh, int level, const double* const u[3], double dt,
                    const double* T, double* T_hat);

/* Coupled time step.  Ra: Rayleigh number; eta = exp(-E T + F (1 - r));
 * dt > 0 fixes the time step, else dt = courant * min_e h_e / |ubar_e|;
 * T_inner / T_outer: temperature on the inner / outer sphere; the energy
 * solve is Jacobi-preconditioned GMRES(energy_restart) to energy_rtol. */
typedef struct {
    double Ra, E, F;
    double dt, courant;
    double T_inner, T_outer;
    double energy_rtol;
    int energy_max_iters, energy_restart;
    /* energy scheme (Sec. 6): 0 = SUPG-stabilised backward Euler; 1 = the
     * modified method of characteristics (eq:mmoc): T at the departure points
     * of the nodes (explicit midpoint rule backwards along u, W1
     * interpolation), then the implicit diffusion step (M/dt + K) T^{n+1} =
     * M (That/dt + H) by the same Jacobi-GMRES; with courant > 0 and dt <= 0
     * the step is courant x the CFL step (MMOC is not CFL-bound, so courant
     * may exceed 1). */
    int scheme;
} tng_step_opts;

typedef struct {
    tng_solve_info stokes;
    int energy_its;
    double energy_rel_res;
    double dt;
    double seconds;
} tng_step_info;

/* One step: eta(T^n), f = Ra T^n rhat, Stokes solve for (u, p), dt, then the
 * energy solve (M/dt + K + C(u) + S(u)) T^{n+1} = M (T^n/dt + H).  H: device
 * FP64 internal heating node field or NULL; T: device FP64, in/out; u[3], p:
 * device FP64 outputs (solver levels 0 / 1).  Synchronises. */
int tng_energy_step(tng_solver* solver, const tng_step_opts* opts, const double* H, double* T,
                    double* const u[3], double* p, tng_step_info* info);

/* ---- serving ------------------------------------------------------------ */
/* Request server for streams of Stokes solves.  levels: nlevels pairs
 * (mt, nr), each kept resident with its multigrid hierarchy, its own HIP
 * stream and one host driver thread.  Requests are admitted FIFO per level
 * into solver slots at iteration boundaries; the running slots of a level
 * advance together, every kernel of an FGMRES iteration launched once for all
 * of them (continuous batching: finished slots are refilled with queued
 * requests at the next boundary), and levels overlap through their streams.
 * A slot is one device allocation holding a whole solver; its size is
 * measured here, by building one slot of each level.  A new slot is created
 * only while that per-slot memory keeps the total within hbm_budget_bytes (an
 * idle slot of another level is released to make room when needed); at most
 * max_slots slots per level, launched in groups of at most 16.  opts: solver
 * options of every slot (normally mixed precision). */
int tng_server_create(tng_ctx* ctx, const int* levels, int nlevels, size_t hbm_budget_bytes, int max_slots,
                      const tng_solver_opts* opts, tng_server** out);
/* Queues a solve with eta = 10^(log10_contrast)^(-T) = exp(-ln(contrast) T)
 * and right-hand side Ra T rhat (buoyancy, g = 0) on level level_idx.  T:
 * device FP64 node field of that level; u_out[3], p_out: device FP64 outputs.
 * All three stay borrowed until the request is done.  Returns a ticket;
 * TNG_E_BUDGET if one slot of the level cannot fit the budget. */
int tng_server_submit(tng_server* srv, int level_idx, const double* T, double log10_contrast, double Ra,
                      double* const u_out[3], double* p_out, long long* ticket);
/* done = 1 when finished; then info, latency (submit -> result on the device)
 * and queueing time (submit -> start) are filled and the request's own
 * status is returned (a failed request does not affect the others). */
int tng_server_poll(tng_server* srv, long long ticket, int* done, tng_solve_info* info, double* latency_s,
                    double* queue_s);
/* Blocks until the ticket (or, for ticket <= 0, every request) is done. */
int tng_server_wait(tng_server* srv, long long ticket);
int tng_server_stats(tng_server* srv, long long* bytes_in_use, int* slots, int* busy, int* queued);
/* Waits for running requests, drops queued ones, frees everything. */
int tng_server_destroy(tng_server* srv);

/* Sum the copies of every duplicate group of a node field and write the sum
 * to all copies (the one-GPU analog of the post-apply halo sum, Sec. 2); with
 * mode 1 instead copy the first copy to all others.  ncomp fields in f[]. */
int tng_interface_sum(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec,
                      int mode, int ncomp, void* const f[]);

#ifdef __cplusplus
}
#endif

#endif /* TNG_H */
