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
 * Memory: "device" pointers must be device memory of the context's GPU (e.g.
 *   torch CUDA tensors); "host" pointers are ordinary host memory.
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
    TNG_OP_DIRICHLET = 8 /* zero-velocity rows on both spheres: identity rows,
                            columns dropped (K_D = [[DAD + I - D, DB^T],[BD, 0]]) */
};

/* Message of the last failed call on this thread ("" if none).  Library-owned. */
const char* tng_last_error(void);

/* ---- context ----------------------------------------------------------- */
/* device: HIP device ordinal.  hip_stream: a hipStream_t owned by the caller
 * (may be NULL for the null stream); the library enqueues all work on it. */
int tng_ctx_create(int device, void* hip_stream, tng_ctx** out);
int tng_ctx_set_stream(tng_ctx* ctx, void* hip_stream);
int tng_ctx_destroy(tng_ctx* ctx);
/* Measurement: with enable != 0, every call records a HIP event pair on the
 * context stream around its main kernel (kernel names: "stokes_apply").
 * tng_ctx_kernel_stats synchronises on the recorded events and returns the
 * summed elapsed milliseconds and the number of launches since profiling was
 * (re)enabled; an unknown name gives 0 and 0. */
int tng_ctx_profile(tng_ctx* ctx, int enable);
int tng_ctx_kernel_stats(tng_ctx* ctx, const char* name, double* total_ms, long long* launches);

/* ---- mesh (Sec. 2, a1) -------------------------------------------------- */
/* Builds the shell with mt lateral intervals per diamond edge (power of two)
 * and nr radial intervals on [r_in, r_out], and uploads `levels` levels to the
 * context's device.  ctx may be NULL: then only the host-side description is
 * built (counts, coordinates, duplicate groups) and the mesh cannot be used by
 * device calls, which reject it with TNG_E_INVAL.  Levels:
 * (level l = (mt/2^l, nr/2^l); both must stay integers >= 1).  The pressure of
 * level l lives on level l + 1, so an operator on level l needs l + 1 < levels. */
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

/* ---- operator (Sec. 3 eq:matfree, eq:epsq, eq:localapply; a3-a5) -------- */
/* y = K(eta) x restricted to the blocks in op_flags, on level `level`.
 * eta_wedge: device wedge field of level `level`.  u[3]: device velocity in;
 * p: device pressure (level + 1) in, may be NULL unless TNG_OP_BT is set.
 * y_u[3]: device velocity out (required if TNG_OP_A or TNG_OP_BT);
 * y_p: device pressure out (required if TNG_OP_B).  Outputs are overwritten
 * (not accumulated) and are assembled: every copy of a duplicate node holds
 * the full sum.  With TNG_OP_DIRICHLET the velocity input is read as zero on
 * both spheres and y_u = u there.  Inputs and outputs must not alias. */
int tng_stokes_apply(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec,
                     unsigned op_flags, const void* eta_wedge,
                     const void* const u[3], const void* p,
                     void* const y_u[3], void* y_p);

/* ---- fields (a2) -------------------------------------------------------- */
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

/* Sum the copies of every duplicate group of a node field and write the sum
 * to all copies (the one-GPU analog of the post-apply halo sum, Sec. 2); with
 * mode 1 instead copy the first copy to all others.  ncomp fields in f[]. */
int tng_interface_sum(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec,
                      int mode, int ncomp, void* const f[]);

#ifdef __cplusplus
}
#endif

#endif /* TNG_H */
