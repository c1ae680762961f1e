// Matrix-free Stokes operator apply y = K(eta) [u; p] (Sec. 3 eq:matfree).
//
// One thread per hexahedral cell, radial index fastest so that a wavefront
// reads 64 consecutive layers of a cell column.  Each thread gathers the 8
// nodes of its cell, evaluates both wedges at their quadrature point
// (wedge.hpp) and adds the element results into the node field with atomics,
// as the paper's textbook kernel does (Sec. 5); the diamond-interface kernel
// then sums the copies of shared nodes.
#include "tng_internal.hpp"
#include "wedge.hpp"

namespace tng {
namespace {

__constant__ IsoWeights c_iso = make_iso_weights();

template <typename T>
struct ApplyArgs {
    const T* __restrict__ eta;
    const T* __restrict__ u[3];
    const T* __restrict__ p;
    T* y[3];
    T* yp;
    const T* __restrict__ geo;
    int m, n;          // fine level
    T r_in, dr;
    int dirichlet;
    long long ncells;
};

template <typename T>
__global__ void fill_kernel(T* __restrict__ a, long long n, T v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = v;
}

template <typename T, bool DO_A, bool DO_BT, bool DO_B>
__global__ void __launch_bounds__(256) stokes_cell_atomic(ApplyArgs<T> a) {
    const long long cid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cid >= a.ncells) return;
    const int m = a.m, n = a.n;
    const int k = (int)(cid % n);
    long long t = cid / n;
    const int j = (int)(t % m);
    t /= m;
    const int i = (int)(t % m);
    const int d = (int)(t / m);

    const long long ldj = n + 1;
    const long long ldi = (long long)(m + 1) * ldj;
    const long long ldd = (long long)(m + 1) * ldi;
    // lateral corners q = di + 2 dj of the cell
    long long base[4];
    base[0] = d * ldd + i * ldi + j * ldj;
    base[1] = base[0] + ldi;
    base[2] = base[0] + ldj;
    base[3] = base[0] + ldi + ldj;

    T uc[4][2][3];
    const bool zb = a.dirichlet && k == 0;
    const bool zt = a.dirichlet && k + 1 == n;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            uc[q][0][c] = (DO_A || DO_B) && !zb ? a.u[c][base[q] + k] : T(0);
            uc[q][1][c] = (DO_A || DO_B) && !zt ? a.u[c][base[q] + k + 1] : T(0);
        }

    const T rm = a.r_in + (T(k) + T(0.5)) * a.dr;
    const T s1 = T(0.5) / rm;
    const T rm2 = rm * rm;
    const T* g = a.geo + (((long long)d * m + i) * m + j) * GEO_PER_COL;
    const long long wid = cid * 2;

    // coarse pressure corners (radially interpolated to this fine layer)
    const int mc = m / 2, nc = n / 2;
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const int ab = i & 1, bb = j & 1, cb = k & 1;
    const long long pldj = nc + 1;
    const long long pldi = (long long)(mc + 1) * pldj;
    const long long pldd = (long long)(mc + 1) * pldi;
    long long pbase[4];
    pbase[0] = d * pldd + I * pldi + J * pldj + K;
    pbase[1] = pbase[0] + pldi;
    pbase[2] = pbase[0] + pldj;
    pbase[3] = pbase[0] + pldi + pldj;
    const T rw0 = T(c_iso.rw[cb][0]), rw1 = T(c_iso.rw[cb][1]);
    T pc[4] = {0, 0, 0, 0};
    if (DO_BT) {
#pragma unroll
        for (int q = 0; q < 4; ++q) pc[q] = rw0 * a.p[pbase[q]] + rw1 * a.p[pbase[q] + 1];
    }

    const int lat[2][3] = {{0, 1, 2}, {3, 2, 1}};
    T tB[4] = {0, 0, 0, 0};
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        T uw[6][3];
#pragma unroll
        for (int jn = 0; jn < 3; ++jn)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                uw[jn][c] = uc[lat[w][jn]][0][c];
                uw[jn + 3][c] = uc[lat[w][jn]][1][c];
            }
        T pbar = 0;
        if (DO_BT) {
#pragma unroll
            for (int q = 0; q < 4; ++q) pbar += T(c_iso.lw[ab][bb][w][q]) * pc[q];
        }
        const T eta = DO_A ? a.eta[wid + w] : T(0);
        WedgeOut<T> o;
        wedge_apply<T, DO_A, DO_BT, DO_B>(uw, g + w * GEO_PER_TRI, s1, rm2, eta, pbar, o);
        if (DO_A || DO_BT) {
#pragma unroll
            for (int jn = 0; jn < 3; ++jn) {
                const long long nb = base[lat[w][jn]];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (!zb) atomicAdd(&a.y[c][nb + k], o.y[jn][c]);
                    if (!zt) atomicAdd(&a.y[c][nb + k + 1], o.y[jn + 3][c]);
                }
            }
        }
        if (DO_B) {
#pragma unroll
            for (int q = 0; q < 4; ++q) tB[q] += T(c_iso.lw[ab][bb][w][q]) * o.dv;
        }
    }
    if (DO_B) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            atomicAdd(&a.yp[pbase[q]], rw0 * tB[q]);
            atomicAdd(&a.yp[pbase[q] + 1], rw1 * tB[q]);
        }
    }
}

template <typename T>
__global__ void interface_kernel(int ngroups, int n1, const int* __restrict__ gptr,
                                 const int* __restrict__ gslot, int mode, int ncomp, T* f0, T* f1,
                                 T* f2, T* f3) {
    long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long long)ngroups * n1) return;
    const int gidx = (int)(tid / n1);
    const int k = (int)(tid % n1);
    const int s0 = gptr[gidx], s1 = gptr[gidx + 1];
    T* fs[4] = {f0, f1, f2, f3};
    for (int c = 0; c < ncomp; ++c) {
        T* f = fs[c];
        T acc = f[(long long)gslot[s0] * n1 + k];
        if (mode == 0)
            for (int s = s0 + 1; s < s1; ++s) acc += f[(long long)gslot[s] * n1 + k];
        for (int s = s0; s < s1; ++s) f[(long long)gslot[s] * n1 + k] = acc;
    }
}

template <typename T>
__global__ void dirichlet_copy_kernel(long long ncol, int n, const T* __restrict__ u0,
                                      const T* __restrict__ u1, const T* __restrict__ u2, T* y0,
                                      T* y1, T* y2) {
    long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 2 * ncol) return;
    const long long col = tid >> 1;
    const long long idx = col * (n + 1) + ((tid & 1) ? n : 0);
    y0[idx] = u0[idx];
    y1[idx] = u1[idx];
    y2[idx] = u2[idx];
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T>
void fill(const tng_ctx* ctx, T* a, long long n) {
    if (n <= 0) return;
    long long nb = std::min<long long>(blocks_for(n, 256), 65536);
    fill_kernel<T><<<(unsigned)nb, 256, 0, ctx->stream>>>(a, n, T(0));
    TNG_HIP(hipGetLastError());
}

template <typename T, bool A, bool BT, bool B>
void launch_cells(const tng_ctx* ctx, const ApplyArgs<T>& args) {
    ScopedKernelTimer timer(ctx, "stokes_apply");
    stokes_cell_atomic<T, A, BT, B><<<blocks_for(args.ncells, 256), 256, 0, ctx->stream>>>(args);
    TNG_HIP(hipGetLastError());
}

template <typename T>
void apply_typed(const tng_ctx* ctx, const Level& L, const Level* Lp, unsigned flags,
                 const void* eta, const void* const u[3], const void* p, void* const yu[3],
                 void* yp) {
    const bool doA = flags & TNG_OP_A, doBT = flags & TNG_OP_BT, doB = flags & TNG_OP_B;
    ApplyArgs<T> a{};
    a.eta = static_cast<const T*>(eta);
    for (int c = 0; c < 3; ++c) {
        a.u[c] = u ? static_cast<const T*>(u[c]) : nullptr;
        a.y[c] = yu ? static_cast<T*>(yu[c]) : nullptr;
    }
    a.p = static_cast<const T*>(p);
    a.yp = static_cast<T*>(yp);
    a.geo = std::is_same<T, double>::value ? reinterpret_cast<const T*>(L.geo64.p)
                                           : reinterpret_cast<const T*>(L.geo32.p);
    a.m = L.m;
    a.n = L.n;
    a.r_in = T(L.r_in);
    a.dr = T(L.dr());
    a.dirichlet = (flags & TNG_OP_DIRICHLET) ? 1 : 0;
    a.ncells = L.cells();
    if (doA || doBT)
        for (int c = 0; c < 3; ++c) fill<T>(ctx, a.y[c], L.node_slots());
    if (doB) fill<T>(ctx, a.yp, Lp->node_slots());
    const int key = (doA ? 1 : 0) | (doBT ? 2 : 0) | (doB ? 4 : 0);
    switch (key) {
        case 1: launch_cells<T, true, false, false>(ctx, a); break;
        case 2: launch_cells<T, false, true, false>(ctx, a); break;
        case 3: launch_cells<T, true, true, false>(ctx, a); break;
        case 4: launch_cells<T, false, false, true>(ctx, a); break;
        case 5: launch_cells<T, true, false, true>(ctx, a); break;
        case 6: launch_cells<T, false, true, true>(ctx, a); break;
        case 7: launch_cells<T, true, true, true>(ctx, a); break;
        default: throw Error(TNG_E_INVAL, "op_flags selects no operator block");
    }
    if (doA || doBT) {
        void* f[3] = {yu[0], yu[1], yu[2]};
        launch_interface(ctx, L, std::is_same<T, double>::value ? TNG_F64 : TNG_F32, 0, 3, f);
        // the identity rows of K_D belong to the viscous block
        if (a.dirichlet && doA)
            launch_dirichlet_copy(ctx, L, std::is_same<T, double>::value ? TNG_F64 : TNG_F32, u, yu);
    }
    if (doB) {
        void* f[1] = {yp};
        launch_interface(ctx, *Lp, std::is_same<T, double>::value ? TNG_F64 : TNG_F32, 0, 1, f);
    }
}

}  // namespace

void launch_stokes_apply(const tng_ctx* ctx, const Level& L, const Level* Lp, tng_prec prec,
                         unsigned flags, const void* eta, const void* const u[3], const void* p,
                         void* const yu[3], void* yp) {
    if (prec == TNG_F64)
        apply_typed<double>(ctx, L, Lp, flags, eta, u, p, yu, yp);
    else
        apply_typed<float>(ctx, L, Lp, flags, eta, u, p, yu, yp);
}

void launch_interface(const tng_ctx* ctx, const Level& L, tng_prec prec, int mode, int ncomp,
                      void* const f[]) {
    TNG_REQUIRE(ncomp >= 1 && ncomp <= 4, "ncomp must be 1..4");
    if (L.n_groups == 0) return;
    const long long nt = (long long)L.n_groups * (L.n + 1);
    void* g[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int c = 0; c < ncomp; ++c) g[c] = f[c];
    if (prec == TNG_F64)
        interface_kernel<double><<<blocks_for(nt, 256), 256, 0, ctx->stream>>>(
            L.n_groups, L.n + 1, L.grp_ptr.p, L.grp_slot.p, mode, ncomp, (double*)g[0],
            (double*)g[1], (double*)g[2], (double*)g[3]);
    else
        interface_kernel<float><<<blocks_for(nt, 256), 256, 0, ctx->stream>>>(
            L.n_groups, L.n + 1, L.grp_ptr.p, L.grp_slot.p, mode, ncomp, (float*)g[0],
            (float*)g[1], (float*)g[2], (float*)g[3]);
    TNG_HIP(hipGetLastError());
}

void launch_dirichlet_copy(const tng_ctx* ctx, const Level& L, tng_prec prec,
                           const void* const u[3], void* const y[3]) {
    const long long ncol = L.lat_slots();
    if (prec == TNG_F64)
        dirichlet_copy_kernel<double><<<blocks_for(2 * ncol, 256), 256, 0, ctx->stream>>>(
            ncol, L.n, (const double*)u[0], (const double*)u[1], (const double*)u[2],
            (double*)y[0], (double*)y[1], (double*)y[2]);
    else
        dirichlet_copy_kernel<float><<<blocks_for(2 * ncol, 256), 256, 0, ctx->stream>>>(
            ncol, L.n, (const float*)u[0], (const float*)u[1], (const float*)u[2], (float*)y[0],
            (float*)y[1], (float*)y[2]);
    TNG_HIP(hipGetLastError());
}

}  // namespace tng
