// Atomic-free streaming kernel for the Stokes apply y = K(eta) [u; p].
//
// Work decomposition (one diamond d, a "band"):
//   * lanes run along the radial direction: lane l of a wave handles the CPL
//     consecutive cells k = k0 + CPL*l + c of one cell column, so every memory
//     access of a wave covers a contiguous radial stretch;
//   * the TI waves of a workgroup handle TI adjacent cell columns i0..i0+TI-1;
//   * the workgroup streams along j over the cell rows of its band, carrying
//     the half-finished node row in registers, so each node of the band's
//     interior is written exactly once, with its complete sum.
// Contributions that cross a wave boundary are combined in LDS (lateral, i
// direction) or with lane shuffles (radial).  A band starts one cell row
// early (the halo row) so that its first node row is complete; nodes on the
// seams between tiles (node columns that are multiples of TI) and between
// radial chunks receive exactly two partial sums, added with atomics to
// memory zeroed beforehand, which keeps the result independent of timing.
//
// The divergence block is accumulated per coarse pressure node in LDS over
// the band and flushed with atomics once a coarse row is complete.
#include "tng_internal.hpp"
#include "wedge.hpp"

namespace tng {
namespace {

__constant__ IsoWeights c_isob = make_iso_weights();
constexpr int TI_MAX = 8;   // cell columns (waves) per workgroup

template <typename T>
struct BandArgs {
    const T* __restrict__ eta;
    const T* __restrict__ u0;
    const T* __restrict__ u1;
    const T* __restrict__ u2;
    const T* __restrict__ p;
    T* y0;
    T* y1;
    T* y2;
    T* yp;
    const T* __restrict__ geo;
    int m, n;
    int TI, TJ, KC;
    int ntile, nband, nchunk;
    T r_in, dr;
    int dirichlet;
};

template <typename T>
__device__ __forceinline__ T shfl_up1(T v, int lane) {
    return __shfl(v, (lane + 63) & 63, 64);
}

// Emit one node value: plain store when this workgroup holds its complete
// sum, atomic add (onto zeroed memory) on tile or chunk seams.
template <typename T>
__device__ __forceinline__ void emit(T* y, long long idx, T v, bool seam) {
    if (seam)
        atomicAdd(y + idx, v);
    else
        y[idx] = v;
}

template <typename T, int CPL, bool DO_A, bool DO_BT, bool DO_B>
__global__ void __launch_bounds__(TI_MAX * 64) stokes_band_kernel(BandArgs<T> a) {
    constexpr int NL = CPL + 1;   // node layers per lane: bottom of each cell + top partial
    constexpr bool DO_U = DO_A || DO_BT;
    constexpr int XW = DO_U ? TI_MAX : 1;
    __shared__ T xch[2][XW][3][NL][64];
    constexpr int PB_I = DO_B ? TI_MAX / 2 + 1 : 1;
    constexpr int PB_K = DO_B ? 32 * CPL + 2 : 1;
    __shared__ T pbuf[2][PB_I][PB_K];

    const int TI = a.TI;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int bid = blockIdx.x;
    const int chunk = bid % a.nchunk;
    bid /= a.nchunk;
    const int band = bid % a.nband;
    bid /= a.nband;
    const int tile = bid % a.ntile;
    const int d = bid / a.ntile;

    const int m = a.m, n = a.n;
    const int i0 = tile * TI;
    const int i = i0 + w;
    const int j0 = band * a.TJ;
    const bool last_band = (band == a.nband - 1);
    const int jfirst = j0 > 0 ? j0 - 1 : 0;            // halo row (computed, not owned)
    const int jlast_cell = last_band ? m - 1 : j0 + a.TJ - 1;
    const int jlast = last_band ? m : jlast_cell;      // last node row emitted
    const int k0 = chunk * a.KC;
    const int kend = min(n, k0 + a.KC);                // cells [k0, kend) of this chunk

    const long long ldj = n + 1;
    const long long ldi = (long long)(m + 1) * ldj;
    const long long colA = (long long)d * (m + 1) * ldi + (long long)i * ldi;   // node column i
    const long long colB = colA + ldi;                                           // node column i + 1

    int kk[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) kk[c] = k0 + CPL * lane + c;
    bool cell_ok[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) cell_ok[c] = kk[c] < kend;
    // the lane holding the chunk's last cell also owns the node layer above it
    const bool top_lane = (kk[0] <= kend - 1) && (kend - 1 <= kk[CPL - 1]);
    const int top_c = kend - kk[0];

    // velocity of node rows: column i (uA/uC) and i+1 (uB/uD); Dirichlet layers read as zero
    T uA[NL][3], uB[NL][3];
    auto load_u = [&](long long col, int jrow, T (&dst)[NL][3]) {
        const long long base = col + (long long)jrow * ldj;
#pragma unroll
        for (int c = 0; c < NL; ++c) {
            const int k = kk[c];
            const bool ok = (DO_A || DO_B) && k <= n && !(a.dirichlet && (k == 0 || k == n));
            dst[c][0] = ok ? a.u0[base + k] : T(0);
            dst[c][1] = ok ? a.u1[base + k] : T(0);
            dst[c][2] = ok ? a.u2[base + k] : T(0);
        }
    };

    // rolling partial sums of node row j+1 (R0: column i, R1: column i+1)
    T R0[NL][3], R1[NL][3];
#pragma unroll
    for (int c = 0; c < NL; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) R0[c][r] = R1[c][r] = T(0);

    if (DO_B)
        for (int t = threadIdx.x; t < 2 * PB_I * PB_K; t += TI * 64) (&pbuf[0][0][0])[t] = T(0);
    load_u(colA, jfirst, uA);
    load_u(colB, jfirst, uB);

    const int mc = m / 2, nc = n / 2;
    const long long pldj = nc + 1;
    const long long pldi = (long long)(mc + 1) * pldj;
    const long long pcol = (long long)d * (mc + 1) * pldi;
    const int I = i >> 1, I0 = i0 >> 1;
    const int ab = i & 1;
    const int K0 = k0 >> 1;

    __syncthreads();

    for (int j = jfirst; j <= jlast; ++j) {
        const bool row_cells = j <= jlast_cell;    // the extra last step only emits
        const bool owned = j >= j0;
        const int par = j & 1;
        const int J = j >> 1, bb = j & 1;
        T Nd[4][NL][3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) Nd[q][c][r] = T(0);
        T uC[NL][3], uD[NL][3];
        if (row_cells) {
            load_u(colA, j + 1, uC);
            load_u(colB, j + 1, uD);
            const T* g = a.geo + (((long long)d * m + i) * m + j) * GEO_PER_COL;
            const long long ecol = ((((long long)d * m + i) * m + j) * n) * 2;
            long long pb[4];
            pb[0] = pcol + (long long)I * pldi + (long long)J * pldj;
            pb[1] = pb[0] + pldi;
            pb[2] = pb[0] + pldj;
            pb[3] = pb[0] + pldi + pldj;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                if (!cell_ok[c]) continue;
                const int k = kk[c];
                const T rm = a.r_in + (T(k) + T(0.5)) * a.dr;
                const T s1 = T(0.5) / rm;
                const T rm2 = rm * rm;
                const int K = k >> 1, cb = k & 1;
                const T rw0 = T(c_isob.rw[cb][0]), rw1 = T(c_isob.rw[cb][1]);
                T pc[4] = {0, 0, 0, 0};
                if (DO_BT) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) pc[q] = rw0 * a.p[pb[q] + K] + rw1 * a.p[pb[q] + K + 1];
                }
                T tB[4] = {0, 0, 0, 0};
#pragma unroll
                for (int wd = 0; wd < 2; ++wd) {
                    // wedge 0: corners (i,j),(i+1,j),(i,j+1); wedge 1: (i+1,j+1),(i,j+1),(i+1,j)
                    T uw[6][3];
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        if (wd == 0) {
                            uw[0][r] = uA[c][r]; uw[1][r] = uB[c][r]; uw[2][r] = uC[c][r];
                            uw[3][r] = uA[c + 1][r]; uw[4][r] = uB[c + 1][r]; uw[5][r] = uC[c + 1][r];
                        } else {
                            uw[0][r] = uD[c][r]; uw[1][r] = uC[c][r]; uw[2][r] = uB[c][r];
                            uw[3][r] = uD[c + 1][r]; uw[4][r] = uC[c + 1][r]; uw[5][r] = uB[c + 1][r];
                        }
                    }
                    T pbar = 0;
                    if (DO_BT) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) pbar += T(c_isob.lw[ab][bb][wd][q]) * pc[q];
                    }
                    const T eta = DO_A ? a.eta[ecol + 2 * k + wd] : T(0);
                    WedgeOut<T> o;
                    wedge_apply<T, DO_A, DO_BT, DO_B>(uw, g + wd * GEO_PER_TRI, s1, rm2, eta, pbar, o);
                    if (DO_U) {
                        // cell corner of each wedge node: 0=(i,j) 1=(i+1,j) 2=(i,j+1) 3=(i+1,j+1)
                        constexpr int cq[2][3] = {{0, 1, 2}, {3, 2, 1}};
#pragma unroll
                        for (int jn = 0; jn < 3; ++jn)
#pragma unroll
                            for (int r = 0; r < 3; ++r) {
                                Nd[cq[wd][jn]][c][r] += o.y[jn][r];
                                Nd[cq[wd][jn]][c + 1][r] += o.y[jn + 3][r];
                            }
                    }
                    if (DO_B) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) tB[q] += T(c_isob.lw[ab][bb][wd][q]) * o.dv;
                    }
                }
                if (DO_B && owned) {
                    // coarse corner q = (I + (q&1), J + (q>>1)), layers K and K+1
                    const int Kl = K - K0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        T* cell = &pbuf[(J + (q >> 1)) & 1][(I - I0) + (q & 1)][Kl];
                        atomicAdd(cell, rw0 * tB[q]);
                        atomicAdd(cell + 1, rw1 * tB[q]);
                    }
                }
            }
        }
        if (DO_U) {
            // radial: the top partial of the lane below completes this lane's bottom node
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const T t = shfl_up1(Nd[q][CPL][r], lane);
                    if (lane > 0) Nd[q][0][r] += t;
                }
            // lateral: this wave's partial of node (i+1, j) goes to the wave on its right
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) xch[par][w][r][c][lane] = R1[c][r] + Nd[1][c][r];
        }
        __syncthreads();
        if (DO_U && owned) {
            const long long rowA = colA + (long long)j * ldj;
            const long long rowB = colB + (long long)j * ldj;
            const bool seamL = (w == 0) && (i0 > 0);
            const bool right = (w == TI - 1);
            const bool seamR = (i0 + TI < m);
#pragma unroll
            for (int c = 0; c < NL; ++c) {
                const int k = kk[c];
                bool live = false, seamK = false;
                if (top_lane && c == top_c) {
                    live = true;
                    seamK = kend < n;                   // chunk top: the next chunk adds the rest
                } else if (c < CPL && cell_ok[c]) {
                    live = true;
                    seamK = (c == 0 && lane == 0 && k0 > 0);   // chunk bottom
                }
                if (a.dirichlet && (k == 0 || k == n)) live = false;   // rows set to u afterwards
                if (!live) continue;
                T v[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    v[r] = R0[c][r] + Nd[0][c][r];
                    if (w > 0) v[r] += xch[par][w - 1][r][c][lane];
                }
                const bool seam = seamL || seamK;
                emit(a.y0, rowA + k, v[0], seam);
                emit(a.y1, rowA + k, v[1], seam);
                emit(a.y2, rowA + k, v[2], seam);
                if (right) {
                    // node column i0 + TI: complete only on the diamond edge
                    const bool s2 = seamR || seamK;
                    emit(a.y0, rowB + k, xch[par][w][0][c][lane], s2);
                    emit(a.y1, rowB + k, xch[par][w][1][c][lane], s2);
                    emit(a.y2, rowB + k, xch[par][w][2][c][lane], s2);
                }
            }
        }
        if (DO_U) {
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    R0[c][r] = Nd[2][c][r];
                    R1[c][r] = Nd[3][c][r];
                }
        }
        if (DO_B && owned && row_cells && (j & 1)) {
            // coarse node row J has received all of this band's cells: flush it
            T* prow = &pbuf[J & 1][0][0];
            for (int t = threadIdx.x; t < PB_I * PB_K; t += TI * 64) {
                const int il = t / PB_K, kl = t % PB_K;
                const int Ig = I0 + il, Kg = K0 + kl;
                const T v = prow[t];
                if (il <= TI / 2 && Ig <= mc && Kg <= nc && v != T(0))
                    atomicAdd(a.yp + pcol + (long long)Ig * pldi + (long long)J * pldj + Kg, v);
                prow[t] = T(0);
            }
            __syncthreads();
        }
        if (row_cells) {
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    uA[c][r] = uC[c][r];
                    uB[c][r] = uD[c][r];
                }
        }
    }
    if (DO_B) {
        // the coarse row above the band's last cell row is still pending
        __syncthreads();
        const int J = (jlast_cell >> 1) + 1;
        T* prow = &pbuf[J & 1][0][0];
        for (int t = threadIdx.x; t < PB_I * PB_K; t += TI * 64) {
            const int il = t / PB_K, kl = t % PB_K;
            const int Ig = I0 + il, Kg = K0 + kl;
            const T v = prow[t];
            if (il <= TI / 2 && Ig <= mc && Kg <= nc && v != T(0))
                atomicAdd(a.yp + pcol + (long long)Ig * pldi + (long long)J * pldj + Kg, v);
        }
    }
}

// Zero the node values that receive two partial sums: node columns on tile
// seams and node layers on radial-chunk seams.
template <typename T>
__global__ void zero_seams_kernel(T* y0, T* y1, T* y2, int m, int n, int TI, int KC, int nchunk) {
    const int nseam_i = m / TI - 1;
    const long long ncol = (long long)10 * nseam_i * (m + 1);       // seam columns x rows
    const long long n1 = n + 1;
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long ldi = (long long)(m + 1) * n1;
    if (t < ncol * n1) {
        const int k = (int)(t % n1);
        long long r = t / n1;
        const int jrow = (int)(r % (m + 1));
        r /= (m + 1);
        const int s = (int)(r % nseam_i);
        const int d = (int)(r / nseam_i);
        const long long idx = ((long long)d * (m + 1) + (long long)(s + 1) * TI) * ldi + (long long)jrow * n1 + k;
        y0[idx] = T(0);
        y1[idx] = T(0);
        y2[idx] = T(0);
        return;
    }
    t -= ncol * n1;
    const long long nlat = (long long)10 * (m + 1) * (m + 1);
    if (t < nlat * (nchunk - 1)) {
        const long long slot = t % nlat;
        const int c = (int)(t / nlat) + 1;
        const long long idx = slot * n1 + (long long)c * KC;
        y0[idx] = T(0);
        y1[idx] = T(0);
        y2[idx] = T(0);
    }
}

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, int CPL, bool A, bool BT, bool B>
void launch_band_t(const tng_ctx* ctx, const BandArgs<T>& args) {
    const long long nb = 10LL * args.ntile * args.nband * args.nchunk;
    ScopedKernelTimer timer(ctx, "stokes_apply");
    stokes_band_kernel<T, CPL, A, BT, B><<<(unsigned)nb, args.TI * 64, 0, ctx->stream>>>(args);
    TNG_HIP(hipGetLastError());
}

template <typename T, int CPL>
void launch_band_ops(const tng_ctx* ctx, const BandArgs<T>& args, int key) {
    switch (key) {
        case 1: launch_band_t<T, CPL, true, false, false>(ctx, args); break;
        case 2: launch_band_t<T, CPL, false, true, false>(ctx, args); break;
        case 3: launch_band_t<T, CPL, true, true, false>(ctx, args); break;
        case 4: launch_band_t<T, CPL, false, false, true>(ctx, args); break;
        case 5: launch_band_t<T, CPL, true, false, true>(ctx, args); break;
        case 6: launch_band_t<T, CPL, false, true, true>(ctx, args); break;
        case 7: launch_band_t<T, CPL, true, true, true>(ctx, args); break;
        default: throw Error(TNG_E_INVAL, "op_flags selects no operator block");
    }
}

template <typename T>
__global__ void fill0_kernel(T* __restrict__ a, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (; i < n; i += stride) a[i] = T(0);
}

template <typename T>
void band_apply(const tng_ctx* ctx, const Level& L, const Level* Lp, unsigned flags,
                const void* eta, const void* const u[3], const void* p, void* const yu[3],
                void* yp) {
    const bool doA = flags & TNG_OP_A, doBT = flags & TNG_OP_BT, doB = flags & TNG_OP_B;
    const bool is64 = std::is_same<T, double>::value;
    BandArgs<T> a{};
    a.eta = static_cast<const T*>(eta);
    a.u0 = u ? static_cast<const T*>(u[0]) : nullptr;
    a.u1 = u ? static_cast<const T*>(u[1]) : nullptr;
    a.u2 = u ? static_cast<const T*>(u[2]) : nullptr;
    a.p = static_cast<const T*>(p);
    a.y0 = yu ? static_cast<T*>(yu[0]) : nullptr;
    a.y1 = yu ? static_cast<T*>(yu[1]) : nullptr;
    a.y2 = yu ? static_cast<T*>(yu[2]) : nullptr;
    a.yp = static_cast<T*>(yp);
    a.geo = is64 ? reinterpret_cast<const T*>(L.geo64.p) : reinterpret_cast<const T*>(L.geo32.p);
    a.m = L.m;
    a.n = L.n;
    a.TI = std::min(TI_MAX, L.m);
    a.TJ = std::min(16, L.m);
    // cells per lane: enough for the whole radial column within the register
    // budget (two or more FP64 cells per lane spill), longer columns are split
    // into radial chunks
    int cpl = (L.n + 63) / 64;
    const int cpl_max = is64 ? 1 : 4;
    cpl = cpl <= 1 ? 1 : (cpl <= 2 ? 2 : 4);
    if (cpl > cpl_max) cpl = cpl_max;
    a.KC = 64 * cpl;
    a.ntile = L.m / a.TI;
    a.nband = L.m / a.TJ;
    a.nchunk = (L.n + a.KC - 1) / a.KC;
    a.r_in = T(L.r_in);
    a.dr = T(L.dr());
    a.dirichlet = (flags & TNG_OP_DIRICHLET) ? 1 : 0;
    if (doB) {
        const long long np = Lp->node_slots();
        fill0_kernel<T><<<std::min<long long>(nblocks(np, 256), 4096), 256, 0, ctx->stream>>>(a.yp, np);
        TNG_HIP(hipGetLastError());
    }
    if ((doA || doBT) && (a.ntile > 1 || a.nchunk > 1)) {
        const long long nz = 10LL * (a.ntile - 1) * (L.m + 1) * (L.n + 1) +
                             10LL * (L.m + 1) * (L.m + 1) * (a.nchunk - 1);
        if (nz > 0) {
            zero_seams_kernel<T><<<nblocks(nz, 256), 256, 0, ctx->stream>>>(
                a.y0, a.y1, a.y2, L.m, L.n, a.TI, a.KC, a.nchunk);
            TNG_HIP(hipGetLastError());
        }
    }
    const int key = (doA ? 1 : 0) | (doBT ? 2 : 0) | (doB ? 4 : 0);
    if constexpr (std::is_same<T, double>::value) {
        launch_band_ops<T, 1>(ctx, a, key);
    } else {
        if (cpl == 1)
            launch_band_ops<T, 1>(ctx, a, key);
        else if (cpl == 2)
            launch_band_ops<T, 2>(ctx, a, key);
        else
            launch_band_ops<T, 4>(ctx, a, key);
    }
    const tng_prec prec = is64 ? TNG_F64 : TNG_F32;
    if (doA || doBT) {
        void* f[3] = {yu[0], yu[1], yu[2]};
        launch_interface(ctx, L, prec, 0, 3, f);
        // identity rows belong to the viscous block; without it the rows are zero
        if (a.dirichlet) launch_dirichlet_copy(ctx, L, prec, doA ? u : nullptr, yu);
    }
    if (doB) {
        void* f[1] = {yp};
        launch_interface(ctx, *Lp, prec, 0, 1, f);
    }
}

}  // namespace

void launch_stokes_apply(const tng_ctx* ctx, const Level& L, const Level* Lp, tng_prec prec,
                         unsigned flags, const void* eta, const void* const u[3], const void* p,
                         void* const yu[3], void* yp) {
    if (prec == TNG_F64)
        band_apply<double>(ctx, L, Lp, flags, eta, u, p, yu, yp);
    else
        band_apply<float>(ctx, L, Lp, flags, eta, u, p, yu, yp);
}

}  // namespace tng
