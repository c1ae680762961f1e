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
__device__ __forceinline__ void emit(T* y, unsigned idx, T v, bool seam) {
    if (seam)
        atomicAdd(y + idx, v);
    else
        y[idx] = v;
}

template <typename T>
struct IsoTable;
template <>
struct IsoTable<float> {
    __device__ static const IsoWeights<float>& get();
};
template <>
struct IsoTable<double> {
    __device__ static const IsoWeights<double>& get();
};
__constant__ IsoWeights<float> c_iso32 = make_iso_weights<float>();
__constant__ IsoWeights<double> c_iso64 = make_iso_weights<double>();
__device__ const IsoWeights<float>& IsoTable<float>::get() { return c_iso32; }
__device__ const IsoWeights<double>& IsoTable<double>::get() { return c_iso64; }

// Coarse-layer slots of the divergence reduction: a lane's cells touch NKL
// consecutive coarse layers starting at layer kb(lane).
template <int CPL>
struct CoarseMap {
    static constexpr int NKL = CPL == 1 ? 2 : CPL / 2 + 1;
};

template <typename T, int CPL, bool DO_A, bool DO_BT, bool DO_B>
__global__ void __launch_bounds__(TI_MAX * 64) stokes_band_kernel(BandArgs<T> a) {
    constexpr int NL = CPL + 1;   // node layers per lane: bottom of each cell + top partial
    constexpr bool DO_U = DO_A || DO_BT;
    constexpr bool LOAD_U = DO_A || DO_B;
    constexpr int XW = DO_U ? TI_MAX : 1;
    __shared__ T xch[2][XW][3][NL][64];
    constexpr int NKC = DO_B ? 32 * CPL + 1 : 1;          // coarse layers per chunk
    constexpr int BW = DO_B ? TI_MAX : 1;
    __shared__ T bsl[2][BW][4][NKC];                      // per-wave coarse partials
    constexpr int NKL = CoarseMap<CPL>::NKL;
    const IsoWeights<T>& iso = IsoTable<T>::get();

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

    // 32-bit offsets: every field of a supported level has < 2^31 entries
    const unsigned ldj = n + 1;
    const unsigned ldi = (unsigned)(m + 1) * ldj;
    const unsigned colA = ((unsigned)d * (m + 1) + i) * ldi;   // node column i
    const unsigned colB = colA + ldi;                          // node column i + 1

    int kk[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) kk[c] = k0 + CPL * lane + c;
    bool cell_ok[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) cell_ok[c] = kk[c] < kend;
    const bool top_lane = (kk[0] <= kend - 1) && (kend - 1 <= kk[CPL - 1]);
    const int top_c = kend - kk[0];
    bool node_ok[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c)
        node_ok[c] = LOAD_U && kk[c] <= n && !(a.dirichlet && (kk[c] == 0 || kk[c] == n));

    auto load_u = [&](unsigned col, int jrow, T (&dst)[NL][3]) {
        const unsigned base = col + (unsigned)jrow * ldj;
#pragma unroll
        for (int c = 0; c < NL; ++c) {
            const unsigned o = base + (unsigned)kk[c];
            dst[c][0] = node_ok[c] ? a.u0[o] : T(0);
            dst[c][1] = node_ok[c] ? a.u1[o] : T(0);
            dst[c][2] = node_ok[c] ? a.u2[o] : T(0);
        }
    };

    const int mc = m / 2, nc = n / 2;
    const unsigned pldj = nc + 1;
    const unsigned pldi = (unsigned)(mc + 1) * pldj;
    const unsigned pcol = (unsigned)d * (mc + 1) * pldi;
    const int I = i >> 1, I0 = i0 >> 1;
    const int ab = i & 1;
    const int K0 = k0 >> 1;

    // per-row inputs of the cell row: viscosities and coarse pressure corners
    struct RowIn {
        T eta[CPL][2];
        T pc[CPL][4];
    };
    auto load_row = [&](int j, RowIn& r) {
        const unsigned ecol = (((unsigned)d * m + i) * m + j) * (unsigned)n * 2u;
        const int J = j >> 1;
        const unsigned pb0 = pcol + (unsigned)I * pldi + (unsigned)J * pldj;
        const unsigned pbq[4] = {pb0, pb0 + pldi, pb0 + pldj, pb0 + pldi + pldj};
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int k = cell_ok[c] ? kk[c] : k0;
            if (DO_A) {
                r.eta[c][0] = a.eta[ecol + 2u * k];
                r.eta[c][1] = a.eta[ecol + 2u * k + 1u];
            }
            if (DO_BT) {
                const int K = k >> 1, cb = k & 1;
                const T rw0 = iso.rw[cb][0], rw1 = iso.rw[cb][1];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    r.pc[c][q] = rw0 * a.p[pbq[q] + K] + rw1 * a.p[pbq[q] + K + 1];
            }
        }
    };

    // rolling partial sums of node row j+1 (R0: column i, R1: column i+1)
    T R0[NL][3], R1[NL][3];
#pragma unroll
    for (int c = 0; c < NL; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) R0[c][r] = R1[c][r] = T(0);

    // divergence: owner threads keep the two open coarse rows in registers
    constexpr int NOWN = 2;
    const int ncoarse = (TI / 2 + 1) * NKC;
    T pacc0[NOWN], pacc1[NOWN];
#pragma unroll
    for (int o = 0; o < NOWN; ++o) pacc0[o] = pacc1[o] = T(0);

    T uA[NL][3], uB[NL][3], uC[NL][3], uD[NL][3];
    RowIn rin;
    load_u(colA, jfirst, uA);
    load_u(colB, jfirst, uB);
    if (jfirst <= jlast_cell) {
        load_u(colA, jfirst + 1, uC);
        load_u(colB, jfirst + 1, uD);
        load_row(jfirst, rin);
    }

    for (int j = jfirst; j <= jlast; ++j) {
        const bool row_cells = j <= jlast_cell;    // the extra last step only emits
        const bool owned = j >= j0;
        const int par = j & 1;
        const int J = j >> 1, bb = j & 1;
        // prefetch the next cell row while this one is computed
        T uE[NL][3], uF[NL][3];
        RowIn rnext;
        const bool pre = j + 1 <= jlast_cell;
        if (pre) {
            load_u(colA, j + 2, uE);
            load_u(colB, j + 2, uF);
            load_row(j + 1, rnext);
        }
        T Nd[4][NL][3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) Nd[q][c][r] = T(0);
        T cp[4][NKL];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int s = 0; s < NKL; ++s) cp[q][s] = T(0);
        if (row_cells) {
            const T* g = a.geo + (((unsigned)d * m + i) * m + j) * (unsigned)GEO_PER_COL;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                if (!cell_ok[c]) continue;
                const int k = kk[c];
                const T rm = a.r_in + (T(k) + T(0.5)) * a.dr;
                const T s1 = T(0.5) / rm;
                const T rm2 = rm * rm;
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
                        for (int q = 0; q < 4; ++q) pbar += iso.lw[ab][bb][wd][q] * rin.pc[c][q];
                    }
                    const T eta = DO_A ? rin.eta[c][wd] : T(0);
                    WedgeOut<T> o;
                    wedge_apply<T, DO_A, DO_BT, DO_B>(uw, g + wd * GEO_PER_TRI, s1, rm2, eta, pbar, o);
                    if (DO_U) {
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
                        for (int q = 0; q < 4; ++q) tB[q] += iso.lw[ab][bb][wd][q] * o.dv;
                    }
                }
                if (DO_B) {
                    // coarse layers of this cell relative to the lane's first coarse layer
                    const int cb = k & 1;
                    const int sl = CPL == 1 ? 0 : ((k >> 1) - ((k0 + CPL * lane) >> 1));
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        cp[q][sl] += iso.rw[cb][0] * tB[q];
                        cp[q][sl + 1] += iso.rw[cb][1] * tB[q];
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
        if (DO_B && owned && row_cells) {
            // radial reduction of the coarse partials to one value per coarse layer
            if (CPL == 1) {
                // lanes 2K' and 2K'+1 share coarse layers K', K'+1
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) cp[q][s2] += __shfl(cp[q][s2], (lane + 1) & 63, 64);
                // the even lane's layer K'+1 part goes to the next even lane
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T t = __shfl(cp[q][1], (lane + 62) & 63, 64);
                    const T top = cp[q][1];
                    if ((lane & 1) == 0) {
                        const int Kl = lane >> 1;
                        bsl[par][w][q][Kl] = cp[q][0] + (lane >= 2 ? t : T(0));
                        if (lane == 62) bsl[par][w][q][32] = top;
                    }
                }
            } else {
                // lane l covers coarse layers CPL/2*l .. CPL/2*l + CPL/2
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T t = __shfl(cp[q][NKL - 1], (lane + 63) & 63, 64);
                    const int Kb = (CPL / 2) * lane;
#pragma unroll
                    for (int s2 = 0; s2 < NKL - 1; ++s2) {
                        T v = cp[q][s2];
                        if (s2 == 0 && lane > 0) v += t;
                        bsl[par][w][q][Kb + s2] = v;
                    }
                    if (lane == 63) bsl[par][w][q][Kb + NKL - 1] = cp[q][NKL - 1];
                }
            }
        }
        __syncthreads();
        if (DO_U && owned) {
            const unsigned rowA = colA + (unsigned)j * ldj;
            const unsigned rowB = colB + (unsigned)j * ldj;
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
                if (a.dirichlet && (k == 0 || k == n)) live = false;   // rows set afterwards
                if (!live) continue;
                T v[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    v[r] = R0[c][r] + Nd[0][c][r];
                    if (w > 0) v[r] += xch[par][w - 1][r][c][lane];
                }
                const bool seam = seamL || seamK;
                const unsigned oa = rowA + (unsigned)k;
                emit(a.y0, oa, v[0], seam);
                emit(a.y1, oa, v[1], seam);
                emit(a.y2, oa, v[2], seam);
                if (right) {
                    // node column i0 + TI: complete only on the diamond edge
                    const bool s2 = seamR || seamK;
                    const unsigned ob = rowB + (unsigned)k;
                    emit(a.y0, ob, xch[par][w][0][c][lane], s2);
                    emit(a.y1, ob, xch[par][w][1][c][lane], s2);
                    emit(a.y2, ob, xch[par][w][2][c][lane], s2);
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
        if (DO_B && owned && row_cells) {
            // owner threads add the (up to four) waves touching each coarse node, in
            // a fixed order, into the open rows J (corners 0, 1) and J+1 (corners 2, 3)
#pragma unroll
            for (int o = 0; o < NOWN; ++o) {
                const int idx = threadIdx.x + o * TI * 64;
                if (idx < ncoarse) {
                    const int il = idx / NKC, kl = idx % NKC;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int ws = 2 * (il - (q & 1));   // waves whose coarse column is il - (q&1)
                        T v = T(0);
                        if (ws >= 0 && ws < TI) v += bsl[par][ws][q][kl];
                        if (ws + 1 >= 0 && ws + 1 < TI) v += bsl[par][ws + 1][q][kl];
                        if (q < 2) pacc0[o] += v; else pacc1[o] += v;
                    }
                }
            }
            if (j & 1) {
                // coarse row J has received all of this band's cells
                const bool rowseam = (J == (j0 >> 1) && j0 > 0);
#pragma unroll
                for (int o = 0; o < NOWN; ++o) {
                    const int idx = threadIdx.x + o * TI * 64;
                    if (idx < ncoarse) {
                        const int il = idx / NKC, kl = idx % NKC;
                        const int Ig = I0 + il, Kg = K0 + kl;
                        if (Ig <= mc && Kg <= nc && kl <= (kend - k0) / 2) {
                            const bool seam = rowseam || (il == 0 && I0 > 0) ||
                                              (il == TI / 2 && Ig < mc) ||
                                              (kl == 0 && K0 > 0) || (Kg < nc && kl == (kend - k0) / 2);
                            emit(a.yp, pcol + (unsigned)Ig * pldi + (unsigned)J * pldj + (unsigned)Kg,
                                 pacc0[o], seam);
                        }
                    }
                    pacc0[o] = pacc1[o];
                    pacc1[o] = T(0);
                }
            }
        }
        if (pre) {
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    uA[c][r] = uC[c][r];
                    uB[c][r] = uD[c][r];
                    uC[c][r] = uE[c][r];
                    uD[c][r] = uF[c][r];
                }
            rin = rnext;
        }
    }
    if (DO_B) {
        // the coarse row above the band's last cell row: complete only on the last band
        const int J = (jlast_cell >> 1) + 1;
#pragma unroll
        for (int o = 0; o < NOWN; ++o) {
            const int idx = threadIdx.x + o * TI * 64;
            if (idx < ncoarse) {
                const int il = idx / NKC, kl = idx % NKC;
                const int Ig = I0 + il, Kg = K0 + kl;
                if (Ig <= mc && Kg <= nc && J <= mc && kl <= (kend - k0) / 2) {
                    const bool seam = !last_band || (il == 0 && I0 > 0) || (il == TI / 2 && Ig < mc) ||
                                      (kl == 0 && K0 > 0) || (Kg < nc && kl == (kend - k0) / 2);
                    emit(a.yp, pcol + (unsigned)Ig * pldi + (unsigned)J * pldj + (unsigned)Kg, pacc0[o],
                         seam);
                }
            }
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
    const int cpl_max = is64 ? 1 : 2;
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
        else
            launch_band_ops<T, 2>(ctx, a, key);
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
