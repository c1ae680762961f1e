// Streaming kernel for the Stokes apply y = K(eta) [u; p] (Sec. 3, one-point
// rule of Sec. 4).
//
// Work decomposition (one diamond d, a "band"):
//   * lanes run along the radial direction: lane l of a wave handles the CPL
//     consecutive cells k = k0 + CPL*l + c of one cell column, so every memory
//     access of a wave covers a contiguous radial stretch of 64 CPL cells;
//   * a workgroup has WG = 4 or 8 waves: TC = WG / RS adjacent cell columns, each
//     column split into RS radial stretches handled by RS waves, so that one
//     workgroup holds whole radial columns (a column split across workgroups
//     costs far more, in memory stalls, than the split inside one);
//   * the workgroup streams along j over the cell rows of its band, carrying
//     the half-finished node row in registers, so each node of the band's
//     interior is written exactly once, with its complete sum.
// Velocity rows are staged in a three-row LDS ring (rows j, j+1 in use, row
// j+2 arriving), copied straight from HBM without passing through registers;
// each node column is read from HBM once per workgroup and shared by the
// waves that touch it.  The nodal differences of a triangle are formed once
// per node layer and shared by the wedges below and above it, and so are the
// test-function sums of the result.  Contributions that cross a wave boundary
// are combined in LDS (lateral, and radial between the stretches of a column)
// or moved one lane up with a DPP wavefront shift (radial, inside a wave).  A
// band starts one cell row early (the halo row; two with the divergence block)
// so that its first node row and its first coarse pressure row are complete, and
// every node row belongs to one band.  Nodes on the seams between tiles (node
// columns that are multiples of TC) receive exactly two partial sums, added
// with atomics to memory zeroed beforehand; two partials sum to the same value
// in either order, so the result does not depend on timing.  Columns longer
// than RS stretches are split into workgroup radial ranges, whose seam layers
// also take two partials; where such a layer crosses a tile seam a node takes
// four, whose order can vary from run to run (levels with more than 256
// radial cells only).
//
// The divergence block is reduced per coarse pressure node through LDS, kept
// by one owner thread per node and flushed once a coarse row is complete.
//
// The band count is chosen per launch from the kernel's resident workgroups
// (bands of unequal length, starting on even rows), and blocks are renumbered
// so that each XCD works on a contiguous run of tiles and bands.
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <type_traits>

#include "batch_dev.hpp"
#include "tng_internal.hpp"
#include "wedge.hpp"

namespace tng {
namespace {

constexpr int TIC = 8;   // widest workgroup: waves (cell columns when a column fits one wave)


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
    int TI, KC;
    int ntile, nband, nchunk;
    T r_in, dr;
    T hg;          // hourglass control: alpha * 5/81 (0 without)
    int ns_in, ns_out;   // no-slip (zero) velocity on the inner / outer sphere
    int fs;              // free slip: bit 0 inner sphere, bit 1 outer sphere
    const T* __restrict__ unit;   // [10][m+1][m+1][3] node unit vectors (free slip)
    const T* __restrict__ rho;    // [n+1] reference density at the node layers (TALA)
};

template <typename T>
__device__ __forceinline__ T shfl_up1(T v, int lane) {
    return __shfl(v, (lane + 63) & 63, 64);
}

// Element idx of a field addressed by a 32-bit byte offset from its (wave-uniform)
// base, so that the compiler can use the scalar-base addressing form (64-bit base in
// scalar registers, 32-bit offset per lane) instead of a 64-bit address per lane; the
// host refuses fields of 4 GiB or more.
template <typename T>
__device__ __forceinline__ T* elem(T* base, unsigned idx) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T& elem(const T* base, unsigned idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}

// Emit one node value: plain store when this workgroup holds its complete
// sum, atomic add (onto zeroed memory) on tile or chunk seams.
template <typename T>
__device__ __forceinline__ void emit(T* y, unsigned idx, T v, bool seam) {
    if (seam)
        atomicAdd(elem(y, idx), v);
    else
        *elem(y, idx) = v;
}

// The three components of one velocity node under a single seam branch.
template <typename T>
__device__ __forceinline__ void emit3(T* const (&y)[3], unsigned idx, const T (&v)[3], bool seam) {
    if (seam) {
#pragma unroll
        for (int r = 0; r < 3; ++r) atomicAdd(elem(y[r], idx), v[r]);
    } else {
#pragma unroll
        for (int r = 0; r < 3; ++r) *elem(y[r], idx) = v[r];
    }
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

// Lane l receives lane l+1 (shl) or lane l-1 (shr); lanes shifted in from
// outside the wavefront read zero (DPP wave shift with bound control).
template <int CTRL>
__device__ __forceinline__ float wave_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double wave_shift(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

// BATCH: copy blockIdx.z works on the fields of slot z of a batch (mesh
// geometry shared); otherwise sb is unused.
// WG: waves per workgroup (4 or 8); a workgroup covers WG / RS cell columns.
// FS: free slip on a sphere (a.fs), staged boundary velocities projected onto the
// tangent plane; TALA: the divergence block tests div(rhobar u) with the mass flux
// rhobar u interpolated nodally; the other kernels compile without these paths.
// TWOPT: the viscous block with the two-radial-point rule (Sec. 4) instead of the one
// point (the divergence blocks keep the one point).
template <typename T, int RS, int CPL, bool DO_A, bool DO_BT, bool DO_B, bool DO_HG, bool BATCH, int WG, bool FS,
          bool TALA, bool TWOPT = false>
__global__ void __launch_bounds__(WG * 64) stokes_band_kernel(BandArgs<T> a, SlotBatch sb) {
    static_assert(!TALA || DO_B, "the reference density enters the divergence block only");
    static_assert(!TWOPT || (DO_A && !DO_HG), "the two-point rule is a form of the viscous block");
    static_assert(DO_A || !DO_HG, "hourglass control belongs to the viscous block");
    if constexpr (BATCH) {
        const long long so = slot_off(sb);
        a.eta = at_slot(a.eta, so);
        a.u0 = at_slot(a.u0, so);
        a.u1 = at_slot(a.u1, so);
        a.u2 = at_slot(a.u2, so);
        a.p = at_slot(a.p, so);
        a.y0 = at_slot(a.y0, so);
        a.y1 = at_slot(a.y1, so);
        a.y2 = at_slot(a.y2, so);
        a.yp = at_slot(a.yp, so);
    }
    constexpr int TC = WG / RS;   // cell columns per workgroup; RS waves share a column radially
    constexpr int NL = CPL + 1;   // node layers per lane: bottom of each cell + top partial
    constexpr bool DO_U = DO_A || DO_BT;
    constexpr bool LOAD_U = DO_A || DO_B;
    constexpr int KC = 64 * CPL;                // cells of one wave's radial stretch
    // velocity rows j, j+1, j+2 of the TC + 1 node columns, radial fastest
    constexpr int KW = RS * KC + 1;             // node layers of the workgroup's radial range
    constexpr int KWP = (KW + 1) & ~1;          // even pitch: lane pairs stay 8-byte aligned
    constexpr int RR = LOAD_U ? 3 : 1;
    constexpr int RW = LOAD_U ? TC + 1 : 1;
    __shared__ T ring[RR][RW][3][KWP];
    constexpr int XW = DO_U ? WG : 1;
    __shared__ T xch[2][XW][3][CPL][64];   // lateral partials of layers 0..CPL-1 of every lane
    __shared__ T xtop[2][XW][3];           // and of the workgroup's top node
    constexpr int RX = (DO_U && RS > 1) ? WG : 1;
    __shared__ T rxs[2][RX][4][3];     // top-layer partials handed to the wave above
    constexpr int NKC = DO_B ? 32 * CPL + 1 : 1;          // coarse layers of one wave
    constexpr int PADW = 2 * RS;                          // two empty columns each side
    constexpr int BW = DO_B ? WG + 2 * PADW : 1;
    __shared__ T bsl[2][BW][4][NKC];   // per-wave coarse partials, wave w in slot w + PADW
    constexpr int NKL = CoarseMap<CPL>::NKL;
    const IsoWeights<T>& iso = IsoTable<T>::get();

    const int TI = a.TI;   // columns, <= TC on small levels; the workgroup has TI * RS waves
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wc = w / RS;       // column of the wave within the tile
    const int h = w % RS;        // radial stretch of the wave within the workgroup
    // XCD-aware order: the dispatcher deals consecutive workgroups to the eight XCDs
    // in turn; each XCD takes a contiguous run of (tile, band) blocks instead, so that
    // the same bands of neighbouring tiles, which share a node column, run together
    // under one L2
    int bid;
    {
        const unsigned nbk = gridDim.x, q = nbk >> 3, r = nbk & 7, x = blockIdx.x & 7;
        bid = (int)(x * q + min(x, r) + (blockIdx.x >> 3));
    }
    const int chunk = bid % a.nchunk;
    bid /= a.nchunk;
    const int band = bid % a.nband;
    bid /= a.nband;
    const int tile = bid % a.ntile;
    const int d = bid / a.ntile;

    const int m = a.m, n = a.n;
    const int i0 = tile * TI;
    const int i = i0 + wc;
    // band b: cell rows [j0, j1), starting on even rows (so that coarse rows stay
    // whole), lengths differing by at most two rows
    const int j0 = 2 * ((band * (m >> 1)) / a.nband);
    const bool last_band = (band == a.nband - 1);
    const int j1 = last_band ? m : 2 * (((band + 1) * (m >> 1)) / a.nband);
    // halo rows (computed, not owned): one for the velocity rows; the divergence
    // kernels take a second one, so that the band's first coarse pressure row is
    // complete in the band and every coarse row belongs to one band
    const int jfirst = j0 > 0 ? j0 - (DO_B ? 2 : 1) : 0;
    const int jlast_cell = j1 - 1;
    const int jlast = last_band ? m : jlast_cell;      // last node row emitted
    const int kc0 = chunk * RS * KC;                   // workgroup's radial range [kc0, kcend)
    const int kcend = min(n, kc0 + RS * KC);
    const int k0 = kc0 + h * KC;                       // even: KC is a multiple of 64
    const int kend = min(kcend, k0 + KC);              // cells [k0, kend) of this wave

    // 32-bit element offsets (and byte offsets: every field is below 4 GiB)
    const unsigned ldj = n + 1;
    const unsigned ldi = (unsigned)(m + 1) * ldj;
    const unsigned colA = ((unsigned)d * (m + 1) + i) * ldi;   // node column i
    const unsigned colB = colA + ldi;                          // node column i + 1

    const int kl0 = CPL * lane;                        // first wave-local layer of the lane
    int kk[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) kk[c] = k0 + kl0 + c;
    // radial factors of the lane's cells; a cell outside the chunk gets a zero
    // volume, which zeroes every contribution it makes
    T s1[CPL], vr[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const T rm = a.r_in + (T(kk[c]) + T(0.5)) * a.dr;
        s1[c] = T(0.5) / rm;
        vr[c] = kk[c] < kend ? rm * rm : T(0);
    }
    // TALA: reference density at the lane's node layers (W1 in the radius, so the
    // nodal mass flux of a layer is rhobar of that layer times u)
    T rho_l[NL];
#pragma unroll
    for (int c = 0; c < NL; ++c) rho_l[c] = TALA ? a.rho[min(kk[c], n)] : T(1);
    // the lane holding the workgroup's top node (layer kcend)
    const bool top_lane = (kk[0] <= kcend - 1) && (kcend - 1 <= kk[CPL - 1]);
    const int top_c = kcend - kk[0];

    // velocity staging: each radial line of a column over the workgroup's range
    // (KW values of one component) is copied straight from HBM into its ring
    // row, 64 dwords per instruction, lane l moving dword l of each 256-byte
    // piece; the RS waves of a column copy consecutive stretches of it, the top
    // one also the range's top node.  Dirichlet layers and layers past the
    // range are never written and keep the zeros the ring starts with.
    constexpr int DW = sizeof(T) / 4;                   // dwords per value
    constexpr int NCH = CPL * DW + 1;                   // 256-byte pieces per wave (+ the top node)
    bool lok[NCH];
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
        const int e = h * KC + (lane + 64 * t) / DW;    // value moved by this lane
        const int k = kc0 + e;
        lok[t] = LOAD_U && e < KW && k <= kcend && (t < NCH - 1 || h == RS - 1) &&
                 !((a.ns_in && k == 0) || (a.ns_out && k == n));
    }
    // free slip: this lane moved the first dword of a node value on a free-slip
    // sphere in piece t, and projects that node's staged velocity onto the
    // sphere's tangent plane once its loads have landed
    bool fsb[NCH];
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
        const int e = h * KC + (lane + 64 * t) / DW;
        const int k = kc0 + e;
        fsb[t] = FS && lok[t] && ((lane + 64 * t) % DW == 0) &&
                 (((a.fs & 1) && k == 0) || ((a.fs & 2) && k == n));
    }
    // u <- u - rhat (rhat . u) at the staged boundary nodes of node row jrow of
    // ring column wl (library column icol); waves touch only values they staged
    auto project_staged = [&](int icol, int jrow, int slot, int wl) {
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
            if (!fsb[t]) continue;
            const int e = h * KC + (lane + 64 * t) / DW;
            const T* nv = a.unit + (((unsigned)d * (m + 1) + icol) * (m + 1) + jrow) * 3u;
            const T n0 = nv[0], n1 = nv[1], n2 = nv[2];
            T* x0 = &ring[slot][wl][0][e];
            T* x1 = &ring[slot][wl][1][e];
            T* x2 = &ring[slot][wl][2][e];
            const T dn = n0 * *x0 + n1 * *x1 + n2 * *x2;
            *x0 -= dn * n0;
            *x1 -= dn * n1;
            *x2 -= dn * n2;
        }
    };
    auto stage = [&](unsigned col, int jrow, int slot, int wl) {
        const unsigned base = col + (unsigned)jrow * ldj + (unsigned)k0;
        const T* const src[3] = {a.u0, a.u1, a.u2};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int t = 0; t < NCH; ++t)
                if (lok[t])
                    __builtin_amdgcn_global_load_lds(
                        reinterpret_cast<const unsigned*>(reinterpret_cast<const char*>(src[r]) +
                                                          (base * (unsigned)sizeof(T) + 4u * (lane + 64 * t))),
                        reinterpret_cast<unsigned*>(&ring[slot][wl][r][0]) + h * KC * DW + 64 * t, 4, 0, 0);
    };

    const int mc = m / 2, nc = n / 2;
    const unsigned pldj = nc + 1;
    const unsigned pldi = (unsigned)(mc + 1) * pldj;
    const unsigned pcol = (unsigned)d * (mc + 1) * pldi;
    const int I = i >> 1, I0 = i0 >> 1;
    const int ab = i & 1;
    const int K0 = kc0 >> 1;

    // per-row inputs of the cell row: viscosities, and the coarse pressure of
    // the four lateral corners on the NKL coarse layers the lane's cells touch
    // (combined only when used, so that the loads stay in flight)
    const int Kb = (k0 + kl0) >> 1;
    int Kp[NKL];
#pragma unroll
    for (int s = 0; s < NKL; ++s) Kp[s] = min(Kb + s, nc);
    struct RowIn {
        T eta[CPL][2];
        T pk[4][NKL];
    };
    auto load_row = [&](int j, RowIn& r) {
        const unsigned ecol = (((unsigned)d * m + i) * m + j) * (unsigned)n * 2u;
        if (DO_A) {
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                // a cell outside the wave's stretch reads the range's first cell: the wave's own
            // first cell lies past the column when the stretch is empty
            const int k = kk[c] < kend ? kk[c] : kc0;
                r.eta[c][0] = elem(a.eta, ecol + 2u * k);
                r.eta[c][1] = elem(a.eta, ecol + 2u * k + 1u);
            }
        }
        if (DO_BT) {
            const unsigned pb0 = pcol + (unsigned)I * pldi + (unsigned)(j >> 1) * pldj;
            const unsigned pbq[4] = {pb0, pb0 + pldi, pb0 + pldj, pb0 + pldi + pldj};
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int s = 0; s < NKL; ++s) r.pk[q][s] = elem(a.p, pbq[q] + Kp[s]);
        }
    };

    // node-row partial sums, [column i / i+1][layer][component]: Rc for node row
    // j (complete after this row's cells), Rn for node row j+1
    T Rc[2][NL][3];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int c = 0; c < NL; ++c)
#pragma unroll
            for (int r = 0; r < 3; ++r) Rc[q][c][r] = T(0);

    // divergence: owner thread t < ncoarse (at most one coarse node per thread,
    // guaranteed by the host's choice of TI, RS and CPL) keeps its two open
    // coarse rows in registers
    constexpr int NKW = RS * (NKC - 1) + 1;               // coarse layers of the workgroup
    const int ncoarse = (TI / 2 + 1) * NKW;
    const bool owner = DO_B && (int)threadIdx.x < ncoarse;
    const int il = (int)threadIdx.x / NKW, kl = (int)threadIdx.x % NKW;
    const int Ig = I0 + il, Kg = K0 + kl;
    const bool own_ok = owner && Ig <= mc && Kg <= nc && kl <= (kcend - kc0) / 2;
    const bool own_seam = (il == 0 && I0 > 0) || (il == TI / 2 && Ig < mc) || (kl == 0 && K0 > 0) ||
                          (Kg < nc && kl == (kcend - kc0) / 2);
    const unsigned own_off = pcol + (unsigned)Ig * pldi + (unsigned)Kg;
    // the owner's coarse layer in the waves' slots: wave stretch hk, local layer klo;
    // a stretch boundary layer is also the top layer of the stretch below
    const int hk = min(kl / (NKC - 1), RS - 1), klo = kl - hk * (NKC - 1);
    const bool below = RS > 1 && klo == 0 && hk > 0;
    if (DO_B) {
        // wave slots without a wave stay zero: two columns below, two from column TI on
        for (int x = threadIdx.x; x < 2 * PADW * 4 * NKC; x += TI * RS * 64) {
            const int sl = x / (4 * NKC), rem = x % (4 * NKC);
            const int slot = sl < PADW ? sl : (TI * RS + sl);
            (&bsl[0][0][0][0])[(size_t)slot * 4 * NKC + rem] = T(0);
            (&bsl[1][0][0][0])[(size_t)slot * 4 * NKC + rem] = T(0);
        }
    }
    T pacc0 = T(0), pacc1 = T(0);

    int sj = 0, sj1 = 1, sj2 = 2;    // ring slots of node rows j, j+1, j+2
    const bool xw = (wc == TI - 1);  // the last column's waves also stage column i0 + TI
    RowIn rin;
    if (LOAD_U) {
        for (int x = threadIdx.x; x < RR * RW * 3 * KWP; x += TI * RS * 64) (&ring[0][0][0][0])[x] = T(0);
        __syncthreads();
        stage(colA, jfirst, sj, wc);
        stage(colA, jfirst + 1, sj1, wc);
        if (xw) {
            stage(colB, jfirst, sj, TI);
            stage(colB, jfirst + 1, sj1, TI);
        }
    }
    load_row(jfirst, rin);
    __builtin_amdgcn_s_waitcnt(0);   // staged rows have landed in LDS
    if constexpr (FS && LOAD_U) {
        project_staged(i, jfirst, sj, wc);
        project_staged(i, jfirst + 1, sj1, wc);
        if (xw) {
            project_staged(i0 + TI, jfirst, sj, TI);
            project_staged(i0 + TI, jfirst + 1, sj1, TI);
        }
    }
    __syncthreads();

    // one cell row: rows alternate between the two register sets, so that the
    // loop carries no copies
    auto step = [&](const int j, T (&Rc)[2][NL][3], T (&Rn)[2][NL][3], const RowIn& rin, RowIn& rnext) {
        const bool row_cells = j <= jlast_cell;    // the extra last step only emits
        const bool owned = j >= j0;
        const int par = j & 1;
        const int J = j >> 1, bb = j & 1;
        // prefetch the next cell row while this one is computed
        const bool pre = j + 1 <= jlast_cell;
        if (pre) {
            // node row j+2 into the slot of row j-1, read for the last time
            // before the previous barrier
            if (LOAD_U) {
                stage(colA, j + 2, sj2, wc);
                if (xw) stage(colB, j + 2, sj2, TI);
            }
            load_row(j + 1, rnext);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) Rn[q][c][r] = T(0);
        T cp[4][NKL];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int s = 0; s < NKL; ++s) cp[q][s] = T(0);
        T top_out[4][3];   // this row's top-layer partials (the DPP shift drops lane 63's)
        if (row_cells) {
            const T* g = a.geo + (((unsigned)d * m + i) * m + j) * (unsigned)GEO_PER_COL;
            // staged velocity of corner q (A=(i,j), B=(i+1,j), C=(i,j+1), D=(i+1,j+1))
            auto rd = [&](int q, int c, int r) -> T {
                return ring[q < 2 ? sj : sj1][wc + (q & 1)][r][h * KC + kl0 + c];
            };
            T top[4][3];   // partials of the lane's top layer, per corner
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                // triangle corners: wedge 0 (A, B, C), wedge 1 (D, C, B)
                const int q0 = t == 0 ? 0 : 3, q1 = t == 0 ? 1 : 2, q2 = t == 0 ? 2 : 1;
                const T* gt = g + t * GEO_PER_TRI;
                // per-layer nodal differences, shared by the wedges below and above:
                // e1 = u1 - u0, e2 = u2 - u0, sm = u0 + u1 + u2
                auto derive = [&](int c, T (&e)[3][3]) {
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const T x0 = LOAD_U ? rd(q0, c, r) : T(0);
                        const T x1 = LOAD_U ? rd(q1, c, r) : T(0);
                        const T x2 = LOAD_U ? rd(q2, c, r) : T(0);
                        e[0][r] = x1 - x0;
                        e[1][r] = x2 - x0;
                        e[2][r] = x0 + x1 + x2;
                    }
                };
                const T r3[3] = {gt[6], gt[7], gt[8]};
                // hourglass control (eq:hgstab over the three barycentric modes): a node
                // of lateral index l and face zeta = -1/+1 receives zeta eps (Du_l - mean Du),
                // Du the top-minus-bottom nodal difference, eps = alpha mean(diag A_e) =
                // alpha 5/27 eta V sum_j |grad phi_j|^2 and sum_j |grad phi_j|^2 =
                // s1^2 hgA + hgB with the triangle's metric sums below
                T hgA = T(0), hgB = T(0);
                if (DO_HG) {
                    hgA = T(4) * (gt[0] * gt[0] + gt[1] * gt[1] + gt[2] * gt[2] + gt[3] * gt[3] + gt[4] * gt[4] +
                                  gt[5] * gt[5] + gt[0] * gt[3] + gt[1] * gt[4] + gt[2] * gt[5]);
                    hgB = T(6) * (gt[6] * gt[6] + gt[7] * gt[7] + gt[8] * gt[8]);
                }
                T hxb[3], hyb[3];   // eps/3 times the e1, e2 differences of the wedge below
                T plat[NKL];   // pressure at the wedge's lateral centroid, per coarse layer
                if (DO_BT) {
#pragma unroll
                    for (int s = 0; s < NKL; ++s) {
                        T v = T(0);
#pragma unroll
                        for (int q = 0; q < 4; ++q) v += iso.lw[ab][bb][t][q] * rin.pk[q][s];
                        plat[s] = v;
                    }
                }
                T dvl[NKL];    // -V div u of the triangle's wedges, per coarse layer
#pragma unroll
                for (int s = 0; s < NKL; ++s) dvl[s] = T(0);
                T lo[3][3], hi[3][3], zb[3][3];
                derive(0, lo);
#pragma unroll
                for (int c = 0; c < CPL; ++c) {
                    derive(c + 1, hi);
                    const T r1[3] = {gt[0] * s1[c], gt[1] * s1[c], gt[2] * s1[c]};
                    const T r2[3] = {gt[3] * s1[c], gt[4] * s1[c], gt[5] * s1[c]};
                    const T V = vr[c] * gt[9];
                    // velocity gradient at q_c: du_r/dx_a = A_r rho1~_a + B_r rho2~_a + C_r rho3'_a
                    T L[3][3];
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const T Ar = lo[0][r] + hi[0][r];
                        const T Br = lo[1][r] + hi[1][r];
                        const T Cr = hi[2][r] - lo[2][r];
#pragma unroll
                        for (int x = 0; x < 3; ++x) L[r][x] = Ar * r1[x] + Br * r2[x] + Cr * r3[x];
                    }
                    const T tr = L[0][0] + L[1][1] + L[2][2];
                    if (DO_B) {
                        // -V div u, split onto the two coarse layers of the cell; with the
                        // reference density -V div(rhobar u): the trace is the sum of a
                        // bottom-layer and a top-layer part, each scaled by its layer's rhobar
                        T trd = tr;
                        if constexpr (TALA) {
                            T tlo = T(0), thi = T(0);
#pragma unroll
                            for (int r = 0; r < 3; ++r) {
                                tlo += lo[0][r] * r1[r] + lo[1][r] * r2[r] - lo[2][r] * r3[r];
                                thi += hi[0][r] * r1[r] + hi[1][r] * r2[r] + hi[2][r] * r3[r];
                            }
                            trd = rho_l[c] * tlo + rho_l[c + 1] * thi;
                        }
                        const T dv = -V * trd;
                        const int cb = (kl0 + c) & 1;
                        const int sl = ((kl0 + c) >> 1) - (kl0 >> 1);
                        dvl[sl] += iso.rw[cb][0] * dv;
                        dvl[sl + 1] += iso.rw[cb][1] * dv;
                    }
                    T za[3][3];   // Z_m = (V sigma) rho_m, rows m = 1, 2, 3
                    T zt[3][3];   // two-point rule: the rows for the wedge's top-face nodes
                    T hx[3], hy[3];
                    if (DO_HG) {
                        const T e3 = a.hg * rin.eta[c][t] * V * (s1[c] * s1[c] * hgA + hgB);
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            hx[r] = e3 * (hi[0][r] - lo[0][r]);
                            hy[r] = e3 * (hi[1][r] - lo[1][r]);
                        }
                    }
                    if (DO_U) {
                        T pbar = T(0);
                        if (DO_BT) {
                            const int cb = (kl0 + c) & 1;
                            const int sl = ((kl0 + c) >> 1) - (kl0 >> 1);
                            pbar = iso.rw[cb][0] * plat[sl] + iso.rw[cb][1] * plat[sl + 1];
                        }
                        T S[3][3];
                        if constexpr (TWOPT) {
                            // two radial points zeta = -+1/sqrt 3, weight 1/2 each, at radius
                            // r_q = r_m + zeta dr/2 (the Jacobian there is G diag(r_q, r_q, dr/2)):
                            // the lateral differences carry (1 -+ zeta) for the bottom / top
                            // layer, and each point's rows Z_1, Z_2 reach the bottom-face
                            // nodes with weight (1 - zeta) and the top-face nodes with (1 + zeta);
                            // B^T stays at q_c (both faces, weight 1)
                            const T rm = a.r_in + (T(kk[c]) + T(0.5)) * a.dr;
                            const T vis = vr[c] != T(0) ? rin.eta[c][t] * gt[9] * T(0.5) : T(0);
#pragma unroll
                            for (int x = 0; x < 3; ++x)
#pragma unroll
                                for (int r = 0; r < 3; ++r) {
                                    const T bt = DO_BT ? -V * pbar * (x == 0 ? r1[r] : (x == 1 ? r2[r] : r3[r]))
                                                       : T(0);
                                    za[x][r] = bt;
                                    zt[x][r] = bt;
                                }
#pragma unroll
                            for (int qq = 0; qq < 2; ++qq) {
                                const T zq = qq == 0 ? T(-0.57735026918962576451) : T(0.57735026918962576451);
                                const T rq = rm + zq * (T(0.5) * a.dr);
                                const T s1q = T(0.5) / rq;
                                const T q1[3] = {gt[0] * s1q, gt[1] * s1q, gt[2] * s1q};
                                const T q2[3] = {gt[3] * s1q, gt[4] * s1q, gt[5] * s1q};
                                T Lq[3][3];
#pragma unroll
                                for (int r = 0; r < 3; ++r) {
                                    const T Ar = (T(1) - zq) * lo[0][r] + (T(1) + zq) * hi[0][r];
                                    const T Br = (T(1) - zq) * lo[1][r] + (T(1) + zq) * hi[1][r];
                                    const T Cr = hi[2][r] - lo[2][r];
#pragma unroll
                                    for (int x = 0; x < 3; ++x) Lq[r][x] = Ar * q1[x] + Br * q2[x] + Cr * r3[x];
                                }
                                const T trq = Lq[0][0] + Lq[1][1] + Lq[2][2];
                                const T e1 = vis * rq * rq;          // eta V_q
                                const T e2 = e1 + e1;
                                const T qd = e2 * trq * T(1.0 / 3.0);
                                T Sq[3][3];
                                Sq[0][0] = e2 * Lq[0][0] - qd;
                                Sq[1][1] = e2 * Lq[1][1] - qd;
                                Sq[2][2] = e2 * Lq[2][2] - qd;
                                Sq[0][1] = Sq[1][0] = e1 * (Lq[0][1] + Lq[1][0]);
                                Sq[0][2] = Sq[2][0] = e1 * (Lq[0][2] + Lq[2][0]);
                                Sq[1][2] = Sq[2][1] = e1 * (Lq[1][2] + Lq[2][1]);
#pragma unroll
                                for (int r = 0; r < 3; ++r) {
                                    const T z1 = Sq[r][0] * q1[0] + Sq[r][1] * q1[1] + Sq[r][2] * q1[2];
                                    const T z2 = Sq[r][0] * q2[0] + Sq[r][1] * q2[1] + Sq[r][2] * q2[2];
                                    const T z3 = Sq[r][0] * r3[0] + Sq[r][1] * r3[1] + Sq[r][2] * r3[2];
                                    za[0][r] += (T(1) - zq) * z1;
                                    za[1][r] += (T(1) - zq) * z2;
                                    za[2][r] += z3;
                                    zt[0][r] += (T(1) + zq) * z1;
                                    zt[1][r] += (T(1) + zq) * z2;
                                    zt[2][r] += z3;
                                }
                            }
                        } else if (DO_A) {
                            const T e1 = rin.eta[c][t] * V;
                            const T e2 = e1 + e1;
                            const T qd = e2 * tr * T(1.0 / 3.0) + (DO_BT ? V * pbar : T(0));
                            S[0][0] = e2 * L[0][0] - qd;
                            S[1][1] = e2 * L[1][1] - qd;
                            S[2][2] = e2 * L[2][2] - qd;
                            S[0][1] = S[1][0] = e1 * (L[0][1] + L[1][0]);
                            S[0][2] = S[2][0] = e1 * (L[0][2] + L[2][0]);
                            S[1][2] = S[2][1] = e1 * (L[1][2] + L[2][1]);
                        } else {
                            const T qd = V * pbar;
#pragma unroll
                            for (int r = 0; r < 3; ++r)
#pragma unroll
                                for (int x = 0; x < 3; ++x) S[r][x] = (r == x) ? -qd : T(0);
                        }
                        if constexpr (!TWOPT) {
#pragma unroll
                            for (int r = 0; r < 3; ++r) {
                                za[0][r] = S[r][0] * r1[0] + S[r][1] * r1[1] + S[r][2] * r1[2];
                                za[1][r] = S[r][0] * r2[0] + S[r][1] * r2[1] + S[r][2] * r2[2];
                                za[2][r] = S[r][0] * r3[0] + S[r][1] * r3[1] + S[r][2] * r3[2];
                            }
                        }
                        // nodal values of layer c: test functions of the wedge above
                        // (g' = (-1,-1,-1), (1,0,-1), (0,1,-1)) and, from c = 1 on,
                        // of the wedge below (g' = (-1,-1,1), (1,0,1), (0,1,1))
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
                            T P1 = za[0][r], P2 = za[1][r], Q = -za[2][r];
                            if (c > 0) {
                                P1 += zb[0][r];
                                P2 += zb[1][r];
                                Q += zb[2][r];
                            }
                            T N0 = Q - (P1 + P2), N1 = P1 + Q, N2 = P2 + Q;
                            if (DO_HG) {
                                // eps c_l of the wedge below minus that of the wedge above
                                const T DX = (c > 0 ? hxb[r] : T(0)) - hx[r];
                                const T DY = (c > 0 ? hyb[r] : T(0)) - hy[r];
                                N0 -= DX + DY;
                                N1 += T(2) * DX - DY;
                                N2 += T(2) * DY - DX;
                            }
                            if (t == 0) {
                                Rc[0][c][r] += N0;
                                Rc[1][c][r] += N1;
                                Rn[0][c][r] += N2;
                            } else {
                                Rn[1][c][r] += N0;
                                Rn[0][c][r] += N1;
                                Rc[1][c][r] += N2;
                            }
                        }
#pragma unroll
                        for (int x = 0; x < 3; ++x)
#pragma unroll
                            for (int r = 0; r < 3; ++r) zb[x][r] = TWOPT ? zt[x][r] : za[x][r];
                        if (DO_HG) {
#pragma unroll
                            for (int r = 0; r < 3; ++r) {
                                hxb[r] = hx[r];
                                hyb[r] = hy[r];
                            }
                        }
                    }
#pragma unroll
                    for (int x = 0; x < 3; ++x)
#pragma unroll
                        for (int r = 0; r < 3; ++r) lo[x][r] = hi[x][r];
                }
                if (DO_B) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int s = 0; s < NKL; ++s) cp[q][s] += iso.lw[ab][bb][t][q] * dvl[s];
                }
                if (DO_U) {
                    // top layer of the lane: the wedge below only
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        const T z12 = zb[0][r] + zb[1][r];
                        T N0 = zb[2][r] - z12, N1 = zb[0][r] + zb[2][r], N2 = zb[1][r] + zb[2][r];
                        if (DO_HG) {
                            N0 -= hxb[r] + hyb[r];
                            N1 += T(2) * hxb[r] - hyb[r];
                            N2 += T(2) * hyb[r] - hxb[r];
                        }
                        if (t == 0) {
                            top[0][r] = N0;
                            top[1][r] = N1;
                            top[2][r] = N2;
                        } else {
                            top[3][r] = N0;
                            top[2][r] += N1;
                            top[1][r] += N2;
                        }
                    }
                }
            }
            if (DO_U) {
                // radial: the top partial of the lane below completes this lane's
                // bottom layer; the top layer itself is kept for the chunk's top node
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    Rc[0][0][r] += wave_shift<DPP_WAVE_SHR1>(top[0][r]);
                    Rc[1][0][r] += wave_shift<DPP_WAVE_SHR1>(top[1][r]);
                    Rn[0][0][r] += wave_shift<DPP_WAVE_SHR1>(top[2][r]);
                    Rn[1][0][r] += wave_shift<DPP_WAVE_SHR1>(top[3][r]);
                    Rc[0][CPL][r] += top[0][r];
                    Rc[1][CPL][r] += top[1][r];
                    Rn[0][CPL][r] += top[2][r];
                    Rn[1][CPL][r] += top[3][r];
#pragma unroll
                    for (int q = 0; q < 4; ++q) top_out[q][r] = top[q][r];
                }
            }
        }
        if (DO_U) {
            // lateral: this wave's partial of node (i+1, j) goes to the wave on its right
#pragma unroll
            for (int c = 0; c < CPL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) xch[par][w][r][c][lane] = Rc[1][c][r];
            if (top_lane && top_c == CPL) {
#pragma unroll
                for (int r = 0; r < 3; ++r) xtop[par][w][r] = Rc[1][CPL][r];
            }
            // radial between the waves of a column: the top lane's new top-layer
            // partials go to lane 0 of the wave above
            if (RS > 1 && h < RS - 1 && lane == 63) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < 3; ++r) rxs[par][w][q][r] = row_cells ? top_out[q][r] : T(0);
            }
        }
        if (DO_B && row_cells) {
            // radial reduction of the coarse partials to one value per coarse layer
            if (CPL == 1) {
                // lanes 2K' and 2K'+1 share coarse layers K', K'+1
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) cp[q][s2] += wave_shift<DPP_WAVE_SHL1>(cp[q][s2]);
                // the even lane's layer K'+1 part goes to the next even lane
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T t = wave_shift<DPP_WAVE_SHR1>(wave_shift<DPP_WAVE_SHR1>(cp[q][1]));
                    if ((lane & 1) == 0) {
                        bsl[par][w + PADW][q][lane >> 1] = cp[q][0] + t;
                        if (lane == 62) bsl[par][w + PADW][q][32] = cp[q][1];
                    }
                }
            } else {
                // lane l covers coarse layers CPL/2*l .. CPL/2*l + CPL/2
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T t = wave_shift<DPP_WAVE_SHR1>(cp[q][NKL - 1]);
                    const int Kb = (CPL / 2) * lane;
#pragma unroll
                    for (int s2 = 0; s2 < NKL - 1; ++s2) bsl[par][w + PADW][q][Kb + s2] = s2 == 0 ? cp[q][0] + t : cp[q][s2];
                    if (lane == 63) bsl[par][w + PADW][q][Kb + NKL - 1] = cp[q][NKL - 1];
                }
            }
        }
        if (LOAD_U && pre) {
            __builtin_amdgcn_s_waitcnt(0);   // row j+2 has landed in LDS
            if constexpr (FS) {
                project_staged(i, j + 2, sj2, wc);
                if (xw) project_staged(i0 + TI, j + 2, sj2, TI);
            }
        }
        __syncthreads();
        if (DO_U && owned) {
            const unsigned rowA = colA + (unsigned)j * ldj;
            const unsigned rowB = colB + (unsigned)j * ldj;
            const bool seamL = (wc == 0) && (i0 > 0);
            const bool rxin = RS > 1 && h > 0 && lane == 0;   // layer 0 also gets the wave below
            const bool seamR = (i0 + TI < m);
#pragma unroll
            for (int c = 0; c < NL; ++c) {
                const int k = kk[c];
                bool live = false, seamK = false;
                if (top_lane && c == top_c) {
                    live = true;
                    seamK = kcend < n;                  // range top: the next range adds the rest
                } else if (c < CPL && k < kend) {
                    live = true;
                    seamK = (c == 0 && lane == 0 && h == 0 && kc0 > 0);   // range bottom
                }
                if ((a.ns_in && k == 0) || (a.ns_out && k == n)) live = false;   // rows set afterwards
                if (!live) continue;
                T v[3], vb[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    v[r] = Rc[0][c][r];
                    vb[r] = Rc[1][c][r];
                    if (wc > 0) v[r] += c < CPL ? xch[par][w - RS][r][c][lane] : xtop[par][w - RS][r];
                    if (c == 0 && rxin) {
                        v[r] += rxs[par][w - 1][0][r];
                        if (wc > 0) v[r] += rxs[par][w - RS - 1][1][r];
                        vb[r] += rxs[par][w - 1][1][r];
                    }
                }
                const bool seam = seamL || seamK;
                const unsigned oa = rowA + (unsigned)k;
                // node column i0 + TI: complete only on the diamond edge
                const bool s2 = seamR || seamK;
                const unsigned ob = rowB + (unsigned)k;
                if constexpr (DO_B) {
                    // full-operator kernels: one seam branch per node (measured 1-2 % faster
                    // there, 2 % slower in the viscous-only FP32 kernel)
                    T* const ys[3] = {a.y0, a.y1, a.y2};
                    emit3(ys, oa, v, seam);
                    if (xw) emit3(ys, ob, vb, s2);
                } else {
                    emit(a.y0, oa, v[0], seam);
                    emit(a.y1, oa, v[1], seam);
                    emit(a.y2, oa, v[2], seam);
                    if (xw) {
                        emit(a.y0, ob, vb[0], s2);
                        emit(a.y1, ob, vb[1], s2);
                        emit(a.y2, ob, vb[2], s2);
                    }
                }
            }
        }
        if (DO_U && RS > 1 && h > 0 && lane == 0 && row_cells) {
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                Rn[0][0][r] += rxs[par][w - 1][2][r];
                Rn[1][0][r] += rxs[par][w - 1][3][r];
            }
        }
        if (DO_B && row_cells) {
            // owner threads add the (up to four) waves touching each coarse node, in
            // a fixed order, into the open rows J (corners 0, 1) and J+1 (corners 2, 3)
            if (owner) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // columns 2 (il - (q&1)) and the next one, stretch hk (and hk - 1 at
                    // its bottom layer), in slots shifted by PADW
                    const int ws = (2 * (il - (q & 1))) * RS + hk + PADW;
                    T v = bsl[par][ws][q][klo] + bsl[par][ws + RS][q][klo];
                    if (below) v += bsl[par][ws - 1][q][NKC - 1] + bsl[par][ws + RS - 1][q][NKC - 1];
                    if (q < 2) pacc0 += v; else pacc1 += v;
                }
            }
            if (j & 1) {
                // coarse row J is complete (the one below the band's first row, from
                // the halo rows, belongs to the band below)
                if (own_ok && J >= (j0 >> 1)) emit(a.yp, own_off + (unsigned)J * pldj, pacc0, own_seam);
                pacc0 = pacc1;
                pacc1 = T(0);
            }
        }
        if (pre) {
            const int s = sj;
            sj = sj1;
            sj1 = sj2;
            sj2 = s;
        }
    };
    // (two rows per trip with the register sets swapped instead of copied costs the
    // compiler 20-40 more registers per lane)
    T Rs[2][NL][3];
    RowIn rin2;
    for (int j = jfirst; j <= jlast; ++j) {
        step(j, Rc, Rs, rin, rin2);
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int c = 0; c < NL; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) Rc[q][c][r] = Rs[q][c][r];
        rin = rin2;
    }
    if (DO_B && last_band) {
        // the coarse row above the last cell row (on other bands, the next band's)
        const int J = (jlast_cell >> 1) + 1;
        if (own_ok && J <= mc) emit(a.yp, own_off + (unsigned)J * pldj, pacc0, own_seam);
    }
}

// The passes before the band kernel in one launch: y_p = 0 (np values, when the
// divergence block is applied), then zeros at the node values that receive two
// partial sums (node columns on tile seams, node layers on radial-range seams).
template <typename T>
__global__ void pre_apply_kernel(T* yp, long long np, T* y0, T* y1, T* y2, int m, int n, int TI, int KC,
                                 int nchunk, long long nz, SlotBatch sb) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long so = slot_off(sb);
    if (t < np) {
        at_slot(yp, so)[t] = T(0);
        return;
    }
    t -= np;
    if (t >= nz) return;
    y0 = at_slot(y0, so);
    y1 = at_slot(y1, so);
    y2 = at_slot(y2, so);
    const int nseam_i = m / TI - 1;
    const long long n1 = n + 1;
    const long long ncol = (long long)10 * nseam_i * (m + 1);
    const long long ldi = (long long)(m + 1) * n1;
    long long idx;
    if (t < ncol * n1) {
        const int k = (int)(t % n1);
        long long r = t / n1;
        const int jrow = (int)(r % (m + 1));
        r /= (m + 1);
        const int s = (int)(r % nseam_i);
        const int d = (int)(r / nseam_i);
        idx = ((long long)d * (m + 1) + (long long)(s + 1) * TI) * ldi + (long long)jrow * n1 + k;
    } else {
        t -= ncol * n1;
        const long long nlat = (long long)10 * (m + 1) * (m + 1);
        idx = (t % nlat) * n1 + (long long)(t / nlat + 1) * KC;
    }
    y0[idx] = T(0);
    y1[idx] = T(0);
    y2[idx] = T(0);
}

// The passes after the band kernel in one launch (disjoint writes, any order):
//  1. the diamond-interface sum of the velocity copies (groups x layers; layers
//     of no-slip spheres are left to part 2; on a free-slip sphere the sum is
//     followed by the boundary row y = P y + N u, P = I - rhat rhat^T, N = rhat rhat^T),
//  2. the boundary rows of every lateral slot at layers 0 and n: no slip y = u
//     (viscous block present) or 0; free slip y = P y + N u (N u with the viscous
//     block only) at slots outside duplicate groups (part 1 does the others),
//  3. the interface sum of the pressure copies.
struct PostArgs {
    int ngu, n1u;                       // velocity groups, layers
    const int* gpu;
    const int* gsu;
    long long nlat_u;                   // lateral slots (boundary part), 0: none
    int ngp, n1p;                       // pressure groups, layers (0 groups: none)
    const int* gpp;
    const int* gsp;
    int ns_in, ns_out;                  // no slip on the inner / outer sphere
    int fs;                             // free slip: bit 0 inner, bit 1 outer
    const double* inv_mult;             // [lateral slots]: 1 / copies of the node
};

// y = P y + N u at one free-slip node, rhat from the unit vector table
template <typename T>
__device__ __forceinline__ void freeslip_row(T (&y)[3], const T (&u)[3], const T* __restrict__ rh, bool with_u) {
    const T n0 = rh[0], n1 = rh[1], n2 = rh[2];
    const T dy = n0 * y[0] + n1 * y[1] + n2 * y[2];
    const T du = with_u ? n0 * u[0] + n1 * u[1] + n2 * u[2] : T(0);
    y[0] += (du - dy) * n0;
    y[1] += (du - dy) * n1;
    y[2] += (du - dy) * n2;
}

template <typename T>
__global__ void post_apply_kernel(PostArgs q, T* y0, T* y1, T* y2, const T* __restrict__ u0,
                                  const T* __restrict__ u1, const T* __restrict__ u2, T* yp,
                                  const T* __restrict__ unit, SlotBatch sb) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long so = slot_off(sb);
    const long long r1 = (long long)q.ngu * q.n1u, r2 = 2 * q.nlat_u, r3 = (long long)q.ngp * q.n1p;
    const int ktop = q.n1u - 1;
    if (t < r1) {
        const int g = (int)(t / q.n1u), k = (int)(t % q.n1u);
        if ((q.ns_in && k == 0) || (q.ns_out && k == ktop)) return;
        const bool fs = ((q.fs & 1) && k == 0) || ((q.fs & 2) && k == ktop);
        const int s0 = q.gpu[g], s1 = q.gpu[g + 1];
        T* ys[3] = {at_slot(y0, so), at_slot(y1, so), at_slot(y2, so)};
        T acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T* f = ys[c];
            acc[c] = f[(long long)q.gsu[s0] * q.n1u + k];
            for (int s = s0 + 1; s < s1; ++s) acc[c] += f[(long long)q.gsu[s] * q.n1u + k];
        }
        if (fs) {
            const long long i0 = (long long)q.gsu[s0] * q.n1u + k;
            const T* us[3] = {at_slot(u0, so), at_slot(u1, so), at_slot(u2, so)};
            T uu[3] = {T(0), T(0), T(0)};
            if (us[0])
                for (int c = 0; c < 3; ++c) uu[c] = us[c][i0];
            freeslip_row(acc, uu, unit + 3LL * q.gsu[s0], us[0] != nullptr);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
            for (int s = s0; s < s1; ++s) ys[c][(long long)q.gsu[s] * q.n1u + k] = acc[c];
        return;
    }
    t -= r1;
    if (t < r2) {
        const long long slot = t >> 1;
        const bool top = t & 1;
        const bool fs = top ? (q.fs & 2) : (q.fs & 1);
        const bool ns = top ? q.ns_out : q.ns_in;
        const long long idx = slot * q.n1u + (top ? ktop : 0);
        const T* us[3] = {at_slot(u0, so), at_slot(u1, so), at_slot(u2, so)};
        T* ys[3] = {at_slot(y0, so), at_slot(y1, so), at_slot(y2, so)};
        if (fs) {
            if (q.inv_mult[slot] < 1.0) return;     // a duplicate group: part 1
            T y[3] = {ys[0][idx], ys[1][idx], ys[2][idx]};
            T uu[3] = {T(0), T(0), T(0)};
            if (us[0])
                for (int c = 0; c < 3; ++c) uu[c] = us[c][idx];
            freeslip_row(y, uu, unit + 3 * slot, us[0] != nullptr);
#pragma unroll
            for (int c = 0; c < 3; ++c) ys[c][idx] = y[c];
        } else if (ns) {
#pragma unroll
            for (int c = 0; c < 3; ++c) ys[c][idx] = us[c] ? us[c][idx] : T(0);
        }
        return;
    }
    t -= r2;
    if (t < r3) {
        const int g = (int)(t / q.n1p), k = (int)(t % q.n1p);
        const int s0 = q.gpp[g], s1 = q.gpp[g + 1];
        T* f = at_slot(yp, so);
        T acc = f[(long long)q.gsp[s0] * q.n1p + k];
        for (int s = s0 + 1; s < s1; ++s) acc += f[(long long)q.gsp[s] * q.n1p + k];
        for (int s = s0; s < s1; ++s) f[(long long)q.gsp[s] * q.n1p + k] = acc;
    }
}

inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Band count of a launch.  The workgroups run in rounds of the chip's resident
// capacity (slots), all bands of a round about equally long, so a launch takes
// about rounds x (band rows + halo row + start-up) row steps, the last round set
// by the longest band; the start-up (ring fill, first loads) is about START_ROWS
// row steps.  Bands have at least four rows, two on the small levels (m <= 16), whose
// launches are latency-bound and fill a fraction of the chip.
constexpr double START_ROWS = 2.0;
inline int choose_bands(int m, long long cols, long long slots) {
    if (m < 4) return 1;
    int best = 1;
    double best_cost = 1e300;
    for (int nb = 1; nb <= (m <= 16 ? m / 2 : m / 4); ++nb) {
        const long long rounds = (cols * nb + slots - 1) / slots;
        const double mean = (double)m / nb, longest = 2.0 * ((m / 2 + nb - 1) / nb);
        const double cost = (rounds - 1) * (mean + 1 + START_ROWS) + (longest + 1 + START_ROWS);
        if (cost < best_cost * (1 - 1e-9)) {
            best_cost = cost;
            best = nb;
        }
    }
    return best;
}

// the solver's combinations (A, B^T, K, each viscous one also with hourglass
// control) have a batched form; the others run one slot at a time
template <typename T, int RS, int CPL, int WG, bool A, bool BT, bool B, bool HG, bool FS, bool TALA = false,
          bool TWOPT = false>
void launch_band_t(const tng_ctx* ctx, BandArgs<T> args, const SlotBatch& sb, int* bands_out) {
    constexpr bool BATCHABLE = !FS && !TALA && !TWOPT && ((A && !BT && !B) || (!A && BT && !B) || (A && BT && B));
    const int block = args.TI * RS * 64;
    const bool batched = sb.nb > 1;
    if (ctx->apply_bands > 0) {
        args.nband = std::max(1, std::min(ctx->apply_bands, std::max(1, args.m / 2)));
    } else {
        // resident workgroups per CU of this kernel at this block size, asked once
        static std::atomic<int> resident[2][TIC + 1];   // per instantiation (one kernel each)
        std::atomic<int>& rc = resident[batched ? 1 : 0][block / 64];
        int per_cu = rc.load(std::memory_order_relaxed);
        if (per_cu == 0) {
            if (batched)
                TNG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, stokes_band_kernel<T, RS, CPL, A, BT, B, HG, BATCHABLE, WG, FS, TALA, TWOPT>, block, 0));
            else
                TNG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, stokes_band_kernel<T, RS, CPL, A, BT, B, HG, false, WG, FS, TALA, TWOPT>, block, 0));
            per_cu = std::max(1, per_cu);
            rc.store(per_cu, std::memory_order_relaxed);
        }
        args.nband = choose_bands(args.m, 10LL * args.ntile * args.nchunk * sb.nb, (long long)per_cu * ctx->n_cu);
    }
    if (bands_out != nullptr) {   // layout query: report the band count, launch nothing
        *bands_out = args.nband;
        return;
    }
    const long long nb = 10LL * args.ntile * args.nband * args.nchunk;
    char detail[64] = {0};
    if (ctx->profile) {
        const char* ops = A ? (BT ? (B ? "K" : "A+BT") : (B ? "A+B" : "A")) : (BT ? (B ? "BT+B" : "BT") : "B");
        std::snprintf(detail, sizeof(detail), "%s/%s%s%s%s%s/%dx%d/b%d%s", std::is_same<T, double>::value ? "f64" : "f32",
                      ops, HG ? "+HG" : "", FS ? "+FS" : "", TALA ? "+TALA" : "", TWOPT ? "+2PT" : "", args.m,
                      args.n, args.nband, sb.nb > 1 ? "/batch" : "");
    }
    ScopedKernelTimer timer(ctx, "stokes_apply", detail);
    if (sb.nb == 1)   // a single slot is always the reference slot (offset 0)
        stokes_band_kernel<T, RS, CPL, A, BT, B, HG, false, WG, FS, TALA, TWOPT>
            <<<(unsigned)nb, args.TI * RS * 64, 0, ctx->stream>>>(args, sb);
    else if constexpr (BATCHABLE)
        stokes_band_kernel<T, RS, CPL, A, BT, B, HG, true, WG, false, false>
            <<<dim3((unsigned)nb, 1, (unsigned)sb.nb), args.TI * RS * 64, 0, ctx->stream>>>(args, sb);
    else
        throw Error(TNG_E_STATE, "this operator combination has no batched form");
    TNG_HIP(hipGetLastError());
}

// key: bit 0 A, bit 1 B^T, bit 2 B, bit 3 hourglass control (with A only), bit 4
// free slip (the full operator and single blocks without hourglass control)
template <typename T, int RS, int CPL, int WG>
void launch_band_ops(const tng_ctx* ctx, const BandArgs<T>& args, const SlotBatch& sb, int key, int* bands_out) {
    switch (key) {
        case 1: launch_band_t<T, RS, CPL, WG, true, false, false, false, false>(ctx, args, sb, bands_out); break;
        case 2: launch_band_t<T, RS, CPL, WG, false, true, false, false, false>(ctx, args, sb, bands_out); break;
        case 3: launch_band_t<T, RS, CPL, WG, true, true, false, false, false>(ctx, args, sb, bands_out); break;
        case 4: launch_band_t<T, RS, CPL, WG, false, false, true, false, false>(ctx, args, sb, bands_out); break;
        case 5: launch_band_t<T, RS, CPL, WG, true, false, true, false, false>(ctx, args, sb, bands_out); break;
        case 6: launch_band_t<T, RS, CPL, WG, false, true, true, false, false>(ctx, args, sb, bands_out); break;
        case 7: launch_band_t<T, RS, CPL, WG, true, true, true, false, false>(ctx, args, sb, bands_out); break;
        case 9: launch_band_t<T, RS, CPL, WG, true, false, false, true, false>(ctx, args, sb, bands_out); break;
        case 11: launch_band_t<T, RS, CPL, WG, true, true, false, true, false>(ctx, args, sb, bands_out); break;
        case 13: launch_band_t<T, RS, CPL, WG, true, false, true, true, false>(ctx, args, sb, bands_out); break;
        case 15: launch_band_t<T, RS, CPL, WG, true, true, true, true, false>(ctx, args, sb, bands_out); break;
        case 16 | 1: launch_band_t<T, RS, CPL, WG, true, false, false, false, true>(ctx, args, sb, bands_out); break;
        case 16 | 4: launch_band_t<T, RS, CPL, WG, false, false, true, false, true>(ctx, args, sb, bands_out); break;
        case 16 | 7: launch_band_t<T, RS, CPL, WG, true, true, true, false, true>(ctx, args, sb, bands_out); break;
        case 128 | 1: launch_band_t<T, RS, CPL, WG, true, false, false, false, false, false, true>(ctx, args, sb, bands_out); break;
        case 128 | 3: launch_band_t<T, RS, CPL, WG, true, true, false, false, false, false, true>(ctx, args, sb, bands_out); break;
        case 128 | 7: launch_band_t<T, RS, CPL, WG, true, true, true, false, false, false, true>(ctx, args, sb, bands_out); break;
        case 64 | 4: launch_band_t<T, RS, CPL, WG, false, false, true, false, false, true>(ctx, args, sb, bands_out); break;
        case 64 | 7: launch_band_t<T, RS, CPL, WG, true, true, true, false, false, true>(ctx, args, sb, bands_out); break;
        case 16 | 64 | 4: launch_band_t<T, RS, CPL, WG, false, false, true, false, true, true>(ctx, args, sb, bands_out); break;
        case 16 | 64 | 7: launch_band_t<T, RS, CPL, WG, true, true, true, false, true, true>(ctx, args, sb, bands_out); break;
        case 16 | 2:   // B^T reads no velocity: its free-slip rows are the post pass's projection
            launch_band_t<T, RS, CPL, WG, false, true, false, false, false>(ctx, args, sb, bands_out);
            break;
        default:
            throw Error(TNG_E_INVAL, "this operator combination has no free-slip, compressible or two-point form "
                                     "(free slip: A, B^T, B or the full operator; TALA: B or the full operator, also "
                                     "with free slip; two-point rule: A, A+B^T or the full operator; none with "
                                     "hourglass control)");
    }
}

// layout != nullptr: fill the decomposition the launch would use (see
// tng_stokes_apply_layout) and launch nothing.
template <typename T>
void band_apply(const tng_ctx* ctx, const Level& L, const Level* Lp, unsigned flags, double hg_alpha,
                const void* eta, const void* const u[3], const void* p, void* const yu[3],
                void* yp, int* layout = nullptr, bool raw = false) {
    const bool doA = flags & TNG_OP_A, doBT = flags & TNG_OP_BT, doB = flags & TNG_OP_B;
    const bool is64 = std::is_same<T, double>::value;
    // the kernel addresses every field by 32-bit byte offsets
    TNG_REQUIRE((double)std::max(L.node_slots(), 2 * L.cells()) * sizeof(T) < 4294967296.0,
                "operator apply: a field of this level reaches 4 GiB");
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
    // cells per lane: enough for a radial stretch of 64 lanes within the
    // register budget (two or more FP64 cells per lane spill); a column longer
    // than one stretch is split among RS waves of the same workgroup (RS
    // columns fewer per workgroup), and only columns longer than RS stretches
    // into workgroup ranges with seams, which cost far more than the split
    int cpl = (L.n + 63) / 64;
    const int cpl_max = is64 ? 1 : 2;
    cpl = cpl <= 1 ? 1 : 2;
    if (cpl > cpl_max) cpl = cpl_max;
    // two cells per lane need at least four columns per workgroup, so that
    // every coarse node of the divergence has one owner thread
    if (std::min(TIC, L.m) < 4) cpl = 1;
    const int stretches = (L.n + 64 * cpl - 1) / (64 * cpl);
    const int rs_max = is64 ? 4 : 2;
    int rs = stretches >= 3 ? 4 : (stretches >= 2 ? 2 : 1);
    if (rs > rs_max) rs = rs_max;
    if (L.m < TIC / rs) rs = 1;                     // the split needs full-width tiles
    // Workgroup width (measured at (128,128)/(256,256)): 4 waves for FP64 columns of up to two
    // stretches (FP64 K 0.90 -> 0.82 ms, A 0.60 -> 0.53 ms) and for the FP32 full operator on
    // one-stretch columns (0.386 -> 0.364 ms): more workgroups per CU (FP32 K: 3 of 52 KB LDS
    // and 135 VGPRs instead of 1 of 90 KB), shorter barriers; 8 waves elsewhere, where narrower
    // tiles cost more in shared edge columns than they gain (FP32 A at (256,256) 2.08 -> 3.76 ms).
    const int wg = ((is64 && rs <= 2) || (!is64 && rs == 1 && doA && doBT && doB)) ? 4 : 8;
    a.TI = std::min(wg / rs, L.m);
    a.KC = rs * 64 * cpl;                           // radial range of a workgroup
    a.ntile = L.m / a.TI;
    a.nchunk = (L.n + a.KC - 1) / a.KC;
    a.nband = 1;   // chosen per kernel at launch
    a.r_in = T(L.r_in);
    a.dr = T(L.dr());
    a.fs = ((flags & TNG_OP_FREESLIP_INNER) ? 1 : 0) | ((flags & TNG_OP_FREESLIP_OUTER) ? 2 : 0);
    a.ns_in = ((flags & TNG_OP_DIRICHLET) && !(a.fs & 1)) ? 1 : 0;
    a.ns_out = ((flags & TNG_OP_DIRICHLET) && !(a.fs & 2)) ? 1 : 0;
    a.unit = is64 ? reinterpret_cast<const T*>(L.unit64.p) : reinterpret_cast<const T*>(L.unit32.p);
    const bool doHG = doA && hg_alpha != 0.0;
    a.hg = T(hg_alpha * (5.0 / 81.0));
    const SlotBatch sb = launch_batch();
    const unsigned nbz = (unsigned)sb.nb;
    const bool tala = (flags & TNG_OP_TALA) != 0;
    if (tala) {
        TNG_REQUIRE(L.rho64.p != nullptr, "TNG_OP_TALA needs the mesh's reference density (tng_mesh_set_density)");
        a.rho = is64 ? reinterpret_cast<const T*>(L.rho64.p) : reinterpret_cast<const T*>(L.rho32.p);
    }
    const bool twopt = doA && (flags & TNG_OP_TWOPOINT) != 0;
    const int key = (doA ? 1 : 0) | (doBT ? 2 : 0) | (doB ? 4 : 0) | (doHG ? 8 : 0) | (a.fs ? 16 : 0) |
                    (tala && doB ? 64 : 0) | (twopt ? 128 : 0);
    auto dispatch = [&](int* bands_out) {
        if constexpr (std::is_same<T, double>::value) {
            if (rs == 1)
                launch_band_ops<T, 1, 1, 4>(ctx, a, sb, key, bands_out);
            else if (rs == 2)
                launch_band_ops<T, 2, 1, 4>(ctx, a, sb, key, bands_out);
            else
                launch_band_ops<T, 4, 1, 8>(ctx, a, sb, key, bands_out);
        } else {
            // FP32 splits only two-cell stretches (one-cell columns fit one stretch)
            if (cpl == 1)
                wg == 4 ? launch_band_ops<T, 1, 1, 4>(ctx, a, sb, key, bands_out)
                        : launch_band_ops<T, 1, 1, 8>(ctx, a, sb, key, bands_out);
            else if (rs == 1)
                wg == 4 ? launch_band_ops<T, 1, 2, 4>(ctx, a, sb, key, bands_out)
                        : launch_band_ops<T, 1, 2, 8>(ctx, a, sb, key, bands_out);
            else
                launch_band_ops<T, 2, 2, 8>(ctx, a, sb, key, bands_out);
        }
    };
    if (layout != nullptr) {
        int bands = 1;
        dispatch(&bands);
        layout[0] = a.TI;
        layout[1] = rs;
        layout[2] = cpl;
        layout[3] = wg;
        layout[4] = a.ntile;
        layout[5] = bands;
        layout[6] = a.nchunk;
        layout[7] = a.KC;
        return;
    }
    {
        // y_p = 0 and the seam zeroing, one launch
        const long long np = doB ? Lp->node_slots() : 0;
        const long long nz = ((doA || doBT) && (a.ntile > 1 || a.nchunk > 1))
                                 ? 10LL * (a.ntile - 1) * (L.m + 1) * (L.n + 1) +
                                       10LL * (L.m + 1) * (L.m + 1) * (a.nchunk - 1)
                                 : 0;
        if (np + nz > 0) {
            pre_apply_kernel<T><<<dim3(nblocks(np + nz, 256), 1, nbz), 256, 0, ctx->stream>>>(
                a.yp, np, a.y0, a.y1, a.y2, L.m, L.n, a.TI, a.KC, a.nchunk, nz, sb);
            TNG_HIP(hipGetLastError());
        }
    }
    dispatch(nullptr);
    if (raw) return;   // the caller completes duplicates and Dirichlet rows
    // interface sums and Dirichlet rows (identity rows belong to the viscous block;
    // without it the rows are zero), one launch
    PostArgs q{};
    if (doA || doBT) {
        q.ngu = L.n_groups;
        q.gpu = L.grp_ptr.p;
        q.gsu = L.grp_slot.p;
        q.nlat_u = (a.ns_in || a.ns_out || a.fs) ? L.lat_slots() : 0;
        q.ns_in = a.ns_in;
        q.ns_out = a.ns_out;
        q.fs = a.fs;
        q.inv_mult = L.inv_mult64.p;
    }
    q.n1u = L.n + 1;
    if (doB) {
        q.ngp = Lp->n_groups;
        q.n1p = Lp->n + 1;
        q.gpp = Lp->grp_ptr.p;
        q.gsp = Lp->grp_slot.p;
    }
    const long long npost = (long long)q.ngu * q.n1u + 2 * q.nlat_u + (long long)q.ngp * q.n1p;
    if (npost > 0) {
        const T* ud[3] = {nullptr, nullptr, nullptr};
        if (doA && u)
            for (int c = 0; c < 3; ++c) ud[c] = static_cast<const T*>(u[c]);
        post_apply_kernel<T><<<dim3(nblocks(npost, 256), 1, nbz), 256, 0, ctx->stream>>>(
            q, a.y0, a.y1, a.y2, ud[0], ud[1], ud[2], a.yp, a.unit, sb);
        TNG_HIP(hipGetLastError());
    }
}

}  // namespace

void launch_stokes_apply(const tng_ctx* ctx, const Level& L, const Level* Lp, tng_prec prec,
                         unsigned flags, double hg_alpha, const void* eta, const void* const u[3], const void* p,
                         void* const yu[3], void* yp) {
    if (prec == TNG_F64)
        band_apply<double>(ctx, L, Lp, flags, hg_alpha, eta, u, p, yu, yp);
    else
        band_apply<float>(ctx, L, Lp, flags, hg_alpha, eta, u, p, yu, yp);
}

void launch_stokes_apply_raw(const tng_ctx* ctx, const Level& L, tng_prec prec, unsigned flags, double hg_alpha,
                             const void* eta, const void* const u[3], void* const yu[3]) {
    TNG_REQUIRE(!(flags & (TNG_OP_BT | TNG_OP_B | TNG_OP_FREESLIP_INNER | TNG_OP_FREESLIP_OUTER)),
                "raw apply: the viscous block with no-slip rows only");
    if (prec == TNG_F64)
        band_apply<double>(ctx, L, nullptr, flags, hg_alpha, eta, u, nullptr, yu, nullptr, nullptr, true);
    else
        band_apply<float>(ctx, L, nullptr, flags, hg_alpha, eta, u, nullptr, yu, nullptr, nullptr, true);
}

void stokes_apply_layout(const tng_ctx* ctx, const Level& L, const Level* Lp, tng_prec prec, unsigned flags,
                         double hg_alpha, int out[8]) {
    if (prec == TNG_F64)
        band_apply<double>(ctx, L, Lp, flags, hg_alpha, nullptr, nullptr, nullptr, nullptr, nullptr, out);
    else
        band_apply<float>(ctx, L, Lp, flags, hg_alpha, nullptr, nullptr, nullptr, nullptr, nullptr, out);
}

}  // namespace tng
