// Streaming form of the SUPG energy apply (Sec. 6 scheme list, Sec. 1 eq:energy
// in Boussinesq form, one-point rule of Sec. 4): y = E(u) T with
//   (E T)_i = sum_e V_e [ T_i / (6 dt) + grad phi_i . grad T + (1/6) ubar . grad T
//                         + tau_e (ubar . grad phi_i)(ubar . grad T) ]
// and the flow data (ubar, tau) formed from the nodal velocity on the fly, so that
// one apply reads T and u once and writes y once.
//
// Work decomposition (one diamond d): lanes run along the radius, lane l of the
// wave of stretch h holding cell k = 64 h + l of one cell column; a workgroup
// holds TC adjacent cell columns (waves) times RS radial stretches (whole
// columns) and streams along j over the cell rows of a band, which starts one
// row early (halo) so that its node rows are complete.  Each wedge is evaluated
// once: its six node contributions go to the node rows j (finished after this
// row) and j+1 (carried in registers).  Radial neighbours exchange by a DPP
// wave shift, and across the stretches and columns of the workgroup through LDS,
// in a fixed order.  The node columns shared by two tiles receive two partial
// sums, added with atomics onto memory zeroed beforehand; two partials give the
// same sum in either order, so the result does not depend on timing.
//
// Per wedge, with e0 = s1 g0, e1 = s1 g1, e2 = g2 (s1 = 1/(2 r_m)) and
// grad T = A e0 + B e1 + C e2 from nodal differences, the wedge volume's radial
// factors (V s1^2 = g9/4, V s1 = r_m g9/2, V = r_m^2 g9) turn V e_a . grad T into
// the per-column metric times (A, B, C).  The SUPG parameter
//   tau = h/(2|ubar|) (coth Pe - 1/Pe) = (h^2/4) F(Pe),  Pe = |ubar| h/2,  h = V^(1/3),
// uses F(x) = (coth x - 1/x)/x: its Taylor series in x^2 (coefficients
// 2^(2n) B_2n / (2n)!, Bernoulli numbers B_2n) for x <= 1, where the closed form
// cancels, and the closed form with coth x = (1 + e^-2x)/(1 - e^-2x) above.
#include <cstdio>
#include <type_traits>

#include "mg.hpp"
#include "tng_internal.hpp"

namespace tng {
namespace {

template <typename T>
struct EStreamArgs {
    const T* __restrict__ Tin;
    const T* __restrict__ u0;
    const T* __restrict__ u1;
    const T* __restrict__ u2;
    T* y;
    const T* __restrict__ eg;   // [10][m][m][2][EG_PER_TRI]
    int m, n;
    int ntile, nband;
    T r_in, dr, inv_dt;
};

// Taylor coefficients of F(x) = (coth x - 1/x)/x in x^2 (exact rationals)
template <typename T>
struct SupgSeries;
template <>
struct SupgSeries<double> {
    static constexpr int N = 17;   // truncation below 3e-17 relative for x <= 1
};
template <>
struct SupgSeries<float> {
    static constexpr int N = 8;    // below 7e-9 relative for x <= 1
};
__device__ __forceinline__ double supg_coef(int k) {
    constexpr double c[17] = {1.0 / 3.0,
                              -1.0 / 45.0,
                              2.0 / 945.0,
                              -1.0 / 4725.0,
                              2.0 / 93555.0,
                              -1382.0 / 638512875.0,
                              4.0 / 18243225.0,
                              -3617.0 / 162820783125.0,
                              87734.0 / 38979295480125.0,
                              -349222.0 / 1531329465290625.0,
                              310732.0 / 13447856940643125.0,
                              -472728182.0 / 201919571963756521875.0,
                              2631724.0 / 11094481976030578125.0,
                              -13571120588.0 / 564653660170076273671875.0,
                              13785346041608.0 / 5660878804669082674070015625.0,
                              -7709321041217.0 / 31245110285511170603633203125.0,
                              303257395102.0 / 12130454581433748587292890625.0};
    return c[k];
}

// hardware reciprocal (square root) estimates
__device__ __forceinline__ float hw_rsq(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double hw_rsq(double v) { return __builtin_amdgcn_rsq(v); }
__device__ __forceinline__ float hw_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double hw_rcp(double v) { return __builtin_amdgcn_rcp(v); }

// F(x) from z = x^2: the series for z <= 1 and the closed form
//   F = (x (1 + e) - (1 - e)) / (z (1 - e)),  e = exp(-2x),
// for z > 1, the reciprocal square root and the reciprocal being the hardware
// estimates refined by two Newton steps each.  FP32: the closed form only when a lane
// of the wave needs it.  FP64: both evaluated and one selected, without a branch (any
// branch here costs the FP64 kernel thirty to fifty registers, and a fourth wave per
// SIMD).
template <typename T>
__device__ __forceinline__ T supg_F(T z) {
    constexpr int N = SupgSeries<T>::N;
    const bool small = z <= T(1);
    const T zs = small ? z : T(1);
    T f = T(supg_coef(N - 1));
#pragma unroll
    for (int k = N - 2; k >= 0; --k) f = f * zs + T(supg_coef(k));
    if constexpr (std::is_same<T, float>::value)
        if (__builtin_amdgcn_ballot_w64(!small) == 0) return f;
    const T zl = small ? T(4) : z;
    T r = hw_rsq(zl);
    r = r * (T(1.5) - T(0.5) * zl * r * r);
    r = r * (T(1.5) - T(0.5) * zl * r * r);
    const T x = zl * r;
    const T e = exp(T(-2) * x);
    const T om = T(1) - e;
    const T den = zl * om;
    T q = hw_rcp(den);
    q = q * (T(2) - den * q);
    q = q * (T(2) - den * q);
    const T fl = (x * (T(1) + e) - om) * q;
    return small ? f : fl;
}

// Element at a 32-bit byte offset from a wave-uniform base: lets the compiler use the
// scalar-base addressing form (64-bit base in scalar registers, 32-bit offset per lane)
template <typename T>
__device__ __forceinline__ const T& at_bytes(const T* base, unsigned off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ T* ptr_bytes(T* base, unsigned off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int SHR1 = 0x138;   // lane l receives lane l-1; lane 0 reads zero

// One node row at the wave's two node columns (i, i+1) and the lane's two node
// layers (k, k+1): the temperatures, and (the velocity enters only through the mean
// over a wedge's six nodes) the velocity summed over both layers, of both columns
// (su) and of column i+1 alone (s1).
template <typename T, bool FLOW>
struct RowV {
    T t[2][2];
    T su[FLOW ? 3 : 1], s1[FLOW ? 3 : 1];
};

template <typename T, bool FLOW, int TC, int RS>
__global__ void __launch_bounds__(TC * RS * 64) energy_stream_kernel(EStreamArgs<T> a) {
    constexpr int NW = TC * RS;
    __shared__ T xr[2][NW][64];    // right-column node sums handed to the next column
    __shared__ T rx[2][NW][2];     // top-layer partials of lane 63 (left, right column)

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = w / RS, h = w % RS;
    int bid;
    {
        // each XCD takes a contiguous run of (tile, band) blocks
        const unsigned nbk = gridDim.x, q = nbk >> 3, r = nbk & 7, x = blockIdx.x & 7;
        bid = (int)(x * q + min(x, r) + (blockIdx.x >> 3));
    }
    const int band = bid % a.nband;
    bid /= a.nband;
    const int tile = bid % a.ntile;
    const int d = bid / a.ntile;
    const int m = a.m, n = a.n;
    const int i0 = tile * TC;
    const int TI = min(TC, m - i0);
    const bool active = c < TI;
    const int i = i0 + c;
    const int j0 = (band * m) / a.nband;
    const int j1 = ((band + 1) * m) / a.nband;
    const bool last_band = band == a.nband - 1;
    const int jfirst = j0 > 0 ? j0 - 1 : 0;
    const int jlast = last_band ? m : j1 - 1;

    const int k = 64 * h + lane;                 // the lane's cell and bottom node layer
    const bool cell = active && k < n;
    const T rm = a.r_in + (T(k) + T(0.5)) * a.dr;
    const T s1 = T(0.5) / rm;
    const T rm2 = cell ? rm * rm : T(0);
    const T r43 = cbrt(rm2 * rm2);               // rm^(4/3): h^2 = rm^(4/3) g9^(2/3)

    // byte offsets (every node field of a supported level is below 4 GiB)
    constexpr unsigned SZ = sizeof(T);
    const unsigned ldj = (n + 1) * SZ;
    const unsigned ldi = (unsigned)(m + 1) * ldj;
    const unsigned colA = ((unsigned)d * (m + 1) + i) * ldi;
    // loads stay inside the diamond's columns and the column's layers for every lane;
    // the wedge of a lane without a cell is zeroed (A = B = C = 0 and no volume)
    const unsigned colL = ((unsigned)d * (m + 1) + min(i, m - 1)) * ldi + (unsigned)min(k, n - 1) * SZ;

    auto load = [&](int jr, RowV<T, FLOW>& v) {
        const unsigned base = colL + (unsigned)jr * ldj;
#pragma unroll
        for (int ic = 0; ic < 2; ++ic) {
            v.t[ic][0] = at_bytes(a.Tin, base + ic * ldi);
            v.t[ic][1] = at_bytes(a.Tin, base + ic * ldi + SZ);
        }
        if constexpr (FLOW) {
            const T* const uu[3] = {a.u0, a.u1, a.u2};
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                const T a0 = at_bytes(uu[x], base), a1 = at_bytes(uu[x], base + SZ);
                const T b0 = at_bytes(uu[x], base + ldi), b1 = at_bytes(uu[x], base + ldi + SZ);
                v.s1[x] = b0 + b1;
                v.su[x] = (a0 + a1) + v.s1[x];
            }
        }
    };

    // the column geometry (uniform over the wave, read-only) is read through the
    // constant address space, so that it is loaded into scalar registers
    using CT = const __attribute__((address_space(4))) T;

    // mean velocity ub = us / 6 of a wedge and V tau = V (h^2/4) F(Pe) of its SUPG
    // parameter (h^2/4 = g16 rm^(4/3))
    auto flow = [&](CT* g, const T (&us)[3], T (&ub)[3]) -> T {
#pragma unroll
        for (int x = 0; x < 3; ++x) ub[x] = us[x] * T(1.0 / 6.0);
        const T hq = g[16] * r43;
        const T z = (ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]) * hq;   // Pe^2
        return (rm2 * g[15]) * hq * supg_F(z);
    };

    // one wedge from the temperatures tv[lat][layer] of its six nodes, its mean
    // velocity ub and V tau (VF); accumulates into out[lat][layer]
    auto wedge = [&](CT* g, const T (&tv)[3][2], const T (&ub)[FLOW ? 3 : 1], T VF, T* (&out)[3]) {
        T A = (tv[1][0] - tv[0][0]) + (tv[1][1] - tv[0][1]);
        T B = (tv[2][0] - tv[0][0]) + (tv[2][1] - tv[0][1]);
        T C = (tv[0][1] + tv[1][1] + tv[2][1]) - (tv[0][0] + tv[1][0] + tv[2][0]);
        if (!cell) A = B = C = T(0);
        const T V = rm2 * g[15];
        const T M = V * a.inv_dt * T(1.0 / 6.0);
        T P0 = g[9] * A + g[10] * B + rm * g[12] * C;
        T P1 = g[10] * A + g[11] * B + rm * g[13] * C;
        T P2 = rm * (g[12] * A + g[13] * B) + rm2 * g[14] * C;
        T Q = T(0);
        if constexpr (FLOW) {
            const T q0 = ub[0] * g[0] + ub[1] * g[1] + ub[2] * g[2];
            const T q1 = ub[0] * g[3] + ub[1] * g[4] + ub[2] * g[5];
            const T q2 = ub[0] * g[6] + ub[1] * g[7] + ub[2] * g[8];
            const T e0 = s1 * q0, e1 = s1 * q1;
            const T adv = A * e0 + B * e1 + C * q2;              // ubar . grad T
            const T wt = VF * adv;                                // V tau (ubar . grad T)
            P0 += wt * e0;
            P1 += wt * e1;
            P2 += wt * q2;
            Q = V * adv * T(1.0 / 6.0);
        }
        const T L0 = -(P0 + P1);
        const T Qb = Q - P2, Qt = Q + P2;
        const T lat[3] = {L0, P0, P1};
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            out[l][0] += (lat[l] + Qb) + M * tv[l][0];
            out[l][1] += (lat[l] + Qt) + M * tv[l][1];
        }
    };

    CT* gcol = (CT*)a.eg;
    const unsigned gbase = (((unsigned)d * m + i) * (unsigned)m) * EG_PER_COL;

    // node-row sums [column][layer]: R0 / R1 alternate between node rows j and j+1
    T R0[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
    T R1[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
    RowV<T, FLOW> V0, V1;
    if (active) load(jfirst, V0);

    auto step = [&](int j, const RowV<T, FLOW>& cur, RowV<T, FLOW>& nxt, T (&Rc)[2][2], T (&Rn)[2][2], int buf) {
        if (j < j1) {
            if (active) {
                load(j + 1, nxt);
                CT* g = gcol + gbase + (unsigned)j * EG_PER_COL;
                {
                    // wedge 0: lateral nodes (i, j), (i+1, j), (i, j+1)
                    T ub[FLOW ? 3 : 1], VF = T(0);
                    if constexpr (FLOW) {
                        T us[3];
#pragma unroll
                        for (int x = 0; x < 3; ++x) us[x] = cur.su[x] + (nxt.su[x] - nxt.s1[x]);
                        VF = flow(g, us, ub);
                    }
                    const T tv[3][2] = {{cur.t[0][0], cur.t[0][1]}, {cur.t[1][0], cur.t[1][1]},
                                        {nxt.t[0][0], nxt.t[0][1]}};
                    T* out[3] = {Rc[0], Rc[1], Rn[0]};
                    wedge(g, tv, ub, VF, out);
                }
                // keeps the second wedge's geometry out of registers until here
                __builtin_amdgcn_sched_barrier(0);
                {
                    // wedge 1: (i+1, j+1), (i, j+1), (i+1, j)
                    CT* g1 = g + EG_PER_TRI;
                    T ub[FLOW ? 3 : 1], VF = T(0);
                    if constexpr (FLOW) {
                        T us[3];
#pragma unroll
                        for (int x = 0; x < 3; ++x) us[x] = cur.s1[x] + nxt.su[x];
                        VF = flow(g1, us, ub);
                    }
                    const T tv[3][2] = {{nxt.t[1][0], nxt.t[1][1]}, {nxt.t[0][0], nxt.t[0][1]},
                                        {cur.t[1][0], cur.t[1][1]}};
                    T* out[3] = {Rn[1], Rn[0], Rc[1]};
                    wedge(g1, tv, ub, VF, out);
                }
            }
        }
        if (j >= j0) {
            // node row j is complete in this workgroup: radial then lateral sums
            T own[2], top63[2];
#pragma unroll
            for (int ic = 0; ic < 2; ++ic) {
                own[ic] = Rc[ic][0] + dpp_shift<SHR1>(Rc[ic][1]);
                top63[ic] = Rc[ic][1];
            }
            xr[buf][w][lane] = own[1];
            if (lane == 63) {
                rx[buf][w][0] = top63[0];
                rx[buf][w][1] = top63[1];
            }
            __syncthreads();
            if (active) {
                T left = own[0];
                if (c > 0) left += xr[buf][w - RS][lane];
                if (lane == 0 && h > 0) {
                    left += rx[buf][w - 1][0];
                    if (c > 0) left += rx[buf][w - RS - 1][1];
                }
                const unsigned row = colA + (unsigned)j * ldj;
                const bool seamL = c == 0 && i0 > 0;
                auto put = [&](unsigned off, T v, bool seam) {
                    if (seam)
                        atomicAdd(ptr_bytes(a.y, off), v);
                    else
                        *ptr_bytes(a.y, off) = v;
                };
                if (k <= n) put(row + (unsigned)k * SZ, left, seamL);
                // the column's top layer when the last stretch's last lane holds the
                // last cell (otherwise lane 0 of the stretch above, or the lane above,
                // holds layer n)
                const bool topn = lane == 63 && k + 1 == n && h == RS - 1;
                if (topn) {
                    T v = top63[0];
                    if (c > 0) v += rx[buf][w - RS][1];
                    put(row + (unsigned)n * SZ, v, seamL);
                }
                if (c == TI - 1) {
                    // the tile's right node column
                    const bool seamR = i0 + TI < m;
                    const unsigned rrow = row + ldi;
                    T right = own[1];
                    if (lane == 0 && h > 0) right += rx[buf][w - 1][1];
                    if (k <= n) put(rrow + (unsigned)k * SZ, right, seamR);
                    if (topn) put(rrow + (unsigned)n * SZ, top63[1], seamR);
                }
            }
        }
#pragma unroll
        for (int ic = 0; ic < 2; ++ic) Rc[ic][0] = Rc[ic][1] = T(0);
    };

    int buf = 0;
    for (int j = jfirst; j <= jlast; j += 2) {
        step(j, V0, V1, R0, R1, buf);
        buf ^= 1;
        if (j + 1 <= jlast) {
            step(j + 1, V1, V0, R1, R0, buf);
            buf ^= 1;
        }
    }
}

// zero the node columns shared by two tiles (i = multiples of TC inside the diamond)
template <typename T>
__global__ void zero_tile_seams_kernel(T* y, int m, int n, int TC, long long total) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const long long colsz = (long long)(m + 1) * (n + 1);
    const int nseam = (m - 1) / TC;
    const long long off = t % colsz;
    const long long r = t / colsz;
    const int s = (int)(r % nseam) + 1;
    const int d = (int)(r / nseam);
    y[((long long)d * (m + 1) + (long long)s * TC) * colsz + off] = T(0);
}

// Dirichlet temperature rows of the result: y = T on k = 0 and k = n
template <typename T>
__global__ void copy_layers_kernel(long long ncol, int n, T* y, const T* src) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * ncol) return;
    const long long idx = (t >> 1) * (n + 1) + ((t & 1) ? n : 0);
    y[idx] = src[idx];
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

template <typename T, bool FLOW, int TC, int RS>
void launch_stream(const tng_ctx* ctx, const Level& L, const EStreamArgs<T>& a0) {
    EStreamArgs<T> a = a0;
    a.ntile = (L.m + TC - 1) / TC;
    // bands of about 32 rows, at least one workgroup per CU
    int nb = std::max(1, L.m / 32);
    while (nb < L.m && 10LL * a.ntile * nb < ctx->n_cu) ++nb;
    a.nband = std::min(nb, L.m);
    const unsigned grid = (unsigned)(10 * a.ntile * a.nband);
    if (L.m > TC) {
        const long long total = 10LL * ((L.m - 1) / TC) * (L.m + 1) * (L.n + 1);
        zero_tile_seams_kernel<T><<<nblk(total, 256), 256, 0, ctx->stream>>>(a.y, L.m, L.n, TC, total);
        TNG_HIP(hipGetLastError());
    }
    char detail[48] = {0};
    if (ctx->profile)
        std::snprintf(detail, sizeof(detail), "%s/%s/%dx%d", std::is_same<T, double>::value ? "f64" : "f32",
                      FLOW ? "SUPG" : "diffusion", L.m, L.n);
    ScopedKernelTimer timer(ctx, "energy_apply", detail);
    energy_stream_kernel<T, FLOW, TC, RS><<<grid, TC * RS * 64, 0, ctx->stream>>>(a);
    TNG_HIP(hipGetLastError());
}

}  // namespace

// at most 256 radial layers (four stretches of 64 cells), node fields below 4 GiB
bool energy_stream_fits(const Level& L) { return L.n <= 256 && L.node_slots() * 8 < (1LL << 32); }

template <typename T>
void energy_apply_stream(const tng_ctx* ctx, const Level& L, const T* const u[3], double dt, const T* Tin, T* y) {
    require_unbatched("energy_apply");
    TNG_REQUIRE(energy_stream_fits(L), "energy apply: more than 256 radial layers");
    EStreamArgs<T> a{};
    a.Tin = Tin;
    if (u) {
        a.u0 = u[0];
        a.u1 = u[1];
        a.u2 = u[2];
    }
    a.y = y;
    a.eg = std::is_same<T, double>::value ? reinterpret_cast<const T*>(L.eg64.p) : reinterpret_cast<const T*>(L.eg32.p);
    a.m = L.m;
    a.n = L.n;
    a.r_in = T(L.r_in);
    a.dr = T(L.dr());
    a.inv_dt = T(1.0 / dt);
    const bool flow = u != nullptr;
    // workgroups of 16 waves: TC columns x RS stretches (four waves per SIMD fit: at
    // most 128 registers per lane)
    if (L.n <= 64) {
        if (flow)
            launch_stream<T, true, 16, 1>(ctx, L, a);
        else
            launch_stream<T, false, 16, 1>(ctx, L, a);
    } else if (L.n <= 128) {
        if (flow)
            launch_stream<T, true, 8, 2>(ctx, L, a);
        else
            launch_stream<T, false, 8, 2>(ctx, L, a);
    } else {
        if (flow)
            launch_stream<T, true, 4, 4>(ctx, L, a);
        else
            launch_stream<T, false, 4, 4>(ctx, L, a);
    }
    void* f[1] = {y};
    launch_interface(ctx, L, prec_of<T>(), 0, 1, f);
    copy_layers_kernel<T><<<nblk(2 * L.lat_slots(), 256), 256, 0, ctx->stream>>>(L.lat_slots(), L.n, y, Tin);
    TNG_HIP(hipGetLastError());
}

template void energy_apply_stream<double>(const tng_ctx*, const Level&, const double* const[3], double, const double*,
                                          double*);
template void energy_apply_stream<float>(const tng_ctx*, const Level&, const float* const[3], double, const float*,
                                         float*);

}  // namespace tng
