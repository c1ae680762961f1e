// Field kernels around the operator: per-wedge viscosity from nodal
// temperature, viscosity coarsening for the multigrid hierarchy.
#include "tng_internal.hpp"

namespace tng {
namespace {

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// eta_e = exp(-E Tbar_e + F (1 - r_m)), Tbar_e = value of the W1 interpolant
// of T at q_c = mean of the wedge's six nodal temperatures (the viscosity at
// the quadrature point, Sec. 4 eq:oneptenergy).
template <typename T>
__global__ void eta_from_T_kernel(const T* __restrict__ Tn, T* __restrict__ eta, int m, int n,
                                  T r_in, T dr, T E, T F, long long ncells) {
    const long long cid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cid >= ncells) return;
    const int k = (int)(cid % n);
    long long t = cid / n;
    const int j = (int)(t % m);
    t /= m;
    const int i = (int)(t % m);
    const int d = (int)(t / m);
    const long long ldj = n + 1, ldi = (long long)(m + 1) * ldj, ldd = (long long)(m + 1) * ldi;
    const long long b00 = d * ldd + i * ldi + j * ldj + k;
    const T t00 = Tn[b00] + Tn[b00 + 1];
    const T t10 = Tn[b00 + ldi] + Tn[b00 + ldi + 1];
    const T t01 = Tn[b00 + ldj] + Tn[b00 + ldj + 1];
    const T t11 = Tn[b00 + ldi + ldj] + Tn[b00 + ldi + ldj + 1];
    const T rm = r_in + (T(k) + T(0.5)) * dr;
    const T depth = F * (T(1) - rm);
    const T sixth = T(1.0 / 6.0);
    eta[2 * cid + 0] = exp(-E * (t00 + t10 + t01) * sixth + depth);
    eta[2 * cid + 1] = exp(-E * (t11 + t01 + t10) * sixth + depth);
}

// Coarse wedge viscosity = mean of its eight children: four lateral child
// triangles (three corner triangles and the centre one) times two layers.
// Coarse wedge 0 of cell (I,J) holds fine (2I,2J,w0), (2I+1,2J,w0),
// (2I,2J+1,w0) and the centre (2I,2J,w1); coarse wedge 1 holds
// (2I+1,2J+1,w1), (2I,2J+1,w1), (2I+1,2J,w1) and the centre (2I+1,2J+1,w0).
template <typename T>
__global__ void eta_coarsen_kernel(const T* __restrict__ ef, T* __restrict__ ec, int mc, int nc,
                                   long long nccells) {
    const long long cid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (cid >= nccells) return;
    const int K = (int)(cid % nc);
    long long t = cid / nc;
    const int J = (int)(t % mc);
    t /= mc;
    const int I = (int)(t % mc);
    const int d = (int)(t / mc);
    const int mf = 2 * mc, nf = 2 * nc;
    auto fw = [&](int a, int b, int c, int w) {
        return ef[((((long long)d * mf + 2 * I + a) * mf + 2 * J + b) * nf + 2 * K + c) * 2 + w];
    };
    T s0 = 0, s1 = 0;
    for (int c = 0; c < 2; ++c) {
        s0 += fw(0, 0, c, 0) + fw(1, 0, c, 0) + fw(0, 1, c, 0) + fw(0, 0, c, 1);
        s1 += fw(1, 1, c, 1) + fw(0, 1, c, 1) + fw(1, 0, c, 1) + fw(1, 1, c, 0);
    }
    ec[2 * cid + 0] = s0 * T(0.125);
    ec[2 * cid + 1] = s1 * T(0.125);
}

}  // namespace

void launch_eta_from_T(const tng_ctx* ctx, const Level& L, tng_prec prec, const void* Tn, void* eta,
                       double E, double F) {
    const long long nc = L.cells();
    if (prec == TNG_F64)
        eta_from_T_kernel<double><<<nblk(nc, 256), 256, 0, ctx->stream>>>(
            (const double*)Tn, (double*)eta, L.m, L.n, L.r_in, L.dr(), E, F, nc);
    else
        eta_from_T_kernel<float><<<nblk(nc, 256), 256, 0, ctx->stream>>>(
            (const float*)Tn, (float*)eta, L.m, L.n, (float)L.r_in, (float)L.dr(), (float)E,
            (float)F, nc);
    TNG_HIP(hipGetLastError());
}

void launch_eta_coarsen(const tng_ctx* ctx, const Level& Lc, tng_prec prec, const void* ef,
                        void* ec) {
    const long long nc = Lc.cells();
    if (prec == TNG_F64)
        eta_coarsen_kernel<double><<<nblk(nc, 256), 256, 0, ctx->stream>>>(
            (const double*)ef, (double*)ec, Lc.m, Lc.n, nc);
    else
        eta_coarsen_kernel<float><<<nblk(nc, 256), 256, 0, ctx->stream>>>(
            (const float*)ef, (float*)ec, Lc.m, Lc.n, nc);
    TNG_HIP(hipGetLastError());
}

}  // namespace tng
