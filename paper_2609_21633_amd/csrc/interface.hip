// Diamond-interface reduction and Dirichlet rows (the one-GPU analog of the
// paper's post-apply halo exchange, Sec. 2): every node on a diamond edge is
// stored once per diamond holding it, each copy receives the partial sum of
// its own diamond's cells, and this pass adds the copies and writes the sum
// back to all of them, in a fixed order.
#include "batch_dev.hpp"
#include "tng_internal.hpp"

namespace tng {
namespace {

template <typename T>
__global__ void interface_kernel(int ngroups, int n1, const int* __restrict__ gptr,
                                 const int* __restrict__ gslot, int mode, int ncomp, T* f0, T* f1,
                                 T* f2, T* f3, SlotBatch sb) {
    const long long so = slot_off(sb);
    f0 = at_slot(f0, so);
    f1 = at_slot(f1, so);
    f2 = at_slot(f2, so);
    f3 = at_slot(f3, so);
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

// Dirichlet rows (layers 0 and n): y = u, or y = 0 when u is NULL.
template <typename T>
__global__ void dirichlet_copy_kernel(long long ncol, int n, const T* __restrict__ u0,
                                      const T* __restrict__ u1, const T* __restrict__ u2, T* y0,
                                      T* y1, T* y2, SlotBatch sb) {
    const long long so = slot_off(sb);
    u0 = at_slot(u0, so);
    u1 = at_slot(u1, so);
    u2 = at_slot(u2, so);
    y0 = at_slot(y0, so);
    y1 = at_slot(y1, so);
    y2 = at_slot(y2, so);
    long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= 2 * ncol) return;
    const long long col = tid >> 1;
    const long long idx = col * (n + 1) + ((tid & 1) ? n : 0);
    y0[idx] = u0 ? u0[idx] : T(0);
    y1[idx] = u1 ? u1[idx] : T(0);
    y2[idx] = u2 ? u2[idx] : T(0);
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_interface(const tng_ctx* ctx, const Level& L, tng_prec prec, int mode, int ncomp,
                      void* const f[]) {
    TNG_REQUIRE(ncomp >= 1 && ncomp <= 4, "ncomp must be 1..4");
    if (L.n_groups == 0) return;
    const long long nt = (long long)L.n_groups * (L.n + 1);
    const SlotBatch sb = launch_batch();
    const dim3 grid(blocks_for(nt, 256), 1, (unsigned)sb.nb);
    void* g[4] = {nullptr, nullptr, nullptr, nullptr};
    for (int c = 0; c < ncomp; ++c) g[c] = f[c];
    if (prec == TNG_F64)
        interface_kernel<double><<<grid, 256, 0, ctx->stream>>>(
            L.n_groups, L.n + 1, L.grp_ptr.p, L.grp_slot.p, mode, ncomp, (double*)g[0],
            (double*)g[1], (double*)g[2], (double*)g[3], sb);
    else
        interface_kernel<float><<<grid, 256, 0, ctx->stream>>>(
            L.n_groups, L.n + 1, L.grp_ptr.p, L.grp_slot.p, mode, ncomp, (float*)g[0],
            (float*)g[1], (float*)g[2], (float*)g[3], sb);
    TNG_HIP(hipGetLastError());
}

void launch_dirichlet_copy(const tng_ctx* ctx, const Level& L, tng_prec prec,
                           const void* const u[3], void* const y[3]) {
    const long long ncol = L.lat_slots();
    const SlotBatch sb = launch_batch();
    const dim3 grid(blocks_for(2 * ncol, 256), 1, (unsigned)sb.nb);
    if (prec == TNG_F64)
        dirichlet_copy_kernel<double><<<grid, 256, 0, ctx->stream>>>(
            ncol, L.n, u ? (const double*)u[0] : nullptr, u ? (const double*)u[1] : nullptr,
            u ? (const double*)u[2] : nullptr,
            (double*)y[0], (double*)y[1], (double*)y[2], sb);
    else
        dirichlet_copy_kernel<float><<<grid, 256, 0, ctx->stream>>>(
            ncol, L.n, u ? (const float*)u[0] : nullptr, u ? (const float*)u[1] : nullptr,
            u ? (const float*)u[2] : nullptr, (float*)y[0],
            (float*)y[1], (float*)y[2], sb);
    TNG_HIP(hipGetLastError());
}

}  // namespace tng
