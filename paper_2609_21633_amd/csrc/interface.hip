// Diamond-interface reduction (the one-GPU analog of the paper's post-apply
// halo exchange, Sec. 2): every node on a diamond edge is stored once per
// diamond holding it, each copy receives the partial sum of its own diamond's
// cells, and this pass adds the copies and writes the sum back to all of them,
// in a fixed order.  (The operator apply does this in its own post-pass.)
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

}  // namespace tng
