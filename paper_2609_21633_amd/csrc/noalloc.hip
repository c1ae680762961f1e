// Chebyshev smoothing without any device allocation: the work vectors of
// tng_smooth (inverted diagonal, right-hand side, iterate, operator output,
// search direction) and the step coefficients live in one file-scope device
// array of fixed size instead of buffers allocated per call.
//
// The array is a device symbol: its name in host code is only a host-side
// stand-in, never a device address.  Its address on each device is asked
// once with hipGetSymbolAddress (tng_noalloc_register_device, called by
// tng_ctx_create with the device current) and only that address is passed
// to kernels and copies.
#include <cmath>
#include <mutex>
#include <vector>

#include "mg.hpp"
#include "tng_internal.hpp"

namespace tng {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(48) << 20;   // 48 MiB per device
constexpr int NOALLOC_MAX_DEGREE = 16;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // device ordinal -> address of `scratch` on it

struct ChebCoefs {
    double ab[2 * NOALLOC_MAX_DEGREE];
    int count;
};

// The coefficients travel as a kernel argument and are written by a kernel, so
// the call has no host-to-device copy and no memset.
__global__ void put_coefs_kernel(ChebCoefs c, double* dst) {
    const int t = threadIdx.x;
    if (t < c.count) dst[t] = c.ab[t];
}

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

template <typename T>
void smooth_noalloc_t(tng_ctx* ctx, const Level& L, const void* eta, double hg_alpha, const void* const diag[3],
                      const void* const b[3], void* const x[3], int degree, int steps, double lmin, double lmax,
                      char* base) {
    const long long ns = L.node_slots(), n3 = 3 * ns;
    const size_t vb = round256((size_t)n3 * sizeof(T));
    T* invd = reinterpret_cast<T*>(base);
    T* bb = reinterpret_cast<T*>(base + vb);
    T* xx = reinterpret_cast<T*>(base + 2 * vb);
    T* y = reinterpret_cast<T*>(base + 3 * vb);
    T* d = reinterpret_cast<T*>(base + 4 * vb);
    double* abd = reinterpret_cast<double*>(base + 5 * vb);
    hipStream_t st = ctx->stream;
    for (int c = 0; c < 3; ++c) {
        TNG_HIP(hipMemcpyAsync(invd + c * ns, diag[c], ns * sizeof(T), hipMemcpyDeviceToDevice, st));
        TNG_HIP(hipMemcpyAsync(bb + c * ns, b[c], ns * sizeof(T), hipMemcpyDeviceToDevice, st));
        TNG_HIP(hipMemcpyAsync(xx + c * ns, x[c], ns * sizeof(T), hipMemcpyDeviceToDevice, st));
    }
    vec_invert<T>(ctx, n3, invd);
    ChebCoefs cc{};
    cc.count = 2 * degree;
    chebyshev_coefficients(degree, lmin, lmax, cc.ab);
    put_coefs_kernel<<<1, 64, 0, st>>>(cc, abd);
    TNG_HIP(hipGetLastError());
    // y and d need no clearing: the first step of a Chebyshev cycle writes y
    // (the operator apply) and d (coefficient alpha_0 = 0, d not read) before
    // reading them, whatever an earlier call left in the array
    chebyshev_steps<T>(ctx, L, (const T*)eta, hg_alpha, invd, bb, xx, y, d, abd, degree, steps, false);
    for (int c = 0; c < 3; ++c)
        TNG_HIP(hipMemcpyAsync(x[c], xx + c * ns, ns * sizeof(T), hipMemcpyDeviceToDevice, st));
}

}  // namespace

// Address of the scratch array on `device` (which must be current), asked once.
void noalloc_register_device(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (device < (int)g_scratch_ptr.size() && g_scratch_ptr[device] != nullptr) return;
    void* p = nullptr;
    TNG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    TNG_REQUIRE(p != nullptr, "hipGetSymbolAddress returned NULL for the scratch array");
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    g_scratch_ptr[device] = p;
}

size_t noalloc_scratch_bytes() { return NOALLOC_SCRATCH_BYTES; }

// Bytes tng_smooth_noalloc needs on a level of ns node slots.
size_t noalloc_smooth_bytes(long long ns, tng_prec prec) {
    const size_t el = prec == TNG_F64 ? sizeof(double) : sizeof(float);
    return 5 * round256((size_t)(3 * ns) * el) + round256(2 * NOALLOC_MAX_DEGREE * sizeof(double));
}

}  // namespace tng

extern "C" int tng_smooth_noalloc(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
                                  double hg_alpha, const void* const diag[3], const void* const b[3], void* const x[3],
                                  int degree, int steps, double lmin, double lmax) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(eta_wedge && diag && b && x, "NULL argument");
    for (int c = 0; c < 3; ++c) TNG_REQUIRE(diag[c] && b[c] && x[c], "NULL field pointer");
    TNG_REQUIRE(degree >= 1 && degree <= tng::NOALLOC_MAX_DEGREE, "degree must be in [1, 16]");
    TNG_REQUIRE(steps >= 0, "steps must be >= 0");
    TNG_REQUIRE(lmin > 0 && lmax > lmin, "need 0 < lmin < lmax");
    TNG_REQUIRE(hg_alpha >= 0.0 && std::isfinite(hg_alpha), "hg_alpha must be finite and >= 0");
    {
        const size_t el = prec == TNG_F64 ? sizeof(double) : sizeof(float);
        tng::require_device(ctx, eta_wedge, (size_t)(2 * L.cells()) * el, "eta_wedge");
        for (int c = 0; c < 3; ++c) {
            tng::require_device(ctx, diag[c], (size_t)L.node_slots() * el, "diag");
            tng::require_device(ctx, b[c], (size_t)L.node_slots() * el, "b");
            tng::require_device(ctx, x[c], (size_t)L.node_slots() * el, "x");
        }
    }
    const size_t need = tng::noalloc_smooth_bytes(L.node_slots(), prec);
    if (need > tng::NOALLOC_SCRATCH_BYTES)
        throw tng::Error(TNG_E_INVAL, "level too large for the no-allocation smoother: needs " +
                                          std::to_string(need) + " bytes of its " +
                                          std::to_string(tng::NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
    TNG_HIP(hipSetDevice(ctx->device));
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(tng::g_scratch_mu);
        if (ctx->device < (int)tng::g_scratch_ptr.size()) base = static_cast<char*>(tng::g_scratch_ptr[ctx->device]);
    }
    TNG_REQUIRE(base != nullptr, "scratch array not registered for this device (context not created by tng_ctx_create)");
    if (prec == TNG_F64)
        tng::smooth_noalloc_t<double>(ctx, L, eta_wedge, hg_alpha, diag, b, x, degree, steps, lmin, lmax, base);
    else
        tng::smooth_noalloc_t<float>(ctx, L, eta_wedge, hg_alpha, diag, b, x, degree, steps, lmin, lmax, base);
    TNG_API_END
}
