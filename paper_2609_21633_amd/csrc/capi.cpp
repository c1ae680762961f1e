// C entry points: argument validation and dispatch to the launchers.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <string>
#include <vector>

#include "mg.hpp"
#include "tng_internal.hpp"

namespace tng {

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }

void build_mesh(tng_mesh* mesh, int levels);

void require_device(const tng_ctx* ctx, const void* p, size_t bytes, const char* what) {
    TNG_REQUIRE(p != nullptr, std::string(what) + " is NULL");
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        throw Error(TNG_E_INVAL, std::string(what) + " is not device memory of the context's GPU");
    }
    if (at.type != hipMemoryTypeDevice || at.isManaged)
        throw Error(TNG_E_INVAL, std::string(what) +
                                     " must be device memory (hipMalloc); host, pinned or managed memory is refused");
    if (at.device != ctx->device)
        throw Error(TNG_E_INVAL, std::string(what) + " lives on device " + std::to_string(at.device) +
                                     ", the context uses device " + std::to_string(ctx->device));
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) == hipSuccess && base != nullptr) {
        const char* b = static_cast<const char*>(base);
        const char* q = static_cast<const char*>(p);
        if (q + bytes > b + size)
            throw Error(TNG_E_INVAL, std::string(what) + " is too small: needs " + std::to_string(bytes) +
                                         " bytes, its allocation ends " + std::to_string(b + size - q) +
                                         " bytes after it");
    } else {
        (void)hipGetLastError();
    }
}

namespace {
size_t elsize(tng_prec prec) { return prec == TNG_F64 ? sizeof(double) : sizeof(float); }
size_t node_bytes(const Level& L, tng_prec prec) { return (size_t)L.node_slots() * elsize(prec); }
size_t wedge_bytes(const Level& L, tng_prec prec) { return (size_t)(2 * L.cells()) * elsize(prec); }
void require_vel(const tng_ctx* ctx, const void* const v[3], const Level& L, tng_prec prec, const char* what) {
    TNG_REQUIRE(v != nullptr, std::string(what) + " is NULL");
    for (int c = 0; c < 3; ++c) require_device(ctx, v[c], node_bytes(L, prec), what);
}
}  // namespace

ScopedKernelTimer::ScopedKernelTimer(const tng_ctx* ctx, const char* kernel, const char* detail)
    : ctx_(const_cast<tng_ctx*>(ctx)) {
    if (!ctx_->profile) return;
    name_ = kernel;
    if (detail) name_ = name_ + "/" + detail;
    TNG_HIP(hipEventCreate(&a_));
    TNG_HIP(hipEventCreate(&b_));
    TNG_HIP(hipEventRecord(a_, ctx_->stream));
}

ScopedKernelTimer::~ScopedKernelTimer() {
    if (!a_) return;
    if (hipEventRecord(b_, ctx_->stream) == hipSuccess)
        ctx_->stats[name_].pending.emplace_back(a_, b_);
}

namespace {
void drain(tng_ctx* ctx) {
    for (auto& kv : ctx->stats) {
        for (auto& ev : kv.second.pending) {
            float ms = 0;
            if (hipEventSynchronize(ev.second) == hipSuccess &&
                hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) {
                kv.second.total_ms += ms;
                kv.second.launches += 1;
            }
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
        kv.second.pending.clear();
    }
}
}  // namespace

}  // namespace tng

tng_ctx::~tng_ctx() { tng::drain(this); }

using tng::Error;

namespace tng {
namespace {
void diag_A_t(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge, double hg_alpha,
              bool twopt, void* const diag[3]) {
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(eta_wedge && diag && diag[0] && diag[1] && diag[2], "NULL argument");
    tng::require_device(ctx, eta_wedge, tng::wedge_bytes(L, prec), "eta_wedge");
    tng::require_vel(ctx, diag, L, prec, "diag");
    TNG_HIP(hipSetDevice(ctx->device));
    if (prec == TNG_F64) {
        double* d[3] = {(double*)diag[0], (double*)diag[1], (double*)diag[2]};
        tng::mg_diag_A<double>(ctx, L, (const double*)eta_wedge, hg_alpha, d, twopt);
    } else {
        float* d[3] = {(float*)diag[0], (float*)diag[1], (float*)diag[2]};
        tng::mg_diag_A<float>(ctx, L, (const float*)eta_wedge, hg_alpha, d, twopt);
    }
}

template <typename T>
void smooth_t(tng_ctx* ctx, const tng::Level& L, const void* eta, double hg_alpha, const void* const diag[3],
              const void* const b[3], void* const x[3], int degree, int steps, double lmin, double lmax) {
    const long long ns = L.node_slots(), n3 = 3 * ns;
    tng::DevBuf<T> invd(n3), bb(n3), xx(n3), y(n3), d(n3);
    hipStream_t st = ctx->stream;
    for (int c = 0; c < 3; ++c) {
        TNG_HIP(hipMemcpyAsync(invd.p + c * ns, diag[c], ns * sizeof(T), hipMemcpyDeviceToDevice, st));
        TNG_HIP(hipMemcpyAsync(bb.p + c * ns, b[c], ns * sizeof(T), hipMemcpyDeviceToDevice, st));
        TNG_HIP(hipMemcpyAsync(xx.p + c * ns, x[c], ns * sizeof(T), hipMemcpyDeviceToDevice, st));
    }
    tng::vec_invert<T>(ctx, n3, invd.p);
    const std::vector<double> ab = tng::chebyshev_coefficients(degree, lmin, lmax);
    tng::DevBuf<double> abd(ab.size());
    abd.upload(ab.data(), ab.size(), st);
    tng::chebyshev_steps<T>(ctx, L, (const T*)eta, hg_alpha, invd.p, bb.p, xx.p, y.p, d.p, abd.p, degree, steps,
                            false);
    for (int c = 0; c < 3; ++c)
        TNG_HIP(hipMemcpyAsync(x[c], xx.p + c * ns, ns * sizeof(T), hipMemcpyDeviceToDevice, st));
    TNG_HIP(hipStreamSynchronize(st));   // scratch is freed on return
}
}  // namespace
}  // namespace tng


extern "C" {

const char* tng_last_error(void) { return tng::g_last_error.c_str(); }

int tng_ctx_create(int device, void* hip_stream, tng_ctx** out) {
    TNG_API_BEGIN
    TNG_REQUIRE(out != nullptr, "out is NULL");
    int ndev = 0;
    TNG_HIP(hipGetDeviceCount(&ndev));
    TNG_REQUIRE(device >= 0 && device < ndev, "device ordinal out of range");
    TNG_HIP(hipSetDevice(device));
    auto* c = new tng_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    try {
        tng::noalloc_register_device(device);
    } catch (...) {
        delete c;
        throw;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->n_cu = prop.multiProcessorCount;
    *out = c;
    TNG_API_END
}

int tng_ctx_set_stream(tng_ctx* ctx, void* hip_stream) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx != nullptr, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    TNG_API_END
}

int tng_ctx_set_apply_bands(tng_ctx* ctx, int bands) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx != nullptr, "ctx is NULL");
    TNG_REQUIRE(bands >= 0, "bands must be >= 0");
    ctx->apply_bands = bands;
    TNG_API_END
}

int tng_ctx_profile(tng_ctx* ctx, int enable) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx != nullptr, "ctx is NULL");
    tng::drain(ctx);
    ctx->profile = enable != 0;
    if (enable) ctx->stats.clear();
    TNG_API_END
}

int tng_ctx_kernel_stats(tng_ctx* ctx, const char* name, double* total_ms, long long* launches) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx != nullptr && name != nullptr, "ctx or name is NULL");
    tng::drain(ctx);
    const std::string key(name), pre = key + "/";
    double ms = 0.0;
    long long n = 0;
    for (const auto& kv : ctx->stats)
        if (kv.first == key || kv.first.compare(0, pre.size(), pre) == 0) {
            ms += kv.second.total_ms;
            n += kv.second.launches;
        }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    TNG_API_END
}

int tng_ctx_kernel_stats_at(tng_ctx* ctx, int index, char* name, int name_len, double* total_ms,
                            long long* launches) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx != nullptr && name != nullptr && name_len > 0, "NULL argument");
    tng::drain(ctx);
    TNG_REQUIRE(index >= 0 && index < (int)ctx->stats.size(), "index out of range");
    auto it = ctx->stats.begin();
    std::advance(it, index);
    std::snprintf(name, (size_t)name_len, "%s", it->first.c_str());
    if (total_ms) *total_ms = it->second.total_ms;
    if (launches) *launches = it->second.launches;
    TNG_API_END
}

int tng_eta_from_temperature(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec,
                             const void* T, double E, double F, void* eta_wedge) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(T != nullptr && eta_wedge != nullptr, "T or eta_wedge is NULL");
    TNG_REQUIRE(std::isfinite(E) && std::isfinite(F), "E and F must be finite");
    tng::require_device(ctx, T, tng::node_bytes(L, prec), "T");
    tng::require_device(ctx, eta_wedge, tng::wedge_bytes(L, prec), "eta_wedge");
    TNG_HIP(hipSetDevice(ctx->device));
    tng::launch_eta_from_T(ctx, L, prec, T, eta_wedge, E, F);
    TNG_API_END
}

int tng_eta_coarsen(tng_ctx* ctx, const tng_mesh* mesh, int fine_level, tng_prec prec,
                    const void* eta_fine, void* eta_coarse) {
    TNG_API_BEGIN
    const tng::Level& Lf = tng::device_level(ctx, mesh, fine_level);
    const tng::Level& Lc = tng::device_level(ctx, mesh, fine_level + 1);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(eta_fine != nullptr && eta_coarse != nullptr, "eta pointer is NULL");
    tng::require_device(ctx, eta_fine, tng::wedge_bytes(Lf, prec), "eta_fine");
    tng::require_device(ctx, eta_coarse, tng::wedge_bytes(Lc, prec), "eta_coarse");
    TNG_HIP(hipSetDevice(ctx->device));
    tng::launch_eta_coarsen(ctx, Lc, prec, eta_fine, eta_coarse);
    TNG_API_END
}

int tng_ctx_destroy(tng_ctx* ctx) {
    TNG_API_BEGIN
    delete ctx;
    TNG_API_END
}

int tng_mesh_create(tng_ctx* ctx, int mt, int nr, double r_in, double r_out, int levels,
                    tng_mesh** out) {
    TNG_API_BEGIN
    TNG_REQUIRE(out != nullptr, "out is NULL");
    TNG_REQUIRE(mt >= 1 && (mt & (mt - 1)) == 0 && mt <= 4096, "mt must be a power of two <= 4096");
    TNG_REQUIRE(nr >= 1 && nr <= 65536, "nr out of range");
    TNG_REQUIRE(levels >= 1, "levels must be >= 1");
    TNG_REQUIRE((mt >> (levels - 1)) >= 1 && ((mt >> (levels - 1)) << (levels - 1)) == mt,
                "mt / 2^(levels-1) must be an integer >= 1");
    TNG_REQUIRE((nr >> (levels - 1)) >= 1 && ((nr >> (levels - 1)) << (levels - 1)) == nr,
                "nr / 2^(levels-1) must be an integer >= 1");
    TNG_REQUIRE(r_in > 0.0 && r_out > r_in, "need 0 < r_in < r_out");
    // the kernels index a field of the finest level with 32-bit offsets
    TNG_REQUIRE(10.0 * (mt + 1.0) * (mt + 1.0) * (nr + 1.0) < 2147483648.0 && 20.0 * mt * (double)mt * nr < 4294967296.0,
                "mesh too large: a node field of the finest level must have fewer than 2^31 values");
    if (ctx) TNG_HIP(hipSetDevice(ctx->device));
    auto* m = new tng_mesh();
    m->ctx = ctx;
    m->mt = mt;
    m->nr = nr;
    m->r_in = r_in;
    m->r_out = r_out;
    try {
        tng::build_mesh(m, levels);
    } catch (...) {
        delete m;
        throw;
    }
    *out = m;
    TNG_API_END
}

int tng_mesh_counts(const tng_mesh* mesh, int level, long long out[8]) {
    TNG_API_BEGIN
    const tng::Level& L = tng::level_of(mesh, level);
    TNG_REQUIRE(out != nullptr, "out is NULL");
    out[0] = L.m;
    out[1] = L.n;
    out[2] = L.lat_slots();
    out[3] = L.n_unique_lat;
    out[4] = L.node_slots();
    out[5] = (long long)L.n_unique_lat * (L.n + 1);
    out[6] = L.cells();
    out[7] = 2 * L.cells();
    TNG_API_END
}

int tng_mesh_coords(const tng_mesh* mesh, int level, double* unit_xyz_host, double* r_host) {
    TNG_API_BEGIN
    const tng::Level& L = tng::level_of(mesh, level);
    if (unit_xyz_host) std::memcpy(unit_xyz_host, L.unit.data(), L.unit.size() * sizeof(double));
    if (r_host) std::memcpy(r_host, L.radii.data(), L.radii.size() * sizeof(double));
    TNG_API_END
}

int tng_mesh_dup_groups(const tng_mesh* mesh, int level, int* unique_id_host) {
    TNG_API_BEGIN
    const tng::Level& L = tng::level_of(mesh, level);
    TNG_REQUIRE(unique_id_host != nullptr, "unique_id_host is NULL");
    std::memcpy(unique_id_host, L.uid.data(), L.uid.size() * sizeof(int));
    TNG_API_END
}

int tng_mesh_set_density(tng_mesh* mesh, const double* rho_host) {
    TNG_API_BEGIN
    TNG_REQUIRE(mesh != nullptr && rho_host != nullptr, "NULL argument");
    TNG_REQUIRE(mesh->ctx != nullptr, "mesh was built without a context (host only)");
    for (int k = 0; k <= mesh->nr; ++k)
        TNG_REQUIRE(std::isfinite(rho_host[k]) && rho_host[k] > 0.0, "reference density must be finite and > 0");
    TNG_HIP(hipSetDevice(mesh->ctx->device));
    for (size_t l = 0; l < mesh->lv.size(); ++l) {
        tng::Level& L = mesh->lv[l];
        const int step = mesh->nr / L.n;
        std::vector<double> r64(L.n + 1);
        std::vector<float> r32(L.n + 1);
        for (int k = 0; k <= L.n; ++k) {
            r64[k] = rho_host[k * step];
            r32[k] = (float)r64[k];
        }
        if (L.rho64.n != r64.size()) L.rho64.alloc(r64.size());
        if (L.rho32.n != r32.size()) L.rho32.alloc(r32.size());
        TNG_HIP(hipMemcpy(L.rho64.p, r64.data(), r64.size() * sizeof(double), hipMemcpyHostToDevice));
        TNG_HIP(hipMemcpy(L.rho32.p, r32.data(), r32.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    TNG_API_END
}

int tng_mesh_destroy(tng_mesh* mesh) {
    TNG_API_BEGIN
    delete mesh;
    TNG_API_END
}

int tng_stokes_apply(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec,
                     unsigned op_flags, double hg_alpha, const void* eta_wedge, const void* const u[3],
                     const void* p, void* const y_u[3], void* y_p) {
    TNG_API_BEGIN
    TNG_REQUIRE(hg_alpha >= 0.0 && std::isfinite(hg_alpha), "hg_alpha must be finite and >= 0");
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE((op_flags & ~255u) == 0, "unknown op_flags bits");
    const bool doA = op_flags & TNG_OP_A, doBT = op_flags & TNG_OP_BT, doB = op_flags & TNG_OP_B;
    TNG_REQUIRE(doA || doBT || doB, "op_flags selects no operator block");
    const tng::Level* Lp = nullptr;
    if (doBT || doB) {
        TNG_REQUIRE(level + 1 < (int)mesh->lv.size(), "pressure level (level + 1) not built");
        Lp = &mesh->lv[level + 1];
        TNG_REQUIRE(L.m % 2 == 0 && L.n % 2 == 0, "B/B^T need even m and n");
    }
    if (doA) TNG_REQUIRE(eta_wedge != nullptr, "eta_wedge is NULL");
    if (doA || doB) {
        TNG_REQUIRE(u != nullptr && u[0] && u[1] && u[2], "u is NULL");
    }
    if (doA || doBT) TNG_REQUIRE(y_u != nullptr && y_u[0] && y_u[1] && y_u[2], "y_u is NULL");
    if (doBT) TNG_REQUIRE(p != nullptr, "p is NULL");
    if (doB) TNG_REQUIRE(y_p != nullptr, "y_p is NULL");
    if ((op_flags & TNG_OP_DIRICHLET) && doA)
        TNG_REQUIRE(u != nullptr && u[0] && u[1] && u[2], "u is NULL");
    if (op_flags & TNG_OP_TALA) {
        TNG_REQUIRE(doB, "TNG_OP_TALA changes the divergence block: it needs TNG_OP_B");
        TNG_REQUIRE(!(doA && hg_alpha != 0.0), "TNG_OP_TALA is not available with hourglass control");
        TNG_REQUIRE(L.rho64.p != nullptr, "TNG_OP_TALA needs the mesh's reference density (tng_mesh_set_density)");
    }
    if (op_flags & TNG_OP_TWOPOINT) {
        TNG_REQUIRE(doA, "TNG_OP_TWOPOINT is a form of the viscous block: it needs TNG_OP_A");
        TNG_REQUIRE(hg_alpha == 0.0, "TNG_OP_TWOPOINT is an alternative to hourglass control");
        TNG_REQUIRE(!(op_flags & (TNG_OP_FREESLIP_INNER | TNG_OP_FREESLIP_OUTER | TNG_OP_TALA)),
                    "TNG_OP_TWOPOINT is not available with free slip or TNG_OP_TALA");
        TNG_REQUIRE(doBT || !doB, "TNG_OP_TWOPOINT: A alone, A + B^T or the full operator");
    }
    if (doA) tng::require_device(ctx, eta_wedge, tng::wedge_bytes(L, prec), "eta_wedge");
    if (doA || doB) tng::require_vel(ctx, u, L, prec, "u");
    if (doA || doBT) tng::require_vel(ctx, y_u, L, prec, "y_u");
    if (doBT) tng::require_device(ctx, p, tng::node_bytes(*Lp, prec), "p");
    if (doB) tng::require_device(ctx, y_p, tng::node_bytes(*Lp, prec), "y_p");
    TNG_HIP(hipSetDevice(ctx->device));
    tng::launch_stokes_apply(ctx, L, Lp, prec, op_flags, hg_alpha, eta_wedge, u, p, y_u, y_p);
    TNG_API_END
}

int tng_stokes_apply_layout(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, unsigned op_flags,
                            double hg_alpha, int out[8]) {
    TNG_API_BEGIN
    TNG_REQUIRE(out != nullptr, "out is NULL");
    TNG_REQUIRE(hg_alpha >= 0.0 && std::isfinite(hg_alpha), "hg_alpha must be finite and >= 0");
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE((op_flags & ~255u) == 0, "unknown op_flags bits");
    const bool doBT = op_flags & TNG_OP_BT, doB = op_flags & TNG_OP_B;
    TNG_REQUIRE(op_flags & 7u, "op_flags selects no operator block");
    const tng::Level* Lp = nullptr;
    if (doBT || doB) {
        TNG_REQUIRE(level + 1 < (int)mesh->lv.size(), "pressure level (level + 1) not built");
        Lp = &mesh->lv[level + 1];
        TNG_REQUIRE(L.m % 2 == 0 && L.n % 2 == 0, "B/B^T need even m and n");
    }
    TNG_HIP(hipSetDevice(ctx->device));
    tng::stokes_apply_layout(ctx, L, Lp, prec, op_flags, hg_alpha, out);
    TNG_API_END
}

int tng_check_device_buffer(tng_ctx* ctx, const void* p, size_t bytes) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx != nullptr, "ctx is NULL");
    tng::require_device(ctx, p, bytes, "buffer");
    TNG_API_END
}

int tng_stream_copy(tng_ctx* ctx, const void* src, void* dst, size_t bytes) {
    TNG_API_BEGIN
    TNG_REQUIRE(ctx != nullptr, "ctx is NULL");
    TNG_REQUIRE(bytes > 0 && bytes % 16 == 0, "bytes must be a positive multiple of 16");
    TNG_REQUIRE(((uintptr_t)src | (uintptr_t)dst) % 16 == 0, "src and dst must be 16-byte aligned");
    tng::require_device(ctx, src, bytes, "src");
    tng::require_device(ctx, dst, bytes, "dst");
    TNG_REQUIRE((const char*)src + bytes <= (const char*)dst || (const char*)dst + bytes <= (const char*)src,
                "src and dst overlap");
    TNG_HIP(hipSetDevice(ctx->device));
    tng::launch_stream_copy(ctx, src, dst, bytes);
    TNG_API_END
}

int tng_interface_sum(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, int mode,
                      int ncomp, void* const f[]) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(mode == 0 || mode == 1, "mode must be 0 (sum) or 1 (copy)");
    TNG_REQUIRE(f != nullptr && ncomp >= 1 && ncomp <= 4, "bad field list");
    for (int c = 0; c < ncomp; ++c) tng::require_device(ctx, f[c], tng::node_bytes(L, prec), "field");
    TNG_HIP(hipSetDevice(ctx->device));
    tng::launch_interface(ctx, L, prec, mode, ncomp, f);
    TNG_API_END
}

int tng_rhs_buoyancy(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* T, double Ra,
                     void* const f[3]) {
    return tng_rhs_buoyancy_bc(ctx, mesh, level, prec, 0u, T, Ra, f);
}

int tng_rhs_buoyancy_bc(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, unsigned bc_flags,
                        const void* T, double Ra, void* const f[3]) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(T && f && f[0] && f[1] && f[2], "NULL argument");
    TNG_REQUIRE(std::isfinite(Ra), "Ra must be finite");
    TNG_REQUIRE((bc_flags & ~(unsigned)(TNG_OP_FREESLIP_INNER | TNG_OP_FREESLIP_OUTER)) == 0,
                "bc_flags: TNG_OP_FREESLIP_INNER and/or TNG_OP_FREESLIP_OUTER only");
    tng::require_device(ctx, T, tng::node_bytes(L, prec), "T");
    tng::require_vel(ctx, f, L, prec, "f");
    TNG_HIP(hipSetDevice(ctx->device));
    const unsigned fs = bc_flags >> 4;
    if (prec == TNG_F64) {
        double* ff[3] = {(double*)f[0], (double*)f[1], (double*)f[2]};
        tng::buoyancy_rhs<double>(ctx, L, (const double*)T, Ra, ff, nullptr, nullptr, fs);
    } else {
        float* ff[3] = {(float*)f[0], (float*)f[1], (float*)f[2]};
        tng::buoyancy_rhs<float>(ctx, L, (const float*)T, Ra, ff, nullptr, nullptr, fs);
    }
    TNG_API_END
}

int tng_rhs_buoyancy_tala(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* T, double Ra,
                          const double* Tbar_host, const double* rhoalpha_host, void* const f[3]) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(T && f && f[0] && f[1] && f[2] && Tbar_host && rhoalpha_host, "NULL argument");
    TNG_REQUIRE(std::isfinite(Ra), "Ra must be finite");
    for (int k = 0; k <= L.n; ++k)
        TNG_REQUIRE(std::isfinite(Tbar_host[k]) && std::isfinite(rhoalpha_host[k]), "profiles must be finite");
    tng::require_device(ctx, T, tng::node_bytes(L, prec), "T");
    tng::require_vel(ctx, f, L, prec, "f");
    TNG_HIP(hipSetDevice(ctx->device));
    tng::DevBuf<double> prof(2 * (L.n + 1));
    prof.upload(Tbar_host, L.n + 1, ctx->stream);
    TNG_HIP(hipMemcpyAsync(prof.p + L.n + 1, rhoalpha_host, (L.n + 1) * sizeof(double), hipMemcpyHostToDevice,
                           ctx->stream));
    if (prec == TNG_F64) {
        double* ff[3] = {(double*)f[0], (double*)f[1], (double*)f[2]};
        tng::buoyancy_rhs<double>(ctx, L, (const double*)T, Ra, ff, prof.p, prof.p + L.n + 1);
    } else {
        float* ff[3] = {(float*)f[0], (float*)f[1], (float*)f[2]};
        tng::buoyancy_rhs<float>(ctx, L, (const float*)T, Ra, ff, prof.p, prof.p + L.n + 1);
    }
    TNG_HIP(hipStreamSynchronize(ctx->stream));   // the profiles are freed on return
    TNG_API_END
}

int tng_energy_apply(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* const u[3],
                     double dt, const void* T, void* y) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(u && u[0] && u[1] && u[2] && T && y, "NULL argument");
    TNG_REQUIRE(dt > 0 && std::isfinite(dt), "dt must be positive");
    tng::require_vel(ctx, u, L, prec, "u");
    tng::require_device(ctx, T, tng::node_bytes(L, prec), "T");
    tng::require_device(ctx, y, tng::node_bytes(L, prec), "y");
    TNG_HIP(hipSetDevice(ctx->device));
    if (prec == TNG_F64) {
        const double* uu[3] = {(const double*)u[0], (const double*)u[1], (const double*)u[2]};
        tng::energy_apply<double>(ctx, L, uu, dt, (const double*)T, (double*)y);
    } else {
        const float* uu[3] = {(const float*)u[0], (const float*)u[1], (const float*)u[2]};
        tng::energy_apply<float>(ctx, L, uu, dt, (const float*)T, (float*)y);
    }
    TNG_API_END
}

int tng_mmoc_advect(tng_ctx* ctx, const tng_mesh* mesh, int level, const double* const u[3], double dt,
                    const double* T, double* T_hat) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(u && u[0] && u[1] && u[2] && T && T_hat, "NULL argument");
    TNG_REQUIRE(std::isfinite(dt) && dt >= 0.0, "dt must be finite and >= 0");
    tng::require_vel(ctx, (const void* const*)u, L, TNG_F64, "u");
    tng::require_device(ctx, T, tng::node_bytes(L, TNG_F64), "T");
    tng::require_device(ctx, T_hat, tng::node_bytes(L, TNG_F64), "T_hat");
    TNG_REQUIRE(T != T_hat, "T and T_hat must not alias");
    TNG_HIP(hipSetDevice(ctx->device));
    tng::mmoc_departure(ctx, L, u, dt, T, T_hat);
    TNG_API_END
}

int tng_diag_A(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
               double hg_alpha, void* const diag[3]) {
    TNG_API_BEGIN
    TNG_REQUIRE(hg_alpha >= 0.0 && std::isfinite(hg_alpha), "hg_alpha must be finite and >= 0");
    tng::diag_A_t(ctx, mesh, level, prec, eta_wedge, hg_alpha, false, diag);
    TNG_API_END
}

int tng_diag_A_twopoint(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
                        void* const diag[3]) {
    TNG_API_BEGIN
    tng::diag_A_t(ctx, mesh, level, prec, eta_wedge, 0.0, true, diag);
    TNG_API_END
}

int tng_pressure_mass(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
                      void* mass) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    const tng::Level& Lp = tng::device_level(ctx, mesh, level + 1);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(eta_wedge && mass, "NULL argument");
    TNG_REQUIRE(L.m % 2 == 0 && L.n % 2 == 0, "needs even m and n");
    tng::require_device(ctx, eta_wedge, tng::wedge_bytes(L, prec), "eta_wedge");
    tng::require_device(ctx, mass, tng::node_bytes(Lp, prec), "mass");
    TNG_HIP(hipSetDevice(ctx->device));
    if (prec == TNG_F64)
        tng::mg_pmass<double>(ctx, L, Lp, (const double*)eta_wedge, (double*)mass);
    else
        tng::mg_pmass<float>(ctx, L, Lp, (const float*)eta_wedge, (float*)mass);
    TNG_API_END
}

int tng_restrict(tng_ctx* ctx, const tng_mesh* mesh, int fine_level, tng_prec prec, const void* const f[3],
                 void* const c[3]) {
    TNG_API_BEGIN
    const tng::Level& Lf = tng::device_level(ctx, mesh, fine_level);
    const tng::Level& Lc = tng::device_level(ctx, mesh, fine_level + 1);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(f && c && f[0] && f[1] && f[2] && c[0] && c[1] && c[2], "NULL argument");
    TNG_REQUIRE(Lf.m % 2 == 0 && Lf.n % 2 == 0, "needs even m and n");
    tng::require_vel(ctx, f, Lf, prec, "f");
    tng::require_vel(ctx, c, Lc, prec, "c");
    TNG_HIP(hipSetDevice(ctx->device));
    if (prec == TNG_F64) {
        const double* ff[3] = {(const double*)f[0], (const double*)f[1], (const double*)f[2]};
        double* cc[3] = {(double*)c[0], (double*)c[1], (double*)c[2]};
        tng::mg_restrict<double>(ctx, Lf, Lc, ff, cc);
    } else {
        const float* ff[3] = {(const float*)f[0], (const float*)f[1], (const float*)f[2]};
        float* cc[3] = {(float*)c[0], (float*)c[1], (float*)c[2]};
        tng::mg_restrict<float>(ctx, Lf, Lc, ff, cc);
    }
    TNG_API_END
}

int tng_prolong(tng_ctx* ctx, const tng_mesh* mesh, int fine_level, tng_prec prec, const void* const c[3],
                void* const f[3]) {
    TNG_API_BEGIN
    const tng::Level& Lf = tng::device_level(ctx, mesh, fine_level);
    const tng::Level& Lc = tng::device_level(ctx, mesh, fine_level + 1);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(f && c && f[0] && f[1] && f[2] && c[0] && c[1] && c[2], "NULL argument");
    TNG_REQUIRE(Lf.m % 2 == 0 && Lf.n % 2 == 0, "needs even m and n");
    tng::require_vel(ctx, c, Lc, prec, "c");
    tng::require_vel(ctx, f, Lf, prec, "f");
    TNG_HIP(hipSetDevice(ctx->device));
    if (prec == TNG_F64) {
        const double* cc[3] = {(const double*)c[0], (const double*)c[1], (const double*)c[2]};
        double* ff[3] = {(double*)f[0], (double*)f[1], (double*)f[2]};
        tng::mg_prolong<double>(ctx, Lf, cc, ff, false);
    } else {
        const float* cc[3] = {(const float*)c[0], (const float*)c[1], (const float*)c[2]};
        float* ff[3] = {(float*)f[0], (float*)f[1], (float*)f[2]};
        tng::mg_prolong<float>(ctx, Lf, cc, ff, false);
    }
    TNG_API_END
}

int tng_smooth(tng_ctx* ctx, const tng_mesh* mesh, int level, tng_prec prec, const void* eta_wedge,
               double hg_alpha, const void* const diag[3], const void* const b[3], void* const x[3], int degree,
               int steps, double lmin, double lmax) {
    TNG_API_BEGIN
    const tng::Level& L = tng::device_level(ctx, mesh, level);
    TNG_REQUIRE(prec == TNG_F64 || prec == TNG_F32, "bad precision");
    TNG_REQUIRE(eta_wedge && diag && b && x, "NULL argument");
    for (int c = 0; c < 3; ++c) TNG_REQUIRE(diag[c] && b[c] && x[c], "NULL field pointer");
    TNG_REQUIRE(degree >= 1 && steps >= 0, "bad degree or steps");
    TNG_REQUIRE(lmin > 0 && lmax > lmin, "need 0 < lmin < lmax");
    tng::require_device(ctx, eta_wedge, tng::wedge_bytes(L, prec), "eta_wedge");
    tng::require_vel(ctx, diag, L, prec, "diag");
    tng::require_vel(ctx, b, L, prec, "b");
    tng::require_vel(ctx, x, L, prec, "x");
    TNG_HIP(hipSetDevice(ctx->device));
    if (prec == TNG_F64)
        tng::smooth_t<double>(ctx, L, eta_wedge, hg_alpha, diag, b, x, degree, steps, lmin, lmax);
    else
        tng::smooth_t<float>(ctx, L, eta_wedge, hg_alpha, diag, b, x, degree, steps, lmin, lmax);
    TNG_API_END
}

}  // extern "C"
