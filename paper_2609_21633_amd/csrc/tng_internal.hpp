// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <map>
#include <vector>

#include "tng.h"

namespace tng {

// Errors travel as exceptions inside the library and become return codes at
// the C boundary (see TNG_API_BEGIN / TNG_API_END).
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void set_last_error(const std::string& msg);
void clear_last_error();

#define TNG_HIP(call)                                                                 \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::tng::Error(TNG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define TNG_REQUIRE(cond, msg)                                                        \
    do {                                                                              \
        if (!(cond)) throw ::tng::Error(TNG_E_INVAL, (msg));                          \
    } while (0)

#define TNG_API_BEGIN try { ::tng::clear_last_error();
#define TNG_API_END                                                                   \
    return TNG_OK;                                                                    \
    }                                                                                 \
    catch (const ::tng::Error& e) {                                                   \
        ::tng::set_last_error(e.what());                                              \
        return e.code;                                                                \
    }                                                                                 \
    catch (const std::bad_alloc&) {                                                   \
        ::tng::set_last_error("host allocation failed");                              \
        return TNG_E_NOMEM;                                                           \
    }                                                                                 \
    catch (const std::exception& e) {                                                 \
        ::tng::set_last_error(e.what());                                              \
        return TNG_E_INVAL;                                                           \
    }

// Device bytes allocated by the calling thread through DevBuf, in whole
// 4 KiB pages; differences around a piece of set-up charge exactly what that
// set-up allocated, whatever other threads do meanwhile.
inline thread_local long long tl_device_bytes = 0;

inline long long devbuf_pages(size_t bytes) { return (long long)((bytes + 4095) & ~size_t(4095)); }

// A bump region of device memory that DevBuf draws from while it is installed
// on the calling thread.  Objects built the same way in two arenas place every
// buffer at the same offset from the arena base, so one kernel launch can
// reach the buffers of several such objects through per-object byte offsets
// (SlotBatch).  Buffers taken from an arena are never freed one by one; the
// arena's owner frees the region.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
};
constexpr size_t ARENA_ALIGN = 256;
inline size_t arena_round(size_t bytes) { return (bytes + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1); }
inline thread_local Arena* tl_arena = nullptr;
// Bytes an arena needs for every DevBuf allocation made so far by this thread
// (never decreases: an arena does not reuse released space).
inline thread_local long long tl_arena_demand = 0;

class ArenaScope {
  public:
    explicit ArenaScope(Arena* a) : prev_(tl_arena) { tl_arena = a; }
    ~ArenaScope() { tl_arena = prev_; }
    ArenaScope(const ArenaScope&) = delete;
    ArenaScope& operator=(const ArenaScope&) = delete;
  private:
    Arena* prev_;
};

// Device buffer: owned (hipMalloc / hipFree), or carved from the installed arena.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    bool owned = false;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), owned(o.owned) { o.p = nullptr; o.n = 0; o.owned = false; }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; owned = o.owned;
            o.p = nullptr; o.n = 0; o.owned = false;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        const size_t bytes = count * sizeof(T);
        tl_arena_demand += (long long)arena_round(bytes);
        if (tl_arena != nullptr) {
            Arena& a = *tl_arena;
            if (a.used + arena_round(bytes) > a.cap)
                throw Error(TNG_E_NOMEM, "arena of " + std::to_string(a.cap) + " bytes exhausted");
            p = reinterpret_cast<T*>(a.base + a.used);
            a.used += arena_round(bytes);
            owned = false;
        } else {
            if (hipMalloc(reinterpret_cast<void**>(&p), bytes) != hipSuccess) {
                p = nullptr;
                (void)hipGetLastError();
                throw Error(TNG_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
            }
            owned = true;
            tl_device_bytes += devbuf_pages(bytes);
        }
        n = count;
    }
    void release() {
        if (p && owned) {
            (void)hipFree(p);
            tl_device_bytes -= devbuf_pages(n * sizeof(T));
        }
        p = nullptr;
        n = 0;
        owned = false;
    }
    void upload(const T* host, size_t count, hipStream_t s) {
        TNG_REQUIRE(count <= n, "upload larger than buffer");
        TNG_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
};

// Slots of one batched launch.  Kernels that take a SlotBatch run gridDim.z =
// nb copies of their grid; copy z works on the buffers of slot z, which sit at
// byte offset off[z] from the buffers named in the launch (arena layout, see
// Arena); mesh arrays are shared and never offset.  With has_cnt, cnt[z]
// replaces the launch's vector count (multi-dots, multi-axpys) or table index
// for copy z.  Outside a batch every launch is the single slot {nb = 1, off 0}.
constexpr int MAX_BATCH = 16;
struct SlotBatch {
    int nb = 1;
    int has_cnt = 0;
    long long off[MAX_BATCH] = {};
    int cnt[MAX_BATCH] = {};
};
inline thread_local const SlotBatch* tl_batch = nullptr;
inline SlotBatch launch_batch() { return tl_batch ? *tl_batch : SlotBatch{}; }
// Launchers whose kernels do not take a SlotBatch refuse to run inside a batch.
inline void require_unbatched(const char* what) {
    if (tl_batch != nullptr && tl_batch->nb > 1)
        throw Error(TNG_E_STATE, std::string(what) + " has no batched form");
}

class BatchScope {
  public:
    explicit BatchScope(const SlotBatch* b) : prev_(tl_batch) { tl_batch = b; }
    ~BatchScope() { tl_batch = prev_; }
    BatchScope(const BatchScope&) = delete;
    BatchScope& operator=(const BatchScope&) = delete;
  private:
    const SlotBatch* prev_;
};

// Number of per-triangle geometry values: rows rho1, rho2 of G^{-1}, row rho3
// of G^{-1} divided by 6h, and h |det G| (see mesh.cpp).
constexpr int GEO_PER_TRI = 10;
constexpr int GEO_PER_COL = 2 * GEO_PER_TRI;
// Per-triangle data of the streaming energy apply (derived from the above):
// g0, g1, g2 (9), the metric g9 (ga . gb) scaled to the wedge volume's radial
// factors (m00, m01, m11 with g9/4; m02, m12 with g9/2; m22 with g9), g9, and the
// SUPG length factor g9^(2/3)/4 (h^2/4 = g9^(2/3)/4 r_m^(4/3) with h = V^(1/3)).
constexpr int EG_PER_TRI = 17;
constexpr int EG_PER_COL = 2 * EG_PER_TRI;

struct Level {
    int m = 0, n = 0;                 // lateral intervals per diamond edge, radial intervals
    double r_in = 0, r_out = 0;
    std::vector<double> unit;         // [10][m+1][m+1][3] unit vectors
    std::vector<double> radii;        // [n+1]
    std::vector<int> uid;             // [10][m+1][m+1] unique lateral id
    int n_unique_lat = 0;
    std::vector<int> grp_ptr_h, grp_slot_h;
    int n_groups = 0;
    std::vector<double> geo_h;        // [10][m][m][GEO_PER_COL] host copy
    // device copies
    DevBuf<double> geo64;             // [10][m][m][GEO_PER_COL]
    DevBuf<float> geo32;
    DevBuf<double> eg64;              // [10][m][m][EG_PER_COL] energy apply geometry
    DevBuf<float> eg32;
    DevBuf<int> grp_ptr, grp_slot;    // duplicate groups (CSR over lateral slots)
    DevBuf<int> lat_grp;              // [10][m+1][m+1]: the slot's duplicate group, -1 for none
    DevBuf<uint8_t> owner;            // [10][m+1][m+1]: 1 for the first copy of a node
    DevBuf<double> inv_mult64;        // [10][m+1][m+1]: 1 / number of copies of the node
    DevBuf<double> unit64;            // [10][m+1][m+1][3] unit vectors
    DevBuf<float> unit32;
    DevBuf<double> rho64;             // [n+1] reference density at the node layers (TALA), if set
    DevBuf<float> rho32;
    DevBuf<float> inv_mult32;

    long long lat_slots() const { return 10LL * (m + 1) * (m + 1); }
    long long node_slots() const { return lat_slots() * (n + 1); }
    long long cells() const { return 10LL * m * m * n; }
    double dr() const { return (r_out - r_in) / n; }
};

}  // namespace tng

namespace tng {
// Optional HIP-event timing of the main kernel of every call, on the stream
// the kernel is launched on.
struct KernelStats {
    double total_ms = 0;
    long long launches = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};
}  // namespace tng

struct tng_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_cu = 256;
    int apply_bands = 0;   // band count of the operator apply; 0 = chosen per launch
    bool profile = false;
    std::map<std::string, tng::KernelStats> stats;
    ~tng_ctx();
};

struct tng_mesh {
    tng_ctx* ctx = nullptr;
    int mt = 0, nr = 0;
    double r_in = 0, r_out = 0;
    std::vector<tng::Level> lv;
};

namespace tng {

inline const Level& level_of(const tng_mesh* mesh, int level) {
    TNG_REQUIRE(mesh != nullptr, "mesh is NULL");
    TNG_REQUIRE(level >= 0 && level < (int)mesh->lv.size(), "level out of range");
    return mesh->lv[level];
}

// Level of a mesh whose arrays live on the device (built with a context).
inline const Level& device_level(const tng_ctx* ctx, const tng_mesh* mesh, int level) {
    TNG_REQUIRE(ctx != nullptr, "ctx is NULL");
    const Level& L = level_of(mesh, level);
    TNG_REQUIRE(mesh->ctx != nullptr, "mesh was built without a context (host only)");
    TNG_REQUIRE(mesh->ctx->device == ctx->device, "mesh belongs to another device");
    return L;
}

// Kernel launchers (defined in the .hip translation units).
// hg_alpha: hourglass-control scale of the viscous block (0: plain one-point operator)
void launch_stokes_apply(const tng_ctx* ctx, const Level& L, const Level* Lp, tng_prec prec,
                         unsigned flags, double hg_alpha, const void* eta, const void* const u[3], const void* p,
                         void* const yu[3], void* yp);
// The velocity apply without its closing pass: y holds each diamond's partial sums on
// the duplicated (diamond-edge) nodes and nothing on Dirichlet rows, for a consumer that
// completes both itself (the fused smoother update).
void launch_stokes_apply_raw(const tng_ctx* ctx, const Level& L, tng_prec prec, unsigned flags, double hg_alpha,
                             const void* eta, const void* const u[3], void* const yu[3]);
// The decomposition launch_stokes_apply would use (tng_stokes_apply_layout);
// launches nothing.
void stokes_apply_layout(const tng_ctx* ctx, const Level& L, const Level* Lp, tng_prec prec, unsigned flags,
                         double hg_alpha, int out[8]);
// Plain streaming copy of `bytes` (a multiple of 16, 16-byte aligned pointers).
void launch_stream_copy(const tng_ctx* ctx, const void* src, void* dst, size_t bytes);
void launch_interface(const tng_ctx* ctx, const Level& L, tng_prec prec, int mode, int ncomp,
                      void* const f[]);
void launch_eta_from_T(const tng_ctx* ctx, const Level& L, tng_prec prec, const void* Tn,
                       void* eta, double E, double F);
void launch_eta_coarsen(const tng_ctx* ctx, const Level& Lc, tng_prec prec, const void* ef,
                        void* ec);

// Argument check of the C entry points: `p` must point at `bytes` bytes of
// ordinary device memory (hipMalloc, hipMemoryTypeDevice) of the context's
// GPU, inside one allocation.  Host, pinned-host and managed memory are
// refused: the kernels' seam sums use FP atomics that are only reliable on
// coarse-grained device memory, and a host pointer handed to a kernel faults.
void require_device(const tng_ctx* ctx, const void* p, size_t bytes, const char* what);

// Scratch array of the no-allocation entry points (noalloc.hip): asks the
// array's address on `device`, which must be current, once per device.
void noalloc_register_device(int device);

// Records a start/stop event pair around a launch when profiling is on.  The
// name is "<kernel>/<detail>" (precision, variant, level size); statistics can
// be read per full name or summed over a kernel prefix.
class ScopedKernelTimer {
  public:
    ScopedKernelTimer(const tng_ctx* ctx, const char* kernel, const char* detail = nullptr);
    ~ScopedKernelTimer();
  private:
    tng_ctx* ctx_;
    std::string name_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace tng

