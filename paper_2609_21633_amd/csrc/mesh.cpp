// Icosahedral shell mesh (Sec. 2 "Grid and Parallelization").
//
// Ten diamonds, each a pair of icosahedron faces, carry an (m+1) x (m+1) grid
// of lateral nodes obtained by recursive geodesic midpoint refinement; the
// surface grid is extruded through n uniform radial intervals.  Each
// hexahedral cell (i, j, k) is split into two wedges along the diagonal that
// is parallel to the diamond's shared diagonal, so that fine wedges nest in
// coarse ones.  Nodes on diamond edges are stored once per diamond; the
// duplicate groups computed here let the interface kernel sum the copies.
//
// Per lateral triangle the kernels need the inverse of
//   G = [s1 - s0 | s2 - s0 | s_c],  s_c = (s0 + s1 + s2) / 3,
// because the isoparametric Jacobian at the quadrature point q_c factors as
// J = G diag(r_m, r_m, h) (r_m the wedge's mid radius, h half its height).
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "tng_internal.hpp"

namespace tng {
namespace {

struct V3 {
    double x, y, z;
};
inline V3 add(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 normalize(V3 a) {
    double s = std::sqrt(a.x * a.x + a.y * a.y + a.z * a.z);
    return {a.x / s, a.y / s, a.z / s};
}

// Icosahedron vertices: 0 north pole, 1..5 upper ring U_k, 6..10 lower ring L_k, 11 south pole.
void ico_vertices(V3 v[12]) {
    const double PI = 3.14159265358979323846;
    const double z = 1.0 / std::sqrt(5.0), rho = 2.0 / std::sqrt(5.0);
    v[0] = {0.0, 0.0, 1.0};
    for (int k = 0; k < 5; ++k) {
        double a = 2.0 * PI * k / 5.0;
        v[1 + k] = {rho * std::cos(a), rho * std::sin(a), z};
        double b = a + PI / 5.0;
        v[6 + k] = {rho * std::cos(b), rho * std::sin(b), -z};
    }
    v[11] = {0.0, 0.0, -1.0};
}

// Corners (0,0), (m,0), (0,m), (m,m) of diamond d as icosahedron vertex ids.
void diamond_corners(int d, int c[4]) {
    auto U = [](int k) { return 1 + ((k % 5) + 5) % 5; };
    auto L = [](int k) { return 6 + ((k % 5) + 5) % 5; };
    if (d < 5) {
        c[0] = 0; c[1] = U(d); c[2] = U(d + 1); c[3] = L(d);
    } else {
        int k = d - 5;
        c[0] = U(k + 1); c[1] = L(k); c[2] = L(k + 1); c[3] = 11;
    }
}

// Lateral unit vectors of one diamond at m = 2^L intervals, [m+1][m+1].
void refine_diamond(int d, int m, std::vector<V3>& s) {
    V3 ico[12];
    ico_vertices(ico);
    int c[4];
    diamond_corners(d, c);
    s.assign((size_t)(m + 1) * (m + 1), V3{0, 0, 0});
    auto at = [&](int i, int j) -> V3& { return s[(size_t)i * (m + 1) + j]; };
    at(0, 0) = ico[c[0]];
    at(m, 0) = ico[c[1]];
    at(0, m) = ico[c[2]];
    at(m, m) = ico[c[3]];
    for (int st = m; st > 1; st /= 2) {
        int h = st / 2;
        for (int i = 0; i <= m; i += h)
            for (int j = 0; j <= m; j += h) {
                bool io = (i % st) != 0, jo = (j % st) != 0;
                if (!io && !jo) continue;
                V3 a, b;
                if (io && !jo) { a = at(i - h, j); b = at(i + h, j); }
                else if (!io && jo) { a = at(i, j - h); b = at(i, j + h); }
                else { a = at(i - h, j + h); b = at(i + h, j - h); }  // midpoint of the split diagonal
                at(i, j) = normalize(add(a, b));
            }
    }
}

// Rows of G^{-1}, G = [a | b | c] given by columns.
bool invert_cols(V3 a, V3 b, V3 c, double inv[9], double& det) {
    // rows of the inverse are cross products divided by the determinant
    V3 bc = {b.y * c.z - b.z * c.y, b.z * c.x - b.x * c.z, b.x * c.y - b.y * c.x};
    V3 ca = {c.y * a.z - c.z * a.y, c.z * a.x - c.x * a.z, c.x * a.y - c.y * a.x};
    V3 ab = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    det = a.x * bc.x + a.y * bc.y + a.z * bc.z;
    if (det == 0.0) return false;
    double r = 1.0 / det;
    inv[0] = bc.x * r; inv[1] = bc.y * r; inv[2] = bc.z * r;
    inv[3] = ca.x * r; inv[4] = ca.y * r; inv[5] = ca.z * r;
    inv[6] = ab.x * r; inv[7] = ab.y * r; inv[8] = ab.z * r;
    return true;
}

void build_level(Level& L, int m, int n, double r_in, double r_out, bool device) {
    L.m = m;
    L.n = n;
    L.r_in = r_in;
    L.r_out = r_out;
    L.radii.resize(n + 1);
    for (int k = 0; k <= n; ++k) L.radii[k] = r_in + (r_out - r_in) * k / n;
    const size_t nl = (size_t)(m + 1) * (m + 1);
    L.unit.resize(10 * nl * 3);
    std::vector<V3> s;
    for (int d = 0; d < 10; ++d) {
        refine_diamond(d, m, s);
        for (size_t q = 0; q < nl; ++q) {
            L.unit[(d * nl + q) * 3 + 0] = s[q].x;
            L.unit[(d * nl + q) * 3 + 1] = s[q].y;
            L.unit[(d * nl + q) * 3 + 2] = s[q].z;
        }
    }
    // duplicate groups: the same geometric node reached from several diamonds
    // is computed from the same parent pairs, so its coordinates agree exactly.
    std::map<std::tuple<long long, long long, long long>, int> key2id;
    std::vector<std::vector<int>> members;
    L.uid.resize(10 * nl);
    for (size_t q = 0; q < 10 * nl; ++q) {
        auto key = std::make_tuple(std::llround(L.unit[q * 3 + 0] * 1e11),
                                   std::llround(L.unit[q * 3 + 1] * 1e11),
                                   std::llround(L.unit[q * 3 + 2] * 1e11));
        auto it = key2id.find(key);
        int id;
        if (it == key2id.end()) {
            id = (int)members.size();
            key2id.emplace(key, id);
            members.emplace_back();
        } else {
            id = it->second;
        }
        members[id].push_back((int)q);
        L.uid[q] = id;
    }
    L.n_unique_lat = (int)members.size();
    if (L.n_unique_lat != 10 * m * m + 2)
        throw Error(TNG_E_INVAL, "mesh build: unexpected number of unique lateral nodes");
    L.grp_ptr_h.assign(1, 0);
    L.grp_slot_h.clear();
    std::vector<uint8_t> owner(10 * nl, 1);
    for (auto& g : members) {
        if (g.size() < 2) continue;
        for (size_t t = 0; t < g.size(); ++t) {
            L.grp_slot_h.push_back(g[t]);
            if (t > 0) owner[g[t]] = 0;
        }
        L.grp_ptr_h.push_back((int)L.grp_slot_h.size());
    }
    L.n_groups = (int)L.grp_ptr_h.size() - 1;
    // per-triangle geometry of every cell column
    const double hh = 0.5 * (r_out - r_in) / n;
    std::vector<double> geo((size_t)10 * m * m * GEO_PER_COL);
    auto S = [&](int d, int i, int j) {
        const double* p = &L.unit[((size_t)d * nl + (size_t)i * (m + 1) + j) * 3];
        return V3{p[0], p[1], p[2]};
    };
    for (int d = 0; d < 10; ++d)
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                V3 tri[2][3] = {{S(d, i, j), S(d, i + 1, j), S(d, i, j + 1)},
                                {S(d, i + 1, j + 1), S(d, i, j + 1), S(d, i + 1, j)}};
                double* g = &geo[(((size_t)d * m + i) * m + j) * GEO_PER_COL];
                for (int t = 0; t < 2; ++t) {
                    V3 s0 = tri[t][0], s1 = tri[t][1], s2 = tri[t][2];
                    V3 sc = {(s0.x + s1.x + s2.x) / 3.0, (s0.y + s1.y + s2.y) / 3.0,
                             (s0.z + s1.z + s2.z) / 3.0};
                    double inv[9], det;
                    if (!invert_cols(sub(s1, s0), sub(s2, s0), sc, inv, det))
                        throw Error(TNG_E_INVAL, "mesh build: degenerate triangle");
                    double* gt = g + t * GEO_PER_TRI;
                    for (int q = 0; q < 6; ++q) gt[q] = inv[q];
                    for (int q = 6; q < 9; ++q) gt[q] = inv[q] / (6.0 * hh);
                    gt[9] = hh * std::fabs(det);
                }
            }
    L.geo_h = geo;
    if (!device) return;
    L.geo64.alloc(geo.size());
    L.geo32.alloc(geo.size());
    std::vector<float> geo32(geo.begin(), geo.end());
    TNG_HIP(hipMemcpy(L.geo64.p, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice));
    TNG_HIP(hipMemcpy(L.geo32.p, geo32.data(), geo32.size() * sizeof(float), hipMemcpyHostToDevice));
    {
        const size_t ncol = (size_t)10 * m * m;
        std::vector<double> eg(ncol * EG_PER_COL);
        for (size_t c = 0; c < ncol; ++c)
            for (int t = 0; t < 2; ++t) {
                const double* g = &geo[c * GEO_PER_COL + t * GEO_PER_TRI];
                double* e = &eg[c * EG_PER_COL + t * EG_PER_TRI];
                auto dot = [&](int a, int b) { return g[a] * g[b] + g[a + 1] * g[b + 1] + g[a + 2] * g[b + 2]; };
                for (int q = 0; q < 9; ++q) e[q] = g[q];
                const double g9 = g[9];
                e[9] = 0.25 * g9 * dot(0, 0);
                e[10] = 0.25 * g9 * dot(0, 3);
                e[11] = 0.25 * g9 * dot(3, 3);
                e[12] = 0.5 * g9 * dot(0, 6);
                e[13] = 0.5 * g9 * dot(3, 6);
                e[14] = g9 * dot(6, 6);
                e[15] = g9;
                const double c13 = std::cbrt(g9);
                e[16] = 0.25 * c13 * c13;
            }
        L.eg64.alloc(eg.size());
        L.eg32.alloc(eg.size());
        std::vector<float> eg32(eg.begin(), eg.end());
        TNG_HIP(hipMemcpy(L.eg64.p, eg.data(), eg.size() * sizeof(double), hipMemcpyHostToDevice));
        TNG_HIP(hipMemcpy(L.eg32.p, eg32.data(), eg32.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    {
        std::vector<int> lg(10 * nl, -1);
        for (int g = 0; g < L.n_groups; ++g)
            for (int q = L.grp_ptr_h[g]; q < L.grp_ptr_h[g + 1]; ++q) lg[L.grp_slot_h[q]] = g;
        L.lat_grp.alloc(lg.size());
        TNG_HIP(hipMemcpy(L.lat_grp.p, lg.data(), lg.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    L.grp_ptr.alloc(L.grp_ptr_h.size());
    TNG_HIP(hipMemcpy(L.grp_ptr.p, L.grp_ptr_h.data(), L.grp_ptr_h.size() * sizeof(int), hipMemcpyHostToDevice));
    L.grp_slot.alloc(L.grp_slot_h.size());
    TNG_HIP(hipMemcpy(L.grp_slot.p, L.grp_slot_h.data(), L.grp_slot_h.size() * sizeof(int), hipMemcpyHostToDevice));
    L.owner.alloc(owner.size());
    TNG_HIP(hipMemcpy(L.owner.p, owner.data(), owner.size(), hipMemcpyHostToDevice));
    std::vector<double> im(10 * nl);
    std::vector<float> im32(10 * nl);
    for (size_t q = 0; q < 10 * nl; ++q) {
        im[q] = 1.0 / (double)members[L.uid[q]].size();
        im32[q] = (float)im[q];
    }
    L.inv_mult64.alloc(im.size());
    TNG_HIP(hipMemcpy(L.inv_mult64.p, im.data(), im.size() * sizeof(double), hipMemcpyHostToDevice));
    L.unit64.alloc(L.unit.size());
    TNG_HIP(hipMemcpy(L.unit64.p, L.unit.data(), L.unit.size() * sizeof(double), hipMemcpyHostToDevice));
    std::vector<float> u32(L.unit.begin(), L.unit.end());
    L.unit32.alloc(u32.size());
    TNG_HIP(hipMemcpy(L.unit32.p, u32.data(), u32.size() * sizeof(float), hipMemcpyHostToDevice));
    L.inv_mult32.alloc(im32.size());
    TNG_HIP(hipMemcpy(L.inv_mult32.p, im32.data(), im32.size() * sizeof(float), hipMemcpyHostToDevice));
}

}  // namespace

void build_mesh(tng_mesh* mesh, int levels) {
    mesh->lv.clear();
    mesh->lv.resize(levels);
    for (int l = 0; l < levels; ++l)
        build_level(mesh->lv[l], mesh->mt >> l, mesh->nr >> l, mesh->r_in, mesh->r_out,
                    mesh->ctx != nullptr);
}

}  // namespace tng
