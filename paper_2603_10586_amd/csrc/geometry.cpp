// Context, geometry and grouping (host side of libqrvie).
//
// Discretisation: each disk becomes 24 in-plane squares of side h = r sqrt(pi/24)
// (centres ((a+1/2)h, (b+1/2)h) with (a+1/2)^2 + (b+1/2)^2 <= 24/pi) in two layers at
// z = -t/4 and z = +t/4; cell volume h^2 t / 2 (48 cells fill the disk volume exactly).
// A sphere (the paper's meta-atom, §6.1) becomes 48 cubes of side h = r (pi/36)^(1/3):
// four layers at z = (-3/2, -1/2, 1/2, 3/2) h, each the 12 squares of a 4 x 4 grid whose
// centres satisfy max(|x|, |y|) < 3h/2 or min(|x|, |y|) < h (the grid without its corners).
// Unknowns are grouped particle by particle (§4, eq. 4.1).
//
// Grouping (§5.1, §5.3, §5.4): a quadtree aligned with the particle lattice, padded to
// 2^L sites per side, or the paper's grid (level 1 is 3 x 3 blocks of the bounding square,
// halving per level) with each particle in the block of its centre.  Both are indexed by
// the finest-level block (i, j): the level-l block is (i, j) >> (L - l).  Particles are
// ordered along a Morton curve of (i, j) so that every tree node is a contiguous range of
// particles (and of DoFs).  At level l the ordered pairs
// (I, J) of occupied nodes whose parents are near (share a grid node: Chebyshev distance
// <= 1) and which are far (Chebyshev >= 2) are compressed; at the finest level, where a
// node holds one particle, the near pairs I != J are compressed too, so the near part
// left is the particle block diagonal.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <unordered_map>

#include "internal.h"

using namespace qrvie;

namespace qrvie {

bool set_err(qrvie_ctx* ctx, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return false;
}

qrvie_status hip_check(qrvie_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return QRVIE_OK;
    set_err(ctx, std::string(what) + ": " + hipGetErrorString(e));
    return QRVIE_ERR_DEVICE;
}

qrvie_status dalloc(qrvie_ctx* ctx, void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (bytes == 0) return QRVIE_OK;
    if (ctx->budget && ctx->in_use.load() + bytes > ctx->budget) {
        set_err(ctx, std::string(what) + ": HBM budget exceeded (" + std::to_string(ctx->in_use.load() + bytes) +
                         " > " + std::to_string(ctx->budget) + " bytes)");
        return QRVIE_ERR_OUT_OF_MEMORY;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        set_err(ctx, std::string(what) + ": hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                         hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? QRVIE_ERR_OUT_OF_MEMORY : QRVIE_ERR_DEVICE;
    }
    const size_t now = (ctx->in_use += bytes);
    size_t pk = ctx->peak.load();
    while (now > pk && !ctx->peak.compare_exchange_weak(pk, now)) {
    }
    return QRVIE_OK;
}

void dfree(qrvie_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    if (ctx) ctx->in_use -= bytes;
}

void particle_offsets(double radius, double height, double* off) {
    const double h = radius * std::sqrt(M_PI / 24.0);
    const double limit = 24.0 / M_PI;
    int c = 0;
    for (int layer = 0; layer < 2; ++layer) {
        const double z = layer == 0 ? -height / 4.0 : height / 4.0;
        for (int b = -3; b < 3; ++b)
            for (int a = -3; a < 3; ++a) {
                const double cx = a + 0.5, cy = b + 0.5;
                if (cx * cx + cy * cy <= limit) {
                    off[3 * c + 0] = cx * h;
                    off[3 * c + 1] = cy * h;
                    off[3 * c + 2] = z;
                    ++c;
                }
            }
    }
}

void sphere_offsets(double radius, double* off) {
    const double h = radius * std::cbrt(M_PI / 36.0);
    int c = 0;
    for (int layer = 0; layer < 4; ++layer)
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                if ((a == 0 || a == 3) && (b == 0 || b == 3)) continue;   // the grid's corners
                off[3 * c + 0] = (a - 1.5) * h;
                off[3 * c + 1] = (b - 1.5) * h;
                off[3 * c + 2] = (layer - 1.5) * h;
                ++c;
            }
}

// The paper's grid over the bounding square of the centres: the finest level L (>= 1) at
// which the blocks of side D / (3 2^(L-1)) hold at most one particle each, and each
// particle's block there.  Returns L, or 0 when two centres share a block at level 20.
int paper_grid(int n, const double* centers, std::vector<int32_t>& ij) {
    double xmin = centers[0], xmax = centers[0], ymin = centers[1], ymax = centers[1];
    for (int p = 1; p < n; ++p) {
        xmin = std::min(xmin, centers[3 * p]); xmax = std::max(xmax, centers[3 * p]);
        ymin = std::min(ymin, centers[3 * p + 1]); ymax = std::max(ymax, centers[3 * p + 1]);
    }
    double side = std::max(xmax - xmin, ymax - ymin);
    if (!(side > 0.0)) side = 1.0;                   // one particle (or all on one point)
    side *= 1.0 + std::ldexp(1.0, -20);
    const double x0 = 0.5 * (xmin + xmax) - 0.5 * side, y0 = 0.5 * (ymin + ymax) - 0.5 * side;
    ij.assign(2 * (size_t)n, 0);
    for (int L = 1; L <= 20; ++L) {
        const int64_t nb = (int64_t)3 << (L - 1);
        const double h = side / (double)nb;
        std::vector<int64_t> keys(n);
        for (int p = 0; p < n; ++p) {
            const int64_t i = std::min<int64_t>(nb - 1, (int64_t)std::floor((centers[3 * p] - x0) / h));
            const int64_t j = std::min<int64_t>(nb - 1, (int64_t)std::floor((centers[3 * p + 1] - y0) / h));
            ij[2 * p] = (int32_t)i;
            ij[2 * p + 1] = (int32_t)j;
            keys[p] = i * nb + j;
        }
        std::sort(keys.begin(), keys.end());
        if (std::adjacent_find(keys.begin(), keys.end()) == keys.end() || n == 1) return L;
    }
    return 0;
}

static uint64_t morton(uint32_t i, uint32_t j) {
    uint64_t code = 0;
    for (int b = 0; b < 31; ++b) {
        code |= (uint64_t)((i >> b) & 1u) << (2 * b);
        code |= (uint64_t)((j >> b) & 1u) << (2 * b + 1);
    }
    return code;
}

static inline int64_t key2(int64_t X, int64_t Y) { return (X << 32) ^ (Y & 0xffffffffLL); }

}  // namespace qrvie

// Per-geometry lattice bookkeeping kept beside the public struct.
struct GeomLattice {
    std::vector<int32_t> li, lj;                                   // internal order, shifted to 0
    std::vector<std::unordered_map<int64_t, int32_t>> level_map;   // key -> node id
    std::vector<std::pair<int32_t, int32_t>> node_xy;              // node id -> (X, Y)
};
static std::map<const qrvie_geom*, GeomLattice>& lattices() {
    static std::map<const qrvie_geom*, GeomLattice> m;
    return m;
}
static std::mutex& lattice_mutex() {   // geometries are created and destroyed from several threads
    static std::mutex mu;
    return mu;
}

namespace qrvie {
// Children of node `id` (level l) at level l+1.
std::vector<int32_t> node_children(const qrvie_geom* g, int32_t id) {
    std::lock_guard<std::mutex> lock(lattice_mutex());
    auto& lat = lattices().at(g);
    const auto& nd = g->nodes[id];
    std::vector<int32_t> out;
    if (nd.level >= g->L) return out;
    const auto xy = lat.node_xy[id];
    const auto& mp = lat.level_map[nd.level + 1];
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
            auto it = mp.find(key2(2 * (int64_t)xy.first + a, 2 * (int64_t)xy.second + b));
            if (it != mp.end()) out.push_back(it->second);
        }
    std::sort(out.begin(), out.end(), [&](int32_t x, int32_t y) { return g->nodes[x].first < g->nodes[y].first; });
    return out;
}
}  // namespace qrvie

extern "C" {

const char* qrvie_status_string(qrvie_status s) {
    switch (s) {
        case QRVIE_OK: return "ok";
        case QRVIE_ERR_INVALID_ARG: return "invalid argument";
        case QRVIE_ERR_GEOMETRY: return "invalid geometry";
        case QRVIE_ERR_OUT_OF_MEMORY: return "out of memory";
        case QRVIE_ERR_DEVICE: return "device error";
        case QRVIE_NOT_CONVERGED: return "not converged";
        case QRVIE_ERR_QUEUE_FULL: return "queue full";
    }
    return "unknown status";
}

qrvie_status qrvie_ctx_create(int hip_device, void* hip_stream, size_t hbm_budget, qrvie_ctx** out) {
    if (!out) return QRVIE_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return QRVIE_ERR_DEVICE;
    }
    if (hip_device < 0 || hip_device >= ndev) return QRVIE_ERR_INVALID_ARG;
    if (hipSetDevice(hip_device) != hipSuccess) return QRVIE_ERR_DEVICE;
    auto* c = new qrvie_ctx;
    c->device = hip_device;
    c->budget = hbm_budget;
    if (!scratch_setup(hip_device, &c->scratch, &c->scratch_err)) c->scratch = nullptr;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return QRVIE_ERR_DEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return QRVIE_OK;
}

void qrvie_ctx_destroy(qrvie_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->own_stream && ctx->stream) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
}

const char* qrvie_last_error(const qrvie_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

size_t qrvie_ctx_bytes_in_use(const qrvie_ctx* ctx) { return ctx ? ctx->in_use.load() : 0; }

size_t qrvie_ctx_peak_bytes(qrvie_ctx* ctx, int32_t reset) {
    if (!ctx) return 0;
    const size_t pk = ctx->peak.load();
    if (reset) ctx->peak.store(ctx->in_use.load());
    return pk;
}

qrvie_status qrvie_geom_create(qrvie_ctx* ctx, const qrvie_array_desc* d, qrvie_geom** out) {
    if (!ctx || !d || !out) return QRVIE_ERR_INVALID_ARG;
    *out = nullptr;
    if (d->n < 1 || !d->centers || !d->radius || !d->height || !d->eps_r ||
        (!d->lattice_ij && d->grid != QRVIE_GRID_PAPER)) {
        set_err(ctx, "geom_create: null pointer or n < 1");
        return QRVIE_ERR_INVALID_ARG;
    }
    if (d->n_eps != 1 && d->n_eps != d->n) { set_err(ctx, "geom_create: n_eps must be 1 or n"); return QRVIE_ERR_INVALID_ARG; }
    if (d->cells_per_particle != kCells) { set_err(ctx, "geom_create: cells_per_particle must be 48"); return QRVIE_ERR_INVALID_ARG; }
    if ((d->shape != QRVIE_SHAPE_DISK && d->shape != QRVIE_SHAPE_SPHERE) ||
        (d->grid != QRVIE_GRID_LATTICE && d->grid != QRVIE_GRID_PAPER)) {
        set_err(ctx, "geom_create: unknown shape or grid");
        return QRVIE_ERR_INVALID_ARG;
    }
    const bool paper = d->grid == QRVIE_GRID_PAPER;
    if (!(d->wavelength > 0.0) || !std::isfinite(d->wavelength)) { set_err(ctx, "geom_create: wavelength must be > 0"); return QRVIE_ERR_INVALID_ARG; }
    const int N = d->n;
    for (int p = 0; p < N; ++p) {
        const qrvie_c128 e = d->eps_r[d->n_eps == 1 ? 0 : p];
        if (!std::isfinite(d->centers[3 * p]) || !std::isfinite(d->centers[3 * p + 1]) ||
            !std::isfinite(d->centers[3 * p + 2]) || !(d->radius[p] > 0.0) || !std::isfinite(d->radius[p]) ||
            (d->shape == QRVIE_SHAPE_DISK && (!(d->height[p] > 0.0) || !std::isfinite(d->height[p]))) ||
            !std::isfinite(e.re) || !std::isfinite(e.im) ||
            (e.re == 1.0 && e.im == 0.0)) {
            set_err(ctx, "geom_create: particle " + std::to_string(p) + " has a non-finite or invalid parameter");
            return QRVIE_ERR_INVALID_ARG;
        }
    }
    // finest-level block of each particle (caller order)
    std::vector<int32_t> bij;
    int L = 0;
    if (paper) {
        L = paper_grid(N, d->centers, bij);
        if (L == 0) { set_err(ctx, "geom_create: two particle centres share a block of the finest grid level"); return QRVIE_ERR_GEOMETRY; }
    } else {
        int32_t imin = INT32_MAX, jmin = INT32_MAX, imax = INT32_MIN, jmax = INT32_MIN;
        for (int p = 0; p < N; ++p) {
            imin = std::min(imin, d->lattice_ij[2 * p]); imax = std::max(imax, d->lattice_ij[2 * p]);
            jmin = std::min(jmin, d->lattice_ij[2 * p + 1]); jmax = std::max(jmax, d->lattice_ij[2 * p + 1]);
        }
        const int64_t nx = (int64_t)imax - imin + 1, ny = (int64_t)jmax - jmin + 1;
        if (nx > (1 << 24) || ny > (1 << 24)) { set_err(ctx, "geom_create: lattice extent too large"); return QRVIE_ERR_GEOMETRY; }
        while ((int64_t(1) << L) < std::max(nx, ny)) ++L;
        bij.resize(2 * (size_t)N);
        for (int p = 0; p < N; ++p) {
            bij[2 * p] = d->lattice_ij[2 * p] - imin;
            bij[2 * p + 1] = d->lattice_ij[2 * p + 1] - jmin;
        }
    }

    auto* g = new qrvie_geom;
    g->ctx = ctx;
    g->N = N;
    g->wavelength = d->wavelength;
    g->k = 2.0 * M_PI / d->wavelength;
    g->L = L;
    g->paper_grid = paper;

    std::vector<std::pair<uint64_t, int32_t>> codes(N);
    for (int p = 0; p < N; ++p) codes[p] = {morton((uint32_t)bij[2 * p], (uint32_t)bij[2 * p + 1]), p};
    std::sort(codes.begin(), codes.end());
    for (int p = 1; p < N; ++p)
        if (codes[p].first == codes[p - 1].first) {
            set_err(ctx, "geom_create: particles " + std::to_string(codes[p - 1].second) + " and " +
                             std::to_string(codes[p].second) + " share a lattice site");
            delete g;
            return QRVIE_ERR_GEOMETRY;
        }
    g->i2c.resize(N);
    g->c2i.resize(N);
    GeomLattice lat;
    lat.li.resize(N);
    lat.lj.resize(N);
    g->center.resize(3 * (size_t)N);
    g->ptype.resize(N);
    std::map<std::vector<uint64_t>, int32_t> tmap;
    for (int p = 0; p < N; ++p) {
        const int c = codes[p].second;
        g->i2c[p] = c;
        g->c2i[c] = p;
        lat.li[p] = bij[2 * c];
        lat.lj[p] = bij[2 * c + 1];
        for (int a = 0; a < 3; ++a) g->center[3 * p + a] = d->centers[3 * c + a];
        const qrvie_c128 e = d->eps_r[d->n_eps == 1 ? 0 : c];
        const bool sphere = d->shape == QRVIE_SHAPE_SPHERE;
        double vals[5] = {d->radius[c], sphere ? 0.0 : d->height[c], e.re, e.im, sphere ? 1.0 : 0.0};
        std::vector<uint64_t> key(5);
        std::memcpy(key.data(), vals, sizeof vals);
        auto it = tmap.find(key);
        if (it == tmap.end()) {
            PType t{};
            t.radius = vals[0]; t.height = vals[1]; t.eps_re = vals[2]; t.eps_im = vals[3];
            if (sphere) {
                const double h = t.radius * std::cbrt(M_PI / 36.0);
                t.vol = h * h * h;
                sphere_offsets(t.radius, t.off);
            } else {
                const double h = t.radius * std::sqrt(M_PI / 24.0);
                t.vol = h * h * t.height / 2.0;
                particle_offsets(t.radius, t.height, t.off);
            }
            t.aeq = std::pow(3.0 * t.vol / (4.0 * M_PI), 1.0 / 3.0);
            it = tmap.emplace(key, (int32_t)g->types.size()).first;
            g->types.push_back(t);
        }
        g->ptype[p] = it->second;
    }

    // nodes per level
    lat.level_map.resize(L + 1);
    g->level_nodes.resize(L + 1);
    for (int l = 0; l <= L; ++l) {
        const int sh = L - l;
        int64_t prev = INT64_MIN;
        for (int p = 0; p < N; ++p) {
            // level 0 is the single root (the paper grid's 3 x 3 level 1 has no 2 x 2 parent)
            const int64_t X = l == 0 ? 0 : lat.li[p] >> sh, Y = l == 0 ? 0 : lat.lj[p] >> sh;
            const int64_t k = key2(X, Y);
            if (k != prev || p == 0) {
                const int32_t id = (int32_t)g->nodes.size();
                g->nodes.push_back(NodeRec{l, p, 0});
                lat.node_xy.push_back({(int32_t)X, (int32_t)Y});
                lat.level_map[l][k] = id;
                g->level_nodes[l].push_back(id);
                prev = k;
            }
            g->nodes.back().count++;
        }
    }
    // blocks
    for (int l = 1; l <= L; ++l) {
        const auto& mp = lat.level_map[l];
        for (int32_t I : g->level_nodes[l]) {
            const auto xy = lat.node_xy[I];
            const int64_t PX = xy.first >> 1, PY = xy.second >> 1;
            for (int64_t dy = -1; dy <= 1; ++dy)
                for (int64_t dx = -1; dx <= 1; ++dx)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const int64_t X = 2 * (PX + dx) + a, Y = 2 * (PY + dy) + b;
                            if (X < 0 || Y < 0) continue;
                            auto it = mp.find(key2(X, Y));
                            if (it == mp.end() || it->second == I) continue;
                            const int64_t cheb = std::max(std::llabs(X - xy.first), std::llabs(Y - xy.second));
                            if (cheb >= 2 || l == L) {
                                const auto& ni = g->nodes[I];
                                const auto& nj = g->nodes[it->second];
                                g->blocks.push_back(BlockRec{l, ni.first, ni.count, nj.first, nj.count, -1,
                                                             ni.first < nj.first ? 1 : 0, I, it->second});
                            }
                        }
        }
    }
    std::sort(g->blocks.begin(), g->blocks.end(), [](const BlockRec& a, const BlockRec& b) {
        if (a.level != b.level) return a.level < b.level;
        if (a.r0 != b.r0) return a.r0 < b.r0;
        return a.c0 < b.c0;
    });

    // device upload
    const int nt = (int)g->types.size();
    std::vector<double> tvol(nt), taeq(nt), toff((size_t)nt * kCells * 3);
    std::vector<c128> tchi(nt);
    std::vector<int32_t> trep(nt, -1);
    for (int t = 0; t < nt; ++t) {
        tvol[t] = g->types[t].vol;
        taeq[t] = g->types[t].aeq;
        tchi[t] = make_double2(g->types[t].eps_re - 1.0, g->types[t].eps_im);
        std::memcpy(&toff[(size_t)t * kCells * 3], g->types[t].off, sizeof(double) * kCells * 3);
    }
    for (int p = 0; p < N; ++p)
        if (trep[g->ptype[p]] < 0) trep[g->ptype[p]] = p;
    qrvie_status st = QRVIE_OK;
    auto up = [&](void** dst, const void* src, size_t bytes, const char* what) {
        if (st != QRVIE_OK) return;
        st = dalloc(ctx, dst, bytes, what);
        if (st != QRVIE_OK) return;
        g->dev_bytes += bytes;
        st = hip_check(ctx, hipMemcpyAsync(*dst, src, bytes, hipMemcpyHostToDevice, ctx->stream), what);
    };
    up((void**)&g->d_center, g->center.data(), sizeof(double) * 3 * N, "geom centers");
    up((void**)&g->d_ptype, g->ptype.data(), sizeof(int32_t) * N, "geom types");
    up((void**)&g->d_i2c, g->i2c.data(), sizeof(int32_t) * N, "geom order");
    up((void**)&g->d_tvol, tvol.data(), sizeof(double) * nt, "geom volumes");
    up((void**)&g->d_taeq, taeq.data(), sizeof(double) * nt, "geom radii");
    up((void**)&g->d_tchi, tchi.data(), sizeof(c128) * nt, "geom chi");
    up((void**)&g->d_toff, toff.data(), sizeof(double) * toff.size(), "geom offsets");
    up((void**)&g->d_trep, trep.data(), sizeof(int32_t) * nt, "geom type representatives");
    if (st == QRVIE_OK) st = hip_check(ctx, hipStreamSynchronize(ctx->stream), "geom upload");
    {
        std::lock_guard<std::mutex> lock(lattice_mutex());
        lattices()[g] = std::move(lat);
    }
    if (st != QRVIE_OK) {
        qrvie_geom_destroy(g);
        return st;
    }
    *out = g;
    return QRVIE_OK;
}

int64_t qrvie_geom_ndof(const qrvie_geom* g) { return g ? g->ndof() : 0; }
int32_t qrvie_geom_nlevels(const qrvie_geom* g) { return g ? g->L : 0; }

qrvie_status qrvie_geom_order(const qrvie_geom* g, int32_t* i2c) {
    if (!g || !i2c) return QRVIE_ERR_INVALID_ARG;
    std::memcpy(i2c, g->i2c.data(), sizeof(int32_t) * g->N);
    return QRVIE_OK;
}

qrvie_status qrvie_geom_blocks(const qrvie_geom* g, int32_t* block_ij) {
    if (!g || !block_ij) return QRVIE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(lattice_mutex());
    const auto& lat = lattices().at(g);
    for (int p = 0; p < g->N; ++p) {
        block_ij[2 * g->i2c[p]] = lat.li[p];
        block_ij[2 * g->i2c[p] + 1] = lat.lj[p];
    }
    return QRVIE_OK;
}

qrvie_status qrvie_geom_cells(const qrvie_geom* g, double* centers, double* volumes) {
    if (!g) return QRVIE_ERR_INVALID_ARG;
    for (int p = 0; p < g->N; ++p) {
        const int c = g->i2c[p];
        const PType& t = g->types[g->ptype[p]];
        for (int cell = 0; cell < kCells; ++cell) {
            const size_t o = (size_t)c * kCells + cell;
            if (centers)
                for (int a = 0; a < 3; ++a) centers[3 * o + a] = g->center[3 * p + a] + t.off[3 * cell + a];
            if (volumes) volumes[o] = t.vol;
        }
    }
    return QRVIE_OK;
}

void qrvie_geom_destroy(qrvie_geom* g) {
    if (!g) return;
    qrvie_ctx* ctx = g->ctx;
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    const int nt = (int)g->types.size();
    dfree(ctx, g->d_center, sizeof(double) * 3 * g->N);
    dfree(ctx, g->d_ptype, sizeof(int32_t) * g->N);
    dfree(ctx, g->d_i2c, sizeof(int32_t) * g->N);
    dfree(ctx, g->d_tvol, sizeof(double) * nt);
    dfree(ctx, g->d_taeq, sizeof(double) * nt);
    dfree(ctx, g->d_tchi, sizeof(c128) * nt);
    dfree(ctx, g->d_toff, sizeof(double) * nt * kCells * 3);
    dfree(ctx, g->d_trep, sizeof(int32_t) * nt);
    {
        std::lock_guard<std::mutex> lock(lattice_mutex());
        lattices().erase(g);
    }
    delete g;
}

qrvie_status qrvie_assemble(qrvie_ctx* ctx, const qrvie_geom* g, int32_t nr, const int32_t* rows, int32_t nc,
                            const int32_t* cols, qrvie_c128* B, int64_t ldb) {
    if (!ctx || !g || !rows || !cols || !B || nr < 1 || nc < 1 || ldb < (int64_t)nr * kNp) {
        if (ctx) set_err(ctx, "assemble: invalid argument");
        return QRVIE_ERR_INVALID_ARG;
    }
    std::vector<int32_t> ri(nr), ci(nc);
    for (int a = 0; a < nr; ++a) {
        if (rows[a] < 0 || rows[a] >= g->N) { set_err(ctx, "assemble: row particle out of range"); return QRVIE_ERR_INVALID_ARG; }
        ri[a] = g->c2i[rows[a]];
    }
    for (int a = 0; a < nc; ++a) {
        if (cols[a] < 0 || cols[a] >= g->N) { set_err(ctx, "assemble: column particle out of range"); return QRVIE_ERR_INVALID_ARG; }
        ci[a] = g->c2i[cols[a]];
    }
    int32_t *dr = nullptr, *dc = nullptr;
    qrvie_status st = dalloc(ctx, (void**)&dr, sizeof(int32_t) * nr, "assemble rows");
    if (st == QRVIE_OK) st = dalloc(ctx, (void**)&dc, sizeof(int32_t) * nc, "assemble cols");
    if (st == QRVIE_OK) st = hip_check(ctx, hipMemcpyAsync(dr, ri.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice, ctx->stream), "assemble");
    if (st == QRVIE_OK) st = hip_check(ctx, hipMemcpyAsync(dc, ci.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, ctx->stream), "assemble");
    if (st == QRVIE_OK) {
        launch_assemble_lists(ctx->stream, g, dr, nr, dc, nc, (c128*)B, ldb);
        st = hip_check(ctx, hipGetLastError(), "assemble launch");
    }
    if (st == QRVIE_OK) st = hip_check(ctx, hipStreamSynchronize(ctx->stream), "assemble");
    dfree(ctx, dr, sizeof(int32_t) * nr);
    dfree(ctx, dc, sizeof(int32_t) * nc);
    return st;
}

qrvie_status qrvie_rhs_plane_waves(qrvie_ctx* ctx, const qrvie_geom* g, int32_t nrhs, const double* theta_deg,
                                   const double* phi_deg, const int32_t* pol, qrvie_c128* v, int64_t ldv) {
    if (!ctx || !g || !theta_deg || !phi_deg || !pol || !v || nrhs < 1 || ldv < g->ndof()) {
        if (ctx) set_err(ctx, "rhs_plane_waves: invalid argument");
        return QRVIE_ERR_INVALID_ARG;
    }
    std::vector<double> par(6 * (size_t)nrhs);
    for (int r = 0; r < nrhs; ++r) {
        if (!std::isfinite(theta_deg[r]) || !std::isfinite(phi_deg[r]) || (pol[r] != 0 && pol[r] != 1)) {
            set_err(ctx, "rhs_plane_waves: bad angle or polarisation");
            return QRVIE_ERR_INVALID_ARG;
        }
        const double t = theta_deg[r] * M_PI / 180.0, f = phi_deg[r] * M_PI / 180.0;
        double* p = &par[6 * r];
        p[0] = std::sin(t) * std::cos(f); p[1] = std::sin(t) * std::sin(f); p[2] = std::cos(t);
        if (pol[r] == 0) { p[3] = -std::sin(f); p[4] = std::cos(f); p[5] = 0.0; }
        else { p[3] = std::cos(t) * std::cos(f); p[4] = std::cos(t) * std::sin(f); p[5] = -std::sin(t); }
    }
    double* dpar = nullptr;
    qrvie_status st = dalloc(ctx, (void**)&dpar, sizeof(double) * par.size(), "rhs params");
    if (st == QRVIE_OK) st = hip_check(ctx, hipMemcpyAsync(dpar, par.data(), sizeof(double) * par.size(), hipMemcpyHostToDevice, ctx->stream), "rhs");
    if (st == QRVIE_OK) {
        launch_rhs(ctx->stream, g, nrhs, dpar, (c128*)v, ldv);
        st = hip_check(ctx, hipGetLastError(), "rhs launch");
    }
    if (st == QRVIE_OK) st = hip_check(ctx, hipStreamSynchronize(ctx->stream), "rhs");
    dfree(ctx, dpar, sizeof(double) * par.size());
    return st;
}

}  // extern "C"
