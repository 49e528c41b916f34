// Host side of the projector: geometry validation, the FP64 per-ray tables
// (stored as exact 32.32 fixed point), their per-device cache, errors and
// library-owned device buffers.
#include <cmath>
#include <cstring>
#include <limits>

#include "common.h"

namespace dect {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

dect_status fail(dect_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

const char *last_error() { return g_last_error.c_str(); }

// ------------------------------------------- device memory, workspace ---
namespace {

struct Arena {
    int device;
    unsigned char *base;
    size_t bytes, used;
};

std::mutex g_arena_mu;
std::vector<Arena> g_arenas;  // at most one per device
thread_local SizingScope *g_sizing = nullptr;

constexpr size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

SizingScope::SizingScope() { g_sizing = this; }

SizingScope::~SizingScope()
{
    tables.clear();  // still counting: their frees do nothing
    g_sizing = nullptr;
}

bool sizing_active() { return g_sizing != nullptr; }

dect_status dev_alloc(void **p, size_t n)
{
    *p = nullptr;
    if (n == 0) return DECT_OK;
    const size_t a = align256(n);
    if (g_sizing) {
        g_sizing->bytes += a;
        *p = (void *)g_sizing->next;
        g_sizing->next += a;
        return DECT_OK;
    }
    int dev = 0;
    DECT_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lk(g_arena_mu);
        for (auto &ar : g_arenas)
            if (ar.device == dev) {
                if (ar.bytes - ar.used < a)
                    return fail(DECT_ERR_INVALID_ARG,
                                "caller workspace exhausted: " + std::to_string(ar.used) + " of " +
                                    std::to_string(ar.bytes) + " bytes used, " +
                                    std::to_string(a) + " more needed");
                *p = ar.base + ar.used;
                ar.used += a;
                return DECT_OK;
            }
    }
    DECT_HIP(hipMalloc(p, n));
    return DECT_OK;
}

void dev_free(void *p)
{
    if (!p || g_sizing) return;
    {
        std::lock_guard<std::mutex> lk(g_arena_mu);
        for (auto &ar : g_arenas)
            if ((unsigned char *)p >= ar.base && (unsigned char *)p < ar.base + ar.bytes) return;
    }
    (void)hipFree(p);
}

dect_status set_workspace(void *p, size_t bytes)
{
    if ((p == nullptr) != (bytes == 0))
        return fail(DECT_ERR_INVALID_ARG, "dect_set_workspace: give both a pointer and a size, or neither");
    if (((uintptr_t)p & 255) != 0)
        return fail(DECT_ERR_INVALID_ARG, "dect_set_workspace: the workspace must be 256-byte aligned");
    int dev = 0;
    DECT_HIP(hipGetDevice(&dev));
    DECT_HIP(hipDeviceSynchronize());
    // every buffer the library holds on this device goes first, while the old
    // workspace (if any) is still known, so its pieces are not passed to hipFree
    release_device_buffers();
    std::lock_guard<std::mutex> lk(g_arena_mu);
    for (auto it = g_arenas.begin(); it != g_arenas.end();) {
        if (it->device == dev) it = g_arenas.erase(it);
        else ++it;
    }
    if (p) g_arenas.push_back(Arena{dev, (unsigned char *)p, bytes, 0});
    return DECT_OK;
}

dect_status workspace_used(size_t *bytes)
{
    if (!bytes) return fail(DECT_ERR_INVALID_ARG, "dect_workspace_used: bytes is NULL");
    int dev = 0;
    DECT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_arena_mu);
    *bytes = 0;
    for (auto &ar : g_arenas)
        if (ar.device == dev) *bytes = ar.used;
    return DECT_OK;
}

// ------------------------------------------------------------ DevBuf ---
dect_status DevBuf::ensure(size_t n, bool zero)
{
    if (n <= bytes && ptr) return DECT_OK;
    if (ptr) {
        if (!g_sizing) (void)hipDeviceSynchronize();
        dev_free(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    if (n == 0) return DECT_OK;
    dect_status st = dev_alloc(&ptr, n);
    if (st) return st;
    bytes = n;
    if (zero && !g_sizing) DECT_HIP(hipMemset(ptr, 0, n));
    return DECT_OK;
}

DevBuf::~DevBuf() { dev_free(ptr); }

// ---------------------------------------------------------- geometry ---
bool GeomKey::operator==(const GeomKey &o) const
{
    return nx == o.nx && ny == o.ny && V == o.V && B == o.B && model == o.model && pixel == o.pixel &&
           bin == o.bin && off == o.off && sod == o.sod && sdd == o.sdd && angles == o.angles &&
           device == o.device;
}

GeomTables::~GeomTables()
{
    dev_free(fwd);
    dev_free(len);
    dev_free(bundles);
    dev_free(views);
    dev_free(adj_bins);
    dev_free(adj_lanes);
    dev_free(sid);
}

dect_status validate_geometry(const dect_geometry *g)
{
    if (!g) return fail(DECT_ERR_INVALID_ARG, "geometry is NULL");
    if (g->nx <= 0 || g->ny <= 0 || g->n_views <= 0 || g->n_bins <= 0)
        return fail(DECT_ERR_INVALID_ARG, "geometry sizes must be positive");
    if (g->model != DECT_JOSEPH && g->model != DECT_SIDDON)
        return fail(DECT_ERR_INVALID_ARG, "geometry model must be DECT_JOSEPH or DECT_SIDDON");
    if (g->nx > 16384 || g->ny > 16384 || g->n_bins > (1 << 20) || g->n_views > (1 << 20))
        return fail(DECT_ERR_INVALID_ARG, "geometry sizes exceed the supported maximum");
    if (!(g->pixel_mm > 0.0) || !(g->bin_mm > 0.0) || !std::isfinite(g->pixel_mm) ||
        !std::isfinite(g->bin_mm) || !std::isfinite(g->det_offset_mm))
        return fail(DECT_ERR_INVALID_ARG, "pixel and bin sizes must be positive and finite");
    double hx = 0.5 * g->nx * g->pixel_mm, hy = 0.5 * g->ny * g->pixel_mm;
    double half_diag = std::sqrt(hx * hx + hy * hy);
    if (!(g->sod_mm > half_diag) || !std::isfinite(g->sod_mm))
        return fail(DECT_ERR_GEOMETRY, "source orbit (SOD) must lie outside the image");
    if (!(g->sdd_mm > g->sod_mm) || !std::isfinite(g->sdd_mm))
        return fail(DECT_ERR_GEOMETRY, "SDD must exceed SOD");
    double half_fan = std::atan((0.5 * g->n_bins * g->bin_mm + std::fabs(g->det_offset_mm)) /
                                g->sdd_mm);
    if (!(half_fan < 0.25 * M_PI))
        return fail(DECT_ERR_GEOMETRY, "fan angle must be below 90 degrees");
    if (g->angles_rad)
        for (int v = 0; v < g->n_views; ++v)
            if (!std::isfinite(g->angles_rad[v]))
                return fail(DECT_ERR_INVALID_ARG, "view angles must be finite");
    return DECT_OK;
}

static constexpr double kTwo32 = 4294967296.0;

// floor(x / 2^32) for int64 x (arithmetic shift floors).
static inline int64_t fx_floor(int64_t x) { return x >> 32; }

// Exact range of lines i in [0, n_line) with floor(q(i)) in [-1, n_q - 1].
static void valid_range(int64_t a, int64_t k, int n_line, int n_q, int *lo, int *hi)
{
    auto ok = [&](int i) {
        int64_t h = fx_floor(a + k * (int64_t)i);
        return h >= -1 && h <= n_q - 1;
    };
    // q is linear in i: locate the crossing points with a double estimate,
    // then settle them exactly with integer evaluation.
    double ad = (double)a / kTwo32, kd = (double)k / kTwo32;
    int l, h;
    if (kd == 0.0) {
        if (ok(0)) { l = 0; h = n_line - 1; }
        else { l = 1; h = 0; }
    } else {
        double t0 = (-1.0 - ad) / kd, t1 = ((double)n_q - ad) / kd;
        double tmin = std::fmin(t0, t1), tmax = std::fmax(t0, t1);
        l = (int)std::max(0.0, std::min((double)n_line - 1, std::floor(tmin)));
        h = (int)std::max(0.0, std::min((double)n_line - 1, std::ceil(tmax)));
        // widen until the outside is invalid, then shrink to valid ends
        while (l > 0 && ok(l - 1)) --l;
        while (h < n_line - 1 && ok(h + 1)) ++h;
        while (l <= h && !ok(l)) ++l;
        while (h >= l && !ok(h)) --h;
    }
    *lo = l;
    *hi = h;
}

static std::mutex g_cache_mu;
static std::vector<std::unique_ptr<GeomTables>> g_cache;

void release_tables()
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int dev = 0;
    (void)hipGetDevice(&dev);
    for (auto it = g_cache.begin(); it != g_cache.end();) {
        if ((*it)->key.device == dev) it = g_cache.erase(it);
        else ++it;
    }
}

dect_status get_tables(const dect_geometry *g, GeomTables **out)
{
    dect_status st = validate_geometry(g);
    if (st != DECT_OK) return st;
    int dev = 0;
    DECT_HIP(hipGetDevice(&dev));
    GeomKey key{g->nx, g->ny, g->n_views, g->n_bins, g->model, g->pixel_mm, g->bin_mm,
                g->det_offset_mm, g->sod_mm, g->sdd_mm, {}, dev};
    if (g->angles_rad) key.angles.assign(g->angles_rad, g->angles_rad + g->n_views);

    std::unique_lock<std::mutex> lk(g_cache_mu, std::defer_lock);
    if (g_sizing) {  // a dry run keeps its own tables and never uses the cache
        for (auto &t : g_sizing->tables)
            if (t->key == key) {
                *out = t.get();
                return DECT_OK;
            }
    } else {
        lk.lock();
        for (auto &t : g_cache)
            if (t->key == key) {
                *out = t.get();
                return DECT_OK;
            }
    }

    const int nx = g->nx, ny = g->ny, V = g->n_views, B = g->n_bins;
    const double dl = g->pixel_mm, R = g->sod_mm, D = g->sdd_mm;
    const int nb = (B + kBundle - 1) / kBundle;
    std::vector<RayFwd> fwd((size_t)V * B);
    std::vector<float> len((size_t)V * B);
    const bool siddon = g->model == DECT_SIDDON;
    std::vector<SidW> sid(siddon ? (size_t)V * B : 0);
    const int nvgrp = (V + kFwdViews - 1) / kFwdViews;
    std::vector<Bundle> bun((size_t)nvgrp * nb);
    // per ray: class and valid driving-line range
    std::vector<int> r_major((size_t)V * B), r_lo((size_t)V * B), r_hi((size_t)V * B);
    std::vector<ViewInfo> views(V);
    int64_t samples = 0;

    for (int v = 0; v < V; ++v) {
        double th = g->angles_rad ? g->angles_rad[v] : 2.0 * M_PI * v / V;
        double ct = std::cos(th), st = std::sin(th);
        double sx = R * ct, sy = R * st;
        std::vector<int> major(B), lo(B), hi(B);
        for (int b = 0; b < B; ++b) {
            double u = (b - (B - 1) / 2.0) * g->bin_mm + g->det_offset_mm;
            double px = -(D - R) * ct - u * st, py = -(D - R) * st + u * ct;
            double dx = px - sx, dy = py - sy;
            double ln = std::sqrt(dx * dx + dy * dy);
            bool xm = std::fabs(dx) >= std::fabs(dy);
            double a, k, L;
            if (xm) {  // q = row coordinate on column c
                k = dy / dx;
                double x0 = (0 - (nx - 1) / 2.0) * dl;
                a = (sy + (x0 - sx) * k) / dl + (ny - 1) / 2.0;
                L = dl * ln / std::fabs(dx);
            } else {   // q = column coordinate on row r
                k = dx / dy;
                double y0 = (0 - (ny - 1) / 2.0) * dl;
                a = (sx + (y0 - sy) * k) / dl + (nx - 1) / 2.0;
                L = dl * ln / std::fabs(dy);
            }
            if (!(std::fabs(a) < 1e6)) a = std::copysign(1e6, a);  // ray far outside
            int64_t afx = (int64_t)std::llround(a * kTwo32);
            int64_t kfx = (int64_t)std::llround(k * kTwo32);
            size_t i = (size_t)v * B + b;
            if (siddon) {
                // |k| <= 1 on the driving axis, so |k_fx| <= 2^32
                const int64_t kabs = kfx < 0 ? -kfx : kfx;
                afx += (int64_t(1) << 31) - (kabs >> 1);
                sid[i].c = kabs ? (uint32_t)((int64_t(1) << 32) - kabs) : 0xFFFFFFFFu;
                sid[i].inv = kabs ? (float)(kTwo32 / (double)kabs) : 0.0f;
            }
            fwd[i] = {afx, kfx};
            len[i] = xm ? (float)L : -(float)L;  // sign marks the class
            major[b] = xm;
            valid_range(afx, kfx, xm ? nx : ny, xm ? ny : nx, &lo[b], &hi[b]);
            // samples with q strictly inside (-1, n): exclude q == -1 exactly
            for (int c = lo[b]; c <= hi[b]; ++c) {
                int64_t q = afx + kfx * (int64_t)c;
                if (q != -(int64_t(1) << 32)) ++samples;
            }
        }
        // class ranges: at most one switch between x-major and y-major bins
        int switches = 0;
        for (int b = 1; b < B; ++b) switches += major[b] != major[b - 1];
        if (switches > 1)
            return fail(DECT_ERR_GEOMETRY, "ray classes are not contiguous within a view");
        ViewInfo vi{(float)ct, (float)st, 0, 0, 0, 0, 0, 0};
        int first_x = -1, last_x = -2, first_y = -1, last_y = -2;
        for (int b = 0; b < B; ++b) {
            if (major[b]) { if (first_x < 0) first_x = b; last_x = b; }
            else { if (first_y < 0) first_y = b; last_y = b; }
        }
        vi.xb0 = first_x < 0 ? 0 : first_x;
        vi.xb1 = first_x < 0 ? 0 : last_x + 1;
        vi.yb0 = first_y < 0 ? 0 : first_y;
        vi.yb1 = first_y < 0 ? 0 : last_y + 1;
        views[v] = vi;
        for (int b = 0; b < B; ++b) {
            r_major[(size_t)v * B + b] = major[b];
            r_lo[(size_t)v * B + b] = lo[b];
            r_hi[(size_t)v * B + b] = hi[b];
        }
    }
    // forward bundles: per (group of kFwdViews views, kBundle bins), the union
    // of the rays' valid line ranges per class
    for (int gi = 0; gi < nvgrp; ++gi)
        for (int j = 0; j < nb; ++j) {
            Bundle bb{1 << 30, -(1 << 30), 1 << 30, -(1 << 30)};
            for (int v = gi * kFwdViews; v < std::min(V, (gi + 1) * kFwdViews); ++v)
                for (int b = j * kBundle; b < std::min(B, (j + 1) * kBundle); ++b) {
                    const size_t i = (size_t)v * B + b;
                    if (r_lo[i] > r_hi[i]) continue;
                    if (r_major[i]) { bb.x0 = std::min(bb.x0, r_lo[i]); bb.x1 = std::max(bb.x1, r_hi[i]); }
                    else { bb.y0 = std::min(bb.y0, r_lo[i]); bb.y1 = std::max(bb.y1, r_hi[i]); }
                }
            if (bb.x0 > bb.x1) { bb.x0 = 1; bb.x1 = 0; }
            if (bb.y0 > bb.y1) { bb.y0 = 1; bb.y1 = 0; }
            bun[(size_t)gi * nb + j] = bb;
        }

    // Adjoint bin ranges: for every strip and view, the bins of the strip's
    // ray class whose rays put a tap inside the strip.  A first guess comes
    // from projecting the strip's corners onto the detector; both ends are
    // then settled exactly on the fixed-point ray table (a ray hits the strip
    // when its line coordinate q, linear along the lane axis, enters the tap
    // interval (t0 - 1, t0 + kSW) somewhere on the strip's lanes).
    const int nsx = adj_strips_x(nx, ny), nst = adj_strips(nx, ny);
    // the adjoint's tables stay below 4 GiB each (2048^2 x 720 views needs
    // 1.5 GB of lane ranges; HBM holds 288 GB)
    if ((double)nst * V * sizeof(BinRange) > (double)(size_t(1) << 32))
        return fail(DECT_ERR_GEOMETRY, "geometry too large for the back-projector's bin table");
    std::vector<BinRange> bins((size_t)nst * V);
    const int64_t one = int64_t(1) << 32;
    for (int v = 0; v < V; ++v) {
        const double th = g->angles_rad ? g->angles_rad[v] : 2.0 * M_PI * v / V;
        const double ct = std::cos(th), st = std::sin(th);
        auto beta = [&](double px, double py) {
            const double pu = -px * st + py * ct, ps = px * ct + py * st;
            return (D * pu / (R - ps) - g->det_offset_mm) / g->bin_mm + (B - 1) / 2.0;
        };
        for (int sI = 0; sI < nst; ++sI) {
            const int cls = sI < nsx ? 0 : 1, sidx = cls ? sI - nsx : sI;
            const int nL = cls ? ny : nx, nT = cls ? nx : ny;
            const int nsL = (nL + kSL - 1) / kSL;
            const int t0 = (sidx / nsL) * kSW, l0 = (sidx % nsL) * kSL;
            const int l1 = std::min(l0 + kSL - 1, nL - 1);
            const int cb0 = cls ? views[v].yb0 : views[v].xb0;
            const int cb1 = cls ? views[v].yb1 : views[v].xb1;
            BinRange r{1, 0, 0, 0};
            if (cb0 < cb1) {
                const int64_t qlo = (int64_t)(t0 - 1) * one, qhi = (int64_t)(t0 + kSW) * one;
                auto hit = [&](int b) {
                    const RayFwd &f = fwd[(size_t)v * B + b];
                    const int64_t qa = f.a_fx + f.k_fx * l0, qb = f.a_fx + f.k_fx * l1;
                    return std::max(qa, qb) > qlo && std::min(qa, qb) < qhi;
                };
                auto mm = [&](int i, int n) { return (i - (n - 1) / 2.0) * dl; };
                double bmin = 1e300, bmax = -1e300;
                for (int li : {l0, l1})
                    for (int ti : {t0 - 1, std::min(t0 + kSW, nT)}) {
                        const double px = cls ? mm(ti, nx) : mm(li, nx);
                        const double py = cls ? mm(li, ny) : mm(ti, ny);
                        const double bb = beta(px, py);
                        bmin = std::min(bmin, bb);
                        bmax = std::max(bmax, bb);
                    }
                int lo = (int)std::max((double)cb0, std::min((double)cb1 - 1, std::floor(bmin) - 2));
                int hi = (int)std::max((double)cb0, std::min((double)cb1 - 1, std::ceil(bmax) + 2));
                while (lo <= hi && !hit(lo)) ++lo;
                while (hi >= lo && !hit(hi)) --hi;
                if (lo > hi) {  // the guess missed: scan the class range
                    for (int b = cb0; b < cb1; ++b)
                        if (hit(b)) {
                            if (lo > hi) lo = hi = b;
                            else hi = b;
                        }
                }
                if (lo <= hi) {
                    while (lo > cb0 && hit(lo - 1)) --lo;
                    while (hi < cb1 - 1 && hit(hi + 1)) ++hi;
                    r = BinRange{lo, hi, 64, 0};
                }
            }
            bins[(size_t)sI * V + v] = r;
        }
    }

    // Per-lane bin ranges inside each strip range.  At a fixed driving line
    // the rays of one view are ordered (they meet only at the source, outside
    // the image), so the line coordinate q is monotone in the bin index and
    // the bins with t0 - 1 < q < t0 + kSW form one interval, whose ends are
    // walked from the previous lane's.  A bin outside it adds nothing to the
    // strip's lines at that lane (q exactly t0 - 1 gives the line t0 weight
    // zero).  Ranges are stored relative to the strip's lo as bytes; a strip
    // range of more than 256 bins stores none (the kernel then gives every
    // lane the whole range, a superset, which changes no result).
    if ((double)nst * V * kSL * sizeof(LaneRange) > (double)(size_t(1) << 32))
        return fail(DECT_ERR_GEOMETRY, "geometry too large for the back-projector's lane table");
    std::vector<LaneRange> lanes((size_t)nst * V * kSL, LaneRange{1, 0});
    for (int sI = 0; sI < nst; ++sI) {
        const int cls = sI < nsx ? 0 : 1, sidx = cls ? sI - nsx : sI;
        const int nL = cls ? ny : nx;
        const int nsL = (nL + kSL - 1) / kSL;
        const int t0 = (sidx / nsL) * kSW, l0 = (sidx % nsL) * kSL;
        const int64_t qlo = (int64_t)(t0 - 1) * one, qhi = (int64_t)(t0 + kSW) * one;
        for (int v = 0; v < V; ++v) {
            BinRange &r = bins[(size_t)sI * V + v];
            if (r.lo > r.hi) continue;
            if (r.hi - r.lo > kLaneRangeMax) continue;  // the kernel takes the whole range
            int longest = 0;
            LaneRange *out = &lanes[((size_t)sI * V + v) * kSL];
            // boundaries of monotone predicates over [lo, hi], walked from the
            // previous lane's (they move by a few bins from lane to lane)
            int gf = r.lo, gl = r.hi;
            for (int l = 0; l < kSL && l0 + l < nL; ++l) {
                const int64_t c = l0 + l;
                auto q = [&](int b) {
                    const RayFwd &f = fwd[(size_t)v * B + b];
                    return f.a_fx + f.k_fx * c;
                };
                const bool up = q(r.hi) >= q(r.lo);
                auto below_hi = [&](int b) { return q(b) < qhi; };
                auto above_lo = [&](int b) { return q(b) > qlo; };
                // smallest b in [lo, hi + 1] where pred (false ... true) holds
                auto first_true = [&](auto pred, int g) {
                    g = std::min(std::max(g, r.lo), r.hi + 1);
                    while (g > r.lo && pred(g - 1)) --g;
                    while (g <= r.hi && !pred(g)) ++g;
                    return g;
                };
                // largest b in [lo - 1, hi] where pred (true ... false) holds
                auto last_true = [&](auto pred, int g) {
                    g = std::min(std::max(g, r.lo - 1), r.hi);
                    while (g < r.hi && pred(g + 1)) ++g;
                    while (g >= r.lo && !pred(g)) --g;
                    return g;
                };
                // in the direction q grows: the first bin past the lower
                // edge, the last before the upper one
                const int first = up ? first_true(above_lo, gf) : first_true(below_hi, gf);
                const int last = up ? last_true(below_hi, gl) : last_true(above_lo, gl);
                gf = first;
                gl = last;
                if (first <= last) {
                    out[l] = LaneRange{(uint8_t)(first - r.lo), (uint8_t)(last - r.lo)};
                    longest = std::max(longest, last - first + 1);
                }
            }
            r.steps = std::min(longest, 64);
        }
    }

    auto t = std::make_unique<GeomTables>();
    t->key = key;
    t->nbundle = nb;
    t->samples = samples;
    auto upload = [&](auto **dst, const auto &v) -> dect_status {
        const size_t n = v.size() * sizeof(v[0]);
        dect_status e = dev_alloc((void **)dst, n);
        if (e) return e;
        if (!g_sizing && n) DECT_HIP(hipMemcpy(*dst, v.data(), n, hipMemcpyHostToDevice));
        return DECT_OK;
    };
    if ((st = upload(&t->fwd, fwd)) || (st = upload(&t->len, len)) ||
        (st = upload(&t->bundles, bun)) || (st = upload(&t->views, views)) ||
        (st = upload(&t->adj_bins, bins)) || (st = upload(&t->adj_lanes, lanes)) ||
        (siddon && (st = upload(&t->sid, sid))))
        return st;
    *out = t.get();
    if (g_sizing) g_sizing->tables.push_back(std::move(t));
    else g_cache.push_back(std::move(t));
    return DECT_OK;
}

}  // namespace dect
