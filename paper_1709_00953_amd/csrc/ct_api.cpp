// Host runtime and C ABI of the block-iterative CT solver.
//
// Geometry validation and device tables, the data-independent block
// schedule of Alg. 5 / Alg. 6, the solver state (z^j, r, work buffers in the
// caller's workspace) and the epoch driver that enqueues, per column block,
// back-projection -> fused forward -> step -> finalize on the caller's stream.
#include "ct.h"
#include "ct_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <map>
#include <mutex>
#include <vector>

using namespace ct;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int ct::fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(CT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
struct ct_geom {
    ct_geom_desc d{};
    int dims = 2;
    int64_t M = 0, N = 0;
    int m = 0, n = 0;
    std::vector<double> views;         // n_views*12
    std::vector<Tile> tiles;
    std::vector<int32_t> rb_tile_ptr, tile_roff;
    std::vector<double> v64;           // float64 per-view frames [n_views][kViewStride]
    std::vector<Chunk> chunks;         // whole row blocks
    std::vector<int32_t> rb_chunk_ptr;
    std::vector<Chunk> wchunks;        // (row block, column block) windows
    std::vector<int32_t> rbj_chunk_ptr;
    std::vector<int64_t> rbj_rays;
    std::vector<int64_t> rb_rays;
    std::vector<Box> boxes;
    std::vector<int32_t> box_tiles;    // back-projection work-groups per group
    std::vector<Entry> all_entries;
    int32_t max_rb_rays = 0, max_cb_vox = 0, max_tiles = 0, total_chunks = 0, max_xg = 0;
    int32_t max_step_wchunks = 0;      // windowed chunks of all row blocks, worst column block
    int32_t vertical = 0;              // cone with detector columns along z (kConeV)
    int device = -1;
    void* dmem = nullptr;               // device tables, uploaded on first use
    bool dmem_owned = true;             // false: placed in caller memory (geom_table_bind)
    size_t dbytes = 0;
    std::mutex mu;
    DGeom G{};
    Entry* d_all = nullptr;
    unsigned long long* d_nnz = nullptr;
    Box* d_boxes = nullptr;            // [n]
    Tune tune{};                       // launch shapes of the projectors (tuner or caller)
};

static void box_tiling(const ct_geom* g, const Box& b, int* tx, int* ty, int* tz) {
    const int nxJ = b.x1 - b.x0, nyJ = b.y1 - b.y0, nzJ = b.z1 - b.z0;
    if (g->dims == 2) {
        *tx = (nxJ + kTile2 - 1) / kTile2;
        *ty = (nyJ + kTile2 - 1) / kTile2;
        *tz = 1;
    } else if (g->vertical) {
        int TZ, CX, CY;
        col_tile_shape(nzJ, TZ, CX, CY);
        *tx = (nxJ + CX - 1) / CX;
        *ty = (nyJ + CY - 1) / CY;
        *tz = (nzJ + TZ - 1) / TZ;
    } else {
        *tx = (nxJ + kTile3x - 1) / kTile3x;
        *ty = (nyJ + kTile3y - 1) / kTile3y;
        *tz = (nzJ + kTile3z - 1) / kTile3z;
    }
}

static inline double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// float64 per-view frames: a(3) c(3) e_u(3) e_v(3) n(3), then
// kappa = cross(d, e_u) (parallel) or sdd, 1/sdd, sigma = cross(n, e_u).
static void build_views(ct_geom* g) {
    const ct_geom_desc& d = g->d;
    g->v64.assign((size_t)d.n_views * kViewStride, 0.0);
    for (int k = 0; k < d.n_views; ++k) {
        const double* V = &g->views[(size_t)k * 12];
        double* W = &g->v64[(size_t)k * kViewStride];
        if (d.kind == CT_PAR2D) {
            const double na = std::hypot(V[0], V[1]);
            W[0] = V[0] / na;
            W[1] = V[1] / na;
            W[3] = V[3];
            W[4] = V[4];
            W[6] = V[6];
            W[7] = V[7];
            W[15] = W[0] * W[7] - W[1] * W[6];
        } else {
            for (int c = 0; c < 12; ++c) W[c] = V[c];
            if (g->dims == 2) W[2] = W[5] = W[8] = W[9] = W[10] = W[11] = 0.0;
            double w[3] = {W[3] - W[0], W[4] - W[1], W[5] - W[2]};
            const double sdd = std::sqrt(dot3(w, w));
            W[12] = w[0] / sdd;
            W[13] = w[1] / sdd;
            W[14] = w[2] / sdd;
            W[15] = sdd;
            W[16] = 1.0 / sdd;
            W[17] = W[12] * W[7] - W[13] * W[6];
        }
    }
}

// Detector rectangle of tile `tl` whose rays can meet box `b`: the bin
// coordinates of the box corners' projections, widened by one bin.  The
// projection of a box lying in front of the source is the hull of its
// corners' projections, so no ray outside the rectangle meets the box.
static void tile_window(const ct_geom* g, const Tile& tl, const Box& b, int* u0, int* u1, int* v0,
                        int* v1) {
    const ct_geom_desc& d = g->d;
    const double* W = &g->v64[(size_t)tl.view * kViewStride];
    const double cu = 0.5 * (d.nu - 1), cv = 0.5 * (d.nv - 1);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    const int nzc = g->dims == 3 ? 2 : 1;
    for (int cz = 0; cz < nzc; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const double p[3] = {d.ox + (cx ? b.x1 : b.x0) * d.vx, d.oy + (cy ? b.y1 : b.y0) * d.vy,
                                     g->dims == 3 ? d.oz + (cz ? b.z1 : b.z0) * d.vz : 0.0};
                double bu = 0.0, bv = cv;
                if (d.kind == CT_PAR2D) {
                    bu = (W[0] * (p[1] - W[4]) - W[1] * (p[0] - W[3])) / W[15] / d.pu + cu;
                } else {
                    const double q[3] = {p[0] - W[0], p[1] - W[1], p[2] - W[2]};
                    const double A = q[0] * W[12] + q[1] * W[13] + q[2] * W[14];
                    const double Bu = q[0] * W[6] + q[1] * W[7] + q[2] * W[8];
                    if (d.kind == CT_FAN2D_CURVED) {
                        bu = std::atan2(Bu, A) / d.pu + cu;
                    } else {
                        bu = W[15] * Bu / A / d.pu + cu;
                    }
                    if (g->dims == 3) {
                        const double Bv = q[0] * W[9] + q[1] * W[10] + q[2] * W[11];
                        bv = W[15] * Bv / A / d.pv + cv;
                    }
                }
                umin = std::min(umin, bu);
                umax = std::max(umax, bu);
                vmin = std::min(vmin, bv);
                vmax = std::max(vmax, bv);
            }
    *u0 = std::max(tl.u0, (int)std::floor(umin) - 1);
    *u1 = std::min(tl.u1, (int)std::ceil(umax) + 2);
    *v0 = std::max(tl.v0, (int)std::floor(vmin) - 1);
    *v1 = std::min(tl.v1, (int)std::ceil(vmax) + 2);
    if (*u1 < *u0) *u1 = *u0;
    if (*v1 < *v0) *v1 = *v0;
}

static void build_windows(ct_geom* g) {
    g->wchunks.clear();
    g->rbj_chunk_ptr.assign(1, 0);
    g->rbj_rays.clear();
    std::vector<int32_t> per_col(g->n, 0);
    for (int b = 0; b < g->m; ++b)
        for (int J = 0; J < g->n; ++J) {
            // chunks of kChunk consecutive rays of a window (row-major, the
            // last one shorter), listed by the detector row of their first
            // ray across the row block's views: the rays of one row of
            // neighbouring views cross the same voxel planes of a 3D box, so
            // work-groups that run together reuse them from L2 (a 2D window
            // is a single row, so its list keeps the view order)
            struct Win {
                int view, u0, v0, w, h;
                int64_t roff;
            };
            std::vector<Win> wins;
            int64_t roff = 0;
            int hmax = 0;
            for (int t = g->rb_tile_ptr[b]; t < g->rb_tile_ptr[b + 1]; ++t) {
                const Tile& tl = g->tiles[t];
                int u0, u1, v0, v1;
                tile_window(g, tl, g->boxes[J], &u0, &u1, &v0, &v1);
                if (u1 <= u0 || v1 <= v0) continue;
                wins.push_back(Win{tl.view, u0, v0, u1 - u0, v1 - v0, roff});
                roff += (int64_t)(u1 - u0) * (v1 - v0);
                hmax = std::max(hmax, v1 - v0);
            }
            const size_t before = g->wchunks.size();
            std::vector<int64_t> next(wins.size(), 0);       // first ray of each window's next chunk
            for (int r = 0; r < hmax; ++r)
                for (size_t i = 0; i < wins.size(); ++i) {
                    const Win& wn = wins[i];
                    const int64_t nr = (int64_t)wn.w * wn.h;
                    for (int64_t& k0 = next[i]; k0 < nr && k0 / wn.w == r; k0 += kChunk)
                        g->wchunks.push_back(Chunk{wn.view, wn.u0, wn.v0, wn.w, (int32_t)k0,
                                                   (int32_t)std::min<int64_t>(kChunk, nr - k0),
                                                   (int32_t)(wn.roff + k0), 0});
                }
            per_col[J] += (int32_t)(g->wchunks.size() - before);
            g->rbj_chunk_ptr.push_back((int32_t)g->wchunks.size());
            g->rbj_rays.push_back(roff);
        }
    g->max_step_wchunks = 0;
    for (int J = 0; J < g->n; ++J) g->max_step_wchunks = std::max(g->max_step_wchunks, per_col[J]);
}

// Validate the description and fill the host-side tables.
static int build_host(ct_geom* g, const ct_geom_desc* d) {
    if (!d) return fail(CT_EINVAL, "desc is NULL");
    if (d->kind < CT_PAR2D || d->kind > CT_CONE3D_FLAT) return fail(CT_EINVAL, "bad kind %d", d->kind);
    g->dims = (d->kind == CT_CONE3D_FLAT) ? 3 : 2;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->nu < 1 || d->nv < 1 || d->n_views < 1)
        return fail(CT_EINVAL, "non-positive size");
    if (g->dims == 2 && (d->nz != 1 || d->nv != 1)) return fail(CT_EINVAL, "2D kinds need nz = nv = 1");
    if (!(d->vx > 0 && d->vy > 0 && d->vz > 0 && d->pu > 0 && d->pv > 0))
        return fail(CT_EINVAL, "non-positive pitch");
    if (!std::isfinite(d->ox) || !std::isfinite(d->oy) || !std::isfinite(d->oz))
        return fail(CT_EINVAL, "non-finite origin");
    if (!d->views || !d->rb_ptr || !d->tiles || !d->boxes) return fail(CT_EINVAL, "NULL array");
    if (d->n_row_blocks < 1 || d->n_col_blocks < 1) return fail(CT_EINVAL, "need >= 1 block");
    const int64_t M = (int64_t)d->n_views * d->nv * d->nu;
    const int64_t N = (int64_t)d->nx * d->ny * d->nz;
    if (M > INT32_MAX || N > INT32_MAX) return fail(CT_EUNSUPPORTED, "more than 2^31 rays or voxels");
    g->d = *d;
    g->d.views = nullptr;
    g->d.rb_ptr = nullptr;
    g->d.tiles = nullptr;
    g->d.boxes = nullptr;
    g->M = M;
    g->N = N;
    g->m = d->n_row_blocks;
    g->n = d->n_col_blocks;
    g->views.assign(d->views, d->views + (size_t)d->n_views * 12);
    for (double v : g->views)
        if (!std::isfinite(v)) return fail(CT_EINVAL, "non-finite view vector");

    // per-view checks
    const double hx = 0.5 * d->vx, hy = 0.5 * d->vy, hz = g->dims == 3 ? 0.5 * d->vz : 0.0;
    const double R = std::sqrt(hx * hx + hy * hy + hz * hz);
    for (int k = 0; k < d->n_views; ++k) {
        const double* V = &g->views[(size_t)k * 12];
        double a[3] = {V[0], V[1], g->dims == 3 ? V[2] : 0.0};
        double c[3] = {V[3], V[4], g->dims == 3 ? V[5] : 0.0};
        double eu[3] = {V[6], V[7], g->dims == 3 ? V[8] : 0.0};
        double ev[3] = {V[9], V[10], V[11]};
        if (std::fabs(std::sqrt(dot3(eu, eu)) - 1.0) > 1e-9) return fail(CT_EINVAL, "view %d: e_u not unit", k);
        if (d->kind == CT_PAR2D) {
            const double na = std::sqrt(dot3(a, a));
            if (!(na > 0)) return fail(CT_EINVAL, "view %d: zero ray direction", k);
            const double kap = (a[0] * eu[1] - a[1] * eu[0]) / na;
            if (std::fabs(kap) < 1e-9) return fail(CT_EINVAL, "view %d: detector parallel to rays", k);
        } else {
            double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            const double sdd = std::sqrt(dot3(w, w));
            if (!(sdd > 0)) return fail(CT_EINVAL, "view %d: source on detector centre", k);
            if (std::fabs(dot3(w, eu)) > 1e-9 * sdd) return fail(CT_EINVAL, "view %d: e_u not perpendicular", k);
            if (g->dims == 3) {
                if (std::fabs(std::sqrt(dot3(ev, ev)) - 1.0) > 1e-9) return fail(CT_EINVAL, "view %d: e_v not unit", k);
                if (std::fabs(dot3(w, ev)) > 1e-9 * sdd || std::fabs(dot3(eu, ev)) > 1e-9)
                    return fail(CT_EINVAL, "view %d: e_v not perpendicular", k);
            }
            // the whole volume must lie in front of the source by more than a voxel
            double nrm[3] = {w[0] / sdd, w[1] / sdd, w[2] / sdd};
            double dmin = INFINITY;
            for (int cz = 0; cz < (g->dims == 3 ? 2 : 1); ++cz)
                for (int cy = 0; cy < 2; ++cy)
                    for (int cx = 0; cx < 2; ++cx) {
                        double p[3] = {d->ox + cx * d->nx * d->vx - a[0], d->oy + cy * d->ny * d->vy - a[1],
                                       g->dims == 3 ? d->oz + cz * d->nz * d->vz - a[2] : 0.0};
                        dmin = std::min(dmin, dot3(p, nrm));
                    }
            if (!(dmin > R * (1 + 1e-6) + 1e-9))
                return fail(CT_EINVAL, "view %d: volume not entirely in front of the source", k);
        }
    }

    // cone views whose detector columns run along z (e_v = +-z, e_u and the
    // source-detector axis in the xy plane): the voxel-column back-projection
    g->vertical = 0;
    if (g->dims == 3) {
        bool vert = true;
        for (int k = 0; k < d->n_views && vert; ++k) {
            const double* V = &g->views[(size_t)k * 12];
            vert = V[9] == 0.0 && V[10] == 0.0 && std::fabs(V[11]) == 1.0 && V[8] == 0.0 && V[5] == V[2];
        }
        g->vertical = vert ? 1 : 0;
    }

    // row blocks: tiles, coverage
    std::vector<uint8_t> cover((size_t)M, 0);
    g->rb_tile_ptr.assign(1, 0);
    g->rb_chunk_ptr.assign(1, 0);
    g->rb_rays.clear();
    const int32_t* rp = d->rb_ptr;
    if (rp[0] != 0) return fail(CT_EINVAL, "rb_ptr[0] != 0");
    for (int b = 0; b < g->m; ++b) {
        if (rp[b + 1] <= rp[b]) return fail(CT_EINVAL, "row block %d has no tiles", b);
        int64_t roff = 0;
        for (int t = rp[b]; t < rp[b + 1]; ++t) {
            const int32_t* T = d->tiles + (size_t)t * 5;
            Tile tl{T[0], T[1], T[2], T[3], T[4]};
            if (tl.view < 0 || tl.view >= d->n_views || tl.u0 < 0 || tl.u1 > d->nu || tl.u0 >= tl.u1 ||
                tl.v0 < 0 || tl.v1 > d->nv || tl.v0 >= tl.v1)
                return fail(CT_EINVAL, "tile %d out of range", t);
            for (int iv = tl.v0; iv < tl.v1; ++iv)
                for (int iu = tl.u0; iu < tl.u1; ++iu) {
                    uint8_t& cv = cover[((size_t)tl.view * d->nv + iv) * d->nu + iu];
                    if (cv) return fail(CT_EINVAL, "row blocks overlap at tile %d", t);
                    cv = 1;
                }
            const int tid = (int)g->tiles.size();
            g->tiles.push_back(tl);
            g->tile_roff.push_back((int32_t)roff);
            const int64_t nr = (int64_t)(tl.u1 - tl.u0) * (tl.v1 - tl.v0);
            (void)tid;
            for (int64_t k0 = 0; k0 < nr; k0 += kChunk) {
                Chunk ch{tl.view, tl.u0, tl.v0, tl.u1 - tl.u0, (int32_t)k0,
                         (int32_t)std::min<int64_t>(kChunk, nr - k0), (int32_t)(roff + k0), 0};
                g->chunks.push_back(ch);
            }
            roff += nr;
        }
        g->rb_tile_ptr.push_back((int32_t)g->tiles.size());
        g->rb_chunk_ptr.push_back((int32_t)g->chunks.size());
        g->rb_rays.push_back(roff);
        g->max_rb_rays = std::max<int32_t>(g->max_rb_rays, (int32_t)roff);
    }
    for (int64_t i = 0; i < M; ++i)
        if (!cover[i]) return fail(CT_EINVAL, "row blocks do not cover ray %lld", (long long)i);
    g->total_chunks = (int32_t)g->chunks.size();

    // column blocks: boxes, coverage
    std::vector<uint8_t> vc((size_t)N, 0);
    for (int b = 0; b < g->n; ++b) {
        const int32_t* B = d->boxes + (size_t)b * 6;
        Box bx{B[0], B[1], B[2], B[3], B[4], B[5]};
        if (bx.x0 < 0 || bx.x1 > d->nx || bx.x0 >= bx.x1 || bx.y0 < 0 || bx.y1 > d->ny || bx.y0 >= bx.y1 ||
            bx.z0 < 0 || bx.z1 > d->nz || bx.z0 >= bx.z1)
            return fail(CT_EINVAL, "box %d out of range", b);
        for (int iz = bx.z0; iz < bx.z1; ++iz)
            for (int iy = bx.y0; iy < bx.y1; ++iy)
                for (int ix = bx.x0; ix < bx.x1; ++ix) {
                    uint8_t& cv = vc[((size_t)iz * d->ny + iy) * d->nx + ix];
                    if (cv) return fail(CT_EINVAL, "column blocks overlap (box %d)", b);
                    cv = 1;
                }
        g->boxes.push_back(bx);
        const int64_t nv = (int64_t)(bx.x1 - bx.x0) * (bx.y1 - bx.y0) * (bx.z1 - bx.z0);
        g->max_cb_vox = std::max<int32_t>(g->max_cb_vox, (int32_t)nv);
        g->max_xg = std::max(g->max_xg, xg_size(bx.x1 - bx.x0, bx.y1 - bx.y0, bx.z1 - bx.z0));
        int tx, ty, tz;
        box_tiling(g, bx, &tx, &ty, &tz);
        g->box_tiles.push_back(tx * ty * tz);
        g->max_tiles = std::max(g->max_tiles, tx * ty * tz);
    }
    for (int64_t i = 0; i < N; ++i)
        if (!vc[i]) return fail(CT_EINVAL, "column blocks do not cover voxel %lld", (long long)i);

    build_views(g);
    build_windows(g);

    // all-row-block launch entries
    g->all_entries.clear();
    int32_t cp = 0, sp = 0;
    for (int b = 0; b < g->m; ++b) {
        g->all_entries.push_back(Entry{b, 0, cp, sp});
        cp += g->rb_chunk_ptr[b + 1] - g->rb_chunk_ptr[b];
        sp += (int32_t)g->rb_rays[b];
    }
    return CT_OK;
}

// 2D per-ray constants and per-view zero-direction flags.
static void build_frames(const ct_geom* g, std::vector<Ray2F>& rayf, std::vector<Ray2B>& rayb,
                         std::vector<Ray2K>& rayk, std::vector<int32_t>& flags) {
    const ct_geom_desc& d = g->d;
    flags.assign(d.n_views, 0);
    const double hx = 0.5 * d.vx, hy = 0.5 * d.vy;
    if (g->dims == 2) {
        rayf.assign((size_t)d.n_views * d.nu, Ray2F{});
        rayb.assign((size_t)d.n_views * d.nu, Ray2B{});
        rayk.assign((size_t)d.n_views * d.nu, Ray2K{});
    }
    for (int k = 0; k < d.n_views; ++k) {
        const double* W = &g->v64[(size_t)k * kViewStride];
        if (g->dims == 2) {
            for (int iu = 0; iu < d.nu; ++iu) {
                const double u = ((double)iu - 0.5 * (double)(d.nu - 1)) * d.pu;
                Ray2B& R = rayb[(size_t)k * d.nu + iu];
                Ray2F& F = rayf[(size_t)k * d.nu + iu];
                double dx, dy;
                if (d.kind == CT_PAR2D) {
                    dx = W[0];
                    dy = W[1];
                    R.p = 1.0;
                    R.q = u * W[15];
                } else if (d.kind == CT_FAN2D_CURVED) {
                    const double cg = std::cos(u), sg = std::sin(u);
                    dx = cg * W[12] + sg * W[6];
                    dy = cg * W[13] + sg * W[7];
                    R.p = W[17] * cg;
                    R.q = W[17] * sg;
                } else {
                    const double sdd = W[15];
                    const double nD = std::hypot(sdd, u);
                    dx = (sdd * W[12] + u * W[6]) / nD;
                    dy = (sdd * W[13] + u * W[7]) / nD;
                    R.p = W[17] * sdd / nD;
                    R.q = W[17] * u / nD;
                }
                if (std::fabs(dx) <= kAxisEps) dx = 0.0;
                if (std::fabs(dy) <= kAxisEps) dy = 0.0;
                F.dx = dx;
                F.dy = dy;
                F.idx = dx != 0.0 ? 1.0 / dx : 0.0;
                F.idy = dy != 0.0 ? 1.0 / dy : 0.0;
                // the origin the forward walk starts from; a ray with a zero
                // component stays in its origin's slab of that axis (the
                // forward kernel's float64 half-open rule, same operations)
                const double o0 = d.kind == CT_PAR2D ? std::fma(u, W[6], W[3]) : W[0];
                const double o1 = d.kind == CT_PAR2D ? std::fma(u, W[7], W[4]) : W[1];
                auto slab = [](double o, double org, double ih) {
                    return (float)std::fmin(std::fmax(std::floor((o - org) * ih), -1e7), 1e7);
                };
                Ray2K& Q = rayk[(size_t)k * d.nu + iu];
                if (dx == 0.0) {
                    R.K = (float)(2.0 * hy / std::fabs(dy));
                    R.M = -1.f;
                    R.hs = slab(o0, d.ox, 1.0 / d.vx);
                    flags[k] |= 1;
                } else if (dy == 0.0) {
                    R.K = (float)(2.0 * hx / std::fabs(dx));
                    R.M = -2.f;
                    R.hs = slab(o1, d.oy, 1.0 / d.vy);
                    flags[k] |= 1;
                } else {
                    const double adx = std::fabs(dx), ady = std::fabs(dy);
                    const double K = 1.0 / (adx * ady);
                    R.hs = hx * ady + hy * adx;
                    R.K = (float)K;
                    R.M = (float)std::min(2.0 * hx / adx, 2.0 * hy / ady);
                    Q.K = R.K;
                    Q.S = (float)(R.hs * K);
                    Q.M = R.M;
                }
            }
        } else {
            // flag views whose rays (as the kernels form them) have a zero component
            // (or one at most kAxisEps)
            const double sdd = W[15];
            bool z = false;
            for (int iv = 0; iv < d.nv && !z; ++iv) {
                const double v = ((double)iv - 0.5 * (double)(d.nv - 1)) * d.pv;
                for (int iu = 0; iu < d.nu && !z; ++iu) {
                    const double u = ((double)iu - 0.5 * (double)(d.nu - 1)) * d.pu;
                    for (int c = 0; c < 3; ++c) {
                        const double Dk = std::fma(v, W[9 + c], std::fma(u, W[6 + c], sdd * W[12 + c]));
                        // the kernels' staged component and their zero test
                        if (std::fabs((float)(Dk * W[16])) <= kAxisEpsF) z = true;
                    }
                }
            }
            if (z) flags[k] |= 1;
        }
    }
}

struct DevLayout {
    size_t off_view, off_rayf, off_rayb, off_rayk, off_cdxy, off_cdz, off_cisv, off_flags, off_tiles, off_rbt, off_troff, off_chunks, off_rbc, off_wch,
        off_rbj, off_all,
        off_nnz, off_boxes, total;
};

// Per-view tables of a vertical cone (see DGeom): the x, y components of a
// ray depend on its detector column only, the z component on its row only.
// Same operations as the kernels' float64 ray vector D = v e_v + u e_u + sdd n
// (with e_v,x = e_v,y = e_u,z = n_z = 0 the other terms are exact zeros).
// The exponent e of the column kernel's interval scale 2^e: the largest
// power of two with 2^e sqrt(vx^2 + vy^2) <= 1.
static int col_scale_exp(const ct_geom_desc& d) {
    const double diag = std::sqrt(d.vx * d.vx + d.vy * d.vy);
    int e = (int)std::floor(std::log2(1.0 / diag));
    while (std::ldexp(diag, e) > 1.0) --e;
    return e;
}

static void build_columns(const ct_geom* g, std::vector<float4>& dxy, std::vector<float>& dz,
                          std::vector<double>& isv) {
    const ct_geom_desc& d = g->d;
    const int ke = col_scale_exp(d);
    dxy.assign((size_t)d.n_views * d.nu, float4{});
    dz.assign((size_t)d.n_views * d.nv, 0.f);
    isv.assign((size_t)d.n_views * d.nv, 0.0);
    for (int k = 0; k < d.n_views; ++k) {
        const double* W = &g->v64[(size_t)k * kViewStride];
        const double sdd = W[15], is = W[16];
        for (int iu = 0; iu < d.nu; ++iu) {
            const double u = ((double)iu - 0.5 * (double)(d.nu - 1)) * d.pu;
            float4& q = dxy[(size_t)k * d.nu + iu];
            const double qx = std::fma(u, W[6], sdd * W[12]) * is, qy = std::fma(u, W[7], sdd * W[13]) * is;
            q.x = (float)qx;
            q.y = (float)qy;
            q.z = (float)(qx * qx + qy * qy);
            q.w = 0.f;
        }
        for (int iv = 0; iv < d.nv; ++iv) {
            const double v = ((double)iv - 0.5 * (double)(d.nv - 1)) * d.pv;
            const double Dz = v * W[11];
            const float f = (float)(Dz * is);
            dz[(size_t)k * d.nv + iv] = f;
            isv[(size_t)k * d.nv + iv] = std::fabs(f) <= kAxisEpsF ? 0.0 : std::ldexp(sdd / Dz, ke);
        }
    }
}

static DevLayout dev_layout(const ct_geom* g) {
    DevLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align256(bytes);
        return r;
    };
    L.off_view = take((size_t)g->d.n_views * kViewStride * sizeof(double));
    L.off_rayf = take(g->dims == 2 ? (size_t)g->d.n_views * g->d.nu * sizeof(Ray2F) : 0);
    L.off_rayb = take(g->dims == 2 ? (size_t)g->d.n_views * g->d.nu * sizeof(Ray2B) : 0);
    L.off_rayk = take(g->dims == 2 ? (size_t)g->d.n_views * g->d.nu * sizeof(Ray2K) : 0);
    L.off_cdxy = take(g->vertical ? (size_t)g->d.n_views * g->d.nu * sizeof(float4) : 0);
    L.off_cdz = take(g->vertical ? (size_t)g->d.n_views * g->d.nv * sizeof(float) : 0);
    L.off_cisv = take(g->vertical ? (size_t)g->d.n_views * g->d.nv * sizeof(double) : 0);
    L.off_flags = take((size_t)g->d.n_views * sizeof(int32_t));
    L.off_tiles = take(g->tiles.size() * sizeof(Tile));
    L.off_rbt = take((g->m + 1) * sizeof(int32_t));
    L.off_troff = take(g->tiles.size() * sizeof(int32_t));
    L.off_chunks = take(g->chunks.size() * sizeof(Chunk));
    L.off_rbc = take((g->m + 1) * sizeof(int32_t));
    L.off_wch = take(g->wchunks.size() * sizeof(Chunk));
    L.off_rbj = take(g->rbj_chunk_ptr.size() * sizeof(int32_t));
    L.off_all = take(g->all_entries.size() * sizeof(Entry));
    L.off_nnz = take((size_t)g->m * g->n * sizeof(unsigned long long));
    L.off_boxes = take(g->boxes.size() * sizeof(Box));
    L.total = o;
    return L;
}

// The device-table image of a geometry (layout dev_layout) packed into host
// memory `dst` of geom_table_bytes(g) bytes.
size_t geom_table_bytes(const ct_geom* g) { return dev_layout(g).total; }

int geom_table_pack(const ct_geom* g, void* dst) {
    const DevLayout L = dev_layout(g);
    std::vector<Ray2F> rayf;
    std::vector<Ray2B> rayb;
    std::vector<Ray2K> rayk;
    std::vector<int32_t> flags;
    build_frames(g, rayf, rayb, rayk, flags);
    std::vector<float4> cdxy;
    std::vector<float> cdz;
    std::vector<double> cisv;
    if (g->vertical) build_columns(g, cdxy, cdz, cisv);
    char* base = (char*)dst;
    std::memset(base, 0, L.total);
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(base + off, src, bytes);
    };
    put(L.off_view, g->v64.data(), g->v64.size() * sizeof(double));
    put(L.off_rayf, rayf.data(), rayf.size() * sizeof(Ray2F));
    put(L.off_rayb, rayb.data(), rayb.size() * sizeof(Ray2B));
    put(L.off_rayk, rayk.data(), rayk.size() * sizeof(Ray2K));
    put(L.off_cdxy, cdxy.data(), cdxy.size() * sizeof(float4));
    put(L.off_cdz, cdz.data(), cdz.size() * sizeof(float));
    put(L.off_cisv, cisv.data(), cisv.size() * sizeof(double));
    put(L.off_flags, flags.data(), flags.size() * sizeof(int32_t));
    put(L.off_tiles, g->tiles.data(), g->tiles.size() * sizeof(Tile));
    put(L.off_rbt, g->rb_tile_ptr.data(), g->rb_tile_ptr.size() * sizeof(int32_t));
    put(L.off_troff, g->tile_roff.data(), g->tile_roff.size() * sizeof(int32_t));
    put(L.off_chunks, g->chunks.data(), g->chunks.size() * sizeof(Chunk));
    put(L.off_rbc, g->rb_chunk_ptr.data(), g->rb_chunk_ptr.size() * sizeof(int32_t));
    put(L.off_wch, g->wchunks.data(), g->wchunks.size() * sizeof(Chunk));
    put(L.off_rbj, g->rbj_chunk_ptr.data(), g->rbj_chunk_ptr.size() * sizeof(int32_t));
    put(L.off_all, g->all_entries.data(), g->all_entries.size() * sizeof(Entry));
    put(L.off_boxes, g->boxes.data(), g->boxes.size() * sizeof(Box));
    return CT_OK;
}

// Point the geometry's device view at a table image in device memory `mem`
// on device `dev`.  owned: the geometry frees it when destroyed.
static void geom_bind(ct_geom* g, void* mem, int dev, bool owned) {
    const DevLayout L = dev_layout(g);
    char* base = (char*)mem;
    DGeom& G = g->G;
    const ct_geom_desc& d = g->d;
    G.kind = d.kind;
    G.nx = d.nx;
    G.ny = d.ny;
    G.nz = d.nz;
    G.nu = d.nu;
    G.nv = d.nv;
    G.n_views = d.n_views;
    G.dims = g->dims;
    G.vx = d.vx;
    G.vy = d.vy;
    G.vz = d.vz;
    G.ox = d.ox;
    G.oy = d.oy;
    G.oz = d.oz;
    G.pu = d.pu;
    G.pv = d.pv;
    const double hz = g->dims == 3 ? 0.5 * d.vz : 0.0;
    G.radius = (float)(std::sqrt(0.25 * d.vx * d.vx + 0.25 * d.vy * d.vy + hz * hz) * (1.0 + 1e-6));
    G.ivx = 1.0 / d.vx;
    G.ivy = 1.0 / d.vy;
    G.ivz = 1.0 / d.vz;
    G.colk_e = col_scale_exp(d);
    G.view64 = (const double*)(base + L.off_view);
    G.ray2f = g->dims == 2 ? (const Ray2F*)(base + L.off_rayf) : nullptr;
    G.ray2b = g->dims == 2 ? (const Ray2B*)(base + L.off_rayb) : nullptr;
    G.ray2k = g->dims == 2 ? (const Ray2K*)(base + L.off_rayk) : nullptr;
    G.cdxy = g->vertical ? (const float4*)(base + L.off_cdxy) : nullptr;
    G.cdz = g->vertical ? (const float*)(base + L.off_cdz) : nullptr;
    G.cisv = g->vertical ? (const double*)(base + L.off_cisv) : nullptr;
    G.view_flags = (const int32_t*)(base + L.off_flags);
    G.tiles = (const Tile*)(base + L.off_tiles);
    G.rb_tile_ptr = (const int32_t*)(base + L.off_rbt);
    G.tile_roff = (const int32_t*)(base + L.off_troff);
    G.chunks = (const Chunk*)(base + L.off_chunks);
    G.rb_chunk_ptr = (const int32_t*)(base + L.off_rbc);
    G.wchunks = (const Chunk*)(base + L.off_wch);
    G.rbj_chunk_ptr = (const int32_t*)(base + L.off_rbj);
    G.n_cols = g->n;
    G.vertical = g->vertical;
    G.mixed_boxes = 0;
    for (const Box& b : g->boxes) {
        const Box& b0 = g->boxes[0];
        if (b.x1 - b.x0 != b0.x1 - b0.x0 || b.y1 - b.y0 != b0.y1 - b0.y0 || b.z1 - b.z0 != b0.z1 - b0.z0)
            G.mixed_boxes = 1;
    }
    g->d_all = (Entry*)(base + L.off_all);
    g->d_nnz = (unsigned long long*)(base + L.off_nnz);
    g->d_boxes = (Box*)(base + L.off_boxes);
    g->dbytes = L.total;
    g->device = dev;
    g->dmem = mem;
    g->dmem_owned = owned;
}

// The tables in caller memory `mem` (device), filled from a packed image
// already copied there (or being copied, in stream order, before any use).
int geom_table_bind(ct_geom* g, void* mem) {
    std::lock_guard<std::mutex> lock(g->mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CT_EDEVICE, "no HIP device");
    if (g->dmem) return fail(CT_EINVAL, "geometry tables are already on a device");
    geom_bind(g, mem, dev, false);
    return CT_OK;
}

// Upload the device tables on first use (the current device becomes the
// geometry's device).  Later calls must be made with that device current.
static int geom_ensure_device(ct_geom* g) {
    std::lock_guard<std::mutex> lock(g->mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CT_EDEVICE, "no HIP device");
    if (g->dmem) {
        if (dev != g->device) return fail(CT_EINVAL, "geometry lives on device %d, current is %d", g->device, dev);
        return CT_OK;
    }
    const size_t bytes = geom_table_bytes(g);
    std::vector<char> img(bytes);
    geom_table_pack(g, img.data());
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess)
        return fail(CT_ENOMEM, "hipMalloc(%zu) for geometry tables failed", bytes);
    const hipError_t e = hipMemcpy(mem, img.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return fail(CT_EDEVICE, "geometry upload: %s", hipGetErrorString(e));
    }
    geom_bind(g, mem, dev, true);
    return CT_OK;
}

extern "C" int ct_geom_create(const ct_geom_desc* desc, ct_geom** out) {
    if (!out) return fail(CT_EINVAL, "out is NULL");
    *out = nullptr;
    ct_geom* g = new (std::nothrow) ct_geom();
    if (!g) return fail(CT_ENOMEM, "host allocation failed");
    int rc = build_host(g, desc);
    if (rc != CT_OK) {
        delete g;
        return rc;
    }
    *out = g;
    return CT_OK;
}

extern "C" void ct_geom_destroy(ct_geom* g) {
    if (!g) return;
    if (g->dmem && g->dmem_owned) (void)hipFree(g->dmem);
    delete g;
}

extern "C" int ct_geom_get_info(const ct_geom* g, ct_geom_info* out) {
    if (!g || !out) return fail(CT_EINVAL, "NULL argument");
    out->n_rays = g->M;
    out->n_vox = g->N;
    out->m = g->m;
    out->n = g->n;
    out->max_rb_rays = g->max_rb_rays;
    out->max_cb_vox = g->max_cb_vox;
    return CT_OK;
}

static int check_device(ct_geom* g) { return geom_ensure_device(g); }

static FwdArgs fwd_all(const ct_geom* g, int J) {
    FwdArgs a{};
    a.box = g->boxes[J];
    a.ent = g->d_all;
    a.n_ent = g->m;
    a.n_chunks = g->total_chunks;
    return a;
}

// The density count enqueued on `st` into the geometry's counter table
// (device [m][n] unsigned 64-bit), without waiting: for callers that read it
// back asynchronously (the serving loop).  The tables must be on the device.
int geom_count_async(ct_geom* g, double tau, unsigned long long** counts, hipStream_t st) {
    if (!g->dmem) return fail(CT_EINVAL, "geometry tables are not on a device");
    HIPCHK(launch_fill_u64(g->d_nnz, (int64_t)g->m * g->n, st));
    for (int J = 0; J < g->n; ++J) {
        FwdArgs a = fwd_all(g, J);
        a.mode = 2;
        a.nnz = g->d_nnz;
        a.n_cols = g->n;
        a.col = J;
        a.tau = tau;
        HIPCHK(launch_fwd(g->G, a, st));
    }
    *counts = g->d_nnz;
    return CT_OK;
}

extern "C" int ct_geom_block_nnz(ct_geom* g, double tau, int64_t* host_nnz, void* stream) {
    if (!g || !host_nnz) return fail(CT_EINVAL, "NULL argument");
    if (!(tau >= 0)) return fail(CT_EINVAL, "tau must be >= 0");
    int rc = check_device(g);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(launch_fill_u64(g->d_nnz, (int64_t)g->m * g->n, st));
    for (int J = 0; J < g->n; ++J) {
        FwdArgs a = fwd_all(g, J);
        a.mode = 2;
        a.nnz = g->d_nnz;
        a.n_cols = g->n;
        a.col = J;
        a.tau = tau;
        HIPCHK(launch_fwd(g->G, a, st));
    }
    std::vector<unsigned long long> tmp((size_t)g->m * g->n);
    HIPCHK(hipMemcpyAsync(tmp.data(), g->d_nnz, tmp.size() * sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < tmp.size(); ++i) host_nnz[i] = (int64_t)tmp[i];
    return CT_OK;
}

// ---------------------------------------------------------------------------
// density table without allocation: counters in a static device array
// ---------------------------------------------------------------------------
// `scratch` is a host-side stand-in in host code: kernels get the device
// address that hipGetSymbolAddress returns for the current device (each GPU
// holds its own copy of the array), looked up once per device.
static __device__ __align__(256) unsigned long long scratch[CT_NNZ_STATIC_MAX];
static std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
static unsigned long long* g_scratch_dev[kMaxDevices] = {};

static int scratch_on_device(unsigned long long** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(CT_EDEVICE, "no HIP device");
    if (dev >= kMaxDevices) return fail(CT_EUNSUPPORTED, "device %d beyond the %d the library tracks", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = (unsigned long long*)p;
    }
    *out = g_scratch_dev[dev];
    return CT_OK;
}

extern "C" int ct_geom_block_nnz_static(ct_geom* g, double tau, int64_t* host_nnz, void* stream) {
    if (!g || !host_nnz) return fail(CT_EINVAL, "NULL argument");
    if (!(tau >= 0)) return fail(CT_EINVAL, "tau must be >= 0");
    const int64_t cells = (int64_t)g->m * g->n;
    if (cells > CT_NNZ_STATIC_MAX)
        return fail(CT_EINVAL, "m * n = %lld exceeds CT_NNZ_STATIC_MAX (%d)", (long long)cells, CT_NNZ_STATIC_MAX);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CT_EDEVICE, "no HIP device");
    {
        std::lock_guard<std::mutex> lock(g->mu);
        if (!g->dmem || g->device != dev)
            return fail(CT_EINVAL, "the geometry's device tables are not on device %d (an earlier call that "
                        "launches work on the geometry uploads them)", dev);
    }
    unsigned long long* cnt = nullptr;
    int rc = scratch_on_device(&cnt);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(launch_fill_u64(cnt, cells, st));          // a kernel, not a memset node
    for (int J = 0; J < g->n; ++J) {
        FwdArgs a = fwd_all(g, J);
        a.mode = 2;
        a.nnz = cnt;
        a.n_cols = g->n;
        a.col = J;
        a.tau = tau;
        HIPCHK(launch_fwd(g->G, a, st));
    }
    static_assert(sizeof(int64_t) == sizeof(unsigned long long), "counts are copied as they are");
    HIPCHK(hipMemcpyAsync(host_nnz, cnt, (size_t)cells * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return CT_OK;
}

// ---------------------------------------------------------------------------
// block primitives
// ---------------------------------------------------------------------------
static int check_rbs(const ct_geom* g, const int32_t* rbs, int32_t n_rb, int32_t col) {
    if (!rbs || n_rb < 1) return fail(CT_EINVAL, "need at least one row block");
    if (col < 0 || col >= g->n) return fail(CT_EINVAL, "column block %d out of range", col);
    std::vector<uint8_t> seen(g->m, 0);
    for (int i = 0; i < n_rb; ++i) {
        if (rbs[i] < 0 || rbs[i] >= g->m) return fail(CT_EINVAL, "row block %d out of range", rbs[i]);
        if (seen[rbs[i]]) return fail(CT_EINVAL, "row block %d listed twice", rbs[i]);
        seen[rbs[i]] = 1;
    }
    return CT_OK;
}

// Fill inline entries for row blocks [i0, i1) of the list; returns chunk count.
template <class A>
static int fill_inline(const ct_geom* g, const int32_t* rbs, int i0, int i1, A& a) {
    int cp = 0, sp = 0, k = 0;
    for (int i = i0; i < i1; ++i, ++k) {
        const int b = rbs[i];
        a.inl[k] = Entry{b, 0, cp, sp};
        cp += g->rb_chunk_ptr[b + 1] - g->rb_chunk_ptr[b];
        sp += (int)g->rb_rays[b];
    }
    a.ent = nullptr;
    a.n_ent = k;
    return cp;
}

extern "C" int ct_block_fwd(ct_geom* g, const int32_t* rbs, int32_t n_rb, int32_t col, const float* x,
                            float* y, int32_t flags, void* stream) {
    if (!g || !x || !y) return fail(CT_EINVAL, "NULL argument");
    int rc = check_rbs(g, rbs, n_rb, col);
    if (rc) return rc;
    if ((rc = check_device(g))) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (int i0 = 0; i0 < n_rb; i0 += kMaxInline) {
        const int i1 = std::min(n_rb, i0 + kMaxInline);
        FwdArgs a{};
        a.box = g->boxes[col];
        a.n_chunks = fill_inline(g, rbs, i0, i1, a);
        a.mode = 0;
        a.flags = flags & CT_ACCUMULATE;
        a.x = x;
        a.out = y;
        HIPCHK(launch_fwd(g->G, a, st));
    }
    return CT_OK;
}

static BackArgs back_common(const ct_geom* g, int col) {
    BackArgs a{};
    a.box = g->boxes[col];
    box_tiling(g, a.box, &a.tiles_x, &a.tiles_y, &a.tiles_z);
    return a;
}

extern "C" int ct_block_back(ct_geom* g, const int32_t* rbs, int32_t n_rb, int32_t col, const float* r,
                             float* gout, int32_t flags, void* stream) {
    if (!g || !r || !gout) return fail(CT_EINVAL, "NULL argument");
    int rc = check_rbs(g, rbs, n_rb, col);
    if (rc) return rc;
    if ((rc = check_device(g))) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (int i0 = 0; i0 < n_rb; i0 += kMaxInline) {
        const int i1 = std::min(n_rb, i0 + kMaxInline);
        BackArgs a = back_common(g, col);
        fill_inline(g, rbs, i0, i1, a);
        a.gptr = nullptr;
        a.flags = (i0 == 0) ? (flags & CT_ACCUMULATE) : CT_ACCUMULATE;
        a.fused = 0;
        a.r = r;
        a.g = gout;
        HIPCHK(launch_back(g->G, a, 1, g->tune.waves, st));
    }
    return CT_OK;
}

// ---------------------------------------------------------------------------
// projection-area densities (Sec. II-C): P_S of every (row block, column block)
// ---------------------------------------------------------------------------
namespace {

struct P2 {
    double x, y;
};

inline double cross2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

// Detector coordinate of the ray through point (px, py) in a 2D view.
double proj2(int kind, const double* V, double px, double py) {
    const double ax = V[0], ay = V[1], cx = V[3], cy = V[4], ux = V[6], uy = V[7];
    if (kind == CT_PAR2D) return cross2(px - cx, py - cy, ax, ay) / cross2(ux, uy, ax, ay);
    const double dx = px - ax, dy = py - ay;
    if (kind == CT_FAN2D_FLAT) return cross2(ax - cx, ay - cy, dx, dy) / cross2(ux, uy, dx, dy);
    const double nx = cx - ax, ny = cy - ay, nn = std::sqrt(nx * nx + ny * ny);
    return std::atan2(dx * ux + dy * uy, (dx * nx + dy * ny) / nn);
}

// Area of the convex polygon `poly` (any orientation) inside [u0,u1] x [v0,v1].
double clipped_area(std::vector<P2> poly, double u0, double u1, double v0, double v1) {
    auto clip = [&](int axis, double bound, bool below) {
        std::vector<P2> outp;
        const size_t k = poly.size();
        auto coord = [&](const P2& q) { return axis == 0 ? q.x : q.y; };
        auto in = [&](const P2& q) { return below ? coord(q) <= bound : coord(q) >= bound; };
        for (size_t i = 0; i < k; ++i) {
            const P2& a = poly[(i + k - 1) % k];
            const P2& b = poly[i];
            const bool ia = in(a), ib = in(b);
            if (ia != ib) {
                const double t = (bound - coord(a)) / (coord(b) - coord(a));
                outp.push_back(P2{a.x + t * (b.x - a.x), a.y + t * (b.y - a.y)});
            }
            if (ib) outp.push_back(b);
        }
        poly.swap(outp);
    };
    clip(0, u0, false);
    if (poly.size() >= 3) clip(0, u1, true);
    if (poly.size() >= 3) clip(1, v0, false);
    if (poly.size() >= 3) clip(1, v1, true);
    if (poly.size() < 3) return 0.0;
    double a = 0.0;
    for (size_t i = 0; i < poly.size(); ++i) {
        const P2& p = poly[(i + poly.size() - 1) % poly.size()];
        const P2& q = poly[i];
        a += p.x * q.y - p.y * q.x;
    }
    return 0.5 * std::fabs(a);
}

// Convex hull of points (counter-clockwise), by gift wrapping from the
// lowest point: fine for the eight projected corners of a box.
std::vector<P2> hull(const std::vector<P2>& pts) {
    std::vector<P2> h;
    size_t start = 0;
    for (size_t i = 1; i < pts.size(); ++i)
        if (pts[i].y < pts[start].y || (pts[i].y == pts[start].y && pts[i].x < pts[start].x)) start = i;
    size_t cur = start;
    for (size_t guard = 0; guard <= pts.size(); ++guard) {
        h.push_back(pts[cur]);
        size_t nxt = (cur + 1) % pts.size();
        for (size_t i = 0; i < pts.size(); ++i) {
            const double c = cross2(pts[nxt].x - pts[cur].x, pts[nxt].y - pts[cur].y, pts[i].x - pts[cur].x,
                                    pts[i].y - pts[cur].y);
            const double dn = std::hypot(pts[nxt].x - pts[cur].x, pts[nxt].y - pts[cur].y);
            const double di = std::hypot(pts[i].x - pts[cur].x, pts[i].y - pts[cur].y);
            if (c < 0 || (c == 0 && di > dn)) nxt = i;          // i is to the right of cur->nxt
        }
        cur = nxt;
        if (cur == start) break;
    }
    return h;
}

}  // namespace

extern "C" int ct_geom_block_area(const ct_geom* g, double* out) {
    if (!g || !out) return fail(CT_EINVAL, "NULL argument");
    const ct_geom_desc& d = g->d;
    const bool cone = d.kind == CT_CONE3D_FLAT;
    const double c0u = 0.5 * (double)(d.nu - 1), c0v = 0.5 * (double)(d.nv - 1);
    for (int I = 0; I < g->m; ++I)
        for (int J = 0; J < g->n; ++J) {
            const Box& b = g->boxes[J];
            const double xs[2] = {d.ox + b.x0 * d.vx, d.ox + b.x1 * d.vx};
            const double ys[2] = {d.oy + b.y0 * d.vy, d.oy + b.y1 * d.vy};
            const double zs[2] = {d.oz + b.z0 * d.vz, d.oz + b.z1 * d.vz};
            double acc = 0.0;
            for (int t = g->rb_tile_ptr[I]; t < g->rb_tile_ptr[I + 1]; ++t) {
                const Tile& tl = g->tiles[t];
                const double* V = &g->views[(size_t)tl.view * 12];
                const double ulo = (tl.u0 - 0.5 - c0u) * d.pu, uhi = (tl.u1 - 0.5 - c0u) * d.pu;
                if (!cone) {
                    double mn = INFINITY, mx = -INFINITY;
                    for (int c = 0; c < 4; ++c) {
                        const double u = proj2(d.kind, V, xs[c & 1], ys[(c >> 1) & 1]);
                        mn = std::min(mn, u);
                        mx = std::max(mx, u);
                    }
                    acc += std::max(0.0, std::min(uhi, mx) - std::max(ulo, mn));
                } else {
                    const double vlo = (tl.v0 - 0.5 - c0v) * d.pv, vhi = (tl.v1 - 0.5 - c0v) * d.pv;
                    const double a[3] = {V[0], V[1], V[2]};
                    double n3[3] = {V[3] - a[0], V[4] - a[1], V[5] - a[2]};
                    const double sdd = std::sqrt(dot3(n3, n3));
                    for (double& q : n3) q /= sdd;
                    std::vector<P2> pts;
                    for (int c = 0; c < 8; ++c) {
                        const double p[3] = {xs[c & 1] - a[0], ys[(c >> 1) & 1] - a[1], zs[(c >> 2) & 1] - a[2]};
                        const double dep = dot3(p, n3);
                        pts.push_back(P2{sdd * dot3(p, V + 6) / dep, sdd * dot3(p, V + 9) / dep});
                    }
                    acc += clipped_area(hull(pts), ulo, uhi, vlo, vhi);
                }
            }
            out[(size_t)I * g->n + J] = acc;
        }
    return CT_OK;
}

// ---------------------------------------------------------------------------
// schedule
// ---------------------------------------------------------------------------
struct ct_schedule {
    int m = 0, n = 0;
    const ct_geom* geom = nullptr;
    std::vector<int32_t> ecp, cols, cgp, grp, rbs;
    std::vector<double> beta;
    // launch tables per column entry (step)
    std::vector<int32_t> step_ent_off;      // [n_cols+1]
    std::vector<int32_t> step_gptr_off;     // [n_cols]: offset into gptr
    std::vector<int32_t> step_chunks, step_slots;
    std::vector<Entry> entries;
    std::vector<int32_t> gptr;
    // union of touched row blocks per epoch
    std::vector<int32_t> uni_off;           // [n_epochs+1]
    std::vector<int32_t> uni_chunks;
    std::vector<Entry> uni;
    int device = -1;
    void* dmem = nullptr;               // device tables, uploaded on first use
    bool dmem_owned = true;             // false: placed in caller memory (sched_table_bind)
    std::mutex mu;
    Entry* d_entries = nullptr;
    int32_t* d_gptr = nullptr;
    double* d_beta = nullptr;
    Entry* d_uni = nullptr;
    StepRec* d_steps = nullptr;         // per step (column entry), for batches
    EpochRec* d_epochs = nullptr;       // per epoch, for batches
};

static std::vector<StepRec> sched_step_recs(const ct_schedule* s) {
    std::vector<StepRec> v(s->cols.size());
    for (size_t c = 0; c < v.size(); ++c) {
        StepRec& r = v[c];
        r.col = s->cols[c];
        r.n_groups = s->cgp[c + 1] - s->cgp[c];
        r.ent_off = s->step_ent_off[c];
        r.n_ent = s->step_ent_off[c + 1] - s->step_ent_off[c];
        r.gptr_off = s->step_gptr_off[c];
        r.beta_off = s->cgp[c];
        r.n_chunks = s->step_chunks[c];
        r.pad = 0;
    }
    return v;
}

static std::vector<EpochRec> sched_epoch_recs(const ct_schedule* s) {
    std::vector<EpochRec> v(s->ecp.size() - 1);
    for (size_t e = 0; e < v.size(); ++e) {
        EpochRec& r = v[e];
        r.step0 = s->ecp[e];
        r.n_steps = s->ecp[e + 1] - s->ecp[e];
        r.uni_off = s->uni_off[e];
        r.n_uni = s->uni_off[e + 1] - s->uni_off[e];
        r.uni_chunks = s->uni_chunks[e];
        r.pad = 0;
    }
    return v;
}

static uint64_t splitmix64(uint64_t seed, uint64_t ctr) {
    uint64_t z = seed + (ctr + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double unit_double(uint64_t seed, uint64_t ctr) {
    return (double)(splitmix64(seed, ctr) >> 11) * (1.0 / 9007199254740992.0);
}

static int count_of(double frac, int total) {
    int k = (int)std::ceil(frac * total - 1e-9);
    return std::max(1, std::min(total, k));
}

static int sched_finish(ct_schedule* s) {
    const ct_geom* g = s->geom;
    const int ncols = (int)s->cols.size();
    s->step_ent_off.assign(1, 0);
    s->step_gptr_off.clear();
    s->step_chunks.clear();
    s->step_slots.clear();
    s->entries.clear();
    s->gptr.clear();
    for (int c = 0; c < ncols; ++c) {
        s->step_gptr_off.push_back((int32_t)s->gptr.size());
        int cp = 0, sp = 0, ne = 0;
        for (int G = s->cgp[c]; G < s->cgp[c + 1]; ++G) {
            s->gptr.push_back(ne);
            for (int k = s->grp[G]; k < s->grp[G + 1]; ++k) {
                const int b = s->rbs[k];
                const int bj = b * g->n + s->cols[c];
                s->entries.push_back(Entry{b, G - s->cgp[c], cp, sp});
                cp += g->rbj_chunk_ptr[bj + 1] - g->rbj_chunk_ptr[bj];
                sp += (int32_t)g->rbj_rays[bj];
                ++ne;
            }
        }
        s->gptr.push_back(ne);
        s->step_ent_off.push_back((int32_t)s->entries.size());
        s->step_chunks.push_back(cp);
        s->step_slots.push_back(sp);
    }
    const int E = (int)s->ecp.size() - 1;
    s->uni_off.assign(1, 0);
    s->uni_chunks.clear();
    s->uni.clear();
    for (int e = 0; e < E; ++e) {
        std::vector<uint8_t> seen(g->m, 0);
        for (int c = s->ecp[e]; c < s->ecp[e + 1]; ++c)
            for (int G = s->cgp[c]; G < s->cgp[c + 1]; ++G)
                for (int k = s->grp[G]; k < s->grp[G + 1]; ++k) seen[s->rbs[k]] = 1;
        int cp = 0;
        for (int b = 0; b < g->m; ++b)
            if (seen[b]) {
                s->uni.push_back(Entry{b, 0, cp, 0});
                cp += g->rb_chunk_ptr[b + 1] - g->rb_chunk_ptr[b];
            }
        s->uni_off.push_back((int32_t)s->uni.size());
        s->uni_chunks.push_back(cp);
    }
    return CT_OK;
}

// The device-table image of a schedule: entries, group offsets, beta, the
// per-epoch unions, step and epoch records, 256-byte aligned segments.
struct SchedLayout {
    size_t ent, gptr, beta, uni, steps, epochs, total;
};
static SchedLayout sched_layout(const ct_schedule* sc, size_t n_steps, size_t n_epochs) {
    SchedLayout L{};
    L.ent = 0;
    L.gptr = L.ent + align256(std::max<size_t>(1, sc->entries.size()) * sizeof(Entry));
    L.beta = L.gptr + align256(std::max<size_t>(1, sc->gptr.size()) * sizeof(int32_t));
    L.uni = L.beta + align256(std::max<size_t>(1, sc->beta.size()) * sizeof(double));
    L.steps = L.uni + align256(std::max<size_t>(1, sc->uni.size()) * sizeof(Entry));
    L.epochs = L.steps + align256(std::max<size_t>(1, n_steps) * sizeof(StepRec));
    L.total = L.epochs + align256(std::max<size_t>(1, n_epochs) * sizeof(EpochRec));
    return L;
}

size_t sched_table_bytes(const ct_schedule* sc) {
    return sched_layout(sc, sc->cols.size(), sc->ecp.size() - 1).total;
}

int sched_table_pack(const ct_schedule* sc, void* dst) {
    const std::vector<StepRec> steps = sched_step_recs(sc);
    const std::vector<EpochRec> epochs = sched_epoch_recs(sc);
    const SchedLayout L = sched_layout(sc, steps.size(), epochs.size());
    char* base = (char*)dst;
    std::memset(base, 0, L.total);
    auto put = [&](size_t off, const void* src, size_t bytes) {
        if (bytes) std::memcpy(base + off, src, bytes);
    };
    put(L.ent, sc->entries.data(), sc->entries.size() * sizeof(Entry));
    put(L.gptr, sc->gptr.data(), sc->gptr.size() * sizeof(int32_t));
    put(L.beta, sc->beta.data(), sc->beta.size() * sizeof(double));
    put(L.uni, sc->uni.data(), sc->uni.size() * sizeof(Entry));
    put(L.steps, steps.data(), steps.size() * sizeof(StepRec));
    put(L.epochs, epochs.data(), epochs.size() * sizeof(EpochRec));
    return CT_OK;
}

static void sched_bind(ct_schedule* sc, void* mem, int dev, bool owned) {
    const SchedLayout L = sched_layout(sc, sc->cols.size(), sc->ecp.size() - 1);
    char* base = (char*)mem;
    sc->d_entries = (Entry*)(base + L.ent);
    sc->d_gptr = (int32_t*)(base + L.gptr);
    sc->d_beta = (double*)(base + L.beta);
    sc->d_uni = (Entry*)(base + L.uni);
    sc->d_steps = (StepRec*)(base + L.steps);
    sc->d_epochs = (EpochRec*)(base + L.epochs);
    sc->device = dev;
    sc->dmem = mem;
    sc->dmem_owned = owned;
}

// The tables in caller device memory `mem` holding (or receiving, in stream
// order before any use) the packed image.
int sched_table_bind(ct_schedule* sc, void* mem) {
    std::lock_guard<std::mutex> lock(sc->mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CT_EDEVICE, "no HIP device");
    if (sc->dmem) return fail(CT_EINVAL, "schedule tables are already on a device");
    sched_bind(sc, mem, dev, false);
    return CT_OK;
}

static int sched_ensure_device(ct_schedule* sc) {
    std::lock_guard<std::mutex> lock(sc->mu);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(CT_EDEVICE, "no HIP device");
    if (sc->dmem) {
        if (dev != sc->device) return fail(CT_EINVAL, "schedule lives on device %d, current is %d", sc->device, dev);
        return CT_OK;
    }
    const size_t bytes = sched_table_bytes(sc);
    std::vector<char> img(bytes);
    sched_table_pack(sc, img.data());
    void* mem = nullptr;
    if (hipMalloc(&mem, bytes) != hipSuccess) return fail(CT_ENOMEM, "hipMalloc for schedule tables failed");
    const hipError_t e = hipMemcpy(mem, img.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        return fail(CT_EDEVICE, "schedule upload: %s", hipGetErrorString(e));
    }
    sched_bind(sc, mem, dev, true);
    return CT_OK;
}

extern "C" void ct_schedule_destroy(ct_schedule* s) {
    if (!s) return;
    if (s->dmem && s->dmem_owned) (void)hipFree(s->dmem);
    delete s;
}

static int sched_check_params(const ct_sched_params* p) {
    if (p->epochs < 0) return fail(CT_EINVAL, "epochs < 0");
    if (!(p->alpha > 0 && p->alpha <= 1) || !(p->gamma > 0 && p->gamma <= 1))
        return fail(CT_EINVAL, "alpha and gamma must lie in (0, 1]");
    if (p->group_size < 1) return fail(CT_EINVAL, "group_size < 1");
    if (!std::isfinite(p->b)) return fail(CT_EINVAL, "b not finite");
    if (p->sampling < CT_SAMPLE_DENSITY || p->sampling > CT_SAMPLE_MIXED) return fail(CT_EINVAL, "bad sampling");
    if (p->sampling == CT_SAMPLE_MIXED && !(p->theta_step >= 0)) return fail(CT_EINVAL, "theta_step < 0");
    return CT_OK;
}

static int sched_draw(const ct_geom* g, const ct_sched_params* p, const std::vector<double>& P,
                      ct_schedule** out);

extern "C" int ct_schedule_create(const ct_geom* g, const ct_sched_params* p, const int64_t* nnz,
                                  ct_schedule** out) {
    if (!g || !p || !nnz || !out) return fail(CT_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = sched_check_params(p);
    if (rc) return rc;
    const int m = g->m, n = g->n;
    for (int i = 0; i < m * n; ++i)
        if (nnz[i] < 0) return fail(CT_EINVAL, "negative density");
    // P(I,J) = nnz / sum_I nnz
    std::vector<double> P((size_t)m * n, 0.0);
    for (int J = 0; J < n; ++J) {
        int64_t col = 0;
        for (int I = 0; I < m; ++I) col += nnz[(size_t)I * n + J];
        if (col > 0)
            for (int I = 0; I < m; ++I) P[(size_t)I * n + J] = (double)nnz[(size_t)I * n + J] / (double)col;
    }
    return sched_draw(g, p, P, out);
}

extern "C" int ct_schedule_create_w(const ct_geom* g, const ct_sched_params* p, const double* w,
                                    ct_schedule** out) {
    if (!g || !p || !w || !out) return fail(CT_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = sched_check_params(p);
    if (rc) return rc;
    const int m = g->m, n = g->n;
    for (int i = 0; i < m * n; ++i)
        if (!(w[i] >= 0) || !std::isfinite(w[i])) return fail(CT_EINVAL, "density weights must be finite and >= 0");
    // P(I,J) = w / sum_I w (ascending I)
    std::vector<double> P((size_t)m * n, 0.0);
    for (int J = 0; J < n; ++J) {
        double col = 0.0;
        for (int I = 0; I < m; ++I) col += w[(size_t)I * n + J];
        if (col > 0)
            for (int I = 0; I < m; ++I) P[(size_t)I * n + J] = w[(size_t)I * n + J] / col;
    }
    return sched_draw(g, p, P, out);
}

static int sched_draw(const ct_geom* g, const ct_sched_params* p, const std::vector<double>& P,
                      ct_schedule** out) {
    const int m = g->m, n = g->n;
    ct_schedule* s = new (std::nothrow) ct_schedule();
    if (!s) return fail(CT_ENOMEM, "host allocation failed");
    s->m = m;
    s->n = n;
    s->geom = g;
    s->ecp.push_back(0);
    s->cgp.push_back(0);
    s->grp.push_back(0);
    const uint64_t seed = p->seed;
    std::vector<int> perm(n), avail;
    std::vector<double> w(m);
    // mixed sampling (Sec. III-D): row blocks whose tiles cover the same set
    // of views are sub-detector areas of one projection; proj[I] is the first
    // row block with I's set of views, and P_max is taken within it
    std::vector<int> proj(m);
    std::vector<double> pmax(m);
    if (p->sampling == CT_SAMPLE_MIXED) {
        std::map<std::vector<int32_t>, int> first;
        for (int I = 0; I < m; ++I) {
            std::vector<int32_t> vs;
            for (int t = g->rb_tile_ptr[I]; t < g->rb_tile_ptr[I + 1]; ++t) vs.push_back(g->tiles[t].view);
            std::sort(vs.begin(), vs.end());
            vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
            proj[I] = first.emplace(std::move(vs), I).first->second;
        }
    }
    for (int e = 0; e < p->epochs; ++e) {
        uint64_t k = 0;
        const uint64_t base = (uint64_t)e << 32;
        for (int i = 0; i < n; ++i) perm[i] = i;
        for (int i = n - 1; i > 0; --i) {
            const int j = (int)std::floor(unit_double(seed, base + k++) * (double)(i + 1));
            std::swap(perm[i], perm[j]);
        }
        const double theta = std::min(1.0, e * p->theta_step);
        const int ncol = count_of(p->gamma, n);
        for (int ci = 0; ci < ncol; ++ci) {
            const int J = perm[ci];
            if (p->sampling == CT_SAMPLE_MIXED) {
                for (int I = 0; I < m; ++I) pmax[I] = 0.0;
                for (int I = 0; I < m; ++I) pmax[proj[I]] = std::max(pmax[proj[I]], P[(size_t)I * n + J]);
            }
            for (int I = 0; I < m; ++I) {
                const double pij = P[(size_t)I * n + J];
                if (p->sampling == CT_SAMPLE_UNIFORM) w[I] = 1.0;
                else if (p->sampling == CT_SAMPLE_MIXED) {
                    const double pm = pmax[proj[I]];
                    w[I] = pm > 0 ? pij + theta * (pm - pij) : 0.0;
                } else w[I] = pij;
            }
            avail.clear();
            for (int I = 0; I < m; ++I)
                if (w[I] > 0) avail.push_back(I);
            const int K = std::min(count_of(p->alpha, m), (int)avail.size());
            std::vector<int> draws;
            for (int t = 0; t < K; ++t) {
                double W = 0.0;
                for (int I : avail) W += w[I];
                const double target = unit_double(seed, base + k++) * W;
                double acc = 0.0;
                size_t pick = avail.size() - 1;
                for (size_t q = 0; q < avail.size(); ++q) {
                    acc += w[avail[q]];
                    if (acc > target) {
                        pick = q;
                        break;
                    }
                }
                draws.push_back(avail[pick]);
                avail.erase(avail.begin() + (long)pick);
            }
            for (int g0 = 0; g0 < K; g0 += p->group_size) {
                double bs = 0.0;
                for (int q = g0; q < std::min(K, g0 + p->group_size); ++q) {
                    s->rbs.push_back(draws[q]);
                    bs += P[(size_t)draws[q] * n + J];
                }
                s->grp.push_back((int32_t)s->rbs.size());
                s->beta.push_back(p->b * bs);
            }
            s->cols.push_back(J);
            s->cgp.push_back((int32_t)s->grp.size() - 1);
        }
        s->ecp.push_back((int32_t)s->cols.size());
    }
    int rc = sched_finish(s);
    if (rc) {
        ct_schedule_destroy(s);
        return rc;
    }
    *out = s;
    return CT_OK;
}

extern "C" int ct_schedule_import(const ct_geom* g, const ct_sched_view* v, ct_schedule** out) {
    if (!g || !v || !out) return fail(CT_EINVAL, "NULL argument");
    *out = nullptr;
    if (v->n_epochs < 0 || !v->epoch_col_ptr) return fail(CT_EINVAL, "bad epoch table");
    const int E = v->n_epochs;
    if (v->epoch_col_ptr[0] != 0) return fail(CT_EINVAL, "epoch_col_ptr[0] != 0");
    for (int e = 0; e < E; ++e)
        if (v->epoch_col_ptr[e + 1] < v->epoch_col_ptr[e]) return fail(CT_EINVAL, "epoch_col_ptr decreasing");
    const int ncols = v->epoch_col_ptr[E];
    if (ncols != v->n_cols) return fail(CT_EINVAL, "n_cols mismatch");
    if (ncols > 0 && (!v->cols || !v->col_group_ptr)) return fail(CT_EINVAL, "NULL column arrays");
    if (v->col_group_ptr && v->col_group_ptr[0] != 0) return fail(CT_EINVAL, "col_group_ptr[0] != 0");
    for (int c = 0; c < ncols; ++c)
        if (v->col_group_ptr[c + 1] < v->col_group_ptr[c]) return fail(CT_EINVAL, "col_group_ptr decreasing");
    const int ngr = ncols ? v->col_group_ptr[ncols] : 0;
    if (ngr != v->n_groups) return fail(CT_EINVAL, "n_groups mismatch");
    if (ngr > 0 && (!v->group_rb_ptr || !v->rbs || !v->beta)) return fail(CT_EINVAL, "NULL group arrays");
    if (ngr > 0 && v->group_rb_ptr[0] != 0) return fail(CT_EINVAL, "group_rb_ptr[0] != 0");
    for (int G = 0; G < ngr; ++G) {
        if (v->group_rb_ptr[G + 1] <= v->group_rb_ptr[G]) return fail(CT_EINVAL, "empty group %d", G);
        if (!std::isfinite(v->beta[G])) return fail(CT_EINVAL, "beta not finite");
    }
    const int nrb = ngr ? v->group_rb_ptr[ngr] : 0;
    if (nrb != v->n_rbs) return fail(CT_EINVAL, "n_rbs mismatch");
    for (int e = 0; e < E; ++e) {
        std::vector<uint8_t> colseen(g->n, 0);
        for (int c = v->epoch_col_ptr[e]; c < v->epoch_col_ptr[e + 1]; ++c) {
            const int J = v->cols[c];
            if (J < 0 || J >= g->n) return fail(CT_EINVAL, "column %d out of range", J);
            if (colseen[J]) return fail(CT_EINVAL, "column %d twice in epoch %d", J, e);
            colseen[J] = 1;
            std::vector<uint8_t> seen(g->m, 0);
            for (int G = v->col_group_ptr[c]; G < v->col_group_ptr[c + 1]; ++G)
                for (int k = v->group_rb_ptr[G]; k < v->group_rb_ptr[G + 1]; ++k) {
                    const int b = v->rbs[k];
                    if (b < 0 || b >= g->m) return fail(CT_EINVAL, "row block %d out of range", b);
                    if (seen[b]) return fail(CT_EINVAL, "row block %d twice for one column", b);
                    seen[b] = 1;
                }
        }
    }
    ct_schedule* s = new (std::nothrow) ct_schedule();
    if (!s) return fail(CT_ENOMEM, "host allocation failed");
    s->m = g->m;
    s->n = g->n;
    s->geom = g;
    s->ecp.assign(v->epoch_col_ptr, v->epoch_col_ptr + E + 1);
    s->cols.assign(v->cols, v->cols + ncols);
    if (ncols) s->cgp.assign(v->col_group_ptr, v->col_group_ptr + ncols + 1);
    else s->cgp.assign(1, 0);
    if (ngr) {
        s->grp.assign(v->group_rb_ptr, v->group_rb_ptr + ngr + 1);
        s->rbs.assign(v->rbs, v->rbs + nrb);
        s->beta.assign(v->beta, v->beta + ngr);
    } else {
        s->grp.assign(1, 0);
    }
    int rc = sched_finish(s);
    if (rc) {
        ct_schedule_destroy(s);
        return rc;
    }
    *out = s;
    return CT_OK;
}

extern "C" int ct_schedule_export(const ct_schedule* s, ct_sched_view* out) {
    if (!s || !out) return fail(CT_EINVAL, "NULL argument");
    out->n_epochs = (int32_t)s->ecp.size() - 1;
    out->n_cols = (int32_t)s->cols.size();
    out->n_groups = (int32_t)s->beta.size();
    out->n_rbs = (int32_t)s->rbs.size();
    out->epoch_col_ptr = s->ecp.data();
    out->cols = s->cols.data();
    out->col_group_ptr = s->cgp.data();
    out->group_rb_ptr = s->grp.data();
    out->rbs = s->rbs.data();
    out->beta = s->beta.data();
    return CT_OK;
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
constexpr int kResBlocks = 1024;        // work-groups of the residual-norm reduction

struct WsLayout {
    size_t z, r, q, xg, pg, pq, mu, part, total;
};

static WsLayout ws_layout(const ct_geom* g) {
    WsLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o += align256(bytes);
        return r;
    };
    L.z = take((size_t)g->n * g->M * sizeof(float));
    L.r = take((size_t)g->M * sizeof(float));
    L.q = take((size_t)g->M * sizeof(float));
    L.xg = take((size_t)g->m * g->max_xg * sizeof(float2));
    L.pg = take((size_t)g->m * g->max_tiles * sizeof(double));
    L.pq = take((size_t)std::max(g->total_chunks, g->max_step_wchunks) * sizeof(double));
    L.mu = take((size_t)g->m * sizeof(double));
    L.part = take((2 * (size_t)kResBlocks + 2) * sizeof(double));
    L.total = o;
    return L;
}

struct ProfRec {
    int kind;
    hipEvent_t a, b;
};

// Per-launch HIP-event timing of a solver or a batch.
struct Prof {
    bool on = false;
    std::vector<ProfRec> recs;          // recorded (kernel class, start, end)
    std::vector<hipEvent_t> pool;       // idle events

    void release() {
        for (auto& r : recs) {
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
    ~Prof() {
        release();
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
    hipEvent_t event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // Enqueue `launch` on `st`, bracketed by events when profiling is on.
    template <class F>
    hipError_t timed(int kind, hipStream_t st, F&& launch) {
        if (!on) return launch();
        hipEvent_t a = event(), b = event();
        if (!a || !b) return hipErrorOutOfMemory;
        hipError_t e = hipEventRecord(a, st);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(b, st);
        recs.push_back(ProfRec{kind, a, b});
        return e;
    }
    int read(ct_kernel_times* out) {
        std::memset(out, 0, sizeof *out);
        for (auto& r : recs) {
            HIPCHK(hipEventSynchronize(r.b));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
            out->ms[r.kind] += ms;
            out->launches[r.kind] += 1;
        }
        release();
        return CT_OK;
    }
};

struct ct_solver {
    Prof prof;
    ct_geom* geom = nullptr;
    ct_solver_params p{};
    char* ws = nullptr;
    size_t ws_bytes = 0;
    float* z = nullptr;
    float* r = nullptr;
    float* q = nullptr;
    float2* xg = nullptr;
    double* pg = nullptr;
    double* pq = nullptr;
    double* mu = nullptr;
    double* part = nullptr;             // residual-norm partials, then the two sums
};

extern "C" int ct_solver_workspace_bytes(const ct_geom* g, const ct_solver_params* p, size_t* bytes) {
    if (!g || !bytes) return fail(CT_EINVAL, "NULL argument");
    if (p && (p->sync < CT_SYNC_COLUMN || p->sync > CT_SYNC_EPOCH)) return fail(CT_EINVAL, "bad sync");
    *bytes = ws_layout(g).total;
    return CT_OK;
}

extern "C" int ct_solver_create(ct_geom* g, const ct_solver_params* p, void* ws, size_t ws_bytes,
                                ct_solver** out) {
    if (!g || !ws || !out) return fail(CT_EINVAL, "NULL argument");
    *out = nullptr;
    ct_solver_params pp{};
    if (p) pp = *p;
    if (pp.sync < CT_SYNC_COLUMN || pp.sync > CT_SYNC_EPOCH) return fail(CT_EINVAL, "bad sync");
    WsLayout L = ws_layout(g);
    if (ws_bytes < L.total) return fail(CT_EINVAL, "workspace too small (%zu < %zu)", ws_bytes, L.total);
    if (((uintptr_t)ws & 255) != 0) return fail(CT_EINVAL, "workspace must be 256-byte aligned");
    ct_solver* s = new (std::nothrow) ct_solver();
    if (!s) return fail(CT_ENOMEM, "host allocation failed");
    s->geom = g;
    s->p = pp;
    s->ws = (char*)ws;
    s->ws_bytes = ws_bytes;
    s->z = (float*)(s->ws + L.z);
    s->r = (float*)(s->ws + L.r);
    s->q = (float*)(s->ws + L.q);
    s->xg = (float2*)(s->ws + L.xg);
    s->pg = (double*)(s->ws + L.pg);
    s->pq = (double*)(s->ws + L.pq);
    s->mu = (double*)(s->ws + L.mu);
    s->part = (double*)(s->ws + L.part);
    *out = s;
    return CT_OK;
}

extern "C" void ct_solver_destroy(ct_solver* s) { delete s; }

template <class F>
static hipError_t timed(ct_solver* s, int kind, hipStream_t st, F&& launch) {
    return s->prof.timed(kind, st, launch);
}

extern "C" int ct_solver_profile(ct_solver* s, int32_t enable) {
    if (!s) return fail(CT_EINVAL, "NULL solver");
    s->prof.on = enable != 0;
    return CT_OK;
}

extern "C" int ct_solver_profile_read(ct_solver* s, ct_kernel_times* out) {
    if (!s || !out) return fail(CT_EINVAL, "NULL argument");
    return s->prof.read(out);
}

extern "C" int ct_solver_state(const ct_solver* s, float** z, float** r) {
    if (!s) return fail(CT_EINVAL, "NULL solver");
    if (z) *z = s->z;
    if (r) *r = s->r;
    return CT_OK;
}

static int residual_all(ct_solver* s, const float* y, hipStream_t st) {
    ct_geom* g = s->geom;
    ResArgs a{};
    a.ent = g->d_all;
    a.n_ent = g->m;
    a.z = s->z;
    a.y = y;
    a.r = s->r;
    a.M = g->M;
    a.n_cols = g->n;
    HIPCHK(launch_residual(g->G, a, g->total_chunks, st));
    return CT_OK;
}

extern "C" int ct_solver_reset(ct_solver* s, const float* y, const float* x, void* stream) {
    if (!s || !y) return fail(CT_EINVAL, "NULL argument");
    ct_geom* g = s->geom;
    int rc = check_device(g);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(launch_fill((float*)s->xg, 2 * (int64_t)g->m * g->max_xg, 0.f, st));  // zero margins
    if (!x) {
        HIPCHK(launch_fill(s->z, (int64_t)g->n * g->M, 0.f, st));
        HIPCHK(hipMemcpyAsync(s->r, y, (size_t)g->M * sizeof(float), hipMemcpyDeviceToDevice, st));
        return CT_OK;
    }
    for (int J = 0; J < g->n; ++J) {
        FwdArgs a = fwd_all(g, J);
        a.mode = 0;
        a.x = x;
        a.out = s->z + (size_t)J * g->M;
        HIPCHK(launch_fwd(g->G, a, st));
    }
    return residual_all(s, y, st);
}

static int enqueue_step(ct_solver* s, const ct_schedule* sc, int c, const float* y, float* x,
                        hipStream_t st) {
    ct_geom* g = s->geom;
    const int J = sc->cols[c];
    const int nG = sc->cgp[c + 1] - sc->cgp[c];
    if (nG <= 0) return CT_OK;
    const Box box = g->boxes[J];
    const int vox_J = (box.x1 - box.x0) * (box.y1 - box.y0) * (box.z1 - box.z0);
    const Entry* ent = sc->d_entries + sc->step_ent_off[c];
    const int n_ent = sc->step_ent_off[c + 1] - sc->step_ent_off[c];
    const int32_t* gptr = sc->d_gptr + sc->step_gptr_off[c];
    const int n_chunks = sc->step_chunks[c];

    BackArgs b = back_common(g, J);
    b.ent = ent;
    b.gptr = gptr;
    b.n_ent = n_ent;
    b.fused = 1;
    b.r = s->r;
    b.x = x;
    b.xg = s->xg;
    b.vox_J = vox_J;
    b.xg_stride = xg_size(box.x1 - box.x0, box.y1 - box.y0, box.z1 - box.z0);
    b.partial = s->pg;
    HIPCHK(timed(s, CT_K_BACK, st, [&] { return launch_back(g->G, b, nG, g->tune.waves, st); }));

    FwdArgs f{};
    f.box = box;
    f.ent = ent;
    f.n_ent = n_ent;
    f.n_chunks = n_chunks;
    f.mode = 1;
    f.split = g->tune.split;
    f.windowed = 1;
    f.col = J;
    f.xg = s->xg;
    f.vox_J = vox_J;
    f.xg_stride = b.xg_stride;
    f.out = s->z + (size_t)J * g->M;
    f.q = s->q;
    f.partial = s->pq;
    HIPCHK(timed(s, CT_K_FWD, st, [&] { return launch_fwd(g->G, f, st); }));

    StepArgs sa{};
    sa.ent = ent;
    sa.gptr = gptr;
    sa.n_chunks = n_chunks;
    sa.n_tiles = b.tiles_x * b.tiles_y * b.tiles_z;
    sa.pg = s->pg;
    sa.pq = s->pq;
    sa.beta = sc->d_beta + sc->cgp[c];
    sa.mu = s->mu;
    HIPCHK(timed(s, CT_K_STEP, st, [&] { return launch_step(sa, nG, st); }));

    FinArgs fa{};
    fa.ent = ent;
    fa.n_ent = n_ent;
    fa.n_chunks = n_chunks;
    fa.mu = s->mu;
    fa.q = s->q;
    fa.z = s->z;
    fa.zJ = s->z + (size_t)J * g->M;
    fa.y = y;
    fa.r = s->r;
    fa.M = g->M;
    fa.n_cols = g->n;
    fa.refresh = (s->p.sync == CT_SYNC_COLUMN) ? 1 : 0;
    fa.col = J;
    fa.box = box;
    fa.vox_J = vox_J;
    fa.xg_stride = b.xg_stride;
    fa.n_groups = nG;
    fa.xg = s->xg;
    fa.x = x;
    fa.nx = g->d.nx;
    fa.ny = g->d.ny;
    HIPCHK(timed(s, CT_K_FINALIZE, st, [&] { return launch_finalize(g->G, fa, (vox_J + 255) / 256, st); }));
    return CT_OK;
}

extern "C" int ct_block_epoch(ct_solver* s, const ct_schedule* sc, int32_t e, const float* y, float* x,
                              void* stream) {
    if (!s || !sc || !y || !x) return fail(CT_EINVAL, "NULL argument");
    ct_geom* g = s->geom;
    if (sc->geom != g) return fail(CT_EINVAL, "schedule was built for another geometry");
    if (e < 0 || e >= (int)sc->ecp.size() - 1) return fail(CT_EINVAL, "epoch %d out of range", e);
    int rc = check_device(g);
    if (rc) return rc;
    if ((rc = sched_ensure_device(const_cast<ct_schedule*>(sc)))) return rc;
    hipStream_t st = (hipStream_t)stream;
    for (int c = sc->ecp[e]; c < sc->ecp[e + 1]; ++c)
        if ((rc = enqueue_step(s, sc, c, y, x, st))) return rc;
    if (s->p.sync == CT_SYNC_EPOCH && sc->uni_chunks[e] > 0) {
        ResArgs a{};
        a.ent = sc->d_uni + sc->uni_off[e];
        a.n_ent = sc->uni_off[e + 1] - sc->uni_off[e];
        a.z = s->z;
        a.y = y;
        a.r = s->r;
        a.M = g->M;
        a.n_cols = g->n;
        const int nch = sc->uni_chunks[e];
        HIPCHK(timed(s, CT_K_RESIDUAL, st, [&] { return launch_residual(g->G, a, nch, st); }));
    }
    return CT_OK;
}

// ||y - A x||^2 and ||y||^2 (float64, fixed order) into s->part[2K], s->part[2K+1].
static int enqueue_norms(ct_solver* s, const float* y, const float* x, hipStream_t st) {
    ct_geom* g = s->geom;
    for (int J = 0; J < g->n; ++J) {
        FwdArgs a = fwd_all(g, J);
        a.mode = 0;
        a.flags = J == 0 ? 0 : CT_ACCUMULATE;
        a.x = x;
        a.out = s->q;
        HIPCHK(launch_fwd(g->G, a, st));
    }
    const int nblk = (int)std::min<int64_t>(kResBlocks, (g->M + 255) / 256);
    HIPCHK(launch_resnorm(y, s->q, g->M, s->part, nblk, st));
    HIPCHK(launch_sum_pairs(s->part, nblk, s->part + 2 * kResBlocks, st));
    return CT_OK;
}

extern "C" int ct_residual_norms(ct_solver* s, const float* y, const float* x, double* out, void* stream) {
    if (!s || !y || !x || !out) return fail(CT_EINVAL, "NULL argument");
    int rc = check_device(s->geom);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = enqueue_norms(s, y, x, st))) return rc;
    HIPCHK(hipMemcpyAsync(out, s->part + 2 * kResBlocks, 2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    return CT_OK;
}

extern "C" int ct_true_residual(ct_solver* s, const float* y, const float* x, double* rel, void* stream) {
    if (!s || !y || !x || !rel) return fail(CT_EINVAL, "NULL argument");
    int rc = check_device(s->geom);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = enqueue_norms(s, y, x, st))) return rc;
    double ab[2];
    HIPCHK(hipMemcpyAsync(ab, s->part + 2 * kResBlocks, sizeof ab, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *rel = ab[1] > 0 ? std::sqrt(ab[0] / ab[1]) : 0.0;
    return CT_OK;
}

// ---------------------------------------------------------------------------
// whole solve
// ---------------------------------------------------------------------------
extern "C" int ct_solve(ct_geom* g, const ct_solve_params* p, const float* y, float* x, void* ws,
                        size_t ws_bytes, ct_solve_stats* st_out, void* stream) {
    if (!g || !p || !y || !x || !ws) return fail(CT_EINVAL, "NULL argument");
    if (p->check_every < 0) return fail(CT_EINVAL, "check_every < 0");
    if (!(p->tau >= 0)) return fail(CT_EINVAL, "tau < 0");
    int rc = sched_check_params(&p->sched);
    if (rc) return rc;
    size_t bytes = 0;
    if ((rc = ct_solver_workspace_bytes(g, &p->solver, &bytes))) return rc;
    if (ws_bytes < bytes) return fail(CT_EINVAL, "workspace too small (%zu < %zu)", ws_bytes, bytes);
    if (((uintptr_t)ws & 255) != 0) return fail(CT_EINVAL, "workspace must be 256-byte aligned");
    if ((rc = check_device(g))) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::vector<int64_t> nnz((size_t)g->m * g->n);
    if ((rc = ct_geom_block_nnz(g, p->tau, nnz.data(), stream))) return rc;
    ct_schedule* sc = nullptr;
    if ((rc = ct_schedule_create(g, &p->sched, nnz.data(), &sc))) return rc;
    ct_solver* s = nullptr;
    rc = ct_solver_create(g, &p->solver, ws, ws_bytes, &s);
    int64_t updates = 0;
    int run = 0;
    double rel = -1.0;
    bool converged = false;
    if (!rc) rc = launch_fill(x, g->N, 0.f, st) == hipSuccess ? CT_OK : fail(CT_EDEVICE, "fill x");
    if (!rc) rc = ct_solver_reset(s, y, nullptr, stream);
    for (int e = 0; !rc && e < p->sched.epochs; ++e) {
        rc = ct_block_epoch(s, sc, e, y, x, stream);
        if (rc) break;
        run = e + 1;
        if (st_out && st_out->r_norm) {
            // ||r||^2 of the tracked residual: the second sum of the norm
            // kernel, sum r^2, with the first taken against r itself
            const int nblk = (int)std::min<int64_t>(kResBlocks, (g->M + 255) / 256);
            double ab[2] = {0.0, 0.0};
            if (launch_resnorm(s->r, s->r, g->M, s->part, nblk, st) != hipSuccess ||
                launch_sum_pairs(s->part, nblk, s->part + 2 * kResBlocks, st) != hipSuccess ||
                hipMemcpyAsync(ab, s->part + 2 * kResBlocks, sizeof ab, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = fail(CT_EDEVICE, "residual norm of epoch %d", e);
                break;
            }
            st_out->r_norm[e] = std::sqrt(ab[1]);
        }
        for (int c = sc->ecp[e]; c < sc->ecp[e + 1]; ++c) {
            const int J = sc->cols[c];
            for (int k = sc->grp[sc->cgp[c]]; k < sc->grp[sc->cgp[c + 1]]; ++k)
                updates += 2 * nnz[(size_t)sc->rbs[k] * g->n + J];
        }
        if (p->check_every > 0 && run % p->check_every == 0) {
            rc = ct_true_residual(s, y, x, &rel, stream);
            if (!rc && rel <= p->rel_tol) {
                converged = true;
                break;
            }
        }
    }
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = fail(CT_EDEVICE, "stream sync failed");
    if (st_out) {
        st_out->epochs_run = run;
        st_out->rel_residual = rel;
        st_out->ray_voxel_updates = updates;
    }
    ct_solver_destroy(s);
    ct_schedule_destroy(sc);
    if (rc) return rc;
    if (p->check_every > 0 && !converged) return CT_NOT_CONVERGED;
    return CT_OK;
}

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
// Device table (one allocation): BJob[cap], int32 ep[cap], then the prefix
// arrays of every launch of a batch epoch.  The host keeps the authoritative
// copy of each job's next epoch and uploads it with the table whenever the
// job set changes; between changes only kb_advance moves the counters, in
// step with the host's own count.
struct BatchSlot {
    int32_t id;
    ct_batch_job job;
    int32_t next;               // next epoch to run
    int32_t n_epochs;
};

struct BatchLaunch {
    int phase, kind, c;
    size_t prefix_off;          // int32 offset of the prefix array in the table
    int blocks;
};

struct ct_batch {
    int cap = 0;
    int next_id = 0;
    std::vector<BatchSlot> jobs;
    bool dirty = true;
    int device = -1;
    // device table and its pinned staging copy
    void* dmem = nullptr;
    size_t dbytes = 0;
    void* hmem = nullptr;
    size_t hbytes = 0;
    hipEvent_t staged = nullptr;    // the last upload from hmem has completed
    bool staged_pending = false;
    std::vector<BatchLaunch> launches;
    // graph of one batch epoch
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_valid = false;
    Prof prof;
    Tune tune[5]{};                 // launch shapes per launch kind (the four kinds and kConeV)
};

// Launch kind of a geometry's projectors: its kind, or kConeV for a cone
// whose detector columns run along z (voxel-column back-projection).
static int launch_kind(const ct_geom* g) { return g->vertical ? kConeV : g->d.kind; }

static BJob make_bjob(const BatchSlot& b) {
    const ct_solver* s = b.job.solver;
    const ct_geom* g = s->geom;
    const ct_schedule* sc = b.job.sched;
    BJob J{};
    J.G = g->G;
    J.boxes = g->d_boxes;
    J.z = s->z;
    J.r = s->r;
    J.q = s->q;
    J.xg = s->xg;
    J.pg = s->pg;
    J.pq = s->pq;
    J.mu = s->mu;
    J.y = b.job.y;
    J.x = b.job.x;
    J.steps = sc->d_steps;
    J.epochs = sc->d_epochs;
    J.ent = sc->d_entries;
    J.gptr = sc->d_gptr;
    J.beta = sc->d_beta;
    J.uni = sc->d_uni;
    J.M = g->M;
    J.n_epochs = (int32_t)sc->ecp.size() - 1;
    J.sync = s->p.sync == CT_SYNC_EPOCH ? 1 : 0;
    J.kind = g->d.kind;
    return J;
}

// Work-groups job b needs in one phase of step index c: the most over all its
// epochs, so that one set of launches (and one graph) serves every epoch.
static int phase_work(const BatchSlot& b, int phase, int c) {
    const ct_solver* s = b.job.solver;
    const ct_geom* g = s->geom;
    const ct_schedule* sc = b.job.sched;
    const int E = (int)sc->ecp.size() - 1;
    int w = 0;
    for (int e = 0; e < E; ++e) {
        if (phase == kPhRes) {
            if (s->p.sync == CT_SYNC_EPOCH) w = std::max(w, (sc->uni_chunks[e] + 3) / 4);
            continue;
        }
        if (c >= sc->ecp[e + 1] - sc->ecp[e]) continue;
        const int k = sc->ecp[e] + c;
        const int nG = sc->cgp[k + 1] - sc->cgp[k];
        if (nG <= 0) continue;
        const Box& box = g->boxes[sc->cols[k]];
        int tx, ty, tz;
        box_tiling(g, box, &tx, &ty, &tz);
        const int vox = (box.x1 - box.x0) * (box.y1 - box.y0) * (box.z1 - box.z0);
        const int nch = sc->step_chunks[k];
        switch (phase) {
            case kPhBack: w = std::max(w, nG * tx * ty * tz); break;
            case kPhFwd: w = std::max(w, nch); break;
            case kPhStep: w = std::max(w, nG); break;
            default: w = std::max(w, (nch + 3) / 4 + (vox + 255) / 256); break;
        }
    }
    return w;
}

static hipError_t batch_wait_staging(ct_batch* b) {
    if (!b->staged_pending) return hipSuccess;
    b->staged_pending = false;
    return hipEventSynchronize(b->staged);
}

// Rebuild the job table and launch list after the job set changed, and
// enqueue its upload on `st`.
static int batch_rebuild(ct_batch* b, hipStream_t st) {
    const int n = (int)b->jobs.size();
    int cmax = 0;
    bool any_epoch_sync = false;
    std::vector<int> kinds;
    for (const BatchSlot& j : b->jobs) {
        const ct_schedule* sc = j.job.sched;
        for (size_t e = 0; e + 1 < sc->ecp.size(); ++e) cmax = std::max(cmax, sc->ecp[e + 1] - sc->ecp[e]);
        any_epoch_sync = any_epoch_sync || j.job.solver->p.sync == CT_SYNC_EPOCH;
        const int k = launch_kind(j.job.solver->geom);
        if (std::find(kinds.begin(), kinds.end(), k) == kinds.end()) kinds.push_back(k);
    }
    std::sort(kinds.begin(), kinds.end());
    // table: jobs, ep, prefix arrays
    const size_t jobs_bytes = align256((size_t)std::max(n, 1) * sizeof(BJob));
    const size_t ep_bytes = align256((size_t)std::max(n, 1) * sizeof(int32_t));
    std::vector<int32_t> pre;
    b->launches.clear();
    auto add_launch = [&](int phase, int kind, int c) {
        BatchLaunch L{phase, kind, c, pre.size(), 0};
        int acc = 0;
        pre.push_back(0);
        for (const BatchSlot& j : b->jobs) {
            const bool mine = (phase != kPhBack && phase != kPhFwd) || launch_kind(j.job.solver->geom) == kind;
            acc += mine ? phase_work(j, phase, c) : 0;
            pre.push_back(acc);
        }
        L.blocks = acc;
        if (acc > 0) b->launches.push_back(L);
        else pre.resize(L.prefix_off);
    };
    for (int c = 0; c < cmax; ++c) {
        for (int k : kinds) add_launch(kPhBack, k, c);
        for (int k : kinds) add_launch(kPhFwd, k, c);
        add_launch(kPhStep, -1, c);
        add_launch(kPhFin, -1, c);
    }
    if (any_epoch_sync) add_launch(kPhRes, -1, 0);
    const size_t total = jobs_bytes + ep_bytes + align256(std::max<size_t>(1, pre.size()) * sizeof(int32_t));
    HIPCHK(batch_wait_staging(b));
    if (total > b->dbytes) {
        // the old table may still be read by enqueued kernels
        if (b->dmem) {
            HIPCHK(hipStreamSynchronize(st));
            (void)hipFree(b->dmem);
            b->dmem = nullptr;
            b->dbytes = 0;
        }
        if (hipMalloc(&b->dmem, total) != hipSuccess) return fail(CT_ENOMEM, "hipMalloc(%zu) for the batch table failed", total);
        b->dbytes = total;
    }
    if (total > b->hbytes) {
        if (b->hmem) (void)hipHostFree(b->hmem);
        b->hmem = nullptr;
        b->hbytes = 0;
        if (hipHostMalloc(&b->hmem, total, hipHostMallocDefault) != hipSuccess)
            return fail(CT_ENOMEM, "hipHostMalloc(%zu) for the batch table failed", total);
        b->hbytes = total;
    }
    char* h = (char*)b->hmem;
    std::memset(h, 0, total);
    BJob* hj = (BJob*)h;
    int32_t* hep = (int32_t*)(h + jobs_bytes);
    int32_t* hpre = (int32_t*)(h + jobs_bytes + ep_bytes);
    for (int k = 0; k < n; ++k) {
        hj[k] = make_bjob(b->jobs[k]);
        hep[k] = b->jobs[k].next;
    }
    if (!pre.empty()) std::memcpy(hpre, pre.data(), pre.size() * sizeof(int32_t));
    HIPCHK(hipMemcpyAsync(b->dmem, b->hmem, total, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(b->staged, st));
    b->staged_pending = true;
    b->dirty = false;
    b->graph_valid = false;
    return CT_OK;
}

static BatchArgs batch_args(const ct_batch* b, const BatchLaunch* L) {
    const int n = (int)b->jobs.size();
    const size_t jobs_bytes = align256((size_t)std::max(n, 1) * sizeof(BJob));
    const size_t ep_bytes = align256((size_t)std::max(n, 1) * sizeof(int32_t));
    char* d = (char*)b->dmem;
    BatchArgs a{};
    a.jobs = (const BJob*)d;
    a.ep = (int32_t*)(d + jobs_bytes);
    a.prefix = L ? (const int32_t*)(d + jobs_bytes + ep_bytes) + L->prefix_off : nullptr;
    a.n_jobs = n;
    a.c = L ? L->c : 0;
    return a;
}

static int batch_enqueue(ct_batch* b, hipStream_t st) {
    static const int kind_of_phase[] = {CT_K_BACK, CT_K_FWD, CT_K_STEP, CT_K_FINALIZE, CT_K_RESIDUAL};
    for (const BatchLaunch& L : b->launches)
        HIPCHK(b->prof.timed(kind_of_phase[L.phase], st,
                             [&] {
                                 return launch_batch(L.phase, L.kind, batch_args(b, &L), L.blocks,
                                                     b->tune[L.kind == kConeV ? (int)CT_CONE3D_FLAT : L.kind], st);
                             }));
    HIPCHK(launch_batch_advance(batch_args(b, nullptr), st));
    return CT_OK;
}

static void batch_drop_graph(ct_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->graph_valid = false;
}

extern "C" int ct_batch_create(int32_t capacity, ct_batch** out) {
    if (!out) return fail(CT_EINVAL, "NULL argument");
    *out = nullptr;
    if (capacity < 1 || capacity > kMaxBatch) return fail(CT_EINVAL, "capacity must lie in [1, %d]", kMaxBatch);
    ct_batch* b = new (std::nothrow) ct_batch();
    if (!b) return fail(CT_ENOMEM, "host allocation failed");
    b->cap = capacity;
    if (hipGetDevice(&b->device) != hipSuccess || hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(CT_EDEVICE, "no HIP device");
    }
    *out = b;
    return CT_OK;
}

extern "C" void ct_batch_destroy(ct_batch* b) {
    if (!b) return;
    (void)batch_wait_staging(b);
    batch_drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->hmem) (void)hipHostFree(b->hmem);
    if (b->staged) (void)hipEventDestroy(b->staged);
    delete b;
}

extern "C" int ct_batch_add(ct_batch* b, const ct_batch_job* job, int32_t* id) {
    if (!b || !job || !id) return fail(CT_EINVAL, "NULL argument");
    if (!job->solver || !job->sched || !job->y || !job->x) return fail(CT_EINVAL, "job has a NULL member");
    if ((int)b->jobs.size() >= b->cap) return fail(CT_EINVAL, "batch is full (%d jobs)", b->cap);
    ct_solver* s = job->solver;
    if (job->sched->geom != s->geom) return fail(CT_EINVAL, "schedule was built for another geometry");
    const int E = (int)job->sched->ecp.size() - 1;
    if (job->epoch < 0 || job->epoch > E) return fail(CT_EINVAL, "first epoch %d out of range [0, %d]", job->epoch, E);
    for (const BatchSlot& j : b->jobs) {
        if (j.job.solver == s) return fail(CT_EINVAL, "solver already in the batch");
        if (j.job.x == job->x) return fail(CT_EINVAL, "x already used by job %d", j.id);
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(CT_EINVAL, "batch lives on device %d, current is %d", b->device, dev);
    int rc = check_device(s->geom);
    if (rc) return rc;
    if ((rc = sched_ensure_device(const_cast<ct_schedule*>(job->sched)))) return rc;
    BatchSlot sl{};
    sl.id = b->next_id++;
    sl.job = *job;
    sl.next = job->epoch;
    sl.n_epochs = E;
    b->jobs.push_back(sl);
    b->dirty = true;
    *id = sl.id;
    return CT_OK;
}

extern "C" int ct_batch_remove(ct_batch* b, int32_t id) {
    if (!b) return fail(CT_EINVAL, "NULL batch");
    for (size_t k = 0; k < b->jobs.size(); ++k)
        if (b->jobs[k].id == id) {
            b->jobs.erase(b->jobs.begin() + (long)k);
            b->dirty = true;
            return CT_OK;
        }
    return fail(CT_EINVAL, "no job %d in the batch", id);
}

extern "C" int ct_batch_profile(ct_batch* b, int32_t enable) {
    if (!b) return fail(CT_EINVAL, "NULL batch");
    b->prof.on = enable != 0;
    return CT_OK;
}

extern "C" int ct_batch_profile_read(ct_batch* b, ct_kernel_times* out) {
    if (!b || !out) return fail(CT_EINVAL, "NULL argument");
    return b->prof.read(out);
}

extern "C" int ct_batch_job_epoch(const ct_batch* b, int32_t id, int32_t* epoch) {
    if (!b || !epoch) return fail(CT_EINVAL, "NULL argument");
    for (const BatchSlot& j : b->jobs)
        if (j.id == id) {
            *epoch = j.next;
            return CT_OK;
        }
    return fail(CT_EINVAL, "no job %d in the batch", id);
}

extern "C" int ct_batch_epoch(ct_batch* b, int32_t flags, int32_t* ran, void* stream) {
    if (!b) return fail(CT_EINVAL, "NULL batch");
    if (flags & ~CT_BATCH_GRAPH) return fail(CT_EINVAL, "unknown flags 0x%x", flags);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return fail(CT_EINVAL, "batch lives on device %d, current is %d", b->device, dev);
    hipStream_t st = (hipStream_t)stream;
    int active = 0;
    for (const BatchSlot& j : b->jobs) active += j.next < j.n_epochs ? 1 : 0;
    if (ran) *ran = active;
    if (active == 0) return CT_OK;
    int rc;
    if (b->dirty && (rc = batch_rebuild(b, st))) return rc;
    if ((flags & CT_BATCH_GRAPH) && !b->prof.on) {
        if (!b->graph_valid) {
            batch_drop_graph(b);
            if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
            HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            rc = batch_enqueue(b, b->cap_stream);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(b->cap_stream, &graph);
            if (rc) {
                if (graph) (void)hipGraphDestroy(graph);
                return rc;
            }
            if (ec != hipSuccess) return fail(CT_EDEVICE, "graph capture: %s", hipGetErrorString(ec));
            const hipError_t ei = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) return fail(CT_EDEVICE, "graph instantiate: %s", hipGetErrorString(ei));
            b->graph_valid = true;
        }
        HIPCHK(hipGraphLaunch(b->exec, st));
    } else {
        if ((rc = batch_enqueue(b, st))) return rc;
    }
    for (BatchSlot& j : b->jobs)
        if (j.next < j.n_epochs) ++j.next;
    return CT_OK;
}

// ---------------------------------------------------------------------------
// launch shapes and their tuner
// ---------------------------------------------------------------------------
namespace {
constexpr int kSplits = 3, kWaves = 5;
constexpr int kSplitVal[kSplits] = {1, 2, 4};
constexpr int kWaveVal[kWaves] = {1, 2, 4, 8, 16};
constexpr int kTuneReps = 3;

struct TuneTable {
    double ms[kSplits][kWaves];     // [pieces per chord][waves per tile]; < 0: not a candidate
};

std::mutex g_tune_mu;
std::map<std::string, TuneTable> g_tune_cache;

int split_index(int v) {
    for (int i = 0; i < kSplits; ++i)
        if (kSplitVal[i] == v) return i;
    return -1;
}
int wave_index(int v) {
    for (int i = 0; i < kWaves; ++i)
        if (kWaveVal[i] == v) return i;
    return -1;
}
}  // namespace

static int check_shape(int dims, int split, int waves) {
    if (split_index(split) < 0) return fail(CT_EINVAL, "fwd_split must be 1, 2 or 4 (got %d)", split);
    if (wave_index(waves) < 0) return fail(CT_EINVAL, "back_waves must be 1, 2, 4, 8 or 16 (got %d)", waves);
    if (dims == 3 && waves != 4) return fail(CT_EINVAL, "the 3D back-projection tile takes 4 waves");
    return CT_OK;
}

// size class: kind, voxels per column block and rays per row block rounded to
// powers of two, GPU architecture
static std::string tune_key(const ct_geom* g) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, g->device) != hipSuccess) prop.gcnArchName[0] = '\0';
    const double vox = (double)g->N / std::max(1, g->n), rays = (double)g->M / std::max(1, g->m);
    char buf[320];
    snprintf(buf, sizeof buf, "%d/%ld/%ld/%s", g->d.kind, std::lround(std::log2(std::max(1.0, vox))),
             std::lround(std::log2(std::max(1.0, rays))), prop.gcnArchName);
    return buf;
}

// Time every shape as kTuneReps epochs (after one untimed) of a scratch solver
// on the schedule's first epoch.
static int tune_measure(ct_geom* g, const ct_schedule* sc, TuneTable* t, hipStream_t st) {
    if (sc->ecp.size() < 2) return fail(CT_EINVAL, "the schedule has no epoch");
    const ct_solver_params p{CT_SYNC_COLUMN};
    size_t wsb = 0;
    int rc = ct_solver_workspace_bytes(g, &p, &wsb);
    if (rc) return rc;
    void* ws = nullptr;
    float *y = nullptr, *x = nullptr;
    ct_solver* s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const Tune keep = g->tune;
    hipError_t e = hipMalloc(&ws, wsb);
    if (e == hipSuccess) e = hipMalloc((void**)&y, (size_t)g->M * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void**)&x, (size_t)g->N * sizeof(float));
    if (e == hipSuccess) e = hipMemsetAsync(y, 0, (size_t)g->M * sizeof(float), st);
    if (e == hipSuccess) e = hipMemsetAsync(x, 0, (size_t)g->N * sizeof(float), st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) rc = fail(CT_EDEVICE, "tuner scratch: %s", hipGetErrorString(e));
    if (!rc) rc = ct_solver_create(g, &p, ws, wsb, &s);
    if (!rc) rc = ct_solver_reset(s, y, nullptr, st);
    for (int i = 0; i < kSplits && !rc; ++i) {
        for (int j = 0; j < kWaves && !rc; ++j) {
            t->ms[i][j] = -1.0;
            if (g->dims == 3 && kWaveVal[j] != 4) continue;
            g->tune.split = kSplitVal[i];
            g->tune.waves = kWaveVal[j];
            rc = ct_block_epoch(s, sc, 0, y, x, st);
            if (!rc && (e = hipEventRecord(e0, st)) != hipSuccess) rc = fail(CT_EDEVICE, "%s", hipGetErrorString(e));
            for (int r = 0; r < kTuneReps && !rc; ++r) rc = ct_block_epoch(s, sc, 0, y, x, st);
            if (!rc && (e = hipEventRecord(e1, st)) != hipSuccess) rc = fail(CT_EDEVICE, "%s", hipGetErrorString(e));
            if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = fail(CT_EDEVICE, "%s", hipGetErrorString(e));
            float ms = 0.f;
            if (!rc && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = fail(CT_EDEVICE, "%s", hipGetErrorString(e));
            if (!rc) t->ms[i][j] = (double)ms / kTuneReps;
        }
    }
    g->tune = keep;
    if (s) ct_solver_destroy(s);
    (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (x) (void)hipFree(x);
    if (y) (void)hipFree(y);
    if (ws) (void)hipFree(ws);
    return rc;
}

// The table of a geometry's size class: from the cache, or timed (and cached).
static int tune_table(ct_geom* g, const ct_schedule* sc, bool refresh, TuneTable* t, bool* cached,
                      hipStream_t st) {
    const std::string key = tune_key(g);
    if (!refresh) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *t = it->second;
            *cached = true;
            return CT_OK;
        }
    }
    int rc = tune_measure(g, sc, t, st);
    if (rc) return rc;
    *cached = false;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = *t;
    return CT_OK;
}

static void tune_pick(const double (&ms)[kSplits][kWaves], int* bi, int* bj) {
    *bi = split_index(kSplit);
    *bj = wave_index(4);
    for (int i = 0; i < kSplits; ++i)
        for (int j = 0; j < kWaves; ++j)
            if (ms[i][j] >= 0 && (ms[*bi][*bj] < 0 || ms[i][j] < ms[*bi][*bj])) {
                *bi = i;
                *bj = j;
            }
}

extern "C" int ct_geom_set_tuning(ct_geom* g, const ct_tuning* t) {
    if (!g || !t) return fail(CT_EINVAL, "NULL argument");
    int rc = check_shape(g->dims, t->fwd_split, t->back_waves);
    if (rc) return rc;
    g->tune.split = t->fwd_split;
    g->tune.waves = t->back_waves;
    return CT_OK;
}

extern "C" int ct_geom_get_tuning(const ct_geom* g, ct_tuning* t) {
    if (!g || !t) return fail(CT_EINVAL, "NULL argument");
    std::memset(t, 0, sizeof *t);
    t->fwd_split = g->tune.split;
    t->back_waves = g->tune.waves;
    return CT_OK;
}

extern "C" int ct_geom_tune(ct_geom* g, const ct_schedule* sc, int32_t flags, ct_tuning* out, void* stream) {
    if (!g || !sc) return fail(CT_EINVAL, "NULL argument");
    if (flags & ~CT_TUNE_REFRESH) return fail(CT_EINVAL, "unknown flags 0x%x", flags);
    if (sc->geom != g) return fail(CT_EINVAL, "schedule was built for another geometry");
    int rc = check_device(g);
    if (rc) return rc;
    TuneTable t{};
    bool cached = false;
    if ((rc = tune_table(g, sc, (flags & CT_TUNE_REFRESH) != 0, &t, &cached, (hipStream_t)stream))) return rc;
    int bi, bj;
    tune_pick(t.ms, &bi, &bj);
    g->tune.split = kSplitVal[bi];
    g->tune.waves = kWaveVal[bj];
    if (out) {
        std::memset(out, 0, sizeof *out);
        out->fwd_split = g->tune.split;
        out->back_waves = g->tune.waves;
        out->ms = t.ms[bi][bj];
        out->ms_default = t.ms[split_index(kSplit)][wave_index(4)];
        out->cached = cached ? 1 : 0;
        if (!cached)
            for (int i = 0; i < kSplits; ++i)
                for (int j = 0; j < kWaves; ++j) out->trials += t.ms[i][j] >= 0 ? 1 : 0;
    }
    return CT_OK;
}

extern "C" int ct_batch_tune(ct_batch* b, int32_t flags, ct_tuning* out, void* stream) {
    if (!b) return fail(CT_EINVAL, "NULL argument");
    if (flags & ~CT_TUNE_REFRESH) return fail(CT_EINVAL, "unknown flags 0x%x", flags);
    if (out) std::memset(out, 0, 4 * sizeof *out);
    double tot[4][kSplits][kWaves] = {};
    bool have[4] = {false, false, false, false};
    int trials[4] = {0, 0, 0, 0}, all_cached[4] = {1, 1, 1, 1};
    std::vector<std::string> refreshed;
    for (const BatchSlot& j : b->jobs) {
        ct_geom* g = j.job.solver->geom;
        const ct_schedule* sc = j.job.sched;
        int rc = check_device(g);
        if (rc) return rc;
        const std::string key = tune_key(g);
        const bool refresh = (flags & CT_TUNE_REFRESH) &&
                             std::find(refreshed.begin(), refreshed.end(), key) == refreshed.end();
        TuneTable t{};
        bool cached = false;
        if ((rc = tune_table(g, sc, refresh, &t, &cached, (hipStream_t)stream))) return rc;
        if (refresh) refreshed.push_back(key);
        const int k = g->d.kind;
        for (int i = 0; i < kSplits; ++i)
            for (int q = 0; q < kWaves; ++q) {
                if (!have[k]) tot[k][i][q] = t.ms[i][q];
                else if (t.ms[i][q] < 0 || tot[k][i][q] < 0) tot[k][i][q] = -1.0;
                else tot[k][i][q] += t.ms[i][q];
                if (!cached && t.ms[i][q] >= 0) ++trials[k];
            }
        if (!cached) all_cached[k] = 0;
        have[k] = true;
    }
    for (int k = 0; k < 4; ++k) {
        if (!have[k]) continue;
        int bi, bj;
        tune_pick(tot[k], &bi, &bj);
        b->tune[k].split = kSplitVal[bi];
        b->tune[k].waves = kWaveVal[bj];
        if (out) {
            out[k].fwd_split = kSplitVal[bi];
            out[k].back_waves = kWaveVal[bj];
            out[k].ms = tot[k][bi][bj];
            out[k].ms_default = tot[k][split_index(kSplit)][wave_index(4)];
            out[k].trials = trials[k];
            out[k].cached = all_cached[k];
        }
    }
    for (BatchSlot& j : b->jobs) j.job.solver->geom->tune = b->tune[j.job.solver->geom->d.kind];
    batch_drop_graph(b);
    return CT_OK;
}

extern "C" int ct_batch_set_tuning(ct_batch* b, int32_t kind, const ct_tuning* t) {
    if (!b || !t) return fail(CT_EINVAL, "NULL argument");
    if (kind < 0 || kind > 3) return fail(CT_EINVAL, "unknown kind %d", kind);
    int rc = check_shape(kind == CT_CONE3D_FLAT ? 3 : 2, t->fwd_split, t->back_waves);
    if (rc) return rc;
    b->tune[kind].split = t->fwd_split;
    b->tune[kind].waves = t->back_waves;
    batch_drop_graph(b);
    return CT_OK;
}

extern "C" int ct_job_footprint(const ct_geom_desc* desc, const ct_solver_params* p, size_t* bytes) {
    if (!bytes) return fail(CT_EINVAL, "NULL argument");
    ct_geom tmp;
    int rc = build_host(&tmp, desc);
    if (rc) return rc;
    (void)p;
    *bytes = dev_layout(&tmp).total + ws_layout(&tmp).total;
    return CT_OK;
}

extern "C" const char* ct_last_error(void) { return g_err.c_str(); }
