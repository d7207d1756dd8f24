// Host runtime of the tpx library: argument validation, the workspace plan,
// geometry tables (interpolation weights and per-tile injection lists), and
// the time-loop drivers behind the C-ABI of include/tpx.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "tpx.h"
#include "tpx_internal.h"

using namespace tpx;

namespace {

thread_local std::string g_err;

tpx_status fail(tpx_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define TPX_HIP(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(TPX_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------------------
// optional per-launch timing with HIP events on the launch stream
// ---------------------------------------------------------------------------
struct ProfRec {
    int kind;
    int64_t launches;
    hipEvent_t a, b;
};

// Consecutive launches of one kernel kind on one stream form a run that is
// bracketed by a single pair of events, so the timing adds no event packets
// between the kernels of a run.
struct Profiler {
    std::mutex mu;
    std::atomic<bool> on{false};   // read without the lock on every launch
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<ProfRec> recs;
    int run_kind = -1;
    int64_t run_launches = 0;
    hipStream_t run_stream = nullptr;
    hipEvent_t run_start = nullptr;
};

Profiler &profiler() {
    static Profiler p;
    return p;
}

hipEvent_t take_event(Profiler &p) {
    if (p.used == p.pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p.pool.push_back(e);
    }
    return p.pool[p.used++];
}

void close_run(Profiler &p) {
    if (p.run_kind < 0) return;
    hipEvent_t b = take_event(p);
    if (b && hipEventRecord(b, p.run_stream) == hipSuccess)
        p.recs.push_back({p.run_kind, p.run_launches, p.run_start, b});
    p.run_kind = -1;
    p.run_launches = 0;
}

enum { KIND_OTHER = 99 };

template <class F>
hipError_t prof(int kind, hipStream_t s, F &&launch) {
    Profiler &p = profiler();
    if (!p.on) return launch();
    std::lock_guard<std::mutex> lk(p.mu);
    if (kind != p.run_kind || s != p.run_stream) {
        close_run(p);
        hipEvent_t a = take_event(p);
        if (!a) return launch();
        hipError_t e = hipEventRecord(a, s);
        if (e != hipSuccess) return e;
        p.run_kind = kind;
        p.run_stream = s;
        p.run_start = a;
        p.run_launches = 0;
    }
    const hipError_t e = launch();
    if (e == hipSuccess) ++p.run_launches;
    return e;
}

// Sum of |weights| of the centred second-difference stencil (Taylor
// coefficients): bounds the spectral radius of the discrete Laplacian.
double stencil_abs_sum(int order) { return order == 4 ? 16.0 / 3.0 : 6.501587301587302; }

// Centred second-derivative weights (Taylor expansion): centre, then distance 1..R.
void stencil_weights(int order, double c[5]) {
    for (int i = 0; i < 5; ++i) c[i] = 0.0;
    if (order == 4) {
        c[0] = -2.5;
        c[1] = 4.0 / 3.0;
        c[2] = -1.0 / 12.0;
    } else {
        c[0] = -205.0 / 72.0;
        c[1] = 1.6;
        c[2] = -0.2;
        c[3] = 8.0 / 315.0;
        c[4] = -1.0 / 560.0;
    }
}

// Most leapfrog steps one 2D launch advances: 3 (default) or 2.  On the
// 16-shot 801 x 301 gradient three-step launches take 11.3 us per step against
// 11.7 for two-step ones; on small problems, bound by each launch's latency,
// a third of the launches go.
std::atomic<int> g_steps2d{3};

struct Problem {
    Layout L;
    Layout L3;          // 2D: tiles and maps of the three-step kernel (valid when `three`)
    bool three = false; // 2D launches may advance three steps
    Physics ph;
    int nt;
    double dt;
    double h;
    int nrec;
};

tpx_status make_problem(const tpx_grid *g, const tpx_geom *geo, Problem *P) {
    if (!g || !geo) return fail(TPX_E_INVAL, "grid and geometry must not be NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(TPX_E_INVAL, "ndim must be 2 or 3");
    if (g->space_order != 4 && g->space_order != 8) return fail(TPX_E_INVAL, "space_order must be 4 or 8");
    if (g->n[0] < 2 || g->n[2] < 2 || (g->ndim == 3 && g->n[1] < 2) || (g->ndim == 2 && g->n[1] != 1))
        return fail(TPX_E_INVAL, "grid sizes: n[0], n[2] >= 2; n[1] >= 2 in 3D and == 1 in 2D");
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(TPX_E_INVAL, "h must be positive");
    if (!(g->dt > 0.0) || !std::isfinite(g->dt)) return fail(TPX_E_INVAL, "dt must be positive");
    if (g->nt < 2) return fail(TPX_E_INVAL, "nt must be >= 2");
    if (g->nbl < 0) return fail(TPX_E_INVAL, "nbl must be >= 0");
    if (!(g->damp_vmax > 0.0)) return fail(TPX_E_INVAL, "damp_vmax must be positive");
    if (!(g->damp_R > 0.0 && g->damp_R <= 1.0)) return fail(TPX_E_INVAL, "damp_R must be in (0, 1]");
    if (geo->nshots < 1 || geo->nrec < 0) return fail(TPX_E_INVAL, "nshots >= 1 and nrec >= 0 required");
    if (!geo->src_pos || (geo->nrec > 0 && !geo->rec_pos))
        return fail(TPX_E_INVAL, "source/receiver positions must not be NULL");
    // leapfrog stability: dt <= 2 h / (vmax sqrt(D sum|c|))
    const double limit = 2.0 * g->h / (g->damp_vmax * std::sqrt((double)g->ndim * stencil_abs_sum(g->space_order)));
    if (g->dt > limit * (1.0 + 1e-12)) {
        char buf[160];
        snprintf(buf, sizeof buf, "dt = %g ms exceeds the stability limit %g ms for vmax = %g km/s", g->dt, limit,
                 g->damp_vmax);
        return fail(TPX_E_CFL, buf);
    }

    Layout &L = P->L;
    L.ndim = g->ndim;
    L.R = g->space_order / 2;
    L.nb = g->nbl;
    L.S = geo->nshots;
    for (int a = 0; a < 3; ++a) L.n[a] = g->n[a];
    L.P[0] = L.n[0] + 2 * L.nb;
    L.P[1] = L.ndim == 3 ? L.n[1] + 2 * L.nb : 1;
    L.P[2] = L.n[2] + 2 * L.nb;
    const int64_t need0 = XO + L.P[0] + L.R;
    L.G[0] = (need0 + 31) / 32 * 32;
    L.G[1] = L.ndim == 3 ? L.P[1] + 2 * L.R : 1;
    L.G[2] = L.P[2] + 2 * L.R;
    L.oy = L.ndim == 3 ? L.R : 0;
    L.shot_floats = L.G[0] * L.G[1] * L.G[2];
    L.slot_floats = L.shot_floats * L.S;
    L.nphys = L.n[0] * L.n[1] * L.n[2];
    L.npad = L.P[0] * L.P[1] * L.P[2];
    if (L.shot_floats >= (int64_t)1 << 31) return fail(TPX_E_INVAL, "one shot's field exceeds 2^31 floats");
    // the step kernels address one shot's field with 32-bit byte offsets
    if (L.shot_floats >= (int64_t)1 << 30) return fail(TPX_E_INVAL, "one shot's field exceeds 2^30 floats");
    if (L.ndim == 2) {
        // tile height: the default unless a launch would give the 256 CUs
        // fewer than two tiles each
        const int64_t tiles32 = L.S * ((L.P[0] + t2x(L.R) - 1) / t2x(L.R)) * ((L.P[2] + T2Z - 1) / T2Z);
        const int tz = tiles32 >= 512 ? T2Z : (tiles32 >= 384 ? T2Z_MID : T2Z_SMALL);
        L.tile[0] = t2x(L.R); L.tile[1] = 1; L.tile[2] = tz;
        L.map[0] = 64; L.map[1] = 1; L.map[2] = tz + 2 * L.R;
        L.map_org[0] = -L.R; L.map_org[1] = 0; L.map_org[2] = -L.R;
    } else {
        // tiles of the two-step kernel, one plane deep; the map of a tile's
        // plane covers the extended region the kernel's first step computes
        L.tile[0] = t2x(L.R); L.tile[1] = T3Y2; L.tile[2] = 1;
        L.map[0] = 64; L.map[1] = T3Y2 + 2 * L.R; L.map[2] = 1;
        L.map_org[0] = -L.R; L.map_org[1] = -L.R; L.map_org[2] = 0;
    }
    for (int a = 0; a < 3; ++a) L.ntiles[a] = (L.P[a] + L.tile[a] - 1) / L.tile[a];
    L.tiles_per_shot = L.ntiles[0] * L.ntiles[1] * L.ntiles[2];
    L.tz3 = 0;
    P->three = false;
    if (L.ndim == 2 && g_steps2d.load() >= 3) {
        // three-step tiles: t3x(R) columns and the two-step tiles' height, maps
        // over the first step's region (the tile plus 2R on every side)
        Layout &L3 = P->L3;
        L3 = L;
        L3.tile[0] = t3x(L.R);
        L3.map[2] = (int)L.tile[2] + 4 * L.R;
        L3.map_org[0] = -2 * L.R;
        L3.map_org[2] = -2 * L.R;
        for (int a = 0; a < 3; ++a) L3.ntiles[a] = (L3.P[a] + L3.tile[a] - 1) / L3.tile[a];
        L3.tiles_per_shot = L3.ntiles[0] * L3.ntiles[1] * L3.ntiles[2];
        P->three = true;
    }
    if (L.ndim == 3) {
        // z chunks of the two-step kernel: about 32 planes, shorter when the
        // launch would otherwise hold fewer than 2048 blocks (8 per CU), never
        // under 8 planes; chunks of one column get equal lengths
        const int64_t cols = L.ntiles[0] * L.ntiles[1] * L.S;
        int64_t nzc = (L.P[2] + 31) / 32;
        const int64_t nzc_max = std::max<int64_t>(1, L.P[2] / 8);
        while (nzc < nzc_max && cols * nzc < 2048) ++nzc;
        L.tz3 = (int)((L.P[2] + nzc - 1) / nzc);
    }

    double c[5];
    stencil_weights(g->space_order, c);
    const double ih2 = 1.0 / (g->h * g->h);
    for (int i = 0; i < 5; ++i) P->ph.c[i] = (float)(c[i] * ih2);
    const double dmax = L.nb > 0 ? 3.0 * g->damp_vmax / (2.0 * L.nb * g->h) * std::log(1.0 / g->damp_R) : 0.0;
    P->ph.hd_max = (float)(0.5 * dmax * g->dt);
    P->ph.inv_nb = L.nb > 0 ? (float)(1.0 / L.nb) : 0.0f;
    P->nt = g->nt;
    P->dt = g->dt;
    P->h = g->h;
    P->nrec = geo->nrec;
    return TPX_OK;
}

// ---------------------------------------------------------------------------
// geometry tables
// ---------------------------------------------------------------------------

struct Corners {
    int cnt;
    int64_t ix[8], iy[8], iz[8];  // padded coordinates
    double w[8];
};

// Bilinear / trilinear weights: base node i0 = min(floor(x/h), n-2),
// fraction x/h - i0; order of corners: z, then y, then x (x fastest).
bool corners_of(const Problem &P, const tpx_grid *g, const double pos[3], Corners *c) {
    const Layout &L = P.L;
    int64_t i0[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < 3; ++a) {
        if (L.ndim == 2 && a == 1) continue;
        const double x = pos[a] / g->h;
        if (!(x >= 0.0) || x > (double)(L.n[a] - 1) * (1.0 + 1e-12)) return false;
        int64_t b = (int64_t)std::floor(x);
        if (b > L.n[a] - 2) b = L.n[a] - 2;
        i0[a] = b;
        f[a] = x - (double)b;
    }
    const int ny = L.ndim == 3 ? 2 : 1;
    const int64_t oyb = L.ndim == 3 ? L.nb : 0;
    c->cnt = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < ny; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                double w = (dx ? f[0] : 1.0 - f[0]) * (dz ? f[2] : 1.0 - f[2]);
                if (L.ndim == 3) w *= (dy ? f[1] : 1.0 - f[1]);
                const int i = c->cnt++;
                c->ix[i] = i0[0] + dx + L.nb;
                c->iy[i] = i0[1] + dy + oyb;
                c->iz[i] = i0[2] + dz + L.nb;
                c->w[i] = w;
            }
    return true;
}

// Host image of the tables, uploaded into the workspace at set-up.  The dense
// injection maps of a large problem run to megabytes, and fresh memory of that
// size costs a page fault per 4 KiB page on every call, all of it before the
// call's first launch.  So each thread keeps one blob's storage between calls
// (up to kBlobKeep bytes); a second blob alive on the same thread at the same
// time gets storage of its own.
constexpr size_t kBlobKeep = size_t(64) << 20;
thread_local std::vector<unsigned char> tl_blob;
thread_local bool tl_blob_busy = false;

struct Blob {
    std::vector<unsigned char> own;
    std::vector<unsigned char> *buf;
    size_t size = 0;   // bytes in use (each part starts kAlign-aligned)
    bool borrowed = false;
    Blob() : buf(&own) {
        if (!tl_blob_busy) {
            tl_blob_busy = borrowed = true;
            buf = &tl_blob;
        }
    }
    ~Blob() {
        if (!borrowed) return;
        if (tl_blob.capacity() > kBlobKeep) std::vector<unsigned char>().swap(tl_blob);
        tl_blob_busy = false;
    }
    Blob(const Blob &) = delete;
    Blob &operator=(const Blob &) = delete;
    // n more bytes at an aligned offset, which is returned; contents undefined
    size_t grow(size_t n) {
        const size_t off = size;
        size = align_up(off + n);
        if (buf->size() < size) buf->resize(std::max(size, buf->size() + buf->size() / 2));
        return off;
    }
    size_t put(const void *p, size_t n) {
        const size_t off = grow(n);
        if (n) memcpy(buf->data() + off, p, n);
        return off;
    }
    unsigned char *data() { return buf->data(); }
    bool empty() const { return size == 0; }
};

struct HostInject {  // offsets into the blob
    size_t tile_dense, dense, seg_ent, ent_idx, ent_w, col_z;
};
struct HostSample {
    size_t base, w;
    int32_t n;
};

struct Entry {
    int64_t tile;
    int32_t local;
    int32_t idx;
    float w;
};

// Injection tables: entries sorted by (tile, target node, source index); a
// segment is the run of entries of one target node.  Every tile that has at
// least one segment gets a dense map "node of the tile -> segment or -1", so a
// step kernel finds the source term of each of its nodes with one load.
HostInject add_inject(Blob &b, const Problem &P, std::vector<Entry> &ent) {
    const Layout &L = P.L;
    std::sort(ent.begin(), ent.end(), [](const Entry &a, const Entry &c) {
        if (a.tile != c.tile) return a.tile < c.tile;
        if (a.local != c.local) return a.local < c.local;
        if (a.idx != c.idx) return a.idx < c.idx;
        return a.w < c.w;
    });
    const int64_t ntile = (int64_t)L.S * L.tiles_per_shot;
    const int64_t tp = (int64_t)L.map[0] * L.map[1] * L.map[2];
    std::vector<int32_t> tile_dense(ntile, -1), seg_ent, ent_idx;
    std::vector<float> ent_w;
    seg_ent.reserve(ent.size() + 1);
    ent_idx.reserve(ent.size());
    ent_w.reserve(ent.size());
    // the dense maps are written straight into the blob
    int64_t nmaps = 0;
    for (size_t i = 0; i < ent.size(); ++i) nmaps += i == 0 || ent[i].tile != ent[i - 1].tile;
    const size_t dense_off = b.grow((size_t)(nmaps * tp) * 4);
    int32_t *dense = (int32_t *)(b.data() + dense_off);   // valid until the next grow
    std::fill(dense, dense + nmaps * tp, -1);
    int32_t nseg = 0, nmap = 0;
    for (size_t i = 0; i < ent.size(); ++i) {
        const bool new_tile = i == 0 || ent[i].tile != ent[i - 1].tile;
        const bool new_seg = new_tile || ent[i].local != ent[i - 1].local;
        if (new_tile) tile_dense[ent[i].tile] = nmap++;
        if (new_seg) {
            dense[(size_t)tile_dense[ent[i].tile] * tp + ent[i].local] = nseg++;
            seg_ent.push_back((int32_t)i);
        }
        ent_idx.push_back(ent[i].idx);
        ent_w.push_back(ent[i].w);
    }
    seg_ent.push_back((int32_t)ent.size());
    // 3D: the first and last plane holding a map, per tile column (shot, y, x)
    const int64_t ncol = L.ndim == 3 ? (int64_t)L.S * L.ntiles[0] * L.ntiles[1] : 0;
    std::vector<int32_t> col_z(2 * ncol);
    for (int64_t c = 0; c < ncol; ++c) {
        col_z[2 * c] = INT32_MAX;
        col_z[2 * c + 1] = -1;
    }
    for (size_t i = 0; i < ent.size() && ncol; ++i) {
        const int64_t t = ent[i].tile, cxy = L.ntiles[0] * L.ntiles[1];
        const int64_t z = (t / cxy) % L.ntiles[2], c = (t / (cxy * L.ntiles[2])) * cxy + t % cxy;
        col_z[2 * c] = std::min<int32_t>(col_z[2 * c], (int32_t)z);
        col_z[2 * c + 1] = std::max<int32_t>(col_z[2 * c + 1], (int32_t)z);
    }
    HostInject h;
    h.col_z = b.put(col_z.data(), col_z.size() * 4);
    h.tile_dense = b.put(tile_dense.data(), tile_dense.size() * 4);
    h.dense = dense_off;
    h.seg_ent = b.put(seg_ent.data(), seg_ent.size() * 4);
    h.ent_idx = b.put(ent_idx.data(), ent_idx.size() * 4);
    h.ent_w = b.put(ent_w.data(), ent_w.size() * 4);
    return h;
}

// Tiles t along one axis whose map [t * tile + org, t * tile + org + extent)
// contains padded index i.
void tiles_covering(int64_t i, int tile, int org, int extent, int64_t ntiles, int64_t *lo, int64_t *hi) {
    // t * tile <= i - org  and  t * tile > i - org - extent
    const int64_t a = i - org - extent + 1, b = i - org;
    *lo = a <= 0 ? 0 : (a + tile - 1) / tile;
    *hi = b < 0 ? -1 : b / tile;
    if (*hi > ntiles - 1) *hi = ntiles - 1;
}

// One entry per (tile whose map contains the corner node, corner).
void push_corners(const Problem &P, const Corners &c, int shot, int idx, std::vector<Entry> &ent) {
    const Layout &L = P.L;
    for (int i = 0; i < c.cnt; ++i) {
        if (c.w[i] == 0.0) continue;  // contributes exactly nothing
        const int64_t pos[3] = {c.ix[i], c.iy[i], c.iz[i]};
        int64_t lo[3], hi[3];
        for (int d = 0; d < 3; ++d) tiles_covering(pos[d], L.tile[d], L.map_org[d], L.map[d], L.ntiles[d], &lo[d], &hi[d]);
        for (int64_t tz = lo[2]; tz <= hi[2]; ++tz)
            for (int64_t ty = lo[1]; ty <= hi[1]; ++ty)
                for (int64_t tx = lo[0]; tx <= hi[0]; ++tx) {
                    const int64_t mx = pos[0] - (tx * L.tile[0] + L.map_org[0]);
                    const int64_t my = pos[1] - (ty * L.tile[1] + L.map_org[1]);
                    const int64_t mz = pos[2] - (tz * L.tile[2] + L.map_org[2]);
                    Entry e;
                    e.tile = (((int64_t)shot * L.ntiles[2] + tz) * L.ntiles[1] + ty) * L.ntiles[0] + tx;
                    e.local = (int32_t)((mz * L.map[1] + my) * L.map[0] + mx);
                    e.idx = idx;
                    e.w = (float)c.w[i];
                    ent.push_back(e);
                }
    }
}

HostSample add_sample(Blob &b, const Problem &P, const std::vector<Corners> &cs) {
    const int nc = P.L.ndim == 3 ? 8 : 4;
    std::vector<int32_t> base(cs.size());
    std::vector<float> w(cs.size() * nc);
    for (size_t i = 0; i < cs.size(); ++i) {
        base[i] = (int32_t)P.L.pad_off(cs[i].ix[0], cs[i].iy[0], cs[i].iz[0]);
        for (int j = 0; j < nc; ++j) w[i * nc + j] = (float)cs[i].w[j];
    }
    HostSample h;
    h.base = b.put(base.data(), base.size() * 4);
    h.w = b.put(w.data(), w.size() * 4);
    return h;
}

struct Tables {
    Blob blob;
    HostInject src_inj, rec_inj;
    HostInject src_inj3, rec_inj3;   // three-step layout (2D, when the problem allows it)
    HostSample rec_smp, src_smp;
};

tpx_status build_tables(const Problem &P, const tpx_grid *g, const tpx_geom *geo, Tables *T) {
    const int S = P.L.S;
    std::vector<Corners> src(S), rec((size_t)S * P.nrec);
    for (int s = 0; s < S; ++s) {
        if (!corners_of(P, g, &geo->src_pos[3 * s], &src[s])) {
            char buf[128];
            snprintf(buf, sizeof buf, "source of shot %d lies outside the physical grid", s);
            return fail(TPX_E_GEOM, buf);
        }
        for (int i = 0; i < P.nrec; ++i)
            if (!corners_of(P, g, &geo->rec_pos[3 * ((int64_t)s * P.nrec + i)], &rec[(size_t)s * P.nrec + i])) {
                char buf[128];
                snprintf(buf, sizeof buf, "receiver %d of shot %d lies outside the physical grid", i, s);
                return fail(TPX_E_GEOM, buf);
            }
    }
    std::vector<Entry> es, er;
    for (int s = 0; s < S; ++s) push_corners(P, src[s], s, 0, es);
    for (int s = 0; s < S; ++s)
        for (int i = 0; i < P.nrec; ++i) push_corners(P, rec[(size_t)s * P.nrec + i], s, i, er);
    T->src_inj = add_inject(T->blob, P, es);
    T->rec_inj = add_inject(T->blob, P, er);
    if (P.three) {
        Problem P3 = P;
        P3.L = P.L3;
        std::vector<Entry> es3, er3;
        for (int s = 0; s < S; ++s) push_corners(P3, src[s], s, 0, es3);
        for (int s = 0; s < S; ++s)
            for (int i = 0; i < P.nrec; ++i) push_corners(P3, rec[(size_t)s * P.nrec + i], s, i, er3);
        T->src_inj3 = add_inject(T->blob, P3, es3);
        T->rec_inj3 = add_inject(T->blob, P3, er3);
    }
    T->rec_smp = add_sample(T->blob, P, rec);
    T->rec_smp.n = P.nrec;
    T->src_smp = add_sample(T->blob, P, src);
    T->src_smp.n = 1;
    return TPX_OK;
}

// ---------------------------------------------------------------------------
// workspace plan
// ---------------------------------------------------------------------------

// Library options (tpx_set_option).  Overlap: probe contractions run on an
// auxiliary stream, concurrently with the next block of time steps.
std::atomic<int> g_overlap{0};
// Matrix-core contractions: 0 never; 1 (default) where they were measured
// faster: the folded adjoint contraction for r >= 32, the accumulations of
// ubar and vbar for r >= 64; 2 every contraction whenever the probes qualify
// (a kind exact in bfloat16 and r a multiple of 16).
std::atomic<int> g_mfma{1};
// Two fused leapfrog steps per 3D launch (2D launches always fuse two).
std::atomic<int> g_fused3d{0};

// Auxiliary streams, created on first use and kept for the process lifetime.
std::mutex g_aux_mu;
std::vector<hipStream_t> g_aux_free;

hipError_t aux_acquire(hipStream_t *s) {
    std::lock_guard<std::mutex> lk(g_aux_mu);
    if (!g_aux_free.empty()) {
        *s = g_aux_free.back();
        g_aux_free.pop_back();
        return hipSuccess;
    }
    return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

void aux_release(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_aux_mu);
    g_aux_free.push_back(s);
}

// Ring slots for a time block of b steps: b + 2 when the contractions run in
// stream order; 2 b + 3 when a block's contraction overlaps the next block.
int ring_slots(int b, bool overlap) { return overlap ? 2 * b + 3 : b + 2; }

// Time steps buffered per probe contraction.  The accumulators' read-modify-
// write costs 8 r / b bytes per point-step against the 4 bytes of the ring
// read, and the ring holds ring_slots(b) wavefield levels.  b starts at 16 r
// (the accumulator traffic at an eighth of the ring's), within 256 .. 1024.
// It is then lowered, in steps of 16 levels, until the ring takes at most
// max(6 x the accumulators, 8 GB): the probed workspace stays a small multiple
// of the r x N accumulators the method keeps, instead of growing with the
// grid to a large share of the GPU's memory.
int default_block(const Layout &L, int nt, bool overlap, int r) {
    const double slot_bytes = (double)L.slot_floats * 4.0;
    const double acc_bytes = (double)L.S * r * L.nphys * 4.0;
    const double cap = std::max(6.0 * acc_bytes, 8e9);
    int b = 256;
    while (b < 1024 && b < 16 * r) b *= 2;
    while (b > 16 && ring_slots(b, overlap) * slot_bytes > cap) b -= 16;
    if (b > nt - 1) b = nt - 1;
    if (b < 1) b = 1;
    return b;
}

struct Plan {
    size_t flags, parts, J, beta, ring, hist, Z, zpk, rfW, rfY, rfX, ubar, vbar, gpart, res, d, tables, total;
    int nslots, block;
    bool overlap;
};

enum Mode { M_FORWARD, M_ADJOINT, M_GRAD_PROBED, M_GRAD_FULL, M_FWD_PROBED, M_BWD_PROBED, M_RANGE_FINDER, M_OBJECTIVE };

// Probes whose count is a multiple of 16 can be contracted on the matrix
// cores: in one bfloat16 part when their entries are exact in bfloat16 (the
// counter-hash kinds and the identity), split in three parts otherwise.
bool mfma_eligible(const tpx_probe *pr) { return pr && pr->r % 16 == 0; }

int probe_parts(const tpx_probe *pr) {
    const bool exact = pr->kind == TPX_PROBE_RADEMACHER || pr->kind == TPX_PROBE_GAUSS_B64 ||
                       pr->kind == TPX_PROBE_IDENTITY;
    return exact ? 1 : 3;
}

enum { MFMA_ACCUM = 1, MFMA_FOLD = 2 };

int mfma_selected(const Layout &L, const tpx_probe *pr) {
    const int opt = g_mfma.load();
    if (!mfma_eligible(pr) || opt == 0) return 0;
    // the matrix-core kernels step from ring slot to ring slot with 32-bit strides
    if (L.slot_floats >= ((int64_t)1 << 32)) return 0;
    // the fold reads the caller's explicit probes as 16-byte vectors
    if (pr->kind == TPX_PROBE_EXPLICIT && ((uintptr_t)pr->Z & 15) != 0) return 0;
    if (opt == 2) return MFMA_ACCUM | MFMA_FOLD;
    return (pr->r >= 64 ? MFMA_ACCUM : 0) | (pr->r >= 32 ? MFMA_FOLD : 0);
}

tpx_status check_probe(const Problem &P, const tpx_probe *pr) {
    if (!pr) return fail(TPX_E_INVAL, "probe must not be NULL for probed calls");
    if (pr->r < 1) return fail(TPX_E_INVAL, "r must be >= 1");
    if (pr->kind < 0 || pr->kind > 4) return fail(TPX_E_INVAL, "unknown probe kind");
    if (pr->kind == TPX_PROBE_RANGE_FINDER && (pr->r > 64 || pr->r > P.nrec || pr->r > P.nt))
        return fail(TPX_E_INVAL, "range-finder probes need r <= min(64, nrec, nt)");
    if (pr->kind == TPX_PROBE_IDENTITY && pr->r != P.nt) return fail(TPX_E_INVAL, "identity probes need r == nt");
    if (pr->kind == TPX_PROBE_EXPLICIT && !pr->Z) return fail(TPX_E_INVAL, "explicit probes need Z");
    if (pr->block < 0) return fail(TPX_E_INVAL, "block must be >= 0");
    if (pr->dtt_side != 0 && pr->dtt_side != 1) return fail(TPX_E_INVAL, "dtt_side must be 0 or 1");
    if (pr->imaging != 0 && pr->imaging != 1) return fail(TPX_E_INVAL, "imaging must be 0 or 1");
    if (pr->imaging == 1 && !pr->keep_vbar) return fail(TPX_E_INVAL, "the gradient imaging condition needs keep_vbar = 1");
    return TPX_OK;
}

Plan make_plan(const Problem &P, Mode mode, const tpx_probe *pr, size_t table_bytes, bool allow_overlap = true) {
    const Layout &L = P.L;
    Plan p;
    memset(&p, 0, sizeof p);
    if (mode == M_RANGE_FINDER) {   // FP64 scratch of the range finder only
        p.rfW = 0;
        p.rfY = align_up((size_t)L.S * P.nrec * pr->r * 8);
        p.rfX = p.rfY + align_up((size_t)L.S * P.nt * pr->r * 8);
        p.total = p.rfX + align_up(rf_scratch_doubles(L.S, P.nt, P.nrec, pr->r) * 8);
        return p;
    }
    const bool probed = mode == M_GRAD_PROBED || mode == M_FWD_PROBED || mode == M_BWD_PROBED;
    const int r = probed ? pr->r : 0;
    const bool plain = mode == M_FORWARD || mode == M_ADJOINT || mode == M_OBJECTIVE;
    p.overlap = allow_overlap && g_overlap.load() != 0 && !plain;
    p.block = default_block(L, P.nt, p.overlap, r);
    if (probed && pr->block > 0) p.block = std::min(pr->block, P.nt - 1);
    if (mode == M_GRAD_FULL) p.block = std::min(32, P.nt - 1);
    // without contractions the ring holds the four levels a launch of two
    // fused steps touches, or six with three-step launches (five touched, and
    // the middle one the next launch samples).  With contractions a launch
    // never crosses a block end, so one block plus two levels suffices.
    p.nslots = plain ? (P.three ? 6 : 4) : ring_slots(p.block, p.overlap);
    const size_t slot = (size_t)L.slot_floats * 4;
    const size_t ntr = (size_t)L.S * P.nt * P.nrec;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o += align_up(bytes);
        return at;
    };
    p.flags = take(64);
    p.parts = take(512 * 8);
    p.J = take(8);
    p.beta = take((size_t)L.shot_floats * 4);
    p.ring = take(slot * p.nslots);
    if (mode == M_GRAD_FULL) p.hist = take(slot * (size_t)P.nt);
    if (probed && pr->kind != TPX_PROBE_EXPLICIT) p.Z = take((size_t)L.S * P.nt * r * 4);
    if (probed && mfma_eligible(pr)) p.zpk = take(pack_probes_bytes(L.S, P.nt, r, probe_parts(pr)));
    if (probed && pr->kind == TPX_PROBE_RANGE_FINDER) {
        p.rfW = take((size_t)L.S * P.nrec * pr->r * 8);
        p.rfY = take((size_t)L.S * P.nt * pr->r * 8);
        p.rfX = take(rf_scratch_doubles(L.S, P.nt, P.nrec, pr->r) * 8);
    }
    if (mode == M_GRAD_PROBED) p.ubar = take((size_t)L.S * r * L.nphys * 4);
    const bool keep_v = probed && pr->keep_vbar;
    if ((mode == M_GRAD_PROBED || mode == M_BWD_PROBED) && keep_v) p.vbar = take((size_t)L.S * r * L.nphys * 4);
    if (mode == M_GRAD_FULL || ((mode == M_GRAD_PROBED || mode == M_BWD_PROBED) && !keep_v))
        p.gpart = take((size_t)L.S * L.nphys * 4);
    if (mode == M_GRAD_PROBED || mode == M_GRAD_FULL || mode == M_OBJECTIVE) {
        p.res = take(ntr * 4);
        p.d = take(ntr * 4);
    }
    p.tables = take(table_bytes);
    p.total = o;
    return p;
}

// ---------------------------------------------------------------------------
// drivers
// ---------------------------------------------------------------------------

struct Ctx {
    Problem P;
    Plan plan;
    unsigned char *ws = nullptr;
    hipStream_t stream = nullptr;
    InjectTables src_inj, rec_inj;
    InjectTables src_inj3, rec_inj3;   // three-step layout
    SampleTables rec_smp, src_smp;  // out/scales filled per use
    float *beta = nullptr;
    float *ring = nullptr;
    const void *zpk = nullptr;   // packed probes when the accumulations run on the matrix cores
    bool fold_mfma = false;      // the folded adjoint contraction runs on the matrix cores
    int zparts = 1;              // bfloat16 parts per probe value on the matrix cores
    // overlap of the contractions: auxiliary stream and per-block events
    // (block i uses slot i & 1; the main stream waits for block i's
    // contraction before block i + 2 starts overwriting its ring slots)
    hipStream_t aux = nullptr;
    hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
    // allocation-free call: tables uploaded from pageable memory (the call
    // waits for that copy), contractions never overlapped
    bool no_alloc = false;

    Ctx() = default;
    Ctx(const Ctx &) = delete;
    Ctx &operator=(const Ctx &) = delete;
    ~Ctx() {
        for (int i = 0; i < 2; ++i) {
            if (ev_ready[i]) (void)hipEventDestroy(ev_ready[i]);
            if (ev_done[i]) (void)hipEventDestroy(ev_done[i]);
        }
        if (aux) aux_release(aux);
    }
};

// Hand a finished time block's contraction to the auxiliary stream.
template <class F>
tpx_status overlap_launch(Ctx &C, int block_idx, int kind, F &&launch) {
    const int e = block_idx & 1;
    TPX_HIP(hipEventRecord(C.ev_ready[e], C.stream));
    TPX_HIP(hipStreamWaitEvent(C.aux, C.ev_ready[e], 0));
    TPX_HIP(prof(kind, C.aux, launch));
    TPX_HIP(hipEventRecord(C.ev_done[e], C.aux));
    return TPX_OK;
}

// Before block `block_idx` overwrites ring slots: wait for the contraction of
// block block_idx - 2 (same event slot).
tpx_status overlap_guard(Ctx &C, int block_idx) {
    if (block_idx >= 2) TPX_HIP(hipStreamWaitEvent(C.stream, C.ev_done[block_idx & 1], 0));
    return TPX_OK;
}

// Join: the main stream waits for every contraction enqueued so far.
tpx_status overlap_join(Ctx &C, int nblocks) {
    if (nblocks >= 1) TPX_HIP(hipStreamWaitEvent(C.stream, C.ev_done[(nblocks - 1) & 1], 0));
    return TPX_OK;
}

InjectTables dev_inject(unsigned char *base, const HostInject &h) {
    InjectTables t;
    t.tile_dense = (const int32_t *)(base + h.tile_dense);
    t.col_z = (const int32_t *)(base + h.col_z);
    t.dense = (const int32_t *)(base + h.dense);
    t.seg_ent = (const int32_t *)(base + h.seg_ent);
    t.ent_idx = (const int32_t *)(base + h.ent_idx);
    t.ent_w = (const float *)(base + h.ent_w);
    return t;
}

SampleTables dev_sample(unsigned char *base, const HostSample &h) {
    SampleTables t;
    memset(&t, 0, sizeof t);
    t.nsmp = h.n;
    t.base = (const int32_t *)(base + h.base);
    t.w = (const float *)(base + h.w);
    return t;
}

// Host-to-device upload of the geometry tables without waiting for the
// stream: the bytes are staged in pinned host memory owned by the library and
// a staging buffer is reused only after the event recorded behind its copy has
// completed.  Buffers are never freed here (freeing pinned memory waits for
// the device): a copy takes the smallest idle buffer that holds it, else a new
// buffer of the next power-of-two size joins the pool.
struct Staging {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
};

std::mutex g_stage_mu;
std::vector<Staging> g_stage;

// Pinned copies of tables uploaded while the stream was being captured into a
// HIP graph: every replay of the graph reads them again, so they are never
// reused or freed.
std::vector<void *> g_captured_tables;

hipError_t upload_async(void *dst, const void *src, size_t n, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t ec = hipStreamIsCapturing(stream, &cs);
    if (ec != hipSuccess) return ec;
    if (cs != hipStreamCaptureStatusNone) {
        void *h = nullptr;
        ec = hipHostMalloc(&h, n, hipHostMallocDefault);
        if (ec != hipSuccess) return ec;
        memcpy(h, src, n);
        g_captured_tables.push_back(h);
        return hipMemcpyAsync(dst, h, n, hipMemcpyHostToDevice, stream);
    }
    Staging *use = nullptr;
    for (Staging &st : g_stage) {
        if (st.cap < n || hipEventQuery(st.done) != hipSuccess) continue;   // too small, or copy pending
        if (!use || st.cap < use->cap) use = &st;
    }
    if (!use) {
        size_t cap = 4096;
        while (cap < n) cap *= 2;
        Staging fresh;
        hipError_t e = hipHostMalloc(&fresh.host, cap, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        fresh.cap = cap;
        e = hipEventCreateWithFlags(&fresh.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(fresh.host);
            return e;
        }
        g_stage.push_back(fresh);
        use = &g_stage.back();
    }
    memcpy(use->host, src, n);
    hipError_t e = hipMemcpyAsync(dst, use->host, n, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return e;
    return hipEventRecord(use->done, stream);
}

hipError_t fill_zero_p(void *ptr, size_t bytes, hipStream_t stream) {
    return prof(KIND_OTHER, stream, [&] { return launch_fill_zero(ptr, bytes, stream); });
}

tpx_status setup(Ctx &C, const tpx_grid *g, const tpx_geom *geo, const tpx_probe *pr, Mode mode, const float *m,
                 void *ws, size_t ws_bytes, void *stream) {
    tpx_status st = make_problem(g, geo, &C.P);
    if (st != TPX_OK) return st;
    const bool probed = mode == M_GRAD_PROBED || mode == M_FWD_PROBED || mode == M_BWD_PROBED;
    if (probed) {
        st = check_probe(C.P, pr);
        if (st != TPX_OK) return st;
    }
    if (!m) return fail(TPX_E_INVAL, "model m must not be NULL");
    if (!geo->wavelet && (mode != M_ADJOINT && mode != M_BWD_PROBED))
        return fail(TPX_E_INVAL, "wavelet must not be NULL");
    Tables T;
    st = build_tables(C.P, g, geo, &T);
    if (st != TPX_OK) return st;
    C.plan = make_plan(C.P, mode, pr, T.blob.size, !C.no_alloc);
    if (!ws || ws_bytes < C.plan.total) {
        char buf[160];
        snprintf(buf, sizeof buf, "workspace of %zu bytes is smaller than the %zu bytes required", ws_bytes,
                 C.plan.total);
        return fail(TPX_E_NOMEM, buf);
    }
    C.ws = (unsigned char *)ws;
    C.stream = (hipStream_t)stream;
    unsigned char *tb = C.ws + C.plan.tables;
    if (!T.blob.empty()) {
        if (C.no_alloc) {
            // no pinned staging: copy from the tables' own (pageable) memory and
            // wait for the copy before that memory is released
            TPX_HIP(hipMemcpyAsync(tb, T.blob.data(), T.blob.size, hipMemcpyHostToDevice, C.stream));
            TPX_HIP(hipStreamSynchronize(C.stream));
        } else {
            TPX_HIP(upload_async(tb, T.blob.data(), T.blob.size, C.stream));
        }
    }
    C.src_inj = dev_inject(tb, T.src_inj);
    C.rec_inj = dev_inject(tb, T.rec_inj);
    if (C.P.three) {
        C.src_inj3 = dev_inject(tb, T.src_inj3);
        C.rec_inj3 = dev_inject(tb, T.rec_inj3);
    }
    C.rec_smp = dev_sample(tb, T.rec_smp);
    C.src_smp = dev_sample(tb, T.src_smp);
    C.beta = (float *)(C.ws + C.plan.beta);
    C.ring = (float *)(C.ws + C.plan.ring);
    if (C.plan.overlap) {
        TPX_HIP(aux_acquire(&C.aux));
        for (int i = 0; i < 2; ++i) {
            TPX_HIP(hipEventCreateWithFlags(&C.ev_ready[i], hipEventDisableTiming));
            TPX_HIP(hipEventCreateWithFlags(&C.ev_done[i], hipEventDisableTiming));
        }
    }
    TPX_HIP(fill_zero_p(C.ws + C.plan.flags, kAlign, C.stream));
    const float m_min = (float)(1.0 / (g->damp_vmax * g->damp_vmax) * (1.0 - 1e-5));
    TPX_HIP(prof(KIND_OTHER, C.stream, [&] {
        return launch_model_prep(C.P.L, m, C.P.dt, m_min, C.beta, (int32_t *)(C.ws + C.plan.flags), C.stream);
    }));
    return TPX_OK;
}

float *slot_ptr(float *base, const Layout &L, int nslots, int k) {
    const int s = ((k % nslots) + nslots) % nslots;
    return base + (int64_t)s * L.slot_floats;
}

// Forward propagation over k = 0..nt-2 in the ring (or the history when
// `hist` is set), sampling traces into d.  When `Z` is set, the probed
// wavefield ubar_j += Z[s,j] u^s is accumulated every `block` steps.
// The loop is resumable: fwd_advance runs at most `max_steps` steps per call.
struct FwdLoop {
    StepArgs a;
    SampleTables smp;
    bool sample = false;  // traces requested
    float *buf = nullptr;
    int ns = 0;
    const float *Z = nullptr;
    int r = 0;
    float *ubar = nullptr;
    int dtt = 0;   // 1: ubar accumulates second time differences of u (Algorithm 1 side)
    int k = 0;
    int s_lo = 1;
    int next_row = 0;  // first trace row not sampled yet
    int blk = 0;   // index of the current time block
    bool finished = false;
};

// Two fused steps are used whenever both steps fall in the caller's budget
// and in one contraction block (the ring holds one block plus the two levels
// around it).  With overlapped contractions too: a block's contraction reads
// levels s_lo - 1 .. s_hi + 1 while the next block writes the b levels beyond
// them, 2 b + 2 distinct levels in a ring of 2 b + 3 slots, however the steps
// are paired.
bool two_steps_allowed(const Ctx &C) { return C.P.L.ndim == 2 || g_fused3d.load() != 0; }

// Most steps per launch.  A three-step launch touches five consecutive levels
// and the next launch samples the middle one of its three, so its ring needs
// at least six slots.
int max_steps_per_launch(const Ctx &C, int ring_slots_used) {
    if (!two_steps_allowed(C)) return 1;
    return C.P.three && ring_slots_used >= 6 ? 3 : 2;
}

// Steps of the next launch: at most `most`, and `left` remain in the current
// segment (the record, the caller's budget, the contraction block).  Four
// left under three-step launches go as two and two: a three-step launch and a
// one-step one cost more than two two-step ones.
int steps_for_launch(int most, int64_t left) {
    int n = (int)std::max<int64_t>(std::min<int64_t>(most, left), 1);
    if (n == 3 && left == 4) n = 2;
    return n;
}

tpx_status fwd_begin(Ctx &C, FwdLoop &f, const float *wavelet, float *d, float *hist, const float *Z, int r,
                     float *ubar, int dtt = 0) {
    const Layout &L = C.P.L;
    const int nt = C.P.nt;
    f.buf = hist ? hist : C.ring;
    f.ns = hist ? nt : C.plan.nslots;
    f.Z = Z;
    f.r = r;
    f.ubar = ubar;
    f.dtt = dtt;
    f.k = 0;
    f.s_lo = 1;
    f.next_row = 0;
    f.blk = 0;
    f.finished = false;
    // u^{-1} = u^0 = 0: the first step reads slot 0 as both levels.  Other
    // slots are written before they are read, and ghost cells are never read.
    TPX_HIP(fill_zero_p(slot_ptr(f.buf, L, f.ns, 0), (size_t)L.slot_floats * 4, C.stream));
    // the second difference at k = 0 reads u^{-1} = 0 from the slot before slot 0
    if (Z && dtt) TPX_HIP(fill_zero_p(slot_ptr(f.buf, L, f.ns, -1), (size_t)L.slot_floats * 4, C.stream));
    if (ubar) TPX_HIP(fill_zero_p(ubar, align_up((size_t)L.S * r * L.nphys * 4), C.stream));
    StepArgs &a = f.a;
    memset(&a, 0, sizeof a);
    a.beta = C.beta;
    a.inject = 1;
    a.inj = C.src_inj;
    a.amp.ptr = wavelet;
    a.amp.shot_stride = nt;
    a.amp.k_stride = 1;
    a.amp.scale = 1.0f;
    f.smp = C.rec_smp;
    f.smp.out = d;
    f.smp.out_shot_stride = (int64_t)nt * C.P.nrec;
    f.smp.out_k_stride = C.P.nrec;
    f.smp.scale = 1.0f;
    f.sample = d && f.smp.nsmp > 0;
    a.smp = f.smp;
    return TPX_OK;
}

tpx_status fwd_advance(Ctx &C, FwdLoop &f, int64_t max_steps, int64_t *used) {
    const Layout &L = C.P.L;
    const int nt = C.P.nt;
    StepArgs &a = f.a;
    int64_t n = 0;
    while (f.k <= nt - 2 && n < max_steps) {
        const int k = f.k;
        const int s = k + 1;
        const bool ovl = f.Z && C.plan.overlap;
        // steps in this launch: within the record, the caller's budget and
        // (with contractions) the current block
        int64_t left = std::min<int64_t>(nt - 1 - k, max_steps - n);
        if (f.Z) left = std::min<int64_t>(left, C.plan.block - (s - f.s_lo));
        const int nstep = steps_for_launch(max_steps_per_launch(C, f.ns), left);
        if (ovl && s == f.s_lo) {
            tpx_status st = overlap_guard(C, f.blk);
            if (st != TPX_OK) return st;
        }
        a.nstep = nstep;
        a.k = k;
        a.k2 = k + 1;
        a.k3 = k + 2;
        a.kp = k - 1;
        a.kp2 = k - 2;
        a.cur = slot_ptr(f.buf, L, f.ns, k);
        a.prev = k == 0 ? a.cur : slot_ptr(f.buf, L, f.ns, k - 1);  // u^{-1} = u^0 = 0
        a.prev2 = k >= 2 ? slot_ptr(f.buf, L, f.ns, k - 2) : nullptr;
        a.next = slot_ptr(f.buf, L, f.ns, k + 1);
        a.next2 = nstep >= 2 ? slot_ptr(f.buf, L, f.ns, k + 2) : nullptr;
        a.next3 = nstep == 3 ? slot_ptr(f.buf, L, f.ns, k + 3) : nullptr;
        a.inj = nstep == 3 ? C.src_inj3 : C.src_inj;
        // sample every level read here that is not sampled yet (after a
        // three-step launch, the level two before `cur` too)
        a.do_sample = f.sample && f.next_row <= k;
        a.sample_prev = f.sample && k >= 1 && f.next_row <= k - 1;
        a.sample_prev2 = f.sample && k >= 2 && f.next_row <= k - 2;
        if (f.sample) f.next_row = k + 1;
        const int kind = nstep == 3 ? TPX_KERNEL_STEP3 : nstep == 2 ? TPX_KERNEL_STEP2 : TPX_KERNEL_STEP;
        const Layout &LL = nstep == 3 ? C.P.L3 : L;
        TPX_HIP(prof(kind, C.stream, [&] { return launch_step(LL, C.P.ph, a, C.stream); }));
        f.k += nstep;
        n += nstep;
        const int s_last = k + nstep;  // last level written
        if (f.Z && (s_last - f.s_lo + 1 == C.plan.block || s_last == nt - 1)) {
            const int s_lo = f.s_lo;
            const int s_hi = s_last;
            // levels s_lo..s_hi are new: contract them (dtt 0), or the second
            // differences centred at k = s_lo-1..s_hi-1, which they complete (dtt 1)
            auto contract = [&](hipStream_t cs) {
                if (C.zpk)
                    return f.dtt ? launch_accum_mfma(L, f.buf, f.ns, s_lo - 1, s_hi - 1, C.zpk, C.zparts, nt, f.r, 1,
                                                     f.ubar, cs)
                                 : launch_accum_mfma(L, f.buf, f.ns, s_lo, s_hi, C.zpk, C.zparts, nt, f.r, 0, f.ubar, cs);
                return f.dtt ? launch_accum_adj(L, f.buf, f.ns, s_lo - 1, s_hi - 1, f.Z, nt, f.r, 0, 1, nullptr, 1.0f,
                                                f.ubar, nullptr, cs)
                             : launch_accum_fwd(L, f.buf, f.ns, s_lo, s_hi, f.Z, nt, f.r, f.ubar, cs);
            };
            if (ovl) {
                tpx_status st = overlap_launch(C, f.blk, TPX_KERNEL_ACCUM_FWD, [&] { return contract(C.aux); });
                if (st != TPX_OK) return st;
            } else {
                TPX_HIP(prof(TPX_KERNEL_ACCUM_FWD, C.stream, [&] { return contract(C.stream); }));
            }
            f.s_lo = s_hi + 1;
            ++f.blk;
        }
    }
    if (f.k > nt - 2 && !f.finished) {
        for (; f.sample && f.next_row <= nt - 1; ++f.next_row) {
            const int row = f.next_row;
            TPX_HIP(prof(KIND_OTHER, C.stream, [&] { return launch_sample_only(L, slot_ptr(f.buf, L, f.ns, row), row, f.smp, C.stream); }));
        }
        if (f.Z && C.plan.overlap) {
            tpx_status st = overlap_join(C, f.blk);
            if (st != TPX_OK) return st;
        }
        f.finished = true;
    }
    if (used) *used = n;
    return TPX_OK;
}

tpx_status run_forward(Ctx &C, const float *wavelet, float *d, float *hist, const float *Z, int r, float *ubar,
                       int dtt = 0) {
    FwdLoop f;
    tpx_status st = fwd_begin(C, f, wavelet, d, hist, Z, r, ubar, dtt);
    if (st != TPX_OK) return st;
    return fwd_advance(C, f, INT64_MAX, nullptr);
}

// Adjoint propagation k = nt-1..1 injecting amp/dt^2 at the receivers.
// Optional: q_adj sampling at the source (scale dt^2), probe accumulation
// (fold into gpart or into vbar), or the full-history imaging term.
struct AdjOut {
    float *q_adj = nullptr;
    const float *Z = nullptr;
    int r = 0;
    int fold = 1;
    int dtt = 0;   // 1: contract lam^k itself (Algorithm 1 side), else its second difference
    const float *ubar = nullptr;
    float c = 1.0f;
    float *vbar = nullptr;
    float *gpart = nullptr;
    const float *hist = nullptr;
};

struct AdjLoop {
    StepArgs a;
    SampleTables smp;
    AdjOut o;
    int k = 0;
    int s_hi = 0;
    int next_row = 0;  // highest sample row not sampled yet
    int blk = 0;   // index of the current time block
    bool finished = false;
};

tpx_status adj_begin(Ctx &C, AdjLoop &b, const float *amp, const AdjOut &o) {
    const Layout &L = C.P.L;
    const int nt = C.P.nt;
    const int ns = C.plan.nslots;
    b.o = o;
    b.k = nt - 1;
    b.s_hi = nt - 1;
    b.next_row = nt - 1;
    b.blk = 0;
    b.finished = false;
    // lambda^{nt} = lambda^{nt-1} = 0; every other slot is written before it is read
    TPX_HIP(fill_zero_p(slot_ptr(C.ring, L, ns, nt), (size_t)L.slot_floats * 4, C.stream));
    TPX_HIP(fill_zero_p(slot_ptr(C.ring, L, ns, nt - 1), (size_t)L.slot_floats * 4, C.stream));
    if (o.gpart) TPX_HIP(fill_zero_p(o.gpart, align_up((size_t)L.S * L.nphys * 4), C.stream));
    if (o.vbar) TPX_HIP(fill_zero_p(o.vbar, align_up((size_t)L.S * o.r * L.nphys * 4), C.stream));
    StepArgs &a = b.a;
    memset(&a, 0, sizeof a);
    a.beta = C.beta;
    a.inject = C.P.nrec > 0 ? 1 : 0;
    a.inj = C.rec_inj;
    a.amp.ptr = amp;
    a.amp.shot_stride = (int64_t)nt * C.P.nrec;
    a.amp.k_stride = C.P.nrec;
    a.amp.scale = (float)(1.0 / (C.P.dt * C.P.dt));
    b.smp = C.src_smp;
    b.smp.out = o.q_adj;
    b.smp.out_shot_stride = nt;
    b.smp.out_k_stride = 1;
    b.smp.scale = (float)(C.P.dt * C.P.dt);
    a.smp = b.smp;
    return TPX_OK;
}

tpx_status adj_advance(Ctx &C, AdjLoop &b, int64_t max_steps, int64_t *used) {
    const Layout &L = C.P.L;
    const int nt = C.P.nt;
    const int ns = C.plan.nslots;
    const AdjOut &o = b.o;
    StepArgs &a = b.a;
    const bool accum = o.Z || o.hist;
    int64_t n = 0;
    while (b.k >= 1 && n < max_steps) {
        const int k = b.k;
        const bool ovl = accum && C.plan.overlap;
        // steps in this launch: down to k = 1, within the caller's budget and
        // (with contractions) the current block
        int64_t left = std::min<int64_t>(k, max_steps - n);
        if (accum) left = std::min<int64_t>(left, C.plan.block - (b.s_hi - k));
        const int nstep = steps_for_launch(max_steps_per_launch(C, ns), left);
        if (ovl && k == b.s_hi) {
            tpx_status st = overlap_guard(C, b.blk);
            if (st != TPX_OK) return st;
        }
        a.nstep = nstep;
        a.k = k;
        a.k2 = k - 1;
        a.k3 = k - 2;
        a.kp = k + 1;
        a.kp2 = k + 2;
        a.cur = slot_ptr(C.ring, L, ns, k);
        a.prev = slot_ptr(C.ring, L, ns, k + 1);
        a.prev2 = slot_ptr(C.ring, L, ns, k + 2);
        a.next = slot_ptr(C.ring, L, ns, k - 1);
        a.next2 = nstep >= 2 ? slot_ptr(C.ring, L, ns, k - 2) : nullptr;
        a.next3 = nstep == 3 ? slot_ptr(C.ring, L, ns, k - 3) : nullptr;
        a.inj = nstep == 3 ? C.rec_inj3 : C.rec_inj;
        // sample every level read here that is not sampled yet (rows nt-1 .. 0)
        const bool smp = o.q_adj != nullptr;
        a.do_sample = smp && b.next_row >= k;
        a.sample_prev = smp && k + 1 <= nt - 1 && b.next_row >= k + 1;
        a.sample_prev2 = smp && k + 2 <= nt - 1 && b.next_row >= k + 2;
        if (smp) b.next_row = k - 1;
        const int skind = nstep == 3 ? TPX_KERNEL_STEP3 : nstep == 2 ? TPX_KERNEL_STEP2 : TPX_KERNEL_STEP;
        const Layout &LL = nstep == 3 ? C.P.L3 : L;
        TPX_HIP(prof(skind, C.stream, [&] { return launch_step(LL, C.P.ph, a, C.stream); }));
        b.k -= nstep;
        n += nstep;
        const int k_last = k - nstep + 1;  // last step taken: lambda^{k_last - 1} is known, w^{k_last} can be formed
        if (accum && (b.s_hi - k_last + 1 == C.plan.block || k_last == 1)) {
            const int s_hi = b.s_hi;
            hipStream_t cs = ovl ? C.aux : C.stream;
            // dtt 0: w^s for s = k_last..s_hi; dtt 1: lam^k itself for k in the same
            // range, lam^0 joining the last block and lam^{nt-1} = 0 left out
            const int lo = o.dtt && k_last == 1 ? 0 : k_last;
            const int hi = o.dtt ? std::min(s_hi, nt - 2) : s_hi;
            auto contract = [&] {
                if (o.hist) return launch_accum_full(L, o.hist, C.ring, ns, k_last, s_hi, o.gpart, cs);
                const int sd = o.dtt ? 0 : 1;
                if (o.fold && C.fold_mfma)
                    return launch_fold_mfma(L, C.ring, ns, lo, hi, o.Z, C.zparts, nt, o.r, sd, o.ubar, o.c, o.gpart,
                                            cs);
                if (!o.fold && C.zpk)
                    return launch_accum_mfma(L, C.ring, ns, lo, hi, C.zpk, C.zparts, nt, o.r, sd, o.vbar, cs);
                return launch_accum_adj(L, C.ring, ns, lo, hi, o.Z, nt, o.r, o.fold, sd, o.ubar, o.c, o.vbar,
                                        o.gpart, cs);
            };
            const int kind = o.hist ? TPX_KERNEL_ACCUM_FULL : TPX_KERNEL_ACCUM_ADJ;
            if (ovl) {
                tpx_status st = overlap_launch(C, b.blk, kind, contract);
                if (st != TPX_OK) return st;
            } else {
                TPX_HIP(prof(kind, C.stream, contract));
            }
            b.s_hi = k_last - 1;
            ++b.blk;
        }
    }
    if (b.k < 1 && !b.finished) {
        for (; o.q_adj && b.next_row >= 0; --b.next_row) {
            const int row = b.next_row;
            TPX_HIP(prof(KIND_OTHER, C.stream, [&] { return launch_sample_only(L, slot_ptr(C.ring, L, ns, row), row, b.smp, C.stream); }));
        }
        if (accum && C.plan.overlap) {
            tpx_status st = overlap_join(C, b.blk);
            if (st != TPX_OK) return st;
        }
        b.finished = true;
    }
    if (used) *used = n;
    return TPX_OK;
}

tpx_status run_adjoint(Ctx &C, const float *amp, const AdjOut &o) {
    AdjLoop b;
    tpx_status st = adj_begin(C, b, amp, o);
    if (st != TPX_OK) return st;
    return adj_advance(C, b, INT64_MAX, nullptr);
}

// Probes of the call on the device: the caller's (EXPLICIT), generated from
// the counter hash, or (RANGE_FINDER) the QR factor of D_obs D_obs^T Z.
const float *probe_matrix_dev(Ctx &C, const tpx_probe *pr, const float *d_obs, tpx_status *st) {
    *st = TPX_OK;
    hipError_t e = hipSuccess;
    const float *Zc = pr->Z;
    if (pr->kind != TPX_PROBE_EXPLICIT) {
        float *Z = (float *)(C.ws + C.plan.Z);
        const bool rf = pr->kind == TPX_PROBE_RANGE_FINDER;
        if (rf && !d_obs) {
            *st = fail(TPX_E_INVAL, "range-finder probes need the observed data");
            return nullptr;
        }
        const int kind = rf ? TPX_PROBE_RADEMACHER : pr->kind;
        e = prof(KIND_OTHER, C.stream, [&] { return launch_probe_gen(kind, pr->r, pr->seed, C.P.nt, 0, C.P.L.S, Z, C.stream); });
        if (e == hipSuccess && rf)
            e = prof(KIND_OTHER, C.stream, [&] {
                return launch_range_finder(C.P.L.S, C.P.nt, C.P.nrec, pr->r, d_obs, Z, (double *)(C.ws + C.plan.rfW),
                                           (double *)(C.ws + C.plan.rfY), (double *)(C.ws + C.plan.rfX), C.stream);
            });
        Zc = Z;
    }
    const int mm = mfma_selected(C.P.L, pr);
    C.zparts = mfma_eligible(pr) ? probe_parts(pr) : 1;
    if (e == hipSuccess && (mm & MFMA_ACCUM)) {
        void *zpk = C.ws + C.plan.zpk;
        e = prof(KIND_OTHER, C.stream, [&] { return launch_pack_probes(C.P.L.S, C.P.nt, pr->r, C.zparts, Zc, zpk, C.stream); });
        C.zpk = zpk;
    }
    C.fold_mfma = (mm & MFMA_FOLD) != 0;
    if (e != hipSuccess) *st = fail(TPX_E_DEVICE, std::string("probe generation: ") + hipGetErrorString(e));
    return Zc;
}

// Imaging of the probed fields: pointwise (Eq. 4) or through the gradient (Eq. 5).
hipError_t image_probed(const Ctx &C, const tpx_probe &pr, float c, const float *ubar, const float *vbar, float *g) {
    if (pr.imaging == 1) return launch_image_graddot(C.P.L, C.P.h, pr.r, c, ubar, vbar, g, C.stream);
    return launch_image_probed(C.P.L, pr.r, c, ubar, vbar, g, C.stream);
}

float probe_scale(const tpx_probe *pr) {
    if (pr->kind == TPX_PROBE_IDENTITY || pr->kind == TPX_PROBE_RANGE_FINDER) return 1.0f;
    if (pr->kind == TPX_PROBE_EXPLICIT) return (float)pr->scale;
    return (float)(1.0 / pr->r);
}

Mode mode_of(int32_t call, bool *ok) {
    *ok = true;
    switch (call) {
    case TPX_CALL_FORWARD: return M_FORWARD;
    case TPX_CALL_ADJOINT: return M_ADJOINT;
    case TPX_CALL_GRADIENT_PROBED: return M_GRAD_PROBED;
    case TPX_CALL_GRADIENT_FULL: return M_GRAD_FULL;
    case TPX_CALL_FORWARD_PROBED: return M_FWD_PROBED;
    case TPX_CALL_BACKWARD_PROBED: return M_BWD_PROBED;
    case TPX_CALL_RANGE_FINDER: return M_RANGE_FINDER;
    case TPX_CALL_OBJECTIVE: return M_OBJECTIVE;
    default: *ok = false; return M_FORWARD;
    }
}

// A probed-gradient job that can be advanced a bounded number of time steps
// at a time (forward with probing, residual/objective, adjoint with probing,
// imaging).  tpx_gradient_probed runs one to the end; a server interleaves
// several.
struct GradJob {
    Ctx C;
    tpx_probe probe;
    const float *wavelet = nullptr;
    const float *d_obs = nullptr;
    float *g = nullptr;
    double *J = nullptr;
    float *d = nullptr;
    float *res = nullptr;
    const float *Z = nullptr;
    float *ubar = nullptr;
    FwdLoop f;
    AdjLoop b;
    int phase = 0;  // 0 forward, 1 adjoint, 2 done
    int64_t done_steps = 0, total_steps = 0;
};

tpx_status job_init(GradJob &J, const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe, const float *m,
                    const float *d_obs, float *g, double *Jout, float *d_out, void *ws, size_t ws_bytes,
                    void *stream, bool no_alloc = false) {
    if ((!d_obs && geom && geom->nrec > 0) || !g || !Jout)
        return fail(TPX_E_INVAL, "d_obs, g and J must not be NULL");
    J.C.no_alloc = no_alloc;
    tpx_status st = setup(J.C, grid, geom, probe, M_GRAD_PROBED, m, ws, ws_bytes, stream);
    if (st != TPX_OK) return st;
    J.probe = *probe;
    J.wavelet = geom->wavelet;
    J.d_obs = d_obs;
    J.g = g;
    J.J = Jout;
    J.d = d_out ? d_out : (float *)(J.C.ws + J.C.plan.d);
    J.res = (float *)(J.C.ws + J.C.plan.res);
    J.ubar = (float *)(J.C.ws + J.C.plan.ubar);
    J.Z = probe_matrix_dev(J.C, probe, d_obs, &st);
    if (st != TPX_OK) return st;
    st = fwd_begin(J.C, J.f, J.wavelet, J.d, nullptr, J.Z, probe->r, J.ubar, probe->dtt_side);
    if (st != TPX_OK) return st;
    J.phase = 0;
    J.done_steps = 0;
    J.total_steps = 2 * (int64_t)(J.C.P.nt - 1);
    return TPX_OK;
}

tpx_status job_advance(GradJob &J, int64_t max_steps) {
    int64_t budget = max_steps;
    tpx_status st;
    if (J.phase == 0) {
        int64_t used = 0;
        if ((st = fwd_advance(J.C, J.f, budget, &used)) != TPX_OK) return st;
        budget -= used;
        J.done_steps += used;
        if (J.f.finished) {
            const Layout &L = J.C.P.L;
            const int64_t ntr = (int64_t)L.S * J.C.P.nt * J.C.P.nrec;
            TPX_HIP(prof(KIND_OTHER, J.C.stream, [&] {
                return launch_residual(J.d, J.d_obs, J.res, ntr, (double *)(J.C.ws + J.C.plan.parts),
                                       residual_parts(ntr), J.J, J.C.stream);
            }));
            AdjOut o;
            o.Z = J.Z;
            o.r = J.probe.r;
            o.fold = J.probe.keep_vbar ? 0 : 1;
            o.dtt = J.probe.dtt_side;
            o.ubar = J.ubar;
            o.c = probe_scale(&J.probe);
            o.vbar = J.probe.keep_vbar ? (float *)(J.C.ws + J.C.plan.vbar) : nullptr;
            o.gpart = J.probe.keep_vbar ? nullptr : (float *)(J.C.ws + J.C.plan.gpart);
            if ((st = adj_begin(J.C, J.b, J.res, o)) != TPX_OK) return st;
            J.phase = 1;
        }
    }
    if (J.phase == 1 && budget > 0) {
        int64_t used = 0;
        if ((st = adj_advance(J.C, J.b, budget, &used)) != TPX_OK) return st;
        J.done_steps += used;
        if (J.b.finished) {
            const Layout &L = J.C.P.L;
            TPX_HIP(prof(KIND_OTHER, J.C.stream, [&] {
                return J.probe.keep_vbar ? image_probed(J.C, J.probe, J.b.o.c, J.ubar, J.b.o.vbar, J.g)
                                         : launch_image_sum(L, J.b.o.gpart, J.g, J.C.stream);
            }));
            J.phase = 2;
        }
    }
    return TPX_OK;
}

template <class F>
tpx_status guarded(F &&f) {
    try {
        return f();
    } catch (const std::exception &e) {
        return fail(TPX_E_INVAL, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(TPX_E_INVAL, "internal error");
    }
}

}  // namespace

namespace {

// ubar occupies the start of a state buffer; the header follows it.
size_t state_ubar_bytes(const Problem &P, const tpx_probe *pr) { return align_up((size_t)P.L.S * pr->r * P.L.nphys * 4); }
size_t state_total_bytes(const Problem &P, const tpx_probe *pr) {
    return state_ubar_bytes(P, pr) + align_up(sizeof(StateHeader));
}

StateHeader state_header(const Problem &P, const tpx_probe *pr) {
    StateHeader h;
    memset(&h, 0, sizeof h);
    h.w[0] = 0x31585054;   // "TPX1"
    h.w[1] = (int32_t)pr->kind;
    h.w[2] = pr->r;
    h.w[3] = (int32_t)(pr->seed & 0xffffffffu);
    h.w[4] = (int32_t)(pr->seed >> 32);
    h.w[5] = pr->dtt_side;
    h.w[6] = P.nt;
    h.w[7] = P.L.S;
    h.w[8] = (int32_t)P.L.n[0];
    h.w[9] = (int32_t)P.L.n[1];
    h.w[10] = (int32_t)P.L.n[2];
    h.w[11] = P.L.R;
    h.w[12] = P.L.nb;
    const uint64_t z = (uint64_t)(uintptr_t)pr->Z;   // explicit probes: the same matrix
    h.w[13] = (int32_t)(z & 0xffffffffu);
    h.w[14] = (int32_t)(z >> 32);
    h.w[15] = (int32_t)(pr->scale * 1e6);
    return h;
}

}  // namespace

namespace tpx {

void set_error(tpx_status st, const char *msg) { (void)fail(st, msg); }

tpx_status gradient_probed_in_scratch(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                                      const float *m, const float *d_obs, float *g, double *J, float *d_out,
                                      void *scratch, size_t scratch_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        // the size check first, with a message that names the limit
        Problem P;
        tpx_status st = make_problem(grid, geom, &P);
        if (st != TPX_OK) return st;
        if ((st = check_probe(P, probe)) != TPX_OK) return st;
        Tables T;
        if ((st = build_tables(P, grid, geom, &T)) != TPX_OK) return st;
        const size_t need = make_plan(P, M_GRAD_PROBED, probe, T.blob.size, false).total;
        if (need > scratch_bytes) {
            char buf[200];
            snprintf(buf, sizeof buf,
                     "the problem needs %zu bytes of scratch; the allocation-free entry point holds %zu bytes per GPU",
                     need, scratch_bytes);
            return fail(TPX_E_NOMEM, buf);
        }
        GradJob job;
        st = job_init(job, grid, geom, probe, m, d_obs, g, J, d_out, scratch, scratch_bytes, stream, true);
        if (st != TPX_OK) return st;
        return job_advance(job, INT64_MAX);
    });
}

}  // namespace tpx

extern "C" {

const char *tpx_last_error(void) { return g_err.c_str(); }
const char *tpx_version(void) { return "tpx 0.1 gfx950"; }

size_t tpx_workspace_bytes(int32_t call, const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe) {
    size_t out = 0;
    guarded([&]() -> tpx_status {
        bool ok;
        const Mode mode = mode_of(call, &ok);
        if (!ok) return fail(TPX_E_INVAL, "unknown call id");
        Problem P;
        tpx_status st = make_problem(grid, geom, &P);
        if (st != TPX_OK) return st;
        const bool probed = mode == M_GRAD_PROBED || mode == M_FWD_PROBED || mode == M_BWD_PROBED;
        if ((probed || mode == M_RANGE_FINDER) && (st = check_probe(P, probe)) != TPX_OK) return st;
        if (mode == M_RANGE_FINDER && probe->kind != TPX_PROBE_RANGE_FINDER)
            return fail(TPX_E_INVAL, "TPX_CALL_RANGE_FINDER needs a range-finder probe");
        if ((mode == M_FWD_PROBED || mode == M_BWD_PROBED) && probe->kind == TPX_PROBE_RANGE_FINDER)
            return fail(TPX_E_INVAL, "range-finder probes need d_obs: pass tpx_range_finder_probes' Q as EXPLICIT");
        Tables T;
        if ((st = build_tables(P, grid, geom, &T)) != TPX_OK) return st;
        out = make_plan(P, mode, probe, T.blob.size).total;
        return TPX_OK;
    });
    return out;
}

size_t tpx_state_bytes(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe) {
    size_t out = 0;
    guarded([&]() -> tpx_status {
        Problem P;
        tpx_status st = make_problem(grid, geom, &P);
        if (st != TPX_OK) return st;
        if ((st = check_probe(P, probe)) != TPX_OK) return st;
        out = state_total_bytes(P, probe);
        return TPX_OK;
    });
    return out;
}

tpx_status tpx_forward(const tpx_grid *grid, const tpx_geom *geom, const float *m, float *d, void *ws,
                       size_t ws_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        if (!d && geom && geom->nrec > 0) return fail(TPX_E_INVAL, "d must not be NULL");
        Ctx C;
        tpx_status st = setup(C, grid, geom, nullptr, M_FORWARD, m, ws, ws_bytes, stream);
        if (st != TPX_OK) return st;
        return run_forward(C, geom->wavelet, d, nullptr, nullptr, 0, nullptr);
    });
}

tpx_status tpx_objective(const tpx_grid *grid, const tpx_geom *geom, const float *m, const float *d_obs, double *J,
                         float *d_out, void *ws, size_t ws_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        if ((!d_obs && geom && geom->nrec > 0) || !J) return fail(TPX_E_INVAL, "d_obs and J must not be NULL");
        Ctx C;
        tpx_status st = setup(C, grid, geom, nullptr, M_OBJECTIVE, m, ws, ws_bytes, stream);
        if (st != TPX_OK) return st;
        float *d = d_out ? d_out : (float *)(C.ws + C.plan.d);
        st = run_forward(C, geom->wavelet, d, nullptr, nullptr, 0, nullptr);
        if (st != TPX_OK) return st;
        const int64_t ntr = (int64_t)C.P.L.S * C.P.nt * C.P.nrec;
        TPX_HIP(prof(KIND_OTHER, C.stream, [&] {
            return launch_residual(d, d_obs, (float *)(C.ws + C.plan.res), ntr, (double *)(C.ws + C.plan.parts),
                                   residual_parts(ntr), J, C.stream);
        }));
        return TPX_OK;
    });
}

tpx_status tpx_adjoint(const tpx_grid *grid, const tpx_geom *geom, const float *m, const float *d_in, float *q_adj,
                       void *ws, size_t ws_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        if ((!d_in && geom && geom->nrec > 0) || !q_adj) return fail(TPX_E_INVAL, "d_in and q_adj must not be NULL");
        Ctx C;
        tpx_status st = setup(C, grid, geom, nullptr, M_ADJOINT, m, ws, ws_bytes, stream);
        if (st != TPX_OK) return st;
        AdjOut o;
        o.q_adj = q_adj;
        return run_adjoint(C, d_in, o);
    });
}

tpx_status tpx_gradient_probed(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe, const float *m,
                               const float *d_obs, float *g, double *J, float *d_out, void *ws, size_t ws_bytes,
                               void *stream) {
    return guarded([&]() -> tpx_status {
        GradJob job;
        tpx_status st = job_init(job, grid, geom, probe, m, d_obs, g, J, d_out, ws, ws_bytes, stream);
        if (st != TPX_OK) return st;
        return job_advance(job, INT64_MAX);
    });
}

struct tpx_job {
    GradJob j;
};

tpx_status tpx_job_create(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe, const float *m,
                          const float *d_obs, float *g, double *J, float *d_out, void *ws, size_t ws_bytes,
                          void *stream, tpx_job **job) {
    return guarded([&]() -> tpx_status {
        if (!job) return fail(TPX_E_INVAL, "job must not be NULL");
        *job = nullptr;
        tpx_job *p = new tpx_job();
        tpx_status st = job_init(p->j, grid, geom, probe, m, d_obs, g, J, d_out, ws, ws_bytes, stream);
        if (st != TPX_OK) {
            delete p;
            return st;
        }
        *job = p;
        return TPX_OK;
    });
}

tpx_status tpx_job_advance(tpx_job *job, int32_t max_steps, void *stream, int32_t *finished) {
    return guarded([&]() -> tpx_status {
        if (!job || max_steps < 1) return fail(TPX_E_INVAL, "job must not be NULL and max_steps >= 1");
        job->j.C.stream = (hipStream_t)stream;
        tpx_status st = job_advance(job->j, max_steps);
        if (finished) *finished = job->j.phase == 2 ? 1 : 0;
        return st;
    });
}

tpx_status tpx_job_progress(const tpx_job *job, int64_t *steps_done, int64_t *steps_total) {
    if (!job || !steps_done || !steps_total) return fail(TPX_E_INVAL, "NULL argument");
    *steps_done = job->j.done_steps;
    *steps_total = job->j.total_steps;
    return TPX_OK;
}

void tpx_job_destroy(tpx_job *job) { delete job; }

tpx_status tpx_gradient_full(const tpx_grid *grid, const tpx_geom *geom, const float *m, const float *d_obs, float *g,
                             double *J, float *d_out, void *ws, size_t ws_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        if ((!d_obs && geom && geom->nrec > 0) || !g || !J) return fail(TPX_E_INVAL, "d_obs, g and J must not be NULL");
        Ctx C;
        tpx_status st = setup(C, grid, geom, nullptr, M_GRAD_FULL, m, ws, ws_bytes, stream);
        if (st != TPX_OK) return st;
        const Layout &L = C.P.L;
        float *hist = (float *)(C.ws + C.plan.hist);
        float *d = d_out ? d_out : (float *)(C.ws + C.plan.d);
        float *res = (float *)(C.ws + C.plan.res);
        st = run_forward(C, geom->wavelet, d, hist, nullptr, 0, nullptr);
        if (st != TPX_OK) return st;
        const int64_t ntr = (int64_t)L.S * C.P.nt * C.P.nrec;
        TPX_HIP(prof(KIND_OTHER, C.stream, [&] {
            return launch_residual(d, d_obs, res, ntr, (double *)(C.ws + C.plan.parts), residual_parts(ntr), J,
                                   C.stream);
        }));
        AdjOut o;
        o.hist = hist;
        o.gpart = (float *)(C.ws + C.plan.gpart);
        st = run_adjoint(C, res, o);
        if (st != TPX_OK) return st;
        TPX_HIP(prof(KIND_OTHER, C.stream, [&] { return launch_image_sum(L, o.gpart, g, C.stream); }));
        return TPX_OK;
    });
}

tpx_status tpx_forward_probed(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe, const float *m,
                              float *d, void *state, size_t state_bytes, void *ws, size_t ws_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        if ((!d && geom && geom->nrec > 0) || !state) return fail(TPX_E_INVAL, "d and state must not be NULL");
        Ctx C;
        tpx_status st = setup(C, grid, geom, probe, M_FWD_PROBED, m, ws, ws_bytes, stream);
        if (st != TPX_OK) return st;
        if (state_bytes < state_total_bytes(C.P, probe))
            return fail(TPX_E_STATE, "state buffer smaller than tpx_state_bytes()");
        const float *Z = probe_matrix_dev(C, probe, nullptr, &st);
        if (st != TPX_OK) return st;
        st = run_forward(C, geom->wavelet, d, nullptr, Z, probe->r, (float *)state, probe->dtt_side);
        if (st != TPX_OK) return st;
        TPX_HIP(prof(KIND_OTHER, C.stream, [&] {
            return launch_state_header(state_header(C.P, probe), (unsigned char *)state + state_ubar_bytes(C.P, probe),
                                       (int32_t *)(C.ws + C.plan.flags), 0, C.stream);
        }));
        return TPX_OK;
    });
}

tpx_status tpx_backward_probed(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe, const float *m,
                               const float *grad_d, const void *state, size_t state_bytes, float *g, void *ws,
                               size_t ws_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        if ((!grad_d && geom && geom->nrec > 0) || !state || !g) return fail(TPX_E_INVAL, "grad_d, state and g must not be NULL");
        Ctx C;
        tpx_status st = setup(C, grid, geom, probe, M_BWD_PROBED, m, ws, ws_bytes, stream);
        if (st != TPX_OK) return st;
        const Layout &L = C.P.L;
        if (state_bytes < state_total_bytes(C.P, probe))
            return fail(TPX_E_STATE, "state buffer smaller than tpx_state_bytes()");
        // the state must come from a forward pass of this problem and probe set
        TPX_HIP(prof(KIND_OTHER, C.stream, [&] {
            return launch_state_header(state_header(C.P, probe),
                                       (unsigned char *)const_cast<void *>(state) + state_ubar_bytes(C.P, probe),
                                       (int32_t *)(C.ws + C.plan.flags), 1, C.stream);
        }));
        const float *Z = probe_matrix_dev(C, probe, nullptr, &st);
        if (st != TPX_OK) return st;
        AdjOut o;
        o.Z = Z;
        o.r = probe->r;
        o.fold = probe->keep_vbar ? 0 : 1;
        o.dtt = probe->dtt_side;
        o.ubar = (const float *)state;
        o.c = probe_scale(probe);
        o.vbar = probe->keep_vbar ? (float *)(C.ws + C.plan.vbar) : nullptr;
        o.gpart = probe->keep_vbar ? nullptr : (float *)(C.ws + C.plan.gpart);
        st = run_adjoint(C, grad_d, o);
        if (st != TPX_OK) return st;
        TPX_HIP(prof(KIND_OTHER, C.stream, [&] {
            return probe->keep_vbar ? image_probed(C, *probe, o.c, o.ubar, o.vbar, g)
                                    : launch_image_sum(L, o.gpart, g, C.stream);
        }));
        return TPX_OK;
    });
}

void tpx_profile_enable(int32_t on) {
    Profiler &p = profiler();
    std::lock_guard<std::mutex> lk(p.mu);
    close_run(p);
    if (on) {
        p.recs.clear();
        p.used = 0;
    }
    p.on = on != 0;
}

tpx_status tpx_profile_read(int32_t kind, double *total_ms, int64_t *launches) {
    return guarded([&]() -> tpx_status {
        if (!total_ms || !launches) return fail(TPX_E_INVAL, "total_ms and launches must not be NULL");
        Profiler &p = profiler();
        std::lock_guard<std::mutex> lk(p.mu);
        close_run(p);
        double tot = 0.0;
        int64_t n = 0;
        for (const ProfRec &r : p.recs) {
            if (r.kind != kind) continue;
            TPX_HIP(hipEventSynchronize(r.b));
            float ms = 0.0f;
            TPX_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            tot += ms;
            n += r.launches;
        }
        *total_ms = tot;
        *launches = n;
        return TPX_OK;
    });
}

tpx_status tpx_set_option(int32_t option, int64_t value) {
    if (option == TPX_OPT_OVERLAP_CONTRACTIONS) {
        g_overlap.store(value ? 1 : 0);
        return TPX_OK;
    }
    if (option == TPX_OPT_STEPS_2D) {
        if (value != 2 && value != 3) return fail(TPX_E_INVAL, "TPX_OPT_STEPS_2D takes 2 or 3");
        g_steps2d.store((int)value);
        return TPX_OK;
    }
    if (option == TPX_OPT_FUSED_STEPS_3D) {
        g_fused3d.store(value ? 1 : 0);
        return TPX_OK;
    }
    if (option == TPX_OPT_MATRIX_CORES) {
        if (value < 0 || value > 2) return fail(TPX_E_INVAL, "TPX_OPT_MATRIX_CORES takes 0, 1 or 2");
        g_mfma.store((int)value);
        return TPX_OK;
    }
    return fail(TPX_E_INVAL, "unknown option");
}

int64_t tpx_get_option(int32_t option) {
    if (option == TPX_OPT_OVERLAP_CONTRACTIONS) return g_overlap.load();
    if (option == TPX_OPT_MATRIX_CORES) return g_mfma.load();
    if (option == TPX_OPT_FUSED_STEPS_3D) return g_fused3d.load();
    if (option == TPX_OPT_STEPS_2D) return g_steps2d.load();
    return -1;
}

tpx_status tpx_check_workspace(const void *ws, void *stream) {
    return guarded([&]() -> tpx_status {
        if (!ws) return fail(TPX_E_INVAL, "ws must not be NULL");
        int32_t flags = 0;
        TPX_HIP(hipStreamSynchronize((hipStream_t)stream));
        TPX_HIP(hipMemcpy(&flags, ws, sizeof flags, hipMemcpyDeviceToHost));
        if (flags & 1) return fail(TPX_E_NUMERIC, "the model holds a non-finite or non-positive value");
        if (flags & 2) return fail(TPX_E_CFL, "the model holds velocities above damp_vmax (dt may be unstable)");
        if (flags & 4)
            return fail(TPX_E_STATE, "the state was written by a forward pass of another problem or probe set");
        return TPX_OK;
    });
}

tpx_status tpx_range_finder_probes(const tpx_grid *grid, const tpx_geom *geom, const tpx_probe *probe,
                                   const float *d_obs, float *Q, void *ws, size_t ws_bytes, void *stream) {
    return guarded([&]() -> tpx_status {
        if (!d_obs || !Q) return fail(TPX_E_INVAL, "d_obs and Q must not be NULL");
        Problem P;
        tpx_status st = make_problem(grid, geom, &P);
        if (st != TPX_OK) return st;
        if ((st = check_probe(P, probe)) != TPX_OK) return st;
        if (probe->kind != TPX_PROBE_RANGE_FINDER) return fail(TPX_E_INVAL, "probe kind must be RANGE_FINDER");
        const Plan plan = make_plan(P, M_RANGE_FINDER, probe, 0);
        if (!ws || ws_bytes < plan.total) return fail(TPX_E_NOMEM, "workspace smaller than required");
        unsigned char *w = (unsigned char *)ws;
        const hipStream_t s = (hipStream_t)stream;
        TPX_HIP(launch_probe_gen(TPX_PROBE_RADEMACHER, probe->r, probe->seed, P.nt, 0, P.L.S, Q, s));
        TPX_HIP(launch_range_finder(P.L.S, P.nt, P.nrec, probe->r, d_obs, Q, (double *)(w + plan.rfW),
                                    (double *)(w + plan.rfY), (double *)(w + plan.rfX), s));
        return TPX_OK;
    });
}

tpx_status tpx_probe_matrix(const tpx_probe *probe, int32_t nt, int32_t shot, float *Z, void *stream) {
    return guarded([&]() -> tpx_status {
        if (!probe || !Z) return fail(TPX_E_INVAL, "probe and Z must not be NULL");
        if (nt < 1 || shot < 0 || probe->r < 1) return fail(TPX_E_INVAL, "nt >= 1, shot >= 0, r >= 1 required");
        if (probe->kind == TPX_PROBE_EXPLICIT || probe->kind < 0 || probe->kind > 3)
            return fail(TPX_E_INVAL, "tpx_probe_matrix generates Rademacher, Gauss-B64 or identity probes");
        if (probe->kind == TPX_PROBE_IDENTITY && probe->r != nt) return fail(TPX_E_INVAL, "identity needs r == nt");
        TPX_HIP(launch_probe_gen(probe->kind, probe->r, probe->seed, nt, shot, 1, Z, (hipStream_t)stream));
        return TPX_OK;
    });
}

}  // extern "C"
