// runtime.hip -- host runtime of libtgf.so: the C ABI declared in tgf.h.
//
// Responsibilities: argument validation (before anything is enqueued),
// carving the caller's workspace into per-configuration buffers, the flow
// schedule (full steps of eps, one shortened last step, measurement rows),
// ordering a batch so that the configurations still flowing at any step form
// a prefix of the tile table (one launch per RK stage for the whole batch),
// capturing the launch sequence of a flow into a HIP graph that is reused
// while the sequence is unchanged, kernel timing with HIP events, and the
// stage-variant autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/tgf.h"
#include "launch.h"
#include "layout.h"

using namespace tgf;

namespace {

thread_local std::string g_err;

tgf_status fail(tgf_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(TGF_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct CfgHost {
    int d[4];
    int tw[6];
    int V;
    int stride;
    int tiles;
    int blk;                 // sites per LDS-staged work-group (default_block, or tuned)
    size_t offW[2], offX;
    int cur = 0;
    double t = 0;
    long long steps = 0;     // RK steps since the links were loaded (reunitarisation schedule)
    bool loaded = false;
};

struct Layout {
    size_t off_desc, off_tiles, off_blocks, off_flag, off_check, off_src, off_partials, off_rows,
        off_meas, off_cfg0;
    size_t total;
    int total_tiles;
    std::vector<CfgHost> cfg;
};

int ne_of(tgf_storage st) { return st == TGF_F32_C12 ? 6 : 9; }

// A storage argument from a C caller may hold any int; it is read as its raw
// value (not as the C++ enum, whose out-of-range values are undefined) and
// only then trusted as a tgf_storage.
bool storage_ok(const tgf_storage &st) {
    int v;
    memcpy(&v, &st, sizeof v);
    return v >= (int)TGF_F64_FULL && v <= (int)TGF_F32_C12;
}

// Sites per work-group of the LDS-staged stage variants: whole (n0, n1) planes
// (so that every neighbour in directions 0 and 1 lies in the block) when at
// least two of them fill half of the 256 threads; otherwise 256.  For the
// L x L x 3L x 3L boxes: L = 6 -> 252, 8 -> 256, 10 -> 200, 12 -> 144.
int default_block(const int d[4]) {
    const int plane = d[0] * d[1];
    if (plane > kBlock) return kBlock;
    const int k = kBlock / plane;
    return k * plane >= kBlock / 2 ? k * plane : kBlock;
}

// Column width of the LDS-staged launch order (block_order): site order while
// an n3 slice spans at most kChunkSlice work-groups (its direction-3
// neighbours are then among the work-groups an XCD runs at a time), else the
// largest divisor of the slice's work-group count up to kChunk.  Stage launch
// on the 32x32x96x96 box (384 work-groups per slice) against site order, for
// columns of 8 / 16 / 32 work-groups: FP32 12-real - / -6.3% / -6.8%,
// FP32 full -8.2% / -11.5% / -9.3%, FP64 -7.3% / -8.3% / +6.9% (the wider the
// column, the more of the XCD's L2 the direction-3 neighbours need; FP64
// holds 144 KB per work-group).
constexpr int kChunk = 16;
constexpr int kChunkSlice = 64;
int block_chunk(const int d[4], int blk) {
    const long long s = (long long)d[0] * d[1] * d[2];
    if (s % blk) return 0;
    const long long slice = s / blk;
    if (slice <= kChunkSlice) return 0;
    for (int ch = kChunk; ch >= 4; ch--)
        if (slice % ch == 0) return ch;
    return 0;
}

// The other candidate the autotuner times for a configuration (0 if none).
int other_block(const int d[4]) {
    const int b = default_block(d);
    return b == kBlock ? 0 : kBlock;
}
size_t cx_bytes(tgf_storage st) { return st == TGF_F64_FULL ? 16 : 8; }

// nc: colours; general: the SU(N) storage (N^2 entries per link)
tgf_status validate_geoms(int32_t n_cfg, const tgf_geom *g, int nc = 3, bool general = false) {
    if (n_cfg <= 0) return fail(TGF_E_INVAL, "n_cfg must be positive");
    if (!g) return fail(TGF_E_INVAL, "geoms is NULL");
    for (int c = 0; c < n_cfg; c++) {
        long long V = 1;
        for (int m = 0; m < 4; m++) {
            if (g[c].dims[m] < 2)
                return fail(TGF_E_INVAL, "config " + std::to_string(c) + ": dims must be >= 2");
            V *= g[c].dims[m];
        }
        // every per-lane byte offset into an entry plane (into the N^2 planes of
        // one direction for the SU(N) storage) must fit in 32 bits
        const long long cap = general ? (1LL << 28) / (nc * nc) - 256 : (1LL << 28) - 256;
        if (V > cap)
            return fail(TGF_E_INVAL, "config " + std::to_string(c) + ": lattice too large");
        for (int k = 0; k < 6; k++)
            if (g[c].twist[k] < 0 || g[c].twist[k] >= nc)
                return fail(TGF_E_INVAL, "config " + std::to_string(c) +
                                             ": twist entries must be in 0.." +
                                             std::to_string(nc - 1));
    }
    return TGF_OK;
}

Layout make_layout(int32_t n_cfg, const tgf_geom *g, tgf_storage st, int nc = 3,
                   bool general = false) {
    Layout L;
    L.cfg.resize(n_cfg);
    int tiles = 0;
    for (int c = 0; c < n_cfg; c++) {
        CfgHost &h = L.cfg[c];
        h.V = 1;
        for (int m = 0; m < 4; m++) { h.d[m] = g[c].dims[m]; h.V *= h.d[m]; }
        for (int k = 0; k < 6; k++) h.tw[k] = g[c].twist[k];
        h.stride = (int)align_up((size_t)h.V, 256);
        h.tiles = (h.V + 63) / 64;
        h.blk = default_block(h.d);
        tiles += h.tiles;
    }
    L.total_tiles = tiles;
    size_t o = 0;
    L.off_desc = o;     o = align_up(o + sizeof(CfgDesc) * n_cfg, 256);
    L.off_tiles = o;    o = align_up(o + sizeof(int) * (n_cfg + 1), 256);
    L.off_blocks = o;   o = align_up(o + sizeof(int) * (n_cfg + 1), 256);
    L.off_flag = o;     o = align_up(o + 64, 256);
    L.off_check = o;    o = align_up(o + 64, 256);
    L.off_src = o;      o = align_up(o + sizeof(void *) * n_cfg, 256);   // batched ingest inputs
    // measurement: 4 doubles per (tile, plane pair); unitarity check: 2 per tile
    size_t partial_doubles = (size_t)tiles * 3 * 4;
    L.off_partials = o; o = align_up(o + sizeof(double) * partial_doubles, 256);
    L.off_rows = o;     o = align_up(o + sizeof(double) * 6 * (size_t)kMaxRows * n_cfg, 256);
    L.off_meas = o;     o = align_up(o + sizeof(MeasSlot) * (size_t)(kMaxRows + 1) * n_cfg, 256);
    L.off_cfg0 = o;
    const size_t e = cx_bytes(st);
    const int NE = general ? nc * nc : ne_of(st);
    for (int c = 0; c < n_cfg; c++) {
        CfgHost &h = L.cfg[c];
        size_t wb = e * 4 * NE * (size_t)h.stride;
        // SU(N): X is a full N x N matrix per link
        size_t xb = e * 4 * (general ? NE : 4) * (size_t)h.stride;
        h.offW[0] = o; o = align_up(o + wb, 256);
        h.offW[1] = o; o = align_up(o + wb, 256);
        h.offX = o;    o = align_up(o + xb, 256);
    }
    L.total = o;
    return L;
}

struct Launch {
    int kind;      // 0 stage, 1 measure, 2 finalize, 3 zero flag
    int grid;      // tiles (stage/measure) or configs (finalize)
    int n_act;
    int step, stage;
    int reunit;    // stage launches: reunit_every (FP32 storages), else 0
    int event;     // measurement event index (slot table row)
    int blocks;    // stage launches: work-groups of the LDS-staged variants
    bool operator==(const Launch &o) const {
        return kind == o.kind && grid == o.grid && n_act == o.n_act && step == o.step &&
               stage == o.stage && reunit == o.reunit && event == o.event && blocks == o.blocks;
    }
};

}  // namespace

struct tgf_ctx {
    int n_cfg;
    tgf_storage st;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    Layout L;
    int variant = -1;
    int nc = 3;              // colours
    bool general = false;    // SU(N) kernels (tgf_create_sun), for any N including 3
    // host pinned staging
    char *h_stage = nullptr;
    size_t h_stage_bytes = 0;
    // cached graph of the last flow
    hipGraphExec_t gexec = nullptr;
    std::vector<Launch> glaunches;
    double geps = 0;
    int gvariant = -2;
    tgf_timing timing{};
    std::vector<hipEvent_t> events;

    CfgDesc *d_desc() { return (CfgDesc *)(ws + L.off_desc); }
    int *d_tiles() { return (int *)(ws + L.off_tiles); }
    int *d_blocks() { return (int *)(ws + L.off_blocks); }
    int *d_flag() { return (int *)(ws + L.off_flag); }
    double *d_check() { return (double *)(ws + L.off_check); }
    const void **d_src() { return (const void **)(ws + L.off_src); }
    double *d_partials() { return (double *)(ws + L.off_partials); }
    double *d_rows() { return (double *)(ws + L.off_rows); }
    MeasSlot *d_meas() { return (MeasSlot *)(ws + L.off_meas); }
    Prec prec() const { return st == TGF_F64_FULL ? P_F64 : P_F32; }
    bool c12() const { return st == TGF_F32_C12; }
    int ne() const { return general ? nc * nc : (st == TGF_F32_C12 ? 6 : 9); }
    int x_entries() const { return general ? nc * nc : 4; }
    int variant_count() const { return general ? sun_variant_count(nc) : V_COUNT; }
    int effective_variant() const {
        if (general) return variant >= 0 ? variant : 0;
        if (variant >= 0) return variant;
        return V_SITE_LDS_XCD;   // the fastest measured for all three storages
    }
};

namespace {

tgf_status ensure_stage(tgf_ctx *c, size_t bytes) {
    if (c->h_stage_bytes >= bytes) return TGF_OK;
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    c->h_stage = nullptr;
    c->h_stage_bytes = 0;
    size_t nb = std::max<size_t>(bytes, 1 << 16);
    HIP_TRY(hipHostMalloc((void **)&c->h_stage, nb, hipHostMallocDefault));
    c->h_stage_bytes = nb;
    return TGF_OK;
}

void fill_desc(const tgf_ctx *c, const CfgHost &h, int user, CfgDesc &d) {
    memset(&d, 0, sizeof d);
    for (int m = 0; m < 4; m++) d.d[m] = h.d[m];
    d.V = h.V;
    d.stride = h.stride;
    for (int k = 0; k < 6; k++) d.tw[k] = h.tw[k];
    d.user = user;
    d.cur = h.cur;
    d.t0 = h.t;
    d.blk = h.blk;
    d.chunk = block_chunk(h.d, h.blk);
    d.W[0] = c->ws + h.offW[0];
    d.W[1] = c->ws + h.offW[1];
    d.X = c->ws + h.offX;
}

bool on_grid(double t, double dt) {
    if (dt <= 0) return false;
    double k = std::floor(t / dt + 0.5);
    return std::fabs(t - k * dt) <= 1e-9;
}

// Step plan of one configuration (same rule as the paper-independent
// schedule stated in tgf.h): t_k = t0 + k*eps while t_k <= t_end + 1e-12,
// then one short step to t_end if more than 1e-12 remains.
struct Plan {
    int n_full;
    int n_steps;
    double eps_last;
    std::vector<std::pair<int, double>> meas;   // (steps done before the row, t)
};

Plan make_plan(double t0, double t_end, double eps, double dt) {
    Plan p;
    long n = 0;
    while (t0 + (n + 1) * eps <= t_end + 1e-12) n++;
    p.n_full = (int)n;
    double t_last = t0 + n * eps;
    bool has_short = (t_end - t_last) > 1e-12;
    p.eps_last = has_short ? t_end - t_last : 0.0;
    p.n_steps = p.n_full + (has_short ? 1 : 0);
    if (on_grid(t0, dt) || p.n_steps == 0) p.meas.push_back({0, t0});
    for (int k = 1; k <= p.n_full; k++) {
        double t = t0 + k * eps;
        bool last = (k == p.n_full) && !has_short;
        if (on_grid(t, dt) || last) p.meas.push_back({k, t});
    }
    if (has_short) p.meas.push_back({p.n_steps, t_end});
    return p;
}

tgf_status run_launches(tgf_ctx *c, const std::vector<Launch> &ls, double eps, bool graph,
                        bool timing) {
    const int variant = c->effective_variant();
    hipStream_t s = c->stream;
    auto issue = [&](const Launch &l) -> hipError_t {
        switch (l.kind) {
            case 0:
                if (c->general)
                    return launch_stage_sun(c->nc, variant, s, c->d_desc(), c->d_tiles(), l.n_act,
                                            l.grid, l.step, l.stage, eps);
                return launch_stage(variant, c->prec(), c->c12(), s, c->d_desc(), c->d_tiles(),
                                    l.n_act, l.grid, c->d_blocks(), l.blocks, l.step, l.stage,
                                    eps, l.reunit);
            case 1:
                if (c->general)
                    return launch_measure_sun(c->nc, variant, s, c->d_desc(), c->d_tiles(),
                                              l.n_act, l.grid,
                                              c->d_meas() + (size_t)l.event * c->n_cfg,
                                              c->d_partials(), l.step);
                return launch_measure(c->prec(), c->c12(), s, c->d_desc(), c->d_tiles(), l.n_act,
                                      l.grid, c->d_meas() + (size_t)l.event * c->n_cfg,
                                      c->d_partials(), l.step);
            case 2:
                return launch_finalize(s, c->d_desc(), c->d_tiles(), l.n_act,
                                       c->d_meas() + (size_t)l.event * c->n_cfg, c->d_partials(),
                                       c->d_rows(), c->n_cfg, c->d_flag(), c->nc);
            default:
                return launch_fill_int(s, c->d_flag(), 1, 0);
        }
    };
    if (timing) {
        size_t need = 2 * ls.size();
        while (c->events.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            c->events.push_back(e);
        }
        for (size_t k = 0; k < ls.size(); k++) {
            HIP_TRY(hipEventRecord(c->events[2 * k], s));
            HIP_TRY(issue(ls[k]));
            HIP_TRY(hipEventRecord(c->events[2 * k + 1], s));
        }
        return TGF_OK;
    }
    if (!graph) {
        for (const Launch &l : ls) HIP_TRY(issue(l));
        return TGF_OK;
    }
    bool reuse = c->gexec && c->glaunches == ls && c->geps == eps && c->gvariant == variant;
    if (!reuse) {
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t err = hipSuccess;
        for (const Launch &l : ls) {
            err = issue(l);
            if (err != hipSuccess) break;
        }
        hipError_t e2 = hipStreamEndCapture(s, &g);
        if (err != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(TGF_E_HIP, std::string("kernel launch during capture: ") +
                                       hipGetErrorString(err));
        }
        HIP_TRY(e2);
        hipError_t e3 = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIP_TRY(e3);
        c->glaunches = ls;
        c->geps = eps;
        c->gvariant = variant;
    }
    HIP_TRY(hipGraphLaunch(c->gexec, s));
    return TGF_OK;
}

tgf_status check_ctx(tgf_ctx *c) {
    if (!c) return fail(TGF_E_INVAL, "context is NULL");
    return TGF_OK;
}

tgf_status check_cfg(tgf_ctx *c, int32_t cfg) {
    if (cfg < 0 || cfg >= c->n_cfg)
        return fail(TGF_E_INVAL, "cfg index " + std::to_string(cfg) + " out of range");
    return TGF_OK;
}

// Unitarity defects of the stored links of config cfg.
tgf_status run_check(tgf_ctx *c, int cfg, const void *src, double out[2]) {
    const CfgHost &h = c->L.cfg[cfg];
    if (c->general)
        HIP_TRY(launch_check_sun(c->nc, false, c->stream, src, h.V, h.stride, c->d_partials(),
                                 c->d_check()));
    else
        HIP_TRY(launch_check(c->prec(), c->c12(), c->stream, src, h.V, h.stride, c->d_partials(),
                             c->d_check()));
    tgf_status st = ensure_stage(c, 64);
    if (st) return st;
    HIP_TRY(hipMemcpyAsync(c->h_stage, c->d_check(), 2 * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    memcpy(out, c->h_stage, 2 * sizeof(double));
    return TGF_OK;
}

// Upload descriptors + tile prefix of the given exec order.
// half_sites: the tiles cover the V/2 sites of one parity (Monte Carlo).
// reunit_every: the flow's reunitarisation period, for each configuration's
// phase (steps done since its load, modulo the period).
tgf_status upload_tables(tgf_ctx *c, const std::vector<int> &order, const std::vector<Plan> *plans,
                         std::vector<int> &tile_start, bool half_sites = false,
                         int reunit_every = 0, std::vector<int> *blk_start = nullptr) {
    const int n = (int)order.size();
    tile_start.assign(n + 1, 0);
    std::vector<int> bs(n + 1, 0);
    for (int k = 0; k < n; k++) {
        const CfgHost &h = c->L.cfg[order[k]];
        const int tiles = half_sites ? (h.V / 2 + 63) / 64 : h.tiles;
        tile_start[k + 1] = tile_start[k] + tiles;
        bs[k + 1] = bs[k] + (h.V + h.blk - 1) / h.blk;
    }
    if (blk_start) *blk_start = bs;
    size_t bytes = sizeof(CfgDesc) * n + 2 * sizeof(int) * (n + 1);
    tgf_status st = ensure_stage(c, bytes);
    if (st) return st;
    CfgDesc *dd = (CfgDesc *)c->h_stage;
    for (int k = 0; k < n; k++) {
        fill_desc(c, c->L.cfg[order[k]], order[k], dd[k]);
        if (reunit_every > 0)
            dd[k].reunit_phase = (int)(c->L.cfg[order[k]].steps % reunit_every);
        if (plans) {
            const Plan &p = (*plans)[order[k]];
            dd[k].n_full = p.n_full;
            dd[k].n_steps = p.n_steps;
            dd[k].eps_last = p.eps_last;
        }
    }
    int *ti = (int *)(c->h_stage + sizeof(CfgDesc) * n);
    memcpy(ti, tile_start.data(), sizeof(int) * (n + 1));
    int *bi = ti + (n + 1);
    memcpy(bi, bs.data(), sizeof(int) * (n + 1));
    HIP_TRY(hipMemcpyAsync(c->d_desc(), dd, sizeof(CfgDesc) * n, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->d_tiles(), ti, sizeof(int) * (n + 1), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->d_blocks(), bi, sizeof(int) * (n + 1), hipMemcpyHostToDevice,
                           c->stream));
    // the staging buffer is reused by the caller: wait for the copies
    HIP_TRY(hipStreamSynchronize(c->stream));
    return TGF_OK;
}

}  // namespace

void tgf::set_last_error(const char *msg) { g_err = msg ? msg : ""; }

// ===========================================================================
// C ABI

extern "C" {

const char *tgf_last_error(void) { return g_err.c_str(); }

size_t tgf_workspace_bytes(int32_t n_cfg, const tgf_geom *geoms, tgf_storage st) {
    if (!storage_ok(st)) return 0;
    if (validate_geoms(n_cfg, geoms) != TGF_OK) return 0;
    return make_layout(n_cfg, geoms, st).total;
}

size_t tgf_workspace_bytes_sun(int32_t nc, int32_t n_cfg, const tgf_geom *geoms,
                               tgf_storage st) {
    if (nc < 2 || nc > 8 || !storage_ok(st) || st != TGF_F64_FULL) return 0;
    if (validate_geoms(n_cfg, geoms, nc, true) != TGF_OK) return 0;
    return make_layout(n_cfg, geoms, st, nc, true).total;
}

static tgf_status create_impl(tgf_ctx **out, int nc, bool general, int32_t n_cfg,
                              const tgf_geom *geoms, tgf_storage st, void *workspace_dev,
                              size_t workspace_bytes, void *hip_stream) {
    g_err.clear();
    if (!out) return fail(TGF_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!storage_ok(st)) return fail(TGF_E_INVAL, "unknown storage");
    if (general && (nc < 2 || nc > 8)) return fail(TGF_E_INVAL, "nc must be 2..8");
    if (general && st != TGF_F64_FULL)
        return fail(TGF_E_UNSUPPORTED, "SU(N) contexts use TGF_F64_FULL storage");
    tgf_status s = validate_geoms(n_cfg, geoms, nc, general);
    if (s) return s;
    if (!workspace_dev) return fail(TGF_E_INVAL, "workspace is NULL");
    if (((uintptr_t)workspace_dev) % 256)
        return fail(TGF_E_INVAL, "workspace must be 256-byte aligned");
    Layout L = make_layout(n_cfg, geoms, st, nc, general);
    if (workspace_bytes < L.total)
        return fail(TGF_E_SIZE, "workspace too small: need " + std::to_string(L.total) +
                                    " bytes, got " + std::to_string(workspace_bytes));
    tgf_ctx *c = new (std::nothrow) tgf_ctx();
    if (!c) return fail(TGF_E_INVAL, "out of host memory");
    c->n_cfg = n_cfg;
    c->st = st;
    c->nc = nc;
    c->general = general;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char *)workspace_dev;
    c->ws_bytes = workspace_bytes;
    c->L = std::move(L);
    *out = c;
    return TGF_OK;
}

tgf_status tgf_create(tgf_ctx **out, int32_t n_cfg, const tgf_geom *geoms, tgf_storage st,
                      void *workspace_dev, size_t workspace_bytes, void *hip_stream) {
    return create_impl(out, 3, false, n_cfg, geoms, st, workspace_dev, workspace_bytes,
                       hip_stream);
}

tgf_status tgf_create_sun(tgf_ctx **out, int32_t nc, int32_t n_cfg, const tgf_geom *geoms,
                          tgf_storage st, void *workspace_dev, size_t workspace_bytes,
                          void *hip_stream) {
    return create_impl(out, nc, true, n_cfg, geoms, st, workspace_dev, workspace_bytes,
                       hip_stream);
}

void tgf_destroy(tgf_ctx *c) {
    if (!c) return;
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
    if (c->h_stage) (void)hipHostFree(c->h_stage);
    delete c;
}

static tgf_status load_impl(tgf_ctx *c, const std::vector<int> &cfgs,
                            const void *const *links, const double *t0) {
    for (size_t k = 0; k < cfgs.size(); k++) {
        if (!links[k]) return fail(TGF_E_INVAL, "links pointer is NULL");
        if (!std::isfinite(t0[k]) || t0[k] < 0) return fail(TGF_E_INVAL, "t0 must be >= 0");
    }
    // SU(3): one launch checks every configuration of the call and packs each
    // into its idle buffer W[cur ^ 1] (the inputs' pointers and the
    // configurations' tables uploaded first), which becomes current only if
    // every link passed; SU(N): one check launch per configuration, then,
    // when all passed, one pack launch each into W[0]
    const bool batch = !c->general;
    std::vector<int> bts;
    if (batch) {
        tgf_status st = upload_tables(c, cfgs, nullptr, bts);   // synchronises
        if (st) return st;
        // staging for the pointers now and the defects read back below (no
        // reallocation while the pointer upload may still be reading it)
        if ((st = ensure_stage(c, sizeof(double) * 2 * cfgs.size()))) return st;
        memcpy(c->h_stage, links, sizeof(void *) * cfgs.size());
        HIP_TRY(hipMemcpyAsync((void *)c->d_src(), c->h_stage, sizeof(void *) * cfgs.size(),
                               hipMemcpyHostToDevice, c->stream));
        HIP_TRY(launch_ingest_batch(c->prec(), c->c12(), c->stream, c->d_src(), c->d_desc(),
                                    c->d_tiles(), (int)cfgs.size(), bts[cfgs.size()],
                                    c->d_partials(), c->d_rows()));
    }
    // check every input before touching storage: each check writes its two
    // defects to its own slot of the rows region, one readback for all
    for (size_t k = 0; k < cfgs.size() && !batch; k++) {
        const CfgHost &h = c->L.cfg[cfgs[k]];
        HIP_TRY(launch_check_sun(c->nc, true, c->stream, links[k], h.V, h.stride,
                                 c->d_partials(), c->d_rows() + 2 * k));
    }
    tgf_status st0 = ensure_stage(c, sizeof(double) * 2 * cfgs.size());
    if (st0) return st0;
    HIP_TRY(hipMemcpyAsync(c->h_stage, c->d_rows(), sizeof(double) * 2 * cfgs.size(),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    int bad = -1;
    double worst[2] = {0, 0};
    for (size_t k = 0; k < cfgs.size(); k++) {
        const double *d = (const double *)c->h_stage + 2 * k;
        if (!(d[0] <= 1e-10) || !(d[1] <= 1e-10)) {
            bad = cfgs[k];
            worst[0] = d[0];
            worst[1] = d[1];
            break;
        }
    }
    if (bad >= 0) {
        char buf[160];
        snprintf(buf, sizeof buf, "config %d: links not in SU(%d): max|UU^+-1| = %.3g, "
                 "max|det-1| = %.3g", bad, c->nc, worst[0], worst[1]);
        return fail(TGF_E_NOT_SU3, buf);
    }
    for (size_t k = 0; k < cfgs.size() && !batch; k++) {
        CfgHost &h = c->L.cfg[cfgs[k]];
        HIP_TRY(launch_pack_sun(c->nc, c->stream, links[k], c->ws + h.offW[0], h.V, h.stride));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < cfgs.size(); k++) {
        CfgHost &h = c->L.cfg[cfgs[k]];
        h.cur = batch ? h.cur ^ 1 : 0;
        h.t = t0[k];
        h.steps = 0;
        h.loaded = true;
    }
    return TGF_OK;
}

tgf_status tgf_load_links(tgf_ctx *c, int32_t cfg, const void *links_dev, double t0) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    std::vector<int> v{cfg};
    const void *p[1] = {links_dev};
    return load_impl(c, v, p, &t0);
}

tgf_status tgf_load_links_all(tgf_ctx *c, const void *const *links_dev, const double *t0) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if (!links_dev || !t0) return fail(TGF_E_INVAL, "links_dev / t0 is NULL");
    std::vector<int> v(c->n_cfg);
    for (int k = 0; k < c->n_cfg; k++) v[k] = k;
    return load_impl(c, v, links_dev, t0);
}

tgf_status tgf_store_links(tgf_ctx *c, int32_t cfg, void *links_dev) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    if (!links_dev) return fail(TGF_E_INVAL, "links pointer is NULL");
    CfgHost &h = c->L.cfg[cfg];
    if (!h.loaded) return fail(TGF_E_STATE, "config not loaded");
    if (c->general)
        HIP_TRY(launch_unpack_sun(c->nc, c->stream, c->ws + h.offW[h.cur], links_dev, h.V,
                                  h.stride));
    else
        HIP_TRY(launch_unpack(c->prec(), c->c12(), c->stream, c->ws + h.offW[h.cur], links_dev,
                              h.V, h.stride));
    return TGF_OK;
}

tgf_status tgf_get_time(tgf_ctx *c, int32_t cfg, double *t) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    if (!t) return fail(TGF_E_INVAL, "t is NULL");
    *t = c->L.cfg[cfg].t;
    return TGF_OK;
}

tgf_status tgf_densities(tgf_ctx *c, int32_t cfg, double *e_dev, double *q_dev) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    if (c->general) return fail(TGF_E_UNSUPPORTED, "densities: SU(3) contexts only");
    const CfgHost &h = c->L.cfg[cfg];
    if (!h.loaded) return fail(TGF_E_STATE, "config not loaded");
    if (!e_dev && !q_dev) return TGF_OK;
    std::vector<int> order(c->n_cfg);
    for (int k = 0; k < c->n_cfg; k++) order[k] = k;
    std::vector<int> ts;
    if ((s = upload_tables(c, order, nullptr, ts))) return s;
    HIP_TRY(launch_densities(c->prec(), c->c12(), c->stream, c->d_desc(), cfg, h.V, e_dev, q_dev));
    return TGF_OK;
}

tgf_status tgf_link_buffer(tgf_ctx *c, int32_t cfg, size_t *offset, size_t *bytes) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    if (!offset || !bytes) return fail(TGF_E_INVAL, "NULL argument");
    const CfgHost &h = c->L.cfg[cfg];
    if (!h.loaded) return fail(TGF_E_STATE, "config not loaded");
    *offset = h.offW[h.cur];
    *bytes = cx_bytes(c->st) * 4 * (size_t)c->ne() * (size_t)h.stride;
    return TGF_OK;
}

tgf_status tgf_unitarity(tgf_ctx *c, int32_t cfg, double *out) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    if (!out) return fail(TGF_E_INVAL, "out is NULL");
    CfgHost &h = c->L.cfg[cfg];
    if (!h.loaded) return fail(TGF_E_STATE, "config not loaded");
    return run_check(c, cfg, c->ws + h.offW[h.cur], out);
}

tgf_status tgf_measure(tgf_ctx *c, tgf_obs *out_host) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if (!out_host) return fail(TGF_E_INVAL, "out_host is NULL");
    for (int k = 0; k < c->n_cfg; k++)
        if (!c->L.cfg[k].loaded)
            return fail(TGF_E_STATE, "config " + std::to_string(k) + " not loaded");
    std::vector<int> order(c->n_cfg);
    for (int k = 0; k < c->n_cfg; k++) order[k] = k;
    std::vector<int> ts;
    if ((s = upload_tables(c, order, nullptr, ts))) return s;
    // one event: every config, row 0
    if ((s = ensure_stage(c, sizeof(MeasSlot) * c->n_cfg))) return s;
    MeasSlot *ms = (MeasSlot *)c->h_stage;
    for (int k = 0; k < c->n_cfg; k++) ms[k] = MeasSlot{0, 0, c->L.cfg[k].t};
    HIP_TRY(hipMemcpyAsync(c->d_meas(), ms, sizeof(MeasSlot) * c->n_cfg, hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(launch_fill_int(c->stream, c->d_flag(), 1, 0));
    if (c->general)
        HIP_TRY(launch_measure_sun(c->nc, c->effective_variant(), c->stream, c->d_desc(),
                                   c->d_tiles(), c->n_cfg, ts[c->n_cfg], c->d_meas(),
                                   c->d_partials(), -1));
    else
        HIP_TRY(launch_measure(c->prec(), c->c12(), c->stream, c->d_desc(), c->d_tiles(),
                               c->n_cfg, ts[c->n_cfg], c->d_meas(), c->d_partials(), -1));
    HIP_TRY(launch_finalize(c->stream, c->d_desc(), c->d_tiles(), c->n_cfg, c->d_meas(),
                            c->d_partials(), c->d_rows(), c->n_cfg, c->d_flag(), c->nc));
    HIP_TRY(hipStreamSynchronize(c->stream));   // the slot upload used the staging buffer
    size_t rb = sizeof(double) * 6 * c->n_cfg;
    HIP_TRY(hipMemcpyAsync(c->h_stage, c->d_rows(), rb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_stage + rb, c->d_flag(), sizeof(int), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    memcpy(out_host, c->h_stage, rb);
    int flag;
    memcpy(&flag, c->h_stage + rb, sizeof(int));
    if (flag) return fail(TGF_E_NONFINITE, "non-finite observable");
    return TGF_OK;
}

tgf_status tgf_flow(tgf_ctx *c, const tgf_flow_params *p, tgf_obs *rows_host, int32_t max_rows,
                    int32_t *n_rows) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if (!p || !p->t_end || !rows_host || !n_rows)
        return fail(TGF_E_INVAL, "NULL argument");
    if (!(p->eps > 0) || !std::isfinite(p->eps)) return fail(TGF_E_INVAL, "eps must be > 0");
    if (!(p->meas_dt >= 0) || !std::isfinite(p->meas_dt))
        return fail(TGF_E_INVAL, "meas_dt must be >= 0");
    if (p->reunit_every < 0) return fail(TGF_E_INVAL, "reunit_every must be >= 0");
    if (max_rows <= 0) return fail(TGF_E_SIZE, "max_rows must be positive");
    const int n = c->n_cfg;
    std::vector<Plan> plans(n);
    int n_rows_max = 0;
    for (int k = 0; k < n; k++) {
        const CfgHost &h = c->L.cfg[k];
        if (!h.loaded) return fail(TGF_E_STATE, "config " + std::to_string(k) + " not loaded");
        double te = p->t_end[k];
        if (!std::isfinite(te) || te < h.t - 1e-12)
            return fail(TGF_E_INVAL, "t_end[" + std::to_string(k) + "] before current t");
        if ((te - h.t) / p->eps > 1e8) return fail(TGF_E_INVAL, "too many steps");
        plans[k] = make_plan(h.t, std::max(te, h.t), p->eps, p->meas_dt);
        n_rows_max = std::max(n_rows_max, (int)plans[k].meas.size());
    }
    if (n_rows_max > max_rows)
        return fail(TGF_E_SIZE, "rows buffer too small: need " + std::to_string(n_rows_max));
    if (n_rows_max > kMaxRows)
        return fail(TGF_E_SIZE, "more than TGF_MAX_ROWS measurement rows in one call");

    // exec order: longest flows first, so the active configs are a prefix
    std::vector<int> order(n);
    for (int k = 0; k < n; k++) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return plans[a].n_steps > plans[b].n_steps; });
    const int max_steps = plans[order[0]].n_steps;

    // measurement events: after `k` steps (k = 0..max_steps), configs measured then
    std::vector<std::vector<std::pair<int, MeasSlot>>> ev(max_steps + 1);
    for (int e = 0; e < n; e++) {
        int cfg = order[e];
        const Plan &pl = plans[cfg];
        for (size_t r = 0; r < pl.meas.size(); r++)
            ev[pl.meas[r].first].push_back({e, MeasSlot{(int)r, 0, pl.meas[r].second}});
    }
    int n_events = 0;
    for (auto &v : ev) n_events += v.empty() ? 0 : 1;
    if (n_events > kMaxRows) return fail(TGF_E_SIZE, "too many measurement events");

    const bool fp32 = c->st != TGF_F64_FULL;
    const int reunit_every = fp32 ? p->reunit_every : 0;
    std::vector<int> ts, bs;
    if ((s = upload_tables(c, order, &plans, ts, false, reunit_every, &bs))) return s;
    // slot table
    if ((s = ensure_stage(c, sizeof(MeasSlot) * (size_t)std::max(n_events, 1) * n))) return s;
    MeasSlot *ms = (MeasSlot *)c->h_stage;
    std::vector<int> event_of_step(max_steps + 1, -1);
    {
        int e = 0;
        for (int k = 0; k <= max_steps; k++) {
            if (ev[k].empty()) continue;
            for (int j = 0; j < n; j++) ms[(size_t)e * n + j] = MeasSlot{-1, 0, 0.0};
            for (auto &pr : ev[k]) ms[(size_t)e * n + pr.first] = pr.second;
            event_of_step[k] = e++;
        }
    }
    if (n_events)
        HIP_TRY(hipMemcpyAsync(c->d_meas(), ms, sizeof(MeasSlot) * (size_t)n_events * n,
                               hipMemcpyHostToDevice, c->stream));

    // active prefix per step
    std::vector<int> active(max_steps, 0);
    for (int k = 0; k < max_steps; k++) {
        int a = 0;
        while (a < n && plans[order[a]].n_steps > k) a++;
        active[k] = a;
    }

    std::vector<Launch> ls;
    ls.push_back(Launch{3, 1, 0, 0, 0, 0, 0, 0});
    auto add_meas = [&](int k) {
        int e = event_of_step[k];
        if (e < 0) return;
        // configs measured at this event are all still "active" up to step k, but a
        // config whose flow ended earlier is never measured here, so n_cfg covers it
        ls.push_back(Launch{1, ts[n], n, 3 * k, 0, 0, e, 0});
        ls.push_back(Launch{2, n, n, 0, 0, 0, e, 0});
    };
    add_meas(0);
    for (int k = 0; k < max_steps; k++) {
        int na = active[k];
        for (int st = 0; st < 3; st++)
            ls.push_back(Launch{0, ts[na], na, k, st, reunit_every, -1, bs[na]});
        add_meas(k + 1);
    }

    const bool timing = (p->flags & TGF_TIMING) != 0;
    // the legacy null stream cannot be captured: launch directly there
    const bool graph = !(p->flags & TGF_NO_GRAPH) && !timing && c->stream != nullptr;
    // the slot upload reads the staging buffer; make sure it is done before reuse
    HIP_TRY(hipStreamSynchronize(c->stream));
    if ((s = run_launches(c, ls, p->eps, graph, timing))) return s;

    // rows back
    size_t rb = sizeof(double) * 6 * (size_t)n * n_rows_max;
    if ((s = ensure_stage(c, rb + 64))) return s;
    HIP_TRY(hipMemcpyAsync(c->h_stage, c->d_rows(), rb, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipMemcpyAsync(c->h_stage + rb, c->d_flag(), sizeof(int), hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));

    if (timing) {
        tgf_timing tm{};
        const double e = (double)cx_bytes(c->st);
        const int NE = c->ne();
        for (size_t k = 0; k < ls.size(); k++) {
            float ms_ = 0;
            HIP_TRY(hipEventElapsedTime(&ms_, c->events[2 * k], c->events[2 * k + 1]));
            const Launch &l = ls[k];
            double sites = 0;
            if (l.kind == 0)
                for (int j = 0; j < l.n_act; j++) sites += c->L.cfg[order[j]].V;
            // algorithmic bytes: every element an operation touches, once
            const double links = 4.0 * NE * e, xs = 4.0 * c->x_entries() * e;
            if (l.kind == 0) {
                tm.stage_ms += ms_;
                tm.stage_launches++;
                // links read + written, X written (stage 0), read+written (1), read (2)
                double xfac = l.stage == 1 ? 2.0 : 1.0;
                tm.stage_bytes += sites * (2.0 * links + xfac * xs);
                tm.stage_site_updates += sites / 3.0;
            } else if (l.kind == 1 || l.kind == 2) {
                tm.measure_ms += ms_;
                tm.measure_launches++;
            }
        }
        c->timing = tm;
    }

    const double *src = (const double *)c->h_stage;
    for (int r = 0; r < n_rows_max; r++)
        for (int k = 0; k < n; k++) {
            int rr = std::min(r, (int)plans[k].meas.size() - 1);
            const double *v = src + ((size_t)rr * n + k) * 6;
            tgf_obs &o = rows_host[(size_t)r * n + k];
            o.t = v[0]; o.E = v[1]; o.t2E = v[2]; o.plaq = v[3]; o.Q = v[4]; o.action = v[5];
        }
    *n_rows = n_rows_max;
    int flag;
    memcpy(&flag, c->h_stage + rb, sizeof(int));
    for (int k = 0; k < n; k++) {
        CfgHost &h = c->L.cfg[k];
        h.cur = (h.cur + 3 * plans[k].n_steps) & 1;
        h.t = std::max(p->t_end[k], h.t);
        h.steps += plans[k].n_steps;
    }
    if (flag) return fail(TGF_E_NONFINITE, "non-finite observable during the flow");
    return TGF_OK;
}

tgf_status tgf_slice_charge(tgf_ctx *c, int32_t dir, double *q_host, int32_t max_slices) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if (dir < 0 || dir > 3) return fail(TGF_E_INVAL, "dir must be 0..3");
    if (!q_host) return fail(TGF_E_INVAL, "q_host is NULL");
    if (c->general) return fail(TGF_E_UNSUPPORTED, "slice charge: SU(3) contexts only");
    size_t total = 0;
    for (int k = 0; k < c->n_cfg; k++) {
        const CfgHost &h = c->L.cfg[k];
        if (!h.loaded) return fail(TGF_E_STATE, "config " + std::to_string(k) + " not loaded");
        if (h.d[dir] > max_slices)
            return fail(TGF_E_SIZE, "max_slices smaller than the extent of direction dir");
        total += (size_t)h.d[dir];
    }
    if (total > (size_t)6 * kMaxRows * c->n_cfg)
        return fail(TGF_E_UNSUPPORTED, "too many slices in total");
    std::vector<int> order(c->n_cfg);
    for (int k = 0; k < c->n_cfg; k++) order[k] = k;
    std::vector<int> ts;
    if ((s = upload_tables(c, order, nullptr, ts))) return s;
    size_t off = 0;
    for (int k = 0; k < c->n_cfg; k++) {
        const CfgHost &h = c->L.cfg[k];
        HIP_TRY(launch_slice_charge(c->prec(), c->c12(), c->stream, c->d_desc(), k, dir,
                                    h.d[dir], h.V / h.d[dir], c->d_partials(), c->d_rows() + off));
        off += (size_t)h.d[dir];
    }
    if ((s = ensure_stage(c, sizeof(double) * total))) return s;
    HIP_TRY(hipMemcpyAsync(c->h_stage, c->d_rows(), sizeof(double) * total, hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const double *src = (const double *)c->h_stage;
    off = 0;
    for (int k = 0; k < c->n_cfg; k++) {
        const int d = c->L.cfg[k].d[dir];
        for (int t = 0; t < max_slices; t++)
            q_host[(size_t)k * max_slices + t] = t < d ? src[off + t] : 0.0;
        off += (size_t)d;
    }
    return TGF_OK;
}

tgf_status tgf_mc(tgf_ctx *c, double b, int32_t n_hybrid, int32_t n_or, uint64_t seed,
                  uint32_t sweep0) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if (c->st != TGF_F64_FULL)
        return fail(TGF_E_INVAL, "Monte Carlo needs TGF_F64_FULL storage");
    if (c->general) return fail(TGF_E_UNSUPPORTED, "Monte Carlo: SU(3) contexts only");
    if (!std::isfinite(b) || b < 0) return fail(TGF_E_INVAL, "b must be finite and >= 0");
    if (n_hybrid < 0 || n_or < 0) return fail(TGF_E_INVAL, "n_hybrid and n_or must be >= 0");
    const uint64_t sweeps = (uint64_t)n_hybrid * (uint64_t)(1 + (int64_t)n_or);
    if ((uint64_t)sweep0 + sweeps > (1ull << 32))
        return fail(TGF_E_INVAL, "sweep counter would pass 2^32");
    for (int k = 0; k < c->n_cfg; k++) {
        const CfgHost &h = c->L.cfg[k];
        if (!h.loaded) return fail(TGF_E_STATE, "config " + std::to_string(k) + " not loaded");
        for (int m = 0; m < 4; m++)
            if (h.d[m] % 2)
                return fail(TGF_E_INVAL, "config " + std::to_string(k) +
                                             ": the checkerboard needs even extents");
    }
    std::vector<int> order(c->n_cfg);
    for (int k = 0; k < c->n_cfg; k++) order[k] = k;
    std::vector<int> ts;
    if ((s = upload_tables(c, order, nullptr, ts, true))) return s;
    const double beta = 18.0 * b;
    uint32_t sweep = sweep0;
    for (int32_t h = 0; h < n_hybrid; h++)
        for (int32_t o = 0; o <= n_or; o++, sweep++)
            for (int mu = 0; mu < 4; mu++)
                for (int par = 0; par < 2; par++)
                    HIP_TRY(launch_mc(c->stream, c->d_desc(), c->d_tiles(), c->n_cfg,
                                      ts[c->n_cfg], mu, par, o == 0 ? 1 : 0, beta, seed, sweep));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int k = 0; k < c->n_cfg; k++) {
        c->L.cfg[k].t = 0;
        c->L.cfg[k].steps = 0;
    }
    return TGF_OK;
}

tgf_status tgf_get_timing(tgf_ctx *c, tgf_timing *out) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if (!out) return fail(TGF_E_INVAL, "out is NULL");
    *out = c->timing;
    return TGF_OK;
}

int32_t tgf_variant_count(void) { return V_COUNT; }

int32_t tgf_sun_variant_count(int32_t nc) { return sun_variant_count(nc); }

int32_t tgf_sun_rows_per_lane(int32_t nc, int32_t variant) {
    return sun_rows_per_lane(nc, variant);
}

int32_t tgf_sun_variant_lds(int32_t nc, int32_t variant) {
    if (nc < 2 || nc > 8) return -1;
    return sun_variant_lds(nc, variant);
}

const char *tgf_variant_name(int32_t v) {
    if (v < 0 || v >= V_COUNT) return "default";
    return variant_name(v);
}

tgf_status tgf_set_variant(tgf_ctx *c, int32_t v) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if (v < -1 || v >= c->variant_count()) return fail(TGF_E_INVAL, "variant out of range");
    c->variant = v;
    return TGF_OK;
}

int32_t tgf_get_variant(tgf_ctx *c) { return c ? c->effective_variant() : -1; }

static std::string arch_name() {
    hipDeviceProp_t prop;
    int dev = 0;
    std::string a = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        a = prop.gcnArchName;
    for (char &ch : a)
        if (ch == ' ') ch = '_';
    return a;
}

// Cache key of the variant choice: device, storage, colours, every extent.
static std::string tune_key(tgf_ctx *c) {
    std::ostringstream k;
    k << arch_name() << "/st" << (int)c->st;
    if (c->general) k << "/nc" << c->nc;
    for (auto &h : c->L.cfg) k << "/" << h.d[0] << "x" << h.d[1] << "x" << h.d[2] << "x" << h.d[3];
    return k.str();
}

// Cache key of one extent class's work-group shape under a variant.
static std::string block_key(tgf_ctx *c, int variant, const int d[4]) {
    std::ostringstream k;
    k << arch_name() << "/st" << (int)c->st << "/v" << variant << "/blk/" << d[0] << "x" << d[1]
      << "x" << d[2] << "x" << d[3];
    return k.str();
}

// A timed candidate replaces the incumbent only when faster by this fraction,
// so that choices within timing noise stay with the default.
constexpr float kTuneMargin = 0.02f;

tgf_status tgf_autotune(tgf_ctx *c, const char *cache_path) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    for (int k = 0; k < c->n_cfg; k++)
        if (!c->L.cfg[k].loaded)
            return fail(TGF_E_STATE, "config " + std::to_string(k) + " not loaded");
    std::vector<std::pair<std::string, int>> cache;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string k2;
        int v;
        while (in >> k2 >> v) cache.push_back({k2, v});
    }
    auto cached = [&](const std::string &key, int &out) {
        for (auto it = cache.rbegin(); it != cache.rend(); ++it)
            if (it->first == key) { out = it->second; return true; }
        return false;
    };
    std::vector<std::pair<std::string, int>> found;

    // classes of configurations with equal extents (the work-group shape is tuned per class)
    std::vector<std::vector<int>> classes;
    for (int k = 0; k < c->n_cfg; k++) {
        bool placed = false;
        for (auto &cl : classes) {
            const CfgHost &h0 = c->L.cfg[cl[0]], &h = c->L.cfg[k];
            if (std::equal(h.d, h.d + 4, h0.d)) { cl.push_back(k); placed = true; break; }
        }
        if (!placed) classes.push_back({k});
    }

    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // stage 0 of the given configurations (reads the current links, writes the
    // other buffer and X, so the loaded state is not modified): the least of
    // three averages over five launches, in ms
    auto time_stage0 = [&](int v, const std::vector<int> &order, float &ms) -> tgf_status {
        const int n = (int)order.size();
        std::vector<Plan> plans(c->n_cfg);
        for (auto &p : plans) { p.n_full = 1; p.n_steps = 1; p.eps_last = 0; }
        std::vector<int> ts, bs;
        tgf_status st = upload_tables(c, order, &plans, ts, false, 0, &bs);
        if (st) return st;
        auto launch = [&]() {
            if (c->general)
                return launch_stage_sun(c->nc, v, c->stream, c->d_desc(), c->d_tiles(), n, ts[n],
                                        0, 0, 0.01);
            return launch_stage(v, c->prec(), c->c12(), c->stream, c->d_desc(), c->d_tiles(), n,
                                ts[n], c->d_blocks(), bs[n], 0, 0, 0.01, 0);
        };
        ms = 1e30f;
        HIP_TRY(launch());
        for (int trial = 0; trial < 3; trial++) {
            HIP_TRY(hipEventRecord(e0, c->stream));
            for (int r = 0; r < 5; r++) HIP_TRY(launch());
            HIP_TRY(hipEventRecord(e1, c->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float t = 0;
            HIP_TRY(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t / 5);
        }
        return TGF_OK;
    };
    auto done = [&](tgf_status st) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return st;
    };

    // (1) the stage variant, on the whole batch.  Candidates: for SU(N) every
    // rows-per-lane build; for SU(3) the XCD-ordered kernels (the plain block
    // order of the same kernel runs as fast with more L2-miss traffic), not the
    // plaquette-sharing one, whose rounding depends on which configurations
    // share a work-group.
    std::vector<int> all(c->n_cfg);
    for (int k = 0; k < c->n_cfg; k++) all[k] = k;
    const std::string vkey = tune_key(c);
    int best = -1;
    if (!cached(vkey, best) || best < 0 || best >= c->variant_count()) {
        std::vector<int> cand;
        if (c->general)
            for (int v = 0; v < c->variant_count(); v++) cand.push_back(v);
        else
            cand = {V_SITE_LDS_XCD, V_SITE_ALG_XCD, V_SITE_ALG3_XCD, V_SITE_XCD, V_LINK_XCD};
        float best_ms = 0;
        for (size_t j = 0; j < cand.size(); j++) {
            float ms = 0;
            if ((s = time_stage0(cand[j], all, ms))) return done(s);
            if (j == 0 || ms < best_ms * (1.0f - kTuneMargin)) { best = cand[j]; best_ms = ms; }
        }
        found.push_back({vkey, best});
    }
    c->variant = best;

    // (2) the work-group shape of the LDS-staged variants, per extent class,
    // timed on that class alone
    if (!c->general && variant_is_lds(best)) {
        for (auto &cl : classes) {
            CfgHost &h0 = c->L.cfg[cl[0]];
            const std::string bkey = block_key(c, best, h0.d);
            int blk = 0;
            if (!cached(bkey, blk) || blk < 1 || blk > kBlock) {
                blk = default_block(h0.d);
                const int alt = other_block(h0.d);
                if (alt) {
                    float ms_def = 0, ms_alt = 0;
                    for (int k : cl) c->L.cfg[k].blk = blk;
                    if ((s = time_stage0(best, cl, ms_def))) return done(s);
                    for (int k : cl) c->L.cfg[k].blk = alt;
                    if ((s = time_stage0(best, cl, ms_alt))) return done(s);
                    if (ms_alt < ms_def * (1.0f - kTuneMargin)) blk = alt;
                }
                found.push_back({bkey, blk});
            }
            for (int k : cl) c->L.cfg[k].blk = blk;
        }
    }
    if (cache_path && !found.empty()) {
        std::ofstream o(cache_path, std::ios::app);
        if (o)
            for (auto &f : found) o << f.first << " " << f.second << "\n";
    }
    return done(TGF_OK);
}

tgf_status tgf_get_block(tgf_ctx *c, int32_t cfg, int32_t *sites) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    if (!sites) return fail(TGF_E_INVAL, "sites is NULL");
    *sites = c->L.cfg[cfg].blk;
    return TGF_OK;
}

tgf_status tgf_set_block(tgf_ctx *c, int32_t cfg, int32_t sites) {
    g_err.clear();
    tgf_status s = check_ctx(c);
    if (s) return s;
    if ((s = check_cfg(c, cfg))) return s;
    if (sites == 0) sites = default_block(c->L.cfg[cfg].d);
    if (sites < 64 || sites > kBlock)
        return fail(TGF_E_INVAL, "sites per work-group must be 64..256 (0 = default)");
    c->L.cfg[cfg].blk = sites;
    return TGF_OK;
}

tgf_status tgf_stream_copy(void *dst_dev, const void *src_dev, size_t bytes, void *hip_stream) {
    g_err.clear();
    if (!dst_dev || !src_dev) return fail(TGF_E_INVAL, "NULL pointer");
    if (((uintptr_t)dst_dev | (uintptr_t)src_dev | bytes) % 16)
        return fail(TGF_E_INVAL, "pointers and size must be 16-byte aligned");
    HIP_TRY(launch_copy((hipStream_t)hip_stream, dst_dev, src_dev, bytes));
    return TGF_OK;
}

}  // extern "C"
