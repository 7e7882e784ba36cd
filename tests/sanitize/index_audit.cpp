// Host audit of the stage kernels' index arithmetic (test infrastructure).
//
// Replays, on the CPU and with the kernels' own index functions (make_geo,
// Geo::up/dn, remap_block, find_cfg, block_order from lattice_dev.h), every work-group,
// wave and lane of the stage launches -- the LDS-staged kernel on its
// per-configuration block table and the tile-based site kernels on the tile
// table, each in both block orders -- and checks every link, accumulator and
// output access they make: site indices inside their configuration, byte
// offsets inside the configuration's buffers (the FP32 paired-entry layout
// and the FP64 entry planes), LDS slots inside the staged block, the source
// lanes of the in-wave plaquette reuse among the wave's active lanes, the
// XCD block remap and the column launch order of large boxes as one-to-one
// maps, and every site updated exactly once.  Each byte offset is also formed
// the kernels' way, as a 32-bit unsigned lane offset ((unsigned)j * 16u, or
// * 8u for entry 8 of the FP32 full storage) on a 64-bit plane base, and must
// equal the 64-bit value; boxes at the runtime's site cap (2^28 - 256) are
// audited on their first and last work-groups, where the offsets are largest.
// The access list per lane follows site_wave_work / site_alg_work /
// update_link_z in kernels.hip.  Built host-only with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitizers.py.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <vector>

#include "lattice_dev.h"
#include "layout.h"

using namespace tgf;

static long long checked = 0, bad = 0;
static void fail(const char *what, int ci, int i, long long v) {
    if (bad < 20) std::fprintf(stderr, "violation: %s cfg %d site %d value %lld\n", what, ci, i, v);
    bad++;
}

struct Case {
    std::vector<CfgDesc> c;
    int ne, rbytes;   // entries per link (6, 9), bytes of a real (4, 8)
};

static int default_blk(const int d[4]) {   // the runtime's default shape rule
    const int plane = d[0] * d[1];
    if (plane > kBlock) return kBlock;
    const int k = kBlock / plane;
    return k * plane >= kBlock / 2 ? k * plane : kBlock;
}

static int chunk_rule(const int d[4], int blk) {   // the runtime's column rule (block_chunk)
    const long long s = (long long)d[0] * d[1] * d[2];
    if (s % blk) return 0;
    const long long slice = s / blk;
    if (slice <= 64) return 0;
    for (int ch = 16; ch >= 4; ch--)
        if (slice % ch == 0) return ch;
    return 0;
}

static Case make_case(const std::vector<std::array<int, 4>> &dims, int ne, int rbytes, bool planes) {
    Case k;
    k.ne = ne;
    k.rbytes = rbytes;
    for (auto &d : dims) {
        CfgDesc c{};
        for (int m = 0; m < 4; m++) c.d[m] = d[m];
        c.V = d[0] * d[1] * d[2] * d[3];
        c.stride = (c.V + 255) / 256 * 256;
        c.blk = planes ? default_blk(c.d) : kBlock;
        c.chunk = chunk_rule(c.d, c.blk);
        k.c.push_back(c);
    }
    return k;
}

// the kernels' per-lane byte offset: 32-bit unsigned, added to a 64-bit plane base
static void check_lane_off(int ci, int j, unsigned unit) {
    const unsigned u = (unsigned)j * unit;
    if ((long long)u != (long long)j * unit) fail("32-bit lane offset wraps", ci, j, (long long)j * unit);
}

// byte range of a link's 16-byte units in its buffer
static void check_link(const Case &k, int ci, int mu, int j) {
    const CfgDesc &c = k.c[ci];
    checked++;
    if (j < 0 || j >= c.V) return fail("link site", ci, j, j);
    check_lane_off(ci, j, 16u);
    if (k.rbytes == 4 && k.ne == 9) check_lane_off(ci, j, 8u);
    const long long wbytes = 4LL * k.ne * c.stride * 2 * k.rbytes;
    if (k.rbytes == 4) {
        const int nu = k.ne == 9 ? 4 : 3;
        for (int e = 0; e < nu; e++) {
            const long long off = (long long)(mu * k.ne) * c.stride * 8 + (long long)e * c.stride * 16 +
                                  (long long)j * 16;
            if (off < 0 || off + 16 > wbytes) fail("link unit", ci, j, off);
        }
        if (k.ne == 9) {
            const long long off = (long long)(mu * 9 + 8) * c.stride * 8 + (long long)j * 8;
            if (off + 8 > wbytes) fail("link entry 8", ci, j, off);
        }
    } else {
        for (int e = 0; e < k.ne; e++) {
            const long long off = ((long long)(mu * k.ne + e) * c.stride + j) * 16;
            if (off < 0 || off + 16 > wbytes) fail("link entry", ci, j, off);
        }
    }
}

static void check_x(const Case &k, int ci, int mu, int i) {
    const CfgDesc &c = k.c[ci];
    checked++;
    const long long xbytes = 4LL * 4 * c.stride * 2 * k.rbytes;
    check_lane_off(ci, i, 16u);
    for (int u = 0; u < (k.rbytes == 4 ? 2 : 4); u++) {
        const long long off = k.rbytes == 4
                                  ? (long long)(mu * 4) * c.stride * 8 + (long long)u * c.stride * 16 + (long long)i * 16
                                  : ((long long)(mu * 4 + u) * c.stride + i) * 16;
        if (off < 0 || off + 16 > xbytes) fail("accumulator", ci, i, off);
    }
}

struct Access {
    int mu, j;
};

// The link reads of one lane in program order (done: lower terms taken from
// the wave, bit 4 mu + nu), as in site_wave_work / site_alg_work.
static void lane_accesses(const CfgDesc &c, int i, unsigned done, bool wave,
                          std::vector<Access> &out, std::vector<Access> &reuse) {
    const Geo g = make_geo(c, i);
    out.clear();
    reuse.clear();
    for (int mu = 0; mu < 4; mu++)
        for (int nu = mu + 1; nu < 4; nu++) {
            out.push_back({nu, i + g.up(mu)});
            out.push_back({mu, i + g.up(nu)});
            if (wave) {
                if ((done >> (4 * mu + nu)) & 1u) reuse.push_back({nu, i + g.dn(nu)});
                if ((done >> (4 * nu + mu)) & 1u) reuse.push_back({mu, i + g.dn(mu)});
            }
        }
    for (int MU = 0; MU < 4; MU++)
        for (int nu = 0; nu < 4; nu++) {
            if (nu == MU || (wave && ((done >> (4 * MU + nu)) & 1u))) continue;
            const int imn = i + g.dn(nu);
            out.push_back({nu, imn + g.up(MU)});
            out.push_back({MU, imn});
            out.push_back({nu, imn});
        }
}

// edge > 0: the block maps are still checked over the whole launch, but only
// the work-groups whose block is among the first or last `edge` blocks of its
// configuration are replayed, and site coverage is not tallied (boxes of
// hundreds of millions of sites)
static void lds_launch(const Case &k, bool xcd, bool wave_reuse, int edge = 0) {
    const int n = (int)k.c.size();
    std::vector<int> bs(n + 1, 0);
    for (int a = 0; a < n; a++) bs[a + 1] = bs[a] + (k.c[a].V + k.c[a].blk - 1) / k.c[a].blk;
    const int nb = bs[n];
    const int grid = xcd ? (nb + 7) / 8 * 8 : nb;
    std::vector<int> seen(nb, 0), order_seen(nb, 0);
    std::vector<std::vector<int>> cover(n);
    if (!edge)
        for (int a = 0; a < n; a++) cover[a].assign(k.c[a].V, 0);
    std::vector<Access> acc, reuse;
    for (int hb = 0; hb < grid; hb++) {
        const int b = remap_block(hb, nb, xcd ? 1 : 0);
        if (b >= nb) continue;
        if (b < 0) { fail("block", -1, hb, b); continue; }
        seen[b]++;
        const int ci = find_cfg(bs.data(), n, b);
        if (!(bs[ci] <= b && b < bs[ci + 1])) { fail("block config", ci, b, b); continue; }
        const CfgDesc &c = k.c[ci];
        const int ob = block_order(b - bs[ci], c);
        if (ob < 0 || ob >= bs[ci + 1] - bs[ci]) { fail("block order", ci, b, ob); continue; }
        order_seen[bs[ci] + ob]++;
        if (edge && ob >= edge && ob < bs[ci + 1] - bs[ci] - edge) continue;
        const int base = ob * c.blk;
        const int nblk = std::min(c.blk, c.V - base);
        if (nblk < 1 || c.blk > kBlock) { fail("block size", ci, base, nblk); continue; }
        for (int t = 0; t < nblk; t++) {       // staging: LDS slot t <- site base + t
            checked++;
            if (t >= kBlock) fail("lds slot", ci, base + t, t);
            check_link(k, ci, 0, base + t);
            check_link(k, ci, 3, base + t);
        }
        for (int w = 0; w * 64 < nblk; w++) {
            const int tb = base + 64 * w, nw = std::min(64, nblk - 64 * w);
            // wave-uniform reuse decisions (the __all votes of site_wave_work)
            unsigned done = 0;
            if (wave_reuse)
                for (int mu = 0; mu < 4; mu++)
                    for (int nu = mu + 1; nu < 4; nu++) {
                        bool all_n = true, all_m = true;
                        for (int l = 0; l < nw; l++) {
                            const Geo g = make_geo(c, tb + l);
                            all_n &= (unsigned)(tb + l + g.dn(nu) - tb) < (unsigned)nw;
                            all_m &= (unsigned)(tb + l + g.dn(mu) - tb) < (unsigned)nw;
                        }
                        if (all_n) done |= 1u << (4 * mu + nu);
                        if (all_m) done |= 1u << (4 * nu + mu);
                    }
            std::vector<std::vector<Access>> lists(nw), reuses(nw);
            for (int l = 0; l < nw; l++) lane_accesses(c, tb + l, done, wave_reuse, lists[l], reuses[l]);
            for (int l = 1; l < nw; l++)
                if (lists[l].size() != lists[0].size()) fail("divergent access list", ci, tb + l, 0);
            for (size_t s = 0; s < lists[0].size(); s++) {
                bool in_block = true;   // wave vote of StagedLinks
                for (int l = 0; l < nw; l++)
                    in_block &= (unsigned)(lists[l][s].j - base) < (unsigned)nblk;
                for (int l = 0; l < nw; l++) {
                    const Access &x = lists[l][s];
                    if (in_block) {
                        checked++;
                        if ((unsigned)(x.j - base) >= (unsigned)nblk) fail("lds read", ci, x.j, x.j - base);
                    } else {
                        check_link(k, ci, x.mu, x.j);
                    }
                }
            }
            for (int l = 0; l < nw; l++) {
                const int i = tb + l;
                for (const Access &x : reuses[l]) {   // shuffle source lane + conjugating link
                    checked++;
                    if ((unsigned)(x.j - tb) >= (unsigned)nw) fail("shuffle lane", ci, i, x.j - tb);
                    check_link(k, ci, x.mu, x.j);
                }
                for (int mu = 0; mu < 4; mu++) {      // own link, X, output
                    check_link(k, ci, mu, i);
                    check_x(k, ci, mu, i);
                }
                if (!edge) cover[ci][i]++;
            }
        }
    }
    for (int b = 0; b < nb; b++) {
        if (seen[b] != 1) fail("block coverage", -1, b, seen[b]);
        if (order_seen[b] != 1) fail("block order coverage", -1, b, order_seen[b]);
    }
    if (edge) return;
    for (int a = 0; a < n; a++)
        for (int i = 0; i < k.c[a].V; i++)
            if (cover[a][i] != 1) fail("site coverage", a, i, cover[a][i]);
}

static void tile_launch(const Case &k, bool xcd) {
    const int n = (int)k.c.size();
    std::vector<int> ts(n + 1, 0);
    for (int a = 0; a < n; a++) ts[a + 1] = ts[a] + (k.c[a].V + 63) / 64;
    const int nt = ts[n];
    const int nb = (nt + 3) / 4;
    const int grid = xcd ? (nb + 7) / 8 * 8 : nb;
    std::vector<std::vector<int>> cover(n);
    for (int a = 0; a < n; a++) cover[a].assign(k.c[a].V, 0);
    std::vector<Access> acc, reuse;
    for (int hb = 0; hb < grid; hb++) {
        const int b = remap_block(hb, nb, xcd ? 1 : 0);
        if (b >= nb) continue;
        for (int w = 0; w < 4; w++) {
            const int tile = b * 4 + w;
            if (tile >= nt) continue;
            const int ci = find_cfg(ts.data(), n, tile);
            const CfgDesc &c = k.c[ci];
            for (int l = 0; l < 64; l++) {
                const int i = (tile - ts[ci]) * 64 + l;
                if (i >= c.V) continue;
                lane_accesses(c, i, 0, false, acc, reuse);
                for (const Access &x : acc) check_link(k, ci, x.mu, x.j);
                for (int mu = 0; mu < 4; mu++) {
                    check_link(k, ci, mu, i);
                    check_x(k, ci, mu, i);
                }
                cover[ci][i]++;
            }
        }
    }
    for (int a = 0; a < n; a++)
        for (int i = 0; i < k.c[a].V; i++)
            if (cover[a][i] != 1) fail("site coverage (tiles)", a, i, cover[a][i]);
}

// block_order alone: a one-to-one map of each configuration's blocks, over a
// range of extents and work-group shapes where the column order applies.
static void order_check() {
    int used = 0;
    for (int d0 : {4, 8, 12, 16, 24, 32, 48})
        for (int d2 : {8, 24, 40, 96, 144})
            for (int d3 : {2, 5, 96}) {
                const int d[4] = {d0, d0, d2, d3};
                for (int blk : {kBlock, default_blk(d), 64, 128, 192, 200}) {
                    CfgDesc c{};
                    for (int m = 0; m < 4; m++) c.d[m] = d[m];
                    c.V = d0 * d0 * d2 * d3;
                    c.blk = blk;
                    c.chunk = chunk_rule(c.d, blk);
                    if (!c.chunk) continue;
                    used++;
                    const int nb = (c.V + blk - 1) / blk;
                    std::vector<int> hit(nb, 0);
                    for (int j = 0; j < nb; j++) {
                        const int b = block_order(j, c);
                        checked++;
                        if (b < 0 || b >= nb) { fail("order range", 0, j, b); continue; }
                        hit[b]++;
                    }
                    for (int b = 0; b < nb; b++)
                        if (hit[b] != 1) fail("order coverage", 0, b, hit[b]);
                }
            }
    if (used < 20) fail("too few column-order shapes", 0, used, used);
}

int main() {
    order_check();
    const std::vector<std::vector<std::array<int, 4>>> batches = {
        {{4, 4, 12, 12}},                                                 // the faulting case's box
        {{6, 6, 18, 18}, {8, 8, 24, 24}, {10, 10, 30, 30}},                // the benchmark's extents
        {{4, 4, 12, 12}, {3, 5, 4, 7}, {10, 10, 6, 6}, {6, 6, 18, 18}},   // ragged, straddling
        {{2, 2, 2, 2}, {8, 8, 4, 6}, {12, 12, 6, 4}, {32, 32, 8, 4}},     // degenerate, planes > 256
        {{16, 16, 72, 2}, {6, 6, 18, 18}, {16, 16, 96, 3}},               // column launch order
    };
    for (auto &dims : batches)
        for (int st = 0; st < 3; st++)
            for (int planes = 0; planes < 2; planes++) {
                const Case k = make_case(dims, st == 2 ? 6 : 9, st == 0 ? 8 : 4, planes);
                for (int xcd = 0; xcd < 2; xcd++) {
                    lds_launch(k, xcd, st == 2);   // 12-real: in-wave plaquette reuse
                    if (planes == 0) tile_launch(k, xcd);
                }
            }
    // the largest boxes: 8x8x1752x1752 (196M sites, replicated in the GPU
    // maximum-size test) and two boxes just under the site cap of 2^28 - 256,
    // one of whole 256-site planes and one of 1020-site planes
    const std::vector<std::array<int, 4>> big = {
        {8, 8, 1752, 1752}, {16, 16, 1024, 1023}, {30, 34, 511, 515}};
    for (auto &d : big) {
        const long long V = (long long)d[0] * d[1] * d[2] * d[3];
        if (V > (1LL << 28) - 256) fail("audit box over the site cap", 0, 0, V);
        for (int st = 0; st < 3; st++) {
            const Case k = make_case({d}, st == 2 ? 6 : 9, st == 0 ? 8 : 4, true);
            for (int xcd = 0; xcd < 2; xcd++) lds_launch(k, xcd, st == 2, 64);
        }
    }
    std::printf("index audit: %lld accesses checked, %lld violations\n", checked, bad);
    return bad ? 1 : 0;
}
