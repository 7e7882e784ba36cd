// Host sanitizer driver for the runtime of libtgf (test infrastructure):
// workspace sizing and layout over many geometries and storages, context
// creation and destruction over a caller workspace that is never touched, the
// per-configuration work-group shapes, variant selection, and every argument
// and state check that returns before a device call.  Linked against stub
// launchers and built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py; needs no GPU.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "tgf.h"

static int fails = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);    \
            fails++;                                                              \
        }                                                                         \
    } while (0)

static tgf_geom geom(int a, int b, int c, int d, int t01 = 1) {
    tgf_geom g{};
    g.dims[0] = a; g.dims[1] = b; g.dims[2] = c; g.dims[3] = d;
    g.twist[0] = t01;
    return g;
}

int main() {
    void *fake = reinterpret_cast<void *>(uintptr_t(1) << 40);   // aligned, never dereferenced
    std::vector<tgf_geom> gs;
    for (int L : {2, 3, 4, 5, 6, 8, 10, 12, 16, 32}) gs.push_back(geom(L, L, 3 * L, 3 * L));
    gs.push_back(geom(3, 5, 4, 7, 2));
    gs.push_back(geom(20, 20, 4, 4, 0));
    for (int st = 0; st < 3; st++) {
        for (auto &g : gs) CHECK(tgf_workspace_bytes(1, &g, (tgf_storage)st) > 0);
        const size_t all = tgf_workspace_bytes((int32_t)gs.size(), gs.data(), (tgf_storage)st);
        CHECK(all > 0);
        tgf_ctx *c = nullptr;
        CHECK(tgf_create(&c, (int32_t)gs.size(), gs.data(), (tgf_storage)st, fake, all, nullptr) ==
              TGF_OK);
        int32_t b = 0;
        for (int k = 0; k < (int)gs.size(); k++) {
            CHECK(tgf_get_block(c, k, &b) == TGF_OK && b >= 64 && b <= 256);
            CHECK(tgf_set_block(c, k, 256) == TGF_OK);
            CHECK(tgf_set_block(c, k, 0) == TGF_OK);
            CHECK(tgf_set_block(c, k, 300) == TGF_E_INVAL);
        }
        for (int v = -1; v < tgf_variant_count(); v++) CHECK(tgf_set_variant(c, v) == TGF_OK);
        CHECK(tgf_set_variant(c, tgf_variant_count()) == TGF_E_INVAL);
        tgf_obs obs[16];
        double te[16];
        for (double &x : te) x = 0.1;
        tgf_flow_params p{0.01, te, 0.02, 10, 0};
        int32_t nr = 0;
        CHECK(tgf_flow(c, &p, obs, 16, &nr) == TGF_E_STATE);
        CHECK(tgf_measure(c, obs) == TGF_E_STATE);
        CHECK(tgf_store_links(c, 0, fake) == TGF_E_STATE);
        CHECK(tgf_autotune(c, nullptr) == TGF_E_STATE);
        double u[2];
        CHECK(tgf_unitarity(c, 0, u) == TGF_E_STATE);
        CHECK(tgf_densities(c, 0, nullptr, nullptr) == TGF_E_STATE);
        size_t off = 0, nb = 0;
        CHECK(tgf_link_buffer(c, 0, &off, &nb) == TGF_E_STATE);
        CHECK(tgf_load_links(c, 0, nullptr, 0.0) == TGF_E_INVAL);
        CHECK(tgf_load_links(c, 99, fake, 0.0) == TGF_E_INVAL);
        CHECK(tgf_slice_charge(c, 5, u, 2) == TGF_E_INVAL);
        tgf_flow_params bad{-1.0, te, 0.0, 0, 0};
        CHECK(tgf_flow(c, &bad, obs, 16, &nr) == TGF_E_INVAL);
        tgf_destroy(c);
        CHECK(tgf_create(&c, (int32_t)gs.size(), gs.data(), (tgf_storage)st, fake, all - 1,
                         nullptr) == TGF_E_SIZE);
    }
    // SU(N) contexts
    for (int nc = 2; nc <= 8; nc++) {
        tgf_geom g = geom(4, 4, 4 * nc, 4 * nc, nc - 1);
        const size_t need = tgf_workspace_bytes_sun(nc, 1, &g, TGF_F64_FULL);
        CHECK(need > 0);
        tgf_ctx *c = nullptr;
        CHECK(tgf_create_sun(&c, nc, 1, &g, TGF_F64_FULL, fake, need, nullptr) == TGF_OK);
        tgf_destroy(c);
    }
    // invalid geometries and storages
    tgf_geom bad = geom(1, 4, 4, 4);
    CHECK(tgf_workspace_bytes(1, &bad, TGF_F64_FULL) == 0);
    tgf_geom big = geom(2048, 2048, 512, 2);
    CHECK(tgf_workspace_bytes(1, &big, TGF_F32_C12) == 0);
    tgf_geom tw = geom(4, 4, 4, 4, 3);
    CHECK(tgf_workspace_bytes(1, &tw, TGF_F64_FULL) == 0);
    CHECK(tgf_workspace_bytes(1, gs.data(), (tgf_storage)7) == 0);
    CHECK(tgf_workspace_bytes(0, gs.data(), TGF_F64_FULL) == 0);
    // allocation-free measurement: host checks only
    tgf_obs *out = reinterpret_cast<tgf_obs *>(fake);
    tgf_geom huge = geom(4096, 4096, 2, 2);
    CHECK(tgf_measure_noalloc(&huge, fake, 0.0, out, nullptr) == TGF_E_SIZE);
    CHECK(tgf_measure_noalloc(&tw, fake, 0.0, out, nullptr) == TGF_E_INVAL);
    CHECK(tgf_measure_noalloc(gs.data(), nullptr, 0.0, out, nullptr) == TGF_E_INVAL);
    CHECK(tgf_measure_noalloc(gs.data(), fake, -1.0, out, nullptr) == TGF_E_INVAL);
    CHECK(tgf_last_error() != nullptr);
    tgf_destroy(nullptr);
    std::printf("runtime driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
