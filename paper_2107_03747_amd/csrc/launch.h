// launch.h -- host-side launchers of the device kernels (internal to libtgf).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "layout.h"

namespace tgf {

enum Prec { P_F64 = 0, P_F32 = 1 };

// Stage-kernel variants (thread <-> link mapping and launch shape).
enum Variant {
    V_SITE = 0,       // one thread per site, 4 links, shared upper plaquettes
    V_LINK = 1,       // one thread per link (wave-uniform mu), no sharing
    V_SITE_XCD = 2,   // V_SITE with XCD-contiguous tile order
    V_LINK_XCD = 3,   // V_LINK with XCD-contiguous tile order
    V_SITE_ALG = 4,   // V_SITE with su(3) (8-real) force accumulators, upper
                      // plaquettes projected from their two computed rows
    V_SITE_ALG_XCD = 5,
    V_SITE_ALG3 = 6,  // V_SITE_ALG capped at 168 registers (three waves per SIMD)
    V_SITE_ALG3_XCD = 7,
    V_SITE_LDS = 8,   // V_SITE_ALG reading links of the work-group's own sites
                      // from an LDS copy
    V_SITE_LDS_XCD = 9,
    V_SITE_PLQ = 10,  // V_SITE_ALG with the block's upper plaquettes kept in LDS and
                      // reused, conjugated, as in-block lower staple terms
    V_SITE_PLQ_XCD = 11,
    V_COUNT = 12
};
const char *variant_name(int v);

// All launchers enqueue on `s` and return the hipError_t of the launch.
// `tile_start` has n_act+1 entries (exec order); tiles are 64 sites.
// `blk_start` (n_act+1 entries) numbers the work-groups of the LDS-staged
// variants: CfgDesc::blk sites each, never more than one configuration.
// One RK stage (staples, force, update of every link) is one launch;
// reunit_every > 0 reunitarises in FP64 at the end of every reunit_every-th
// step of each configuration (counted from its load, CfgDesc::reunit_phase).
hipError_t launch_stage(int variant, Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs,
                        const int *tile_start, int n_act, int n_tiles, const int *blk_start,
                        int n_blocks, int step, int stage, double eps, int reunit_every);
inline bool variant_is_lds(int v) { return v == V_SITE_LDS || v == V_SITE_LDS_XCD; }

hipError_t launch_measure(Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs,
                          const int *tile_start, int n_cfg, int n_tiles, const MeasSlot *slots,
                          double *partials, int buf_sel);

// nc: colours (the plaquette is normalised by 6 nc V)
hipError_t launch_finalize(hipStream_t s, const CfgDesc *cfgs, const int *tile_start, int n_cfg,
                           const MeasSlot *slots, const double *partials, double *rows,
                           int n_cfg_total, int *flag, int nc);

// storage buffer W (of config c) -> canonical complex128 [V][4][3][3]
hipError_t launch_unpack(Prec p, bool c12, hipStream_t s, const void *W, void *dst, int V,
                         int stride);

// Ingest of one or more configurations in one go (canonical complex128
// inputs srcs[k], a device array of n_cfg pointers; descriptors and tile
// table of those configurations in order): checks every link (unitarity
// defects max|UU^+ - 1|, max|det U - 1| of configuration k to out[2k],
// out[2k+1]; partials holds 2 doubles per tile) and packs each configuration
// into its idle buffer W[cur ^ 1], which the caller makes current when every
// defect is within the tolerance.
hipError_t launch_ingest_batch(Prec p, bool c12, hipStream_t s, const void *srcs,
                               const CfgDesc *cfgs, const int *tile_start, int n_cfg, int n_tiles,
                               double *partials, double *out);
// Unitarity defects of stored links.  Partials need ceil(V/64)*2 doubles;
// out 2 doubles.
hipError_t launch_check(Prec p, bool c12, hipStream_t s, const void *src, int V, int stride,
                        double *partials, double *out);

// Topological charge per slice of direction `dir` for config ci (exec-order
// descriptor at cfgs[ci]); partials need n_slices * ceil(slice_sites/256)
// doubles, out n_slices doubles.
hipError_t launch_slice_charge(Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs, int ci,
                               int dir, int n_slices, int slice_sites, double *partials,
                               double *out);

// Per-site e(n) and q(n) of config ci (exec-order descriptor at cfgs[ci]), V
// doubles each in site order; either output may be null.
hipError_t launch_densities(Prec p, bool c12, hipStream_t s, const CfgDesc *cfgs, int ci, int V,
                            double *e_out, double *q_out);

// One Monte Carlo launch: the links of direction mu on the sites of parity
// par (0 even, 1 odd) of every configuration, heat bath (heatbath = 1) or
// over-relaxation, in place in W[cur].  FP64 full storage only.  tile_start
// counts tiles of 64 sites of one parity (ceil(V/2 / 64) per configuration).
hipError_t launch_mc(hipStream_t s, const CfgDesc *cfgs, const int *tile_start, int n_cfg,
                     int n_tiles, int mu, int par, int heatbath, double beta, uint64_t seed,
                     uint32_t sweep);

// max over ntiles pairs of defects in partials -> out[2]
hipError_t launch_check_final(hipStream_t s, const double *partials, int ntiles, double *out);

// General SU(N), FP64 full storage [mu][N^2][stride], 2 <= nc <= 8 (sun.hip).
// Same tile table, ping-pong and partials conventions as the SU(3) launchers.
// variant selects the rows held per lane (sun_rows_per_lane) and whether the
// products exchange rows through cross-lane permutes or LDS (sun_variant_lds);
// -1 = 0.
int sun_variant_count(int nc);
int sun_rows_per_lane(int nc, int variant);   // 0 if the variant does not exist
int sun_variant_lds(int nc, int variant);     // 1 LDS operands, 0 permutes, -1 no such variant
hipError_t launch_stage_sun(int nc, int variant, hipStream_t s, const CfgDesc *cfgs,
                            const int *tile_start, int n_act, int n_tiles, int step, int stage,
                            double eps);
hipError_t launch_measure_sun(int nc, int variant, hipStream_t s, const CfgDesc *cfgs,
                              const int *tile_start, int n_cfg, int n_tiles, const MeasSlot *slots,
                              double *partials, int buf_sel);
hipError_t launch_pack_sun(int nc, hipStream_t s, const void *src, void *W, int V, int stride);
hipError_t launch_unpack_sun(int nc, hipStream_t s, const void *W, void *dst, int V, int stride);
hipError_t launch_check_sun(int nc, bool canon, hipStream_t s, const void *src, int V, int stride,
                            double *partials, double *out);

// Set the thread-local message returned by tgf_last_error.
void set_last_error(const char *msg);

hipError_t launch_fill_int(hipStream_t s, int *dst, int n, int value);
hipError_t launch_copy(hipStream_t s, void *dst, const void *src, size_t bytes);

}  // namespace tgf
