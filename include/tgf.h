/*
 * tgf.h -- C ABI of libtgf.so: twisted Wilson flow of SU(3) lattice gauge
 * fields on MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem (Bribian, Dasilva
 * Golan, Garcia Perez, Ramos, arXiv 2107.03747, sec. 3.1): SU(3) links
 * U_mu(n) on an L x L x 3L x 3L torus whose short-short plane carries
 * twisted boundary conditions through the factors Z_{mu nu}(n) of the Wilson
 * action; the links are evolved with the Wilson-flow discretisation of the
 * gradient flow equation (sec. 1) to flow time t, and at t the clover energy
 * density E_cl (eq. gmunu), t^2 <E>, the plaquette and the topological charge
 * Q (eq. qlatt) are measured.
 *
 * Conventions
 *   - Directions mu = 0..3 are the paper's 1..4.  The twisted plane of the
 *     paper is (0, 1) here; dims = {d0, d1, d2, d3} = {L, L, 3L, 3L}.  Any
 *     d_mu >= 2 is accepted.
 *   - twist[6] = n_01, n_02, n_03, n_12, n_13, n_23 in {0, 1, 2}; the paper's
 *     setting is {1,0,0,0,0,0}.  Z_{mu nu}(n) = exp(2 pi i n_{mu nu}/3) when
 *     n_mu = n_nu = 0 (the 0-based form of the paper's x_1 = x_2 = 1) and 1
 *     elsewhere; Z_{nu mu} = Z_{mu nu}^*.
 *   - Canonical link layout (every links_dev argument): complex128 (two
 *     doubles, re then im), C-contiguous [d3][d2][d1][d0][4][3][3], site
 *     index n0 + d0*(n1 + d1*(n2 + d2*n3)), row-major 3x3, device memory.
 *   - Flow: Luscher's three-stage Runge-Kutta scheme with force
 *     F = -P_ah(Omega) (P_ah = traceless anti-Hermitian part, Omega the
 *     twisted staple sum), step eps, a shortened last step to reach t_end.
 *   - Observables (FP64, tgf_obs): E = site average of
 *     e(n) = 1/2 sum_{mu,nu} Tr G_{mu nu} G_{mu nu}; t2E = t^2 E;
 *     plaq = (1/18V) sum_n sum_{mu<nu} Re Tr[Z^* P_{mu nu}(n)];
 *     Q = (1/16 pi^2) sum_n Tr G G~ with eps_{0123} = +1;
 *     action = sum_n sum_{mu<nu} Re Tr[1 - Z^* P_{mu nu}(n)].
 *
 * Ownership: the caller owns all device memory -- the workspace (one
 * allocation of tgf_workspace_bytes), every link buffer -- and the HIP
 * stream.  The library never allocates or frees device memory; a context
 * owns only host state (including a pinned staging buffer) and its cached
 * HIP graph.
 *
 * Ordering and threading: every call enqueues on the context's stream.
 * tgf_load_links*, tgf_measure, tgf_flow and tgf_unitarity synchronise that
 * stream before returning.  A context is not thread-safe; contexts on
 * different streams are independent.
 *
 * Errors: every call returns a tgf_status and never aborts or throws.
 * Arguments are validated on the host before anything is enqueued; on a
 * validation error nothing is enqueued and the context is unchanged.
 * tgf_last_error() gives a thread-local message for the last failure.
 */
#ifndef TGF_H
#define TGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TGF_OK = 0,
    TGF_E_INVAL = -1,       /* bad argument (dims, twist, eps, t, pointer, cfg index) */
    TGF_E_SIZE = -2,        /* workspace or row buffer too small */
    TGF_E_HIP = -3,         /* a HIP runtime call failed */
    TGF_E_NOT_SU3 = -4,     /* loaded links not in SU(3) within 1e-10, or non-finite */
    TGF_E_NONFINITE = -5,   /* a measured sum was not finite; links are undefined */
    TGF_E_STATE = -6,       /* call not valid in this state (e.g. flow before load) */
    TGF_E_UNSUPPORTED = -7  /* option not supported for this storage */
} tgf_status;

/* Device storage of the flowed links and RK accumulator. */
typedef enum {
    TGF_F64_FULL = 0,   /* FP64, all 9 complex entries (the plain path) */
    TGF_F32_FULL = 1,   /* FP32, all 9 complex entries */
    TGF_F32_C12 = 2     /* FP32, rows 0 and 1 only; row 2 = conj(row0 x row1) */
} tgf_storage;

typedef struct {
    int32_t dims[4];    /* d0, d1 (twisted plane), d2, d3; each >= 2, product <= 2^28 - 256 */
    int32_t twist[6];   /* n01, n02, n03, n12, n13, n23 in {0,1,2} */
} tgf_geom;

typedef struct {
    double t, E, t2E, plaq, Q, action;
} tgf_obs;

/* tgf_flow_params.flags */
#define TGF_NO_GRAPH 1u   /* launch kernels directly instead of a cached HIP graph
                             (always the case on the null stream) */
#define TGF_TIMING 2u     /* time every kernel with HIP events (implies NO_GRAPH) */

typedef struct {
    double eps;            /* step size, > 0 */
    const double *t_end;   /* [n_cfg] host array, t_end[c] >= current t of cfg c */
    double meas_dt;        /* measurement grid spacing; 0 = only at t_end */
    int32_t reunit_every;  /* FP32 storages: reunitarise in FP64 at the end of every R-th
                              step of each configuration, steps counted from its last
                              tgf_load_links* (or tgf_mc), so the schedule is the same
                              however a flow is split into calls (0 = never);
                              ignored for TGF_F64_FULL */
    uint32_t flags;        /* TGF_NO_GRAPH | TGF_TIMING */
} tgf_flow_params;

/* Kernel time of the last tgf_flow run with TGF_TIMING (HIP events around
 * every launch on the context's stream). */
typedef struct {
    double stage_ms;          /* total duration of the RK stage (force + update) kernels */
    int64_t stage_launches;   /* number of those launches (one per stage) */
    double stage_bytes;       /* algorithmic HBM bytes of those launches */
    double stage_site_updates;/* site-stage updates / 3 (= site-updates) */
    double measure_ms;        /* measurement + reduction kernels */
    int64_t measure_launches;
} tgf_timing;

/* Maximum rows (measurement times) one tgf_flow call can return per config. */
#define TGF_MAX_ROWS 4096

typedef struct tgf_ctx tgf_ctx;

/* Bytes of device workspace needed for n_cfg configurations with geometries
 * geoms[n_cfg] (the L x L x 3L x 3L boxes of sec. 3.1, or any extents) in
 * storage st: per site 1408 (FP64), 704 (FP32 full) or 512 (FP32 12-real)
 * bytes plus small shared tables.  Returns 0 on invalid arguments. */
size_t tgf_workspace_bytes(int32_t n_cfg, const tgf_geom *geoms, tgf_storage st);

/* Create a context for a batch of configurations (the paper's ensembles,
 * sec. 3.1 and Table A.1) with their extents and twist tensors (the twist
 * factors Z_{mu nu} of the action, sec. 3.1), over caller-owned device memory
 * workspace_dev (at least tgf_workspace_bytes, 256-byte aligned) and the HIP
 * stream hip_stream (hipStream_t; NULL = the null stream).  Configurations
 * start unloaded.  TGF_E_INVAL for bad geometry, twist, storage or pointers,
 * TGF_E_SIZE for a workspace that is too small; nothing is touched. */
tgf_status tgf_create(tgf_ctx **out, int32_t n_cfg, const tgf_geom *geoms, tgf_storage st,
                      void *workspace_dev, size_t workspace_bytes, void *hip_stream);

/* General SU(N), 2 <= nc <= 8 (sec. 1: the TGF scheme is defined for SU(N) on
 * an l^2 x (N l)^2 box whose short plane is twisted by Z_12 = exp(2 pi i k/N),
 * k coprime to N; the action, clover and charge of sec. 3.1 with N colours).
 * A context made by tgf_create_sun runs the general-N kernels (for nc = 3 as
 * well; tgf_create is the SU(3)-specialised path) and accepts every call
 * above and below with these differences:
 *   - storage must be TGF_F64_FULL (TGF_E_UNSUPPORTED otherwise);
 *   - links are complex128 [d3][d2][d1][d0][4][nc][nc] (row-major nc x nc);
 *     tgf_load_links* require SU(nc) within 1e-10 (TGF_E_NOT_SU3 otherwise);
 *   - twist entries n_{mu nu} are in 0..nc-1, Z_{mu nu} = exp(2 pi i n/nc);
 *   - sites per configuration <= 2^28 / nc^2 - 256;
 *   - plaq = (1/(6 nc V)) sum_n sum_{mu<nu} Re Tr[Z^* P], action =
 *     sum_n sum_{mu<nu} Re Tr[1 - Z^* P], force -P_ah with the trace/nc part;
 *   - the variants are the rows of each link matrix held per lane (a link
 *     spread over nc / rows lanes, rows = nc: one thread per link), and how a
 *     product reaches the rows other lanes hold: cross-lane permutes, or (the
 *     LDS-operand variant, one row per lane) a per-wave LDS copy of the right
 *     operand; tgf_set_variant accepts -1 .. tgf_sun_variant_count(nc) - 1 and
 *     tgf_autotune times them; tgf_mc and tgf_slice_charge return
 *     TGF_E_UNSUPPORTED.
 * tgf_workspace_bytes_sun returns 0 on invalid arguments. */
size_t tgf_workspace_bytes_sun(int32_t nc, int32_t n_cfg, const tgf_geom *geoms,
                               tgf_storage st);
/* Number of SU(nc) stage variants (0 for nc outside 2..8), the matrix rows
 * per lane of variant v (-1 = the default, 0; returns 0 for no such variant),
 * and whether v reads product operands from LDS (1) or through cross-lane
 * permutes (0; -1 for no such variant). */
int32_t tgf_sun_variant_count(int32_t nc);
int32_t tgf_sun_rows_per_lane(int32_t nc, int32_t variant);
int32_t tgf_sun_variant_lds(int32_t nc, int32_t variant);
tgf_status tgf_create_sun(tgf_ctx **out, int32_t nc, int32_t n_cfg, const tgf_geom *geoms,
                          tgf_storage st, void *workspace_dev, size_t workspace_bytes,
                          void *hip_stream);

/* Copy the SU(3) links U_mu(n) (sec. 3.1) of configuration cfg from
 * canonical device memory into the context's storage and set its flow time to
 * t0 (and its step count, which schedules reunitarisation, to 0).  The input is checked:
 * max |U U^+ - 1| and |det U - 1| above 1e-10 (or any non-finite entry)
 * return TGF_E_NOT_SU3 and change nothing (a configuration that was not
 * loaded stays unloaded, a loaded one keeps its links, time and step count).
 * Synchronises. */
tgf_status tgf_load_links(tgf_ctx *c, int32_t cfg, const void *links_dev, double t0);

/* Same for every configuration at once: links_dev[n_cfg] (host array of
 * device pointers), t0[n_cfg] (host).  SU(3): one launch checks and packs all
 * of them; one synchronisation.  If any link of any configuration fails the
 * check, TGF_E_NOT_SU3 names the first such configuration and no
 * configuration changes. */
tgf_status tgf_load_links_all(tgf_ctx *c, const void *const *links_dev, const double *t0);

/* Write the current (flowed) links of cfg, the field V_t of sec. 1, in
 * canonical layout (FP64; C12 rebuilds row 2): a checkpoint that
 * tgf_load_links resumes with t0.  Enqueued only; the caller synchronises
 * the stream. */
tgf_status tgf_store_links(tgf_ctx *c, int32_t cfg, void *links_dev);

/* Current flow time of cfg. */
tgf_status tgf_get_time(tgf_ctx *c, int32_t cfg, double *t);

/* Per-site densities of cfg at its current flow time (sec. 3.1, eq. gmunu and
 * eq. qlatt), FP64, canonical site order (n0 fastest), V doubles each in
 * device memory owned by the caller (either pointer may be NULL):
 *   e_dev[n] = sum_{mu<nu} Tr G_{mu nu}(n)^2, so that E = (1/V) sum_n e(n);
 *   q_dev[n] = (1/16 pi^2) Tr G G~ (n), so that Q = sum_n q(n).
 * The clover G is computed in the context's precision (FP32 for the FP32
 * storages) and each site's sum is converted to FP64.  TGF_E_STATE if cfg is
 * not loaded.  Enqueued only; the caller synchronises the stream. */
tgf_status tgf_densities(tgf_ctx *c, int32_t cfg, double *e_dev, double *q_dev);

/* Where cfg's links are stored now: *offset = byte offset within the
 * workspace, *bytes = size of that storage buffer (structure of arrays
 * [mu][entry][site], FP32 entries paired; the layout is internal to the
 * library).  For callers that checksum, snapshot or poison the stored field in
 * place; the buffer alternates with every RK stage, so the answer holds until
 * the next tgf_flow or tgf_load_links*.  TGF_E_STATE if cfg is not loaded. */
tgf_status tgf_link_buffer(tgf_ctx *c, int32_t cfg, size_t *offset, size_t *bytes);

/* Measure every loaded configuration at its current flow time: the clover
 * energy density E (eq. gmunu), t^2 E, the plaquette and action (sec. 3.1)
 * and the topological charge Q (eq. qlatt), FP64 sums: out_host[n_cfg].
 * TGF_E_STATE if a configuration is not loaded, TGF_E_NONFINITE if a sum is
 * not finite.  Synchronises. */
tgf_status tgf_measure(tgf_ctx *c, tgf_obs *out_host);

/* Flow every configuration from its current t to p->t_end[cfg] with the
 * gradient flow of the twisted Wilson action (sec. 1 and sec. 3.1, the
 * "Wilson flow discretization"; Luscher's RK3, step p->eps) -- the paper runs
 * it to sqrt(8t) = c Lt; the benchmark configurations to t = c^2 L^2 / 8 --
 * measuring as tgf_measure does.  Rows go to
 * rows_host[max_rows][n_cfg] (row-major, config fastest): a row at the start
 * time if it lies on the meas_dt grid, after every step that ends on the
 * grid, and at t_end; a configuration with fewer rows repeats its last row.
 * *n_rows = rows written.  Synchronises.  TGF_E_NONFINITE if any measured
 * sum was not finite. */
tgf_status tgf_flow(tgf_ctx *c, const tgf_flow_params *p, tgf_obs *rows_host, int32_t max_rows,
                    int32_t *n_rows);

/* Kernel timings of the last flow run with TGF_TIMING. */
tgf_status tgf_get_timing(tgf_ctx *c, tgf_timing *out);

/* max |U U^+ - 1| and max |det U - 1| over the current links of cfg (FP64
 * reduction): out[2], how far the flowed links are from SU(3) (sec. 3.1).
 * TGF_E_STATE if cfg is not loaded.  Synchronises. */
tgf_status tgf_unitarity(tgf_ctx *c, int32_t cfg, double *out);

/* Tune the stage kernel on the loaded links (stage 0 timed with HIP events,
 * links restored afterwards; the batched ensemble of the paper's Table A.1
 * mixes extents, so shapes are tuned per extent):
 *   (1) the variant, timed on the whole batch, among the XCD-ordered site and
 *       link kernels (the LDS-staged one first); a candidate replaces the
 *       current choice only when it is more than 2% faster;
 *   (2) for the LDS-staged variants, the work-group shape of each class of
 *       configurations with equal extents: whole (n0, n1) planes (the
 *       default, tgf_get_block) against 256 consecutive sites, timed on that
 *       class alone, with the same 2% rule.
 * The plaquette-sharing variants, whose rounding depends on the other
 * configurations of a work-group, are never chosen (tgf_set_variant still
 * selects them).  cache_path (may be NULL): a text file of "key value" lines
 * (one per variant choice and per class shape) read before and appended
 * after tuning.  Synchronises. */
tgf_status tgf_autotune(tgf_ctx *c, const char *cache_path);

/* Sites per work-group of the LDS-staged variants for configuration cfg
 * (64..256).  Default: whole (n0, n1) planes -- the largest multiple of
 * d0 d1 not above 256 when that is at least 128 (L = 6: 252, L = 10: 200,
 * L = 12: 144), else 256.  tgf_set_block(c, cfg, 0) restores the default.
 * Results do not depend on the shape beyond rounding order. */
tgf_status tgf_get_block(tgf_ctx *c, int32_t cfg, int32_t *sites);
tgf_status tgf_set_block(tgf_ctx *c, int32_t cfg, int32_t sites);

/* Select a stage-kernel variant by index (0 .. tgf_variant_count()-1), or
 * -1 for the built-in default ("site_lds_xcd", the LDS-staged site kernel;
 * general SU(N) contexts: variant 0). */
tgf_status tgf_set_variant(tgf_ctx *c, int32_t variant);
int32_t tgf_get_variant(tgf_ctx *c);
int32_t tgf_variant_count(void);
const char *tgf_variant_name(int32_t variant);

/* Plain device copy of bytes (16-byte aligned pointers) on hip_stream: the
 * calibration kernel for HBM counters (no counterpart in the paper).
 * TGF_E_INVAL for misaligned pointers or size.  Enqueued only. */
tgf_status tgf_stream_copy(void *dst_dev, const void *src_dev, size_t bytes, void *hip_stream);

/* Topological charge per slice of direction dir (0..3; the paper uses a long
 * direction): q_host[cfg * max_slices + s] = (1/16 pi^2) sum over the sites with
 * n_dir = s of Tr G G~ (the charge density of eq. qlatt summed over the three
 * other directions, sec. 4), for s < dims[dir]; later entries are zero.  FP64
 * sums in a fixed order.  Synchronises. */
tgf_status tgf_slice_charge(tgf_ctx *c, int32_t dir, double *q_host, int32_t max_slices);

/* Monte Carlo generation (sec. 3.1): hybrid over-relaxation of the twisted
 * Wilson action with bare coupling b = 1/lambda_0 (beta = 18 b), applied in
 * place to the current links of every configuration of the context:
 * n_hybrid times { one heat-bath sweep, then n_or over-relaxation sweeps }.
 * The paper takes n_or = Lt (the long extent) and Lt such hybrid sweeps
 * between measurements.  Updates are SU(2)-subgroup (Cabibbo-Marinari) on a
 * checkerboard; random numbers are Philox4x32-10 keyed by seed, with the
 * counter (site, sweep index, direction/subgroup/attempt, configuration
 * index); sweeps are numbered from sweep0 (heat-bath sweep of hybrid h:
 * sweep0 + h (1 + n_or)), so a chain continued with the next sweep0 is the
 * same chain.  Requires TGF_F64_FULL storage, every configuration loaded and
 * every extent even (TGF_E_INVAL / TGF_E_STATE otherwise, nothing enqueued);
 * b >= 0 finite; sweep0 + n_hybrid (1 + n_or) <= 2^32.  Afterwards every
 * configuration is at flow time 0.  Synchronises. */
tgf_status tgf_mc(tgf_ctx *c, double b, int32_t n_hybrid, int32_t n_or, uint64_t seed,
                  uint32_t sweep0);

/* --- ensemble statistics (host FP64, no device work) --------------------- */

/* Lattice normalisation N(c, Lt) of the twisted gradient-flow coupling
 * (sec. 3.1, eq. latt_norm): N^{-1} = c^4/128 sum_{mu!=nu} sum'_q
 * exp(-c^2 Lt^2 qhat^2/4) sin^2(q_nu) cos^2(q_mu/2) / qhat^2 over
 * q_mu = 2 pi n_mu / Lt, n_mu = 0..Lt-1, leaving out the momenta whose two
 * twisted-plane (directions 0, 1) components both have Lt q_i a multiple of
 * 2 pi N (n_i = 0 mod N).  Lt <= 512. */
tgf_status tgf_latt_norm(double c, int32_t Lt, int32_t N, double *out);

/* lambda_TGF = N(c, Lt) <t2E delta_Q> / (3 <delta_Q>) with delta_Q = 1 iff
 * |Q| < 0.5 (sec. 3.1, eq. lambdat_latt), over n configurations' t2E[n], Q[n]
 * at sqrt(8t) = c Lt; err (may be NULL): delete-one jackknife error.
 * TGF_E_STATE if no configuration has |Q| < 0.5. */
tgf_status tgf_coupling(const double *t2E, const double *Q, int32_t n, double c, int32_t Lt,
                        int32_t N, double *lambda, double *err);

/* C(x0) = <q(x0) q(0) delta_Q> / <delta_Q> (sec. 4, eq. qcorr), averaged over
 * the origin: q[k * ld + x] is configuration k's slice charge (x < T), Q[k] its
 * total charge; C[T] and err[T] (jackknife, may be NULL) are written. */
tgf_status tgf_charge_correlator(const double *q, const double *Q, int32_t n, int32_t T,
                                 int32_t ld, double *C, double *err);

/* Topological susceptibility chi = <Q^2> / V (sec. 4.2) over the n
 * configurations' total charges Q[n] (no sector filter), V the number of
 * sites; err (may be NULL): delete-one jackknife error (NaN for n = 1). */
tgf_status tgf_susceptibility(const double *Q, int32_t n, double V, double *chi, double *err);

/* Message of the last failing statistics call ("" if none). */
const char *tgf_stats_last_error(void);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the
 * measurement of tgf_measure (E, t2E, plaquette, Q, action; FP64) on links the
 * caller holds in canonical layout, with no context and no workspace.
 *   geom:      extents (each >= 2, at most TGF_NOALLOC_MAX_SITES sites in
 *              all, else TGF_E_SIZE) and twist (entries 0..2);
 *   links_dev: complex128 [d3][d2][d1][d0][4][3][3], device memory (not
 *              checked for SU(3));
 *   t:         flow time written to out (t2E = t^2 E), finite, >= 0;
 *   out_dev:   one tgf_obs in device memory, written by the last kernel;
 *   hip_stream: hipStream_t (NULL = the null stream) of the current device.
 * Nothing is allocated (no hipMalloc, no pinned staging): the reduction
 * partials live in a fixed device array of the library (18 MiB, one per GPU,
 * held until the process ends), fully rewritten by every call.  Calls that
 * overlap on one GPU race on that array; serialise them (one stream).
 * Arguments are checked on the host; then two kernels are enqueued and the
 * call returns without synchronising.  A non-finite sum shows as non-finite
 * entries of *out_dev (there is no status word).  The result equals that of
 * tgf_measure on a TGF_F64_FULL context holding the same links. */
#define TGF_NOALLOC_MAX_SITES 12582912
tgf_status tgf_measure_noalloc(const tgf_geom *geom, const void *links_dev, double t,
                               tgf_obs *out_dev, void *hip_stream);

/* Thread-local message of the last failing call ("" if none). */
const char *tgf_last_error(void);

/* Free host state and the cached graph; never touches caller memory. */
void tgf_destroy(tgf_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* TGF_H */
