// noalloc.hip -- tgf_measure_noalloc: the measurement of tgf_measure (clover
// E, t^2 E, plaquette, Q and action of eq. gmunu / eq. qlatt, sec. 3.1) on
// caller links in canonical layout, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).  No context and no workspace: the per-tile reduction
// partials live in `scratch`, a file-scope device array of fixed size that
// every GPU the library runs on holds until the process ends.
//
// The kernels are the ones of the context path (measure_dev.h) with a
// canonical-layout link accessor; the partials have the same (tile, pair)
// layout and are summed in the same order, so the result equals that of
// tgf_measure on a TGF_F64_FULL context holding the same links.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "../../include/tgf.h"
#include "launch.h"
#include "lattice_dev.h"
#include "layout.h"
#include "measure_dev.h"

namespace tgf {

constexpr int kNoallocMaxTiles = TGF_NOALLOC_MAX_SITES / kTile;
constexpr size_t kScratchDoubles = (size_t)kNoallocMaxTiles * 3 * 4;   // [tile][pair][4]

// Reduction partials of tgf_measure_noalloc (18 MiB).  In host code this name
// is a host-side stand-in: only the address from hipGetSymbolAddress may be
// passed to kernels or copies.
static __device__ __align__(256) double scratch[kScratchDoubles];

// Canonical caller links: complex128 [site][mu][3][3].
struct CanonLinks {
    const double2 *p;
    __device__ __forceinline__ M3<double> operator()(int mu, int i) const {
        const double2 *s = p + ((size_t)i * 4 + mu) * 9;
        M3<double> U;
#pragma unroll
        for (int e = 0; e < 9; e++) U.e[e / 3][e % 3] = {s[e].x, s[e].y};
        return U;
    }
};

// One work-group per tile of 64 sites, one wave per dual plane pair; the
// wave's FP64 sums go to partials[tile][pair][4] (as measure_kernel).
__global__ __launch_bounds__(192) void measure_canon_kernel(CfgDesc c, const double2 *links,
                                                            double *partials) {
    const int tile = blockIdx.x;
    const int pair = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tb = tile * kTile;                               // site of lane 0
    const int i = tb + (threadIdx.x & 63);
    double v[4] = {0, 0, 0, 0};
    if (i < c.V) {
        const CanonLinks W{links};
        const Geo g = make_geo(c, i);
        const int nw = min(kTile, c.V - tb);
        switch (pair) {
            case 0: measure_pair<double, 0>(W, c, g, v, tb, nw); break;
            case 1: measure_pair<double, 1>(W, c, g, v, tb, nw); break;
            default: measure_pair<double, 2>(W, c, g, v, tb, nw); break;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = wave_sum(v[k]);
    if ((threadIdx.x & 63) == 0) {
        double *o = partials + ((size_t)tile * 3 + pair) * 4;
        o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    }
}

// One work-group: the fixed-order sum of the n_tiles x 3 partials, written as
// one tgf_obs {t, E, t^2 E, plaq, Q, action} to out.
__global__ __launch_bounds__(256) void finalize_canon_kernel(int V, int n_tiles, double t,
                                                             const double *partials,
                                                             double *out) {
    double tot[4];
    sum_tile_partials(partials, 0, n_tiles * 3, tot);
    if (threadIdx.x == 0) {
        const double E = tot[0] / (double)V;
        out[0] = t;
        out[1] = E;
        out[2] = t * t * E;
        out[3] = tot[2] / (6.0 * 3 * (double)V);
        out[4] = tot[1];
        out[5] = tot[3];
    }
}

namespace {

constexpr int kMaxDevices = 64;
double *g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device, looked up once per
// device (each GPU holds its own copy at its own address).
hipError_t scratch_ptr(double **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = (double *)p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

tgf_status nfail(tgf_status s, const std::string &msg) {
    set_last_error(msg.c_str());
    return s;
}

}  // namespace
}  // namespace tgf

using namespace tgf;

extern "C" tgf_status tgf_measure_noalloc(const tgf_geom *geom, const void *links_dev, double t,
                                          tgf_obs *out_dev, void *hip_stream) {
    set_last_error("");
    if (!geom || !links_dev || !out_dev) return nfail(TGF_E_INVAL, "NULL argument");
    if (!std::isfinite(t) || t < 0) return nfail(TGF_E_INVAL, "t must be finite and >= 0");
    long long V = 1;
    for (int m = 0; m < 4; m++) {
        if (geom->dims[m] < 2) return nfail(TGF_E_INVAL, "dims must be >= 2");
        V *= geom->dims[m];
        if (V > TGF_NOALLOC_MAX_SITES)
            return nfail(TGF_E_SIZE, "more than TGF_NOALLOC_MAX_SITES sites");
    }
    for (int k = 0; k < 6; k++)
        if (geom->twist[k] < 0 || geom->twist[k] > 2)
            return nfail(TGF_E_INVAL, "twist entries must be in 0..2");
    double *part = nullptr;
    hipError_t e = scratch_ptr(&part);
    if (e != hipSuccess)
        return nfail(TGF_E_HIP, std::string("scratch address: ") + hipGetErrorString(e));
    CfgDesc c{};
    for (int m = 0; m < 4; m++) c.d[m] = geom->dims[m];
    for (int k = 0; k < 6; k++) c.tw[k] = geom->twist[k];
    c.V = (int)V;
    const int n_tiles = (int)((V + kTile - 1) / kTile);
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(measure_canon_kernel, dim3(n_tiles), dim3(192), 0, s, c,
                       (const double2 *)links_dev, part);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(finalize_canon_kernel, dim3(1), dim3(256), 0, s, (int)V, n_tiles, t,
                           (const double *)part, (double *)out_dev);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return nfail(TGF_E_HIP, std::string("launch: ") + hipGetErrorString(e));
    return TGF_OK;
}
