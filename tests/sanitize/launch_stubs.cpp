// Stand-ins for the device launchers of libtgf (test infrastructure): the
// host-side sanitizer build of the runtime links these instead of the
// kernels.  Every one reports that no device is there; the driver only takes
// paths that return before any launch.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace tgf {

const char *variant_name(int) { return "stub"; }
hipError_t launch_stage(int, Prec, bool, hipStream_t, const CfgDesc *, const int *, int, int,
                        const int *, int, int, int, double, int) {
    return hipErrorNoDevice;
}
hipError_t launch_measure(Prec, bool, hipStream_t, const CfgDesc *, const int *, int, int,
                          const MeasSlot *, double *, int) {
    return hipErrorNoDevice;
}
hipError_t launch_finalize(hipStream_t, const CfgDesc *, const int *, int, const MeasSlot *,
                           const double *, double *, int, int *, int) {
    return hipErrorNoDevice;
}
hipError_t launch_unpack(Prec, bool, hipStream_t, const void *, void *, int, int) {
    return hipErrorNoDevice;
}
hipError_t launch_check(Prec, bool, hipStream_t, const void *, int, int, double *, double *) {
    return hipErrorNoDevice;
}
hipError_t launch_ingest_batch(Prec, bool, hipStream_t, const void *, const CfgDesc *,
                               const int *, int, int, double *, double *) {
    return hipErrorNoDevice;
}
hipError_t launch_check_final(hipStream_t, const double *, int, double *) {
    return hipErrorNoDevice;
}
hipError_t launch_slice_charge(Prec, bool, hipStream_t, const CfgDesc *, int, int, int, int,
                               double *, double *) {
    return hipErrorNoDevice;
}
hipError_t launch_densities(Prec, bool, hipStream_t, const CfgDesc *, int, int, double *,
                            double *) {
    return hipErrorNoDevice;
}
hipError_t launch_mc(hipStream_t, const CfgDesc *, const int *, int, int, int, int, int, double,
                     uint64_t, uint32_t) {
    return hipErrorNoDevice;
}
int sun_variant_count(int nc) { return nc >= 2 && nc <= 8 ? 2 : 0; }
int sun_rows_per_lane(int nc, int v) { return (nc >= 2 && nc <= 8 && v >= -1 && v < 2) ? nc : 0; }
int sun_variant_lds(int nc, int v) { return (nc >= 2 && nc <= 8 && v >= -1 && v < 2) ? (v == 1) : -1; }
hipError_t launch_stage_sun(int, int, hipStream_t, const CfgDesc *, const int *, int, int, int,
                            int, double) {
    return hipErrorNoDevice;
}
hipError_t launch_measure_sun(int, int, hipStream_t, const CfgDesc *, const int *, int, int,
                              const MeasSlot *, double *, int) {
    return hipErrorNoDevice;
}
hipError_t launch_pack_sun(int, hipStream_t, const void *, void *, int, int) {
    return hipErrorNoDevice;
}
hipError_t launch_unpack_sun(int, hipStream_t, const void *, void *, int, int) {
    return hipErrorNoDevice;
}
hipError_t launch_check_sun(int, bool, hipStream_t, const void *, int, int, double *, double *) {
    return hipErrorNoDevice;
}
hipError_t launch_fill_int(hipStream_t, int *, int, int) { return hipErrorNoDevice; }
hipError_t launch_copy(hipStream_t, void *, const void *, size_t) { return hipErrorNoDevice; }

}  // namespace tgf
