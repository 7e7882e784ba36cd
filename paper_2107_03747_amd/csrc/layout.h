// layout.h -- device-side layout of a flow context (host and device code).
//
// Every configuration c owns, inside the caller's workspace:
//   W[0], W[1]  ping-pong link buffers, structure of arrays
//               [mu (4)][entry (NE)][site (stride)] of complex R, where NE = 9
//               (full storage, row-major entries) or 6 (rows 0 and 1 only);
//               FP32 pairs the entries, [mu][pair][site][2] (12-real: 3
//               pairs; full: 4 pairs and entry 8 alone, [mu][8][site]), so
//               that one 16-byte access moves two complex numbers
//               (entry_index);
//   X           RK accumulator [mu (4)][slot (4)][site (stride)] of complex R:
//               slots 0..2 = X01, X02, X12, slot 3 = (Im X00, Im X11); FP32
//               pairs the slots, [mu][pair (2)][site][2].
// Bytes per site: FP64 full 2 x 576 + 256 = 1408, FP32 full 2 x 288 + 128 =
// 704, FP32 12-real 2 x 192 + 128 = 512.
// `stride` is the site count rounded up to a multiple of 256 so that every
// entry plane starts 256-byte aligned and a wavefront's 64 consecutive sites
// read 64 consecutive complex numbers (fully coalesced).
//
// Shared regions: the descriptor table, the per-block reduction partials
// (4 doubles per block: e, q, plaq, action), the FP64 observable rows, the
// flow schedule and a status word.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace tgf {

constexpr int kBlock = 256;          // threads per work-group for site kernels
constexpr int kMaxRows = 4096;       // rows per flow call (TGF_MAX_ROWS)

struct CfgDesc {
    int32_t d[4];         // extents
    int32_t V;            // sites
    int32_t stride;       // site stride of an entry plane
    int32_t tw[6];        // twist n01 n02 n03 n12 n13 n23 (0..2)
    int32_t user;         // index of this config in the caller's order
    int32_t cur;          // which W buffer holds the links at step 0 of this flow
    int32_t n_full;       // full steps of size eps this flow
    int32_t n_steps;      // n_full + (short final step ? 1 : 0)
    int32_t reunit_phase; // steps since the load, before this flow, mod reunit_every
    int32_t blk;          // sites per work-group of the LDS-staged stage variants (<= 256)
    int32_t chunk;        // their launch order: 0 = site order, else columns of chunk blocks
    double eps_last;      // size of the short final step (0 if none)
    double t0;            // flow time at the start of this flow
    void *W[2];
    void *X;
};

// Index (in complex elements) of entry e of link (mu, site i) in a link buffer.
template <class R, int NE>
__host__ __device__ inline size_t entry_index(int mu, int e, int stride, int i) {
    if (sizeof(R) == 4 && e < 8) {
        const size_t base = (size_t)(mu * NE) * stride;   // direction mu starts here
        return base + (((size_t)(e >> 1) * stride + i) << 1) + (e & 1);
    }
    return (size_t)(mu * NE + e) * stride + i;
}

// Per-measurement-event schedule entry for one config (exec order).
struct MeasSlot {
    int32_t row;          // output row, or -1 when this config is not measured
    int32_t pad;
    double t;             // flow time of the measurement
};

}  // namespace tgf
