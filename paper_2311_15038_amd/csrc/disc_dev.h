// The kept disc of container removal (Section III-B) as seen by the kernels
// that read a volume: for image row y, the run of columns [x0, x1] whose
// pixels satisfy (x - cx)^2 + (y - cy)^2 <= R^2, from the circle record
// written by vr_find_container.
#pragma once

#include "common.h"

namespace vr {
namespace disc {

// circle record fields
enum { kFound = 0, kCx = 1, kCy = 2, kR = 3, kKeepR = 4, kVotes = 5, kRadiusVotes = 6, kEdges = 7 };

struct Disc {
    int found, cx, cy;
    int64_t R2;
};

__device__ __forceinline__ Disc load_disc(const int32_t* __restrict__ rec)
{
    Disc d;
    d.found = rec[kFound];
    d.cx = rec[kCx];
    d.cy = rec[kCy];
    const int64_t R = rec[kKeepR];
    d.R2 = R * R;
    return d;
}

// floor(sqrt(h)) for 0 <= h < 2^52, exact
__device__ __forceinline__ int64_t isqrt64(int64_t h)
{
    int64_t w = (int64_t)sqrt((double)h);
    while (w * w > h) --w;
    while ((w + 1) * (w + 1) <= h) ++w;
    return w;
}

// Columns [x0, x1] of row y kept by the disc, clipped to [0, nx); x0 > x1
// when none is.  A circle that was not found keeps the whole row.
__device__ __forceinline__ void row_span(const Disc& d, int64_t y, int64_t nx, int64_t& x0, int64_t& x1)
{
    if (!d.found) {
        x0 = 0;
        x1 = nx - 1;
        return;
    }
    const int64_t dy = y - d.cy, h = d.R2 - dy * dy;
    if (h < 0) {
        x0 = 1;
        x1 = 0;
        return;
    }
    const int64_t w = isqrt64(h);
    x0 = d.cx - w < 0 ? 0 : d.cx - w;
    x1 = d.cx + w > nx - 1 ? nx - 1 : d.cx + w;
}

}  // namespace disc
}  // namespace vr
