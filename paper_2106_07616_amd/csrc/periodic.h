// Device-side construction of periodic clouds (Sec. 3.1): the bounding box,
// the ghost images within a band of the periodic faces, the check that every
// cloud lies within the band, and the map from image rows back to points.
#pragma once

#include "internal.h"

namespace rbffd {

// Bounding box of xyz [n][dim], copied to the host; E_ARG for non-finite
// coordinates.
int device_bbox(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, double *lo, double *hi, hipStream_t s);

// Shift m[k] moves a point by +L, -L or 0 along each axis; an image is kept
// when it lies within band of the box [lo, hi] along every periodic axis
// (L > 0).
struct PeriodicShifts {
    int count = 0;
    int m[26][3] = {};
    double L[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    double band = 0.0;
};

// The points followed by their kept images, shift by shift in order and point
// by point within a shift: *aug [*naug][dim] and *owner [*naug] (the point each
// row stands for), both allocated from the context (abytes, obytes to free).
int launch_periodic_images(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, const PeriodicShifts &P,
                           double **aug, int32_t **owner, int64_t *naug, size_t *abytes, size_t *obytes,
                           hipStream_t s);

// Queries of a periodic cloud, in place: a coordinate outside [lo, lo + L)
// along a periodic axis becomes lo + r, r = fmod(x - lo, L) taken into
// [0, L); margin[t] is then the query's largest distance outside the box
// [lo, hi] along an axis (0 inside). *nonfinite (device int, cleared here)
// becomes 1 for a non-finite coordinate.
int launch_periodic_wrap(int dim, int64_t nq, double *qxyz, const PeriodicShifts &P, double *margin, int *nonfinite,
                         hipStream_t s);

// *outside (device int, cleared here) becomes 1 when some query's q-th
// neighbour among the aug rows lies farther than band, less the query's
// margin when margin is not null.
int launch_periodic_inside(int dim, int64_t nq, const double *qxyz, const double *aug, int q, const int32_t *nbr,
                           double band, const double *margin, int *outside, hipStream_t s);

// nbr[i][a] = owner[nbr[i][a]]; *first_dup (device, set to INT64_MAX here)
// becomes the lowest point whose cloud then holds one point twice.
int launch_periodic_remap(int64_t n, int q, const int32_t *owner, int32_t *nbr, int64_t *first_dup,
                          hipStream_t s);

}  // namespace rbffd
