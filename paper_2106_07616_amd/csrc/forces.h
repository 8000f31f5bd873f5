// Surface forces on a cylinder (Sec. 4, Eqs. cylinder forces and cylinder
// stress): the device part of rbffd_cylinder_forces.
#pragma once

#include "internal.h"

namespace rbffd {

// Traction sigma . n at ns surface points from fld [5][ns] (p, du/dx, du/dy,
// dv/dx, dv/dy) and cs [2][ns] (cos t, sin t); force [2] = scale times the
// Simpson sum of the traction (weights 2, 4, 2, 4, ...); trac [2][ns] optional.
int launch_surface_traction(int ns, const double *fld, const double *cs, double mu, double scale, double *trac,
                            double *force, hipStream_t s);

}  // namespace rbffd
