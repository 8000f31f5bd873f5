// Forces on a circular cylinder from its surface stresses (Sec. 4, Eqs.
// cylinder forces, cylinder stress and cylinder lift drag).
//
// The host entry point differentiates the velocity with the cloud's d/dx and
// d/dy operators and interpolates the pressure and the four strain rates to
// uniform points on the circle. The one-block kernel here then forms the
// stress at each surface point, its traction on the normal (cos t, sin t) that
// points from the cylinder into the fluid, and the composite Simpson sum of
// the traction over the closed curve.
//
// The work is a few hundred points: one block of kBlock threads, with a
// fixed-order block sum so that the result is the same run to run.
#include "forces.h"

namespace rbffd {

namespace {

// fld:   [5][ns] pressure, du/dx, du/dy, dv/dx, dv/dy at the surface points
// cs:    [2][ns] cos t_j and sin t_j
// trac:  optional [2][ns] traction sigma . n
// force: [2] scale * sum_j c_j trac_j, c_j = 2 at even j and 4 at odd j
__global__ __launch_bounds__(kBlock) void surface_traction(int ns, const double *__restrict__ fld,
                                                           const double *__restrict__ cs, double mu, double scale,
                                                           double *__restrict__ trac, double *__restrict__ force)
{
    __shared__ double lds[kBlock / 64];
    double sx = 0.0, sy = 0.0;
    for (int j = threadIdx.x; j < ns; j += kBlock) {
        const double p = fld[j], ux = fld[ns + j], uy = fld[2 * ns + j];
        const double vx = fld[3 * ns + j], vy = fld[4 * ns + j];
        const double c = cs[j], s = cs[ns + j];
        const double sxx = -p + 2.0 * mu * ux;
        const double syy = -p + 2.0 * mu * vy;
        const double sxy = mu * (uy + vx);
        const double tx = sxx * c + sxy * s;
        const double ty = sxy * c + syy * s;
        if (trac) {
            trac[j] = tx;
            trac[ns + j] = ty;
        }
        // the curve's end point repeats its start, so the Simpson weights
        // alternate 2, 4 around the whole curve
        const double wgt = (j & 1) ? 4.0 : 2.0;
        sx += wgt * tx;
        sy += wgt * ty;
    }
    const double fx = block_sum(sx, lds);
    const double fy = block_sum(sy, lds);
    if (threadIdx.x == 0) {
        force[0] = scale * fx;
        force[1] = scale * fy;
    }
}

}  // namespace

int launch_surface_traction(int ns, const double *fld, const double *cs, double mu, double scale, double *trac,
                            double *force, hipStream_t s)
{
    if (ns <= 0) return fail(RBFFD_E_ARG, "no surface points");
    hipLaunchKernelGGL(surface_traction, dim3(1), dim3(kBlock), 0, s, ns, fld, cs, mu, scale, trac, force);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

}  // namespace rbffd
