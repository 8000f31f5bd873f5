// One BDF time step of the semi-implicit outer iteration (Sec. 3, Eqs. u:n+1
// ... p:correction, Eq. normal momentum, and the step list of Sec. 3.2), and
// the Courant-number eigenvalue estimate of Sec. 3.2.
//
// Per outer iteration: momentum matrix + right-hand sides (one streaming pass
// over the stored operators), d-right-hand-side BiCGSTAB sharing each matrix
// pass, divergence right-hand side, pressure-correction BiCGSTAB, interior
// pressure update, boundary-pressure block solve, velocity correction fused
// with the change Delta. Only Delta (8 bytes) returns to the host per
// iteration.
#include <cmath>
#include <vector>

#include "internal.h"

namespace rbffd {

namespace {

__device__ inline int lb() { return xcd_block(gridDim.x); }

inline int blocks_for(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b >= 64) b = (b + 7) / 8 * 8;   // whole rows per thread; multiple of 8 for the XCD mapping
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (int)std::max<int64_t>(1, b);
}

// constant body force per unit volume (the mean pressure gradient of a periodic
// channel), passed by value
struct Force3 {
    double v[3];
};

// u^r = u^n with the Dirichlet values of t^{n+1} on velocity-prescribed points; p^r = p^n
__global__ void k_start(int64_t n, int dim, const uint8_t *__restrict__ kind, const double *__restrict__ u,
                        const double *__restrict__ ubc, const double *__restrict__ p, double *__restrict__ ur,
                        double *__restrict__ pr)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool b = kind[i] == RBFFD_DIRICHLET || kind[i] == RBFFD_PRESCRIBED_PRESSURE;
    for (int e = 0; e < dim; ++e) ur[e * n + i] = b ? ubc[e * n + i] : u[e * n + i];
    pr[i] = p[i];
}

// Momentum matrix (Eqs. u:tilde, v:tilde, with u^r linearising advection):
//   interior:  M_ij = rho a1/dt d_ij + rho sum_e u^r_e,i D_e,ij - mu L_ij
//              b_e,i = -rho (a2 u^n_e,i + a3 u^{n-1}_e,i)/dt - (D_e p^r)_i
//   velocity-prescribed boundary:  identity row, b_e,i = u_bc,e,i
//   outlet and symmetry:  zero normal derivative (Sec. 3.1),
//              M_ij = sum_d N_d D_d,ij, b_e,i = 0 (the normal component of a
//              symmetry point is switched to u = 0 per solve by k_sym_rows)
// With `cd` set it writes instead C = -rho (u . grad) + mu L on interior rows and
// zero rows on the boundary (the convection-diffusion operator of Sec. 3.2).
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_momentum(int64_t n, int q, const int32_t *__restrict__ col,
                                                     const double *__restrict__ val, int64_t vs,
                                                     const uint8_t *__restrict__ kind,
                                                     const double *__restrict__ normal, const double *__restrict__ ur,
                                                     const double *__restrict__ un, const double *__restrict__ up,
                                                     const double *__restrict__ ubc, const double *__restrict__ pr,
                                                     double rho, double mu, double dt, double a1, double a2, double a3,
                                                     Force3 f, int cd, double *__restrict__ mval,
                                                     double *__restrict__ mdinv, double *__restrict__ bm)
{
    const int64_t i = (int64_t)lb() * kBlock + threadIdx.x;
    if (i >= pad64(n)) return;
    const int64_t base = ((i >> 6) * (int64_t)q) * 64 + (i & 63);
    if (i >= n) {
        for (int a = 0; a < q; ++a) mval[base + (int64_t)a * 64] = 0.0;
        mdinv[i] = 0.0;
        return;
    }
    if ((kind[i] == RBFFD_OUTLET || kind[i] == RBFFD_SYMMETRY) && !cd) {
        double diag = 0.0;
        for (int a = 0; a < q; ++a) {
            const int64_t slot = base + (int64_t)a * 64;
            double v = 0.0;
            for (int d = 0; d < DIM; ++d) v = fma(normal[i * DIM + d], val[d * vs + slot], v);
            mval[slot] = v;
            if (col[slot] == i) diag += v;
        }
        mdinv[i] = (diag != 0.0) ? 1.0 / diag : 1.0;
        for (int e = 0; e < DIM; ++e) bm[e * n + i] = 0.0;
        return;
    }
    if (kind[i] != RBFFD_INTERIOR) {
        for (int a = 0; a < q; ++a) {
            const int64_t slot = base + (int64_t)a * 64;
            mval[slot] = (!cd && col[slot] == i) ? 1.0 : 0.0;
        }
        mdinv[i] = 1.0;
        if (!cd)
            for (int e = 0; e < DIM; ++e) bm[e * n + i] = ubc[e * n + i];
        return;
    }
    double uc[DIM];
    for (int e = 0; e < DIM; ++e) uc[e] = ur[e * n + i];
    const double mass = rho * a1 / dt;
    double g[DIM];
    for (int e = 0; e < DIM; ++e) g[e] = 0.0;
    double diag = 0.0;
    for (int a = 0; a < q; ++a) {
        const int64_t slot = base + (int64_t)a * 64;
        const int32_t c = col[slot];
        double conv = 0.0;
        for (int e = 0; e < DIM; ++e) conv = conv + uc[e] * val[e * vs + slot];
        double v;
        if (cd) {
            v = -rho * conv + mu * val[DIM * vs + slot];
        } else {
            v = rho * conv - mu * val[DIM * vs + slot];
            if (c == i) v = v + mass;
            const double pc = pr[c];
            for (int e = 0; e < DIM; ++e) g[e] = fma(val[e * vs + slot], pc, g[e]);
        }
        mval[slot] = v;
        if (c == i) diag += v;
    }
    mdinv[i] = (diag != 0.0) ? 1.0 / diag : 1.0;
    if (!cd)
        for (int e = 0; e < DIM; ++e)
            bm[e * n + i] = -rho * (a2 * un[e * n + i] + a3 * up[e * n + i]) / dt - g[e] + f.v[e];
}

// Symmetry rows of the momentum matrix for velocity component e (Sec. 3.1):
// u_e = 0 where e is the normal axis of the point's plane, N . grad u_e = 0
// otherwise. The right-hand side stays 0 on both.
// The component that carries u . n = 0 at a symmetry point: the largest |n_s|,
// the lowest index on ties.
template <int DIM>
__device__ inline int sym_component(const double *nv)
{
    int sc = 0;
#pragma unroll
    for (int d = 1; d < DIM; ++d)
        if (fabs(nv[d]) > fabs(nv[sc])) sc = d;
    return sc;
}

// Momentum rows of component e at symmetry points (Sec. 3.1: no flow through
// the plane, no normal derivative of the tangential velocity). With the unit
// normal n, component s takes u . n = 0 as the row n_s u_s; every other
// component a takes the tangent t_a = e_a - n_a n as the row
// (1 - n_a^2) N.grad u_a. A normal along an axis gives u_s = 0 and N.grad u_a
// = 0 (unit scale). The other components enter the right-hand side (k_sym_rhs).
template <int DIM>
__global__ void k_sym_rows(int64_t n, int q, const int32_t *__restrict__ col, const double *__restrict__ val,
                           int64_t vs, const uint8_t *__restrict__ kind, const double *__restrict__ normal, int e,
                           double *__restrict__ mval, double *__restrict__ mdinv)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || kind[i] != RBFFD_SYMMETRY) return;
    const int64_t base = ((i >> 6) * (int64_t)q) * 64 + (i & 63);
    const double *nv = normal + i * DIM;
    const int sc = sym_component<DIM>(nv);
    const bool axis = fabs(nv[sc]) == 1.0;
    const double scale = (e == sc) ? (axis ? 1.0 : nv[sc]) : (axis ? 1.0 : 1.0 - nv[e] * nv[e]);
    double diag = 0.0;
    for (int a = 0; a < q; ++a) {
        const int64_t slot = base + (int64_t)a * 64;
        double v;
        if (e == sc) {
            v = (col[slot] == i) ? scale : 0.0;
        } else {
            v = 0.0;
            for (int d = 0; d < DIM; ++d) v = fma(nv[d], val[d * vs + slot], v);
            v = scale * v;
        }
        mval[slot] = v;
        if (col[slot] == i) diag += v;
    }
    mdinv[i] = (diag != 0.0) ? 1.0 / diag : 1.0;
}

// Right-hand side of component e at symmetry points with a normal off the
// axes: -sum_{d != s} n_d u_d for the normal component s, and
// sum_{d != e} n_e n_d (N.grad u_d) for a tangential one, the other
// components at the outer iterate ur [DIM][n]. Axis normals keep 0.
template <int DIM>
__global__ void k_sym_rhs(int64_t n, int q, const int32_t *__restrict__ col, const double *__restrict__ val,
                          int64_t vs, const uint8_t *__restrict__ kind, const double *__restrict__ normal,
                          const double *__restrict__ ur, int e, double *__restrict__ b)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n || kind[i] != RBFFD_SYMMETRY) return;
    const double *nv = normal + i * DIM;
    const int sc = sym_component<DIM>(nv);
    if (fabs(nv[sc]) == 1.0) return;
    double r = 0.0;
    if (e == sc) {
        for (int d = 0; d < DIM; ++d)
            if (d != sc) r = r - nv[d] * ur[d * n + i];
    } else {
        const int64_t base = ((i >> 6) * (int64_t)q) * 64 + (i & 63);
        for (int d = 0; d < DIM; ++d) {
            if (d == e) continue;
            double g = 0.0;   // (N . grad u_d)(x_i) at the iterate
            for (int a = 0; a < q; ++a) {
                const int64_t slot = base + (int64_t)a * 64;
                double w = 0.0;
                for (int c = 0; c < DIM; ++c) w = fma(nv[c], val[c * vs + slot], w);
                g = fma(w, ur[d * n + col[slot]], g);
            }
            r = r + nv[e] * nv[d] * g;
        }
    }
    b[i] = r;
}

// f_i = (rho a1 / dt) sum_e (D_e u~_e)_i on interior rows other than the pin; 0 elsewhere
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_div_rhs(int64_t n, int q, const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, int64_t vs,
                                                    const uint8_t *__restrict__ kind, int64_t pin,
                                                    const double *__restrict__ ut, double coef, double *__restrict__ f)
{
    const int64_t i = (int64_t)lb() * kBlock + threadIdx.x;
    if (i >= n) return;
    if (kind[i] != RBFFD_INTERIOR || i == pin) {
        f[i] = 0.0;
        return;
    }
    const int64_t base = ((i >> 6) * (int64_t)q) * 64 + (i & 63);
    double dv = 0.0;
    for (int e = 0; e < DIM; ++e) {
        double s = 0.0;
        for (int a = 0; a < q; ++a) {
            const int64_t slot = base + (int64_t)a * 64;
            s = fma(val[e * vs + slot], ut[e * n + col[slot]], s);
        }
        dv = dv + s;
    }
    f[i] = coef * dv;
}

// p_a = p^r + p' on interior points, the prescribed value on prescribed-pressure
// points, p^r on velocity-Dirichlet points (replaced by the normal-momentum solve)
__global__ void k_p_interior(int64_t n, const uint8_t *__restrict__ kind, const double *__restrict__ pr,
                             const double *__restrict__ pc, const double *__restrict__ pbc, double *__restrict__ pa)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int kd = kind[i];
    pa[i] = (kd == RBFFD_INTERIOR) ? pr[i] + pc[i]
                                   : ((kd == RBFFD_PRESCRIBED_PRESSURE || kd == RBFFD_OUTLET) ? pbc[i] : pr[i]);
}

// Boundary-pressure right-hand side (Eq. normal momentum) for boundary row b:
//   R_b = sum_c N_c [ -rho (a1 u~_c + a2 u^n_c + a3 u^{n-1}_c)/dt - rho (u~ . grad) u~_c + mu L u~_c ]_b
//         - sum_{j not velocity-Dirichlet} G_bj p_a,j
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_boundary_rhs(int64_t n, int64_t nb, int q, const int32_t *__restrict__ col,
                                                         const double *__restrict__ val, int64_t vs,
                                                         const double *__restrict__ pval,
                                                         const uint8_t *__restrict__ kind,
                                                         const double *__restrict__ normal,
                                                         const int32_t *__restrict__ bidx, const double *__restrict__ ut,
                                                         const double *__restrict__ un, const double *__restrict__ up,
                                                         const double *__restrict__ pa, const double *__restrict__ pr,
                                                         double rho, double mu, double dt, double a1, double a2,
                                                         double a3, Force3 f, double *__restrict__ bb,
                                                         double *__restrict__ pb)
{
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int64_t i = bidx[b];
    const int64_t base = ((i >> 6) * (int64_t)q) * 64 + (i & 63);
    double grad[DIM][DIM], lap[DIM], off = 0.0;
    for (int c = 0; c < DIM; ++c) {
        lap[c] = 0.0;
        for (int g = 0; g < DIM; ++g) grad[g][c] = 0.0;
    }
    for (int a = 0; a < q; ++a) {
        const int64_t slot = base + (int64_t)a * 64;
        const int32_t j = col[slot];
        for (int c = 0; c < DIM; ++c) {
            const double uj = ut[c * n + j];
            for (int g = 0; g < DIM; ++g) grad[g][c] = fma(val[g * vs + slot], uj, grad[g][c]);
            lap[c] = fma(val[DIM * vs + slot], uj, lap[c]);
        }
        if (!neumann_p(kind[j])) off = fma(pval[slot], pa[j], off);
    }
    double rhs = 0.0;
    for (int c = 0; c < DIM; ++c) {
        const double dudt = rho * (a1 * ut[c * n + i] + a2 * un[c * n + i] + a3 * up[c * n + i]) / dt;
        double adv = 0.0;
        for (int g = 0; g < DIM; ++g) adv = adv + ut[g * n + i] * grad[g][c];
        const double comp = -dudt - rho * adv + mu * lap[c] + f.v[c];
        rhs = rhs + normal[i * DIM + c] * comp;
    }
    bb[b] = rhs - off;
    pb[b] = pr[i];
}

__global__ void k_p_scatter(int64_t n, const uint8_t *__restrict__ kind, const int32_t *__restrict__ bpos,
                            const double *__restrict__ pa, const double *__restrict__ pb, double *__restrict__ pr)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    pr[i] = neumann_p(kind[i]) ? pb[bpos[i]] : pa[i];
}

// u^{r+1} = u~ - coef D p' on interior points (Eqs. u:correction, v:correction),
// u~ on boundary points; partials of sum_i |u^{r+1}_e - u^r_e| per component.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_correct(int64_t n, int q, const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, int64_t vs,
                                                    const uint8_t *__restrict__ kind, const double *__restrict__ pc,
                                                    const double *__restrict__ ut, const double *__restrict__ ur,
                                                    double coef, double *__restrict__ unew, double *__restrict__ part)
{
    __shared__ double lds[kBlock / 64];
    double acc[DIM];
    for (int e = 0; e < DIM; ++e) acc[e] = 0.0;
    for (int64_t i = (int64_t)lb() * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        if (kind[i] != RBFFD_INTERIOR) {
            for (int e = 0; e < DIM; ++e) {
                const double v = ut[e * n + i];
                unew[e * n + i] = v;
                acc[e] += fabs(v - ur[e * n + i]);
            }
            continue;
        }
        const int64_t base = ((i >> 6) * (int64_t)q) * 64 + (i & 63);
        double g[DIM];
        for (int e = 0; e < DIM; ++e) g[e] = 0.0;
        for (int a = 0; a < q; ++a) {
            const int64_t slot = base + (int64_t)a * 64;
            const double pj = pc[col[slot]];
            for (int e = 0; e < DIM; ++e) g[e] = fma(val[e * vs + slot], pj, g[e]);
        }
        for (int e = 0; e < DIM; ++e) {
            const double v = ut[e * n + i] - coef * g[e];
            unew[e * n + i] = v;
            acc[e] += fabs(v - ur[e * n + i]);
        }
    }
    for (int e = 0; e < DIM; ++e) {
        const double s = block_sum(acc[e], lds);
        if (threadIdx.x == 0) part[e * kMaxBlocks + blockIdx.x] = s;
    }
}

// partials of sum_i |a_e - b_e|
__global__ __launch_bounds__(kBlock) void k_absdiff(int64_t n, int dim, const double *__restrict__ a,
                                                    const double *__restrict__ b, double *__restrict__ part)
{
    __shared__ double lds[kBlock / 64];
    for (int e = 0; e < dim; ++e) {
        double acc = 0.0;
        for (int64_t i = (int64_t)lb() * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
            acc += fabs(a[e * n + i] - b[e * n + i]);
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0) part[e * kMaxBlocks + blockIdx.x] = s;
    }
}

// Discrete continuity error of the new velocity: per-block sums of
// |sum_e (D_e u_e)_i| and of the count over interior points i (Eq.
// continuity:n+1), in part[0..] and part[kMaxBlocks..].
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_div_abs(int64_t n, int q, const int32_t *__restrict__ col,
                                                    const double *__restrict__ val, int64_t vs,
                                                    const uint8_t *__restrict__ kind, const double *__restrict__ u,
                                                    double *__restrict__ part)
{
    __shared__ double lds[kBlock / 64];
    double acc = 0.0, cnt = 0.0;
    for (int64_t i = (int64_t)lb() * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        if (kind[i] != RBFFD_INTERIOR) continue;
        const int64_t base = ((i >> 6) * (int64_t)q) * 64 + (i & 63);
        double dv = 0.0;
        for (int e = 0; e < DIM; ++e) {
            double s = 0.0;
            for (int a = 0; a < q; ++a) {
                const int64_t slot = base + (int64_t)a * 64;
                s = fma(val[e * vs + slot], u[e * n + col[slot]], s);
            }
            dv = dv + s;
        }
        acc += fabs(dv);
        cnt += 1.0;
    }
    const double sa = block_sum(acc, lds), sc = block_sum(cnt, lds);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sa;
        part[kMaxBlocks + blockIdx.x] = sc;
    }
}

__global__ __launch_bounds__(kBlock) void k_finish_ratio(const double *__restrict__ part, int np,
                                                         double *__restrict__ out)
{
    __shared__ double lds[kBlock / 64];
    const double a = sum_partials(part, np, lds);
    const double c = sum_partials(part + kMaxBlocks, np, lds);
    if (threadIdx.x == 0) out[0] = (c > 0.0) ? a / c : 0.0;
}

// out[0] = sum_e S_e / n (Delta); out[1] = max_e S_e / n / dt (steady rate)
__global__ __launch_bounds__(kBlock) void k_finish_sums(const double *__restrict__ part, int np, int dim, int64_t n,
                                                        double dt, double *__restrict__ out)
{
    __shared__ double lds[kBlock / 64];
    double tot = 0.0, mx = 0.0;
    for (int e = 0; e < dim; ++e) {
        const double s = sum_partials(part + e * kMaxBlocks, np, lds) / (double)n;
        tot += s;
        mx = fmax(mx, s / dt);
    }
    if (threadIdx.x == 0) {
        out[0] = tot;
        out[1] = mx;
    }
}

// ---- power iteration -------------------------------------------------------
__global__ void k_pow_start(int64_t n, double *__restrict__ x)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) x[i] = 1.0 + (double)(i % 7) / 7.0;
}

__global__ __launch_bounds__(kBlock) void k_sq_partial(int64_t n, const double *__restrict__ y,
                                                       double *__restrict__ part)
{
    __shared__ double lds[kBlock / 64];
    double acc = 0.0;
    for (int64_t i = (int64_t)lb() * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) acc += y[i] * y[i];
    const double s = block_sum(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_normalise(int64_t n, const double *__restrict__ y, double *__restrict__ x,
                                                      const double *__restrict__ part, int np,
                                                      double *__restrict__ norm_out)
{
    __shared__ double lds[kBlock / 64];
    const double nrm = sqrt(sum_partials(part, np, lds));
    if (blockIdx.x == 0 && threadIdx.x == 0) *norm_out = nrm;
    if (nrm == 0.0) return;
    for (int64_t i = (int64_t)lb() * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) x[i] = y[i] / nrm;
}

struct StepBufs {
    double *ur, *ut, *un, *bm, *pr, *pa, *pc, *f, *part, *scal;
    double *bb, *pb;
};

}  // namespace

int run_step(rbffd_ctx *ctx, const rbffd_ops *ops, double *u, double *u_prev, double *p, const double *u_bc,
             const double *p_bc, const rbffd_step_opts *o, rbffd_step_stats *st, hipStream_t s)
{
    const int dim = ops->dim, q = ops->q;
    const int64_t n = ops->n, vs = ops->npad * q;
    const size_t vec = sizeof(double) * n;
    StepBufs B;
    char *w = nullptr;
    const size_t partb = sizeof(double) * (kMaxRhs * kMaxBlocks + 8);
    RB_CHECK(workspace(ctx, WS_STEP, vec * (4 * dim + 4) + partb, (void **)&w));
    B.ur = (double *)w;
    B.ut = B.ur + dim * n;
    B.un = B.ut + dim * n;
    B.bm = B.un + dim * n;
    B.pr = B.bm + dim * n;
    B.pa = B.pr + n;
    B.pc = B.pa + n;
    B.f = B.pc + n;
    B.part = B.f + n;
    B.scal = B.part + kMaxRhs * kMaxBlocks;
    char *w2 = nullptr;
    const int64_t nbv = std::max<int64_t>(ops->nb, 1);
    RB_CHECK(workspace(ctx, WS_STEP2, sizeof(double) * 2 * nbv, (void **)&w2));
    B.bb = (double *)w2;
    B.pb = B.bb + nbv;
    double *hs = nullptr;
    RB_CHECK(host_scratch(ctx, kHostStep, sizeof(double) * 6, (void **)&hs));

    const double rho = o->rho, mu = o->mu, dt = o->dt;
    const double a1 = o->alpha[0], a2 = o->alpha[1], a3 = o->alpha[2];
    const Force3 force{{o->force[0], o->force[1], o->force[2]}};
    const int gn = (int)((n + kBlock - 1) / kBlock);
    const int gpad = (int)((ops->npad + kBlock - 1) / kBlock);
    const int nblk = blocks_for(n);
    const bool fp32 = o->precision != RBFFD_FP64;

    hipLaunchKernelGGL(k_start, dim3(gn), dim3(kBlock), 0, s, n, dim, ops->kind, u, u_bc, p, B.ur, B.pr);
    RB_HIP(hipGetLastError());

    int status = RBFFD_OK, outer = 0, kit_m = 0, kit_p = 0, kit_b = 0;
    double delta = 0.0, relres_p = 0.0, relres_max = 0.0;
    for (outer = 1; outer <= o->max_outer; ++outer) {
        // step 2: momentum matrix, right-hand sides, and the solves from u^r
        if (dim == 2)
            hipLaunchKernelGGL(k_momentum<2>, dim3(gpad), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                               ops->normal, B.ur, u, u_prev, u_bc, B.pr, rho, mu, dt, a1, a2, a3, force, 0, ops->mval,
                               ops->mdinv, B.bm);
        else
            hipLaunchKernelGGL(k_momentum<3>, dim3(gpad), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                               ops->normal, B.ur, u, u_prev, u_bc, B.pr, rho, mu, dt, a1, a2, a3, force, 0, ops->mval,
                               ops->mdinv, B.bm);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(B.ut, B.ur, vec * dim, hipMemcpyDeviceToDevice, s));
        // the d components share one matrix, unless symmetry rows differ between them
        const int groups = ops->n_symmetry > 0 ? dim : 1;
        const int nrhs = ops->n_symmetry > 0 ? 1 : dim;
        for (int g = 0; g < groups; ++g) {
            if (ops->n_symmetry > 0) {
                if (dim == 2) {
                    hipLaunchKernelGGL(k_sym_rows<2>, dim3(gn), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs,
                                       ops->kind, ops->normal, g, ops->mval, ops->mdinv);
                    hipLaunchKernelGGL(k_sym_rhs<2>, dim3(gn), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs,
                                       ops->kind, ops->normal, B.ur, g, B.bm + (int64_t)g * n);
                } else {
                    hipLaunchKernelGGL(k_sym_rows<3>, dim3(gn), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs,
                                       ops->kind, ops->normal, g, ops->mval, ops->mdinv);
                    hipLaunchKernelGGL(k_sym_rhs<3>, dim3(gn), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs,
                                       ops->kind, ops->normal, B.ur, g, B.bm + (int64_t)g * n);
                }
                RB_HIP(hipGetLastError());
            }
            const double *bg = B.bm + (int64_t)g * n;
            double *xg = B.ut + (int64_t)g * n;
            KrylovResult km;
            if (fp32) {
                RB_CHECK(launch_to_fp32(ops->mval, ops->mval32, vs, s));
                RB_CHECK(launch_to_fp32(ops->mdinv, ops->mdinv32, ops->npad, s));
                RB_CHECK(bicgstab_mixed(ctx, o->precision, n, q, cols_of(ops), ops->mval, ops->mval32, ops->mdinv32,
                                        ops->mdinv, kNoBlockInv, nrhs, bg, xg, o->tol_krylov, o->max_krylov, &km,
                                        nullptr, s));
            } else {
                RB_CHECK(bicgstab(ctx, n, q, cols_of(ops), ops->mval, ops->mdinv, nrhs, bg, xg, o->tol_krylov,
                                  o->max_krylov, &km, s));
            }
            for (int e = 0; e < nrhs; ++e) {
                kit_m += km.iters[e];
                relres_max = std::max(relres_max, km.relres[e]);
                if (km.status[e] != RBFFD_OK && status == RBFFD_OK) status = km.status[e];
            }
        }
        // step 3: pressure correction from p' = 0
        const double mass = rho * a1 / dt;
        if (dim == 2)
            hipLaunchKernelGGL(k_div_rhs<2>, dim3(gn), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                               ops->pin, B.ut, mass, B.f);
        else
            hipLaunchKernelGGL(k_div_rhs<3>, dim3(gn), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                               ops->pin, B.ut, mass, B.f);
        RB_HIP(hipMemsetAsync(B.pc, 0, vec, s));
        KrylovResult kp;
        const bool block = o->preconditioner == RBFFD_PREC_BLOCK64;
        if (block) RB_CHECK(ensure_block_inverse(ops, s));
        if (fp32)
            RB_CHECK(bicgstab_mixed(ctx, o->precision, n, q, cols_of(ops), ops->pval, ops->pval32, ops->pdinv32,
                                    ops->pdinv, block ? binv_of(ops) : kNoBlockInv, 1, B.f, B.pc, o->tol_krylov,
                                    o->max_krylov, &kp, nullptr, s));
        else if (block)
            RB_CHECK(bicgstab_block(ctx, n, q, cols_of(ops), ops->pval, binv_of(ops), B.f, B.pc, o->tol_krylov,
                                    o->max_krylov, &kp, s));
        else
            RB_CHECK(bicgstab(ctx, n, q, cols_of(ops), ops->pval, ops->pdinv, 1, B.f, B.pc, o->tol_krylov, o->max_krylov,
                              &kp, s));
        kit_p += kp.iters[0];
        relres_p = kp.relres[0];
        relres_max = std::max(relres_max, kp.relres[0]);
        if (kp.status[0] != RBFFD_OK && status == RBFFD_OK) status = kp.status[0];
        // step 4: interior pressure
        hipLaunchKernelGGL(k_p_interior, dim3(gn), dim3(kBlock), 0, s, n, ops->kind, B.pr, B.pc, p_bc ? p_bc : B.pr,
                           B.pa);
        // step 5: boundary pressure from the normal momentum equation
        if (ops->nb > 0) {
            const unsigned gb = (unsigned)((ops->nb + kBlock - 1) / kBlock);
            if (dim == 2)
                hipLaunchKernelGGL(k_boundary_rhs<2>, dim3(gb), dim3(kBlock), 0, s, n, ops->nb, q, ops->col, ops->val, vs,
                                   ops->pval, ops->kind, ops->normal, ops->bidx, B.ut, u, u_prev, B.pa, B.pr, rho, mu,
                                   dt, a1, a2, a3, force, B.bb, B.pb);
            else
                hipLaunchKernelGGL(k_boundary_rhs<3>, dim3(gb), dim3(kBlock), 0, s, n, ops->nb, q, ops->col, ops->val, vs,
                                   ops->pval, ops->kind, ops->normal, ops->bidx, B.ut, u, u_prev, B.pa, B.pr, rho, mu,
                                   dt, a1, a2, a3, force, B.bb, B.pb);
            RB_HIP(hipGetLastError());
            KrylovResult kb;
            RB_CHECK(bicgstab(ctx, ops->nb, q, cols_plain(ops->gcol), ops->gval, ops->gdinv, 1, B.bb, B.pb, o->tol_krylov,
                              o->max_krylov, &kb, s));
            kit_b += kb.iters[0];
            relres_max = std::max(relres_max, kb.relres[0]);
            if (kb.status[0] != RBFFD_OK && status == RBFFD_OK) status = kb.status[0];
        }
        hipLaunchKernelGGL(k_p_scatter, dim3(gn), dim3(kBlock), 0, s, n, ops->kind, ops->bpos, B.pa, B.pb, B.pr);
        // step 6 + 7: velocity correction and Delta
        const double coef = dt / (rho * a1);
        if (dim == 2)
            hipLaunchKernelGGL(k_correct<2>, dim3(nblk), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                               B.pc, B.ut, B.ur, coef, B.un, B.part);
        else
            hipLaunchKernelGGL(k_correct<3>, dim3(nblk), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                               B.pc, B.ut, B.ur, coef, B.un, B.part);
        hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(kBlock), 0, s, B.part, nblk, dim, n, dt, B.scal);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(hs, B.scal, sizeof(double), hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        delta = hs[0];
        std::swap(B.ur, B.un);
        // step 8
        if (delta < o->tol_outer) break;
    }
    if (outer > o->max_outer) {
        outer = o->max_outer;
        // tol_outer <= 0 asks for exactly max_outer iterations: not a failure
        if (status == RBFFD_OK && o->tol_outer > 0.0) status = RBFFD_E_NOCONV;
    }
    // steady rate, then rotate the time levels
    hipLaunchKernelGGL(k_absdiff, dim3(nblk), dim3(kBlock), 0, s, n, dim, B.ur, u, B.part);
    hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(kBlock), 0, s, B.part, nblk, dim, n, dt, B.scal + 2);
    // discrete continuity error of the new velocity
    if (dim == 2)
        hipLaunchKernelGGL(k_div_abs<2>, dim3(nblk), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind, B.ur,
                           B.part);
    else
        hipLaunchKernelGGL(k_div_abs<3>, dim3(nblk), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind, B.ur,
                           B.part);
    hipLaunchKernelGGL(k_finish_ratio, dim3(1), dim3(kBlock), 0, s, B.part, nblk, B.scal + 4);
    RB_HIP(hipGetLastError());
    RB_HIP(hipMemcpyAsync(u_prev, u, vec * dim, hipMemcpyDeviceToDevice, s));
    RB_HIP(hipMemcpyAsync(u, B.ur, vec * dim, hipMemcpyDeviceToDevice, s));
    RB_HIP(hipMemcpyAsync(p, B.pr, vec, hipMemcpyDeviceToDevice, s));
    RB_HIP(hipMemcpyAsync(hs + 2, B.scal + 2, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    st->outer_iters = outer;
    st->krylov_mom = kit_m;
    st->krylov_p = kit_p;
    st->krylov_b = kit_b;
    st->status = status;
    st->delta = delta;
    st->eps_steady = hs[3];
    st->div_l1 = hs[4];
    st->final_relres_p = relres_p;
    st->krylov_relres_max = relres_max;
    if (status != RBFFD_OK)
        return fail(status, status == RBFFD_E_NOCONV ? "simple_step: an iteration limit was reached"
                                                     : "simple_step: Krylov breakdown");
    return RBFFD_OK;
}

// ---- one time step of many independent clouds -------------------------------
// The outer iteration of run_step on every cloud at once: the per-cloud kernels
// (momentum matrix and right-hand sides, divergence, pressure updates,
// corrections, Delta) are launched cloud by cloud, and each Krylov stage is one
// batched solve over the clouds still iterating (bicgstab_batched: every
// system owns its blocks and reductions, so a cloud's result does not depend on
// the others). A cloud leaves the outer loop when its own Delta meets its own
// tolerance. FP64; no symmetry points (their momentum rows differ between
// components).
int run_step_batched(rbffd_ctx *ctx, int count, const rbffd_ops *const *ops, double *const *u,
                     double *const *u_prev, double *const *p, const double *const *u_bc, const double *const *p_bc,
                     const rbffd_step_opts *o, rbffd_step_stats *st, hipStream_t s)
{
    // per-cloud workspace: the run_step buffers, packed
    std::vector<StepBufs> B(count);
    std::vector<size_t> off(count + 1, 0);
    for (int j = 0; j < count; ++j) {
        const int64_t n = ops[j]->n, nbv = std::max<int64_t>(ops[j]->nb, 1);
        const int dim = ops[j]->dim;
        const size_t words = (size_t)n * (4 * dim + 4) + (kMaxRhs * kMaxBlocks + 8) + 2 * (size_t)nbv;
        off[j + 1] = off[j] + (words + 31) / 32 * 32;
    }
    char *w = nullptr;
    RB_CHECK(workspace(ctx, WS_STEP, sizeof(double) * (off[count] + 2 * (size_t)count), (void **)&w));
    double *base = (double *)w;
    double *deltas = base + off[count];   // [count][2] (Delta, rate) of each cloud, one read-back
    for (int j = 0; j < count; ++j) {
        const int64_t n = ops[j]->n, nbv = std::max<int64_t>(ops[j]->nb, 1);
        const int dim = ops[j]->dim;
        double *b = base + off[j];
        B[j].ur = b;
        B[j].ut = B[j].ur + dim * n;
        B[j].un = B[j].ut + dim * n;
        B[j].bm = B[j].un + dim * n;
        B[j].pr = B[j].bm + dim * n;
        B[j].pa = B[j].pr + n;
        B[j].pc = B[j].pa + n;
        B[j].f = B[j].pc + n;
        B[j].part = B[j].f + n;
        B[j].scal = B[j].part + kMaxRhs * kMaxBlocks;
        B[j].bb = B[j].scal + 8;
        B[j].pb = B[j].bb + nbv;
    }
    std::vector<double> hdelta(count, 0.0);
    std::vector<int> active(count, 1), outer(count, 0), kit_m(count, 0), kit_p(count, 0), kit_b(count, 0),
        status(count, RBFFD_OK);
    std::vector<double> relres_p(count, 0.0), relres_max(count, 0.0);
    for (int j = 0; j < count; ++j) {
        const rbffd_ops *op = ops[j];
        const int gn = (int)((op->n + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_start, dim3(gn), dim3(kBlock), 0, s, op->n, op->dim, op->kind, u[j], u_bc[j], p[j], B[j].ur,
                           B[j].pr);
    }
    RB_HIP(hipGetLastError());
    int max_outer = 0;
    for (int j = 0; j < count; ++j) max_outer = std::max(max_outer, o[j].max_outer);
    std::vector<BatchSystem> sys;
    std::vector<int> owner, it_v, st_v;
    std::vector<double> rr_v;
    auto solve = [&](int kind) -> int {
        // kind 0: momentum (one system per component), 1: pressure correction, 2: boundary pressure
        if (sys.empty()) return RBFFD_OK;
        it_v.assign(sys.size(), 0);
        st_v.assign(sys.size(), 0);
        rr_v.assign(sys.size(), 0.0);
        // one batched call per (tolerance, iteration limit): clouds usually share them
        std::vector<char> done(sys.size(), 0);
        for (size_t a = 0; a < sys.size(); ++a) {
            if (done[a]) continue;
            const rbffd_step_opts &oa = o[owner[a]];
            std::vector<size_t> idx;
            for (size_t b = a; b < sys.size(); ++b)
                if (!done[b] && o[owner[b]].tol_krylov == oa.tol_krylov && o[owner[b]].max_krylov == oa.max_krylov) {
                    idx.push_back(b);
                    done[b] = 1;
                }
            std::vector<BatchSystem> sub;
            for (size_t b : idx) sub.push_back(sys[b]);
            std::vector<int> si(sub.size()), ss(sub.size());
            std::vector<double> sr(sub.size());
            RB_CHECK(bicgstab_batched(ctx, (int)sub.size(), sub.data(), oa.tol_krylov, oa.max_krylov, si.data(),
                                      ss.data(), sr.data(), s));
            for (size_t t = 0; t < idx.size(); ++t) {
                it_v[idx[t]] = si[t];
                st_v[idx[t]] = ss[t];
                rr_v[idx[t]] = sr[t];
            }
        }
        for (size_t a = 0; a < sys.size(); ++a) {
            const int j = owner[a];
            (kind == 0 ? kit_m : kind == 1 ? kit_p : kit_b)[j] += it_v[a];
            relres_max[j] = std::max(relres_max[j], rr_v[a]);
            if (kind == 1) relres_p[j] = rr_v[a];
            if (st_v[a] != RBFFD_OK && status[j] == RBFFD_OK) status[j] = st_v[a];
        }
        return RBFFD_OK;
    };
    for (int it = 1; it <= max_outer; ++it) {
        bool any = false;
        for (int j = 0; j < count; ++j) {
            if (active[j] && it > o[j].max_outer) active[j] = 0;
            any = any || active[j];
        }
        if (!any) break;
        // step 2: momentum matrices and right-hand sides, then one batched solve
        sys.clear();
        owner.clear();
        for (int j = 0; j < count; ++j) {
            if (!active[j]) continue;
            const rbffd_ops *op = ops[j];
            const rbffd_step_opts &oj = o[j];
            const int64_t n = op->n, vs = op->npad * op->q;
            const int gpad = (int)((op->npad + kBlock - 1) / kBlock);
            const Force3 force{{oj.force[0], oj.force[1], oj.force[2]}};
            if (op->dim == 2)
                hipLaunchKernelGGL(k_momentum<2>, dim3(gpad), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs,
                                   op->kind, op->normal, B[j].ur, u[j], u_prev[j], u_bc[j], B[j].pr, oj.rho, oj.mu, oj.dt,
                                   oj.alpha[0], oj.alpha[1], oj.alpha[2], force, 0, op->mval, op->mdinv, B[j].bm);
            else
                hipLaunchKernelGGL(k_momentum<3>, dim3(gpad), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs,
                                   op->kind, op->normal, B[j].ur, u[j], u_prev[j], u_bc[j], B[j].pr, oj.rho, oj.mu, oj.dt,
                                   oj.alpha[0], oj.alpha[1], oj.alpha[2], force, 0, op->mval, op->mdinv, B[j].bm);
            RB_HIP(hipMemcpyAsync(B[j].ut, B[j].ur, sizeof(double) * n * op->dim, hipMemcpyDeviceToDevice, s));
            for (int e = 0; e < op->dim; ++e) {
                BatchSystem y{};
                y.n = n;
                y.q = op->q;
                y.col = cols_of(op);
                y.val = op->mval;
                y.dinv = op->mdinv;
                y.b = B[j].bm + (int64_t)e * n;
                y.x = B[j].ut + (int64_t)e * n;
                y.binv = kNoBlockInv;
                y.val32 = nullptr;
                sys.push_back(y);
                owner.push_back(j);
            }
        }
        RB_HIP(hipGetLastError());
        RB_CHECK(solve(0));
        // step 3: pressure corrections from p' = 0, one batched solve
        sys.clear();
        owner.clear();
        for (int j = 0; j < count; ++j) {
            if (!active[j]) continue;
            const rbffd_ops *op = ops[j];
            const rbffd_step_opts &oj = o[j];
            const int64_t n = op->n, vs = op->npad * op->q;
            const int gn = (int)((n + kBlock - 1) / kBlock);
            const double mass = oj.rho * oj.alpha[0] / oj.dt;
            if (op->dim == 2)
                hipLaunchKernelGGL(k_div_rhs<2>, dim3(gn), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs, op->kind,
                                   op->pin, B[j].ut, mass, B[j].f);
            else
                hipLaunchKernelGGL(k_div_rhs<3>, dim3(gn), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs, op->kind,
                                   op->pin, B[j].ut, mass, B[j].f);
            RB_HIP(hipMemsetAsync(B[j].pc, 0, sizeof(double) * n, s));
            BatchSystem y{};
            y.n = n;
            y.q = op->q;
            y.col = cols_of(op);
            y.val = op->pval;
            y.dinv = op->pdinv;
            y.b = B[j].f;
            y.x = B[j].pc;
            if (oj.preconditioner == RBFFD_PREC_BLOCK64) RB_CHECK(ensure_block_inverse(op, s));
            y.binv = oj.preconditioner == RBFFD_PREC_BLOCK64 ? binv_of(op) : kNoBlockInv;
            y.val32 = nullptr;
            sys.push_back(y);
            owner.push_back(j);
        }
        RB_HIP(hipGetLastError());
        RB_CHECK(solve(1));
        // steps 4-5: interior pressure; boundary pressures, one batched solve
        sys.clear();
        owner.clear();
        for (int j = 0; j < count; ++j) {
            if (!active[j]) continue;
            const rbffd_ops *op = ops[j];
            const rbffd_step_opts &oj = o[j];
            const int64_t n = op->n, vs = op->npad * op->q;
            const int gn = (int)((n + kBlock - 1) / kBlock);
            const Force3 force{{oj.force[0], oj.force[1], oj.force[2]}};
            hipLaunchKernelGGL(k_p_interior, dim3(gn), dim3(kBlock), 0, s, n, op->kind, B[j].pr, B[j].pc,
                               p_bc[j] ? p_bc[j] : B[j].pr, B[j].pa);
            if (op->nb > 0) {
                const unsigned gb = (unsigned)((op->nb + kBlock - 1) / kBlock);
                if (op->dim == 2)
                    hipLaunchKernelGGL(k_boundary_rhs<2>, dim3(gb), dim3(kBlock), 0, s, n, op->nb, op->q, op->col,
                                       op->val, vs, op->pval, op->kind, op->normal, op->bidx, B[j].ut, u[j], u_prev[j],
                                       B[j].pa, B[j].pr, oj.rho, oj.mu, oj.dt, oj.alpha[0], oj.alpha[1], oj.alpha[2],
                                       force, B[j].bb, B[j].pb);
                else
                    hipLaunchKernelGGL(k_boundary_rhs<3>, dim3(gb), dim3(kBlock), 0, s, n, op->nb, op->q, op->col,
                                       op->val, vs, op->pval, op->kind, op->normal, op->bidx, B[j].ut, u[j], u_prev[j],
                                       B[j].pa, B[j].pr, oj.rho, oj.mu, oj.dt, oj.alpha[0], oj.alpha[1], oj.alpha[2],
                                       force, B[j].bb, B[j].pb);
                BatchSystem y{};
                y.n = op->nb;
                y.q = op->q;
                y.col = cols_plain(op->gcol);
                y.val = op->gval;
                y.dinv = op->gdinv;
                y.b = B[j].bb;
                y.x = B[j].pb;
                y.binv = kNoBlockInv;
                y.val32 = nullptr;
                sys.push_back(y);
                owner.push_back(j);
            }
        }
        RB_HIP(hipGetLastError());
        RB_CHECK(solve(2));
        // steps 6-7: scatter the pressures, correct the velocities, Delta
        for (int j = 0; j < count; ++j) {
            if (!active[j]) continue;
            const rbffd_ops *op = ops[j];
            const rbffd_step_opts &oj = o[j];
            const int64_t n = op->n, vs = op->npad * op->q;
            const int gn = (int)((n + kBlock - 1) / kBlock);
            const int nblk = blocks_for(n);
            const double coef = oj.dt / (oj.rho * oj.alpha[0]);
            hipLaunchKernelGGL(k_p_scatter, dim3(gn), dim3(kBlock), 0, s, n, op->kind, op->bpos, B[j].pa, B[j].pb,
                               B[j].pr);
            if (op->dim == 2)
                hipLaunchKernelGGL(k_correct<2>, dim3(nblk), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs, op->kind,
                                   B[j].pc, B[j].ut, B[j].ur, coef, B[j].un, B[j].part);
            else
                hipLaunchKernelGGL(k_correct<3>, dim3(nblk), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs, op->kind,
                                   B[j].pc, B[j].ut, B[j].ur, coef, B[j].un, B[j].part);
            hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(kBlock), 0, s, B[j].part, nblk, op->dim, n, oj.dt,
                               deltas + 2 * j);
        }
        RB_HIP(hipGetLastError());
        double *hd = nullptr;   // pinned; the batched solves are done with their staging by now
        RB_CHECK(workspace(ctx, WS_BATCH_HOST, sizeof(double) * 2 * (size_t)count, (void **)&hd));
        RB_HIP(hipMemcpyAsync(hd, deltas, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        for (int j = 0; j < count; ++j) {
            if (!active[j]) continue;
            hdelta[j] = hd[2 * j];
            outer[j] = it;
            std::swap(B[j].ur, B[j].un);
            if (hdelta[j] < o[j].tol_outer) active[j] = 0;
        }
    }
    // steady rates, continuity errors, time-level rotation, statistics
    for (int j = 0; j < count; ++j) {
        const rbffd_ops *op = ops[j];
        const int64_t n = op->n, vs = op->npad * op->q;
        const int nblk = blocks_for(n);
        hipLaunchKernelGGL(k_absdiff, dim3(nblk), dim3(kBlock), 0, s, n, op->dim, B[j].ur, u[j], B[j].part);
        hipLaunchKernelGGL(k_finish_sums, dim3(1), dim3(kBlock), 0, s, B[j].part, nblk, op->dim, n, o[j].dt,
                           B[j].scal + 2);
        if (op->dim == 2)
            hipLaunchKernelGGL(k_div_abs<2>, dim3(nblk), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs, op->kind,
                               B[j].ur, B[j].part);
        else
            hipLaunchKernelGGL(k_div_abs<3>, dim3(nblk), dim3(kBlock), 0, s, n, op->q, op->col, op->val, vs, op->kind,
                               B[j].ur, B[j].part);
        hipLaunchKernelGGL(k_finish_ratio, dim3(1), dim3(kBlock), 0, s, B[j].part, nblk, B[j].scal + 4);
        const size_t vec = sizeof(double) * n;
        RB_HIP(hipMemcpyAsync(u_prev[j], u[j], vec * op->dim, hipMemcpyDeviceToDevice, s));
        RB_HIP(hipMemcpyAsync(u[j], B[j].ur, vec * op->dim, hipMemcpyDeviceToDevice, s));
        RB_HIP(hipMemcpyAsync(p[j], B[j].pr, vec, hipMemcpyDeviceToDevice, s));
    }
    RB_HIP(hipGetLastError());
    std::vector<double> sc(3 * (size_t)count);
    for (int j = 0; j < count; ++j)
        RB_HIP(hipMemcpyAsync(&sc[3 * j], B[j].scal + 2, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    int first_fail = RBFFD_OK;
    for (int j = 0; j < count; ++j) {
        if (outer[j] >= o[j].max_outer && hdelta[j] >= o[j].tol_outer && status[j] == RBFFD_OK &&
            o[j].tol_outer > 0.0)
            status[j] = RBFFD_E_NOCONV;   // tol_outer <= 0 asks for exactly max_outer iterations
        rbffd_step_stats &t = st[j];
        t.outer_iters = outer[j];
        t.krylov_mom = kit_m[j];
        t.krylov_p = kit_p[j];
        t.krylov_b = kit_b[j];
        t.status = status[j];
        t.delta = hdelta[j];
        t.eps_steady = sc[3 * j + 1];
        t.div_l1 = sc[3 * j + 2];
        t.final_relres_p = relres_p[j];
        t.krylov_relres_max = relres_max[j];
        if (status[j] != RBFFD_OK && first_fail == RBFFD_OK) first_fail = status[j];
    }
    if (first_fail != RBFFD_OK)
        return fail(first_fail, "simple_step_batched: an iteration limit was reached or a Krylov solve broke down "
                                "(per-cloud status in stats)");
    return RBFFD_OK;
}

int convdiff_lambda(rbffd_ctx *ctx, const rbffd_ops *ops, const double *u0, double rho, double mu, int iters,
                    double *lambda, hipStream_t s)
{
    const int dim = ops->dim, q = ops->q;
    const int64_t n = ops->n, vs = ops->npad * q;
    char *w = nullptr;
    RB_CHECK(workspace(ctx, WS_STEP, sizeof(double) * (2 * n + kMaxBlocks + 8), (void **)&w));
    double *x = (double *)w, *y = x + n, *part = y + n, *nrm = part + kMaxBlocks;
    const int gpad = (int)((ops->npad + kBlock - 1) / kBlock);
    const int gn = (int)((n + kBlock - 1) / kBlock);
    const int nblk = blocks_for(n);
    if (dim == 2)
        hipLaunchKernelGGL(k_momentum<2>, dim3(gpad), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                           ops->normal, u0, u0, u0, u0, u0, rho, mu, 1.0, 0.0, 0.0, 0.0, Force3{}, 1, ops->mval,
                           ops->mdinv, y);
    else
        hipLaunchKernelGGL(k_momentum<3>, dim3(gpad), dim3(kBlock), 0, s, n, q, ops->col, ops->val, vs, ops->kind,
                           ops->normal, u0, u0, u0, u0, u0, rho, mu, 1.0, 0.0, 0.0, 0.0, Force3{}, 1, ops->mval,
                           ops->mdinv, y);
    hipLaunchKernelGGL(k_pow_start, dim3(gn), dim3(kBlock), 0, s, n, y);
    hipLaunchKernelGGL(k_sq_partial, dim3(nblk), dim3(kBlock), 0, s, n, y, part);
    hipLaunchKernelGGL(k_normalise, dim3(nblk), dim3(kBlock), 0, s, n, y, x, part, nblk, nrm);
    for (int it = 0; it < iters; ++it) {
        RB_CHECK(spmv(n, q, cols_of(ops), ops->mval, x, y, s));
        hipLaunchKernelGGL(k_sq_partial, dim3(nblk), dim3(kBlock), 0, s, n, y, part);
        hipLaunchKernelGGL(k_normalise, dim3(nblk), dim3(kBlock), 0, s, n, y, x, part, nblk, nrm);
    }
    RB_HIP(hipGetLastError());
    double *hs = nullptr;
    RB_CHECK(host_scratch(ctx, kHostStep, sizeof(double), (void **)&hs));
    RB_HIP(hipMemcpyAsync(hs, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    *lambda = hs[0];
    return RBFFD_OK;
}

}  // namespace rbffd
