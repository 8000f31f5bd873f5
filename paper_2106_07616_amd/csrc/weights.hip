// Local PHS-RBF + polynomial differentiation weights (Sec. 2, Eqs. RBF_interp,
// RBF_constraint, RBF_interp_mat_vec, RBF_interp_phi, RBF_interp_poly,
// RBF_interp_L ... RBF_interp_mat_vec_L_solve).
//
// For each point the saddle system A = [Phi P; P^T 0] (ns = q + m) and one
// right-hand side per operator (d/dx, d/dy, (d/dz), Laplacian at the centre)
// are built in coordinates centred at the point and scaled by the distance to
// its q-th neighbour, then solved by LU with partial pivoting; since A is
// symmetric, the centre row of B1 = [L Phi  L P] A^{-1} is the first q entries
// of A^{-1} b_L.
//
// Layout on gfx950: one wavefront per system, lane r owns row r of [A | B] in
// registers (ns <= 64). The pivot search is a wave max-reduction, the pivot row
// is broadcast lane-to-scalar with readlane, and the rank-1 update is one FP64
// FMA per entry. On gfx950 the FP64 matrix-core rate equals the FP64 vector
// rate, so the unblocked register LU runs against the same FP64 ceiling a
// blocked MFMA factorisation would, without its panel/broadcast overheads.
#include <cfloat>
#include <climits>
#include <cmath>

#include "internal.h"

namespace rbffd {

namespace {

__device__ inline double readlane_d(double v, int lane)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

template <int DIM>
__device__ inline double sqdist_exact(const double *a, const double *b)
{
#pragma clang fp contract(off)
    double dx = b[0] - a[0];
    double dy = b[1] - a[1];
    double d2 = dx * dx + dy * dy;
    if (DIM == 3) {
        double dz = b[2] - a[2];
        d2 = d2 + dz * dz;
    }
    return d2;
}

__device__ inline double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r = r * x;
    return r;
}

template <int DIM>
__device__ inline double monomial(const int *ex, const double *x)
{
    double v = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) v = v * ipow(x[d], ex[d]);
    return v;
}

// graded monomial order: by total degree, then descending x power, then y power
template <int DIM>
__device__ inline void monomial_exponents(int alpha, int *ex)
{
    int idx = 0;
    for (int t = 0; t <= 16; ++t) {
        for (int a = t; a >= 0; --a) {
            if (DIM == 2) {
                if (idx == alpha) {
                    ex[0] = a;
                    ex[1] = t - a;
                    ex[2] = 0;
                    return;
                }
                ++idx;
            } else {
                for (int b = t - a; b >= 0; --b) {
                    if (idx == alpha) {
                        ex[0] = a;
                        ex[1] = b;
                        ex[2] = t - a - b;
                        return;
                    }
                    ++idx;
                }
            }
        }
    }
}

template <int NSP, int DIM>
__global__ __launch_bounds__(64) void weights_kernel(const double *__restrict__ xyz, const int32_t *__restrict__ nbr,
                                                     int64_t n, int q, int m, int phs, double *__restrict__ w,
                                                     int64_t *__restrict__ bad)
{
    constexpr int R = DIM + 1;
    constexpr int NC = NSP + R;
    __shared__ double xs[kMaxQ * DIM];
    __shared__ int exs[64 * 3];
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const int ns = q + m;

    // centre and scale: s = distance to the q-th neighbour
    double c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) c[d] = xyz[i * DIM + d];
    const int64_t jl = nbr[i * q + q - 1];
    const double s = sqrt(sqdist_exact<DIM>(c, xyz + jl * DIM));
    for (int a = lane; a < q; a += 64) {
        const int64_t j = nbr[i * q + a];
        for (int d = 0; d < DIM; ++d) xs[a * DIM + d] = (xyz[j * DIM + d] - c[d]) / s;
    }
    if (lane < m) {
        int ex[3];
        monomial_exponents<DIM>(lane, ex);
        exs[lane * 3 + 0] = ex[0];
        exs[lane * 3 + 1] = ex[1];
        exs[lane * 3 + 2] = ex[2];
    }
    __syncthreads();

    // ---- row `lane` of [A | B] ---------------------------------------------
    double a_[NC];
    double mine[3] = {0, 0, 0};
    if (lane < q)
        for (int d = 0; d < DIM; ++d) mine[d] = xs[lane * DIM + d];
    int myex[3] = {0, 0, 0};
    if (lane >= q && lane < ns) {
        myex[0] = exs[(lane - q) * 3 + 0];
        myex[1] = exs[(lane - q) * 3 + 1];
        myex[2] = exs[(lane - q) * 3 + 2];
    }
#pragma unroll
    for (int b = 0; b < NSP; ++b) {
        double v = 0.0;
        if (lane < q) {
            if (b < q) {
                const double r = sqrt(sqdist_exact<DIM>(mine, xs + b * DIM));
                v = (phs == 3) ? r * r * r : r * r * r * r * r;
            } else if (b < ns) {
                v = monomial<DIM>(exs + (b - q) * 3, mine);
            }
        } else if (lane < ns) {
            if (b < q) v = monomial<DIM>(myex, xs + b * DIM);
        }
        a_[b] = v;
    }
    {
        // right-hand sides: L phi(|x - x_lane|) and L P_alpha at the centre
        double rhs[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rhs[r] = 0.0;
        if (lane < q) {
            double rr = 0.0;
            for (int d = 0; d < DIM; ++d) rr = rr + mine[d] * mine[d];
            const double r = sqrt(rr);
            const double rp2 = (phs == 3) ? r : r * r * r;
#pragma unroll
            for (int d = 0; d < DIM; ++d) rhs[d] = -(double)phs * rp2 * mine[d];
            rhs[DIM] = (double)(phs * (phs + DIM - 2)) * rp2;
        } else if (lane < ns) {
            const int tot = myex[0] + myex[1] + myex[2];
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (tot == 1 && myex[d] == 1) rhs[d] = 1.0;
                if (tot == 2 && myex[d] == 2) rhs[DIM] = 2.0;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) a_[NSP + r] = rhs[r];
    }

    // ---- LU with partial pivoting (largest |a|, ties to the lowest row) -----
    double amax = 0.0;
#pragma unroll
    for (int b = 0; b < NSP; ++b) amax = fmax(amax, fabs(a_[b]));
    amax = wave_max(amax);
    bool active = lane < ns;
    int mystep = -1;
    bool singular = false;
#pragma unroll
    for (int k = 0; k < NSP; ++k) {
        if (k < ns) {
            const double v = active ? fabs(a_[k]) : -1.0;
            const double mx = wave_max(v);
            const uint64_t msk = __ballot(active && v == mx);
            const int p = msk ? (__ffsll((unsigned long long)msk) - 1) : 0;
            if (!(mx > 1e-13 * amax)) singular = true;
            double piv = readlane_d(a_[k], p);
            if (singular) piv = 1.0;
            if (lane == p) {
                active = false;
                mystep = k;
            }
            const double l = active ? a_[k] / piv : 0.0;
#pragma unroll
            for (int j = k + 1; j < NC; ++j) {
                const double u = readlane_d(a_[j], p);
                a_[j] = fma(-l, u, a_[j]);
            }
        }
    }

    // ---- back substitution; lane c keeps unknown c ---------------------------
    double xout[R];
#pragma unroll
    for (int r = 0; r < R; ++r) xout[r] = 0.0;
#pragma unroll
    for (int k = NSP - 1; k >= 0; --k) {
        if (k < ns) {
            const uint64_t msk = __ballot(mystep == k);
            const int p = msk ? (__ffsll((unsigned long long)msk) - 1) : 0;
            double dgl = readlane_d(a_[k], p);
            if (singular) dgl = 1.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double y = readlane_d(a_[NSP + r], p);
                const double xk = y / dgl;
                if (lane == k) xout[r] = xk;
                if (mystep >= 0 && mystep < k) a_[NSP + r] = fma(-a_[k], xk, a_[NSP + r]);
            }
        }
    }

    // ---- unscale and store (cloud order) -------------------------------------
    if (lane < q) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double sc = (r < DIM) ? s : s * s;
            w[(int64_t)r * n * q + i * q + lane] = xout[r] / sc;
        }
    }
    if (singular && lane == 0) atomicMin((unsigned long long *)bad, (unsigned long long)i);
}

}  // namespace

int launch_weights(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int q, const int32_t *nbr, int k,
                   int phs, double *w, int64_t *bad_dev, hipStream_t s)
{
    (void)ctx;
    long mm = 1, den = 1;
    for (int i = 1; i <= dim; ++i) {
        mm *= (k + i);
        den *= i;
    }
    const int m = (int)(mm / den);
    const int ns = q + m;
    const long long init = LLONG_MAX;
    RB_HIP(hipMemcpyAsync(bad_dev, &init, sizeof(init), hipMemcpyHostToDevice, s));
    const dim3 grid((unsigned)n), block(64);
    // the register row holds NSP + R doubles: NSP is the smallest instantiated
    // size >= ns, so little work goes to padding columns
#define RB_WEIGHTS(NSP_)                                                                                  \
    if (ns <= NSP_) {                                                                                     \
        if (dim == 2)                                                                                     \
            hipLaunchKernelGGL((weights_kernel<NSP_, 2>), grid, block, 0, s, xyz, nbr, n, q, m, phs, w, bad_dev); \
        else                                                                                              \
            hipLaunchKernelGGL((weights_kernel<NSP_, 3>), grid, block, 0, s, xyz, nbr, n, q, m, phs, w, bad_dev); \
        RB_HIP(hipGetLastError());                                                                        \
        return RBFFD_OK;                                                                                  \
    }
    RB_WEIGHTS(16)
    RB_WEIGHTS(24)
    RB_WEIGHTS(32)
    RB_WEIGHTS(40)
    RB_WEIGHTS(48)
    RB_WEIGHTS(56)
    RB_WEIGHTS(64)
#undef RB_WEIGHTS
    return fail(RBFFD_E_ARG, "collocation systems larger than 64 are not supported");
}

}  // namespace rbffd
