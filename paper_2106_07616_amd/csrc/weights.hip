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
// Layout on gfx950, by system size:
//  - up to 64 unknowns: one wavefront per system, lane r owns row r of [A | B]
//    in registers; the pivot search is a DPP wave max-reduction, the pivot row
//    is broadcast lane-to-scalar with readlane, and the rank-1 update is one
//    FP64 FMA per entry (LU, then back substitution);
//  - 65 unknowns and up, at most 128 columns with the right-hand sides (2D
//    degree 6, 3D degree 4): blocked Gauss-Jordan in panels of four columns
//    whose rank-4 updates run on v_mfma_f64_16x16x4, the matrix in registers
//    as MFMA tiles spread over three or four wavefronts (below);
//  - up to 128 unknowns with more columns: the same elimination with the
//    tiles in LDS (up to 159 KB), and an unblocked LDS kernel on devices whose
//    workgroups cannot hold those tiles.
// On gfx950 the FP64 matrix-core rate equals the FP64 vector rate: the MFMA
// path pays by replacing per-entry LDS traffic and broadcasts with one
// instruction per 16 x 16 tile, not by a higher ceiling.
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

// Wave maximum through DPP within rows of 16 lanes, then the four row maxima.
__device__ inline double dpp_max_step(double v, int ctrl_sel)
{
    int lo = __double2loint(v), hi = __double2hiint(v);
    int lo2, hi2;
    switch (ctrl_sel) {
    case 0:   // quad_perm [1, 0, 3, 2]
        lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0xB1, 0xF, 0xF, false);
        hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0xB1, 0xF, 0xF, false);
        break;
    case 1:   // quad_perm [2, 3, 0, 1]
        lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x4E, 0xF, 0xF, false);
        hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x4E, 0xF, 0xF, false);
        break;
    case 2:   // row_half_mirror
        lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x141, 0xF, 0xF, false);
        hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x141, 0xF, 0xF, false);
        break;
    default:  // row_mirror
        lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x140, 0xF, 0xF, false);
        hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x140, 0xF, 0xF, false);
        break;
    }
    return fmax(v, __hiloint2double(hi2, lo2));
}

__device__ inline double wave_max_dpp(double v)
{
    v = dpp_max_step(v, 0);
    v = dpp_max_step(v, 1);
    v = dpp_max_step(v, 2);
    v = dpp_max_step(v, 3);
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// The same maximum with the cross-row steps as DPP row broadcasts (rows 1
// and 3 take lane 15 of the row before, then rows 2 and 3 take lane 31), so
// that lane 63 holds it: one readlane instead of four.
__device__ inline double dpp_bcast_max(double v, int sel)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int lo2, hi2;
    if (sel == 0) {   // row_bcast:15 into rows 1 and 3
        lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x142, 0xA, 0xF, false);
        hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x142, 0xA, 0xF, false);
    } else {          // row_bcast:31 into rows 2 and 3
        lo2 = __builtin_amdgcn_update_dpp(lo, lo, 0x143, 0xC, 0xF, false);
        hi2 = __builtin_amdgcn_update_dpp(hi, hi, 0x143, 0xC, 0xF, false);
    }
    return fmax(v, __hiloint2double(hi2, lo2));
}

__device__ inline double wave_max_bcast(double v)
{
    v = dpp_max_step(v, 0);
    v = dpp_max_step(v, 1);
    v = dpp_max_step(v, 2);
    v = dpp_max_step(v, 3);
    v = dpp_bcast_max(v, 0);
    v = dpp_bcast_max(v, 1);
    return readlane_d(v, 63);
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

// graded monomial order: by total degree, then descending x power, then
// descending y power. Closed form: the degree t is the first with more than
// alpha monomials of degree <= t, and the position r within degree t fixes the
// powers (a short loop over the x power in 3-D). A search that returns from a
// nested loop unrolls into a divergent branch chain whose saved exec masks
// spill scalar registers.
template <int DIM>
__device__ inline int monomials_below(int t)
{
    return DIM == 2 ? t * (t + 1) / 2 : t * (t + 1) * (t + 2) / 6;
}

template <int DIM>
__device__ inline void monomial_exponents(int alpha, int *ex)
{
    int t = 0;
#pragma unroll 1
    while (monomials_below<DIM>(t + 1) <= alpha) ++t;
    int r = alpha - monomials_below<DIM>(t);
    if (DIM == 2) {
        ex[0] = t - r;
        ex[1] = r;
        ex[2] = 0;
    } else {
        int a = t;
#pragma unroll 1
        while (r > t - a) {
            r -= t - a + 1;
            --a;
        }
        ex[0] = a;
        ex[1] = t - a - r;
        ex[2] = r;
    }
}

// With INTERP set, the kernel gives interpolation weights at off-node points
// instead, as the LDS kernel below does in that mode: centre ctr[i], scale the
// distance to the farthest cloud point, one right-hand side, unscaled weights.
//
// The work of one point lives in weights_point, so that the batched kernel
// below runs the same arithmetic for the points of many clouds. xs and exs are
// the block's LDS buffers (kMaxQ * DIM doubles, 64 * 3 ints).
// Elimination segment length of the register kernel by system width: fully
// unrolled (1) up to 32 unknowns, pairs of steps above (measured on MI355X
// against lengths 3, 4, 8 and 16 and a fully unrolled kernel, whose 48- and
// 64-wide bodies are 140-220 KB of code).
template <int NSP>
constexpr int weights_segment()
{
    return NSP <= 32 ? 1 : 2;
}

template <int NSP, int DIM, bool INTERP>
__device__ __forceinline__ void weights_point(const double *__restrict__ xyz, const double *__restrict__ ctr,
                                     const int32_t *__restrict__ nbr, int64_t n, int q, int m, int phs,
                                     double *__restrict__ w, int64_t *__restrict__ bad, int64_t i, double *xs,
                                     int *exs)
{
    constexpr int R = INTERP ? 1 : DIM + 1;
    constexpr int NC = NSP + R;
    const int lane = threadIdx.x;
    const int ns = q + m;

    // centre and scale: s = distance to the q-th neighbour
    double c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) c[d] = ctr[i * DIM + d];
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
    // Columns are computed in a runtime loop per segment of SEG and dropped into
    // their (constant-index) registers by a select, which keeps the code small.
    constexpr int SEG = weights_segment<NSP>();
#pragma unroll
    for (int b0 = 0; b0 < NSP; b0 += SEG) {
#pragma unroll 1
        for (int t = 0; t < SEG; ++t) {
            const int b = b0 + t;
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
#pragma unroll
            for (int tt = 0; tt < SEG; ++tt)
                if (b0 + tt < NSP && t == tt) a_[b0 + tt] = v;
        }
    }
    {
        // right-hand sides: L phi(|x - x_lane|) and L P_alpha at the centre
        double rhs[R];
#pragma unroll
        for (int r = 0; r < R; ++r) rhs[r] = 0.0;
        if constexpr (INTERP) {
            // phi(|x_lane - x*|) and the monomials at the centre x*
            if (lane < q) {
                double rr = 0.0;
                for (int d = 0; d < DIM; ++d) rr = rr + mine[d] * mine[d];
                const double r = sqrt(rr);
                rhs[0] = (phs == 3) ? r * r * r : r * r * r * r * r;
            } else if (lane < ns) {
                rhs[0] = (myex[0] + myex[1] + myex[2] == 0) ? 1.0 : 0.0;
            }
        } else if (lane < q) {
            double rr = 0.0;
            for (int d = 0; d < DIM; ++d) rr = rr + mine[d] * mine[d];
            const double r = sqrt(rr);
            const double rp2 = (phs == 3) ? r : r * r * r;
#pragma unroll
            for (int d = 0; d < DIM; ++d) rhs[d] = -(double)phs * rp2 * mine[d];
            rhs[R - 1] = (double)(phs * (phs + DIM - 2)) * rp2;
        } else if (lane < ns) {
            const int tot = myex[0] + myex[1] + myex[2];
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                if (tot == 1 && myex[d] == 1) rhs[d] = 1.0;
                if (tot == 2 && myex[d] == 2) rhs[R - 1] = 2.0;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) a_[NSP + r] = rhs[r];
    }

    // ---- LU with partial pivoting (largest |a|, ties to the lowest row) -----
    double amax = 0.0;
#pragma unroll
    for (int b = 0; b < NSP; ++b) amax = fmax(amax, fabs(a_[b]));
    amax = wave_max_dpp(amax);
    bool active = lane < ns;
    int mystep = -1;
    bool singular = false;
    // The steps run in segments of SEG: the segment loop is unrolled (so every
    // register index is a constant) and the steps inside a segment are a
    // runtime loop that updates the segment's remaining columns. A fully
    // unrolled elimination is over 100 KB of code for 45+ unknowns, more than
    // the instruction cache; segmenting costs ~15% extra column updates and
    // gives the same arithmetic, column by column.
#pragma unroll
    for (int k0 = 0; k0 < NSP; k0 += SEG) {
        const int kend = min(k0 + SEG, ns);
#pragma unroll 1
        for (int k = k0; k < kend; ++k) {
            double ak = a_[k0];
#pragma unroll
            for (int t = 1; t < SEG; ++t)
                if (k0 + t < NSP && k == k0 + t) ak = a_[k0 + t];
            const double v = active ? fabs(ak) : -1.0;
            const double mx = wave_max_bcast(v);
            const uint64_t msk = __ballot(active && v == mx);
            const int p = msk ? (__ffsll((unsigned long long)msk) - 1) : 0;
            if (!(mx > 1e-13 * amax)) singular = true;
            double piv = readlane_d(ak, p);
            if (singular) piv = 1.0;
            if (lane == p) {
                active = false;
                mystep = k;
            }
            const double l = active ? ak / piv : 0.0;
#pragma unroll
            for (int j = k0 + 1; j < NC; ++j) {
                if (j >= k0 + SEG || j > k) {
                    const double u = readlane_d(a_[j], p);
                    a_[j] = fma(-l, u, a_[j]);
                }
            }
        }
    }

    // ---- back substitution; lane c keeps unknown c ---------------------------
    double xout[R];
#pragma unroll
    for (int r = 0; r < R; ++r) xout[r] = 0.0;
#pragma unroll
    for (int k0 = ((NSP - 1) / SEG) * SEG; k0 >= 0; k0 -= SEG) {
#pragma unroll 1
        for (int k = min(k0 + SEG, ns) - 1; k >= k0; --k) {
            double ak = a_[k0];
#pragma unroll
            for (int t = 1; t < SEG; ++t)
                if (k0 + t < NSP && k == k0 + t) ak = a_[k0 + t];
            const uint64_t msk = __ballot(mystep == k);
            const int p = msk ? (__ffsll((unsigned long long)msk) - 1) : 0;
            double dgl = readlane_d(ak, p);
            if (singular) dgl = 1.0;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const double y = readlane_d(a_[NSP + r], p);
                const double xk = y / dgl;
                if (lane == k) xout[r] = xk;
                if (mystep >= 0 && mystep < k) a_[NSP + r] = fma(-ak, xk, a_[NSP + r]);
            }
        }
    }

    // ---- unscale and store (cloud order) -------------------------------------
    if (lane < q) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double sc = INTERP ? 1.0 : ((r < DIM) ? s : s * s);
            w[(int64_t)r * n * q + i * q + lane] = INTERP ? xout[r] : xout[r] / sc;
        }
    }
    if (singular && lane == 0) atomicMin((unsigned long long *)bad, (unsigned long long)i);
}

template <int NSP, int DIM, bool INTERP>
__global__ __launch_bounds__(64) void weights_kernel(const double *__restrict__ xyz, const double *__restrict__ ctr,
                                                     const int32_t *__restrict__ nbr, int64_t n, int q, int m, int phs,
                                                     double *__restrict__ w, int64_t *__restrict__ bad)
{
    __shared__ double xs[kMaxQ * DIM];
    __shared__ int exs[64 * 3];
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    weights_point<NSP, DIM, INTERP>(xyz, ctr, nbr, n, q, m, phs, w, bad, i, xs, exs);
}

// Weights of the points of many clouds in one launch, all with the register
// width NSP: block b takes point b - first_block of the last cloud whose
// first_block <= b (binary search over the clouds) and runs weights_point
// with that cloud's sizes, so every point gets exactly the arithmetic of the
// one-cloud kernel. Each cloud has its own singular-point slot. Clouds of
// different widths go to different launches: one kernel covering every width
// would hold the widest path's registers (167 VGPRs against 58 at width 16)
// and run the narrow systems at a third of their occupancy.
template <int NSP, int DIM>
__global__ __launch_bounds__(64) void weights_batched_kernel(const WeightSys *__restrict__ sys, int count,
                                                             int64_t *__restrict__ bad)
{
    __shared__ double xs[kMaxQ * DIM];
    __shared__ int exs[64 * 3];
    const int64_t b = blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sys[mid].first_block <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    const WeightSys S = sys[lo];
    const int64_t i = b - S.first_block;
    if (i < 0 || i >= S.n) return;
    weights_point<NSP, DIM, false>(S.xyz, S.xyz, S.nbr, S.n, S.q, S.m, S.phs, S.w, bad + lo, i, xs, exs);
}

// Systems of 65-128 unknowns: one workgroup of 128 x kRowThreads threads per
// system. [A | B] lives in LDS column-major (entry (t, j) at j*128 + t, up to
// 132 KiB), so the lanes of a wavefront touch consecutive addresses. Row t is
// shared by the threads (t, h), h < kRowThreads, each updating the columns
// j = h mod kRowThreads; the threads with h = 0 (wavefronts 0 and 1) run the
// pivot search and the back substitution. The arithmetic per entry is the
// one-wavefront kernel's. A double-buffered LDS pair carries the two
// wavefronts' pivot candidates, so one barrier per elimination step orders
// every cross-row read.
//
// With INTERP set the same kernel gives interpolation weights at off-node
// points (evaluation of the local PHS + polynomial interpolant, Sec. 2, Eq.
// RBF_interp): the system is centred at query point i (ctr[i]), scaled by the
// distance to its farthest cloud point, and its one right-hand side is
// [phi(|x_j - x*|); P(x*)], where only the constant monomial is nonzero at the
// centre. Interpolation weights are scale-free, so they are stored unscaled.
constexpr int kRowThreads = 8;

template <int DIM, bool INTERP>
__global__ __launch_bounds__(128 * kRowThreads) void weights_kernel_lds(
    const double *__restrict__ xyz, const double *__restrict__ ctr, const int32_t *__restrict__ nbr, int64_t n,
    int q, int m, int phs, double *__restrict__ w, int64_t *__restrict__ bad)
{
    constexpr int R = INTERP ? 1 : DIM + 1;
    constexpr int NW = 128 * kRowThreads / 64;   // wavefronts per workgroup
    extern __shared__ double A[];   // [ns + R][128]: columns 0..ns-1 the matrix, ns..ns+R-1 the right-hand sides
    __shared__ double xs[kMaxQ * DIM];
    __shared__ int exs[128 * 3];
    __shared__ double red[2][2];
    __shared__ int redi[2][2];
    __shared__ double redm[NW];
    __shared__ int prow_of[128];    // pivot row of each elimination step
    const int tid = threadIdx.x;
    const int t = tid & 127, h = tid >> 7;
    const int lane = tid & 63, wv = tid >> 6;
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const int ns = q + m, nc = ns + R;
#define RB_AT(ptr, j) (ptr)[(j) * 128]

    double c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) c[d] = ctr[i * DIM + d];
    const int64_t jl = nbr[i * q + q - 1];
    const double s = sqrt(sqdist_exact<DIM>(c, xyz + jl * DIM));
    for (int a = tid; a < q; a += blockDim.x) {
        const int64_t j = nbr[i * q + a];
        for (int d = 0; d < DIM; ++d) xs[a * DIM + d] = (xyz[j * DIM + d] - c[d]) / s;
    }
    if (tid < m) {
        int ex[3];
        monomial_exponents<DIM>(tid, ex);
        exs[tid * 3 + 0] = ex[0];
        exs[tid * 3 + 1] = ex[1];
        exs[tid * 3 + 2] = ex[2];
    }
    __syncthreads();

    double *row = A + t;   // RB_AT(row, j): entry (t, j)
    double amax = 0.0;
    double mine[3] = {0, 0, 0};
    int myex[3] = {0, 0, 0};
    if (t < ns) {
        if (t < q)
            for (int d = 0; d < DIM; ++d) mine[d] = xs[t * DIM + d];
        if (t >= q) {
            myex[0] = exs[(t - q) * 3 + 0];
            myex[1] = exs[(t - q) * 3 + 1];
            myex[2] = exs[(t - q) * 3 + 2];
        }
        for (int b = h; b < ns; b += kRowThreads) {
            double v = 0.0;
            if (t < q) {
                if (b < q) {
                    const double r = sqrt(sqdist_exact<DIM>(mine, xs + b * DIM));
                    v = (phs == 3) ? r * r * r : r * r * r * r * r;
                } else {
                    v = monomial<DIM>(exs + (b - q) * 3, mine);
                }
            } else if (b < q) {
                v = monomial<DIM>(myex, xs + b * DIM);
            }
            RB_AT(row, b) = v;
            amax = fmax(amax, fabs(v));
        }
        if (h == 0) {
            double rhs[R];
#pragma unroll
            for (int r = 0; r < R; ++r) rhs[r] = 0.0;
            if (INTERP) {
                if (t < q) {
                    double rr = 0.0;
                    for (int d = 0; d < DIM; ++d) rr = rr + mine[d] * mine[d];
                    const double r = sqrt(rr);
                    rhs[0] = (phs == 3) ? r * r * r : r * r * r * r * r;
                } else {
                    rhs[0] = (myex[0] + myex[1] + myex[2] == 0) ? 1.0 : 0.0;
                }
            } else if (t < q) {
                double rr = 0.0;
                for (int d = 0; d < DIM; ++d) rr = rr + mine[d] * mine[d];
                const double r = sqrt(rr);
                const double rp2 = (phs == 3) ? r : r * r * r;
#pragma unroll
                for (int d = 0; d < DIM; ++d) rhs[d] = -(double)phs * rp2 * mine[d];
                rhs[R - 1] = (double)(phs * (phs + DIM - 2)) * rp2;
            } else {
                const int tot = myex[0] + myex[1] + myex[2];
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    if (tot == 1 && myex[d] == 1) rhs[d] = 1.0;
                    if (tot == 2 && myex[d] == 2) rhs[R - 1] = 2.0;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) RB_AT(row, ns + r) = rhs[r];
        }
    }
    amax = wave_max(amax);
    if (lane == 0) redm[wv] = amax;
    __syncthreads();
    amax = 0.0;
#pragma unroll
    for (int u = 0; u < NW; ++u) amax = fmax(amax, redm[u]);

    // LU with partial pivoting (largest |a|, ties to the lowest row); a row
    // that has served as pivot keeps its U part and is no longer updated
    bool active = t < ns;
    int mystep = -1;
    bool singular = false;
    for (int k = 0; k < ns; ++k) {
        const int buf = k & 1;
        if (h == 0) {
            const double v = active ? fabs(RB_AT(row, k)) : -1.0;
            const double mx_w = wave_max(v);
            const uint64_t msk = __ballot(active && v == mx_w);
            if (lane == 0) {
                red[buf][wv] = mx_w;
                redi[buf][wv] = msk ? wv * 64 + (__ffsll((unsigned long long)msk) - 1) : INT_MAX;
            }
        }
        __syncthreads();   // every row's step k-1 update and both candidates are visible
        const double mx = fmax(red[buf][0], red[buf][1]);
        const int p = (red[buf][0] >= red[buf][1]) ? redi[buf][0] : redi[buf][1];
        if (!(mx > 1e-13 * amax)) singular = true;
        if (t == p) {
            active = false;
            mystep = k;
            if (h == 0) prow_of[k] = t;
        }
        const double *pr = A + p;
        const double piv = singular ? 1.0 : RB_AT(pr, k);
        if (active) {
            // rw and pp are different rows (the pivot row is inactive)
            double *__restrict__ rw = row;
            const double *__restrict__ pp = pr;
            const double l = RB_AT(rw, k) / piv;
            int j = k + 1 + h;
            for (; j + kRowThreads < nc; j += 2 * kRowThreads) {
                const double p0 = RB_AT(pp, j), p1 = RB_AT(pp, j + kRowThreads);
                const double r0 = RB_AT(rw, j), r1 = RB_AT(rw, j + kRowThreads);
                RB_AT(rw, j) = fma(-l, p0, r0);
                RB_AT(rw, j + kRowThreads) = fma(-l, p1, r1);
            }
            if (j < nc) RB_AT(rw, j) = fma(-l, RB_AT(pp, j), RB_AT(rw, j));
        }
    }

    // back substitution by the h = 0 threads; thread c keeps unknown c
    double xout[R];
#pragma unroll
    for (int r = 0; r < R; ++r) xout[r] = 0.0;
    for (int k = ns - 1; k >= 0; --k) {
        __syncthreads();   // the pivot row's right-hand sides are final for step k
        if (h != 0) continue;
        const double *pr = A + prow_of[k];
        const double dgl = singular ? 1.0 : RB_AT(pr, k);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double xk = RB_AT(pr, ns + r) / dgl;
            if (t == k) xout[r] = xk;
            if (mystep >= 0 && mystep < k) RB_AT(row, ns + r) = fma(-RB_AT(row, k), xk, RB_AT(row, ns + r));
        }
    }
#undef RB_AT

    if (h == 0 && t < q) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double sc = INTERP ? 1.0 : ((r < DIM) ? s : s * s);
            w[(int64_t)r * n * q + i * q + t] = xout[r] / sc;
        }
    }
    if (singular && tid == 0) atomicMin((unsigned long long *)bad, (unsigned long long)i);
}

// ---- blocked Gauss-Jordan with FP64 MFMA trailing updates ------------------
//
// The same saddle systems, solved by Gauss-Jordan elimination with partial
// pivoting in panels of four columns. A panel is factored by one wavefront
// (pivot search, multipliers, updates of the panel's own columns); the rest of
// the augmented matrix then takes the panel's rank-4 update, one
// v_mfma_f64_16x16x4 per 16 x 16 tile. Rows never move: a row that has served
// as pivot stays where it is, and Gauss-Jordan eliminates each pivot column
// from every other row, including earlier pivot rows, so the matrix ends as a
// permuted diagonal and no back substitution follows; unknown k is the pivot
// row's right-hand side over its pivot. The pivot rule is that of the LU
// kernels above (largest |a| among rows not yet pivots, ties to the lowest row;
// singular below 1e-13 max|A|).
//
// The matrix lives in LDS tile by tile in the MFMA accumulator layout, so a
// tile's C operand is two 16-byte reads per lane without bank conflicts.

typedef double v4d __attribute__((ext_vector_type(4)));

// LDS slot of entry (i, j): tile (i / 16, j / 16) holds 256 doubles; within a
// tile, lane 16 * (i % 4) + j % 16 keeps rows 4 v + l / 16 at v = (i % 16) / 4
// (the 16x16x4 FP64 MFMA's C/D layout on gfx950: column l % 16, rows
// l / 16, 4 + l / 16, 8 + l / 16, 12 + l / 16 in its four registers).
__device__ inline int gj_slot(int i, int j, int tc)
{
    return ((((i >> 4) * tc + (j >> 4)) * 64 + 16 * (i & 3) + (j & 15)) << 2) + ((i & 15) >> 2);
}

// Entry (i, j) of the augmented system [A | B] of a point: rows and columns
// beyond ns (and beyond ns + R) are zero padding. xs holds the scaled cloud
// (q x DIM), exs the monomial exponents.
template <int DIM, bool INTERP>
__device__ inline double gj_entry(int i, int j, int q, int ns, int phs, const double *xs, const int *exs)
{
    constexpr int R = INTERP ? 1 : DIM + 1;
    if (i >= ns || j >= ns + R) return 0.0;
    if (j < ns) {
        if (i < q) {
            if (j < q) {
                const double r = sqrt(sqdist_exact<DIM>(xs + i * DIM, xs + j * DIM));
                return (phs == 3) ? r * r * r : r * r * r * r * r;
            }
            return monomial<DIM>(exs + (j - q) * 3, xs + i * DIM);
        }
        if (j < q) return monomial<DIM>(exs + (i - q) * 3, xs + j * DIM);
        return 0.0;
    }
    const int r = j - ns;
    if (INTERP) {
        if (i < q) {
            double rr = 0.0;
            for (int d = 0; d < DIM; ++d) rr = rr + xs[i * DIM + d] * xs[i * DIM + d];
            const double rad = sqrt(rr);
            return (phs == 3) ? rad * rad * rad : rad * rad * rad * rad * rad;
        }
        const int *ex = exs + (i - q) * 3;
        return (ex[0] + ex[1] + ex[2] == 0) ? 1.0 : 0.0;
    }
    if (i < q) {
        double rr = 0.0;
        for (int d = 0; d < DIM; ++d) rr = rr + xs[i * DIM + d] * xs[i * DIM + d];
        const double rad = sqrt(rr);
        const double rp2 = (phs == 3) ? rad : rad * rad * rad;
        if (r < DIM) return -(double)phs * rp2 * xs[i * DIM + r];
        return (double)(phs * (phs + DIM - 2)) * rp2;
    }
    const int *ex = exs + (i - q) * 3;
    const int tot = ex[0] + ex[1] + ex[2];
    if (r < DIM) return (tot == 1 && ex[r] == 1) ? 1.0 : 0.0;
    int two = 0;
    for (int d = 0; d < DIM; ++d) two += (ex[d] == 2);
    return (tot == 2 && two == 1) ? 2.0 : 0.0;
}

// LDS bytes of one system: matrix tiles, two panels' multipliers, pivots,
// two panels' pivot-row multipliers, the scaled cloud.
__host__ __device__ inline size_t gj_lds_bytes(int q, int ns, int nc, int dim)
{
    const int tr = (ns + 15) >> 4, tc = (nc + 15) >> 4;
    return sizeof(double) * ((size_t)tr * tc * 256 + 2 * (size_t)tr * 64 + (size_t)ns + 32 + (size_t)q * dim);
}

// Factor the panel of columns c0 .. c0 + np - 1 (np <= 4; wavefront 0): rows
// lane + 64 h in registers, pivot by the rule above, every row but the pivot
// eliminates the column from the panel's later columns. Writes -L to Lbuf in the
// MFMA A layout, the pivot rows' multipliers for earlier panel columns to lpb,
// and the pivot rows and values.
// ld(i, cc) gives entry (i, c0 + cc) for the rows i < rows.
template <int RPL, typename Load>
__device__ inline void gj_factor_panel_with(Load ld, int rows, int c0, int np, bool *act, double amax,
                                            bool &singular, double *Lbuf, double *lpb, int *prow, double *pv,
                                            int *sflag, int lane)
{
    double a[RPL][4], l[RPL][4];
#pragma unroll
    for (int h = 0; h < RPL; ++h)
#pragma unroll
        for (int cc = 0; cc < 4; ++cc) {
            const int i = lane + 64 * h;
            a[h][cc] = (cc < np && i < rows) ? ld(i, cc) : 0.0;
            l[h][cc] = 0.0;
        }
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        if (cc < np) {
            double best = -1.0;
#pragma unroll
            for (int h = 0; h < RPL; ++h) best = fmax(best, act[h] ? fabs(a[h][cc]) : -1.0);
            const double mx = wave_max_bcast(best);
            // 1 / |pivot| = 1 / mx (hardware reciprocal, two Newton steps),
            // started while the pivot row is still being found; every step is
            // odd in its argument, so the signed reciprocal is its negation
            // for a negative pivot, bit for bit
            double rm = __builtin_amdgcn_rcp(mx);
            rm = fma(rm, fma(-mx, rm, 1.0), rm);
            rm = fma(rm, fma(-mx, rm, 1.0), rm);
            int p = 0;
#pragma unroll
            for (int h = RPL - 1; h >= 0; --h) {
                const uint64_t msk = __ballot(act[h] && fabs(a[h][cc]) == mx);
                if (msk) p = 64 * h + (__ffsll((unsigned long long)msk) - 1);
            }
            if (!(mx > 1e-13 * amax)) singular = true;
            const int ph = p >> 6, pl = p & 63;
            double prw[4];
#pragma unroll
            for (int c2 = 0; c2 < 4; ++c2) {
                double src = a[0][c2];
#pragma unroll
                for (int h = 1; h < RPL; ++h)
                    if (ph == h) src = a[h][c2];
                prw[c2] = readlane_d(src, pl);
            }
            const double piv = singular ? 1.0 : prw[cc];
            const double rp = singular ? 1.0 : (prw[cc] < 0.0 ? -rm : rm);
#pragma unroll
            for (int h = 0; h < RPL; ++h) {
                const bool me = (lane + 64 * h) == p;
                if (me) act[h] = false;
                const double mul = me ? 0.0 : a[h][cc] * rp;
                l[h][cc] = mul;
#pragma unroll
                for (int c2 = cc + 1; c2 < 4; ++c2) a[h][c2] = fma(-mul, prw[c2], a[h][c2]);
                if (me)
#pragma unroll
                    for (int c2 = 0; c2 < cc; ++c2) lpb[cc * 4 + c2] = l[h][c2];
            }
            if (lane == 0) {
                prow[c0 + cc] = p;
                pv[c0 + cc] = piv;
                *sflag = singular;
            }
        }
    }
#pragma unroll
    for (int h = 0; h < RPL; ++h) {
        const int i = lane + 64 * h;
        if (i < rows)
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) Lbuf[(i >> 4) * 64 + (i & 15) + 16 * cc] = -l[h][cc];
    }
}

template <int RPL>
__device__ inline void gj_factor_panel(const double *M, int tr, int tc, int c0, int np, bool *act, double amax,
                                       bool &singular, double *Lbuf, double *lpb, int *prow, double *pv, int *sflag,
                                       int lane)
{
    gj_factor_panel_with<RPL>([=](int i, int cc) { return M[gj_slot(i, c0 + cc, tc)]; }, tr * 16, c0, np, act,
                              amax, singular, Lbuf, lpb, prow, pv, sflag, lane);
}

// Panel c0's rank-np update of tile column J, by the one wavefront that owns
// the column for this panel: its B operand holds the panel's U rows, by forward
// substitution over the pivot rows (u_c[j] = a[p_c][j] - sum_{c' < c}
// L[p_c][c'] u_c'[j]), all read before the column's first write; then one MFMA
// per row tile. Columns up to the panel's last get B = 0 and stay as they are.
__device__ inline void gj_update_column(double *M, int tr, int tc, int J, int c0, int np, const int *prow,
                                        const double *lpb, const double *Lbuf, int lane)
{
    const int cend = c0 + np, cl = lane >> 4, j = 16 * J + (lane & 15);
    double u[4], bv = 0.0;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
        double x = 0.0;
        if (cc < np && j >= cend) {
            x = M[gj_slot(prow[c0 + cc], j, tc)];
#pragma unroll
            for (int c2 = 0; c2 < cc; ++c2) x = fma(-lpb[cc * 4 + c2], u[c2], x);
        }
        u[cc] = x;
        if (cc == cl) bv = x;
    }
    for (int I = 0; I < tr; ++I) {
        const double av = Lbuf[I * 64 + lane];
        double2 *cp = (double2 *)(M + (((I * tc + J) * 64 + lane) << 2));
        const double2 c01 = cp[0], c23 = cp[1];
        v4d acc = {c01.x, c01.y, c23.x, c23.y};
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        cp[0] = make_double2(acc[0], acc[1]);
        cp[1] = make_double2(acc[2], acc[3]);
    }
}

// NW wavefronts per system; RPL rows per lane in the panel factorization
// (ns <= 64 * RPL).
template <int DIM, bool INTERP, int NW, int RPL>
__global__ __launch_bounds__(64 * NW) void weights_kernel_gj(const double *__restrict__ xyz,
                                                             const double *__restrict__ ctr,
                                                             const int32_t *__restrict__ nbr, int64_t n, int q, int m,
                                                             int phs, double *__restrict__ w,
                                                             int64_t *__restrict__ bad)
{
    constexpr int R = INTERP ? 1 : DIM + 1;
    constexpr int NT = 64 * NW;
    extern __shared__ __attribute__((aligned(16))) double gsm[];
    __shared__ int exs[128 * 3];
    __shared__ int prow[128];
    __shared__ double redm[NW];
    __shared__ int sflag;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t i0 = blockIdx.x;
    if (i0 >= n) return;
    const int ns = q + m, nc = ns + R;
    const int tr = (ns + 15) >> 4, tc = (nc + 15) >> 4;
    double *M = gsm;                      // tr * tc tiles of 256
    double *Lb = M + tr * tc * 256;       // [2][tr][64]: -L of a panel in the MFMA A layout
    double *pv = Lb + 2 * tr * 64;        // [ns] pivot values
    double *lp = pv + ns;                 // [2][4][4] multipliers of a panel's pivot rows
    double *xs = lp + 32;                 // [q][DIM] scaled cloud

    // centre and scale: s = distance to the q-th neighbour (interpolation:
    // to the farthest cloud point, the same point in distance order)
    double c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) c[d] = ctr[i0 * DIM + d];
    const int64_t jl = nbr[i0 * q + q - 1];
    const double s = sqrt(sqdist_exact<DIM>(c, xyz + jl * DIM));
    for (int a = tid; a < q; a += NT) {
        const int64_t j = nbr[i0 * q + a];
        for (int d = 0; d < DIM; ++d) xs[a * DIM + d] = (xyz[j * DIM + d] - c[d]) / s;
    }
    if (tid < m) {
        int ex[3];
        monomial_exponents<DIM>(tid, ex);
        exs[tid * 3 + 0] = ex[0];
        exs[tid * 3 + 1] = ex[1];
        exs[tid * 3 + 2] = ex[2];
    }
    __syncthreads();

    // the matrix, slot by slot (slot order: conflict-free LDS writes)
    double amax = 0.0;
    const int nslot = tr * tc * 256;
    for (int e = tid; e < nslot; e += NT) {
        const int v = e & 3, l = (e >> 2) & 63, t = e >> 8;
        const int I = t / tc, J = t - I * tc;
        const int i = 16 * I + 4 * v + (l >> 4), j = 16 * J + (l & 15);
        const double a = gj_entry<DIM, INTERP>(i, j, q, ns, phs, xs, exs);
        M[e] = a;
        if (j < ns) amax = fmax(amax, fabs(a));
    }
    amax = wave_max_dpp(amax);
    if (lane == 0) redm[wv] = amax;
    __syncthreads();
    amax = 0.0;
#pragma unroll
    for (int u = 0; u < NW; ++u) amax = fmax(amax, redm[u]);

    bool act[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) act[h] = lane + 64 * h < ns;
    bool singular = false;
    if (tid == 0) sflag = 0;   // ordered before its readers by the panels' barriers
    // Look-ahead: while the other wavefronts apply panel c0's update to their
    // tile columns, wavefront 0 updates tile column J0 (which holds the next
    // panel) and factors the next panel, so one barrier per panel orders all.
    // Lb and lp are double-buffered by panel parity.
    if (wv == 0) gj_factor_panel<RPL>(M, tr, tc, 0, min(4, ns), act, amax, singular, Lb, lp, prow, pv, &sflag, lane);
    __syncthreads();
    for (int c0 = 0; c0 < ns; c0 += 4) {
        const int np = min(4, ns - c0), cend = c0 + np, J0 = cend >> 4, buf = (c0 >> 2) & 1;
        const double *Lcur = Lb + buf * tr * 64;
        const double *lcur = lp + buf * 16;
        if (wv == 0) {
            if (J0 < tc) gj_update_column(M, tr, tc, J0, c0, np, prow, lcur, Lcur, lane);
            if (cend < ns)
                gj_factor_panel<RPL>(M, tr, tc, cend, min(4, ns - cend), act, amax, singular,
                                     Lb + (buf ^ 1) * tr * 64, lp + (buf ^ 1) * 16, prow, pv, &sflag, lane);
        }
        if (NW == 1 || wv > 0) {
            const int step = (NW == 1) ? 1 : NW - 1;
            for (int J = J0 + ((NW == 1) ? 1 : wv); J < tc; J += step)
                gj_update_column(M, tr, tc, J, c0, np, prow, lcur, Lcur, lane);
        }
        __syncthreads();
    }

    // unknown k = right-hand side of its pivot row over the pivot
    singular = sflag != 0;
    for (int k = tid; k < q; k += NT) {
        const int p = prow[k];
        const double dg = singular ? 1.0 : pv[k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double x = M[gj_slot(p, ns + r, tc)] / dg;
            const double sc = INTERP ? 1.0 : ((r < DIM) ? s : s * s);
            w[(int64_t)r * n * q + i0 * q + k] = INTERP ? x : x / sc;
        }
    }
    if (singular && tid == 0) atomicMin((unsigned long long *)bad, (unsigned long long)i0);
}

// Calls f(std::integral_constant<int, k>) for k = 0 .. N - 1, so that f can
// index register arrays with k.
template <int K>
struct IntC {
    static constexpr int value = K;
};
template <int N, int K = 0, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    if constexpr (K < N) {
        f(IntC<K>{});
        static_for<N, K + 1>(f);
    }
}

// Systems of 65 unknowns and up, at most 128 columns with the right-hand
// sides, with the matrix in registers: TR x TC tiles of 16 x 16 in the MFMA
// accumulator layout (lane l: column l % 16, rows 4 v + l / 16 in register
// v), tile column J held by wavefront J % NW, and the same Gauss-Jordan in
// panels of four columns as
// the kernel above. Per panel, the panel's owner passes its columns through
// LDS to the register factorisation (pivot rule, multipliers, -L in the A
// layout); every wavefront passes its part of the raw pivot rows through LDS to
// its B operands (forward substitution over the pivot rows), and every tile
// takes its rank-4 update in one MFMA. With no matrix in LDS, three or four
// systems share a CU and one's serial panel chain overlaps the others'
// updates. WPE is the wavefronts per SIMD that the register budget allows.
template <int DIM, bool INTERP, int TR, int TC, int NW, int WPE>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(WPE))) void weights_kernel_gjr(
    const double *__restrict__ xyz, const double *__restrict__ ctr, const int32_t *__restrict__ nbr, int64_t n, int q,
    int m, int phs, double *__restrict__ w, int64_t *__restrict__ bad)
{
    constexpr int R = INTERP ? 1 : DIM + 1;
    constexpr int RPL = (TR * 16 + 63) / 64;
    constexpr int TCW = (TC + NW - 1) / NW;   // tile columns per wavefront
    constexpr int NT = 64 * NW;
    __shared__ double xs[kMaxQ * DIM];
    __shared__ int exs[128 * 3];
    __shared__ __attribute__((aligned(16))) double S[TR * 256];   // a tile column; the right-hand sides
    __shared__ double P[TR * 64];                                  // the panel: row i, column c0 + cc at 4 i + cc
    __shared__ double Lb[2][TR * 64];                              // -L of a panel, MFMA A layout (by parity)
    __shared__ double Ur[NW][4][TCW * 16];                         // raw pivot rows, a wavefront's tile columns
    __shared__ double lp[2][16];
    __shared__ double pv[TR * 16];
    __shared__ int prow[TR * 16];
    __shared__ double redm[NW];
    __shared__ int sflag;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, g = lane >> 4, cl = lane & 15;
    const int64_t i0 = blockIdx.x;
    if (i0 >= n) return;
    const int ns = q + m;

    double c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) c[d] = ctr[i0 * DIM + d];
    const int64_t jl = nbr[i0 * q + q - 1];
    const double s = sqrt(sqdist_exact<DIM>(c, xyz + jl * DIM));
    for (int a = tid; a < q; a += NT) {
        const int64_t j = nbr[i0 * q + a];
        for (int d = 0; d < DIM; ++d) xs[a * DIM + d] = (xyz[j * DIM + d] - c[d]) / s;
    }
    for (int a = tid; a < m; a += NT) {
        int ex[3];
        monomial_exponents<DIM>(a, ex);
        exs[a * 3 + 0] = ex[0];
        exs[a * 3 + 1] = ex[1];
        exs[a * 3 + 2] = ex[2];
    }
    if (tid == 0) sflag = 0;
    __syncthreads();

    // the matrix, a tile column at a time through LDS (entries in slot order),
    // each column into its owner's registers
    v4d T[TR][TCW];
    double amax = 0.0;
#pragma unroll
    for (int J = 0; J < TC; ++J) {
#pragma unroll 1
        for (int e = tid; e < TR * 256; e += NT) {
            const int v = e & 3, l = (e >> 2) & 63, I = e >> 8;
            const int i = 16 * I + 4 * v + (l >> 4), j = 16 * J + (l & 15);
            const double a = gj_entry<DIM, INTERP>(i, j, q, ns, phs, xs, exs);
            S[e] = a;
            if (j < ns) amax = fmax(amax, fabs(a));
        }
        __syncthreads();
        if (wv == J % NW)
#pragma unroll
            for (int I = 0; I < TR; ++I) {
                const double2 *sp = (const double2 *)(S + ((I * 64 + lane) << 2));
                const double2 a01 = sp[0], a23 = sp[1];
                T[I][J / NW] = (v4d){a01.x, a01.y, a23.x, a23.y};
            }
        __syncthreads();
    }
    amax = wave_max_dpp(amax);
    if (lane == 0) redm[wv] = amax;
    __syncthreads();
    amax = 0.0;
#pragma unroll
    for (int u = 0; u < NW; ++u) amax = fmax(amax, redm[u]);

    bool act[RPL];
#pragma unroll
    for (int h = 0; h < RPL; ++h) act[h] = lane + 64 * h < ns;

    // Factor the panel at column c1 (its owner only): its columns through LDS
    // to the register factorisation, -L and the pivot-row multipliers into the
    // buffers of parity b.
    auto factor = [&](int c1, int b) {
        const int J1 = c1 >> 4, sp = (c1 >> 2) & 3;
        const int cc = cl - 4 * sp;
        const bool inp = cc >= 0 && cc < 4;
#pragma unroll
        for (int jj = 0; jj < TCW; ++jj)
            if (jj == J1 / NW) {
                if (inp)
#pragma unroll
                    for (int I = 0; I < TR; ++I)
#pragma unroll
                        for (int v = 0; v < 4; ++v) P[(16 * I + 4 * v + g) * 4 + cc] = T[I][jj][v];
            }
        bool singular = sflag != 0;
        gj_factor_panel_with<RPL>([&](int i, int cc2) { return P[i * 4 + cc2]; }, TR * 16, c1, min(4, ns - c1), act,
                                  amax, singular, Lb[b], lp[b], prow, pv, &sflag, lane);
    };
    if (wv == 0) factor(0, 0);
    __syncthreads();

    // One runtime loop over the panels; tile accesses stay constant-indexed in
    // loops over the wavefront's tile columns under uniform tests. Look-ahead:
    // the owner of the next panel's tile column updates that column first and
    // factors the next panel while the other wavefronts update theirs, so one
    // barrier per panel orders everything.
#pragma unroll 1
    for (int c0 = 0; c0 < ns; c0 += 4) {
        const int np = min(4, ns - c0), cend = c0 + np, J0 = c0 >> 4, buf = (c0 >> 2) & 1;
        // the panel's pivot rows leave the active set; the raw pivot rows of
        // this wavefront's tile columns to its LDS rows (row p sits in
        // register (p % 16) / 4 of row tile p / 16, lanes 16 (p % 4) + 0..15)
        for (int cc = 0; cc < np; ++cc) {
            const int p = __builtin_amdgcn_readfirstlane(prow[c0 + cc]);
#pragma unroll
            for (int h = 0; h < RPL; ++h)
                if (lane + 64 * h == p) act[h] = false;
            const int pI = p >> 4, pv4 = (p & 15) >> 2;
            const bool mine = g == (p & 3);
#pragma unroll
            for (int I = 0; I < TR; ++I)
                if (I == pI)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (v == pv4) {
                            if (mine)
#pragma unroll
                                for (int jj = 0; jj < TCW; ++jj) Ur[wv][cc][16 * jj + cl] = T[I][jj][v];
                        }
        }
        double av[TR], lpv[6];
#pragma unroll
        for (int I = 0; I < TR; ++I) av[I] = Lb[buf][I * 64 + lane];
        // the pivot rows' multipliers of earlier panel columns: (1,0) (2,0)
        // (2,1) (3,0) (3,1) (3,2)
        lpv[0] = lp[buf][4];
        lpv[1] = lp[buf][8];
        lpv[2] = lp[buf][9];
        lpv[3] = lp[buf][12];
        lpv[4] = lp[buf][13];
        lpv[5] = lp[buf][14];
        // rank-4 update of tile column jj (columns left of the panel's tile
        // column are finished and skipped; B is zero up to the panel's end)
        auto update = [&](auto jjc) {
            constexpr int jj = decltype(jjc)::value;
            const int J = NW * jj + wv;
            if (J >= TC || J < J0) return;
            const int j = 16 * J + cl;
            double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
            if (j >= cend) {
                const double *ur = &Ur[wv][0][16 * jj + cl];
                u0 = ur[0];
                if (np > 1) u1 = fma(-lpv[0], u0, ur[TCW * 16]);
                if (np > 2) u2 = fma(-lpv[2], u1, fma(-lpv[1], u0, ur[2 * TCW * 16]));
                if (np > 3) u3 = fma(-lpv[5], u2, fma(-lpv[4], u1, fma(-lpv[3], u0, ur[3 * TCW * 16])));
            }
            const double bv = (g == 0) ? u0 : (g == 1) ? u1 : (g == 2) ? u2 : u3;
#pragma unroll
            for (int I = 0; I < TR; ++I)
                T[I][jj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[I], bv, T[I][jj], 0, 0, 0);
        };
        const int J1 = cend >> 4;
        const bool ahead = cend < ns && wv == J1 % NW;
        if (ahead) {
            static_for<TCW>([&](auto jjc) {
                if (decltype(jjc)::value == J1 / NW) update(jjc);
            });
            factor(cend, buf ^ 1);
            static_for<TCW>([&](auto jjc) {
                if (decltype(jjc)::value != J1 / NW) update(jjc);
            });
        } else {
            static_for<TCW>([&](auto jjc) { update(jjc); });
        }
        __syncthreads();
    }

    // unknown k = right-hand side of its pivot row over the pivot
#pragma unroll
    for (int jj = 0; jj < TCW; ++jj) {
        const int r = 16 * (NW * jj + wv) + cl - ns;
        if (r >= 0 && r < R)
#pragma unroll
            for (int I = 0; I < TR; ++I)
#pragma unroll
                for (int v = 0; v < 4; ++v) S[(16 * I + 4 * v + g) * 4 + r] = T[I][jj][v];
    }
    __syncthreads();
    const bool singular = sflag != 0;
    for (int k = tid; k < q; k += NT) {
        const int p = prow[k];
        const double dg = singular ? 1.0 : pv[k];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double x = S[p * 4 + r] / dg;
            const double sc = INTERP ? 1.0 : ((r < DIM) ? s : s * s);
            w[(int64_t)r * n * q + i0 * q + k] = INTERP ? x : x / sc;
        }
    }
    if (singular && tid == 0) atomicMin((unsigned long long *)bad, (unsigned long long)i0);
}

// The register Gauss-Jordan kernel for tiles (TR, TC) = (ceil(ns / 16),
// ceil((ns + R) / 16)) when an instance exists; false otherwise. NW, the
// wavefronts per system, and WPE, the wavefronts the compiler budgets per
// SIMD (three: 168 VGPRs), set how many systems share a CU: three wavefronts
// up to six tile columns (four systems per CU), four at seven and eight
// (three per CU; the widest shapes spill up to 40 dwords). Measured on
// MI355X: 2D k = 6 (84 unknowns) 7.7 ms, against 8.0 with two wavefronts at
// two per SIMD and 12.3 with four; 3D k = 4 (105 unknowns) 17.8 ms, against
// 20.8 at two per SIMD and 24.3 with two wavefronts; 8 x 8 tiles (121
// unknowns) 17.5 ms at three per SIMD, 20.2 at two.
template <bool INTERP>
bool launch_gjr(int dim, int ns, int nc, dim3 grid, hipStream_t s, const double *xyz, const double *ctr,
                const int32_t *nbr, int64_t n, int q, int m, int phs, double *w, int64_t *bad)
{
    const int tr = (ns + 15) >> 4, tc = (nc + 15) >> 4;
#define RB_GJR(TR_, TC_, NW_)                                                                              \
    if (tr == TR_ && tc == TC_) {                                                                          \
        constexpr int wpe = 3;                                                                             \
        if (dim == 2)                                                                                      \
            hipLaunchKernelGGL((weights_kernel_gjr<2, INTERP, TR_, TC_, NW_, wpe>), grid, dim3(64 * NW_), 0, s,   \
                               xyz, ctr, nbr, n, q, m, phs, w, bad);                                       \
        else                                                                                               \
            hipLaunchKernelGGL((weights_kernel_gjr<3, INTERP, TR_, TC_, NW_, wpe>), grid, dim3(64 * NW_), 0, s,   \
                               xyz, ctr, nbr, n, q, m, phs, w, bad);                                       \
        return true;                                                                                       \
    }
    RB_GJR(5, 5, 3)
    RB_GJR(5, 6, 3)
    RB_GJR(6, 6, 3)
    RB_GJR(6, 7, 4)
    RB_GJR(7, 7, 4)
    RB_GJR(7, 8, 4)
    RB_GJR(8, 8, 4)
#undef RB_GJR
    return false;
}

// out[f][j] = sum_a w[j][a] field_f[nbr[j][a]], in cloud order a = 0..q-1
__global__ __launch_bounds__(kBlock) void interp_apply(int64_t nq, int q, const int32_t *__restrict__ nbr,
                                                       const double *__restrict__ w, int nfield, int64_t n,
                                                       const double *__restrict__ fields, double *__restrict__ out)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= nq) return;
    for (int f = 0; f < nfield; ++f) {
        double acc = 0.0;
        for (int a = 0; a < q; ++a) acc = fma(w[j * q + a], fields[(int64_t)f * n + nbr[j * q + a]], acc);
        out[(int64_t)f * nq + j] = acc;
    }
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
            hipLaunchKernelGGL((weights_kernel<NSP_, 2, false>), grid, block, 0, s, xyz, xyz, nbr, n, q, m, phs, w,   \
                               bad_dev);                                                                  \
        else                                                                                              \
            hipLaunchKernelGGL((weights_kernel<NSP_, 3, false>), grid, block, 0, s, xyz, xyz, nbr, n, q, m, phs, w,   \
                               bad_dev);                                                                  \
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
    if (launch_gjr<false>(dim, ns, ns + dim + 1, grid, s, xyz, xyz, nbr, n, q, m, phs, w, bad_dev)) {
        RB_HIP(hipGetLastError());
        return RBFFD_OK;
    }
    if (ns <= 128) {
        // systems of 65-128 unknowns: the matrix lives in LDS
        const int R = dim + 1;
        int dev = 0, lim = 0;
        RB_HIP(hipGetDevice(&dev));
        RB_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const size_t gjl = gj_lds_bytes(q, ns, ns + R, dim);
        if (gjl + 2048 <= (size_t)lim) {
            // blocked Gauss-Jordan, MFMA trailing updates, four wavefronts
            if (dim == 2) {
                RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_gj<2, false, 4, 2>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)gjl));
                hipLaunchKernelGGL((weights_kernel_gj<2, false, 4, 2>), grid, dim3(256), gjl, s, xyz, xyz, nbr, n, q,
                                   m, phs, w, bad_dev);
            } else {
                RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_gj<3, false, 4, 2>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)gjl));
                hipLaunchKernelGGL((weights_kernel_gj<3, false, 4, 2>), grid, dim3(256), gjl, s, xyz, xyz, nbr, n, q,
                                   m, phs, w, bad_dev);
            }
            RB_HIP(hipGetLastError());
            return RBFFD_OK;
        }
        const size_t lds = sizeof(double) * (size_t)(ns + R) * 128;
        const size_t fixed = sizeof(double) * (kMaxQ * 3 + 4 + 2 * kRowThreads) + sizeof(int) * (128 * 3 + 4 + 128);
        if (lds + fixed > (size_t)lim)
            return fail(RBFFD_E_ARG, "collocation system needs " + std::to_string(lds + fixed) +
                                         " bytes of LDS per workgroup; the device allows " + std::to_string(lim));
        const dim3 block2(128 * kRowThreads);
        if (dim == 2) {
            RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_lds<2, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL((weights_kernel_lds<2, false>), grid, block2, lds, s, xyz, xyz, nbr, n, q, m, phs, w,
                               bad_dev);
        } else {
            RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_lds<3, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL((weights_kernel_lds<3, false>), grid, block2, lds, s, xyz, xyz, nbr, n, q, m, phs, w,
                               bad_dev);
        }
        RB_HIP(hipGetLastError());
        return RBFFD_OK;
    }
    return fail(RBFFD_E_ARG, "collocation systems larger than 128 are not supported");
}

// smallest instantiated register width >= ns (systems of at most 64 unknowns)
int weight_width(int ns)
{
    for (int wdt = 16; wdt <= 64; wdt += 8)
        if (ns <= wdt) return wdt;
    return 0;
}

int launch_weights_batched(int dim, int width, int count, const WeightSys *sys_dev, int64_t total_blocks,
                           int64_t *bad_dev, hipStream_t s)
{
    if (count <= 0 || total_blocks <= 0) return RBFFD_OK;
    if (total_blocks > INT_MAX) return fail(RBFFD_E_ARG, "too many points in one batched build");
    const dim3 grid((unsigned)total_blocks), block(64);
#define RB_WB(NSP_)                                                                                          \
    if (width == NSP_) {                                                                                     \
        if (dim == 2)                                                                                        \
            hipLaunchKernelGGL((weights_batched_kernel<NSP_, 2>), grid, block, 0, s, sys_dev, count, bad_dev); \
        else                                                                                                 \
            hipLaunchKernelGGL((weights_batched_kernel<NSP_, 3>), grid, block, 0, s, sys_dev, count, bad_dev); \
        RB_HIP(hipGetLastError());                                                                           \
        return RBFFD_OK;                                                                                     \
    }
    RB_WB(16)
    RB_WB(24)
    RB_WB(32)
    RB_WB(40)
    RB_WB(48)
    RB_WB(56)
    RB_WB(64)
#undef RB_WB
    return fail(RBFFD_E_ARG, "no register width " + std::to_string(width));
}

int launch_interp(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int64_t nq, const double *qxyz, int q,
                  const int32_t *nbr, int k, int phs, double *w, int64_t *bad_dev, int nfield, const double *fields,
                  double *out, hipStream_t s)
{
    (void)ctx;
    long mm = 1, den = 1;
    for (int i = 1; i <= dim; ++i) {
        mm *= (k + i);
        den *= i;
    }
    const int m = (int)(mm / den);
    const int ns = q + m;
    if (ns > 128) return fail(RBFFD_E_ARG, "collocation systems larger than 128 are not supported");
    const long long init = LLONG_MAX;
    RB_HIP(hipMemcpyAsync(bad_dev, &init, sizeof(init), hipMemcpyHostToDevice, s));
    if (nq == 0) return RBFFD_OK;
    // up to 64 unknowns: one wavefront per query point, the row in registers
    bool launched = false;
    const dim3 grid1((unsigned)nq), block1(64);
#define RB_INTERP(NSP_)                                                                                   \
    if (!launched && ns <= NSP_) {                                                                        \
        if (dim == 2)                                                                                     \
            hipLaunchKernelGGL((weights_kernel<NSP_, 2, true>), grid1, block1, 0, s, xyz, qxyz, nbr, nq, q, m, phs, \
                               w, bad_dev);                                                               \
        else                                                                                              \
            hipLaunchKernelGGL((weights_kernel<NSP_, 3, true>), grid1, block1, 0, s, xyz, qxyz, nbr, nq, q, m, phs, \
                               w, bad_dev);                                                               \
        launched = true;                                                                                  \
    }
    RB_INTERP(16)
    RB_INTERP(24)
    RB_INTERP(32)
    RB_INTERP(40)
    RB_INTERP(48)
    RB_INTERP(56)
    RB_INTERP(64)
#undef RB_INTERP
    int dev = 0, lim = 0;
    RB_HIP(hipGetDevice(&dev));
    RB_HIP(hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    if (!launched)
        launched = launch_gjr<true>(dim, ns, ns + 1, dim3((unsigned)nq), s, xyz, qxyz, nbr, nq, q, m, phs, w, bad_dev);
    if (!launched) {
        // 65-128 unknowns: one workgroup per query point, the matrix in LDS
        const size_t gjl = gj_lds_bytes(q, ns, ns + 1, dim);
        if (gjl + 2048 <= (size_t)lim) {
            if (dim == 2) {
                RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_gj<2, true, 4, 2>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)gjl));
                hipLaunchKernelGGL((weights_kernel_gj<2, true, 4, 2>), dim3((unsigned)nq), dim3(256), gjl, s, xyz,
                                   qxyz, nbr, nq, q, m, phs, w, bad_dev);
            } else {
                RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_gj<3, true, 4, 2>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)gjl));
                hipLaunchKernelGGL((weights_kernel_gj<3, true, 4, 2>), dim3((unsigned)nq), dim3(256), gjl, s, xyz,
                                   qxyz, nbr, nq, q, m, phs, w, bad_dev);
            }
            launched = true;
        }
    }
    if (!launched) {
        const size_t lds = sizeof(double) * (size_t)(ns + 1) * 128;
        const size_t fixed =
            sizeof(double) * (kMaxQ * 3 + 4 + 2 * kRowThreads) + sizeof(int) * (128 * 3 + 4 + 128);
        if (lds + fixed > (size_t)lim) return fail(RBFFD_E_ARG, "interpolation system does not fit the device's LDS");
        const dim3 grid((unsigned)nq), block(128 * kRowThreads);
        if (dim == 2) {
            RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_lds<2, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL((weights_kernel_lds<2, true>), grid, block, lds, s, xyz, qxyz, nbr, nq, q, m, phs, w,
                               bad_dev);
        } else {
            RB_HIP(hipFuncSetAttribute((const void *)weights_kernel_lds<3, true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
            hipLaunchKernelGGL((weights_kernel_lds<3, true>), grid, block, lds, s, xyz, qxyz, nbr, nq, q, m, phs, w,
                               bad_dev);
        }
    }
    RB_HIP(hipGetLastError());
    return launch_interp_apply(nq, q, nbr, w, nfield, n, fields, out, s);
}

int launch_interp_apply(int64_t nq, int q, const int32_t *nbr, const double *w, int nfield, int64_t n,
                        const double *fields, double *out, hipStream_t s)
{
    if (nfield <= 0 || nq == 0) return RBFFD_OK;
    hipLaunchKernelGGL(interp_apply, dim3((unsigned)((nq + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, nq, q, nbr, w,
                       nfield, n, fields, out);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

}  // namespace rbffd
