// Sparse matrix-vector products and preconditioned BiCGSTAB (Sec. 3: the
// momentum and pressure-correction equations are solved "using a
// preconditioned BiCGSTAB"; the preconditioner is the Jacobi diagonal applied
// on the right).
//
// Every kernel streams the sliced-ELL matrix with one thread per row: entry a of
// 64 consecutive rows is one contiguous run, so column indices and values are
// read fully coalesced, and the gathered vector entries of Morton-ordered points
// hit in cache. Each BiCGSTAB iteration is four kernels:
//   KV  v = A p-hat, r-hat.v                 (convergence test on ||r|| first)
//   KS  alpha; s = r - alpha v, s-hat = D^-1 s, s.s, r-hat.s
//   KT  t = A s-hat, t.s, t.t, r-hat.t       (or x += alpha p-hat if ||s|| is small)
//   KX  omega; x += alpha p-hat + omega s-hat; r = s - omega t; r.r; and the next
//       search direction p-hat = D^-1 r + beta (p-hat - omega D^-1 v), with
//       beta = (rho'/rho)(alpha/omega) and rho' = r-hat.r taken as
//       r-hat.s - omega r-hat.t (the same inner product, by linearity), so the
//       search-direction update needs no kernel of its own.
// Global dot products are finished redundantly by every block of the consuming
// kernel from per-block partials in a fixed order, so the scalars never travel
// to the host and results are deterministic run to run. The host only reads a
// small state record every few iterations to stop.
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace rbffd {

namespace {

// Per right-hand-side solver state. A kernel launch that finishes a solve
// records its launch sequence number in done_at; blocks of that same launch keep
// working (they may still owe updates of their rows), later launches skip.
// Fields written by block 0 during a launch are read by other blocks only in
// later launches.
struct KState {
    double rho;       // r-hat . r of the current iteration (set by KV)
    double rho_next;  // r-hat . r of the next iteration (set by KX, taken over by the next KV)
    double alpha, omega;
    double rr, bb;    // ||r||^2 (recursive) at the start of the last iteration, ||b||^2
    int done_at;      // 0 running, else sequence number of the launch that finished
    int iters;        // completed iterations
    int status;       // RBFFD_OK / RBFFD_E_BREAKDOWN
    int restart;      // r-hat was reset to r: rho = r.r at the next KV
    int refresh;      // r was replaced by a true residual: rho = r-hat.r at the next KV
    int fresh;        // batched systems: to be initialised by the next KB_INIT
    int moved;        // batched systems: block range changed, ||r||^2 is in rr
};

// BiCGSTAB kernels run 512-thread blocks on at most 512 blocks (two per CU),
// so that a consumer kernel re-reduces at most 512 partials per dot product;
// larger systems loop over rows. Measured at 1.06M rows: 258 us per iteration
// with 512 blocks, 272 us with 1024, 282 us with 256.
constexpr int kKB = 512;
constexpr int kKMaxBlocks = 512;
static_assert(kKMaxBlocks <= kMaxBlocks, "partial arrays hold kMaxBlocks entries");

__device__ inline double kblock_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kKB / 64; ++i) t += lds[i];
    return t;
}

__device__ inline bool finished_before(const KState &s, int phase) { return s.done_at != 0 && s.done_at < phase; }

enum { P_RHR = 0, P_RR, P_BB, P_RV, P_SS, P_RS, P_TS, P_TT, P_RT, P_COUNT };

struct Work {
    // vectors, [nrhs][npad] each
    void *r, *rh, *ph, *v, *s, *sh, *t;
    double *part;   // [P_COUNT][kMaxRhs][kMaxBlocks]
    KState *st;     // [kMaxRhs]
};

__device__ inline double *partial(double *base, int kind, int r) { return base + ((int64_t)kind * kMaxRhs + r) * kMaxBlocks; }

template <typename T>
__device__ inline int64_t row_base(int64_t i, int q) { return ((i >> 6) * (int64_t)q) * 64 + (i & 63); }

// Matrix loads. With NT set they are non-temporal: the values and column
// indices are read once per product, and keeping them out of the caches leaves
// the L2 and the Infinity Cache to the gathered vector and the Krylov vectors.
// That pays where the matrix outgrows the Infinity Cache (1.06M rows at q = 40:
// 255 -> 239 us per BiCGSTAB iteration) and costs where it would stay there
// (250k rows at q = 30: 45.8 -> 52.6 us), so matrix_nt() picks it by size.
template <bool NT, typename X>
__device__ inline X mload(const X *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NARROW, bool NT = false>
__device__ inline int32_t col_at(const ColIdx &ci, int64_t slot, int32_t cb)
{
    if constexpr (NARROW)
        return cb + (int32_t)mload<NT>(ci.col16 + slot);
    else
        return mload<NT>(ci.col + slot);
}

// acc[r] = sum_a A[i,a] x_r[col] for the right-hand sides with act[r]; entries in
// column order. The activity test sits outside the entry loop so the loop body
// is branch-free and the compiler can keep several column/value/gather loads in
// flight. Rows accumulate in FP64 also for FP32 operands: Laplacian-like rows
// cancel terms ~1/h^2 larger than their sum, and FP32 accumulation of that
// cancellation makes FP32 BiCGSTAB diverge on fine clouds.
template <bool NARROW, typename TM, typename TX, int NRHS, int U, bool NT>
__device__ inline void row_dot_cols(int64_t base, int q, const ColIdx &ci, int32_t cb, const TM *__restrict__ val,
                                    const TX *__restrict__ x, int64_t xs, const bool *act, bool all, double *acc)
{
    if (all) {
        double s[NRHS];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) s[r] = 0.0;
#pragma unroll U
        for (int a = 0; a < q; ++a) {
            const int64_t slot = base + (int64_t)a * 64;
            const int32_t c = col_at<NARROW, NT>(ci, slot, cb);
            const double v = (double)mload<NT>(val + slot);
#pragma unroll
            for (int r = 0; r < NRHS; ++r) s[r] = fma(v, (double)x[r * xs + c], s[r]);
        }
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[r] = s[r];
        return;
    }
    for (int r = 0; r < NRHS; ++r) {
        if (!act[r]) continue;
        double s1 = 0.0;
#pragma unroll 4
        for (int a = 0; a < q; ++a) {
            const int64_t slot = base + (int64_t)a * 64;
            s1 = fma((double)mload<NT>(val + slot), (double)x[r * xs + col_at<NARROW, NT>(ci, slot, cb)], s1);
        }
        acc[r] = s1;
    }
}

// U is the unroll depth of the entry loop. It changes only the schedule of the
// loads, never the order of the sums; row_unroll() picks it for a stencil width.
template <typename TM, typename TX, int NRHS, int U = 4, bool NT = false>
__device__ inline void row_dot(int64_t i, int q, const ColIdx &ci, const TM *__restrict__ val,
                               const TX *__restrict__ x, int64_t xs, const bool *act, double *acc)
{
    const int64_t base = row_base<TM>(i, q);
    bool all = true, any = false;
#pragma unroll
    for (int r = 0; r < NRHS; ++r) {
        all = all && act[r];
        any = any || act[r];
    }
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = 0.0;
    if (!any) return;
    // one 64-row slice per wavefront: the branch is uniform across the wave
    const int32_t cb = ci.cbase ? ci.cbase[i >> 6] : -1;
    if (cb >= 0)
        row_dot_cols<true, TM, TX, NRHS, U, NT>(base, q, ci, cb, val, x, xs, act, all, acc);
    else
        row_dot_cols<false, TM, TX, NRHS, U, NT>(base, q, ci, cb, val, x, xs, act, all, acc);
}

__device__ inline int logical_block() { return xcd_block(gridDim.x); }

// Unroll depth of the row loop in the SpMV kernels of the Krylov iteration.
// Measured at the two benchmark widths: q = 30 runs 3.5% faster unrolled by 3
// than by 4, q = 40 5% slower. Each kernel holds one loop (a run-time choice
// inside the kernel slowed the 3D iteration by 10%).
inline bool row_unroll3(int q) { return q % 3 == 0 && q % 4 != 0; }

// Non-temporal matrix loads for matrices beyond half of the 256 MB Infinity
// Cache (values of val_bytes plus up to 4-byte column indices per entry).
constexpr size_t kNtBytes = size_t(128) << 20;
inline bool matrix_nt(int64_t n, int q, size_t val_bytes) { return (size_t)pad64(n) * q * (val_bytes + 4) > kNtBytes; }

// ---- plain SpMV ------------------------------------------------------------
template <typename T, int U, bool NT>
__global__ __launch_bounds__(kBlock) void spmv_kernel(int64_t n, int q, ColIdx col,
                                                      const T *__restrict__ val, const T *__restrict__ x,
                                                      T *__restrict__ y)
{
    const int64_t i = (int64_t)logical_block() * kBlock + threadIdx.x;
    if (i >= n) return;
    const bool act[1] = {true};
    double acc[1];
    row_dot<T, T, 1, U, NT>(i, q, col, val, x, 0, act, acc);
    y[i] = (T)acc[0];
}

// ---- BiCGSTAB ---------------------------------------------------------------
// The state records, read at a kernel's start: their loads then overlap the
// partial loads. A field block 0 writes during a launch is read by other
// blocks only in later launches, so the early copy is the current value.
template <int NRHS>
__device__ inline void load_states(const KState *st, KState *out)
{
#pragma unroll
    for (int r = 0; r < NRHS; ++r) out[r] = st[r];
}

template <int NRHS>
__device__ inline bool all_done(const KState *st, int phase)
{
    bool d = true;
#pragma unroll
    for (int r = 0; r < NRHS; ++r) d = d && finished_before(st[r], phase);
    return d;
}

// Block sums of NV per-thread values, written as partial blk of NV arrays.
template <int NV>
__device__ inline void write_partials(const double *v, double *const *parts)
{
    __shared__ double red[NV][kKB / 64];
    double w[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) w[m] = v[m];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int m = 0; m < NV; ++m) w[m] += __shfl_xor(w[m], o, 64);
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0)
#pragma unroll
        for (int m = 0; m < NV; ++m) red[m][wv] = w[m];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int m = 0; m < NV; ++m) {
            double t = 0.0;
#pragma unroll
            for (int j = 0; j < kKB / 64; ++j) t += red[m][j];
            parts[m][blockIdx.x] = t;
        }
}

// Partials each thread loads per array: thread t holds entries t, t + kKB, ...
constexpr int kPartPer = (kKMaxBlocks + kKB - 1) / kKB;

// Sums of NV partial arrays (np entries each) in a fixed order, identical in
// every block, in two phases: the loads, then one block reduction. A kernel may
// issue its own row loads between the two, so that waiting for the partials
// does not also wait for those rows.
template <int NV>
__device__ inline void load_partials_n(const double *const *parts, int np, double (&ld)[NV][kPartPer])
{
#pragma unroll
    for (int j = 0; j < kPartPer; ++j) {
        const int i = threadIdx.x + j * kKB;
#pragma unroll
        for (int m = 0; m < NV; ++m) ld[m][j] = (i < np) ? parts[m][i] : 0.0;
    }
}

template <int NV>
__device__ inline void reduce_partials_n(const double (&ld)[NV][kPartPer], double *out)
{
    __shared__ double red[NV][kKB / 64];
    double v[NV];
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        v[m] = 0.0;
#pragma unroll
        for (int j = 0; j < kPartPer; ++j) v[m] += ld[m][j];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int m = 0; m < NV; ++m) v[m] += __shfl_xor(v[m], o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0)
#pragma unroll
        for (int m = 0; m < NV; ++m) red[m][w] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < kKB / 64; ++j) t += red[m][j];
        out[m] = t;
    }
}

template <int NV>
__device__ inline void sum_partials_n(const double *const *parts, int np, double *out)
{
    double ld[NV][kPartPer];
    load_partials_n<NV>(parts, np, ld);
    reduce_partials_n<NV>(ld, out);
}

// r = b - A x, r-hat = r, p-hat = D^-1 r; partials r.r and b.b
template <typename T, int NRHS>
__global__ __launch_bounds__(kKB) void k_init(int64_t n, int64_t np, int q, ColIdx col, const T *__restrict__ val,
                                              const T *__restrict__ dinv, const T *__restrict__ b, int64_t bs,
                                              const T *__restrict__ x, int64_t xs, T *__restrict__ r,
                                              T *__restrict__ rh, T *__restrict__ ph, double *__restrict__ part)
{
    double acc[2 * NRHS];
#pragma unroll
    for (int k = 0; k < 2 * NRHS; ++k) acc[k] = 0.0;
    bool act[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) act[k] = true;
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
        double ax[NRHS];
        row_dot<T, T, NRHS>(i, q, col, val, x, xs, act, ax);
        const T di = dinv[i];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            const double bi = (double)b[k * bs + i];
            const T ri = (T)(bi - ax[k]);
            r[k * np + i] = ri;
            rh[k * np + i] = ri;
            ph[k * np + i] = di * ri;
            acc[2 * k] += (double)ri * (double)ri;
            acc[2 * k + 1] += bi * bi;
        }
    }
    double *ps[2 * NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        ps[2 * k] = partial(part, P_RR, k);
        ps[2 * k + 1] = partial(part, P_BB, k);
    }
    write_partials<2 * NRHS>(acc, ps);
}

// KV: convergence test on ||r||; v = A p-hat; partial r-hat.v. With check_only
// set, only the test runs (after the last permitted iteration).
template <typename T, typename TM, int NRHS, int U, bool NT>
__global__ __launch_bounds__(kKB) void k_v(int64_t n, int64_t np, int q, ColIdx col, const TM *__restrict__ val,
                                           const T *__restrict__ rh, const T *__restrict__ ph, T *__restrict__ v,
                                           T *__restrict__ x, int64_t xs, double *__restrict__ part,
                                           KState *__restrict__ st, int nblk, double tol2, int check_only, int phase)
{
    KState st0[NRHS];
    load_states<NRHS>(st, st0);
    double sums[3 * NRHS];
    {
        const double *ps[3 * NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            ps[3 * k] = partial(part, P_RR, k);
            ps[3 * k + 1] = partial(part, P_BB, k);
            ps[3 * k + 2] = partial(part, P_RHR, k);
        }
        sum_partials_n<3 * NRHS>(ps, nblk, sums);
    }
    if (all_done<NRHS>(st0, phase)) return;
    bool act[NRHS], zero[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        const KState s = st0[k];
        const double rr = sums[3 * k], bb = sums[3 * k + 1];
        act[k] = !finished_before(s, phase);
        zero[k] = act[k] && bb == 0.0;
        const bool conv = act[k] && !zero[k] && rr <= tol2 * bb;
        if (act[k] && blockIdx.x == 0 && threadIdx.x == 0) {
            st[k].rr = rr;
            st[k].bb = bb;
            if (s.refresh)
                st[k].rho = sums[3 * k + 2];
            else if (s.iters == 0 || s.restart)
                st[k].rho = rr;
            else
                st[k].rho = s.rho_next;
            if (zero[k] || conv) {
                st[k].done_at = phase;
                st[k].status = RBFFD_OK;
            }
        }
        if (conv || check_only) act[k] = false;
    }
    double srv[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) srv[k] = 0.0;
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
        bool sp[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            sp[k] = act[k] && !zero[k];
            if (act[k] && zero[k]) x[k * xs + i] = (T)0;
        }
        double av[NRHS];
        row_dot<TM, T, NRHS, U, NT>(i, q, col, val, ph, np, sp, av);
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            if (!sp[k]) continue;
            const T vi = (T)av[k];
            v[k * np + i] = vi;
            srv[k] += (double)rh[k * np + i] * (double)vi;
        }
    }
    double *ps[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) ps[k] = partial(part, P_RV, k);
    write_partials<NRHS>(srv, ps);
}

// KS: alpha = rho / r-hat.v; s = r - alpha v; s-hat = D^-1 s; partials s.s, r-hat.s
template <typename T, int NRHS>
__global__ __launch_bounds__(kKB) void k_s(int64_t n, int64_t np, const T *__restrict__ dinv,
                                           const T *__restrict__ r, const T *__restrict__ rh, const T *__restrict__ v,
                                           T *__restrict__ s, T *__restrict__ sh, double *__restrict__ part,
                                           KState *__restrict__ st, int nblk, int phase)
{
    KState st0[NRHS];
    load_states<NRHS>(st, st0);
    double ld[NRHS][kPartPer];
    {
        const double *ps[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) ps[k] = partial(part, P_RV, k);
        load_partials_n<NRHS>(ps, nblk, ld);
    }
    // the first row's operands, requested after the partials: the wait for the
    // partials leaves them in flight through the reduction
    const int64_t i0 = (int64_t)logical_block() * kKB + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kKB;
    T d0 = (T)0, r0[NRHS], v0[NRHS], rh0[NRHS];
    if (i0 < n) {
        d0 = dinv[i0];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            r0[k] = r[k * np + i0];
            v0[k] = v[k * np + i0];
            rh0[k] = rh[k * np + i0];
        }
    }
    double rvs[NRHS];
    reduce_partials_n<NRHS>(ld, rvs);
    if (all_done<NRHS>(st0, phase)) return;
    bool act[NRHS];
    double alpha[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        const KState stk = st0[k];
        act[k] = !finished_before(stk, phase);
        const double rv = rvs[k];
        alpha[k] = (rv != 0.0) ? stk.rho / rv : 0.0;
        if (act[k] && blockIdx.x == 0 && threadIdx.x == 0) {
            st[k].alpha = alpha[k];
            st[k].restart = 0;
            st[k].refresh = 0;
            if (rv == 0.0) {
                st[k].done_at = phase;
                st[k].status = RBFFD_E_BREAKDOWN;
            }
        }
        if (rv == 0.0) act[k] = false;
    }
    double acc[2 * NRHS];
#pragma unroll
    for (int k = 0; k < 2 * NRHS; ++k) acc[k] = 0.0;
    for (int64_t i = i0; i < n; i += stride) {
        const bool first = i == i0;
        const T di = first ? d0 : dinv[i];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            if (!act[k]) continue;
            const T ri = first ? r0[k] : r[k * np + i];
            const T vi = first ? v0[k] : v[k * np + i];
            const T rhi = first ? rh0[k] : rh[k * np + i];
            const T si = (T)((double)ri - alpha[k] * (double)vi);
            s[k * np + i] = si;
            sh[k * np + i] = di * si;
            acc[2 * k] += (double)si * (double)si;
            acc[2 * k + 1] += (double)rhi * (double)si;
        }
    }
    double *ps[2 * NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        ps[2 * k] = partial(part, P_SS, k);
        ps[2 * k + 1] = partial(part, P_RS, k);
    }
    write_partials<2 * NRHS>(acc, ps);
}

// KT: if ||s|| is small, x += alpha p-hat and stop; else t = A s-hat and
// partials t.s, t.t, r-hat.t
template <typename T, typename TM, int NRHS, int U, bool NT>
__global__ __launch_bounds__(kKB) void k_t(int64_t n, int64_t np, int q, ColIdx col, const TM *__restrict__ val,
                                           T *__restrict__ x, int64_t xs, const T *__restrict__ ph,
                                           const T *__restrict__ s, const T *__restrict__ sh,
                                           const T *__restrict__ rh, T *__restrict__ t, double *__restrict__ part,
                                           KState *__restrict__ st, int nblk, double tol2, int phase)
{
    KState st0[NRHS];
    load_states<NRHS>(st, st0);
    double ss[NRHS];
    {
        const double *ps[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) ps[k] = partial(part, P_SS, k);
        sum_partials_n<NRHS>(ps, nblk, ss);
    }
    if (all_done<NRHS>(st0, phase)) return;
    bool act[NRHS], half[NRHS], sp[NRHS];
    double alpha[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        const KState stk = st0[k];
        act[k] = !finished_before(stk, phase);
        alpha[k] = stk.alpha;
        half[k] = act[k] && ss[k] <= tol2 * stk.bb;
        sp[k] = act[k] && !half[k];
        if (half[k] && blockIdx.x == 0 && threadIdx.x == 0) {
            st[k].done_at = phase;
            st[k].status = RBFFD_OK;
            st[k].iters = stk.iters + 1;
        }
    }
    double acc[3 * NRHS];
#pragma unroll
    for (int k = 0; k < 3 * NRHS; ++k) acc[k] = 0.0;
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
#pragma unroll
        for (int k = 0; k < NRHS; ++k)
            if (half[k]) x[k * xs + i] = (T)((double)x[k * xs + i] + alpha[k] * (double)ph[k * np + i]);
        double at[NRHS];
        row_dot<TM, T, NRHS, U, NT>(i, q, col, val, sh, np, sp, at);
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            if (!sp[k]) continue;
            const T ti = (T)at[k];
            t[k * np + i] = ti;
            acc[3 * k] += (double)ti * (double)s[k * np + i];
            acc[3 * k + 1] += (double)ti * (double)ti;
            acc[3 * k + 2] += (double)rh[k * np + i] * (double)ti;
        }
    }
    double *ps[3 * NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        ps[3 * k] = partial(part, P_TS, k);
        ps[3 * k + 1] = partial(part, P_TT, k);
        ps[3 * k + 2] = partial(part, P_RT, k);
    }
    write_partials<3 * NRHS>(acc, ps);
}

// KX: omega = t.s / t.t; x += alpha p-hat + omega s-hat; r = s - omega t;
// rho' = r-hat.s - omega r-hat.t; restart (r-hat = r) when rho' has vanished
// relative to r.r (both by linearity from the dots of s and t); p-hat = D^-1 r + beta (p-hat - omega D^-1 v); partial r.r.
// s-hat is formed again from s and D^-1, as KS formed it (the same rounded
// product), which saves reading it back.
template <typename T, int NRHS>
__global__ __launch_bounds__(kKB) void k_x(int64_t n, int64_t np, const T *__restrict__ dinv, T *__restrict__ x,
                                           int64_t xs, T *__restrict__ ph, const T *__restrict__ s,
                                           const T *__restrict__ t,
                                           const T *__restrict__ v, T *__restrict__ r, T *__restrict__ rh,
                                           double *__restrict__ part, KState *__restrict__ st, int nblk, int phase)
{
    KState st0[NRHS];
    load_states<NRHS>(st, st0);
    double ld[5 * NRHS][kPartPer];
    {
        const double *ps[5 * NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            ps[5 * k] = partial(part, P_TS, k);
            ps[5 * k + 1] = partial(part, P_TT, k);
            ps[5 * k + 2] = partial(part, P_RS, k);
            ps[5 * k + 3] = partial(part, P_RT, k);
            ps[5 * k + 4] = partial(part, P_SS, k);
        }
        load_partials_n<5 * NRHS>(ps, nblk, ld);
    }
    // the first row's operands, requested after the partials (as in k_s)
    const int64_t i0 = (int64_t)logical_block() * kKB + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * kKB;
    T d0 = (T)0, x0[NRHS], ph0[NRHS], s0[NRHS], t0[NRHS], v0[NRHS];
    if (i0 < n) {
        d0 = dinv[i0];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            x0[k] = x[k * xs + i0];
            ph0[k] = ph[k * np + i0];
            s0[k] = s[k * np + i0];
            t0[k] = t[k * np + i0];
            v0[k] = v[k * np + i0];
        }
    }
    double sums[5 * NRHS];
    reduce_partials_n<5 * NRHS>(ld, sums);
    if (all_done<NRHS>(st0, phase)) return;
    bool act[NRHS], restart[NRHS];
    double alpha[NRHS], omega[NRHS], beta[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        const KState stk = st0[k];
        act[k] = !finished_before(stk, phase);
        alpha[k] = stk.alpha;
        const double ts = sums[5 * k], tt = sums[5 * k + 1], rs = sums[5 * k + 2], rt = sums[5 * k + 3];
        const double ssk = sums[5 * k + 4];
        omega[k] = (tt > 0.0) ? ts / tt : 0.0;
        const double rho1 = rs - omega[k] * rt;
        // ||r||^2 of the new residual r = s - omega t, by linearity
        const double rrk = fmax(ssk - 2.0 * omega[k] * ts + omega[k] * omega[k] * tt, 0.0);
        restart[k] = fabs(rho1) < 1e-300 || fabs(rho1) < 1e-30 * rrk;
        beta[k] = (restart[k] || omega[k] == 0.0) ? 0.0 : (rho1 / stk.rho) * (alpha[k] / omega[k]);
        if (act[k] && blockIdx.x == 0 && threadIdx.x == 0) {
            st[k].omega = omega[k];
            st[k].iters = stk.iters + 1;
            st[k].rho_next = rho1;
            st[k].restart = restart[k];
            if (omega[k] == 0.0) {
                st[k].done_at = phase;
                st[k].status = RBFFD_E_BREAKDOWN;
            }
        }
    }
    double srr[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) srr[k] = 0.0;
    for (int64_t i = i0; i < n; i += stride) {
        const bool first = i == i0;
        const T di = first ? d0 : dinv[i];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            if (!act[k]) continue;
            const T phi = first ? ph0[k] : ph[k * np + i];
            const T si = first ? s0[k] : s[k * np + i];
            const T xi = first ? x0[k] : x[k * xs + i];
            const T ti = first ? t0[k] : t[k * np + i];
            const T shi = di * si;
            x[k * xs + i] = (T)((double)xi + alpha[k] * (double)phi + omega[k] * (double)shi);
            const T ri = (T)((double)si - omega[k] * (double)ti);
            r[k * np + i] = ri;
            if (restart[k]) rh[k * np + i] = ri;
            const T pn = (beta[k] == 0.0) ? (T)(di * ri)
                                          : (T)(di * ri + beta[k] * ((double)phi - omega[k] * (double)(di * (first ? v0[k] : v[k * np + i]))));
            ph[k * np + i] = pn;
            srr[k] += (double)ri * (double)ri;
        }
    }
    double *ps[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) ps[k] = partial(part, P_RR, k);
    write_partials<NRHS>(srr, ps);
}

// The instantiation of KV and KT for a stencil width (row unroll depth) and a
// matrix size (non-temporal matrix loads).
template <typename T, typename TM, int NRHS>
inline auto kv_for(int q, bool nt)
{
    if (row_unroll3(q)) return nt ? k_v<T, TM, NRHS, 3, true> : k_v<T, TM, NRHS, 3, false>;
    return nt ? k_v<T, TM, NRHS, 4, true> : k_v<T, TM, NRHS, 4, false>;
}

template <typename T, typename TM, int NRHS>
inline auto kt_for(int q, bool nt)
{
    if (row_unroll3(q)) return nt ? k_t<T, TM, NRHS, 3, true> : k_t<T, TM, NRHS, 3, false>;
    return nt ? k_t<T, TM, NRHS, 4, true> : k_t<T, TM, NRHS, 4, false>;
}

// ||b - A x||^2 and ||b||^2 per right-hand side (FP64), partials then one block
__global__ __launch_bounds__(kBlock) void k_resid(int64_t n, int q, int nrhs, ColIdx col,
                                                  const double *__restrict__ val, const double *__restrict__ b,
                                                  int64_t bs, const double *__restrict__ x, int64_t xs,
                                                  double *__restrict__ part)
{
    __shared__ double lds[kBlock / 64];
    for (int k = 0; k < nrhs; ++k) {
        double srr = 0.0, sbb = 0.0;
        const bool act[1] = {true};
        for (int64_t i = (int64_t)logical_block() * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
            double ax[1];
            row_dot<double, double, 1>(i, q, col, val, x + k * xs, 0, act, ax);
            const double ri = b[k * bs + i] - ax[0];
            srr += ri * ri;
            sbb += b[k * bs + i] * b[k * bs + i];
        }
        const double a = block_sum(srr, lds), c = block_sum(sbb, lds);
        if (threadIdx.x == 0) {
            part[(2 * k) * kMaxBlocks + blockIdx.x] = a;
            part[(2 * k + 1) * kMaxBlocks + blockIdx.x] = c;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_resid_final(const double *__restrict__ part, int np, int nrhs,
                                                        double *__restrict__ out)
{
    __shared__ double lds[kBlock / 64];
    for (int k = 0; k < nrhs; ++k) {
        const double a = sum_partials(part + (2 * k) * kMaxBlocks, np, lds);
        const double c = sum_partials(part + (2 * k + 1) * kMaxBlocks, np, lds);
        if (threadIdx.x == 0) out[k] = (c > 0.0) ? sqrt(a / c) : sqrt(a);
    }
}

// Reliable update of the mixed-precision solve, part 1: x (FP64) += d (FP32
// correction accumulated since the last update), d = 0.
template <typename T>
__global__ void k_refine_add(int64_t n, int nrhs, double *__restrict__ x, int64_t xs, T *__restrict__ d, int64_t np)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < nrhs; ++k) {
        x[k * xs + i] += (double)d[k * np + i];
        d[k * np + i] = (T)0;
    }
}

// Part 2: the true residual r = b - A x in FP64 replaces the FP32 recursive
// residual; partials r-hat.r and r.r for the FP32 iteration, and ||r||^2,
// ||b||^2 of the FP64 residual for the host. With init set, r-hat = r,
// p-hat = D^-1 r and the ||b||^2 partials of the iteration are written as well.
template <typename T, int NRHS>
__global__ __launch_bounds__(kKB) void k_rel_resid(int64_t n, int64_t np, int q, ColIdx col,
                                                   const double *__restrict__ val, const double *__restrict__ b,
                                                   int64_t bs, const double *__restrict__ x, int64_t xs,
                                                   const T *__restrict__ dinv, T *__restrict__ r, T *__restrict__ rh,
                                                   T *__restrict__ ph, int init, double *__restrict__ part,
                                                   double *__restrict__ tpart)
{
    __shared__ double lds[kKB / 64];
    double rhr[NRHS], rr[NRHS], tr[NRHS], bb[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) rhr[k] = rr[k] = tr[k] = bb[k] = 0.0;
    bool act[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) act[k] = true;
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kKB) {
        double ax[NRHS];
        row_dot<double, double, NRHS>(i, q, col, val, x, xs, act, ax);
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            const double bi = b[k * bs + i];
            const double ri = bi - ax[k];
            const T rf = (T)ri;
            r[k * np + i] = rf;
            T hf;
            if (init) {
                rh[k * np + i] = rf;
                ph[k * np + i] = dinv[i] * rf;
                hf = rf;
            } else {
                hf = rh[k * np + i];
            }
            rhr[k] += (double)hf * (double)rf;
            rr[k] += (double)rf * (double)rf;
            tr[k] += ri * ri;
            bb[k] += bi * bi;
        }
    }
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        const double a1 = kblock_sum(rhr[k], lds);
        const double a2 = kblock_sum(rr[k], lds);
        const double a3 = kblock_sum(tr[k], lds);
        const double a4 = kblock_sum(bb[k], lds);
        if (threadIdx.x == 0) {
            partial(part, P_RHR, k)[blockIdx.x] = a1;
            partial(part, P_RR, k)[blockIdx.x] = a2;
            if (init) partial(part, P_BB, k)[blockIdx.x] = a4;
            tpart[(2 * k) * kMaxBlocks + blockIdx.x] = a3;
            tpart[(2 * k + 1) * kMaxBlocks + blockIdx.x] = a4;
        }
    }
}

// r-hat = r and p-hat = D^-1 r for the right-hand sides in mask (a solve that
// continues after its recursion had stopped)
template <typename T>
__global__ void k_dir_reset(int64_t n, int64_t np, int nrhs, unsigned mask, const T *__restrict__ dinv,
                            const T *__restrict__ r, T *__restrict__ rh, T *__restrict__ ph)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < nrhs; ++k) {
        if (!((mask >> k) & 1u)) continue;
        const T ri = r[k * np + i];
        rh[k * np + i] = ri;
        ph[k * np + i] = dinv[i] * ri;
    }
}

// Zeroes the solver state records (a kernel rather than a memset, so that the
// solve also runs inside a captured graph).
// After each chunk of iterations every finished solve's stamp becomes 1, below
// the phase numbers (2, 3, ...) that a chunk's launches carry. Every chunk of
// one length then launches the same kernels with the same arguments, so it can
// be captured once as a HIP graph and replayed.
__global__ void k_stamp_done(KState *__restrict__ st, int nrhs)
{
    const int k = threadIdx.x;
    if (k < nrhs && st[k].done_at != 0) st[k].done_at = 1;
}

__global__ void k_clear_states(KState *__restrict__ st)
{
    if (threadIdx.x < kMaxRhs) st[threadIdx.x] = KState{};
}

template <typename T>
__global__ void k_zero(T *__restrict__ y, int64_t m)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) y[i] = (T)0;
}

inline int grid_blocks(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b >= 64) b = (b + 7) / 8 * 8;   // multiple of 8 for the XCD-aware mapping
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (int)std::max<int64_t>(1, b);
}

inline int krylov_blocks(int64_t n)
{
    int64_t b = (n + kKB - 1) / kKB;
    if (b >= 64) b = (b + 7) / 8 * 8;   // multiple of 8 for the XCD-aware mapping
    if (b > kKMaxBlocks) b = kKMaxBlocks;
    return (int)std::max<int64_t>(1, b);
}

template <typename T>
int get_work(rbffd_ctx *ctx, int64_t npad, int nrhs, Work *w)
{
    const size_t vec = sizeof(T) * npad * nrhs;
    char *base = nullptr;
    RB_CHECK(workspace(ctx, sizeof(T) == 4 ? WS_KRYLOV32 : WS_KRYLOV, 7 * vec, (void **)&base));
    w->r = base;
    w->rh = base + vec;
    w->ph = base + 2 * vec;
    w->v = base + 3 * vec;
    w->s = base + 4 * vec;
    w->sh = base + 5 * vec;
    w->t = base + 6 * vec;
    RB_CHECK(workspace(ctx, sizeof(T) == 4 ? WS_PARTIAL32 : WS_PARTIAL,
                       sizeof(double) * P_COUNT * kMaxRhs * kMaxBlocks + sizeof(KState) * kMaxRhs, (void **)&w->part));
    w->st = (KState *)(w->part + P_COUNT * kMaxRhs * kMaxBlocks);
    return RBFFD_OK;
}

// ---- one-workgroup BiCGSTAB: the whole solve of a small system in one kernel --
// The four-kernel iteration has a latency floor of about 22 us however small
// the system. Here one workgroup runs the entire solve instead: the same
// iteration as KV, KS, KT, KX (same dot products, convergence tests, restart
// rule and breakdown handling), with block barriers in place of kernel
// boundaries and block-wide sums in a fixed order in place of partials. Thread
// t owns rows t, t + BS, ... in every row loop, so row-local updates need no
// barrier; the SpMVs gather neighbour entries and follow a barrier. It is a
// path the autotuner (or the caller) may pick per system size; on MI355X one
// CU streams about two matrix entries per cycle, which keeps it behind the
// four-kernel iteration at every size measured (26 vs 22 us per iteration at
// 1,760 rows).
struct WGSys {
    int64_t n, np, xs;      // rows, vector stride, stride of x between right-hand sides
    int q, max_iter;
    double tol2;
    ColIdx col;
    const double *val, *dinv, *b;   // b: [nrhs][n]
    double *x;
    double *r, *rh, *ph, *v, *s, *sh, *t;   // [nrhs][np] each
    KState *st;             // out: iters, status, done_at (1 = finished)
};

// Wave sum through DPP: butterflies within rows of 16 lanes, then the row
// broadcasts, leaving the total in lane 63 (a fixed order of additions).
template <int CTRL, int ROWS>
__device__ inline double dpp_add(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return v + __hiloint2double(hi, lo);
}

__device__ inline double wave_sum_dpp63(double v)
{
    v = dpp_add<0xB1, 0xF>(v);    // quad_perm [1, 0, 3, 2]
    v = dpp_add<0x4E, 0xF>(v);    // quad_perm [2, 3, 0, 1]
    v = dpp_add<0x141, 0xF>(v);   // row_half_mirror
    v = dpp_add<0x140, 0xF>(v);   // row_mirror
    v = dpp_add<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
    return v;                     // lane 63: the wave's sum
}

template <int NV, int BS>
__device__ inline void wg_sum(double (&v)[NV], double (*red)[BS / 64])
{
#pragma unroll
    for (int m = 0; m < NV; ++m) v[m] = wave_sum_dpp63(v[m]);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 63)
#pragma unroll
        for (int m = 0; m < NV; ++m) red[m][w] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < BS / 64; ++j) t += red[m][j];
        v[m] = t;
    }
    __syncthreads();   // red is reused by the next sum
}

template <int NRHS, int BS, int U>
__device__ inline void wg_solve(const WGSys &S, double (*red)[BS / 64])
{
    const int tid = threadIdx.x;
    const int64_t n = S.n, np = S.np;
    double rr[NRHS], bb[NRHS], rho[NRHS];
    bool act[NRHS];
    int iters[NRHS], status[NRHS];
    bool all[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) all[k] = true;
    {
        double acc[2 * NRHS];
#pragma unroll
        for (int k = 0; k < 2 * NRHS; ++k) acc[k] = 0.0;
        for (int64_t i = tid; i < n; i += BS) {
            double ax[NRHS];
            row_dot<double, double, NRHS, U>(i, S.q, S.col, S.val, S.x, S.xs, all, ax);
            const double di = S.dinv[i];
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                const double bi = S.b[k * n + i];
                const double ri = bi - ax[k];
                S.r[k * np + i] = ri;
                S.rh[k * np + i] = ri;
                S.ph[k * np + i] = di * ri;
                acc[2 * k] += ri * ri;
                acc[2 * k + 1] += bi * bi;
            }
        }
        wg_sum<2 * NRHS, BS>(acc, red);
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            rr[k] = acc[2 * k];
            bb[k] = acc[2 * k + 1];
        }
    }
    bool zero[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        iters[k] = 0;
        status[k] = RBFFD_OK;
        rho[k] = rr[k];
        zero[k] = bb[k] == 0.0;
        act[k] = !zero[k] && !(rr[k] <= S.tol2 * bb[k]);
    }
    for (int64_t i = tid; i < n; i += BS)
#pragma unroll
        for (int k = 0; k < NRHS; ++k)
            if (zero[k]) S.x[k * S.xs + i] = 0.0;
    for (int it = 0; it < S.max_iter; ++it) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < NRHS; ++k) any = any || act[k];
        if (!any) break;
        __syncthreads();   // p-hat of every row is written
        // v = A p-hat, r-hat.v
        double rv[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) rv[k] = 0.0;
        for (int64_t i = tid; i < n; i += BS) {
            double av[NRHS];
            row_dot<double, double, NRHS, U>(i, S.q, S.col, S.val, S.ph, np, act, av);
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                if (!act[k]) continue;
                S.v[k * np + i] = av[k];
                rv[k] += S.rh[k * np + i] * av[k];
            }
        }
        wg_sum<NRHS, BS>(rv, red);
        double alpha[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            alpha[k] = (rv[k] != 0.0) ? rho[k] / rv[k] : 0.0;
            if (act[k] && rv[k] == 0.0) {
                status[k] = RBFFD_E_BREAKDOWN;
                act[k] = false;
            }
        }
        // s = r - alpha v, s-hat = D^-1 s, s.s, r-hat.s
        double sacc[2 * NRHS];
#pragma unroll
        for (int k = 0; k < 2 * NRHS; ++k) sacc[k] = 0.0;
        for (int64_t i = tid; i < n; i += BS) {
            const double di = S.dinv[i];
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                if (!act[k]) continue;
                const double si = S.r[k * np + i] - alpha[k] * S.v[k * np + i];
                S.s[k * np + i] = si;
                S.sh[k * np + i] = di * si;
                sacc[2 * k] += si * si;
                sacc[2 * k + 1] += S.rh[k * np + i] * si;
            }
        }
        wg_sum<2 * NRHS, BS>(sacc, red);
        bool half[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            half[k] = act[k] && sacc[2 * k] <= S.tol2 * bb[k];
            if (half[k]) {
                iters[k] += 1;
                act[k] = false;
            }
        }
        for (int64_t i = tid; i < n; i += BS)
#pragma unroll
            for (int k = 0; k < NRHS; ++k)
                if (half[k]) S.x[k * S.xs + i] = S.x[k * S.xs + i] + alpha[k] * S.ph[k * np + i];
        __syncthreads();   // s-hat of every row is written
        // t = A s-hat, t.s, t.t, r-hat.t
        double tacc[3 * NRHS];
#pragma unroll
        for (int k = 0; k < 3 * NRHS; ++k) tacc[k] = 0.0;
        for (int64_t i = tid; i < n; i += BS) {
            double at[NRHS];
            row_dot<double, double, NRHS, U>(i, S.q, S.col, S.val, S.sh, np, act, at);
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                if (!act[k]) continue;
                S.t[k * np + i] = at[k];
                tacc[3 * k] += at[k] * S.s[k * np + i];
                tacc[3 * k + 1] += at[k] * at[k];
                tacc[3 * k + 2] += S.rh[k * np + i] * at[k];
            }
        }
        wg_sum<3 * NRHS, BS>(tacc, red);
        double omega[NRHS], beta[NRHS], rho1[NRHS];
        bool restart[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            const double ts = tacc[3 * k], tt = tacc[3 * k + 1], rt = tacc[3 * k + 2];
            const double ss = sacc[2 * k], rs = sacc[2 * k + 1];
            omega[k] = (tt > 0.0) ? ts / tt : 0.0;
            rho1[k] = rs - omega[k] * rt;
            const double rrk = fmax(ss - 2.0 * omega[k] * ts + omega[k] * omega[k] * tt, 0.0);
            restart[k] = fabs(rho1[k]) < 1e-300 || fabs(rho1[k]) < 1e-30 * rrk;
            beta[k] = (restart[k] || omega[k] == 0.0) ? 0.0 : (rho1[k] / rho[k]) * (alpha[k] / omega[k]);
        }
        // x += alpha p-hat + omega s-hat; r = s - omega t; next p-hat; r.r
        double racc[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) racc[k] = 0.0;
        for (int64_t i = tid; i < n; i += BS) {
            const double di = S.dinv[i];
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                if (!act[k]) continue;
                const double phi = S.ph[k * np + i], si = S.s[k * np + i];
                const double shi = S.sh[k * np + i];
                S.x[k * S.xs + i] = S.x[k * S.xs + i] + alpha[k] * phi + omega[k] * shi;
                const double ri = si - omega[k] * S.t[k * np + i];
                S.r[k * np + i] = ri;
                if (restart[k]) S.rh[k * np + i] = ri;
                S.ph[k * np + i] = (beta[k] == 0.0) ? di * ri
                                                    : di * ri + beta[k] * (phi - omega[k] * (di * S.v[k * np + i]));
                racc[k] += ri * ri;
            }
        }
        wg_sum<NRHS, BS>(racc, red);
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            if (!act[k]) continue;
            iters[k] += 1;
            rr[k] = racc[k];
            rho[k] = restart[k] ? rr[k] : rho1[k];
            if (omega[k] == 0.0) {
                status[k] = RBFFD_E_BREAKDOWN;
                act[k] = false;
            } else if (rr[k] <= S.tol2 * bb[k]) {
                act[k] = false;
            }
        }
    }
    if (tid == 0)
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            S.st[k].iters = iters[k];
            S.st[k].status = status[k];
            S.st[k].done_at = act[k] ? 0 : 1;
        }
}

template <int NRHS, int BS, int U>
__global__ __launch_bounds__(BS) void k_bicgstab_wg1(WGSys S)
{
    __shared__ double red[3 * NRHS][BS / 64];
    wg_solve<NRHS, BS, U>(S, red);
}

// Row-loop unroll of the one-workgroup solver: deep, so that one thread has
// many entries' loads in flight (one workgroup has few threads per row).
inline int wg_unroll(int q) { return (q % 10 == 0) ? 10 : (q % 6 == 0) ? 6 : 8; }

template <int NRHS>
int launch_wg1(const WGSys &S, int bs, hipStream_t s)
{
    const int u = wg_unroll(S.q);
#define RB_WG1(BS_)                                                                                   \
    if (bs == BS_) {                                                                                  \
        if (u == 10)                                                                                  \
            hipLaunchKernelGGL((k_bicgstab_wg1<NRHS, BS_, 10>), dim3(1), dim3(BS_), 0, s, S);         \
        else if (u == 6)                                                                              \
            hipLaunchKernelGGL((k_bicgstab_wg1<NRHS, BS_, 6>), dim3(1), dim3(BS_), 0, s, S);          \
        else                                                                                          \
            hipLaunchKernelGGL((k_bicgstab_wg1<NRHS, BS_, 8>), dim3(1), dim3(BS_), 0, s, S);          \
        RB_HIP(hipGetLastError());                                                                    \
        return RBFFD_OK;                                                                              \
    }
    RB_WG1(256)
    RB_WG1(512)
    RB_WG1(1024)
#undef RB_WG1
    return fail(RBFFD_E_ARG, "one-workgroup solver: block size must be 256, 512 or 1024");
}

// Path of a solve: 0 the multi-kernel iteration, else the one-workgroup
// solver's block size. Without a recorded choice the multi-kernel iteration
// runs: on MI355X one workgroup streams about two matrix entries per cycle,
// so even at 1,760 rows (26 us per iteration) it does not beat the four-kernel
// iteration's latency floor (22 us), and from 10k rows it is 8x slower or more.
int solver_choice(const rbffd_ctx *ctx, int64_t n, int q)
{
    auto it = ctx->solver_choice.find({n, q});
    return it != ctx->solver_choice.end() ? it->second : 0;
}

// the autotuner tries the one-workgroup solver up to this size
constexpr int64_t kWGTuneMaxRows = 65536;

// ---- HIP graphs of iteration chunks ------------------------------------------
// A chunk (its KV, KS, KT, KX launches, the closing convergence test and the
// stamp) is captured on the context's own stream the first time its exact
// launch sequence occurs, and replayed on the caller's stream after that. The
// key holds every kernel argument of the chunk, so a replay launches exactly
// what the direct path would: results are bitwise the same either way.
struct ChunkKey {
    const void *kv, *kt, *ks, *kx;
    const void *col, *cbase, *col16, *val, *dinv, *x;
    const void *r, *rh, *ph, *v, *s, *sh, *t, *part, *st;
    int64_t n, xs;
    int q, nblk, todo, nrhs;
    double tol2;
};

struct GraphCache {
    struct Entry {
        ChunkKey key;
        hipGraphExec_t exec;
        uint64_t used;
    };
    hipStream_t cs = nullptr;
    std::vector<Entry> e;
    uint64_t clock = 0;
};
constexpr size_t kMaxGraphs = 32;

template <typename F>
int chunk_graph(rbffd_ctx *ctx, const ChunkKey &key, F &&launch, hipGraphExec_t *out)
{
    GraphCache *gc = (GraphCache *)ctx->graphs;
    if (!gc) {
        gc = new GraphCache();
        ctx->graphs = gc;
    }
    for (auto &en : gc->e)
        if (std::memcmp(&en.key, &key, sizeof(ChunkKey)) == 0) {
            en.used = ++gc->clock;
            *out = en.exec;
            return RBFFD_OK;
        }
    if (!gc->cs) RB_HIP(hipStreamCreateWithFlags(&gc->cs, hipStreamNonBlocking));
    RB_HIP(hipStreamBeginCapture(gc->cs, hipStreamCaptureModeRelaxed));
    launch(gc->cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(gc->cs, &g);
    if (e != hipSuccess) return hip_fail(e, "capturing a BiCGSTAB chunk");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "instantiating a BiCGSTAB chunk graph");
    if (gc->e.size() >= kMaxGraphs) {
        size_t lru = 0;
        for (size_t i = 1; i < gc->e.size(); ++i)
            if (gc->e[i].used < gc->e[lru].used) lru = i;
        (void)hipGraphExecDestroy(gc->e[lru].exec);
        gc->e.erase(gc->e.begin() + lru);
    }
    gc->e.push_back({key, ex, ++gc->clock});
    *out = ex;
    return RBFFD_OK;
}

template <typename T, int NRHS>
int bicgstab_t(int64_t n, int q, ColIdx col, const T *val, const T *dinv, const T *b, int64_t bs, T *x, int64_t xs,
               double tol, int max_iter, KrylovResult *res, Work &w, KState *hst, hipStream_t s,
               rbffd_ctx *gctx = nullptr)
{
    const int64_t np = pad64(n);
    const int nblk = krylov_blocks(n);
    const dim3 g(nblk), bl(kKB);
    T *r = (T *)w.r, *rh = (T *)w.rh, *ph = (T *)w.ph, *v = (T *)w.v, *sv = (T *)w.s, *sh = (T *)w.sh, *t = (T *)w.t;
    const double tol2 = tol * tol;
    hipLaunchKernelGGL(k_clear_states, dim3(1), dim3(64), 0, s, w.st);
    hipLaunchKernelGGL((k_init<T, NRHS>), g, bl, 0, s, n, np, q, col, val, dinv, b, bs, x, xs, r, rh, ph, w.part);
    RB_HIP(hipGetLastError());
    const bool nt = matrix_nt(n, q, sizeof(T));
    const auto kv = kv_for<T, T, NRHS>(q, nt);
    const auto kt = kt_for<T, T, NRHS>(q, nt);
    const auto ks = k_s<T, NRHS>;
    const auto kx = k_x<T, NRHS>;
    // one chunk: todo iterations, the convergence test on the last residual (so
    // the host sees it now) and the stamp; phases 2, 3, ... within the chunk
    auto launch_chunk = [&](hipStream_t st_, int todo) {
        int phase = 1;
        for (int c = 0; c < todo; ++c) {
            hipLaunchKernelGGL(kv, g, bl, 0, st_, n, np, q, col, val, rh, ph, v, x, xs, w.part, w.st, nblk,
                               tol2, 0, ++phase);
            hipLaunchKernelGGL(ks, g, bl, 0, st_, n, np, dinv, r, rh, v, sv, sh, w.part, w.st, nblk, ++phase);
            hipLaunchKernelGGL(kt, g, bl, 0, st_, n, np, q, col, val, x, xs, ph, sv, sh, rh, t, w.part,
                               w.st, nblk, tol2, ++phase);
            hipLaunchKernelGGL(kx, g, bl, 0, st_, n, np, dinv, x, xs, ph, sv, t, v, r, rh, w.part, w.st,
                               nblk, ++phase);
        }
        hipLaunchKernelGGL(kv, g, bl, 0, st_, n, np, q, col, val, rh, ph, v, x, xs, w.part, w.st, nblk,
                           tol2, 1, ++phase);
        hipLaunchKernelGGL(k_stamp_done, dim3(1), dim3(64), 0, st_, w.st, NRHS);
    };
    int it = 0, chunk = 4;
    bool finished = false;
    while (!finished) {
        const int todo = std::max(std::min(chunk, max_iter - it), 0);
        if (gctx && gctx->use_graphs) {
            ChunkKey key;
            std::memset(&key, 0, sizeof(key));
            key.kv = (const void *)kv;
            key.kt = (const void *)kt;
            key.ks = (const void *)ks;
            key.kx = (const void *)kx;
            key.col = col.col;
            key.cbase = col.cbase;
            key.col16 = col.col16;
            key.val = val;
            key.dinv = dinv;
            key.x = x;
            key.r = r;
            key.rh = rh;
            key.ph = ph;
            key.v = v;
            key.s = sv;
            key.sh = sh;
            key.t = t;
            key.part = w.part;
            key.st = w.st;
            key.n = n;
            key.xs = xs;
            key.q = q;
            key.nblk = nblk;
            key.todo = todo;
            key.nrhs = NRHS;
            key.tol2 = tol2;
            hipGraphExec_t ge = nullptr;
            if (chunk_graph(gctx, key, [&](hipStream_t cs) { launch_chunk(cs, todo); }, &ge) == RBFFD_OK) {
                RB_HIP(hipGraphLaunch(ge, s));
            } else {
                // a capture that fails (another thread synchronised the whole
                // device meanwhile, for instance) launched nothing: this chunk
                // and the context's later solves launch kernel by kernel
                (void)hipGetLastError();
                gctx->use_graphs = false;
                launch_chunk(s, todo);
            }
        } else {
            launch_chunk(s, todo);
        }
        it += todo;
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(hst, w.st, sizeof(KState) * kMaxRhs, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        bool done = true;
        for (int k = 0; k < NRHS; ++k) done = done && hst[k].done_at != 0;
        finished = done || it >= max_iter;
        chunk = std::min(chunk * 2, 32);
    }
    for (int k = 0; k < NRHS; ++k) {
        res->iters[k] = hst[k].iters;
        res->status[k] = hst[k].done_at ? hst[k].status : RBFFD_E_NOCONV;
    }
    return RBFFD_OK;
}

// ---- BiCGSTAB with the block-Jacobi preconditioner (FP64, one right-hand side)
// The preconditioner blocks are the 64-row slices, and a slice is one
// wavefront, so z = M^-1 y is a wave-local 64x64 matrix-vector product: lane l
// holds y_l, and z_l = sum_j Minv[l][j] y_j with y_j broadcast across the wave.
// The row loops therefore run over whole slices (up to npad) so that every
// lane takes part in the broadcasts; loads and stores stay within n.
__device__ inline double bj_apply(const BlockInv &bi, int64_t slice, double y, int lane)
{
    const __half *__restrict__ blk = bi.val + slice * 4096;
    double z = 0.0;
#pragma unroll 8
    for (int j = 0; j < 64; ++j) z = fma((double)__half2float(blk[j * 64 + lane]), __shfl(y, j, 64), z);
    return z * (double)bi.scale[slice];
}

// r = b - A x, r-hat = r, p = r, p-hat = M^-1 r; partials r.r and b.b
__global__ __launch_bounds__(kKB) void kbj_init(int64_t n, int64_t np, int q, ColIdx col, const double *__restrict__ val,
                                                BlockInv binv, const double *__restrict__ b,
                                                const double *__restrict__ x, double *__restrict__ r,
                                                double *__restrict__ rh, double *__restrict__ p,
                                                double *__restrict__ ph, double *__restrict__ part)
{
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    const bool act[1] = {true};
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < np; i += (int64_t)gridDim.x * kKB) {
        double ri = 0.0;
        if (i < n) {
            double ax[1];
            row_dot<double, double, 1>(i, q, col, val, x, 0, act, ax);
            const double bi = b[i];
            ri = bi - ax[0];
            r[i] = ri;
            rh[i] = ri;
            p[i] = ri;
            acc[0] += ri * ri;
            acc[1] += bi * bi;
        }
        const double z = bj_apply(binv, i >> 6, ri, lane);
        if (i < n) ph[i] = z;
    }
    double *ps[2] = {partial(part, P_RR, 0), partial(part, P_BB, 0)};
    write_partials<2>(acc, ps);
}

// KS: alpha = rho / r-hat.v; s = r - alpha v; s-hat = M^-1 s; partials s.s, r-hat.s
template <typename T>
__global__ __launch_bounds__(kKB) void kbj_s(int64_t n, int64_t np, BlockInv binv,
                                             const T *__restrict__ r, const T *__restrict__ rh,
                                             const T *__restrict__ v, T *__restrict__ s,
                                             T *__restrict__ sh, double *__restrict__ part, KState *__restrict__ st,
                                             int nblk, int phase)
{
    KState st0[1];
    load_states<1>(st, st0);
    double rv;
    {
        const double *ps[1] = {partial(part, P_RV, 0)};
        sum_partials_n<1>(ps, nblk, &rv);
    }
    if (all_done<1>(st0, phase)) return;
    const KState stk = st0[0];
    const double alpha = (rv != 0.0) ? stk.rho / rv : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[0].alpha = alpha;
        st[0].restart = 0;
        st[0].refresh = 0;
        if (rv == 0.0) {
            st[0].done_at = phase;
            st[0].status = RBFFD_E_BREAKDOWN;
        }
    }
    if (rv == 0.0) return;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < np; i += (int64_t)gridDim.x * kKB) {
        double si = 0.0;
        if (i < n) {
            const T sv = (T)((double)r[i] - alpha * (double)v[i]);
            s[i] = sv;
            si = (double)sv;
            acc[0] += si * si;
            acc[1] += (double)rh[i] * si;
        }
        const double z = bj_apply(binv, i >> 6, si, lane);
        if (i < n) sh[i] = (T)z;
    }
    double *ps[2] = {partial(part, P_SS, 0), partial(part, P_RS, 0)};
    write_partials<2>(acc, ps);
}

// KX: omega; x += alpha p-hat + omega s-hat; r = s - omega t; p = r + beta (p -
// omega v); p-hat = M^-1 p; partial r.r (restart and beta as in k_x)
template <typename T>
__global__ __launch_bounds__(kKB) void kbj_x(int64_t n, int64_t np, BlockInv binv,
                                             T *__restrict__ x, T *__restrict__ p, T *__restrict__ ph,
                                             const T *__restrict__ s, const T *__restrict__ sh,
                                             const T *__restrict__ t, const T *__restrict__ v,
                                             T *__restrict__ r, T *__restrict__ rh,
                                             double *__restrict__ part, KState *__restrict__ st, int nblk, int phase)
{
    KState st0[1];
    load_states<1>(st, st0);
    double sums[5];
    {
        const double *ps[5] = {partial(part, P_TS, 0), partial(part, P_TT, 0), partial(part, P_RS, 0),
                               partial(part, P_RT, 0), partial(part, P_SS, 0)};
        sum_partials_n<5>(ps, nblk, sums);
    }
    if (all_done<1>(st0, phase)) return;
    const KState stk = st0[0];
    const double ts = sums[0], tt = sums[1], rs = sums[2], rt = sums[3], ssk = sums[4];
    const double omega = (tt > 0.0) ? ts / tt : 0.0;
    const double rho1 = rs - omega * rt;
    const double rrk = fmax(ssk - 2.0 * omega * ts + omega * omega * tt, 0.0);   // ||s - omega t||^2
    const bool restart = fabs(rho1) < 1e-300 || fabs(rho1) < 1e-30 * rrk;
    const double beta = (restart || omega == 0.0) ? 0.0 : (rho1 / stk.rho) * (stk.alpha / omega);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[0].omega = omega;
        st[0].iters = stk.iters + 1;
        st[0].rho_next = rho1;
        st[0].restart = restart;
        if (omega == 0.0) {
            st[0].done_at = phase;
            st[0].status = RBFFD_E_BREAKDOWN;
        }
    }
    const int lane = threadIdx.x & 63;
    double srr = 0.0;
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < np; i += (int64_t)gridDim.x * kKB) {
        double pn = 0.0;
        if (i < n) {
            x[i] = (T)((double)x[i] + (stk.alpha * (double)ph[i] + omega * (double)sh[i]));
            const T rt = (T)((double)s[i] - omega * (double)t[i]);
            const double ri = (double)rt;
            r[i] = rt;
            if (restart) rh[i] = rt;
            const T pt = (beta == 0.0) ? rt : (T)(ri + beta * ((double)p[i] - omega * (double)v[i]));
            p[i] = pt;
            pn = (double)pt;
            srr += ri * ri;
        }
        const double z = bj_apply(binv, i >> 6, pn, lane);
        if (i < n) ph[i] = (T)z;
    }
    double *ps[1] = {partial(part, P_RR, 0)};
    write_partials<1>(&srr, ps);
}

// Reliable update with the block preconditioner (one right-hand side): the
// FP64 residual r = b - A x replaces the recursive one; partials r-hat.r and
// r.r for the iteration and ||r||^2, ||b||^2 for the host. With init set,
// r-hat = p = r, p-hat = M^-1 r and the ||b||^2 partials are written as well.
template <typename T>
__global__ __launch_bounds__(kKB) void kbj_rel_resid(int64_t n, int64_t np, int q, ColIdx col,
                                                     const double *__restrict__ val, BlockInv binv,
                                                     const double *__restrict__ b, const double *__restrict__ x,
                                                     T *__restrict__ r, T *__restrict__ rh, T *__restrict__ p,
                                                     T *__restrict__ ph, int init, double *__restrict__ part,
                                                     double *__restrict__ tpart)
{
    __shared__ double lds[kKB / 64];
    const int lane = threadIdx.x & 63;
    double rhr = 0.0, rr = 0.0, tr = 0.0, bb = 0.0;
    const bool act[1] = {true};
    for (int64_t i = (int64_t)logical_block() * kKB + threadIdx.x; i < np; i += (int64_t)gridDim.x * kKB) {
        double rf = 0.0;
        if (i < n) {
            double ax[1];
            row_dot<double, double, 1>(i, q, col, val, x, n, act, ax);
            const double bi = b[i];
            const double ri = bi - ax[0];
            const T rt = (T)ri;
            rf = (double)rt;
            r[i] = rt;
            double hf = rf;
            if (init) {
                rh[i] = rt;
                p[i] = rt;
            } else {
                hf = (double)rh[i];
            }
            rhr += hf * rf;
            rr += rf * rf;
            tr += ri * ri;
            bb += bi * bi;
        }
        if (init) {
            const double z = bj_apply(binv, i >> 6, rf, lane);
            if (i < n) ph[i] = (T)z;
        }
    }
    const double a1 = kblock_sum(rhr, lds);
    const double a2 = kblock_sum(rr, lds);
    const double a3 = kblock_sum(tr, lds);
    const double a4 = kblock_sum(bb, lds);
    if (threadIdx.x == 0) {
        partial(part, P_RHR, 0)[blockIdx.x] = a1;
        partial(part, P_RR, 0)[blockIdx.x] = a2;
        if (init) partial(part, P_BB, 0)[blockIdx.x] = a4;
        tpart[blockIdx.x] = a3;
        tpart[kMaxBlocks + blockIdx.x] = a4;
    }
}

// r-hat = p = r, p-hat = M^-1 r (a solve that continues after its recursion
// had stopped); one thread per row, whole slices per wavefront
template <typename T>
__global__ void kbj_dir_reset(int64_t n, int64_t np, BlockInv binv, const T *__restrict__ r,
                              T *__restrict__ rh, T *__restrict__ p, T *__restrict__ ph)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= np) return;   // np is a multiple of 64 and blockDim.x of 64: whole wavefronts leave
    double ri = 0.0;
    if (i < n) {
        const T rt = r[i];
        rh[i] = rt;
        p[i] = rt;
        ri = (double)rt;
    }
    const double z = bj_apply(binv, i >> 6, ri, threadIdx.x & 63);
    if (i < n) ph[i] = (T)z;
}

// ---- batched BiCGSTAB (FP64, one right-hand side per system) ---------------
// System j owns blocks [boff, boff + nblk); block b belongs to system bmap[b].
// Partials live at part[kind * pstride + b], so every system reduces over its
// own blocks in block order. A system with block inverses (binv) is
// preconditioned by them and keeps its unpreconditioned direction in p; its
// row loops run over whole 64-row slices (a block's first row and its stride
// are multiples of 64, so each wavefront holds one slice).
struct BSys {
    int64_t n, np;
    int q, boff, nblk, pad;
    double tol2;
    ColIdx col;
    const double *val, *dinv, *b;
    const float *val32;   // FP32 matrix for the Krylov SpMVs, or nullptr (FP64)
    BlockInv binv;        // block-Jacobi inverses (binv.val nullptr: Jacobi)
    double *x;
    double *r, *rh, *ph, *v, *s, *sh, *t, *p;
};
constexpr int kBatchVecs = 8;   // work vectors per system: r r-hat p-hat v s s-hat t p

__device__ inline const double *bpart(const double *part, int kind, int pstride, int boff)
{
    return part + (int64_t)kind * pstride + boff;
}

__global__ __launch_bounds__(kKB) void kb_init(const BSys *__restrict__ sys, const int *__restrict__ bmap,
                                               double *__restrict__ part, int pstride, const KState *__restrict__ st)
{
    const int j = bmap[blockIdx.x];
    const BSys S = sys[j];
    if (!st[j].fresh) return;
    const int lb = blockIdx.x - S.boff;
    const bool bj = S.binv.val != nullptr;
    const int64_t lim = bj ? S.np : S.n;
    const int lane = threadIdx.x & 63;
    double rr = 0.0, bb = 0.0;
    const bool act[1] = {true};
    for (int64_t i = (int64_t)lb * kKB + threadIdx.x; i < lim; i += (int64_t)S.nblk * kKB) {
        double ri = 0.0;
        if (i < S.n) {
            double ax[1];
            row_dot<double, double, 1>(i, S.q, S.col, S.val, S.x, 0, act, ax);
            const double bi = S.b[i];
            ri = bi - ax[0];
            S.r[i] = ri;
            S.rh[i] = ri;
            if (bj)
                S.p[i] = ri;
            else
                S.ph[i] = S.dinv[i] * ri;
            rr += ri * ri;
            bb += bi * bi;
        }
        if (bj) {
            const double z = bj_apply(S.binv, i >> 6, ri, lane);
            if (i < S.n) S.ph[i] = z;
        }
    }
    const double acc[2] = {rr, bb};
    double *ps[2] = {part + (int64_t)P_RR * pstride, part + (int64_t)P_BB * pstride};
    write_partials<2>(acc, ps);
}

__global__ __launch_bounds__(kKB) void kb_v(const BSys *__restrict__ sys, const int *__restrict__ bmap,
                                            double *__restrict__ part, int pstride, KState *__restrict__ st,
                                            int check_only, int phase)
{
    const int j = bmap[blockIdx.x];
    const BSys S = sys[j];
    double sums[2];
    {
        const double *ps[2] = {bpart(part, P_RR, pstride, S.boff), bpart(part, P_BB, pstride, S.boff)};
        sum_partials_n<2>(ps, S.nblk, sums);
    }
    const KState k0 = st[j];
    if (finished_before(k0, phase)) return;
    // ||b||^2 is taken from the partials of KB_INIT once, then from the state;
    // after a change of block ranges ||r||^2 also comes from the state
    const double rr = k0.moved ? k0.rr : sums[0];
    const double bb = (k0.iters == 0 && !k0.moved) ? sums[1] : k0.bb;
    const bool zero = bb == 0.0;
    const bool conv = !zero && rr <= S.tol2 * bb;
    const bool lead = blockIdx.x == S.boff && threadIdx.x == 0;
    if (lead) {
        st[j].rr = rr;
        st[j].bb = bb;
        st[j].rho = (k0.iters == 0 || k0.restart) ? rr : k0.rho_next;
        if (zero || conv) {
            st[j].done_at = phase;
            st[j].status = RBFFD_OK;
        }
    }
    if (conv || (check_only && !zero)) return;
    const int lb = blockIdx.x - S.boff;
    double srv = 0.0;
    const bool act[1] = {!zero};
    for (int64_t i = (int64_t)lb * kKB + threadIdx.x; i < S.n; i += (int64_t)S.nblk * kKB) {
        if (zero) {
            S.x[i] = 0.0;
            continue;
        }
        double av[1];
        if (S.val32)
            row_dot<float, double, 1>(i, S.q, S.col, S.val32, S.ph, 0, act, av);
        else
            row_dot<double, double, 1>(i, S.q, S.col, S.val, S.ph, 0, act, av);
        S.v[i] = av[0];
        srv += S.rh[i] * av[0];
    }
    double *ps[1] = {part + (int64_t)P_RV * pstride};
    write_partials<1>(&srv, ps);
}

__global__ __launch_bounds__(kKB) void kb_s(const BSys *__restrict__ sys, const int *__restrict__ bmap,
                                            double *__restrict__ part, int pstride, KState *__restrict__ st, int phase)
{
    const int j = bmap[blockIdx.x];
    const BSys S = sys[j];
    const KState k0 = st[j];   // loaded early: overlaps the partial loads
    double rv;
    {
        const double *ps[1] = {bpart(part, P_RV, pstride, S.boff)};
        sum_partials_n<1>(ps, S.nblk, &rv);
    }
    if (finished_before(k0, phase)) return;
    const double alpha = (rv != 0.0) ? k0.rho / rv : 0.0;
    if (blockIdx.x == S.boff && threadIdx.x == 0) {
        st[j].alpha = alpha;
        st[j].restart = 0;
        st[j].fresh = 0;
        st[j].moved = 0;
        if (rv == 0.0) {
            st[j].done_at = phase;
            st[j].status = RBFFD_E_BREAKDOWN;
        }
    }
    if (rv == 0.0) return;
    const int lb = blockIdx.x - S.boff;
    const bool bj = S.binv.val != nullptr;
    const int64_t lim = bj ? S.np : S.n;
    const int lane = threadIdx.x & 63;
    double acc[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)lb * kKB + threadIdx.x; i < lim; i += (int64_t)S.nblk * kKB) {
        double si = 0.0;
        if (i < S.n) {
            si = S.r[i] - alpha * S.v[i];
            S.s[i] = si;
            if (!bj) S.sh[i] = S.dinv[i] * si;
            acc[0] += si * si;
            acc[1] += S.rh[i] * si;
        }
        if (bj) {
            const double z = bj_apply(S.binv, i >> 6, si, lane);
            if (i < S.n) S.sh[i] = z;
        }
    }
    double *ps[2] = {part + (int64_t)P_SS * pstride, part + (int64_t)P_RS * pstride};
    write_partials<2>(acc, ps);
}

__global__ __launch_bounds__(kKB) void kb_t(const BSys *__restrict__ sys, const int *__restrict__ bmap,
                                            double *__restrict__ part, int pstride, KState *__restrict__ st, int phase)
{
    const int j = bmap[blockIdx.x];
    const BSys S = sys[j];
    const KState k0 = st[j];   // loaded early: overlaps the partial loads
    double ss;
    {
        const double *ps[1] = {bpart(part, P_SS, pstride, S.boff)};
        sum_partials_n<1>(ps, S.nblk, &ss);
    }
    if (finished_before(k0, phase)) return;
    const bool half = ss <= S.tol2 * k0.bb;
    if (half && blockIdx.x == S.boff && threadIdx.x == 0) {
        st[j].done_at = phase;
        st[j].status = RBFFD_OK;
        st[j].iters = k0.iters + 1;
    }
    const int lb = blockIdx.x - S.boff;
    double acc[3] = {0.0, 0.0, 0.0};
    const bool act[1] = {true};
    for (int64_t i = (int64_t)lb * kKB + threadIdx.x; i < S.n; i += (int64_t)S.nblk * kKB) {
        if (half) {
            S.x[i] += k0.alpha * S.ph[i];
            continue;
        }
        double at[1];
        if (S.val32)
            row_dot<float, double, 1>(i, S.q, S.col, S.val32, S.sh, 0, act, at);
        else
            row_dot<double, double, 1>(i, S.q, S.col, S.val, S.sh, 0, act, at);
        S.t[i] = at[0];
        acc[0] += at[0] * S.s[i];
        acc[1] += at[0] * at[0];
        acc[2] += S.rh[i] * at[0];
    }
    if (half) return;
    double *ps[3] = {part + (int64_t)P_TS * pstride, part + (int64_t)P_TT * pstride, part + (int64_t)P_RT * pstride};
    write_partials<3>(acc, ps);
}

__global__ __launch_bounds__(kKB) void kb_x(const BSys *__restrict__ sys, const int *__restrict__ bmap,
                                            double *__restrict__ part, int pstride, KState *__restrict__ st, int phase)
{
    const int j = bmap[blockIdx.x];
    const BSys S = sys[j];
    const KState k0 = st[j];   // loaded early: overlaps the partial loads
    double sums[5];
    {
        const double *ps[5] = {bpart(part, P_TS, pstride, S.boff), bpart(part, P_TT, pstride, S.boff),
                               bpart(part, P_RS, pstride, S.boff), bpart(part, P_RT, pstride, S.boff),
                               bpart(part, P_SS, pstride, S.boff)};
        sum_partials_n<5>(ps, S.nblk, sums);
    }
    if (finished_before(k0, phase)) return;
    const double ts = sums[0], tt = sums[1], rs = sums[2], rt = sums[3], ssk = sums[4];
    const double omega = (tt > 0.0) ? ts / tt : 0.0;
    const double rho1 = rs - omega * rt;
    const double rrk = fmax(ssk - 2.0 * omega * ts + omega * omega * tt, 0.0);   // ||s - omega t||^2
    const bool restart = fabs(rho1) < 1e-300 || fabs(rho1) < 1e-30 * rrk;
    const double beta = (restart || omega == 0.0) ? 0.0 : (rho1 / k0.rho) * (k0.alpha / omega);
    if (blockIdx.x == S.boff && threadIdx.x == 0) {
        st[j].omega = omega;
        st[j].iters = k0.iters + 1;
        st[j].rho_next = rho1;
        st[j].restart = restart;
        if (omega == 0.0) {
            st[j].done_at = phase;
            st[j].status = RBFFD_E_BREAKDOWN;
        }
    }
    const int lb = blockIdx.x - S.boff;
    double srr = 0.0;
    if (S.binv.val == nullptr) {
        for (int64_t i = (int64_t)lb * kKB + threadIdx.x; i < S.n; i += (int64_t)S.nblk * kKB) {
            const double di = S.dinv[i];
            const double phi = S.ph[i];
            S.x[i] += k0.alpha * phi + omega * S.sh[i];
            const double ri = S.s[i] - omega * S.t[i];
            S.r[i] = ri;
            if (restart) S.rh[i] = ri;
            S.ph[i] = (beta == 0.0) ? di * ri : di * ri + beta * (phi - omega * (di * S.v[i]));
            srr += ri * ri;
        }
    } else {
        // p = r + beta (p - omega v), p-hat = M^-1 p over whole slices
        const int lane = threadIdx.x & 63;
        for (int64_t i = (int64_t)lb * kKB + threadIdx.x; i < S.np; i += (int64_t)S.nblk * kKB) {
            double pn = 0.0;
            if (i < S.n) {
                S.x[i] += k0.alpha * S.ph[i] + omega * S.sh[i];
                const double ri = S.s[i] - omega * S.t[i];
                S.r[i] = ri;
                if (restart) S.rh[i] = ri;
                pn = (beta == 0.0) ? ri : ri + beta * (S.p[i] - omega * S.v[i]);
                S.p[i] = pn;
                srr += ri * ri;
            }
            const double z = bj_apply(S.binv, i >> 6, pn, lane);
            if (i < S.n) S.ph[i] = z;
        }
    }
    double *ps[1] = {part + (int64_t)P_RR * pstride};
    write_partials<1>(&srr, ps);
}

// true residual ||b - A x|| / ||b|| per system (||b - A x|| when b = 0)
__global__ __launch_bounds__(kKB) void kb_resid(const BSys *__restrict__ sys, const int *__restrict__ bmap,
                                                double *__restrict__ part, int pstride)
{
    const int j = bmap[blockIdx.x];
    const BSys S = sys[j];
    const int lb = blockIdx.x - S.boff;
    double acc[2] = {0.0, 0.0};
    const bool act[1] = {true};
    for (int64_t i = (int64_t)lb * kKB + threadIdx.x; i < S.n; i += (int64_t)S.nblk * kKB) {
        double ax[1];
        row_dot<double, double, 1>(i, S.q, S.col, S.val, S.x, 0, act, ax);
        const double ri = S.b[i] - ax[0];
        acc[0] += ri * ri;
        acc[1] += S.b[i] * S.b[i];
    }
    double *ps[2] = {part + (int64_t)P_TS * pstride, part + (int64_t)P_TT * pstride};
    write_partials<2>(acc, ps);
}

__global__ __launch_bounds__(kKB) void kb_resid_final(const BSys *__restrict__ sys, const double *__restrict__ part,
                                                      int pstride, double *__restrict__ out)
{
    const BSys S = sys[blockIdx.x];
    double sums[2];
    const double *ps[2] = {bpart(part, P_TS, pstride, S.boff), bpart(part, P_TT, pstride, S.boff)};
    sum_partials_n<2>(ps, S.nblk, sums);
    if (threadIdx.x == 0) out[blockIdx.x] = (sums[1] > 0.0) ? sqrt(sums[0] / sums[1]) : sqrt(sums[0]);
}

}  // namespace

int spmv(int64_t n, int q, ColIdx col, const double *val, const double *x, double *y, hipStream_t s)
{
    const int64_t nb = (n + kBlock - 1) / kBlock;
    const bool nt = matrix_nt(n, q, sizeof(double));
    const auto kern = row_unroll3(q) ? (nt ? spmv_kernel<double, 3, true> : spmv_kernel<double, 3, false>)
                                     : (nt ? spmv_kernel<double, 4, true> : spmv_kernel<double, 4, false>);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kBlock), 0, s, n, q, col, val, x, y);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

// One solve (nrhs right-hand sides) by the one-workgroup solver with bs
// threads, in the vectors and state records of w; hst receives the records.
static int wg_solve_one(int64_t n, int q, ColIdx col, const double *val, const double *dinv, int nrhs,
                        const double *b, double *x, double tol, int max_iter, Work &w, KState *hst, int bs,
                        KrylovResult *res, hipStream_t s)
{
    WGSys S;
    std::memset(&S, 0, sizeof(S));
    S.n = n;
    S.np = pad64(n);
    S.xs = n;
    S.q = q;
    S.max_iter = std::max(max_iter, 0);
    S.tol2 = tol * tol;
    S.col = col;
    S.val = val;
    S.dinv = dinv;
    S.b = b;
    S.x = x;
    S.r = (double *)w.r;
    S.rh = (double *)w.rh;
    S.ph = (double *)w.ph;
    S.v = (double *)w.v;
    S.s = (double *)w.s;
    S.sh = (double *)w.sh;
    S.t = (double *)w.t;
    S.st = w.st;
    switch (nrhs) {
    case 1: RB_CHECK(launch_wg1<1>(S, bs, s)); break;
    case 2: RB_CHECK(launch_wg1<2>(S, bs, s)); break;
    case 3: RB_CHECK(launch_wg1<3>(S, bs, s)); break;
    default: return fail(RBFFD_E_ARG, "nrhs must be 1..3");
    }
    RB_HIP(hipMemcpyAsync(hst, w.st, sizeof(KState) * nrhs, hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nrhs; ++k) {
        res->iters[k] = hst[k].iters;
        res->status[k] = hst[k].done_at ? hst[k].status : RBFFD_E_NOCONV;
    }
    return RBFFD_OK;
}

static int bicgstab_once(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val,
                         const double *dinv, int nrhs, const double *b, double *x, double tol, int max_iter,
                         KrylovResult *res, hipStream_t s)
{
    Work w;
    RB_CHECK(get_work<double>(ctx, pad64(n), nrhs, &w));
    KState *hst = nullptr;
    RB_CHECK(host_scratch(ctx, kHostKrylov, sizeof(KState) * kMaxRhs, (void **)&hst));
    const int bs = solver_choice(ctx, n, q);
    if (bs > 0) return wg_solve_one(n, q, col, val, dinv, nrhs, b, x, tol, max_iter, w, hst, bs, res, s);
    switch (nrhs) {
    case 1: return bicgstab_t<double, 1>(n, q, col, val, dinv, b, n, x, n, tol, max_iter, res, w, hst, s, ctx);
    case 2: return bicgstab_t<double, 2>(n, q, col, val, dinv, b, n, x, n, tol, max_iter, res, w, hst, s, ctx);
    case 3: return bicgstab_t<double, 3>(n, q, col, val, dinv, b, n, x, n, tol, max_iter, res, w, hst, s, ctx);
    default: return fail(RBFFD_E_ARG, "nrhs must be 1..3");
    }
}

static int bicgstab_block_once(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, BlockInv binv,
                               const double *b, double *x, double tol, int max_iter, KrylovResult *res,
                               hipStream_t s)
{
    Work w;
    RB_CHECK(get_work<double>(ctx, pad64(n), 1, &w));
    double *pv = nullptr;   // unpreconditioned search direction
    RB_CHECK(workspace(ctx, WS_MISC, sizeof(double) * pad64(n), (void **)&pv));
    const int64_t np = pad64(n);
    const int nblk = krylov_blocks(n);
    const dim3 g(nblk), bl(kKB);
    double *r = (double *)w.r, *rh = (double *)w.rh, *ph = (double *)w.ph, *v = (double *)w.v, *sv = (double *)w.s,
           *sh = (double *)w.sh, *t = (double *)w.t;
    const double tol2 = tol * tol;
    hipLaunchKernelGGL(k_clear_states, dim3(1), dim3(64), 0, s, w.st);
    hipLaunchKernelGGL(kbj_init, g, bl, 0, s, n, np, q, col, val, binv, b, x, r, rh, pv, ph, w.part);
    RB_HIP(hipGetLastError());
    KState *hst = nullptr;
    RB_CHECK(host_scratch(ctx, kHostKrylov, sizeof(KState) * kMaxRhs, (void **)&hst));
    const bool nt = matrix_nt(n, q, sizeof(double));
    const auto kv = kv_for<double, double, 1>(q, nt);
    const auto kt = kt_for<double, double, 1>(q, nt);
    int it = 0, chunk = 4, phase = 0;
    bool finished = false;
    while (!finished) {
        const int todo = std::min(chunk, max_iter - it);
        for (int c = 0; c < todo; ++c) {
            hipLaunchKernelGGL(kv, g, bl, 0, s, n, np, q, col, val, rh, ph, v, x, n, w.part,
                               w.st, nblk, tol2, 0, ++phase);
            hipLaunchKernelGGL(kbj_s<double>, g, bl, 0, s, n, np, binv, r, rh, v, sv, sh, w.part, w.st, nblk, ++phase);
            hipLaunchKernelGGL(kt, g, bl, 0, s, n, np, q, col, val, x, n, ph, sv, sh, rh, t,
                               w.part, w.st, nblk, tol2, ++phase);
            hipLaunchKernelGGL(kbj_x<double>, g, bl, 0, s, n, np, binv, x, pv, ph, sv, sh, t, v, r, rh, w.part, w.st,
                               nblk, ++phase);
        }
        it += std::max(todo, 0);
        hipLaunchKernelGGL(kv, g, bl, 0, s, n, np, q, col, val, rh, ph, v, x, n, w.part, w.st,
                           nblk, tol2, 1, ++phase);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(hst, w.st, sizeof(KState) * kMaxRhs, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        finished = hst[0].done_at != 0 || it >= max_iter;
        chunk = std::min(chunk * 2, 32);
    }
    res->iters[0] = hst[0].iters;
    res->status[0] = hst[0].done_at ? hst[0].status : RBFFD_E_NOCONV;
    return RBFFD_OK;
}

int bicgstab_block(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, BlockInv binv,
                   const double *b, double *x, double tol, int max_iter, KrylovResult *res, hipStream_t s)
{
    KrylovResult acc;
    for (int attempt = 0; attempt < 3; ++attempt) {
        const int left = max_iter - acc.iters[0];
        KrylovResult r1;
        RB_CHECK(bicgstab_block_once(ctx, n, q, col, val, binv, b, x, tol, std::max(left, 0), &r1, s));
        acc.iters[0] += r1.iters[0];
        acc.status[0] = r1.status[0];
        double rr[kMaxRhs];
        RB_CHECK(residual_norms(ctx, n, q, col, val, 1, b, x, rr, s));
        acc.relres[0] = rr[0];
        if (r1.status[0] != RBFFD_OK || left <= 0 || rr[0] <= 10.0 * tol) break;
    }
    // the recursion converged but the true residual still misses 10 tol after
    // the restarts: not converged, as in the batched and served solves
    if (acc.status[0] == RBFFD_OK && !(acc.relres[0] <= 10.0 * tol)) acc.status[0] = RBFFD_E_NOCONV;
    *res = acc;
    return RBFFD_OK;
}

// BiCGSTAB with up to two restarts from the true residual: when the recursive
// residual has met tol but ||b - A x|| exceeds 10 tol ||b||, iterate again from x.
int bicgstab(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, const double *dinv, int nrhs,
             const double *b, double *x, double tol, int max_iter, KrylovResult *res, hipStream_t s)
{
    KrylovResult acc;
    for (int attempt = 0; attempt < 3; ++attempt) {
        int left = max_iter;
        for (int k = 0; k < nrhs; ++k) left = std::min(left, max_iter - acc.iters[k]);
        KrylovResult r1;
        RB_CHECK(bicgstab_once(ctx, n, q, col, val, dinv, nrhs, b, x, tol, std::max(left, 0), &r1, s));
        bool ok = true;
        for (int k = 0; k < nrhs; ++k) {
            acc.iters[k] += r1.iters[k];
            acc.status[k] = r1.status[k];
            ok = ok && r1.status[k] == RBFFD_OK;
        }
        double rr[kMaxRhs];
        RB_CHECK(residual_norms(ctx, n, q, col, val, nrhs, b, x, rr, s));
        bool good = true;
        for (int k = 0; k < nrhs; ++k) {
            acc.relres[k] = rr[k];
            good = good && rr[k] <= 10.0 * tol;
        }
        if (!ok || left <= 0 || good) break;
    }
    for (int k = 0; k < nrhs; ++k)
        if (acc.status[k] == RBFFD_OK && !(acc.relres[k] <= 10.0 * tol)) acc.status[k] = RBFFD_E_NOCONV;
    *res = acc;
    return RBFFD_OK;
}

// Mixed precision: BiCGSTAB with FP32 matrix values (and in one mode FP32
// vectors; rows and dots accumulated in FP64) inside FP64 iterative
// refinement: whenever the recursive residual has fallen by the inner factor
// since the last refinement (or the recursion reports convergence), the
// correction is added to the FP64 iterate, the FP64 residual b - A x replaces
// the recursive one, and BiCGSTAB restarts from it (r-hat = r, fresh
// directions). Inner factors: 0.1 with FP32 vectors, 0.01 with FP64 vectors
// (a CPU emulation on the pressure-correction matrices of 17k and 66k-point
// Taylor-Green clouds: continuing in the same Krylov space instead took 1.35x
// the FP64 iterations with FP64 vectors and diverged with FP32 vectors).
// The solve stops when the FP64 residual meets tol. If a refinement finds a
// non-finite or growing FP64 residual, or FP32 BiCGSTAB breaks down, the best
// iterate is restored and the solve finishes in FP64. With block inverses
// (binv, one right-hand side) the iteration is right-preconditioned by them
// instead of the diagonal, and keeps its unpreconditioned direction p.
template <typename T>
constexpr double inner_factor()
{
    return sizeof(T) == sizeof(float) ? 0.1 : 0.01;
}
constexpr int kStallIters = 1000;   // forced update; less than 2x progress since the last one = stall

template <typename T, int NRHS>
static int bicgstab_reliable(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val,
                             const float *val32, const T *dinv, const double *dinv64, BlockInv binv,
                             const double *b, double *x, double tol, int max_iter, KrylovResult *res,
                             int *refinements, hipStream_t s)
{
    if (binv.val && NRHS != 1) return fail(RBFFD_E_ARG, "the block preconditioner takes one right-hand side");
    const int64_t np = pad64(n);
    Work w;
    RB_CHECK(get_work<T>(ctx, np, NRHS, &w));
    char *scr = nullptr;
    const size_t tbytes = sizeof(double) * (2 * kMaxRhs * kMaxBlocks + kMaxRhs);
    const size_t xbytes = sizeof(double) * n * NRHS;
    const size_t dbytes = sizeof(T) * np * NRHS;
    RB_CHECK(workspace(ctx, WS_REFINE, tbytes + xbytes + dbytes + (binv.val ? dbytes : 0), (void **)&scr));
    double *tpart = (double *)scr;
    double *rout = tpart + 2 * kMaxRhs * kMaxBlocks;
    double *xgood = (double *)(scr + tbytes);       // iterate with the lowest FP64 residual so far
    T *d = (T *)(scr + tbytes + xbytes);            // correction accumulated since the last update
    T *pv = binv.val ? (T *)(scr + tbytes + xbytes + dbytes) : nullptr;   // unpreconditioned direction
    double *rr = nullptr;
    RB_CHECK(host_scratch(ctx, kHostRefine, sizeof(double) * kMaxRhs, (void **)&rr));
    KState *hst = nullptr;
    RB_CHECK(host_scratch(ctx, kHostKrylov, sizeof(KState) * kMaxRhs, (void **)&hst));

    const int nblk = krylov_blocks(n);
    const dim3 g(nblk), bl(kKB);
    const unsigned gb = (unsigned)((n + kBlock - 1) / kBlock);
    T *r = (T *)w.r, *rh = (T *)w.rh, *ph = (T *)w.ph, *v = (T *)w.v, *sv = (T *)w.s, *sh = (T *)w.sh, *t = (T *)w.t;
    const double tol2 = tol * tol;

    // true residual of x: replaces r (and r-hat when init), norms to the host
    auto true_residual = [&](int init) -> int {
        if (binv.val)
            hipLaunchKernelGGL(kbj_rel_resid<T>, g, bl, 0, s, n, np, q, col, val, binv, b, x, r, rh, pv, ph, init,
                               w.part, tpart);
        else
            hipLaunchKernelGGL((k_rel_resid<T, NRHS>), g, bl, 0, s, n, np, q, col, val, b, n, x, n, dinv, r, rh, ph,
                               init, w.part, tpart);
        hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(kBlock), 0, s, tpart, nblk, NRHS, rout);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(rr, rout, sizeof(double) * NRHS, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        return RBFFD_OK;
    };

    hipLaunchKernelGGL(k_clear_states, dim3(1), dim3(64), 0, s, w.st);
    hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((np * NRHS + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d,
                       np * NRHS);
    RB_CHECK(true_residual(1));
    double best[NRHS], rmax[NRHS];
    bool conv = true;
    for (int k = 0; k < NRHS; ++k) {
        best[k] = rmax[k] = rr[k];
        conv = conv && rr[k] <= tol;
    }
    RB_HIP(hipMemcpyAsync(xgood, x, xbytes, hipMemcpyDeviceToDevice, s));
    double prev[NRHS];
    for (int k = 0; k < NRHS; ++k) prev[k] = rr[k];
    const bool nt = matrix_nt(n, q, sizeof(float));
    const auto kv = kv_for<T, float, NRHS>(q, nt);
    const auto kt = kt_for<T, float, NRHS>(q, nt);
    int it = 0, chunk = 4, phase = 0, nref = 0, last_update = 0;
    bool fallback = false;
    while (!conv && it < max_iter) {
        const int todo = std::min(chunk, max_iter - it);
        for (int c = 0; c < todo; ++c) {
            hipLaunchKernelGGL(kv, g, bl, 0, s, n, np, q, col, val32, rh, ph, v, d, np, w.part,
                               w.st, nblk, tol2, 0, ++phase);
            if (binv.val)
                hipLaunchKernelGGL(kbj_s<T>, g, bl, 0, s, n, np, binv, r, rh, v, sv, sh, w.part, w.st, nblk, ++phase);
            else
                hipLaunchKernelGGL((k_s<T, NRHS>), g, bl, 0, s, n, np, dinv, r, rh, v, sv, sh, w.part, w.st, nblk,
                                   ++phase);
            hipLaunchKernelGGL(kt, g, bl, 0, s, n, np, q, col, val32, d, np, ph, sv, sh, rh, t,
                               w.part, w.st, nblk, tol2, ++phase);
            if (binv.val)
                hipLaunchKernelGGL(kbj_x<T>, g, bl, 0, s, n, np, binv, d, pv, ph, sv, sh, t, v, r, rh, w.part, w.st,
                                   nblk, ++phase);
            else
                hipLaunchKernelGGL((k_x<T, NRHS>), g, bl, 0, s, n, np, dinv, d, np, ph, sv, t, v, r, rh, w.part,
                                   w.st, nblk, ++phase);
        }
        it += todo;
        hipLaunchKernelGGL(kv, g, bl, 0, s, n, np, q, col, val32, rh, ph, v, d, np, w.part, w.st,
                           nblk, tol2, 1, ++phase);
        chunk = std::min(chunk * 2, 32);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(hst, w.st, sizeof(KState) * kMaxRhs, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        bool update = it >= max_iter || it - last_update >= kStallIters, broke = false;
        for (int k = 0; k < NRHS; ++k) {
            if (hst[k].done_at != 0) {
                update = true;
                // b == 0 (x = 0) and breakdowns are left to the FP64 solver
                broke = broke || hst[k].status != RBFFD_OK || hst[k].bb == 0.0;
            } else if (hst[k].bb > 0.0 &&
                       hst[k].rr <= inner_factor<T>() * inner_factor<T>() * rmax[k] * rmax[k] * hst[k].bb) {
                update = true;
            }
        }
        if (!update) continue;
        // FP64 refinement
        hipLaunchKernelGGL(k_refine_add<T>, dim3(gb), dim3(kBlock), 0, s, n, NRHS, x, n, d, np);
        RB_CHECK(true_residual(0));
        ++nref;
        bool finite = true, worse = false, stalled = false;
        conv = true;
        for (int k = 0; k < NRHS; ++k) {
            finite = finite && std::isfinite(rr[k]);
            worse = worse || rr[k] > 2.0 * best[k];
            conv = conv && rr[k] <= tol;
            stalled = stalled || (rr[k] > tol && rr[k] > 0.5 * prev[k]);
            prev[k] = rr[k];
        }
        last_update = it;
        if (!finite || worse || broke || (stalled && !conv)) {
            fallback = true;
            break;
        }
        bool improved = true;
        for (int k = 0; k < NRHS; ++k) improved = improved && rr[k] <= best[k];
        if (improved) {
            RB_HIP(hipMemcpyAsync(xgood, x, xbytes, hipMemcpyDeviceToDevice, s));
            for (int k = 0; k < NRHS; ++k) best[k] = rr[k];
        }
        if (conv) break;
        // restart from the replaced residual (r-hat = r, fresh directions) every
        // right-hand side that has not met tol
        unsigned mask = 0;
        for (int k = 0; k < NRHS; ++k) {
            rmax[k] = rr[k];
            if (rr[k] > tol) {
                hst[k].done_at = 0;
                hst[k].restart = 1;
                hst[k].refresh = 0;
                mask |= 1u << k;
            } else {
                hst[k].refresh = 1;
            }
        }
        if (mask && binv.val)
            hipLaunchKernelGGL(kbj_dir_reset<T>, dim3((unsigned)((np + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n,
                               np, binv, r, rh, pv, ph);
        else if (mask)
            hipLaunchKernelGGL(k_dir_reset<T>, dim3(gb), dim3(kBlock), 0, s, n, np, NRHS, mask, dinv, r, rh, ph);
        RB_HIP(hipMemcpyAsync(w.st, hst, sizeof(KState) * kMaxRhs, hipMemcpyHostToDevice, s));
    }
    int total_it[kMaxRhs] = {0, 0, 0};
    for (int k = 0; k < NRHS; ++k) total_it[k] = (it > 0) ? hst[k].iters : 0;
    if (fallback) {
        RB_HIP(hipMemcpyAsync(x, xgood, xbytes, hipMemcpyDeviceToDevice, s));
        for (int k = 0; k < NRHS; ++k) rr[k] = best[k];
    }
    if (fallback && it < max_iter) {
        const int left = max_iter - it;
        KrylovResult fr;
        if (binv.val)
            RB_CHECK(bicgstab_block(ctx, n, q, col, val, binv, b, x, tol, left, &fr, s));
        else
            RB_CHECK(bicgstab(ctx, n, q, col, val, dinv64, NRHS, b, x, tol, left, &fr, s));
        conv = true;
        for (int k = 0; k < NRHS; ++k) {
            total_it[k] += fr.iters[k];
            rr[k] = fr.relres[k];
            conv = conv && fr.status[k] == RBFFD_OK;
        }
        ++nref;
    }
    for (int k = 0; k < NRHS; ++k) {
        res->iters[k] = total_it[k];
        res->status[k] = (rr[k] <= tol || (fallback && conv)) ? RBFFD_OK : RBFFD_E_NOCONV;
        res->relres[k] = rr[k];
    }
    res->fp64_fallback = fallback;
    if (refinements) *refinements = nref;
    return RBFFD_OK;
}

int bicgstab_mixed(rbffd_ctx *ctx, int precision, int64_t n, int q, ColIdx col, const double *val,
                   const float *val32, const float *dinv32, const double *dinv64, BlockInv binv, int nrhs,
                   const double *b, double *x, double tol, int max_iter, KrylovResult *res, int *refinements,
                   hipStream_t s)
{
    if (nrhs < 1 || nrhs > kMaxRhs) return fail(RBFFD_E_ARG, "nrhs must be 1..3");
    if (binv.val && nrhs != 1) return fail(RBFFD_E_ARG, "the block preconditioner takes one right-hand side");
    if (precision == RBFFD_FP32_IR) {
        // FP32 vectors and Jacobi diagonal, FP32 matrix
        switch (nrhs) {
        case 1: return bicgstab_reliable<float, 1>(ctx, n, q, col, val, val32, dinv32, dinv64, binv, b, x, tol,
                                                   max_iter, res, refinements, s);
        case 2: return bicgstab_reliable<float, 2>(ctx, n, q, col, val, val32, dinv32, dinv64, binv, b, x, tol,
                                                   max_iter, res, refinements, s);
        default: return bicgstab_reliable<float, 3>(ctx, n, q, col, val, val32, dinv32, dinv64, binv, b, x, tol,
                                                    max_iter, res, refinements, s);
        }
    }
    if (precision == RBFFD_FP32_MATRIX) {
        // FP64 vectors and Jacobi diagonal, FP32 matrix
        switch (nrhs) {
        case 1: return bicgstab_reliable<double, 1>(ctx, n, q, col, val, val32, dinv64, dinv64, binv, b, x, tol,
                                                    max_iter, res, refinements, s);
        case 2: return bicgstab_reliable<double, 2>(ctx, n, q, col, val, val32, dinv64, dinv64, binv, b, x, tol,
                                                    max_iter, res, refinements, s);
        default: return bicgstab_reliable<double, 3>(ctx, n, q, col, val, val32, dinv64, dinv64, binv, b, x, tol,
                                                     max_iter, res, refinements, s);
        }
    }
    return fail(RBFFD_E_ARG, "unknown mixed precision mode");
}

// ||b - A x|| / ||b|| per right-hand side. dev: device [2 kMaxRhs kMaxBlocks +
// kMaxRhs] doubles; hout: host [kMaxRhs] doubles the result is copied through.
static int residual_norms_in(int64_t n, int q, ColIdx col, const double *val, int nrhs, const double *b,
                             const double *x, double *dev, double *hout, double *relres_out, hipStream_t s)
{
    const int nblk = grid_blocks(n);
    double *out = dev + 2 * kMaxRhs * kMaxBlocks;
    hipLaunchKernelGGL(k_resid, dim3(nblk), dim3(kBlock), 0, s, n, q, nrhs, col, val, b, n, x, n, dev);
    hipLaunchKernelGGL(k_resid_final, dim3(1), dim3(kBlock), 0, s, dev, nblk, nrhs, out);
    RB_HIP(hipGetLastError());
    RB_HIP(hipMemcpyAsync(hout, out, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < nrhs; ++k) relres_out[k] = hout[k];
    return RBFFD_OK;
}

int residual_norms(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, int nrhs,
                   const double *b, const double *x, double *relres_out, hipStream_t s)
{
    double *dev = nullptr;
    RB_CHECK(workspace(ctx, WS_RESID, sizeof(double) * (2 * kMaxRhs * kMaxBlocks + kMaxRhs), (void **)&dev));
    double *hout = nullptr;
    RB_CHECK(host_scratch(ctx, kHostMisc, sizeof(double) * kMaxRhs, (void **)&hout));
    return residual_norms_in(n, q, col, val, nrhs, b, x, dev, hout, relres_out, s);
}


int bicgstab_batched(rbffd_ctx *ctx, int count, const BatchSystem *sys, double tol, int max_iter, int *iters,
                     int *status, double *relres, hipStream_t s)
{
    if (count < 1) return fail(RBFFD_E_ARG, "batch is empty");
    // block ranges: the same for a system alone or in any batch
    std::vector<int> boff(count), nblk(count);
    int64_t total = 0, vec = 0;
    for (int j = 0; j < count; ++j) {
        int64_t b = (sys[j].n + kKB - 1) / kKB;
        if (b > kKMaxBlocks) b = kKMaxBlocks;
        nblk[j] = (int)std::max<int64_t>(1, b);
        boff[j] = (int)total;
        total += nblk[j];
        vec += pad64(sys[j].n);
    }
    if (total > (int64_t)INT32_MAX / P_COUNT) return fail(RBFFD_E_ARG, "batch too large");
    const int pstride = (int)total;
    // device: descriptors | block map | states | partials | 7 vectors per system
    const size_t dsz = sizeof(BSys) * count, msz = sizeof(int) * total, ssz = sizeof(KState) * count;
    const size_t psz = sizeof(double) * P_COUNT * total, vsz = sizeof(double) * kBatchVecs * vec;
    const size_t o1 = (dsz + 255) / 256 * 256, o2 = o1 + (msz + 255) / 256 * 256, o3 = o2 + (ssz + 255) / 256 * 256,
                 o4 = o3 + (psz + 255) / 256 * 256, dtot = o4 + vsz + (size_t)count * sizeof(double) + 256;
    char *dev = nullptr;
    RB_CHECK(workspace(ctx, WS_BATCH, dtot, (void **)&dev));
    BSys *dsys = (BSys *)dev;
    int *dmap = (int *)(dev + o1);
    KState *dst = (KState *)(dev + o2);
    double *part = (double *)(dev + o3);
    double *vecs = (double *)(dev + o4);
    double *dout = vecs + kBatchVecs * vec;
    // pinned host staging: descriptors | block map | states | residuals
    const size_t htot = o3 + (size_t)count * sizeof(double) + 256;
    char *host = nullptr;
    RB_CHECK(workspace(ctx, WS_BATCH_HOST, htot, (void **)&host));
    BSys *hsys = (BSys *)host;
    int *hmap = (int *)(host + o1);
    KState *hst = (KState *)(host + o2);
    double *hout = (double *)(host + o3);
    int64_t voff = 0;
    for (int j = 0; j < count; ++j) {
        BSys &B = hsys[j];
        B.n = sys[j].n;
        B.np = pad64(sys[j].n);
        B.q = sys[j].q;
        B.boff = boff[j];
        B.nblk = nblk[j];
        B.pad = 0;
        B.tol2 = tol * tol;
        B.col = sys[j].col;
        B.val = sys[j].val;
        B.dinv = sys[j].dinv;
        B.val32 = sys[j].val32;
        B.binv = sys[j].binv;
        B.b = sys[j].b;
        B.x = sys[j].x;
        double *base = vecs + kBatchVecs * voff;
        B.r = base;
        B.rh = base + B.np;
        B.ph = base + 2 * B.np;
        B.v = base + 3 * B.np;
        B.s = base + 4 * B.np;
        B.sh = base + 5 * B.np;
        B.t = base + 6 * B.np;
        B.p = base + 7 * B.np;
        voff += B.np;
        for (int b = 0; b < nblk[j]; ++b) hmap[boff[j] + b] = j;
    }
    RB_HIP(hipMemcpyAsync(dsys, hsys, dsz, hipMemcpyHostToDevice, s));
    RB_HIP(hipMemcpyAsync(dmap, hmap, msz, hipMemcpyHostToDevice, s));
    const dim3 g((unsigned)total), bl(kKB);
    std::vector<int> it_total(count, 0), good(count, 0);
    for (int j = 0; j < count; ++j) status[j] = RBFFD_E_NOCONV;
    int phase = 0;
    for (int attempt = 0; attempt < 3; ++attempt) {
        // systems already within 10 tol of their true residual stay finished
        for (int j = 0; j < count; ++j) {
            KState z{};
            z.done_at = good[j] ? 1 : 0;
            z.fresh = good[j] ? 0 : 1;
            z.status = RBFFD_OK;
            hst[j] = z;
        }
        RB_HIP(hipMemcpyAsync(dst, hst, ssz, hipMemcpyHostToDevice, s));
        ++phase;   // 1: the "finished" stamp above precedes every later launch
        hipLaunchKernelGGL(kb_init, g, bl, 0, s, dsys, dmap, part, pstride, dst);
        int it = 0, chunk = 4;
        int left = max_iter;
        for (int j = 0; j < count; ++j)
            if (!good[j]) left = std::min(left, max_iter - it_total[j]);
        bool finished = left <= 0;
        while (!finished) {
            const int todo = std::min(chunk, left - it);
            for (int c = 0; c < todo; ++c) {
                hipLaunchKernelGGL(kb_v, g, bl, 0, s, dsys, dmap, part, pstride, dst, 0, ++phase);
                hipLaunchKernelGGL(kb_s, g, bl, 0, s, dsys, dmap, part, pstride, dst, ++phase);
                hipLaunchKernelGGL(kb_t, g, bl, 0, s, dsys, dmap, part, pstride, dst, ++phase);
                hipLaunchKernelGGL(kb_x, g, bl, 0, s, dsys, dmap, part, pstride, dst, ++phase);
            }
            it += todo;
            hipLaunchKernelGGL(kb_v, g, bl, 0, s, dsys, dmap, part, pstride, dst, 1, ++phase);
            RB_HIP(hipGetLastError());
            RB_HIP(hipMemcpyAsync(hst, dst, ssz, hipMemcpyDeviceToHost, s));
            RB_HIP(hipStreamSynchronize(s));
            bool done = true;
            for (int j = 0; j < count; ++j) done = done && hst[j].done_at != 0;
            finished = done || it >= left;
            chunk = std::min(chunk * 2, 32);
        }
        hipLaunchKernelGGL(kb_resid, g, bl, 0, s, dsys, dmap, part, pstride);
        hipLaunchKernelGGL(kb_resid_final, dim3((unsigned)count), bl, 0, s, dsys, part, pstride, dout);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(hout, dout, sizeof(double) * count, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        bool retry = false;
        for (int j = 0; j < count; ++j) {
            if (good[j]) continue;
            it_total[j] += hst[j].iters;
            relres[j] = hout[j];
            const bool stopped = hst[j].done_at != 0;
            status[j] = stopped ? hst[j].status : RBFFD_E_NOCONV;
            if (stopped && status[j] == RBFFD_OK) {
                if (hout[j] <= 10.0 * tol)
                    good[j] = 1;
                else
                    retry = true;   // recursive residual drifted: iterate again from x
            }
        }
        if (!retry) break;
    }
    for (int j = 0; j < count; ++j) {
        iters[j] = it_total[j];
        if (!good[j] && status[j] == RBFFD_OK) status[j] = RBFFD_E_NOCONV;
    }
    return RBFFD_OK;
}


// ---- continuous batching ------------------------------------------------------
// Systems join and leave a running batch between chunks of iterations. Each
// system keeps its own work vectors and state; when the set changes the block
// ranges are rebuilt (a system's result does not depend on its range: its
// reductions always run over its own blocks in order), states move with their
// systems, and ||r||^2 of moved systems is taken from their state once.
struct ServerSys {
    int64_t ticket = 0;
    BatchSystem sys{};
    double tol = 0.0;
    int max_iter = 0;
    double *vec = nullptr;
    size_t vbytes = 0;
    KState st{};
    int iters_done = 0;   // iterations of finished attempts
    int attempts = 0;
};

struct Server {
    rbffd_ctx *ctx = nullptr;
    std::vector<ServerSys> active;
    std::vector<ServerSys> finished;
    std::vector<int> fin_status;
    std::vector<double> fin_relres;
    int64_t next_ticket = 1;
    int phase = 0;
    bool dirty = true;
    // layout buffers
    char *dev = nullptr;
    size_t dev_bytes = 0;
    char *host = nullptr;
    size_t host_bytes = 0;
    int total_blocks = 0;
    BSys *dsys = nullptr;
    int *dmap = nullptr;
    KState *dst = nullptr;
    double *part = nullptr, *dout = nullptr;
    BSys *hsys = nullptr;
    int *hmap = nullptr;
    KState *hst = nullptr;
    double *hout = nullptr;
};

int server_create(rbffd_ctx *ctx, Server **out)
{
    Server *sv = new Server();
    sv->ctx = ctx;
    *out = sv;
    return RBFFD_OK;
}

void server_destroy(Server *sv)
{
    if (!sv) return;
    (void)hipDeviceSynchronize();
    for (auto &a : sv->active) dev_free(sv->ctx, a.vec, a.vbytes);
    for (auto &a : sv->finished) dev_free(sv->ctx, a.vec, a.vbytes);
    if (sv->dev) dev_free(sv->ctx, sv->dev, sv->dev_bytes);
    if (sv->host) (void)hipHostFree(sv->host);
    delete sv;
}

int server_submit(Server *sv, const BatchSystem &sys, double tol, int max_iter, int64_t *ticket)
{
    ServerSys a;
    a.sys = sys;
    a.tol = tol;
    a.max_iter = max_iter;
    a.vbytes = sizeof(double) * kBatchVecs * pad64(sys.n);
    RB_CHECK(dev_alloc(sv->ctx, (void **)&a.vec, a.vbytes));
    a.ticket = sv->next_ticket++;
    a.st = KState{};
    a.st.fresh = 1;
    a.st.status = RBFFD_OK;
    sv->active.push_back(a);
    sv->dirty = true;
    *ticket = a.ticket;
    return RBFFD_OK;
}

static int server_layout(Server *sv, hipStream_t s)
{
    const int count = (int)sv->active.size();
    int64_t total = 0;
    std::vector<int> boff(count), nblk(count);
    for (int j = 0; j < count; ++j) {
        int64_t b = (sv->active[j].sys.n + kKB - 1) / kKB;
        if (b > kKMaxBlocks) b = kKMaxBlocks;
        nblk[j] = (int)std::max<int64_t>(1, b);
        boff[j] = (int)total;
        total += nblk[j];
    }
    if (total > (int64_t)INT32_MAX / P_COUNT) return fail(RBFFD_E_ARG, "batch too large");
    const size_t dsz = sizeof(BSys) * count, msz = sizeof(int) * total, ssz = sizeof(KState) * count;
    const size_t psz = sizeof(double) * P_COUNT * total;
    const size_t o1 = (dsz + 255) / 256 * 256, o2 = o1 + (msz + 255) / 256 * 256, o3 = o2 + (ssz + 255) / 256 * 256,
                 o4 = o3 + (psz + 255) / 256 * 256, dtot = o4 + sizeof(double) * count + 256;
    if (sv->dev_bytes < dtot) {
        RB_HIP(hipStreamSynchronize(s));
        if (sv->dev) dev_free(sv->ctx, sv->dev, sv->dev_bytes);
        sv->dev = nullptr;
        sv->dev_bytes = 0;
        RB_CHECK(dev_alloc(sv->ctx, (void **)&sv->dev, dtot + dtot / 4));
        sv->dev_bytes = dtot + dtot / 4;
    }
    const size_t htot = o3 + sizeof(double) * count + 256;
    if (sv->host_bytes < htot) {
        RB_HIP(hipStreamSynchronize(s));
        if (sv->host) (void)hipHostFree(sv->host);
        sv->host = nullptr;
        sv->host_bytes = 0;
        RB_HIP(hipHostMalloc((void **)&sv->host, htot + htot / 4, hipHostMallocDefault));
        sv->host_bytes = htot + htot / 4;
    }
    sv->dsys = (BSys *)sv->dev;
    sv->dmap = (int *)(sv->dev + o1);
    sv->dst = (KState *)(sv->dev + o2);
    sv->part = (double *)(sv->dev + o3);
    sv->dout = (double *)(sv->dev + o4);
    sv->hsys = (BSys *)sv->host;
    sv->hmap = (int *)(sv->host + o1);
    sv->hst = (KState *)(sv->host + o2);
    sv->hout = (double *)(sv->host + o3);
    sv->total_blocks = (int)total;
    for (int j = 0; j < count; ++j) {
        ServerSys &a = sv->active[j];
        BSys &B = sv->hsys[j];
        B.n = a.sys.n;
        B.np = pad64(a.sys.n);
        B.q = a.sys.q;
        B.boff = boff[j];
        B.nblk = nblk[j];
        B.pad = 0;
        B.tol2 = a.tol * a.tol;
        B.col = a.sys.col;
        B.val = a.sys.val;
        B.dinv = a.sys.dinv;
        B.val32 = a.sys.val32;
        B.binv = a.sys.binv;
        B.b = a.sys.b;
        B.x = a.sys.x;
        B.r = a.vec;
        B.rh = a.vec + B.np;
        B.ph = a.vec + 2 * B.np;
        B.v = a.vec + 3 * B.np;
        B.s = a.vec + 4 * B.np;
        B.sh = a.vec + 5 * B.np;
        B.t = a.vec + 6 * B.np;
        B.p = a.vec + 7 * B.np;
        for (int b = 0; b < nblk[j]; ++b) sv->hmap[boff[j] + b] = j;
        KState k = a.st;
        if (!k.fresh) k.moved = 1;
        sv->hst[j] = k;
    }
    RB_HIP(hipMemcpyAsync(sv->dsys, sv->hsys, dsz, hipMemcpyHostToDevice, s));
    RB_HIP(hipMemcpyAsync(sv->dmap, sv->hmap, msz, hipMemcpyHostToDevice, s));
    RB_HIP(hipMemcpyAsync(sv->dst, sv->hst, ssz, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(kb_init, dim3((unsigned)total), dim3(kKB), 0, s, sv->dsys, sv->dmap, sv->part, (int)total,
                       sv->dst);
    RB_HIP(hipGetLastError());
    sv->dirty = false;
    return RBFFD_OK;
}

int server_run(Server *sv, int iterations, int *n_active, hipStream_t s)
{
    if (sv->active.empty()) {
        *n_active = 0;
        return RBFFD_OK;
    }
    if (sv->dirty) RB_CHECK(server_layout(sv, s));
    const int count = (int)sv->active.size();
    const int total = sv->total_blocks;
    const dim3 g((unsigned)total), bl(kKB);
    int budget = iterations;
    for (auto &a : sv->active) budget = std::min(budget, a.max_iter - a.iters_done - a.st.iters);
    budget = std::max(budget, 1);
    int it = 0, chunk = 4;
    bool all_done = false;
    while (it < budget && !all_done) {
        const int todo = std::min(chunk, budget - it);
        for (int c = 0; c < todo; ++c) {
            hipLaunchKernelGGL(kb_v, g, bl, 0, s, sv->dsys, sv->dmap, sv->part, total, sv->dst, 0, ++sv->phase);
            hipLaunchKernelGGL(kb_s, g, bl, 0, s, sv->dsys, sv->dmap, sv->part, total, sv->dst, ++sv->phase);
            hipLaunchKernelGGL(kb_t, g, bl, 0, s, sv->dsys, sv->dmap, sv->part, total, sv->dst, ++sv->phase);
            hipLaunchKernelGGL(kb_x, g, bl, 0, s, sv->dsys, sv->dmap, sv->part, total, sv->dst, ++sv->phase);
        }
        it += todo;
        hipLaunchKernelGGL(kb_v, g, bl, 0, s, sv->dsys, sv->dmap, sv->part, total, sv->dst, 1, ++sv->phase);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(sv->hst, sv->dst, sizeof(KState) * count, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        all_done = true;
        for (int j = 0; j < count; ++j) all_done = all_done && sv->hst[j].done_at != 0;
        chunk = std::min(chunk * 2, 32);
    }
    for (int j = 0; j < count; ++j) sv->active[j].st = sv->hst[j];
    // systems that stopped or used their iterations: true residual
    bool any = false;
    for (auto &a : sv->active)
        any = any || a.st.done_at != 0 || a.iters_done + a.st.iters >= a.max_iter;
    if (any) {
        hipLaunchKernelGGL(kb_resid, g, bl, 0, s, sv->dsys, sv->dmap, sv->part, total);
        hipLaunchKernelGGL(kb_resid_final, dim3((unsigned)count), bl, 0, s, sv->dsys, sv->part, total, sv->dout);
        RB_HIP(hipGetLastError());
        RB_HIP(hipMemcpyAsync(sv->hout, sv->dout, sizeof(double) * count, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        std::vector<ServerSys> keep;
        for (int j = 0; j < count; ++j) {
            ServerSys &a = sv->active[j];
            const bool stopped = a.st.done_at != 0;
            const bool out_of_iters = a.iters_done + a.st.iters >= a.max_iter;
            if (!stopped && !out_of_iters) {
                keep.push_back(a);
                continue;
            }
            const double rel = sv->hout[j];
            int status = stopped ? a.st.status : RBFFD_E_NOCONV;
            if (stopped && status == RBFFD_OK && rel > 10.0 * a.tol && a.attempts < 2 && !out_of_iters) {
                // the recursive residual drifted: iterate again from x
                a.iters_done += a.st.iters;
                a.attempts += 1;
                a.st = KState{};
                a.st.fresh = 1;
                a.st.status = RBFFD_OK;
                keep.push_back(a);
                sv->dirty = true;
                continue;
            }
            if (status == RBFFD_OK && rel > 10.0 * a.tol) status = RBFFD_E_NOCONV;
            a.iters_done += a.st.iters;
            dev_free(sv->ctx, a.vec, a.vbytes);
            a.vec = nullptr;
            sv->finished.push_back(a);
            sv->fin_status.push_back(status);
            sv->fin_relres.push_back(rel);
            sv->dirty = true;
        }
        sv->active.swap(keep);
    }
    *n_active = (int)sv->active.size();
    return RBFFD_OK;
}

int server_poll(Server *sv, int max, int64_t *tickets, int *iters, int *status, double *relres, int *count)
{
    const int m = std::min<int>(max, (int)sv->finished.size());
    for (int i = 0; i < m; ++i) {
        tickets[i] = sv->finished[i].ticket;
        iters[i] = sv->finished[i].iters_done;
        status[i] = sv->fin_status[i];
        relres[i] = sv->fin_relres[i];
    }
    sv->finished.erase(sv->finished.begin(), sv->finished.begin() + m);
    sv->fin_status.erase(sv->fin_status.begin(), sv->fin_status.begin() + m);
    sv->fin_relres.erase(sv->fin_relres.begin(), sv->fin_relres.begin() + m);
    *count = m;
    return RBFFD_OK;
}


// ---- kernel times of the Krylov iteration --------------------------------
// Mean durations of the four kernels of one FP64 Jacobi BiCGSTAB iteration on
// one system, for roofline measurement. With tolerance 0 nothing stops the
// solve, and KV, KS and KT are idempotent within an iteration (they read the
// state and vectors the previous kernels left and rewrite the same outputs), so
// each is timed by `reps` back-to-back launches between two events on the
// stream; whole iterations are timed the same way, and KX is the remainder.
int krylov_kernel_times(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, const double *dinv,
                        const double *b, double *x, int reps, double *us, hipStream_t s)
{
    Work w;
    RB_CHECK(get_work<double>(ctx, pad64(n), 1, &w));
    KState *hst = nullptr;
    RB_CHECK(host_scratch(ctx, kHostKrylov, sizeof(KState) * kMaxRhs, (void **)&hst));
    const int64_t np = pad64(n);
    const int nblk = krylov_blocks(n);
    const dim3 g(nblk), bl(kKB);
    double *r = (double *)w.r, *rh = (double *)w.rh, *ph = (double *)w.ph, *v = (double *)w.v, *sv = (double *)w.s,
           *sh = (double *)w.sh, *t = (double *)w.t;
    const bool nt = matrix_nt(n, q, sizeof(double));
    const auto kv = kv_for<double, double, 1>(q, nt);
    const auto kt = kt_for<double, double, 1>(q, nt);
    int phase = 0;
    auto iteration = [&]() {
        hipLaunchKernelGGL(kv, g, bl, 0, s, n, np, q, col, val, rh, ph, v, x, n, w.part, w.st, nblk, 0.0, 0, ++phase);
        hipLaunchKernelGGL((k_s<double, 1>), g, bl, 0, s, n, np, dinv, r, rh, v, sv, sh, w.part, w.st, nblk, ++phase);
        hipLaunchKernelGGL(kt, g, bl, 0, s, n, np, q, col, val, x, n, ph, sv, sh, rh, t, w.part, w.st, nblk, 0.0,
                           ++phase);
        hipLaunchKernelGGL((k_x<double, 1>), g, bl, 0, s, n, np, dinv, x, n, ph, sv, t, v, r, rh, w.part, w.st, nblk,
                           ++phase);
    };
    hipLaunchKernelGGL(k_clear_states, dim3(1), dim3(64), 0, s, w.st);
    hipLaunchKernelGGL((k_init<double, 1>), g, bl, 0, s, n, np, q, col, val, dinv, b, n, x, n, r, rh, ph, w.part);
    for (int i = 0; i < 3; ++i) iteration();
    RB_HIP(hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RB_HIP(hipEventCreate(&e0));
    hipError_t err = hipEventCreate(&e1);
    if (err != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(err, "hipEventCreate");
    }
    float ms[4] = {0, 0, 0, 0};
    // KV, then KS, then KT, each repeated in place; then whole iterations
    for (int stage = 0; stage < 4 && err == hipSuccess; ++stage) {
        err = hipEventRecord(e0, s);
        for (int r_ = 0; r_ < reps && err == hipSuccess; ++r_) {
            if (stage == 0)
                hipLaunchKernelGGL(kv, g, bl, 0, s, n, np, q, col, val, rh, ph, v, x, n, w.part, w.st, nblk, 0.0, 0,
                                   phase + 1);
            else if (stage == 1)
                hipLaunchKernelGGL((k_s<double, 1>), g, bl, 0, s, n, np, dinv, r, rh, v, sv, sh, w.part, w.st, nblk,
                                   phase + 2);
            else if (stage == 2)
                hipLaunchKernelGGL(kt, g, bl, 0, s, n, np, q, col, val, x, n, ph, sv, sh, rh, t, w.part, w.st, nblk,
                                   0.0, phase + 3);
            else
                iteration();
        }
        if (stage == 2) {
            hipLaunchKernelGGL((k_x<double, 1>), g, bl, 0, s, n, np, dinv, x, n, ph, sv, t, v, r, rh, w.part, w.st,
                               nblk, phase + 4);
            phase += 4;
        }
        if (err == hipSuccess) err = hipGetLastError();
        if (err == hipSuccess) err = hipEventRecord(e1, s);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms[stage], e0, e1);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(err, "krylov_kernel_times");
    RB_HIP(hipMemcpyAsync(hst, w.st, sizeof(KState), hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    if (hst[0].done_at != 0)
        return fail(RBFFD_E_BREAKDOWN, "the timed BiCGSTAB iteration broke down; no kernel times");
    for (int i = 0; i < 4; ++i) us[i] = 1e3 * ms[i] / reps;
    us[4] = us[3];                          // whole iteration
    us[3] = us[4] - us[0] - us[1] - us[2];  // KX: the remainder
    return RBFFD_OK;
}

// ---- allocation-free pressure-correction solve -----------------------------
// For callers that cannot allocate (graph capture, serving loops): the Krylov
// vectors, partials and state records live in a fixed device array of this
// file instead of the context's workspace. Every device that loads the library
// holds one copy of the array until the process ends; calls on one device share
// it, so calls that overlap on one device race. Its address on each device is
// taken once, by the context's set-up on that device (noalloc_init), and only
// that address is handed to kernels: in host code the array's name is not a
// device address.
constexpr size_t kNoAllocFixed = size_t(1) << 20;   // partials, states, residual partials
static_assert((size_t)RBFFD_NOALLOC_SCRATCH_BYTES == kNoAllocFixed + (size_t)RBFFD_NOALLOC_MAX_N * 7 * sizeof(double),
              "the scratch array holds the fixed region and 7 FP64 vectors of RBFFD_NOALLOC_MAX_N rows");
static_assert(RBFFD_NOALLOC_MAX_N % 64 == 0, "whole 64-row slices");
static_assert(sizeof(double) * (P_COUNT * kMaxRhs * kMaxBlocks + 2 * kMaxRhs * kMaxBlocks + kMaxRhs) +
                      sizeof(KState) * kMaxRhs + 256 <= kNoAllocFixed,
              "fixed region too small");

static __device__ __align__(256) unsigned char scratch[RBFFD_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
unsigned char *g_noalloc_ptr[kNoAllocDevices] = {};
}  // namespace

__global__ void k_tune_rhs(int64_t n, double *__restrict__ b, double *__restrict__ x)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    b[i] = sin(0.37 * (double)i) + 0.5 * cos(1.3 * (double)i);
    x[i] = 0.0;
}

int autotune_solver(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, const double *dinv,
                    int iterations, int *choice, double *us_per_iter, hipStream_t s)
{
    if (iterations < 4) return fail(RBFFD_E_ARG, "autotune needs at least 4 iterations");
    double *bx = nullptr;
    RB_CHECK(dev_alloc(ctx, (void **)&bx, sizeof(double) * 2 * (size_t)n));
    const int cand[4] = {0, 256, 512, 1024};
    double best = 0.0;
    int bestc = 0;
    bool have = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = RBFFD_OK;
    const auto saved = ctx->solver_choice.find({n, q});
    const bool had = saved != ctx->solver_choice.end();
    const int old = had ? saved->second : 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = fail(RBFFD_E_DEVICE, "hipEventCreate");
    for (int c = 0; c < 4 && st == RBFFD_OK; ++c) {
        // one workgroup cannot compete beyond this size: not tried
        const bool tried = cand[c] == 0 || n <= kWGTuneMaxRows;
        double us = -1.0;
        if (tried) {
            ctx->solver_choice[{n, q}] = cand[c];
            for (int rep = 0; rep < 2 && st == RBFFD_OK; ++rep) {   // the first run captures graphs
                hipLaunchKernelGGL(k_tune_rhs, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, bx,
                                   bx + n);
                KrylovResult r;
                (void)hipEventRecord(e0, s);
                st = bicgstab_once(ctx, n, q, col, val, dinv, 1, bx, bx + n, 0.0, iterations, &r, s);
                (void)hipEventRecord(e1, s);
                (void)hipEventSynchronize(e1);
                float ms = 0.0f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                us = 1e3 * ms / std::max(r.iters[0], 1);
            }
        }
        if (us_per_iter) us_per_iter[c] = us;
        if (tried && (!have || us < best)) {
            best = us;
            bestc = cand[c];
            have = true;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free(ctx, bx, sizeof(double) * 2 * (size_t)n);
    if (st != RBFFD_OK) {
        if (had)
            ctx->solver_choice[{n, q}] = old;
        else
            ctx->solver_choice.erase({n, q});
        return st;
    }
    ctx->solver_choice[{n, q}] = bestc;
    if (choice) *choice = bestc;
    return RBFFD_OK;
}

void graph_cache_destroy(rbffd_ctx *ctx)
{
    GraphCache *gc = (GraphCache *)ctx->graphs;
    if (!gc) return;
    for (auto &en : gc->e) (void)hipGraphExecDestroy(en.exec);
    if (gc->cs) (void)hipStreamDestroy(gc->cs);
    delete gc;
    ctx->graphs = nullptr;
}

int noalloc_init(int device)
{
    if (device < 0 || device >= kNoAllocDevices) return fail(RBFFD_E_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return RBFFD_OK;
    void *ptr = nullptr;
    RB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(RBFFD_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
    g_noalloc_ptr[device] = (unsigned char *)ptr;
    return RBFFD_OK;
}

int poisson_solve_noalloc_impl(int device, int64_t n, int q, ColIdx col, const double *val, const double *dinv,
                               const double *b, double *x, double tol, int max_iter, KrylovResult *res,
                               double *relres, hipStream_t s)
{
    if (device < 0 || device >= kNoAllocDevices) return fail(RBFFD_E_ARG, "device index beyond the scratch table");
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        base = g_noalloc_ptr[device];
    }
    if (!base) return fail(RBFFD_E_ARG, "the scratch array of this device was not set up (no context was created on it)");
    const int64_t np = pad64(n);
    if (np > RBFFD_NOALLOC_MAX_N)
        return fail(RBFFD_E_ARG, "poisson_solve_noalloc: " + std::to_string(n) + " rows exceed the scratch limit of " +
                                     std::to_string(RBFFD_NOALLOC_MAX_N));
    // fixed region: partials, state records, residual partials; then the vectors
    Work w;
    w.part = (double *)base;
    w.st = (KState *)(w.part + P_COUNT * kMaxRhs * kMaxBlocks);
    double *rdev = (double *)(base + (((char *)(w.st + kMaxRhs) - (char *)base + 255) / 256) * 256);
    unsigned char *vb = base + kNoAllocFixed;
    const size_t vec = sizeof(double) * np;
    w.r = vb;
    w.rh = vb + vec;
    w.ph = vb + 2 * vec;
    w.v = vb + 3 * vec;
    w.s = vb + 4 * vec;
    w.sh = vb + 5 * vec;
    w.t = vb + 6 * vec;
    // host copies go through the caller's stack (pageable memory, no pinned staging)
    KState hst[kMaxRhs];
    double hout[kMaxRhs];
    KrylovResult acc;
    for (int attempt = 0; attempt < 3; ++attempt) {
        const int left = max_iter - acc.iters[0];
        KrylovResult r1;
        RB_CHECK((bicgstab_t<double, 1>(n, q, col, val, dinv, b, n, x, n, tol, std::max(left, 0), &r1, w, hst, s)));
        acc.iters[0] += r1.iters[0];
        acc.status[0] = r1.status[0];
        RB_CHECK(residual_norms_in(n, q, col, val, 1, b, x, rdev, hout, acc.relres, s));
        if (r1.status[0] != RBFFD_OK || left <= 0 || acc.relres[0] <= 10.0 * tol) break;
    }
    if (acc.status[0] == RBFFD_OK && !(acc.relres[0] <= 10.0 * tol)) acc.status[0] = RBFFD_E_NOCONV;
    *res = acc;
    *relres = acc.relres[0];
    return RBFFD_OK;
}

}  // namespace rbffd
