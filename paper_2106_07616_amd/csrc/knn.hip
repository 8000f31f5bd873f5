// Cloud selection (Sec. 2: a cloud of neighbouring points; Sec. 3.1: one-sided
// clouds at boundaries): the q nearest points of every point, itself included,
// in the total order (squared distance, index).
//
// Points are binned into a uniform grid (a few points per cell) with a count
// sort. One wavefront serves one query: it visits shells of cells of growing
// Chebyshev radius around the query's cell, keeps the q best keys in LDS, and
// stops as soon as the q-th key is closer than every point the visited box
// could have missed. Because the selection is by a total order on exactly
// computed keys, the result does not depend on visiting order.
#include <cfloat>
#include <cmath>

#include "internal.h"
#include "periodic.h"

namespace rbffd {

namespace {

struct Grid {
    double lo[3];
    double cs[3];
    double inv[3];
    int nc[3];
};

// Squared distance without contraction: ((dx*dx + dy*dy) + dz*dz).
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

__device__ inline bool key_less(double d1, int i1, double d2, int i2)
{
    return d1 < d2 || (d1 == d2 && i1 < i2);
}

template <int DIM>
__device__ inline int cell_coord(double x, const Grid &g, int d)
{
    double t = floor((x - g.lo[d]) * g.inv[d]);
    int c = (t < 0.0) ? 0 : (t > (double)(g.nc[d] - 1) ? g.nc[d] - 1 : (int)t);
    return c;
}

template <int DIM>
__device__ inline int64_t cell_linear(const int *c, const Grid &g)
{
    int64_t id = c[0] + (int64_t)g.nc[0] * c[1];
    if (DIM == 3) id += (int64_t)g.nc[0] * g.nc[1] * c[2];
    return id;
}

// ---- bounding box --------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kBlock) void bbox_partial(const double *__restrict__ xyz, int64_t n,
                                                       double *__restrict__ part)
{
    __shared__ double lds[6][kBlock / 64];
    double mn[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, mx[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        for (int d = 0; d < DIM; ++d) {
            double v = xyz[i * DIM + d];
            // fmin/fmax skip NaN: a NaN coordinate widens the box to +-infinity
            // instead, so the host's finiteness check sees it
            mn[d] = (v != v) ? -INFINITY : fmin(mn[d], v);
            mx[d] = (v != v) ? INFINITY : fmax(mx[d], v);
        }
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    for (int d = 0; d < DIM; ++d) {
        double a = mn[d], b = mx[d];
        for (int o = 32; o > 0; o >>= 1) {
            a = fmin(a, __shfl_xor(a, o, 64));
            b = fmax(b, __shfl_xor(b, o, 64));
        }
        if (l == 0) {
            lds[d][w] = a;
            lds[3 + d][w] = b;
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const bool isMin = threadIdx.x < 3;
        double r = isMin ? DBL_MAX : -DBL_MAX;
        for (int j = 0; j < kBlock / 64; ++j) r = isMin ? fmin(r, lds[threadIdx.x][j]) : fmax(r, lds[threadIdx.x][j]);
        part[blockIdx.x * 6 + threadIdx.x] = r;
    }
}

// One wavefront (64 threads): lane l folds partials l, l + 64, ... of the six
// extents, then a shuffle reduction finishes them. Minima and maxima are exact
// in any order, and the partials hold no NaN (bbox_partial widens the box to
// +-infinity instead).
__global__ __launch_bounds__(64) void bbox_final(const double *__restrict__ part, int np, double *__restrict__ out)
{
    const int l = threadIdx.x;
    double r[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) r[d] = (d < 3) ? DBL_MAX : -DBL_MAX;
    for (int j = l; j < np; j += 64)
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const double v = part[j * 6 + d];
            r[d] = (d < 3) ? fmin(r[d], v) : fmax(r[d], v);
        }
#pragma unroll
    for (int d = 0; d < 6; ++d)
        for (int o = 32; o > 0; o >>= 1) {
            const double u = __shfl_xor(r[d], o, 64);
            r[d] = (d < 3) ? fmin(r[d], u) : fmax(r[d], u);
        }
    if (l == 0)
#pragma unroll
        for (int d = 0; d < 6; ++d) out[d] = r[d];
}

// ---- binning ------------------------------------------------------------
template <int DIM>
__global__ void cell_count(const double *__restrict__ xyz, int64_t n, Grid g, int32_t *__restrict__ cell_of,
                           int32_t *__restrict__ count)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) c[d] = cell_coord<DIM>(xyz[i * DIM + d], g, d);
    int32_t id = (int32_t)cell_linear<DIM>(c, g);
    cell_of[i] = id;
    atomicAdd(&count[id], 1);
}

template <int DIM>
__global__ void cell_scatter(const double *__restrict__ xyz, int64_t n, const int32_t *__restrict__ cell_of,
                             const int32_t *__restrict__ start, int32_t *__restrict__ cursor,
                             int32_t *__restrict__ sidx, double *__restrict__ sxyz)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = cell_of[i];
    int32_t pos = start[c] + atomicAdd(&cursor[c], 1);
    sidx[pos] = (int32_t)i;
    for (int d = 0; d < DIM; ++d) sxyz[(int64_t)pos * DIM + d] = xyz[i * DIM + d];
}

// ---- query ---------------------------------------------------------------
template <int DIM>
struct QueryState {
    double Ld[2][kMaxQ];
    int Li[2][kMaxQ];
    double Bd[64];
    int Bi[64];
};

// Merge the batch (nbat keys) into the sorted list (cnt keys) keeping the q
// smallest; every key lands at its rank in the union.
template <int DIM>
__device__ inline void merge_batch(QueryState<DIM> &S, int &cur, int &cnt, int nbat, int q)
{
    __syncthreads();
    const int lane = threadIdx.x;
    const int nxt = cur ^ 1;
    if (lane < nbat) {
        const double bd = S.Bd[lane];
        const int bi = S.Bi[lane];
        int rb = 0;
        for (int m = 0; m < nbat; ++m) rb += key_less(S.Bd[m], S.Bi[m], bd, bi);
        int lo = 0, hi = cnt;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (key_less(S.Ld[cur][mid], S.Li[cur][mid], bd, bi))
                lo = mid + 1;
            else
                hi = mid;
        }
        const int pos = lo + rb;
        if (pos < q) {
            S.Ld[nxt][pos] = bd;
            S.Li[nxt][pos] = bi;
        }
    }
    for (int j = lane; j < cnt; j += 64) {
        const double ld = S.Ld[cur][j];
        const int li = S.Li[cur][j];
        int rb = 0;
        for (int m = 0; m < nbat; ++m) rb += key_less(S.Bd[m], S.Bi[m], ld, li);
        const int pos = j + rb;
        if (pos < q) {
            S.Ld[nxt][pos] = ld;
            S.Li[nxt][pos] = li;
        }
    }
    cnt = min(q, cnt + nbat);
    cur = nxt;
    __syncthreads();
}

template <int DIM>
__device__ inline void scan_range(QueryState<DIM> &S, const double *xq, int32_t start, int32_t end,
                                  const int32_t *__restrict__ sidx, const double *__restrict__ sxyz,
                                  int &cur, int &cnt, int &nbat, int q)
{
    const int lane = threadIdx.x;
    for (int32_t base = start; base < end; base += 64) {
        const int32_t pidx = base + lane;
        const bool valid = pidx < end;
        double d2 = DBL_MAX;
        int id = 0x7fffffff;
        if (valid) {
            id = sidx[pidx];
            double pc[3];
            for (int d = 0; d < DIM; ++d) pc[d] = sxyz[(int64_t)pidx * DIM + d];
            d2 = sqdist_exact<DIM>(xq, pc);
        }
        bool cand = valid && (cnt < q || key_less(d2, id, S.Ld[cur][q - 1], S.Li[cur][q - 1]));
        uint64_t mask = __ballot(cand);
        int nnew = __popcll(mask);
        if (nnew == 0) continue;
        if (nbat + nnew > 64) {
            merge_batch<DIM>(S, cur, cnt, nbat, q);
            nbat = 0;
        }
        if (cand) {
            int pos = nbat + __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
            S.Bd[pos] = d2;
            S.Bi[pos] = id;
        }
        nbat += nnew;
        __syncthreads();
    }
}

template <int DIM>
__global__ __launch_bounds__(64) void knn_query(const double *__restrict__ qxyz, const int32_t *__restrict__ cstart,
                                                const int32_t *__restrict__ sidx, const double *__restrict__ sxyz,
                                                Grid g, int64_t nq, int q, int32_t *__restrict__ nbr)
{
    __shared__ QueryState<DIM> S;
    const int64_t i = blockIdx.x;
    if (i >= nq) return;
    double xq[3] = {0.0, 0.0, 0.0};
    int c[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) {
        xq[d] = qxyz[i * DIM + d];
        c[d] = cell_coord<DIM>(xq[d], g, d);
    }
    double csmin = g.cs[0];
    for (int d = 1; d < DIM; ++d) csmin = fmin(csmin, g.cs[d]);
    int cur = 0, cnt = 0, nbat = 0;
    for (int R = 0;; ++R) {
        // rows of the shell at Chebyshev radius R: (dy) in 2D, (dy, dz) in 3D
        const int zlo = (DIM == 3) ? -R : 0, zhi = (DIM == 3) ? R : 0;
        for (int dz = zlo; dz <= zhi; ++dz) {
            const int cz = c[2] + dz;
            if (DIM == 3 && (cz < 0 || cz >= g.nc[2])) continue;
            for (int dy = -R; dy <= R; ++dy) {
                const int cy = c[1] + dy;
                if (cy < 0 || cy >= g.nc[1]) continue;
                const int64_t rowbase = (int64_t)g.nc[0] * cy + (DIM == 3 ? (int64_t)g.nc[0] * g.nc[1] * cz : 0);
                const bool full = (abs(dy) == R) || (DIM == 3 && abs(dz) == R);
                if (full) {
                    const int xa = max(c[0] - R, 0), xb = min(c[0] + R, g.nc[0] - 1);
                    scan_range<DIM>(S, xq, cstart[rowbase + xa], cstart[rowbase + xb + 1], sidx, sxyz, cur, cnt, nbat, q);
                } else {
                    if (c[0] - R >= 0)
                        scan_range<DIM>(S, xq, cstart[rowbase + c[0] - R], cstart[rowbase + c[0] - R + 1], sidx, sxyz,
                                        cur, cnt, nbat, q);
                    if (c[0] + R < g.nc[0])
                        scan_range<DIM>(S, xq, cstart[rowbase + c[0] + R], cstart[rowbase + c[0] + R + 1], sidx, sxyz,
                                        cur, cnt, nbat, q);
                }
            }
        }
        if (nbat > 0) {
            merge_batch<DIM>(S, cur, cnt, nbat, q);
            nbat = 0;
        }
        // Stop when the box of radius R covers the grid, or when the q-th key is
        // closer than the nearest face of the box that has points beyond it.
        bool covers = true;
        double rg = DBL_MAX;
        for (int d = 0; d < DIM; ++d) {
            if (c[d] - R > 0) {
                covers = false;
                rg = fmin(rg, xq[d] - (g.lo[d] + (double)(c[d] - R) * g.cs[d]));
            }
            if (c[d] + R < g.nc[d] - 1) {
                covers = false;
                rg = fmin(rg, (g.lo[d] + (double)(c[d] + R + 1) * g.cs[d]) - xq[d]);
            }
        }
        if (covers) break;
        if (cnt == q) {
            rg -= 1e-7 * csmin;   // margin against rounding of the binning
            if (rg > 0.0 && S.Ld[cur][q - 1] < rg * rg) break;
        }
    }
    for (int a = threadIdx.x; a < q; a += 64) nbr[i * q + a] = S.Li[cur][a];
}

}  // namespace

// ---- exclusive scan (int32) ------------------------------------------------
namespace {
constexpr int kScanPer = 4;
constexpr int kScanTile = kBlock * kScanPer;

__global__ __launch_bounds__(kBlock) void scan_tile(const int32_t *__restrict__ in, int32_t *__restrict__ out,
                                                    int64_t n, int32_t *__restrict__ tile_sum)
{
    __shared__ int32_t wsum[kBlock / 64];
    const int64_t base = blockIdx.x * (int64_t)kScanTile + threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int32_t t = 0;
    for (int j = 0; j < kScanPer; ++j) {
        v[j] = (base + j < n) ? in[base + j] : 0;
        t += v[j];
    }
    // inclusive wave scan of per-thread totals
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t incl = t;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int32_t woff = 0;
    for (int j = 0; j < w; ++j) woff += wsum[j];
    int32_t run = woff + incl - t;
    for (int j = 0; j < kScanPer; ++j) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == kBlock - 1) tile_sum[blockIdx.x] = woff + incl;
}

__global__ void scan_add(int32_t *__restrict__ out, int64_t n, const int32_t *__restrict__ tile_off)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / kScanTile];
}
}  // namespace

int scan_exclusive(rbffd_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, hipStream_t s)
{
    // out[0..n) = exclusive scan, out[n] = total
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    int32_t *tsum = nullptr, *toff = nullptr;
    RB_CHECK(dev_alloc(ctx, (void **)&tsum, sizeof(int32_t) * (tiles + 1) * 2));
    toff = tsum + tiles + 1;
    hipLaunchKernelGGL(scan_tile, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, out, n, tsum);
    RB_HIP(hipGetLastError());
    int st = RBFFD_OK;
    if (tiles > 1) {
        st = scan_exclusive(ctx, tsum, toff, tiles, s);
        if (st == RBFFD_OK) {
            hipLaunchKernelGGL(scan_add, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, out, n, toff);
            if (hipGetLastError() != hipSuccess) st = fail(RBFFD_E_DEVICE, "scan_add launch failed");
        }
        if (st == RBFFD_OK)
            (void)hipMemcpyAsync(out + n, toff + tiles, sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    } else {
        (void)hipMemcpyAsync(out + n, tsum, sizeof(int32_t), hipMemcpyDeviceToDevice, s);
    }
    (void)hipStreamSynchronize(s);
    dev_free(ctx, tsum, sizeof(int32_t) * (tiles + 1) * 2);
    return st;
}

// ---- periodic clouds (Sec. 3.1) -------------------------------------------
// Image of point j under shift k: x + L or x - L along the shifted axes (the
// same floating-point operations as any host-side construction), kept when
// within band of the box along every periodic axis.
template <int DIM>
__device__ inline bool periodic_image(const double *__restrict__ xyz, int64_t j, const PeriodicShifts &P, int k,
                                      double *y)
{
    bool keep = true;
    for (int d = 0; d < DIM; ++d) {
        const double v = xyz[j * DIM + d];
        const int md = P.m[k][d];
        y[d] = (md > 0) ? v + P.L[d] : ((md < 0) ? v - P.L[d] : v);
        if (P.L[d] > 0.0 && (y[d] < P.lo[d] - P.band || y[d] > P.hi[d] + P.band)) keep = false;
    }
    return keep;
}

// flag[k n + j] = 1 when point j's image under shift k is kept
template <int DIM>
__global__ void periodic_flags(const double *__restrict__ xyz, int64_t n, PeriodicShifts P, int32_t *__restrict__ flag)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx >= n * P.count) return;
    const int k = (int)(idx / n);
    const int64_t j = idx - (int64_t)k * n;
    double y[3];
    flag[idx] = periodic_image<DIM>(xyz, j, P, k, y) ? 1 : 0;
}

// rows 0..n-1: the points; row n + pos[k n + j]: the kept image of point j
// under shift k
template <int DIM>
__global__ void periodic_scatter(const double *__restrict__ xyz, int64_t n, PeriodicShifts P,
                                 const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                                 double *__restrict__ aug, int32_t *__restrict__ owner)
{
    const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (idx < n) {
        for (int d = 0; d < DIM; ++d) aug[idx * DIM + d] = xyz[idx * DIM + d];
        owner[idx] = (int32_t)idx;
        return;
    }
    const int64_t t = idx - n;
    if (t >= n * P.count || !flag[t]) return;
    const int k = (int)(t / n);
    const int64_t j = t - (int64_t)k * n;
    double y[3];
    periodic_image<DIM>(xyz, j, P, k, y);
    const int64_t r = n + pos[t];
    for (int d = 0; d < DIM; ++d) aug[r * DIM + d] = y[d];
    owner[r] = (int32_t)j;
}

template <int DIM>
__global__ void periodic_inside(const double *__restrict__ qxyz, int64_t nq, const double *__restrict__ aug, int q,
                                const int32_t *__restrict__ nbr, double band, const double *__restrict__ margin,
                                int *__restrict__ outside)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nq) return;
    const int64_t j = nbr[t * q + q - 1];
    const double d2 = sqdist_exact<DIM>(qxyz + t * DIM, aug + j * DIM);
    if (!(sqrt(d2) <= (margin ? band - margin[t] : band))) atomicOr(outside, 1);
}

template <int DIM>
__global__ void periodic_wrap(double *__restrict__ qxyz, int64_t nq, PeriodicShifts P, double *__restrict__ margin,
                              int *__restrict__ nonfinite)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nq) return;
    double out = 0.0;
    for (int d = 0; d < DIM; ++d) {
        double v = qxyz[t * DIM + d];
        if (!isfinite(v)) {
            atomicOr(nonfinite, 1);
            return;
        }
        if (!(P.L[d] > 0.0)) continue;
        if (v < P.lo[d] || v >= P.lo[d] + P.L[d]) {
            double r = fmod(v - P.lo[d], P.L[d]);
            if (r < 0.0) r += P.L[d];
            v = P.lo[d] + r;
            qxyz[t * DIM + d] = v;
        }
        out = fmax(out, fmax(P.lo[d] - v, v - P.hi[d]));
    }
    margin[t] = out;
}

__global__ void periodic_remap(int64_t n, int q, const int32_t *__restrict__ owner, int32_t *__restrict__ nbr,
                               unsigned long long *__restrict__ first_dup)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t *row = nbr + i * q;
    for (int a = 0; a < q; ++a) row[a] = owner[row[a]];
    bool dup = false;
    for (int a = 0; a < q && !dup; ++a)
        for (int b = a + 1; b < q; ++b)
            if (row[a] == row[b]) {
                dup = true;
                break;
            }
    if (dup) atomicMin(first_dup, (unsigned long long)i);
}

// Duplicate points (an input error). A point that coincides with another has
// that point at squared distance 0 among its two nearest, since clouds are in
// (d^2, index) order, so the first two entries of each cloud decide it: the
// first entry is another point, or the second lies at distance 0. The lowest
// such point goes to *first (which the launcher sets to INT64_MAX first).
template <int DIM>
__global__ void dup_check_kernel(const double *__restrict__ xyz, const int32_t *__restrict__ nbr, int64_t n, int q,
                                 unsigned long long *__restrict__ first)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j0 = nbr[i * q];
    bool dup = j0 != i;
    if (!dup && q > 1) dup = sqdist_exact<DIM>(xyz + i * DIM, xyz + (int64_t)nbr[i * q + 1] * DIM) == 0.0;
    if (dup) atomicMin(first, (unsigned long long)i);
}

int launch_dup_check(int dim, int64_t n, const double *xyz, int q, const int32_t *nbr, int64_t *first, hipStream_t s)
{
    const long long init = LLONG_MAX;
    RB_HIP(hipMemcpyAsync(first, &init, sizeof(init), hipMemcpyHostToDevice, s));
    if (n <= 0) return RBFFD_OK;
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
    if (dim == 2)
        hipLaunchKernelGGL(dup_check_kernel<2>, grid, block, 0, s, xyz, nbr, n, q, (unsigned long long *)first);
    else
        hipLaunchKernelGGL(dup_check_kernel<3>, grid, block, 0, s, xyz, nbr, n, q, (unsigned long long *)first);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

int device_bbox(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, double *lo, double *hi, hipStream_t s)
{
    const int nbb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + kBlock - 1) / kBlock));
    double *part = nullptr;
    RB_CHECK(dev_alloc(ctx, (void **)&part, sizeof(double) * (nbb * 6 + 6)));
    double *bb = part + nbb * 6;
    if (dim == 2)
        hipLaunchKernelGGL(bbox_partial<2>, dim3(nbb), dim3(kBlock), 0, s, xyz, n, part);
    else
        hipLaunchKernelGGL(bbox_partial<3>, dim3(nbb), dim3(kBlock), 0, s, xyz, n, part);
    hipLaunchKernelGGL(bbox_final, dim3(1), dim3(64), 0, s, part, nbb, bb);
    double hb[6];
    hipError_t e = hipMemcpyAsync(hb, bb, sizeof(hb), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(ctx, part, sizeof(double) * (nbb * 6 + 6));
    if (e != hipSuccess) return hip_fail(e, "bounding box");
    for (int d = 0; d < dim; ++d) {
        if (!std::isfinite(hb[d]) || !std::isfinite(hb[3 + d])) return fail(RBFFD_E_ARG, "non-finite coordinates");
        lo[d] = hb[d];
        hi[d] = hb[3 + d];
    }
    return RBFFD_OK;
}

int launch_periodic_images(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, const PeriodicShifts &P,
                           double **aug, int32_t **owner, int64_t *naug, size_t *abytes, size_t *obytes,
                           hipStream_t s)
{
    *aug = nullptr;
    *owner = nullptr;
    const int64_t m = n * P.count;
    int32_t *flag = nullptr;
    const size_t fbytes = sizeof(int32_t) * (2 * m + 1);
    RB_CHECK(dev_alloc(ctx, (void **)&flag, fbytes));
    int32_t *pos = flag + m;
    int st = RBFFD_OK;
    int32_t total = 0;
    if (m > 0) {
        const dim3 g((unsigned)((m + kBlock - 1) / kBlock));
        if (dim == 2)
            hipLaunchKernelGGL(periodic_flags<2>, g, dim3(kBlock), 0, s, xyz, n, P, flag);
        else
            hipLaunchKernelGGL(periodic_flags<3>, g, dim3(kBlock), 0, s, xyz, n, P, flag);
        if (hipGetLastError() != hipSuccess) st = fail(RBFFD_E_DEVICE, "periodic image flags launch failed");
        if (st == RBFFD_OK) st = scan_exclusive(ctx, flag, pos, m, s);
        if (st == RBFFD_OK) {
            hipError_t e = hipMemcpyAsync(&total, pos + m, sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(e, "periodic image count");
        }
    }
    const int64_t rows = n + (int64_t)total;
    if (st == RBFFD_OK && rows >= (int64_t(1) << 31)) st = fail(RBFFD_E_ARG, "too many periodic images");
    *abytes = sizeof(double) * (size_t)rows * dim;
    *obytes = sizeof(int32_t) * (size_t)rows;
    if (st == RBFFD_OK) st = dev_alloc(ctx, (void **)aug, *abytes);
    if (st == RBFFD_OK) {
        st = dev_alloc(ctx, (void **)owner, *obytes);
        if (st != RBFFD_OK) {
            dev_free(ctx, *aug, *abytes);
            *aug = nullptr;
        }
    }
    if (st == RBFFD_OK) {
        const dim3 g((unsigned)((n + m + kBlock - 1) / kBlock));
        if (dim == 2)
            hipLaunchKernelGGL(periodic_scatter<2>, g, dim3(kBlock), 0, s, xyz, n, P, flag, pos, *aug, *owner);
        else
            hipLaunchKernelGGL(periodic_scatter<3>, g, dim3(kBlock), 0, s, xyz, n, P, flag, pos, *aug, *owner);
        if (hipGetLastError() != hipSuccess) st = fail(RBFFD_E_DEVICE, "periodic image scatter launch failed");
        (void)hipStreamSynchronize(s);
    }
    dev_free(ctx, flag, fbytes);
    *naug = rows;
    if (st != RBFFD_OK && *aug) {
        dev_free(ctx, *aug, *abytes);
        dev_free(ctx, *owner, *obytes);
        *aug = nullptr;
        *owner = nullptr;
    }
    return st;
}

int launch_periodic_inside(int dim, int64_t nq, const double *qxyz, const double *aug, int q, const int32_t *nbr,
                           double band, const double *margin, int *outside, hipStream_t s)
{
    const int zero = 0;
    RB_HIP(hipMemcpyAsync(outside, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    if (nq <= 0) return RBFFD_OK;
    const dim3 g((unsigned)((nq + kBlock - 1) / kBlock));
    if (dim == 2)
        hipLaunchKernelGGL(periodic_inside<2>, g, dim3(kBlock), 0, s, qxyz, nq, aug, q, nbr, band, margin, outside);
    else
        hipLaunchKernelGGL(periodic_inside<3>, g, dim3(kBlock), 0, s, qxyz, nq, aug, q, nbr, band, margin, outside);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

int launch_periodic_wrap(int dim, int64_t nq, double *qxyz, const PeriodicShifts &P, double *margin, int *nonfinite,
                         hipStream_t s)
{
    const int zero = 0;
    RB_HIP(hipMemcpyAsync(nonfinite, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    if (nq <= 0) return RBFFD_OK;
    const dim3 g((unsigned)((nq + kBlock - 1) / kBlock));
    if (dim == 2)
        hipLaunchKernelGGL(periodic_wrap<2>, g, dim3(kBlock), 0, s, qxyz, nq, P, margin, nonfinite);
    else
        hipLaunchKernelGGL(periodic_wrap<3>, g, dim3(kBlock), 0, s, qxyz, nq, P, margin, nonfinite);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

int launch_periodic_remap(int64_t n, int q, const int32_t *owner, int32_t *nbr, int64_t *first_dup, hipStream_t s)
{
    const long long init = LLONG_MAX;
    RB_HIP(hipMemcpyAsync(first_dup, &init, sizeof(init), hipMemcpyHostToDevice, s));
    if (n <= 0) return RBFFD_OK;
    hipLaunchKernelGGL(periodic_remap, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n, q, owner,
                       nbr, (unsigned long long *)first_dup);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

int launch_knn(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int q, int32_t *nbr, hipStream_t s)
{
    return launch_knn_points(ctx, dim, n, xyz, n, xyz, q, nbr, s);
}

// The q nearest cloud points of each of nq query points (qxyz [nq][dim]); a
// query outside the cloud's bounding box starts from the nearest cell and
// widens its shells until the box covers the grid.
int launch_knn_points(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int64_t nq, const double *qxyz, int q,
                      int32_t *nbr, hipStream_t s)
{
    if (qxyz != xyz && nq > 0) {
        // query coordinates must be finite (their bounding box is)
        const int nbq = (int)std::min<int64_t>(1024, (nq + kBlock - 1) / kBlock);
        double *qpart = nullptr;
        RB_CHECK(dev_alloc(ctx, (void **)&qpart, sizeof(double) * (nbq * 6 + 6)));
        double *qbb = qpart + nbq * 6;
        if (dim == 2)
            hipLaunchKernelGGL(bbox_partial<2>, dim3(nbq), dim3(kBlock), 0, s, qxyz, nq, qpart);
        else
            hipLaunchKernelGGL(bbox_partial<3>, dim3(nbq), dim3(kBlock), 0, s, qxyz, nq, qpart);
        hipLaunchKernelGGL(bbox_final, dim3(1), dim3(64), 0, s, qpart, nbq, qbb);
        double hq[6];
        hipError_t eq = hipMemcpyAsync(hq, qbb, sizeof(hq), hipMemcpyDeviceToHost, s);
        if (eq == hipSuccess) eq = hipStreamSynchronize(s);
        dev_free(ctx, qpart, sizeof(double) * (nbq * 6 + 6));
        if (eq != hipSuccess) return hip_fail(eq, "query bounding box");
        for (int d = 0; d < dim; ++d)
            if (!std::isfinite(hq[d]) || !std::isfinite(hq[3 + d])) return fail(RBFFD_E_ARG, "non-finite query coordinates");
    }
    // bounding box
    const int nbb = (int)std::min<int64_t>(1024, (n + kBlock - 1) / kBlock);
    double *part = nullptr;
    RB_CHECK(dev_alloc(ctx, (void **)&part, sizeof(double) * (nbb * 6 + 6)));
    double *bb = part + nbb * 6;
    if (dim == 2)
        hipLaunchKernelGGL(bbox_partial<2>, dim3(nbb), dim3(kBlock), 0, s, xyz, n, part);
    else
        hipLaunchKernelGGL(bbox_partial<3>, dim3(nbb), dim3(kBlock), 0, s, xyz, n, part);
    hipLaunchKernelGGL(bbox_final, dim3(1), dim3(64), 0, s, part, nbb, bb);
    double hb[6];
    hipError_t e = hipMemcpyAsync(hb, bb, sizeof(hb), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(ctx, part, sizeof(double) * (nbb * 6 + 6));
    if (e != hipSuccess) return hip_fail(e, "bounding box");
    for (int d = 0; d < dim; ++d)
        if (!std::isfinite(hb[d]) || !std::isfinite(hb[3 + d])) return fail(RBFFD_E_ARG, "non-finite coordinates");

    // grid: about q/2 (2D) or q/3 (3D) points per cell
    Grid g{};
    double span[3] = {1, 1, 1}, vol = 1.0;
    int live = 0;
    for (int d = 0; d < dim; ++d) {
        span[d] = hb[3 + d] - hb[d];
        if (span[d] > 0) {
            vol *= span[d];
            ++live;
        }
    }
    const double target = std::max(2.0, dim == 2 ? q / 2.0 : q / 3.0);
    const double hc = live ? std::pow(target * vol / (double)n, 1.0 / live) : 1.0;
    int64_t ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (d >= dim || !(span[d] > 0)) {
            g.lo[d] = (d < dim) ? hb[d] : 0.0;
            g.nc[d] = 1;
            g.cs[d] = 1.0;
            g.inv[d] = 0.0;
            continue;
        }
        int64_t k = (int64_t)std::floor(span[d] / hc);
        k = std::max<int64_t>(1, std::min<int64_t>(k, 1 << 20));
        g.lo[d] = hb[d];
        g.nc[d] = (int)k;
        g.cs[d] = span[d] / (double)k;
        g.inv[d] = 1.0 / g.cs[d];
        ncell *= k;
    }
    if (ncell > (int64_t)4 * n + 64) return fail(RBFFD_E_ARG, "degenerate point distribution");

    // count sort into cells
    // layout: sxyz [n*dim] doubles first (aligned), then the int32 arrays
    const size_t bytes = sizeof(double) * n * dim + sizeof(int32_t) * (2 * n + 3 * (ncell + 1));
    char *buf = nullptr;
    RB_CHECK(dev_alloc(ctx, (void **)&buf, bytes));
    double *sxyz = (double *)buf;
    int32_t *cell_of = (int32_t *)(sxyz + n * dim);
    int32_t *count = cell_of + n;
    int32_t *cstart = count + (ncell + 1);
    int32_t *cursor = cstart + (ncell + 1);
    int32_t *sidx = cursor + (ncell + 1);
    int st = RBFFD_OK;
    e = hipMemsetAsync(count, 0, sizeof(int32_t) * (ncell + 1) * 3, s);
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    if (e == hipSuccess) {
        if (dim == 2)
            hipLaunchKernelGGL(cell_count<2>, dim3(nb), dim3(kBlock), 0, s, xyz, n, g, cell_of, count);
        else
            hipLaunchKernelGGL(cell_count<3>, dim3(nb), dim3(kBlock), 0, s, xyz, n, g, cell_of, count);
        e = hipGetLastError();
    }
    if (e == hipSuccess) st = scan_exclusive(ctx, count, cstart, ncell, s);
    if (e == hipSuccess && st == RBFFD_OK) {
        if (dim == 2)
            hipLaunchKernelGGL(cell_scatter<2>, dim3(nb), dim3(kBlock), 0, s, xyz, n, cell_of, cstart, cursor, sidx, sxyz);
        else
            hipLaunchKernelGGL(cell_scatter<3>, dim3(nb), dim3(kBlock), 0, s, xyz, n, cell_of, cstart, cursor, sidx, sxyz);
        e = hipGetLastError();
    }
    if (e == hipSuccess && st == RBFFD_OK && nq > 0) {
        if (dim == 2)
            hipLaunchKernelGGL(knn_query<2>, dim3((unsigned)nq), dim3(64), 0, s, qxyz, cstart, sidx, sxyz, g, nq, q, nbr);
        else
            hipLaunchKernelGGL(knn_query<3>, dim3((unsigned)nq), dim3(64), 0, s, qxyz, cstart, sidx, sxyz, g, nq, q, nbr);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    dev_free(ctx, buf, bytes);
    if (st != RBFFD_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "neighbour search");
    return RBFFD_OK;
}

}  // namespace rbffd
