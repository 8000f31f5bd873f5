// Assembly of the stored operators (Sec. 2 closing remark: B1 precomputed and
// kept for the whole run) and of the pressure-correction matrix (Eq. pressure
// poisson with the boundary conditions of Sec. 3.1).
//
// Storage is sliced ELL with exactly q entries per row: each row's columns
// ascending (the CSR order), entry a of 64 consecutive rows contiguous, so a
// wavefront streams one 512-byte run of values and a 256-byte run of columns
// per entry.
#include <cmath>

#include <climits>
#include <vector>

#include "internal.h"

namespace rbffd {

namespace {

// One workgroup per 64-row slice: the slice's clouds are staged in LDS, each
// lane ranks its row's neighbours by index and writes the column indices in
// rank order; then the workgroup copies the weights in cloud order (coalesced
// reads) into the slot of each entry's rank.
__global__ __launch_bounds__(64) void sort_rows(const int32_t *__restrict__ nbr, const double *__restrict__ w,
                                                int64_t n, int q, int R, int32_t *__restrict__ col,
                                                double *__restrict__ val, int64_t vstride)
{
    extern __shared__ int32_t sh[];                  // [64][q+1] neighbour indices
    int16_t *rk = (int16_t *)(sh + 64 * (q + 1));    // [64][q] ranks
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int t = threadIdx.x;
    const int rows = (int)min((int64_t)64, n - i0);
    for (int e = t; e < rows * q; e += 64) {
        const int r = e / q, a = e % q;
        sh[r * (q + 1) + a] = nbr[(i0 + r) * q + a];
    }
    __syncthreads();
    const int64_t i = i0 + t;
    if (t >= rows) {
        for (int a = 0; a < q; ++a) {
            const int64_t slot = ell_at(i, a, q);
            col[slot] = 0;
            for (int r = 0; r < R; ++r) val[r * vstride + slot] = 0.0;
        }
    } else {
        const int32_t *mine = sh + t * (q + 1);
        for (int a = 0; a < q; ++a) {
            const int32_t c = mine[a];
            int rank = 0;
            for (int b = 0; b < q; ++b) rank += (mine[b] < c);
            rk[t * q + a] = (int16_t)rank;
            col[ell_at(i, rank, q)] = c;
        }
    }
    __syncthreads();
    for (int r = 0; r < R; ++r)
        for (int e = t; e < rows * q; e += 64) {
            const int row = e / q;
            val[r * vstride + ell_at(i0 + row, rk[e], q)] = w[(int64_t)r * n * q + i0 * q + e];
        }
}

// Pressure-correction matrix rows and its Jacobi diagonal.
template <int DIM>
__global__ void poisson_rows(const int32_t *__restrict__ col, const double *__restrict__ val, int64_t vstride,
                             const uint8_t *__restrict__ kind, const double *__restrict__ normal, int64_t pin,
                             int64_t n, int q, double *__restrict__ pval, double *__restrict__ pdinv)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= pad64(n)) return;
    if (i >= n) {
        for (int a = 0; a < q; ++a) pval[ell_at(i, a, q)] = 0.0;
        pdinv[i] = 0.0;
        return;
    }
    const int kd = kind[i];
    double nv[3] = {0, 0, 0};
    if (kd != RBFFD_INTERIOR)
        for (int d = 0; d < DIM; ++d) nv[d] = normal[i * DIM + d];
    double diag = 0.0;
    for (int a = 0; a < q; ++a) {
        const int64_t slot = ell_at(i, a, q);
        const int32_t c = col[slot];
        double v;
        if (i == pin || kd == RBFFD_PRESCRIBED_PRESSURE || kd == RBFFD_OUTLET) {
            v = (c == i) ? 1.0 : 0.0;
        } else if (kd == RBFFD_INTERIOR) {
            v = val[DIM * vstride + slot];
        } else {
            v = nv[0] * val[slot] + nv[1] * val[vstride + slot];
            if (DIM == 3) v = v + nv[2] * val[2 * vstride + slot];
        }
        pval[slot] = v;
        if (c == i) diag += v;
    }
    pdinv[i] = (diag != 0.0) ? 1.0 / diag : 1.0;
}

__global__ void boundary_flags(const uint8_t *__restrict__ kind, int64_t n, int32_t *__restrict__ flag,
                               int32_t *__restrict__ flag2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) {
        flag[i] = neumann_p(kind[i]);
        flag2[i] = kind[i] == RBFFD_PRESCRIBED_PRESSURE || kind[i] == RBFFD_OUTLET;
    }
}

__global__ void boundary_index(const uint8_t *__restrict__ kind, const int32_t *__restrict__ pos, int64_t n,
                               int32_t *__restrict__ bidx, int32_t *__restrict__ bpos)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (neumann_p(kind[i])) {
        bidx[pos[i]] = (int32_t)i;
        bpos[i] = pos[i];
    } else {
        bpos[i] = -1;
    }
}

// Block of the normal-derivative rows over velocity-Dirichlet and symmetry points: entries of
// the other columns are kept as explicit zeros on the row's own (block-local)
// column, so every row keeps q entries.
__global__ void boundary_block(const int32_t *__restrict__ col, const double *__restrict__ pval,
                               const uint8_t *__restrict__ kind, const int32_t *__restrict__ bidx,
                               const int32_t *__restrict__ bpos, int64_t nb, int q, int32_t *__restrict__ gcol,
                               double *__restrict__ gval, double *__restrict__ gdinv)
{
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= pad64(nb)) return;
    if (b >= nb) {
        for (int a = 0; a < q; ++a) {
            gcol[ell_at(b, a, q)] = 0;
            gval[ell_at(b, a, q)] = 0.0;
        }
        gdinv[b] = 0.0;
        return;
    }
    const int64_t i = bidx[b];
    double diag = 0.0;
    for (int a = 0; a < q; ++a) {
        const int64_t si = ell_at(i, a, q), sb = ell_at(b, a, q);
        const int32_t j = col[si];
        if (neumann_p(kind[j])) {
            gcol[sb] = bpos[j];
            gval[sb] = pval[si];
            if (bpos[j] == b) diag += pval[si];
        } else {
            gcol[sb] = (int32_t)b;
            gval[sb] = 0.0;
        }
    }
    gdinv[b] = (diag != 0.0) ? 1.0 / diag : 1.0;
}

__global__ void to_fp32(const double *__restrict__ x, float *__restrict__ y, int64_t m)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) y[i] = (float)x[i];
}

__global__ void ell_to_csr(const int32_t *__restrict__ col, const double *__restrict__ val, int64_t vstride,
                           const double *__restrict__ pval, int64_t n, int q, int R, int32_t *__restrict__ ocol,
                           double *__restrict__ oval)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n * q) return;
    const int64_t i = e / q;
    const int a = (int)(e % q);
    const int64_t slot = ell_at(i, a, q);
    ocol[e] = col[slot];
    for (int r = 0; r < R; ++r) oval[r * n * q + e] = val[r * vstride + slot];
    oval[(int64_t)R * n * q + e] = pval[slot];
}

// Per 64-row slice: the smallest column and, when the slice's columns span
// fewer than 65536 indices, 16-bit offsets from it (one wavefront per slice).
__global__ __launch_bounds__(64) void slice_offsets(const int32_t *__restrict__ col, int64_t n, int q,
                                                    int32_t *__restrict__ cbase, uint16_t *__restrict__ col16)
{
    const int64_t sl = blockIdx.x;
    const int64_t i = sl * 64 + threadIdx.x;
    int32_t mn = INT32_MAX, mx = INT32_MIN;
    if (i < n)
        for (int a = 0; a < q; ++a) {
            const int32_t c = col[ell_at(i, a, q)];
            mn = min(mn, c);
            mx = max(mx, c);
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = min(mn, __shfl_xor(mn, o, 64));
        mx = max(mx, __shfl_xor(mx, o, 64));
    }
    const bool narrow = mx >= mn && (int64_t)mx - (int64_t)mn < 65536;
    if (threadIdx.x == 0) cbase[sl] = narrow ? mn : -1;
    if (narrow && i < n)
        for (int a = 0; a < q; ++a) {
            const int64_t slot = ell_at(i, a, q);
            col16[slot] = (uint16_t)(col[slot] - mn);
        }
}

// Inverse of the 64x64 diagonal block of each 64-row slice of the
// pressure-correction matrix (a block-Jacobi preconditioner whose blocks are
// Morton-compact patches of 64 points): Gauss-Jordan elimination with partial
// pivoting (largest |a|, ties to the lowest row) in LDS, one wavefront per
// slice, one row per lane. Stored in FP16 divided by the inverse's largest
// |entry| (kept in FP32 per block), column-major per block: entry (row l,
// column j) at j*64 + l. Padding rows are identity rows. A block whose pivot
// falls to 1e-13 max|block| or below keeps the Jacobi diagonal.
__global__ __launch_bounds__(64) void block_inverse(const int32_t *__restrict__ col, const double *__restrict__ pval,
                                                    int64_t n, int q, __half *__restrict__ binv,
                                                    float *__restrict__ bscale)
{
    __shared__ double A[64][65];
    __shared__ double B[64][65];
    const int l = threadIdx.x;
    const int64_t sl = blockIdx.x;
    const int64_t i = sl * 64 + l;
    for (int j = 0; j < 64; ++j) {
        A[l][j] = 0.0;
        B[l][j] = (j == l) ? 1.0 : 0.0;
    }
    if (i < n) {
        for (int a = 0; a < q; ++a) {
            const int64_t slot = ell_at(i, a, q);
            const int32_t c = col[slot];
            if ((int64_t)(c >> 6) == sl) A[l][c & 63] += pval[slot];
        }
    } else {
        A[l][l] = 1.0;
    }
    const double diag = A[l][l];
    double amax = 0.0;
    for (int j = 0; j < 64; ++j) amax = fmax(amax, fabs(A[l][j]));
    amax = wave_max(amax);
    __syncthreads();
    bool singular = false;
    for (int k = 0; k < 64; ++k) {
        const double v = (l >= k) ? fabs(A[l][k]) : -1.0;
        const double mx = wave_max(v);
        if (!(mx > 1e-13 * amax)) {
            singular = true;
            break;
        }
        const uint64_t msk = __ballot(l >= k && v == mx);
        const int p = msk ? (__ffsll((unsigned long long)msk) - 1) : k;
        if (p != k) {
            double t = A[k][l];
            A[k][l] = A[p][l];
            A[p][l] = t;
            t = B[k][l];
            B[k][l] = B[p][l];
            B[p][l] = t;
        }
        __syncthreads();
        const double inv = 1.0 / A[k][k];
        __syncthreads();
        A[k][l] *= inv;
        B[k][l] *= inv;
        __syncthreads();
        if (l != k) {
            const double f = A[l][k];
            for (int j = 0; j < 64; ++j) {
                A[l][j] -= f * A[k][j];
                B[l][j] -= f * B[k][j];
            }
        }
        __syncthreads();
    }
    double emax = 0.0;
    for (int j = 0; j < 64; ++j) {
        const double e = singular ? ((j == l && diag != 0.0) ? 1.0 / diag : 0.0) : B[l][j];
        emax = fmax(emax, fabs(e));
    }
    emax = wave_max(emax);
    const double sc = (emax > 0.0 && emax < 3.0e38) ? emax : 1.0;
    __half *out = binv + sl * 4096;
    for (int j = 0; j < 64; ++j) {
        const double e = singular ? ((j == l && diag != 0.0) ? 1.0 / diag : 0.0) : B[l][j];
        out[j * 64 + l] = __float2half((float)(e / sc));
    }
    if (l == 0) bscale[sl] = (float)sc;
}

// FP32 copy of the block inverses (value x scale), for export
__global__ void expand_blocks(int64_t total, const __half *__restrict__ v, const float *__restrict__ sc,
                              float *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < total) out[e] = __half2float(v[e]) * sc[e >> 12];
}

template <typename T>
int alloc_ops(rbffd_ops *ops, T **p, size_t count)
{
    void *v = nullptr;
    const size_t bytes = sizeof(T) * count;
    RB_CHECK(dev_alloc(ops->ctx, &v, bytes));
    // the context charge moves to the operator object
    ops->bytes += bytes;
    *p = (T *)v;
    return RBFFD_OK;
}

}  // namespace

int assemble_ops(rbffd_ctx *ctx, const rbffd_cloud *cloud, int q, int k, int phs, const int32_t *nbr,
                 const double *w, int precision, rbffd_ops *ops, hipStream_t s)
{
    const int dim = cloud->dim;
    const int64_t n = cloud->n, npad = pad64(n);
    ops->ctx = ctx;
    ops->dim = dim;
    ops->q = q;
    ops->R = dim + 1;
    ops->k = k;
    ops->phs = phs;
    ops->n = n;
    ops->npad = npad;
    ops->pin = cloud->pin;
    ops->precision = precision;
    const int64_t nnz = npad * q;
    RB_CHECK(alloc_ops(ops, &ops->kind, (size_t)n));
    RB_CHECK(alloc_ops(ops, &ops->normal, (size_t)n * dim));
    RB_CHECK(alloc_ops(ops, &ops->col, (size_t)nnz));
    RB_CHECK(alloc_ops(ops, &ops->cbase, (size_t)(npad / 64)));
    RB_CHECK(alloc_ops(ops, &ops->col16, (size_t)nnz));
    RB_CHECK(alloc_ops(ops, &ops->val, (size_t)nnz * ops->R));
    RB_CHECK(alloc_ops(ops, &ops->pval, (size_t)nnz));
    RB_CHECK(alloc_ops(ops, &ops->pdinv, (size_t)npad));
    RB_CHECK(alloc_ops(ops, &ops->mval, (size_t)nnz));
    RB_CHECK(alloc_ops(ops, &ops->mdinv, (size_t)npad * kMaxRhs));
    RB_HIP(hipMemcpyAsync(ops->kind, cloud->kind, n, hipMemcpyDeviceToDevice, s));
    RB_HIP(hipMemcpyAsync(ops->normal, cloud->normal, sizeof(double) * n * dim, hipMemcpyDeviceToDevice, s));
    {
        // symmetry points: count them, and check that each normal has unit
        // length (their rows differ per velocity component)
        std::vector<uint8_t> hk((size_t)n);
        RB_HIP(hipMemcpyAsync(hk.data(), cloud->kind, (size_t)n, hipMemcpyDeviceToHost, s));
        RB_HIP(hipStreamSynchronize(s));
        int64_t nsym = 0;
        for (uint8_t v : hk) nsym += (v == RBFFD_SYMMETRY);
        ops->n_symmetry = nsym;
        if (nsym > 0) {
            std::vector<double> hn((size_t)n * dim);
            RB_HIP(hipMemcpyAsync(hn.data(), cloud->normal, sizeof(double) * n * dim, hipMemcpyDeviceToHost, s));
            RB_HIP(hipStreamSynchronize(s));
            for (int64_t i = 0; i < n; ++i) {
                if (hk[i] != RBFFD_SYMMETRY) continue;
                double len2 = 0.0;
                for (int d = 0; d < dim; ++d) len2 += hn[i * dim + d] * hn[i * dim + d];
                if (!(std::fabs(len2 - 1.0) <= 1e-12))
                    return fail(RBFFD_E_ARG, "symmetry point " + std::to_string(i) +
                                                 ": the normal is not a unit vector");
            }
        }
    }

    const unsigned nslices = (unsigned)(npad / 64);
    hipLaunchKernelGGL(sort_rows, dim3(nslices), dim3(64), sizeof(int32_t) * 64 * (q + 1) + sizeof(int16_t) * 64 * q,
                       s, nbr, w, n, q, ops->R, ops->col, ops->val, nnz);
    RB_HIP(hipGetLastError());
    hipLaunchKernelGGL(slice_offsets, dim3(nslices), dim3(64), 0, s, ops->col, n, q, ops->cbase, ops->col16);
    RB_HIP(hipGetLastError());
    const unsigned gb = (unsigned)((npad + kBlock - 1) / kBlock);
    if (dim == 2)
        hipLaunchKernelGGL(poisson_rows<2>, dim3(gb), dim3(kBlock), 0, s, ops->col, ops->val, nnz, ops->kind,
                           ops->normal, ops->pin, n, q, ops->pval, ops->pdinv);
    else
        hipLaunchKernelGGL(poisson_rows<3>, dim3(gb), dim3(kBlock), 0, s, ops->col, ops->val, nnz, ops->kind,
                           ops->normal, ops->pin, n, q, ops->pval, ops->pdinv);
    RB_HIP(hipGetLastError());

    // the block-Jacobi inverses of the pressure-correction matrix are built at
    // the first solve that asks for them (ensure_block_inverse)

    // boundary numbering
    int32_t *flag = nullptr, *pos = nullptr, *flag2 = nullptr, *pos2 = nullptr;
    const size_t fbytes = sizeof(int32_t) * (4 * n + 2);
    RB_CHECK(dev_alloc(ctx, (void **)&flag, fbytes));
    pos = flag + n;
    flag2 = pos + n + 1;
    pos2 = flag2 + n;
    const unsigned gn = (unsigned)((n + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(boundary_flags, dim3(gn), dim3(kBlock), 0, s, ops->kind, n, flag, flag2);
    int st = scan_exclusive(ctx, flag, pos, n, s);
    if (st == RBFFD_OK) st = scan_exclusive(ctx, flag2, pos2, n, s);
    int32_t nb32 = 0, np32 = 0;
    if (st == RBFFD_OK) {
        hipError_t e = hipMemcpyAsync(&nb32, pos + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&np32, pos2 + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "boundary count");
        ops->n_prescribed = np32;
    }
    if (st == RBFFD_OK) {
        ops->nb = nb32;
        ops->nbpad = pad64(nb32 > 0 ? nb32 : 1);
        st = alloc_ops(ops, &ops->bidx, (size_t)ops->nbpad);
        if (st == RBFFD_OK) st = alloc_ops(ops, &ops->bpos, (size_t)n);
        if (st == RBFFD_OK) st = alloc_ops(ops, &ops->gcol, (size_t)ops->nbpad * q);
        if (st == RBFFD_OK) st = alloc_ops(ops, &ops->gval, (size_t)ops->nbpad * q);
        if (st == RBFFD_OK) st = alloc_ops(ops, &ops->gdinv, (size_t)ops->nbpad);
    }
    if (st == RBFFD_OK) {
        hipLaunchKernelGGL(boundary_index, dim3(gn), dim3(kBlock), 0, s, ops->kind, pos, n, ops->bidx, ops->bpos);
        const unsigned gbb = (unsigned)((ops->nbpad + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(boundary_block, dim3(gbb), dim3(kBlock), 0, s, ops->col, ops->pval, ops->kind, ops->bidx,
                           ops->bpos, ops->nb, q, ops->gcol, ops->gval, ops->gdinv);
        if (hipGetLastError() != hipSuccess) st = fail(RBFFD_E_DEVICE, "boundary block launch failed");
    }
    (void)hipStreamSynchronize(s);
    dev_free(ctx, flag, fbytes);
    RB_CHECK(st);

    if (precision != RBFFD_FP64) {
        RB_CHECK(alloc_ops(ops, &ops->pval32, (size_t)nnz));
        RB_CHECK(alloc_ops(ops, &ops->pdinv32, (size_t)npad));
        RB_CHECK(alloc_ops(ops, &ops->mval32, (size_t)nnz));
        RB_CHECK(alloc_ops(ops, &ops->mdinv32, (size_t)npad * kMaxRhs));
        hipLaunchKernelGGL(to_fp32, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, ops->pval,
                           ops->pval32, nnz);
        hipLaunchKernelGGL(to_fp32, dim3(gb), dim3(kBlock), 0, s, ops->pdinv, ops->pdinv32, npad);
        RB_HIP(hipGetLastError());
    }
    RB_HIP(hipStreamSynchronize(s));
    return RBFFD_OK;
}

int launch_to_fp32(const double *x, float *y, int64_t m, hipStream_t s)
{
    hipLaunchKernelGGL(to_fp32, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, x, y, m);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

int ensure_block_inverse(const rbffd_ops *cops, hipStream_t s)
{
    if (cops->pbinv) return RBFFD_OK;
    // the inverses depend on the pressure-correction values only, which stay as
    // assembled: building them late gives what building them at assembly would
    rbffd_ops *ops = const_cast<rbffd_ops *>(cops);
    const unsigned nslices = (unsigned)(ops->npad / 64);
    __half *bi = nullptr;
    float *bs = nullptr;
    RB_CHECK(alloc_ops(ops, &bi, (size_t)ops->npad * 64));
    int st = alloc_ops(ops, &bs, (size_t)nslices);
    if (st != RBFFD_OK) {
        (void)hipFree(bi);
        ops->ctx->in_use -= sizeof(__half) * (size_t)ops->npad * 64;
        ops->bytes -= sizeof(__half) * (size_t)ops->npad * 64;
        return st;
    }
    hipLaunchKernelGGL(block_inverse, dim3(nslices), dim3(64), 0, s, ops->col, ops->pval, ops->n, ops->q, bi, bs);
    RB_HIP(hipGetLastError());
    ops->pbinv = bi;
    ops->pbscale = bs;
    return RBFFD_OK;
}

int expand_block_inverse(const rbffd_ops *ops, float *out, hipStream_t s)
{
    const int64_t total = ops->npad * 64;
    hipLaunchKernelGGL(expand_blocks, dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, total,
                       ops->pbinv, ops->pbscale, out);
    RB_HIP(hipGetLastError());
    return RBFFD_OK;
}

int export_csr(const rbffd_ops *ops, int32_t *col, double *val, hipStream_t s)
{
    const int64_t m = ops->n * ops->q;
    hipLaunchKernelGGL(ell_to_csr, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, ops->col,
                       ops->val, ops->npad * ops->q, ops->pval, ops->n, ops->q, ops->R, col, val);
    RB_HIP(hipGetLastError());
    RB_HIP(hipStreamSynchronize(s));
    return RBFFD_OK;
}

int apply_op(rbffd_ctx *ctx, const rbffd_ops *ops, int which, const double *x, double *y, hipStream_t s)
{
    (void)ctx;
    const double *v = (which <= ops->dim) ? ops->val + (int64_t)which * ops->npad * ops->q : ops->pval;
    return spmv(ops->n, ops->q, cols_of(ops), v, x, y, s);
}

}  // namespace rbffd
