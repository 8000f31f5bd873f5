// Internal declarations of the gfx950 PHS-RBF library: context and operator
// objects, device helpers, kernel launch wrappers. Not part of the C ABI.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <set>
#include <string>

#include "../../include/rbffd.h"

namespace rbffd {

constexpr int kWave = 64;
constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kMaxBlocks = 2048;     // grid cap of reducing kernels (partials <= this)
constexpr int kSlice = 64;           // rows per slice of the sliced-ELL layout
constexpr int kMaxQ = 128;           // largest cloud
constexpr int kMaxRhs = 3;           // velocity components solved together

// ---------------------------------------------------------------------------
// error handling
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define RB_HIP(call)                                        \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(e_, #call);   \
    } while (0)

#define RB_CHECK(call)                       \
    do {                                     \
        int s_ = (call);                     \
        if (s_ != RBFFD_OK) return s_;       \
    } while (0)

// ---------------------------------------------------------------------------
// sliced ELL: row i, entry a lives at ((i / 64) * q + a) * 64 + (i % 64), so a
// wavefront of 64 consecutive rows reads entry a of all its rows as one
// contiguous 64-element run. Rows are padded to a multiple of 64; padding rows
// hold column 0 and value 0.
// ---------------------------------------------------------------------------
__host__ __device__ inline int64_t ell_at(int64_t i, int a, int q)
{
    return ((i >> 6) * (int64_t)q + a) * 64 + (i & 63);
}
__host__ __device__ inline int64_t pad64(int64_t n) { return (n + 63) / 64 * 64; }

// ---------------------------------------------------------------------------
// context: device, HBM budget, workspace buffers grown on demand
// ---------------------------------------------------------------------------
struct Buffer {
    void *ptr = nullptr;
    size_t bytes = 0;
};

enum WorkSlot {
    WS_KRYLOV = 0,   // FP64 Krylov vectors
    WS_KRYLOV32,     // FP32 Krylov vectors (inner solves of the refinement)
    WS_PARTIAL,      // FP64 solve: reduction partials + state records
    WS_PARTIAL32,    // FP32 solve: reduction partials + state records
    WS_REFINE,       // refinement residual / correction
    WS_STEP,         // time-step fields
    WS_STEP2,        // boundary-pressure solve and step reductions
    WS_MISC,
    WS_RESID,        // true-residual partials
    WS_BATCH,        // batched solves: descriptors, block map, partials, states, vectors
    WS_BATCH_HOST,   // batched solves: pinned host staging
    WS_HOST_PINNED,  // pinned host staging for small read-backs
    WS_BUILD,        // batched stencil builds: cloud descriptors, singular-point slots
    WS_BUILD_HOST,   // batched stencil builds: pinned host staging
    WS_COUNT
};

// fixed regions of the pinned host staging buffer
constexpr size_t kHostKrylov = 0;      // Krylov state records
constexpr size_t kHostRefine = 1024;   // refinement residual norms
constexpr size_t kHostStep = 2048;     // time-step scalars
constexpr size_t kHostMisc = 3072;
constexpr size_t kHostBytes = 4096;

}  // namespace rbffd

struct rbffd_server;
struct rbffd_ctx {
    int device = 0;
    size_t budget = 0;        // 0 = unlimited
    size_t in_use = 0;
    rbffd::Buffer ws[rbffd::WS_COUNT];
    // objects created under this context: destroying the context releases
    // their device memory and leaves them orphaned (freeing them later is safe)
    std::set<rbffd_ops *> ops;
    std::set<rbffd_server *> servers;
    // HIP graphs of BiCGSTAB iteration chunks (krylov.hip), and whether the
    // solves replay them
    void *graphs = nullptr;
    bool use_graphs = false;
    // solver path per system size (n, q) for FP64 Jacobi BiCGSTAB: 0 = the
    // multi-kernel iteration, 256 / 512 / 1024 = the one-workgroup solver with
    // that many threads; sizes not listed take the multi-kernel iteration
    std::map<std::pair<int64_t, int>, int> solver_choice;
};

namespace rbffd {
// release the context's captured graphs (and their capture stream)
void graph_cache_destroy(rbffd_ctx *ctx);
int dev_alloc(rbffd_ctx *ctx, void **p, size_t bytes);
void dev_free(rbffd_ctx *ctx, void *p, size_t bytes);
// workspace slot of at least `bytes` (contents are not preserved on growth)
int workspace(rbffd_ctx *ctx, int slot, size_t bytes, void **p);
// region [off, off + bytes) of the pinned host staging buffer
int host_scratch(rbffd_ctx *ctx, size_t off, size_t bytes, void **p);
}  // namespace rbffd

// Operators of one cloud, resident on the device.
struct rbffd_ops {
    rbffd_ctx *ctx = nullptr;
    int dim = 2, q = 0, R = 3, k = 0, phs = 3;
    int64_t n = 0, npad = 0, pin = 0;
    int64_t nb = 0, nbpad = 0;          // velocity-Dirichlet boundary points (normal momentum block)
    int64_t n_prescribed = 0;           // prescribed-pressure and outlet points
    int64_t n_symmetry = 0;             // symmetry-plane points (momentum solved per component)
    int precision = RBFFD_FP64;
    size_t bytes = 0;                   // device bytes charged to ctx
    // cloud copies
    uint8_t *kind = nullptr;            // [n]
    double *normal = nullptr;           // [n][dim]
    // sliced-ELL operators
    int32_t *col = nullptr;             // [npad*q]
    int32_t *cbase = nullptr;           // [npad/64] smallest column of each 64-row slice, -1 = wide slice
    uint16_t *col16 = nullptr;          // [npad*q]  col - cbase on slices whose columns span < 65536
    double *val = nullptr;              // [R][npad*q]  d/dx, d/dy, (d/dz), Laplacian
    double *pval = nullptr;             // [npad*q]     pressure-correction matrix
    double *pdinv = nullptr;            // [npad]       1 / diag(P)
    __half *pbinv = nullptr;            // [npad/64][64][64] inverse of each 64-row diagonal block of P
                                        //              (FP16 divided by pbscale, column-major per block)
    float *pbscale = nullptr;           // [npad/64]    largest |entry| of each block's inverse
    float *pval32 = nullptr;            // [npad*q]     FP32 copy (RBFFD_FP32_IR)
    float *pdinv32 = nullptr;           // [npad]
    double *mval = nullptr;             // [npad*q]     momentum matrix (rebuilt per outer iteration)
    double *mdinv = nullptr;            // [npad]
    float *mval32 = nullptr;            // [npad*q]
    float *mdinv32 = nullptr;           // [npad]
    // block of the normal-derivative rows over velocity-Dirichlet points
    int32_t *bidx = nullptr;            // [nb]   global row of block row b
    int32_t *bpos = nullptr;            // [n]    block row of global row i, or -1
    int32_t *gcol = nullptr;            // [nbpad*q] sliced-ELL, boundary-local columns
    double *gval = nullptr;             // [nbpad*q]
    double *gdinv = nullptr;            // [nbpad]
};

namespace rbffd {

// Column indices of a sliced-ELL matrix. Where a 64-row slice's columns span
// fewer than 65536 indices (nearly all slices of a Morton-ordered cloud), the
// kernels read 16-bit offsets from the slice's smallest column instead of
// 32-bit indices. cbase == nullptr: 32-bit indices only.
struct ColIdx {
    const int32_t *col;
    const int32_t *cbase;
    const uint16_t *col16;
};

inline ColIdx cols_of(const rbffd_ops *ops) { return ColIdx{ops->col, ops->cbase, ops->col16}; }
inline ColIdx cols_plain(const int32_t *col) { return ColIdx{col, nullptr, nullptr}; }

// Block-Jacobi preconditioner: the inverse of each 64-row slice's diagonal
// block in FP16, divided by the block's largest |entry| (scale), so every
// stored value lies in [-1, 1]. val == nullptr: no block preconditioner.
struct BlockInv {
    const __half *val;
    const float *scale;
};

inline BlockInv binv_of(const rbffd_ops *ops) { return BlockInv{ops->pbinv, ops->pbscale}; }
// build the operators' block inverses if no solve has asked for them yet
int ensure_block_inverse(const rbffd_ops *ops, hipStream_t s);

// Points whose pressure correction has a homogeneous Neumann row and whose
// pressure comes from the normal momentum equation (Sec. 3.1).
__host__ __device__ inline bool neumann_p(int kd) { return kd == RBFFD_DIRICHLET || kd == RBFFD_SYMMETRY; }
constexpr BlockInv kNoBlockInv{nullptr, nullptr};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Fixed-order block sum (blockDim.x == kBlock): identical result in every block
// for identical inputs. `lds` holds kBlock/64 doubles.
__device__ inline double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) t += lds[i];
    return t;
}

// Sum of np partials in a fixed order, computed identically by every block.
__device__ inline double sum_partials(const double *part, int np, double *lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < np; i += kBlock) v += part[i];
    return block_sum(v, lds);
}

// XCD-aware block order: consecutive logical blocks land on the same XCD (the
// hardware deals blocks round-robin over 8 XCDs), so neighbouring rows share an L2.
__device__ inline int xcd_block(int nblocks)
{
    const int b = blockIdx.x;
    const int per = nblocks / 8;
    if (per == 0 || (nblocks & 7)) return b;
    return (b & 7) * per + (b >> 3);
}

// ---------------------------------------------------------------------------
// launch wrappers (defined in the .hip files)
// ---------------------------------------------------------------------------
// Lowest point whose cloud shows a coincident point (INT64_MAX when none), in
// device memory at *first.
int launch_dup_check(int dim, int64_t n, const double *xyz, int q, const int32_t *nbr, int64_t *first,
                     hipStream_t s);
int launch_knn(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int q, int32_t *nbr,
               hipStream_t s);
int launch_weights(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int q, const int32_t *nbr,
                   int k, int phs, double *w, int64_t *bad_dev, hipStream_t s);
// One cloud of a batched weight build (systems of at most 64 unknowns): its
// points take the blocks [first_block, first_block + n) of the launch.
struct WeightSys {
    const double *xyz;
    const int32_t *nbr;
    double *w;
    int64_t n, first_block;
    int q, m, phs, width;
};
// smallest register width of the weight kernels >= ns, or 0 above 64 unknowns
int weight_width(int ns);
// one launch over the points of `count` clouds of dimension dim and register
// width `width` (all of them); bad_dev[j] is cloud j's lowest singular point
// (INT64_MAX if none; set by the caller)
int launch_weights_batched(int dim, int width, int count, const WeightSys *sys_dev, int64_t total_blocks,
                           int64_t *bad_dev, hipStream_t s);
// The q nearest cloud points of nq arbitrary query points.
int launch_knn_points(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int64_t nq, const double *qxyz, int q,
                      int32_t *nbr, hipStream_t s);
// Interpolation weights at nq query points (clouds in nbr) and, when nfield > 0,
// the interpolated fields: out[f][j] = sum_a w[j][a] fields[f][nbr[j][a]].
int launch_interp(rbffd_ctx *ctx, int dim, int64_t n, const double *xyz, int64_t nq, const double *qxyz, int q,
                  const int32_t *nbr, int k, int phs, double *w, int64_t *bad_dev, int nfield, const double *fields,
                  double *out, hipStream_t s);
// out[f][j] = sum_a w[j][a] fields[f][nbr[j][a]] for nq points (fields [nfield][n]).
int launch_interp_apply(int64_t nq, int q, const int32_t *nbr, const double *w, int nfield, int64_t n,
                        const double *fields, double *out, hipStream_t s);
int assemble_ops(rbffd_ctx *ctx, const rbffd_cloud *cloud, int q, int k, int phs,
                 const int32_t *nbr, const double *w, int precision, rbffd_ops *ops, hipStream_t s);
int export_csr(const rbffd_ops *ops, int32_t *col, double *val, hipStream_t s);
// FP32 copy of the block-Jacobi inverses (FP16 value x block scale), out [npad*64]
int expand_block_inverse(const rbffd_ops *ops, float *out, hipStream_t s);
int apply_op(rbffd_ctx *ctx, const rbffd_ops *ops, int which, const double *x, double *y,
             hipStream_t s);

int launch_to_fp32(const double *x, float *y, int64_t m, hipStream_t s);

// exclusive scan of int32 counts (n + 1 outputs: out[n] = total)
int scan_exclusive(rbffd_ctx *ctx, const int32_t *in, int32_t *out, int64_t n, hipStream_t s);

// Krylov: BiCGSTAB on a sliced-ELL matrix with nrhs right-hand sides
struct KrylovResult {
    int iters[kMaxRhs] = {0, 0, 0};
    int status[kMaxRhs] = {0, 0, 0};
    double relres[kMaxRhs] = {0, 0, 0};
    bool fp64_fallback = false;   // FP32 sweeps stalled; finished in FP64
};
// FP64 BiCGSTAB right-preconditioned by the inverses of the 64x64 diagonal
// blocks of the 64-row slices (one right-hand side).
int bicgstab_block(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, BlockInv binv,
                   const double *b, double *x, double tol, int max_iter, KrylovResult *res, hipStream_t s);
// time `iterations` FP64 Jacobi BiCGSTAB iterations of the system (n, q, col,
// val, dinv) on each solver path and record the fastest for (n, q)
int autotune_solver(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, const double *dinv,
                    int iterations, int *choice, double *us_per_iter, hipStream_t s);
int bicgstab(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val,
             const double *dinv, int nrhs, const double *b, double *x, double tol, int max_iter,
             KrylovResult *res, hipStream_t s);
// FP32 matrix values with FP64 row accumulation and FP64 reliable updates;
// precision RBFFD_FP32_IR keeps the Krylov vectors in FP32, RBFFD_FP32_MATRIX in FP64.
// binv: block-Jacobi inverses (one right-hand side), or binv.val nullptr for Jacobi.
int bicgstab_mixed(rbffd_ctx *ctx, int precision, int64_t n, int q, ColIdx col, const double *val,
                   const float *val32, const float *dinv32, const double *dinv64, BlockInv binv, int nrhs,
                   const double *b, double *x, double tol, int max_iter, KrylovResult *res, int *refinements,
                   hipStream_t s);
// One system of a batched solve (host description).
struct BatchSystem {
    int64_t n;
    int q;
    ColIdx col;
    const double *val, *dinv, *b;
    double *x;
    BlockInv binv;        // block-Jacobi inverses (binv.val nullptr: Jacobi)
    const float *val32;   // FP32 matrix for the Krylov SpMVs (FP64 residuals), or nullptr
};
// FP64 BiCGSTAB on many independent systems at once: every kernel stage is one
// launch over all systems, each system owns a fixed range of blocks and its own
// reductions, so its result does not depend on the other systems in the batch.
int bicgstab_batched(rbffd_ctx *ctx, int count, const BatchSystem *sys, double tol, int max_iter, int *iters,
                     int *status, double *relres, hipStream_t s);
// Continuous batching of FP64 pressure-correction solves: systems join and
// leave a running batch between chunks of iterations.
struct Server;
int server_create(rbffd_ctx *ctx, Server **out);
void server_destroy(Server *sv);
int server_submit(Server *sv, const BatchSystem &sys, double tol, int max_iter, int64_t *ticket);
int server_run(Server *sv, int iterations, int *n_active, hipStream_t s);
int server_poll(Server *sv, int max, int64_t *tickets, int *iters, int *status, double *relres, int *count);
int spmv(int64_t n, int q, ColIdx col, const double *val, const double *x, double *y,
         hipStream_t s);
// Mean kernel durations (us) of one FP64 Jacobi BiCGSTAB iteration on one system:
// us[0] KV, us[1] KS, us[2] KT, us[3] KX, us[4] the whole iteration.
int krylov_kernel_times(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val, const double *dinv,
                        const double *b, double *x, int reps, double *us, hipStream_t s);
// Allocation-free solve: takes the address of the fixed scratch array on the
// current device (once per device), and runs the FP64 Jacobi BiCGSTAB of
// poisson_solve with its workspace there.
int noalloc_init(int device);
int poisson_solve_noalloc_impl(int device, int64_t n, int q, ColIdx col, const double *val, const double *dinv,
                               const double *b, double *x, double tol, int max_iter, KrylovResult *res,
                               double *relres, hipStream_t s);
int residual_norms(rbffd_ctx *ctx, int64_t n, int q, ColIdx col, const double *val,
                   int nrhs, const double *b, const double *x, double *relres_out, hipStream_t s);

int run_step_batched(rbffd_ctx *ctx, int count, const rbffd_ops *const *ops, double *const *u,
                     double *const *u_prev, double *const *p, const double *const *u_bc, const double *const *p_bc,
                     const rbffd_step_opts *o, rbffd_step_stats *st, hipStream_t s);
int run_step(rbffd_ctx *ctx, const rbffd_ops *ops, double *u, double *u_prev, double *p,
             const double *u_bc, const double *p_bc, const rbffd_step_opts *o, rbffd_step_stats *st,
             hipStream_t s);
int convdiff_lambda(rbffd_ctx *ctx, const rbffd_ops *ops, const double *u0, double rho, double mu,
                    int iters, double *lambda, hipStream_t s);

}  // namespace rbffd
