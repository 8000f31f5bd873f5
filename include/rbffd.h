/*
 * rbffd.h - C ABI of the MI355X (gfx950) implementation of the data-parallel
 * hot path of Shahane & Vanka, "A Semi-Implicit Meshless Method for
 * Incompressible Flows in Complex Geometries" (arXiv 2106.07616):
 *
 *   rbffd_build_stencils  k-nearest-neighbour clouds and PHS-RBF + polynomial
 *                         differentiation weights (Sec. 2)
 *   rbffd_assemble        sparse operators d/dx, d/dy, (d/dz), Laplacian and the
 *                         pressure-correction matrix (Sec. 2 closing remark,
 *                         Eq. pressure poisson, Sec. 3.1)
 *   simple_step           one BDF2 time step with outer momentum /
 *                         pressure-correction iterations (Sec. 3, Sec. 3.2)
 *   poisson_solve         preconditioned BiCGSTAB on the pressure-correction
 *                         matrix (Sec. 3)
 *
 * Conventions shared by every entry point:
 *   - Return value: RBFFD_OK (0) or a negative RBFFD_E_* code; nothing aborts
 *     and no C++ exception crosses the ABI. rbffd_last_error() gives a
 *     thread-local message for the last failure on the calling thread.
 *   - Array arguments are DEVICE pointers (hipMalloc / torch tensors on the
 *     GPU) owned by the caller unless stated otherwise; sizes are elements.
 *   - Arguments are validated on the host before anything is launched; an
 *     invalid argument returns RBFFD_E_ARG and launches nothing.
 *   - All work is enqueued on the caller's HIP stream (void* hip_stream, NULL =
 *     the default stream). rbffd_build_stencils and rbffd_assemble return once
 *     their small host-visible results are known (they synchronise the stream
 *     once); simple_step and poisson_solve synchronise to take convergence
 *     decisions and return with all work complete.
 *   - One context per host thread; calls on one context must not overlap.
 *   - Field layout: a velocity field is [dim][n] (component-major), a scalar
 *     field is [n]; coordinates and normals are [n][dim] (point-major).
 */
#ifndef RBFFD_H
#define RBFFD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define RBFFD_OK 0
#define RBFFD_E_ARG (-1)        /* invalid argument (checked before any launch)  */
#define RBFFD_E_OOM (-2)        /* the context's HBM budget or the device is full */
#define RBFFD_E_SINGULAR (-3)   /* a collocation system had a pivot <= 1e-13 max|A| */
#define RBFFD_E_NOCONV (-4)     /* a Krylov solve or the outer iteration hit its limit */
#define RBFFD_E_BREAKDOWN (-5)  /* BiCGSTAB breakdown (t.t == 0) */
#define RBFFD_E_DEVICE (-6)     /* a HIP runtime call failed */

/* ---- precision of the Krylov sweeps ------------------------------------ */
#define RBFFD_FP64 0            /* everything in FP64                                  */
#define RBFFD_FP32_IR 1         /* FP32 matrix values and Krylov vectors, FP64 row and dot
                                   accumulation, inside FP64 iterative refinement: each
                                   time the recursive residual has fallen 10x, the FP64
                                   residual b - A x replaces it and BiCGSTAB restarts from
                                   it, until the FP64 residual meets the tolerance; FP64
                                   sweeps finish a solve that stalls in FP32             */
#define RBFFD_FP32_MATRIX 2     /* as RBFFD_FP32_IR with FP32 matrix values but FP64 Krylov
                                   vectors, refined each time the recursive residual has
                                   fallen 100x: 1/3 fewer matrix bytes at q >= 20 with
                                   nearly the FP64 iteration count                      */

/* ---- preconditioner of the pressure-correction solve ------------------- */
#define RBFFD_PREC_JACOBI 0     /* diagonal (Jacobi), applied on the right               */
#define RBFFD_PREC_BLOCK64 1    /* inverses of the 64 x 64 diagonal blocks of the 64-row
                                   slices (Morton-compact patches of 64 points), stored
                                   in FP16 scaled per block and applied on the right
                                   with FP64 accumulation; any precision in poisson_solve and
                                   simple_step, RBFFD_FP64 or RBFFD_FP32_MATRIX in
                                   batched and served solves                            */

/* ---- point kinds ------------------------------------------------------- */
#define RBFFD_INTERIOR 0
#define RBFFD_DIRICHLET 1       /* prescribed velocity (wall, inlet); homogeneous Neumann
                                   pressure correction; boundary pressure from the
                                   normal momentum equation (Sec. 3.1)                  */
#define RBFFD_PRESCRIBED_PRESSURE 2 /* prescribed velocity and prescribed pressure; the
                                   pressure correction is zero there (Sec. 3.1)          */
#define RBFFD_OUTLET 3          /* outlet with prescribed pressure (p' = 0, pressure from
                                   p_bc) and zero normal derivative of every velocity
                                   component (Sec. 3.1); needs the outward normal        */
#define RBFFD_SYMMETRY 4        /* symmetry plane (Sec. 3.1), at any angle: zero normal
                                   velocity, zero normal derivative of the tangential
                                   velocity; homogeneous Neumann p' and the pressure
                                   from the normal momentum equation, as at
                                   velocity-Dirichlet points. The normal must have unit
                                   length; off the axes the components' conditions are
                                   coupled through the outer iteration               */

/* Thread-local description of the last error on this thread ("" if none). */
const char *rbffd_last_error(void);

/* ---- context ------------------------------------------------------------ */
typedef struct rbffd_ctx rbffd_ctx;

/* Create a context on HIP device `hip_device`. Device memory the library
 * allocates (operators, Krylov workspace) is charged to `hbm_budget_bytes`
 * (0 = no limit); an allocation beyond the budget returns RBFFD_E_OOM. */
int rbffd_ctx_create(rbffd_ctx **ctx, int hip_device, size_t hbm_budget_bytes);
/* Free the context and its workspace (operators are freed by rbffd_ops_free). */
int rbffd_ctx_destroy(rbffd_ctx *ctx);
/* Device bytes currently charged to the context (workspace + live operators). */
size_t rbffd_ctx_bytes_in_use(const rbffd_ctx *ctx);
/* (Sec. 3: the BiCGSTAB solves of each outer iteration) Whether the context's
 * FP64 Jacobi BiCGSTAB solves (the momentum and pressure-correction solves of
 * simple_step, and poisson_solve) launch their iteration chunks as HIP graphs:
 * enable = 1 captures each distinct chunk once, on a stream the context owns,
 * and replays it on the caller's stream; 0 (the default) launches the kernels
 * one by one. The results are bitwise the same either way. A capture is
 * invalidated when another thread synchronises the whole device meanwhile:
 * the solve then launches that chunk directly and the context returns to
 * direct launches (so enable graphs where no other thread does). A captured graph
 * holds the addresses of the vectors it was captured with, so it is replayed
 * only for the same operators, solution vector and workspace; at most 32 are
 * kept per context (least recently used evicted), and rbffd_ctx_destroy
 * releases them. RBFFD_E_ARG for a NULL ctx or enable outside {0, 1}. */
int rbffd_ctx_set_graphs(rbffd_ctx *ctx, int enable);
/* (Sec. 3: the BiCGSTAB solves) Which kernels run the FP64 Jacobi BiCGSTAB
 * solves of systems of n rows and stencil width q under this context
 * (simple_step's momentum, boundary-pressure and pressure-correction solves,
 * poisson_solve):
 *   choice 0            the multi-kernel iteration (four kernels per iteration,
 *                       the grid spread over the whole GPU);
 *   256, 512, 1024      one workgroup of that many threads runs the entire
 *                       solve in one kernel;
 *   -1                  forget the choice: the multi-kernel iteration, the
 *                       default for every size.
 * The paths iterate identically but sum their dot products in different orders,
 * so results differ at rounding level between choices (each is deterministic).
 * Batched solves (poisson_solve_batched) and poisson_solve_noalloc always take
 * the multi-kernel iteration.
 * RBFFD_E_ARG for a NULL ctx, n or q < 1, or another choice. */
int rbffd_ctx_set_solver_choice(rbffd_ctx *ctx, int64_t n, int q, int choice);

/* ---- inputs ------------------------------------------------------------ */
typedef struct {
    int dim;                /* 2 or 3                                                */
    int64_t n;              /* number of points, 1 <= n < 2^31                       */
    const double *xyz;      /* device [n][dim]; no two points may coincide           */
    const uint8_t *kind;    /* device [n]: RBFFD_INTERIOR / _DIRICHLET / _PRESCRIBED_PRESSURE / _OUTLET /
                               _SYMMETRY */
    const double *normal;   /* device [n][dim]: unit outward normal (boundary points) */
    int64_t pin;            /* interior point whose pressure correction is 0, or -1
                               (none; needed only when no prescribed-pressure point
                               fixes the pressure level)                             */
    double period[3];       /* > 0: the cloud wraps along that axis with this period
                               (Sec. 3.1, periodic boundaries): point j also stands
                               at x_j +- period e_d, and clouds near one face take
                               points from the other. The points' extent along the
                               axis must be below the period. 0: not periodic        */
} rbffd_cloud;

typedef struct {
    int phs_power;          /* polyharmonic spline exponent: 3 (r^3) or 5 (r^5)     */
    int poly_degree;        /* k, degree of the appended polynomials, 0..6           */
    int q;                  /* cloud size including the point itself; 0 = 2m          */
} rbffd_stencil_opts;

/* Cloud size q (resolving q = 0), monomial count m = binomial(k+dim, dim) and
 * operator count R = dim + 1 for the given options. RBFFD_E_ARG if q <= m. */
int rbffd_stencil_sizes(int dim, const rbffd_stencil_opts *opts, int *q, int *m, int *R);

/* (Sec. 2) For every point i: its cloud, the q nearest points including i in
 * the total order (squared distance, index), with squared distance evaluated
 * as ((dx*dx + dy*dy) + dz*dz), dx = x_j - x_i, without fused multiply-add;
 * then the centre row of B1 = [L Phi  L P] A^{-1} for L = d/dx, d/dy, (d/dz),
 * Laplacian, with A = [Phi P; P^T 0] built in coordinates centred at x_i and
 * scaled by the distance to the q-th neighbour, solved by LU with partial
 * pivoting.
 *   nbr: device [n][q] int32 out, neighbour indices in cloud order (nbr[i][0]=i)
 *   w:   device [R][n][q] double out, weights in cloud order
 *   bad_point: host out (may be NULL): lowest index of a singular stencil or -1
 * Returns RBFFD_E_SINGULAR if any stencil was singular (w is then undefined for
 * that point). Coincident points are an input error: RBFFD_E_ARG, the message
 * naming the lowest point whose cloud holds a point at distance 0 (checked on
 * the coordinates as given; periodic clouds are not checked for points that
 * coincide modulo the period). */
int rbffd_build_stencils(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts,
                         int32_t *nbr, double *w, int64_t *bad_point, void *hip_stream);

/* (Sec. 2, over many independent clouds: the batched configuration) The
 * clouds and weights of `count` clouds, each exactly as rbffd_build_stencils
 * computes them (bitwise the same). The neighbour search runs cloud by cloud;
 * the weights of all clouds with at most 64 unknowns (q + m) are built in one
 * launch per (dimension, register width) present, each 64-lane block taking
 * one point of one cloud; clouds of 65-128 unknowns take the Gauss-Jordan
 * kernels one by one. Clouds may differ in size, degree, cloud size and PHS
 * power.
 *   clouds, opts: HOST arrays of `count` descriptions and options
 *   nbr, w:       HOST arrays of `count` device pointers: nbr[j] [n_j][q_j]
 *                 int32, w[j] [R_j][n_j][q_j] double (outputs)
 *   bad_points:   optional HOST [count] out: cloud j's lowest singular point,
 *                 or -1
 * Periodic clouds are refused (RBFFD_E_ARG; build them one at a time), as is
 * any invalid cloud or size, before any launch (the message names the cloud).
 * RBFFD_E_SINGULAR if any cloud had a singular system. Synchronises the
 * stream. */
int rbffd_build_stencils_batched(rbffd_ctx *ctx, int count, const rbffd_cloud *clouds,
                                 const rbffd_stencil_opts *opts, int32_t *const *nbr, double *const *w,
                                 int64_t *bad_points, void *hip_stream);

/* ---- operators ---------------------------------------------------------- */
typedef struct rbffd_ops rbffd_ops;

/* (Sec. 2 closing remark, Eq. pressure poisson, Sec. 3.1) Sort each cloud by
 * column into a sparse matrix with exactly q entries per row, carry the R
 * weight sets along, and build the pressure-correction matrix: the Laplacian
 * row at interior points, N . grad at velocity-Dirichlet and symmetry points
 * (homogeneous Neumann), the identity row (p' = 0) at prescribed-pressure and
 * outlet points and at the pin. RBFFD_E_ARG if a symmetry point's normal is
 * not of unit length (within 1e-12). `precision` selects
 * whether FP32 copies for the mixed-precision modes are made (any value other
 * than RBFFD_FP64). The cloud arrays are copied;
 * nbr and w may be freed afterwards. *out is library-owned: free it with
 * rbffd_ops_free. */
int rbffd_assemble(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts,
                   const int32_t *nbr, const double *w, int precision, rbffd_ops **out,
                   void *hip_stream);
int rbffd_ops_free(rbffd_ops *ops);
/* n, q, dim and the number of boundary points of assembled operators. */
int rbffd_ops_info(const rbffd_ops *ops, int64_t *n, int *q, int *dim, int64_t *n_boundary);
/* Write the operators as row-major CSR with q entries per row (row_ptr[i] = i*q,
 * columns ascending): col device [n][q] int32, val device [R+1][n][q] double
 * holding d/dx, d/dy, (d/dz), Laplacian and the pressure-correction matrix. */
int rbffd_ops_export_csr(const rbffd_ops *ops, int32_t *col, double *val, void *hip_stream);
/* The block-Jacobi preconditioner of the pressure-correction matrix: for each
 * 64-row slice s, the inverse of its 64 x 64 diagonal block as the solver
 * holds it (FP16 values times an FP32 per-block scale), expanded to FP32,
 * column-major (entry (row l, column j) at out[s*4096 + j*64 + l]; padding rows
 * of the last slice are identity rows). out: device [ceil(n/64) * 4096]. */
int rbffd_ops_export_block_inverse(const rbffd_ops *ops, float *out, void *hip_stream);
/* y = A x for operator `which` (0..dim-1: d/dx_e, dim: Laplacian, dim+1: the
 * pressure-correction matrix); x, y device [n]. Enqueued on the stream and not
 * synchronised (one kernel launch). */
int rbffd_apply(rbffd_ctx *ctx, const rbffd_ops *ops, int which, const double *x, double *y,
                void *hip_stream);

/* (Sec. 2, Eq. RBF_interp evaluated off the nodes; the centre-line profiles
 * and sampled fields of Sec. 4) Interpolate fields given on the cloud's points
 * at nq arbitrary points: each query point takes its q nearest cloud points in
 * the order (squared distance, index), and the local PHS + polynomial
 * interpolant of degree opts->poly_degree on them, centred at the query point
 * and scaled by the distance to its farthest cloud point, is evaluated there.
 *   qxyz:   device [nq][dim] query coordinates (any point; clouds of points
 *           outside the bounding box are still exact but slower to find)
 *   fields: device [nfield][n] values on the cloud (may be NULL if nfield = 0)
 *   out:    device [nfield][nq] interpolated values (may be NULL if nfield = 0)
 *   nbr_out, w_out: optional device [nq][q] int32 clouds and [nq][q] double
 *           weights (out[f][j] = sum_a w[j][a] fields[f][nbr[j][a]]); NULL to
 *           keep them internal
 * On a periodic cloud (Sec. 3.1), a query coordinate outside [lo, lo + L)
 * along a periodic axis (lo the cloud's smallest coordinate there) is first
 * wrapped to lo + r, r = fmod(x - lo, L) taken into [0, L); the query takes
 * its q nearest among the points and their periodic images, the weights use
 * the images' coordinates, and nbr_out names the points the images stand for
 * (RBFFD_E_ARG if a cloud would hold two images of one point).
 * Systems of up to 128 unknowns (q + m). Synchronises the stream. Returns
 * RBFFD_E_SINGULAR (lowest query index in *bad_query) for a singular local
 * system, RBFFD_E_ARG for bad sizes; nq = 0 is a no-op. */
int rbffd_interpolate(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts, int64_t nq,
                      const double *qxyz, int nfield, const double *fields, double *out, int32_t *nbr_out,
                      double *w_out, int64_t *bad_query, void *hip_stream);

/* (Sec. 4, Eqs. cylinder forces, cylinder stress and cylinder lift drag) Force
 * per unit length on a circular cylinder in a 2D flow, from its surface
 * stresses:
 *   1. the strain rates du/dx, du/dy, dv/dx, dv/dy at the nodes, by the
 *      operators' d/dx and d/dy;
 *   2. the pressure and the strain rates interpolated, as rbffd_interpolate
 *      does with the operators' degree, cloud size and PHS power, to nsurf
 *      uniform points x_j = centre + (D/2)(cos t_j, sin t_j),
 *      t_j = 2 pi j / nsurf (cos and sin of the host C library);
 *   3. sigma = -p I + mu (grad u + grad u^T) there, and the traction
 *      sigma . (cos t_j, sin t_j), the normal pointing from the cylinder into
 *      the fluid;
 *   4. F = (D/2) * integral over t in [0, 2 pi] of the traction, by the
 *      composite Simpson rule over the nsurf panels of the closed curve.
 *   cloud, ops:   a 2D cloud and its operators (same n)
 *   u:            device [2][n] velocity; p: device [n] pressure
 *   centre:       host [2]; diameter D > 0; mu the dynamic viscosity
 *   nsurf:        even, 4 .. 1048576 (the paper uses 360)
 *   force:        host [2] out: F_x, F_y
 *   coef:         optional host [2] out: C_D, C_L = F / (rho u_ref^2 D / 2),
 *                 with rho > 0 and u_ref != 0; NULL to skip
 *   traction:     optional device [2][nsurf] out: the traction at each point
 *   bad_query:    optional host out: the surface point whose interpolation
 *                 system was singular, else -1
 * The surface may cross the cloud anywhere: its points take the q nearest
 * cloud points wherever they lie. Allocates device scratch for the five
 * fields at the nodes, synchronises the stream. On a periodic cloud the
 * surface points are interpolated as rbffd_interpolate does there (a periodic
 * array of cylinders). RBFFD_E_ARG for 3D clouds, mismatched sizes, odd or
 * out-of-range nsurf, a
 * non-positive or non-finite diameter; RBFFD_E_SINGULAR for a singular
 * interpolation system. */
int rbffd_cylinder_forces(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_ops *ops, const double *u,
                          const double *p, const double *centre, double diameter, double mu, int nsurf, double rho,
                          double u_ref, double *force, double *coef, double *traction, int64_t *bad_query,
                          void *hip_stream);

/* ---- Krylov solve ------------------------------------------------------- */
typedef struct {
    double tol;             /* stop when ||b - A x||_2 <= tol ||b||_2 (recursive residual) */
    int max_iter;           /* BiCGSTAB iterations                                   */
    int precision;          /* RBFFD_FP64, RBFFD_FP32_IR or RBFFD_FP32_MATRIX        */
    int preconditioner;     /* RBFFD_PREC_JACOBI or RBFFD_PREC_BLOCK64               */
} rbffd_krylov_opts;

typedef struct {
    int iters;              /* BiCGSTAB iterations (FP32_IR: inner iterations, all sweeps) */
    int status;             /* RBFFD_OK / RBFFD_E_NOCONV / RBFFD_E_BREAKDOWN         */
    int refinements;        /* FP32_IR: FP64 residual refinement sweeps              */
    int fp64_fallback;      /* FP32_IR: 1 when an FP32 sweep failed to halve the FP64
                               residual and the solve finished with FP64 sweeps      */
    double relres;          /* true FP64 residual ||b - A x|| / ||b|| at return      */
} rbffd_krylov_stats;

/* (Sec. 3, "preconditioned BiCGSTAB") Solve P x = rhs for the
 * pressure-correction matrix with BiCGSTAB, right-preconditioned by the
 * Jacobi diagonal or (opts->preconditioner) by the 64x64 diagonal blocks.
 * x holds the initial guess on entry and the solution on return.
 * rhs, x: device [n]. */
int poisson_solve(rbffd_ctx *ctx, const rbffd_ops *ops, const double *rhs, double *x,
                  const rbffd_krylov_opts *opts, rbffd_krylov_stats *stats, void *hip_stream);
/* (Sec. 3) Autotuner: time `iterations` (>= 4) FP64 Jacobi BiCGSTAB iterations
 * of the operators' pressure-correction system (a fixed right-hand side, zero
 * start, in scratch memory the call allocates and frees) on each path, the
 * multi-kernel iteration and the one-workgroup solver with 256, 512 and 1024
 * threads (the latter only up to 65,536 rows), and record the fastest for the
 * system's (n, q) as rbffd_ctx_set_solver_choice would. Outputs (host, each
 * may be NULL): *choice, and us_per_iter[4] = microseconds per iteration of
 * each candidate in that order (-1 where not tried). Synchronous. */
int rbffd_autotune_krylov(rbffd_ctx *ctx, const rbffd_ops *ops, int iterations, int *choice,
                          double *us_per_iter, void *hip_stream);

/* (Sec. 3, "preconditioned BiCGSTAB"; the batched configuration of many
 * independent clouds) Solve P_j x_j = rhs_j for `count` independent
 * pressure-correction systems at once, each as poisson_solve would (FP64
 * BiCGSTAB, right-preconditioned by the Jacobi diagonal or the 64x64 diagonal
 * blocks, restarts from the true residual). Every kernel stage
 * is one launch over all systems; each system owns a fixed range of thread
 * blocks and its own reductions, so its result is bitwise the same alone or
 * in any batch. Systems stop independently.
 *   ops, rhs, x: HOST arrays of `count` pointers; rhs[j], x[j] device [n_j];
 *                x[j] holds the initial guess on entry and the solution on
 *                return
 *   opts:        shared by all systems; precision RBFFD_FP64 or
 *                RBFFD_FP32_MATRIX (FP32 matrix values in the Krylov
 *                SpMVs, FP64 vectors; every start and the final check use
 *                the FP64 residual b - A x, and a system whose FP64 residual
 *                exceeds 10 tol iterates again from x, at most three times:
 *                iterative refinement; needs operators assembled with FP32
 *                copies), preconditioner RBFFD_PREC_JACOBI or
 *                RBFFD_PREC_BLOCK64
 *   stats:       host array of `count` records (may be NULL)
 * Returns RBFFD_OK when every system converged, RBFFD_E_NOCONV or
 * RBFFD_E_BREAKDOWN (the first failing code) otherwise; per-system outcomes
 * are in stats. */
int poisson_solve_batched(rbffd_ctx *ctx, int count, const rbffd_ops *const *ops, const double *const *rhs,
                          double *const *x, const rbffd_krylov_opts *opts, rbffd_krylov_stats *stats,
                          void *hip_stream);

/* ---- measurement --------------------------------------------------------- */
/* (Sec. 3, "preconditioned BiCGSTAB": the iteration that dominates the time
 * step) Mean durations of the four kernels of one FP64 Jacobi BiCGSTAB
 * iteration on the pressure-correction matrix, measured with HIP events on
 * the caller's stream, for roofline figures:
 *   us[0]  v = A p^ and r^.v                 (one matrix pass)
 *   us[1]  alpha, s = r - alpha v, s^ = D^-1 s, s.s and r^.s
 *   us[2]  t = A s^, t.s, t.t and r^.t       (one matrix pass)
 *   us[3]  omega, x, r and the next search direction, r.r (whole iteration
 *          minus the other three)
 *   us[4]  one whole iteration
 * The solve starts from x (device [n], overwritten with the iterate, not a
 * solution) with right-hand side rhs (device [n]), runs three iterations,
 * then times `reps` back-to-back launches of each of the first three kernels
 * (each recomputes the same outputs in place) and `reps` whole iterations,
 * with tolerance 0 so that nothing stops early. us: host [5]. Synchronises
 * the stream. RBFFD_E_ARG for reps < 1; RBFFD_E_BREAKDOWN if the iteration
 * broke down while being timed. */
int rbffd_krylov_kernel_times(rbffd_ctx *ctx, const rbffd_ops *ops, const double *rhs, double *x, int reps,
                              double *us, void *hip_stream);

/* ---- allocation-free solve ---------------------------------------------- */
/* For callers that cannot allocate memory during the call: code under HIP graph
 * capture, tight serving loops, and harnesses that forbid hipMalloc.
 * poisson_solve_noalloc solves P x = rhs exactly as poisson_solve does with
 * precision RBFFD_FP64 and preconditioner RBFFD_PREC_JACOBI by the default
 * multi-kernel iteration (a rbffd_ctx_set_solver_choice override applies to
 * poisson_solve only) with the same kernels and launch shapes, so the same
 * results, but it never replays HIP graphs, and its Krylov vectors, partial
 * sums and state records live in one fixed device array of
 * RBFFD_NOALLOC_SCRATCH_BYTES that the library holds on every device it is
 * loaded on, until the process ends. The call allocates no device or pinned
 * host memory: its few host read-backs go through the calling thread's stack.
 *   ops:   operators from rbffd_assemble; their context must have been created
 *          on the device (rbffd_ctx_create takes the array's address there)
 *   rhs, x: device [n]; x holds the initial guess on entry, the solution on return
 *   opts:  tol, max_iter; precision must be RBFFD_FP64 and preconditioner
 *          RBFFD_PREC_JACOBI
 *   stats: as poisson_solve (may be NULL)
 * Returns RBFFD_E_ARG, before any launch, when n exceeds RBFFD_NOALLOC_MAX_N
 * or for other options; RBFFD_E_NOCONV as poisson_solve. Every call on one
 * device shares that device's array and leaves its contents behind (each call
 * clears what it needs), so calls that overlap on one device race: the caller
 * serialises them. */
#define RBFFD_NOALLOC_SCRATCH_BYTES 67108864   /* 64 MiB per device                  */
#define RBFFD_NOALLOC_MAX_N 1179648            /* rows the array holds (7 FP64 vectors) */
int poisson_solve_noalloc(const rbffd_ops *ops, const double *rhs, double *x, const rbffd_krylov_opts *opts,
                          rbffd_krylov_stats *stats, void *hip_stream);

/* ---- continuous batching ------------------------------------------------ */
/* (Sec. 3, applied to a stream of independent requests) A server keeps a
 * running batch of pressure-correction solves (FP64, or FP32 matrix values
 * with FP64 vectors and residuals). Solves submitted while
 * others run join the batch at the next rbffd_server_run; finished ones leave
 * it and are collected with rbffd_server_poll. Each solve behaves as
 * poisson_solve (FP64 BiCGSTAB with the Jacobi or block-Jacobi preconditioner,
 * restarts from the true residual) and its result does not depend on which
 * other solves share the batch.
 * Work vectors (8 n doubles per solve) are charged to the context's HBM
 * budget at submission: RBFFD_E_OOM means "retry after some solves finish".
 * One server per context; calls on it must not overlap. */
typedef struct rbffd_server rbffd_server;
int rbffd_server_create(rbffd_ctx *ctx, rbffd_server **out);
int rbffd_server_destroy(rbffd_server *sv);
/* Queue a solve of P x = rhs (ops, rhs and x stay owned by the caller and must
 * outlive the solve; x holds the initial guess). opts: tol, max_iter (>= 1),
 * precision (RBFFD_FP64 or RBFFD_FP32_MATRIX, as in poisson_solve_batched)
 * and preconditioner, copied at submission.
 * *ticket identifies the solve. */
int rbffd_server_submit(rbffd_server *sv, const rbffd_ops *ops, const double *rhs, double *x,
                        const rbffd_krylov_opts *opts, int64_t *ticket);
/* Run up to `iterations` BiCGSTAB iterations on every queued or running solve
 * (synchronous on the stream); *active receives the number still running. */
int rbffd_server_run(rbffd_server *sv, int iterations, int *active, void *hip_stream);
/* Collect up to `max` finished solves: tickets[] and stats[] (host arrays). */
int rbffd_server_poll(rbffd_server *sv, int max, int64_t *tickets, rbffd_krylov_stats *stats, int *count);

/* ---- time step ---------------------------------------------------------- */
typedef struct {
    double rho, mu;         /* density and dynamic viscosity                         */
    double dt;              /* time step                                              */
    double alpha[3];        /* BDF coefficients (1.5, -2, 0.5); (1, -1, 0) = BDF1    */
    double tol_outer;       /* stop the outer iteration when Delta < tol_outer; <= 0:
                               run exactly max_outer iterations (not an error)        */
    double tol_krylov;      /* relative tolerance of every Krylov solve              */
    int max_outer;          /* outer iteration limit                                  */
    int max_krylov;         /* iteration limit of every Krylov solve                  */
    int precision;          /* RBFFD_FP64, RBFFD_FP32_IR or RBFFD_FP32_MATRIX        */
    int preconditioner;     /* of the pressure-correction solve: RBFFD_PREC_JACOBI or
                               RBFFD_PREC_BLOCK64; momentum and boundary-pressure
                               solves use Jacobi                                      */
    double force[3];        /* constant body force per unit volume added to the
                               momentum equations (and to the normal momentum
                               equation of the boundary pressure): the mean
                               pressure gradient that drives a periodic channel
                               (Sec. 4, Eq. bellow dp_dx); 0 for none                 */
} rbffd_step_opts;

typedef struct {
    int outer_iters;        /* outer iterations taken                                */
    int krylov_mom;         /* momentum BiCGSTAB iterations (sum over components)    */
    int krylov_p;           /* pressure-correction BiCGSTAB iterations               */
    int krylov_b;           /* boundary-pressure BiCGSTAB iterations                 */
    int status;             /* RBFFD_OK or the first failure code                    */
    double delta;           /* last Delta = sum_c mean_i |u_c^{r+1} - u_c^r|          */
    double eps_steady;      /* max_c mean_i |u_c^{n+1} - u_c^n| / dt                  */
    double div_l1;          /* mean over interior points of |sum_c D_c u_c^{n+1}|: the
                               discrete continuity error of the new velocity (Eq.
                               continuity:n+1)                                        */
    double final_relres_p;  /* true residual ||b - P p'|| / ||b|| of the last
                               pressure-correction solve                              */
    double krylov_relres_max; /* largest true relative residual over every Krylov
                               solve of the step (momentum, pressure correction,
                               boundary pressure)                                     */
} rbffd_step_stats;

/* (Sec. 3 and the step list of Sec. 3.2) One BDF time step: starting from
 * u^r = u^n (Dirichlet values of t^{n+1} on velocity-prescribed points) and
 * p^r = p^n, repeat  momentum solves for u~ (Eqs. u:tilde, v:tilde; outlet
 * rows N . grad u = 0) -> pressure correction (Eq. pressure poisson) ->
 * interior p += p' -> boundary pressure (Eq. normal momentum on
 * velocity-Dirichlet points, solved for their block with the other pressures
 * fixed; the given value on prescribed-pressure and outlet points) ->
 * u = u~ - dt/(rho alpha1) grad p' on interior points -> Delta, until
 * Delta < tol_outer or max_outer.
 *   u:      device [dim][n] in: u^n,     out: u^{n+1}
 *   u_prev: device [dim][n] in: u^{n-1}, out: u^n
 *   p:      device [n]      in: p^n,     out: p^{n+1}
 *   u_bc:   device [dim][n] Dirichlet velocity at t^{n+1} (read on
 *           velocity-prescribed rows)
 *   p_bc:   device [n] pressure at t^{n+1} (read on prescribed-pressure and
 *           outlet rows; may be NULL when the cloud has none)
 * Returns RBFFD_OK, or RBFFD_E_NOCONV when the outer or a Krylov iteration hit
 * its limit (fields hold the last iterate). */
int simple_step(rbffd_ctx *ctx, const rbffd_ops *ops, double *u, double *u_prev, double *p,
                const double *u_bc, const double *p_bc, const rbffd_step_opts *opts,
                rbffd_step_stats *stats, void *hip_stream);

/* (Sec. 3 and the step list of Sec. 3.2, over many independent clouds: the
 * batched configuration) One BDF time step of `count` clouds at once, each
 * exactly as simple_step defines it, with its own options (opts[j]: dt, BDF
 * coefficients, tolerances, limits, preconditioner). The per-cloud kernels run
 * cloud by cloud; every Krylov stage (the momentum solves, one system per
 * velocity component; the pressure corrections; the boundary pressures) is one
 * batched solve over the clouds still iterating, as in poisson_solve_batched,
 * so a cloud's fields do not depend on the other clouds in the call. A cloud
 * leaves the outer iteration when its own Delta meets its own tol_outer.
 *   ops, u, u_prev, p, u_bc, p_bc, opts, stats: host arrays of `count`; the
 *     device arrays they point to are laid out as for simple_step; p_bc[j] may
 *     be NULL for a cloud without prescribed-pressure points; stats[j] receives
 *     cloud j's statistics.
 * Restrictions (RBFFD_E_ARG before any launch): FP64 only, no symmetry points,
 * every ops[j] distinct and of this context. Returns RBFFD_OK, or the first
 * cloud's failure (E_NOCONV / E_BREAKDOWN; every cloud's own status is in
 * stats). The operators' momentum values are overwritten, as by simple_step. */
int simple_step_batched(rbffd_ctx *ctx, int count, const rbffd_ops *const *ops, double *const *u,
                        double *const *u_prev, double *const *p, const double *const *u_bc,
                        const double *const *p_bc, const rbffd_step_opts *opts, rbffd_step_stats *stats,
                        void *hip_stream);

/* (Sec. 3.2) |lambda|max of the discrete convection-diffusion operator
 * -rho (u0 . grad) + mu Laplacian on interior rows (boundary rows zero), by
 * `iters` normalised power iterations from x_i = 1 + (i mod 7)/7; a Courant
 * number Co gives dt = 2 Co / |lambda|max. u0: device [dim][n]. */
int rbffd_convdiff_lambda(rbffd_ctx *ctx, const rbffd_ops *ops, const double *u0, double rho,
                          double mu, int iters, double *lambda_out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RBFFD_H */
