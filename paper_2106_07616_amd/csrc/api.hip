// C ABI entry points, context and error handling.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include <vector>

#include "forces.h"
#include "internal.h"
#include "periodic.h"

namespace rbffd {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return (e == hipErrorOutOfMemory) ? RBFFD_E_OOM : RBFFD_E_DEVICE;
}

int dev_alloc(rbffd_ctx *ctx, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) return RBFFD_OK;
    if (ctx->budget && ctx->in_use + bytes > ctx->budget)
        return fail(RBFFD_E_OOM, "allocation of " + std::to_string(bytes) +
                                     " bytes exceeds the context's HBM budget");
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    ctx->in_use += bytes;
    return RBFFD_OK;
}

void dev_free(rbffd_ctx *ctx, void *p, size_t bytes)
{
    if (!p) return;
    (void)hipFree(p);
    if (ctx) ctx->in_use -= bytes;
}

int workspace(rbffd_ctx *ctx, int slot, size_t bytes, void **p)
{
    Buffer &b = ctx->ws[slot];
    if (b.bytes < bytes) {
        size_t grow = bytes + bytes / 4;
        if (slot == WS_HOST_PINNED || slot == WS_BATCH_HOST || slot == WS_BUILD_HOST) {
            if (b.ptr) (void)hipHostFree(b.ptr);
            b.ptr = nullptr;
            b.bytes = 0;
            RB_HIP(hipHostMalloc(&b.ptr, grow, hipHostMallocDefault));
        } else {
            if (b.ptr) {
                RB_HIP(hipDeviceSynchronize());
                dev_free(ctx, b.ptr, b.bytes);
            }
            b.ptr = nullptr;
            b.bytes = 0;
            RB_CHECK(dev_alloc(ctx, &b.ptr, grow));
        }
        b.bytes = grow;
    }
    *p = b.ptr;
    return RBFFD_OK;
}

int host_scratch(rbffd_ctx *ctx, size_t off, size_t bytes, void **p)
{
    if (off + bytes > kHostBytes) return fail(RBFFD_E_ARG, "host staging request too large");
    char *base = nullptr;
    RB_CHECK(workspace(ctx, WS_HOST_PINNED, kHostBytes, (void **)&base));
    *p = base + off;
    return RBFFD_OK;
}

static int check_cloud(const rbffd_cloud *c)
{
    if (!c) return fail(RBFFD_E_ARG, "cloud is NULL");
    if (c->dim != 2 && c->dim != 3) return fail(RBFFD_E_ARG, "dim must be 2 or 3");
    if (c->n < 1 || c->n >= (int64_t(1) << 31)) return fail(RBFFD_E_ARG, "n out of range");
    if (!c->xyz) return fail(RBFFD_E_ARG, "cloud.xyz is NULL");
    for (int d = 0; d < 3; ++d) {
        if (!(c->period[d] >= 0.0) || !std::isfinite(c->period[d]))
            return fail(RBFFD_E_ARG, "cloud.period must be finite and >= 0");
        if (d >= c->dim && c->period[d] != 0.0) return fail(RBFFD_E_ARG, "cloud.period set beyond dim");
    }
    return RBFFD_OK;
}

static bool is_periodic(const rbffd_cloud *c)
{
    for (int d = 0; d < c->dim; ++d)
        if (c->period[d] > 0.0) return true;
    return false;
}

// The periodic box of a cloud (Sec. 3.1) for images: its bounds (from the
// device), a first band width (twice the radius holding q points at the mean
// density) and the shift vectors m in {-1, 0, 1}^3, nonzero only along
// periodic axes, in lexicographic order.
static int periodic_setup(rbffd_ctx *ctx, const rbffd_cloud *cloud, int q, hipStream_t s, PeriodicShifts *P,
                          double *band)
{
    const int dim = cloud->dim;
    const int64_t n = cloud->n;
    const double *L = cloud->period;
    RB_CHECK(device_bbox(ctx, dim, n, cloud->xyz, P->lo, P->hi, s));
    double vol = 1.0;
    for (int d = 0; d < dim; ++d) {
        P->L[d] = L[d];
        if (L[d] > 0.0 && !(P->hi[d] - P->lo[d] < L[d]))
            return fail(RBFFD_E_ARG, "the cloud's extent along a periodic axis is not below its period");
        vol *= (L[d] > 0.0) ? L[d] : std::max(P->hi[d] - P->lo[d], 1e-300);
    }
    const double pi = 3.14159265358979323846;
    *band = 2.0 * ((dim == 2) ? std::sqrt(q * vol / (pi * (double)n))
                              : std::cbrt(3.0 * q * vol / (4.0 * pi * (double)n)));
    P->count = 0;
    for (int a = -1; a <= 1; ++a)
        for (int bb = -1; bb <= 1; ++bb)
            for (int c = -1; c <= 1; ++c) {
                const int m[3] = {a, bb, c};
                bool ok = !(a == 0 && bb == 0 && c == 0);
                for (int d = 0; d < 3; ++d)
                    if (m[d] != 0 && (d >= dim || !(L[d] > 0.0))) ok = false;
                if (!ok) continue;
                for (int d = 0; d < 3; ++d) P->m[P->count][d] = m[d];
                ++P->count;
            }
    return RBFFD_OK;
}

// Stencils of a cloud that wraps along its periodic axes (Sec. 3.1): ghost
// images x_j +- period e_d of the points within a band of each periodic face
// are appended, the neighbour search and the weights run on the augmented
// points (the images' own coordinates: clouds near one face take points from
// the other), and neighbour indices are mapped back to the points they are
// images of. The band starts at twice the radius that holds q points at the
// mean density and doubles until every point's q-th neighbour lies within it,
// which makes the search exact. Every step over the points runs on the
// device; the host sees the bounding box, the image count and two flags.
static int stencils_periodic(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts, int q,
                             int32_t *nbr, double *w, int64_t *bad_point, hipStream_t s)
{
    const int dim = cloud->dim;
    const int64_t n = cloud->n;
    PeriodicShifts P;
    double band = 0.0;
    RB_CHECK(periodic_setup(ctx, cloud, q, s, &P, &band));
    int64_t *flags = nullptr;   // [0]: singular point, [1]: cloud with a repeated point, [2]: q-th beyond the band
    RB_CHECK(workspace(ctx, WS_MISC, 3 * sizeof(int64_t), (void **)&flags));
    int64_t *hf = nullptr;
    RB_CHECK(host_scratch(ctx, kHostMisc, 3 * sizeof(int64_t), (void **)&hf));
    for (int attempt = 0; attempt < 12; ++attempt, band *= 2.0) {
        P.band = band;
        double *aug = nullptr;
        int32_t *owner = nullptr;
        int64_t naug = 0;
        size_t abytes = 0, obytes = 0;
        RB_CHECK(launch_periodic_images(ctx, dim, n, cloud->xyz, P, &aug, &owner, &naug, &abytes, &obytes, s));
        int st = launch_knn_points(ctx, dim, naug, aug, n, aug, q, nbr, s);
        if (st == RBFFD_OK) st = launch_periodic_inside(dim, n, aug, aug, q, nbr, band, nullptr, (int *)(flags + 2), s);
        if (st == RBFFD_OK) {
            hipError_t e = hipMemcpyAsync(hf + 2, flags + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(e, "periodic neighbours");
        }
        if (st == RBFFD_OK && *(const int *)(hf + 2) != 0) {
            dev_free(ctx, aug, abytes);
            dev_free(ctx, owner, obytes);
            continue;   // a q-th neighbour beyond the band: widen it
        }
        if (st == RBFFD_OK)
            st = launch_weights(ctx, dim, n, aug, q, nbr, opts->poly_degree, opts->phs_power, w, flags, s);
        // neighbour indices back to the points they are images of; a point may
        // appear in a cloud only once
        if (st == RBFFD_OK) st = launch_periodic_remap(n, q, owner, nbr, flags + 1, s);
        if (st == RBFFD_OK) {
            hipError_t e = hipMemcpyAsync(hf, flags, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(e, "periodic weights");
        }
        (void)hipStreamSynchronize(s);
        dev_free(ctx, aug, abytes);
        dev_free(ctx, owner, obytes);
        RB_CHECK(st);
        if (hf[1] != INT64_MAX)
            return fail(RBFFD_E_ARG, "point " + std::to_string(hf[1]) +
                                         ": its cloud holds two images of one point (period too small for q)");
        const int64_t bad = (hf[0] == INT64_MAX) ? -1 : hf[0];
        if (bad_point) *bad_point = bad;
        if (bad >= 0) return fail(RBFFD_E_SINGULAR, "singular collocation system at point " + std::to_string(bad));
        return RBFFD_OK;
    }
    return fail(RBFFD_E_ARG, "no band of periodic images holds every cloud");
}

static int binom(int a, int b)
{
    long r = 1;
    for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
    return (int)r;
}

static int resolve_sizes(int dim, const rbffd_stencil_opts *o, int *q, int *m, int *R)
{
    if (!o) return fail(RBFFD_E_ARG, "stencil options are NULL");
    if (dim != 2 && dim != 3) return fail(RBFFD_E_ARG, "dim must be 2 or 3");
    if (o->phs_power != 3 && o->phs_power != 5) return fail(RBFFD_E_ARG, "phs_power must be 3 or 5");
    if (o->poly_degree < 0 || o->poly_degree > 6) return fail(RBFFD_E_ARG, "poly_degree must be 0..6");
    int mm = binom(o->poly_degree + dim, dim);
    int qq = o->q ? o->q : 2 * mm;
    if (qq <= mm) return fail(RBFFD_E_ARG, "cloud size q must exceed the monomial count m");
    if (qq > kMaxQ) return fail(RBFFD_E_ARG, "cloud size q exceeds 128");
    *q = qq;
    *m = mm;
    *R = dim + 1;
    return RBFFD_OK;
}

}  // namespace rbffd

using namespace rbffd;

extern "C" {

const char *rbffd_last_error(void) { return g_last_error.c_str(); }

int rbffd_ctx_create(rbffd_ctx **ctx, int hip_device, size_t hbm_budget_bytes)
{
    if (!ctx) return fail(RBFFD_E_ARG, "ctx is NULL");
    *ctx = nullptr;
    int ndev = 0;
    RB_HIP(hipGetDeviceCount(&ndev));
    if (hip_device < 0 || hip_device >= ndev) return fail(RBFFD_E_ARG, "no such HIP device");
    RB_HIP(hipSetDevice(hip_device));
    // the allocation-free solve's scratch array: its address on this device
    RB_CHECK(noalloc_init(hip_device));
    rbffd_ctx *c = new (std::nothrow) rbffd_ctx();
    if (!c) return fail(RBFFD_E_OOM, "host allocation failed");
    c->device = hip_device;
    c->budget = hbm_budget_bytes;
    *ctx = c;
    g_last_error.clear();
    return RBFFD_OK;
}

struct rbffd_server {
    rbffd_ctx *ctx;
    rbffd::Server *impl;
};

static void release_ops_memory(rbffd_ops *ops);

int rbffd_ctx_destroy(rbffd_ctx *ctx)
{
    if (!ctx) return RBFFD_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (rbffd_server *sv : ctx->servers) {
        server_destroy(sv->impl);
        sv->impl = nullptr;
        sv->ctx = nullptr;
    }
    for (rbffd_ops *ops : ctx->ops) {
        release_ops_memory(ops);
        ops->ctx = nullptr;
    }
    graph_cache_destroy(ctx);
    for (int s = 0; s < WS_COUNT; ++s) {
        if (!ctx->ws[s].ptr) continue;
        if (s == WS_HOST_PINNED || s == WS_BATCH_HOST || s == WS_BUILD_HOST)
            (void)hipHostFree(ctx->ws[s].ptr);
        else
            dev_free(ctx, ctx->ws[s].ptr, ctx->ws[s].bytes);
    }
    delete ctx;
    return RBFFD_OK;
}

size_t rbffd_ctx_bytes_in_use(const rbffd_ctx *ctx) { return ctx ? ctx->in_use : 0; }

int rbffd_ctx_set_solver_choice(rbffd_ctx *ctx, int64_t n, int q, int choice)
{
    if (!ctx) return fail(RBFFD_E_ARG, "ctx is NULL");
    if (n < 1 || q < 1) return fail(RBFFD_E_ARG, "n and q must be positive");
    if (choice == -1) {
        ctx->solver_choice.erase({n, q});
        return RBFFD_OK;
    }
    if (choice != 0 && choice != 256 && choice != 512 && choice != 1024)
        return fail(RBFFD_E_ARG, "choice must be -1, 0, 256, 512 or 1024");
    ctx->solver_choice[{n, q}] = choice;
    return RBFFD_OK;
}

int rbffd_autotune_krylov(rbffd_ctx *ctx, const rbffd_ops *ops, int iterations, int *choice, double *us_per_iter,
                          void *hip_stream)
{
    if (!ctx || !ops) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    RB_HIP(hipSetDevice(ctx->device));
    return autotune_solver(ctx, ops->n, ops->q, cols_of(ops), ops->pval, ops->pdinv, iterations, choice, us_per_iter,
                           (hipStream_t)hip_stream);
}

int rbffd_ctx_set_graphs(rbffd_ctx *ctx, int enable)
{
    if (!ctx) return fail(RBFFD_E_ARG, "ctx is NULL");
    if (enable != 0 && enable != 1) return fail(RBFFD_E_ARG, "enable must be 0 or 1");
    ctx->use_graphs = enable != 0;
    return RBFFD_OK;
}

int rbffd_stencil_sizes(int dim, const rbffd_stencil_opts *opts, int *q, int *m, int *R)
{
    int qq, mm, rr;
    RB_CHECK(resolve_sizes(dim, opts, &qq, &mm, &rr));
    if (q) *q = qq;
    if (m) *m = mm;
    if (R) *R = rr;
    return RBFFD_OK;
}

int rbffd_build_stencils(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts,
                         int32_t *nbr, double *w, int64_t *bad_point, void *hip_stream)
{
    if (!ctx) return fail(RBFFD_E_ARG, "ctx is NULL");
    RB_CHECK(check_cloud(cloud));
    int q, m, R;
    RB_CHECK(resolve_sizes(cloud->dim, opts, &q, &m, &R));
    if (q > cloud->n) return fail(RBFFD_E_ARG, "cloud size q exceeds the number of points");
    if (!nbr || !w) return fail(RBFFD_E_ARG, "nbr or w is NULL");
    if (q + m > 128) return fail(RBFFD_E_ARG, "collocation systems larger than 128 (q + m) are not supported");
    RB_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    if (bad_point) *bad_point = -1;
    if (is_periodic(cloud)) return stencils_periodic(ctx, cloud, opts, q, nbr, w, bad_point, s);
    RB_CHECK(launch_knn(ctx, cloud->dim, cloud->n, cloud->xyz, q, nbr, s));
    int64_t *bad_dev = nullptr;   // [0] singular stencil, [1] duplicate point
    RB_CHECK(workspace(ctx, WS_MISC, 2 * sizeof(int64_t), (void **)&bad_dev));
    RB_CHECK(launch_dup_check(cloud->dim, cloud->n, cloud->xyz, q, nbr, bad_dev + 1, s));
    RB_CHECK(launch_weights(ctx, cloud->dim, cloud->n, cloud->xyz, q, nbr, opts->poly_degree,
                            opts->phs_power, w, bad_dev, s));
    int64_t *hb = nullptr;
    RB_CHECK(host_scratch(ctx, kHostMisc, 2 * sizeof(int64_t), (void **)&hb));
    RB_HIP(hipMemcpyAsync(hb, bad_dev, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    if (hb[1] != INT64_MAX)
        return fail(RBFFD_E_ARG, "duplicate points: point " + std::to_string(hb[1]) + " coincides with another point");
    int64_t bad = (*hb == INT64_MAX) ? -1 : *hb;
    if (bad_point) *bad_point = bad;
    if (bad >= 0) return fail(RBFFD_E_SINGULAR, "singular collocation system at point " + std::to_string(bad));
    return RBFFD_OK;
}

int rbffd_build_stencils_batched(rbffd_ctx *ctx, int count, const rbffd_cloud *clouds,
                                 const rbffd_stencil_opts *opts, int32_t *const *nbr, double *const *w,
                                 int64_t *bad_points, void *hip_stream)
{
    if (!ctx) return fail(RBFFD_E_ARG, "ctx is NULL");
    if (count < 0) return fail(RBFFD_E_ARG, "count must be >= 0");
    if (count == 0) return RBFFD_OK;
    if (!clouds || !opts || !nbr || !w) return fail(RBFFD_E_ARG, "NULL argument");
    // every check before any launch
    std::vector<int> qs(count), ms(count), width(count);
    for (int j = 0; j < count; ++j) {
        const rbffd_cloud *c = &clouds[j];
        const std::string at = " (cloud " + std::to_string(j) + ")";
        int st = check_cloud(c);
        if (st != RBFFD_OK) return fail(st, rbffd_last_error() + at);
        int R;
        st = resolve_sizes(c->dim, &opts[j], &qs[j], &ms[j], &R);
        if (st != RBFFD_OK) return fail(st, rbffd_last_error() + at);
        if (qs[j] > c->n) return fail(RBFFD_E_ARG, "cloud size q exceeds the number of points" + at);
        if (!nbr[j] || !w[j]) return fail(RBFFD_E_ARG, "nbr or w is NULL" + at);
        if (qs[j] + ms[j] > 128) return fail(RBFFD_E_ARG, "collocation systems larger than 128 are not supported" + at);
        if (is_periodic(c)) return fail(RBFFD_E_ARG, "periodic clouds are built one at a time (rbffd_build_stencils)" + at);
        width[j] = weight_width(qs[j] + ms[j]);   // 0: 65-128 unknowns, the Gauss-Jordan kernels
    }
    RB_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    if (bad_points)
        for (int j = 0; j < count; ++j) bad_points[j] = -1;
    // neighbour search, cloud by cloud
    for (int j = 0; j < count; ++j)
        RB_CHECK(launch_knn(ctx, clouds[j].dim, clouds[j].n, clouds[j].xyz, qs[j], nbr[j], s));
    // launch groups: one per (dimension, register width) present; the clouds
    // of a group are contiguous in `order`, and so are their descriptors and
    // singular-point slots (slot t belongs to cloud order[t])
    std::vector<int> order;
    std::vector<std::pair<int, int>> groups;   // (dim, width) of each launch, width 0 = LDS
    std::vector<size_t> gstart;
    for (int dim = 2; dim <= 3; ++dim)
        for (int wd : {16, 24, 32, 40, 48, 56, 64, 0}) {
            const size_t before = order.size();
            for (int j = 0; j < count; ++j)
                if (clouds[j].dim == dim && width[j] == wd) order.push_back(j);
            if (order.size() > before) {
                groups.push_back({dim, wd});
                gstart.push_back(before);
            }
        }
    gstart.push_back(order.size());
    std::vector<WeightSys> sys(count);
    std::vector<int64_t> blocks(groups.size(), 0);
    for (size_t g = 0; g < groups.size(); ++g)
        for (size_t t = gstart[g]; t < gstart[g + 1]; ++t) {
            const int j = order[t];
            sys[t] = WeightSys{clouds[j].xyz, nbr[j], w[j], clouds[j].n, blocks[g], qs[j], ms[j],
                               opts[j].phs_power, width[j]};
            blocks[g] += clouds[j].n;
        }
    // descriptors, singular-point and duplicate-point slots:
    // [sys: count][pad][bad: count][dup: count]
    const size_t dbytes = (sizeof(WeightSys) * (size_t)count + 255) / 256 * 256;
    const size_t bytes = dbytes + 2 * sizeof(int64_t) * (size_t)count;
    char *dev = nullptr, *host = nullptr;
    RB_CHECK(workspace(ctx, WS_BUILD, bytes, (void **)&dev));
    RB_CHECK(workspace(ctx, WS_BUILD_HOST, bytes, (void **)&host));
    // the staging buffer is free: every batched build synchronises the stream
    // before it returns
    std::memcpy(host, sys.data(), sizeof(WeightSys) * (size_t)count);
    int64_t *hbad = (int64_t *)(host + dbytes);
    for (int j = 0; j < count; ++j) hbad[j] = INT64_MAX;
    RB_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, s));
    const WeightSys *dsys = (const WeightSys *)dev;
    int64_t *dbad = (int64_t *)(dev + dbytes);
    int64_t *ddup = dbad + count;
    for (int j = 0; j < count; ++j)
        RB_CHECK(launch_dup_check(clouds[j].dim, clouds[j].n, clouds[j].xyz, qs[j], nbr[j], ddup + j, s));
    for (size_t g = 0; g < groups.size(); ++g) {
        const int dim = groups[g].first, wd = groups[g].second;
        const size_t t0 = gstart[g], nt = gstart[g + 1] - gstart[g];
        if (wd > 0) {
            RB_CHECK(launch_weights_batched(dim, wd, (int)nt, dsys + t0, blocks[g], dbad + t0, s));
        } else {
            // systems of 65-128 unknowns: the Gauss-Jordan kernels, cloud by cloud
            for (size_t t = t0; t < t0 + nt; ++t) {
                const int j = order[t];
                RB_CHECK(launch_weights(ctx, dim, clouds[j].n, clouds[j].xyz, qs[j], nbr[j], opts[j].poly_degree,
                                        opts[j].phs_power, w[j], dbad + t, s));
            }
        }
    }
    RB_HIP(hipMemcpyAsync(hbad, dbad, 2 * sizeof(int64_t) * (size_t)count, hipMemcpyDeviceToHost, s));
    RB_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < count; ++j)
        if (hbad[count + j] != INT64_MAX)
            return fail(RBFFD_E_ARG, "duplicate points: point " + std::to_string(hbad[count + j]) + " of cloud " +
                                         std::to_string(j) + " coincides with another point");
    int first_bad = -1;
    for (int t = 0; t < count; ++t) {
        const int j = order[t];
        const int64_t bp = (hbad[t] == INT64_MAX) ? -1 : hbad[t];
        if (bad_points) bad_points[j] = bp;
        if (bp >= 0 && (first_bad < 0 || j < first_bad)) first_bad = j;
    }
    if (first_bad >= 0)
        return fail(RBFFD_E_SINGULAR, "singular collocation system in cloud " + std::to_string(first_bad));
    return RBFFD_OK;
}

int rbffd_assemble(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts,
                   const int32_t *nbr, const double *w, int precision, rbffd_ops **out,
                   void *hip_stream)
{
    if (!ctx || !out) return fail(RBFFD_E_ARG, "ctx or out is NULL");
    *out = nullptr;
    RB_CHECK(check_cloud(cloud));
    if (!cloud->kind || !cloud->normal) return fail(RBFFD_E_ARG, "cloud.kind or cloud.normal is NULL");
    if (cloud->pin < -1 || cloud->pin >= cloud->n) return fail(RBFFD_E_ARG, "pin out of range");
    if (precision != RBFFD_FP64 && precision != RBFFD_FP32_IR && precision != RBFFD_FP32_MATRIX)
        return fail(RBFFD_E_ARG, "unknown precision");
    int q, m, R;
    RB_CHECK(resolve_sizes(cloud->dim, opts, &q, &m, &R));
    if (q > cloud->n) return fail(RBFFD_E_ARG, "cloud size q exceeds the number of points");
    if (!nbr || !w) return fail(RBFFD_E_ARG, "nbr or w is NULL");
    RB_HIP(hipSetDevice(ctx->device));
    rbffd_ops *ops = new (std::nothrow) rbffd_ops();
    if (!ops) return fail(RBFFD_E_OOM, "host allocation failed");
    int st = assemble_ops(ctx, cloud, q, opts->poly_degree, opts->phs_power, nbr, w, precision, ops,
                          (hipStream_t)hip_stream);
    if (st != RBFFD_OK) {
        std::string msg = g_last_error;
        rbffd_ops_free(ops);
        return fail(st, msg);
    }
    ctx->ops.insert(ops);
    *out = ops;
    return RBFFD_OK;
}

// device memory of an operator object (the object itself stays)
static void release_ops_memory(rbffd_ops *ops)
{
    void **ptrs[] = {(void **)&ops->kind,   (void **)&ops->normal, (void **)&ops->col,    (void **)&ops->cbase,
                     (void **)&ops->col16,  (void **)&ops->val,    (void **)&ops->pval,   (void **)&ops->pdinv, (void **)&ops->pbinv, (void **)&ops->pbscale,
                     (void **)&ops->pval32, (void **)&ops->pdinv32, (void **)&ops->mval, (void **)&ops->mdinv,
                     (void **)&ops->mval32, (void **)&ops->mdinv32, (void **)&ops->bidx, (void **)&ops->bpos,
                     (void **)&ops->gcol,   (void **)&ops->gval,   (void **)&ops->gdinv};
    for (void **p : ptrs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    if (ops->ctx) ops->ctx->in_use -= ops->bytes;
    ops->bytes = 0;
}

int rbffd_ops_free(rbffd_ops *ops)
{
    if (!ops) return RBFFD_OK;
    rbffd_ctx *ctx = ops->ctx;
    if (ctx) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        ctx->ops.erase(ops);
        release_ops_memory(ops);
    }
    delete ops;
    return RBFFD_OK;
}

int rbffd_ops_info(const rbffd_ops *ops, int64_t *n, int *q, int *dim, int64_t *n_boundary)
{
    if (!ops) return fail(RBFFD_E_ARG, "ops is NULL");
    if (n) *n = ops->n;
    if (q) *q = ops->q;
    if (dim) *dim = ops->dim;
    if (n_boundary) *n_boundary = ops->nb;
    return RBFFD_OK;
}

int rbffd_ops_export_csr(const rbffd_ops *ops, int32_t *col, double *val, void *hip_stream)
{
    if (!ops || !col || !val) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    RB_HIP(hipSetDevice(ops->ctx->device));
    return export_csr(ops, col, val, (hipStream_t)hip_stream);
}

int rbffd_ops_export_block_inverse(const rbffd_ops *ops, float *out, void *hip_stream)
{
    if (!ops || !out) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    RB_HIP(hipSetDevice(ops->ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    RB_CHECK(ensure_block_inverse(ops, s));
    RB_CHECK(expand_block_inverse(ops, out, s));
    RB_HIP(hipStreamSynchronize(s));
    return RBFFD_OK;
}

int rbffd_apply(rbffd_ctx *ctx, const rbffd_ops *ops, int which, const double *x, double *y,
                void *hip_stream)
{
    if (!ctx || !ops || !x || !y) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    if (which < 0 || which > ops->dim + 1) return fail(RBFFD_E_ARG, "operator index out of range");
    RB_HIP(hipSetDevice(ctx->device));
    return apply_op(ctx, ops, which, x, y, (hipStream_t)hip_stream);
}

// Interpolation on a periodic cloud (Sec. 2 off the nodes, Sec. 3.1 periodic
// boundaries). Query coordinates outside [lo, lo + L) along a periodic axis
// are wrapped to lo + r, r = fmod(x - lo, L) taken into [0, L). Each query
// takes its q nearest among the points and their images within a band of the
// box; the band widens until every q-th neighbour lies closer than the band
// less the query's own distance outside the box, so no image left out can be
// nearer. Weights use the images' coordinates; the clouds are then written
// with the indices of the points the images stand for, and the fields are
// sampled through them.
static int interpolate_periodic(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts, int q,
                                int64_t nq, const double *qxyz, int nfield, const double *fields, double *out,
                                int32_t *nbr, double *w, int64_t *bad_query, hipStream_t s)
{
    const int dim = cloud->dim;
    const int64_t n = cloud->n;
    PeriodicShifts P;
    double band = 0.0;
    RB_CHECK(periodic_setup(ctx, cloud, q, s, &P, &band));
    // the queries, wrapped into the box, and their margins, on the device
    const size_t qbytes = sizeof(double) * nq * (dim + 1);
    double *qdev = nullptr;
    RB_CHECK(dev_alloc(ctx, (void **)&qdev, qbytes));
    double *margin = qdev + nq * dim;
    int64_t *flags = nullptr, *hf = nullptr;   // [0]: singular query, [1]: cloud with a repeated point, [2]: flag
    int st = workspace(ctx, WS_MISC, 3 * sizeof(int64_t), (void **)&flags);
    if (st == RBFFD_OK) st = host_scratch(ctx, kHostMisc, 3 * sizeof(int64_t), (void **)&hf);
    hipError_t e = hipSuccess;
    if (st == RBFFD_OK && nq > 0) {
        e = hipMemcpyAsync(qdev, qxyz, sizeof(double) * nq * dim, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) st = hip_fail(e, "periodic queries");
    }
    if (st == RBFFD_OK) st = launch_periodic_wrap(dim, nq, qdev, P, margin, (int *)(flags + 2), s);
    if (st == RBFFD_OK) {
        e = hipMemcpyAsync(hf + 2, flags + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "periodic queries");
        else if (*(const int *)(hf + 2) != 0) st = fail(RBFFD_E_ARG, "non-finite query coordinates");
    }
    bool done = false;
    for (int attempt = 0; st == RBFFD_OK && !done && attempt < 12; ++attempt, band *= 2.0) {
        P.band = band;
        double *aug = nullptr;
        int32_t *owner = nullptr;
        int64_t naug = 0;
        size_t abytes = 0, obytes = 0;
        st = launch_periodic_images(ctx, dim, n, cloud->xyz, P, &aug, &owner, &naug, &abytes, &obytes, s);
        if (st != RBFFD_OK) break;
        st = launch_knn_points(ctx, dim, naug, aug, nq, qdev, q, nbr, s);
        // no image left out can be nearer than band less the query's margin
        if (st == RBFFD_OK) st = launch_periodic_inside(dim, nq, qdev, aug, q, nbr, band, margin, (int *)(flags + 2), s);
        if (st == RBFFD_OK) {
            e = hipMemcpyAsync(hf + 2, flags + 2, sizeof(int64_t), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) st = hip_fail(e, "periodic neighbours");
        }
        if (st == RBFFD_OK && *(const int *)(hf + 2) == 0) {
            done = true;
            st = launch_interp(ctx, dim, naug, aug, nq, qdev, q, nbr, opts->poly_degree, opts->phs_power, w, flags, 0,
                               nullptr, nullptr, s);
            // image indices back to the points they stand for; a point may
            // appear in a cloud only once
            if (st == RBFFD_OK) st = launch_periodic_remap(nq, q, owner, nbr, flags + 1, s);
            if (st == RBFFD_OK) {
                e = hipMemcpyAsync(hf, flags, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e != hipSuccess) st = hip_fail(e, "periodic interpolation weights");
            }
            if (st == RBFFD_OK && hf[1] != INT64_MAX)
                st = fail(RBFFD_E_ARG, "query " + std::to_string(hf[1]) +
                                           ": its cloud holds two images of one point (period too small for q)");
        }
        (void)hipStreamSynchronize(s);
        dev_free(ctx, aug, abytes);
        dev_free(ctx, owner, obytes);
    }
    if (st == RBFFD_OK && !done) st = fail(RBFFD_E_ARG, "no band of periodic images holds every cloud");
    const int64_t bad = (st == RBFFD_OK && hf[0] != INT64_MAX) ? hf[0] : -1;
    if (st == RBFFD_OK && bad < 0) st = launch_interp_apply(nq, q, nbr, w, nfield, n, fields, out, s);
    (void)hipStreamSynchronize(s);
    dev_free(ctx, qdev, qbytes);
    RB_CHECK(st);
    if (bad_query) *bad_query = bad;
    if (bad >= 0) return fail(RBFFD_E_SINGULAR, "singular interpolation system at query " + std::to_string(bad));
    return RBFFD_OK;
}

int rbffd_interpolate(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_stencil_opts *opts, int64_t nq,
                      const double *qxyz, int nfield, const double *fields, double *out, int32_t *nbr_out,
                      double *w_out, int64_t *bad_query, void *hip_stream)
{
    if (!ctx) return fail(RBFFD_E_ARG, "ctx is NULL");
    if (bad_query) *bad_query = -1;
    RB_CHECK(check_cloud(cloud));
    int q, m, R;
    RB_CHECK(resolve_sizes(cloud->dim, opts, &q, &m, &R));
    if (q > cloud->n) return fail(RBFFD_E_ARG, "cloud size q exceeds the number of points");
    if (q + m > 128) return fail(RBFFD_E_ARG, "collocation systems larger than 128 (q + m) are not supported");
    if (nq < 0 || nfield < 0) return fail(RBFFD_E_ARG, "nq and nfield must be >= 0");
    if (nq > INT32_MAX) return fail(RBFFD_E_ARG, "too many query points");
    if (nq == 0) return RBFFD_OK;
    if (!qxyz) return fail(RBFFD_E_ARG, "qxyz is NULL");
    if (nfield > 0 && (!fields || !out)) return fail(RBFFD_E_ARG, "fields or out is NULL");
    RB_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t nb = sizeof(int32_t) * nq * q, wb = sizeof(double) * nq * q;
    int32_t *nbr = nbr_out;
    double *w = w_out;
    if (!nbr) RB_CHECK(dev_alloc(ctx, (void **)&nbr, nb));
    if (!w) {
        const int st = dev_alloc(ctx, (void **)&w, wb);
        if (st != RBFFD_OK) {
            if (!nbr_out) dev_free(ctx, nbr, nb);
            return st;
        }
    }
    int64_t *bad_dev = nullptr;
    int64_t *hb = nullptr;
    int st = workspace(ctx, WS_MISC, sizeof(int64_t), (void **)&bad_dev);
    if (st == RBFFD_OK) st = host_scratch(ctx, kHostMisc, sizeof(int64_t), (void **)&hb);
    if (st == RBFFD_OK && is_periodic(cloud)) {
        st = interpolate_periodic(ctx, cloud, opts, q, nq, qxyz, nfield, fields, out, nbr, w, bad_query, s);
        if (!w_out) dev_free(ctx, w, wb);
        if (!nbr_out) dev_free(ctx, nbr, nb);
        return st;
    }
    if (st == RBFFD_OK) st = launch_knn_points(ctx, cloud->dim, cloud->n, cloud->xyz, nq, qxyz, q, nbr, s);
    if (st == RBFFD_OK)
        st = launch_interp(ctx, cloud->dim, cloud->n, cloud->xyz, nq, qxyz, q, nbr, opts->poly_degree,
                           opts->phs_power, w, bad_dev, nfield, fields, out, s);
    hipError_t e = hipSuccess;
    if (st == RBFFD_OK) {
        e = hipMemcpyAsync(hb, bad_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    } else {
        (void)hipStreamSynchronize(s);
    }
    if (!w_out) dev_free(ctx, w, wb);
    if (!nbr_out) dev_free(ctx, nbr, nb);
    if (st != RBFFD_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "interpolation");
    const int64_t bad = (*hb == INT64_MAX) ? -1 : *hb;
    if (bad_query) *bad_query = bad;
    if (bad >= 0) return fail(RBFFD_E_SINGULAR, "singular interpolation system at query " + std::to_string(bad));
    return RBFFD_OK;
}

// most surface points of one force evaluation
static constexpr int kMaxSurface = 1 << 20;

int rbffd_cylinder_forces(rbffd_ctx *ctx, const rbffd_cloud *cloud, const rbffd_ops *ops, const double *u,
                          const double *p, const double *centre, double diameter, double mu, int nsurf, double rho,
                          double u_ref, double *force, double *coef, double *traction, int64_t *bad_query,
                          void *hip_stream)
{
    if (bad_query) *bad_query = -1;
    if (!ctx || !ops || !u || !p || !centre || !force) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    RB_CHECK(check_cloud(cloud));
    if (cloud->dim != 2 || ops->dim != 2) return fail(RBFFD_E_ARG, "cylinder forces are defined for 2D clouds");
    if (cloud->n != ops->n) return fail(RBFFD_E_ARG, "the cloud and the operators differ in size");
    if (nsurf < 4 || (nsurf & 1) || nsurf > kMaxSurface)
        return fail(RBFFD_E_ARG, "nsurf must be even, at least 4 and at most " + std::to_string(kMaxSurface));
    if (!(diameter > 0.0) || !std::isfinite(diameter) || !std::isfinite(centre[0]) || !std::isfinite(centre[1]) ||
        !std::isfinite(mu))
        return fail(RBFFD_E_ARG, "the centre, diameter and viscosity must be finite, the diameter positive");
    if (coef && !(rho > 0.0 && std::isfinite(rho) && u_ref != 0.0 && std::isfinite(u_ref)))
        return fail(RBFFD_E_ARG, "coefficients need a positive density and a nonzero reference speed");
    const int q = ops->q, k = ops->k, phs = ops->phs;
    const int m = (k + 1) * (k + 2) / 2;
    if (q + m > 128) return fail(RBFFD_E_ARG, "collocation systems larger than 128 (q + m) are not supported");
    RB_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = ops->n, ns = nsurf;
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_fld = up(sizeof(double) * 5 * n), b_q = up(sizeof(double) * 2 * ns),
                 b_cs = up(sizeof(double) * 2 * ns), b_fs = up(sizeof(double) * 5 * ns),
                 b_nbr = up(sizeof(int32_t) * ns * q), b_w = up(sizeof(double) * ns * q),
                 b_res = up(sizeof(double) * 2 + sizeof(int64_t));
    const size_t total = b_fld + b_q + b_cs + b_fs + b_nbr + b_w + b_res;
    char *base = nullptr;
    RB_CHECK(dev_alloc(ctx, (void **)&base, total));
    double *fld = (double *)base;
    double *qxyz = (double *)(base + b_fld);
    double *cs = (double *)(base + b_fld + b_q);
    double *fs = (double *)(base + b_fld + b_q + b_cs);
    int32_t *nbr = (int32_t *)(base + b_fld + b_q + b_cs + b_fs);
    double *w = (double *)(base + b_fld + b_q + b_cs + b_fs + b_nbr);
    double *res = (double *)(base + b_fld + b_q + b_cs + b_fs + b_nbr + b_w);
    int64_t *bad_dev = (int64_t *)(res + 2);
    // uniform surface points t_j = 2 pi j / nsurf (host cos and sin)
    const double r = 0.5 * diameter;
    std::vector<double> hq(2 * ns), hcs(2 * ns);
    for (int64_t j = 0; j < ns; ++j) {
        const double t = 2.0 * M_PI * (double)j / (double)nsurf;
        const double c = std::cos(t), sn = std::sin(t);
        const double dx = r * c, dy = r * sn;
        hq[2 * j] = centre[0] + dx;
        hq[2 * j + 1] = centre[1] + dy;
        hcs[j] = c;
        hcs[ns + j] = sn;
    }
    const double h = 2.0 * M_PI / (double)nsurf;
    double *hres = nullptr;
    int st = host_scratch(ctx, kHostMisc, sizeof(double) * 3, (void **)&hres);
    hipError_t e = hipSuccess;
    if (st == RBFFD_OK) e = hipMemcpyAsync(qxyz, hq.data(), sizeof(double) * 2 * ns, hipMemcpyHostToDevice, s);
    if (st == RBFFD_OK && e == hipSuccess)
        e = hipMemcpyAsync(cs, hcs.data(), sizeof(double) * 2 * ns, hipMemcpyHostToDevice, s);
    if (st == RBFFD_OK && e == hipSuccess) e = hipMemcpyAsync(fld, p, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) st = hip_fail(e, "cylinder forces");
    // strain rates at the nodes: du/dx, du/dy, dv/dx, dv/dy
    if (st == RBFFD_OK) st = apply_op(ctx, ops, 0, u, fld + n, s);
    if (st == RBFFD_OK) st = apply_op(ctx, ops, 1, u, fld + 2 * n, s);
    if (st == RBFFD_OK) st = apply_op(ctx, ops, 0, u + n, fld + 3 * n, s);
    if (st == RBFFD_OK) st = apply_op(ctx, ops, 1, u + n, fld + 4 * n, s);
    // pressure and strain rates at the surface points (a periodic cloud takes
    // the periodic interpolation, which reports a singular system itself)
    const bool periodic = is_periodic(cloud);
    if (st == RBFFD_OK && periodic) {
        rbffd_stencil_opts o;
        o.phs_power = phs;
        o.poly_degree = k;
        o.q = q;
        st = interpolate_periodic(ctx, cloud, &o, q, ns, qxyz, 5, fld, fs, nbr, w, bad_query, s);
    } else {
        if (st == RBFFD_OK) st = launch_knn_points(ctx, 2, n, cloud->xyz, ns, qxyz, q, nbr, s);
        if (st == RBFFD_OK)
            st = launch_interp(ctx, 2, n, cloud->xyz, ns, qxyz, q, nbr, k, phs, w, bad_dev, 5, fld, fs, s);
    }
    if (st == RBFFD_OK) st = launch_surface_traction(nsurf, fs, cs, mu, r * (h / 3.0), traction, res, s);
    if (st == RBFFD_OK) {
        e = hipMemcpyAsync(hres, res, sizeof(double) * 2 + sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    } else {
        (void)hipStreamSynchronize(s);
    }
    dev_free(ctx, base, total);
    if (st != RBFFD_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "cylinder forces");
    int64_t bad = INT64_MAX;
    if (!periodic) std::memcpy(&bad, hres + 2, sizeof(bad));
    if (bad != INT64_MAX) {
        if (bad_query) *bad_query = bad;
        return fail(RBFFD_E_SINGULAR, "singular interpolation system at surface point " + std::to_string(bad));
    }
    force[0] = hres[0];
    force[1] = hres[1];
    if (coef) {
        const double den = 0.5 * rho * u_ref * u_ref * diameter;
        coef[0] = force[0] / den;
        coef[1] = force[1] / den;
    }
    return RBFFD_OK;
}

int poisson_solve(rbffd_ctx *ctx, const rbffd_ops *ops, const double *rhs, double *x,
                  const rbffd_krylov_opts *opts, rbffd_krylov_stats *stats, void *hip_stream)
{
    if (!ctx || !ops || !rhs || !x || !opts) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    if (!(opts->tol >= 0.0) || opts->max_iter < 0) return fail(RBFFD_E_ARG, "bad Krylov options");
    if (opts->precision != RBFFD_FP64 && opts->precision != RBFFD_FP32_IR && opts->precision != RBFFD_FP32_MATRIX)
        return fail(RBFFD_E_ARG, "unknown precision");
    if (opts->precision != RBFFD_FP64 && !ops->pval32)
        return fail(RBFFD_E_ARG, "operators were assembled without FP32 copies");
    RB_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)hip_stream;
    KrylovResult res;
    int refine = 0;
    int st;
    if (opts->preconditioner != RBFFD_PREC_JACOBI && opts->preconditioner != RBFFD_PREC_BLOCK64)
        return fail(RBFFD_E_ARG, "unknown preconditioner");
    const bool block = opts->preconditioner == RBFFD_PREC_BLOCK64;
    if (block) RB_CHECK(ensure_block_inverse(ops, s));
    if (block && opts->precision == RBFFD_FP64)
        st = bicgstab_block(ctx, ops->n, ops->q, cols_of(ops), ops->pval, binv_of(ops), rhs, x, opts->tol,
                            opts->max_iter, &res, s);
    else if (opts->precision == RBFFD_FP64)
        st = bicgstab(ctx, ops->n, ops->q, cols_of(ops), ops->pval, ops->pdinv, 1, rhs, x, opts->tol,
                      opts->max_iter, &res, s);
    else
        st = bicgstab_mixed(ctx, opts->precision, ops->n, ops->q, cols_of(ops), ops->pval, ops->pval32, ops->pdinv32,
                            ops->pdinv, block ? binv_of(ops) : kNoBlockInv, 1, rhs, x, opts->tol, opts->max_iter, &res,
                            &refine, s);
    if (st != RBFFD_OK) return st;
    double rr = 0.0;
    RB_CHECK(residual_norms(ctx, ops->n, ops->q, cols_of(ops), ops->pval, 1, rhs, x, &rr, s));
    if (stats) {
        stats->iters = res.iters[0];
        stats->status = res.status[0];
        stats->refinements = refine;
        stats->fp64_fallback = res.fp64_fallback ? 1 : 0;
        stats->relres = rr;
    }
    if (res.status[0] != RBFFD_OK)
        return fail(res.status[0], "poisson_solve did not converge in " + std::to_string(res.iters[0]) +
                                       " iterations (relres " + std::to_string(rr) + ")");
    return RBFFD_OK;
}

int rbffd_krylov_kernel_times(rbffd_ctx *ctx, const rbffd_ops *ops, const double *rhs, double *x, int reps,
                              double *us, void *hip_stream)
{
    if (!ctx || !ops || !rhs || !x || !us) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    if (reps < 1) return fail(RBFFD_E_ARG, "reps must be >= 1");
    RB_HIP(hipSetDevice(ctx->device));
    return krylov_kernel_times(ctx, ops->n, ops->q, cols_of(ops), ops->pval, ops->pdinv, rhs, x, reps, us,
                               (hipStream_t)hip_stream);
}

int poisson_solve_noalloc(const rbffd_ops *ops, const double *rhs, double *x, const rbffd_krylov_opts *opts,
                          rbffd_krylov_stats *stats, void *hip_stream)
{
    if (!ops || !rhs || !x || !opts) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    if (!(opts->tol >= 0.0) || opts->max_iter < 0) return fail(RBFFD_E_ARG, "bad Krylov options");
    if (opts->precision != RBFFD_FP64 || opts->preconditioner != RBFFD_PREC_JACOBI)
        return fail(RBFFD_E_ARG, "poisson_solve_noalloc takes precision RBFFD_FP64 and the Jacobi preconditioner");
    if (pad64(ops->n) > RBFFD_NOALLOC_MAX_N)
        return fail(RBFFD_E_ARG, "poisson_solve_noalloc: " + std::to_string(ops->n) +
                                     " rows exceed RBFFD_NOALLOC_MAX_N (" + std::to_string(RBFFD_NOALLOC_MAX_N) + ")");
    RB_HIP(hipSetDevice(ops->ctx->device));
    KrylovResult res;
    double rr = 0.0;
    RB_CHECK(poisson_solve_noalloc_impl(ops->ctx->device, ops->n, ops->q, cols_of(ops), ops->pval, ops->pdinv, rhs, x,
                                        opts->tol, opts->max_iter, &res, &rr, (hipStream_t)hip_stream));
    if (stats) {
        stats->iters = res.iters[0];
        stats->status = res.status[0];
        stats->refinements = 0;
        stats->fp64_fallback = 0;
        stats->relres = rr;
    }
    if (res.status[0] != RBFFD_OK)
        return fail(res.status[0], "poisson_solve_noalloc did not converge in " + std::to_string(res.iters[0]) +
                                       " iterations (relres " + std::to_string(rr) + ")");
    return RBFFD_OK;
}

int poisson_solve_batched(rbffd_ctx *ctx, int count, const rbffd_ops *const *ops, const double *const *rhs,
                          double *const *x, const rbffd_krylov_opts *opts, rbffd_krylov_stats *stats,
                          void *hip_stream)
{
    if (!ctx || !ops || !rhs || !x || !opts) return fail(RBFFD_E_ARG, "NULL argument");
    if (count < 1) return fail(RBFFD_E_ARG, "count must be >= 1");
    if (!(opts->tol >= 0.0) || opts->max_iter < 0) return fail(RBFFD_E_ARG, "bad Krylov options");
    if (opts->precision != RBFFD_FP64 && opts->precision != RBFFD_FP32_MATRIX)
        return fail(RBFFD_E_ARG, "batched solves run in RBFFD_FP64 or RBFFD_FP32_MATRIX");
    if (opts->preconditioner != RBFFD_PREC_JACOBI && opts->preconditioner != RBFFD_PREC_BLOCK64)
        return fail(RBFFD_E_ARG, "unknown preconditioner");
    const bool block = opts->preconditioner == RBFFD_PREC_BLOCK64;
    const bool f32 = opts->precision == RBFFD_FP32_MATRIX;
    std::vector<BatchSystem> sys((size_t)count);
    for (int j = 0; j < count; ++j) {
        if (!ops[j] || !rhs[j] || !x[j])
            return fail(RBFFD_E_ARG, "NULL operator, right-hand side or solution of system " + std::to_string(j));
        if (!ops[j]->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
        if (f32 && !ops[j]->pval32)
            return fail(RBFFD_E_ARG, "system " + std::to_string(j) + " was assembled without FP32 copies");
        if (block) {
            RB_HIP(hipSetDevice(ctx->device));
            RB_CHECK(ensure_block_inverse(ops[j], (hipStream_t)hip_stream));
        }
        sys[j] = BatchSystem{ops[j]->n, ops[j]->q, cols_of(ops[j]), ops[j]->pval, ops[j]->pdinv, rhs[j], x[j],
                             block ? binv_of(ops[j]) : kNoBlockInv, f32 ? ops[j]->pval32 : nullptr};
    }
    RB_HIP(hipSetDevice(ctx->device));
    std::vector<int> iters((size_t)count), status((size_t)count);
    std::vector<double> relres((size_t)count);
    RB_CHECK(bicgstab_batched(ctx, count, sys.data(), opts->tol, opts->max_iter, iters.data(), status.data(),
                              relres.data(), (hipStream_t)hip_stream));
    int first = RBFFD_OK;
    for (int j = 0; j < count; ++j) {
        if (stats) {
            stats[j].iters = iters[j];
            stats[j].status = status[j];
            stats[j].refinements = 0;
            stats[j].fp64_fallback = 0;
            stats[j].relres = relres[j];
        }
        if (status[j] != RBFFD_OK && first == RBFFD_OK) first = status[j];
    }
    if (first != RBFFD_OK) return fail(first, "a batched system did not converge");
    return RBFFD_OK;
}

int rbffd_server_create(rbffd_ctx *ctx, rbffd_server **out)
{
    if (!ctx || !out) return fail(RBFFD_E_ARG, "NULL argument");
    rbffd::Server *impl = nullptr;
    RB_CHECK(server_create(ctx, &impl));
    *out = new rbffd_server{ctx, impl};
    ctx->servers.insert(*out);
    return RBFFD_OK;
}

int rbffd_server_destroy(rbffd_server *sv)
{
    if (!sv) return RBFFD_OK;
    if (sv->ctx) {
        (void)hipSetDevice(sv->ctx->device);
        sv->ctx->servers.erase(sv);
        server_destroy(sv->impl);
    }
    delete sv;
    return RBFFD_OK;
}

int rbffd_server_submit(rbffd_server *sv, const rbffd_ops *ops, const double *rhs, double *x,
                        const rbffd_krylov_opts *opts, int64_t *ticket)
{
    if (!sv || !ops || !rhs || !x || !opts || !ticket) return fail(RBFFD_E_ARG, "NULL argument");
    if (!sv->impl) return fail(RBFFD_E_ARG, "the server's context was destroyed");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    if (!(opts->tol >= 0.0) || opts->max_iter < 1) return fail(RBFFD_E_ARG, "bad Krylov options");
    if (opts->precision != RBFFD_FP64 && opts->precision != RBFFD_FP32_MATRIX)
        return fail(RBFFD_E_ARG, "served solves run in RBFFD_FP64 or RBFFD_FP32_MATRIX");
    if (opts->preconditioner != RBFFD_PREC_JACOBI && opts->preconditioner != RBFFD_PREC_BLOCK64)
        return fail(RBFFD_E_ARG, "unknown preconditioner");
    const bool f32 = opts->precision == RBFFD_FP32_MATRIX;
    if (f32 && !ops->pval32) return fail(RBFFD_E_ARG, "operators were assembled without FP32 copies");
    RB_HIP(hipSetDevice(sv->ctx->device));
    if (opts->preconditioner == RBFFD_PREC_BLOCK64 && !ops->pbinv) {
        // built once, on the null stream, and finished before the server uses it
        RB_CHECK(ensure_block_inverse(ops, nullptr));
        RB_HIP(hipStreamSynchronize(nullptr));
    }
    const BatchSystem sys{ops->n, ops->q, cols_of(ops), ops->pval, ops->pdinv, rhs, x,
                          opts->preconditioner == RBFFD_PREC_BLOCK64 ? binv_of(ops) : kNoBlockInv,
                          f32 ? ops->pval32 : nullptr};
    return server_submit(sv->impl, sys, opts->tol, opts->max_iter, ticket);
}

int rbffd_server_run(rbffd_server *sv, int iterations, int *active, void *hip_stream)
{
    if (!sv || !active || iterations < 1) return fail(RBFFD_E_ARG, "bad argument");
    if (!sv->impl) return fail(RBFFD_E_ARG, "the server's context was destroyed");
    RB_HIP(hipSetDevice(sv->ctx->device));
    return server_run(sv->impl, iterations, active, (hipStream_t)hip_stream);
}

int rbffd_server_poll(rbffd_server *sv, int max, int64_t *tickets, rbffd_krylov_stats *stats, int *count)
{
    if (!sv || !tickets || !stats || !count || max < 0) return fail(RBFFD_E_ARG, "bad argument");
    if (!sv->impl) return fail(RBFFD_E_ARG, "the server's context was destroyed");
    std::vector<int> iters((size_t)std::max(max, 1)), status((size_t)std::max(max, 1));
    std::vector<double> relres((size_t)std::max(max, 1));
    RB_CHECK(server_poll(sv->impl, max, tickets, iters.data(), status.data(), relres.data(), count));
    for (int i = 0; i < *count; ++i) {
        stats[i].iters = iters[i];
        stats[i].status = status[i];
        stats[i].refinements = 0;
        stats[i].fp64_fallback = 0;
        stats[i].relres = relres[i];
    }
    return RBFFD_OK;
}

int simple_step(rbffd_ctx *ctx, const rbffd_ops *ops, double *u, double *u_prev, double *p,
                const double *u_bc, const double *p_bc, const rbffd_step_opts *opts,
                rbffd_step_stats *stats, void *hip_stream)
{
    if (!ctx || !ops || !u || !u_prev || !p || !u_bc || !opts) return fail(RBFFD_E_ARG, "NULL argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    if (ops->n_prescribed > 0 && !p_bc) return fail(RBFFD_E_ARG, "p_bc is required: the cloud has prescribed-pressure points");
    if (!(opts->rho > 0.0) || !(opts->mu >= 0.0) || !(opts->dt > 0.0) || !std::isfinite(opts->dt))
        return fail(RBFFD_E_ARG, "rho, mu, dt must be positive and finite");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(opts->force[d])) return fail(RBFFD_E_ARG, "the body force must be finite");
    if (!(opts->alpha[0] != 0.0) || !std::isfinite(opts->alpha[1]) || !std::isfinite(opts->alpha[2]))
        return fail(RBFFD_E_ARG, "bad BDF coefficients");
    if (opts->max_outer < 1 || opts->max_krylov < 1 || !(opts->tol_krylov >= 0.0) || !(opts->tol_outer >= 0.0))
        return fail(RBFFD_E_ARG, "bad iteration limits or tolerances");
    if (opts->precision != RBFFD_FP64 && opts->precision != RBFFD_FP32_IR && opts->precision != RBFFD_FP32_MATRIX)
        return fail(RBFFD_E_ARG, "unknown precision");
    if (opts->precision != RBFFD_FP64 && !ops->pval32)
        return fail(RBFFD_E_ARG, "operators were assembled without FP32 copies");
    if (opts->preconditioner != RBFFD_PREC_JACOBI && opts->preconditioner != RBFFD_PREC_BLOCK64)
        return fail(RBFFD_E_ARG, "unknown preconditioner");
    RB_HIP(hipSetDevice(ctx->device));
    rbffd_step_stats local{};
    int st = run_step(ctx, ops, u, u_prev, p, u_bc, p_bc, opts, stats ? stats : &local, (hipStream_t)hip_stream);
    return st;
}

int simple_step_batched(rbffd_ctx *ctx, int count, const rbffd_ops *const *ops, double *const *u,
                        double *const *u_prev, double *const *p, const double *const *u_bc,
                        const double *const *p_bc, const rbffd_step_opts *opts, rbffd_step_stats *stats,
                        void *hip_stream)
{
    if (!ctx || !ops || !u || !u_prev || !p || !u_bc || !p_bc || !opts || !stats)
        return fail(RBFFD_E_ARG, "NULL argument");
    if (count < 1) return fail(RBFFD_E_ARG, "count must be >= 1");
    std::set<const rbffd_ops *> seen;
    for (int j = 0; j < count; ++j) {
        const std::string at = " (cloud " + std::to_string(j) + ")";
        const rbffd_ops *op = ops[j];
        const rbffd_step_opts *o = &opts[j];
        if (!op || !u[j] || !u_prev[j] || !p[j] || !u_bc[j]) return fail(RBFFD_E_ARG, "NULL argument" + at);
        if (!op->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed" + at);
        if (op->ctx != ctx) return fail(RBFFD_E_ARG, "operators of another context" + at);
        if (!seen.insert(op).second) return fail(RBFFD_E_ARG, "the same operators appear twice" + at);
        if (op->n_prescribed > 0 && !p_bc[j])
            return fail(RBFFD_E_ARG, "p_bc is required: the cloud has prescribed-pressure points" + at);
        if (op->n_symmetry > 0) return fail(RBFFD_E_ARG, "clouds with symmetry points step one at a time" + at);
        if (!(o->rho > 0.0) || !(o->mu >= 0.0) || !(o->dt > 0.0) || !std::isfinite(o->dt))
            return fail(RBFFD_E_ARG, "rho, mu, dt must be positive and finite" + at);
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(o->force[d])) return fail(RBFFD_E_ARG, "the body force must be finite" + at);
        if (!(o->alpha[0] != 0.0) || !std::isfinite(o->alpha[1]) || !std::isfinite(o->alpha[2]))
            return fail(RBFFD_E_ARG, "bad BDF coefficients" + at);
        if (o->max_outer < 1 || o->max_krylov < 1 || !(o->tol_krylov >= 0.0) || !(o->tol_outer >= 0.0))
            return fail(RBFFD_E_ARG, "bad iteration limits or tolerances" + at);
        if (o->precision != RBFFD_FP64) return fail(RBFFD_E_ARG, "batched steps run in FP64" + at);
        if (o->preconditioner != RBFFD_PREC_JACOBI && o->preconditioner != RBFFD_PREC_BLOCK64)
            return fail(RBFFD_E_ARG, "unknown preconditioner" + at);
    }
    RB_HIP(hipSetDevice(ctx->device));
    return run_step_batched(ctx, count, ops, u, u_prev, p, u_bc, p_bc, opts, stats, (hipStream_t)hip_stream);
}

int rbffd_convdiff_lambda(rbffd_ctx *ctx, const rbffd_ops *ops, const double *u0, double rho,
                          double mu, int iters, double *lambda_out, void *hip_stream)
{
    if (!ctx || !ops || !u0 || !lambda_out || iters < 1) return fail(RBFFD_E_ARG, "bad argument");
    if (!ops->ctx) return fail(RBFFD_E_ARG, "the operators' context was destroyed");
    RB_HIP(hipSetDevice(ctx->device));
    return convdiff_lambda(ctx, ops, u0, rho, mu, iters, lambda_out, (hipStream_t)hip_stream);
}

}  // extern "C"
