// C-ABI entry points of raybornhf: argument validation, geometry cache, workspace, and the
// orchestration of one frequency step (Section 3 and Section 6.3.2(a) of the paper).
#include "rb_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <vector>

rb_status rb_launch_gather_mask(rb_ctx *ctx, const double *c, double *cq);
rb_status rb_launch_rough_part(rb_ctx *ctx, const double *cq, const float *n_s, double c0,
                               double w, float *sv);
rb_status rb_launch_backproject_finish_acc(rb_ctx *ctx, int mblocks, const float *parts,
                                           const double *c_mask, double omega, double d_omega,
                                           double *dm_acc);
rb_status rb_launch_zero_f64(rb_ctx *ctx, double *x, int n);
rb_status rb_launch_update(rb_ctx *ctx, const double *cq, const double *dm, double tau,
                           double *c_new);
rb_status rb_launch_commit(rb_ctx *ctx, const double *c_new, double *c, const int32_t *flag);
rb_status rb_launch_note_fail(rb_ctx *ctx, int step);

rb_status rb_fail(rb_ctx *ctx, rb_status st, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return st;
}

void rb_prof_begin(rb_ctx *ctx, int stage) {
    if (!ctx->prof || ctx->n_ev >= rb_ctx::kMaxEv) return;
    int i = ctx->n_ev;
    if (i >= ctx->n_ev_created) {
        if (hipEventCreate(&ctx->ev[i][0]) != hipSuccess ||
            hipEventCreate(&ctx->ev[i][1]) != hipSuccess) {
            ctx->prof = false;
            return;
        }
        ctx->n_ev_created = i + 1;
    }
    ctx->ev_stage[i] = stage;
    (void)hipEventRecord(ctx->ev[i][0], ctx->stream);
}

void rb_prof_end(rb_ctx *ctx) {
    if (!ctx->prof || ctx->n_ev >= rb_ctx::kMaxEv) return;
    (void)hipEventRecord(ctx->ev[ctx->n_ev][1], ctx->stream);
    ctx->n_ev++;
}

rb_status rb_arena_reserve(rb_ctx *ctx, rb_arena *a, size_t bytes) {
    if (bytes <= a->cap) return RB_OK;
    if (ctx->fixed)
        return rb_fail(ctx, RB_ENOMEM,
                       "the call needs %zu workspace bytes, %zu were reserved (rb_reserve)", bytes,
                       a->cap);
    if (ctx->capturing) {  // no allocation inside a graph capture: grow it and capture again
        a->want = std::max(a->want, bytes);
        return RB_ERETRY;
    }
    ++ctx->gen;
    if (a->base) {
        // kernels queued on the stream may still read the old block
        RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        RB_HIP(ctx, hipFree(a->base));
        a->base = nullptr;
        a->cap = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return rb_fail(ctx, RB_ENOMEM, "workspace allocation of %zu bytes failed", bytes);
    }
    a->base = static_cast<char *>(p);
    a->cap = bytes;
    return RB_OK;
}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

rb_status rb_check_grid(rb_ctx *ctx, const rb_grid *g) {
    if (!g) return rb_fail(ctx, RB_EINVAL, "grid is NULL");
    if (g->nx < 4 || g->ny < 4) return rb_fail(ctx, RB_EINVAL, "grid must be at least 4x4");
    if ((int64_t)g->nx * g->ny > (int64_t)1 << 30 || g->nx > 65535)
        return rb_fail(ctx, RB_EINVAL, "grid too large (at most 2^30 nodes, 65535 per row)");
    if (!finite_pos(g->dx) || !std::isfinite(g->x0) || !std::isfinite(g->y0) ||
        !finite_pos(g->mask_radius))
        return rb_fail(ctx, RB_EINVAL, "grid spacing, origin and mask radius must be finite");
    return RB_OK;
}

rb_status rb_check_ring(rb_ctx *ctx, const rb_grid *g, const rb_ring *r) {
    if (!r) return rb_fail(ctx, RB_EINVAL, "ring is NULL");
    if (r->n < 3 || r->n > 65536) return rb_fail(ctx, RB_EINVAL, "ring needs 3..65536 elements");
    if (!finite_pos(r->radius) || !std::isfinite(r->psi0))
        return rb_fail(ctx, RB_EINVAL, "ring radius must be positive");
    if (g->mask_radius >= r->radius)
        return rb_fail(ctx, RB_EINVAL, "imaging mask must lie inside the ring");
    double xmax = g->x0 + (g->nx - 1) * g->dx, ymax = g->y0 + (g->ny - 1) * g->dx;
    if (g->x0 > -r->radius || g->y0 > -r->radius || xmax < r->radius || ymax < r->radius)
        return rb_fail(ctx, RB_EINVAL, "the grid must cover the ring");
    return RB_OK;
}

rb_status rb_check_trace(rb_ctx *ctx, const rb_trace_params *tp) {
    if (!tp) return rb_fail(ctx, RB_EINVAL, "trace parameters are NULL");
    if (tp->n_rays < 2 || tp->n_rays > 2048)
        return rb_fail(ctx, RB_EINVAL, "n_rays must be in 2..2048");
    if (tp->max_steps < 1 || tp->max_steps > 100000)
        return rb_fail(ctx, RB_EINVAL, "max_steps must be in 1..100000");
    if ((uint64_t)tp->n_rays * (uint64_t)(tp->max_steps + 1) * 2 >= ((uint64_t)1 << 32))
        return rb_fail(ctx, RB_EINVAL, "n_rays * (max_steps + 1) too large for triangle ids");
    if (!finite_pos(tp->ds) || !finite_pos(tp->c0))
        return rb_fail(ctx, RB_EINVAL, "ds and c0 must be positive");
    return RB_OK;
}

static int64_t mask_list(const rb_grid *g, std::vector<int32_t> *idx, std::vector<int32_t> *map) {
    int64_t n = 0;
    double r2 = g->mask_radius * g->mask_radius;
    if (map) map->assign((size_t)g->nx * g->ny, -1);
    for (int j = 0; j < g->ny; ++j) {
        double y = g->y0 + j * g->dx;
        for (int i = 0; i < g->nx; ++i) {
            double x = g->x0 + i * g->dx;
            if (x * x + y * y <= r2) {
                if (idx) idx->push_back(j * g->nx + i);
                if (map) (*map)[(size_t)j * g->nx + i] = (int32_t)n;
                ++n;
            }
        }
    }
    return n;
}

rb_status rb_prepare_grid(rb_ctx *ctx, const rb_grid *g) {
    if (ctx->have_grid && std::memcmp(&ctx->grid, g, sizeof(rb_grid)) == 0) return RB_OK;
    if (ctx->fixed)
        return rb_fail(ctx, RB_EINVAL, "the grid differs from the one given to rb_reserve");
    if (ctx->capturing) return rb_fail(ctx, RB_EINVAL, "grid changed inside a graph capture");
    ++ctx->gen;
    std::vector<int32_t> idx, map;
    int64_t n = mask_list(g, &idx, &map);
    if (n < 1) return rb_fail(ctx, RB_EINVAL, "the imaging mask holds no grid node");
    RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->d_mask_index) RB_HIP(ctx, hipFree(ctx->d_mask_index));
    if (ctx->d_qmap) RB_HIP(ctx, hipFree(ctx->d_qmap));
    if (ctx->d_qrow) RB_HIP(ctx, hipFree(ctx->d_qrow));
    ctx->d_mask_index = nullptr;
    ctx->d_qmap = nullptr;
    ctx->d_qrow = nullptr;
    ctx->have_grid = false;
    RB_HIP(ctx, hipMalloc(&ctx->d_mask_index, n * sizeof(int32_t)));
    RB_HIP(ctx, hipMalloc(&ctx->d_qmap, map.size() * sizeof(int32_t)));
    RB_HIP(ctx, hipMemcpy(ctx->d_mask_index, idx.data(), n * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    RB_HIP(ctx, hipMemcpy(ctx->d_qmap, map.data(), map.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    // the mask is a disc: each row's nodes are one run of consecutive indices
    std::vector<int2> qrow((size_t)g->ny, make_int2(1, 0));  // empty: first > last
    for (int j = 0; j < g->ny; ++j) {
        int lo = -1, hi = -1;
        for (int i = 0; i < g->nx; ++i)
            if (map[(size_t)j * g->nx + i] >= 0) {
                if (lo < 0) lo = i;
                hi = i;
            }
        if (lo >= 0)
            qrow[j] = make_int2((int)((uint32_t)lo | ((uint32_t)hi << 16)),
                                map[(size_t)j * g->nx + lo] - lo);
    }
    RB_HIP(ctx, hipMalloc(&ctx->d_qrow, qrow.size() * sizeof(int2)));
    RB_HIP(ctx, hipMemcpy(ctx->d_qrow, qrow.data(), qrow.size() * sizeof(int2),
                          hipMemcpyHostToDevice));
    int imin = g->nx, imax = -1, jmin = g->ny, jmax = -1;
    for (int32_t p : idx) {
        int i = p % g->nx, j = p / g->nx;
        imin = std::min(imin, i);
        imax = std::max(imax, i);
        jmin = std::min(jmin, j);
        jmax = std::max(jmax, j);
    }
    ctx->tile_i0 = imin;
    ctx->tile_j0 = jmin;
    ctx->tiles_x = (imax - imin + RB_WALK_TX) / RB_WALK_TX;
    ctx->tiles_y = (jmax - jmin + RB_WALK_TY) / RB_WALK_TY;
    ctx->grid = *g;
    ctx->n_mask = n;
    ctx->have_grid = true;
    return RB_OK;
}

static rb_status check_tables(rb_ctx *ctx, const rb_tables *tb, int n, int64_t n_mask) {
    if (!tb) return rb_fail(ctx, RB_EINVAL, "tables are NULL");
    if (tb->n != n || tb->n_mask != n_mask)
        return rb_fail(ctx, RB_EINVAL, "tables sized [%d][%d], expected [%d][%lld]", tb->n,
                       tb->n_mask, n, (long long)n_mask);
    if (!tb->T || !tb->A || !tb->ux || !tb->uy || !tb->flags || !tb->rx_T || !tb->rx_A ||
        !tb->rx_flags)
        return rb_fail(ctx, RB_EINVAL, "a table pointer is NULL");
    return RB_OK;
}

static rb_status check_green(rb_ctx *ctx, const rb_green *gr) {
    if (!gr) return rb_fail(ctx, RB_EINVAL, "green operands are NULL");
    if (gr->n < 1 || gr->n_mask < 1 || !gr->G || !gr->H)
        return rb_fail(ctx, RB_EINVAL, "green operands incomplete");
    if (!rb_prec_valid(gr->prec))
        return rb_fail(ctx, RB_EINVAL, "unknown operand precision %d", (int)gr->prec);
    if (gr->prec != RB_F32 && !gr->scales)
        return rb_fail(ctx, RB_EINVAL, "16-bit operands need their per-row scales");
    return RB_OK;
}

static rb_status check_step_args(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                                 const rb_trace_params *tp, const double *c, int32_t smooth_w,
                                 int32_t n_omega, const double *omega, const double *d_omega,
                                 const float *data, double tau, rb_mode mode, rb_prec prec) {
    RB_TRY(rb_check_grid(ctx, grid));
    RB_TRY(rb_check_ring(ctx, grid, ring));
    RB_TRY(rb_check_trace(ctx, tp));
    if (!c || !data) return rb_fail(ctx, RB_EINVAL, "c and data must be device pointers");
    if (n_omega < 1 || !omega || !d_omega)
        return rb_fail(ctx, RB_EINVAL, "need at least one frequency (host arrays)");
    for (int k = 0; k < n_omega; ++k)
        if (!finite_pos(omega[k]) || !finite_pos(d_omega[k]))
            return rb_fail(ctx, RB_EINVAL, "frequencies and spacings must be positive");
    if (smooth_w < 1 || (smooth_w & 1) == 0)
        return rb_fail(ctx, RB_EINVAL, "smoothing window must be odd and >= 1");
    if (!std::isfinite(tau)) return rb_fail(ctx, RB_EINVAL, "tau must be finite");
    if (mode != RB_RAY_BORN && mode != RB_RAY_ONLY)
        return rb_fail(ctx, RB_EINVAL, "unknown mode");
    if (!rb_prec_valid(prec)) return rb_fail(ctx, RB_EINVAL, "unknown operand precision");
    return RB_OK;
}

// Scratch of the allocation-free back-projection (rb_backproject_noalloc): one file-scope
// device array per GPU, held by the loaded code object until the process ends. In host code
// `scratch` names a host-side stand-in; its device address on each GPU comes from
// hipGetSymbolAddress (once per device, at the first rb_create there) and only that address
// is used.
static __device__ __align__(256) char scratch[RB_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// With ctx->device current: record the device address of `scratch` on this device.
static rb_status scratch_setup(rb_ctx *ctx) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device >= kMaxDevices) return RB_OK;  // the allocation-free form reports it
    if (g_scratch_ptr[ctx->device]) return RB_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return RB_EDEVICE;
    }
    g_scratch_ptr[ctx->device] = p;
    return RB_OK;
}

static void *scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

// Low parts of a split operand's H (they follow the three components' planes), or NULL.
static const void *h_low(const rb_green *gr) {
    if (!rb_prec_split(gr->prec)) return nullptr;
    return static_cast<const char *>(gr->H) +
           6 * (size_t)gr->n_mask * rb_lp_pad(gr->n) * sizeof(uint16_t);
}

// Workspace of rb_build_green with 16-bit operands: the tables' per-row amplitude maxima.
static size_t green_ws_bytes(int n) { return rb_align((size_t)2 * n * sizeof(unsigned int)); }

// Workspace bytes of the standalone contractions (rb_born_adjoint, rb_backproject).
static size_t adjoint_ws_bytes(int n, int nm, bool lp) {
    if (!lp)
        return rb_align((size_t)2 * rb_rowred_mblocks(n) * nm * sizeof(float)) +
               rb_align((size_t)2 * n * n * sizeof(float));
    const size_t np = (size_t)rb_lp_pad(n);
    return rb_align((size_t)2 * rb_rowred_lp_mblocks(n) * nm * sizeof(float)) +
           rb_align(2 * (size_t)n * np * sizeof(uint16_t)) + rb_align(8) +
           rb_align(2 * (size_t)nm * np * sizeof(uint16_t));
}

static size_t backproject_ws_bytes(int n, int nm, bool lp) {
    const int mb = lp ? rb_rowred_lp_mblocks(n) : rb_rowred_mblocks(n);
    const size_t nnp = (size_t)n * rb_lp_pad(n);
    return rb_align((size_t)2 * mb * nm * sizeof(float)) + rb_align(2 * nnp * sizeof(uint16_t)) +
           rb_align(8) + rb_align(2 * (size_t)n * n * sizeof(float));
}

// Bytes of the step arena for N transducers, nm mask nodes and P grid nodes.
static size_t step_arena_bytes(int N, int nm, size_t P, rb_prec prec);

struct GeomSizes {
    int64_t nm = 0;
    size_t tiles = 0;
};

static GeomSizes geom_sizes(const rb_grid *grid) {
    GeomSizes gs;
    std::vector<int32_t> idx;
    gs.nm = mask_list(grid, &idx, nullptr);
    if (gs.nm < 1) return gs;
    int imin = grid->nx, imax = -1, jmin = grid->ny, jmax = -1;
    for (int32_t p : idx) {
        const int i = p % grid->nx, j = p / grid->nx;
        imin = std::min(imin, i);
        imax = std::max(imax, i);
        jmin = std::min(jmin, j);
        jmax = std::max(jmax, j);
    }
    gs.tiles = (size_t)((imax - imin + RB_WALK_TX) / RB_WALK_TX) *
               ((jmax - jmin + RB_WALK_TY) / RB_WALK_TY);
    return gs;
}

static int device_cus() {
    int n_cu = 256, dev = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipGetLastError();
    return n_cu > 0 ? n_cu : 256;
}

// Largest scratch arena any entry point takes for this geometry (any operand precision).
static size_t ws_need(const rb_grid *grid, const rb_ring *ring, const rb_trace_params *tp,
                      const GeomSizes &gs, size_t sample_budget, int n_cu) {
    const int N = ring->n, nm = (int)gs.nm;
    const size_t P = (size_t)grid->nx * grid->ny;
    size_t ws = 2 * rb_align(P * sizeof(double));  // smoothing (both maps when lossy)
    ws = std::max(ws, rb_trace_ws_bytes(grid, ring, tp, gs.nm, gs.tiles, sample_budget));
    ws = std::max(ws, rb_forward_ws_bytes(N, nm));
    ws = std::max(ws, rb_forward_lp_ws_bytes(N, nm, std::max(8, n_cu)));
    ws = std::max(ws, green_ws_bytes(N));
    for (int lp = 0; lp < 2; ++lp) {
        ws = std::max(ws, adjoint_ws_bytes(N, nm, lp != 0));
        ws = std::max(ws, backproject_ws_bytes(N, nm, lp != 0));
    }
    return ws;
}

extern "C" {

rb_status rb_create(rb_ctx **out, int device, void *hip_stream) {
    if (!out) return RB_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return RB_EDEVICE;
    }
    if (hipSetDevice(device) != hipSuccess) return RB_EDEVICE;
    rb_ctx *ctx = new rb_ctx();
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    if (hipMalloc(&ctx->d_flag, RB_W_COUNT * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&ctx->d_red, RB_RED_PARTS * sizeof(float)) != hipSuccess ||
        hipHostMalloc(&ctx->h_flag, RB_W_COUNT * sizeof(int32_t), hipHostMallocDefault) !=
            hipSuccess ||
        hipMemset(ctx->d_flag, 0, RB_W_COUNT * sizeof(int32_t)) != hipSuccess) {
        rb_destroy(ctx);
        return RB_EDEVICE;
    }
    if (scratch_setup(ctx) != RB_OK) {
        rb_destroy(ctx);
        return RB_EDEVICE;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        ncu > 0)
        ctx->n_cu = ncu;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
        ctx->sample_budget = std::min(std::max(free_b / 4, (size_t)1 << 30), (size_t)48 << 30);
    *out = ctx;
    return RB_OK;
}

void rb_destroy(rb_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws.base) (void)hipFree(ctx->ws.base);
    if (ctx->step.base) (void)hipFree(ctx->step.base);
    if (ctx->gn.base) (void)hipFree(ctx->gn.base);
    if (ctx->d_mask_index) (void)hipFree(ctx->d_mask_index);
    if (ctx->d_qmap) (void)hipFree(ctx->d_qmap);
    if (ctx->d_qrow) (void)hipFree(ctx->d_qrow);
    if (ctx->d_flag) (void)hipFree(ctx->d_flag);
    if (ctx->d_red) (void)hipFree(ctx->d_red);
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->h_flag) (void)hipHostFree(ctx->h_flag);
    for (int i = 0; i < ctx->n_ev_created; ++i) {
        (void)hipEventDestroy(ctx->ev[i][0]);
        (void)hipEventDestroy(ctx->ev[i][1]);
    }
    delete ctx;
}

const char *rb_last_error(const rb_ctx *ctx) { return ctx ? ctx->err : "no context"; }

int64_t rb_trace_lost_nodes(const rb_ctx *ctx) { return ctx ? ctx->lost_nodes : -1; }

int64_t rb_trace_samples(const rb_ctx *ctx) { return ctx ? ctx->ray_samples : -1; }

rb_status rb_profile_enable(rb_ctx *ctx, int32_t on) {
    if (!ctx) return RB_EINVAL;
    ctx->prof = on != 0;
    ctx->n_ev = 0;
    return RB_OK;
}

rb_status rb_profile_read(rb_ctx *ctx, double *total_ms, int64_t *launches) {
    if (!ctx || !total_ms || !launches) return RB_EINVAL;
    RB_HIP(ctx, hipSetDevice(ctx->device));
    RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int s = 0; s < RB_N_STAGES; ++s) {
        total_ms[s] = 0.0;
        launches[s] = 0;
    }
    for (int i = 0; i < ctx->n_ev; ++i) {
        float ms = 0.f;
        RB_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[i][0], ctx->ev[i][1]));
        total_ms[ctx->ev_stage[i]] += ms;
        launches[ctx->ev_stage[i]] += 1;
    }
    ctx->n_ev = 0;
    return RB_OK;
}

const char *rb_stage_name(int32_t stage) {
    static const char *names[RB_N_STAGES] = {
        "smooth", "trace", "raster", "resolve", "receivers", "build_green", "forward_gemm",
        "forward_reduce", "residual", "backproject_gemm", "finish", "update"};
    return (stage >= 0 && stage < RB_N_STAGES) ? names[stage] : "unknown";
}

int64_t rb_mask_count(const rb_grid *grid) {
    if (!grid || grid->nx < 1 || grid->ny < 1 || !(grid->dx > 0)) return -1;
    return mask_list(grid, nullptr, nullptr);
}

rb_status rb_refractive_index(rb_ctx *ctx, const rb_grid *grid, const double *c, double c0,
                              int32_t w, float *n_s) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(rb_check_grid(ctx, grid));
    if (!c || !n_s) return rb_fail(ctx, RB_EINVAL, "c and n_s must be device pointers");
    if (w < 1 || (w & 1) == 0) return rb_fail(ctx, RB_EINVAL, "window must be odd and >= 1");
    if (!finite_pos(c0)) return rb_fail(ctx, RB_EINVAL, "c0 must be positive");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    return rb_launch_refractive_index(ctx, grid, c, c0, w, n_s);
}

rb_status rb_trace_rays(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                        const rb_trace_params *tp, const float *n_s, const rb_tables *out) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(rb_check_grid(ctx, grid));
    RB_TRY(rb_check_ring(ctx, grid, ring));
    RB_TRY(rb_check_trace(ctx, tp));
    if (!n_s) return rb_fail(ctx, RB_EINVAL, "n_s is NULL");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    RB_TRY(rb_prepare_grid(ctx, grid));
    RB_TRY(check_tables(ctx, out, ring->n, ctx->n_mask));
    return rb_launch_trace(ctx, grid, ring, tp, n_s, out);
}

rb_status rb_build_green(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                         const rb_green *out) {
    if (!ctx) return RB_EINVAL;
    if (!tb) return rb_fail(ctx, RB_EINVAL, "tables are NULL");
    RB_TRY(check_tables(ctx, tb, tb->n, tb->n_mask));
    RB_TRY(check_green(ctx, out));
    if (out->n != tb->n || out->n_mask != tb->n_mask)
        return rb_fail(ctx, RB_EINVAL, "green operands and tables differ in size");
    if (tb->n < 3 || tb->n_mask < 1) return rb_fail(ctx, RB_EINVAL, "empty tables");
    if (!finite_pos(omega) || !finite_pos(c0))
        return rb_fail(ctx, RB_EINVAL, "omega and c0 must be positive");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    if (out->prec != RB_F32) {
        ctx->ws.used = 0;
        RB_TRY(rb_arena_reserve(ctx, &ctx->ws, green_ws_bytes(tb->n)));
        unsigned int *rowmax = rb_carve<unsigned int>(&ctx->ws, 2 * (size_t)tb->n);
        return rb_launch_green_lp(ctx, tb, omega, c0, out, nullptr, nullptr, 1, rowmax);
    }
    return rb_launch_green(ctx, tb, omega, c0, out, nullptr, nullptr, 1);
}

rb_status rb_born_forward(rb_ctx *ctx, const rb_green *gr, const float *w, const float *delta,
                          float *d) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(check_green(ctx, gr));
    if (!d || !w != !delta)
        return rb_fail(ctx, RB_EINVAL, "d must be non-NULL, w and delta both given or both NULL");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    if (gr->prec != RB_F32) return rb_launch_forward_lp(ctx, gr, w, delta, d, nullptr);
    return rb_launch_forward(ctx, gr, w, delta, d, nullptr);
}

rb_status rb_born_adjoint(rb_ctx *ctx, const rb_green *gr, const float *w, const float *R,
                          float *grad) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(check_green(ctx, gr));
    if (!w || !R || !grad) return rb_fail(ctx, RB_EINVAL, "w, R and grad must be non-NULL");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    const bool lp = gr->prec != RB_F32;
    int mb = lp ? rb_rowred_lp_mblocks(gr->n) : rb_rowred_mblocks(gr->n);
    ctx->ws.used = 0;
    const size_t nn = (size_t)gr->n * gr->n;
    RB_TRY(rb_arena_reserve(ctx, &ctx->ws, adjoint_ws_bytes(gr->n, gr->n_mask, lp)));
    float *parts = rb_carve<float>(&ctx->ws, (size_t)2 * mb * gr->n_mask);
    if (lp) {
        // conj(G) node-major, R rounded with its range scale, the one-component contraction
        const size_t np = (size_t)rb_lp_pad(gr->n);
        uint16_t *Rp = rb_carve<uint16_t>(&ctx->ws, 2 * (size_t)gr->n * np);
        float *rscale = rb_carve<float>(&ctx->ws, 2);
        uint16_t *Gt = rb_carve<uint16_t>(&ctx->ws, 2 * (size_t)gr->n_mask * np);
        // G is never split: the split form's adjoint is the FP16 one
        const rb_prec kp = rb_prec_split(gr->prec) ? RB_F16 : gr->prec;
        RB_TRY(rb_launch_to_planar(ctx, kp, R, gr->n, Rp, rscale, gr->scales));
        RB_TRY(rb_launch_transpose_conj(ctx, gr, Gt));
        RB_TRY(rb_launch_rowred_lp(ctx, kp, gr->n, gr->n_mask, Rp, Gt, 1, parts, &mb));
        RB_TRY(rb_launch_unscale(ctx, parts, (size_t)2 * mb * gr->n_mask, rscale));
        return rb_launch_adjoint_finish(ctx, gr->n_mask, mb, parts, w, grad);
    }
    float *rsym = rb_carve<float>(&ctx->ws, 2 * nn);
    RB_TRY(rb_launch_rowred(ctx, gr->n, gr->n_mask, R, (const float *)gr->G, 1, 1, rsym, parts,
                            &mb));
    return rb_launch_adjoint_finish(ctx, gr->n_mask, mb, parts, w, grad);
}

rb_status rb_residual(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                      const float *d_born, const float *data, float *R) {
    if (!ctx) return RB_EINVAL;
    if (!tb) return rb_fail(ctx, RB_EINVAL, "tables are NULL");
    RB_TRY(check_tables(ctx, tb, tb->n, tb->n_mask));
    if (!data || !R) return rb_fail(ctx, RB_EINVAL, "data and R must be non-NULL");
    if (!finite_pos(omega) || !finite_pos(c0))
        return rb_fail(ctx, RB_EINVAL, "omega and c0 must be positive");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    return rb_launch_residual(ctx, tb, omega, c0, d_born, data, R, nullptr);
}

static rb_status check_backproject(rb_ctx *ctx, const rb_green *gr, const float *R,
                                   const double *c_mask, double omega, double d_omega,
                                   const float *dm) {
    RB_TRY(check_green(ctx, gr));
    if (!R || !c_mask || !dm) return rb_fail(ctx, RB_EINVAL, "R, c_mask and dm must be non-NULL");
    if (!finite_pos(omega) || !finite_pos(d_omega))
        return rb_fail(ctx, RB_EINVAL, "omega and d_omega must be positive");
    return RB_OK;
}

// The back-projection's contraction with its scratch (partial sums, the residual operand)
// carved from `a`, which holds at least backproject_ws_bytes: complex partial sums
// parts[2][mb][n_mask] of sum_{e,r} R[e][r] (H_e H_r + H^x_e H^x_r + H^y_e H^y_r).
static rb_status backproject_parts(rb_ctx *ctx, rb_arena *a, const rb_green *gr, const float *R,
                                   float **parts_out, int *mb_out) {
    const bool lp = gr->prec != RB_F32;
    int mb = lp ? rb_rowred_lp_mblocks(gr->n) : rb_rowred_mblocks(gr->n);
    const size_t nn = (size_t)gr->n * gr->n;
    const size_t nnp = (size_t)gr->n * rb_lp_pad(gr->n);
    a->used = 0;
    float *parts = rb_carve<float>(a, (size_t)2 * mb * gr->n_mask);
    if (lp) {
        uint16_t *Rp = rb_carve<uint16_t>(a, 2 * nnp);
        float *rscale = rb_carve<float>(a, 2);
        RB_TRY(rb_launch_to_planar(ctx, gr->prec, R, gr->n, Rp, rscale, gr->scales + gr->n));
        RB_TRY(rb_launch_rowred_lp(ctx, gr->prec, gr->n, gr->n_mask, Rp, gr->H, 3, parts, &mb,
                                   h_low(gr)));
        RB_TRY(rb_launch_unscale(ctx, parts, (size_t)2 * mb * gr->n_mask, rscale));
    } else {
        float *rsym = rb_carve<float>(a, 2 * nn);
        RB_TRY(rb_launch_rowred(ctx, gr->n, gr->n_mask, R, (const float *)gr->H, 3, 0, rsym,
                                parts, &mb));
    }
    *parts_out = parts;
    *mb_out = mb;
    return RB_OK;
}

static rb_status backproject_with(rb_ctx *ctx, rb_arena *a, const rb_green *gr, const float *R,
                                  const double *c_mask, double omega, double d_omega, float *dm,
                                  int32_t accumulate) {
    int mb = 0;
    float *parts = nullptr;
    RB_TRY(backproject_parts(ctx, a, gr, R, &parts, &mb));
    return rb_launch_backproject_finish(ctx, gr->n_mask, mb, parts, c_mask, omega, d_omega, dm,
                                        accumulate);
}

static rb_status check_absorption(rb_ctx *ctx, const rb_absorption *abs);

rb_status rb_backproject_lossy(rb_ctx *ctx, const rb_green *gr, const float *R,
                               const double *c_mask, const double *alpha0_mask, double y,
                               double omega, double d_omega, float *dm, int32_t accumulate) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(check_backproject(ctx, gr, R, c_mask, omega, d_omega, dm));
    const rb_absorption abs{alpha0_mask, y};
    RB_TRY(check_absorption(ctx, &abs));
    RB_HIP(ctx, hipSetDevice(ctx->device));
    const bool lp = gr->prec != RB_F32;
    ctx->ws.used = 0;
    RB_TRY(rb_arena_reserve(ctx, &ctx->ws, backproject_ws_bytes(gr->n, gr->n_mask, lp)));
    int mb = 0;
    float *parts = nullptr;
    RB_TRY(backproject_parts(ctx, &ctx->ws, gr, R, &parts, &mb));
    return rb_launch_backproject_finish_lossy(ctx, gr->n_mask, mb, parts, c_mask, alpha0_mask,
                                              omega, d_omega, y, nullptr, dm, accumulate);
}

rb_status rb_backproject(rb_ctx *ctx, const rb_green *gr, const float *R, const double *c_mask,
                         double omega, double d_omega, float *dm, int32_t accumulate) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(check_backproject(ctx, gr, R, c_mask, omega, d_omega, dm));
    RB_HIP(ctx, hipSetDevice(ctx->device));
    ctx->ws.used = 0;
    RB_TRY(rb_arena_reserve(ctx, &ctx->ws,
                            backproject_ws_bytes(gr->n, gr->n_mask, gr->prec != RB_F32)));
    return backproject_with(ctx, &ctx->ws, gr, R, c_mask, omega, d_omega, dm, accumulate);
}

rb_status rb_backproject_noalloc(rb_ctx *ctx, const rb_green *gr, const float *R,
                                 const double *c_mask, double omega, double d_omega, float *dm,
                                 int32_t accumulate) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(check_backproject(ctx, gr, R, c_mask, omega, d_omega, dm));
    const size_t need = backproject_ws_bytes(gr->n, gr->n_mask, gr->prec != RB_F32);
    if (need > RB_SCRATCH_BYTES)
        return rb_fail(ctx, RB_EINVAL,
                       "n = %d, n_mask = %d needs %zu scratch bytes; the allocation-free "
                       "back-projection holds %zu",
                       gr->n, gr->n_mask, need, (size_t)RB_SCRATCH_BYTES);
    void *base = scratch_of(ctx->device);
    if (!base)
        return rb_fail(ctx, RB_EDEVICE, "no scratch address for device %d", ctx->device);
    RB_HIP(ctx, hipSetDevice(ctx->device));
    rb_arena a;
    a.base = static_cast<char *>(base);
    a.cap = RB_SCRATCH_BYTES;
    // profiling creates its events on first use: off for this call
    const bool prof = ctx->prof;
    ctx->prof = false;
    const rb_status st = backproject_with(ctx, &a, gr, R, c_mask, omega, d_omega, dm, accumulate);
    ctx->prof = prof;
    return st;
}

// One frequency step (rows a1-a9) enqueued on ctx->stream. With ctx->deferred nothing
// synchronises with the host: errors stay in d_flag and the commit kernel checks them.
// Device buffers of one frequency step, carved from the context's step arena.
struct StepBufs {
    int N = 0, nm = 0, mb = 0;
    bool lp = false;
    size_t NN = 0;
    float *n_s = nullptr;
    rb_tables tb{};
    float4 *rec = nullptr;
    double2 *ringpos = nullptr;
    rb_green gr{};
    float *d_born = nullptr, *R = nullptr, *rsym = nullptr;
    uint16_t *Rp = nullptr;
    uint8_t *Rp8 = nullptr;  // split form: FP8 planes of Rs (the correction term's operand)
    uint16_t *Rf = nullptr;  // 16-bit forms: the whole Rs (Rp itself in the split form)
    float *rscale = nullptr, *wv = nullptr, *svscale = nullptr;
    unsigned int *rowmax = nullptr;  // per-row amplitude maxima of the binning (16-bit form)
    double *cq = nullptr, *dm = nullptr, *c_new = nullptr;
    float *parts = nullptr;
    // absorbing media: row passes of c0/c and alpha0, the maps of the current frequency and
    // alpha0 at the mask nodes
    double *tn = nullptr, *ta = nullptr, *aq = nullptr;
    float *n_w = nullptr, *a_w = nullptr;
};

static size_t step_arena_bytes(int N, int nm, size_t P, rb_prec prec) {
    const size_t NP = (size_t)N * nm, NN = (size_t)N * N;
    const size_t NPp = (size_t)rb_lp_pad(N) * nm;  // padded operand rows (16-bit form)
    const size_t NNp = (size_t)rb_lp_pad(N) * N;
    const bool lp = prec != RB_F32;
    const size_t NG = lp ? (size_t)N * rb_lp_pad(nm) : NP;  // G rows padded (16-bit form)
    const int mb = lp ? rb_rowred_lp_mblocks(N) : rb_rowred_mblocks(N);
    const size_t opb = lp ? 4 : 8;  // bytes per complex operand
    const size_t hparts = rb_prec_split(prec) ? 2 : 1;  // H and its low parts
    // node tables: ABI layout for the FP32 form, compact records (+ ring) for 16-bit
    const size_t tab_bytes = lp ? rb_align(NP * 16) + rb_align((size_t)N * 16)
                                : rb_align(NP * 8) + 3 * rb_align(NP * 4) + rb_align(NP);
    return rb_align(P * 4) + tab_bytes + rb_align(NN * 8) + rb_align(NN * 4) + rb_align(NN) +
           rb_align(NG * opb) + rb_align(hparts * 3 * NPp * opb) + 3 * rb_align(NN * 8) +
           rb_align(NNp * 4) +
           (rb_prec_split(prec) ? rb_align((size_t)2 * N * rb_lp8_pad(N)) : 0) +
           (lp && !rb_prec_split(prec) ? rb_align(NNp * 4) : 0) +
           rb_align((size_t)nm * 8) + rb_align((size_t)nm * 4) +
           3 * rb_align((size_t)nm * 8) + rb_align((size_t)2 * mb * nm * 4) + rb_align(8) +
           rb_align(8) + 2 * rb_align((size_t)2 * N * 4) + 2 * rb_align(P * 8) +
           2 * rb_align(P * 4) + rb_align((size_t)nm * 8);
}

static rb_status step_carve(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring, rb_prec prec,
                            StepBufs *b) {
    RB_TRY(rb_prepare_grid(ctx, grid));
    const int N = ring->n;
    const int nm = (int)ctx->n_mask;
    const size_t P = (size_t)grid->nx * grid->ny;
    const size_t NP = (size_t)N * nm, NN = (size_t)N * N;
    const size_t NPp = (size_t)rb_lp_pad(N) * nm;
    const size_t NNp = (size_t)rb_lp_pad(N) * N;
    const bool lp = prec != RB_F32;
    const size_t NG = lp ? (size_t)N * rb_lp_pad(nm) : NP;
    const size_t opb = lp ? 4 : 8;
    ctx->step.used = 0;
    RB_TRY(rb_arena_reserve(ctx, &ctx->step, step_arena_bytes(N, nm, P, prec)));
    rb_arena *a = &ctx->step;
    b->N = N;
    b->nm = nm;
    b->NN = NN;
    b->lp = lp;
    b->mb = lp ? rb_rowred_lp_mblocks(N) : rb_rowred_mblocks(N);
    b->n_s = rb_carve<float>(a, P);
    rb_tables &tb = b->tb;
    tb.n = N;
    tb.n_mask = nm;
    if (lp) {
        tb.T = nullptr;
        tb.A = tb.ux = tb.uy = nullptr;
        tb.flags = nullptr;
        b->rec = rb_carve<float4>(a, NP);
        b->ringpos = rb_carve<double2>(a, N);
    } else {
        tb.T = rb_carve<double>(a, NP);
        tb.A = rb_carve<float>(a, NP);
        tb.ux = rb_carve<float>(a, NP);
        tb.uy = rb_carve<float>(a, NP);
        tb.flags = rb_carve<uint8_t>(a, NP);
    }
    tb.rx_T = rb_carve<double>(a, NN);
    tb.rx_A = rb_carve<float>(a, NN);
    tb.rx_flags = rb_carve<uint8_t>(a, NN);
    rb_green &gr = b->gr;
    gr.n = N;
    gr.n_mask = nm;
    gr.prec = prec;
    gr.G = rb_carve<char>(a, NG * opb);
    gr.H = rb_carve<char>(a, (rb_prec_split(prec) ? 2 : 1) * 3 * (lp ? NPp : NP) * opb);
    gr.scales = rb_carve<float>(a, 2 * (size_t)N);
    b->rowmax = rb_carve<unsigned int>(a, 2 * (size_t)N);
    b->d_born = rb_carve<float>(a, 2 * NN);
    b->R = rb_carve<float>(a, 2 * NN);
    b->rsym = rb_carve<float>(a, 2 * NN);
    b->Rp = rb_carve<uint16_t>(a, 2 * NNp);
    if (rb_prec_split(prec)) b->Rp8 = rb_carve<uint8_t>(a, (size_t)2 * N * rb_lp8_pad(N));
    if (lp) b->Rf = rb_prec_split(prec) ? b->Rp : rb_carve<uint16_t>(a, 2 * NNp);
    b->rscale = rb_carve<float>(a, 2);
    b->wv = rb_carve<float>(a, 2 * (size_t)nm);
    b->svscale = rb_carve<float>(a, 2);
    b->cq = rb_carve<double>(a, nm);
    b->dm = rb_carve<double>(a, nm);
    b->c_new = rb_carve<double>(a, nm);
    b->parts = rb_carve<float>(a, (size_t)2 * b->mb * nm);
    b->tn = rb_carve<double>(a, P);
    b->ta = rb_carve<double>(a, P);
    b->n_w = rb_carve<float>(a, P);
    b->a_w = rb_carve<float>(a, P);
    b->aq = rb_carve<double>(a, nm);
    return RB_OK;
}

// a1: tracing map; a2-a3: rays and tables (independent of omega when lossless). In an
// absorbing medium (abs != NULL) the rays depend on omega: here only the row passes of both
// maps, the sound-speed part n_s and alpha0 at the nodes; step_trace_lossy per frequency.
static rb_status step_begin(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                            const rb_trace_params *tp, double *c, int32_t smooth_w,
                            double *residual_norm, StepBufs &b,
                            const rb_absorption *abs = nullptr) {
    if (abs) {
        RB_TRY(rb_launch_lossy_rows(ctx, grid, c, tp->c0, abs->alpha0, smooth_w, b.tn, b.ta,
                                    b.n_s));
        RB_TRY(rb_launch_gather_mask(ctx, abs->alpha0, b.aq));
    } else {
        RB_TRY(rb_launch_refractive_index(ctx, grid, c, tp->c0, smooth_w, b.n_s));
        RB_TRY(rb_launch_trace(ctx, grid, ring, tp, b.n_s, &b.tb, b.rec, b.ringpos, b.rowmax));
    }
    RB_TRY(rb_launch_gather_mask(ctx, c, b.cq));
    RB_TRY(rb_launch_zero_f64(ctx, b.dm, b.nm));
    if (residual_norm) RB_TRY(rb_launch_zero_f64(ctx, residual_norm, 1));
    return RB_OK;
}

// a1-a3 of one frequency in an absorbing medium: the maps n_w, a_w of omega (Eq.
// wave-number in units of k0; alpha = alpha0 omega^y), then rays and tables with A_abs.
static rb_status step_trace_lossy(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                                  const rb_trace_params *tp, int32_t smooth_w, double om,
                                  const rb_absorption *abs, StepBufs &b) {
    const double kd = tp->c0 * tan(0.5 * RB_PI * abs->y) * pow(om, abs->y - 1.0);
    RB_TRY(rb_launch_lossy_map(ctx, grid, b.tn, b.ta, smooth_w, kd, pow(om, abs->y), b.n_w,
                               b.a_w));
    return rb_launch_trace(ctx, grid, ring, tp, b.n_w, &b.tb, b.rec, b.ringpos, b.rowmax, b.a_w);
}

// a4: Green's functions and back-projection operands. In ray_born mode G is stored as
// G sqrt(v), v = Upsilon_m h^2 (m - m_s) (Upsilon_m = omega^2 lossless, omega c k~ in an
// absorbing medium), so that a5 is the plain symmetric product; ray_only needs no G.
static rb_status step_green(rb_ctx *ctx, const rb_grid *grid, const rb_trace_params *tp,
                            double om, rb_mode mode, StepBufs &b,
                            const rb_absorption *abs = nullptr) {
    const bool born_term = mode == RB_RAY_BORN;
    if (born_term) {
        if (abs)
            RB_TRY(rb_launch_rough_part_lossy(ctx, b.cq, b.aq, b.n_s, tp->c0, om, abs->y,
                                              grid->dx * grid->dx, b.wv));
        else
            RB_TRY(rb_launch_rough_part(ctx, b.cq, b.n_s, tp->c0, om * om * grid->dx * grid->dx,
                                        b.wv));
        // power-of-two scale that brings max |sqrt(v)| to [1, 2) (range of 16-bit types)
        RB_TRY(rb_launch_range_scale(ctx, b.wv, (size_t)b.nm, 1, b.svscale));
    }
    const float *gs = born_term ? b.wv : nullptr;
    if (b.lp)
        return rb_launch_green_lp_rec(ctx, b.rec, b.ringpos, b.N, om, tp->c0, &b.gr, gs,
                                      b.svscale, born_term, b.rowmax);
    return rb_launch_green(ctx, &b.tb, om, tp->c0, &b.gr, gs, b.svscale, born_term);
}

// a6: residual of the predicted data (ray part + Born term in b.d_born if `born`), and the
// 16-bit back-projection operand.
static rb_status step_residual(rb_ctx *ctx, const rb_trace_params *tp, double om, bool born,
                               const float *data_k, double *residual_norm, rb_prec prec,
                               StepBufs &b) {
    RB_TRY(rb_launch_residual(ctx, &b.tb, om, tp->c0, born ? b.d_born : nullptr, data_k, b.R,
                              residual_norm));
    if (b.lp)
        RB_TRY(rb_launch_to_planar(ctx, prec, b.R, b.N, b.Rp, b.rscale, b.gr.scales + b.N,
                                   b.Rp8, b.Rf));
    return RB_OK;
}

// a8 tail: undo the operand scale and accumulate the direction over the set in FP64.
static rb_status step_accumulate(rb_ctx *ctx, double om, double d_om, StepBufs &b,
                                 const rb_absorption *abs = nullptr) {
    if (b.lp) RB_TRY(rb_launch_unscale(ctx, b.parts, (size_t)2 * b.mb * b.nm, b.rscale));
    if (abs)
        return rb_launch_backproject_finish_lossy(ctx, b.nm, b.mb, b.parts, b.cq, b.aq, om, d_om,
                                                  abs->y, b.dm, nullptr, 0);
    return rb_launch_backproject_finish_acc(ctx, b.mb, b.parts, b.cq, om, d_om, b.dm);
}

// a9: model update, committed only if every value is finite.
static rb_status step_end(rb_ctx *ctx, double *c, double tau, int step_index, StepBufs &b) {
    if (ctx->deferred) {
        RB_TRY(rb_launch_update(ctx, b.cq, b.dm, tau, b.c_new));
        RB_TRY(rb_launch_note_fail(ctx, step_index));
        return rb_launch_commit(ctx, b.c_new, c, ctx->d_flag);
    }
    RB_TRY(rb_launch_fill_i32(ctx, ctx->d_flag, 1, 0));
    RB_TRY(rb_launch_update(ctx, b.cq, b.dm, tau, b.c_new));
    RB_HIP(ctx, hipMemcpyAsync(ctx->h_flag, ctx->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost,
                               ctx->stream));
    RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (*ctx->h_flag & 2)
        return rb_fail(ctx, RB_ENONFINITE, "non-finite model update rejected; c unchanged");
    return rb_launch_commit(ctx, b.c_new, c, nullptr);
}

static rb_status step_enqueue(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                              const rb_trace_params *tp, double *c, int32_t smooth_w,
                              int32_t n_omega, const double *omega, const double *d_omega,
                              const float *data, double tau, rb_mode mode, rb_prec prec,
                              double *residual_norm, int step_index,
                              const rb_absorption *abs = nullptr) {
    StepBufs b;
    RB_TRY(step_carve(ctx, grid, ring, prec, &b));
    RB_TRY(step_begin(ctx, grid, ring, tp, c, smooth_w, residual_norm, b, abs));
    for (int k = 0; k < n_omega; ++k) {
        const double om = omega[k];
        const bool born = mode == RB_RAY_BORN;
        if (abs) RB_TRY(step_trace_lossy(ctx, grid, ring, tp, smooth_w, om, abs, b));
        RB_TRY(step_green(ctx, grid, tp, om, mode, b, abs));
        // a5: Born term of the rough part in the predicted data
        if (born) {
            if (b.lp)
                RB_TRY(rb_launch_forward_lp(ctx, &b.gr, nullptr, nullptr, b.d_born, b.svscale));
            else
                RB_TRY(rb_launch_forward(ctx, &b.gr, nullptr, nullptr, b.d_born, b.svscale));
        }
        RB_TRY(step_residual(ctx, tp, om, born, data + 2 * b.NN * (size_t)k, residual_norm, prec,
                             b));
        // a8: Hessian-free back-projection
        if (b.lp) {
            RB_TRY(rb_launch_rowred_lp(ctx, prec, b.N, b.nm, b.Rp, b.gr.H, 3, b.parts, nullptr,
                                       h_low(&b.gr), b.Rp8, b.Rf));
        } else {
            int mbo = b.mb;
            RB_TRY(rb_launch_rowred(ctx, b.N, b.nm, b.R, (const float *)b.gr.H, 3, 0, b.rsym,
                                    b.parts, &mbo));
        }
        RB_TRY(step_accumulate(ctx, om, d_omega[k], b, abs));
    }
    return step_end(ctx, c, tau, step_index, b);
}


// The frequency step with its report handling (abs: absorbing medium or NULL).
static rb_status frequency_step_with(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                                     const rb_trace_params *tp, double *c, int32_t smooth_w,
                                     int32_t n_omega, const double *omega,
                                     const double *d_omega, const float *data, double tau,
                                     rb_mode mode, rb_prec prec, double *residual_norm,
                                     rb_report *report, const rb_absorption *abs) {
    RB_HIP(ctx, hipSetDevice(ctx->device));
    if (!report) {
        ctx->deferred = false;
        return step_enqueue(ctx, grid, ring, tp, c, smooth_w, n_omega, omega, d_omega, data,
                            tau, mode, prec, residual_norm, 0, abs);
    }
    // asynchronous form: the checks stay on the device (as in a sweep of one step) and the
    // status goes to the caller's report
    RB_TRY(rb_prepare_grid(ctx, grid));
    ctx->deferred = true;
    rb_status st = rb_launch_fill_i32(ctx, ctx->d_flag, RB_W_COUNT, 0);
    if (st == RB_OK) st = rb_launch_fill_i32(ctx, ctx->d_flag + RB_W_FAIL_STEP, 1, -1);
    if (st == RB_OK)
        st = step_enqueue(ctx, grid, ring, tp, c, smooth_w, n_omega, omega, d_omega, data, tau,
                          mode, prec, residual_norm, 0, abs);
    if (st == RB_OK) st = rb_launch_report(ctx, report);
    ctx->deferred = false;
    return st;
}

rb_status rb_frequency_step(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                            const rb_trace_params *tp, double *c, int32_t smooth_w,
                            int32_t n_omega, const double *omega, const double *d_omega,
                            const float *data, double tau, rb_mode mode, rb_prec prec,
                            double *residual_norm, rb_report *report) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(check_step_args(ctx, grid, ring, tp, c, smooth_w, n_omega, omega, d_omega, data, tau,
                           mode, prec));
    return frequency_step_with(ctx, grid, ring, tp, c, smooth_w, n_omega, omega, d_omega, data,
                               tau, mode, prec, residual_norm, report, nullptr);
}

static rb_status check_absorption(rb_ctx *ctx, const rb_absorption *abs) {
    if (!abs || !abs->alpha0)
        return rb_fail(ctx, RB_EINVAL, "absorption needs a device alpha0 map");
    if (!(abs->y > 0.0 && abs->y <= 2.0) || !(fabs(abs->y - 1.0) >= 1e-3))
        return rb_fail(ctx, RB_EINVAL, "power-law exponent y = %g outside (0, 2] or within "
                       "1e-3 of 1", abs->y);
    return RB_OK;
}

rb_status rb_lossy_maps(rb_ctx *ctx, const rb_grid *grid, const double *c,
                        const rb_absorption *abs, double c0, double omega, int32_t w,
                        float *n_w, float *a_w) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(rb_check_grid(ctx, grid));
    RB_TRY(check_absorption(ctx, abs));
    if (!c || !n_w || !a_w)
        return rb_fail(ctx, RB_EINVAL, "c, n_w and a_w must be device pointers");
    if (w < 1 || (w & 1) == 0) return rb_fail(ctx, RB_EINVAL, "window must be odd and >= 1");
    if (!finite_pos(c0) || !finite_pos(omega))
        return rb_fail(ctx, RB_EINVAL, "c0 and omega must be positive");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    const size_t P = (size_t)grid->nx * grid->ny;
    ctx->ws.used = 0;
    RB_TRY(rb_arena_reserve(ctx, &ctx->ws, 2 * rb_align(P * sizeof(double))));
    double *tn = rb_carve<double>(&ctx->ws, P);
    double *ta = rb_carve<double>(&ctx->ws, P);
    RB_TRY(rb_launch_lossy_rows(ctx, grid, c, c0, abs->alpha0, w, tn, ta, nullptr));
    const double kd = c0 * tan(0.5 * RB_PI * abs->y) * pow(omega, abs->y - 1.0);
    return rb_launch_lossy_map(ctx, grid, tn, ta, w, kd, pow(omega, abs->y), n_w, a_w);
}

rb_status rb_trace_rays_lossy(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                              const rb_trace_params *tp, const float *n_w, const float *a_w,
                              const rb_tables *out) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(rb_check_grid(ctx, grid));
    RB_TRY(rb_check_ring(ctx, grid, ring));
    RB_TRY(rb_check_trace(ctx, tp));
    if (!n_w || !a_w) return rb_fail(ctx, RB_EINVAL, "n_w and a_w must be device pointers");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    RB_TRY(rb_prepare_grid(ctx, grid));
    RB_TRY(check_tables(ctx, out, ring->n, ctx->n_mask));
    return rb_launch_trace(ctx, grid, ring, tp, n_w, out, nullptr, nullptr, nullptr, a_w);
}

rb_status rb_frequency_step_lossy(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                                  const rb_trace_params *tp, double *c,
                                  const rb_absorption *abs, int32_t smooth_w, int32_t n_omega,
                                  const double *omega, const double *d_omega, const float *data,
                                  double tau, rb_mode mode, rb_prec prec,
                                  double *residual_norm, rb_report *report) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(check_step_args(ctx, grid, ring, tp, c, smooth_w, n_omega, omega, d_omega, data, tau,
                           mode, prec));
    RB_TRY(check_absorption(ctx, abs));
    return frequency_step_with(ctx, grid, ring, tp, c, smooth_w, n_omega, omega, d_omega, data,
                               tau, mode, prec, residual_norm, report, abs);
}

// Gauss-Newton step ----------------------------------------------------------------------
// Its workspace lies outside rb_reserve: grown on demand whatever the reservation.
static rb_status gn_reserve(rb_ctx *ctx, size_t bytes) {
    rb_arena *a = &ctx->gn;
    if (bytes <= a->cap) return RB_OK;
    if (a->base) {
        RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        RB_HIP(ctx, hipFree(a->base));
        a->base = nullptr;
        a->cap = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return rb_fail(ctx, RB_ENOMEM, "Gauss-Newton workspace of %zu bytes failed", bytes);
    }
    a->base = static_cast<char *>(p);
    a->cap = bytes;
    return RB_OK;
}

static rb_status gn_enqueue(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                            const rb_trace_params *tp, double *c, int32_t smooth_w,
                            int32_t n_omega, const double *omega, const float *data, double tau,
                            int32_t n_inner, rb_green_model model, rb_prec prec,
                            double *residual_norm, double *cg_norms) {
    StepBufs b;
    RB_TRY(step_carve(ctx, grid, ring, prec, &b));
    const int N = b.N, nm = b.nm;
    const bool lp = b.lp;
    const rb_prec kp = rb_prec_split(prec) ? RB_F16 : prec;  // G itself is never split
    const size_t Np = (size_t)rb_lp_pad(N), Mp = (size_t)rb_lp_pad(nm);
    const int mb = lp ? rb_rowred_lp_mblocks(N) : rb_rowred_mblocks(N);
    const size_t gbytes = lp ? 2 * (size_t)N * Mp * 2 : (size_t)N * nm * 8;
    const size_t gtbytes = lp ? 2 * (size_t)nm * Np * 2 : 0;
    const size_t per = rb_align(gbytes) + rb_align(gtbytes) + rb_align(2 * (size_t)N * 4) +
                       rb_align((size_t)nm * 8);
    const size_t need = n_omega * per + 5 * rb_align((size_t)nm * 8) +
                        2 * rb_align((size_t)nm * 4) + rb_align(b.NN * 8) +
                        rb_align(2 * (size_t)N * Np * 2) + rb_align(8) + rb_align(b.NN * 8) +
                        rb_align((size_t)2 * mb * nm * 4) + rb_gn_scalar_bytes() +
                        rb_align((size_t)N * 16);
    RB_TRY(gn_reserve(ctx, need));
    rb_arena *a = &ctx->gn;
    a->used = 0;
    rb_green gk[8];
    void *Gt[8];
    float *wk[8];
    for (int k = 0; k < n_omega; ++k) {
        gk[k] = rb_green{N, nm, kp, rb_carve<char>(a, gbytes), b.gr.H, nullptr};
        Gt[k] = lp ? rb_carve<char>(a, gtbytes) : nullptr;
        gk[k].scales = rb_carve<float>(a, 2 * (size_t)N);
        wk[k] = rb_carve<float>(a, 2 * (size_t)nm);
    }
    double *x = rb_carve<double>(a, nm), *r = rb_carve<double>(a, nm);
    double *pv = rb_carve<double>(a, nm), *hp = rb_carve<double>(a, nm);
    double *grad = rb_carve<double>(a, nm);
    float *pf = rb_carve<float>(a, nm), *delta = rb_carve<float>(a, nm);
    float *d = rb_carve<float>(a, 2 * b.NN);
    uint16_t *Rp = rb_carve<uint16_t>(a, 2 * (size_t)N * Np);
    float *rscale = rb_carve<float>(a, 2);
    float *rsym = rb_carve<float>(a, 2 * b.NN);
    float *parts = rb_carve<float>(a, (size_t)2 * mb * nm);
    double *scal = reinterpret_cast<double *>(rb_carve<char>(a, rb_gn_scalar_bytes()));
    double2 *ringpos = lp ? b.ringpos : rb_carve<double2>(a, N);

    // a1-a3 or the analytic water tables
    if (model == RB_GREEN_RAY) {
        RB_TRY(rb_launch_refractive_index(ctx, grid, c, tp->c0, smooth_w, b.n_s));
        RB_TRY(rb_launch_trace(ctx, grid, ring, tp, b.n_s, &b.tb, b.rec, b.ringpos, b.rowmax));
    } else {
        RB_TRY(rb_launch_water_tables(ctx, ring, tp->c0, &b.tb, b.rec, ringpos,
                                      lp ? b.rowmax : nullptr));
    }
    RB_TRY(rb_launch_gather_mask(ctx, c, b.cq));
    RB_TRY(rb_launch_gn_delta(ctx, b.cq, model == RB_GREEN_RAY ? b.n_s : nullptr, tp->c0, delta));
    if (residual_norm) RB_TRY(rb_launch_zero_f64(ctx, residual_norm, 1));

    auto forward = [&](int k, const float *dl, float *out) -> rb_status {
        return lp ? rb_launch_forward_lp(ctx, &gk[k], wk[k], dl, out, nullptr)
                  : rb_launch_forward(ctx, &gk[k], wk[k], dl, out, nullptr);
    };
    // Q = 1 adjoint of the pair data R (zero off the kept pairs), added to acc in FP64
    auto adjoint = [&](int k, const float *R, double *acc, int first) -> rb_status {
        int mbo = mb;
        if (lp) {
            RB_TRY(rb_launch_to_planar(ctx, kp, R, N, Rp, rscale, gk[k].scales));
            RB_TRY(rb_launch_rowred_lp(ctx, kp, N, nm, Rp, Gt[k], 1, parts, &mbo));
            RB_TRY(rb_launch_unscale(ctx, parts, (size_t)2 * mb * nm, rscale));
        } else {
            RB_TRY(rb_launch_rowred(ctx, N, nm, R, (const float *)gk[k].G, 1, 1, rsym, parts,
                                    &mbo));
        }
        return rb_launch_gn_adjoint_acc(ctx, mb, parts, wk[k], acc, first);
    };
    // operands, predicted data, residual and gradient of every frequency of the set
    const double h2 = grid->dx * grid->dx;
    for (int k = 0; k < n_omega; ++k) {
        const double om = omega[k];
        RB_TRY(rb_launch_gn_weight(ctx, wk[k], nm, om * om * h2));
        if (lp)
            RB_TRY(rb_launch_green_lp_rec(ctx, b.rec, ringpos, N, om, tp->c0, &gk[k], nullptr,
                                          nullptr, 1, b.rowmax));
        else
            RB_TRY(rb_launch_green(ctx, &b.tb, om, tp->c0, &gk[k], nullptr, nullptr, 1));
        RB_TRY(forward(k, delta, d));  // Born term of m - m_s in the predicted data
        RB_TRY(rb_launch_residual(ctx, &b.tb, om, tp->c0, d, data + 2 * b.NN * (size_t)k, b.R,
                                  residual_norm));
        if (lp) RB_TRY(rb_launch_transpose_conj(ctx, &gk[k], Gt[k]));
        RB_TRY(adjoint(k, b.R, grad, k == 0));
    }
    // conjugate gradients on H x = -grad
    RB_TRY(rb_launch_gn_cg(ctx, 0, x, r, pv, hp, pf, grad, scal, cg_norms, 0));
    for (int it = 0; it < n_inner; ++it) {
        for (int k = 0; k < n_omega; ++k) {
            RB_TRY(forward(k, pf, d));
            RB_TRY(rb_launch_gn_mask_pairs(ctx, d, b.tb.rx_flags, N));
            RB_TRY(adjoint(k, d, hp, k == 0));
        }
        RB_TRY(rb_launch_gn_cg(ctx, 1, x, r, pv, hp, pf, nullptr, scal, cg_norms, it + 1));
    }
    // a9: m <- m + tau x, committed only if finite
    RB_TRY(rb_launch_update(ctx, b.cq, x, tau, b.c_new));
    RB_TRY(rb_launch_note_fail(ctx, 0));
    return rb_launch_commit(ctx, b.c_new, c, ctx->d_flag);
}

rb_status rb_gauss_newton_step(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                               const rb_trace_params *tp, double *c, int32_t smooth_w,
                               int32_t n_omega, const double *omega, const float *data,
                               double tau, int32_t n_inner, rb_green_model model, rb_prec prec,
                               double *residual_norm, double *cg_norms, rb_report *report) {
    if (!ctx) return RB_EINVAL;
    if (n_omega < 1 || n_omega > 8)
        return rb_fail(ctx, RB_EINVAL, "a Gauss-Newton set holds 1..8 frequencies, not %d",
                       n_omega);
    if (n_inner < 1 || n_inner > 256)
        return rb_fail(ctx, RB_EINVAL, "n_inner must be in 1..256, not %d", n_inner);
    if (model != RB_GREEN_RAY && model != RB_GREEN_WATER)
        return rb_fail(ctx, RB_EINVAL, "unknown Green's-function model %d", (int)model);
    std::vector<double> dom(n_omega, 1.0);  // no spacing in this method; validated as positive
    RB_TRY(check_step_args(ctx, grid, ring, tp, c, model == RB_GREEN_RAY ? smooth_w : 1, n_omega,
                           omega, dom.data(), data, tau, RB_RAY_BORN, prec));
    RB_HIP(ctx, hipSetDevice(ctx->device));
    RB_TRY(rb_prepare_grid(ctx, grid));
    ctx->deferred = true;
    rb_status st = rb_launch_fill_i32(ctx, ctx->d_flag, RB_W_COUNT, 0);
    if (st == RB_OK) st = rb_launch_fill_i32(ctx, ctx->d_flag + RB_W_FAIL_STEP, 1, -1);
    if (st == RB_OK)
        st = gn_enqueue(ctx, grid, ring, tp, c, smooth_w, n_omega, omega, data, tau, n_inner,
                        model, prec, residual_norm, cg_norms);
    if (st == RB_OK && report) st = rb_launch_report(ctx, report);
    ctx->deferred = false;
    if (st != RB_OK || report) return st;
    RB_HIP(ctx, hipMemcpyAsync(ctx->h_flag, ctx->d_flag, RB_W_COUNT * sizeof(int32_t),
                               hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->lost_nodes = ctx->h_flag[RB_W_LOST];
    ctx->ray_samples = *reinterpret_cast<const int64_t *>(ctx->h_flag + RB_W_SAMPLES);
    const int32_t fl = ctx->h_flag[RB_W_FLAGS];
    if (fl)
        return rb_fail(ctx, RB_ENONFINITE, "the Gauss-Newton step failed (%s); c unchanged",
                       (fl & 1) ? "a ray did not reach the ring within max_steps"
                                : "non-finite model update");
    return RB_OK;
}

size_t rb_workspace_bytes(const rb_grid *grid, const rb_ring *ring, const rb_trace_params *tp,
                          rb_prec prec, size_t sample_budget) {
    if (!grid || !ring || !tp || grid->nx < 1 || grid->ny < 1 || ring->n < 1 || tp->n_rays < 1 ||
        tp->max_steps < 1 || !rb_prec_valid(prec))
        return 0;
    const GeomSizes gs = geom_sizes(grid);
    if (gs.nm < 1) return 0;
    const size_t P = (size_t)grid->nx * grid->ny;
    const size_t lists = rb_align((size_t)gs.nm * 4) + rb_align(P * 4);
    return step_arena_bytes(ring->n, (int)gs.nm, P, prec) +
           ws_need(grid, ring, tp, gs, sample_budget, device_cus()) + lists;
}

rb_status rb_reserve(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                     const rb_trace_params *tp, rb_prec prec) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(rb_check_grid(ctx, grid));
    RB_TRY(rb_check_ring(ctx, grid, ring));
    RB_TRY(rb_check_trace(ctx, tp));
    if (!rb_prec_valid(prec))
        return rb_fail(ctx, RB_EINVAL, "unknown operand precision %d", (int)prec);
    if (ctx->capturing) return rb_fail(ctx, RB_EINVAL, "rb_reserve inside a graph capture");
    RB_HIP(ctx, hipSetDevice(ctx->device));
    ctx->fixed = false;
    RB_TRY(rb_prepare_grid(ctx, grid));
    const GeomSizes gs = geom_sizes(grid);
    const size_t P = (size_t)grid->nx * grid->ny;
    const size_t step = step_arena_bytes(ring->n, (int)gs.nm, P, prec);
    const size_t ws = ws_need(grid, ring, tp, gs, ctx->sample_budget, ctx->n_cu);
    // exactly these sizes: release larger blocks of an earlier geometry as well
    for (rb_arena *a : {&ctx->step, &ctx->ws}) {
        const size_t want = a == &ctx->step ? step : ws;
        if (a->base && a->cap != want) {
            RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
            RB_HIP(ctx, hipFree(a->base));
            a->base = nullptr;
            a->cap = 0;
            ++ctx->gen;
        }
        RB_TRY(rb_arena_reserve(ctx, a, want));
    }
    ctx->fixed = true;
    return RB_OK;
}

size_t rb_step_bytes(const rb_grid *grid, const rb_ring *ring, const rb_trace_params *tp,
                     rb_prec prec, size_t sample_budget) {
    if (!grid || !ring || !tp || grid->nx < 1 || grid->ny < 1 || ring->n < 1 || tp->n_rays < 1 ||
        tp->max_steps < 1)
        return 0;
    const GeomSizes gs = geom_sizes(grid);
    const int64_t nm = gs.nm;
    if (nm < 1) return 0;
    const size_t tiles = gs.tiles;
    const size_t P = (size_t)grid->nx * grid->ny;
    const int N = ring->n;
    const int n_cu = device_cus();
    size_t ws = rb_align(P * sizeof(double));  // smoothing
    ws = std::max(ws, rb_trace_ws_bytes(grid, ring, tp, nm, tiles, sample_budget));
    ws = std::max(ws, prec == RB_F32 ? rb_forward_ws_bytes(N, (int)nm)
                                     : rb_forward_lp_ws_bytes(N, (int)nm, std::max(8, n_cu)));
    const size_t fixed = (size_t)nm * 4 + P * 4 + RB_W_COUNT * 4 + RB_RED_PARTS * 4;
    return step_arena_bytes(N, (int)nm, P, prec) + ws + fixed;
}

rb_status rb_set_receiver_linking(rb_ctx *ctx, int32_t max_iter, double tol) {
    if (!ctx) return RB_EINVAL;
    if (max_iter < 0 || max_iter > 64)
        return rb_fail(ctx, RB_EINVAL, "linking takes 0 .. 64 rays per pair, not %d", max_iter);
    if (max_iter > 0 && !(tol > 0.0 && tol <= RB_LINK_ACCEPT))
        return rb_fail(ctx, RB_EINVAL, "linking tolerance %g outside (0, %g] radians", tol,
                       RB_LINK_ACCEPT);
    if (max_iter != ctx->link_iter || (max_iter > 0 && tol != ctx->link_tol)) ++ctx->gen;
    ctx->link_iter = max_iter;
    if (max_iter > 0) ctx->link_tol = tol;
    return RB_OK;
}

rb_status rb_set_sample_budget(rb_ctx *ctx, size_t bytes) {
    if (!ctx) return RB_EINVAL;
    if (bytes < ((size_t)1 << 20)) return rb_fail(ctx, RB_EINVAL, "sample budget below 1 MiB");
    ctx->sample_budget = bytes;
    return RB_OK;
}

// Install t in the context's table (replacing the record of its shape), or remove the record
// of t's shape with remove = true.
static rb_status tune_put(rb_ctx *ctx, const rb_tuning &t, bool remove = false) {
    int i = 0;
    while (i < ctx->n_tune && !(ctx->tune[i].n == t.n && ctx->tune[i].n_mask == t.n_mask &&
                                ctx->tune[i].prec == t.prec))
        ++i;
    if (remove) {
        if (i < ctx->n_tune) ctx->tune[i] = ctx->tune[--ctx->n_tune];
    } else if (i < ctx->n_tune) {
        ctx->tune[i] = t;
    } else {
        if (ctx->n_tune == rb_ctx::kMaxTune)
            return rb_fail(ctx, RB_EUNSUPPORTED, "at most %d tunings per context",
                           rb_ctx::kMaxTune);
        ctx->tune[ctx->n_tune++] = t;
    }
    ++ctx->gen;  // cached graphs hold the old launches
    return RB_OK;
}

rb_status rb_set_tuning(rb_ctx *ctx, const rb_tuning *t) {
    if (!ctx) return RB_EINVAL;
    if (!t) {
        if (ctx->n_tune) ++ctx->gen;
        ctx->n_tune = 0;
        return RB_OK;
    }
    if (t->n < 1 || t->n_mask < 1)
        return rb_fail(ctx, RB_EINVAL, "tuning for n = %d, n_mask = %d", t->n, t->n_mask);
    if (!rb_prec_valid(t->prec))
        return rb_fail(ctx, RB_EINVAL, "tuning for an unknown precision %d", (int)t->prec);
    if (t->fwd_tile != RB_TILE_256x128 && t->fwd_tile != RB_TILE_128x128)
        return rb_fail(ctx, RB_EINVAL, "unknown forward tile %d", (int)t->fwd_tile);
    if (t->prec == RB_F32 && t->fwd_tile != RB_TILE_128x128)
        return rb_fail(ctx, RB_EINVAL, "the FP32 forward has 128 x 128 tiles only");
    if (t->fwd_splitk < 1 || t->fwd_splitk > 1024)
        return rb_fail(ctx, RB_EINVAL, "forward K split %d outside 1..1024", t->fwd_splitk);
    return tune_put(ctx, *t);
}

rb_status rb_get_tuning(const rb_ctx *ctx, rb_tuning *out) {
    if (!ctx || !out) return RB_EINVAL;
    const rb_tuning *t = rb_tuned(ctx, out->n, out->n_mask, out->prec);
    if (!t) return RB_EINVAL;
    *out = *t;
    return RB_OK;
}

rb_status rb_autotune(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring, rb_prec prec,
                      rb_tuning *out) {
    if (!ctx) return RB_EINVAL;
    RB_TRY(rb_check_grid(ctx, grid));
    RB_TRY(rb_check_ring(ctx, grid, ring));
    if (!rb_prec_valid(prec)) return rb_fail(ctx, RB_EINVAL, "unknown precision %d", (int)prec);
    RB_HIP(ctx, hipSetDevice(ctx->device));
    StepBufs b;
    RB_TRY(step_carve(ctx, grid, ring, prec, &b));
    RB_TRY(rb_launch_tune_fill(ctx, &b.gr, b.svscale));
    const int N = b.N, nm = b.nm;
    // candidates: each tile with K splits 8, 16, ..., RB_TUNE_SPLITK_MAX and its built-in one
    std::vector<rb_tuning> cand;
    const rb_tile tiles[2] = {RB_TILE_256x128, RB_TILE_128x128};
    for (int ti = prec == RB_F32 ? 1 : 0; ti < 2; ++ti) {
        std::vector<int> splits;
        for (int s = 8; s <= RB_TUNE_SPLITK_MAX; s += 8) splits.push_back(s);
        splits.push_back(prec == RB_F32 ? rb_forward_default_splitk(N, nm)
                                        : rb_forward_lp_default_splitk(N, nm, ti == 0,
                                                                       ctx->n_cu));
        std::sort(splits.begin(), splits.end());
        splits.erase(std::unique(splits.begin(), splits.end()), splits.end());
        for (int sk : splits) {
            rb_tuning t{};
            t.n = N;
            t.n_mask = nm;
            t.prec = prec;
            t.fwd_tile = tiles[ti];
            t.fwd_splitk = sk;
            cand.push_back(t);
        }
    }
    const bool prof = ctx->prof;
    ctx->prof = false;
    // the shape's current record, restored if tuning fails
    const rb_tuning *cur = rb_tuned(ctx, N, nm, prec);
    const bool had = cur != nullptr;
    const rb_tuning old = had ? *cur : rb_tuning{};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rb_status st = RB_OK;
    rb_tuning best{};
    float best_ms = 3.0e38f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        st = rb_fail(ctx, RB_EDEVICE, "event creation failed");
    }
    auto forward = [&]() {
        return prec == RB_F32
                   ? rb_launch_forward(ctx, &b.gr, nullptr, nullptr, b.d_born, b.svscale)
                   : rb_launch_forward_lp(ctx, &b.gr, nullptr, nullptr, b.d_born, b.svscale);
    };
    constexpr int kReps = 3;
    for (size_t i = 0; i < cand.size() && st == RB_OK; ++i) {
        st = tune_put(ctx, cand[i]);
        if (st == RB_OK) st = forward();  // first launch of the configuration, untimed
        if (st == RB_OK && hipEventRecord(e0, ctx->stream) != hipSuccess) st = RB_EDEVICE;
        for (int r = 0; r < kReps && st == RB_OK; ++r) st = forward();
        float ms = 0.f;
        if (st == RB_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                            hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
            (void)hipGetLastError();
            st = rb_fail(ctx, RB_EDEVICE, "timing the forward failed");
        }
        if (st == RB_OK && ms / kReps < best_ms) {
            best_ms = ms / kReps;
            best = cand[i];
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    ctx->prof = prof;
    if (st != RB_OK) {
        rb_tuning key{};
        key.n = N;
        key.n_mask = nm;
        key.prec = prec;
        (void)(had ? tune_put(ctx, old) : tune_put(ctx, key, true));
        return st;
    }
    best.fwd_ms = best_ms;
    RB_TRY(tune_put(ctx, best));
    if (out) *out = best;
    return RB_OK;
}

// Frequency steps of several scans, enqueued together. The per-scan stages run on each scan's
// own stream (the batch's scans overlap on the device); for each frequency index k, the Born
// forward terms and the back-projections of every scan with a k-th frequency run as one
// grouped launch each, on the first scan's stream, ordered by events.
static rb_status batch_enqueue(const rb_scan_step *st, int count, rb_prec prec,
                               StepBufs *bufs) {
    rb_ctx *lead = st[0].ctx;
    hipStream_t ls = lead->stream;
    int kmax = 0;
    for (int i = 0; i < count; ++i) {
        rb_ctx *ctx = st[i].ctx;
        RB_TRY(step_carve(ctx, st[i].grid, st[i].ring, prec, &bufs[i]));
        RB_TRY(rb_launch_fill_i32(ctx, ctx->d_flag, RB_W_COUNT, 0));
        RB_TRY(rb_launch_fill_i32(ctx, ctx->d_flag + RB_W_FAIL_STEP, 1, -1));
        RB_TRY(step_begin(ctx, st[i].grid, st[i].ring, st[i].tp, st[i].c, st[i].smooth_w,
                          st[i].residual_norm, bufs[i]));
        kmax = std::max(kmax, st[i].n_omega);
    }
    for (int k = 0; k < kmax; ++k) {
        int act[RB_GROUP_MAX], na = 0;
        for (int i = 0; i < count; ++i)
            if (st[i].n_omega > k) act[na++] = i;
        for (int a = 0; a < na; ++a) {
            const rb_scan_step &s = st[act[a]];
            RB_TRY(step_green(s.ctx, s.grid, s.tp, s.omega[k], s.mode, bufs[act[a]]));
            if (s.ctx->stream != ls) {
                RB_HIP(s.ctx, hipEventRecord(s.ctx->ev_join, s.ctx->stream));
                RB_HIP(lead, hipStreamWaitEvent(ls, s.ctx->ev_join, 0));
            }
        }
        // contractions and residuals of every active scan on the lead stream
        rb_status res = RB_OK;
        hipStream_t saved[RB_GROUP_MAX];
        for (int a = 0; a < na; ++a) {
            saved[a] = st[act[a]].ctx->stream;
            st[act[a]].ctx->stream = ls;
        }
        do {
            rb_fwd_plan plans[RB_GROUP_MAX];
            int np = 0, born[RB_GROUP_MAX] = {0};
            for (int a = 0; a < na && res == RB_OK; ++a) {
                const rb_scan_step &s = st[act[a]];
                StepBufs &b = bufs[act[a]];
                if (s.mode != RB_RAY_BORN) continue;
                born[a] = 1;
                if (b.lp) {
                    res = rb_forward_lp_plan(s.ctx, &b.gr, b.svscale, &plans[np]);
                    if (res == RB_OK && !plans[np].pipe)  // too large for the grouped kernel
                        res = rb_launch_forward_lp(s.ctx, &b.gr, nullptr, nullptr, b.d_born,
                                                   b.svscale);
                    else if (res == RB_OK)
                        ++np;
                } else {
                    res = rb_launch_forward(s.ctx, &b.gr, nullptr, nullptr, b.d_born, b.svscale);
                }
            }
            if (res != RB_OK) break;
            if (np > 0) res = rb_launch_forward_lp_group(lead, prec, plans, np);
            for (int a = 0, j = 0; a < na && res == RB_OK; ++a) {
                const rb_scan_step &s = st[act[a]];
                StepBufs &b = bufs[act[a]];
                if (born[a] && b.lp && j < np && plans[j].gr.G == b.gr.G)
                    res = rb_forward_lp_reduce(s.ctx, &plans[j++], b.d_born);
                if (res == RB_OK)
                    res = step_residual(s.ctx, s.tp, s.omega[k], born[a] != 0,
                                        s.data + 2 * b.NN * (size_t)k, s.residual_norm, prec, b);
            }
            if (res != RB_OK) break;
            if (prec != RB_F32) {
                rb_rowred_prob pr[RB_GROUP_MAX];
                for (int a = 0; a < na; ++a) {
                    StepBufs &b = bufs[act[a]];
                    pr[a] = rb_rowred_prob{b.Rp,  b.gr.H,        b.parts, b.N,
                                           b.nm,  h_low(&b.gr),  b.Rp8,   b.Rf};
                }
                res = rb_launch_rowred_lp_group(lead, prec, pr, na, 3);
            } else {
                for (int a = 0; a < na && res == RB_OK; ++a) {
                    StepBufs &b = bufs[act[a]];
                    res = rb_launch_rowred(st[act[a]].ctx, b.N, b.nm, b.R, (const float *)b.gr.H,
                                           3, 0, b.rsym, b.parts, nullptr);
                }
            }
        } while (false);
        for (int a = 0; a < na; ++a) st[act[a]].ctx->stream = saved[a];
        if (res != RB_OK) return res;
        RB_HIP(lead, hipEventRecord(lead->ev_join, ls));
        for (int a = 0; a < na; ++a) {
            const rb_scan_step &s = st[act[a]];
            if (s.ctx->stream != ls) RB_HIP(s.ctx, hipStreamWaitEvent(s.ctx->stream, lead->ev_join, 0));
            RB_TRY(step_accumulate(s.ctx, s.omega[k], s.d_omega[k], bufs[act[a]]));
        }
    }
    for (int i = 0; i < count; ++i)
        RB_TRY(step_end(st[i].ctx, st[i].c, st[i].tau, 0, bufs[i]));
    // later work on the lead stream waits for every scan's last kernel
    for (int i = 1; i < count; ++i) {
        rb_ctx *ctx = st[i].ctx;
        if (ctx->stream == ls) continue;
        RB_HIP(ctx, hipEventRecord(ctx->ev_join, ctx->stream));
        RB_HIP(lead, hipStreamWaitEvent(ls, ctx->ev_join, 0));
    }
    return RB_OK;
}

rb_status rb_frequency_step_batch(const rb_scan_step *steps, int32_t count, rb_prec prec,
                                  rb_status *status) {
    if (!steps || count < 1 || count > RB_GROUP_MAX) return RB_EINVAL;
    for (int i = 0; i < count; ++i) {
        rb_ctx *ctx = steps[i].ctx;
        if (!ctx) return RB_EINVAL;
        ctx->err[0] = 0;
        if (status) status[i] = RB_OK;
        for (int j = 0; j < i; ++j)
            if (steps[j].ctx == ctx)
                return rb_fail(ctx, RB_EINVAL, "a batch takes each context once");
        if (ctx->device != steps[0].ctx->device)
            return rb_fail(ctx, RB_EINVAL, "the scans of a batch share one device");
        RB_TRY(check_step_args(ctx, steps[i].grid, steps[i].ring, steps[i].tp, steps[i].c,
                               steps[i].smooth_w, steps[i].n_omega, steps[i].omega,
                               steps[i].d_omega, steps[i].data, steps[i].tau, steps[i].mode,
                               prec));
    }
    rb_ctx *lead = steps[0].ctx;
    RB_HIP(lead, hipSetDevice(lead->device));
    bool prof[RB_GROUP_MAX];
    for (int i = 0; i < count; ++i) {
        rb_ctx *ctx = steps[i].ctx;
        if (!ctx->ev_join)
            RB_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
    }
    for (int i = 0; i < count; ++i) {
        prof[i] = steps[i].ctx->prof;
        steps[i].ctx->prof = false;
        steps[i].ctx->deferred = true;
    }
    StepBufs bufs[RB_GROUP_MAX];
    rb_status st = batch_enqueue(steps, count, prec, bufs);
    for (int i = 0; i < count; ++i) {
        steps[i].ctx->prof = prof[i];
        steps[i].ctx->deferred = false;
    }
    if (st != RB_OK) return st;
    // each scan's checks: a failed step left its model unchanged
    rb_status first = RB_OK;
    for (int i = 0; i < count; ++i) {
        rb_ctx *ctx = steps[i].ctx;
        RB_HIP(ctx, hipMemcpyAsync(ctx->h_flag, ctx->d_flag, RB_W_COUNT * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, ctx->stream));
        RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        ctx->lost_nodes = ctx->h_flag[RB_W_LOST];
        ctx->ray_samples = *reinterpret_cast<const int64_t *>(ctx->h_flag + RB_W_SAMPLES);
        const int32_t fl = ctx->h_flag[RB_W_FLAGS];
        rb_status si = RB_OK;
        if (fl)
            si = rb_fail(ctx, RB_ENONFINITE, "the step failed (%s); c holds the model before it",
                         (fl & 1) ? "a ray did not reach the ring within max_steps"
                                  : "non-finite model update");
        if (status) status[i] = si;
        if (first == RB_OK) first = si;
    }
    return first;
}

// The steps of a sweep, enqueued with deferred checks (also the body of the captured graph).
static rb_status sweep_enqueue(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                               const rb_trace_params *tp, double *c, int32_t n_steps,
                               const int32_t *smooth_w, const int32_t *n_omega,
                               const double *omega, const double *d_omega, const float *data,
                               double tau, rb_mode mode, rb_prec prec, double *residual_norms) {
    const size_t NN = (size_t)ring->n * ring->n;
    RB_TRY(rb_launch_fill_i32(ctx, ctx->d_flag, RB_W_COUNT, 0));
    RB_TRY(rb_launch_fill_i32(ctx, ctx->d_flag + RB_W_FAIL_STEP, 1, -1));
    size_t f0 = 0;
    for (int k = 0; k < n_steps; ++k) {
        RB_TRY(step_enqueue(ctx, grid, ring, tp, c, smooth_w[k], n_omega[k], omega + f0,
                            d_omega + f0, data + 2 * NN * f0, tau, mode, prec,
                            residual_norms ? residual_norms + k : nullptr, k));
        f0 += (size_t)n_omega[k];
    }
    return RB_OK;
}

static void key_add(std::string &key, const void *p, size_t n) {
    key.append(static_cast<const char *>(p), n);
}

// Capture the sweep into a graph on the library stream; workspaces that must grow are grown
// outside the capture and the capture is redone.
static rb_status sweep_capture(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                               const rb_trace_params *tp, double *c, int32_t n_steps,
                               const int32_t *smooth_w, const int32_t *n_omega,
                               const double *omega, const double *d_omega, const float *data,
                               double tau, rb_mode mode, rb_prec prec, double *residual_norms,
                               hipGraphExec_t *exec) {
    if (!ctx->cap_stream)
        RB_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    for (int attempt = 0; attempt < 8; ++attempt) {
        hipStream_t user = ctx->stream;
        const bool prof = ctx->prof;
        ctx->stream = ctx->cap_stream;
        ctx->prof = false;
        ctx->capturing = true;
        rb_status st = RB_OK;
        hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess)
            st = sweep_enqueue(ctx, grid, ring, tp, c, n_steps, smooth_w, n_omega, omega,
                               d_omega, data, tau, mode, prec, residual_norms);
        hipGraph_t graph = nullptr;
        hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(ctx->cap_stream, &graph) : e;
        ctx->capturing = false;
        ctx->stream = user;
        ctx->prof = prof;
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            return rb_fail(ctx, RB_EDEVICE, "graph capture failed: %s",
                           hipGetErrorString(e != hipSuccess ? e : e2));
        }
        if (st == RB_ERETRY) {
            (void)hipGraphDestroy(graph);
            RB_TRY(rb_arena_reserve(ctx, &ctx->ws, ctx->ws.want));
            RB_TRY(rb_arena_reserve(ctx, &ctx->step, ctx->step.want));
            continue;
        }
        if (st != RB_OK) {
            (void)hipGraphDestroy(graph);
            return st;
        }
        hipError_t e3 = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess)
            return rb_fail(ctx, RB_EDEVICE, "graph instantiation failed: %s",
                           hipGetErrorString(e3));
        return RB_OK;
    }
    return rb_fail(ctx, RB_EDEVICE, "graph capture did not settle its workspace");
}

rb_status rb_frequency_sweep(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                             const rb_trace_params *tp, double *c, int32_t n_steps,
                             const int32_t *smooth_w, const int32_t *n_omega,
                             const double *omega, const double *d_omega, const float *data,
                             double tau, rb_mode mode, rb_prec prec, int32_t use_graph,
                             double *residual_norms) {
    if (!ctx) return RB_EINVAL;
    if (n_steps < 1 || !smooth_w || !n_omega)
        return rb_fail(ctx, RB_EINVAL, "need n_steps >= 1 and host arrays smooth_w, n_omega");
    size_t f0 = 0;
    for (int k = 0; k < n_steps; ++k) {
        if (n_omega[k] < 1) return rb_fail(ctx, RB_EINVAL, "step %d has no frequency", k);
        RB_TRY(check_step_args(ctx, grid, ring, tp, c, smooth_w[k], n_omega[k],
                               omega ? omega + f0 : nullptr, d_omega ? d_omega + f0 : nullptr,
                               data, tau, mode, prec));
        f0 += (size_t)n_omega[k];
    }
    RB_HIP(ctx, hipSetDevice(ctx->device));
    RB_TRY(rb_prepare_grid(ctx, grid));
    ctx->deferred = true;
    rb_status st = RB_OK;
    if (use_graph) {
        std::string key;
        key_add(key, grid, sizeof(*grid));
        key_add(key, ring, sizeof(*ring));
        key_add(key, tp, sizeof(*tp));
        key_add(key, &c, sizeof(c));
        key_add(key, &n_steps, sizeof(n_steps));
        key_add(key, smooth_w, n_steps * sizeof(int32_t));
        key_add(key, n_omega, n_steps * sizeof(int32_t));
        key_add(key, omega, f0 * sizeof(double));
        key_add(key, d_omega, f0 * sizeof(double));
        key_add(key, &data, sizeof(data));
        key_add(key, &tau, sizeof(tau));
        key_add(key, &mode, sizeof(mode));
        key_add(key, &prec, sizeof(prec));
        key_add(key, &residual_norms, sizeof(residual_norms));
        std::string full = key;
        key_add(full, &ctx->gen, sizeof(ctx->gen));
        if (!ctx->gexec || ctx->gkey != full) {
            if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
            ctx->gexec = nullptr;
            ctx->gkey.clear();
            hipGraphExec_t exec = nullptr;
            st = sweep_capture(ctx, grid, ring, tp, c, n_steps, smooth_w, n_omega, omega, d_omega,
                               data, tau, mode, prec, residual_norms, &exec);
            if (st == RB_OK) {
                ctx->gexec = exec;
                ctx->gkey = key;
                key_add(ctx->gkey, &ctx->gen, sizeof(ctx->gen));
            }
        }
        if (st == RB_OK && hipGraphLaunch(ctx->gexec, ctx->stream) != hipSuccess) {
            (void)hipGetLastError();
            st = rb_fail(ctx, RB_EDEVICE, "graph launch failed");
        }
    } else {
        st = sweep_enqueue(ctx, grid, ring, tp, c, n_steps, smooth_w, n_omega, omega, d_omega,
                           data, tau, mode, prec, residual_norms);
    }
    ctx->deferred = false;
    if (st != RB_OK) return st;
    RB_HIP(ctx, hipMemcpyAsync(ctx->h_flag, ctx->d_flag, RB_W_COUNT * sizeof(int32_t),
                               hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->lost_nodes = ctx->h_flag[RB_W_LOST];
    ctx->ray_samples = *reinterpret_cast<const int64_t *>(ctx->h_flag + RB_W_SAMPLES);
    const int32_t fl = ctx->h_flag[RB_W_FLAGS];
    if (fl)
        return rb_fail(ctx, RB_ENONFINITE,
                       "step %d of the sweep failed (%s); c holds the model before it",
                       ctx->h_flag[RB_W_FAIL_STEP],
                       (fl & 1) ? "a ray did not reach the ring within max_steps"
                                : "non-finite model update");
    return RB_OK;
}

}  // extern "C"
