// Internal declarations shared by the raybornhf HIP sources (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "raybornhf.h"

#define RB_PI 3.14159265358979323846
#define RB_TWO_PI 6.28318530717958647692

// Device workspace owned by a context: one growing allocation, carved into aligned parts.
struct rb_arena {
    char *base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    size_t want = 0;  // largest size asked for during a graph capture
};

// Internal status (never returned through the ABI): a workspace had to grow while a graph
// was being captured; the capture is discarded, the workspace grown, and the capture redone.
#define RB_ERETRY ((rb_status)-100)

// Workgroups (and partial maxima) of a range-scale reduction.
#define RB_RED_PARTS 512

// Ray linking: a linked ray further from its receiver than this (radians of exit angle) is
// not accepted.
#define RB_LINK_ACCEPT 1e-6

// Node tile of one binning-walk workgroup (the walk's starting offsets are per tile).
#define RB_WALK_TX 16
#define RB_WALK_TY 16

// Scratch bytes of the allocation-free back-projection (one device array per GPU).
#define RB_SCRATCH_BYTES ((size_t)64 << 20)

// Scans one batch (and one grouped launch) may hold.
#define RB_GROUP_MAX 16

// Words of rb_ctx::d_flag: error bits (1 ray overflow, 2 non-finite update), index of the
// first failing step of a sweep, mask nodes the binning could not place, and (as int64 at
// word 4) the ray samples of the last trace.
enum { RB_W_FLAGS = 0, RB_W_FAIL_STEP = 1, RB_W_LOST = 2, RB_W_SAMPLES = 4, RB_W_COUNT = 8 };

struct rb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char err[512] = {0};

    // geometry cache: mask node list and node -> mask index map of the last grid seen
    rb_grid grid{};
    bool have_grid = false;
    int64_t n_mask = 0;
    int32_t *d_mask_index = nullptr;  // [n_mask] flat node index of each mask node
    int32_t *d_qmap = nullptr;        // [nx*ny] mask index of each node, -1 outside
    int2 *d_qrow = nullptr;           // [ny] mask row: (first | last << 16, index - i)
    int tile_i0 = 0, tile_j0 = 0;     // walk tiles (RB_WALK_TX x RB_WALK_TY nodes) over the mask bbox
    int tiles_x = 0, tiles_y = 0;

    // per-stage event timing (rb_profile_enable / rb_profile_read)
    bool prof = false;
    static constexpr int kMaxEv = 8192;
    hipEvent_t ev[kMaxEv][2] = {};
    int ev_stage[kMaxEv] = {0};
    int n_ev = 0, n_ev_created = 0;

    rb_arena ws;                      // scratch of the current call
    rb_arena step;                    // persistent buffers of rb_frequency_step
    rb_arena gn;                      // per-frequency operands and CG state of a Gauss-Newton step
    int32_t *d_flag = nullptr;        // device words RB_W_* (flags, counters)
    float *d_red = nullptr;           // [RB_RED_PARTS] per-block partials of range scales
    int32_t *h_flag = nullptr;        // pinned host mirror of d_flag
    int64_t lost_nodes = 0;           // mask nodes the last binning could not place
    int64_t ray_samples = 0;          // ray samples written by the last trace
    // Bytes of ray samples one tracer launch may hold: a quarter of the device memory free
    // when the context was created, at most 48 GiB. All transducers in one launch keeps the
    // GPU full until the longest rays finish (one chunk at N = 1024 on a 288 GB device).
    size_t sample_budget = (size_t)6 << 30;
    int n_cu = 256;                   // compute units of the device (persistent grids)

    // Deferred checks (rb_frequency_sweep): no host synchronisation inside a step; errors
    // stay in d_flag and the commit kernel skips the update once any is set.
    bool deferred = false;
    bool capturing = false;           // a graph capture is in progress on `stream`
    // rb_reserve: workspaces are fixed (no allocation, free or host wait after it); a call
    // needing more fails with RB_ENOMEM, a call on another grid with RB_EINVAL
    bool fixed = false;
    uint64_t gen = 0;                 // bumped whenever a device buffer is reallocated
    hipStream_t cap_stream = nullptr; // library stream the sweep is captured on
    hipGraphExec_t gexec = nullptr;   // cached sweep graph
    hipEvent_t ev_join = nullptr;     // orders this context's stream in a batch
    // Receiver tables by secant ray linking (rb_set_receiver_linking): traced rays per pair
    // (0: interpolation in exit angle over the fan) and the exit-angle tolerance (radians).
    int link_iter = 0;
    double link_tol = 1e-8;
    static constexpr int kMaxTune = 16;
    rb_tuning tune[kMaxTune] = {};    // forward launch configurations (rb_autotune), by shape
    int n_tune = 0;
    std::string gkey;                 // the arguments (and gen) it was captured with
};

// Stages timed by the profiler (order = rb_stage_name).
enum rb_stage {
    ST_SMOOTH = 0, ST_TRACE, ST_RASTER, ST_RESOLVE, ST_RECEIVERS, ST_GREEN, ST_FORWARD,
    ST_FORWARD_REDUCE, ST_RESIDUAL, ST_BACKPROJECT, ST_FINISH, ST_UPDATE
};
// Gauss-Newton step (rb_gn.hip) ----------------------------------------------------------
// Analytic water tables: the C-ABI tables (rec == NULL) or compact records, the receiver
// tables, transducer positions and (nullable) the rows' amplitude maxima.
rb_status rb_launch_water_tables(rb_ctx *ctx, const rb_ring *ring, double c0,
                                 const rb_tables *tb, float4 *rec, double2 *ringpos,
                                 unsigned int *rowmax);
// delta = m - m_s on the mask nodes (n_s NULL: m_s = c0^-2).
rb_status rb_launch_gn_delta(rb_ctx *ctx, const double *cq, const float *n_s, double c0,
                             float *delta);
rb_status rb_launch_gn_weight(rb_ctx *ctx, float *w, int n, double value);
rb_status rb_launch_gn_mask_pairs(rb_ctx *ctx, float *d, const uint8_t *rx_flags, int N);
rb_status rb_launch_gn_adjoint_acc(rb_ctx *ctx, int mblocks, const float *parts, const float *w,
                                   double *acc, int first);
size_t rb_gn_scalar_bytes();
// op 0: start from grad (norms[k] = |r_0|); op 1: the update after H p (norms[k] = |r_k|).
rb_status rb_launch_gn_cg(rb_ctx *ctx, int op, double *x, double *r, double *p, double *hp,
                          float *pf, const double *grad, double *scal, double *norms, int k);

// Copy the context's status words into a caller's device rb_report (one small kernel).
rb_status rb_launch_report(rb_ctx *ctx, rb_report *rep);
// Fill n int32 words with a value (a kernel: also inside graph captures).
rb_status rb_launch_fill_i32(rb_ctx *ctx, int32_t *x, int n, int32_t value);
// Record the start / end event of a launch of `stage` (no-ops unless profiling is on).
void rb_prof_begin(rb_ctx *ctx, int stage);
void rb_prof_end(rb_ctx *ctx);

// Error reporting -------------------------------------------------------------------------
rb_status rb_fail(rb_ctx *ctx, rb_status st, const char *fmt, ...);

#define RB_HIP(ctx, call)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return rb_fail((ctx), RB_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define RB_CHECK_LAUNCH(ctx) RB_HIP(ctx, hipGetLastError())

#define RB_TRY(x)                       \
    do {                                \
        rb_status s_ = (x);             \
        if (s_ != RB_OK) return s_;     \
    } while (0)

// Workspace -------------------------------------------------------------------------------
// Ensure the arena holds at least `bytes` (reallocates, dropping old contents).
rb_status rb_arena_reserve(rb_ctx *ctx, rb_arena *a, size_t bytes);
inline size_t rb_align(size_t x) { return (x + 255) & ~size_t(255); }

// Operand types: valid values of rb_prec, and the split form (FP16 operands with the
// back-projection operand H stored as a high and a low FP16 part).
inline bool rb_prec_valid(int p) {
    return p == RB_F32 || p == RB_BF16 || p == RB_F16 || p == RB_F16X;
}
inline bool rb_prec_split(int p) { return p == RB_F16X; }

// Transducer dimension of the 16-bit operand rows (H, residual): a whole number of 32-deep
// contraction steps, zeros past n.
__host__ __device__ inline int rb_lp_pad(int n) { return (n + 31) & ~31; }
// Row length of the 8-bit operand planes of the split back-projection (K steps of 64 bytes).
__host__ __device__ inline int rb_lp8_pad(int n) { return (n + 63) & ~63; }
template <typename T> T *rb_carve(rb_arena *a, size_t count) {
    T *p = reinterpret_cast<T *>(a->base + a->used);
    a->used += rb_align(count * sizeof(T));
    return p;
}

// Geometry --------------------------------------------------------------------------------
rb_status rb_check_grid(rb_ctx *ctx, const rb_grid *g);
rb_status rb_check_ring(rb_ctx *ctx, const rb_grid *g, const rb_ring *r);
rb_status rb_check_trace(rb_ctx *ctx, const rb_trace_params *tp);
// Upload the mask list for this grid if it differs from the cached one.
rb_status rb_prepare_grid(rb_ctx *ctx, const rb_grid *g);

// Stage launchers (each validates nothing; callers have validated) -------------------------
rb_status rb_launch_refractive_index(rb_ctx *ctx, const rb_grid *g, const double *c, double c0,
                                     int w, float *n_s);
// Trace and bin. The receiver tables always go to `out`. The node tables go to `out` as well
// unless `rec` is given ([n][n_mask] float4, inside a frequency step): then each
// (transducer, node) gets one compact record (dT, A, theta, flags) with dT = T - d / c0 (d:
// distance from the transducer, recomputed by the reader), theta = atan2(u_y, u_x) and the
// flag bits of rb_tables stored as the bits of the fourth float. ring_out (nullable, double2
// [n]) receives the transducer positions. rowmax (nullable, with rec; [n][2]) receives for
// each transducer the bits of the largest A and of the largest 1/A over its valid records.
// a_w (nullable, float [ny][nx]): absorption map alpha (Np/m) of an absorbing medium; its
// line integral along each ray is subtracted from the log-amplitude (A = A_geom A_abs).
rb_status rb_launch_trace(rb_ctx *ctx, const rb_grid *g, const rb_ring *r,
                          const rb_trace_params *tp, const float *n_s, const rb_tables *out,
                          float4 *rec = nullptr, double2 *ring_out = nullptr,
                          unsigned int *rowmax = nullptr, const float *a_w = nullptr);
// Absorbing media (Szabo's model): row passes of the box window over c0/c (tn) and alpha0
// (ta), double [ny][nx] each, and n_s = box(c0/c); then per frequency the traced map
// n_w = box(c0/c) + kd box(alpha0) and the absorption map a_w = ky box(alpha0) (float),
// kd = c0 tan(pi y/2) omega^(y-1), ky = omega^y.
rb_status rb_launch_lossy_rows(rb_ctx *ctx, const rb_grid *g, const double *c, double c0,
                               const double *alpha0, int w, double *tn, double *ta,
                               float *n_s);
rb_status rb_launch_lossy_map(rb_ctx *ctx, const rb_grid *g, const double *tn, const double *ta,
                              int w, double kd, double ky, float *n_w, float *a_w);
// Lossy scattering potential and back-projection weight (rb_green.hip): sv = sqrt(v) with
// v = Upsilon_m h^2 (m - m_s), Upsilon_m = omega^2 [1 + omega^(y-1) c alpha0 (tan + i)];
// the finish with the complex weight S (accumulating into dm_acc, or into/over float dm).
rb_status rb_launch_rough_part_lossy(rb_ctx *ctx, const double *cq, const double *aq,
                                     const float *n_s, double c0, double omega, double y,
                                     double h2, float *sv);
rb_status rb_launch_backproject_finish_lossy(rb_ctx *ctx, int n_mask, int mblocks,
                                             const float *parts, const double *c_mask,
                                             const double *a_mask, double omega, double d_omega,
                                             double y, double *dm_acc, float *dm,
                                             int accumulate);
// gs (nullable): complex per-node factor on G; write_g = 0 leaves G unwritten.
rb_status rb_launch_green(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                          const rb_green *out, const float *gs, const float *gscale,
                          int write_g);
rb_status rb_launch_residual(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                             const float *d_born, const float *data, float *R,
                             double *residual_norm);
// w, delta nullable together: then v = 1 (the operand already carries the node weights).
// gscale (nullable, device): the operand carries sqrt(v) gscale[0]; d is divided by
// gscale[0]^2 (multiplied by gscale[1]^2).
rb_status rb_launch_forward(rb_ctx *ctx, const rb_green *gr, const float *w, const float *delta,
                            float *d, const float *gscale);
// Row-reduced complex GEMM: parts[2][mblocks][n_mask] (re, im) of
// sum_e E_c[e][q] (R B_c)[e][q] summed over the n_comp components c (E_c = B_c, conjugated
// with conj_b). rsym: workspace of n x n complex64 for the block upper triangle of the
// symmetric part of R (rb_gemm.hip).
rb_status rb_launch_rowred(rb_ctx *ctx, int n, int n_mask, const float *R, const float *B,
                           int n_comp, int conj_b, float *rsym, float *parts, int *mblocks);
rb_status rb_launch_adjoint_finish(rb_ctx *ctx, int n_mask, int mblocks, const float *parts,
                                   const float *w, float *grad);
rb_status rb_launch_backproject_finish(rb_ctx *ctx, int n_mask, int mblocks, const float *parts,
                                       const double *c_mask, double omega, double d_omega,
                                       float *dm, int accumulate);
int rb_rowred_mblocks(int n);
// Workspace bytes the FP32 forward of n transducers over n_mask nodes reserves.
size_t rb_forward_ws_bytes(int n, int n_mask);
// Workspace bytes of one tracer launch under a sample budget (tiles: walk tiles).
size_t rb_trace_ws_bytes(const rb_grid *g, const rb_ring *r, const rb_trace_params *tp,
                         int64_t n_mask, size_t tiles, size_t sample_budget);

// Reduced-precision (BF16 / FP16 operand) form: layouts in rb_lowp.hip.
// Writes out->scales (per-row powers of two) with the operands; rowmax: workspace of [n][2]
// words for the tables' row maxima.
rb_status rb_launch_green_lp(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                             const rb_green *out, const float *gs, const float *gscale,
                             int write_g, unsigned int *rowmax);
// The same from the compact records of rb_launch_trace (ring: transducer positions; rowmax:
// the binning's per-row amplitude maxima), for the frequency step's back-projection: the
// three operand components are the rotated ones, H, b = H (u_x - i u_y) and a = H (u_x +
// i u_y) (a^T Rs b = (H u_x)^T Rs (H u_x) + (H u_y)^T Rs (H u_y)). In the split form the low
// parts of H, b and a, times 2^6, are FP8 (E4M3) at the start of the three low-part slots,
// each [2][rb_lp8_pad(n) / 64][n_mask][64] (blocks of 64 transducers, node-major inside).
rb_status rb_launch_green_lp_rec(rb_ctx *ctx, const float4 *rec, const double2 *ring, int n,
                                 double omega, double c0, const rb_green *out, const float *gs,
                                 const float *gscale, int write_g, const unsigned int *rowmax);
// R -> planar 16-bit operand of the back-projection: the block upper triangle of the
// symmetric part of R (the bilinear forms h^T R h see nothing else; rb_lowp.hip), divided by
// rows[e] rows[r] (the per-row scales of the other operand; nullable) and scaled by a power
// of two kept in scale[0..1] (device, 2 floats).
// R8 (nullable, split form of the frequency step): also the symmetric part Rs in FP8 (E4M3)
// planes [2][n][rb_lp8_pad(n)] (zero past n), at the 16-bit operand's scale times 2^-6.
// Rfull (nullable, plain 16-bit forms of the frequency step): also the whole Rs as 16-bit
// planes like Rp (the operand of the rotated bilinear form).
rb_status rb_launch_to_planar(rb_ctx *ctx, rb_prec prec, const float *R, int n, void *Rp,
                              float *scale, const float *rows, void *R8 = nullptr,
                              void *Rfull = nullptr);
rb_status rb_launch_unscale(rb_ctx *ctx, float *parts, size_t count, const float *scale);
// 16-bit G [2][n][m_pad] -> conj(G) node-major [2][n_mask][n_pad] (operand of the adjoint).
rb_status rb_launch_transpose_conj(rb_ctx *ctx, const rb_green *gr, void *Gt);
// Hlo (nullable): low parts of a split operand (RB_F16X), added with weight 2 in the epilogue.
// Rf (nullable, with the frequency step's operands H, b, a of rb_launch_green_lp_rec): the
// rotated form, two contractions (n_comp is then 2): h^T R h over Rp, then a^T Rs b with Rs
// = Rf (the whole symmetric part; Rp itself in the split form, whose low parts Hlo and FP8
// Rs R8 it also takes).
rb_status rb_launch_rowred_lp(rb_ctx *ctx, rb_prec prec, int n, int n_mask, const void *Rp,
                              const void *Ht, int n_comp, float *parts, int *mblocks,
                              const void *Hlo = nullptr, const void *R8 = nullptr,
                              const void *Rf = nullptr);
rb_status rb_launch_forward_lp(rb_ctx *ctx, const rb_green *gr, const float *w,
                               const float *delta, float *d, const float *gscale);

// Grouped launches (rb_frequency_step_batch): the contractions of several scans in one launch,
// each problem computing exactly what its single launch computes.
struct rb_rowred_prob {
    const void *Rp;   // planar 16-bit block upper triangle of R (rb_launch_to_planar)
    const void *Ht;   // 16-bit H planes of the green record
    float *parts;     // [2][mblocks][n_mask] partial sums
    int n, n_mask;
    const void *Hlo;  // low parts of H (split form) or NULL
    const void *R8;   // FP8 planes of Rs (rotated split form) or NULL
    const void *Rf;   // 16-bit planes of the whole Rs (rotated forms) or NULL
};
rb_status rb_launch_rowred_lp_group(rb_ctx *ctx, rb_prec prec, const rb_rowred_prob *probs,
                                    int count, int n_comp);
// Launch plan of the pipelined forward on operands that carry sqrt(v) (w = delta = NULL):
// tiles, K split and partial-sum buffer (in the workspace of the context that planned it).
struct rb_fwd_plan {
    rb_green gr;
    const float *gscale;
    bool pipe;  // the pipelined kernel applies (G's planes fit one buffer descriptor)
    int n, ld, nT, tiles, kchunk, splitk;
    unsigned nblk;
    float2 *dpart;
    float *vscale;
};
rb_status rb_forward_lp_plan(rb_ctx *ctx, const rb_green *gr, const float *gscale,
                             rb_fwd_plan *plan);
// Plans of pipe == true, one prec; the range-scale factors of each plan are applied first.
rb_status rb_launch_forward_lp_group(rb_ctx *ctx, rb_prec prec, const rb_fwd_plan *plans,
                                     int count);
rb_status rb_forward_lp_reduce(rb_ctx *ctx, const rb_fwd_plan *plan, float *d);
// Workspace bytes the forward of n transducers over n_mask nodes reserves (at most, over
// the configurations the autotuner may choose).
size_t rb_forward_lp_ws_bytes(int n, int n_mask, int n_cu);
// K splits the autotuner tries besides the built-in choice.
#define RB_TUNE_SPLITK_MAX 64
// The context's tuning if it applies to this shape and precision, else NULL.
inline const rb_tuning *rb_tuned(const rb_ctx *ctx, int n, int n_mask, rb_prec prec) {
    for (int i = 0; i < ctx->n_tune; ++i)
        if (ctx->tune[i].n == n && ctx->tune[i].n_mask == n_mask && ctx->tune[i].prec == prec)
            return &ctx->tune[i];
    return nullptr;
}
// Seeded operand values of the shape of gr (autotuner input) and gscale = {1, 1}.
rb_status rb_launch_tune_fill(rb_ctx *ctx, const rb_green *gr, float *gscale);
// Built-in K splits of the forwards (the autotuner's reference candidates).
int rb_forward_lp_default_splitk(int n, int n_mask, int pipe, int n_cu);
int rb_forward_default_splitk(int n, int n_mask);
// scale[0] = 2^(top - e), scale[1] = 1 / scale[0] with 2^(e-1) <= max |x| < 2^e (complex x).
rb_status rb_launch_range_scale(rb_ctx *ctx, const float *x, size_t count, int top, float *scale);
int rb_rowred_lp_mblocks(int n);
