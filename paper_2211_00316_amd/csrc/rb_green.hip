// Green's-function assembly, residual, back-projection scaling and model update (gfx950).
//
// Eq. 2D_greens: g = A exp(i [phi + pi/4]) with A_geom = A_tab / sqrt(k0);
// Eq. phase-discretised: phi = omega T - (pi/2) K (lossless);
// Eq. greens-time-reversed: g_dagger = A^-1 exp(-i [phi + pi/4]);
// Eq. sound_speed_update2: angular weights |d gamma_e / d e| De (central difference over
// neighbouring transducers), pair weight |kbar| |d|kbar|/d omega| = (2k/c)(1 + u_e . u_r)
// split into the three operands H, H u_x, H u_y; scale S = (Domega/(2 pi)^3)(2k/c)/omega^2.
// Eq. residual: g_res = g - data; Section 3.4: m <- m + tau dm, c = m^-1/2 (FP64).
//
// These kernels are elementwise and bound by HBM bandwidth: each reads its table entries
// once and writes the operands with coalesced 8-byte stores; only the phase is in FP64.
#include "rb_internal.h"

namespace {

__device__ __forceinline__ double reduce_phase(double ph) {
    return ph - RB_TWO_PI * floor(ph / RB_TWO_PI);
}

// One thread per (transducer e, mask node q); grid.y = e.
// gs (nullable): per-node complex factor applied to G (the frequency step stores
// G sqrt(v), so that the Born term is the plain symmetric product); write_g = 0 skips G.
__global__ void __launch_bounds__(256) green_kernel(rb_tables tb, int N, int n_mask,
                                                    double omega, double c0,
                                                    const float2 *__restrict__ gs,
                                                    const float *__restrict__ gscale, int write_g,
                                                    float2 *__restrict__ G,
                                                    float2 *__restrict__ H) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    int e = blockIdx.y;
    if (q >= n_mask) return;
    size_t o = (size_t)e * n_mask + q;
    size_t plane = (size_t)N * n_mask;
    uint8_t f = tb.flags[o];
    if (!(f & 0x80)) {
        if (write_g) G[o] = make_float2(0.f, 0.f);
        H[o] = make_float2(0.f, 0.f);
        H[plane + o] = make_float2(0.f, 0.f);
        H[2 * plane + o] = make_float2(0.f, 0.f);
        return;
    }
    double k0 = omega / c0;
    double ph = reduce_phase(omega * tb.T[o] + 0.25 * RB_PI - (double)(f & 3) * 0.5 * RB_PI);
    float s, c;
    sincosf((float)ph, &s, &c);
    float A = tb.A[o];
    float sk = (float)sqrt(k0);
    float ga = A / sk;
    if (write_g) {
        float gr = ga * c, gi = ga * s;
        if (gs) {
            float2 f2 = gs[q];
            float sc = gscale[0];
            float tr = (gr * f2.x - gi * f2.y) * sc;
            gi = (gr * f2.y + gi * f2.x) * sc;
            gr = tr;
        }
        G[o] = make_float2(gr, gi);
    }

    // angular weight: angle between the ray directions of the neighbouring transducers
    int em = (e + N - 1) % N, ep = (e + 1) % N;
    size_t om = (size_t)em * n_mask + q, op = (size_t)ep * n_mask + q;
    bool vm = tb.flags[om] & 0x80, vp = tb.flags[op] & 0x80;
    float ux = tb.ux[o], uy = tb.uy[o];
    float a = 0.f;
    if (vm && vp) {
        float ax = tb.ux[om], ay = tb.uy[om], bx = tb.ux[op], by = tb.uy[op];
        a = 0.5f * fabsf(atan2f(ax * by - ay * bx, ax * bx + ay * by));
    } else if (vp) {
        float bx = tb.ux[op], by = tb.uy[op];
        a = fabsf(atan2f(ux * by - uy * bx, ux * bx + uy * by));
    } else if (vm) {
        float ax = tb.ux[om], ay = tb.uy[om];
        a = fabsf(atan2f(ax * uy - ay * ux, ax * ux + ay * uy));
    }
    float ha = a * sk / A;
    float hr = ha * c, hi = -ha * s;
    H[o] = make_float2(hr, hi);
    H[plane + o] = make_float2(hr * ux, hi * ux);
    H[2 * plane + o] = make_float2(hr * uy, hi * uy);
}

// R[e][r] = g_rx + d_born - data on valid pairs with e != r; sum |R|^2 into *norm. One
// workgroup per emitter row e: one atomic per row for the norm.
__global__ void __launch_bounds__(256) residual_kernel(const double *__restrict__ rx_T,
                                                       const float *__restrict__ rx_A,
                                                       const uint8_t *__restrict__ rx_flags,
                                                       int N, double omega, double c0,
                                                       const float2 *__restrict__ d_born,
                                                       const float2 *__restrict__ data,
                                                       float2 *__restrict__ R, double *norm) {
    __shared__ double red[4];
    const int e = blockIdx.x;
    const double isk = 1.0 / sqrt(omega / c0);
    double v = 0.0;
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        const size_t o = (size_t)e * N + r;
        const uint8_t f = rx_flags[o];
        float2 out = make_float2(0.f, 0.f);
        if ((f & 0x80) && r != e) {
            double ph =
                reduce_phase(omega * rx_T[o] + 0.25 * RB_PI - (double)(f & 3) * 0.5 * RB_PI);
            double sn, cs;
            sincos(ph, &sn, &cs);
            double a = (double)rx_A[o] * isk;
            double gr = a * cs, gi = a * sn;
            if (d_born) {
                gr += d_born[o].x;
                gi += d_born[o].y;
            }
            float2 dd = data[o];
            out = make_float2((float)(gr - dd.x), (float)(gi - dd.y));
        }
        R[o] = out;
        v += (double)out.x * out.x + (double)out.y * out.y;
    }
    if (norm) {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(norm, (red[0] + red[1]) + (red[2] + red[3]));
    }
}

__global__ void adjoint_finish_kernel(int n_mask, int mblocks, const float *__restrict__ parts,
                                      const float2 *__restrict__ w, float *__restrict__ grad) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    float sr = 0.f, si = 0.f;
    for (int b = 0; b < mblocks; ++b) {
        sr += parts[(size_t)b * n_mask + q];
        si += parts[(size_t)(mblocks + b) * n_mask + q];
    }
    float2 ww = w[q];
    grad[q] = ww.x * sr + ww.y * si;  // Re{ conj(w) (sr + i si) }
}

template <typename OutT>
__global__ void backproject_finish_kernel(int n_mask, int mblocks, const float *__restrict__ parts,
                                          const double *__restrict__ c_mask, double omega,
                                          double d_omega, OutT *__restrict__ dm, int accumulate) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    double sr = 0.0;
    for (int b = 0; b < mblocks; ++b) sr += (double)parts[(size_t)b * n_mask + q];
    double c = c_mask[q];
    double S = 2.0 * d_omega / (RB_TWO_PI * RB_TWO_PI * RB_TWO_PI * omega * c * c);
    double v = -S * sr;
    if (accumulate) v += (double)dm[q];
    dm[q] = (OutT)v;
}

// c at the mask nodes (double) gathered from the full map.
__global__ void gather_mask(const double *__restrict__ c, const int32_t *__restrict__ mask_index,
                            int n_mask, double *__restrict__ cq) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n_mask) cq[q] = c[mask_index[q]];
}

// sv = sqrt(w delta) at the mask nodes (complex: i sqrt(w |delta|) for delta < 0), with
// w = omega^2 h^2 and delta = m - m_s, where m_s = (n_s / c0)^2 is the squared slowness of
// the smoothed map the rays were traced on. Then sum_q G[e,q] v[q] G[r,q] with v = w delta
// is the symmetric product of G sv with itself.
__global__ void rough_part(const double *__restrict__ cq, const float *__restrict__ n_s,
                           const int32_t *__restrict__ mask_index, int n_mask, double c0,
                           double w, float2 *__restrict__ sv) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    double c = cq[q];
    double ns = (double)n_s[mask_index[q]];
    double v = w * (1.0 / (c * c) - ns * ns / (c0 * c0));
    float r = (float)sqrt(fabs(v));
    sv[q] = v >= 0.0 ? make_float2(r, 0.f) : make_float2(0.f, r);
}

// Absorbing media (Szabo's model, Section 2.2; Eq. scattering-potential): sv = sqrt(v) with
// v = Upsilon_m h^2 delta complex, Upsilon_m = omega c k~ = omega^2 z, z = 1 + omega^(y-1)
// c alpha0 (tan(pi y/2) + i) from the model's c and alpha0 at the node. The principal square
// root in the cancellation-free form; with alpha0 = 0 it is the lossless root.
__global__ void rough_part_lossy(const double *__restrict__ cq, const double *__restrict__ aq,
                                 const float *__restrict__ n_s,
                                 const int32_t *__restrict__ mask_index, int n_mask, double c0,
                                 double w, double wy1, double tanpy, float2 *__restrict__ sv) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    const double c = cq[q];
    const double ns = (double)n_s[mask_index[q]];
    const double delta = 1.0 / (c * c) - ns * ns / (c0 * c0);
    const double t = wy1 * c * aq[q];
    const double vr = w * (1.0 + t * tanpy) * delta, vi = w * t * delta;
    double sr = 0.0, si = 0.0;
    if (vi == 0.0) {
        const double r = sqrt(fabs(vr));
        if (vr >= 0.0) sr = r;
        else si = r;
    } else {
        const double m = sqrt(vr * vr + vi * vi);
        if (vr >= 0.0) {
            sr = sqrt(0.5 * (m + vr));
            si = vi / (2.0 * sr);
        } else {
            const double u = sqrt(0.5 * (m - vr));
            si = copysign(u, vi);
            sr = fabs(vi) / (2.0 * u);
        }
    }
    sv[q] = make_float2((float)sr, (float)si);
}

// Hessian-free direction of an absorbing medium (Eq. sound_speed_update2 with Section 3.4's
// d|kbar|/domega): S = Domega / (2 pi)^3 (2k/c + 2k y tan(pi y/2) omega^(y-1) alpha0)
// / (omega^2 z), k = omega/c + alpha0 tan(pi y/2) omega^y, z as in rough_part_lossy; S is
// complex and dm = -Re{S (sr + i si)} over the complex double sum of the contraction.
template <typename OutT>
__global__ void backproject_finish_lossy_kernel(int n_mask, int mblocks,
                                                const float *__restrict__ parts,
                                                const double *__restrict__ c_mask,
                                                const double *__restrict__ a_mask, double omega,
                                                double base, double tanpy, double wy, double wy1,
                                                double y, OutT *__restrict__ dm, int accumulate) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < mblocks; ++b) {
        sr += (double)parts[(size_t)b * n_mask + q];
        si += (double)parts[(size_t)(mblocks + b) * n_mask + q];
    }
    const double c = c_mask[q], a0 = a_mask[q];
    const double k = omega / c + a0 * tanpy * wy;
    const double s = base * (2.0 * k / c + 2.0 * k * (y * tanpy * wy1 * a0));  // base: Dw/(2pi)^3 w^2
    const double t = wy1 * c * a0;
    const double zr = 1.0 + t * tanpy, zi = t;
    const double iz = 1.0 / (zr * zr + zi * zi);
    const double Sr = s * zr * iz, Si = -s * zi * iz;
    double v = -(Sr * sr - Si * si);
    if (accumulate) v += (double)dm[q];
    dm[q] = (OutT)v;
}

// m <- m + tau dm (FP64); the candidate c is kept aside until every value is finite.
__global__ void update_kernel(const double *__restrict__ cq, const double *__restrict__ dm,
                              int n_mask, double tau, double *__restrict__ c_new, int *flag) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    double c = cq[q];
    double m = 1.0 / (c * c) + tau * dm[q];
    double cn = 1.0 / sqrt(m);
    if (!(m > 0.0) || !isfinite(cn)) atomicOr(flag, 2);
    c_new[q] = cn;
}

// Writes the new model on the mask; with `flag` (deferred checks) only while no error bit
// is set, so a failed step and every later one leave c as it was.
__global__ void commit_kernel(const double *__restrict__ c_new,
                              const int32_t *__restrict__ mask_index, int n_mask,
                              const int32_t *__restrict__ flag, double *__restrict__ c) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask || (flag && flag[RB_W_FLAGS] != 0)) return;
    c[mask_index[q]] = c_new[q];
}

// Deferred checks: remember the first step that raised an error bit.
__global__ void note_fail_kernel(int32_t *flag, int step) {
    if (threadIdx.x == 0 && flag[RB_W_FLAGS] != 0 && flag[RB_W_FAIL_STEP] < 0)
        flag[RB_W_FAIL_STEP] = step;
}

// Status of a step for the caller, from the context's device words (no host round trip).
__global__ void report_kernel(const int32_t *__restrict__ flag, rb_report *__restrict__ rep) {
    if (threadIdx.x != 0) return;
    const int32_t fl = flag[RB_W_FLAGS];
    rep->status = fl ? (int32_t)RB_ENONFINITE : (int32_t)RB_OK;
    rep->flags = fl;
    rep->lost_nodes = flag[RB_W_LOST];
    rep->reserved = 0;
    rep->ray_samples = *reinterpret_cast<const int64_t *>(flag + RB_W_SAMPLES);
}

__global__ void fill_i32(int32_t *x, int n, int32_t v) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) x[q] = v;
}

__global__ void zero_f64(double *x, int n) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) x[q] = 0.0;
}

inline unsigned blocks(size_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

rb_status rb_launch_green(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                          const rb_green *out, const float *gs, const float *gscale,
                          int write_g) {
    dim3 grd(blocks(tb->n_mask), tb->n);
    rb_prof_begin(ctx, ST_GREEN);
    hipLaunchKernelGGL(green_kernel, grd, dim3(256), 0, ctx->stream, *tb, tb->n, tb->n_mask, omega,
                       c0, (const float2 *)gs, gscale, write_g, (float2 *)out->G,
                       (float2 *)out->H);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_residual(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                             const float *d_born, const float *data, float *R,
                             double *residual_norm) {
    rb_prof_begin(ctx, ST_RESIDUAL);
    hipLaunchKernelGGL(residual_kernel, dim3(tb->n), dim3(256), 0, ctx->stream, tb->rx_T, tb->rx_A,
                       tb->rx_flags, tb->n, omega, c0, (const float2 *)d_born,
                       (const float2 *)data, (float2 *)R, residual_norm);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_adjoint_finish(rb_ctx *ctx, int n_mask, int mblocks, const float *parts,
                                   const float *w, float *grad) {
    rb_prof_begin(ctx, ST_FINISH);
    hipLaunchKernelGGL(adjoint_finish_kernel, dim3(blocks(n_mask)), dim3(256), 0, ctx->stream,
                       n_mask, mblocks, parts, (const float2 *)w, grad);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_backproject_finish(rb_ctx *ctx, int n_mask, int mblocks, const float *parts,
                                       const double *c_mask, double omega, double d_omega,
                                       float *dm, int accumulate) {
    rb_prof_begin(ctx, ST_FINISH);
    hipLaunchKernelGGL(backproject_finish_kernel<float>, dim3(blocks(n_mask)), dim3(256), 0,
                       ctx->stream, n_mask, mblocks, parts, c_mask, omega, d_omega, dm,
                       accumulate);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

// Internal helpers of rb_frequency_step --------------------------------------------------
rb_status rb_launch_gather_mask(rb_ctx *ctx, const double *c, double *cq) {
    int n = (int)ctx->n_mask;
    hipLaunchKernelGGL(gather_mask, dim3(blocks(n)), dim3(256), 0, ctx->stream, c,
                       ctx->d_mask_index, n, cq);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_rough_part(rb_ctx *ctx, const double *cq, const float *n_s, double c0,
                               double w, float *sv) {
    int n = (int)ctx->n_mask;
    hipLaunchKernelGGL(rough_part, dim3(blocks(n)), dim3(256), 0, ctx->stream, cq, n_s,
                       ctx->d_mask_index, n, c0, w, (float2 *)sv);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_backproject_finish_acc(rb_ctx *ctx, int mblocks, const float *parts,
                                           const double *c_mask, double omega, double d_omega,
                                           double *dm_acc) {
    int n = (int)ctx->n_mask;
    rb_prof_begin(ctx, ST_FINISH);
    hipLaunchKernelGGL(backproject_finish_kernel<double>, dim3(blocks(n)), dim3(256), 0,
                       ctx->stream, n, mblocks, parts, c_mask, omega, d_omega, dm_acc, 1);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_rough_part_lossy(rb_ctx *ctx, const double *cq, const double *aq,
                                     const float *n_s, double c0, double omega, double y,
                                     double h2, float *sv) {
    int n = (int)ctx->n_mask;
    hipLaunchKernelGGL(rough_part_lossy, dim3(blocks(n)), dim3(256), 0, ctx->stream, cq, aq, n_s,
                       ctx->d_mask_index, n, c0, omega * omega * h2, pow(omega, y - 1.0),
                       tan(0.5 * RB_PI * y), (float2 *)sv);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_backproject_finish_lossy(rb_ctx *ctx, int n_mask, int mblocks,
                                             const float *parts, const double *c_mask,
                                             const double *a_mask, double omega, double d_omega,
                                             double y, double *dm_acc, float *dm,
                                             int accumulate) {
    const double base = d_omega / (RB_TWO_PI * RB_TWO_PI * RB_TWO_PI) / (omega * omega);
    const double tanpy = tan(0.5 * RB_PI * y), wy = pow(omega, y), wy1 = pow(omega, y - 1.0);
    rb_prof_begin(ctx, ST_FINISH);
    if (dm_acc)
        hipLaunchKernelGGL(backproject_finish_lossy_kernel<double>, dim3(blocks(n_mask)),
                           dim3(256), 0, ctx->stream, n_mask, mblocks, parts, c_mask, a_mask,
                           omega, base, tanpy, wy, wy1, y, dm_acc, 1);
    else
        hipLaunchKernelGGL(backproject_finish_lossy_kernel<float>, dim3(blocks(n_mask)),
                           dim3(256), 0, ctx->stream, n_mask, mblocks, parts, c_mask, a_mask,
                           omega, base, tanpy, wy, wy1, y, dm, accumulate);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_zero_f64(rb_ctx *ctx, double *x, int n) {
    hipLaunchKernelGGL(zero_f64, dim3(blocks(n)), dim3(256), 0, ctx->stream, x, n);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_update(rb_ctx *ctx, const double *cq, const double *dm, double tau,
                           double *c_new) {
    int n = (int)ctx->n_mask;
    rb_prof_begin(ctx, ST_UPDATE);
    hipLaunchKernelGGL(update_kernel, dim3(blocks(n)), dim3(256), 0, ctx->stream, cq, dm, n, tau,
                       c_new, ctx->d_flag);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_commit(rb_ctx *ctx, const double *c_new, double *c, const int32_t *flag) {
    int n = (int)ctx->n_mask;
    hipLaunchKernelGGL(commit_kernel, dim3(blocks(n)), dim3(256), 0, ctx->stream, c_new,
                       ctx->d_mask_index, n, flag, c);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_note_fail(rb_ctx *ctx, int step) {
    hipLaunchKernelGGL(note_fail_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->d_flag, step);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_report(rb_ctx *ctx, rb_report *rep) {
    hipLaunchKernelGGL(report_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->d_flag, rep);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_fill_i32(rb_ctx *ctx, int32_t *x, int n, int32_t value) {
    hipLaunchKernelGGL(fill_i32, dim3(blocks(n)), dim3(256), 0, ctx->stream, x, n, value);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}
