// Gauss-Newton inversion of one frequency set (Section 6.3.2 b: the Hessian-based ray-Born
// method; c: the prototype Born method with the Green's functions of water): conjugate
// gradients on the Hessian action H x = Re sum_w J_w^H J_w x (Eq. hessian-action, Q = 1)
// against the gradient Re sum_w J_w^H g_res,w (Eq. functional-gradient). J_w is the Born
// operator of Eqs. perturb1 and derivative on the kept emitter-receiver pairs; both products
// reuse the contractions of the Hessian-free step (the weighted forward, and the
// one-component row-reduced product as the adjoint). This file holds the kernels the
// iteration adds: the analytic tables of water, the rough part of the model, the pair mask,
// the FP64 accumulation of the adjoint, and the CG vector updates with their scalars kept on
// the device (no host round trip inside the iteration).
#include "rb_internal.h"

#include <algorithm>

namespace {

inline unsigned blocks_of(size_t n) { return (unsigned)((n + 255) / 256); }

__global__ void gn_ring_positions(double R, double psi0, int N, double2 *pos) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < N) {
        const double psi = psi0 + RB_TWO_PI * (double)e / (double)N;
        pos[e] = make_double2(R * cos(psi), R * sin(psi));
    }
}

// Water (App. B): straight rays, T = d / c0, A = (8 pi d)^-1/2 (amplitude times sqrt(k0)),
// direction along x - x_e, no caustics; every mask node is valid. Writes the tables of the
// C ABI (FP32 form) or the compact records (16-bit form: dT = 0, A, ray angle, flags).
__global__ void __launch_bounds__(256) water_nodes(const int32_t *__restrict__ mask_index,
                                                   double x0, double y0, double dx, int nx,
                                                   int n_mask, const double2 *__restrict__ ring,
                                                   double c0, rb_tables tb,
                                                   float4 *__restrict__ rec) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
    if (q >= n_mask) return;
    const int p = mask_index[q];
    const double2 xe = ring[e];
    const double ddx = x0 + (p % nx) * dx - xe.x, ddy = y0 + (p / nx) * dx - xe.y;
    const double d = sqrt(ddx * ddx + ddy * ddy);
    const float A = (float)(1.0 / sqrt(8.0 * RB_PI * d));
    const size_t o = (size_t)e * n_mask + q;
    if (rec) {
        rec[o] = make_float4(0.f, A, (float)atan2(ddy, ddx), __int_as_float(0x80));
        return;
    }
    tb.T[o] = d / c0;
    tb.A[o] = A;
    tb.ux[o] = (float)(ddx / d);
    tb.uy[o] = (float)(ddy / d);
    tb.flags[o] = 0x80;
}

__global__ void water_receivers(const double2 *__restrict__ ring, int N, double c0, rb_tables tb) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
    if (r >= N) return;
    const size_t o = (size_t)e * N + r;
    if (r == e) {
        tb.rx_T[o] = 0.0;
        tb.rx_A[o] = 0.f;
        tb.rx_flags[o] = 0;
        return;
    }
    const double ddx = ring[r].x - ring[e].x, ddy = ring[r].y - ring[e].y;
    const double d = sqrt(ddx * ddx + ddy * ddy);
    tb.rx_T[o] = d / c0;
    tb.rx_A[o] = (float)(1.0 / sqrt(8.0 * RB_PI * d));
    tb.rx_flags[o] = 0x80;
}

// Largest A and 1/A of each transducer's water records (one workgroup per transducer), the
// row maxima the 16-bit operand scales come from.
__global__ void __launch_bounds__(256) water_rowmax(const int32_t *__restrict__ mask_index,
                                                    double x0, double y0, double dx, int nx,
                                                    int n_mask, const double2 *__restrict__ ring,
                                                    unsigned int *__restrict__ rowmax) {
    __shared__ double red[2][4];
    const int e = blockIdx.x;
    const double2 xe = ring[e];
    double dmin = 1e300, dmax = 0.0;
    for (int q = threadIdx.x; q < n_mask; q += blockDim.x) {
        const int p = mask_index[q];
        const double ddx = x0 + (p % nx) * dx - xe.x, ddy = y0 + (p / nx) * dx - xe.y;
        const double d = sqrt(ddx * ddx + ddy * ddy);
        dmin = fmin(dmin, d);
        dmax = fmax(dmax, d);
    }
    for (int o = 32; o > 0; o >>= 1) {
        dmin = fmin(dmin, __shfl_xor(dmin, o));
        dmax = fmax(dmax, __shfl_xor(dmax, o));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = dmin;
        red[1][threadIdx.x >> 6] = dmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        dmin = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
        dmax = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        // the records' A is rounded to float: bound it from above
        rowmax[2 * e] = __float_as_uint((float)(1.0 / sqrt(8.0 * RB_PI * dmin)) * 1.0000002f);
        rowmax[2 * e + 1] = __float_as_uint((float)sqrt(8.0 * RB_PI * dmax) * 1.0000002f);
    }
}

// delta = m - m_s at the mask nodes: the part of the model the Green's functions do not see
// (m_s = (n_s / c0)^2 of the traced map, or c0^-2 for water).
__global__ void gn_delta(const double *__restrict__ cq, const float *__restrict__ n_s,
                         const int32_t *__restrict__ mask_index, int n_mask, double c0,
                         float *__restrict__ delta) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    const double c = cq[q];
    double ms = 1.0 / (c0 * c0);
    if (n_s) {
        const double n = (double)n_s[mask_index[q]];
        ms = n * n / (c0 * c0);
    }
    delta[q] = (float)(1.0 / (c * c) - ms);
}

__global__ void gn_fill_weight(float2 *__restrict__ w, int n, float v) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) w[q] = make_float2(v, 0.f);
}

// J x on the kept pairs only: zero where the residual is zero (e = r, or no valid receiver).
__global__ void gn_mask_pairs(float2 *__restrict__ d, const uint8_t *__restrict__ rx_flags,
                              int N) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
    if (r >= N) return;
    const size_t o = (size_t)e * N + r;
    if (r == e || !(rx_flags[o] & 0x80)) d[o] = make_float2(0.f, 0.f);
}

// acc[q] (+)= Re{ conj(w[q]) sum_b parts } in FP64: the Q = 1 adjoint summed over frequencies.
__global__ void gn_adjoint_acc(int n_mask, int mblocks, const float *__restrict__ parts,
                               const float2 *__restrict__ w, double *__restrict__ acc,
                               int first) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_mask) return;
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < mblocks; ++b) {
        sr += (double)parts[(size_t)b * n_mask + q];
        si += (double)parts[(size_t)(mblocks + b) * n_mask + q];
    }
    const float2 ww = w[q];
    const double v = (double)ww.x * sr + (double)ww.y * si;
    acc[q] = first ? v : acc[q] + v;
}

// CG scalars (device doubles): rr = r.r of the current iterate, alpha, beta.
// S_STOP: the iteration has ended (converged, or p.Hp not positive); later iterations keep x.
enum { S_RR = 0, S_ALPHA = 1, S_BETA = 2, S_STOP = 3, S_COUNT = 4 };
constexpr int DOT_BLOCKS = 256;

__global__ void __launch_bounds__(256) gn_dot_part(const double *__restrict__ a,
                                                   const double *__restrict__ b, int n,
                                                   double *__restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        s += a[i] * b[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__device__ double sum_parts(const double *__restrict__ part) {
    __shared__ double red[4];
    double s = part[threadIdx.x];  // DOT_BLOCKS == blockDim.x
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// r = -grad, p = r, x = 0, pf = (float) p
__global__ void gn_init(const double *__restrict__ grad, double *__restrict__ x,
                        double *__restrict__ r, double *__restrict__ p, float *__restrict__ pf,
                        int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = -grad[i];
    x[i] = 0.0;
    r[i] = v;
    p[i] = v;
    pf[i] = (float)v;
}

// rr from the partials of r.r; norms[k] = sqrt(rr)
__global__ void __launch_bounds__(256) gn_set_rr(const double *__restrict__ part,
                                                 double *__restrict__ s, double *norms, int k) {
    const double rr = sum_parts(part);
    if (threadIdx.x == 0) {
        s[S_RR] = rr;
        s[S_STOP] = 0.0;
        if (norms) norms[k] = sqrt(rr);
    }
}

// alpha = rr / p.Hp (0 once the iteration has converged or lost positivity)
__global__ void __launch_bounds__(256) gn_alpha(const double *__restrict__ part,
                                                double *__restrict__ s) {
    const double pap = sum_parts(part);
    if (threadIdx.x == 0) {
        const double rr = s[S_RR];
        const bool go = s[S_STOP] == 0.0 && rr > 0.0 && pap > 0.0 && isfinite(pap);
        s[S_ALPHA] = go ? rr / pap : 0.0;
        if (!go) s[S_STOP] = 1.0;
    }
}

__global__ void gn_update_xr(double *__restrict__ x, double *__restrict__ r,
                             const double *__restrict__ p, const double *__restrict__ hp,
                             const double *__restrict__ s, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = s[S_ALPHA];
    x[i] += a * p[i];
    r[i] -= a * hp[i];
}

// beta = rr_new / rr (0 when alpha was 0), rr = rr_new, norms[k] = sqrt(rr_new)
__global__ void __launch_bounds__(256) gn_beta(const double *__restrict__ part,
                                               double *__restrict__ s, double *norms, int k) {
    const double rrn = sum_parts(part);
    if (threadIdx.x == 0) {
        const double rr = s[S_RR];
        s[S_BETA] = (s[S_STOP] == 0.0 && rr > 0.0) ? rrn / rr : 0.0;
        s[S_RR] = rrn;
        if (norms) norms[k] = sqrt(rrn);
    }
}

__global__ void gn_update_p(double *__restrict__ p, const double *__restrict__ r,
                            const double *__restrict__ s, float *__restrict__ pf, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = r[i] + s[S_BETA] * p[i];
    p[i] = v;
    pf[i] = (float)v;
}

}  // namespace

rb_status rb_launch_water_tables(rb_ctx *ctx, const rb_ring *ring, double c0,
                                 const rb_tables *tb, float4 *rec, double2 *ringpos,
                                 unsigned int *rowmax) {
    const rb_grid &g = ctx->grid;
    const int N = ring->n, nm = (int)ctx->n_mask;
    hipLaunchKernelGGL(gn_ring_positions, dim3(blocks_of(N)), dim3(256), 0, ctx->stream,
                       ring->radius, ring->psi0, N, ringpos);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_begin(ctx, ST_TRACE);
    hipLaunchKernelGGL(water_nodes, dim3(blocks_of(nm), N), dim3(256), 0, ctx->stream,
                       ctx->d_mask_index, g.x0, g.y0, g.dx, g.nx, nm, (const double2 *)ringpos,
                       c0, *tb, rec);
    RB_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(water_receivers, dim3(blocks_of(N), N), dim3(256), 0, ctx->stream,
                       (const double2 *)ringpos, N, c0, *tb);
    RB_CHECK_LAUNCH(ctx);
    if (rowmax) {
        hipLaunchKernelGGL(water_rowmax, dim3(N), dim3(256), 0, ctx->stream, ctx->d_mask_index,
                           g.x0, g.y0, g.dx, g.nx, nm, (const double2 *)ringpos, rowmax);
        RB_CHECK_LAUNCH(ctx);
    }
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_gn_delta(rb_ctx *ctx, const double *cq, const float *n_s, double c0,
                             float *delta) {
    const int nm = (int)ctx->n_mask;
    hipLaunchKernelGGL(gn_delta, dim3(blocks_of(nm)), dim3(256), 0, ctx->stream, cq, n_s,
                       ctx->d_mask_index, nm, c0, delta);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_gn_weight(rb_ctx *ctx, float *w, int n, double value) {
    hipLaunchKernelGGL(gn_fill_weight, dim3(blocks_of(n)), dim3(256), 0, ctx->stream,
                       (float2 *)w, n, (float)value);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_gn_mask_pairs(rb_ctx *ctx, float *d, const uint8_t *rx_flags, int N) {
    hipLaunchKernelGGL(gn_mask_pairs, dim3(blocks_of(N), N), dim3(256), 0, ctx->stream,
                       (float2 *)d, rx_flags, N);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_gn_adjoint_acc(rb_ctx *ctx, int mblocks, const float *parts, const float *w,
                                   double *acc, int first) {
    const int nm = (int)ctx->n_mask;
    rb_prof_begin(ctx, ST_FINISH);
    hipLaunchKernelGGL(gn_adjoint_acc, dim3(blocks_of(nm)), dim3(256), 0, ctx->stream, nm,
                       mblocks, parts, (const float2 *)w, acc, first);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

size_t rb_gn_scalar_bytes() { return rb_align((DOT_BLOCKS + S_COUNT) * sizeof(double)); }

// The CG state: x, r, p, Hp (double [n]), pf (float [n]); scal: rb_gn_scalar_bytes.
rb_status rb_launch_gn_cg(rb_ctx *ctx, int op, double *x, double *r, double *p, double *hp,
                          float *pf, const double *grad, double *scal, double *norms, int k) {
    const int n = (int)ctx->n_mask;
    double *part = scal + S_COUNT;
    const dim3 vb(blocks_of(n)), db(DOT_BLOCKS), t(256);
    switch (op) {
    case 0:  // start: x = 0, r = p = -grad, rr
        hipLaunchKernelGGL(gn_init, vb, t, 0, ctx->stream, grad, x, r, p, pf, n);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(gn_dot_part, db, t, 0, ctx->stream, r, r, n, part);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(gn_set_rr, dim3(1), t, 0, ctx->stream, part, scal, norms, k);
        break;
    case 1:  // after H p: alpha, x += alpha p, r -= alpha H p, beta, p = r + beta p
        hipLaunchKernelGGL(gn_dot_part, db, t, 0, ctx->stream, p, hp, n, part);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(gn_alpha, dim3(1), t, 0, ctx->stream, part, scal);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(gn_update_xr, vb, t, 0, ctx->stream, x, r, p, hp, scal, n);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(gn_dot_part, db, t, 0, ctx->stream, r, r, n, part);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(gn_beta, dim3(1), t, 0, ctx->stream, part, scal, norms, k);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(gn_update_p, vb, t, 0, ctx->stream, p, r, scal, pf, n);
        break;
    default:
        return rb_fail(ctx, RB_EINVAL, "unknown CG operation");
    }
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}
