// Complex GEMMs of the Born operator on MFMA (gfx950, FP32 matrix cores).
//
// Forward (Eqs. perturb1, derivative): d[e][r] = sum_q G[e][q] v[q] G[r][q] with
// v = w delta. Both operands are K-contiguous ([row][q]); d is symmetric (reciprocity), so
// only tiles with tile(e) <= tile(r) are computed. K = number of mask nodes is long, so the
// K range is split across workgroups (split-K) into FP32 partial tiles that a second kernel
// sums in a fixed order (deterministic) and mirrors.
//
// Row-reduced NN GEMM (Eq. functional-gradient with Q = 1, Eq. sound_speed_update2):
// for each component c, Y_c = R B_c with R [n][n] and B_c [n][n_mask]; the epilogue
// multiplies Y_c by the same operand at the output position (E_c[e][q] = B_c[e][q]) and
// sums over the rows e of the tile, giving per-column partial sums (re, im) per row block.
//
// A complex product is four real MFMAs (v_mfma_f32_32x32x2f32): re += ar br - ai bi,
// im += ar bi + ai br. Operand tiles are staged through LDS as planar re/im arrays laid
// out [k][row] so that the 32 lanes reading one MFMA operand touch 32 consecutive words.
#include "rb_internal.h"

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ floatx16 mfma32(float a, float b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Output element held by (lane, register i) of a 32x32 MFMA tile.
__device__ __forceinline__ int mfma_row(int lane, int i) {
    return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
}

constexpr int RR_BM = 256, RR_BN = 64, RR_BK = 16;

// The row-reduced products are bilinear forms x^T R x (the same operand E = B on both
// sides), which see only the symmetric part Rs = (R + R^T) / 2. With row and column blocks
// of RR_BM transducers, x^T Rs x = sum_I x_I^T Rs_II x_I + 2 sum_{J > I} x_I^T Rs_IJ x_J, so
// the operand is the block upper triangle R' = Rs on diagonal blocks, R + R^T above them, 0
// below, and row block I contracts over columns from its own block on.
__global__ void sym_upper_kernel(const float2 *__restrict__ R, int n, float2 *__restrict__ Rs) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)n * n) return;
    const int row = (int)(i / n), col = (int)(i - (size_t)row * n);
    const int bi = row / RR_BM, bj = col / RR_BM;
    float2 v = make_float2(0.f, 0.f);
    if (bj >= bi) {
        const float2 a = R[i], b = R[(size_t)col * n + row];
        const float f = bj == bi ? 0.5f : 1.0f;
        v = make_float2(f * (a.x + b.x), f * (a.y + b.y));
    }
    Rs[i] = v;
}

// parts: [2][mblocks][n_cols] (re plane, then im plane).
__global__ void __launch_bounds__(256) rowred_kernel(const float2 *__restrict__ R,
                                                     const float2 *__restrict__ B, int n,
                                                     int n_cols, int n_comp, int conj_b,
                                                     int mblocks, int nblocks,
                                                     float *__restrict__ parts) {
    __shared__ float a_re[RR_BK][RR_BM], a_im[RR_BK][RR_BM];
    __shared__ float b_re[RR_BK][RR_BN], b_im[RR_BK][RR_BN];
    __shared__ float red[2][4][RR_BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float bsign = conj_b ? -1.f : 1.f;
    // Persistent: one workgroup per CU walks a static list of items, each one column block
    // and a pair of row blocks (i, mblocks - 1 - i) whose contractions (from the diagonal
    // block on) together span mblocks + 1 blocks, so every item costs the same. Each XCD
    // walks a contiguous range of items.
    const int n_pairs = (mblocks + 1) / 2, n_items = nblocks * n_pairs;
    const int L = gridDim.x >> 3, xcd = blockIdx.x & 7;
    const int per = (((n_items + 7) / 8) + 1) & ~1;
    for (int k = blockIdx.x >> 3; k < per; k += L) {
        const int item = xcd * per + k;
        if (item >= n_items) break;
        const int nb = item / n_pairs, pr = item - nb * n_pairs;
        for (int half = 0; half < 2; ++half) {
            const int mb = half == 0 ? pr : mblocks - 1 - pr;
            if (half == 1 && mb == pr) break;  // middle block of an odd count

            const int row0 = mb * RR_BM, col0 = nb * RR_BN;

            float cs_re[2] = {0.f, 0.f}, cs_im[2] = {0.f, 0.f};  // per n-tile column sums

            for (int c = 0; c < n_comp; ++c) {
                const float2 *Bc = B + (size_t)c * n * n_cols;
                floatx16 acc_re[2][2], acc_im[2][2];
#pragma unroll
                for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            acc_re[mt][nt][i] = 0.f;
                            acc_im[mt][nt][i] = 0.f;
                        }
                for (int k0 = row0; k0 < n; k0 += RR_BK) {  // R' is zero left of the diagonal block
                    // A tile: row (row0 + tid), 16 consecutive k of R
                    {
                        int gr = row0 + tid;
                        const float2 *src = R + (size_t)gr * n + k0;
#pragma unroll
                        for (int kk = 0; kk < RR_BK; ++kk) {
                            float2 v = make_float2(0.f, 0.f);
                            if (gr < n && k0 + kk < n) v = src[kk];
                            a_re[kk][tid] = v.x;
                            a_im[kk][tid] = v.y;
                        }
                    }
                    // B tile: 16 rows (k) x 64 columns; each thread 4 consecutive columns
                    {
                        int kk = tid >> 4, cc = (tid & 15) * 4;
                        int gk = k0 + kk;
                        const float2 *src = Bc + (size_t)gk * n_cols + col0 + cc;
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            float2 v = make_float2(0.f, 0.f);
                            if (gk < n && col0 + cc + u < n_cols) v = src[u];
                            b_re[kk][cc + u] = v.x;
                            b_im[kk][cc + u] = bsign * v.y;
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int kp = 0; kp < RR_BK / 2; ++kp) {
                        int k = 2 * kp + (lane >> 5);
                        float ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
                        for (int mt = 0; mt < 2; ++mt) {
                            int m = wave * 64 + mt * 32 + (lane & 31);
                            ar[mt] = a_re[k][m];
                            ai[mt] = a_im[k][m];
                            nai[mt] = -ai[mt];
                        }
#pragma unroll
                        for (int nt = 0; nt < 2; ++nt) {
                            int cn = nt * 32 + (lane & 31);
                            br[nt] = b_re[k][cn];
                            bi[nt] = b_im[k][cn];
                        }
#pragma unroll
                        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                            for (int nt = 0; nt < 2; ++nt) {
                                acc_re[mt][nt] = mfma32(ar[mt], br[nt], acc_re[mt][nt]);
                                acc_re[mt][nt] = mfma32(nai[mt], bi[nt], acc_re[mt][nt]);
                                acc_im[mt][nt] = mfma32(ar[mt], bi[nt], acc_im[mt][nt]);
                                acc_im[mt][nt] = mfma32(ai[mt], br[nt], acc_im[mt][nt]);
                            }
                    }
                    __syncthreads();
                }
                // epilogue: sum over the rows of E_c[e][q] Y_c[e][q]
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    int gc = col0 + nt * 32 + (lane & 31);
                    if (gc >= n_cols) continue;
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            int gr = row0 + wave * 64 + mt * 32 + mfma_row(lane, i);
                            if (gr < n) {
                                float2 ev = Bc[(size_t)gr * n_cols + gc];
                                float er = ev.x, ei = bsign * ev.y;
                                float yr = acc_re[mt][nt][i], yi = acc_im[mt][nt][i];
                                cs_re[nt] += er * yr - ei * yi;
                                cs_im[nt] += er * yi + ei * yr;
                            }
                        }
                }
            }
            // combine the two lane halves (rows 4..7 of each group of 8), then the four waves
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                cs_re[nt] += __shfl_xor(cs_re[nt], 32);
                cs_im[nt] += __shfl_xor(cs_im[nt], 32);
                if (lane < 32) {
                    red[0][wave][nt * 32 + lane] = cs_re[nt];
                    red[1][wave][nt * 32 + lane] = cs_im[nt];
                }
            }
            __syncthreads();
            if (tid < RR_BN) {
                int gc = col0 + tid;
                if (gc < n_cols) {
                    float sr = red[0][0][tid] + red[0][1][tid] + red[0][2][tid] + red[0][3][tid];
                    float si = red[1][0][tid] + red[1][1][tid] + red[1][2][tid] + red[1][3][tid];
                    parts[(size_t)mb * n_cols + gc] = sr;
                    parts[(size_t)(mblocks + mb) * n_cols + gc] = si;
                }
            }
            __syncthreads();  // red[] and the LDS tiles are reused by the next block
        }
    }
}

constexpr int FW_B = 128, FW_BK = 16;

// Upper-triangular tile index -> (tm, tn) with tm <= tn.
__device__ __forceinline__ void upper_tile(int idx, int T, int &tm, int &tn) {
    int r = 0, rem = idx;
    while (rem >= T - r) {
        rem -= T - r;
        ++r;
    }
    tm = r;
    tn = r + rem;
}

// dpart: [splitk][n][n] complex partial sums (only upper tiles written).
__global__ void __launch_bounds__(256) forward_kernel(const float2 *__restrict__ G,
                                                      const float2 *__restrict__ w,
                                                      const float *__restrict__ delta, int n,
                                                      int K, int T, int kchunk,
                                                      float2 *__restrict__ dpart) {
    __shared__ float a_re[FW_BK][FW_B], a_im[FW_BK][FW_B];
    __shared__ float b_re[FW_BK][FW_B], b_im[FW_BK][FW_B];
    int tm, tn;
    upper_tile(blockIdx.x, T, tm, tn);
    const int split = blockIdx.y;
    const int kbeg = split * kchunk, kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int row0 = tm * FW_B, col0 = tn * FW_B;

    floatx16 acc_re[2][2], acc_im[2][2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                acc_re[mt][nt][i] = 0.f;
                acc_im[mt][nt][i] = 0.f;
            }

    const int lr = tid >> 1, kh = (tid & 1) * 8;  // loader: row, first k of 8
    for (int k0 = kbeg; k0 < kend; k0 += FW_BK) {
        {
            int gr = row0 + lr;
            const float2 *src = G + (size_t)gr * K + k0 + kh;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                int gk = k0 + kh + u;
                float2 g = make_float2(0.f, 0.f);
                if (gr < n && gk < kend) {
                    float2 gv = src[u];
                    if (w) {  // v = w delta (absent: the operand already carries it)
                        float2 wv = w[gk];
                        float dl = delta[gk];
                        float vr = wv.x * dl, vi = wv.y * dl;
                        g = make_float2(gv.x * vr - gv.y * vi, gv.x * vi + gv.y * vr);
                    } else {
                        g = gv;
                    }
                }
                a_re[kh + u][lr] = g.x;
                a_im[kh + u][lr] = g.y;
            }
        }
        {
            int gr = col0 + lr;
            const float2 *src = G + (size_t)gr * K + k0 + kh;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                int gk = k0 + kh + u;
                float2 g = make_float2(0.f, 0.f);
                if (gr < n && gk < kend) g = src[u];
                b_re[kh + u][lr] = g.x;
                b_im[kh + u][lr] = g.y;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kp = 0; kp < FW_BK / 2; ++kp) {
            int k = 2 * kp + (lane >> 5);
            float ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                int m = wm * 64 + mt * 32 + (lane & 31);
                ar[mt] = a_re[k][m];
                ai[mt] = a_im[k][m];
                nai[mt] = -ai[mt];
            }
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                int cn = wn * 64 + nt * 32 + (lane & 31);
                br[nt] = b_re[k][cn];
                bi[nt] = b_im[k][cn];
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    acc_re[mt][nt] = mfma32(ar[mt], br[nt], acc_re[mt][nt]);
                    acc_re[mt][nt] = mfma32(nai[mt], bi[nt], acc_re[mt][nt]);
                    acc_im[mt][nt] = mfma32(ar[mt], bi[nt], acc_im[mt][nt]);
                    acc_im[mt][nt] = mfma32(ai[mt], br[nt], acc_im[mt][nt]);
                }
        }
        __syncthreads();
    }
    float2 *out = dpart + (size_t)split * n * n;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            int gc = col0 + wn * 64 + nt * 32 + (lane & 31);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                int gr = row0 + wm * 64 + mt * 32 + mfma_row(lane, i);
                if (gr < n && gc < n)
                    out[(size_t)gr * n + gc] = make_float2(acc_re[mt][nt][i], acc_im[mt][nt][i]);
            }
        }
}

// d[e][r] = d[r][e] = sum over splits of the partial at (min(e,r), max(e,r)), which lies in
// a computed upper tile; both entries come from the same sums, so d is exactly symmetric.
__global__ void forward_reduce(const float2 *__restrict__ dpart, int n, int splitk,
                               const float *__restrict__ gscale, float2 *__restrict__ d) {
    int r = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
    if (r >= n) return;
    size_t src = (e <= r) ? (size_t)e * n + r : (size_t)r * n + e;
    float sr = 0.f, si = 0.f;
    for (int s = 0; s < splitk; ++s) {
        float2 v = dpart[(size_t)s * n * n + src];
        sr += v.x;
        si += v.y;
    }
    float inv = gscale ? gscale[1] * gscale[1] : 1.f;  // the operand carried sqrt(v) s
    d[(size_t)e * n + r] = make_float2(sr * inv, si * inv);
}

}  // namespace

int rb_rowred_mblocks(int n) { return (n + RR_BM - 1) / RR_BM; }

rb_status rb_launch_rowred(rb_ctx *ctx, int n, int n_mask, const float *R, const float *B,
                           int n_comp, int conj_b, float *rsym, float *parts, int *mblocks_out) {
    int mblocks = rb_rowred_mblocks(n);
    int nblocks = (n_mask + RR_BN - 1) / RR_BN;
    int grid = std::max(8, ctx->n_cu / 8 * 8);  // one workgroup per CU (persistent)
    rb_prof_begin(ctx, ST_BACKPROJECT);
    hipLaunchKernelGGL(sym_upper_kernel, dim3((unsigned)(((size_t)n * n + 255) / 256)), dim3(256),
                       0, ctx->stream, (const float2 *)R, n, (float2 *)rsym);
    RB_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(rowred_kernel, dim3(grid), dim3(256), 0, ctx->stream,
                       (const float2 *)rsym, (const float2 *)B, n, n_mask, n_comp, conj_b,
                       mblocks, nblocks, parts);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    if (mblocks_out) *mblocks_out = mblocks;
    return RB_OK;
}

// K split of the FP32 forward: the built-in rule, or `want` (a tuned configuration).
static int forward_splitk(int n, int n_mask, int want, int *kchunk_out) {
    const int T = (n + FW_B - 1) / FW_B;
    const int tiles = T * (T + 1) / 2;
    const int ksteps = (n_mask + FW_BK - 1) / FW_BK;
    int splitk = want > 0 ? want : (1024 + tiles - 1) / tiles;
    splitk = want > 0 ? std::max(1, std::min(splitk, ksteps))
                      : std::max(1, std::min(splitk, std::max(1, ksteps / 4)));
    const int kchunk = ((ksteps + splitk - 1) / splitk) * FW_BK;
    if (kchunk_out) *kchunk_out = kchunk;
    return (n_mask + kchunk - 1) / kchunk;
}

int rb_forward_default_splitk(int n, int n_mask) { return forward_splitk(n, n_mask, 0, nullptr); }

size_t rb_forward_ws_bytes(int n, int n_mask) {
    const int spk = std::max(rb_forward_default_splitk(n, n_mask),
                             forward_splitk(n, n_mask, RB_TUNE_SPLITK_MAX, nullptr));
    return rb_align((size_t)spk * n * n * sizeof(float2));
}

rb_status rb_launch_forward(rb_ctx *ctx, const rb_green *gr, const float *w, const float *delta,
                            float *d, const float *gscale) {
    const int n = gr->n, K = gr->n_mask;
    const int T = (n + FW_B - 1) / FW_B;
    const int tiles = T * (T + 1) / 2;
    const rb_tuning *t = rb_tuned(ctx, n, K, RB_F32);
    int kchunk = 0;
    const int splitk = forward_splitk(n, K, t ? t->fwd_splitk : 0, &kchunk);
    ctx->ws.used = 0;
    size_t bytes = rb_align((size_t)splitk * n * n * sizeof(float2));
    rb_status st = rb_arena_reserve(ctx, &ctx->ws, bytes);
    if (st != RB_OK) return st;
    float2 *dpart = rb_carve<float2>(&ctx->ws, (size_t)splitk * n * n);
    rb_prof_begin(ctx, ST_FORWARD);
    hipLaunchKernelGGL(forward_kernel, dim3(tiles, splitk), dim3(256), 0, ctx->stream,
                       (const float2 *)gr->G, (const float2 *)w, delta, n, K, T, kchunk, dpart);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    rb_prof_begin(ctx, ST_FORWARD_REDUCE);
    hipLaunchKernelGGL(forward_reduce, dim3((n + 255) / 256, n), dim3(256), 0, ctx->stream, dpart,
                       n, splitk, gscale, (float2 *)d);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}
