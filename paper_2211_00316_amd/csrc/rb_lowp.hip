// Reduced-precision form of the Born operator (BF16 / FP16 operands, FP32 accumulation).
//
// The same mathematics as rb_green.hip / rb_gemm.hip (Eqs. 2D_greens, greens-time-reversed,
// perturb1, derivative, sound_speed_update2), with the Green's-function operands stored in a
// 16-bit type and the complex contractions on the 16-bit matrix cores
// (v_mfma_f32_32x32x16_bf16 / _f16: K = 16 per instruction, 8 consecutive K per lane).
// The phase omega T + pi/4 - K pi/2 is still reduced in FP64 and the sincos is FP32; only
// the stored operands are rounded.
//
// Layouts (planar re / im, so that one 16-byte load gives 8 consecutive K of one part):
//   Gp  [2][N][P_m]      G rows (transducer-major, node-contiguous): the forward operator
//                        d = G diag(v) G^T contracts over nodes, K-contiguous for both sides;
//   Ht  [3][2][P_m][Np]  H, H u_x, H u_y transposed (node-major, transducer-contiguous): the
//                        back-projection Y_c = R H_c contracts over transducers;
//   Rp  [2][N][Np]       residual rows.
// Np = N rounded up to a multiple of 32 (zeros beyond N), so that every operand row starts
// 16-byte aligned and the contraction runs over whole 32-deep steps.
// The green kernel transposes H through LDS so that both layouts are written coalesced.
#include "rb_internal.h"

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

template <typename T> struct Lp;
template <> struct Lp<__bf16> {
    typedef bf16x8 vec;
    static __device__ __forceinline__ floatx16 mfma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Lp<_Float16> {
    typedef halfx8 vec;
    static __device__ __forceinline__ floatx16 mfma(vec a, vec b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

template <typename T> __device__ __forceinline__ T to_lp(float x) { return (T)x; }
template <typename T> __device__ __forceinline__ float from_lp(T x) { return (float)x; }

// Negate eight packed 16-bit values (both types keep the sign in bit 15).
__device__ __forceinline__ uint4 neg8(uint4 v) {
    return make_uint4(v.x ^ 0x80008000u, v.y ^ 0x80008000u, v.z ^ 0x80008000u,
                      v.w ^ 0x80008000u);
}

template <typename T> __device__ __forceinline__ typename Lp<T>::vec as_vec(uint4 v) {
    return __builtin_bit_cast(typename Lp<T>::vec, v);
}

__device__ __forceinline__ int mfma_row(int lane, int i) {
    return (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
}

__device__ __forceinline__ double reduce_phase(double ph) {
    return ph - RB_TWO_PI * floor(ph / RB_TWO_PI);
}

// Green's functions --------------------------------------------------------------------
// A workgroup covers 64 mask nodes (one per lane) x 64 transducers (16 consecutive ones per
// wave). A lane keeps the directions and flags of its 16 transducers and their two
// neighbours in registers, writes G rows coalesced over the nodes, and writes its 16 entries
// of each transposed H row as two 16-byte stores.
constexpr int GQ = 64;
constexpr int GW = 16;       // transducers per wave
constexpr int GE = 4 * GW;   // transducers per workgroup

// Bit pattern of a value rounded to the 16-bit type.
template <typename T>
__device__ __forceinline__ uint32_t lp_bits(float x) {
    T b = to_lp<T>(x);
    uint16_t u;
    __builtin_memcpy(&u, &b, 2);
    return u;
}

// Bit pattern of the rounding error of x in the 16-bit type, itself rounded (the low part of
// a split operand: x ~ hi + lo with hi = the rounded x).
template <typename T>
__device__ __forceinline__ uint32_t lp_lo_bits(float x) {
    return lp_bits<T>(x - from_lp<T>(to_lp<T>(x)));
}

// Angle between two unit directions.
__device__ __forceinline__ float angle_between(float ax, float ay, float bx, float by) {
    return fabsf(atan2f(ax * by - ay * bx, ax * bx + ay * by));
}

// Lanes of the nodes past the last one write G's zero padding (rows are rb_lp_pad(n_mask)
// long) and nothing else.
template <typename T>
__device__ __forceinline__ void green_pad_g(T *Gp, size_t gplane, int Mp, int N, int e0, int q) {
#pragma unroll
    for (int r = 0; r < GW; ++r) {
        const int e = e0 + r;
        if (e < N) {
            Gp[(size_t)e * Mp + q] = to_lp<T>(0.f);
            Gp[gplane + (size_t)e * Mp + q] = to_lp<T>(0.f);
        }
    }
}

// G = A k0^-1/2 e^{i phi} and H = a k0^1/2 A^-1 e^{-i phi}, phi = omega T + pi/4 - K pi/2
// reduced modulo 2 pi in FP64 (Eqs. 2D_greens, greens-time-reversed; a: angular weight).
__device__ __forceinline__ void green_entry(double omega, double Tt, uint32_t K, float A, float a,
                                            float sk, float isk, float &gr, float &gi, float &hr,
                                            float &hi) {
    double ph = omega * Tt + 0.25 * RB_PI - (double)(K & 3) * 0.5 * RB_PI;
    ph -= RB_TWO_PI * floor(ph * (1.0 / RB_TWO_PI));
    float sn, cs;
    __sincosf((float)ph, &sn, &cs);
    const float ga = A * isk;
    gr = ga * cs;
    gi = ga * sn;
    const float ha = a * sk * __builtin_amdgcn_rcpf(A);
    hr = ha * cs;
    hi = -ha * sn;
}

// Per-transducer operand scales. With the largest amplitude A and the largest 1/A of row e
// (bits in rowmax[2e], rowmax[2e+1]), |G[e][q]| <= A k0^-1/2 gmax (gmax bounds the per-node
// factor sqrt(v) carried by G) and |H_c[e][q]| <= pi k0^1/2 / A (angular weight <= pi, |u| <= 1).
// The scale is the power of two that brings the bound to [2^13, 2^14): the largest stored
// value stays below 2^14 (inside the FP16 range) and a row's small values stay far above the
// FP16 subnormals. A row without a valid entry gets 1.
__device__ __forceinline__ float pow2_scale(float bound) {
    if (!(bound > 0.f) || !isfinite(bound)) return 1.f;
    int e = 0;
    frexpf(bound, &e);  // 2^(e-1) <= bound < 2^e
    return ldexpf(1.f, 14 - e);
}

__device__ __forceinline__ void row_scales(const unsigned int *__restrict__ rowmax, int e,
                                           float sk, float isk, float gmax, float &sg,
                                           float &sh) {
    const float amax = __uint_as_float(rowmax[2 * e]);
    const float iamax = __uint_as_float(rowmax[2 * e + 1]);
    sg = pow2_scale(amax * isk * gmax);
    sh = pow2_scale((float)RB_PI * sk * iamax);
}

// The scales of every row for one frequency, scales[e] (G) and scales[N + e] (H), before the
// assembly from compact records, which then reads them instead of recomputing them in every
// lane.
__global__ void __launch_bounds__(256) row_scale_kernel(const unsigned int *__restrict__ rowmax,
                                                        int N, double omega, double c0,
                                                        float gmax, float *__restrict__ scales) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const double k0 = omega / c0;
    const float sk = (float)sqrt(k0), isk = 1.0f / sk;
    float sg, sh;
    row_scales(rowmax, e, sk, isk, gmax, sg, sh);
    scales[e] = sg;
    scales[N + e] = sh;
}

// Largest A and 1/A over the valid entries of each row of the ABI tables (one workgroup per
// transducer), as the bits rowmax[2e], rowmax[2e+1].
__global__ void __launch_bounds__(256) row_amax_kernel(rb_tables tb, int n_mask,
                                                       unsigned int *__restrict__ rowmax) {
    __shared__ float red[2][4];
    const int e = blockIdx.x;
    float m0 = 0.f, m1 = 0.f;
    for (int q = threadIdx.x; q < n_mask; q += blockDim.x) {
        const size_t o = (size_t)e * n_mask + q;
        const float A = tb.A[o];
        if ((tb.flags[o] & 0x80) && A > 0.f) {
            m0 = fmaxf(m0, A);
            m1 = fmaxf(m1, 1.0f / A);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        m0 = fmaxf(m0, __shfl_xor(m0, o));
        m1 = fmaxf(m1, __shfl_xor(m1, o));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = m0;
        red[1][threadIdx.x >> 6] = m1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        rowmax[2 * e] = __float_as_uint(fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3])));
        rowmax[2 * e + 1] =
            __float_as_uint(fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3])));
    }
}

template <typename T, bool SPLIT>
__global__ void __launch_bounds__(256) green_lp_kernel(rb_tables tb, int N, int n_mask,
                                                       double omega, double c0,
                                                       const float2 *__restrict__ gs,
                                                       const float *__restrict__ gscale,
                                                       int write_g, T *__restrict__ Gp,
                                                       T *__restrict__ Ht,
                                                       const unsigned int *__restrict__ rowmax,
                                                       float gmax, float *__restrict__ scales,
                                                       T *__restrict__ Htlo) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int q = blockIdx.x * GQ + lane;
    const int e0 = blockIdx.y * GE + w * GW;
    const int Np = rb_lp_pad(N), Mp = rb_lp_pad(n_mask);
    const size_t gplane = (size_t)N * Mp;
    if (q >= Mp || e0 >= Np) return;  // no barrier in this kernel
    if (q >= n_mask) {
        if (write_g) green_pad_g(Gp, gplane, Mp, N, e0, q);
        return;
    }
    // rows e0 - 1 .. e0 + GW (indices mod N)
    float ux[GW + 2], uy[GW + 2];
    uint32_t valid = 0;
#pragma unroll
    for (int r = 0; r < GW + 2; ++r) {
        int e = e0 - 1 + r;
        e = e < 0 ? e + N : (e >= N ? e - N : e);
        if (e >= N) e = 0;  // rows past the padding end: never used
        size_t o = (size_t)e * n_mask + q;
        valid |= (tb.flags[o] & 0x80) ? (1u << r) : 0u;
        ux[r] = tb.ux[o];
        uy[r] = tb.uy[o];
    }
    const double k0 = omega / c0;
    const float sk = (float)sqrt(k0), isk = 1.0f / sk;
    float2 f2 = make_float2(1.f, 0.f);
    if (write_g && gs) {
        f2 = gs[q];
        float sc = gscale[0];
        f2.x *= sc;
        f2.y *= sc;
    }
    uint32_t hp[6][GW / 2];  // (c, part) rows, two transducers per dword
    uint32_t hl[6][GW / 2];  // their low parts (split form)
#pragma unroll
    for (int r = 0; r < GW; ++r) {
        const int e = e0 + r;
        float gr = 0.f, gi = 0.f, hr = 0.f, hi = 0.f, vx = 0.f, vy = 0.f;
        if (e < N) {
            float sg, sh;
            row_scales(rowmax, e, sk, isk, gmax, sg, sh);
            if (blockIdx.x == 0 && lane == 0) {
                scales[e] = sg;
                scales[N + e] = sh;
            }
            size_t o = (size_t)e * n_mask + q;
            if (valid >> (r + 1) & 1u) {
                vx = ux[r + 1];
                vy = uy[r + 1];
                const bool vm = valid >> r & 1u, vp = valid >> (r + 2) & 1u;
                float a = 0.f;
                if (vm && vp) a = 0.5f * angle_between(ux[r], uy[r], ux[r + 2], uy[r + 2]);
                else if (vp) a = angle_between(vx, vy, ux[r + 2], uy[r + 2]);
                else if (vm) a = angle_between(ux[r], uy[r], vx, vy);
                green_entry(omega, tb.T[o], tb.flags[o], tb.A[o], a, sk, isk, gr, gi, hr, hi);
                gr *= sg;
                gi *= sg;
                hr *= sh;
                hi *= sh;
            }
            if (write_g) {
                const size_t og = (size_t)e * Mp + q;
                float tr = gr * f2.x - gi * f2.y;
                gi = gr * f2.y + gi * f2.x;
                Gp[og] = to_lp<T>(tr);
                Gp[gplane + og] = to_lp<T>(gi);
            }
        }
        float v[6] = {hr, hi, hr * vx, hi * vx, hr * vy, hi * vy};
#pragma unroll
        for (int cp = 0; cp < 6; ++cp) {
            if (r & 1) hp[cp][r >> 1] |= lp_bits<T>(v[cp]) << 16;
            else hp[cp][r >> 1] = lp_bits<T>(v[cp]);
            if constexpr (SPLIT) {
                if (r & 1) hl[cp][r >> 1] |= lp_lo_bits<T>(v[cp]) << 16;
                else hl[cp][r >> 1] = lp_lo_bits<T>(v[cp]);
            }
        }
    }
    // transposed rows (c, part, q), Np long (zeros past N)
    const size_t hplane = (size_t)n_mask * Np;
    auto store = [&](const uint32_t (&src)[6][GW / 2], T *base) {
#pragma unroll
        for (int cp = 0; cp < 6; ++cp) {
            T *dst = base + (size_t)cp * hplane + (size_t)q * Np + e0;
            *reinterpret_cast<uint4 *>(dst) =
                make_uint4(src[cp][0], src[cp][1], src[cp][2], src[cp][3]);
            if (e0 + 8 < Np)
                *reinterpret_cast<uint4 *>(dst + 8) =
                    make_uint4(src[cp][4], src[cp][5], src[cp][6], src[cp][7]);
        }
    };
    store(hp, Ht);
    if constexpr (SPLIT) store(hl, Htlo);
}

// The same assembly from the compact records of a frequency step (rb_launch_trace): one
// 16-byte load per (transducer, node) gives dT, A, the ray angle theta and the flags;
// T = dT + d / c0 with d the node's distance from the transducer, and the angle between
// neighbouring transducers' rays is the wrapped difference of their thetas.
__device__ __forceinline__ float wrap_pi(float x) {
    return x - (float)RB_TWO_PI * rintf(x * (float)(1.0 / RB_TWO_PI));
}

// Distance from the squared distance a > 0 (normal): the hardware FP32 square root and one
// Newton step in FP64, relative error about 1e-14 (the phase needs about 1e-9 of T), in a
// third of the instructions of the correctly rounded FP64 square root.
__device__ __forceinline__ double dist_newton(double a) {
    const float s0 = __builtin_amdgcn_sqrtf((float)a);
    const double s = (double)s0;
    return fma(fma(-s, s, a), (double)(0.5f * __builtin_amdgcn_rcpf(s0)), s);
}

// Stores go through LDS: the workgroup's tile of G (4 GWt transducers x 64 nodes) leaves
// as 16-byte pieces of rows (over nodes), and each node's 4 GWt transducers of H as one row
// piece written by consecutive threads, 16 bytes each (H in two halves of three planes; one
// buffer for all, its pitch 8 elements longer than a row so 16-byte lane writes miss no bank).

template <typename T, bool SPLIT, int GWt, int NW>
__global__ void __launch_bounds__(64 * NW) green_lp_rec_kernel(
    const float4 *__restrict__ rec, const int32_t *__restrict__ mask_index,
    const double2 *__restrict__ ring, double x0, double y0, double dx, int nx, int N, int n_mask,
    double omega, double c0, const float2 *__restrict__ gs, const float *__restrict__ gscale,
    int write_g, T *__restrict__ Gp, T *__restrict__ Ht, const float *__restrict__ scales,
    T *__restrict__ Htlo) {
    constexpr int GEt = NW * GWt, GHL = GEt + 8;  // transducers per workgroup, staging pitch
    constexpr int NT = 64 * NW;                   // threads
    __shared__ __attribute__((aligned(16))) T stage[3 * GQ * GHL];
    // w is the wave's index (uniform), so the rows' scales are scalar loads
    const int tid = threadIdx.x, lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q0 = blockIdx.x * GQ, E0 = blockIdx.y * GEt;
    const int q = q0 + lane;
    const int e0 = E0 + w * GWt;
    const int Np = rb_lp_pad(N), Mp = rb_lp_pad(n_mask);
    const size_t gplane = (size_t)N * Mp;
    const bool node = q < n_mask;
    float th[GWt + 2], dTr[GWt], Ar[GWt];
    uint32_t valid = 0, Kb = 0;
    double px = 0.0, py = 0.0;
    float2 f2 = make_float2(1.f, 0.f);
    if (node) {
        const int p = mask_index[q];
        px = x0 + (p % nx) * dx;
        py = y0 + (p / nx) * dx;
        // records of rows e0 - 1 .. e0 + GWt (indices mod N)
#pragma unroll
        for (int r = 0; r < GWt + 2; ++r) {
            int e = e0 - 1 + r;
            e = e < 0 ? e + N : (e >= N ? e - N : e);
            if (e >= N) e = 0;  // rows past the padding end: never used
            const float4 v = rec[(size_t)e * n_mask + q];
            const uint32_t f = __float_as_uint(v.w);
            valid |= (f & 0x80) ? (1u << r) : 0u;
            th[r] = v.z;
            if (r >= 1 && r <= GWt) {
                dTr[r - 1] = v.x;
                Ar[r - 1] = v.y;
                Kb |= (f & 3) << (2 * (r - 1));
            }
        }
        if (write_g && gs) {
            f2 = gs[q];
            float sc = gscale[0];
            f2.x *= sc;
            f2.y *= sc;
        }
    }
    const double k0 = omega / c0, ic0 = 1.0 / c0;
    const float sk = (float)sqrt(k0), isk = 1.0f / sk;
    T *sg = stage;  // G tile [2][GEt][GQ]
    uint32_t hp[6][GWt / 2];  // (c, part) rows, two transducers per dword
    uint32_t b8[6][GWt / 4];  // split form: their low parts times 2^6 as FP8, four per dword
    float b8p[6];
#pragma unroll
    for (int cp = 0; cp < 6; ++cp) {
        b8p[cp] = 0.f;
#pragma unroll
        for (int u = 0; u < GWt / 4; ++u) b8[cp][u] = 0u;
    }
#pragma unroll
    for (int r = 0; r < GWt; ++r) {
        const int e = e0 + r;
        float gr = 0.f, gi = 0.f, hr = 0.f, hi = 0.f, vx = 0.f, vy = 0.f;
        float rsg = 1.f, rsh = 1.f;
        if (e < N) {  // row_scale_kernel's
            rsg = scales[e];
            rsh = scales[N + e];
        }
        if (node && e < N && (valid >> (r + 1) & 1u)) {
            __sincosf(th[r + 1], &vy, &vx);
            const bool vm = valid >> r & 1u, vp = valid >> (r + 2) & 1u;
            float a = 0.f;
            if (vm && vp) a = 0.5f * fabsf(wrap_pi(th[r + 2] - th[r]));
            else if (vp) a = fabsf(wrap_pi(th[r + 2] - th[r + 1]));
            else if (vm) a = fabsf(wrap_pi(th[r + 1] - th[r]));
            const double2 xe = ring[e];
            const double ddx = px - xe.x, ddy = py - xe.y;
            const double Tt = (double)dTr[r] + dist_newton(ddx * ddx + ddy * ddy) * ic0;
            green_entry(omega, Tt, Kb >> (2 * r), Ar[r], a, sk, isk, gr, gi, hr, hi);
            gr *= rsg;
            gi *= rsg;
            hr *= rsh;
            hi *= rsh;
        }
        const float tr = gr * f2.x - gi * f2.y, ti = gr * f2.y + gi * f2.x;
        sg[(w * GWt + r) * GQ + lane] = to_lp<T>(tr);
        sg[(GEt + w * GWt + r) * GQ + lane] = to_lp<T>(ti);
        // the rotated components H, b = H (u_x - i u_y), a = H (u_x + i u_y): the bilinear
        // form a^T Rs b is the sum of the quadratic forms of H u_x and H u_y (Rs symmetric),
        // so the back-projection needs two contractions
        const float v[6] = {hr, hi, hr * vx + hi * vy, hi * vx - hr * vy, hr * vx - hi * vy,
                            hi * vx + hr * vy};
#pragma unroll
        for (int cp = 0; cp < 6; ++cp) {
            if (r & 1) hp[cp][r >> 1] |= lp_bits<T>(v[cp]) << 16;
            else hp[cp][r >> 1] = lp_bits<T>(v[cp]);
            if constexpr (SPLIT) {
                // low part: |lo| <= 4 (half an FP16 ulp below 2^14), times 2^6 in FP8 (E4M3);
                // a correction of relative size 2^-11 needs no more than its 3 bits. Clamped
                // to the format's largest value (448; beyond it the conversion gives NaN), which
                // only a value rounded up to 2^14 itself could reach.
                const float lo = fminf(fmaxf(64.f * (v[cp] - from_lp<T>(to_lp<T>(v[cp]))), -448.f),
                                       448.f);
                if (!(r & 1))
                    b8p[cp] = lo;
                else if ((r >> 1) & 1)  // bytes 2, 3 of the dword
                    b8[cp][r >> 2] = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(
                        b8p[cp], lo, (int)b8[cp][r >> 2], true);
                else  // bytes 0, 1
                    b8[cp][r >> 2] = (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(
                        b8p[cp], lo, (int)b8[cp][r >> 2], false);
            }
        }
    }
    __syncthreads();
    if (write_g) {
        // 2 planes x GEt rows x 8 pieces of 8 nodes
#pragma unroll
        for (int k = 0; k < 2 * GEt * 8 / NT; ++k) {
            const int id = tid + NT * k;
            const int part = id / (GEt * 8), row = (id >> 3) % GEt, ch = id & 7;
            const int e = E0 + row, qq = q0 + ch * 8;
            if (e < N && qq < Mp)
                *reinterpret_cast<uint4 *>(Gp + part * gplane + (size_t)e * Mp + qq) =
                    *reinterpret_cast<const uint4 *>(&sg[(part * GEt + row) * GQ + ch * 8]);
        }
    }
    const size_t hplane = (size_t)n_mask * Np;
    auto store = [&](const uint32_t (&src)[6][GWt / 2], T *base) {
        constexpr int PC = GEt / 8;  // pieces of 8 transducers per node row
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            __syncthreads();  // the staging buffer is free again
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int cp = 3 * half + k;
                uint4 *dst = reinterpret_cast<uint4 *>(&stage[(k * GQ + lane) * GHL + w * GWt]);
#pragma unroll
                for (int u = 0; u < GWt / 8; ++u)
                    dst[u] = make_uint4(src[cp][4 * u], src[cp][4 * u + 1], src[cp][4 * u + 2],
                                        src[cp][4 * u + 3]);
            }
            __syncthreads();
            // 3 planes x GQ node rows x PC pieces of 8 transducers
#pragma unroll
            for (int k = 0; k < 3 * GQ * PC / NT; ++k) {
                const int id = tid + NT * k;
                const int pl = id / (GQ * PC), qr = (id / PC) % GQ, ch = id % PC;
                const int qq = q0 + qr, e = E0 + ch * 8;
                const int plane = 3 * half + pl;
                if (qq < n_mask && e < Np)
                    *reinterpret_cast<uint4 *>(base + (size_t)plane * hplane +
                                               (size_t)qq * Np + e) =
                        *reinterpret_cast<const uint4 *>(&stage[(pl * GQ + qr) * GHL + ch * 8]);
            }
        }
    };
    if constexpr (SPLIT) {
        // FP8 low parts: component c's planes [2][Np8 / 64][n_mask][64 bytes] at the start
        // of its low-part slot (a block of 64 transducers per workgroup: its 64 nodes are
        // 4 KiB in a row), staged [plane][node][GEt bytes]
        constexpr int PP = GEt / 16;  // pieces per node row of one plane
        static_assert(6 * GQ * GEt <= (int)sizeof(stage) && (6 * GQ * PP) % NT == 0 &&
                          GWt == 8 && GEt == 64,
                      "FP8 staging: one block of 64 transducers per workgroup");
        const int Np8 = rb_lp8_pad(N);
        uint8_t *s8 = reinterpret_cast<uint8_t *>(stage);
        __syncthreads();  // the staging buffer is free again
#pragma unroll
        for (int cp = 0; cp < 6; ++cp)
            *reinterpret_cast<uint2 *>(&s8[(cp * GQ + lane) * GEt + w * GWt]) =
                make_uint2(b8[cp][0], b8[cp][1]);
        __syncthreads();
        uint8_t *base8 = reinterpret_cast<uint8_t *>(Htlo);
#pragma unroll
        for (int k = 0; k < 6 * GQ * PP / NT; ++k) {
            const int id = tid + NT * k;
            const int cp = id / (GQ * PP), qr = (id / PP) % GQ, ch = id % PP;
            const int qq = q0 + qr;
            // slot of component cp / 2 (4 hplane bytes), part cp % 2
            const size_t o = (size_t)(cp >> 1) * 4 * hplane + (size_t)(cp & 1) * n_mask * Np8 +
                             (size_t)(E0 >> 6) * n_mask * 64 + (size_t)qq * 64 + 16 * ch;
            if (qq < n_mask)
                *reinterpret_cast<uint4 *>(base8 + o) =
                    *reinterpret_cast<const uint4 *>(&s8[(cp * GQ + qr) * GEt + 16 * ch]);
        }
    }
    store(hp, Ht);
}

// conj(G) in the back-projection's operand layout, for the 16-bit adjoint: G planar
// [2][n][Mp] (rows over nodes) -> planar node-major [2][n_mask][Np] with the imaginary part
// negated and zeros past n. The adjoint's double sum is the bilinear form h^T R h with
// h = conj(G), the same contraction as the back-projection's with h = H. Raw 16-bit words
// (both types keep the sign in bit 15); a 64 x 64 tile per workgroup through LDS.
__global__ void __launch_bounds__(256) transpose_conj_kernel(const uint16_t *__restrict__ Gp,
                                                             int n, int n_mask,
                                                             uint16_t *__restrict__ Gt) {
    __shared__ uint16_t tile[2][64][66];
    const int q0 = blockIdx.x * 64, e0 = blockIdx.y * 64;
    const int Mp = rb_lp_pad(n_mask), Np = rb_lp_pad(n);
    const size_t gplane = (size_t)n * Mp, tplane = (size_t)n_mask * Np;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int e = e0 + r, q = q0 + tx;
        uint16_t vr = 0, vi = 0;
        if (e < n && q < n_mask) {
            vr = Gp[(size_t)e * Mp + q];
            vi = Gp[gplane + (size_t)e * Mp + q] ^ (uint16_t)0x8000u;
        }
        tile[0][r][tx] = vr;
        tile[1][r][tx] = vi;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int q = q0 + r, e = e0 + tx;
        if (q < n_mask && e < Np) {
            Gt[(size_t)q * Np + e] = tile[0][tx][r];
            Gt[tplane + (size_t)q * Np + e] = tile[1][tx][r];
        }
    }
}

// Power-of-two range scale of an operand: scale[0] = 2^(top - e) and scale[1] = 1/scale[0]
// with 2^(e-1) <= max |x| < 2^e, so the largest scaled magnitude lies in [2^(top-1), 2^top)
// (top = 14: inside the FP16 range, far from its subnormals). |x| of a complex value is the
// larger of |re| and |im| (times |y| when y is given). Exact: per-workgroup maxima, then one
// workgroup over them.
__global__ void __launch_bounds__(256) range_max_kernel(const float2 *__restrict__ x,
                                                        size_t count, const float *__restrict__ y,
                                                        const float *__restrict__ rows, int n,
                                                        float *__restrict__ part) {
    __shared__ float red[4];
    float m = 0.f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x) {
        float2 v = x[i];
        float a = fmaxf(fabsf(v.x), fabsf(v.y));
        if (y) a *= fabsf(y[i]);
        if (rows) a /= rows[i / n] * rows[i % n];  // exact: powers of two
        m = fmaxf(m, a);
    }
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ void __launch_bounds__(256) range_finish_kernel(const float *__restrict__ part,
                                                           int n_part, int top,
                                                           float *__restrict__ scale) {
    __shared__ float red[4];
    float m = 0.f;
    for (int i = threadIdx.x; i < n_part; i += blockDim.x) m = fmaxf(m, part[i]);
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float mm = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        int e = 0;
        if (mm > 0.f && isfinite(mm)) frexpf(mm, &e);
        float s = ldexpf(1.f, top - e);
        scale[0] = s;
        scale[1] = 1.f / s;
    }
}

rb_status launch_range_scale(rb_ctx *ctx, const float2 *x, size_t count, const float *y, int top,
                             float *scale, const float *rows = nullptr, int n = 1) {
    const int nb = (int)std::min<size_t>(RB_RED_PARTS, std::max<size_t>(1, (count + 1023) / 1024));
    hipLaunchKernelGGL(range_max_kernel, dim3(nb), dim3(256), 0, ctx->stream, x, count, y, rows,
                       n, ctx->d_red);
    RB_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(range_finish_kernel, dim3(1), dim3(256), 0, ctx->stream,
                       (const float *)ctx->d_red, nb, top, scale);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

// The back-projection needs R only through the bilinear forms h^T R h (the same operand on
// both sides), which depend on R only through its symmetric part Rs = (R + R^T) / 2. With
// row and column blocks of `bm` transducers, h^T Rs h = sum_I h_I^T Rs_II h_I +
// 2 sum_{J > I} h_I^T Rs_IJ h_J, so the operand is the block upper triangle
//   R'[e][r] = Rs[e][r] (same block), 2 Rs[e][r] = R[e][r] + R[r][e] (block J > I), 0 (J < I)
// and the product for row block I runs over column blocks J >= I only.
// complex64 [n][n] -> planar T [2][n][np] of R' (zero past n), multiplied by scale[0]. With
// per-row operand scales (rows, nullable) the operand is R'[e][r] / (rows[e] rows[r]), so
// that the bilinear form of the scaled operands h'_e = rows[e] h_e is unchanged.
template <typename T>
__global__ void to_planar_kernel(const float2 *__restrict__ src, int n, int np, int bm,
                                 const float *__restrict__ scale, const float *__restrict__ rows,
                                 T *__restrict__ dst) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t nn = (size_t)n * np;
    if (i >= nn) return;
    int row = (int)(i / np), col = (int)(i - (size_t)row * np);
    float s = scale[0];
    float2 v = make_float2(0.f, 0.f);
    const int bi = row / bm, bj = col / bm;
    if (col < n && bj >= bi) {
        const float2 a = src[(size_t)row * n + col], b = src[(size_t)col * n + row];
        const float f = bj == bi ? 0.5f : 1.0f;
        v = make_float2(f * (a.x + b.x), f * (a.y + b.y));
        if (rows) {
            const float ir = 1.0f / (rows[row] * rows[col]);
            v.x *= ir;
            v.y *= ir;
        }
    }
    dst[i] = to_lp<T>(v.x * s);
    dst[nn + i] = to_lp<T>(v.y * s);
}

// The symmetric part Rs of R (divided by rows[e] rows[r] when given) at the 16-bit operand's
// scale times 2^-6, as FP8 (E4M3) planes [2][n][np8] (zero past n): the operand of the split
// back-projection's correction term. |Rs scale| < 2^13, so the values stay below 2^7 (the
// format's largest finite value is 448). One thread per four columns of a row.
__global__ void to_fp8_kernel(const float2 *__restrict__ src, int n, int np8,
                              const float *__restrict__ scale, const float *__restrict__ rows,
                              uint32_t *__restrict__ dst) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int w4 = np8 / 4;
    const size_t nw = (size_t)n * w4;
    if (i >= nw) return;
    const int row = (int)(i / w4), col0 = (int)(i - (size_t)row * w4) * 4;
    const float s = scale[0] * (1.f / 64.f);
    float re[4], im[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int col = col0 + k;
        re[k] = im[k] = 0.f;
        if (col < n) {
            const float2 a = src[(size_t)row * n + col], b = src[(size_t)col * n + row];
            float f = 0.5f * s;
            if (rows) f /= rows[row] * rows[col];
            re[k] = f * (a.x + b.x);
            im[k] = f * (a.y + b.y);
        }
    }
    int pr = __builtin_amdgcn_cvt_pk_fp8_f32(re[0], re[1], 0, false);
    pr = __builtin_amdgcn_cvt_pk_fp8_f32(re[2], re[3], pr, true);
    int pi = __builtin_amdgcn_cvt_pk_fp8_f32(im[0], im[1], 0, false);
    pi = __builtin_amdgcn_cvt_pk_fp8_f32(im[2], im[3], pi, true);
    dst[i] = (uint32_t)pr;
    dst[nw + i] = (uint32_t)pi;
}

__global__ void square_scale_kernel(const float *__restrict__ g, float *scale) {
    float inv = g ? g[1] : 1.f;
    scale[0] = 1.f;
    scale[1] = inv * inv;
}

// parts *= scale[1] (undo the residual's range scale before the final sum)
__global__ void unscale_kernel(float *__restrict__ parts, size_t count,
                               const float *__restrict__ scale) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) parts[i] *= scale[1];
}

// Back-projection: Y_c = R H_c, epilogue sums over the tile's rows of H_c[e][q] Y_c[e][q] --
// Workgroup tile 256 (transducers e) x 128 (nodes q), eight waves of 64 x 64 complex (four
// 32 x 32 MFMA tiles, 128 FP32 accumulators per lane, two waves per SIMD so that one
// wave's MFMAs run while the other waits for LDS). K (transducers r) in steps of 32
// (two MFMA sub-steps of 16). The operands go from global memory straight into LDS
// (buffer loads with the LDS bit, 16 bytes per lane), three K steps in flight: while step
// k is multiplied, step k+1 has landed or is landing and step k+2 is being fetched; one
// barrier per step. The MFMA fragments of the next sub-step are read from LDS while the
// current sub-step's MFMAs run (across the barrier for the first sub-step of the next
// step). Global operands are read through one wave-uniform buffer descriptor per operand
// spanning its two part planes (loads past the end return zero); rows are whole K steps
// long. Rows past the last transducer or node read other (finite) data: they only reach
// output rows that meet zero padding or are never stored.
constexpr int LR_BM = 256, LR_BN = 128, LR_BK = 32;
// Waves of a workgroup: LR_WM along M times 2 along N; a wave owns LR_BM / LR_WM rows and 64
// columns (LR_MT tiles of 32 x 32 by 2).
constexpr int LR_WM = 4;
constexpr int LR_MT = LR_BM / (32 * LR_WM);
constexpr int LR_THREADS = 64 * 2 * LR_WM;
// One LDS stage holds one K step: the A part planes (LR_BM rows of LR_BK values each) then
// the B part planes (LR_BN rows). A row is four 16-byte chunks; chunk c of row r sits in slot
// c ^ ((r >> 2) & 3), so that the 16 lanes of a fragment read (16 consecutive rows, one
// chunk) hit all 64 banks once. A loader instruction of a wave fills 1 KiB of a stage, 16
// rows: lane l writes slot l & 3 of row l >> 2 and so fetches chunk (l & 3) ^ ((l >> 4) & 3).
constexpr int LR_AP = LR_BM * LR_BK, LR_BP = LR_BN * LR_BK;  // part plane sizes (values)
constexpr int LR_STAGE = 2 * LR_AP + 2 * LR_BP;                // values per stage
constexpr int LR_AU = 2 * LR_AP * 2 / 1024 / (LR_THREADS / 64);  // A loads per lane and step
constexpr int LR_BU = 2 * LR_BP * 2 / 1024 / (LR_THREADS / 64);  // B loads per lane and step
static_assert(LR_THREADS == 512 && LR_AU == 4 && LR_BU == 2, "loader layout");
constexpr size_t LR_SPAN = 0xfffffff0u;  // vector + scalar byte offsets stay below this

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

// 16 bytes per lane from the buffer to LDS: lane l writes lds + 16 l (lds wave-uniform).
template <typename T>
__device__ __forceinline__ void load_lds16(__amdgpu_buffer_rsrc_t r, T *lds, uint32_t off,
                                           uint32_t soff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(
        r, (__attribute__((address_space(3))) void *)lds, 16, (int)off, (int)soff, 0, 0);
}

// Wait until at most N global loads of this wave are outstanding and its LDS operations are
// done, then meet the other waves. Loads return in order, so the older step's operands are in
// LDS; after the barrier every wave's are.
template <int N>
__device__ __forceinline__ void lr_sync() {
    static_assert(N >= 0 && N < 64, "vmcnt");
    if constexpr (N == 0) asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    else asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(N) : "memory");
}

// MFMA operands of one 16-deep sub-step of a wave: A rows (re, im) of its 32-row tiles, B
// columns (re, im, -im) of its two 32-column tiles.
struct LrFrag {
    uint4 ar[LR_MT], ai[LR_MT], br[2], bi[2], bn[2];
};

// Fragments of sub-step `sub` (0 or 1) of the stage st.
template <typename T>
__device__ __forceinline__ void lr_read(LrFrag &f, const T *st, int wm, int wn, int lane,
                                        int sub) {
    const int co = (((sub * 2 + (lane >> 5)) ^ ((lane >> 2) & 3)) * 8);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int o = 2 * LR_AP + (wn * 64 + nt * 32 + (lane & 31)) * LR_BK + co;
        f.br[nt] = *reinterpret_cast<const uint4 *>(st + o);
        f.bi[nt] = *reinterpret_cast<const uint4 *>(st + o + LR_BP);
    }
#pragma unroll
    for (int mt = 0; mt < LR_MT; ++mt) {
        const int o = (wm * (32 * LR_MT) + mt * 32 + (lane & 31)) * LR_BK + co;
        f.ar[mt] = *reinterpret_cast<const uint4 *>(st + o);
        f.ai[mt] = *reinterpret_cast<const uint4 *>(st + o + LR_AP);
    }
}

template <typename T>
__device__ __forceinline__ void lr_mfma(LrFrag &f, floatx16 (&acc_re)[LR_MT][2],
                                        floatx16 (&acc_im)[LR_MT][2]) {
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) f.bn[nt] = neg8(f.bi[nt]);
#pragma unroll
    for (int mt = 0; mt < LR_MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            acc_re[mt][nt] = Lp<T>::mfma(as_vec<T>(f.ar[mt]), as_vec<T>(f.br[nt]), acc_re[mt][nt]);
            acc_im[mt][nt] = Lp<T>::mfma(as_vec<T>(f.ar[mt]), as_vec<T>(f.bi[nt]), acc_im[mt][nt]);
            acc_re[mt][nt] = Lp<T>::mfma(as_vec<T>(f.ai[mt]), as_vec<T>(f.bn[nt]), acc_re[mt][nt]);
            acc_im[mt][nt] = Lp<T>::mfma(as_vec<T>(f.ai[mt]), as_vec<T>(f.br[nt]), acc_im[mt][nt]);
        }
}

// Loader offsets of a lane (bytes, buffer-relative): the A rows it fetches are
// a_row0 + 16 w + (l >> 2) (+ 128) of both part planes, the B rows b_row0 + 16 w + (l >> 2)
// of both planes; ld = values per row.
struct LrLoad {
    __amdgpu_buffer_rsrc_t ra, rb;
    uint32_t a_off, a_half, a_plane, b_off, b_plane;
};

template <typename T>
__device__ __forceinline__ LrLoad lr_load(const void *A, size_t a_plane, int a_row0,
                                          const void *B, size_t b_plane, int b_row0, int ld) {
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int kc = (l & 3) ^ ((l >> 4) & 3);
    LrLoad L;
    L.ra = plane_rsrc(A, 2 * a_plane * sizeof(T));
    L.rb = plane_rsrc(B, 2 * b_plane * sizeof(T));
    L.a_off = (uint32_t)(((size_t)(a_row0 + 16 * w + (l >> 2)) * ld + kc * 8) * sizeof(T));
    L.b_off = (uint32_t)(((size_t)(b_row0 + 16 * w + (l >> 2)) * ld + kc * 8) * sizeof(T));
    L.a_half = (uint32_t)((size_t)128 * ld * sizeof(T));
    L.a_plane = (uint32_t)(a_plane * sizeof(T));
    L.b_plane = (uint32_t)(b_plane * sizeof(T));
    return L;
}

// K step kp of both operands into stage st: LR_AU + LR_BU loads per lane.
template <typename T>
__device__ __forceinline__ void lr_fetch(const LrLoad &L, T *st, int kp) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t kb = (uint32_t)(kp * LR_BK * sizeof(T));
#pragma unroll
    for (int u = 0; u < LR_AU; ++u)  // A block w + 8 u: plane u >> 1, rows 16 w + 128 (u & 1)
        load_lds16(L.ra, st + (w + 8 * u) * 512,
                   L.a_off + (u & 1) * L.a_half + (u >> 1) * L.a_plane, kb);
#pragma unroll
    for (int u = 0; u < LR_BU; ++u)  // B block w + 8 u: plane u, rows 16 w
        load_lds16(L.rb, st + 2 * LR_AP + (w + 8 * u) * 512, L.b_off + u * L.b_plane, kb);
}

// The back-projection epilogue's operand: Ht_c[col0 + q][row0 + e] for q < LR_BN, e < LR_BM,
// both parts, into the stages: rows e in chunks of LR_ECH, LR_ECH, LR_BM - 2 LR_ECH (one
// per stage), each stage laid out [part][q][e] with the 16-byte piece k of a row in slot
// k ^ lr_eswz(q, pieces per row), so that 16 consecutive q of one read hit distinct banks. A loader
// instruction fills 1 KiB of a stage lane-contiguously; each lane fetches the piece that
// lands in its slot. Coalesced: a row's pieces are contiguous in Ht_c.
constexpr int LR_ECH = 96;
__device__ __forceinline__ int lr_eswz(int q, int pr) {
    return pr == 8 ? (q >> 1) & 7 : (q >> 2) & 3;  // rows of 128 or 192 bytes
}
static_assert(LR_ECH % 32 == 0 && 2 * LR_ECH < LR_BM && LR_BM - 2 * LR_ECH <= LR_ECH &&
                  2 * LR_BN * LR_ECH <= LR_STAGE,
              "epilogue chunks");
template <typename T>
__device__ __forceinline__ void lr_fetch_e(const T *Hc, size_t hplane, int np, int row0,
                                           int col0, T *s0, T *s1, T *s2) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(Hc, 2 * hplane * sizeof(T));
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        T *st = ch == 0 ? s0 : (ch == 1 ? s1 : s2);
        constexpr int waves = LR_THREADS / 64;
        const int len = ch == 2 ? LR_BM - 2 * LR_ECH : LR_ECH;
        const int pr = len / 8;                 // pieces per row
        const int nu = 2 * LR_BN * pr / 64 / waves;  // loads per lane
#pragma unroll
        for (int u = 0; u < nu; ++u) {
            const int b = w + waves * u;
            const int P = b * 64 + l;
            const int row = P / pr, slot = P - row * pr;
            const int part = row / LR_BN, q = row - part * LR_BN;
            const int piece = slot ^ lr_eswz(q, pr);
            const uint32_t off = (uint32_t)((part * hplane + (size_t)(col0 + q) * np + row0 +
                                             ch * LR_ECH + piece * 8) *
                                            sizeof(T));
            load_lds16(r, st + b * 512, off, 0u);
        }
    }
}

// The same for an FP8 operand (the low parts of the rotated split form, [part][block of 64
// transducers][n_cols nodes][64 bytes]): rows e in chunks of LR_ECH8 (stage s0) and
// LR_BM - LR_ECH8 (s1), laid out [part][q][e] with the 16-byte piece k of a row in slot
// k ^ ((q >> 2) & 3).
constexpr int LR_ECH8 = 192;
static_assert(2 * LR_BN * LR_ECH8 == 2 * LR_STAGE && LR_ECH8 % 32 == 0 && LR_ECH8 % 16 == 0,
              "FP8 epilogue chunks");
template <typename T>
__device__ __forceinline__ void lr_fetch_e8(const uint8_t *Hc, size_t plane8, int n_cols,
                                            int row0, int col0, T *s0, T *s1) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(Hc, 2 * plane8);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), l = threadIdx.x & 63;
#pragma unroll
    for (int ch = 0; ch < 2; ++ch) {
        T *st = ch == 0 ? s0 : s1;
        constexpr int waves = LR_THREADS / 64;
        const int len = ch == 1 ? LR_BM - LR_ECH8 : LR_ECH8;
        const int pr = len / 16;                     // pieces per row
        const int nu = 2 * LR_BN * pr / 64 / waves;  // loads per lane
#pragma unroll
        for (int u = 0; u < nu; ++u) {
            const int b = w + waves * u;
            const int P = b * 64 + l;
            const int row = P / pr, slot = P - row * pr;
            const int part = row / LR_BN, q = row - part * LR_BN;
            const int piece = slot ^ ((q >> 2) & 3);
            const int e = row0 + ch * LR_ECH8 + piece * 16;  // 16-aligned, inside one block
            const uint32_t off = (uint32_t)(part * plane8 + (size_t)(e >> 6) * n_cols * 64 +
                                            (size_t)(col0 + q) * 64 + (e & 63));
            load_lds16(r, st + b * 512, off, 0u);
        }
    }
}

// Epilogue of an FP8 operand staged by lr_fetch_e8: four consecutive rows e per register
// group are one 4-byte LDS read per part; the values carry 2^6, folded into f.
template <typename T>
__device__ __forceinline__ void lr_epilogue8(const T *s0, const T *s1, int row0, int np,
                                             const floatx16 (&acc_re)[LR_MT][2],
                                             const floatx16 (&acc_im)[LR_MT][2], float f,
                                             float (&cs_re)[2], float (&cs_im)[2]) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int q = wn * 64 + nt * 32 + (lane & 31);
        const int hq = (q >> 2) & 3;
#pragma unroll
        for (int mt = 0; mt < LR_MT; ++mt) {
            const int eb = wm * (32 * LR_MT) + mt * 32;  // wave-uniform
            const int ch = eb / LR_ECH8;
            const uint8_t *st = reinterpret_cast<const uint8_t *>(ch == 0 ? s0 : s1);
            const int pr = ch == 1 ? (LR_BM - LR_ECH8) / 16 : LR_ECH8 / 16;
            const float rm = row0 + eb < np ? f : 0.f;
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int el = eb - ch * LR_ECH8 + g * 8 + (lane >> 5) * 4;
                const int o = (q * pr + ((el >> 4) ^ hq)) * 16 + (el & 15);
                const int wr = *reinterpret_cast<const int *>(st + o);
                const int wi = *reinterpret_cast<const int *>(st + o + LR_BN * pr * 16);
                const f2v r01 = __builtin_amdgcn_cvt_pk_f32_fp8(wr, false);
                const f2v r23 = __builtin_amdgcn_cvt_pk_f32_fp8(wr, true);
                const f2v i01 = __builtin_amdgcn_cvt_pk_f32_fp8(wi, false);
                const f2v i23 = __builtin_amdgcn_cvt_pk_f32_fp8(wi, true);
                const float er[4] = {r01[0], r01[1], r23[0], r23[1]};
                const float ei[4] = {i01[0], i01[1], i23[0], i23[1]};
#pragma unroll
                for (int z = 0; z < 4; ++z) {
                    const float yr = acc_re[mt][nt][g * 4 + z];
                    const float yi = acc_im[mt][nt][g * 4 + z];
                    sr += er[z] * yr - ei[z] * yi;
                    si += er[z] * yi + ei[z] * yr;
                }
            }
            cs_re[nt] += rm * sr;
            cs_im[nt] += rm * si;
        }
    }
}

// Issue order of one sub-step: its 16 MFMAs carry the 8 LDS reads of the next sub-step and,
// in the first sub-step, the 6 loads of step k+2.
__device__ __forceinline__ void lr_sched_first() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x020, 2, 0);
}

__device__ __forceinline__ void lr_sched_second() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
}

// The pipelined K loop: acc += A B^T over K steps [kt0, kt1) of LR_BK, complex operands in two
// part planes, through the LDS stages s0, s1, s2 (step kt0 + i in stage i mod 3). DESC walks
// the K steps from kt1 - 1 down to kt0. The stages are distinct arrays so that the compiler
// sees that the loads in flight into one do not feed the LDS reads of another. No load is
// outstanding when it returns, but the stages are still being read: a barrier must precede
// their next fill.
template <typename T, bool DESC>
__device__ __forceinline__ void lr_mainloop(T *s0, T *s1, T *s2, const LrLoad &L, int kt0,
                                            int kt1, floatx16 (&acc_re)[LR_MT][2],
                                            floatx16 (&acc_im)[LR_MT][2]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    auto kp = [&](int kt) { return DESC ? kt0 + kt1 - 1 - kt : kt; };
    LrFrag f0, f1;
    // one K step whose successor is in flight and whose second successor is fetched now
    auto step = [&](T *cur, T *nxt, T *nn, int kt) {
        lr_read<T>(f1, cur, wm, wn, lane, 1);
        lr_mfma<T>(f0, acc_re, acc_im);
        lr_fetch<T>(L, nn, kp(kt + 2));
        lr_sched_first();
        lr_sync<LR_AU + LR_BU>();
        lr_read<T>(f0, nxt, wm, wn, lane, 0);
        lr_mfma<T>(f1, acc_re, acc_im);
        lr_sched_second();
    };
    // one of the last two K steps (nothing left to fetch)
    auto last = [&](T *cur, T *nxt, int kt) {
        lr_read<T>(f1, cur, wm, wn, lane, 1);
        lr_mfma<T>(f0, acc_re, acc_im);
        if (kt + 1 < kt1) {
            lr_sync<0>();
            lr_read<T>(f0, nxt, wm, wn, lane, 0);
        }
        lr_mfma<T>(f1, acc_re, acc_im);
    };
    lr_fetch<T>(L, s0, kp(kt0));
    if (kt0 + 1 >= kt1) {  // a single step
        lr_sync<0>();
        lr_read<T>(f0, s0, wm, wn, lane, 0);
        last(s0, s1, kt0);
        return;
    }
    lr_fetch<T>(L, s1, kp(kt0 + 1));
    lr_sync<LR_AU + LR_BU>();
    lr_read<T>(f0, s0, wm, wn, lane, 0);
    int kt = kt0;
    // steady state, branch-free: the stages rotate with the unrolled steps, so that each
    // step names its stages statically
    for (; kt + 4 < kt1; kt += 3) {
        step(s0, s1, s2, kt);
        step(s1, s2, s0, kt + 1);
        step(s2, s0, s1, kt + 2);
    }
    T *c0 = s0, *c1 = s1, *c2 = s2;
    for (; kt + 2 < kt1; ++kt) {
        step(c0, c1, c2, kt);
        T *t = c0;
        c0 = c1;
        c1 = c2;
        c2 = t;
    }
    for (; kt < kt1; ++kt) {
        last(c0, c1, kt);
        T *t = c0;
        c0 = c1;
        c1 = c2;
        c2 = t;
    }
}

// FP8 (E4M3) K loop of the rotated split form's correction term: acc += A B^T with 8-bit
// operands, K steps of 64 values (64-byte rows, the same bytes per stage as a 16-bit step of
// 32), loaded by the same loader into the same swizzled stages (the planes seen as 16-bit
// values). A lane's 32 bytes of a 32 x 32 x 64 MFMA operand are the two 16-byte chunks its
// half of the wave reads in the two sub-steps of a 16-bit step (chunks h and 2 + h): the same
// K values on both operands, so every K value meets its partner once.
typedef int intx8 __attribute__((ext_vector_type(8)));

// A fragments of a wave's 32-row tiles (re, im); the B fragments of its two 32-column tiles are
// read one tile at a time inside the MFMA sequence (fewer live registers).
struct Lr8Frag {
    intx8 ar[LR_MT], ai[LR_MT];
};

__device__ __forceinline__ intx8 lr_rd8(const void *p, int c0, int c1) {
    const char *b = static_cast<const char *>(p);
    const uint4 x = *reinterpret_cast<const uint4 *>(b + 2 * c0);
    const uint4 y = *reinterpret_cast<const uint4 *>(b + 2 * c1);
    intx8 r;
    r[0] = (int)x.x; r[1] = (int)x.y; r[2] = (int)x.z; r[3] = (int)x.w;
    r[4] = (int)y.x; r[5] = (int)y.y; r[6] = (int)y.z; r[7] = (int)y.w;
    return r;
}

template <typename T>
__device__ __forceinline__ void lr_read8(Lr8Frag &f, const T *st, int wm, int lane) {
    const int h = lane >> 5, sw = (lane >> 2) & 3;
    const int c0 = (h ^ sw) * 8, c1 = ((2 + h) ^ sw) * 8;
#pragma unroll
    for (int mt = 0; mt < LR_MT; ++mt) {
        const int o = (wm * (32 * LR_MT) + mt * 32 + (lane & 31)) * LR_BK;
        f.ar[mt] = lr_rd8(st + o, c0, c1);
        f.ai[mt] = lr_rd8(st + o + LR_AP, c0, c1);
    }
}

__device__ __forceinline__ floatx16 mfma_fp8(intx8 a, intx8 b, floatx16 c) {
    // E4M3 operands (format 0 on both sides), no block scales
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

template <typename T>
__device__ __forceinline__ void lr_mfma8(const Lr8Frag &f, const T *st, int wn, int lane,
                                         floatx16 (&acc_re)[LR_MT][2],
                                         floatx16 (&acc_im)[LR_MT][2]) {
    const int h = lane >> 5, sw = (lane >> 2) & 3;
    const int c0 = (h ^ sw) * 8, c1 = ((2 + h) ^ sw) * 8;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int o = 2 * LR_AP + (wn * 64 + nt * 32 + (lane & 31)) * LR_BK;
        const intx8 br = lr_rd8(st + o, c0, c1), bi = lr_rd8(st + o + LR_BP, c0, c1);
        intx8 bn;  // -b_im: the sign bit of every byte flipped
#pragma unroll
        for (int k = 0; k < 8; ++k) bn[k] = bi[k] ^ (int)0x80808080u;
#pragma unroll
        for (int mt = 0; mt < LR_MT; ++mt) {
            acc_re[mt][nt] = mfma_fp8(f.ar[mt], br, acc_re[mt][nt]);
            acc_im[mt][nt] = mfma_fp8(f.ar[mt], bi, acc_im[mt][nt]);
            acc_re[mt][nt] = mfma_fp8(f.ai[mt], bn, acc_re[mt][nt]);
            acc_im[mt][nt] = mfma_fp8(f.ai[mt], br, acc_im[mt][nt]);
        }
    }
}

// Loader of the FP8 pass: A = Rs in FP8 rows of a_ld bytes (a K step is the next 64 bytes of
// each row); B = the low part of b in blocks of 64 transducers, [part][block][node][64 bytes]
// (a K step is the next block, b_step bytes further). Same lane layout as lr_load.
__device__ __forceinline__ LrLoad lr_load8(const void *A, size_t a_plane, int a_row0, int a_ld,
                                           const void *B, size_t b_plane, int b_row0) {
    const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
    const int kc = (l & 3) ^ ((l >> 4) & 3);
    LrLoad L;
    L.ra = plane_rsrc(A, 2 * a_plane);
    L.rb = plane_rsrc(B, 2 * b_plane);
    L.a_off = (uint32_t)((size_t)(a_row0 + 16 * w + (l >> 2)) * a_ld + kc * 16);
    L.b_off = (uint32_t)((size_t)(b_row0 + 16 * w + (l >> 2)) * 64 + kc * 16);
    L.a_half = (uint32_t)((size_t)128 * a_ld);
    L.a_plane = (uint32_t)a_plane;
    L.b_plane = (uint32_t)b_plane;
    return L;
}

template <typename T>
__device__ __forceinline__ void lr_fetch8(const LrLoad &L, T *st, int kp, uint32_t b_step) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t ka = (uint32_t)kp * 64u, kb = (uint32_t)kp * b_step;
#pragma unroll
    for (int u = 0; u < LR_AU; ++u)
        load_lds16(L.ra, st + (w + 8 * u) * 512,
                   L.a_off + (u & 1) * L.a_half + (u >> 1) * L.a_plane, ka);
#pragma unroll
    for (int u = 0; u < LR_BU; ++u)
        load_lds16(L.rb, st + 2 * LR_AP + (w + 8 * u) * 512, L.b_off + u * L.b_plane, kb);
}

// Steps kt0 .. kt1 - 1 (step kt0 + i in stage i mod 3): after the barrier of step k its
// fragments are read and step k + 2 is fetched into the stage of step k - 1, which every
// wave finished reading before that barrier. The stages must be free when it starts (a
// barrier after their last reads); no load is outstanding when it returns.
template <typename T>
__device__ __forceinline__ void lr_mainloop8(T *s0, T *s1, T *s2, const LrLoad &L,
                                             uint32_t b_step, int kt0, int kt1,
                                             floatx16 (&acc_re)[LR_MT][2],
                                             floatx16 (&acc_im)[LR_MT][2]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    auto step = [&](T *cur, T *nn, int kt) {
        if (kt + 1 < kt1) lr_sync<LR_AU + LR_BU>();
        else lr_sync<0>();
        Lr8Frag f;
        lr_read8<T>(f, cur, wm, lane);
        if (kt + 2 < kt1) lr_fetch8<T>(L, nn, kt + 2, b_step);
        lr_mfma8<T>(f, cur, wn, lane, acc_re, acc_im);
    };
    if (kt0 >= kt1) return;
    lr_fetch8<T>(L, s0, kt0, b_step);
    if (kt0 + 1 < kt1) lr_fetch8<T>(L, s1, kt0 + 1, b_step);
    int kt = kt0;
    for (; kt + 3 <= kt1; kt += 3) {
        step(s0, s2, kt);
        step(s1, s0, kt + 1);
        step(s2, s1, kt + 2);
    }
    if (kt < kt1) step(s0, s2, kt);
    if (kt + 1 < kt1) step(s1, s0, kt + 1);
}

// The back-projection contractions of one launch: `count` independent problems (one per scan
// of a batch; count = 1 for a single call). Problem p owns items item0[p] .. item0[p+1]-1 of
// the launch's item list; XCD x walks items xcd0[x] .. xcd0[x+1]-1.
// With `full`, R' is the whole symmetric part of R and every row slab contracts over all of
// K (the split form: the epilogue's operand is h_hi + 2 h_lo, and the cross term
// 2 h_lo^T Rs h_hi needs Rs h_hi in every row); Hlo[p] (nullable) are the low parts.
struct RowGroup {
    int count;
    int full;
    // rot: the rotated operands of the frequency step (H, b, a). Component 0 is h = H as
    // before (over the block triangle Rp, or all of Rs in the split form); component 1
    // contracts b over the whole Rs in Rf[p] (in the split form then b's FP8 low part
    // against the FP8 Rs in R8[p], into the same accumulators, so Y = Rs b to first order),
    // and its epilogue takes a (component 2; split: a_hi + a_lo, weight 1).
    int rot;
    const void *R8[RB_GROUP_MAX];
    const void *Rf[RB_GROUP_MAX];
    int item0[RB_GROUP_MAX + 1];
    int xcd0[9];
    int n[RB_GROUP_MAX], n_cols[RB_GROUP_MAX];
    const void *Rp[RB_GROUP_MAX];
    const void *Ht[RB_GROUP_MAX];
    const void *Hlo[RB_GROUP_MAX];
    float *parts[RB_GROUP_MAX];
};

// Epilogue of one component: adds f sum_e E[e][q] Y[e][q] over the tile's rows to cs, with
// E staged in the three LDS stages by lr_fetch_e: four consecutive rows e per register group,
// one 8-byte LDS read per part. Rows are padded with zeros to np, a multiple of 32, so a
// 32-row group lies wholly inside np or wholly past it (uniform; such groups get weight 0 and
// read other finite data), and rows beyond n carry E = 0. Lanes of nodes past the last read
// other finite data; their sums are never stored.
template <typename T>
__device__ __forceinline__ void lr_epilogue(const T *s0, const T *s1, const T *s2, int row0,
                                            int np, const floatx16 (&acc_re)[LR_MT][2],
                                            const floatx16 (&acc_im)[LR_MT][2], float f,
                                            float (&cs_re)[2], float (&cs_im)[2]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int q = wn * 64 + nt * 32 + (lane & 31);
#pragma unroll
        for (int mt = 0; mt < LR_MT; ++mt) {
            const int eb = wm * (32 * LR_MT) + mt * 32;  // wave-uniform
            const int ch = eb / LR_ECH;
            const T *st = ch == 0 ? s0 : (ch == 1 ? s1 : s2);
            const int pr = ch == 2 ? (LR_BM - 2 * LR_ECH) / 8 : LR_ECH / 8;
            const int hq = lr_eswz(q, pr);
            const float rm = row0 + eb < np ? f : 0.f;
            float sr = 0.f, si = 0.f;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int el = eb - ch * LR_ECH + g * 8 + (lane >> 5) * 4;
                const int o = (q * pr + ((el >> 3) ^ hq)) * 8 + (el & 7);
                T vr[4], vi[4];
                __builtin_memcpy(vr, st + o, 8);
                __builtin_memcpy(vi, st + o + LR_BN * pr * 8, 8);
#pragma unroll
                for (int z = 0; z < 4; ++z) {
                    const float er = from_lp<T>(vr[z]), ei = from_lp<T>(vi[z]);
                    const float yr = acc_re[mt][nt][g * 4 + z];
                    const float yi = acc_im[mt][nt][g * 4 + z];
                    sr += er * yr - ei * yi;
                    si += er * yi + ei * yr;
                }
            }
            cs_re[nt] += rm * sr;
            cs_im[nt] += rm * si;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(LR_THREADS) rowred_lp_kernel(const RowGroup grp, int n_comp) {
    __shared__ __attribute__((aligned(1024))) T s0[LR_STAGE];
    __shared__ __attribute__((aligned(1024))) T s1[LR_STAGE];
    __shared__ __attribute__((aligned(1024))) T s2[LR_STAGE];
    __shared__ float red[2][LR_WM][LR_BN];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;  // LR_WM x 2 waves of 32 LR_MT x 64

    // Persistent: one workgroup per CU walks a static list of work items. An item is one
    // node tile and a pair of row slabs (i, mblocks - 1 - i), whose contractions start at
    // their diagonal blocks and together span mblocks + 1 blocks of K, so every item of a
    // problem costs the same. Workgroups are dealt to the 8 XCDs round-robin; each XCD walks
    // a contiguous range of items (both pairs of a node tile next to each other, sharing its
    // H tile in L2). Every slab walks K from the last block down: the two workgroups of a
    // node tile read the same rows of H at the same time for most of their first slabs, and
    // each slab's epilogue finds its diagonal block, read last, still in L2.
    const int L = gridDim.x >> 3, xcd = blockIdx.x & 7;
    const int x1 = grp.xcd0[xcd + 1];
    for (int item = grp.xcd0[xcd] + (blockIdx.x >> 3); item < x1; item += L) {
        int p = 0;
        while (p + 1 < grp.count && item >= grp.item0[p + 1]) ++p;
        const T *__restrict__ Rp = static_cast<const T *>(grp.Rp[p]);
        const T *__restrict__ Ht = static_cast<const T *>(grp.Ht[p]);
        const T *__restrict__ Hlo = static_cast<const T *>(grp.Hlo[p]);
        float *__restrict__ parts = grp.parts[p];
        const int n = grp.n[p], n_cols = grp.n_cols[p];
        const int mblocks = (n + LR_BM - 1) / LR_BM, n_pairs = (mblocks + 1) / 2;
        const int np = rb_lp_pad(n);  // padded row length (zeros past n), a multiple of LR_BK
        const size_t rplane = (size_t)n * np;
        const size_t hplane = (size_t)n_cols * np;
        const int KT = np / LR_BK;
        const int local = item - grp.item0[p];
        const int nb = local / n_pairs, pr = local - nb * n_pairs;
        for (int half = 0; half < 2; ++half) {
            const int mb = half == 0 ? pr : mblocks - 1 - pr;
            if (half == 1 && mb == pr) break;  // middle slab of an odd count
            const int row0 = mb * LR_BM, col0 = nb * LR_BN;
            // R' is zero left of the diagonal block (the whole row in the full form)
            const int KT0 = grp.full ? 0 : row0 / LR_BK;
            float cs_re[2] = {0.f, 0.f}, cs_im[2] = {0.f, 0.f};

            for (int c = 0; c < n_comp; ++c) {
                const T *Hc = Ht + (size_t)(2 * c) * hplane;
                const bool corr = grp.rot && c == 1;  // b over all of Rs, epilogue with a
                const int ce = corr ? 2 : c;          // component of the epilogue operand
                const T *Ra = corr ? static_cast<const T *>(grp.Rf[p]) : Rp;
                const LrLoad ld = lr_load<T>(Ra, rplane, row0, Hc, hplane, col0, np);
                floatx16 acc_re[LR_MT][2], acc_im[LR_MT][2];
#pragma unroll
                for (int mt = 0; mt < LR_MT; ++mt)
#pragma unroll
                    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                        for (int i = 0; i < 16; ++i) {
                            acc_re[mt][nt][i] = 0.f;
                            acc_im[mt][nt][i] = 0.f;
                        }
                lr_mainloop<T, true>(s0, s1, s2, ld, corr ? 0 : KT0, KT, acc_re, acc_im);
                if (corr && grp.R8[p]) {
                    // + Rs b_lo on FP8 operands (R8 = Rs / 2^6 in rows of rb_lp8_pad(n)
                    // bytes; b_lo times 2^6 in blocks of 64 transducers), K steps of 64
                    const int np8 = rb_lp8_pad(n);
                    const T *B8 = Hlo + (size_t)2 * hplane;  // the second low-part slot
                    const LrLoad l8 = lr_load8(grp.R8[p], (size_t)n * np8, row0, np8, B8,
                                               (size_t)n_cols * np8, col0);
                    __syncthreads();  // every wave is done with the 16-bit loop's stages
                    lr_mainloop8<T>(s0, s1, s2, l8, (uint32_t)n_cols * 64u, 0, np8 / 64, acc_re,
                                    acc_im);
                }
                // epilogue: E_c[e][q] = Ht_c[q][e] for the tile's 256 rows e and 128 nodes q,
                // staged through the three LDS stages (coalesced loads of row pieces of Ht_c);
                // a split operand adds its low part with weight 2 (h_hi + 2 h_lo against
                // Y = Rs h_hi: the first-order rounding of h on both sides), the rotated
                // form's second component a_hi + a_lo against Y = Rs b with weight 1
                const T *He = Ht + (size_t)(2 * ce) * hplane;
                __syncthreads();  // every wave is done with the K loop's stages
                lr_fetch_e<T>(He, hplane, np, row0, col0, s0, s1, s2);
                lr_sync<0>();
                lr_epilogue<T>(s0, s1, s2, row0, np, acc_re, acc_im, 1.f, cs_re, cs_im);
                __syncthreads();  // LDS buffers are refilled next
                if (Hlo && grp.rot) {
                    // FP8 low part (times 2^6) at the start of the component's low-part slot
                    const int np8 = rb_lp8_pad(n);
                    const uint8_t *lo8 = reinterpret_cast<const uint8_t *>(Hlo) +
                                         (size_t)ce * 4 * hplane;
                    lr_fetch_e8<T>(lo8, (size_t)n_cols * np8, n_cols, row0, col0, s0, s1);
                    lr_sync<0>();
                    lr_epilogue8<T>(s0, s1, row0, np, acc_re, acc_im,
                                    (corr ? 1.f : 2.f) * (1.f / 64.f), cs_re, cs_im);
                    __syncthreads();
                } else if (Hlo) {
                    lr_fetch_e<T>(Hlo + (size_t)(2 * ce) * hplane, hplane, np, row0, col0, s0,
                                  s1, s2);
                    lr_sync<0>();
                    lr_epilogue<T>(s0, s1, s2, row0, np, acc_re, acc_im, 2.f, cs_re, cs_im);
                    __syncthreads();
                }
            }
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                cs_re[nt] += __shfl_xor(cs_re[nt], 32);
                cs_im[nt] += __shfl_xor(cs_im[nt], 32);
                if (lane < 32) {
                    red[0][wm][wn * 64 + nt * 32 + lane] = cs_re[nt];
                    red[1][wm][wn * 64 + nt * 32 + lane] = cs_im[nt];
                }
            }
            __syncthreads();
            if (tid < LR_BN) {
                const int gc = col0 + tid;
                if (gc < n_cols) {
                    float sr = red[0][0][tid], si = red[1][0][tid];
#pragma unroll
                    for (int w2 = 1; w2 < LR_WM; ++w2) {
                        sr += red[0][w2][tid];
                        si += red[1][w2][tid];
                    }
                    parts[(size_t)mb * n_cols + gc] = sr;
                    parts[(size_t)(mblocks + mb) * n_cols + gc] = si;
                }
            }
            __syncthreads();  // red[] and the LDS tiles are reused by the next slab
        }
    }
}

// Forward: d[e][r] = sum_q G[e][q] v[q] G[r][q] on 16-bit operands, split-K, upper tiles ----
constexpr int LF_B = 128, LF_BK = 32, LF_LD = LF_BK + 8;

__device__ __forceinline__ void upper_tile(int idx, int T_, int &tm, int &tn) {
    int r = 0, rem = idx;
    while (rem >= T_ - r) {
        rem -= T_ - r;
        ++r;
    }
    tm = r;
    tn = r + rem;
}

template <typename T>
__global__ void __launch_bounds__(256) forward_lp_kernel(const T *__restrict__ Gp,
                                                         const float2 *__restrict__ w,
                                                         const float *__restrict__ delta, int n,
                                                         int K, int ld, int nT, int kchunk,
                                                         int splitk,
                                                         const float *__restrict__ vscale,
                                                         float2 *__restrict__ dpart) {
    __shared__ __attribute__((aligned(16))) T a_s[2][LF_B][LF_LD];
    const float vs = vscale[0];
    __shared__ __attribute__((aligned(16))) T b_s[2][LF_B][LF_LD];
    // Workgroups are dealt to the 8 XCDs round-robin. Every tile of one K chunk goes to the
    // same XCD (chunk s to XCD s mod 8), so the chunk's columns of G come from HBM once and
    // serve all tiles from that XCD's L2.
    const int tiles = nT * (nT + 1) / 2;
    const int kq = blockIdx.x >> 3;
    const int split = (kq / tiles) * 8 + (blockIdx.x & 7);
    if (split >= splitk) return;
    int tm, tn;
    upper_tile(kq % tiles, nT, tm, tn);
    const int kbeg = split * kchunk, kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int row0 = tm * LF_B, col0 = tn * LF_B;
    const size_t gplane = (size_t)n * ld;

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

    // each tile: 128 rows x 4 chunks of 8 K = 512 (row, chunk) pairs, 2 per thread
    const bool kvec = (ld % 8) == 0;
    for (int k0 = kbeg; k0 < kend; k0 += LF_BK) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int idx = tid + u * 256;
            int ch = idx & 3, row = idx >> 2;
            int gk = k0 + ch * 8;
            int ge = row0 + row, gr = col0 + row;
            // v = w delta for the 8 node indices of this chunk (absent: G carries it)
            float vr[8], vi[8];
            if (w) {
#pragma unroll
                for (int z = 0; z < 8; ++z) {
                    int k = gk + z;
                    float2 wv = make_float2(0.f, 0.f);
                    float dl = 0.f;
                    if (k < kend) {
                        wv = w[k];
                        dl = delta[k] * vs;
                    }
                    vr[z] = wv.x * dl;
                    vi[z] = wv.y * dl;
                }
            }
            // 8 consecutive K of one row of G (both parts), zero beyond the chunk end
            auto row8 = [&](int grow, T *re, T *im) {
                if (grow < n && kvec && gk + 7 < kend) {
                    uint4 a = *reinterpret_cast<const uint4 *>(Gp + (size_t)grow * ld + gk);
                    uint4 b = *reinterpret_cast<const uint4 *>(Gp + gplane + (size_t)grow * ld + gk);
                    __builtin_memcpy(re, &a, 16);
                    __builtin_memcpy(im, &b, 16);
                } else {
#pragma unroll
                    for (int z = 0; z < 8; ++z) {
                        bool ok = grow < n && gk + z < kend;
                        re[z] = ok ? Gp[(size_t)grow * ld + gk + z] : to_lp<T>(0.f);
                        im[z] = ok ? Gp[gplane + (size_t)grow * ld + gk + z] : to_lp<T>(0.f);
                    }
                }
            };
            T ar[8], ai[8], br[8], bi[8];
            row8(ge, ar, ai);
            row8(gr, br, bi);
            // A = G v, complex product in FP32 rounded once to the operand type
            if (w) {
#pragma unroll
                for (int z = 0; z < 8; ++z) {
                    float gre = from_lp<T>(ar[z]), gim = from_lp<T>(ai[z]);
                    ar[z] = to_lp<T>(gre * vr[z] - gim * vi[z]);
                    ai[z] = to_lp<T>(gre * vi[z] + gim * vr[z]);
                }
            }
            *reinterpret_cast<uint4 *>(&a_s[0][row][ch * 8]) = __builtin_bit_cast(uint4, ar);
            *reinterpret_cast<uint4 *>(&a_s[1][row][ch * 8]) = __builtin_bit_cast(uint4, ai);
            *reinterpret_cast<uint4 *>(&b_s[0][row][ch * 8]) = __builtin_bit_cast(uint4, br);
            *reinterpret_cast<uint4 *>(&b_s[1][row][ch * 8]) = __builtin_bit_cast(uint4, bi);
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < LF_BK; ks += 16) {
            int kk = ks + (lane >> 5) * 8;
            uint4 ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                int m = wm * 64 + mt * 32 + (lane & 31);
                ar[mt] = *reinterpret_cast<const uint4 *>(&a_s[0][m][kk]);
                ai[mt] = *reinterpret_cast<const uint4 *>(&a_s[1][m][kk]);
                nai[mt] = neg8(ai[mt]);
            }
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                int cn = wn * 64 + nt * 32 + (lane & 31);
                br[nt] = *reinterpret_cast<const uint4 *>(&b_s[0][cn][kk]);
                bi[nt] = *reinterpret_cast<const uint4 *>(&b_s[1][cn][kk]);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 2; ++nt) {
                    acc_re[mt][nt] =
                        Lp<T>::mfma(as_vec<T>(ar[mt]), as_vec<T>(br[nt]), acc_re[mt][nt]);
                    acc_re[mt][nt] =
                        Lp<T>::mfma(as_vec<T>(nai[mt]), as_vec<T>(bi[nt]), acc_re[mt][nt]);
                    acc_im[mt][nt] =
                        Lp<T>::mfma(as_vec<T>(ar[mt]), as_vec<T>(bi[nt]), acc_im[mt][nt]);
                    acc_im[mt][nt] =
                        Lp<T>::mfma(as_vec<T>(ai[mt]), as_vec<T>(br[nt]), acc_im[mt][nt]);
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

// Forward on operands that already carry sqrt(v): d[e][r] = sum_q G[e][q] G[r][q], on the
// pipelined K loop of the back-projection. Tiles LR_BM (e) x LR_BN (r) cover the upper
// triangle (row block tm takes column blocks from tm LR_BM / LR_BN on); K (nodes) is split
// into chunks of kchunk steps, each workgroup writing its chunk's partial sums of the tile's
// elements with e <= r. Workgroups are dealt to the 8 XCDs round-robin: every tile of one
// chunk goes to the same XCD, so the chunk's columns of G come from HBM once. Rows of G are
// ld long with zeros past the last node; rows past n read other finite data or zeros and
// only reach outputs that are not stored. A launch serves `count` independent problems (the
// scans of a batch; one for a single call): problem p takes workgroups blk0[p] ..
// blk0[p+1]-1, blk0[p] a multiple of 8, so the XCD of a workgroup is that of its local index.
struct FwdGroup {
    int count;
    int blk0[RB_GROUP_MAX + 1];
    int n[RB_GROUP_MAX], ld[RB_GROUP_MAX], nT[RB_GROUP_MAX], tiles[RB_GROUP_MAX];
    int kchunk[RB_GROUP_MAX], splitk[RB_GROUP_MAX];
    const void *G[RB_GROUP_MAX];
    float2 *dpart[RB_GROUP_MAX];
};

template <typename T>
__global__ void __launch_bounds__(LR_THREADS) forward_pipe_kernel(const FwdGroup grp) {
    __shared__ __attribute__((aligned(1024))) T s0[LR_STAGE];
    __shared__ __attribute__((aligned(1024))) T s1[LR_STAGE];
    __shared__ __attribute__((aligned(1024))) T s2[LR_STAGE];
    int p = 0;
    while (p + 1 < grp.count && (int)blockIdx.x >= grp.blk0[p + 1]) ++p;
    const T *__restrict__ Gp = static_cast<const T *>(grp.G[p]);
    float2 *__restrict__ dpart = grp.dpart[p];
    const int n = grp.n[p], ld = grp.ld[p], nTn = grp.nT[p], tiles = grp.tiles[p];
    const int kchunk = grp.kchunk[p], splitk = grp.splitk[p];
    const int blk = (int)blockIdx.x - grp.blk0[p];
    const int kq = blk >> 3;
    const int split = (kq / tiles) * 8 + (blk & 7);
    if (split >= splitk) return;  // whole workgroup: no barrier is skipped by part of it
    constexpr int RB = LR_BM / LR_BN;  // column blocks per row block
    int rem = kq % tiles, tm = 0;
    while (rem >= nTn - tm * RB) {
        rem -= nTn - tm * RB;
        ++tm;
    }
    const int tn = tm * RB + rem;
    const int row0 = tm * LR_BM, col0 = tn * LR_BN;
    const int KT = ld / LR_BK;
    const int kt0 = split * kchunk, kt1 = min(KT, kt0 + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const size_t gplane = (size_t)n * ld;
    const LrLoad L = lr_load<T>(Gp, gplane, row0, Gp, gplane, col0, ld);
    floatx16 acc_re[LR_MT][2], acc_im[LR_MT][2];
#pragma unroll
    for (int mt = 0; mt < LR_MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                acc_re[mt][nt][i] = 0.f;
                acc_im[mt][nt][i] = 0.f;
            }
    lr_mainloop<T, false>(s0, s1, s2, L, kt0, kt1, acc_re, acc_im);
    float2 *out = dpart + (size_t)split * n * n;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int gc = col0 + wn * 64 + nt * 32 + (lane & 31);
        if (gc >= n) continue;
#pragma unroll
        for (int mt = 0; mt < LR_MT; ++mt)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int gr = row0 + wm * (32 * LR_MT) + mt * 32 + mfma_row(lane, i);
                if (gr <= gc)
                    out[(size_t)gr * n + gc] = make_float2(acc_re[mt][nt][i], acc_im[mt][nt][i]);
            }
    }
}

__global__ void forward_reduce_lp(const float2 *__restrict__ dpart, int n, int splitk,
                                  const float *__restrict__ vscale,
                                  const float *__restrict__ rows, float2 *__restrict__ d) {
    int r = blockIdx.x * blockDim.x + threadIdx.x, e = blockIdx.y;
    if (r >= n) return;
    size_t src = (e <= r) ? (size_t)e * n + r : (size_t)r * n + e;
    float sr = 0.f, si = 0.f;
    for (int s = 0; s < splitk; ++s) {
        float2 v = dpart[(size_t)s * n * n + src];
        sr += v.x;
        si += v.y;
    }
    // the rows of G carry the per-transducer scales (powers of two: exact)
    float inv = vscale[1] / (rows[e] * rows[r]);
    d[(size_t)e * n + r] = make_float2(sr * inv, si * inv);
}

// Seeded operand of the autotuner: magnitude in [0.5, 1), sign and phase from a hash of the
// index; zeros in the padding past n_mask (as rb_build_green writes).
template <typename T>
__global__ void tune_fill_kernel(T *__restrict__ G, int n, int ld, int n_mask) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = 2 * (size_t)n * ld;
    if (i >= total) return;
    const int k = (int)(i % (size_t)ld);
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    const float v = (0.5f + 0.5f * (float)(h & 0xffff) / 65536.f) * ((h & 0x10000) ? -1.f : 1.f);
    G[i] = to_lp<T>(k < n_mask ? v : 0.f);
}

__global__ void tune_fill_f32_kernel(float *__restrict__ G, size_t count) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    G[i] = (0.5f + 0.5f * (float)(h & 0xffff) / 65536.f) * ((h & 0x10000) ? -1.f : 1.f);
}

__global__ void ones_kernel(float *x, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 1.f;
}

__global__ void unit_scale_kernel(float *s) {
    s[0] = 1.f;
    s[1] = 1.f;
}

}  // namespace

rb_status rb_launch_tune_fill(rb_ctx *ctx, const rb_green *gr, float *gscale) {
    const int n = gr->n, nm = gr->n_mask;
    if (gr->prec == RB_F32) {
        const size_t count = 2 * (size_t)n * nm;
        hipLaunchKernelGGL(tune_fill_f32_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256),
                           0, ctx->stream, (float *)gr->G, count);
    } else {
        const int ld = rb_lp_pad(nm);
        const size_t total = 2 * (size_t)n * ld;
        if (gr->prec == RB_BF16)
            hipLaunchKernelGGL(tune_fill_kernel<__bf16>, dim3((unsigned)((total + 255) / 256)),
                               dim3(256), 0, ctx->stream, (__bf16 *)gr->G, n, ld, nm);
        else
            hipLaunchKernelGGL(tune_fill_kernel<_Float16>, dim3((unsigned)((total + 255) / 256)),
                               dim3(256), 0, ctx->stream, (_Float16 *)gr->G, n, ld, nm);
    }
    RB_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(unit_scale_kernel, dim3(1), dim3(1), 0, ctx->stream, gscale);
    RB_CHECK_LAUNCH(ctx);
    if (gr->prec != RB_F32 && gr->scales) {  // unscaled rows
        hipLaunchKernelGGL(ones_kernel, dim3((2 * n + 255) / 256), dim3(256), 0, ctx->stream,
                           gr->scales, 2 * n);
        RB_CHECK_LAUNCH(ctx);
    }
    return RB_OK;
}

// Launchers ------------------------------------------------------------------------------
// Bound of |sqrt(v)| scaled to [1, 2) per part, as G carries it: |re|, |im| < 2.
constexpr float GS_MAX = 2.8285f;

rb_status rb_launch_green_lp(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                             const rb_green *out, const float *gs, const float *gscale,
                             int write_g, unsigned int *rowmax) {
    dim3 grd((tb->n_mask + GQ - 1) / GQ, (tb->n + GE - 1) / GE);
    rb_prof_begin(ctx, ST_GREEN);
    hipLaunchKernelGGL(row_amax_kernel, dim3(tb->n), dim3(256), 0, ctx->stream, *tb, tb->n_mask,
                       rowmax);
    RB_CHECK_LAUNCH(ctx);
    const float gmax = gs ? GS_MAX : 1.f;
    const size_t hlo = 6 * (size_t)tb->n_mask * rb_lp_pad(tb->n);  // low parts follow H
    if (out->prec == RB_BF16)
        hipLaunchKernelGGL((green_lp_kernel<__bf16, false>), grd, dim3(256), 0, ctx->stream, *tb,
                           tb->n, tb->n_mask, omega, c0, (const float2 *)gs, gscale, write_g,
                           (__bf16 *)out->G, (__bf16 *)out->H, rowmax, gmax, out->scales,
                           nullptr);
    else if (rb_prec_split(out->prec))
        hipLaunchKernelGGL((green_lp_kernel<_Float16, true>), grd, dim3(256), 0, ctx->stream, *tb,
                           tb->n, tb->n_mask, omega, c0, (const float2 *)gs, gscale, write_g,
                           (_Float16 *)out->G, (_Float16 *)out->H, rowmax, gmax, out->scales,
                           (_Float16 *)out->H + hlo);
    else
        hipLaunchKernelGGL((green_lp_kernel<_Float16, false>), grd, dim3(256), 0, ctx->stream,
                           *tb, tb->n, tb->n_mask, omega, c0, (const float2 *)gs, gscale,
                           write_g, (_Float16 *)out->G, (_Float16 *)out->H, rowmax, gmax,
                           out->scales, nullptr);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_green_lp_rec(rb_ctx *ctx, const float4 *rec, const double2 *ring, int n,
                                 double omega, double c0, const rb_green *out, const float *gs,
                                 const float *gscale, int write_g, const unsigned int *rowmax) {
    const int nm = (int)ctx->n_mask;
    const rb_grid &g = ctx->grid;
    // the split form holds twice the packed rows per lane: 8 transducers per wave (8 waves
    // per workgroup, so a workgroup still writes 128-byte row pieces of H) keep it at 4 waves
    // per SIMD
    constexpr int GWS = 8;
    dim3 grd((nm + GQ - 1) / GQ, (n + GE - 1) / GE);
    const float gmax = gs ? GS_MAX : 1.f;
    const size_t hlo = 6 * (size_t)nm * rb_lp_pad(n);  // low parts follow H
    rb_prof_begin(ctx, ST_GREEN);
    hipLaunchKernelGGL(row_scale_kernel, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, rowmax,
                       n, omega, c0, gmax, out->scales);
    RB_CHECK_LAUNCH(ctx);
    if (out->prec == RB_BF16)
        hipLaunchKernelGGL((green_lp_rec_kernel<__bf16, false, GW, 4>), grd, dim3(256), 0, ctx->stream,
                           rec, ctx->d_mask_index, ring, g.x0, g.y0, g.dx, g.nx, n, nm, omega,
                           c0, (const float2 *)gs, gscale, write_g, (__bf16 *)out->G,
                           (__bf16 *)out->H, out->scales, nullptr);
    else if (rb_prec_split(out->prec))
        hipLaunchKernelGGL((green_lp_rec_kernel<_Float16, true, GWS, 8>), grd, dim3(512), 0, ctx->stream,
                           rec, ctx->d_mask_index, ring, g.x0, g.y0, g.dx, g.nx, n, nm, omega,
                           c0, (const float2 *)gs, gscale, write_g, (_Float16 *)out->G,
                           (_Float16 *)out->H, out->scales, (_Float16 *)out->H + hlo);
    else
        hipLaunchKernelGGL((green_lp_rec_kernel<_Float16, false, GW, 4>), grd, dim3(256), 0,
                           ctx->stream, rec, ctx->d_mask_index, ring, g.x0, g.y0, g.dx, g.nx, n,
                           nm, omega, c0, (const float2 *)gs, gscale, write_g,
                           (_Float16 *)out->G, (_Float16 *)out->H, out->scales, nullptr);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_to_planar(rb_ctx *ctx, rb_prec prec, const float *R, int n, void *Rp,
                              float *scale, const float *rows, void *R8, void *Rfull) {
    size_t nn = (size_t)n * n;
    const int np = rb_lp_pad(n);
    rb_prof_begin(ctx, ST_RESIDUAL);
    // |R'| <= 2 max |R|: scale max |R| to [2^12, 2^13) so R' stays below 2^14
    RB_TRY(launch_range_scale(ctx, (const float2 *)R, nn, nullptr, 13, scale, rows, n));
    size_t npad = (size_t)n * np;
    dim3 grd((unsigned)((npad + 255) / 256));
    // block size of the triangle; one block (the whole symmetric part) for the split form
    const int bm = rb_prec_split(prec) ? np : LR_BM;
    if (prec == RB_BF16)
        hipLaunchKernelGGL(to_planar_kernel<__bf16>, grd, dim3(256), 0, ctx->stream,
                           (const float2 *)R, n, np, bm, scale, rows, (__bf16 *)Rp);
    else
        hipLaunchKernelGGL(to_planar_kernel<_Float16>, grd, dim3(256), 0, ctx->stream,
                           (const float2 *)R, n, np, bm, scale, rows, (_Float16 *)Rp);
    RB_CHECK_LAUNCH(ctx);
    if (Rfull && Rfull != Rp) {  // one block: the whole symmetric part
        if (prec == RB_BF16)
            hipLaunchKernelGGL(to_planar_kernel<__bf16>, grd, dim3(256), 0, ctx->stream,
                               (const float2 *)R, n, np, np, scale, rows, (__bf16 *)Rfull);
        else
            hipLaunchKernelGGL(to_planar_kernel<_Float16>, grd, dim3(256), 0, ctx->stream,
                               (const float2 *)R, n, np, np, scale, rows, (_Float16 *)Rfull);
        RB_CHECK_LAUNCH(ctx);
    }
    if (R8) {
        const size_t nw = (size_t)n * (rb_lp8_pad(n) / 4);
        hipLaunchKernelGGL(to_fp8_kernel, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0,
                           ctx->stream, (const float2 *)R, n, rb_lp8_pad(n), scale, rows,
                           (uint32_t *)R8);
        RB_CHECK_LAUNCH(ctx);
    }
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_transpose_conj(rb_ctx *ctx, const rb_green *gr, void *Gt) {
    const int Np = rb_lp_pad(gr->n);
    dim3 grd((gr->n_mask + 63) / 64, (Np + 63) / 64);
    hipLaunchKernelGGL(transpose_conj_kernel, grd, dim3(256), 0, ctx->stream,
                       (const uint16_t *)gr->G, gr->n, gr->n_mask, (uint16_t *)Gt);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

rb_status rb_launch_range_scale(rb_ctx *ctx, const float *x, size_t count, int top, float *scale) {
    return launch_range_scale(ctx, (const float2 *)x, count, nullptr, top, scale);
}

rb_status rb_launch_unscale(rb_ctx *ctx, float *parts, size_t count, const float *scale) {
    hipLaunchKernelGGL(unscale_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                       ctx->stream, parts, count, scale);
    RB_CHECK_LAUNCH(ctx);
    return RB_OK;
}

int rb_rowred_lp_mblocks(int n) { return (n + LR_BM - 1) / LR_BM; }

rb_status rb_launch_rowred_lp_group(rb_ctx *ctx, rb_prec prec, const rb_rowred_prob *pr,
                                    int count, int n_comp) {
    if (count < 1 || count > RB_GROUP_MAX)
        return rb_fail(ctx, RB_EINVAL, "grouped back-projection of %d problems", count);
    RowGroup g{};
    g.count = count;
    g.full = rb_prec_split(prec) ? 1 : 0;
    g.rot = pr[0].Rf ? 1 : 0;
    if (g.rot) n_comp = 2;
    int64_t items = 0, cost = 0;
    int64_t pcost[RB_GROUP_MAX];  // cost of one item of each problem (K blocks it walks)
    for (int i = 0; i < count; ++i) {
        const int n = pr[i].n, n_mask = pr[i].n_mask;
        const int mblocks = rb_rowred_lp_mblocks(n);
        const int nblocks = (n_mask + LR_BN - 1) / LR_BN;
        // byte offsets into the two part planes of an operand, padding rows included, must
        // stay below LR_SPAN (32-bit buffer offsets)
        const size_t np = (size_t)rb_lp_pad(n);
        const size_t span = (2 * (size_t)n_mask + LR_BN + (size_t)mblocks * LR_BM) * np * 2 + 64;
        if (span >= LR_SPAN)
            return rb_fail(ctx, RB_EUNSUPPORTED,
                           "16-bit back-projection: H planes of %d nodes x %zu exceed 4 GiB",
                           n_mask, np);
        g.item0[i] = (int)items;
        g.n[i] = n;
        g.n_cols[i] = n_mask;
        g.Rp[i] = pr[i].Rp;
        g.Ht[i] = pr[i].Ht;
        g.Hlo[i] = pr[i].Hlo;
        g.R8[i] = pr[i].R8;
        g.Rf[i] = pr[i].Rf;
        // rotated forms: Rf everywhere; split: its low parts and FP8 Rs everywhere too
        if ((pr[i].Rf != nullptr) != (g.rot != 0) ||
            (g.rot && g.full && (!pr[i].Hlo || !pr[i].R8)) || (!g.full && pr[i].R8))
            return rb_fail(ctx, RB_EINVAL, "grouped back-projection: mixed operand forms");
        g.parts[i] = pr[i].parts;
        const int64_t it = (int64_t)nblocks * ((mblocks + 1) / 2);
        // K blocks of 256 an item walks (per component; rotated: in all, the FP8 pass as half)
        pcost[i] = !g.rot ? (g.full ? 2 * mblocks : mblocks + 1)
                          : (g.full ? 5 * mblocks : 3 * mblocks + 1);
        items += it;
        cost += it * pcost[i];
    }
    if (items >= (int64_t)1 << 30)
        return rb_fail(ctx, RB_EUNSUPPORTED, "grouped back-projection of %lld items",
                       (long long)items);
    g.item0[count] = (int)items;
    if (count == 1) {
        // even-sized ranges: both slab pairs of a node tile stay on one XCD
        const int per = (int)((((items + 7) / 8) + 1) & ~int64_t(1));
        for (int x = 0; x <= 8; ++x) g.xcd0[x] = (int)std::min<int64_t>((int64_t)x * per, items);
    } else {
        // XCD ranges of equal cost: the items of different problems cost differently
        g.xcd0[0] = 0;
        for (int x = 1; x < 8; ++x) {
            const int64_t target = cost * x / 8;
            int64_t cum = 0;
            int i = 0;
            for (; i + 1 < count; ++i) {
                const int64_t c_i = (int64_t)(g.item0[i + 1] - g.item0[i]) * pcost[i];
                if (cum + c_i > target) break;
                cum += c_i;
            }
            const int64_t n_i = g.item0[i + 1] - g.item0[i];
            int64_t local = (target - cum + pcost[i] - 1) / pcost[i];
            local = std::min<int64_t>((local + 1) & ~int64_t(1), n_i);
            g.xcd0[x] = std::max<int>(g.xcd0[x - 1], (int)(g.item0[i] + local));
        }
        g.xcd0[8] = (int)items;
    }
    const int grid = std::max(8, ctx->n_cu / 8 * 8);  // one workgroup per CU (persistent)
    rb_prof_begin(ctx, ST_BACKPROJECT);
    if (prec == RB_BF16)
        hipLaunchKernelGGL(rowred_lp_kernel<__bf16>, dim3(grid), dim3(LR_THREADS), 0, ctx->stream,
                           g, n_comp);
    else
        hipLaunchKernelGGL(rowred_lp_kernel<_Float16>, dim3(grid), dim3(LR_THREADS), 0,
                           ctx->stream, g, n_comp);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_rowred_lp(rb_ctx *ctx, rb_prec prec, int n, int n_mask, const void *Rp,
                              const void *Ht, int n_comp, float *parts, int *mblocks_out,
                              const void *Hlo, const void *R8, const void *Rf) {
    const rb_rowred_prob pr{Rp, Ht, parts, n, n_mask, Hlo, R8, Rf};
    RB_TRY(rb_launch_rowred_lp_group(ctx, prec, &pr, 1, n_comp));
    if (mblocks_out) *mblocks_out = rb_rowred_lp_mblocks(n);
    return RB_OK;
}

namespace {
struct FwdShape {
    int nT, tiles, kchunk, splitk;
    unsigned nblk;
};

// Tiles and K split of the 16-bit forward for n transducers over K nodes (rows ld long).
// pipe: the pipelined kernel (256 x 128 upper tiles); else the 128 x 128 kernel. splitk > 0
// overrides the built-in K split (a tuned configuration).
FwdShape forward_shape(int n, int K, int ld, bool pipe, int n_cu, int splitk = 0) {
    FwdShape f{};
    const int ksteps = pipe ? ld / LR_BK : (K + LF_BK - 1) / LF_BK;
    if (splitk > 0) {
        f.nT = pipe ? (n + LR_BN - 1) / LR_BN : (n + LF_B - 1) / LF_B;
        f.tiles = 0;
        if (pipe)
            for (int tm = 0; tm * (LR_BM / LR_BN) < f.nT; ++tm)
                f.tiles += f.nT - tm * (LR_BM / LR_BN);
        else
            f.tiles = f.nT * (f.nT + 1) / 2;
        f.splitk = std::max(1, std::min(splitk, ksteps));
    } else if (pipe) {
        f.nT = (n + LR_BN - 1) / LR_BN;
        f.tiles = 0;
        for (int tm = 0; tm * (LR_BM / LR_BN) < f.nT; ++tm) f.tiles += f.nT - tm * (LR_BM / LR_BN);
        // K chunks in multiples of 8 (one XCD per chunk group): the fewest that fill the
        // device at least 1.5 times over with at most 7 % of the last round idle
        const int cu = std::max(8, n_cu);
        f.splitk = 8;
        for (int s8 = 8; s8 <= 1024; s8 += 8) {
            const long blocks = (long)f.tiles * s8, rounds = (blocks + cu - 1) / cu;
            f.splitk = s8;
            if (ksteps / s8 < 8) break;
            if (2 * blocks >= 3L * cu && (double)blocks / (double)(rounds * cu) >= 0.93) break;
        }
        f.splitk = std::max(1, std::min(f.splitk, ksteps));
    } else {
        f.nT = (n + LF_B - 1) / LF_B;
        f.tiles = f.nT * (f.nT + 1) / 2;
        f.splitk = (1024 + f.tiles - 1) / f.tiles;
        f.splitk = std::max(1, std::min(f.splitk, std::max(1, ksteps / 4)));
        f.splitk = (f.splitk + 7) / 8 * 8;  // K chunks spread evenly over the 8 XCDs
    }
    f.kchunk = (ksteps + f.splitk - 1) / f.splitk;
    f.splitk = (ksteps + f.kchunk - 1) / f.kchunk;
    f.nblk = (unsigned)(f.tiles * ((f.splitk + 7) / 8) * 8);
    return f;
}

bool forward_pipe_fits(int n, int n_mask) {
    return 2 * (size_t)n * rb_lp_pad(n_mask) * 2 <= LR_SPAN;
}
}  // namespace

int rb_forward_lp_default_splitk(int n, int n_mask, int pipe, int n_cu) {
    return forward_shape(n, n_mask, rb_lp_pad(n_mask), pipe && forward_pipe_fits(n, n_mask),
                         n_cu).splitk;
}

size_t rb_forward_lp_ws_bytes(int n, int n_mask, int n_cu) {
    int spk = RB_TUNE_SPLITK_MAX;
    spk = std::max(spk, rb_forward_lp_default_splitk(n, n_mask, 1, n_cu));
    spk = std::max(spk, rb_forward_lp_default_splitk(n, n_mask, 0, n_cu));
    return rb_align((size_t)spk * n * n * sizeof(float2)) + rb_align(8);
}

// Tuned configuration of the forward on operands that carry sqrt(v): kernel and K split.
static void forward_choice(const rb_ctx *ctx, const rb_green *gr, bool *pipe, int *splitk) {
    *pipe = forward_pipe_fits(gr->n, gr->n_mask);
    *splitk = 0;
    if (const rb_tuning *t = rb_tuned(ctx, gr->n, gr->n_mask, gr->prec)) {
        *pipe = *pipe && t->fwd_tile == RB_TILE_256x128;
        *splitk = t->fwd_splitk;
    }
}

rb_status rb_forward_lp_plan(rb_ctx *ctx, const rb_green *gr, const float *gscale,
                             rb_fwd_plan *pl) {
    const int n = gr->n, K = gr->n_mask, ld = rb_lp_pad(K);
    int spk = 0;
    forward_choice(ctx, gr, &pl->pipe, &spk);
    const FwdShape f = forward_shape(n, K, ld, pl->pipe, ctx->n_cu, spk);
    ctx->ws.used = 0;
    RB_TRY(rb_arena_reserve(
        ctx, &ctx->ws, rb_align((size_t)f.splitk * n * n * sizeof(float2)) + rb_align(8)));
    pl->gr = *gr;
    pl->gscale = gscale;
    pl->n = n;
    pl->ld = ld;
    pl->nT = f.nT;
    pl->tiles = f.tiles;
    pl->kchunk = f.kchunk;
    pl->splitk = f.splitk;
    pl->nblk = f.nblk;
    pl->dpart = rb_carve<float2>(&ctx->ws, (size_t)f.splitk * n * n);
    pl->vscale = rb_carve<float>(&ctx->ws, 2);
    return RB_OK;
}

rb_status rb_launch_forward_lp_group(rb_ctx *ctx, rb_prec prec, const rb_fwd_plan *pl,
                                     int count) {
    if (count < 1 || count > RB_GROUP_MAX)
        return rb_fail(ctx, RB_EINVAL, "grouped forward of %d problems", count);
    FwdGroup g{};
    g.count = count;
    int64_t blk = 0;
    for (int i = 0; i < count; ++i) {
        if (!pl[i].pipe || pl[i].gr.prec != prec)
            return rb_fail(ctx, RB_EINVAL, "grouped forward: problem %d does not fit", i);
        g.blk0[i] = (int)blk;
        g.n[i] = pl[i].n;
        g.ld[i] = pl[i].ld;
        g.nT[i] = pl[i].nT;
        g.tiles[i] = pl[i].tiles;
        g.kchunk[i] = pl[i].kchunk;
        g.splitk[i] = pl[i].splitk;
        g.G[i] = pl[i].gr.G;
        g.dpart[i] = pl[i].dpart;
        blk += pl[i].nblk;
    }
    if (blk >= (int64_t)1 << 30)
        return rb_fail(ctx, RB_EUNSUPPORTED, "grouped forward of %lld workgroups", (long long)blk);
    g.blk0[count] = (int)blk;
    rb_prof_begin(ctx, ST_FORWARD);
    // G already carries sqrt(v) s: undo s^2 (or nothing) in the reduction
    for (int i = 0; i < count; ++i) {
        hipLaunchKernelGGL(square_scale_kernel, dim3(1), dim3(1), 0, ctx->stream, pl[i].gscale,
                           pl[i].vscale);
        RB_CHECK_LAUNCH(ctx);
    }
    if (prec == RB_BF16)
        hipLaunchKernelGGL(forward_pipe_kernel<__bf16>, dim3((unsigned)blk), dim3(LR_THREADS), 0,
                           ctx->stream, g);
    else
        hipLaunchKernelGGL(forward_pipe_kernel<_Float16>, dim3((unsigned)blk), dim3(LR_THREADS),
                           0, ctx->stream, g);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_forward_lp_reduce(rb_ctx *ctx, const rb_fwd_plan *pl, float *d) {
    rb_prof_begin(ctx, ST_FORWARD_REDUCE);
    hipLaunchKernelGGL(forward_reduce_lp, dim3((pl->n + 255) / 256, pl->n), dim3(256), 0,
                       ctx->stream, pl->dpart, pl->n, pl->splitk, pl->vscale, pl->gr.scales,
                       (float2 *)d);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_forward_lp(rb_ctx *ctx, const rb_green *gr, const float *w,
                               const float *delta, float *d, const float *gscale) {
    const int n = gr->n, K = gr->n_mask, ld = rb_lp_pad(K);
    // Operands that carry sqrt(v) take the pipelined kernel while G's two planes fit one
    // buffer descriptor (unless a tuning chose the 128 x 128 tiles); the node weights of the
    // standalone call are folded in on the fly.
    bool pipe = false;
    int spk = 0;
    if (!w) forward_choice(ctx, gr, &pipe, &spk);
    if (pipe) {
        rb_fwd_plan pl;
        RB_TRY(rb_forward_lp_plan(ctx, gr, gscale, &pl));
        RB_TRY(rb_launch_forward_lp_group(ctx, gr->prec, &pl, 1));
        return rb_forward_lp_reduce(ctx, &pl, d);
    }
    const FwdShape f = forward_shape(n, K, ld, false, ctx->n_cu, spk);
    ctx->ws.used = 0;
    RB_TRY(rb_arena_reserve(
        ctx, &ctx->ws, rb_align((size_t)f.splitk * n * n * sizeof(float2)) + rb_align(8)));
    rb_fwd_plan pl;
    pl.gr = *gr;
    pl.n = n;
    pl.splitk = f.splitk;
    pl.dpart = rb_carve<float2>(&ctx->ws, (size_t)f.splitk * n * n);
    pl.vscale = rb_carve<float>(&ctx->ws, 2);
    rb_prof_begin(ctx, ST_FORWARD);
    if (w) {
        // range scale of v = w delta (the node weights are folded into the A operand): the
        // parts of v below 1, so that |G v| < 2^15 with G's rows scaled below 2^14 per part
        RB_TRY(launch_range_scale(ctx, (const float2 *)w, (size_t)K, delta, 0, pl.vscale));
    } else {
        hipLaunchKernelGGL(square_scale_kernel, dim3(1), dim3(1), 0, ctx->stream, gscale,
                           pl.vscale);
        RB_CHECK_LAUNCH(ctx);
    }
    if (gr->prec == RB_BF16)
        hipLaunchKernelGGL(forward_lp_kernel<__bf16>, dim3(f.nblk), dim3(256), 0, ctx->stream,
                           (const __bf16 *)gr->G, (const float2 *)w, delta, n, K, ld, f.nT,
                           f.kchunk * LF_BK, f.splitk, pl.vscale, pl.dpart);
    else
        hipLaunchKernelGGL(forward_lp_kernel<_Float16>, dim3(f.nblk), dim3(256), 0, ctx->stream,
                           (const _Float16 *)gr->G, (const float2 *)w, delta, n, K, ld, f.nT,
                           f.kchunk * LF_BK, f.splitk, pl.vscale, pl.dpart);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return rb_forward_lp_reduce(ctx, &pl, d);
}
