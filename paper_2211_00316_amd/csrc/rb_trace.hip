// Ray tracing and ray-to-grid binning on gfx950.
//
// Section 4 of the paper: Hamiltonian ray equations (Eq. ray-equation-reference) and the
// paraxial system (Eq. ray-equation-paraxial) integrated together by Heun's method with the
// wave-vector normalisations of Algorithm 1; initial conditions of Section 4.4; ray
// sampling of Definition 1 (last step lands on the ring); travel time by the trapezoid rule
// (Eq. phase-discretised / omega), caustic count from sign changes of the Jacobian, and the
// geometric amplitude of Eq. amplitude-geom-discretised referenced to the first sample by
// Eq. attenuation_geom_reference. Section 4.5: the map is the uniform cubic B-spline of the
// grid samples; ray-to-grid by linear interpolation over the triangulated ray samples.
// Absorbing media (Section 2.2, Szabo's model; Eq. amplitude-abs-discretised): the rays of one
// frequency follow its dispersive map, and the line integral of the absorption map
// alpha = alpha0 omega^y (Np/m, the same cubic B-spline, value only) is taken by the
// trapezoid rule beside the travel time and subtracted from the log-amplitude, so that the
// interpolated amplitude is A_geom A_abs and nothing downstream changes.
//
// GPU design: one lane per ray, the 64 lanes of a wavefront are 64 neighbouring rays of one
// transducer, so the per-step sample stores are coalesced ([emitter][step][ray] planes).
// Positions and the travel time are kept in FP64 (one FMA each per step); the rest of the
// ray and paraxial state is FP32. The spline at the new point is reused as the first
// evaluation of the next step.
//
// Binning. The samples of one transducer form a structured mesh (ray j, step i). Where the
// fan does not fold (no ray of that transducer meets a caustic), every mask node lies in
// exactly one triangle (up to shared edges), so each (transducer, node) lane walks the mesh
// from the straight-ray guess to its triangle and writes the tables directly: no atomics,
// coalesced stores. A transducer whose fan folds goes through the general path instead:
// one lane per quad keeps, per covered node, the smallest (travel-time, triangle-id) 64-bit
// key by atomicMin (order independent, hence deterministic), and a resolve pass
// re-interpolates the winning triangle.
#include "rb_internal.h"

#include <cmath>

namespace {

struct GridP {
    int nx, ny;
    double dx, x0, y0, idx;  // idx = 1 / dx
};

// The spline map is stored with MPAD replicated nodes on every side, so the four control
// points of a cell are always in the array. Clamping the cell index to [-2, n] then gives
// exactly the values of clamping each control point index to [0, n-1]: beyond that range all
// four control points are the edge value either way.
constexpr int MPAD = 3;

// The map holds n - 1, not n: the index stays within a few percent of 1, and weighted sums
// of control points near 1 would lose most of the FP32 digits of the Hessian (about 1e-4
// per node^2) to cancellation. Near a focus the amplitude is sensitive to exactly those
// digits.
// The cubic B-spline of the map n - 1 (Section 5: the map's samples as control points),
// stored per cell as the bicubic in the cell's local coordinates (tx, ty) in [0, 1):
// coef[cell][j] = (a_j0, a_j1, a_j2, a_j3) with value sum_{j,i} a_ji tx^i ty^j. Cells
// (iu, iv), iu in [-2, nx], iv in [-2, ny], have index (iv + 2) (nx + 3) + iu + 2.
constexpr int PATCH_STRIDE = 256;  // threads of a tracing workgroup

struct SplineMap {
    const float4 *coef;  // [(ny + 3) (nx + 3)][4]
    int nx, ny, ncx;     // ncx = nx + 3 cells per row
    float ih;            // 1 / dx
    float4 *patch;       // this lane's cell cache in LDS: 4 float4 at stride PATCH_STRIDE
};

struct Spline {
    float v, gx, gy, hxx, hxy, hyy;
};

// Four consecutive floats of a row, 4-byte aligned: one 16-byte load.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef int i2u __attribute__((ext_vector_type(2), aligned(4)));

// The cell a lane evaluated last; its 16 coefficients stay in the lane's LDS slot
// (m.patch). A step is shorter than a cell, so consecutive evaluations (predictor,
// corrector, next predictor) mostly fall in the same cell and read them from LDS instead of
// loading them again; kept in LDS rather than in registers, they cost no register copies.
struct Patch {
    int cell = -1;  // (iv + 2) (nx + 3) + iu + 2 of the stored cell, -1 for none
};

// Value, gradient and Hessian (per metre) of the spline at node-index coordinates (u, v).
__device__ __forceinline__ Spline spline_eval(const SplineMap &m, double u, double v,
                                              Patch &pc) {
    double fu = floor(u), fv = floor(v);
    const float tx = (float)(u - fu), ty = (float)(v - fv);
    int iu = min(max((int)fu, -2), m.nx), iv = min(max((int)fv, -2), m.ny);
    const int cell = (iv + 2) * m.ncx + (iu + 2);
    if (cell != pc.cell) {
        const float4 *p = m.coef + (size_t)cell * 4;
#pragma unroll
        for (int b = 0; b < 4; ++b) m.patch[b * PATCH_STRIDE] = p[b];
        pc.cell = cell;
    }
    float f[16];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float4 q = m.patch[b * PATCH_STRIDE];
        f[4 * b] = q.x;
        f[4 * b + 1] = q.y;
        f[4 * b + 2] = q.z;
        f[4 * b + 3] = q.w;
    }
    // Row polynomials Q_j(tx) = sum_i a_ji tx^i and their first two tx-derivatives (Horner),
    // then the same in ty: value, gradient and Hessian of the bicubic.
    float q0[4], q1[4], q2[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float a0 = f[4 * j], a1 = f[4 * j + 1], a2 = f[4 * j + 2];
        const float a3 = f[4 * j + 3];
        const float b3 = 3.0f * a3, b2 = a2 + a2;
        q0[j] = fmaf(fmaf(fmaf(a3, tx, a2), tx, a1), tx, a0);
        q1[j] = fmaf(fmaf(b3, tx, b2), tx, a1);
        q2[j] = fmaf(b3 + b3, tx, b2);
    }
    const float s_v = fmaf(fmaf(fmaf(q0[3], ty, q0[2]), ty, q0[1]), ty, q0[0]);
    const float s_gx = fmaf(fmaf(fmaf(q1[3], ty, q1[2]), ty, q1[1]), ty, q1[0]);
    const float s_xx = fmaf(fmaf(fmaf(q2[3], ty, q2[2]), ty, q2[1]), ty, q2[0]);
    const float c3 = 3.0f * q0[3], c2 = q0[2] + q0[2];
    const float s_gy = fmaf(fmaf(c3, ty, c2), ty, q0[1]);
    const float s_xy = fmaf(fmaf(3.0f * q1[3], ty, q1[2] + q1[2]), ty, q1[1]);
    const float s_yy = fmaf(c3 + c3, ty, c2);
    float ih = m.ih, ih2 = ih * ih;
    return Spline{s_v + 1.0f, s_gx * ih, s_gy * ih, s_xx * ih2, s_xy * ih2, s_yy * ih2};
}

// Absorption map alpha (Np/m) with MPAD replicated nodes on every side, as stored by pad_map
// with offset 0; p == nullptr for a lossless medium.
struct AbsMap {
    const float *p;
    int nx, ny, nxp;  // nxp = nx + 2 MPAD
};

// Value of the uniform cubic B-spline of the absorption map at node-index coordinates (u, v):
// the sixteen control points around the cell weighted by the basis functions (cell index
// clamped as in spline_eval, which with the padding equals clamping each control point).
__device__ __forceinline__ float abs_value(const AbsMap &a, double u, double v) {
    const double fu = floor(u), fv = floor(v);
    const float tx = (float)(u - fu), ty = (float)(v - fv);
    const int iu = min(max((int)fu, -2), a.nx), iv = min(max((int)fv, -2), a.ny);
    float wx[4], wy[4];
    {
        const float s = 1.0f - tx, t2 = tx * tx, t3 = t2 * tx;
        wx[0] = s * s * s * (1.0f / 6.0f);
        wx[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * (1.0f / 6.0f);
        wx[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * tx + 1.0f) * (1.0f / 6.0f);
        wx[3] = t3 * (1.0f / 6.0f);
    }
    {
        const float s = 1.0f - ty, t2 = ty * ty, t3 = t2 * ty;
        wy[0] = s * s * s * (1.0f / 6.0f);
        wy[1] = (3.0f * t3 - 6.0f * t2 + 4.0f) * (1.0f / 6.0f);
        wy[2] = (-3.0f * t3 + 3.0f * t2 + 3.0f * ty + 1.0f) * (1.0f / 6.0f);
        wy[3] = t3 * (1.0f / 6.0f);
    }
    float acc = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const f4u row = *reinterpret_cast<const f4u *>(
            a.p + (size_t)(iv - 1 + b + MPAD) * a.nxp + (iu - 1 + MPAD));
        acc = fmaf(wy[b], wx[0] * row.x + wx[1] * row.y + wx[2] * row.z + wx[3] * row.w, acc);
    }
    return acc;
}

// Ray state; the position is in node-index units (u, v) = ((x - x0) / dx, (y - y0) / dx).
// What a ray integrates over its whole length is FP64: position, wave vector and the
// paraxial dx (FP32 rounding of the direction, repeated every step, moves the far end of
// the ray by about 1e-3 node, enough to shift the interpolation in the thin triangles of a
// focus by percents). The right-hand sides are evaluated in FP32.
struct Ray {
    double u, v;
    double kx, ky, dxx, dxy;
    float dkx, dky;
};

// 1 / sqrt(a) from the FP32 estimate and one Newton step (relative error about the square
// of the FP32 one). The estimate is the hardware reciprocal square root alone: its arguments
// here are squared wave-vector norms near n^2, never denormal, so the library's rescaling
// for tiny arguments would only add instructions.
__device__ __forceinline__ double rsqrt_newton(double a) {
    const double y = (double)__builtin_amdgcn_rsqf((float)a);
    return y * fma(-0.5 * a * y, y, 1.5);
}

// Paraxial right-hand side (Eq. ray-equation-paraxial with k -> n).
__device__ __forceinline__ void paraxial_rhs(const Spline &s, float kx, float ky, float dxx,
                                             float dxy, float dkx, float dky, float q[4]) {
    float n = s.v, in = __builtin_amdgcn_rcpf(n), in2 = in * in;
    float gdx = s.gx * dxx + s.gy * dxy;
    float kdk = kx * dkx + ky * dky;
    q[0] = -gdx * in2 * kx + dkx * in;
    q[1] = -gdx * in2 * ky + dky * in;
    q[2] = s.hxx * dxx + s.hxy * dxy - gdx * in * s.gx + kdk * in2 * s.gx;
    q[3] = s.hxy * dxx + s.hyy * dxy - gdx * in * s.gy + kdk * in2 * s.gy;
}

// One step of Algorithm 1 of length h (metres), given the spline at the current point.
__device__ __forceinline__ Ray heun_step(const SplineMap &m, const Spline &s1, const Ray &r,
                                         double h, double idx, Patch &pc) {
    float hf = (float)h;
    double hu = h * idx;                                    // step in node units
    float n = s1.v;
    const double ikn = rsqrt_newton(r.kx * r.kx + r.ky * r.ky);
    const double kxd = (double)n * (r.kx * ikn), kyd = (double)n * (r.ky * ikn);
    float qxx = (float)(r.kx * ikn), qxy = (float)(r.ky * ikn);  // unit ray direction
    float kx = (float)kxd, ky = (float)kyd;                 // normalised wave vector
    float kpx = kx + hf * s1.gx, kpy = ky + hf * s1.gy;     // auxiliary ray direction
    Spline s2 = spline_eval(m, r.u + hu * (double)qxx, r.v + hu * (double)qxy, pc);
    float n2 = s2.v;
    float ikpn = __builtin_amdgcn_rsqf(kpx * kpx + kpy * kpy);
    float qxx2 = kpx * ikpn, qxy2 = kpy * ikpn;
    kpx = n2 * qxx2;
    kpy = n2 * qxy2;
    float sx = qxx + qxx2, sy = qxy + qxy2;
    float isn = __builtin_amdgcn_rsqf(sx * sx + sy * sy);
    Ray o;
    o.u = r.u + hu * (double)(sx * isn);                    // position along mean direction
    o.v = r.v + hu * (double)(sy * isn);
    o.kx = kxd + (double)(hf * (s1.gx + s2.gx) * 0.5f);
    o.ky = kyd + (double)(hf * (s1.gy + s2.gy) * 0.5f);
    float a[4], b[4];
    const float dxx = (float)r.dxx, dxy = (float)r.dxy;
    paraxial_rhs(s1, kx, ky, dxx, dxy, r.dkx, r.dky, a);
    float dkpx = r.dkx + hf * a[2], dkpy = r.dky + hf * a[3];
    float dxpx = dxx + hf * a[0], dxpy = dxy + hf * a[1];
    paraxial_rhs(s2, kpx, kpy, dxpx, dxpy, dkpx, dkpy, b);
    o.dxx = r.dxx + (double)(hf * (a[0] + b[0]) * 0.5f);
    o.dxy = r.dxy + (double)(hf * (a[1] + b[1]) * 0.5f);
    o.dkx = r.dkx + hf * (a[2] + b[2]) * 0.5f;
    o.dky = r.dky + hf * (a[3] + b[3]) * 0.5f;
    return o;
}

// Square root of a positive double from the FP32 estimate and one Newton step (relative
// error about the square of the FP32 one). The estimate is the hardware square root (about
// one ulp, not correctly rounded): the Newton step in FP64 removes its error either way.
__device__ __forceinline__ double sqrt_newton(double a) {
    float s0 = __builtin_amdgcn_sqrtf((float)a);
    double s = (double)s0;
    return fma(a - s * s, (double)(0.5f * __builtin_amdgcn_rcpf(s0)), s);
}

struct SampleBufs {
    float2 *pos;                       // [E][S][n_rays] position in node-index units
    float4 *fld;                       // [E][S][n_rays] (dT, L, t_x, t_y)
    uint8_t *K;                        // [E][S][n_rays] caustic count, stored where > 0 only
    int32_t *kfirst;                   // [E][n_rays] first sample with K > 0, S if none
    int32_t *M;                        // [E][n_rays] last sample index, -1 if invalid
    double *ex_beta;                   // [E][n_rays] exit angle from psi_e in [0, 2 pi)
    float *ex_dT, *ex_L;
    uint8_t *ex_K;
    int32_t *folded;                   // [E] nonzero if a ray of the transducer met a caustic
    const double2 *ring;               // [N] transducer positions
};

// Terminal state of a traced ray (linking): travel time, distance from the source, exit
// angle from psi_e in [0, 2 pi), log-amplitude L = ln A + ln(d) / 2 and caustic count.
struct RayEnd {
    double T, d, beta;
    float L;
    int K;
};

// One ray from the transducer at xy (angle psi on the ring) with launch direction (cg, sg):
// Algorithm 1 with the paraxial system, Definition 1's last step. STORE: the samples of fan
// ray j of chunk transducer el go to sb; otherwise only the terminal state goes to *end.
// Returns the index of the last sample, -1 if the ray did not reach the ring within
// max_steps.
template <bool STORE, bool ABS>
__device__ __forceinline__ int trace_core(const SplineMap &m, const AbsMap &am, const GridP &g,
                                          double R, double psi, double2 xy, double cg,
                                          double sg, int n_rays, int max_steps, double ds,
                                          double c0, int el, int j, const SampleBufs &sb,
                                          int *flag, RayEnd *end) {
    const int S = max_steps + 1;
    const double ue = (xy.x - g.x0) * g.idx, ve = (xy.y - g.y0) * g.idx;
    const double uc = -g.x0 * g.idx, vc = -g.y0 * g.idx;  // ring centre
    const double Ru2 = R * R * g.idx * g.idx;              // ring radius squared, node units
    Patch pc;
    Ray r;
    r.u = ue;
    r.v = ve;
    Spline sc = spline_eval(m, r.u, r.v, pc);
    float n_cur = sc.v;
    r.kx = (double)n_cur * cg;
    r.ky = (double)n_cur * sg;
    r.dxx = 0.0;
    r.dxy = 0.0;
    r.dkx = (float)(-(double)n_cur * sg);
    r.dky = (float)((double)n_cur * cg);
    double T = 0.0;
    double Babs = 0.0;  // int alpha ds from the source (absorbing media)
    float a_cur = 0.0f;
    if constexpr (ABS) a_cur = abs_value(am, r.u, r.v);

    size_t o = (size_t)el * S * n_rays + j;
    if constexpr (STORE) {
        sb.pos[o] = make_float2((float)r.u, (float)r.v);
        sb.fld[o] = make_float4(0.0f, 0.0f, (float)cg, (float)sg);
    }
    int kfirst = S;  // K is monotone along a ray: zero before kfirst, stored from it on

    float J_prev = 0.0f;
    float lnc1 = 0.0f;  // (1/2) ln(n_1 J_1 / (8 pi s_1)) of the first sample
    int K = 0;
    int M = -1;
    const double ic0 = 1.0 / c0;
    double h = ds;
    bool last = false;
    int i = 0;
    while (i < max_steps) {
        Ray nr = heun_step(m, sc, r, h, g.idx, pc);
        if (!last) {
            double pu = nr.u - uc, pv = nr.v - vc;
            if (pu * pu + pv * pv >= Ru2) {
                // Definition 1: redo the step with ds' = distance along the unit direction
                // to the ring.
                double kn = sqrt(r.kx * r.kx + r.ky * r.ky);
                double tx = r.kx / kn, ty = r.ky / kn;
                double qu = r.u - uc, qv = r.v - vc;
                double b = (qu * tx + qv * ty) * g.dx;
                double disc = b * b + R * R - (qu * qu + qv * qv) * g.dx * g.dx;
                h = fmin(fmax(-b + sqrt(fmax(disc, 0.0)), 0.0), ds);
                last = true;
                continue;
            }
        }
        r = nr;
        sc = spline_eval(m, r.u, r.v, pc);
        float n_new = sc.v;
        T += h * 0.5 * ic0 * ((double)n_cur + (double)n_new);
        if constexpr (ABS) {
            const float a_new = abs_value(am, r.u, r.v);
            Babs += h * 0.5 * ((double)a_cur + (double)a_new);
            a_cur = a_new;
        }
        const float kxf = (float)r.kx, kyf = (float)r.ky;
        float ikn = __builtin_amdgcn_rsqf(kxf * kxf + kyf * kyf);
        float tx = kxf * ikn, ty = kyf * ikn;
        float J = (float)r.dxx * (-ty) + (float)r.dxy * tx;
        if (i >= 1 && J * J_prev < 0.0f) ++K;
        double du = r.u - ue, dv = r.v - ve;
        double d = sqrt_newton(du * du + dv * dv) * g.dx;   // distance from the source
        float df = (float)d;
        float nJ = n_new * fabsf(J);
        // Eq. attenuation_geom_reference with the first sample as reference, as a logarithm:
        // L = ln A + ln(d)/2 = lnc1 + ln(d / (n |J|)) / 2 with
        // lnc1 = ln(n_1 |J_1| / (8 pi d_1)) / 2 = -ln(d_1 / (n_1 |J_1|)) / 2 - ln(8 pi) / 2,
        // so one logarithm per sample (hardware log2; its argument is of order d / |J|, far
        // from the denormal range).
        const float lh = (0.5f * 0.693147181f) *
                         __builtin_amdgcn_logf(df * __builtin_amdgcn_rcpf(nJ));
        if (i == 0) lnc1 = -lh - 0.5f * 3.22417143f;  // ln(8 pi) = 3.2241714...
        float L = lnc1 + lh;
        if constexpr (ABS) L -= (float)Babs;  // ln A_abs (Eq. amplitude-abs-discretised)
        float dT = (float)(T - d * ic0);
        ++i;
        o += n_rays;
        if constexpr (STORE) {
            sb.pos[o] = make_float2((float)r.u, (float)r.v);
            sb.fld[o] = make_float4(dT, L, tx, ty);
            if (K > 0) {
                sb.K[o] = (uint8_t)min(K, 255);
                if (kfirst == S) kfirst = i;
            }
        }
        J_prev = J;
        n_cur = n_new;
        if (last) {
            M = i;
            if constexpr (STORE) {
                size_t x = (size_t)el * n_rays + j;
                sb.ex_dT[x] = dT;
                sb.ex_L[x] = L;
                sb.ex_K[x] = (uint8_t)min(K, 255);
            } else {
                end->T = T;
                end->d = d;
                end->L = L;
                end->K = K;
            }
            break;
        }
    }
    if (M >= 0) {
        double beta = atan2(r.v - vc, r.u - uc) - psi;
        beta -= RB_TWO_PI * floor(beta * (1.0 / RB_TWO_PI));
        if constexpr (STORE) sb.ex_beta[(size_t)el * n_rays + j] = beta;
        else end->beta = beta;
    }
    if constexpr (STORE) {
        sb.M[(size_t)el * n_rays + j] = M;
        sb.kfirst[(size_t)el * n_rays + j] = kfirst;
        if (M < 0) atomicOr(flag, 1);
        if (K > 0) atomicOr(sb.folded + el, 1);
    }
    return M;
}

// Fan ray j of transducer e0 + el (Section 4.4: launch angle gamma = psi + pi + delta,
// |delta| < pi / 2), samples to sb.
template <bool ABS>
__device__ __forceinline__ int trace_ray(const SplineMap &m, const AbsMap &am, const GridP &g,
                                         double R,
                                         double psi0, int N, int n_rays, int max_steps,
                                         double ds, double c0, int e0, int el, int j,
                                         const SampleBufs &sb, int *flag) {
    const int e = e0 + el;
    const double psi = psi0 + RB_TWO_PI * (double)e / (double)N;
    const double2 xy = sb.ring[e];
    double sd, cd;
    sincospi(((double)j + 0.5 - 0.5 * (double)n_rays) / (double)n_rays, &sd, &cd);
    const double cp = xy.x / R, sp = xy.y / R;
    const double cg = -(cp * cd - sp * sd), sg = -(sp * cd + cp * sd);
    return trace_core<true, ABS>(m, am, g, R, psi, xy, cg, sg, n_rays, max_steps, ds, c0, el,
                                 j, sb, flag, nullptr);
}

// One lane per ray; a wavefront holds 64 neighbouring rays of one transducer, so the
// per-step sample stores are coalesced. Rays near the middle of a fan cross the whole disk
// and take the most steps, so wavefronts are dispatched by the distance of their ray group
// from the fan's middle (rank r: groups mid, mid - 1, mid + 1, ...), over all transducers:
// the longest run first and the shortest fill the end of the launch. Also counts the
// samples written (one atomic per wavefront; the workgroup is a whole number of them).
// Four waves per SIMD (128 registers, a few spilled) hide more of the coefficient loads'
// latency than three without spills.
// Workgroups (four transducers of one rank) are dealt to the 8 XCDs round-robin by launch
// index. When E is a multiple of 32 the transducer groups of a rank are renamed so that each
// XCD traces one contiguous arc of E / 8 transducers: same-rank rays of neighbouring
// transducers cross nearly the same cells at about the same time, so that XCD's L2 fetches
// their spline coefficients once instead of once per group of four. (Which wave traces which
// ray changes nothing in the results.)
template <bool ABS>
__global__ void __launch_bounds__(PATCH_STRIDE) __attribute__((amdgpu_waves_per_eu(4))) trace_kernel(SplineMap m, AbsMap am, GridP g,
                                                             double R, double psi0, int N,
                                                             int n_rays, int max_steps,
                                                             double ds, double c0, int e0, int E,
                                                             SampleBufs sb, int *flag,
                                                             unsigned long long *n_samples) {
    __shared__ float4 s_patch[4 * PATCH_STRIDE];
    m.patch = s_patch + threadIdx.x;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int n_groups = (n_rays + 63) / 64;
    const int rank = wave / E;
    int el = wave % E;
    if ((E & 31) == 0) {  // group g of four -> (g mod 8) (E / 32) + g / 8
        const int g = el >> 2;
        el = (((g & 7) * (E >> 5) + (g >> 3)) << 2) | (el & 3);
    }
    int M = -1;
    if (rank < n_groups) {
        const int mid = n_groups / 2;
        const int grp = (rank & 1) ? mid - 1 - (rank >> 1) : mid + (rank >> 1);
        const int j = grp * 64 + (threadIdx.x & 63);
        if (j < n_rays)
            M = trace_ray<ABS>(m, am, g, R, psi0, N, n_rays, max_steps, ds, c0, e0, el, j, sb,
                               flag);
    }
    int cnt = M >= 0 ? M + 1 : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt > 0) atomicAdd(n_samples, (unsigned long long)cnt);
}

// Map minus `off` (the index map stores n - 1, exact in FP32 for n in [1/2, 2]; the absorption
// map off = 0) with MPAD replicated nodes on every side.
__global__ void pad_map(const float *__restrict__ ns, int nx, int ny, float off,
                        float *__restrict__ out) {
    const int nxp = nx + 2 * MPAD;
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= nxp) return;
    int si = min(max(i - MPAD, 0), nx - 1), sj = min(max(j - MPAD, 0), ny - 1);
    out[(size_t)j * nxp + i] = ns[(size_t)sj * nx + si] - off;
}

// Monomial coefficients of the uniform cubic B-spline on cell (iu, iv) = (ci - 2, cj - 2),
// whose control points are the padded samples iu - 1 .. iu + 2, iv - 1 .. iv + 2. The
// weights of control point k at offset t are sum_p B[k][p] t^p with 6 B = [[1, -3, 3, -1],
// [4, 0, -6, 3], [1, 3, 3, -3], [0, 0, 0, 1]]; a = B^T C B (rows: powers of ty, columns:
// powers of tx), formed in FP64 from the FP32 samples and rounded once.
__global__ void spline_coef(const float *__restrict__ padded, int nx, int ny,
                            float4 *__restrict__ coef) {
    const int nxp = nx + 2 * MPAD, ncx = nx + 3;
    const int ci = blockIdx.x * blockDim.x + threadIdx.x, cj = blockIdx.y;
    if (ci >= ncx) return;
    const int iu = ci - 2, iv = cj - 2;
    constexpr double B[4][4] = {{1.0, -3.0, 3.0, -1.0},
                                {4.0, 0.0, -6.0, 3.0},
                                {1.0, 3.0, 3.0, -3.0},
                                {0.0, 0.0, 0.0, 1.0}};
    double D[4][4];  // D[b][p] = sum_k C[b][k] B[k][p] / 6 (row b of control points)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float *row = padded + (size_t)(iv - 1 + b + MPAD) * nxp + (iu - 1 + MPAD);
        const double c0 = row[0], c1 = row[1], c2 = row[2], c3 = row[3];
#pragma unroll
        for (int p = 0; p < 4; ++p)
            D[b][p] = (c0 * B[0][p] + c1 * B[1][p] + c2 * B[2][p] + c3 * B[3][p]) * (1.0 / 6.0);
    }
    float4 *out = coef + ((size_t)cj * ncx + ci) * 4;
#pragma unroll
    for (int q = 0; q < 4; ++q) {  // power of ty
        double a[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
            a[p] = (B[0][q] * D[0][p] + B[1][q] * D[1][p] + B[2][q] * D[2][p] +
                    B[3][q] * D[3][p]) * (1.0 / 6.0);
        out[q] = make_float4((float)a[0], (float)a[1], (float)a[2], (float)a[3]);
    }
}

__device__ __forceinline__ unsigned long long ordered_bits64(double f) {
    unsigned long long u = (unsigned long long)__double_as_longlong(f);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

__device__ __forceinline__ uint32_t ordered_bits(float f) {
    uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Barycentric coordinates of node (pu, pv) in triangle (a, b, c), node-index units.
__device__ __forceinline__ bool barycentric(float au, float av, float bu, float bv, float cu,
                                            float cv, float pu, float pv, float &la, float &lb,
                                            float &lc) {
    float area = (bu - au) * (cv - av) - (bv - av) * (cu - au);
    if (!(fabsf(area) > 1e-30f)) return false;
    float ia = __builtin_amdgcn_rcpf(area);
    la = ((bu - pu) * (cv - pv) - (bv - pv) * (cu - pu)) * ia;
    lb = ((cu - pu) * (av - pv) - (cv - pv) * (au - pu)) * ia;
    lc = ((au - pu) * (bv - pv) - (av - pv) * (bu - pu)) * ia;
    return true;
}

// Coverage tolerance of the barycentric test in FP32: nodes on a shared edge are claimed by
// both triangles (the smallest-key rule picks one), so no node falls between triangles.
#define RB_BARY_EPS 1e-5f

// Where binning writes: the tables of the C ABI, or (rec != nullptr, inside a frequency step)
// one compact record per (transducer, node), see rb_launch_trace. With compact records the
// binning also keeps, per transducer, the largest A and 1/A it wrote (the per-row operand
// scales of the 16-bit form come from them): per walk workgroup in tmax[2 (el ntiles + t)],
// and, for nodes the folded-fan resolve writes, directly in rowmax[2 e] (bits of positive
// floats, which order as unsigned integers).
struct TableOut {
    rb_tables tb;
    float4 *rec;
    float *tmax;
    unsigned int *rowmax;
};

// Travel-time residual of a triangle at barycentric (la, lb, lc): one fixed order of
// operations, so that binning by walk and by rasterisation build identical keys.
__device__ __forceinline__ float tri_dT(float la, float lb, float lc, float d0, float d1,
                                        float d2) {
    return fmaf(lc, d2, fmaf(lb, d1, la * d0));
}

// Key of a candidate triangle at a node: smallest travel time first, then lowest triangle id.
__device__ __forceinline__ unsigned long long tri_key(float dT, uint32_t id) {
    return ((unsigned long long)ordered_bits(dT) << 32) | id;
}

// Nodes in 8 x 8 tiles, one mark byte per (transducer, tile): set where more than one
// triangle may cover a node. In a fan whose triangles all keep one orientation (negative
// area in node coordinates, rays in launch order) no point is covered twice; in general the
// positive minus the negative covers of a point is the winding number of the fan's boundary
// about it (0 or 1), so a point covered twice is covered by an inverted triangle. Inverted
// and near-degenerate triangles mark the tiles their bounding box touches, and a node whose
// walk failed marks its own tile; the rasterisation skips triangles that touch no marked tile.
constexpr int MT_SHIFT = 3;
constexpr float AREA_MARK = -1e-3f;  // node^2: above this a triangle counts as inverted

__device__ __forceinline__ void bbox_tiles(const float *tu, const float *tv, int nx, int ny,
                                           int &ti0, int &ti1, int &tj0, int &tj1) {
    float umin = fminf(fminf(tu[0], tu[1]), tu[2]), umax = fmaxf(fmaxf(tu[0], tu[1]), tu[2]);
    float vmin = fminf(fminf(tv[0], tv[1]), tv[2]), vmax = fmaxf(fmaxf(tv[0], tv[1]), tv[2]);
    int i0 = max((int)ceilf(umin - 1e-4f), 0), i1 = min((int)floorf(umax + 1e-4f), nx - 1);
    int j0 = max((int)ceilf(vmin - 1e-4f), 0), j1 = min((int)floorf(vmax + 1e-4f), ny - 1);
    ti0 = i0 >> MT_SHIFT;
    ti1 = i1 >> MT_SHIFT;
    tj0 = j0 >> MT_SHIFT;
    tj1 = j1 >> MT_SHIFT;
}

// Interpolate the fields of triangle vb[] at barycentric lam[] and write table entry `out`;
// K: the largest caustic count of the three vertices. Returns the interpolated dT.
// Polar angle of (x, y) in [-pi, pi] within 3e-7 rad (atan2f: 2 ulp): octant reduction
// and an odd polynomial of degree 15 for atan on [0, 1], the least-squares fit on 2000
// Chebyshev nodes (4.1e-8 rad in exact arithmetic; fit_atan.py rebuilds it).
__device__ __forceinline__ float ray_atan2(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(fmaxf(ax, ay), 1e-30f));
    const float t2 = t * t;
    float p = -0.0040733092f;
    p = fmaf(p, t2, 0.021946611f);
    p = fmaf(p, t2, -0.056063175f);
    p = fmaf(p, t2, 0.096562564f);
    p = fmaf(p, t2, -0.13915803f);
    p = fmaf(p, t2, 0.19948509f);
    p = fmaf(p, t2, -0.33330107f);
    p = fmaf(p, t2, 0.99999946f);
    float a = t * p;
    if (ay > ax) a = 1.57079633f - a;
    if (x < 0.f) a = 3.14159265f - a;
    return y < 0.f ? -a : a;
}

// Table rows of transducer e (uniform over a workgroup): entry q of the row is out + q.
__device__ __forceinline__ TableOut table_row(const TableOut &to, size_t off) {
    TableOut r = to;
    if (to.rec) {
        r.rec = to.rec + off;
    } else {
        r.tb.T = to.tb.T + off;
        r.tb.A = to.tb.A + off;
        r.tb.ux = to.tb.ux + off;
        r.tb.uy = to.tb.uy + off;
        r.tb.flags = to.tb.flags + off;
    }
    return r;
}

// REC: compact records (to.rec); otherwise the tables of the C ABI, whose T needs the FP64
// distance d (df: the same distance in FP32, for the amplitude; a positive normal number).
// `to` holds the rows of the entry's transducer (table_row), out is the node's mask index.
template <bool REC>
__device__ __forceinline__ float write_entry_f(const float4 f0, const float4 f1, const float4 f2,
                                               const float lam[3], int K, float df, double d,
                                               double c0, const TableOut &to, uint32_t out,
                                               float &A) {
    const float dT = tri_dT(lam[0], lam[1], lam[2], f0.x, f1.x, f2.x);
    const float L = tri_dT(lam[0], lam[1], lam[2], f0.y, f1.y, f2.y);
    const float tx = tri_dT(lam[0], lam[1], lam[2], f0.z, f1.z, f2.z);
    const float ty = tri_dT(lam[0], lam[1], lam[2], f0.w, f1.w, f2.w);
    // exp(L) = 2^(L log2 e); L is far from the range where exp2 loses precision
    A = __builtin_amdgcn_exp2f(L * 1.44269504f) * __builtin_amdgcn_rsqf(df);
    if constexpr (REC) {
        to.rec[out] = make_float4(dT, A, ray_atan2(ty, tx), __int_as_float(0x80 | (K & 3)));
        return dT;
    }
    const rb_tables &tb = to.tb;
    float itn = rsqrtf(tx * tx + ty * ty);
    tb.T[out] = (double)dT + d / c0;
    tb.A[out] = A;
    tb.ux[out] = tx * itn;
    tb.uy[out] = ty * itn;
    tb.flags[out] = (uint8_t)(0x80 | (K & 3));
    return dT;
}

template <bool REC>
__device__ __forceinline__ void write_invalid(const TableOut &to, uint32_t out) {
    if constexpr (REC) {
        to.rec[out] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        return;
    }
    const rb_tables &tb = to.tb;
    tb.T[out] = 0.0;
    tb.A[out] = 0.0f;
    tb.ux[out] = 0.0f;
    tb.uy[out] = 0.0f;
    tb.flags[out] = 0;
}

// Walk over the ray mesh of one transducer, from quad (j, i), to the triangle that
// contains the point (pu, pv) (node-index units). Returns false if the walk leaves the
// mesh or does not settle within LOCATE_MAX_IT quads.
constexpr int LOCATE_MAX_IT = 96;
// In a fan that folds, inverted triangles mislead the walk's edge tests; a walk that does not
// settle soon is given up and its node left to the rasterisation.
constexpr int LOCATE_MAX_IT_FOLD = 16;
constexpr int LTX = RB_WALK_TX, LTY = RB_WALK_TY;  // node tile of one locate workgroup
constexpr int LOCATE_NPL = 2;  // nodes per lane (rows jj and jj + LTY / 2; folded: jj + 1)
constexpr int LOCATE_THREADS = LTX * LTY / LOCATE_NPL;
constexpr int LOCATE_WAVES = LOCATE_THREADS / 64;
constexpr int LOCATE_GROUP_ROWS = 2;  // tile rows per XCD group

// The two triangles of quad (j, i) with corners p00 (ray j, step i), p10 (ray j + 1, step i),
// p01 (ray j, step i + 1), p11: half 0 = (p00, p10, p11), half 1 = (p00, p11, p01). Returns
// the half that holds (pu, pv) with its barycentric coordinates, or -1.
__device__ __forceinline__ int quad_test(float2 p00, float2 p10, float2 p01, float2 p11,
                                         float pu, float pv, float lam[3]) {
    float la, lb, lc;
    if (barycentric(p00.x, p00.y, p10.x, p10.y, p11.x, p11.y, pu, pv, la, lb, lc) &&
        la >= -RB_BARY_EPS && lb >= -RB_BARY_EPS && lc >= -RB_BARY_EPS) {
        lam[0] = la;
        lam[1] = lb;
        lam[2] = lc;
        return 0;
    }
    if (barycentric(p00.x, p00.y, p11.x, p11.y, p01.x, p01.y, pu, pv, la, lb, lc) &&
        la >= -RB_BARY_EPS && lb >= -RB_BARY_EPS && lc >= -RB_BARY_EPS) {
        lam[0] = la;
        lam[1] = lb;
        lam[2] = lc;
        return 1;
    }
    return -1;
}

// posE, Mrow: the transducer's samples and last-sample indices (uniform over a workgroup in
// the walk); vb: the found triangle's vertices as sample offsets from posE.
__device__ __forceinline__ bool mesh_walk(const float2 *__restrict__ posE,
                                          const int32_t *__restrict__ Mrow, int n_rays, float pu,
                                          float pv, int &j, int &i, uint32_t vb[3], float lam[3],
                                          int &half, int max_it = LOCATE_MAX_IT) {
    for (int it = 0; it < max_it; ++it) {
        // rays j and j+1 are adjacent in memory: one load per pair (j <= n_rays - 2)
        const i2u Mv = *reinterpret_cast<const i2u *>(Mrow + j);
        const int Mj = Mv.x, Mj1 = Mv.y;
        int top = min(Mj, Mj1) - 1;  // last quad index along the rays
        if (Mj < 0 || Mj1 < 0 || top < 1) return false;
        if (i > top) i = top;
        const uint32_t b00 = (uint32_t)(i * n_rays + j), b01 = b00 + (uint32_t)n_rays;
        const f4u q0 = *reinterpret_cast<const f4u *>(posE + b00);
        const f4u q1 = *reinterpret_cast<const f4u *>(posE + b01);
        const float2 p00 = make_float2(q0.x, q0.y), p10 = make_float2(q0.z, q0.w);
        const float2 p01 = make_float2(q1.x, q1.y), p11 = make_float2(q1.z, q1.w);
        const int h = quad_test(p00, p10, p01, p11, pu, pv, lam);
        if (h >= 0) {
            vb[0] = b00;
            vb[1] = h == 0 ? b00 + 1 : b01 + 1;
            vb[2] = h == 0 ? b01 + 1 : b01;
            half = h;
            return true;
        }
        // step across the quad edge the point lies farthest outside of
        float area = (p10.x - p00.x) * (p01.y - p00.y) - (p10.y - p00.y) * (p01.x - p00.x);
        float sg = area >= 0.f ? 1.f : -1.f;
        auto side = [&](float2 a, float2 b) {
            float ex = b.x - a.x, ey = b.y - a.y;
            float cr = ex * (pv - a.y) - ey * (pu - a.x);
            return sg * cr * __builtin_amdgcn_rsqf(ex * ex + ey * ey + 1e-30f);
        };
        float s_i0 = side(p00, p10);   // edge at step i
        float s_j1 = side(p10, p11);   // edge along ray j+1
        float s_i1 = side(p11, p01);   // edge at step i+1
        float s_j0 = side(p01, p00);   // edge along ray j
        float worst = fminf(fminf(s_i0, s_j1), fminf(s_i1, s_j0));
        if (worst >= 0.f) return false;  // inside the quad but in neither triangle
        if (worst == s_i0) {
            if (i <= 1) return false;
            --i;
        } else if (worst == s_i1) {
            if (i >= top) return false;
            ++i;
        } else if (worst == s_j0) {
            if (j <= 0) return false;
            --j;
        } else {
            if (j >= n_rays - 2) return false;
            ++j;
        }
    }
    return false;
}

// Straight-ray guess of the quad holding the point at (ddx, ddy) from the source: launch
// angle and arc length of the straight ray.
// Polar angle of (x, y) in [-pi, pi] to 1e-4 rad: octant reduction and an odd polynomial of
// degree 7 for atan on [0, 1], the least-squares fit on 2000 Chebyshev nodes (fit_atan.py).
// Only the walk's starting quad depends on it (a tenth of a ray spacing at 1024 rays), not
// where a walk ends.
__device__ __forceinline__ float guess_atan2(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float t = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(fmaxf(ax, ay), 1e-30f));
    const float t2 = t * t;
    float a = t * fmaf(fmaf(fmaf(-0.039134149f, t2, 0.14661528f), t2, -0.32143047f), t2,
                       0.9992677f);
    if (ay > ax) a = 1.57079633f - a;
    if (x < 0.f) a = 3.14159265f - a;
    return y < 0.f ? -a : a;
}

// Fan ray and step of the straight ray from the transducer (angle psi on the ring, psi_pi =
// psi + pi in FP32) to the node at offset (ddx, ddy), distance d; ids = 1 / ds. A guess only.
__device__ __forceinline__ void straight_guess(float ddx, float ddy, float d, float psi_pi,
                                               float ids, int n_rays, int S, int &j, int &i) {
    float rel = guess_atan2(ddy, ddx) - psi_pi;
    rel -= (float)RB_TWO_PI * floorf((rel + (float)RB_PI) * (float)(1.0 / RB_TWO_PI));
    j = (int)floorf((rel + 0.5f * (float)RB_PI) * (float)n_rays * (float)(1.0 / RB_PI) - 0.5f);
    j = min(max(j, 0), n_rays - 2);
    i = min(max((int)(d * ids), 1), S - 2);
}

// Pre-pass: one lane per (transducer, node tile) walks the tile centre from its straight-ray
// guess and stores the offset of the quad it reached (the local bending of the rays).
__global__ void __launch_bounds__(256) tile_offset_kernel(SampleBufs sb, int n_rays, int S, int E,
                                                          int e0, GridP g, double psi0, int N,
                                                          double ds, int tile_i0, int tile_j0,
                                                          int tiles_x, int tiles_y,
                                                          float dpsi, double ids,
                                                          int2 *__restrict__ off) {
    const int ntiles = tiles_x * tiles_y;
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= E * ntiles) return;
    const int el = tid / ntiles, t = tid - el * ntiles;
    int2 o = make_int2(0, 0);
    {
        const int ti = t % tiles_x, tj = t / tiles_x;
        const int e = e0 + el;
        const float psi_pi = (float)(psi0 + RB_PI) + (float)e * dpsi;
        const double2 xy = sb.ring[e];
        double cu = tile_i0 + ti * LTX + 0.5 * (LTX - 1);
        double cv = tile_j0 + tj * LTY + 0.5 * (LTY - 1);
        double ddx = g.x0 + cu * g.dx - xy.x, ddy = g.y0 + cv * g.dx - xy.y;
        double d = sqrt(ddx * ddx + ddy * ddy);
        int j, i, jw, iw;
        straight_guess((float)ddx, (float)ddy, (float)d, psi_pi, (float)ids, n_rays, S, jw, iw);
        j = jw;
        i = iw;
        uint32_t vb[3];
        float lam[3];
        int half;
        if (d >= 2.0 * ds && mesh_walk(sb.pos + (size_t)el * S * n_rays, sb.M + (size_t)el * n_rays,
                                       n_rays, (float)cu, (float)cv, j, i, vb, lam, half))
            o = make_int2(j - jw, i - iw);
    }
    off[tid] = o;
}

// Caustic count of a triangle (vertices (ray, sample): (j, i), (j + 1, i), (j + 1, i + 1) for
// half 0; (j, i), (j + 1, i + 1), (j, i + 1) for half 1): the largest of its vertices', K being
// stored from the first sample of a ray where it is positive.
__device__ __forceinline__ int tri_K(const SampleBufs &sb, int n_rays, int S, int el, int j,
                                     int i, int half, const uint32_t vb[3]) {
    const uint8_t *KE = sb.K + (size_t)el * S * n_rays;
    const int kf0 = sb.kfirst[(size_t)el * n_rays + j], kf1 = sb.kfirst[(size_t)el * n_rays + j + 1];
    const int vi[3] = {i, half ? i + 1 : i, i + 1};
    const int kf[3] = {kf0, kf1, half ? kf0 : kf1};
    int K = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (vi[k] >= kf[k]) K = max(K, (int)KE[vb[k]]);
    return K;
}

// One (transducer, grid node) of the walk: for a mask node (q >= 0) writes its table entry
// (and, in a folded fan, its seed key); returns the amplitude written (0 for an invalid entry,
// a node outside the mask or a node left to the rasterisation).
template <bool REC, bool fold>
__device__ __forceinline__ float locate_node(const SampleBufs &sb, int n_rays, int S, int el,
                                             int e0, const GridP &g, float two_ds, double c0,
                                             int n_mask, int ii, int jj, int q, int2 o,
                                             const float4 wc, const TableOut &toE,
                                             unsigned long long *__restrict__ keys,
                                             uint8_t *__restrict__ changed,
                                             uint8_t *__restrict__ marks, int mtx, int mtiles,
                                             int *lost, float ids, int &js, int &is) {
    const int e = e0 + el;
    // Distance from the transducer. Records: FP32 (it decides validity, the walk's start and
    // A = exp(L) / sqrt(d); the reader rebuilds T from its own FP64 distance). ABI tables:
    // FP64, for T = dT + d / c0.
    float ddx, ddy, df;
    double d = 0.0;
    if constexpr (REC) {
        ddx = fmaf((float)ii, (float)g.dx, wc.x);
        ddy = fmaf((float)jj, (float)g.dx, wc.y);
        df = __builtin_amdgcn_sqrtf(fmaf(ddx, ddx, ddy * ddy));
    } else {
        const double2 xy = sb.ring[e];
        const double px = g.x0 + ii * g.dx, py = g.y0 + jj * g.dx;
        const double dx64 = px - xy.x, dy64 = py - xy.y;
        d = sqrt_newton(dx64 * dx64 + dy64 * dy64);
        ddx = (float)dx64;
        ddy = (float)dy64;
        df = (float)d;
    }
    // start: in a folded fan the quad where the lane's previous walk (the node one row below)
    // ended, else the straight-ray guess plus the tile's offset. (In an unfolded fan the two
    // walks of a lane stay independent, so that their loads overlap: chaining them there
    // made the walk slower.)
    int j = fold ? js : -1, i = is;
    if (j < 0) {
        straight_guess(ddx, ddy, df, wc.z, ids, n_rays, S, j, i);
        j = min(max(j + o.x, 0), n_rays - 2);
        i = min(max(i + o.y, 1), S - 2);
    }
    js = -1;
    if (q < 0) return 0.f;  // outside the mask
    const uint32_t out = (uint32_t)q;
    const size_t kq = (size_t)el * n_mask + q;
    const size_t mq = (size_t)el * mtiles + (jj >> MT_SHIFT) * mtx + (ii >> MT_SHIFT);
    if (df < two_ds || (fold && marks[mq])) {
        write_invalid<REC>(toE, out);
        if (fold) {
            keys[kq] = ~0ull;
            changed[kq] = 0;
        }
        return 0.f;
    }
    const size_t ebase = (size_t)el * S * n_rays;  // the transducer's samples
    uint32_t vb[3];
    float lam[3];
    int half;
    if (mesh_walk(sb.pos + ebase, sb.M + (size_t)el * n_rays, n_rays, (float)ii, (float)jj, j, i,
                  vb, lam, half, fold ? LOCATE_MAX_IT_FOLD : LOCATE_MAX_IT)) {
        js = j;
        is = i;
        // no ray of an unfolded fan has K > 0
        const int K = fold ? tri_K(sb, n_rays, S, el, j, i, half, vb) : 0;
        const float4 *fldE = sb.fld + ebase;
        float A;
        const float dT = write_entry_f<REC>(fldE[vb[0]], fldE[vb[1]], fldE[vb[2]], lam, K, df, d,
                                            c0, toE, out, A);
        if (fold) {
            keys[kq] = tri_key(dT, (uint32_t)(((size_t)j * S + i) * 2 + half));
            changed[kq] = 0;
        }
        return A;
    }
    write_invalid<REC>(toE, out);
    if (fold) {  // left to the rasterisation
        keys[kq] = ~0ull;
        changed[kq] = 0;
        marks[mq] = 1;
    } else {
        atomicAdd(lost, 1);
    }
    return 0.f;
}

// Largest value over the 64 lanes of a wave (non-negative inputs), returned in every lane:
// row reductions by DPP lane swaps, then the row results broadcast across rows (GFX9 DPP).
// Non-negative floats order as their bit patterns, so the maxima are unsigned-integer ones:
// one v_max_u32 with a DPP operand per stage (a float max would also quiet NaNs first).
__device__ __forceinline__ float wave_max(float x) {
    uint32_t v = __float_as_uint(x);
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)v, 63));
}

// One lane per (transducer, mask node); a workgroup covers a 16 x 16 tile of grid nodes of
// one transducer and starts every walk from the straight-ray guess plus the tile's offset.
// In a fan that folds, the walk's triangle is one candidate of the smallest-key rule: its
// record is written and its key seeds keys[] (changed[] cleared); the rasterisation of the
// fan then replaces it where a triangle with a smaller key covers the node.
// Workgroups are dealt to the 8 XCDs round-robin by launch index. The (transducer, tile)
// sequence is cut into groups of LOCATE_GROUP_ROWS tile rows and group g goes to XCD g mod 8,
// so neighbouring tiles share their ray samples through one L2 while every XCD still gets an
// even mix of the disk-shaped mask. The launch is padded to a multiple of 8 groups.
template <bool REC>
__global__ void __launch_bounds__(LOCATE_THREADS, 8) locate_kernel(SampleBufs sb, int n_rays, int S, int E,
                                                     int e0, GridP g, double R, double psi0,
                                                     int N, double ds, double c0, int n_mask,
                                                     int tile_i0, int tile_j0, int tiles_x,
                                                     int tiles_y, const int32_t *__restrict__ qmap,
                                                     const int2 *__restrict__ off, TableOut to,
                                                     unsigned long long *__restrict__ keys,
                                                     uint8_t *__restrict__ changed,
                                                     uint8_t *__restrict__ marks, int mtx,
                                                     int mtiles, int *lost, float idsf,
                                                     float two_ds, float cxn, float cyn,
                                                     float r2n, const float4 *__restrict__ wcon) {
    const int ntiles = tiles_x * tiles_y;
    const int G = LOCATE_GROUP_ROWS * tiles_x;
    const int L = blockIdx.x, xcd = L & 7, k = L >> 3;
    const int item = ((k / G) * 8 + xcd) * G + k % G;
    if (item >= E * ntiles) return;  // the whole workgroup
    const int el = item / ntiles, t = item - el * ntiles;
    const bool fold = sb.folded[el] != 0;  // uniform over the block
    const int ti = t % tiles_x, tj = t / tiles_x;
    const int ii = tile_i0 + ti * LTX + (threadIdx.x % LTX);
    const TableOut toE = table_row(to, (size_t)(e0 + el) * n_mask);
    const int2 o = off[item];
    const float4 wc = wcon[e0 + el];
    // largest A and 1/A of the lane's records (bits of non-negative floats)
    uint32_t amax = 0u, iamax = 0u;
    int js = -1, is = 0;  // quad of the lane's last successful walk (folded fans)
#pragma unroll
    for (int h = 0; h < LOCATE_NPL; ++h) {
        const int jj = tile_j0 + tj * LTY +
                       (fold ? LOCATE_NPL * (threadIdx.x / LTX) + h
                             : h * (LOCATE_THREADS / LTX) + (threadIdx.x / LTX));
        float A = 0.f;
        // nodes clearly outside the mask disc (node units; the margin leaves the decision on
        // the circle to qmap) issue nothing
        const float ru = (float)ii - cxn, rv = (float)jj - cyn;
        if (ii < g.nx && jj < g.ny && ru * ru + rv * rv <= r2n) {
            const int q = qmap[(size_t)jj * g.nx + ii];
            if (fold)
                A = locate_node<REC, true>(sb, n_rays, S, el, e0, g, two_ds, c0, n_mask, ii, jj,
                                           q, o, wc, toE, keys, changed, marks, mtx, mtiles,
                                           lost, idsf, js, is);
            else
                A = locate_node<REC, false>(sb, n_rays, S, el, e0, g, two_ds, c0, n_mask, ii, jj,
                                            q, o, wc, toE, keys, changed, marks, mtx, mtiles,
                                            lost, idsf, js, is);
        }
        amax = max(amax, __float_as_uint(A));
        iamax = max(iamax, __float_as_uint(A > 0.f ? __builtin_amdgcn_rcpf(A) : 0.f));
    }
    if (REC && to.tmax) {
        // each wave's largest A and 1/A (0 where no record was written); no barrier, so a
        // wave whose walks end early leaves at once
        const float m0 = wave_max(__uint_as_float(amax)), m1 = wave_max(__uint_as_float(iamax));
        if ((threadIdx.x & 63) == 0) {
            const size_t o = 2 * ((size_t)item * LOCATE_WAVES + (threadIdx.x >> 6));
            to.tmax[o] = m0;
            to.tmax[o + 1] = m1;
        }
    }
}


// Offer triangle tid to every mask node it covers. Keys only decrease, so a stale read of a
// node's key costs at most a needless atomic; a node whose key this triangle lowers is
// marked changed (its record is then rebuilt by the resolve pass).
// qrow: per grid row, the mask's run of nodes (first | last << 16) and the mask index of node
// i of the row minus i (the mask is a disc: one run per row).
__device__ __forceinline__ void raster_tri(const float *tu, const float *tv,
                                           const float4 *__restrict__ fld, const size_t *vb,
                                           int nx, int ny, const int2 *qrow,
                                           unsigned long long *__restrict__ keys,
                                           uint8_t *__restrict__ changed,
                                           const uint8_t *__restrict__ marks, int mtx,
                                           uint32_t tid) {
    {
        int ti0, ti1, tj0, tj1;
        bbox_tiles(tu, tv, nx, ny, ti0, ti1, tj0, tj1);
        bool any = false;
        for (int tj = tj0; tj <= tj1; ++tj)
            for (int ti = ti0; ti <= ti1; ++ti) any |= marks[tj * mtx + ti] != 0;
        if (!any) return;
    }
    const float tdT[3] = {fld[vb[0]].x, fld[vb[1]].x, fld[vb[2]].x};
    float umin = fminf(fminf(tu[0], tu[1]), tu[2]), umax = fmaxf(fmaxf(tu[0], tu[1]), tu[2]);
    float vmin = fminf(fminf(tv[0], tv[1]), tv[2]), vmax = fmaxf(fmaxf(tv[0], tv[1]), tv[2]);
    int i0 = max((int)ceilf(umin - 1e-4f), 0), i1 = min((int)floorf(umax + 1e-4f), nx - 1);
    int j0 = max((int)ceilf(vmin - 1e-4f), 0), j1 = min((int)floorf(vmax + 1e-4f), ny - 1);
    // Scanline bounds: on row jj only the nodes within m of the triangle's extent over the
    // strip |v - jj| <= m are tested (the edges clipped to the strip bound it). m covers the
    // coverage tolerance and the rounding of the barycentric test, so the nodes skipped are
    // nodes the test rejects; long thin triangles of a folding fan cost their rows and the
    // nodes they cover instead of their bounding box.
    const float m = 0.05f + 1e-4f * ((umax - umin) + (vmax - vmin));
    for (int jj = j0; jj <= j1; ++jj) {
        const float y = (float)jj;
        float lo = 3.0e38f, hi = -3.0e38f;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int k1 = k == 2 ? 0 : k + 1;
            const float ua = tu[k], va = tv[k], ub = tu[k1], vb_ = tv[k1];
            if (fmaxf(va, vb_) < y - m || fminf(va, vb_) > y + m) continue;
            float t0 = 0.f, t1 = 1.f;
            if (va != vb_) {
                const float ia = 1.0f / (vb_ - va);
                const float s0 = (y - m - va) * ia, s1 = (y + m - va) * ia;
                t0 = fmaxf(fminf(s0, s1), 0.f);
                t1 = fminf(fmaxf(s0, s1), 1.f);
            }
            const float x0 = fmaf(t0, ub - ua, ua), x1 = fmaf(t1, ub - ua, ua);
            lo = fminf(lo, fminf(x0, x1));
            hi = fmaxf(hi, fmaxf(x0, x1));
        }
        if (!(lo <= hi)) continue;
        const int2 qr = qrow[jj];
        const int ia = max(max(i0, (int)ceilf(lo - m)), (int)((uint32_t)qr.x & 0xffffu));
        const int ib = min(min(i1, (int)floorf(hi + m)), (int)((uint32_t)qr.x >> 16));
        for (int ii = ia; ii <= ib; ++ii) {
            const int q = qr.y + ii;
            float la, lb, lc;
            if (!barycentric(tu[0], tv[0], tu[1], tv[1], tu[2], tv[2], (float)ii, (float)jj, la,
                             lb, lc))
                return;
            if (la < -RB_BARY_EPS || lb < -RB_BARY_EPS || lc < -RB_BARY_EPS) continue;
            const unsigned long long key = tri_key(tri_dT(la, lb, lc, tdT[0], tdT[1], tdT[2]), tid);
            if (key < keys[q]) {
                const unsigned long long old = atomicMin(keys + q, key);
                if (key < old) changed[q] = 1;
            }
        }
    }
}

// The general path runs over the folded transducers of a chunk only: flist[0] = their count,
// flist[1 ..] = their chunk indices in increasing order. Its kernels are grid-stride loops
// over that list, so a chunk without folded fans costs one short launch each.
__global__ void folded_list(const int32_t *__restrict__ folded, int E, int32_t *flist,
                            unsigned long long *next) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int c = 0;
        for (int el = 0; el < E; ++el)
            if (folded[el]) flist[1 + c++] = el;
        flist[0] = c;
        *next = 0ull;  // the smallest-key pass's work counter
    }
}

constexpr int FOLD_GRID = 2048;  // workgroups of the grid-stride kernels

// One item per run of RCH quads along a pair of neighbouring rays (j, j+1; samples i to
// i + RCH, i >= 1, i + 1 <= min(M_j, M_j+1)). The edge at sample i + 1 of one quad is the
// edge at sample i of the next, so each step loads one new pair of positions (one 16-byte
// load: rays j, j+1 are adjacent) and the two travel-time residuals; consecutive items
// are consecutive ray pairs, so their loads are coalesced.
constexpr int RCH = 8;

template <bool MARK>
__device__ __forceinline__ void raster_run(const SampleBufs &sb, int n_rays, int S, int el,
                                           int c, int j, int nx, int ny, int n_mask,
                                           const int2 *qrow,
                                           unsigned long long *__restrict__ keys,
                                           uint8_t *__restrict__ changed,
                                           uint8_t *__restrict__ marks, int mtx, int mtiles) {
    const i2u Mv = *reinterpret_cast<const i2u *>(sb.M + (size_t)el * n_rays + j);
    if (Mv.x < 0 || Mv.y < 0) return;
    const int top = min(Mv.x, Mv.y);  // quads i with i + 1 <= top
    const int i0 = max(c * RCH, 1), i1 = min(c * RCH + RCH, top);
    if (i0 >= i1) return;
    unsigned long long *ek = keys + (size_t)el * n_mask;
    uint8_t *ec = changed + (size_t)el * n_mask;
    uint8_t *em = marks + (size_t)el * mtiles;
    if (!MARK) {
        // The run's bounding box holds every triangle's: if its tiles hold no mark, no
        // triangle of the run touches a marked tile and each would return at its own test.
        float umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
        size_t bb = ((size_t)el * S + i0) * n_rays + j;
        for (int i = i0; i <= i1; ++i, bb += n_rays) {
            const f4u q = *reinterpret_cast<const f4u *>(sb.pos + bb);
            umin = fminf(umin, fminf(q.x, q.z));
            umax = fmaxf(umax, fmaxf(q.x, q.z));
            vmin = fminf(vmin, fminf(q.y, q.w));
            vmax = fmaxf(vmax, fmaxf(q.y, q.w));
        }
        const float bu[3] = {umin, umax, umax}, bv[3] = {vmin, vmax, vmax};
        int ti0, ti1, tj0, tj1;
        bbox_tiles(bu, bv, nx, ny, ti0, ti1, tj0, tj1);
        bool any = false;
        for (int tj = tj0; tj <= tj1 && !any; ++tj)
            for (int ti = ti0; ti <= ti1; ++ti) any |= em[tj * mtx + ti] != 0;
        if (!any) return;
    }
    size_t b = ((size_t)el * S + i0) * n_rays + j;
    f4u q = *reinterpret_cast<const f4u *>(sb.pos + b);
    float u0 = q.x, v0 = q.y, u1 = q.z, v1 = q.w;
    for (int i = i0; i < i1; ++i) {
        const size_t bp = b;  // row i
        b += n_rays;          // row i + 1
        q = *reinterpret_cast<const f4u *>(sb.pos + b);
        const float u2 = q.z, v2 = q.w, u3 = q.x, v3 = q.y;  // (j+1, i+1), (j, i+1)
        const uint32_t id0 = (uint32_t)(((size_t)j * S + i) * 2);
        float tu0[3] = {u0, u1, u2}, tv0[3] = {v0, v1, v2};
        float tu1[3] = {u0, u2, u3}, tv1[3] = {v0, v2, v3};
        const size_t vb0[3] = {bp, bp + 1, b + 1}, vb1[3] = {bp, b + 1, b};
        if (MARK) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float *tu = h ? tu1 : tu0, *tv = h ? tv1 : tv0;
                const float area =
                    (tu[1] - tu[0]) * (tv[2] - tv[0]) - (tv[1] - tv[0]) * (tu[2] - tu[0]);
                if (area > AREA_MARK) {
                    int ti0, ti1, tj0, tj1;
                    bbox_tiles(tu, tv, nx, ny, ti0, ti1, tj0, tj1);
                    for (int tj = tj0; tj <= tj1; ++tj)
                        for (int ti = ti0; ti <= ti1; ++ti) em[tj * mtx + ti] = 1;
                }
            }
        } else {
            raster_tri(tu0, tv0, sb.fld, vb0, nx, ny, qrow, ek, ec, em, mtx, id0);
            raster_tri(tu1, tv1, sb.fld, vb1, nx, ny, qrow, ek, ec, em, mtx, id0 + 1);
        }
        u0 = u3; v0 = v3;  // (j, i+1)
        u1 = u2; v1 = v2;  // (j+1, i+1)
    }
}

constexpr int RASTER_ROWS = 4096;  // grid rows of the LDS copy of the mask's row table

// Dynamic LDS of the smallest-key pass: the mask's row table when the grid has at most
// RASTER_ROWS rows (the kernel then reads it from LDS), else none (read from memory).
inline size_t raster_lds_bytes(int ny) {
    return ny <= RASTER_ROWS ? (size_t)ny * sizeof(int2) : 0;
}

constexpr int RCHUNK = 1024;  // items a wave of the smallest-key pass takes at a time

template <bool MARK>
__global__ void __launch_bounds__(256) raster_kernel(SampleBufs sb, int n_rays, int S, int nx,
                                                     int ny, int n_mask,
                                                     const int2 *__restrict__ qrow_g,
                                                     const int32_t *__restrict__ flist,
                                                     unsigned long long *__restrict__ keys,
                                                     uint8_t *__restrict__ changed,
                                                     uint8_t *__restrict__ marks, int mtx,
                                                     int mtiles, unsigned long long *next) {
    extern __shared__ int2 s_qrow[];  // raster_lds_bytes(ny) in the smallest-key pass
    const int2 *qrow = qrow_g;
    if (!MARK && ny <= RASTER_ROWS) {
        for (int r = threadIdx.x; r < ny; r += blockDim.x) s_qrow[r] = qrow_g[r];
        __syncthreads();
        qrow = s_qrow;
    }
    const size_t nq = (size_t)n_rays - 1, nc = (size_t)(S + RCH - 1) / RCH, per = nc * nq;
    const size_t total = (size_t)flist[0] * per;
    auto item = [&](size_t t) {
        const int f = (int)(t / per);
        const size_t rest = t - (size_t)f * per;
        const int c = (int)(rest / nq), j = (int)(rest - (size_t)c * nq);
        raster_run<MARK>(sb, n_rays, S, flist[1 + f], c, j, nx, ny, n_mask, qrow, keys, changed,
                         marks, mtx, mtiles);
    };
    if (MARK) {
        for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
             t += (size_t)gridDim.x * blockDim.x)
            item(t);
        return;
    }
    // Runs differ widely in cost (those near marked tiles rasterise, the others return after
    // their bounding-box test), so each wave takes RCHUNK consecutive items at a time from a
    // counter (zeroed by folded_list) instead of a fixed share; every wave leaves once the
    // counter has passed the last item.
    if (total == 0) return;  // no folded fan: not even one atomic per wave
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(next, (unsigned long long)RCHUNK);
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
        const size_t b0 = ((size_t)hi << 32) | lo;
        if (b0 >= total) break;
        const size_t b1 = min(b0 + (size_t)RCHUNK, total);
        for (size_t t = b0 + lane; t < b1; t += 64) item(t);
    }
}

// General path: per (folded transducer, mask node) whose walk result the rasterisation
// replaced, interpolate the winning triangle. Returns the amplitude written (0 if none).
__device__ __forceinline__ float resolve_node(const SampleBufs &sb, int n_rays, int S, int el,
                                             int q, int e0, const GridP &g, double ds, double c0,
                                             int n_mask, const int32_t *__restrict__ mask_index,
                                             const unsigned long long *__restrict__ keys,
                                             const uint8_t *__restrict__ changed,
                                             const TableOut &to) {
    const size_t tid = (size_t)el * n_mask + q;
    if (!changed[tid]) return 0.f;
    int e = e0 + el;
    const TableOut toE = table_row(to, (size_t)e * n_mask);
    const uint32_t out = (uint32_t)q;
    unsigned long long key = keys[tid];
    int p = mask_index[q];
    int ii = p % g.nx, jj = p / g.nx;
    const double2 xy = sb.ring[e];
    double xe = xy.x, ye = xy.y;
    double px = g.x0 + ii * g.dx, py = g.y0 + jj * g.dx;
    double d = sqrt_newton((px - xe) * (px - xe) + (py - ye) * (py - ye));
    if (key == ~0ull || d < 2.0 * ds) {
        if (to.rec) write_invalid<true>(toE, out);
        else write_invalid<false>(toE, out);
        return 0.f;
    }
    uint32_t tri = (uint32_t)(key & 0xffffffffu);
    int half = tri & 1;
    uint32_t rest = tri >> 1;
    int j = (int)(rest / S), i = (int)(rest % S);
    const size_t ebase = (size_t)el * S * n_rays;  // the transducer's samples
    const uint32_t b00 = (uint32_t)(i * n_rays + j), b01 = b00 + (uint32_t)n_rays;
    uint32_t vb[3];
    vb[0] = b00;
    vb[1] = half ? b01 + 1 : b00 + 1;
    vb[2] = half ? b01 : b01 + 1;
    float tu[3], tv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float2 pk = sb.pos[ebase + vb[k]];
        tu[k] = pk.x;
        tv[k] = pk.y;
    }
    float la, lb, lc;
    barycentric(tu[0], tv[0], tu[1], tv[1], tu[2], tv[2], (float)ii, (float)jj, la, lb, lc);
    float lam[3] = {la, lb, lc};
    const int K = tri_K(sb, n_rays, S, el, j, i, half, vb);
    const float4 *fldE = sb.fld + ebase;
    float A;
    if (to.rec)
        write_entry_f<true>(fldE[vb[0]], fldE[vb[1]], fldE[vb[2]], lam, K, (float)d, d, c0, toE,
                            out, A);
    else
        write_entry_f<false>(fldE[vb[0]], fldE[vb[1]], fldE[vb[2]], lam, K, (float)d, d, c0, toE,
                             out, A);
    return A;
}

__global__ void __launch_bounds__(256) resolve_kernel(SampleBufs sb, int n_rays, int S, int e0,
                                                      GridP g, double ds, double c0, int n_mask,
                                                      const int32_t *__restrict__ mask_index,
                                                      const int32_t *__restrict__ flist,
                                                      const unsigned long long *__restrict__ keys,
                                                      const uint8_t *__restrict__ changed,
                                                      TableOut to) {
    // A workgroup takes 256 consecutive nodes of one folded transducer, so the largest A and
    // 1/A it writes reach the per-row maxima as one atomic pair per wave (the walk's are
    // folded in by tile_max_fold; max is order-independent).
    const int per = (n_mask + 255) / 256;
    const size_t total = (size_t)flist[0] * per;
    for (size_t b = blockIdx.x; b < total; b += gridDim.x) {  // uniform over the workgroup
        const int f = (int)(b / per);
        const int el = flist[1 + f];
        const int q = (int)(b - (size_t)f * per) * 256 + (int)threadIdx.x;
        float A = 0.f;
        if (q < n_mask)
            A = resolve_node(sb, n_rays, S, el, q, e0, g, ds, c0, n_mask, mask_index, keys,
                             changed, to);
        if (to.rowmax) {
            const float m0 = wave_max(A), m1 = wave_max(A > 0.f ? 1.0f / A : 0.f);
            if ((threadIdx.x & 63) == 0 && m0 > 0.f) {
                atomicMax(to.rowmax + 2 * (e0 + el), __float_as_uint(m0));
                atomicMax(to.rowmax + 2 * (e0 + el) + 1, __float_as_uint(m1));
            }
        }
    }
}

// Receiver tables: per emitter, bracket each receiver's angle between neighbouring exit
// angles and interpolate dT and L linearly; the smallest travel time wins (lowest ray on a
// tie); unbracketed pairs are invalid. When every ray is valid and the exit angles increase
// strictly with the ray index, the bracket of a receiver is unique and found by bisection.
// rx_j (nullable, [E][N]): the fan ray j of the chosen bracket (j, j + 1) of each receiver,
// -1 if none (the starting points of ray linking).
__global__ void __launch_bounds__(256) receiver_kernel(SampleBufs sb, int n_rays, int e0, double R,
                                                       double psi0, int N, double c0,
                                                       rb_tables tb, int32_t *rx_j) {
    extern __shared__ __attribute__((aligned(16))) char smem[];  // 64-bit LDS atomics below
    double *beta = reinterpret_cast<double *>(smem);
    float *dTs = reinterpret_cast<float *>(beta + n_rays);
    float *Ls = dTs + n_rays;
    int *ok = reinterpret_cast<int *>(Ls + n_rays);
    uint8_t *Ks = reinterpret_cast<uint8_t *>(ok + n_rays);
    // per receiver (index rel = (r - e) mod N): smallest travel time, then its lowest ray pair
    unsigned long long *rkey =
        reinterpret_cast<unsigned long long *>(smem + ((n_rays * 21 + 7) & ~7));
    int *rwin = reinterpret_cast<int *>(rkey + N);
    __shared__ int not_monotone;
    int el = blockIdx.x, e = e0 + el;
    if (threadIdx.x == 0) not_monotone = 0;
    for (int j = threadIdx.x; j < n_rays; j += blockDim.x) {
        size_t x = (size_t)el * n_rays + j;
        int good = sb.M[x] >= 0;
        ok[j] = good;
        beta[j] = good ? sb.ex_beta[x] : 0.0;
        dTs[j] = good ? sb.ex_dT[x] : 0.0f;
        Ls[j] = good ? sb.ex_L[x] : 0.0f;
        Ks[j] = good ? sb.ex_K[x] : 0;
    }
    __syncthreads();
    for (int j = threadIdx.x; j + 1 < n_rays; j += blockDim.x)
        if (!(ok[j] && ok[j + 1] && beta[j + 1] > beta[j])) not_monotone = 1;
    __syncthreads();
    const bool mono = !not_monotone;
    // Without monotone exit angles every ray pair offers itself to the receivers whose angle
    // it brackets (the scan's test and interpolation): the smallest travel time wins, then the
    // lowest pair, as in a scan over the pairs in order.
    auto dT_at = [&](int j, double br) {
        double b0 = beta[j], b1 = beta[j + 1];
        double lam = (br - b0) / (b1 - b0);
        return (1.0 - lam) * (double)dTs[j] + lam * (double)dTs[j + 1];
    };
    auto pair_range = [&](int j, int &rl0, int &rl1) {  // receivers (rel) pair j may bracket
        const double lo = fmin(beta[j], beta[j + 1]), hi = fmax(beta[j], beta[j + 1]);
        rl0 = max(1, (int)floor(lo * (double)N / RB_TWO_PI) - 1);
        rl1 = min(N - 1, (int)ceil(hi * (double)N / RB_TWO_PI) + 1);
    };
    auto brackets = [&](int j, double br) {
        double b0 = beta[j], b1 = beta[j + 1];
        return ok[j] && ok[j + 1] && !(b0 == b1 || br < fmin(b0, b1) || br > fmax(b0, b1));
    };
    if (!mono) {
        for (int k = threadIdx.x; k < N; k += blockDim.x) {
            rkey[k] = ~0ull;
            rwin[k] = INT_MAX;
        }
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            for (int j = threadIdx.x; j + 1 < n_rays; j += blockDim.x) {
                if (!(ok[j] && ok[j + 1])) continue;
                int rl0, rl1;
                pair_range(j, rl0, rl1);
                for (int rel = rl0; rel <= rl1; ++rel) {
                    const double br = RB_TWO_PI * (double)rel / (double)N;
                    if (!brackets(j, br)) continue;
                    const unsigned long long k = ordered_bits64(dT_at(j, br));
                    if (pass == 0) atomicMin(rkey + rel, k);
                    else if (k == rkey[rel]) atomicMin(rwin + rel, j);
                }
            }
            __syncthreads();
        }
    }
    const double2 xy = sb.ring[e];
    double xe = xy.x, ye = xy.y;
    for (int r = threadIdx.x; r < N; r += blockDim.x) {
        size_t out = (size_t)e * N + r;
        int rel = ((r - e) % N + N) % N;
        double br = RB_TWO_PI * (double)rel / (double)N;
        bool found = false;
        double best = 0.0, bestL = 0.0;
        int bestK = 0, bestJ = -1;
        auto take = [&](int j) {
            double b0 = beta[j], b1 = beta[j + 1];
            double lam = (br - b0) / (b1 - b0);
            double dT = (1.0 - lam) * (double)dTs[j] + lam * (double)dTs[j + 1];
            if (!found || dT < best) {
                found = true;
                bestJ = j;
                best = dT;
                bestL = (1.0 - lam) * (double)Ls[j] + lam * (double)Ls[j + 1];
                bestK = max((int)Ks[j], (int)Ks[j + 1]);
            }
        };
        if (r != e) {
            if (mono) {
                if (br >= beta[0] && br <= beta[n_rays - 1]) {
                    int lo = 0, hi = n_rays - 1;  // beta[lo] <= br <= beta[hi]
                    while (hi - lo > 1) {
                        int mid = (lo + hi) >> 1;
                        if (beta[mid] <= br) lo = mid;
                        else hi = mid;
                    }
                    // a receiver exactly on a ray's exit angle is bracketed on both sides;
                    // the lower pair wins the tie as in the full scan
                    if (lo > 0 && beta[lo] == br) take(lo - 1);
                    take(lo);
                }
            } else if (rwin[rel] != INT_MAX) {
                take(rwin[rel]);
            }
        }
        if (found) {
            const double2 rr = sb.ring[r];
            double xr = rr.x, yr = rr.y;
            double dist = sqrt((xr - xe) * (xr - xe) + (yr - ye) * (yr - ye));
            tb.rx_T[out] = best + dist / c0;
            tb.rx_A[out] = (float)(exp(bestL) / sqrt(dist));
            tb.rx_flags[out] = (uint8_t)(0x80 | (bestK & 3));
        } else {
            tb.rx_T[out] = 0.0;
            tb.rx_A[out] = 0.0f;
            tb.rx_flags[out] = 0;
        }
        if (rx_j) rx_j[(size_t)el * N + r] = found ? bestJ : -1;
    }
}

// Ray linking (Sections 4 and 6.3): one lane per (chunk transducer el, receiver r). The
// launch angle is adjusted by a safeguarded secant on f(gamma) = beta(gamma) - beta_r, from
// the two fan rays of the receiver's bracket (their exit angles are known): the secant
// point of the last two iterates when it lies inside the bracket, else the bracket's
// midpoint; each traced ray keeps a sign change of f inside the bracket. Stops at |f| <=
// tol or after max_iter rays; the traced ray closest to its receiver gives the receiver
// tables if |f| <= accept, else the pair is invalid. Pairs without a bracket keep the
// receiver kernel's invalid entry.
template <bool ABS>
__global__ void __launch_bounds__(PATCH_STRIDE) __attribute__((amdgpu_waves_per_eu(2))) link_kernel(SplineMap m, AbsMap am, GridP g, double R, double psi0,
                                                   int N, int n_rays, int max_steps, double ds,
                                                   double c0, int e0, int E, SampleBufs sb,
                                                   const int32_t *__restrict__ rx_j,
                                                   int max_iter, double tol, double accept,
                                                   rb_tables tb) {
    __shared__ float4 s_patch[4 * PATCH_STRIDE];
    m.patch = s_patch + threadIdx.x;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= E * N) return;
    const int el = t / N, r = t - el * N, e = e0 + el;
    const int j = rx_j[t];
    if (j < 0) return;
    const double psi = psi0 + RB_TWO_PI * (double)e / (double)N;
    const double br = RB_TWO_PI * (double)(((r - e) % N + N) % N) / (double)N;
    const double2 xy = sb.ring[e];
    const double dgam = RB_PI / (double)n_rays;
    double lo = psi + RB_PI + ((double)j + 0.5 - 0.5 * (double)n_rays) * dgam;
    double hi = lo + dgam;
    const size_t x = (size_t)el * n_rays + j;
    double flo = sb.ex_beta[x] - br, fhi = sb.ex_beta[x + 1] - br;
    double xp = lo, fp = flo, xc = hi, fc = fhi;
    double best_f = 1e300;
    RayEnd best{};
    for (int it = 0; it < max_iter && best_f > tol; ++it) {
        double cand = xc - fc * (xc - xp) / (fc - fp);
        const double a = fmin(lo, hi), b = fmax(lo, hi);
        if (!(cand > a && cand < b)) cand = 0.5 * (lo + hi);  // also catches NaN
        double sgm, cgm;
        sincos(cand, &sgm, &cgm);
        RayEnd end;
        if (trace_core<false, ABS>(m, am, g, R, psi, xy, cgm, sgm, n_rays, max_steps, ds, c0, el,
                                   0, sb, nullptr, &end) < 0)
            break;  // the ray did not reach the ring: the pair ends here
        const double f = end.beta - br;
        if (fabs(f) < best_f) {
            best_f = fabs(f);
            best = end;
        }
        if ((f < 0.0) == (flo < 0.0)) {
            lo = cand;
            flo = f;
        } else {
            hi = cand;
            fhi = f;
        }
        xp = xc;
        fp = fc;
        xc = cand;
        fc = f;
    }
    const size_t out = (size_t)e * N + r;
    if (best_f <= accept) {
        tb.rx_T[out] = best.T;
        tb.rx_A[out] = (float)(exp((double)best.L) / sqrt(best.d));
        tb.rx_flags[out] = (uint8_t)(0x80 | (best.K & 3));
    } else {
        tb.rx_T[out] = 0.0;
        tb.rx_A[out] = 0.0f;
        tb.rx_flags[out] = 0;
    }
}

// n = c0 / c followed by a separable odd box window with replicated edges (FP64 sums).
__global__ void box_rows(const double *__restrict__ c, double c0, int nx, int ny, int w,
                         double *__restrict__ tmp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= nx) return;
    int h = w / 2;
    double acc = 0.0;
    for (int s = -h; s <= h; ++s) {
        int k = min(max(i + s, 0), nx - 1);
        acc += c0 / c[(size_t)j * nx + k];
    }
    tmp[(size_t)j * nx + i] = acc / w;
}

__global__ void box_cols(const double *__restrict__ tmp, int nx, int ny, int w,
                         float *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= nx) return;
    int h = w / 2;
    double acc = 0.0;
    for (int s = -h; s <= h; ++s) {
        int k = min(max(j + s, 0), ny - 1);
        acc += tmp[(size_t)k * nx + i];
    }
    out[(size_t)j * nx + i] = (float)(acc / w);
}

// Row pass of the box window over a plain map (the absorption alpha0), FP64 sums.
__global__ void box_rows_plain(const double *__restrict__ f, int nx, int ny, int w,
                               double *__restrict__ tmp) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= nx) return;
    int h = w / 2;
    double acc = 0.0;
    for (int s = -h; s <= h; ++s) acc += f[(size_t)j * nx + min(max(i + s, 0), nx - 1)];
    tmp[(size_t)j * nx + i] = acc / w;
}

// Column pass of both maps and the maps of one frequency (Section 2.2, Eq. wave-number):
// n_w = box(c0/c) + kd box(alpha0) with kd = c0 tan(pi y/2) omega^(y-1) (the wavenumber in
// units of k0), a_w = ky box(alpha0) with ky = omega^y (the absorption in Np/m). With
// alpha0 = 0 the index is box(c0/c) to the bit.
__global__ void box_cols_lossy(const double *__restrict__ tn, const double *__restrict__ ta,
                               int nx, int ny, int w, double kd, double ky,
                               float *__restrict__ n_w, float *__restrict__ a_w) {
    int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= nx) return;
    int h = w / 2;
    double an = 0.0, aa = 0.0;
    for (int s = -h; s <= h; ++s) {
        const size_t o = (size_t)min(max(j + s, 0), ny - 1) * nx + i;
        an += tn[o];
        aa += ta[o];
    }
    const double al = aa / w;
    n_w[(size_t)j * nx + i] = (float)(an / w + kd * al);
    a_w[(size_t)j * nx + i] = (float)(ky * al);
}

// Transducer positions, and the walk's per-transducer constants in FP32: the grid origin
// relative to the transducer (x0 - x_e, y0 - y_e) and psi_e + pi (its straight-ray guess).
__global__ void ring_positions(double R, double psi0, int N, double2 *pos, GridP g, float dpsi,
                               float4 *wcon) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < N) {
        double psi = psi0 + RB_TWO_PI * (double)e / (double)N;
        const double2 xy = make_double2(R * cos(psi), R * sin(psi));
        pos[e] = xy;
        wcon[e] = make_float4((float)(g.x0 - xy.x), (float)(g.y0 - xy.y),
                              (float)(psi0 + RB_PI) + (float)e * dpsi, 0.f);
    }
}

// Per-transducer maxima of the walk's waves (tmax, one pair per (transducer, tile, wave) of a
// chunk) folded into rowmax; one workgroup per transducer of the chunk.
__global__ void __launch_bounds__(256) tile_max_fold(const float *__restrict__ tmax, int ntiles,
                                                     int e0, unsigned int *__restrict__ rowmax) {
    __shared__ float red[2][4];
    const int el = blockIdx.x;
    const int per = ntiles * LOCATE_WAVES;
    float m0 = 0.f, m1 = 0.f;
    for (int t = threadIdx.x; t < per; t += blockDim.x) {
        const size_t o = 2 * ((size_t)el * per + t);
        m0 = fmaxf(m0, tmax[o]);
        m1 = fmaxf(m1, tmax[o + 1]);
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
        m0 = fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3]));
        m1 = fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3]));
        atomicMax(rowmax + 2 * (e0 + el), __float_as_uint(m0));
        atomicMax(rowmax + 2 * (e0 + el) + 1, __float_as_uint(m1));
    }
}

__global__ void zero_i32(int32_t *x, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0;
}

}  // namespace

rb_status rb_launch_refractive_index(rb_ctx *ctx, const rb_grid *g, const double *c, double c0,
                                     int w, float *n_s) {
    ctx->ws.used = 0;
    size_t P = (size_t)g->nx * g->ny;
    rb_status st = rb_arena_reserve(ctx, &ctx->ws, rb_align(P * sizeof(double)));
    if (st != RB_OK) return st;
    double *tmp = rb_carve<double>(&ctx->ws, P);
    dim3 blk(256), grd((g->nx + 255) / 256, g->ny);
    rb_prof_begin(ctx, ST_SMOOTH);
    hipLaunchKernelGGL(box_rows, grd, blk, 0, ctx->stream, c, c0, g->nx, g->ny, w, tmp);
    RB_CHECK_LAUNCH(ctx);
    hipLaunchKernelGGL(box_cols, grd, blk, 0, ctx->stream, tmp, g->nx, g->ny, w, n_s);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

// Absorbing media: the row passes of both maps (kept for the maps of every frequency of a
// step) and the sound-speed part n_s = box(c0/c) (skipped for n_s == nullptr).
rb_status rb_launch_lossy_rows(rb_ctx *ctx, const rb_grid *g, const double *c, double c0,
                               const double *alpha0, int w, double *tn, double *ta,
                               float *n_s) {
    dim3 blk(256), grd((g->nx + 255) / 256, g->ny);
    rb_prof_begin(ctx, ST_SMOOTH);
    hipLaunchKernelGGL(box_rows, grd, blk, 0, ctx->stream, c, c0, g->nx, g->ny, w, tn);
    RB_CHECK_LAUNCH(ctx);
    if (n_s) {
        hipLaunchKernelGGL(box_cols, grd, blk, 0, ctx->stream, tn, g->nx, g->ny, w, n_s);
        RB_CHECK_LAUNCH(ctx);
    }
    hipLaunchKernelGGL(box_rows_plain, grd, blk, 0, ctx->stream, alpha0, g->nx, g->ny, w, ta);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

rb_status rb_launch_lossy_map(rb_ctx *ctx, const rb_grid *g, const double *tn, const double *ta,
                              int w, double kd, double ky, float *n_w, float *a_w) {
    dim3 blk(256), grd((g->nx + 255) / 256, g->ny);
    rb_prof_begin(ctx, ST_SMOOTH);
    hipLaunchKernelGGL(box_cols_lossy, grd, blk, 0, ctx->stream, tn, ta, g->nx, g->ny, w, kd, ky,
                       n_w, a_w);
    RB_CHECK_LAUNCH(ctx);
    rb_prof_end(ctx);
    return RB_OK;
}

// Emitters per tracer launch so that the ray samples of one chunk fit the budget.
static int trace_chunk(size_t budget, const rb_ring *r, const rb_trace_params *tp,
                       int64_t n_mask) {
    size_t S = (size_t)tp->max_steps + 1;
    size_t per = S * tp->n_rays * (sizeof(float2) + sizeof(float4) + 1) + (size_t)n_mask * 8 +
                 (size_t)tp->n_rays * 32;
    size_t c = budget / per;
    if (c < 1) c = 1;
    if (c > (size_t)r->n) c = r->n;
    return (int)c;
}

static size_t mtiles_of(const rb_grid *g) {
    const size_t mtx = (g->nx + (1 << MT_SHIFT) - 1) >> MT_SHIFT;
    const size_t mty = (g->ny + (1 << MT_SHIFT) - 1) >> MT_SHIFT;
    return mtx * mty;
}

// Workspace of one tracer launch of C emitters (`tiles` walk tiles over the mask).
static size_t trace_bytes(const rb_grid *g, const rb_ring *r, const rb_trace_params *tp,
                          int64_t n_mask, int C, size_t tiles) {
    const size_t nr = tp->n_rays, S = (size_t)tp->max_steps + 1;
    const size_t plane = (size_t)C * S * nr;
    return rb_align(plane * sizeof(float2)) + rb_align(plane * sizeof(float4)) +
           rb_align(plane) + 2 * rb_align((size_t)C * nr * sizeof(int32_t)) +
           rb_align((size_t)C * nr * sizeof(double)) +
           2 * rb_align((size_t)C * nr * sizeof(float)) + rb_align((size_t)C * nr) +
           rb_align((size_t)C * sizeof(int32_t)) + rb_align(((size_t)C + 4) * sizeof(int32_t)) +
           rb_align((size_t)r->n * sizeof(double2)) + rb_align((size_t)r->n * sizeof(float4)) +
           rb_align((size_t)C * tiles * sizeof(int2)) +
           rb_align((size_t)C * n_mask * sizeof(unsigned long long)) +
           rb_align((size_t)C * n_mask) + rb_align(mtiles_of(g) * (size_t)C + 4) +
           2 * rb_align((size_t)(g->nx + 2 * MPAD) * (g->ny + 2 * MPAD) * sizeof(float)) +
           rb_align((size_t)(g->nx + 3) * (g->ny + 3) * 4 * sizeof(float4)) +
           rb_align((size_t)C * r->n * sizeof(int32_t)) +
           rb_align((size_t)C * tiles * LOCATE_WAVES * 2 * sizeof(float));
}

size_t rb_trace_ws_bytes(const rb_grid *g, const rb_ring *r, const rb_trace_params *tp,
                         int64_t n_mask, size_t tiles, size_t sample_budget) {
    return trace_bytes(g, r, tp, n_mask, trace_chunk(sample_budget, r, tp, n_mask), tiles);
}

rb_status rb_launch_trace(rb_ctx *ctx, const rb_grid *g, const rb_ring *r,
                          const rb_trace_params *tp, const float *n_s, const rb_tables *out,
                          float4 *rec, double2 *ring_out, unsigned int *rowmax,
                          const float *a_w) {
    const int N = r->n, nr = tp->n_rays, S = tp->max_steps + 1;
    const int n_mask = (int)ctx->n_mask;
    const int C = trace_chunk(ctx->sample_budget, r, tp, n_mask);
    size_t plane = (size_t)C * S * nr;
    const size_t bytes =
        trace_bytes(g, r, tp, n_mask, C, (size_t)ctx->tiles_x * ctx->tiles_y);
    ctx->ws.used = 0;
    rb_status st = rb_arena_reserve(ctx, &ctx->ws, bytes);
    if (st != RB_OK) return st;
    SampleBufs sb;
    sb.pos = rb_carve<float2>(&ctx->ws, plane);
    sb.fld = rb_carve<float4>(&ctx->ws, plane);
    sb.K = rb_carve<uint8_t>(&ctx->ws, plane);
    sb.M = rb_carve<int32_t>(&ctx->ws, (size_t)C * nr);
    sb.kfirst = rb_carve<int32_t>(&ctx->ws, (size_t)C * nr);
    sb.ex_beta = rb_carve<double>(&ctx->ws, (size_t)C * nr);
    sb.ex_dT = rb_carve<float>(&ctx->ws, (size_t)C * nr);
    sb.ex_L = rb_carve<float>(&ctx->ws, (size_t)C * nr);
    sb.ex_K = rb_carve<uint8_t>(&ctx->ws, (size_t)C * nr);
    sb.folded = rb_carve<int32_t>(&ctx->ws, (size_t)C);
    int32_t *flist = rb_carve<int32_t>(&ctx->ws, (size_t)C + 4);  // + the 8-byte counter
    unsigned long long *rnext = reinterpret_cast<unsigned long long *>(flist + ((C + 2) & ~1));
    double2 *ringpos = rb_carve<double2>(&ctx->ws, (size_t)N);
    float4 *wcon = rb_carve<float4>(&ctx->ws, (size_t)N);
    if (ring_out) ringpos = ring_out;
    int2 *toff = rb_carve<int2>(&ctx->ws, (size_t)C * ctx->tiles_x * ctx->tiles_y);
    float *tmax =
        rb_carve<float>(&ctx->ws, (size_t)C * ctx->tiles_x * ctx->tiles_y * LOCATE_WAVES * 2);
    const bool rows = rec && rowmax;
    const TableOut to{*out, rec, rows ? tmax : nullptr, rows ? rowmax : nullptr};
    sb.ring = ringpos;
    unsigned long long *keys = rb_carve<unsigned long long>(&ctx->ws, (size_t)C * n_mask);
    uint8_t *changed = rb_carve<uint8_t>(&ctx->ws, (size_t)C * n_mask);
    const int mtx = (g->nx + (1 << MT_SHIFT) - 1) >> MT_SHIFT;
    const int mtiles = (int)mtiles_of(g);
    uint8_t *marks = rb_carve<uint8_t>(&ctx->ws, (size_t)C * mtiles + 4);  // whole words zeroed
    const int nxp = g->nx + 2 * MPAD, nyp = g->ny + 2 * MPAD;
    float *padded = rb_carve<float>(&ctx->ws, (size_t)nxp * nyp);
    float *apad = rb_carve<float>(&ctx->ws, (size_t)nxp * nyp);
    const AbsMap amap{a_w ? apad : nullptr, g->nx, g->ny, nxp};
    int32_t *rx_j = rb_carve<int32_t>(&ctx->ws, (size_t)C * N);
    float4 *coef = rb_carve<float4>(&ctx->ws, (size_t)(g->nx + 3) * (g->ny + 3) * 4);
    SplineMap smap{coef, g->nx, g->ny, g->nx + 3, (float)(1.0 / g->dx)};

    GridP gp{g->nx, g->ny, g->dx, g->x0, g->y0, 1.0 / g->dx};
    // counters of this trace; the error bits start clear unless a sweep collects them
    int32_t *lost = ctx->d_flag + RB_W_LOST;
    unsigned long long *nsamp = reinterpret_cast<unsigned long long *>(ctx->d_flag + RB_W_SAMPLES);
    if (!ctx->deferred) RB_TRY(rb_launch_fill_i32(ctx, ctx->d_flag, RB_W_COUNT, 0));
    else RB_TRY(rb_launch_fill_i32(ctx, ctx->d_flag + RB_W_LOST, RB_W_COUNT - RB_W_LOST, 0));
    hipLaunchKernelGGL(ring_positions, dim3((N + 255) / 256), dim3(256), 0, ctx->stream,
                       r->radius, r->psi0, N, ringpos, gp, (float)(RB_TWO_PI / N), wcon);
    RB_CHECK_LAUNCH(ctx);
    if (rows) RB_TRY(rb_launch_fill_i32(ctx, reinterpret_cast<int32_t *>(rowmax), 2 * N, 0));
    hipLaunchKernelGGL(pad_map, dim3((nxp + 255) / 256, nyp), dim3(256), 0, ctx->stream, n_s,
                       g->nx, g->ny, 1.0f, padded);
    RB_CHECK_LAUNCH(ctx);
    if (a_w) {
        hipLaunchKernelGGL(pad_map, dim3((nxp + 255) / 256, nyp), dim3(256), 0, ctx->stream, a_w,
                           g->nx, g->ny, 0.0f, apad);
        RB_CHECK_LAUNCH(ctx);
    }
    hipLaunchKernelGGL(spline_coef, dim3((g->nx + 3 + 255) / 256, g->ny + 3), dim3(256), 0,
                       ctx->stream, padded, g->nx, g->ny, coef);
    RB_CHECK_LAUNCH(ctx);
    for (int e0 = 0; e0 < N; e0 += C) {
        int E = std::min(C, N - e0);
        hipLaunchKernelGGL(zero_i32, dim3((E + 255) / 256), dim3(256), 0, ctx->stream, sb.folded,
                           E);
        RB_CHECK_LAUNCH(ctx);
        const int mwords = (int)(((size_t)E * mtiles + 3) / 4);
        hipLaunchKernelGGL(zero_i32, dim3((mwords + 255) / 256), dim3(256), 0, ctx->stream,
                           reinterpret_cast<int32_t *>(marks), mwords);
        RB_CHECK_LAUNCH(ctx);
        rb_prof_begin(ctx, ST_TRACE);
        const int waves = E * ((nr + 63) / 64);
        hipLaunchKernelGGL(a_w ? trace_kernel<true> : trace_kernel<false>,
                           dim3((waves + 3) / 4), dim3(256), 0, ctx->stream, smap, amap, gp,
                           r->radius, r->psi0, N, nr, tp->max_steps, tp->ds, tp->c0, e0, E, sb,
                           ctx->d_flag, nsamp);
        RB_CHECK_LAUNCH(ctx);
        rb_prof_end(ctx);
        // folded fans: tiles near inverted triangles
        rb_prof_begin(ctx, ST_RASTER);
        hipLaunchKernelGGL(folded_list, dim3(1), dim3(64), 0, ctx->stream, sb.folded, E, flist,
                           rnext);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(raster_kernel<true>, dim3(FOLD_GRID), dim3(256), 0, ctx->stream, sb,
                           nr, S, g->nx, g->ny, n_mask, ctx->d_qrow, flist, keys, changed, marks,
                           mtx, mtiles, rnext);
        RB_CHECK_LAUNCH(ctx);
        rb_prof_end(ctx);
        // every fan: walk per (transducer, node); for folded fans also the seed keys
        rb_prof_begin(ctx, ST_RESOLVE);
        int ntiles = ctx->tiles_x * ctx->tiles_y;
        hipLaunchKernelGGL(tile_offset_kernel, dim3((E * ntiles + 255) / 256), dim3(256), 0,
                           ctx->stream, sb, nr, S, E, e0, gp, r->psi0, N, tp->ds, ctx->tile_i0,
                           ctx->tile_j0, ctx->tiles_x, ctx->tiles_y, (float)(RB_TWO_PI / N),
                           1.0 / tp->ds, toff);
        RB_CHECK_LAUNCH(ctx);
        const long G = (long)LOCATE_GROUP_ROWS * ctx->tiles_x;
        const long groups = ((long)E * ntiles + G - 1) / G;
        const long nblk = (groups + 7) / 8 * 8 * G;
        hipLaunchKernelGGL(rec ? locate_kernel<true> : locate_kernel<false>, dim3((unsigned)nblk),
                           dim3(LOCATE_THREADS), 0, ctx->stream,
                           sb, nr,
                           S, E, e0, gp, r->radius, r->psi0, N, tp->ds, tp->c0, n_mask,
                           ctx->tile_i0, ctx->tile_j0, ctx->tiles_x, ctx->tiles_y, ctx->d_qmap,
                           toff, to, keys, changed, marks, mtx, mtiles, lost,
                           (float)(1.0 / tp->ds), (float)(2.0 * tp->ds), (float)(-g->x0 / g->dx),
                           (float)(-g->y0 / g->dx),
                           (float)((g->mask_radius / g->dx + 2.0) * (g->mask_radius / g->dx + 2.0)),
                           wcon);
        RB_CHECK_LAUNCH(ctx);
        if (rows) {
            hipLaunchKernelGGL(tile_max_fold, dim3(E), dim3(256), 0, ctx->stream, tmax, ntiles,
                               e0, rowmax);
            RB_CHECK_LAUNCH(ctx);
        }
        rb_prof_end(ctx);
        // folded fans: smallest-key rasterisation against the walk's keys, and resolve of
        // the nodes it changed
        rb_prof_begin(ctx, ST_RASTER);
        // as many workgroups as are resident at once (with 2048, registers and LDS let 5 or 6
        // per CU run and the rest waited for a second round); their waves take the items from
        // the counter folded_list zeroed
        const size_t rlds = raster_lds_bytes(g->ny);
        int rpc = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&rpc, raster_kernel<false>, 256, rlds) !=
                hipSuccess ||
            rpc < 1) {
            (void)hipGetLastError();  // a failed query is no launch error
            rpc = 4;
        }
        hipLaunchKernelGGL(raster_kernel<false>, dim3(rpc * ctx->n_cu), dim3(256), rlds,
                           ctx->stream, sb, nr, S, g->nx, g->ny, n_mask, ctx->d_qrow, flist, keys,
                           changed, marks, mtx, mtiles, rnext);
        RB_CHECK_LAUNCH(ctx);
        hipLaunchKernelGGL(resolve_kernel, dim3(FOLD_GRID), dim3(256), 0, ctx->stream, sb, nr, S,
                           e0, gp, tp->ds, tp->c0, n_mask, ctx->d_mask_index, flist, keys,
                           changed, to);
        RB_CHECK_LAUNCH(ctx);
        rb_prof_end(ctx);
        rb_prof_begin(ctx, ST_RECEIVERS);
        size_t smem = (((size_t)nr * 21 + 7) & ~(size_t)7) + (size_t)N * 12;
        if (smem > (size_t)160 * 1024)
            return rb_fail(ctx, RB_EINVAL, "n_rays=%d with n=%d needs %zu bytes of LDS for the "
                           "receiver tables (at most 160 KiB)", nr, N, smem);
        if (smem > (size_t)64 * 1024)
            RB_HIP(ctx, hipFuncSetAttribute((const void *)receiver_kernel,
                                            hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)smem));
        hipLaunchKernelGGL(receiver_kernel, dim3(E), dim3(256), smem, ctx->stream, sb, nr, e0,
                           r->radius, r->psi0, N, tp->c0, *out,
                           ctx->link_iter > 0 ? rx_j : nullptr);
        RB_CHECK_LAUNCH(ctx);
        if (ctx->link_iter > 0) {
            const long lanes = (long)E * N;
            hipLaunchKernelGGL(a_w ? link_kernel<true> : link_kernel<false>,
                               dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0,
                               ctx->stream, smap, amap, gp, r->radius, r->psi0, N, nr, tp->max_steps,
                               tp->ds, tp->c0, e0, E, sb, rx_j, ctx->link_iter, ctx->link_tol,
                               RB_LINK_ACCEPT, *out);
            RB_CHECK_LAUNCH(ctx);
        }
        rb_prof_end(ctx);
    }
    if (ctx->deferred) return RB_OK;  // read back at the end of the sweep
    RB_HIP(ctx, hipMemcpyAsync(ctx->h_flag, ctx->d_flag, RB_W_COUNT * sizeof(int32_t),
                               hipMemcpyDeviceToHost, ctx->stream));
    RB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->lost_nodes = ctx->h_flag[RB_W_LOST];
    ctx->ray_samples = *reinterpret_cast<const int64_t *>(ctx->h_flag + RB_W_SAMPLES);
    if (ctx->h_flag[RB_W_FLAGS] & 1)
        return rb_fail(ctx, RB_ENONFINITE, "a ray did not reach the ring within max_steps=%d",
                       tp->max_steps);
    return RB_OK;
}
