/*
 * raybornhf: one Hessian-free ray-Born frequency step on an AMD MI355X (gfx950).
 *
 * Method: A. Javaherian, "Hessian-free ray-Born inversion for quantitative ultrasound
 * tomography of weakly heterogeneous media" (arXiv 2211.00316).
 *   - problem setting: Section 2.1 (ring of point emitters/receivers, sound speed c(x),
 *     c0 outside the imaging region); unknown m = c^-2 (Section 3);
 *   - ray tracing: Section 4 (Hamiltonian and paraxial ray equations, Algorithm 1);
 *   - ray-to-grid interpolation: Section 4.5; receivers: Section 6.3;
 *   - ray Green's function: Eqs. 2D_greens, phase-discretised, amplitude-geom-discretised;
 *   - Born operator: Eqs. perturb1, derivative, scattering-potential;
 *   - Q=1 gradient: Eq. functional-gradient; Hessian-free direction: Eqs.
 *     sound_speed_update, sound_speed_update2; update m <- m + tau dm (Section 3.4);
 *   - absorbing, dispersive media (Szabo's model, Section 2.2): Eqs.
 *     szabo_dispersion_equation, wave-number, amplitude-abs-discretised, the complex
 *     scattering potential and Section 3.4's d|kbar|/domega (rb_absorption, *_lossy).
 *
 * Conventions (every entry point):
 *   - Lengths in metres, times in seconds, angular frequencies in rad/s.
 *   - Grid node (j, i) sits at (x0 + i dx, y0 + j dx); flat index p = j nx + i (x fastest).
 *     The imaging mask keeps nodes with x^2 + y^2 <= mask_radius^2; "mask nodes" are listed
 *     in ascending flat index, P_m of them (rb_mask_count).
 *   - Transducer e sits at R (cos psi_e, sin psi_e), psi_e = psi0 + 2 pi e / N.
 *   - Every array argument is a DEVICE pointer allocated and owned by the caller; the
 *     library never frees it. Complex numbers are interleaved (re, im) float pairs.
 *   - Calls are asynchronous on the context's stream; outputs are ready when that stream is.
 *     Exceptions, which wait for the stream before they return: rb_trace_rays (it reports a
 *     ray that exceeded max_steps), rb_frequency_step without a report, rb_frequency_sweep,
 *     rb_frequency_step_batch, rb_autotune and rb_profile_read.
 *   - Workspace: a context allocates device memory when a call first needs it and grows it
 *     on demand (freeing the old block after waiting for the stream). After rb_reserve for a
 *     geometry, no entry point allocates, frees or waits for the stream on account of its
 *     workspace: a call that would need more than was reserved fails with RB_ENOMEM before
 *     launching anything. A reserved context with a report pointer can therefore be captured
 *     into a HIP graph one rb_frequency_step at a time.
 *   - Every entry point validates its arguments before launching anything and returns an
 *     rb_status; on RB_EINVAL / RB_EUNSUPPORTED nothing was launched (outputs unchanged).
 *     RB_ENONFINITE is reported after the kernels ran (outputs unspecified, except that
 *     rb_frequency_step then leaves the model unchanged); RB_EDEVICE reports a failed HIP
 *     call. rb_last_error() describes the problem.
 *   - A context may be used from one host thread at a time.
 */
#ifndef RAYBORNHF_H
#define RAYBORNHF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RB_OK = 0,
    RB_EINVAL = -1,       /* invalid argument (null pointer, size, geometry) */
    RB_ENOMEM = -2,       /* device workspace allocation failed */
    RB_EDEVICE = -3,      /* a HIP runtime call failed */
    RB_ENONFINITE = -4,   /* a ray exceeded max_steps, or a non-finite update was rejected */
    RB_EUNSUPPORTED = -5  /* requested mode / precision not available */
} rb_status;

/* Operand type of the Born contractions. RB_F16X: FP16 operands, with the back-projection
 * operand H stored as two FP16 parts, h = h_hi + h_lo (h_lo: the rounding error of h_hi),
 * and the back-projection's epilogue weighting the low part twice against R h_hi (R's whole
 * symmetric part): the bilinear form h^T R h is then free of the first-order rounding of h,
 * which dominates the error of the plain 16-bit forms. Inside rb_frequency_step (and the
 * sweep, the batch and the lossy step) the same form runs on the step's own operands: H and,
 * for the two angular components (Eq. sound_speed_update2's weight 1 + u_e . u_r), one
 * bilinear form a^T Rs b with a = H (u_x + i u_y), b = H (u_x - i u_y), which equals the sum
 * of their quadratic forms; the low parts are FP8 (E4M3) there, and b's enters the
 * contraction on FP8 matrix instructions. The operands passed through this header keep the
 * layout below. */
typedef enum { RB_F32 = 1, RB_BF16 = 2, RB_F16 = 3, RB_F16X = 4 } rb_prec;

/* Predicted data of the frequency step: ray Green's function at the receivers plus, in
 * RB_RAY_BORN mode, the first-order Born term of the part of the model removed by the
 * smoothing window (m - m_s); RB_RAY_ONLY omits that term. */
typedef enum { RB_RAY_BORN = 0, RB_RAY_ONLY = 1 } rb_mode;

/* Absorbing, dispersive medium (Section 2.2, Szabo's model): the complex wavenumber is
 * k~ = omega/c + alpha0 omega^y [tan(pi y/2) + i] (Eq. szabo_dispersion_equation), with the
 * power-law absorption alpha = alpha0 omega^y and the real part k = omega/c + alpha0
 * tan(pi y/2) omega^y = omega / c_p(omega) (Eq. wave-number). alpha0: DEVICE double [ny][nx]
 * in Np (rad/s)^-y m^-1 (>= 0; 0 in water); y: exponent in (0, 2], at least 1e-3 from 1
 * (soft tissue: 1 < y <= 1.5). The alpha0 map is a known property of the medium, not an
 * unknown: the steps update c only. */
typedef struct {
    const double *alpha0;
    double y;
} rb_absorption;

/* Ring of n point transducers of radius `radius` (Section 2.1); each emits and receives. */
typedef struct {
    int32_t n;
    double radius;
    double psi0;
} rb_ring;

/* Square-spaced Cartesian grid and circular imaging mask (Section 6.3: 90 % of the ring). */
typedef struct {
    int32_t nx, ny;
    double dx, x0, y0;
    double mask_radius;
} rb_grid;

/* Fan of n_rays launch angles per transducer over the inward half-plane,
 * gamma0_j = psi_e + pi + (j + 1/2 - n_rays/2) pi / n_rays; Heun step ds (Algorithm 1);
 * a ray still inside the ring after max_steps steps makes the call fail (RB_ENONFINITE). */
typedef struct {
    int32_t n_rays;
    int32_t max_steps;
    double ds;
    double c0;
} rb_trace_params;

/* Per-transducer tables (outputs of rb_trace_rays, inputs of rb_build_green).
 * Grid tables over the mask nodes, row e = transducer, shape [n][n_mask]:
 *   T  travel time from transducer e (s);
 *   A  geometric amplitude times sqrt(k0): A_geom = A / sqrt(omega / c0);
 *   ux, uy unit direction of the ray from e at the node;
 *   flags bit 7 = valid, bits 0-1 = caustic count mod 4.
 * Receiver tables, row = emitter, column = receiver, shape [n][n]: rx_T, rx_A, rx_flags. */
typedef struct {
    int32_t n;
    int32_t n_mask;
    double *T;
    float *A;
    float *ux;
    float *uy;
    uint8_t *flags;
    double *rx_T;
    float *rx_A;
    uint8_t *rx_flags;
} rb_tables;

/* Green's-function operands of one frequency (output of rb_build_green):
 *   G  g(omega, x, e) = A exp(i (phi + pi/4))  (Eq. 2D_greens);
 *   H  back-projection operands a_e g_dagger, a_e g_dagger u_x, a_e g_dagger u_y
 *      (Eq. greens-time-reversed times the angular weight |d gamma_e / d e| De of
 *      Eq. sound_speed_update2).
 * Layout by precision:
 *   RB_F32:  G complex64 [n][n_mask];  H complex64 [3][n][n_mask].
 *   RB_BF16, RB_F16 (16-bit operands, FP32 accumulation in every contraction):
 *            G planar [2 (re, im)][n][m_pad], m_pad = n_mask rounded up to a multiple of
 *            32;  H planar, node-major [3][2 (re, im)][n_mask][n_pad] (transducer index
 *            contiguous), n_pad = n rounded up to a multiple of 32. rb_build_green writes
 *            zeros past n_mask in G and past n in H.
 *   RB_F16X: as RB_F16, with H followed by its low parts: [2 (hi, lo)][3][2][n_mask][n_pad].
 *            scales float [2][n]: per-transducer powers of two s_e (row e of G) and t_e
 *            (the rows of transducer e in H), chosen by rb_build_green from the largest
 *            amplitude of each row so that the row's largest value sits near 2^13 before it
 *            is rounded: the stored operands are s_e G[e] and t_e H[e]. The contractions
 *            divide the scales out exactly. A caller filling 16-bit operands itself sets
 *            them (ones: unscaled). Not used for RB_F32 (may be NULL). */
typedef struct {
    int32_t n;
    int32_t n_mask;
    rb_prec prec;
    void *G;
    void *H;
    float *scales;
} rb_green;

/* Status of one rb_frequency_step written to DEVICE memory by the step's last kernel, so
 * that the call needs no host synchronisation (graph capture, tight loops). */
typedef struct {
    int32_t status;       /* RB_OK, or RB_ENONFINITE when the step committed nothing */
    int32_t flags;        /* bit 0: a ray exceeded max_steps; bit 1: non-finite model update */
    int32_t lost_nodes;   /* mask nodes the binning walk could not place (0 normally) */
    int32_t reserved;
    int64_t ray_samples;  /* ray samples the tracer wrote */
} rb_report;

typedef struct rb_ctx rb_ctx;

/* Create a context on HIP device `device` that launches on `hip_stream` (a hipStream_t,
 * borrowed, may be NULL for the null stream). Returns RB_EDEVICE if the device is absent. */
rb_status rb_create(rb_ctx **ctx, int device, void *hip_stream);
/* Device bytes rb_reserve allocates for this geometry (workspace of every entry point with
 * operands of any precision, the frequency step's buffers for `prec`, the mask lists), with
 * ray samples of one tracer launch limited to sample_budget bytes (rb_set_sample_budget).
 * Host arithmetic only; 0 if the geometry is invalid. */
size_t rb_workspace_bytes(const rb_grid *grid, const rb_ring *ring, const rb_trace_params *tp,
                          rb_prec prec, size_t sample_budget);
/* Allocate, once, every device buffer the context's entry points need for this geometry
 * (rb_workspace_bytes with the context's sample budget) and fix it: afterwards no call
 * allocates, frees or synchronises for workspace; a call on another grid returns RB_EINVAL,
 * one needing more than the reservation (another ring, more rays, a frequency step of a
 * wider precision, a larger sample budget) RB_ENOMEM, both before launching anything.
 * Calling rb_reserve again replaces the reservation (it waits for the stream first). */
rb_status rb_reserve(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                     const rb_trace_params *tp, rb_prec prec);
/* Release the context's workspace. The caller's buffers are untouched. */
void rb_destroy(rb_ctx *ctx);
/* Message of the last error of this context (static storage inside the context). */
const char *rb_last_error(const rb_ctx *ctx);
/* Number of mask nodes of a grid (host arithmetic only; -1 if the grid is invalid). */
int64_t rb_mask_count(const rb_grid *grid);

/* Box-smoothed refractive index n_s = box_w(c0 / c) (Section 6.3.2: odd averaging window,
 * edges replicated) as float [ny][nx], from c (double [ny][nx]). w must be odd and >= 1. */
rb_status rb_refractive_index(rb_ctx *ctx, const rb_grid *grid, const double *c, double c0,
                              int32_t w, float *n_s);

/* Trace the fan of every transducer through the refractive-index map n_s (float [ny][nx],
 * the uniform cubic B-spline of these samples is the medium; Section 4.5) with the paraxial
 * Heun scheme of Algorithm 1, bin the rays onto the mask nodes by linear interpolation over
 * the triangulated ray samples (Section 4.5), and fill the receiver tables from the rays'
 * exit points (Section 6.3). Writes every field of `out` (sizes must match). Where several
 * triangles cover a node (a folded fan), the smallest travel time wins, ties to the lowest
 * triangle id. */
rb_status rb_trace_rays(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                        const rb_trace_params *tp, const float *n_s, const rb_tables *out);

/* Maps of one frequency omega in an absorbing medium, float [ny][nx] each:
 *   n_w = box_w(c0/c) + c0 tan(pi y/2) omega^(y-1) box_w(alpha0), the real wavenumber k of Eq.
 *         wave-number in units of k0 = omega/c0 (the map the rays of omega follow: with
 *         dispersion they differ between frequencies);
 *   a_w = omega^y box_w(alpha0), the absorption alpha (Np/m) the rays integrate.
 * box_w: the odd box window of rb_refractive_index, applied to both maps (the wavenumber map
 * is linear in them). With alpha0 = 0, n_w equals rb_refractive_index's n_s bit for bit. */
rb_status rb_lossy_maps(rb_ctx *ctx, const rb_grid *grid, const double *c,
                        const rb_absorption *abs, double c0, double omega, int32_t w,
                        float *n_w, float *a_w);

/* rb_trace_rays through the map n_w of an absorbing medium: the same rays, binning and
 * receivers, with the amplitude tables A and rx_A carrying the absorption along each ray,
 * A = A_geom sqrt(k0) A_abs, A_abs = exp(-int a_w ds) (Eq. amplitude-abs-discretised;
 * trapezoid rule at the ray samples on the cubic B-spline of a_w, value only). The tables then
 * belong to the frequency of n_w and a_w (rb_lossy_maps); rb_build_green and rb_residual take
 * them as they are. Receiver linking (rb_set_receiver_linking) applies as in rb_trace_rays. */
rb_status rb_trace_rays_lossy(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                              const rb_trace_params *tp, const float *n_w, const float *a_w,
                              const rb_tables *out);

/* Diagnostic of the last rb_trace_rays / rb_frequency_step on this context: the number of
 * (transducer, mask node) pairs that the mesh walk of an unfolded fan could not place in a
 * triangle (reported as invalid table entries). Zero in normal operation. */
int64_t rb_trace_lost_nodes(const rb_ctx *ctx);

/* Diagnostic of the last rb_trace_rays / rb_frequency_step on this context: the number of ray
 * samples the tracer wrote (source samples included), summed over all rays that reached the
 * ring; the unit of the tracer's work. -1 for a null context. */
int64_t rb_trace_samples(const rb_ctx *ctx);

/* Assemble G and the back-projection operands H of angular frequency omega from the tables
 * (Eqs. 2D_greens, phase-discretised, greens-time-reversed). The phase omega T + pi/4 -
 * K pi/2 is reduced modulo 2 pi in FP64. Invalid table entries give zeros. */
rb_status rb_build_green(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                         const rb_green *out);

/* Born forward operator (Eqs. perturb1, derivative): d[e][r] = sum_q G[e][q] w[q] delta[q]
 * G[r][q] for all (e, r) including e = r. w: complex64 [n_mask] (Upsilon h^2, e.g.
 * omega^2 dx^2 for dm = delta m); delta: float [n_mask]; d: complex64 [n][n]. w and delta
 * may both be NULL: then w delta = 1, for operands that already carry sqrt(w delta) (as G
 * does inside rb_frequency_step). */
rb_status rb_born_forward(rb_ctx *ctx, const rb_green *gr, const float *w, const float *delta,
                          float *d);

/* Adjoint of rb_born_forward for real delta (Eq. functional-gradient with Q = 1):
 * grad[q] = Re{ conj(w[q]) sum_e conj(G[e][q]) sum_r R[e][r] conj(G[r][q]) }.
 * R: complex64 [n][n]; w: complex64 [n_mask]; grad: float [n_mask]. With 16-bit operands
 * (RB_BF16, RB_F16) G is first transposed (node-major, conjugated) in the workspace and R is
 * rounded to the operand type with a power-of-two range scale; every product accumulates in
 * FP32. Only the symmetric part of R enters (the double sum is a bilinear form in conj(G)). */
rb_status rb_born_adjoint(rb_ctx *ctx, const rb_green *gr, const float *w, const float *R,
                          float *grad);

/* Residual of one frequency (Eq. residual): R[e][r] = g(omega, r, e) + d_born[e][r] - data[e][r]
 * on valid pairs with e != r, zero elsewhere, where g(omega, r, e) = rx_A / sqrt(k0)
 * exp(i (omega rx_T + pi/4 - K pi/2)) is the ray Green's function at the receivers.
 * d_born: complex64 [n][n] or NULL; data, R: complex64 [n][n]. */
rb_status rb_residual(rb_ctx *ctx, const rb_tables *tb, double omega, double c0,
                      const float *d_born, const float *data, float *R);

/* Hessian-free search direction of one frequency (Eqs. sound_speed_update,
 * sound_speed_update2): dm[q] = -S[q] Re sum_{e,r} R[e][r] [H_e H_r + H^x_e H^x_r +
 * H^y_e H^y_r](q), with S[q] = 2 d_omega / ((2 pi)^3 omega c[q]^2) (lossless, two-way
 * isochron gradient k (u_e + u_r)). c: double [n_mask] sound speed at the mask nodes;
 * dm: float [n_mask], overwritten unless `accumulate` != 0 (then added). */
rb_status rb_backproject(rb_ctx *ctx, const rb_green *gr, const float *R, const double *c_mask,
                         double omega, double d_omega, float *dm, int32_t accumulate);

/* rb_backproject in an absorbing medium (operands from lossy tables): the weight becomes
 * complex, S[q] = d_omega / (2 pi)^3 2 k dk/domega / Upsilon_m with the dispersive
 * k = omega/c + alpha0 tan(pi y/2) omega^y, dk/domega = 1/c + y tan(pi y/2) omega^(y-1)
 * alpha0 (Section 3.4) and Upsilon_m = omega c k~ (Eq. scattering-potential), at the node's
 * c and alpha0; dm[q] = -Re{ S[q] sum_{e,r} R[e][r] [H_e H_r + H^x_e H^x_r + H^y_e H^y_r](q) }.
 * alpha0_mask: double [n_mask] (alpha0 at the mask nodes); y as in rb_absorption. */
rb_status rb_backproject_lossy(rb_ctx *ctx, const rb_green *gr, const float *R,
                               const double *c_mask, const double *alpha0_mask, double y,
                               double omega, double d_omega, float *dm, int32_t accumulate);

/* rb_backproject without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, hosts that forbid it): the same kernels
 * and result, with the partial sums and the rounded residual in a fixed 64 MiB device array
 * of the library (one per GPU, held until the process ends) instead of the context's
 * workspace. The array's address on a device is taken at the first rb_create there. Sizes
 * whose scratch exceeds 64 MiB (about 2 (n/256 + 1) n_mask 4 + 12 n^2 bytes; n = 1024 with
 * 636 160 mask nodes takes 33 MB) return RB_EINVAL before any launch. Every call on one GPU
 * shares the array: calls that overlap on a GPU (different streams or contexts) race and
 * must be ordered by the caller. Nothing needs to be zero beforehand: every scratch word a
 * call reads it has written itself. */
rb_status rb_backproject_noalloc(rb_ctx *ctx, const rb_green *gr, const float *R,
                                 const double *c_mask, double omega, double d_omega, float *dm,
                                 int32_t accumulate);

/* One frequency step (the unit of the benchmark). c: double [ny][nx] sound speed, updated
 * in place on the mask nodes (m <- m + tau sum_omega dm_omega, c = m^-1/2, FP64); omega and
 * d_omega: HOST arrays of n_omega values; data: complex64 [n_omega][n][n] measured Green's
 * functions (row = emitter). smooth_w: odd window of the tracing map. If a ray exceeds
 * max_steps or any updated value is not finite the model is left unchanged.
 * residual_norm (device double, may be NULL) receives sum |g_res|^2 over all frequencies.
 * prec selects the operand type of the Born contractions (RB_F32 plain form; RB_BF16 /
 * RB_F16 reduced form); tracing, phases and the model update are the same in all forms.
 * report == NULL: the call waits for the stream and returns RB_ENONFINITE for a step that
 * committed nothing. report != NULL (device rb_report): nothing waits for the stream; the
 * step's last kernel writes the status there and the call returns RB_OK once the step is
 * enqueued (argument errors are still returned before any launch). */
rb_status rb_frequency_step(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                            const rb_trace_params *tp, double *c, int32_t smooth_w,
                            int32_t n_omega, const double *omega, const double *d_omega,
                            const float *data, double tau, rb_mode mode, rb_prec prec,
                            double *residual_norm, rb_report *report);

/* rb_frequency_step in an absorbing, dispersive medium (abs: alpha0 map and exponent y; the
 * other arguments as in rb_frequency_step). Per frequency the rays are traced again on that
 * frequency's map (rb_lossy_maps, rb_trace_rays_lossy), so the Green's functions carry its
 * dispersion and A_abs; the Born term of the rough part uses w = Upsilon_m h^2 with the
 * complex Upsilon_m = omega c k~ of the model's c and alpha0 at the node (the rough part
 * m - m_s keeps m_s = (box_w(c0/c)/c0)^2), and the back-projection the complex weight of
 * rb_backproject_lossy. With alpha0 = 0 the step computes the lossless step's quantities.
 * rb_trace_lost_nodes / rb_trace_samples and the report's counters describe the last
 * frequency's trace. */
rb_status rb_frequency_step_lossy(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                                  const rb_trace_params *tp, double *c,
                                  const rb_absorption *abs, int32_t smooth_w, int32_t n_omega,
                                  const double *omega, const double *d_omega, const float *data,
                                  double tau, rb_mode mode, rb_prec prec,
                                  double *residual_norm, rb_report *report);

/* Green's functions of a Gauss-Newton step: traced rays (the Hessian-based ray-Born method of
 * Section 6.3.2 b) or water's, computed analytically (App. B; the prototype Born method of
 * Section 6.3.2 c, where the sound speed enters only the scattering potential). */
typedef enum { RB_GREEN_RAY = 0, RB_GREEN_WATER = 1 } rb_green_model;

/* One Gauss-Newton update of the frequency set (Section 6.3.2 b, c): the linearised
 * subproblem (Eq. linearised-linearised-subproblem, Q = 1) solved by n_inner conjugate-
 * gradient iterations on the Hessian action H x = Re sum_w J_w^H J_w x (Eq. hessian-action)
 * from x = 0 against -grad, grad = Re sum_w J_w^H g_res,w (Eq. functional-gradient), with
 * J_w the Born operator (Eqs. perturb1, derivative; w = omega^2 dx^2) on the pairs the
 * residual keeps (valid, e != r); then m <- m + tau x on the mask (tau = 1: the Gauss-Newton
 * step), c = m^-1/2, committed only if finite. The iteration stops early (keeps x) once
 * r.r = 0 or p.Hp <= 0. RB_GREEN_RAY: tables, Green's functions and predicted data as in
 * rb_frequency_step (rays on box_w(c0/c), smooth_w odd; the rough part m - m_s in the data);
 * RB_GREEN_WATER: T = |x - x_e| / c0, A = (8 pi |x - x_e|)^-1/2, predicted data
 * g0 + F0 (m - c0^-2); no rays are traced and smooth_w is ignored. prec as in
 * rb_frequency_step (16-bit operands with FP32 accumulation; RB_F16X behaves as RB_F16);
 * the CG vectors and scalars are FP64 on the device. omega: HOST [n_omega] (1..8); data:
 * complex64 [n_omega][n][n]; 1 <= n_inner <= 256. residual_norm (device double or NULL):
 * sum |g_res|^2 before the update; cg_norms (device double [n_inner + 1] or NULL): |r_k| of
 * the normal equations at each iterate. report: as in rb_frequency_step. The operands of
 * all n_omega frequencies stay resident during the iteration, in a workspace of their own
 * that rb_reserve does not cover (allocated on first use, grown when a call needs more). */
rb_status rb_gauss_newton_step(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                               const rb_trace_params *tp, double *c, int32_t smooth_w,
                               int32_t n_omega, const double *omega, const float *data,
                               double tau, int32_t n_inner, rb_green_model model, rb_prec prec,
                               double *residual_norm, double *cg_norms, rb_report *report);

/* Several frequency steps in a row: the frequency continuation of Section 6.3.2 (one step
 * per frequency set, sets ordered low to high by the caller). Step k uses smoothing window
 * smooth_w[k] and the next n_omega[k] entries of omega / d_omega (HOST arrays, sets
 * concatenated) with the matching [n][n] slices of data (complex64, one slice per frequency,
 * in the same order). No step synchronises with the host: a ray exceeding max_steps or a
 * non-finite update is recorded on the device, that step and every later one commit
 * nothing (c keeps the model from before the failing step), and the call returns
 * RB_ENONFINITE naming the step after the last kernel. residual_norms: device
 * double[n_steps] (per-step sum |g_res|^2) or NULL.
 * use_graph != 0: the whole sweep is captured into one HIP graph on a stream of the
 * library and replayed on the context's stream (one launch for all steps). The graph is
 * kept in the context and replayed while the arguments (pointer values included) and the
 * context's workspace are unchanged; otherwise it is captured again. The caller keeps c,
 * data and residual_norms valid between replays. Returns after the last kernel (the
 * host waits for the context's stream). */
rb_status rb_frequency_sweep(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring,
                             const rb_trace_params *tp, double *c, int32_t n_steps,
                             const int32_t *smooth_w, const int32_t *n_omega,
                             const double *omega, const double *d_omega, const float *data,
                             double tau, rb_mode mode, rb_prec prec, int32_t use_graph,
                             double *residual_norms);

/* One scan's step inside a batch: the arguments of rb_frequency_step for that scan. */
typedef struct {
    rb_ctx *ctx;                 /* the scan's context (its stream, workspace and mask) */
    const rb_grid *grid;         /* HOST structs, as in rb_frequency_step */
    const rb_ring *ring;
    const rb_trace_params *tp;
    double *c;                   /* device [ny][nx] model, updated in place */
    int32_t smooth_w;
    int32_t n_omega;
    const double *omega;         /* HOST [n_omega] */
    const double *d_omega;       /* HOST [n_omega] */
    const float *data;           /* device complex64 [n_omega][n][n] */
    double tau;
    rb_mode mode;
    double *residual_norm;       /* device double or NULL */
} rb_scan_step;

/* The frequency steps of `count` scans (1 <= count <= 16) at once: each scan's step is the
 * one rb_frequency_step computes for it (the same kernels on the same values, so results are
 * identical to the scan stepped alone). This is the serving form of the continuation
 * (Section 6.3.2) over several reconstructions: the per-scan stages (map, rays, binning,
 * Green's functions) of different scans run on their contexts' streams and overlap on the
 * device; for each frequency index k, the Born forward terms (Eq. perturb1) of all scans
 * with a k-th frequency run as one grouped launch, and so do their back-projections (Eq.
 * sound_speed_update2), on the stream of steps[0].ctx, ordered against the scans' streams by
 * events. Scans may differ in n, grid and frequency count. The contexts must be distinct and
 * on one device; prec applies to every scan. Returns after the last kernel of every scan
 * (the host waits). status (HOST rb_status[count], may be NULL) receives each scan's result:
 * a scan whose step fails (ray beyond max_steps, non-finite update) keeps its model and gets
 * RB_ENONFINITE (its context's rb_last_error says why) while the other scans commit; the
 * return value is the first non-OK status. Arguments are validated before any launch. */
rb_status rb_frequency_step_batch(const rb_scan_step *steps, int32_t count, rb_prec prec,
                                  rb_status *status);

/* Peak device bytes a context holds for frequency steps of this geometry and precision
 * (workspaces, tables, operands, mask lists), for a tracer sample budget of sample_budget
 * bytes (rb_set_sample_budget). For admission by memory; 0 if the geometry is invalid. */
size_t rb_step_bytes(const rb_grid *grid, const rb_ring *ring, const rb_trace_params *tp,
                     rb_prec prec, size_t sample_budget);

/* Receiver tables by ray linking (Sections 4 and 6.3: one ray per emitter-receiver pair,
 * its launch angle adjusted by the secant method until it crosses the ring at the
 * receiver). With max_iter > 0, every later rb_trace_rays and frequency step of this
 * context computes rx_T, rx_A and rx_flags from the linked ray's terminal sample instead of
 * interpolating the fan in exit angle. Per pair: starting points are the two fan rays of the
 * receiver's bracket; at most max_iter rays are traced, stopping once the exit angle is
 * within tol radians of the receiver's (0 < tol <= 1e-6); the traced ray closest to the
 * receiver is taken if within 1e-6 radians, else the pair is invalid. Pairs without a
 * bracket are invalid as before. max_iter = 0 returns to interpolation (the default).
 * RB_EINVAL for max_iter outside 0 .. 64 or tol outside (0, 1e-6]. */
rb_status rb_set_receiver_linking(rb_ctx *ctx, int32_t max_iter, double tol);

/* Bytes of ray samples one tracer launch of this context may hold (default: a quarter of the
 * device memory free at rb_create, at most 48 GiB). Emitters are traced in chunks that fit;
 * a smaller budget means more launches. RB_EINVAL below 1 MiB. */
rb_status rb_set_sample_budget(rb_ctx *ctx, size_t bytes);

/* Launch configuration of the Born forward contraction (Eq. perturb1) for one shape: the
 * workgroup tile (rows e x columns r of d) and the number of K chunks (mask nodes split over
 * workgroups, partial sums added in a fixed order). Applies to calls with n, n_mask and prec
 * equal to the record's and, for 16-bit operands, to operands that carry sqrt(v)
 * (rb_frequency_step, rb_frequency_sweep, rb_frequency_step_batch, rb_born_forward with
 * w = delta = NULL); FP32 calls with weights use it too. Other calls use a built-in rule. */
typedef enum { RB_TILE_256x128 = 0, RB_TILE_128x128 = 1 } rb_tile;
typedef struct {
    int32_t n, n_mask;
    rb_prec prec;
    rb_tile fwd_tile;      /* RB_TILE_256x128: pipelined 16-bit kernel; FP32 takes 128x128 */
    int32_t fwd_splitk;    /* K chunks, 1 .. 1024 */
    float fwd_ms;          /* rb_autotune: measured time of this configuration (ms) */
} rb_tuning;

/* Autotuner: times every candidate forward configuration (both tiles for 16-bit operands,
 * K splits from 8 to 64 and the built-in choice) on this context's device, on operands of
 * the shape of `grid`'s mask and `ring` (seeded values in the context's step workspace, so
 * nothing else is overwritten), keeps the fastest in the context and writes it to *out
 * (may be NULL). A context keeps up to 16 tunings, one per (n, n_mask, prec). Synchronizes
 * the context's stream. Results of the tuned and untuned launches differ only by the order
 * of the FP32 partial sums. */
rb_status rb_autotune(rb_ctx *ctx, const rb_grid *grid, const rb_ring *ring, rb_prec prec,
                      rb_tuning *out);
/* Install a tuning (e.g. one saved from rb_autotune), replacing the record of its shape;
 * NULL removes every tuning. RB_EINVAL for a configuration that is not valid for its
 * precision. rb_step_bytes covers K splits up to 64 (the autotuner's range); a larger one
 * set here takes more workspace. */
rb_status rb_set_tuning(rb_ctx *ctx, const rb_tuning *t);
/* The tuning of the shape given in out->n, out->n_mask, out->prec; RB_EINVAL if none. */
rb_status rb_get_tuning(const rb_ctx *ctx, rb_tuning *out);

/* Measurement: per-stage GPU time from HIP events recorded around every kernel launch on
 * the context's stream while profiling is on (small overhead; off by default). Stages are
 * numbered 0 .. RB_N_STAGES-1 (rb_stage_name). rb_profile_read synchronizes the stream,
 * writes for each stage the summed kernel time in milliseconds and the launch count, and
 * clears the record. */
#define RB_N_STAGES 12
rb_status rb_profile_enable(rb_ctx *ctx, int32_t on);
rb_status rb_profile_read(rb_ctx *ctx, double *total_ms, int64_t *launches);
const char *rb_stage_name(int32_t stage);

#ifdef __cplusplus
}
#endif
#endif /* RAYBORNHF_H */
