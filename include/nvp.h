/*
 * nvp — nested-mesh Helmholtz volume potentials on MI355X (gfx950).
 *
 * C ABI of the library that computes the higher harmonics p_2..p_n of the
 * weakly nonlinear (Westervelt) field of a focused-ultrasound source, each on
 * its own voxel grid, following Groth et al., "Accelerating frequency-domain
 * numerical methods for weakly nonlinear focused ultrasound using nested
 * meshes" (arXiv 2011.03009):
 *
 *   harmonic cascade  (Section 2, eq. cascade_2; Section 3, eqs. harm2-harm5)
 *       p_n = C_n * int_{D_n} G_{k_n}(x, y) f_n(y) dy,
 *       f_n = sum_{m=1}^{n-1} p_m p_{n-m},  C_n = -beta w^2 n^2 / (2 rho0 c0^4),
 *       k_n = n w / c0 + i alpha(n w)  (eq. power_law);
 *   quadrature        (Section 3.1, eq. quad): midpoint rule off the diagonal,
 *       equal-volume sphere on the self voxel; the Toeplitz operator is applied
 *       through a circulant embedding and 3-D FFTs;
 *   nested meshes     (Section 6): harmonic n on its own box and spacing; lower
 *       harmonics are interpolated onto the new mesh (step 2(a)).
 *
 * Conventions for every call:
 *   - Returns an nvp_status; never throws.  On failure the context's
 *     nvp_last_error() holds a message.
 *   - Field buffers are DEVICE pointers owned by the caller, C order [n0][n1][n2]
 *     (z fastest), complex interleaved re/im: complex64 for NVP_C64,
 *     complex128 for NVP_C128.
 *   - execute* calls only enqueue work on the context's stream and return;
 *     asynchronous faults surface at nvp_ctx_sync().
 *   - Contexts and plans are owned by the library and released only by their
 *     _destroy call.  A plan is bound to its context's device and stream.
 *   - A context outlives the plans, batches and networks made with it:
 *     nvp_ctx_destroy fails with NVP_E_STATE, and frees nothing, while any
 *     of them has not been destroyed.
 */
#ifndef NVP_H
#define NVP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nvp_status;
#define NVP_OK 0
#define NVP_E_INVALID 1     /* bad argument: null pointer, h <= 0, n < 1, bad precision, ... */
#define NVP_E_NOMEM 2       /* device or host allocation failed; no partial state kept */
#define NVP_E_HIP 3         /* a HIP runtime call or kernel launch failed */
#define NVP_E_UNSUPPORTED 4 /* valid request outside what the library handles: an axis beyond 4096 voxels, a grid beyond a fixed scratch, a transfer order other than 1 or 3, the source kernel for grids only the fused path takes */
#define NVP_E_STATE 5       /* call out of order (e.g. timing read while disabled) */
/* Fault injection for tests: with the environment variable
 * NVP_DEVICE_ALLOC_LIMIT set to a byte count, every device allocation of the
 * runtime (plans, batches, the volume-potential cache, twiddle tables, the
 * autotuner's scratch) larger than that fails as out of memory; calls then
 * return NVP_E_NOMEM and keep no partial state. */

typedef enum { NVP_C64 = 0, NVP_C128 = 1 } nvp_prec;

/* Medium (Section 2; medium table of Section 3.2).  alpha0_db is the
 * attenuation in dB/m at 1 MHz and eta its frequency exponent, so that
 * alpha(f) = alpha0_db (f / 1 MHz)^eta / (20 log10 e) Np/m. */
typedef struct {
    double c0, rho0, beta, alpha0_db, eta;
} nvp_medium;

/* Uniform voxel grid: centre(i, j, k) = origin + (i, j, k) h. */
typedef struct {
    double origin[3];
    double h;
    int64_t n[3];
} nvp_grid;

typedef struct nvp_ctx nvp_ctx;
typedef struct nvp_plan nvp_plan;

/* ---- status and context ------------------------------------------------ */

const char *nvp_status_str(nvp_status s);
/* Last error message of a context (empty string if none); ctx may be NULL
 * for errors of nvp_ctx_create. */
const char *nvp_last_error(const nvp_ctx *ctx);

/* device: HIP device ordinal; hip_stream: a hipStream_t (NULL = the null
 * stream) on which all work of this context is enqueued. */
nvp_status nvp_ctx_create(int device, void *hip_stream, nvp_ctx **out);
nvp_status nvp_ctx_destroy(nvp_ctx *ctx);
/* Waits for the context's stream; reports asynchronous HIP errors. */
nvp_status nvp_ctx_sync(nvp_ctx *ctx);

/* ---- quadrature rule ------------------------------------------------------ */

/* The rule by which the volume potential is discretised (Section 3.1).
 * NVP_QUAD_BALL, the default, is the paper's equation "quad": the midpoint
 * rule on every other voxel, the integral over the equal-volume ball on the
 * target's own.  NVP_QUAD_CORRECTED is the higher-order rule that the paper
 * leaves open there: the midpoint sum over the other voxels with the error of
 * G's singularity removed by weights on the target voxel and its six face
 * neighbours (a corrected trapezoidal rule for singular integrands, with the
 * Epstein zeta values of the cubic lattice Z(1/2), Z(-1/2)):
 *   K(0)        = h^2 (Z(-1/2) - Z(1/2)) / (4 pi) + i k h^3 / (4 pi) + k^2 h^4 Z(-1/2) / (8 pi),
 *   K(face) adds  -h^2 Z(-1/2) / (24 pi)  to the midpoint value h^3 G(h).
 * It costs nothing extra: the operator stays a convolution. */
#define NVP_QUAD_BALL 0
#define NVP_QUAD_CORRECTED 1
/* Rule of every volume potential, box potential, VIE solve and plan made
 * with this context from now on (a plan keeps the rule it was made with).
 * NVP_E_INVALID for another value. */
nvp_status nvp_ctx_set_quadrature(nvp_ctx *ctx, int rule);
/* Host only: w[0] + i w[1] = the self-voxel value K(0) of `rule`, w[2] + i
 * w[3] = what the rule adds at the six face neighbours (0 for the ball rule).
 * NVP_E_INVALID for a bad rule, k = 0, non-finite k or h <= 0. */
nvp_status nvp_quadrature_weights(int rule, double k_re, double k_im, double h, double w[4]);

/* ---- constants and grids (host only) ------------------------------------ */

/* k_n = 2 pi n f0 / c0 + i alpha(n f0)  (Section 2, eq. power_law with n w). */
nvp_status nvp_wavenumber(const nvp_medium *med, double f0, int n, double *k_re, double *k_im);
/* C_n = -beta (2 pi f0)^2 n^2 / (2 rho0 c0^4)  (eqs. cascade_2 and harm2-harm5). */
nvp_status nvp_cascade_constant(const nvp_medium *med, double f0, int n, double *c);
/* delta x = c0 / (n f0 n_w): n_w voxels per own wavelength (Section 3.3 uses 6). */
nvp_status nvp_spacing(const nvp_medium *med, double f0, int n, int n_w, double *h);
/* Grid with n[a] voxels per axis whose voxel i_f[a] is centred on focus[a]. */
nvp_status nvp_grid_from_counts(const double focus[3], double h, const int64_t n[3],
                                const int64_t i_f[3], nvp_grid *out);
/* Grid covering the cuboid [lo, hi] at spacing h with the focus on a voxel
 * centre: n = max(1, floor((hi - lo)/h + 1/2)), i_f = floor((focus - lo)/h + 1/2).
 * i_f_out may be NULL. */
nvp_status nvp_grid_from_box(const double focus[3], const double lo[3], const double hi[3],
                             double h, nvp_grid *out, int64_t i_f_out[3]);
/* Box D_n of the paper's rule of thumb (Section 5): D_2 = [l - L, l + d] x [-R, R]^2
 * with L = sqrt(l^2 - R^2) - eps (eq. domain); for n > 2 the pre-focal length
 * and the width are scaled by lambda_n / lambda_2 = 2 / n, d is kept. */
nvp_status nvp_rule_of_thumb_box(int n, double l, double R, double d, double eps,
                                 double lo[3], double hi[3]);
/* Transfer table of one axis (Section 6, step 2(a)): for target centres
 * dst_origin + i dst_h, i < dst_n, the first source index base[i] and the
 * order + 1 weights w[i*(order+1) + j] of source nodes base[i] + j, for a
 * source axis src_origin + j src_h, j < src_n.  Targets are clamped into the
 * source hull; order 1: linear (the paper's choice), order 3: four-point
 * Lagrange with the stencil shifted inward at the edges.  Host buffers.
 * NVP_E_INVALID if src_n < order + 1. */
nvp_status nvp_transfer_axis(double dst_origin, double dst_h, int64_t dst_n, double src_origin, double src_h,
                             int64_t src_n, int order, int32_t *base, double *w);
/* Circulant length used for an axis of n voxels: the smallest compiled
 * transform length M >= 2 n - 1 (the embedding of Section 3.1 is exact for any
 * such M).  The compiled lengths are 2,3,5,7-smooth multiples of 8 from 16
 * to 8192 (nvp_transform_lengths), spaced so that from n = 128 on M exceeds
 * 2 n - 1 by less than 12.5%.  NVP_E_UNSUPPORTED for n > 4096. */
nvp_status nvp_circulant_size(int64_t n, int64_t *m);
/* The compiled transform lengths in increasing order: *count receives how
 * many there are, and the first min(count, capacity) go to lengths (host). */
nvp_status nvp_transform_lengths(int32_t *lengths, int capacity, int *count);

/* ---- the incident field ---------------------------------------------------- */

/* The incident (first-harmonic) field of a transducer modelled as n_points
 * equal-weight point sources on its surface (Section 3.2, incident-field
 * equation), at the voxel centres x_i = origin + (ix, iy, iz) h of grid g:
 *   out[i] = (s_re + i s_im) * sum_j exp(i k r_ij) / (4 pi r_ij),  r_ij = |x_i - p_j|,
 * k = k_re + i k_im with k_im >= 0 (outgoing, decaying waves).  The caller
 * folds the weights and the source strength into the scale s (a bowl of area
 * A with surface pressure p0: s = -2 i k p0 A / n_points).
 *   points_dev: n_points x 3 doubles (x, y, z), device memory, caller-owned;
 *   out_dev: g->n[0]*g->n[1]*g->n[2] complex values [Nx][Ny][Nz] in prec,
 *            device memory, caller-owned, written in full.
 * complex64: distances, phases and the phase reduction in FP64, sine and
 * cosine of the reduced phase, decay and 1/r in FP32, sums in FP64 (relative
 * L2 error ~6e-8 at the paper's scale); complex128: FP64 throughout.  A voxel centre on a point (r = 0) receives a non-finite value.
 * Enqueued on the context stream.  NVP_E_INVALID: null pointers,
 * n_points < 1, a bad grid or precision, non-finite k or s, k_im < 0. */
nvp_status nvp_incident_field(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im,
                              const double *points_dev, int64_t n_points, const nvp_grid *g, void *out_dev,
                              nvp_prec prec);

/* The same sum at n_targets arbitrary points: targets_dev n_targets x 3
 * doubles (device, caller-owned); out_dev n_targets complex values in prec. */
nvp_status nvp_incident_at(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im,
                           const double *points_dev, int64_t n_points, const double *targets_dev,
                           int64_t n_targets, void *out_dev, nvp_prec prec);
/* Power radiated through the disc of the given radius centred at centre[3]
 * in the plane x = centre[0] (the transducer axis is the x axis), for the
 * field of nvp_incident_field with the same k, scale and points (Section 3.2,
 * the radiated-power integral over a disc covering the open end of a bowl):
 *   power = 1/(2 rho0 c0) * int_0^{2 pi} int_0^radius |p(r, theta)|^2 r dr dtheta,
 * by the midpoint rule with n_r x n_theta nodes (1..4096 each), the field
 * evaluated in complex128.  The paper's normalisation to a prescribed power
 * P0 multiplies the scale by sqrt(P0 / power).  Synchronous: waits for the
 * context stream; allocates n_r * n_theta * 40 bytes of device scratch for
 * the call.  NVP_E_INVALID for bad arguments as nvp_incident_field and for
 * non-positive radius, rho0 or c0. */
nvp_status nvp_radiated_power(nvp_ctx *ctx, double k_re, double k_im, double s_re, double s_im,
                              const double *points_dev, int64_t n_points, const double centre[3], double radius,
                              double rho0, double c0, int n_r, int n_theta, double *power);

/* ---- the raw operator ---------------------------------------------------- */

/* u = -sum_j K(x_i - x_j) f_j on grid g (eqs. vol_pot_approx and quad), any
 * complex wavenumber k with Im k >= 0, K of the context's quadrature rule.
 * f_dev and u_dev are device buffers of g->n[0]*g->n[1]*g->n[2] complex
 * elements (may not alias).  The context keeps the kernel spectrum of the
 * last (rule, k, g, prec) for reuse. */
nvp_status nvp_volume_potential(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g,
                                const void *f_dev, void *u_dev, nvp_prec prec);


/* The volume potential of a source restricted to a box, scaled:
 *   u_i = scale * sum_{j in box} K(x_i - x_j) f_j   at every voxel i of g,
 * K as in nvp_volume_potential (which is the case box = NULL, scale = -1).
 * With scale = C_n this is p_n computed from the source f_n cut to an
 * integration domain D (the truncated potentials of the domain study of
 * Section 5, evaluated on the whole grid).  box: host, 6 int64 = inclusive
 * voxel indices lo_x, lo_y, lo_z, hi_x, hi_y, hi_z inside the grid, or NULL
 * for the whole grid.  Shares the context's kernel-spectrum cache with
 * nvp_volume_potential.  NVP_E_INVALID: bad arguments, an empty box or one
 * reaching outside the grid. */
nvp_status nvp_volume_potential_box(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g,
                                    const void *f_dev, const int64_t *box, double scale, void *u_dev,
                                    nvp_prec prec);

/* Field arithmetic of the drivers built on the operator (the fixed-point
 * sweeps of the full cascade, iterative solvers), on n complex values in
 * prec, device buffers:
 *   nvp_field_lin3:       out = a + al b + be c  (al, be complex: {re, im});
 *                         a null a, b or c counts as zero; out may alias any
 *                         operand.  Enqueued on the context stream.
 *   nvp_field_diff_norms: out[0] = sum |a - b|^2, out[1] = sum |a|^2,
 *                         accumulated in FP64; waits for the result. */
nvp_status nvp_field_lin3(nvp_ctx *ctx, int64_t n, void *out_dev, const void *a_dev, const void *b_dev,
                          const void *c_dev, const double al[2], const double be[2], nvp_prec prec);
nvp_status nvp_field_diff_norms(nvp_ctx *ctx, int64_t n, const void *a_dev, const void *b_dev, nvp_prec prec,
                                double out[2]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operator and arguments as nvp_volume_potential, computed with the same
 * kernels, but with every work buffer (the kernel-spectrum octant and the two
 * pass buffers) inside one fixed device array of NVP_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device it runs on until the process ends.
 * The call allocates nothing and keeps no cache: the kernel spectrum is made
 * again on every call.  Grids whose buffers exceed the array are refused with
 * NVP_E_UNSUPPORTED (the message gives both sizes); complex64 cubes up to
 * 128^3 voxels fit, complex128 cubes up to 96^3 (the exact limit follows
 * from the circulant lengths, nvp_circulant_size).  Every call on one GPU
 * shares that GPU's array, so calls that may overlap on one GPU (other
 * streams, other contexts, other threads) race; calls on one stream run in
 * turn.  Each call writes every scratch byte before reading it.  The transform
 * tables come from the context (made at nvp_ctx_create).  Enqueued on the
 * context stream; errors as nvp_volume_potential. */
#define NVP_NOALLOC_SCRATCH_BYTES (128u << 20)
nvp_status nvp_volume_potential_noalloc(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g,
                                        const void *f_dev, void *u_dev, nvp_prec prec);

/* Volume integral equation of an inhomogeneous medium (Section 7, the
 * equations of the harmonics in an inhomogeneous domain): with background
 * wavenumber kb (Im kb >= 0) and contrast q_j = k(x_j)^2 - kb^2 per voxel,
 *   p_i - sum_j K_kb(x_i - x_j) q_j p_j = rhs_i   on grid g,
 * K the midpoint-rule kernel of nvp_volume_potential.  Solved by BiCGStab
 * with that operator: p_dev holds the initial guess on entry and the solution
 * on return; stops when the recursive residual falls to tol * ||rhs|| or after
 * max_iter iterations.  *iters receives the iterations taken and *relres the
 * true relative residual ||rhs - A p|| / ||rhs|| of the returned p (check it:
 * reaching max_iter is not an error).  q_dev, rhs_dev, p_dev: N complex values
 * in prec (device, caller-owned; p may not alias q or rhs).  Synchronous:
 * the recurrence's scalars stay on the device and each iteration waits once
 * for the context stream, to read the residual norm.  Allocates 8 N complex
 * values for the call; uses the context's volume-potential cache.
 * NVP_E_INVALID: bad arguments; NVP_E_STATE: a breakdown of the recurrence. */
nvp_status nvp_vie_solve(nvp_ctx *ctx, double kb_re, double kb_im, const nvp_grid *g, const void *q_dev,
                         const void *rhs_dev, void *p_dev, nvp_prec prec, double tol, int max_iter, int *iters,
                         double *relres);

/* Difference-frequency term of the full harmonic cascade (Section 2, the
 * products 2 p_m conj(p_{m-n}), m > n, of equation cascade_1 that equation
 * cascade_2 drops): out += scale * T_a(a) * conj(T_b(b)) at the centres of
 * grid gt.  T_x interpolates field x from its grid g_x with the cascade's
 * transfer of order `order` (1 or 3; see nvp_transfer_axis); zero_x != 0
 * makes it zero at targets outside the hull of g_x's voxel centres (more than
 * 1e-9 source voxels beyond it on some axis), as for a higher harmonic that
 * vanishes outside its own box; a field on gt itself is used as is.  Sums in
 * FP64.  out_dev, a_dev, b_dev: device, complex in prec, C order of their own
 * grids; out may not alias a or b.  Waits for the result (the stencil tables
 * it allocates are freed on return).  NVP_E_INVALID for bad arguments or a
 * source axis shorter than order + 1. */
nvp_status nvp_difference_term(nvp_ctx *ctx, const nvp_grid *gt, void *out_dev, const nvp_grid *ga,
                               const void *a_dev, int zero_a, const nvp_grid *gb, const void *b_dev, int zero_b,
                               int order, double scale, nvp_prec prec);

/* ---- the nested-mesh cascade (Section 6) ----------------------------------- */

/* Plan harmonics 2..n_harm.  g1: grid of the incident field p_1 (Section 3.2);
 * gn[0..n_harm-2]: grids of p_2..p_n_harm.  transfer_order: 1 = trilinear
 * (the paper's choice), 3 = tricubic Lagrange (the higher-order option the
 * paper recommends); target centres are clamped into the source grid's hull,
 * and a field on the very grid it is needed on is used as is.  Every axis
 * of a source grid needs at least transfer_order + 1 voxels, and every axis
 * a circulant length (nvp_circulant_size; up to 4096 voxels per axis).
 * The plan discretises with the context's quadrature rule at creation. */
nvp_status nvp_plan_cascade(nvp_ctx *ctx, const nvp_medium *med, double f0, int n_harm,
                            const nvp_grid *g1, const nvp_grid *gn, nvp_prec prec,
                            int transfer_order, nvp_plan **out);
/* Replaces the grid of harmonic n (2 <= n <= n_harm) of a plan with g, as if
 * the plan had been made with it: the transfer tables of every harmonic are
 * laid out again (later harmonics transfer from harmonic n), harmonic n's
 * kernel spectrum and launch choices start afresh, and the other harmonics
 * keep their kernel spectra.  Device memory is reused where it is large
 * enough and grown where not.  Waits for the plan's queued work.  For the
 * guarded runs of predicted truncation boxes, whose fallback replaces one
 * harmonic's box with the full one.  NVP_E_INVALID: a bad n or grid, a source
 * axis shorter than the transfer stencil, or a caller workspace too small
 * for the new grid (the plan then unchanged); NVP_E_NOMEM: allocation failed
 * (the plan unchanged). */
nvp_status nvp_plan_regrid(nvp_plan *plan, int n, const nvp_grid *g);
/* Device bytes held by the plan: its tables and kernel spectra, plus its own
 * work buffers unless a caller workspace replaces them. */
nvp_status nvp_plan_workspace_bytes(const nvp_plan *plan, size_t *bytes);
/* Size of the plan's transient work buffers (the two pass buffers and the
 * scratch of the overlapped kernel spectra): the least workspace that
 * nvp_plan_set_workspace accepts. */
nvp_status nvp_plan_work_bytes(const nvp_plan *plan, size_t *bytes);
/* Caller-owned work buffers.  dev: device memory on the context's device,
 * 256-byte aligned, of bytes >= nvp_plan_work_bytes; the plan waits for its
 * queued work, frees its own work buffers and from then on runs in
 * [dev, dev + bytes).  The caller keeps that memory alive, and free of other
 * use while the plan's work may run, until nvp_plan_destroy or the next call.
 * Plans that share one workspace must not run concurrently.  dev null: the
 * plan allocates work buffers of its own again.  Tables and kernel spectra
 * stay plan-owned.  NVP_E_INVALID for a short or misaligned workspace (the
 * plan unchanged); NVP_E_NOMEM if dev is null and the allocation fails (the
 * plan then has no work buffers and its executions return NVP_E_STATE). */
nvp_status nvp_plan_set_workspace(nvp_plan *plan, void *dev, size_t bytes);
/* 1 (default): keep each harmonic's kernel spectrum after its first use;
 * 0: tabulate and transform the kernel again on every execution. */
nvp_status nvp_plan_set_kernel_cache(nvp_plan *plan, int enable);
/* 1 (default): nvp_execute_cascade computes the kernel spectra it needs on a
 * second stream of the plan, each from the moment the context stream reaches
 * its harmonic (after all earlier work there), concurrently with that
 * harmonic's source build and forward x and y passes; the z pass waits for
 * it.  The second stream uses scratch of its own.  0: spectra computed in line.  Ignored while timing is on and while
 * the context stream is being captured into a graph; off for the plans of a
 * batch.  Results are the same either way. */
nvp_status nvp_plan_set_overlap(nvp_plan *plan, int enable);
/* One harmonic: fields[m-1] = p_m on its grid for m = 1..n-1; writes p_n. */
nvp_status nvp_execute_harmonic(nvp_plan *plan, int n, const void *const *fields, void *pn_dev);
/* The whole cascade: p1 in, pn_dev[i] = p_{i+2} out, computed in order. */
nvp_status nvp_execute_cascade(nvp_plan *plan, const void *p1_dev, void *const *pn_dev);
nvp_status nvp_plan_destroy(nvp_plan *plan);

/* The source term of harmonic n (eqs. harm2-harm5: f_n = sum over m of
 * p_m p_{n-m}, no conjugates) on the plan's grid of harmonic n, with the
 * fields transferred exactly as nvp_execute_harmonic does: fields[m-1] = p_m
 * on its plan grid for m = 1..n-1; f_dev receives N_n complex elements in the
 * grid's [Nx][Ny][Nz] layout.  Enqueued on the context stream.
 * NVP_E_UNSUPPORTED when this grid pair takes the fused source path only. */
nvp_status nvp_source_term(nvp_plan *plan, int n, const void *const *fields, void *f_dev);

/* ---- truncation boxes (Section 5) ------------------------------------------ */

#define NVP_QBOX_MAX_COUNT 32

/* Localisation boxes of a source term by the measure Q(x) = log10(|f(x)| /
 * max |f|) of Section 5: for each threshold q0[i] <= 0 (i < count <= 32), the
 * smallest voxel box outside which Q < q0[i], written as box[6i .. 6i+5] =
 * lo_x, lo_y, lo_z, hi_x, hi_y, hi_z (inclusive voxel indices).  A voxel is
 * inside when |f|^2 >= 10^(2 q0) max |f|^2, evaluated in FP64 (the power by
 * the C library's pow); an all-zero f gives the whole grid.  f_dev: device,
 * n[0] n[1] n[2] complex elements, [Nx][Ny][Nz]; q0, box: host.  Waits for
 * the result. */
nvp_status nvp_qbox(nvp_ctx *ctx, const int64_t n[3], const void *f_dev, nvp_prec prec, int count,
                    const double *q0, int64_t *box);

/* Truncated potentials at one voxel (the sums of eq. quad restricted to
 * boxes, for the truncation-convergence sweeps of Section 5): out[2i] + i
 * out[2i+1] = -sum over voxels j inside box i of K(x_t - x_j) f_j, with the
 * kernel of Section 3.1 for wavenumber k under the context's quadrature
 * rule, FP64 kernel and accumulation.  t: target voxel index on g; box:
 * host, count * 6 int64 as in nvp_qbox, each non-empty box inside the grid
 * (a box with hi < lo on an axis is empty and sums to 0); out: host, 2 count
 * doubles.  count <= 32.  Waits for the result. */
nvp_status nvp_box_potential(nvp_ctx *ctx, double k_re, double k_im, const nvp_grid *g, const void *f_dev,
                             nvp_prec prec, const int64_t t[3], int count, const int64_t *box, double *out);

/* ---- learned box predictor ------------------------------------------------- */

/* A 5-64-64-64-3 tanh MLP in FP32 that maps a transducer and harmonic
 * (aperture, focal length, frequency, source pressure, harmonic index) to the
 * three box fractions of that harmonic's truncation box (the paper's
 * fractions of the reference domain, Section 5 and its domain table; the
 * paper itself chooses boxes by a rule of thumb instead).  Inputs are
 * standardised by (x - mean) / std inside the forward pass.  Parameters
 * (float, row-major W[out][in]): W1[64][5] b1[64] W2[64][64] b2[64]
 * W3[64][64] b3[64] W4[3][64] b4[3].  Training minimises the pinball loss of
 * quantile tau averaged over the batch and the outputs,
 * L = (1 / 3B) sum rho_tau(t - y), rho_tau(u) = u (tau - [u < 0]), with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).  All x, y, t, grad buffers are device
 * arrays in sample-major layout ([B][5], [B][3], [B][3], [8899]). */
#define NVP_BOXNET_IN 5
#define NVP_BOXNET_OUT 3
#define NVP_BOXNET_PARAMS 8899
#define NVP_BOXNET_MAX_BATCH 65536
#define NVP_BOXNET_BETA1 0.9f
#define NVP_BOXNET_BETA2 0.999f
#define NVP_BOXNET_EPS 1e-8f

typedef struct nvp_boxnet nvp_boxnet;

/* Network for batches of up to max_batch samples; parameters and Adam state
 * zero, mean 0 and std 1.  Owned by the caller until nvp_boxnet_destroy. */
nvp_status nvp_boxnet_create(nvp_ctx *ctx, int max_batch, nvp_boxnet **out);
/* Host copy in/out of the NVP_BOXNET_PARAMS parameters (n must equal it);
 * setting them also clears the Adam moments and step count.  Both wait. */
nvp_status nvp_boxnet_set_params(nvp_boxnet *bn, const float *params, int64_t n);
nvp_status nvp_boxnet_get_params(nvp_boxnet *bn, float *params, int64_t n);
/* Input standardisation (host arrays of 5; std > 0). */
nvp_status nvp_boxnet_set_norm(nvp_boxnet *bn, const float *mean, const float *stdev);
/* y = net(x) for batch samples; enqueued on the context stream. */
nvp_status nvp_boxnet_predict(nvp_boxnet *bn, int batch, const float *x_dev, float *y_dev);
/* grad_dev = dL/dparams for targets t_dev, 0 < tau < 1, without updating the
 * parameters; loss_host (optional) receives L and makes the call wait.
 * Weight gradients are summed over the batch in sample order (no atomics),
 * so repeated calls give identical bits. */
nvp_status nvp_boxnet_grads(nvp_boxnet *bn, int batch, const float *x_dev, const float *t_dev, float tau,
                            float *grad_dev, float *loss_host);
/* One Adam step of learning rate lr on the batch; loss_host (optional)
 * receives the loss before the step and makes the call wait. */
nvp_status nvp_boxnet_train_step(nvp_boxnet *bn, int batch, const float *x_dev, const float *t_dev, float tau,
                                 float lr, float *loss_host);
nvp_status nvp_boxnet_destroy(nvp_boxnet *bn);

/* ---- autotuning and batches ------------------------------------------------ */

/* Times the launch choices of every harmonic of the plan and keeps the
 * fastest: the column tile of the x and the y passes (default or half), the
 * pencil quads per z-pass workgroup (1 or 2), the source build (its own
 * kernel or fused into the x pass) and, with its own kernel, the target x
 * planes per source workgroup (the default, or chunks for about half or
 * twice as many workgroups).  Each choice is timed over reps
 * executions on zero-filled fields (the kernels have no data-dependent
 * control flow).  cache_path (optional): a text file of earlier choices,
 * keyed by device, precision, transfer order and shapes; entries found there
 * are used without timing, new ones are written back.  Waits for the device.
 * Results of a tuned plan differ from the default only by the rounding order
 * of the source build. */
nvp_status nvp_plan_autotune(nvp_plan *plan, const char *cache_path, int reps);
/* The launch choices of harmonic n: choice[5] = x tile, y tile (0 default,
 * 1 half), z quads (0 default, 1, 2), source (-1 default, 1 its own kernel,
 * 0 fused into the x pass), source x chunk (0 default, else 1..64 target x
 * planes per workgroup of the source kernel). */
nvp_status nvp_plan_get_tuning(const nvp_plan *plan, int n, int *choice);
/* Sets the launch choices of harmonic n (choice[5], as above), e.g. ones
 * found by nvp_plan_autotune in an earlier process.  NVP_E_INVALID for a
 * choice out of range; NVP_E_UNSUPPORTED for the source kernel (1) where the
 * plan's grids take the fused path only.  Results differ from the default's
 * only by the rounding order of the source build. */
nvp_status nvp_plan_set_tuning(nvp_plan *plan, int n, const int *choice);

/* One problem of a batch: the arguments of nvp_plan_cascade. */
typedef struct {
    nvp_medium med;
    double f0;
    int n_harm;
    nvp_grid g1;
    const nvp_grid *gn; /* n_harm - 1 grids, read during nvp_batch_create only */
} nvp_problem;

typedef struct nvp_batch nvp_batch;

/* Many cascades (e.g. one per transducer) planned together.  Outputs are
 * numbered problem by problem: problem i writes p_2..p_{n_harm} to output
 * slots off_i .. off_i + n_harm - 2, off_i = sum over earlier problems of
 * (n_harm - 1); nvp_batch_outputs gives the total.  Each problem keeps its
 * own plan (workspace and kernel spectra). */
nvp_status nvp_batch_create(nvp_ctx *ctx, int count, const nvp_problem *problems, nvp_prec prec,
                            int transfer_order, nvp_batch **out);
nvp_status nvp_batch_outputs(const nvp_batch *batch, int64_t *n_out);
/* enable != 0 (default): from the second execution on, the whole batch runs as
 * one HIP graph in which problem i is recorded on branch i mod branches
 * (1..16, default 4) so that independent problems may overlap.  The graph is
 * recorded again whenever the buffer pointers change.  enable = 0: every
 * execution launches the kernels one by one on the context stream. */
nvp_status nvp_batch_set_graph(nvp_batch *batch, int enable, int branches);
/* enable != 0: run the batch level by level (harmonic n of every problem that
 * has it) with each pass of the convolution as one multi-task launch over the
 * problems that share its transform length (a task table in device memory
 * maps each workgroup to its problem), instead of one launch per problem;
 * inside a graph when nvp_batch_set_graph enables one (as by default).
 * Problems whose harmonic takes the fused source path run that harmonic on
 * their own.  Results are the same bits as per-problem execution. */
nvp_status nvp_batch_set_grouped(nvp_batch *batch, int enable);
/* nvp_plan_autotune for every problem, sharing one cache (identical shapes
 * are timed once). */
nvp_status nvp_batch_autotune(nvp_batch *batch, const char *cache_path, int reps);
/* p1_dev[i]: p_1 of problem i; pn_dev[slot]: outputs as numbered above.  The
 * first execution (and every execution with the kernel cache of some problem
 * off) runs eagerly and fills the kernel-spectrum caches; later ones launch
 * the graph.  Enqueued on the context stream. */
nvp_status nvp_batch_execute(nvp_batch *batch, const void *const *p1_dev, void *const *pn_dev);
nvp_status nvp_batch_destroy(nvp_batch *batch);

/* ---- timing of the plan's kernels ---------------------------------------- */

/* Kinds of kernel timed by nvp_plan_get_timing. */
#define NVP_T_KTAB 0   /* kernel tabulation fused with the first (z) FP64 FFT pass */
#define NVP_T_KFFT 1   /* kernel spectrum: the y and x FP64 FFT passes and the downcast */
#define NVP_T_XFWD 2   /* forward x pass (with the source build fused in, when that path is used) */
#define NVP_T_YFWD 3   /* forward y pass */
#define NVP_T_ZCONV 4  /* z pass: forward FFT, spectral multiply, inverse FFT */
#define NVP_T_YINV 5   /* inverse y pass */
#define NVP_T_XINV 6   /* inverse x pass with the C_n / M scale */
#define NVP_T_SRC 7    /* transfer + source build as its own tiled kernel */
#define NVP_T_KINDS 8

/* enable != 0: bracket every kernel launch with HIP events on the plan's
 * stream from now on (adds no device work between kernels). */
nvp_status nvp_plan_set_timing(nvp_plan *plan, int enable);
/* Waits for the recorded events; ms[k] = summed kernel time of kind k and
 * count[k] = launches since the last call (both arrays of n_kinds entries);
 * then clears the record. */
nvp_status nvp_plan_get_timing(nvp_plan *plan, double *ms, int64_t *count, int n_kinds);

#ifdef __cplusplus
}
#endif
#endif /* NVP_H */
