/*
 * asn.h - C ABI of the MI355X artificial-scattering S_N (as-S_N) library.
 *
 * The library advances the as-S_N equations (Camminady, Frank, Hauck, Kusch,
 * arXiv:1911.08801, Section 3.2, eq. asSNeq) on a uniform 2-D Cartesian grid
 * with an explicit forward-Euler, first-order donor-cell step:
 *
 *   psi_q^{n+1} = psi_q - dt * div(F_upwind(psi_q))
 *                 - dt (sigma_a + sigma_s + sigma_as) psi_q
 *                 + dt sigma_s Phi / W
 *                 + dt sigma_as sum_p K_qp psi_p
 *                 + dt q,
 *
 * where Phi = sum_q w_q psi_q is the scalar flux (Section 2.2), W = sum_q w_q,
 * and K is the quadrature-normalised artificial in-scattering matrix built
 * from the kernel s_eps(mu) ~ exp(-((1 - mu)/eps)^2) of eq. (5) with
 * eps = beta / N_q (Section 2.3).  Boundaries are vacuum (no incoming flux).
 *
 * Conventions for every entry point:
 *   - All functions return asn_status; nothing throws or aborts across the ABI.
 *     On failure a thread-local message is available from asn_last_error().
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *     pointers are HIP device memory on the problem's device.
 *   - Grids are row-major: cell (j, i) (row j along y, column i along x) is at
 *     flat index c = j * nx + i.  Angular fluxes are ordinate-major:
 *     psi[q][j][i], q = 0 .. Q-1.
 *   - A problem handle is used by one host thread at a time.  Work is enqueued
 *     on the handle's HIP stream; entry points that return data to the host
 *     synchronise that stream.
 */
#ifndef ASN_H
#define ASN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ASN_OK = 0,
    ASN_E_INVALID = -1,      /* an argument is out of range or inconsistent          */
    ASN_E_OOM = -2,          /* device allocation failed or workspace too small      */
    ASN_E_HIP = -3,          /* a HIP runtime call failed (message holds its text)   */
    ASN_E_UNSTABLE = -4,     /* CFL above 1, or the solution became non-finite       */
    ASN_E_STATE = -5,        /* handle used in a state that does not allow the call  */
    ASN_E_UNSUPPORTED = -6   /* valid request this build does not implement          */
} asn_status;

/* Operand type of the artificial-scattering contraction sum_p K_qp psi_p. */
enum { ASN_GEMM_F32 = 0, ASN_GEMM_BF16 = 1, ASN_GEMM_F16 = 2 };

/* Normalisation of K (Section 3.2 normalisation factors).
 * ASN_NORM_SYM: K = diag(d) S diag(w d), rows and w-weighted columns sum to one,
 *               so the discrete operator conserves particles.
 * ASN_NORM_ROW: the paper's K_qp = w_p c_q^(eps) s_eps(Omega_q . Omega_p),
 *               c_q^(eps) = 1 / sum_p w_p s_eps(Omega_q . Omega_p). */
enum { ASN_NORM_SYM = 0, ASN_NORM_ROW = 1 };

/* Explicit time scheme.
 * ASN_SCHEME_EULER: forward Euler with first-order donor-cell (upwind) fluxes.
 * ASN_SCHEME_HEUN:  the paper's explicit scheme (Section 3.1): Heun's method with
 *                   second-order upwind fluxes from a minmod-limited linear
 *                   reconstruction per axis (slope minmod(psi_i - psi_{i-1},
 *                   psi_{i+1} - psi_i), face value psi_i +- slope / 2 on the upwind
 *                   side, zero ghost cells); psi^1 = psi + dt R(psi),
 *                   psi^{n+1} = (psi + psi^1 + dt R(psi^1)) / 2. */
/* ASN_SCHEME_IMPLICIT: the paper's implicit scheme (Sections 3.4-3.5, Algorithms 1-3):
 *                   implicit Euler, faces carry 3/2 psi_up - 1/2 psi_upup (no limiter),
 *                   the artificial scattering is resolved inside the sweep by source
 *                   iteration (Algorithm 1: stop once ||psi^(l+1) - psi^(l)||_2 <
 *                   source_tol (1 - T)/T, T the a-priori contraction bound
 *                   max sigma_as / (sigma_a + sigma_s + sigma_as + 1/dt); the norm is
 *                   Euclidean over all ordinates and cells; at most 500 sweeps),
 *                   and GMRES (restart 30, relative residual implicit_tol) solves for
 *                   the scalar flux.  FP64 on the device; cfl above 1 is allowed;
 *                   nx <= 2048; such problems step alone (no batches); asn_step blocks
 *                   until its steps are done. */
enum { ASN_SCHEME_EULER = 0, ASN_SCHEME_HEUN = 1, ASN_SCHEME_IMPLICIT = 2 };

/* Stopping test of the implicit scheme's source iteration (Algorithm 1).
 * ASN_SOURCE_TEST_ABSOLUTE: ||psi^(l+1) - psi^(l)||_2 < source_tol (1 - T)/T, as printed
 *                           (the estimated distance to the fixed point below source_tol).
 * ASN_SOURCE_TEST_RELATIVE: ... < source_tol (1 - T)/T ||psi^(l+1)||_2, a scale-free
 *                           variant for right-hand sides far from unit size. */
enum { ASN_SOURCE_TEST_ABSOLUTE = 0, ASN_SOURCE_TEST_RELATIVE = 1 };

/* Time-step rule.  Both start from dt_max = cfl / max_q(|xi_q|/dx + |eta_q|/dy)
 * and take dt = t_final / n, n = ceil(t_final / dt_max).
 * ASN_DT_STREAMING: that rule alone (Section 4.1; CFL on the streaming).
 * ASN_DT_STIFF:     dt_max is also limited so that the stability number (see
 *                   asn_stability) is at most 2 cfl.  For strongly absorbing cells
 *                   on coarse grids the streaming rule alone leaves the explicit
 *                   schemes' stability interval and the discrete solution grows
 *                   without bound; this rule keeps every problem inside it. */
enum { ASN_DT_STREAMING = 0, ASN_DT_STIFF = 1 };

/* Kernel form of a forward-Euler step (results agree to FP32 rounding across forms).
 * ASN_FORM_FUSED:    the stream + collide update runs in the contraction kernel's
 *                    epilogue; the contraction output Y never reaches memory.
 * ASN_FORM_SEPARATE: contraction, then a separate stencil kernel (Y through memory).
 * ASN_FORM_BANDED:   product sets only: the set is invariant under rotation by
 *                    2 pi / n_azim about the polar axis, so K restricted to two polar
 *                    levels is circulant along the azimuth, and K couples only nearby
 *                    levels (forward peak, Section 3.5 notes S_as^+ is sparse).  One kernel
 *                    per step applies K level pair by level pair and the update, reading
 *                    psi^n once.  FP32: short circular convolutions on the vector units,
 *                    n_azim in {8, 16, ..., 64}.  BF16 / FP16: each coupled pair's
 *                    n_azim x n_azim circulant block of the rounded K on the matrix
 *                    cores, the update as ASN_FORM_FUSED (the same rounding recipe and
 *                    pending per-cell correction), n_azim 32, 48 or 64.  Needs levels at
 *                    most 3 apart coupled (BF16 at 48 or 64 azimuths: 2) and the stored K exactly
 *                    circulant (checked at asn_create; ASN_E_UNSUPPORTED otherwise).
 * ASN_FORM_AUTO:     the banded form where it applies; else BF16/FP16 fuse, and FP32
 *                    runs separate kernels from 2^25 cell-ordinates (nx <= 4088) and
 *                    fuses smaller problems, the faster forms on MI355X at the sizes
 *                    measured.  asn_workspace_size covers every form AUTO may take. */
enum { ASN_FORM_AUTO = 0, ASN_FORM_SEPARATE = 1, ASN_FORM_FUSED = 2, ASN_FORM_BANDED = 3 };

#define ASN_BUDGET_LEN 8

/* Uniform grid of nx * ny cells covering [x_min, x_max] x [y_min, y_max]. */
typedef struct {
    int32_t nx, ny;
    double x_min, x_max, y_min, y_max;
} asn_grid;

/* Angular quadrature.  Default: product set of n_polar Gauss-Legendre nodes in
 * mu (axis normal to the grid) times n_azim uniform azimuths
 * phi_k = (k + 1/2) 2 pi / n_azim, ordinate q = i * n_azim + k (Q = n_polar *
 * n_azim).  q_custom > 0: Q = q_custom ordinates from omega_xyz[Q][3] (unit
 * vectors, host) and weights[Q] (positive, host).  icosahedron_order >= 2 (and
 * q_custom == 0): the icosahedron set of paper Section 3.3, see
 * asn_build_icosahedron.  The streaming uses the x-y projection (Section 4). */
typedef struct {
    int32_t n_polar, n_azim;
    int32_t q_custom;
    const double* omega_xyz;
    const double* weights;
    int32_t icosahedron_order;
} asn_quadrature;

typedef struct {
    int32_t gemm_dtype;     /* ASN_GEMM_F32 (default), ASN_GEMM_BF16, ASN_GEMM_F16              */
    int32_t normalization;  /* ASN_NORM_SYM (default) or ASN_NORM_ROW                             */
    double cfl;             /* 0 < cfl <= 1 bounds dt * max_q(|xi|/dx + |eta|/dy); default 0.95   */
    double eps_override;    /* > 0: kernel width eps used instead of beta / Q                     */
    double dt_override;     /* > 0: fixed dt (still subject to the CFL bound)                     */
    int32_t scale_block;    /* ASN_GEMM_BF16 / _F16: cells per block of the operand's power-of-two
                               scale (flat cell index c = y nx + x, blocks [b n, (b + 1) n));
                               a power of two from 64 to 4096, default 256; 0 means 256.
                               Ignored for FP32, still checked.                           */
    int32_t scheme;         /* ASN_SCHEME_EULER (default) or ASN_SCHEME_HEUN                     */
    int32_t dt_rule;        /* ASN_DT_STREAMING (default) or ASN_DT_STIFF                        */
    int32_t step_form;      /* ASN_FORM_AUTO (default), _SEPARATE, _FUSED or _BANDED:       
                               kernel form of forward-Euler steps (other schemes: separate)   */
    double implicit_tol;    /* ASN_SCHEME_IMPLICIT: GMRES relative residual (0: 1.5e-8, paper 4.1) */
    double source_tol;      /* ASN_SCHEME_IMPLICIT: source-iteration tolerance (0: 1e-4, paper 4.1) */
    int32_t source_test;    /* ASN_SCHEME_IMPLICIT: ASN_SOURCE_TEST_ABSOLUTE (default) or _RELATIVE */
} asn_options;

typedef struct asn_problem_s* asn_problem;

/* Fill *opt with the defaults listed above.  Errors: ASN_E_INVALID if opt is NULL. */
asn_status asn_options_default(asn_options* opt);

/* Device bytes asn_create needs when the caller supplies the workspace.
 * Errors: ASN_E_INVALID on inconsistent grid/quadrature/options. */
asn_status asn_workspace_size(const asn_grid* grid, const asn_quadrature* quad,
                              const asn_options* opt, size_t* bytes);

/* Build a problem: quadrature, kernel matrix K (FP64 on the host, then cast),
 * time step dt = t_final / ceil(t_final / dt_max) and the per-cell fields.
 * sigma_s, sigma_a, sigma_as, source: host float[ny * nx] (source may be NULL =
 * 0; it is the isotropic per-steradian q of eq. asSNeq).  kernel_beta > 0 sets
 * eps = kernel_beta / Q (Section 2.3).  hip_stream: a hipStream_t (NULL = the
 * null stream).  workspace: device memory of at least asn_workspace_size bytes,
 * owned by the caller and kept alive until asn_destroy, or NULL for memory the
 * library allocates and frees.  The state starts at psi = 0.
 * Errors: ASN_E_INVALID (nx, ny < 1, empty domain, Q < 1, non-unit omega,
 * weight <= 0, negative or non-finite sigma, beta <= 0, cfl <= 0, t_final <= 0),
 * ASN_E_UNSTABLE (cfl > 1, or dt_override above the CFL bound), ASN_E_OOM, ASN_E_HIP. */
asn_status asn_create(const asn_grid* grid, const asn_quadrature* quad,
                      const float* sigma_s, const float* sigma_a, const float* sigma_as,
                      const float* source, double kernel_beta, double t_final,
                      const asn_options* opt, void* hip_stream,
                      void* workspace, size_t workspace_bytes, asn_problem* out);

/* Set the angular flux: psi float[Q][ny][nx], host (on_device = 0) or device
 * (on_device = 1).  Resets the step counter and the particle budget.
 * Errors: ASN_E_INVALID (NULL), ASN_E_HIP. */
asn_status asn_set_state(asn_problem p, const float* psi, int32_t on_device);

/* Set an isotropic state psi_q(c) = psi_cell[c] for every ordinate; psi_cell is
 * float[ny][nx] on the host or the device.  Same effects as asn_set_state. */
asn_status asn_set_state_isotropic(asn_problem p, const float* psi_cell, int32_t on_device);

/* Copy the angular flux float[Q][ny][nx] to host or device memory; synchronises. */
asn_status asn_get_state(asn_problem p, float* psi, int32_t on_device);

/* Enqueue n_steps explicit steps on the problem's stream (asynchronous).
 * n_steps may exceed the remaining steps to t_final (the solution keeps evolving).
 * Errors: ASN_E_INVALID (n_steps < 0), ASN_E_HIP. */
asn_status asn_step(asn_problem p, int64_t n_steps);

/* Advance n problems by n_steps each with one fused launch per kernel per step
 * (asn_batch_create + asn_batch_step + asn_batch_destroy).  Results equal
 * asn_step on each problem alone, bit for bit.
 * Errors: those of asn_batch_create and asn_batch_step. */
asn_status asn_step_batch(asn_problem* probs, int32_t n, int64_t n_steps);

/* asn_step_batch for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same steps with
 * the same results, bit for bit, and no hipMalloc, hipFree, graph instantiation or
 * other allocating call.  The batch tables live in a static device array of 64 KiB
 * per GPU (held until the process ends), which bounds the batch to what fits (every
 * batch of up to 64 problems does).  Launches are eager on the problems' stream and
 * the call waits for them before it returns.  Every call on one GPU shares that array
 * and overwrites it: calls that overlap on one GPU (other host threads, or problems on
 * another stream of the same device while a call runs) race and must not be issued.
 * Errors: those of asn_batch_create (ASN_E_INVALID, ASN_E_UNSUPPORTED), ASN_E_INVALID
 * (n_steps outside [0, 2^20]), ASN_E_HIP. */
asn_status asn_step_batch_noalloc(asn_problem* probs, int32_t n, int64_t n_steps);

/* A batch groups 1..64 problems for fused stepping: every kernel of a step covers
 * all of them in one launch.  Problems keep their own grid, ordinates, kernel
 * matrix and buffers (ordinate counts may differ); they must share the operand
 * type, the time scheme, the kernel form (asn_step_form: with ASN_FORM_AUTO it
 * follows the problem size, so ask for one form for problems of different sizes)
 * and the HIP stream.  The batch holds small device tables (hipMalloc).
 * A problem may be stepped alone while in a batch; the batch reads each
 * problem's current buffer at every asn_batch_step.  Errors: ASN_E_INVALID,
 * ASN_E_OOM, ASN_E_HIP. */
typedef struct asn_batch_s* asn_batch;
asn_status asn_batch_create(asn_problem* probs, int32_t n, asn_batch* out);

/* Enqueue n_steps fused steps (asynchronous).  Problem i takes min(n_steps,
 * limit[i]) of them and its blocks exit at once afterwards (limit may be NULL =
 * all take n_steps), so problems with different horizons share the launches.
 * On a non-null stream the sequence of n_steps steps is captured once into a HIP
 * graph and replayed on later calls with the same n_steps.
 * Errors: ASN_E_INVALID (n_steps < 0 or > 2^20), ASN_E_HIP. */
asn_status asn_batch_step(asn_batch b, int64_t n_steps, const int64_t* limit);

/* Synchronise the batch's stream and free its tables and graphs.  NULL accepted. */
asn_status asn_batch_destroy(asn_batch b);

/* Stability number of the problem's dt:
 *   z = dt [ 2 max_q (|xi_q|/dx + |eta_q|/dy)
 *            + max_c (sigma_a + sigma_s + 2 (1 - min_q K_qq) sigma_as) ].
 * In a region of uniform material, a state that alternates in sign from cell to
 * cell decays at a rate given by the eigenvalues of 2 diag(r_q) + (sigma_a +
 * sigma_s + sigma_as) I - sigma_as K - sigma_s (isotropic projection); for the
 * symmetric normalisation these are real and at most the bracket (Weyl's
 * inequality, with the eigenvalues of K at least 2 min_q K_qq - 1 by
 * Gershgorin's theorem).  Forward Euler and Heun are stable for a real decay
 * rate only while dt times it lies in [0, 2]; z <= 2 therefore rules out the
 * growth of such modes, and z above 2 is where the streaming rule alone can let
 * the run grow without bound (coarse grids, strong absorbers).
 * Errors: ASN_E_INVALID. */
asn_status asn_stability(asn_problem p, double* z);

/* ASN_SCHEME_IMPLICIT: transport sweeps and GMRES matrix-vector products since the
 * last set_state (0 for the explicit schemes).  Errors: ASN_E_INVALID. */
asn_status asn_iteration_counts(asn_problem p, int64_t* sweeps, int64_t* matvecs);

/* Run n_steps exactly like asn_step while recording HIP events on the problem's
 * stream between its kernels; synchronises.  kernel_ms[k] receives the average
 * duration per step of kernel k: 0 the ordinate contraction Y = K Psi, 1 stream
 * + collide, 2 moment finalize, 3 budget fold (for ASN_SCHEME_HEUN, the sum over
 * its two passes); kernel_ms[4] the average span of a whole step.  Measurement
 * support for benchmarks; results equal asn_step.
 * Errors: ASN_E_INVALID (n_steps < 1), ASN_E_HIP. */
asn_status asn_step_timed(asn_problem p, int64_t n_steps, double kernel_ms[5]);

/* Scalar flux Phi = sum_q w_q psi_q in FP64 into phi_host double[ny][nx]; synchronises. */
asn_status asn_scalar_flux(asn_problem p, double* phi_host);

/* Particle budget since the last set_state, FP64, synchronises:
 * out[0] current mass M = dx dy sum_c Phi_c, out[1] initial mass,
 * out[2] cumulative absorption dt sum_n dx dy sum_c sigma_a Phi^n,
 * out[3] cumulative outflow through the boundary, out[4] cumulative source,
 * out[5] cumulative artificial-scattering defect dt sum_n dx dy sum_c sigma_as
 *        sum_q w_q (Y_q - psi_q) (zero up to rounding for ASN_NORM_SYM),
 * out[6] max over steps of |M^{n+1} - M^n - dt(-A - O + S + D)| / max(M^0, M^n),
 * out[7] steps covered by the budget.
 * Errors: ASN_E_UNSTABLE if the mass is not finite, ASN_E_HIP. */
asn_status asn_mass_budget(asn_problem p, double out[ASN_BUDGET_LEN]);

/* Kernel form of the problem's steps: ASN_FORM_FUSED, ASN_FORM_SEPARATE or
 * ASN_FORM_BANDED (what ASN_FORM_AUTO chose at asn_create; Heun and implicit steps
 * report ASN_FORM_SEPARATE).  Problems of one batch must share it.  Errors: ASN_E_INVALID
 * for a NULL argument. */
asn_status asn_step_form(asn_problem p, int32_t* form);

/* Problem facts: time step, steps taken, steps to t_final, ordinate count.
 * Any output pointer may be NULL. */
asn_status asn_info(asn_problem p, double* dt, int64_t* steps_done, int64_t* steps_to_tfinal,
                    int32_t* q);

/* Arithmetic of one contraction Y = K Psi: dense_flops = 2 Q^2 C; tile_flops =
 * 2 C times the number of K entries in the blocks the kernel multiplies (banded
 * step: the runs it multiplies, see asn_contraction_nonzero; in BF16 / FP16 every
 * coupled pair's whole n_azim x n_azim block, not counting the zero operands that fill a
 * level's pair slots up to 2 reach + 1).  K is
 * forward peaked (paper Section 3.5: the discrete artificial in-scattering is a
 * sparse matrix), so blocks whose entries are all zero in the stored operand type
 * are skipped: 128-row x 32-column tiles for BF16/FP16, and for FP32 the 16-row x
 * 4-column blocks (the K operand of one MFMA).  The skipped products are exact zeros
 * and the result is unchanged.  Either pointer may be NULL. */
asn_status asn_contraction_work(asn_problem p, double* dense_flops, double* tile_flops);

/* The contraction's own arithmetic: nonzero_flops = 2 C times the number of nonzero
 * entries of K in the stored operand type (FP32, or the BF16/FP16 copy), the products
 * the method needs (paper Section 3.5: S_as^+ is sparse).  The banded step
 * (ASN_FORM_BANDED) multiplies every stored nonzero of a pair's run plus the zeros that
 * pad wide runs to a multiple of four, which asn_contraction_work reports as its
 * tile_flops.  Errors: ASN_E_INVALID (NULL problem or pointer). */
asn_status asn_contraction_nonzero(asn_problem p, double* nonzero_flops);

/* Free the handle and any memory the library allocated.  NULL is accepted. */
asn_status asn_destroy(asn_problem p);

const char* asn_status_string(asn_status s);
const char* asn_last_error(void);

/* ---- Host-side builders (no GPU needed); they are the set-up asn_create runs. ---- */

/* Product quadrature (see asn_quadrature): omega_xyz double[Q][3], weights double[Q]. */
asn_status asn_build_quadrature(int32_t n_polar, int32_t n_azim, double* omega_xyz,
                                double* weights);

/* Icosahedron set (paper Section 3.3) of the given order >= 2, Q = 10 (order - 1)^2
 * + 2 ordinates (12, 42, 92, 162, ...): every face of a regular icosahedron with a
 * vertex at (0, 0, 1) is split by equidistant points on its edges (and the
 * corresponding interior points) into (order - 1)^2 triangles, the nodes are
 * projected onto the unit sphere, and a node's weight is the area of the spherical
 * polygon that joins the centres of its surrounding triangles (weights sum to
 * 4 pi).  Ordinates are sorted by decreasing z, then increasing azimuth.
 * omega_xyz double[Q][3], weights double[Q], host.  Errors: ASN_E_INVALID. */
asn_status asn_build_icosahedron(int32_t order, double* omega_xyz, double* weights);

/* Normalised kernel matrix K double[Q][Q] (row-major, K[q][p]) for unit ordinates
 * omega_xyz[Q][3] and weights[Q], width eps > 0, normalisation ASN_NORM_*.
 * Errors: ASN_E_INVALID; ASN_E_UNSUPPORTED if the symmetric scaling fails to converge. */
asn_status asn_build_kernel(int32_t q, const double* omega_xyz, const double* weights,
                            double eps, int32_t normalization, double* k_out);

/* Reduced-precision copy of a kernel matrix as used by the contraction with
 * gemm_dtype ASN_GEMM_BF16 or ASN_GEMM_F16: k_bits[Q][Q] receives the 16-bit
 * patterns of T(fp32(K)) rounded to nearest even, row_defect[Q] the values
 * fp32(1 - sum_p T(K)_qp) (sum in FP64).  k_in is double[Q][Q] row-major.
 * Errors: ASN_E_INVALID. */
asn_status asn_build_kernel_lowp(int32_t q, const double* k_in, int32_t gemm_dtype,
                                 uint16_t* k_bits, float* row_defect);

/* The banded form ASN_FORM_BANDED takes of a product set's kernel matrix, expanded
 * back (host only): from fp32(k_in) (double[Q][Q] row-major, Q = n_polar * n_azim,
 * ordinate q = i * n_azim + k) the library builds per pair of polar levels i, j one
 * row of coefficients c_ij(delta) over azimuth offsets, and k_out[Q][Q] receives
 * k_out[(i,k)][(j,k')] = c_ij(k' - k mod n_azim) (zero outside the stored runs);
 * *reach is the largest level distance coupled.  The step applies K in this form.
 * Errors: ASN_E_INVALID (NULL, sizes); ASN_E_UNSUPPORTED if fp32(K) is not circulant
 * along the azimuth per level pair, couples levels more than 3 apart, or n_azim is odd. */
asn_status asn_band_expand(int32_t n_polar, int32_t n_azim, const double* k_in, float* k_out,
                           int32_t* reach);

/* Time step for a grid: dt = t_final / n, n = ceil(t_final / dt_max),
 * dt_max = cfl / max_q(|xi_q|/dx + |eta_q|/dy).  Errors: ASN_E_INVALID, ASN_E_UNSTABLE. */
asn_status asn_time_step(const asn_grid* grid, int32_t q, const double* omega_xyz, double cfl,
                         double t_final, double* dt, int64_t* n_steps);

#ifdef __cplusplus
}
#endif
#endif /* ASN_H */
