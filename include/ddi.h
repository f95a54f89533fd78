/*
 * ddi.h -- C ABI of the MI355X (gfx950) NUFFT dipole-dipole interaction library.
 *
 * The library evaluates the dipolar potential Phi = U_dip * rho on a uniform
 * grid (Bao, Tang & Zhang, Sec. 1, Eqs. DipGPE0 and dipole-poten0) by the
 * Fourier quadrature of Sec. 2.1: the inverse transform of Eq. DDI-Con is
 * truncated to a ball and written in spherical (3D) or polar (2D)
 * coordinates, whose Jacobian |k|^(d-1) cancels the singularity of the
 * symbol at k = 0 (Eq. DDI-Trun1); the tensor quadrature sum is evaluated by
 * a type-2 NUFFT (grid -> quadrature nodes), a multiplication by the weighted
 * symbol and a type-1 NUFFT (nodes -> grid), all in hand-written HIP kernels.
 *
 * Discrete operator (what every entry point computes, up to the NUFFT
 * tolerance):
 *     rhohat_q = prod(h) sum_l rho_l exp(-i k_q . x_l)
 *     Phi_l    = sum_q c_q Re[rhohat_q exp(+i k_q . x_l)],
 *     c_q      = W_q Uhat(k_q) / (2 pi)^d
 * with x_l = -L + l h on the half-open box [-L, L), N points per axis, the
 * symbol Uhat of Eq. DipKer (two axes: Eq. dipmn), Gauss-Legendre nodes in
 * |k| on [0, Kmax] and in cos(theta) on [-1, 1], uniform azimuths, and the
 * nodes outside the Nyquist box |k_i| <= pi/h_i removed.
 *
 * Conventions for every entry point
 *  - Grids are C-ordered (last axis fastest).  3D arrays are [n0][n1][n2];
 *    2D arrays are [n0][n1] (the paper's x, y).
 *  - Element types follow the plan's precision: DDI_FP64 -> double grids and
 *    complex double (interleaved re, im) node arrays; DDI_MIXED -> float grids
 *    and complex float node arrays.  Plan tables (nodes, weights, symbol,
 *    deconvolution) are FP64 in both forms.
 *  - Buffers named *_dev are device pointers owned by the caller, on the
 *    device that was current when the plan was made; they must not alias
 *    each other.  Inputs are never modified.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *    enqueued asynchronously; no entry point synchronises the host except
 *    gpe_energy_grad (which returns host values) and ddi_plan/ddi_plan_nodes.
 *  - A plan owns its device workspace: calls that use one plan must be
 *    ordered (one stream, or explicit events).  ddi_apply, ddi_apply_adjoint,
 *    ddi_type2 and ddi_type1 allocate no memory.
 *  - Errors: every call returns a ddi_status; on failure ddi_last_error()
 *    returns a message (thread-local).  No exception crosses the ABI.  NaN or
 *    Inf inputs propagate to the outputs; they are not detected.
 */
#ifndef DDI_H
#define DDI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddi_plan_s* ddi_plan_t;

typedef enum {
  DDI_OK = 0,
  DDI_EINVAL = 1,     /* invalid argument (sizes, NULL pointers, unit vectors) */
  DDI_ENOMEM = 2,     /* device or host allocation failed */
  DDI_EDEVICE = 3,    /* a HIP runtime call failed */
  DDI_ENOTSUP = 4,    /* valid but unsupported configuration (e.g. grid size) */
  DDI_EINTERNAL = 5
} ddi_status;

typedef enum { DDI_FP64 = 0, DDI_MIXED = 1 } ddi_precision;

/*
 * Plan parameters (Sec. 2.1).
 *  dim          2 or 3.
 *  n[3]         grid points per axis (n[2] ignored for dim 2); powers of two or
 *               three times a power of two (e.g. 96), 8 <= n <= 512 in 3D,
 *               32 <= n <= 512 in 2D, and in 2D a first axis of the form 3 * 2^a
 *               must be at least 96 (its oversampled axis holds whole 64-point tiles).
 *  L[3]         half box lengths; the box is [-L_i, L_i), h_i = 2 L_i / n_i.
 *  dip_n[3]     unit dipole axis n, used as given (not renormalised; must be
 *               non-zero and finite).
 *               In 2D n_perp = (dip_n[0], dip_n[1]) and n3 = dip_n[2].
 *  dip_m[3]     second dipole axis m of Eq. dipmn; all zero means m = n.
 *  n_rad, n_pol, n_azi  quadrature sizes (n_pol ignored in 2D); n_azi even.
 *  kmax         radius of the Fourier ball; <= 0 selects pi*sqrt(sum_i 1/h_i^2).
 *  nyquist_mask 1: drop nodes with |k_i| > pi/h_i (the default reading);
 *               0: keep them (then nodes outside the box alias).
 *  tol          requested relative accuracy of the NUFFT; picks the kernel
 *               width w = ceil(-log10(tol)) + 1 (clamped to [4, 16]).
 *  prec         DDI_FP64 or DDI_MIXED (FP32 grids, spread, interp and FFT).
 *  kernel_width 0 = from tol; else the width w (4..16) of the
 *               exponential-of-semicircle kernel.
 *  split        0: the quadrature over the whole ball (above).  1: the split of
 *               Sec. 2.1, Eq. 3.9, Phi = I_1 + I_2 with the partition
 *               q(k) = exp(-|k|^2/s^2) in 3D and q(k) = erfc(|k|/s) in 2D (where
 *               the symbol grows like |k|: with 1 - q = erf(|k|/s), (1 - q) Uhat
 *               is smooth):
 *                 I_1 = (2 pi)^-d int over the Nyquist box |k_i| < pi/h_i of
 *                       exp(i k.x) (1 - q(k)) Uhat(k) rhohat(k) dk, by the
 *                       trapezoid rule of the box zero-padded to 2 n_i points
 *                       per axis (k_m = pi m / (2 L_i), |m| < n_i; the Nyquist
 *                       planes m_i = -n_i are left out), i.e. a padded FFT,
 *                       a multiplication and an inverse FFT;
 *                 I_2 = the quadrature sum above over the ball of radius kmax
 *                       with every weight c_q multiplied by q(k_q).
 *               The quadrature sizes and kmax are then those of I_2, and
 *               kmax <= 0 selects s sqrt(ln(1/tol)) (divided by the smallest
 *               stretch factor).  ddi_type2 / ddi_type1 act on the I_2 nodes.
 *  split_s      s of the partition (split = 1); <= 0 selects
 *               sqrt(ln(1/tol)) / min_i L_i, which puts the decay
 *               exp(-s^2 r^2/4) of the short-range kernel at tol at the
 *               nearest image 2 L_min away.  With kernel_width set and tol
 *               outside (0, 1), tol is taken as 10^-(w-1).
 *  stretch[3]   per-axis factors S_i of the quadrature (a reading for anisotropic
 *               boxes such as Tables 4-5): nodes k = S k' with k' on the rule
 *               above, weights times det S; the Jacobian still cancels the
 *               singularity (Uhat is homogeneous of degree 0).  kmax (of k')
 *               <= 0 then selects pi sqrt(sum 1/(h_i S_i)^2).  Values <= 0 mean
 *               1 (the plain rule); stretch[2] is ignored in 2D.
 */
typedef struct {
  int32_t dim;
  int64_t n[3];
  double L[3];
  double dip_n[3];
  double dip_m[3];
  int64_t n_rad, n_pol, n_azi;
  double kmax;
  int32_t nyquist_mask;
  double tol;
  int32_t prec;
  int32_t kernel_width;
  int32_t split;
  double split_s;
  double stretch[3];
} ddi_params;

/*
 * GPE parameters for gpe_energy_grad / gpe_gf_step (Sec. 1, Eqs. DipGPE0,
 * Vpoten, energy).  V(x) = 1/2 sum_i gamma_i^2 x_i^2 unless V_dev is a device
 * grid of the plan's real type, which then replaces it.
 */
typedef struct {
  double beta;
  double lambda;
  double gamma[3];
  const void* V_dev;
} gpe_params;

typedef struct {
  int64_t m_eff;        /* quadrature nodes kept after the mask */
  int64_t m_nominal;    /* n_rad * n_pol * n_azi (3D) or n_rad * n_azi (2D) */
  int64_t m_half;       /* nodes interpolated and spread by ddi_apply: one per +-k pair */
  int64_t apply_window; /* positions along the fine grid's last axis that ddi_apply transforms:
                           the kept member of each pair lies on one side, so their supports
                           cover a window of n_fine[2] (a multiple of 8 in FP64, 16 in mixed;
                           n_fine[2] if there is no gap) */
  int64_t n_fine[3];    /* oversampled FFT grid (n_fine[0] = 1 in 2D) */
  int32_t width;        /* kernel width w */
  double es_beta;       /* kernel shape parameter */
  double kmax;
  int64_t spread_items; /* spread work items (tiles, tile chunks, and empty items that even out the per-XCD regions) */
  int64_t spread_entries; /* (tile, node) pairs visited by one spread */
  int64_t workspace_bytes;
  int32_t split;        /* 1 for the split of Eq. 3.9 */
  double split_s;       /* s of the partition as used (0 without the split) */
} ddi_plan_info_t;

/* Build a plan: quadrature nodes and weights, mask, symbol, kernel and
 * deconvolution tables, the node-to-tile schedule, and the device workspace.
 * Synchronises `stream` before returning.  *out is NULL on failure. */
ddi_status ddi_plan(const ddi_params* params, void* stream, ddi_plan_t* out);

/* Phi = A rho (Sec. 2.1, Eqs. DDI-Con, DDI-Trun1).  rho_dev, phi_dev: real grids.
 * A split plan returns I_1 + I_2 (Eq. 3.9): I_1 is computed on a stream the plan owns (default
 * priority), forked from `stream` by an event, concurrently with I_2 on `stream`, and added to
 * phi after I_2; `stream` waits for it before any later work, so the call is ordered on
 * `stream` like every other. */
ddi_status ddi_apply(ddi_plan_t plan, const void* rho_dev, void* phi_dev, void* stream);

/* rhobar = A^T phibar, executed literally: transform with exp(+i k.x) to the
 * nodes, weights c_q, transform back with exp(-i k.x), real part.  In exact
 * arithmetic A^T = A; used for gradients.  A split plan returns the transpose of
 * I_2 plus I_1 (the padded convolution with an even real multiplier over a
 * symmetric set of modes is its own transpose). */
ddi_status ddi_apply_adjoint(ddi_plan_t plan, const void* phibar_dev, void* rhobar_dev, void* stream);

/* New dipole axes for a plan (Eq. DipKer; two axes: Eq. dipmn), for a time-dependent orientation
 * such as Eq. dip_rot: every node coefficient c_q = W_q Uhat(k_q; n, m) / (2 pi)^d (times
 * q(k_q) for a split plan) is re-evaluated on the device from the stored nodes, and a split
 * plan's I_1 takes the new axes.  dip_n: 3 host doubles, used as given (non-zero, finite);
 * dip_m: NULL or all zero means m = n.  The first call on a plan allocates and uploads the node
 * coordinates and symbol-free weights (3 M_eff doubles) and synchronises; later calls enqueue
 * one small kernel on `stream` and allocate nothing.  Calls of the plan after it, on the same
 * stream, see the new axes; ddi_plan_nodes returns the new coefficients. */
ddi_status ddi_set_dipole(ddi_plan_t plan, const double* dip_n, const double* dip_m, void* stream);

/* Type-2 half: rhohat_q = prod(h) sum_l rho_l exp(-i k_q . x_l) for the M_eff
 * nodes in plan order (see ddi_plan_nodes).  rhohat_dev: complex array [M_eff]. */
ddi_status ddi_type2(ddi_plan_t plan, const void* rho_dev, void* rhohat_dev, void* stream);

/* Type-1 half: Phi_l = Re sum_q g_q exp(+i k_q . x_l), g_dev complex [M_eff] in plan order. */
ddi_status ddi_type1(ddi_plan_t plan, const void* g_dev, void* phi_dev, void* stream);

/*
 * GPE energy split (Sec. 3.2) and gradient.  psi_dev: complex grid.
 *   E_out[0] E_kin = 1/2 prod(h)/prod(n) sum_p |mu_p|^2 |psihat_p|^2 (spectral)
 *   E_out[1] E_pot = prod(h) sum V |psi|^2
 *   E_out[2] E_int = beta/2 prod(h) sum |psi|^4
 *   E_out[3] E_dip = lambda/2 prod(h) sum Phi |psi|^2, Phi = A |psi|^2
 *   E_out[4] total
 * grad_dev (nullable, complex grid): G = dE/d conj(psi) =
 *   prod(h) [-1/2 Lap psi + V psi + beta |psi|^2 psi + lambda/2 (A rho + A^T rho) psi].
 * E_out is a host pointer; the call synchronises `stream`.  The first call on
 * a plan allocates the GPE workspace (4 complex grids).
 */
ddi_status gpe_energy_grad(ddi_plan_t plan, const gpe_params* gp, const void* psi_dev,
                           double E_out[5], void* grad_dev, void* stream);

/*
 * gpe_energy_grad for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The same energies and gradient as
 * gpe_energy_grad, with its GPE workspace (three real grids, one complex grid and the reduction
 * partials of the plan's grid) taken from a static device array of 96 MiB that the library holds
 * on every GPU it runs on until the process ends, instead of the plan's own workspace.
 *   E_dev      device pointer to 5 doubles (kin, pot, int, dip, total), written on `stream`;
 *   grad_dev   as in gpe_energy_grad (nullable).
 * Allocates nothing (no hipMalloc, hipFree or allocating library call) and does not synchronise.
 * A grid whose workspace exceeds 96 MiB (20 bytes per point in mixed precision, 40 in FP64 plus the
 * partials: up to about 2.4M points in FP64, e.g. 128^3, and 4.8M in mixed) is rejected with
 * DDI_EINVAL before any work.  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (different streams, or different host threads) race and must be ordered by the caller.
 * Nothing in the array needs to start at zero: every call writes each part before reading it.
 */
ddi_status gpe_energy_grad_noalloc(ddi_plan_t plan, const gpe_params* gp, const void* psi_dev, double* E_dev,
                                   void* grad_dev, void* stream);

/*
 * One step of the gradient flow with discrete normalisation (Sec. 3.1,
 * Eqs. gf-eq2, gf-colb2, gffg33): Phi^n = A |psi_in|^2 once, then n_inner
 * stabilised Fourier iterations for (1/dt - 1/2 Lap + B) phi1 = psi_in/dt,
 * B = V + beta |psi_in|^2 + lambda Phi^n, alpha = (max B + min B)/2:
 *   (1/dt + alpha - 1/2 Lap) phi1_{j+1} = psi_in/dt + (alpha - B) phi1_j,  phi1_0 = psi_in,
 * then psi_out = phi1 / sqrt(prod(h) sum |phi1|^2).  psi_in, psi_out: complex
 * grids (may be the same buffer).  residual_dev (nullable): one device double that receives
 * the stopping quantity of Sec. 3.1, max_l |psi_out_l - psi_in_l| / dt, computed from the stored
 * values.  Does not synchronise.
 */
ddi_status gpe_gf_step(ddi_plan_t plan, const gpe_params* gp, double dt, int32_t n_inner,
                       const void* psi_in_dev, void* psi_out_dev, double* residual_dev, void* stream);

/*
 * One step of the second-order time splitting for the dipolar GPE dynamics (Sec. 4.1,
 * Eq. tssp2; the equation is Eq. DipGPE1 with the cubic nonlinearity and a time-independent
 * dipole axis), damping f = delta >= 0 (Case I: delta = 0; Case II, linear damping: delta > 0):
 *   psi1     = IDFT[exp(-i dt |mu|^2/4) DFT(psi_in)]
 *   psi2     = psi1 exp(-i [dt V + s (beta |psi1|^2 + lambda Phi)]) exp(-delta dt),  Phi = A |psi1|^2,
 *              s = dt (delta = 0) or (1 - exp(-2 delta dt)) / (2 delta)
 *   psi_out  = IDFT[exp(-i dt |mu|^2/4) DFT(psi2)]
 * with mu_p = pi p / L_i, p in [-N_i/2, N_i/2).  psi_in, psi_out: complex grids (may be the same
 * buffer).  dt may be negative (a step back in time); delta must be >= 0.  The first GPE call on
 * a plan allocates the GPE workspace.  Does not synchronise.
 */
ddi_status gpe_ts_step(ddi_plan_t plan, const gpe_params* gp, double dt, double delta,
                       const void* psi_in_dev, void* psi_out_dev, void* stream);

/*
 * The same step with the particle loss f(rho) = delta rho^q (Sec. 4.1, Case III of Eqs.
 * fun1-fun2; q = 1 two-body, q = 2 three-body), cubic nonlinearity, time-independent axis.  With
 * rho1 = |psi1|^2 the closed forms share one function
 *   w = [(1 + 2 q delta dt rho1^q)^(1 - 1/q) - 1] / (2 delta (q - 1) rho1^(q-1))   (q != 1),
 *   w = ln(1 + 2 delta dt rho1) / (2 delta)                                           (q = 1),
 * and psi2 = psi1 exp(-i [dt V + beta w + lambda (A w)]) (1 + 2 q delta dt rho1^q)^(-1/(2q)).
 * dt > 0, delta > 0 and q > 0 (finite) are required.  Otherwise as gpe_ts_step.
 */
ddi_status gpe_ts_step_loss(ddi_plan_t plan, const gpe_params* gp, double dt, double delta, double q,
                            const void* psi_in_dev, void* psi_out_dev, void* stream);

/*
 * Per-kernel timing of ddi_apply (sign = +1) or ddi_apply_adjoint (sign = -1):
 * runs the operator `reps` times on `stream` with HIP events between its
 * kernels and writes the mean duration in milliseconds of each stage to
 * stage_ms[DDI_NSTAGES] (host):
 *   0 last-axis FFT with deconvolution and zero-padding   5 spread reduce (split tiles)
 *   1 axis-1 FFT (pruned)                                 6 axis-0 FFT (pruned)
 *   2 axis-0 FFT (pruned; 0 in 2D)                        7 axis-1 FFT (pruned)
 *   3 interpolation at the nodes and weighting            8 last-axis FFT, truncation,
 *   4 spread to the fine grid                               deconvolution and real part
 * The outputs are the same as those of ddi_apply / ddi_apply_adjoint.  For a
 * split plan the stages are those of I_2; I_1 runs after stage 8 and is not
 * timed.  Synchronises `stream`.
 */
#define DDI_NSTAGES 9
ddi_status ddi_profile_apply(ddi_plan_t plan, const void* in_dev, void* out_dev, int32_t sign, int32_t reps,
                             double* stage_ms, void* stream);

/* Sizes and kernel parameters of a plan. */
ddi_status ddi_plan_info(ddi_plan_t plan, ddi_plan_info_t* info);

/* Host copies of the plan's node tables in plan order (any pointer may be NULL):
 *   index_host [M_eff][3] int32: (radial, polar, azimuthal) quadrature indices (polar = 0 in 2D)
 *   k_host     [M_eff][3] double: node k (k[2] = 0 in 2D)
 *   c_host     [M_eff] double: c_q = W_q Uhat(k_q)/(2 pi)^d */
ddi_status ddi_plan_nodes(ddi_plan_t plan, int32_t* index_host, double* k_host, double* c_host);

/* Release a plan and its device memory (NULL is ignored).  The caller must
 * make sure no work using the plan is still pending. */
void ddi_destroy(ddi_plan_t plan);

/* Message of the last failed call on this thread ("" if none). */
const char* ddi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDI_H */
