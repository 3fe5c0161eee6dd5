/*
 * phenomd.h — C ABI of the MI355X (gfx950) library for batched IMRPhenomD-structured
 * waveforms and the noise-weighted products built on them.
 *
 * Paper: "ripple: Differentiable and Hardware-Accelerated Waveforms for Gravitational
 * Wave Data Analysis" (arXiv:2302.05329).  The waveform is the aligned-spin IMRPhenomD
 * model the paper re-implements (Sec. 2); the products are the noise-weighted inner
 * product (Eq. 1), the Gaussian likelihood of the HMC study (Sec. 3.3), the Fisher matrix
 * (Sec. 3.2, Eq. 8) and the mismatch over the 209 fit coefficients (Sec. 3.1, Eqs. 2-5
 * and 7).
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller, unless stated.
 *     Arrays are dense, row-major, float64; complex arrays are interleaved (re, im).
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream) and is
 *     asynchronous: outputs are valid once the stream has synchronised.
 *   - The library allocates no device memory.  Calls that need scratch take a
 *     caller-owned `workspace` of at least the size the matching *_workspace_bytes()
 *     query returns; two calls that run concurrently must not share a workspace.
 *   - pd_loglike_and_grad and pd_mismatch_grad run two of the three phase-region
 *     launches of their per-bin pass, and pd_loglike_and_grad with a gradient also the record
 *     tangents, on side streams (default priority) created once per host thread and device,
 *     forked from and joined back to `stream` with events inside the call; the calls stay
 *     asynchronous and their results are ordered on `stream` as for any other call.  The calls
 *     built on them (the network, posterior, HMC, random-walk and coefficient-descent entries)
 *     inherit this.
 *   - A negative return value is a batch-level error (bad pointer, size, grid or
 *     enum); nothing is launched and pd_last_error() describes it.  Nothing throws.
 *   - Per-point physical-domain errors (non-finite input, masses <= 0, eta outside
 *     (0, 1/4], |chi| > 1, D <= 0, or a source whose model transition frequencies are
 *     out of order) do not fail the call: the point's outputs are NaN and, when a
 *     `status` array is given, status[i] = PD_EDOMAIN (else PD_OK).
 *   - The model is zero outside f_min <= f and M f <= 0.2 (M in seconds).
 */
#ifndef PHENOMD_H
#define PHENOMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PD_OK = 0,
    PD_EINVAL = -1,       /* bad argument: null pointer, size, grid, enum */
    PD_EDOMAIN = -2,      /* per-point: parameters outside the model's domain */
    PD_EHIP = -3,         /* a HIP runtime call failed */
    PD_ENOMEM = -4,       /* workspace too small */
    PD_EUNSUPPORTED = -5  /* valid but not supported (e.g. an FFT length that is not 2^6..2^16) */
} pd_status;

/* Arithmetic of the per-bin model.  Only PD_FP64 is implemented: the phase needs FP64 (its
 * summands reach 1e5 rad and the likelihood is sensitive to 1e-6 rad), and the amplitude shares the
 * phase's FP64 intermediates, so a separate FP32 amplitude path saves little on a pass bound by
 * FP64 issue.  PD_MIXED is reserved for that path and every entry point taking a precision
 * returns PD_EUNSUPPORTED for it, launching nothing. */
typedef enum {
    PD_FP64 = 0,   /* everything in FP64 */
    PD_MIXED = 1   /* reserved (FP32 amplitude ratio): PD_EUNSUPPORTED */
} pd_precision;

/* Layout of one parameter row theta[7]; derivatives are taken w.r.t. the same 7 numbers.
 * Masses in solar masses, D in Mpc, tc in s, phic in rad (orbital phase: h ~ exp(+2 i phic)). */
typedef enum {
    PD_PARAM_MC_ETA = 0,       /* (Mc, eta, chi1, chi2, D, tc, phic)           Sec. 3.3 set  */
    PD_PARAM_LNMC_ETA_LND = 1, /* (ln Mc, eta, chi1, chi2, ln D, tc, phic)     Fisher set    */
    PD_PARAM_MC_Q = 2,         /* (Mc, q = m2/m1, chi1, chi2, D, tc, phic)     sampler set   */
    PD_PARAM_M1M2 = 3          /* (m1, m2, chi1, chi2, D, tc, phic), unsorted               */
} pd_param;

/* Uniform frequency grid f_k = f0 + k*df (k < n_bins), f in Hz.  Bins with f_k < f_min
 * carry no signal; f_ref is the physical frequency where the phase is referenced.
 * 1 <= n_bins <= 2^28 (the per-bin tables are addressed with 32-bit byte offsets); a grid
 * outside that range is a batch-level error (PD_EINVAL). */
typedef struct {
    double f0;
    double df;
    int64_t n_bins;
    double f_min;
    double f_ref;
} pd_grid;

/* Operations for the workspace queries. */
typedef enum {
    PD_OP_WAVEFORM = 0,
    PD_OP_LOGLIKE = 1,        /* value only */
    PD_OP_LOGLIKE_GRAD = 2,
    PD_OP_FISHER = 3,
    PD_OP_MISMATCH_GRAD = 4
} pd_op;

/* Bytes of workspace an operation needs for n points (targets) on an n_bins grid. */
size_t pd_workspace_bytes(int op, int64_t n, int64_t n_bins);

/* Frequency-domain strain, Sec. 2 (the model the paper implements):
 *   h_k = A(f_k) exp(-i Psi(f_k)) for each parameter row.
 * theta   [n][7]              parameter rows, layout `param`
 * lambda  [209]               fit coefficients, 19 rows x 11 columns (Sec. 3.1)
 * h_out   [n][n_bins][2]      output, complex128 (zeros on inactive bins)
 * status  [n] int32 or NULL   per-point status (PD_OK / PD_EDOMAIN)
 */
int pd_waveform_eval(const double* theta, int64_t n, int param, const pd_grid* grid,
                     const double* lambda, int precision, double* h_out, int32_t* status,
                     void* workspace, size_t workspace_bytes, void* stream);

/* Gaussian log-likelihood of Sec. 3.3 with the inner product of Eq. 1 as a Riemann sum:
 *   lnL = (d|h) - (h|h)/2,  (a|b) = 4 df Re sum_k conj(a_k) b_k / S_k,
 * fused so the strain is never written, and optionally its gradient w.r.t. theta
 * (hand-written forward-mode tangents of the per-point coefficients contracted with
 * per-bin moments; Sec. 2 on derivatives).
 * data    [n_bins][2]         complex128 data d_k (shared by all points)
 * inv_psd [n_bins]            1 / S_n(f_k), one-sided PSD in 1/Hz
 * lnl     [n]                 output
 * grad    [n][7] or NULL      output d lnL / d theta (NULL: value only)
 */
int pd_loglike_and_grad(const double* theta, int64_t n, int param, const pd_grid* grid,
                        const double* lambda, const double* data, const double* inv_psd,
                        int precision, double* lnl, double* grad, int32_t* status,
                        void* workspace, size_t workspace_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): pd_loglike_and_grad with its workspace in a fixed
 * device array of PD_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on (one
 * copy per GPU, kept until the process ends).  Arguments and results as for pd_loglike_and_grad,
 * without the workspace; every launch is enqueued on `stream` (no side streams).
 * The call allocates nothing (no hipMalloc, hipFree, stream or event creation).  A batch whose
 * pd_loglike_and_grad workspace (pd_workspace_bytes) exceeds the array, e.g. more than about
 * 20 700 points on a 16 225-bin grid (4096 points x 8033 bins need 16.8 MB), returns
 * PD_EUNSUPPORTED and launches nothing.  All calls on one GPU share that GPU's array: calls
 * that overlap on one GPU (other streams, other host threads) race and must be serialised by
 * the caller.  Nothing in the array needs to be cleared between calls. */
#define PD_NOALLOC_SCRATCH_BYTES (64u << 20)
int pd_loglike_and_grad_noalloc(const double* theta, int64_t n, int param, const pd_grid* grid,
                                const double* lambda, const double* data, const double* inv_psd, int precision,
                                double* lnl, double* grad, int32_t* status, void* stream);

/* Fisher information of one detector, Sec. 3.2 Eq. 8: F_pq = (d_p h | d_q h),
 * p, q over the 7 entries of theta in layout `param`.
 * F       [n][7][7]           output, symmetric
 */
int pd_fisher(const double* theta, int64_t n, int param, const pd_grid* grid,
              const double* lambda, const double* inv_psd, double* F, int32_t* status,
              void* workspace, size_t workspace_bytes, void* stream);

/* Mismatch against fixed targets and its gradient w.r.t. the 209 fit coefficients,
 * Sec. 3.1 Eqs. 5 and 7:
 *   z_j = sum_k w_k conj(h_k) t_k exp(+2 pi i k j / N), j < N = n_bins,
 *   m = max_j |z_j| / sqrt((h|h)(t|t)),  M = 1 - m   (max over lag and phase),
 *   dsum_dlambda = sum over targets of dM / dlambda at the maximising lag.
 * n_bins must be a power of two from 2^6 to 2^16 (the FFT length; PD_EUNSUPPORTED otherwise).
 * theta        [nt][7]           source of each target (layout `param`)
 * targets      [nt][n_bins][2]   target strains t_k, complex128
 * inv_psd      [n_bins]          1 / S_n (use ones for a flat PSD)
 * mismatch     [nt]              output
 * dsum_dlambda [209] or NULL     output (NULL: mismatch only)
 * lag          [nt] int32 or NULL  output, maximising lag j* (ties: lowest j)
 */
int pd_mismatch_grad(const double* theta, int64_t nt, int param, const pd_grid* grid,
                     const double* lambda, const double* targets, const double* inv_psd,
                     double* mismatch, double* dsum_dlambda, int32_t* lag,
                     void* workspace, size_t workspace_bytes, void* stream);

/* One gradient-descent step on the 209 fit coefficients (Sec. 3.1, Eq. 6 on the mean loss of
 * Eq. 7):  L = (1/nt) sum_i M_i,  lambda_j <- lambda_j - alpha P_j dL/dlambda_j.
 * Arguments as for pd_mismatch_grad, except:
 * lambda       [209] device, in/out: read by the mismatch pass, then updated in place
 * alpha        learning rate (finite, >= 0)
 * precond      [209] device or NULL: per-coefficient factors P_j (NULL: P_j = 1, Eq. 6 as
 *              printed).  P_j = lambda0_j^2 makes the step Eq. 6 in the relative coordinates
 *              u_j = lambda_j / lambda0_j - 1 (dL/du_j = lambda0_j dL/dlambda_j).  Must not alias
 *              lambda or dsum_dlambda.
 * mismatch     [nt]  output: M_i at the coefficients on entry
 * dsum_dlambda [209] output (required, must not alias lambda): sum over targets of dM/dlambda
 *              at the coefficients on entry
 * Workspace as for PD_OP_MISMATCH_GRAD.  Steps issued on one stream run in order, so a loop
 * of calls is the descent of Sec. 3.1 with no host synchronisation.
 */
int pd_fit_lambda_step(const double* theta, int64_t nt, int param, const pd_grid* grid, double* lambda,
                       const double* targets, const double* inv_psd, double alpha, const double* precond,
                       double* mismatch, double* dsum_dlambda, void* workspace, size_t workspace_bytes,
                       void* stream);

/* ---------------------------------------------------------------------------------------
 * Detector network: the two-detector injection of Sec. 3.3 and the network setups of the
 * Fisher forecasts (Sec. 3.2).  The paper does not print the detector response; the one used
 * is the standard response to the dominant (2,2) mode:
 *   h_d(f) = (F+ h+ + Fx hx) exp(-2 pi i f dt_d),  h+ = h0 (1 + cos^2 iota)/2,  hx = -i cos iota h0,
 * with h0 the face-on, optimally oriented strain of pd_waveform_eval, the antenna patterns
 *   F+ = D : (XX - YY),  Fx = D : (XY + YX),  D = (x x^T - y y^T)/2  (unit arm vectors x, y),
 * in the Earth-fixed frame: source direction n = (cos dec cos l, cos dec sin l, sin dec),
 * l = ra - gmst; a = (sin l, -cos l, 0), b = n x a; X = cos psi a + sin psi b,
 * Y = -sin psi a + cos psi b; and the arrival delay dt_d = -(r_d . n)/c at the site vertex r_d.
 * Network ln L = sum over sites of (d_d|h_d) - (h_d|h_d)/2 (Eq. 1 per site).
 * ------------------------------------------------------------------------------------- */
#define PD_NETWORK_MAX_DETECTORS 8

typedef struct {
    double vertex[3];   /* site position, Earth-fixed Cartesian, metres */
    double xarm[3];     /* unit vector along the x arm */
    double yarm[3];     /* unit vector along the y arm */
} pd_detector;

size_t pd_network_workspace_bytes(int64_t n, int64_t n_bins, int n_det);

/* Network ln L and its gradient over 11 parameters for n points.
 * theta     [n][11]          the 7 entries of layout `param`, then (iota, psi, ra, dec) in rad
 * n_det     1..PD_NETWORK_MAX_DETECTORS;  detectors [n_det] HOST array
 * gmst      Greenwich sidereal angle at the reference time (rad)
 * data      [n_det][n_bins][2]  complex128 data of each site;  inv_psd [n_det][n_bins]
 * lnl [n]; grad [n][11] or NULL (value only); status [n] or NULL (PD_OK / PD_EDOMAIN with NaN
 *           outputs for a point outside the model's domain).  A site whose response
 *           F+ (1+cos^2 iota)/2 - i Fx cos iota is exactly zero records no signal and adds nothing.
 * Each site runs one fused pass of pd_loglike_and_grad at the site's effective parameters
 * (D / |c|, tc + dt, phic + arg(c)/2 with c the complex response above), one after another on
 * `stream`.  Workspace: pd_network_workspace_bytes(n, n_bins, n_det), 256-byte aligned.
 */
int pd_network_loglike_and_grad(const double* theta, int64_t n, int param, const pd_grid* grid,
                                const double* lambda, int n_det, const pd_detector* detectors, double gmst,
                                const double* data, const double* inv_psd, double* lnl, double* grad,
                                int32_t* status, void* workspace, size_t workspace_bytes, void* stream);

size_t pd_network_strain_workspace_bytes(int64_t n, int64_t n_bins);

/* Strain recorded at one site, h_d(f) = (F+ h+ + Fx hx) exp(-2 pi i f dt) (the response above),
 * for n rows theta [n][11]; h_out [n][n_bins][2] complex128 (zeros on inactive bins); status [n]
 * or NULL.  Computed as pd_waveform_eval at the site's effective parameters.
 * Workspace: pd_network_strain_workspace_bytes(n, n_bins), 256-byte aligned. */
int pd_network_strain(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                      const pd_detector* detector, double gmst, double* h_out, int32_t* status, void* workspace,
                      size_t workspace_bytes, void* stream);

size_t pd_network_fisher_workspace_bytes(int64_t n, int64_t n_bins, int n_det);

/* Network Fisher matrix over the same 11 parameters (Eq. 8 summed over sites):
 *   F_pq = sum over sites of (d_p h_d | d_q h_d),
 * computed as sum over sites of J^T F_d J with F_d the single-site Fisher matrix (pd_fisher) at
 * the site's effective parameters and J the 7 x 11 Jacobian of those parameters.
 * theta [n][11], detectors, gmst, inv_psd [n_det][n_bins] as for pd_network_loglike_and_grad;
 * F [n][11][11] output (symmetric); status [n] or NULL.
 * Workspace: pd_network_fisher_workspace_bytes(n, n_bins, n_det), 256-byte aligned.
 */
int pd_network_fisher(const double* theta, int64_t n, int param, const pd_grid* grid, const double* lambda,
                      int n_det, const pd_detector* detectors, double gmst, const double* inv_psd, double* F,
                      int32_t* status, void* workspace, size_t workspace_bytes, void* stream);

/* Per-point model quantities used to account the work of a batch (Sec. 2): for each row,
 * out[i] = {M T_sun [s], Mf of the phase join intermediate->merger-ringdown (f_RD / 2),
 *           Mf of the amplitude join intermediate->merger-ringdown (f_peak), valid (1/0)}.
 * out     [n][4]              output
 * Workspace as for PD_OP_WAVEFORM.
 */
int pd_transition_frequencies(const double* theta, int64_t n, int param, const pd_grid* grid,
                              const double* lambda, double* out, void* workspace,
                              size_t workspace_bytes, void* stream);

/* Kernel timing for benchmarks.  While enabled, every call brackets its dominant per-bin
 * kernel with HIP events recorded on the call's own stream.  pd_profile_read() waits for
 * the recorded events, returns the summed elapsed time (ms) and launch count of one kernel
 * and clears its record.  Kernel ids: */
enum {
    PD_K_LOGLIKE_GRAD = 0,    /* fused lnL + gradient moments */
    PD_K_LOGLIKE = 1,         /* fused lnL (value only) */
    PD_K_FISHER = 2,          /* Fisher accumulation */
    PD_K_WAVEFORM = 3,        /* strain output */
    PD_K_MISMATCH_INPUT = 4,  /* overlap input (model per bin) fused with the column FFT pass */
    PD_K_MISMATCH_FFT = 5,    /* row FFT pass with the fused arg-max */
    PD_K_MISMATCH_ADJ = 6,    /* mismatch adjoint moments */
    PD_K_OVERLAP = 7,         /* template-bank overlap GEMM (generation + FP64 MFMA) */
    PD_K_COUNT = 8
};
int pd_profile_enable(int on);
int pd_profile_read(int kernel, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------------------------
 * Sampling (Sec. 3.3).  A posterior in unconstrained coordinates x in R^7:
 *   PD_TARGET_GW     theta = (Mc, q, chi1, chi2, D, tc, phic) with theta_i = lo_i +
 *                    (hi_i - lo_i) sigmoid(x_i) for i < 6 (uniform priors) and phic = x_6;
 *                    log pi(x) = lnL(theta(x)) + log |d theta / d x|, lnL as in
 *                    pd_loglike_and_grad (FP64).
 *   PD_TARGET_GW_NETWORK  as PD_TARGET_GW with lnL the network likelihood of
 *                    pd_network_loglike_and_grad over n_det sites, the orientation and sky
 *                    position (iota, psi, ra, dec) held at `orient` (the two-detector
 *                    injection of Sec. 3.3 fixes them); data [n_det][n_bins][2] and
 *                    inv_psd [n_det][n_bins].
 *   PD_TARGET_GAUSS  log pi(x) = -1/2 sum_j (x_j - mu_j)^2 isig2_j (tests the samplers
 *                    against a known answer).
 * Random numbers are inputs: every call is a deterministic function of its arguments.
 * ------------------------------------------------------------------------------------- */
typedef enum { PD_TARGET_GW = 0, PD_TARGET_GAUSS = 1, PD_TARGET_GW_NETWORK = 2 } pd_target;

typedef struct {
    int kind;                 /* pd_target */
    pd_grid grid;             /* GW: frequency grid of data and inv_psd */
    const double* lambda;     /* GW: [209] device */
    const double* data;       /* GW: [n_bins][2] device (GW_NETWORK: [n_det][n_bins][2]) */
    const double* inv_psd;    /* GW: [n_bins] device (GW_NETWORK: [n_det][n_bins]) */
    double lo[7], hi[7];      /* GW: prior bounds of (Mc, q, chi1, chi2, D, tc, phic); 0 < q <= 1.
                                 The likelihood has period pi in phic, so a phic interval of
                                 length pi is the whole circle. */
    double mu[7], isig2[7];   /* GAUSS: means and inverse variances */
    int n_det;                /* GW_NETWORK: number of sites, 1..PD_NETWORK_MAX_DETECTORS */
    pd_detector detectors[PD_NETWORK_MAX_DETECTORS];  /* GW_NETWORK: site geometry */
    double gmst;              /* GW_NETWORK: Greenwich sidereal angle at the reference time */
    double orient[4];         /* GW_NETWORK: fixed (iota, psi, ra, dec) */
} pd_posterior;

size_t pd_posterior_workspace_bytes(const pd_posterior* post, int64_t n);

/* log pi(x) [n] and its gradient [n][7] (or NULL) for n points x [n][7]. */
int pd_posterior_logp(const pd_posterior* post, const double* x, int64_t n, double* logp, double* grad,
                      void* workspace, size_t workspace_bytes, void* stream);

size_t pd_hmc_workspace_bytes(const pd_posterior* post, int64_t n);

/* One Hamiltonian Monte Carlo transition for n independent chains (Sec. 3.3; leapfrog
 * integrator with a diagonal mass matrix, Metropolis accept on the Hamiltonian):
 *   p ~ N(0, diag(mass));  n_leapfrog leapfrog steps of size eps;  accept if log u < -dH,
 * with H = -log pi(x) + sum_j p_j^2 / (2 mass_j).
 * x [n][7], logp [n], grad [n][7]   in/out: the chains' state with its cached log pi and
 *                                   gradient (from pd_posterior_logp or a previous step)
 * xi [n][7]      standard-normal momentum draws (p_j = sqrt(mass_j) xi_j);  u [n] uniform(0,1) draws
 * mass [7]       HOST array, diagonal mass matrix
 * accepted [n]   out (or NULL): 1 accepted, 0 rejected, -1 rejected as divergent
 *                (non-finite dH or |dH| > 1000)
 * dh [n]         out (or NULL): H(end) - H(start)
 */
int pd_hmc_step(const pd_posterior* post, int64_t n, double* x, double* logp, double* grad, const double* xi,
                const double* u, int n_leapfrog, double eps, const double* mass, int32_t* accepted,
                double* dh, void* workspace, size_t workspace_bytes, void* stream);

/* As pd_hmc_step with a dense metric: the inverse mass matrix (the covariance the momenta move
 * along) is L L^T for the row-major lower-triangular chol [7][7] (HOST array, positive diagonal;
 * entries above the diagonal are ignored), i.e. p ~ N(0, (L L^T)^-1) and
 * H = -log pi(x) + p^T L L^T p / 2.  The chains carry r = L^T p = xi, so the drift is
 * x += eps L r and the kick r += eps L^T grad log pi.  With L the Cholesky factor of the posterior
 * covariance the trajectories see an isotropic target.  Workspace as pd_hmc_workspace_bytes.
 * PD_EINVAL (nothing launched) for a NULL chol, a non-finite entry or a non-positive diagonal. */
int pd_hmc_step_dense(const pd_posterior* post, int64_t n, double* x, double* logp, double* grad, const double* xi,
                      const double* u, int n_leapfrog, double eps, const double* chol, int32_t* accepted,
                      double* dh, void* workspace, size_t workspace_bytes, void* stream);

size_t pd_rwmh_workspace_bytes(const pd_posterior* post, int64_t n);

/* One random-walk Metropolis-Hastings transition for n independent chains: the baseline
 * sampler that Sec. 3.3 compares HMC with (Metropolis et al. 1953, Gaussian steps):
 *   x' = x + scale * xi (per coordinate);  accept if log u < log pi(x') - log pi(x).
 * A non-finite log pi(x') rejects; a chain whose log pi is not finite takes any finite x'.
 * x [n][7], logp [n]   in/out: the chains' state and its cached log pi (from
 *                      pd_posterior_logp or a previous step)
 * xi [n][7]      standard-normal step draws;  u [n] uniform(0,1) draws
 * scale [7]      HOST array, step standard deviation per coordinate (finite, >= 0)
 * accepted [n]   out (or NULL): 1 accepted, 0 rejected
 * Uses log pi only (value-only likelihood); a cached gradient of the chains is not updated.
 */
int pd_rwmh_step(const pd_posterior* post, int64_t n, double* x, double* logp, const double* xi, const double* u,
                 const double* scale, int32_t* accepted, void* workspace, size_t workspace_bytes, void* stream);

/* As pd_rwmh_step with correlated Gaussian steps x' = x + L xi, the proposal covariance L L^T
 * given by the row-major lower-triangular chol [7][7] (HOST array, finite; entries above the
 * diagonal are ignored).  Workspace as pd_rwmh_workspace_bytes.  PD_EINVAL (nothing launched)
 * for a NULL chol or a non-finite entry. */
int pd_rwmh_step_dense(const pd_posterior* post, int64_t n, double* x, double* logp, const double* xi,
                       const double* u, const double* chol, int32_t* accepted, void* workspace, size_t workspace_bytes,
                       void* stream);

/* Independence Metropolis-Hastings accept (the learned proposal of the sampler): for each
 * chain, accept x' (drawn from q) with probability min(1, pi(x') q(x) / (pi(x) q(x'))).
 * x [n][7], logp [n], logq [n]   in/out current state, log pi and log q at it
 * xp [n][7], logp_p [n], logq_p [n]  proposals with their log pi and log q
 * grad [n][7], grad_p [n][7]  (both NULL, or both set) gradient of log pi at the current
 *                state (in/out) and at the proposals, carried along so that HMC can continue
 * u [n] uniform(0,1) draws;  accepted [n] out (or NULL)
 */
int pd_independence_mh(int64_t n, double* x, double* logp, double* logq, double* grad, const double* xp,
                       const double* logp_p, const double* logq_p, const double* grad_p, const double* u,
                       int32_t* accepted, void* stream);

/* ---------------------------------------------------------------------------------------
 * Learned proposal: a RealNVP normalising flow on R^7 (the flow + GPU + gradient-sampler
 * combination announced at the end of Sec. 3.3).  Fixed architecture: standardisation
 * y = (x - mu) isd, then 8 affine coupling layers alternately conditioning on dims {0,1,2}
 * and {3..6}, each with an MLP 7 -> 128 -> 128 -> 14 (tanh hidden units), log-scale bounded
 * as 2 tanh(./2).  log q(x) = log N(z; 0, I) + sum of log-determinants + sum log isd.
 * params: float32, per layer W1[7][128] b1[128] W2[128][128] b2[128] W3[128][14] b3[14],
 * 8 layers, then mu[7] and isd[7] (not trained).  x, z, log q in FP64.
 * mode: PD_FLOW_FP32 (all FP32 arithmetic) or PD_FLOW_BF16 (the hidden and output layers,
 * and in training their gradient products, on the bfloat16 matrix cores with FP32
 * accumulation; the rest FP32).  In either mode a fixed parameter vector defines a bijection
 * whose log-determinant is the sum of the log-scales (s and t depend only on the dims a layer
 * keeps), so the flow is a valid independence proposal; use the same mode for sampling and
 * for log q.  Inverse-then-forward reproduces z to rounding except where rounding of the data
 * coordinates moves an operand across a bfloat16 rounding boundary (then at bfloat16 level).
 * ------------------------------------------------------------------------------------- */
typedef enum { PD_FLOW_FP32 = 0, PD_FLOW_BF16 = 1 } pd_flow_mode;
int64_t pd_flow_param_count(void);
size_t pd_flow_workspace_bytes(int64_t n);

/* data -> latent: z [n][7] (or NULL) and log q(x) [n] for x [n][7]. */
int pd_flow_forward(const float* params, const double* x, int64_t n, double* z, double* logq, int mode,
                    void* stream);

/* latent -> data: x [n][7] = f^-1(z) and log q(x) [n], for z [n][7] (standard-normal draws). */
int pd_flow_sample(const float* params, const double* z, int64_t n, double* x, double* logq, int mode,
                   void* stream);

/* Maximum-likelihood training objective loss = -mean_b log q(x_b) over x [n][7] and its
 * gradient grad [P] w.r.t. params (the 14 standardisation entries get zero); loss [1] or NULL.
 * Workspace of pd_flow_workspace_bytes(n). */
int pd_flow_loss_grad(const float* params, const double* x, int64_t n, float* grad, double* loss,
                      void* workspace, size_t workspace_bytes, int mode, void* stream);

/* Adam (Kingma & Ba 2015) on count float32 parameters, step t >= 1 (bias-corrected). */
int pd_adam_step(float* params, const float* grad, float* m, float* v, int64_t count, double lr,
                 double beta1, double beta2, double eps, int64_t t, void* stream);

/* ---------------------------------------------------------------------------------------
 * Template-bank overlaps (Eq. 1 for many templates against many data streams), the one dense
 * contraction of the path:
 *   overlap[t][s] = sum_k w_k conj(h_t(f_k)) d_s(f_k),  w_k = 4 df inv_psd[k],
 * so Re overlap = (h_t | d_s), |overlap| is the phase-maximised overlap, and with
 * hh[t] = (h_t | h_t) one has ln L[t][s] = Re overlap[t][s] - hh[t] / 2.  Templates are
 * generated in registers/LDS and contracted on the FP64 matrix cores; they are never stored.
 * theta [nt][7] in the pd_param parameterisation, data [ns][n_bins][2] complex, 1 <= ns <= 64;
 * overlap [nt][ns][2] out; hh [nt] out or NULL; status [nt] out or NULL (domain errors give
 * NaN rows).  Templates ordered by total mass run faster (each block of 64 contracts only the
 * bins where one of its templates is active).
 * ------------------------------------------------------------------------------------- */
#define PD_OVERLAP_MAX_STREAMS 64
size_t pd_overlap_workspace_bytes(int64_t nt, int64_t ns, int64_t n_bins);
int pd_overlap(const double* theta, int64_t nt, int param, const pd_grid* grid, const double* lambda,
               const double* data, int64_t ns, const double* inv_psd, double* overlap, double* hh,
               int32_t* status, void* workspace, size_t workspace_bytes, void* stream);

/* Diagnostic: the kernels' own FP64 elementary functions applied elementwise, out[i] = fn(x[i])
 * for x [n], out [n] (device).  fn: PD_FN_SIN, PD_FN_COS (one shared argument reduction by
 * pi/256 with a two-part split, then a 512-entry (sin, cos) table and short polynomials;
 * |x| > 2^24 falls back to the device library), PD_FN_ATAN (two-level reduction: 1/u above 1,
 * then pi/6 above tan(pi/12), and an 11-term polynomial), PD_FN_ATAN_TABLE (the form the fused
 * likelihood's merger-ringdown loop uses: atan c + atan((|u| - c)/(1 + |u| c)) with c from a
 * 321-entry table indexed by the exponent and top mantissa bits of |u|, and a 3-term
 * polynomial), PD_FN_EXP, PD_FN_RCP (hardware estimate + two Newton steps).  Exposed so that
 * their ulp error can be measured against a high-precision reference.  Unknown fn:
 * PD_EINVAL. */
typedef enum {
    PD_FN_SIN = 0,
    PD_FN_COS = 1,
    PD_FN_ATAN = 2,
    PD_FN_EXP = 3,
    PD_FN_RCP = 4,
    PD_FN_ATAN_TABLE = 5
} pd_fn;
int pd_elementary_eval(int fn, const double* x, int64_t n, double* out, void* stream);

/* Text of the last batch-level error on the calling thread (library-owned, never NULL). */
const char* pd_last_error(void);

/* Library version string (library-owned). */
const char* pd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PHENOMD_H */
