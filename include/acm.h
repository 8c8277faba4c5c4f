/*
 * acm.h - C ABI of the MI355X (gfx950) unit-cell solvers for periodic porous
 * media, following Karimi & Bhattacharya, "Accelerated Computational
 * Micromechanics for Reactive Flow in Porous Media" (arXiv 2312.15554).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Unit cell Y = [0,1)^d (Section 2), grid n[0] x n[1] (x n[2]) voxels,
 *   h_j = 1/n_j.  Every n_j must be one of 8, 16, 24, 32, 48, 64, 96, 128,
 *   192, 256, 512; nx = n[0] must also be at most 512.  dim is 2 or 3; for
 *   dim 2 set n[2] = 1.
 * - Real fields are structure-of-arrays [component][z][y][x], x fastest, in
 *   the precision selected by `precision` (ACM_FP32: float, ACM_FP64: double).
 *   Half spectra are [field][z][y][x_half] of interleaved complex values with
 *   x_half = nx/2 + 1.
 * - H is the solid indicator of Section 3 (eq. Heaviside): one uint8 per
 *   voxel, 1 = solid, 0 = pore, same [z][y][x] order.
 * - ALL array arguments except the small double arrays (g, B0, K, D, mass,
 *   history) are DEVICE pointers on the current HIP device.  The caller owns
 *   every buffer; the library owns only its internal workspace and tables.
 * - `stream` is a hipStream_t (NULL = default stream).  Every call is ordered
 *   after prior work on `stream` and returns only when its results are
 *   complete (the call synchronises).
 * - Derivatives use the central-difference symbol s_j = sin(2 pi m_j/n_j)/h_j
 *   for first derivatives and the compact symbol 4 sin^2(pi m_j/n_j)/h_j^2 for
 *   second derivatives (Section 3.2, eq. fft_app), for both problems.
 * - No exception or abort crosses the ABI.  On a negative status, outputs are
 *   left untouched and acm_last_error() describes the failure.
 */
#ifndef ACM_H_
#define ACM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ACM_OK = 0,
  ACM_NOT_CONVERGED = 1,       /* max_iter reached; outputs hold the last iterate */
  ACM_E_INVALID = -1,          /* bad argument (null pointer, bad dim, all-pore H, ...) */
  ACM_E_UNSUPPORTED_SIZE = -2, /* grid length not in the supported set */
  ACM_E_NOMEM = -3,            /* device allocation failed */
  ACM_E_HIP = -4,              /* a HIP runtime call failed */
  ACM_E_DIVERGED = -5          /* a residual became non-finite */
} acm_status;

enum { ACM_FP32 = 0, ACM_FP64 = 1 };

typedef struct {
  int32_t dim;  /* 2 or 3 */
  int32_t n[3]; /* nx, ny, nz (nz = 1 when dim = 2) */
} acm_grid;

/* ADMM penalties (Section 3.1, eq. Lagrangian with auxiliary variable) and
 * their adaptive update (Section 4.1, eq. varying algorithm).  Order of every
 * triple: {alpha, beta, b}; alpha pairs with constraint 1 (ut = 0 in the
 * solid), beta with constraint 2 (div u = 0), b with constraint 3 (u = ut). */
typedef struct {
  double alpha, beta, b;  /* initial penalties; <= 0 selects nu * max(n) */
  double phi[3];          /* growth factors (paper: 1.1) */
  double tau[3];          /* ratio thresholds (paper: {20,10,30} model cell, {5,10,5} random) */
  double psi_min[3];      /* floors; <= 0 selects 1e-3 * initial value */
  int32_t adaptive;       /* 0: fixed penalties */
} acm_penalty;

typedef struct {
  double eps;           /* epsilon = eps_abs = eps_rel of the stopping test (Section 3.1, Step 4) */
  int64_t max_iter;     /* iteration cap (per time step for transport) */
  int32_t precision;    /* ACM_FP32 or ACM_FP64: field and transform precision */
  int32_t check_every;  /* iterations between host convergence checks; 0 = automatic */
  int32_t warm_start;   /* Stokes only: 1 = u (and q if non-NULL) hold an initial guess */
  int32_t use_graph;    /* 1 = replay the iterations as a captured HIP graph */
  int32_t profile;      /* 1 = launch eagerly and time every kernel kind with HIP events */
  int32_t history_cap;  /* > 0: keep the residuals of the last history_cap iterations */
  int32_t pass_mode;    /* Stokes 3D: 0 automatic, 1 separate x and y passes,
                           2 fused xy-slab passes (needs nx == ny <= 128 and
                           16-byte aligned u and H; otherwise ACM_E_INVALID),
                           3 fused xy-slab passes with the local and rhs passes
                           in one launch joined by a device-wide gate (needs, in
                           addition, a single cell whose nz * 3 workgroups are
                           all resident at once; otherwise ACM_E_INVALID),
                           4 fused xy-slab passes where, after the first 64
                           iterations, a one-workgroup kernel forms Step 4 in
                           place of the rhs pass (the local pass has formed r
                           with the b of its iteration); a Step 4 that changes
                           b (rare after the first iterations) holds the
                           iterations until the host has formed r again.  Same
                           iterates as 2, bit for bit (needs a single cell;
                           otherwise ACM_E_INVALID).
                           5 row-step passes (any grid, a single cell with
                           32-byte aligned u and 16-byte aligned H; otherwise
                           ACM_E_INVALID): one pass over x rows takes the
                           spectra back to real space, applies Steps 2-3 and
                           forms the next right-hand side with the b of its
                           iteration, transformed in place (y transforms in
                           their own passes in 3D); a one-workgroup kernel
                           forms Step 4, and only when that changes b is the
                           right-hand side formed again.
                           Automatic picks 4 for a single cell where the
                           slab passes apply, 2 for a batch of such cells,
                           5 for any other single 3D cell, else 1. */
  int32_t green_variant; /* Stokes: kernel of the last-axis (green) pass. 0 automatic:
                           the first solve of a grid times every variant over a few
                           iterations and keeps the fastest for that grid; 1-3 force
                           the LDS-staged kernel with the default, half and double
                           pencil count per workgroup; 4-5 force the register-resident
                           kernel with the default and half pencil count (lengths with
                           a radix-3 factor use the LDS-staged kernel instead); 6-7
                           force the LDS-staged kernel with one thread group per
                           field during the transforms (default and half pencil
                           count).  All variants compute the same iterates up to
                           rounding. */
  int32_t derivative;   /* derivative symbols: 0 the central-difference symbol and
                           compact Laplacian (Section 3.2, eq. fft_app; the
                           paper's scheme), 1 the exact spectral symbols i k and
                           |k|^2 (the exact-FFT alternative of Section 4).  The
                           Stokes warm start needs 0; the transport slab form
                           folds central differences and is replaced by the row
                           form with 1. */
  int32_t step1_form;   /* Stokes: 0 automatic (2 for FP32 with pass modes 2, 4
                           and 5, else 1); 1 Step 1 solved
                           for u from r = b ut - a (the paper's form); 2 increment
                           form: while b is unchanged the spectra carry the change
                           X of Step 1's right-hand side since the last solve and
                           Step 1 is solved for the change of u, which the local
                           pass adds to u (the same iterates in exact arithmetic;
                           FP32 transforms then round quantities that vanish at
                           convergence instead of the O(1) reaction in the solid,
                           so the residuals keep falling below the FP32 floor of
                           form 1); the first 64 iterations, and an iteration
                           after a change of b, are in form 1.
                           Form 2 needs pass mode 2, 4 or 5 (ACM_E_INVALID otherwise). */
  int32_t transport_form; /* transport: 0 the literal form (Section 3.2 with the
                           central symbols: the divergence of (A - A0)(grad chi +
                           g) by central differences, so A0 leaves an O(h^2) term
                           in the fixed point); 1 the flux form: the diffusive
                           flux through each face is A_f (D+ chi + g) with the
                           forward difference D+ and the harmonic mean A_f of the
                           two voxels' diffusivities, its divergence the backward
                           difference, so the fixed point does not depend on A0
                           or B0 and pure diffusion conserves solute mass exactly
                           (advection keeps the central gradient).  Form 1 needs
                           derivative 0 and runs the row form of the passes. */
} acm_opts;

/* Kernel kinds reported in acm_stats.kernel_ms (with opts.profile = 1).  Each
 * kernel is timed by start/stop events attached to its own dispatch; those
 * include a per-launch overhead of a few microseconds, which ACM_K_OTHER
 * measures on an empty kernel launched the same way once per iteration. */
enum {
  ACM_K_GREEN = 0,   /* Stokes: last-axis FFT pair + Step 1 + q update */
  ACM_K_LOCAL = 1,   /* Stokes: x inverse transform + Steps 2-3 (+ Step 4 on the row
                        path; local and rhs together with pass_mode 3) */
  ACM_K_RHS = 2,     /* Stokes: (Step 4 on the slab path +) right-hand side of Step 1
                        + x forward transform; with pass_mode 4 also the Step 4
                        kernel */
  ACM_K_YINV = 3,    /* y inverse transform (3D) */
  ACM_K_YFWD = 4,    /* y forward transform (3D) */
  ACM_K_T_GREEN = 5, /* transport: last-axis FFT pair + LS update */
  ACM_K_T_LOCAL = 6, /* transport: x transforms + local residual F */
  ACM_K_OTHER = 7    /* Stokes profiling: the empty calibration kernel */
};

typedef struct {
  int64_t iters;        /* iterations performed (summed over time steps for transport) */
  double r_p[3], r_d[3];        /* last primal/dual residuals (transport: r_1, r_2 in r_p[0..1]) */
  double tol_p[3], tol_d[3];    /* their tolerances */
  double psi[3];                /* penalties after the last iteration */
  double seconds;               /* wall time of the iteration loop */
  int32_t converged;
  int32_t status;
  double kernel_ms[8];          /* opts.profile: summed kernel time per kind */
  int64_t kernel_calls[8];
} acm_stats;

/* Fill *p / *o with the defaults (adaptive, phi = 1.1, tau = {5,10,5},
 * eps = 1e-6, FP32, HIP graph on). */
void acm_default_penalty(acm_penalty* p);
void acm_default_opts(acm_opts* o);

/* Message of the last failing call on this thread ("" if none).  Valid until
 * the next call on the same thread. */
const char* acm_last_error(void);

/* ABI version (incremented on any signature or struct change): 6. */
int32_t acm_version(void);

/*
 * Unit-cell Stokes flow (Section 2, eq. unit cell, first two lines) solved on
 * the extended domain by ADMM (Section 3.1: Steps 1-4, eq. FFT step1,
 * eq. u_tilde, eq. Lagrange-multipliers, eq. constrains) with adaptive
 * penalties (Section 4.1, eq. varying algorithm).
 *   grid   cell size; H   solid indicator (device, ntot bytes, needs >= 1 solid voxel)
 *   g_p    body force / imposed pressure gradient, dim entries used
 *   nu     viscosity (> 0)
 *   pen    penalties (NULL = defaults); opts (NULL = defaults)
 *   u      inout device field, dim components: on entry the initial guess if
 *          opts->warm_start, otherwise ignored; on exit the velocity.
 *   q      out device scalar field (may be NULL): the pressure multiplier q.
 *          With warm_start it is also read as the initial guess.
 *   stats  out (may be NULL); history: host array of history_cap*15 doubles
 *          (may be NULL): per iteration r_p[3], r_d[3], tol_p[3], tol_d[3],
 *          psi[3], oldest first.
 * Convergence: every residual within its tolerance (all six, Step 4).
 * Returns ACM_OK, ACM_NOT_CONVERGED (outputs valid), or a negative status.
 */
acm_status acm_stokes_solve(const acm_grid* grid, const uint8_t* H, const double* g_p, double nu,
                            const acm_penalty* pen, const acm_opts* opts, void* u, void* q,
                            acm_stats* stats, double* history, void* stream);

/*
 * Many independent Stokes cells (possibly of different sizes) in one call.
 * Cells with the same grid share every launch of a pass (the cell index is a
 * grid dimension of each kernel); different sizes run as parallel branches of
 * one captured HIP graph.  Each cell keeps its own control block: penalties,
 * residuals and convergence are per cell (as acm_stokes_solve), and a cell
 * that has converged is skipped by every later launch.
 *   ncell  number of cells; grids[i] its grid; H[i], u[i] device pointers
 *   g_p    host array ncell x 3 (entries beyond a cell's dim ignored)
 *   q      NULL or array of ncell device pointers (entries may be NULL)
 *   stats  NULL or host array of ncell records; stats[i].seconds is the time
 *          from the first iteration until cell i was seen converged.
 * Returns ACM_OK if every cell converged, ACM_NOT_CONVERGED if any did not
 * (per-cell status in stats), or a negative status.
 */
acm_status acm_stokes_solve_batched(int32_t ncell, const acm_grid* grids, const uint8_t* const* H,
                                    const double* g_p, double nu, const acm_penalty* pen,
                                    const acm_opts* opts, void* const* u, void* const* q,
                                    acm_stats* stats, void* stream);

/*
 * Penalised advection-diffusion (Section 3.2, eq. penalization) by the
 * Lippmann-Schwinger iteration (eq. iter solved by eq. fft_solute, stopping
 * test eq. tol_solute):
 *   A = diffusivity (1-H) + eta H,  B = Pe (1-H) u,  calF = Pe (1-H) ubar . g_chi.
 *   dt = +INFINITY: the steady cell problem (mean-zero chi); n_steps must be 1.
 *   dt finite: n_steps backward-Euler steps of d chi/dt + operator = calF,
 *   each converged by the LS iteration with comparison symbol
 *   1/dt + A0 L + i B0 . s.
 *   u    device flow field (dim components, as passed: no normalisation)
 *   chi  inout device scalar field: initial value on entry, result on exit.
 *   A0 > 0; B0: dim entries (host).
 * The LS iteration contracts only for a large enough comparison medium A0
 * (Section 3.2); ACM_E_DIVERGED is returned as soon as r_1 becomes non-finite
 * or grows a millionfold over its smallest value within a time step.
 */
acm_status acm_transport_step(const acm_grid* grid, const uint8_t* H, const void* u,
                              const double* g_chi, double Pe, double diffusivity, double eta,
                              double A0, const double* B0, double dt, int32_t n_steps,
                              const acm_opts* opts, void* chi, acm_stats* stats, void* stream);

/*
 * Effective properties (Section 2, eq. K and eq. D), FP64 reductions.
 *   K (host, n_flow x dim, row i = flow i):  K_ij = (1/nu) h^d sum_Y u^i_j
 *     (equals the integral of grad u^i . grad u^j at a converged solution).
 *   D (host, dim x n_chi, column j = chi^j):
 *     D_ij = porosity delta_ij + Pe h^d sum_pore (ubar_i - u_i) chi^j
 *            + h^d sum_pore (grad_c chi^j)_i
 *     with u = u_transport (the flow used for chi) and grad_c the central
 *     difference.  mass (host, n_chi): h^d sum_Y chi^j.
 *   Any of K / D / mass may be NULL to skip it.
 */
acm_status acm_effective_props(const acm_grid* grid, int32_t precision, const uint8_t* H,
                               int32_t n_flow, const void* const* u, int32_t n_chi,
                               const void* const* chi, const void* u_transport, double nu,
                               double Pe, double* K, double* D, double* mass, void* stream);

/*
 * acm_effective_props without any allocation, for callers that cannot
 * allocate memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and error statuses as
 * acm_effective_props, bit for bit, with two differences:
 *   - at most 16 flows and 16 chi fields per call (ACM_E_INVALID beyond);
 *   - the kernels run on `stream` itself (the caller's stream, NULL = the
 *     default stream); the call returns after synchronising it.
 * The FP64 partial sums live in a fixed 36,864-byte device array that the
 * library holds on every GPU it runs on until the process ends; nothing is
 * allocated on the host or the device on the success path (the device address
 * of the array is looked up once per device on the first call).  Calls that
 * overlap on one GPU share that array and race: serialise them.
 */
acm_status acm_effective_props_noalloc(const acm_grid* grid, int32_t precision, const uint8_t* H,
                                       int32_t n_flow, const void* const* u, int32_t n_chi,
                                       const void* const* chi, const void* u_transport, double nu,
                                       double Pe, double* K, double* D, double* mass,
                                       void* stream);

/* Multi-dimensional real FFT of nfields fields (forward unnormalised /
 * inverse normalised by 1/ntot), half spectra as described above.  These are
 * the transforms every solver pass is built from. */
acm_status acm_fft_r2c(const acm_grid* grid, int32_t precision, int32_t nfields, const void* in,
                       void* out, void* stream);
acm_status acm_fft_c2r(const acm_grid* grid, int32_t precision, int32_t nfields, const void* in,
                       void* out, void* stream);

/*
 * Fourier-neural-operator warm start for the Stokes ADMM (g = e_x).  The
 * network (Li et al., ICLR 2021) maps H to (u_x, u_y, u_z, p):
 *   v0 = Pw H + Pb;  v_{l+1} = act(W_l v_l + b_l + K_l v_l), act = GELU except
 *   after the last layer; K_l = inverse real FFT of R_l (complex C x C per kept
 *   mode: kx < m, ky, kz in [0,m) U [n-m,n)) applied to the forward real FFT;
 *   out = Q2 GELU(Q1 v_L + c1) + c2.
 * Parameters: one flat array (layout Pw[C] Pb[C] | per layer R[nm][C][C]
 * complex as (re,im), W[C][C], b[C] | Q1[Cp][C] c1[Cp] Q2[4][Cp] c2[4],
 * nm = (2m)^2 m); kernels read the BF16 copy, Adam updates the FP32 master
 * and refreshes the BF16 copy.  Activations and accumulations are FP32.
 * params_bf16 must be 4-byte aligned (the mode weights are read as (re, im)
 * pairs); otherwise the call returns ACM_E_INVALID.
 * Grids must be cubic 3D with n in the supported set, channels in
 * {4, 8, 16, 32}, hidden * channels <= 4096, 2 * modes <= n.
 * H: uint8 [batch][n^3]; out, dout: float [batch][4][n^3] (device).
 * The workspace (device, caller-owned) keeps the activations of a training
 * forward pass for the following backward pass with the same arguments.
 */
typedef struct {
  int32_t channels; /* C */
  int32_t hidden;   /* Cp, projection width */
  int32_t modes;    /* m, kept modes per axis */
  int32_t layers;   /* L, Fourier layers */
} acm_fno_shape;

int64_t acm_fno_param_count(const acm_fno_shape* shape);  /* floats; -1 if invalid */
int64_t acm_fno_workspace_bytes(const acm_fno_shape* shape, const acm_grid* grid, int32_t batch,
                                int32_t train);            /* -1 if invalid */
acm_status acm_fno_forward(const acm_fno_shape* shape, const acm_grid* grid, int32_t batch,
                           const uint16_t* params_bf16, const uint8_t* H, float* out,
                           void* workspace, int64_t workspace_bytes, int32_t train, void* stream);
/* grad (device, param_count floats) receives d(sum dout * out)/d(params);
 * complex weights get (d/dRe, d/dIm). */
acm_status acm_fno_backward(const acm_fno_shape* shape, const acm_grid* grid, int32_t batch,
                            const uint16_t* params_bf16, const uint8_t* H, const float* dout,
                            float* grad, void* workspace, int64_t workspace_bytes, void* stream);
/* One Adam step (Kingma & Ba) on n parameters; step counts from 1. */
acm_status acm_fno_adam(int64_t n, float* params, uint16_t* params_bf16, const float* grad,
                        float* m, float* v, int64_t step, double lr, double beta1, double beta2,
                        double eps, void* stream);
acm_status acm_fno_to_bf16(int64_t n, const float* params, uint16_t* params_bf16, void* stream);
/* loss = mean (out - target)^2 (FP64 sum, host); dout = 2 (out - target) / n. */
acm_status acm_fno_mse(int64_t n, const float* out, const float* target, float* dout,
                       double* loss, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ACM_H_ */
