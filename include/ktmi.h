/*
 * ktmi.h -- C ABI of libktmi, an MI355X (gfx950) library for the hot path of
 * CLVisc (arXiv:1802.04449): one RK2 step of the Kurganov-Tadmor central scheme
 * for (3+1)D second-order viscous hydrodynamics in Milne coordinates
 * (tau, x, y, eta_s).
 *
 * What one step computes (Sec. II eqns. Ttilde, pitilde, Ipi; Sec. III eqns.
 * common_form, kt, flux_out and the RK2 predictor-corrector flow chart):
 *   - KT flux divergence of T~^{tau mu} = tau T^{tau mu} and u~^tau pi~^{mu nu}
 *     from a minmod piecewise-linear reconstruction of the primitive fields,
 *   - the geometric source S_T and the Israel-Stewart source S_pi,
 *   - predictor (T', pi' with u* = 2u^n - u^{n-1}), then corrector (pi^{n+1}
 *     first, then T^{n+1} with S_T evaluated on pi^{n+1}),
 *   - after each stage the per-cell root solve T_ideal = T - pi -> (e, u~)
 *     with a tabulated or ideal-gas EoS (Sec. III, EoS options),
 *   - the energy-density cutoff (Sec. V.A), diagnostics reductions (App. A.2).
 * Tilde variables as in Sec. II: u~ = (u^tau, u^x, u^y, tau u^eta),
 * pi~ components ordered (tt, tx, ty, te, xx, xy, xe, yy, ye, ee).
 * Units: e, P in GeV/fm^3; T in GeV; lengths and tau in fm.
 *
 * Conventions for every call:
 *   - Return value 0 on success; a negative KTMI_E* code on error, with a
 *     message available from ktmi_last_error(h).  No exception crosses the ABI.
 *   - Field arrays are device pointers to FP64 data of nx*ny*ne elements in C
 *     order (x slowest, eta fastest) unless a call says "host".
 *   - The library never allocates device memory: the caller supplies one
 *     workspace of ktmi_workspace_bytes() bytes (ktmi_bind) and owns it; the
 *     library owns its layout.  All work is enqueued on the bound HIP stream;
 *     calls marked "synchronizes" wait for that stream.
 *   - A handle is not thread safe; distinct handles are independent.
 */
#ifndef KTMI_H
#define KTMI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    KTMI_OK = 0,
    KTMI_EINVAL = -22, /* bad argument or descriptor */
    KTMI_ESTATE = -5,  /* call out of order (e.g. step before bind / initial state) */
    KTMI_EHIP = -71    /* a HIP runtime call failed; see ktmi_last_error */
};

enum { KTMI_FP64 = 0, KTMI_MIXED = 1 };                               /* precision */
/* Start of the per-cell root solve: the cell's e from the previous stage, E
 * itself (cold), or the learned guess (ktmi_set_mlp; used by the initial state's
 * and the predictor's solves, while the corrector's solve starts from the
 * predictor's e, which is closer).  The result does not depend on the start
 * beyond the solve tolerance (a polish step follows). */
enum { KTMI_GUESS_PREV = 0, KTMI_GUESS_COLD = 1, KTMI_GUESS_MLP = 2 };
enum { KTMI_MLP_FP32 = 0, KTMI_MLP_BF16 = 1 }; /* forward of the learned guess */

/* Field ids for ktmi_read. */
enum {
    KTMI_F_EPS = 0,   /* e */
    KTMI_F_UX = 1,    /* u~^x, u~^y, u~^eta: 1..3 */
    KTMI_F_PI = 4,    /* pi~ components: 4..13 in the order above */
    KTMI_F_T = 14,    /* T~^{tau mu}: 14..17 */
    KTMI_F_UPREV = 18, /* u~ at the previous time level: 18..20 */
    KTMI_F_BULK = 21,  /* bulk pressure Pi (zero without bulk viscosity) */
    KTMI_F_NB = 22     /* net-baryon density n (zero unless transported) */
};

typedef struct ktmi_desc {
    int nx, ny, ne;      /* cells per axis, each >= 1 */
    double dx, dy, de;   /* spacings in fm, fm, and units of eta_s */
    double tau0, h;      /* initial proper time and time step (fm) */
    double etas;         /* eta_v / s; must be > 0 when viscous */
    int viscous;         /* 1: evolve the 10 pi~ components; 0: ideal (pi~ = 0) */
    int cartesian;       /* 1: tau == 1 in every metric factor, no Milne sources */
    double eps_cut;      /* energy-density cutoff, 1e-7 GeV/fm^3 in the paper */
    double theta;        /* generalised minmod parameter in [1, 2] */
    double newton_tol;   /* relative tolerance of the root solve */
    int newton_maxit;    /* iteration cap of the root solve */
    double pi_reg;       /* cap on sqrt(|pi~:pi~|)/(e+P); <= 0 disables */
    int precision;       /* KTMI_FP64, or KTMI_MIXED: FP32 reconstruction, fluxes, local
                            speed and shear relaxation source, and pi~ stored in FP32;
                            FP64 root solve, geometric source, e, u~, T~ and
                            accumulators.  ktmi_read returns every field in FP64. */
    int guess;           /* KTMI_GUESS_* */
    int tile;            /* workgroup tile shape index (ktmi_tile_shape); -1 = automatic */
    double taupi_coef;   /* tau_pi = taupi_coef (eta/s) hbarc / T; 5 in Sec. II.  Must be > 0
                            when viscous.  The Sec. V.C viscous Gubser solution needs
                            4 lambda1_hat^2 / 9 (its condition eta^ lambda1^2 = 3 tau_pi^) */
    double lambda1_hat;  /* second-order term of eqn. pimn, -(lambda_1/tau_pi) pi^<mu_l pi^nu>l,
                            with lambda_1 = lambda1_hat / e (the dimensionless lambda1_hat = lambda_1 e
                            of Sec. V.C); 0 = the equations of Sec. II.  Must be finite */
    double zetas;        /* zeta / s of the bulk pressure Pi (eqn. Pitilde; 0 in every run of the
                            paper, which is the default: no bulk pressure).  Must be finite, >= 0 */
    double taubulk_coef; /* tau_Pi = taubulk_coef (zeta/s) hbarc / T (default 5); > 0 with bulk */
    int baryon;          /* 1: transport the net-baryon density n (eqn. Ntilde; passive, the EoS
                            tables here being those of zero baryon chemical potential); 0 default.
                            Bulk pressure and baryon density need viscous mode, FP64 and
                            lambda1_hat = 0, and do not use the learned guess.  Pi and n obey
                            d~_tau(u~^tau X) + d~_i(u~^i X) = S_X with
                            S_Pi = -(Pi + zeta theta)/tau_Pi - Pi theta/3 - Pi u~^tau/tau,
                            zeta = (zeta/s)(e+P) hbarc/T, S_n = -n u~^tau/tau; Pi adds to P in
                            T^{mu nu} and in the root solve; the regulator clips Pi to [-P, P] */
    double cfl_limit;    /* largest c h / Delta over faces and stages that raises no
                            KTMI_ERR_CFL (default 0.5); must be > 0 */
} ktmi_desc;

/* Error bits of ktmi_diagnostics.errors, set from the counters accumulated since
 * the initial state.  The root solve (Sec. III flow chart) takes a varying
 * number of iterations (App. A.3) and the energy-density cutoff turns dilute
 * cells into vacuum (Sec. V.A); these bits flag the cases that mean the run
 * left the method's assumptions:
 *   KTMI_ERR_NAN     a NaN reached a root solve (the cell became vacuum),
 *   KTMI_ERR_NEG_EPS a root solve saw K^tau < 0, a negative energy density (the
 *                    cell became vacuum),
 *   KTMI_ERR_NONCONV a root solve stopped at newton_maxit iterations,
 *   KTMI_ERR_CFL     a face's c h / Delta exceeded cfl_limit (the KT scheme's
 *                    stability needs c h / Delta well below 1). */
enum { KTMI_ERR_NAN = 1, KTMI_ERR_NEG_EPS = 2, KTMI_ERR_NONCONV = 4, KTMI_ERR_CFL = 8 };

typedef struct ktmi_diagnostics {
    double tau;          /* proper time after the last step */
    long step;           /* steps taken since the initial state */
    double eps_max;      /* max e after the last step (App. A.2 stop criterion) */
    double sum_Ttt;      /* sum of T~^{tau tau} dx dy deta after the last step */
    double geo_src;      /* accumulated sum of h/2 (S_T1 + S_T2)^tau dx dy deta */
    double max_cfl;      /* max over faces and stages of c h / Delta */
    double newton_mean;  /* mean iterations per root solve (incl. the polish step) */
    long newton_max;     /* max iterations of one root solve */
    long solves, fallbacks, nonconv, nans, vacuum, clamps; /* counters */
    long negative;       /* root solves that saw K^tau < 0 */
    int errors;          /* KTMI_ERR_* bits */
} ktmi_diagnostics;

typedef struct ktmi_handle ktmi_handle;

/* Fills d with the defaults: cutoff 1e-7, theta 1.8, tolerance 1e-12, 100
 * iterations, regulator 0.3, FP64, previous-stage guess, automatic tile,
 * taupi_coef 5, lambda1_hat 0, zetas 0, taubulk_coef 5, baryon 0, cfl_limit
 * 0.5.  Sizes are zero. */
void ktmi_desc_default(ktmi_desc *d);

/* Validates d and creates a handle (host memory only).  KTMI_EINVAL if a size
 * is < 1, the grid has more than 2^29 - 256 cells (the kernels address a
 * field by 32-bit byte offsets), a spacing, tau0 or h is not > 0, viscous with etas <= 0 or
 * taupi_coef <= 0, lambda1_hat is not finite, zetas is not finite and >= 0,
 * baryon is not 0 or 1, or bulk/baryon is asked for without viscous mode, FP64
 * and lambda1_hat = 0, or with taubulk_coef <= 0, or cfl_limit is not > 0. */
int ktmi_create(const ktmi_desc *d, ktmi_handle **out);

/* Bytes of device workspace the handle needs (0 if d is invalid). */
size_t ktmi_workspace_bytes(const ktmi_desc *d);

/* Binds caller-owned device memory (>= ktmi_workspace_bytes, 256-byte aligned)
 * and a hipStream_t (passed as void*; NULL = default stream).  May be called
 * again to move the handle to another stream; the workspace must not change
 * after an initial state is set. */
int ktmi_bind(ktmi_handle *h, void *dev_workspace, size_t bytes, void *hip_stream);

/* Ideal-gas EoS P = e/3 (EOSI), T = (e/c_sb)^(1/4).  Sec. III, EoS options. */
int ktmi_set_eos_conformal(ktmi_handle *h, double c_sb);

/* Uniform-e table: row i holds (e0 + i de, P[i], T[i], cs2[i]); host arrays of
 * n >= 2 rows, copied to the workspace.  Linear interpolation between rows; past
 * the last row P continues with the last slope, cs2 is held and
 * T = T_last ((e+P)/(e_last+P_last))^(1/4).  KTMI_EINVAL if n < 2 or de <= 0. */
int ktmi_set_eos_table(ktmi_handle *h, double e0, double de, int n, const double *P,
                       const double *T, const double *cs2);

/* Initial primitive state (device arrays): e, u~x, u~y, u~eta and optionally 10
 * pi~ blocks (pi10 may be NULL for pi~ = 0; ignored in ideal mode).  Applies the
 * cutoff, forms T~^{tau mu}, and estimates u~^{-1} by one ideal forward-Euler
 * step (Sec. III: ideal hydrodynamics estimates u*1 on the first step).
 * Resets the diagnostics.  With KTMI_MIXED the stored pi~ is the input rounded
 * to FP32 (T~ is formed from the FP64 input). */
int ktmi_set_initial_primitive(ktmi_handle *h, const double *e, const double *ux,
                               const double *uy, const double *ue, const double *pi10);

/* As ktmi_set_initial_primitive, plus the bulk pressure Pi and the net-baryon
 * density n (eqns. Pitilde, Ntilde): device arrays of nx*ny*ne doubles, NULL for
 * zero; Pi is ignored unless zetas > 0, n unless baryon.  T~ is formed with
 * P + Pi; Pi and n are zero below the cutoff. */
int ktmi_set_initial_primitive_ext(ktmi_handle *h, const double *e, const double *ux,
                                   const double *uy, const double *ue, const double *pi10,
                                   const double *Pi, const double *n);

/* Initial conserved state: 4 device blocks of T~^{tau mu} and optional pi~
 * (Pi = n = 0 with bulk/baryon);
 * the root solve (starting from E) yields (e, u~).  Then as above. */
int ktmi_set_initial_conserved(ktmi_handle *h, const double *T4, const double *pi10);

/* Enqueues n RK2 steps on the bound stream (asynchronous).  Device-side
 * failures (NaN, negative energy density, non-converged solves, CFL excess) are
 * counted in the diagnostics and flagged in its error bits, not returned here
 * (no host synchronisation). */
int ktmi_step(ktmi_handle *h, int n);

/* Copies one field (ids above) to device array dst (stream-ordered, async). */
int ktmi_read(ktmi_handle *h, int field, double *dst);

/* Diagnostics accumulated since the initial state.  Synchronizes. */
int ktmi_diag(ktmi_handle *h, ktmi_diagnostics *out);

/* Per-kernel timing with HIP events recorded on the bound stream around every
 * launch (on = 1) or off (0; the default).  Turning it on clears the totals. */
int ktmi_set_timing(ktmi_handle *h, int on);

/* Kernel names of the step, in the order used by ktmi_timing. */
int ktmi_kernel_count(void);
const char *ktmi_kernel_name(int k);

/* Total milliseconds and launch count of kernel k since timing was turned on.
 * Synchronizes. */
int ktmi_timing(ktmi_handle *h, int k, double *total_ms, long *launches);

/* Workgroup tile shapes of the stencil kernels: each workgroup of 256 threads
 * owns tx*ty*tz cells (x, y, eta).  Any shape gives the same results up to
 * rounding of the diagnostics sums; the speed differs with the grid. */
int ktmi_tile_count(void);
int ktmi_tile_shape(int t, int *tx, int *ty, int *tz);

/* Selects the tile shape used by later launches (-1 = automatic: fewest padded
 * thread slots).  The workspace is sized for every shape. */
int ktmi_set_tile(ktmi_handle *h, int t);
int ktmi_get_tile(const ktmi_handle *h);

/* Replays one captured step as a HIP graph on every later ktmi_step (on = 1).
 * Every step issues identical launches (time and buffer parity live in device
 * memory), so the graph of one step is valid for all steps.  Needs a
 * non-default stream; ignored while timing is on.  KTMI_EINVAL on the default
 * stream. */
int ktmi_set_graph(ktmi_handle *h, int on);

/* Quiet-tile skipping (off by default; not part of the paper's method).  A
 * tile whose cells were vacuum before and after the last step (e = 0 before,
 * after stage 1 and after the step, pi~ = 0 after stage 1 and after the step,
 * K^tau below the cutoff) is quiet; a step skips every tile whose neighbours
 * within 6 cells are all quiet, because each pass would rewrite exactly the
 * values its buffers hold (zero fluxes, zero sources, T~ unchanged).  Fields
 * and diagnostics equal those of the full computation bit for bit.  Needs an
 * EoS with P(0) = 0 (KTMI_ESTATE otherwise, also when a later table breaks
 * it).  Turning it on or off, or changing the tile shape, marks every tile
 * as not quiet, so the next step computes all of them.  A group uses the
 * setting its members had when it was created. */
int ktmi_set_quiet_skip(ktmi_handle *h, int on);

/* Number of quiet tiles after the last step, and of tiles.  Synchronizes. */
int ktmi_quiet_tiles(ktmi_handle *h, long *quiet, long *total);

/* Groups: step many events (possibly of different grids and modes) together.
 * Events are sorted into classes of equal (viscous, precision, tile); per class
 * and stage a single launch covers the tiles of all its events (at most 128 per
 * class), and one reduce launch serves them all.  The handles keep their own
 * workspaces and states; the group only needs a device table of
 * ktmi_group_workspace_bytes(nev) bytes (256-byte aligned, caller-owned).  All
 * handles must share one stream and have an initial state; rebuild the group
 * after changing a handle's tile, EoS, guess mode or network.  ktmi_read /
 * ktmi_diag on a member handle see the grouped steps. */
typedef struct ktmi_group ktmi_group;
size_t ktmi_group_workspace_bytes(int nev);
int ktmi_group_create(ktmi_handle *const *hs, int nev, void *dev_ws, size_t bytes,
                      ktmi_group **out);
int ktmi_group_step(ktmi_group *g, int n);
int ktmi_group_set_graph(ktmi_group *g, int on);
int ktmi_group_class_count(const ktmi_group *g);
const char *ktmi_group_last_error(const ktmi_group *g);
void ktmi_group_destroy(ktmi_group *g);

/* Learned root-solve guess (not part of the paper's method; the paper notes
 * only that the root solve needs a varying number of iterations, App. A.3).
 * Network 4 -> 32 -> 32 -> 1 with tanh hidden layers on the features
 * f = (ln E / 5, M/E, (M/E)^2, ln(max(lo/E, 1e-30)) / 10) of K = (E, K^i),
 * M = |K^i|, lo = max(0, E - M^2/E); guess = lo + sigmoid(z) (E - lo), inside
 * the root bracket [lo, E].  Parameters: ktmi_mlp_nparam() FP32 values,
 * W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3 (device arrays).
 * KTMI_MLP_FP32 evaluates per thread in FP32; KTMI_MLP_BF16 runs the 32 x 32
 * layer on the BF16 matrix cores (FP32 accumulation) for 64 cells at a time. */
int ktmi_mlp_nparam(void);

/* Copies the parameters (device) into h's workspace and selects the forward
 * mode; later steps with guess KTMI_GUESS_MLP use them.  Stream-ordered. */
int ktmi_set_mlp(ktmi_handle *h, const float *params, int mode);

/* Changes the guess mode of h (KTMI_GUESS_*; MLP needs ktmi_set_mlp first).
 * Groups that hold h must be rebuilt. */
int ktmi_set_guess(ktmi_handle *h, int guess);

/* Training samples from h's current state, one per cell (device arrays of
 * nx*ny*ne): E = K^tau, M = |K^i| with K = T~^{tau .}/tau - pi~^{tau .}, and
 * eps = the cell's e (the root of that K; 0 in vacuum).  Async. */
int ktmi_harvest(ktmi_handle *h, double *E, double *M, double *eps);

/* guess[i] for n samples (device arrays E, M); samples with E < emin or not
 * finite get guess = E.  mode KTMI_MLP_*.  Async on stream (hipStream_t). */
int ktmi_mlp_forward(const float *params, int n, const double *E, const double *M, double emin,
                     double *guess, int mode, void *stream);

/* Gradient of the mean over the samples with E >= emin (finite) of
 * ((guess - eps)/E)^2.  out (device, ktmi_mlp_nparam() + 2 floats): the
 * gradient, then the mean loss, then the sample count.  The backward pass is
 * FP32; mode selects the forward as above.  Deterministic (fixed reduction
 * order).  ws: caller-owned device scratch of ktmi_mlp_grad_workspace_bytes(n)
 * bytes.  KTMI_EINVAL on bad arguments or a short workspace.  Async. */
size_t ktmi_mlp_grad_workspace_bytes(int n);
int ktmi_mlp_grad(const float *params, int n, const double *E, const double *M, const double *eps,
                  double emin, int mode, float *out, void *ws, size_t bytes, void *stream);

/* ktmi_mlp_grad for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight training loops, harnesses that
 * forbid allocation).  Same arguments and result as ktmi_mlp_grad, bitwise, but
 * the per-workgroup partial sums go to a scratch array inside the library: one
 * 2.56 MB copy per GPU (512 records of ktmi_mlp_nparam() + 2 floats), held
 * until the process ends.  That covers every sample count the call accepts:
 * 1 <= n <= 2^31 - 129 (KTMI_EINVAL outside, as for a bad pointer or mode).
 * No allocation of any kind; the first call on a GPU looks up the array's
 * device address (KTMI_EHIP if that fails).  The array is shared by every call
 * on one GPU and keeps the last call's contents: calls that overlap on one GPU
 * (on different streams, or from several threads) race and must be ordered by
 * the caller.  Async on stream. */
int ktmi_mlp_grad_noalloc(const float *params, int n, const double *E, const double *M,
                          const double *eps, double emin, int mode, float *out, void *stream);

/* One Adam step (Kingma & Ba 2015; bias-corrected moments, t counts from 1) on
 * params with gradient grad and moment arrays m, v (device, updated).  Async. */
int ktmi_mlp_adam(float *params, const float *grad, float *m, float *v, int t, float lr, float b1,
                  float b2, float epsilon, void *stream);

/* ------------------------------------------------------------------------ */
/* End of the evolution and the freeze-out surface (Sec. IV; App. A.2).      */
/* ------------------------------------------------------------------------ */

/* Steps h in chunks of check_every steps until the maximum energy density after
 * a chunk falls below eps_stop (the freeze-out energy density: App. A.2 stops the
 * evolution there), or max_steps steps are taken; *taken receives the number of
 * steps taken (>= 1 when max_steps >= 1).  Reads one diagnostics record per chunk
 * (a stream synchronisation).  KTMI_EINVAL if max_steps < 0, check_every < 1 or
 * taken is NULL. */
int ktmi_step_until(ktmi_handle *h, double eps_stop, int max_steps, int check_every, int *taken);

/* A time slice of h's state for the surface finder: with_pi = 0 gives 4 fields
 * (e, u~x, u~y, u~eta), 1 gives 14 (then pi~ in the order of KTMI_F_PI, zero in
 * vacuum), each nx*ny*ne doubles in the cell order of ktmi_read, field after
 * field.  ktmi_snapshot_doubles returns the size; ktmi_snapshot writes it to the
 * caller's device buffer dst (async on h's stream). */
size_t ktmi_snapshot_doubles(const ktmi_handle *h, int with_pi);
int ktmi_snapshot(ktmi_handle *h, double *dst, int with_pi);

#define KTMI_SURF_REC 24 /* doubles per surface element */

/* Freeze-out surface of constant energy density eps_f between two slices of h's
 * grid (device buffers from ktmi_snapshot with the same with_pi): A at tau_A and
 * B at tau_B > tau_A.  Every hypercube of 2x2x2x2 grid points (an axis with one
 * cell spans its width) whose corners straddle eps_f gives one element: the zero
 * set of the piecewise-linear interpolant of e - eps_f on the Kuhn triangulation
 * of the hypercube, with the covector dSigma_mu = sqrt(-g) S_mu pointing out of
 * the region e > eps_f, S_mu = V_mu (f_lo - f_hi) from the hot volume fractions of
 * the hypercube's faces normal to mu (divergence theorem; sums over hypercubes
 * telescope exactly), sqrt(-g) = tau at the element's centre (1 in Cartesian
 * mode).  Record (KTMI_SURF_REC doubles): [0] hypercube index (i cy + j) cz + k
 * with cy, cz the hypercube counts along y and eta, [1..4] centre (tau, x, y,
 * eta_s; the mean of the sign changes along the 32 edges), [5..8] dSigma_mu in
 * the coordinates (tau, x, y, eta_s), [9..11] u~ and [12..21] pi~ at the centre
 * (multilinear in the corners; pi~ zero for 4-field slices), [22] e at the
 * centre, [23] zero.  Records are in increasing hypercube order and reproducible
 * bit for bit.  The first capacity records go to out (device); *count (device, 8
 * bytes) receives the number of elements, which may exceed capacity (then call
 * again with a larger buffer).  Uses scratch in h's workspace (calls on one
 * handle must not overlap).  Async on h's stream.  KTMI_EINVAL on bad arguments,
 * KTMI_ESTATE without a bound workspace. */
int ktmi_surface(ktmi_handle *h, const double *A, double tau_A, const double *B, double tau_B,
                 int with_pi, double eps_f, double *out, long capacity,
                 unsigned long long *count);

/* Smooth Cooper-Frye spectra (Sec. IV, eq. cooper_frye with f_eq and delta f of
 * eqn. feq; App. A.2) of n surface records (device, as written by ktmi_surface)
 * for ns species (host arrays: mass in GeV, degeneracy dof, stat = +1
 * Fermi-Dirac, -1 Bose-Einstein, 0 Boltzmann, chemical potential mu in GeV) on
 * the bins Y[nY] x pt[npt] (GeV) x phi[nphi] (host arrays):
 *   out[((s nY + iy) npt + ip) nphi + iphi] = dN/(dY pT dpT dphi) in GeV^-2
 *   = dof / (2 pi hbarc)^3 sum_elements p^mu dSigma_mu f (1 + df),
 * p~ = (m_T cosh(Y - eta_s), pT cos phi, pT sin phi, m_T sinh(Y - eta_s)) at the element's
 * centre, p^mu dSigma_mu = p~^tau dS_tau + p~^x dS_x + p~^y dS_y + (p~^eta/tau) dS_eta,
 * f = 1/(exp((p.u - mu)/T) + stat), df = (1 - stat f) p~_a p~_b pi~^{ab} / (2 T^2 e_plus_P)
 * (eps_plus_P = e + P at freeze-out in GeV/fm^3; 0 leaves delta f out).  out is
 * device memory; ws is caller-owned device scratch of ktmi_spectra_workspace_bytes
 * bytes.  The result does not depend on scheduling (fixed summation order).
 * Synchronises stream once (upload of the small tables), then runs async on it.
 * KTMI_EINVAL on bad arguments or a short workspace. */
size_t ktmi_spectra_workspace_bytes(long n, int ns, int nY, int npt, int nphi);
int ktmi_spectra(const double *elements, long n, double T, double eps_plus_P, int ns,
                 const double *mass, const double *dof, const int *stat, const double *mu, int nY,
                 const double *Y, int npt, const double *pt, int nphi, const double *phi,
                 double *out, void *ws, size_t ws_bytes, void *stream);

/* Message of the last error on h (or of the last failed ktmi_create if h is
 * NULL).  Valid until the next call on h. */
const char *ktmi_last_error(const ktmi_handle *h);

/* Releases host resources; the caller frees the workspace afterwards. */
void ktmi_destroy(ktmi_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* KTMI_H */
