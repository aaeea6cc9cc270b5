/*
 * lbm.h -- C ABI of the MI355X (gfx950) semiclassical lattice Boltzmann library.
 *
 * Method: Coelho & Doria, "Lattice Boltzmann method for semiclassical fluids". The
 * library advances the isothermal electron model of Sec. 9.1: BGK relaxation toward
 * the second-order Fermi-Dirac equilibrium of eq. (feq-reduced-applied-electrons-in-
 * metals-eq), expanded in the generalised polynomials of Sec. 3 and discretised on the
 * D2V9 (Sec. 8) or D3V19 (Table 1) quadrature; the Lorentz forcing term of Sec. 7 with
 * the velocity-dependent acceleration a = E + xi x B; streaming on the lattice vectors
 * e_a; halfway bounce-back on solid nodes.
 *
 * Conventions used by every call:
 *   - Nodes are numbered n = x + nx*(y + ny*z); 2D grids have nz = 1.
 *   - Velocities are in xi-units, the paper's units where the Fermi speed is 1
 *     (xi_a = e_a / c_s). rho u = sum_a f_a xi_a, rho = sum_a f_a.
 *   - E and B are given in xi-units per time step (Delta t = 1): the field adds
 *     rho E to rho u per step and B rotates u by |B| radians per step. In 2D only
 *     E_x, E_y and B_z may be non-zero.
 *   - Every device pointer is borrowed: the library owns no device memory. The caller
 *     allocates state and work buffers of the sizes lbm_workspace_bytes reports and keeps
 *     them (and the mask and s arrays) alive while the handle exists.
 *   - All device work is enqueued on the HIP stream given to lbm_create; only
 *     lbm_current synchronises. A handle is not thread-safe.
 *   - Status codes: LBM_OK (0) or a negative LBM_E* value; no C++ exception crosses
 *     the ABI. lbm_last_error gives a message for the last failing call on a handle.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_s *lbm_t;

/* Lattices (Sec. 8, Table 1, App. A). D3V15 is listed only so that it can be rejected:
 * under the electron weight its rest weight is negative, which Sec. 8 forbids.
 * LBM_D1V7 (App. A, e = 0, +-1, +-2, +-3, quadrature of order 9) carries the
 * fourth-order thermal model: the equilibrium expanded to K = 4 (Sec. 3-6; K = 3 with
 * lbm_params.order = 3), periodic in x (ny = nz = 1), FP32 or 16-bit storage, no fields, solids or
 * porosity, two state buffers or one (the in-place step, as for the other lattices);
 * see lbm_init_thermal. */
enum { LBM_D2V9 = 0, LBM_D3V19 = 1, LBM_D3V15 = 2, LBM_D1V7 = 3 };

/* Weight functions: the Fermi-Dirac electron weight 1/(exp((xi^2 - mu)/theta) + 1) of
 * eq. (weight-func-isotherm-eq), Sec. 9.1; the Bose-Einstein weight
 * 1/(exp((xi^2 - mu)/theta) - 1), the other semiclassical form of eq. (be-fd-dist-eq),
 * Sec. 2 (needs mu < 0, fugacity z = e^(mu/theta) < 1; the paper gives no parameters);
 * or the Hermite weight of eq. (hermite-weight-eq), Sec. 2 (theta and mu ignored),
 * which yields textbook D2Q9/D3Q19. */
enum { LBM_FERMI_DIRAC = 0, LBM_BOSE_EINSTEIN = 1, LBM_HERMITE = 2 };

/* Population storage. All arithmetic is FP32; storage holds deviations
 * d_a = f_a - what_a rho0 from the rest equilibrium (what_a = w_a / I_0):
 *   LBM_F32  : float d_a
 *   LBM_F16  : IEEE half of d_a * 2^dev_scale_log2
 *   LBM_BF16 : bfloat16 of d_a
 * 16-bit values are rounded to nearest even, or stochastically (lbm_params.rounding). */
enum { LBM_F32 = 0, LBM_F16 = 1, LBM_BF16 = 2 };

/* Rounding of the 16-bit stored values written by the time steps (not in the paper):
 *   LBM_ROUND_NEAREST    : round to nearest even (the default);
 *   LBM_ROUND_STOCHASTIC : stochastic rounding (gfx950 v_cvt_sr_*): up or down with
 *                          probabilities given by the distance to the two neighbours, so
 *                          that a change smaller than half a unit in the last place is kept
 *                          on average instead of lost at every step. The random bits are a
 *                          hash of (node, population, step index): runs repeat bit for bit,
 *                          and the in-place and two-buffer steps agree bit for bit.
 * Initial states (lbm_init) are always rounded to nearest. LBM_F16 and LBM_BF16 only. */
enum { LBM_ROUND_NEAREST = 0, LBM_ROUND_STOCHASTIC = 1 };

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,        /* bad argument (sizes, tau <= 1/2, null pointer, ...) */
    LBM_EUNSUPPORTED = -2,  /* valid but not supported (e.g. a non-positive weight) */
    LBM_EDEVICE = -3,       /* a HIP call failed */
    LBM_ENONFINITE = -4,    /* a reduction found NaN or Inf */
    LBM_ESTATE = -5         /* call out of order (e.g. step before init) */
};

/* Forcing scheme of E and B (Sec. 7):
 *   LBM_FORCE_SOURCE : the xi-dependent source S_a = (E + xi_a x B) . grad_u f^eq_a added
 *                      to the BGK update (Sec. 7, forcing-term-integrals-eq);
 *   LBM_FORCE_SHIFT  : velocity shift, f^eq evaluated at u + tau (E + u x B) and no source
 *                      (eq. u-update-force-term-eq; the scheme of the runs of Sec. 9). */
enum { LBM_FORCE_SOURCE = 0, LBM_FORCE_SHIFT = 1 };

/* Free-slip walls (Sec. 9.4): LBM_SLIP_Y makes the planes y = 0 and y = ny-1 solid walls
 * that reflect specularly (a population keeps its motion along the wall and reverses
 * the normal component, arriving beside the node that emitted it); LBM_SLIP_Z the
 * same for z = 0 and z = nz-1. Obstacles of the mask keep halfway bounce-back, also
 * when a reflection would land on one. */
enum { LBM_SLIP_Y = 1, LBM_SLIP_Z = 2 };

typedef struct {
    int lattice;        /* LBM_D2V9, LBM_D3V19, or LBM_D1V7 (thermal model) */
    int stats;          /* LBM_FERMI_DIRAC or LBM_HERMITE */
    int storage;        /* LBM_F32, LBM_F16 or LBM_BF16 */
    int nx, ny, nz;     /* grid; nz = 1 for D2V9, ny = nz = 1 for D1V7; each >= 1, nx*ny*nz*Q < 2^31 */
    double theta, mu;   /* weight parameters (electron model: 1/270 and 1) */
    double tau;         /* BGK relaxation time in steps, > 1/2 */
    double E[3];        /* electric acceleration, xi-units per step */
    double B[3];        /* magnetic field: rotation angle of u per step */
    double rho0;        /* reference density of the stored deviations (> 0) */
    int dev_scale_log2; /* LBM_F16 only: stored value is d * 2^dev_scale_log2 (0..40) */
    int forcing;        /* LBM_FORCE_SOURCE or LBM_FORCE_SHIFT */
    int slip;           /* free-slip wall planes: 0, or LBM_SLIP_Y | LBM_SLIP_Z (3D only) */
    int order;          /* D1V7 only: truncation order K of the equilibrium expansion, 3 (the
                         * momentum equation, Sec. 6) or 4 (also the energy equation); 0 = 4.
                         * Must be 0 for D2V9/D3V19 (second order, Sec. 9.1). */
    int rounding;       /* LBM_ROUND_NEAREST or LBM_ROUND_STOCHASTIC (16-bit D2V9/D3V19 only) */
} lbm_params;

/* Constants the library derives from the parameters (host FP64), exposed for
 * checking. Shell index k = |e|^2 (0 rest, 1 axis, 2 face diagonal); unused
 * shells are 0. */
typedef struct {
    double I0, I2, I4;            /* weight integrals, eq. (i2n-cont2), Sec. 3 */
    double c0, c1, c2, c2bar, c2p;/* polynomial coefficients, Sec. 3 (K <= 2) */
    double J2, Delta2;            /* J_2 = I_2^2/(I_4 I_0), Delta_2, Sec. 3 */
    double theta_bar;             /* I_2 / I_0, Sec. 9.1 */
    double cs;                    /* reference speed sqrt(I_2/(3 I_4)), Sec. 8 */
    double w[4];                  /* quadrature weights by shell, Sec. 8 / Table 1 */
    double what[4];               /* w / I_0 (sum over the lattice = 1) */
    double A, Bc;                 /* equilibrium f_a = rho what_a [1 + A (xi.u) */
    double C[4];                  /*   + Bc (xi.u)^2 + C_k u^2], the reduced EDF of Sec. 9.1 */
} lbm_constants;

/* Host only, no device work. Computes the constants of Sec. 3, 8 and 9.1 for the
 * lattice, weight, theta and mu of *p (other fields ignored). Returns LBM_EINVAL for
 * an unknown lattice/weight or non-finite parameters and LBM_EUNSUPPORTED when a
 * weight comes out <= 0 (D3V15 under the electron weight). */
int lbm_compute_constants(const lbm_params *p, lbm_constants *out);

/* Host only. Q, D and the library's lattice vectors e (Q x 3 ints, row a = e_a) of the
 * quadratures of Sec. 8, Table 1 and App. A, in the order used by every Q-indexed buffer
 * of this library. e may be NULL. LBM_EINVAL for an unknown lattice and for D3V15. */
int lbm_lattice_info(int lattice, int *Q, int *D, int *e);

/* Host only; not in the paper (buffer sizing of this library). Sizes of the device
 * buffers a handle with parameters *p needs, so that the caller can allocate them (the
 * library owns no device memory):
 *   state_bytes : one population state (Q arrays of `stride` elements, storage type)
 *   work_bytes  : scratch for reductions, link masks and held adjoint partials
 *                 (8-byte aligned; any initial content)
 * Same validation and errors as lbm_create (LBM_EINVAL, e.g. Q * N >= 2^31). Either
 * output pointer may be NULL. */
int lbm_workspace_bytes(const lbm_params *p, size_t *state_bytes, size_t *work_bytes);

/* Host only; not in the paper. lbm_workspace_bytes plus the sizes the adjoint and the
 * caller's own indexing need:
 *   adjoint_bytes : one adjoint field (Q x stride floats)
 *   stride      : elements between population arrays (>= nx*ny*nz)
 * Any output pointer may be NULL. */
int lbm_buffer_sizes(const lbm_params *p, size_t *state_bytes, size_t *work_bytes,
                     size_t *adjoint_bytes, size_t *stride);

/* Validate *p, compute the constants and bind the buffers: the problem statement of the
 * electron model of Sec. 9.1 (lattice and weight, relaxation time tau, fields E and B,
 * solids), with the constants of Sec. 3 and the quadrature weights of Sec. 8 / Table 1.
 *   mask    : device uint8[N], 1 = solid, or NULL (no solids)
 *   s       : device float[N] in [0, 1], partial bounce-back fraction (Walsh et al.
 *             2009 gray lattice, not in the paper), or NULL
 *   state_a, state_b : two device state buffers of state_bytes each (ping-pong); with
 *             state_b = NULL the handle keeps one buffer and every step updates it in
 *             place (the AA access pattern of Bailey et al. 2009, not in the paper): a
 *             step that starts from the two-buffer layout writes each node's
 *             post-collision values where it pulled the opposite populations from (the
 *             populations end up streamed), and the next step reads them at the node
 *             and writes the two-buffer layout again. Same results, bit for bit, as two
 *             buffers, with half the state memory; lbm_get_state always returns the
 *             two-buffer layout.
 *   work    : device buffer of work_bytes
 *   stream  : hipStream_t (NULL = default stream)
 * Errors: LBM_EINVAL (tau <= 1/2, bad sizes, B_x/B_y or E_z in 2D, nz != 1 for D2V9,
 * null state_a or work, state_a == state_b, F16 scale out of range, unknown forcing,
 * slip bits other than Y/Z, Z slip in 2D, a slip axis with fewer than 3 planes),
 * LBM_EUNSUPPORTED (non-positive weight), LBM_EDEVICE. On error *out is NULL. */
int lbm_create(const lbm_params *p, const uint8_t *mask, const float *s, void *state_a,
               void *state_b, void *work, void *stream, lbm_t *out);

/* Initial state f_a(x) = f^eq_a(rho(x), u(x)) (reduced EDF,
 * eq. (feq-reduced-applied-electrons-in-metals-eq), Sec. 9.1), no force correction, as
 * the runs of Sec. 9.2-9.4 start from an equilibrium. rho: device double[N]; u: device
 * double[D*N] SoA (u_x block, then u_y, ...), xi-units, or NULL for u = 0. The fields are
 * FP64 (not float) so that a density given to more digits than FP32 holds, e.g.
 * rho(mu) from lbm_density_from_mu, is rounded once, inside the kernel, to the deviation
 * it stores. Values at solid nodes are ignored. Async. */
int lbm_init(lbm_t h, const double *rho, const double *u);

/* Initial state of the fourth-order thermal model (LBM_D1V7 only, LBM_EUNSUPPORTED
 * otherwise): f_a(x) = f^eq_a(rho(x), u(x), thetabar(x)), the equilibrium expanded to
 * K = 4 in the polynomials orthonormal under the weight (eq. feq-complete-exp-eq,
 * Sec. 3-5), i.e. w_a p(xi_a) with the polynomial p of degree 4 whose moments on the
 * lattice are those of the local distribution, M_0..M_4 = rho, rho u, rho (thetabar + u^2),
 * rho (u^3 + 3 u thetabar), rho (u^4 + 6 u^2 thetabar + 3 thetabar^2 g) (eqs. rho-def-eq,
 * vel-def-eq, theta-bar-def-eq, gz-def-eq). g is held at the weight's own value
 * I_4 I_0 / I_2^2, as Sec. 9.1 holds thetabar for the isothermal model (a g that follows
 * the local state makes the model unstable in the degenerate regime). rho: device
 * double[N]; u, thetabar: device double[N] or NULL (0, and the weight's I_2/I_0). The
 * lattice moves e = 0, +-1, +-2, +-3 per step; xi = e / c_s with the c_s of App. A.
 * lbm_step then relaxes to this equilibrium (BGK) and streams, periodic in x; the
 * energy equation of Sec. 6 follows, with the heat flux of eq. (pseudo-heat-flux-eq).
 * Async. */
int lbm_init_thermal(lbm_t h, const double *rho, const double *u, const double *thetabar);

/* Advance nsteps >= 0 time steps (collide, force, partial bounce-back, stream,
 * halfway bounce-back and free-slip walls: the discrete BGK update of Sec. 9.1 with
 * the forcing of Sec. 7). With one state buffer (state_b = NULL) the steps alternate
 * between the two in-place kernels. Async. */
int lbm_step(lbm_t h, int nsteps);

/* One step of the discrete BGK update of Sec. 9.1 (as lbm_step) from the state in `src`
 * into `dst` (device state buffers of state_bytes,
 * distinct, neither need be the handle's own; two-buffer layout, as lbm_get_state
 * writes it); the handle's state is not touched, its step index advances by one (it
 * selects the random bits of stochastic rounding). Used to recompute trajectories for
 * the adjoint. Async. */
int lbm_step_from(lbm_t h, const void *src, void *dst);

/* Not in the paper. The index of the handle's next time step (steps since lbm_init, which
 * sets it to 0, as lbm_set_state does); lbm_step and lbm_step_from advance it by one per
 * step. With LBM_ROUND_STOCHASTIC the random bits of step t are a function of t, so a
 * caller that recomputes steps (checkpointed adjoints, restarts) sets the index of the
 * first one here to repeat the run bit for bit; it has no effect otherwise. Host only. */
int lbm_set_step_index(lbm_t h, unsigned long long t);

/* Macroscopic fields of eq. (mac-fields-model-sec-eq), Sec. 9.1, of the current state
 * (pre-collision): rho = sum_a f_a (device float[N]) and u = sum_a f_a xi_a / rho (device
 * float[D*N] SoA, xi-units). Solid nodes get 0. Either pointer may be NULL. Async. */
int lbm_moments(lbm_t h, float *rho, float *u);

/* Thermal model (LBM_D1V7) only: thetabar of the current state, device float[N], defined
 * by rho (thetabar + u^2) = sum_a f_a xi_a^2 (eq. theta-bar-def-eq). Async. */
int lbm_thetabar(lbm_t h, float *thetabar);

/* Thermal model (LBM_D1V7) only: sum over nodes of sum_a f_a xi_a^2 (twice the kinetic
 * energy, the second moment the energy equation of Sec. 6 conserves, eq. energy-cons-eq),
 * FP64 into host *out. Synchronises the stream. */
int lbm_energy(lbm_t h, double *out);

/* Totals over fluid nodes of the current state, accumulated in FP64: the mass and the
 * current of Sec. 9.4 (Ohm's law: the current through the sample is rho times the mean
 * velocity over its cross-section), out[0] = sum rho, out[1..3] = sum rho u (xi-units;
 * out[3] = 0 in 2D), with rho and u of eq. (mac-fields-model-sec-eq). out is host
 * memory. Synchronises the stream. LBM_ENONFINITE if any total is NaN/Inf. */
int lbm_current(lbm_t h, double out[4]);

/* For callers that cannot allocate device memory or synchronise (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the totals of
 * lbm_current, computed the same way (same kernels, same FP64 reduction order, the same
 * bits), written asynchronously into device memory out[4] = (sum rho, sum rho u) on the
 * handle's stream. The reduction partials live in a fixed device-resident scratch array of
 * the library (64 KiB per GPU, held until the process ends; the totals use 57 KiB whatever
 * the grid size, LBM_EINVAL if that ever exceeded the array) instead of the workspace; no
 * hipMalloc, hipFree, memset or host synchronisation. Every call on one GPU shares that
 * GPU's array, and each call overwrites every part of it that it reads, so calls that
 * overlap on one GPU (concurrent streams or threads) race and must be serialised by the
 * caller. No NaN/Inf check (that needs the host): non-finite totals arrive as such.
 * D2V9 and D3V19 only (LBM_EUNSUPPORTED for D1V7). out: device double[4]. */
int lbm_current_noalloc(lbm_t h, double *out);

/* Convergence measure of the Ohm's-law runs (Sec. 9.4, stopped when it falls below 1e-7):
 * the average, over the nodes whose speed |u_new| is non-zero (fluid nodes; solids have
 * u = 0), of | |u_new| - |u_old| | / |u_new|. u (device float[D*N], the layout lbm_moments
 * writes) holds the new velocity field; speed (device float[N], caller-owned) holds |u_old|
 * on entry when have_previous != 0 and |u_new| on return (any content when have_previous
 * is 0, and then *out = 0). Per-node terms in FP64, summed in FP64; *out is host memory.
 * Synchronises the stream; LBM_ENONFINITE if the average is NaN/Inf. */
int lbm_speed_change(lbm_t h, const float *u, float *speed, int have_previous, double *out);

/* Not in the paper (state I/O for checkpointing and restarts). Copy the current state
 * to / from a caller device buffer of state_bytes (the library's opaque two-buffer
 * layout: post-collision populations of the previous step).
 * With one state buffer after an odd number of steps, lbm_get_state rearranges the
 * in-place layout into dst with a kernel (dst must not be state_a, LBM_EINVAL);
 * lbm_set_state restarts the in-place sequence from the two-buffer layout and sets the
 * step index to 0 (lbm_set_step_index). Async. */
int lbm_get_state(lbm_t h, void *dst);
int lbm_set_state(lbm_t h, const void *src);

/* Not in the paper (state I/O, for checking). Pre-collision populations f_a (full
 * values, not deviations) of a state in FP64:
 * dst is device double[Q*N], f_a of node n at dst[a*N + n] in lbm_lattice_info order.
 * state = NULL means the current state. Solid nodes get 0. Async. */
int lbm_export_f64(lbm_t h, const void *state, double *dst);

/* Change the fields of the Lorentz acceleration a = E + xi x B of Sec. 7 on an existing
 * handle (same validation as lbm_create), e.g. for the field sweep of Sec. 9.4. */
int lbm_set_fields(lbm_t h, const double E[3], const double B[3]);

/* Change the relaxation time tau of the discrete BGK update of Sec. 9.1 on an existing
 * handle (tau > 1/2, LBM_EINVAL otherwise), e.g. for the tau sweep of Sec. 9.3. */
int lbm_set_tau(lbm_t h, double tau);

/* Not in the paper (the adjoint is a growth of the method). Adjoint seed for the mean
 * current of Sec. 9.4 as the objective, J = (1/norm) sum over fluid nodes x and a of
 * f_a(x, T) xi_a[axis]:
 * lam[a*stride + n] = xi_a[axis]/norm at fluid nodes, 0 at solids (obstacles and free-slip
 * wall planes). LBM_EUNSUPPORTED for the D1V7 thermal model. lam: device float
 * buffer of adjoint_bytes. Starts a reverse pass: held dJ/dE, dJ/dtau contributions of
 * lbm_adjoint_step are discarded. Async. */
int lbm_adjoint_seed(lbm_t h, int axis, double norm, float *lam);

/* One reverse step of the discrete adjoint of lbm_step (not in the paper), for either
 * forcing (the source term of Sec. 7, or the velocity shift of eq. (u-update-force-term-eq)
 * used in Sec. 9.3), bounce-back
 * obstacles, partial bounce-back and the free-slip wall planes of Sec. 9.4:
 * LBM_EUNSUPPORTED for the D1V7 thermal model (as lbm_adjoint_seed).
 *   state   : the state buffer whose populations are pre-collision at step t (what the
 *             handle held before the forward step t -> t+1)
 *   lam_in  : dJ/df(t+1) (adjoint_bytes); lam_out: dJ/df(t) (distinct buffer)
 *   grad_s  : device float[N]; += dJ/ds through this step; may be NULL
 *   grad_scalars : device double[4]; += (dJ/dE_x, dJ/dE_y, dJ/dE_z, dJ/dtau) of this step
 *             and of every earlier step since the last call that passed one. NULL keeps
 *             this step's contribution as FP64 per-wave partials in the workspace (no
 *             reduction kernels), to be added by a later call; lbm_adjoint_seed discards
 *             contributions still held (a new reverse pass).
 * Async. */
int lbm_adjoint_step(lbm_t h, const void *state, const float *lam_in, float *lam_out,
                     float *grad_s, double *grad_scalars);

/* Density from chemical potential, Sec. 9.1-9.2: rho = (pi theta)^(D/2) g_(D/2)(e^(mu/theta))
 * with g_nu(z) = -Li_nu(-z) (LBM_FERMI_DIRAC) or Li_nu(z) (LBM_BOSE_EINSTEIN); D from
 * p->lattice, the weight from p->stats, theta from p->theta (other fields ignored). In 2D
 * g_1 is elementary; in 3D g_3/2 is integrated in FP64 per element (~1e-14 relative).
 * mu, rho: device double[n]. Async on `stream` (hipStream_t, NULL = default). The
 * Bose-Einstein weight needs mu < 0 (NaN otherwise). Errors: LBM_EINVAL (Hermite
 * weight, theta <= 0, null pointers), LBM_EDEVICE. Not part of the time step: the paper
 * uses it to set initial conditions and to report fields. */
int lbm_density_from_mu(const lbm_params *p, const double *mu, double *rho, size_t n, void *stream);

/* The inverse of the density relation of Sec. 9.1-9.2: mu from rho > 0 (closed form in
 * 2D, Newton's method on g_3/2 in 3D, where the paper inverts it numerically).
 * NaN where no mu exists: rho <= 0, and Bose-Einstein 3D densities at or above
 * (pi theta)^(3/2) zeta(3/2) (condensation). Same arguments and errors as above. */
int lbm_mu_from_density(const lbm_params *p, const double *rho, double *mu, size_t n, void *stream);

/* Not in the paper (handle lifetime and error reporting of this library). lbm_destroy
 * frees the host-side handle (NULL is a no-op) and no device memory, which the caller
 * owns; lbm_last_error gives the message of the last failing call on h (h = NULL: of the
 * last failing call that had no handle, on this thread); lbm_status_string names a
 * status code. The strings are owned by the library. */
void lbm_destroy(lbm_t h);
const char *lbm_last_error(lbm_t h);
const char *lbm_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
