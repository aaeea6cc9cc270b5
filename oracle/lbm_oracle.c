/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the semiclassical lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY. This file is the reference against which the GPU path is
 * checked. Only the tests, the package smoke check and the benchmark's CPU-baseline
 * leg load it; the product path never does, and this file shares no code, header,
 * table or constant with the GPU library.
 *
 * Method: Coelho & Doria, "Lattice Boltzmann method for semiclassical fluids".
 * Readings of the paper that this file takes (the paper is silent or garbled there):
 *   - moments are rho = sum_a f_a, rho u = sum_a f_a xi_a with xi_a = e_a / c_s
 *     (the printed moment formula of Sec. 9.1 carries an extra w_a that only fits
 *     populations stored divided by w_a);
 *   - the Lorentz source enters with a plus sign, S_a = +a_a . grad_u f^eq_a, so that
 *     sum_a S_a xi_a = +rho (E + u x B) (Sec. 7 has sign slips);
 *   - E and B are in xi-units per time step, Delta t = 1;
 *   - walls are halfway (link) bounce-back against solid nodes (mask = 1);
 *   - the optional partial bounce-back g_a = (1-s) f*_a + s f_abar is the
 *     Walsh-Burwinkle-Saar (2009) gray-lattice rule; it is not in the paper;
 *   - the velocity-shift forcing of Sec. 7 (the scheme of the experiments of Sec. 9)
 *     evaluates f^eq at u + tau a with the macroscopic acceleration a = E + u x B and
 *     adds no source term;
 *   - free-slip walls (Sec. 9.4) are the domain planes y = 0, ny-1 (and z = 0, nz-1)
 *     reflecting specularly: a population pushed into a wall plane keeps its motion
 *     along the wall and reverses its normal component, arriving beside its emitter;
 *     if that node is an obstacle it bounces back instead.
 *
 * Layout: full populations (not deviations), f[a*N + n], n = x + nx*(y + ny*z).
 * Rows (y, z) are split over OpenMP threads; that is the only optimisation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QMAX 27

typedef struct {
    int D, Q;
    int nx, ny, nz;
    double tau;
    double E[3], B[3];
    /* second-order polynomial coefficients, Sec. 3 */
    double c0, c1, c2, c2bar, c2p;
    /* reference speed c_s, Sec. 8 */
    double cs;
    double w[ORC_QMAX];     /* quadrature weights w_a (not divided by I_0) */
    int e[ORC_QMAX][3];     /* integer lattice vectors e_a */
    double xi[ORC_QMAX][3]; /* discrete velocities xi_a = e_a / c_s, Sec. 8 */
    int opp[ORC_QMAX];      /* index of -e_a */
    int forcing;            /* 0: xi-dependent source term; 1: velocity shift */
    int slip;               /* free-slip wall planes: bit 0 y, bit 1 z */
} orc_model;

int orc_model_size(void) { return (int)sizeof(orc_model); }

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Build the model. `ev` holds Q integer vectors (3 ints each, unused components 0) in
 * the oracle's own order; `w_by_norm2[k]` is the weight of every vector with |e|^2 = k
 * (Sec. 8 and Table 1 give one weight per fully symmetric shell); `coef` holds
 * c0, c1, c2, cbar2, c'2, c_s.
 * Returns 0, or -1 if a vector has no opposite in the set.
 */
int orc_init_model(orc_model *m, int D, int Q, const int *ev, int nx, int ny, int nz,
                   double tau, const double *E, const double *B, const double *coef,
                   const double *w_by_norm2)
{
    memset(m, 0, sizeof(*m));
    m->D = D;
    m->Q = Q;
    m->nx = nx;
    m->ny = ny;
    m->nz = nz;
    m->tau = tau;
    for (int i = 0; i < 3; ++i) {
        m->E[i] = E[i];
        m->B[i] = B[i];
    }
    m->c0 = coef[0];
    m->c1 = coef[1];
    m->c2 = coef[2];
    m->c2bar = coef[3];
    m->c2p = coef[4];
    m->cs = coef[5];
    for (int a = 0; a < Q; ++a) {
        int n2 = 0;
        for (int i = 0; i < 3; ++i) {
            m->e[a][i] = ev[3 * a + i];
            n2 += m->e[a][i] * m->e[a][i];
            m->xi[a][i] = (double)m->e[a][i] / m->cs;
        }
        m->w[a] = w_by_norm2[n2];
    }
    for (int a = 0; a < Q; ++a) {
        m->opp[a] = -1;
        for (int b = 0; b < Q; ++b)
            if (m->e[b][0] == -m->e[a][0] && m->e[b][1] == -m->e[a][1] &&
                m->e[b][2] == -m->e[a][2])
                m->opp[a] = b;
        if (m->opp[a] < 0) return -1;
    }
    return 0;
}

/* Forcing scheme (0 source, 1 velocity shift) and free-slip planes (bit 0 y, bit 1 z). */
int orc_set_scheme(orc_model *m, int forcing, int slip)
{
    if (forcing != 0 && forcing != 1) return -1;
    if (slip < 0 || slip > 3 || (m->D == 2 && (slip & 2))) return -1;
    m->forcing = forcing;
    m->slip = slip;
    return 0;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Macroscopic fields of one node (Sec. 9.1, moment definitions, read as above). */
void orc_node_moments(const orc_model *m, const double *f, double *rho, double *u)
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < m->Q; ++a) {
        r += f[a];
        for (int i = 0; i < 3; ++i) j[i] += f[a] * m->xi[a][i];
    }
    *rho = r;
    for (int i = 0; i < 3; ++i) u[i] = j[i] / r;
}

/*
 * Reduced second-order equilibrium used by the electron model, eq.
 * (feq-reduced-applied-electrons-in-metals-eq), Sec. 9.1:
 *   f^eq_a = rho w_a { c0^2 + c1^2 (xi.u) + c2^2/2 (xi.u)^2 + 1/2 c2 cbar2 u^2 xi^2
 *                      + 1/2 (cbar2 xi^2 + c'2)(c2 + D cbar2) u^2 }.
 */
void orc_equilibrium(const orc_model *m, double rho, const double *u, double *feq)
{
    const double D = (double)m->D;
    const double u2 = dot3(u, u);
    for (int a = 0; a < m->Q; ++a) {
        const double xu = dot3(m->xi[a], u);
        const double xi2 = dot3(m->xi[a], m->xi[a]);
        const double brace = m->c0 * m->c0 + m->c1 * m->c1 * xu + 0.5 * m->c2 * m->c2 * xu * xu +
                             0.5 * m->c2 * m->c2bar * u2 * xi2 +
                             0.5 * (m->c2bar * xi2 + m->c2p) * (m->c2 + D * m->c2bar) * u2;
        feq[a] = rho * m->w[a] * brace;
    }
}

/*
 * The vector G_a(u) = grad_u f^eq_a / (rho w_a) of Sec. 7:
 *   G_a = c1^2 xi + c2^2 (xi.u) xi + (2 c2 cbar2 + D cbar2^2) xi^2 u + (c2 c'2 + D cbar2 c'2) u.
 */
static void grad_u_feq_unit(const orc_model *m, int a, const double *u, double *G)
{
    const double D = (double)m->D;
    const double *xi = m->xi[a];
    const double xu = dot3(xi, u);
    const double xi2 = dot3(xi, xi);
    const double k1 = 2.0 * m->c2 * m->c2bar + D * m->c2bar * m->c2bar;
    const double k2 = m->c2 * m->c2p + D * m->c2bar * m->c2p;
    for (int i = 0; i < 3; ++i)
        G[i] = m->c1 * m->c1 * xi[i] + m->c2 * m->c2 * xu * xi[i] + k1 * xi2 * u[i] + k2 * u[i];
}

/* Lorentz acceleration of population a (Sec. 7): a_E = E plus a_B = xi_a x B. */
static void lorentz_accel(const orc_model *m, int a, double *acc)
{
    double xb[3];
    cross3(m->xi[a], m->B, xb);
    for (int i = 0; i < 3; ++i) acc[i] = m->E[i] + xb[i];
    if (m->D == 2) acc[2] = 0.0; /* the 2D model lives in the x-y plane */
}

/*
 * Forcing term of Sec. 7, S_a = a_a . grad_u f^eq_a = rho w_a G_a(u) . a_a, with the
 * xi-dependent Lorentz acceleration a_a = E + xi_a x B.
 */
void orc_source(const orc_model *m, double rho, const double *u, double *S)
{
    for (int a = 0; a < m->Q; ++a) {
        double G[3], acc[3];
        grad_u_feq_unit(m, a, u, G);
        lorentz_accel(m, a, acc);
        S[a] = rho * m->w[a] * dot3(G, acc);
    }
}

/*
 * Collision of one node: BGK relaxation with the source (discrete BGK of Sec. 9.1,
 * Delta t = 1), f*_a = f_a - (f_a - f^eq_a)/tau + S_a, then the optional partial
 * bounce-back g_a = (1 - s) f*_a + s f_abar.
 */
void orc_collide_node(const orc_model *m, const double *f, double s, double *g)
{
    double rho, u[3], feq[ORC_QMAX], S[ORC_QMAX], fs[ORC_QMAX];
    orc_node_moments(m, f, &rho, u);
    if (m->forcing == 1) {
        /* velocity shift, eq. (u-update-force-term-eq): f^eq at u + tau a, a = E + u x B */
        double ub[3], ueq[3];
        cross3(u, m->B, ub);
        for (int i = 0; i < 3; ++i) ueq[i] = u[i] + m->tau * (m->E[i] + ub[i]);
        if (m->D == 2) ueq[2] = 0.0;
        orc_equilibrium(m, rho, ueq, feq);
        for (int a = 0; a < m->Q; ++a) S[a] = 0.0;
    } else {
        orc_equilibrium(m, rho, u, feq);
        orc_source(m, rho, u, S);
    }
    for (int a = 0; a < m->Q; ++a) fs[a] = f[a] - (f[a] - feq[a]) / m->tau + S[a];
    for (int a = 0; a < m->Q; ++a) g[a] = (1.0 - s) * fs[a] + s * f[m->opp[a]];
}

static long node_index(const orc_model *m, int x, int y, int z)
{
    return (long)x + (long)m->nx * ((long)y + (long)m->ny * (long)z);
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Initial state f = f^eq(rho(x), u(x)) (no force correction). u is SoA [D][N]. */
void orc_init_state(const orc_model *m, const uint8_t *mask, const double *rho, const double *u,
                    double *f)
{
    const long N = (long)m->nx * m->ny * m->nz;
    for (long n = 0; n < N; ++n) {
        double uu[3] = {0.0, 0.0, 0.0}, feq[ORC_QMAX];
        if (mask && mask[n]) {
            for (int a = 0; a < m->Q; ++a) f[a * N + n] = 0.0;
            continue;
        }
        if (u)
            for (int i = 0; i < m->D; ++i) uu[i] = u[i * N + n];
        orc_equilibrium(m, rho[n], uu, feq);
        for (int a = 0; a < m->Q; ++a) f[a * N + n] = feq[a];
    }
}

/* index of the vector e with the components of the axes in `flip` (bit 1 y, bit 2 z) reversed */
static int reflected(const orc_model *m, int a, int flip)
{
    const int ex = m->e[a][0], ey = (flip & 1) ? -m->e[a][1] : m->e[a][1];
    const int ez = (flip & 2) ? -m->e[a][2] : m->e[a][2];
    for (int b = 0; b < m->Q; ++b)
        if (m->e[b][0] == ex && m->e[b][1] == ey && m->e[b][2] == ez) return b;
    return -1;
}

/*
 * One time step: collide every fluid node, then push each post-collision population
 * g_a(x) to x + e_a (periodic wrap). If x + e_a lies in a free-slip wall plane, the
 * population is reflected there: it arrives at x + e_a with the wall-axis coordinates
 * of x, in the direction with those components of e_a reversed. If its destination is
 * solid (an obstacle), it returns to x in the opposite direction (halfway bounce-back).
 * Solid nodes (mask = 1; the caller includes the wall planes) hold zero.
 * `s` (per node, may be NULL) is the partial bounce-back fraction.
 */
void orc_step(const orc_model *m, const uint8_t *mask, const double *s, const double *fin,
              double *fout)
{
    const long N = (long)m->nx * m->ny * m->nz;
    const int Q = m->Q;
    memset(fout, 0, sizeof(double) * (size_t)Q * (size_t)N);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < m->nz; ++z)
        for (int y = 0; y < m->ny; ++y)
            for (int x = 0; x < m->nx; ++x) {
                const long n = node_index(m, x, y, z);
                if (mask && mask[n]) continue;
                double f[ORC_QMAX], g[ORC_QMAX];
                for (int a = 0; a < Q; ++a) f[a] = fin[a * N + n];
                orc_collide_node(m, f, s ? s[n] : 0.0, g);
                for (int a = 0; a < Q; ++a) {
                    int tx = wrap(x + m->e[a][0], m->nx), ty = wrap(y + m->e[a][1], m->ny);
                    int tz = wrap(z + m->e[a][2], m->nz), b = a;
                    const int flip = (((m->slip & 1) && m->e[a][1] != 0 && (ty == 0 || ty == m->ny - 1)) ? 1 : 0) |
                                     (((m->slip & 2) && m->e[a][2] != 0 && (tz == 0 || tz == m->nz - 1)) ? 2 : 0);
                    if (flip) {
                        if (flip & 1) ty = y;
                        if (flip & 2) tz = z;
                        b = reflected(m, a, flip);
                    }
                    const long d = node_index(m, tx, ty, tz);
                    if (mask && mask[d])
                        fout[m->opp[a] * N + n] = g[a];
                    else
                        fout[b * N + d] = g[a];
                }
            }
}

/* nsteps steps in place on f (uses a scratch copy). Returns 0, -1 on allocation failure. */
int orc_run(const orc_model *m, const uint8_t *mask, const double *s, double *f, int nsteps)
{
    const size_t len = (size_t)m->Q * (size_t)m->nx * m->ny * m->nz;
    double *tmp = (double *)malloc(sizeof(double) * len);
    if (!tmp) return -1;
    for (int t = 0; t < nsteps; ++t) {
        orc_step(m, mask, s, f, tmp);
        memcpy(f, tmp, sizeof(double) * len);
    }
    free(tmp);
    return 0;
}

/* rho and u fields of a state (pre-collision); solid nodes report 0. u is SoA [D][N]. */
void orc_moments(const orc_model *m, const uint8_t *mask, const double *fin, double *rho,
                 double *u)
{
    const long N = (long)m->nx * m->ny * m->nz;
    for (long n = 0; n < N; ++n) {
        double f[ORC_QMAX], r = 0.0, uu[3] = {0.0, 0.0, 0.0};
        if (!(mask && mask[n])) {
            for (int a = 0; a < m->Q; ++a) f[a] = fin[a * N + n];
            orc_node_moments(m, f, &r, uu);
        }
        rho[n] = r;
        for (int i = 0; i < m->D; ++i) u[i * N + n] = uu[i];
    }
}

/* Totals over fluid nodes: out = {sum rho, sum rho u_x, sum rho u_y, sum rho u_z}. */
void orc_totals(const orc_model *m, const uint8_t *mask, const double *fin, double *out)
{
    const long N = (long)m->nx * m->ny * m->nz;
    for (int i = 0; i < 4; ++i) out[i] = 0.0;
    for (long n = 0; n < N; ++n) {
        if (mask && mask[n]) continue;
        for (int a = 0; a < m->Q; ++a) {
            const double fa = fin[a * N + n];
            out[0] += fa;
            for (int i = 0; i < 3; ++i) out[1 + i] += fa * m->xi[a][i];
        }
    }
}

/*
 * Discrete adjoint of one time step (not in the paper; it differentiates the map
 * F_t -> F_{t+1} that orc_step computes).
 *
 * Inputs: the forward pre-collision state F_t (`fin`), and lam_in = dJ/dF_{t+1}.
 * Output: lam_out = dJ/dF_t. Accumulates grad_s[n] += dJ/ds(n) through step t when
 * grad_s is given, and grad[0..2] += dJ/dE, grad[3] += dJ/dtau.
 *
 * Per fluid node y:
 *   gbar_a = adjoint of g_a(y): lam_in where orc_step writes g_a(y): at (y + e_a, a),
 *            at the reflected destination and direction beside a free-slip plane, or at
 *            (y, abar) when that destination is solid (transpose of the push);
 *   hbar_a = (1 - s) gbar_a                      (adjoint of f*_a);
 *   dJ/ds  = sum_a gbar_a (f_abar - f*_a);
 *   dJ/dtau = sum_a hbar_a (f_a - f^eq_a) / tau^2;
 *   dJ/dE_i = sum_a hbar_a rho w_a G_ai;
 *   with Phi_a = f^eq_a/tau + S_a (linear in rho at fixed u):
 *   rhobar = sum_a hbar_a Phi_a / rho,  ubar_i = sum_a hbar_a dPhi_a/du_i,
 *     dPhi_a/du_i = rho w_a [ G_ai / tau + c2^2 xi_ai (xi_a . a_a) + (k1 xi_a^2 + k2) a_ai ];
 *   lam_out_b = (1 - 1/tau) hbar_b + s gbar_abar(b) + rhobar + ubar . (xi_b - u) / rho.
 * Velocity shift (eq. u-update-force-term-eq): Phi_a = f^eq_a(rho, u') / tau with
 * u' = u + tau (E + u x B) and no source; with Gs = sum_a hbar_a rho w_a G_a(u')
 * (the adjoint of u'): rhobar = sum_a hbar_a f^eq_a / (tau rho), ubar = (Gs + tau B x Gs)
 * / tau, dJ/dE = Gs, dJ/dtau = sum_a hbar_a (f_a - f^eq_a) / tau^2 + Gs . (E + u x B) / tau.
 * Solid nodes get lam_out = 0.
 */
void orc_adjoint_step(const orc_model *m, const uint8_t *mask, const double *s,
                      const double *fin, const double *lam_in, double *lam_out,
                      double *grad_s, double *grad)
{
    const long N = (long)m->nx * m->ny * m->nz;
    const int Q = m->Q;
    const double D = (double)m->D;
    const double tau = m->tau;
    const double k1 = 2.0 * m->c2 * m->c2bar + D * m->c2bar * m->c2bar;
    const double k2 = m->c2 * m->c2p + D * m->c2bar * m->c2p;
    double gE0 = 0.0, gE1 = 0.0, gE2 = 0.0, gT = 0.0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : gE0, gE1, gE2, gT)
    for (int z = 0; z < m->nz; ++z)
        for (int y = 0; y < m->ny; ++y)
            for (int x = 0; x < m->nx; ++x) {
                const long n = node_index(m, x, y, z);
                if (mask && mask[n]) {
                    for (int a = 0; a < Q; ++a) lam_out[a * N + n] = 0.0;
                    continue;
                }
                double f[ORC_QMAX], gbar[ORC_QMAX], hbar[ORC_QMAX];
                double feq[ORC_QMAX], S[ORC_QMAX], fs[ORC_QMAX];
                double rho, u[3];
                const double sn = s ? s[n] : 0.0;
                for (int a = 0; a < Q; ++a) {
                    f[a] = fin[a * N + n];
                    /* where orc_step sends g_a(x): slot b of d (reflected at a free-slip
                     * plane), or slot opp(a) of x when d is solid */
                    int tx = wrap(x + m->e[a][0], m->nx), ty = wrap(y + m->e[a][1], m->ny);
                    int tz = wrap(z + m->e[a][2], m->nz), b = a;
                    const int flip = (((m->slip & 1) && m->e[a][1] != 0 && (ty == 0 || ty == m->ny - 1)) ? 1 : 0) |
                                     (((m->slip & 2) && m->e[a][2] != 0 && (tz == 0 || tz == m->nz - 1)) ? 2 : 0);
                    if (flip) {
                        if (flip & 1) ty = y;
                        if (flip & 2) tz = z;
                        b = reflected(m, a, flip);
                    }
                    const long d = node_index(m, tx, ty, tz);
                    gbar[a] = (mask && mask[d]) ? lam_in[m->opp[a] * N + n] : lam_in[b * N + d];
                    hbar[a] = (1.0 - sn) * gbar[a];
                }
                orc_node_moments(m, f, &rho, u);
                if (m->forcing == 1) {
                    /* velocity shift: Phi_a = f^eq_a(rho, u') / tau, u' = u + tau (E + u x B) */
                    double ub[3], up[3], sh[3], Gs[3] = {0.0, 0.0, 0.0};
                    cross3(u, m->B, ub);
                    for (int i = 0; i < 3; ++i) {
                        sh[i] = m->E[i] + ub[i];
                        up[i] = u[i] + tau * sh[i];
                    }
                    if (m->D == 2) up[2] = sh[2] = 0.0;
                    orc_equilibrium(m, rho, up, feq);
                    for (int a = 0; a < Q; ++a) fs[a] = f[a] - (f[a] - feq[a]) / tau;
                    double ds = 0.0, rhobar = 0.0;
                    for (int a = 0; a < Q; ++a) {
                        double G[3];
                        grad_u_feq_unit(m, a, up, G); /* d f^eq_a / d u' = rho w_a G */
                        ds += gbar[a] * (f[m->opp[a]] - fs[a]);
                        gT += hbar[a] * ((f[a] - feq[a]) / (tau * tau) + rho * m->w[a] * dot3(G, sh) / tau);
                        for (int i = 0; i < 3; ++i) Gs[i] += hbar[a] * rho * m->w[a] * G[i];
                        rhobar += hbar[a] * feq[a] / (tau * rho);
                    }
                    gE0 += Gs[0];
                    gE1 += Gs[1];
                    gE2 += Gs[2];
                    /* du'/du = 1 + tau [. x B]: ubar = (Gs + tau B x Gs) / tau */
                    double bg[3], ubar[3];
                    cross3(m->B, Gs, bg);
                    for (int i = 0; i < 3; ++i) ubar[i] = (Gs[i] + tau * bg[i]) / tau;
                    if (grad_s) grad_s[n] += ds;
                    for (int b = 0; b < Q; ++b) {
                        double uterm = 0.0;
                        for (int i = 0; i < m->D; ++i) uterm += ubar[i] * (m->xi[b][i] - u[i]) / rho;
                        lam_out[b * N + n] =
                            (1.0 - 1.0 / tau) * hbar[b] + sn * gbar[m->opp[b]] + rhobar + uterm;
                    }
                    continue;
                }
                orc_equilibrium(m, rho, u, feq);
                orc_source(m, rho, u, S);
                for (int a = 0; a < Q; ++a) fs[a] = f[a] - (f[a] - feq[a]) / tau + S[a];

                double ds = 0.0, rhobar = 0.0, ubar[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < Q; ++a) {
                    double G[3], acc[3];
                    grad_u_feq_unit(m, a, u, G);
                    lorentz_accel(m, a, acc);
                    const double *xi = m->xi[a];
                    const double xi2 = dot3(xi, xi);
                    const double xa = dot3(xi, acc);
                    ds += gbar[a] * (f[m->opp[a]] - fs[a]);
                    gT += hbar[a] * (f[a] - feq[a]) / (tau * tau);
                    gE0 += hbar[a] * rho * m->w[a] * G[0];
                    gE1 += hbar[a] * rho * m->w[a] * G[1];
                    gE2 += hbar[a] * rho * m->w[a] * G[2];
                    rhobar += hbar[a] * (feq[a] / tau + S[a]) / rho;
                    for (int i = 0; i < m->D; ++i)
                        ubar[i] += hbar[a] * rho * m->w[a] *
                                   (G[i] / tau + m->c2 * m->c2 * xi[i] * xa + (k1 * xi2 + k2) * acc[i]);
                }
                if (grad_s) grad_s[n] += ds;
                for (int b = 0; b < Q; ++b) {
                    double uterm = 0.0;
                    for (int i = 0; i < m->D; ++i) uterm += ubar[i] * (m->xi[b][i] - u[i]) / rho;
                    lam_out[b * N + n] =
                        (1.0 - 1.0 / tau) * hbar[b] + sn * gbar[m->opp[b]] + rhobar + uterm;
                }
            }
    grad[0] += gE0;
    grad[1] += gE1;
    grad[2] += gE2;
    grad[3] += gT;
}

/* Adjoint seed for J = (1/norm) sum_{fluid x} sum_a F_T(x, a) xi_a[axis]. */
void orc_seed_current(const orc_model *m, const uint8_t *mask, int axis, double norm,
                      double *lam)
{
    const long N = (long)m->nx * m->ny * m->nz;
    for (long n = 0; n < N; ++n)
        for (int a = 0; a < m->Q; ++a)
            lam[a * N + n] = (mask && mask[n]) ? 0.0 : m->xi[a][axis] / norm;
}
