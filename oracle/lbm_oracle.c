/*
 * FP64 CPU oracle of the thermal lattice Boltzmann scheme with arbitrary
 * specific-heat ratio (Hu, Zhang & Geng, arXiv:1608.06345).
 *
 * TEST INFRASTRUCTURE ONLY.  The HIP product path never links or calls this
 * file; it shares no code, header or table with it.  It is plain, slow and
 * written to be checked against the paper by eye:
 *
 *   state      two reduced distributions per cell, g_i (mass) and h_i
 *              (energy), Sec. II; stored cell-major: g[cell * Q + i].
 *   moments    rho = sum g_i, rho u = sum g_i xi_i,
 *              rho E = sum (1/2) xi_i^2 g_i + sum h_i            (Sec. II)
 *   temperature  E = u^2/2 + (D + delta) T / 2  (dimensionless energy,
 *              Sec. II), so T = (2E - u^2) / (D + delta)
 *   equilibrium  F_i = w_i rho sum_{k<=4} a(k).H(k) / k!         (Sec. IV)
 *              with the Hermite contractions written out below
 *   collision  g_i <- g_i - (g_i - F_i) / tau_f,
 *              h_i <- h_i - (h_i - (delta/2) T F_i) / tau_g     (Sec. II/III)
 *   streaming  population i moves e_i cells per step (the lattice time step
 *              Delta x = r Delta t implied by the time conversion of Sec. V)
 *
 * One step is S_{n+1} = Stream(Collide(S_n)); the initial state is the
 * equilibrium of the initial fields.
 *
 * The finite-difference form of Sec. III (orc_fd_step) advances the same two
 * distributions explicitly in time with a free time step dt (grid step 1,
 * particle speeds xi_i = r e_i):
 *   g_i(t+dt) = g_i - dt xi_i . grad g_i - (dt/tau_f) (g_i - F_i),
 *   h_i(t+dt) = h_i - dt xi_i . grad h_i - (dt/tau_g) (h_i - (delta/2) T F_i),
 * everything on the right at time t, the convection term per axis by the
 * third-order upwind-biased difference of Sec. III.  There tau_f and tau_g
 * are relaxation times in the units of dt.
 *
 * Boundary conditions, per axis: periodic (wrap) or open.  The paper leaves
 * the open condition unspecified (Sec. V); it is read as zero gradient: the
 * populations that stream in from beyond an open end are the post-collision
 * populations of the end cell itself, i.e. the pull source coordinate is
 * clamped to [0, n-1].
 *
 * Parallelism: OpenMP over cells (static schedule); no blocking, no fusion.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QMAX 128

typedef struct {
    int D;             /* 2 or 3 */
    int Q;             /* 37 or 107 */
    const long *e;     /* Q x D integer lattice vectors, row-major */
    const double *w;   /* Q weights */
    double r;          /* scale: xi_i = r e_i */
    double delta;      /* internal degrees of freedom */
    double tau_f;      /* relaxation time of g */
    double tau_g;      /* relaxation time of h */
    long n[3];         /* grid size per axis; n[2] = 1 in 2D */
    int open_end[3];   /* 1: zero-gradient (open) axis, 0: periodic */
    int energy_fix;    /* 1: energy-conserving collision for tau_f != tau_g */
} orc_model;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Equilibrium of the mass distribution at one cell (Sec. IV): the
 * fourth-order Hermite expansion of the reduced Maxwellian
 * rho (2 pi theta)^(-D/2) exp(-|xi - u|^2 / (2 theta)).
 *
 * With c = xi.u, U = |u|^2, q = |xi|^2 and t = theta - 1, the contractions
 * a(k).H(k) / rho are
 *   k=0: 1
 *   k=1: c
 *   k=2: c^2 - U + t (q - D)
 *   k=3: c (c^2 - 3U + 3 t (q - D - 2))
 *   k=4: c^4 - 6 c^2 U + 3 U^2 + 6 t (c^2 (q - D - 4) + (D + 2 - q) U)
 *        + 3 t^2 (q^2 - 2 (D + 2) q + D (D + 2))
 * The printed k = 2..4 lines exchange xi and u (or theta) in several places;
 * the forms above are the ones that follow from contracting the Hermite
 * tensors H(2..4) with the Maxwellian coefficients
 * a(2) = rho (uu + t I), a(3) = rho (uuu + t [I u]_3),
 * a(4) = rho (uuuu + t [I uu]_6 + t^2 [I I]_3). */
void orc_feq(const orc_model *m, double rho, const double *u, double theta,
             double *F)
{
    const int D = m->D;
    double U = 0.0;
    for (int k = 0; k < D; ++k) U += u[k] * u[k];
    const double t = theta - 1.0;
    for (int i = 0; i < m->Q; ++i) {
        double c = 0.0, q = 0.0;
        for (int k = 0; k < D; ++k) {
            const double xi = m->r * (double)m->e[i * D + k];
            c += xi * u[k];
            q += xi * xi;
        }
        const double h0 = 1.0;
        const double h1 = c;
        const double h2 = c * c - U + t * (q - D);
        const double h3 = c * (c * c - 3.0 * U + 3.0 * t * (q - D - 2.0));
        const double h4 = c * c * c * c - 6.0 * c * c * U + 3.0 * U * U
                        + 6.0 * t * (c * c * (q - D - 4.0) + (D + 2.0 - q) * U)
                        + 3.0 * t * t * (q * q - 2.0 * (D + 2.0) * q + D * (D + 2.0));
        F[i] = m->w[i] * rho * (h0 + h1 + h2 / 2.0 + h3 / 6.0 + h4 / 24.0);
    }
}

/* Macroscopic fields of one cell (Sec. II): rho, u (D), specific total
 * energy E and temperature T. */
void orc_macro(const orc_model *m, const double *g, const double *h,
               double *rho_out, double *u_out, double *E_out, double *T_out)
{
    const int D = m->D;
    double rho = 0.0, mom[3] = {0.0, 0.0, 0.0}, rhoE = 0.0;
    for (int i = 0; i < m->Q; ++i) {
        double q = 0.0;
        for (int k = 0; k < D; ++k) {
            const double xi = m->r * (double)m->e[i * D + k];
            mom[k] += g[i] * xi;
            q += xi * xi;
        }
        rho += g[i];
        rhoE += 0.5 * q * g[i] + h[i];
    }
    double U = 0.0;
    for (int k = 0; k < D; ++k) {
        u_out[k] = mom[k] / rho;
        U += u_out[k] * u_out[k];
    }
    const double E = rhoE / rho;
    *rho_out = rho;
    *E_out = E;
    *T_out = (2.0 * E - U) / (D + m->delta);
}

/* Energy-conserving collision (not part of the paper; a separate mode).
 * With rates a_f, a_g (1/tau, or dt/tau in the finite-difference form) the
 * BGK step changes the cell's total energy by
 *   (a_f - a_g) (E_tr^eq - E_tr),   E_tr = sum xi^2 g / 2,
 * E_tr^eq = rho (u^2 + D T) / 2 its equilibrium value, because the internal
 * part sum h relaxes at the other rate toward the complement.  Relaxing h
 * toward ((delta/2) T + kappa) F instead, with
 *   kappa rho = (1 - a_f / a_g) (E_tr^eq - E_tr),
 * makes the step conserve energy exactly; kappa = 0 when tau_f = tau_g.
 * Returns kappa (0 when the mode is off). */
static double energy_fix_kappa(const orc_model *m, const double *g, double rho,
                               const double *u, double T)
{
    if (!m->energy_fix) return 0.0;
    const int D = m->D;
    double e_tr = 0.0, U = 0.0;
    for (int i = 0; i < m->Q; ++i) {
        double q = 0.0;
        for (int k = 0; k < D; ++k) {
            const double xi = m->r * (double)m->e[i * D + k];
            q += xi * xi;
        }
        e_tr += 0.5 * q * g[i];
    }
    for (int k = 0; k < D; ++k) U += u[k] * u[k];
    const double e_tr_eq = 0.5 * rho * (U + D * T);
    /* a_f / a_g = tau_g / tau_f in both forms */
    return (1.0 - m->tau_g / m->tau_f) * (e_tr_eq - e_tr) / rho;
}

/* BGK relaxation of one cell in place (Sec. II reduced equations, explicit
 * in time as in Sec. III): g toward F, h toward (delta/2) T F (plus kappa F
 * in the energy-conserving mode). */
void orc_collide_cell(const orc_model *m, double *g, double *h)
{
    double rho, u[3], E, T;
    double F[ORC_QMAX];
    orc_macro(m, g, h, &rho, u, &E, &T);
    orc_feq(m, rho, u, T, F);
    const double kappa = energy_fix_kappa(m, g, rho, u, T);
    for (int i = 0; i < m->Q; ++i) {
        g[i] = g[i] - (g[i] - F[i]) / m->tau_f;
        h[i] = h[i] - (h[i] - (0.5 * m->delta * T + kappa) * F[i]) / m->tau_g;
    }
}

static long ncells(const orc_model *m) { return m->n[0] * m->n[1] * m->n[2]; }

/* Pull source coordinate along one axis for destination x and shift e
 * (also: the coordinate of the neighbour x + d is source_coord(x, -d, ...)). */
static long source_coord(long x, long e, long n, int open_end)
{
    long s = x - e;
    if (open_end) {
        if (s < 0) s = 0;
        if (s > n - 1) s = n - 1;
        return s;
    }
    s %= n;
    if (s < 0) s += n;
    return s;
}

/* Initial state: g_i = F_i(rho, u, T), h_i = (delta/2) T F_i.
 * rho, T: [cells]; u: [D][cells]; cell = x + nx (y + ny z). */
void orc_init(const orc_model *m, const double *rho, const double *u,
              const double *T, double *g, double *h)
{
    const long N = ncells(m);
    const int Q = m->Q, D = m->D;
    #pragma omp parallel
    {
        double *F = (double *)malloc(sizeof(double) * (size_t)Q);
        #pragma omp for schedule(static)
        for (long c = 0; c < N; ++c) {
            double uc[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < D; ++k) uc[k] = u[k * N + c];
            orc_feq(m, rho[c], uc, T[c], F);
            for (int i = 0; i < Q; ++i) {
                g[c * Q + i] = F[i];
                h[c * Q + i] = 0.5 * m->delta * T[c] * F[i];
            }
        }
        free(F);
    }
}

/* n time steps in place: collide every cell, then stream every population. */
int orc_step(const orc_model *m, double *g, double *h, long nsteps)
{
    const long N = ncells(m);
    const int Q = m->Q, D = m->D;
    double *gp = (double *)malloc(sizeof(double) * (size_t)(N * Q));
    double *hp = (double *)malloc(sizeof(double) * (size_t)(N * Q));
    if (!gp || !hp) { free(gp); free(hp); return -2; }
    for (long step = 0; step < nsteps; ++step) {
        /* collision: post-collision copy gp, hp */
        #pragma omp parallel for schedule(static)
        for (long c = 0; c < N; ++c) {
            memcpy(gp + c * Q, g + c * Q, sizeof(double) * (size_t)Q);
            memcpy(hp + c * Q, h + c * Q, sizeof(double) * (size_t)Q);
            orc_collide_cell(m, gp + c * Q, hp + c * Q);
        }
        /* streaming: S(x, i) = P(x - e_i, i) with the boundary rule above */
        #pragma omp parallel for schedule(static)
        for (long c = 0; c < N; ++c) {
            long x[3];
            x[0] = c % m->n[0];
            x[1] = (c / m->n[0]) % m->n[1];
            x[2] = c / (m->n[0] * m->n[1]);
            for (int i = 0; i < Q; ++i) {
                long s[3] = {0, 0, 0};
                for (int k = 0; k < 3; ++k) {
                    const long ek = k < D ? m->e[i * D + k] : 0;
                    s[k] = source_coord(x[k], ek, m->n[k], m->open_end[k]);
                }
                const long src = s[0] + m->n[0] * (s[1] + m->n[1] * s[2]);
                g[c * Q + i] = gp[src * Q + i];
                h[c * Q + i] = hp[src * Q + i];
            }
        }
    }
    free(gp);
    free(hp);
    return 0;
}


/* xi_a d(p)/dx_a of one population along one axis at x (Sec. III): the
 * third-order upwind-biased difference, its stencil leaning against the
 * direction of xi_a, grid step 1:
 *   xi > 0:  xi [p(x-2) - 6 p(x-1) + 3 p(x) + 2 p(x+1)] / 6
 *   xi < 0:  xi [-p(x+2) + 6 p(x+1) - 3 p(x) - 2 p(x-1)] / 6
 * (the paper writes both halves at once with (xi +- |xi|)/2).  p_at(d)
 * is the population at the neighbour x + d along the axis. */
static double upwind_convection(double xi, const double p_at[5])
{
    /* p_at[d + 2] = p(x + d), d = -2..2 */
    const double plus = (p_at[0] - 6.0 * p_at[1] + 3.0 * p_at[2] + 2.0 * p_at[3]) / 6.0;
    const double minus = (-p_at[4] + 6.0 * p_at[3] - 3.0 * p_at[2] - 2.0 * p_at[1]) / 6.0;
    return 0.5 * (xi + fabs(xi)) * plus + 0.5 * (xi - fabs(xi)) * minus;
}

/* nsteps explicit steps of the finite-difference form (see the header).
 * Open ends: a neighbour beyond the end takes the end cell's value (zero
 * gradient), the same reading as for streaming. */
int orc_fd_step(const orc_model *m, double *g, double *h, long nsteps, double dt)
{
    const long N = ncells(m);
    const int Q = m->Q, D = m->D;
    double *gn = (double *)malloc(sizeof(double) * (size_t)(N * Q));
    double *hn = (double *)malloc(sizeof(double) * (size_t)(N * Q));
    if (!gn || !hn) { free(gn); free(hn); return -2; }
    for (long step = 0; step < nsteps; ++step) {
        #pragma omp parallel for schedule(static)
        for (long c = 0; c < N; ++c) {
            long x[3];
            x[0] = c % m->n[0];
            x[1] = (c / m->n[0]) % m->n[1];
            x[2] = c / (m->n[0] * m->n[1]);
            double rho, u[3] = {0.0, 0.0, 0.0}, E, T;
            double F[ORC_QMAX];
            orc_macro(m, g + c * Q, h + c * Q, &rho, u, &E, &T);
            orc_feq(m, rho, u, T, F);
            const double kappa = energy_fix_kappa(m, g + c * Q, rho, u, T);
            for (int i = 0; i < Q; ++i) {
                double conv_g = 0.0, conv_h = 0.0;
                for (int a = 0; a < D; ++a) {
                    const double xi = m->r * (double)m->e[i * D + a];
                    if (xi == 0.0) continue;
                    double pg[5], ph[5];
                    for (int d = -2; d <= 2; ++d) {
                        long y[3] = {x[0], x[1], x[2]};
                        y[a] = source_coord(x[a], -d, m->n[a], m->open_end[a]);
                        const long nb = y[0] + m->n[0] * (y[1] + m->n[1] * y[2]);
                        pg[d + 2] = g[nb * Q + i];
                        ph[d + 2] = h[nb * Q + i];
                    }
                    conv_g += upwind_convection(xi, pg);
                    conv_h += upwind_convection(xi, ph);
                }
                const double gi = g[c * Q + i], hi = h[c * Q + i];
                gn[c * Q + i] = gi - dt * conv_g - dt / m->tau_f * (gi - F[i]);
                hn[c * Q + i] = hi - dt * conv_h
                              - dt / m->tau_g * (hi - (0.5 * m->delta * T + kappa) * F[i]);
            }
        }
        memcpy(g, gn, sizeof(double) * (size_t)(N * Q));
        memcpy(h, hn, sizeof(double) * (size_t)(N * Q));
    }
    free(gn);
    free(hn);
    return 0;
}

/* Per-cell moments of the state: rho [cells], u [D][cells], E [cells]. */
void orc_moments(const orc_model *m, const double *g, const double *h,
                 double *rho, double *u, double *E)
{
    const long N = ncells(m);
    const int Q = m->Q, D = m->D;
    #pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
        double r_, uc[3], e_, t_;
        orc_macro(m, g + c * Q, h + c * Q, &r_, uc, &e_, &t_);
        rho[c] = r_;
        for (int k = 0; k < D; ++k) u[k * N + c] = uc[k];
        E[c] = e_;
    }
}

/* Domain totals: mass, momentum (D), total energy; plain serial sums. */
void orc_totals(const orc_model *m, const double *g, const double *h,
                double *mass, double *mom, double *energy)
{
    const long N = ncells(m);
    const int Q = m->Q, D = m->D;
    double M = 0.0, P[3] = {0.0, 0.0, 0.0}, En = 0.0;
    for (long c = 0; c < N; ++c) {
        for (int i = 0; i < Q; ++i) {
            double q = 0.0;
            for (int k = 0; k < D; ++k) {
                const double xi = m->r * (double)m->e[i * D + k];
                P[k] += g[c * Q + i] * xi;
                q += xi * xi;
            }
            M += g[c * Q + i];
            En += 0.5 * q * g[c * Q + i] + h[c * Q + i];
        }
    }
    *mass = M;
    for (int k = 0; k < D; ++k) mom[k] = P[k];
    *energy = En;
}
