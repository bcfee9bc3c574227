/*
 * dpml_oracle.c -- plain FP64 CPU oracle for the reflectionless discrete PML
 * of A. Chern, "A Reflectionless Discrete Perfectly Matched Layer"
 * (J. Comput. Phys.; arXiv 1804.01390).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * What it computes (paper notation, grid spacing h, per-axis shift tau_a):
 *
 *   Eq. (DiscretePML a):
 *     U_tt = c^2 * sum_a (tau_a^-1 U - 2U + tau_a U)/h^2
 *            + sum_a (1/h) ( sigma_a * tau_a Psi_a - (tau_a^-1 sigma_a)(tau_a^-1 Phi_a) )
 *   Eq. (DiscretePML b):
 *     Phi_a,t = -1/2 ( (tau_a^-1 sigma_a)(tau_a^-1 Phi_a) + sigma_a Phi_a )
 *               - (tau_a U - tau_a^-1 U)/(2h)
 *   Eq. (DiscretePML c):
 *     Psi_a,t = -1/2 ( (tau_a^-1 sigma_a) Psi_a + sigma_a (tau_a Psi_a) )
 *               - (tau_a U - tau_a^-1 U)/(2h)
 *
 * The equations are evaluated at EVERY cell of the grid (the paper states
 * them on all of Z^d; the restriction of Phi/Psi to the layer in Sec. 1.1.2
 * is an economy, not part of the definition).  Each axis is truncated either
 * periodically (Sec. 1.1.3, the runs of Figs. 2 and 3) or by reflecting walls
 * (the truncation the paper analyses with Eq. (IntroReflectedDecayBound)):
 * U, Phi and Psi vanish on the ghost cells -1 and N, and the ghost edge
 * [-1, 0] carries no damping.  The coefficient c^2 multiplies the
 * Laplacian only; it must equal 1 wherever a damping term acts (the paper
 * uses unit wave speed).
 *
 * Time discretisation (the paper's runs use RK4 with an unstated step; this
 * oracle follows the leapfrog reading): U by the explicit central
 * second difference, Phi and Psi by a forward step, and every right-hand
 * side of one step evaluated from time-level-n data only:
 *
 *   U^{n+1}   = 2 U^n - U^{n-1} + dt^2 * A(U^n, Phi^n, Psi^n)
 *   Phi^{n+1} = Phi^n + dt * B(U^n, Phi^n)
 *   Psi^{n+1} = Psi^n + dt * C(U^n, Psi^n)
 *
 * With that placement the Fourier-domain derivation of Sec. 3.3 carries over
 * with -omega^2 -> (z - 2 + 1/z)/dt^2 in Eq. (UEquationFourier) and
 * -i omega -> (z - 1)/dt in Eqs. (PhiEquationFourier), (PsiEquationFourier),
 * z the one-step amplification factor; the discrete plane waves of Thm. 1
 * then continue into the layer exactly, with decay factor rho(s, k, omega')
 * and omega' = i (z - 1)/dt.
 *
 * Start (zero or given initial velocity, Phi = Psi = 0):
 *   U^{-1} = U^0 - dt V^0 + dt^2/2 * A(U^0, 0, 0)
 *
 * Point sources (not in the paper): after step n (U^n -> U^{n+1}),
 *   U^{n+1}[s] += dt^2 * w_s[n] / h^d,  and receivers record U^{n+1}[r].
 *
 * Arrays are row-major with axis 0 (x) fastest: cell (x, y, z) sits at
 * x + N0*(y + N1*z).  Unused axes have extent 1.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t ndim;            /* 1, 2 or 3 */
    int32_t pad_;
    int64_t N[3];            /* cells per axis, axis 0 fastest; unused axes 1 */
    double h;                /* grid spacing */
    double dt;               /* time step */
    const double *c2;        /* NULL: c^2 = 1; else one value per cell */
    const double *sigma[3];  /* sigma_a(i_a), N[a] values each; NULL = all 0 */
    int32_t wall[3];         /* 0: periodic axis; 1: reflecting walls, i.e. U, Phi,
                                Psi vanish on ghost cells -1 and N[a], and the
                                ghost edge [-1, 0] carries no damping */
    int32_t pad2_;
} orc_grid;

static int64_t orc_wrap(int64_t i, int64_t n)
{
    if (i < 0) return i + n;
    if (i >= n) return i - n;
    return i;
}

static double orc_sigma(const orc_grid *g, int a, int64_t i)
{
    if (i < 0) return 0.0;          /* ghost edge outside a wall */
    return g->sigma[a] ? g->sigma[a][i] : 0.0;
}

/* Value of array X at flat index c, or 0 for a ghost cell (c < 0). */
static double orc_at(const double *X, int64_t c)
{
    return c < 0 ? 0.0 : X[c];
}

/* Decompose a flat cell index into per-axis indices. */
static void orc_coords(const orc_grid *g, int64_t c, int64_t ii[3])
{
    ii[0] = c % g->N[0];
    ii[1] = (c / g->N[0]) % g->N[1];
    ii[2] = c / (g->N[0] * g->N[1]);
}

static int64_t orc_stride(const orc_grid *g, int a)
{
    if (a == 0) return 1;
    if (a == 1) return g->N[0];
    return g->N[0] * g->N[1];
}

/* Flat index of the cell one step along axis a (dir = +1 or -1): periodic,
 * or -1 (a ghost cell) past a wall. */
static int64_t orc_shift(const orc_grid *g, int64_t c, const int64_t ii[3], int a, int dir)
{
    int64_t t = ii[a] + dir;
    if (g->wall[a] && (t < 0 || t >= g->N[a])) return -1;
    int64_t j = orc_wrap(t, g->N[a]);
    return c + (j - ii[a]) * orc_stride(g, a);
}

/* Index of the edge left of cell i along axis a: i-1, periodic or -1 at a wall. */
static int64_t orc_left(const orc_grid *g, int a, int64_t i)
{
    if (g->wall[a] && i == 0) return -1;
    return orc_wrap(i - 1, g->N[a]);
}

static int64_t orc_ncells(const orc_grid *g)
{
    return g->N[0] * g->N[1] * g->N[2];
}

/* Right-hand side of Eq. (DiscretePML a) at cell c. Phi/Psi may be NULL
 * (treated as zero, used at the start). */
static double orc_rhs_u(const orc_grid *g, const double *U,
                        double *const Phi[3], double *const Psi[3], int64_t c)
{
    int64_t ii[3];
    double lap = 0.0, damp = 0.0;
    orc_coords(g, c, ii);
    for (int a = 0; a < g->ndim; ++a) {
        int64_t cp = orc_shift(g, c, ii, a, +1);
        int64_t cm = orc_shift(g, c, ii, a, -1);
        int64_t im = orc_left(g, a, ii[a]);
        lap += (orc_at(U, cm) - 2.0 * U[c] + orc_at(U, cp)) / (g->h * g->h);
        if (Phi && Psi) {
            double s_here = orc_sigma(g, a, ii[a]);   /* sigma_a        */
            double s_left = orc_sigma(g, a, im);      /* tau^-1 sigma_a */
            damp += (s_here * orc_at(Psi[a], cp) - s_left * orc_at(Phi[a], cm)) / g->h;
        }
    }
    return (g->c2 ? g->c2[c] : 1.0) * lap + damp;
}

/* Right-hand side of Eq. (DiscretePML b) for Phi_a at cell c. */
static double orc_rhs_phi(const orc_grid *g, const double *U, const double *Phi_a,
                          int a, int64_t c)
{
    int64_t ii[3];
    orc_coords(g, c, ii);
    int64_t cp = orc_shift(g, c, ii, a, +1);
    int64_t cm = orc_shift(g, c, ii, a, -1);
    int64_t im = orc_left(g, a, ii[a]);
    double s_here = orc_sigma(g, a, ii[a]);
    double s_left = orc_sigma(g, a, im);
    return -0.5 * (s_left * orc_at(Phi_a, cm) + s_here * Phi_a[c])
           - (orc_at(U, cp) - orc_at(U, cm)) / (2.0 * g->h);
}

/* Right-hand side of Eq. (DiscretePML c) for Psi_a at cell c. */
static double orc_rhs_psi(const orc_grid *g, const double *U, const double *Psi_a,
                          int a, int64_t c)
{
    int64_t ii[3];
    orc_coords(g, c, ii);
    int64_t cp = orc_shift(g, c, ii, a, +1);
    int64_t cm = orc_shift(g, c, ii, a, -1);
    int64_t im = orc_left(g, a, ii[a]);
    double s_here = orc_sigma(g, a, ii[a]);
    double s_left = orc_sigma(g, a, im);
    return -0.5 * (s_left * Psi_a[c] + s_here * orc_at(Psi_a, cp))
           - (orc_at(U, cp) - orc_at(U, cm)) / (2.0 * g->h);
}

/* Start: U^{-1} = U^0 - dt V^0 + dt^2/2 A(U^0, 0, 0).  V0 may be NULL. */
void orc_start(const orc_grid *g, const double *U0, const double *V0, double *Um1)
{
    int64_t n = orc_ncells(g);
    double dt = g->dt;
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        double a = orc_rhs_u(g, U0, NULL, NULL, c);
        double v = V0 ? V0[c] : 0.0;
        Um1[c] = U0[c] - dt * v + 0.5 * dt * dt * a;
    }
}

/* One step of the scheme from time-n data only.
 * Inputs: Un, Unm1, Phi[a], Psi[a] (time n).  Outputs: Unp1, PhiN[a], PsiN[a]
 * (time n+1); outputs must not alias inputs. */
void orc_step(const orc_grid *g, const double *Un, const double *Unm1,
              double *const Phi[3], double *const Psi[3],
              double *Unp1, double *const PhiN[3], double *const PsiN[3])
{
    int64_t n = orc_ncells(g);
    double dt = g->dt;
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        double a = orc_rhs_u(g, Un, Phi, Psi, c);
        Unp1[c] = 2.0 * Un[c] - Unm1[c] + dt * dt * a;
        for (int ax = 0; ax < g->ndim; ++ax) {
            PhiN[ax][c] = Phi[ax][c] + dt * orc_rhs_phi(g, Un, Phi[ax], ax, c);
            PsiN[ax][c] = Psi[ax][c] + dt * orc_rhs_psi(g, Un, Psi[ax], ax, c);
        }
    }
}

/* Add the point-source term of step `n` to U^{n+1} and record receivers.
 * wavelets: [ns][nt] row-major; traces: [nr][nt] row-major. */
static void orc_sources_receivers(const orc_grid *g, double *Unp1, int64_t n,
                                  int64_t ns, const int64_t *src, const double *wav,
                                  int64_t nr, const int64_t *rec, double *traces,
                                  int64_t nt)
{
    double hd = 1.0;
    for (int a = 0; a < g->ndim; ++a) hd *= g->h;
    if (n < nt) {
        for (int64_t s = 0; s < ns; ++s)
            Unp1[src[s]] += g->dt * g->dt * wav[s * nt + n] / hd;
        for (int64_t r = 0; r < nr; ++r)
            traces[r * nt + n] = Unp1[rec[r]];
    }
}

/* Run `nsteps` steps in place.  On entry U = U^{n0}, Uprev = U^{n0-1},
 * Phi/Psi at n0; on return they hold time n0+nsteps.  Step n0+k uses wavelet
 * sample n0+k and writes trace column n0+k (when n0+k < nt).
 * The run works on private copies, so the caller's arrays are only read at
 * entry and written at exit.  Returns 0, or -1 if out of memory. */
int orc_run(const orc_grid *g, double *U, double *Uprev,
            double *const Phi[3], double *const Psi[3],
            int64_t n0, int64_t nsteps,
            int64_t ns, const int64_t *src, const double *wav,
            int64_t nr, const int64_t *rec, double *traces, int64_t nt)
{
    int64_t n = orc_ncells(g);
    size_t bytes = (size_t)n * sizeof(double);
    /* private buffers: u[0..2] for U, f[a][0..1] for Phi_a, p[a][0..1] for Psi_a */
    double *u[3] = {0, 0, 0};
    double *f[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    double *p[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    int ok = 1;
    for (int k = 0; k < 3; ++k) ok &= (u[k] = malloc(bytes)) != NULL;
    for (int a = 0; a < g->ndim; ++a)
        for (int k = 0; k < 2; ++k) {
            ok &= (f[a][k] = malloc(bytes)) != NULL;
            ok &= (p[a][k] = malloc(bytes)) != NULL;
        }
    if (ok) {
        memcpy(u[0], U, bytes);      /* U^n     */
        memcpy(u[1], Uprev, bytes);  /* U^{n-1} */
        for (int a = 0; a < g->ndim; ++a) {
            memcpy(f[a][0], Phi[a], bytes);
            memcpy(p[a][0], Psi[a], bytes);
        }
        int inow = 0, iold = 1, inew = 2, cur = 0;
        for (int64_t k = 0; k < nsteps; ++k) {
            double *phi_now[3] = {0, 0, 0}, *psi_now[3] = {0, 0, 0};
            double *phi_new[3] = {0, 0, 0}, *psi_new[3] = {0, 0, 0};
            for (int a = 0; a < g->ndim; ++a) {
                phi_now[a] = f[a][cur]; phi_new[a] = f[a][1 - cur];
                psi_now[a] = p[a][cur]; psi_new[a] = p[a][1 - cur];
            }
            orc_step(g, u[inow], u[iold], phi_now, psi_now, u[inew], phi_new, psi_new);
            orc_sources_receivers(g, u[inew], n0 + k, ns, src, wav, nr, rec, traces, nt);
            int t = iold; iold = inow; inow = inew; inew = t;
            cur = 1 - cur;
        }
        memcpy(U, u[inow], bytes);
        memcpy(Uprev, u[iold], bytes);
        for (int a = 0; a < g->ndim; ++a) {
            memcpy(Phi[a], f[a][cur], bytes);
            memcpy(Psi[a], p[a][cur], bytes);
        }
    }
    for (int k = 0; k < 3; ++k) free(u[k]);
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 2; ++k) { free(f[a][k]); free(p[a][k]); }
    return ok ? 0 : -1;
}

/* Plain discrete wave equation, Eq. (DiscreteWaveEquation), leapfrog, with no
 * damping terms at all: the untruncated "free space" reference.
 * On entry U = U^{n0}, Uprev = U^{n0-1}; on return time n0+nsteps. */
int orc_wave_run(const orc_grid *g, double *U, double *Uprev, int64_t nsteps)
{
    int64_t n = orc_ncells(g);
    size_t bytes = (size_t)n * sizeof(double);
    double *u[3] = {malloc(bytes), malloc(bytes), malloc(bytes)};
    double dt2 = g->dt * g->dt;
    if (!u[0] || !u[1] || !u[2]) {
        free(u[0]); free(u[1]); free(u[2]);
        return -1;
    }
    memcpy(u[0], U, bytes);
    memcpy(u[1], Uprev, bytes);
    int inow = 0, iold = 1, inew = 2;
    const int64_t rows = g->N[1] * g->N[2];
    for (int64_t k = 0; k < nsteps; ++k) {
        const double *un = u[inow], *uo = u[iold];
        double *uw = u[inew];
        /* one row of cells (fixed y, z) per iteration: the same per-cell
         * expression, without recovering the coordinates by division */
        #pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < rows; ++r) {
            const int64_t N0 = g->N[0], base = r * N0;
            int64_t ii[3] = {0, r % g->N[1], r / g->N[1]};
            /* the rows above/below and the planes before/after (index of the
             * row's first cell; -1 for a ghost row past a wall) */
            int64_t nb[3][2] = {{0, 0}, {0, 0}, {0, 0}};
            for (int a = 1; a < g->ndim; ++a) {
                nb[a][0] = orc_shift(g, base, ii, a, -1);
                nb[a][1] = orc_shift(g, base, ii, a, +1);
            }
            const double h2 = g->h * g->h;
            for (int64_t x = 0; x < N0; ++x) {
                const int64_t c = base + x;
                double lap = 0.0;
                ii[0] = x;
                {
                    int64_t cp = orc_shift(g, c, ii, 0, +1);
                    int64_t cm = orc_shift(g, c, ii, 0, -1);
                    lap += (orc_at(un, cm) - 2.0 * un[c] + orc_at(un, cp)) / h2;
                }
                for (int a = 1; a < g->ndim; ++a) {
                    double um = nb[a][0] < 0 ? 0.0 : un[nb[a][0] + x];
                    double up = nb[a][1] < 0 ? 0.0 : un[nb[a][1] + x];
                    lap += (um - 2.0 * un[c] + up) / h2;
                }
                uw[c] = 2.0 * un[c] - uo[c] + dt2 * (g->c2 ? g->c2[c] : 1.0) * lap;
            }
        }
        int t = iold; iold = inow; inow = inew; inew = t;
    }
    memcpy(U, u[inow], bytes);
    memcpy(Uprev, u[iold], bytes);
    free(u[0]); free(u[1]); free(u[2]);
    return 0;
}

/* ------------------------------------------------------------------------
 * Discrete adjoint (reverse mode) of orc_start + orc_run with point sources
 * and receivers, for the misfit J = 1/2 sum_{r,n} (d_r[n] - obs_r[n])^2 where
 * d_r[n] = U^{n+1}[rec_r] after step n.  The caller passes the residual
 * resid[r][n] = d_r[n] - obs_r[n]; the routine returns
 *   grad_c2[c]   = dJ/dc^2(c)       (c^2 given per cell; NULL c2 means 1)
 *   grad_w[s][n] = dJ/dw_s[n]
 * The forward levels U^0..U^{N-1} are recomputed and stored in full (plain,
 * no checkpointing).  Zero initial velocity and Phi = Psi = 0 at start.
 *
 * Transposing one step (x^{n+1} = T x^n + b^n) gives, with a^k the adjoint
 * of U^k and p_a, q_a those of Phi_a, Psi_a at level n+1:
 *   grad_c2   += dt^2 a^{n+1} * (L U^n)                (L: periodic Laplacian)
 *   a^n        = 2 a^{n+1} - a^{n+2} + dt^2 L(c^2 a^{n+1})
 *                + dt sum_a G_a(p_a + q_a)             (G_a^T = -G_a)
 *   p_a^n(i)   = p_a(i) - dt/2 sigma(i)(p_a(i) + p_a(i+e))   - dt^2/h sigma(i)   a^{n+1}(i+e)
 *   q_a^n(i)   = q_a(i) - dt/2 sigma(i-1)(q_a(i) + q_a(i-e)) + dt^2/h sigma(i-1) a^{n+1}(i-e)
 * with G_a U = (U(i+e) - U(i-e))/(2h).  The start U^{-1} = U^0 + dt^2/2 c^2 L U^0
 * adds  grad_c2 += dt^2/2 a^{-1} L U^0, with a^{-1} = -a^1.
 * ------------------------------------------------------------------------ */
static double orc_lap(const orc_grid *g, const double *U, int64_t c)
{
    int64_t ii[3];
    double lap = 0.0;
    orc_coords(g, c, ii);
    for (int a = 0; a < g->ndim; ++a) {
        int64_t cp = orc_shift(g, c, ii, a, +1);
        int64_t cm = orc_shift(g, c, ii, a, -1);
        lap += (orc_at(U, cm) - 2.0 * U[c] + orc_at(U, cp)) / (g->h * g->h);
    }
    return lap;
}

int orc_adjoint(const orc_grid *g, const double *U0, int64_t nsteps,
                int64_t ns, const int64_t *src, const double *wav,
                int64_t nr, const int64_t *rec, const double *resid,
                double *grad_c2, double *grad_w)
{
    int64_t n = orc_ncells(g);
    int d = g->ndim;
    size_t bytes = (size_t)n * sizeof(double);
    double hd = 1.0;
    for (int a = 0; a < d; ++a) hd *= g->h;
    double dt = g->dt, dt2 = dt * dt;
    int ok = 1;
    /* forward: store U^0 .. U^{N-1} */
    double *hist = malloc(bytes * (size_t)(nsteps > 0 ? nsteps : 1));
    double *Uprev = malloc(bytes), *U = malloc(bytes);
    double *Phi[3] = {0, 0, 0}, *Psi[3] = {0, 0, 0};
    ok &= hist && Uprev && U;
    for (int a = 0; a < d; ++a) {
        ok &= (Phi[a] = calloc((size_t)n, sizeof(double))) != NULL;
        ok &= (Psi[a] = calloc((size_t)n, sizeof(double))) != NULL;
    }
    /* adjoint buffers */
    double *a_next = calloc((size_t)n, sizeof(double));   /* a^{n+2} */
    double *a_cur = calloc((size_t)n, sizeof(double));    /* a^{n+1} */
    double *a_new = calloc((size_t)n, sizeof(double));
    double *c2a = malloc(bytes);
    double *p[3] = {0, 0, 0}, *q[3] = {0, 0, 0}, *pn[3] = {0, 0, 0}, *qn[3] = {0, 0, 0};
    ok &= a_next && a_cur && a_new && c2a;
    for (int a = 0; a < d; ++a) {
        ok &= (p[a] = calloc((size_t)n, sizeof(double))) != NULL;
        ok &= (q[a] = calloc((size_t)n, sizeof(double))) != NULL;
        ok &= (pn[a] = calloc((size_t)n, sizeof(double))) != NULL;
        ok &= (qn[a] = calloc((size_t)n, sizeof(double))) != NULL;
    }
    if (ok) {
        memcpy(U, U0, bytes);
        orc_start(g, U0, NULL, Uprev);
        for (int64_t k = 0; k < nsteps; ++k) {
            memcpy(hist + (size_t)k * (size_t)n, U, bytes);
            /* one step with a scratch traces array (not needed here) */
            orc_run(g, U, Uprev, Phi, Psi, k, 1, ns, src, wav, 0, NULL, NULL, nsteps);
        }
        memset(grad_c2, 0, bytes);
        for (int64_t k = nsteps - 1; k >= 0; --k) {
            const double *Un = hist + (size_t)k * (size_t)n;
            /* receivers read U^{k+1}: seed its adjoint with the residual */
            for (int64_t r = 0; r < nr; ++r) a_cur[rec[r]] += resid[r * nsteps + k];
            /* sources were added to U^{k+1} */
            for (int64_t s = 0; s < ns; ++s) grad_w[s * nsteps + k] = dt2 / hd * a_cur[src[s]];
            for (int64_t c = 0; c < n; ++c) c2a[c] = (g->c2 ? g->c2[c] : 1.0) * a_cur[c];
            #pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < n; ++c) {
                int64_t ii[3];
                orc_coords(g, c, ii);
                grad_c2[c] += dt2 * a_cur[c] * orc_lap(g, Un, c);
                double v = 2.0 * a_cur[c] - a_next[c] + dt2 * orc_lap(g, c2a, c);
                for (int a = 0; a < d; ++a) {
                    int64_t cp = orc_shift(g, c, ii, a, +1);
                    int64_t cm = orc_shift(g, c, ii, a, -1);
                    int64_t im = orc_left(g, a, ii[a]);
                    double s_here = orc_sigma(g, a, ii[a]);
                    double s_left = orc_sigma(g, a, im);
                    v += dt * ((orc_at(p[a], cp) + orc_at(q[a], cp)) - (orc_at(p[a], cm) + orc_at(q[a], cm)))
                         / (2.0 * g->h);
                    pn[a][c] = p[a][c] - 0.5 * dt * s_here * (p[a][c] + orc_at(p[a], cp))
                               - dt2 / g->h * s_here * orc_at(a_cur, cp);
                    qn[a][c] = q[a][c] - 0.5 * dt * s_left * (q[a][c] + orc_at(q[a], cm))
                               + dt2 / g->h * s_left * orc_at(a_cur, cm);
                }
                a_new[c] = v;
            }
            double *t = a_next; a_next = a_cur; a_cur = a_new; a_new = t;
            for (int a = 0; a < d; ++a) {
                double *tp = p[a]; p[a] = pn[a]; pn[a] = tp;
                double *tq = q[a]; q[a] = qn[a]; qn[a] = tq;
            }
        }
        /* start: a^{-1} = -a^1 (a_next now holds a^1) */
        for (int64_t c = 0; c < n; ++c)
            grad_c2[c] += 0.5 * dt2 * (-a_next[c]) * orc_lap(g, U0, c);
    }
    free(hist); free(Uprev); free(U); free(a_next); free(a_cur); free(a_new); free(c2a);
    for (int a = 0; a < 3; ++a) {
        free(Phi[a]); free(Psi[a]); free(p[a]); free(q[a]); free(pn[a]); free(qn[a]);
    }
    return ok ? 0 : -1;
}

/* ------------------------------------------------------------------------
 * The paper's own time integrator (Sec. 1.1.3: the runs use RK4): classic
 * fourth-order Runge-Kutta on the first-order system
 *   U_t = V,  V_t = A(U, Phi, Psi),  Phi_a,t = B_a(U, Phi_a),  Psi_a,t = C_a(U, Psi_a)
 * with A, B, C the right-hand sides of Eq. (DiscretePML a, b, c).
 * ------------------------------------------------------------------------ */
static void orc_rk_rhs(const orc_grid *g, const double *U, const double *V,
                       double *const Phi[3], double *const Psi[3],
                       double *dU, double *dV, double *const dPhi[3], double *const dPsi[3])
{
    int64_t n = orc_ncells(g);
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        dU[c] = V[c];
        dV[c] = orc_rhs_u(g, U, Phi, Psi, c);
        for (int a = 0; a < g->ndim; ++a) {
            dPhi[a][c] = orc_rhs_phi(g, U, Phi[a], a, c);
            dPsi[a][c] = orc_rhs_psi(g, U, Psi[a], a, c);
        }
    }
}

/* nsteps RK4 steps in place on (U, V, Phi, Psi).  Returns 0 or -1 (memory). */
int orc_rk4_run(const orc_grid *g, double *U, double *V,
                double *const Phi[3], double *const Psi[3], int64_t nsteps)
{
    int64_t n = orc_ncells(g);
    int d = g->ndim;
    size_t bytes = (size_t)n * sizeof(double);
    /* 4 stage derivatives k[s] and one stage state y, each (U, V, Phi_a, Psi_a) */
    int nf = 2 + 2 * d;
    double *buf[5][8];
    int ok = 1;
    for (int s = 0; s < 5; ++s)
        for (int f = 0; f < 8; ++f) {
            buf[s][f] = NULL;
            if (f < nf) ok &= (buf[s][f] = malloc(bytes)) != NULL;
        }
    if (ok) {
        double dt = g->dt;
        const double cst[4] = {0.0, 0.5, 0.5, 1.0};   /* stage offsets */
        const double wgt[4] = {1.0 / 6.0, 2.0 / 6.0, 2.0 / 6.0, 1.0 / 6.0};
        double *y0[8] = {U, V, 0, 0, 0, 0, 0, 0};
        for (int a = 0; a < d; ++a) { y0[2 + a] = Phi[a]; y0[2 + d + a] = Psi[a]; }
        double **ys = buf[4];
        for (int64_t k = 0; k < nsteps; ++k) {
            for (int s = 0; s < 4; ++s) {
                /* stage state y_s = y0 + cst[s] dt k_{s-1} */
                for (int f = 0; f < nf; ++f) {
                    if (s == 0) { memcpy(ys[f], y0[f], bytes); continue; }
                    const double *kp = buf[s - 1][f];
                    for (int64_t c = 0; c < n; ++c) ys[f][c] = y0[f][c] + cst[s] * dt * kp[c];
                }
                double *phs[3] = {0, 0, 0}, *pss[3] = {0, 0, 0}, *dph[3] = {0, 0, 0}, *dps[3] = {0, 0, 0};
                for (int a = 0; a < d; ++a) {
                    phs[a] = ys[2 + a]; pss[a] = ys[2 + d + a];
                    dph[a] = buf[s][2 + a]; dps[a] = buf[s][2 + d + a];
                }
                orc_rk_rhs(g, ys[0], ys[1], phs, pss, buf[s][0], buf[s][1], dph, dps);
            }
            for (int f = 0; f < nf; ++f)
                for (int64_t c = 0; c < n; ++c)
                    y0[f][c] = y0[f][c] + dt * (wgt[0] * buf[0][f][c] + wgt[1] * buf[1][f][c]
                                                + wgt[2] * buf[2][f][c] + wgt[3] * buf[3][f][c]);
        }
    }
    for (int s = 0; s < 5; ++s)
        for (int f = 0; f < 8; ++f) free(buf[s][f]);
    return ok ? 0 : -1;
}
