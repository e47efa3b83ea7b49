/*
 * osbli_oracle.c -- plain, slow, FP64 CPU oracle for the per-Runge-Kutta-
 * substage residual of the explicit compressible Navier-Stokes method of
 * Lusher, Jammy & Sandham, "OpenSBLI: automated code-generation for
 * heterogeneous computing architectures applied to compressible fluid
 * dynamics on structured grids" (arXiv 2007.14933).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; the two meet only in the
 * seeded input generators and in the array layout, which is an interface.
 *
 * Every function follows a passage of the paper, cited by section and
 * equation label.  Where the paper is silent or garbled the reading that is
 * taken is stated in place; all of them are collected in the design notes.
 * No blocking, fusion or reordering: each routine is the definition written
 * out, one interface / one node at a time.  The only parallelism is an
 * OpenMP "parallel for" over independent grid lines, which does not change
 * any arithmetic.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA, no
 * fast-math), so every operation is a correctly rounded IEEE FP64 operation
 * in the order written.
 *
 * Array layout (the interface shared with the GPU library):
 *   conserved state U[c][k][j][i], c = (rho, rho*u_0..rho*u_{ndim-1}, rho*E),
 *   i fastest, each active direction padded by 3 ghost nodes per side,
 *   inactive directions have extent 1 and no ghosts;
 *   residual / RK register arrays R[c][k][j][i], dU[c][k][j][i] over interior
 *   nodes only (no ghosts).
 *   Metrics (oracle private): S[d][m][ext] (area vector of direction d,
 *   component m, 3 components always), J[ext], on the ghost-extended grid.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NGHOST 3
#define NCMAX 5

enum { BC_PERIODIC = 0, BC_EXTRAPOLATE = 1, BC_ISOTHERMAL = 2, BC_ADIABATIC = 3, BC_DIRICHLET = 4 };
enum { SCHEME_WENOZ5 = 0, SCHEME_TENO5 = 1, SCHEME_TENO6 = 2, SCHEME_WENOJS5 = 3, SCHEME_WENOZ3 = 4,
       SCHEME_CENTRAL4 = 5, SCHEME_WENOZ7 = 6 };
enum { RK3_WILLIAMSON = 0, RK3_SSP = 1, RK4_CK = 2 };

typedef struct {
    int32_t ndim;
    int32_t pad0;
    int64_t n[3];
    double gamma, Re, Pr, Minf;   /* Re <= 0: inviscid (Euler) */
    int32_t sutherland;           /* 1: Sutherland's law, 0: mu = 1 */
    int32_t scheme;               /* SCHEME_* */
    double Ts_over_Tref;
    double teno_CT;
    double eps;                   /* epsilon of the nonlinear weights */
    int32_t roe_avg;              /* 1: Roe average, 0: arithmetic mean */
    int32_t rk;                   /* RK3_WILLIAMSON, RK3_SSP or RK4_CK */
    int32_t bc[3][2];
    double wall_T[3][2];
    double period[3];
    double body_force;            /* test-only x-momentum source (channel) */
} orc_params;

/* ------------------------------------------------------------------ grid */

typedef struct {
    int nd, nc;
    int64_t n[3], h[3], e[3], s[3];
    int64_t npts, nint;
} grid_t;

static void grid_make(const orc_params *P, grid_t *g)
{
    g->nd = P->ndim;
    g->nc = P->ndim + 2;
    for (int d = 0; d < 3; d++) {
        g->n[d] = d < P->ndim ? P->n[d] : 1;
        g->h[d] = d < P->ndim ? NGHOST : 0;
        g->e[d] = g->n[d] + 2 * g->h[d];
    }
    g->s[0] = 1;
    g->s[1] = g->e[0];
    g->s[2] = g->e[0] * g->e[1];
    g->npts = g->e[0] * g->e[1] * g->e[2];
    g->nint = g->n[0] * g->n[1] * g->n[2];
}

static int64_t gidx(const grid_t *g, int64_t i, int64_t j, int64_t k)
{
    return (i + g->h[0]) + (j + g->h[1]) * g->s[1] + (k + g->h[2]) * g->s[2];
}

static int64_t cidx(const grid_t *g, int64_t i, int64_t j, int64_t k)
{
    return i + g->n[0] * (j + g->n[1] * k);
}

static int64_t wrap(int64_t p, int64_t n) { int64_t r = p % n; return r < 0 ? r + n : r; }

/* ------------------------------------------------- state, EOS and flux --
 * Governing equations (section 2.1, eq. ns_eqn): conserved variables
 * (rho, rho u_i, rho E).  Pressure, temperature and sound speed from the
 * equation of state (eq. pressure_eqn): p = (gamma-1)(rho E - rho u_i u_i/2),
 * p = rho T / (gamma M^2), a = sqrt(gamma p / rho).
 */
typedef struct { double rho, u[3], p, T, a, H; } prim_t;

static void to_prim(const orc_params *P, int nd, const double *U, prim_t *w)
{
    double ke = 0.0;
    w->rho = U[0];
    for (int m = 0; m < 3; m++) w->u[m] = 0.0;
    for (int m = 0; m < nd; m++) {
        w->u[m] = U[1 + m] / U[0];
        ke += w->u[m] * w->u[m];
    }
    w->p = (P->gamma - 1.0) * (U[nd + 1] - 0.5 * w->rho * ke);
    w->T = P->gamma * P->Minf * P->Minf * w->p / w->rho;
    w->a = sqrt(P->gamma * w->p / w->rho);
    w->H = (U[nd + 1] + w->p) / w->rho;
}

/* Physical inviscid flux projected on the unit vector nv (the convective part
 * of eq. ns_eqn contracted with n): (rho u_n, rho u_i u_n + p n_i, (rho E + p) u_n). */
static void phys_flux(int nd, const double *U, const prim_t *w, const double *nv, double *f)
{
    double un = 0.0;
    for (int m = 0; m < nd; m++) un += w->u[m] * nv[m];
    f[0] = U[0] * un;
    for (int m = 0; m < nd; m++) f[1 + m] = U[1 + m] * un + w->p * nv[m];
    f[nd + 1] = (U[nd + 1] + w->p) * un;
}

/* ----------------------------------------- eigensystem in direction n --
 * Characteristic decomposition (section 2.2, enumerated algorithm, step 2b).
 * The paper does not print the eigenvectors; these are the textbook ones of
 * the Euler equations for a direction n.  Field order:
 *   0: u_n - a,  1: u_n (entropy),  2..nd: u_n (shear, tangents t_1..),
 *   nd+1: u_n + a.
 * Reading for the repeated eigenvalue: t_1 = normalise(e_{d+1} - (e_{d+1}.n)n),
 * t_2 = n x t_1 (indices cyclic).  Rows of L are left eigenvectors, columns of
 * R right eigenvectors, L R = I.
 */
static void tangents(int nd, int d, const double *nv, double t[2][3])
{
    memset(t, 0, sizeof(double) * 6);
    if (nd < 2) return;
    double e[3] = {0.0, 0.0, 0.0};
    e[(d + 1) % nd] = 1.0;
    double en = 0.0;
    for (int m = 0; m < nd; m++) en += e[m] * nv[m];
    double nrm = 0.0;
    for (int m = 0; m < nd; m++) { t[0][m] = e[m] - en * nv[m]; nrm += t[0][m] * t[0][m]; }
    nrm = sqrt(nrm);
    for (int m = 0; m < nd; m++) t[0][m] /= nrm;
    if (nd == 3) {
        t[1][0] = nv[1] * t[0][2] - nv[2] * t[0][1];
        t[1][1] = nv[2] * t[0][0] - nv[0] * t[0][2];
        t[1][2] = nv[0] * t[0][1] - nv[1] * t[0][0];
    }
}

/* Average state at the half node from nodes i (left) and i+1 (right):
 * Roe average (default; the scheme listing of section 3 selects it) or the
 * arithmetic mean of u and H (flag).  Returns a^2. */
static double half_state(const orc_params *P, int nd, const prim_t *L, const prim_t *R,
                         double *u, double *Hh)
{
    if (P->roe_avg) {
        double sl = sqrt(L->rho), sr = sqrt(R->rho);
        for (int m = 0; m < 3; m++) u[m] = 0.0;
        for (int m = 0; m < nd; m++) u[m] = (sl * L->u[m] + sr * R->u[m]) / (sl + sr);
        *Hh = (sl * L->H + sr * R->H) / (sl + sr);
    } else {
        for (int m = 0; m < 3; m++) u[m] = 0.0;
        for (int m = 0; m < nd; m++) u[m] = 0.5 * (L->u[m] + R->u[m]);
        *Hh = 0.5 * (L->H + R->H);
    }
    double ke = 0.0;
    for (int m = 0; m < nd; m++) ke += u[m] * u[m];
    return (P->gamma - 1.0) * (*Hh - 0.5 * ke);
}

static void eigvecs(const orc_params *P, int nd, int d, const double *u, double Hh, double a,
                    const double *nv, double Lm[NCMAX][NCMAX], double Rm[NCMAX][NCMAX])
{
    int nc = nd + 2;
    double t[2][3];
    tangents(nd, d, nv, t);
    double K = 0.0, un = 0.0;
    for (int m = 0; m < nd; m++) { K += 0.5 * u[m] * u[m]; un += u[m] * nv[m]; }
    double b = (P->gamma - 1.0) / (a * a);
    memset(Lm, 0, sizeof(double) * NCMAX * NCMAX);
    memset(Rm, 0, sizeof(double) * NCMAX * NCMAX);
    int jp = nd + 1;
    /* right eigenvectors (columns) */
    Rm[0][0] = 1.0; Rm[0][1] = 1.0; Rm[0][jp] = 1.0;
    for (int m = 0; m < nd; m++) {
        Rm[1 + m][0] = u[m] - a * nv[m];
        Rm[1 + m][1] = u[m];
        Rm[1 + m][jp] = u[m] + a * nv[m];
    }
    Rm[nd + 1][0] = Hh - a * un;
    Rm[nd + 1][1] = K;
    Rm[nd + 1][jp] = Hh + a * un;
    for (int s = 0; s < nd - 1; s++) {
        double ut = 0.0;
        for (int m = 0; m < nd; m++) { Rm[1 + m][2 + s] = t[s][m]; ut += u[m] * t[s][m]; }
        Rm[nd + 1][2 + s] = ut;
    }
    /* left eigenvectors (rows) */
    Lm[0][0] = 0.5 * (b * K + un / a);
    Lm[1][0] = 1.0 - b * K;
    Lm[jp][0] = 0.5 * (b * K - un / a);
    for (int m = 0; m < nd; m++) {
        Lm[0][1 + m] = -0.5 * (b * u[m] + nv[m] / a);
        Lm[1][1 + m] = b * u[m];
        Lm[jp][1 + m] = -0.5 * (b * u[m] - nv[m] / a);
    }
    Lm[0][nd + 1] = 0.5 * b;
    Lm[1][nd + 1] = -b;
    Lm[jp][nd + 1] = 0.5 * b;
    for (int s = 0; s < nd - 1; s++) {
        double ut = 0.0;
        for (int m = 0; m < nd; m++) { Lm[2 + s][1 + m] = t[s][m]; ut += u[m] * t[s][m]; }
        Lm[2 + s][0] = -ut;
        Lm[2 + s][nd + 1] = 0.0;
    }
    (void)nc;
}

/* ------------------------------------------- WENO-Z5 / TENO5 (per scalar) --
 * Input f[0..4] = f_{i-2..i+2}; returns the reconstruction at x_{i+1/2}.
 * Candidate stencils S_r = {i-r .. i-r+2} (eq. eno_rhs) with the standard
 * third-order coefficients and optimal weights d = (3/10, 3/5, 1/10);
 * Jiang-Shu indicators exactly as eq. fifth_smoothness; tau_5 = |beta_0 -
 * beta_2| (section 2.4 and eq. tau_5).
 *   WENO-Z (eq. wenoz_weights, sigma_r read as beta_r):
 *       alpha_r = d_r (1 + (tau/(beta_r + eps))^2),  omega = alpha / sum alpha
 *   TENO5 (section 2.5): gamma_r = (1 + tau/(beta_r + eps))^6,
 *       chi_r = gamma_r / sum gamma, delta_r = 0 if chi_r < C_T else 1,
 *       omega_r = d_r delta_r / sum d delta.
 * delta (may be NULL) receives the TENO cut-off flags (all 1 for WENO-Z).
 */
static void smoothness5(const double *f, double *beta)
{
    const double fm2 = f[0], fm1 = f[1], f0 = f[2], fp1 = f[3], fp2 = f[4];
    double s, t;
    s = f0 - 2.0 * fp1 + fp2;   t = 3.0 * f0 - 4.0 * fp1 + fp2;
    beta[0] = (13.0 / 12.0) * s * s + 0.25 * t * t;
    s = fm1 - 2.0 * f0 + fp1;   t = fm1 - fp1;
    beta[1] = (13.0 / 12.0) * s * s + 0.25 * t * t;
    s = fm2 - 2.0 * fm1 + f0;   t = fm2 - 4.0 * fm1 + 3.0 * f0;
    beta[2] = (13.0 / 12.0) * s * s + 0.25 * t * t;
}

static double recon5(int scheme, double CT, double eps, const double *f, int *delta)
{
    const double fm2 = f[0], fm1 = f[1], f0 = f[2], fp1 = f[3], fp2 = f[4];
    double q[3], beta[3], w[3];
    q[0] = (1.0 / 3.0) * f0 + (5.0 / 6.0) * fp1 - (1.0 / 6.0) * fp2;
    q[1] = -(1.0 / 6.0) * fm1 + (5.0 / 6.0) * f0 + (1.0 / 3.0) * fp1;
    q[2] = (1.0 / 3.0) * fm2 - (7.0 / 6.0) * fm1 + (11.0 / 6.0) * f0;
    smoothness5(f, beta);
    const double dr[3] = {3.0 / 10.0, 3.0 / 5.0, 1.0 / 10.0};
    double tau = fabs(beta[0] - beta[2]);
    if (scheme == SCHEME_WENOZ5) {
        double a[3], sum = 0.0;
        for (int r = 0; r < 3; r++) {
            double x = tau / (beta[r] + eps);
            a[r] = dr[r] * (1.0 + x * x);
            sum += a[r];
        }
        for (int r = 0; r < 3; r++) w[r] = a[r] / sum;
        if (delta) delta[0] = delta[1] = delta[2] = 1;
    } else {
        double g[3], sum = 0.0;
        for (int r = 0; r < 3; r++) {
            double c = 1.0 + tau / (beta[r] + eps);
            double c3 = c * c * c;
            g[r] = c3 * c3;
            sum += g[r];
        }
        int dl[3];
        double sd = 0.0;
        for (int r = 0; r < 3; r++) {
            double chi = g[r] / sum;
            dl[r] = chi < CT ? 0 : 1;
            sd += dr[r] * dl[r];
        }
        for (int r = 0; r < 3; r++) w[r] = dr[r] * dl[r] / sd;
        if (delta) { delta[0] = dl[0]; delta[1] = dl[1]; delta[2] = dl[2]; }
    }
    return w[0] * q[0] + w[1] * q[1] + w[2] * q[2];
}

/* ------------------------------------------------------ TENO6 (per scalar) --
 * Sixth-order TENO (section 2.5 with K = 6): four candidate stencils, the
 * three three-point ones of the fifth-order scheme, S_0 = {i..i+2},
 * S_1 = {i-1..i+1}, S_2 = {i-2..i}, and the four-point S_3 = {i..i+3}, so the
 * reconstruction at x_{i+1/2} reads f_{i-2..i+3} (f[0..5]).
 * S_3's value is the cell-average reconstruction of its cubic,
 *   (1/4) f_i + (13/12) f_{i+1} - (5/12) f_{i+2} + (1/12) f_{i+3},
 * and its indicator is the Jiang-Shu integral (eq. smoothness_indicator)
 * of that cubic over cell i, which works out to
 *   beta_3 = (1/36)(-11 f_i + 18 f_{i+1} - 9 f_{i+2} + 2 f_{i+3})^2
 *          + (13/12)(2 f_i - 5 f_{i+1} + 4 f_{i+2} - f_{i+3})^2
 *          + (781/720)(-f_i + 3 f_{i+1} - 3 f_{i+2} + f_{i+3})^2.
 * tau_6 = |beta_3 - (beta_0 + beta_2 + 4 beta_1)/6| (eq. tau_5, second
 * line; beta_1 is the central stencil's).  gamma_r = (1 + tau_6/(beta_r +
 * eps))^6 (eq. TENO_weights, C = 1, q = 6), chi_r = gamma_r / sum gamma,
 * delta_r = 0 if chi_r < C_T (eq. cutoff_eqn), omega_r = d_r delta_r /
 * sum d delta.
 * Reading (the optimal weights are not printed): d = (3/10, 9/20, 1/20, 1/5),
 * the unique weights whose combination of the four candidates is the
 * sixth-order reconstruction (1, -8, 37, 37, -8, 1)/60 on i-2..i+3.  Four
 * stencils can never all be cut (max chi >= 1/4 > C_T).
 */
/* the four indicators and tau_6 of f_{i-2..i+3} */
static double smoothness6(const double *f, double *beta)
{
    const double f0 = f[2], fp1 = f[3], fp2 = f[4], fp3 = f[5];
    smoothness5(f, beta);
    const double a = -11.0 * f0 + 18.0 * fp1 - 9.0 * fp2 + 2.0 * fp3;
    const double b = 2.0 * f0 - 5.0 * fp1 + 4.0 * fp2 - fp3;
    const double c = -f0 + 3.0 * fp1 - 3.0 * fp2 + fp3;
    beta[3] = (1.0 / 36.0) * a * a + (13.0 / 12.0) * b * b + (781.0 / 720.0) * c * c;
    return fabs(beta[3] - (beta[0] + beta[2] + 4.0 * beta[1]) / 6.0);
}

static double recon_teno6(double CT, double eps, const double *f, int *delta)
{
    const double fm2 = f[0], fm1 = f[1], f0 = f[2], fp1 = f[3], fp2 = f[4], fp3 = f[5];
    double q[4], beta[4];
    q[0] = (1.0 / 3.0) * f0 + (5.0 / 6.0) * fp1 - (1.0 / 6.0) * fp2;
    q[1] = -(1.0 / 6.0) * fm1 + (5.0 / 6.0) * f0 + (1.0 / 3.0) * fp1;
    q[2] = (1.0 / 3.0) * fm2 - (7.0 / 6.0) * fm1 + (11.0 / 6.0) * f0;
    q[3] = 0.25 * f0 + (13.0 / 12.0) * fp1 - (5.0 / 12.0) * fp2 + (1.0 / 12.0) * fp3;
    const double tau = smoothness6(f, beta);
    const double dr[4] = {3.0 / 10.0, 9.0 / 20.0, 1.0 / 20.0, 1.0 / 5.0};
    double g[4], sum = 0.0;
    for (int r = 0; r < 4; r++) {
        double c = 1.0 + tau / (beta[r] + eps);
        double c3 = c * c * c;
        g[r] = c3 * c3;
        sum += g[r];
    }
    int dl[4];
    double sd = 0.0;
    for (int r = 0; r < 4; r++) {
        double chi = g[r] / sum;
        dl[r] = chi < CT ? 0 : 1;
        sd += dr[r] * dl[r];
    }
    double v = 0.0;
    for (int r = 0; r < 4; r++) v += (dr[r] * dl[r] / sd) * q[r];
    if (delta) for (int r = 0; r < 4; r++) delta[r] = dl[r];
    return v;
}

/* ---------------------------------------------- WENO-JS5 (per scalar) --
 * The original weights (eqs. omega and alpha): alpha_r = d_r / (eps +
 * beta_r)^p with p = 2, omega = alpha / sum alpha; the same candidates,
 * indicators and optimal weights as the fifth-order WENO-Z.  The paper sets
 * eps = 1e-6 for this scheme; eps is the caller's. */
static double recon_wenojs5(double eps, const double *f)
{
    const double fm2 = f[0], fm1 = f[1], f0 = f[2], fp1 = f[3], fp2 = f[4];
    double q[3], beta[3], a[3], sum = 0.0;
    q[0] = (1.0 / 3.0) * f0 + (5.0 / 6.0) * fp1 - (1.0 / 6.0) * fp2;
    q[1] = -(1.0 / 6.0) * fm1 + (5.0 / 6.0) * f0 + (1.0 / 3.0) * fp1;
    q[2] = (1.0 / 3.0) * fm2 - (7.0 / 6.0) * fm1 + (11.0 / 6.0) * f0;
    smoothness5(f, beta);
    const double dr[3] = {3.0 / 10.0, 3.0 / 5.0, 1.0 / 10.0};
    for (int r = 0; r < 3; r++) {
        double e = eps + beta[r];
        a[r] = dr[r] / (e * e);
        sum += a[r];
    }
    return (a[0] / sum) * q[0] + (a[1] / sum) * q[1] + (a[2] / sum) * q[2];
}

/* ---------------------------------------------- WENO-3Z (per scalar) --
 * Third-order WENO-Z (k = 2, section 2.4; the order used in section 5.2):
 * candidates S_0 = {i, i+1}, S_1 = {i-1, i} (eq. eno_rhs with r = 0, 1):
 * q_0 = (f_i + f_{i+1})/2, q_1 = (3 f_i - f_{i-1})/2; indicators of their
 * linear polynomials (eq. smoothness_indicator): beta_0 = (f_{i+1} - f_i)^2,
 * beta_1 = (f_i - f_{i-1})^2; optimal weights (2/3, 1/3), whose combination
 * is the third-order (-1/6, 5/6, 1/3) on i-1..i+1; alpha_r = d_r (1 +
 * (tau/(beta_r + eps))^2) (eq. wenoz_weights).  Reading: tau_3 = |beta_0 -
 * beta_1| (the paper prints only the fifth-order tau).  Reads f[1..3]. */
static double recon_wenoz3(double eps, const double *f)
{
    const double fm1 = f[1], f0 = f[2], fp1 = f[3];
    const double q0 = 0.5 * f0 + 0.5 * fp1, q1 = -0.5 * fm1 + 1.5 * f0;
    const double b0 = (fp1 - f0) * (fp1 - f0), b1 = (f0 - fm1) * (f0 - fm1);
    const double tau = fabs(b0 - b1);
    const double x0 = tau / (b0 + eps), x1 = tau / (b1 + eps);
    const double a0 = (2.0 / 3.0) * (1.0 + x0 * x0), a1 = (1.0 / 3.0) * (1.0 + x1 * x1);
    const double sum = a0 + a1;
    return (a0 / sum) * q0 + (a1 / sum) * q1;
}

/* ---------------------------------------------- WENO-7Z (per scalar) --
 * Seventh-order WENO-Z (k = 4; the highest order of section 5.2), written
 * from the definitions: four candidate stencils S_r = {i-r .. i-r+3} of
 * f_{i-3..i+3} (f[0..6]); on each, the cubic p_r whose averages over the
 * cells [x_j - 1/2, x_j + 1/2] (unit spacing, cell i = [-1/2, 1/2]) are the
 * stencil's values; candidate q_r = p_r(1/2); indicator (eq.
 * smoothness_indicator) beta_r = sum_{l=1..3} integral over cell i of
 * (p_r^(l))^2, the integrals by three-point Gauss-Legendre quadrature (exact
 * for these polynomial degrees); alpha_r = d_r (1 + (tau/(beta_r + eps))^2)
 * (eq. wenoz_weights).  Readings (not printed): the optimal weights
 * d = (4/35, 18/35, 12/35, 1/35) of the cited source (the unique weights
 * whose combination of the candidates is the seven-cell reconstruction), and
 * tau_7 = |beta_0 + 3 beta_1 - 3 beta_2 - beta_3| (Castro et al., the paper
 * prints only the fifth-order tau). */
static double wz7_basis[4][4][4];  /* [r][j][k]: coefficient of x^k of the cubic of unit data at node j of S_r */

/* the cubics of unit data (called before any reconstruction; idempotent) */
static void wz7_init(void)
{
    for (int r = 0; r < 4; r++)
        for (int j = 0; j < 4; j++) {
            /* cell-average conditions: sum_k c_k int_{x_m-1/2}^{x_m+1/2} x^k dx = [m == j] */
            double A[4][5];
            for (int m = 0; m < 4; m++) {
                const double xm = (double)(m - r), lo = xm - 0.5, hi = xm + 0.5;
                double plo = lo, phi = hi;
                for (int k = 0; k < 4; k++) {
                    A[m][k] = (phi - plo) / (k + 1);
                    plo *= lo;
                    phi *= hi;
                }
                A[m][4] = m == j ? 1.0 : 0.0;
            }
            for (int c = 0; c < 4; c++) {  /* Gauss-Jordan with partial pivoting */
                int pv = c;
                for (int m = c + 1; m < 4; m++)
                    if (fabs(A[m][c]) > fabs(A[pv][c])) pv = m;
                for (int k = 0; k < 5; k++) {
                    double t = A[c][k];
                    A[c][k] = A[pv][k];
                    A[pv][k] = t;
                }
                for (int m = 0; m < 4; m++) {
                    if (m == c) continue;
                    const double fac = A[m][c] / A[c][c];
                    for (int k = 0; k < 5; k++) A[m][k] -= fac * A[c][k];
                }
            }
            for (int k = 0; k < 4; k++) wz7_basis[r][j][k] = A[k][4] / A[k][k];
        }
}

/* the four indicators of f_{i-3..i+3}, and the candidates if q != NULL */
static void smoothness7(const double *f, double *beta, double *q)
{
    const double gx[3] = {-0.5 * sqrt(0.6), 0.0, 0.5 * sqrt(0.6)};  /* Gauss-Legendre on [-1/2, 1/2] */
    const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
    for (int r = 0; r < 4; r++) {
        double c[4] = {0.0, 0.0, 0.0, 0.0};
        for (int j = 0; j < 4; j++)
            for (int k = 0; k < 4; k++) c[k] += wz7_basis[r][j][k] * f[3 - r + j];
        double b = 0.0;
        for (int t = 0; t < 3; t++) {
            const double x = gx[t];
            const double d1 = c[1] + 2.0 * c[2] * x + 3.0 * c[3] * x * x;
            const double d2 = 2.0 * c[2] + 6.0 * c[3] * x;
            const double d3 = 6.0 * c[3];
            b += gw[t] * (d1 * d1 + d2 * d2 + d3 * d3);
        }
        beta[r] = b;
        if (q) q[r] = c[0] + 0.5 * c[1] + 0.25 * c[2] + 0.125 * c[3];
    }
}

static double recon_wenoz7(double eps, const double *f)
{
    double q[4], beta[4];
    smoothness7(f, beta, q);
    const double tau = fabs(beta[0] + 3.0 * beta[1] - 3.0 * beta[2] - beta[3]);
    const double dr[4] = {4.0 / 35.0, 18.0 / 35.0, 12.0 / 35.0, 1.0 / 35.0};
    double a[4], sum = 0.0;
    for (int r = 0; r < 4; r++) {
        const double x = tau / (beta[r] + eps);
        a[r] = dr[r] * (1.0 + x * x);
        sum += a[r];
    }
    double v = 0.0;
    for (int r = 0; r < 4; r++) v += (a[r] / sum) * q[r];
    return v;
}

/* Reconstruction of the scheme at x_{i+1/2} from f[0..5] = f_{i-2..i+3}
 * (the fifth-order schemes read f[0..4], WENO-3Z f[1..3]; WENO-7Z reads
 * f[0..6] = f_{i-3..i+3}).  delta (may be NULL) receives four cut-off flags;
 * stencils a scheme does not have, and every stencil of a WENO scheme,
 * read 1. */
static double recon(int scheme, double CT, double eps, const double *f, int *delta)
{
    int dl[4] = {1, 1, 1, 1};
    double v;
    switch (scheme) {
    case SCHEME_TENO6: v = recon_teno6(CT, eps, f, dl); break;
    case SCHEME_WENOJS5: v = recon_wenojs5(eps, f); break;
    case SCHEME_WENOZ3: v = recon_wenoz3(eps, f); break;
    case SCHEME_WENOZ7: v = recon_wenoz7(eps, f); break;
    default: v = recon5(scheme, CT, eps, f, dl); break;
    }
    if (delta) for (int r = 0; r < 4; r++) delta[r] = dl[r];
    return v;
}

/* --------------------------------------------- characteristic LLF flux --
 * One half node x_{i+1/2} in direction d (section 2.2, enumerated algorithm):
 *   n = S/|S| with S the half-node area vector; for k = i-2..i+3:
 *   V_k = L U_k, g_k = L f_k(n); alpha_j = max_k |lambda_j(U_k)| over the six
 *   stencil points (reading of "local stencil points k", pointwise
 *   eigenvalues, the averaged state's own eigenvalue not included);
 *   g^{+-}_k = (g_k +- alpha_j V_k)/2 (eq. lax_scalar per field);
 *   ghat^+ from g^+_{i-2..i+3}, ghat^- from the mirror image
 *   g^-_{i+3..i-2} (the fifth-order schemes use the first five of each,
 *   g^+_{i-2..i+2} and g^-_{i+3..i-1}); F = |S| R (ghat^+ + ghat^-).
 * Uk holds the six stencil states, Uk[k*nc + c].  delta (may be NULL)
 * receives the TENO flags as delta[(j*2 + side)*4 + r], side 0 = plus.
 */
static void iface_flux(const orc_params *P, int d, const double *Uk, const double *S,
                       double *F, int *delta)
{
    const int nd = P->ndim, nc = nd + 2;
    const int W = P->scheme == SCHEME_WENOZ7 ? 8 : 6;  /* stencil points i-W/2+1 .. i+W/2 */
    double Smag = 0.0, nv[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < nd; m++) Smag += S[m] * S[m];
    Smag = sqrt(Smag);
    for (int m = 0; m < nd; m++) nv[m] = S[m] / Smag;

    prim_t w[8];
    double fk[8][NCMAX], lam[8][NCMAX];
    for (int k = 0; k < W; k++) {
        to_prim(P, nd, Uk + k * nc, &w[k]);
        phys_flux(nd, Uk + k * nc, &w[k], nv, fk[k]);
        double un = 0.0;
        for (int m = 0; m < nd; m++) un += w[k].u[m] * nv[m];
        lam[k][0] = un - w[k].a;
        for (int j = 1; j <= nd; j++) lam[k][j] = un;
        lam[k][nd + 1] = un + w[k].a;
    }
    double uh[3], Hh;
    double a2 = half_state(P, nd, &w[W / 2 - 1], &w[W / 2], uh, &Hh);
    double ah = sqrt(a2);
    double Lm[NCMAX][NCMAX], Rm[NCMAX][NCMAX];
    eigvecs(P, nd, d, uh, Hh, ah, nv, Lm, Rm);

    double V[8][NCMAX], G[8][NCMAX];
    for (int k = 0; k < W; k++)
        for (int j = 0; j < nc; j++) {
            double sv = 0.0, sg = 0.0;
            for (int c = 0; c < nc; c++) {
                sv += Lm[j][c] * Uk[k * nc + c];
                sg += Lm[j][c] * fk[k][c];
            }
            V[k][j] = sv;
            G[k][j] = sg;
        }
    double ghat[NCMAX];
    for (int j = 0; j < nc; j++) {
        double alpha = 0.0;
        for (int k = 0; k < W; k++) alpha = fmax(alpha, fabs(lam[k][j]));
        double gp[8], gm[8];
        for (int m = 0; m < W; m++) {
            gp[m] = 0.5 * (G[m][j] + alpha * V[m][j]);                  /* k = i-W/2+1+m */
            gm[m] = 0.5 * (G[W - 1 - m][j] - alpha * V[W - 1 - m][j]);  /* k = i+W/2-m   */
        }
        int *dp = delta ? delta + (j * 2 + 0) * 4 : NULL;
        int *dm = delta ? delta + (j * 2 + 1) * 4 : NULL;
        ghat[j] = recon(P->scheme, P->teno_CT, P->eps, gp, dp)
                + recon(P->scheme, P->teno_CT, P->eps, gm, dm);
    }
    for (int c = 0; c < nc; c++) {
        double s = 0.0;
        for (int j = 0; j < nc; j++) s += Rm[c][j] * ghat[j];
        F[c] = Smag * s;
    }
}

/* --------------------------------------- fourth-order central operators --
 * First derivative per unit index spacing (section 2.6).  Interior:
 * (f_{i-2} - 8 f_{i-1} + 8 f_{i+1} - f_{i+2})/12; the sign of the printed
 * interior formula is taken from the generated OPS kernel of section 4 (the
 * displayed equation has both signs flipped), written difference-first so a
 * constant gives exactly zero.  Non-periodic ends: the one-sided closures at
 * nodes 0, 1, N-2, N-1 exactly as printed.  Periodic: wrap-around.
 * fn(ctx, pos) evaluates the operand at index pos along the line (for
 * periodic lines it is called with pos outside [0, N)).
 */
typedef double (*line_fn)(const void *ctx, int64_t pos);

static double dline(line_fn fn, const void *ctx, int64_t N, int periodic, int64_t p)
{
    if (periodic || (p >= 2 && p <= N - 3)) {
        return (2.0 / 3.0) * (fn(ctx, p + 1) - fn(ctx, p - 1))
             - (1.0 / 12.0) * (fn(ctx, p + 2) - fn(ctx, p - 2));
    }
    if (p == 0)
        return (-25.0 * fn(ctx, 0) + 48.0 * fn(ctx, 1) - 36.0 * fn(ctx, 2)
                + 16.0 * fn(ctx, 3) - 3.0 * fn(ctx, 4)) / 12.0;
    if (p == 1)
        return (-3.0 * fn(ctx, 0) - 10.0 * fn(ctx, 1) + 18.0 * fn(ctx, 2)
                - 6.0 * fn(ctx, 3) + fn(ctx, 4)) / 12.0;
    if (p == N - 2)
        return (-fn(ctx, N - 5) + 6.0 * fn(ctx, N - 4) - 18.0 * fn(ctx, N - 3)
                + 10.0 * fn(ctx, N - 2) + 3.0 * fn(ctx, N - 1)) / 12.0;
    /* p == N - 1 */
    return (3.0 * fn(ctx, N - 5) - 16.0 * fn(ctx, N - 4) + 36.0 * fn(ctx, N - 3)
            - 48.0 * fn(ctx, N - 2) + 25.0 * fn(ctx, N - 1)) / 12.0;
}

/* operand = plain array over interior nodes, periodic lines wrapped */
typedef struct { const grid_t *g; const double *a; int dir; int64_t i, j, k; } arr_line;

static double arr_line_at(const void *vctx, int64_t pos)
{
    const arr_line *c = (const arr_line *)vctx;
    int64_t q[3] = {c->i, c->j, c->k};
    q[c->dir] = wrap(pos, c->g->n[c->dir]);
    return c->a[cidx(c->g, q[0], q[1], q[2])];
}

static int is_periodic(const orc_params *P, int d) { return P->bc[d][0] == BC_PERIODIC; }

/* D_dir of an interior-node array at node (i, j, k) */
static double darr(const orc_params *P, const grid_t *g, const double *a, int dir,
                   int64_t i, int64_t j, int64_t k)
{
    arr_line c = {g, a, dir, i, j, k};
    int64_t q[3] = {i, j, k};
    return dline(arr_line_at, &c, g->n[dir], is_periodic(P, dir), q[dir]);
}

/* --------------------------------------------------------------- metrics --
 * Curvilinear transformation (section 2.6, last paragraph): metrics computed
 * once, with the same central scheme and boundary closures, multiplied into
 * the derivatives.  The discrete form is not printed; the reading taken is
 * the strong-conservation one: area vectors S_d = grad(xi_d)/J,
 *   1D: S = 1, J = 1/x_xi;
 *   2D: S_xi = (y_eta, -x_eta), S_eta = (-y_xi, x_xi),
 *       J = 1/(x_xi y_eta - x_eta y_xi);
 *   3D: S_a = x_b x x_c for (a,b,c) cyclic, each component written in the
 *       conservative Thomas-Lombard form D_c(x_q D_b x_p) - D_b(x_q D_c x_p),
 *       J = 1/det(dx/dxi).
 * Periodic directions: coordinate component d of a node shifted by N_d is
 * shifted by period[d].  Ghost-node metrics: periodic copy, otherwise copied
 * from the boundary node (zero-order extension).
 */
typedef struct {
    const orc_params *P; const grid_t *g; const double *X[3];
    int comp; int dir; int64_t i, j, k;
} coord_line;

/* coordinate component comp at a node whose index along dir may be outside */
static double coord_at(const orc_params *P, const grid_t *g, const double *const *X, int comp,
                       int64_t i, int64_t j, int64_t k)
{
    int64_t q[3] = {i, j, k};
    double shift = 0.0;
    for (int d = 0; d < g->nd; d++) {
        int64_t N = g->n[d];
        if (q[d] < 0 || q[d] >= N) {
            int64_t m = (q[d] >= 0) ? q[d] / N : -((-q[d] + N - 1) / N);
            q[d] -= m * N;
            if (comp == d) shift += (double)m * P->period[d];
        }
    }
    return X[comp][cidx(g, q[0], q[1], q[2])] + shift;
}

static double coord_line_at(const void *vctx, int64_t pos)
{
    const coord_line *c = (const coord_line *)vctx;
    int64_t q[3] = {c->i, c->j, c->k};
    q[c->dir] = pos;
    return coord_at(c->P, c->g, c->X, c->comp, q[0], q[1], q[2]);
}

/* D_dir x_comp at node */
static double dcoord(const orc_params *P, const grid_t *g, const double *const *X, int comp,
                     int dir, int64_t i, int64_t j, int64_t k)
{
    coord_line c = {P, g, {X[0], X[1], X[2]}, comp, dir, i, j, k};
    int64_t q[3] = {i, j, k};
    return dline(coord_line_at, &c, g->n[dir], is_periodic(P, dir), q[dir]);
}

/* operand x_q * Xpb where Xpb (= D_b x_p) is periodic without shift */
typedef struct {
    const orc_params *P; const grid_t *g; const double *X[3]; const double *Xpb;
    int q; int dir; int64_t i, j, k;
} prod_line;

static double prod_line_at(const void *vctx, int64_t pos)
{
    const prod_line *c = (const prod_line *)vctx;
    int64_t qq[3] = {c->i, c->j, c->k};
    qq[c->dir] = pos;
    double xq = coord_at(c->P, c->g, c->X, c->q, qq[0], qq[1], qq[2]);
    int64_t w[3] = {qq[0], qq[1], qq[2]};
    w[c->dir] = wrap(pos, c->g->n[c->dir]);
    return xq * c->Xpb[cidx(c->g, w[0], w[1], w[2])];
}

static void fill_ghost_metrics(const orc_params *P, const grid_t *g, double *A)
{
    /* A on the extended grid; interior filled.  Fill ghosts direction by
     * direction over the full extent of the other directions. */
    for (int d = 0; d < g->nd; d++) {
        int64_t lo[3], hi[3];
        for (int e = 0; e < 3; e++) { lo[e] = -g->h[e]; hi[e] = g->n[e] + g->h[e]; }
        for (int64_t k = lo[2]; k < hi[2]; k++)
            for (int64_t j = lo[1]; j < hi[1]; j++)
                for (int64_t i = lo[0]; i < hi[0]; i++) {
                    int64_t q[3] = {i, j, k};
                    int64_t N = g->n[d];
                    if (q[d] >= 0 && q[d] < N) continue;
                    int64_t src[3] = {i, j, k};
                    if (is_periodic(P, d)) src[d] = wrap(q[d], N);
                    else src[d] = q[d] < 0 ? 0 : N - 1;
                    A[gidx(g, i, j, k)] = A[gidx(g, src[0], src[1], src[2])];
                }
    }
}

/* X[3]: coordinates on interior nodes (compact, x fastest; unused comps may be
 * NULL).  S: 9*npts doubles, J: npts doubles (extended grid). */
int orc_metrics(const orc_params *P, const double *x, const double *y, const double *z,
                double *S, double *J)
{
    grid_t g;
    grid_make(P, &g);
    const int nd = g.nd;
    const double *X[3] = {x, y, z};
    memset(S, 0, sizeof(double) * 9 * g.npts);
    memset(J, 0, sizeof(double) * g.npts);
    double *Xd = (double *)malloc(sizeof(double) * 9 * g.nint); /* Xd[(p*3+b)] = D_b x_p */
    if (!Xd) return -1;
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g.n[2]; k++)
        for (int64_t j = 0; j < g.n[1]; j++)
            for (int64_t i = 0; i < g.n[0]; i++)
                for (int p = 0; p < nd; p++)
                    for (int b = 0; b < nd; b++)
                        Xd[(p * 3 + b) * g.nint + cidx(&g, i, j, k)] = dcoord(P, &g, X, p, b, i, j, k);

    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g.n[2]; k++)
        for (int64_t j = 0; j < g.n[1]; j++)
            for (int64_t i = 0; i < g.n[0]; i++) {
                int64_t c = cidx(&g, i, j, k), e = gidx(&g, i, j, k);
#define XD(p, b) Xd[((p) * 3 + (b)) * g.nint + c]
                if (nd == 1) {
                    S[0 * g.npts + e] = 1.0;
                    J[e] = 1.0 / XD(0, 0);
                } else if (nd == 2) {
                    S[(0 * 3 + 0) * g.npts + e] = XD(1, 1);
                    S[(0 * 3 + 1) * g.npts + e] = -XD(0, 1);
                    S[(1 * 3 + 0) * g.npts + e] = -XD(1, 0);
                    S[(1 * 3 + 1) * g.npts + e] = XD(0, 0);
                    J[e] = 1.0 / (XD(0, 0) * XD(1, 1) - XD(0, 1) * XD(1, 0));
                } else {
                    for (int a = 0; a < 3; a++) {
                        int b = (a + 1) % 3, cc = (a + 2) % 3;
                        for (int m = 0; m < 3; m++) {
                            int p = (m + 1) % 3, q = (m + 2) % 3;
                            /* D_c(x_q D_b x_p) - D_b(x_q D_c x_p) */
                            prod_line c1 = {P, &g, {x, y, z}, Xd + (p * 3 + b) * g.nint, q, cc, i, j, k};
                            prod_line c2 = {P, &g, {x, y, z}, Xd + (p * 3 + cc) * g.nint, q, b, i, j, k};
                            int64_t qq[3] = {i, j, k};
                            double t1 = dline(prod_line_at, &c1, g.n[cc], is_periodic(P, cc), qq[cc]);
                            double t2 = dline(prod_line_at, &c2, g.n[b], is_periodic(P, b), qq[b]);
                            S[(a * 3 + m) * g.npts + e] = t1 - t2;
                        }
                    }
                    double det = XD(0, 0) * (XD(1, 1) * XD(2, 2) - XD(1, 2) * XD(2, 1))
                               - XD(0, 1) * (XD(1, 0) * XD(2, 2) - XD(1, 2) * XD(2, 0))
                               + XD(0, 2) * (XD(1, 0) * XD(2, 1) - XD(1, 1) * XD(2, 0));
                    J[e] = 1.0 / det;
                }
#undef XD
            }
    free(Xd);
    for (int q = 0; q < 9; q++) fill_ghost_metrics(P, &g, S + q * g.npts);
    fill_ghost_metrics(P, &g, J);
    return 0;
}

/* Half-node area vector of direction d between nodes p and p+1:
 * S_{i+1/2} = (-S_{i-1} + 7 S_i + 7 S_{i+1} - S_{i+2})/12 (reading: the
 * four-point interpolation whose difference is the interior operator D, so
 * the discrete geometric conservation law holds). */
static void half_area(const grid_t *g, const double *S, int d, int64_t e, double *Sh)
{
    int64_t st = g->s[d];
    for (int m = 0; m < 3; m++) {
        const double *A = S + (d * 3 + m) * g->npts;
        Sh[m] = (-A[e - st] + 7.0 * A[e] + 7.0 * A[e + st] - A[e + 2 * st]) / 12.0;
    }
}

/* ----------------------------------------------------- boundary conditions --
 * Section 3.1 (boundary and initial conditions): BCs per (direction, side),
 * enforced through three ghost nodes.
 *   periodic: copy; extrapolation (reading: zero-gradient copy of the
 *   boundary node); Dirichlet (the Shu-Osher case of section 5.2): the
 *   ghost values are the boundary data, set with the initial state and
 *   left unchanged;
 *   isothermal wall (eq. wall_energy, eq. halo_density and the momentum
 *   reflection): wall node momentum = 0, rho E_w = rho_w T_w/(M^2 gamma
 *   (gamma-1)) with rho_w floating; p_w = rho_w T_w/(gamma M^2) (reading);
 *   ghost T_{-i} = (i+1) T_w - i T_1; rho_{-i} = gamma M^2 p_w / T_{-i}
 *   (the printed rho_{-1} read as rho_{-i}); rho u_{-i} = -rho_{-i} u_i;
 *   rho E_{-i} = p_w/(gamma-1) + rho_{-i}|u_i|^2/2 (reading: zero normal
 *   pressure gradient).
 *   adiabatic wall: T_w from the fourth-order one-sided dT/dn = 0 closure,
 *   T_w = (48 T_1 - 36 T_2 + 16 T_3 - 3 T_4)/25, then as isothermal.
 * Phase 1 sets the wall-node values of every wall face; phase 2 fills
 * ghosts direction by direction over the full extent of the other
 * directions (corner ghosts are never read by the stencils).
 */
static void node_T(const orc_params *P, int nd, const double *U, int64_t e, int64_t npts,
                   double *T, double *u)
{
    double Uc[NCMAX];
    for (int c = 0; c < nd + 2; c++) Uc[c] = U[c * npts + e];
    prim_t w;
    to_prim(P, nd, Uc, &w);
    *T = w.T;
    if (u) for (int m = 0; m < 3; m++) u[m] = w.u[m];
}

void orc_apply_bc(const orc_params *P, double *U)
{
    grid_t g;
    grid_make(P, &g);
    const int nd = g.nd, nc = g.nc;
    const double gm = P->gamma, M2 = P->Minf * P->Minf;
    /* phase 1: wall nodes */
    for (int d = 0; d < nd; d++)
        for (int side = 0; side < 2; side++) {
            int kind = P->bc[d][side];
            if (kind != BC_ISOTHERMAL && kind != BC_ADIABATIC) continue;
            int64_t N = g.n[d];
            int64_t lo[3], hi[3];
            for (int e = 0; e < 3; e++) { lo[e] = 0; hi[e] = g.n[e]; }
            lo[d] = side ? N - 1 : 0; hi[d] = lo[d] + 1;
            int sgn = side ? -1 : 1;
            for (int64_t k = lo[2]; k < hi[2]; k++)
                for (int64_t j = lo[1]; j < hi[1]; j++)
                    for (int64_t i = lo[0]; i < hi[0]; i++) {
                        int64_t ew = gidx(&g, i, j, k);
                        double Tw;
                        if (kind == BC_ISOTHERMAL) {
                            Tw = P->wall_T[d][side];
                        } else {
                            double Tm[5];
                            for (int m = 1; m <= 4; m++) {
                                node_T(P, nd, U, ew + sgn * m * g.s[d], g.npts, &Tm[m], NULL);
                            }
                            Tw = (48.0 * Tm[1] - 36.0 * Tm[2] + 16.0 * Tm[3] - 3.0 * Tm[4]) / 25.0;
                        }
                        double rw = U[ew];
                        for (int m = 0; m < nd; m++) U[(1 + m) * g.npts + ew] = 0.0;
                        U[(nd + 1) * g.npts + ew] = rw * Tw / (M2 * gm * (gm - 1.0));
                    }
        }
    /* phase 2: ghosts */
    for (int d = 0; d < nd; d++) {
        int64_t N = g.n[d];
        for (int side = 0; side < 2; side++) {
            int kind = P->bc[d][side];
            int64_t lo[3], hi[3];
            for (int e = 0; e < 3; e++) { lo[e] = -g.h[e]; hi[e] = g.n[e] + g.h[e]; }
            lo[d] = 0; hi[d] = 1;  /* iterate the face; ghost index set below */
            int sgn = side ? -1 : 1;
            for (int64_t k = lo[2]; k < hi[2]; k++)
                for (int64_t j = lo[1]; j < hi[1]; j++)
                    for (int64_t i = lo[0]; i < hi[0]; i++) {
                        int64_t q[3] = {i, j, k};
                        q[d] = side ? N - 1 : 0;
                        int64_t ew = gidx(&g, q[0], q[1], q[2]);   /* boundary node */
                        for (int m = 1; m <= NGHOST; m++) {
                            int64_t eg = ew - sgn * m * g.s[d];      /* ghost m */
                            if (kind == BC_PERIODIC) {
                                int64_t es = ew - sgn * m * g.s[d] + sgn * N * g.s[d];
                                for (int c = 0; c < nc; c++) U[c * g.npts + eg] = U[c * g.npts + es];
                            } else if (kind == BC_EXTRAPOLATE) {
                                for (int c = 0; c < nc; c++) U[c * g.npts + eg] = U[c * g.npts + ew];
                            } else if (kind == BC_DIRICHLET) {
                                /* boundary data: the ghost values the state
                                 * was given, never overwritten */
                            } else {
                                double Tw, T1, ui[3], Ti;
                                node_T(P, nd, U, ew, g.npts, &Tw, NULL);
                                node_T(P, nd, U, ew + sgn * g.s[d], g.npts, &T1, NULL);
                                node_T(P, nd, U, ew + sgn * m * g.s[d], g.npts, &Ti, ui);
                                (void)Ti;
                                double rw = U[ew];
                                double pw = rw * Tw / (gm * M2);
                                double Tg = (m + 1) * Tw - m * T1;
                                double rg = gm * M2 * pw / Tg;
                                double ke = 0.0;
                                U[eg] = rg;
                                for (int c = 0; c < nd; c++) {
                                    U[(1 + c) * g.npts + eg] = -rg * ui[c];
                                    ke += ui[c] * ui[c];
                                }
                                U[(nd + 1) * g.npts + eg] = pw / (gm - 1.0) + 0.5 * rg * ke;
                            }
                        }
                    }
        }
    }
}

/* ------------------------------------------------------- viscous terms --
 * Heat flux (eq. heat_flux), stress tensor (eq. stress_tensor), Sutherland's
 * law (eq. sutherland).  Discrete form (reading: divergence form):
 *   gradients at nodes  d phi/dx_j = J sum_k (S_k)_j D_k phi,
 *   Fv_j = (0, tau_1j .. tau_nj, u_i tau_ij - q_j),
 *   G_k = sum_j (S_k)_j Fv_j at nodes,
 *   R_visc = J sum_k D_k G_k,
 * with D the central operator above (closures at non-periodic ends, wrap on
 * periodic ones); ghost nodes are never used.
 */
static double viscosity(const orc_params *P, double T)
{
    if (!P->sutherland) return 1.0;
    double Ts = P->Ts_over_Tref;
    return pow(T, 1.5) * (1.0 + Ts) / (T + Ts);
}

static void viscous_residual(const orc_params *P, const grid_t *g, const double *S,
                             const double *J, const double *U, double *R)
{
    const int nd = g->nd, nv = nd + 1;  /* velocity comps + T */
    const int64_t ni = g->nint;
    double *phi = (double *)malloc(sizeof(double) * nv * ni);
    double *Gv = (double *)malloc(sizeof(double) * nd * nv * ni);
    if (!phi || !Gv) { free(phi); free(Gv); return; }
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                double T, u[3];
                node_T(P, nd, U, gidx(g, i, j, k), g->npts, &T, u);
                int64_t c = cidx(g, i, j, k);
                for (int m = 0; m < nd; m++) phi[m * ni + c] = u[m];
                phi[nd * ni + c] = T;
            }
    const double Re = P->Re, Pr = P->Pr, gm = P->gamma, M2 = P->Minf * P->Minf;
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                int64_t c = cidx(g, i, j, k), e = gidx(g, i, j, k);
                double Dk[4][3], grad[4][3];
                for (int v = 0; v < nv; v++)
                    for (int kk = 0; kk < nd; kk++)
                        Dk[v][kk] = darr(P, g, phi + v * ni, kk, i, j, k);
                for (int v = 0; v < nv; v++)
                    for (int jj = 0; jj < nd; jj++) {
                        double s = 0.0;
                        for (int kk = 0; kk < nd; kk++) s += S[(kk * 3 + jj) * g->npts + e] * Dk[v][kk];
                        grad[v][jj] = J[e] * s;
                    }
                double T = phi[nd * ni + c];
                double mu = viscosity(P, T);
                double divu = 0.0;
                for (int m = 0; m < nd; m++) divu += grad[m][m];
                double tau[3][3], q[3], Fv[3][4];
                for (int a = 0; a < nd; a++)
                    for (int b = 0; b < nd; b++)
                        tau[a][b] = mu / Re * (grad[a][b] + grad[b][a] - (a == b ? 2.0 / 3.0 * divu : 0.0));
                for (int b = 0; b < nd; b++)
                    q[b] = -mu / ((gm - 1.0) * M2 * Pr * Re) * grad[nd][b];
                for (int b = 0; b < nd; b++) {
                    double work = 0.0;
                    for (int a = 0; a < nd; a++) { Fv[b][a] = tau[a][b]; work += phi[a * ni + c] * tau[a][b]; }
                    Fv[b][nd] = work - q[b];
                }
                for (int kk = 0; kk < nd; kk++)
                    for (int v = 0; v < nv; v++) {
                        double s = 0.0;
                        for (int b = 0; b < nd; b++) s += S[(kk * 3 + b) * g->npts + e] * Fv[b][v];
                        Gv[(kk * nv + v) * ni + c] = s;
                    }
            }
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                int64_t c = cidx(g, i, j, k), e = gidx(g, i, j, k);
                for (int v = 0; v < nv; v++) {
                    double s = 0.0;
                    for (int kk = 0; kk < nd; kk++) s += darr(P, g, Gv + (kk * nv + v) * ni, kk, i, j, k);
                    R[(1 + v) * ni + c] += J[e] * s;
                }
            }
    free(phi);
    free(Gv);
}

/* ---------------------------------------------- fourth-order central path --
 * Section 2.6: central differences for the convective terms of smooth
 * problems and for the viscous terms, the scheme of the paper's central TGV
 * benchmark (section 6.1).  Second-derivative operator per unit index
 *   f''_i = (-f_{i-2} + 16 f_{i-1} - 30 f_i + 16 f_{i+1} - f_{i+2}) / 12
 * (written difference-first, so a constant gives exactly 0) with the printed
 * one-sided closures at nodes 0 and 1, mirrored at N-1 and N-2 (a second
 * derivative does not change sign under x -> -x); periodic: wrap-around.
 * Readings (the generated code is not printed):
 *  - convection in conservative form, R_c -= sum_d D_d(F_d,c) / h_d, with
 *    F_d the physical flux along e_d at the nodes, on separable meshes of
 *    uniform spacing h_d per direction (the benchmark's), 1/h_d = J S_dd;
 *  - viscous and heat-flux terms in the expanded form that differentiating
 *    the printed equations term by term gives: with g_ij = d_j u_i,
 *    mu~ = mu(T)/Re and kappa = mu~ / ((gamma-1) M^2 Pr),
 *      d_j tau_ij = sum_j d_j mu~ (g_ij + g_ji) - (2/3) d_i mu~ div
 *                 + mu~ [sum_j d_jj u_i + sum_j d_j(g_ji) - (2/3) sum_k d_i(g_kk)],
 *      d_j (u_i tau_ij - q_j) = sum_ij g_ij tau_ij + sum_i u_i d_j tau_ij
 *                 + sum_j (d_j kappa d_j T + kappa d_jj T);
 *    a pure second derivative d_jj (and d_j(g_jj)) takes the second-
 *    derivative operator, a mixed one d_j(g_ji), i != j, the first
 *    derivative of the first derivative (outer index as written); d_j mu~
 *    and d_j kappa are first derivatives of their node values.
 */
static double d2line(line_fn fn, const void *ctx, int64_t N, int periodic, int64_t p)
{
    if (periodic || (p >= 2 && p <= N - 3)) {
        const double c = fn(ctx, p);
        return ((4.0 / 3.0) * ((fn(ctx, p + 1) - c) + (fn(ctx, p - 1) - c))
                - (1.0 / 12.0) * ((fn(ctx, p + 2) - c) + (fn(ctx, p - 2) - c)));
    }
    /* the closures' coefficients sum to zero: written on differences from
     * the boundary node, so a constant gives exactly 0 */
    const int m = p <= 1 ? 1 : -1;           /* direction into the domain */
    const int64_t b = p <= 1 ? 0 : N - 1;    /* boundary node */
    const double f0 = fn(ctx, b);
    const double d1 = fn(ctx, b + m) - f0, d2 = fn(ctx, b + 2 * m) - f0;
    const double d3 = fn(ctx, b + 3 * m) - f0, d4 = fn(ctx, b + 4 * m) - f0;
    if (p == 0 || p == N - 1)
        return (-104.0 * d1 + 114.0 * d2 - 56.0 * d3 + 11.0 * d4) / 12.0;
    /* p == 1 or p == N - 2 */
    return (-20.0 * d1 + 6.0 * d2 + 4.0 * d3 - d4) / 12.0;
}

static double d2arr(const orc_params *P, const grid_t *g, const double *a, int dir,
                    int64_t i, int64_t j, int64_t k)
{
    arr_line c = {g, a, dir, i, j, k};
    int64_t q[3] = {i, j, k};
    return d2line(arr_line_at, &c, g->n[dir], is_periodic(P, dir), q[dir]);
}

static void central_residual(const orc_params *P, const grid_t *g, const double *S,
                             const double *J, const double *U, double *R)
{
    const int nd = g->nd, nc = g->nc;
    const int64_t ni = g->nint;
    double ih[3] = {0.0, 0.0, 0.0};
    {
        const int64_t e0 = gidx(g, 0, 0, 0);
        for (int d = 0; d < nd; d++) ih[d] = J[e0] * S[(d * 3 + d) * g->npts + e0];
    }
    /* convective fluxes F_d at the interior nodes, then their derivatives */
    double *F = (double *)malloc(sizeof(double) * nd * nc * ni);
    if (!F) return;
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                const int64_t e = gidx(g, i, j, k), c = cidx(g, i, j, k);
                double Uc[NCMAX], f[NCMAX];
                for (int q = 0; q < nc; q++) Uc[q] = U[q * g->npts + e];
                prim_t w;
                to_prim(P, nd, Uc, &w);
                for (int d = 0; d < nd; d++) {
                    double nv[3] = {0.0, 0.0, 0.0};
                    nv[d] = 1.0;
                    phys_flux(nd, Uc, &w, nv, f);
                    for (int q = 0; q < nc; q++) F[(d * nc + q) * ni + c] = f[q];
                }
            }
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                const int64_t c = cidx(g, i, j, k);
                for (int q = 0; q < nc; q++) {
                    double s = 0.0;
                    for (int d = 0; d < nd; d++) s += ih[d] * darr(P, g, F + (d * nc + q) * ni, d, i, j, k);
                    R[q * ni + c] -= s;
                }
            }
    free(F);
    if (!(P->Re > 0.0)) return;

    /* node values: u_m (nd), T, mu~, kappa; then the first derivatives g */
    const int nv = nd + 1;
    const double gm = P->gamma, M2 = P->Minf * P->Minf;
    double *phi = (double *)malloc(sizeof(double) * (nv + 2) * ni);
    double *gr = (double *)malloc(sizeof(double) * nv * nd * ni);
    if (!phi || !gr) { free(phi); free(gr); return; }
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                double T, u[3];
                node_T(P, nd, U, gidx(g, i, j, k), g->npts, &T, u);
                const int64_t c = cidx(g, i, j, k);
                const double mut = viscosity(P, T) / P->Re;
                for (int m = 0; m < nd; m++) phi[m * ni + c] = u[m];
                phi[nd * ni + c] = T;
                phi[(nd + 1) * ni + c] = mut;
                phi[(nd + 2) * ni + c] = mut / ((gm - 1.0) * M2 * P->Pr);
            }
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                const int64_t c = cidx(g, i, j, k);
                for (int v = 0; v < nv; v++)
                    for (int jj = 0; jj < nd; jj++)
                        gr[(v * nd + jj) * ni + c] = ih[jj] * darr(P, g, phi + v * ni, jj, i, j, k);
            }
    #pragma omp parallel for collapse(2)
    for (int64_t k = 0; k < g->n[2]; k++)
        for (int64_t j = 0; j < g->n[1]; j++)
            for (int64_t i = 0; i < g->n[0]; i++) {
                const int64_t c = cidx(g, i, j, k);
                double G[4][3], dmu[3], dka[3];
                for (int v = 0; v < nv; v++)
                    for (int jj = 0; jj < nd; jj++) G[v][jj] = gr[(v * nd + jj) * ni + c];
                for (int jj = 0; jj < nd; jj++) {
                    dmu[jj] = ih[jj] * darr(P, g, phi + (nd + 1) * ni, jj, i, j, k);
                    dka[jj] = ih[jj] * darr(P, g, phi + (nd + 2) * ni, jj, i, j, k);
                }
                const double mut = phi[(nd + 1) * ni + c], kap = phi[(nd + 2) * ni + c];
                double div = 0.0;
                for (int m = 0; m < nd; m++) div += G[m][m];
                double dtau[3], work = 0.0;
                for (int a = 0; a < nd; a++) {
                    double first = -(2.0 / 3.0) * dmu[a] * div, second = 0.0;
                    for (int b = 0; b < nd; b++) {
                        first += dmu[b] * (G[a][b] + G[b][a]);
                        /* d_bb u_a */
                        second += ih[b] * ih[b] * d2arr(P, g, phi + a * ni, b, i, j, k);
                        /* d_b (g_ba) */
                        if (a == b) second += ih[b] * ih[b] * d2arr(P, g, phi + b * ni, b, i, j, k);
                        else second += ih[b] * darr(P, g, gr + (b * nd + a) * ni, b, i, j, k);
                        /* -(2/3) d_a (g_bb) */
                        if (a == b) second -= (2.0 / 3.0) * ih[a] * ih[a] * d2arr(P, g, phi + b * ni, a, i, j, k);
                        else second -= (2.0 / 3.0) * ih[a] * darr(P, g, gr + (b * nd + b) * ni, a, i, j, k);
                    }
                    dtau[a] = first + mut * second;
                }
                for (int a = 0; a < nd; a++) {
                    for (int b = 0; b < nd; b++) {
                        const double tau = mut * (G[a][b] + G[b][a] - (a == b ? (2.0 / 3.0) * div : 0.0));
                        work += G[a][b] * tau;
                    }
                    work += phi[a * ni + c] * dtau[a];
                    R[(1 + a) * ni + c] += dtau[a];
                }
                double heat = 0.0;
                for (int b = 0; b < nd; b++)
                    heat += dka[b] * G[nd][b] + kap * ih[b] * ih[b] * d2arr(P, g, phi + nd * ni, b, i, j, k);
                R[(nd + 1) * ni + c] += work + heat;
            }
    free(phi);
    free(gr);
}

/* ------------------------------------------------------------ residual --
 * R = dU/dt on interior nodes: convective part -J sum_d (F_{i+1/2} -
 * F_{i-1/2}) (eq. FD_reconstruct in computational space, all directions,
 * enumerated algorithm step 4), plus the viscous part when Re > 0, plus the
 * test-only body force.
 */
int orc_residual(const orc_params *P, const double *S, const double *J, const double *U, double *R)
{
    grid_t g;
    grid_make(P, &g);
    const int nd = g.nd, nc = g.nc;
    const int64_t ni = g.nint;
    memset(R, 0, sizeof(double) * nc * ni);
    if (P->scheme == SCHEME_CENTRAL4) {
        central_residual(P, &g, S, J, U, R);
        goto body_force;
    }
    const int W = P->scheme == SCHEME_WENOZ7 ? 8 : 6;
    if (P->scheme == SCHEME_WENOZ7) wz7_init();
    for (int d = 0; d < nd; d++) {
        int64_t N = g.n[d];
        int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
        int64_t n1 = g.n[o1], n2 = g.n[o2];
        #pragma omp parallel for collapse(2)
        for (int64_t b = 0; b < n2; b++)
            for (int64_t a = 0; a < n1; a++) {
                double *Fl = (double *)malloc(sizeof(double) * nc * (N + 1));
                for (int64_t p = -1; p < N; p++) {
                    int64_t q[3];
                    q[d] = p; q[o1] = a; q[o2] = b;
                    int64_t e = gidx(&g, q[0], q[1], q[2]);
                    double Uk[8 * NCMAX], Sh[3];
                    for (int k = 0; k < W; k++) {
                        int64_t pos = p + k - (W / 2 - 1);
                        /* WENO-7Z reads one node past the three ghost layers at the
                           outermost interfaces: the wrapped interior on periodic
                           lines, else the third ghost layer again */
                        if (pos < -NGHOST) pos = is_periodic(P, d) ? N + pos : -NGHOST;
                        if (pos > N - 1 + NGHOST) pos = is_periodic(P, d) ? pos - N : N - 1 + NGHOST;
                        for (int c = 0; c < nc; c++) Uk[k * nc + c] = U[c * g.npts + e + (pos - p) * g.s[d]];
                    }
                    half_area(&g, S, d, e, Sh);
                    iface_flux(P, d, Uk, Sh, Fl + (p + 1) * nc, NULL);
                }
                for (int64_t p = 0; p < N; p++) {
                    int64_t q[3];
                    q[d] = p; q[o1] = a; q[o2] = b;
                    int64_t e = gidx(&g, q[0], q[1], q[2]);
                    int64_t ci = cidx(&g, q[0], q[1], q[2]);
                    for (int c = 0; c < nc; c++)
                        R[c * ni + ci] -= J[e] * (Fl[(p + 1) * nc + c] - Fl[p * nc + c]);
                }
                free(Fl);
            }
    }
    if (P->Re > 0.0) viscous_residual(P, &g, S, J, U, R);
body_force:
    if (P->body_force != 0.0) {
        for (int64_t k = 0; k < g.n[2]; k++)
            for (int64_t j = 0; j < g.n[1]; j++)
                for (int64_t i = 0; i < g.n[0]; i++) {
                    double T, u[3];
                    node_T(P, nd, U, gidx(&g, i, j, k), g.npts, &T, u);
                    int64_t ci = cidx(&g, i, j, k);
                    R[1 * ni + ci] += P->body_force;
                    R[(nd + 1) * ni + ci] += P->body_force * u[0];
                }
    }
    return 0;
}

/* --------------------------------------------------------- time stepping --
 * Low-storage Runge-Kutta in Williamson's 2N form (section 2.7):
 *   dU^(s) = A_s dU^(s-1) + dt R(U^(s-1)),  U^(s) = U^(s-1) + B_s dU^(s),
 * A_1 = 0 (stage 0 does not read dU).  The coefficients are not printed;
 * they are cited to Carpenter & Kennedy (third and fourth order) and to
 * Gottlieb (the strong-stability-preserving third-order version).  Readings:
 *   RK3_WILLIAMSON: the three-stage third-order 2N scheme
 *       A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15);
 *   RK4_CK: Carpenter & Kennedy's five-stage fourth-order 2N scheme (their
 *       published rational coefficients, below);
 *   RK3_SSP: the three-stage third-order 2N scheme of Gottlieb & Shu with
 *       c_2 = B_1 = 0.924574 (the member of the one-parameter 2N family that
 *       they found to be strong-stability preserving); the other four
 *       coefficients follow from c_2 by the third-order conditions and the
 *       2N structure (ssp_rk3 below).
 */
static const double RK3W_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK3W_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
static const double RK4CK_A[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                                  -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
static const double RK4CK_B[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                                  1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                                  2277821191437.0 / 14882151754819.0};

/* The 2N third-order family given c_2.  With k_s = dt R(U^(s-1)), the 2N
 * update is the explicit RK scheme with a_21 = B_1, a_31 = B_1 + B_2 A_2,
 * a_32 = B_2, b_1 = a_31 + B_3 A_3 A_2, b_2 = B_2 + B_3 A_3, b_3 = B_3.
 * Third order fixes, for nodes c_2 and c_3 = a_31 + a_32,
 *   b_3 = (1/3 - c_2/2) / (c_3 (c_3 - c_2)),  b_2 = (1/3 - c_3/2) / (c_2 (c_2 - c_3)),
 *   a_32 = 1 / (6 b_3 c_2),  b_1 = 1 - b_2 - b_3,
 * and the 2N structure then gives B_2 = a_32, A_2 = (c_3 - a_32 - c_2)/a_32,
 * B_3 = b_3, A_3 = (b_2 - B_2)/B_3, and leaves one condition on c_3:
 *   resid(c_3) = b_1 - (c_2 + B_2 A_2 + B_3 A_3 A_2) = 0. */
static double ssp_resid(double c2, double c3, double *A, double *B)
{
    const double b3 = (1.0 / 3.0 - c2 / 2.0) / (c3 * (c3 - c2));
    const double b2 = (1.0 / 3.0 - c3 / 2.0) / (c2 * (c2 - c3));
    const double a32 = 1.0 / (6.0 * b3 * c2);
    const double b1 = 1.0 - b2 - b3;
    A[0] = 0.0;
    B[0] = c2;
    B[1] = a32;
    A[1] = (c3 - a32 - c2) / a32;
    B[2] = b3;
    A[2] = (b2 - B[1]) / B[2];
    return b1 - (B[0] + B[1] * A[1] + B[2] * A[2] * A[1]);
}

/* c_3 by bisection on [0.2, 0.6], where resid changes sign once for
 * c_2 = 0.924574 (c_3 = 0.37346...); 200 halvings reach the double
 * closest to the root. */
static void ssp_rk3(double *A, double *B)
{
    const double c2 = 0.924574;
    double lo = 0.2, hi = 0.6;
    double flo = ssp_resid(c2, lo, A, B);
    for (int it = 0; it < 200; it++) {
        const double mid = 0.5 * (lo + hi);
        const double fm = ssp_resid(c2, mid, A, B);
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
    }
    ssp_resid(c2, 0.5 * (lo + hi), A, B);
}

static int rk_stages(const orc_params *P) { return P->rk == RK4_CK ? 5 : 3; }

static void rk_coeffs(const orc_params *P, double *A, double *B)
{
    if (P->rk == RK4_CK) {
        for (int s = 0; s < 5; s++) { A[s] = RK4CK_A[s]; B[s] = RK4CK_B[s]; }
    } else if (P->rk == RK3_SSP) {
        ssp_rk3(A, B);
    } else {
        for (int s = 0; s < 3; s++) { A[s] = RK3W_A[s]; B[s] = RK3W_B[s]; }
    }
}

void orc_rk_coeffs(const orc_params *P, double *A, double *B, int *nstages)
{
    rk_coeffs(P, A, B);
    *nstages = rk_stages(P);
}

int orc_rk_update(const orc_params *P, int stage, double dt, const double *R, double *U, double *dU)
{
    grid_t g;
    grid_make(P, &g);
    const int64_t ni = g.nint;
    double RK_A[5], RK_B[5];
    rk_coeffs(P, RK_A, RK_B);
    for (int c = 0; c < g.nc; c++)
        for (int64_t k = 0; k < g.n[2]; k++)
            for (int64_t j = 0; j < g.n[1]; j++)
                for (int64_t i = 0; i < g.n[0]; i++) {
                    int64_t ci = c * ni + cidx(&g, i, j, k);
                    int64_t e = c * g.npts + gidx(&g, i, j, k);
                    double du = (stage == 0 ? 0.0 : RK_A[stage] * dU[ci]) + dt * R[ci];
                    dU[ci] = du;
                    U[e] = U[e] + RK_B[stage] * du;
                }
    return 0;
}

int orc_rk_substep(const orc_params *P, const double *S, const double *J, int stage, double dt,
                   double *U, double *dU)
{
    grid_t g;
    grid_make(P, &g);
    double *R = (double *)malloc(sizeof(double) * g.nc * g.nint);
    if (!R) return -1;
    orc_residual(P, S, J, U, R);
    orc_rk_update(P, stage, dt, R, U, dU);
    free(R);
    return 0;
}

/* Time step (the paper advances with a constant dt; reading for a CFL
 * number): dt = CFL / max over interior nodes of
 *   sum_d J|S_d| (|u.n_d| + a) + 2 nu_eff sum_d (J|S_d|)^2,
 * nu_eff = max(4/3, gamma/Pr) mu / (rho Re) when viscous, else 0. */
double orc_compute_dt(const orc_params *P, const double *S, const double *J, const double *U, double cfl)
{
    grid_t g;
    grid_make(P, &g);
    const int nd = g.nd;
    double smax = 0.0;
    for (int64_t k = 0; k < g.n[2]; k++)
        for (int64_t j = 0; j < g.n[1]; j++)
            for (int64_t i = 0; i < g.n[0]; i++) {
                int64_t e = gidx(&g, i, j, k);
                double Uc[NCMAX];
                for (int c = 0; c < g.nc; c++) Uc[c] = U[c * g.npts + e];
                prim_t w;
                to_prim(P, nd, Uc, &w);
                double nu = 0.0;
                if (P->Re > 0.0) {
                    double f = fmax(4.0 / 3.0, P->gamma / P->Pr);
                    nu = f * viscosity(P, w.T) / (w.rho * P->Re);
                }
                double conv = 0.0, diff = 0.0;
                for (int d = 0; d < nd; d++) {
                    double s2 = 0.0, us = 0.0;
                    for (int m = 0; m < nd; m++) {
                        double sm = S[(d * 3 + m) * g.npts + e];
                        s2 += sm * sm;
                        us += w.u[m] * sm;
                    }
                    double smag = sqrt(s2);
                    double js = J[e] * smag;
                    conv += js * (fabs(us / smag) + w.a);
                    diff += js * js;
                }
                double s = conv + 2.0 * nu * diff;
                if (s > smax) smax = s;
            }
    return cfl / smax;
}

/* Whole run: BCs at t = 0, then per step dt (fixed, or from CFL, clipped to
 * t_end), the scheme's substeps (three or five) each followed by the BCs. */
int orc_run(const orc_params *P, const double *S, const double *J, double *U, double *dU,
            int64_t nsteps, double cfl, double dt_fixed, double t_end, double *t_out)
{
    double t = t_out ? *t_out : 0.0;
    orc_apply_bc(P, U);
    for (int64_t it = 0; it < nsteps; it++) {
        if (t_end > 0.0 && t >= t_end) break;
        double dt = dt_fixed > 0.0 ? dt_fixed : orc_compute_dt(P, S, J, U, cfl);
        if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
        for (int s = 0; s < rk_stages(P); s++) {
            orc_rk_substep(P, S, J, s, dt, U, dU);
            orc_apply_bc(P, U);
        }
        t += dt;
    }
    if (t_out) *t_out = t;
    return 0;
}

/* ------------------------------------------------ exported unit pieces -- */

void orc_smoothness5(const double *f, double *beta) { smoothness5(f, beta); }

double orc_recon(int scheme, double CT, double eps, const double *f, int *delta)
{
    return recon(scheme, CT, eps, f, delta);
}

double orc_smoothness6(const double *f, double *beta) { return smoothness6(f, beta); }

/* WENO-7Z at x_{i+1/2} from f_{i-3..i+3}; its indicators and candidates */
double orc_recon_wenoz7(double eps, const double *f)
{
    wz7_init();
    return recon_wenoz7(eps, f);
}

void orc_smoothness7(const double *f, double *beta, double *q)
{
    wz7_init();
    smoothness7(f, beta, q);
}

double orc_recon5(int scheme, double CT, double eps, const double *f, int *delta)
{
    return recon5(scheme, CT, eps, f, delta);
}

void orc_iface_flux(const orc_params *P, int d, const double *Uk, const double *S, double *F, int *delta)
{
    iface_flux(P, d, Uk, S, F, delta);
}

void orc_phys_flux(const orc_params *P, const double *U, const double *nv, double *f)
{
    prim_t w;
    to_prim(P, P->ndim, U, &w);
    phys_flux(P->ndim, U, &w, nv, f);
}

/* averaged state and eigenvectors at the half node between UL and UR */
void orc_eigen(const orc_params *P, int d, const double *UL, const double *UR, const double *nv,
               double *Lout, double *Rout, double *lam)
{
    const int nd = P->ndim, nc = nd + 2;
    prim_t wl, wr;
    to_prim(P, nd, UL, &wl);
    to_prim(P, nd, UR, &wr);
    double uh[3], Hh;
    double a = sqrt(half_state(P, nd, &wl, &wr, uh, &Hh));
    double Lm[NCMAX][NCMAX], Rm[NCMAX][NCMAX];
    eigvecs(P, nd, d, uh, Hh, a, nv, Lm, Rm);
    double un = 0.0;
    for (int m = 0; m < nd; m++) un += uh[m] * nv[m];
    for (int j = 0; j < nc; j++)
        for (int c = 0; c < nc; c++) { Lout[j * nc + c] = Lm[j][c]; Rout[c * nc + j] = Rm[c][j]; }
    lam[0] = un - a;
    for (int j = 1; j <= nd; j++) lam[j] = un;
    lam[nd + 1] = un + a;
}

/* D of a 1D array (n points; periodic flag) */
void orc_deriv2_line(const double *f, int64_t n, int periodic, double *out)
{
    orc_params P;
    memset(&P, 0, sizeof(P));
    P.ndim = 1;
    P.n[0] = n;
    P.bc[0][0] = P.bc[0][1] = periodic ? BC_PERIODIC : BC_EXTRAPOLATE;
    grid_t g;
    grid_make(&P, &g);
    for (int64_t i = 0; i < n; i++) out[i] = d2arr(&P, &g, f, 0, i, 0, 0);
}

void orc_deriv_line(const double *f, int64_t n, int periodic, double *out)
{
    orc_params P;
    memset(&P, 0, sizeof(P));
    P.ndim = 1;
    P.n[0] = n;
    P.bc[0][0] = P.bc[0][1] = periodic ? BC_PERIODIC : BC_EXTRAPOLATE;
    grid_t g;
    grid_make(&P, &g);
    for (int64_t i = 0; i < n; i++) out[i] = darr(&P, &g, f, 0, i, 0, 0);
}

/* D along direction dir of an interior-node array (for the GCL test) */
void orc_deriv_field(const orc_params *P, const double *a, int dir, double *out)
{
    grid_t g;
    grid_make(P, &g);
    for (int64_t k = 0; k < g.n[2]; k++)
        for (int64_t j = 0; j < g.n[1]; j++)
            for (int64_t i = 0; i < g.n[0]; i++)
                out[cidx(&g, i, j, k)] = darr(P, &g, a, dir, i, j, k);
}

double orc_viscosity(const orc_params *P, double T) { return viscosity(P, T); }

int orc_abi_version(void) { return 1; }

/* viscous part of the residual alone (interior nodes, R overwritten) */
int orc_viscous_residual(const orc_params *P, const double *S, const double *J, const double *U, double *R)
{
    grid_t g;
    grid_make(P, &g);
    memset(R, 0, sizeof(double) * g.nc * g.nint);
    viscous_residual(P, &g, S, J, U, R);
    return 0;
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* threads the OpenMP loops of this library use */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------- learned-sensor support --
 * Not in the paper: the paper names sensor-switched hybrids of central and
 * shock-capturing fluxes (section 2, introduction) as hard to design by
 * hand.  The routed form replaces the characteristic TENO flux at an
 * interface the sensor calls smooth by the exact all-stencils-kept limit of
 * the same flux (cheap flux), and keeps the full flux elsewhere.
 *
 * Cheap flux: summing the split upwind-5 reconstructions of g+ and g- gives
 *   F = |S| [ C6 f + R diag(alpha) L D6 U ],
 *   C6 = (1, -8, 37, 37, -8, 1)/60,  D6 = (1, -5, 10, -10, 5, -1)/60 on
 *   i-2..i+3, with the averaged state, L, R and alpha of the full flux.
 */
void orc_cheap_flux(const orc_params *P, int d, const double *Uk, const double *S, double *F)
{
    const int nd = P->ndim, nc = nd + 2;
    double Smag = 0.0, nv[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < nd; m++) Smag += S[m] * S[m];
    Smag = sqrt(Smag);
    for (int m = 0; m < nd; m++) nv[m] = S[m] / Smag;
    prim_t w[6];
    double fk[6][NCMAX], lam[6][NCMAX];
    for (int k = 0; k < 6; k++) {
        to_prim(P, nd, Uk + k * nc, &w[k]);
        phys_flux(nd, Uk + k * nc, &w[k], nv, fk[k]);
        double un = 0.0;
        for (int m = 0; m < nd; m++) un += w[k].u[m] * nv[m];
        lam[k][0] = un - w[k].a;
        for (int j = 1; j <= nd; j++) lam[k][j] = un;
        lam[k][nd + 1] = un + w[k].a;
    }
    double uh[3], Hh;
    double ah = sqrt(half_state(P, nd, &w[2], &w[3], uh, &Hh));
    double Lm[NCMAX][NCMAX], Rm[NCMAX][NCMAX];
    eigvecs(P, nd, d, uh, Hh, ah, nv, Lm, Rm);
    const double C6[6] = {1.0 / 60.0, -8.0 / 60.0, 37.0 / 60.0, 37.0 / 60.0, -8.0 / 60.0, 1.0 / 60.0};
    const double D6[6] = {1.0 / 60.0, -5.0 / 60.0, 10.0 / 60.0, -10.0 / 60.0, 5.0 / 60.0, -1.0 / 60.0};
    double cf[NCMAX], du[NCMAX], v[NCMAX];
    for (int c = 0; c < nc; c++) {
        cf[c] = 0.0;
        du[c] = 0.0;
        for (int k = 0; k < 6; k++) {
            cf[c] += C6[k] * fk[k][c];
            du[c] += D6[k] * Uk[k * nc + c];
        }
    }
    for (int j = 0; j < nc; j++) {
        double alpha = 0.0, s = 0.0;
        for (int k = 0; k < 6; k++) alpha = fmax(alpha, fabs(lam[k][j]));
        for (int c = 0; c < nc; c++) s += Lm[j][c] * du[c];
        v[j] = alpha * s;
    }
    for (int c = 0; c < nc; c++) {
        double s = 0.0;
        for (int j = 0; j < nc; j++) s += Rm[c][j] * v[j];
        F[c] = Smag * (cf[c] + s);
    }
}

/* Sensor features of interface i+1/2 (ten values; reading of the sensor
 * inputs "smoothness indicators + normalised rho/p jumps"):
 *   f0..f3: Jiang-Shu three-point indicators B(a,b,c) = 13/12 (a-2b+c)^2 +
 *     1/4 (a-c)^2 of rho/rho_bar + p/p_bar + (u.t_s)/a_bar summed over the
 *     tangents, on the substencils {i-2..i}, {i-1..i+1}, {i..i+2},
 *     {i+1..i+3}, divided by their sum (+1e-20, so variations at rounding
 *     level read as a uniform state), with a_bar = sqrt(gamma p_bar/rho_bar);
 *   f4..f6: jumps J = |rho_{k+1} - rho_k| / (rho_{k+1} + rho_k) over (i-1,i),
 *     (i,i+1), (i+1,i+2), log-normalised as log10(1 + 1e6 J)/6;  f7..f9: the
 *     same for p.
 * rho_bar, p_bar: means of nodes i, i+1.
 * Label: 1 iff every TENO stencil of every field and both splits is kept. */
static double js3(const double *q, int m)
{
    const double a1 = q[m] - 2.0 * q[m + 1] + q[m + 2], a2 = q[m] - q[m + 2];
    return (13.0 / 12.0) * a1 * a1 + 0.25 * a2 * a2;
}

void orc_features(const orc_params *P, int d, const double *Uk, const double *S, double *feat, int *label)
{
    const int nd = P->ndim, nc = nd + 2;
    double Smag = 0.0, nv[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < nd; m++) Smag += S[m] * S[m];
    Smag = sqrt(Smag);
    for (int m = 0; m < nd; m++) nv[m] = S[m] / Smag;
    double t[2][3];
    tangents(nd, d, nv, t);
    prim_t w[6];
    for (int k = 0; k < 6; k++) to_prim(P, nd, Uk + k * nc, &w[k]);
    const double rb = 0.5 * (w[2].rho + w[3].rho), pb = 0.5 * (w[2].p + w[3].p);
    const double ab = sqrt(P->gamma * pb / rb);
    /* the normalised variables, then the indicators of their substencils */
    double r[6], q[6], vt[2][6];
    for (int k = 0; k < 6; k++) {
        r[k] = w[k].rho / rb;
        q[k] = w[k].p / pb;
        for (int s = 0; s < nd - 1; s++) {
            double ut = 0.0;
            for (int m = 0; m < nd; m++) ut += w[k].u[m] * t[s][m];
            vt[s][k] = ut / ab;
        }
    }
    double beta[4], sum = 0.0;
    for (int m = 0; m < 4; m++) {
        double b = js3(r, m) + js3(q, m);
        for (int s = 0; s < nd - 1; s++) b += js3(vt[s], m);
        beta[m] = b;
        sum += b;
    }
    for (int m = 0; m < 4; m++) feat[m] = beta[m] / (sum + 1e-20);
    for (int m = 0; m < 3; m++) {
        double jr = fabs(w[m + 2].rho - w[m + 1].rho) / (w[m + 2].rho + w[m + 1].rho);
        double jp = fabs(w[m + 2].p - w[m + 1].p) / (w[m + 2].p + w[m + 1].p);
        feat[4 + m] = log10(1.0 + 1e6 * jr) / 6.0;
        feat[7 + m] = log10(1.0 + 1e6 * jp) / 6.0;
    }
    if (label) {
        int dl[NCMAX * 2 * 4];
        double F[NCMAX];
        iface_flux(P, d, Uk, S, F, dl);
        int all = 1;
        for (int i = 0; i < nc * 2 * 4; i++) all &= dl[i];
        *label = all;
    }
}
