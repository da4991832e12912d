/*
 * lbref.c -- FP64 CPU oracle for the improved MRT pseudopotential D2Q9 step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  It is loaded by the test-suite, by the
 * package smoke check and by the benchmark's CPU-baseline leg, and by nothing
 * else.  It shares no source, header, table or helper with the GPU library.
 *
 * Every quantity is double precision.  The update follows the paper
 * (Li, Luo & Li, "Lattice Boltzmann modeling of multiphase flows at large
 * density ratio with an improved pseudopotential model"):
 *
 *   Sec. II   Eq. (1)  velocity-space MRT evolution (dense-matrix form, kept
 *                      for cross-checking the moment form on tiny grids)
 *             Eq. (2)  relaxation rates Lambda
 *             Eq. (3)  moment equilibria m_eq
 *             Eq. (4)  moment-space collision m* = m - L(m - m_eq) + (I - L/2) Sbar
 *             Eq. (5)  streaming f(x + e, t + 1) = f*(x, t), f* = M^-1 m*
 *             Eq. (6)  rho = sum f,  rho v = sum e f + F/2
 *             Eq. (7)  interaction force, w(1) = 1/3, w(2) = 1/12 (nearest
 *                      neighbours), or the 24-site stencil of nearest and
 *                      next-nearest neighbours (Sec. III.B, epsilon = 10/31)
 *             Eq. (10) kinematic viscosity nu = (tau_nu - 1/2)/3
 *   Sec. III  Eq. (24) psi = sqrt(2 (p_EOS - rho c_s^2) / (G c^2))  (psi_form 0)
 *             Eq. (23) Sbragaglia-Shan psi = exp(-1/rho) (eps = 0) or
 *                      (rho / (eps + rho))^(1/eps)                     (psi_form 1)
 *             Eq. (25) improved forcing term Sbar
 *   Sec. IV   Eq. (30) Carnahan-Starling p_EOS
 *   Sec. IV.C density-dependent viscosity nu(rho) = nu_l if rho >= rho_c else nu_g
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - velocity ordering e_0..e_8 and the orthogonal matrix M are the standard
 *     Lallemand-Luo D2Q9 ones (the paper names M but does not print it);
 *   - halfway bounce-back at the two y walls when bc == 1; the pseudopotential
 *     beyond a wall equals the value of the adjacent fluid row, same column;
 *   - the velocity that enters m_eq and Sbar is the half-force-corrected v of
 *     Eq. (6).
 *
 * State convention: f[alpha][y][x] holds the post-streaming distributions at
 * time t (row-major, x fastest, alpha-major planes).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9

enum { LBREF_OK = 0, LBREF_EINVAL = -1, LBREF_ENOMEM = -2, LBREF_EUNSTABLE = -4 };
enum { LBREF_PERIODIC = 0, LBREF_WALLS_Y = 1 };
enum { LBREF_FORM_MOMENT = 0, LBREF_FORM_VELOCITY = 1 };
enum { LBREF_PSI_CS = 0, LBREF_PSI_SS = 1 };

typedef struct {
    int32_t nx, ny, bc, pad_;
    double a, b, R, T, G, sigma;        /* Eq. (30), Eq. (7)/(24), Eq. (25) */
    double s_rho, s_e, s_zeta, s_j, s_q;/* Eq. (2), as rates 1/tau         */
    double nu_l, nu_g, rho_switch;      /* Sec. IV.C viscosity switch      */
    int32_t psi_form;                   /* Eq. (24) (0) or Eq. (23) (1)    */
    int32_t stencil;                    /* interaction range of Eq. (7)    */
    double psi_eps;                     /* epsilon of Eq. (23)             */
} lbref_params;

/* Interaction stencils of Eq. (7), F = -G psi(x) sum_e w(|e|^2) psi(x + e) e:
 *   LBREF_NEAREST    the eight nearest neighbours, w(1) = 1/3, w(2) = 1/12 (Sec. II);
 *   LBREF_MULTIRANGE nearest and next-nearest neighbours: the 24 sites with
 *                    |e|^2 in {1, 2, 4, 5, 8}.  Sec. III.B quotes epsilon = 10/31 for
 *                    such interactions without printing weights.  The weights used
 *                    are the unique ones that make the stencil's moments isotropic up
 *                    to eighth order with sum w e_x^2 = 1 (the normalisation of the
 *                    nearest-neighbour weights, so the bulk term G psi^2 / 2 of
 *                    Eq. (19) and Eq. (24) are unchanged):
 *                    w(1) = 4/21, w(2) = 4/45, w(4) = 1/60, w(5) = 2/315,
 *                    w(8) = 1/5040.  The isotropy conditions and the epsilon = 10/31
 *                    of a flat interface are checked by the tests. */
enum { LBREF_NEAREST = 0, LBREF_MULTIRANGE = 1 };

/* Weight of a neighbour at squared distance q for the given stencil (0 if absent). */
static double stencil_weight(int stencil, int q)
{
    if (stencil == LBREF_MULTIRANGE) {
        switch (q) {
        case 1: return 4.0 / 21.0;
        case 2: return 4.0 / 45.0;
        case 4: return 1.0 / 60.0;
        case 5: return 2.0 / 315.0;
        case 8: return 1.0 / 5040.0;
        default: return 0.0;
        }
    }
    return q == 1 ? 1.0 / 3.0 : (q == 2 ? 1.0 / 12.0 : 0.0);
}

static int stencil_reach(int stencil) { return stencil == LBREF_MULTIRANGE ? 2 : 1; }

void lbref_stencil_weights(int stencil, double *w9)
{
    for (int q = 0; q < 9; ++q) w9[q] = stencil_weight(stencil, q);
}

/* D2Q9 velocities (standard ordering: rest, 4 axis, 4 diagonal). */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

/* Orthogonal transformation matrix M, rows = (rho, e, eps, jx, qx, jy, qy,
 * pxx, pxy).  The paper refers to it (Sec. II) without printing it. */
static const double MROWS[Q][Q] = {
    { 1,  1,  1,  1,  1,  1,  1,  1,  1},
    {-4, -1, -1, -1, -1,  2,  2,  2,  2},
    { 4, -2, -2, -2, -2,  1,  1,  1,  1},
    { 0,  1,  0, -1,  0,  1, -1, -1,  1},
    { 0, -2,  0,  2,  0,  1, -1, -1,  1},
    { 0,  0,  1,  0, -1,  1,  1, -1, -1},
    { 0,  0, -2,  0,  2,  1,  1, -1, -1},
    { 0,  1, -1,  1, -1,  0,  0,  0,  0},
    { 0,  0,  0,  0,  0,  1, -1,  1, -1},
};

/* Plain Gauss-Jordan inversion with partial pivoting (no use is made of the
 * orthogonality of M, so that a test can check that property separately). */
static int invert9(const double A[Q][Q], double Ainv[Q][Q])
{
    double w[Q][2 * Q];
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) {
            w[i][j] = A[i][j];
            w[i][Q + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int c = 0; c < Q; ++c) {
        int piv = c;
        for (int r = c + 1; r < Q; ++r)
            if (fabs(w[r][c]) > fabs(w[piv][c])) piv = r;
        if (w[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int j = 0; j < 2 * Q; ++j) {
                double t = w[c][j]; w[c][j] = w[piv][j]; w[piv][j] = t;
            }
        double d = w[c][c];
        for (int j = 0; j < 2 * Q; ++j) w[c][j] /= d;
        for (int r = 0; r < Q; ++r) {
            if (r == c) continue;
            double m = w[r][c];
            if (m == 0.0) continue;
            for (int j = 0; j < 2 * Q; ++j) w[r][j] -= m * w[c][j];
        }
    }
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) Ainv[i][j] = w[i][Q + j];
    return 0;
}

static double MINV[Q][Q];
static int minv_ready = 0;

static void ensure_minv(void)
{
    /* Idempotent: concurrent first calls compute the same values. */
    if (!minv_ready) {
        double tmp[Q][Q];
        invert9(MROWS, tmp);
        memcpy(MINV, tmp, sizeof(tmp));
        minv_ready = 1;
    }
}

void lbref_matrices(double *M_out, double *Minv_out)
{
    ensure_minv();
    for (int i = 0; i < Q; ++i)
        for (int j = 0; j < Q; ++j) {
            if (M_out) M_out[i * Q + j] = MROWS[i][j];
            if (Minv_out) Minv_out[i * Q + j] = MINV[i][j];
        }
}

/* Eq. (30): Carnahan-Starling equation of state. */
double lbref_p_eos(const lbref_params *p, double rho)
{
    double eta = p->b * rho / 4.0;
    double num = 1.0 + eta + eta * eta - eta * eta * eta;
    double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
    return rho * p->R * p->T * num / den - p->a * rho * rho;
}

/* psi^2 of the chosen pseudopotential.  Eq. (24) with c = 1, c_s^2 = 1/3:
 * psi^2 = 2 (p_EOS - rho/3) / G.  Eq. (23): psi = exp(-1/rho) for eps = 0,
 * (rho / (eps + rho))^(1/eps) otherwise. */
double lbref_psi2(const lbref_params *p, double rho)
{
    if (p->psi_form == LBREF_PSI_SS) {
        double psi = (p->psi_eps == 0.0) ? exp(-1.0 / rho) : pow(rho / (p->psi_eps + rho), 1.0 / p->psi_eps);
        return psi * psi;
    }
    return 2.0 * (lbref_p_eos(p, rho) - rho / 3.0) / p->G;
}

/* Bulk pressure of the model, rho c_s^2 + G c^2 psi^2 / 2 (the bulk terms of
 * Eqs. (19)-(21)); for the Eq. (24) psi this is p_EOS itself. */
double lbref_pressure(const lbref_params *p, double rho)
{
    if (p->psi_form == LBREF_PSI_SS) return rho / 3.0 + 0.5 * p->G * lbref_psi2(p, rho);
    return lbref_p_eos(p, rho);
}

/* Eq. (3): moment equilibria. */
static void moment_equilibrium(double rho, double vx, double vy, double meq[Q])
{
    double v2 = vx * vx + vy * vy;
    meq[0] = rho;
    meq[1] = rho * (-2.0 + 3.0 * v2);
    meq[2] = rho * (1.0 - 3.0 * v2);
    meq[3] = rho * vx;
    meq[4] = -rho * vx;
    meq[5] = rho * vy;
    meq[6] = -rho * vy;
    meq[7] = rho * (vx * vx - vy * vy);
    meq[8] = rho * vx * vy;
}

/* Eq. (25): improved forcing term in moment space (sigma = 0 gives Eq. (9)).
 * Written literally, with tau_e = 1/s_e and tau_zeta = 1/s_zeta, dt = 1. */
static void forcing_moments(const lbref_params *p, double vx, double vy,
                            double Fx, double Fy, double psi2, double S[Q])
{
    double vF = vx * Fx + vy * Fy;
    double F2 = Fx * Fx + Fy * Fy;
    double tau_e = 1.0 / p->s_e, tau_z = 1.0 / p->s_zeta;
    S[0] = 0.0;
    S[1] = 6.0 * vF + 12.0 * p->sigma * F2 / (psi2 * (tau_e - 0.5));
    S[2] = -6.0 * vF - 12.0 * p->sigma * F2 / (psi2 * (tau_z - 0.5));
    S[3] = Fx;
    S[4] = -Fx;
    S[5] = Fy;
    S[6] = -Fy;
    S[7] = 2.0 * (vx * Fx - vy * Fy);
    S[8] = vx * Fy + vy * Fx;
}

/* Eq. (2) with the density-dependent shear rate of Sec. IV.C:
 * nu(rho) = nu_l for rho >= rho_switch else nu_g; tau_nu = 3 nu + 1/2 (Eq. 10). */
static void relaxation_rates(const lbref_params *p, double rho, double s[Q])
{
    double nu = (rho >= p->rho_switch) ? p->nu_l : p->nu_g;
    double s_nu = 1.0 / (3.0 * nu + 0.5);
    s[0] = p->s_rho; s[1] = p->s_e; s[2] = p->s_zeta;
    s[3] = p->s_j;   s[4] = p->s_q; s[5] = p->s_j;
    s[6] = p->s_q;   s[7] = s_nu;   s[8] = s_nu;
}

/* One-site collision, moment form, Eqs. (3), (4) and (25); f* = M^-1 m*. */
static void collide_moment(const lbref_params *p, const double f[Q], double rho,
                           double vx, double vy, double Fx, double Fy,
                           double psi2, double fstar[Q])
{
    double m[Q], meq[Q], S[Q], s[Q], mstar[Q];
    for (int k = 0; k < Q; ++k) {
        m[k] = 0.0;
        for (int a = 0; a < Q; ++a) m[k] += MROWS[k][a] * f[a];
    }
    moment_equilibrium(rho, vx, vy, meq);
    forcing_moments(p, vx, vy, Fx, Fy, psi2, S);
    relaxation_rates(p, rho, s);
    for (int k = 0; k < Q; ++k)
        mstar[k] = m[k] - s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * s[k]) * S[k];
    for (int a = 0; a < Q; ++a) {
        fstar[a] = 0.0;
        for (int k = 0; k < Q; ++k) fstar[a] += MINV[a][k] * mstar[k];
    }
}

/* One-site collision, velocity-space form of Eq. (1):
 *   f* = f - Lbar (f - f_eq) + (S - Lbar S / 2),  Lbar = M^-1 Lambda M,
 * with f_eq = M^-1 m_eq and S = M^-1 Sbar.  Dense 9x9 products throughout. */
static void collide_velocity(const lbref_params *p, const double f[Q], double rho,
                             double vx, double vy, double Fx, double Fy,
                             double psi2, double fstar[Q])
{
    double meq[Q], Sm[Q], s[Q], feq[Q], Sv[Q], Lbar[Q][Q];
    moment_equilibrium(rho, vx, vy, meq);
    forcing_moments(p, vx, vy, Fx, Fy, psi2, Sm);
    relaxation_rates(p, rho, s);
    for (int a = 0; a < Q; ++a) {
        feq[a] = 0.0; Sv[a] = 0.0;
        for (int k = 0; k < Q; ++k) {
            feq[a] += MINV[a][k] * meq[k];
            Sv[a] += MINV[a][k] * Sm[k];
        }
    }
    for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b) {
            double acc = 0.0;
            for (int k = 0; k < Q; ++k) acc += MINV[a][k] * s[k] * MROWS[k][b];
            Lbar[a][b] = acc;
        }
    for (int a = 0; a < Q; ++a) {
        double relax = 0.0, lsv = 0.0;
        for (int b = 0; b < Q; ++b) {
            relax += Lbar[a][b] * (f[b] - feq[b]);
            lsv += Lbar[a][b] * Sv[b];
        }
        fstar[a] = f[a] - relax + (Sv[a] - 0.5 * lsv);
    }
}

int lbref_collide_site(const lbref_params *p, const double *f9, double rho,
                       double vx, double vy, double Fx, double Fy, double psi2,
                       int form, double *fstar9)
{
    ensure_minv();
    if (form == LBREF_FORM_MOMENT)
        collide_moment(p, f9, rho, vx, vy, Fx, Fy, psi2, fstar9);
    else
        collide_velocity(p, f9, rho, vx, vy, Fx, Fy, psi2, fstar9);
    return LBREF_OK;
}

static int validate(const lbref_params *p)
{
    if (!p || p->nx < 1 || p->ny < 1) return LBREF_EINVAL;
    if (p->bc != LBREF_PERIODIC && p->bc != LBREF_WALLS_Y) return LBREF_EINVAL;
    if (p->stencil != LBREF_NEAREST && p->stencil != LBREF_MULTIRANGE) return LBREF_EINVAL;
    if (!(p->G < 0.0)) return LBREF_EINVAL;
    if (p->psi_form == LBREF_PSI_CS) {
        if (!(p->b > 0.0) || !(p->T > 0.0)) return LBREF_EINVAL;
    } else if (p->psi_form == LBREF_PSI_SS) {
        if (!(p->psi_eps >= 0.0) || !isfinite(p->psi_eps)) return LBREF_EINVAL;
    } else {
        return LBREF_EINVAL;
    }
    return LBREF_OK;
}

static inline size_t IDX(const lbref_params *p, int a, int y, int x)
{
    return ((size_t)a * p->ny + (size_t)y) * p->nx + (size_t)x;
}

static inline int wrap(int i, int n) { return ((i % n) + n) % n; }

/* psi at one site (Eq. (30) + Eq. (24), or Eq. (23)).  Sets *bad (and returns
 * 0) for a non-finite density, or, for Eq. (24), b rho / 4 >= 1 or psi^2 <= 0,
 * or, for Eq. (23), rho <= 0. */
static double psi_site(const lbref_params *p, double r, int *bad)
{
    int ok;
    double s2 = 0.0;
    if (p->psi_form == LBREF_PSI_SS) {
        ok = isfinite(r) && r > 0.0;
        if (ok) s2 = lbref_psi2(p, r);
    } else {
        s2 = lbref_psi2(p, r);
        ok = isfinite(r) && (p->b * r / 4.0 < 1.0) && (s2 > 0.0);
    }
    if (!ok) {
        *bad = 1;
        return 0.0;
    }
    return sqrt(s2);
}

/* psi at every site of a density field; LBREF_EUNSTABLE (psi set to 0 there)
 * if some site is invalid as in psi_site. */
static int psi_of(const lbref_params *p, const double *rho, double *psi)
{
    const int nx = p->nx, ny = p->ny;
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            int b = 0;
            psi[i] = psi_site(p, rho[i], &b);
            bad |= b;
        }
    return bad ? LBREF_EUNSTABLE : LBREF_OK;
}

/* sum_e w(|e|^2) psi(x + e) e of Eq. (7) from the neighbourhood P[dy + 2][dx + 2]
 * (|dx|, |dy| <= 2).  Written as differences psi(x + e) - psi(x - e), with the
 * partners at +e_y and -e_y (or +e_x, -e_x) added as one pair, so that mirroring or
 * transposing the neighbourhood mirrors or swaps (sx, sy) exactly in floating point. */
static void stencil_sum(int stencil, const double P[5][5], double *sx, double *sy)
{
    const int r = stencil_reach(stencil);
    double ax = 0.0, ay = 0.0;
    for (int u = 1; u <= r; ++u)
        for (int v = 0; v <= r; ++v) {
            double w = stencil_weight(stencil, u * u + v * v);
            if (w == 0.0) continue;
            double dx, dy;
            if (v == 0) {
                dx = P[2][2 + u] - P[2][2 - u];
                dy = P[2 + u][2] - P[2 - u][2];
            } else {
                dx = (P[2 + v][2 + u] - P[2 + v][2 - u]) + (P[2 - v][2 + u] - P[2 - v][2 - u]);
                dy = (P[2 + u][2 + v] - P[2 - u][2 + v]) + (P[2 + u][2 - v] - P[2 - u][2 - v]);
            }
            ax += w * u * dx;
            ay += w * u * dy;
        }
    *sx = ax;
    *sy = ay;
}

/* psi around (x, y) into P[dy + 2][dx + 2] for |dx|, |dy| <= reach: x periodic; y
 * periodic, or clamped to the nearest fluid row beyond a wall. */
static void gather_psi(const lbref_params *p, const double *psi, int x, int y, double P[5][5])
{
    const int r = stencil_reach(p->stencil);
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            int xn = wrap(x + dx, p->nx), yn = y + dy;
            if (p->bc == LBREF_PERIODIC) yn = wrap(yn, p->ny);
            else if (yn < 0) yn = 0;
            else if (yn >= p->ny) yn = p->ny - 1;
            P[dy + 2][dx + 2] = psi[(size_t)yn * p->nx + xn];
        }
}

/* Eq. (7): F = -G psi(x) sum_e w(|e|^2) psi(x + e) e over the stencil's
 * neighbours.  Walls: psi beyond a wall equals the nearest fluid row, same column. */
static void force_of(const lbref_params *p, const double *psi, double *Fx, double *Fy)
{
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            double P[5][5], sx, sy;
            gather_psi(p, psi, x, y, P);
            stencil_sum(p->stencil, P, &sx, &sy);
            Fx[i] = -p->G * psi[i] * sx;
            Fy[i] = -p->G * psi[i] * sy;
        }
}

/* Initial state (post-streaming, t = 0): f = M^-1 m_eq(rho0, u_eq) at every
 * site.  u0 (NULL = zero) is the Eq. (6) fluid velocity, so the equilibrium
 * is taken at u_eq = u0 - F / (2 rho0) with F the Eq. (7) force of the
 * initial density field: then sum e f + F/2 = rho0 u0 and the moments at
 * t = 0 return (rho0, u0).  LBREF_EINVAL if rho0 gives an invalid psi. */
int lbref_init(const lbref_params *p, const double *rho0, const double *ux0,
               const double *uy0, double *f)
{
    int st = validate(p);
    if (st) return st;
    ensure_minv();
    const size_t n = (size_t)p->nx * p->ny;
    double *psi = (double *)malloc(n * sizeof(double));
    double *Fx = (double *)malloc(n * sizeof(double));
    double *Fy = (double *)malloc(n * sizeof(double));
    if (!psi || !Fx || !Fy) {
        free(psi); free(Fx); free(Fy);
        return LBREF_ENOMEM;
    }
    st = psi_of(p, rho0, psi);
    if (st) {
        free(psi); free(Fx); free(Fy);
        return LBREF_EINVAL;
    }
    force_of(p, psi, Fx, Fy);
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t i = (size_t)y * p->nx + x;
            double ux = (ux0 ? ux0[i] : 0.0) - Fx[i] / (2.0 * rho0[i]);
            double uy = (uy0 ? uy0[i] : 0.0) - Fy[i] / (2.0 * rho0[i]);
            double meq[Q];
            moment_equilibrium(rho0[i], ux, uy, meq);
            for (int a = 0; a < Q; ++a) {
                double acc = 0.0;
                for (int k = 0; k < Q; ++k) acc += MINV[a][k] * meq[k];
                f[IDX(p, a, y, x)] = acc;
            }
        }
    free(psi); free(Fx); free(Fy);
    return LBREF_OK;
}

/* Density, pseudopotential, force and velocity of the post-streaming state f
 * (Eqs. 6, 7, 24, 30).  Any output pointer may be NULL except rho/psi2
 * scratch, which are allocated here when NULL.  Returns LBREF_EUNSTABLE if
 * some site has a non-finite density or psi^2 <= 0. */
static int fields(const lbref_params *p, const double *f, double *rho,
                  double *psi, double *Fx, double *Fy, double *vx, double *vy)
{
    const int nx = p->nx, ny = p->ny;
    /* Eq. (6) density */
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            double r = 0.0;
            for (int a = 0; a < Q; ++a) r += f[IDX(p, a, y, x)];
            rho[(size_t)y * nx + x] = r;
        }
    if (psi_of(p, rho, psi)) return LBREF_EUNSTABLE;
    const size_t n = (size_t)nx * ny;
    double *fx = Fx ? Fx : (double *)malloc(n * sizeof(double));
    double *fy = Fy ? Fy : (double *)malloc(n * sizeof(double));
    if (!fx || !fy) {
        if (!Fx) free(fx);
        if (!Fy) free(fy);
        return LBREF_ENOMEM;
    }
    force_of(p, psi, fx, fy);
    if (vx || vy) {
#pragma omp parallel for
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t i = (size_t)y * nx + x;
                double jx = 0.0, jy = 0.0;
                for (int a = 0; a < Q; ++a) {
                    double fa = f[IDX(p, a, y, x)];
                    jx += EX[a] * fa;
                    jy += EY[a] * fa;
                }
                if (vx) vx[i] = (jx + 0.5 * fx[i]) / rho[i];
                if (vy) vy[i] = (jy + 0.5 * fy[i]) / rho[i];
            }
    }
    if (!Fx) free(fx);
    if (!Fy) free(fy);
    return LBREF_OK;
}

/* Macroscopic fields of the current state; any output may be NULL. */
int lbref_moments(const lbref_params *p, const double *f, double *rho_out,
                  double *ux, double *uy, double *Fx_out, double *Fy_out,
                  double *psi_out)
{
    int st = validate(p);
    if (st) return st;
    size_t n = (size_t)p->nx * p->ny;
    double *rho = rho_out ? rho_out : (double *)malloc(n * sizeof(double));
    double *psi = psi_out ? psi_out : (double *)malloc(n * sizeof(double));
    if (!rho || !psi) return LBREF_ENOMEM;
    st = fields(p, f, rho, psi, Fx_out, Fy_out, ux, uy);
    if (!rho_out) free(rho);
    if (!psi_out) free(psi);
    return st;
}

/* Eq. (5), push form: f(x + e_a) = f*_a(x).  x is periodic; y is periodic or
 * bounded by halfway bounce-back walls, where a population leaving through a
 * wall returns to its own site reversed. */
static void stream(const lbref_params *p, const double *fstar, double *f)
{
    const int nx = p->nx, ny = p->ny;
#pragma omp parallel for
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
            for (int a = 0; a < Q; ++a) {
                double v = fstar[IDX(p, a, y, x)];
                int xd = wrap(x + EX[a], nx);
                int yd = y + EY[a];
                if (p->bc == LBREF_PERIODIC)
                    f[IDX(p, a, wrap(yd, ny), xd)] = v;
                else if (yd < 0 || yd >= ny)
                    f[IDX(p, OPP[a], y, x)] = v;
                else
                    f[IDX(p, a, yd, xd)] = v;
            }
}

int lbref_stream(const lbref_params *p, const double *fstar, double *f)
{
    int st = validate(p);
    if (st) return st;
    stream(p, fstar, f);
    return LBREF_OK;
}

/* Post-collision distributions f*(x) (Eq. 4 with Eq. 25) at n listed sites
 * (flat indices y * nx + x) of the post-streaming state f; out is [n][9].
 * Only the neighbourhood the stencil reaches (3 x 3 or 5 x 5) of each site is
 * evaluated. */
int lbref_collide_at(const lbref_params *p, const double *f, int64_t n, const int64_t *sites,
                     double *out)
{
    int st = validate(p);
    if (st) return st;
    ensure_minv();
    const int nx = p->nx, ny = p->ny, r = stencil_reach(p->stencil);
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int64_t s = 0; s < n; ++s) {
        int x = (int)(sites[s] % nx), y = (int)(sites[s] / nx);
        double psi_n[5][5] = {{0.0}}, rho_c = 0.0, fl[Q];
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                int xn = wrap(x + dx, nx), yn = y + dy;
                if (p->bc == LBREF_PERIODIC) yn = wrap(yn, ny);
                else if (yn < 0) yn = 0;
                else if (yn >= ny) yn = ny - 1;
                double rr = 0.0;
                for (int a = 0; a < Q; ++a) rr += f[IDX(p, a, yn, xn)];
                int b = 0;
                psi_n[dy + 2][dx + 2] = psi_site(p, rr, &b);
                bad |= b;
                if (dx == 0 && dy == 0) rho_c = rr;
            }
        double sx, sy;
        stencil_sum(p->stencil, psi_n, &sx, &sy);
        double psi = psi_n[2][2];
        double Fx = -p->G * psi * sx, Fy = -p->G * psi * sy;
        double jx = 0.0, jy = 0.0;
        for (int a = 0; a < Q; ++a) {
            fl[a] = f[IDX(p, a, y, x)];
            jx += EX[a] * fl[a];
            jy += EY[a] * fl[a];
        }
        double vx = (jx + 0.5 * Fx) / rho_c, vy = (jy + 0.5 * Fy) / rho_c;
        collide_moment(p, fl, rho_c, vx, vy, Fx, Fy, psi * psi, out + 9 * s);
    }
    return bad ? LBREF_EUNSTABLE : LBREF_OK;
}

/* Advance nsteps.  f holds the post-streaming state at time t on entry and at
 * t + nsteps on success.  work must hold 9 * nx * ny doubles.  On an unstable
 * state the function returns LBREF_EUNSTABLE and *done gives the number of
 * completed steps (f then holds the state at t + *done). */
int lbref_step(const lbref_params *p, double *f, double *work, int64_t nsteps,
               int form, int64_t *done)
{
    int st = validate(p);
    if (st) return st;
    ensure_minv();
    const int nx = p->nx, ny = p->ny;
    size_t n = (size_t)nx * ny;
    double *rho = (double *)malloc(n * sizeof(double));
    double *psi = (double *)malloc(n * sizeof(double));
    double *Fx = (double *)malloc(n * sizeof(double));
    double *Fy = (double *)malloc(n * sizeof(double));
    double *vx = (double *)malloc(n * sizeof(double));
    double *vy = (double *)malloc(n * sizeof(double));
    if (!rho || !psi || !Fx || !Fy || !vx || !vy) {
        free(rho); free(psi); free(Fx); free(Fy); free(vx); free(vy);
        return LBREF_ENOMEM;
    }
    int64_t k = 0;
    st = LBREF_OK;
    for (; k < nsteps; ++k) {
        st = fields(p, f, rho, psi, Fx, Fy, vx, vy);
        if (st) break;
        /* Collision (Eq. 4 or Eq. 1) then streaming (Eq. 5), push form. */
#pragma omp parallel for
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t i = (size_t)y * nx + x;
                double fl[Q], fs[Q];
                for (int a = 0; a < Q; ++a) fl[a] = f[IDX(p, a, y, x)];
                double s2 = psi[i] * psi[i];
                if (form == LBREF_FORM_MOMENT)
                    collide_moment(p, fl, rho[i], vx[i], vy[i], Fx[i], Fy[i], s2, fs);
                else
                    collide_velocity(p, fl, rho[i], vx[i], vy[i], Fx[i], Fy[i], s2, fs);
                for (int a = 0; a < Q; ++a) work[IDX(p, a, y, x)] = fs[a];
            }
        stream(p, work, f);
    }
    if (done) *done = k;
    free(rho); free(psi); free(Fx); free(Fy); free(vx); free(vy);
    return st;
}

#ifdef _OPENMP
#include <omp.h>
#endif

/* Number of threads the oracle's parallel loops use. */
int lbref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
