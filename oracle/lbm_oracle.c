/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference of the lattice update studied in
 * Han, Ooka & Kikumoto, "A wall function approach in lattice Boltzmann
 * method: algorithm and validation using turbulent channel flow"
 * (arXiv 2009.04352).  It exists so that the GPU library can be checked
 * against something written independently from the paper; it shares no
 * code, header, table or helper with the GPU library and must never be
 * called from the product path (only from tests, the smoke check and the
 * CPU-baseline leg of the benchmark).
 *
 * What one time step computes, for every cell c = (x, y, z) of an
 * nx * ny * nz channel (x, z periodic; walls below y = 0 and above
 * y = ny - 1, halfway between the last cell and its missing neighbour):
 *
 *   1. gather   f_a(c) = fpost_a(c - e_a)                         (Eq. 1)
 *               wall-crossing links: bounce-back (Eq. 3, 3-D form) or
 *               mirror reflection (free-slip, Eq. 4, 3-D form).
 *   2. WFB      at wall cells, Spalding's law (Eq. 16-17) solved by Newton
 *               for u_tau, tau_w split along the wall velocity (Eq. 15),
 *               and the four reflected diagonal populations shifted by
 *               +-tau/2 (Eq. 13-14).
 *   3. moments  rho, u (Eq. 2), with the half-force velocity shift.
 *   4. SGS      Smagorinsky eddy viscosity (Cs, Sec. 3.1) from the local
 *               non-equilibrium stress.
 *   5. collide  BGK towards the second-order equilibrium, plus the body
 *               force term F_a of Eq. 1.
 *
 * Readings of points the paper leaves open (all are listed with reasons in
 * the project's design notes):
 *   - walls are link-wise (halfway); WFB acts on the first fluid layer;
 *   - y1 (distance used in y+) is a parameter, default one lattice spacing;
 *   - the velocity fed to Spalding's law is the free-slip (gathered)
 *     tangential velocity, including the half-force shift;
 *   - Newton starts from the viscous-sublayer guess u_tau = sqrt(nu U / y1)
 *     and stops on a relative step below newton_tol;
 *   - U = 0 gives tau_w = 0;
 *   - the top wall is the bottom wall mirrored in y;
 *   - collision is single-relaxation-time (BGK); the Smagorinsky closure is
 *     tau_e = (tau0 + sqrt(tau0^2 + 18 Cs^2 Q / rho)) / 2 with
 *     Q = sqrt(2 Pi:Pi), Pi the non-equilibrium second moment;
 *   - F_a is the Guo et al. (2002) force term with u = (sum e f + F/2)/rho;
 *   - MRT (optional, the paper's collision, Sec. 3.1 [40]): the moment basis
 *     of d'Humieres et al. (2002) for D3Q19, equilibrium moments taken as the
 *     moments of the same second-order equilibrium (so equal rates give BGK),
 *     the stress moments relaxed at 1/tau_e, the others at given rates, the
 *     force term added as (I - S/2) M F in moment space;
 *   - van Driest damping (optional, Sec. 3.1 [42]): Cs (1 - exp(-y+/A+)) with
 *     y+ = d u_tau,ref / nu0, d = min(y, ny - 1 - y) + y1 (the distance used
 *     for the first layer) and u_tau,ref the given friction velocity, or
 *     sqrt(|Fx| ny / 2) from the force balance when none is given.
 *
 * Arithmetic is IEEE FP64 throughout, summation order a = 0..18, built
 * with -ffp-contract=off.  Populations are stored as full f (not f - w).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19

/* Discrete velocities of D3Q19 in the paper's numbering (Table A-1). */
static const int E[Q][3] = {
    {0, 0, 0},                            /* 0 */
    {1, 0, 0},   {-1, 0, 0},              /* 1, 2 */
    {0, 1, 0},   {0, -1, 0},              /* 3, 4 */
    {0, 0, 1},   {0, 0, -1},              /* 5, 6 */
    {1, 1, 0},   {-1, -1, 0},             /* 7, 8 */
    {1, 0, 1},   {-1, 0, -1},             /* 9, 10 */
    {0, 1, 1},   {0, -1, -1},             /* 11, 12 */
    {1, -1, 0},  {-1, 1, 0},              /* 13, 14 */
    {1, 0, -1},  {-1, 0, 1},              /* 15, 16 */
    {0, 1, -1},  {0, -1, 1},              /* 17, 18 */
};

static double W[Q];  /* weights, Qian et al. (1992): 1/3, 1/18, 1/36 by |e|^2 */
static int OPP[Q];   /* e_opp(a) = -e_a */
static int MIR[Q];   /* e_mir(a) = (e_ax, -e_ay, e_az): reflection in the wall */
static int tables_ready = 0;

static void tables_init(void)
{
    if (tables_ready) return;
    for (int a = 0; a < Q; ++a) {
        int n2 = E[a][0] * E[a][0] + E[a][1] * E[a][1] + E[a][2] * E[a][2];
        W[a] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1) ? 1.0 / 18.0 : 1.0 / 36.0;
        OPP[a] = -1;
        MIR[a] = -1;
        for (int b = 0; b < Q; ++b) {
            if (E[b][0] == -E[a][0] && E[b][1] == -E[a][1] && E[b][2] == -E[a][2]) OPP[a] = b;
            if (E[b][0] == E[a][0] && E[b][1] == -E[a][1] && E[b][2] == E[a][2]) MIR[a] = b;
        }
    }
    tables_ready = 1;
}

enum { ORC_BB = 0, ORC_WFB = 1, ORC_FREESLIP = 2 };
enum { ORC_BGK = 0, ORC_MRT = 1 };
enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_NONFINITE = -5, ORC_E_NEWTON = -6 };

typedef struct {
    int32_t nx, ny, nz;
    int32_t bc;          /* ORC_BB, ORC_WFB or ORC_FREESLIP */
    double tau0;         /* molecular relaxation time, nu0 = (tau0 - 1/2) / 3 */
    double cs;           /* Smagorinsky constant */
    double kappa, bconst;/* Spalding's law constants */
    double fx;           /* body force density along x */
    double y1;           /* wall distance of the first fluid layer in y+ */
    double newton_tol;   /* relative step that ends Newton */
    int32_t newton_maxit;
    int32_t stats_every; /* sample statistics on steps t with t % every == 0; 0 = off */
    int32_t collision;   /* ORC_BGK or ORC_MRT */
    double s_e, s_eps;   /* MRT rates of the energy and energy-square moments */
    double s_q;          /* MRT rate of the heat-flux moments */
    double s_pi;         /* MRT rate of the fourth-order normal-stress moments */
    double s_m;          /* MRT rate of the third-order m moments */
    double vd_aplus;     /* van Driest A+; <= 0: no damping */
    double vd_utau;      /* friction velocity for the damping's y+; <= 0: sqrt(|Fx| ny / 2) */
    int32_t wall_nodes;  /* 0: link-wise walls halfway below row 0 and above row ny - 1, WFB on the
                          * first fluid layer; 1: wall nodes at y = -1 and y = ny (Sec. 2.1-2.2,
                          * Eq. 3, 4 and 14 applied at the wall grid), the stress of a step's
                          * wall-node collision from the first layer's velocity of the previous
                          * step; 2: the same wall nodes, the stress from the first layer's
                          * velocity of the same step */
} orc_params;

typedef struct {
    orc_params p;
    int64_t ncell;
    double *fpost, *fnew;   /* [a][z][y][x], post-collision populations */
    int64_t steps;
    int status;
    int64_t first_bad_step;
    int32_t max_newton_iters;
    double *stats;          /* [y][8]: sums of ux uy uz ux^2 uy^2 uz^2 ux*uy, count */
    int64_t nsamples;
    /* wall nodes (p.wall_nodes): the five populations each wall node sends
     * into the fluid, [w][k][z][x] with k indexing the directions IN_W[w],
     * and the first layer's rho, u_x, u_z of the latest step, [w][z][x][3],
     * from which the next wall-node collision takes its stress */
    double *fw, *fw_new;
    double *urec, *urec_new;
} orc;

/* ------------------------------------------------------------ threads */

/* Threads the OpenMP loops over z use (1 without OpenMP), and a way to set
 * them; the results do not depend on the count (cells are independent and
 * every sum runs in a fixed order). */
int32_t orc_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads((int)n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------- tables */

void orc_tables(int32_t* e, double* w, int32_t* opp, int32_t* mir)
{
    tables_init();
    for (int a = 0; a < Q; ++a) {
        for (int d = 0; d < 3; ++d) e[3 * a + d] = E[a][d];
        w[a] = W[a];
        opp[a] = OPP[a];
        mir[a] = MIR[a];
    }
}

/* ------------------------------------------------------- Spalding's law */

/* Eq. 16: y+ as an explicit function of u+. */
double orc_spalding_yplus(double up, double kappa, double b)
{
    double k = kappa * up;
    return up + exp(-kappa * b) * (exp(k) - 1.0 - k - k * k / 2.0 - k * k * k / 6.0);
}

/* Invert Eq. 16 for u+ at a given y+ by bisection on [0, y+] (Sp(p) >= p).
 * Used for the initial profile and for workload parameters only. */
double orc_spalding_uplus(double yplus, double kappa, double b)
{
    if (!(yplus > 0.0)) return 0.0;
    double lo = 0.0, hi = yplus;
    for (int i = 0; i < 200; ++i) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (orc_spalding_yplus(mid, kappa, b) < yplus) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Wall-function Newton solve (Sec. 2.3).  With y+ = y1 u_tau / nu and
 * u+ = U / u_tau (Eq. 17), writing p = u+ and R = y1 U / nu turns Eq. 16
 * into H(p) = p Sp(p) - R = 0.  Start: viscous sublayer u+ = y+, i.e.
 * u_tau = sqrt(nu U / y1), p0 = sqrt(R).  Returns u_tau, or -1 on failure. */
double orc_wall_utau(double U, double y1, double nu, double kappa, double b,
                     double tol, int maxit, int32_t* iters_out)
{
    if (iters_out) *iters_out = 0;
    if (U == 0.0) return 0.0;
    double R = y1 * U / nu;
    double p = sqrt(R);
    double ekb = exp(-kappa * b);
    for (int it = 1; it <= maxit; ++it) {
        double k = kappa * p;
        double ek = exp(k);
        double sp = p + ekb * (ek - 1.0 - k - k * k / 2.0 - k * k * k / 6.0);
        double dsp = 1.0 + kappa * ekb * (ek - 1.0 - k - k * k / 2.0);
        double h = p * sp - R;
        double dh = sp + p * dsp;
        double pn = p - h / dh;
        if (iters_out) *iters_out = it;
        if (fabs(pn - p) <= tol * pn) return U / pn;
        p = pn;
    }
    return -1.0;
}

/* ------------------------------------------------------ one-cell pieces */

/* Second-order equilibrium (Qian et al. 1992), c_s^2 = 1/3. */
static double feq(int a, double rho, const double u[3])
{
    double eu = E[a][0] * u[0] + E[a][1] * u[1] + E[a][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return W[a] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

void orc_feq(double rho, const double* u, double* out)
{
    tables_init();
    for (int a = 0; a < Q; ++a) out[a] = feq(a, rho, u);
}

/* Eq. 2 with the half-force shift: rho = sum f, rho u = sum e f + F/2. */
static void moments(const double f[Q], double fx, double* rho, double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < Q; ++a) {
        r += f[a];
        for (int d = 0; d < 3; ++d) j[d] += E[a][d] * f[a];
    }
    j[0] += 0.5 * fx;
    *rho = r;
    for (int d = 0; d < 3; ++d) u[d] = j[d] / r;
}

/* WFB correction of the gathered populations of one wall cell, Eqs. 13-17.
 * wall = 0: bottom (wall below, +y into the flow, the paper's setting);
 * wall = 1: top (the bottom case mirrored in y).
 * rec (may be NULL) receives tau_x, tau_z, u_tau, U. */
/* The wall stress of Eq. 15-17 for density rho and wall-parallel velocity
 * (vx, vz): u_tau from Spalding's law by Newton, tau_w = rho u_tau^2, split
 * against the velocity.  rec receives tau_x, tau_z, u_tau, U. */
int orc_wall_tau(const orc_params* p, double rho, double vx, double vz, double rec[4], int32_t* iters)
{
    double U = sqrt(vx * vx + vz * vz);
    double taux = 0.0, tauz = 0.0, utau = 0.0;
    int32_t it = 0;
    if (iters) *iters = 0;
    if (U > 0.0) {
        double nu0 = (p->tau0 - 0.5) / 3.0;
        utau = orc_wall_utau(U, p->y1, nu0, p->kappa, p->bconst, p->newton_tol,
                             p->newton_maxit, &it);
        if (iters) *iters = it;
        if (utau < 0.0) return ORC_E_NEWTON;
        double tauw = rho * utau * utau;           /* Eq. 17 */
        taux = -(vx / U) * tauw;                   /* Eq. 15 */
        tauz = -(vz / U) * tauw;
    }
    rec[0] = taux; rec[1] = tauz; rec[2] = utau; rec[3] = U;
    return ORC_OK;
}

int orc_wfb_cell(const orc_params* p, int wall, double f[Q], double rec[4], int32_t* iters)
{
    tables_init();
    double rho = 0.0, jx = 0.0, jz = 0.0;
    for (int a = 0; a < Q; ++a) {
        rho += f[a];
        jx += E[a][0] * f[a];
        jz += E[a][2] * f[a];
    }
    jx += 0.5 * p->fx;
    double vx = jx / rho, vz = jz / rho;          /* free-slip velocity v, Eq. 7-10 */
    double r[4];
    int32_t it = 0;
    int st = orc_wall_tau(p, rho, vx, vz, r, &it);
    if (st != ORC_OK) {
        if (iters) *iters = it;
        return st;
    }
    double taux = r[0], tauz = r[1], utau = r[2], U = r[3];
    /* Eq. 13 (dt = dy = 1): the in-pointing diagonals of the bottom wall are
     * 7 and 14 (x) and 11 and 17 (z); the top wall uses their mirror images. */
    int a7 = 7, a14 = 14, a11 = 11, a17 = 17;
    if (wall == 1) { a7 = MIR[7]; a14 = MIR[14]; a11 = MIR[11]; a17 = MIR[17]; }
    f[a7] += 0.5 * taux;
    f[a14] -= 0.5 * taux;
    f[a11] += 0.5 * tauz;
    f[a17] -= 0.5 * tauz;
    if (rec) { rec[0] = taux; rec[1] = tauz; rec[2] = utau; rec[3] = U; }
    if (iters) *iters = it;
    return ORC_OK;
}

/* Populations a wall node sends into the fluid (e_y = +1 at the bottom
 * wall, -1 at the top), in the order k = 0..4 of the wall-node arrays. */
static const int IN_W[2][5] = {{3, 7, 11, 14, 17}, {4, 13, 18, 8, 12}};

/* The collision of a wall node (Sec. 2.1-2.2, applied at the wall grid
 * itself), literally, on all 19 populations f that reached it:
 *   bounce-back (Eq. 3 in 3-D form): every population reversed;
 *   WFB (Eq. 14): the wall-normal and in-plane populations reversed (14c),
 *     the in-pointing diagonals from their mirror images plus or minus
 *     tau/2 (14a-b), the out-pointing diagonals equal to the corrected
 *     in-pointing ones (14c); the rest population unchanged;
 *   free-slip (Eq. 4 in 3-D form): Eq. 14 with tau = 0.
 * wall = 1 (top) is the bottom rule mirrored in y. */
void orc_wall_node_collide(const orc_params* p, int wall, const double f[Q], double taux, double tauz, double out[Q])
{
    tables_init();
    double g[Q], o[Q];
    for (int a = 0; a < Q; ++a) g[a] = (wall == 0) ? f[a] : f[MIR[a]];   /* the bottom picture */
    if (p->bc == ORC_BB) {
        for (int a = 0; a < Q; ++a) o[a] = g[OPP[a]];
    } else {
        double tx = (p->bc == ORC_WFB) ? taux : 0.0, tz = (p->bc == ORC_WFB) ? tauz : 0.0;
        o[0] = g[0];
        o[7] = g[13] + 0.5 * tx;                       /* 14a */
        o[14] = g[8] - 0.5 * tx;
        o[11] = g[18] + 0.5 * tz;                      /* 14b */
        o[17] = g[12] - 0.5 * tz;
        o[1] = g[2]; o[2] = g[1]; o[3] = g[4]; o[4] = g[3]; o[5] = g[6]; o[6] = g[5];   /* 14c */
        o[8] = o[7]; o[9] = g[10]; o[10] = g[9]; o[12] = o[11]; o[13] = o[14];
        o[15] = g[16]; o[16] = g[15]; o[18] = o[17];
    }
    for (int a = 0; a < Q; ++a) {
        if (wall == 0) out[a] = o[a];
        else out[MIR[a]] = o[a];
    }
}

static double cs_at(const orc_params* p, int y);
static double mrate(const orc_params* p, int k, double omega);
static double mrow(int k, int a);

/* Collision + Smagorinsky + body force on gathered (and WFB-corrected) f of
 * a cell in row y (y < 0: no van Driest damping).  BGK, or MRT in the
 * moment basis.  out receives the post-collision populations; taue_out
 * (may be NULL) the effective relaxation time. */
void orc_collide_cell_at(const orc_params* p, int y, const double f[Q], double out[Q], double* taue_out)
{
    tables_init();
    double rho, u[3], fe[Q];
    moments(f, p->fx, &rho, u);
    for (int a = 0; a < Q; ++a) fe[a] = feq(a, rho, u);
    double pi[3][3] = {{0}};
    for (int a = 0; a < Q; ++a)
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) pi[i][j] += E[a][i] * E[a][j] * (f[a] - fe[a]);
    double pp = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) pp += pi[i][j] * pi[i][j];
    double qn = sqrt(2.0 * pp);
    double cs = cs_at(p, y);
    double taue = 0.5 * (p->tau0 + sqrt(p->tau0 * p->tau0 + 18.0 * cs * cs * qn / rho));
    double fvec[3] = {p->fx, 0.0, 0.0};
    double force[Q];
    for (int a = 0; a < Q; ++a) {
        double eu = E[a][0] * u[0] + E[a][1] * u[1] + E[a][2] * u[2];
        double ef = E[a][0] * fvec[0] + E[a][1] * fvec[1] + E[a][2] * fvec[2];
        double emuf = (E[a][0] - u[0]) * fvec[0] + (E[a][1] - u[1]) * fvec[1] + (E[a][2] - u[2]) * fvec[2];
        force[a] = W[a] * (3.0 * emuf + 9.0 * eu * ef);
    }
    if (p->collision == ORC_MRT) {
        /* m* = m - S (m - m_eq) + (I - S/2) M F, then f* = M^-1 m* with
         * M^-1 = M^T diag(1 / |row k|^2) (the rows are orthogonal) */
        double mstar[Q];
        for (int k = 0; k < Q; ++k) {
            double m = 0.0, meq = 0.0, mf = 0.0;
            for (int a = 0; a < Q; ++a) {
                double c = mrow(k, a);
                m += c * f[a];
                meq += c * fe[a];
                mf += c * force[a];
            }
            double sk = mrate(p, k, 1.0 / taue);
            mstar[k] = m - sk * (m - meq) + (1.0 - 0.5 * sk) * mf;
        }
        for (int a = 0; a < Q; ++a) {
            double v = 0.0;
            for (int k = 0; k < Q; ++k) {
                double n2 = 0.0;
                for (int b = 0; b < Q; ++b) n2 += mrow(k, b) * mrow(k, b);
                v += mrow(k, a) * mstar[k] / n2;
            }
            out[a] = v;
        }
    } else {
        for (int a = 0; a < Q; ++a)
            out[a] = f[a] - (f[a] - fe[a]) / taue + (1.0 - 1.0 / (2.0 * taue)) * force[a];
    }
    if (taue_out) *taue_out = taue;
}

void orc_collide_cell(const orc_params* p, const double f[Q], double out[Q], double* taue_out)
{
    orc_collide_cell_at(p, -1, f, out, taue_out);
}

/* ------------------------------------------------------------------ MRT */

/* Row k of the D3Q19 moment basis of d'Humieres et al. (2002) at velocity e:
 * the polynomials 1, e2 = |e|^2, energy and energy square, momentum and heat
 * flux, the normal and off-diagonal stresses with their fourth-order
 * partners, and the three third-order m moments, orthogonal over the 19
 * velocities. */
static double mrow(int k, int a)
{
    const double ex = E[a][0], ey = E[a][1], ez = E[a][2];
    const double e2 = ex * ex + ey * ey + ez * ez;
    switch (k) {
        case 0: return 1.0;                                            /* rho */
        case 1: return 19.0 * e2 - 30.0;                               /* e */
        case 2: return (21.0 * e2 * e2 - 53.0 * e2 + 24.0) / 2.0;      /* epsilon */
        case 3: return ex;                                             /* j_x */
        case 4: return (5.0 * e2 - 9.0) * ex;                          /* q_x */
        case 5: return ey;                                             /* j_y */
        case 6: return (5.0 * e2 - 9.0) * ey;                          /* q_y */
        case 7: return ez;                                             /* j_z */
        case 8: return (5.0 * e2 - 9.0) * ez;                          /* q_z */
        case 9: return 3.0 * ex * ex - e2;                             /* 3 p_xx */
        case 10: return (3.0 * e2 - 5.0) * (3.0 * ex * ex - e2);       /* 3 pi_xx */
        case 11: return ey * ey - ez * ez;                             /* p_ww */
        case 12: return (3.0 * e2 - 5.0) * (ey * ey - ez * ez);        /* pi_ww */
        case 13: return ex * ey;                                       /* p_xy */
        case 14: return ey * ez;                                       /* p_yz */
        case 15: return ex * ez;                                       /* p_xz */
        case 16: return (ey * ey - ez * ez) * ex;                      /* m_x */
        case 17: return (ez * ez - ex * ex) * ey;                      /* m_y */
        default: return (ex * ex - ey * ey) * ez;                      /* m_z */
    }
}

void orc_mrt_basis(double* m)
{
    tables_init();
    for (int k = 0; k < Q; ++k)
        for (int a = 0; a < Q; ++a) m[k * Q + a] = mrow(k, a);
}

/* Relaxation rate of moment k: the stress moments (and the conserved ones,
 * whose rate does not matter) at omega = 1/tau_e, the others at theirs. */
static double mrate(const orc_params* p, int k, double omega)
{
    switch (k) {
        case 1: return p->s_e;
        case 2: return p->s_eps;
        case 4: case 6: case 8: return p->s_q;
        case 10: case 12: return p->s_pi;
        case 16: case 17: case 18: return p->s_m;
        default: return omega;
    }
}

/* Smagorinsky constant at row y with the van Driest damping. */
static double cs_at(const orc_params* p, int y)
{
    if (!(p->vd_aplus > 0.0) || y < 0) return p->cs;
    int dy = y < p->ny - 1 - y ? y : p->ny - 1 - y;
    double d = (double)dy + p->y1;
    double ut = p->vd_utau > 0.0 ? p->vd_utau : sqrt(fabs(p->fx) * p->ny / 2.0);
    double nu0 = (p->tau0 - 0.5) / 3.0;
    return p->cs * (1.0 - exp(-(d * ut / nu0) / p->vd_aplus));
}

/* ------------------------------------------------------------ gathering */

/* A source of post-collision populations: either a stored array or the
 * analytic initial state (used to check single cells of huge grids). */
typedef struct {
    const orc_params* p;
    const double* fpost;  /* if non-NULL: [a][z][y][x] */
    /* analytic initial state */
    const double* profile;/* [y] streamwise velocity of the initial profile */
    double noise;
    uint64_t seed;
    /* or, if tab_cells is non-NULL: a table of cells (ascending indices
     * x + nx (y + ny z)) and their populations [k][a]; a lookup of a cell
     * that is not in it sets *missing */
    const int64_t* tab_cells;
    const double* tab_f;
    int64_t ntab;
    int* missing;
    /* wall nodes: their outputs [w][k][z][x] (p->wall_nodes) */
    const double* fw;
} src_t;

static int64_t cell_index(const orc_params* p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * (int64_t)z);
}

/* splitmix64 (Steele, Lea & Flood 2014): output k (k = 0, 1, ...) of the
 * generator whose state starts at seed. */
static uint64_t splitmix64_at(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double uniform01(uint64_t seed, uint64_t k)
{
    return (double)(splitmix64_at(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

/* Initial velocity of a cell: profile value times (1 + d0, d1, d2) with
 * d_i uniform in [-noise, noise), drawn from counter 3 * cell + i. */
static void initial_velocity(const src_t* s, int x, int y, int z, double u[3])
{
    uint64_t c = (uint64_t)cell_index(s->p, x, y, z);
    double up = s->profile[y];
    double d[3];
    for (int i = 0; i < 3; ++i) d[i] = s->noise * (2.0 * uniform01(s->seed, 3u * c + (uint64_t)i) - 1.0);
    u[0] = up * (1.0 + d[0]);
    u[1] = up * d[1];
    u[2] = up * d[2];
}

static double src_get(const src_t* s, int a, int x, int y, int z)
{
    if (s->tab_cells) {
        int64_t c = cell_index(s->p, x, y, z), lo = 0, hi = s->ntab;
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (s->tab_cells[mid] < c) lo = mid + 1; else hi = mid;
        }
        if (lo < s->ntab && s->tab_cells[lo] == c) return s->tab_f[Q * lo + a];
        *s->missing = 1;
        return NAN;
    }
    if (s->fpost) return s->fpost[(int64_t)a * ((int64_t)s->p->nx * s->p->ny * s->p->nz) + cell_index(s->p, x, y, z)];
    double u[3];
    initial_velocity(s, x, y, z, u);
    return feq(a, 1.0, u);
}

static int wrap(int i, int n) { return ((i % n) + n) % n; }

static int in_index(int wall, int a)
{
    for (int k = 0; k < 5; ++k)
        if (IN_W[wall][k] == a) return k;
    return -1;
}

/* Streaming by pull (Eq. 1) with the wall rules for links that cross a wall:
 * BB: the population returns on its own link (Eq. 3 in 3-D form);
 * WFB / free-slip: the wall-normal population is bounced back, the
 * diagonal ones are mirror images from the in-plane neighbour (Eq. 4 in
 * 3-D form; pairs 7-13, 14-8, 11-18, 17-12 as listed with Eq. 14).
 * Wall nodes: a population entering from the wall comes from the wall node
 * it left, x - e_a in the wall plane. */
static void gather(const src_t* s, int x, int y, int z, double f[Q])
{
    const orc_params* p = s->p;
    for (int a = 0; a < Q; ++a) {
        int sx = wrap(x - E[a][0], p->nx);
        int sy = y - E[a][1];
        int sz = wrap(z - E[a][2], p->nz);
        if (sy >= 0 && sy < p->ny) {
            f[a] = src_get(s, a, sx, sy, sz);
        } else if (p->wall_nodes) {
            int w = sy < 0 ? 0 : 1;
            f[a] = s->fw[(((int64_t)w * 5 + in_index(w, a)) * p->nz + sz) * p->nx + sx];
        } else if (p->bc == ORC_BB || (E[a][0] == 0 && E[a][2] == 0)) {
            f[a] = src_get(s, OPP[a], x, y, z);
        } else {
            f[a] = src_get(s, MIR[a], sx, y, sz);
        }
    }
}

static int wall_of_row(const orc_params* p, int y)
{
    if (y == 0) return 0;
    if (y == p->ny - 1) return 1;
    return -1;
}

/* Gather + WFB (when active) at one cell: the "pre-collision state". */
static int precollision(const src_t* s, int x, int y, int z, double f[Q], double rec[4], int32_t* iters)
{
    const orc_params* p = s->p;
    gather(s, x, y, z, f);
    if (rec) rec[0] = rec[1] = rec[2] = rec[3] = 0.0;
    if (iters) *iters = 0;
    int w = wall_of_row(p, y);
    if (p->bc == ORC_WFB && w >= 0 && !p->wall_nodes) {
        if (p->ny == 1) return ORC_E_ARG;
        return orc_wfb_cell(p, w, f, rec, iters);
    }
    return ORC_OK;
}

/* ----------------------------------------------------------- the object */

static int params_ok(const orc_params* p)
{
    if (p->nx < 1 || p->ny < 2 || p->nz < 1) return 0;
    if (!(p->tau0 > 0.5) || !(p->cs >= 0.0) || !(p->kappa > 0.0)) return 0;
    if (!isfinite(p->tau0) || !isfinite(p->cs) || !isfinite(p->kappa) || !isfinite(p->bconst)) return 0;
    if (!isfinite(p->fx) || !(p->y1 > 0.0) || !(p->newton_tol > 0.0) || p->newton_maxit < 1) return 0;
    if (p->bc < 0 || p->bc > 2 || p->stats_every < 0) return 0;
    if (p->wall_nodes < 0 || p->wall_nodes > 2) return 0;
    if (p->collision != ORC_BGK && p->collision != ORC_MRT) return 0;
    if (p->collision == ORC_MRT) {
        const double r[5] = {p->s_e, p->s_eps, p->s_q, p->s_pi, p->s_m};
        for (int i = 0; i < 5; ++i)
            if (!(r[i] > 0.0 && r[i] < 2.0)) return 0;
    }
    if (!isfinite(p->vd_aplus) || !isfinite(p->vd_utau)) return 0;
    return 1;
}

orc* orc_create(const orc_params* p)
{
    tables_init();
    if (!params_ok(p)) return NULL;
    orc* o = (orc*)calloc(1, sizeof(orc));
    if (!o) return NULL;
    o->p = *p;
    o->ncell = (int64_t)p->nx * p->ny * p->nz;
    o->fpost = (double*)calloc((size_t)(Q * o->ncell), sizeof(double));
    o->fnew = (double*)calloc((size_t)(Q * o->ncell), sizeof(double));
    o->stats = (double*)calloc((size_t)p->ny * 8, sizeof(double));
    int ok = o->fpost && o->fnew && o->stats;
    if (ok && p->wall_nodes) {
        size_t m = (size_t)2 * p->nx * p->nz;
        o->fw = (double*)calloc(m * 5, sizeof(double));
        o->fw_new = (double*)calloc(m * 5, sizeof(double));
        o->urec = (double*)calloc(m * 3, sizeof(double));
        o->urec_new = (double*)calloc(m * 3, sizeof(double));
        ok = o->fw && o->fw_new && o->urec && o->urec_new;
    }
    if (!ok) {
        free(o->fpost); free(o->fnew); free(o->stats);
        free(o->fw); free(o->fw_new); free(o->urec); free(o->urec_new); free(o);
        return NULL;
    }
    o->first_bad_step = -1;
    return o;
}

void orc_destroy(orc* o)
{
    if (!o) return;
    free(o->fpost);
    free(o->fnew);
    free(o->stats);
    free(o->fw);
    free(o->fw_new);
    free(o->urec);
    free(o->urec_new);
    free(o);
}

int orc_set_param_bc(orc* o, int32_t bc)
{
    if (bc < 0 || bc > 2) return ORC_E_ARG;
    o->p.bc = bc;
    return ORC_OK;
}

/* The wall-node collision of one step for every wall node W = (x, z) of
 * both walls: the populations the first layer sent towards W on the
 * previous step (o->fpost, taken from the cells x - e_b in the wall plane)
 * collide by orc_wall_node_collide with the stress of Eq. 15-17 from the
 * first layer's density and velocity at W's column in urec (those of the
 * previous step, or of this step with wall_nodes = 2); the five outputs
 * that stream into the fluid go to fw_out.  Returns ORC_E_NEWTON if a
 * Newton solve fails. */
static int wall_node_update(const orc* o, const double* urec, double* fw_out, int32_t* maxit)
{
    const orc_params* p = &o->p;
    int bad = 0;
    int32_t mx = 0;
    for (int w = 0; w < 2; ++w) {
        int y = (w == 0) ? 0 : p->ny - 1;
        for (int z = 0; z < p->nz; ++z)
            for (int x = 0; x < p->nx; ++x) {
                double f[Q], out[Q], rec[4] = {0.0, 0.0, 0.0, 0.0};
                for (int b = 0; b < Q; ++b) {
                    f[b] = 0.0;   /* populations that never reach the fluid are not tracked */
                    if ((w == 0 && E[b][1] == -1) || (w == 1 && E[b][1] == 1)) {
                        int sx = wrap(x - E[b][0], p->nx), sz = wrap(z - E[b][2], p->nz);
                        f[b] = o->fpost[(int64_t)b * o->ncell + cell_index(p, sx, y, sz)];
                    }
                }
                const double* u = urec + 3 * (((int64_t)w * p->nz + z) * p->nx + x);
                int32_t it = 0;
                if (p->bc == ORC_WFB && orc_wall_tau(p, u[0], u[1], u[2], rec, &it) != ORC_OK) bad = 1;
                if (it > mx) mx = it;
                orc_wall_node_collide(p, w, f, rec[0], rec[1], out);
                for (int k = 0; k < 5; ++k)
                    fw_out[(((int64_t)w * 5 + k) * p->nz + z) * p->nx + x] = out[IN_W[w][k]];
            }
    }
    if (maxit && mx > *maxit) *maxit = mx;
    return bad ? ORC_E_NEWTON : ORC_OK;
}

/* Wall nodes at a state set from outside (initial state, orc_set_state):
 * the first layer's density and velocity are the plain moments of its
 * post-collision populations, and the wall nodes hold what they would send
 * had the state also been the previous step's (one wall-node collision of
 * the given populations with that stress). */
static int wall_node_start(orc* o)
{
    const orc_params* p = &o->p;
    if (!p->wall_nodes) return ORC_OK;
    for (int w = 0; w < 2; ++w) {
        int y = (w == 0) ? 0 : p->ny - 1;
        for (int z = 0; z < p->nz; ++z)
            for (int x = 0; x < p->nx; ++x) {
                int64_t c = cell_index(p, x, y, z);
                double r = 0.0, jx = 0.0, jz = 0.0;
                for (int a = 0; a < Q; ++a) {
                    double v = o->fpost[(int64_t)a * o->ncell + c];
                    r += v;
                    jx += E[a][0] * v;
                    jz += E[a][2] * v;
                }
                double* u = o->urec + 3 * (((int64_t)w * p->nz + z) * p->nx + x);
                u[0] = r; u[1] = jx / r; u[2] = jz / r;
            }
    }
    return wall_node_update(o, o->urec, o->fw, NULL);
}

void orc_set_state(orc* o, const double* fpost)
{
    memcpy(o->fpost, fpost, sizeof(double) * Q * o->ncell);
    o->status = wall_node_start(o);
}
void orc_get_state(const orc* o, double* fpost) { memcpy(fpost, o->fpost, sizeof(double) * Q * o->ncell); }
int64_t orc_steps(const orc* o) { return o->steps; }
int32_t orc_max_newton_iters(const orc* o) { return o->max_newton_iters; }
int64_t orc_first_bad_step(const orc* o) { return o->first_bad_step; }

/* Streamwise velocity of the initial profile per layer: Spalding's law at
 * distance d_y = min(y, ny - 1 - y) + y1 from the nearer wall. */
static void initial_profile(const orc_params* p, double u_tau, double* prof)
{
    double nu0 = (p->tau0 - 0.5) / 3.0;
    for (int y = 0; y < p->ny; ++y) {
        int dy = y < p->ny - 1 - y ? y : p->ny - 1 - y;
        double d = (double)dy + p->y1;
        prof[y] = u_tau * orc_spalding_uplus(d * u_tau / nu0, p->kappa, p->bconst);
    }
}

void orc_initial_profile(const orc_params* p, double u_tau, double* prof) { initial_profile(p, u_tau, prof); }

/* fpost(0) = f_eq(1, u0): Spalding profile plus seeded uniform noise. */
int orc_init_spalding(orc* o, double u_tau, double noise, uint64_t seed)
{
    const orc_params* p = &o->p;
    double* prof = (double*)malloc(sizeof(double) * p->ny);
    if (!prof) return ORC_E_ARG;
    initial_profile(p, u_tau, prof);
    src_t s = {p, NULL, prof, noise, seed, NULL, NULL, 0, NULL, NULL};
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t c = cell_index(p, x, y, z);
                double u[3];
                initial_velocity(&s, x, y, z, u);
                for (int a = 0; a < Q; ++a) o->fpost[(int64_t)a * o->ncell + c] = feq(a, 1.0, u);
            }
    free(prof);
    o->steps = 0;
    o->status = wall_node_start(o);
    o->first_bad_step = -1;
    return o->status;
}

/* Full update of one cell from a source of post-collision populations. */
static int cell_update(const src_t* s, int x, int y, int z, double out[Q], double mom[4], int32_t* iters)
{
    double f[Q];
    int st = precollision(s, x, y, z, f, NULL, iters);
    if (st != ORC_OK) return st;
    double rho, u[3];
    moments(f, s->p->fx, &rho, u);
    if (mom) { mom[0] = rho; mom[1] = u[0]; mom[2] = u[1]; mom[3] = u[2]; }
    if (!(rho > 0.0) || !isfinite(rho)) return ORC_E_NONFINITE;
    orc_collide_cell_at(s->p, y, f, out, NULL);
    return ORC_OK;
}

int orc_step(orc* o, int64_t n)
{
    const orc_params* p = &o->p;
    const int64_t nc = o->ncell;
    for (int64_t t = 0; t < n; ++t) {
        const int64_t step = o->steps + 1;
        const int sample = p->stats_every > 0 && (step % p->stats_every) == 0;
        src_t s = {p, o->fpost, NULL, 0.0, 0, NULL, NULL, 0, NULL, o->fw};
        int bad = 0;
        int32_t maxit = o->max_newton_iters;
        /* wall nodes: their collision of this step, of the populations the first
         * layer sent on the previous step, with the stress from the first
         * layer's velocity of the previous step (after the cells: of this step) */
        if (p->wall_nodes == 1 && wall_node_update(o, o->urec, o->fw_new, &maxit) != ORC_OK) bad |= 2;
        double* srow = NULL;
        if (sample) {
            srow = (double*)calloc((size_t)p->nz * p->ny * 7, sizeof(double));
            if (!srow) return ORC_E_ARG;
        }
#pragma omp parallel for schedule(static) reduction(| : bad) reduction(max : maxit)
        for (int z = 0; z < p->nz; ++z) {
            for (int y = 0; y < p->ny; ++y) {
                for (int x = 0; x < p->nx; ++x) {
                    double out[Q], mom[4];
                    int32_t it = 0;
                    int st = cell_update(&s, x, y, z, out, mom, &it);
                    if (it > maxit) maxit = it;
                    if (st != ORC_OK) {
                        bad |= (st == ORC_E_NEWTON) ? 2 : 1;
                        for (int a = 0; a < Q; ++a) out[a] = NAN;
                    }
                    int64_t c = cell_index(p, x, y, z);
                    for (int a = 0; a < Q; ++a) o->fnew[(int64_t)a * nc + c] = out[a];
                    if (p->wall_nodes && (y == 0 || y == p->ny - 1)) {
                        /* the first layer's density and velocity for the next wall-node collision */
                        double* u = o->urec_new + 3 * (((int64_t)(y == 0 ? 0 : 1) * p->nz + z) * p->nx + x);
                        u[0] = mom[0]; u[1] = mom[1]; u[2] = mom[3];
                    }
                    if (sample) {
                        double* r = srow + 7 * ((int64_t)z * p->ny + y);
                        r[0] += mom[1]; r[1] += mom[2]; r[2] += mom[3];
                        r[3] += mom[1] * mom[1]; r[4] += mom[2] * mom[2]; r[5] += mom[3] * mom[3];
                        r[6] += mom[1] * mom[2];
                    }
                }
            }
        }
        if (p->wall_nodes == 2 && wall_node_update(o, o->urec_new, o->fw_new, &maxit) != ORC_OK) bad |= 2;
        if (sample) {
            for (int y = 0; y < p->ny; ++y) {
                for (int z = 0; z < p->nz; ++z)
                    for (int k = 0; k < 7; ++k) o->stats[8 * y + k] += srow[7 * ((int64_t)z * p->ny + y) + k];
                o->stats[8 * y + 7] += (double)p->nx * p->nz;
            }
            o->nsamples += 1;
            free(srow);
        }
        o->max_newton_iters = maxit;
        double* tmp = o->fpost; o->fpost = o->fnew; o->fnew = tmp;
        if (p->wall_nodes) {
            tmp = o->fw; o->fw = o->fw_new; o->fw_new = tmp;
            tmp = o->urec; o->urec = o->urec_new; o->urec_new = tmp;
        }
        o->steps = step;
        if (bad) {
            if (o->first_bad_step < 0) o->first_bad_step = step;
            o->status = (bad & 2) ? ORC_E_NEWTON : ORC_E_NONFINITE;
            return o->status;
        }
    }
    return ORC_OK;
}

/* Observables of the current state (steps 1-3 applied to fpost, no write):
 * rho, ux, uy, uz per cell (any pointer may be NULL). */
int orc_observe(const orc* o, double* rho, double* ux, double* uy, double* uz)
{
    const orc_params* p = &o->p;
    src_t s = {p, o->fpost, NULL, 0.0, 0, NULL, NULL, 0, NULL, o->fw};
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double f[Q], r, u[3];
                if (precollision(&s, x, y, z, f, NULL, NULL) != ORC_OK) bad = 1;
                moments(f, p->fx, &r, u);
                int64_t c = cell_index(p, x, y, z);
                if (rho) rho[c] = r;
                if (ux) ux[c] = u[0];
                if (uy) uy[c] = u[1];
                if (uz) uz[c] = u[2];
            }
    return bad ? ORC_E_NEWTON : ORC_OK;
}

/* Wall records of the current state, layout [w][z][x] with w = 0 bottom,
 * 1 top.  WFB: tau_x, tau_z, u_tau, U of the WFB correction the next step
 * applies.  BB: force on the fluid by momentum exchange (the change of
 * momentum of the reflected populations), u_tau = sqrt(|tau| / rho).
 * Free-slip: zeros, U the tangential speed. */
int orc_wall(const orc* o, double* taux, double* tauz, double* utau, double* uu)
{
    const orc_params* p = &o->p;
    src_t s = {p, o->fpost, NULL, 0.0, 0, NULL, NULL, 0, NULL, o->fw};
    if (p->wall_nodes) {
        /* the stress from the first layer's latest density and velocity (WFB:
         * what the next wall-node collision applies, or with wall_nodes = 2 what
         * the latest one applied); bounce-back: the momentum
         * exchange of the populations the first layer sends towards the wall
         * node; free-slip: no stress */
        for (int w = 0; w < 2; ++w) {
            int y = (w == 0) ? 0 : p->ny - 1;
            for (int z = 0; z < p->nz; ++z)
                for (int x = 0; x < p->nx; ++x) {
                    int64_t k = (int64_t)w * p->nx * p->nz + (int64_t)z * p->nx + x;
                    const double* u = o->urec + 3 * k;
                    double rec[4] = {0.0, 0.0, 0.0, sqrt(u[1] * u[1] + u[2] * u[2])};
                    if (p->bc == ORC_WFB) {
                        if (orc_wall_tau(p, u[0], u[1], u[2], rec, NULL) != ORC_OK) return ORC_E_NEWTON;
                    } else if (p->bc == ORC_BB) {
                        double tx = 0.0, tz = 0.0;
                        for (int b = 0; b < Q; ++b) {
                            if (!((w == 0 && E[b][1] == -1) || (w == 1 && E[b][1] == 1))) continue;
                            int sx = wrap(x - E[b][0], p->nx), sz = wrap(z - E[b][2], p->nz);
                            double fb = o->fpost[(int64_t)b * o->ncell + cell_index(p, sx, y, sz)];
                            tx += -2.0 * E[b][0] * fb;
                            tz += -2.0 * E[b][2] * fb;
                        }
                        rec[0] = tx; rec[1] = tz;
                        rec[2] = sqrt(sqrt(tx * tx + tz * tz) / u[0]);
                    }
                    if (taux) taux[k] = rec[0];
                    if (tauz) tauz[k] = rec[1];
                    if (utau) utau[k] = rec[2];
                    if (uu) uu[k] = rec[3];
                }
        }
        return ORC_OK;
    }
    for (int w = 0; w < 2; ++w) {
        int y = (w == 0) ? 0 : p->ny - 1;
        for (int z = 0; z < p->nz; ++z)
            for (int x = 0; x < p->nx; ++x) {
                double f[Q], rec[4];
                int64_t k = (int64_t)w * p->nx * p->nz + (int64_t)z * p->nx + x;
                if (precollision(&s, x, y, z, f, rec, NULL) != ORC_OK) return ORC_E_NEWTON;
                double r, u[3];
                moments(f, p->fx, &r, u);
                if (p->bc == ORC_BB) {
                    /* every population leaving the cell through the wall comes back
                     * reversed: momentum change -2 e_b fpost_b */
                    double tx = 0.0, tz = 0.0;
                    int64_t c = cell_index(p, x, y, z);
                    for (int b = 0; b < Q; ++b) {
                        int dy = y + E[b][1];
                        if (dy >= 0 && dy < p->ny) continue;
                        double fb = o->fpost[(int64_t)b * o->ncell + c];
                        tx += -2.0 * E[b][0] * fb;
                        tz += -2.0 * E[b][2] * fb;
                    }
                    rec[0] = tx; rec[1] = tz;
                    rec[2] = sqrt(sqrt(tx * tx + tz * tz) / r);
                    rec[3] = sqrt(u[0] * u[0] + u[2] * u[2]);
                } else if (p->bc == ORC_FREESLIP) {
                    rec[0] = rec[1] = rec[2] = 0.0;
                    rec[3] = sqrt(u[0] * u[0] + u[2] * u[2]);
                }
                if (taux) taux[k] = rec[0];
                if (tauz) tauz[k] = rec[1];
                if (utau) utau[k] = rec[2];
                if (uu) uu[k] = rec[3];
            }
    }
    return ORC_OK;
}

/* Wall-node state: fw [2][5][nz][nx], the populations the wall nodes send
 * into the fluid at the next step, in the direction order of IN_W (bottom
 * 3, 7, 11, 14, 17; top 4, 13, 18, 8, 12); urec [2][nz][nx][3], the first
 * layer's rho, u_x, u_z of the latest step.  ORC_E_ARG without wall nodes. */
int orc_get_wall_nodes(const orc* o, double* fw, double* urec)
{
    if (!o->p.wall_nodes) return ORC_E_ARG;
    size_t m = (size_t)2 * o->p.nx * o->p.nz;
    if (fw) memcpy(fw, o->fw, sizeof(double) * 5 * m);
    if (urec) memcpy(urec, o->urec, sizeof(double) * 3 * m);
    return ORC_OK;
}

/* Sets the wall-node state (same layout as orc_get_wall_nodes), e.g. to
 * continue from another implementation's state after orc_set_state. */
int orc_set_wall_nodes(orc* o, const double* fw, const double* urec)
{
    if (!o->p.wall_nodes) return ORC_E_ARG;
    size_t m = (size_t)2 * o->p.nx * o->p.nz;
    if (fw) memcpy(o->fw, fw, sizeof(double) * 5 * m);
    if (urec) memcpy(o->urec, urec, sizeof(double) * 3 * m);
    return ORC_OK;
}

void orc_stats_sums(const orc* o, double* out, int64_t* nsamples)
{
    memcpy(out, o->stats, sizeof(double) * 8 * o->p.ny);
    if (nsamples) *nsamples = o->nsamples;
}

void orc_stats_reset(orc* o)
{
    memset(o->stats, 0, sizeof(double) * 8 * o->p.ny);
    o->nsamples = 0;
}

/* --------------------------------------- single cells of the initial state */

/* Initial state, one step and observables at selected cells of a grid too
 * large to hold twice, computed from the analytic initial state. */
int orc_init_cells(const orc_params* p, double u_tau, double noise, uint64_t seed,
                   int64_t n, const int64_t* cells, double* fpost_out /* [n][19] */)
{
    tables_init();
    if (!params_ok(p) || p->wall_nodes) return ORC_E_ARG;
    double* prof = (double*)malloc(sizeof(double) * p->ny);
    if (!prof) return ORC_E_ARG;
    initial_profile(p, u_tau, prof);
    src_t s = {p, NULL, prof, noise, seed, NULL, NULL, 0, NULL, NULL};
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = cells[i];
        int x = (int)(c % p->nx), y = (int)((c / p->nx) % p->ny), z = (int)(c / ((int64_t)p->nx * p->ny));
        for (int a = 0; a < Q; ++a) fpost_out[Q * i + a] = src_get(&s, a, x, y, z);
    }
    free(prof);
    return ORC_OK;
}

int orc_step1_cells(const orc_params* p, double u_tau, double noise, uint64_t seed,
                    int64_t n, const int64_t* cells, double* fpost_out /* [n][19] */,
                    double* mom_out /* [n][4]: observables of the initial state */)
{
    tables_init();
    if (!params_ok(p) || p->wall_nodes) return ORC_E_ARG;
    double* prof = (double*)malloc(sizeof(double) * p->ny);
    if (!prof) return ORC_E_ARG;
    initial_profile(p, u_tau, prof);
    src_t s = {p, NULL, prof, noise, seed, NULL, NULL, 0, NULL, NULL};
    int st = ORC_OK;
    for (int64_t i = 0; i < n && st == ORC_OK; ++i) {
        int64_t c = cells[i];
        int x = (int)(c % p->nx), y = (int)((c / p->nx) % p->ny), z = (int)(c / ((int64_t)p->nx * p->ny));
        st = cell_update(&s, x, y, z, fpost_out + Q * i, mom_out ? mom_out + 4 * i : NULL, NULL);
    }
    free(prof);
    return st;
}

/* One step at selected cells from a table of post-collision populations of
 * the cells around them (any cells, ascending indices; e.g. the 3 x 3 x 3
 * neighbourhoods of the selected cells): the same update as orc_step, for
 * checking single cells of grids too large for the oracle's arrays.
 * Returns ORC_E_ARG if the gather needs a cell that is not in the table. */
int orc_step_cells_table(const orc_params* p, int64_t ntab, const int64_t* tab_cells, const double* tab_f,
                         int64_t n, const int64_t* cells, double* fpost_out /* [n][19] */,
                         double* mom_out /* [n][4]: observables of the table's state, may be NULL */)
{
    tables_init();
    if (!params_ok(p) || p->wall_nodes) return ORC_E_ARG;
    for (int64_t k = 1; k < ntab; ++k)
        if (tab_cells[k] <= tab_cells[k - 1]) return ORC_E_ARG;
    int missing = 0;
    src_t s = {p, NULL, NULL, 0.0, 0, tab_cells, tab_f, ntab, &missing, NULL};
    int st = ORC_OK;
    for (int64_t i = 0; i < n && st == ORC_OK; ++i) {
        int64_t c = cells[i];
        int x = (int)(c % p->nx), y = (int)((c / p->nx) % p->ny), z = (int)(c / ((int64_t)p->nx * p->ny));
        st = cell_update(&s, x, y, z, fpost_out + Q * i, mom_out ? mom_out + 4 * i : NULL, NULL);
        if (missing) st = ORC_E_ARG;
    }
    return st;
}
