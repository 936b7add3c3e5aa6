/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the double-MRT lattice Boltzmann
 * method for natural convection in a differentially heated cubic cavity
 * (Li, Yang & Zhang, arXiv:1511.04633).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker that the
 * GPU library is compared against.  Only the test suite, the package smoke
 * check and the CPU-baseline leg of the benchmark may load it; the GPU
 * library never links, includes or calls it, and it shares no code, table or
 * header with that library.
 *
 * It is written to be read against the paper, not to be fast:
 *   - the D3Q19 velocity set, weights and transform matrix M are typed in
 *     from Eqs. (12), (18) and (21); M^-1 is obtained by Gauss-Jordan
 *     elimination at start-up, never from an orthogonality shortcut;
 *   - the collision is the dense matrix form of Eq. (19), the force term is
 *     Eq. (15) with Eq. (17), added after the collision as Eq. (14) reads;
 *   - the energy lattice is Eqs. (28)-(37): dense N, n^eq, and Q obtained by
 *     inverting the Q^-1 of Eq. (35);
 *   - streaming is push-style: every post-collision population moves to its
 *     neighbour, or is reflected at the wall it would cross.
 *
 * Readings of points the paper leaves open, silent or garbled:
 *   R1  row 14 of M (Eq. 21) is misprinted; the oracle uses p_xy = e_x e_y,
 *       i.e. (+1,-1,-1,+1) on directions 8..11 (Eq. 22 names that moment).
 *   R3  the "/p" of Eq. (15) is read as division by c_s^2 with the density
 *       carried by f^eq, so that sum_i F_i = 0 and sum_i e_i F_i = rho G.
 *   R5  Eq. (20): rho V = sum_i e_i f_i.
 *   R6  T_l is the mean wall temperature: theta_ref = 0 for theta_h = +1/2,
 *       theta_c = -1/2.
 *   R7  gravity points along -z (Eq. 4), so G = (0, 0, g beta (theta - theta_ref)).
 *   R9  nodes sit at cell centres (i + 1/2); walls lie half way between the
 *       outermost nodes and the (virtual) outside nodes; H = N.
 *   R10 thermal walls: Dirichlet walls use the half-way anti-bounce-back
 *       g_ibar = -g*_i + 2 w_T,ibar theta_W, adiabatic walls plain bounce-back.
 *   R11 theta_W on a linear wall is taken at the wall point the link crosses,
 *       whose y equals the node's y = j + 1/2 (Eqs. 9-10 with y/H = (j+1/2)/N).
 *   R12 any D3Q19 link leaving the cube, through a face, edge or corner, is
 *       reflected at its own node (half-way bounce-back, walls at rest, Eq. 8).
 *   R14 the force uses theta(t) and the energy equilibrium uses V(t) of the
 *       same node (same-time coupling).
 *   R15 Eq. (17) (with rho) is the f^eq inside the force; Eq. (24) (with
 *       rho_0 = 1) gives the equilibrium moments of the collision.
 *   R16 isotropic diffusion: tau_xx = tau_yy = tau_zz = 1/2 + 4 alpha (Eq. 36,
 *       epsilon = 1/4, D = alpha I), off-diagonals 0, tau_1 = tau_5 = tau_6 =
 *       tau_7 = 1 (end of Sec. 3.2).
 *   R17 Nu of Eq. (39): second-order one-sided difference through the wall
 *       value and the first two nodes, dtheta/dy|_0 = (9 th_0 - th_1 - 8 th_w)/3.
 *   R18 Nu_2D (Eq. 41) on the X = 0.5 line: the centre column for odd N, the
 *       mean of the two central columns for even N; Nu_max without interpolation.
 *
 * Variants beyond the paper's own choices (ablations of the readings above):
 *   force model 1: the other reading of Eq. (15), division by rho c_s^2, so that
 *       sum_i e_i F_i = G (force density G instead of rho G);
 *   force model 2: Guo-type forcing written in moment space (Guo, Zheng & Shi,
 *       Phys. Rev. E 65, 046308 (2002), in its MRT form): V = (sum_i e_i f_i +
 *       rho G / 2) / rho, m^eq of Eq. (24) with j = rho V, and
 *       M^-1 (I - S/2) M Fbar added, Fbar_i = w_i rho [3 (e_i - V) + 9 (e_i . V) e_i] . G;
 *       the energy equilibrium and the reported velocity use the same V;
 *   anisotropic diffusion: D = alpha A for a symmetric positive definite A,
 *       the full tau-bar block of Eq. (35) from Eq. (36);
 *   Nu stencils: 0 = R17; 1 = first order, dtheta/dy|_0 = 2 (th_0 - th_w);
 *       2 = energy flux of the wall links, q = g_in - g*_out through the hot
 *       wall, Nu = H q / D_yy (the conductive flux that crosses the wall).
 *
 * A fully periodic mode (wall_type 0) exists only here, for the transport
 * coefficient checks (decay of a shear wave and of a temperature sine mode).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q19 19
#define Q7 7

/* Eq. (12): D3Q19 velocities, columns i = 1..19 in the paper's order. */
static const int E19[Q19][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, 1, 0}, {1, -1, 0}, {-1, -1, 0},
    {1, 0, 1},  {-1, 0, 1}, {1, 0, -1}, {-1, 0, -1},
    {0, 1, 1},  {0, -1, 1}, {0, 1, -1}, {0, -1, -1}};

/* Eq. (18): D3Q19 weights. */
static const double W19[Q19] = {
    1.0 / 3,
    1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* Eq. (21): transform matrix M.  Row 14 (p_xy) carries the correction of
 * reading R1; every other row is as printed. */
static const double M19[Q19][Q19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-30, -11, -11, -11, -11, -11, -11, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8, 8},
    {12, -4, -4, -4, -4, -4, -4, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, -4, 4, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, -4, 4, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, -4, 4, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, -4, -4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, -2, -2, 2, 2, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0}, /* R1 */
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, -1, -1, 1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1}};

/* Eq. (28): D3Q7 velocities. */
static const int E7[Q7][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Eq. (31): D3Q7 weights. */
static const double W7[Q7] = {1.0 / 4, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8};

/* Eq. (32): transform matrix N. */
static const double N7[Q7][Q7] = {
    {1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0},
    {0, 0, 0, 0, 0, 1, -1},
    {6, -1, -1, -1, -1, -1, -1},
    {0, 2, 2, -1, -1, -1, -1},
    {0, 0, 0, 1, 1, -1, -1}};

/* Eq. (34): a = 7 w_T,1 - 1. */
#define A_THERMAL (7.0 * (1.0 / 4) - 1.0)
/* Eq. (13) with c = 1. */
#define CS2 (1.0 / 3.0)
/* Eq. (36): epsilon = 1/4 in three dimensions. */
#define EPS_T 0.25

typedef struct oracle {
    int n, wall_type;
    int force_model;           /* 0, 1, 2: see the header */
    double tau_wall;           /* tau-bar_yy of Q^-1, for the wall-flux Nu */
    double theta_hot, theta_cold, theta_ref;
    double gbeta;              /* g beta per unit theta, lattice units */
    double u_c, nu, alpha, s_nu, tau_t;
    double s[Q19];             /* diagonal of S, Eq. (23) */
    double minv[Q19][Q19];     /* M^-1 */
    double ninv[Q7][Q7];       /* N^-1 */
    double qmat[Q7][Q7];       /* Q = (Q^-1)^-1, Eq. (35) */
    double *f, *g;             /* state at time t (pre-collision), [i][cell] */
    double *fp, *gp;           /* post-collision scratch */
    long t;
} oracle;

static int opposite19(int i)
{
    for (int k = 0; k < Q19; ++k)
        if (E19[k][0] == -E19[i][0] && E19[k][1] == -E19[i][1] && E19[k][2] == -E19[i][2])
            return k;
    return -1;
}

static int opposite7(int i)
{
    for (int k = 0; k < Q7; ++k)
        if (E7[k][0] == -E7[i][0] && E7[k][1] == -E7[i][1] && E7[k][2] == -E7[i][2])
            return k;
    return -1;
}

/* Gauss-Jordan elimination with partial pivoting; a (n x n) is destroyed.
 * Returns 0 on success, -1 if singular. */
static int invert(int n, double *a, double *inv)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            inv[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r * n + c]) > fabs(a[piv * n + c]))
                piv = r;
        if (fabs(a[piv * n + c]) < 1e-300)
            return -1;
        if (piv != c) {
            for (int j = 0; j < n; ++j) {
                double t = a[c * n + j]; a[c * n + j] = a[piv * n + j]; a[piv * n + j] = t;
                t = inv[c * n + j]; inv[c * n + j] = inv[piv * n + j]; inv[piv * n + j] = t;
            }
        }
        double d = a[c * n + c];
        for (int j = 0; j < n; ++j) {
            a[c * n + j] /= d;
            inv[c * n + j] /= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c)
                continue;
            double m = a[r * n + c];
            if (m == 0.0)
                continue;
            for (int j = 0; j < n; ++j) {
                a[r * n + j] -= m * a[c * n + j];
                inv[r * n + j] -= m * inv[c * n + j];
            }
        }
    }
    return 0;
}

/* Sec. 4, Eq. (38) with Ma = u_c / c_s, Eq. (26) and Eq. (36).
 * out = {u_c, gbeta, nu, alpha, s_nu, tau_t}. */
void oracle_derive(int n, double ra, double pr, double ma, double *out)
{
    double u_c = ma * sqrt(CS2);              /* Ma = u_c / c_s            */
    double gbeta = u_c * u_c / n;             /* u_c^2 = g beta dT H, dT=1 */
    double nu = u_c * n * sqrt(pr / ra);      /* Ra = g beta dT H^3 Pr/nu^2 */
    double alpha = nu / pr;                   /* Pr = nu / alpha           */
    out[0] = u_c;
    out[1] = gbeta;
    out[2] = nu;
    out[3] = alpha;
    out[4] = 1.0 / (3.0 * nu + 0.5);          /* Eq. (26)                  */
    out[5] = 0.5 + alpha / EPS_T;             /* Eq. (36), dt = dx = 1     */
}

void oracle_matrices(double *m, double *minv, double *nmat, double *ninv)
{
    double a[Q19 * Q19], b[Q7 * Q7];
    for (int k = 0; k < Q19; ++k)
        for (int i = 0; i < Q19; ++i) {
            a[k * Q19 + i] = M19[k][i];
            if (m)
                m[k * Q19 + i] = M19[k][i];
        }
    double tmp[Q19 * Q19];
    invert(Q19, a, tmp);
    if (minv)
        memcpy(minv, tmp, sizeof(tmp));
    for (int k = 0; k < Q7; ++k)
        for (int i = 0; i < Q7; ++i) {
            b[k * Q7 + i] = N7[k][i];
            if (nmat)
                nmat[k * Q7 + i] = N7[k][i];
        }
    double tmp7[Q7 * Q7];
    invert(Q7, b, tmp7);
    if (ninv)
        memcpy(ninv, tmp7, sizeof(tmp7));
}

void oracle_velocities(int *e19, double *w19, int *e7, double *w7)
{
    for (int i = 0; i < Q19; ++i) {
        for (int d = 0; d < 3; ++d)
            if (e19) e19[i * 3 + d] = E19[i][d];
        if (w19) w19[i] = W19[i];
    }
    for (int i = 0; i < Q7; ++i) {
        for (int d = 0; d < 3; ++d)
            if (e7) e7[i * 3 + d] = E7[i][d];
        if (w7) w7[i] = W7[i];
    }
}

/* Eq. (24), with rho_0 = 1 (the mean density, Sec. 3.1). */
void oracle_meq(double rho, double jx, double jy, double jz, double *meq)
{
    const double rho0 = 1.0;
    double jj = jx * jx + jy * jy + jz * jz;
    meq[0] = rho;
    meq[1] = -11.0 * rho + 19.0 * jj / rho0;
    meq[2] = 3.0 * rho - 5.5 * jj / rho0;
    meq[3] = jx;
    meq[4] = -2.0 / 3.0 * jx;
    meq[5] = jy;
    meq[6] = -2.0 / 3.0 * jy;
    meq[7] = jz;
    meq[8] = -2.0 / 3.0 * jz;
    meq[9] = (2.0 * jx * jx - (jy * jy + jz * jz)) / rho0;
    meq[10] = -0.5 * (2.0 * jx * jx - (jy * jy + jz * jz)) / rho0;
    meq[11] = (jy * jy - jz * jz) / rho0;
    meq[12] = -0.5 * (jy * jy - jz * jz) / rho0;
    meq[13] = jx * jy / rho0;
    meq[14] = jy * jz / rho0;
    meq[15] = jx * jz / rho0;
    meq[16] = 0.0;
    meq[17] = 0.0;
    meq[18] = 0.0;
}

/* Eq. (17). */
void oracle_feq(double rho, const double *v, double *feq)
{
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    for (int i = 0; i < Q19; ++i) {
        double ev = E19[i][0] * v[0] + E19[i][1] * v[1] + E19[i][2] * v[2];
        feq[i] = rho * W19[i] *
                 (1.0 + ev / CS2 + ev * ev / (2.0 * CS2 * CS2) - vv / (2.0 * CS2));
    }
}

/* Eq. (33): equilibrium moments of the energy populations. */
static void thermal_neq(double theta, const double *v, double *neq)
{
    neq[0] = theta;
    neq[1] = v[0] * theta;
    neq[2] = v[1] * theta;
    neq[3] = v[2] * theta;
    neq[4] = A_THERMAL * theta;
    neq[5] = 0.0;
    neq[6] = 0.0;
}

/* The energy populations whose moments are n^eq of Eq. (33): N^-1 n^eq. */
void oracle_geq(double theta, const double *v, double *geq)
{
    double ninv[Q7 * Q7], neq[Q7];
    oracle_matrices(NULL, NULL, NULL, ninv);
    thermal_neq(theta, v, neq);
    for (int i = 0; i < Q7; ++i) {
        geq[i] = 0.0;
        for (int k = 0; k < Q7; ++k)
            geq[i] += ninv[i * Q7 + k] * neq[k];
    }
}

/* Eq. (15) under reading R3, with G = (0, 0, gz) (Eq. 16, reading R7), dt = 1. */
void oracle_force(double rho, const double *v, double gz, double *force)
{
    double feq[Q19];
    oracle_feq(rho, v, feq);
    const double gvec[3] = {0.0, 0.0, gz};
    for (int i = 0; i < Q19; ++i) {
        double gdot = 0.0;
        for (int d = 0; d < 3; ++d)
            gdot += gvec[d] * (E19[i][d] - v[d]);
        force[i] = gdot / CS2 * feq[i];
    }
}

/* Guo's forcing term (force model 2): Fbar_i = w_i rho [3 (e_i - V) + 9 (e_i . V) e_i] . G,
 * G = (0, 0, gz); c_s^2 = 1/3. */
void oracle_guo_force(double rho, const double *v, double gz, double *fbar)
{
    const double gvec[3] = {0.0, 0.0, gz};
    for (int i = 0; i < Q19; ++i) {
        double ev = 0.0, t = 0.0;
        for (int d = 0; d < 3; ++d)
            ev += E19[i][d] * v[d];
        for (int d = 0; d < 3; ++d)
            t += ((E19[i][d] - v[d]) / CS2 + ev * E19[i][d] / (CS2 * CS2)) * gvec[d];
        fbar[i] = W19[i] * rho * t;
    }
}

/* One node's collision: Eqs. (19)-(20), (14)-(17) for f; Eqs. (29)-(35) for g. */
static void collide_node(const oracle *o, const double *f, const double *g,
                         double *fo, double *go)
{
    /* Eq. (20), reading R5: density and momentum. */
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q19; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d)
            j[d] += E19[i][d] * f[i];
    }
    /* Eq. (30): temperature; Eq. (16): buoyancy along +z (reading R7). */
    double theta = 0.0;
    for (int i = 0; i < Q7; ++i)
        theta += g[i];
    const double gz = o->gbeta * (theta - o->theta_ref);
    /* Momentum of the equilibrium: j itself, or j + rho G / 2 (force model 2). */
    double jeq[3] = {j[0], j[1], j[2]};
    if (o->force_model == 2)
        jeq[2] += 0.5 * rho * gz;
    double v[3] = {jeq[0] / rho, jeq[1] / rho, jeq[2] / rho};

    /* Eq. (20): m = M f;  Eq. (24): m^eq;  Eq. (19): Omega = -M^-1 S (m - m^eq). */
    double m[Q19], meq[Q19], dm[Q19];
    for (int k = 0; k < Q19; ++k) {
        m[k] = 0.0;
        for (int i = 0; i < Q19; ++i)
            m[k] += M19[k][i] * f[i];
    }
    oracle_meq(rho, jeq[0], jeq[1], jeq[2], meq);
    for (int k = 0; k < Q19; ++k)
        dm[k] = o->s[k] * (m[k] - meq[k]);

    double force[Q19];
    if (o->force_model == 2) {
        /* Guo: the source (I - S/2) M Fbar joins the moment-space update. */
        double fbar[Q19], mf[Q19];
        oracle_guo_force(rho, v, gz, fbar);
        for (int k = 0; k < Q19; ++k) {
            mf[k] = 0.0;
            for (int i = 0; i < Q19; ++i)
                mf[k] += M19[k][i] * fbar[i];
            dm[k] -= (1.0 - 0.5 * o->s[k]) * mf[k];
        }
        for (int i = 0; i < Q19; ++i)
            force[i] = 0.0;
    } else {
        /* Eqs. (15)-(17); force model 1 divides by rho as well. */
        oracle_force(rho, v, gz, force);
        if (o->force_model == 1)
            for (int i = 0; i < Q19; ++i)
                force[i] /= rho;
    }

    /* Eq. (14): post-collision value f + Omega + F. */
    for (int i = 0; i < Q19; ++i) {
        double omega = 0.0;
        for (int k = 0; k < Q19; ++k)
            omega -= o->minv[i][k] * dm[k];
        fo[i] = f[i] + omega + force[i];
    }

    /* Eq. (30): n = N g;  Eq. (33): n^eq;  Eq. (29): -N^-1 Q (n - n^eq). */
    double n[Q7], neq[Q7], dn[Q7];
    for (int k = 0; k < Q7; ++k) {
        n[k] = 0.0;
        for (int i = 0; i < Q7; ++i)
            n[k] += N7[k][i] * g[i];
    }
    thermal_neq(theta, v, neq);
    for (int k = 0; k < Q7; ++k) {
        dn[k] = 0.0;
        for (int l = 0; l < Q7; ++l)
            dn[k] += o->qmat[k][l] * (n[l] - neq[l]);
    }
    for (int i = 0; i < Q7; ++i) {
        double om = 0.0;
        for (int k = 0; k < Q7; ++k)
            om -= o->ninv[i][k] * dn[k];
        go[i] = g[i] + om;
    }
}

void oracle_collide_node(const oracle *o, const double *f, const double *g, double *fo, double *go)
{
    collide_node(o, f, g, fo, go);
}

/* Eq. (9)-(10): wall temperature of a linear wall at node height j. */
static double theta_linear(const oracle *o, int y)
{
    return o->theta_hot + (o->theta_cold - o->theta_hot) * (y + 0.5) / o->n;
}

/* Thermal condition of the wall crossed by a D3Q7 link leaving node (x,y,z)
 * along axis `axis` towards side `side` (+1 high, -1 low).  Returns 1 and sets
 * *theta_w for a Dirichlet wall, 0 for an adiabatic wall.  Eqs. (6)-(7), (9), (10). */
static int thermal_wall(const oracle *o, int axis, int side, int y, double *theta_w)
{
    if (axis == 1) { /* y = 0 hot, y = H cold: Eqs. (6)-(7) */
        *theta_w = side < 0 ? o->theta_hot : o->theta_cold;
        return 1;
    }
    if (o->wall_type == 1) /* Type 1: the four other walls adiabatic */
        return 0;
    if (axis == 0 || o->wall_type == 2) { /* Eq. (9); Eq. (10) for x walls */
        *theta_w = theta_linear(o, y);
        return 1;
    }
    return 0; /* Type 3, z walls: Eq. (10), adiabatic */
}

/* The parameter part of an oracle, without state arrays: enough for the
 * single-node step and the Nusselt numbers of a state held elsewhere. */
oracle *oracle_create_params(int n, int wall_type, double ra, double pr, double ma,
                             double theta_hot, double theta_cold, double theta_ref,
                             double buoyancy_scale, const double *s19, const double *tau7,
                             const double *aniso6, int force_model)
{
    if (n < 2 || wall_type < 0 || wall_type > 3 || ra <= 0 || pr <= 0 || ma <= 0 ||
        force_model < 0 || force_model > 2)
        return NULL;
    oracle *o = (oracle *)calloc(1, sizeof(oracle));
    if (!o)
        return NULL;
    o->n = n;
    o->wall_type = wall_type;
    o->force_model = force_model;
    o->theta_hot = theta_hot;
    o->theta_cold = theta_cold;
    o->theta_ref = theta_ref;
    double d[6];
    oracle_derive(n, ra, pr, ma, d);
    o->u_c = d[0];
    o->gbeta = d[1] * buoyancy_scale;
    o->nu = d[2];
    o->alpha = d[3];
    o->s_nu = d[4];
    o->tau_t = d[5];

    /* Eq. (26). */
    if (s19) {
        memcpy(o->s, s19, sizeof(o->s));
    } else {
        double s[Q19] = {1.0, 1.19, 1.4, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2, o->s_nu,
                         1.4, o->s_nu, 1.4, o->s_nu, o->s_nu, o->s_nu, 1.98, 1.98, 1.98};
        memcpy(o->s, s, sizeof(o->s));
    }
    double mi[Q19 * Q19], ni[Q7 * Q7];
    oracle_matrices(NULL, mi, NULL, ni);
    memcpy(o->minv, mi, sizeof(mi));
    memcpy(o->ninv, ni, sizeof(ni));

    /* Eq. (35) with reading R16; Q is the inverse of Q^-1.  With aniso6 =
     * (A_xx, A_yy, A_zz, A_xy, A_xz, A_yz), D = alpha A and the tau-bar block
     * of rows/columns 2..4 is Eq. (36): 1/2 delta_ij + D_ij / epsilon. */
    double qinv[Q7 * Q7], qm[Q7 * Q7];
    memset(qinv, 0, sizeof(qinv));
    double tau_default[Q7] = {1.0, o->tau_t, o->tau_t, o->tau_t, 1.0, 1.0, 1.0};
    for (int k = 0; k < Q7; ++k)
        qinv[k * Q7 + k] = tau7 ? tau7[k] : tau_default[k];
    if (aniso6) {
        const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
        for (int q = 0; q < 6; ++q) {
            double t = (ia[q] == ib[q] ? 0.5 : 0.0) + o->alpha * aniso6[q] / EPS_T;
            qinv[(1 + ia[q]) * Q7 + (1 + ib[q])] = t;
            qinv[(1 + ib[q]) * Q7 + (1 + ia[q])] = t;
        }
    }
    o->tau_wall = qinv[2 * Q7 + 2];
    if (invert(Q7, qinv, qm) != 0) {
        free(o);
        return NULL;
    }
    memcpy(o->qmat, qm, sizeof(qm));
    o->t = 0;
    return o;
}

oracle *oracle_create(int n, int wall_type, double ra, double pr, double ma,
                      double theta_hot, double theta_cold, double theta_ref,
                      double buoyancy_scale, const double *s19, const double *tau7,
                      const double *aniso6, int force_model, const double *theta0)
{
    oracle *o = oracle_create_params(n, wall_type, ra, pr, ma, theta_hot, theta_cold, theta_ref,
                                     buoyancy_scale, s19, tau7, aniso6, force_model);
    if (!o)
        return NULL;
    size_t cells = (size_t)n * n * n;
    o->f = (double *)malloc(sizeof(double) * Q19 * cells);
    o->fp = (double *)malloc(sizeof(double) * Q19 * cells);
    o->g = (double *)malloc(sizeof(double) * Q7 * cells);
    o->gp = (double *)malloc(sizeof(double) * Q7 * cells);
    if (!o->f || !o->fp || !o->g || !o->gp) {
        free(o->f); free(o->fp); free(o->g); free(o->gp); free(o);
        return NULL;
    }
    /* Initial state (the paper is silent, reading R13): fluid at rest with
     * rho = 1, f_i = w_i, and g_i = w_T,i theta0 (zero velocity). */
    for (size_t c = 0; c < cells; ++c) {
        for (int i = 0; i < Q19; ++i)
            o->f[i * cells + c] = W19[i];
        double th = theta0 ? theta0[c] : 0.0;
        for (int i = 0; i < Q7; ++i)
            o->g[i * cells + c] = W7[i] * th;
    }
    o->t = 0;
    return o;
}

void oracle_destroy(oracle *o)
{
    if (!o)
        return;
    free(o->f); free(o->fp); free(o->g); free(o->gp);
    free(o);
}

void oracle_derived_of(const oracle *o, double *out)
{
    out[0] = o->u_c; out[1] = o->gbeta; out[2] = o->nu;
    out[3] = o->alpha; out[4] = o->s_nu; out[5] = o->tau_t;
}

long oracle_time(const oracle *o) { return o->t; }

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One time step: collide every node (Eqs. 14, 19, 29), then stream every
 * post-collision population to its neighbour or reflect it at the wall. */
void oracle_step(oracle *o, long nsteps)
{
    const int n = o->n;
    const size_t cells = (size_t)n * n * n;
    for (long s = 0; s < nsteps; ++s) {
#pragma omp parallel for schedule(static)
        for (int z = 0; z < n; ++z) {
            double f[Q19], g[Q7], fo[Q19], go[Q7];
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    size_t c = (size_t)x + (size_t)n * (y + (size_t)n * z);
                    for (int i = 0; i < Q19; ++i) f[i] = o->f[i * cells + c];
                    for (int i = 0; i < Q7; ++i) g[i] = o->g[i * cells + c];
                    collide_node(o, f, g, fo, go);
                    for (int i = 0; i < Q19; ++i) o->fp[i * cells + c] = fo[i];
                    for (int i = 0; i < Q7; ++i) o->gp[i * cells + c] = go[i];
                }
        }
        /* Streaming.  Each destination slot receives exactly one value. */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < n; ++z)
            for (int y = 0; y < n; ++y)
                for (int x = 0; x < n; ++x) {
                    size_t c = (size_t)x + (size_t)n * (y + (size_t)n * z);
                    int pos[3] = {x, y, z};
                    for (int i = 0; i < Q19; ++i) {
                        int t[3], inside = 1;
                        for (int d = 0; d < 3; ++d) {
                            t[d] = pos[d] + E19[i][d];
                            if (o->wall_type == 0)
                                t[d] = (t[d] + n) % n;
                            else if (t[d] < 0 || t[d] >= n)
                                inside = 0;
                        }
                        double v = o->fp[i * cells + c];
                        if (inside) {
                            size_t tc = (size_t)t[0] + (size_t)n * (t[1] + (size_t)n * t[2]);
                            o->f[i * cells + tc] = v;
                        } else {
                            /* Half-way bounce-back at a wall at rest (Eq. 8, R12). */
                            o->f[opposite19(i) * cells + c] = v;
                        }
                    }
                    for (int i = 0; i < Q7; ++i) {
                        int t[3], inside = 1, axis = -1, side = 0;
                        for (int d = 0; d < 3; ++d) {
                            t[d] = pos[d] + E7[i][d];
                            if (o->wall_type == 0)
                                t[d] = (t[d] + n) % n;
                            else if (t[d] < 0 || t[d] >= n) {
                                inside = 0;
                                axis = d;
                                side = E7[i][d];
                            }
                        }
                        double v = o->gp[i * cells + c];
                        if (inside) {
                            size_t tc = (size_t)t[0] + (size_t)n * (t[1] + (size_t)n * t[2]);
                            o->g[i * cells + tc] = v;
                        } else {
                            int ib = opposite7(i);
                            double tw;
                            if (thermal_wall(o, axis, side, y, &tw))
                                o->g[ib * cells + c] = -v + 2.0 * W7[ib] * tw; /* R10 */
                            else
                                o->g[ib * cells + c] = v;                     /* R10 */
                        }
                    }
                }
        o->t += 1;
    }
}

/* Macroscopic fields of the current state: Eqs. (20), (25), (30) (with the
 * half-force velocity of force model 2).  Arrays hold n^3 values, x fastest;
 * any pointer may be NULL. */
void oracle_macro(const oracle *o, double *rho, double *ux, double *uy, double *uz, double *theta)
{
    const int n = o->n;
    const size_t cells = (size_t)n * n * n;
    for (size_t c = 0; c < cells; ++c) {
        double r = 0.0, j[3] = {0.0, 0.0, 0.0}, th = 0.0;
        for (int i = 0; i < Q19; ++i) {
            double fi = o->f[i * cells + c];
            r += fi;
            for (int d = 0; d < 3; ++d)
                j[d] += E19[i][d] * fi;
        }
        for (int i = 0; i < Q7; ++i)
            th += o->g[i * cells + c];
        if (o->force_model == 2) /* V = (j + rho G / 2) / rho */
            j[2] += 0.5 * r * o->gbeta * (th - o->theta_ref);
        if (rho) rho[c] = r;
        if (ux) ux[c] = j[0] / r;
        if (uy) uy[c] = j[1] / r;
        if (uz) uz[c] = j[2] / r;
        if (theta) theta[c] = th;
    }
}

/* Hot-wall Nusselt numbers, Eqs. (39)-(41) with readings R17, R18 and the
 * stencil choice of the header (theta_h - theta_c = 1, as in Eq. 38).
 * out = {Nu_3D, Nu_2D, Nu_max}; map (n*n, x fastest then z) may be NULL. */
static void nusselt_of(const oracle *o, const double *gs, int stencil, double *out, double *map);

void oracle_nusselt(const oracle *o, int stencil, double *out, double *map)
{
    nusselt_of(o, o->g, stencil, out, map);
}

/* The same for a state g held by the caller (n^3 per population, [i][cell]). */
void oracle_nusselt_state(const oracle *o, const double *g, int stencil, double *out, double *map)
{
    nusselt_of(o, g, stencil, out, map);
}

static void nusselt_of(const oracle *o, const double *gs, int stencil, double *out, double *map)
{
    const int n = o->n;
    const size_t cells = (size_t)n * n * n;
    /* D_yy from the tau-bar actually used (Eq. 36 solved for D). */
    const double d_yy = EPS_T * (o->tau_wall - 0.5);
    double sum = 0.0, line = 0.0, mx = -INFINITY;
    for (int z = 0; z < n; ++z)
        for (int x = 0; x < n; ++x) {
            double th0 = 0.0, th1 = 0.0;
            size_t c0 = (size_t)x + (size_t)n * (0 + (size_t)n * z);
            size_t c1 = (size_t)x + (size_t)n * (1 + (size_t)n * z);
            for (int i = 0; i < Q7; ++i) {
                th0 += gs[i * cells + c0];
                th1 += gs[i * cells + c1];
            }
            /* Nu = -d theta / dY with Y = y / H, H = n. */
            double nu_loc;
            if (stencil == 1) {
                nu_loc = -2.0 * (th0 - o->theta_hot) * n;
            } else if (stencil == 2) {
                /* g_+y at the wall node entered from the wall in the last
                 * streaming: g_in = -g*_out + 2 w_T theta_h, so the net flux
                 * into the fluid is g_in - g*_out = 2 (g_in - w_T theta_h). */
                const double g_in = gs[3 * cells + c0];
                const double q = 2.0 * (g_in - W7[3] * o->theta_hot);
                nu_loc = n * q / d_yy;
            } else {
                double dth = (9.0 * th0 - th1 - 8.0 * o->theta_hot) / 3.0;
                nu_loc = -dth * n;
            }
            if (map) map[(size_t)x + (size_t)n * z] = nu_loc;
            sum += nu_loc;
            if (nu_loc > mx) mx = nu_loc;
            if (n % 2 == 1) {
                if (x == n / 2) line += nu_loc;
            } else if (x == n / 2 - 1 || x == n / 2) {
                line += 0.5 * nu_loc;
            }
        }
    out[0] = sum / ((double)n * n); /* Eq. (40), midpoint rule */
    out[1] = line / n;              /* Eq. (41), midpoint rule */
    out[2] = mx;
}

/* Copy the state (pre-collision populations at time t) out / in. */
void oracle_get_state(const oracle *o, double *f, double *g)
{
    size_t cells = (size_t)o->n * o->n * o->n;
    if (f) memcpy(f, o->f, sizeof(double) * Q19 * cells);
    if (g) memcpy(g, o->g, sizeof(double) * Q7 * cells);
}

void oracle_set_state(oracle *o, const double *f, const double *g, long t)
{
    size_t cells = (size_t)o->n * o->n * o->n;
    if (f) memcpy(o->f, f, sizeof(double) * Q19 * cells);
    if (g) memcpy(o->g, g, sizeof(double) * Q7 * cells);
    o->t = t;
}

/* One time step at the single node (x, y, z), for a state S_t held by the
 * caller (f: 19 n^3, g: 7 n^3, [i][cell]): the streaming of oracle_step read
 * from the destination's side.  Population i arrives from x - e_i after that
 * node's collision; where x - e_i lies outside, it is node x's own
 * post-collision population of the opposite direction reflected at the wall
 * (Eq. 8, R12; for g the rule of the wall crossed, R10).  fo, go: S_{t+1}. */
void oracle_step_node(const oracle *o, const double *f, const double *g, int x, int y, int z,
                      double *fo, double *go)
{
    const int n = o->n;
    const size_t cells = (size_t)n * n * n;
    double fi[Q19], gi[Q7], fp[Q19], gp[Q7], own_f[Q19], own_g[Q7];
    const int pos[3] = {x, y, z};
    size_t c = (size_t)x + (size_t)n * (y + (size_t)n * z);
    for (int i = 0; i < Q19; ++i) fi[i] = f[i * cells + c];
    for (int i = 0; i < Q7; ++i) gi[i] = g[i * cells + c];
    collide_node(o, fi, gi, own_f, own_g);

    for (int i = 0; i < Q19; ++i) {
        int sp[3], inside = 1;
        for (int d = 0; d < 3; ++d) {
            sp[d] = pos[d] - E19[i][d];
            if (o->wall_type == 0)
                sp[d] = (sp[d] + n) % n;
            else if (sp[d] < 0 || sp[d] >= n)
                inside = 0;
        }
        if (!inside) {
            fo[i] = own_f[opposite19(i)];  /* half-way bounce-back */
            continue;
        }
        size_t sc = (size_t)sp[0] + (size_t)n * (sp[1] + (size_t)n * sp[2]);
        for (int k = 0; k < Q19; ++k) fi[k] = f[k * cells + sc];
        for (int k = 0; k < Q7; ++k) gi[k] = g[k * cells + sc];
        collide_node(o, fi, gi, fp, gp);
        fo[i] = fp[i];
    }
    for (int i = 0; i < Q7; ++i) {
        int sp[3], inside = 1, axis = -1, side = 0;
        for (int d = 0; d < 3; ++d) {
            sp[d] = pos[d] - E7[i][d];
            if (o->wall_type == 0)
                sp[d] = (sp[d] + n) % n;
            else if (sp[d] < 0 || sp[d] >= n) {
                inside = 0;
                axis = d;
                side = -E7[i][d];  /* the opposite direction leaves through this side */
            }
        }
        if (!inside) {
            const int ib = opposite7(i);
            double tw;
            if (thermal_wall(o, axis, side, y, &tw))
                go[i] = -own_g[ib] + 2.0 * W7[i] * tw; /* R10 */
            else
                go[i] = own_g[ib];                     /* R10 */
            continue;
        }
        size_t sc = (size_t)sp[0] + (size_t)n * (sp[1] + (size_t)n * sp[2]);
        for (int k = 0; k < Q19; ++k) fi[k] = f[k * cells + sc];
        for (int k = 0; k < Q7; ++k) gi[k] = g[k * cells + sc];
        collide_node(o, fi, gi, fp, gp);
        go[i] = gp[i];
    }
}
