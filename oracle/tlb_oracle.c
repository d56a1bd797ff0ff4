/*
 * Plain FP64 CPU oracle of the ternary free-energy lattice Boltzmann step
 * (Semprebon, Krueger & Kusumaatmaja, "Ternary free energy lattice Boltzmann
 * model with tunable surface tensions and contact angles", arXiv:1511.02155).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no source with the HIP library.
 *
 * Conventions (the state and one step):
 *   - populations f (density), g (phi = C1 - C2), k (psi = C3), Sec. IV;
 *   - the state s_t is the set of post-propagation populations;
 *   - one step: moments -> wetting ghosts -> stencils -> chemical potentials
 *     and pressure terms -> equilibria -> BGK collision -> propagation with
 *     half-way bounce-back, in that order;
 *   - node index n = x + nx*(y + ny*z); populations stored [species][q][n].
 *
 * Readings of the paper used here:
 *   R1  mu_phi and mu_psi are written in the equivalent compact form
 *       mu_phi = (mu1 - mu2)/2, mu_psi = mu3 - (mu1 + mu2)/2 with
 *       mu_m = kappa_m C_m (1-C_m)(1-2C_m) - alpha^2 kappa_m lap C_m
 *       (Sec. III chemical potentials; algebraically identical to the printed
 *       expressions in rho, phi, psi).
 *   R2  the bulk pressure is p_b = rho c_s^2 + sum_m kappa_m/2 C_m^2 (1-C_m)
 *       (1-3C_m), the thermodynamic identity p_b = rho c_s^2 + sum X mu_X - F;
 *       the printed polynomial of Sec. III carries an extra 3 kappa_3 psi^2/2.
 *   R3  every gradient term of f^eq carries alpha^2, as in the pressure tensor
 *       of Sec. III (the printed equilibrium omits it; configurations use
 *       alpha = 1 where it makes no difference).
 *   R4  off-diagonal gradient terms are read symmetrically, so the gradient
 *       part of f^eq is 3 sum_{ab} w_i^{ab} T_ab with
 *       T_ab = alpha^2 sum_m kappa_m d_a C_m d_b C_m.
 *   R5  D3Q19 weights are assigned by velocity class (the printed index sets
 *       need 11-14 to be the yz diagonals and 15-18 the zx diagonals).
 *   R6  D2Q9 gradient weights (not in the paper): w^xx = 1/9 on (+-1,0),
 *       -1/18 on (0,+-1), -1/72 on diagonals; w^xy = e_x e_y / 12.
 *   R7  derivatives use the isotropic lattice stencils
 *       d_a X = (1/c_s^2) sum_i w_i e_ia X(r+e_i),
 *       lap X = (2/c_s^2) sum_i w_i [X(r+e_i) - X(r)].
 *   R8  the wetting condition alpha^2 kappa_m grad_perp C_m = -h_m is imposed
 *       on a half-way wall through a ghost row:
 *       C_m(ghost) = C_m(adjacent fluid node) + h_m / (alpha^2 kappa_m).
 *   R9  bounce-back is the half-way, stationary-wall rule in pull form.
 *   R18 the multiple-relaxation-time collision (Sec. IV names the extension,
 *       after the binary model's, without a moment basis) acts on f only:
 *       f* = f - M^-1 S M (f - f^eq) with the orthogonal polynomial bases of
 *       Lallemand & Luo (D2Q9) and d'Humieres et al. (D3Q19); the viscous
 *       stress moments relax at 1/tau_f, the energy moment at 1/tau_bulk and
 *       every other moment at 1/tau_ghost (the conserved ones have no
 *       non-equilibrium part).  g and k keep the BGK rule.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 19

typedef struct {
    int32_t lattice; /* 0: D2Q9, 1: D3Q19 */
    int32_t nx, ny, nz;
    int32_t walls_y; /* 0: periodic in y; 1: half-way walls below y=0 and above y=ny-1 */
    double kappa[3];
    double alpha;
    double tau_f, tau_g, tau_k;
    double gamma_phi, gamma_psi;
    int32_t no_advection; /* 1: g^eq and k^eq without the velocity terms (diffusive Cahn-Hilliard) */
    int32_t collision;    /* 0: BGK; 1: multiple relaxation times for f (reading R18) */
    double tau_bulk, tau_ghost; /* MRT relaxation times of the energy moment and of the other moments */
} orc_params;

typedef struct {
    int Q, D;
    int e[ORC_MAXQ][3];
    double w[ORC_MAXQ];
    int opp[ORC_MAXQ];
    /* gradient weights w_i^{ab}, components ordered xx, yy, zz, xy, yz, zx */
    double wab[ORC_MAXQ][6];
} orc_lattice;

/* ------------------------------------------------------------------------ */
/* Lattices.  D3Q19 velocity set of Sec. IV; the index order follows the     */
/* weight index sets printed there (axes 1-6, xy diagonals 7-10, yz           */
/* diagonals 11-14, zx diagonals 15-18; within a plane (+,+),(+,-),(-,+),     */
/* (-,-)).  D2Q9 uses the same order restricted to the plane.                 */
/* ------------------------------------------------------------------------ */
static void build_lattice(int lattice, orc_lattice* L)
{
    static const int e2[9][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                 {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0}};
    static const int e3[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                                  {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {1, -1, 0}, {-1, 1, 0},
                                  {-1, -1, 0}, {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1},
                                  {1, 0, 1},  {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1}};
    memset(L, 0, sizeof(*L));
    if (lattice == 0) {
        L->Q = 9;
        L->D = 2;
        memcpy(L->e, e2, sizeof(e2));
    } else {
        L->Q = 19;
        L->D = 3;
        memcpy(L->e, e3, sizeof(e3));
    }
    for (int i = 0; i < L->Q; ++i) {
        int e2n = L->e[i][0] * L->e[i][0] + L->e[i][1] * L->e[i][1] + L->e[i][2] * L->e[i][2];
        /* lattice weights: D2Q9 4/9, 1/9, 1/36 (standard); D3Q19 1/3, 1/18, 1/36 (Sec. IV) */
        if (L->D == 2)
            L->w[i] = (e2n == 0) ? 4.0 / 9.0 : (e2n == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        else
            L->w[i] = (e2n == 0) ? 1.0 / 3.0 : (e2n == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        for (int j = 0; j < L->Q; ++j)
            if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] && L->e[j][2] == -L->e[i][2])
                L->opp[i] = j;
        if (e2n == 0)
            continue; /* rest population is fixed by the mass constraint */
        /* diagonal gradient weights w^{aa} by velocity class (readings R5, R6) */
        for (int a = 0; a < L->D; ++a) {
            int ea = L->e[i][a];
            double v;
            if (e2n == 1) {
                if (ea != 0)
                    v = (L->D == 2) ? 1.0 / 9.0 : 5.0 / 36.0;
                else
                    v = (L->D == 2) ? -1.0 / 18.0 : -1.0 / 9.0;
            } else {
                if (ea != 0)
                    v = -1.0 / 72.0;
                else
                    v = 1.0 / 36.0; /* only occurs in D3Q19 */
            }
            L->wab[i][a] = v;
        }
        /* off-diagonal gradient weights w^{ab} = e_a e_b / 12 on diagonals */
        if (e2n == 2) {
            L->wab[i][3] = L->e[i][0] * L->e[i][1] / 12.0;
            if (L->D == 3) {
                L->wab[i][4] = L->e[i][1] * L->e[i][2] / 12.0;
                L->wab[i][5] = L->e[i][2] * L->e[i][0] / 12.0;
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Local thermodynamics.                                                     */
/* ------------------------------------------------------------------------ */

/* Concentrations from the auxiliary variables, Sec. II.C. */
static void concentrations(double rho, double phi, double psi, double C[3])
{
    C[0] = 0.5 * (rho + phi - psi);
    C[1] = 0.5 * (rho - phi - psi);
    C[2] = psi;
}

/* Chemical potentials mu_phi, mu_psi (Sec. III, reading R1), bulk pressure
 * p_b (reading R2), and Lambda = alpha^2 sum_m kappa_m C_m lap C_m, the
 * isotropic Laplacian part of the pressure tensor of Sec. III. */
static void local_thermo(const orc_params* P, double rho, const double C[3], const double lapC[3],
                         double* mu_phi, double* mu_psi, double* p_b, double* Lambda)
{
    double a2 = P->alpha * P->alpha;
    double mu[3];
    double pb = rho / 3.0;
    double lam = 0.0;
    for (int m = 0; m < 3; ++m) {
        double c = C[m], km = P->kappa[m];
        mu[m] = km * c * (1.0 - c) * (1.0 - 2.0 * c) - a2 * km * lapC[m];
        pb += 0.5 * km * c * c * (1.0 - c) * (1.0 - 3.0 * c);
        lam += a2 * km * c * lapC[m];
    }
    *mu_phi = 0.5 * (mu[0] - mu[1]);
    *mu_psi = mu[2] - 0.5 * (mu[0] + mu[1]);
    *p_b = pb;
    *Lambda = lam;
}

/* Equilibria f^eq, g^eq, k^eq of Sec. IV (eq. eqdistfbinary) for i > 0 with
 * readings R3, R4; the rest populations follow from the mass constraints
 * sum_i f^eq_i = rho, sum_i g^eq_i = phi, sum_i k^eq_i = psi.  With
 * no_advection the velocity terms of g^eq and k^eq are left out, which
 * removes the advection term from the Cahn-Hilliard equations (the diffusive
 * runs of Sec. V.C). */
static void equilibria(const orc_params* P, const orc_lattice* L, double rho, const double v[3],
                       double phi, double psi, const double C[3], const double gradC[3][3],
                       const double lapC[3], double* feq, double* geq, double* keq)
{
    const double cs2 = 1.0 / 3.0;
    double mu_phi, mu_psi, pb, lam;
    local_thermo(P, rho, C, lapC, &mu_phi, &mu_psi, &pb, &lam);
    double a2 = P->alpha * P->alpha;
    double T[6] = {0, 0, 0, 0, 0, 0}; /* xx yy zz xy yz zx */
    static const int ia[6] = {0, 1, 2, 0, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 0};
    for (int c = 0; c < 6; ++c)
        for (int m = 0; m < 3; ++m)
            T[c] += a2 * P->kappa[m] * gradC[m][ia[c]] * gradC[m][ib[c]];
    double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double fs = 0.0, gs = 0.0, ks = 0.0;
    for (int i = 1; i < L->Q; ++i) {
        double ev = L->e[i][0] * v[0] + L->e[i][1] * v[1] + L->e[i][2] * v[2];
        double vel = ev / cs2 + ev * ev / (2.0 * cs2 * cs2) - vv / (2.0 * cs2);
        double grad = 0.0;
        for (int c = 0; c < 6; ++c)
            grad += L->wab[i][c] * T[c];
        feq[i] = L->w[i] * ((pb - lam) / cs2 + rho * vel) + grad / cs2;
        const double cvel = P->no_advection ? 0.0 : vel;
        geq[i] = L->w[i] * (P->gamma_phi * mu_phi / cs2 + phi * cvel);
        keq[i] = L->w[i] * (P->gamma_psi * mu_psi / cs2 + psi * cvel);
        fs += feq[i];
        gs += geq[i];
        ks += keq[i];
    }
    feq[0] = rho - fs;
    geq[0] = phi - gs;
    keq[0] = psi - ks;
}

/* ------------------------------------------------------------------------ */
/* Lattice-wide helpers.                                                     */
/* ------------------------------------------------------------------------ */
static inline long node_index(const orc_params* P, int x, int y, int z)
{
    return (long)x + (long)P->nx * ((long)y + (long)P->ny * (long)z);
}

static inline int wrap(int a, int n) { return ((a % n) + n) % n; }

/* Concentration fields with ghost rows y = -1 and y = ny: array
 * [3][nz][ny+2][nx]; row index yy = y + 1. */
static inline long cg_index(const orc_params* P, int m, int x, int yy, int z)
{
    return (long)x + (long)P->nx * ((long)yy + (long)(P->ny + 2) * ((long)z + (long)P->nz * m));
}

/* Moments of Sec. IV (eq. lbconstraint) at every node, and C_m (Sec. II.C). */
static void moments(const orc_params* P, const orc_lattice* L, const double* pop, double* rho,
                    double* vel /*[3][N]*/, double* phi, double* psi, double* Cg)
{
    long N = (long)P->nx * P->ny * P->nz;
    const double* f = pop;
    const double* g = pop + (long)L->Q * N;
    const double* k = pop + 2L * L->Q * N;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long n = node_index(P, x, y, z);
                double r = 0, j[3] = {0, 0, 0}, ph = 0, ps = 0;
                for (int i = 0; i < L->Q; ++i) {
                    double fi = f[(long)i * N + n];
                    r += fi;
                    for (int a = 0; a < 3; ++a)
                        j[a] += fi * L->e[i][a];
                    ph += g[(long)i * N + n];
                    ps += k[(long)i * N + n];
                }
                rho[n] = r;
                for (int a = 0; a < 3; ++a)
                    vel[a * N + n] = j[a] / r;
                phi[n] = ph;
                psi[n] = ps;
                double C[3];
                concentrations(r, ph, ps, C);
                for (int m = 0; m < 3; ++m)
                    Cg[cg_index(P, m, x, y + 1, z)] = C[m];
            }
}

/* Ghost rows (reading R8 of the wetting condition of Sec. II.B, eq.
 * cahn_gradient; the equivalent conditions on rho, phi, psi are those of
 * Sec. II.C).  With periodic y the ghost rows are periodic images. */
static void fill_ghosts(const orc_params* P, const double* h, double* Cg)
{
    double a2 = P->alpha * P->alpha;
    long nxz = (long)P->nx * P->nz;
    for (int m = 0; m < 3; ++m)
        for (int z = 0; z < P->nz; ++z)
            for (int x = 0; x < P->nx; ++x) {
                if (P->walls_y) {
                    double hb = h ? h[(0 * 3 + m) * nxz + x + (long)P->nx * z] : 0.0;
                    double ht = h ? h[(1 * 3 + m) * nxz + x + (long)P->nx * z] : 0.0;
                    Cg[cg_index(P, m, x, 0, z)] =
                        Cg[cg_index(P, m, x, 1, z)] + hb / (a2 * P->kappa[m]);
                    Cg[cg_index(P, m, x, P->ny + 1, z)] =
                        Cg[cg_index(P, m, x, P->ny, z)] + ht / (a2 * P->kappa[m]);
                } else {
                    Cg[cg_index(P, m, x, 0, z)] = Cg[cg_index(P, m, x, P->ny, z)];
                    Cg[cg_index(P, m, x, P->ny + 1, z)] = Cg[cg_index(P, m, x, 1, z)];
                }
            }
}

/* Gradient and Laplacian of C_m at node (x,y,z) with the stencils of
 * reading R7 (x and z periodic; y through the ghost rows). */
static void stencil(const orc_params* P, const orc_lattice* L, const double* Cg, int x, int y, int z,
                    double gradC[3][3], double lapC[3])
{
    for (int m = 0; m < 3; ++m) {
        double c0 = Cg[cg_index(P, m, x, y + 1, z)];
        double gr[3] = {0, 0, 0}, lp = 0.0;
        for (int i = 0; i < L->Q; ++i) {
            int xn = wrap(x + L->e[i][0], P->nx);
            int yn = y + L->e[i][1] + 1;
            int zn = wrap(z + L->e[i][2], P->nz);
            double c = Cg[cg_index(P, m, xn, yn, zn)];
            for (int a = 0; a < 3; ++a)
                gr[a] += L->w[i] * L->e[i][a] * c;
            lp += L->w[i] * (c - c0);
        }
        for (int a = 0; a < 3; ++a)
            gradC[m][a] = 3.0 * gr[a];
        lapC[m] = 6.0 * lp;
    }
}

/* Propagation (eq. latboltPropagation) in pull form with half-way
 * bounce-back at the y walls (reading R9). */
static void propagate(const orc_params* P, const orc_lattice* L, const double* post, double* pop)
{
    long N = (long)P->nx * P->ny * P->nz;
    for (int s = 0; s < 3; ++s)
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < P->nz; ++z)
            for (int y = 0; y < P->ny; ++y)
                for (int x = 0; x < P->nx; ++x) {
                    long n = node_index(P, x, y, z);
                    for (int i = 0; i < L->Q; ++i) {
                        int ys = y - L->e[i][1];
                        double val;
                        if (P->walls_y && (ys < 0 || ys >= P->ny)) {
                            val = post[((long)s * L->Q + L->opp[i]) * N + n];
                        } else {
                            int xs = wrap(x - L->e[i][0], P->nx);
                            int zs = wrap(z - L->e[i][2], P->nz);
                            ys = wrap(ys, P->ny);
                            val = post[((long)s * L->Q + i) * N + node_index(P, xs, ys, zs)];
                        }
                        pop[((long)s * L->Q + i) * N + n] = val;
                    }
                }
}

/* ------------------------------------------------------------------------ */
/* Exported API.                                                             */
/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Moment basis of the multiple-relaxation-time collision (reading R18).     */
/* Row k of M holds moment k as a polynomial of the velocity c = e_i; cls[k] */
/* is its class: 0 conserved, 1 energy (bulk viscosity), 2 viscous stress,   */
/* 3 other.                                                                   */
/*   D2Q9:  rho, e, eps, jx, qx, jy, qy, pxx, pxy                             */
/*   D3Q19: rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww,      */
/*          pxy, pyz, pxz, mx, my, mz                                          */
/* ------------------------------------------------------------------------ */
static void mrt_basis(const orc_lattice* L, double M[ORC_MAXQ][ORC_MAXQ], int cls[ORC_MAXQ])
{
    for (int i = 0; i < L->Q; ++i) {
        const double x = L->e[i][0], y = L->e[i][1], z = L->e[i][2];
        const double c2 = x * x + y * y + z * z;
        double r[ORC_MAXQ];
        if (L->Q == 9) {
            r[0] = 1.0;
            r[1] = -4.0 + 3.0 * c2;
            r[2] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
            r[3] = x;
            r[4] = (-5.0 + 3.0 * c2) * x;
            r[5] = y;
            r[6] = (-5.0 + 3.0 * c2) * y;
            r[7] = x * x - y * y;
            r[8] = x * y;
        } else {
            r[0] = 1.0;
            r[1] = 19.0 * c2 - 30.0;
            r[2] = (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
            r[3] = x;
            r[4] = (5.0 * c2 - 9.0) * x;
            r[5] = y;
            r[6] = (5.0 * c2 - 9.0) * y;
            r[7] = z;
            r[8] = (5.0 * c2 - 9.0) * z;
            r[9] = 3.0 * x * x - c2;
            r[10] = (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
            r[11] = y * y - z * z;
            r[12] = (3.0 * c2 - 5.0) * (y * y - z * z);
            r[13] = x * y;
            r[14] = y * z;
            r[15] = x * z;
            r[16] = (y * y - z * z) * x;
            r[17] = (z * z - x * x) * y;
            r[18] = (x * x - y * y) * z;
        }
        for (int k = 0; k < L->Q; ++k)
            M[k][i] = r[k];
    }
    static const int c9[9] = {0, 1, 3, 0, 3, 0, 3, 2, 2};
    static const int c19[19] = {0, 1, 3, 0, 3, 0, 3, 0, 3, 2, 3, 2, 3, 2, 2, 2, 3, 3, 3};
    for (int k = 0; k < L->Q; ++k)
        cls[k] = L->Q == 9 ? c9[k] : c19[k];
}

/* Inverse of an n x n matrix by Gauss-Jordan elimination with partial pivoting; 0 on success. */
static int invert(int n, double A[ORC_MAXQ][ORC_MAXQ], double X[ORC_MAXQ][ORC_MAXQ])
{
    double W[ORC_MAXQ][2 * ORC_MAXQ];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            W[r][c] = c < n ? A[r][c] : (c - n == r ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(W[r][c]) > fabs(W[piv][c]))
                piv = r;
        if (W[piv][c] == 0.0)
            return -1;
        for (int k = 0; k < 2 * n; ++k) {
            const double t = W[c][k];
            W[c][k] = W[piv][k];
            W[piv][k] = t;
        }
        const double d = W[c][c];
        for (int k = 0; k < 2 * n; ++k)
            W[c][k] /= d;
        for (int r = 0; r < n; ++r)
            if (r != c && W[r][c] != 0.0) {
                const double f = W[r][c];
                for (int k = 0; k < 2 * n; ++k)
                    W[r][k] -= f * W[c][k];
            }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c)
            X[r][c] = W[r][n + c];
    return 0;
}

/* Moment basis of a lattice for the tests: M[Q][Q] (row = moment) and the classes. */
int orc_mrt_basis(int lattice, double* M, int* cls)
{
    if (lattice != 0 && lattice != 1)
        return -1;
    orc_lattice L;
    build_lattice(lattice, &L);
    double B[ORC_MAXQ][ORC_MAXQ];
    mrt_basis(&L, B, cls);
    for (int k = 0; k < L.Q; ++k)
        for (int i = 0; i < L.Q; ++i)
            M[k * L.Q + i] = B[k][i];
    return L.Q;
}

int orc_check_params(const orc_params* P)
{
    if (!P || (P->lattice != 0 && P->lattice != 1))
        return -1;
    if (P->nx < 3 || P->ny < 3 || P->nz < 1)
        return -1;
    if ((P->lattice == 0) != (P->nz == 1))
        return -1;
    if (P->lattice == 1 && P->nz < 3)
        return -1;
    if (!(P->tau_f > 0.5 && P->tau_g > 0.5 && P->tau_k > 0.5))
        return -1;
    if (!(P->alpha > 0.0))
        return -1;
    if (P->no_advection != 0 && P->no_advection != 1)
        return -1;
    if (P->collision != 0 && P->collision != 1)
        return -1;
    if (P->collision == 1 && !(P->tau_bulk > 0.5 && P->tau_ghost > 0.5))
        return -1;
    for (int m = 0; m < 3; ++m)
        if (!(P->kappa[m] > 0.0))
            return -1;
    return 0;
}

int orc_lattice_info(int lattice, int* Q, int* e /*[Q][3]*/, double* w, double* wab /*[Q][6]*/,
                     int* opp)
{
    orc_lattice L;
    build_lattice(lattice, &L);
    *Q = L.Q;
    for (int i = 0; i < L.Q; ++i) {
        if (e)
            for (int a = 0; a < 3; ++a)
                e[i * 3 + a] = L.e[i][a];
        if (w)
            w[i] = L.w[i];
        if (wab)
            for (int c = 0; c < 6; ++c)
                wab[i * 6 + c] = L.wab[i][c];
        if (opp)
            opp[i] = L.opp[i];
    }
    return 0;
}

/* Single-node thermodynamics and equilibria, for the unit pins. */
int orc_node_thermo(const orc_params* P, double rho, const double* C, const double* lapC,
                    double* out /* mu_phi, mu_psi, p_b, Lambda */)
{
    local_thermo(P, rho, C, lapC, &out[0], &out[1], &out[2], &out[3]);
    return 0;
}

int orc_node_equilibria(const orc_params* P, double rho, const double* v, double phi, double psi,
                        const double* gradC /*[3][3]*/, const double* lapC, double* feq,
                        double* geq, double* keq)
{
    orc_lattice L;
    build_lattice(P->lattice, &L);
    double C[3], g3[3][3], vv[3] = {v[0], v[1], L.D == 3 ? v[2] : 0.0};
    concentrations(rho, phi, psi, C);
    for (int m = 0; m < 3; ++m)
        for (int a = 0; a < 3; ++a)
            g3[m][a] = (a < L.D) ? gradC[m * 3 + a] : 0.0;
    equilibria(P, &L, rho, vv, phi, psi, C, g3, lapC, feq, geq, keq);
    return 0;
}

/* Gradient and Laplacian of three given concentration fields C[3][N] with
 * the ghost rows of the wetting condition, for the stencil pins. */
int orc_gradients(const orc_params* P, const double* h, const double* C, double* grad /*[3][3][N]*/,
                  double* lap /*[3][N]*/)
{
    if (orc_check_params(P))
        return -1;
    orc_lattice L;
    build_lattice(P->lattice, &L);
    long N = (long)P->nx * P->ny * P->nz;
    double* Cg = (double*)calloc((size_t)3 * P->nx * (P->ny + 2) * P->nz, sizeof(double));
    if (!Cg)
        return -2;
    for (int m = 0; m < 3; ++m)
        for (int z = 0; z < P->nz; ++z)
            for (int y = 0; y < P->ny; ++y)
                for (int x = 0; x < P->nx; ++x)
                    Cg[cg_index(P, m, x, y + 1, z)] = C[m * N + node_index(P, x, y, z)];
    fill_ghosts(P, h, Cg);
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                double gc[3][3], lc[3];
                long n = node_index(P, x, y, z);
                stencil(P, &L, Cg, x, y, z, gc, lc);
                for (int m = 0; m < 3; ++m) {
                    for (int a = 0; a < 3; ++a)
                        grad[(m * 3 + a) * N + n] = gc[m][a];
                    lap[m * N + n] = lc[m];
                }
            }
    free(Cg);
    return 0;
}

/* Initial state: populations equal to the equilibria of the given fields
 * C[3][N] and velocity u[D][N] (NULL: at rest), with rho = sum_m C_m,
 * phi = C1 - C2, psi = C3 (Sec. II.C) and the gradient terms evaluated from
 * the same fields. */
int orc_init_equilibrium(const orc_params* P, const double* h, const double* C, const double* u,
                         double* pop)
{
    if (orc_check_params(P))
        return -1;
    orc_lattice L;
    build_lattice(P->lattice, &L);
    long N = (long)P->nx * P->ny * P->nz;
    double* Cg = (double*)calloc((size_t)3 * P->nx * (P->ny + 2) * P->nz, sizeof(double));
    if (!Cg)
        return -2;
    for (int m = 0; m < 3; ++m)
        for (int z = 0; z < P->nz; ++z)
            for (int y = 0; y < P->ny; ++y)
                for (int x = 0; x < P->nx; ++x)
                    Cg[cg_index(P, m, x, y + 1, z)] = C[m * N + node_index(P, x, y, z)];
    fill_ghosts(P, h, Cg);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long n = node_index(P, x, y, z);
                double c[3], gc[3][3], lc[3], v[3] = {0, 0, 0};
                for (int m = 0; m < 3; ++m)
                    c[m] = C[m * N + n];
                if (u)
                    for (int a = 0; a < L.D; ++a)
                        v[a] = u[a * N + n];
                double rho = c[0] + c[1] + c[2], phi = c[0] - c[1], psi = c[2];
                double cc[3];
                concentrations(rho, phi, psi, cc);
                stencil(P, &L, Cg, x, y, z, gc, lc);
                double feq[ORC_MAXQ], geq[ORC_MAXQ], keq[ORC_MAXQ];
                equilibria(P, &L, rho, v, phi, psi, cc, gc, lc, feq, geq, keq);
                for (int i = 0; i < L.Q; ++i) {
                    pop[(0L * L.Q + i) * N + n] = feq[i];
                    pop[(1L * L.Q + i) * N + n] = geq[i];
                    pop[(2L * L.Q + i) * N + n] = keq[i];
                }
            }
    free(Cg);
    return 0;
}

/* Advance the state s_t (post-propagation populations [3][Q][N]) by nsteps
 * time steps: moments, ghosts, stencils, thermodynamics, equilibria, BGK
 * collision (eq. latboltCollision; multiple relaxation times for f with
 * collision == 1, reading R18) and propagation. */
int orc_step(const orc_params* P, const double* h, double* pop, long nsteps)
{
    if (orc_check_params(P))
        return -1;
    orc_lattice L;
    build_lattice(P->lattice, &L);
    long N = (long)P->nx * P->ny * P->nz;
    double* post = (double*)malloc(sizeof(double) * 3 * L.Q * N);
    double* rho = (double*)malloc(sizeof(double) * N);
    double* vel = (double*)malloc(sizeof(double) * 3 * N);
    double* phi = (double*)malloc(sizeof(double) * N);
    double* psi = (double*)malloc(sizeof(double) * N);
    double* Cg = (double*)calloc((size_t)3 * P->nx * (P->ny + 2) * P->nz, sizeof(double));
    if (!post || !rho || !vel || !phi || !psi || !Cg) {
        free(post), free(rho), free(vel), free(phi), free(psi), free(Cg);
        return -2;
    }
    const double itau[3] = {1.0 / P->tau_f, 1.0 / P->tau_g, 1.0 / P->tau_k};
    /* multiple relaxation times for f (reading R18): K = M^-1 S M */
    double K[ORC_MAXQ][ORC_MAXQ];
    if (P->collision == 1) {
        double M[ORC_MAXQ][ORC_MAXQ], Mi[ORC_MAXQ][ORC_MAXQ];
        int cls[ORC_MAXQ];
        mrt_basis(&L, M, cls);
        if (invert(L.Q, M, Mi)) {
            free(post), free(rho), free(vel), free(phi), free(psi), free(Cg);
            return -3;
        }
        double S[ORC_MAXQ];
        for (int k = 0; k < L.Q; ++k)
            S[k] = cls[k] == 2 ? 1.0 / P->tau_f : (cls[k] == 1 ? 1.0 / P->tau_bulk : 1.0 / P->tau_ghost);
        for (int i = 0; i < L.Q; ++i)
            for (int j = 0; j < L.Q; ++j) {
                double a = 0.0;
                for (int k = 0; k < L.Q; ++k)
                    a += Mi[i][k] * S[k] * M[k][j];
                K[i][j] = a;
            }
    }
    for (long t = 0; t < nsteps; ++t) {
        moments(P, &L, pop, rho, vel, phi, psi, Cg);
        fill_ghosts(P, h, Cg);
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < P->nz; ++z)
            for (int y = 0; y < P->ny; ++y)
                for (int x = 0; x < P->nx; ++x) {
                    long n = node_index(P, x, y, z);
                    double gc[3][3], lc[3], C[3], v[3];
                    stencil(P, &L, Cg, x, y, z, gc, lc);
                    concentrations(rho[n], phi[n], psi[n], C);
                    for (int a = 0; a < 3; ++a)
                        v[a] = vel[a * N + n];
                    double eq[3][ORC_MAXQ];
                    equilibria(P, &L, rho[n], v, phi[n], psi[n], C, gc, lc, eq[0], eq[1], eq[2]);
                    for (int s = 0; s < 3; ++s) {
                        if (s == 0 && P->collision == 1) {
                            double d[ORC_MAXQ];
                            for (int j = 0; j < L.Q; ++j)
                                d[j] = pop[(long)j * N + n] - eq[0][j];
                            for (int i = 0; i < L.Q; ++i) {
                                double r = 0.0;
                                for (int j = 0; j < L.Q; ++j)
                                    r += K[i][j] * d[j];
                                post[(long)i * N + n] = pop[(long)i * N + n] - r;
                            }
                            continue;
                        }
                        for (int i = 0; i < L.Q; ++i) {
                            long a = ((long)s * L.Q + i) * N + n;
                            post[a] = pop[a] - itau[s] * (pop[a] - eq[s][i]);
                        }
                    }
                }
        propagate(P, &L, post, pop);
    }
    free(post), free(rho), free(vel), free(phi), free(psi), free(Cg);
    return 0;
}

/* Macroscopic fields of the state s_t, out[11][N] in the order
 * C1, C2, C3, rho, phi, psi, ux, uy, uz, mu_phi, mu_psi. */
int orc_fields(const orc_params* P, const double* h, const double* pop, double* out)
{
    if (orc_check_params(P))
        return -1;
    orc_lattice L;
    build_lattice(P->lattice, &L);
    long N = (long)P->nx * P->ny * P->nz;
    double* Cg = (double*)calloc((size_t)3 * P->nx * (P->ny + 2) * P->nz, sizeof(double));
    if (!Cg)
        return -2;
    moments(P, &L, pop, out + 3 * N, out + 6 * N, out + 4 * N, out + 5 * N, Cg);
    fill_ghosts(P, h, Cg);
    for (int z = 0; z < P->nz; ++z)
        for (int y = 0; y < P->ny; ++y)
            for (int x = 0; x < P->nx; ++x) {
                long n = node_index(P, x, y, z);
                double gc[3][3], lc[3], C[3], th[4];
                stencil(P, &L, Cg, x, y, z, gc, lc);
                concentrations(out[3 * N + n], out[4 * N + n], out[5 * N + n], C);
                for (int m = 0; m < 3; ++m)
                    out[m * N + n] = C[m];
                local_thermo(P, out[3 * N + n], C, lc, &th[0], &th[1], &th[2], &th[3]);
                out[9 * N + n] = th[0];
                out[10 * N + n] = th[1];
            }
    free(Cg);
    return 0;
}
