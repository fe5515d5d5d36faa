/*
 * lbm_oracle.c -- FP64 CPU oracle for one time step of the bump-function D3Q19 lattice
 * Boltzmann scheme of Afrasiabian & Denniston, "A Novel Velocity Discretization for Lattice
 * Boltzmann Method: Application to Compressible Flow" (arXiv:2501.00620).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * load this library. It shares no code, header, table or helper with the GPU library, and the
 * GPU library never calls it.
 *
 * Written to be checked by eye against the paper: plain loops over sites, double precision, no
 * blocking or fusion, built with -O2 -ffp-contract=off. Every quantity keeps the paper's name.
 *
 * State (the auxiliary variables of Sec. II C): per site the 19 post-stream populations
 * fbar_i (Eq. 49-50) and the 6 components of the auxiliary variance bbar_ab (Eq. 62), both in
 * structure-of-arrays order  field[k][z][y][x]  (x fastest).  Periodic in all three directions.
 * Lattice units: dx = dt = c = 1.
 *
 * One step (Sec. II C), read as follows where the paper leaves room:
 *   1. predictor moments from the post-stream state: rho = sum fbar (Eq. 56),
 *      j* = sum fbar e, u* = j* / rho, Pi* = sum fbar e e;  temperature T* from the total second
 *      moment trace of the bump expansion (Eq. 26) in the energy-conserving mode, or the
 *      prescribed T in the isothermal mode;  beq* = beq(u*, T*) (Appendix A, Eq. 36);
 *      physical b = bbar - (omega/2)(bbar - beq*)   (Eqs. 62-65, 67-68), omega = 1/(tau+1/2);
 *   2. gradient sources R_ab = rho b_ab and X_abg = rho u*_g b_ab, and their isotropic finite
 *      differences  F_b = -d_a R_ab  (Eq. 59)  and  S_bg = -d_a (X_abg + X_agb)  (Eq. 61);
 *   3. corrected moments u = (j* + F/2)/rho (Eq. 57) and, energy-conserving mode,
 *      3 rho T = tr Pi* + rho tr bbar + tr S / 2 - rho |u|^2;
 *   4. feq(rho,u) and beq(u,T) (Appendix A), forcing Phi from its moments (Eqs. 58-61) through
 *      the inverse of the transformation matrix of Appendix B (Table I);
 *   5. BGK collision (Eq. 55): fbar* = fbar - omega (fbar - feq) + (1 - omega/2) Phi,
 *      and bbar* = bbar - omega (bbar - beq) (Eq. 65);
 *   6. stream fbar*_i along e_i (Eq. 49) and gather bbar with the arriving populations as
 *      weights (Eq. 66): bbar(x) = sum_i fbar*_i(x-e_i) bbar*(x-e_i) / rho(x).
 *
 * The readings behind steps 1, 3, 6 (temperature closure, which velocity enters the gradient
 * sources, post-collision gather weights, the D3Q19 finite-difference stencil) are listed with
 * their reasons in the design notes of the repository.
 *
 * Walls (the channels of Sec. III A and C): optionally two planar walls normal to z, half-way
 * between the last fluid plane and its periodic image (z = -1/2 and z = nz - 1/2), with
 * tangential velocities u_b (bottom) and u_t (top); x and y stay periodic.  Read as follows:
 *   - half-way bounce-back with the moving-wall momentum of Ladd: a population that would stream
 *     through a wall returns to its site reversed, plus 6 w_i rho(x) e_i.u_w, which is
 *     feq_i(rho, u_w) - feq_opp(i)(rho, u_w) of Appendix A (its odd part is exactly linear in u);
 *   - it carries the variance of the site it left, which is also its destination (a full reversal
 *     maps a second moment onto itself);
 *   - the gradient sources one plane beyond a wall, in the same (x, y) column:
 *       R = rho b (the variance part of the pressure) is mirrored, R(-1) = R(0), as bounce-back
 *       mirrors the populations' own second moment (a reversal maps a second moment onto itself);
 *       X = rho u* b is extrapolated to second order, X(-1) = 3 X(0) - 3 X(1) + X(2), so its
 *       z-derivative at a wall-adjacent site is the one-sided second-order difference.
 *     Extrapolating R as well destabilises the energy-conserving mode below T = 1/3 and moving
 *     walls under gravity; mirroring X spoils the viscous stress at a no-slip wall and the
 *     hydrostatic balance (u* carries half the body force).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
#define NB 6 /* b components: xx yy zz xy xz yz */

/* Velocity set, read off rows 2-4 of Table I (Appendix B); c = 1. */
static const int E[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0},
    {1, 0, 1}, {1, 0, -1}, {-1, 0, 1}, {-1, 0, -1},
    {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1},
};

/* Weights w_i = feq_i(u = 0)/rho, read off the Appendix A closed forms at u = 0. */
static const double W[Q] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
};

/* index pairs of the symmetric tensor components, in storage order */
static const int BA[NB] = {0, 1, 2, 0, 0, 1};
static const int BB[NB] = {0, 1, 2, 1, 2, 2};

static int comp(int a, int b) /* storage slot of the symmetric pair (a,b) */
{
    if (a == b) return a;
    if ((a == 0 && b == 1) || (a == 1 && b == 0)) return 3;
    if ((a == 0 && b == 2) || (a == 2 && b == 0)) return 4;
    return 5;
}

void orc_velocity_set(int *e, double *w)
{
    for (int i = 0; i < Q; i++) {
        for (int a = 0; a < 3; a++) e[3 * i + a] = E[i][a];
        w[i] = W[i];
    }
}

/* ---------------------------------------------------------------------------------------------
 * Equilibrium populations, Appendix A, written term by term as printed (c kept explicit).
 * ------------------------------------------------------------------------------------------- */
void orc_feq(double rho, double ux, double uy, double uz, double *f)
{
    const double c = 1.0;
    const double c2 = c * c, c3 = c2 * c, c4 = c2 * c2;
    const double x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    f[0] = rho * (3 * c4 - 2 * (x2 + y2 + z2) * c2 - 6 * ((y2 + z2) * x2 + y2 * z2)) / (9 * c4);
    f[1] = rho * (c4 + 3 * ux * c3 + 2 * (x2 - y2 - z2) * c2 + 6 * x2 * (y2 + z2)) / (18 * c4);
    f[2] = rho * (c4 + 3 * uy * c3 - 2 * (x2 - y2 + z2) * c2 + 6 * y2 * (x2 + z2)) / (18 * c4);
    f[3] = rho * (c4 - 3 * ux * c3 + 2 * (x2 - y2 - z2) * c2 + 6 * x2 * (y2 + z2)) / (18 * c4);
    f[4] = rho * (c4 - 3 * uy * c3 - 2 * (x2 - y2 + z2) * c2 + 6 * y2 * (x2 + z2)) / (18 * c4);
    f[5] = rho * (c4 + 3 * uz * c3 - 2 * (x2 + y2 - z2) * c2 + 6 * (x2 + y2) * z2) / (18 * c4);
    f[6] = rho * (c4 - 3 * uz * c3 - 2 * (x2 + y2 - z2) * c2 + 6 * (x2 + y2) * z2) / (18 * c4);
    f[7] = rho * (c4 + 3 * (ux + uy) * c3 + 2 * (x2 + 3 * uy * ux + y2) * c2 - 6 * x2 * y2) / (36 * c4);
    f[8] = rho * (c4 + 3 * (ux - uy) * c3 + 2 * (x2 - 3 * uy * ux + y2) * c2 - 6 * x2 * y2) / (36 * c4);
    f[9] = rho * (c4 - 3 * (ux - uy) * c3 + 2 * (x2 - 3 * uy * ux + y2) * c2 - 6 * x2 * y2) / (36 * c4);
    f[10] = rho * (c4 - 3 * (ux + uy) * c3 + 2 * (x2 + 3 * uy * ux + y2) * c2 - 6 * x2 * y2) / (36 * c4);
    f[11] = rho * (c4 + 3 * (ux + uz) * c3 + 2 * (x2 + 3 * uz * ux + z2) * c2 - 6 * x2 * z2) / (36 * c4);
    f[12] = rho * (c4 + 3 * (ux - uz) * c3 + 2 * (x2 - 3 * uz * ux + z2) * c2 - 6 * x2 * z2) / (36 * c4);
    f[13] = rho * (c4 - 3 * (ux - uz) * c3 + 2 * (x2 - 3 * uz * ux + z2) * c2 - 6 * x2 * z2) / (36 * c4);
    f[14] = rho * (c4 - 3 * (ux + uz) * c3 + 2 * (x2 + 3 * uz * ux + z2) * c2 - 6 * x2 * z2) / (36 * c4);
    f[15] = rho * (c4 + 3 * (uy + uz) * c3 + 2 * (y2 + 3 * uz * uy + z2) * c2 - 6 * y2 * z2) / (36 * c4);
    f[16] = rho * (c4 + 3 * (uy - uz) * c3 + 2 * (y2 - 3 * uz * uy + z2) * c2 - 6 * y2 * z2) / (36 * c4);
    f[17] = rho * (c4 - 3 * (uy - uz) * c3 + 2 * (y2 - 3 * uz * uy + z2) * c2 - 6 * y2 * z2) / (36 * c4);
    f[18] = rho * (c4 - 3 * (uy + uz) * c3 + 2 * (y2 + 3 * uz * uy + z2) * c2 - 6 * y2 * z2) / (36 * c4);
}

/* Equilibrium variance, Appendix A (the P = rho T delta case of Eq. 36). Order xx yy zz xy xz yz. */
void orc_beq(double ux, double uy, double uz, double T, double *b)
{
    const double c = 1.0;
    b[0] = (-c * c + ux * ux + 3 * T) / 3.0;
    b[1] = (-c * c + uy * uy + 3 * T) / 3.0;
    b[2] = (-c * c + uz * uz + 3 * T) / 3.0;
    b[3] = ux * uy / 3.0;
    b[4] = ux * uz / 3.0;
    b[5] = uy * uz / 3.0;
}

/* ---------------------------------------------------------------------------------------------
 * Table I of Appendix B (population-to-moment transformation), c = 1, row a, column i.
 * ------------------------------------------------------------------------------------------- */
static const double T3 = 1.0 / 3.0, T23 = 2.0 / 3.0, T6 = 1.0 / 6.0;
static const double TABLE_M[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0},
    {0, 0, 1, 0, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1},
    {-T3, T23, -T3, T23, -T3, -T3, -T3, T23, T23, T23, T23, T23, T23, T23, T23, -T3, -T3, -T3, -T3},
    {-T3, -T3, T23, -T3, T23, -T3, -T3, T23, T23, T23, T23, -T3, -T3, -T3, -T3, T23, T23, T23, T23},
    {-T3, -T3, -T3, -T3, -T3, T23, T23, -T3, -T3, -T3, -T3, T23, T23, T23, T23, T23, T23, T23, T23},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, -T23, 0, T23, 0, 0, 0, T3, T3, -T3, -T3, T3, T3, -T3, -T3, 0, 0, 0, 0},
    {0, 0, -T23, 0, T23, 0, 0, T3, -T3, T3, -T3, 0, 0, 0, 0, T3, T3, -T3, -T3},
    {0, 0, 0, 0, 0, -T23, T23, 0, 0, 0, 0, T3, -T3, T3, -T3, T3, -T3, T3, -T3},
    {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, -1, -1, 1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, -1, -1, 1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1},
    {0, 0.5, 0.5, 0.5, 0.5, -1, -1, -1, -1, -1, -1, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5, 0.5},
    {0, 0.5, -0.5, 0.5, -0.5, 0, 0, 0, 0, 0, 0, -0.5, -0.5, -0.5, -0.5, 0.5, 0.5, 0.5, 0.5},
    {T6, -T3, -T3, -T3, -T3, -T3, -T3, T6, T6, T6, T6, T6, T6, T6, T6, T6, T6, T6, T6},
};

void orc_table_m(double *m)
{
    for (int a = 0; a < Q; a++)
        for (int i = 0; i < Q; i++) m[a * Q + i] = TABLE_M[a][i];
}

/* Forcing populations from their moments (Eqs. 58-61): the moment vector in the Table I basis is
 * (0, F, S_xx, S_yy, S_zz, S_xy, S_xz, S_yz, 0, ..., 0) -- rows 4-6 of Table I are e_a^2 - 1/3,
 * whose Phi-moment is S_aa because sum Phi = 0 -- and Phi_i = w_i sum_a m^a_i N^a M^a with
 * N^a = 1 / sum_j w_j (m^a_j)^2 (Eq. B2; this inverse holds because the rows are orthogonal under
 * the weights w).  S is ordered xx yy zz xy xz yz. */
void orc_forcing(const double *Fv, const double *S, double *phi)
{
    double mom[Q];
    for (int a = 0; a < Q; a++) mom[a] = 0.0;
    mom[1] = Fv[0];
    mom[2] = Fv[1];
    mom[3] = Fv[2];
    mom[4] = S[0];
    mom[5] = S[1];
    mom[6] = S[2];
    mom[7] = S[3];
    mom[8] = S[4];
    mom[9] = S[5];
    for (int i = 0; i < Q; i++) phi[i] = 0.0;
    for (int a = 0; a < Q; a++) {
        if (mom[a] == 0.0) continue; /* rows with a zero moment add nothing */
        double norm = 0.0;
        for (int j = 0; j < Q; j++) norm += W[j] * TABLE_M[a][j] * TABLE_M[a][j];
        double Na = 1.0 / norm;
        for (int i = 0; i < Q; i++) phi[i] += W[i] * TABLE_M[a][i] * Na * mom[a];
    }
}

/* ---------------------------------------------------------------------------------------------
 * Lattice helpers.
 * ------------------------------------------------------------------------------------------- */
static long site(int nx, int ny, int x, int y, int z) { return ((long)z * ny + y) * nx + x; }

static int wrap(int v, int n) { return ((v % n) + n) % n; }

/* Flat indices of the 19 sites x + e_i (periodic), e_0 = 0 first. */
static void neighbours(int nx, int ny, int nz, int x, int y, int z, long *nbr)
{
    for (int i = 0; i < Q; i++)
        nbr[i] = site(nx, ny, wrap(x + E[i][0], nx), wrap(y + E[i][1], ny), wrap(z + E[i][2], nz));
}

/* Index of the velocity -e_i. */
static int opp(int i)
{
    for (int j = 0; j < Q; j++)
        if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1] && E[j][2] == -E[i][2]) return j;
    return -1;
}

/* phi at (x, y, z) with x, y periodic and z either periodic (walls = 0) or bounded by the two
 * walls (walls = 1): one plane beyond a wall is the mirror image of the wall-adjacent plane
 * (extrap = 0) or extrapolated from the three planes inside it (extrap = 1). */
static double value_at(const double *phi, int nx, int ny, int nz, int walls, int extrap, int x, int y, int z)
{
    x = wrap(x, nx);
    y = wrap(y, ny);
    if (!walls) return phi[site(nx, ny, x, y, wrap(z, nz))];
    if (z < 0 || z >= nz) {
        const int z0 = z < 0 ? 0 : nz - 1, d = z < 0 ? 1 : -1;
        const double p0 = phi[site(nx, ny, x, y, z0)];
        if (!extrap) return p0;
        return 3.0 * p0 - 3.0 * phi[site(nx, ny, x, y, z0 + d)] + phi[site(nx, ny, x, y, z0 + 2 * d)];
    }
    return phi[site(nx, ny, x, y, z)];
}

/* The stencil below with the neighbour values from value_at (used when walls bound z). */
static double fd_walls(const double *phi, int nx, int ny, int nz, int extrap, int x, int y, int z, int a)
{
    double s = 0.0;
    for (int i = 1; i < Q; i++) {
        if (E[i][a] == 0) continue;
        s += W[i] * E[i][a] * value_at(phi, nx, ny, nz, 1, extrap, x + E[i][0], y + E[i][1], z + E[i][2]);
    }
    return 3.0 * s;
}

/* Isotropic finite difference d_a phi(x) = (1/cs^2) sum_i w_i e_ia phi(x + e_i), cs^2 = 1/3,
 * over the 18 D3Q19 neighbours (nbr from neighbours()). */
static double fd(const double *phi, const long *nbr, int a)
{
    double s = 0.0;
    for (int i = 1; i < Q; i++) {
        if (E[i][a] == 0) continue;
        s += W[i] * E[i][a] * phi[nbr[i]];
    }
    return 3.0 * s;
}

/* Public wrapper of the stencil for the tests: out[n] = d_a phi at every site. */
void orc_gradient(int nx, int ny, int nz, const double *phi, int a, double *out)
{
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long nbr[Q];
                neighbours(nx, ny, nz, x, y, z, nbr);
                out[site(nx, ny, x, y, z)] = fd(phi, nbr, a);
            }
}

/* Predictor moments at one site from the post-stream state (step 1). */
typedef struct {
    double rho, j[3], u[3], Pi[6], trb, T, b[6];
} predictor;

static void predict(const double *Fsite /*19*/, const double *bbar /*6*/, double Tiso, int iso,
                    double omega, predictor *p)
{
    p->rho = 0.0;
    for (int a = 0; a < 3; a++) p->j[a] = 0.0;
    for (int k = 0; k < NB; k++) p->Pi[k] = 0.0;
    for (int i = 0; i < Q; i++) {
        p->rho += Fsite[i];
        for (int a = 0; a < 3; a++) p->j[a] += Fsite[i] * E[i][a];
        for (int k = 0; k < NB; k++) p->Pi[k] += Fsite[i] * E[i][BA[k]] * E[i][BB[k]];
    }
    for (int a = 0; a < 3; a++) p->u[a] = p->j[a] / p->rho;
    p->trb = bbar[0] + bbar[1] + bbar[2];
    if (iso) {
        p->T = Tiso;
    } else {
        double trPi = p->Pi[0] + p->Pi[1] + p->Pi[2];
        double u2 = p->u[0] * p->u[0] + p->u[1] * p->u[1] + p->u[2] * p->u[2];
        p->T = (trPi + p->rho * p->trb - p->rho * u2) / (3.0 * p->rho);
    }
    double beq[6];
    orc_beq(p->u[0], p->u[1], p->u[2], p->T, beq);
    for (int k = 0; k < NB; k++) p->b[k] = bbar[k] - 0.5 * omega * (bbar[k] - beq[k]);
}

/* Gradient sources over the whole lattice: src[0..5] = R_k = rho b_k and, for the second-moment
 * forcing, the products rho u*_g b_ab stored as src[6 + 3k + g]. */
#define NSRC (NB + 3 * NB)
static void sources(int nx, int ny, int nz, double tau, int mode, const double *Tf, const double *F,
                    const double *b, double *src /* NSRC * n */)
{
    const long n = (long)nx * ny * nz;
    const double omega = 1.0 / (tau + 0.5);
#pragma omp parallel for schedule(static)
    for (long s = 0; s < n; s++) {
        double Fs[Q], bs[NB];
        for (int i = 0; i < Q; i++) Fs[i] = F[i * n + s];
        for (int k = 0; k < NB; k++) bs[k] = b[k * n + s];
        predictor p;
        predict(Fs, bs, mode ? Tf[s] : 0.0, mode, omega, &p);
        for (int k = 0; k < NB; k++) {
            src[k * n + s] = p.rho * p.b[k];
            for (int g = 0; g < 3; g++) src[(NB + 3 * k + g) * n + s] = p.rho * p.u[g] * p.b[k];
        }
    }
}

/* Corrected moments at one site (steps 1-3): rho, u, T and the forcing moments F, S. */
typedef struct {
    double rho, u[3], T, Fv[3], S[6];
    predictor p;
} corrected;

/* accel: a body-force acceleration field (3 planes) or NULL.  It enters the forcing moments in
 * the manner of a Guo forcing: F += rho a, S += rho (u a + a u) with the corrected u, which then
 * carries half of rho a as well (Eq. 57); the predictor sources stay force-free (as the paper
 * keeps the uncorrected u there). */
static void correct(int nx, int ny, int nz, double tau, int mode, const double *Tf, const double *accel,
                    int walls, const double *F, const double *b, const double *src, int x, int y, int z,
                    corrected *c)
{
    const long n = (long)nx * ny * nz;
    const long s = site(nx, ny, x, y, z);
    const double omega = 1.0 / (tau + 0.5);
    double Fs[Q], bs[NB];
    for (int i = 0; i < Q; i++) Fs[i] = F[i * n + s];
    for (int k = 0; k < NB; k++) bs[k] = b[k * n + s];
    predict(Fs, bs, mode ? Tf[s] : 0.0, mode, omega, &c->p);
    long nbr[Q];
    neighbours(nx, ny, nz, x, y, z, nbr);
#define D(plane, a) (walls ? fd_walls(src + (long)(plane) * n, nx, ny, nz, (plane) >= NB, x, y, z, a) \
                           : fd(src + (long)(plane) * n, nbr, a))

    /* F_b = - d_a (rho b_ab)  (Eq. 59) */
    for (int bb = 0; bb < 3; bb++) {
        double acc = 0.0;
        for (int a = 0; a < 3; a++) acc += D(comp(a, bb), a);
        c->Fv[bb] = -acc;
    }
    /* S_bg = - d_a (rho u_g b_ab + rho u_b b_ga)  (Eq. 61) */
    for (int k = 0; k < NB; k++) {
        int bb = BA[k], g = BB[k];
        double acc = 0.0;
        for (int a = 0; a < 3; a++) {
            acc += D(NB + 3 * comp(a, bb) + g, a);
            acc += D(NB + 3 * comp(g, a) + bb, a);
        }
        c->S[k] = -acc;
    }
#undef D
    c->rho = c->p.rho;
    if (accel)
        for (int a = 0; a < 3; a++) c->Fv[a] += c->rho * accel[a * n + s];
    for (int a = 0; a < 3; a++) c->u[a] = (c->p.j[a] + 0.5 * c->Fv[a]) / c->rho; /* Eq. 57 */
    if (accel)
        for (int k = 0; k < NB; k++) {
            const int bb = BA[k], g = BB[k];
            c->S[k] += c->rho * (c->u[bb] * accel[g * n + s] + c->u[g] * accel[bb * n + s]);
        }
    if (mode) {
        c->T = Tf[s];
    } else {
        double trPi = c->p.Pi[0] + c->p.Pi[1] + c->p.Pi[2];
        double trS = c->S[0] + c->S[1] + c->S[2];
        double u2 = c->u[0] * c->u[0] + c->u[1] * c->u[1] + c->u[2] * c->u[2];
        c->T = (trPi + c->rho * c->p.trb + 0.5 * trS - c->rho * u2) / (3.0 * c->rho);
    }
}

/* Collision at one site (steps 4-5): post-collision fbar* (19) and bbar* (6).
 *
 * omega_g: relaxation factor of the nine non-hydrodynamic moments, rows 11-19 of Table I
 * (omega_g = omega is the single-relaxation-time step of Eq. 55).  With a collision matrix
 * L = M^-1 diag(lambda_a) M in the Table I basis, the general update of the auxiliary populations
 * (the form with (I + L dt/2)^-1 that leads to Eq. 55) relaxes moment a with
 * omega_a = lambda_a / (1 + lambda_a / 2) and weighs its forcing moment with 1 - omega_a / 2.
 * Rows 1-10 (rho, j, the second moments) keep omega, and Phi has no components on rows 11-19,
 * so this differs from the single-rate update only by (omega - omega_g) (m_a - m_a^eq) on those
 * rows, mapped back with the inverse of Table I (w_i m^a_i N^a, as in orc_forcing). */
static void collide(const double *Fs, const double *bs, const corrected *c, double omega, double omega_g,
                    double *Fpost, double *bpost)
{
    double feq[Q], beq[NB], phi[Q];
    orc_feq(c->rho, c->u[0], c->u[1], c->u[2], feq);
    orc_beq(c->u[0], c->u[1], c->u[2], c->T, beq);
    orc_forcing(c->Fv, c->S, phi);
    for (int i = 0; i < Q; i++)
        Fpost[i] = Fs[i] - omega * (Fs[i] - feq[i]) + (1.0 - 0.5 * omega) * phi[i];
    if (omega_g != omega) {
        for (int a = 10; a < Q; a++) {
            double ma = 0.0, norm = 0.0;
            for (int i = 0; i < Q; i++) {
                ma += TABLE_M[a][i] * (Fs[i] - feq[i]);
                norm += W[i] * TABLE_M[a][i] * TABLE_M[a][i];
            }
            for (int i = 0; i < Q; i++) Fpost[i] += W[i] * TABLE_M[a][i] / norm * (omega - omega_g) * ma;
        }
    }
    for (int k = 0; k < NB; k++) bpost[k] = bs[k] - omega * (bs[k] - beq[k]);
}

/* ---------------------------------------------------------------------------------------------
 * Public entry points (all arrays owned by the caller).
 * ------------------------------------------------------------------------------------------- */

/* Initialisation: fbar = feq(rho0, u0), bbar = beq(u0, T0) at every site. u is 3 planes. */
void orc_init(int nx, int ny, int nz, const double *rho, const double *u, const double *T, double *F,
              double *b)
{
    const long n = (long)nx * ny * nz;
    for (long s = 0; s < n; s++) {
        double feq[Q], beq[NB];
        orc_feq(rho[s], u[s], u[n + s], u[2 * n + s], feq);
        orc_beq(u[s], u[n + s], u[2 * n + s], T[s], beq);
        for (int i = 0; i < Q; i++) F[i * n + s] = feq[i];
        for (int k = 0; k < NB; k++) b[k * n + s] = beq[k];
    }
}

/* Wall velocities uw = (u_b, u_t) must be tangential, and the extrapolation needs 3 planes. */
static int walls_invalid(int nz, const double *uw)
{
    return uw && (nz < 3 || uw[2] != 0.0 || uw[5] != 0.0);
}

/* nsteps full steps in place. mode 0 = energy-conserving temperature, 1 = prescribed T field.
 * tau_ghost: relaxation time of the non-hydrodynamic moments (rows 11-19 of Table I; see
 * collide); tau_ghost = tau is the single-relaxation-time scheme of the paper.
 * uw: NULL (periodic in z) or the bottom and top wall velocities (6 values; see the header). */
int orc_step_walls(int nx, int ny, int nz, double tau, double tau_ghost, int mode, const double *Tf,
                   const double *accel, const double *uw, double *F, double *b, long nsteps)
{
    const long n = (long)nx * ny * nz;
    const double omega = 1.0 / (tau + 0.5);
    const double omega_g = tau_ghost == tau ? omega : 1.0 / (tau_ghost + 0.5);
    const int walls = uw != NULL;
    if (walls_invalid(nz, uw)) return -3;
    double *src = malloc(sizeof(double) * NSRC * n);
    double *Fp = malloc(sizeof(double) * Q * n);
    double *bp = malloc(sizeof(double) * NB * n);
    double *rp = malloc(sizeof(double) * n);
    if (!src || !Fp || !bp || !rp) {
        free(src);
        free(Fp);
        free(bp);
        free(rp);
        return -1;
    }
    for (long it = 0; it < nsteps; it++) {
        sources(nx, ny, nz, tau, mode, Tf, F, b, src);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    long s = site(nx, ny, x, y, z);
                    corrected c;
                    correct(nx, ny, nz, tau, mode, Tf, accel, walls, F, b, src, x, y, z, &c);
                    double Fs[Q], bs[NB], Fo[Q], bo[NB];
                    for (int i = 0; i < Q; i++) Fs[i] = F[i * n + s];
                    for (int k = 0; k < NB; k++) bs[k] = b[k * n + s];
                    collide(Fs, bs, &c, omega, omega_g, Fo, bo);
                    for (int i = 0; i < Q; i++) Fp[i * n + s] = Fo[i];
                    for (int k = 0; k < NB; k++) bp[k * n + s] = bo[k];
                    rp[s] = c.rho;
                }
        /* step 6: stream and gather */
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    long s = site(nx, ny, x, y, z);
                    double rho = 0.0, acc[NB] = {0, 0, 0, 0, 0, 0};
                    for (int i = 0; i < Q; i++) {
                        const int zf = z - E[i][2];
                        long from;
                        double fi;
                        if (walls && (zf < 0 || zf >= nz)) {
                            /* bounce-back: the population that left x towards the wall */
                            const double *u_w = zf < 0 ? uw : uw + 3;
                            from = s;
                            fi = Fp[opp(i) * n + s] +
                                 6.0 * W[i] * rp[s] * (E[i][0] * u_w[0] + E[i][1] * u_w[1] + E[i][2] * u_w[2]);
                        } else {
                            from = site(nx, ny, wrap(x - E[i][0], nx), wrap(y - E[i][1], ny), wrap(zf, nz));
                            fi = Fp[i * n + from];
                        }
                        F[i * n + s] = fi;
                        rho += fi;
                        for (int k = 0; k < NB; k++) acc[k] += fi * bp[k * n + from];
                    }
                    for (int k = 0; k < NB; k++) b[k * n + s] = acc[k] / rho;
                }
    }
    free(src);
    free(Fp);
    free(bp);
    free(rp);
    return 0;
}

/* Periodic in all three directions. */
int orc_step_ext(int nx, int ny, int nz, double tau, double tau_ghost, int mode, const double *Tf,
                 const double *accel, double *F, double *b, long nsteps)
{
    return orc_step_walls(nx, ny, nz, tau, tau_ghost, mode, Tf, accel, NULL, F, b, nsteps);
}

/* The same without a body force. */
int orc_step_mrt(int nx, int ny, int nz, double tau, double tau_ghost, int mode, const double *Tf, double *F,
                 double *b, long nsteps)
{
    return orc_step_ext(nx, ny, nz, tau, tau_ghost, mode, Tf, NULL, F, b, nsteps);
}

/* nsteps single-relaxation-time steps (Eq. 55) in place. */
int orc_step(int nx, int ny, int nz, double tau, int mode, const double *Tf, double *F, double *b,
             long nsteps)
{
    return orc_step_mrt(nx, ny, nz, tau, tau, mode, Tf, F, b, nsteps);
}

/* Reported moments of the current state: rho, corrected u (3 planes), T (steps 1-3).
 * walls: nonzero when walls bound z (only the gradient stencil depends on it). */
int orc_moments_walls(int nx, int ny, int nz, double tau, int mode, const double *Tf, const double *accel,
                      int walls, const double *F, const double *b, double *rho, double *u, double *T)
{
    const long n = (long)nx * ny * nz;
    if (walls && nz < 3) return -3;
    double *src = malloc(sizeof(double) * NSRC * n);
    if (!src) return -1;
    sources(nx, ny, nz, tau, mode, Tf, F, b, src);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(nx, ny, x, y, z);
                corrected c;
                correct(nx, ny, nz, tau, mode, Tf, accel, walls, F, b, src, x, y, z, &c);
                rho[s] = c.rho;
                for (int a = 0; a < 3; a++) u[a * n + s] = c.u[a];
                T[s] = c.T;
            }
    free(src);
    return 0;
}

int orc_moments_ext(int nx, int ny, int nz, double tau, int mode, const double *Tf, const double *accel,
                    const double *F, const double *b, double *rho, double *u, double *T)
{
    return orc_moments_walls(nx, ny, nz, tau, mode, Tf, accel, 0, F, b, rho, u, T);
}

int orc_moments(int nx, int ny, int nz, double tau, int mode, const double *Tf, const double *F,
                const double *b, double *rho, double *u, double *T)
{
    return orc_moments_ext(nx, ny, nz, tau, mode, Tf, NULL, F, b, rho, u, T);
}

/* Forcing moments F (3 planes) and S (6 planes) of the current state, for the tests. */
int orc_forcing_moments(int nx, int ny, int nz, double tau, int mode, const double *Tf,
                        const double *F, const double *b, double *Fv, double *S)
{
    const long n = (long)nx * ny * nz;
    double *src = malloc(sizeof(double) * NSRC * n);
    if (!src) return -1;
    sources(nx, ny, nz, tau, mode, Tf, F, b, src);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                long s = site(nx, ny, x, y, z);
                corrected c;
                correct(nx, ny, nz, tau, mode, Tf, NULL, 0, F, b, src, x, y, z, &c);
                for (int a = 0; a < 3; a++) Fv[a * n + s] = c.Fv[a];
                for (int k = 0; k < NB; k++) S[k * n + s] = c.S[k];
            }
    free(src);
    return 0;
}

/* Global invariants of the auxiliary state: mass, momentum (3), energy
 * E = 1/2 sum_x (sum_i fbar_i |e_i|^2 + rho tr bbar)  (second moment trace of Eq. 26). */
void orc_invariants(int nx, int ny, int nz, const double *F, const double *b, double *out)
{
    const long n = (long)nx * ny * nz;
    for (int k = 0; k < 5; k++) out[k] = 0.0;
    for (long s = 0; s < n; s++) {
        double rho = 0.0, e2 = 0.0;
        for (int i = 0; i < Q; i++) {
            double fi = F[i * n + s];
            rho += fi;
            out[1] += fi * E[i][0];
            out[2] += fi * E[i][1];
            out[3] += fi * E[i][2];
            e2 += fi * (E[i][0] * E[i][0] + E[i][1] * E[i][1] + E[i][2] * E[i][2]);
        }
        out[0] += rho;
        out[4] += 0.5 * (e2 + rho * (b[s] + b[n + s] + b[2 * n + s]));
    }
}

/* One step evaluated only at the listed sites of a full-size state, without stepping the rest:
 * Fout[19*m], bout[6*m] receive the post-stream state after one step at sites[m]; if bstar is
 * not NULL, bstar[6*m] receives the post-collision bbar*(x) at the site itself (before it is
 * carried along, i.e. the i = 0 upstream term).  The output at
 * x needs the collision at the 19 upstream sites x - e_i, and each of those needs the gradient
 * sources one hop further, so a 5x5x5 copy of the state centred on x (periodic wrap applied when
 * copying) holds everything; the same per-site functions as orc_step run on that copy, whose
 * own wrap-around is never read for the centre's result. */
int orc_step_sites(int nx, int ny, int nz, double tau, int mode, const double *Tf, const double *F,
                   const double *b, long nsites, const long *sites, double *Fout, double *bout, double *bstar)
{
    const long n = (long)nx * ny * nz;
    const int L = 5;
    const long nb = (long)L * L * L;
    const double omega = 1.0 / (tau + 0.5);
    double *Fb = malloc(sizeof(double) * Q * nb);
    double *bb = malloc(sizeof(double) * NB * nb);
    double *Tb = malloc(sizeof(double) * nb);
    double *src = malloc(sizeof(double) * NSRC * nb);
    if (!Fb || !bb || !Tb || !src) {
        free(Fb);
        free(bb);
        free(Tb);
        free(src);
        return -1;
    }
    for (long m = 0; m < nsites; m++) {
        long s0 = sites[m];
        if (s0 < 0 || s0 >= n) {
            free(Fb);
            free(bb);
            free(Tb);
            free(src);
            return -2;
        }
        int x0 = (int)(s0 % nx), y0 = (int)((s0 / nx) % ny), z0 = (int)(s0 / ((long)nx * ny));
        for (int dz = 0; dz < L; dz++)
            for (int dy = 0; dy < L; dy++)
                for (int dx = 0; dx < L; dx++) {
                    long g = site(nx, ny, wrap(x0 + dx - 2, nx), wrap(y0 + dy - 2, ny), wrap(z0 + dz - 2, nz));
                    long l = site(L, L, dx, dy, dz);
                    for (int i = 0; i < Q; i++) Fb[i * nb + l] = F[i * n + g];
                    for (int k = 0; k < NB; k++) bb[k * nb + l] = b[k * n + g];
                    Tb[l] = mode ? Tf[g] : 0.0;
                }
        sources(L, L, L, tau, mode, Tb, Fb, bb, src);
        double rho = 0.0, acc[NB] = {0, 0, 0, 0, 0, 0};
        for (int i = 0; i < Q; i++) {
            int xu = 2 - E[i][0], yu = 2 - E[i][1], zu = 2 - E[i][2];
            long su = site(L, L, xu, yu, zu);
            corrected c;
            correct(L, L, L, tau, mode, Tb, NULL, 0, Fb, bb, src, xu, yu, zu, &c);
            double Fs[Q], bs[NB], Fo[Q], bo[NB];
            for (int q = 0; q < Q; q++) Fs[q] = Fb[q * nb + su];
            for (int k = 0; k < NB; k++) bs[k] = bb[k * nb + su];
            collide(Fs, bs, &c, omega, omega, Fo, bo);
            Fout[m * Q + i] = Fo[i];
            rho += Fo[i];
            for (int k = 0; k < NB; k++) acc[k] += Fo[i] * bo[k];
            if (i == 0 && bstar)
                for (int k = 0; k < NB; k++) bstar[m * NB + k] = bo[k];
        }
        for (int k = 0; k < NB; k++) bout[m * NB + k] = acc[k] / rho;
    }
    free(Fb);
    free(bb);
    free(Tb);
    free(src);
    return 0;
}


/* ---------------------------------------------------------------------------------------------
 * Standard lattice Boltzmann comparator (Sec. I, Eq. 4): D3Q19 populations without a variance,
 * equilibrium = the second-order Hermite expansion of the Maxwell-Boltzmann distribution at
 * temperature T, written in lattice units (c = 1, so 1/c_s^2 = 3 and the Hermite temperature
 * offset is T - 1/3):
 *     feq_i = rho w_i [1 + 3 e_i.u + 9/2 (u_a u_b + (T - 1/3) delta_ab)(e_ia e_ib - delta_ab/3)].
 * The paper uses it as the contrast to the bump scheme in the Galilean-invariance experiment of
 * Sec. III C.  One step: BGK with the same relaxation factor omega = 1/(tau + 1/2) (Eq. 55),
 * then streaming; T is a prescribed field.  A body force enters as in the bump scheme: the
 * forcing Phi built from F = rho a and S = rho (u a + a u) (orc_forcing), weighted by
 * 1 - omega/2, with u = (j + F/2)/rho; there is no gradient forcing (no variance).  The walls
 * are those of the bump scheme (half-way bounce-back with the moving-wall momentum
 * 6 w_i rho e_i.u_w, which is also the odd part of this equilibrium).
 * ------------------------------------------------------------------------------------------- */
void orc_feq_std(double rho, double ux, double uy, double uz, double T, double *f)
{
    const double u[3] = {ux, uy, uz};
    for (int i = 0; i < Q; i++) {
        double eu = 0.0, second = 0.0;
        for (int a = 0; a < 3; a++) eu += E[i][a] * u[a];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                const double d = a == b ? 1.0 : 0.0;
                second += (u[a] * u[b] + (T - 1.0 / 3.0) * d) * (E[i][a] * E[i][b] - d / 3.0);
            }
        f[i] = rho * W[i] * (1.0 + 3.0 * eu + 4.5 * second);
    }
}

void orc_init_std(int nx, int ny, int nz, const double *rho, const double *u, const double *T, double *F)
{
    const long n = (long)nx * ny * nz;
    for (long s = 0; s < n; s++) {
        double feq[Q];
        orc_feq_std(rho[s], u[s], u[n + s], u[2 * n + s], T[s], feq);
        for (int i = 0; i < Q; i++) F[i * n + s] = feq[i];
    }
}

/* Velocity of the standard model at one site: (j + rho a / 2) / rho, a = accel or none. */
static void std_velocity(const double *Fsite, const double *a, double *rho, double *u)
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; i++) {
        r += Fsite[i];
        for (int c = 0; c < 3; c++) j[c] += Fsite[i] * E[i][c];
    }
    *rho = r;
    for (int c = 0; c < 3; c++) u[c] = (j[c] + (a ? 0.5 * r * a[c] : 0.0)) / r;
}

int orc_step_std_walls(int nx, int ny, int nz, double tau, const double *Tf, const double *accel,
                       const double *uw, double *F, long nsteps)
{
    const long n = (long)nx * ny * nz;
    const double omega = 1.0 / (tau + 0.5);
    const int walls = uw != NULL;
    if (uw && (uw[2] != 0.0 || uw[5] != 0.0)) return -3;
    double *Fp = malloc(sizeof(double) * Q * n);
    double *rp = malloc(sizeof(double) * n);
    if (!Fp || !rp) {
        free(Fp);
        free(rp);
        return -1;
    }
    for (long it = 0; it < nsteps; it++) {
#pragma omp parallel for schedule(static)
        for (long s = 0; s < n; s++) {
            double Fs[Q], a[3], rho, u[3], feq[Q], phi[Q];
            for (int i = 0; i < Q; i++) Fs[i] = F[i * n + s];
            if (accel)
                for (int c = 0; c < 3; c++) a[c] = accel[c * n + s];
            std_velocity(Fs, accel ? a : NULL, &rho, u);
            orc_feq_std(rho, u[0], u[1], u[2], Tf[s], feq);
            for (int i = 0; i < Q; i++) phi[i] = 0.0;
            if (accel) {
                const double Fv[3] = {rho * a[0], rho * a[1], rho * a[2]};
                double S[NB];
                for (int k = 0; k < NB; k++) S[k] = rho * (u[BA[k]] * a[BB[k]] + u[BB[k]] * a[BA[k]]);
                orc_forcing(Fv, S, phi);
            }
            for (int i = 0; i < Q; i++) Fp[i * n + s] = Fs[i] - omega * (Fs[i] - feq[i]) + (1.0 - 0.5 * omega) * phi[i];
            rp[s] = rho;
        }
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    const long s = site(nx, ny, x, y, z);
                    for (int i = 0; i < Q; i++) {
                        const int zf = z - E[i][2];
                        if (walls && (zf < 0 || zf >= nz)) {
                            const double *u_w = zf < 0 ? uw : uw + 3;
                            F[i * n + s] = Fp[opp(i) * n + s] +
                                           6.0 * W[i] * rp[s] * (E[i][0] * u_w[0] + E[i][1] * u_w[1] + E[i][2] * u_w[2]);
                        } else {
                            F[i * n + s] = Fp[i * n + site(nx, ny, wrap(x - E[i][0], nx), wrap(y - E[i][1], ny), wrap(zf, nz))];
                        }
                    }
                }
    }
    free(Fp);
    free(rp);
    return 0;
}

int orc_step_std(int nx, int ny, int nz, double tau, const double *Tf, double *F, long nsteps)
{
    return orc_step_std_walls(nx, ny, nz, tau, Tf, NULL, NULL, F, nsteps);
}

/* Moments of the standard model: rho = sum f, u = (sum f e + rho a / 2) / rho (accel or NULL). */
void orc_moments_std_ext(int nx, int ny, int nz, const double *accel, const double *F, double *rho, double *u)
{
    const long n = (long)nx * ny * nz;
    for (long s = 0; s < n; s++) {
        double Fs[Q], a[3], uu[3];
        for (int i = 0; i < Q; i++) Fs[i] = F[i * n + s];
        if (accel)
            for (int c = 0; c < 3; c++) a[c] = accel[c * n + s];
        std_velocity(Fs, accel ? a : NULL, rho + s, uu);
        for (int c = 0; c < 3; c++) u[c * n + s] = uu[c];
    }
}

void orc_moments_std(int nx, int ny, int nz, const double *F, double *rho, double *u)
{
    orc_moments_std_ext(nx, ny, nz, NULL, F, rho, u);
}
