/*
 * lbfd_oracle.c -- plain, slow FP64 CPU reference ("the oracle") of one time
 * step of the hybrid lattice-Boltzmann colour-gradient / finite-difference
 * method for two-phase flow with soluble surfactants of Ba, Liu, Li and Yang
 * (arXiv 2311.15242).
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only users of this library. The
 * product path (the HIP library) shares no code, header, table or generator
 * with it, and neither side includes or loads the other.
 *
 * Every routine follows the paper passage named in its comment, in the paper's
 * order and notation. There is no blocking, fusion or reordering: the lattice
 * matrices are the printed ones (Appendix A, eqs 36 and 39), M^-1 is obtained
 * by Gauss-Jordan elimination at start-up, and the moment-space products are
 * dense loops. OpenMP only splits loops over independent nodes; every global
 * sum is a serial loop in node order, and the implicit solve is plain
 * lexicographic SOR. Where the paper is silent or garbled the choice made is
 * marked "Reading:" in place.
 *
 * Pins: the tests check this library against closed forms, invariants, a
 * separately written NumPy brute force and exact dense solves. Parity partly
 * pinned: rows 16-18 of the 3-D moment equilibrium (eq 40) beyond u = 0
 * (pinned at u = 0 and by covariance under the lattice symmetries only).
 * The rescaling of the total surfactant (Sec 2.2 cites it without giving it)
 * is pinned to its reading: one factor for psi and phi from the new level's
 * weights, checked against the factor summed from an unrescaled step.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define QMAX 19

/* ---------------------------------------------------------------- params */

typedef struct {
    int32_t lattice;          /* 0 = D2Q9, 1 = D3Q19 (Sec 2.1) */
    int32_t nx, ny, nz;       /* nz = 1 in 2-D */
    int32_t bc[3];            /* per axis: 0 periodic, 1 half-way bounce-back walls on both faces */
    double wall_u[6][3];      /* velocity of the walls at -x,+x,-y,+y,-z,+z */
    double rhoR0, rhoB0;      /* pure-fluid densities (eq 6) */
    double muR0, muB0;        /* pure-fluid dynamic viscosities (eq 43) */
    double alphaR;            /* free sound-speed parameter of red; alphaB from eq 42 */
    double beta;              /* recolouring segregation parameter (0.7, Sec 2.1) */
    double sigma0, E0, psi_inf, sigma_min_ratio; /* modified Langmuir EOS (eq 8) */
    double Ds, Db, ra, rd;    /* diffusivities, adsorption/desorption coefficients (eqs 20-22) */
    int32_t source_mode;      /* 0: j of eq 22; 1: adsorption-only j = ra psi_inf phi (Sec 3.1) */
    double gravity[3];        /* buoyancy F_b = (rho - rhoB0) gravity (Sec 3.4) */
    double sor_omega, sor_tol;
    int32_t sor_max_sweeps;
    double weno_eps;          /* epsilon of the WENO3 weights (1e-6, Sec 2.2) */
    int32_t rescale;          /* 1: restore the total surfactant after each step (Sec 2.2) */
    int32_t fd_enable;        /* 0: psi, phi frozen (LB only) */
    int32_t q_literal;        /* 3-D correction factor: 0 = [1 - 3 cs^2] (reading), 1 = printed [1 - cs^2] */
    double eps_n;             /* regularisation of the normal where |grad rhoN| -> 0 */
    int32_t recolour_literal; /* eq 11 weight: 0 = local rest equilibrium per unit density (reading), 1 = lattice w_i */
    double fd_eps;          /* background added to the FD weights G = |grad rhoN| and X = 1 - rhoN */
    double upwind_eps;      /* |u_a| at or below this takes both one-sided WENO differences by halves */
    int32_t buoyancy_ref;   /* F_b = (rho - rho_ref) g: 0 = rhoB0 as printed (Sec 3.4), 1 = the mean
                               density of the domain (no net force on a periodic domain) */
    int32_t eos_mode;       /* 0: Langmuir law of eq 8 with the CMC floor; 1: the linear law
                               sigma = sigma0 (1 - E0 psi / psi_inf) of Sec 3.2, no floor */
} orc_params;

typedef struct {
    int32_t n;                /* number of red drops/bubbles */
    double cx[16], cy[16], cz[16], r[16];
    double width;             /* tanh profile width W */
    double psi0, phi0_out, phi0_in;
    double shear_rate;        /* initial u_x = shear_rate * (y - (ny-1)/2) */
} orc_init_spec;

typedef struct {
    int64_t step;
    double mass_R, mass_B;
    double total_surf;        /* sum over nodes of (G psi + X phi), the conserved integrand of eqs 20-21 */
    double drift_pre;         /* relative change of total_surf in the last step before rescaling */
    double velocity[3];       /* sum u N / sum N with N of eq 34 (eq 33 per component) */
    double centroid[3];       /* weight (1 + rhoN)/2 */
    double second[6];         /* xx, yy, zz, xy, xz, yz central second moments, same weight */
    double wsum, nsum;
    double psi_av, psi_min, psi_max;
    double p_in, p_out;
    int32_t sor_sweeps[2];
    int32_t status;
} orc_obs;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ESOR = -5, ORC_ENONFINITE = -4 };

enum {
    FLD_F = 0, FLD_FR = 1, FLD_FB = 2, FLD_RHOR = 3, FLD_RHOB = 4, FLD_RHON = 5,
    FLD_U = 6, FLD_PSI = 7, FLD_PHI = 8, FLD_FORCE = 9, FLD_G = 10,
    FLD_SPREV = 11, FLD_BPREV = 12, FLD_KAPPA = 13
};

/* ---------------------------------------------------------------- lattices */

/* D2Q9 velocities in the column order of the printed M (eq 36). */
static const int E2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W2[9] = {4. / 9., 1. / 9., 1. / 9., 1. / 9., 1. / 9.,
                             1. / 36., 1. / 36., 1. / 36., 1. / 36.};
/* eq 36 */
static const int M2[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* D3Q19 velocities: the columns of rows 1-3 of the printed M (eq 39). */
static const int E3[19][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W3[19] = {1. / 3.,
                              1. / 18., 1. / 18., 1. / 18., 1. / 18., 1. / 18., 1. / 18.,
                              1. / 36., 1. / 36., 1. / 36., 1. / 36., 1. / 36., 1. / 36.,
                              1. / 36., 1. / 36., 1. / 36., 1. / 36., 1. / 36., 1. / 36.};
/* eq 39 */
static const int M3[19][19] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
    {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2},
    {0, 2, 2, -1, -1, -1, -1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
    {0, 0, 0, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1},
    {0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1}};

/* ---------------------------------------------------------------- state */

typedef struct orc_state {
    orc_params p;
    int Q, D;
    long nx, ny, nz, N;
    int e[QMAX][3];
    double w[QMAX];
    int opp[QMAX];
    double M[QMAX][QMAX], Minv[QMAX][QMAX];
    double alpha[2], cs2[2];  /* [0] red, [1] blue */
    double phi_rest[2][QMAX]; /* rest equilibrium of each colour per unit density, M^-1 m^eq(1, alpha^k, 0) */
    double *fR, *fB, *fR2, *fB2;
    double *psi, *phi, *Sprev, *Bprev;
    long step;
    double M0, drift_pre;
    int sweeps[2];
    /* work arrays of the force stage */
    double *rhoR, *rhoB, *rho, *rhoN, *j[3], *g[3], *G, *nrm[3], *kappa, *gpsi[3];
    double *F[3], *u[3], *sv, *ku[2][3], *dku[2][3];
    /* work arrays of the FD stage */
    double *rhoN1, *G1, *g1[3], *X0, *X1, *Psi[3], *Phi[3], *divPsi, *divPhi;
    double *S, *B, *rhsP, *rhsF, *tmp, *Gw;
    double *dump_fdag;        /* when set, the LB stage also stores f_dag here (Q x N) */
} orc_state;

static long IDX(const orc_state *s, long x, long y, long z) { return x + s->nx * (y + s->ny * z); }

/* Gauss-Jordan inverse with partial pivoting of the Q x Q lattice matrix. */
static int invert(int n, double A[QMAX][QMAX], double Ainv[QMAX][QMAX])
{
    double a[QMAX][2 * QMAX];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            a[r][c] = c < n ? A[r][c] : (c - n == r ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (a[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int k = 0; k < 2 * n; ++k) { double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
        double d = a[c][c];
        for (int k = 0; k < 2 * n; ++k) a[c][k] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c || a[r][c] == 0.0) continue;
            double f = a[r][c];
            for (int k = 0; k < 2 * n; ++k) a[r][k] -= f * a[c][k];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r][c] = a[r][n + c];
    return 0;
}

static void setup_lattice(orc_state *s)
{
    int three = s->p.lattice == 1;
    s->Q = three ? 19 : 9;
    s->D = three ? 3 : 2;
    for (int i = 0; i < s->Q; ++i) {
        for (int a = 0; a < 3; ++a) s->e[i][a] = three ? E3[i][a] : E2[i][a];
        s->w[i] = three ? W3[i] : W2[i];
        for (int k = 0; k < s->Q; ++k) s->M[i][k] = three ? M3[i][k] : M2[i][k];
    }
    for (int i = 0; i < s->Q; ++i)
        for (int k = 0; k < s->Q; ++k)
            if (s->e[k][0] == -s->e[i][0] && s->e[k][1] == -s->e[i][1] && s->e[k][2] == -s->e[i][2])
                s->opp[i] = k;
    invert(s->Q, s->M, s->Minv);
    /* Appendix A: (cs^k)^2 = 0.6 (1 - alpha^k) in 2-D and 0.5 (1 - alpha^k) in 3-D;
       eq 42: gamma = rhoR0/rhoB0 = (1 - alphaB)/(1 - alphaR). */
    s->alpha[0] = s->p.alphaR;
    s->alpha[1] = 1.0 - (s->p.rhoR0 / s->p.rhoB0) * (1.0 - s->p.alphaR);
    for (int k = 0; k < 2; ++k) s->cs2[k] = (three ? 0.5 : 0.6) * (1.0 - s->alpha[k]);
}

/* ---------------------------------------------------------------- ghosts */

/* Map a coordinate along one axis. Periodic axes wrap. Wall axes carry
   half-way walls at -1/2 and n-1/2; for the finite-difference stencils the
   values beyond them are mirror images (c = -1-k -> k, c = n+k -> n-1-k).
   Reading: mirror ghosts give zero normal gradient of rhoN, psi, phi and zero
   normal flux of surfactant through a wall. */
static long map_coord(long c, long n, int wall, int *mirrored)
{
    if (c >= 0 && c < n) return c;
    if (!wall) {
        c %= n;
        if (c < 0) c += n;
        return c;
    }
    *mirrored = 1;
    return c < 0 ? -1 - c : 2 * n - 1 - c;
}

/* Node index of (x,y,z)+(dx,dy,dz) and the sign of a field there: odd_axis is
   -1 for a scalar, or the axis a for the a-component of a vector, which changes
   sign in a mirror normal to that axis. */
static long nbr(const orc_state *s, long x, long y, long z, int dx, int dy, int dz, int odd_axis, double *sign)
{
    int mx = 0, my = 0, mz = 0;
    long X = map_coord(x + dx, s->nx, s->p.bc[0], &mx);
    long Y = map_coord(y + dy, s->ny, s->p.bc[1], &my);
    long Z = map_coord(z + dz, s->nz, s->p.bc[2], &mz);
    *sign = 1.0;
    if ((odd_axis == 0 && mx) || (odd_axis == 1 && my) || (odd_axis == 2 && mz)) *sign = -1.0;
    return IDX(s, X, Y, Z);
}

static double at(const orc_state *s, const double *f, long x, long y, long z, int dx, int dy, int dz, int odd_axis)
{
    double sg;
    long k = nbr(s, x, y, z, dx, dy, dz, odd_axis, &sg);
    return sg * f[k];
}

#define FOR_NODES(s)                                                    \
    _Pragma("omp parallel for collapse(2) schedule(static)")            \
    for (long z = 0; z < (s)->nz; ++z)                                  \
        for (long y = 0; y < (s)->ny; ++y)                              \
            for (long x = 0; x < (s)->nx; ++x)

/* ---------------------------------------------------------------- operators */

/* Isotropic lattice derivative, the "fourth-order isotropic finite
   difference" with which eq 9 evaluates every partial derivative.
   Reading: d_a chi(x) = (1/cs^2) sum_i w_i chi(x + e_i) e_ia with cs^2 = 1/3
   and the weights of the flow lattice. */
static void op_deriv(const orc_state *s, const double *chi, int odd_axis, int a, double *out)
{
    FOR_NODES(s) {
        double acc = 0.0;
        for (int i = 0; i < s->Q; ++i) {
            if (s->e[i][a] == 0) continue;
            acc += s->w[i] * at(s, chi, x, y, z, s->e[i][0], s->e[i][1], s->e[i][2], odd_axis) * s->e[i][a];
        }
        out[IDX(s, x, y, z)] = 3.0 * acc;
    }
}

/* Colour function (eq 6) and the per-colour densities (after eq 13). */
static void macro(orc_state *s, const double *fR, const double *fB, double *rhoR, double *rhoB,
                  double *rho, double *rhoN, double **j)
{
    long N = s->N;
    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double r = 0.0, b = 0.0, jj[3] = {0, 0, 0};
        for (int i = 0; i < s->Q; ++i) {
            r += fR[i * N + n];
            b += fB[i * N + n];
            for (int a = 0; a < 3; ++a) jj[a] += (fR[i * N + n] + fB[i * N + n]) * s->e[i][a];
        }
        rhoR[n] = r;
        rhoB[n] = b;
        if (rho) rho[n] = r + b;
        double rr = r / s->p.rhoR0, bb = b / s->p.rhoB0;
        rhoN[n] = (rr - bb) / (rr + bb);
        if (j)
            for (int a = 0; a < s->D; ++a) j[a][n] = jj[a];
    }
}

/* Interface geometry, forces and velocity at the current time level:
   grad rhoN and n (below eq 6), curvature (eq 7), EOS (eq 8), interfacial force
   (eq 9), buoyancy (Sec 3.4), velocity (eq 10) and the relaxation rate s_v
   (Appendix A, eq 43). */
static void force_stage(orc_state *s)
{
    const orc_params *p = &s->p;
    long N = s->N;
    int D = s->D;
    macro(s, s->fR, s->fB, s->rhoR, s->rhoB, s->rho, s->rhoN, s->j);
    for (int a = 0; a < D; ++a) op_deriv(s, s->rhoN, -1, a, s->g[a]);
    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double G2 = 0.0;
        for (int a = 0; a < D; ++a) G2 += s->g[a][n] * s->g[a][n];
        s->G[n] = sqrt(G2);
        /* n = -grad rhoN / |grad rhoN|.  Reading: regularised by eps_n so that it is
           defined (and zero) where the colour field is uniform. */
        double den = sqrt(G2 + p->eps_n * p->eps_n);
        for (int a = 0; a < D; ++a) s->nrm[a][n] = den > 0.0 ? -s->g[a][n] / den : 0.0;
    }
    /* eq 7: kappa = -div n */
    for (long n = 0; n < N; ++n) s->kappa[n] = 0.0;
    for (int a = 0; a < D; ++a) {
        op_deriv(s, s->nrm[a], a, a, s->tmp);
        for (long n = 0; n < N; ++n) s->kappa[n] -= s->tmp[n];
    }
    for (int a = 0; a < D; ++a) op_deriv(s, s->psi, -1, a, s->gpsi[a]);

    double sig_min = p->sigma_min_ratio * p->sigma0;
    /* reference density of the buoyancy: rhoB0, or the domain mean (exactly conserved) */
    double rho_ref = p->rhoB0;
    if (p->buoyancy_ref == 1) {
        double m = 0.0;
        for (long n = 0; n < N; ++n) m += s->rho[n];
        rho_ref = m / (double)N;
    }
    /* CMC below eq 8: the psi at which sigma reaches sigma_min. */
    double cmc = p->E0 > 0.0 ? p->psi_inf * (1.0 - exp(-(1.0 - p->sigma_min_ratio) / p->E0)) : p->psi_inf;
    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double psi = s->psi[n], Fs[3] = {0, 0, 0};
        if (p->E0 == 0.0) {
            for (int a = 0; a < D; ++a) Fs[a] = -0.5 * p->sigma0 * s->kappa[n] * s->g[a][n];
        } else if (p->eos_mode == 1) {
            /* Sec 3.2: sigma linear in psi, so d sigma / d psi = -sigma0 E0 / psi_inf everywhere */
            double sigma = p->sigma0 * (1.0 - p->E0 * psi / p->psi_inf);
            double ndg = 0.0;
            for (int a = 0; a < D; ++a) ndg += s->nrm[a][n] * s->gpsi[a][n];
            double mar = 0.5 * s->G[n] * p->sigma0 * p->E0 / p->psi_inf;
            for (int a = 0; a < D; ++a)
                Fs[a] = -0.5 * sigma * s->kappa[n] * s->g[a][n] - mar * (s->gpsi[a][n] - ndg * s->nrm[a][n]);
        } else if (psi < cmc) {
            double sigma = p->sigma0 * (1.0 + p->E0 * log(1.0 - psi / p->psi_inf));
            double ndg = 0.0;
            for (int a = 0; a < D; ++a) ndg += s->nrm[a][n] * s->gpsi[a][n];
            double mar = 0.5 * s->G[n] * p->sigma0 * p->E0 / (p->psi_inf - psi);
            for (int a = 0; a < D; ++a)
                Fs[a] = -0.5 * sigma * s->kappa[n] * s->g[a][n] - mar * (s->gpsi[a][n] - ndg * s->nrm[a][n]);
        } else {
            for (int a = 0; a < D; ++a) Fs[a] = -0.5 * sig_min * s->kappa[n] * s->g[a][n];
        }
        double rho = s->rho[n];
        for (int a = 0; a < D; ++a) {
            /* Sec 3.4: F_b = (rho - rhoB0) g k, added like F_s. Reading: gravity is a signed vector.
               buoyancy_ref = 1 takes the mean density of the domain instead of rhoB0. */
            s->F[a][n] = Fs[a] + (rho - rho_ref) * p->gravity[a];
            s->u[a][n] = (s->j[a][n] + 0.5 * s->F[a][n]) / rho; /* eq 10 */
        }
        /* eq 43 and the mu-s_v relation of Appendix A (delta_t = 1). */
        double rN = s->rhoN[n];
        double inv_mu = (1.0 + rN) / (2.0 * p->muR0) + (1.0 - rN) / (2.0 * p->muB0);
        double mu = 1.0 / inv_mu;
        double pk = s->rhoR[n] * s->cs2[0] + s->rhoB[n] * s->cs2[1];
        s->sv[n] = 1.0 / (mu / pk + 0.5);
    }
}

/* Moment equilibrium of colour k: eq 37 (2-D) or eq 40 (3-D), written out. */
static void moment_eq(const orc_state *s, int k, double rho, const double *u, double *m)
{
    double al = s->alpha[k];
    double ux = u[0], uy = u[1], uz = s->D == 3 ? u[2] : 0.0;
    double u2 = ux * ux + uy * uy + uz * uz;
    if (s->D == 2) {
        m[0] = rho;
        m[1] = rho * (-3.6 * al - 0.4 + 3.0 * u2);
        m[2] = rho * (5.4 * al - 1.4 - 3.0 * u2);
        m[3] = rho * ux;
        m[4] = rho * (-1.8 * al - 0.2) * ux;
        m[5] = rho * uy;
        m[6] = rho * (-1.8 * al - 0.2) * uy;
        m[7] = rho * (ux * ux - uy * uy);
        m[8] = rho * ux * uy;
    } else {
        double pk = rho * s->cs2[k];
        m[0] = rho;
        m[1] = rho * ux;
        m[2] = rho * uy;
        m[3] = rho * uz;
        m[4] = 3.0 * pk + rho * u2;
        m[5] = rho * (2.0 * ux * ux - uy * uy - uz * uz);
        m[6] = rho * (uy * uy - uz * uz);
        m[7] = rho * ux * uy;
        m[8] = rho * ux * uz;
        m[9] = rho * uy * uz;
        m[10] = pk * uy;
        m[11] = pk * ux;
        m[12] = pk * uz;
        m[13] = pk * ux;
        m[14] = pk * uz;
        m[15] = pk * uy;
        m[16] = rho * ((1.0 - al - u2) + 2.0 * (ux * ux + uy * uy)) / 6.0;
        m[17] = rho * ((1.0 - al - u2) + 2.0 * (ux * ux + uz * uz)) / 6.0;
        m[18] = rho * ((1.0 - al - u2) + 2.0 * (uy * uy + uz * uz)) / 6.0;
    }
}

/* Prefactor of the correction Q_a = c_k d_a(rho^k u_a) (Appendix A, below eq 42).
   2-D as printed: 1.8 alpha^k - 0.8. 3-D: printed c^2 - (cs^k)^2; Reading:
   c^2 - 3 (cs^k)^2 with c = 1, which, like the 2-D form (= 1 - 3 (cs^k)^2), vanishes
   at the standard sound speed. q_literal selects the printed form. */
static double q_coef(const orc_state *s, int k)
{
    if (s->D == 2) return 1.8 * s->alpha[k] - 0.8;
    return s->p.q_literal ? 1.0 - s->cs2[k] : 1.0 - 3.0 * s->cs2[k];
}

/* Relaxation matrix: eq 38 (2-D), eq 41 (3-D). */
static void relax_diag(const orc_state *s, double sv, double *S)
{
    if (s->D == 2) {
        const double s2[9] = {0.0, 1.25, 1.14, 0.0, 1.6, 0.0, 1.6, 0.0, 0.0};
        for (int i = 0; i < 9; ++i) S[i] = s2[i];
        S[7] = S[8] = sv;
    } else {
        for (int i = 0; i < 19; ++i) S[i] = 1.0;
        for (int i = 5; i <= 9; ++i) S[i] = sv;
    }
}

/* Collision (eqs 1-4) and recolouring (eqs 11-12) at every node, followed by
   propagation (eq 13) with periodic wrap or half-way bounce-back walls.
   Writes the next populations into fR2/fB2. */
static void lb_stage(orc_state *s)
{
    const orc_params *p = &s->p;
    long N = s->N;
    int Q = s->Q, D = s->D;
    const double cs2 = 1.0 / 3.0; /* lattice sound speed of eq 4 */

    /* d_a(rho^k u_a) for the correction term, same derivative operator. */
    for (int k = 0; k < 2; ++k)
        for (int a = 0; a < D; ++a) {
            const double *rk = k == 0 ? s->rhoR : s->rhoB;
            for (long n = 0; n < N; ++n) s->ku[k][a][n] = rk[n] * s->u[a][n];
            op_deriv(s, s->ku[k][a], a, a, s->dku[k][a]);
        }

    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double f[QMAX], m[QMAX], meq[QMAX], mk[QMAX], C[QMAX], Fm[QMAX], S[QMAX];
        double fdag[QMAX], fRr[QMAX], fBr[QMAX];
        double u[3] = {0, 0, 0}, F[3] = {0, 0, 0}, g[3] = {0, 0, 0};
        for (int a = 0; a < D; ++a) { u[a] = s->u[a][n]; F[a] = s->F[a][n]; g[a] = s->g[a][n]; }
        double rR = s->rhoR[n], rB = s->rhoB[n], rho = s->rho[n];

        for (int i = 0; i < Q; ++i) f[i] = s->fR[i * N + n] + s->fB[i * N + n];
        for (int r = 0; r < Q; ++r) {
            m[r] = 0.0;
            for (int i = 0; i < Q; ++i) m[r] += s->M[r][i] * f[i];
        }
        /* sum over colours of the equilibria and corrections (eq 2) */
        for (int r = 0; r < Q; ++r) { meq[r] = 0.0; C[r] = 0.0; }
        for (int k = 0; k < 2; ++k) {
            moment_eq(s, k, k == 0 ? rR : rB, u, mk);
            for (int r = 0; r < Q; ++r) meq[r] += mk[r];
            double c = q_coef(s, k), Qa[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) Qa[a] = c * s->dku[k][a][n];
            if (D == 2) {
                C[1] += 3.0 * Qa[0] + 3.0 * Qa[1];      /* eq 37 */
                C[7] += Qa[0] - Qa[1];
            } else {
                C[4] += Qa[0] + Qa[1] + Qa[2];          /* eq 40 */
                C[5] += 2.0 * Qa[0] - Qa[1] - Qa[2];
                C[6] += Qa[1] - Qa[2];
            }
        }
        /* eq 4 */
        for (int r = 0; r < Q; ++r) {
            double acc = 0.0;
            for (int i = 0; i < Q; ++i) {
                double eu = 0.0, t = 0.0;
                for (int a = 0; a < D; ++a) eu += s->e[i][a] * u[a];
                for (int a = 0; a < D; ++a)
                    t += ((s->e[i][a] - u[a]) / cs2 + eu * s->e[i][a] / (cs2 * cs2)) * F[a];
                acc += s->M[r][i] * s->w[i] * t;
            }
            Fm[r] = acc;
        }
        relax_diag(s, s->sv[n], S);
        /* eqs 1-3: f_dag = f + Omega + Phi */
        for (int i = 0; i < Q; ++i) {
            double om = 0.0, ph = 0.0;
            for (int r = 0; r < Q; ++r) {
                double mis = s->Minv[i][r] * S[r];
                om += -mis * (m[r] - meq[r]) + (s->Minv[i][r] - 0.5 * mis) * C[r];
                ph += (s->Minv[i][r] - 0.5 * mis) * Fm[r];
            }
            fdag[i] = f[i] + om + ph;
            if (s->dump_fdag) s->dump_fdag[i * N + n] = fdag[i];
        }
        /* eqs 11-12. cos(theta_i)|e_i| = e_i . grad rhoN / |grad rhoN|.
           Reading: the term is zero for i = 0 and where |grad rhoN| = 0.
           Reading: the weight w_i is the rest equilibrium of the local mixture
           per unit density, sum_k rho^k phi_i(alpha^k) / rho. It equals the
           lattice weight when both colours have the standard sound speed
           (density ratio 1); with the lattice weight a static bubble at density
           ratio 10 blows up. recolour_literal selects the lattice weight. */
        double Gn = s->G[n];
        double rr = rR * rB / rho;
        for (int i = 0; i < Q; ++i) {
            double ce = 0.0;
            if (Gn > 0.0) {
                double eg = 0.0;
                for (int a = 0; a < D; ++a) eg += s->e[i][a] * g[a];
                ce = eg / Gn;
            }
            double wi = p->recolour_literal ? s->w[i]
                                            : (rR * s->phi_rest[0][i] + rB * s->phi_rest[1][i]) / rho;
            fRr[i] = rR / rho * fdag[i] + p->beta * wi * rr * ce;
            fBr[i] = rB / rho * fdag[i] - p->beta * wi * rr * ce;
        }
        /* eq 13, push form. Half-way bounce-back: a population leaving through a
           wall returns to the same node in the opposite direction one step later.
           Reading (moving walls): Ladd's momentum term -2 w_i rho^k (e_i . u_w)/cs^2,
           with rho^k of the node; at a corner the first crossed axis (x, y, z)
           names the wall. */
        for (int i = 0; i < Q; ++i) {
            long X = x + s->e[i][0], Y = y + s->e[i][1], Z = z + s->e[i][2];
            int wall = -1;
            long c[3] = {X, Y, Z}, lim[3] = {s->nx, s->ny, s->nz};
            for (int a = 0; a < 3 && wall < 0; ++a)
                if (p->bc[a] == 1 && (c[a] < 0 || c[a] >= lim[a])) wall = 2 * a + (c[a] >= lim[a] ? 1 : 0);
            if (wall >= 0) {
                double eu = 0.0;
                for (int a = 0; a < 3; ++a) eu += s->e[i][a] * p->wall_u[wall][a];
                int o = s->opp[i];
                s->fR2[o * N + n] = fRr[i] - 2.0 * s->w[i] * rR * eu / cs2;
                s->fB2[o * N + n] = fBr[i] - 2.0 * s->w[i] * rB * eu / cs2;
            } else {
                int dm = 0;
                X = map_coord(X, s->nx, 0, &dm);
                Y = map_coord(Y, s->ny, 0, &dm);
                Z = map_coord(Z, s->nz, 0, &dm);
                long d = IDX(s, X, Y, Z);
                s->fR2[i * N + d] = fRr[i];
                s->fB2[i * N + d] = fBr[i];
            }
        }
    }
}

/* WENO3 convective derivative of eqs 25-27 along every axis:
   out = sum_a [H+(u_a) D-_a Psi_a + H-(u_a) D+_a Psi_a], with
   H+ = u^+/|u|, H- = |u^-|/|u|. Reading: the printed u^-/|u| is negative for
   u < 0; its magnitude is meant. Reading: where |u_a| <= upwind_eps (and at
   u_a = 0, where the printed form is 0/0) both are 1/2, so that the upwind
   choice never rests on the sign of a velocity at the level of rounding. */
static void op_weno_div(const orc_state *s, double *const *Psi, double *const *u, double *out)
{
    double eps = s->p.weno_eps;
    int D = s->D;
    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double acc = 0.0;
        for (int a = 0; a < D; ++a) {
            double P[5];
            for (int k = -2; k <= 2; ++k) {
                int d[3] = {0, 0, 0};
                d[a] = k;
                P[k + 2] = at(s, Psi[a], x, y, z, d[0], d[1], d[2], a);
            }
#define DP(k) (P[(k) + 3] - P[(k) + 2])                     /* forward difference at i+k */
#define DD(k) (P[(k) + 3] - 2.0 * P[(k) + 2] + P[(k) + 1])  /* second difference at i+k */
            double rm = (eps + DD(-1) * DD(-1)) / (eps + DD(0) * DD(0));
            double wm = 1.0 / (1.0 + 2.0 * rm * rm);
            double Dm = 0.5 * ((DP(-1) + DP(0)) - wm * (DP(-2) - 2.0 * DP(-1) + DP(0)));
            double rp = (eps + DD(1) * DD(1)) / (eps + DD(0) * DD(0));
            double wp = 1.0 / (1.0 + 2.0 * rp * rp);
            double Dp = 0.5 * ((DP(-1) + DP(0)) - wp * (DP(1) - 2.0 * DP(0) + DP(-1)));
#undef DP
#undef DD
            double ua = u[a][n], hp, hm;
            if (fabs(ua) <= s->p.upwind_eps) { hp = 0.5; hm = 0.5; }
            else { hp = fmax(ua, 0.0) / fabs(ua); hm = fabs(fmin(ua, 0.0)) / fabs(ua); }
            acc += hp * Dm + hm * Dp;
        }
        out[n] = acc;
    }
}

/* Conservative diffusion operator of eq 28, written as printed:
   sum_f W_f chi_f - (sum_f W_f) chi, with half-point W_f the mean of the two
   nodes. Faces whose neighbour is the node's own mirror image carry no flux. */
static void op_diffusion(const orc_state *s, const double *W, const double *chi, double *out)
{
    int D = s->D;
    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double sw = 0.0, swc = 0.0, sg;
        for (int a = 0; a < D; ++a)
            for (int d = -1; d <= 1; d += 2) {
                int o[3] = {0, 0, 0};
                o[a] = d;
                long k = nbr(s, x, y, z, o[0], o[1], o[2], -1, &sg);
                double wf = 0.5 * (W[n] + W[k]);
                swc += wf * chi[k];
                sw += wf;
            }
        out[n] = swc - sw * chi[n];
    }
}

/* Solve [diag(W) - (Dc/2) L_W] chi = rhs by SOR (Sec 2.2, relaxation factor
   omega), lexicographic order, from the initial guess in chi. Reading: rows
   with zero diagonal (W = 0 at the node and all its face neighbours) are
   decoupled and keep their value; convergence is max |residual| over the
   other rows <= tol * max |rhs|. Returns the number of sweeps or -1. */
static int op_solve(const orc_state *s, const double *W, double Dc, const double *rhs, double *chi)
{
    const orc_params *p = &s->p;
    int D = s->D, nf = 2 * s->D;
    long N = s->N;
    double hd = 0.5 * Dc;
    /* the matrix: face neighbours, off-diagonal weights (Dc/2) W_f and diagonal */
    long *nb = (long *)malloc(sizeof(long) * N * nf);
    double *wf = (double *)malloc(sizeof(double) * N * nf);
    double *dg = (double *)malloc(sizeof(double) * N);
    if (!nb || !wf || !dg) { free(nb); free(wf); free(dg); return -1; }
    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double diag = W[n], sg;
        int f = 0;
        for (int a = 0; a < D; ++a)
            for (int d = -1; d <= 1; d += 2, ++f) {
                int o[3] = {0, 0, 0};
                o[a] = d;
                long k = nbr(s, x, y, z, o[0], o[1], o[2], -1, &sg);
                nb[n * nf + f] = k;
                wf[n * nf + f] = k == n ? 0.0 : hd * 0.5 * (W[n] + W[k]);
                diag += wf[n * nf + f];
            }
        dg[n] = diag;
    }
    double rmax = 0.0;
    for (long n = 0; n < N; ++n)
        if (dg[n] > 0.0) rmax = fmax(rmax, fabs(rhs[n]));
    int result = -1;
    for (int sweep = 0; sweep <= p->sor_max_sweeps; ++sweep) {
        /* residual of the current iterate */
        double res = 0.0;
        for (long n = 0; n < N; ++n) {
            if (!(dg[n] > 0.0)) continue;
            double off = 0.0;
            for (int f = 0; f < nf; ++f) off += wf[n * nf + f] * chi[nb[n * nf + f]];
            res = fmax(res, fabs(rhs[n] - (dg[n] * chi[n] - off)));
        }
        if (res <= p->sor_tol * rmax) { result = sweep; break; }
        if (sweep == p->sor_max_sweeps) break;
        /* one lexicographic SOR sweep */
        for (long n = 0; n < N; ++n) {
            if (!(dg[n] > 0.0)) continue;
            double off = 0.0;
            for (int f = 0; f < nf; ++f) off += wf[n * nf + f] * chi[nb[n * nf + f]];
            chi[n] = (1.0 - p->sor_omega) * chi[n] + p->sor_omega * (rhs[n] + off) / dg[n];
        }
    }
    free(nb);
    free(wf);
    free(dg);
    return result;
}

/* Weight of a node in the surfactant equations. Reading: the delta function
   |grad rhoN|/2 and the indicator (1 - rhoN)/2 of eqs 20-21 carry a small
   uniform background fd_eps, so that psi (phi) stays defined where the
   weight itself vanishes. Without it, the weights of the tanh tails shrink
   as the interface sharpens, psi = (G psi)/G grows like G^t/G^{t+1} step
   after step and the source G j feeds it back until overflow. */
static double fd_weight(const orc_state *s, double w) { return w + s->p.fd_eps; }

/* Conserved integrand of eqs 20-21, summed serially in node order. */
static double total_surfactant(const orc_state *s, const double *G, const double *X, const double *psi,
                               const double *phi)
{
    double acc = 0.0;
    for (long n = 0; n < s->N; ++n) acc += G[n] * psi[n] + X[n] * phi[n];
    return acc;
}

/* Finite-difference transport of psi and phi over one step (Sec 2.2):
   eqs 20-22, modified Crank-Nicolson (eq 23 at the first step, eq 24 after),
   WENO3 convection (eqs 25-27), diffusion (eq 28), SOR solve and rescaling.
   Reading of the time levels: G^{t+1} comes from the populations just
   streamed; convection and sources use u, G, rhoN of the LB step just taken. */
static int fd_transport(orc_state *s);

static int fd_stage(orc_state *s)
{
    long N = s->N;
    int D = s->D;

    macro(s, s->fR2, s->fB2, s->tmp, s->divPhi, NULL, s->rhoN1, NULL); /* divPhi as scratch */
    for (int a = 0; a < D; ++a) op_deriv(s, s->rhoN1, -1, a, s->g1[a]);
    for (long n = 0; n < N; ++n) {
        double G2 = 0.0;
        for (int a = 0; a < D; ++a) G2 += s->g1[a][n] * s->g1[a][n];
        s->G1[n] = fd_weight(s, sqrt(G2));
        s->X1[n] = fd_weight(s, 1.0 - s->rhoN1[n]);
        s->X0[n] = fd_weight(s, 1.0 - s->rhoN[n]);
        s->Gw[n] = fd_weight(s, s->G[n]);
    }
    return fd_transport(s);
}

/* The transport itself, from the weights G1, X1 (time t+1), Gw, X0 (time t),
   u and psi, phi at time t. */
static int fd_transport(orc_state *s)
{
    const orc_params *p = &s->p;
    long N = s->N;
    int D = s->D;
    int status = ORC_OK;
    /* fluxes Psi = psi |grad rhoN| u and Phi = phi (1 - rhoN) u at time t */
    for (int a = 0; a < D; ++a)
        for (long n = 0; n < N; ++n) {
            s->Psi[a][n] = s->psi[n] * s->Gw[n] * s->u[a][n];
            s->Phi[a][n] = s->phi[n] * s->X0[n] * s->u[a][n];
        }
    op_weno_div(s, s->Psi, s->u, s->divPsi);
    op_weno_div(s, s->Phi, s->u, s->divPhi);
    for (long n = 0; n < N; ++n) {
        double psi = s->psi[n], phi = s->phi[n];
        double jj = p->source_mode == 1 ? p->ra * p->psi_inf * phi
                                        : p->ra * phi * (p->psi_inf - psi) - p->rd * psi; /* eq 22 */
        s->S[n] = -s->divPsi[n] + s->Gw[n] * jj;
        s->B[n] = -s->divPhi[n] - s->Gw[n] * jj;
    }
    /* explicit half of the diffusion, then the right-hand sides of eqs 23/24 */
    op_diffusion(s, s->Gw, s->psi, s->rhsP);
    op_diffusion(s, s->X0, s->phi, s->rhsF);
    for (long n = 0; n < N; ++n) {
        double eS = s->step == 0 ? s->S[n] : 1.5 * s->S[n] - 0.5 * s->Sprev[n];
        double eB = s->step == 0 ? s->B[n] : 1.5 * s->B[n] - 0.5 * s->Bprev[n];
        s->rhsP[n] = s->Gw[n] * s->psi[n] + 0.5 * p->Ds * s->rhsP[n] + eS;
        s->rhsF[n] = s->X0[n] * s->phi[n] + 0.5 * p->Db * s->rhsF[n] + eB;
    }
    /* implicit half: psi, phi at t+1, initial guess the values at t */
    s->sweeps[0] = op_solve(s, s->G1, p->Ds, s->rhsP, s->psi);
    s->sweeps[1] = op_solve(s, s->X1, p->Db, s->rhsF, s->phi);
    if (s->sweeps[0] < 0 || s->sweeps[1] < 0) status = ORC_ESOR;
    /* rescaling: one common factor restores the initial total (Sec 2.2, Xu et al.).
       Reading: the conserved total is sum(G psi + X phi). */
    double Mt = total_surfactant(s, s->G1, s->X1, s->psi, s->phi);
    s->drift_pre = s->M0 != 0.0 ? (Mt - s->M0) / s->M0 : 0.0;
    if (p->rescale && s->M0 != 0.0 && Mt != 0.0) {
        double sc = s->M0 / Mt;
        for (long n = 0; n < N; ++n) { s->psi[n] *= sc; s->phi[n] *= sc; }
    }
    for (long n = 0; n < N; ++n) { s->Sprev[n] = s->S[n]; s->Bprev[n] = s->B[n]; }
    return status;
}

/* ---------------------------------------------------------------- API */

static double *alloc0(long n) { return (double *)calloc((size_t)n, sizeof(double)); }

void orc_destroy(orc_state *s);

orc_state *orc_create(const orc_params *p)
{
    if (!p || (p->lattice != 0 && p->lattice != 1)) return NULL;
    if (p->nx < 4 || p->ny < 4 || (p->lattice == 1 ? p->nz < 4 : p->nz != 1)) return NULL;
    if (!(p->rhoR0 > 0 && p->rhoB0 > 0 && p->muR0 > 0 && p->muB0 > 0)) return NULL;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->p = *p;
    if (p->lattice == 0) s->p.bc[2] = 0;
    setup_lattice(s);
    if (!(s->alpha[1] > 0.0 && s->alpha[1] < 1.0 && s->alpha[0] > 0.0 && s->alpha[0] < 1.0)) { free(s); return NULL; }
    for (int k = 0; k < 2; ++k) {
        double u0[3] = {0, 0, 0}, m[QMAX];
        moment_eq(s, k, 1.0, u0, m);
        for (int i = 0; i < s->Q; ++i) {
            double a = 0.0;
            for (int r = 0; r < s->Q; ++r) a += s->Minv[i][r] * m[r];
            s->phi_rest[k][i] = a;
        }
    }
    s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
    s->N = s->nx * s->ny * s->nz;
    long N = s->N, Q = s->Q;
    int ok = 1;
#define A(ptr, cnt) do { (ptr) = alloc0(cnt); ok = ok && (ptr); } while (0)
    A(s->fR, Q * N); A(s->fB, Q * N); A(s->fR2, Q * N); A(s->fB2, Q * N);
    A(s->psi, N); A(s->phi, N); A(s->Sprev, N); A(s->Bprev, N);
    A(s->rhoR, N); A(s->rhoB, N); A(s->rho, N); A(s->rhoN, N); A(s->G, N); A(s->kappa, N); A(s->sv, N);
    A(s->rhoN1, N); A(s->G1, N); A(s->X0, N); A(s->X1, N); A(s->divPsi, N); A(s->divPhi, N);
    A(s->S, N); A(s->B, N); A(s->rhsP, N); A(s->rhsF, N); A(s->tmp, N); A(s->Gw, N);
    for (int a = 0; a < 3; ++a) {
        A(s->j[a], N); A(s->g[a], N); A(s->nrm[a], N); A(s->gpsi[a], N); A(s->F[a], N); A(s->u[a], N);
        A(s->g1[a], N); A(s->Psi[a], N); A(s->Phi[a], N);
        for (int k = 0; k < 2; ++k) { A(s->ku[k][a], N); A(s->dku[k][a], N); }
    }
#undef A
    if (!ok) { orc_destroy(s); return NULL; }
    return s;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    double **all[] = {&s->fR, &s->fB, &s->fR2, &s->fB2, &s->psi, &s->phi, &s->Sprev, &s->Bprev,
                      &s->rhoR, &s->rhoB, &s->rho, &s->rhoN, &s->G, &s->kappa, &s->sv, &s->rhoN1, &s->G1,
                      &s->X0, &s->X1, &s->divPsi, &s->divPhi, &s->S, &s->B, &s->rhsP, &s->rhsF, &s->tmp, &s->Gw};
    for (size_t i = 0; i < sizeof(all) / sizeof(all[0]); ++i) free(*all[i]);
    for (int a = 0; a < 3; ++a) {
        free(s->j[a]); free(s->g[a]); free(s->nrm[a]); free(s->gpsi[a]); free(s->F[a]); free(s->u[a]);
        free(s->g1[a]); free(s->Psi[a]); free(s->Phi[a]);
        for (int k = 0; k < 2; ++k) { free(s->ku[k][a]); free(s->dku[k][a]); }
    }
    free(s);
}

/* Initial state. Reading: rhoN = tanh(2 (R - r)/W) (the largest over drops),
   rho^R = rhoR0 (1 + rhoN)/2, rho^B = rhoB0 (1 - rhoN)/2, each colour at its
   moment equilibrium with the initial velocity; psi uniform; phi a step at
   rhoN = 0. */
int orc_init(orc_state *s, const orc_init_spec *in)
{
    if (!s || !in || in->n < 0 || in->n > 16 || !(in->width > 0.0)) return ORC_EINVAL;
    long N = s->N;
    int Q = s->Q;
    FOR_NODES(s) {
        long n = IDX(s, x, y, z);
        double rN = -1.0;
        for (int d = 0; d < in->n; ++d) {
            double dx = x - in->cx[d], dy = y - in->cy[d], dz = s->D == 3 ? z - in->cz[d] : 0.0;
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double v = tanh(2.0 * (in->r[d] - r) / in->width);
            if (d == 0 || v > rN) rN = v;
        }
        double rR = s->p.rhoR0 * (1.0 + rN) / 2.0, rB = s->p.rhoB0 * (1.0 - rN) / 2.0;
        double u[3] = {in->shear_rate * (y - 0.5 * (s->ny - 1)), 0.0, 0.0};
        double mR[QMAX], mB[QMAX];
        moment_eq(s, 0, rR, u, mR);
        moment_eq(s, 1, rB, u, mB);
        for (int i = 0; i < Q; ++i) {
            double a = 0.0, b = 0.0;
            for (int r = 0; r < Q; ++r) { a += s->Minv[i][r] * mR[r]; b += s->Minv[i][r] * mB[r]; }
            s->fR[i * N + n] = a;
            s->fB[i * N + n] = b;
        }
        s->psi[n] = in->psi0;
        s->phi[n] = rN < 0.0 ? in->phi0_out : in->phi0_in;
        s->Sprev[n] = 0.0;
        s->Bprev[n] = 0.0;
    }
    s->step = 0;
    s->drift_pre = 0.0;
    s->sweeps[0] = s->sweeps[1] = 0;
    force_stage(s);
    for (long n = 0; n < N; ++n) { s->X0[n] = fd_weight(s, 1.0 - s->rhoN[n]); s->Gw[n] = fd_weight(s, s->G[n]); }
    s->M0 = total_surfactant(s, s->Gw, s->X0, s->psi, s->phi);
    return ORC_OK;
}

/* One time step: force stage, LB collision/recolouring/propagation, FD transport. */
static int step_once(orc_state *s)
{
    force_stage(s);
    lb_stage(s);
    int st = ORC_OK;
    if (s->p.fd_enable) st = fd_stage(s);
    double *t;
    t = s->fR; s->fR = s->fR2; s->fR2 = t;
    t = s->fB; s->fB = s->fB2; s->fB2 = t;
    s->step += 1;
    return st;
}

/* k transport updates of psi and phi with the flow frozen at the current state:
   rhoN, G and u from the current populations, and the weights of the new time
   level equal to those of the old one (G^{t+1} = G^t, X^{t+1} = X^t). The LB
   populations and the step counter are left as they are. This defines the
   quantity the learned surrogate approximates (k substeps of the FD update of
   Sec 2.2 with the flow held fixed). */
int orc_fd_substeps(orc_state *s, int64_t k)
{
    if (!s || k < 0) return ORC_EINVAL;
    if (!s->p.fd_enable || k == 0) return ORC_OK;
    force_stage(s);
    for (long n = 0; n < s->N; ++n) {
        s->Gw[n] = fd_weight(s, s->G[n]);
        s->G1[n] = s->Gw[n];
        s->X0[n] = fd_weight(s, 1.0 - s->rhoN[n]);
        s->X1[n] = s->X0[n];
    }
    for (int64_t i = 0; i < k; ++i) {
        int st = fd_transport(s);
        if (st != ORC_OK) return st;
    }
    return ORC_OK;
}

int orc_step(orc_state *s, int64_t nsteps)
{
    if (!s || nsteps < 0) return ORC_EINVAL;
    for (int64_t k = 0; k < nsteps; ++k) {
        int st = step_once(s);
        if (st != ORC_OK) return st;
    }
    return ORC_OK;
}

int64_t orc_nodes(const orc_state *s) { return s ? s->N : 0; }

/* Threads the OpenMP loops use (for reporting the CPU baseline). */
/* Set the OpenMP threads of the node loops (timing only: results do not
   depend on it beyond the summation order of the observables). */
void orc_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int orc_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
int orc_lattice_q(const orc_state *s) { return s ? s->Q : 0; }
double orc_initial_total(const orc_state *s) { return s ? s->M0 : 0.0; }

/* Copy a field out as FP64. Derived fields (u, force, G, kappa) are evaluated
   at the current time level from the current state. */
int orc_get_field(orc_state *s, int id, double *out)
{
    if (!s || !out) return ORC_EINVAL;
    long N = s->N;
    int Q = s->Q, D = s->D;
    switch (id) {
    case FLD_F: for (long k = 0; k < Q * N; ++k) out[k] = s->fR[k] + s->fB[k]; return ORC_OK;
    case FLD_FR: memcpy(out, s->fR, sizeof(double) * Q * N); return ORC_OK;
    case FLD_FB: memcpy(out, s->fB, sizeof(double) * Q * N); return ORC_OK;
    case FLD_PSI: memcpy(out, s->psi, sizeof(double) * N); return ORC_OK;
    case FLD_PHI: memcpy(out, s->phi, sizeof(double) * N); return ORC_OK;
    case FLD_SPREV: memcpy(out, s->Sprev, sizeof(double) * N); return ORC_OK;
    case FLD_BPREV: memcpy(out, s->Bprev, sizeof(double) * N); return ORC_OK;
    default: break;
    }
    force_stage(s);
    switch (id) {
    case FLD_RHOR: memcpy(out, s->rhoR, sizeof(double) * N); return ORC_OK;
    case FLD_RHOB: memcpy(out, s->rhoB, sizeof(double) * N); return ORC_OK;
    case FLD_RHON: memcpy(out, s->rhoN, sizeof(double) * N); return ORC_OK;
    case FLD_G: memcpy(out, s->G, sizeof(double) * N); return ORC_OK;
    case FLD_KAPPA: memcpy(out, s->kappa, sizeof(double) * N); return ORC_OK;
    case FLD_U: for (int a = 0; a < D; ++a) memcpy(out + a * N, s->u[a], sizeof(double) * N); return ORC_OK;
    case FLD_FORCE: for (int a = 0; a < D; ++a) memcpy(out + a * N, s->F[a], sizeof(double) * N); return ORC_OK;
    default: return ORC_EINVAL;
    }
}

int orc_set_field(orc_state *s, int id, const double *in)
{
    if (!s || !in) return ORC_EINVAL;
    long N = s->N;
    int Q = s->Q;
    switch (id) {
    case FLD_FR: memcpy(s->fR, in, sizeof(double) * Q * N); return ORC_OK;
    case FLD_FB: memcpy(s->fB, in, sizeof(double) * Q * N); return ORC_OK;
    case FLD_PSI: memcpy(s->psi, in, sizeof(double) * N); return ORC_OK;
    case FLD_PHI: memcpy(s->phi, in, sizeof(double) * N); return ORC_OK;
    case FLD_SPREV: memcpy(s->Sprev, in, sizeof(double) * N); return ORC_OK;
    case FLD_BPREV: memcpy(s->Bprev, in, sizeof(double) * N); return ORC_OK;
    default: return ORC_EINVAL;
    }
}

/* Set the step counter (selects eq 23 at 0, eq 24 after) and the target total. */
int orc_set_clock(orc_state *s, int64_t step, double M0)
{
    if (!s || step < 0) return ORC_EINVAL;
    s->step = step;
    s->M0 = M0;
    return ORC_OK;
}

/* Observables: masses, total surfactant, the droplet velocity of eqs 33-34,
   centroid and second moments, the interface surfactant statistics and the
   bulk pressures inside and outside. Reading: centroid weight (1 + rhoN)/2;
   psi_av = sum G psi / sum G; psi_min/max over |rhoN| <= 0.5; p = sum_k rho^k
   (cs^k)^2 averaged over rhoN > 0.99 (inside) and rhoN < -0.99 (outside). */
int orc_observables(orc_state *s, orc_obs *o)
{
    if (!s || !o) return ORC_EINVAL;
    memset(o, 0, sizeof(*o));
    force_stage(s);
    for (long n = 0; n < s->N; ++n) { s->X0[n] = fd_weight(s, 1.0 - s->rhoN[n]); s->Gw[n] = fd_weight(s, s->G[n]); }
    o->step = s->step;
    o->total_surf = total_surfactant(s, s->Gw, s->X0, s->psi, s->phi);
    o->drift_pre = s->drift_pre;
    o->sor_sweeps[0] = s->sweeps[0];
    o->sor_sweeps[1] = s->sweeps[1];
    double sw = 0, sx[3] = {0, 0, 0}, sN = 0, su[3] = {0, 0, 0}, sG = 0, sGp = 0;
    double pin = 0, nin = 0, pout = 0, nout = 0, pmin = INFINITY, pmax = -INFINITY;
    for (long z = 0; z < s->nz; ++z)
        for (long y = 0; y < s->ny; ++y)
            for (long x = 0; x < s->nx; ++x) {
                long n = IDX(s, x, y, z);
                double rN = s->rhoN[n], c[3] = {(double)x, (double)y, (double)z};
                o->mass_R += s->rhoR[n];
                o->mass_B += s->rhoB[n];
                double w = 0.5 * (1.0 + rN);
                sw += w;
                for (int a = 0; a < 3; ++a) sx[a] += w * c[a];
                if (rN >= 0.0) { /* eq 34 */
                    sN += 1.0;
                    for (int a = 0; a < s->D; ++a) su[a] += s->u[a][n];
                }
                sG += s->G[n];
                sGp += s->G[n] * s->psi[n];
                if (fabs(rN) <= 0.5) { pmin = fmin(pmin, s->psi[n]); pmax = fmax(pmax, s->psi[n]); }
                double pr = s->rhoR[n] * s->cs2[0] + s->rhoB[n] * s->cs2[1];
                if (rN > 0.99) { pin += pr; nin += 1.0; }
                if (rN < -0.99) { pout += pr; nout += 1.0; }
            }
    o->wsum = sw;
    o->nsum = sN;
    for (int a = 0; a < 3; ++a) {
        o->centroid[a] = sw > 0 ? sx[a] / sw : 0.0;
        o->velocity[a] = sN > 0 ? su[a] / sN : 0.0;
    }
    double m2[6] = {0, 0, 0, 0, 0, 0};
    for (long z = 0; z < s->nz; ++z)
        for (long y = 0; y < s->ny; ++y)
            for (long x = 0; x < s->nx; ++x) {
                long n = IDX(s, x, y, z);
                double w = 0.5 * (1.0 + s->rhoN[n]);
                double d[3] = {x - o->centroid[0], y - o->centroid[1], z - o->centroid[2]};
                m2[0] += w * d[0] * d[0]; m2[1] += w * d[1] * d[1]; m2[2] += w * d[2] * d[2];
                m2[3] += w * d[0] * d[1]; m2[4] += w * d[0] * d[2]; m2[5] += w * d[1] * d[2];
            }
    for (int k = 0; k < 6; ++k) o->second[k] = sw > 0 ? m2[k] / sw : 0.0;
    o->psi_av = sG > 0 ? sGp / sG : 0.0;
    o->psi_min = pmin;
    o->psi_max = pmax;
    o->p_in = nin > 0 ? pin / nin : 0.0;
    o->p_out = nout > 0 ? pout / nout : 0.0;
    o->status = ORC_OK;
    return ORC_OK;
}

/* ----------------------------------------------------- operator-level entry points
   for the pin tests: each applies one operator of the step to caller arrays. */

void orc_lattice(const orc_state *s, int *Q, int *D, int *e, double *w, double *M, double *Minv,
                 double *alpha, double *cs2)
{
    *Q = s->Q;
    *D = s->D;
    for (int i = 0; i < s->Q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = s->e[i][a];
        w[i] = s->w[i];
        for (int k = 0; k < s->Q; ++k) { M[i * s->Q + k] = s->M[i][k]; Minv[i * s->Q + k] = s->Minv[i][k]; }
    }
    alpha[0] = s->alpha[0]; alpha[1] = s->alpha[1];
    cs2[0] = s->cs2[0]; cs2[1] = s->cs2[1];
}

void orc_moment_eq(const orc_state *s, int k, double rho, const double *u, double *m) { moment_eq(s, k, rho, u, m); }

double orc_sigma(const orc_state *s, double psi)
{
    const orc_params *p = &s->p;
    if (p->E0 == 0.0) return p->sigma0;
    if (p->eos_mode == 1) return p->sigma0 * (1.0 - p->E0 * psi / p->psi_inf); /* Sec 3.2 */
    return fmax(p->sigma0 * (1.0 + p->E0 * log(1.0 - psi / p->psi_inf)), p->sigma_min_ratio * p->sigma0); /* eq 8 */
}

void orc_op_deriv(const orc_state *s, const double *chi, int odd_axis, int a, double *out)
{
    op_deriv(s, chi, odd_axis, a, out);
}

void orc_op_weno_div(const orc_state *s, const double *Psi, const double *u, double *out)
{
    double *P[3], *U[3];
    for (int a = 0; a < 3; ++a) { P[a] = (double *)Psi + a * s->N; U[a] = (double *)u + a * s->N; }
    op_weno_div(s, P, U, out);
}

void orc_op_diffusion(const orc_state *s, const double *W, const double *chi, double *out)
{
    op_diffusion(s, W, chi, out);
}

int orc_op_solve(const orc_state *s, const double *W, double Dc, const double *rhs, double *chi)
{
    return op_solve(s, W, Dc, rhs, chi);
}

/* Collision and recolouring without propagation: returns f_dag, f^R and f^B
   after recolouring (each Q x N) for the current state. */
int orc_collide_only(orc_state *s, double *fdag, double *fRr, double *fBr)
{
    if (!s) return ORC_EINVAL;
    orc_params keep = s->p;
    long N = s->N;
    int Q = s->Q;
    force_stage(s);
    /* run the LB stage on fully periodic copies so that no population bounces */
    for (int a = 0; a < 3; ++a) s->p.bc[a] = 0;
    s->dump_fdag = fdag;
    lb_stage(s);
    s->dump_fdag = NULL;
    s->p = keep;
    /* undo propagation: the population that arrived at x + e_i came from x */
    for (long z = 0; z < s->nz; ++z)
        for (long y = 0; y < s->ny; ++y)
            for (long x = 0; x < s->nx; ++x) {
                long n = IDX(s, x, y, z);
                for (int i = 0; i < Q; ++i) {
                    int dm = 0;
                    long X = map_coord(x + s->e[i][0], s->nx, 0, &dm);
                    long Y = map_coord(y + s->e[i][1], s->ny, 0, &dm);
                    long Z = map_coord(z + s->e[i][2], s->nz, 0, &dm);
                    long d = IDX(s, X, Y, Z);
                    fRr[i * N + n] = s->fR2[i * N + d];
                    fBr[i * N + n] = s->fB2[i * N + d];
                }
            }
    return ORC_OK;
}
