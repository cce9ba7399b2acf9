/*
 * Plain FP64 CPU oracle of the iterative discrete-velocity scheme for the
 * steady Shakhov model equation (Zhu, Wang, Chen, Guo, Zhang, "GPU
 * acceleration of an iterative scheme for gas-kinetic model equations with
 * memory reduction techniques", arXiv:1810.00348).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it exists so that the tests, the smoke check and the CPU
 * baseline of the benchmark have an independent, slow, obviously correct
 * reference.  It shares no code, header or table with the HIP library.
 *
 * What it computes (one outer iteration n -> n+1):
 *   - per cell: rho, U, T, tau from the conserved moments of iteration n
 *     (Sec. 2.1, eqs. "shak", "feq", "mom"; viscosity law and mu_ref from
 *     Sec. 4, eq. "mu_ref"), the Shakhov equilibrium f^S (eq. "feq") with the
 *     heat flux q^n, plus the conservative correction that makes the discrete
 *     mass, momentum and energy of the equilibrium equal those of f;
 *   - per discrete velocity, ONE velocity at a time (the velocity-space
 *     memory reduction of Sec. 2.2): a first-order upwind sweep along the
 *     characteristic direction (eqs. "iter_outer", "sweeping_example"), the
 *     boundary values being the diffuse-wall emission (eqs. "maxwell_wall",
 *     "rho_wall"), the free-stream equilibrium, or the specular mirror image;
 *     optionally (orc_set_order) the second-order upwind sweep that the
 *     paper's closing section proposes (three consecutive cells per axis:
 *     each face carries the upwind cell's value extrapolated linearly from
 *     that cell and its own upwind neighbour, with the cells' sizes on a
 *     stretched mesh);
 *   - optionally (orc_set_model) the ES-BGK model in place of Shakhov's:
 *     an anisotropic Gaussian built from the stress of the iterate,
 *     relaxing with frequency Pr p / mu, corrected the same way;
 *   - the discrete moments of eq. "macros" of the new f.  The heat flux uses
 *     the NEW bulk velocity U^{n+1}, so each velocity is swept twice: once for
 *     rho, rho U, rho E and the wall fluxes, once for q (the sweep is a
 *     deterministic function of the iteration-n state, so both passes
 *     produce the same f);
 *   - wall densities from the non-penetration condition (discrete
 *     normalisation), total-mass rescaling for a closed domain (Sec. 3.4),
 *     and the relative change of the conserved fields (Sec. 4.1).
 *
 * The velocity axes are uniform with trapezoid weights (Sec. 4.1) unless
 * orc_set_velocity_axis supplies other nodes and weights.
 *
 * Normalisation: lengths by the reference length L that defines Kn,
 * velocities by sqrt(2 R T0), temperature by T0, density by rho0.  Hence
 * R T = T/2, p = rho T/2, f^M = rho (pi T)^{-3/2} exp(-|c|^2/T),
 * rho E = rho |U|^2/2 + 3 rho T/4, tau = kappa Kn T^(omega-1) / rho with
 * kappa = 15 sqrt(pi) / ((5 - 2 omega)(7 - 2 omega)).
 *
 * Parity pins for every function here live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR -1

/* face kinds */
#define FACE_WALL 0       /* Maxwell diffuse wall                         */
#define FACE_FREE 1       /* free stream: incoming particles equilibrium */
#define FACE_SPECULAR 2   /* symmetry plane: mirror reflection           */

typedef struct {
    int nx, ny, nz;
    double lx, ly, lz;
    int m[3];
    double vmax[3];
    double kn, omega, pr;
    int correction;         /* 1: conservative correction of f^S          */
    int face_kind[6];       /* x-, x+, y-, y+, z-, z+                       */
    double face_u[6][3];
    double face_T[6];
    double face_rho[6];     /* free-stream density (FACE_FREE only)       */
    int closed;             /* 1: rescale total mass every iteration       */
    double solid_u[3];
    double solid_T;
    int threads;            /* 0: OpenMP default                           */
} orc_case;

typedef struct {
    orc_case c;
    int N, NV;
    double dx[3];
    double *h[3];           /* cell size along each axis, per index (the
                               paper's cube runs use stretched meshes,
                               Sec. 4.2); uniform lx/nx ... by default     */
    double *xi[3], *w1[3];
    unsigned char *solid;   /* N, may be all zero                          */
    /* wall / free-stream emission shapes: kinds 0..5 = the six domain
       faces, kind 6 = the solid body                                         */
    double *ghat[7];        /* NV each: unit-density corrected Maxwellian  */
    double gout[7][6];      /* sum over emitted velocities of w (xi.n) ghat */
    /* state */
    double *W;              /* 5 x N: rho, rho Ux, rho Uy, rho Uz, rho E   */
    double *q;              /* 3 x N                                       */
    double *rho_w;          /* 6 x N: wall density of each wall face       */
    double M0;
    double res[5];
    int iter;
    int order;              /* 1: first-order upwind (the paper's scheme);
                               2: second-order upwind (Sec. 6 outlook)    */
    int model;              /* 0: Shakhov (the paper's), 1: ES-BGK         */
    double *P;              /* 6 x N: Theta = (1/rho) sum w c c f, the
                               stress of the current iterate per unit mass
                               (xx, yy, zz, xy, xz, yz; ES-BGK only)      */
} orc_state;

/* ----------------------------------------------------------------------- */
/* velocity grid: M uniform nodes on [-V, V] including both end points,     */
/* trapezoidal weights (Sec. 4.1: uniform grid, trapezoidal rule).          */
/* ----------------------------------------------------------------------- */
int orc_velocity_axis(int M, double V, double *xi, double *w)
{
    if (M < 2 || !(V > 0)) return ORC_ERR;
    double h = 2.0 * V / (M - 1);
    double half = V / (M - 1);
    for (int a = 0; a < M; ++a) {
        /* (2a - (M-1)) is an exact integer, so xi_{M-1-a} = -xi_a exactly */
        xi[a] = (double)(2 * a - (M - 1)) * half;
        w[a] = (a == 0 || a == M - 1) ? 0.5 * h : h;
    }
    return ORC_OK;
}

double orc_kappa(double omega)
{
    /* tau = mu / p with mu = mu_ref (T/T_ref)^omega and mu_ref of eq.
       "mu_ref"; in the units above tau(rho=1,T=1) = kappa * Kn.             */
    return 15.0 * sqrt(M_PI) / ((5.0 - 2.0 * omega) * (7.0 - 2.0 * omega));
}

static int cell_index(const orc_case *c, int i, int j, int k)
{
    return i + c->nx * (j + c->ny * k);
}

/* Solve the symmetric positive definite 5x5 system A x = b (Cholesky). */
static int spd_solve5(double A[5][5], double b[5], double x[5])
{
    double L[5][5] = {{0}};
    for (int i = 0; i < 5; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0)) return ORC_ERR;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double y[5];
    for (int i = 0; i < 5; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
    for (int i = 4; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 5; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return ORC_OK;
}

/*
 * Shakhov equilibrium on the discrete velocity set (eq. "feq"), written in
 * the normalised units, followed (if correct != 0) by the conservative
 * correction: f~ = f^S + f^M * sum_k lambda_k phi_k with
 * phi = (1, c_x, c_y, c_z, |c|^2), lambda chosen so that
 *   sum_a w_a phi_l(c_a) f~_a = (rho, 0, 0, 0, 3 rho T / 2),
 * i.e. the discrete mass, momentum and energy of f~ are exactly those the
 * state (rho, U, T) was computed from.  All sums run over the full grid.
 */
/* ES-BGK (Holway's ellipsoidal statistical model; the paper states that the
   scheme applies to other model equations than Shakhov's, Sec. 2.1).  In the
   normalised units (R T = T/2) its Gaussian is
     G = rho (2 pi)^{-3/2} det(Lam)^{-1/2} exp(-c^T Lam^{-1} c / 2),
     Lam = (T/2) I / Pr + (1 - 1/Pr) Theta,
   Theta the stress per unit mass; it relaxes with frequency Pr p / mu, so
   that both the viscosity and the Prandtl number are those of the gas.     */
static int es_tensor(double T, const double th[6], double pr, double inv[6], double *det)
{
    /* Lam in (xx, yy, zz, xy, xz, yz) order */
    double L[6];
    for (int k = 0; k < 6; ++k) L[k] = (1.0 - 1.0 / pr) * th[k];
    for (int k = 0; k < 3; ++k) L[k] += 0.5 * T / pr;
    const double a = L[0], b = L[1], c = L[2], d = L[3], e = L[4], f = L[5];
    /* cofactors of the symmetric matrix [[a d e] [d b f] [e f c]] */
    const double A = b * c - f * f, B = a * c - e * e, C = a * b - d * d;
    const double D = e * f - d * c, E = d * f - e * b, F = d * e - a * f;
    const double dt = a * A + d * D + e * E;
    if (!(dt > 0) || !(A > 0) || !(C > 0)) return ORC_ERR;   /* not positive definite */
    inv[0] = A / dt; inv[1] = B / dt; inv[2] = C / dt;
    inv[3] = D / dt; inv[4] = E / dt; inv[5] = F / dt;
    *det = dt;
    return ORC_OK;
}

static double es_exponent(const double inv[6], double cx, double cy, double cz)
{
    return 0.5 * (inv[0] * cx * cx + inv[1] * cy * cy + inv[2] * cz * cz) +
           inv[3] * cx * cy + inv[4] * cx * cz + inv[5] * cy * cz;
}

/* The ES-BGK Gaussian (no correction) on the velocity grid. */
int orc_esbgk_gaussian(const int m[3], const double *const xi[3], double rho, const double U[3],
                       double T, const double theta[6], double pr, double *out)
{
    double inv[6], det;
    if (!(rho > 0) || !(T > 0) || es_tensor(T, theta, pr, inv, &det)) return ORC_ERR;
    const double pre = rho * pow(2.0 * M_PI, -1.5) / sqrt(det);
    for (int c3 = 0; c3 < m[2]; ++c3)
        for (int b3 = 0; b3 < m[1]; ++b3)
            for (int a3 = 0; a3 < m[0]; ++a3) {
                int al = a3 + m[0] * (b3 + m[1] * c3);
                out[al] = pre * exp(-es_exponent(inv, xi[0][a3] - U[0], xi[1][b3] - U[1], xi[2][c3] - U[2]));
            }
    return ORC_OK;
}

int orc_equilibrium(const int m[3], const double *const xi[3],
                    const double *const w1[3], double rho, const double U[3],
                    double T, const double qv[3], double pr, int correct,
                    double *out)
{
    if (!(rho > 0) || !(T > 0)) return ORC_ERR;
    int NV = m[0] * m[1] * m[2];
    double pre = rho * pow(M_PI * T, -1.5);
    double sig = (1.0 - pr) * 4.0 / (5.0 * rho * T * T);
    double A[5][5] = {{0}}, b[5] = {0};
    for (int c3 = 0; c3 < m[2]; ++c3)
        for (int b3 = 0; b3 < m[1]; ++b3)
            for (int a3 = 0; a3 < m[0]; ++a3) {
                int al = a3 + m[0] * (b3 + m[1] * c3);
                double cx = xi[0][a3] - U[0];
                double cy = xi[1][b3] - U[1];
                double cz = xi[2][c3] - U[2];
                double c2 = cx * cx + cy * cy + cz * cz;
                double fm = pre * exp(-c2 / T);
                double cq = cx * qv[0] + cy * qv[1] + cz * qv[2];
                double fs = fm * (1.0 + sig * cq * (2.0 * c2 / T - 5.0));
                out[al] = fs;
                if (correct) {
                    double w = w1[0][a3] * w1[1][b3] * w1[2][c3];
                    double phi[5] = {1.0, cx, cy, cz, c2};
                    for (int l = 0; l < 5; ++l) {
                        b[l] -= w * phi[l] * fs;
                        for (int k = 0; k < 5; ++k)
                            A[l][k] += w * phi[l] * phi[k] * fm;
                    }
                }
            }
    if (!correct) return ORC_OK;
    b[0] += rho;
    b[4] += 1.5 * rho * T;
    double lam[5];
    if (spd_solve5(A, b, lam) != ORC_OK) return ORC_ERR;
    for (int c3 = 0; c3 < m[2]; ++c3)
        for (int b3 = 0; b3 < m[1]; ++b3)
            for (int a3 = 0; a3 < m[0]; ++a3) {
                int al = a3 + m[0] * (b3 + m[1] * c3);
                double cx = xi[0][a3] - U[0];
                double cy = xi[1][b3] - U[1];
                double cz = xi[2][c3] - U[2];
                double c2 = cx * cx + cy * cy + cz * cz;
                double fm = pre * exp(-c2 / T);
                out[al] += fm * (lam[0] + lam[1] * cx + lam[2] * cy +
                                 lam[3] * cz + lam[4] * c2);
            }
    (void)NV;
    return ORC_OK;
}

/* primitive variables of a cell from its conserved moments (eq. "mom") */
static int primitives(const double *W, int N, int cell, double *rho,
                      double U[3], double *T)
{
    double r = W[0 * N + cell];
    if (!(r > 0)) return ORC_ERR;
    U[0] = W[1 * N + cell] / r;
    U[1] = W[2 * N + cell] / r;
    U[2] = W[3 * N + cell] / r;
    double ke = 0.5 * r * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
    double t = (W[4 * N + cell] - ke) / (0.75 * r);
    if (!(t > 0)) return ORC_ERR;
    *rho = r;
    *T = t;
    return ORC_OK;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    for (int d = 0; d < 3; ++d) { free(s->xi[d]); free(s->w1[d]); free(s->h[d]); }
    for (int k = 0; k < 7; ++k) free(s->ghat[k]);
    free(s->solid); free(s->W); free(s->q); free(s->rho_w); free(s->P);
    free(s);
}

/* volume of cell id (finite-volume cell of a tensor-product mesh) */
static double cell_volume(const orc_state *s, int id)
{
    const orc_case *c = &s->c;
    const int i = id % c->nx, j = (id / c->nx) % c->ny, k = id / (c->nx * c->ny);
    return s->h[0][i] * s->h[1][j] * s->h[2][k];
}

/* Non-uniform cell sizes along each axis (NULL keeps that axis uniform);
   before the initial state is set.  The sizes must be positive. */
int orc_set_spacing(orc_state *s, const double *hx, const double *hy, const double *hz)
{
    const double *in[3] = {hx, hy, hz};
    const int n3[3] = {s->c.nx, s->c.ny, s->c.nz};
    for (int d = 0; d < 3; ++d) {
        if (!in[d]) continue;
        for (int i = 0; i < n3[d]; ++i)
            if (!(in[d][i] > 0)) return ORC_ERR;
    }
    for (int d = 0; d < 3; ++d)
        if (in[d]) memcpy(s->h[d], in[d], sizeof(double) * n3[d]);
    return ORC_OK;
}

/* Spatial order of the upwind scheme (1 or 2).  The second order is the one
   the paper's closing section proposes, built from three consecutive cells
   along each axis (see sweep_velocity); on uniform and stretched meshes.   */
int orc_set_order(orc_state *s, int order)
{
    if (order != 1 && order != 2) return ORC_ERR;
    s->order = order;
    return ORC_OK;
}

/* Collision model: 0 Shakhov (default), 1 ES-BGK. */
int orc_set_model(orc_state *s, int model)
{
    if (model != 0 && model != 1) return ORC_ERR;
    s->model = model;
    return ORC_OK;
}

int orc_get_stress(const orc_state *s, double *P)
{
    memcpy(P, s->P, sizeof(double) * 6 * s->N);
    return ORC_OK;
}

/* side s of a cell: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+; the normal pointing
   from that face INTO the cell (into the gas) is -(side odd ? +e_d : -e_d). */
static double into_gas_normal_sign(int side) { return (side & 1) ? -1.0 : 1.0; }

/* Unit-density emission shapes of the six faces and the solid body (the
   corrected Maxwellian of each face's wall or free-stream state) and their
   emitted-flux normalisers for every face orientation, on the current
   velocity axes.                                                           */
static int emission_tables(orc_state *s)
{
    const double zero3[3] = {0, 0, 0};
    int any_solid = 0;
    for (int id = 0; id < s->N; ++id) any_solid |= s->solid[id];
    for (int k = 0; k < 7; ++k) {
        if (k == 6 && !any_solid) continue;
        const double *u = k < 6 ? s->c.face_u[k] : s->c.solid_u;
        double T = k < 6 ? s->c.face_T[k] : s->c.solid_T;
        if (k < 6 && s->c.face_kind[k] == FACE_SPECULAR) continue;
        if (!(T > 0)) return ORC_ERR;
        free(s->ghat[k]);
        s->ghat[k] = (double *)malloc(sizeof(double) * s->NV);
        if (orc_equilibrium(s->c.m, (const double *const *)s->xi,
                            (const double *const *)s->w1, 1.0, u, T, zero3,
                            s->c.pr, s->c.correction, s->ghat[k])) {
            return ORC_ERR;
        }
        /* emitted-flux normaliser for each possible face orientation */
        for (int side = 0; side < 6; ++side) {
            int d = side >> 1;
            double ns = into_gas_normal_sign(side);
            double g = 0;
            for (int c3 = 0; c3 < s->c.m[2]; ++c3)
                for (int b3 = 0; b3 < s->c.m[1]; ++b3)
                    for (int a3 = 0; a3 < s->c.m[0]; ++a3) {
                        int idx[3] = {a3, b3, c3};
                        double xn = s->xi[d][idx[d]] * ns;
                        if (xn > 0) {
                            int al = a3 + s->c.m[0] * (b3 + s->c.m[1] * c3);
                            double w = s->w1[0][a3] * s->w1[1][b3] * s->w1[2][c3];
                            g += w * xn * s->ghat[k][al];
                        }
                    }
            s->gout[k][side] = g;
        }
    }
    return ORC_OK;
}

/* Nodes and quadrature weights of velocity axis d (m[d] values each) in
   place of the uniform trapezoid axis -- the non-uniform velocity grids the
   paper recommends over very large uniform ones (Sec. 5.2).  The nodes must
   increase and be symmetric about 0 (xi[M-1-a] = -xi[a]), the weights be
   positive and symmetric.  Before the initial state is set.                */
int orc_set_velocity_axis(orc_state *s, int d, const double *xi, const double *w)
{
    if (!s || d < 0 || d > 2 || !xi || !w) return ORC_ERR;
    const int M = s->c.m[d];
    double big = 0;
    for (int a = 0; a < M; ++a) big = fmax(big, fabs(xi[a]));
    for (int a = 0; a < M; ++a) {
        if (!(w[a] > 0) || !isfinite(xi[a])) return ORC_ERR;
        if (a > 0 && !(xi[a] > xi[a - 1])) return ORC_ERR;
        if (fabs(xi[a] + xi[M - 1 - a]) > 1e-12 * big) return ORC_ERR;
        if (fabs(w[a] - w[M - 1 - a]) > 1e-12 * w[a]) return ORC_ERR;
    }
    memcpy(s->xi[d], xi, sizeof(double) * M);
    memcpy(s->w1[d], w, sizeof(double) * M);
    return emission_tables(s);
}

orc_state *orc_create(const orc_case *cfg, const unsigned char *solid)
{
    if (!cfg) return NULL;
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return NULL;
    if (!(cfg->lx > 0) || !(cfg->ly > 0) || !(cfg->lz > 0)) return NULL;
    if (!(cfg->kn > 0) || !(cfg->pr > 0)) return NULL;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    s->c = *cfg;
    s->N = cfg->nx * cfg->ny * cfg->nz;
    s->NV = cfg->m[0] * cfg->m[1] * cfg->m[2];
    s->dx[0] = cfg->lx / cfg->nx;
    s->dx[1] = cfg->ly / cfg->ny;
    s->dx[2] = cfg->lz / cfg->nz;
    {
        const int n3[3] = {cfg->nx, cfg->ny, cfg->nz};
        for (int d = 0; d < 3; ++d) {
            s->h[d] = (double *)malloc(sizeof(double) * n3[d]);
            for (int i = 0; i < n3[d]; ++i) s->h[d][i] = s->dx[d];
        }
    }
    for (int d = 0; d < 3; ++d) {
        s->xi[d] = (double *)malloc(sizeof(double) * cfg->m[d]);
        s->w1[d] = (double *)malloc(sizeof(double) * cfg->m[d]);
        if (orc_velocity_axis(cfg->m[d], cfg->vmax[d], s->xi[d], s->w1[d])) {
            orc_destroy(s);
            return NULL;
        }
    }
    s->order = 1;
    s->solid = (unsigned char *)calloc(s->N, 1);
    if (solid) memcpy(s->solid, solid, s->N);
    if (emission_tables(s)) {
        orc_destroy(s);
        return NULL;
    }
    s->W = (double *)calloc((size_t)5 * s->N, sizeof(double));
    s->q = (double *)calloc((size_t)3 * s->N, sizeof(double));
    s->rho_w = (double *)calloc((size_t)6 * s->N, sizeof(double));
    s->P = (double *)calloc((size_t)6 * s->N, sizeof(double));
    return s;
}

/* what lies beyond side `side` of fluid cell (i,j,k):
   returns -1 for an interior fluid neighbour (its index in *nb),
   otherwise the emission kind index (0..5 domain face, 6 solid body),
   or 100 + FACE_SPECULAR for a symmetry plane.                             */
static int face_type(const orc_state *s, int i, int j, int k, int side, int *nb)
{
    const orc_case *c = &s->c;
    int d = side >> 1, up = side & 1;
    int ii = i, jj = j, kk = k;
    int *p = d == 0 ? &ii : d == 1 ? &jj : &kk;
    int n = d == 0 ? c->nx : d == 1 ? c->ny : c->nz;
    *p += up ? 1 : -1;
    if (*p < 0 || *p >= n) {
        if (c->face_kind[side] == FACE_SPECULAR) return 100 + FACE_SPECULAR;
        return side;
    }
    int id = cell_index(c, ii, jj, kk);
    if (s->solid[id]) return 6;
    *nb = id;
    return -1;
}

/* is the emission kind a diffuse wall (density from non-penetration)?    */
static int kind_is_wall(const orc_state *s, int kind)
{
    if (kind == 6) return 1;
    return s->c.face_kind[kind] == FACE_WALL;
}

typedef struct {
    double *rho, *U, *T, *nu, *q;   /* per cell */
    double *esinv, *espre;           /* ES-BGK: Lam^{-1} (6) and prefactor */
} cellprm;

/* One upwind sweep of discrete velocity al (eq. "sweeping_example" in the
 * finite-volume flux form: the upwind value at a boundary or solid face is
 * that face's inflow value).  feq: corrected equilibrium of this velocity
 * at every cell (nu-weighted source).  spec_mirror: the z=0 plane of the
 * mirrored velocity (symmetry plane), two planes of nx*ny values -- its f,
 * then what it carries through z = 0 (its fo along z) -- or NULL.  The
 * mirror image stands for the cell beyond the plane, so with the second
 * order the plane is an interior face.
 *
 * fo[d] (3 x N): the value this velocity carries through each cell's
 * downstream face along axis d.  First order: the cell value.  Second
 * order: the linear profile through the centres of the cell and of its
 * upwind neighbour along d, evaluated at the cell's downstream face:
 * f + theta (f - f_up) with theta = h / (h + h_up), h and h_up the two cells'
 * sizes along d (1/2 on a uniform mesh; the mirror image beyond a symmetry
 * plane has the cell's own size), or the cell value when the upwind side is
 * a boundary.  The cell balance is then, per axis with a = |xi_d| / h,
 * a (fo_d(cell) - fo_d(upwind)) (the boundary's inflow value in place of
 * fo_d(upwind) at a boundary), so that the unknown f enters with
 * coefficient (1 + theta) a behind an interior face and a behind a
 * boundary.                                                                 */
static void sweep_velocity(const orc_state *s, int a3, int b3, int c3,
                           const double *feq, const double *nu,
                           const double *spec_mirror, double *f, double *fo)
{
    const int N = s->N;
    const orc_case *c = &s->c;
    int al = a3 + c->m[0] * (b3 + c->m[1] * c3);
    double xv[3] = {s->xi[0][a3], s->xi[1][b3], s->xi[2][c3]};
    int sg[3];
    for (int d = 0; d < 3; ++d) sg[d] = xv[d] >= 0 ? 1 : -1;
    for (int kq = 0; kq < c->nz; ++kq) {
        int k = sg[2] > 0 ? kq : c->nz - 1 - kq;
        for (int jq = 0; jq < c->ny; ++jq) {
            int j = sg[1] > 0 ? jq : c->ny - 1 - jq;
            for (int iq = 0; iq < c->nx; ++iq) {
                int i = sg[0] > 0 ? iq : c->nx - 1 - iq;
                int id = cell_index(c, i, j, k);
                if (s->solid[id]) {
                    f[id] = 0;
                    for (int d = 0; d < 3; ++d) fo[(size_t)d * N + id] = 0;
                    continue;
                }
                double num = nu[id] * feq[id];
                double den = nu[id];
                double up[3] = {0, 0, 0};  /* f of the interior upwind cell */
                double th[3] = {0, 0, 0};  /* second order: extrapolation weight */
                int interior[3] = {0, 0, 0};
                /* |xi_d| / (cell size along d): the flux through the cell's
                   upwind face per unit volume                               */
                const double ad[3] = {fabs(xv[0]) / s->h[0][i], fabs(xv[1]) / s->h[1][j],
                                      fabs(xv[2]) / s->h[2][k]};
                for (int d = 0; d < 3; ++d) {
                    if (ad[d] == 0) continue;
                    int side = 2 * d + (sg[d] > 0 ? 0 : 1); /* upwind side */
                    int nb = -1;
                    int t = face_type(s, i, j, k, side, &nb);
                    double fu;
                    if (s->order == 2 && (t < 0 || t == 100 + FACE_SPECULAR)) {
                        /* inflow = the upwind cell's downstream face value;
                           own outflow f + (f - f_up)/2 adds a/2 (f - f_up) */
                        const int nxy = c->nx * c->ny, ij = i + c->nx * j;
                        const double fup = t < 0 ? f[nb] : spec_mirror[ij];
                        const double fin = t < 0 ? fo[(size_t)d * N + nb] : spec_mirror[nxy + ij];
                        const int pos[3] = {i, j, k};
                        const double hc = s->h[d][pos[d]];
                        const double hu = t < 0 ? s->h[d][pos[d] - sg[d]] : hc;
                        th[d] = hc / (hc + hu);
                        interior[d] = 1;
                        up[d] = fup;
                        num += ad[d] * (fin + th[d] * fup);
                        den += (1.0 + th[d]) * ad[d];
                        continue;
                    }
                    if (t < 0) fu = f[nb];
                    else if (t == 100 + FACE_SPECULAR) fu = spec_mirror[i + c->nx * j];
                    else if (kind_is_wall(s, t)) fu = s->rho_w[side * s->N + id] * s->ghat[t][al];
                    else fu = c->face_rho[t] * s->ghat[t][al];
                    num += ad[d] * fu;
                    den += ad[d];
                }
                f[id] = num / den;
                for (int d = 0; d < 3; ++d)
                    fo[(size_t)d * N + id] = interior[d] ? f[id] + th[d] * (f[id] - up[d]) : f[id];
            }
        }
    }
}

/* is z- a specular plane? */
static int has_specular(const orc_state *s) { return s->c.face_kind[4] == FACE_SPECULAR; }

int orc_init_fields(orc_state *s, const double *rho, const double *u,
                    const double *T)
{
    int N = s->N;
    for (int id = 0; id < N; ++id) {
        if (s->solid[id]) {
            for (int v = 0; v < 5; ++v) s->W[v * N + id] = 0;
            continue;
        }
        if (!(rho[id] > 0) || !(T[id] > 0) || !isfinite(u[id]) ||
            !isfinite(u[N + id]) || !isfinite(u[2 * N + id]))
            return ORC_ERR;
        double U[3] = {u[id], u[N + id], u[2 * N + id]};
        s->W[0 * N + id] = rho[id];
        s->W[1 * N + id] = rho[id] * U[0];
        s->W[2 * N + id] = rho[id] * U[1];
        s->W[3 * N + id] = rho[id] * U[2];
        s->W[4 * N + id] = 0.5 * rho[id] * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]) +
                           0.75 * rho[id] * T[id];
    }
    memset(s->q, 0, sizeof(double) * 3 * N);
    /* equilibrium stress per unit mass: (T/2) I */
    memset(s->P, 0, sizeof(double) * 6 * N);
    for (int id = 0; id < N; ++id)
        if (!s->solid[id])
            for (int k = 0; k < 3; ++k) s->P[k * N + id] = 0.5 * T[id];
    double m0 = 0;
    for (int id = 0; id < N; ++id) if (!s->solid[id]) m0 += s->W[id] * cell_volume(s, id);
    s->M0 = m0;
    /* initial wall densities: non-penetration with the equilibrium of the
       initial state at the wall-adjacent cell                              */
    memset(s->rho_w, 0, sizeof(double) * 6 * N);
    const orc_case *c = &s->c;
    double *fe = (double *)malloc(sizeof(double) * s->NV);
    for (int k = 0; k < c->nz; ++k)
        for (int j = 0; j < c->ny; ++j)
            for (int i = 0; i < c->nx; ++i) {
                int id = cell_index(c, i, j, k);
                if (s->solid[id]) continue;
                int any = 0;
                int kinds[6];
                for (int side = 0; side < 6; ++side) {
                    int nb;
                    kinds[side] = face_type(s, i, j, k, side, &nb);
                    if (kinds[side] >= 0 && kinds[side] < 100 && kind_is_wall(s, kinds[side])) any = 1;
                }
                if (!any) continue;
                double r, U[3], T0;
                primitives(s->W, N, id, &r, U, &T0);
                const double q0[3] = {0, 0, 0};
                orc_equilibrium(c->m, (const double *const *)s->xi,
                                (const double *const *)s->w1, r, U, T0, q0,
                                c->pr, c->correction, fe);
                for (int side = 0; side < 6; ++side) {
                    int t = kinds[side];
                    if (t < 0 || t >= 100 || !kind_is_wall(s, t)) continue;
                    int d = side >> 1;
                    double ns = into_gas_normal_sign(side);
                    double flux = 0;
                    for (int c3 = 0; c3 < c->m[2]; ++c3)
                        for (int b3 = 0; b3 < c->m[1]; ++b3)
                            for (int a3 = 0; a3 < c->m[0]; ++a3) {
                                int idx[3] = {a3, b3, c3};
                                double xn = s->xi[d][idx[d]] * ns;
                                if (xn < 0) {
                                    int al = a3 + c->m[0] * (b3 + c->m[1] * c3);
                                    double w = s->w1[0][a3] * s->w1[1][b3] * s->w1[2][c3];
                                    flux += w * (-xn) * fe[al];
                                }
                            }
                    s->rho_w[side * N + id] = flux / s->gout[t][side];
                }
            }
    free(fe);
    s->iter = 0;
    for (int v = 0; v < 5; ++v) s->res[v] = 0;
    return ORC_OK;
}

int orc_init_uniform(orc_state *s, double rho, const double u[3], double T)
{
    int N = s->N;
    double *r = (double *)malloc(sizeof(double) * N);
    double *uu = (double *)malloc(sizeof(double) * 3 * N);
    double *t = (double *)malloc(sizeof(double) * N);
    for (int id = 0; id < N; ++id) {
        r[id] = rho; t[id] = T;
        uu[id] = u[0]; uu[N + id] = u[1]; uu[2 * N + id] = u[2];
    }
    int st = orc_init_fields(s, r, uu, t);
    free(r); free(uu); free(t);
    return st;
}

/* per-cell equilibrium parameters of the current state */
static int cell_params(const orc_state *s, cellprm *p)
{
    int N = s->N;
    double kap = orc_kappa(s->c.omega);
    for (int id = 0; id < N; ++id) {
        if (s->solid[id]) { p->nu[id] = 0; continue; }
        double r, U[3], T;
        if (primitives(s->W, N, id, &r, U, &T)) return ORC_ERR;
        p->rho[id] = r; p->T[id] = T;
        for (int d = 0; d < 3; ++d) {
            p->U[d * N + id] = U[d];
            p->q[d * N + id] = s->q[d * N + id];
        }
        double tau = kap * s->c.kn * pow(T, s->c.omega - 1.0) / r;
        p->nu[id] = 1.0 / tau;
        if (s->model == 1) {
            /* ES-BGK relaxes with Pr p / mu */
            p->nu[id] = s->c.pr / tau;
            double th[6], det;
            for (int k = 0; k < 6; ++k) th[k] = s->P[k * N + id];
            if (es_tensor(T, th, s->c.pr, p->esinv + 6 * (size_t)id, &det)) return ORC_ERR;
            p->espre[id] = r * pow(2.0 * M_PI, -1.5) / sqrt(det);
        }
    }
    return ORC_OK;
}

/* Velocity al's corrected equilibrium at every fluid cell. */
static void velocity_feq(const orc_state *s, const cellprm *p, const double *lam,
                         int a3, int b3, int c3, double *feq)
{
    int N = s->N;
    double pr = s->c.pr;
    for (int id = 0; id < N; ++id) {
        if (s->solid[id]) { feq[id] = 0; continue; }
        double rho = p->rho[id], T = p->T[id];
        double cx = s->xi[0][a3] - p->U[id];
        double cy = s->xi[1][b3] - p->U[N + id];
        double cz = s->xi[2][c3] - p->U[2 * N + id];
        double c2 = cx * cx + cy * cy + cz * cz;
        double fm, v;
        if (s->model == 1) {
            fm = p->espre[id] * exp(-es_exponent(p->esinv + 6 * (size_t)id, cx, cy, cz));
            v = fm;
        } else {
            fm = rho * pow(M_PI * T, -1.5) * exp(-c2 / T);
            double cq = cx * p->q[id] + cy * p->q[N + id] + cz * p->q[2 * N + id];
            double sig = (1.0 - pr) * 4.0 / (5.0 * rho * T * T);
            v = fm * (1.0 + sig * cq * (2.0 * c2 / T - 5.0));
        }
        if (lam) {
            const double *L = lam + 5 * (size_t)id;
            v += fm * (L[0] + L[1] * cx + L[2] * cy + L[3] * cz + L[4] * c2);
        }
        feq[id] = v;
    }
}

/* Correction multipliers lambda (5 per cell) obtained with the same plain
   O(M^3) sums as orc_equilibrium.                                           */
static int cell_lambdas(const orc_state *s, const cellprm *p, double *lam)
{
    int N = s->N;
    const orc_case *c = &s->c;
    int err = 0;
#pragma omp parallel for schedule(static)
    for (int id = 0; id < N; ++id) {
        if (s->solid[id]) { for (int l = 0; l < 5; ++l) lam[5 * (size_t)id + l] = 0; continue; }
        double rho = p->rho[id], T = p->T[id];
        double U[3] = {p->U[id], p->U[N + id], p->U[2 * N + id]};
        double qv[3] = {p->q[id], p->q[N + id], p->q[2 * N + id]};
        double pre = rho * pow(M_PI * T, -1.5);
        double sig = (1.0 - c->pr) * 4.0 / (5.0 * rho * T * T);
        double A[5][5] = {{0}}, b[5] = {0};
        for (int c3 = 0; c3 < c->m[2]; ++c3)
            for (int b3 = 0; b3 < c->m[1]; ++b3)
                for (int a3 = 0; a3 < c->m[0]; ++a3) {
                    double cx = s->xi[0][a3] - U[0];
                    double cy = s->xi[1][b3] - U[1];
                    double cz = s->xi[2][c3] - U[2];
                    double c2 = cx * cx + cy * cy + cz * cz;
                    double fm, fs;
                    if (s->model == 1) {
                        /* correct the ES-BGK Gaussian with the same basis */
                        fm = p->espre[id] * exp(-es_exponent(p->esinv + 6 * (size_t)id, cx, cy, cz));
                        fs = fm;
                    } else {
                        fm = pre * exp(-c2 / T);
                        double cq = cx * qv[0] + cy * qv[1] + cz * qv[2];
                        fs = fm * (1.0 + sig * cq * (2.0 * c2 / T - 5.0));
                    }
                    double w = s->w1[0][a3] * s->w1[1][b3] * s->w1[2][c3];
                    double phi[5] = {1.0, cx, cy, cz, c2};
                    for (int l = 0; l < 5; ++l) {
                        b[l] -= w * phi[l] * fs;
                        for (int k = 0; k < 5; ++k) A[l][k] += w * phi[l] * phi[k] * fm;
                    }
                }
        b[0] += rho;
        b[4] += 1.5 * rho * T;
        if (spd_solve5(A, b, lam + 5 * (size_t)id)) {
#pragma omp atomic write
            err = 1;
        }
    }
    return err ? ORC_ERR : ORC_OK;
}

static int nthreads_of(const orc_state *s)
{
#ifdef _OPENMP
    return s->c.threads > 0 ? s->c.threads : omp_get_max_threads();
#else
    (void)s;
    return 1;
#endif
}

/* One outer iteration (eq. "iter_outer").  Returns ORC_OK or ORC_ERR on a
   non-physical state (the state is then left unchanged).                    */
int orc_iterate(orc_state *s)
{
    const orc_case *c = &s->c;
    int N = s->N, NV = s->NV;
    int nth = nthreads_of(s);
#ifdef _OPENMP
    omp_set_num_threads(nth);
#endif
    cellprm p;
    p.rho = (double *)malloc(sizeof(double) * N);
    p.T = (double *)malloc(sizeof(double) * N);
    p.nu = (double *)malloc(sizeof(double) * N);
    p.U = (double *)malloc(sizeof(double) * 3 * N);
    p.q = (double *)malloc(sizeof(double) * 3 * N);
    p.esinv = (double *)malloc(sizeof(double) * 6 * N);
    p.espre = (double *)malloc(sizeof(double) * N);
    double *lam = c->correction ? (double *)malloc(sizeof(double) * 5 * (size_t)N) : NULL;
    int err = cell_params(s, &p);
    if (!err && lam) err = cell_lambdas(s, &p, lam);
    if (err) {
        free(p.rho); free(p.T); free(p.nu); free(p.U); free(p.q); free(p.esinv); free(p.espre); free(lam);
        return ORC_ERR;
    }
    int spec = has_specular(s);
    int nxy = c->nx * c->ny;
    /* z=0 plane values of every velocity moving towards -z (symmetry plane) */
    double *specbuf = spec ? (double *)calloc((size_t)NV * 2 * nxy, sizeof(double)) : NULL;

    /* per-thread accumulators: 5 conserved moments, 3 heat flux, 6 wall
       fluxes (pass 1), then the heat flux (pass 2)                          */
    double *acc = (double *)calloc((size_t)nth * 11 * N, sizeof(double));
    double *Wn = (double *)malloc(sizeof(double) * 5 * N);
    double *qn = (double *)malloc(sizeof(double) * 3 * N);
    double *flux = (double *)malloc(sizeof(double) * 6 * N);
    double *Pn = (double *)calloc((size_t)6 * N, sizeof(double));

    for (int pass = 0; pass < 2; ++pass) {
        memset(acc, 0, sizeof(double) * (size_t)nth * 11 * N);
        /* velocities with xi_z < 0 first, so that with a symmetry plane the
           xi_z > 0 velocities can read their mirror images                   */
        for (int half = 0; half < 2; ++half) {
#pragma omp parallel num_threads(nth)
            {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                double *f = (double *)malloc(sizeof(double) * N);
                double *fo = (double *)malloc(sizeof(double) * 3 * N);
                double *feq = (double *)malloc(sizeof(double) * N);
                double *A = acc + (size_t)tid * 11 * N;
#pragma omp for schedule(static)
                for (int al = 0; al < NV; ++al) {
                    int a3 = al % c->m[0];
                    int b3 = (al / c->m[0]) % c->m[1];
                    int c3 = al / (c->m[0] * c->m[1]);
                    double xz = s->xi[2][c3];
                    if ((half == 0) != (xz < 0)) continue;
                    double xv[3] = {s->xi[0][a3], s->xi[1][b3], xz};
                    double w = s->w1[0][a3] * s->w1[1][b3] * s->w1[2][c3];
                    velocity_feq(s, &p, lam, a3, b3, c3, feq);
                    const double *mir = NULL;
                    if (spec && xz > 0) {
                        int cm = c->m[2] - 1 - c3; /* mirrored z index */
                        int alm = a3 + c->m[0] * (b3 + c->m[1] * cm);
                        mir = specbuf + (size_t)alm * 2 * nxy;
                    }
                    sweep_velocity(s, a3, b3, c3, feq, p.nu, mir, f, fo);
                    /* the mirror image takes what crosses the plane z = 0 */
                    if (spec && xz < 0 && pass == 0)
                        for (int ij = 0; ij < nxy; ++ij) {
                            specbuf[(size_t)al * 2 * nxy + ij] = f[ij];
                            specbuf[((size_t)al * 2 + 1) * nxy + ij] = fo[(size_t)2 * N + ij];
                        }
                    double x2 = xv[0] * xv[0] + xv[1] * xv[1] + xv[2] * xv[2];
                    for (int k = 0; k < c->nz; ++k)
                        for (int j = 0; j < c->ny; ++j)
                            for (int i = 0; i < c->nx; ++i) {
                                int id = cell_index(c, i, j, k);
                                if (s->solid[id]) continue;
                                double wf = w * f[id];
                                if (pass == 0) {
                                    A[0 * N + id] += wf;
                                    A[1 * N + id] += xv[0] * wf;
                                    A[2 * N + id] += xv[1] * wf;
                                    A[3 * N + id] += xv[2] * wf;
                                    A[4 * N + id] += 0.5 * x2 * wf;
                                    /* flux into each diffuse wall face */
                                    for (int side = 0; side < 6; ++side) {
                                        int d = side >> 1;
                                        double xn = xv[d] * into_gas_normal_sign(side);
                                        if (!(xn < 0)) continue;
                                        int nb;
                                        int t = face_type(s, i, j, k, side, &nb);
                                        if (t < 0 || t >= 100 || !kind_is_wall(s, t)) continue;
                                        /* what crosses the wall face */
                                        A[(5 + side) * N + id] += -xn * (w * fo[(size_t)d * N + id]);
                                    }
                                } else {
                                    /* heat flux about the NEW bulk velocity */
                                    double cx = xv[0] - Wn[1 * N + id] / Wn[id];
                                    double cy = xv[1] - Wn[2 * N + id] / Wn[id];
                                    double cz = xv[2] - Wn[3 * N + id] / Wn[id];
                                    double cc = cx * cx + cy * cy + cz * cz;
                                    A[0 * N + id] += 0.5 * cx * cc * wf;
                                    A[1 * N + id] += 0.5 * cy * cc * wf;
                                    A[2 * N + id] += 0.5 * cz * cc * wf;
                                    /* the stress about the new bulk velocity */
                                    A[3 * N + id] += cx * cx * wf;
                                    A[4 * N + id] += cy * cy * wf;
                                    A[5 * N + id] += cz * cz * wf;
                                    A[6 * N + id] += cx * cy * wf;
                                    A[7 * N + id] += cx * cz * wf;
                                    A[8 * N + id] += cy * cz * wf;
                                }
                            }
                }
                free(f); free(fo); free(feq);
            }
        }
        /* fixed-order reduction over threads */
        int nv = pass == 0 ? 11 : 9;
        for (int v = 0; v < nv; ++v)
            for (int id = 0; id < N; ++id) {
                double t = 0;
                for (int th = 0; th < nth; ++th) t += acc[((size_t)th * 11 + v) * N + id];
                if (pass == 0) {
                    if (v < 5) Wn[v * N + id] = t;
                    else flux[(v - 5) * N + id] = t;
                } else if (v < 3) {
                    qn[v * N + id] = t;
                } else {
                    Pn[(v - 3) * N + id] = (s->solid[id] || !(Wn[id] > 0)) ? 0.0 : t / Wn[id];
                }
            }
        if (pass == 0) {
            for (int id = 0; id < N; ++id)
                if (!s->solid[id] && !(Wn[id] > 0)) err = 1;
            if (err) break;
        }
    }
    if (!err) {
        /* new wall densities (non-penetration, discrete normalisation) */
        double *rw = (double *)calloc((size_t)6 * N, sizeof(double));
        for (int k = 0; k < c->nz; ++k)
            for (int j = 0; j < c->ny; ++j)
                for (int i = 0; i < c->nx; ++i) {
                    int id = cell_index(c, i, j, k);
                    if (s->solid[id]) continue;
                    for (int side = 0; side < 6; ++side) {
                        int nb;
                        int t = face_type(s, i, j, k, side, &nb);
                        if (t < 0 || t >= 100 || !kind_is_wall(s, t)) continue;
                        rw[side * N + id] = flux[side * N + id] / s->gout[t][side];
                    }
                }
        /* closed domain: rescale so that the total mass stays M0 */
        if (c->closed) {
            double m = 0;
            for (int id = 0; id < N; ++id) if (!s->solid[id]) m += Wn[id] * cell_volume(s, id);
            double sc = s->M0 / m;
            for (int v = 0; v < 5 * N; ++v) Wn[v] *= sc;
            for (int v = 0; v < 3 * N; ++v) qn[v] *= sc;
            for (int v = 0; v < 6 * N; ++v) rw[v] *= sc;
        }
        /* relative change of rho, rho U, rho E (global L2 per field) */
        for (int v = 0; v < 5; ++v) {
            double dn = 0, nn = 0;
            for (int id = 0; id < N; ++id) {
                if (s->solid[id]) continue;
                double dd = Wn[v * N + id] - s->W[v * N + id];
                dn += dd * dd;
                nn += Wn[v * N + id] * Wn[v * N + id];
            }
            s->res[v] = nn > 0 ? sqrt(dn / nn) : (dn > 0 ? sqrt(dn) : 0.0);
        }
        memcpy(s->W, Wn, sizeof(double) * 5 * N);
        memcpy(s->q, qn, sizeof(double) * 3 * N);
        memcpy(s->P, Pn, sizeof(double) * 6 * N);
        memcpy(s->rho_w, rw, sizeof(double) * 6 * N);
        free(rw);
        s->iter++;
    }
    free(acc); free(Wn); free(qn); free(flux); free(specbuf); free(Pn);
    free(p.rho); free(p.T); free(p.nu); free(p.U); free(p.q); free(p.esinv); free(p.espre); free(lam);
    return err ? ORC_ERR : ORC_OK;
}

/* ---- accessors ---------------------------------------------------------- */
double orc_residual(const orc_state *s, double *per_field)
{
    double r = 0;
    for (int v = 0; v < 5; ++v) {
        if (per_field) per_field[v] = s->res[v];
        if (s->res[v] > r) r = s->res[v];
    }
    return r;
}

int orc_get_state(const orc_state *s, double *W, double *q, double *rho_w)
{
    int N = s->N;
    if (W) memcpy(W, s->W, sizeof(double) * 5 * N);
    if (q) memcpy(q, s->q, sizeof(double) * 3 * N);
    if (rho_w) memcpy(rho_w, s->rho_w, sizeof(double) * 6 * N);
    return ORC_OK;
}

int orc_set_state(orc_state *s, const double *W, const double *q,
                  const double *rho_w, double M0)
{
    int N = s->N;
    memcpy(s->W, W, sizeof(double) * 5 * N);
    memcpy(s->q, q, sizeof(double) * 3 * N);
    memcpy(s->rho_w, rho_w, sizeof(double) * 6 * N);
    s->M0 = M0;
    /* the stress restarts at the equilibrium of the given state */
    memset(s->P, 0, sizeof(double) * 6 * N);
    for (int id = 0; id < N; ++id) {
        double r, U[3], T;
        if (s->solid[id] || primitives(s->W, N, id, &r, U, &T)) continue;
        for (int k = 0; k < 3; ++k) s->P[k * N + id] = 0.5 * T;
    }
    return ORC_OK;
}

double orc_total_mass(const orc_state *s)
{
    double m = 0;
    for (int id = 0; id < s->N; ++id) if (!s->solid[id]) m += s->W[id] * cell_volume(s, id);
    return m;
}

double orc_initial_mass(const orc_state *s) { return s->M0; }

/* rho, U (3 x N), T, q (3 x N) of the current state; solid cells get 0 */
int orc_get_fields(const orc_state *s, double *rho, double *u, double *T, double *q)
{
    int N = s->N;
    for (int id = 0; id < N; ++id) {
        double r = 0, U[3] = {0, 0, 0}, t = 0;
        if (!s->solid[id]) primitives(s->W, N, id, &r, U, &t);
        if (rho) rho[id] = r;
        if (T) T[id] = t;
        if (u) for (int d = 0; d < 3; ++d) u[d * N + id] = U[d];
        if (q) for (int d = 0; d < 3; ++d) q[d * N + id] = s->solid[id] ? 0 : s->q[d * N + id];
    }
    return ORC_OK;
}

/* emission shape of kind k (0..5 domain faces, 6 solid) and its emitted flux
   normaliser for each face orientation; for test pins                         */
int orc_get_ghat(const orc_state *s, int kind, double *g, double *gout6)
{
    if (kind < 0 || kind > 6 || !s->ghat[kind]) return ORC_ERR;
    if (g) memcpy(g, s->ghat[kind], sizeof(double) * s->NV);
    if (gout6) for (int side = 0; side < 6; ++side) gout6[side] = s->gout[kind][side];
    return ORC_OK;
}

/* The f field of one discrete velocity produced by the sweep of the NEXT
   iteration from the current state (for the brute-force dense check).
   spec_mirror: z=0 planes of the mirrored velocity (its f, then its fo
   along z; the second plane is read with the second order only) or NULL.   */
int orc_sweep_one(const orc_state *s, int al, const double *spec_mirror,
                  double *f_out, double *feq_out, double *nu_out)
{
    const orc_case *c = &s->c;
    int N = s->N;
    if (al < 0 || al >= s->NV) return ORC_ERR;
    cellprm p;
    p.rho = (double *)malloc(sizeof(double) * N);
    p.T = (double *)malloc(sizeof(double) * N);
    p.nu = (double *)malloc(sizeof(double) * N);
    p.U = (double *)malloc(sizeof(double) * 3 * N);
    p.q = (double *)malloc(sizeof(double) * 3 * N);
    p.esinv = (double *)malloc(sizeof(double) * 6 * N);
    p.espre = (double *)malloc(sizeof(double) * N);
    double *lam = c->correction ? (double *)malloc(sizeof(double) * 5 * (size_t)N) : NULL;
    int err = cell_params(s, &p);
    if (!err && lam) err = cell_lambdas(s, &p, lam);
    if (!err) {
        int a3 = al % c->m[0];
        int b3 = (al / c->m[0]) % c->m[1];
        int c3 = al / (c->m[0] * c->m[1]);
        double *feq = (double *)malloc(sizeof(double) * N);
        double *fo = (double *)malloc(sizeof(double) * 3 * N);
        velocity_feq(s, &p, lam, a3, b3, c3, feq);
        sweep_velocity(s, a3, b3, c3, feq, p.nu, spec_mirror, f_out, fo);
        free(fo);
        if (feq_out) memcpy(feq_out, feq, sizeof(double) * N);
        if (nu_out) memcpy(nu_out, p.nu, sizeof(double) * N);
        free(feq);
    }
    free(p.rho); free(p.T); free(p.nu); free(p.U); free(p.q); free(p.esinv); free(p.espre); free(lam);
    return err ? ORC_ERR : ORC_OK;
}

int orc_num_threads(const orc_state *s) { return nthreads_of(s); }
