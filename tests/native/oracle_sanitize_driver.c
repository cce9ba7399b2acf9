/*
 * Runs the FP64 oracle (test infrastructure) through every option on tiny
 * cases in one translation unit built with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py builds and runs
 * it; OpenMP is off, so the loops run serially).  Exit status 0 = all calls
 * returned success and the sanitizers stayed quiet.
 */
#include "../../oracle/dvm_oracle.c"

#include <stdio.h>

static int fail(const char *what)
{
    fprintf(stderr, "oracle call failed: %s\n", what);
    return 1;
}

static orc_case cavity(int nx, int ny, int nz, int m)
{
    orc_case c;
    memset(&c, 0, sizeof c);
    c.nx = nx; c.ny = ny; c.nz = nz;
    c.lx = c.ly = c.lz = 1.0;
    c.m[0] = c.m[1] = c.m[2] = m;
    c.vmax[0] = c.vmax[1] = c.vmax[2] = 5.0;
    c.kn = 0.5; c.omega = 0.81; c.pr = 2.0 / 3.0; c.correction = 1;
    for (int f = 0; f < 6; ++f) { c.face_kind[f] = FACE_WALL; c.face_T[f] = 1.0; c.face_rho[f] = 1.0; }
    c.face_u[3][0] = 0.3;
    c.closed = 1; c.solid_T = 1.0; c.threads = 1;
    return c;
}

static int run(orc_case c, const unsigned char *solid, int order, int model, int axes, int spacing)
{
    orc_state *s = orc_create(&c, solid);
    if (!s) return fail("create");
    if (spacing) {
        double hx[16];
        double sum = 0;
        for (int i = 0; i < c.nx; ++i) { hx[i] = 1.0 + 0.1 * i; sum += hx[i]; }
        for (int i = 0; i < c.nx; ++i) hx[i] *= c.lx / sum;
        if (orc_set_spacing(s, hx, NULL, NULL)) return fail("spacing");
    }
    if (axes) {
        double xi[32], w[32];
        const int M = c.m[0];
        for (int a = 0; a < M; ++a) { xi[a] = 4.0 * (2.0 * a - (M - 1)) / (M - 1); w[a] = 8.0 / (M - 1); }
        w[0] *= 0.5; w[M - 1] *= 0.5;
        for (int a = 0; a < M; ++a) xi[a] = xi[a] * (0.6 + 0.4 * fabs(xi[a]) / 4.0);
        for (int a = 1; a < M - 1; ++a) w[a] = 0.5 * (xi[a + 1] - xi[a - 1]);
        w[0] = 0.5 * (xi[1] - xi[0]); w[M - 1] = w[0];
        if (orc_set_velocity_axis(s, 0, xi, w)) return fail("velocity axis");
    }
    if (order != 1 && orc_set_order(s, order)) return fail("order");
    if (model && orc_set_model(s, model)) return fail("model");
    const double u[3] = {0.1, 0.0, 0.0};
    if (orc_init_uniform(s, 1.0, u, 1.0)) return fail("init");
    for (int k = 0; k < 2; ++k)
        if (orc_iterate(s)) return fail("iterate");
    const int N = s->N;
    double *W = malloc(sizeof(double) * 5 * N), *q = malloc(sizeof(double) * 3 * N);
    double *rw = malloc(sizeof(double) * 6 * N), *P = malloc(sizeof(double) * 6 * N);
    double *f = malloc(sizeof(double) * N), *feq = malloc(sizeof(double) * N), *nu = malloc(sizeof(double) * N);
    double *mir = calloc((size_t)2 * c.nx * c.ny, sizeof(double));
    double r5[5];
    int bad = orc_get_state(s, W, q, rw) || orc_get_stress(s, P) || orc_set_state(s, W, q, rw, s->M0) ||
              orc_sweep_one(s, s->NV / 3, mir, f, feq, nu) || orc_iterate(s);
    orc_residual(s, r5);
    free(W); free(q); free(rw); free(P); free(f); free(feq); free(nu); free(mir);
    orc_destroy(s);
    return bad ? fail("state / sweep") : 0;
}

int main(void)
{
    int bad = 0;
    orc_case c = cavity(5, 4, 6, 6);
    bad |= run(c, NULL, 1, 0, 0, 0);
    bad |= run(c, NULL, 2, 0, 0, 0);
    bad |= run(c, NULL, 1, 1, 0, 0);
    bad |= run(c, NULL, 2, 1, 1, 0);
    bad |= run(c, NULL, 1, 0, 1, 1);
    orc_case o = cavity(4, 3, 5, 7);       /* odd node count: xi = 0 */
    bad |= run(o, NULL, 1, 0, 0, 0);
    /* half-domain body with a mirror plane and free-stream faces */
    orc_case h = cavity(6, 4, 3, 6);
    unsigned char solid[6 * 4 * 3];
    memset(solid, 0, sizeof solid);
    solid[2 + 6 * (1 + 4 * 0)] = solid[3 + 6 * (1 + 4 * 0)] = solid[2 + 6 * (2 + 4 * 0)] = 1;
    for (int f = 0; f < 6; ++f) { h.face_kind[f] = FACE_FREE; h.face_u[f][0] = 0.8; }
    h.face_kind[4] = FACE_SPECULAR;
    h.closed = 0;
    bad |= run(h, solid, 1, 0, 0, 0);
    bad |= run(h, solid, 2, 0, 0, 0);
    bad |= run(h, solid, 2, 1, 0, 0);
    if (!bad) printf("oracle sanitized run: ok\n");
    return bad;
}
