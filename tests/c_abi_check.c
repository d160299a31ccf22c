/* Plain C11 client of the library's C ABI (no GPU needed): the header must
 * compile as C, every host-side call must work from C, and argument errors
 * must come back as status codes with a message.  Prints "ok" and exits 0
 * on success. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "dsn.h"

#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            printf("FAILED line %d: %s (%s)\n", __LINE__, #cond, dsn_last_error()); \
            return 1;                                                    \
        }                                                                \
    } while (0)

int main(void)
{
    /* S4 quadrature: 24 directions, unit vectors, weights summing to 4 pi */
    double om[24 * 3], w[24];
    CHECK(dsn_quadrature(4, om, w) == DSN_OK);
    double sw = 0.0;
    for (int n = 0; n < 24; ++n) {
        sw += w[n];
        CHECK(fabs(om[3 * n] * om[3 * n] + om[3 * n + 1] * om[3 * n + 1] + om[3 * n + 2] * om[3 * n + 2] - 1.0) <
              1e-14);
    }
    CHECK(fabs(sw - 4.0 * 3.14159265358979323846) < 1e-13);
    CHECK(dsn_quadrature(5, om, w) != DSN_OK && strlen(dsn_last_error()) > 0);

    /* a 3 x 2 x 2 one-material problem */
    uint8_t mat[12];
    memset(mat, 0, sizeof(mat));
    double st[2] = {0.5, 0.7}, ss[2 * 2 * 2];
    memset(ss, 0, sizeof(ss));
    ss[0 * 4 + 0 * 2 + 0] = 0.2; /* l = 0, g = 0 <- 0 */
    ss[0 * 4 + 1 * 2 + 0] = 0.1; /* l = 0, g = 1 <- 0 */
    ss[0 * 4 + 1 * 2 + 1] = 0.3; /* l = 0, g = 1 <- 1 */
    ss[1 * 4 + 0 * 2 + 0] = 0.05;
    dsn_problem_desc d;
    memset(&d, 0, sizeof(d));
    d.nx = 3; d.ny = 2; d.nz = 2;
    d.dx = d.dy = d.dz = 1.0;
    d.material = mat;
    d.n_materials = 1;
    d.n_groups = 2;
    d.sigma_t = st;
    d.legendre_order = 1;
    d.sigma_s = ss;
    d.sn_order = 4;
    d.fixup = 1;
    d.precision = DSN_FP32;
    dsn_problem *p = NULL;
    CHECK(dsn_create(&d, &p) == DSN_OK && p != NULL);
    CHECK(dsn_sweep_tuning(p, NULL, NULL, NULL, NULL, NULL, 0) == 0);

    /* upscatter is rejected */
    dsn_problem *q = NULL;
    ss[0 * 4 + 0 * 2 + 1] = 0.1; /* l = 0, g = 0 <- 1 */
    CHECK(dsn_create(&d, &q) == DSN_ERR_INVALID_ARG && q == NULL);
    ss[0 * 4 + 0 * 2 + 1] = 0.0;

    /* solve-argument errors are found before any device work */
    double spec[2] = {1.0, 0.0};
    dsn_source s;
    memset(&s, 0, sizeof(s));
    s.position[0] = -2.0; s.position[1] = 1.1; s.position[2] = 0.9;
    s.axis[0] = 1.0;
    s.half_angle = 0.5;
    s.spectrum = spec;
    dsn_solve_opts o;
    memset(&o, 0, sizeof(o));
    o.tol = -1.0;
    o.max_iters = 10;
    dsn_solve_info info;
    memset(&info, 0, sizeof(info));
    double fake;
    CHECK(dsn_solve(p, &s, 1, &o, &fake, NULL, &info) == DSN_ERR_INVALID_ARG);
    o.tol = 1e-6;
    o.autotune = 2;
    CHECK(dsn_solve(p, &s, 1, &o, &fake, NULL, &info) == DSN_ERR_INVALID_ARG);
    o.autotune = 0;
    o.stop_rule = 2;
    CHECK(dsn_solve(p, &s, 1, &o, &fake, NULL, &info) == DSN_ERR_INVALID_ARG);
    o.stop_rule = 1;
    o.batch_mode = 2;
    CHECK(dsn_solve(p, &s, 1, &o, &fake, NULL, &info) == DSN_ERR_INVALID_ARG);
    {
        dsn_problem *pp[1] = {p};
        const dsn_source *sp[1] = {&s};
        int32_t ns[1] = {1};
        double *outs[1] = {&fake};
        CHECK(dsn_solve_batch(pp, 1, sp, ns, &o, outs, &info) == DSN_ERR_INVALID_ARG);
    }
    o.batch_mode = 0;
    s.half_angle = 0.3;
    s.fan_half_thickness = 0.1; /* fan with a normal parallel to the axis */
    s.fan_normal[0] = 1.0;
    CHECK(dsn_solve(p, &s, 1, &o, &fake, NULL, &info) == DSN_ERR_INVALID_ARG);
    double k[2] = {1.0, NAN};
    CHECK(dsn_dose(p, &fake, 1, k, &fake, NULL) == DSN_ERR_INVALID_ARG);
    CHECK(dsn_workspace_bytes(p) > 0); /* the estimate for a one-source solve */
    CHECK(dsn_set_sweep_shape(NULL, 1, 64, 0, 0) == DSN_ERR_INVALID_ARG);
    CHECK(dsn_set_sweep_shape(p, 7, 64, 0, 0) == DSN_ERR_INVALID_ARG); /* not a built choice */
    CHECK(dsn_set_sweep_shape(p, 1, 0, 0, 0) == DSN_ERR_INVALID_ARG);
    CHECK(dsn_set_sweep_shape(p, 1, 64, -1, 0) == DSN_ERR_INVALID_ARG);
    CHECK(dsn_set_sweep_shape(p, 1, 64, 0, 3) == DSN_ERR_INVALID_ARG); /* no relay of 3 roles */
    CHECK(dsn_set_sweep_shape(p, 1, 64, 8, 2) == DSN_ERR_INVALID_ARG); /* relays use the global queue */
    dsn_destroy(p);
    printf("ok\n");
    return 0;
}
