/*
 * Host-side memory and undefined-behaviour check of the FP64 oracle.
 *
 * TEST INFRASTRUCTURE ONLY. Built together with nnp_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (see oracle.build_sanitized) and run by the CPU test suite: every
 * exported entry point is called on small problems of each network shape and feature set (the
 * C0 6-16-2 network, the 8-32-32-2 network, the paper's 5-10-10-2 with the steering-rate limit),
 * with no obstacle points, one point, moving points and a point inside the start footprint, and
 * every rounding mode of the rollout. The sanitizers abort on the first invalid access or
 * undefined operation; the few consistency checks below return a non-zero status instead.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "nnp_oracle.h"

#define PI_D 3.14159265358979323846

static int failures = 0;

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);        \
            ++failures;                                                               \
        }                                                                             \
    } while (0)

/* A small linear congruential generator for the scene layout (not the method's arithmetic). */
static uint64_t lcg_state = 12345u;
static double uniform(double lo, double hi)
{
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (hi - lo) * (double)(lcg_state >> 11) / 9007199254740992.0;
}

static orc_model model_of(int which)
{
    orc_model m;
    memset(&m, 0, sizeof m);
    m.dt = 0.1;
    m.norm_xi = 30.0;
    m.norm_eta = 3.5;
    m.norm_phi = 2.0 * PI_D;
    m.norm_v = 120.0 / 3.6;
    m.d_cap = 20.0;
    m.effort_weight = 0.1;
    m.eps_xi = 1.0;
    m.eps_eta = 0.25;
    m.eps_phi = 10.0 * PI_D / 180.0;
    m.eps_v = 5.0 / 3.6;
    if (which == 2) {                       /* paper preset, NN-[5,10,10,2] */
        m.lf = 1.1;
        m.lr = 1.4;
        m.front = 1.8;
        m.rear = 2.0;
        m.half_width = 1.0;
        m.delta_max = 40.0 * PI_D / 180.0;
        m.delta_rate_max = 20.0 * PI_D / 180.0;
        m.u_min = -4.0;
        m.u_max = 2.0;
        m.v_min = -INFINITY;
        m.v_max = INFINITY;
        m.n_layers = 3;
        m.widths[0] = 5;
        m.widths[1] = 10;
        m.widths[2] = 10;
        m.widths[3] = 2;
        m.feature_set = ORC_FEAT_PAPER;
        m.goal_heading_weight = 2.0;
        m.goal_speed_weight = 0.5;
        return m;
    }
    m.lf = 1.35;
    m.lr = 1.35;
    m.front = 2.25;
    m.rear = 2.25;
    m.half_width = 0.9;
    m.delta_max = 0.6;
    m.u_min = -3.0;
    m.u_max = 3.0;
    m.v_min = -3.0;
    m.v_max = 15.0;
    if (which == 0) {                       /* 6-16-2 */
        m.n_layers = 2;
        m.widths[0] = 6;
        m.widths[1] = 16;
        m.widths[2] = 2;
        m.feature_set = ORC_FEAT_SIX;
    } else {                                /* 8-32-32-2 */
        m.n_layers = 3;
        m.widths[0] = 8;
        m.widths[1] = 32;
        m.widths[2] = 32;
        m.widths[3] = 2;
        m.feature_set = ORC_FEAT_EIGHT;
    }
    return m;
}

static void run_case(const orc_model *m, int P, int moving, int blocked, int T, int N)
{
    double *pts = (double *)malloc(sizeof(double) * 4 * (size_t)(P > 0 ? P : 1));
    for (int j = 0; j < P; ++j) {
        pts[4 * j] = uniform(-15.0, 15.0);
        pts[4 * j + 1] = uniform(-15.0, 15.0);
        pts[4 * j + 2] = moving ? uniform(-5.0, 5.0) : 0.0;
        pts[4 * j + 3] = moving ? uniform(-5.0, 5.0) : 0.0;
    }
    if (blocked && P > 0) {
        pts[0] = 0.3;
        pts[1] = 0.1;
        pts[2] = pts[3] = 0.0;
    }
    orc_scene sc;
    memset(&sc, 0, sizeof sc);
    sc.z0[2] = 0.3;
    sc.z0[3] = 2.0;
    sc.goal[0] = 12.0;
    sc.goal[1] = -4.0;
    sc.goal[2] = 1.0;
    sc.a_prev[1] = -1.0 - 2.0 * m->u_min / (m->u_max - m->u_min);
    sc.points = pts;
    sc.P = P;
    sc.T = T;

    const int nt = orc_n_theta(m);
    double *cost = (double *)malloc(sizeof(double) * (size_t)N);
    double *theta = (double *)malloc(sizeof(double) * (size_t)nt);
    double *traj = (double *)malloc(sizeof(double) * 4 * (size_t)(T + 1));
    double *ctrl = (double *)malloc(sizeof(double) * 2 * (size_t)T);
    int best = -1, reached = -1;
    int status = orc_plan(m, &sc, N, 7u, 3u, cost, &best, theta, traj, ctrl, &reached);
    int b2 = -1;
    CHECK(orc_argmin(cost, N, &b2) == status && b2 == best);
    CHECK(best >= 0 && best < N);
    if (blocked && P > 0) CHECK(status == 1 && best == 0);

    /* per-sample rollouts in every rounding mode, with every output array */
    uint32_t idx[5] = {0u, 1u, (uint32_t)best, (uint32_t)(N - 1), (uint32_t)(N / 2)};
    const int M = 5;
    double *tr = (double *)malloc(sizeof(double) * M * 4 * (size_t)(T + 1));
    double *co = (double *)malloc(sizeof(double) * M * 2 * (size_t)T);
    double *dn = (double *)malloc(sizeof(double) * M * (size_t)(T + 1));
    double c[5], mm[5], mf[5];
    int col[5], first[5];
    for (int mode = 0; mode <= 4; ++mode) {
        orc_rollout_samples(m, &sc, 7u, 3u, idx, M, mode, tr, co, dn, c, col, first, mm, mf);
        if (mode == 0) CHECK(c[2] == cost[best] || (isinf(c[2]) && isinf(cost[best])));
    }
    orc_rollout_samples(m, &sc, 7u, 3u, idx, M, 0, NULL, NULL, NULL, c, NULL, NULL, NULL, NULL);

    /* the step evaluated at the rollout's own states reproduces the rollout */
    orc_rollout_samples(m, &sc, 7u, 3u, idx + 2, 1, 0, tr, co, dn, c, col, first, mm, mf);
    double *ap = (double *)malloc(sizeof(double) * 2 * (size_t)T);
    int *steps = (int *)malloc(sizeof(int) * (size_t)T);
    double *aout = (double *)malloc(sizeof(double) * 2 * (size_t)T);
    double *zn = (double *)malloc(sizeof(double) * 4 * (size_t)T);
    double *dd = (double *)malloc(sizeof(double) * (size_t)T);
    for (int h = 0; h < T; ++h) {
        steps[h] = h;
        ap[2 * h] = h ? co[2 * (h - 1)] : sc.a_prev[0];
        ap[2 * h + 1] = h ? co[2 * (h - 1) + 1] : sc.a_prev[1];
    }
    orc_step_at_states(m, &sc, theta, tr, ap, steps, T, aout, zn, dd);
    for (int h = 0; h < T; ++h) {
        CHECK(aout[2 * h] == co[2 * h] && aout[2 * h + 1] == co[2 * h + 1]);
        for (int k = 0; k < 4; ++k) CHECK(zn[4 * h + k] == tr[4 * (h + 1) + k]);
    }

    /* flags at the rollout's poses */
    double *poses = (double *)malloc(sizeof(double) * 3 * (size_t)(T + 1));
    int *psteps = (int *)malloc(sizeof(int) * (size_t)(T + 1));
    int *flags = (int *)malloc(sizeof(int) * (size_t)(T + 1));
    for (int h = 0; h <= T; ++h) {
        poses[3 * h] = tr[4 * h];
        poses[3 * h + 1] = tr[4 * h + 1];
        poses[3 * h + 2] = tr[4 * h + 2];
        psteps[h] = h;
    }
    orc_flags_at_poses(m, pts, P, m->dt, poses, psteps, T + 1, 1e-5, flags);
    if (first[0] >= 0) CHECK(flags[first[0]] != 0);

    /* the single-point primitives */
    double pose[3] = {0.5, -0.25, 0.7}, p[2] = {1.0, 0.5}, q[2], s[ORC_MAX_WIDTH], a[2], lim[2];
    double zz[4] = {1.0, 2.0, 3.1, -2.0}, znext[4], delta, u;
    (void)orc_point_inside(m, pose, p);
    (void)orc_face_distance(m, pose, p);
    (void)orc_margin(m, pose, p);
    orc_extrapolate(pts, 0.7, q);
    orc_features(m, zz, sc.goal, 3.0, sc.a_prev, s);
    orc_mlp(m, theta, s, a);
    orc_limit_rate(m, a, sc.a_prev, lim);
    orc_control_map(m, lim, &delta, &u);
    orc_vehicle_step(m, zz, delta, u, znext);
    CHECK(fabs(orc_wrap_angle(3.0 * PI_D)) <= PI_D + 1e-12);

    free(pts); free(cost); free(theta); free(traj); free(ctrl); free(tr); free(co); free(dn);
    free(ap); free(steps); free(aout); free(zn); free(dd); free(poses); free(psteps); free(flags);
}

int main(void)
{
    uint32_t ctr[4] = {0u, 0u, 0u, 0u}, key[2] = {0u, 0u}, out[4];
    orc_philox4x32_10(ctr, key, out);
    double th[3 * 146];
    orc_draw_theta(0x1234abcdull, 2u, 100u, 3u, 146u, th);
    for (int k = 0; k < 3 * 146; ++k) CHECK(th[k] > -1.0 && th[k] < 1.0 && th[k] != 0.0);
    CHECK(th[146 + 5] == orc_theta_value(0x1234abcdull, 2u, 0u, 101u, 5u));
    CHECK(orc_num_threads() >= 1);

    for (int which = 0; which < 3; ++which) {
        orc_model m = model_of(which);
        run_case(&m, 0, 0, 0, 6, 9);
        run_case(&m, 1, 0, 0, 5, 7);
        run_case(&m, 37, 1, 0, 8, 12);
        run_case(&m, 20, 0, 1, 4, 5);
    }
    if (failures) {
        fprintf(stderr, "%d consistency checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
