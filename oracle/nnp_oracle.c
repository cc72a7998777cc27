/*
 * FP64 CPU oracle of the sampling planner of M. G. Plessen, "Online Sampling in the Parameter
 * Space of a Neural Network for GPU-accelerated Motion Planning of Autonomous Vehicles".
 *
 * TEST INFRASTRUCTURE ONLY: it checks the HIP planner and is never on the product path. Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * The code follows the paper's steps in the paper's order and names, one function per step:
 *   Step 5 of Alg. 1 (Sect. II-E) as a plain sampler: N parameter vectors theta are drawn, each is
 *   held constant over the horizon, the closed loop
 *       features s_{t+h} (eq. (3)) -> a_{t+h} = X(s_{t+h}, theta) (eq. (4), a tanh MLP)
 *       -> control map and kinematic model (Sect. II-F, eq. (5), Table I)
 *   is simulated for h = 0..H, obstacle points are extrapolated at constant velocity
 *   (Sect. II-E items (ii)-(iv)) and tested against the vehicle rectangle with the linear
 *   inequalities of eq. (2) at every h, and the lowest-cost parameter vector is returned.
 * Readings of what the paper leaves open (cost, feature variants, sampler distribution, Philox
 * counter layout, wrap conventions) are listed in the design notes of the repository.
 */
#include "nnp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORC_PI = 3.14159265358979323846;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of a multiply-hi/lo S-box      */
/* bijection on a 128-bit counter, keyed by a 64-bit key that is advanced by a Weyl sequence    */
/* between rounds.                                                                              */
/* ------------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;      /* golden ratio                */
            k1 += 0xBB67AE85u;      /* sqrt(3) - 1                 */
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Parameter k of sample i: counter (k / 4, i, stream, inst), key (seed low, seed high), word
 * k mod 4. The top 24 bits m of that word give theta = (2m + 1 - 2^24) / 2^24, an odd multiple
 * of 2^-24 in (-1, 1): uniform on (-1, 1) and exact in float and double alike. */
double orc_theta_value(uint64_t seed, uint32_t inst, uint32_t stream, uint32_t i, uint32_t k)
{
    uint32_t ctr[4] = { k >> 2, i, stream, inst };
    uint32_t key[2] = { (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32) };
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    uint32_t m = out[k & 3u] >> 8;
    return ((double)(2.0 * (double)m + 1.0 - 16777216.0)) / 16777216.0;
}

void orc_draw_theta(uint64_t seed, uint32_t inst, uint32_t i0, uint32_t n, uint32_t n_theta,
                    double *out)
{
    for (uint32_t r = 0; r < n; ++r)
        for (uint32_t k = 0; k < n_theta; ++k)
            out[(size_t)r * n_theta + k] = orc_theta_value(seed, inst, 0u, i0 + r, k);
}

/* Table III counts weights and biases: layer l contributes n_l * n_{l-1} + n_l. */
int orc_n_theta(const orc_model *m)
{
    int n = 0;
    for (int l = 0; l < m->n_layers; ++l)
        n += m->widths[l + 1] * m->widths[l] + m->widths[l + 1];
    return n;
}

/* ------------------------------------------------------------------------------------------ */
/* Controller: a_{t+h} = X(s_{t+h}, theta), eq. (4). "Standard multilayer perceptron" (Sect. III)*/
/* with tanh units; the output is tanh as well because both controls live in [-1, 1]            */
/* (Sect. II-F control map). theta is stored layer by layer: W_l row-major [n_l][n_{l-1}], then */
/* b_l.                                                                                         */
/* ------------------------------------------------------------------------------------------ */
void orc_mlp(const orc_model *m, const double *theta, const double *s, double *a)
{
    double x[ORC_MAX_WIDTH], y[ORC_MAX_WIDTH];
    int n_in = m->widths[0];
    for (int i = 0; i < n_in; ++i) x[i] = s[i];
    const double *p = theta;
    for (int l = 0; l < m->n_layers; ++l) {
        int nin = m->widths[l], nout = m->widths[l + 1];
        const double *W = p;
        const double *b = p + (size_t)nout * nin;
        for (int o = 0; o < nout; ++o) {
            double acc = b[o];
            for (int i = 0; i < nin; ++i) acc += W[(size_t)o * nin + i] * x[i];
            y[o] = tanh(acc);
        }
        for (int o = 0; o < nout; ++o) x[o] = y[o];
        p += (size_t)nout * nin + nout;
    }
    a[0] = x[0];
    a[1] = x[1];
}

/* The same controller evaluated at binary32 precision, for the float-rounding mode 3 of
 * orc_rollout: the inputs, every partial sum of each unit's weighted sum (in index order) and
 * every activation are rounded to float. This does not reproduce any particular float
 * implementation bit for bit; it perturbs the controller by errors of the size such an
 * implementation makes. */
static double f32r(double v) { return (double)(float)v; }

static void mlp_binary32(const orc_model *m, const double *theta, const double *s, double *a)
{
    double x[ORC_MAX_WIDTH], y[ORC_MAX_WIDTH];
    int n_in = m->widths[0];
    for (int i = 0; i < n_in; ++i) x[i] = f32r(s[i]);
    const double *p = theta;
    for (int l = 0; l < m->n_layers; ++l) {
        int nin = m->widths[l], nout = m->widths[l + 1];
        const double *W = p;
        const double *b = p + (size_t)nout * nin;
        for (int o = 0; o < nout; ++o) {
            double acc = f32r(b[o]);
            for (int i = 0; i < nin; ++i) acc = f32r(acc + W[(size_t)o * nin + i] * x[i]);
            y[o] = f32r(tanh(acc));
        }
        for (int o = 0; o < nout; ++o) x[o] = y[o];
        p += (size_t)nout * nin + nout;
    }
    a[0] = x[0];
    a[1] = x[1];
}

/* Mode 4 of orc_rollout: the whole step at binary32, i.e. the oracle's own formulas below
 * (features, controller, rate limit, control map, kinematic model) evaluated in C float arithmetic
 * with the math library's float functions, so that every operation, not only the stored values,
 * carries a binary32 rounding error. Like mode 3 it reproduces no particular float implementation;
 * it gives the closed loop perturbations of the size a binary32 implementation makes. */
static float wrap_f(float a)
{
    const float pi = (float)ORC_PI, two_pi = (float)(2.0 * ORC_PI);
    if (a >= pi) a -= two_pi;
    else if (a < -pi) a += two_pi;
    return a;
}

static void step_binary32(const orc_model *m, const double *theta, const float z[4],
                          const float goal[4], float d_near, const float a_prev[2], float a[2],
                          float zn[4])
{
    /* features, eq. (3) */
    float s[ORC_MAX_WIDTH];
    const float c = cosf(z[2]), sn = sinf(z[2]);
    const float gx = goal[0] - z[0], gy = goal[1] - z[1];
    const float xi_g = c * gx + sn * gy, eta_g = -sn * gx + c * gy;
    const float dphi = wrap_f(goal[2] - z[2]);
    const float dcap = (float)m->d_cap, dn = d_near < dcap ? d_near : dcap;
    if (m->feature_set == ORC_FEAT_PAPER) {
        s[0] = xi_g / (float)m->norm_xi;
        s[1] = eta_g / (float)m->norm_eta;
        s[2] = dphi / (float)m->norm_phi;
        s[3] = (goal[3] - z[3]) / (float)m->norm_v;
        s[4] = a_prev[0];
    } else {
        s[0] = xi_g / (float)m->norm_xi;
        s[1] = eta_g / (float)m->norm_eta;
        s[2] = dphi / (float)m->norm_phi;
        s[3] = z[3] / (float)m->norm_v;
        s[4] = dn / dcap;
        s[5] = a_prev[0];
        if (m->feature_set == ORC_FEAT_EIGHT) {
            s[6] = (goal[3] - z[3]) / (float)m->norm_v;
            s[7] = a_prev[1];
        }
    }
    /* controller, eq. (4) */
    float x[ORC_MAX_WIDTH], y[ORC_MAX_WIDTH];
    for (int i = 0; i < m->widths[0]; ++i) x[i] = s[i];
    const double *p = theta;
    for (int l = 0; l < m->n_layers; ++l) {
        const int nin = m->widths[l], nout = m->widths[l + 1];
        const double *W = p, *b = p + (size_t)nout * nin;
        for (int o = 0; o < nout; ++o) {
            float acc = (float)b[o];
            for (int i = 0; i < nin; ++i) acc += (float)W[(size_t)o * nin + i] * x[i];
            y[o] = tanhf(acc);
        }
        for (int o = 0; o < nout; ++o) x[o] = y[o];
        p += (size_t)nout * nin + nout;
    }
    a[0] = x[0];
    a[1] = x[1];
    /* rate limit, control map and model, Sect. II-F */
    if (m->delta_rate_max > 0.0) {
        const float r = (float)m->delta_rate_max * (float)m->dt / (float)m->delta_max;
        if (a[0] < a_prev[0] - r) a[0] = a_prev[0] - r;
        if (a[0] > a_prev[0] + r) a[0] = a_prev[0] + r;
    }
    const float delta = (float)m->delta_max * a[0];
    const float u = (float)m->u_min + (a[1] + 1.0f) / 2.0f * ((float)m->u_max - (float)m->u_min);
    const float L = (float)m->lf + (float)m->lr, dt = (float)m->dt;
    const float beta = atanf((float)m->lr * tanf(delta) / L);
    const float xd = z[3] * cosf(z[2] + beta) / cosf(beta);
    const float yd = z[3] * sinf(z[2] + beta) / cosf(beta);
    const float phid = z[3] * tanf(delta) / L;
    zn[0] = z[0] + dt * xd;
    zn[1] = z[1] + dt * yd;
    zn[2] = wrap_f(z[2] + dt * phid);
    float vn = z[3] + dt * u;
    if (vn < (float)m->v_min) vn = (float)m->v_min;
    if (vn > (float)m->v_max) vn = (float)m->v_max;
    zn[3] = vn;
}

/* Heading angles are kept in [-pi, pi). Every difference wrapped here is within one turn of
 * that range, so a single correction suffices. */
double orc_wrap_angle(double a)
{
    if (a >= ORC_PI) a -= 2.0 * ORC_PI;
    else if (a < -ORC_PI) a += 2.0 * ORC_PI;
    return a;
}

/* Feature vector s_{t+h}, eq. (3): deviations from the goal setpoint expressed in the
 * vehicle-aligned (xi, eta) frame of step h, scaled by the Delta constants of Table II, plus the
 * previous steering output. The six- and eight-input variants add speed and the distance to the
 * nearest extrapolated obstacle point, capped at d_cap. */
void orc_features(const orc_model *m, const double z[4], const double goal[4], double d_near,
                  const double a_prev[2], double *s)
{
    double c = cos(z[2]), sn = sin(z[2]);
    double gx = goal[0] - z[0], gy = goal[1] - z[1];
    double xi_g = c * gx + sn * gy;
    double eta_g = -sn * gx + c * gy;
    double dphi = orc_wrap_angle(goal[2] - z[2]);
    double dn = d_near < m->d_cap ? d_near : m->d_cap;
    switch (m->feature_set) {
    case ORC_FEAT_PAPER:
        s[0] = xi_g / m->norm_xi;
        s[1] = eta_g / m->norm_eta;
        s[2] = dphi / m->norm_phi;
        s[3] = (goal[3] - z[3]) / m->norm_v;
        s[4] = a_prev[0];
        break;
    case ORC_FEAT_SIX:
    case ORC_FEAT_EIGHT:
        s[0] = xi_g / m->norm_xi;
        s[1] = eta_g / m->norm_eta;
        s[2] = dphi / m->norm_phi;
        s[3] = z[3] / m->norm_v;
        s[4] = dn / m->d_cap;
        s[5] = a_prev[0];
        if (m->feature_set == ORC_FEAT_EIGHT) {
            s[6] = (goal[3] - z[3]) / m->norm_v;
            s[7] = a_prev[1];
        }
        break;
    default:
        break;
    }
}

/* Steering-rate limit of Table I: the steering output may move by at most
 * delta_rate_max * T_s / delta_max per step in normalised units. Off when delta_rate_max = 0. */
void orc_limit_rate(const orc_model *m, const double a_raw[2], const double a_prev[2],
                    double a[2])
{
    a[0] = a_raw[0];
    a[1] = a_raw[1];
    if (m->delta_rate_max > 0.0) {
        double r = m->delta_rate_max * m->dt / m->delta_max;
        double lo = a_prev[0] - r, hi = a_prev[0] + r;
        if (a[0] < lo) a[0] = lo;
        if (a[0] > hi) a[0] = hi;
    }
}

/* Control map of Sect. II-F: delta = delta_max a[0], u = u_min + (a[1] + 1)/2 (u_max - u_min). */
void orc_control_map(const orc_model *m, const double a[2], double *delta, double *u)
{
    *delta = m->delta_max * a[0];
    *u = m->u_min + (a[1] + 1.0) / 2.0 * (m->u_max - m->u_min);
}

/* Kinematic model of Sect. II-F, eq. (5), one explicit Euler step of length T_s:
 *   x' = v cos(phi + beta)/cos(beta),  y' = v sin(phi + beta)/cos(beta),
 *   phi' = v tan(delta)/(l_f + l_r),   v' = u,   beta = atan(l_r tan(delta)/(l_f + l_r)).
 * The heading is wrapped to [-pi, pi) and the speed clamped to [v_min, v_max]. */
void orc_vehicle_step(const orc_model *m, const double z[4], double delta, double u,
                      double z_next[4])
{
    double L = m->lf + m->lr;
    double beta = atan(m->lr * tan(delta) / L);
    double x = z[0], y = z[1], phi = z[2], v = z[3];
    double xd = v * cos(phi + beta) / cos(beta);
    double yd = v * sin(phi + beta) / cos(beta);
    double phid = v * tan(delta) / L;
    z_next[0] = x + m->dt * xd;
    z_next[1] = y + m->dt * yd;
    z_next[2] = orc_wrap_angle(phi + m->dt * phid);
    double vn = v + m->dt * u;
    if (vn < m->v_min) vn = m->v_min;
    if (vn > m->v_max) vn = m->v_max;
    z_next[3] = vn;
}

/* Constant-velocity extrapolation, Sect. II-E items (ii)-(iv): m_{t+h} = m_t + (h T_s) v. */
void orc_extrapolate(const double point[4], double t, double out[2])
{
    out[0] = point[0] + t * point[2];
    out[1] = point[1] + t * point[3];
}

/* Collision test of eq. (2) for the rectangle: A(phi)(p - [x, y]) < b(phi) row by row, with the
 * four outward face normals of the rectangle as the rows of A and the face offsets as b. Strict:
 * a point on a face does not collide. */
int orc_point_inside(const orc_model *m, const double pose[3], const double p[2])
{
    double c = cos(pose[2]), s = sin(pose[2]);
    double d0 = p[0] - pose[0], d1 = p[1] - pose[1];
    double A[4][2] = { { c, s }, { -c, -s }, { -s, c }, { s, -c } };
    double b[4] = { m->front, m->rear, m->half_width, m->half_width };
    for (int r = 0; r < 4; ++r)
        if (!(A[r][0] * d0 + A[r][1] * d1 < b[r])) return 0;
    return 1;
}

static void body_frame(const double pose[3], const double p[2], double *xi, double *eta)
{
    double c = cos(pose[2]), s = sin(pose[2]);
    double d0 = p[0] - pose[0], d1 = p[1] - pose[1];
    *xi = c * d0 + s * d1;
    *eta = -s * d0 + c * d1;
}

/* Signed distance of the point to the nearest face in the max sense: negative inside, zero on
 * the boundary. A perturbation of the point smaller than |value| cannot change the test. */
double orc_face_distance(const orc_model *m, const double pose[3], const double p[2])
{
    double xi, eta;
    body_frame(pose, p, &xi, &eta);
    double oc = 0.5 * (m->front - m->rear), hl = 0.5 * (m->front + m->rear);
    double a = fabs(xi - oc) - hl, b = fabs(eta) - m->half_width;
    return a > b ? a : b;
}

/* Normalised penetration margin: below 1 exactly when the point is inside. */
double orc_margin(const orc_model *m, const double pose[3], const double p[2])
{
    double xi, eta;
    body_frame(pose, p, &xi, &eta);
    double oc = 0.5 * (m->front - m->rear), hl = 0.5 * (m->front + m->rear);
    double a = fabs(xi - oc) / hl, b = fabs(eta) / m->half_width;
    return a > b ? a : b;
}

static int goal_reached(const orc_model *m, const double z[4], const double goal[4])
{
    double c = cos(z[2]), sn = sin(z[2]);
    double gx = goal[0] - z[0], gy = goal[1] - z[1];
    double xi_g = c * gx + sn * gy, eta_g = -sn * gx + c * gy;
    double dphi = orc_wrap_angle(goal[2] - z[2]);
    return fabs(xi_g) <= m->eps_xi && fabs(eta_g) <= m->eps_eta && fabs(dphi) <= m->eps_phi &&
           fabs(goal[3] - z[3]) <= m->eps_v;
}

/* ------------------------------------------------------------------------------------------ */
/* One sample: the parameters are held constant over the horizon (Sect. IV, first comment), the */
/* closed loop runs for h = 0..H, collision is checked at every h including h = 0 (eq. (2)), and */
/* the cost is the terminal distance to the goal position plus effort_weight * T_s * sum |a|^2, */
/* +inf on any collision. Two optional terms (weights 0 by default) add the terminal heading and */
/* speed errors to the goal setpoint, for missions whose setpoints prescribe them (Sect. III).   */
/* fp32_state = 1 rounds the state to float after every step; 2 also rounds the features and the */
/* applied controls; 3 in addition evaluates the controller at binary32 precision (mlp_binary32); */
/* 4 computes the nearest distance and the whole step at binary32 (step_binary32), the effort and */
/* the terminal distance in float as well (collision tests stay binary64 at the float states).   */
/* The tests use the gap to the plain run to recognise samples whose outcome is ill-conditioned  */
/* at float precision.                                                                           */
/* ------------------------------------------------------------------------------------------ */
void orc_rollout(const orc_model *m, const orc_scene *sc, const double *theta, int fp32_state,
                 orc_record *rec)
{
    double z[4], ap[2];
    for (int q = 0; q < 4; ++q) z[q] = sc->z0[q];
    ap[0] = sc->a_prev[0];
    ap[1] = sc->a_prev[1];
    double effort = 0.0;
    float effort_f = 0.0f;
    int collided = 0, first = -1;
    double min_margin = INFINITY, min_abs_face = INFINITY;
    for (int h = 0; h <= sc->T; ++h) {
        double t = (double)h * m->dt;
        double pose[3] = { z[0], z[1], z[2] };
        double d2min = INFINITY;
        float d2min_f = INFINITY;
        int hit = 0;
        for (int j = 0; j < sc->P; ++j) {
            double p[2];
            orc_extrapolate(sc->points + 4 * (size_t)j, t, p);
            if (fp32_state == 4) {
                const double *q = sc->points + 4 * (size_t)j;
                const float tf = (float)h * (float)m->dt;
                const float dxf = ((float)q[0] + tf * (float)q[2]) - (float)z[0];
                const float dyf = ((float)q[1] + tf * (float)q[3]) - (float)z[1];
                const float d2f = dxf * dxf + dyf * dyf;
                if (d2f < d2min_f) d2min_f = d2f;
            }
            if (orc_point_inside(m, pose, p)) hit = 1;
            double mg = orc_margin(m, pose, p);
            if (mg < min_margin) min_margin = mg;
            if (!collided) {
                double fd = fabs(orc_face_distance(m, pose, p));
                if (fd < min_abs_face) min_abs_face = fd;
            }
            double dx = p[0] - z[0], dy = p[1] - z[1];
            double d2 = dx * dx + dy * dy;
            if (d2 < d2min) d2min = d2;
        }
        double d_near = sqrt(d2min);
        if (rec->traj)
            for (int q = 0; q < 4; ++q) rec->traj[4 * (size_t)h + q] = z[q];
        if (rec->d_near) rec->d_near[h] = d_near;
        if (rec->step_flags) rec->step_flags[h] = hit;
        if (hit && !collided) {
            collided = 1;
            first = h;
        }
        if (h == sc->T) break;

        if (fp32_state == 4) {
            float zf[4], gf[4], apf[2] = { (float)ap[0], (float)ap[1] }, af[2], znf[4];
            for (int q = 0; q < 4; ++q) {
                zf[q] = (float)z[q];
                gf[q] = (float)sc->goal[q];
            }
            step_binary32(m, theta, zf, gf, sqrtf(d2min_f), apf, af, znf);
            effort_f += af[0] * af[0] + af[1] * af[1];
            if (rec->controls) {
                rec->controls[2 * (size_t)h] = af[0];
                rec->controls[2 * (size_t)h + 1] = af[1];
            }
            for (int q = 0; q < 4; ++q) z[q] = znf[q];
            ap[0] = af[0];
            ap[1] = af[1];
            continue;
        }
        double s[ORC_MAX_WIDTH], a_raw[2], a[2], delta, u, zn[4];
        orc_features(m, z, sc->goal, d_near, ap, s);
        if (fp32_state >= 2)
            for (int i = 0; i < m->widths[0]; ++i) s[i] = (double)(float)s[i];
        if (fp32_state == 3) mlp_binary32(m, theta, s, a_raw);
        else orc_mlp(m, theta, s, a_raw);
        orc_limit_rate(m, a_raw, ap, a);
        if (fp32_state >= 2) {
            a[0] = (double)(float)a[0];
            a[1] = (double)(float)a[1];
        }
        orc_control_map(m, a, &delta, &u);
        orc_vehicle_step(m, z, delta, u, zn);
        effort += a[0] * a[0] + a[1] * a[1];
        if (rec->controls) {
            rec->controls[2 * (size_t)h] = a[0];
            rec->controls[2 * (size_t)h + 1] = a[1];
        }
        for (int q = 0; q < 4; ++q) z[q] = fp32_state ? (double)(float)zn[q] : zn[q];
        ap[0] = a[0];
        ap[1] = a[1];
    }
    double gx = z[0] - sc->goal[0], gy = z[1] - sc->goal[1];
    double cost = sqrt(gx * gx + gy * gy) + m->effort_weight * m->dt * effort;
    if (fp32_state == 4) {
        const float gxf = (float)z[0] - (float)sc->goal[0], gyf = (float)z[1] - (float)sc->goal[1];
        cost = sqrtf(gxf * gxf + gyf * gyf) +
               (float)m->effort_weight * (float)m->dt * effort_f;
    }
    cost += m->goal_heading_weight * fabs(orc_wrap_angle(sc->goal[2] - z[2]));
    cost += m->goal_speed_weight * fabs(sc->goal[3] - z[3]);
    if (collided || isnan(cost)) cost = INFINITY;
    rec->cost = cost;
    rec->collided = collided;
    rec->first_collision = first;
    rec->min_margin = min_margin;
    rec->min_abs_face = min_abs_face;
    rec->goal_reached = goal_reached(m, z, sc->goal);
}

/* Rollouts of the listed samples with their Philox parameters (OpenMP over the list). */
void orc_rollout_samples(const orc_model *m, const orc_scene *sc, uint64_t seed, uint32_t inst,
                         const uint32_t *idx, int count, int fp32_state,
                         double *traj, double *controls, double *d_near, double *cost,
                         int *collided, int *first_collision, double *min_margin,
                         double *min_abs_face)
{
    int nt = orc_n_theta(m);
    int T = sc->T;
#pragma omp parallel for schedule(dynamic, 1)
    for (int r = 0; r < count; ++r) {
        double *theta = (double *)malloc(sizeof(double) * (size_t)nt);
        orc_draw_theta(seed, inst, idx[r], 1u, (uint32_t)nt, theta);
        orc_record rec;
        memset(&rec, 0, sizeof rec);
        rec.traj = traj ? traj + (size_t)r * (T + 1) * 4 : NULL;
        rec.controls = controls ? controls + (size_t)r * T * 2 : NULL;
        rec.d_near = d_near ? d_near + (size_t)r * (T + 1) : NULL;
        orc_rollout(m, sc, theta, fp32_state, &rec);
        if (cost) cost[r] = rec.cost;
        if (collided) collided[r] = rec.collided;
        if (first_collision) first_collision[r] = rec.first_collision;
        if (min_margin) min_margin[r] = rec.min_margin;
        if (min_abs_face) min_abs_face[r] = rec.min_abs_face;
        free(theta);
    }
}

/* Lowest cost wins, the lowest index wins ties. Returns 1 (infeasible) when no cost is finite;
 * the winner is then index 0. */
int orc_argmin(const double *cost, int n, int *best)
{
    int b = 0;
    double bc = INFINITY;
    for (int i = 0; i < n; ++i)
        if (cost[i] < bc) {
            bc = cost[i];
            b = i;
        }
    *best = b;
    return isinf(bc) ? 1 : 0;
}

/* The whole plan: every sample, then the argmin, then the winner's outputs. */
int orc_plan(const orc_model *m, const orc_scene *sc, int N, uint64_t seed, uint32_t inst,
             double *cost, int *best, double *theta_best, double *traj_best,
             double *controls_best, int *goal_reached_out)
{
    int nt = orc_n_theta(m);
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < N; ++i) {
        double *theta = (double *)malloc(sizeof(double) * (size_t)nt);
        orc_draw_theta(seed, inst, (uint32_t)i, 1u, (uint32_t)nt, theta);
        orc_record rec;
        memset(&rec, 0, sizeof rec);
        orc_rollout(m, sc, theta, 0, &rec);
        cost[i] = rec.cost;
        free(theta);
    }
    int status = orc_argmin(cost, N, best);
    double *theta = (double *)malloc(sizeof(double) * (size_t)nt);
    orc_draw_theta(seed, inst, (uint32_t)*best, 1u, (uint32_t)nt, theta);
    orc_record rec;
    memset(&rec, 0, sizeof rec);
    rec.traj = traj_best;
    rec.controls = controls_best;
    orc_rollout(m, sc, theta, 0, &rec);
    if (theta_best) memcpy(theta_best, theta, sizeof(double) * (size_t)nt);
    if (goal_reached_out) *goal_reached_out = rec.goal_reached;
    free(theta);
    return status;
}

/* Eq. (2) re-evaluated at given poses (x, y, phi) and steps h, in double precision. flag[i] is
 * 1 when some point is inside by more than eps, else 2 when some point lies within eps of a
 * face (undecidable at that precision), else 0. */
void orc_flags_at_poses(const orc_model *m, const double *points, int P, double dt,
                        const double *poses, const int *steps, int M, double eps, int *flag)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < M; ++i) {
        double t = (double)steps[i] * dt;
        int f = 0;
        for (int j = 0; j < P; ++j) {
            double p[2];
            orc_extrapolate(points + 4 * (size_t)j, t, p);
            double fd = orc_face_distance(m, poses + 3 * (size_t)i, p);
            if (fd < -eps) {
                f = 1;
                break;
            }
            if (fabs(fd) <= eps) f = 2;
        }
        flag[i] = f;
    }
}

/* One closed-loop step evaluated at given states: for each (z_h, a_{h-1}, h) the nearest
 * extrapolated obstacle distance, the features, the controller, the rate limit and the model
 * step, exactly as inside orc_rollout. Used to check a float implementation step by step at its
 * own states, apart from the drift its rounding builds up over a whole horizon. */
void orc_step_at_states(const orc_model *m, const orc_scene *sc, const double *theta,
                        const double *states, const double *a_prev, const int *steps, int M,
                        double *a_out, double *z_next, double *d_near)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < M; ++i) {
        const double *z = states + 4 * (size_t)i;
        const double *ap = a_prev + 2 * (size_t)i;
        double t = (double)steps[i] * m->dt;
        double d2min = INFINITY;
        for (int j = 0; j < sc->P; ++j) {
            double p[2];
            orc_extrapolate(sc->points + 4 * (size_t)j, t, p);
            double dx = p[0] - z[0], dy = p[1] - z[1];
            double d2 = dx * dx + dy * dy;
            if (d2 < d2min) d2min = d2;
        }
        double dn = sqrt(d2min);
        double s[ORC_MAX_WIDTH], a_raw[2], a[2], delta, u;
        orc_features(m, z, sc->goal, dn, ap, s);
        orc_mlp(m, theta, s, a_raw);
        orc_limit_rate(m, a_raw, ap, a);
        orc_control_map(m, a, &delta, &u);
        orc_vehicle_step(m, z, delta, u, z_next + 4 * (size_t)i);
        a_out[2 * (size_t)i] = a[0];
        a_out[2 * (size_t)i + 1] = a[1];
        if (d_near) d_near[i] = dn;
    }
}
