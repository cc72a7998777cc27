/*
 * FP64 CPU oracle of the sampling planner of M. G. Plessen, "Online Sampling in the Parameter
 * Space of a Neural Network for GPU-accelerated Motion Planning of Autonomous Vehicles".
 *
 * TEST INFRASTRUCTURE ONLY. This library exists to check the HIP planner; it is plain, slow and
 * written to be read against the paper. Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it. It shares no source with the GPU library.
 *
 * Everything is double precision. Inputs that the GPU receives as float are handed to the oracle
 * as the same float values widened to double, so both sides start from identical numbers.
 */
#ifndef NNP_ORACLE_H
#define NNP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_LAYERS 3
#define ORC_MAX_WIDTH 64

/* Feature vectors (Sect. II-E, eq. (3), and the configuration readings):
 * ORC_FEAT_PAPER  5 inputs  [xi_g/dxi, eta_g/deta, wrap(phi_g-phi)/dphi, (v_g-v)/dv, a_prev[0]]
 * ORC_FEAT_SIX    6 inputs  [xi_g/dxi, eta_g/deta, wrap(phi_g-phi)/dphi, v/dv, min(d,dcap)/dcap, a_prev[0]]
 * ORC_FEAT_EIGHT  8 inputs  the six above, then [(v_g-v)/dv, a_prev[1]]                          */
enum { ORC_FEAT_PAPER = 0, ORC_FEAT_SIX = 1, ORC_FEAT_EIGHT = 2 };

typedef struct {
    double dt;                    /* sampling time T_s (Table II)                              */
    double lf, lr;                /* CoG to front / rear axle (Table I)                        */
    double front, rear, half_width; /* rectangle extents from the CoG: +xi, -xi, |eta|          */
    double delta_max;             /* steering limit (Table I)                                  */
    double delta_rate_max;        /* steering-rate limit, 0 = off (Table I)                    */
    double u_min, u_max;          /* longitudinal acceleration range (Table I)                 */
    double v_min, v_max;          /* speed clamp (may be -inf/+inf)                            */
    int n_layers;                 /* weight layers (2 or 3)                                    */
    int widths[ORC_MAX_LAYERS + 1]; /* widths[0] = inputs ... widths[n_layers] = 2             */
    int feature_set;              /* ORC_FEAT_*                                                */
    double norm_xi, norm_eta, norm_phi, norm_v; /* Delta constants of eq. (3), Table II         */
    double d_cap;                 /* cap of the nearest-obstacle distance feature              */
    double effort_weight;         /* weight of the control-effort term of the cost             */
    double eps_xi, eps_eta, eps_phi, eps_v; /* goal tolerances (Table II)                       */
    double goal_heading_weight;   /* optional terminal cost terms (0 = off): weight of          */
    double goal_speed_weight;     /* |wrap(phi_g - phi_T)| and of |v_g - v_T|                   */
} orc_model;

typedef struct {
    double z0[4];                 /* x, y, phi, v                                              */
    double goal[4];               /* x, y, phi, v   (eq. (1))                                  */
    double a_prev[2];             /* a_{t-1}                                                   */
    const double *points;         /* [P][4]: x, y, vx, vy at time t                            */
    int P;
    int T;                        /* horizon length in steps                                   */
} orc_scene;

/* Per-sample rollout record. Array members may be NULL. */
typedef struct {
    double *traj;                 /* [T+1][4] states z_0..z_T                                  */
    double *controls;             /* [T][2] applied normalised controls a_0..a_{T-1}           */
    double *d_near;               /* [T+1] nearest obstacle distance (uncapped; +inf if P = 0) */
    int *step_flags;              /* [T+1] 1 if some point is strictly inside at step h        */
    double cost;                  /* +inf on collision                                          */
    int collided;
    int first_collision;          /* -1 if none                                                */
    double min_margin;            /* min over h, j of max(|xi_c|/hl, |eta|/hw)                  */
    double min_abs_face;          /* min |face distance| over points and steps h <= first hit  */
    int goal_reached;             /* tolerance test of Table II at z_T                         */
} orc_record;

int    orc_n_theta(const orc_model *m);
int    orc_num_threads(void);

void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_theta_value(uint64_t seed, uint32_t inst, uint32_t stream, uint32_t i, uint32_t k);
void   orc_draw_theta(uint64_t seed, uint32_t inst, uint32_t i0, uint32_t n, uint32_t n_theta,
                      double *out);

double orc_wrap_angle(double a);
void   orc_mlp(const orc_model *m, const double *theta, const double *s, double *a);
void   orc_features(const orc_model *m, const double z[4], const double goal[4], double d_near,
                    const double a_prev[2], double *s);
void   orc_limit_rate(const orc_model *m, const double a_raw[2], const double a_prev[2],
                      double a[2]);
void   orc_control_map(const orc_model *m, const double a[2], double *delta, double *u);
void   orc_vehicle_step(const orc_model *m, const double z[4], double delta, double u,
                        double z_next[4]);
void   orc_extrapolate(const double point[4], double t, double out[2]);
int    orc_point_inside(const orc_model *m, const double pose[3], const double p[2]);
double orc_face_distance(const orc_model *m, const double pose[3], const double p[2]);
double orc_margin(const orc_model *m, const double pose[3], const double p[2]);

/* fp32_state: 0 binary64 throughout; 1..4 inject binary32 rounding (1: state after every step,
 * 2: also features and applied controls, 3: also the controller, 4: the whole step computed in
 * binary32), used by the tests to recognise samples whose outcome is ill-conditioned. */
void   orc_rollout(const orc_model *m, const orc_scene *sc, const double *theta,
                   int fp32_state, orc_record *rec);
void   orc_rollout_samples(const orc_model *m, const orc_scene *sc, uint64_t seed, uint32_t inst,
                           const uint32_t *idx, int count, int fp32_state,
                           double *traj, double *controls, double *d_near, double *cost,
                           int *collided, int *first_collision, double *min_margin,
                           double *min_abs_face);
int    orc_argmin(const double *cost, int n, int *best);
int    orc_plan(const orc_model *m, const orc_scene *sc, int N, uint64_t seed, uint32_t inst,
                double *cost, int *best, double *theta_best, double *traj_best,
                double *controls_best, int *goal_reached);
void   orc_step_at_states(const orc_model *m, const orc_scene *sc, const double *theta,
                          const double *states, const double *a_prev, const int *steps, int M,
                          double *a_out, double *z_next, double *d_near);
void   orc_flags_at_poses(const orc_model *m, const double *points, int P, double dt,
                          const double *poses, const int *steps, int M, double eps, int *flag);

#ifdef __cplusplus
}
#endif

#endif
