/*
 * nnplan: MI355X (gfx950) batched closed-loop rollout planner.
 *
 * The method is the one of M. G. Plessen, "Online Sampling in the Parameter Space of a Neural
 * Network for GPU-accelerated Motion Planning of Autonomous Vehicles": at every sampling time a
 * population of neural-network parameter vectors theta is drawn, each theta is held constant and
 * rolled over the prediction horizon in closed loop (features s_{t+h} of eq. (3), controls
 * a_{t+h} = X(s_{t+h}, theta) of eq. (4), kinematic model of Sect. II-F), constant-velocity
 * extrapolated obstacle points are tested against the vehicle rectangle with the linear
 * inequalities of eq. (2) at every step, and the best parameter vector is returned (Step 5 of
 * Alg. 1, Sect. II-E).
 *
 * Conventions for every entry point:
 *  - All float arithmetic on the device is IEEE binary32.
 *  - "device" pointers are HIP global-memory addresses on the handle's device; "host" pointers are
 *    ordinary CPU memory that the call reads before returning. The library never frees or keeps
 *    caller memory.
 *  - hip_stream is a hipStream_t (NULL = the default stream). Device work is enqueued on it and
 *    the call returns without waiting; device outputs are valid once the stream has been
 *    synchronised. Calls on one handle must be ordered (one stream, or explicit events).
 *  - Return values: NNP_OK on success, a negative NNP_E* code on failure (nothing is enqueued on
 *    failure). nnp_last_error() gives a readable reason for the handle's last failure.
 *  - A handle is not thread-safe; use one handle per host thread.
 */
#ifndef NNPLAN_H
#define NNPLAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NNP_OK 0
#define NNP_INFEASIBLE 1      /* device status value: every sample collides                 */
#define NNP_EINVAL (-1)       /* bad argument: null pointer, size out of range, non-finite   */
#define NNP_ENOMEM (-2)       /* device allocation failed                                    */
#define NNP_EDEVICE (-3)      /* a HIP call failed; see nnp_last_error()                     */
#define NNP_EUNSUPPORTED (-4) /* network shape / lane layout without a compiled kernel       */

#define NNP_MAX_LAYERS 3
#define NNP_MAX_T 4096        /* longest horizon accepted                                    */
#define NNP_MAX_P (1 << 22)   /* most obstacle points accepted                               */
#define NNP_MAX_BATCH 65535   /* most problems in one nnp_plan_batch call                    */
#define NNP_NOALLOC_SCRATCH_BYTES (4 << 20) /* device scratch of nnp_plan_noalloc, per GPU      */

/* Feature vectors of eq. (3) (Sect. II-E) and the two extended variants:
 * NNP_FEAT_PAPER  5 inputs: [xi_g/dxi, eta_g/deta, wrap(phi_g-phi)/dphi, (v_g-v)/dv, a_prev[0]]
 * NNP_FEAT_SIX    6 inputs: [xi_g/dxi, eta_g/deta, wrap(phi_g-phi)/dphi, v/dv,
 *                            min(d_near,d_cap)/d_cap, a_prev[0]]
 * NNP_FEAT_EIGHT  8 inputs: the six, then [(v_g-v)/dv, a_prev[1]]
 * (xi_g, eta_g) is the goal position in the vehicle frame of step h; d_near the distance from the
 * reference point to the nearest extrapolated obstacle point at step h.                          */
#define NNP_FEAT_PAPER 0
#define NNP_FEAT_SIX 1
#define NNP_FEAT_EIGHT 2

/* Vehicle, controller and cost constants (Sect. II-F, Table I, Table II). Copied at creation. */
typedef struct nnp_model {
    float dt;                        /* sampling time T_s [s]                                   */
    float lf, lr;                    /* reference point (CoG) to front / rear axle [m]          */
    float front, rear, half_width;   /* rectangle extents from the reference point [m]: ahead,  */
                                     /* behind, to each side                                    */
    float delta_max;                 /* steering limit [rad]: delta = delta_max * a[0]          */
    float delta_rate_max;            /* steering-rate limit [rad/s]; 0 disables it              */
    float u_min, u_max;              /* acceleration range [m/s^2] mapped from a[1] in [-1, 1]   */
    float v_min, v_max;              /* speed clamp after every step (+-INFINITY = none)        */
    int32_t n_layers;                /* weight layers of the tanh MLP: 2 or 3                   */
    int32_t widths[NNP_MAX_LAYERS + 1]; /* widths[0] = inputs, ..., widths[n_layers] = 2       */
    int32_t feature_set;             /* NNP_FEAT_*; must match widths[0]                        */
    float norm_xi, norm_eta, norm_phi, norm_v; /* Delta normalisers of eq. (3)                  */
    float d_cap;                     /* cap of the nearest-obstacle distance feature [m]        */
    float effort_weight;             /* cost = |p_T - g_xy| + effort_weight*T_s*sum|a_h|^2     */
    float eps_xi, eps_eta, eps_phi, eps_v; /* goal tolerances for the goal_reached flag          */
    int32_t lanes_per_sample;        /* 0 = library default for the network; 1, 2, 4, 8, 16    */
    float goal_heading_weight;       /* optional terminal terms of the cost (>= 0; 0 = off):   */
    float goal_speed_weight;         /* + w_phi |wrap(phi_g - phi_T)| + w_v |v_g - v_T|        */
    int32_t block_threads;           /* rollout workgroup size; 0 = default for the layout      */
    int32_t tile_pairs;              /* point pairs per LDS buffer; 0 = default for the layout   */
                                     /* (lanes_per_sample, block_threads, tile_pairs): one of   */
                                     /* the compiled launch shapes, else NNP_EUNSUPPORTED; all  */
                                     /* shapes give the same results bit for bit                */
    int32_t all_points;              /* 0: the obstacle pass skips groups of 64 points whose     */
                                     /* bounding box is, for every sample of a wavefront,       */
                                     /* beyond both the rectangle's corner distance and either  */
                                     /* d_cap (distance features) or a bound on the step's      */
                                     /* nearest distance carried from the previous step: such   */
                                     /* points cannot change a collision, a margin below 1 or   */
                                     /* the capped nearest distance; 1: every point is tested.  */
                                     /* Same results bit for bit either way.                    */
} nnp_model;

/* One planning problem at sampling time t (Sect. II-E, fourth comment: what is passed to the GPU
 * every t: theta source (seed), m_t^z, a_{t-1}, zeta_t^goal, m_t^ext). */
typedef struct nnp_problem {
    float z0[4];              /* host copy: x, y, heading phi in [-pi, pi], speed v             */
    float goal[4];            /* host copy: zeta^goal = x, y, phi in [-pi, pi], v (eq. (1))     */
    const float *a_prev;      /* host [2] previous controls a_{t-1}; NULL = [0, a_idle]         */
                              /* (zero acceleration, Sect. III)                                 */
    const float *obst;        /* device [P][4] rows x, y, vx, vy of the obstacle points at t;   */
                              /* may be NULL when P = 0                                         */
    int32_t P;                /* number of obstacle points, 0..NNP_MAX_P                        */
    int32_t N;                /* number of parameter samples, >= 1                              */
    int32_t T;                /* horizon steps H, 1..NNP_MAX_T                                  */
    uint32_t inst;            /* Philox instance word (fourth counter word)                     */
    uint64_t seed;            /* Philox key                                                     */
    const float *warm_theta;  /* device [n_theta] or NULL: replaces sample 0 (warm start of    */
                              /* the first restart with theta*_{t-1}, Sect. II-E fifth comment) */
    int32_t n_prop;           /* 0..N: samples 0..n_prop-1 come from the Gaussian proposal      */
                              /* theta_k = mu_k + exp(log_sigma_k) z_k (z: Box-Muller on Philox  */
                              /* stream 1, see nnp_sample_gauss); samples n_prop..N-1 are the    */
                              /* uniform draws 0..N-n_prop-1 of stream 0. 0 = plain sampler.     */
    const float *prop_mu;        /* device [n_theta] proposal mean (may be NULL if n_prop = 0)   */
    const float *prop_log_sigma; /* device [n_theta] proposal log standard deviation             */
    int32_t own_goal_weights;    /* 1: this problem's cost takes the two weights below instead   */
                                 /* of the model's goal_heading_weight / goal_speed_weight       */
                                 /* (finite, >= 0); 0: the model's (missions of different kinds  */
                                 /* in one batch may weigh the goal's heading and speed apart)   */
    float goal_heading_weight;
    float goal_speed_weight;
} nnp_problem;

/* Outputs of nnp_plan: caller-owned device buffers; any member may be NULL to skip it. */
typedef struct nnp_result {
    float *theta;             /* [n_theta] best parameter vector theta*                          */
    float *controls;          /* [T][2] normalised controls a_h of theta* (after rate limit)     */
    float *controls_phys;     /* [T][2] steering delta [rad], acceleration u [m/s^2]             */
    float *traj;              /* [T+1][4] states z_h of theta*                                   */
    float *cost;              /* [1] best cost (+INFINITY when infeasible)                       */
    int32_t *best_index;      /* [1] sample index of theta* (lowest index among equal costs)     */
    int32_t *status;          /* [1] NNP_OK, or NNP_INFEASIBLE when every sample collides (the   */
                              /*     outputs then describe sample 0)                             */
    int32_t *goal_reached;    /* [1] 1 if z_T is within the eps tolerances of the goal           */
} nnp_result;

/* Per-sample outputs of nnp_rollout: caller-owned device buffers; NULL skips a member. */
typedef struct nnp_rollout_out {
    float *cost;              /* [N] cost per sample, +INFINITY if it collides at some h in 0..T */
    int32_t *collided;        /* [N] 0/1                                                         */
    int32_t *first_collision; /* [N] first step h with a point inside, -1 if none               */
    float *min_margin;        /* [N] min over h and points of max(|xi_c|/hl, |eta|/hw): < 1      */
                              /*     exactly when some point is inside (diagnostic)              */
    float *traj;              /* [N][T+1][4] states                                              */
    float *controls;          /* [N][T][2] normalised controls                                   */
} nnp_rollout_out;

typedef struct nnp_handle nnp_handle;

/* Create a planner for model *m on HIP device `device`. Validates the model (finite constants,
 * positive extents, supported network shape, feature set consistent with widths[0]) and
 * allocates the handle's small device workspace. Returns NNP_EINVAL / NNP_EUNSUPPORTED /
 * NNP_ENOMEM / NNP_EDEVICE on failure, with *h set to NULL. */
int nnp_create(nnp_handle **h, const nnp_model *m, int device);

/* Release the handle and its workspace. NULL is accepted. Waits for the handle's device work. */
void nnp_destroy(nnp_handle *h);

/* Number of parameters of the handle's network (Table III counts: weights plus biases). */
int nnp_n_theta(const nnp_handle *h);

/* Step 5 of Alg. 1 as a plain sampler (Sect. II-E): draw N parameter vectors from Philox, roll
 * each over h = 0..T with collision checks of eq. (2) at every h, cost every sample, and return
 * the lowest-cost one (lowest index on ties) with its controls and trajectory. Every sample is
 * simulated over the whole horizon. The winner's controls come from per-sample records of the
 * applied controls that the rollout writes into the handle's workspace (8 N T bytes, grown on
 * demand like the extrapolation table) and its states from z0 and those controls by the model
 * step alone, when that size is within the handle's record limit and below 2^31 bytes; else the
 * winner is re-simulated with its obstacle passes. Both give the same bits. */
int nnp_plan(nnp_handle *h, const nnp_problem *p, nnp_result *r, void *hip_stream);

/* Largest per-sample record workspace nnp_plan and nnp_plan_batch may use (default 2^32 bytes;
 * a batch needs the sum over its problems); 0 makes every plan re-simulate its winner instead.
 * Results do not depend on it. Returns NNP_EINVAL for h == NULL. */
int nnp_set_record_limit(nnp_handle *h, uint64_t bytes);

/* Cap on the device workspace the handle grows on demand (extrapolation table, per-sample
 * records, batch tables and descriptors; default: none). nnp_plan leaves the records out when
 * they would exceed it; a call that still needs more fails with NNP_ENOMEM before any device work
 * and names the buffer in nnp_last_error. Lowering the cap frees nothing already allocated.
 * Returns NNP_EINVAL for h == NULL. */
int nnp_set_workspace_limit(nnp_handle *h, uint64_t bytes);

/* nnp_plan for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): same arguments, same validation and the same
 * outputs bit for bit as nnp_plan, but the call allocates nothing, on the device or the host. Its
 * argmin key and extrapolation table live in a fixed file-scope device array of
 * NNP_NOALLOC_SCRATCH_BYTES (4 MiB) that every GPU the library runs on holds until the process
 * ends; the winner's outputs are re-simulated (no per-sample records). Limit: the table of
 * (T + 1) * (P rounded up to a multiple of 64) / 2 point pairs of 16 bytes, plus 64 pairs of
 * slack, the boxes of its groups of 32 pairs, the spatial order of up to 2^20 points and 256
 * bytes for the key, must fit (T = 50 allows P up to 9856); larger problems
 * return NNP_EINVAL with the sizes in nnp_last_error. The key is reset by the call itself. All
 * calls on one GPU share that GPU's array: calls that overlap on one GPU (on different streams,
 * from different threads or handles) race and must be serialised by the caller; consecutive
 * calls on one stream are ordered. The handle's timing instrumentation does not record these
 * calls. Returns the codes of nnp_plan. */
int nnp_plan_noalloc(nnp_handle *h, const nnp_problem *p, nnp_result *r, void *hip_stream);

/* Many independent problems in one call: the same plan as nnp_plan for every probs[i] (each with
 * its own N, T, P, obstacles, seed and warm start), written to results[i]. All problems are
 * rolled out by one launch of one workgroup per (problem, block of samples) item, longest
 * problems first, so uneven sizes share the GPU without a launch per problem.
 * The call copies `count` problem descriptors to the device through a pinned staging buffer
 * owned by the handle (it waits for the previous batch's copy before reusing it) and enqueues
 * four kernels. The winners' outputs are gathered from per-sample records, one region per
 * problem, when the batch's 8 * sum(N T) bytes fit the record limit and the workspace cap, and
 * re-simulated otherwise. Results are bit-identical to nnp_plan on each problem and to every lane
 * layout.
 * Returns NNP_EINVAL if count is outside 1..NNP_MAX_BATCH or any problem is invalid
 * (nnp_last_error names it).
 * HIP graph capture: the call records one host-to-device copy from the staging buffer and four
 * kernels (no memsets, no host synchronisation). The handle's batch workspace must already be
 * large enough, i.e. an uncaptured call with at least as many problems, samples-times-points and
 * table entries must come first, else NNP_EINVAL; records are used under capture only when the
 * allocation made before holds them (else the winners are re-simulated). Replays re-read the staging buffer, so between
 * the capture and the graph's last replay no other nnp_plan_batch call may be made on the same
 * handle (use a second handle for other batches); nnp_plan and nnp_rollout do not touch it. */
int nnp_plan_batch(nnp_handle *h, const nnp_problem *probs, int count, nnp_result *results,
                   void *hip_stream);

/* Step 5 of Alg. 1 (Sect. II-E) without the final selection: every sample's closed loop over the
 * horizon (features eq. (3), controller eq. (4), model eq. (5) of Sect. II-F, obstacle points
 * extrapolated at constant velocity and tested with eq. (2) at every h = 0..T), with per-sample
 * outputs instead of the argmin: o->cost[N] (f32, +inf after any collision), o->collided[N]
 * (i32 0/1), o->first_collision[N] (i32, first step with a point inside, -1 if none),
 * o->min_margin[N] (f32, smallest normalised margin over steps and points, < 1 inside; when it
 * is requested the call tests every point, since skipped groups would leave it out), and
 * optionally o->traj[N][T+1][4] (z_h) and o->controls[N][T][2] (normalised a_h). Every output
 * pointer is a caller-owned device buffer and may be NULL (not written). Same kernel and device
 * functions as nnp_plan, so the costs are bit-identical to the ones nnp_plan minimises.
 * theta, if not NULL, is a device [N][n_theta] array of parameters used instead of the Philox
 * draws (explicit-parameter hook for tests and for externally proposed samples, the theta that
 * Sect. II-E's fourth comment lists among the host-to-GPU inputs); p->warm_theta is ignored
 * then. Asynchronous on hip_stream. Returns NNP_OK, NNP_EINVAL (null handle/problem/output
 * struct, N < 1, T outside 1..4096, P outside 0..2^22, non-finite or out-of-range z0, goal or
 * a_prev), NNP_ENOMEM (workspace) or NNP_EDEVICE (HIP error; nnp_last_error has the text). */
int nnp_rollout(nnp_handle *h, const nnp_problem *p, const float *theta, nnp_rollout_out *o,
                void *hip_stream);

/* The parameter draws of nnp_plan for samples i0..i0+N-1 into device out[N][n_theta]. Sect.
 * II-E's fourth comment has the host pass the parameter samples and the current random seed to
 * the GPU at every sampling time; here the samples are a pure function of (seed, inst, i), so
 * only the seed crosses, and this call materialises the same values: theta_k of sample i =
 * (2m + 1 - 2^24) 2^-24, m the top 24 bits of word k mod 4 of Philox4x32-10(counter = (k / 4,
 * i, 0, inst), key = (seed low 32, seed high 32)), i.e. uniform in (-1, 1) (the reading of the
 * unbounded parameter range of Sect. III-A as the uniform box the plain sampler draws from),
 * exact in binary32. out is caller-owned; layout sample-major, parameters layer by layer (W_l
 * row-major, then b_l). Asynchronous on hip_stream, on the current HIP device. Returns NNP_OK,
 * NNP_EINVAL (out == NULL, N == 0, n_theta == 0 or N * n_theta >= 2^40) or NNP_EDEVICE. */
int nnp_sample_theta(uint64_t seed, uint32_t inst, uint32_t i0, uint32_t N, uint32_t n_theta,
                     float *out, void *hip_stream);

/* The proposal draws of nnp_plan (samples with index < n_prop) for Philox sample words
 * i0..i0+N-1 into device out[N][n_theta]: theta_k = mu_k + exp(log_sigma_k) z_k, rounded once
 * (fused multiply-add), with z the Box-Muller normals of Philox4x32-10(counter = (k / 4, i, 1,
 * inst), key = (seed low 32, seed high 32)): words (0, 1) serve k mod 4 in {0, 1}, words (2, 3)
 * serve {2, 3}; u = (m + 1/2) 2^-23 with m the top 23 bits of a word; z = sqrt(-2 ln u_a)
 * cos(2 pi u_b) for even k, sin for odd k. mu and log_sigma are device [n_theta]. Runs on the
 * current HIP device. Bit-identical to the draws inside nnp_plan. */
int nnp_sample_gauss(uint64_t seed, uint32_t inst, uint32_t i0, uint32_t N, uint32_t n_theta,
                     const float *mu, const float *log_sigma, float *out, void *hip_stream);

/* Text of the handle's last error ("" if none). With h == NULL: the last nnp_create failure. */
const char *nnp_last_error(const nnp_handle *h);

/* Device-time instrumentation of the rollout kernel: when enabled, nnp_plan and nnp_rollout
 * bracket the rollout-kernel launch with HIP events on the caller's stream. nnp_kernel_time
 * synchronises on the last recorded event and returns the summed kernel milliseconds and the
 * number of launches since the last reset. */
int nnp_set_timing(nnp_handle *h, int enable);
int nnp_kernel_time(nnp_handle *h, double *ms, int64_t *launches, int reset);

/* Work counter of the obstacle pass's group skipping (nnp_model.all_points = 0): when enabled,
 * every rollout kernel launched through the handle (nnp_plan, nnp_plan_noalloc, nnp_plan_batch,
 * nnp_rollout) adds, per wavefront and step (and tile), the number of point groups it tested and
 * the number the step has; nnp_cull_stats synchronises the device and returns both sums since
 * the last reset (their ratio is the share of the point tests actually executed). Enabling
 * allocates and clears a 16-byte device counter (synchronously; not under stream capture);
 * disabling keeps it but stops the counting. Counting costs two device atomics per wavefront and
 * launch. Returns NNP_OK, NNP_EINVAL (null handle) or NNP_ENOMEM / NNP_EDEVICE. */
int nnp_set_cull_stats(nnp_handle *h, int enable);
int nnp_cull_stats(nnp_handle *h, uint64_t *tested, uint64_t *total, int reset);

/* Library version string. */
const char *nnp_version(void);

#ifdef __cplusplus
}
#endif

#endif
