/*
 * nnfleet: the closed-loop algorithm (Alg. 1, Sect. II) served for many vehicles at once on one
 * MI355X (gfx950).
 *
 * Every call of nnp_fleet_step is one sampling time t for every vehicle whose mission is not yet
 * complete: measurement m_t^z = z_t (Sect. II-B, simplest case), the current waypoint of the
 * vehicle's mission as goal setpoint zeta_t^goal (Sect. II-D, switched to the next waypoint once
 * the vehicle is within the tolerances), the control a_t from one batched plan (Step 5; the
 * previous best parameters theta*_{t-1} warm-start sample 0 and a_{t-1} feeds the features, Sect.
 * II-E), application of a_t (the vehicle follows the kinematic model of Sect. II-F, i.e. z_{t+1}
 * is the plan's first predicted state), the mission check (Step 7), and the obstacles' constant-
 * velocity motion to t+1. Samples per plan: n_prop draws from the learned proposal (encoding and
 * network of include/nnproposal.h, evaluated on the GPU every step) plus n_uniform uniform draws;
 * the Philox key of vehicle i is seed + i and the instance word is the step index, so vehicles
 * and steps draw independent samples.
 *
 * Conventions are those of include/nnplan.h.
 */
#ifndef NNFLEET_H
#define NNFLEET_H

#include <stdint.h>

#include "nnplan.h"
#include "nnproposal.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnp_fleet_config {
    int32_t n_vehicles;        /* 1..65535                                                    */
    int32_t T;                 /* horizon of every plan                                       */
    int32_t n_uniform;         /* uniform samples per plan (>= 1)                             */
    int32_t n_prop;            /* proposal samples per plan (0 = plain sampler)                */
    uint64_t seed;             /* Philox key of vehicle i's plans: seed + i                    */
    int32_t warm_start;        /* 1: theta*_{t-1} replaces sample 0 from the second step on    */
    float dt;                  /* sampling time T_s (obstacle motion between steps)           */
    float eps_xi, eps_eta, eps_phi, eps_v; /* waypoint tolerances (Table II)                  */
    int32_t switch_rule;       /* NNP_SWITCH_STATE or NNP_SWITCH_PLAN (below)                  */
} nnp_fleet_config;

/* Waypoint switching (Step 4 of Alg. 1, Sect. II-D). NNP_SWITCH_STATE: the next waypoint becomes
 * the goal setpoint once the vehicle's own state z_{t+1} is within the tolerances.
 * NNP_SWITCH_PLAN: the recursive logic the goal-setpoint discussion names, based on whether the
 * last plan reached the setpoint over its horizon: an intermediate waypoint is passed once the
 * best plan's predicted trajectory comes within the tolerances at any step h = 1..T; the final
 * waypoint (mission completion, Step 7) still needs the vehicle's own state within them. */
#define NNP_SWITCH_STATE 0
#define NNP_SWITCH_PLAN 1

typedef struct nnp_vehicle_spec {
    float z0[4];               /* initial state x, y, phi in [-pi, pi], v                     */
    const float *waypoints;    /* host [n_waypoints][4] goal setpoints x, y, phi, v, in order  */
    int32_t n_waypoints;       /* >= 1; the mission is complete when the last one is reached   */
    const float *obst;         /* device [P][4] obstacle points (x, y, vx, vy) at t = 0; copied */
    int32_t P;                 /* 0..NNP_MAX_P                                                 */
    int32_t own_goal_weights;  /* 1: this vehicle's plans weigh the goal's heading and speed    */
    float goal_heading_weight; /* with these (nnp_problem's fields of the same names); 0: the   */
    float goal_speed_weight;   /* planner model's                                              */
} nnp_vehicle_spec;

/* Per-vehicle status after a step (host copy). */
typedef struct nnp_vehicle_state {
    float z[4];                /* current state z_t                                           */
    float a[2];                /* last applied normalised controls a_{t-1}; before the first   */
                               /* step a[1] is NaN (idle acceleration is used)                 */
    float cost;                /* best cost of the last plan (+INFINITY if it was infeasible)  */
    int32_t waypoint;          /* index of the current waypoint (n_waypoints when complete)    */
    int32_t steps;             /* sampling times taken                                         */
    int32_t done;              /* 1 once the mission is complete                               */
    int32_t infeasible_steps;  /* plans in which every sample collided                         */
} nnp_vehicle_state;

typedef struct nnp_fleet nnp_fleet;

/* Create a fleet served by `planner` (and `proposal` when n_prop > 0; it must have been created
 * with max_batch >= n_vehicles and the planner's n_theta). Copies the specs (waypoints to host
 * memory, obstacles to device memory owned by the fleet). The handles are borrowed: they must
 * outlive the fleet and must not be used by others during nnp_fleet_step. */
int nnp_fleet_create(nnp_fleet **f, nnp_handle *planner, nnp_proposal *proposal,
                     const nnp_fleet_config *c, const nnp_vehicle_spec *vehicles);

/* One sampling time for every vehicle whose mission is not complete (see above). Synchronises
 * hip_stream before returning (the controls must reach the vehicles). *latency_ms (may be NULL)
 * receives the host wall time of the call; *active (may be NULL) the number of vehicles planned.
 * Returns NNP_OK, or a negative code. */
int nnp_fleet_step(nnp_fleet *f, void *hip_stream, double *latency_ms, int32_t *active);

/* Copy the vehicles' status to host states[n_vehicles]. */
int nnp_fleet_state(const nnp_fleet *f, nnp_vehicle_state *states);

/* Release the fleet (waits for its device work). NULL is accepted. */
void nnp_fleet_destroy(nnp_fleet *f);

/* Text of the fleet's last error ("" if none); NULL: the last create failure. */
const char *nnp_fleet_last_error(const nnp_fleet *f);

#ifdef __cplusplus
}
#endif

#endif
