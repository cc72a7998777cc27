// nnfleet: closed-loop receding-horizon planning served for many vehicles (declarations in
// include/nnfleet.h). Host runtime around the batched planner and the proposal network; the
// per-step device work is one encoding + forward pass, one batched plan, one status kernel and
// the obstacles' motion.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <chrono>
#include <string>
#include <vector>

#include "../../include/nnfleet.h"
#include "rollout.hpp"

namespace {

struct StatusRec {
    float z[4];
    float a[2];
    float cost;
    int32_t reached;           // z_{t+1} within the tolerances
    int32_t status;
    int32_t plan_reached;      // some predicted state z_h, h = 1..T, within the tolerances
    int32_t pad[2];
};

struct FleetEps {
    float xi, eta, phi, v;
};

// z_{t+1} = the plan's first predicted state, a_t = its first control; waypoint check at z_{t+1}
// and over the whole predicted trajectory. One vehicle per workgroup of 64 lanes: lane h tests
// the predicted states h + 1, h + 65, ... (infeasible plans never count as reaching).
__global__ void fleet_status_kernel(int n, int T, const float *__restrict__ traj,
                                    const float *__restrict__ controls,
                                    const float *__restrict__ cost,
                                    const int32_t *__restrict__ status,
                                    const float *__restrict__ goals, FleetEps eps,
                                    StatusRec *__restrict__ out)
{
    const int j = blockIdx.x;
    if (j >= n) return;
    const float *tr = traj + (size_t)j * (T + 1) * 4;
    const float g[4] = {goals[4 * j], goals[4 * j + 1], goals[4 * j + 2], goals[4 * j + 3]};
    int any = 0;
    for (int h = 1 + (int)threadIdx.x; h <= T; h += 64) {
        const float *z = tr + 4 * (size_t)h;
        float sn, cs;
        sincosf(z[2], &sn, &cs);
        any |= nnp::within_tolerance(eps.xi, eps.eta, eps.phi, eps.v, g, z[0], z[1], z[2], z[3],
                                     cs, sn);
    }
    any = __any(any);
    if (threadIdx.x != 0) return;
    const float *z = tr + 4;
    const float *a = controls + (size_t)j * T * 2;
    StatusRec r;
    for (int k = 0; k < 4; ++k) r.z[k] = z[k];
    r.a[0] = a[0];
    r.a[1] = a[1];
    r.cost = cost[j];
    r.status = status[j];
    float sn, cs;
    sincosf(r.z[2], &sn, &cs);
    r.reached = nnp::within_tolerance(eps.xi, eps.eta, eps.phi, eps.v, g, r.z[0], r.z[1], r.z[2],
                                      r.z[3], cs, sn);
    r.plan_reached = any && r.status != NNP_INFEASIBLE;
    r.pad[0] = r.pad[1] = 0;
    out[j] = r;
}

// Constant-velocity motion of every obstacle point over one sampling time.
__global__ void advance_obstacles_kernel(float4 *__restrict__ pts, long long n, float dt)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float4 p = pts[i];
    p.x = fmaf(dt, p.z, p.x);
    p.y = fmaf(dt, p.w, p.y);
    pts[i] = p;
}

}  // namespace

struct nnp_fleet {
    nnp_handle *planner = nullptr;
    nnp_proposal *prop = nullptr;
    nnp_fleet_config cfg{};
    int n_theta = 0, device = 0;
    long long tick = 0;
    int parity = 0;
    // vehicles (host)
    std::vector<nnp_vehicle_state> st;
    std::vector<std::vector<float>> wps;
    std::vector<long long> obst_off;
    std::vector<int> obst_n;
    std::vector<nnp_vehicle_spec> spec;   // the specs as given (pointers not used after create)
    // device
    float4 *d_obst = nullptr;
    long long n_points = 0;
    float *d_warm = nullptr;                    // [2][n][n_theta]
    float *d_enc = nullptr, *d_mu = nullptr, *d_ls = nullptr;
    float *d_ctrl = nullptr, *d_traj = nullptr, *d_cost = nullptr, *d_goal = nullptr;
    int32_t *d_status = nullptr;
    StatusRec *d_rec = nullptr, *h_rec = nullptr;
    float *h_goal = nullptr, *h_aprev = nullptr;
    std::string err;
};

namespace {

std::string g_fleet_error;

int ffail(nnp_fleet *f, int code, const std::string &msg)
{
    if (f) f->err = msg;
    else g_fleet_error = msg;
    return code;
}

}  // namespace

extern "C" {

void nnp_fleet_destroy(nnp_fleet *f)
{
    if (!f) return;
    hipSetDevice(f->device);
    hipDeviceSynchronize();
    for (void *p : {(void *)f->d_obst, (void *)f->d_warm, (void *)f->d_enc, (void *)f->d_mu,
                    (void *)f->d_ls, (void *)f->d_ctrl, (void *)f->d_traj, (void *)f->d_cost,
                    (void *)f->d_goal, (void *)f->d_status, (void *)f->d_rec})
        if (p) hipFree(p);
    for (void *p : {(void *)f->h_rec, (void *)f->h_goal, (void *)f->h_aprev})
        if (p) hipHostFree(p);
    delete f;
}

int nnp_fleet_create(nnp_fleet **out, nnp_handle *planner, nnp_proposal *proposal,
                     const nnp_fleet_config *c, const nnp_vehicle_spec *veh)
{
    if (!out) return ffail(nullptr, NNP_EINVAL, "null fleet pointer");
    *out = nullptr;
    if (!planner || !c || !veh) return ffail(nullptr, NNP_EINVAL, "null argument");
    const int n = c->n_vehicles;
    if (n < 1 || n > 65535) return ffail(nullptr, NNP_EINVAL, "n_vehicles must be in [1, 65535]");
    if (c->T < 1 || c->T > NNP_MAX_T) return ffail(nullptr, NNP_EINVAL, "T out of range");
    if (c->n_uniform < 1 || c->n_prop < 0) return ffail(nullptr, NNP_EINVAL, "sample counts");
    if (c->n_prop > 0 && !proposal)
        return ffail(nullptr, NNP_EINVAL, "n_prop > 0 needs a proposal network");
    if (!(c->dt > 0.0f) || !(c->eps_xi >= 0.0f) || !(c->eps_eta >= 0.0f) ||
        !(c->eps_phi >= 0.0f) || !(c->eps_v >= 0.0f))
        return ffail(nullptr, NNP_EINVAL, "dt / tolerances");
    if (c->switch_rule != NNP_SWITCH_STATE && c->switch_rule != NNP_SWITCH_PLAN)
        return ffail(nullptr, NNP_EINVAL, "switch_rule must be NNP_SWITCH_STATE or NNP_SWITCH_PLAN");
    nnp_fleet *f = new nnp_fleet();
    f->planner = planner;
    f->prop = c->n_prop > 0 ? proposal : nullptr;
    f->cfg = *c;
    f->n_theta = nnp_n_theta(planner);
    hipGetDevice(&f->device);
    f->st.resize((size_t)n);
    f->wps.resize((size_t)n);
    f->obst_off.resize((size_t)n);
    f->obst_n.resize((size_t)n);
    f->spec.assign(veh, veh + n);
    long long total = 0;
    for (int i = 0; i < n; ++i) {
        const nnp_vehicle_spec &v = veh[i];
        const bool weights_ok =
            v.own_goal_weights == 0 ||
            (v.own_goal_weights == 1 && v.goal_heading_weight >= 0.0f &&
             v.goal_speed_weight >= 0.0f && isfinite(v.goal_heading_weight) &&
             isfinite(v.goal_speed_weight));
        if (v.n_waypoints < 1 || !v.waypoints || v.P < 0 || v.P > NNP_MAX_P ||
            (v.P > 0 && !v.obst) || !weights_ok) {
            delete f;
            return ffail(nullptr, NNP_EINVAL, "vehicle " + std::to_string(i) + ": bad spec");
        }
        nnp_vehicle_state &s = f->st[(size_t)i];
        memset(&s, 0, sizeof s);
        memcpy(s.z, v.z0, sizeof s.z);
        s.a[0] = 0.0f;
        s.a[1] = NAN;                 // idle acceleration until the first plan (a_prev = NULL)
        s.cost = INFINITY;
        f->wps[(size_t)i].assign(v.waypoints, v.waypoints + 4 * (size_t)v.n_waypoints);
        f->obst_off[(size_t)i] = total;
        f->obst_n[(size_t)i] = v.P;
        total += v.P;
    }
    f->n_points = total;
    const size_t nt = (size_t)f->n_theta, T = (size_t)c->T;
    bool ok = true;
    auto dm = [&](void **p, size_t bytes) {
        if (ok && hipMalloc(p, bytes > 0 ? bytes : 16) != hipSuccess) ok = false;
    };
    dm((void **)&f->d_obst, (size_t)total * sizeof(float4));
    dm((void **)&f->d_warm, 2 * (size_t)n * nt * sizeof(float));
    dm((void **)&f->d_enc, (size_t)n * NNP_PROP_ENC * sizeof(float));
    dm((void **)&f->d_mu, (size_t)n * nt * sizeof(float));
    dm((void **)&f->d_ls, (size_t)n * nt * sizeof(float));
    dm((void **)&f->d_ctrl, (size_t)n * T * 2 * sizeof(float));
    dm((void **)&f->d_traj, (size_t)n * (T + 1) * 4 * sizeof(float));
    dm((void **)&f->d_cost, (size_t)n * sizeof(float));
    dm((void **)&f->d_goal, (size_t)n * 4 * sizeof(float));
    dm((void **)&f->d_status, (size_t)n * sizeof(int32_t));
    dm((void **)&f->d_rec, (size_t)n * sizeof(StatusRec));
    if (ok && hipHostMalloc((void **)&f->h_rec, (size_t)n * sizeof(StatusRec), 0) != hipSuccess)
        ok = false;
    if (ok && hipHostMalloc((void **)&f->h_goal, (size_t)n * 4 * sizeof(float), 0) != hipSuccess)
        ok = false;
    if (ok && hipHostMalloc((void **)&f->h_aprev, (size_t)n * 2 * sizeof(float), 0) != hipSuccess)
        ok = false;
    for (int i = 0; ok && i < n; ++i)
        if (veh[i].P > 0 &&
            hipMemcpy(f->d_obst + f->obst_off[(size_t)i], veh[i].obst,
                      (size_t)veh[i].P * sizeof(float4), hipMemcpyDeviceToDevice) != hipSuccess)
            ok = false;
    if (!ok) {
        nnp_fleet_destroy(f);
        return ffail(nullptr, NNP_ENOMEM, "fleet allocation or obstacle copy failed");
    }
    *out = f;
    return NNP_OK;
}

int nnp_fleet_step(nnp_fleet *f, void *hip_stream, double *latency_ms, int32_t *active)
{
    if (!f) return NNP_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)hip_stream;
    const nnp_fleet_config &c = f->cfg;
    const size_t nt = (size_t)f->n_theta, T = (size_t)c.T;
    std::vector<int> act;
    for (int i = 0; i < c.n_vehicles; ++i)
        if (!f->st[(size_t)i].done) act.push_back(i);
    const int na = (int)act.size();
    if (active) *active = na;
    if (na == 0) {
        if (latency_ms) *latency_ms = 0.0;
        return NNP_OK;
    }
    float *warm_in = f->d_warm + (size_t)f->parity * c.n_vehicles * nt;
    float *warm_out = f->d_warm + (size_t)(f->parity ^ 1) * c.n_vehicles * nt;
    std::vector<nnp_problem> probs((size_t)na);
    std::vector<nnp_result> res((size_t)na);
    for (int j = 0; j < na; ++j) {
        const int i = act[(size_t)j];
        const nnp_vehicle_state &v = f->st[(size_t)i];
        nnp_problem &p = probs[(size_t)j];
        memset(&p, 0, sizeof p);
        memcpy(p.z0, v.z, sizeof p.z0);
        memcpy(p.goal, &f->wps[(size_t)i][4 * (size_t)v.waypoint], sizeof p.goal);
        memcpy(f->h_goal + 4 * j, p.goal, sizeof p.goal);
        if (isnan(v.a[1])) {
            p.a_prev = nullptr;
        } else {
            f->h_aprev[2 * j] = v.a[0];
            f->h_aprev[2 * j + 1] = v.a[1];
            p.a_prev = f->h_aprev + 2 * j;
        }
        p.obst = reinterpret_cast<const float *>(f->d_obst + f->obst_off[(size_t)i]);
        p.P = f->obst_n[(size_t)i];
        p.N = c.n_prop + c.n_uniform;
        p.T = c.T;
        p.inst = (uint32_t)f->tick;
        p.seed = c.seed + (uint64_t)i;      // one Philox key per vehicle
        p.warm_theta = (c.warm_start && v.steps > 0) ? warm_in + (size_t)i * nt : nullptr;
        p.own_goal_weights = f->spec[(size_t)i].own_goal_weights;
        p.goal_heading_weight = f->spec[(size_t)i].goal_heading_weight;
        p.goal_speed_weight = f->spec[(size_t)i].goal_speed_weight;
        if (f->prop) {
            p.n_prop = c.n_prop;
            p.prop_mu = f->d_mu + (size_t)j * nt;
            p.prop_log_sigma = f->d_ls + (size_t)j * nt;
        }
        nnp_result &r = res[(size_t)j];
        memset(&r, 0, sizeof r);
        r.theta = warm_out + (size_t)i * nt;
        r.controls = f->d_ctrl + (size_t)j * T * 2;
        r.traj = f->d_traj + (size_t)j * (T + 1) * 4;
        r.cost = f->d_cost + j;
        r.status = f->d_status + j;
    }
    int rc;
    if (f->prop) {
        rc = nnp_proposal_encode(f->prop, probs.data(), na, f->d_enc, s);
        if (!rc) rc = nnp_proposal_forward(f->prop, f->d_enc, na, f->d_mu, f->d_ls, s);
        if (rc) return ffail(f, rc, std::string("proposal: ") + nnp_proposal_last_error(f->prop));
    }
    rc = nnp_plan_batch(f->planner, probs.data(), na, res.data(), s);
    if (rc) return ffail(f, rc, std::string("plan: ") + nnp_last_error(f->planner));
    if (hipMemcpyAsync(f->d_goal, f->h_goal, (size_t)na * 4 * sizeof(float),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return ffail(f, NNP_EDEVICE, "goal copy failed");
    const FleetEps eps{c.eps_xi, c.eps_eta, c.eps_phi, c.eps_v};
    hipLaunchKernelGGL(fleet_status_kernel, dim3(na), dim3(64), 0, s, na, c.T, f->d_traj,
                       f->d_ctrl, f->d_cost, f->d_status, f->d_goal, eps, f->d_rec);
    if (hipMemcpyAsync(f->h_rec, f->d_rec, (size_t)na * sizeof(StatusRec), hipMemcpyDeviceToHost,
                       s) != hipSuccess)
        return ffail(f, NNP_EDEVICE, "status copy failed");
    if (f->n_points > 0)
        hipLaunchKernelGGL(advance_obstacles_kernel, dim3((unsigned)((f->n_points + 255) / 256)),
                           dim3(256), 0, s, f->d_obst, f->n_points, c.dt);
    if (hipGetLastError() != hipSuccess) return ffail(f, NNP_EDEVICE, "kernel launch failed");
    if (hipStreamSynchronize(s) != hipSuccess) return ffail(f, NNP_EDEVICE, "stream sync failed");
    for (int j = 0; j < na; ++j) {
        const int i = act[(size_t)j];
        nnp_vehicle_state &v = f->st[(size_t)i];
        const StatusRec &r = f->h_rec[j];
        memcpy(v.z, r.z, sizeof v.z);
        v.a[0] = r.a[0];
        v.a[1] = r.a[1];
        v.cost = r.cost;
        v.steps += 1;
        if (r.status == NNP_INFEASIBLE) v.infeasible_steps += 1;
        const bool last = v.waypoint + 1 >= (int)(f->wps[(size_t)i].size() / 4);
        const bool passed = c.switch_rule == NNP_SWITCH_PLAN && !last ? r.plan_reached != 0
                                                                      : r.reached != 0;
        if (passed) {
            v.waypoint += 1;
            if (last) v.done = 1;
        }
    }
    f->parity ^= 1;
    f->tick += 1;
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                t0).count();
    f->err.clear();
    return NNP_OK;
}

int nnp_fleet_state(const nnp_fleet *f, nnp_vehicle_state *states)
{
    if (!f || !states) return NNP_EINVAL;
    memcpy(states, f->st.data(), f->st.size() * sizeof(nnp_vehicle_state));
    return NNP_OK;
}

const char *nnp_fleet_last_error(const nnp_fleet *f)
{
    return f ? f->err.c_str() : g_fleet_error.c_str();
}

}  // extern "C"
