"""Closed-loop harness for the shielded workload (test infrastructure).

A controller runs the receding-horizon loop of Alg. 1 on the synthetic ellipse track: at closed-loop
step n it solves from the plant state (solve index n), applies v+_0 to the plant and shifts its warm
start.  The plant is the double-precision single-track car of the oracle plus a disturbance on
(vx, vy, r) of standard deviation sigma_w drawn from Philox4x32-10 with tag 3: counter
(n, 0, 0, 3 << 28) under the problem's seed, normals z0, z1 and z2 of that block.  The same plant
serves every controller, so only the controller differs between runs.

Episode rules: a crash (|e_y| > w_T after a plant step) ends the episode; a new start pose is drawn
(arc length uniform along the track from generator seed (plant seed, episode)) and the warm start
is reset to zero, until the step budget is used.  Statistics per run:
  crashes            episodes ended by a crash,
  collision_steps    plant steps with |e_y| > 0.9 w_T (the paper's collision/crash ratio of the
                     deviation thresholds),
  dcbf_ok / dcbf_n   plant steps satisfying the discrete barrier condition
                     h(x_{n+1}) >= (1 - gamma) h(x_n) with h = w_T^2 - e_y^2 on the realised states
                     (the plant state is known exactly, so the belief's covariance term vanishes),
  half_width_steps   plant steps with |e_y| > 0.5 w_T,
  sum_abs_ey, sum_ey2, max_abs_ey, sum_vx   sums for the mean / RMS / maximum lateral deviation
                     and the mean speed over the plant steps.
"""
import math

import numpy as np

import oracle
from paper_2408_00494_amd import workloads as W

PLANT_TAG = 3


def plant_noise(seed, n):
    ctr = np.array([n & 0xFFFFFFFF, 0, 0, PLANT_TAG << 28], dtype=np.uint32)
    return oracle.normals(seed, ctr)[:3]


def lateral_deviation(prob, x):
    return oracle.ellipse_sdf(prob["ell_a"], prob["ell_b"], x[0], x[1])[0]


def start_pose(prob, episode):
    rng = np.random.default_rng([int(prob["seed"]), int(episode)])
    return W.random_start(prob["ell_a"], prob["ell_b"], rng)


class OracleController:
    def __init__(self, prob, nthreads):
        self.prob, self.nthreads = prob, nthreads
        self.reset()

    def reset(self):
        self.v = np.zeros((self.prob["T"], 2))

    def act(self, x, n):
        r = oracle.solve(self.prob, n, x, self.v, want_traces=False, nthreads=self.nthreads)
        self.v = oracle.step_shift(r["v"])
        return np.array(r["v"][0])


def window_stats(series, wT, begin, end):
    """Aggregate statistics of steps [begin, end) from the per-step series of a run."""
    ey = np.abs(np.asarray(series["ey"][begin:end]))
    return {"steps": int(ey.size), "crashes": int(np.sum(series["crash"][begin:end])),
            "collision_steps": int(np.sum(ey > 0.9 * wT)),
            "half_width_steps": int(np.sum(ey > 0.5 * wT)),
            "dcbf_ok": int(np.sum(series["dcbf"][begin:end])), "dcbf_n": int(ey.size),
            "sum_abs_ey": float(np.sum(ey)), "sum_vx": float(np.sum(series["vx"][begin:end]))}


def run(prob, steps, controller, record=False, keep_series=False):
    """Closed loop of `steps` plant steps; returns (stats dict, records).  records (if asked) hold
    (n, x_n, warm start used at n, u0) for every step; stats["series"] (with record or
    keep_series) holds the per-step e_y, crash flag, barrier flag and vx."""
    wT, gamma = prob["half_width"], prob["gamma"]
    sw = np.asarray(prob["sigma_w"], dtype=np.float64)
    st = {"steps": 0, "crashes": 0, "collision_steps": 0, "dcbf_ok": 0, "dcbf_n": 0,
          "episodes": 1, "half_width_steps": 0, "sum_abs_ey": 0.0, "sum_ey2": 0.0,
          "max_abs_ey": 0.0, "sum_vx": 0.0}
    episode = 0
    x = start_pose(prob, episode)
    controller.reset()
    h_prev = wT * wT - lateral_deviation(prob, x) ** 2
    recs = []
    series = {"ey": [], "crash": [], "dcbf": [], "vx": []}
    for n in range(steps):
        v_used = controller.warm_start() if record and hasattr(controller, "warm_start") else None
        u0 = controller.act(x, n)
        xn = oracle.model_step(prob, x, u0)
        xn[3:] += sw * plant_noise(prob["seed"], n)
        ey = lateral_deviation(prob, xn)
        h = wT * wT - ey * ey
        st["steps"] += 1
        st["dcbf_n"] += 1
        st["dcbf_ok"] += int(h >= (1.0 - gamma) * h_prev)
        st["collision_steps"] += int(abs(ey) > 0.9 * wT)
        st["half_width_steps"] += int(abs(ey) > 0.5 * wT)
        st["sum_abs_ey"] += abs(ey)
        st["sum_ey2"] += ey * ey
        st["max_abs_ey"] = max(st["max_abs_ey"], abs(ey))
        st["sum_vx"] += xn[3]
        crash = not math.isfinite(ey) or abs(ey) > wT
        series["ey"].append(float(ey))
        series["crash"].append(int(crash))
        series["dcbf"].append(int(h >= (1.0 - gamma) * h_prev))
        series["vx"].append(float(xn[3]))
        if record:
            recs.append((n, x.copy(), v_used, np.array(u0)))
        if crash:
            st["crashes"] += 1
            episode += 1
            st["episodes"] += 1
            x = start_pose(prob, episode)
            controller.reset()
            h_prev = wT * wT - lateral_deviation(prob, x) ** 2
        else:
            x = xn
            h_prev = h
    if record or keep_series:
        st["series"] = series
    return st, recs


COMBOS = [(d, g) for d in (0.01, 0.05, 0.1) for g in (0.1, 0.3)]


def combo_problem(i):
    d, g = COMBOS[i]
    prob, _, _ = W.config_shielded(delta=d, gamma=g, seed=3000 + i)
    return prob
