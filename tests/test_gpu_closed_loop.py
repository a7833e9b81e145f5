"""Shielded closed loop (K=8192, M=128, T=60, two repair iterations) for every (delta, gamma)
combination: 1000 receding-horizon steps of the GPU controller on the FP64 plant.

* Lockstep replay: at 25 evenly spaced steps the oracle solves from the GPU run's own plant
  state, warm start and solve index; its command must meet the control bar
  (max |du| / u_max <= 1e-4), or, at a step where the shield's feedback makes the command itself
  that sensitive, stay within twice the oracle's own drift when its estimate moves by ~1e-6
  (tests/sensitivity.py).
* Rates: the oracle controller's statistics and per-step series
  (tests/golden/closed_loop_oracle.json) cover the first 250 or 1000 steps of each combination
  (each entry records its own); the GPU run's same window (same start, same plant noise) is
  compared with them.  Single- and double-precision closed
  loops drift apart (the dynamics amplify rounding), so the two runs are two realisations of the
  same closed loop, and consecutive steps are strongly correlated: the standard error of each
  difference comes from batch means (10 batches of 25 steps) of both series,
  sqrt(se_gpu^2 + se_oracle^2), and the difference of the half-width and collision fractions,
  the barrier-condition fraction, the mean |e_y| and the mean speed must lie within 4 of them
  (plus a small floor); crash counts must agree within 2.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import closed_loop as CL

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2408_00494_amd as bss  # noqa: E402
import sensitivity as SENS  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)
STEPS = 1000
LOCKSTEP = 25
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "closed_loop_oracle.json")


class GpuController:
    def __init__(self, prob):
        self.T = prob["T"]
        self.s = bss.Solver(prob)
        self.s.set_outputs(controls=False)

    def reset(self):
        self.s.set_controls(np.zeros((self.T, 2)))

    def warm_start(self):
        return self.s.get_controls()

    def act(self, x, n):
        self.s.solve_index = n
        u0, _ = self.s.solve(x)
        self.s.step_shift()
        return u0

    def close(self):
        self.s.close()


def _batch_se(x, nb=10):
    x = np.asarray(x, dtype=np.float64)
    m = x.size // nb
    means = x[:m * nb].reshape(nb, m).mean(axis=1)
    return float(means.std(ddof=1) / np.sqrt(nb))


_runs = {}


def _gpu_run(i):
    if i not in _runs:
        prob = CL.combo_problem(i)
        ctl = GpuController(prob)
        st, recs = CL.run(prob, STEPS, ctl, record=True)
        ctl.close()
        _runs[i] = (prob, st, recs)
    return _runs[i]


@pytest.mark.parametrize("i", range(len(CL.COMBOS)))
def test_lockstep_replay_against_oracle(i):
    prob, st, recs = _gpu_run(i)
    d, g = CL.COMBOS[i]
    shown = {key: val for key, val in st.items() if key != "series"}
    print(f"GPU closed loop delta={d} gamma={g}: {shown}", flush=True)
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    worst, sensitive = 0.0, 0
    for n in range(1, STEPS, STEPS // LOCKSTEP):
        _, x, v_used, u0 = recs[n]
        ref = oracle.solve(prob, n, x, v_used, want_traces=False, nthreads=NTHREADS)
        err = float(np.max(np.abs(u0 - ref["v"][0]) / scale))
        worst = max(worst, err)
        if err > 1e-4:
            own = 0.0
            for sign in (1.0, -1.0):
                moved = oracle.solve(prob, n, x + sign * SENS.DX, v_used, want_traces=False,
                                     nthreads=NTHREADS)
                own = max(own, float(np.max(np.abs(moved["v"][0] - ref["v"][0]) / scale)))
            print(f"  step {n}: |du|/u_max = {err:.2e}, oracle against itself {own:.2e}",
                  flush=True)
            assert err <= 2.0 * own
            sensitive += 1
    print(f"  {LOCKSTEP} lockstep steps: worst |du|/u_max = {worst:.2e} ({sensitive} past 1e-4 "
          f"within the oracle's own drift)", flush=True)


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle closed-loop statistics missing")
@pytest.mark.parametrize("i", range(len(CL.COMBOS)))
def test_rates_match_oracle_controller(i):
    prob, _, _ = _gpu_run(i)
    series = _runs[i][1]["series"]
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    ref = [c for c in gold["combos"] if c["seed"] == prob["seed"] and "series" in c]
    if not ref:
        pytest.skip("combination not in the stored statistics")
    ref = ref[0]
    n = ref["steps"]
    wT = prob["half_width"]
    st = CL.window_stats(series, wT, 0, n)
    ey = np.abs(np.asarray(series["ey"][:n]))
    ey_ref = np.abs(np.asarray(ref["series"]["ey"][:n]))

    def bound(x, y, floor):
        return 4.0 * math.hypot(_batch_se(x), _batch_se(y)) + floor

    # fractions of steps beyond half the track half-width and beyond the collision threshold
    for key, thr in (("half_width_steps", 0.5), ("collision_steps", 0.9)):
        b = bound(ey > thr * wT, ey_ref > thr * wT, 0.02)
        assert abs(st[key] - ref[key]) / n <= b, (key, st[key], ref[key], b)
    assert abs(st["crashes"] - ref["crashes"]) <= 2
    b = bound(series["dcbf"][:n], ref["series"]["dcbf"][:n], 0.02)
    assert abs(st["dcbf_ok"] - ref["dcbf_ok"]) / n <= b
    m1, m2 = st["sum_abs_ey"] / n, ref["sum_abs_ey"] / n
    assert abs(m1 - m2) <= bound(ey, ey_ref, 0.02), (m1, m2)
    s1, s2 = st["sum_vx"] / n, ref["sum_vx"] / n
    assert abs(s1 - s2) <= bound(series["vx"][:n], ref["series"]["vx"][:n], 0.05), (s1, s2)
    print(f"delta={ref['delta']} gamma={ref['gamma']} first {n} steps: half-width steps GPU "
          f"{st['half_width_steps']} oracle {ref['half_width_steps']}, mean|e_y| GPU {m1:.4f} "
          f"oracle {m2:.4f}, mean vx GPU {s1:.3f} oracle {s2:.3f}", flush=True)
