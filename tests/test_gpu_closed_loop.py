"""Shielded closed loop (K=8192, M=128, T=60, two repair iterations) for every (delta, gamma)
combination: 1000 receding-horizon steps of the GPU controller on the FP64 plant.

* Lockstep replay: at sampled steps the oracle solves from the GPU run's own plant state, warm
  start and solve index; its command must meet the control bar (max |du| / u_max <= 1e-4).
* Rates: single- and double-precision closed loops diverge (the dynamics are chaotic at the
  scale of rounding), so the GPU run's statistics are compared with the oracle controller's
  (tests/golden/closed_loop_oracle.json) as distributions: two-proportion z-tests at z = 4 for the
  crash, collision, half-width and barrier rates, and the mean |e_y| and mean speed within
  stated relative bounds.
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

NTHREADS = min(16, os.cpu_count() or 1)
STEPS = 1000
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


def _two_prop_ok(k1, n1, k2, n2, z=4.0):
    p1, p2 = k1 / n1, k2 / n2
    p = (k1 + k2) / (n1 + n2)
    se = math.sqrt(max(p * (1 - p), 1e-12) * (1 / n1 + 1 / n2))
    return abs(p1 - p2) <= z * se + 1e-12


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
    print(f"GPU closed loop delta={d} gamma={g}: {st}", flush=True)
    rng = np.random.default_rng(100 + i)
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    for n in (1, int(rng.integers(2, STEPS))):
        _, x, v_used, u0 = recs[n]
        ref = oracle.solve(prob, n, x, v_used, want_traces=False, nthreads=NTHREADS)
        err = float(np.max(np.abs(u0 - ref["v"][0]) / scale))
        print(f"  step {n}: |du|/u_max = {err:.2e}", flush=True)
        assert err <= 1e-4


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle closed-loop statistics missing")
@pytest.mark.parametrize("i", range(len(CL.COMBOS)))
def test_rates_match_oracle_controller(i):
    prob, st, _ = _gpu_run(i)
    with open(GOLDEN) as fh:
        gold = json.load(fh)
    ref = [c for c in gold["combos"] if c["seed"] == prob["seed"]]
    if not ref:
        pytest.skip("combination not in the stored statistics")
    ref = ref[0]
    n1, n2 = st["steps"], ref["steps"]
    for key in ("crashes", "collision_steps", "half_width_steps"):
        assert _two_prop_ok(st[key], n1, ref[key], n2), key
    assert _two_prop_ok(st["dcbf_ok"], st["dcbf_n"], ref["dcbf_ok"], ref["dcbf_n"])
    m1, m2 = st["sum_abs_ey"] / n1, ref["sum_abs_ey"] / n2
    assert abs(m1 - m2) <= 0.3 * m2 + 0.02, (m1, m2)
    s1, s2 = st["sum_vx"] / n1, ref["sum_vx"] / n2
    assert abs(s1 - s2) <= 0.05 * s2, (s1, s2)
    print(f"delta={ref['delta']} gamma={ref['gamma']}: mean|e_y| GPU {m1:.4f} oracle {m2:.4f}, "
          f"mean vx GPU {s1:.3f} oracle {s2:.3f}", flush=True)
