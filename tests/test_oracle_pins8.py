"""Pins of the oracle's 8-state vehicle (the Simulation Study's single-track model with wheel
speeds, Pacejka tires and the friction ellipse, in the road-aligned frame), against closed forms,
invariants, geometry and brute force.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_00494_amd import workloads as W


def _prob(**kw):
    return W.vehicle8_problem(**kw)


# ---- tires ---------------------------------------------------------------------------------
def test_magic_formula_small_slip_slope_is_BCD():
    """d/dz D sin(C atan(Bz - E(Bz - atan Bz))) at 0 = B C D: the small-slip limit is the
    linear tire with stiffness mu Fz B C D."""
    prob = _prob(pac_B=8.0, pac_C=1.6, pac_D=0.9, pac_E=0.5)
    z = 1e-7
    slope = (oracle.magic8(prob, z) - oracle.magic8(prob, -z)) / (2 * z)
    assert slope == pytest.approx(8.0 * 1.6 * 0.9, rel=1e-8)
    Fz = 120.0
    F = oracle.tire8(prob, Fz, 0.0, 1e-6)
    assert F[1] == pytest.approx(prob["mu"] * Fz * 8.0 * 1.6 * 0.9 * 1e-6, rel=1e-6)


def test_magic_formula_is_odd_and_peaks_at_D():
    prob = _prob()
    zs = np.linspace(0.0, 1.0, 1001)
    f = np.array([oracle.magic8(prob, z) for z in zs])
    g = np.array([oracle.magic8(prob, -z) for z in zs])
    assert np.array_equal(g, -f)                             # odd, bit for bit
    fine = np.linspace(0.0, 0.6, 60001)
    peak = max(oracle.magic8(prob, z) for z in fine)
    assert peak == pytest.approx(prob["pac_D"], abs=1e-7)    # C > 1: the sine reaches 1
    assert oracle.magic8(prob, 0.0) == 0.0


def test_friction_ellipse_bounds_the_combined_force():
    prob = _prob()
    rng = np.random.default_rng(3)
    for _ in range(2000):
        Fz = rng.uniform(10, 200)
        slip, alpha = rng.uniform(-1, 1), rng.uniform(-0.8, 0.8)
        F = oracle.tire8(prob, Fz, slip, alpha)
        fmax = prob["mu"] * prob["pac_D"] * Fz
        assert (F[0] / fmax) ** 2 + (F[1] / fmax) ** 2 <= 1.0 + 1e-12
        # odd symmetry of the combined tire
        G = oracle.tire8(prob, Fz, -slip, -alpha)
        assert np.array_equal(G, -F)
    # either pure-slip case is reproduced exactly
    Fz = 100.0
    assert oracle.tire8(prob, Fz, 0.0, 0.2)[1] == prob["mu"] * Fz * oracle.magic8(prob, 0.2)
    assert oracle.tire8(prob, Fz, 0.0, 0.2)[0] == 0.0
    assert oracle.tire8(prob, Fz, 0.1, 0.0)[0] == prob["mu"] * Fz * oracle.magic8(prob, 0.1)
    assert oracle.tire8(prob, Fz, 0.1, 0.0)[1] == 0.0


# ---- vehicle and road frame ------------------------------------------------------------------
def test_rolling_straight_is_an_equilibrium():
    """Straight track (kappa = 0), no steering, no throttle, rolling wheels: no slip, no force,
    so one period keeps every velocity and advances s by vX dt exactly."""
    prob = _prob(track_len=math.inf, kappa_amp=0.0)
    vX = 5.0
    w = vX / prob["Rw"]
    x = np.array([vX, 0.0, 0.0, w, w, 0.0, 0.0, 7.0])
    xn = oracle.model_step8(prob, x, [0.0, 0.0])
    assert np.array_equal(xn[:7], x[:7])
    assert xn[7] == pytest.approx(7.0 + vX * prob["dt"], rel=1e-15)


def test_wheel_spin_decays_and_conserves_momentum():
    """Rear wheel spinning 20 % fast, no throttle, straight: the tire force moves momentum between
    the wheels and the body, m vX + (Iw / Rw)(wF + wR) is conserved (the midpoint rule keeps
    linear invariants), and the wheels end rolling (Rw w = vX)."""
    prob = _prob(track_len=math.inf, kappa_amp=0.0)
    vX, Rw, Iw, m = 5.0, prob["Rw"], prob["Iw"], prob["m"]
    x = np.array([vX, 0.0, 0.0, vX / Rw, 1.2 * vX / Rw, 0.0, 0.0, 0.0])
    inv0 = m * x[0] + Iw / Rw * (x[3] + x[4])
    for _ in range(400):
        x = oracle.model_step8(prob, x, [0.0, 0.0])
    inv = m * x[0] + Iw / Rw * (x[3] + x[4])
    assert inv == pytest.approx(inv0, rel=1e-12)
    assert x[0] > vX                                        # the spinning wheel pushed the car
    assert abs(Rw * x[4] - x[0]) / x[0] < 1e-6
    assert abs(Rw * x[3] - x[0]) / x[0] < 1e-6


def test_road_frame_kinematics_match_global_geometry():
    """No tire forces (mu = 0): the body velocities are constant and the car moves on a straight
    line in the plane.  On a circular track of radius R = L / (2 pi) (no curvature variation),
    its road-frame coordinates follow from plane geometry: with the centre at the origin and the
    path starting at (R, 0) heading +Y (counter-clockwise, eY positive towards the centre),
    s = R theta, eY = R - |p|, epsi = psi - (theta + pi / 2)."""
    L = 60.0
    R = L / (2 * math.pi)
    prob = _prob(mu=0.0, track_len=L, kappa_amp=0.0, n_sub=200)
    vX, vY, eY0, epsi0 = 5.0, 0.4, 0.3, 0.2
    x = np.array([vX, vY, 0.0, 0.0, 0.0, epsi0, eY0, 0.0])
    psi = math.pi / 2 + epsi0
    p0 = np.array([R - eY0, 0.0])
    vel = np.array([vX * math.cos(psi) - vY * math.sin(psi), vX * math.sin(psi) + vY * math.cos(psi)])
    worst = 0.0
    for n in range(1, 21):
        x = oracle.model_step8(prob, x, [0.0, 0.0])
        p = p0 + vel * n * prob["dt"]
        theta = math.atan2(p[1], p[0])
        want = np.array([R * theta, R - np.hypot(*p), psi - (theta + math.pi / 2)])
        got = np.array([x[7], x[6], x[5]])
        worst = max(worst, float(np.max(np.abs(got - want))))
    assert worst < 1e-6, worst


def test_kappa_profile_turns_once_per_lap():
    prob = _prob()
    L = prob["track_len"]
    s = np.linspace(0.0, L, 200001)
    k = np.array([oracle.kappa8(prob, v) for v in s])
    turn = float(np.sum(0.5 * (k[1:] + k[:-1]) * np.diff(s)))
    assert turn == pytest.approx(2 * math.pi, rel=1e-9)
    assert min(k) == pytest.approx(2 * math.pi / L * (1 - prob["kappa_amp"]), rel=1e-6)


# ---- belief, barrier, cost -------------------------------------------------------------------
def test_record_barrier_and_cost_closed_forms():
    prob = _prob()
    rng = np.random.default_rng(4)
    part = rng.normal(size=(7, 8))
    rec = oracle.moments8(part)
    assert np.allclose(rec[:8], part.mean(axis=0), atol=1e-15)
    assert rec[8] == pytest.approx(np.var(part[:, 6], ddof=1), rel=1e-13)
    assert oracle.moments8(part[:1])[8] == 0.0
    nu = oracle.backoff(prob["delta"])
    rec = np.array([5.5, 0.1, 0.2, 50.0, 51.0, 0.05, 0.7, 12.0, 0.09])
    wT = prob["half_width"]
    assert oracle.barrier8(prob, nu, rec) == pytest.approx((wT - nu * 0.3) ** 2 - 0.49, rel=1e-14)
    q = (5.5 - 6.0) ** 2 + 1.0 * 0.05 ** 2 + 0.1 * 0.49
    assert oracle.stage_cost8(prob, rec) == pytest.approx(q, rel=1e-14)
    out = rec.copy()
    out[6] = -2.0
    assert oracle.stage_cost8(prob, out) == pytest.approx((5.5 - 6) ** 2 + 0.0025 + 0.4 + 1000.0)


def test_repair8_steers_back_toward_the_centerline():
    """Near the left edge (eY = 1.7 m) heading further left: the condition is violated for u = 0,
    and one damped Gauss-Newton step steers right (negative) and lowers the one-step residual
    (the residual is not monotone in the steering once the front tire passes its force peak, so
    later steps may bounce; one step is the pinned behaviour)."""
    prob = _prob(shield_iters=1, gamma=0.05, kappa_amp=0.0, track_len=math.inf)
    nu = oracle.backoff(prob["delta"])
    w = 5.5 / prob["Rw"]
    rec = np.array([5.5, 0.0, 0.0, w, w, 0.15, 1.7, 0.0, 1e-3])

    def resid(u):
        xn = oracle.model_step8(prob, rec[:8], u)
        return -oracle.barrier8(prob, nu, np.concatenate([xn, [rec[8]]])) + \
            (1 - prob["gamma"]) * oracle.barrier8(prob, nu, rec)
    assert resid([0.0, 0.0]) > 0
    u = oracle.repair8(prob, nu, rec, [0.0, 0.0])
    assert u[0] < 0.0 and resid(u) < resid([0.0, 0.0])
    assert oracle.repair8(dict(prob, shield_iters=0), nu, rec, [0.0, 0.0]).tolist() == [0.0, 0.0]


# ---- solves ------------------------------------------------------------------------------------
def test_zero_noise_solve8_is_deterministic_integration():
    prob = _prob(K=5, M=8, T=6, sigma_eps=[0.0, 0.0], sigma_w=[0.0, 0.0, 0.0])
    x0 = W.vehicle8_start(prob, np.random.default_rng(1))
    v = np.column_stack([0.05 * np.ones(6), 0.3 * np.sin(np.arange(6))])
    r = oracle.solve8(prob, 3, x0, v, nthreads=2)
    x = x0.copy()
    for t in range(6):
        x = oracle.model_step8(prob, x, np.clip(v[t], [-0.4, -1], [0.4, 1]))
        for k in range(5):
            # the mean of M equal values is the value up to the rounding of the running sum
            assert np.allclose(r["mom"][k, t + 1, :8], x, rtol=8 * 2.0 ** -52, atol=0)
            assert abs(r["mom"][k, t + 1, 8]) <= 1e-28
    assert np.all(r["S"] == r["S"][0])
    assert np.array_equal(r["v"], v)


def test_brute_force_tiny_solve8():
    """K = 2, M = 5, T = 2: a literal evaluator that stores every particle (normals from the
    Philox blocks dealt three per particle from each quad), NumPy moments, the closed-form barrier
    and cost, and unshifted long-double weights agrees with the solve."""
    prob = _prob(K=2, M=5, T=2, C_cbf=50.0, sigma_w=[0.3, 0.3, 0.2])
    K, M, T, s = 2, 5, 2, 9
    x0 = W.vehicle8_start(prob, np.random.default_rng(2))
    v = np.array([[0.04, 0.5], [-0.03, -0.2]])
    nu = oracle.backoff(prob["delta"])
    wT, g = prob["half_width"], prob["gamma"]
    inv_var = 1.0 / np.array(prob["sigma_eps"]) ** 2

    def h(rec):
        return max(wT - nu * math.sqrt(rec[8]), 0.0) ** 2 - rec[6] ** 2

    def q(rec):
        return ((rec[0] - 6.0) ** 2 + prob["q_epsi"] * rec[5] ** 2 + prob["q_ey"] * rec[6] ** 2
                + (prob["C_obs"] if abs(rec[6]) >= wT else 0.0))

    S, U = [], []
    for k in range(K):
        X = np.tile(x0, (M, 1))
        recs = [np.concatenate([x0, [0.0]])]
        u_k = []
        for t in range(T):
            z = oracle.normals(prob["seed"], [t, 0, k, s])
            u = np.clip(v[t] + np.array(prob["sigma_eps"]) * z[:2], [-0.4, -1.0], [0.4, 1.0])
            u_k.append(u)
            Xn = np.zeros_like(X)
            for m in range(M):
                qd, i = divmod(m, 4)
                z12 = np.concatenate([oracle.normals(prob["seed"], [t, 3 * qd + b, k, (1 << 28) | s])
                                      for b in range(3)])
                Xn[m] = oracle.model_step8(prob, X[m], u)
                Xn[m, :3] += np.array(prob["sigma_w"]) * z12[3 * i:3 * i + 3]
            X = Xn
            recs.append(np.concatenate([X.mean(axis=0), [np.var(X[:, 6], ddof=1)]]))
        cost = 0.0
        for t in range(T):
            cost += q(recs[t]) + float(np.dot(v[t] * inv_var, u_k[t]))
            if t > 0:
                cost += prob["C_cbf"] * max(-h(recs[t]) + (1 - g) * h(recs[t - 1]), 0.0)
        cost += q(recs[T]) + prob["C_cbf"] * max(-h(recs[T]) + (1 - g) * h(recs[T - 1]), 0.0)
        S.append(cost)
        U.append(np.array(u_k))
    r = oracle.solve8(prob, s, x0, v, nthreads=1)
    assert np.allclose(r["S"], S, rtol=1e-12, atol=0)
    w = np.array([np.exp(np.longdouble(-c / prob["lambda"])) for c in S])
    vplus = v + sum(w[k] * (U[k] - v) for k in range(K)) / w.sum()
    assert np.allclose(r["v"], vplus.astype(np.float64), rtol=0, atol=1e-13)


def test_paper_size_solve8_runs_and_is_deterministic():
    prob, x0, v = W.config_vehicle8()
    a = oracle.solve8(prob, 0, x0, v, nthreads=8)
    b = oracle.solve8(prob, 0, x0, v, nthreads=3)
    assert a["status"] == 0 and np.all(np.isfinite(a["S"]))
    assert np.array_equal(a["v"], b["v"]) and np.array_equal(a["S"], b["S"])
    assert a["stats"][2] > 2.0                           # the weights are not degenerate


# ---- integration -----------------------------------------------------------------------------
def test_substeps_converge_at_second_order_to_an_independent_ode_solution():
    """The period step is n_sub explicit-midpoint substeps of the vector field.  Against SciPy's
    adaptive Runge-Kutta solution of the same field (tolerances 1e-13), the error of one period
    falls by about four per doubling of n_sub (second order: a first-order slip, e.g. the
    endpoint slope in place of the midpoint's, would give two), and a fine subdivision agrees
    with the independent solution."""
    from scipy.integrate import solve_ivp
    prob = _prob()   # the 0.05 s period
    x0 = np.array([5.0, 0.3, 0.5, 55.0, 60.0, 0.1, 0.5, 10.0])
    u = np.array([0.15, 0.4])
    sol = solve_ivp(lambda t, x: oracle.deriv8(prob, x, u), (0.0, prob["dt"]), x0,
                    method="DOP853", rtol=1e-13, atol=1e-13)
    ref = sol.y[:, -1]
    errs = [float(np.max(np.abs(oracle.model_step8(dict(prob, n_sub=n), x0, u) - ref)))
            for n in (4, 8, 16, 32)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.3 < r < 4.7 for r in ratios), (errs, ratios)
    fine = oracle.model_step8(dict(prob, n_sub=1024), x0, u)
    assert np.max(np.abs(fine - ref)) < 1e-6
