"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test checks an oracle function against something other than itself: published known-answer
values, a library routine, a closed form, an invariant, a special case that reduces to a textbook
result, or brute force.  See the module docstring of each group for what a mistake would break.
"""
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import special, stats

import oracle
from paper_2408_00494_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ================================== random numbers ==========================================
def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers():
    """Random123's published known-answer vectors for Philox4x32-10 (Salmon et al., SC'11)."""
    for row in _kat_rows():
        out = oracle.philox(row[:4], row[4:6])
        assert [int(x) for x in out] == row[6:]


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_engine():
    """Bit-exact agreement with rocRAND's Philox4x32-10 engine (independent implementation,
    compiled from the installed header) on counters of the shape the solver uses."""
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rocrand_philox_ref.cpp")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "ref")
        subprocess.run(["hipcc", "-O1", "-o", exe, src], check=True, cwd=tmp,
                       capture_output=True)
        rng = np.random.default_rng(7)
        cases = []
        for i in range(300):
            seed = int(rng.integers(0, 2**63))
            c0 = int(rng.integers(0, 200))                 # time step
            c1 = int(rng.integers(0, 300))                 # particle
            c2 = int(rng.integers(0, 9000))                # sample
            c3 = (int(rng.integers(0, 3)) << 28) | int(rng.integers(0, 2**28))  # tag | solve
            cases.append((seed, c0, c1, c2, c3))
        inp = "".join(f"{s} {a} {b} {c} {d}\n" for s, a, b, c, d in cases)
        res = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
        lines = res.stdout.strip().splitlines()
        assert len(lines) == len(cases)
        for (seed, c0, c1, c2, c3), line in zip(cases, lines):
            want = [int(x) for x in line.split()]
            got = oracle.philox([c0, c1, c2, c3], [seed & 0xFFFFFFFF, seed >> 32])
            assert [int(x) for x in got] == want


def test_uniform_exact_and_open_interval():
    """u = ((r >> 9) + 1/2) 2^-23 lies in (0, 1) and is exact in float32 (both sides can form it
    without rounding)."""
    rs = [0, 1, 511, 512, 2**31, 2**32 - 1] + list(np.random.default_rng(1).integers(0, 2**32, 1000))
    for r in rs:
        u = oracle.uniform(int(r))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        assert u == ((int(r) >> 9) + 0.5) / 2**23
    assert oracle.uniform(0) == 2.0**-24
    assert oracle.uniform(2**32 - 1) == 1.0 - 2.0**-24


def test_box_muller_is_standard_normal():
    """Box-Muller pairs from Philox blocks: mean 0, variance 1, uncorrelated pairs, and a
    Kolmogorov-Smirnov test against N(0, 1).  A wrong 2 pi, a missing factor -2 or a reused
    uniform fails this."""
    n = 20000
    z = np.empty((n, 4))
    for i in range(n):
        z[i] = oracle.normals(12345, [i % 97, i // 97, 3, (1 << 28) | 5])
    for j in range(4):
        col = z[:, j]
        assert abs(col.mean()) < 5.0 / math.sqrt(n)
        assert abs(col.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
        assert stats.kstest(col, "norm").pvalue > 1e-4
    for a, b in ((0, 1), (2, 3), (0, 2)):
        assert abs(np.corrcoef(z[:, a], z[:, b])[0, 1]) < 5.0 / math.sqrt(n)
    # tails are bounded by the smallest uniform 2^-24
    assert np.abs(z).max() <= math.sqrt(-2.0 * math.log(2.0**-24)) + 1e-12


# ================================== back-off coefficient =====================================
def test_backoff_textbook_values():
    """Remark 1: Gaussian nu = Phi^-1(1 - delta) (standard normal quantiles), Cantelli
    nu = sqrt((1 - delta)/delta)."""
    with open(os.path.join(GOLDEN, "backoff_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            kind, d, nu = line.split()
            got = oracle.backoff(float(d), 0 if kind == "gaussian" else 1)
            assert got == pytest.approx(float(nu), rel=1e-12, abs=1e-12)


def test_backoff_matches_library_quantile():
    for d in (1e-6, 1e-3, 0.01, 0.05, 0.1, 0.2, 0.4, 0.49):
        assert oracle.backoff(d, 0) == pytest.approx(-special.ndtri(d), rel=1e-12)
        assert oracle.backoff(d, 0) == pytest.approx(math.sqrt(2) * special.erfcinv(2 * d),
                                                     rel=1e-12)
        if d >= 1e-3:
            assert oracle.backoff(d, 0) == pytest.approx(
                math.sqrt(2) * special.erfinv(1 - 2 * d), rel=1e-10)


# ======================================= track geometry ======================================
def test_sdf_circle_closed_form():
    """a = b = R: signed distance |p| - R and normal p / |p|."""
    R = 25.0
    rng = np.random.default_rng(3)
    for _ in range(500):
        p = rng.uniform(-40, 40, size=2)
        if np.hypot(*p) < 1e-3:
            continue
        sd, n = oracle.ellipse_sdf(R, R, p[0], p[1])
        assert sd == pytest.approx(np.hypot(*p) - R, abs=1e-12)
        assert n == pytest.approx(p / np.hypot(*p), abs=1e-12)


@pytest.mark.parametrize("a,b", [(30.0, 20.0), (20.0, 30.0), (50.0, 15.0)])
def test_sdf_vertices(a, b):
    """Points on the axes beyond/inside the vertices within the curvature radius: the distance is
    the offset along the axis and the normal is the axis direction."""
    for d in (-2.5, -1.0, -0.1, 0.0, 0.1, 1.0, 2.5):
        for sx in (1, -1):
            sd, n = oracle.ellipse_sdf(a, b, sx * (a + d), 0.0)
            assert sd == pytest.approx(d, abs=1e-12)
            assert n == pytest.approx([sx, 0.0], abs=1e-12)
            sd, n = oracle.ellipse_sdf(a, b, 0.0, sx * (b + d))
            assert sd == pytest.approx(d, abs=1e-12)
            assert n == pytest.approx([0.0, sx], abs=1e-12)


@pytest.mark.parametrize("a,b", [(30.0, 20.0), (18.0, 47.0)])
def test_sdf_brute_force_and_gradient(a, b):
    """|sd| equals the minimum distance to a dense sampling of the ellipse, the sign is negative
    inside, and n is the finite-difference gradient of sd."""
    th = np.linspace(0.0, 2 * np.pi, 400001)
    cx, cy = a * np.cos(th), b * np.sin(th)
    rng = np.random.default_rng(11)
    for _ in range(60):
        t0 = rng.uniform(0, 2 * np.pi)
        off = rng.uniform(-4.0, 4.0)
        base = np.array([a * np.cos(t0), b * np.sin(t0)])
        nrm = np.array([np.cos(t0) / a, np.sin(t0) / b])
        nrm /= np.hypot(*nrm)
        p = base + off * nrm
        sd, n = oracle.ellipse_sdf(a, b, p[0], p[1])
        dmin = np.min(np.hypot(cx - p[0], cy - p[1]))
        assert abs(sd) == pytest.approx(dmin, abs=2e-7)
        inside = (p[0] / a) ** 2 + (p[1] / b) ** 2 < 1
        assert (sd < 0) == inside
        h = 1e-6
        gx = (oracle.ellipse_sdf(a, b, p[0] + h, p[1])[0] - oracle.ellipse_sdf(a, b, p[0] - h, p[1])[0]) / (2 * h)
        gy = (oracle.ellipse_sdf(a, b, p[0], p[1] + h)[0] - oracle.ellipse_sdf(a, b, p[0], p[1] - h)[0]) / (2 * h)
        assert n == pytest.approx([gx, gy], abs=1e-6)


# ========================================= dynamics ==========================================
def test_rk2_straight_line_is_exact():
    """No steering and no lateral motion with constant acceleration: the midpoint rule
    integrates the quadratic X(t) = X0 + v0 t + a t^2 / 2 exactly."""
    cfg = W.default_problem()
    x = np.array([1.0, 2.0, 0.0, 5.0, 0.0, 0.0])
    a = 1.3
    for i in range(1, 41):
        x = oracle.model_step(cfg, x, [0.0, a])
        t = i * cfg["dt"]
        assert x[0] == pytest.approx(1.0 + 5.0 * t + 0.5 * a * t * t, abs=1e-12)
        assert x[3] == pytest.approx(5.0 + a * t, abs=1e-12)
        assert x[1] == 2.0 and x[2] == 0.0 and x[4] == 0.0 and x[5] == 0.0


def test_rk2_is_midpoint_on_rigid_rotation():
    """Without tire forces and throttle the body velocities obey the linear rotation
    d(vx, vy)/dt = r (vy, -vx); one midpoint step is exactly (I + dt W + dt^2 W^2 / 2) v, and the
    position moves by dt times the midpoint global velocity."""
    cfg = W.default_problem(Cf=0.0, Cr=0.0)
    dt = cfg["dt"]
    x = np.array([3.0, -1.0, 0.4, 6.0, 0.7, 0.9])
    xn = oracle.model_step(cfg, x, [0.0, 0.0])
    r = x[5]
    Wm = np.array([[0.0, r], [-r, 0.0]])
    v = x[3:5]
    vm = v + 0.5 * dt * Wm @ v
    psim = x[2] + 0.5 * dt * r
    assert xn[3:5] == pytest.approx((np.eye(2) + dt * Wm + 0.5 * dt * dt * Wm @ Wm) @ v, abs=1e-13)
    assert xn[2] == pytest.approx(x[2] + dt * r, abs=1e-14)
    gX = vm[0] * math.cos(psim) - vm[1] * math.sin(psim)
    gY = vm[0] * math.sin(psim) + vm[1] * math.cos(psim)
    assert xn[0] == pytest.approx(x[0] + dt * gX, abs=1e-13)
    assert xn[1] == pytest.approx(x[1] + dt * gY, abs=1e-13)
    assert xn[5] == r


def test_lateral_dynamics_match_linear_bicycle_model():
    """At zero slip the Jacobian of (dvy/dt, dr/dt) w.r.t. (vy, r, steer) equals the textbook
    linear single-track (bicycle) model with axle cornering stiffnesses Cf, Cr (e.g. Rajamani,
    Vehicle Dynamics and Control, lateral dynamics in body velocities)."""
    cfg = W.default_problem()
    m, Iz, lf, lr, Cf, Cr = (cfg[k] for k in ("m", "Iz", "lf", "lr", "Cf", "Cr"))
    vx = 10.0
    A = np.array([[-(Cf + Cr) / (m * vx), -vx - (lf * Cf - lr * Cr) / (m * vx)],
                  [-(lf * Cf - lr * Cr) / (Iz * vx), -(lf * lf * Cf + lr * lr * Cr) / (Iz * vx)]])
    B = np.array([Cf / m, lf * Cf / Iz])
    x0 = np.array([0.0, 0.0, 0.3, vx, 0.0, 0.0])
    h = 1e-6
    J = np.zeros((2, 3))
    for j, idx in enumerate((4, 5)):
        xp, xm = x0.copy(), x0.copy()
        xp[idx] += h
        xm[idx] -= h
        J[:, j] = (oracle.car_deriv(cfg, xp, [0, 0])[4:6] - oracle.car_deriv(cfg, xm, [0, 0])[4:6]) / (2 * h)
    J[:, 2] = (oracle.car_deriv(cfg, x0, [h, 0])[4:6] - oracle.car_deriv(cfg, x0, [-h, 0])[4:6]) / (2 * h)
    assert J[:, :2] == pytest.approx(A, rel=1e-6)
    assert J[:, 2] == pytest.approx(B, rel=1e-6)
    # longitudinal: accel enters dvx/dt one-to-one; global velocity is the rotated body velocity
    d = oracle.car_deriv(cfg, np.array([0, 0, 0.3, vx, 0.5, 0.0]), [0.0, 2.0])
    assert d[3] == pytest.approx(2.0, abs=1e-12)
    assert d[0] == pytest.approx(vx * math.cos(0.3) - 0.5 * math.sin(0.3), abs=1e-12)
    assert d[1] == pytest.approx(vx * math.sin(0.3) + 0.5 * math.cos(0.3), abs=1e-12)


def test_friction_saturation_and_mirror_symmetry():
    cfg = W.default_problem()
    m, g, mu, lf, lr = cfg["m"], cfg["g"], cfg["mu"], cfg["lf"], cfg["lr"]
    Ff_max = mu * m * g * lr / (lf + lr)
    d = oracle.car_deriv(cfg, np.array([0, 0, 0, 8.0, 0, 0]), [0.4, 0.0])
    # front force saturated at the static front axle load, rear force zero at zero slip
    assert d[4] == pytest.approx(Ff_max * math.cos(0.4) / m, rel=1e-12)
    assert d[5] == pytest.approx(lf * Ff_max * math.cos(0.4) / cfg["Iz"], rel=1e-12)
    # mirror: (Y, psi, vy, r, steer) -> -(...)
    rng = np.random.default_rng(5)
    for _ in range(50):
        x = rng.normal(size=6) * [5, 5, 1, 1, 0.5, 0.5] + [0, 0, 0, 6, 0, 0]
        u = rng.normal(size=2) * [0.2, 1.0]
        xm = x * [1, -1, -1, 1, -1, -1]
        um = u * [-1, 1]
        a = oracle.model_step(cfg, x, u)
        b = oracle.model_step(cfg, xm, um)
        assert b == pytest.approx(a * [1, -1, -1, 1, -1, -1], abs=1e-12)


# ======================================== moments ============================================
def test_moments_match_library_and_two_particle_form():
    rng = np.random.default_rng(2)
    P = rng.normal(size=(37, 6)) * 3 + 10
    mom = oracle.moments(P)
    assert mom[:6] == pytest.approx(P.mean(axis=0), abs=1e-12)
    C = np.cov(P[:, :2].T, ddof=1)
    assert mom[6:] == pytest.approx([C[0, 0], C[0, 1], C[1, 1]], abs=1e-12)
    P2 = P[:2]
    d = P2[0, :2] - P2[1, :2]
    m2 = oracle.moments(P2)
    assert m2[6:] == pytest.approx([d[0] * d[0] / 2, d[0] * d[1] / 2, d[1] * d[1] / 2], abs=1e-12)
    m1 = oracle.moments(P[:1])
    assert list(m1[6:]) == [0.0, 0.0, 0.0]
    assert m1[:6] == pytest.approx(P[0], abs=0)


def _linear_problem(M, K=1, T=8, sigma_w=(0.3, 0.2, 0.1)):
    dt = 0.1
    A = np.eye(6)
    A[0, 3] = dt          # X += dt vx
    A[1, 4] = dt          # Y += dt vy
    A[2, 5] = dt          # psi += dt r
    A[3, 3] = 0.9
    A[4, 4] = 0.95
    A[4, 5] = 0.1
    A[5, 5] = 0.8
    A[1, 3] = 0.02
    B = np.zeros((6, 2))
    B[3, 1] = dt
    B[5, 0] = 0.5
    cfg = W.default_problem(model=1, K=K, M=M, T=T, sigma_w=list(sigma_w),
                            sigma_eps=[0.0, 0.0])
    cfg["lin_A"] = A
    cfg["lin_B"] = B
    Q = np.diag([0, 0, 0, sigma_w[0] ** 2, sigma_w[1] ** 2, sigma_w[2] ** 2])
    return cfg, A, Q


def test_linear_model_covariance_matches_closed_form():
    """Linear-Gaussian propagation: Sigma_{t+1} = A Sigma_t A^T + Q (the analytic case the paper
    mentions); the Monte-Carlo estimate at M = 2^16 agrees within 5 standard errors."""
    M = 1 << 16
    cfg, A, Q = _linear_problem(M)
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    _, _, mom = oracle.rollout(cfg, 0, 0, x0, np.zeros((cfg["T"], 2)))
    Sig = np.zeros((6, 6))
    mean = x0.copy()
    for t in range(1, cfg["T"] + 1):
        Sig = A @ Sig @ A.T + Q
        mean = A @ mean
        got = mom[t]
        assert np.all(np.abs(got[:6] - mean) <= 5 * np.sqrt(np.diag(Sig) / M) + 1e-10)
        for val, (i, j) in zip(got[6:], ((0, 0), (0, 1), (1, 1))):
            se = math.sqrt((Sig[i, i] * Sig[j, j] + Sig[i, j] ** 2) / (M - 1))
            assert abs(val - Sig[i, j]) <= 5 * se + 1e-15


def test_covariance_estimate_is_unbiased_at_small_M():
    """The 1/(M-1) normalisation: averaged over many independent samples with M = 3 particles,
    the estimate converges to the true covariance (1/M would give 2/3 of it)."""
    K = 4000
    cfg, A, Q = _linear_problem(3, K=K, T=3)
    x0 = np.zeros(6)
    res = oracle.solve(cfg, 0, x0, np.zeros((3, 2)))
    Sig = np.zeros((6, 6))
    for _ in range(3):
        Sig = A @ Sig @ A.T + Q
    est = res["mom"][:, 3, 6:].mean(axis=0)
    want = np.array([Sig[0, 0], Sig[0, 1], Sig[1, 1]])
    sd = res["mom"][:, 3, 6:].std(axis=0) / math.sqrt(K)
    assert np.all(np.abs(est - want) < 5 * sd)


def test_initial_spread_follows_given_covariance():
    """With a state-estimate covariance Sigma_0 the particles start at xbar_0 + L_0 xi; on the
    linear model the position covariance at t = 1 is (A Sigma_0 A^T + Q)_pos (w does not reach
    positions in one step)."""
    M = 1 << 15
    cfg, A, Q = _linear_problem(M, T=1)
    rng = np.random.default_rng(9)
    G = rng.normal(size=(6, 6)) * 0.3
    Sigma0 = G @ G.T + 0.05 * np.eye(6)
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    _, _, mom = oracle.rollout(cfg, 0, 0, x0, np.zeros((1, 2)), Sigma0=Sigma0)
    assert mom[0, 6:] == pytest.approx([Sigma0[0, 0], Sigma0[0, 1], Sigma0[1, 1]], abs=0)
    S1 = A @ Sigma0 @ A.T + Q
    for val, (i, j) in zip(mom[1, 6:], ((0, 0), (0, 1), (1, 1))):
        se = math.sqrt((S1[i, i] * S1[j, j] + S1[i, j] ** 2) / (M - 1))
        assert abs(val - S1[i, j]) <= 5 * se


# ===================================== heuristic and costs ====================================
def test_barrier_closed_forms():
    """h = max(w_T - nu sigma_y, 0)^2 - e_y^2 (eq. 33): with no spread h = w_T^2 - e_y^2; at the
    vertex (a, 0) the normal is the X axis so sigma_y = sqrt(Sigma_xx); past nu sigma_y > w_T
    the margin is clamped at 0."""
    cfg = W.default_problem()
    a, wT = cfg["ell_a"], cfg["half_width"]
    nu = oracle.backoff(cfg["delta"])
    mom = np.array([a + 0.5, 0, 0, 5, 0, 0, 0, 0, 0])
    assert oracle.barrier(cfg, nu, mom) == pytest.approx(wT ** 2 - 0.25, abs=1e-12)
    mom = np.array([a - 0.3, 0, 0, 5, 0, 0, 0.04, 0.01, 0.5])
    assert oracle.barrier(cfg, nu, mom) == pytest.approx((wT - nu * 0.2) ** 2 - 0.09, abs=1e-12)
    mom = np.array([a + 0.3, 0, 0, 5, 0, 0, 4.0, 0.0, 0.0])
    assert oracle.barrier(cfg, nu, mom) == pytest.approx(-0.09, abs=1e-12)


def test_stage_cost_closed_form_and_collision_penalty():
    """q at the vertex (a + e, 0) heading along +Y (the counter-clockwise tangent there):
    q_vx (vx - v_g)^2 + q_vy vy^2 + q_r r^2 + q_ey e^2, zero heading error; turning the heading by
    pi/2 adds q_epsi * 2; crossing |e_y| >= w_T adds C_obs."""
    cfg = W.default_problem(q_vy=0.3, q_r=0.7)
    a = cfg["ell_a"]
    mom = np.array([a + 1.0, 0, math.pi / 2, 4.0, 0.2, -0.1, 0, 0, 0])
    want = 1.0 * 4.0 + 0.3 * 0.04 + 0.7 * 0.01 + 0.1 * 1.0
    assert oracle.stage_cost(cfg, mom) == pytest.approx(want, abs=1e-12)
    mom[2] = math.pi
    assert oracle.stage_cost(cfg, mom) == pytest.approx(want + 2.0, abs=1e-12)
    mom[2] = math.pi / 2
    mom[0] = a + 2.0
    assert oracle.stage_cost(cfg, mom) == pytest.approx(4.0 + 0.012 + 0.007 + 0.4 + 1000.0, abs=1e-9)


def test_score_bookkeeping_small_horizon():
    """Alg. 1's sums with eq. 25: q and the control cost at t = 0..T-1, C_safe on the transitions
    t-1 -> t for t = 1..T (C_safe(z_0) = 0), phi at T.  Checked on injected moments where only one
    transition violates the condition."""
    cfg = W.default_problem(T=2, q_vx=0.0, q_ey=0.0, q_epsi=0.0, C_obs=0.0, gamma_u=2.0)
    nu = oracle.backoff(cfg["delta"])
    a, wT, g, C = cfg["ell_a"], cfg["half_width"], cfg["gamma"], cfg["C_cbf"]
    # e_y = 0, 1.5, 0.5 along the trajectory: h = 4, 1.75, 3.75
    mom = np.zeros((3, 9))
    mom[:, 0] = [a, a + 1.5, a + 0.5]
    h = [wT ** 2, wT ** 2 - 2.25, wT ** 2 - 0.25]
    u = np.array([[0.1, -0.5], [0.2, 0.3]])
    v = np.array([[0.05, 0.4], [-0.1, 1.0]])
    ctrl = 2.0 * sum(v[t, 0] * u[t, 0] / 0.01 + v[t, 1] * u[t, 1] / 1.0 for t in range(2))
    safe = C * max(-h[1] + (1 - g) * h[0], 0) + C * max(-h[2] + (1 - g) * h[1], 0)
    assert C * max(-h[2] + (1 - g) * h[1], 0) == 0.0
    assert oracle.score(cfg, nu, mom, u, v) == pytest.approx(ctrl + safe, abs=1e-10)


# ===================================== rollout invariants =====================================
def test_zero_noise_reduces_to_deterministic_integration():
    """sigma_w = 0 and sigma_eps = 0: all particles coincide, the covariance vanishes, the mean is
    the noise-free integration of v, all costs are equal, weights are 1/K and v+ = v exactly
    (the covariance only up to the rounding of the running sum in the mean, ~ulp(X)^2)."""
    prob, x0, _ = W.config_small()
    prob = dict(prob, sigma_w=[0, 0, 0], sigma_eps=[0, 0], K=16, M=5)
    T = prob["T"]
    v = np.column_stack([0.1 * np.sin(np.arange(T) * 0.3), 0.5 * np.cos(np.arange(T) * 0.2)])
    res = oracle.solve(prob, 3, x0, v)
    x = x0.copy()
    for t in range(T):
        x = oracle.model_step(prob, x, v[t])
        for k in range(prob["K"]):
            assert res["mom"][k, t + 1, :6] == pytest.approx(x, abs=1e-12)
            assert np.all(np.abs(res["mom"][k, t + 1, 6:]) <= 1e-24)
    assert np.all(res["S"] == res["S"][0])
    assert res["stats"][2] == pytest.approx(prob["K"], rel=1e-12)   # ESS = K
    assert np.array_equal(res["v"], v)


def test_results_independent_of_M_without_disturbance():
    prob, x0, v = W.config_small()
    outs = []
    for M in (1, 2, 7, 64):
        res = oracle.solve(dict(prob, sigma_w=[0, 0, 0], M=M, K=32), 0, x0, v)
        outs.append(res)
    for r in outs[1:]:
        assert r["S"] == pytest.approx(outs[0]["S"], rel=1e-12)
        assert r["v"] == pytest.approx(outs[0]["v"], abs=1e-12)


def test_position_covariance_vanishes_at_first_step():
    """With a known initial state, positions at t = 1 depend only on x_0 and u_0 (the disturbance
    enters the velocities), so Sigma_pos(1) = 0 up to the rounding of the mean (~ulp(X)^2),
    while at t = 2 it is of order (dt^2 sigma_w)^2."""
    prob, x0, v = W.config_small()
    res = oracle.solve(dict(prob, K=8), 0, x0, v)
    assert np.all(np.abs(res["mom"][:, 1, 6:]) <= 1e-24)
    assert np.all(res["mom"][:, 2, 6] > 1e-10)


def _plain_mppi(prob, s, x0, v):
    """Independent plain MPPI (deterministic rollouts, eqs. 6-8) for the special case M = 1,
    sigma_w = 0, C_cbf = 0, no repair."""
    K, T, lam = prob["K"], prob["T"], prob["lambda"]
    seed = prob["seed"]
    inv_var = [1.0 / s_ ** 2 for s_ in prob["sigma_eps"]]
    S = np.zeros(K)
    U = np.zeros((K, T, 2))
    for k in range(K):
        x = np.array(x0, dtype=float)
        cost = 0.0
        for t in range(T):
            z = oracle.normals(seed, [t, 0, k, s])
            u = np.clip(v[t] + np.array(prob["sigma_eps"]) * z[:2],
                        [-prob["steer_max"], -prob["accel_max"]],
                        [prob["steer_max"], prob["accel_max"]])
            U[k, t] = u
            cost += oracle.stage_cost(prob, np.concatenate([x, [0, 0, 0]]))
            cost += prob["gamma_u"] * (v[t, 0] * inv_var[0] * u[0] + v[t, 1] * inv_var[1] * u[1])
            x = oracle.model_step(prob, x, u)
        cost += prob["phi_scale"] * oracle.stage_cost(prob, np.concatenate([x, [0, 0, 0]]))
        S[k] = cost
    w = np.exp(-(S - S.min()) / lam)
    return S, (w[:, None, None] * U).sum(axis=0) / w.sum()


def test_special_case_is_plain_mppi():
    prob, x0, _ = W.config_small()
    prob = dict(prob, K=24, M=1, sigma_w=[0, 0, 0], C_cbf=0.0, shield_iters=0)
    T = prob["T"]
    v = np.column_stack([0.05 * np.ones(T), 0.3 * np.ones(T)])
    res = oracle.solve(prob, 7, x0, v)
    S, vplus = _plain_mppi(prob, 7, x0, v)
    assert res["S"] == pytest.approx(S, rel=1e-13, abs=1e-12)
    assert res["v"] == pytest.approx(vplus, abs=1e-12)


def test_brute_force_tiny_solve():
    """K = 2, M = 5, T = 2 with Sigma_0 != 0: a literal evaluator that stores every particle and
    uses the unshifted weights in extended precision agrees with the solve.  The disturbance
    normals of step t are dealt from the twelve normals of each particle quad's three blocks
    (t, 3q + b, k), three per particle; M = 5 spans two quads."""
    prob, x0, _ = W.config_small()
    prob = dict(prob, K=2, M=5, T=2, C_cbf=50.0)
    T, K, M = 2, 2, 5
    s = 11
    v = np.array([[0.05, 0.5], [-0.02, -0.3]])
    Sigma0 = np.diag([0.04, 0.09, 0.001, 0.01, 0.01, 0.001])
    L0 = np.linalg.cholesky(Sigma0)
    nu = oracle.backoff(prob["delta"])
    S_all, U_all = [], []
    for k in range(K):
        X = np.zeros((T + 1, M, 6))
        for m in range(M):
            xi = np.concatenate([oracle.normals(prob["seed"], [b, m, k, (2 << 28) | s])[:3]
                                 for b in (0, 1)])
            X[0, m] = x0 + L0 @ xi
        U = np.zeros((T, 2))
        moms = [np.concatenate([x0, [Sigma0[0, 0], Sigma0[0, 1], Sigma0[1, 1]]])]
        for t in range(T):
            z = oracle.normals(prob["seed"], [t, 0, k, s])
            U[t] = np.clip(v[t] + np.array(prob["sigma_eps"]) * z[:2], [-0.4, -4], [0.4, 4])
            for m in range(M):
                X[t + 1, m] = oracle.model_step(prob, X[t, m], U[t])
                q, i = divmod(m, 4)
                z12 = np.concatenate([oracle.normals(prob["seed"], [t, 3 * q + b, k, (1 << 28) | s])
                                      for b in range(3)])
                X[t + 1, m, 3:] += np.array(prob["sigma_w"]) * z12[3 * i:3 * i + 3]
            mean = X[t + 1].mean(axis=0)
            C = np.cov(X[t + 1, :, :2].T, ddof=1)
            moms.append(np.concatenate([mean, [C[0, 0], C[0, 1], C[1, 1]]]))
        hs = [oracle.barrier(prob, nu, mm) for mm in moms]
        cost = 0.0
        for t in range(T):
            cost += oracle.stage_cost(prob, moms[t])
            cost += prob["gamma_u"] * (v[t, 0] * U[t, 0] / 0.01 + v[t, 1] * U[t, 1] / 1.0)
        for t in range(1, T + 1):
            cost += prob["C_cbf"] * max(-hs[t] + (1 - prob["gamma"]) * hs[t - 1], 0.0)
        cost += oracle.stage_cost(prob, moms[T])
        S_all.append(cost)
        U_all.append(U)
    S_all = np.array(S_all, dtype=np.longdouble)
    w = np.exp(-S_all / np.longdouble(prob["lambda"]))
    vplus = (w[:, None, None] * np.array(U_all, dtype=np.longdouble)).sum(axis=0) / w.sum()
    res = oracle.solve(prob, s, x0, v, Sigma0=Sigma0)
    assert res["S"] == pytest.approx(np.array(S_all, dtype=float), rel=1e-12)
    assert res["v"] == pytest.approx(np.array(vplus, dtype=float), abs=1e-12)


# ========================================= MPPI update ========================================
def test_update_weights_sum_to_one_and_shift_invariance():
    rng = np.random.default_rng(4)
    K, T = 300, 7
    cfg = W.default_problem(K=K, T=T)
    S = rng.uniform(10, 20, K)
    v = rng.normal(size=(T, 2))
    c = rng.normal(size=(T, 2))
    u = v[None] + c[None]                               # every sample deviates by the same c
    _, vp, st = oracle.update(cfg, S, np.ascontiguousarray(np.broadcast_to(u, (K, T, 2))), v)
    assert vp == pytest.approx(v + c, abs=K * 2.0**-52 * 10)
    u = rng.normal(size=(K, T, 2))
    _, v1, s1 = oracle.update(cfg, S, u, v)
    _, v2, s2 = oracle.update(cfg, S + 1234.5, u, v)
    assert v1 == pytest.approx(v2, abs=1e-12)
    assert s1[1] == pytest.approx(s2[1], rel=1e-12) and s1[2] == pytest.approx(s2[2], rel=1e-12)
    assert s2[0] == pytest.approx(S.min() + 1234.5)


def test_update_temperature_limits_and_nonfinite_costs():
    rng = np.random.default_rng(6)
    K, T = 50, 4
    S = rng.uniform(0, 5, K)
    u = rng.normal(size=(K, T, 2))
    v = np.zeros((T, 2))
    _, vp, _ = oracle.update(W.default_problem(K=K, T=T, **{"lambda": 1e-6}), S, u, v)
    assert vp == pytest.approx(u[np.argmin(S)], abs=1e-12)
    _, vp, st = oracle.update(W.default_problem(K=K, T=T, **{"lambda": 1e12}), S, u, v)
    assert vp == pytest.approx(u.mean(axis=0), abs=1e-9)
    assert st[2] == pytest.approx(K, rel=1e-9)
    S2 = S.copy()
    S2[np.argmin(S)] = np.nan
    S2[3] = np.inf
    _, vp, st = oracle.update(W.default_problem(K=K, T=T, **{"lambda": 1e-6}), S2, u, v)
    keep = np.isfinite(S2)
    best = np.flatnonzero(keep)[np.argmin(S2[keep])]
    assert vp == pytest.approx(u[best], abs=1e-12)
    assert st[3] == K - 2
    rc, vp, _ = oracle.update(W.default_problem(K=K, T=T), np.full(K, np.nan), u, v + 1.0)
    assert rc == 1 and np.all(vp == 1.0)


# ========================================= shield repair ======================================
def _repair_setup(**kw):
    prob = W.default_problem(shield_iters=kw.pop("iters", 2), **kw)
    nu = oracle.backoff(prob["delta"])
    return prob, nu


def test_repair_identity_cases():
    """No iterations, or a control that already satisfies the condition, leave u unchanged."""
    prob, nu = _repair_setup(iters=0)
    a = prob["ell_a"]
    mom = np.array([a + 1.9, 0.0, 0.0, 6.0, 0, 0, 0.01, 0, 0.01])   # heading outward near the wall
    assert list(oracle.repair(prob, nu, mom, [0.0, 0.0])) == [0.0, 0.0]
    prob, nu = _repair_setup(iters=3)
    safe = np.array([a, 0.0, math.pi / 2, 5.0, 0, 0, 1e-4, 0, 1e-4])  # centerline, along tangent
    assert list(oracle.repair(prob, nu, safe, [0.01, 0.2])) == [0.01, 0.2]


def _residual_fn(prob, nu, mom):
    """r(u) = -h(f(xbar, u); sigma_t) + (1 - gamma) h_t from the oracle's model, distance and
    barrier primitives (pinned above)."""
    a, b, wT, g = prob["ell_a"], prob["ell_b"], prob["half_width"], prob["gamma"]
    _, nn = oracle.ellipse_sdf(a, b, mom[0], mom[1])
    sig = math.sqrt(nn @ np.array([[mom[6], mom[7]], [mom[7], mom[8]]]) @ nn)
    h_t = oracle.barrier(prob, nu, mom)

    def resid(u):
        xn = oracle.model_step(prob, mom[:6], u)
        sd, _ = oracle.ellipse_sdf(a, b, xn[0], xn[1])
        return -(max(wT - nu * sig, 0) ** 2 - sd ** 2) + (1 - g) * h_t
    return resid


def test_repair_restores_the_condition():
    """Drifting outward near the outer wall with a tight rate (gamma = 0.05): r > 0 for u = 0.
    Each damped Gauss-Newton step steers back toward the centerline (positive steer), and a few
    steps drive the residual to a small fraction of its start, inside the control box."""
    prob, nu = _repair_setup(iters=6, gamma=0.05)
    mom = np.array([prob["ell_a"] + 1.0, 0.3, math.pi / 2 - 0.2, 6.0, 0, 0, 0.002, 0, 0.002])
    resid = _residual_fn(prob, nu, mom)
    u0 = np.array([0.0, 0.0])
    r0 = resid(u0)
    assert r0 > 0
    u = oracle.repair(prob, nu, mom, u0)
    assert abs(u[0]) <= 0.4 and abs(u[1]) <= 4.0
    assert u[0] > 0.0
    assert resid(u) < 0.01 * r0
    u1 = oracle.repair(dict(prob, shield_iters=1), nu, mom, u0)
    assert 0.0 < resid(u1) < 0.5 * r0


def test_repair_step_is_the_damped_gauss_newton_step():
    """One iteration equals clip(u - r g / (|g|^2 + gmin^2)) with g the gradient of r, here taken
    by a finer central difference than the oracle's (they agree to the difference truncation)."""
    prob, nu = _repair_setup(iters=1, gamma=0.05)
    mom = np.array([prob["ell_a"] + 1.3, -0.4, math.pi / 2 - 0.3, 5.5, 0.1, 0.05, 0.004, 0.001,
                    0.003])
    resid = _residual_fn(prob, nu, mom)
    u0 = np.array([0.05, -0.5])
    r0 = resid(u0)
    assert r0 > 0
    h = 1e-6
    g = np.array([(resid(u0 + [h, 0]) - resid(u0 - [h, 0])) / (2 * h),
                  (resid(u0 + [0, h]) - resid(u0 - [0, h])) / (2 * h)])
    want = np.clip(u0 - r0 * g / (g @ g + prob["shield_gmin"] ** 2), [-0.4, -4.0], [0.4, 4.0])
    got = oracle.repair(prob, nu, mom, u0)
    assert abs(got[1] - u0[1]) > 1e-4           # the accel channel moved and is not clipped
    assert got == pytest.approx(want, abs=1e-6)


@pytest.mark.parametrize("iters", [1, 2, 5])
def test_repair_on_an_affine_residual_contracts_in_closed_form(iters):
    """Linear test model x+ = A x + B u with one binding speed limit a^T x <= b (a = e_vx) and the
    track term slack (the mean on the centerline, positions independent of u).  Then
    r(u) = a^T (A xbar + B u) - b + nu sigma + (1 - gamma) h_t is affine with gradient
    g = B^T a, each damped step multiplies r by rho = gmin^2 / (|g|^2 + gmin^2), and n unclipped
    steps give u_n = u_0 - r_0 (1 - rho^n) g / |g|^2 and r(u_n) = rho^n r_0.  Every quantity
    below is computed from the model's matrices and the heuristic of eq. 13, not from the
    oracle's repair."""
    dt = 0.05
    A = np.eye(6)
    A[3, 3], A[3, 4], A[5, 5] = 0.98, 0.01, 0.9
    B = np.zeros((6, 2))
    B[3, 0], B[3, 1] = 0.02, dt          # both controls act on vx; positions are not touched
    B[5, 0] = 0.5
    gmin, gam, b_lim, var_c = 0.05, 0.2, 6.0, 1e-4
    a_con = np.array([0.0, 0.0, 0.0, 1.0, 0.0, 0.0])
    prob = W.default_problem(model=1, shield_iters=iters, shield_gmin=gmin, gamma=gam, n_con=1,
                             con_a=list(np.concatenate([a_con, np.zeros(18)])),
                             con_b=[b_lim, 0.0, 0.0, 0.0])
    prob["lin_A"], prob["lin_B"] = A, B
    nu = oracle.backoff(prob["delta"])
    xbar = np.array([prob["ell_a"], 0.0, math.pi / 2, 5.9, 0.1, 0.0])
    mom = np.concatenate([xbar, [0.0, 0.0, 0.0]])
    sig = math.sqrt(var_c)
    h_track = prob["half_width"] ** 2            # e_y = 0 and Sigma_pos = 0 on the centerline
    h_t = min(h_track, b_lim - a_con @ xbar - nu * sig)

    def r_of(u):
        return a_con @ (A @ xbar + B @ u) - b_lim + nu * sig + (1.0 - gam) * h_t

    u0 = np.array([0.05, 3.0])
    g = B.T @ a_con
    r0 = r_of(u0)
    assert r0 > 0
    rho = gmin ** 2 / (g @ g + gmin ** 2)
    want = u0 - r0 * (1.0 - rho ** iters) * g / (g @ g)
    got = oracle.repair(prob, nu, mom, u0, con_var=[var_c])
    assert np.all(np.abs(want) < [prob["steer_max"], prob["accel_max"]])      # no clipping
    assert got == pytest.approx(want, rel=1e-9, abs=1e-12)
    assert r_of(got) == pytest.approx(rho ** iters * r0, rel=1e-7)
    # the track term stays slack at every point the repair evaluates
    xn = A @ xbar + B @ got
    assert h_track > b_lim - a_con @ xn - nu * sig


def test_repair_is_continuous():
    """Small changes of the sampled control or of the belief change the repaired control by a
    bounded multiple (the damping caps the gain where the control has little authority)."""
    prob, nu = _repair_setup(iters=3, gamma=0.05)
    rng = np.random.default_rng(8)
    a = prob["ell_a"]
    worst = 0.0
    for _ in range(200):
        mom = np.array([a + rng.uniform(-2.5, 2.5), rng.uniform(-1, 1),
                        math.pi / 2 + rng.uniform(-0.4, 0.4), rng.uniform(3, 8),
                        rng.normal() * 0.2, rng.normal() * 0.2, 0.003, 0.0005, 0.002])
        u0 = rng.uniform([-0.4, -4], [0.4, 4])
        base = oracle.repair(prob, nu, mom, u0)
        d = 1e-7
        du = rng.normal(size=2) * d
        dm = np.zeros(9)
        dm[:2] = rng.normal(size=2) * d
        out1 = oracle.repair(prob, nu, mom, u0 + du)
        out2 = oracle.repair(prob, nu, mom + dm, u0)
        worst = max(worst, np.max(np.abs(out1 - base)) / d, np.max(np.abs(out2 - base)) / d)
    assert worst < 100.0


def test_step_shift():
    v = np.arange(10, dtype=float).reshape(5, 2)
    s = oracle.step_shift(v)
    assert s.tolist() == [[2, 3], [4, 5], [6, 7], [8, 9], [8, 9]]


# ============================ Gaussian re-sampling reading (Alg. 2) ============================
def test_semidefinite_factor():
    """The re-sampling factor: the Cholesky factor on positive definite input, L L^T = A with the
    rank's number of nonzero pivots on semi-definite input, and a zero column for a variance at
    the rounding level of an exactly degenerate set."""
    rng = np.random.default_rng(3)
    B = rng.normal(size=(6, 6))
    A = B @ B.T + 0.1 * np.eye(6)
    assert np.max(np.abs(oracle.chol_psd6(A) - np.linalg.cholesky(A))) <= 1e-13
    B3 = rng.normal(size=(6, 3))
    A3 = B3 @ B3.T
    L3 = oracle.chol_psd6(A3)
    assert np.max(np.abs(L3 @ L3.T - A3)) <= 1e-12 * np.max(np.abs(A3))
    assert np.count_nonzero(np.diag(L3)) == 3
    Z = A.copy()
    Z[0, :] = 0.0
    Z[:, 0] = 0.0
    LZ = oracle.chol_psd6(Z)
    assert np.all(LZ[:, 0] == 0.0)
    assert np.max(np.abs(LZ[1:, 1:] - np.linalg.cholesky(A[1:, 1:]))) <= 1e-13
    R = A.copy()
    R[0, 0] = 1e-30
    R[1:, 0] = R[0, 1:] = 1e-18
    LR = oracle.chol_psd6(R)
    assert np.all(LR[:, 0] == 0.0)


def test_resampling_with_one_particle_is_the_persistent_recursion():
    """M = 1: the covariance is 0, so every redraw returns the particle itself."""
    prob, x0, v = W.config_small()
    prob = dict(prob, K=16, M=1, T=12)
    a = oracle.solve(prob, 3, x0, v[:12])
    b = oracle.solve(dict(prob, belief=1), 3, x0, v[:12])
    for key in ("v", "mom", "S", "u"):
        assert np.array_equal(a[key], b[key]), key


def test_resampling_without_disturbance_is_deterministic_integration():
    """No disturbance and a known start: every particle stays on the deterministic trajectory, the
    covariance stays (numerically) zero, and the redraw only moves particles to the mean."""
    prob, x0, v = W.config_small()
    prob = dict(prob, K=8, M=7, T=15, sigma_w=[0.0, 0.0, 0.0])
    a = oracle.solve(prob, 1, x0, v[:15])
    b = oracle.solve(dict(prob, belief=1), 1, x0, v[:15])
    assert np.max(np.abs(a["mom"] - b["mom"])) <= 1e-12 * np.max(np.abs(a["mom"]))
    assert np.max(np.abs(a["S"] - b["S"])) <= 1e-12 * np.max(np.abs(a["S"]))


def test_resampling_linear_gaussian_matches_closed_form():
    """Linear-Gaussian model: redrawing from the sample mean and covariance keeps
    Sigma_{t+1} = A Sigma_t A^T + Q in expectation; each redraw adds one sampling error, so the
    bound grows like sqrt(t) standard errors."""
    M = 1 << 14
    cfg, A, Q = _linear_problem(M, T=6)
    cfg = dict(cfg, belief=1)
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    mom = oracle.propagate(cfg, 0, 0, x0, np.zeros((cfg["T"], 2)))
    Sig = np.zeros((6, 6))
    mean = x0.copy()
    for t in range(1, cfg["T"] + 1):
        Sig = A @ Sig @ A.T + Q
        mean = A @ mean
        got = mom[t]
        tol = 6.0 * math.sqrt(t)
        assert np.all(np.abs(got[:6] - mean) <= tol * np.sqrt(np.diag(Sig) / M) + 1e-10)
        for val, (i, j) in zip(got[6:], ((0, 0), (0, 1), (1, 1))):
            se = math.sqrt((Sig[i, i] * Sig[j, j] + Sig[i, j] ** 2) / (M - 1))
            assert abs(val - Sig[i, j]) <= tol * se + 1e-15


def test_resampling_changes_a_nonlinear_belief():
    """On the car the two readings differ (the redraw projects the particle cloud onto a
    Gaussian every step) while both stay finite and close in the mean."""
    prob, x0, v = W.config_small()
    prob = dict(prob, K=4, M=32, T=20)
    a = oracle.solve(prob, 2, x0, v[:20])
    b = oracle.solve(dict(prob, belief=1), 2, x0, v[:20])
    assert np.all(np.isfinite(b["mom"]))
    assert np.max(np.abs(a["mom"][:, 2:, 6:] - b["mom"][:, 2:, 6:])) > 1e-9
    assert np.max(np.abs(a["mom"][:, :, :2] - b["mom"][:, :, :2])) < 0.5


# ============== disturbance variants: common random numbers, state-dependent std ==============
def test_common_random_numbers_leave_sample_zero_unchanged():
    """With common random numbers every sample draws the disturbance stream of sample 0, so sample
    0 itself is bit-identical to the independent-stream solve."""
    prob, x0, v = W.config_small()
    prob = dict(prob, K=6, M=8, T=10)
    a = oracle.solve(prob, 4, x0, v[:10])
    b = oracle.solve(dict(prob, crn=1), 4, x0, v[:10])
    assert np.array_equal(a["mom"][0], b["mom"][0])
    assert a["S"][0] == b["S"][0]
    assert not np.array_equal(a["mom"][1:], b["mom"][1:])


def test_common_random_numbers_without_control_noise_give_identical_samples():
    """No control noise and common disturbances: every sample is the same rollout, all weights are
    equal and the update returns the mean sequence; independent disturbances separate them."""
    prob, x0, _ = W.config_small()
    prob = dict(prob, K=5, M=8, T=12, sigma_eps=[0.0, 0.0], crn=1)
    v = np.column_stack([0.05 * np.ones(12), 0.5 * np.ones(12)])
    r = oracle.solve(prob, 0, x0, v)
    assert np.all(r["S"] == r["S"][0])
    assert np.all(r["mom"] == r["mom"][0])
    assert np.max(np.abs(r["v"] - v)) <= 1e-15
    r2 = oracle.solve(dict(prob, crn=0), 0, x0, v)
    assert len(set(r2["S"].tolist())) == 5


def test_state_dependent_disturbance_scales_the_covariance():
    """p(w | x) with std sigma_w (1 + kappa |vx|): from a known start every particle has the same
    vx_0, so the position covariance at t = 2 is the closed form of the linear model with Q scaled
    by (1 + kappa |vx_0|)^2; kappa = 0 is the plain model."""
    M = 1 << 16
    cfg, A, Q = _linear_problem(M, T=2)
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    kappa = 0.2
    f0 = 1.0 + kappa * abs(x0[3])
    mom = oracle.propagate(dict(cfg, sigma_w_speed=kappa), 0, 0, x0, np.zeros((2, 2)))
    Sig = A @ (f0 * f0 * Q) @ A.T
    for val, (i, j) in zip(mom[2][6:], ((0, 0), (0, 1), (1, 1))):
        se = math.sqrt((Sig[i, i] * Sig[j, j] + Sig[i, j] ** 2) / (M - 1))
        assert abs(val - Sig[i, j]) <= 5 * se + 1e-15
    base = oracle.propagate(cfg, 0, 0, x0, np.zeros((2, 2)))
    same = oracle.propagate(dict(cfg, sigma_w_speed=0.0), 0, 0, x0, np.zeros((2, 2)))
    assert np.array_equal(base, same)


# ======================= sigma-point belief propagation (belief = 2) ========================
def test_sigma_points_are_exact_on_the_linear_model():
    """The 12-point cubature set reproduces the linear-Gaussian recursion exactly (up to rounding):
    mean A xbar + B u and covariance A Sigma A^T + Q, from a nonzero Sigma_0."""
    cfg, A, Q = _linear_problem(12, T=6)
    cfg = dict(cfg, belief=2)
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    G = np.random.default_rng(1).normal(size=(6, 6)) * 0.1
    S0 = G @ G.T
    mom = oracle.propagate(cfg, 0, 0, x0, np.zeros((cfg["T"], 2)), Sigma0=S0)
    Sig, mean = S0.copy(), x0.copy()
    for t in range(1, cfg["T"] + 1):
        Sig = A @ Sig @ A.T + Q
        mean = A @ mean
        assert np.max(np.abs(mom[t][:6] - mean)) <= 1e-12 * (1 + np.max(np.abs(mean)))
        want = np.array([Sig[0, 0], Sig[0, 1], Sig[1, 1]])
        assert np.max(np.abs(mom[t][6:] - want)) <= 1e-12 * np.max(np.abs(want)) + 1e-24


def test_sigma_points_state_dependent_disturbance_closed_form():
    """With std sigma_w (1 + kappa |vx|) and every point at positive vx, the points' mean of
    (1 + kappa vx)^2 is (1 + kappa mu)^2 + kappa^2 Sigma_vx, exactly."""
    cfg, A, Q = _linear_problem(12, T=4)
    kappa = 0.1
    cfg = dict(cfg, belief=2, sigma_w_speed=kappa)
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    mom = oracle.propagate(cfg, 0, 0, x0, np.zeros((cfg["T"], 2)))
    Sig, mean = np.zeros((6, 6)), x0.copy()
    for t in range(1, cfg["T"] + 1):
        scale = (1 + kappa * mean[3]) ** 2 + kappa ** 2 * Sig[3, 3]
        Sig = A @ Sig @ A.T + scale * Q
        mean = A @ mean
        want = np.array([Sig[0, 0], Sig[0, 1], Sig[1, 1]])
        assert np.max(np.abs(mom[t][6:] - want)) <= 1e-12 * np.max(np.abs(want)) + 1e-24


def test_sigma_points_without_uncertainty_are_deterministic_integration():
    prob, x0, v = W.config_small()
    prob = dict(prob, K=4, T=15, sigma_w=[0.0, 0.0, 0.0])
    a = oracle.solve(dict(prob, M=1), 2, x0, v[:15])
    b = oracle.solve(dict(prob, M=12, belief=2), 2, x0, v[:15])
    assert np.max(np.abs(a["mom"] - b["mom"])) <= 1e-12 * np.max(np.abs(a["mom"]))
    assert np.max(np.abs(b["mom"][:, :, 6:])) <= 1e-24   # rounding of the points' mean
    assert np.max(np.abs(a["S"] - b["S"])) <= 1e-12 * np.max(np.abs(a["S"]))


def test_sigma_point_belief_needs_twelve_points():
    prob, x0, v = W.config_small()
    with pytest.raises(ValueError):
        oracle.solve(dict(prob, K=2, M=16, belief=2), 0, x0, v)


# ======================= more constraints: circular obstacles (eq. 16) ========================
def _obstacle_problem(obstacles, **kw):
    prob, x0, v = W.config_small()
    flat = [c for ob in obstacles for c in ob] + [0.0] * (12 - 3 * len(obstacles))
    return dict(prob, n_obs=len(obstacles), obs=flat, **kw), x0, v


def test_far_obstacle_changes_nothing():
    """h = min over the constraints: an obstacle far from the track never attains the minimum and
    never holds the mean, so the solve is bit-identical to the track-only one."""
    base, x0, v = W.config_small()
    base = dict(base, K=32, shield_iters=2)
    prob, _, _ = _obstacle_problem([(500.0, 500.0, 2.0)], K=32, shield_iters=2)
    a = oracle.solve(base, 1, x0, v)
    b = oracle.solve(prob, 1, x0, v)
    for key in ("v", "mom", "S", "u"):
        assert np.array_equal(a[key], b[key]), key


def test_obstacle_barrier_closed_form():
    """h_i = max(d_i - nu sqrt(eta^T Sigma_pos eta), 0)^2 - r_i^2 with eta the unit vector from the
    centre to the mean, and h = min(track, obstacles)."""
    prob, _, _ = _obstacle_problem([(31.0, 2.0, 0.8), (29.0, -3.0, 0.5)])
    nu = 1.6448536269514722
    mom = np.array([30.2, 0.4, 1.5, 5.0, 0.0, 0.0, 0.04, 0.01, 0.09])
    S = np.array([[mom[6], mom[7]], [mom[7], mom[8]]])
    hs = []
    for ox, oy, r in ((31.0, 2.0, 0.8), (29.0, -3.0, 0.5)):
        d = np.hypot(mom[0] - ox, mom[1] - oy)
        eta = np.array([mom[0] - ox, mom[1] - oy]) / d
        sig = math.sqrt(eta @ S @ eta)
        hs.append(max(d - nu * sig, 0.0) ** 2 - r * r)
    h_track = oracle.barrier(dict(prob, n_obs=0), nu, mom)
    assert abs(oracle.barrier(prob, nu, mom) - min([h_track] + hs)) <= 1e-12
    assert min(hs) < h_track          # the near obstacle binds here


def test_obstacle_collision_indicator():
    prob, _, _ = _obstacle_problem([(30.0, 0.5, 1.0)])
    inside = np.array([30.2, 0.4, 1.5, 5.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    base = oracle.stage_cost(dict(prob, n_obs=0), inside)
    assert oracle.stage_cost(prob, inside) - base == prob["C_obs"]
    outside = inside.copy()
    outside[1] = 3.0
    assert oracle.stage_cost(prob, outside) == oracle.stage_cost(dict(prob, n_obs=0), outside)


def test_repair_steers_away_from_an_obstacle():
    """An obstacle just ahead of the one-step prediction violates the condition; the repaired
    control raises the barrier of the predicted mean (known state, so the spreads are zero)."""
    prob, _, _ = _obstacle_problem([(30.35, 0.45, 0.3)], shield_iters=4)
    nu = oracle.backoff(prob["delta"])
    mom = np.array([30.0, 0.0, math.pi / 2, 5.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    u = np.array([0.0, 0.0])

    def h_pred(uu):
        xn = oracle.model_step(prob, mom[:6], uu)
        return oracle.barrier(prob, nu, np.concatenate([xn, [0.0, 0.0, 0.0]]))

    h_t = oracle.barrier(prob, nu, mom)
    assert -h_pred(u) + (1 - prob["gamma"]) * h_t > 0      # violated before the repair
    u_rep = oracle.repair(prob, nu, mom, u)
    assert h_pred(u_rep) > h_pred(u)


# ---- repair of the updated sequence from the estimate (local repair of v+, Alg. 1) ----------

LOCAL_REPAIR_KEY = 0x5DEECE66DA3B9F1B     # documented stream of the repair rollout


def _local_repair_problem(**kw):
    base = dict(K=64, M=4, T=20, shield_iters=8, gamma=0.3, sigma_w=[0.0, 0.0, 0.0])
    base.update(kw)
    return W.default_problem(**base)


def test_local_repair_on_a_deterministic_belief():
    """No disturbance and no initial spread: every particle is the mean, so each belief step is
    the model step of the control the repair chose.  Heading outward near the outer wall with
    v+ = 0, the unrepaired controls violate the discrete barrier condition from some step on.
    Where they satisfy it the control is clip(v+_t) unchanged; where they do not it is the shield
    repair of clip(v+_t) against the repair rollout's own belief at t (pinned above), the first
    such repair lowers the one-step violation, and the repaired trajectory ends with a larger
    barrier value than the unrepaired one (one-step repairs with little steering authority cannot
    always restore the condition; the control box binds here)."""
    prob = _local_repair_problem()
    nu = oracle.backoff(prob["delta"])
    a = prob["ell_a"]
    x0 = np.array([a + 0.8, 0.0, math.pi / 2 - 0.35, 6.0, 0.0, 0.0])
    v_plus = np.zeros((prob["T"], 2))
    v_safe, mom = oracle.local_repair(prob, 7, x0, v_plus)
    assert np.all(mom[:, 6:] == 0.0)
    active = []
    for t in range(prob["T"]):
        assert np.array_equal(mom[t + 1, :6], oracle.model_step(prob, mom[t, :6], v_safe[t]))
        resid = _residual_fn(prob, nu, mom[t])
        r_before = resid(v_plus[t])
        if r_before > 0:
            active.append(t)
            assert np.array_equal(v_safe[t], oracle.repair(prob, nu, mom[t], v_plus[t]))
        else:
            assert np.array_equal(v_safe[t], v_plus[t])
    assert len(active) >= 3
    first = active[0]
    resid = _residual_fn(prob, nu, mom[first])
    assert resid(v_safe[first]) < 0.9 * resid(v_plus[first])
    unrepaired = oracle.propagate(prob, 7, 0, x0, v_plus)
    assert np.array_equal(unrepaired[:first + 1], mom[:first + 1])
    assert oracle.barrier(prob, nu, mom[-1]) > oracle.barrier(prob, nu, unrepaired[-1]) + 1.0


def test_local_repair_rollout_draws_its_own_stream():
    """With disturbance and an initial spread, the repair rollout's belief is the propagation of
    v_safe by sample 0 under the key seed ^ 0x5DEECE66DA3B9F1B (and not the samples' stream)."""
    prob = _local_repair_problem(sigma_w=[0.3, 0.3, 0.2], M=16, seed=11)
    x0 = np.array([prob["ell_a"] + 0.8, 0.0, math.pi / 2 - 0.35, 6.0, 0.0, 0.0])
    Sigma0 = np.diag([0.01, 0.01, 0.001, 0.02, 0.01, 0.005])
    v_plus = np.tile([0.05, 0.3], (prob["T"], 1))
    v_safe, mom = oracle.local_repair(prob, 5, x0, v_plus, Sigma0=Sigma0)
    same = oracle.propagate(dict(prob, seed=prob["seed"] ^ LOCAL_REPAIR_KEY), 5, 0, x0, v_safe,
                            Sigma0=Sigma0)
    assert np.array_equal(mom, same)
    other = oracle.propagate(prob, 5, 0, x0, v_safe, Sigma0=Sigma0)
    assert np.max(np.abs(other[1:, :2] - mom[1:, :2])) > 1e-6
    assert not np.array_equal(v_safe, v_plus)       # the repair was active somewhere


def test_solve_with_local_repair_is_update_then_repair():
    """local_repair = 1: the solve's v is the repair of the update of the shielded solve; = 2:
    the repair of the update of the solve whose samples are not repaired."""
    prob = _local_repair_problem(sigma_w=[0.3, 0.3, 0.2], K=48, M=8, T=15,
                                 sigma_eps=[0.1, 1.0])
    x0 = np.array([prob["ell_a"] + 1.0, 0.0, math.pi / 2 - 0.3, 6.0, 0.0, 0.0])
    v = np.tile([0.0, 0.5], (prob["T"], 1))
    s = 3
    plain = oracle.solve(prob, s, x0, v, want_traces=False, nthreads=2)
    with_lr = oracle.solve(dict(prob, local_repair=1), s, x0, v, want_traces=False, nthreads=2)
    assert np.array_equal(with_lr["v"], oracle.local_repair(prob, s, x0, plain["v"])[0])
    assert np.array_equal(with_lr["stats"], plain["stats"])
    unrepaired = oracle.solve(dict(prob, shield_iters=0), s, x0, v, want_traces=False,
                              nthreads=2)
    only_lr = oracle.solve(dict(prob, local_repair=2), s, x0, v, want_traces=False, nthreads=2)
    assert np.array_equal(only_lr["v"], oracle.local_repair(prob, s, x0, unrepaired["v"])[0])
    assert not np.array_equal(only_lr["v"], with_lr["v"])


def test_local_repair_argument_checks():
    with pytest.raises(ValueError):
        oracle.make_params(W.default_problem(local_repair=3))
    with pytest.raises(ValueError):
        oracle.make_params(W.default_problem(local_repair=1, shield_iters=0))


# ============================ half-space constraints on the state ============================
def _con_problem(rows, bounds, **kw):
    """Problem with len(rows) half-space constraints a_i^T x <= b_i."""
    a = np.zeros(24)
    b = np.zeros(4)
    for i, (row, bound) in enumerate(zip(rows, bounds)):
        a[6 * i:6 * i + 6] = row
        b[i] = bound
    return W.default_problem(n_con=len(rows), con_a=list(a), con_b=list(b), **kw)


def test_full_covariance_matches_library():
    """The full 6x6 estimate equals NumPy's unbiased covariance, its position block is the
    record's (same two-pass sums), and a single particle gives zero."""
    rng = np.random.default_rng(7)
    P = rng.normal(size=(50, 6)) * [3.0, 2.0, 0.5, 1.0, 0.2, 0.1] + [100.0, -40.0, 1.0, 6.0, 0, 0]
    cov = oracle.full_cov(P)
    want = np.cov(P.T, ddof=1)
    assert np.max(np.abs(cov - want)) <= 1e-12 * np.max(np.abs(want))
    m = oracle.moments(P)
    assert [cov[0, 0], cov[0, 1], cov[1, 1]] == list(m[6:])
    assert np.array_equal(oracle.full_cov(P[:1]), np.zeros((6, 6)))


def test_constraint_spread_is_variance_of_the_projection():
    """a^T Sigma a equals the unbiased variance of the projected particles a^T x^n (brute force
    on the scalars); entries beyond n_con are zero."""
    rng = np.random.default_rng(8)
    P = rng.normal(size=(40, 6)) * [3.0, 2.0, 0.5, 1.0, 0.2, 0.1]
    rows = [rng.normal(size=6), [0, 0, 0, 1.0, 0, 0], rng.normal(size=6)]
    cfg = _con_problem(rows, [1.0, 2.0, 3.0])
    got = oracle.con_spreads(cfg, oracle.full_cov(P))
    for i, a in enumerate(rows):
        y = P @ np.asarray(a, dtype=np.float64)
        want = np.sum((y - y.mean()) ** 2) / (len(y) - 1)
        assert got[i] == pytest.approx(want, rel=1e-12)
    assert got[3] == 0.0


def test_constraint_variance_linear_model_closed_form():
    """On the linear-Gaussian model the recorded a^T Sigma_t a of constraints on the velocity
    states and on mixed directions follows a^T (A Sigma A^T + Q) a within 5 standard errors of a
    sample variance (sqrt(2 / (M - 1)) relative) at M = 2^16."""
    M = 1 << 16
    base, A, Q = _linear_problem(M)
    rows = [np.array([0, 0, 0, 1.0, 0, 0]), np.array([0, 0, 1.0, 0, 0, 2.0]),
            np.array([0.5, 0, 0, 0, -1.0, 0]), np.array([1.0, 1.0, 0, 0.3, 0, 0])]
    cfg = dict(_con_problem(rows, [10.0] * 4), **{k: base[k] for k in
                                                  ("model", "lin_A", "lin_B", "K", "M", "T",
                                                   "sigma_w", "sigma_eps")})
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    mom, cv = oracle.propagate(cfg, 0, 0, x0, np.zeros((cfg["T"], 2)), with_con=True)
    assert cv.shape == (cfg["T"] + 1, 4)
    assert np.array_equal(cv[0], np.zeros(4))
    Sig = np.zeros((6, 6))
    for t in range(1, cfg["T"] + 1):
        Sig = A @ Sig @ A.T + Q
        for i, a in enumerate(rows):
            want = a @ Sig @ a
            assert abs(cv[t, i] - want) <= 5 * want * math.sqrt(2.0 / (M - 1)) + 1e-15


def test_constraint_variance_sigma_points_exact_with_initial_spread():
    """Sigma points on the linear model: the recorded a^T Sigma_t a equals the exact recursion from
    a nonzero Sigma_0 (record 0 is a^T Sigma_0 a), disturbance covariance included."""
    base, A, Q = _linear_problem(12, T=6)
    rows = [np.array([0, 0, 0, 1.0, 0, 0]), np.array([0.3, -0.2, 0.1, 0.5, 1.0, -2.0])]
    cfg = dict(_con_problem(rows, [10.0, 10.0]), belief=2,
               **{k: base[k] for k in ("model", "lin_A", "lin_B", "K", "M", "T", "sigma_w",
                                       "sigma_eps")})
    x0 = np.array([1.0, 2.0, 0.0, 3.0, 0.5, 0.1])
    G = np.random.default_rng(1).normal(size=(6, 6)) * 0.1
    S0 = G @ G.T
    _, cv = oracle.propagate(cfg, 0, 0, x0, np.zeros((cfg["T"], 2)), Sigma0=S0, with_con=True)
    Sig = S0.copy()
    for t in range(cfg["T"] + 1):
        if t > 0:
            Sig = A @ Sig @ A.T + Q
        want = np.array([a @ Sig @ a for a in rows])
        assert np.max(np.abs(cv[t] - want)) <= 1e-12 * np.max(np.abs(want))


def test_position_constraints_reproduce_the_position_block():
    """On the car with persistent particles, constraints along X, along Y and along X + Y record
    Sigma_XX, Sigma_YY and Sigma_XX + 2 Sigma_XY + Sigma_YY of the same particle sets."""
    rows = [np.array([1.0, 0, 0, 0, 0, 0]), np.array([0, 1.0, 0, 0, 0, 0]),
            np.array([1.0, 1.0, 0, 0, 0, 0])]
    cfg = _con_problem(rows, [1e3] * 3, K=4, M=24, T=20, sigma_w=[0.3, 0.3, 0.2])
    x0 = W.pose_on_centerline(cfg["ell_a"], cfg["ell_b"], 0.4, vx=6.0)
    Sigma0 = np.diag([0.04, 0.09, 0.01, 0.2, 0.05, 0.02])
    mom, cv = oracle.propagate(cfg, 3, 1, x0, np.tile([0.05, 0.5], (20, 1)), Sigma0=Sigma0,
                               with_con=True)
    assert np.array_equal(cv[:, 0], mom[:, 6])
    assert np.array_equal(cv[:, 1], mom[:, 8])
    s = mom[:, 6] + 2 * mom[:, 7] + mom[:, 8]
    assert np.max(np.abs(cv[:, 2] - s)) <= 1e-12 * np.max(np.abs(s))
    assert np.all(cv[1:, 2] > 0)


def test_constraint_barrier_closed_form_and_minimum():
    """h = min(track, constraints): with a wide track a speed limit vx <= b is the minimum and
    equals b - vx - nu sqrt(var); a far bound leaves the track's h; a negative rounding variance
    counts as zero."""
    nu = oracle.backoff(0.05)
    rows = [np.array([0, 0, 0, 1.0, 0, 0])]
    rec = np.array([30.5, 0.2, 1.7, 6.0, 0.1, 0.02, 0.04, 0.01, 0.09])
    wide = _con_problem(rows, [6.5], half_width=50.0)
    h = oracle.barrier(wide, nu, rec, [0.16])
    assert h == pytest.approx(6.5 - 6.0 - nu * 0.4, rel=1e-14)
    track_only = oracle.barrier(dict(wide, n_con=0), nu, rec)
    assert track_only > h
    far = _con_problem(rows, [1e6], half_width=50.0)
    assert oracle.barrier(far, nu, rec, [0.16]) == track_only
    assert oracle.barrier(wide, nu, rec, [-1e-18]) == pytest.approx(0.5, rel=1e-14)
    mixed = _con_problem([np.array([0.5, 0, 0, -1.0, 0, 2.0])], [0.0], half_width=50.0)
    want = 0.0 - (0.5 * 30.5 - 6.0 + 2 * 0.02) - nu * math.sqrt(0.25)
    assert oracle.barrier(mixed, nu, rec, [0.25]) == pytest.approx(want, rel=1e-14)


def test_constraint_repair_brakes_at_a_speed_limit():
    """A speed limit that the full-throttle control would cross: the repair lowers the
    acceleration, reduces the one-step residual r(u) = -h(f(xbar, u)) + (1 - gamma) h_t (spread
    frozen; zero position covariance so the track term is spread-free) and leaves a control that
    already satisfies the condition unchanged."""
    nu = oracle.backoff(0.05)
    limit = 6.3
    cfg = _con_problem([np.array([0, 0, 0, 1.0, 0, 0])], [limit], half_width=50.0,
                       shield_iters=6)
    xb = W.pose_on_centerline(cfg["ell_a"], cfg["ell_b"], 0.3, vx=6.0)
    rec = np.concatenate([xb, [0.0, 0.0, 0.0]])
    cvar = [0.01]
    h_t = oracle.barrier(cfg, nu, rec, cvar)

    def resid(u):
        xn = oracle.model_step(cfg, xb, u)
        return -oracle.barrier(cfg, nu, np.concatenate([xn, [0.0, 0.0, 0.0]]), cvar) + \
            (1 - cfg["gamma"]) * h_t

    u = np.array([0.0, 4.0])
    assert resid(u) > 0
    ur = oracle.repair(cfg, nu, rec, u, cvar)
    assert ur[1] < u[1]
    assert resid(ur) < 0.05 * resid(u)
    ok = np.array([0.0, -2.0])
    assert resid(ok) <= 0
    assert np.array_equal(oracle.repair(cfg, nu, rec, ok, cvar), ok)


def test_constraint_score_term_closed_form():
    """With the constraint as the minimum everywhere, the score's safety part is
    C sum_{t>=1} max(-h_t + (1 - gamma) h_{t-1}, 0) with h_t = b - vx_t - nu sqrt(var_t)."""
    nu = oracle.backoff(0.05)
    T = 12
    rng = np.random.default_rng(3)
    cfg = _con_problem([np.array([0, 0, 0, 1.0, 0, 0])], [7.0], half_width=50.0, T=T)
    mom = np.zeros((T + 1, 9))
    mom[:, 0] = cfg["ell_a"]
    mom[:, 2] = math.pi / 2
    mom[:, 3] = 6.0 + 0.08 * np.arange(T + 1) + 0.05 * rng.normal(size=T + 1)
    var = 0.01 + 0.002 * np.arange(T + 1)
    u = rng.normal(size=(T, 2)) * 0.1
    v = rng.normal(size=(T, 2)) * 0.1
    with_c = oracle.score(cfg, nu, mom, u, v, var[:, None])
    without = oracle.score(dict(cfg, C_cbf=0.0), nu, mom, u, v, var[:, None])
    h = 7.0 - mom[:, 3] - nu * np.sqrt(var)
    viol = np.maximum(-h[1:] + (1 - cfg["gamma"]) * h[:-1], 0.0)
    assert viol.sum() > 0
    assert with_c - without == pytest.approx(cfg["C_cbf"] * viol.sum(), rel=1e-12)


def test_inactive_constraint_leaves_the_solve_unchanged():
    """A bound no belief comes near gives h = the track's everywhere: the solve is bitwise the
    unconstrained one."""
    prob, x0, v = W.config_small()
    prob = dict(prob, K=32, T=12, shield_iters=2)
    v = v[:12]
    a = oracle.solve(prob, 1, x0, v, nthreads=2)
    rows = [np.array([0, 0, 0, 1.0, 0, 0])]
    far = dict(prob, n_con=1, con_a=list(np.concatenate([rows[0], np.zeros(18)])),
               con_b=[1e9, 0.0, 0.0, 0.0])
    b = oracle.solve(far, 1, x0, v, nthreads=2)
    for key in ("v", "u", "mom", "S", "stats"):
        assert np.array_equal(a[key], b[key]), key
    assert b["con_var"].shape == (32, 13, 1)


def test_constraint_argument_checks():
    with pytest.raises(ValueError):
        oracle.make_params(W.default_problem(n_con=5))
