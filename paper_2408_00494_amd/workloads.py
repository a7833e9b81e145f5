"""Seeded synthetic workloads (problem descriptions and start states).

This module only generates inputs: parameter sets, start poses on the synthetic elliptical track,
warm-start sequences and the per-instance draws of the batched and serving workloads.  It holds
none of the method's arithmetic, and both the GPU path and the oracle take their inputs from it.

The paper's experiments use the AutoRally track and simulator, which are not available; a
synthetic ellipse track (centerline semi-axes a x b, constant half-width w_T) stands in for them,
with the paper's goal speed (6 m/s), lateral-deviation weight (0.1) and half-width (2 m).
"""
import math

import numpy as np

# Problem description shared by both implementations.  Car data beyond the mass and the tire
# stiffness are not given anywhere, so the remaining values are stated choices.
_DEFAULTS = dict(
    # single-track car with linear tires
    m=1500.0, Iz=2500.0, lf=1.2, lr=1.6, Cf=5.0e4, Cr=5.0e4, mu=1.0, g=9.81, v_min=3.0,
    dt=0.05,
    # control box and noise
    steer_max=0.4, accel_max=4.0,
    sigma_eps=[0.1, 1.0],
    sigma_w=[0.1, 0.1, 0.05],
    # sizes
    K=256, M=16, T=30,
    # chance constraint and DCBF
    delta=0.05, gamma=0.2, backoff=0,
    # MPPI and costs
    **{"lambda": 1.0},
    gamma_u=1.0, v_goal=6.0, q_vx=1.0, q_vy=0.0, q_r=0.0, q_ey=0.1, q_epsi=1.0,
    C_cbf=100.0, C_obs=1000.0, phi_scale=1.0,
    # track
    ell_a=30.0, ell_b=20.0, half_width=2.0,
    # shield repair (0 iterations = off)
    shield_iters=0, shield_gmin=0.05, shield_fd=1.0e-2,
    # random numbers, belief propagation (0 persistent particles, 1 Gaussian re-sampling every
    # step), common random numbers for the disturbance across samples, speed dependence of the
    # disturbance std (sigma_w (1 + sigma_w_speed |vx|)) and model selector (0 = car)
    seed=1, belief=0, crn=0, sigma_w_speed=0.0, model=0,
    # circular obstacles (up to 4): n_obs and the flat list (x, y, radius) per obstacle
    n_obs=0, obs=[0.0] * 12,
    # repair of the updated sequence from the state estimate: 0 off, 1 in addition to the repair
    # of every sample, 2 instead of it (uses the shield_* settings)
    local_repair=0,
    # half-space constraints on the whole state (up to 4): a_i^T x <= b_i with
    # a_i = con_a[6i..6i+5] over (X, Y, psi, vx, vy, r) and b_i = con_b[i]
    n_con=0, con_a=[0.0] * 24, con_b=[0.0] * 4,
    # vehicle: 0 = the 6-state car above, 1 = the paper's 8-state single-track vehicle with wheel
    # speeds in the road-aligned frame (config_vehicle8 sets its values): wheel radius, drive-line
    # inertia per axle, rear drive torque at full throttle, magic-formula coefficients, track
    # length and curvature amplitude, midpoint substeps per control period
    vehicle=0, Rw=0.095, Iw=0.3, T_max=8.0, pac_B=10.0, pac_C=1.9, pac_D=1.0, pac_E=0.97,
    track_len=120.0, kappa_amp=0.8, n_sub=4,
)


def default_problem(**overrides) -> dict:
    """The small single-solve problem (K=256, M=16, T=30) with optional overrides."""
    p = {k: (list(v) if isinstance(v, list) else v) for k, v in _DEFAULTS.items()}
    for k, v in overrides.items():
        if k not in p:
            raise KeyError(f"unknown problem key {k!r}")
        p[k] = v
    return p


# ------------------------------------------------------------------------------------------------
# start poses on the ellipse track
# ------------------------------------------------------------------------------------------------
def _arclength_table(a: float, b: float, n: int = 4096):
    """Cumulative arc length of (a cos th, b sin th) at n+1 equally spaced th in [0, 2 pi]."""
    th = np.linspace(0.0, 2.0 * math.pi, n + 1)
    speed = np.hypot(a * np.sin(th), b * np.cos(th))
    seg = 0.5 * (speed[1:] + speed[:-1]) * (th[1] - th[0])
    return th, np.concatenate([[0.0], np.cumsum(seg)])


def pose_on_centerline(a: float, b: float, theta: float, vx: float = 5.0) -> np.ndarray:
    """State [X, Y, psi, vx, vy, r] on the centerline at parameter theta, heading along the
    counter-clockwise tangent."""
    X, Y = a * math.cos(theta), b * math.sin(theta)
    psi = math.atan2(b * math.cos(theta), -a * math.sin(theta))
    return np.array([X, Y, psi, vx, 0.0, 0.0])


def random_start(a: float, b: float, rng: np.random.Generator, vx: float = 5.0) -> np.ndarray:
    """Start pose with arc length uniform on [0, perimeter) (4096-point arc-length table)."""
    th, cum = _arclength_table(a, b)
    s = rng.uniform(0.0, cum[-1])
    theta = float(np.interp(s, cum, th))
    return pose_on_centerline(a, b, theta, vx)


# ------------------------------------------------------------------------------------------------
# the five workloads
# ------------------------------------------------------------------------------------------------
def config_small():
    """Plain solve, K=256, M=16, T=30, seed 1; start at (30, 0) heading +Y at 5 m/s, v = 0."""
    prob = default_problem(K=256, M=16, T=30, seed=1)
    x0 = pose_on_centerline(prob["ell_a"], prob["ell_b"], 0.0, 5.0)
    v = np.zeros((prob["T"], 2))
    return prob, x0, v


def config_paper_scale(seed: int = 2):
    """Paper-scale solve: K=4096, M=64, T=50, disturbance std x2, start uniform along the track."""
    base = default_problem()
    prob = default_problem(K=4096, M=64, T=50, seed=seed,
                           sigma_w=[2.0 * s for s in base["sigma_w"]])
    rng = np.random.default_rng(seed)
    x0 = random_start(prob["ell_a"], prob["ell_b"], rng)
    v = np.zeros((prob["T"], 2))
    return prob, x0, v


def config_shielded(delta: float = 0.05, gamma: float = 0.1, seed: int = 3000):
    """Shielded solve: the paper-scale problem with K=8192, M=128, T=60 and the repair on."""
    base = default_problem()
    prob = default_problem(K=8192, M=128, T=60, seed=seed, delta=delta, gamma=gamma,
                           sigma_w=[2.0 * s for s in base["sigma_w"]], shield_iters=2)
    rng = np.random.default_rng(seed)
    x0 = random_start(prob["ell_a"], prob["ell_b"], rng)
    v = np.zeros((prob["T"], 2))
    return prob, x0, v


def config_constrained(seed: int = 2):
    """The paper-scale solve with four half-space constraints on the state: a speed limit
    vx <= 6.5, the yaw rate within +-0.8 (two half-spaces) and vy + 0.5 r <= 1.0."""
    prob, x0, v = config_paper_scale(seed)
    a = np.zeros(24)
    a[3] = 1.0                 # vx
    a[6 + 5] = 1.0             # r
    a[12 + 5] = -1.0           # -r
    a[18 + 4], a[18 + 5] = 1.0, 0.5
    prob = dict(prob, n_con=4, con_a=list(a), con_b=[6.5, 0.8, 0.8, 1.0])
    return prob, x0, v


def config_batch(n: int = 64, seed: int = 4):
    """64 independent instances with K in {512..8192}, M in {16..256}, T uniform in [20, 80],
    ellipse semi-axes uniform 15-50 m, half-width 1.5-3 m, disturbance std x U[0.5, 3]."""
    rng = np.random.default_rng(seed)
    base = default_problem()
    out = []
    for i in range(n):
        K = int(rng.choice([512, 1024, 2048, 4096, 8192]))
        M = int(rng.choice([16, 32, 64, 128, 256]))
        T = int(rng.integers(20, 81))
        a = float(rng.uniform(15.0, 50.0))
        b = float(rng.uniform(15.0, 50.0))
        wT = float(rng.uniform(1.5, 3.0))
        mult = float(rng.uniform(0.5, 3.0))
        prob = default_problem(K=K, M=M, T=T, seed=seed * 1000 + i, ell_a=a, ell_b=b,
                               half_width=wT, sigma_w=[mult * s for s in base["sigma_w"]])
        x0 = random_start(a, b, rng)
        out.append((prob, x0, np.zeros((T, 2))))
    return out


def serving_fleet(n_vehicles: int = 256, seed: int = 5):
    """Vehicles of the serving workload, each with its own problem: ellipse track with semi-axes
    a ~ U[25, 35] m, b ~ U[18, 22] m and half-width 2 m (the small problem's track type), its own
    seed, and a start arc length uniform along its track.  Returns (problems, start arc lengths);
    K, M and delta of a problem are replaced per request."""
    rng = np.random.default_rng(seed)
    probs, s0 = [], []
    for veh in range(n_vehicles):
        a = float(rng.uniform(25.0, 35.0))
        b = float(rng.uniform(18.0, 22.0))
        probs.append(default_problem(T=50, seed=seed * 100000 + veh, ell_a=a, ell_b=b,
                                     half_width=2.0))
        _, cum = _arclength_table(a, b)
        s0.append(float(rng.uniform(0.0, cum[-1])))
    return probs, np.array(s0)


def serving_trace(fleet, duration_s: float = 60.0, rate_hz: float = 20.0, seed: int = 5,
                  K_range=(1024, 8192), M_range=(32, 128), delta_range=(0.01, 0.1),
                  speed: float = 5.0):
    """Poisson request trace of a fleet: per vehicle exponential inter-arrival times with mean
    1 / rate_hz over duration_s.  Each request draws K ~ U{K_range}, M ~ U{M_range} (inclusive
    integers) and delta ~ U(delta_range); its state estimate is the vehicle's pose on its
    centerline after driving `speed` m/s since t = 0.  Returns a dict of arrays sorted by arrival:
    t, vehicle, K, M, delta, x0 [n, 6]."""
    probs, s0 = fleet
    rng = np.random.default_rng(seed + 1)
    ts, vs = [], []
    for veh in range(len(probs)):
        t = rng.exponential(1.0 / rate_hz)
        while t < duration_s:
            ts.append(t)
            vs.append(veh)
            t += rng.exponential(1.0 / rate_hz)
    order = np.argsort(np.array(ts), kind="stable")
    t = np.array(ts)[order]
    veh = np.array(vs, dtype=np.int32)[order]
    n = t.shape[0]
    K = rng.integers(K_range[0], K_range[1] + 1, n).astype(np.int32)
    M = rng.integers(M_range[0], M_range[1] + 1, n).astype(np.int32)
    delta = rng.uniform(delta_range[0], delta_range[1], n)
    x0 = np.zeros((n, 6))
    tables = {}
    for i in range(n):
        p = probs[veh[i]]
        key = (p["ell_a"], p["ell_b"])
        if key not in tables:
            tables[key] = _arclength_table(*key)
        th, cum = tables[key]
        sarc = (s0[veh[i]] + speed * t[i]) % cum[-1]
        x0[i] = pose_on_centerline(p["ell_a"], p["ell_b"], float(np.interp(sarc, cum, th)), speed)
    return {"t": t, "vehicle": veh, "K": K, "M": M, "delta": delta, "x0": x0}


# ------------------------------------------------------------------------------------------------
# the paper's 8-state vehicle (vehicle = 1)
# ------------------------------------------------------------------------------------------------
def vehicle8_problem(**overrides) -> dict:
    """The 8-state single-track vehicle with wheel speeds, x = [vX, vY, r, wF, wR, epsi, eY, s],
    u = [steer, throttle].  The paper gives the AutoRally's size (1 m long, 22 kg) but none of
    its inertia, tire, wheel or track data, so the values are stated choices: a 22 kg car with
    lf = 0.34 m, lr = 0.23 m, Iz = 1.1 kg m^2, wheel radius 0.095 m, drive-line inertia 0.3 kg m^2
    per axle, 8 N m of rear drive torque at full throttle (throttle in [-1, 1]), the generic
    dry-road magic-formula coefficients B = 10, C = 1.9, D = 1, E = 0.97 for both slip
    directions with mu = 0.9, slip denominators floored at 2 m/s, four midpoint substeps per
    0.05 s period, and a closed synthetic track of length 120 m with curvature
    (2 pi / 120)(1 + 0.8 sin(4 pi s / 120)) (radii 10.6 m to 95 m); the paper's goal speed
    (6 m/s), lateral-deviation weight (0.1) and half-width (2 m)."""
    base = dict(vehicle=1, m=22.0, Iz=1.1, lf=0.34, lr=0.23, mu=0.9, g=9.81, v_min=2.0, dt=0.05,
                Rw=0.095, Iw=0.3, T_max=8.0, pac_B=10.0, pac_C=1.9, pac_D=1.0, pac_E=0.97,
                track_len=120.0, kappa_amp=0.8, n_sub=4,
                steer_max=0.4, accel_max=1.0, sigma_eps=[0.1, 0.3], sigma_w=[0.05, 0.05, 0.05],
                v_goal=6.0, q_vx=1.0, q_vy=0.0, q_r=0.0, q_ey=0.1, q_epsi=1.0,
                half_width=2.0, delta=0.05, gamma=0.2)
    base.update(overrides)
    return default_problem(**base)


def vehicle8_start(prob: dict, rng: np.random.Generator, vX: float = 5.0) -> np.ndarray:
    """Start on the centerline (eY = epsi = 0) at a path coordinate uniform along the track,
    rolling (wheel speeds vX / Rw) at vX."""
    s0 = rng.uniform(0.0, prob["track_len"])
    w = vX / prob["Rw"]
    return np.array([vX, 0.0, 0.0, w, w, 0.0, 0.0, s0])


def config_vehicle8(seed: int = 6):
    """The paper's largest BSS-MPPI setting of its Table 1 (1000 control samples x 20 particles,
    horizon 20) on the 8-state vehicle: K=1000, M=20, T=20, seeded start along the track."""
    prob = vehicle8_problem(K=1000, M=20, T=20, seed=seed)
    rng = np.random.default_rng(seed)
    x0 = vehicle8_start(prob, rng)
    v = np.zeros((prob["T"], 2))
    return prob, x0, v
