"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` import this
package.  It loads ``oracle/liboracle.so`` (building it with gcc when it is absent) and exposes the
oracle's C functions on numpy arrays.  It shares no code with the GPU library.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


class OrcParams(C.Structure):
    """Mirror of ``orc_params`` in bss_oracle.h (field order matters)."""
    _fields_ = [
        ("m", C.c_double), ("Iz", C.c_double), ("lf", C.c_double), ("lr", C.c_double),
        ("Cf", C.c_double), ("Cr", C.c_double), ("mu", C.c_double), ("g", C.c_double),
        ("v_min", C.c_double), ("dt", C.c_double),
        ("steer_max", C.c_double), ("accel_max", C.c_double),
        ("sigma_eps", C.c_double * 2), ("sigma_w", C.c_double * 3),
        ("K", C.c_int32), ("M", C.c_int32), ("T", C.c_int32),
        ("delta", C.c_double), ("gamma", C.c_double),
        ("backoff", C.c_int32),
        ("lambda_", C.c_double), ("gamma_u", C.c_double), ("v_goal", C.c_double),
        ("q_vx", C.c_double), ("q_vy", C.c_double), ("q_r", C.c_double), ("q_ey", C.c_double),
        ("q_epsi", C.c_double), ("C_cbf", C.c_double), ("C_obs", C.c_double),
        ("phi_scale", C.c_double),
        ("ell_a", C.c_double), ("ell_b", C.c_double), ("half_width", C.c_double),
        ("shield_iters", C.c_int32), ("shield_gmin", C.c_double), ("shield_fd", C.c_double),
        ("seed", C.c_uint64),
        ("belief", C.c_int32),
        ("crn", C.c_int32),
        ("sigma_w_speed", C.c_double),
        ("n_obs", C.c_int32), ("obs", C.c_double * 12),
        ("local_repair", C.c_int32),
        ("model", C.c_int32),
        ("lin_A", C.c_double * 36), ("lin_B", C.c_double * 12),
        ("n_con", C.c_int32), ("con_a", C.c_double * 24), ("con_b", C.c_double * 4),
        ("vehicle", C.c_int32),
        ("Rw", C.c_double), ("Iw", C.c_double), ("T_max", C.c_double),
        ("pac_B", C.c_double), ("pac_C", C.c_double), ("pac_D", C.c_double),
        ("pac_E", C.c_double),
        ("track_len", C.c_double), ("kappa_amp", C.c_double),
        ("n_sub", C.c_int32),
    ]


# one belief record: mean (6), position covariance (3), a_i^T Sigma a_i of the half-space
# constraints (4, zero beyond n_con)
NMOM = 13


def make_params(cfg: dict) -> OrcParams:
    """Build an ``OrcParams`` from a problem dict (keys as in ``workloads.default_problem``)."""
    if cfg.get("belief", 0) == 2 and cfg.get("M") != 12:
        raise ValueError("the sigma-point belief uses M = 12 points")
    if cfg.get("local_repair", 0) not in (0, 1, 2):
        raise ValueError("local_repair is 0, 1 or 2")
    if cfg.get("local_repair", 0) and cfg.get("shield_iters", 0) < 1:
        raise ValueError("the repair of the update needs shield_iters >= 1")
    if not 0 <= cfg.get("n_con", 0) <= 4:
        raise ValueError("n_con is 0..4")
    p = OrcParams()
    for name, _ in OrcParams._fields_:
        key = "lambda" if name == "lambda_" else name
        if key not in cfg:
            continue
        val = cfg[key]
        if name in ("sigma_eps", "sigma_w", "lin_A", "lin_B", "obs", "con_a", "con_b"):
            arr = getattr(p, name)
            flat = np.asarray(val, dtype=np.float64).ravel()
            for i, x in enumerate(flat):
                arr[i] = float(x)
        else:
            setattr(p, name, type(getattr(p, name))(val))
    return p


def _load():
    path = os.path.join(_HERE, "liboracle.so")
    if not os.path.exists(path):
        _build.build()
    lib = C.CDLL(path)
    P = C.POINTER(OrcParams)
    lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.orc_philox4x32_10.restype = None
    lib.orc_philox_many.argtypes = [_u32p, _u32p, _u32p, C.c_int64]
    lib.orc_philox_many.restype = None
    lib.orc_normals_many.argtypes = [C.c_uint64, _u32p, _f64p, C.c_int64]
    lib.orc_normals_many.restype = None
    lib.orc_uniform.argtypes = [C.c_uint32]
    lib.orc_uniform.restype = C.c_double
    lib.orc_normals.argtypes = [C.c_uint64, _u32p, _f64p]
    lib.orc_normals.restype = None
    lib.orc_disturbance_normals.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                            C.c_uint32, _f64p]
    lib.orc_disturbance_normals.restype = None
    lib.orc_backoff.argtypes = [C.c_double, C.c_int32]
    lib.orc_backoff.restype = C.c_double
    lib.orc_car_deriv.argtypes = [P, _f64p, _f64p, _f64p]
    lib.orc_car_deriv.restype = None
    lib.orc_model_step.argtypes = [P, _f64p, _f64p, _f64p]
    lib.orc_model_step.restype = None
    lib.orc_ellipse_sdf.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.POINTER(C.c_double), _f64p]
    lib.orc_ellipse_sdf.restype = None
    lib.orc_barrier.argtypes = [P, C.c_double, _f64p]
    lib.orc_barrier.restype = C.c_double
    lib.orc_stage_cost.argtypes = [P, _f64p]
    lib.orc_stage_cost.restype = C.c_double
    lib.orc_moments.argtypes = [_f64p, C.c_int32, _f64p]
    lib.orc_moments.restype = None
    lib.orc_full_cov.argtypes = [_f64p, C.c_int32, _f64p]
    lib.orc_full_cov.restype = None
    lib.orc_con_spreads.argtypes = [P, _f64p, _f64p]
    lib.orc_con_spreads.restype = None
    lib.orc_repair.argtypes = [P, C.c_double, _f64p, _f64p]
    lib.orc_repair.restype = None
    lib.orc_score.argtypes = [P, C.c_double, _f64p, _f64p, _f64p]
    lib.orc_score.restype = C.c_double
    lib.orc_rollout.argtypes = [P, C.c_double, C.c_uint32, C.c_int32, _f64p, C.c_void_p,
                                C.c_void_p, _f64p, _f64p, _f64p]
    lib.orc_rollout.restype = C.c_double
    lib.orc_propagate.argtypes = [P, C.c_uint32, C.c_int32, _f64p, C.c_void_p, C.c_void_p,
                                  _f64p, _f64p]
    lib.orc_propagate.restype = None
    lib.orc_update.argtypes = [P, _f64p, _f64p, _f64p, _f64p]
    lib.orc_update.restype = C.c_int32
    lib.orc_solve.argtypes = [P, C.c_uint32, _f64p, C.c_void_p, _f64p, C.c_void_p, C.c_void_p,
                              C.c_void_p, _f64p, C.c_int32]
    lib.orc_solve.restype = C.c_int32
    lib.orc_local_repair.argtypes = [P, C.c_uint32, _f64p, C.c_void_p, _f64p, _f64p, _f64p]
    lib.orc_local_repair.restype = None
    lib.orc_step_shift.argtypes = [C.c_int32, _f64p]
    lib.orc_step_shift.restype = None
    lib.orc_chol_psd6.argtypes = [_f64p, _f64p]
    lib.orc_chol_psd6.restype = None
    # the 8-state vehicle
    lib.orc8_magic.argtypes = [P, C.c_double]
    lib.orc8_magic.restype = C.c_double
    lib.orc8_tire.argtypes = [P, C.c_double, C.c_double, C.c_double, _f64p]
    lib.orc8_tire.restype = None
    lib.orc8_kappa.argtypes = [P, C.c_double]
    lib.orc8_kappa.restype = C.c_double
    lib.orc8_deriv.argtypes = [P, _f64p, _f64p, _f64p]
    lib.orc8_deriv.restype = None
    lib.orc8_step.argtypes = [P, _f64p, _f64p, _f64p]
    lib.orc8_step.restype = None
    lib.orc8_moments.argtypes = [_f64p, C.c_int32, _f64p]
    lib.orc8_moments.restype = None
    lib.orc8_barrier.argtypes = [P, C.c_double, _f64p]
    lib.orc8_barrier.restype = C.c_double
    lib.orc8_stage_cost.argtypes = [P, _f64p]
    lib.orc8_stage_cost.restype = C.c_double
    lib.orc8_repair.argtypes = [P, C.c_double, _f64p, _f64p]
    lib.orc8_repair.restype = None
    lib.orc8_score.argtypes = [P, C.c_double, _f64p, _f64p, _f64p]
    lib.orc8_score.restype = C.c_double
    lib.orc8_solve.argtypes = [P, C.c_uint32, _f64p, _f64p, C.c_void_p, C.c_void_p, C.c_void_p,
                               _f64p, C.c_int32]
    lib.orc8_solve.restype = C.c_int32
    return lib


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = _load()
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    """Philox4x32-10 of one counter (4 uint32) under one key (2 uint32)."""
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(np.ascontiguousarray(ctr, dtype=np.uint32),
                            np.ascontiguousarray(key, dtype=np.uint32), out)
    return out


def philox_many(ctr, seed):
    """Philox4x32-10 of counters ctr [n, 4] under the key (lo32 seed, hi32 seed)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros_like(ctr)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)
    lib().orc_philox_many(ctr, key, out, int(ctr.shape[0]))
    return out


def normals_many(seed, ctr):
    """Four Box-Muller normals per counter: [n, 4] float64."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32)
    z = np.zeros(ctr.shape, dtype=np.float64)
    lib().orc_normals_many(int(seed), ctr, z, int(ctr.shape[0]))
    return z


def normals(seed, ctr):
    z = np.zeros(4)
    lib().orc_normals(int(seed), np.ascontiguousarray(ctr, dtype=np.uint32), z)
    return z


def disturbance_normals(seed, s, k, t, m):
    """The three disturbance normals of particle m at step t of sample word k (solve index s)."""
    w = np.zeros(3)
    lib().orc_disturbance_normals(int(seed), int(s), int(k), int(t), int(m), w)
    return w


def uniform(r):
    return lib().orc_uniform(int(r))


def backoff(delta, kind=0):
    return lib().orc_backoff(float(delta), int(kind))


def car_deriv(cfg, x, u):
    p = make_params(cfg)
    dx = np.zeros(6)
    lib().orc_car_deriv(C.byref(p), np.ascontiguousarray(x, dtype=np.float64),
                        np.ascontiguousarray(u, dtype=np.float64), dx)
    return dx


def model_step(cfg, x, u):
    p = make_params(cfg)
    xn = np.zeros(6)
    lib().orc_model_step(C.byref(p), np.ascontiguousarray(x, dtype=np.float64),
                         np.ascontiguousarray(u, dtype=np.float64), xn)
    return xn


def ellipse_sdf(a, b, X, Y):
    sd = C.c_double()
    n = np.zeros(2)
    lib().orc_ellipse_sdf(float(a), float(b), float(X), float(Y), C.byref(sd), n)
    return sd.value, n


def _records(mom, con_var=None):
    """Belief records [..., NMOM] from position records [..., 9] and the constraint variances
    [..., n_con] (zero when not given)."""
    mom = np.asarray(mom, dtype=np.float64)
    rec = np.zeros(mom.shape[:-1] + (NMOM,))
    rec[..., :9] = mom[..., :9]
    if con_var is not None:
        cv = np.asarray(con_var, dtype=np.float64)
        rec[..., 9:9 + cv.shape[-1]] = cv
    return rec


def barrier(cfg, nu, mom, con_var=None):
    """Belief heuristic h of one record (9 entries), with the variances a_i^T Sigma a_i of the
    half-space constraints when there are any."""
    p = make_params(cfg)
    return lib().orc_barrier(C.byref(p), float(nu), _records(mom, con_var))


def stage_cost(cfg, mom):
    p = make_params(cfg)
    return lib().orc_stage_cost(C.byref(p), np.ascontiguousarray(mom, dtype=np.float64))


def moments(particles):
    particles = np.ascontiguousarray(particles, dtype=np.float64)
    out = np.zeros(9)
    lib().orc_moments(particles, int(particles.shape[0]), out)
    return out


def full_cov(particles):
    """Unbiased full 6x6 covariance of a particle set [M][6] (zero for one particle)."""
    particles = np.ascontiguousarray(particles, dtype=np.float64)
    out = np.zeros(36)
    lib().orc_full_cov(particles, int(particles.shape[0]), out)
    return out.reshape(6, 6)


def con_spreads(cfg, cov):
    """a_i^T Sigma a_i of the half-space constraints (four entries, zero beyond n_con)."""
    p = make_params(cfg)
    rec = np.zeros(NMOM)
    lib().orc_con_spreads(C.byref(p), np.ascontiguousarray(cov, dtype=np.float64).ravel(), rec)
    return rec[9:]


def repair(cfg, nu, mom_t, u, con_var=None):
    p = make_params(cfg)
    uu = np.array(u, dtype=np.float64)
    lib().orc_repair(C.byref(p), float(nu), _records(mom_t, con_var), uu)
    return uu


def score(cfg, nu, mom, u, v, con_var=None):
    """Trajectory cost of one sample from injected moments [T+1][9] (and constraint variances
    [T+1][n_con]), controls [T][2], v [T][2]."""
    p = make_params(cfg)
    return lib().orc_score(C.byref(p), float(nu), _records(mom, con_var),
                           np.ascontiguousarray(u, dtype=np.float64),
                           np.ascontiguousarray(v, dtype=np.float64))


def _split(rec, n_con):
    return rec[..., :9], rec[..., 9:9 + n_con]


def rollout(cfg, s, k, x0, v, Sigma0=None, with_con=False):
    """One sample's rollout: returns (S_k, u [T][2], moments [T+1][9]), and the constraint
    variances [T+1][n_con] as a fourth item with with_con."""
    p = make_params(cfg)
    T = cfg["T"]
    nu = backoff(cfg["delta"], cfg.get("backoff", 0))
    u = np.zeros((T, 2))
    mom = np.zeros((T + 1, NMOM))
    L0 = None
    S0 = None
    if Sigma0 is not None:
        S0 = np.ascontiguousarray(Sigma0, dtype=np.float64)
        L0 = np.linalg.cholesky(S0 + 0.0) if np.any(S0 != 0) else None
    Sk = lib().orc_rollout(C.byref(p), nu, int(s), int(k),
                           np.ascontiguousarray(x0, dtype=np.float64), _ptr(S0),
                           _ptr(None if L0 is None else np.ascontiguousarray(L0)),
                           np.ascontiguousarray(v, dtype=np.float64), u, mom)
    m9, cv = _split(mom, cfg.get("n_con", 0))
    return (Sk, u, m9, cv) if with_con else (Sk, u, m9)


def propagate(cfg, s, k, x0, u, Sigma0=None, with_con=False):
    """Belief trajectory [T+1][9] of sample k under the given controls u [T][2] (and the
    constraint variances [T+1][n_con] with with_con)."""
    p = make_params(cfg)
    T = cfg["T"]
    mom = np.zeros((T + 1, NMOM))
    S0 = None if Sigma0 is None else np.ascontiguousarray(Sigma0, dtype=np.float64)
    L0 = None
    if S0 is not None and np.any(S0 != 0):
        L0 = np.ascontiguousarray(np.linalg.cholesky(S0))
    lib().orc_propagate(C.byref(p), int(s), int(k), np.ascontiguousarray(x0, dtype=np.float64),
                        _ptr(S0), _ptr(L0), np.ascontiguousarray(u, dtype=np.float64), mom)
    m9, cv = _split(mom, cfg.get("n_con", 0))
    return (m9, cv) if with_con else m9


def update(cfg, S, u, v):
    """MPPI update from injected costs [K] and controls [K][T][2]; returns (rc, v+, stats)."""
    p = make_params(cfg)
    vv = np.array(v, dtype=np.float64)
    stats = np.zeros(4)
    rc = lib().orc_update(C.byref(p), np.ascontiguousarray(S, dtype=np.float64),
                          np.ascontiguousarray(u, dtype=np.float64), vv, stats)
    return rc, vv, stats


def solve(cfg, s, x0, v, Sigma0=None, want_traces=True, nthreads=None):
    """One full solve.  Returns dict(rc, v (updated), u, mom, con_var, S, stats)."""
    p = make_params(cfg)
    K, T = cfg["K"], cfg["T"]
    vv = np.array(v, dtype=np.float64).reshape(T, 2).copy()
    stats = np.zeros(4)
    u = np.zeros((K, T, 2)) if want_traces else None
    mom = np.zeros((K, T + 1, NMOM)) if want_traces else None
    S = np.zeros(K)
    S0 = None if Sigma0 is None else np.ascontiguousarray(Sigma0, dtype=np.float64)
    if nthreads is None:
        nthreads = min(8, os.cpu_count() or 1)
    rc = lib().orc_solve(C.byref(p), int(s), np.ascontiguousarray(x0, dtype=np.float64),
                         _ptr(S0), vv, _ptr(u), _ptr(mom), _ptr(S), stats, int(nthreads))
    m9, cv = _split(mom, cfg.get("n_con", 0)) if want_traces else (None, None)
    return {"rc": rc, "v": vv, "u": u, "mom": m9, "con_var": cv, "S": S, "stats": stats}


def local_repair(cfg, s, x0, v_plus, Sigma0=None):
    """Repair of an updated sequence v+ [T][2] from the estimate (solve index s): returns
    (v_safe [T][2], the repair rollout's belief [T+1][9])."""
    p = make_params(cfg)
    T = cfg["T"]
    v_safe = np.zeros((T, 2))
    mom = np.zeros((T + 1, NMOM))
    S0 = None if Sigma0 is None else np.ascontiguousarray(Sigma0, dtype=np.float64)
    lib().orc_local_repair(C.byref(p), int(s), np.ascontiguousarray(x0, dtype=np.float64),
                           _ptr(S0), np.ascontiguousarray(v_plus, dtype=np.float64), v_safe, mom)
    return v_safe, mom[:, :9]


def step_shift(v):
    vv = np.array(v, dtype=np.float64)
    lib().orc_step_shift(int(vv.shape[0]), vv)
    return vv


def chol_psd6(A):
    """Semi-definite lower factor of a 6x6 matrix (the re-sampling draw's factor)."""
    L = np.zeros(36)
    lib().orc_chol_psd6(np.ascontiguousarray(A, dtype=np.float64).ravel(), L)
    return L.reshape(6, 6)


# ---- the paper's 8-state vehicle (vehicle = 1): x = [vX, vY, r, wF, wR, epsi, eY, s] ----------
NREC8 = 9


def magic8(cfg, z):
    return lib().orc8_magic(C.byref(make_params(cfg)), float(z))


def tire8(cfg, Fz, slip, alpha):
    F = np.zeros(2)
    lib().orc8_tire(C.byref(make_params(cfg)), float(Fz), float(slip), float(alpha), F)
    return F


def kappa8(cfg, s):
    return lib().orc8_kappa(C.byref(make_params(cfg)), float(s))


def deriv8(cfg, x, u):
    dx = np.zeros(8)
    lib().orc8_deriv(C.byref(make_params(cfg)), np.ascontiguousarray(x, dtype=np.float64),
                     np.ascontiguousarray(u, dtype=np.float64), dx)
    return dx


def model_step8(cfg, x, u):
    xn = np.zeros(8)
    lib().orc8_step(C.byref(make_params(cfg)), np.ascontiguousarray(x, dtype=np.float64),
                    np.ascontiguousarray(u, dtype=np.float64), xn)
    return xn


def moments8(particles):
    part = np.ascontiguousarray(particles, dtype=np.float64)
    rec = np.zeros(NREC8)
    lib().orc8_moments(part.ravel(), part.shape[0], rec)
    return rec


def barrier8(cfg, nu, rec):
    return lib().orc8_barrier(C.byref(make_params(cfg)), float(nu),
                              np.ascontiguousarray(rec, dtype=np.float64))


def stage_cost8(cfg, rec):
    return lib().orc8_stage_cost(C.byref(make_params(cfg)),
                                 np.ascontiguousarray(rec, dtype=np.float64))


def repair8(cfg, nu, rec_t, u):
    uu = np.array(u, dtype=np.float64)
    lib().orc8_repair(C.byref(make_params(cfg)), float(nu),
                      np.ascontiguousarray(rec_t, dtype=np.float64), uu)
    return uu


def score8(cfg, nu, rec, u, v):
    return lib().orc8_score(C.byref(make_params(cfg)), float(nu),
                            np.ascontiguousarray(rec, dtype=np.float64).ravel(),
                            np.ascontiguousarray(u, dtype=np.float64).ravel(),
                            np.ascontiguousarray(v, dtype=np.float64).ravel())


def solve8(cfg, s, x0, v, want_traces=True, nthreads=None):
    """One solve of the 8-state problem from the estimate x0 [8] (known exactly) and warm start
    v [T][2]: returns dict(v=v+, u [K][T][2], mom [K][T+1][9], S [K], stats [4], status)."""
    p = make_params(cfg)
    K, T = cfg["K"], cfg["T"]
    vv = np.array(v, dtype=np.float64).reshape(T, 2).copy()
    stats = np.zeros(4)
    out = {}
    if want_traces:
        u = np.zeros((K, T, 2))
        mom = np.zeros((K, T + 1, NREC8))
        S = np.zeros(K)
        ptrs = [_ptr(u), _ptr(mom), _ptr(S)]
    else:
        ptrs = [None, None, None]
    rc = lib().orc8_solve(C.byref(p), int(s), np.ascontiguousarray(x0, dtype=np.float64), vv,
                          *ptrs, stats, int(nthreads or os.cpu_count() or 1))
    out.update(v=vv, stats=stats, status=int(rc))
    if want_traces:
        out.update(u=u, mom=mom, S=S)
    return out
