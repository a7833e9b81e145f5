"""GPU-vs-oracle parity of the HIP path (run on an MI355X; every call goes through the C ABI).

Staged checks give each stage the other side's inputs so errors do not compound; end-to-end
checks compare whole solves.  Tolerances (floating point; integer work is bit-exact):
  controls v+      : max |dv| / u_max <= 1e-4 (full-scale relative, per control channel)
  moments          : |d mom[k,t,i]| / max_t |mom_ref[k,t,i]| <= 1e-3 (trajectory-scale relative)
  costs            : |dS_k| / |S_k| <= 1e-3
The single-precision rollout against the double-precision oracle is the only source of
difference; staged double-precision stages are held to ~1e-12.
"""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2408_00494_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2408_00494_amd as bss  # noqa: E402
import sensitivity as SENS  # noqa: E402

NTHREADS = min(16, os.cpu_count() or 1)


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def ctrl_err(v_gpu, v_ref, prob):
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    return float(np.max(np.abs(np.asarray(v_gpu) - v_ref) / scale))


def mom_err(m_gpu, m_ref):
    """|d| / max_t |ref| per record entry and sample.  The off-diagonal position covariance S_XY
    is bounded by sqrt(S_XX S_YY), so it is measured against at least the geometric mean of the
    spans of S_XX and S_YY: over a million samples some have position spreads that are nearly
    uncorrelated by chance, and their S_XY span sits at the rounding level of the block."""
    span = np.max(np.abs(m_ref), axis=1, keepdims=True)
    span[..., 7] = np.maximum(span[..., 7], np.sqrt(span[..., 6] * span[..., 8]))
    span = np.where(span > 0, span, 1.0)
    return float(np.max(np.abs(m_gpu - m_ref) / span))


def cost_err(S_gpu, S_ref):
    return float(np.max(np.abs(S_gpu - S_ref) / np.abs(S_ref)))


# ================================= random numbers (bit-exact) ==================================
def _counters_of(prob, s, n_sample=None, rng=None):
    """Counters a solve of `prob` at solve index s draws (tag 0: (t, 0, k); tag 1: (t, 3q + b, k)
    for the particle quads q < ceil(M / 4) and b < 3)."""
    K, M, T = prob["K"], prob["M"], prob["T"]
    nb = 3 * ((M + 3) // 4)
    if n_sample is None:
        t, m, k = np.meshgrid(np.arange(T), np.arange(nb), np.arange(K), indexing="ij")
        t, m, k = t.ravel(), m.ravel(), k.ravel()
        te, ke = np.meshgrid(np.arange(T), np.arange(K), indexing="ij")
        te, ke = te.ravel(), ke.ravel()
    else:
        t, m, k = rng.integers(0, T, n_sample), rng.integers(0, nb, n_sample), rng.integers(0, K, n_sample)
        te, ke = rng.integers(0, T, n_sample), rng.integers(0, K, n_sample)
    w = np.stack([t, m, k, np.full_like(t, (1 << 28) | (s & 0x0FFFFFFF))], axis=1)
    e = np.stack([te, np.zeros_like(te), ke, np.full_like(te, s & 0x0FFFFFFF)], axis=1)
    return np.concatenate([w, e]).astype(np.uint32)


def test_philox_bit_exact_on_solve_counters():
    prob, _, _ = W.config_small()
    rng = np.random.default_rng(0)
    sets = [(_counters_of(prob, 0), prob["seed"]), (_counters_of(prob, 77), prob["seed"])]
    p2, _, _ = W.config_paper_scale()
    sets.append((_counters_of(p2, 5, 400000, rng), p2["seed"]))
    p3, _, _ = W.config_shielded()
    sets.append((_counters_of(p3, 3, 400000, rng), p3["seed"]))
    for ctr, seed in sets:
        got = bss.dev_philox(seed, dev(ctr.view(np.int32))).cpu().numpy().view(np.uint32)
        want = oracle.philox_many(ctr, seed)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("K,M,T,lanes,ppl,crn", [
    (5, 13, 4, 16, 1, False),    # one particle per lane: lane quads share a particle quad
    (3, 30, 3, 16, 2, False),    # two per lane, ragged last quad
    (4, 64, 3, 16, 4, False),    # the paper-scale shape
    (3, 37, 2, 16, 4, False),    # ragged M with whole quads per lane
    (3, 128, 2, 16, 8, False),   # the shielded shape (two quads per lane)
    (2, 300, 2, 64, 8, False),   # 64 lanes, ragged
    (3, 16, 3, 8, 2, True),      # common random numbers (sample word 0 for every sample)
    (2, 20, 2, 32, 1, False),
])
def test_solve_noise_path_matches_oracle(K, M, T, lanes, ppl, crn):
    """The solve kernel's disturbance path (shared first rounds, per-block tails, quad dealing,
    lane placement) against the oracle: every Philox word bit-exact, every dealt normal within
    the single-precision Box-Muller bound."""
    seed, s = 0x1234ABCD9876, 19
    w, words = bss.dev_disturbance(seed, s, K, M, T, lanes, ppl, crn)
    w = w.cpu().numpy().astype(np.float64)
    words = words.cpu().numpy().view(np.uint32)
    nblk = 3 * ((M + 3) // 4)
    t, b, k = np.meshgrid(np.arange(T), np.arange(nblk), np.arange(K), indexing="ij")
    kw = np.zeros_like(k) if crn else k
    ctr = np.stack([t.ravel(), b.ravel(), kw.ravel(),
                    np.full(t.size, (1 << 28) | s)], axis=1).astype(np.uint32)
    want = oracle.philox_many(ctr, seed).reshape(T, nblk, K, 4).transpose(2, 0, 1, 3)
    assert np.array_equal(words, want)
    err = 0.0
    for kk in range(K):
        for tt in range(T):
            for m in range(M):
                ref = oracle.disturbance_normals(seed, s, 0 if crn else kk, tt, m)
                err = max(err, float(np.max(np.abs(w[kk, tt, m] - ref))))
    assert err <= 2e-6, err


def test_philox_known_answers_on_device():
    rows = [[0, 0, 0, 0, 0, 0], [0xFFFFFFFF] * 6,
            [0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344, 0xa4093822, 0x299f31d0]]
    for r in rows:
        ctr = np.array([r[:4]], dtype=np.uint32)
        seed = r[4] | (r[5] << 32)
        got = bss.dev_philox(seed, dev(ctr.view(np.int32))).cpu().numpy().view(np.uint32)
        assert np.array_equal(got[0], oracle.philox(r[:4], r[4:6]))


def test_normals_match_oracle():
    prob, _, _ = W.config_small()
    ctr = _counters_of(prob, 0)
    z_gpu = bss.dev_normals(prob["seed"], dev(ctr.view(np.int32))).cpu().numpy().astype(np.float64)
    z_ref = oracle.normals_many(prob["seed"], ctr)
    err = np.max(np.abs(z_gpu - z_ref))
    assert err <= 2e-6, err


# ====================================== dynamics =============================================
def test_model_step_matches_oracle():
    prob, _, _ = W.config_small()
    rng = np.random.default_rng(1)
    n = 4096
    x = np.column_stack([rng.uniform(-40, 40, n), rng.uniform(-40, 40, n), rng.uniform(-7, 7, n),
                         rng.uniform(0.5, 12, n), rng.normal(0, 1.0, n), rng.normal(0, 0.8, n)])
    u = np.column_stack([rng.uniform(-0.4, 0.4, n), rng.uniform(-4, 4, n)])
    x32, u32 = x.astype(np.float32), u.astype(np.float32)
    got = bss.dev_model_step(prob, dev(x32), dev(u32)).cpu().numpy().astype(np.float64)
    want = np.array([oracle.model_step(prob, x32[i].astype(np.float64), u32[i].astype(np.float64))
                     for i in range(n)])
    # per-component scale: position/heading change over one step, velocities
    d = np.abs(got - want)
    step = np.abs(want - x32.astype(np.float64))
    tol = 2e-6 * (np.abs(want) + 1.0) + 1e-5 * step
    assert np.all(d <= tol), float(np.max(d / tol))


def test_sdf_matches_oracle():
    rng = np.random.default_rng(2)
    for a, b in ((30.0, 20.0), (18.0, 47.0), (25.0, 25.0)):
        th = rng.uniform(0, 2 * np.pi, 3000)
        off = rng.uniform(-5, 5, 3000)
        pts = np.column_stack([(a + off) * np.cos(th), (b + off) * np.sin(th)])
        pts = np.concatenate([pts, [[a, 0.0], [0.0, b], [a + 1, 0], [0, -b - 1], [3.0, 0.0],
                                    [0.0, 2.0], [a - 0.5, 1e-12], [1e-13, b - 0.3]]])
        got = bss.dev_sdf(a, b, dev(pts)).cpu().numpy()
        for i, (X, Y) in enumerate(pts):
            sd, n = oracle.ellipse_sdf(a, b, X, Y)
            assert abs(got[i, 0] - sd) <= 1e-10, (a, b, X, Y, got[i], sd)
            assert np.all(np.abs(got[i, 1:] - n) <= 1e-8), (a, b, X, Y, got[i], n)


# ================================ score, update, repair (FP64) ================================
def test_score_from_injected_moments():
    prob, x0, v = W.config_small()
    prob = dict(prob, K=64)
    ref = oracle.solve(prob, 0, x0, v)
    u32 = ref["u"].astype(np.float32)
    S_gpu = bss.dev_score(prob, dev(ref["mom"]), dev(u32), dev(v)).cpu().numpy()
    nu = oracle.backoff(prob["delta"])
    S_ref = np.array([oracle.score(prob, nu, ref["mom"][k], u32[k].astype(np.float64), v)
                      for k in range(prob["K"])])
    assert np.max(np.abs(S_gpu - S_ref) / np.abs(S_ref)) <= 1e-12


def test_update_from_injected_costs():
    rng = np.random.default_rng(3)
    for K, T, lam in ((256, 30, 1.0), (4096, 50, 1.0), (1000, 7, 25.0), (300, 80, 0.05)):
        prob = W.default_problem(K=K, T=T, **{"lambda": lam})
        S = rng.uniform(20, 60, K)
        S[rng.integers(0, K, 3)] = np.nan
        u = rng.normal(size=(K, T, 2)).astype(np.float32)
        v = rng.normal(size=(T, 2))
        v_gpu, st_gpu = bss.dev_update(prob, dev(S), dev(u), dev(v))
        rc, v_ref, st_ref = oracle.update(prob, S, u.astype(np.float64), v)
        assert rc == 0
        assert np.max(np.abs(v_gpu.cpu().numpy() - v_ref)) <= 1e-12
        st = st_gpu.cpu().numpy()
        assert st[0] == pytest.approx(st_ref[0], rel=1e-15)
        assert st[1] == pytest.approx(st_ref[1], rel=1e-12)
        assert st[2] == pytest.approx(st_ref[2], rel=1e-12)
        assert st[3] == st_ref[3] and st[4] == 0.0
    # every cost non-finite: v unchanged, status 5
    prob = W.default_problem(K=100, T=5)
    v = rng.normal(size=(5, 2))
    v_gpu, st = bss.dev_update(prob, dev(np.full(100, np.inf)), dev(np.zeros((100, 5, 2), np.float32)),
                               dev(v))
    assert np.array_equal(v_gpu.cpu().numpy(), v) and st.cpu().numpy()[4] == 5.0


def test_repair_from_injected_beliefs():
    prob = W.default_problem(shield_iters=3, gamma=0.05)
    rng = np.random.default_rng(4)
    a = prob["ell_a"]
    n = 300
    mom = np.zeros((n, 9))
    for i in range(n):
        mom[i] = [a + rng.uniform(-2.5, 2.5), rng.uniform(-1, 1), np.pi / 2 + rng.uniform(-0.4, 0.4),
                  rng.uniform(3, 8), rng.normal() * 0.2, rng.normal() * 0.2, 0.003, 0.0005, 0.002]
    u = rng.uniform([-0.4, -4], [0.4, 4], size=(n, 2))
    got = bss.dev_repair(prob, dev(mom), dev(u)).cpu().numpy()
    nu = oracle.backoff(prob["delta"])
    want = np.array([oracle.repair(prob, nu, mom[i], u[i]) for i in range(n)])
    assert np.sum(np.any(got != u, axis=1)) > 10     # the repair acted on some controls
    # the projection divides by |dr/du|^2 from central differences, which turns last-bit
    # differences of the two libm's (atan, sin, cos) into ~1e-7 differences where the gradient
    # is small; the bound is full-scale relative 1e-6 per channel
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    assert np.max(np.abs(got - want) / scale) <= 1e-6


# ======================================== end to end ==========================================
def _compare_solve(prob, x0, v, s=0, Sigma0=None, lanes=0, ctrl_tol=1e-4):
    solver = bss.Solver(prob, lanes=lanes)
    solver.set_controls(v)
    solver.solve_index = s
    u0, info = solver.solve(x0, Sigma0)
    b = solver.buffers()
    got = {"v": solver.get_controls(), "u": b["u"].cpu().numpy().astype(np.float64),
           "mom": b["mom"].cpu().numpy(), "S": b["S"].cpu().numpy()}
    solver.close()
    ref = oracle.solve(prob, s, x0, v, Sigma0=Sigma0, nthreads=NTHREADS)
    errs = {"u": float(np.max(np.abs(got["u"] - ref["u"]))),
            "mom": mom_err(got["mom"], ref["mom"]),
            "S": cost_err(got["S"], ref["S"]),
            "v": ctrl_err(got["v"], ref["v"], prob)}
    print(f"K={prob['K']} M={prob['M']} T={prob['T']} lanes={info['lanes']}x{info['ppl']} "
          f"ess={info['ess']:.3f} errs={errs}", flush=True)
    assert errs["u"] <= 1e-5
    assert errs["mom"] <= 1e-3
    assert errs["S"] <= 1e-3
    assert errs["v"] <= ctrl_tol
    assert np.allclose(u0, got["v"][0], atol=0, rtol=0)
    return got, ref, info


def test_small_solve_matches_oracle():
    prob, x0, v = W.config_small()
    _compare_solve(prob, x0, v)


@pytest.mark.parametrize("lanes", [8, 16, 32, 64])
def test_every_launch_shape_matches_oracle(lanes):
    prob, x0, v = W.config_small()
    _compare_solve(dict(prob, K=96), x0, v, s=3, lanes=lanes)


def test_closed_loop_sequence_matches_oracle():
    """Five receding-horizon periods: solve, apply u0 to a noise-free plant, shift the warm start;
    the oracle is fed the same states (taken from the GPU run) at every period."""
    prob, x0, v = W.config_small()
    prob = dict(prob, K=128)
    solver = bss.Solver(prob)
    v_ref = v.copy()
    x = x0.copy()
    for s in range(5):
        u0, _ = solver.solve(x)
        ref = oracle.solve(prob, s, x, v_ref, nthreads=NTHREADS)
        v_gpu = solver.get_controls()
        assert ctrl_err(v_gpu, ref["v"], prob) <= 1e-4
        v_ref = oracle.step_shift(v_gpu)
        solver.step_shift()
        assert np.array_equal(solver.get_controls(), v_ref)
        x = oracle.model_step(prob, x, u0)
    solver.close()


def test_paper_scale_solve_matches_oracle():
    """K=4096, M=64, T=50, disturbance x2, random start on the track (the benchmark workload)."""
    prob, x0, v = W.config_paper_scale()
    _compare_solve(prob, x0, v, s=1)


def test_shielded_solve_matches_oracle():
    """K=8192, M=128, T=60 with the shield repair (delta=0.05, gamma=0.1).

    Inside a sample the repair feeds the belief of step t back into u_t, so single- vs
    double-precision particle differences are re-amplified at every step of the horizon.  The
    implementation is therefore checked stage by stage on the other side's inputs (the repair
    from the GPU's own belief and pre-repair control to 1e-6, the propagation under the GPU's
    repaired controls to 1e-3), and end to end against the method's own sensitivity (the oracle
    against itself with the estimate moved by ~1e-6; tests/sensitivity.py)."""
    prob, x0, v = W.config_shielded(delta=0.05, gamma=0.1)
    s = 2
    solver = bss.Solver(prob)
    solver.set_controls(v)
    solver.solve_index = s
    solver.solve(x0)
    b = solver.buffers()
    got = {"u": b["u"].cpu().numpy().astype(np.float64), "mom": b["mom"].cpu().numpy(),
           "S": b["S"].cpu().numpy(), "v": solver.get_controls()}
    solver.close()
    ref = oracle.solve(prob, s, x0, v, nthreads=NTHREADS)
    span = np.max(np.abs(ref["mom"]), axis=1, keepdims=True)
    per_k = np.max(np.abs(got["mom"] - ref["mom"]) / np.where(span > 0, span, 1.0), axis=(1, 2))

    # the repair acted on this workload
    eps_only = oracle.solve(dict(prob, shield_iters=0), s, x0, v, nthreads=NTHREADS)
    assert np.mean(np.any(np.abs(ref["u"] - eps_only["u"]) > 1e-12, axis=2)) > 1e-3

    # stage checks on the worst and on random samples.  The repair stage starts from the GPU's
    # own pre-repair control (its single-precision clip(v + sigma z) with the device normals), so
    # it compares the double-precision repair alone.
    rng = np.random.default_rng(0)
    ks = np.unique(np.concatenate([np.argsort(per_k)[-16:], rng.integers(0, prob["K"], 48)]))
    nu = oracle.backoff(prob["delta"])
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    ctr = np.array([[t, 0, k, s] for k in ks for t in range(prob["T"])], dtype=np.uint32)
    z = bss.dev_normals(prob["seed"], dev(ctr.view(np.int32))).cpu().numpy()
    sig32 = np.array(prob["sigma_eps"], dtype=np.float32)
    worst_rep, worst_prop = 0.0, 0.0
    row = 0
    for k in ks:
        for t in range(prob["T"]):
            v32 = v[t].astype(np.float32)
            # fmaf(sigma, z, v) in single precision (exact product, one rounding)
            pre = (sig32.astype(np.float64) * z[row, :2].astype(np.float64)
                   + v32.astype(np.float64)).astype(np.float32)
            pre = np.clip(pre, -scale.astype(np.float32), scale.astype(np.float32))
            row += 1
            u_rep = oracle.repair(prob, nu, got["mom"][k, t], pre.astype(np.float64))
            u_rep32 = u_rep.astype(np.float32).astype(np.float64)
            worst_rep = max(worst_rep, float(np.max(np.abs(u_rep32 - got["u"][k, t]) / scale)))
        mom_k = oracle.propagate(prob, s, int(k), x0, got["u"][k])
        worst_prop = max(worst_prop, mom_err(got["mom"][k:k + 1], mom_k[None]))
    print(f"shield stages: repair {worst_rep:.2e}  propagation {worst_prop:.2e}", flush=True)
    assert worst_rep <= 1e-6
    assert worst_prop <= 1e-3

    # end to end, against the oracle's own sensitivity
    gpu = SENS.drift(prob, got, ref)
    own = SENS.self_drift(prob, s, x0, v, ref, nthreads=NTHREADS)
    SENS.check(gpu, own, "shielded workload")


@pytest.mark.parametrize("K,M,T,lanes", [(1, 1, 1, 0), (3, 13, 7, 8), (257, 16, 30, 0),
                                         (5, 512, 4, 64), (2, 37, 256, 16), (70, 2, 3, 32),
                                         (1 << 20, 16, 3, 0), (9, 512, 256, 0)])
def test_edge_sizes_match_oracle(K, M, T, lanes):
    """Ragged and extreme sizes, among them the maxima K = 2^20, M = 512 (64 lanes x 8) and
    T = 256 together with M = 512."""
    prob, x0, _ = W.config_small()
    prob = dict(prob, K=K, M=M, T=T)
    v = np.column_stack([0.05 * np.sin(np.arange(T)), 0.5 * np.cos(np.arange(T))])
    _compare_solve(prob, x0, v, s=9, lanes=lanes)


@pytest.mark.parametrize("K,M,T,ppl", [(4096, 64, 50, 4), (4096, 64, 50, 2), (333, 37, 23, 8),
                                       (70, 5, 9, 1), (3, 200, 4, 4)])
def test_noise_split_is_bitwise_identical(K, M, T, ppl):
    """Generating the disturbance normals in separate waves changes no result bit."""
    prob, x0, _ = W.config_paper_scale()
    prob = dict(prob, K=K, M=M, T=T)
    v = np.column_stack([0.05 * np.sin(np.arange(T)), 0.5 * np.cos(np.arange(T))])
    out = []
    for split in (0, 1):
        s = bss.Solver(prob)
        s.set_shape(ppl=ppl, split=split)
        s.set_controls(v)
        s.solve_index = 7
        s.solve(x0)
        s.solve(x0)                 # second solve reads the first one's update
        b = s.buffers()
        out.append((s.get_controls(), b["mom"].cpu().numpy(), b["S"].cpu().numpy(),
                    b["u"].cpu().numpy()))
        s.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("belief,K,M,T,ppl", [(1, 4096, 64, 50, 4), (1, 333, 37, 23, 2),
                                              (1, 70, 5, 9, 1), (2, 512, 12, 30, 1),
                                              (1, 200, 30, 12, 2)])
def test_resampling_noise_split_is_bitwise_identical(belief, K, M, T, ppl):
    """With the noise split the noise waves also draw the re-sampling normals (belief 1) ahead of
    the integrating waves; no result bit changes (sigma points: the integrating waves use no
    normals)."""
    prob, x0, _ = W.config_paper_scale()
    prob = dict(prob, K=K, M=M, T=T, belief=belief)
    v = np.column_stack([0.05 * np.sin(np.arange(T)), 0.5 * np.cos(np.arange(T))])
    out = []
    for split in (0, 1):
        s = bss.Solver(prob)
        s.set_shape(ppl=ppl, split=split)
        assert s.info()["split"] == bool(split)
        s.set_controls(v)
        s.solve_index = 7
        s.solve(x0)
        s.solve(x0)
        b = s.buffers()
        out.append((s.get_controls(), b["mom"].cpu().numpy(), b["S"].cpu().numpy(),
                    b["u"].cpu().numpy()))
        s.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("K,M,T,shape", [(1000, 20, 20, (32, 1)), (512, 64, 30, (64, 1)),
                                         (2048, 32, 25, (32, 1)), (4096, 64, 20, (16, 4)),
                                         (256, 16, 30, (16, 1))])
def test_default_shape_of_small_launches_matches_oracle(K, M, T, shape):
    """The automatic launch shape spreads the particles of a launch with fewer sample lanes than
    one wave per SIMD over more lanes (fewer per lane); every shape meets the oracle bars."""
    prob, x0, _ = W.config_small()
    prob = dict(prob, K=K, M=M, T=T, seed=K + M)
    t = np.arange(T)
    v = np.column_stack([0.05 * np.sin(0.3 * t), 0.5 * np.cos(0.2 * t)])
    solver = bss.Solver(prob)
    assert (solver.info()["lanes"], solver.info()["ppl"]) == shape
    solver.close()
    _compare_solve(prob, x0, v, s=2)


def test_cantelli_backoff_solve_matches_oracle():
    """Distribution-free back-off nu = sqrt((1 - delta)/delta) (Remark 1) instead of the Gaussian
    quantile: larger nu, so the barrier binds earlier."""
    prob, x0, v = W.config_small()
    prob = dict(prob, K=128, backoff=1, delta=0.1)
    assert abs(bss.backoff(prob) - 3.0) <= 1e-15
    _compare_solve(prob, x0, v, s=6)


def test_initial_spread_matches_oracle():
    prob, x0, v = W.config_small()
    rng = np.random.default_rng(5)
    G = rng.normal(size=(6, 6)) * 0.05
    Sigma0 = G @ G.T + np.diag([0.02, 0.02, 1e-3, 0.01, 0.01, 1e-3])
    _compare_solve(dict(prob, K=128), x0, v, s=4, Sigma0=Sigma0)


def test_zero_noise_keeps_the_mean_sequence():
    prob, x0, _ = W.config_small()
    prob = dict(prob, sigma_w=[0.0, 0.0, 0.0], sigma_eps=[0.0, 0.0], K=64)
    T = prob["T"]
    v = np.column_stack([0.1 * np.sin(np.arange(T) * 0.3), 0.5 * np.cos(np.arange(T) * 0.2)])
    solver = bss.Solver(prob)
    solver.set_controls(v)
    solver.solve(x0)
    b = solver.buffers()
    mom = b["mom"].cpu().numpy()
    S = b["S"].cpu().numpy()
    # every sample is the same deterministic rollout; covariances vanish
    assert np.all(S == S[0])
    assert np.max(np.abs(mom[:, :, 6:])) <= 1e-20
    # v+ = v up to the single-precision storage of the sampled controls
    assert np.max(np.abs(solver.get_controls() - v)) <= 1e-7
    solver.close()


def test_solves_are_deterministic_and_resumable():
    prob, x0, v = W.config_small()
    a = bss.Solver(prob)
    a.solve(x0)
    a.solve(x0)
    va = a.get_controls()
    Sa = a.buffers()["S"].cpu().numpy()
    b = bss.Solver(prob)
    b.solve(x0)
    v1 = b.get_controls()
    c = bss.Solver(prob)          # resume from the state after the first solve
    c.set_controls(v1)
    c.solve_index = 1
    c.solve(x0)
    assert np.array_equal(c.get_controls(), va)
    assert np.array_equal(c.buffers()["S"].cpu().numpy(), Sa)
    for s_ in (a, b, c):
        s_.close()


def test_non_finite_state_reports_numeric_status():
    prob, x0, v = W.config_small()
    solver = bss.Solver(prob)
    v0 = np.full((prob["T"], 2), 0.1)
    solver.set_controls(v0)
    x_bad = dev(np.array([np.nan, 0, 0, 5, 0, 0]))
    solver.solve_async(x_bad)
    torch.cuda.synchronize()
    st = solver.buffers()["stats"].cpu().numpy()
    assert st[4] == 5.0 and st[3] == 0
    assert np.array_equal(solver.get_controls(), v0)
    with pytest.raises(bss.BssError) as ei:
        solver.solve(np.array([0, np.inf, 0, 5, 0, 0]))
    assert ei.value.status == 1
    solver.close()


# ===================== Gaussian re-sampling reading of Alg. 2 (belief = 1) =====================
@pytest.mark.parametrize("K,M,T,lanes", [(128, 16, 30, 0), (96, 64, 40, 16), (64, 37, 25, 8),
                                         (40, 128, 20, 32), (1024, 64, 50, 0)])
def test_resampling_solve_matches_oracle(K, M, T, lanes):
    prob, x0, _ = W.config_paper_scale()
    prob = dict(prob, K=K, M=M, T=T, belief=1)
    v = np.column_stack([0.05 * np.sin(np.arange(T) * 0.4), 0.5 * np.cos(np.arange(T) * 0.3)])
    _compare_solve(prob, x0, v, s=5, lanes=lanes)


def test_resampling_with_one_particle_is_the_persistent_recursion_on_device():
    prob, x0, v = W.config_small()
    outs = []
    for belief in (0, 1):
        s = bss.Solver(dict(prob, K=64, M=1, belief=belief))
        s.set_controls(v)
        s.solve(x0)
        outs.append((s.get_controls(), s.buffers()["mom"].cpu().numpy()))
        s.close()
    assert np.max(np.abs(outs[0][0] - outs[1][0])) <= 1e-12
    assert np.max(np.abs(outs[0][1] - outs[1][1])) <= 1e-9


# ============== disturbance variants: common random numbers, state-dependent std ==============
@pytest.mark.parametrize("crn,kappa", [(1, 0.0), (0, 0.15), (1, 0.15)])
def test_disturbance_variants_match_oracle(crn, kappa):
    prob, x0, v = W.config_paper_scale()
    prob = dict(prob, K=512, M=32, T=40, crn=crn, sigma_w_speed=kappa)
    v = np.column_stack([0.05 * np.sin(np.arange(40) * 0.4), 0.5 * np.cos(np.arange(40) * 0.3)])
    _compare_solve(prob, x0, v, s=8)


def test_common_random_numbers_give_identical_samples_without_control_noise():
    prob, x0, _ = W.config_small()
    prob = dict(prob, K=64, sigma_eps=[0.0, 0.0], crn=1)
    v = np.column_stack([0.05 * np.ones(prob["T"]), 0.5 * np.ones(prob["T"])])
    s = bss.Solver(prob)
    s.set_controls(v)
    s.solve(x0)
    b = s.buffers()
    S = b["S"].cpu().numpy()
    mom = b["mom"].cpu().numpy()
    assert np.all(S == S[0])
    assert np.all(mom == mom[0])
    # v+ = v up to the single-precision storage of the sampled controls
    assert np.max(np.abs(s.get_controls() - v)) <= 1e-7
    s.close()


# ======================= sigma-point belief propagation (belief = 2) ========================
@pytest.mark.parametrize("K,T,lanes,kappa", [(128, 30, 0, 0.0), (300, 50, 8, 0.0),
                                             (64, 40, 16, 0.1)])
def test_sigma_point_solve_matches_oracle(K, T, lanes, kappa):
    prob, x0, _ = W.config_paper_scale()
    prob = dict(prob, K=K, M=12, T=T, belief=2, sigma_w_speed=kappa)
    v = np.column_stack([0.05 * np.sin(np.arange(T) * 0.4), 0.5 * np.cos(np.arange(T) * 0.3)])
    _compare_solve(prob, x0, v, s=3, lanes=lanes)


def test_sigma_point_solve_with_initial_covariance_matches_oracle():
    prob, x0, v = W.config_small()
    rng = np.random.default_rng(8)
    G = rng.normal(size=(6, 6)) * 0.05
    Sigma0 = G @ G.T + np.diag([0.02, 0.02, 1e-3, 0.01, 0.01, 1e-3])
    _compare_solve(dict(prob, K=96, M=12, belief=2), x0, v, s=2, Sigma0=Sigma0)


def test_sigma_point_belief_rejects_other_particle_counts():
    prob, _, _ = W.config_small()
    with pytest.raises(bss.BssError):
        bss.Solver(dict(prob, M=16, belief=2))


# ======================= more constraints: circular obstacles (eq. 16) ========================
def _with_obstacles(prob, obstacles):
    flat = [c for ob in obstacles for c in ob] + [0.0] * (12 - 3 * len(obstacles))
    return dict(prob, n_obs=len(obstacles), obs=flat)


_OBSTACLES = [(30.3, 3.0, 0.5), (29.2, 6.0, 0.7)]   # next to the centerline ahead of the start


def test_obstacle_solve_matches_oracle():
    """Two obstacles next to the centerline ahead of the start (the car heads +Y from (30, 0))."""
    prob, x0, v = W.config_small()
    prob = _with_obstacles(dict(prob, K=512, M=32), _OBSTACLES)
    _compare_solve(prob, x0, v, s=4)


def test_shielded_obstacle_solve_matches_oracle():
    """The repair against the obstacles as well as the walls.  As for the shielded workload, the
    repair feeds each step's belief back into u: the repair is checked as a stage on the GPU's
    own beliefs and pre-repair controls (1e-6), and the solve end to end against the oracle's own
    sensitivity (tests/sensitivity.py)."""
    prob, x0, v = W.config_small()
    prob = _with_obstacles(dict(prob, K=512, M=32, shield_iters=2), _OBSTACLES)
    s = 4
    solver = bss.Solver(prob)
    solver.set_controls(v)
    solver.solve_index = s
    solver.solve(x0)
    b = solver.buffers()
    got = {"u": b["u"].cpu().numpy().astype(np.float64), "mom": b["mom"].cpu().numpy(),
           "S": b["S"].cpu().numpy(), "v": solver.get_controls()}
    solver.close()
    ref = oracle.solve(prob, s, x0, v, nthreads=NTHREADS)
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    per_k = np.max(np.abs(got["u"] - ref["u"]) / scale, axis=(1, 2))
    # the repair acted on this workload
    plain = oracle.solve(dict(prob, shield_iters=0), s, x0, v, nthreads=NTHREADS)
    assert np.mean(np.any(np.abs(ref["u"] - plain["u"]) > 1e-12, axis=2)) > 1e-3
    # stage check on the worst samples: repair from the GPU's belief and pre-repair control
    nu = oracle.backoff(prob["delta"])
    ks = np.argsort(per_k)[-12:]
    ctr = np.array([[t, 0, k, s] for k in ks for t in range(prob["T"])], dtype=np.uint32)
    z = bss.dev_normals(prob["seed"], dev(ctr.view(np.int32))).cpu().numpy()
    sig32 = np.array(prob["sigma_eps"], dtype=np.float32)
    worst, row = 0.0, 0
    for k in ks:
        for t in range(prob["T"]):
            pre = (sig32.astype(np.float64) * z[row, :2].astype(np.float64)
                   + v[t].astype(np.float32).astype(np.float64)).astype(np.float32)
            pre = np.clip(pre, -scale.astype(np.float32), scale.astype(np.float32))
            row += 1
            u_rep = oracle.repair(prob, nu, got["mom"][k, t], pre.astype(np.float64))
            u_rep32 = u_rep.astype(np.float32).astype(np.float64)
            worst = max(worst, float(np.max(np.abs(u_rep32 - got["u"][k, t]) / scale)))
    print(f"obstacles + shield: repair stage {worst:.2e}", flush=True)
    assert worst <= 1e-6
    SENS.check(SENS.drift(prob, got, ref), SENS.self_drift(prob, s, x0, v, ref, nthreads=NTHREADS),
               "obstacles + shield")


def test_far_obstacle_changes_nothing_on_device():
    prob, x0, v = W.config_small()
    prob = dict(prob, K=128, shield_iters=2)
    outs = []
    for p in (prob, _with_obstacles(prob, [(500.0, 500.0, 2.0)])):
        s = bss.Solver(p)
        s.set_controls(v)
        s.solve(x0)
        b = s.buffers()
        outs.append((s.get_controls(), b["S"].cpu().numpy(), b["mom"].cpu().numpy()))
        s.close()
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("mode", [1, 2])
def test_local_repair_matches_oracle(mode):
    """Repair of the updated sequence (local_repair): one shielded rollout of v+ from the estimate
    on its own stream replaces v+ by v_safe.  Staged: the GPU's v_safe against the oracle's repair
    of the GPU's own v+ (the same solve with the repair of the update off: the samples run the
    same launch, with the per-sample repair for mode 1 and without for mode 2); the returned
    command is v_safe_0; end to end against the oracle's solve with the same setting."""
    prob, _, v = W.config_small()
    prob = dict(prob, shield_iters=4, gamma=0.3)
    x0 = np.array([prob["ell_a"] + 0.8, 0.0, math.pi / 2 - 0.3, 6.0, 0.0, 0.0])
    s = 4
    pre_prob = dict(prob, local_repair=0) if mode == 1 else dict(prob, shield_iters=0)
    outs = {}
    for name, p in (("pre", pre_prob), ("repaired", dict(prob, local_repair=mode))):
        solver = bss.Solver(p)
        solver.set_controls(v)
        solver.solve_index = s
        u0, _ = solver.solve(x0)
        outs[name] = (solver.get_controls(), np.asarray(u0))
        solver.close()
    v_plus = outs["pre"][0]
    v_safe, u0 = outs["repaired"]
    assert np.array_equal(u0, v_safe[0])
    ref_safe, _ = oracle.local_repair(prob, s, x0, v_plus)
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    assert np.max(np.abs(ref_safe - np.clip(v_plus, -scale, scale))) > 1e-2   # the repair acted
    e_stage = ctrl_err(v_safe, ref_safe, prob)
    ref = oracle.solve(dict(prob, local_repair=mode), s, x0, v, want_traces=False,
                       nthreads=NTHREADS)
    e_end = ctrl_err(v_safe, ref["v"], prob)
    print(f"local repair mode {mode}: stage {e_stage:.2e} end-to-end {e_end:.2e}", flush=True)
    assert e_stage <= 1e-4
    assert e_end <= 1e-4


def test_local_repair_is_rejected_in_batches():
    prob, _, _ = W.config_small()
    solver = bss.Solver(dict(prob, shield_iters=2, local_repair=1))
    with pytest.raises(RuntimeError, match="local_repair"):
        bss.Batch([solver])
    solver.close()


@pytest.mark.parametrize("belief", [0, 1])
def test_local_repair_with_initial_spread_matches_oracle(belief):
    """The repair of the update from an uncertain estimate (Sigma0), with persistent particles and
    with the Gaussian re-sampling reading (the repair rollout's own key also drives its
    re-sampling draws): staged against the oracle's repair of the GPU's own v+."""
    prob, _, v = W.config_small()
    prob = dict(prob, K=128, M=16, T=20, shield_iters=4, gamma=0.3, belief=belief)
    x0 = np.array([prob["ell_a"] + 0.8, 0.0, math.pi / 2 - 0.3, 6.0, 0.0, 0.0])
    Sigma0 = np.diag([0.02, 0.02, 0.002, 0.05, 0.02, 0.01])
    v = v[:prob["T"]]
    s = 6
    outs = {}
    for name, p in (("pre", prob), ("repaired", dict(prob, local_repair=1))):
        solver = bss.Solver(p)
        solver.set_controls(v)
        solver.solve_index = s
        u0, _ = solver.solve(x0, Sigma0)
        outs[name] = (solver.get_controls(), np.asarray(u0))
        solver.close()
    v_plus = outs["pre"][0]
    v_safe, u0 = outs["repaired"]
    assert np.array_equal(u0, v_safe[0])
    ref_safe, _ = oracle.local_repair(prob, s, x0, v_plus, Sigma0=Sigma0)
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    assert np.max(np.abs(ref_safe - np.clip(v_plus, -scale, scale))) > 1e-2   # the repair acted
    e_stage = ctrl_err(v_safe, ref_safe, prob)
    print(f"local repair, Sigma0, belief {belief}: stage {e_stage:.2e}", flush=True)
    assert e_stage <= 1e-4


def _violations(prob, mom, nu):
    """DCBF violations of belief records [K][T+1][9]: transitions with
    -h_t + (1 - gamma) h_{t-1} > 0 (eq. 24), h from the oracle's barrier."""
    K, T1 = mom.shape[0], mom.shape[1]
    h = np.array([[oracle.barrier(prob, nu, mom[k, t]) for t in range(T1)] for k in range(K)])
    return int(np.sum(-h[:, 1:] + (1.0 - prob["gamma"]) * h[:, :-1] > 0.0))


def test_info_counts_dcbf_violations_and_times_the_kernel():
    """bss_info.dcbf_violations equals the count the oracle's barrier gives on the GPU's own belief
    records (the same decision in double precision), and on the oracle's own records to within
    the samples whose decision sits at the rounding level; kernel_ms is the timed launch."""
    prob, x0, v = W.config_small()
    prob = dict(prob, gamma=0.05, sigma_w=[0.4, 0.4, 0.2])
    s = 5
    solver = bss.Solver(prob)
    solver.set_controls(v)
    solver.solve_index = s
    solver.timing(True)
    _, info = solver.solve(x0)
    mom = solver.buffers()["mom"].cpu().numpy()
    solver.close()
    nu = oracle.backoff(prob["delta"])
    staged = _violations(prob, mom, nu)
    ref = oracle.solve(prob, s, x0, v, nthreads=NTHREADS)
    end = _violations(prob, ref["mom"], nu)
    print(f"DCBF violations: GPU {info['dcbf_violations']}, oracle on the GPU's records {staged}, "
          f"oracle {end}; kernel {info['kernel_ms']:.4f} ms", flush=True)
    assert info["dcbf_violations"] > 0
    assert info["dcbf_violations"] == staged
    assert abs(end - staged) <= max(2, staged // 1000)
    assert 0.0 < info["kernel_ms"] < 1000.0


# ======================= belief records kept on chip (BSS_OUT_BELIEFS off) =======================
def _config_variant(name):
    prob, x0, _ = W.config_paper_scale()
    if name == "plain_split":
        return dict(prob, K=1024), x0, True
    if name == "paper_scale":
        return prob, x0, True
    if name == "many_blocks":      # needs four blocks per CU: the records stay in HBM
        return dict(prob, K=16384, T=30), x0, False
    if name == "shielded":
        p, x, _ = W.config_shielded()
        return dict(p, K=512), x, True
    if name == "resampled":
        return dict(prob, K=512, belief=1), x0, True
    if name == "sigma_points":
        return dict(prob, K=512, M=12, belief=2), x0, True
    if name == "constrained":
        p, x, _ = W.config_constrained()
        return dict(p, K=1024), x, True
    raise KeyError(name)


@pytest.mark.parametrize("name", ["plain_split", "paper_scale", "many_blocks", "shielded",
                                  "resampled", "sigma_points", "constrained"])
def test_records_on_chip_give_identical_results(name):
    """Without the belief-record output a context's solve keeps the records in the block's LDS
    when they fit beside the resident blocks; costs, updates and stats are the same bit for bit
    over three receding-horizon periods."""
    prob, x0, on_chip = _config_variant(name)
    T = prob["T"]
    t = np.arange(T)
    v = np.column_stack([0.05 * np.sin(0.3 * t), 0.3 * np.cos(0.2 * t)])
    out = []
    for beliefs in (True, False):
        s = bss.Solver(prob)
        s.set_outputs(controls=False, beliefs=beliefs)
        s.set_controls(v)
        res = []
        for _ in range(3):
            u0, info = s.solve(x0)
            b = s.buffers()
            res.append((u0, s.get_controls(), b["S"].cpu().numpy(), b["stats"].cpu().numpy(),
                        info["dcbf_violations"]))
            s.step_shift()
        out.append((res, s.info()["records_on_chip"]))
        s.close()
    (ref, chip_ref), (got, chip_got) = out
    assert not chip_ref
    assert chip_got == on_chip
    for (a, b) in zip(ref, got):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
