"""The solve that allocates nothing (bss_solve_noalloc, the library's static scratch) against the
context path (bss_create + bss_solve_async at the same solve index and mean sequence): the same
kernels and launch shape, so v+ and the stats must agree bit for bit.  Two calls in a row, the
second with a smaller problem, so the second reuses scratch the first left behind."""
import numpy as np
import pytest

from paper_2408_00494_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

import paper_2408_00494_amd as bss  # noqa: E402


def _context_solve(prob, s, x0, v, Sigma0=None):
    solver = bss.Solver(prob)
    solver.set_outputs(controls=False)
    solver.set_controls(v)
    solver.solve_index = s
    x0_dev = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
    S0 = None if Sigma0 is None else torch.as_tensor(Sigma0, dtype=torch.float64, device="cuda")
    solver.solve_async(x0_dev, S0)
    torch.cuda.synchronize()
    v_out = solver.get_controls()
    stats = solver.buffers()["stats"].cpu().numpy().copy()
    solver.close()
    return v_out, stats


def _noalloc_solve(prob, s, x0, v, Sigma0=None):
    x0_dev = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
    S0 = None if Sigma0 is None else torch.as_tensor(Sigma0, dtype=torch.float64, device="cuda")
    v_in = torch.as_tensor(v, dtype=torch.float64, device="cuda")
    v_out = torch.full_like(v_in, float("nan"))
    stats = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    bss.solve_noalloc(prob, s, x0_dev, v_in, v_out, stats, Sigma0=S0)
    torch.cuda.synchronize()
    assert np.array_equal(v_in.cpu().numpy(), v)   # v_in is only read
    return v_out.cpu().numpy(), stats.cpu().numpy()


def test_noalloc_solve_equals_context_solve_twice_in_a_row():
    big, x0_big, _ = W.config_paper_scale()                  # K=4096, M=64, T=50 (noise split)
    T = big["T"]
    v_big = np.column_stack([0.05 * np.sin(np.arange(T) * 0.3), 0.4 * np.cos(np.arange(T) * 0.2)])
    small, x0_small, _ = W.config_small()
    small = dict(small, K=200, M=12, T=24, shield_iters=2)   # smaller, shielded (P = 8 variant)
    v_small = np.column_stack([0.02 * np.ones(24), 0.3 * np.sin(np.arange(24) * 0.5)])
    Sigma0 = np.diag([0.01, 0.01, 1e-4, 0.02, 0.01, 1e-3])
    assert bss.noalloc_scratch_bytes(small) < bss.noalloc_scratch_bytes(big)
    for prob, x0, v, S0, s in ((big, x0_big, v_big, None, 7), (small, x0_small, v_small, Sigma0, 3)):
        got_v, got_stats = _noalloc_solve(prob, s, x0, v, S0)
        want_v, want_stats = _context_solve(prob, s, x0, v, S0)
        print(f"K={prob['K']} M={prob['M']} T={prob['T']}: max |dv| "
              f"{np.max(np.abs(got_v - want_v)):.3e}, ess {got_stats[2]:.2f}", flush=True)
        assert got_stats[4] == 0.0
        assert np.array_equal(got_v, want_v)
        assert np.array_equal(got_stats, want_stats)


def test_noalloc_rejects_problems_beyond_the_scratch():
    prob, x0, v = W.config_shielded()
    prob = dict(prob, T=200)                       # K=8192, M=128, T=200: ~118 MB of records
    need = bss.noalloc_scratch_bytes(prob)
    assert need > (48 << 20)
    x0_dev = torch.as_tensor(x0, dtype=torch.float64, device="cuda")
    v_in = torch.zeros((prob["T"], 2), dtype=torch.float64, device="cuda")
    v_out = torch.zeros_like(v_in)
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="scratch"):
        bss.solve_noalloc(prob, 0, x0_dev, v_in, v_out, stats)
    torch.cuda.synchronize()
    assert not torch.any(v_out != 0)              # nothing was enqueued
