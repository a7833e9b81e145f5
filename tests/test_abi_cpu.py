"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every declared entry
point, its struct layouts match the header, and parameter validation behaves as documented."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_2408_00494_amd import _lib, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bssmppi.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libbssmppi.so not built")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bss_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = _lib.lib()
    declared = _declared_functions()
    assert sorted(_lib.EXPORTS) == declared
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header():
    fields = [f for f, _ in _lib.BssParams._fields_]
    prog = ["#include <stdio.h>", "#include <stddef.h>", '#include "bssmppi.h"', "int main(void){",
            'printf("%zu\\n", sizeof(bss_params));']
    for f in fields:
        cf = "lambda" if f == "lambda_" else f
        prog.append(f'printf("%zu\\n", offsetof(bss_params, {cf}));')
    for s, fl in (("bss_buffers", _lib.BssBuffers), ("bss_info", _lib.BssInfo),
                  ("bss_allocator", _lib.BssAllocator), ("bss_server_config", _lib.BssServerConfig),
                  ("bss_completion", _lib.BssCompletion)):
        prog.append(f'printf("%zu\\n", sizeof({s}));')
    for s, fl in (("bss_server_config", _lib.BssServerConfig),
                  ("bss_completion", _lib.BssCompletion)):
        for f, _ in fl._fields_:
            prog.append(f'printf("%zu\\n", offsetof({s}, {f}));')
    prog.append("return 0;}")
    with tempfile.TemporaryDirectory() as tmp:
        c_file = os.path.join(tmp, "layout.c")
        open(c_file, "w").write("\n".join(prog))
        exe = os.path.join(tmp, "layout")
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), "-o", exe, c_file], check=True)
        out = [int(x) for x in subprocess.run([exe], capture_output=True, text=True,
                                              check=True).stdout.split()]
    assert out[0] == C.sizeof(_lib.BssParams)
    for f, off in zip(fields, out[1:1 + len(fields)]):
        assert getattr(_lib.BssParams, f).offset == off, f
    rest = out[1 + len(fields):]
    sizes = [C.sizeof(_lib.BssBuffers), C.sizeof(_lib.BssInfo), C.sizeof(_lib.BssAllocator),
             C.sizeof(_lib.BssServerConfig), C.sizeof(_lib.BssCompletion)]
    assert rest[:len(sizes)] == sizes
    offs = rest[len(sizes):]
    want = [getattr(fl, f).offset for fl in (_lib.BssServerConfig, _lib.BssCompletion)
            for f, _ in fl._fields_]
    assert offs == want


def test_defaults_match_reference_problem():
    p = _lib.BssParams()
    _lib.lib().bss_params_default(C.byref(p))
    ref = W.default_problem()
    for name, _ in _lib.BssParams._fields_:
        key = "lambda" if name == "lambda_" else name
        if key == "lanes":
            assert p.lanes == 0
            continue
        val = getattr(p, name)
        if name in ("sigma_eps", "sigma_w", "obs", "con_a", "con_b"):
            assert list(val) == ref[key]
        else:
            assert val == ref[key], name


def _validate(**kw):
    p = _lib.params_from_problem(W.default_problem(**{k: v for k, v in kw.items() if k != "lanes"}))
    if "lanes" in kw:
        p.lanes = kw["lanes"]
    st = _lib.lib().bss_validate(C.byref(p))
    return st, _lib.lib().bss_last_error().decode()


def test_validation_accepts_workloads():
    assert _validate()[0] == _lib.BSS_OK
    for prob, _, _ in W.config_batch(8):
        st, msg = _lib.lib().bss_validate(C.byref(_lib.params_from_problem(prob))), None
        assert st == _lib.BSS_OK


@pytest.mark.parametrize("kw,frag", [
    (dict(K=0), "K="), (dict(K=(1 << 20) + 1), "K="), (dict(M=0), "M="), (dict(M=513), "M="),
    (dict(T=0), "T="),
    (dict(T=257), "T="), (dict(delta=0.0), "delta"), (dict(delta=0.5), "delta"),
    (dict(gamma=0.0), "gamma"), (dict(gamma=1.5), "gamma"), (dict(**{"lambda": 0.0}), "lambda"),
    (dict(dt=-1.0), "dt"), (dict(sigma_w=[0.1, -1.0, 0.0]), "sigma_w"),
    (dict(sigma_eps=[float("nan"), 1.0]), "sigma_eps"), (dict(half_width=14.0), "track"),
    (dict(ell_a=0.0), "semi-axes"), (dict(shield_iters=17), "shield_iters"),
    (dict(lanes=12), "lanes"), (dict(M=200, lanes=8), "particles per lane"),
    (dict(C_obs=float("inf")), "cost weights"), (dict(m=0.0), "m, Iz"),
    (dict(belief=3), "belief"), (dict(belief=2, M=16), "M = 12"), (dict(crn=2), "crn"),
    (dict(sigma_w_speed=-0.1), "sigma_w_speed"), (dict(n_obs=5), "n_obs"),
    (dict(n_obs=1, obs=[1.0, 2.0, 0.0] + [0.0] * 9), "obstacle 0"),
    (dict(local_repair=3), "local_repair"), (dict(local_repair=1), "shield_iters >= 1"),
    (dict(n_con=5), "n_con"), (dict(n_con=-1), "n_con"),
    (dict(n_con=1, con_a=[float("nan")] + [0.0] * 23), "half-space constraint 0: a"),
    (dict(n_con=2, con_b=[1.0, float("inf"), 0.0, 0.0]), "half-space constraint 1: b"),
])
def test_validation_rejects(kw, frag):
    st, msg = _validate(**kw)
    assert st == _lib.BSS_E_INVAL
    assert frag in msg


def test_backoff_matches_oracle():
    for d in (1e-6, 1e-3, 0.01, 0.05, 0.1, 0.3, 0.49):
        for kind in (0, 1):
            p = _lib.params_from_problem(W.default_problem(delta=d, backoff=kind))
            nu = C.c_double()
            assert _lib.lib().bss_backoff(C.byref(p), C.byref(nu)) == _lib.BSS_OK
            assert nu.value == pytest.approx(oracle.backoff(d, kind), rel=1e-13)


def test_null_and_invalid_handles():
    lib = _lib.lib()
    lib.bss_destroy(None)
    assert lib.bss_create(None, None, None, None) == _lib.BSS_E_INVAL
    out = C.c_void_p()
    bad = _lib.params_from_problem(W.default_problem(K=0))
    assert lib.bss_create(C.byref(bad), None, None, C.byref(out)) == _lib.BSS_E_INVAL
    assert out.value is None
    assert lib.bss_solve(None, None, None, None, None) == _lib.BSS_E_INVAL
    assert lib.bss_step_shift(None) == _lib.BSS_E_INVAL
    assert lib.bss_set_solve_index(None, 3) == _lib.BSS_E_INVAL
    assert lib.bss_dev_philox(1, None, None, -1, None) == _lib.BSS_E_INVAL
    assert lib.bss_dev_update_workspace(0, 5) == 0
    assert lib.bss_dev_update_workspace(300, 5) >= 256 + 2 * (2 * 5 + 4) * 8
    assert "NULL" in lib.bss_last_error().decode() or lib.bss_last_error() is not None


def test_server_and_batch_argument_checks():
    """Argument and configuration errors are reported before any device work."""
    lib = _lib.lib()
    lib.bss_server_destroy(None)
    lib.bss_batch_destroy(None)
    out = C.c_void_p()
    assert lib.bss_server_create(None, None, C.byref(out)) == _lib.BSS_E_INVAL
    cfg = _lib.BssServerConfig()
    lib.bss_server_config_default(C.byref(cfg))
    assert (cfg.n_vehicles, cfg.T, cfg.K_max, cfg.M_max) == (256, 50, 8192, 128)
    assert cfg.hbm_budget == 32 << 30
    veh = (_lib.BssParams * 1)(_lib.params_from_problem(W.default_problem()))
    for field, value in (("n_vehicles", 0), ("T", 0), ("T", 257), ("K_max", 0), ("M_max", 513),
                         ("ppl", 3), ("n_streams", 0), ("n_streams", 17), ("max_batch", 0),
                         ("hbm_budget", 1 << 20)):
        bad = _lib.BssServerConfig.from_buffer_copy(cfg)
        bad.n_vehicles = 1
        setattr(bad, field, value)
        assert lib.bss_server_create(C.byref(bad), veh, C.byref(out)) == _lib.BSS_E_INVAL, field
        assert out.value is None
    bad = _lib.BssServerConfig.from_buffer_copy(cfg)
    bad.n_vehicles, bad.M_max, bad.ppl = 1, 512, 4          # 128 lanes per sample
    assert lib.bss_server_create(C.byref(bad), veh, C.byref(out)) == _lib.BSS_E_INVAL
    assert "64" in lib.bss_last_error().decode()
    bad_veh = (_lib.BssParams * 1)(_lib.params_from_problem(W.default_problem(delta=0.7)))
    one = _lib.BssServerConfig.from_buffer_copy(cfg)
    one.n_vehicles = 1
    assert lib.bss_server_create(C.byref(one), bad_veh, C.byref(out)) == _lib.BSS_E_INVAL
    # the repair of the update runs per context, not in the server's batched launches
    lr_veh = (_lib.BssParams * 1)(_lib.params_from_problem(
        W.default_problem(shield_iters=2, local_repair=1)))
    assert lib.bss_server_create(C.byref(one), lr_veh, C.byref(out)) == _lib.BSS_E_INVAL
    assert "local_repair" in lib.bss_last_error().decode()
    x0 = (C.c_double * 6)()
    assert lib.bss_server_submit(None, 0, 1, 1, 0.05, x0, None) == _lib.BSS_E_INVAL
    assert lib.bss_server_pump(None, None) == _lib.BSS_E_INVAL
    assert lib.bss_server_poll(None, None, 4) == 0
    assert lib.bss_server_drain(None) == _lib.BSS_E_INVAL
    assert lib.bss_batch_create(None, 0, 0, 0, C.byref(out)) == _lib.BSS_E_INVAL
    assert lib.bss_batch_solve(None) == _lib.BSS_E_INVAL
    assert lib.bss_set_shape(None, 16, 4, -1) == _lib.BSS_E_INVAL


def test_noalloc_rejects_oversized_problems_before_any_device_call():
    """The solve that allocates nothing checks its scratch need against the static array before
    touching a device (so this runs without a GPU; the pointers are never dereferenced)."""
    lib = _lib.lib()
    prob, _, _ = W.config_shielded()
    big = _lib.params_from_problem(dict(prob, T=200))
    need = lib.bss_noalloc_scratch_bytes(C.byref(big))
    assert need > (48 << 20)
    fake = C.c_void_p(256)
    st = lib.bss_solve_noalloc(C.byref(big), 0, fake, None, fake, C.c_void_p(512), fake, None)
    assert st == 1                                            # BSS_E_INVAL
    msg = lib.bss_last_error().decode()
    assert "scratch" in msg and str(48 << 20) in msg, msg
    small = _lib.params_from_problem(W.config_small()[0])
    assert 0 < lib.bss_noalloc_scratch_bytes(C.byref(small)) < (48 << 20)
    assert lib.bss_solve_noalloc(C.byref(small), 0, fake, None, fake, fake, fake, None) == 1
    assert "distinct" in lib.bss_last_error().decode()


def test_create_reports_nomem_when_the_allocator_fails():
    """An allocator that returns NULL makes bss_create fail with BSS_E_NOMEM before any device
    call, leave *out NULL and release the host state (repeated failures do not grow the
    process)."""
    import resource
    lib = _lib.lib()
    calls = []

    def alloc(nbytes, _user):
        calls.append(int(nbytes))
        return None

    def release(ptr, _user):
        calls.append(-1)

    a_cb = _lib.BssAllocator._fields_[0][1](alloc)
    r_cb = _lib.BssAllocator._fields_[1][1](release)
    allocator = _lib.BssAllocator(a_cb, r_cb, None)
    p = _lib.params_from_problem(W.config_small()[0])
    ctx = C.c_void_p(1234)
    assert lib.bss_create(C.byref(p), C.byref(allocator), None, C.byref(ctx)) == 2
    assert ctx.value is None
    assert "allocator returned NULL" in lib.bss_last_error().decode()
    assert calls and calls[0] > 0 and -1 not in calls
    rss0 = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss
    for _ in range(20000):
        assert lib.bss_create(C.byref(p), C.byref(allocator), None, C.byref(ctx)) == 2
    rss1 = resource.getrusage(resource.RUSAGE_SELF).ru_maxrss
    assert rss1 - rss0 < 16 * 1024          # KiB: a leaked context per call would be ~MBs
