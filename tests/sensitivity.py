"""End-to-end bars of shielded solves, measured from the method's own sensitivity (test
infrastructure, used by the GPU parity tests).

With the repair of the samples active, the belief of step t feeds back into the control u_t at
every step, so a difference of the belief of the size the single-precision particles make (about
1e-6 of the state) can move a sample's later controls, beliefs and cost by far more: the repair
divides the residual by |dr/du|^2 + gmin^2 (a large gain where the controls have little authority
over the constraint), and the collision indicator C_obs [|e_y| >= w_T] of the running cost jumps
when a mean crosses the wall.  The oracle shows the same spread against itself when its state
estimate moves by that much.

The bars of a shielded end-to-end comparison are therefore taken from the oracle run against
itself with the estimate moved by +DX and by -DX (the larger of the two spreads):
  * per sample, the number of samples past each fixed bar (controls 1e-4 of full scale, moments
    1e-3 of the trajectory scale, costs 1e-3 relative) may exceed the oracle's own number by at
    most a factor two plus three samples;
  * the weighted controls v+ may differ by at most max(1e-4, 2 x the oracle's own drift).
Where the oracle's own spread is zero the fixed bars hold up to three samples.
"""
import numpy as np

import oracle

DX = np.array([1e-6, 1e-6, 1e-7, 1e-6, 1e-7, 1e-7])
U_BAR, MOM_BAR, S_BAR, V_BAR = 1e-4, 1e-3, 1e-3, 1e-4


def drift(prob, a, b):
    """Shares of samples of solve `a` past the fixed bars against solve `b` (dicts with u [K][T][2],
    mom [K][T+1][9], S [K] and v [T][2]; u and mom optional) and the v+ difference."""
    scale = np.array([prob["steer_max"], prob["accel_max"]])
    out = {"K": int(np.asarray(b["S"]).shape[0])}
    out["n_S"] = int(np.sum(np.abs(a["S"] - b["S"]) / np.abs(b["S"]) > S_BAR))
    out["S_max"] = float(np.max(np.abs(a["S"] - b["S"]) / np.abs(b["S"])))
    if a.get("u") is not None and b.get("u") is not None:
        per_k = np.max(np.abs(a["u"] - b["u"]) / scale, axis=(1, 2))
        out["n_u"] = int(np.sum(per_k > U_BAR))
    if a.get("mom") is not None and b.get("mom") is not None:
        span = np.max(np.abs(b["mom"]), axis=1, keepdims=True)
        per_k = np.max(np.abs(a["mom"] - b["mom"]) / np.where(span > 0, span, 1.0), axis=(1, 2))
        out["n_mom"] = int(np.sum(per_k > MOM_BAR))
        out["mom_max"] = float(per_k.max())
    out["v"] = float(np.max(np.abs(a["v"] - b["v"]) / scale))
    return out


def self_drift(prob, s, x0, v, ref, Sigma0=None, nthreads=16):
    """The oracle against itself with the estimate moved by +DX and -DX: the larger spread."""
    own = None
    for sign in (1.0, -1.0):
        moved = oracle.solve(prob, s, np.asarray(x0) + sign * DX, v, Sigma0=Sigma0,
                             nthreads=nthreads)
        d = drift(prob, moved, ref)
        own = d if own is None else {key: max(own[key], d[key]) for key in d}
    return own


def check(gpu, own, label=""):
    """Assert the GPU's spread against the oracle stays within the oracle's own (see above)."""
    print(f"{label}: GPU vs oracle {gpu}; oracle vs itself (estimate moved by ~1e-6) {own}",
          flush=True)
    for key in ("n_u", "n_mom", "n_S"):
        if key in gpu and key in own:
            assert gpu[key] <= 2 * own[key] + 3, (key, gpu[key], own[key])
    assert gpu["v"] <= max(V_BAR, 2.0 * own["v"]), (gpu["v"], own["v"])
