"""Writes closed_loop_oracle.json: closed-loop statistics of the FP64 oracle controller on the
shielded workload (K=8192, M=128, T=60, two repair iterations) for every (delta, gamma)
combination, with the plant and episode rules of tests/closed_loop.py, and the per-step series
(e_y, crash flag, barrier flag, vx) they come from.  Calls only the oracle and the input
generators.  The file is updated in place: each combination, once finished, replaces the entry of
the same seed (each entry records its own number of steps), so a longer run can extend an
existing file one combination at a time.

    python tests/golden/make_closed_loop_oracle.py [steps] [nthreads] [output path] [first combo]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))            # tests/
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))   # repository root

import closed_loop as CL  # noqa: E402


def main():
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 250
    nthreads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    out_path = sys.argv[3] if len(sys.argv) > 3 else os.path.join(HERE, "closed_loop_oracle.json")
    first = int(sys.argv[4]) if len(sys.argv) > 4 else 0
    res = {"controller": "oracle", "combos": []}
    if os.path.exists(out_path):
        with open(out_path) as fh:
            res = json.load(fh)
        res.pop("steps_per_combo", None)
    for i, (d, g) in enumerate(CL.COMBOS):
        if i < first:
            continue
        prob = CL.combo_problem(i)
        t0 = time.time()
        st, _ = CL.run(prob, steps, CL.OracleController(prob, nthreads), keep_series=True)
        st.update({"delta": d, "gamma": g, "seed": prob["seed"]})
        res["combos"] = [c for c in res["combos"] if c["seed"] != prob["seed"]] + [st]
        res["combos"].sort(key=lambda c: (c["delta"], c["gamma"]))
        shown = {key: val for key, val in st.items() if key != "series"}
        print(f"delta={d} gamma={g}: {shown} ({time.time() - t0:.0f} s)", flush=True)
        with open(out_path, "w") as fh:
            json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
