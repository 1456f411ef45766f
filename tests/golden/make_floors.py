"""Writes the oracle's own round-off floors of two long runs:
  tube_1024x128_floor.json  1024 x 128 one-step detonation tube (seed 2504, CFL 0.5),
                            N = 100, 200, ..., 1000 steps;
  ensemble_64_floor.json    64-instance one-step ensemble (32 1-D, 32 2-D; seed 2025),
                            N = 25, 50, 100 steps.

The detonation fronts are unstable, so a change at the level of one rounding grows
with N. The floor at N is, per field, the larger of two relative differences
(field-max normalization) from the oracle's reference run:
  "ulp": the oracle run from the same state with every initial density one ulp larger;
  "fma": the same source built with fused multiply-add contraction (every a*b+c rounded
         once instead of twice, as in the GPU build) run from the same state.
A second implementation of the same arithmetic cannot be expected to agree with the
oracle more closely than this; the GPU parity tests of these runs hold each field to
max(1e-10, 2 x floor).

Calls only the oracle (both builds) and the seeded case generators:
    python tests/golden/make_floors.py tube        (about 10 minutes on 8 cores)
    python tests/golden/make_floors.py ensemble    (about 8 minutes on 8 cores)
"""

import json
import os
import subprocess
import sys
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

STEPS = {"tube": [100, 200, 300, 400, 500, 600, 700, 800, 900, 1000], "ensemble": [25, 50, 100]}
OUT = {"tube": "tube_1024x128_floor.json", "ensemble": "ensemble_64_floor.json"}
WHAT = {"tube": "1024 x 128 one-step detonation tube (seed 2504, CFL 0.5)",
        "ensemble": "64-instance one-step ensemble, 32 1-D and 32 2-D instances (seed 2025)"}


def rel_err(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    return [float(np.max(np.abs(a[f] - b[f])) / np.max(np.abs(b[f]))) for f in range(a.shape[0])]


def states(workload, steps, ulp=False):
    """Conserved state after each N in steps, from the oracle this process loaded."""
    import copy
    import oracle
    from cases import detonation_tube_case, ensemble_case
    out = {}
    n = 0
    if workload == "tube":
        case = detonation_tube_case()
        W = case.W.copy()
        if ulp:
            W[0] = np.nextafter(W[0], np.inf)
        U, T = oracle.init_state(case.model, W, case.mech, case.gamma, case.R, case.Q)
        t = 0.0
        for N in steps:
            U, T, t, _, _ = oracle.step(case, U, T, N - n, t=t)
            n = N
            out[N] = U.copy()
    else:
        case = ensemble_case()
        if ulp:
            case = copy.copy(case)
            case.W = case.W.copy()
            case.W[0] = np.nextafter(case.W[0], np.inf)
        U, T = oracle.block_state(case)
        t = None
        for N in steps:
            U, T, t, _, _ = oracle.step_blocks(case, U, T, N - n, t=t)
            n = N
            out[N] = U.copy()
    return out


def run_variant(workload, steps, variant, ulp, path):
    env = dict(os.environ)
    if variant:
        env["JANC_ORACLE_VARIANT"] = variant
    else:
        env.pop("JANC_ORACLE_VARIANT", None)
    cmd = [sys.executable, os.path.abspath(__file__), "--states", workload, path]
    if ulp:
        cmd.append("--ulp")
    subprocess.run(cmd, env=env, check=True)
    with np.load(path) as z:
        return {N: z[str(N)] for N in steps}


def floors(workload, steps, verbose=False):
    with tempfile.TemporaryDirectory() as d:
        base = run_variant(workload, steps, None, False, os.path.join(d, "base.npz"))
        ulp = run_variant(workload, steps, None, True, os.path.join(d, "ulp.npz"))
        fma = run_variant(workload, steps, "fma", False, os.path.join(d, "fma.npz"))
    table = {}
    for N in steps:
        eu, ef = rel_err(ulp[N], base[N]), rel_err(fma[N], base[N])
        table[N] = {"ulp": eu, "fma": ef, "floor": [max(a, b) for a, b in zip(eu, ef)]}
        if verbose:
            print(N, "ulp", ["%.2e" % x for x in eu], "fma", ["%.2e" % x for x in ef], flush=True)
    return table


def main():
    if sys.argv[1] == "--states":
        workload, path = sys.argv[2], sys.argv[3]
        res = states(workload, STEPS[workload], ulp="--ulp" in sys.argv)
        np.savez(path, **{str(k): v for k, v in res.items()})
        return
    workload = sys.argv[1]
    table = floors(workload, STEPS[workload], verbose=True)
    doc = {
        "what": f"oracle round-off floor, {WHAT[workload]}: per field, max|U_x - U_ref| / "
                "max|U_ref| after N steps for x = ulp (initial densities one ulp larger) and "
                "x = fma (the oracle built with fused multiply-add contraction); floor = the "
                "larger of the two",
        "fields": ["rho", "rho u", "rho v", "E", "rho Y"],
        "script": "tests/golden/make_floors.py " + workload,
        "floor": {str(k): v["floor"] for k, v in table.items()},
        "ulp": {str(k): v["ulp"] for k, v in table.items()},
        "fma": {str(k): v["fma"] for k, v in table.items()},
    }
    with open(os.path.join(HERE, OUT[workload]), "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", OUT[workload])


if __name__ == "__main__":
    main()
