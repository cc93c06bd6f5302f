"""Write the oracle's one-step results at the workloads' full sizes, sampled.

A ROK step at 256^3 (N = 83.9 M) or 2048^2 (N = 16.8 M) takes the oracle
minutes to a quarter of an hour, too long for a test; the GPU tests compare
with what this script stores instead: the step's result y_1 at 8192 seeded
sample indices (element by element) and, over the whole vector, the sum and
the sum of squares of each conserved variable.  Calls only the oracle and the
seeded input generators (rok_inputs).

Cases (one ROK4 step from the seeded state, or from that state with every
primitive variable seeded-perturbed, `perturb_generic`):
  tgv256_3d_fd       256^3 viscous Taylor-Green, M = 16, CFL 10, FD products
                     (the plain FP64 method at the benchmark size)
  tgv256_3d_exact_g  the same, perturbed state, exact products
  tgv2048_exact_g    2048^2 viscous Taylor-Green, M = 20, CFL 50, perturbed
                     state, exact products
  vortex1024_pert_fd 1024^2 MUSCL vortex with the +/-1 % density
                     perturbation, M = 16, CFL 10, FD products

Usage: python tests/golden/make_fullsize_golden.py [case ...]   (default: all)
Writes tests/golden/fullsize_<case>.json.
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import rok_inputs as ri  # noqa: E402
from oracle import fv, rok  # noqa: E402

NSAMPLE = 8192
SAMPLE_SEED = 8192

CASES = {
    "tgv256_3d_fd": dict(workload="tgv256_3d_fp64", generic=False, mode="fd", M=16, cfl=10.0),
    "tgv256_3d_exact_g": dict(workload="tgv256_3d", generic=True, mode="exact", M=16, cfl=10.0),
    "tgv2048_exact_g": dict(workload="tgv2048_ns", generic=True, mode="exact", M=20, cfl=50.0),
    "vortex1024_pert_fd": dict(workload="vortex1024_muscl", generic=False, perturb=True, mode="fd", M=16, cfl=10.0),
}


def case_input(name):
    """(problem, y0, h, settings) of a case: the inputs the GPU test rebuilds the same way."""
    c = CASES[name]
    pb, y0, _ = ri.workload(c["workload"])
    if c.get("perturb"):
        y0 = ri.perturb_density(pb, y0)
    if c["generic"]:
        y0 = ri.perturb_generic(pb, y0)
    h = ri.cfl_step(pb, y0, c["cfl"])
    return pb, y0, h, c


def sample_indices(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, size=min(NSAMPLE, n), replace=False))


def main(names):
    torch.set_default_dtype(torch.float64)
    for name in names:
        t0 = time.time()
        pb, y0, h, c = case_input(name)
        P = fv.Problem(n=tuple(pb["n"]), lo=tuple(pb["lo"]), hi=tuple(pb["hi"]), physics=pb["physics"],
                       recon=pb["recon"], gamma=pb["gamma"], mu=pb["mu"], prandtl=pb["prandtl"])
        f, mv = rok.fv_system(P, c["mode"])
        rec = {}
        y1 = rok.rok_step(f, mv, ri.rok4_tableau(), c["M"], h, torch.from_numpy(np.asarray(y0)), record=rec)
        a = y1.numpy()
        idx = sample_indices(a.size)
        nvar = len(pb["n"]) + 2
        per = a.reshape(nvar, -1)
        out = {"case": name, "settings": c, "h": h, "N": int(a.size), "M_eff": int(rec["M_eff"]),
               "sample_seed": SAMPLE_SEED, "index": idx.tolist(), "y1": [float(x) for x in a[idx]],
               "var_sum": [float(np.sum(per[v])) for v in range(nvar)],
               "var_sumsq": [float(np.sum(per[v] * per[v])) for v in range(nvar)],
               "oracle_seconds": round(time.time() - t0, 1), "torch_threads": torch.get_num_threads()}
        path = os.path.join(HERE, f"fullsize_{name}.json")
        with open(path, "w") as fh:
            json.dump(out, fh)
        print(f"{name}: wrote {path} ({out['oracle_seconds']} s)", flush=True)
        del y1, rec, a, per


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
