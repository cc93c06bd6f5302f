"""Write the oracle's directional derivatives for the differentiation workload.

Differentiation workload: 512 x 512 first-order Rusanov vortex (density
perturbed, seeded), ROK4 with exact products, M = 16, 50 steps at CFL 2;
L = integrated kinetic energy of y_50.  For directions d seeded 1..3
(Gaussian, ||d|| = ||y_0||) this records <grad L(y_0), d>, computed by
forward-mode differentiation of the oracle's differentiable step
(oracle.rok_ad), and L itself.  Calls only the oracle and the seeded input
generators.  Runtime: minutes per direction on a few CPU cores.

Usage: python tests/golden/make_adjoint_golden.py [seed ...]
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
from oracle import fv, rok_ad  # noqa: E402

OUT = os.path.join(HERE, "vortex512_adjoint_directional.json")


def main(seeds):
    torch.set_default_dtype(torch.float64)
    pb, y0, st = ri.workload("vortex512_adjoint")
    P = fv.Problem(n=tuple(pb["n"]), lo=tuple(pb["lo"]), hi=tuple(pb["hi"]), physics=pb["physics"],
                   recon=pb["recon"], gamma=pb["gamma"], mu=pb["mu"], prandtl=pb["prandtl"])
    tab = ri.rok4_tableau()
    h = ri.cfl_step(pb, y0, st["cfl"])
    y = torch.from_numpy(np.asarray(y0, dtype=np.float64))
    ny = float(torch.linalg.norm(y))
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    res.update({"workload": "vortex512_adjoint", "steps": st["steps"], "M": st["M"], "cfl": st["cfl"], "h": h,
                "direction": "random_direction(N, seed) scaled to ||y_0||"})
    dirs = res.setdefault("directional", {})
    for seed in seeds:
        d = torch.from_numpy(np.asarray(ri.random_direction(y.numel(), seed), dtype=np.float64))
        d = d * (ny / float(torch.linalg.norm(d)))
        t0 = time.time()

        def L(z):
            return rok_ad.kinetic_energy(P, rok_ad.trajectory(P, tab, st["M"], h, z, st["steps"], forward=True))

        Lv, t = torch.func.jvp(L, (y,), (d,))
        dirs[str(seed)] = {"L": float(Lv), "dLd": float(t), "seconds": round(time.time() - t0, 1)}
        print(seed, dirs[str(seed)], flush=True)
        cur = json.load(open(OUT)) if os.path.exists(OUT) else {}
        cur.update({k: v for k, v in res.items() if k != "directional"})
        cur.setdefault("directional", {}).update(dirs)
        json.dump(cur, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1, 2, 3])
