"""Helpers shared by the tests (conversion of plain inputs to oracle objects)."""
import numpy as np
import torch

from oracle import fv


def oracle_problem(pb):
    return fv.Problem(n=tuple(pb["n"]), lo=tuple(pb["lo"]), hi=tuple(pb["hi"]), physics=pb["physics"],
                      recon=pb["recon"], gamma=pb["gamma"], mu=pb["mu"], prandtl=pb["prandtl"],
                      flux=pb.get("flux", "rusanov"), sutherland=pb.get("sutherland", 0.0),
                      t_ref=pb.get("t_ref", 1.0))


def t64(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64))


def relerr(a, b):
    a = torch.as_tensor(a, dtype=torch.float64).reshape(-1)
    b = torch.as_tensor(b, dtype=torch.float64).reshape(-1)
    nb = float(torch.linalg.norm(b))
    return float(torch.linalg.norm(a - b)) / (nb if nb > 0 else 1.0)
