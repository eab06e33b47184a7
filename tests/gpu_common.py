"""Helpers shared by the GPU tests: run the HIP library and the CPU oracle on
the same inputs and compare fields."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2501_04920_amd import lbm_ehd

FIELDS8 = ("phi", "psi", "cp", "cm", "rhoe", "ux", "uy", "p")


def floors(params: dict, ncell: int) -> dict:
    """Absolute floor of the rel-L2 denominator per field: the field's natural
    scale times sqrt(cells) times 1e-5, so that fields that are still ~0
    (velocity at early times) are compared on that scale."""
    dpsi = max(abs(params.get("dpsi", 0.0)), 1e-3)
    c0 = params.get("c0", 1.0)
    qc = max(abs(params.get("q", 0.0)) * c0, 1e-12)
    s = dict(phi=1.0, psi=dpsi, cp=c0, cm=c0, rhoe=qc, ux=1e-2, uy=1e-2, p=1e-4,
             Ex=dpsi / params["ny"], Ey=dpsi / params["ny"])
    return {k: v * np.sqrt(ncell) * 1e-5 for k, v in s.items()}


def rel_l2(got: dict, ref: dict, params: dict, names=FIELDS8) -> dict:
    fl = floors(params, ref["phi"].size)
    out = {}
    for k in names:
        den = max(np.linalg.norm(ref[k]), fl[k])
        out[k] = float(np.linalg.norm(got[k] - ref[k]) / den)
    return out


def e_vec_rel(got: dict, ref: dict) -> float:
    """rel-L2 of the field vector E = (Ex, Ey) over the grid.  Where E is
    nearly parallel to y, the per-component error of Ex divides a rounding
    difference by a small norm; the vector measure does not."""
    num = np.sqrt(np.sum((got["Ex"] - ref["Ex"]) ** 2 + (got["Ey"] - ref["Ey"]) ** 2))
    return float(num / np.sqrt(np.sum(ref["Ex"] ** 2 + ref["Ey"] ** 2)))


def run_gpu(params, precision, *, droplet=None, fields=None, presolve=0, steps=0):
    sim = lbm_ehd.Simulation(dict(params, precision=precision), device="cuda:0")
    if droplet is not None:
        sim.init_droplet(droplet["xc"], droplet["yc"], droplet["radius"], droplet["noise"],
                         droplet["seed"], presolve=presolve)
    else:
        sim.init_fields(*fields)
        if presolve:
            sim.presolve(presolve)
    if steps:
        sim.step(steps)
    return sim


def run_oracle(params, *, droplet=None, fields=None, presolve=0, steps=0):
    o = oracle.Oracle(params)
    if droplet is not None:
        o.init_droplet(droplet["xc"], droplet["yc"], droplet["radius"], droplet["noise"],
                       droplet["seed"], presolve=presolve)
    else:
        o.init_fields(*fields)
        if presolve:
            o.presolve(presolve)
    if steps:
        o.step(steps)
    return o
