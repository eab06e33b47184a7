"""The ion LBEs on D2Q9 (lbm_ehd_params.ion_q9 = 1) against the CPU oracle
run with the same option.

* FP64 storage on the 128^2 droplet case, on ragged variants with and
  without side walls, and on the enclosure of Sec. 6 (rel-L2 <= 1e-10 on
  every field);
* FP32 storage on the ragged case with and without side walls and on the
  enclosure (the FP32 bar, 2e-5);
* D2Q9 ions differ from D2Q5 ions (the option is not a no-op) while phi is
  conserved to rounding;
* batches that mix D2Q9 and D2Q5 members give every member bitwise its
  results alone; a checkpoint does not load across the two ion lattices.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import FIELDS8, rel_l2, run_gpu, run_oracle  # noqa: E402

from paper_2501_04920_amd import lbm_ehd, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

ALL10 = FIELDS8 + ("Ex", "Ey")


def _report(tag, errs):
    print("%s: %s" % (tag, " ".join("%s=%.2e" % kv for kv in errs.items())), flush=True)


def test_config1_droplet_ions_d2q9_fp64():
    cfg = workloads.config1()
    p, d = dict(cfg["params"], ion_q9=1), cfg["droplet"]
    sim = run_gpu(p, "fp64", droplet=d, presolve=cfg["presolve"], steps=cfg["steps"])
    o = run_oracle(p, droplet=d, presolve=cfg["presolve"], steps=cfg["steps"])
    errs = rel_l2(sim.fields(), o.fields(), p, ALL10)
    _report("config1 ions d2q9 fp64", errs)
    assert max(errs.values()) <= 1e-10
    sim.close()


def _ragged(**over):
    p = workloads.lattice_params(70, 12.0, nx=100)
    p.update(over, ion_q9=1)
    d = dict(xc=49.3, yc=33.7, radius=12.0, noise=1e-3, seed=7)
    return p, d


VARIANTS = {
    "base": {},
    "periodic": dict(walls=2),
    "insulating": dict(walls=1),
    "poisson_iters": dict(poisson_iters=3),
    "reaction_off": dict(reaction=0),
    "no_ion_force": dict(ion_force=0),
    "ratios": dict(rho_r=2.0, eta_r=3.0, mu_r=0.5, m_ratio=1.5, eps_r=0.5),
    "bgk_masks": dict(mask_f=0x1FF, mask_h=0x1FF, mask_p=0x1FF, mask_n=0x1FF, mask_g=0x1F),
    "s_free": dict(s_free=1.3),
    "side_walls": dict(side_walls=1),
    "side_walls_insulating": dict(side_walls=1, walls=1),
    "side_walls_periodic": dict(side_walls=1, walls=2),
    "side_walls_bgk": dict(side_walls=1, mask_p=0x1FF, mask_n=0x1FF),
}


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_ragged_variants_ions_d2q9_fp64(name):
    """100 x 70 (a ragged strip and band), off-centre droplet, 61 steps."""
    p, d = _ragged(**VARIANTS[name])
    sim = run_gpu(p, "fp64", droplet=d, presolve=10, steps=61)
    o = run_oracle(p, droplet=d, presolve=10, steps=61)
    errs = rel_l2(sim.fields(), o.fields(), p, ALL10)
    _report("ragged ions d2q9 %s" % name, errs)
    assert max(errs.values()) <= 1e-10
    sim.close()


@pytest.mark.parametrize("side_walls", [0, 1])
@pytest.mark.parametrize("precision", ["fp32", "fp32f64"])
def test_ragged_ions_d2q9_fp32_storage(precision, side_walls):
    p, d = _ragged(side_walls=side_walls)
    sim = run_gpu(p, precision, droplet=d, presolve=10, steps=200)
    o = run_oracle(p, droplet=d, presolve=10, steps=200)
    errs = rel_l2(sim.fields(), o.fields(), p, ALL10)
    _report("ragged ions d2q9 %s side walls %d" % (precision, side_walls), errs)
    assert max(errs.values()) <= 2e-5
    sim.close()


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32", 2e-5)])
def test_enclosure_ions_d2q9(precision, bar):
    """The enclosure of Sec. 6 (256^2, side walls, electrodes) with the ions
    on D2Q9: 2000 pre-solve sweeps and 1000 steps against the oracle."""
    case = workloads.enclosure(256)
    p, d = dict(case["params"], ion_q9=1), case["droplet"]
    sim = run_gpu(p, precision, droplet=d, presolve=2000, steps=1000)
    o = run_oracle(p, droplet=d, presolve=2000, steps=1000)
    errs = rel_l2(sim.fields(), o.fields(), p, ALL10)
    _report("enclosure ions d2q9 %s" % precision, errs)
    assert max(errs.values()) <= bar
    sim.close()


def test_d2q9_ions_differ_from_d2q5_and_conserve():
    p, d = _ragged()
    p5 = dict(p, ion_q9=0)
    a = run_gpu(p, "fp64", droplet=d, presolve=10, steps=200)
    b = run_gpu(p5, "fp64", droplet=d, presolve=10, steps=200)
    fa, fb = a.fields(), b.fields()
    # the same physics to the lattices' truncation error, not the same numbers
    diff = np.linalg.norm(fa["cp"] - fb["cp"]) / np.linalg.norm(fb["cp"])
    print("d2q9 vs d2q5 ions: rel diff of c+ %.2e" % diff, flush=True)
    assert 1e-12 < diff < 1e-2
    z = run_gpu(p, "fp64", droplet=d, presolve=10)
    da0, da = z.diagnostics(), a.diagnostics()
    assert abs(da["sum_phi"] / da0["sum_phi"] - 1) <= 1e-12
    for s in (a, b, z):
        s.close()


def _member(nx, ny, r, seed, q9, precision, side=0):
    p = workloads.lattice_params(ny, r, nx=nx)
    s = lbm_ehd.Simulation(dict(p, precision=precision, ion_q9=q9, side_walls=side),
                           device="cuda:0")
    s.init_droplet((nx - 1) / 2 + 0.3, (ny - 1) / 2 - 0.2, r, 1e-3, seed, presolve=6)
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ions_d2q9_batch_equals_members_alone(precision):
    shapes = [(64, 64, 10.0, 1, 1, 0), (100, 70, 12.0, 2, 0, 0), (128, 96, 15.0, 3, 1, 1),
              (37, 41, 6.0, 4, 1, 0), (90, 60, 11.0, 5, 0, 1)]
    steps = 37
    alone = []
    for nx, ny, r, seed, q9, side in shapes:
        s = _member(nx, ny, r, seed, q9, precision, side)
        s.step(steps)
        alone.append(s.fields())
        s.close()
    sims = [_member(nx, ny, r, seed, q9, precision, side)
            for nx, ny, r, seed, q9, side in shapes]
    b = lbm_ehd.Batch(sims)
    b.set_launch(2, 8)
    b.run(16)
    b.set_launch(1, 4)
    b.run(steps - 16)
    b.synchronize()
    for s, ref in zip(sims, alone):
        assert s.time == steps
        f = s.fields()
        for k in ALL10:
            assert np.array_equal(f[k], ref[k]), k
    b.close()
    for s in sims:
        s.close()


def test_ions_d2q9_checkpoint():
    """A D2Q9-ion state continues bitwise after a save and load, and does not
    load into a D2Q5-ion simulation."""
    p, d = _ragged()
    a = run_gpu(p, "fp32", droplet=d, presolve=7, steps=21)
    state = a.save_state()
    a.step(10)
    b = lbm_ehd.Simulation(dict(p, precision="fp32"), device="cuda:0")
    b.load_state(state)
    b.step(10)
    fa, fb = a.fields(), b.fields()
    for k in ALL10:
        assert np.array_equal(fa[k], fb[k]), k
    c = lbm_ehd.Simulation(dict(p, precision="fp32", ion_q9=0), device="cuda:0")
    with pytest.raises(lbm_ehd.LbmError) as e:
        c.load_state(state)
    assert e.value.code == lbm_ehd.LBM_EINVAL
    for s in (a, b, c):
        s.close()
