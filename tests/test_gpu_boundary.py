"""GPU tests of the C ABI's guards and run modes: the diag_every watchdog,
graph-replayed runs, the batch-member guard and the references recorded in
a checkpoint."""
import ctypes

import numpy as np
import pytest

from paper_2501_04920_amd import lbm_ehd, workloads

pytestmark = pytest.mark.gpu

ALL10 = ("phi", "psi", "cp", "cm", "rhoe", "ux", "uy", "p", "Ex", "Ey")


def _droplet_fields(n, p):
    y, x = np.mgrid[0:n, 0:n]
    phi = 0.5 * (1 + np.tanh(2 * (10.0 - np.hypot(x - 31.5, y - 31.5)) / p["W"]))
    psi = p["dpsi"] * (n - 0.5 - y) / n
    return phi, psi


@pytest.mark.parametrize("precision,inplace", [("fp32", 0), ("fp16", 1), ("fp64", 1)])
def test_watchdog_stops_a_run_at_the_first_check_after_a_nan(precision, inplace):
    """With diag_every = 8 a NaN in one cell of the initial phi stops the
    run with LBM_ENONFINITE at step 8 (the first check), and the step count
    says so; with the watchdog off the same run completes, and a clean state
    passes every check (two buffers and in place)."""
    n = 64
    p = dict(workloads.lattice_params(n, 10.0), precision=precision, inplace=inplace)
    phi, psi = _droplet_fields(n, p)
    clean = lbm_ehd.Simulation(dict(p, diag_every=8), device="cuda:0")
    clean.init_fields(phi, 1.0, 1.0, psi)
    clean.step(40)
    assert clean.time == 40
    clean.close()
    phi[20, 30] = np.nan
    for every in (8, 0):
        sim = lbm_ehd.Simulation(dict(p, diag_every=every), device="cuda:0")
        sim.init_fields(phi, 1.0, 1.0, psi)
        code = lbm_ehd.lib().lbm_ehd_run(sim.handle, 40)
        if every:
            assert code == lbm_ehd.LBM_ENONFINITE
            assert "step 8" in lbm_ehd.lbm_ehd_last_error()
            assert sim.time == 8
        else:
            assert code == lbm_ehd.LBM_OK and sim.time == 40
        sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_graph_replayed_run_equals_single_steps(precision):
    """lbm_ehd_run replays blocks of 16 captured sweeps; the result is
    bitwise that of the same steps taken one lbm_ehd_step at a time, from
    either buffer parity and across a change of launch shape."""
    p, d = workloads.config1()["params"], workloads.config1()["droplet"]
    p = dict(p, nx=96, ny=80)
    a = lbm_ehd.Simulation(dict(p, precision=precision), device="cuda:0")
    b = lbm_ehd.Simulation(dict(p, precision=precision), device="cuda:0")
    for s in (a, b):
        s.init_droplet(47.5, 39.5, 12.0, d["noise"], d["seed"], presolve=20)
    a.step(37)                       # 2 graph blocks + 5 single steps: odd parity after
    a.step(35)
    a.set_launch(1, 4)               # drops the captured graphs
    a.step(20)
    for _ in range(37 + 35):
        lbm_ehd.lbm_ehd_step(b.handle)
    b.set_launch(1, 4)
    for _ in range(20):
        lbm_ehd.lbm_ehd_step(b.handle)
    assert a.time == b.time == 92
    fa, fb = a.fields(), b.fields()
    for k in ALL10:
        assert np.array_equal(fa[k], fb[k]), k
    a.close()
    b.close()


def test_batch_members_refuse_their_own_steps():
    """Calls that move or replace a member's state return LBM_ESTATE while it
    is in a batch, work again once it is removed, and a member belongs to one
    batch only; destroying a member removes it from its batch."""
    p = workloads.lattice_params(48, 8.0)
    sims = []
    for _ in range(3):
        s = lbm_ehd.Simulation(dict(p, precision="fp32"), device="cuda:0")
        s.init_droplet(23.5, 23.5, 8.0)
        sims.append(s)
    b = lbm_ehd.Batch(sims[:2])
    h = sims[0].handle
    L = lbm_ehd.lib()
    state = sims[0].save_state()              # saving is allowed
    calls = [lambda: L.lbm_ehd_step(h), lambda: L.lbm_ehd_run(h, 4),
             lambda: L.lbm_ehd_presolve(h, 2),
             lambda: L.lbm_ehd_presolve_to(h, 1e-6, 10, 5, None, None),
             lambda: L.lbm_ehd_init_droplet(h, 23.5, 23.5, 8.0, 0.0, 0),
             lambda: L.lbm_ehd_set_launch(h, 1, 4),
             lambda: L.lbm_ehd_load_state(h, state.ctypes.data_as(ctypes.c_void_p), state.size)]
    for c in calls:
        assert c() == lbm_ehd.LBM_ESTATE
    other = lbm_ehd.lbm_ehd_batch_create([])
    assert L.lbm_ehd_batch_add(other, h) == lbm_ehd.LBM_EINVAL
    b.run(4)
    b.synchronize()
    assert sims[0].time == 4
    b.remove(sims[0])
    sims[0].step(2)
    assert sims[0].time == 6
    assert L.lbm_ehd_batch_add(other, h) == lbm_ehd.LBM_OK
    lbm_ehd.lbm_ehd_batch_destroy(other)      # releases its members
    sims[0].step(2)
    sims[1].close()                           # a member: leaves the batch first
    assert len(b) == 0
    b.add(sims[2])
    b.run(2)
    b.synchronize()
    b.close()
    sims[2].step(1)
    for s in sims:
        s.close()


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_checkpoint_refuses_other_references(precision):
    """A saved state holds deviations from references set by dpsi, c0, the
    wall types and the g rates (and, with 16-bit storage, the ion offsets):
    loading it where any of these differ is LBM_EINVAL; where only other
    parameters differ it loads."""
    p = workloads.lattice_params(48, 8.0)
    a = lbm_ehd.Simulation(dict(p, precision=precision), device="cuda:0")
    a.init_droplet(23.5, 23.5, 8.0)
    a.step(3)
    state = a.save_state()
    for change in (dict(dpsi=p["dpsi"] * 1.5), dict(c0=2.0), dict(theta=0.5),
                   dict(walls="insulating"), dict(side_walls=1)):
        s = lbm_ehd.Simulation(dict(p, precision=precision, **change), device="cuda:0")
        with pytest.raises(lbm_ehd.LbmError) as e:
            s.load_state(state)
        assert e.value.code == lbm_ehd.LBM_EINVAL, change
        s.close()
    ok = lbm_ehd.Simulation(dict(p, precision=precision, zeta=2e-3, eta_r=2.0), device="cuda:0")
    ok.load_state(state)
    assert ok.time == 3
    ok.step(2)
    for s in (a, ok):
        s.close()
