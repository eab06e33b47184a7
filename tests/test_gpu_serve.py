"""Serving with continuous batching: requests admitted by HBM footprint while
others run, their work sharing one sweep launch per step; each result equals
the same simulation run alone (bitwise: the arithmetic per node does not
depend on the mix), and the budget is never exceeded.
"""
import numpy as np
import pytest

from paper_2501_04920_amd import lbm_ehd, workloads

pytestmark = pytest.mark.gpu

ALL10 = ("phi", "psi", "cp", "cm", "rhoe", "ux", "uy", "p", "Ex", "Ey")

# (nx, ny, radius, eps_r, mu_r, Ca_E, steps)
REQUESTS = [(64, 64, 10.0, 2.0, 1.0, 0.5, 30), (100, 70, 12.0, 0.5, 2.0, 0.25, 57),
            (128, 128, 20.0, 4.0, 0.25, 1.0, 80), (200, 150, 24.0, 0.25, 4.0, 0.5, 44),
            (96, 96, 14.0, 1.0, 1.0, 0.5, 101), (37, 41, 6.0, 1.0, 1.0, 0.5, 0)]


def _params(i, precision, inplace=0):
    nx, ny, r, er, mr, ca, _ = REQUESTS[i]
    p = workloads.lattice_params(ny, r, nx=nx, eps_r=er, mu_r=mr, Ca_E=ca)
    return lbm_ehd.make_params(**dict(p, precision=precision, inplace=inplace))


def _drop(i):
    nx, ny, r = REQUESTS[i][:3]
    return dict(xc=(nx - 1) / 2 + 0.25, yc=(ny - 1) / 2, radius=r, noise=1e-3, seed=100 + i)


def _alone(i, precision, inplace=0):
    sim = lbm_ehd.Simulation(_params(i, precision, inplace), device="cuda:0")
    d = _drop(i)
    sim.init_droplet(d["xc"], d["yc"], d["radius"], d["noise"], d["seed"])
    sim.step(REQUESTS[i][6])
    f = sim.fields()
    sim.close()
    return f


@pytest.mark.parametrize("precision,inplace", [("fp32", 0), ("fp16", 0), ("fp32", 1), ("fp16", 1)])
def test_each_result_is_the_same_alone_and_in_the_mix(precision, inplace):
    fps = [lbm_ehd.lbm_ehd_footprint_bytes(_params(i, precision, inplace))
           for i in range(len(REQUESTS))]
    budget = sorted(fps)[-1] + sorted(fps)[-2]      # two large ones at most at a time
    srv = lbm_ehd.Server(budget, block_steps=16)
    ids, got, infos = [], {}, {}
    max_running, saw_wait = 0, False
    pending = list(range(len(REQUESTS)))
    rounds = 0
    while True:
        # requests arrive over the first rounds, while others are running
        if pending and rounds % 2 == 0:
            i = pending.pop(0)
            d = _drop(i)
            ids.append(srv.submit(_params(i, precision, inplace), d["xc"], d["yc"], d["radius"],
                                  d["noise"], d["seed"], REQUESTS[i][6]))
        running, queued = srv.advance()
        assert srv.used_bytes <= budget
        max_running = max(max_running, running)
        saw_wait |= queued > 0 and running > 0
        # a client collects finished results and releases their memory
        for i, rid in enumerate(ids):
            if i in got:
                continue
            inf = srv.info(rid)
            if inf["state"] == lbm_ehd.REQ_DONE:
                nx, ny = REQUESTS[i][:2]
                got[i] = srv.fields(rid, ny, nx)
                infos[i] = inf
                srv.release(rid)
        rounds += 1
        if not pending and running == 0 and queued == 0 and len(got) == len(REQUESTS):
            break
        assert rounds < 1000
    assert max_running >= 2 and saw_wait
    assert srv.used_bytes == 0
    for i in range(len(REQUESTS)):
        inf = infos[i]
        assert inf["steps_done"] == REQUESTS[i][6]
        assert inf["t_submit"] <= inf["t_start"] <= inf["t_done"]
        want = _alone(i, precision, inplace)
        for k in ALL10:
            assert np.array_equal(got[i][k], want[k]), (i, k)
    srv.close()


def test_server_rejects_and_guards():
    p32 = _params(0, "fp32")
    fp = lbm_ehd.lbm_ehd_footprint_bytes(p32)
    srv = lbm_ehd.Server(fp, block_steps=8)
    with pytest.raises(lbm_ehd.LbmError) as e:
        srv.submit(_params(2, "fp32"), 63.5, 63.5, 20.0, steps=10)   # larger than the budget
    assert e.value.code == lbm_ehd.LBM_ERANGE
    a = srv.submit(p32, 31.5, 31.5, 10.0, steps=10)
    with pytest.raises(lbm_ehd.LbmError) as e:
        srv.submit(_params(0, "fp16"), 31.5, 31.5, 10.0, steps=10)  # another precision
    assert e.value.code == lbm_ehd.LBM_EINVAL
    srv.advance()
    with pytest.raises(lbm_ehd.LbmError) as e:
        srv.release(a)                                                # still running
    assert e.value.code == lbm_ehd.LBM_ESTATE
    with pytest.raises(lbm_ehd.LbmError):
        lbm_ehd.Server(fp, block_steps=7)
    while srv.advance() != (0, 0):
        pass
    assert srv.info(a)["state"] == lbm_ehd.REQ_DONE
    srv.release(a)
    srv.close()
