"""The largest grids the population buffers allow (below 4 GiB each: the
kernels address a buffer with 32-bit byte offsets), at 2048 columns in FP64,
FP32 and FP16 storage, and FP32 and FP16 with in-place streaming.

An x-uniform state (a flat heavy layer between the electrodes, ion and
potential profiles in y only) stays x-uniform: every column of the GPU result
must be bitwise the same (every column runs the same arithmetic, whatever its
strip, band or offset in the buffer), and equal to the oracle run on two
columns (an x-periodic x-uniform state does not see nx) within the storage
form's bar.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from gpu_common import rel_l2, run_gpu, run_oracle  # noqa: E402

from paper_2501_04920_amd import workloads  # noqa: E402

pytestmark = pytest.mark.gpu

NAMES = ("phi", "psi", "cp", "cm", "uy", "p")


def largest_ny(nx, lines, size):
    pitch = (nx + 63) // 64 * 64
    ny = (1 << 32) // (lines * pitch * size) - 2
    while lines * (ny + 2) * pitch * size >= 1 << 32:
        ny -= 1
    return ny


@pytest.mark.parametrize("precision,size,bar,inplace", [("fp64", 8, 1e-10, 0), ("fp32", 4, 2e-5, 0),
                                                        ("fp16", 2, 3e-3, 0), ("fp32", 4, 2e-5, 1),
                                                        ("fp16", 2, 3e-3, 1)])
def test_largest_grid_x_uniform_state(precision, size, bar, inplace):
    nx = 2048
    ny = largest_ny(nx, 33, size)
    p = workloads.lattice_params(ny, 20.0, nx=nx)
    y = np.arange(ny, dtype=np.float64)[:, None]
    y1, y2, W = 0.3 * ny, 0.7 * ny, p["W"]
    phi = 0.5 * (np.tanh(2 * (y - y1) / W) - np.tanh(2 * (y - y2) / W))
    cp = p["c0"] * (1 + 1e-3 * np.sin(2 * np.pi * y / 97.0))
    cm = p["c0"] * (1 - 1e-3 * np.sin(2 * np.pi * y / 61.0))
    psi = p["dpsi"] * (ny - 0.5 - y) / ny
    steps = 20
    print("largest %s grid: %d x %d, in place %d" % (precision, nx, ny, inplace), flush=True)
    o = run_oracle(dict(p, nx=2), fields=(phi, cp, cm, psi), steps=steps)
    ref = {k: v[:, :1] for k, v in o.fields().items()}
    sim = run_gpu(dict(p, inplace=inplace), precision, fields=(phi, cp, cm, psi), steps=steps)
    got = sim.fields(NAMES)
    sim.close()
    for k in NAMES:
        assert np.array_equal(got[k], np.broadcast_to(got[k][:, :1], got[k].shape)), k
    col = {k: got[k][:, :1] for k in NAMES}
    errs = rel_l2(col, ref, dict(p, nx=1), NAMES)
    print("largest %s: %s" % (precision, " ".join("%s=%.2e" % kv for kv in errs.items())),
          flush=True)
    assert max(errs.values()) <= bar
