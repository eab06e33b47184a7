"""Python binding of the lbm_ehd C ABI (include/lbm_ehd.h).

Argument marshalling only: every step of the method runs in the HIP library
``liblbm_ehd.so`` built from ``csrc/``.  PyTorch supplies device memory and
the stream (see :class:`Simulation`).  If the library is missing the import of
any entry point raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LBM_EHD_LIB", os.path.join(HERE, "liblbm_ehd.so"))

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE, LBM_ERANGE = (
    0, -1, -2, -3, -4, -5, -6)
PRECISIONS = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp32f64": 5}
WALLS = {"electrodes": 0, "insulating": 1, "periodic": 2}
FIELDS = ("phi", "psi", "cp", "cm", "rhoe", "ux", "uy", "p", "Ex", "Ey")
FIELD_BITS = {name: 1 << i for i, name in enumerate(FIELDS)}


class LbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("lbm_ehd error %d: %s" % (code, message))
        self.code = code


class lbm_ehd_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("walls", ctypes.c_int32),
        ("reaction", ctypes.c_int32), ("poisson_form", ctypes.c_int32),
        ("poisson_norm", ctypes.c_int32), ("flow", ctypes.c_int32),
        ("ion_force", ctypes.c_int32), ("poisson_iters", ctypes.c_int32),
        ("mask_f", ctypes.c_int32), ("mask_h", ctypes.c_int32),
        ("mask_p", ctypes.c_int32), ("mask_n", ctypes.c_int32),
        ("mask_g", ctypes.c_int32), ("side_walls", ctypes.c_int32),
        ("local_field", ctypes.c_int32), ("poisson_max", ctypes.c_int32),
        ("rho_v", ctypes.c_double), ("rho_r", ctypes.c_double),
        ("eta_v", ctypes.c_double), ("eta_r", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("W", ctypes.c_double), ("zeta", ctypes.c_double),
        ("theta", ctypes.c_double), ("dpsi", ctypes.c_double),
        ("eps_v", ctypes.c_double), ("eps_r", ctypes.c_double),
        ("mu_v", ctypes.c_double), ("mu_r", ctypes.c_double),
        ("m_ratio", ctypes.c_double), ("v_th", ctypes.c_double),
        ("c0", ctypes.c_double), ("q", ctypes.c_double), ("gamma_v", ctypes.c_double),
        ("force_x", ctypes.c_double), ("force_y", ctypes.c_double),
        ("s_free", ctypes.c_double), ("poisson_tol", ctypes.c_double),
        ("n_eps", ctypes.c_double), ("diag_every", ctypes.c_int32), ("inplace", ctypes.c_int32),
        ("ion_q9", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class lbm_ehd_groups(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("radius", ctypes.c_double), ("W", ctypes.c_double), ("Ca_E", ctypes.c_double),
        ("W0", ctypes.c_double), ("beta", ctypes.c_double),
        ("eps_r", ctypes.c_double), ("mu_r", ctypes.c_double), ("rho_r", ctypes.c_double),
        ("eta_r", ctypes.c_double), ("m_ratio", ctypes.c_double), ("sigma_r", ctypes.c_double),
        ("reaction", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("U", ctypes.c_double), ("alpha", ctypes.c_double), ("zeta", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("eta_v", ctypes.c_double), ("eps_v", ctypes.c_double),
    ]


class lbm_ehd_device(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_void_p),
        ("pop", ctypes.c_void_p * 2), ("pop_bytes", ctypes.c_size_t),
        ("aux", ctypes.c_void_p), ("aux_bytes", ctypes.c_size_t),
    ]


class lbm_ehd_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("sum_phi", ctypes.c_double), ("sum_rhoe", ctypes.c_double),
        ("sum_p", ctypes.c_double), ("sum_n", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
        ("D", ctypes.c_double), ("L", ctypes.c_double), ("H", ctypes.c_double),
        ("presolve_iters", ctypes.c_int64), ("presolve_residual", ctypes.c_double),
    ]


class lbm_ehd_request_info(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("state", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("steps_done", ctypes.c_int64), ("steps_total", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("footprint", ctypes.c_size_t),
                ("diag", lbm_ehd_diag)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib() -> ctypes.CDLL:
    """The HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm_ehd.so is not built (run __graft_entry__.build()); "
                               "there is no CPU fallback")
        # torch ships its own HIP runtime and loads it into the global symbol
        # scope.  Importing torch first makes the library's HIP calls bind to
        # that same runtime: one runtime per process, so the buffers, streams
        # and events torch hands over and the library's kernels share queues
        # (with two runtimes, whichever initialises second finds no GPU).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        sig = {
            "lbm_ehd_params_default": [P(lbm_ehd_params)],
            "lbm_ehd_params_from_groups": [P(lbm_ehd_groups), P(lbm_ehd_params)],
            "lbm_ehd_required_bytes": [P(lbm_ehd_params), P(ctypes.c_size_t),
                                       P(ctypes.c_size_t)],
            "lbm_ehd_create": [P(lbm_ehd_params), P(lbm_ehd_device), P(vp)],
            "lbm_ehd_init_droplet": [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_uint64],
            "lbm_ehd_init_fields": [vp, _dp, _dp, _dp, _dp, _dp, _dp],
            "lbm_ehd_presolve": [vp, ctypes.c_int32],
            "lbm_ehd_presolve_to": [vp, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    P(ctypes.c_int32), P(ctypes.c_double)],
            "lbm_ehd_step": [vp],
            "lbm_ehd_run": [vp, ctypes.c_int64],
            "lbm_ehd_get_fields": [vp, ctypes.c_uint32, _dp, ctypes.c_size_t],
            "lbm_ehd_diagnostics": [vp, P(lbm_ehd_diag)],
            "lbm_ehd_invariants_noalloc": [vp, P(lbm_ehd_diag)],
            "lbm_ehd_synchronize": [vp],
            "lbm_ehd_destroy": [vp],
            "lbm_ehd_state_bytes": [vp, P(ctypes.c_size_t)],
            "lbm_ehd_save_state": [vp, vp, ctypes.c_size_t],
            "lbm_ehd_load_state": [vp, vp, ctypes.c_size_t],
            "lbm_ehd_set_launch": [vp, ctypes.c_int32, ctypes.c_int32],
            "lbm_ehd_get_launch": [vp, P(ctypes.c_int32), P(ctypes.c_int32)],
            "lbm_ehd_batch_create": [P(vp), ctypes.c_int32, vp, P(vp)],
            "lbm_ehd_batch_add": [vp, vp],
            "lbm_ehd_batch_remove": [vp, vp],
            "lbm_ehd_batch_set_launch": [vp, ctypes.c_int32, ctypes.c_int32],
            "lbm_ehd_batch_get_launch": [vp, P(ctypes.c_int32), P(ctypes.c_int32)],
            "lbm_ehd_batch_set_graph_steps": [vp, ctypes.c_int32],
            "lbm_ehd_batch_run": [vp, ctypes.c_int64],
            "lbm_ehd_batch_autotune": [vp, ctypes.c_int32, P(ctypes.c_int32),
                                       P(ctypes.c_int32), P(ctypes.c_int64)],
            "lbm_ehd_batch_synchronize": [vp],
            "lbm_ehd_batch_destroy": [vp],
            "lbm_ehd_footprint_bytes": [P(lbm_ehd_params), P(ctypes.c_size_t)],
            "lbm_ehd_server_create": [ctypes.c_size_t, ctypes.c_int32, P(vp)],
            "lbm_ehd_server_submit": [vp, P(lbm_ehd_params), ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.c_int64, P(ctypes.c_int64)],
            "lbm_ehd_server_advance": [vp, P(ctypes.c_int32), P(ctypes.c_int32)],
            "lbm_ehd_server_info": [vp, ctypes.c_int64, P(lbm_ehd_request_info)],
            "lbm_ehd_server_fields": [vp, ctypes.c_int64, ctypes.c_uint32, _dp, ctypes.c_size_t],
            "lbm_ehd_server_release": [vp, ctypes.c_int64],
            "lbm_ehd_server_destroy": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int32
        L.lbm_ehd_server_used_bytes.argtypes = [vp]
        L.lbm_ehd_server_used_bytes.restype = ctypes.c_size_t
        L.lbm_ehd_server_last_error.argtypes = []
        L.lbm_ehd_server_last_error.restype = ctypes.c_char_p
        L.lbm_ehd_batch_size.argtypes = [vp]
        L.lbm_ehd_batch_size.restype = ctypes.c_int32
        L.lbm_ehd_time.argtypes = [vp]
        L.lbm_ehd_time.restype = ctypes.c_int64
        L.lbm_ehd_last_error.argtypes = []
        L.lbm_ehd_last_error.restype = ctypes.c_char_p
        L.lbm_ehd_stream_copy.argtypes = [vp, vp, ctypes.c_size_t, vp, ctypes.c_int32]
        L.lbm_ehd_stream_copy.restype = ctypes.c_int32
        L.lbm_ehd_bytes_per_lup.argtypes = [ctypes.c_int32]
        L.lbm_ehd_bytes_per_lup.restype = ctypes.c_double
        _lib = L
    return _lib


def _check(code: int):
    if code != LBM_OK:
        raise LbmError(code, lbm_ehd_last_error())


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI).
# ---------------------------------------------------------------------------
def lbm_ehd_last_error() -> str:
    return lib().lbm_ehd_last_error().decode()


def lbm_ehd_params_default() -> lbm_ehd_params:
    p = lbm_ehd_params()
    _check(lib().lbm_ehd_params_default(ctypes.byref(p)))
    return p


def lbm_ehd_params_from_groups(g: lbm_ehd_groups) -> lbm_ehd_params:
    p = lbm_ehd_params()
    _check(lib().lbm_ehd_params_from_groups(ctypes.byref(g), ctypes.byref(p)))
    return p


def lbm_ehd_required_bytes(p: lbm_ehd_params):
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().lbm_ehd_required_bytes(ctypes.byref(p), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def lbm_ehd_create(p: lbm_ehd_params, dev: lbm_ehd_device | None = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().lbm_ehd_create(ctypes.byref(p), ctypes.byref(dev) if dev is not None else None,
                                ctypes.byref(h)))
    return h


def lbm_ehd_init_droplet(h, xc, yc, radius, noise=0.0, seed=0):
    _check(lib().lbm_ehd_init_droplet(h, xc, yc, radius, noise, seed))


def _host(a, shape):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64)
    return arr, arr.ctypes.data_as(_dp)


def lbm_ehd_init_fields(h, ny, nx, phi, cp, cm, psi, ux=None, uy=None):
    keep = [_host(a, (ny, nx)) for a in (phi, cp, cm, psi, ux, uy)]
    _check(lib().lbm_ehd_init_fields(h, *[k[1] for k in keep]))


def lbm_ehd_presolve(h, iters: int):
    _check(lib().lbm_ehd_presolve(h, int(iters)))


def lbm_ehd_presolve_to(h, tol: float, max_iters: int, check_every: int = 100):
    """Returns (sweeps done, last convergence residual)."""
    it, r = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib().lbm_ehd_presolve_to(h, float(tol), int(max_iters), int(check_every),
                                      ctypes.byref(it), ctypes.byref(r)))
    return it.value, r.value


def lbm_ehd_step(h):
    _check(lib().lbm_ehd_step(h))


def lbm_ehd_run(h, nsteps: int):
    _check(lib().lbm_ehd_run(h, int(nsteps)))


def lbm_ehd_get_fields(h, ny, nx, mask=0x3FF) -> np.ndarray:
    nsel = bin(mask & 0x3FF).count("1")
    out = np.empty((nsel, ny, nx))
    _check(lib().lbm_ehd_get_fields(h, mask, out.ctypes.data_as(_dp), out.size))
    return out


def lbm_ehd_diagnostics(h) -> lbm_ehd_diag:
    d = lbm_ehd_diag()
    code = lib().lbm_ehd_diagnostics(h, ctypes.byref(d))
    if code not in (LBM_OK, LBM_ENONFINITE):
        _check(code)
    return d


def lbm_ehd_invariants_noalloc(h) -> lbm_ehd_diag:
    d = lbm_ehd_diag()
    code = lib().lbm_ehd_invariants_noalloc(h, ctypes.byref(d))
    if code not in (LBM_OK, LBM_ENONFINITE):
        _check(code)
    return d


def lbm_ehd_state_bytes(h) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbm_ehd_state_bytes(h, ctypes.byref(n)))
    return n.value


def lbm_ehd_save_state(h) -> np.ndarray:
    buf = np.empty(lbm_ehd_state_bytes(h), dtype=np.uint8)
    _check(lib().lbm_ehd_save_state(h, buf.ctypes.data_as(ctypes.c_void_p), buf.size))
    return buf


def lbm_ehd_load_state(h, state: np.ndarray):
    state = np.ascontiguousarray(state, dtype=np.uint8)
    _check(lib().lbm_ehd_load_state(h, state.ctypes.data_as(ctypes.c_void_p), state.size))


def lbm_ehd_time(h) -> int:
    return int(lib().lbm_ehd_time(h))


def lbm_ehd_synchronize(h):
    _check(lib().lbm_ehd_synchronize(h))


def lbm_ehd_destroy(h):
    _check(lib().lbm_ehd_destroy(h))


def lbm_ehd_set_launch(h, waves: int, tile_rows: int):
    _check(lib().lbm_ehd_set_launch(h, waves, tile_rows))


def lbm_ehd_get_launch(h):
    w, r = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lbm_ehd_get_launch(h, ctypes.byref(w), ctypes.byref(r)))
    return w.value, r.value


def lbm_ehd_batch_create(handles, stream_ptr=None) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * max(1, len(handles)))(*handles)
    out = ctypes.c_void_p()
    _check(lib().lbm_ehd_batch_create(arr, len(handles), stream_ptr, ctypes.byref(out)))
    return out


def lbm_ehd_batch_add(b, h):
    _check(lib().lbm_ehd_batch_add(b, h))


def lbm_ehd_batch_remove(b, h):
    _check(lib().lbm_ehd_batch_remove(b, h))


def lbm_ehd_batch_size(b) -> int:
    return int(lib().lbm_ehd_batch_size(b))


def lbm_ehd_batch_set_launch(b, waves: int, tile_rows: int):
    _check(lib().lbm_ehd_batch_set_launch(b, waves, tile_rows))


def lbm_ehd_batch_get_launch(b):
    w, r = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().lbm_ehd_batch_get_launch(b, ctypes.byref(w), ctypes.byref(r)))
    return w.value, r.value


def lbm_ehd_batch_set_graph_steps(b, steps: int):
    _check(lib().lbm_ehd_batch_set_graph_steps(b, steps))


def lbm_ehd_batch_run(b, nsteps: int):
    _check(lib().lbm_ehd_batch_run(b, nsteps))


def lbm_ehd_batch_autotune(b, steps_per_trial: int):
    w, r, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().lbm_ehd_batch_autotune(b, steps_per_trial, ctypes.byref(w), ctypes.byref(r),
                                        ctypes.byref(n)))
    return w.value, r.value, n.value


def lbm_ehd_batch_synchronize(b):
    _check(lib().lbm_ehd_batch_synchronize(b))


def lbm_ehd_batch_destroy(b):
    _check(lib().lbm_ehd_batch_destroy(b))


def lbm_ehd_stream_copy(src_ptr: int, dst_ptr: int, nbytes: int, stream_ptr: int, width=4):
    _check(lib().lbm_ehd_stream_copy(src_ptr, dst_ptr, nbytes, stream_ptr, width))


def lbm_ehd_bytes_per_lup(precision) -> float:
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    return float(lib().lbm_ehd_bytes_per_lup(precision))


# ---------------------------------------------------------------------------
# Convenience owner: torch allocates the state and provides the stream.
# ---------------------------------------------------------------------------
def make_params(**kw) -> lbm_ehd_params:
    """Library defaults overridden by keyword values; ``precision`` and
    ``walls`` may be given by name."""
    p = lbm_ehd_params_default()
    names = {f[0] for f in lbm_ehd_params._fields_}
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "walls" and isinstance(v, str):
            v = WALLS[v]
        if k not in names:
            raise KeyError("unknown parameter %r" % k)
        setattr(p, k, v)
    return p


class Simulation:
    """One simulation whose state lives in torch-allocated HBM.

    The population ping-pong buffers and the (phi u) buffer are torch uint8
    tensors on ``device``; the library launches on torch's current stream of
    that device at creation time."""

    def __init__(self, params, device="cuda"):
        import torch

        self.params = params if isinstance(params, lbm_ehd_params) else make_params(**params)
        self.nx, self.ny = self.params.nx, self.params.ny
        pop_bytes, aux_bytes = lbm_ehd_required_bytes(self.params)
        self.device = torch.device(device)
        nbuf = 1 if self.params.inplace else 2
        with torch.cuda.device(self.device):
            self._bufs = [torch.empty(pop_bytes, dtype=torch.uint8, device=self.device)
                          for _ in range(nbuf)]
            self._aux = torch.empty(aux_bytes, dtype=torch.uint8, device=self.device)
            self.stream = torch.cuda.current_stream(self.device)
            dev = lbm_ehd_device()
            dev.stream = ctypes.c_void_p(self.stream.cuda_stream)
            dev.pop[0] = self._bufs[0].data_ptr()
            dev.pop[1] = self._bufs[1].data_ptr() if nbuf == 2 else None
            dev.pop_bytes = pop_bytes
            dev.aux = self._aux.data_ptr()
            dev.aux_bytes = aux_bytes
            self.handle = lbm_ehd_create(self.params, dev)

    def close(self):
        if getattr(self, "handle", None):
            lbm_ehd_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_droplet(self, xc, yc, radius, noise=0.0, seed=0, presolve=0):
        lbm_ehd_init_droplet(self.handle, xc, yc, radius, noise, seed)
        if presolve:
            lbm_ehd_presolve(self.handle, presolve)
        return self

    def init_fields(self, phi, cp, cm, psi, ux=None, uy=None):
        lbm_ehd_init_fields(self.handle, self.ny, self.nx, phi, cp, cm, psi, ux, uy)
        return self

    def presolve(self, iters):
        lbm_ehd_presolve(self.handle, iters)
        return self

    def presolve_to(self, tol, max_iters, check_every=100):
        """(sweeps done, convergence residual) of a pre-solve to `tol`."""
        return lbm_ehd_presolve_to(self.handle, tol, max_iters, check_every)

    def step(self, n=1):
        lbm_ehd_run(self.handle, n)
        return self

    @property
    def time(self):
        return lbm_ehd_time(self.handle)

    def fields(self, names=FIELDS) -> dict:
        mask = 0
        for n in names:
            mask |= FIELD_BITS[n]
        arr = lbm_ehd_get_fields(self.handle, self.ny, self.nx, mask)
        order = [n for n in FIELDS if mask & FIELD_BITS[n]]
        return {n: arr[i] for i, n in enumerate(order)}

    def diagnostics(self) -> dict:
        d = lbm_ehd_diagnostics(self.handle)
        return {f[0]: getattr(d, f[0]) for f in lbm_ehd_diag._fields_}

    def synchronize(self):
        lbm_ehd_synchronize(self.handle)

    def save_state(self) -> np.ndarray:
        """Checkpoint: the whole state as host bytes."""
        return lbm_ehd_save_state(self.handle)

    def load_state(self, state: np.ndarray):
        """Resume from save_state() of a simulation of the same grid and
        storage precision."""
        lbm_ehd_load_state(self.handle, state)
        return self

    def set_launch(self, waves: int, tile_rows: int):
        lbm_ehd_set_launch(self.handle, waves, tile_rows)
        return self

    @property
    def launch(self):
        return lbm_ehd_get_launch(self.handle)


class Batch:
    """Simulations advanced together by one launch per step (see
    lbm_ehd_batch_create).  Members are Simulation objects on one device; the
    batch runs on the first member's stream unless another is given."""

    def __init__(self, sims=(), stream=None):
        self.members = list(sims)
        sp = None if stream is None else ctypes.c_void_p(stream.cuda_stream)
        self.handle = lbm_ehd_batch_create([m.handle for m in self.members], sp)

    def add(self, sim):
        lbm_ehd_batch_add(self.handle, sim.handle)
        self.members.append(sim)
        return self

    def remove(self, sim):
        lbm_ehd_batch_remove(self.handle, sim.handle)
        self.members.remove(sim)
        return self

    def __len__(self):
        return lbm_ehd_batch_size(self.handle)

    def set_launch(self, waves: int, tile_rows: int):
        lbm_ehd_batch_set_launch(self.handle, waves, tile_rows)
        return self

    @property
    def launch(self):
        return lbm_ehd_batch_get_launch(self.handle)

    def set_graph_steps(self, steps: int):
        lbm_ehd_batch_set_graph_steps(self.handle, steps)
        return self

    def run(self, nsteps: int):
        lbm_ehd_batch_run(self.handle, nsteps)
        return self

    def autotune(self, steps_per_trial: int = 10):
        """Returns (waves, tile_rows, steps taken by the trials)."""
        return lbm_ehd_batch_autotune(self.handle, steps_per_trial)

    def synchronize(self):
        lbm_ehd_batch_synchronize(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            lbm_ehd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbm_ehd_footprint_bytes(p: lbm_ehd_params) -> int:
    n = ctypes.c_size_t()
    _check(lib().lbm_ehd_footprint_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def _scheck(code: int):
    if code != LBM_OK:
        raise LbmError(code, lib().lbm_ehd_server_last_error().decode())


class Server:
    """Continuous-batching request server (see lbm_ehd_server_create)."""

    def __init__(self, hbm_budget_bytes: int, block_steps: int = 256):
        self.handle = ctypes.c_void_p()
        _scheck(lib().lbm_ehd_server_create(int(hbm_budget_bytes), block_steps,
                                            ctypes.byref(self.handle)))

    def submit(self, params, xc, yc, radius, noise=0.0, seed=0, steps=0) -> int:
        p = params if isinstance(params, lbm_ehd_params) else make_params(**params)
        rid = ctypes.c_int64()
        _scheck(lib().lbm_ehd_server_submit(self.handle, ctypes.byref(p), xc, yc, radius, noise,
                                            seed, steps, ctypes.byref(rid)))
        return rid.value

    def advance(self):
        """One scheduling round; returns (running, queued)."""
        r, q = ctypes.c_int32(), ctypes.c_int32()
        _scheck(lib().lbm_ehd_server_advance(self.handle, ctypes.byref(r), ctypes.byref(q)))
        return r.value, q.value

    def info(self, rid: int) -> dict:
        i = lbm_ehd_request_info()
        _scheck(lib().lbm_ehd_server_info(self.handle, rid, ctypes.byref(i)))
        out = {f[0]: getattr(i, f[0]) for f in lbm_ehd_request_info._fields_ if f[0] != "diag"}
        out["diag"] = {f[0]: getattr(i.diag, f[0]) for f in lbm_ehd_diag._fields_}
        return out

    def fields(self, rid: int, ny: int, nx: int, names=FIELDS) -> dict:
        mask = 0
        for n in names:
            mask |= FIELD_BITS[n]
        order = [n for n in FIELDS if mask & FIELD_BITS[n]]
        out = np.empty((len(order), ny, nx))
        _scheck(lib().lbm_ehd_server_fields(self.handle, rid, mask,
                                            out.ctypes.data_as(_dp), out.size))
        return {n: out[i] for i, n in enumerate(order)}

    def release(self, rid: int):
        _scheck(lib().lbm_ehd_server_release(self.handle, rid))

    @property
    def used_bytes(self) -> int:
        return int(lib().lbm_ehd_server_used_bytes(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            _scheck(lib().lbm_ehd_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
