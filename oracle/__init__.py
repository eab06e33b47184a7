"""FP64 CPU oracle for the phase-field MRT lattice Boltzmann EHD method.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, plain reference the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product package
never does.  It shares no code with the GPU library: its C source
(``lbm_ehd_oracle.c``) is compiled here with gcc and driven through ctypes.

Every function follows Sec. 4 of Zheng, Wang, Xiong, Huang, Luo,
"Phase-field lattice Boltzmann method for two-phase electrohydrodynamic flows
induced by Onsager-Wien effect" (arXiv 2501.04920); the C source cites the
equation behind each step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_ehd_oracle.c")
LIB = os.path.join(HERE, "liblbm_ehd_oracle.so")

FIELDS = ("phi", "psi", "cp", "cm", "rhoe", "ux", "uy", "p", "Ex", "Ey")

WALLS = {"electrodes": 0, "insulating": 1, "periodic": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("walls", ctypes.c_int32), ("reaction", ctypes.c_int32),
        ("poisson_form", ctypes.c_int32), ("flow", ctypes.c_int32),
        ("ion_force", ctypes.c_int32), ("poisson_iters", ctypes.c_int32),
        ("mask_f", ctypes.c_int32), ("mask_h", ctypes.c_int32),
        ("mask_p", ctypes.c_int32), ("mask_n", ctypes.c_int32),
        ("mask_g", ctypes.c_int32), ("poisson_norm", ctypes.c_int32),
        ("side_walls", ctypes.c_int32), ("local_field", ctypes.c_int32),
        ("rho_v", ctypes.c_double), ("rho_r", ctypes.c_double),
        ("eta_v", ctypes.c_double), ("eta_r", ctypes.c_double),
        ("M_phi", ctypes.c_double), ("W", ctypes.c_double), ("zeta", ctypes.c_double),
        ("theta", ctypes.c_double), ("dpsi", ctypes.c_double),
        ("eps_v", ctypes.c_double), ("eps_r", ctypes.c_double),
        ("mu_v", ctypes.c_double), ("mu_r", ctypes.c_double),
        ("m_ratio", ctypes.c_double), ("v_th", ctypes.c_double),
        ("c0", ctypes.c_double), ("q", ctypes.c_double), ("gamma_v", ctypes.c_double),
        ("force_x", ctypes.c_double), ("force_y", ctypes.c_double),
        ("s_free", ctypes.c_double), ("n_eps", ctypes.c_double),
        ("ion_q9", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.POINTER(OracleParams)
        L.orc_sizeof_params.restype = ctypes.c_int
        L.orc_params_default.argtypes = [pp]
        L.orc_create.argtypes = [pp]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_init_droplet.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_uint64]
        L.orc_init_fields.argtypes = [ctypes.c_void_p, dp, dp, dp, dp, dp, dp]
        L.orc_poisson_presolve.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_step.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_get_step.argtypes = [ctypes.c_void_p]
        L.orc_get_step.restype = ctypes.c_long
        L.orc_fields.argtypes = [ctypes.c_void_p, dp]
        L.orc_sums.argtypes = [ctypes.c_void_p, dp]
        L.orc_get_state.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_set_state.argtypes = [ctypes.c_void_p, dp, dp]
        L.orc_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_splitmix64.restype = ctypes.c_uint64
        L.orc_noise.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_noise.restype = ctypes.c_double
        L.orc_lattice.argtypes = [ip, ip, dp, ip, ip, dp]
        L.orc_matrices.argtypes = [dp, dp, dp, dp]
        L.orc_matrices.restype = ctypes.c_int
        L.orc_mrt.argtypes = [ctypes.c_int, dp, dp, dp]
        L.orc_feq.argtypes = [ctypes.c_double] * 4 + [dp]
        L.orc_fforce.argtypes = [ctypes.c_double] * 6 + [dp]
        L.orc_heq.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_hforce.argtypes = [ctypes.c_double] * 6 + [dp]
        L.orc_unit_normal.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_ioneq.argtypes = [ctypes.c_int] + [ctypes.c_double] * 3 + [dp]
        L.orc_ionsrc.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [ctypes.c_int, dp]
        L.orc_iondrift.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [dp]
        L.orc_npop.argtypes = [ctypes.c_void_p]
        L.orc_npop.restype = ctypes.c_int
        L.orc_geq.argtypes = [ctypes.c_double, dp]
        L.orc_ion_solve.argtypes = [ctypes.c_double] * 3 + [dp]
        L.orc_stencil_field.argtypes = [pp, dp, ctypes.c_int, dp, dp, dp]
        if L.orc_sizeof_params() != ctypes.sizeof(OracleParams):
            raise RuntimeError("oracle parameter struct layout mismatch")
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(**kw) -> OracleParams:
    """Oracle parameters: library defaults overridden by keyword values.

    ``walls`` may be given by name ("electrodes", "insulating", "periodic")."""
    p = OracleParams()
    lib().orc_params_default(ctypes.byref(p))
    names = {f[0] for f in OracleParams._fields_}
    for k, v in kw.items():
        if k == "walls" and isinstance(v, str):
            v = WALLS[v]
        if k not in names:
            raise KeyError("unknown oracle parameter %r" % k)
        setattr(p, k, v)
    return p


class Oracle:
    """One simulation held by the oracle."""

    def __init__(self, params: dict):
        self.params = make_params(**params)
        self.nx, self.ny = self.params.nx, self.params.ny
        self._h = lib().orc_create(ctypes.byref(self.params))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def init_droplet(self, xc, yc, radius, noise=0.0, seed=0, presolve=0):
        lib().orc_init_droplet(self._h, xc, yc, radius, noise, seed)
        if presolve:
            lib().orc_poisson_presolve(self._h, int(presolve))
        return self

    def init_fields(self, phi, cp, cm, psi, ux=None, uy=None):
        """Equilibrium populations for the given fields [ny][nx] (pressure 0)."""
        shp = (self.ny, self.nx)
        arrs = [np.ascontiguousarray(np.broadcast_to(a, shp), dtype=np.float64)
                for a in (phi, cp, cm, psi)]
        vel = [None if a is None else
               np.ascontiguousarray(np.broadcast_to(a, shp), dtype=np.float64) for a in (ux, uy)]
        self._keep = arrs + vel
        lib().orc_init_fields(self._h, *[_dp(a) for a in arrs],
                              *[None if a is None else _dp(a) for a in vel])
        return self

    def presolve(self, iters: int):
        lib().orc_poisson_presolve(self._h, int(iters))
        return self

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))
        return self

    @property
    def time(self) -> int:
        return int(lib().orc_get_step(self._h))

    def fields(self) -> dict:
        out = np.empty((len(FIELDS), self.ny, self.nx))
        lib().orc_fields(self._h, _dp(out))
        return {k: out[i] for i, k in enumerate(FIELDS)}

    def sums(self) -> dict:
        out = np.empty(4)
        lib().orc_sums(self._h, _dp(out))
        return {"sum_phi": out[0], "sum_rhoe": out[1], "sum_p": out[2], "sum_n": out[3]}

    @property
    def npop(self) -> int:
        """Populations per cell: 33, or 41 with the ions on D2Q9."""
        return int(lib().orc_npop(self._h))

    def get_state(self):
        pop = np.empty((self.npop, self.ny, self.nx))
        jp = np.empty((2, self.ny, self.nx))
        lib().orc_get_state(self._h, _dp(pop), _dp(jp))
        return pop, jp

    def set_state(self, pop: np.ndarray, jprev: np.ndarray):
        pop = np.ascontiguousarray(pop, dtype=np.float64)
        jprev = np.ascontiguousarray(jprev, dtype=np.float64)
        assert pop.shape == (self.npop, self.ny, self.nx) and jprev.shape == (2, self.ny, self.nx)
        lib().orc_set_state(self._h, _dp(pop), _dp(jprev))


# ---------------------------------------------------------------------------
# Pieces, for the pins.
# ---------------------------------------------------------------------------
def lattice():
    ci = (ctypes.c_int * 9)
    cx9, cy9, cx5, cy5 = ci(), ci(), (ctypes.c_int * 5)(), (ctypes.c_int * 5)()
    w9, w5 = np.empty(9), np.empty(5)
    lib().orc_lattice(cx9, cy9, _dp(w9), cx5, cy5, _dp(w5))
    return (np.array(cx9[:]), np.array(cy9[:]), w9, np.array(cx5[:]), np.array(cy5[:]), w5)


def matrices():
    m9, m9i, n5, n5i = np.empty((9, 9)), np.empty((9, 9)), np.empty((5, 5)), np.empty((5, 5))
    rc = lib().orc_matrices(_dp(m9), _dp(m9i), _dp(n5), _dp(n5i))
    if rc:
        raise RuntimeError("singular transformation matrix")
    return m9, m9i, n5, n5i


def mrt(q: int, s):
    s = np.ascontiguousarray(s, dtype=np.float64)
    A, B = np.empty((q, q)), np.empty((q, q))
    lib().orc_mrt(q, _dp(s), _dp(A), _dp(B))
    return A, B


def _vec(fn, n, *args):
    out = np.empty(n)
    fn(*args, _dp(out))
    return out


def feq(p, rho, ux, uy):
    return _vec(lib().orc_feq, 9, p, rho, ux, uy)


def fforce(ux, uy, grx, gry, Fx, Fy):
    return _vec(lib().orc_fforce, 9, ux, uy, grx, gry, Fx, Fy)


def heq(phi, ux, uy):
    return _vec(lib().orc_heq, 9, phi, ux, uy)


def unit_normal(gx, gy, n_eps):
    return _vec(lib().orc_unit_normal, 2, gx, gy, n_eps)


def hforce(dJx, dJy, nx, ny, phi, W):
    return _vec(lib().orc_hforce, 9, dJx, dJy, nx, ny, phi, W)


def ioneq(c, ux, uy, q=5):
    """Eq. (38) on the ion lattice of q = 5 or 9 velocities."""
    return _vec(lib().orc_ioneq, q, int(q), c, ux, uy)


def ionsrc(R, c, Fx, Fy, with_L=1, q=5):
    return _vec(lib().orc_ionsrc, q, int(q), R, c, Fx, Fy, int(with_L))


def iondrift(mu, c, gx, gy, q=5):
    return _vec(lib().orc_iondrift, q, int(q), mu, c, gx, gy)


def geq(psi):
    return _vec(lib().orc_geq, 5, psi)


def ion_solve(cbp, cbm, lam0):
    return _vec(lib().orc_ion_solve, 2, cbp, cbm, lam0)


def splitmix64(seed: int, n: int) -> int:
    return int(lib().orc_splitmix64(seed, n))


def noise(seed: int, n: int) -> float:
    return float(lib().orc_noise(seed, n))


def stencil_field(field: np.ndarray, ghost: int = 0, **params):
    """grad_x, grad_y and Laplacian of ``field`` [ny][nx] by Eq. (59) and the
    isotropic Laplacian, with the wall ghost rule ``ghost`` (0 mirror, 1 odd
    about the electrode potentials)."""
    f = np.ascontiguousarray(field, dtype=np.float64)
    ny, nx = f.shape
    p = make_params(nx=nx, ny=ny, **params)
    gx, gy, lap = np.empty_like(f), np.empty_like(f), np.empty_like(f)
    lib().orc_stencil_field(ctypes.byref(p), _dp(f), int(ghost), _dp(gx), _dp(gy), _dp(lap))
    return gx, gy, lap


from .deformation import deformation  # noqa: E402  (numpy post-processing)
