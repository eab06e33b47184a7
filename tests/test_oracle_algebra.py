"""Exact-algebra pins of the CPU oracle (no GPU).

Each check compares an oracle piece with something fixed independently of it:
lattice isotropy identities, the raw-moment definition of the MRT rows
(Eq. 28, 46), textbook moment identities of the equilibria and forcing terms,
the quadratic that Eq. (41)-(43) define, exactness of the isotropic finite
differences (Eq. 59) on quadratics, published SplitMix64 outputs, and the
deformation factor of an analytic ellipse.
"""
import math

import numpy as np
import pytest


def test_lattice_isotropy(orc):
    cx9, cy9, w9, cx5, cy5, w5 = orc.lattice()
    c9 = np.stack([cx9, cy9], 1).astype(float)
    c5 = np.stack([cx5, cy5], 1).astype(float)
    d = np.eye(2)
    for c, w in ((c9, w9), (c5, w5)):
        assert math.isclose(w.sum(), 1.0, abs_tol=1e-15)
        assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)
        assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), d / 3, atol=1e-16)
        assert np.allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-16)
        # every velocity has its opposite
        for v in c:
            assert any(np.array_equal(-v, u) for u in c)
    # D2Q9 fourth-order isotropy
    t4 = np.einsum("i,ia,ib,ic,id->abcd", w9, c9, c9, c9, c9)
    ref = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.allclose(t4, ref, atol=1e-16)
    # weights: rest, axis, diagonal classes
    assert np.allclose(w9, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    assert np.allclose(w5, [1 / 3] + [1 / 6] * 4)


def test_transform_rows_are_raw_moments(orc):
    cx9, cy9, _, cx5, cy5, _ = orc.lattice()
    m9, m9i, n5, n5i = orc.matrices()
    mono9 = [lambda x, y: 1, lambda x, y: x, lambda x, y: y, lambda x, y: x * x,
             lambda x, y: y * y, lambda x, y: x * y, lambda x, y: x * y * y,
             lambda x, y: x * x * y, lambda x, y: x * x * y * y]
    ref9 = np.array([[f(x, y) for x, y in zip(cx9, cy9)] for f in mono9], float)
    assert np.array_equal(m9, ref9)
    ref5 = np.array([[f(x, y) for x, y in zip(cx5, cy5)] for f in mono9[:5]], float)
    assert np.array_equal(n5, ref5)


def test_inverses_exact(orc):
    m9, m9i, n5, n5i = orc.matrices()
    assert np.array_equal(m9 @ m9i, np.eye(9))
    assert np.array_equal(m9i @ m9, np.eye(9))
    assert np.array_equal(n5 @ n5i, np.eye(5))
    allowed = {0.0, 0.25, -0.25, 0.5, -0.5, 1.0, -1.0}
    assert set(m9i.ravel()) <= allowed and set(n5i.ravel()) <= allowed


@pytest.mark.parametrize("q", [9, 5])
def test_mrt_operators(orc, q):
    m9, m9i, n5, n5i = orc.matrices()
    M, Mi = (m9, m9i) if q == 9 else (n5, n5i)
    # uniform rates: the MRT operator is the BGK operator
    A, B = orc.mrt(q, np.full(q, 1 / 0.8))
    assert np.allclose(A, np.eye(q) / 0.8, atol=1e-15)
    assert np.allclose(B, np.eye(q) * (1 - 0.5 / 0.8), atol=1e-15)
    # general rates: each moment relaxes with its own rate
    s = np.linspace(0.7, 1.9, q)
    A, B = orc.mrt(q, s)
    assert np.allclose(M @ A @ Mi, np.diag(s), atol=1e-14)
    assert np.allclose(M @ B @ Mi, np.diag(1 - s / 2), atol=1e-14)


def _mom(pop, cx, cy):
    c = np.stack([cx, cy], 1).astype(float)
    return pop.sum(), c.T @ pop, np.einsum("i,ia,ib->ab", pop, c, c)


def test_equilibrium_moments(orc):
    cx9, cy9, w9, cx5, cy5, w5 = orc.lattice()
    rng = np.random.default_rng(1)
    for _ in range(5):
        p, rho, phi, c, psi = rng.uniform(0.1, 2.0, 5)
        u = rng.uniform(-0.1, 0.1, 2)
        # Eq. (52)-(53): pressure-based equilibrium, zeroth moment 0,
        # momentum rho u, momentum flux p I + rho u u
        m0, m1, m2 = _mom(orc.feq(p, rho, *u), cx9, cy9)
        assert abs(m0) < 1e-15
        assert np.allclose(m1, rho * u, atol=1e-15)
        assert np.allclose(m2, p * np.eye(2) + rho * np.outer(u, u), atol=1e-14)
        # Eq. (57) applied to an equilibrium returns its pressure
        fe = orc.feq(p, rho, *u)
        r0 = w9[0] * (-1.5 * (u @ u))
        assert math.isclose(3 / 5 * (fe[1:].sum() + rho * r0), p, rel_tol=1e-13)
        # Eq. (31): phi, phi u, phi I / 3
        m0, m1, m2 = _mom(orc.heq(phi, *u), cx9, cy9)
        assert math.isclose(m0, phi, rel_tol=1e-15)
        assert np.allclose(m1, phi * u, atol=1e-15)
        assert np.allclose(m2, phi * np.eye(2) / 3, atol=1e-15)
        # Eq. (38) on D2Q5 and on D2Q9 (the lattice of Eq. 34-35 as printed)
        for q, cx, cy in ((5, cx5, cy5), (9, cx9, cy9)):
            m0, m1, m2 = _mom(orc.ioneq(c, *u, q=q), cx, cy)
            assert math.isclose(m0, c, rel_tol=1e-15)
            assert np.allclose(m1, c * u, atol=1e-15)
            assert np.allclose(m2, c * np.eye(2) / 3, atol=1e-15)
        # Eq. (45): zero sum, Eq. (49) recovers psi, second moment psi I / 3
        g = orc.geq(psi)
        m0, m1, m2 = _mom(g, cx5, cy5)
        assert abs(m0) < 1e-15 and np.allclose(m1, 0)
        assert math.isclose(g[1:].sum() / (1 - w5[0]), psi, rel_tol=1e-15)
        assert np.allclose(m2, psi * np.eye(2) / 3, atol=1e-15)


def test_forcing_moments(orc):
    cx9, cy9, w9, cx5, cy5, w5 = orc.lattice()
    rng = np.random.default_rng(2)
    for _ in range(5):
        u, gr, F, dJ = (rng.uniform(-0.1, 0.1, 2) for _ in range(4))
        nh = rng.normal(size=2)
        nh /= np.linalg.norm(nh)
        phi, W, R, c, mu = rng.uniform(0.1, 0.9), 4.0, *rng.uniform(0.1, 2.0, 3)
        # Eq. (54): zeroth u.grad(rho), first F, second (u.gr I + u gr + gr u)/3
        m0, m1, m2 = _mom(orc.fforce(*u, *gr, *F), cx9, cy9)
        assert math.isclose(m0, u @ gr, rel_tol=1e-12, abs_tol=1e-17)
        assert np.allclose(m1, F, atol=1e-15)
        ref = ((u @ gr) * np.eye(2) + np.outer(u, gr) + np.outer(gr, u)) / 3
        assert np.allclose(m2, ref, atol=1e-15)
        # Eq. (32): zero sum, first moment d(phi u)/dt + lambda n / 3 ...
        lam = 4 * phi * (1 - phi) / W
        m0, m1, m2 = _mom(orc.hforce(*dJ, *nh, phi, W), cx9, cy9)
        assert abs(m0) < 1e-16
        assert np.allclose(m1, dJ + lam * nh / 3, atol=1e-15)
        assert np.allclose(m2, 0, atol=1e-16)
        for q, cx, cy in ((5, cx5, cy5), (9, cx9, cy9)):
            # Eq. (39): R, c F, R I / 3 (and no first moment without L_i)
            m0, m1, m2 = _mom(orc.ionsrc(R, c, *F, 1, q=q), cx, cy)
            assert math.isclose(m0, R, rel_tol=1e-15)
            assert np.allclose(m1, c * F, atol=1e-15)
            assert np.allclose(m2, R * np.eye(2) / 3, atol=1e-15)
            m0, m1, _ = _mom(orc.ionsrc(R, c, *F, 0, q=q), cx, cy)
            assert np.allclose(m1, 0, atol=1e-16)
            # Eq. (40): G_i carries the drift flux mu c grad(psi) and nothing else
            m0, m1, m2 = _mom(orc.iondrift(mu, c, *gr, q=q), cx, cy)
            assert abs(m0) < 1e-16
            assert np.allclose(m1, mu * c * gr, atol=1e-15)
            assert np.allclose(m2, 0, atol=1e-16)


def test_ion_solve_quadratic(orc):
    """Eq. (41)-(43): c+ = cb+ - lam0 c+ c-, c- = cb- - lam0 c+ c-."""
    rng = np.random.default_rng(3)
    for lam0 in [0.0, 1e-8, 1e-4, 4.44e-4, 0.01, 0.5, 3.0]:
        for _ in range(20):
            cbp, cbm = rng.uniform(0.0, 2.0, 2)
            cp, cm = orc.ion_solve(cbp, cbm, lam0)
            assert cp >= 0 and cm >= 0
            scale = cbp + cbm + lam0 * cp * cm + cp + cm  # magnitude of the terms
            assert abs(cp - (cbp - lam0 * cp * cm)) <= 4e-16 * scale
            assert abs(cm - (cbm - lam0 * cp * cm)) <= 4e-16 * scale
            if lam0 >= 1e-4:
                # the form printed in Eq. (42); it loses about eps/lam0 to cancellation
                lit = ((lam0 * cbp - lam0 * cbm - 1)
                       + math.sqrt((1 - lam0 * cbp + lam0 * cbm) ** 2 + 4 * lam0 * cbp)) / (2 * lam0)
                assert abs(lit - cp) <= 1e-15 / lam0 * max(1, cp)
            if lam0 == 0:
                assert cp == cbp and cm == cbm


def test_stencils_exact_on_quadratics(orc):
    ny, nx = 12, 16
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    a, b, c, d, e, f = 0.3, -1.2, 0.7, 0.05, -0.02, 0.03
    chi = a + b * x + c * y + d * x * x + e * x * y + f * y * y
    gx, gy, lap = orc.stencil_field(chi, 0, walls=2)
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    assert np.allclose(gx[inner], (b + 2 * d * x + e * y)[inner], atol=1e-13)
    assert np.allclose(gy[inner], (c + e * x + 2 * f * y)[inner], atol=1e-13)
    assert np.allclose(lap[inner], 2 * d + 2 * f, atol=1e-12)


def test_stencil_wall_ghosts(orc):
    ny, nx, dpsi = 10, 6, 0.8
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    # linear potential between psi(-1/2) = dpsi and psi(ny - 1/2) = 0: the odd
    # ghost makes the gradient exact on every row, including the wall rows
    psi = dpsi * (ny - 0.5 - y) / ny
    gx, gy, lap = orc.stencil_field(psi, 1, walls=0, dpsi=dpsi)
    assert np.allclose(gy, -dpsi / ny, atol=1e-15) and np.allclose(gx, 0, atol=1e-15)
    assert np.allclose(lap, 0, atol=1e-14)
    # mirror ghost for phi: on the wall rows the normal derivative is the
    # central difference with phi(-1) = phi(0) and phi(ny) = phi(ny-1)
    phi = np.cos(np.pi * (y + 0.5) / ny) ** 2 + 0.1 * y
    gx, gy, lap = orc.stencil_field(phi, 0, walls=0)
    assert np.allclose(gy[0], (phi[1] - phi[0]) / 2, atol=1e-15)
    assert np.allclose(gy[-1], (phi[-1] - phi[-2]) / 2, atol=1e-15)
    assert np.allclose(lap[0], 2 * (phi[1] - phi[0]) * (1 / 9 + 2 / 36) * 3, atol=1e-14)
    # periodic in x: the derivative of sin(2 pi x / nx) is the central
    # difference on every column, the wrapped ones included
    xx = np.arange(nx)[None, :] * np.ones((ny, 1))
    k = 2 * np.pi / nx
    gx, _, _ = orc.stencil_field(np.sin(k * xx), 0, walls=2)
    assert np.allclose(gx, np.sin(k) * np.cos(k * xx), atol=1e-15)


def test_splitmix64_published_outputs(orc):
    # First outputs of SplitMix64 started at 0 (reference C code of Vigna).
    assert orc.splitmix64(0, 1) == 0xE220A8397B1DCDAF
    assert orc.splitmix64(0, 2) == 0x6E789E6AA1B965F4
    assert orc.splitmix64(0, 3) == 0x06C45D188009454F
    xs = np.array([orc.noise(7, n) for n in range(1, 20001)])
    assert xs.min() >= -1.0 and xs.max() < 1.0
    assert abs(xs.mean()) < 0.02 and abs(xs.var() - 1 / 3) < 0.01


@pytest.mark.parametrize("a,b", [(30.0, 20.0), (20.0, 28.0), (24.0, 24.0)])
def test_deformation_of_analytic_ellipse(orc, a, b):
    """D = (a - b)/(a + b) for an ellipse of semi-axes a (along y, the field)
    and b (along x) with a tanh rim."""
    ny = nx = 128
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    xc, yc = 63.3, 64.6
    rr = np.sqrt(((x - xc) / b) ** 2 + ((y - yc) / a) ** 2)
    # signed distance to the rim, to first order, along the axes
    dist = (1 - rr) * np.sqrt(a * b)
    phi = 0.5 * (1 + np.tanh(2 * dist / 4.0))
    D, L, H = orc.deformation(phi)
    assert abs(L - 2 * a) < 0.1 and abs(H - 2 * b) < 0.1
    assert abs(D - (a - b) / (a + b)) < 1e-3


def test_unit_normal_reading(orc):
    """grad(phi)/|grad(phi)| of Eq. (1), (32): where the gradient is well
    above the regularisation it is the unit vector along grad(phi) to second
    order in n_eps/|g|; it never exceeds unit length, points along grad(phi)
    and goes to 0 continuously with the gradient; the bare form (n_eps = 0)
    is the unit vector itself, and 0 below 1e-12."""
    rng = np.random.default_rng(7)
    eps = 1e-4
    for _ in range(50):
        g = rng.normal(size=2) * 10.0 ** rng.uniform(-8, 0)
        gn = np.linalg.norm(g)
        n = orc.unit_normal(*g, eps)
        assert np.linalg.norm(n) < 1.0
        assert abs(n[0] * g[1] - n[1] * g[0]) <= 1e-15 * gn   # parallel to g
        assert n @ g > 0
        if gn > 100 * eps:
            assert np.linalg.norm(n - g / gn) <= (eps / gn) ** 2
        if gn < 1e-2 * eps:
            assert np.linalg.norm(n) <= gn / eps                 # continuous at 0
        bare = orc.unit_normal(*g, 0.0)
        assert abs(np.linalg.norm(bare) - 1.0) < 1e-15
    assert np.array_equal(orc.unit_normal(0.0, 0.0, eps), [0.0, 0.0])
    assert np.array_equal(orc.unit_normal(3e-13, 4e-13, 0.0), [0.0, 0.0])
