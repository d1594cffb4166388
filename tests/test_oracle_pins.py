"""Pins of the CPU oracle against what the mathematics fixes.

Each test checks an oracle function against something other than itself: a
closed form, an invariant, a special case with a textbook answer, or an
independent brute-force evaluation written from a different definition
(e.g. the B-spline's piecewise formula instead of the oracle's weights).
"""
import math
from dataclasses import replace as dataclasses_replace
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_2204_12837_amd import inputs as I


# --------------------------------------------------------------------------
# helpers written from definitions, not from the oracle's code

def bspline2(t):
    """Quadratic B-spline M2 (three unit boxes convolved), piecewise form."""
    t = abs(t)
    if t <= 0.5:
        return 0.75 - t * t
    if t <= 1.5:
        return 0.5 * (1.5 - t) ** 2
    return 0.0


def tent_cdf(z):
    """CDF of the linear B-spline (tent on [-1, 1])."""
    if z <= -1:
        return 0.0
    if z < 0:
        return 0.5 * (1 + z) ** 2
    if z < 1:
        return 1 - 0.5 * (1 - z) ** 2
    return 1.0


class _G:
    def __init__(self, dim, n, d=0.1, patch=None, dt=None):
        self.dim = dim
        self.n = tuple(n) + (1,) * (3 - len(n))
        self.d = tuple(d) if isinstance(d, tuple) else (d, d, d)
        self.patch = tuple(patch or self.n[:dim]) + (1,) * (3 - dim)
        self.dt = dt if dt is not None else I.cfl_dt(self.d, dim)

    @property
    def n_patches(self):
        return int(np.prod([self.n[a] // self.patch[a] for a in range(self.dim)]))


STAG_E = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
STAG_B = [(0, 1, 1), (1, 0, 1), (1, 1, 0)]


def field_shape(g):
    return (g.n[2] if g.dim == 3 else 1, g.n[1], g.n[0])


# --------------------------------------------------------------------------
# shape function

def test_shape_matches_bspline_definition():
    rng = np.random.default_rng(1)
    for xi in rng.uniform(-3, 70, 2000):
        for s in (0, 1):
            i, S = O.shape(xi, s)
            for k in range(3):
                node = (i - 1 + k) + 0.5 * s
                assert abs(S[k] - bspline2(xi - node)) <= 1e-15
            # nodes outside the stencil carry no weight
            assert bspline2(xi - (i - 2 + 0.5 * s)) == 0.0 or abs(xi - (i - 2 + 0.5 * s)) >= 1.5 - 1e-12
            assert bspline2(xi - (i + 2 + 0.5 * s)) == 0.0 or abs(xi - (i + 2 + 0.5 * s)) >= 1.5 - 1e-12


def test_shape_moments():
    rng = np.random.default_rng(2)
    for xi in rng.uniform(0, 64, 1000):
        for s in (0, 1):
            i, S = O.shape(xi, s)
            delta = (xi - 0.5 * s) - i
            k = np.array([-1.0, 0.0, 1.0])
            assert abs(S.sum() - 1) <= 4e-16
            assert abs((k * S).sum() - delta) <= 4e-16
            assert abs(((k - delta) ** 2 * S).sum() - 0.25) <= 4e-16
            assert -0.5 - 1e-15 <= delta < 0.5


def test_shape_exact_dyadic_and_tie():
    i, S = O.shape(5.25, 0)
    assert i == 5
    assert [Fraction(v) for v in S] == [Fraction(1, 32), Fraction(11, 16), Fraction(9, 32)]
    # a half-integer position sits between two nodes with weight 1/2 each
    for xi in (3.5, 10.5, 0.5):
        i, S = O.shape(xi, 0)
        w = {i - 1 + k: S[k] for k in range(3) if S[k] != 0}
        assert w == {int(xi - 0.5): 0.5, int(xi + 0.5): 0.5}
    # dual stagger: a position on a dual node has weights (1/8, 3/4, 1/8)
    i, S = O.shape(7.5, 1)
    assert i == 7 and list(S) == [0.125, 0.75, 0.125]


# --------------------------------------------------------------------------
# interpolation

def _rand_fields(g, rng, amp=1.0):
    shp = field_shape(g)
    return rng.uniform(-amp, amp, (3,) + shp), rng.uniform(-amp, amp, (3,) + shp)


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_constant_exact(dim):
    g = _G(dim, (8, 8, 8)[:dim])
    shp = field_shape(g)
    c = np.array([0.3, -1.25, 2.0, 0.5, -0.75, 1.0])
    E = np.stack([np.full(shp, c[k]) for k in range(3)])
    B = np.stack([np.full(shp, c[3 + k]) for k in range(3)])
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 0.8, (dim, 500))
    F = O.interp(g, E, B, x)
    assert np.max(np.abs(F - c[:, None])) <= 4e-16 * np.abs(c).max()


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_linear_and_quadratic(dim):
    """Quadratic B-splines reproduce linear functions exactly and map x^2 to
    x^2 + d^2/4 (second moment 1/4 in cell units)."""
    n = 32
    g = _G(dim, (n,) * dim, d=0.1)
    shp = field_shape(g)
    rng = np.random.default_rng(4)
    a, b = rng.normal(size=dim), rng.normal()
    x = rng.uniform(0.8, 2.4, (dim, 400))  # stencil never wraps
    comps_E, comps_B, expect_lin, expect_q = [], [], [], []
    for st_list, out in ((STAG_E, comps_E), (STAG_B, comps_B)):
        for st in st_list:
            coords = np.meshgrid(*[(np.arange(g.n[ax]) + 0.5 * st[ax]) * g.d[ax] for ax in range(dim)][::-1],
                                 indexing="ij")[::-1]
            lin = b + sum(a[ax] * coords[ax] for ax in range(dim))
            out.append((lin, coords[0] ** 2))
    E = np.stack([c[0].reshape(shp) for c in comps_E])
    B = np.stack([c[0].reshape(shp) for c in comps_B])
    F = O.interp(g, E, B, x)
    lin_exact = b + sum(a[ax] * x[ax] for ax in range(dim))
    assert np.max(np.abs(F - lin_exact[None])) <= 1e-14 * np.abs(lin_exact).max()
    E2 = np.stack([c[1].reshape(shp) for c in comps_E])
    B2 = np.stack([c[1].reshape(shp) for c in comps_B])
    F2 = O.interp(g, E2, B2, x)
    q_exact = x[0] ** 2 + g.d[0] ** 2 / 4
    assert np.max(np.abs(F2 - q_exact[None])) <= 1e-14 * q_exact.max()


@pytest.mark.parametrize("dim", [2, 3])
def test_interp_bruteforce_full_sum(dim):
    """Interpolation equals the sum over every grid node of M2(dx) M2(dy)
    (M2(dz)) F, with periodic images, evaluated by brute force."""
    n = (6, 7, 5)[:dim]
    g = _G(dim, n)
    rng = np.random.default_rng(5)
    E, B = _rand_fields(g, rng)
    L = np.array([g.n[a] * g.d[a] for a in range(dim)])
    x = rng.uniform(0, 1, (dim, 60)) * L[:, None]
    x[0, :4] = [0.0, L[0] * (1 - 1e-16), g.d[0] * 0.5, g.d[0] * 3]  # edges, nodes
    F = O.interp(g, E, B, x)
    for p in range(x.shape[1]):
        for c in range(6):
            st = (STAG_E + STAG_B)[c]
            arr = (E if c < 3 else B)[c % 3]
            tot = 0.0
            for idx in np.ndindex(*arr.shape):
                kk, jj, ii = idx
                ijk = (ii, jj, kk)
                w = 1.0
                for ax in range(dim):
                    pos = x[ax, p] / g.d[ax]
                    nd = ijk[ax] + 0.5 * st[ax]
                    dist = (pos - nd + g.n[ax] / 2) % g.n[ax] - g.n[ax] / 2  # nearest image
                    w *= bspline2(dist)
                tot += w * arr[idx]
            assert abs(F[c, p] - tot) <= 1e-14 * np.abs(arr).max()


# --------------------------------------------------------------------------
# Boris push

def test_boris_pure_B_invariants():
    q, m, dt, Bz = -1.0, 1.0, 0.067175144212722, 1.0
    u0 = np.array([0.3, -0.2, 0.1])
    n = 10000
    xs, us = O.boris_traj(q, m, dt, 2, [0, 0, 0], [0, 0, Bz], [0.5, 0.5, 0], u0, n)
    umag = np.linalg.norm(us, axis=1)
    assert np.max(np.abs(umag - umag[0])) <= 1e-13 * umag[0]
    assert np.all(us[:, 2] == u0[2])  # parallel momentum untouched
    gam = math.sqrt(1 + u0 @ u0)
    omega = abs(q) * Bz / (m * gam)
    theta = 2 * math.atan(omega * dt / 2)
    phase = np.unwrap(np.arctan2(us[:, 1], us[:, 0]))
    expect = phase[0] + (-np.sign(q)) * theta * np.arange(n + 1)
    assert np.max(np.abs(phase - expect)) <= 1e-11


def test_boris_pure_E_exact_and_decimal_positions():
    # dyadic values: every momentum increment is exact
    q, m, dt = -1.0, 1.0, 0.0625
    E = np.array([0.5, -0.25, 0.125])
    u0 = np.array([0.125, 0.0, -0.5])
    n = 200
    xs, us = O.boris_traj(q, m, dt, 3, E, [0, 0, 0], [0, 0, 0], u0, n)
    for k in range(n + 1):
        assert np.array_equal(us[k], u0 + (q / m) * E * dt * k)
    # positions: the leapfrog sum x_{k+1} = x_k + dt u_{k+1/2}/gamma in 50 digits
    getcontext().prec = 50
    x = [Decimal(0)] * 3
    for k in range(1, n + 1):
        u = [Decimal(float(v)) for v in us[k]]
        g = (Decimal(1) + sum(v * v for v in u)).sqrt()
        x = [x[a] + Decimal(dt) * u[a] / g for a in range(3)]
    assert np.max(np.abs(xs[n] - np.array([float(v) for v in x]))) <= 1e-14 * np.abs(xs[n]).max()


def test_boris_pure_E_converges_second_order():
    """x(t) = x0 + (sqrt(1+(u0+a t)^2) - sqrt(1+u0^2))/a for a = qE/m along x;
    the leapfrog with u given at t = -dt/2 is second-order accurate."""
    q, m, Ex, u0, T = 1.0, 1.0, 0.7, 0.4, 2.0
    a = q * Ex / m
    exact = (math.sqrt(1 + (u0 + a * T) ** 2) - math.sqrt(1 + u0 ** 2)) / a
    errs = []
    for nst in (50, 100, 200, 400):
        dt = T / nst
        xs, us = O.boris_traj(q, m, dt, 1, [Ex, 0, 0], [0, 0, 0], [0, 0, 0],
                              [u0 - a * dt / 2, 0, 0], nst)
        errs.append(abs(xs[nst, 0] - exact))
    ratios = [errs[k] / errs[k + 1] for k in range(3)]
    for r in ratios:
        assert abs(r - 4) <= 0.2, ratios


def test_boris_ExB_drift():
    q, m, dt = -1.0, 1.0, 0.067175144212722
    E = np.array([0.0, 0.01, 0.0])
    B = np.array([0.0, 0.0, 1.0])
    vd = np.cross(E, B) / (B @ B)  # (0.01, 0, 0)
    gd = 1 / math.sqrt(1 - vd @ vd)
    n = 2000
    xs, us = O.boris_traj(q, m, dt, 2, E, B, [0, 0, 0], gd * vd, n)
    v = us / np.sqrt(1 + (us ** 2).sum(axis=1))[:, None]
    assert np.max(np.abs(v[1:] - vd)) <= 1e-6 * np.linalg.norm(vd)
    # a gyrating start drifts at vd on average over whole gyro-periods
    # (period from the discrete rotation angle 2 atan(Omega dt / 2), Omega = |q| B / (m gamma))
    u0 = np.array([0.0, 0.05, 0.0])
    omega = abs(q) * 1.0 / (m * math.sqrt(1 + u0 @ u0))
    per = 2 * math.pi * dt / (2 * math.atan(omega * dt / 2))
    nper = 100
    n2 = int(round(nper * per / dt))
    xs, us = O.boris_traj(q, m, dt, 2, E, B, [0, 0, 0], u0, n2)
    mean_v = (xs[n2] - xs[0]) / (n2 * dt)
    # residual of an incomplete last gyration: at most 2 r_L / T_total
    resid = 2 * 0.05 / (n2 * dt) * dt * 2
    assert abs(mean_v[0] - vd[0]) <= 1e-3 * vd[0] + resid
    assert abs(mean_v[1]) <= 1e-3 * vd[0] + resid


# --------------------------------------------------------------------------
# Esirkepov deposit

def _dep(g, q, w, x0, x1, vz=0.0):
    J = np.zeros((3,) + field_shape(g))
    O.deposit(g, q, w, x0, x1, vz, J)
    return J


def _div(g, J):
    out = np.zeros(J.shape[1:])
    for a in range(g.dim):
        ax = 2 - a
        out += (J[a] - np.roll(J[a], 1, axis=ax)) / g.d[a]
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_deposit_continuity_and_total_current(dim):
    g = _G(dim, (8, 9, 7)[:dim])
    rng = np.random.default_rng(7)
    L = np.array([g.n[a] * g.d[a] for a in range(dim)])
    for trial in range(200):
        x0 = rng.uniform(0, 1, dim) * L
        v = rng.uniform(-1, 1, 3)
        v *= rng.uniform(0, 0.999) / np.linalg.norm(v)
        x1 = x0 + g.dt * v[:dim]
        q, w = rng.choice([-1.0, 1.0]), rng.uniform(0.1, 2)
        J = _dep(g, q, w, x0, x1, v[2])
        r0 = O.rho(g, q, x0[:, None], np.array([w]))
        x1w = np.mod(x1, L)
        r1 = O.rho(g, q, x1w[:, None], np.array([w]))
        res = (r1 - r0) / g.dt + _div(g, J)
        scale = abs(q * w) / g.dt
        assert np.max(np.abs(res)) <= 1e-12 * scale
        for a in range(dim):
            assert abs(J[a].sum() - q * w * (x1[a] - x0[a]) / g.dt) <= 1e-12 * scale * g.d[a]
        if dim == 2:
            assert abs(J[2].sum() - q * w * v[2]) <= 1e-14


@pytest.mark.parametrize("dim", [2, 3])
def test_deposit_stationary_and_single_axis(dim):
    g = _G(dim, (10,) * dim)
    rng = np.random.default_rng(8)
    x0 = np.array([0.43, 0.571, 0.66])[:dim]
    J = _dep(g, -1.0, 1.0, x0, x0, 0.0)
    assert np.all(J == 0)
    # motion along x only: Jx(face i+1/2) = q w dx/dt * prod_other S *
    # [Phi(xi1 - i - 1/2) - Phi(xi0 - i - 1/2)], Phi = CDF of the tent
    for trial in range(50):
        x0 = rng.uniform(0.3, 0.7, dim)
        x1 = x0.copy()
        x1[0] += rng.uniform(-0.9, 0.9) * g.d[0]
        q, w = -1.0, 0.7
        J = _dep(g, q, w, x0, x1)
        for a in range(1, dim):
            assert np.all(J[a] == 0) or np.max(np.abs(J[a])) <= 1e-16
        xi0, xi1 = x0 / g.d[0], x1 / g.d[0]
        expect = np.zeros_like(J[0])
        for idx in np.ndindex(*J[0].shape):
            kk, jj, ii = idx
            ijk = (ii, jj, kk)
            wt = 1.0
            for a in range(1, dim):
                wt *= bspline2(x0[a] / g.d[a] - ijk[a])
            face = ii + 0.5
            expect[idx] = q * w * g.d[0] / g.dt * wt * (tent_cdf(xi1[0] - face) - tent_cdf(xi0[0] - face))
        assert np.max(np.abs(J[0] - expect)) <= 1e-13 * abs(q * w) * g.d[0] / g.dt


def test_deposit_transpose_symmetry_2d():
    g = _G(2, (10, 10))
    rng = np.random.default_rng(9)
    for trial in range(50):
        x0 = rng.uniform(0.2, 0.8, 2)
        x1 = x0 + rng.uniform(-0.06, 0.06, 2)
        J = _dep(g, 1.0, 1.0, x0, x1, 0.3)
        Jt = _dep(g, 1.0, 1.0, x0[::-1], x1[::-1], 0.3)
        # swapping x and y swaps Jx with Jy and transposes every grid array
        assert np.allclose(J[0, 0], Jt[1, 0].T, atol=1e-15, rtol=0)
        assert np.allclose(J[1, 0], Jt[0, 0].T, atol=1e-15, rtol=0)
        assert np.allclose(J[2, 0], Jt[2, 0].T, atol=1e-16, rtol=0)


def test_deposit_cyclic_symmetry_3d():
    g = _G(3, (8, 8, 8))
    rng = np.random.default_rng(10)
    for trial in range(20):
        x0 = rng.uniform(0.2, 0.6, 3)
        x1 = x0 + rng.uniform(-0.05, 0.05, 3)
        J = _dep(g, 1.0, 1.0, x0, x1)
        # rotate axes (x, y, z) -> (y, z, x): new position p' = (p_y, p_z, p_x)
        Jr = _dep(g, 1.0, 1.0, np.roll(x0, -1), np.roll(x1, -1))
        # component a of J corresponds to component a-1 of Jr; array axes are (z, y, x)
        for a in range(3):
            A = J[a]                       # A[z, y, x]
            Br = Jr[(a - 1) % 3]           # Br[z', y', x'] with x'=y, y'=z, z'=x
            # explicit index check: A[z, y, x] == Br[x, z, y]
            for (z, y, x) in [(1, 2, 3), (2, 3, 1), (3, 1, 2), (2, 2, 2), (1, 1, 4)]:
                assert abs(A[z, y, x] - Br[x, z, y]) <= 1e-15


def test_deposit_jz_is_path_average_2d():
    """Esirkepov's out-of-plane weight is the average over the straight path
    of the product of linearly varying node weights; Simpson's rule is exact
    for that quadratic in the path parameter."""
    g = _G(2, (10, 10))
    rng = np.random.default_rng(11)
    for trial in range(30):
        x0 = rng.uniform(0.3, 0.7, 2)
        x1 = x0 + rng.uniform(-0.06, 0.06, 2)
        vz, q, w = 0.37, -1.0, 0.5
        J = _dep(g, q, w, x0, x1, vz)

        def nodew(x, ii, jj):
            return bspline2(x[0] / g.d[0] - ii) * 1.0, bspline2(x[1] / g.d[1] - jj)

        for jj in range(10):
            for ii in range(10):
                a0x, a0y = nodew(x0, ii, jj)
                a1x, a1y = nodew(x1, ii, jj)
                f = lambda tau: (a0x + tau * (a1x - a0x)) * (a0y + tau * (a1y - a0y))
                avg = (f(0) + 4 * f(0.5) + f(1)) / 6
                assert abs(J[2, 0, jj, ii] - q * w * vz * avg) <= 1e-15


def test_deposit_cfl_error():
    g = _G(2, (10, 10))
    with pytest.raises(O.OracleError):
        _dep(g, 1.0, 1.0, [0.5, 0.5], [0.5 + 2.1 * g.d[0], 0.5])


# --------------------------------------------------------------------------
# sort / pre-BC / boundary condition

def test_bin_counts_bounds_and_stability():
    wl = I.custom(2, (48, 40), (8, 8), ppc=3, seed=12)
    inp = I.generate(wl)
    sp = O.species_from(inp)[0]
    L = np.array([wl.n[0] * wl.d[0], wl.n[1] * wl.d[1]])
    # push some particles out of the box by less than one period
    sp.x[0, :50] += L[0]
    sp.x[1, 50:100] -= L[1] * 0.999
    ids_in = sp.id.copy()
    O.bin(wl, sp)
    assert np.all(sp.x >= 0) and np.all(sp.x[0] < L[0]) and np.all(sp.x[1] < L[1])
    cells = np.floor(sp.x / np.array(wl.d[:2])[:, None]).astype(np.int64)
    cells = np.minimum(cells, np.array(wl.n[:2])[:, None] - 1)
    P = cells[0] // wl.patch[0] + (wl.n[0] // wl.patch[0]) * (cells[1] // wl.patch[1])
    cnt = np.bincount(P, minlength=wl.n_patches)
    assert np.array_equal(np.diff(sp.off), cnt)
    assert np.all(np.diff(P) >= 0)
    assert np.array_equal(np.sort(sp.id), np.sort(ids_in))
    # stable: within a patch, ids keep their input order (input ids increase)
    for Pp in range(wl.n_patches):
        seg = sp.id[sp.off[Pp]:sp.off[Pp + 1]]
        assert np.all(np.diff(seg) > 0)


def test_bin_wrap_rounding_edge():
    wl = I.custom(2, (16, 16), (8, 8), ppc=1, seed=13)
    inp = I.generate(wl)
    sp = O.species_from(inp)[0]
    L = wl.n[0] * wl.d[0]
    sp.x[0, 0] = -1e-18     # x + L rounds to L: must become 0
    sp.x[0, 1] = L          # exactly L: becomes 0
    sp.x[0, 2] = np.nextafter(L, 0)  # just below L stays, clamped to the last cell
    idx = sp.id[:3].copy()
    O.bin(wl, sp)
    pos = {int(i): k for k, i in enumerate(sp.id)}
    assert sp.x[0, pos[idx[0]]] == 0.0
    assert sp.x[0, pos[idx[1]]] == 0.0
    assert sp.x[0, pos[idx[2]]] == np.nextafter(L, 0)
    assert pos[idx[2]] >= sp.off[1] - (sp.off[1] - sp.off[0])  # in a last-column patch
    k = pos[idx[2]]
    Pp = np.searchsorted(sp.off, k, side="right") - 1
    assert Pp % (wl.n[0] // wl.patch[0]) == wl.n[0] // wl.patch[0] - 1


# --------------------------------------------------------------------------
# whole step

def _run_step(wl, inp, nsteps=1):
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    J = None
    for _ in range(nsteps):
        J = O.step(wl, sps, inp.E, inp.B)
    return sps, J


@pytest.mark.parametrize("dim", [2, 3])
def test_step_continuity_and_total_current(dim):
    if dim == 2:
        wl = I.workload("uniform64")
    else:
        wl = I.custom(3, (16, 16, 16), (8, 8, 8), ppc=2, seed=14, n_species=2, sigma=0.05)
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    rho0 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    x_before = {}
    for k, s in enumerate(sps):
        order = np.argsort(s.id)
        x_before[k] = s.x[:, order].copy()
    J = O.step(wl, sps, inp.E, inp.B)
    rho1 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    res = (rho1 - rho0) / wl.dt + _div(wl, J)
    assert np.max(np.abs(res)) <= 1e-13 * np.abs(rho0).max() / wl.dt
    L = np.array([wl.n[a] * wl.d[a] for a in range(dim)])
    for a in range(dim):
        tot = 0.0
        for k, s in enumerate(sps):
            order = np.argsort(s.id)
            dx = s.x[a, order] - x_before[k][a]
            dx = (dx + L[a] / 2) % L[a] - L[a] / 2
            tot += (s.q * s.w[order] * dx).sum() / wl.dt
        assert abs(J[a].sum() - tot) <= 1e-12 * max(1.0, abs(tot))


def test_step_free_streaming():
    wl = I.custom(2, (32, 32), (8, 8), ppc=2, seed=15, sigma=0.2)
    inp = I.generate(wl)
    inp.E[:] = 0
    inp.B[:] = 0
    sps = O.species_from(inp)
    O.bin(wl, sps[0])
    s = sps[0]
    o0 = np.argsort(s.id)
    x0, u0 = s.x[:, o0].copy(), s.u[:, o0].copy()
    O.step(wl, sps, inp.E, inp.B)
    o1 = np.argsort(s.id)
    assert np.array_equal(s.u[:, o1], u0)
    gam = np.sqrt(1 + (u0 ** 2).sum(axis=0))
    L = wl.n[0] * wl.d[0]
    expect = np.mod(x0 + wl.dt * (u0[:2] * (1 / gam)), L)
    assert np.max(np.abs(s.x[:, o1] - expect)) <= 1e-15 * L


def test_step_species_linearity_and_order_invariance():
    wl = I.custom(2, (24, 24), (8, 8), ppc=4, seed=16, n_species=2, sigma=0.05)
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    parts = []
    for s in sps:
        t = O.OSpecies(s.q, s.m, s.x, s.u, s.w, s.id, wl.n_patches)
        t.off[:] = s.off
        parts.append(O.step(wl, [t], inp.E, inp.B))
    # the combined call needs valid offsets too
    c = [O.OSpecies(s.q, s.m, s.x, s.u, s.w, s.id, wl.n_patches) for s in sps]
    for ci, s in zip(c, sps):
        ci.off[:] = s.off
    J_both = O.step(wl, c, inp.E, inp.B)
    assert np.max(np.abs(J_both - (parts[0] + parts[1]))) <= 1e-15 * np.abs(J_both).max() * 10
    # reversing particle order inside every patch changes J by rounding only
    s = sps[0]
    r = O.OSpecies(s.q, s.m, s.x, s.u, s.w, s.id, wl.n_patches)
    r.off[:] = s.off
    for P in range(wl.n_patches):
        a, b = s.off[P], s.off[P + 1]
        for arr in (r.x, r.u):
            arr[:, a:b] = arr[:, a:b][:, ::-1]
        r.w[a:b] = r.w[a:b][::-1]
        r.id[a:b] = r.id[a:b][::-1]
    Jr = O.step(wl, [r], inp.E, inp.B)
    assert np.max(np.abs(Jr - parts[0])) <= 1e-14 * np.abs(parts[0]).max()
    o1, o2 = np.argsort(t.id), np.argsort(r.id)
    # particles are identical bit for bit (each particle is independent)
    s_again = O.OSpecies(s.q, s.m, s.x, s.u, s.w, s.id, wl.n_patches)
    s_again.off[:] = s.off
    O.step(wl, [s_again], inp.E, inp.B)
    oa = np.argsort(s_again.id)
    assert np.array_equal(s_again.x[:, oa], r.x[:, o2])
    assert np.array_equal(s_again.u[:, oa], r.u[:, o2])


# --------------------------------------------------------------------------
# reflecting walls (particle boundary condition)

def _walls(wl, axes):
    import dataclasses
    return dataclasses.replace(wl, particle_bc=tuple(int(a in axes) for a in range(3)))


def _fold(y, L):
    """Straight-line coordinate y unfolded past walls at 0 and L, folded back
    into [0, L] (a triangle wave), and the parity of the number of walls hit."""
    m = np.mod(y, 2 * L)
    back = m > L
    return np.where(back, 2 * L - m, m), back


@pytest.mark.parametrize("axes", [(0,), (1,), (0, 1)])
def test_walls_free_streaming_is_the_folded_line(axes):
    """Without fields every particle moves on a straight line; walls fold that
    line into the box.  After k steps each position is the fold of x0 + k dt v
    and each momentum component has the sign of the fold's parity."""
    wl = _walls(I.custom(2, (24, 16), (8, 8), ppc=3, seed=41, sigma=0.8), axes)
    inp = I.generate(wl)
    inp.E[:] = 0
    inp.B[:] = 0
    sps = O.species_from(inp)
    s = sps[0]
    O.bin(wl, s)
    o = np.argsort(s.id)
    x0, u0 = s.x[:, o].copy(), s.u[:, o].copy()
    k = 12
    for _ in range(k):
        O.step(wl, sps, inp.E, inp.B)
    o = np.argsort(s.id)
    x, u = s.x[:, o], s.u[:, o]
    gam = np.sqrt(1 + (u0 ** 2).sum(axis=0))
    hits = 0
    for a in range(2):
        L = wl.n[a] * wl.d[a]
        y = x0[a] + k * wl.dt * u0[a] / gam
        if a in axes:
            want, flipped = _fold(y, L)
            # particles whose line ends within rounding of a wall are ambiguous
            ok = (np.abs(np.mod(y + L / 2, L) - L / 2) > 1e-9) & (np.abs(np.mod(y, L) - L / 2) < L / 2 - 1e-9)
            assert np.array_equal(u[a, ok], np.where(flipped, -u0[a], u0[a])[ok])
            hits += int(flipped[ok].sum())
        else:
            want = np.mod(y, L)
            ok = np.abs(np.mod(y + L / 2, L) - L / 2) > 1e-9
            assert np.array_equal(u[a], u0[a])
        assert np.max(np.abs(x[a, ok] - want[ok])) <= 1e-13 * L
        assert np.all(x[a] >= 0) and np.all(x[a] < L)
    assert np.array_equal(u[2], u0[2])
    assert hits > 50  # many particles met a wall
    # every particle sits in the patch its offsets say
    cells = np.minimum(np.floor(s.x / np.array(wl.d[:2])[:, None]).astype(np.int64),
                       np.array(wl.n[:2])[:, None] - 1)
    P = cells[0] // wl.patch[0] + (wl.n[0] // wl.patch[0]) * (cells[1] // wl.patch[1])
    assert np.array_equal(np.diff(s.off), np.bincount(P, minlength=wl.n_patches))
    assert np.all(np.diff(P) >= 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_walls_keep_charge_continuity(dim):
    """A mirrored particle deposits the current of the move from its start to
    its mirrored position, so the deposit still satisfies the discrete
    continuity equation at every node, and the total current is the sum of
    q w (x1 - x0) / dt over those moves (no wrap on a walled axis).  A deposit
    along the unmirrored path would leave a charge residual at the walls."""
    if dim == 2:
        wl = _walls(I.custom(2, (16, 24), (8, 8), ppc=6, seed=42, sigma=0.5, n_species=2), (0, 1))
    else:
        wl = _walls(I.custom(3, (16, 8, 8), (8, 8, 8), ppc=3, seed=43, sigma=0.5, n_species=2), (0, 2))
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    rho0 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    before = []
    for s in sps:
        o = np.argsort(s.id)
        before.append((s.x[:, o].copy(), s.u[:, o].copy()))
    J = O.step(wl, sps, inp.E, inp.B)
    rho1 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    res = (rho1 - rho0) / wl.dt + _div(wl, J)
    assert np.max(np.abs(res)) <= 1e-13 * np.abs(rho0).max() / wl.dt
    flips = 0
    for a in range(dim):
        L = wl.n[a] * wl.d[a]
        tot = 0.0
        for s, (xb, ub) in zip(sps, before):
            o = np.argsort(s.id)
            dx = s.x[a, o] - xb[a]
            if not wl.particle_bc[a]:
                dx = (dx + L / 2) % L - L / 2
            else:
                flips += int((np.sign(s.u[a, o]) != np.sign(ub[a])).sum())
            tot += (s.q * s.w[o] * dx).sum() / wl.dt
        assert abs(J[a].sum() - tot) <= 1e-12 * max(1.0, abs(tot))
    assert flips > 0


def test_walls_bin_rejects_positions_outside_the_box():
    """On a walled axis a position outside [0, L) is an error, not wrapped;
    the periodic axis still wraps."""
    wl = _walls(I.custom(2, (16, 16), (8, 8), ppc=1, seed=44), (0,))
    inp = I.generate(wl)
    sp = O.species_from(inp)[0]
    L = wl.n[1] * wl.d[1]
    sp.x[1, 0] = -0.25 * L
    O.bin(wl, sp)
    assert np.all(sp.x[1] >= 0)
    for bad in (-1e-3, wl.n[0] * wl.d[0]):
        sp2 = O.species_from(inp)[0]
        sp2.x[0, 3] = bad
        with pytest.raises(O.OracleError):
            O.bin(wl, sp2)


def _bcs(wl, bc):
    import dataclasses
    return dataclasses.replace(wl, particle_bc=tuple(bc) + (0,) * (3 - len(bc)))


@pytest.mark.parametrize("bc", [(2, 0), (0, 2), (2, 1)])
def test_remove_free_streaming_keeps_exactly_the_particles_inside(bc):
    """Without fields every particle moves on a straight line, monotone along
    each axis: after k steps the survivors are exactly the particles whose
    line ends inside [0, L) on every removing axis (the others left through a
    wall and were deleted), at their straight-line positions (folded at a
    reflecting wall, wrapped on a periodic axis), and every patch's particles
    stay contiguous in input order."""
    wl = _bcs(I.custom(2, (24, 16), (8, 8), ppc=3, seed=47, sigma=0.8), bc)
    inp = I.generate(wl)
    inp.E[:] = 0
    inp.B[:] = 0
    sps = O.species_from(inp)
    s = sps[0]
    O.bin(wl, s)
    o = np.argsort(s.id)
    ids0, x0, u0 = s.id[o].copy(), s.x[:, o].copy(), s.u[:, o].copy()
    k = 10
    for _ in range(k):
        O.step(wl, sps, inp.E, inp.B)
    gam = np.sqrt(1 + (u0 ** 2).sum(axis=0))
    y = x0 + k * wl.dt * u0[:2] / gam
    L = np.array([wl.n[a] * wl.d[a] for a in range(2)])
    inside = np.ones(ids0.size, bool)
    sure = np.ones(ids0.size, bool)
    for a in range(2):
        if bc[a] == 2:
            inside &= (y[a] >= 0) & (y[a] < L[a])
            sure &= (np.abs(y[a]) > 1e-9) & (np.abs(y[a] - L[a]) > 1e-9)
    got = np.isin(ids0, s.id)
    assert np.array_equal(got[sure], inside[sure])
    assert 100 < int((~inside).sum()) < ids0.size - 100  # many deleted, many kept
    # survivors: straight-line positions, momenta unchanged but for mirrors
    o = np.argsort(s.id)
    keep = np.isin(ids0, s.id)
    for a in range(2):
        want = y[a, keep]
        if bc[a] == 0:
            want = np.mod(want, L[a])
        elif bc[a] == 1:
            want, flip = _fold(want, L[a])
        ok = np.abs(np.mod(want + L[a] / 2, L[a]) - L[a] / 2) > 1e-9
        assert np.max(np.abs(s.x[a, o][ok] - want[ok])) <= 1e-13 * L[a]
    assert np.array_equal(np.abs(s.u[:, o]), np.abs(u0[:, keep]))
    assert s.off[-1] == s.id.size and np.all(np.diff(s.off) >= 0)


@pytest.mark.parametrize("dim", [2, 3])
def test_remove_continuity_holds_for_the_survivors(dim):
    """A particle that leaves through a removing wall deposits nothing in that
    step and is deleted, so the deposit satisfies the discrete continuity
    equation of the survivors: (rho1 - (rho0 - rho_removed)) / dt + div J = 0
    at every node, where rho_removed is the removed particles' density at
    their start positions; the total charge falls by theirs."""
    if dim == 2:
        wl = _bcs(I.custom(2, (16, 24), (8, 8), ppc=6, seed=48, sigma=0.5, n_species=2), (2, 1))
    else:
        wl = _bcs(I.custom(3, (16, 8, 8), (8, 8, 8), ppc=3, seed=49, sigma=0.5, n_species=2),
                  (2, 0, 2))
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    before = [(s.q, s.x.copy(), s.w.copy(), s.id.copy()) for s in sps]
    rho0 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    J = O.step(wl, sps, inp.E, inp.B)
    rho1 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    rho_rm = 0.0
    n_rm = 0
    for (q, x, w, ids), s in zip(before, sps):
        gone = ~np.isin(ids, s.id)
        n_rm += int(gone.sum())
        rho_rm = rho_rm + O.rho(wl, q, x[:, gone], w[gone])
    assert n_rm > 20
    res = (rho1 - (rho0 - rho_rm)) / wl.dt + _div(wl, J)
    assert np.max(np.abs(res)) <= 1e-13 * np.abs(rho0).max() / wl.dt
    # the removed particles' charge did leave: plain continuity fails
    assert np.max(np.abs((rho1 - rho0) / wl.dt + _div(wl, J))) > 1e-3 * np.abs(rho0).max() / wl.dt
    q_rm = sum(q * w[~np.isin(ids, s.id)].sum() for (q, x, w, ids), s in zip(before, sps))
    assert abs((rho0 - rho1).sum() - q_rm) <= 1e-12 * np.abs(rho0).sum()


def test_remove_bin_deletes_positions_outside_the_box():
    """orc_bin deletes a particle outside a removing axis (and still wraps
    the periodic one); the rest keep their stable order."""
    wl = _bcs(I.custom(2, (16, 16), (8, 8), ppc=2, seed=50), (2, 0))
    inp = I.generate(wl)
    sp = O.species_from(inp)[0]
    Lx, Ly = wl.n[0] * wl.d[0], wl.n[1] * wl.d[1]
    sp.x[0, 3] = -1e-12
    sp.x[0, 7] = Lx
    sp.x[1, 9] = -0.5 * Ly
    gone = sp.id[[3, 7]].copy()
    n0 = sp.n
    O.bin(wl, sp)
    assert sp.n == n0 - 2 and sp.off[-1] == n0 - 2
    assert not np.isin(gone, sp.id).any()
    assert np.all(sp.x[1] >= 0)
    for P in range(wl.n_patches):
        assert np.all(np.diff(sp.id[sp.off[P]:sp.off[P + 1]]) > 0)


# --------------------------------------------------------------------------
# derivatives

def _small_adjoint_case(seed=17, steps=4):
    wl = I.custom(2, (16, 16), (8, 8), ppc=3, seed=seed, sigma=0.05, bz0=1.0, steps=steps)
    inp = I.generate(wl, with_W=True)
    sp = O.species_from(inp)[0]
    O.bin(wl, sp)
    return wl, inp, sp


def test_jvp_matches_extended_precision_fd():
    wl, inp, sp = _small_adjoint_case()
    rng = np.random.default_rng(18)
    shp = inp.E.shape
    for kind in ("u", "E", "B", "all"):
        du = rng.normal(size=sp.u.shape) if kind in ("u", "all") else None
        dE = rng.normal(size=shp) * 0.01 if kind in ("E", "all") else None
        dB = rng.normal(size=shp) * 0.01 if kind in ("B", "all") else None
        J, dJ = O.jvp(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, du, dE, dB)
        g = math.fsum((inp.W * dJ).ravel())
        fd, L0 = O.fd(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, inp.W, du, dE, dB, h=1e-6)
        assert abs(L0 - math.fsum((inp.W * J).ravel())) <= 1e-13 * max(1, abs(L0))
        assert abs(g - fd) <= 1e-7 * abs(fd), (kind, g, fd)


def test_jvp_with_walls_matches_extended_precision_fd():
    """Through reflecting walls (fast particles, so many mirror images in
    four steps) the tangent still equals the central difference."""
    wl = _walls(I.custom(2, (16, 16), (8, 8), ppc=3, seed=45, sigma=0.6, bz0=1.0, steps=4),
                (0, 1))
    inp = I.generate(wl, with_W=True)
    sp = O.species_from(inp)[0]
    O.bin(wl, sp)
    rng = np.random.default_rng(46)
    du = rng.normal(size=sp.u.shape)
    dE = rng.normal(size=inp.E.shape) * 0.01
    J, dJ = O.jvp(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, du, dE, None)
    g = math.fsum((inp.W * dJ).ravel())
    fd, L0 = O.fd(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, inp.W, du, dE, None, h=1e-6)
    assert abs(L0 - math.fsum((inp.W * J).ravel())) <= 1e-13 * max(1, abs(L0))
    assert abs(g - fd) <= 1e-7 * abs(fd), (g, fd)
    # the walls matter: the periodic run's J differs
    Jp, _ = O.jvp(dataclasses_replace(wl, particle_bc=(0, 0, 0)), sp.q, sp.m, sp.x, sp.u, sp.w,
                  inp.E, inp.B, du, dE, None)
    assert np.abs(Jp - J).max() > 1e-6 * np.abs(J).max()


def test_jvp_with_removing_walls_matches_extended_precision_fd():
    """Particles deleted at a removing wall stop contributing; the tangent of
    the survivors' current still equals the central difference."""
    wl = _bcs(I.custom(2, (16, 16), (8, 8), ppc=3, seed=51, sigma=0.6, bz0=1.0, steps=4), (2, 1))
    inp = I.generate(wl, with_W=True)
    sp = O.species_from(inp)[0]
    O.bin(wl, sp)
    rng = np.random.default_rng(52)
    du = rng.normal(size=sp.u.shape)
    dB = rng.normal(size=inp.B.shape) * 0.01
    J, dJ = O.jvp(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, du, None, dB)
    g = math.fsum((inp.W * dJ).ravel())
    fd, L0 = O.fd(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, inp.W, du, None, dB, h=1e-6)
    assert abs(L0 - math.fsum((inp.W * J).ravel())) <= 1e-13 * max(1, abs(L0))
    assert abs(g - fd) <= 1e-7 * abs(fd), (g, fd)
    # J equals the step oracle's after the same steps
    c = O.OSpecies(sp.q, sp.m, sp.x, sp.u, sp.w, sp.id, wl.n_patches)
    c.off[:] = sp.off
    Js = None
    for _ in range(wl.steps):
        Js = O.step(wl, [c], inp.E, inp.B)
    assert c.n < sp.n
    assert np.max(np.abs(J - Js)) <= 1e-14 * np.abs(Js).max()


def test_jvp_is_linear_in_direction():
    wl, inp, sp = _small_adjoint_case(seed=19, steps=3)
    rng = np.random.default_rng(20)
    du1, du2 = rng.normal(size=sp.u.shape), rng.normal(size=sp.u.shape)
    dE1 = rng.normal(size=inp.E.shape)
    _, a = O.jvp(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, du1, dE1, None)
    _, b = O.jvp(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, du2, None, None)
    _, c = O.jvp(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B, du1 + 2 * du2, dE1, None)
    assert np.max(np.abs(c - (a + 2 * b))) <= 1e-12 * np.abs(c).max()


def test_jvp_J_equals_step_J():
    """The per-particle derivative code's J_final equals the step oracle's."""
    wl, inp, sp = _small_adjoint_case(seed=21, steps=3)
    J, _ = O.jvp(wl, sp.q, sp.m, sp.x, sp.u, sp.w, inp.E, inp.B)
    c = O.OSpecies(sp.q, sp.m, sp.x, sp.u, sp.w, sp.id, wl.n_patches)
    c.off[:] = sp.off
    Js = None
    for _ in range(wl.steps):
        Js = O.step(wl, [c], inp.E, inp.B)
    assert np.max(np.abs(J - Js)) <= 1e-14 * np.abs(Js).max()


def test_extended_build_is_extended():
    assert O.real_size(False) == 8
    assert O.real_size(True) >= 10


def test_step_rejects_unsorted_offsets():
    wl = I.custom(2, (16, 16), (8, 8), ppc=2, seed=22)
    inp = I.generate(wl)
    sp = O.species_from(inp)[0]  # offsets never computed
    with pytest.raises(O.OracleError):
        O.step(wl, [sp], inp.E, inp.B)


@pytest.mark.parametrize("dim", [2, 3])
def test_window_of_particles_reproduces_the_full_run(dim):
    """Finite propagation: the particles within the margin of a window of
    patches give the full run's counts, particles and J inside it (the
    reduction the full-size GPU parity tests rely on).  Fast particles
    (sigma 0.4) and a window across the periodic corner."""
    import _window as Wn

    if dim == 2:
        wl = I.custom(2, (64, 48), (8, 8), ppc=3, seed=150, sigma=0.4)
        a0, npw, steps = [-8, -8, 0], [3, 2, 1], 6
    else:
        wl = I.custom(3, (24, 24, 24), (4, 4, 4), ppc=1, seed=151, sigma=0.4, n_species=2)
        a0, npw, steps = [-4, 4, -4], [2, 2, 2], 3
    inp = I.generate(wl)
    full = O.species_from(inp)
    for s in full:
        O.bin(wl, s)
    for _ in range(steps):
        J, A = O.step(wl, full, inp.E, inp.B, with_abs=True)
    margin = Wn.margin_cells(wl, steps)
    sub, Js, _ = Wn.oracle_window(wl, inp, steps, a0, npw, margin)
    assert sum(s.n for s in sub) < sum(s.n for s in full)
    patches = Wn.window_patches(wl, a0, npw)
    for f, s in zip(full, sub):
        assert np.array_equal(np.diff(f.off)[patches], np.diff(s.off)[patches])
        for P in patches:
            fi, si = np.arange(f.off[P], f.off[P + 1]), np.arange(s.off[P], s.off[P + 1])
            assert np.array_equal(f.id[fi], s.id[si])  # stable sort keeps the order
            assert np.array_equal(f.x[:, fi], s.x[:, si])
            assert np.array_equal(f.u[:, fi], s.u[:, si])
    nodes = Wn.window_nodes(wl, a0, npw)
    for c in range(3):
        assert np.all(np.abs(J[c][nodes] - Js[c][nodes]) <= 1e-12 * A[c][nodes])
    # the margin is needed: without it the window's particle sets differ
    sub0, _, _ = Wn.oracle_window(wl, inp, steps, a0, npw, 0)
    ids = lambda sps: [np.sort(np.concatenate([s.id[s.off[P]:s.off[P + 1]] for P in patches]))
                       for s in sps]
    assert any(not np.array_equal(a, b) for a, b in zip(ids(sub0), ids(full)))


# --------------------------------------------------------------------------
# field solver (Yee): pins from the Fourier symbol of the staggered
# differences, the vector identities div curl = 0, the continuity of the
# deposit, and energy conservation of the leapfrog

E_STAG = ((1, 0, 0), (0, 1, 0), (0, 0, 1))
B_STAG = ((0, 1, 1), (1, 0, 1), (1, 1, 0))


def _phase(g, st, k):
    """k . x at every entry of a component with stagger bits st."""
    nz, ny, nx = field_shape(g)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ph = k[0] * (x + st[0] / 2) * g.d[0] + k[1] * (y + st[1] / 2) * g.d[1]
    if g.dim == 3:
        ph = ph + k[2] * (z + st[2] / 2) * g.d[2]
    return ph


def _mode(g, amp, stag, k, t_phase):
    return np.stack([np.real(amp[c] * np.exp(1j * (_phase(g, stag[c], k) - t_phase)))
                     for c in range(3)])


@pytest.mark.parametrize("dim", [2, 3])
def test_maxwell_plane_wave_follows_the_yee_dispersion(dim):
    """A Fourier mode of the staggered grid evolves exactly as the Yee
    scheme's symbol says: the differences act as i kappa with
    kappa_a = 2 sin(k_a d_a / 2) / d_a, and the leapfrog turns |kappa| into
    the frequency omega with sin(omega dt / 2) = dt |kappa| / 2.  Two
    polarisations, unequal cell sizes, 40 steps."""
    n = (24, 20, 16)[:dim]
    d = (0.1, 0.13, 0.08)
    dt = 0.9 * I.cfl_dt(d, dim)
    g = _G(dim, n, d=d, dt=dt)
    m = (3, -2, 1)
    k = np.array([2 * np.pi * m[a] / (g.n[a] * d[a]) if a < dim else 0.0 for a in range(3)])
    kap = np.array([2 * np.sin(k[a] * d[a] / 2) / d[a] if a < dim else 0.0 for a in range(3)])
    om_t = np.linalg.norm(kap)
    omega = 2 / dt * np.arcsin(dt * om_t / 2)
    a1 = np.cross(kap, [0.3, -0.2, 1.0])
    a1 /= np.linalg.norm(a1)
    a2 = np.cross(kap, a1) / om_t
    N = 40
    for A in (a1, a2):
        A = A * np.exp(0.7j)
        Bh = np.cross(kap, A) / om_t
        E0 = _mode(g, A, E_STAG, k, 0.0)
        B0 = _mode(g, Bh, B_STAG, k, omega * dt / 2)
        E1, B1 = O.maxwell(g, E0, B0, np.zeros_like(E0), N)
        Ee = _mode(g, A, E_STAG, k, omega * N * dt)
        Be = _mode(g, Bh, B_STAG, k, omega * (N + 0.5) * dt)
        assert np.abs(E1 - Ee).max() <= 1e-11, np.abs(E1 - Ee).max()
        assert np.abs(B1 - Be).max() <= 1e-11, np.abs(B1 - Be).max()
        assert np.abs(E1 - E0).max() > 0.1  # the wave moved


def _divB(g, B):
    out = np.zeros(B.shape[1:])
    for a in range(g.dim):
        ax = 2 - a
        out += (np.roll(B[a], -1, axis=ax) - B[a]) / g.d[a]
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_maxwell_keeps_div_b(dim):
    """div B at cell centres is unchanged by any number of steps (the
    discrete divergence of a discrete curl vanishes), whatever E, B and J."""
    g = _G(dim, (10, 12, 8)[:dim], d=(0.1, 0.12, 0.09))
    rng = np.random.default_rng(31)
    shp = (3,) + field_shape(g)
    E, B, J = rng.standard_normal(shp), rng.standard_normal(shp), rng.standard_normal(shp)
    E1, B1 = O.maxwell(g, E, B, J, 5)
    assert np.abs(B1 - B).max() > 0.1
    assert np.abs(_divB(g, B1) - _divB(g, B)).max() <= 1e-12 / min(g.d[:dim])


@pytest.mark.parametrize("dim", [2, 3])
def test_maxwell_keeps_gauss_law_with_the_deposited_current(dim):
    """With the current of a particle step, div E changes by exactly the
    change of the charge density: Gauss's law is preserved (Yee's Ampere
    update plus the deposit's discrete continuity)."""
    if dim == 2:
        wl = I.workload("uniform64")
    else:
        wl = I.custom(3, (16, 16, 16), (8, 8, 8), ppc=2, seed=15, n_species=2, sigma=0.05)
    inp = I.generate(wl)
    sps = O.species_from(inp)
    for s in sps:
        O.bin(wl, s)
    rho0 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    J = O.step(wl, sps, inp.E, inp.B)
    rho1 = sum(O.rho(wl, s.q, s.x, s.w) for s in sps)
    E1, _ = O.maxwell(wl, inp.E, inp.B, J, 1)
    res = _div(wl, E1) - _div(wl, inp.E) - (rho1 - rho0)
    scale = max(np.abs(rho0).max(), np.abs(inp.E).max() / min(wl.d[:dim]))
    assert np.abs(res).max() <= 1e-12 * scale
    assert np.abs(rho1 - rho0).max() > 1e-6 * np.abs(rho0).max()  # charges moved


def test_maxwell_conserves_the_leapfrog_energy():
    """Without current, sum |E^n|^2 + B^(n-1/2) . B^(n+1/2) is conserved by the
    Yee leapfrog (to rounding) while the fields change."""
    g = _G(2, (16, 14), d=(0.1, 0.11, 1.0))
    rng = np.random.default_rng(32)
    shp = (3,) + field_shape(g)
    E, B = rng.standard_normal(shp), rng.standard_normal(shp)
    E_init = E.copy()
    Z = np.zeros(shp)
    W = []
    for _ in range(50):
        E1, B1 = O.maxwell(g, E, B, Z, 1)
        W.append((E1 * E1).sum() + (B * B1).sum())
        E, B = E1, B1
    W = np.array(W)
    assert np.abs(W - W[0]).max() <= 1e-12 * W[0]
    assert np.abs(E - E_init).max() > 0.1


@pytest.mark.parametrize("dim", [2, 3])
def test_maxwell_uniform_fields_and_current(dim):
    """Uniform fields have no curl: B stays, E changes by -dt J exactly."""
    g = _G(dim, (8, 6, 4)[:dim])
    shp = (3,) + field_shape(g)
    E = np.ones(shp) * np.array([0.3, -0.7, 1.1])[:, None, None, None]
    B = np.ones(shp) * np.array([-0.2, 0.5, 0.9])[:, None, None, None]
    J = np.ones(shp) * np.array([0.01, 0.02, -0.03])[:, None, None, None]
    E1, B1 = O.maxwell(g, E, B, J, 1)
    assert np.array_equal(B1, B)
    assert np.array_equal(E1, E - g.dt * J)


@pytest.mark.parametrize("dim", [2, 3])
def test_maxwell_adjoint_is_the_transpose(dim):
    """<F(E, B, J), (Eb, Bb)> = <(E, B, J), F^T(Eb, Bb)> for the oracle's
    field steps F and its reverse mode F^T, with random vectors (unequal
    cell sizes, 4 steps): any wrong sign, index or coefficient in the
    transpose breaks the identity."""
    g = _G(dim, (10, 9, 8)[:dim], d=(0.1, 0.12, 0.09))
    rng = np.random.default_rng(33 + dim)
    shp = (3,) + field_shape(g)
    E, B, J = (rng.standard_normal(shp) for _ in range(3))
    Eb, Bb = rng.standard_normal(shp), rng.standard_normal(shp)
    E1, B1 = O.maxwell(g, E, B, J, 4)
    Ea, Ba, Ja = O.maxwell_adjoint(g, Eb, Bb, 4)
    lhs = (E1 * Eb).sum() + (B1 * Bb).sum()
    rhs = (E * Ea).sum() + (B * Ba).sum() + (J * Ja).sum()
    scale = np.abs(E1 * Eb).sum() + np.abs(B1 * Bb).sum()
    assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs)
    # Jb accumulates
    _, _, Jb2 = O.maxwell_adjoint(g, Eb, Bb, 4, Jb=Ja)
    assert np.allclose(Jb2, 2 * Ja, rtol=1e-13, atol=1e-13)


def test_oracle_matches_its_stored_digest():
    """Regression guard: the oracle's state after 10 steps of uniform64, and
    of a fast plasma between removing and reflecting walls, equals the digest
    written by tests/golden/make_golden.py (the paper prints no
    worked example with values for these operators, so the golden file is
    the oracle's own, pinned output; a change to the oracle's arithmetic has
    to rewrite it on purpose)."""
    import json
    import os
    import sys

    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    try:
        import make_golden
    finally:
        sys.path.remove(here)
    with open(os.path.join(here, "oracle_uniform64_digest.json")) as fh:
        stored = json.load(fh)
    assert make_golden.digest() == stored
    with open(os.path.join(here, "oracle_walls_digest.json")) as fh:
        stored = json.load(fh)
    got = make_golden.digest(walls=True)
    assert got == stored
    assert got["particles"] < 32 * 24 * 6  # particles were deleted


def test_adjoint256_fd_golden_is_the_oracles():
    """tests/golden/adjoint256_fd.json (the expected values of the adjoint's
    finite-difference check at full size) belongs to the current inputs and
    oracle: the input digest matches; a few sampled scalars recomputed now
    give the stored numbers exactly; and every stored binary128 central
    difference agrees with the stored forward-mode derivative (two
    independent computations) to 1e-10 (directions) and 1e-8 (sampled
    scalars, where not negligible)."""
    import json
    import os
    import sys

    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, os.path.join(here, "golden"))
    import make_adjoint256_fd as G

    with open(os.path.join(here, "golden", "adjoint256_fd.json")) as fh:
        gold = json.load(fh)
    wl, inp, x = G.setup()
    assert G.inputs_sha(inp, x) == gold["inputs_sha256"]
    assert gold["h"] == G.H and len(gold["directions"]) == 8 and len(gold["scalars"]) == 96
    assert [(k, c, i) for k, c, i in G.samples(wl, x.shape[1])] == \
        [(e["kind"], e["component"], e["index"]) for e in gold["scalars"]]
    G._STATE.update(wl=wl, inp=inp, x=x)
    for e in (gold["scalars"][0], gold["scalars"][1], gold["scalars"][32], gold["scalars"][64]):
        again = G.scalar_task((e["kind"], e["component"], e["index"]))
        assert again["fd"] == e["fd"] and again["jvp"] == e["jvp"], (e, again)
    # binary128 differences against the double forward mode: the difference
    # quotient's error O(h^2) and the forward mode's rounding stay far below
    # the 1e-7 the adjoint is held to
    for d in gold["directions"]:
        assert abs(d["fd"] - d["jvp"]) <= 1e-10 * abs(d["fd"]), d
    for kind in ("u", "E", "B"):
        sc = [e for e in gold["scalars"] if e["kind"] == kind]
        top = max(abs(e["fd"]) for e in sc)
        for e in sc:
            if abs(e["fd"]) > 1e-3 * top:
                assert abs(e["fd"] - e["jvp"]) <= 1e-8 * abs(e["fd"]), e
