"""Pins of two parts of the FP64 oracle that the other pins leave open (no GPU):

* the Roe-average arm of the local Lax-Friedrichs wave speed (Section 2.1,
  numerical flux: lambda is the largest |u_n| + a over the two face states and
  their Roe average, the average defined in Toro's book, which the paper cites);
* the mirror ghost rows next to the slip walls and on both sides of the lid
  (Appendix B; the cell gradients of the rows next to a horizontal boundary).

The Roe pin rests on Roe's defining property: for the sqrt(rho)-weighted
velocity and total enthalpy, the flux Jacobian A evaluated there maps the state
jump onto the flux jump exactly, f_n(qR) - f_n(qL) = A (qR - qL), and its
spectral radius is |u_n| + a of that average.  Neither a rho-weighted nor an
arithmetic mean has the property, so the test's average is the Roe average by
mathematics, not by restating the oracle's code; the wave speed read back from
the oracle's flux must then equal the largest of the one-sided speeds and that
spectral radius.

The mirror pin rests on geometry: a domain of 2 nz rows whose lower half is the
mirror image (rho, rho u, -rho w, rho E) of its upper half has, on its upper
half, exactly the cell gradients and face states that the one-row mirror ghost
gives the single domain at its wall.  So the two RHS agree on every row, except
where the reading of the boundary flux itself differs from an interior face:
the normal viscous stress, which the doubled domain keeps and the slip wall
sets to zero, and the lid's viscous flux, which the single domain adds.  Both
differences are checked in closed form.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2202_11890_amd import inputs

G = 1.4


# --------------------------------------------------------------------------
# Roe average (Section 2.1, numerical flux)
# --------------------------------------------------------------------------
def _primitives(q):
    rho = q[0]
    vel = q[1:-1] / rho
    p = (G - 1) * (q[-1] - 0.5 * rho * vel @ vel)
    return rho, vel, p


def _phys_flux(q, d):
    rho, vel, p = _primitives(q)
    un = vel[d]
    f = np.empty_like(q)
    f[0] = rho * un
    f[1:-1] = q[1:-1] * un
    f[1 + d] += p
    f[-1] = (q[-1] + p) * un
    return f


def _jacobian(vel, H, d):
    """Flux Jacobian of the Euler equations in direction d, written in the
    velocity and the total enthalpy (conserved variables rho, rho u.., rho E)."""
    nd = len(vel)
    n = np.zeros(nd)
    n[d] = 1.0
    un = vel[d]
    k = 0.5 * (G - 1) * vel @ vel
    A = np.zeros((nd + 2, nd + 2))
    A[0, 1:-1] = n
    A[1:-1, 0] = k * n - vel * un
    A[1:-1, 1:-1] = np.outer(vel, n) - (G - 1) * np.outer(n, vel) + un * np.eye(nd)
    A[1:-1, -1] = (G - 1) * n
    A[-1, 0] = un * (k - H)
    A[-1, 1:-1] = H * n - (G - 1) * un * vel
    A[-1, -1] = G * un
    return A


def _weighted(qL, qR, wL, wR):
    rL, vL, pL = _primitives(qL)
    rR, vR, pR = _primitives(qR)
    HL, HR = (qL[-1] + pL) / rL, (qR[-1] + pR) / rR
    return (wL * vL + wR * vR) / (wL + wR), (wL * HL + wR * HR) / (wL + wR)


def _pair(rng, nd, d, shear):
    """Two physical states, densities over a factor 40, velocities up to a few
    sound speeds; with `shear`, a cold pair whose normal velocity (direction
    d) is small, so the tangential jump dominates the wave speeds."""
    out = []
    for _ in range(2):
        rho = np.exp(rng.uniform(np.log(0.05), np.log(2.0)))
        vel = rng.uniform(-3.0, 3.0, nd)
        p = rng.uniform(0.2, 2.0)
        if shear:
            rho = np.exp(rng.uniform(np.log(0.3), np.log(3.0)))
            vel[d] *= 0.1
            p = rng.uniform(0.1, 0.4)
        out.append(np.concatenate([[rho], rho * vel, [p / (G - 1) + 0.5 * rho * vel @ vel]]))
    return out


def _llf(qL, qR, d):
    return oracle.llf(qL, qR, d) if len(qL) == 4 else oracle.llf3(qL, qR, d)


@pytest.mark.parametrize("nd", [2, 3])
def test_roe_average_speed_of_the_llf_flux(nd):
    rng = np.random.default_rng(2202 + nd)
    roe_binds = 0
    trials = 400
    for t in range(trials):
        d = t % nd
        qL, qR = _pair(rng, nd, d, shear=(t // nd) % 2 == 1)
        dq = qR - qL
        # The dissipation coefficient read back from the oracle's flux.
        fL, fR = _phys_flux(qL, d), _phys_flux(qR, d)
        F = _llf(qL, qR, d)
        lam = -2.0 * (F[0] - 0.5 * (fL[0] + fR[0])) / dq[0]

        # Roe's property fixes the average: only sqrt(rho) weights satisfy it.
        vel, H = _weighted(qL, qR, np.sqrt(qL[0]), np.sqrt(qR[0]))
        A = _jacobian(vel, H, d)
        scale = np.abs(fR - fL).max() + np.abs(fL).max()
        assert np.abs((fR - fL) - A @ dq).max() <= 1e-13 * scale
        for wts in ((qL[0], qR[0]), (1.0, 1.0)):
            v2, H2 = _weighted(qL, qR, *wts)
            assert np.abs((fR - fL) - _jacobian(v2, H2, d) @ dq).max() > 1e-6 * scale

        # Spectral radius of the Roe matrix = |u_n| + a of the average.
        radius = np.abs(np.linalg.eigvals(A)).max()
        one_sided = []
        for q in (qL, qR):
            rho, v, p = _primitives(q)
            one_sided.append(abs(v[d]) + np.sqrt(G * p / rho))
        expect = max(max(one_sided), radius)
        assert lam == pytest.approx(expect, rel=1e-12), (t, lam, expect)

        if radius > max(one_sided) * (1 + 1e-6):
            roe_binds += 1
            # The test has power here: another average would give another lambda.
            for wts in ((qL[0], qR[0]), (1.0, 1.0)):
                v2, H2 = _weighted(qL, qR, *wts)
                r2 = np.abs(np.linalg.eigvals(_jacobian(v2, H2, d))).max()
                if abs(r2 - radius) > 1e-9 * radius:
                    assert lam != pytest.approx(max(max(one_sided), r2), rel=1e-12)
    # Shear makes the Roe arm the largest in a good share of the pairs.
    assert roe_binds >= trials // 5, roe_binds


# --------------------------------------------------------------------------
# Mirror-doubled domains (Appendix B; ghost rows at walls and at the lid)
# --------------------------------------------------------------------------
def _mirror2(q):
    """[4, nz, nx] -> rows in reverse order with rho w negated."""
    return q[:, ::-1, :] * np.array([1.0, 1.0, -1.0, 1.0])[:, None, None]


def _problem2(w, nzl, nzu, mu=(2e-3, 7e-4)):
    return oracle.Problem(w.nx, nzl, nzu, w.dx, w.dz_lower, w.dz_upper, n_buffer=2,
                          mu_lower=mu[0], mu_upper=mu[1])


def _dx_c(f, dx):
    """Central x-difference of a periodic row."""
    return (np.roll(f, -1, axis=-1) - np.roll(f, 1, axis=-1)) / (2 * dx)


def _szz2(q_row, above_w, below_w, dz, dx, mu):
    """Normal viscous stress of an interior z-face whose two cells have the
    same u (mirror pair): mu (4/3 dw/dz - 2/3 du/dx)."""
    u = q_row[1] / q_row[0]
    return mu * (4.0 / 3.0 * (above_w - below_w) / dz - 2.0 / 3.0 * _dx_c(u, dx))


def _case2(seed):
    w = inputs.small().with_(nx=14, nz_lower=6, nz_upper=5, lz_lower=1.5, lz_upper=2.5)
    ql, qu = inputs.random_state(w, seed, amp=0.2)
    return w, ql, qu


def _scale(r):
    return np.abs(r).max(axis=(1, 2))[:, None, None] + 1e-300


@pytest.mark.parametrize("seed", [1, 2])
def test_wall_rows_equal_a_mirror_doubled_domain_2d(seed):
    w, ql, qu = _case2(seed)
    nzl, nzu = ql.shape[1], qu.shape[1]
    mu = (2e-3, 7e-4)
    rl, ru = oracle.rhs(_problem2(w, nzl, nzu, mu), ql, qu)

    # Bottom wall of the lower domain: mirror image below it.
    ql2 = np.ascontiguousarray(np.concatenate([_mirror2(ql), ql], axis=1))
    rl2, ru2 = oracle.rhs(_problem2(w, 2 * nzl, nzu, mu), ql2, qu)
    assert np.array_equal(ru2, ru)
    got = rl2[:, nzl:].copy()
    wv = ql[2, 0] / ql[0, 0]
    # Slip wall: sigma_zz = 0; the doubled domain's face carries it.
    got[2, 0] += _szz2(ql[:, 0], wv, -wv, w.dz_lower, w.dx, mu[0]) / w.dz_lower
    assert np.abs(got - rl).max() <= 1e-13 * _scale(rl).max()
    assert np.all(np.abs(got - rl) <= 1e-13 * _scale(rl))

    # Top wall of the upper domain: mirror image above it.
    qu2 = np.ascontiguousarray(np.concatenate([qu, _mirror2(qu)], axis=1))
    rl3, ru3 = oracle.rhs(_problem2(w, nzl, 2 * nzu, mu), ql, qu2)
    assert np.array_equal(rl3, rl)
    got = ru3[:, :nzu].copy()
    wv = qu[2, -1] / qu[0, -1]
    got[2, -1] -= _szz2(qu[:, -1], -wv, wv, w.dz_upper, w.dx, mu[1]) / w.dz_upper
    assert np.all(np.abs(got - ru) <= 1e-13 * _scale(ru))


@pytest.mark.parametrize("seed", [3, 4])
def test_lid_rows_equal_a_mirror_doubled_domain_2d(seed):
    """On each side of the lid the ghost row is the mirror of the row next to
    it; the lid adds its viscous flux (0, sigma_xz, 0, u_w sigma_xz - Pi_z) in
    +z, leaving the lower domain and entering the upper one."""
    w, ql, qu = _case2(seed)
    nzl, nzu = ql.shape[1], qu.shape[1]
    mu = (2e-3, 7e-4)
    pb = _problem2(w, nzl, nzu, mu)
    rl, ru = oracle.rhs(pb, ql, qu)
    ifc = oracle.interface(pb, ql, qu)
    fvg = np.stack([np.zeros(w.nx), ifc[:, 0], np.zeros(w.nx), ifc[:, 2] * ifc[:, 0] - ifc[:, 1]])

    # Upper domain: its mirror image below it, the lid below the image.
    qu2 = np.ascontiguousarray(np.concatenate([_mirror2(qu), qu], axis=1))
    _, ru2 = oracle.rhs(_problem2(w, nzl, 2 * nzu, mu), ql, qu2)
    got = ru2[:, nzu:].copy()
    wv = qu[2, 0] / qu[0, 0]
    got[2, 0] += _szz2(qu[:, 0], wv, -wv, w.dz_upper, w.dx, mu[1]) / w.dz_upper
    got[:, 0] -= fvg / w.dz_upper
    assert np.all(np.abs(got - ru) <= 1e-13 * _scale(ru))

    # Lower domain: its mirror image above it, the lid above the image.
    ql2 = np.ascontiguousarray(np.concatenate([ql, _mirror2(ql)], axis=1))
    rl2, _ = oracle.rhs(_problem2(w, 2 * nzl, nzu, mu), ql2, qu)
    got = rl2[:, :nzl].copy()
    wv = ql[2, -1] / ql[0, -1]
    got[2, -1] -= _szz2(ql[:, -1], -wv, wv, w.dz_lower, w.dx, mu[0]) / w.dz_lower
    got[:, -1] += fvg / w.dz_lower
    assert np.all(np.abs(got - rl) <= 1e-13 * _scale(rl))


def test_mirror_pin_detects_a_copied_ghost_row():
    """Negative control of the doubled-domain argument: a doubled domain whose
    lower half copies the upper half without negating rho w (what a copy
    ghost would give) differs from the single domain on the wall rows by far
    more than the tolerance."""
    w, ql, qu = _case2(5)
    nzl, nzu = ql.shape[1], qu.shape[1]
    rl, _ = oracle.rhs(_problem2(w, nzl, nzu), ql, qu)
    ql2 = np.ascontiguousarray(np.concatenate([ql[:, ::-1], ql], axis=1))
    rl2, _ = oracle.rhs(_problem2(w, 2 * nzl, nzu), ql2, qu)
    diff = np.abs(rl2[:, nzl:] - rl)
    assert diff[[0, 1, 3], :2].max() > 1e-6 * _scale(rl).max()


# ---- 3D ----------------------------------------------------------------------
def _mirror3(q):
    return q[:, ::-1] * np.array([1.0, 1.0, 1.0, -1.0, 1.0])[:, None, None, None]


def _problem3(w, nzl, nzu, mu=(2e-3, 7e-4)):
    return oracle.Problem3(w.nx, w.ny, nzl, nzu, w.dx, w.dy, w.dz_lower, w.dz_upper,
                           n_buffer=2, mu_lower=mu[0], mu_upper=mu[1])


def _szz3(q_plane, above_w, below_w, dz, dx, dy, mu):
    u = q_plane[1] / q_plane[0]
    v = q_plane[2] / q_plane[0]
    dudx = _dx_c(u, dx)
    dvdy = (np.roll(v, -1, axis=0) - np.roll(v, 1, axis=0)) / (2 * dy)
    return mu * (4.0 / 3.0 * (above_w - below_w) / dz - 2.0 / 3.0 * (dudx + dvdy))


def _case3(seed):
    w = inputs.small3d().with_(nx=9, ny=7, nz_lower=5, nz_upper=4)
    ql, qu = inputs.random_state3(w, seed, amp=0.2)
    return w, ql, qu


def _scale3(r):
    return np.abs(r).max(axis=(1, 2, 3))[:, None, None, None] + 1e-300


def test_wall_and_lid_planes_equal_mirror_doubled_domains_3d():
    w, ql, qu = _case3(6)
    nzl, nzu = ql.shape[1], qu.shape[1]
    mu = (2e-3, 7e-4)
    pb = _problem3(w, nzl, nzu, mu)
    rl, ru = oracle.rhs3(pb, ql, qu)
    ifc = oracle.interface3(pb, ql, qu)  # [ny, nx, 8]
    z = np.zeros((w.ny, w.nx))
    fvg = np.stack([z, ifc[..., 0], ifc[..., 1], z,
                    ifc[..., 3] * ifc[..., 0] + ifc[..., 4] * ifc[..., 1] - ifc[..., 2]])

    def wz(q, k):
        return q[3, k] / q[0, k]

    # Bottom wall of the lower domain.
    ql2 = np.ascontiguousarray(np.concatenate([_mirror3(ql), ql], axis=1))
    rl2, ru2 = oracle.rhs3(_problem3(w, 2 * nzl, nzu, mu), ql2, qu)
    assert np.array_equal(ru2, ru)
    got = rl2[:, nzl:].copy()
    got[3, 0] += _szz3(ql[:, 0], wz(ql, 0), -wz(ql, 0), w.dz_lower, w.dx, w.dy, mu[0]) / w.dz_lower
    assert np.all(np.abs(got - rl) <= 1e-13 * _scale3(rl))

    # Top wall of the upper domain.
    qu2 = np.ascontiguousarray(np.concatenate([qu, _mirror3(qu)], axis=1))
    rl3, ru3 = oracle.rhs3(_problem3(w, nzl, 2 * nzu, mu), ql, qu2)
    assert np.array_equal(rl3, rl)
    got = ru3[:, :nzu].copy()
    got[3, -1] -= _szz3(qu[:, -1], -wz(qu, -1), wz(qu, -1), w.dz_upper, w.dx, w.dy, mu[1]) / w.dz_upper
    assert np.all(np.abs(got - ru) <= 1e-13 * _scale3(ru))

    # Lid, upper side.
    qu4 = np.ascontiguousarray(np.concatenate([_mirror3(qu), qu], axis=1))
    _, ru4 = oracle.rhs3(_problem3(w, nzl, 2 * nzu, mu), ql, qu4)
    got = ru4[:, nzu:].copy()
    got[3, 0] += _szz3(qu[:, 0], wz(qu, 0), -wz(qu, 0), w.dz_upper, w.dx, w.dy, mu[1]) / w.dz_upper
    got[:, 0] -= fvg / w.dz_upper
    assert np.all(np.abs(got - ru) <= 1e-13 * _scale3(ru))

    # Lid, lower side.
    ql4 = np.ascontiguousarray(np.concatenate([ql, _mirror3(ql)], axis=1))
    rl4, _ = oracle.rhs3(_problem3(w, 2 * nzl, nzu, mu), ql4, qu)
    got = rl4[:, :nzl].copy()
    got[3, -1] -= _szz3(ql[:, -1], -wz(ql, -1), wz(ql, -1), w.dz_lower, w.dx, w.dy, mu[0]) / w.dz_lower
    got[:, -1] += fvg / w.dz_lower
    assert np.all(np.abs(got - rl) <= 1e-13 * _scale3(rl))
