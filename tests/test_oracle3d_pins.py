"""Pins of the 3D oracle (Appendix B in three dimensions) against what the
paper and mathematics fix, independently of the oracle itself:

* a state that does not depend on y and has v = 0 is the 2D problem, so the
  3D RHS and MPRK step must reproduce the (separately pinned) 2D oracle bit
  for bit, with a zero y-momentum RHS;
* exchanging the x and y axes (and u with v) exchanges the results;
* the spatial discretization converges at second order to the exact PDE
  right-hand side of Section 2 (sympy), which pins every term, including the
  cross-derivative stresses that the 2D reduction leaves out;
* free stream, conservation across the interface, the bulk interface flux of
  a piecewise-linear profile, and LLF consistency.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2202_11890_amd import inputs


def prob3(w, **over):
    kw = dict(fast_is_lower=w.fast_is_lower, n_buffer=w.n_buffer, gamma=w.gamma,
              prandtl=w.prandtl, mu_lower=w.mu_lower, mu_upper=w.mu_upper, gravity=w.gravity)
    kw.update(over)
    return oracle.Problem3(w.nx, w.ny, w.nz_lower, w.nz_upper, w.dx, w.dy, w.dz_lower, w.dz_upper,
                           **kw)


def to3(q2, ny):
    """2D state [4, nz, nx] -> y-invariant 3D state [5, nz, ny, nx] with v = 0."""
    nz, nx = q2.shape[1:]
    q3 = np.zeros((5, nz, ny, nx))
    for c3, c2 in ((0, 0), (1, 1), (3, 2), (4, 3)):
        q3[c3] = q2[c2][:, None, :]
    return q3


def flux_scale(q, hmin, gamma=1.4):
    rho = q[0]
    vel = q[1:4] / rho
    p = (gamma - 1) * (q[4] - 0.5 * rho * (vel ** 2).sum(axis=0))
    a = np.sqrt(gamma * p / rho)
    s = np.abs(vel).sum(axis=0) + a
    return float(((np.abs(q).max(axis=0) + p) * s).max()) / hmin


@pytest.mark.parametrize("gravity", [0.0, -0.05])
def test_y_invariant_state_reduces_to_2d_bitwise(gravity):
    w2 = inputs.small().with_(nx=20, nz_lower=9, nz_upper=11, lz_lower=2.0, mu_lower=3e-3,
                              mu_upper=5e-4, gravity=gravity, t_lower=4.0)
    ql, qu = inputs.random_state(w2, 4, amp=0.1)
    pb2 = oracle.Problem(w2.nx, w2.nz_lower, w2.nz_upper, w2.dx, w2.dz_lower, w2.dz_upper,
                         n_buffer=w2.n_buffer, mu_lower=w2.mu_lower, mu_upper=w2.mu_upper,
                         gravity=gravity)
    ny = 3
    pb3 = oracle.Problem3(w2.nx, ny, w2.nz_lower, w2.nz_upper, w2.dx, 0.7, w2.dz_lower,
                          w2.dz_upper, n_buffer=w2.n_buffer, mu_lower=w2.mu_lower,
                          mu_upper=w2.mu_upper, gravity=gravity)
    rl2, ru2 = oracle.rhs(pb2, ql, qu)
    rl3, ru3 = oracle.rhs3(pb3, to3(ql, ny), to3(qu, ny))
    for r2, r3 in ((rl2, rl3), (ru2, ru3)):
        assert np.array_equal(to3(r2, ny)[[0, 1, 3, 4]], r3[[0, 1, 3, 4]])
        assert np.all(r3[2] == 0.0)
    # and one MPRK step
    a2, b2 = ql.copy(), qu.copy()
    oracle.mprk_step(pb2, 2, 2, 0.01, a2, b2)
    a3, b3 = to3(ql, ny), to3(qu, ny)
    oracle.mprk_run3(pb3, 2, 2, 0.01, 1, a3, b3)
    assert np.array_equal(to3(a2, ny), a3) and np.array_equal(to3(b2, ny), b3)


def test_xy_exchange_symmetry():
    w = inputs.small3d().with_(nx=14, ny=10, nz_lower=6, nz_upper=5, ly=7.0)
    ql, qu = inputs.random_state3(w, 7, amp=0.1)
    pb = prob3(w)
    rl, ru = oracle.rhs3(pb, ql, qu)

    def swap(q):
        t = np.ascontiguousarray(np.swapaxes(q, 2, 3))
        t[[1, 2]] = t[[2, 1]]
        return np.ascontiguousarray(t)

    pbs = oracle.Problem3(w.ny, w.nx, w.nz_lower, w.nz_upper, w.dy, w.dx, w.dz_lower, w.dz_upper,
                          n_buffer=w.n_buffer)
    sl, su = oracle.rhs3(pbs, swap(ql), swap(qu))
    for r, s, q in ((rl, sl, ql), (ru, su, qu)):
        tol = 1e-14 * flux_scale(q, min(w.dx, w.dy, w.dz_lower))
        assert np.abs(swap(r) - s).max() <= tol


def test_free_stream_preserved_3d():
    w = inputs.small3d().with_(nx=10, ny=8, nz_lower=6, nz_upper=7)
    ql, qu = inputs.uniform_state3(w, 1.0, 0.3, -0.2, 0.0, 1 / 1.4)
    a, b = ql.copy(), qu.copy()
    oracle.mprk_run3(prob3(w), 3, 2, 0.01, 3, a, b)
    assert np.array_equal(a, ql) and np.array_equal(b, qu)


def test_conservation_3d():
    w = inputs.small3d().with_(nx=12, ny=10, nz_lower=8, nz_upper=8, n_buffer=5)
    ql, qu = inputs.random_state3(w, 3, amp=0.05)
    pb = prob3(w)
    t0 = oracle.totals3(pb, ql, qu)
    dt = oracle.dt_rule3(pb, ql, qu, w.m)
    oracle.mprk_run3(pb, w.base, w.m, dt, 6, ql, qu)
    t1 = oracle.totals3(pb, ql, qu)
    # mass per domain; x, y momentum and energy in total (z momentum meets the
    # walls and the lid)
    assert abs(t1[0, 0] - t0[0, 0]) <= 1e-13 * t0[0, 0]
    assert abs(t1[1, 0] - t0[1, 0]) <= 1e-13 * t0[1, 0]
    for v in (1, 2):
        assert abs(t1[:, v].sum() - t0[:, v].sum()) <= 1e-13 * t0[:, 0].sum()
    assert abs(t1[:, 4].sum() - t0[:, 4].sum()) <= 1e-13 * t0[:, 4].sum()


def test_interface_flux_of_piecewise_linear_profiles():
    """Linear u(z), v(z), T(z) in each domain with continuous flux mu du/dz,
    kappa dT/dz across the lid: the bulk formulas give exactly that flux, and
    both sides' wall states agree."""
    w = inputs.small3d().with_(nx=4, ny=4, nz_lower=4, nz_upper=6, mu_lower=2e-3, mu_upper=5e-4)
    pb = prob3(w)
    g, pr = w.gamma, w.prandtl
    k1, k2 = w.mu_lower / ((g - 1) * pr), w.mu_upper / ((g - 1) * pr)
    su, sv, q_ = 0.3, -0.2, 0.05          # sigma_xz, sigma_yz, heat flux -Pi_z
    z1 = -(np.arange(w.nz_lower)[::-1] + 0.5) * w.dz_lower
    z2 = (np.arange(w.nz_upper) + 0.5) * w.dz_upper
    out = []
    for z, mu, k in ((z1, w.mu_lower, k1), (z2, w.mu_upper, k2)):
        u = 0.1 + su / mu * z
        v = -0.05 + sv / mu * z
        T = 1.0 + q_ / k * z
        nz = len(z)
        q = np.zeros((5, nz, w.ny, w.nx))
        rho = 1.0
        q[0] = rho
        q[1] = (rho * u)[:, None, None]
        q[2] = (rho * v)[:, None, None]
        q[4] = (rho * T / g / (g - 1) + 0.5 * rho * (u * u + v * v))[:, None, None]
        out.append(q)
    ifc = oracle.interface3(pb, out[0], out[1])
    assert np.allclose(ifc[..., 0], su, rtol=1e-12)
    assert np.allclose(ifc[..., 1], sv, rtol=1e-12)
    assert np.allclose(ifc[..., 2], -q_, rtol=1e-12)
    assert np.allclose(ifc[..., 3], ifc[..., 6], rtol=1e-12, atol=1e-15)
    assert np.allclose(ifc[..., 3], 0.1, rtol=1e-12) and np.allclose(ifc[..., 4], -0.05, rtol=1e-12)


def test_llf3_consistency_and_rotation():
    q = np.array([1.1, 0.2, -0.1, 0.3, 2.5])
    for d in range(3):
        un = q[1 + d] / q[0]
        u = q[1:4] / q[0]
        p = 0.4 * (q[4] - 0.5 * q[0] * (u ** 2).sum())
        f = q * un
        f[1 + d] += p
        f[4] = (q[4] + p) * un
        assert np.allclose(oracle.llf3(q, q, d), f, rtol=1e-15, atol=1e-16)
    qL = np.array([1.0, 0.1, 0.05, -0.02, 2.4])
    qR = np.array([0.9, -0.1, 0.02, 0.03, 2.2])
    perm = [0, 2, 1, 3, 4]                        # exchange x and y
    assert np.allclose(oracle.llf3(qL, qR, 0), oracle.llf3(qL[perm], qR[perm], 1)[perm],
                       rtol=1e-15, atol=1e-16)


def _exact3(gamma, prandtl, mu, L):
    import sympy as sp
    x, y, z = sp.symbols("x y z", real=True)
    kx, ky, kz = [2 * sp.pi / v for v in L]
    r = sp.Rational
    rho = 1 + r(1, 5) * sp.sin(kx * x + r(3, 10)) * sp.cos(ky * y) * sp.cos(kz * z + r(1, 7))
    u = r(3, 10) + r(1, 10) * sp.cos(kx * x) * sp.sin(ky * y + r(1, 5)) * sp.cos(kz * z)
    v = -r(1, 5) + r(1, 10) * sp.sin(kx * x + r(2, 5)) * sp.cos(ky * y) * sp.sin(kz * z + r(1, 3))
    w = r(1, 10) * sp.sin(kx * x + r(1, 2)) * sp.cos(ky * y + r(1, 4)) * sp.cos(kz * z + r(1, 10))
    p = (1 + r(1, 10) * sp.cos(kx * x + r(7, 10)) * sp.sin(ky * y + r(1, 9)) * sp.sin(kz * z)) / gamma
    g = sp.nsimplify(gamma)
    E = p / (g - 1) + rho * (u * u + v * v + w * w) / 2
    T = g * p / rho
    d = sp.diff
    X = (x, y, z)
    U = (u, v, w)
    div = d(u, x) + d(v, y) + d(w, z)
    sig = [[mu * (d(U[a], X[b]) + d(U[b], X[a])) - (2 * mu * div / 3 if a == b else 0)
            for b in range(3)] for a in range(3)]
    kap = mu / ((g - 1) * prandtl)
    q = [rho, rho * u, rho * v, rho * w, E]
    R = []
    for comp in range(5):
        tot = 0
        for a in range(3):
            un = U[a]
            if comp == 0:
                fi, fv = rho * un, 0
            elif comp <= 3:
                c = comp - 1
                fi = rho * U[c] * un + (p if c == a else 0)
                fv = sig[a][c]
            else:
                fi = (E + p) * un
                fv = sum(U[c] * sig[a][c] for c in range(3)) + kap * d(T, X[a])
            tot += -d(fi, X[a]) + d(fv, X[a])
        R.append(tot)
    return sp.lambdify(X, q, "numpy"), sp.lambdify(X, R, "numpy")


def test_spatial_second_order_against_exact_pde_3d():
    gamma, pr, mu = 1.4, 0.72, 0.05
    L = (10.0, 8.0, 5.0)
    qf, rf = _exact3(gamma, pr, mu, L)
    errs = []
    for n in (16, 32, 64):
        w = inputs.small3d().with_(nx=n, ny=n, nz_lower=n // 2, nz_upper=n // 2, lx=L[0], ly=L[1],
                                   lz_lower=L[2], lz_upper=L[2], mu_lower=mu, mu_upper=mu)
        pb = prob3(w)
        x = -L[0] / 2 + (np.arange(n) + 0.5) * w.dx
        y = -L[1] / 2 + (np.arange(n) + 0.5) * w.dy
        qs, rs = [], []
        for z0, dz, nz in ((-L[2], w.dz_lower, n // 2), (0.0, w.dz_upper, n // 2)):
            z = z0 + (np.arange(nz) + 0.5) * dz
            Z, Y, Xg = np.meshgrid(z, y, x, indexing="ij")
            qs.append(np.array([np.broadcast_to(v, Xg.shape) for v in qf(Xg, Y, Z)], dtype=np.float64))
            rs.append(np.array([np.broadcast_to(v, Xg.shape) for v in rf(Xg, Y, Z)], dtype=np.float64))
        rl, ru = oracle.rhs3(pb, np.ascontiguousarray(qs[0]), np.ascontiguousarray(qs[1]))
        out = []
        for r, rex in ((rl, rs[0]), (ru, rs[1])):
            nz = r.shape[1]
            sl = slice(2, nz - 2)           # away from walls and the interface
            out.append(np.abs(r[:, sl] - rex[:, sl]).max(axis=(1, 2, 3)))
        errs.append(np.max(out, axis=0))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(rates[-1] > 1.85), (errs, rates)
    assert np.all(errs[-1] < 2e-3)
