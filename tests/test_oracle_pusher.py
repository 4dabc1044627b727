"""Pins of the oracle's Boris pusher (the push that feeds the run-time deposit)."""
import math

import numpy as np


def test_uniform_electric_field_is_exact_for_momentum(oracle_mod):
    """A uniform E kicks u by qm E dt per step exactly; from rest the position
    follows hyperbolic motion, x(t) = (sqrt(1 + (qm E t)^2) - 1) / (qm E), to second
    order in dt."""
    E = np.array([0.0, 0.0, 0.3])
    qm = -1.0
    errs = []
    for n in (100, 200, 400):
        T = 10.0
        x, u = oracle_mod.boris_push(np.zeros((3, 1)), np.zeros((3, 1)), qm, T / n, n, {"E": E})
        t = np.arange(n + 1) * (T / n)
        np.testing.assert_allclose(u[2, :, 0], qm * E[2] * t, rtol=1e-13, atol=1e-15)
        a = qm * E[2]
        exact = (np.sqrt(1 + (a * t) ** 2) - 1) / a
        errs.append(np.abs(x[2, :, 0] - exact).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 0.15), orders


def test_uniform_magnetic_field_rotates_by_the_boris_angle(oracle_mod):
    """In a uniform B, |u| is kept exactly and u turns by 2 atan(|qm| B dt / (2 gamma))
    per step: the Boris map's rotation, which tends to the gyration angle omega dt."""
    B = np.array([0.0, 0.0, 2.0])
    qm, dt, n = -1.0, 0.05, 300
    u0 = np.array([[3.0], [0.0], [0.5]])
    x, u = oracle_mod.boris_push(np.zeros((3, 1)), u0, qm, dt, n, {"B": B})
    g = math.sqrt(1 + (u0 ** 2).sum())
    np.testing.assert_allclose(np.linalg.norm(u[:, :, 0], axis=0), math.sqrt(g * g - 1), rtol=1e-14)
    ang = np.unwrap(np.arctan2(u[1, :, 0], u[0, :, 0]))
    step = 2 * math.atan(abs(qm) * B[2] * dt / (2 * g))
    # an electron (qm < 0) turns counter-clockwise about +z
    np.testing.assert_allclose(ang, step * np.arange(n + 1), rtol=0, atol=1e-11)
    np.testing.assert_allclose(u[2, :, 0], 0.5, rtol=0, atol=1e-14)


def test_plane_wave_follows_the_exact_solution(oracle_mod):
    """An electron at rest in a linearly polarised plane wave along x: u_y = qm (a/omega)
    sin(phase) (canonical momentum) and u_x = u_y^2 / 2 (light-front invariant
    gamma - u_x = 1), as functions of the phase omega (t - x); second order in dt."""
    a, om, qm = 2.0, 1.0, -1.0
    fields = {"wave_amplitude": a, "wave_dir": [1.0, 0.0, 0.0], "wave_pol": [0.0, 1.0, 0.0],
              "wave_omega": om, "wave_phase": 0.0}
    errs = []
    for n in (400, 800, 1600):
        T = 4 * math.pi
        dt = T / n
        x, u = oracle_mod.boris_push(np.zeros((3, 1)), np.zeros((3, 1)), qm, dt, n, fields)
        t = np.arange(n + 1) * dt
        ph = om * (t - x[0, :, 0])
        uy = qm * (a / om) * np.sin(ph)
        errs.append(max(np.abs(u[1, :, 0] - uy).max(), np.abs(u[0, :, 0] - uy ** 2 / 2).max()))
        g = np.sqrt(1 + (u[:, :, 0] ** 2).sum(axis=0))
        np.testing.assert_allclose(g - u[0, :, 0], 1.0, rtol=0, atol=50 * dt ** 2)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.8), orders
