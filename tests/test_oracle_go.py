"""Pins of the gradient-optimisation step (Eqs. (3) and (6)).

The Eq. (3) estimator, averaged exactly (weights W^2/Z over every S^z = 0
configuration) on a lattice small enough for the exact regime, must equal the
derivative of the energy E(T) = <psi|H|psi>/<psi|psi> taken by central finite
differences, with psi from brute-force contraction and H from exact
diagonalisation's sector operators (neither uses the boundary-MPS code).
"""
import numpy as np
import pytest

from oracle import brute, ed, go
from paper_1611_09467_amd import workloads as wl

N, M, D = 2, 3, 2
J1, J2 = 1.0, 0.5


def _energy(T):
    states, hnn, hnnn = ed.hamiltonian_blocks(N, M)
    psi = np.array([brute.amplitude(T, ed.config_of_state(int(st), N, M)) for st in states])
    H = J1 * hnn + J2 * hnnn
    return float(psi @ (H @ psi) / (psi @ psi))


def test_eq3_exact_average_is_the_energy_gradient():
    T = wl.make_peps(N, M, D, seed=31, bias=0.2)
    states, _, _ = ed.hamiltonian_blocks(N, M)
    configs = [ed.config_of_state(int(st), N, M).reshape(-1) for st in states]
    w2 = np.array([brute.amplitude(T, c.reshape(N, M)) ** 2 for c in configs])
    sd, sde, n, se, _ = go.accumulate(T, configs, D ** 2, J1, J2, weights=w2 / w2.sum())
    g = go.gradient(sd, sde, n, se)
    rng = np.random.default_rng(0)
    h = 1e-6
    checked = 0
    for k in (0, 2, 4):
        i, j = divmod(k, M)
        for _ in range(3):
            idx = tuple(int(rng.integers(0, d)) for d in T[i][j].shape)
            Tp = [[t.copy() for t in row] for row in T]
            Tm = [[t.copy() for t in row] for row in T]
            Tp[i][j][idx] += h
            Tm[i][j][idx] -= h
            fd = (_energy(Tp) - _energy(Tm)) / (2 * h)
            assert g[k][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8), (k, idx)
            checked += 1
    assert checked == 9


def test_eq6_sign_update():
    T = wl.make_peps(2, 2, 2, seed=1)
    grad = [np.where(np.arange(t.size).reshape(t.shape) % 3 == 0, 0.0,
                     np.where(np.arange(t.size).reshape(t.shape) % 2 == 0, 2.5, -1e-9))
            for row in T for t in row]
    p = [np.full(t.shape, 0.25) for row in T for t in row]
    T2 = go.sign_update(T, grad, 0.01, p)
    for k, (t, t2) in enumerate(zip([t for row in T for t in row], [t for row in T2 for t in row])):
        assert np.allclose(t2 - t, -0.0025 * np.sign(grad[k]), atol=1e-15, rtol=0)
        assert np.array_equal(t2 == t, grad[k] == 0)
