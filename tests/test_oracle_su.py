"""Pins of the simple-update initialiser (oracle.su).

* The gate against the closed form of exp(-tau J S.S): the bond term has the
  singlet at -3J/4 and the triplet at +J/4, so
  exp(-tau h) = e^{-tau J/4} (1 - P_s) + e^{3 tau J/4} P_s.
* On open chains whose bond dimension D never forces a truncation (1x3 and
  3x1 with D = 2, 1x4 with D = 4, where the end bonds carry rank 2 < D and the
  zero weights are skipped) the simple update is exact: the state after n
  steps equals the product of the full-space bond propagators, applied in the
  same group order, to the initial state (brute-force contraction of the
  network, operators built from Kronecker products).
* Many small steps on a single bond reach the singlet, E = -3/4 J.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import brute, su
from paper_1611_09467_amd import workloads as wl


def test_gate_closed_form():
    J, tau = 1.3, 0.07
    ps = np.zeros((4, 4))
    ps[1, 1] = ps[2, 2] = 0.5
    ps[1, 2] = ps[2, 1] = -0.5
    ref = np.exp(-tau * J / 4) * (np.eye(4) - ps) + np.exp(3 * tau * J / 4) * ps
    assert np.allclose(su.gate(J, tau), ref, rtol=0, atol=1e-14)
    w = np.linalg.eigvalsh(su.bond_hamiltonian(J))
    assert np.allclose(w, [-0.75 * J, 0.25 * J, 0.25 * J, 0.25 * J])


def _full_bond(n, a, b, J):
    """J S_a.S_b on the 2^n space, bit k of the basis index = s of site k (s=1: S^z=-1/2)."""
    sx = np.array([[0, 0.5], [0.5, 0]], dtype=complex)
    sy = np.array([[0, -0.5j], [0.5j, 0]])
    sz = np.array([[0.5, 0], [0, -0.5]], dtype=complex)
    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for op in (sx, sy, sz):
        mats = [np.eye(2, dtype=complex)] * n
        mats = list(mats)
        mats[a], mats[b] = op, op
        full = mats[n - 1]
        for k in range(n - 2, -1, -1):
            full = np.kron(full, mats[k])
        H += full
    assert np.allclose(H.imag, 0)
    return J * H.real


@pytest.mark.parametrize("N,M,D", [(1, 3, 2), (3, 1, 2), (1, 4, 4), (4, 1, 4)])
def test_exact_on_chains(N, M, D):
    J, dtau, nsteps = 1.0, 0.05, 6
    G = wl.make_peps(N, M, D, seed=31 + N + 7 * M)
    lam = su.initial_weights(N, M, D)
    psi = brute.state_vector(su.to_peps(G, lam), N, M)
    n = N * M
    for _ in range(nsteps):
        for grp in su.bond_groups(N, M):
            for kind, i, j in grp:
                a = i * M + j
                b = a + 1 if kind == "h" else a + M
                psi = sla.expm(-dtau * _full_bond(n, a, b, J)) @ psi
    G2, lam2 = su.evolve(G, lam, J, dtau, nsteps, D)
    got = brute.state_vector(su.to_peps(G2, lam2), N, M)
    ov = abs(got @ psi) / (np.linalg.norm(got) * np.linalg.norm(psi))
    assert ov == pytest.approx(1.0, abs=1e-12)
    for row in lam2["h"] + lam2["v"]:
        for w in row:
            assert np.linalg.norm(w) == pytest.approx(1.0, abs=1e-14)
            assert np.all(np.diff(w) <= 0)


def test_single_bond_reaches_singlet():
    G = wl.make_peps(1, 2, 2, seed=3)
    lam = su.initial_weights(1, 2, 2)
    G2, lam2 = su.evolve(G, lam, 1.0, 0.05, 400, 2)
    psi = brute.state_vector(su.to_peps(G2, lam2), 1, 2)
    H = _full_bond(2, 0, 1, 1.0)
    assert psi @ H @ psi / (psi @ psi) == pytest.approx(-0.75, abs=1e-10)
    assert np.allclose(lam2["h"][0][0], [np.sqrt(0.5), np.sqrt(0.5)], atol=1e-10)


def test_grow_keeps_the_state_and_stays_exact():
    # 1x4 chain: evolve at D=2 (truncating the middle bond), grow to D=4, evolve on;
    # the grown state equals the D=2 state, and the steps at D=4 are exact again
    N, M, J, dtau = 1, 4, 1.0, 0.05
    G = wl.make_peps(N, M, 2, seed=8)
    G1, lam1 = su.evolve(G, su.initial_weights(N, M, 2), J, dtau, 3, 2)
    psi1 = brute.state_vector(su.to_peps(G1, lam1), N, M)
    G2, lam2 = su.grow(G1, lam1, 4)
    psi2 = brute.state_vector(su.to_peps(G2, lam2), N, M)
    assert np.allclose(psi1, psi2, rtol=0, atol=1e-15)
    assert all(t.shape[2] in (1, 4) for t in G2[0])
    G3, lam3 = su.evolve(G2, lam2, J, dtau, 4, 4)
    psi = psi2.copy()
    for _ in range(4):
        for grp in su.bond_groups(N, M):
            for kind, i, j in grp:
                psi = sla.expm(-dtau * _full_bond(N * M, j, j + 1, J)) @ psi
    got = brute.state_vector(su.to_peps(G3, lam3), N, M)
    ov = abs(got @ psi) / (np.linalg.norm(got) * np.linalg.norm(psi))
    assert ov == pytest.approx(1.0, abs=1e-12)
