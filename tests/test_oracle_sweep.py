"""Pins of the environment-reusing Metropolis sweep (oracle/sweep.py).

  * exact regime (nothing truncated): every ratio a sweep decides with equals
    W(S')/W(S) of the configuration at that moment, both W by brute-force
    contraction of the whole network;
  * the chain of sweeps has W(S)^2 as its stationary distribution: visit
    frequencies on 2x3 against brute-force W^2 (far from |W| or W^4);
  * under truncation the incremental environments give the decisions and
    ratios of a full evaluation of the current configuration before every
    single proposal (oracle.metropolis.shared_ratio_step applied bond by bond).
"""
import itertools
import math

import numpy as np

from oracle import brute, metropolis, sweep
from paper_1611_09467_amd import workloads as wl


def test_exact_regime_ratios_are_brute_force_ratios():
    N, M, D = 3, 3, 2
    T = wl.make_peps(N, M, D, seed=41, bias=0.1)
    rng = np.random.default_rng(42)
    order = sweep.bond_order(N, M)
    for S in wl.random_sz0_configs(N, M, 3, 43):
        u = rng.random(len(order))
        new, acc, ratios = sweep.sweep(T, D * D, S, u)
        cur = S.copy()
        nprop = 0
        for k, (a, b) in enumerate(order):
            if cur[a] == cur[b]:
                assert math.isnan(ratios[k]) and not acc[k]
                continue
            nprop += 1
            nxt = cur.copy()
            nxt[a], nxt[b] = cur[b], cur[a]
            r = brute.amplitude(T, nxt.reshape(N, M)) / brute.amplitude(T, cur.reshape(N, M))
            assert abs(ratios[k] - r) <= 1e-10 * max(1.0, abs(r)), (k, ratios[k], r)
            assert acc[k] == (u[k] < min(1.0, r * r))
            if acc[k]:
                cur = nxt
        assert nprop > 0 and np.array_equal(cur, new)


def test_sweeps_sample_w_squared_on_2x3():
    N, M, D = 2, 3, 2
    T = wl.make_peps(N, M, D, seed=11)
    states = [np.array(c, dtype=np.uint8) for c in itertools.product((0, 1), repeat=N * M)
              if sum(c) == N * M // 2]
    w2 = np.array([brute.amplitude(T, s.reshape(N, M)) ** 2 for s in states])
    p = w2 / w2.sum()
    keys = {tuple(s): k for k, s in enumerate(states)}
    rng = np.random.default_rng(5)
    nb = len(sweep.bond_order(N, M))
    s = states[0]
    counts = np.zeros(len(states))
    for t in range(8000):
        s, _, _ = sweep.sweep(T, D * D, s, rng.random(nb))
        if t >= 200:
            counts[keys[tuple(s)]] += 1
    freq = counts / counts.sum()
    assert np.abs(freq - p).max() < 0.03, (freq, p)
    for wrong in (np.sqrt(w2) / np.sqrt(w2).sum(), w2 ** 2 / (w2 ** 2).sum()):
        assert np.abs(wrong - p).max() > 0.15


def test_truncated_sweep_equals_bond_by_bond_full_evaluations():
    N, M, D, Dc = 5, 4, 3, 4
    T = wl.make_peps(N, M, D, seed=61, bias=0.1)
    order = sweep.bond_order(N, M)
    rng = np.random.default_rng(62)
    for S in wl.random_sz0_configs(N, M, 2, 63):
        u = rng.random(len(order))
        new, acc, ratios = sweep.sweep(T, Dc, S, u)
        cur = S.copy()
        for k, (a, b) in enumerate(order):
            if cur[a] == cur[b]:
                continue
            _, nxt, ok, R = metropolis.shared_ratio_step(T, Dc, cur, (a, b), u[k])
            assert abs(ratios[k] - R) <= 1e-9 * max(1.0, abs(R)), (k, ratios[k], R)
            assert ok == acc[k], k
            cur = nxt
        assert np.array_equal(cur, new)
