"""Host side of the optimisation protocols (paper_1611_09467_amd/protocols.py).

The schedule of Sec. III: 50 steps at dt = 0.005 with M from 5e4 to 1e5, 50
steps with dt(n+1) = 0.968 dt(n) ending near 0.001 with M rising to 5e5, and
20 steps at dt = 0.001 with M = 5e5; the S^z = 0 enumeration used for exact
energies.
"""
import math

import numpy as np
import pytest

from paper_1611_09467_amd import protocols as pr


def test_go_schedule_phases():
    s = pr.go_schedule()
    assert len(s) == 120
    dt = [a for a, _ in s]
    m = [b for _, b in s]
    assert all(x == 0.005 for x in dt[:50])
    assert dt[50] == pytest.approx(0.005 * 0.968)
    for n in range(51, 100):
        assert dt[n] == pytest.approx(dt[n - 1] * 0.968, rel=1e-15)
    assert dt[99] == pytest.approx(0.001, rel=0.02)          # "from 0.005 to 0.001"
    assert all(x == 0.001 for x in dt[100:])
    assert m[0] == 50000 and m[49] == 100000
    assert all(b > a for a, b in zip(m[50:100], m[51:100]))
    assert m[99] == 500000 and all(x == 500000 for x in m[100:])
    assert all(b >= a for a, b in zip(m, m[1:]))


def test_scaled_schedule_keeps_its_phases():
    s = pr.go_schedule(first=4, decay=3, last=2, m0=100, m1=200, m_max=400)
    assert [a for a, _ in s][:4] == [0.005] * 4 and [a for a, _ in s][-2:] == [0.001] * 2
    assert [b for _, b in s] == [100, 133, 167, 200, 267, 333, 400, 400, 400]


@pytest.mark.parametrize("N,M", [(2, 2), (2, 3), (4, 4)])
def test_sz0_enumeration(N, M):
    S = pr.sz0_configs(N, M)
    n = N * M
    assert len(S) == math.comb(n, n // 2)
    assert np.all(S.sum(axis=1) == n // 2)
    assert len({bytes(c) for c in S}) == len(S)
