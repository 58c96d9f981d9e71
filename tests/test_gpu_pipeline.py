"""The optimisation loop end to end on the device, checked step by step.

Simple-update start (Sec. III), then two gradient steps, each made of
Metropolis steps (one exchange proposal per chain and step, each costing a whole evaluation) of 32 chains (weight W^2, Sec. II), the Eq. (3) sums over
every visited configuration and the Eq. (6) sign update, all through the
C-ABI.  At every stage the oracle is run on the same inputs: the simple-update
state, the chains' configurations before each move (so one borderline accept
decision cannot make the two sides drift apart), and the same p.
"""
import numpy as np
import pytest

from oracle import brute, go, metropolis, su
from paper_1611_09467_amd import binding as bd
from paper_1611_09467_amd import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    c = bd.Context(0)
    yield c
    c.close()


def _flat(parts):
    return np.concatenate([a.ravel() for a in parts])


def test_su_then_two_gradient_steps_4x4(ctx):
    N, M, D, Dc, J1, J2 = 4, 4, 2, 4, 1.0, 0.0
    chains, steps, dt = 32, 6, 0.005  # the first step size of the paper's schedule
    G = wl.make_peps(N, M, D, seed=77)
    P = bd.Peps(ctx, N, M, D, wl.pack_peps(G))
    gam, lam = P.su_start()
    print("[gpu] pipeline 4x4 D=2: simple update 30 steps", flush=True)
    P.su_evolve(gam, lam, J1, 0.05, 30)
    P.su_to_peps(gam, lam)
    T_gpu = P.read().cpu().numpy()
    Go, lo = su.evolve(G, su.initial_weights(N, M, D), J1, 0.05, 30, D)
    a = brute.state_vector(wl.unpack_peps(T_gpu, N, M, D), N, M)
    b = brute.state_vector(su.to_peps(Go, lo), N, M)
    assert np.linalg.norm(a - b) <= 1e-8 * np.linalg.norm(b)

    starts, picks, uniforms = wl.chain_draws(N, M, chains, 2 * steps, 78)
    bonds = wl.nn_bonds(N, M)
    cfg = torch.from_numpy(np.ascontiguousarray(starts)).cuda()
    rng = np.random.default_rng(79)
    for step in range(2):
        T = wl.unpack_peps(T_gpu, N, M, D)
        sums, visited = None, []
        print(f"[gpu] pipeline gradient step {step}: {steps} Metropolis steps x {chains} chains",
              flush=True)
        for t in range(step * steps, (step + 1) * steps):
            before = cfg.cpu().numpy().copy()
            bt = torch.from_numpy(picks[:, t].astype(np.int32)).cuda()
            ut = torch.from_numpy(uniforms[:, t].copy()).cuda()
            out, acc = P.metropolis_step(cfg, bt, ut, Dc, J1, J2, want_grad=True)
            sums = P.go_accumulate(torch.from_numpy(before).cuda(), out, sums)
            torch.cuda.synchronize()
            after, acc = cfg.cpu().numpy(), acc.cpu().numpy()
            for c in range(chains):
                o, s2, oacc, R = metropolis.shared_ratio_step(T, Dc, before[c], bonds[picks[c, t]],
                                                              uniforms[c, t], J1, J2)
                if np.isfinite(R) and abs(uniforms[c, t] - min(1.0, R * R)) <= 1e-9:
                    continue  # borderline: either decision is right
                assert bool(acc[c]) == bool(oacc), (step, t, c)
                assert np.array_equal(after[c], s2), (step, t, c)
            visited.append(before)
        torch.cuda.synchronize()
        visited = np.concatenate(visited)
        sd, sde, n, se, se2 = go.accumulate(T, visited, Dc, J1, J2)
        assert sums["stats"][0].item() == n == len(visited)
        o_sd, o_sde = _flat(sd), _flat(sde)
        assert np.linalg.norm(sums["sum_delta"].cpu().numpy() - o_sd) <= 1e-8 * np.linalg.norm(o_sd)
        assert np.linalg.norm(sums["sum_delta_e"].cpu().numpy() - o_sde) <= 1e-8 * np.linalg.norm(o_sde)
        p = rng.random(P.nparams)
        P.go_update(sums, dt, torch.from_numpy(p).cuda())
        T_new = P.read().cpu().numpy()
        grad = go.gradient(sd, sde, n, se)
        g = _flat(grad)
        scale = 2.0 * (np.abs(o_sde) + np.abs(o_sd) * abs(se / n)) / n
        decided = np.abs(g) > 1e-7 * scale + 1e-9 * np.abs(g).max()
        step_gpu = T_new - T_gpu
        assert np.allclose(step_gpu[decided], -p[decided] * dt * np.sign(g[decided]), rtol=0,
                           atol=1e-15)
        assert np.all(np.isclose(np.abs(step_gpu[~decided]), 0, atol=1e-15)
                      | np.isclose(np.abs(step_gpu[~decided]), p[~decided] * dt, atol=1e-15))
        print(f"  step {step}: {len(visited)} samples, <E>/site {se / n / (N * M):.5f}, "
              f"{int(decided.sum())} of {g.size} elements decided", flush=True)
        T_gpu = T_new
    P.free()
