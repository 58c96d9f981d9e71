"""Write the stored Metropolis-chain configurations of a named workload.

    python -m oracle.make_chains 10x10_D6_Dc12 [--procs 8]

Input-generation infrastructure: the chains need amplitudes, which come from
this float64 CPU reference (``oracle.metropolis``); the random draws come
from ``workloads.chain_draws`` with the workload's seed.  The output file is
read by ``workloads.metropolis_configs`` and holds the configurations as
packed bits together with the parameters that made them.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np  # noqa: E402

from paper_1611_09467_amd import workloads as wl  # noqa: E402

from . import metropolis  # noqa: E402

_STATE = {}


def _init(name):
    w = wl.WORKLOADS[name]
    _STATE["T"] = wl.make_peps(w["N"], w["M"], w["D"], seed=w["seed"], bias=w["bias"])
    _STATE["Dc"] = w["Dc"]
    _STATE["bonds"] = wl.nn_bonds(w["N"], w["M"])


def _chain(args):
    start, picks, uniforms = args
    return metropolis.run_chain(_STATE["T"], _STATE["Dc"], start, picks, uniforms,
                                _STATE["bonds"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    w = wl.WORKLOADS[a.name]
    seed = w["seed"] + 1000
    starts, picks, uniforms = wl.chain_draws(w["N"], w["M"], w["chains"], w["steps"], seed)
    t0 = time.time()
    import multiprocessing as mp
    with mp.get_context("fork").Pool(a.procs, initializer=_init, initargs=(a.name,)) as pool:
        parts = pool.map(_chain, list(zip(starts, picks, uniforms)), chunksize=1)
    S = np.concatenate(parts).astype(np.uint8)
    moved = float(np.mean(np.any(S[1:] != S[:-1], axis=1)))
    wl.DATA_DIR.mkdir(exist_ok=True)
    f = wl.metropolis_file(a.name)
    np.savez_compressed(f, bits=np.packbits(S.ravel()), count=S.shape[0], sites=S.shape[1],
                        seed=seed, chains=w["chains"], steps=w["steps"], Dc=w["Dc"],
                        sha256=hashlib.sha256(S.tobytes()).hexdigest())
    print(f"{a.name}: {S.shape[0]} configs in {time.time() - t0:.0f} s, "
          f"fraction of steps that moved {moved:.3f} -> {f}")


if __name__ == "__main__":
    main()
