"""Oracle evaluations of many samples in worker processes.

The workers are spawned (fresh interpreters that import only numpy and the
oracle), so they never touch the GPU of the test process; each uses one BLAS
thread.  At most 16 workers.
"""
from __future__ import annotations

import multiprocessing as mp
import os

from oracle import conditioning, correlations, peps

_STATE = {}


def _init(T, Dc, J1, J2, want_grad, want_eloc):
    _STATE.update(T=T, Dc=Dc, J1=J1, J2=J2, want_grad=want_grad, want_eloc=want_eloc)


def _evaluate(s):
    st = _STATE
    return peps.evaluate(st["T"], s, st["Dc"], st["J1"], st["J2"], want_grad=st["want_grad"],
                         want_eloc=st["want_eloc"])


def _kappa(s):
    st = _STATE
    return conditioning.kappa(st["T"], s, st["Dc"], st["J1"], st["J2"],
                              want_grad=st["want_grad"])[1]


def _ratios(args):
    s, window = args
    return correlations.ratio_matrix(_STATE["T"], s, _STATE["Dc"], window)


def _kappa_ratios(args):
    s, window = args
    return conditioning.kappa_ratios(_STATE["T"], s, _STATE["Dc"], window)[1]


class OraclePool:
    """map(evaluate), map(kappa) and the exchange ratios over configurations of one PEPS."""

    def __init__(self, T, Dc, J1=1.0, J2=0.0, want_grad=True, want_eloc=True, workers=None):
        n = workers or min(16, os.cpu_count() or 1)
        saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
        os.environ["OMP_NUM_THREADS"] = os.environ["OPENBLAS_NUM_THREADS"] = "1"
        try:
            self.pool = mp.get_context("spawn").Pool(
                n, initializer=_init, initargs=(T, Dc, J1, J2, want_grad, want_eloc))
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v

    def evaluate(self, configs):
        return self.pool.map(_evaluate, list(configs), chunksize=4)

    def kappa(self, configs):
        return self.pool.map(_kappa, list(configs), chunksize=1)

    def ratios(self, configs, window):
        """correlations.ratio_matrix of each configuration on ``window``."""
        return self.pool.map(_ratios, [(s, tuple(window)) for s in configs], chunksize=1)

    def kappa_ratios(self, configs, window):
        """Per-pair kappa of the exchange ratios (conditioning.kappa_ratios)."""
        return self.pool.map(_kappa_ratios, [(s, tuple(window)) for s in configs], chunksize=1)

    def close(self):
        self.pool.close()
        self.pool.join()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
