"""ctypes binding of the pepsgo C-ABI (include/pepsgo.h).

Argument marshalling only: every step of the evaluation runs in the HIP
library.  The low-level functions carry the C names and take plain integer
addresses; ``Peps.evaluate`` is a convenience wrapper that allocates the
output and workspace buffers as torch tensors on the device.  Loading fails
loudly when the built library is absent.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(HERE, "libpepsgo.so")

PEPSGO_OK = 0
PEPSGO_EINVAL = -1
PEPSGO_ENOMEM = -2
PEPSGO_EUNSUPPORTED = -3
PEPSGO_EDEVICE = -4
PEPSGO_EBUSY = -5
PEPSGO_WARN_SAMPLES = 1
PEPSGO_FP64 = 0
PEPSGO_FP32 = 1
PEPSGO_BF16_MIXED = 2
PEPSGO_BF16 = 3
PRECISIONS = {"fp64": PEPSGO_FP64, "fp32": PEPSGO_FP32, "bf16x6": PEPSGO_BF16_MIXED,
              "bf16": PEPSGO_BF16}
PEPSGO_GRAD_NONE = 0
PEPSGO_GRAD_PER_SAMPLE = 1
PEPSGO_GRAD_REDUCED = 2
F_ZERO_PSI = 1
F_NONFINITE = 2
F_NEAR_TIE = 4
F_REFINED = 8

# every entry point declared in include/pepsgo.h
EXPORTS = (
    "pepsgo_version", "pepsgo_last_error", "pepsgo_create", "pepsgo_destroy", "pepsgo_peps_load",
    "pepsgo_peps_update", "pepsgo_peps_free", "pepsgo_grad_layout", "pepsgo_workspace_bytes",
    "pepsgo_evaluate", "pepsgo_profile", "pepsgo_profile_read", "pepsgo_serve_create",
    "pepsgo_serve_submit", "pepsgo_serve_poll", "pepsgo_serve_pending", "pepsgo_serve_destroy",
    "pepsgo_tune_get", "pepsgo_tune_set", "pepsgo_autotune", "pepsgo_tune_save", "pepsgo_tune_load",
    "pepsgo_graph_create", "pepsgo_graph_launch", "pepsgo_graph_free", "pepsgo_metropolis_step",
    "pepsgo_go_accumulate", "pepsgo_go_update", "pepsgo_peps_read", "pepsgo_su_workspace_bytes",
    "pepsgo_su_evolve", "pepsgo_su_to_peps", "pepsgo_su_pad", "pepsgo_sz_counts", "pepsgo_structure_factor",
    "pepsgo_evaluate_noalloc", "pepsgo_metropolis_sweep", "pepsgo_transverse_workspace_bytes",
    "pepsgo_transverse", "pepsgo_spin_structure_factor", "pepsgo_serve_stats", "pepsgo_peak_probe",
)
NOALLOC_SCRATCH_BYTES = 128 << 20  # PEPSGO_NOALLOC_SCRATCH_BYTES
KERNEL_CLASSES = ("edges", "zip", "sandwich", "strip", "finalize")


class EvalParams(ctypes.Structure):
    _fields_ = [("Dc", ctypes.c_int), ("J1", ctypes.c_double), ("J2", ctypes.c_double),
                ("precision", ctypes.c_int), ("grad_mode", ctypes.c_int), ("want_eloc", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("zip_lds_bytes", ctypes.c_int), ("sandwich_lds_bytes", ctypes.c_int),
                ("strip_lds_bytes", ctypes.c_int), ("strip_xc", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServeConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_size_t), ("streams", ctypes.c_int),
                ("max_chunk", ctypes.c_int), ("min_chunk", ctypes.c_int),
                ("max_pending", ctypes.c_int)]


class ServeStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("samples", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("samples_per_s", ctypes.c_double), ("pending", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServeDone(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int), ("batch", ctypes.c_int),
                ("t_submit_ns", ctypes.c_int64), ("t_start_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class PepsgoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pepsgo error {code}: {msg}")
        self.code = code


_vp = ctypes.c_void_p
_i64p = ctypes.POINTER(ctypes.c_int64)


def load_library(path: str | None = None) -> ctypes.CDLL:
    path = path or os.environ.get("PEPSGO_LIB", DEFAULT_LIB)
    if not os.path.exists(path):
        raise RuntimeError(f"pepsgo HIP library not found at {path}; build it with "
                           "`python -m paper_1611_09467_amd.build`")
    lib = ctypes.CDLL(path)
    lib.pepsgo_version.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.pepsgo_last_error.restype = ctypes.c_char_p
    lib.pepsgo_create.argtypes = [ctypes.c_int, ctypes.POINTER(_vp)]
    lib.pepsgo_destroy.argtypes = [_vp]
    lib.pepsgo_peps_load.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     _vp, ctypes.c_int, ctypes.POINTER(_vp)]
    lib.pepsgo_peps_update.argtypes = [_vp, _vp, ctypes.c_int, _vp]
    lib.pepsgo_peps_free.argtypes = [_vp]
    lib.pepsgo_grad_layout.argtypes = [_vp, _i64p, _i64p]
    lib.pepsgo_workspace_bytes.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_size_t)]
    lib.pepsgo_evaluate.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp, _vp, _vp,
                                    _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pepsgo_evaluate_noalloc.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp,
                                            _vp, _vp, _vp, _vp, _vp, _vp]
    lib.pepsgo_metropolis_sweep.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp,
                                            _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pepsgo_profile.argtypes = [_vp, ctypes.c_int]
    lib.pepsgo_profile_read.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                        _i64p]
    lib.pepsgo_metropolis_step.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp, _vp,
                                           _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                           ctypes.c_size_t, _vp]
    lib.pepsgo_su_workspace_bytes.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.pepsgo_su_evolve.argtypes = [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     _vp, ctypes.c_size_t, _vp]
    lib.pepsgo_su_to_peps.argtypes = [_vp, _vp, _vp, _vp]
    lib.pepsgo_su_pad.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.pepsgo_sz_counts.argtypes = [ctypes.c_int] * 7 + [_vp, _vp, _vp, _vp, _vp]
    lib.pepsgo_structure_factor.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, _vp, _vp]
    lib.pepsgo_transverse_workspace_bytes.argtypes = [_vp, ctypes.POINTER(EvalParams)] + \
        [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_size_t)]
    lib.pepsgo_transverse.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp] + \
        [ctypes.c_int] * 4 + [_vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
    lib.pepsgo_spin_structure_factor.argtypes = [ctypes.c_int, ctypes.c_int, _vp, _vp, _vp, _vp,
                                                 ctypes.c_double, ctypes.c_double, _vp, _vp]
    lib.pepsgo_peps_read.argtypes = [_vp, _vp, ctypes.c_int, _vp]
    lib.pepsgo_go_accumulate.argtypes = [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.pepsgo_go_update.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_double, _vp, _vp]
    lib.pepsgo_graph_create.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp, _vp,
                                        _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                        ctypes.POINTER(_vp)]
    lib.pepsgo_graph_launch.argtypes = [_vp, _vp]
    lib.pepsgo_graph_free.argtypes = [_vp]
    lib.pepsgo_tune_get.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(Tuning)]
    lib.pepsgo_tune_set.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(Tuning)]
    lib.pepsgo_autotune.argtypes = [_vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp, _vp,
                                    ctypes.POINTER(Tuning)]
    lib.pepsgo_tune_save.argtypes = [_vp, ctypes.c_char_p]
    lib.pepsgo_tune_load.argtypes = [_vp, ctypes.c_char_p]
    lib.pepsgo_serve_create.argtypes = [_vp, ctypes.POINTER(ServeConfig), ctypes.POINTER(_vp)]
    lib.pepsgo_serve_submit.argtypes = [_vp, _vp, ctypes.POINTER(EvalParams), ctypes.c_int, _vp,
                                        _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.pepsgo_serve_poll.argtypes = [_vp, ctypes.POINTER(ServeDone), ctypes.c_int, ctypes.c_int64]
    lib.pepsgo_serve_pending.argtypes = [_vp, ctypes.POINTER(ctypes.c_int)]
    lib.pepsgo_serve_destroy.argtypes = [_vp]
    lib.pepsgo_serve_stats.argtypes = [_vp, ctypes.POINTER(ServeStats), ctypes.c_int]
    lib.pepsgo_peak_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                      ctypes.POINTER(ctypes.c_double), _vp]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype or ctypes.c_int
    lib.pepsgo_last_error.restype = ctypes.c_char_p
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def check(rc: int, L=None) -> int:
    if rc < 0:
        L = L or lib()
        raise PepsgoError(rc, (L.pepsgo_last_error() or b"").decode())
    return rc


# ---- C names, addresses as Python ints -------------------------------------------------

def pepsgo_version(L=None):
    L = L or lib()
    a, b = ctypes.c_int(), ctypes.c_int()
    check(L.pepsgo_version(ctypes.byref(a), ctypes.byref(b)), L)
    return a.value, b.value


def pepsgo_create(device: int = 0, L=None) -> int:
    L = L or lib()
    h = _vp()
    check(L.pepsgo_create(device, ctypes.byref(h)), L)
    return h.value


def pepsgo_destroy(ctx: int, L=None):
    L = L or lib()
    check(L.pepsgo_destroy(ctx), L)


def pepsgo_peps_load(ctx: int, nrows: int, ncols: int, d: int, D: int, tensors_addr: int,
                     on_device: bool, L=None) -> int:
    L = L or lib()
    h = _vp()
    check(L.pepsgo_peps_load(ctx, nrows, ncols, d, D, tensors_addr, int(on_device),
                             ctypes.byref(h)), L)
    return h.value


def pepsgo_peps_update(peps: int, tensors_addr: int, on_device: bool, stream: int = 0, L=None):
    L = L or lib()
    check(L.pepsgo_peps_update(peps, tensors_addr, int(on_device), stream or None), L)


def pepsgo_peps_free(peps: int, L=None):
    L = L or lib()
    check(L.pepsgo_peps_free(peps), L)


def pepsgo_grad_layout(peps: int, nsites: int, L=None):
    L = L or lib()
    n = ctypes.c_int64()
    offs = (ctypes.c_int64 * (nsites + 1))()
    check(L.pepsgo_grad_layout(peps, ctypes.byref(n), offs), L)
    return n.value, list(offs)


def make_params(Dc: int, J1: float = 1.0, J2: float = 0.0, precision: int = PEPSGO_FP64,
                grad_mode: int = PEPSGO_GRAD_PER_SAMPLE, want_eloc: bool = True) -> EvalParams:
    return EvalParams(Dc, J1, J2, precision, grad_mode, int(want_eloc))


def pepsgo_workspace_bytes(peps: int, params: EvalParams, batch: int, L=None) -> int:
    L = L or lib()
    n = ctypes.c_size_t()
    check(L.pepsgo_workspace_bytes(peps, ctypes.byref(params), batch, ctypes.byref(n)), L)
    return n.value


def pepsgo_evaluate(peps: int, params: EvalParams, batch: int, configs: int, logabs: int,
                    sign: int, eloc: int, flags: int, grad: int, workspace: int,
                    workspace_bytes: int, stream: int = 0, L=None) -> int:
    L = L or lib()
    return check(L.pepsgo_evaluate(peps, ctypes.byref(params), batch, configs, logabs, sign,
                                   eloc, flags, grad or None, workspace, workspace_bytes,
                                   stream or None), L)


def pepsgo_evaluate_noalloc(peps: int, params: EvalParams, batch: int, configs: int, logabs: int,
                            sign: int, eloc: int, flags: int, grad: int, stream: int = 0,
                            L=None) -> int:
    L = L or lib()
    return check(L.pepsgo_evaluate_noalloc(peps, ctypes.byref(params), batch, configs, logabs,
                                           sign, eloc, flags, grad or None, stream or None), L)


def pepsgo_metropolis_sweep(peps: int, params: EvalParams, batch: int, configs: int,
                            uniforms: int, accepted: int, ratios: int, workspace: int,
                            workspace_bytes: int, stream: int = 0, L=None) -> int:
    L = L or lib()
    return check(L.pepsgo_metropolis_sweep(peps, ctypes.byref(params), batch, configs, uniforms,
                                           accepted, ratios or None, workspace, workspace_bytes,
                                           stream or None), L)


def pepsgo_transverse_workspace_bytes(peps: int, params: EvalParams, r0: int, c0: int, h: int,
                                      w: int, batch: int, L=None) -> int:
    L = L or lib()
    out = ctypes.c_size_t()
    check(L.pepsgo_transverse_workspace_bytes(peps, ctypes.byref(params), r0, c0, h, w, batch,
                                              ctypes.byref(out)), L)
    return out.value


def pepsgo_transverse(peps: int, params: EvalParams, batch: int, configs: int, r0: int, c0: int,
                      h: int, w: int, ratios: int, sums: int, count: int, flags: int,
                      workspace: int, workspace_bytes: int, stream: int = 0, L=None) -> int:
    L = L or lib()
    return check(L.pepsgo_transverse(peps, ctypes.byref(params), batch, configs, r0, c0, h, w,
                                     ratios or None, sums, count, flags, workspace,
                                     workspace_bytes, stream or None), L)


def pepsgo_spin_structure_factor(h: int, w: int, same: int, nsamples: int, trans: int,
                                 ntrans: int, kx: float, ky: float, out: int, stream: int = 0,
                                 L=None):
    L = L or lib()
    return check(L.pepsgo_spin_structure_factor(h, w, same, nsamples, trans, ntrans, kx, ky, out,
                                                stream or None), L)


def pepsgo_profile(ctx: int, enable: int, L=None):
    L = L or lib()
    check(L.pepsgo_profile(ctx, enable), L)


def pepsgo_profile_read(ctx: int, kernel_class: int, L=None):
    L = L or lib()
    ms, n = ctypes.c_double(), ctypes.c_int64()
    check(L.pepsgo_profile_read(ctx, kernel_class, ctypes.byref(ms), ctypes.byref(n)), L)
    return ms.value, n.value


def pepsgo_metropolis_step(peps: int, params: EvalParams, batch: int, configs: int, bonds: int,
                           uniforms: int, accepted: int, logabs: int, sign: int, eloc: int,
                           flags: int, grad: int, workspace: int, workspace_bytes: int,
                           stream: int = 0, L=None) -> int:
    L = L or lib()
    return check(L.pepsgo_metropolis_step(peps, ctypes.byref(params), batch, configs, bonds,
                                          uniforms, accepted, logabs, sign, eloc, flags,
                                          grad or None, workspace, workspace_bytes,
                                          stream or None), L)


def pepsgo_su_workspace_bytes(peps: int, L=None) -> int:
    L = L or lib()
    n = ctypes.c_size_t()
    check(L.pepsgo_su_workspace_bytes(peps, ctypes.byref(n)), L)
    return n.value


def pepsgo_su_evolve(peps: int, gamma: int, lambdas: int, J1: float, dtau: float, nsteps: int,
                     workspace: int, workspace_bytes: int, stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_su_evolve(peps, gamma, lambdas, J1, dtau, nsteps, workspace or None,
                                    workspace_bytes, stream or None), L)


def pepsgo_su_pad(src: int, gamma: int, lambdas: int, dst: int, gamma_out: int,
                  lambdas_out: int, stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_su_pad(src, gamma, lambdas, dst, gamma_out, lambdas_out,
                                 stream or None), L)


def pepsgo_su_to_peps(peps: int, gamma: int, lambdas: int, stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_su_to_peps(peps, gamma, lambdas, stream or None), L)


def pepsgo_sz_counts(nrows: int, ncols: int, r0: int, c0: int, h: int, w: int, batch: int,
                     configs: int, flags: int, same: int, nsamples: int, stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_sz_counts(nrows, ncols, r0, c0, h, w, batch, configs, flags or None,
                                    same, nsamples, stream or None), L)


def pepsgo_structure_factor(h: int, w: int, same: int, nsamples: int, kx: float, ky: float,
                            factor: float, out: int, stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_structure_factor(h, w, same, nsamples, kx, ky, factor, out,
                                           stream or None), L)


def sz_correlations(configs, nrows: int, ncols: int, window, flags=None, counts=None):
    """Add a batch of device configurations to the equal-spin counts of ``window``
    = (r0, c0, h, w); returns the dict {"same", "n", "window"} (int64 device tensors)."""
    import torch
    r0, c0, h, w = window
    dev = configs.device
    if counts is None:
        counts = dict(same=torch.zeros((h * w, h * w), dtype=torch.int64, device=dev),
                      n=torch.zeros(1, dtype=torch.int64, device=dev), window=tuple(window))
    s = torch.cuda.current_stream(dev)
    pepsgo_sz_counts(nrows, ncols, r0, c0, h, w, configs.shape[0], configs.data_ptr(),
                     flags.data_ptr() if flags is not None else 0, counts["same"].data_ptr(),
                     counts["n"].data_ptr(), s.cuda_stream)
    return counts


def structure_factor(counts, kx: float, ky: float, factor: float = 1.0):
    """factor / N^2 sum_pq <S^z_p S^z_q> cos(k.(r_p - r_q)) over the counted window (device scalar)."""
    import torch
    _, _, h, w = counts["window"]
    dev = counts["same"].device
    out = torch.empty(1, dtype=torch.float64, device=dev)
    pepsgo_structure_factor(h, w, counts["same"].data_ptr(), counts["n"].data_ptr(), kx, ky, factor,
                            out.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    return out


def spin_structure_factor(counts, trans, kx: float, ky: float):
    """m_s^2(k) = 1/N^2 sum_pq <S_p . S_q> cos(k.(r_p - r_q)) over the window, from the
    equal-spin ``counts`` (sz_correlations) and the transverse sums ``trans``
    (Peps.transverse) of the same window (device scalar)."""
    import torch
    _, _, h, w = counts["window"]
    if tuple(trans["window"]) != tuple(counts["window"]):
        raise ValueError("counts and transverse sums of different windows")
    dev = counts["same"].device
    out = torch.empty(1, dtype=torch.float64, device=dev)
    pepsgo_spin_structure_factor(h, w, counts["same"].data_ptr(), counts["n"].data_ptr(),
                                 trans["sums"].data_ptr(), trans["n"].data_ptr(), kx, ky,
                                 out.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    return out


def pepsgo_peps_read(peps: int, tensors: int, on_device: bool, stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_peps_read(peps, tensors, int(on_device), stream or None), L)


def pepsgo_go_accumulate(peps: int, batch: int, configs: int, grad: int, eloc: int, flags: int,
                         sum_delta: int, sum_delta_e: int, stats: int, stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_go_accumulate(peps, batch, configs, grad, eloc, flags, sum_delta,
                                        sum_delta_e, stats, stream or None), L)


def pepsgo_go_update(peps: int, sum_delta: int, sum_delta_e: int, stats: int, dt: float, p: int,
                     stream: int = 0, L=None):
    L = L or lib()
    return check(L.pepsgo_go_update(peps, sum_delta, sum_delta_e, stats, dt, p, stream or None), L)


def pepsgo_graph_create(peps: int, params: EvalParams, batch: int, configs: int, logabs: int,
                        sign: int, eloc: int, flags: int, grad: int, workspace: int,
                        workspace_bytes: int, L=None) -> int:
    L = L or lib()
    h = _vp()
    check(L.pepsgo_graph_create(peps, ctypes.byref(params), batch, configs, logabs, sign, eloc,
                                flags, grad or None, workspace, workspace_bytes, ctypes.byref(h)), L)
    return h.value


def pepsgo_graph_launch(graph: int, stream: int = 0, L=None):
    L = L or lib()
    check(L.pepsgo_graph_launch(graph, stream or None), L)


def pepsgo_graph_free(graph: int, L=None):
    L = L or lib()
    check(L.pepsgo_graph_free(graph), L)


def pepsgo_tune_get(ctx: int, D: int, Dc: int, precision: int, L=None) -> Tuning:
    L = L or lib()
    t = Tuning()
    check(L.pepsgo_tune_get(ctx, D, Dc, precision, ctypes.byref(t)), L)
    return t


def pepsgo_tune_set(ctx: int, D: int, Dc: int, precision: int, t: Tuning | None, L=None):
    L = L or lib()
    check(L.pepsgo_tune_set(ctx, D, Dc, precision, ctypes.byref(t) if t is not None else None), L)


def pepsgo_autotune(peps: int, params: EvalParams, batch: int, configs: int, stream: int = 0,
                    L=None) -> Tuning:
    L = L or lib()
    t = Tuning()
    check(L.pepsgo_autotune(peps, ctypes.byref(params), batch, configs, stream or None,
                            ctypes.byref(t)), L)
    return t


def pepsgo_tune_save(ctx: int, path: str, L=None):
    L = L or lib()
    check(L.pepsgo_tune_save(ctx, path.encode()), L)


def pepsgo_tune_load(ctx: int, path: str, L=None) -> int:
    L = L or lib()
    return check(L.pepsgo_tune_load(ctx, path.encode()), L)


def pepsgo_serve_create(ctx: int, cfg: ServeConfig, L=None) -> int:
    L = L or lib()
    h = _vp()
    check(L.pepsgo_serve_create(ctx, ctypes.byref(cfg), ctypes.byref(h)), L)
    return h.value


def pepsgo_serve_submit(srv: int, peps: int, params: EvalParams, batch: int, configs: int,
                        logabs: int, sign: int, eloc: int, flags: int, grad: int, L=None) -> int:
    L = L or lib()
    rid = ctypes.c_uint64()
    check(L.pepsgo_serve_submit(srv, peps, ctypes.byref(params), batch, configs, logabs, sign,
                                eloc, flags, grad or None, ctypes.byref(rid)), L)
    return rid.value


def pepsgo_serve_poll(srv: int, max_done: int, timeout_us: int, L=None) -> list:
    L = L or lib()
    buf = (ServeDone * max(1, max_done))()
    n = check(L.pepsgo_serve_poll(srv, buf, max_done, timeout_us), L)
    return [buf[k] for k in range(n)]


def pepsgo_serve_pending(srv: int, L=None) -> int:
    L = L or lib()
    n = ctypes.c_int()
    check(L.pepsgo_serve_pending(srv, ctypes.byref(n)), L)
    return n.value


def pepsgo_serve_stats(srv: int, reset: bool = False, L=None) -> ServeStats:
    L = L or lib()
    out = ServeStats()
    check(L.pepsgo_serve_stats(srv, ctypes.byref(out), int(reset)), L)
    return out


PROBES = {"fp64_vector_fma": 0, "fp64_mfma_16x16x4": 1, "fp32_mfma_16x16x4": 2,
          "bf16_mfma_16x16x16": 3}


def pepsgo_peak_probe(kind: int, blocks: int, iters: int, sink: int, stream: int = 0, L=None) -> float:
    """Launch one throughput probe; returns its flop count (time it on `stream`)."""
    L = L or lib()
    flops = ctypes.c_double()
    check(L.pepsgo_peak_probe(kind, blocks, iters, sink, ctypes.byref(flops), stream or None), L)
    return flops.value


def pepsgo_serve_destroy(srv: int, L=None):
    L = L or lib()
    check(L.pepsgo_serve_destroy(srv), L)


# ---- torch convenience layer -----------------------------------------------------------

class Context:
    def __init__(self, device: int = 0):
        self.device = device
        self.handle = pepsgo_create(device)

    def close(self):
        if self.handle:
            pepsgo_destroy(self.handle)
            self.handle = 0


class Peps:
    """A PEPS resident on the device.  ``flat`` is the packed float64 tensor vector."""

    def __init__(self, ctx: Context, N: int, M: int, D: int, flat, d: int = 2):
        import numpy as np
        import torch
        self.ctx, self.N, self.M, self.D, self.d = ctx, N, M, D, d
        if isinstance(flat, torch.Tensor):
            t = flat.detach().to(dtype=torch.float64).contiguous()
            on_dev = t.is_cuda
            keep = t
            addr = t.data_ptr()
        else:
            keep = np.ascontiguousarray(flat, dtype=np.float64)
            on_dev = False
            addr = keep.ctypes.data
        self.handle = pepsgo_peps_load(ctx.handle, N, M, d, D, addr, on_dev)
        self.nparams = int(keep.numel() if on_dev else keep.size)
        del keep
        self.grad_elems, self.grad_offsets = pepsgo_grad_layout(self.handle, N * M)
        self._ws = None
        self._su_ws = None

    def free(self):
        if self.handle:
            pepsgo_peps_free(self.handle)
            self.handle = 0

    def workspace_bytes(self, params: EvalParams, batch: int) -> int:
        return pepsgo_workspace_bytes(self.handle, params, batch)

    def metropolis_step(self, configs, bonds, uniforms, Dc: int, J1: float = 1.0, J2: float = 0.0,
                        precision: int = PEPSGO_FP64, want_grad: bool = False, sums=None,
                        stream=None):
        """One device Metropolis step (one exchange proposal per chain, at the cost of
        one whole evaluation: psi, every Delta and every strip): evaluates ``configs``
        (uint8 device tensor, updated in place) and applies the accepted exchanges.
        ``bonds`` int32 and ``uniforms`` float64 device tensors of length B.  Returns
        (outputs of the states before the move, accepted uint8 tensor).

        ``sums`` (a dict from ``new_sums`` or an earlier call) selects the REDUCED
        gradient mode: the Eq. (3) sums of the states before the move are added to
        it inside the call, before the configurations change, and no per-sample
        Delta is returned.  With ``want_grad`` instead, the returned per-sample Delta
        belong to the configurations as they were before this call: to feed them to
        ``go_accumulate`` pass a copy of ``configs`` taken before the call."""
        import torch
        dev = configs.device
        B = configs.shape[0]
        mode = (PEPSGO_GRAD_REDUCED if sums is not None else
                PEPSGO_GRAD_PER_SAMPLE if want_grad else PEPSGO_GRAD_NONE)
        want_grad = mode == PEPSGO_GRAD_PER_SAMPLE
        params = make_params(Dc, J1, J2, precision, mode, True)
        out = dict(
            logabs=torch.empty(B, dtype=torch.float64, device=dev),
            sign=torch.empty(B, dtype=torch.int8, device=dev),
            eloc=torch.empty(B, dtype=torch.float64, device=dev),
            flags=torch.empty(B, dtype=torch.int32, device=dev),
            grad=torch.empty((B, self.grad_elems) if want_grad else (0,), dtype=torch.float64,
                             device=dev),
        )
        acc = torch.empty(B, dtype=torch.uint8, device=dev)
        nbytes = self.workspace_bytes(params, B)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        gptr = (sums["flat"].data_ptr() if sums is not None else
                out["grad"].data_ptr() if want_grad else 0)
        pepsgo_metropolis_step(self.handle, params, B, configs.data_ptr(), bonds.data_ptr(),
                               uniforms.data_ptr(), acc.data_ptr(), out["logabs"].data_ptr(),
                               out["sign"].data_ptr(), out["eloc"].data_ptr(),
                               out["flags"].data_ptr(), gptr, self._ws.data_ptr(),
                               self._ws.numel(), s.cuda_stream)
        return out, acc

    @property
    def nbonds(self) -> int:
        """Nearest-neighbour bonds of the lattice (proposals of one sweep)."""
        return self.N * (self.M - 1) + (self.N - 1) * self.M

    def metropolis_sweep(self, configs, uniforms, Dc: int, want_ratios: bool = False,
                         stream=None):
        """One Metropolis sweep per chain on the device (every bond once, row by row,
        environments reused; about the cost of one evaluation).  ``configs`` (uint8
        [B, N*M]) are updated in place; ``uniforms`` float64 [B, nbonds].  Returns
        (accepted uint8 [B, nbonds], ratios float64 [B, nbonds] or None)."""
        import torch
        dev = configs.device
        B = configs.shape[0]
        params = make_params(Dc, 1.0, 0.0, PEPSGO_FP64, PEPSGO_GRAD_NONE, True)
        acc = torch.empty((B, self.nbonds), dtype=torch.uint8, device=dev)
        rat = torch.empty((B, self.nbonds), dtype=torch.float64, device=dev) if want_ratios else None
        nbytes = self.workspace_bytes(params, B)
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        pepsgo_metropolis_sweep(self.handle, params, B, configs.data_ptr(), uniforms.data_ptr(),
                                acc.data_ptr(), rat.data_ptr() if want_ratios else 0,
                                self._ws.data_ptr(), self._ws.numel(), s.cuda_stream)
        return acc, rat

    def transverse(self, configs, window, Dc: int, acc=None, want_ratios: bool = False,
                   max_workspace_bytes: int = 0, stream=None):
        """Transverse correlations on ``window`` = (r0, c0, h, w): adds the batch's
        sums of 1/2 [s_p != s_q] W(S^{pq})/W(S) (1/2 on the diagonal) and its
        counted samples to ``acc`` = {"sums" float64 [n, n], "n" int64 [1], "window"}
        (created when None) and returns (acc, flags uint32 [B], ratios float64
        [B, n, n] or None).  ``max_workspace_bytes`` caps the workspace (0: the
        whole batch at once, or 8 GiB, whichever is smaller)."""
        import torch
        dev = configs.device
        B = configs.shape[0]
        r0, c0, h, w = window
        n = h * w
        if acc is None:
            acc = dict(sums=torch.zeros((n, n), dtype=torch.float64, device=dev),
                       n=torch.zeros(1, dtype=torch.int64, device=dev), window=tuple(window))
        params = make_params(Dc, 1.0, 0.0, PEPSGO_FP64, PEPSGO_GRAD_NONE, False)
        per = pepsgo_transverse_workspace_bytes(self.handle, params, r0, c0, h, w, 1)
        cap = max_workspace_bytes or (8 << 30)
        nbytes = max(per, min(per * max(B, 1), cap))
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        flags = torch.empty(B, dtype=torch.int32, device=dev)
        rat = torch.empty((B, n, n), dtype=torch.float64, device=dev) if want_ratios else None
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        pepsgo_transverse(self.handle, params, B, configs.data_ptr(), r0, c0, h, w,
                          rat.data_ptr() if want_ratios else 0, acc["sums"].data_ptr(),
                          acc["n"].data_ptr(), flags.data_ptr(), self._ws.data_ptr(), nbytes,
                          s.cuda_stream)
        return acc, flags, rat

    def new_sums(self, device="cuda"):
        """Zeroed Eq. (3) sums in the layout of the REDUCED gradient mode: one
        float64 buffer ``flat`` of 2 nparams + 3 and its views ``sum_delta``,
        ``sum_delta_e`` and ``stats`` (n, sum E, sum E^2), as go_update takes them."""
        import torch
        flat = torch.zeros(2 * self.nparams + 3, dtype=torch.float64, device=device)
        n = self.nparams
        return dict(flat=flat, sum_delta=flat[:n], sum_delta_e=flat[n:2 * n], stats=flat[2 * n:])

    def update(self, flat, stream=None):
        """Overwrite the device tensors with ``flat`` (a float64 device tensor)."""
        import torch
        t = flat.detach().to(dtype=torch.float64).contiguous()
        s = stream if stream is not None else torch.cuda.current_stream(t.device)
        pepsgo_peps_update(self.handle, t.data_ptr(), True, s.cuda_stream)

    def read(self):
        """The packed float64 tensors as they are on the device now (a device tensor)."""
        import torch
        t = torch.empty(self.nparams, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        pepsgo_peps_read(self.handle, t.data_ptr(), True,
                         torch.cuda.current_stream(t.device).cuda_stream)
        return t

    def su_start(self):
        """A simple-update state (gamma, lambdas) starting from the loaded tensors
        with all bond weights 1 (device tensors)."""
        import torch
        nb = self.N * (self.M - 1) + (self.N - 1) * self.M
        lam = torch.ones(nb * self.D, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        return self.read(), lam

    def su_evolve(self, gamma, lambdas, J1: float, dtau: float, nsteps: int, stream=None):
        """nsteps simple-update steps of exp(-dtau J1 S.S) on (gamma, lambdas) in place."""
        import torch
        nbytes = pepsgo_su_workspace_bytes(self.handle)
        if self._su_ws is None or self._su_ws.numel() < nbytes:
            self._su_ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=gamma.device)
        s = stream if stream is not None else torch.cuda.current_stream(gamma.device)
        pepsgo_su_evolve(self.handle, gamma.data_ptr(), lambdas.data_ptr(), J1, dtau, nsteps,
                         self._su_ws.data_ptr(), self._su_ws.numel(), s.cuda_stream)

    def su_pad(self, gamma, lambdas, target: "Peps", stream=None):
        """This handle's simple-update state at ``target``'s (larger) bond dimension."""
        import torch
        nb = self.N * (self.M - 1) + (self.N - 1) * self.M
        g2 = torch.empty(target.nparams, dtype=torch.float64, device=gamma.device)
        l2 = torch.empty(nb * target.D, dtype=torch.float64, device=gamma.device)
        s = stream if stream is not None else torch.cuda.current_stream(gamma.device)
        pepsgo_su_pad(self.handle, gamma.data_ptr(), lambdas.data_ptr(), target.handle,
                      g2.data_ptr(), l2.data_ptr(), s.cuda_stream)
        return g2, l2

    def su_to_peps(self, gamma, lambdas, stream=None):
        """Load the PEPS represented by (gamma, lambdas) as this handle's tensors."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(gamma.device)
        pepsgo_su_to_peps(self.handle, gamma.data_ptr(), lambdas.data_ptr(), s.cuda_stream)

    def go_accumulate(self, configs, out, sums=None, stream=None):
        """Add one evaluated batch (``out`` from evaluate / metropolis_step with
        per-sample gradients and energies) to the sums of Eq. (3).  ``configs``
        must be the configurations that were evaluated: each sample's Delta goes
        to the slice of its own spins (after a metropolis_step, the copy taken
        before the move; or use metropolis_step(..., sums=...), which sums before
        moving).  ``sums`` is the dict returned by a previous call (or by
        ``new_sums``), or None to start from zero."""
        import torch
        dev = configs.device
        if sums is None:
            sums = dict(sum_delta=torch.zeros(self.nparams, dtype=torch.float64, device=dev),
                        sum_delta_e=torch.zeros(self.nparams, dtype=torch.float64, device=dev),
                        stats=torch.zeros(3, dtype=torch.float64, device=dev))
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        pepsgo_go_accumulate(self.handle, configs.shape[0], configs.data_ptr(),
                             out["grad"].data_ptr(), out["eloc"].data_ptr(),
                             out["flags"].data_ptr(), sums["sum_delta"].data_ptr(),
                             sums["sum_delta_e"].data_ptr(), sums["stats"].data_ptr(),
                             s.cuda_stream)
        return sums

    def go_update(self, sums, dt: float, p, stream=None):
        """Eq. (6) sign step of every tensor element in place; ``p`` is a float64
        device tensor of per-element factors in [0, 1]."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(p.device)
        pepsgo_go_update(self.handle, sums["sum_delta"].data_ptr(), sums["sum_delta_e"].data_ptr(),
                         sums["stats"].data_ptr(), dt, p.data_ptr(), s.cuda_stream)

    def capture(self, configs, Dc: int, J1: float = 1.0, J2: float = 0.0,
                precision: int = PEPSGO_FP64, want_grad: bool = True, want_eloc: bool = True,
                workspace=None, out=None) -> "Graph":
        """Capture evaluate(configs, ...) into a replayable graph over fixed buffers."""
        import torch
        dev = configs.device
        B = configs.shape[0]
        params = make_params(Dc, J1, J2, precision,
                             PEPSGO_GRAD_PER_SAMPLE if want_grad else PEPSGO_GRAD_NONE, want_eloc)
        if out is None:
            out = dict(
                logabs=torch.empty(B, dtype=torch.float64, device=dev),
                sign=torch.empty(B, dtype=torch.int8, device=dev),
                eloc=torch.empty(B, dtype=torch.float64, device=dev),
                flags=torch.empty(B, dtype=torch.int32, device=dev),
                grad=torch.empty((B, self.grad_elems) if want_grad else (0,),
                                 dtype=torch.float64, device=dev),
            )
        if workspace is None:
            workspace = torch.empty(self.workspace_bytes(params, B), dtype=torch.uint8,
                                    device=dev)
        h = pepsgo_graph_create(self.handle, params, B, configs.data_ptr(),
                                out["logabs"].data_ptr(), out["sign"].data_ptr(),
                                out["eloc"].data_ptr(), out["flags"].data_ptr(),
                                out["grad"].data_ptr() if want_grad else 0,
                                workspace.data_ptr(), workspace.numel())
        return Graph(h, configs, out, workspace)

    def autotune(self, configs, Dc: int, J1: float = 1.0, J2: float = 0.0,
                 precision: int = PEPSGO_FP64, want_grad: bool = True, want_eloc: bool = True,
                 stream=None) -> dict:
        """Pick the LDS budgets of this (D, Dc, precision) on a device config batch."""
        import torch
        params = make_params(Dc, J1, J2, precision,
                             PEPSGO_GRAD_PER_SAMPLE if want_grad else PEPSGO_GRAD_NONE, want_eloc)
        s = stream if stream is not None else torch.cuda.current_stream(configs.device)
        t = pepsgo_autotune(self.handle, params, configs.shape[0], configs.data_ptr(), s.cuda_stream)
        self._ws = None
        return t.as_dict()

    def evaluate(self, configs, Dc: int, J1: float = 1.0, J2: float = 0.0,
                 precision: int = PEPSGO_FP64, want_grad: bool = True, want_eloc: bool = True,
                 workspace=None, out=None, stream=None, sums=None):
        """Evaluate a uint8 device tensor [B, N*M]; returns a dict of device tensors.

        With ``sums`` (a dict from ``new_sums``) the gradient mode is REDUCED: the
        Eq. (3) sums of this batch are added to it and ``out["grad"]`` is empty."""
        import torch
        dev = configs.device
        B = configs.shape[0]
        mode = (PEPSGO_GRAD_REDUCED if sums is not None else
                PEPSGO_GRAD_PER_SAMPLE if want_grad else PEPSGO_GRAD_NONE)
        want_grad = mode == PEPSGO_GRAD_PER_SAMPLE
        params = make_params(Dc, J1, J2, precision, mode, want_eloc)
        if out is None:
            out = dict(
                logabs=torch.empty(B, dtype=torch.float64, device=dev),
                sign=torch.empty(B, dtype=torch.int8, device=dev),
                eloc=torch.empty(B, dtype=torch.float64, device=dev),
                flags=torch.empty(B, dtype=torch.int32, device=dev),
                grad=torch.empty((B, self.grad_elems) if want_grad else (0,), dtype=torch.float64,
                                 device=dev),
            )
        if workspace is None:
            nbytes = self.workspace_bytes(params, B)
            if self._ws is None or self._ws.numel() < nbytes:
                self._ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            workspace = self._ws
        s = stream if stream is not None else torch.cuda.current_stream(dev)
        gptr = (sums["flat"].data_ptr() if sums is not None else
                out["grad"].data_ptr() if want_grad else 0)
        pepsgo_evaluate(self.handle, params, B, configs.data_ptr(), out["logabs"].data_ptr(),
                        out["sign"].data_ptr(), out["eloc"].data_ptr(), out["flags"].data_ptr(),
                        gptr, workspace.data_ptr(), workspace.numel(), s.cuda_stream)
        return out


class Graph:
    """A captured evaluation; ``out`` are its fixed output tensors."""

    def __init__(self, handle: int, configs, out: dict, workspace):
        self.handle, self.configs, self.out, self.workspace = handle, configs, out, workspace

    def launch(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.configs.device)
        pepsgo_graph_launch(self.handle, s.cuda_stream)
        return self.out

    def free(self):
        if self.handle:
            pepsgo_graph_free(self.handle)
            self.handle = 0


class Server:
    """Request loop of the library (pepsgo_serve_*): submit batches, poll completions.

    ``submit`` allocates the request's output tensors on the device and keeps
    them (and the configuration tensor) alive until the request is polled.
    """

    def __init__(self, ctx: Context, pool_bytes: int = 0, streams: int = 0, max_chunk: int = 0,
                 min_chunk: int = 0, max_pending: int = 0):
        self.ctx = ctx
        self.handle = pepsgo_serve_create(ctx.handle, ServeConfig(pool_bytes, streams, max_chunk,
                                                                  min_chunk, max_pending))
        self._live = {}

    def submit(self, peps: Peps, configs, Dc: int, J1: float = 1.0, J2: float = 0.0,
               precision: int = PEPSGO_FP64, want_grad: bool = True, want_eloc: bool = True) -> int:
        import torch
        dev = configs.device
        B = configs.shape[0]
        params = make_params(Dc, J1, J2, precision,
                             PEPSGO_GRAD_PER_SAMPLE if want_grad else PEPSGO_GRAD_NONE, want_eloc)
        out = dict(
            logabs=torch.empty(B, dtype=torch.float64, device=dev),
            sign=torch.empty(B, dtype=torch.int8, device=dev),
            eloc=torch.empty(B, dtype=torch.float64, device=dev),
            flags=torch.empty(B, dtype=torch.int32, device=dev),
            grad=torch.empty((B, peps.grad_elems) if want_grad else (0,), dtype=torch.float64,
                             device=dev),
        )
        # the server's streams do not wait for torch's: inputs must be complete
        torch.cuda.current_stream(dev).synchronize()
        rid = pepsgo_serve_submit(self.handle, peps.handle, params, B, configs.data_ptr(),
                                  out["logabs"].data_ptr(), out["sign"].data_ptr(),
                                  out["eloc"].data_ptr(), out["flags"].data_ptr(),
                                  out["grad"].data_ptr() if want_grad else 0)
        self._live[rid] = (configs, out)
        return rid

    def poll(self, timeout_s: float = 0.0, max_done: int = 256):
        """[(ServeDone, outputs)] of requests completed since the last poll."""
        done = pepsgo_serve_poll(self.handle, max_done, int(timeout_s * 1e6))
        return [(d, self._live.pop(d.id)[1]) for d in done]

    def pending(self) -> int:
        return pepsgo_serve_pending(self.handle)

    def stats(self, reset: bool = False) -> dict:
        """Request and sample counts, p50/p99 latency (ms) and samples/s (pepsgo_serve_stats)."""
        return pepsgo_serve_stats(self.handle, reset).as_dict()

    def close(self):
        if self.handle:
            pepsgo_serve_destroy(self.handle)
            self.handle = 0
            self._live.clear()
