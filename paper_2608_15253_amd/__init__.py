"""Python binding of libmmx (argument marshalling only).

Every function below calls the C entry point of the same name in
``libmmx.so`` (declared in ``include/mmx.h``); all computation happens in the
library's HIP kernels.  Device arrays are passed as raw pointers, typically
``torch.Tensor.data_ptr()`` of CUDA (HIP) tensors; streams as the integer
handle ``torch.cuda.current_stream().cuda_stream``.

Importing this package loads the library and fails loudly if it is missing:
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch is imported first so that libmmx's libamdhip64.so.7 dependency binds to
# the HIP runtime torch already loaded (same SONAME): one runtime per process,
# so device pointers and streams from torch are valid inside the library.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmmx.so")

MMX_F32, MMX_F64 = 1, 2
MMX_OK = 0
STATUS = {0: "MMX_OK", -1: "MMX_EINVAL", -2: "MMX_ESHAPE", -3: "MMX_EHIP",
          -4: "MMX_ESTATE", -5: "MMX_EUNSUP", -6: "MMX_ENONFINITE", -8: "MMX_EDTMIN"}
MMX_EXCH, MMX_DMI_INTERFACIAL, MMX_ANIS_UNIAXIAL = 1, 2, 4
MMX_ZEEMAN, MMX_DEMAG, MMX_THERMAL = 8, 16, 32
MMX_STT = 64
MMX_DMI_BULK = 128
MMX_ANIS_CUBIC = 256
MMX_RKKY = 512
MMX_ALL_TERMS = 1023
DEFAULT_TERMS = MMX_EXCH | MMX_DMI_INTERFACIAL | MMX_ANIS_UNIAXIAL | MMX_ZEEMAN | MMX_DEMAG


class mmx_group(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("cell", ctypes.c_double * 3),
                ("pbc", ctypes.c_int32 * 3), ("pbc_images", ctypes.c_int32 * 3),
                ("replicas", ctypes.c_int32)]


class mmx_material(ctypes.Structure):
    _fields_ = [("Ms", ctypes.c_double), ("A", ctypes.c_double), ("alpha", ctypes.c_double),
                ("Ku", ctypes.c_double), ("u", ctypes.c_double * 3), ("D", ctypes.c_double)]


class mmx_material_ext(ctypes.Structure):
    _fields_ = [("Kc1", ctypes.c_double), ("Kc2", ctypes.c_double),
                ("c1", ctypes.c_double * 3), ("c2", ctypes.c_double * 3),
                ("Db", ctypes.c_double), ("rkky", ctypes.c_double),
                ("rkky_z", ctypes.c_int32 * 2)]


class mmx_rk_stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("err", ctypes.c_double),
                ("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64)]


class mmx_surrogate_stats(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("err", ctypes.c_double),
                ("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("surrogate_steps", ctypes.c_int64), ("exact_steps", ctypes.c_int64),
                ("gate_checks", ctypes.c_int64), ("gate_failures", ctypes.c_int64),
                ("surrogate_rejected", ctypes.c_int64), ("gate_max_passed", ctypes.c_double)]


class MMXError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} -> {STATUS.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950) first")
_lib = ctypes.CDLL(LIB_PATH)

_P = ctypes.c_void_p
_SIGS = {
    "mmx_create": [ctypes.POINTER(mmx_group), ctypes.c_int32, ctypes.c_int, ctypes.POINTER(_P)],
    "mmx_set_stream": [_P, _P],
    "mmx_set_material": [_P, ctypes.c_int32, ctypes.POINTER(mmx_material)],
    "mmx_set_terms": [_P, ctypes.c_uint32],
    "mmx_set_field": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "mmx_set_thermal": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_uint64)],
    "mmx_build_demag": [_P],
    "mmx_field": [_P, _P, _P, ctypes.c_uint64, ctypes.c_double],
    "mmx_torque": [_P, _P, _P, ctypes.c_uint64, ctypes.c_double],
    "mmx_heun": [_P, _P, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, _P],
    "mmx_depondt": [_P, _P, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, _P],
    "mmx_set_stt": [_P, ctypes.c_int32, _P, _P, ctypes.c_double, ctypes.c_double,
                    ctypes.c_double],
    "mmx_rk4": [_P, _P, ctypes.c_double, ctypes.c_int64],
    "mmx_set_material_ext": [_P, ctypes.c_int32, _P],
    "mmx_set_exchange_cells": [_P, ctypes.c_int32, _P],
    "mmx_set_material_cells": [_P, ctypes.c_int32, _P, _P, _P, _P, _P],
    "mmx_set_precession": [_P, ctypes.c_int32],
    "mmx_relax": [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _P],
    "mmx_depondt_refill": [_P, _P, _P, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64, _P,
                           ctypes.c_int32, _P],
    "mmx_rk45": [_P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                 ctypes.POINTER(ctypes.c_double), ctypes.c_int64, _P, ctypes.c_int64,
                 ctypes.POINTER(mmx_rk_stats)],
    "mmx_sync": [_P],
    "mmx_workspace_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "mmx_bind": [_P, _P, ctypes.c_size_t, _P],
    "mmx_checkpoint": [_P, _P, ctypes.POINTER(ctypes.c_size_t)],
    "mmx_restore": [_P, _P, ctypes.c_size_t],
    "mmx_rk45_resume": [_P, _P, ctypes.c_double, ctypes.c_double, _P, ctypes.c_int64,
                        ctypes.POINTER(mmx_rk_stats)],
    "mmx_rk45_dts": [_P, ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                     ctypes.POINTER(ctypes.c_int64)],
    "mmx_energy": [_P, _P, _P],
    "mmx_topological_charge": [_P, _P, _P],
    "mmx_topological_charge_noalloc": [_P, _P, _P],
    "mmx_fno_create": [ctypes.c_int32] * 9 + [ctypes.POINTER(_P)],
    "mmx_fno_set_stream": [_P, _P],
    "mmx_fno_param_count": [_P, ctypes.POINTER(ctypes.c_int64)],
    "mmx_fno_init": [_P, _P, ctypes.c_uint64],
    "mmx_fno_forward": [_P, _P, _P, _P, ctypes.c_int32],
    "mmx_fno_backward": [_P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_double)],
    "mmx_fno_adam": [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int64],
    "mmx_rk45_surrogate": [_P, _P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(ctypes.c_double), ctypes.c_int64,
                           ctypes.POINTER(mmx_surrogate_stats)],
    "mmx_set_path": [_P, ctypes.c_int32],
    "mmx_set_tiles": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "mmx_get_tiles": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "mmx_autotune": [_P],
    "mmx_profile_enable": [_P, ctypes.c_int32],
    "mmx_profile_get": [_P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                        ctypes.POINTER(ctypes.c_int32)],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.mmx_destroy.argtypes = [_P]
_lib.mmx_destroy.restype = None
_lib.mmx_fno_destroy.argtypes = [_P]
_lib.mmx_fno_destroy.restype = None
_lib.mmx_last_error.argtypes = []
_lib.mmx_last_error.restype = ctypes.c_char_p

EXPORTED = list(_SIGS) + ["mmx_destroy", "mmx_last_error", "mmx_fno_destroy"]


def mmx_last_error() -> str:
    return _lib.mmx_last_error().decode()


def _check(fn, status):
    if status != MMX_OK:
        raise MMXError(fn, status, mmx_last_error())


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, (int, np.integer)):
        return int(x)
    return x.data_ptr()


def _dbl(seq):
    arr = (ctypes.c_double * len(seq))(*[float(v) for v in seq])
    return arr


def make_group(n, cell, pbc=(0, 0, 0), images=(0, 0, 0), replicas=1) -> mmx_group:
    g = mmx_group()
    g.n[:] = [int(v) for v in n]
    g.cell[:] = [float(v) for v in cell]
    g.pbc[:] = [int(v) for v in pbc]
    g.pbc_images[:] = [int(v) for v in images]
    g.replicas = int(replicas)
    return g


def mmx_create(groups, prec) -> int:
    arr = (mmx_group * len(groups))(*groups)
    out = _P()
    _check("mmx_create", _lib.mmx_create(arr, len(groups), int(prec), ctypes.byref(out)))
    return out.value


def mmx_destroy(ctx) -> None:
    _lib.mmx_destroy(ctx)


def mmx_set_stream(ctx, stream) -> None:
    _check("mmx_set_stream", _lib.mmx_set_stream(ctx, stream))


def mmx_set_material(ctx, group, Ms, A, alpha, Ku=0.0, u=(0.0, 0.0, 1.0), D=0.0) -> None:
    m = mmx_material(Ms, A, alpha, Ku, (ctypes.c_double * 3)(*u), D)
    _check("mmx_set_material", _lib.mmx_set_material(ctx, group, ctypes.byref(m)))


def mmx_set_terms(ctx, mask) -> None:
    _check("mmx_set_terms", _lib.mmx_set_terms(ctx, int(mask)))


def mmx_set_field(ctx, group, B) -> None:
    _check("mmx_set_field", _lib.mmx_set_field(ctx, group, _dbl(B)))


def mmx_set_thermal(ctx, group, T_per_replica, seeds) -> None:
    n = len(T_per_replica)
    Ta = (ctypes.c_double * n)(*[float(v) for v in T_per_replica])
    Sa = (ctypes.c_uint64 * n)(*[int(v) for v in seeds])
    _check("mmx_set_thermal", _lib.mmx_set_thermal(ctx, group, Ta, Sa))


def mmx_build_demag(ctx) -> None:
    _check("mmx_build_demag", _lib.mmx_build_demag(ctx))


def mmx_field(ctx, m, H, step=0, dt=0.0) -> None:
    _check("mmx_field", _lib.mmx_field(ctx, _ptr(m), _ptr(H), int(step), float(dt)))


def mmx_torque(ctx, m, dmdt, step=0, dt=0.0) -> None:
    _check("mmx_torque", _lib.mmx_torque(ctx, _ptr(m), _ptr(dmdt), int(step), float(dt)))


def mmx_heun(ctx, m, dt, n_steps, step0=0, t_switch=None) -> None:
    _check("mmx_heun", _lib.mmx_heun(ctx, _ptr(m), float(dt), int(n_steps), int(step0),
                                     _ptr(t_switch)))


def mmx_set_stt(ctx, group, J, p=(0.0, 0.0, 1.0), P=0.0, Lambda=1.0, eps_prime=0.0) -> None:
    Ja = np.ascontiguousarray(np.asarray(J, dtype=np.float64).ravel())
    pa = (ctypes.c_double * 3)(*[float(x) for x in p])
    _check("mmx_set_stt", _lib.mmx_set_stt(ctx, int(group),
                                           Ja.ctypes.data_as(ctypes.c_void_p), pa, float(P),
                                           float(Lambda), float(eps_prime)))


def mmx_set_material_ext(ctx, group, Kc1=0.0, Kc2=0.0, c1=(1.0, 0.0, 0.0), c2=(0.0, 1.0, 0.0),
                         Db=0.0, rkky=0.0, rkky_z=(0, 1)) -> None:
    e = mmx_material_ext(float(Kc1), float(Kc2), (ctypes.c_double * 3)(*map(float, c1)),
                         (ctypes.c_double * 3)(*map(float, c2)), float(Db), float(rkky),
                         (ctypes.c_int32 * 2)(*map(int, rkky_z)))
    _check("mmx_set_material_ext", _lib.mmx_set_material_ext(ctx, int(group), ctypes.byref(e)))


def mmx_set_exchange_cells(ctx, group, A) -> None:
    """A: per-cell stiffness array (nz, ny, nx) or None."""
    if A is None:
        _check("mmx_set_exchange_cells", _lib.mmx_set_exchange_cells(ctx, int(group), None))
        return
    Aa = np.ascontiguousarray(np.asarray(A, dtype=np.float64).ravel())
    _check("mmx_set_exchange_cells", _lib.mmx_set_exchange_cells(
        ctx, int(group), Aa.ctypes.data_as(ctypes.c_void_p)))


def mmx_set_material_cells(ctx, group, Ms=None, A=None, alpha=None, Ku=None, D=None) -> None:
    """Per-cell Ms, A, alpha, Ku, D of a group: device tensors of the context's
    element type with one value per cell (None: uniform)."""
    _check("mmx_set_material_cells",
           _lib.mmx_set_material_cells(ctx, int(group), _ptr(Ms), _ptr(A), _ptr(alpha),
                                       _ptr(Ku), _ptr(D)))


def mmx_rk4(ctx, m, dt, n_steps) -> None:
    _check("mmx_rk4", _lib.mmx_rk4(ctx, _ptr(m), float(dt), int(n_steps)))


def mmx_set_precession(ctx, on) -> None:
    _check("mmx_set_precession", _lib.mmx_set_precession(ctx, int(bool(on))))


def mmx_relax(ctx, m, torque_tol, t_max, tol=1e-6):
    """Returns (stats, final max |dm/dt|)."""
    st = mmx_rk_stats()
    tq = ctypes.c_double(0.0)
    _check("mmx_relax", _lib.mmx_relax(ctx, _ptr(m), float(torque_tol), float(t_max), float(tol),
                                       ctypes.byref(st), ctypes.byref(tq)))
    return st, tq.value


def mmx_depondt(ctx, m, dt, n_steps, step0=0, t_switch=None) -> None:
    _check("mmx_depondt", _lib.mmx_depondt(ctx, _ptr(m), float(dt), int(n_steps), int(step0),
                                           _ptr(t_switch)))


def mmx_depondt_refill(ctx, m, m_init, dt, n_steps, times, cap, counts, step0=0) -> None:
    _check("mmx_depondt_refill",
           _lib.mmx_depondt_refill(ctx, _ptr(m), _ptr(m_init), float(dt), int(n_steps),
                                   int(step0), _ptr(times), int(cap), _ptr(counts)))


def mmx_rk45(ctx, m, t0, t_end, tol, dt0=1e-14, dt_replay=None, energy_trace=None,
             trace_cap=0) -> mmx_rk_stats:
    st = mmx_rk_stats()
    rp = _dbl(dt_replay) if dt_replay is not None else None
    nrp = len(dt_replay) if dt_replay is not None else 0
    _check("mmx_rk45", _lib.mmx_rk45(ctx, _ptr(m), float(t0), float(t_end), float(tol),
                                     float(dt0), rp, nrp, _ptr(energy_trace), int(trace_cap),
                                     ctypes.byref(st)))
    return st


def mmx_rk45_surrogate(ctx, net, params, m, t0, t_end, tol, dt0=1e-14, gate_tol=1e-3,
                       residual_mz=True, exact_after_fail=10, gate_cap=0):
    """RK45 whose stages 2-6 use the network's demag field, gated at every
    accepted step by the exact field; returns (stats, gate errors list)."""
    st = mmx_surrogate_stats()
    log = (ctypes.c_double * max(int(gate_cap), 1))()
    _check("mmx_rk45_surrogate",
           _lib.mmx_rk45_surrogate(ctx, net, _ptr(params), _ptr(m), float(t0), float(t_end),
                                   float(tol), float(dt0), float(gate_tol), int(bool(residual_mz)),
                                   int(exact_after_fail), log if gate_cap else None,
                                   int(gate_cap), ctypes.byref(st)))
    n = min(int(gate_cap), st.gate_checks)
    return st, [log[i] for i in range(n)]


def mmx_sync(ctx) -> None:
    """Synchronise the bound stream; raises MMXError (MMX_ENONFINITE) if a
    non-finite state was produced since the last check."""
    _check("mmx_sync", _lib.mmx_sync(ctx))


def mmx_workspace_bytes(ctx) -> int:
    n = ctypes.c_size_t()
    _check("mmx_workspace_bytes", _lib.mmx_workspace_bytes(ctx, ctypes.byref(n)))
    return n.value


def mmx_bind(ctx, workspace, stream) -> None:
    """Move the context's device workspace into ``workspace`` (a device tensor
    of at least mmx_workspace_bytes bytes, or None for a library allocation)
    and bind ``stream``."""
    nbytes = 0 if workspace is None else workspace.numel() * workspace.element_size()
    _check("mmx_bind", _lib.mmx_bind(ctx, _ptr(workspace), nbytes, stream))


def mmx_checkpoint(ctx) -> bytes:
    n = ctypes.c_size_t()
    _check("mmx_checkpoint", _lib.mmx_checkpoint(ctx, None, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check("mmx_checkpoint", _lib.mmx_checkpoint(ctx, buf, ctypes.byref(n)))
    return buf.raw[:n.value]


def mmx_restore(ctx, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check("mmx_restore", _lib.mmx_restore(ctx, buf, len(blob)))


def mmx_rk45_resume(ctx, m, t_end, tol, energy_trace=None, trace_cap=0) -> mmx_rk_stats:
    st = mmx_rk_stats()
    _check("mmx_rk45_resume", _lib.mmx_rk45_resume(ctx, _ptr(m), float(t_end), float(tol),
                                                   _ptr(energy_trace), int(trace_cap),
                                                   ctypes.byref(st)))
    return st


def mmx_rk45_dts(ctx, cap=None):
    count = ctypes.c_int64()
    _check("mmx_rk45_dts", _lib.mmx_rk45_dts(ctx, None, 0, ctypes.byref(count)))
    n = count.value if cap is None else min(cap, count.value)
    buf = (ctypes.c_double * max(n, 1))()
    _check("mmx_rk45_dts", _lib.mmx_rk45_dts(ctx, buf, n, ctypes.byref(count)))
    return [buf[i] for i in range(n)]


def mmx_energy(ctx, m, E) -> None:
    _check("mmx_energy", _lib.mmx_energy(ctx, _ptr(m), _ptr(E)))


def mmx_topological_charge(ctx, m, Q) -> None:
    _check("mmx_topological_charge", _lib.mmx_topological_charge(ctx, _ptr(m), _ptr(Q)))


MMX_PATH_AUTO, MMX_PATH_STAGED, MMX_PATH_FUSED = 0, 1, 2


def mmx_topological_charge_noalloc(ctx, m, Q) -> None:
    """Topological charges with the library's static scratch (no allocation,
    no synchronisation)."""
    _check("mmx_topological_charge_noalloc",
           _lib.mmx_topological_charge_noalloc(ctx, _ptr(m), _ptr(Q)))


def mmx_set_path(ctx, path) -> None:
    _check("mmx_set_path", _lib.mmx_set_path(ctx, int(path)))


def mmx_set_tiles(ctx, group, tiles) -> None:
    arr = (ctypes.c_int32 * 3)(*[int(v) for v in tiles])
    _check("mmx_set_tiles", _lib.mmx_set_tiles(ctx, group, arr))


def mmx_get_tiles(ctx, group) -> tuple:
    arr = (ctypes.c_int32 * 3)()
    _check("mmx_get_tiles", _lib.mmx_get_tiles(ctx, group, arr))
    return tuple(arr)


def mmx_autotune(ctx) -> None:
    _check("mmx_autotune", _lib.mmx_autotune(ctx))


def mmx_profile_enable(ctx, on) -> None:
    _check("mmx_profile_enable", _lib.mmx_profile_enable(ctx, 1 if on else 0))


def mmx_profile_get(ctx) -> dict:
    """{kernel name: (total ms, launches)} of the events recorded so far."""
    n = ctypes.c_int32()
    _check("mmx_profile_get", _lib.mmx_profile_get(ctx, -1, None, 0, None, None,
                                                   ctypes.byref(n)))
    out = {}
    for i in range(n.value):
        name = ctypes.create_string_buffer(64)
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check("mmx_profile_get", _lib.mmx_profile_get(ctx, i, name, 64, ctypes.byref(ms),
                                                       ctypes.byref(cnt), ctypes.byref(n)))
        out[name.value.decode()] = (ms.value, cnt.value)
    return out


# --------------------------------------------------------------------------
# learned demag surrogate
# --------------------------------------------------------------------------
def mmx_fno_create(H, W, C=32, M1=12, M2=12, L=4, Cp=128, batch_max=32, use_mfma=True) -> int:
    out = _P()
    _check("mmx_fno_create", _lib.mmx_fno_create(H, W, C, M1, M2, L, Cp, batch_max,
                                                 1 if use_mfma else 0, ctypes.byref(out)))
    return out.value


def mmx_fno_destroy(f) -> None:
    _lib.mmx_fno_destroy(f)


def mmx_fno_set_stream(f, stream) -> None:
    _check("mmx_fno_set_stream", _lib.mmx_fno_set_stream(f, stream))


def mmx_fno_param_count(f) -> int:
    n = ctypes.c_int64()
    _check("mmx_fno_param_count", _lib.mmx_fno_param_count(f, ctypes.byref(n)))
    return n.value


def mmx_fno_init(f, params, seed) -> None:
    _check("mmx_fno_init", _lib.mmx_fno_init(f, _ptr(params), int(seed)))


def mmx_fno_forward(f, params, m, h, batch) -> None:
    _check("mmx_fno_forward", _lib.mmx_fno_forward(f, _ptr(params), _ptr(m), _ptr(h), int(batch)))


def mmx_fno_backward(f, params, h, target, grads, want_loss=True):
    """Gradients of the last forward; returns the loss (synchronous) or None."""
    loss = ctypes.c_double()
    _check("mmx_fno_backward", _lib.mmx_fno_backward(f, _ptr(params), _ptr(h), _ptr(target),
                                                     _ptr(grads),
                                                     ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def mmx_fno_adam(f, params, grads, moments, lr, t) -> None:
    _check("mmx_fno_adam", _lib.mmx_fno_adam(f, _ptr(params), _ptr(grads), _ptr(moments),
                                             float(lr), int(t)))
