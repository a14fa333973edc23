"""ctypes binding of the etdpic C ABI (include/etdpic.h).

Argument marshalling only: every function has the name of the C entry point it
calls, converts numpy arrays and device addresses to pointers, and raises
``EtdpicError`` on a non-zero status.  All computation happens in the HIP
library; if ``libetdpic.so`` is missing, loading fails loudly.
"""
import ctypes
import os

import numpy as np

from . import build as _build

EP_OK, EP_EINVAL, EP_ENOMEM, EP_EHIP, EP_ESTATE, EP_ENOTRAINED, EP_EIO = 0, -1, -2, -3, -4, -5, -6
EP_FIELD_ZERO, EP_FIELD_DUFFING, EP_FIELD_POISSON = 0, 1, 2
EP_DEPOSIT_ATOMIC, EP_DEPOSIT_SORTED = 0, 1
(EP_PUSH_PLAIN, EP_PUSH_LEARNED, EP_PUSH_RK4, EP_PUSH_IMPROVED_ETD, EP_PUSH_CLASSIC_ETD,
 EP_PUSH_MODIFIED_ETD) = 0, 1, 2, 3, 4, 5
EP_MLP_BF16, EP_MLP_FP16 = 0, 1

STATUS_NAMES = {0: "EP_OK", -1: "EP_EINVAL", -2: "EP_ENOMEM", -3: "EP_EHIP", -4: "EP_ESTATE",
                -5: "EP_ENOTRAINED", -6: "EP_EIO"}

# Every symbol include/etdpic.h declares (checked by the CPU test-suite).
EXPORTS = (
    "ep_create", "ep_destroy", "ep_last_error", "ep_set_particles", "ep_bind_particles",
    "ep_step", "ep_moments_get", "ep_get_particles", "ep_get_field", "ep_set_push_mode",
    "ep_sync", "ep_timing_enable", "ep_timing_get", "ep_mlp_set_weights", "ep_mlp_get_weights",
    "ep_mlp_set_projection", "ep_mlp_labels", "ep_mlp_grad", "ep_mlp_train", "ep_mlp_collect",
    "ep_mlp_get_samples",
    "ep_save", "ep_load", "ep_set_fine_solver", "ep_get_periods", "ep_compute_periods",
    "ep_copy_bandwidth", "ep_mlp_set_precision", "ep_step_noalloc",
)


class EtdpicError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))


class ep_config(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_uint64), ("n_cells", ctypes.c_uint32),
                ("substeps", ctypes.c_uint32), ("r_max", ctypes.c_double),
                ("deposit", ctypes.c_int32), ("device", ctypes.c_int32),
                ("hip_stream", ctypes.c_void_p)]


class ep_moments(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("phase", ctypes.c_double), ("charge", ctypes.c_double),
                ("rms_radius", ctypes.c_double), ("energy", ctypes.c_double),
                ("kinetic", ctypes.c_double), ("potential", ctypes.c_double),
                ("n_steps", ctypes.c_uint64), ("n_offmesh", ctypes.c_uint64),
                ("n_nan", ctypes.c_uint64), ("n_fallback", ctypes.c_uint64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ep_train_cfg(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("eps", ctypes.c_double), ("field", ctypes.c_int32),
                ("fine_substeps", ctypes.c_uint32), ("batch", ctypes.c_uint32),
                ("epochs", ctypes.c_uint32), ("lr", ctypes.c_double),
                ("lr_final", ctypes.c_double), ("s_in", ctypes.c_double)]


class ep_train_report(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("loss_first", ctypes.c_double),
                ("loss_last", ctypes.c_double), ("mu_delta", ctypes.c_double),
                ("sig_delta", ctypes.c_double), ("mu_kappa", ctypes.c_double),
                ("sig_kappa", ctypes.c_double), ("label_ms", ctypes.c_double),
                ("train_ms", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None

# The HIP runtime the library is linked against (ROCm's).
ROCM_HIP_RUNTIME = "/opt/rocm/lib/libamdhip64.so.7"
# normalisation of a corrector: s_in, s_t, s_E, mu_d, sig_d, mu_k, sig_k, output
# map, base push substeps
NORM_LEN = 9


def library_path():
    return _build.LIB


def foreign_hip_runtimes(maps="/proc/self/maps"):
    """Paths of HIP runtimes mapped into this process from anywhere but the
    directory of the runtime the library links (e.g. the copy a framework
    wheel bundles).  Two runtimes in one process do not share devices,
    streams or allocations, and a profiler attached to such a process has
    aborted inside its own tool library."""
    own = os.path.dirname(os.path.realpath(ROCM_HIP_RUNTIME))
    found = set()
    try:
        with open(maps) as f:
            for line in f:
                parts = line.split()
                if len(parts) >= 6 and "libamdhip64" in os.path.basename(parts[-1]):
                    found.add(parts[-1])
    except OSError:
        return []
    return sorted(p for p in found if os.path.dirname(os.path.realpath(p)) != own)


def lib():
    """Load libetdpic.so (raises if it has not been built, or if another HIP
    runtime is already loaded into this process)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError("etdpic HIP library not built: %s is missing "
                              "(run __graft_entry__.build())" % path)
        foreign = foreign_hip_runtimes()
        if foreign:
            raise ImportError("another HIP runtime is already loaded in this process (%s); "
                              "libetdpic uses %s and cannot share a process with it -- "
                              "load the library in a process that does not import it"
                              % (", ".join(foreign), ROCM_HIP_RUNTIME))
        L = ctypes.CDLL(path)
        vp, d, u64, u32, i32 = (ctypes.c_void_p, ctypes.c_double, ctypes.c_uint64,
                                ctypes.c_uint32, ctypes.c_int32)
        pd = ctypes.POINTER(ctypes.c_double)
        pf = ctypes.POINTER(ctypes.c_float)
        sigs = {
            "ep_create": ([ctypes.POINTER(ep_config), ctypes.POINTER(vp)], i32),
            "ep_destroy": ([vp], i32),
            "ep_last_error": ([vp], ctypes.c_char_p),
            "ep_set_particles": ([vp, pd, pd, u64, d], i32),
            "ep_bind_particles": ([vp, vp, vp, u64, d], i32),
            "ep_step": ([vp, d, d, i32, u64], i32),
            "ep_moments_get": ([vp, d, i32, ctypes.POINTER(ep_moments)], i32),
            "ep_get_particles": ([vp, pd, pd, u64, u64], i32),
            "ep_get_field": ([vp, pd, pd, pd, pd, u32], i32),
            "ep_set_push_mode": ([vp, i32, d, u32], i32),
            "ep_sync": ([vp], i32),
            "ep_timing_enable": ([vp, i32], i32),
            "ep_timing_get": ([vp, ctypes.c_char_p, pd, ctypes.POINTER(u64)], i32),
            "ep_mlp_set_weights": ([vp, pf, u32, pd], i32),
            "ep_mlp_set_precision": ([vp, i32], i32),
            "ep_mlp_set_projection": ([vp, i32], i32),
            "ep_mlp_get_weights": ([vp, pf, u32, pd], i32),
            "ep_mlp_labels": ([vp, d, d, u32, pd, pd, u64, pf, pf], i32),
            "ep_mlp_grad": ([vp, pf, pf, u32, pf, pd], i32),
            "ep_mlp_train": ([vp, ctypes.POINTER(ep_train_cfg), pd, pd, u64,
                              ctypes.POINTER(ep_train_report)], i32),
            "ep_mlp_collect": ([vp, d, d, u32, u64, u64, i32, ctypes.POINTER(u64)], i32),
            "ep_mlp_get_samples": ([vp, u64, u64, pf, pf], i32),
            "ep_set_fine_solver": ([vp, d, u64, i32], i32),
            "ep_copy_bandwidth": ([i32, u64, i32, pd], i32),
            "ep_compute_periods": ([vp, d, i32, ctypes.POINTER(u64)], i32),
            "ep_get_periods": ([vp, pd, ctypes.POINTER(ctypes.c_int64), u64, u64,
                                ctypes.POINTER(u64)], i32),
            "ep_save": ([vp, ctypes.c_char_p], i32),
            "ep_load": ([vp, ctypes.c_char_p, ctypes.POINTER(u64)], i32),
            "ep_step_noalloc": ([vp, vp, u64, d, u32, d, u32, d, d, i32, u64, pd, i32, vp], i32),
        }
        for name, (args, res) in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(ctx, status):
    if status != EP_OK:
        msg = lib().ep_last_error(ctx)
        raise EtdpicError(status, msg.decode() if msg else "")


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _pf(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def ep_create(n_particles, n_cells=256, substeps=1, r_max=5.0, deposit=EP_DEPOSIT_ATOMIC,
              device=0, hip_stream=None):
    cfg = ep_config(n_particles, n_cells, substeps, r_max, deposit, device, hip_stream)
    out = ctypes.c_void_p()
    _check(None, lib().ep_create(ctypes.byref(cfg), ctypes.byref(out)))
    return out


def ep_destroy(ctx):
    _check(None, lib().ep_destroy(ctx))


def ep_last_error(ctx):
    m = lib().ep_last_error(ctx)
    return m.decode() if m else ""


def ep_set_particles(ctx, R, V, w):
    R = _f64(R)
    V = _f64(V)
    if R.shape != V.shape:
        raise ValueError("R and V must have the same shape")
    _check(ctx, lib().ep_set_particles(ctx, _p(R), _p(V), R.size, float(w)))


def ep_bind_particles(ctx, zR_ptr, zV_ptr, n, w):
    """zR_ptr, zV_ptr: addresses (ints) of caller-owned FP32 device arrays of n
    particles in the rotating frame, allocated through the library's HIP
    runtime (e.g. hipMalloc of ROCM_HIP_RUNTIME)."""
    _check(ctx, lib().ep_bind_particles(ctx, ctypes.c_void_p(int(zR_ptr)),
                                        ctypes.c_void_p(int(zV_ptr)), int(n), float(w)))


def ep_step(ctx, dt, eps, field, n_steps=1):
    _check(ctx, lib().ep_step(ctx, float(dt), float(eps), int(field), int(n_steps)))


def ep_moments_get(ctx, eps, field):
    m = ep_moments()
    _check(ctx, lib().ep_moments_get(ctx, float(eps), int(field), ctypes.byref(m)))
    return m.as_dict()


def ep_get_particles(ctx, count, offset=0):
    R = np.empty(count)
    V = np.empty(count)
    _check(ctx, lib().ep_get_particles(ctx, _p(R), _p(V), int(offset), int(count)))
    return R, V


def ep_get_field(ctx, n_nodes):
    rho = np.empty(n_nodes)
    E = np.empty(n_nodes)
    Psi = np.empty(n_nodes)
    Qb = ctypes.c_double(0.0)
    _check(ctx, lib().ep_get_field(ctx, _p(rho), _p(E), _p(Psi), ctypes.byref(Qb), n_nodes))
    return rho, E, Psi, Qb.value


def ep_set_push_mode(ctx, push, drift_tol=1e-5, fallback_substeps=0):
    _check(ctx, lib().ep_set_push_mode(ctx, int(push), float(drift_tol), int(fallback_substeps)))


def ep_sync(ctx):
    _check(ctx, lib().ep_sync(ctx))


def ep_timing_enable(ctx, on=True):
    """on: False/0 off, True/1 every launch, n > 1 every n-th launch of each kernel."""
    n = (1 if on else 0) if isinstance(on, bool) else int(on)
    _check(ctx, lib().ep_timing_enable(ctx, n))


def ep_timing_get(ctx, kernel):
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_uint64(0)
    _check(ctx, lib().ep_timing_get(ctx, kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def ep_mlp_set_weights(ctx, params, norm):
    params = _f32(params)
    norm = _f64(norm)
    if norm.size == 8:     # no base push
        norm = np.append(norm, 0.0)
    if norm.size != NORM_LEN:
        raise ValueError("norm must hold %d values (or 8: no base push)" % NORM_LEN)
    _check(ctx, lib().ep_mlp_set_weights(ctx, _pf(params), params.size, _p(norm)))


def ep_mlp_set_precision(ctx, precision):
    """Inference operand type: EP_MLP_BF16 (default) or EP_MLP_FP16."""
    _check(ctx, lib().ep_mlp_set_precision(ctx, int(precision)))


def ep_mlp_set_projection(ctx, on=True):
    """Energy projection of the particles that pass the learned push's check."""
    _check(ctx, lib().ep_mlp_set_projection(ctx, 1 if on else 0))


def mlp_n_params(n_in):
    """Parameter count of the n_in -> 64 -> 64 -> 2 corrector."""
    return 64 * n_in + 64 + 64 * 64 + 64 + 2 * 64 + 2


def ep_mlp_get_weights(ctx, n_params):
    params = np.empty(n_params, dtype=np.float32)
    norm = np.empty(NORM_LEN)
    _check(ctx, lib().ep_mlp_get_weights(ctx, _pf(params), n_params, _p(norm)))
    return params, norm


def ep_mlp_labels(ctx, dt, eps, fine_substeps, R, V):
    R = _f64(R)
    V = _f64(V)
    delta = np.empty(R.size, dtype=np.float32)
    kappa = np.empty(R.size, dtype=np.float32)
    _check(ctx, lib().ep_mlp_labels(ctx, float(dt), float(eps), int(fine_substeps), _p(R), _p(V),
                                    R.size, _pf(delta), _pf(kappa)))
    return delta, kappa


def ep_mlp_grad(ctx, X, Y, n_params):
    X = _f32(X)
    Y = _f32(Y)
    grad = np.empty(n_params, dtype=np.float32)
    loss = ctypes.c_double(0.0)
    _check(ctx, lib().ep_mlp_grad(ctx, _pf(X), _pf(Y), X.shape[0], _pf(grad), ctypes.byref(loss)))
    return grad, loss.value


def ep_mlp_train(ctx, R, V, dt, eps, fine_substeps, batch, epochs, lr, lr_final, s_in,
                 field=EP_FIELD_DUFFING):
    """Duffing field: trains on the samples (R, V).  Poisson field: pass
    R = V = None; trains on the set collected with ep_mlp_collect."""
    cfg = ep_train_cfg(dt, eps, field, fine_substeps, batch, epochs, lr, lr_final, s_in)
    rep = ep_train_report()
    if R is None:
        _check(ctx, lib().ep_mlp_train(ctx, ctypes.byref(cfg), None, None, 0, ctypes.byref(rep)))
    else:
        R = _f64(R)
        V = _f64(V)
        _check(ctx, lib().ep_mlp_train(ctx, ctypes.byref(cfg), _p(R), _p(V), R.size,
                                       ctypes.byref(rep)))
    return rep.as_dict()


def ep_mlp_collect(ctx, dt, eps, fine_substeps, first=0, stride=1, reset=False):
    """Appends self-generated Poisson-field samples; returns the set's size."""
    n = ctypes.c_uint64(0)
    _check(ctx, lib().ep_mlp_collect(ctx, float(dt), float(eps), int(fine_substeps), int(first),
                                     int(stride), 1 if reset else 0, ctypes.byref(n)))
    return int(n.value)


def ep_mlp_get_samples(ctx, first, count):
    """Rows [first, first + count) of the collected set: (X [count, 6], Y [count, 2])."""
    X = np.empty((count, 6), dtype=np.float32)
    Y = np.empty((count, 2), dtype=np.float32)
    _check(ctx, lib().ep_mlp_get_samples(ctx, int(first), int(count), _pf(X), _pf(Y)))
    return X, Y


def ep_set_fine_solver(ctx, h_fine=0.0, max_fine=10000, periods_once=True):
    """Fine step of the reference RK4 and improved-ETD modes (<= 0: 2 pi eps/100),
    the period-search bound, and whether Duffing improved-ETD steps reuse the
    periods found once."""
    _check(ctx, lib().ep_set_fine_solver(ctx, float(h_fine), int(max_fine), int(periods_once)))


def ep_copy_bandwidth(n_bytes, reps=10, device=0):
    """GB/s (read + written) of a plain device copy of n_bytes."""
    out = ctypes.c_double(0.0)
    _check(None, lib().ep_copy_bandwidth(int(device), int(n_bytes), int(reps), ctypes.byref(out)))
    return out.value


def ep_compute_periods(ctx, eps, field):
    """Periods of the current state (no step); returns the unresolved count."""
    un = ctypes.c_uint64(0)
    _check(ctx, lib().ep_compute_periods(ctx, float(eps), int(field), ctypes.byref(un)))
    return int(un.value)


def ep_get_periods(ctx, count, offset=0):
    """(T [count] FP64, N [count] int64, n_unresolved) of the last improved-ETD step."""
    T = np.empty(count)
    N = np.empty(count, dtype=np.int64)
    un = ctypes.c_uint64(0)
    _check(ctx, lib().ep_get_periods(ctx, _p(T), N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     int(offset), int(count), ctypes.byref(un)))
    return T, N, int(un.value)


def ep_save(ctx, path):
    _check(ctx, lib().ep_save(ctx, os.fsencode(path)))


def ep_load(ctx, path):
    """Restores a checkpoint; returns the restored particle count."""
    n = ctypes.c_uint64(0)
    _check(ctx, lib().ep_load(ctx, os.fsencode(path), ctypes.byref(n)))
    return int(n.value)


def ep_step_noalloc(zR_ptr, zV_ptr, n, w, dt, eps, field, n_steps, phase, n_cells=256,
                    r_max=5.0, substeps=1, device=0, hip_stream=None):
    """The plain step on caller-owned FP32 device arrays (addresses as ints) at
    the fast phase `phase`, without allocating; returns the phase after the
    steps.  The work is queued on hip_stream (an address, or None)."""
    ph = ctypes.c_double(float(phase))
    _check(None, lib().ep_step_noalloc(ctypes.c_void_p(int(zR_ptr)), ctypes.c_void_p(int(zV_ptr)),
                                       int(n), float(w), int(n_cells), float(r_max),
                                       int(substeps), float(dt), float(eps), int(field),
                                       int(n_steps), ctypes.byref(ph), int(device),
                                       None if hip_stream is None else ctypes.c_void_p(hip_stream)))
    return ph.value
