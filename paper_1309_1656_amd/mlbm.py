"""ctypes binding of libmlbm.so: the C ABI of include/mlbm.h with the same names.

Argument marshalling only.  Fields and per-cell arrays are torch tensors in
device memory (contiguous, on the current device); this module checks their
dtype, size and placement and passes raw pointers and the current torch
stream.  All computation happens in the library's HIP kernels.  If the
library has not been built, the first call raises.
"""
import ctypes
import os

import numpy as np

MLBM_D2Q9, MLBM_D3Q19 = 9, 19
MLBM_STORE_F64, MLBM_STORE_F32, MLBM_STORE_F16DEV = 0, 1, 2
MLBM_EQ_DIRECT, MLBM_EQ_EIGEN, MLBM_EQ_ISOTHERMAL = 0, 1, 2
MLBM_ORDER_AUTO, MLBM_ORDER_NATURAL, MLBM_ORDER_XCD_RANGE, MLBM_ORDER_INTERLEAVE8 = -1, 0, 1, 2
MLBM_ADJ_AUTO, MLBM_ADJ_CHANNEL, MLBM_ADJ_CELL = 0, 1, 2
MLBM_OK, MLBM_EINVAL, MLBM_EDOMAIN, MLBM_EHIP, MLBM_ENOMEM, MLBM_ENONFINITE, MLBM_ENOCONV = 0, -1, -2, -3, -4, -5, -6

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmlbm.so")

EXPORTS = (
    "mlbm_create", "mlbm_destroy", "mlbm_get_info", "mlbm_field_bytes", "mlbm_set_tau", "mlbm_set_eq_mode",
    "mlbm_init_equilibrium", "mlbm_step", "mlbm_collide", "mlbm_stream", "mlbm_moments", "mlbm_spin_loss",
    "mlbm_adjoint_step", "mlbm_adjoint_segment", "mlbm_step_states", "mlbm_adjoint_sweep", "mlbm_set_f16_reference", "mlbm_set_launch",
    "mlbm_set_magnetic_field", "mlbm_set_magnetic_field_map", "mlbm_init_chemical", "mlbm_relaxation", "mlbm_set_positivity",
    "mlbm_device_copy", "mlbm_set_store_policy", "mlbm_set_adjoint_launch", "mlbm_moments_noalloc",
    "mlbm_step_post", "mlbm_adjoint_sweep_post", "mlbm_last_error",
)


class MlbmError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"mlbm status {code}: {message}")
        self.code = code


class Info(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int), ("d", ctypes.c_int), ("storage", ctypes.c_int), ("eq_mode", ctypes.c_int),
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64), ("ncell", ctypes.c_int64),
        ("tau", ctypes.c_double), ("omega", ctypes.c_double), ("beta0", ctypes.c_double),
        ("xi", ctypes.c_double), ("a", ctypes.c_double),
        ("w", ctypes.c_double * 19), ("c", (ctypes.c_int * 3) * 19),
        ("a1_0", ctypes.c_double), ("a1_b", ctypes.c_double), ("a2_0", ctypes.c_double),
        ("a2_b", ctypes.c_double), ("a3", ctypes.c_double), ("a4", ctypes.c_double), ("a5", ctypes.c_double),
        ("launch_block_x", ctypes.c_int), ("launch_order", ctypes.c_int),
        ("f16_scale", ctypes.c_double), ("f16_ref", (ctypes.c_double * 19) * 4),
        ("launch_blocks_per_cu", ctypes.c_int), ("launch_temporal_stores", ctypes.c_int),
        ("adjoint_form", ctypes.c_int), ("adjoint_block_x", ctypes.c_int), ("adjoint_order", ctypes.c_int),
        ("adjoint_blocks_per_cu", ctypes.c_int), ("adjoint_temporal_stores", ctypes.c_int),
    ]


_lib_handle = None


def load_library(path=LIB_PATH):
    """Load libmlbm.so once and declare its signatures."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1309_1656_amd.build`")
    # torch ships its own HIP runtime under another file name (same soname).
    # Loaded first, it is the runtime the library binds to; loaded after the
    # library, it would be a second HIP runtime in the process, and one of the
    # two then finds no device.  So torch's runtime goes in first.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
    sig = {
        "mlbm_create": ([ctypes.POINTER(vp), ctypes.c_int, i64p, ctypes.c_double, ctypes.c_double, ctypes.c_int], ctypes.c_int),
        "mlbm_destroy": ([vp], None),
        "mlbm_get_info": ([vp, ctypes.POINTER(Info)], ctypes.c_int),
        "mlbm_field_bytes": ([vp, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "mlbm_set_tau": ([vp, ctypes.c_double], ctypes.c_int),
        "mlbm_set_eq_mode": ([vp, ctypes.c_int], ctypes.c_int),
        "mlbm_init_equilibrium": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_step": ([vp, vp, vp, ctypes.c_int, vp], ctypes.c_int),
        "mlbm_collide": ([vp, vp, vp, vp], ctypes.c_int),
        "mlbm_stream": ([vp, vp, vp, vp], ctypes.c_int),
        "mlbm_moments": ([vp, vp, vp, vp, vp, dp, i64p, vp], ctypes.c_int),
        "mlbm_moments_noalloc": ([vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_spin_loss": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_adjoint_step": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_adjoint_segment": ([vp, vp, vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_adjoint_sweep": ([vp, vp, vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_step_states": ([vp, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp], ctypes.c_int),
        "mlbm_step_post": ([vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, vp], ctypes.c_int),
        "mlbm_adjoint_sweep_post": ([vp, vp, vp, ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_set_f16_reference": ([vp, dp, ctypes.c_double], ctypes.c_int),
        "mlbm_set_launch": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "mlbm_set_magnetic_field": ([vp, dp], ctypes.c_int),
        "mlbm_set_magnetic_field_map": ([vp, vp], ctypes.c_int),
        "mlbm_init_chemical": ([vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "mlbm_relaxation": ([vp, vp, dp, vp], ctypes.c_int),
        "mlbm_set_positivity": ([vp, ctypes.c_int], ctypes.c_int),
        "mlbm_device_copy": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "mlbm_set_store_policy": ([vp, ctypes.c_int], ctypes.c_int),
        "mlbm_set_adjoint_launch": ([vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int],
                                    ctypes.c_int),
        "mlbm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib_handle = lib
    return lib


def mlbm_last_error():
    return load_library().mlbm_last_error().decode()


def _check(code):
    if code != MLBM_OK:
        raise MlbmError(code, mlbm_last_error())


class Handle:
    """Owns one mlbm_handle; destroyed with the object."""

    def __init__(self, ptr, info):
        self._ptr = ptr
        self.info = info

    @property
    def ptr(self):
        if self._ptr is None:
            raise MlbmError(MLBM_EINVAL, "handle already destroyed")
        return self._ptr

    def destroy(self):
        if self._ptr is not None:
            load_library().mlbm_destroy(self._ptr)
            self._ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    # field geometry -------------------------------------------------------
    @property
    def Q(self):
        return self.info["lattice"]

    @property
    def grid(self):
        i = self.info
        return (i["ny"], i["nx"]) if i["d"] == 2 else (i["nz"], i["ny"], i["nx"])

    @property
    def field_shape(self):
        """Library layout: [ny, 4, Q, nx] (2D) or [nz, ny, 4, Q, nx] (3D)."""
        i = self.info
        if i["d"] == 2:
            return (i["ny"], 4, self.Q, i["nx"])
        return (i["nz"], i["ny"], 4, self.Q, i["nx"])

    @property
    def field_dtype(self):
        import torch
        return {MLBM_STORE_F64: torch.float64, MLBM_STORE_F32: torch.float32,
                MLBM_STORE_F16DEV: torch.float16}[self.info["storage"]]

    def empty_field(self, device="cuda"):
        import torch
        return torch.empty(self.field_shape, dtype=self.field_dtype, device=device)

    def pauli_view(self, W):
        """View of a field as [4, Q, *grid] (Pauli component, velocity, cells); no copy."""
        return W.permute(1, 2, 0, 3) if self.info["d"] == 2 else W.permute(2, 3, 0, 1, 4)

    def field_from_pauli(self, a, device="cuda"):
        """Contiguous field in the library layout from values shaped [4, Q, *grid]."""
        import torch
        t = torch.as_tensor(a)
        t = t.permute(2, 0, 1, 3) if self.info["d"] == 2 else t.permute(2, 3, 0, 1, 4)
        return t.to(device=device, dtype=self.field_dtype).contiguous()


def _info_dict(h_ptr):
    info = Info()
    _check(load_library().mlbm_get_info(h_ptr, ctypes.byref(info)))
    Q = info.lattice
    out = {f: getattr(info, f) for f, _ in Info._fields_ if f not in ("w", "c", "f16_ref")}
    out["w"] = np.array(info.w[:Q])
    out["c"] = np.array([[info.c[i][a] for a in range(3)] for i in range(Q)], dtype=np.int64)
    out["f16_ref"] = np.array([[info.f16_ref[k][i] for i in range(Q)] for k in range(4)])
    return out


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))


def _dev_ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise MlbmError(MLBM_EINVAL, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise MlbmError(MLBM_EINVAL, f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise MlbmError(MLBM_EINVAL, f"{name} has dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise MlbmError(MLBM_EINVAL, f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _field_ptr(h, t, name):
    return _dev_ptr(t, h.field_dtype, 4 * h.Q * h.info["ncell"], name)


def _f64_ptr(h, t, rows, name):
    import torch
    return _dev_ptr(t, torch.float64, None if t is None else rows * h.info["ncell"], name)


# ---- the C ABI, one wrapper per entry point -----------------------------------

def mlbm_create(lattice, dims, tau, beta0=1.0, storage=MLBM_STORE_F64):
    """dims = (nx, ny, nz); nz = 1 for D2Q9."""
    lib = load_library()
    ptr = ctypes.c_void_p()
    d = (ctypes.c_int64 * 3)(*[int(v) for v in dims])
    _check(lib.mlbm_create(ctypes.byref(ptr), int(lattice), d, float(tau), float(beta0), int(storage)))
    return Handle(ptr, _info_dict(ptr))


def mlbm_destroy(h):
    h.destroy()


def mlbm_get_info(h):
    h.info = _info_dict(h.ptr)
    return h.info


def mlbm_field_bytes(h):
    n = ctypes.c_size_t()
    _check(load_library().mlbm_field_bytes(h.ptr, ctypes.byref(n)))
    return n.value


def mlbm_set_tau(h, tau):
    _check(load_library().mlbm_set_tau(h.ptr, float(tau)))
    mlbm_get_info(h)


def mlbm_set_eq_mode(h, mode):
    _check(load_library().mlbm_set_eq_mode(h.ptr, int(mode)))
    mlbm_get_info(h)


def mlbm_init_equilibrium(h, W, rho4, u, T, stream=None):
    d = h.info["d"]
    _check(load_library().mlbm_init_equilibrium(
        h.ptr, _field_ptr(h, W, "W"), _f64_ptr(h, rho4, 4, "rho4"), _f64_ptr(h, u, d, "u"),
        _f64_ptr(h, T, 1, "T"), _stream_ptr(stream)))
    mlbm_get_info(h)


def mlbm_init_chemical(h, W, nu, u, T, axis=None, stream=None):
    """Equilibrium from nu = beta mu per spin channel ([2, *grid]) and an optional spin axis ([3, *grid])."""
    d = h.info["d"]
    _check(load_library().mlbm_init_chemical(
        h.ptr, _field_ptr(h, W, "W"), _f64_ptr(h, nu, 2, "nu"), _f64_ptr(h, axis, 3, "axis"),
        _f64_ptr(h, u, d, "u"), _f64_ptr(h, T, 1, "T"), _stream_ptr(stream)))
    mlbm_get_info(h)


def mlbm_step(h, W, scratch, nsteps, stream=None):
    _check(load_library().mlbm_step(h.ptr, _field_ptr(h, W, "W"), _field_ptr(h, scratch, "scratch"),
                                    int(nsteps), _stream_ptr(stream)))


def _states_ptr(h, states, nfields, what):
    """Device pointer of a contiguous tensor holding at least nfields fields (None when nfields <= 0)."""
    if nfields <= 0 and states is None:
        return None
    need = nfields * 4 * h.Q * h.info["ncell"]
    if states is None or states.dtype != h.field_dtype or states.numel() < need or not states.is_contiguous():
        raise MlbmError(MLBM_EINVAL, f"{what} must hold {nfields} contiguous fields")
    return _dev_ptr(states, name=what)


def mlbm_step_states(h, src, dst, states, nsteps, nstates=None, stream=None):
    """Out-of-place steps keeping the post-collision states: step j's goes to field j mod nstates of
    `states` (default nstates: the number of fields the tensor holds)."""
    if nstates is None:
        nstates = 0 if states is None else states.numel() // (4 * h.Q * h.info["ncell"])
    _check(load_library().mlbm_step_states(
        h.ptr, _field_ptr(h, src, "src"), _field_ptr(h, dst, "dst"),
        _states_ptr(h, states, nstates if nsteps > 0 else 0, "states"), int(nstates), int(nsteps),
        _stream_ptr(stream)))


def mlbm_step_post(h, src, nsteps, states=None, dst=None, src_post=False, nstates=None, stream=None):
    """Steps keeping post-collision states only: step j's state goes to field j mod nstates of `states`
    (default nstates: the number of fields the tensor holds), the last one to dst when given."""
    kept = nsteps - (1 if dst is not None else 0)
    if nstates is None:
        nstates = 0 if states is None else states.numel() // (4 * h.Q * h.info["ncell"])
    _check(load_library().mlbm_step_post(
        h.ptr, _field_ptr(h, src, "src"), int(bool(src_post)), None if dst is None else _field_ptr(h, dst, "dst"),
        _states_ptr(h, states, min(max(kept, 0), nstates), "states"), int(nstates), int(nsteps),
        _stream_ptr(stream)))


def mlbm_collide(h, src, dst, stream=None):
    _check(load_library().mlbm_collide(h.ptr, _field_ptr(h, src, "src"), _field_ptr(h, dst, "dst"),
                                       _stream_ptr(stream)))


def mlbm_stream(h, src, dst, stream=None):
    _check(load_library().mlbm_stream(h.ptr, _field_ptr(h, src, "src"), _field_ptr(h, dst, "dst"),
                                      _stream_ptr(stream)))


def mlbm_moments(h, W, rho4=None, u=None, eps=None, host=True, stream=None):
    """Returns (global8 as numpy array, n_neg_eig) when host=True, else None.

    Raises MlbmError(MLBM_ENONFINITE) when the field holds NaN or infinity.
    """
    g = (ctypes.c_double * 8)()
    nneg = ctypes.c_int64()
    _check(load_library().mlbm_moments(
        h.ptr, _field_ptr(h, W, "W"), _f64_ptr(h, rho4, 4, "rho4"), _f64_ptr(h, u, h.info["d"], "u"),
        _f64_ptr(h, eps, 1, "eps"), g if host else None, ctypes.byref(nneg) if host else None,
        _stream_ptr(stream)))
    if host:
        return np.array(g[:]), int(nneg.value)
    return None


def mlbm_moments_noalloc(h, W, rho4=None, u=None, eps=None, sums=None, stream=None):
    """mlbm_moments without allocation or synchronisation; sums: float64 device tensor of 10 values or None."""
    import torch
    _check(load_library().mlbm_moments_noalloc(
        h.ptr, _field_ptr(h, W, "W"), _f64_ptr(h, rho4, 4, "rho4"), _f64_ptr(h, u, h.info["d"], "u"),
        _f64_ptr(h, eps, 1, "eps"), _dev_ptr(sums, torch.float64, 10, "sums"), _stream_ptr(stream)))


RELAXATION_KEYS = ("max_drho", "max_du", "max_detot", "internal_energy", "kinetic_energy",
                   "rms_drho", "rms_du", "rms_detot")


def mlbm_relaxation(h, W, stream=None):
    """Distances from the uniform equilibrium and the energy split, as a dict (RELAXATION_KEYS)."""
    out = (ctypes.c_double * 8)()
    _check(load_library().mlbm_relaxation(h.ptr, _field_ptr(h, W, "W"), out, _stream_ptr(stream)))
    return dict(zip(RELAXATION_KEYS, out[:]))


def mlbm_spin_loss(h, W, r_target, loss=None, lam=None, stream=None):
    import torch
    _check(load_library().mlbm_spin_loss(
        h.ptr, _field_ptr(h, W, "W"), _f64_ptr(h, r_target, 3, "r_target"),
        _dev_ptr(loss, torch.float64, 1, "loss"), None if lam is None else _field_ptr(h, lam, "lam"),
        _stream_ptr(stream)))


def mlbm_adjoint_step(h, W_n, lam_next, lam_n, dL_domega=None, stream=None):
    import torch
    _check(load_library().mlbm_adjoint_step(
        h.ptr, _field_ptr(h, W_n, "W_n"), _field_ptr(h, lam_next, "lam_next"), _field_ptr(h, lam_n, "lam_n"),
        _dev_ptr(dL_domega, torch.float64, 1, "dL_domega"), _stream_ptr(stream)))


def mlbm_set_magnetic_field(h, mu_b):
    """Uniform mu B (three numbers), or None to switch the field off."""
    arr = None if mu_b is None else (ctypes.c_double * 3)(*[float(v) for v in mu_b])
    _check(load_library().mlbm_set_magnetic_field(h.ptr, arr))
    mlbm_get_info(h)


def mlbm_set_magnetic_field_map(h, mu_b):
    """Per-cell mu B as a float64 device tensor [3, *grid] (kept alive by the caller), or None."""
    if mu_b is None:
        _check(load_library().mlbm_set_magnetic_field_map(h.ptr, None))
        h._field_map = None
        mlbm_get_info(h)
        return
    ptr = _f64_ptr(h, mu_b, 3, "mu_b")
    _check(load_library().mlbm_set_magnetic_field_map(h.ptr, ptr))
    h._field_map = mu_b          # keep the device memory alive while the handle uses it
    mlbm_get_info(h)


def mlbm_set_positivity(h, on):
    _check(load_library().mlbm_set_positivity(h.ptr, int(on)))
    mlbm_get_info(h)


def mlbm_set_launch(h, block_x=0, order=MLBM_ORDER_AUTO, blocks_per_cu=-1):
    _check(load_library().mlbm_set_launch(h.ptr, int(block_x), int(order), int(blocks_per_cu)))
    mlbm_get_info(h)


def mlbm_set_store_policy(h, policy=-1):
    """-1 automatic, 0 streaming (non-temporal) field writes, 1 temporal."""
    _check(load_library().mlbm_set_store_policy(h.ptr, int(policy)))
    mlbm_get_info(h)


def mlbm_set_adjoint_launch(h, form=MLBM_ADJ_AUTO, block_x=0, order=MLBM_ORDER_AUTO, blocks_per_cu=-1, stores=-1):
    _check(load_library().mlbm_set_adjoint_launch(h.ptr, int(form), int(block_x), int(order), int(blocks_per_cu),
                                                  int(stores)))
    mlbm_get_info(h)


def mlbm_adjoint_segment(h, W, states, nsteps, lam, lam_tmp, dL_domega=None, stream=None):
    """states: device tensor holding at least nsteps - 1 fields (e.g. shape [n - 1, *field_shape]) or None."""
    import torch
    if nsteps > 1:
        need = (nsteps - 1) * 4 * h.Q * h.info["ncell"]
        if states is None or states.dtype != h.field_dtype or states.numel() < need or not states.is_contiguous():
            raise MlbmError(MLBM_EINVAL, f"states must hold {nsteps - 1} contiguous fields")
    _check(load_library().mlbm_adjoint_segment(
        h.ptr, _field_ptr(h, W, "W"), None if states is None else _dev_ptr(states, name="states"), int(nsteps),
        _field_ptr(h, lam, "lam"), _field_ptr(h, lam_tmp, "lam_tmp"),
        _dev_ptr(dL_domega, torch.float64, 1, "dL_domega"), _stream_ptr(stream)))


def mlbm_adjoint_sweep(h, W, states, nsteps, lam, lam_tmp, dL_domega=None, stream=None):
    """states: the nsteps - 1 post-collision states after W (e.g. from mlbm_step_states), or None for nsteps <= 1."""
    import torch
    _check(load_library().mlbm_adjoint_sweep(
        h.ptr, _field_ptr(h, W, "W"), _states_ptr(h, states, nsteps - 1, "states"), int(nsteps),
        _field_ptr(h, lam, "lam"), _field_ptr(h, lam_tmp, "lam_tmp"),
        _dev_ptr(dL_domega, torch.float64, 1, "dL_domega"), _stream_ptr(stream)))


def mlbm_adjoint_sweep_post(h, S_prev, states, nsteps, lam, lam_tmp, dL_domega=None, stream=None):
    """As mlbm_adjoint_sweep, with the segment's first state pulled from the post-collision state S_prev."""
    import torch
    _check(load_library().mlbm_adjoint_sweep_post(
        h.ptr, _field_ptr(h, S_prev, "S_prev"), _states_ptr(h, states, nsteps - 1, "states"), int(nsteps),
        _field_ptr(h, lam, "lam"), _field_ptr(h, lam_tmp, "lam_tmp"),
        _dev_ptr(dL_domega, torch.float64, 1, "dL_domega"), _stream_ptr(stream)))


def mlbm_device_copy(src, dst, nbytes=None, stream=None):
    """Diagnostic plain copy of nbytes (default: all of src) between two device tensors."""
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    if n > src.numel() * src.element_size() or n > dst.numel() * dst.element_size():
        raise MlbmError(MLBM_EINVAL, "nbytes exceeds a tensor")
    _check(load_library().mlbm_device_copy(_dev_ptr(src, name="src"), _dev_ptr(dst, name="dst"), n,
                                           _stream_ptr(stream)))


def mlbm_set_f16_reference(h, ref, scale):
    ref = np.ascontiguousarray(ref, dtype=np.float64).reshape(-1)
    if ref.size != 4 * h.Q:
        raise MlbmError(MLBM_EINVAL, f"reference needs {4 * h.Q} values")
    _check(load_library().mlbm_set_f16_reference(
        h.ptr, ref.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(scale)))
    mlbm_get_info(h)
