"""qk: kernelized state-vector simulation on one AMD MI355X (gfx950).

Thin ctypes binding over ``libqk.so`` (declared in ``include/qk.h``).  Every
step of the simulation runs in the library's HIP kernels; this module only
marshals arguments.  Importing it fails loudly when the library has not been
built (``python paper_2408_09055_amd/build.py``).

PyTorch provides device memory and the stream: ``State.from_torch`` wraps a
``torch.complex64``/``complex128`` CUDA tensor, and contexts bind to
``torch.cuda.current_stream()`` by default.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libqk.so not found at {LIB_PATH}: build it with `python paper_2408_09055_amd/build.py` "
        "(there is no fallback implementation)")

# libqk links libamdhip64.so.7.  Importing torch first makes the process use
# torch's HIP runtime for both (one runtime per process); loading libqk first
# would bring in a second runtime that cannot see the device torch holds.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

QK_OK, QK_EINVAL, QK_ENOMEM, QK_EDEVICE, QK_ESTATE, QK_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
QK_C64, QK_C128 = 0, 1
QK_COST_ANALYTIC, QK_COST_LEARNED = 0, 1
QK_KERNEL_FUSED, QK_KERNEL_LDS = 0, 1
QK_CTX_HOST_ONLY = 1
QK_NOALLOC_SCRATCH_BYTES = 4 << 20
QK_IMPL_LDS_SEQUENCE, QK_IMPL_REGISTER, QK_IMPL_LDS_DENSE, QK_IMPL_MFMA_DENSE = 0, 1, 2, 3
QK_KERNELIZE_ORDERED, QK_KERNELIZE_FULL, QK_KERNELIZE_DP = 0, 1, 2
QK_ABSORB_ANTIDIAG = 2
QK_DP_ATTACH_1Q, QK_DP_SUBSUME, QK_DP_PACK, QK_DP_FUSED, QK_DP_COMMUTE = 1, 2, 4, 8, 16
IMPL_NAMES = ["lds_sequence", "register", "lds_dense", "mfma_dense"]
NUM_CLASSES = 7

_ERRNAMES = {QK_EINVAL: "QK_EINVAL", QK_ENOMEM: "QK_ENOMEM", QK_EDEVICE: "QK_EDEVICE",
             QK_ESTATE: "QK_ESTATE", QK_EUNSUPPORTED: "QK_EUNSUPPORTED"}


class QkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------- structures
class qk_circuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_gates", ctypes.c_int64), ("gates", ctypes.c_void_p)]


class qk_cost_tables(ctypes.Structure):
    _fields_ = [("fused_ps", ctypes.c_int64 * 8), ("lds_alpha_ps", ctypes.c_int64),
                ("lds_gate_ps", ctypes.c_int64 * NUM_CLASSES)]


class qk_kopts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("cost_model", ctypes.c_int32), ("k_max", ctypes.c_int32),
                ("m_max", ctypes.c_int32), ("ell", ctypes.c_int32), ("absorb_swaps", ctypes.c_int32),
                ("allow_fused", ctypes.c_int32), ("allow_lds", ctypes.c_int32),
                ("block_qubits", ctypes.c_int32), ("insular", ctypes.c_int32),
                ("kernelizer", ctypes.c_int32), ("dp_prune", ctypes.c_int32), ("dp_flags", ctypes.c_int32),
                ("local_qubits", ctypes.c_int32), ("fuse_gates", ctypes.c_int32), ("tables", ctypes.POINTER(qk_cost_tables))]


class qk_kernel_info(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("k", ctypes.c_int32), ("gate_begin", ctypes.c_int64),
                ("gate_end", ctypes.c_int64), ("qubit_mask", ctypes.c_uint64), ("cost_ps", ctypes.c_int64),
                ("block_qubits", ctypes.c_int32), ("n_ops", ctypes.c_int32), ("impl", ctypes.c_int32),
                ("n_phases", ctypes.c_int32), ("n_transposes", ctypes.c_int32), ("stage", ctypes.c_int32)]


class qk_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("val_frac", ctypes.c_float), ("seed", ctypes.c_uint64)]


class qk_train_report(ctypes.Structure):
    _fields_ = [("train_mse", ctypes.c_float), ("val_mse", ctypes.c_float), ("train_mape", ctypes.c_double),
                ("val_mape", ctypes.c_double), ("n_train", ctypes.c_int64), ("n_val", ctypes.c_int64)]


class qk_batch_stats(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("items", ctypes.c_int64), ("whole_circuits", ctypes.c_int32),
                ("errors", ctypes.c_int32)]


NUM_FEATURES = 20
DATA_DIR = os.path.join(_HERE, "data")


def costmodel_path(dtype: int) -> str:
    """Default location of the trained cost model for a dtype."""
    return os.path.join(DATA_DIR, f"costmodel_gfx950_{'c64' if dtype == 0 else 'c128'}.txt")


def autotune_path(dtype: int) -> str:
    """Default location of the shipped autotuner cache for a dtype."""
    return os.path.join(DATA_DIR, f"autotune_gfx950_{'c64' if dtype == 0 else 'c128'}.txt")


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_i32, _i64, _u64, _u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32
_dbl_p = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "qk_ctx_create": [_P, _u32, _PP], "qk_ctx_free": [_P], "qk_sync": [_P],
    "qk_debug_set_max_groups": [ctypes.c_int],
    "sv_alloc": [_P, ctypes.c_int, ctypes.c_int, _PP],
    "sv_wrap": [_P, _P, ctypes.c_int, ctypes.c_int, _PP], "sv_free": [_P],
    "sv_device_ptr": [_P, _PP], "sv_info": [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "sv_layout": [_P, _P], "sv_init_basis": [_P, _u64], "sv_upload": [_P, _P], "sv_download": [_P, _P],
    "sv_download_physical": [_P, _P],
    "sv_download_range": [_P, _u64, _u64, _P], "sv_restore": [_P], "sv_permute": [_P, _P],
    "sv_permute_inplace": [_P, _P],
    "sv_norm2": [_P, _dbl_p], "sv_overlap_host": [_P, _P, _u64, _u64, _P],
    "sv_gather": [_P, _P, _u64, _P],
    "kernelize": [_P, ctypes.POINTER(qk_circuit), ctypes.POINTER(qk_kopts), _PP],
    "plan_num_kernels": [_P, ctypes.POINTER(_i64)],
    "plan_kernel_info": [_P, _i64, ctypes.POINTER(qk_kernel_info)],
    "plan_total_cost": [_P, ctypes.POINTER(_i64)], "plan_num_gates": [_P, ctypes.POINTER(_i64)],
    "plan_gate_source": [_P, _i64, ctypes.POINTER(_i64)], "plan_final_layout": [_P, _P],
    "plan_num_stages": [_P, ctypes.POINTER(_i64)], "plan_stage_map": [_P, _i64, _P],
    "plan_free": [_P],
    "apply_kernel": [_P, _P, _i64, _P], "plan_finish": [_P, _P, _P],
    "simulate": [_P, ctypes.POINTER(qk_circuit), ctypes.POINTER(qk_kopts), _P],
    "simulate_noalloc": [_P, ctypes.POINTER(qk_circuit), ctypes.POINTER(qk_kopts), _P],
    "sv_alloc_host": [_P, ctypes.c_int, ctypes.c_int, _PP],
    "simulate_offload": [_P, ctypes.POINTER(qk_circuit), ctypes.POINTER(qk_kopts), _P],
    "execute_plan": [_P, _P, _P],
    "plan_cost_model": [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "qk_ctx_set_tables": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qk_cost_tables)],
    "qk_ctx_get_tables": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qk_cost_tables), ctypes.POINTER(ctypes.c_int)],
    "costmodel_calibrate": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qk_cost_tables)],
    "kernelize_single": [_P, ctypes.POINTER(qk_circuit), ctypes.POINTER(qk_kopts), ctypes.c_int, _PP],
    "plan_kernel_features": [_P, _i64, _P],
    "time_kernel": [_P, _P, _i64, _P, ctypes.c_int, _dbl_p],
    "costmodel_collect": [_P, _P, _P, _P, _i64, ctypes.POINTER(qk_kopts), ctypes.c_int, _P, _P, _P,
                          ctypes.POINTER(_i64)],
    "costmodel_train": [_P, ctypes.c_int, _P, _P, _i64, ctypes.POINTER(qk_train_opts), ctypes.POINTER(qk_train_report)],
    "costmodel_save": [_P, ctypes.c_int, ctypes.c_char_p], "costmodel_load": [_P, ctypes.c_int, ctypes.c_char_p],
    "costmodel_unload": [_P, ctypes.c_int], "costmodel_loaded": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "costmodel_training_range": [_P, ctypes.c_int, _P, _P],
    "costmodel_predict": [_P, ctypes.c_int, _P, _i64, _P],
    "mlp_forward_backward": [_P, _P, _P, _P, _i64, _P, _P, _P],
    "mlp_adam_step": [_P, _P, _P, _P, _P, ctypes.c_float, ctypes.c_int],
    "simulate_batch": [_P, _P, _P, _i64, _P, _P, ctypes.POINTER(qk_batch_stats)],
    "simulate_batch_persistent": [_P, _P, _P, _i64, _P, _P, ctypes.POINTER(qk_batch_stats)],
    "simulate_batch_check": [_P, _P, _i64, ctypes.c_int, _P, ctypes.POINTER(_i64)],
    "qk_autotune": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_char_p],
    "qk_autotune_load": [_P, ctypes.c_int, ctypes.c_char_p],
    "qk_set_tuned": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qk_kopts)],
    "qk_get_tuned": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(qk_kopts), ctypes.POINTER(ctypes.c_int)],
}
for _name, _args in _SIGS.items():
    try:
        _f = getattr(_lib, _name)
    except AttributeError as _e:
        raise ImportError(f"{LIB_PATH} lacks {_name}: it is older than the sources, rebuild it with "
                          "`python paper_2408_09055_amd/build.py`") from _e
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.qk_last_error.restype = ctypes.c_char_p
_lib.qk_last_error.argtypes = []
_lib.qk_version.restype = ctypes.c_char_p
_lib.qk_kopts_default.restype = None
_lib.qk_kopts_default.argtypes = [ctypes.POINTER(qk_kopts)]
_lib.mlp_num_params.restype = ctypes.c_int
_lib.mlp_num_params.argtypes = []


def lib():
    return _lib


def _check(rc: int):
    if rc != QK_OK:
        raise QkError(rc, _lib.qk_last_error().decode(errors="replace"))


def version() -> str:
    return _lib.qk_version().decode()


def set_max_groups(groups: int):
    """Test hook: bound the workgroups of persistent launches (0 = default)."""
    _check(_lib.qk_debug_set_max_groups(int(groups)))


# ---------------------------------------------------------------- options
def kopts(dtype=QK_C64, cost_model=QK_COST_ANALYTIC, k_max=None, m_max=None, ell=None,
          absorb_swaps=None, allow_fused=None, allow_lds=None, block_qubits=None, tables=None,
          insular=None, kernelizer=None, dp_prune=None, dp_flags=None, fuse_gates=None, local_qubits=None) -> qk_kopts:
    ko = qk_kopts()
    _lib.qk_kopts_default(ctypes.byref(ko))
    ko.dtype = int(dtype)
    ko.cost_model = int(cost_model)
    for name, val in (("k_max", k_max), ("m_max", m_max), ("ell", ell), ("absorb_swaps", absorb_swaps),
                      ("allow_fused", allow_fused), ("allow_lds", allow_lds), ("block_qubits", block_qubits),
                      ("insular", insular), ("kernelizer", kernelizer), ("dp_prune", dp_prune),
                      ("dp_flags", dp_flags), ("fuse_gates", fuse_gates),
                      ("local_qubits", local_qubits)):
        if val is not None:
            setattr(ko, name, int(val))
    if tables is not None:
        t = tables if isinstance(tables, qk_cost_tables) else make_tables(*tables)
        ko._tables_keep = t
        ko.tables = ctypes.pointer(t)
    return ko


def tables_tuple(t: qk_cost_tables):
    return ([int(t.fused_ps[k]) for k in range(8)], int(t.lds_alpha_ps),
            [int(t.lds_gate_ps[c]) for c in range(NUM_CLASSES)])


def make_tables(fused, alpha, gate) -> qk_cost_tables:
    t = qk_cost_tables()
    for k in range(8):
        t.fused_ps[k] = int(fused[k])
    t.lds_alpha_ps = int(alpha)
    for c in range(NUM_CLASSES):
        t.lds_gate_ps[c] = int(gate[c])
    return t


def _circuit_struct(circ) -> qk_circuit:
    gates = np.ascontiguousarray(circ.gates)
    assert gates.dtype.itemsize == 48
    c = qk_circuit()
    c.n_qubits = circ.n_qubits
    c.n_gates = len(gates)
    c.gates = gates.ctypes.data if len(gates) else None
    c._keep = gates
    return c


# ---------------------------------------------------------------- objects
class Context:
    """A libqk context bound to a HIP stream (default: torch's current stream)."""

    def __init__(self, stream=None, host_only: bool = False):
        self.host_only = host_only
        if stream is None and not host_only:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        self._stream = stream
        h = ctypes.c_void_p()
        _check(_lib.qk_ctx_create(ctypes.c_void_p(stream or 0), QK_CTX_HOST_ONLY if host_only else 0,
                                  ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            _lib.qk_ctx_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        _check(_lib.qk_sync(self.h))

    def set_tables(self, n: int, dtype: int, tables):
        t = tables if isinstance(tables, qk_cost_tables) else make_tables(*tables)
        _check(_lib.qk_ctx_set_tables(self.h, n, dtype, ctypes.byref(t)))

    def get_tables(self, n: int, dtype: int):
        t = qk_cost_tables()
        d = ctypes.c_int()
        _check(_lib.qk_ctx_get_tables(self.h, n, dtype, ctypes.byref(t), ctypes.byref(d)))
        return tables_tuple(t), bool(d.value)

    def calibrate(self, n: int, dtype: int, reps: int = 3):
        """Measure the analytic cost constants for (n, dtype) on the device."""
        t = qk_cost_tables()
        _check(_lib.costmodel_calibrate(self.h, n, dtype, reps, ctypes.byref(t)))
        return tables_tuple(t)

    def load_costmodel(self, dtype: int, path: str | None = None) -> bool:
        p = path or costmodel_path(dtype)
        if not os.path.exists(p):
            return False
        _check(_lib.costmodel_load(self.h, dtype, p.encode()))
        return True

    def save_costmodel(self, dtype: int, path: str):
        _check(_lib.costmodel_save(self.h, dtype, path.encode()))

    def unload_costmodel(self, dtype: int):
        _check(_lib.costmodel_unload(self.h, dtype))

    def costmodel_loaded(self, dtype: int) -> bool:
        v = ctypes.c_int()
        _check(_lib.costmodel_loaded(self.h, dtype, ctypes.byref(v)))
        return bool(v.value)

    def training_range(self, dtype: int):
        """(x_min, x_max) over the loaded model's training rows, per feature."""
        lo = np.zeros(NUM_FEATURES, np.float32)
        hi = np.zeros(NUM_FEATURES, np.float32)
        _check(_lib.costmodel_training_range(self.h, dtype, lo.ctypes.data, hi.ctypes.data))
        return lo, hi

    def predict(self, dtype: int, feats: np.ndarray) -> np.ndarray:
        f = np.ascontiguousarray(feats, np.float32).reshape(-1, NUM_FEATURES)
        out = np.zeros(f.shape[0], np.float32)
        _check(_lib.costmodel_predict(self.h, dtype, f.ctypes.data, f.shape[0], out.ctypes.data))
        return out

    def train_costmodel(self, dtype: int, feats: np.ndarray, targets: np.ndarray, epochs=200, batch=256,
                        lr=1e-3, val_frac=0.2, seed=3) -> dict:
        f = np.ascontiguousarray(feats, np.float32).reshape(-1, NUM_FEATURES)
        t = np.ascontiguousarray(targets, np.float32)
        o = qk_train_opts(epochs, batch, lr, val_frac, seed)
        r = qk_train_report()
        _check(_lib.costmodel_train(self.h, dtype, f.ctypes.data, t.ctypes.data, f.shape[0], ctypes.byref(o),
                                    ctypes.byref(r)))
        return {"train_mse": r.train_mse, "val_mse": r.val_mse, "train_mape": r.train_mape,
                "val_mape": r.val_mape, "n_train": r.n_train, "n_val": r.n_val}


class State:
    """A 2^n-amplitude state vector on the device."""

    def __init__(self, ctx: Context, handle, n: int, dtype: int, keep=None):
        self.ctx = ctx
        self.h = handle
        self.n = n
        self.dtype = dtype
        self._keep = keep

    @classmethod
    def alloc(cls, ctx: Context, n: int, dtype: int = QK_C64) -> "State":
        h = ctypes.c_void_p()
        _check(_lib.sv_alloc(ctx.h, n, dtype, ctypes.byref(h)))
        return cls(ctx, h, n, dtype)

    @classmethod
    def from_torch(cls, ctx: Context, t) -> "State":
        import torch
        assert t.is_cuda and t.is_contiguous() and t.dim() == 1
        dtype = {torch.complex64: QK_C64, torch.complex128: QK_C128}[t.dtype]
        n = int(t.numel()).bit_length() - 1
        assert (1 << n) == t.numel()
        h = ctypes.c_void_p()
        _check(_lib.sv_wrap(ctx.h, ctypes.c_void_p(t.data_ptr()), n, dtype, ctypes.byref(h)))
        return cls(ctx, h, n, dtype, keep=t)

    def free(self):
        if self.h:
            _lib.sv_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def np_dtype(self):
        return np.complex64 if self.dtype == QK_C64 else np.complex128

    def device_ptr(self) -> int:
        p = ctypes.c_void_p()
        _check(_lib.sv_device_ptr(self.h, ctypes.byref(p)))
        return p.value

    def layout(self) -> list:
        out = np.zeros(self.n, np.int32)
        _check(_lib.sv_layout(self.h, out.ctypes.data))
        return [int(x) for x in out]

    def init_basis(self, x: int = 0):
        _check(_lib.sv_init_basis(self.h, int(x)))

    def upload(self, host: np.ndarray):
        a = np.ascontiguousarray(host, dtype=self.np_dtype)
        assert a.size == (1 << self.n)
        _check(_lib.sv_upload(self.h, a.ctypes.data))

    def download(self) -> np.ndarray:
        out = np.empty(1 << self.n, self.np_dtype)
        _check(_lib.sv_download(self.h, out.ctypes.data))
        return out

    def download_physical(self) -> np.ndarray:
        out = np.empty(1 << self.n, self.np_dtype)
        _check(_lib.sv_download_physical(self.h, out.ctypes.data))
        return out

    def download_range(self, offset: int, count: int) -> np.ndarray:
        out = np.empty(count, self.np_dtype)
        _check(_lib.sv_download_range(self.h, offset, count, out.ctypes.data))
        return out

    def restore(self):
        _check(_lib.sv_restore(self.h))

    def permute(self, perm):
        p = np.ascontiguousarray(perm, np.int32)
        _check(_lib.sv_permute(self.h, p.ctypes.data))

    def permute_inplace(self, perm):
        p = np.ascontiguousarray(perm, np.int32)
        _check(_lib.sv_permute_inplace(self.h, p.ctypes.data))

    def norm2(self) -> float:
        out = ctypes.c_double()
        _check(_lib.sv_norm2(self.h, ctypes.byref(out)))
        return out.value

    def overlap_host(self, ref: np.ndarray, offset: int = 0) -> complex:
        r = np.ascontiguousarray(ref, np.complex128)
        out = np.zeros(2)
        _check(_lib.sv_overlap_host(self.h, r.ctypes.data, offset, r.size, out.ctypes.data))
        return complex(out[0], out[1])

    def gather(self, idx) -> np.ndarray:
        i = np.ascontiguousarray(idx, np.uint64)
        out = np.zeros(i.size, np.complex128)
        _check(_lib.sv_gather(self.h, i.ctypes.data, i.size, out.ctypes.data))
        return out


class KernelInfo:
    def __init__(self, s: qk_kernel_info):
        self.type = s.type
        self.k = s.k
        self.gate_begin = s.gate_begin
        self.gate_end = s.gate_end
        self.qubit_mask = s.qubit_mask
        self.cost_ps = s.cost_ps
        self.block_qubits = s.block_qubits
        self.n_ops = s.n_ops
        self.impl = s.impl
        self.n_phases = s.n_phases
        self.n_transposes = s.n_transposes
        self.stage = s.stage

    def as_tuple(self):
        return (self.gate_begin, self.gate_end, self.type, self.cost_ps)

    def __repr__(self):
        t = "fused" if self.type == QK_KERNEL_FUSED else "lds"
        return f"<{t} k={self.k} gates[{self.gate_begin}:{self.gate_end}] cost={self.cost_ps}>"


class Plan:
    """Output of ``kernelize``: a kernel sequence ready to run."""

    def __init__(self, ctx: Context, handle, n: int):
        self.ctx = ctx
        self.h = handle
        self.n = n

    def free(self):
        if self.h:
            _lib.plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __len__(self):
        v = ctypes.c_int64()
        _check(_lib.plan_num_kernels(self.h, ctypes.byref(v)))
        return v.value

    def kernel(self, i: int) -> KernelInfo:
        s = qk_kernel_info()
        _check(_lib.plan_kernel_info(self.h, i, ctypes.byref(s)))
        return KernelInfo(s)

    def kernels(self) -> list:
        return [self.kernel(i) for i in range(len(self))]

    def total_cost(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.plan_total_cost(self.h, ctypes.byref(v)))
        return v.value

    def num_gates(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.plan_num_gates(self.h, ctypes.byref(v)))
        return v.value

    def gate_source(self, i: int) -> int:
        v = ctypes.c_int64()
        _check(_lib.plan_gate_source(self.h, i, ctypes.byref(v)))
        return v.value

    def features(self, i: int) -> np.ndarray:
        out = np.zeros(NUM_FEATURES, np.float32)
        _check(_lib.plan_kernel_features(self.h, i, out.ctypes.data))
        return out

    def cost_model(self):
        u, f = ctypes.c_int(), ctypes.c_int()
        _check(_lib.plan_cost_model(self.h, ctypes.byref(u), ctypes.byref(f)))
        return {"learned_used": bool(u.value), "learned_fallback": bool(f.value)}

    def final_layout(self) -> list:
        out = np.zeros(self.n, np.int32)
        _check(_lib.plan_final_layout(self.h, out.ctypes.data))
        return [int(x) for x in out]

    def num_stages(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.plan_num_stages(self.h, ctypes.byref(v)))
        return v.value

    def stage_map(self, s: int) -> list:
        out = np.zeros(self.n, np.int32)
        _check(_lib.plan_stage_map(self.h, s, out.ctypes.data))
        return [int(x) for x in out]


# ---------------------------------------------------------------- entry points
def sv_alloc(ctx: Context, n: int, dtype: int = QK_C64) -> State:
    return State.alloc(ctx, n, dtype)


def kernelize(ctx: Context, circuit, ko: qk_kopts | None = None) -> Plan:
    c = _circuit_struct(circuit)
    h = ctypes.c_void_p()
    _check(_lib.kernelize(ctx.h, ctypes.byref(c), ctypes.byref(ko) if ko is not None else None,
                          ctypes.byref(h)))
    return Plan(ctx, h, circuit.n_qubits)


def apply_kernel(ctx: Context, plan: Plan, i: int, state: State):
    _check(_lib.apply_kernel(ctx.h, plan.h, i, state.h))


def plan_finish(ctx: Context, plan: Plan, state: State):
    _check(_lib.plan_finish(ctx.h, plan.h, state.h))


def execute_plan(ctx: Context, plan: Plan, state: State):
    _check(_lib.execute_plan(ctx.h, plan.h, state.h))


def simulate(ctx: Context, circuit, state: State, ko: qk_kopts | None = None):
    c = _circuit_struct(circuit)
    _check(_lib.simulate(ctx.h, ctypes.byref(c), ctypes.byref(ko) if ko is not None else None, state.h))


def sv_alloc_host(ctx: Context, n: int, dtype: int = QK_C64) -> State:
    """A state in pinned host memory, for simulate_offload."""
    h = ctypes.c_void_p()
    _check(_lib.sv_alloc_host(ctx.h, n, dtype, ctypes.byref(h)))
    return State(ctx, h, n, dtype)


def simulate_offload(ctx: Context, circuit, state: State, ko: qk_kopts):
    c = _circuit_struct(circuit)
    _check(_lib.simulate_offload(ctx.h, ctypes.byref(c), ctypes.byref(ko), state.h))


def simulate_noalloc(ctx: Context, circuit, state: State, ko: qk_kopts | None = None):
    c = _circuit_struct(circuit)
    _check(_lib.simulate_noalloc(ctx.h, ctypes.byref(c), ctypes.byref(ko) if ko is not None else None, state.h))


def kernelize_single(ctx: Context, circuit, ko: qk_kopts | None, ktype: int) -> Plan:
    c = _circuit_struct(circuit)
    h = ctypes.c_void_p()
    _check(_lib.kernelize_single(ctx.h, ctypes.byref(c), ctypes.byref(ko) if ko is not None else None, ktype,
                                 ctypes.byref(h)))
    return Plan(ctx, h, circuit.n_qubits)


def time_kernel(ctx: Context, plan: Plan, i: int, state: State, reps: int = 3) -> float:
    v = ctypes.c_double()
    _check(_lib.time_kernel(ctx.h, plan.h, i, state.h, reps, ctypes.byref(v)))
    return v.value


def costmodel_collect(ctx: Context, state: State, circuits, types, ko: qk_kopts | None = None, reps: int = 3):
    """Times each candidate circuit as one kernel of its type on a view of
    `state` (libqk's costmodel_collect).  Returns (features, log ps per
    amplitude, ms) as arrays of len(circuits) rows."""
    cnt = len(circuits)
    assert len(types) == cnt
    feats = np.zeros((cnt, NUM_FEATURES), np.float32)
    log_ps = np.zeros(cnt, np.float32)
    ms = np.zeros(cnt, np.float64)
    if cnt == 0:
        return feats, log_ps, ms
    cstructs, keep = _circuit_array(circuits)
    ty = np.ascontiguousarray(types, np.int32)
    done = _i64()
    _check(_lib.costmodel_collect(ctx.h, state.h, cstructs, ty.ctypes.data, cnt,
                                  ctypes.byref(ko) if ko is not None else None, reps, feats.ctypes.data,
                                  log_ps.ctypes.data, ms.ctypes.data, ctypes.byref(done)))
    return feats, log_ps, ms


def mlp_num_params() -> int:
    return int(_lib.mlp_num_params())


def mlp_forward_backward(ctx: Context, params: np.ndarray, x: np.ndarray, t: np.ndarray | None = None):
    """One device pass of the cost-model network: returns (y, loss, grads)."""
    p = np.ascontiguousarray(params, np.float32)
    assert p.size == mlp_num_params()
    xx = np.ascontiguousarray(x, np.float32).reshape(-1, NUM_FEATURES)
    B = xx.shape[0]
    y = np.zeros(B, np.float32)
    loss = np.zeros(1, np.float32)
    grads = np.zeros(p.size, np.float32)
    tt = None if t is None else np.ascontiguousarray(t, np.float32)
    _check(_lib.mlp_forward_backward(ctx.h, p.ctypes.data, xx.ctypes.data,
                                     None if tt is None else tt.ctypes.data, B, y.ctypes.data,
                                     loss.ctypes.data, grads.ctypes.data))
    return y, (float(loss[0]) if tt is not None else None), (grads if tt is not None else None)


def mlp_adam_step(ctx: Context, params, grads, m, v, lr: float, step: int):
    """One device Adam step; returns updated (params, m, v) copies."""
    p = np.array(params, np.float32)
    g = np.ascontiguousarray(grads, np.float32)
    mm = np.array(m, np.float32)
    vv = np.array(v, np.float32)
    _check(_lib.mlp_adam_step(ctx.h, p.ctypes.data, g.ctypes.data, mm.ctypes.data, vv.ctypes.data, lr, step))
    return p, mm, vv


def _circuit_array(circuits):
    n = len(circuits)
    cstructs = (qk_circuit * n)()
    keep = []
    for i, c in enumerate(circuits):
        cs = _circuit_struct(c)
        keep.append(cs)
        ctypes.memmove(ctypes.byref(cstructs, i * ctypes.sizeof(qk_circuit)), ctypes.byref(cs),
                       ctypes.sizeof(qk_circuit))
    return cstructs, keep


def simulate_batch_persistent(ctx: Context, circuits, states, kos=None):
    """Run many circuits in one persistent launch.  Returns (stats dict,
    per-circuit latency in ms from the first workgroup's start)."""
    n = len(circuits)
    assert len(states) == n and n > 0
    cstructs, keep = _circuit_array(circuits)
    sptr = (ctypes.c_void_p * n)(*[s.h.value if isinstance(s.h, ctypes.c_void_p) else s.h for s in states])
    karr = (qk_kopts * n)(*kos) if kos is not None else None
    lat = np.zeros(n, np.float64)
    st = qk_batch_stats()
    _check(_lib.simulate_batch_persistent(ctx.h, ctypes.cast(cstructs, ctypes.c_void_p),
                                          ctypes.cast(sptr, ctypes.c_void_p), n,
                                          ctypes.cast(karr, ctypes.c_void_p) if karr is not None else None,
                                          lat.ctypes.data, ctypes.byref(st)))
    return ({"total_ms": st.total_ms, "items": st.items, "whole_circuits": st.whole_circuits,
             "errors": st.errors}, lat)


def simulate_batch_check(ctx: Context, circuits, dtype: int, kos=None) -> int:
    """Plan a batch and bounds-check its persistent-launch descriptors on the
    host; returns the number of kernels."""
    n = len(circuits)
    cstructs, keep = _circuit_array(circuits)
    karr = (qk_kopts * n)(*kos) if kos is not None else None
    nk = ctypes.c_int64()
    _check(_lib.simulate_batch_check(ctx.h, ctypes.cast(cstructs, ctypes.c_void_p), n, dtype,
                                     ctypes.cast(karr, ctypes.c_void_p) if karr is not None else None,
                                     ctypes.byref(nk)))
    return nk.value


def simulate_batch(ctx: Context, circuits, states, kos=None):
    """Run many circuits, dealt over the library's HIP streams.  Returns
    (stats dict, per-circuit latency in ms from the batch start)."""
    n = len(circuits)
    assert len(states) == n and n > 0
    cstructs = (qk_circuit * n)()
    keep = []
    for i, c in enumerate(circuits):
        cs = _circuit_struct(c)
        keep.append(cs)
        ctypes.memmove(ctypes.byref(cstructs, i * ctypes.sizeof(qk_circuit)), ctypes.byref(cs),
                       ctypes.sizeof(qk_circuit))
    sptr = (ctypes.c_void_p * n)(*[s.h.value if isinstance(s.h, ctypes.c_void_p) else s.h for s in states])
    karr = None
    if kos is not None:
        karr = (qk_kopts * n)(*kos)
    lat = np.zeros(n, np.float64)
    st = qk_batch_stats()
    _check(_lib.simulate_batch(ctx.h, ctypes.cast(cstructs, ctypes.c_void_p), ctypes.cast(sptr, ctypes.c_void_p), n,
                               ctypes.cast(karr, ctypes.c_void_p) if karr is not None else None,
                               lat.ctypes.data, ctypes.byref(st)))
    return ({"total_ms": st.total_ms, "items": st.items, "whole_circuits": st.whole_circuits,
             "errors": st.errors}, lat)


def autotune(ctx: Context, dtype: int, n_lo: int, n_hi: int, reps: int = 3, cache_path: str | None = None):
    _check(_lib.qk_autotune(ctx.h, dtype, n_lo, n_hi, reps, cache_path.encode() if cache_path else None))


def autotune_load(ctx: Context, dtype: int, path: str):
    _check(_lib.qk_autotune_load(ctx.h, dtype, path.encode()))


def get_tuned(ctx: Context, dtype: int, n: int):
    ko = qk_kopts()
    f = ctypes.c_int()
    _check(_lib.qk_get_tuned(ctx.h, dtype, n, ctypes.byref(ko), ctypes.byref(f)))
    return ko, bool(f.value)
