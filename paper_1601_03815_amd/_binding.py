"""ctypes binding of libdhit.so: argument marshalling only.

Every function here calls the C function of the same name declared in
include/dhit.h; all arithmetic runs in the library's HIP kernels.  The
library must have been built (``python paper_1601_03815_amd/build.py`` or
``__graft_entry__.build()``); importing this module raises ImportError when
it has not.
"""
import ctypes
import os

import numpy as np

# One HIP runtime per process: PyTorch ships its own copy of the HIP
# runtime, hipFFT and the HSA runtime (same sonames as the system ROCm).
# Importing torch first makes libdhit.so bind to the copies torch already
# loaded; loading the system copies next to torch's gives two runtimes that
# both try to own the device.
try:
    import torch  # noqa: F401
except ImportError:  # a caller without PyTorch uses the system ROCm runtime
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdhit.so")

DHIT_OK = 0
DHIT_EINVAL = -1
DHIT_ENOMEM = -2
DHIT_EDEVICE = -3
DHIT_EMETHOD = -4
DHIT_ENONFINITE = -5

LBE_BGK, LBE_MRT, DUGKS = 0, 1, 2
FP64, FP32 = 0, 1
VARIANT_DEFAULT, VARIANT_TWO_PASS = 0, 1

METHODS = {"bgk": LBE_BGK, "mrt": LBE_MRT, "dugks": DUGKS}
PRECISIONS = {"fp64": FP64, "fp32": FP32}

Q = 19


class DhitError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("dhit error %d: %s" % (code, message))
        self.code = code


class NonFiniteError(DhitError):
    pass


class Params(ctypes.Structure):
    """Mirror of struct dhit_params."""
    _fields_ = [
        ("n", ctypes.c_int32), ("method", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("variant", ctypes.c_int32), ("tile_width", ctypes.c_int32), ("z_chunk", ctypes.c_int32),
        ("nu", ctypes.c_double), ("rho0", ctypes.c_double), ("dt", ctypes.c_double),
        ("s1", ctypes.c_double), ("s2", ctypes.c_double), ("s4", ctypes.c_double), ("s9", ctypes.c_double),
        ("s10", ctypes.c_double), ("s13", ctypes.c_double), ("s16", ctypes.c_double),
        ("w_eps", ctypes.c_double), ("w_epsj", ctypes.c_double), ("w_xx", ctypes.c_double),
        ("stream", ctypes.c_void_p), ("f_a", ctypes.c_void_p), ("f_b", ctypes.c_void_p),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdhit.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(Params)
    box = ctypes.c_void_p
    dp = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    sig = {
        "default_params": ([i32, i32, i32, ctypes.c_double, P], i32),
        "population_buffer_bytes": ([P], i64),
        "box_bytes": ([P], i64),
        "spectrum_bytes": ([P], i64),
        "fused_work_items": ([P, i32, ctypes.POINTER(i32)], i32),
        "fused_work_item": ([P, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "create_box": ([P, ctypes.POINTER(ctypes.c_void_p)], i32),
        "destroy_box": ([box], i32),
        "init_velocity_field": ([box, dp, dp], i32),
        "init_velocity_field_device": ([box, ctypes.c_void_p, ctypes.c_void_p], i32),
        "init_consistent": ([box, dp, dp, i32, dp], i32),
        "set_mesh": ([box, dp], i32),
        "step_lbe": ([box, i32], i32),
        "step_dugks": ([box, i32], i32),
        "moments": ([box, dp, dp, dp], i32),
        "sums_history": ([box, dp, i32], i32),
        "energy_spectrum": ([box, dp, i32, dp], i32),
        "vorticity": ([box, dp], i32),
        "initial_pressure": ([box, dp, dp], i32),
        "get_populations": ([box, dp], i32),
        "set_populations": ([box, dp], i32),
        "steps_taken": ([box], i64),
        "box_synchronize": ([box], i32),
        "current_populations": ([box, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int64)], i32),
        "step_batch": ([ctypes.POINTER(ctypes.c_void_p), i32, i32], i32),
        "create_batch": ([ctypes.POINTER(ctypes.c_void_p), i32, i32, ctypes.POINTER(ctypes.c_void_p)], i32),
        "batch_step": ([ctypes.c_void_p, i32], i32),
        "batch_set_stream": ([ctypes.c_void_p, ctypes.c_void_p], i32),
        "batch_update": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), i32], i32),
        "batch_info": ([ctypes.c_void_p, dp], i32),
        "destroy_batch": ([ctypes.c_void_p], i32),
        "set_kernel_timing": ([box, i32], i32),
        "read_kernel_timings": ([box, dp, dp], i32),
        "device_copy": ([ctypes.c_void_p, ctypes.c_void_p, i64, ctypes.c_void_p], i32),
        "step_noalloc": ([P, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], i32),
        "dhit_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def last_error():
    return _lib.dhit_last_error().decode()


def _check(code):
    if code < 0:
        msg = last_error()
        if code == DHIT_ENONFINITE:
            raise NonFiniteError(code, msg)
        raise DhitError(code, msg)
    return code


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64_out(shape):
    return np.zeros(shape, dtype=np.float64)


def _f64_in(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (tuple(shape), a.shape))
    return a


# ----------------------------------------------------------------------------
# Functions with the names of the C ABI
# ----------------------------------------------------------------------------

def default_params(n, method, precision, nu):
    """method: 'bgk' | 'mrt' | 'dugks' or the enum value; precision: 'fp64' |
    'fp32' or the enum value."""
    p = Params()
    m = METHODS.get(method, method)
    pr = PRECISIONS.get(precision, precision)
    _check(_lib.default_params(int(n), int(m), int(pr), float(nu), ctypes.byref(p)))
    return p


def population_buffer_bytes(p):
    return _check(_lib.population_buffer_bytes(ctypes.byref(p)))


def box_bytes(p):
    return _check(_lib.box_bytes(ctypes.byref(p)))


def spectrum_bytes(p):
    return _check(_lib.spectrum_bytes(ctypes.byref(p)))


def fused_work_items(p, slots):
    """(work items of the fused DUGKS launch, z_chunk setting in effect) on a
    device holding `slots` blocks of the kernel at once."""
    z = ctypes.c_int32()
    items = _check(_lib.fused_work_items(ctypes.byref(p), int(slots), ctypes.byref(z)))
    return items, z.value


def fused_work_item(p, slots, item):
    """(tile, z0, planes) that work item `item` of that launch marches."""
    t, z, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.fused_work_item(ctypes.byref(p), int(slots), int(item), ctypes.byref(t), ctypes.byref(z),
                                ctypes.byref(k)))
    return t.value, z.value, k.value


def create_box(p):
    h = ctypes.c_void_p()
    _check(_lib.create_box(ctypes.byref(p), ctypes.byref(h)))
    return h


def destroy_box(h):
    _check(_lib.destroy_box(h))


def init_velocity_field(h, n, u, drho=None):
    u = _f64_in(u, (3, n, n, n))
    d = None if drho is None else _f64_in(drho, (n, n, n))
    _check(_lib.init_velocity_field(h, _ptr(u), _ptr(d)))


def init_velocity_field_device(h, u_ptr, drho_ptr=None):
    """Initial state from device fields: u_ptr, drho_ptr are device addresses
    of (3, n^3) and (n^3) doubles (drho_ptr None = 0); asynchronous on the
    box's stream (the caller keeps the fields until the stream has passed)."""
    _check(_lib.init_velocity_field_device(h, ctypes.c_void_p(u_ptr), ctypes.c_void_p(drho_ptr or 0)))


def set_mesh(h, n, widths=None):
    """Stretched mesh of a DUGKS box: widths (3, n) cell widths per axis, or
    None for unit cells."""
    w = None if widths is None else _f64_in(widths, (3, n))
    _check(_lib.set_mesh(h, _ptr(w)))


def init_consistent(h, n, u, drho=None, iters=0):
    """Consistent initial state of an LBE box; returns the largest change
    of drho over the last pass."""
    u = _f64_in(u, (3, n, n, n))
    d = None if drho is None else _f64_in(drho, (n, n, n))
    res = np.zeros(1, dtype=np.float64)
    _check(_lib.init_consistent(h, _ptr(u), _ptr(d), int(iters), _ptr(res)))
    return float(res[0])


def step_lbe(h, nsteps=1):
    _check(_lib.step_lbe(h, int(nsteps)))


def step_dugks(h, nsteps=1):
    _check(_lib.step_dugks(h, int(nsteps)))


def moments(h, n, want_fields=True):
    """(drho[n,n,n], j[3,n,n,n], sums[5]); fields are None if not wanted."""
    d = _f64_out((n, n, n)) if want_fields else None
    j = _f64_out((3, n, n, n)) if want_fields else None
    s = _f64_out(5)
    _check(_lib.moments(h, _ptr(d), _ptr(j), _ptr(s)))
    return d, j, s


def sums_history(h, count):
    out = _f64_out((count, 5))
    _check(_lib.sums_history(h, _ptr(out), int(count)))
    return out


def energy_spectrum(h, kmax):
    E = _f64_out(kmax + 1)
    st = _f64_out(4)
    _check(_lib.energy_spectrum(h, _ptr(E), int(kmax), _ptr(st)))
    return E, dict(K=st[0], eps=st[1], S=st[2], F=st[3])


def initial_pressure(h, n, u):
    """drho = 3 p of the incompressible pressure of velocity field u (3, n, n, n)."""
    u = _f64_in(u, (3, n, n, n))
    d = _f64_out((n, n, n))
    _check(_lib.initial_pressure(h, _ptr(u), _ptr(d)))
    return d


def vorticity(h, n):
    """omega = curl(j/rho0) as (3, n, n, n) doubles."""
    w = _f64_out((3, n, n, n))
    _check(_lib.vorticity(h, _ptr(w)))
    return w


def get_populations(h, n):
    f = _f64_out((Q, n, n, n))
    _check(_lib.get_populations(h, _ptr(f)))
    return f


def set_populations(h, n, f):
    f = _f64_in(f, (Q, n, n, n))
    _check(_lib.set_populations(h, _ptr(f)))


def steps_taken(h):
    return _check(_lib.steps_taken(h))


def box_synchronize(h):
    _check(_lib.box_synchronize(h))


def current_populations(h):
    ptr = ctypes.c_void_p()
    stride = ctypes.c_int64()
    _check(_lib.current_populations(h, ctypes.byref(ptr), ctypes.byref(stride)))
    return ptr.value, stride.value


def _handle_array(handles):
    return (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in handles])


def step_batch(handles, nsteps=1):
    _check(_lib.step_batch(_handle_array(handles), len(handles), int(nsteps)))


def create_batch(handles, autotune=True):
    out = ctypes.c_void_p()
    _check(_lib.create_batch(_handle_array(handles), len(handles), 1 if autotune else 0, ctypes.byref(out)))
    return out


def batch_update(bt, handles):
    _check(_lib.batch_update(bt, _handle_array(handles), len(handles)))


def batch_step(bt, nsteps=1):
    _check(_lib.batch_step(bt, int(nsteps)))


def batch_set_stream(bt, stream):
    """Issue the batch's later work on `stream` (a hipStream_t as an int,
    or 0 for the null stream)."""
    _check(_lib.batch_set_stream(bt, ctypes.c_void_p(int(stream) or None)))


def batch_info(bt):
    info = np.zeros(6, dtype=np.int64)
    _check(_lib.batch_info(bt, _ptr(info)))
    return dict(grid=int(info[0]), chunk=int(info[1]), items=int(info[2]), graph_steps=int(info[3]),
                tuned=bool(info[4]), tile=int(info[5]))


def destroy_batch(bt):
    _check(_lib.destroy_batch(bt))


KERNEL_NAMES = ["lbe", "dugks_transform", "dugks_face", "dugks_fused", "finalize"]


def set_kernel_timing(h, enable=True):
    _check(_lib.set_kernel_timing(h, 1 if enable else 0))


def read_kernel_timings(h):
    """{kernel name: (total ms, launches)} since the last read."""
    ms = np.zeros(len(KERNEL_NAMES))
    cnt = np.zeros(len(KERNEL_NAMES), dtype=np.int64)
    _check(_lib.read_kernel_timings(h, _ptr(ms), _ptr(cnt)))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_NAMES)}


def device_copy(dst_ptr, src_ptr, nbytes, stream_handle=0):
    _check(_lib.device_copy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), int(nbytes),
                            ctypes.c_void_p(stream_handle)))


def step_noalloc(p, src_ptr, dst_ptr, sums_ptr=None):
    """One step of the method in params p from device buffer src_ptr to
    dst_ptr (integers: device addresses), sums to device double[5] at
    sums_ptr (or None); the library allocates nothing."""
    _check(_lib.step_noalloc(ctypes.byref(p), ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr),
                             None if sums_ptr is None else ctypes.c_void_p(sums_ptr)))


EXPORTED = [
    "default_params", "population_buffer_bytes", "box_bytes", "spectrum_bytes", "fused_work_items",
    "fused_work_item", "create_box", "destroy_box",
    "init_velocity_field", "init_velocity_field_device", "init_consistent", "set_mesh", "step_lbe", "step_dugks", "moments", "sums_history", "energy_spectrum", "vorticity", "initial_pressure",
    "get_populations", "set_populations", "steps_taken", "box_synchronize", "current_populations",
    "step_batch", "create_batch", "batch_update", "batch_set_stream", "batch_step", "batch_info", "destroy_batch",
    "set_kernel_timing", "read_kernel_timings", "device_copy", "step_noalloc", "dhit_last_error",
]
