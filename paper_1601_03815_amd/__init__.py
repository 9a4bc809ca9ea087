"""LBE and DUGKS time steps for decaying isotropic turbulence on MI355X.

The compute path is the HIP library libdhit.so (kernels for gfx950 behind the
C ABI of include/dhit.h).  This package binds it with ctypes under the same
function names, and adds `Box`, a small owner object that lets PyTorch
provide the device memory and the stream.  There is no CPU fallback: when
the library is missing, importing this package raises ImportError.
"""
from ._binding import (  # noqa: F401
    DUGKS, FP32, FP64, LBE_BGK, LBE_MRT, METHODS, PRECISIONS, VARIANT_DEFAULT, VARIANT_TWO_PASS,
    DhitError, NonFiniteError, Params, box_bytes, spectrum_bytes, box_synchronize, create_box, current_populations,
    default_params, destroy_box, energy_spectrum, get_populations, init_velocity_field, init_velocity_field_device,
    init_consistent, set_mesh, last_error,
    moments, vorticity, initial_pressure, population_buffer_bytes, set_populations, step_batch, step_dugks, step_lbe, steps_taken,
    sums_history, set_kernel_timing, read_kernel_timings, device_copy, step_noalloc, KERNEL_NAMES,
    fused_work_items, fused_work_item,
    create_batch, batch_update, batch_set_stream, batch_step, batch_info, destroy_batch,
)
from . import _binding

import itertools as _itertools

_uids = _itertools.count()


class Box:
    """One periodic n^3 box of one method and precision.

    Device memory for the two population buffers comes from PyTorch
    (``torch.empty`` on the current CUDA/HIP device) and the library works on
    a PyTorch stream (``stream``, else PyTorch's current stream, else - when
    that is PyTorch's default null stream - a new ``torch.cuda.Stream``),
    exposed as ``self.stream`` so that callers can order PyTorch work and
    record events around the box's kernels.  With ``torch_memory=False`` the
    library allocates the buffers and creates its own stream.  Extra keyword
    arguments override fields of the parameter struct (e.g.
    ``variant=VARIANT_TWO_PASS``, ``dt=0.35``, ``s1=1.5``).
    """

    def __init__(self, n, method, precision="fp64", nu=0.01, torch_memory=True, stream=None, **overrides):
        self.uid = next(_uids)   # unique for the process (never reused, unlike id())
        self.n = int(n)
        self.method = method
        self.params = default_params(n, method, precision, nu)
        if "nu" in overrides:
            raise ValueError("pass nu as the positional/keyword argument, not as an override")
        for k, v in overrides.items():
            if not hasattr(self.params, k):
                raise AttributeError("dhit_params has no field %r" % k)
            setattr(self.params, k, v)
        self._buffers = None
        self.stream = None
        if torch_memory:
            import torch
            nbytes = population_buffer_bytes(self.params)
            self._buffers = (torch.empty(nbytes, dtype=torch.uint8, device="cuda"),
                             torch.empty(nbytes, dtype=torch.uint8, device="cuda"))
            self.params.f_a = self._buffers[0].data_ptr()
            self.params.f_b = self._buffers[1].data_ptr()
            if stream is None:
                stream = torch.cuda.current_stream()
                if stream.cuda_stream == 0:
                    stream = torch.cuda.Stream()
            self.stream = stream
            self.params.stream = stream.cuda_stream
        elif stream is not None:
            self.params.stream = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        self.handle = create_box(self.params)

    # lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None) is not None:
            destroy_box(self.handle)
            self.handle = None
        self._buffers = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # verbs ------------------------------------------------------------------
    def init_velocity_field(self, u, drho=None):
        init_velocity_field(self.handle, self.n, u, drho)

    def init_velocity_field_device(self, u, drho=None):
        """The same initial state from PyTorch device tensors u (3, n, n, n)
        and drho (n, n, n) of float64, without host copies; enqueued on the
        box's stream after the work queued on PyTorch's current stream
        (boxes without a PyTorch stream: the caller has synchronised)."""
        import torch
        n = self.n
        for t, shape in ((u, (3, n, n, n)), (drho, (n, n, n))):
            if t is not None and (t.dtype != torch.float64 or not t.is_cuda or tuple(t.shape) != shape
                                  or not t.is_contiguous()):
                raise ValueError("expected a contiguous float64 CUDA tensor of shape %s" % (shape,))
        if self.stream is not None:
            self.stream.wait_stream(torch.cuda.current_stream())
            # the allocator must not hand the fields' memory to other streams
            # before the box's stream has read them
            for t in (u, drho):
                if t is not None:
                    t.record_stream(self.stream)
        init_velocity_field_device(self.handle, u.data_ptr(), None if drho is None else drho.data_ptr())

    def set_mesh(self, widths=None):
        """DUGKS boxes: cell widths (3, n) per axis of a stretched periodic
        mesh (None: unit cells).  The step sums become volume-weighted."""
        set_mesh(self.handle, self.n, widths)

    def init_consistent(self, u, drho=None, iters=50):
        """LBE boxes: start from (u, drho) and iterate the scheme with the
        velocity held at u, so that the density and the non-equilibrium part
        become the scheme's own (Sec. IV.A).  Returns the largest change of
        drho over the last pass."""
        return init_consistent(self.handle, self.n, u, drho, iters)

    def step(self, nsteps=1):
        if self.params.method == DUGKS:
            step_dugks(self.handle, nsteps)
        else:
            step_lbe(self.handle, nsteps)

    def moments(self, want_fields=True):
        return moments(self.handle, self.n, want_fields)

    def sums_history(self, count):
        return sums_history(self.handle, count)

    def energy_spectrum(self, kmax=None):
        if kmax is None:
            kmax = self.n // 2
        return energy_spectrum(self.handle, kmax)

    def initial_pressure(self, u):
        """drho = 3 p consistent with velocity field u (3, n, n, n), on the GPU
        (the box's state is not touched)."""
        return initial_pressure(self.handle, self.n, u)

    def vorticity(self):
        """Vorticity of the current velocity field, (3, n, n, n) doubles in
        lattice units."""
        return vorticity(self.handle, self.n)

    def get_populations(self):
        return get_populations(self.handle, self.n)

    def set_populations(self, f):
        set_populations(self.handle, self.n, f)

    def synchronize(self):
        box_synchronize(self.handle)

    @property
    def steps(self):
        return steps_taken(self.handle)

    def populations_tensor(self):
        """A PyTorch view (19, n^3) of the current population buffer
        (only for boxes whose memory PyTorch provides).  Waits for the box's
        queued work first, since the box's stream is not always PyTorch's
        current stream."""
        import torch
        if self._buffers is None:
            raise RuntimeError("populations_tensor needs torch_memory=True")
        self.synchronize()
        ptr, stride = current_populations(self.handle)
        buf = self._buffers[0] if ptr == self._buffers[0].data_ptr() else self._buffers[1]
        dt = torch.float64 if self.params.precision == FP64 else torch.float32
        return buf.view(dt).view(19, stride)[:, : self.n ** 3]


def step_boxes(boxes, nsteps=1):
    """Advance several boxes of one method/precision with one batched launch
    per step (no tuning, no graph)."""
    step_batch([b.handle for b in boxes], nsteps)


class Batch:
    """Boxes of one method and precision advanced together: one launch per
    step over all of them (one block per work item or a persistent grid),
    autotuned, replayed from a captured hipGraph."""

    def __init__(self, boxes, autotune=True, stream=None):
        self.boxes = list(boxes)
        self.handle = create_batch([b.handle for b in self.boxes], autotune)
        self.stream = stream
        if stream is not None:
            self.set_stream(stream)

    def set_stream(self, stream):
        """Issue later steps on `stream` (a torch.cuda.Stream) instead of the
        first box's stream; each box's own stream is still ordered after the
        steps it takes part in."""
        batch_set_stream(self.handle, stream.cuda_stream)
        self.stream = stream

    def step(self, nsteps=1):
        batch_step(self.handle, nsteps)

    def update(self, boxes):
        """Replace the batch's boxes (same method and precision), keeping
        its device tables and tuned settings."""
        batch_update(self.handle, [b.handle for b in boxes])
        self.boxes = list(boxes)

    def info(self):
        return batch_info(self.handle)

    def close(self):
        if getattr(self, "handle", None) is not None:
            destroy_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
