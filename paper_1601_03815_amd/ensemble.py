"""Batched ensembles of independent decaying-turbulence runs.

An ensemble is many boxes (distinct seeds, mixed grid sizes) of one method
and precision advanced together by `Batch` (one launch per step over all
boxes, graph replays, autotuned grid).  Also runs the same boxes one launch per box
for comparison, and averages energy spectra over the realisations of each
grid size.
"""
import numpy as np

from . import Batch, Box


def make_ensemble(sizes, method="mrt", precision="fp32", nu=0.01, fields=None, stream=None):
    """Boxes for grid sizes `sizes`; box i starts from `fields(i, n)`
    (a velocity field [3, n, n, n])."""
    boxes = []
    for i, n in enumerate(sizes):
        b = Box(n, method, precision, nu, stream=stream)
        if fields is not None:
            b.init_velocity_field(fields(i, n))
        boxes.append(b)
    return boxes


def run_batched(boxes, steps, autotune=True, torch=None):
    """Advances the boxes by `steps` with one Batch; returns (ms, batch info).
    The time is taken with events on the batch's stream (the first box's)."""
    import torch as _torch
    torch = torch or _torch
    stream = boxes[0].stream
    with Batch(boxes, autotune=autotune) as bt:
        info = bt.info()
        bt.step(1)   # warm-up (graph capture happens on the first run of >= 8 steps)
        bt.step(8)
        torch.cuda.synchronize()
        for b in boxes:
            b.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        bt.step(steps)
        e1.record(stream)
        e1.synchronize()
    return e0.elapsed_time(e1), info


def run_unbatched(boxes, steps, torch=None):
    """Advances every box by `steps`, one launch per box and step, all on
    the first box's stream order; returns ms."""
    import torch as _torch
    torch = torch or _torch
    torch.cuda.synchronize()
    for b in boxes:
        b.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    streams = {id(b.stream): b.stream for b in boxes}
    first = boxes[0].stream
    e0.record(first)
    for _ in range(steps):
        for b in boxes:
            b.step(1)
    for s in streams.values():
        ev = torch.cuda.Event()
        ev.record(s)
        first.wait_event(ev)
    e1.record(first)
    e1.synchronize()
    return e0.elapsed_time(e1)


def ensemble_spectra(boxes):
    """{n: (mean E(k) over the boxes of size n, count, mean K, mean eps)}."""
    acc = {}
    for b in boxes:
        E, st = b.energy_spectrum(b.n // 2)
        e, c, K, eps = acc.get(b.n, (np.zeros_like(E), 0, 0.0, 0.0))
        acc[b.n] = (e + E, c + 1, K + st["K"], eps + st["eps"])
    return {n: (e / c, c, K / c, eps / c) for n, (e, c, K, eps) in sorted(acc.items())}
