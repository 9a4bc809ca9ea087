"""The allocation-free step (step_noalloc) against the box step it is a
variant of (step_lbe / step_dugks): same kernels and launch, so the new
state and the global sums must agree bit for bit.  Two calls in a row, the
second on a smaller box, so that the static work space is reused with
fewer blocks than the previous call left in it."""
import numpy as np
import pytest

import paper_1601_03815_amd as dhit
import synth

pytestmark = pytest.mark.gpu

CASES = [(m, p) for p in ("fp64", "fp32") for m in ("bgk", "mrt", "dugks")]


def _noalloc_against_box(torch, method, precision, n, seed):
    nu = 0.01
    f0 = synth.random_populations(n, seed=seed, amplitude=0.01)
    if precision == "fp32":
        f0 = f0.astype(np.float32).astype(np.float64)
    print("step_noalloc: %s %s n=%d" % (method, precision, n), flush=True)
    with dhit.Box(n, method, precision, nu) as box:
        box.set_populations(f0)
        box.synchronize()
        ptr, stride = dhit.current_populations(box.handle)
        nbytes = dhit.population_buffer_bytes(box.params)
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        sums = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        dhit.device_copy(src.data_ptr(), ptr, nbytes, box.stream.cuda_stream)
        p = dhit.default_params(n, method, precision, nu)
        p.stream = box.stream.cuda_stream
        dhit.step_noalloc(p, src.data_ptr(), dst.data_ptr(), sums.data_ptr())
        box.step(1)
        box.synchronize()
        ref = box.populations_tensor()
        dt = torch.float64 if precision == "fp64" else torch.float32
        got = dst.view(dt).view(19, stride)[:, : n ** 3]
        assert torch.equal(got, ref), (method, precision, n)
        hist = box.sums_history(1)[0]
        np.testing.assert_array_equal(sums.cpu().numpy(), hist)
        # the source buffer is left as it was
        assert torch.equal(src.view(dt).view(19, stride)[:, : n ** 3],
                           torch.from_numpy(f0.reshape(19, -1)).to(device="cuda", dtype=dt))


@pytest.mark.parametrize("method,precision", CASES)
def test_noalloc_step_equals_box_step(method, precision):
    import torch
    _noalloc_against_box(torch, method, precision, 40, seed=11)
    _noalloc_against_box(torch, method, precision, 9, seed=12)


def test_noalloc_rejects_what_it_cannot_hold():
    """Host-side checks: a box whose reduction exceeds the static work space,
    the two-pass DUGKS form, a shared source and destination."""
    import torch
    buf = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    big = dhit.default_params(323, "bgk", "fp64", 0.01)
    with pytest.raises(dhit.DhitError) as e:
        dhit.step_noalloc(big, buf.data_ptr(), buf.data_ptr() + 256)
    assert e.value.code == -1 and "322" in str(e.value)
    tp = dhit.default_params(8, "dugks", "fp64", 0.01)
    tp.variant = dhit.VARIANT_TWO_PASS
    with pytest.raises(dhit.DhitError):
        dhit.step_noalloc(tp, buf.data_ptr(), buf.data_ptr() + 256)
    same = dhit.default_params(8, "bgk", "fp64", 0.01)
    with pytest.raises(dhit.DhitError):
        dhit.step_noalloc(same, buf.data_ptr(), buf.data_ptr())
