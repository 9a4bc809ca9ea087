"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/dhit.h declares, and validates parameters before touching
the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dhit.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"(?m)^(?:const\s+)?(?:int32_t|int64_t|char|void)\s*\*?\s*([a-z_][a-z0-9_]*)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("create_box", "init_velocity_field", "step_lbe", "step_dugks", "moments",
                     "energy_spectrum"):
        assert required in names
    assert len(names) >= 15


def test_library_exports_every_declared_symbol():
    import paper_1601_03815_amd._binding as b
    lib = ctypes.CDLL(b.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(b.EXPORTED) == declared_functions()


def test_default_params_are_the_papers():
    import paper_1601_03815_amd as dhit
    p = dhit.default_params(128, "mrt", "fp64", 0.012395)
    assert (p.s1, p.s2, p.s4, p.s10, p.s16) == (1.19, 1.4, 1.2, 1.4, 1.98)
    assert p.s9 == p.s13 == 1.0 / (3 * 0.012395 + 0.5)
    assert (p.w_eps, p.w_epsj, p.w_xx) == (0.0, -475.0 / 63.0, 0.0)
    assert p.dt == 1.0 and p.rho0 == 1.0
    assert dhit.default_params(64, "dugks", "fp32", 0.01).dt == 0.5


def test_buffer_sizes():
    import paper_1601_03815_amd as dhit
    p64 = dhit.default_params(256, "bgk", "fp64", 0.01)
    p32 = dhit.default_params(256, "bgk", "fp32", 0.01)
    b64 = dhit.population_buffer_bytes(p64)
    b32 = dhit.population_buffer_bytes(p32)
    assert b64 >= 19 * 256 ** 3 * 8 and b64 < 19 * 256 ** 3 * 8 * 1.01
    assert b32 >= 19 * 256 ** 3 * 4 and b32 < 19 * 256 ** 3 * 4 * 1.01
    assert dhit.box_bytes(p64) >= 2 * b64
    pd = dhit.default_params(256, "dugks", "fp64", 0.01)
    assert 2 * b64 <= dhit.box_bytes(pd) < 2.1 * b64      # fused kernel: no scratch field
    pd.variant = dhit.VARIANT_TWO_PASS
    assert dhit.box_bytes(pd) >= 3 * b64                  # two-pass: transform scratch field


@pytest.mark.parametrize("field,value", [("n", 3), ("n", 2000), ("nu", 0.0), ("nu", -1.0),
                                          ("rho0", 0.0), ("method", 7), ("precision", 5),
                                          ("dt", 0.5), ("variant", 9)])
def test_invalid_parameters_are_rejected(field, value):
    import paper_1601_03815_amd as dhit
    p = dhit.default_params(8, "bgk", "fp64", 0.01)
    setattr(p, field, value)
    with pytest.raises(dhit.DhitError) as e:
        dhit.create_box(p)
    assert e.value.code == -1
    assert dhit.last_error()


def test_dugks_cfl_is_checked():
    import paper_1601_03815_amd as dhit
    p = dhit.default_params(8, "dugks", "fp64", 0.01)
    p.dt = 0.75   # CFL = 0.75 sqrt(2) > 1
    with pytest.raises(dhit.DhitError):
        dhit.create_box(p)


def test_mrt_rates_are_checked():
    import paper_1601_03815_amd as dhit
    p = dhit.default_params(8, "mrt", "fp64", 0.01)
    p.s1 = 2.5
    with pytest.raises(dhit.DhitError):
        dhit.create_box(p)
