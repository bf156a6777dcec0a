"""CPU checks of the C-ABI boundary: the library loads, exports every entry
point declared in include/mmx.h, and rejects bad arguments before touching the
GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmx.h")


def _declared():
    text = open(HEADER).read()
    decl = r"^\s*(?:mmx_status|void|const char\s*\*)\s*(mmx_[a-z0-9_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mmx_create", "mmx_destroy", "mmx_set_material", "mmx_build_demag",
                 "mmx_field", "mmx_torque", "mmx_heun", "mmx_rk45", "mmx_energy",
                 "mmx_topological_charge", "mmx_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2608_15253_amd as mmx
    lib = ctypes.CDLL(mmx.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(mmx.EXPORTED) == _declared()


def test_argument_errors_are_reported_without_a_gpu():
    import paper_2608_15253_amd as mmx
    with pytest.raises(mmx.MMXError) as e:
        mmx.mmx_create([], mmx.MMX_F32)
    assert e.value.status == -1
    g = mmx.make_group((4, 4, 1), (1e-9, 1e-9, 1e-9), replicas=0)
    with pytest.raises(mmx.MMXError) as e:
        mmx.mmx_create([g], mmx.MMX_F32)
    assert e.value.status == -2
    g = mmx.make_group((4, 4, 1), (1e-9, 1e-9, 1e-9))
    with pytest.raises(mmx.MMXError) as e:
        mmx.mmx_create([g], 7)
    assert e.value.status == -1
    with pytest.raises(mmx.MMXError):
        mmx.mmx_set_terms(None, 1)
    assert "context" in mmx.mmx_last_error()


def test_library_has_no_oracle_dependency():
    # the product path never imports the oracle
    pkg = os.path.join(ROOT, "paper_2608_15253_amd")
    files = [os.path.join(pkg, f) for f in os.listdir(pkg) if f.endswith(".py")]
    files += [os.path.join(pkg, "csrc", f) for f in os.listdir(os.path.join(pkg, "csrc"))]
    for f in files:
        src = open(f).read()
        assert "import oracle" not in src and "from oracle" not in src, f
