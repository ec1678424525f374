"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/ucp.h, and rejects bad arguments before touching the
device.  No compute calls are made here."""
import ctypes as C
import os
import re

import pytest

from paper_0709_3331_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ucp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ucp_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = L.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_oracle_is_not_linked_into_the_library():
    with open(L.LIBPATH, "rb") as fh:
        blob = fh.read()
    assert b"orc_tree_new" not in blob and b"ucp_oracle" not in blob


def test_default_params_and_version():
    p = L.default_params()
    assert p.theta == 0.5 and p.key_bits == 63 and p.leaf_cap == 24 and p.group_size == 64
    assert p.precision == L.UCP_SPLIT and p.group_mode == L.UCP_GROUP_CHUNK
    assert p.pair_law == L.UCP_PAIR_PLUMMER and p.lambda_ei == 0.0
    assert p.expansion == L.UCP_EXPANSION_QUADRUPOLE
    assert p.curve == L.UCP_CURVE_HILBERT
    assert L.ucp_version() >= 100


@pytest.mark.parametrize("over", [dict(theta=-0.1), dict(theta=1.2), dict(eps=0.0),
                                  dict(key_bits=32), dict(leaf_cap=0), dict(leaf_cap=65),
                                  dict(group_size=0), dict(group_size=65), dict(list_len=8), dict(list_len=600),
                                  dict(precision=3), dict(group_mode=2), dict(group_mode=-1),
                                  dict(pair_law=2), dict(pair_law=1, lambda_ei=0.0),
                                  dict(pair_law=1, lambda_ei=-0.5),
                                  dict(pair_law=1, lambda_ei=0.1, eps=-1.0),
                                  dict(expansion=2), dict(expansion=-1),
                                  dict(curve=2), dict(curve=-1)])
def test_create_rejects_bad_params_without_gpu(over):
    p = L.default_params(**over)
    with pytest.raises(L.UcpError) as ei:
        L.ucp_create(1000, 1, p)
    assert ei.value.status == L.UCP_EINVAL


def test_create_rejects_bad_sizes_without_gpu():
    p = L.default_params()
    for n_max, clouds in [(0, 1), (-5, 1), (1 << 29, 1), (10, 0), (10, 70000)]:
        with pytest.raises(L.UcpError) as ei:
            L.ucp_create(n_max, clouds, p)
        assert ei.value.status == L.UCP_EINVAL
    assert "n_max" in L.ucp_last_error(None) or "clouds" in L.ucp_last_error(None)


def test_null_context_is_rejected():
    lib = L.load()
    assert lib.ucp_build_tree(None, None, None, 0, None) == L.UCP_EINVAL
    assert lib.ucp_compute_forces(None, None, None, None) == L.UCP_EINVAL
    st = L.ucp_stats()
    assert lib.ucp_get_stats(None, C.byref(st), None) == L.UCP_EINVAL
