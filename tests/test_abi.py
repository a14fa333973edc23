"""The C-ABI library loads and exports every symbol its header declares (no GPU)."""
import os
import re

import pytest

from paper_1404_1160_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(ep_[a-z_0-9]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(capi.library_path()):
        from paper_1404_1160_amd import build
        build.build()
    return capi.lib()


def test_header_declares_the_binding_names():
    assert _header_symbols() == set(capi.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _header_symbols():
        assert hasattr(lib, name), name


def test_library_is_gfx950_code_object():
    data = open(capi.library_path(), "rb").read()
    assert b"gfx950" in data


def test_create_rejects_bad_configuration(lib):
    """Host-side validation returns EP_EINVAL before any device work."""
    for kw in [dict(n_cells=255), dict(n_cells=0), dict(substeps=0), dict(r_max=-1.0),
               dict(n_cells=16384), dict(deposit=7)]:
        args = dict(n_particles=16, n_cells=256, substeps=1, r_max=5.0)
        args.update(kw)
        with pytest.raises(capi.EtdpicError) as ei:
            capi.ep_create(**args)
        assert ei.value.status == capi.EP_EINVAL
        assert capi.ep_last_error(None)
    with pytest.raises(capi.EtdpicError):
        capi.ep_create(n_particles=0)


def test_null_context_is_rejected(lib):
    assert lib.ep_step(None, 0.1, 0.1, 1, 1) == capi.EP_EINVAL
    assert lib.ep_sync(None) == capi.EP_EINVAL
    assert lib.ep_destroy(None) == capi.EP_OK
