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


def test_create_rejects_more_particles_than_the_charge_scan_holds(lib):
    """The exact-integer trapezoid scan sums up to 2 N 2^32 in u64, and the
    learned fallback queue holds 32-bit indices: N >= 2^31 is refused before
    any device work."""
    for n in (2 ** 31, 2 ** 40):
        with pytest.raises(capi.EtdpicError) as ei:
            capi.ep_create(n_particles=n)
        assert ei.value.status == capi.EP_EINVAL
        assert "2^31" in capi.ep_last_error(None)


def test_foreign_hip_runtime_is_detected(tmp_path):
    """A process map naming a HIP runtime outside ROCm's library directory is
    reported (the library refuses to load beside it); ROCm's own is not."""
    own = os.path.realpath(capi.ROCM_HIP_RUNTIME)
    other = "/usr/lib/python3/site-packages/framework/lib/libamdhip64.so"
    maps = tmp_path / "maps"
    maps.write_text("7f00-7f10 r-xp 00000000 08:01 1 %s\n7f20-7f30 r--p 00000000 08:01 2 %s\n"
                    "7f40-7f50 r--p 00000000 08:01 3 /usr/lib/libc.so.6\n" % (own, other))
    assert capi.foreign_hip_runtimes(str(maps)) == [other]
    maps.write_text("7f00-7f10 r-xp 00000000 08:01 1 %s\n" % own)
    assert capi.foreign_hip_runtimes(str(maps)) == []


def test_library_refuses_a_process_with_another_hip_runtime():
    """In a process that has loaded a framework's bundled HIP runtime (here
    PyTorch's, if importable), loading the library raises instead of sharing
    the process with a second runtime."""
    import subprocess
    import sys
    code = ("import torch\n"
            "from paper_1404_1160_amd import capi\n"
            "if not capi.foreign_hip_runtimes():\n"
            "    print('NO_FOREIGN_RUNTIME'); raise SystemExit(0)\n"
            "try:\n"
            "    capi.lib()\n"
            "except ImportError as e:\n"
            "    print('REFUSED', e); raise SystemExit(0)\n"
            "raise SystemExit('loaded beside a foreign HIP runtime')\n")
    try:
        import importlib.util
        if importlib.util.find_spec("torch") is None:
            pytest.skip("no framework with a bundled HIP runtime is installed")
    except ImportError:
        pytest.skip("no framework with a bundled HIP runtime is installed")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    if "NO_FOREIGN_RUNTIME" in r.stdout:
        pytest.skip("this framework build maps no HIP runtime of its own")
    assert "REFUSED" in r.stdout


def test_null_context_is_rejected(lib):
    assert lib.ep_step(None, 0.1, 0.1, 1, 1) == capi.EP_EINVAL
    assert lib.ep_sync(None) == capi.EP_EINVAL
    assert lib.ep_mlp_set_projection(None, 1) == capi.EP_EINVAL
    assert lib.ep_mlp_set_precision(None, 0) == capi.EP_EINVAL
    assert lib.ep_timing_enable(None, 5) == capi.EP_EINVAL
    assert lib.ep_destroy(None) == capi.EP_OK
