"""The C-ABI library loads and exports every function include/*.h declares
(no compute: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(coop_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1707_01989_amd import coop
    so = coop.library_path()
    if not os.path.exists(so):
        from paper_1707_01989_amd import build
        build.build_coop()
    return coop.load_library()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("coop_init", "coop_bfs", "coop_sssp", "coop_color", "coop_mis", "coop_wait",
                 "coop_set_target", "coop_fork_groups", "coop_injector_start", "coop_barrier_bench"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1707_01989_amd import coop
    assert sorted(coop.EXPORTS) == declared_functions()


def test_strerror_and_defaults_without_gpu(lib):
    from paper_1707_01989_amd import coop
    assert coop.coop_strerror(coop.COOP_E_TIMEOUT).startswith("barrier watchdog")
    assert coop.coop_strerror(0) == "ok"
    o = coop.make_opts()
    assert o.mode == coop.COOP_MODE_PLAIN and o.num_groups == 0


def test_init_rejects_bad_device_without_gpu(lib):
    h = ctypes.c_void_p()
    assert lib.coop_init(1 << 20, ctypes.byref(h)) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_1707_01989_amd import coop
    monkeypatch.setattr(coop, "_lib", None)
    monkeypatch.setattr(coop, "library_path", lambda: str(tmp_path / "missing.so"))
    with pytest.raises(coop.CoopLibraryMissing):
        coop.load_library()
