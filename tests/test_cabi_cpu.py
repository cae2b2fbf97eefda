"""The C-ABI library loads and exports every function include/gdn.h declares.
Only host-side entry points are called (no GPU in this tier)."""
import ctypes as C
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def libgdn():
    from paper_2512_10386_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gdn.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gdn_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["gdn_default_params", "gdn_create", "gdn_destroy", "gdn_workspace_size",
              "gdn_denoise", "gdn_debug_dump", "gdn_status_string", "gdn_last_error"]:
        assert f in names


def test_library_exports_every_declared_symbol(libgdn):
    lib = C.CDLL(libgdn.LIB_PATH)
    for f in declared_functions():
        assert hasattr(lib, f), f


def test_defaults_match_the_paper_and_the_oracle(libgdn, oracle):
    p = libgdn.gdn_default_params()
    o = oracle.default_params()
    for f, _ in libgdn.gdn_params._fields_:
        if f == "knn_chunk":  # work split of the kNN kernel: speed only, not a method parameter
            assert p.knn_chunk == 0
            continue
        a, b = getattr(p, f), o[f]
        assert a == b or (math.isnan(a) and math.isnan(b)), f
    assert (p.k, p.rho_percentile, p.min_vox_count) == (12, 0.2, 4)


def test_workspace_size_and_validation_on_host(libgdn):
    p = libgdn.make_params(k=32, leaf_cap=1024)
    small = libgdn.gdn_workspace_size(0, p, 1000)
    big = libgdn.gdn_workspace_size(0, p, 120000)
    assert 0 < small < big
    assert libgdn.gdn_workspace_size(0, p, 0) == 0
    with pytest.raises(libgdn.GdnError) as e:
        libgdn.gdn_workspace_size(0, libgdn.make_params(k=65), 10)
    assert e.value.status == libgdn.GDN_EINVAL
    with pytest.raises(libgdn.GdnError) as e:
        libgdn.gdn_workspace_size(0, p, 1 << 30)
    assert e.value.status == libgdn.GDN_ECAPACITY
    assert libgdn.lib().gdn_status_string(libgdn.GDN_ENOMEM) == b"workspace too small"


def test_batch_workspace_size_and_validation_on_host(libgdn):
    p = libgdn.make_params(k=32, leaf_cap=1024)
    one = libgdn.gdn_workspace_size(0, p, 120000)
    assert libgdn.gdn_workspace_size_batch(0, p, 120000, 1) == one
    many = libgdn.gdn_workspace_size_batch(0, p, 120000, 64)
    assert many > one  # frame table, frame ids and kept ranks
    assert libgdn.gdn_workspace_size_batch(0, p, 0, 5) == 0
    for nf, status in ((0, libgdn.GDN_EINVAL), (libgdn.GDN_MAX_FRAMES + 1, libgdn.GDN_ECAPACITY)):
        with pytest.raises(libgdn.GdnError) as e:
            libgdn.gdn_workspace_size_batch(0, p, 1000, nf)
        assert e.value.status == status
    libgdn.gdn_workspace_size_batch(0, p, 1000, libgdn.GDN_MAX_FRAMES)
    with pytest.raises(libgdn.GdnError) as e:
        libgdn.gdn_workspace_size(0, libgdn.make_params(knn_chunk=-1), 10)
    assert e.value.status == libgdn.GDN_EINVAL


def test_library_matches_its_sources(libgdn, monkeypatch):
    """The loaded library carries the hash of the sources it was built from;
    a library built from other sources is refused."""
    from paper_2512_10386_amd import build
    lib = C.CDLL(libgdn.LIB_PATH)
    lib.gdn_source_hash.restype = C.c_char_p
    assert lib.gdn_source_hash().decode() == build.source_hash()
    monkeypatch.setattr(libgdn, "_lib", None)
    monkeypatch.setattr(build, "source_hash", lambda: "0" * 64)
    with pytest.raises(RuntimeError, match="stale"):
        libgdn.lib()
