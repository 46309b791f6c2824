"""Host-side checks of libpyjac_mi355x.so that need no GPU: the library loads,
exports every entry point include/pyjac.h declares, and its mechanism loader
rejects malformed or unsupported mechanisms before touching a device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT, tiny

HEADER = os.path.join(ROOT, "include", "pyjac.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1605_03262_amd import _lib
    return _lib.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pyjac_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    from paper_1605_03262_amd import _lib
    assert sorted(_lib.EXPORTED) == names


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        s = lib.pyjac_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.pyjac_status_string(-99).decode() == "unknown status"


def _load_status(lib, text):
    h = ctypes.c_void_p()
    rc = lib.pyjac_mech_load_string(text.encode(), 0, ctypes.byref(h))
    return rc, lib.pyjac_last_error().decode(), h.value


def test_loader_rejects_unbalanced(lib):
    mech = tiny(301, {"elementary": 2})
    text = mech.to_text()
    r = mech.reactions[0]
    names = [sp.name for sp in mech.species]
    prod = "products %d " % len(r.prod) + " ".join(f"{names[k]} {n}" for k, n in r.prod)
    bad = text.replace(prod, f"products 1 {names[-1]} 1", 1)   # inert Ar as the only product
    assert bad != text
    rc, msg, h = _load_status(lib, bad)
    assert rc == -7 and "not conserved" in msg and not h


@pytest.mark.parametrize("mutation,code", [
    (lambda t: t.replace("pyjac-mech 1", "pyjac-mech 2"), -3),
    (lambda t: t.replace("reactions ", "reactionz ", 1), -2),
    (lambda t: t.replace(" end\n", "\n").rstrip() [:-3], -2),
    (lambda t: t.replace("reaction elementary kc", "reaction photolysis kc", 1), -3),
])
def test_loader_rejects_malformed(lib, mutation, code):
    text = tiny(302, {"elementary": 2, "thirdbody": 1}).to_text()
    rc, msg, h = _load_status(lib, mutation(text))
    assert rc == code, msg
    assert msg and not h


def test_loader_null_arguments(lib):
    assert lib.pyjac_mech_load_string(None, 0, None) == -1
    h = ctypes.c_void_p()
    assert lib.pyjac_mech_load(b"/nonexistent/mech.txt", 0, ctypes.byref(h)) == -6
    assert lib.pyjac_mech_free(None) == 0


def test_python_binding_refuses_missing_library(monkeypatch, tmp_path):
    from paper_1605_03262_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load_library()
