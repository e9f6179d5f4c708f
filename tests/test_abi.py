"""The C-ABI library builds for gfx950, loads, and exports every declared entry point (no GPU needed)."""
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:gz_status|const\s+char\s*\*|void|uint32_t|int32_t|uint64_t)\s+"
                             r"\**\s*(gz_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def libgz():
    from paper_2203_14927_amd import LIB_PATH, lib

    if not os.path.exists(LIB_PATH):
        from paper_2203_14927_amd import build_lib

        build_lib.build()
    return lib()


def test_headers_declare_the_boundary():
    names = _declared()
    for required in ["gz_sketch_init", "gz_update_sketch_batch", "gz_ingest", "gz_ingest_multi",
                     "gz_flush", "gz_connected_components", "gz_list_spanning_forest",
                     "gz_export_sketches", "gz_free", "gz_status_str"]:
        assert required in names


def test_library_exports_every_declared_symbol(libgz):
    from paper_2203_14927_amd import LIB_PATH

    out = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    for n in _declared():
        assert hasattr(libgz, n)


def test_library_is_built_for_gfx950():
    from paper_2203_14927_amd import LIB_PATH

    data = open(LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_status_strings(libgz):
    assert libgz.gz_status_str(0) == b"GZ_OK"
    assert libgz.gz_status_str(4) == b"GZ_ESKETCH_FAIL"
    assert libgz.gz_status_str(99) == b"GZ_UNKNOWN"


def test_package_has_no_cpu_fallback():
    """The product path never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2203_14927_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*.py"), recursive=True):
        src = open(path).read()
        assert "import oracle" not in src and "from oracle" not in src, path


def _prototypes():
    """name -> list of parameter type strings, parsed from include/*.h."""
    protos = {}
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        for m in re.finditer(r"(?:gz_status|const\s+char\s*\*|void|uint32_t|int32_t|uint64_t)\s+"
                             r"\**\s*(gz_\w+)\s*\(([^)]*)\)\s*;", text):
            params = [p.strip() for p in m.group(2).replace("\n", " ").split(",")]
            params = [] if params == ["void"] or params == [""] else params
            protos[m.group(1)] = [re.sub(r"\s+\w+$", "", p) for p in params]
    return protos


def _kind_of_c(t):
    t = t.replace("const ", "").strip()
    if "*" in t or t in ("hipStream_t",):
        return "ptr"
    return {"uint32_t": "u32", "int32_t": "i32", "uint64_t": "u64", "int": "i32",
            "gz_status": "i32"}[t]


def _kind_of_ctypes(ct):
    import ctypes

    if ct in (ctypes.c_void_p, ctypes.c_char_p) or hasattr(ct, "_type_") and ct.__name__.startswith("LP_"):
        return "ptr"
    return {ctypes.c_uint32: "u32", ctypes.c_int32: "i32", ctypes.c_uint64: "u64",
            ctypes.c_int: "i32"}[ct]


def test_binding_signatures_follow_the_header(libgz):
    """Every entry point the binding declares has the header's parameter list (count and kinds);
    in particular gz_ingest takes (g, src, dst, op, N, flags, stream)."""
    protos = _prototypes()
    assert protos["gz_ingest"] == ["gz_graph*", "const uint32_t*", "const uint32_t*",
                                   "const uint8_t*", "uint64_t", "uint32_t", "hipStream_t"]
    checked = 0
    for name, proto in protos.items():
        fn = getattr(libgz, name)
        if fn.argtypes is None:
            continue
        assert len(fn.argtypes) == len(proto), name
        assert [_kind_of_ctypes(a) for a in fn.argtypes] == [_kind_of_c(p) for p in proto], name
        checked += 1
    assert checked >= 30
