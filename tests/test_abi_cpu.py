"""CPU-side checks of the boundary: the library loads without a GPU and
exports every entry point declared in include/*.h; the Python binding's
struct layouts match the header's field order."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hprqp_[a-z_0-9]+)\s*\(", src)))


def _lib():
    from paper_2507_02470_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.skip("libhprqp.so not built (run __graft_entry__.build())")
    return _native.load()


def test_library_exports_every_declared_symbol():
    lib = _lib()
    names = _declared("hprqp.h")
    assert "hprqp_create" in names and "hprqp_solve_batch" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_default_options_without_gpu():
    lib = _lib()
    from paper_2507_02470_amd.solver import default_options
    o = default_options()
    assert o.tol == 1e-8 and o.check_every == 100
    assert (o.alpha1, o.alpha2, o.alpha3) == (0.2, 0.8, 0.5)
    assert o.enable_restart == 1 and o.enable_sigma_update == 1
    assert o.precondition == 0 and o.ruiz_iters == 10 and o.spmv_lanes == -1 and o.method == 0
    assert o.kron_kernel == -1 and o.small_path == -1


def _struct_fields(header, name):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    end = re.search(r"\}\s*" + name + r"\s*;", src).start()
    start = src.rindex("typedef struct {", 0, end) + len("typedef struct {")
    body = src[start:end]
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        decl = re.sub(r"^(const\s+)?\w+\s*", "", decl)       # drop the type
        for part in decl.split(","):
            fields.append(part.strip().lstrip("*").strip())
    return fields


@pytest.mark.parametrize("cname,pyname", [("hprqp_problem", "hprqp_problem"), ("hprqp_options", "hprqp_options"),
                                          ("hprqp_info", "hprqp_info")])
def test_binding_structs_follow_the_header(cname, pyname):
    from paper_2507_02470_amd import _native
    hdr = _struct_fields("hprqp.h", cname)
    py = [f[0] for f in getattr(_native, pyname)._fields_]
    assert hdr == py


def test_product_path_raises_without_library(tmp_path, monkeypatch):
    from paper_2507_02470_amd import _native
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(RuntimeError, match="not found"):
        _native.load()
