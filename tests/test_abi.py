"""The C-ABI library loads and exports every entry point that include/lbm.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("lbm_create", "lbm_set_solids", "lbm_step", "lbm_force_torque", "lbm_macros",
                 "lbm_workspace_bytes", "lbm_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol():
    so = os.path.join(ROOT, "paper_1906_05445_amd", "liblbm.so")
    if not os.path.exists(so):
        import sys

        sys.path.insert(0, ROOT)
        from paper_1906_05445_amd import build

        build.build()
    lib = ctypes.CDLL(so)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    from paper_1906_05445_amd import lbm

    assert sorted(lbm.EXPORTED) == _declared()


def test_workspace_sizing_and_validation_without_gpu():
    from paper_1906_05445_amd import lbm

    p, _ = lbm.make_params("D3Q19", "MRT", "F32", (128, 128, 128), 0.8)
    n = lbm.lbm_workspace_bytes(ctypes.byref(p), 1, 0, 0)
    assert n > 2 * 19 * 128 ** 3 * 4
    bad, _ = lbm.make_params("D3Q19", "MRT", "F32", (16, 16, 16), 0.5)
    assert lbm.lbm_workspace_bytes(ctypes.byref(bad), 1, 0, 0) == 0
    bad2, _ = lbm.make_params("D2Q9", "BGK", "F64", (16, 16, 2), 0.8)
    assert lbm.lbm_workspace_bytes(ctypes.byref(bad2), 1, 0, 0) == 0
    assert lbm.lbm_status_string(-4) == b"non-finite populations"


# the calls of the boundary that carry a step or a result of the method: each
# declaration's comment names the passage of the paper that defines it
CITED = ["lbm_workspace_bytes", "lbm_create", "lbm_set_solids", "lbm_set_lagrangian", "lbm_step",
         "lbm_force_torque", "lbm_force_history", "lbm_macros", "lbm_strain", "lbm_link_list",
         "lbm_get_f", "lbm_set_equilibrium", "lbm_batch_create", "lbm_batch_admit", "lbm_batch_step",
         "lbm_batch_poll", "lbm_batch_release"]


def _comment_before(src, name):
    """The comment block that documents `name`: the last /* ... */ before its
    declaration, with only declarations (no other comment) in between."""
    m = re.search(r"\b" + name + r"\s*\(", src)
    assert m, name
    head = src[: m.start()]
    end = head.rfind("*/")
    start = head.rfind("/*", 0, end)
    assert end > 0 and start >= 0, name
    between = head[end + 2:]
    assert "/*" not in between, name
    return head[start:end]


def test_declarations_cite_the_paper():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    missing = [n for n in CITED if not re.search(r"(Eq\.|Sec\.|Fig\.|App\.)\s*\d", _comment_before(src, n))]
    assert not missing, missing


def test_domain_boundaries_validate():
    """Domain boundaries (Sec. 3.4): open on x only, D2Q9 keeps z periodic, an
    open x axis needs nx >= 8 and |inflow| < 0.3; the outlet plane's buffer is
    part of the workspace."""
    from paper_1906_05445_amd import lbm

    def nbytes(lat, shape, bnd, inflow=0.0):
        p, _ = lbm.make_params(lat, "MRT", "F32", shape, 0.8, boundary=bnd, inflow=inflow)
        return lbm._lib.lbm_workspace_bytes(ctypes.byref(p), 1, 0, 0)

    per = nbytes("D3Q19", (32, 24, 20), ("periodic", "periodic", "periodic"))
    assert per > 0
    assert nbytes("D3Q19", (32, 24, 20), ("slip", "slip", "slip")) == per
    assert nbytes("D3Q19", (32, 24, 20), ("open", "slip", "slip"), 0.05) >= per + 24 * 20 * 4
    assert nbytes("D3Q19", (32, 24, 20), ("periodic", "open", "periodic")) == 0
    assert nbytes("D3Q19", (32, 24, 20), ("periodic", "periodic", "open")) == 0
    assert nbytes("D3Q19", (7, 24, 20), ("open", "slip", "slip")) == 0
    assert nbytes("D3Q19", (32, 24, 20), ("open", "slip", "slip"), 0.3) == 0
    assert nbytes("D2Q9", (32, 24, 1), ("open", "slip", "periodic"), 0.05) > 0
    assert nbytes("D2Q9", (32, 24, 1), ("open", "slip", "slip")) == 0


def test_lattice_size_limit():
    """Up to 2^31 - 1 cells (32-bit cell indices); population offsets are 64-bit, so the arrays may hold
    more than 2^31 values."""
    from paper_1906_05445_amd import lbm

    def nbytes(shape):
        p, _ = lbm.make_params("D3Q19", "MRT", "F32", shape, 0.8)
        return lbm._lib.lbm_workspace_bytes(ctypes.byref(p), 1, 4096, 1024)

    assert nbytes((1152, 576, 576)) > 0          # 3.8e8 cells, 7.3e9 values per array
    assert nbytes((2048, 1024, 1024)) == 0       # 2^31 cells
