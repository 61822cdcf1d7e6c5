"""The C-ABI library loads and exports every entry point declared in
include/lp.h (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(lp_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("lp_compress", "lp_decompress", "lp_cluster", "lp_contract", "lp_edge_cut",
                     "lp_graph_free", "lp_strerror", "lp_graph_info"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2410_19119_amd as m
    lib = m._load()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    assert set(m.exported_symbols()) == set(declared_symbols())
    assert lib.lp_strerror(-3).decode() == "coarse weight exceeds INT32_MAX"
    assert b"gfx950" in lib.lp_version()


def test_library_is_built_for_gfx950():
    import paper_2410_19119_amd as m
    data = open(m._LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_product_path_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2410_19119_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f), errors="ignore").read()
                assert "import oracle" not in src and "liboracle" not in src, f
