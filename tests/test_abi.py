"""The C interface: header and library agree (CPU only, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtmc.h")
LIB = os.path.join(ROOT, "paper_1806_00205_amd", "librtmc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtmc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rtmc_load_mesh", "rtmc_build_bvh", "rtmc_load_tables", "rtmc_trace", "rtmc_trace_batch",
                     "rtmc_first_hit", "rtmc_create", "rtmc_destroy", "rtmc_last_error"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_export():
    import paper_1806_00205_amd as rt
    assert sorted(rt.EXPORTS) == declared_functions()


def test_package_import_does_not_load_the_library():
    import paper_1806_00205_amd as rt
    assert rt.LIB_PATH.endswith("librtmc.so")


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1806_00205_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "rtmc_oracle" not in text and "liboracle" not in text, f


def test_committed_traffic_counters_match_the_kernel_sources():
    """The traffic figure bench.py reports comes from a committed counter
    summary keyed by a hash of the traversal kernel's sources: it must belong
    to the kernel as it stands (else the figure would be reported as null)."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    for cfg in ("c3", "c1"):
        t = bench.load_traffic(cfg)
        assert t is not None, f"profiles/k_traverse_{cfg}_traffic.json was measured on other kernel sources"
        assert t["kernel"] == "k_traverse" and 0.0 < t["fetch_plus_write_bytes_per_alg_byte"] < 2.0
        assert t["bound"] in ("hbm", "alu")
