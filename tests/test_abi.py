"""The C-ABI library loads and exports every symbol include/binv.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2305_11103_amd", "libbinv.so")


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "binv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(binv_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ("binv_create", "binv_destroy", "binv_invert", "binv_last_error"):
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s), s


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_declared_symbol():
    from paper_2305_11103_amd import binv
    assert sorted(binv.EXPORTS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_version_string():
    from paper_2305_11103_amd import binv
    lib = binv.load_library()
    assert lib.binv_version().decode().startswith("binv")


def test_tier_shape_table():
    """Launch-shape table of the batched tiers (host-only query)."""
    from paper_2305_11103_amd import binv
    for t, count in enumerate(binv.TIER_SHAPES):
        for v in range(count):
            rpl, cpw, nwv, sub = binv.batch_shape(t, v)
            limit = binv.TIER_LIMITS[t]
            assert nwv * cpw >= limit and nwv * cpw <= 64 * rpl  # columns cover the tier, rows cover the columns
            assert 64 * nwv * sub <= 1024
        with pytest.raises(binv.BinvError):
            binv.batch_shape(t, count)


def test_binding_shares_torch_hip_runtime():
    """Loading the library through the binding, before anything imports
    torch, maps a single HIP runtime: torch's (it ships its own copy)."""
    import subprocess
    import sys
    code = ("from paper_2305_11103_amd import binv\n"
            "binv.load_library()\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    import ast
    libs = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1 and "torch" in libs[0], libs


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_level_partition_is_table2():
    """binv_level_partition (host only) against the rows printed in Table 2
    and the oracle's partitioner for every order up to 4096."""
    from oracle import level_scheme as ls
    from paper_2305_11103_amd import binv
    rows = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "table2_partitions.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, v = line.split(":")
            rows[int(k)] = [int(x) for x in v.split()]
    for m, blocks in rows.items():
        assert binv.level_partition(m) == blocks
    for m in range(1, 4097):
        assert binv.level_partition(m) == ls.table2_partition(m)
    with pytest.raises(binv.BinvError):
        binv.level_partition(0)
