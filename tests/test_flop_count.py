"""The flop counts that bench.py uses for the arithmetic roofline of the operator kernels
match the element code: tests/native/flop_count.cpp instantiates the library's element
header on a counting scalar type."""

import ctypes
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def counts():
    out = os.path.join(tempfile.mkdtemp(prefix="nc_flops_"), "libflops.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", out,
                           os.path.join(HERE, "native", "flop_count.cpp")])
    lib = ctypes.CDLL(out)
    arr = (ctypes.c_long * 6)()
    lib.fc_counts(arr)
    return dict(zip(["lin", "jv5", "jtw5", "jv2", "jtw2", "residual5"], arr))


def test_bench_flop_constants_match_element_code():
    import bench
    c = counts()
    assert bench.FLOPS_PER_ELEM["jv"] == c["lin"] + c["jv2"]
    assert bench.FLOPS_PER_ELEM["jtw"] == c["lin"] + c["jtw2"]
    assert bench.FLOPS_PER_ELEM["smooth"] == c["lin"] + c["jv2"]
    assert bench.FLOPS_PER_ELEM["smooth_T"] == c["lin"] + c["jtw2"]
    assert bench.FLOPS_PER_ELEM["pt_residual"] == c["lin"] + c["jv2"]


def test_counts_are_plausible():
    """The five-field apply does strictly more work than the two-field one, and the
    element work sits in the range of a sum-factorised trilinear element (1-3 kflop)."""
    c = counts()
    assert c["jv5"] > c["jv2"] and c["jtw5"] > c["jtw2"]
    assert 1000 <= c["lin"] + c["jtw5"] <= 3000 or 900 <= c["lin"] + c["jv5"] <= 3000
