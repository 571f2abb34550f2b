"""The C-ABI library loads and exports every entry point its header declares;
argument checks that need no device answer on any machine."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import paper_2602_20826_amd as db
from paper_2602_20826_amd import dagbound as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dagbound.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dagbound_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = db.load_library()
    names = declared_functions()
    assert "dagbound_create_batch" in names and "dagbound_best_allocation" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTS) == names


def test_header_constants_match_binding():
    text = open(HEADER).read()
    for name, val in [("DAGBOUND_E_ARG", -1), ("DAGBOUND_E_CYCLE", -2), ("DAGBOUND_E_RANGE", -3),
                      ("DAGBOUND_E_DUP_EDGE", -4), ("DAGBOUND_E_OOM", -5), ("DAGBOUND_E_DEVICE", -6),
                      ("DAGBOUND_E_STATE", -7), ("DAGBOUND_E_OVERFLOW", -8),
                      ("DAGBOUND_E_UNSUPPORTED", -9)]:
        assert re.search(rf"{name}\s*=\s*{val}\b", text), name
    assert f"DAGBOUND_MAX_NODES_PER_DAG {binding.MAX_NODES_PER_DAG}" in text


def test_version_string():
    assert "gfx950" in db.version()


def _empty(d=1):
    return (np.zeros(d + 1, np.int64), np.zeros(d + 1, np.int64), np.zeros(0, np.int32),
            np.zeros(0, np.int32), np.zeros(0, np.int64), np.zeros(0, np.int32))


@pytest.mark.parametrize("M", [0, -3, 65536])
def test_bad_num_cus_rejected_before_device(M):
    with pytest.raises(db.DagboundError) as e:
        db.create_batch(*_empty(), M)
    assert e.value.code == binding.E_ARG


def test_null_arguments_rejected():
    lib = db.load_library()
    out = ctypes.c_void_p()
    no = np.zeros(2, np.int64)
    assert lib.dagbound_create_batch(1, no.ctypes.data, no.ctypes.data, None, None, None, None, 8, 0,
                                     None, None) == binding.E_ARG
    assert lib.dagbound_create_batch(-1, no.ctypes.data, no.ctypes.data, None, None, None, None, 8, 0,
                                     None, ctypes.byref(out)) == binding.E_ARG
    assert lib.dagbound_create_batch(1, None, None, None, None, None, None, 8, 0, None,
                                     ctypes.byref(out)) == binding.E_ARG
    assert lib.dagbound_create_batch(1, no.ctypes.data, no.ctypes.data, None, None, None, None, 8, 7,
                                     None, ctypes.byref(out)) == binding.E_ARG
    assert lib.dagbound_set_allocations(None, 4, 0, None, 0, 0) == binding.E_ARG
    assert lib.dagbound_eval_bounds(None, None, None, None, 0, None) == binding.E_ARG
    assert lib.dagbound_best_allocation(None, 0, 0, None, None, None, 0, None) == binding.E_ARG
    assert lib.dagbound_get_division(None, 0, None, None, None, None) == binding.E_ARG
    lib.dagbound_destroy_batch(None)
    assert "NULL" in db.last_error()


def test_binding_dtype_checks():
    with pytest.raises(TypeError):
        binding._marshal([(np.zeros(2, np.int32), "int64")])


def test_missing_library_fails_loudly():
    # with the shared library absent the binding raises on first use; there
    # is no other path that could compute a bound
    code = (
        "import numpy as np, workloads as W\n"
        "import paper_2602_20826_amd.dagbound as d\n"
        "d._lib = None\n"
        "d.load_library.__defaults__ = ('/nonexistent/libdagbound.so',)\n"
        "b = W.from_dags([(2, [0], [1], [3, 4], [1, 2])])\n"
        "try:\n"
        "    d.create_batch(b.node_off, b.edge_off, b.src, b.dst, b.wcet, b.par, 4)\n"
        "except ImportError as e:\n"
        "    print('raised', 'is not built' in str(e))\n"
    )
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "raised True"
