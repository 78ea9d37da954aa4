"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and reports errors instead of aborting."""

import ctypes
import json
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "g6mi.h")
GOLDEN = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_constants.json")))


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(g6\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def g6():
    import paper_0902_4463_amd as g6
    return g6


def test_header_declares_grape_sequence():
    names = declared_functions()
    for n in ("g6_open", "g6_close", "g6_npipes", "g6_set_j_particle", "g6_set_ti",
              "g6calc_firsthalf", "g6calc_lasthalf", "g6calc_lasthalf2", "g6_nearest_neighbour",
              "g6_read_neighbour_list", "g6_get_neighbour_list", "g6mi_calc_device"):
        assert n in names
        assert n + "_" in names or n.startswith("g6mi")  # every GRAPE call has its Fortran alias


def test_every_declared_symbol_is_exported(g6):
    lib = ctypes.CDLL(g6.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_c_names(g6):
    for n in declared_functions():
        if n.endswith("_") and not n.startswith("g6mi"):
            continue  # Fortran aliases are for Fortran callers
        assert hasattr(g6, n), n


def test_constants_match_paper(g6):
    assert g6.g6mi_nb_max() == GOLDEN["neighbour_list_cap"]["value"]
    assert g6.NB_MAX == g6.g6mi_nb_max()
    old = os.environ.pop("G6MI_NPIPES", None)
    try:
        assert g6.g6_npipes() == GOLDEN["npipes"]["value"]
        os.environ["G6MI_NPIPES"] = "1048576"
        assert g6.g6_npipes() == 1048576
        os.environ["G6MI_NPIPES"] = "0"
        assert g6.g6_npipes() == GOLDEN["npipes"]["value"]
    finally:
        os.environ.pop("G6MI_NPIPES", None)
        if old is not None:
            os.environ["G6MI_NPIPES"] = old


def test_header_constants_agree_with_binding(g6):
    text = open(HEADER).read()
    consts = dict(re.findall(r"#define\s+(G6MI_\w+)\s+\(?(-?\d+)\)?", text))
    assert int(consts["G6MI_NB_MAX"]) == g6.NB_MAX
    assert int(consts["G6MI_NPIPES_DEFAULT"]) == g6.NPIPES_DEFAULT
    assert int(consts["G6MI_PREC_DS"]) == g6.PREC_DS
    assert int(consts["G6MI_EDEVICE"]) == g6.EDEVICE
    assert int(consts["G6MI_MAX_HANDLES"]) == g6.MAX_HANDLES


def _struct_fields(text, name):
    body = re.search(r"typedef struct " + name + r" \{(.*?)\} " + name + ";", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return re.findall(r"\b(int|double)\s+(\w+);", body)


def test_batch_structs_match_header(g6):
    """The binding's mirrors of g6mi_cluster and g6mi_batch_tuning have the
    header's fields, in order, with the same sizes."""
    text = open(HEADER).read()
    cl = _struct_fields(text, "g6mi_cluster")
    assert [n for _, n in cl] == list(g6.CLUSTER_DTYPE.names)
    size = {"int": 4, "double": 8}
    for (ty, n) in cl:
        assert g6.CLUSTER_DTYPE[n].itemsize == size[ty]
    assert sum(size[t] for t, _ in cl) == g6.CLUSTER_DTYPE.itemsize == 32
    tu = _struct_fields(text, "g6mi_batch_tuning")
    assert [n for _, n in tu] == [n for n, _ in g6.BatchTuning._fields_]


def test_errors_not_aborts_without_gpu(g6):
    """In a process that has no GPU, g6_open reports G6MI_EDEVICE and every
    handle call reports that the handle is not open."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert g6.g6_open(0) == g6.EDEVICE
    assert "device" in g6.last_error(0)
    assert g6.g6_open(-1) == g6.EINVAL
    assert g6.g6_open(g6.MAX_HANDLES) == g6.EINVAL
    z = np.zeros(3)
    assert g6.g6_set_j_particle(0, 0, 0, 0.0, 0.0, 1.0, z, z, z, z, z) == g6.ESTATE
    assert g6.g6calc_firsthalf(0, 0, 0, [], np.zeros((0, 3)), np.zeros((0, 3)), None, None, None, 0.0, None) == g6.ESTATE
    acc = np.zeros((0, 3))
    assert g6.g6calc_lasthalf(0, 0, 0, [], None, None, 0.0, None, acc, acc, np.zeros(0)) == g6.ESTATE
    assert g6.g6_read_neighbour_list(0) == g6.ESTATE
    assert g6.g6mi_set_precision(0, "ds") == g6.ESTATE
    assert g6.g6_close(0) == g6.ESTATE
    assert g6.g6_close(g6.MAX_HANDLES + 1) == g6.EINVAL
    cl = g6.clusters([0], [1], [0], [1], [0.0], [0.0])
    assert g6.g6mi_batch_calc(0, cl, 1, 1, 1, 1, 1, 1, 1, 1) == g6.ESTATE
    assert g6.g6mi_batch_calc_device(0, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1) == g6.ESTATE
    assert g6.g6mi_batch_use_graph(0, 1) == g6.ESTATE
    assert g6.g6mi_batch_set_tuning(0, None) == g6.ESTATE
    flags = np.zeros(1, dtype=np.int32)
    assert g6._L().g6mi_last_status(0, g6._pi(flags)) == g6.ESTATE


def test_fortran_aliases_take_addresses(g6):
    lib = ctypes.CDLL(g6.LIB_PATH)
    f = lib.g6_npipes_
    f.restype = ctypes.c_int
    assert f() == g6.g6_npipes()
    op = lib.g6_open_
    op.restype = ctypes.c_int
    op.argtypes = [ctypes.POINTER(ctypes.c_int)]
    bad = ctypes.c_int(-5)
    assert op(ctypes.byref(bad)) == g6.EINVAL


def test_nearest_neighbour_alias_forwards(g6):
    """The Fortran alias reads id and ni by address and returns what the C
    call returns (here: the error for a handle that is not open)."""
    lib = ctypes.CDLL(g6.LIB_PATH)
    f = lib.g6_nearest_neighbour_
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.c_void_p]
    nnb = np.zeros(4, dtype=np.int32)
    r2 = np.zeros(4)
    for hid in (0, 7, -3):
        want = g6.g6_nearest_neighbour(hid, 4, nnb, r2)
        got = f(ctypes.byref(ctypes.c_int(hid)), ctypes.byref(ctypes.c_int(4)), nnb.ctypes.data, r2.ctypes.data)
        assert got == want and got < 0


def test_header_compiles_as_c11_and_links(g6, tmp_path):
    """A C11 translation unit that includes g6mi.h, takes the address of
    every declared function (Fortran aliases included), checks the public
    struct sizes and calls the GPU-free entry points by C and by Fortran
    convention compiles warning-free under -pedantic, links against
    libg6mi.so and runs."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    names = declared_functions()
    table = ",\n    ".join(f"(fn){n}" for n in names)
    src = f"""
#include "g6mi.h"
#include <stdio.h>
#include <string.h>
typedef void (*fn)(void);
_Static_assert(sizeof(g6mi_cluster) == 32, "g6mi_cluster is 32 bytes");
_Static_assert(sizeof(g6mi_batch_tuning) == 16, "g6mi_batch_tuning is 16 bytes");
static const fn every[] = {{
    {table}
}};
int main(void) {{
  int i, n = 0, id = -5;
  for (i = 0; i < (int)(sizeof every / sizeof every[0]); ++i) n += every[i] != 0;
  /* C and Fortran call sites of calls that need no GPU */
  if (g6mi_nb_max() != G6MI_NB_MAX) return 2;
  if (g6_npipes_() != g6_npipes()) return 3;
  if (g6_open_(&id) != G6MI_EINVAL || g6_open(-5) != G6MI_EINVAL) return 4;
  if (g6mi_last_error(-5) == 0 || strlen(g6mi_last_error(-5)) == 0) return 5;
  printf("%d\\n", n);
  return 0;
}}
"""
    c = tmp_path / "abi_check.c"
    c.write_text(src)
    exe = tmp_path / "abi_check"
    libdir = os.path.dirname(g6.LIB_PATH)
    cmd = [cc, "-std=c11", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
           str(c), "-o", str(exe), "-L", libdir, "-lg6mi", f"-Wl,-rpath,{libdir}"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stderr)
    assert int(r.stdout.strip()) == len(names)
