"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, validates arguments on the host before touching the
device, and its footprint arithmetic is consistent."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2301_06384_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gk", "graph_kernel.h")

gk = pytest.importorskip("paper_2301_06384_amd.gk")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|const char\*|char\*)\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_symbols_exported():
    names = _declared_functions()
    assert len(names) >= 15
    lib = C.CDLL(gk.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(names) == set(gk.EXPORTED)


def test_strerror_and_version():
    assert gk.strerror(0) == "ok"
    assert "duplicate" in gk.strerror(gk.EDUPSAMPLE)
    assert gk.version().startswith("gk")


def _lap():
    return I.grid((4, 3))


def test_init_rejects_bad_csr_on_host():
    L = _lap()
    with pytest.raises(gk.GKError) as e:
        gk.Graph(0, [0], [], [])
    assert e.value.code == gk.EINVAL
    # column out of range
    ci = L.col_idx.copy()
    ci[3] = 99
    with pytest.raises(gk.GKError) as e:
        gk.Graph(L.n, L.row_ptr, ci, L.vals)
    assert e.value.code == gk.EINVAL
    # non-symmetric values
    v = L.vals.copy()
    v[1] -= 0.5
    with pytest.raises(gk.GKError) as e:
        gk.Graph(L.n, L.row_ptr, L.col_idx, v)
    assert e.value.code == gk.ENOTSYM
    # positive off-diagonal (both triangles, so symmetric)
    A = L.to_scipy().tolil()
    A[0, 1] = A[1, 0] = 0.5
    A = A.tocsr()
    A.sort_indices()
    with pytest.raises(gk.GKError) as e:
        gk.Graph(L.n, A.indptr, A.indices, A.data)
    assert e.value.code == gk.ENOTLAP
    # negative diagonal excess without ASSUME_PSD
    B = L.to_scipy().tolil()
    B[2, 2] = B[2, 2] - 1.0
    B = B.tocsr()
    B.sort_indices()
    with pytest.raises(gk.GKError) as e:
        gk.Graph(L.n, B.indptr, B.indices, B.data)
    assert e.value.code == gk.ENOTLAP
    # non-finite
    v = L.vals.copy()
    v[0] = np.nan
    with pytest.raises(gk.GKError) as e:
        gk.Graph(L.n, L.row_ptr, L.col_idx, v)
    assert e.value.code == gk.EINVAL
    # unsorted columns
    ci = L.col_idx.copy()
    ci[0], ci[1] = ci[1], ci[0]
    with pytest.raises(gk.GKError) as e:
        gk.Graph(L.n, L.row_ptr, ci, L.vals)
    assert e.value.code == gk.EINVAL


def test_valid_csr_reaches_device_check():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: covered by the GPU tests")
    L = _lap()
    with pytest.raises(gk.GKError) as e:
        gk.Graph.from_laplacian(L)
    assert e.value.code == gk.EDEVICE


def test_footprint_arithmetic():
    # basis storage dominates (Table 2): fp64 ~ m n s 8 bytes, mixed ~ m n s 4 + 3 n s 8
    n, s, m = 100_000, 64, 40
    f64 = gk.request_footprint(n, s, m, "cbl", "fp64")
    fmx = gk.request_footprint(n, s, m, "cbl", "mixed")
    basis64 = m * n * s * 8
    assert basis64 < f64 < basis64 * 1.3
    assert fmx < f64 * 0.7
    # Chebyshev needs O(n s) storage independent of m (Table 2)
    c1 = gk.request_footprint(n, s, 10, "cheb", "fp64")
    c2 = gk.request_footprint(n, s, 400, "cheb", "fp64")
    assert c1 == c2 and c1 < f64 / 5
    # the 128^3-grid request (s=512, m=30): the fp64 basis alone is 257.7 GB,
    # beyond 90% of a 288 GB device; the mixed path (float32 archive) fits
    n5, s5, m5 = 128 ** 3, 512, 30
    assert gk.request_footprint(n5, s5, m5, "cbl", "fp64") > 0.9 * 288e9
    assert gk.request_footprint(n5, s5, m5, "cbl", "mixed") < 0.7 * 288e9
    with pytest.raises(gk.GKError):
        gk.request_footprint(0, 4, 4)
    with pytest.raises(gk.GKError):
        gk.request_footprint(10, 2000, 4)


def test_struct_layouts_match_header(tmp_path):
    # the ctypes structures of the binding against the C header: every field
    # offset and every struct size, from a program compiled with the header
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"gk_phi": gk.Phi, "gk_stats": gk.Stats, "gk_request": gk.Request, "gk_result": gk.Result,
               "gk_kernel_timing": gk.KernelTiming}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gk/graph_kernel.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            cname, field, val = line.split()
            got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
