"""Host check (no GPU) of the scatter epilogue's tables: in the batched corner
chain, step 2's GEMM writes its products straight into step 3's A panels, and
every product must land on the position step 3's gather would copy it to
(tests/host/scatter_check.cpp, compiled here against the library's planner),
for seeded draws of the batched workload in the three bf16 precisions."""
import ctypes as C
import os
import subprocess

import pytest

import paper_1808_10804_amd as st
from paper_1808_10804_amd import _lib
from oracle import u1
from synth import config, batched_draws

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PREC = {"bf16": 2, "bf16x3": 3, "bf16x6": 4}


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    lib = os.path.dirname(_lib.LIB_PATH)
    out = str(tmp_path_factory.mktemp("scatter") / "scatter_check.so")
    cmd = ["hipcc", "-std=c++17", "-O2", "-fPIC", "-shared", "-x", "hip",
           os.path.join(ROOT, "tests", "host", "scatter_check.cpp"),
           "-I", os.path.join(ROOT, "paper_1808_10804_amd", "csrc"), "-L" + lib, "-l:" + os.path.basename(_lib.LIB_PATH),
           "-Wl,-rpath," + lib, "-o", out]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-3000:]
    _lib.lib()
    L = C.CDLL(out)
    L.scatter_check.argtypes = [C.c_void_p] * 3 + [C.c_int]
    L.scatter_check.restype = C.c_longlong
    return L


@pytest.mark.parametrize("prec", sorted(PREC))
def test_every_product_lands_where_the_gather_puts_it(checker, prec):
    c5 = config(5)
    draws = batched_draws(c5["seed"], c5["batch"], c5["D_choices"], c5["chi_range"])
    total = 0
    for d in draws[:: 8]:   # 8 of the 64 draws (D 4..8, chi 32..160)
        w = u1.Workload(c5["phys"], d["virt"], d["chi"], c5["flux"])
        dd, chi = w.a_legs[0].sectors(), d["chi"]
        a = st.Tensor.meta([(dd, 1), (dd, 1), (dd, -1), (dd, -1)], 0, "f32")
        C1 = st.Tensor.meta([(chi, 1), (chi, -1)], 0, "f32")
        T1 = st.Tensor.meta([(chi, 1), (dd, -1), (chi, -1)], 0, "f32")
        T4 = st.Tensor.meta([(chi, 1), (dd, -1), (chi, -1)], 0, "f32")
        # the batched chain: step 1's output ordered [xa, x1, u]
        _, s1 = st.plan_info(C1, T1, [1], [0], out_perm=[0, 2, 1])
        n = checker.scatter_check(s1._h, T4._h, a._h, PREC[prec])
        assert n > 0, (d["D"], chi, n)
        total += n
    assert total > 10 ** 6
