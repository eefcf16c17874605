"""The C ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_29257_amd", "librisp.so")
HEADER = os.path.join(ROOT, "include", "risp.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(risp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("risp_build_factors", "risp_sigma", "risp_davidson", "risp_ctx_create", "risp_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librisp.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="librisp.so not built")
def test_binding_struct_layouts_match_header(tmp_path):
    import subprocess
    from paper_2603_29257_amd import abi
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "risp.h"\nint main(){printf("%zu %zu %zu %zu %zu %zu",'
                   'sizeof(risp_shell),sizeof(risp_system),sizeof(risp_params),sizeof(risp_dav_opts),'
                   'sizeof(risp_dav_info),sizeof(risp_factors_desc));}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o", str(exe)], check=True)
    got = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    want = [ctypes.sizeof(t) for t in (abi.Shell, abi.SystemC, abi.ParamsC, abi.DavOptsC, abi.DavInfoC,
                                       abi.FactorsDescC)]
    assert [int(x) for x in got] == want


@pytest.mark.skipif(not os.path.exists(LIB), reason="librisp.so not built")
def test_host_side_argument_errors_without_gpu():
    """risp_select_aux is host logic: it validates and selects without touching a device."""
    import numpy as np
    from paper_2603_29257_amd import abi
    import synth
    mol = synth.make_config0()
    sysc = abi.System(mol)
    prm = abi.Params().c()
    J = (abi.Shell * 64)()
    K = (abi.Shell * 64)()
    nj, nk = ctypes.c_int32(), ctypes.c_int32()
    rc = abi._LIB.risp_select_aux(ctypes.byref(sysc.c), ctypes.byref(prm), 64, J, ctypes.byref(nj), K,
                                  ctypes.byref(nk))
    assert rc == 0 and nj.value == 24 and nk.value == 12
    rc = abi._LIB.risp_select_aux(ctypes.byref(sysc.c), ctypes.byref(prm), 4, J, ctypes.byref(nj), K,
                                  ctypes.byref(nk))
    assert rc == abi.RISP_E_SHAPE and b"cap" in abi._LIB.risp_last_error()
    bad = abi.Params(theta=-1.0).c()
    rc = abi._LIB.risp_select_aux(ctypes.byref(sysc.c), ctypes.byref(bad), 64, J, ctypes.byref(nj), K,
                                  ctypes.byref(nk))
    assert rc == abi.RISP_E_ARG
    assert np.all([J[k].atom < 12 for k in range(24)])


@pytest.mark.skipif(not os.path.exists(LIB), reason="librisp.so not built")
def test_job_footprint_host_model():
    """The admission footprint is host logic: it grows with size, precision and subspace."""
    from paper_2603_29257_amd import abi
    import synth
    small = abi.System(synth.make_chain_ring(40, 40))
    big = abi.System(synth.make_config0())
    f_small = abi.job_footprint(small, abi.Params(precision=abi.FP32), nstates=5)
    f_big = abi.job_footprint(big, abi.Params(precision=abi.FP32), nstates=5)
    assert 0 < f_small
    f64 = abi.job_footprint(small, abi.Params(precision=abi.FP64), nstates=5)
    assert f64 > f_small
    more = abi.job_footprint(small, abi.Params(precision=abi.FP32), nstates=5, max_space=200)
    assert more >= f_small
    assert f_big != f_small
    with pytest.raises(abi.RispError):
        bad = synth.make_chain_ring(40, 40)
        bad.nocc = 0
        abi.job_footprint(abi.System(bad), abi.Params(), nstates=5)


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: --gpus N > 1 exits with status 2 and a JSON line saying so, before touching a GPU
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
