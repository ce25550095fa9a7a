"""The C-ABI library loads and exports every function include/sph.h
declares, and the ctypes mirror of each struct has the C layout.  CPU only:
no compute calls."""
import ctypes as C
import os
import subprocess
import sys
import tempfile

import pytest

from paper_2206_14780_amd import sph as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(S.LIB_PATH):
        from paper_2206_14780_amd import build
        build.build()
    return C.CDLL(S.LIB_PATH)


def test_header_declares_the_entry_points():
    names = S.header_functions()
    for f in ("sph_build_neighbors", "sph_visc_apply", "sph_visc_solve", "sph_create",
              "sph_destroy", "sph_neighbors_export", "sph_neighbors_free", "sph_status_str",
              "sph_mlp_samples", "sph_mlp_warmstart", "sph_mlp_forward", "sph_mlp_grad",
              "sph_mlp_train_step"):
        assert f in names


def test_mlp_constants_agree():
    from oracle import mlp as M
    txt = open(S.HEADER).read()
    assert f"#define SPH_MLP_NPARAM {M.NPARAM}" in txt
    assert f"#define SPH_MLP_SAMPLE {M.SAMPLE}" in txt
    assert S.SPH_MLP_NPARAM == M.NPARAM and S.SPH_MLP_SAMPLE == M.SAMPLE


def test_every_declared_symbol_is_exported(lib):
    for name in S.header_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    lib.sph_status_str.restype = C.c_char_p
    lib.sph_status_str.argtypes = [C.c_int]
    assert lib.sph_status_str(0) == b"ok"
    assert lib.sph_status_str(-5) == b"non-finite input"


def test_null_context_is_an_argument_error(lib):
    lib.sph_visc_solve.restype = C.c_int
    assert lib.sph_visc_solve(None, None, None, None, None, 0, None, None, None, None) == -1
    lib.sph_create.restype = C.c_int
    assert lib.sph_create(None, 0, None) == -1


STRUCT_NAMES = ["sph_particles", "sph_domain", "sph_visc_params", "sph_solve_opts",
                "sph_solve_report", "sph_step_params"]
# every field of every ctypes mirror, in declaration order
STRUCTS = {st: [f[0] for f in getattr(S, st)._fields_] for st in STRUCT_NAMES}


def test_ctypes_layout_matches_c():
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sph.h"', "int main(void){"]
    for st, fields in STRUCTS.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fields:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(l.split() for l in out if l.strip())
    for st, fields in STRUCTS.items():
        cls = getattr(S, st)
        assert int(got[st]) == C.sizeof(cls), st
        for f in fields:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, f"{st}.{f}"


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: the solver has no multi-GPU decomposition, and the check
    # comes before anything touches a device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "--gpus 2" in r.stderr and r.stdout == ""


def test_traffic_summary_is_machine_readable():
    # bench.py reads the dominant kernel's measured HBM bytes per launch from
    # the committed counter summary, and reports them only while the listed
    # kernel sources hash to the recorded value: the three fields are there,
    # the byte count is a positive integer, and every listed source exists
    import bench
    txt = open(bench.TRAFFIC_PROFILE).read()
    fields = dict(l.split(": ", 1) for l in txt.splitlines()
                  if l.startswith(("traffic_bytes_per_launch:", "source_sha256:", "source_files:")))
    assert set(fields) == {"traffic_bytes_per_launch", "source_sha256", "source_files"}
    assert int(fields["traffic_bytes_per_launch"]) > 0
    assert len(fields["source_sha256"].strip()) == 64
    files = fields["source_files"].split()
    assert files and all(os.path.exists(os.path.join(ROOT, f)) for f in files)
