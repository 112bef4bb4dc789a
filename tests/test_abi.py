"""The C ABI without a GPU: the library loads, exports every function that
include/pdd.h declares, and the binding's structures have the C layout."""
import ctypes as C
import os
import re
import shutil
import subprocess
import sys
import tempfile

import pytest

from paper_1512_02818_amd import pdd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdd.h")


@pytest.fixture(scope="module")
def built_lib():
    if not os.path.exists(pdd.LIB_PATH):
        from paper_1512_02818_amd import build
        build.build()
    return pdd.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:pdd_status|void|const char\s*\*)\s*\*?\s*(pdd_\w+)\s*\(",
                                 text, flags=re.M)))


def test_every_declared_symbol_is_exported(built_lib):
    names = declared_functions()
    assert len(names) == 27, names
    for n in names:
        assert hasattr(built_lib, n), n
    assert set(names) == set(pdd.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", pdd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (pdd_\w+)", out))
    assert exported == set(names), exported ^ set(names)


def test_last_error_is_empty_string_initially(built_lib):
    # a fresh process: other tests in this one leave messages behind
    code = ("import ctypes as C, sys; L = C.CDLL(sys.argv[1]); L.pdd_last_error.restype = C.c_char_p; "
            "sys.exit(0 if L.pdd_last_error() == b'' else 1)")
    subprocess.run([sys.executable, "-c", code, pdd.LIB_PATH], check=True)


def test_null_arguments_are_rejected_without_gpu(built_lib):
    # argument checks run before any HIP call
    assert built_lib.pdd_init(None, 0) == -1
    assert b"NULL" in built_lib.pdd_last_error()
    assert built_lib.pdd_create_problem(None, None, None) == -1
    assert built_lib.pdd_create_problem_tabulated(None, None, None, None) == -1
    assert built_lib.pdd_solve_nodes(None, None, 0, None, None, None) == -1
    assert built_lib.pdd_solve_ito(None, None, None, 0, None, None, None) == -1
    assert built_lib.pdd_solve_batch(None, None, 0, None) == -1
    assert built_lib.pdd_server_create(None, None, None) == -1
    assert built_lib.pdd_server_submit(None, None, None) == -1
    assert built_lib.pdd_server_poll(None, None, 0, None, 0) == -1
    assert built_lib.pdd_server_report_get(None, None) == -1
    built_lib.pdd_server_destroy(None)
    assert built_lib.pdd_autotune(None, None, None) == -1
    assert built_lib.pdd_set_tuning(None, None, None) == -1
    assert built_lib.pdd_glm_fit(None, None, 0, 0, None, None, None) == -1
    assert built_lib.pdd_grid_gradient(None, None, None, None) == -1
    assert built_lib.pdd_grid_residual(None, None, None, None) == -1
    assert built_lib.pdd_fit_constants(None, None, None, 0, 0, 1.0, None, None) == -1


STRUCTS = {
    "pdd_problem_desc": (pdd.ProblemDesc, ["dim", "lo", "radius", "sigma", "B", "c_b", "n_gx",
                                           "trig", "mono", "fx", "gx", "seed"]),
    "pdd_grid": (pdd.Grid, ["dtype", "n", "lo", "hi", "data"]),
    "pdd_coef_grids": (pdd.CoefGrids, ["b", "c", "f", "g"]),
    "pdd_tuning": (pdd.Tuning, ["block", "grab", "max_launch_paths", "refill", "bridge"]),
    "pdd_solve_opts": (pdd.SolveOpts, ["dt", "n_paths_per_node", "path_offset", "stream_id",
                                       "max_steps", "flags", "rec_phi", "rec_steps", "tuning"]),
    "pdd_node_stats": (pdd.NodeStats, ["mean", "stderr_", "vr_opt", "sums"]),
    "pdd_work_item": (pdd.WorkItem, ["nodes", "n_nodes", "opts", "resid", "out", "grad"]),
    "pdd_tuning_key": (pdd.TuningKey, ["precision", "dim", "correction", "generic"]),
    "pdd_node_constants": (pdd.NodeConstants, ["E_phi", "se_beta", "alpha", "E_tau", "se_E_tau", "iterations"]),
    "pdd_server_opts": (pdd.ServerOpts, ["memory_budget", "max_queued", "n_pilot", "epoch_paths", "pipeline",
                                         "reserved"]),
    "pdd_request": (pdd.Request, ["n_nodes", "target_se", "stream_id", "u_prev", "resid", "out",
                                  "user_tag", "grad"]),
    "pdd_completion": (pdd.Completion, ["status", "queued_ms", "latency_ms", "path_steps", "n_nodes"]),
    "pdd_server_report": (pdd.ServerReport, ["shed", "mem_fixed", "p50_ms", "wall_s",
                                             "node_solves_per_s", "epoch_s", "p99_done_ms", "busy_s",
                                             "paths_run"]),
}


def test_struct_layouts_match_the_header():
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pdd.h"', "int main(void){"]
    for name, (_, fields) in STRUCTS.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f in fields:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    d = tempfile.mkdtemp()
    try:
        src = os.path.join(d, "l.c")
        open(src, "w").write("\n".join(lines))
        exe = os.path.join(d, "l")
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    finally:
        shutil.rmtree(d, ignore_errors=True)
    got = dict(l.split() for l in out if l.strip())
    for name, (cls, fields) in STRUCTS.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f in fields:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, (name, f)
