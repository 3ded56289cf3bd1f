"""CPU checks of the C ABI: the library loads, exports every function that
include/dnls.h declares, and rejects malformed problems before touching the
device (no kernel launches here)."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2207_09442_amd as P
    if not os.path.exists(P.LIB_PATH):
        pytest.skip("libdnls.so not built (run __graft_entry__.build())")
    return P


def _declared():
    src = open(os.path.join(ROOT, "include", "dnls.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dnls_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["dnls_plan_create", "dnls_plan_workspace", "dnls_plan_flops", "dnls_solve", "dnls_backward",
              "dnls_project_grad", "dnls_plan_destroy", "dnls_last_error", "dnls_version"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    P = _lib()
    L = ctypes.CDLL(P.LIB_PATH)
    for n in _declared():
        assert hasattr(L, n), n


def _create(P, p, **opt):
    pr = P._Problem()
    keep = []
    pr.batch = len(p["pose_off"]) - 1
    pr.group = P.GROUPS[p["group"]]
    for name in ["pose_off", "edge_off", "prior_off", "prior_var"]:
        a, ptr = P._i32(p[name])
        keep.append(a)
        setattr(pr, name, ptr)
    a, ptr = P._i32(np.asarray(p["edge_ij"]).reshape(-1))
    keep.append(a)
    pr.edge_ij = ptr
    o = P._Options(opt.get("solver", 0), opt.get("precision", 0), opt.get("iterations", 3),
                   opt.get("refine", 0), opt.get("lam", 0.0), opt.get("sparse_solve", 0), opt.get("flags", 0),
                   opt.get("radius", 0.0))
    h = ctypes.c_void_p()
    code = P.lib().dnls_plan_create(ctypes.byref(h), ctypes.byref(pr), ctypes.byref(o))
    return code, P.lib().dnls_last_error().decode()


def test_invalid_problems_are_rejected_with_a_message():
    P = _lib()
    p = synth.walk_se3(batch=2, n_poses=5, n_loops=2)
    bad = dict(p)
    bad["edge_ij"] = p["edge_ij"].copy()
    bad["edge_ij"][0, 1] = p["pose_off"][1] + 1          # index in the other graph
    code, msg = _create(P, bad)
    assert code == 1 and "outside its graph" in msg
    bad = dict(p)
    bad["edge_ij"] = p["edge_ij"].copy()
    bad["edge_ij"][0, 1] = bad["edge_ij"][0, 0]           # self edge
    assert _create(P, bad)[0] == 1
    bad = dict(p)
    bad["pose_off"] = np.array([0, 7, 5], np.int32)       # decreasing offsets
    assert _create(P, bad)[0] == 1
    bad = dict(p)
    bad["prior_var"] = np.array([0, 0], np.int32)         # prior of graph 1 on a pose of graph 0
    assert _create(P, bad)[0] == 1
    assert _create(P, p, iterations=-1)[0] == 1
    assert _create(P, p, lam=-1.0)[0] == 1
    assert _create(P, p, refine=9)[0] == 1
    assert _create(P, p, precision=5)[0] == 1
    assert _create(P, p, sparse_solve=6)[0] == 1
    assert _create(P, p, flags=32)[0] == 1
    assert _create(P, p, flags=8, solver=1)[0] == 2       # kept iterates: pose-graph solvers only
    assert _create(P, p, flags=10)[0] == 2                # kept iterates with adaptive damping
    assert _create(P, p, flags=4)[0] == 1                 # dogleg without a trust radius
    assert _create(P, p, flags=4, radius=float("nan"))[0] == 1
    assert _create(P, p, flags=6, radius=1.0)[0] == 1     # dogleg and adaptive damping


def test_null_arguments():
    P = _lib()
    L = P.lib()
    assert L.dnls_plan_create(None, None, None) == 1
    assert L.dnls_plan_destroy(None) == 0
    assert L.dnls_solve(None, None, None) == 1
    assert L.dnls_solve_noalloc(None, None, None) == 1
    assert L.dnls_backward(None, None, None) == 1
    assert L.dnls_project_grad(7, 1, None, None, None, None) == 1
    assert L.dnls_project_grad(3, 0, None, None, None, None) == 0
    assert L.dnls_version().decode().startswith("dnls")
