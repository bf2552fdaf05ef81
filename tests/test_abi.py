"""Host-side checks of the C ABI (no GPU needed): the built library exports
every entry point the header declares, the binding's structs have the C
layout, and configuration validation rejects what the header says it does."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "metade.h")


def _lib():
    from paper_2502_10470_amd import metade as M
    if not os.path.exists(M.LIB_PATH):
        pytest.skip("libmetade.so not built")
    return M


def test_header_symbols_exported():
    M = _lib()
    text = open(HEADER).read()
    declared = set(re.findall(r"\b(metade_[a-z_]+)\s*\(", text))
    assert len(declared) >= 20
    L = M.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(M.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", M.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared:
        assert re.search(rf"\bT {name}\b", out), name


def test_struct_layout_matches_c(tmp_path):
    M = _lib()
    src = tmp_path / "lay.c"
    fields_p = [f[0] for f in M.MetadeProblem._fields_]
    fields_c = [f[0] for f in M.MetadeConfig._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "metade.h"', 'int main(void){']
    lines.append('printf("%zu %zu\\n", sizeof(metade_problem), sizeof(metade_config));')
    lines.append('printf("%zu %zu\\n", sizeof(metade_tuning), offsetof(metade_tuning, mfma_rows));')
    for f in fields_p:
        lines.append(f'printf("%zu\\n", offsetof(metade_problem, {f}));')
    for f in fields_c:
        lines.append(f'printf("%zu\\n", offsetof(metade_config, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(M.MetadeProblem) and vals[1] == ctypes.sizeof(M.MetadeConfig)
    assert vals[2] == ctypes.sizeof(M.MetadeTuning) and vals[3] == M.MetadeTuning.mfma_rows.offset
    k = 4
    for f in fields_p:
        assert vals[k] == getattr(M.MetadeProblem, f).offset, f
        k += 1
    for f in fields_c:
        assert vals[k] == getattr(M.MetadeConfig, f).offset, f
        k += 1


def _cfg(M, N=(32,), D=10, kind="rastrigin", lb=-100.0, ub=100.0, n_cs=2, precision=0):
    n = len(N)
    keep = {}
    keep["N"] = np.array(N, np.uint32)
    keep["P"] = np.zeros(n, np.uint32)
    keep["S"] = np.zeros(n, np.uint32)
    probs = (M.MetadeProblem * 1)()
    probs[0].kind = M.FN[kind]
    probs[0].D = D
    probs[0].bias = 100.0
    probs[0].o = 0x1000      # never dereferenced by size queries
    probs[0].R = 0x2000
    cfg = M.MetadeConfig()
    cfg.n_runs = n
    cfg.N = keep["N"].ctypes.data
    cfg.problem = keep["P"].ctypes.data
    cfg.stream_id = keep["S"].ctypes.data
    cfg.n_problems = 1
    cfg.problems = ctypes.addressof(probs)
    cfg.lb, cfg.ub, cfg.n_cs, cfg.precision = lb, ub, n_cs, precision
    keep["probs"] = probs
    return cfg, keep


def test_query_sizes_packing():
    M = _lib()
    cfg, keep = _cfg(M, N=(32, 50, 10), D=7)
    pop, fit, by, bx, scratch = M.metade_query_sizes(cfg)
    assert pop == 4 * 7 * (32 + 50 + 10) and fit == 4 * 92 and by == 8 * 3 and bx == 4 * 21
    assert scratch > 0


@pytest.mark.parametrize("kw,msg", [
    ({"N": (9,)}, "N must be"),
    ({"N": (257,)}, "N must be"),
    ({"D": 0}, "D must be"),
    ({"D": 129}, "D must be"),
    ({"lb": 1.0, "ub": 1.0}, "lb < ub"),
    ({"n_cs": 4}, "n_cs"),
])
def test_validation_rejects(kw, msg):
    M = _lib()
    cfg, keep = _cfg(M, **kw)
    with pytest.raises(M.MetadeError) as ei:
        M.metade_query_sizes(cfg)
    assert "status -1" in str(ei.value) and msg in str(ei.value)


def test_unknown_kind_rejected():
    M = _lib()
    cfg, keep = _cfg(M)
    keep["probs"][0].kind = 99
    with pytest.raises(M.MetadeError) as ei:
        M.metade_query_sizes(cfg)
    assert "unsupported kind" in str(ei.value)


def _ctrl_cfg(M, N=(256,), obs=17, act=6, hidden=(64, 64), D=None, steps=200, plant=True):
    """Control-workload configuration; D defaults to the policy's weight count."""
    h1, h2 = hidden
    if D is None:
        D = h1 * obs + h1 + h2 * h1 + h2 + act * h2 + act
    cfg, keep = _cfg(M, N=N, D=D, kind="lqr_mlp", lb=-1.0, ub=1.0)
    q = keep["probs"][0]
    q.o = q.R = None
    q.bias = 0.0
    q.obs, q.act, q.hidden1, q.hidden2 = obs, act, h1, h2
    q.steps, q.n_rollouts, q.ctrl_weight = steps, 1, 0.01
    if plant:
        q.A, q.B, q.x0 = 0x1000, 0x2000, 0x3000   # never dereferenced by size queries
    return cfg, keep


def test_control_query_sizes():
    M = _lib()
    cfg, keep = _ctrl_cfg(M, N=(256, 100))
    pop, fit, by, bx, scratch = M.metade_query_sizes(cfg)
    D = 5702   # 17 -> 64 -> 64 -> 6 tanh policy (weights and biases)
    assert pop == 4 * D * 356 and fit == 4 * 356 and by == 16 and bx == 8 * D
    assert scratch >= 4 * D * 356   # pending trial rows


@pytest.mark.parametrize("obs,act,D", [(11, 3, 1539), (8, 2, 1410), (11, 2, 1506)])
def test_control_query_sizes_table7_policies(obs, act, D):
    """The 32 x 32 policies of Table VII are accepted with their weight counts."""
    M = _lib()
    cfg, keep = _ctrl_cfg(M, N=(100,), obs=obs, act=act, hidden=(32, 32))
    pop, fit, by, bx, scratch = M.metade_query_sizes(cfg)
    assert pop == 4 * D * 100 and fit == 4 * 100 and bx == 4 * D
    cfg, keep = _ctrl_cfg(M, N=(100,), obs=obs, act=act, hidden=(32, 32), D=D + 1)
    with pytest.raises(M.MetadeError) as ei:
        M.metade_query_sizes(cfg)
    assert "weight count " + str(D) in str(ei.value)


def test_control_mixed_hidden_widths_rejected():
    """All control policies of one context share one hidden width."""
    M = _lib()
    cfg, keep = _ctrl_cfg(M, N=(100, 100))
    probs = (M.MetadeProblem * 2)()
    ctypes.memmove(ctypes.addressof(probs), ctypes.addressof(keep["probs"]),
                   ctypes.sizeof(M.MetadeProblem))
    ctypes.memmove(ctypes.addressof(probs) + ctypes.sizeof(M.MetadeProblem),
                   ctypes.addressof(keep["probs"]), ctypes.sizeof(M.MetadeProblem))
    probs[1].hidden1 = probs[1].hidden2 = 32
    probs[1].D = 32 * 17 + 32 + 32 * 32 + 32 + 32 * 6 + 6
    keep["probs2"] = probs
    keep["P"][1] = 1
    cfg.n_problems = 2
    cfg.problems = ctypes.addressof(probs)
    with pytest.raises(M.MetadeError) as ei:
        M.metade_query_sizes(cfg)
    assert "status -1" in str(ei.value) and "same hidden width" in str(ei.value)
    probs[1].hidden1 = probs[1].hidden2 = 64
    probs[1].D = 5702
    M.metade_query_sizes(cfg)


@pytest.mark.parametrize("kw,msg", [
    ({"hidden": (48, 48)}, "32 or both 64"),
    ({"hidden": (32, 64)}, "32 or both 64"),
    ({"hidden": (64, 32)}, "32 or both 64"),
    ({"obs": 21}, "obs"),
    ({"act": 9}, "act"),
    ({"D": 5701}, "weight count"),
    ({"plant": False}, "A, B and x0"),
    ({"steps": 0}, "steps"),
    ({"N": (1025,)}, "10..1024"),
    ({"N": (9,)}, "10..1024"),
])
def test_control_validation_rejects(kw, msg):
    M = _lib()
    cfg, keep = _ctrl_cfg(M, **kw)
    with pytest.raises(M.MetadeError) as ei:
        M.metade_query_sizes(cfg)
    assert "status -1" in str(ei.value) and msg in str(ei.value)


def test_init_requires_buffers():
    M = _lib()
    cfg, keep = _cfg(M)
    with pytest.raises(M.MetadeError) as ei:
        M.metade_init(cfg)
    assert "device buffers" in str(ei.value)


def test_unknown_evolver_rejected():
    M = _lib()
    cfg, keep = _cfg(M)
    cfg.evolver = 9
    with pytest.raises(M.MetadeError) as ei:
        M.metade_query_sizes(cfg)
    assert "evolver must be" in str(ei.value)


def test_cso_swarm_size_limit():
    M = _lib()
    cfg, keep = _cfg(M, N=(32,) * 1025)
    cfg.evolver = M.EVOLVER_CSO
    with pytest.raises(M.MetadeError) as ei:
        M.metade_query_sizes(cfg)
    assert "1024" in str(ei.value)
