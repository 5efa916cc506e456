"""Graph replay of the Arnoldi steps (rsfde_set_graph): each step's launches are
captured once and replayed as a graph.  Every step of every run must come out
bit for bit as with direct launches (same kernels and arguments), with the
replays interleaved with the solver's own direct work (source operator,
right-hand side, cycle start, update, summary reads), across time steps, new e
buffers, kernel timing switched on and off, restarts and the batched form."""
import os
from dataclasses import replace

import numpy as np
import pytest

from paper_2404_10221_amd import rsfde as R
from rsfde_workloads import config, with_grid

from gpu_helpers import empty, host, say

pytestmark = pytest.mark.gpu


def _run(insts, graphs, precision=R.RSFDE_FP64, fresh_e=False, timing_at=None, batched=True,
         method=R.RSFDE_OPGM):
    """Step all instances through M steps with rsfde_step; returns per step the host
    copies of u and the iteration counts."""
    old = os.environ.get("RSFDE_NO_BATCH")
    os.environ["RSFDE_NO_BATCH"] = "0" if batched else "1"
    try:
        S = R.Solver([R.params_from_instance(i, precision=precision, method=method) for i in insts])
    finally:
        if old is None:
            del os.environ["RSFDE_NO_BATCH"]
        else:
            os.environ["RSFDE_NO_BATCH"] = old
    R.rsfde_set_graph(S.h, graphs)
    for k, inst in enumerate(insts):
        R.rsfde_set_fields(S.h, k, inst.e, inst.f, inst.psi)
        R.rsfde_prescan_ebar(S.h, k, inst.M)
    us = [empty(i.size) for i in insts]
    for k in range(len(insts)):
        R.rsfde_eval_field(S.h, k, R.WHICH_PSI, 0.0, us[k])
    ebufs = [[empty(i.size) for i in insts] for _ in range(2)]
    fs = [empty(int(np.prod([v + 2 for v in i.n]))) for i in insts]
    out = []
    dt = insts[0].dt
    for m in range(insts[0].M):
        if timing_at is not None and m == timing_at[0]:
            R.rsfde_set_timing(S.h, 0x1FF, 1)
        if timing_at is not None and m == timing_at[1]:
            R.rsfde_set_timing(S.h, 0, 1)
        es = ebufs[m % 2] if fresh_e else ebufs[0]
        th = (m + 0.5) * dt
        R.rsfde_eval_field_batch(S.h, R.WHICH_E, th, es)
        R.rsfde_eval_field_batch(S.h, R.WHICH_F, th, fs)
        st, stats = R.rsfde_step(S.h, m * dt, es, fs, us)
        assert st == R.RSFDE_OK
        out.append(([host(u) for u in us], [s["iters"] for s in stats]))
    if graphs:
        R.rsfde_set_graph(S.h, False)
    S.close()
    return out


def _same(a, b):
    for m, ((ua, ia), (ub, ib)) in enumerate(zip(a, b)):
        assert ia == ib, f"step {m}: iterations {ia} vs {ib}"
        for k in range(len(ua)):
            assert np.array_equal(ua[k], ub[k]), f"step {m} instance {k}"


@pytest.mark.parametrize("name,grid", [("C1", (127,)), ("C2", (63, 47)), ("C3", (31, 23, 15))])
def test_graph_replay_equals_direct(name, grid):
    inst = with_grid(config(name), grid, M=5)
    say(f"[graphs] {name} grid {grid}, 5 steps")
    a = _run([inst], graphs=True)
    b = _run([inst], graphs=False)
    say(f"   iterations per step {[i[0] for _, i in a]}")
    _same(a, b)


def test_graph_replay_mixed_precision():
    inst = with_grid(config("C2"), (63, 63), M=4)
    a = _run([inst], graphs=True, precision=R.RSFDE_MIXED)
    b = _run([inst], graphs=False, precision=R.RSFDE_MIXED)
    _same(a, b)


def test_graph_replay_new_e_buffers_and_timing_switches():
    # e alternates between two buffers (captured steps are rebuilt when e moves);
    # timing on for steps 2..3 (direct launches then), off again afterwards
    inst = with_grid(config("C3"), (31, 31, 31), M=6)
    a = _run([inst], graphs=True, fresh_e=True, timing_at=(2, 4))
    b = _run([inst], graphs=False, fresh_e=True)
    _same(a, b)


@pytest.mark.parametrize("name,grid", [("C1", (63,)), ("C2", (47, 31)), ("C3", (15, 23, 11))])
def test_graph_replay_two_sided(name, grid):
    # the two-sided form's steps start with the P^{-1/2} passes
    inst = replace(with_grid(config(name), grid, M=4), restart=4, max_cycles=60)
    a = _run([inst], graphs=True, method=R.RSFDE_TPGM)
    b = _run([inst], graphs=False, method=R.RSFDE_TPGM)
    _same(a, b)


def test_graph_replay_strang():
    # the Strang-circulant form's steps end with the Hartley passes
    inst = replace(with_grid(config("C2"), (47, 31), M=3), restart=5, max_cycles=60)
    a = _run([inst], graphs=True, method=R.RSFDE_SPGM)
    b = _run([inst], graphs=False, method=R.RSFDE_SPGM)
    _same(a, b)


def test_graph_replay_restarts():
    # GMRES(3): several cycles per step, with and without a pending resolve
    inst = replace(with_grid(config("C2"), (47, 47), M=3), restart=3, max_cycles=60)
    a = _run([inst], graphs=True)
    b = _run([inst], graphs=False)
    _same(a, b)


def test_graph_replay_batched():
    # the batched form replays graphs captured on the full-set plan; restart cycles
    # on a partial set of instances launch directly
    sizes = [(15, 31), (31, 15), (47, 23), (23, 47), (31, 31)]
    c4 = config("C4")
    insts = [replace(with_grid(c4[i], sizes[i], M=4), restart=4, max_cycles=60) for i in range(5)]
    tols = [1e-6, 1e-12, 1e-8, 1e-10, 1e-11]
    insts = [replace(i, rtol=t) for i, t in zip(insts, tols)]
    a = _run(insts, graphs=True, fresh_e=True)
    b = _run(insts, graphs=False, fresh_e=True)
    c = _run(insts, graphs=False, fresh_e=True, batched=False)
    _same(a, b)
    _same(a, c)


@pytest.mark.parametrize("method", [R.RSFDE_TPGM, R.RSFDE_SPGM], ids=["two_sided", "strang"])
def test_graph_replay_batched_other_forms(method):
    # batched two-sided (right factor stopping on the pending step's status) and
    # Strang (batched Hartley passes) forms replayed from graphs, against direct
    # batched and one-at-a-time launches
    sizes = [(15, 31), (31, 15), (23, 23)]
    c4 = config("C4")
    insts = [replace(with_grid(c4[i], sizes[i], M=3), restart=5, max_cycles=60) for i in range(3)]
    a = _run(insts, graphs=True, method=method)
    b = _run(insts, graphs=False, method=method)
    c = _run(insts, graphs=False, batched=False, method=method)
    _same(a, b)
    _same(a, c)
