"""The C-ABI library loads and exports every symbol include/mcf.h declares, and
its host-side validation answers without a GPU.  CPU only."""
import os
import re

import numpy as np
import pytest

from paper_2501_17996_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mcf.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mcf_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def mcf():
    from paper_2501_17996_amd import build, mcf as M
    if not os.path.exists(M.LIB_PATH):
        build.build()
    return M


def test_every_declared_symbol_is_exported(mcf):
    L = mcf.lib()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(mcf.EXPORTED)


def test_options_defaults_are_the_papers(mcf):
    import json
    o = mcf.mcf_options_default()
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    assert o.rho == g["rho"]["value"] and o.theta == g["theta"]["value"] and o.tau == g["tau"]["value"]
    assert o.k_adapt == g["k_adapt"]["value"] and o.omega0 == g["omega0"]["value"]
    assert o.tol == 1e-4 and o.precision == mcf.MCF_FP64 and o.check_every == 1


def test_workspace_bytes(mcf):
    a = mcf.mcf_workspace_bytes(200, 2000, mcf.MCF_FP32)
    b = mcf.mcf_workspace_bytes(200, 2000, mcf.MCF_FP64)
    assert 0 < a < b
    # four n x m iterate arrays dominate: 4 * 256 * 2000 * 4 bytes in FP32 (ld = n padded to 64)
    assert a >= 4 * 256 * 2000 * 4
    assert mcf.mcf_workspace_bytes(1, 10, 0) == 0
    assert mcf.mcf_workspace_bytes(10, 0, 0) == 0
    assert mcf.mcf_workspace_bytes(16385, 10, 0) == 0


def test_strerror(mcf):
    assert mcf.mcf_strerror(0) == "ok"
    assert "strongly" in mcf.mcf_strerror(mcf.MCF_E_GRAPH)
    assert mcf.mcf_strerror(-99) == "unknown error"


def _expect(mcf, code, **kw):
    inst = I.config1(0)
    args = dict(n=inst.n, tail=inst.tail, head=inst.head, cap=inst.cap, utility=inst.utility, gamma=inst.gamma,
                w=inst.w)
    args.update(kw)
    with pytest.raises(mcf.MCFError) as ei:
        mcf.mcf_create(args["n"], args["tail"], args["head"], args["cap"], args["utility"], args["gamma"],
                       args["w"], kw.get("opt"))
    assert ei.value.code == code


def test_validation_errors(mcf):
    inst = I.config1(0)
    E = mcf.MCF_E_ARG
    t = inst.tail.copy(); t[3] = 10
    _expect(mcf, E, tail=t)                                   # index out of range
    t = inst.tail.copy(); t[0] = inst.head[0]
    _expect(mcf, E, tail=t)                                   # self-loop
    c = inst.cap.copy(); c[5] = 0.0
    _expect(mcf, E, cap=c)                                    # c <= 0
    c = inst.cap.copy(); c[5] = np.inf
    _expect(mcf, E, cap=c)
    w = inst.w.copy(); w[1] = np.nan
    _expect(mcf, E, w=w)                                      # NaN weight off the diagonal
    w = inst.w.copy(); w[0] = np.nan                          # the diagonal is ignored ...
    _expect(mcf, E, w=w, utility=1, gamma=1.0)                # ... but gamma must be in (0, 1)
    _expect(mcf, E, utility=7)
    for a in (0.0, -1.0, 1.0, 16.5, np.nan, np.inf):          # alpha-fair: 0 < alpha <= 16, alpha != 1
        _expect(mcf, E, utility=mcf.MCF_UTIL_ALPHA, gamma=a)
    _expect(mcf, E, n=1)
    o = mcf.mcf_options_default(); o.tol = 0.0
    _expect(mcf, E, opt=o)
    o = mcf.mcf_options_default(); o.rho = 2.0
    _expect(mcf, E, opt=o)


def test_forced_launch_shapes_are_validated(mcf):
    """A forced two-phase shape must be compiled and hold the columns; a node block is 64 or 256."""
    E = mcf.MCF_E_ARG

    def opt(**kw):
        o = mcf.mcf_options_default()
        for k, v in kw.items():
            setattr(o, k, v)
        return o
    _expect(mcf, E, opt=opt(edge_waves=3, edge_vectors=1))      # not a compiled shape
    _expect(mcf, E, opt=opt(edge_waves=4))                      # the pair is given together
    _expect(mcf, E, opt=opt(edge_vectors=2))
    _expect(mcf, E, opt=opt(node_block=128))
    _expect(mcf, E, opt=opt(node_form=3))                       # 0 by size, 1 latency, 2 streaming
    _expect(mcf, E, opt=opt(node_form=-1))
    _expect(mcf, E, opt=opt(precision=0, edge_waves=8, edge_vectors=3))   # compiled for FP32 only ...
    big = I.ring_instance(3000, 2, seed=1)                       # ... and columns of 64*1*2*2 < 3000
    with pytest.raises(mcf.MCFError) as ei:
        mcf.mcf_create(big.n, big.tail, big.head, big.cap, big.utility, big.gamma, big.w,
                       opt(edge_waves=1, edge_vectors=2))
    assert ei.value.code == E
    with pytest.raises(mcf.MCFError) as ei:                     # the flat form has one wave per column too
        mcf.mcf_create(big.n, big.tail, big.head, big.cap, big.utility, big.gamma, big.w,
                       opt(edge_waves=-1, edge_vectors=2))
    assert ei.value.code == E
    _expect(mcf, E, opt=opt(edge_waves=-1, edge_vectors=3))    # not a compiled flat shape
    assert (8, 3) in mcf.mcf_edge_shapes(1) and (8, 3) not in mcf.mcf_edge_shapes(0)
    for precision in (0, 1):
        assert {(-1, v) for v in (1, 2, 4, 8)} <= set(mcf.mcf_edge_shapes(precision))
    assert mcf.mcf_edge_shapes(7) == []


def test_tuned_table_is_well_formed(mcf):
    """Every entry of the measured table names a compiled shape that holds its n_max, with
    n_max ascending per iterate size."""
    import re
    path = os.path.join(os.path.dirname(mcf.LIB_PATH), "csrc", "tuned_shapes.inc")
    ent = re.findall(r"\{(\d+), (\d+), \{(\d+), (\d+), (\d+)\}, (\d+)\}", open(path).read())
    last = {}
    for b, n_max, waves, vectors, par, nb in (tuple(map(int, e)) for e in ent):
        if b == 0:
            continue   # sentinel
        precision = 1 if b == 4 else 0
        assert b in (4, 8) and nb in (64, 256)
        if par == 2:   # the flat edge phase: one wave per edge, listed as waves -1
            assert waves == 1 and (-1, vectors) in mcf.mcf_edge_shapes(precision)
        else:
            assert par == (1 if waves == 1 else 0)
            assert (waves, vectors) in mcf.mcf_edge_shapes(precision)
        assert n_max <= 64 * waves * vectors * (16 // b)
        assert n_max > last.get(b, 0)
        last[b] = n_max


def test_graph_not_strongly_connected(mcf):
    # a directed path 0 -> 1 -> 2 plus 2 -> 1: node 0 is never reached back
    tail = np.array([0, 1, 2], np.int32)
    head = np.array([1, 2, 1], np.int32)
    w = np.ones(9)
    with pytest.raises(mcf.MCFError) as ei:
        mcf.mcf_create(3, tail, head, np.ones(3), 0, 0.0, w)
    assert ei.value.code == mcf.MCF_E_GRAPH


def test_pool_argument_validation(mcf):
    """Invalid pool options are refused on the host, before any device call."""
    bad = [dict(precision=7), dict(max_slots=0), dict(max_slots=mcf.MCF_POOL_MAX_SLOTS + 1), dict(check_every=0),
           dict(n_max=1), dict(n_max=513), dict(waves=6), dict(waves=16), dict(waves=3), dict(precision=0, waves=4),
           dict(precision=0, waves=2),
]
    for kw in bad:
        args = {"precision": 1, "hbm_budget": 0, "max_slots": 4, "check_every": 20}
        args.update(kw)
        with pytest.raises(mcf.MCFError) as ei:
            mcf.mcf_pool_create(**args)
        assert ei.value.code == mcf.MCF_E_ARG, kw


def test_pool_options_defaults(mcf):
    o = mcf.mcf_pool_options_default()
    assert (o.precision, o.max_slots, o.check_every, o.n_max, o.graphs) == (mcf.MCF_FP32, 64, 20, 512, 1)
    assert (o.waves, o.hbm_budget, o.stream) == (0, 0, None)
