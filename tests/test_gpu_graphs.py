"""GPU: the captured-graph launch mode against one-by-one launches.

A batch replays one HIP graph per run chunk; the same batch launched kernel by
kernel runs the same kernels on the same arguments, so every iterate, every
per-plan statistic and every stopping decision must agree bit for bit.  The
replays are interleaved with the program's own eager work (statistics
read-back and synchronisation after each chunk, the export of the iterates,
the step-size rescale kernels and the upload of the frozen-plan mask inside a
converging run), and every replay is checked, not only the last.
"""
import sys

import numpy as np
import pytest

from synth import cases

pytestmark = pytest.mark.gpu

ladmm = pytest.importorskip("paper_2509_08602_amd.ladmm")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    return ladmm.Context(0)


@pytest.fixture(scope="module")
def c0():
    return cases.make_case(0)


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("precision", ["f64", "f32", "bf16x3"])
def test_graph_replays_match_eager_launches(ctx, c0, precision):
    say("graph vs eager c0", precision)
    w = cases.config_weights(0)
    dc = ladmm.Case.from_case(ctx, c0, precision)
    opts = ladmm.Options(max_iter=3000, check_every=25, tol_gap=1e-4, tol_pri=1e-4, tol_dual=1e-4,
                         rho0=1e4, w0_bot=cases.W0_BOT, adapt_rho=True)
    g = ladmm.Batch(dc, w, opts=opts)
    e = ladmm.Batch(dc, w, opts=opts)
    e.set_graphs(False)
    for rep in range(4):
        g.iterate(25)
        if rep == 0:
            # the tiles g's autotuner chose, pinned on e (tiles never change
            # results; this keeps the comparison to the launch mode alone)
            e.set_tiles(*g.tiles())
        e.iterate(25)
        assert _same(g.export(), e.export()), f"replay {rep}"
        rg, re = g.results(), e.results()
        for key in ("objective", "rel_gap", "r_pri", "r_dual"):
            assert np.array_equal(rg[key], re[key]), (rep, key)
    # a shorter chunk captures a second graph; the first is replayed after it
    g.iterate(7)
    e.iterate(7)
    g.iterate(25)
    e.iterate(25)
    assert _same(g.export(), e.export())
    # a converging run: replays with step-size switches and frozen plans between them
    g.run()
    e.run()
    rg, re = g.results(), e.results()
    for key in rg:
        assert np.array_equal(rg[key], re[key]), key
    assert _same(g.export(), e.export())
    say("graph vs eager", precision, "iters", rg["iters"].tolist())
    g.close()
    e.close()
    dc.close()
