"""Block windows replayed from a captured HIP graph (ctaux_set_graph) against
the same chains launched block by block.

The graph holds the same kernels in the same order, so every result must be
identical bit for bit: decisions, ratios, configurations, N and the
accumulated observables.  The runs have lengths that are not multiples of the
window, and the refinement schedule starts at one block and grows, so graph
replays alternate with blocks launched one by one and with refinements (the
program's own work between replays); each replay is checked through the
decisions of the proposals it ran.
"""

from __future__ import annotations

import numpy as np
import pytest

from ctaux_inputs import dca_square

pytestmark = pytest.mark.gpu


def _ctaux():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1010_3690_amd import ctaux
    return ctaux


def _pair(ctaux, ws, window, **kw):
    opts = dict(k_max=32, k_cap=32, n_cap=512, recompute_every=16, meas_every=32, n_tau_out=8, seed=11,
                log_cap=32 * 400)
    opts.update(kw)
    eager = ctaux.CtauxBatch(ws, ctaux.Options(**opts))
    graph = ctaux.CtauxBatch(ws, ctaux.Options(**opts))
    graph.set_graph(window)
    return eager, graph


def _same(ctaux, eager, graph, n_chains, n_prop):
    for c in range(n_chains):
        se, sg = eager.stats(c), graph.stats(c)
        assert se["proposals"] == sg["proposals"] == n_prop
        for key in ("accepted", "blocks", "order", "sign"):
            assert se[key] == sg[key], (c, key, se[key], sg[key])
        ae, re = eager.decisions(c, 0, n_prop)
        ag, rg = graph.decisions(c, 0, n_prop)
        assert np.array_equal(ae, ag), c
        assert np.array_equal(re, rg), c
        for a, b in zip(eager.config(c), graph.config(c)):
            assert np.array_equal(a, b), c
        for sec in (0, 1):
            assert np.array_equal(eager.N(c, sec), graph.N(c, sec)), (c, sec)
        assert np.array_equal(eager.obs(c), graph.obs(c)), c


@pytest.mark.parametrize("n_chains", [2, 8])
def test_graph_windows_reproduce_block_launches(n_chains):
    ctaux = _ctaux()
    ws = [dca_square(beta=4.0, U=4.0 + 0.5 * (c % 3), K=1.0, n_tau=4096, n_fine=16,
                     superlattice=[[2, 0], [0, 2]]) for c in range(n_chains)]
    eager, graph = _pair(ctaux, ws, 4)
    done = 0
    # uneven run lengths: windows start at multiples of 4 blocks, the rest is
    # launched block by block, refinements fall between windows
    for blocks in (3, 9, 14, 1, 23, 30, 17, 40):
        eager.run(32 * blocks)
        graph.run(32 * blocks)
        done += 32 * blocks
        _same(ctaux, eager, graph, n_chains, done)
    assert graph.graph_launches >= 10, graph.graph_launches
    assert eager.graph_launches == 0


def test_graph_window_validation():
    ctaux = _ctaux()
    eager, graph = _pair(ctaux, [dca_square(beta=2.0, U=4.0, K=1.0, n_tau=1024, n_fine=8,
                                            superlattice=[[2, 0], [0, 2]])], 2)
    for bad in (-1, 3, 128):
        with pytest.raises(ctaux.CtauxError) as e:
            graph.set_graph(bad)
        assert e.value.code == ctaux.CTAUX_EINVAL
    graph.set_graph(0)
    graph.run(32 * 10)
    assert graph.graph_launches == 0
