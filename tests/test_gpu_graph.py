"""Replayed step graphs give the same results as kernel-by-kernel launches.

The step graph is replayed several times with eager work (mass reports,
field exports, a variant change) in between, and every replay is checked."""
import numpy as np
import pytest

from paper_2207_13962_amd import inputs as I

pytestmark = pytest.mark.gpu


def _pair(setup):
    import torch
    from paper_2207_13962_amd.fslbm import Simulation
    st = torch.cuda.Stream()
    a = Simulation(setup, stream=st)
    b = Simulation(setup, stream=st)
    b.set_graphs(False)
    return a, b


@pytest.mark.parametrize("storage", [I.F64, I.F32])
def test_graph_replays_match_plain_launches(storage):
    s = I.rect_dam_break(nx=48, ny=32, nz=16, wx=16, hy=24, g=1e-4, nu=0.005, storage=storage)
    a, b = _pair(s)
    for r in range(5):
        a.step(8)
        b.step(8)
        fa, fb = a.fields(), b.fields()
        for k in ("type", "pdf", "mass", "phi"):
            assert np.array_equal(fa[k], fb[k]), (r, k)
        assert a.mass() == b.mass()
    # a variant change recaptures
    a.set_variant(I.NBKC)
    b.set_variant(I.NBKC)
    a.step(19)
    b.step(19)
    fa, fb = a.fields(), b.fields()
    assert np.array_equal(fa["pdf"], fb["pdf"]) and np.array_equal(fa["type"], fb["type"])


def test_odd_plain_steps_between_replays():
    """The step graph holds the buffer pointers and counter slots of the step
    parity it was captured at. Calls of odd length between replays (plain
    launches) change the parity; the next replay must still continue the run
    exactly: bitwise equal to a run launched kernel by kernel. The graph is
    captured eagerly by set_graphs, before any step."""
    s = I.rect_dam_break(nx=48, ny=32, nz=16, wx=16, hy=24, g=1e-4, nu=0.005, storage=I.F64,
                         variant=I.OM3)
    a, b = _pair(s)
    a.set_graphs(True)  # captures now, at step 0
    for n in (3, 8, 1, 9, 16, 5, 8, 8, 7, 24):
        a.step(n)
        b.step(n)
    fa, fb = a.fields(), b.fields()
    for k in ("type", "pdf", "mass", "phi"):
        assert np.array_equal(fa[k], fb[k]), k
    assert a.mass() == b.mass()


def test_runs_on_separate_streams_side_by_side():
    """Runs stepped side by side on streams of their own (their launches
    overlap on the device) equal the same runs stepped in turn on one stream,
    bitwise: each context owns its arena, lists and counters."""
    import torch
    from paper_2207_13962_amd.fslbm import Simulation
    setups = [I.rect_dam_break(nx=48, ny=32, nz=16, wx=16, hy=24, g=1e-4, nu=0.005, storage=I.F32, variant=v)
              for v in (I.NBRC, I.NBKC, I.OM, I.OM3)]
    setups.append(I.Setup(setups[2].params.with_(layout=I.AA), setups[2].type, setups[2].phi, setups[2].rho,
                          setups[2].ux, setups[2].uy, setups[2].uz))
    one = torch.cuda.Stream()
    seq = [Simulation(s, stream=one) for s in setups]
    streams = [torch.cuda.Stream() for _ in setups]
    par = [Simulation(s, stream=st) for s, st in zip(setups, streams)]
    for _ in range(4):
        for s in seq:
            s.step(37)
        for s in par:
            s.step(37)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(seq, par)):
        fa, fb = a.fields(), b.fields()
        for k in ("type", "pdf", "mass", "phi"):
            assert np.array_equal(fa[k], fb[k]), (i, k)
        assert a.mass() == b.mass()
        a.close()
        b.close()
