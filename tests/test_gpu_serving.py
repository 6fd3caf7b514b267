"""Serving through the C ABI (fslbm_server_*): a run's results are the same
alone, in a mix and in a single context; the FP64 served run matches the
oracle; admission respects the pool budget; an unstable run is retired with
its error while the others finish unaffected."""
import numpy as np
import pytest

from paper_2207_13962_amd import inputs as I

pytestmark = pytest.mark.gpu

MB = 1 << 20


def _mix():
    """Small runs of both kinds, all four variants, different sizes."""
    reqs = [
        I.droplet_impact(L=24, velocity=0.03, variant=I.NBRC),
        I.wave_slab(L=32, amp_frac=0.02, variant=I.NBKC),
        I.droplet_impact(L=28, velocity=0.04, variant=I.OM),
        I.wave_slab(L=40, amp_frac=0.01, variant=I.OM3),
        I.droplet_impact(L=20, velocity=0.02, variant=I.OM3),
    ]
    steps = [90, 60, 75, 50, 110]
    return reqs, steps


def _serve(setups, steps, budget=512 * MB, max_slots=8, ticks=7, order=None):
    from paper_2207_13962_amd.fslbm import Server
    srv = Server(budget, max_slots=max_slots)
    order = list(range(len(setups))) if order is None else order
    ids = {}
    for i in order:
        ids[srv.submit(setups[i], steps[i])] = i
    out = {}
    peak = 0
    budget_calls = 10 * sum(steps) // ticks + 100
    while len(out) < len(setups):
        budget_calls -= 1
        assert budget_calls > 0, "runs did not finish"
        srv.advance(ticks)
        st = srv.stats()
        peak = max(peak, st["resident"])
        assert st["bytes_in_use"] <= st["budget_bytes"]
        for rid, status in srv.poll():
            rep, phi = srv.result(rid)
            out[ids[rid]] = (status, rep, phi)
    stats = srv.stats()
    srv.close()
    return out, peak, stats


def test_same_alone_in_mix_and_single_context():
    from paper_2207_13962_amd.fslbm import Simulation
    setups, steps = _mix()
    mixed, peak, _ = _serve(setups, steps)
    assert peak == len(setups)  # every run resident at once
    for i, s in enumerate(setups):
        alone, _, _ = _serve([s], [steps[i]])
        st_m, rep_m, phi_m = mixed[i]
        st_a, rep_a, phi_a = alone[0]
        assert st_m == st_a == 0
        assert np.array_equal(phi_m, phi_a), i
        assert rep_m["total_mass"] == rep_a["total_mass"]
        sim = Simulation(s)
        sim.step(steps[i])
        r = sim.mass()
        phi_s = sim.fields(pdf=False)["phi"]
        sim.close()
        assert np.array_equal(phi_m, phi_s), i
        assert rep_m["total_mass"] == r["total_mass"]
        assert rep_m["n_interface"] == r["n_interface"]


def test_served_fp64_run_matches_oracle():
    from oracle import Oracle
    setups = [I.droplet_impact(L=20, velocity=0.03, variant=v, storage=I.F64) for v in (I.OM, I.NBKC)]
    setups.append(I.wave_slab(L=24, amp_frac=0.02, variant=I.NBRC, storage=I.F64))
    steps = [40, 33, 25]
    out, _, _ = _serve(setups, steps, ticks=5)
    for i, s in enumerate(setups):
        o = Oracle(s)
        assert o.step(steps[i]) == 0
        f = o.fields()
        st, rep, phi = out[i]
        assert st == 0
        assert np.allclose(phi, f["phi"], rtol=0, atol=1e-12), i
        r = o.mass()
        assert abs(rep["total_mass"] - r.total_mass) <= 1e-12 * r.total_mass
        assert rep["n_interface"] == r.n_interface


def test_budget_limits_residency():
    from paper_2207_13962_amd.fslbm import workspace_bytes
    setups, steps = _mix()
    need = sorted(workspace_bytes(s.params) for s in setups)
    budget = need[-1] + need[-2] + 4096  # room for two of the largest at most
    out, peak, stats = _serve(setups, steps, budget=budget)
    assert 1 <= peak <= 3
    assert stats["peak_bytes_in_use"] <= budget
    assert all(out[i][0] == 0 for i in range(len(setups)))
    # same results as with a large pool (admission order does not change a run)
    ref, _, _ = _serve(setups, steps)
    for i in range(len(setups)):
        assert np.array_equal(out[i][2], ref[i][2])


def test_rejects_what_it_cannot_serve():
    from paper_2207_13962_amd.fslbm import FslbmError, Server
    srv = Server(8 * MB, max_slots=2)
    with pytest.raises(FslbmError):
        srv.submit(I.wave_slab(L=96), 10)  # workspace above the budget
    with pytest.raises(FslbmError):
        srv.submit(I.wave_slab(L=16), 0)
    srv.close()


def test_unstable_run_is_retired_others_unaffected():
    setups, steps = _mix()
    bad = I.droplet_impact(L=24, velocity=0.6, variant=I.OM)  # drop faster than c_s
    ref, _, _ = _serve(setups, steps)
    out, _, _ = _serve(setups + [bad], steps + [120], order=[5, 0, 1, 2, 3, 4])
    assert out[5][0] == -4  # FSLBM_EUNSTABLE
    for i in range(len(setups)):
        assert out[i][0] == 0
        assert np.array_equal(out[i][2], ref[i][2])
    # the failed run itself: the same state as in a single context
    from paper_2207_13962_amd.fslbm import Simulation
    sim = Simulation(bad)
    sim.step(120)
    f = sim.fields(pdf=False, check=False)
    sim.close()
    assert f["status"] == -4
    assert np.array_equal(out[5][2], f["phi"], equal_nan=True)


def test_unstable_run_stops_advancing():
    """After the step that flags an instability no step kernel changes the
    state (two further steps bring back the same buffers)."""
    from paper_2207_13962_amd.fslbm import Simulation
    sim = Simulation(I.droplet_impact(L=24, velocity=0.6, variant=I.OM))
    sim.step(10)
    a = sim.fields(pdf=True, check=False)
    sim.step(2)
    b = sim.fields(pdf=True, check=False)
    sim.step(30)
    c = sim.fields(pdf=True, check=False)
    sim.close()
    assert a["status"] == b["status"] == -4
    for k in ("type", "phi", "mass", "pdf"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k
        assert np.array_equal(a[k], c[k], equal_nan=True), k


def _aux_mix(storage=I.F32):
    """Runs that need the launches beside the step: surface tension with one
    enclosed bubble (a rising bubble in a tube), surface tension alone (a
    resting drop), one enclosed bubble without surface tension (a closed dam
    break), and a plain drop impact, all in one launch group."""
    taylor = I.taylor_bubble(nx=20, ny=20, nz=40, tube_radius=8.5, bubble_radius=5.0, z0=10.0, length=10.0,
                             g=1e-5, nu=0.01, sigma=1e-3, storage=storage, variant=I.OM, collision=I.SRT,
                             q=19)
    drop = I.sphere_drop_static(L=20, radius=5.0, sigma=2e-3, storage=storage)
    dam = I.rect_dam_break(nx=32, ny=24, nz=12, wx=10, hy=18, g=2e-4, nu=5e-3, collision=I.SRT,
                           storage=storage, variant=I.NBKC)
    dam.params = dam.params.with_(bubble_model=1)
    plain = I.droplet_impact(L=24, velocity=0.03, variant=I.NBRC, storage=storage)
    return [taylor, drop, dam, plain], [70, 45, 60, 50]


def test_surface_tension_and_bubble_runs_served():
    """Served runs with surface tension or the single-bubble model equal
    their single-context runs bitwise (fill levels, total mass, volume
    pressure), alone and in the mix."""
    from paper_2207_13962_amd.fslbm import Simulation
    setups, steps = _aux_mix()
    mixed, peak, _ = _serve(setups, steps)
    assert peak == len(setups)
    for i, s in enumerate(setups):
        alone, _, _ = _serve([s], [steps[i]])
        st_m, rep_m, phi_m = mixed[i]
        st_a, rep_a, phi_a = alone[0]
        assert st_m == st_a == 0
        assert np.array_equal(phi_m, phi_a), i
        sim = Simulation(s)
        sim.step(steps[i])
        r = sim.mass()
        phi_s = sim.fields(pdf=False)["phi"]
        sim.close()
        assert np.array_equal(phi_m, phi_s), i
        assert rep_m["total_mass"] == r["total_mass"]
        assert rep_m["p_volume"] == r["p_volume"] == rep_a["p_volume"], i
        assert rep_m["bubble_volume"] == r["bubble_volume"]


def test_served_surface_tension_run_matches_oracle():
    """A served FP64 rising bubble (surface tension, volume pressure) against
    the oracle: fill levels and mass within 1e-12, the volume pressure too."""
    from oracle import Oracle
    setups, steps = _aux_mix(I.F64)
    out, _, _ = _serve(setups[:3], steps[:3], ticks=9)
    for i in range(3):
        o = Oracle(setups[i])
        assert o.step(steps[i]) == 0
        f, r = o.fields(), o.mass()
        st, rep, phi = out[i]
        assert st == 0
        ifc = f["type"] == I.INTERFACE
        assert np.abs(phi[ifc] - f["phi"][ifc]).max() < 1e-12, i
        assert abs(rep["total_mass"] - r.total_mass) <= 1e-12 * r.total_mass
        assert abs(rep["p_volume"] - r.p_volume) <= 1e-12 * r.p_volume


def _tracked_mix():
    """Runs with tracked bubbles (merging, splitting, across a periodic face,
    D3Q27, a rising bubble with surface tension in a tube, and one in the
    in-place layout) beside runs without them, in several launch groups."""
    merge = I.bubble_pair("merge", storage=I.F64, g=1e-4)
    split = I.bubble_pair("split", q=27, storage=I.F32, g=1e-4)
    straddle = I.bubble_pair("straddle", periodic_x=True, g=2e-4, storage=I.F64)
    taylor = I.taylor_bubble(nx=20, ny=20, nz=40, tube_radius=8.5, bubble_radius=5.0, z0=10.0, length=10.0,
                             g=1e-5, nu=0.01, sigma=1e-3, storage=I.F32, variant=I.OM, collision=I.SRT, q=19)
    taylor.params = taylor.params.with_(bubble_model=2)
    plain = I.droplet_impact(L=24, velocity=0.03, variant=I.NBRC)
    single = I.rect_dam_break(nx=32, ny=24, nz=12, wx=10, hy=18, g=2e-4, nu=5e-3, collision=I.SRT,
                              storage=I.F32, variant=I.NBKC)
    single.params = single.params.with_(bubble_model=1)
    inplace = I.bubble_pair("merge", storage=I.F32, g=1e-4)
    inplace.params = inplace.params.with_(layout=I.AA)
    return [merge, split, straddle, taylor, plain, single, inplace], [41, 37, 60, 55, 45, 52, 43]


def test_tracked_bubble_runs_served():
    """Served runs with tracked bubbles equal their single-context runs
    bitwise (fill levels, total mass, bubble volume, volume pressure), alone
    and in a mix with other runs; the per-bubble totals are order-free sums,
    so this holds whatever shares the launches."""
    from paper_2207_13962_amd.fslbm import Simulation
    setups, steps = _tracked_mix()
    mixed, peak, _ = _serve(setups, steps, ticks=6)
    assert peak == len(setups)
    # two slots: runs are admitted at later ticks of either parity
    staged, peak2, _ = _serve(setups, steps, max_slots=2, ticks=5)
    assert peak2 == 2
    for i in range(len(setups)):
        assert staged[i][0] == 0 and np.array_equal(staged[i][2], mixed[i][2]), i
    for i, s in enumerate(setups):
        alone, _, _ = _serve([s], [steps[i]], ticks=13)
        st_m, rep_m, phi_m = mixed[i]
        st_a, rep_a, phi_a = alone[0]
        assert st_m == st_a == 0, i
        assert np.array_equal(phi_m, phi_a), i
        sim = Simulation(s)
        sim.step(steps[i])
        r = sim.mass()
        phi_s = sim.fields(pdf=False)["phi"]
        sim.close()
        assert np.array_equal(phi_m, phi_s), i
        for k in ("total_mass", "bubble_volume", "p_volume"):
            assert rep_m[k] == r[k] == rep_a[k], (i, k)


def test_served_tracked_bubbles_match_oracle():
    """A served FP64 merge of two bubbles against the oracle: fill levels and
    total mass within 1e-12."""
    from oracle import Oracle
    s = I.bubble_pair("merge", storage=I.F64, g=1e-4)
    out, _, _ = _serve([s, I.droplet_impact(L=20, velocity=0.02)], [40, 30], ticks=9)
    o = Oracle(s)
    assert o.step(40) == 0
    f, r = o.fields(), o.mass()
    st, rep, phi = out[0]
    assert st == 0
    ifc = f["type"] == I.INTERFACE
    assert np.abs(phi[ifc] - f["phi"][ifc]).max() < 1e-12
    assert abs(rep["total_mass"] - r.total_mass) <= 1e-12 * r.total_mass
