"""Batched ensembles through the C ABI: every member of a batch must come out
bit for bit as the same simulation stepped alone (the per-site update does not
depend on how tiles are grouped into launches), across mixed sizes and
precisions, follow-wall members, graph re-capture and membership changes."""
import numpy as np
import pytest

import synth_inputs as si

pytestmark = pytest.mark.gpu


def _solo(cfg, steps):
    from paper_2303_02210_amd import Sim
    s = Sim(cfg)
    s.step(steps)
    out = (s.populations(), s.front_heights(), s.diagnostics())
    s.close()
    return out


def _same(member, ref, tag):
    f, h, d = ref
    assert np.array_equal(member.populations(), f), tag
    assert np.array_equal(member.front_heights(), h), tag
    dm = member.diagnostics()
    for k in ("step", "y_wall", "h_hi", "status", "hbar", "W", "divisions", "lam", "rows_swept"):
        assert dm[k] == d[k], (tag, k, dm[k], d[k])
    for k in ("mass", "src_total", "fix_total", "retired"):
        assert abs(dm[k] - d[k]) <= 1e-12 * max(1.0, abs(d["mass"])), (tag, k)


MIXED = [
    si.cfg(L=128, H=256, init_rows=64, growth_rate=1e-3, sigma=1e-3, precision="fp32", seed=1, replica=1),
    si.cfg(L=256, H=192, init_rows=40, growth_rate=2e-3, sigma=1e-3, precision="fp32", seed=2, replica=2),
    si.cfg(L=64, H=64, init_rows=16, growth_rate=1e-3, precision="fp64", seed=3),
    si.cfg(L=96, H=128, init_rows=30, tau=0.8, growth_rate=1e-3, sigma=1e-3, region="front_band",
           region_width=8, precision="fp16", seed=4),
    si.cfg(L=200, H=96, init_rows=30, growth_rate=1e-3, sigma=1e-3, precision="bf16", seed=5),
    si.cfg(L=130, H=80, init_rows=20, growth_rate=1e-3, sigma=1e-3, precision="fp32", seed=6),
    si.cfg(L=72, H=128, init_rows=90, sigma=1e-2, growth_rate=1e-2, ybc="follow", wall_min_gap=20,
           precision="fp64", seed=7),
    si.cfg(L=128, H=256, init_rows=40, sigma=1e-3, growth_rate=3e-3, window=True, precision="fp32",
           seed=8),
    si.cfg(L=96, H=160, init_rows=100, sigma=1e-2, growth_rate=1e-2, ybc="follow", wall_min_gap=10,
           window=True, precision="fp64", seed=9),
    si.cfg(L=128, H=192, init_rows=100, sigma=1e-3, growth_rate=5e-3, ybc="follow", wall_min_gap=10,
           window=True, precision="fp16", seed=10),
]


def test_batch_members_match_solo_runs_bitwise():
    from paper_2303_02210_amd import Ensemble
    ens = Ensemble(MIXED)
    for n in (10, 10, 17):          # graph captured for 10, replayed, re-captured for 17
        ens.step(n)
    ens.synchronize()
    for i, (c, m) in enumerate(zip(MIXED, ens.members)):
        _same(m, _solo(c, 37), i)


DIVISION = [
    si.cfg(L=128, H=192, init_rows=48, growth="division", growth_rate=5e-3, sigma=1e-3,
           precision="fp32", seed=11),
    si.cfg(L=128, H=192, init_rows=48, growth_rate=5e-3, sigma=1e-3, precision="fp32", seed=11),
    si.cfg(L=96, H=96, init_rows=30, growth="division_density", growth_rate=1e-2, sigma=1e-2,
           precision="fp64", seed=12),
    si.cfg(L=130, H=128, init_rows=30, tau=0.8, growth="division", growth_rate=5e-3, sigma=1e-3,
           region="front_band", region_width=6, precision="fp16", seed=13),
    si.cfg(L=96, H=160, init_rows=100, sigma=1e-2, growth="division", growth_rate=1e-2,
           ybc="follow", wall_min_gap=10, window=True, precision="fp64", seed=14),
    si.cfg(L=200, H=96, init_rows=30, growth="division_density", growth_rate=5e-3, sigma=1e-3,
           precision="bf16", seed=15),
]


def test_batch_division_members_match_solo_runs_bitwise():
    """Division-law members (their per-step rate is reduced on the device from
    the previous step's tallies) batched beside a bulk-growth member of the
    same kernel form."""
    from paper_2303_02210_amd import Ensemble
    ens = Ensemble(DIVISION)
    for n in (8, 8, 13):
        ens.step(n)
    ens.synchronize()
    for i, (c, m) in enumerate(zip(DIVISION, ens.members)):
        ref = _solo(c, 29)
        _same(m, ref, i)
        if c["growth"] != "bulk":
            assert ref[2]["divisions"] > 0, i


def test_batch_membership_changes_and_solo_steps():
    from paper_2303_02210_amd import Ensemble
    a, b, c = MIXED[0], MIXED[2], MIXED[6]
    ens = Ensemble([a, b])
    ens.step(5)
    ma, mb = ens.members
    mb.step(3)                          # stepped on its own in between
    mc = ens.add(c)                     # joins late
    ens.step(7)
    ens.remove(ma)
    ens.step(4)
    ens.synchronize()
    _same(ma, _solo(a, 12), "a")
    _same(mb, _solo(b, 19), "b")
    _same(mc, _solo(c, 11), "c")


def test_large_members_step_alone_and_match():
    """With a size threshold, members at or above it without a window step
    by their own launches, the rest through the batch (a windowed member
    above it stays batched); every member matches its solo run, also after
    a member leaves, and an ensemble whose members all step alone works."""
    from paper_2303_02210_amd import Ensemble
    ens = Ensemble(MIXED, solo_min_sites=128 * 192)
    members = list(ens.members)                 # in the order of MIXED
    alone = ens.stepped_alone
    assert {(m.cfg["L"], m.cfg["H"]) for m in alone} == {(128, 256), (256, 192)}
    ens.step(6)
    ens.remove(alone[0])
    ens.step(5)
    ens.synchronize()
    for c, m in zip(MIXED, members):
        _same(m, _solo(c, 6 if m is alone[0] else 11), (c["L"], c["H"]))
    ens.close()
    ens = Ensemble(MIXED[:2], solo_min_sites=1)
    assert len(ens.stepped_alone) == 2
    ens.step(4)
    ens.step(4)                                 # the graph replayed: the steps go on
    ens.synchronize()
    for c, m in zip(MIXED[:2], ens.members):
        _same(m, _solo(c, 8), "all alone")
    # a member must use the ensemble's stream, whichever way it is stepped
    from paper_2303_02210_amd import LbmError, Sim
    other = Sim(dict(MIXED[0], batch_own=True))
    with pytest.raises(LbmError):
        ens.add(other)
    other.close()
    ens.close()


def test_batch_on_null_stream_runs_without_graph():
    import torch
    from paper_2303_02210_amd import Ensemble
    ens = Ensemble(MIXED[:3], stream=torch.cuda.default_stream())
    ens.step(6)
    ens.synchronize()
    for i in range(3):
        _same(ens.members[i], _solo(MIXED[i], 6), i)


def test_batch_member_fault_is_its_own():
    from paper_2303_02210_amd import Ensemble, LbmError
    full = si.cfg(L=64, H=24, init_rows=20, growth_rate=5e-2, precision="fp32")
    ok = MIXED[0]
    ens = Ensemble([full, ok])
    ens.step(400)
    ens.synchronize()
    bad, good = ens.members
    with pytest.raises(LbmError, match="DOMAIN_FULL"):
        bad.front_heights()
    with pytest.raises(LbmError, match="STATE"):
        ens.step(1)
    ens.remove(bad)
    ens.step(3)
    ens.synchronize()
    _same(good, _solo(ok, 403), "good")


def test_server_results_equal_solo_runs():
    """Continuous batching: requests join and leave the running batches (one
    per lane: storage type and width class, each on its own stream) at
    different times; each finished run equals the same run stepped alone."""
    from paper_2303_02210_amd.serve import Server, lane_index
    reqs = []
    for k, (L, H, prec, steps, t) in enumerate([
            (128, 256, "fp32", 230, 0.0), (64, 192, "fp64", 150, 0.0), (256, 512, "fp16", 310, 0.0),
            (128, 384, "fp32", 120, 0.05), (192, 256, "bf16", 90, 0.1), (64, 128, "fp64", 260, 0.1),
            (1024, 192, "fp16", 70, 0.05), (1024, 160, "fp32", 110, 0.1)]):
        reqs.append(si.cfg(name=f"r{k}", L=L, H=H, init_rows=100, sigma=1e-3, growth_rate=2e-3,
                           ybc="follow", wall_min_gap=20, window=True, precision=prec,
                           steps=steps, seed=k, arrival_s=t))
    srv = Server(hbm_budget=4e9, tick_steps=40, keep_results=True)
    summ = srv.serve(reqs)
    srv.close()
    assert summ["completed"] == len(reqs) and summ["p99_latency_s"] is not None
    for r in srv.done:
        f, h, d = r.result
        ref = _solo(r.req, r.req["steps"])
        assert np.array_equal(f, ref[0]), r.req["name"]
        assert np.array_equal(h, ref[1]), r.req["name"]
        assert d["step"] == r.req["steps"] and d["y_wall"] == ref[2]["y_wall"]
        assert r.h_updates >= r.req["steps"] // 40
    # the runs were spread over five of the six lanes
    assert len({lane_index(q, 6) for q in reqs}) == 5
    assert len({id(r.lane) for r in srv.done}) == 5


def test_persistent_batch_matches_solo_runs_bitwise():
    """lbm_batch_persistent: the table groups of members that neither move
    their wall or window nor divide run each lbm_batch_step in one
    cooperative launch with a grid-wide barrier between steps; the others
    (follow wall, window, division laws) launch per step.  Every member
    matches its solo run bit for bit, across runs of different lengths, a
    member stepped on its own in between, and a membership change, and no
    barrier gives up."""
    from paper_2303_02210_amd import Ensemble
    from paper_2303_02210_amd import _ffi
    cfgs = MIXED + DIVISION[:2]
    ens = Ensemble(cfgs, solo_min_sites=None, persistent=True)
    members = list(ens.members)
    for n in (1, 9, 9, 16):
        ens.step(n)
    members[1].step(2)                  # on its own in between
    ens.remove(members[2])
    ens.step(5)
    ens.synchronize()
    for i, (c, m) in enumerate(zip(cfgs, members)):
        steps = 35 + (5 if i != 2 else 0) + (2 if i == 1 else 0)
        _same(m, _solo(c, steps), ("persistent", i))
        assert not (m.diagnostics()["status"] & _ffi.ST_SYNC_LOST)
    ens.close()
