"""The batched ensemble (one persistent launch per stage over members of
uneven order and resolution) against the plain per-member path, graphs
against eager launches, and the autotuner's schedule."""
import os
import sys

import numpy as np
import pytest

from dg_inputs import band_limited_state, ensemble_members, lake_at_rest_state
from oracle import SphereDG
from parity_util import TOL, errors

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MEMBERS = [
    {"n_lon": 24, "n_lat": 12, "order": 2},
    {"n_lon": 40, "n_lat": 20, "order": 4},
    {"n_lon": 13, "n_lat": 7, "order": 3},
    {"n_lon": 90, "n_lat": 45, "order": 3},
    {"n_lon": 32, "n_lat": 16, "order": 1},
    {"n_lon": 9, "n_lat": 1, "order": 0},
    {"n_lon": 36, "n_lat": 18, "order": 5},
    {"n_lon": 20, "n_lat": 10, "order": 7},
]


@pytest.fixture(scope="module")
def dg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2303_11767_amd as dg
    return dg


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def build(dg, dtype, members=MEMBERS):
    href = 1e4 if dtype == "f32" else 0.0
    ens = dg.Ensemble(members, dtype=dtype, h_ref=href)
    q = ens.empty_state()
    infos = []
    for k, (m, v) in enumerate(zip(ens.members, ens.views(q))):
        qh, info = band_limited_state(m.n_lon, m.n_lat, m.order, 4, 900 + k)
        v.copy_(torch.from_numpy(qh).to(v.dtype))
        infos.append(info)
    dts = [dg.cfl_time_step(m, i.cmax, 0.1) for m, i in zip(ens.members, infos)]
    ens.set_dt(dts)
    return ens, q, dts


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ensemble_stage_equals_plain_members(dg, dtype):
    say("ensemble stage vs plain", dtype)
    ens, q, dts = build(dg, dtype)
    out = ens.empty_state()
    ens.rk_stage(q, None, out, 0.0, 1.0)
    for k, (m, qv, ov) in enumerate(zip(ens.members, ens.views(q), ens.views(out))):
        ref = torch.empty_like(qv)
        m.rk_stage(qv.contiguous(), None, ref, 0.0, 1.0, dts[k])
        same = torch.equal(ov, ref)
        err = (ov.double() - ref.double()).abs().max().item() / max(ref.double().abs().max().item(), 1e-300)
        say("  member", k, m.n_lon, m.n_lat, m.order, "bitwise" if same else f"rel {err:.2e}")
        assert err <= (1e-14 if dtype == "f64" else 1e-6)
    # gaps between members are untouched
    for k in range(ens.n):
        lo, hi = ens.offsets[k] + ens.members[k].state_size(), ens.offsets[k + 1]
        assert torch.all(out[lo:hi] == 0)


def test_ensemble_rhs_vs_oracle(dg):
    """Every member's RHS from one ensemble launch against the oracle, FP64
    and FP32 (componentwise bar)."""
    for dtype in ("f64", "f32"):
        say("ensemble rhs vs oracle", dtype)
        ens, q, dts = build(dg, dtype)
        out = ens.rhs(q)
        for k, m in enumerate(ens.members):
            qh = ens.views(q)[k].cpu().numpy().astype(np.float64)
            got = ens.views(out)[k].cpu().numpy()
            o = SphereDG(m.n_lon, m.n_lat, m.order)
            comp, norm = errors(got, o.rhs(qh), o.rhs_scale(qh))
            say("  member", k, m.n_lon, m.n_lat, m.order, "componentwise", comp)
            assert np.all(comp <= TOL[dtype])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ensemble_steps_equal_plain_steps(dg, dtype):
    say("ensemble steps vs plain", dtype)
    ens, q, dts = build(dg, dtype)
    q_plain = [v.clone() for v in ens.views(q)]
    ens.rk_step(q, ens.empty_work(), nsteps=20)
    for k, (m, qv) in enumerate(zip(ens.members, ens.views(q))):
        m.rk_step(q_plain[k], m.empty_work(), dts[k], nsteps=20)
        err = (qv.double() - q_plain[k].double()).abs().max().item() / q_plain[k].double().abs().max().item()
        say("  member", k, "bitwise" if torch.equal(qv, q_plain[k]) else f"rel {err:.2e}")
        assert err <= (1e-13 if dtype == "f64" else 1e-6)


ORDERS = sorted({m["order"] for m in MEMBERS})


def test_schedule_does_not_change_results(dg):
    """With every member in the line layout (the fused launch runs that layout
    only): per-order and fused schedules of any shape give the same stage to
    rounding (each schedule runs its own compiled kernel, whose multiply-add
    contraction may differ), and every schedule is bitwise reproducible."""
    say("schedules")
    ens, q, dts = build(dg, "f32")
    for o in ORDERS:
        ens.set_kernel(o, "line")
    ref = ens.empty_state()
    ens.rk_stage(q, None, ref, 0.0, 1.0)

    def rel_err(out):
        # per member and variable, against that variable's largest value
        worst = 0.0
        for m, o, r in zip(ens.members, ens.views(out), ens.views(ref)):
            o3, r3 = o.double().view(m.E, 3, -1), r.double().view(m.E, 3, -1)
            for v in range(3):
                d = (o3[:, v] - r3[:, v]).abs().max().item()
                worst = max(worst, d / max(r3[:, v].abs().max().item(), 1e-300))
        return worst

    for w, g, f in [(1, 1, 0), (1, 7, 1), (2, 64, 0), (4, 3, 1), (4, 1000, 0), (2, 100000, 1), (4, 0, 0), (2, 0, 1)]:
        ens.set_schedule(w, g, f)
        out, again = ens.empty_state(), ens.empty_state()
        ens.rk_stage(q, None, out, 0.0, 1.0)
        ens.rk_stage(q, None, again, 0.0, 1.0)
        err = rel_err(out)
        say("  schedule", w, g, f, "bitwise" if torch.equal(out, ref) else f"rel {err:.2e}")
        assert torch.equal(out, again), (w, g, f)
        assert err <= 1e-6, (w, g, f, err)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_layouts_per_order_match_plain_members(dg, dtype):
    """Every order of the ensemble in each stage-kernel layout: one batched
    stage equals each member's own stage in the same layout (to roundoff; the
    same arithmetic), under per-order flat and persistent schedules; the
    fused launch refuses other layouts than the line one."""
    say("ensemble layouts", dtype)
    ens, q, dts = build(dg, dtype)
    for lay in ("line", "half"):
        for o in ORDERS:
            ens.set_kernel(o, lay)
            assert ens.kernel(o) == lay
            for sched in ((4, 0, 0), (2, 300, 0)):
                ens.set_schedule(*sched)
                out = ens.empty_state()
                ens.rk_stage(q, None, out, 0.0, 1.0)
                for k, (m, qv, ov) in enumerate(zip(ens.members, ens.views(q), ens.views(out))):
                    m.kernel = ens.kernel(m.order)
                    ref = torch.empty_like(qv)
                    m.rk_stage(qv.contiguous(), None, ref, 0.0, 1.0, dts[k])
                    err = (ov.double() - ref.double()).abs().max().item() / ref.double().abs().max().item()
                    assert err <= (1e-14 if dtype == "f64" else 1e-6), (lay, o, sched, k, err)
            if lay != "line":
                with pytest.raises(dg.DGError) as ei:
                    ens.set_schedule(4, 0, 1)
                assert ei.value.code == dg._lib.DG_EINVAL
            ens.set_kernel(o, "line")
    with pytest.raises(dg.DGError):
        ens.set_kernel(6, "half")          # no member of order 6


def test_autotune_and_cache(dg, tmp_path):
    say("autotune")
    ens, q, dts = build(dg, "f32")
    path = str(tmp_path / "tune.txt")
    w, g, f = ens.autotune(q, ens.empty_work(), path)
    lays = {o: ens.kernel(o) for o in ORDERS}
    say("  chosen", (w, g, f), lays)
    assert w in (1, 2, 4) and g >= 0          # 0: flat, one workgroup per w items
    # one line: key, the schedule and one layout per order 0..7
    assert os.path.exists(path) and len(open(path).read().split()) == 4 + 8
    for o in ORDERS:
        ens.set_kernel(o, "line")
    ens.set_schedule(1, 1, not f if all(v == "line" for v in lays.values()) else 0)
    assert ens.autotune(q, ens.empty_work(), path) == (w, g, f)
    assert {o: ens.kernel(o) for o in ORDERS} == lays
    # the tuned configuration still computes the members' own stages
    out = ens.empty_state()
    ens.rk_stage(q, None, out, 0.0, 1.0)
    for k, (m, qv, ov) in enumerate(zip(ens.members, ens.views(q), ens.views(out))):
        m.kernel = ens.kernel(m.order)
        ref = torch.empty_like(qv)
        m.rk_stage(qv.contiguous(), None, ref, 0.0, 1.0, dts[k])
        err = (ov.double() - ref.double()).abs().max().item() / ref.double().abs().max().item()
        assert err <= 1e-6, (k, err)


def test_graph_replays_match_eager(dg):
    """A captured 5-step graph replayed three times, with eager work and
    synchronisation between replays, equals 5-step eager runs each time."""
    say("graph replays")
    ens, q, dts = build(dg, "f64")
    work = ens.empty_work()
    qg = q.clone()
    g = ens.graph(qg, work, nsteps=5)
    qe = q.clone()
    we = ens.empty_work()
    for rep in range(3):
        g.launch()
        ens.rk_step(qe, we, nsteps=5)
        torch.cuda.synchronize()
        _ = (qe * 2).sum().item()          # eager work between replays
        assert torch.equal(qg, qe), rep
    g.close()
    # single-mesh graph
    m = ens.members[3]
    qm = ens.views(q)[3].clone()
    wm = m.empty_work()
    gm = m.graph(qm, wm, dts[3], nsteps=4)
    qref = qm.clone()
    for rep in range(3):
        gm.launch()
        m.rk_step(qref, m.empty_work(), dts[3], nsteps=4)
        torch.cuda.synchronize()
        assert torch.equal(qm, qref), rep
    gm.close()


def test_graph_pins_schedule_and_owner(dg):
    """A live graph bakes in the ensemble's schedule and tables: changing the
    schedule or autotuning is refused while it lives, and freeing the
    ensemble (or a mesh) under a live graph defers the release, so the graph
    still replays correctly; after the graph is freed the schedule can
    change again."""
    say("graph pins schedule and owner")
    ens, q, dts = build(dg, "f32")
    work = ens.empty_work()
    qe, we = q.clone(), ens.empty_work()
    ens.rk_step(qe, we, nsteps=2)
    qg = q.clone()
    g = ens.graph(qg, work, nsteps=2)
    with pytest.raises(dg.DGError) as ei:
        ens.set_schedule(2, 64, 0)
    assert ei.value.code == -1
    with pytest.raises(dg.DGError):
        ens.autotune(q, ens.empty_work())
    g.close()
    ens.set_schedule(2, 64, 0)                       # no live graph: allowed again
    # free under a live graph: the C release is deferred to dg_graph_free
    lib = ens._lib
    import ctypes
    gh = ctypes.c_void_p()
    qg2 = q.clone()
    assert lib.dg_graph_ens(ens._e, ctypes.c_void_p(qg2.data_ptr()), ctypes.c_void_p(work.data_ptr()),
                            2, ctypes.byref(gh)) == 0
    for m in ens.members:
        m._ctx = None
    assert lib.dg_ens_free(ens._e) == 0
    ens._e = None
    assert lib.dg_graph_launch(gh, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(qg2, qe)
    assert lib.dg_graph_free(gh) == 0
    # the same for a single mesh
    mesh = dg.Mesh(24, 12, 2, dtype="f64")
    qm, _ = band_limited_state(24, 12, 2, 4, 77)
    qa = torch.from_numpy(qm).cuda()
    qb = qa.clone()
    mesh.rk_step(qb, mesh.empty_work(), 10.0, nsteps=3)
    wm = mesh.empty_work()
    gm = ctypes.c_void_p()
    assert lib.dg_graph_rk(mesh._ctx, ctypes.c_void_p(qa.data_ptr()), ctypes.c_void_p(wm.data_ptr()),
                           10.0, 3, 3, ctypes.byref(gm)) == 0
    assert lib.dg_free(mesh._ctx) == 0
    mesh._ctx = None
    assert lib.dg_graph_launch(gm, None) == 0
    torch.cuda.synchronize()
    assert torch.equal(qa, qb)
    assert lib.dg_graph_free(gm) == 0


def test_full_ensemble_sampled_members_vs_oracle(dg):
    """The 64-member FP32 ensemble of the benchmark (orders 2-4, 90x45 ..
    360x180) in its autotuned launch configuration: three members (the first,
    the first of the largest shape and one of another order) hold seeded
    band-limited states and are checked against the oracle one by one; the
    other members hold a lake at rest and must stay finite."""
    mem = ensemble_members(64, seed=4)
    say("full ensemble", len(mem), "members")
    ens = dg.Ensemble(mem, dtype="f32", h_ref=1e4)
    q = ens.empty_state()
    big = next(k for k, m in enumerate(mem) if (m["n_lon"], m["n_lat"], m["order"]) == (360, 180, 4))
    other = next(k for k, m in enumerate(mem) if m["order"] != mem[0]["order"] and k != big)
    sampled = {0, big, other}
    states = {}
    for k, (m, v) in enumerate(zip(ens.members, ens.views(q))):
        if k in sampled:
            qh, _ = band_limited_state(m.n_lon, m.n_lat, m.order, 8, 7000 + k)
            states[k] = qh
        else:
            qh = lake_at_rest_state(m.n_lon, m.n_lat, m.order)
        v.copy_(torch.from_numpy(qh).to(v.dtype))
    ens.autotune(q, ens.empty_work())
    out = ens.rhs(q)
    assert torch.isfinite(out).all()
    for k in sorted(sampled):
        m = ens.members[k]
        qin = states[k].astype(np.float32).astype(np.float64)
        o = SphereDG(m.n_lon, m.n_lat, m.order)
        comp, _ = errors(ens.views(out)[k].cpu().numpy(), o.rhs(qin), o.rhs_scale(qin))
        say("  member", k, m.n_lon, m.n_lat, m.order, "componentwise", comp)
        assert np.all(comp <= TOL["f32"]), (k, comp)
