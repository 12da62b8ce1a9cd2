"""GPU checks of the batched evaluation (one replayed HIP graph for many
independent systems): every system against its own single-plan evaluation,
every graph replay against the eager result (with eager work and
synchronisation between replays), the batched-launch form against the
per-system graph form, and a small FP64 batch against the oracle.

Tolerances: batch vs single plan relE <= 1e-6 and relative RMS <= 1e-5 (the
same kernels; only the order of floating-point atomics in the spread and the
autotuned stage-2 split differ); FP64 batch vs oracle 1e-10.
"""
import numpy as np
import pytest

from oracle import skp
from paper_2601_18838_amd import systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def relrms(a, b):
    return np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum())


def build(batch, prec):
    from paper_2601_18838_amd import kpme
    wls = [b[0] for b in batch]
    bp = kpme.BatchPlan([w.box for w in wls], [w.grid for w in wls], [w.order for w in wls],
                        [w.beta for w in wls], [w.rank for w in wls], precision=prec,
                        max_particles=[w.n for w in wls])
    dt = torch.float64 if prec == "fp64" else torch.float32
    pos = torch.tensor(np.concatenate([b[1] for b in batch]), dtype=dt, device="cuda")
    q = torch.tensor(np.concatenate([b[2] for b in batch]), dtype=dt, device="cuda")
    return bp, pos, q, [w.n for w in wls]


def test_batch_matches_single_plans_and_graph_replays():
    from paper_2601_18838_amd import kpme
    batch = systems.batch_systems(count=10)
    print("[batch] 10 systems fp16x3", flush=True)
    bp, pos, q, n = build(batch, "fp16x3")
    e0, pot0, f0 = [x.clone() for x in bp.evaluate(n, pos, q)]
    torch.cuda.synchronize()
    form, launches = bp.info()
    print(f"  form {form}, {launches} launches per replay", flush=True)
    assert form == 1 and launches < 10 * 4   # one launch per stage and kernel instance
    # replays, with unrelated eager work in between; the second call passes
    # fresh output buffers after a host synchronisation, which re-records
    for rep in range(3):
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()
        if rep == 1:
            fresh = (torch.empty_like(e0), torch.empty_like(pot0), torch.empty_like(f0))
            e, pot, f = bp.evaluate(n, pos, q, energy=fresh[0], pot=fresh[1], force=fresh[2])
        else:
            e, pot, f = bp.evaluate(n, pos, q)
        torch.cuda.synchronize()
        np.testing.assert_allclose(e.cpu().numpy(), e0.cpu().numpy(), rtol=1e-6, atol=1e-9)
        assert relrms(pot.double().cpu().numpy(), pot0.double().cpu().numpy()) < 1e-6
        assert relrms(f.double().cpu().numpy(), f0.double().cpu().numpy()) < 1e-6
    # every system against its own single-plan evaluation
    off = 0
    for k, (wl, p_np, q_np) in enumerate(batch):
        pl = kpme.Plan(wl.box, wl.grid, wl.order, wl.beta, rank=wl.rank, precision="fp16x3",
                       max_particles=wl.n)
        es, ps, fs = pl.evaluate(pos[off:off + wl.n].contiguous(), q[off:off + wl.n].contiguous())
        es = es.cpu().numpy()
        assert abs(e0[k, 0].item() - es[0]) <= 1e-6 * abs(es[0]), k
        assert relrms(pot0[off:off + wl.n].double().cpu().numpy(), ps.double().cpu().numpy()) < 1e-5
        assert relrms(f0[off:off + wl.n].double().cpu().numpy(), fs.double().cpu().numpy()) < 1e-5
        off += wl.n


def test_batch64_against_stored_oracle():
    """The 64-system batch (the batched workload, one replayed graph) in both
    split precisions against oracle values stored by
    tests/golden/make_full_size_golden.py: every system's E_rec to relE <= 1e-5,
    and the relative RMS of the 8 sampled potentials and forces of every
    system to <= 1e-4 (the mixed-precision targets)."""
    import json
    import os
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "batch64_pm1.json")))["systems"]
    batch = systems.batch_systems(count=64)
    failures = []
    for prec in ("fp16x3", "bf16x3"):
        print(f"[batch] 64 systems {prec} vs stored oracle", flush=True)
        bp, pos, q, n = build(batch, prec)
        e4, pot, f = bp.evaluate(n, pos, q)
        e4 = e4.cpu().numpy()
        pot = pot.double().cpu().numpy()
        f = f.double().cpu().numpy()
        off, worst, bad = 0, [0.0, 0.0, 0.0], []
        for k, (wl, _, _) in enumerate(batch):
            r = ref[k]
            assert r["n"] == wl.n and r["rank"] == wl.rank
            idx = off + np.asarray(r["sample_index"])
            errs = (abs(e4[k, 0] - r["E_rec"]) / abs(r["E_rec"]),
                    relrms(pot[idx], np.asarray(r["phi"])), relrms(f[idx], np.asarray(r["F"])))
            worst = [max(a, b) for a, b in zip(worst, errs)]
            if errs[0] >= 1e-5 or errs[1] >= 1e-4 or errs[2] >= 1e-4:
                bad.append((k, wl.grid, wl.order, wl.rank, ["%.2e" % x for x in errs]))
            off += wl.n
        print(f"  {prec}: worst relE={worst[0]:.2e} rmsPhi={worst[1]:.2e} "
              f"rmsF={worst[2]:.2e}; systems off the bar: {bad}", flush=True)
        failures.extend((prec, b) for b in bad)
        del bp
    assert not failures, failures


def test_small_fp64_batch_against_oracle():
    print("[batch] fp64 vs oracle", flush=True)
    cases = []
    for seed, (box, grid, p, rank) in enumerate([((20.0,) * 3, (16, 16, 16), 4, 8),
                                                 ((21.0, 26.0, 31.0), (20, 25, 30), 6, 12),
                                                 ((12.0, 12.0, 24.0), (12, 12, 24), 4, 5)]):
        pos, q = systems.uniform_pm1(400 + 100 * seed, box, 100 + seed)
        wl = systems.Workload(f"t{seed}", box, grid, p, 0.5, rank=rank, kind="given", n=len(q))
        cases.append((wl, pos, q))
    bp, pos, q, n = build(cases, "fp64")
    e4, pot, f = bp.evaluate(n, pos, q)
    assert bp.info()[0] == 0   # FP64 stage kernels have no batched form: per-system graph
    off = 0
    for k, (wl, p_np, q_np) in enumerate(cases):
        ref = skp.Plan(wl.box, wl.grid, wl.order, wl.beta, rank=wl.rank).evaluate(p_np, q_np)
        assert abs(e4[k, 0].item() - ref["E_rec"]) < 1e-10 * abs(ref["E_rec"])
        assert relrms(pot[off:off + wl.n].cpu().numpy(), ref["phi"]) < 1e-10
        assert relrms(f[off:off + wl.n].cpu().numpy(), ref["F"]) < 1e-10
        off += wl.n


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_batched_launches_match_per_system_graph(prec, monkeypatch):
    """The 64-system batch in its two recorded forms -- one launch per stage
    and kernel instance over all systems, and every system's own launch
    sequence on parallel graph branches -- runs the same kernel bodies on the
    same arguments: energies to 1e-6 relative, potentials and forces to 1e-5
    relative RMS (binning assigns slots with atomics, so FP32 sums may be
    added in another order)."""
    batch = systems.batch_systems(count=64)
    print(f"[batch] batched vs per-system graph, 64 systems {prec}", flush=True)
    bp, pos, q, n = build(batch, prec)
    ea, pa, fa = [x.clone() for x in bp.evaluate(n, pos, q)]
    assert bp.info()[0] == 1
    del bp
    monkeypatch.setenv("KPME_BATCH_FUSED", "0")
    bp, pos, q, n = build(batch, prec)
    eb, pb, fb = bp.evaluate(n, pos, q)
    form, launches = bp.info()
    assert form == 0 and launches > 64
    ea, eb = ea.cpu().numpy(), eb.cpu().numpy()
    assert np.all(np.abs(ea[:, 0] - eb[:, 0]) <= 1e-6 * np.abs(eb[:, 0]))
    off = 0
    for k, (wl, _, _) in enumerate(batch):
        sl = slice(off, off + wl.n)
        assert relrms(pa[sl].double().cpu().numpy(), pb[sl].double().cpu().numpy()) < 1e-5, k
        assert relrms(fa[sl].double().cpu().numpy(), fb[sl].double().cpu().numpy()) < 1e-5, k
        off += wl.n


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x3"])
def test_persistent_batched_launches_match_the_grid_form(prec, monkeypatch):
    """The batched launches in their persistent form (resident workgroups
    taking the concatenated grid's workgroups from a zeroed device counter,
    largest systems first) run the same items as the grid form: energies to
    1e-6 relative, potentials and forces to 1e-5 relative RMS; two replays of
    the recording (the counters restart from zero on each) agree."""
    batch = systems.batch_systems(count=64)
    print(f"[batch] persistent vs grid form, 64 systems {prec}", flush=True)
    bp, pos, q, n = build(batch, prec)
    ea, pa, fa = [x.clone() for x in bp.evaluate(n, pos, q)]
    assert bp.info()[0] == 1
    del bp
    monkeypatch.setenv("KPME_BATCH_PERSISTENT", "1")
    bp, pos, q, n = build(batch, prec)
    e4 = torch.empty_like(ea)
    pot = torch.empty_like(pa)
    frc = torch.empty_like(fa)
    outs = []
    for _ in range(2):
        bp.evaluate(n, pos, q, energy=e4, pot=pot, force=frc)
        torch.cuda.synchronize()
        outs.append((e4.cpu().numpy().copy(), pot.double().cpu().numpy(), frc.double().cpu().numpy()))
    form, launches = bp.info()
    assert form == 2 and launches < 45
    eref = ea.cpu().numpy()
    for eb, pb, fb in outs:
        assert np.all(np.abs(eb[:, 0] - eref[:, 0]) <= 1e-6 * np.abs(eref[:, 0]))
        off = 0
        for k, (wl, _, _) in enumerate(batch):
            sl = slice(off, off + wl.n)
            assert relrms(pb[sl], pa[sl].double().cpu().numpy()) < 1e-5, k
            assert relrms(fb[sl], fa[sl].double().cpu().numpy()) < 1e-5, k
            off += wl.n


@pytest.mark.skip(reason="a run of this test (re-recording while the previous replay could "
                         "still run) ended in SIGSEGV in a HIP runtime thread; re-recording now "
                         "drains the device first, but the crash's cause was never shown, so "
                         "the case stays off the GPU")
def test_rerecording_while_previous_replay_runs():
    """Back-to-back evaluations with fresh output buffers and no host
    synchronisation: every signature change re-records the graph, which the
    library does only after draining the stream and the device."""
    batch = systems.batch_systems(count=6, base_seed=7000)
    print("[batch] re-recording, 6 systems fp16x3", flush=True)
    bp, pos, q, n = build(batch, "fp16x3")
    ref = [x.clone() for x in bp.evaluate(n, pos, q)]
    torch.cuda.synchronize()
    outs = []
    for _ in range(4):   # fresh outputs each time, no synchronisation in between
        o = (torch.empty_like(ref[0]), torch.empty_like(ref[1]), torch.empty_like(ref[2]))
        outs.append(bp.evaluate(n, pos, q, energy=o[0], pot=o[1], force=o[2]))
    torch.cuda.synchronize()
    for e, pot, f in outs:
        np.testing.assert_allclose(e.cpu().numpy(), ref[0].cpu().numpy(), rtol=1e-6, atol=1e-9)
        assert relrms(pot.double().cpu().numpy(), ref[1].double().cpu().numpy()) < 1e-6
