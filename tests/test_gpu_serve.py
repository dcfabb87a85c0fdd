"""GPU tests of the serving loop (mpm_server_*): continuous batching gives
every fit the same result as running it alone (small JTV-MAP fits in batched
groups included), admission respects the memory budget, an over-budget
request is rejected, and a cancelled request (queued, running, or running in a
group) leaves the others intact."""
import time

import numpy as np
import pytest

from conftest import cuda, f32, observations
from paper_2102_01604_amd import _lib, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _lib.load()
    return torch


def _requests(orc, torch):
    """A mix of ML and MAP fits of uneven sizes (inputs resident on the GPU)."""
    specs = [("map", (40, 33, 12), 1), ("ml", (64, 64, 16), 2), ("map", (24, 20, 30), 3), ("ml", (17, 9, 5), 4),
             ("map", (64, 48, 20), 5), ("map", (31, 31, 9), 6), ("ml", (96, 40, 8), 7)]
    out = []
    for mode, dims, seed in specs:
        c = synth.make_case("map_brain", dims=dims, seed=seed)
        c["b1"] = f32(c["b1"])
        x = observations(orc, c)
        opts = dict(c["opts"], mode=mode, n_outer=3, n_gn=3, n_cg=12) if mode == "map" else {"mode": "ml", "n_gn": 15}
        out.append({"case": c, "opts": opts, "X": cuda(x), "b1": cuda(c["b1"].astype(np.float32)),
                    "N": x.shape[1]})
    return out


def _drive(srv, tickets, timeout=120.0):
    reports = {}
    t0 = time.time()
    while len(reports) < len(tickets):
        srv.step()
        for t in tickets:
            if t not in reports:
                r = srv.poll(t)
                if r is not None:
                    reports[t] = r
        assert time.time() - t0 < timeout, "server did not finish in time"
    return reports


def test_mix_equals_alone(torch_cuda, orc):
    torch = torch_cuda
    reqs = _requests(orc, torch)
    alone = []
    for r in reqs:
        maps = torch.zeros((4, r["N"]), dtype=torch.float32, device="cuda")
        rep, _ = _lib.mpm_fit(r["case"]["proto"], r["case"]["dims"], r["X"], r["b1"], r["opts"], maps)
        alone.append((maps.cpu().numpy(), rep))
    with _lib.MpmServer(hbm_budget=64 << 30, max_active=4) as srv:
        outs = [torch.zeros((4, r["N"]), dtype=torch.float32, device="cuda") for r in reqs]
        tickets = [srv.submit(r["case"]["proto"], r["case"]["dims"], r["X"], r["b1"], r["opts"], o)
                   for r, o in zip(reqs, outs)]
        reports = _drive(srv, tickets)
    torch.cuda.synchronize()
    nbit = 0
    for (ref, rep_a), o, t in zip(alone, outs, tickets):
        got = o.cpu().numpy()
        nbit += int(np.array_equal(got, ref))
        rel = np.abs(got.astype(np.float64) - ref).max(axis=1) / np.abs(ref).max(axis=1)
        assert (rel <= 1e-6).all(), rel
        assert reports[t]["gn_done"] == rep_a["gn_done"]
        assert reports[t]["objective"] == pytest.approx(rep_a["objective"], rel=1e-9)
    print(f"{nbit}/{len(reqs)} fits bitwise identical alone and in the mix")
    assert nbit == len(reqs)


def test_budget_admission_and_rejection(torch_cuda, orc):
    torch = torch_cuda
    reqs = _requests(orc, torch)[:4]
    fps = [_lib.mpm_footprint_bytes(r["case"]["proto"], r["case"]["dims"], 0, 1 if r["opts"]["mode"] == "map" else 0)
           for r in reqs]
    budget = max(fps)  # at most one fit can be admitted at a time
    with _lib.MpmServer(hbm_budget=budget, max_active=4) as srv:
        outs = [torch.zeros((4, r["N"]), dtype=torch.float32, device="cuda") for r in reqs]
        tickets = [srv.submit(r["case"]["proto"], r["case"]["dims"], r["X"], r["b1"], r["opts"], o)
                   for r, o in zip(reqs, outs)]
        reports = _drive(srv, tickets)
        assert all(reports[t]["nonfinite_voxels"] == 0 for t in tickets)
        # a request bigger than the whole budget fails with MPM_ERR_OUT_OF_MEMORY
        big = synth.make_case("map_brain", dims=(80, 80, 40), seed=9)
        Xb = torch.zeros((22, 80 * 80 * 40), dtype=torch.float32, device="cuda") + 10.0
        mb = torch.zeros((4, 80 * 80 * 40), dtype=torch.float32, device="cuda")
        t = srv.submit(big["proto"], big["dims"], Xb, None, big["opts"], mb)
        with pytest.raises(_lib.MpmError) as ei:
            for _ in range(1000):
                srv.step()
                if srv.poll(t) is not None:
                    break
        assert ei.value.status == 3


def test_background_thread(torch_cuda, orc):
    torch = torch_cuda
    reqs = _requests(orc, torch)[:3]
    with _lib.MpmServer(hbm_budget=64 << 30, max_active=2, thread=True) as srv:
        outs = [torch.zeros((4, r["N"]), dtype=torch.float32, device="cuda") for r in reqs]
        tickets = [srv.submit(r["case"]["proto"], r["case"]["dims"], r["X"], r["b1"], r["opts"], o)
                   for r, o in zip(reqs, outs)]
        t0 = time.time()
        done = {}
        while len(done) < len(tickets):
            for t in tickets:
                if t not in done:
                    r = srv.poll(t)
                    if r is not None:
                        done[t] = r
            assert time.time() - t0 < 120
            time.sleep(0.002)
    assert all(d["gn_done"] > 0 for d in done.values())


def test_cancel_queued_and_running(torch_cuda, orc):
    """mpm_server_cancel: a queued request finishes at once as cancelled, a
    running MAP fit is released after its pieces in flight, and the request
    behind them still equals its solo fit."""
    torch = torch_cuda
    reqs = [_requests(orc, torch)[i] for i in (0, 2, 5)]  # three MAP fits
    r3 = reqs[2]
    solo = torch.zeros((4, r3["N"]), dtype=torch.float32, device="cuda")
    rep_solo, _ = _lib.mpm_fit(r3["case"]["proto"], r3["case"]["dims"], r3["X"], r3["b1"], r3["opts"], solo)
    # one stream, no groups: one fit runs at a time
    with _lib.MpmServer(hbm_budget=16 << 30, max_active=1, groups=False) as srv:
        outs = [torch.zeros((4, r["N"]), dtype=torch.float32, device="cuda") for r in reqs]
        tickets = [srv.submit(r["case"]["proto"], r["case"]["dims"], r["X"], r["b1"], r["opts"], o)
                   for r, o in zip(reqs, outs)]
        srv.step()  # admits the first fit and enqueues its first piece; the others wait
        srv.cancel(tickets[1])
        with pytest.raises(_lib.MpmError) as ei:
            srv.poll(tickets[1])
        assert ei.value.status == 7
        srv.cancel(tickets[0])
        t0, cancelled = time.time(), False
        while not cancelled:
            srv.step()
            try:
                assert srv.poll(tickets[0]) is None, "a cancelled fit reported success"
            except _lib.MpmError as e:
                assert e.status == 7
                cancelled = True
            assert time.time() - t0 < 60.0
        rep = _drive(srv, [tickets[2]])[tickets[2]]
        srv.cancel(tickets[2])  # finished: no effect
        assert srv.poll(tickets[2]) is not None
        with pytest.raises(_lib.MpmError) as ei:
            srv.cancel(10 ** 9)
        assert ei.value.status == 6
    torch.cuda.synchronize()
    assert np.array_equal(outs[2].cpu().numpy(), solo.cpu().numpy())
    assert rep["objective"] == rep_solo["objective"]


def test_group_runs_batched_and_cancel_in_group(torch_cuda, orc):
    """Small MAP fits waiting together run as one batched group: with one
    stream, all four are running after the first step and each equals its fit
    alone bit for bit; a member cancelled while running finishes with its
    group as cancelled, the others are unaffected."""
    torch = torch_cuda
    reqs = []
    for dims, seed in (((40, 33, 12), 11), ((24, 20, 30), 12), ((31, 31, 9), 13), ((30, 25, 20), 14)):
        c = synth.make_case("map_brain", dims=dims, seed=seed)  # sizes within 2x of each other
        c["b1"] = f32(c["b1"])
        x = observations(orc, c)
        reqs.append({"case": c, "opts": dict(c["opts"], n_outer=3, n_gn=3, n_cg=12), "X": cuda(x),
                     "b1": cuda(c["b1"].astype(np.float32)), "N": x.shape[1]})
    solo = []
    for r in reqs:
        m = torch.zeros((4, r["N"]), dtype=torch.float32, device="cuda")
        rep, _ = _lib.mpm_fit(r["case"]["proto"], r["case"]["dims"], r["X"], r["b1"], r["opts"], m)
        solo.append((m.cpu().numpy(), rep))
    with _lib.MpmServer(hbm_budget=64 << 30, max_active=1) as srv:
        outs = [torch.zeros((4, r["N"]), dtype=torch.float32, device="cuda") for r in reqs]
        tickets = [srv.submit(r["case"]["proto"], r["case"]["dims"], r["X"], r["b1"], r["opts"], o)
                   for r, o in zip(reqs, outs)]
        assert srv.step() == 4
        srv.cancel(tickets[3])  # running in the group: with one stream, only as a member of it
        assert srv.poll(tickets[3]) is None
        srv.cancel(tickets[1])  # running in the group
        assert srv.poll(tickets[1]) is None  # finishes with its group
        live = [t for i, t in enumerate(tickets) if i not in (1, 3)]
        reports = _drive(srv, live)
        for i in (1, 3):
            with pytest.raises(_lib.MpmError) as ei:
                srv.poll(tickets[i])
            assert ei.value.status == 7
    torch.cuda.synchronize()
    for i, ((ref, rep_a), o, t) in enumerate(zip(solo, outs, tickets)):
        if i in (1, 3):
            continue
        assert np.array_equal(o.cpu().numpy(), ref), i
        assert reports[t] == rep_a
