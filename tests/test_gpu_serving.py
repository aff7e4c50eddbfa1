"""Serving: continuous batching over several resident materials (FP16 and FP32), admission by
memory budget, and every result bitwise equal to the same request decoded alone."""
import time

import numpy as np
import pytest

from paper_2305_02678_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def nam(torch):
    from paper_2305_02678_amd import nam as n
    n.lib()
    return n


@pytest.fixture(scope="module")
def ctx(nam):
    return nam.Context(0)


@pytest.fixture(scope="module")
def materials(nam, ctx):
    mats = wl.serving_materials(seed=77, count=4, sides=(64, 128, 256))
    out = []
    for i, m in enumerate(mats):
        mm = nam.Material.from_workload(ctx, m)
        if i % 2 == 0:
            mm.set_precision(nam.F16)
        out.append(mm)
    return mats, out


def _requests(torch, nam, mats, count, seed, lo=100, hi=300000):
    reqs = wl.request_stream(seed, mats, count, rate_per_s=1e4, lo=lo, hi=hi)
    dev = []
    for r in reqs:
        dq = nam.to_device(r.queries)
        dev.append((r, dq, torch.full((len(r.queries), 3), -1.0, device="cuda")))
    return dev


def test_results_in_the_mix_equal_alone(nam, ctx, torch, materials):
    mats, handles = materials
    srv = nam.Server(ctx, budget_bytes=64 << 20, n_streams=4, max_tile=65536)
    ids = [srv.add_material(h) for h in handles]
    reqs = _requests(torch, nam, mats, 40, seed=3)
    tickets = [srv.submit(ids[r.material], *dq, out) for r, dq, out in reqs]
    srv.wait_all()
    for (r, dq, out), tk in zip(reqs, tickets):
        done, lat = srv.poll(tk)
        assert done and lat >= 0.0
        alone = nam.decode(handles[r.material], *dq)
        torch.cuda.synchronize()
        assert torch.equal(out, alone), (r.material, len(r.queries))
    st = srv.stats()
    assert st["completed"] == 40 and st["p50_s"] <= st["p99_s"] <= st["max_s"]
    assert 0 < st["peak_reserved_bytes"] <= 64 << 20
    srv.close()


def test_host_buffers_are_staged_through_the_budget(nam, ctx, torch, materials):
    mats, handles = materials
    srv = nam.Server(ctx, budget_bytes=48 * 20000, n_streams=3, max_tile=20000)   # forces waits
    ids = [srv.add_material(h) for h in handles]
    reqs = wl.request_stream(5, mats, 12, rate_per_s=1e4, lo=1000, hi=90000)
    host = []
    for r in reqs:
        arrs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).pin_memory()
                for a in (r.queries.uv, r.queries.lod, r.queries.wi, r.queries.wo)]
        out = torch.empty((len(r.queries), 3), dtype=torch.float32).pin_memory()
        host.append((r, arrs, out))
    for r, arrs, out in host:
        srv.submit(ids[r.material], *arrs, out)
    srv.wait_all()
    for r, arrs, out in host:
        alone = nam.decode(handles[r.material], *nam.to_device(r.queries)).cpu()
        assert torch.equal(out, alone)
    assert srv.stats()["peak_reserved_bytes"] <= 48 * 20000
    srv.close()


def test_replayed_arrivals_overlap_and_latency(nam, ctx, torch, materials):
    """Requests arriving while others run are admitted as streams free up; latency counts from
    the replayed arrival time."""
    mats, handles = materials
    srv = nam.Server(ctx, budget_bytes=256 << 20, n_streams=4, max_tile=1 << 18)
    ids = [srv.add_material(h) for h in handles]
    reqs = _requests(torch, nam, mats, 60, seed=9)
    srv.reset_stats()                   # replayed arrival times count from here
    t = 0.0
    tickets = []
    for r, dq, out in reqs:
        t += 0.0005
        tickets.append(srv.submit(ids[r.material], *dq, out, arrival_s=t))
    srv.wait_all()
    lats = [srv.poll(tk)[1] for tk in tickets]
    assert min(lats) >= 0.0
    st = srv.stats()
    print(f"replayed arrivals: {st['completed']} requests, at most {st['peak_requests_on_device']} requests and "
          f"{st['peak_launches_on_device']} launches on the device at once, p50 {st['p50_s'] * 1e3:.3f} ms, "
          f"p99 {st['p99_s'] * 1e3:.3f} ms", flush=True)
    assert st["completed"] == 60 and st["span_s"] >= 0.03 - 1e-3
    for (r, dq, out) in reqs[:10]:
        assert torch.equal(out, nam.decode(handles[r.material], *dq))
    srv.close()


def test_burst_of_arrivals_overlaps_on_the_device(nam, ctx, torch, materials):
    """Continuous batching, from the server's own counters: 60 replayed arrivals 5 us apart
    (requests of 100 to 300,000 queries over 4 resident materials) are admitted while earlier
    ones are still on the device, so several requests and several launches are in flight at
    once, and each result is still the one nam_decode gives alone."""
    mats, handles = materials
    srv = nam.Server(ctx, budget_bytes=256 << 20, n_streams=4, max_tile=1 << 18)
    ids = [srv.add_material(h) for h in handles]
    reqs = _requests(torch, nam, mats, 60, seed=11)
    srv.reset_stats()                   # replayed arrival times count from here
    tickets = [srv.submit(ids[r.material], *dq, out, arrival_s=0.002 + 5e-6 * k)
               for k, (r, dq, out) in enumerate(reqs)]
    srv.wait_all()
    st = srv.stats()
    print(f"burst: {st['completed']} requests in {st['launches']} launches ({st['tiles']} tiles); at most "
          f"{st['peak_requests_on_device']} requests and {st['peak_launches_on_device']} launches on the device "
          f"at once; p50 {st['p50_s'] * 1e3:.3f} ms, p99 {st['p99_s'] * 1e3:.3f} ms", flush=True)
    assert st["completed"] == 60 and st["p99_s"] < 0.1
    assert st["peak_requests_on_device"] >= 2
    assert st["peak_launches_on_device"] >= 2
    assert all(srv.poll(tk)[0] for tk in tickets)
    for (r, dq, out) in reqs:
        assert torch.equal(out, nam.decode(handles[r.material], *dq))
    srv.close()


def test_cancel_queued_request(nam, ctx, torch, materials):
    mats, handles = materials
    srv = nam.Server(ctx, budget_bytes=64 << 20, n_streams=1, max_tile=65536)
    mid = srv.add_material(handles[0])
    q = wl.uniform_queries(np.random.default_rng(0), 5000, 0, 3)
    dq = nam.to_device(q)
    out = torch.full((5000, 3), -7.0, device="cuda")
    tk = srv.submit(mid, *dq, out, arrival_s=30.0)    # far in the future: still queued
    srv.cancel(tk)
    with pytest.raises(nam.NamError):
        srv.poll(tk)
    srv.wait_all()
    assert bool((out == -7.0).all())
    srv.close()


def test_budget_and_argument_errors(nam, ctx, torch, materials):
    mats, handles = materials
    with pytest.raises(nam.NamError) as e:
        nam.Server(ctx, budget_bytes=1000, n_streams=2, max_tile=65536)
    assert e.value.status == nam.NAM_E_BUDGET
    srv = nam.Server(ctx, budget_bytes=64 << 20, n_streams=2, max_tile=65536)
    mid = srv.add_material(handles[1])
    with pytest.raises(nam.NamError) as e:
        handles[1].set_precision(nam.F16)             # held by the server
    assert e.value.status == nam.NAM_E_BUSY
    with pytest.raises(nam.NamError) as e:
        handles[1].free()
    assert e.value.status == nam.NAM_E_BUSY
    L = nam.lib()
    import ctypes
    tk = ctypes.c_uint64(0)
    assert L.nam_server_submit(srv.handle, 99, 10, None, None, None, None, None, 0, -1.0, ctypes.byref(tk)) == nam.NAM_E_INVALID_ARG
    assert L.nam_server_submit(srv.handle, mid, -1, None, None, None, None, None, 0, -1.0, ctypes.byref(tk)) == nam.NAM_E_INVALID_ARG
    srv.close()
    handles[1].set_precision(nam.F32)                  # released by the server


def test_grouped_launch_over_materials(nam, ctx, torch):
    """Tiles of several materials that share a matrix-core kernel go out as grouped launches
    (fewer launches than tiles), and every result is still bitwise the one decoded alone; with
    grouping off every tile is its own launch."""
    mats = [wl.make_material(*wl.rngs(300 + i)[:2], 128 >> (i % 2), 128 >> (i % 2), 16, 6, [64] * 3,
                             n_frames=2 if i >= 4 else 0) for i in range(6)]
    handles = []
    for m in mats:
        h = nam.Material.from_workload(ctx, m)
        h.set_precision(nam.F16)
        handles.append(h)
    rng = np.random.default_rng(9)
    reqs = []
    for k in range(40):
        mid = int(rng.integers(0, 6))
        q = wl.uniform_queries(rng, int(rng.integers(100, 40000)), 0, 6)
        dq = nam.to_device(q)
        reqs.append((mid, dq, torch.full((len(q), 3), -1.0, device="cuda")))
    for group in (8, 1):
        srv = nam.Server(ctx, budget_bytes=64 << 20, n_streams=2, max_tile=16384)
        srv.set_group(group)
        ids = [srv.add_material(h) for h in handles]
        for _, _, out in reqs:
            out.fill_(-1.0)
        torch.cuda.synchronize()
        for mid, dq, out in reqs:
            srv.submit(ids[mid], *dq, out)
        srv.wait_all()
        st = srv.stats()
        for mid, dq, out in reqs:
            assert torch.equal(out, nam.decode(handles[mid], *dq)), (group, mid)
        print(f"group {group}: {st['tiles']} tiles in {st['launches']} launches", flush=True)
        assert st["completed"] == len(reqs)
        if group == 1:
            assert st["launches"] == st["tiles"]
        else:
            assert st["launches"] < st["tiles"]
        srv.close()
    with pytest.raises(nam.NamError, match="NAM_E_INVALID_ARG"):
        nam.Server(ctx, budget_bytes=64 << 20, n_streams=2, max_tile=16384).set_group(9)
