"""Continuous batching (bos_sort_step) and the serving loop on the GPU.

Every request served in a mix must come out byte-identical to the same request
sorted alone (bos_sort) and to the oracle's sort, with the same number of
routing attempts; admission must keep the resident footprint under the budget.
"""
import numpy as np
import pytest

import closed_forms as cf
from gpu_util import record_checksum
from paper_2008_01765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_01765_amd import bos, serving  # noqa: E402


def _hosts(sizes, rec, data_seed):
    return [inputs.records(int(n), rec, data_seed + i, key_bits=(20 if rec == 16 else None))
            for i, n in enumerate(sizes)]


@pytest.mark.parametrize("rec,z,pipeline", [(16, 512, True), (8, 512, True), (16, 256, True), (16, 512, False)])
def test_mix_equals_alone(rec, z, pipeline):
    sizes = [4096, 1 << 16, 0, 1, 5000, 70000, 1 << 12, 333, 1 << 18, 9999]
    hosts = _hosts(sizes, rec, 300)
    srv = serving.Server(hbm_budget_bytes=1 << 34, z=z, min_security_bits=0, pipeline=pipeline)
    futs = []
    ts = [bos.from_numpy(h) for h in hosts]
    # requests join while others are mid-flight
    for i, t in enumerate(ts):
        futs.append(srv.submit(t, seed=50 + i))
        if i % 3 == 2:
            srv.step()
    srv.run_until_idle()
    for h, t, f in zip(hosts, ts, futs):
        got = bos.to_numpy(f.result())
        np.testing.assert_array_equal(got, cf.sorted_records(h))
        if len(h):
            alone, rep = bos.sort(t, seed=f.seed, z=z, min_security_bits=0, report=True)
            np.testing.assert_array_equal(got, bos.to_numpy(alone))
            assert f.attempts + 1 == rep["attempts"]
    assert srv.used == 0


@pytest.mark.parametrize("rec,tile,pipeline", [(8, 1024, True), (16, 2048, False), (16, 1024, True)])
def test_mix_four_way_merge_phases(rec, tile, pipeline):
    # Jobs whose merge phases are four-way passes from the start, two-way then
    # four-way, or two-way only, admitted while others run: each equals the
    # request sorted alone.
    sizes = [1 << 18, 300000, 5000, 70001, 4 * tile + 3, 1 << 16, 2 * tile + 1, 1]
    hosts = _hosts(sizes, rec, 520)
    srv = serving.Server(hbm_budget_bytes=1 << 34, z=512, tile=tile, pipeline=pipeline)
    ts = [bos.from_numpy(h) for h in hosts]
    futs = []
    for i, t in enumerate(ts):
        futs.append(srv.submit(t, seed=90 + i))
        if i % 2 == 1:
            srv.step()
    srv.run_until_idle()
    for h, t, f in zip(hosts, ts, futs):
        assert f.status == bos.OK
        got = bos.to_numpy(f.result())
        np.testing.assert_array_equal(got, cf.sorted_records(h))
        alone = bos.to_numpy(bos.sort(t, seed=f.seed, z=512, tile=tile))
        np.testing.assert_array_equal(got, alone)
    assert srv.used == 0


@pytest.mark.parametrize("pipeline", [True, False])
def test_side_stream_server(pipeline):
    # The server runs on a stream of its own: inputs produced on the caller's
    # stream just before submission, outputs read on the caller's stream
    # right after result(), buffers of finished requests released while
    # later ones still run.  Every result equals the sort alone.
    side = torch.cuda.Stream()
    sizes = [1 << 16, 4096, 70000, 1 << 18, 333, 9999, 1 << 12, 5000] * 2
    hosts = _hosts(sizes, 16, 1300)
    srv = serving.Server(hbm_budget_bytes=1 << 34, z=512, min_security_bits=0, pipeline=pipeline, stream=side)
    futs, srcs = [], []
    for i, h in enumerate(hosts):
        staged = bos.from_numpy(h)
        t = staged.clone()  # written on the caller's stream, read on the server's
        srcs.append(t)
        futs.append(srv.submit(t, seed=70 + i))
        if i % 4 == 3:
            srv.step()
    outs = [f.result() for f in futs]
    srv.run_until_idle()
    for h, o in zip(hosts, outs):
        chk = o.clone()  # read on the caller's stream after result()
        np.testing.assert_array_equal(bos.to_numpy(chk), cf.sorted_records(h))
    assert srv.used == 0


def test_budget_bounds_resident_footprint():
    sizes = [1 << 16] * 6 + [1 << 14] * 4
    hosts = _hosts(sizes, 16, 900)
    probe = serving.Server(hbm_budget_bytes=1 << 40, min_security_bits=0)
    one = probe.footprint(1 << 16, 16)
    srv = serving.Server(hbm_budget_bytes=2 * one + one // 2, min_security_bits=0)
    futs = [srv.submit(bos.from_numpy(h), seed=i) for i, h in enumerate(hosts)]
    while not srv.idle():
        srv.step()
        assert srv.used <= srv.budget
        assert sum(f.footprint for f in srv.active) == srv.used
    assert srv.peak_used <= srv.budget
    assert srv.completed == len(futs)
    # first come, first served: admission times follow submission order
    adm = [f.admitted for f in futs]
    assert adm == sorted(adm)
    for h, f in zip(hosts, futs):
        np.testing.assert_array_equal(bos.to_numpy(f.out), cf.sorted_records(h))


@pytest.mark.parametrize("pipeline", [True, False])
def test_overflow_retries_in_mix_match_alone(pipeline):
    # Z = 32 overflows often at these sizes; a job that overflows retries from
    # pass 0 with the next attempt, as bos_sort does.  The oracle fixes the
    # attempt count of every job.
    import oracle
    oracle.build(force=False)
    sizes = [1 << 14, 9000, 1 << 13, 6000, 20000]
    hosts = _hosts(sizes, 8, 5)
    seeds = [11, 12, 13, 14, 15]
    srv = serving.Server(hbm_budget_bytes=1 << 34, z=32, min_security_bits=0, max_retries=30, pipeline=pipeline)
    futs = [srv.submit(bos.from_numpy(h), seed=s) for h, s in zip(hosts, seeds)]
    srv.run_until_idle()
    retried = 0
    for h, f, s in zip(hosts, futs, seeds):
        want = oracle.sort(h, s, z=32, max_retries=30)
        assert want["rc"] == 0 and f.status == bos.OK
        assert f.attempts + 1 == want["report"]["attempts"]
        retried += f.attempts > 0
        np.testing.assert_array_equal(bos.to_numpy(f.out), want["out"])
    assert retried > 0


def test_trace_replay_and_sequential_agree():
    sizes = inputs.request_sizes(12, lo_log2=10, hi_log2=16, seed=3)
    hosts = _hosts(sizes, 16, 77)
    ts = [bos.from_numpy(h) for h in hosts]
    arr = serving.poisson_arrivals(len(ts), rate_per_s=2000.0, seed=5)
    srv = serving.Server(hbm_budget_bytes=1 << 34, min_security_bits=0)
    futs = serving.run_trace(srv, ts, arr)
    lat, outs = serving.run_trace_sequential(ts, arr)
    assert len(lat) == len(futs) == len(ts)
    for h, f, o in zip(hosts, futs, outs):
        np.testing.assert_array_equal(bos.to_numpy(f.out), cf.sorted_records(h))
        np.testing.assert_array_equal(bos.to_numpy(o), cf.sorted_records(h))
        assert f.latency >= 0


def test_step_rejects_small_workspace():
    t = bos.from_numpy(inputs.records(5000, 16, 1))
    out = torch.empty_like(t)
    p = bos.params(0, 512, 0, 0, 3, 0)
    ws = torch.empty(bos.workspace_bytes(5000, 16, p), dtype=torch.uint8, device="cuda")
    jobs = (bos.Job * 1)()
    jobs[0].in_, jobs[0].out, jobs[0].n, jobs[0].seed = t.data_ptr(), out.data_ptr(), 5000, 1
    jobs[0].ws, jobs[0].ws_bytes = ws.data_ptr(), ws.numel() - 256
    sws = torch.empty(bos.step_workspace_bytes(1), dtype=torch.uint8, device="cuda")
    with pytest.raises(bos.BosError) as e:
        bos.sort_step(jobs, 16, p, sws)
    assert e.value.status == bos.WORKSPACE
    jobs[0].ws_bytes = ws.numel()
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(bos.BosError) as e:
        bos.sort_step(jobs, 16, p, small)
    assert e.value.status == bos.WORKSPACE
    while bos.sort_step(jobs, 16, p, sws):
        pass
    np.testing.assert_array_equal(bos.to_numpy(out), cf.sorted_records(bos.to_numpy(t)))


def test_request_over_budget_rejected():
    srv = serving.Server(hbm_budget_bytes=1 << 20, min_security_bits=0)
    with pytest.raises(bos.BosError):
        srv.submit(bos.from_numpy(inputs.records(1 << 16, 16, 1)))


def test_server_freed_without_cycle_collector():
    # futures refer to their server weakly: dropping the server frees it and
    # its workspaces at once, while the futures keep their outputs
    import gc
    import weakref

    hosts = _hosts([3000, 70000], 16, 41)
    gc.disable()
    try:
        srv = serving.Server(hbm_budget_bytes=1 << 34, min_security_bits=0)
        futs = [srv.submit(bos.from_numpy(h), seed=i) for i, h in enumerate(hosts)]
        srv.run_until_idle()
        assert srv.completed == 2
        ref = weakref.ref(srv)
        del srv
        assert ref() is None
    finally:
        gc.enable()
    for h, f in zip(hosts, futs):
        np.testing.assert_array_equal(bos.to_numpy(f.out), cf.sorted_records(h))


def _job(t, out, ws, seed):
    j = bos.Job()
    j.in_, j.out, j.n, j.seed = t.data_ptr(), out.data_ptr(), t.shape[0], seed
    j.ws, j.ws_bytes = ws.data_ptr(), ws.numel()
    return j


def test_stepper_jobs_matched_by_workspace():
    # the pipelined engine finds its jobs by workspace: the array is reversed
    # after every call, a job joins mid-way and finished jobs leave; outputs
    # and attempt counts equal bos_sort's (Z = 32 so that some attempts
    # overflow and roll back)
    import oracle
    oracle.build(force=False)
    sizes = [1 << 14, 9000, 1 << 13, 6000, 20000]
    hosts = _hosts(sizes, 8, 5)
    p = bos.params(0, 32, 0, 0, 30, 0)
    ts = [bos.from_numpy(h) for h in hosts]
    outs = [torch.empty_like(t) for t in ts]
    wss = [torch.empty(bos.workspace_bytes(t.shape[0], 8, p), dtype=torch.uint8, device="cuda") for t in ts]
    jobs = [_job(t, o, w, 11 + i) for i, (t, o, w) in enumerate(zip(ts, outs, wss))]
    late = jobs.pop()  # joins after two calls
    st = bos.Stepper()
    sws = torch.empty(2 * bos.step_workspace_bytes(len(sizes)), dtype=torch.uint8, device="cuda")
    done = {}
    calls = 0
    while jobs or late is not None:
        arr = (bos.Job * len(jobs))(*jobs)
        st.step(arr, 8, p, sws)
        calls += 1
        jobs = []
        for j in arr:
            if j.phase == bos.PHASE_DONE:
                done[j.ws] = (j.status, j.attempt)
            else:
                jobs.append(j)
        jobs.reverse()
        if calls == 2 and late is not None:
            jobs.append(late)
            late = None
        assert calls < 10000
    st.close()
    retried = 0
    for i, (h, w) in enumerate(zip(hosts, wss)):
        want = oracle.sort(h, 11 + i, z=32, max_retries=30)
        status, attempt = done[w.data_ptr()]
        assert status == bos.OK and attempt + 1 == want["report"]["attempts"]
        retried += attempt > 0
        np.testing.assert_array_equal(bos.to_numpy(outs[i]), want["out"])
    assert retried > 0


def test_stepper_rejects_null_and_small_workspace():
    t = bos.from_numpy(inputs.records(5000, 16, 1))
    out = torch.empty_like(t)
    p = bos.params(0, 512, 0, 0, 3, 0)
    ws = torch.empty(bos.workspace_bytes(5000, 16, p), dtype=torch.uint8, device="cuda")
    arr = (bos.Job * 1)(_job(t, out, ws, 1))
    one = bos.step_workspace_bytes(1)
    rc = bos.lib().bos_sort_step_async(None, arr, 1, 16, bos.C.byref(p), bos.C.c_void_p(ws.data_ptr()), one, None)
    assert rc == bos.INVALID_ARG
    st = bos.Stepper()
    small = torch.empty(one, dtype=torch.uint8, device="cuda")  # one half is too small
    with pytest.raises(bos.BosError) as e:
        st.step(arr, 16, p, small)
    assert e.value.status == bos.WORKSPACE
    sws = torch.empty(2 * one, dtype=torch.uint8, device="cuda")
    for _ in range(1000):
        st.step(arr, 16, p, sws)
        if arr[0].phase == bos.PHASE_DONE:
            break
    assert arr[0].status == bos.OK
    np.testing.assert_array_equal(bos.to_numpy(out), cf.sorted_records(bos.to_numpy(t)))
    st.close()


def test_serving_workload_shape():
    # Requests of the serving workload's shape (16-byte records, sizes
    # log-uniform in [2^12, 2^24], slices of one device array at pseudo-random
    # offsets) replayed with Poisson arrivals through the pipelined server:
    # every output is sorted and a permutation of its request, and 4 sampled
    # requests are compared whole with numpy's sort.
    sizes = inputs.request_sizes(64, 12, 24, seed=7)
    master_n = 1 << 25
    host = inputs.records(master_n, 16, 44)
    master = bos.from_numpy(host)
    starts = (inputs.splitmix64(99, 0, len(sizes)) % np.uint64(master_n - (1 << 24) + 1)).astype(np.int64)
    reqs = [master[int(s0):int(s0) + int(n)] for s0, n in zip(starts, sizes)]
    arr = serving.poisson_arrivals(len(reqs), rate_per_s=400.0, seed=11)
    srv = serving.Server(hbm_budget_bytes=64 << 30)
    futs = serving.run_trace(srv, reqs, arr)
    assert srv.idle() and srv.completed == len(reqs)
    for f in futs:
        assert f.status == bos.OK
        o = bos.to_numpy(f.out)
        k, p = o[:, 0], o[:, 1]
        assert bool(np.all((k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (p[1:] >= p[:-1]))))
        h = host[int(starts[f.id]):int(starts[f.id]) + f.n]
        assert record_checksum(o) == record_checksum(h)
    for i in np.random.default_rng(3).choice(len(reqs), 4, replace=False):
        h = host[int(starts[i]):int(starts[i]) + int(sizes[i])]
        np.testing.assert_array_equal(bos.to_numpy(futs[i].out), cf.sorted_records(h))
