"""lsb_batch_run_static, the allocation-free batched call: its results equal
those of a plan (lsb_plan_create + lsb_plan_run) on the same jobs, byte for
byte, on two calls in a row (the second with fewer jobs), and job counts
beyond its fixed table, or a stream that is capturing a graph, are refused
before anything runs."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_0947_amd import batch
from paper_0912_0947_amd._lib import E_ARG, E_CAPACITY, OK, OP_EMBED, OP_EXTRACT, OP_MIXED, LsbError
from paper_0912_0947_amd.workloads import BatchWorkload

from gpu_helpers import DEV

pytestmark = pytest.mark.gpu


def _plan_run(jobs, op, cover, stego, msg, lens, status):
    plan = batch.Plan(jobs.size, op, jobs)
    try:
        plan.run(cover, stego, msg, lens, status)
        torch.cuda.synchronize()
    finally:
        plan.close()


def test_static_equals_plan_on_two_calls():
    wl = BatchWorkload(600, oracle.capacity, seed=3101, lo=16, hi=700, ks=(1, 2, 3, 4, 8))
    cover, _, msg, _ = wl.allocate(DEV, pixel_seed=3102, msg_seed=3103)
    emb = wl.jobs(OP_EMBED)
    emb["len"][[5, 77, 300]] = wl.cap[[5, 77, 300]] + 1  # over capacity: status only, no work
    # call 1: every job an embed
    st_plan = torch.zeros_like(cover)
    st_static = torch.zeros_like(cover)
    s_plan = torch.full((wl.count,), 99, dtype=torch.int32, device=DEV)
    s_static = torch.full((wl.count,), 99, dtype=torch.int32, device=DEV)
    _plan_run(emb, OP_EMBED, cover, st_plan, msg, None, s_plan)
    batch.run_static(emb, OP_EMBED, cover, st_static, msg, None, s_static)
    torch.cuda.synchronize()
    assert torch.equal(s_static, s_plan)
    assert int((s_plan == E_CAPACITY).sum()) == 3 and int((s_plan == OK).sum()) == wl.count - 3
    assert torch.equal(st_static, st_plan), "static embed differs from the plan's"
    # call 2, fewer jobs: a mixed list of extracts (shuffled) and re-embeds
    g = np.random.default_rng(3104)
    pick = g.permutation(np.setdiff1d(np.arange(wl.count), [5, 77, 300]))[:250]
    mixed = wl.jobs(OP_EXTRACT)[pick]
    mixed["op"] = OP_EXTRACT
    re = g.choice(pick, size=40, replace=False)
    mixed["op"][np.isin(pick, re)] = OP_EMBED
    mixed["len"][np.isin(pick, re)] = wl.len[pick[np.isin(pick, re)]]
    out_plan, out_static = torch.zeros_like(msg), torch.zeros_like(msg)
    # extract jobs write msg_off of the message arena; embed jobs of the
    # mixed list read it: give each side the same message bytes
    out_plan.copy_(msg)
    out_static.copy_(msg)
    for j in np.nonzero(mixed["op"] == OP_EXTRACT)[0]:
        o, ln = int(mixed["msg_off"][j]), int(mixed["msg_cap"][j])
        out_plan[o:o + ln] = 0
        out_static[o:o + ln] = 0
    re_plan, re_static = st_plan.clone(), st_plan.clone()
    l_plan = torch.zeros(mixed.size, dtype=torch.int32, device=DEV)
    l_static = torch.full((mixed.size,), 7, dtype=torch.int32, device=DEV)
    s_plan = torch.full((mixed.size,), 99, dtype=torch.int32, device=DEV)
    s_static = torch.full((mixed.size,), 98, dtype=torch.int32, device=DEV)
    _plan_run(mixed, OP_MIXED, cover, re_plan, out_plan, l_plan, s_plan)
    batch.run_static(mixed, OP_MIXED, cover, re_static, out_static, l_static, s_static)
    torch.cuda.synchronize()
    assert bool((s_plan == OK).all())
    assert torch.equal(s_static, s_plan) and torch.equal(l_static, l_plan)
    assert torch.equal(out_static, out_plan), "static extract differs from the plan's"
    assert torch.equal(re_static, re_plan), "static re-embed differs from the plan's"
    # the extracted messages are the embedded ones
    for j in np.nonzero(mixed["op"] == OP_EXTRACT)[0]:
        o, ln = int(mixed["msg_off"][j]), int(mixed["msg_cap"][j])
        assert int(l_static[j]) == ln and torch.equal(out_static[o:o + ln], msg[o:o + ln])


def test_static_refuses_more_jobs_than_its_table():
    wl = BatchWorkload(batch.STATIC_MAX_JOBS + 1, oracle.capacity, seed=3111, lo=16, hi=24)
    cover, stego, msg, _ = wl.allocate(DEV)
    jobs = wl.jobs(OP_EMBED)
    status = torch.full((jobs.size,), 99, dtype=torch.int32, device=DEV)
    with pytest.raises(LsbError) as e:
        batch.run_static(jobs, OP_EMBED, cover, stego, msg, None, status)
    assert e.value.code == E_ARG
    torch.cuda.synchronize()
    assert bool((status == 99).all()), "a refused call ran"
    batch.run_static(jobs[:batch.STATIC_MAX_JOBS], OP_EMBED, cover, stego, msg, None, status)
    torch.cuda.synchronize()
    assert bool((status[:batch.STATIC_MAX_JOBS] == OK).all()) and int(status[-1]) == 99


def test_static_refuses_a_capturing_stream():
    """Under stream capture the table upload would be a graph node reading
    the library's shared staging buffer at replay time: the call is refused
    before anything is enqueued, and the same call outside capture runs."""
    wl = BatchWorkload(8, oracle.capacity, seed=3121, lo=16, hi=64)
    cover, stego, msg, _ = wl.allocate(DEV)
    jobs = wl.jobs(OP_EMBED)
    status = torch.full((jobs.size,), 99, dtype=torch.int32, device=DEV)
    mark = torch.zeros(1, dtype=torch.int32, device=DEV)
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        graph.capture_begin()
        try:
            mark.add_(1)  # the captured graph is not empty
            with pytest.raises(LsbError) as e:
                batch.run_static(jobs, OP_EMBED, cover, stego, msg, None, status, stream=side)
        finally:
            graph.capture_end()
    assert e.value.code == E_ARG and "capturing" in str(e.value)
    del graph
    torch.cuda.synchronize()
    assert bool((status == 99).all()) and int(mark) == 0, "nothing ran during the capture"
    batch.run_static(jobs, OP_EMBED, cover, stego, msg, None, status)
    torch.cuda.synchronize()
    assert bool((status == OK).all())
