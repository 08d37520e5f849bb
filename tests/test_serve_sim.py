"""The serving scheduler on the host (lsb_serve_simulate): the same C++ loop
as lsb_serve, with modelled launches on a virtual clock and no GPU.  Checks
admission order, the HBM budget, eviction, extract targeting, continuous
batching and rejection of requests that can never fit."""
import numpy as np
import pytest

import oracle
from paper_0912_0947_amd import serve
from paper_0912_0947_amd._lib import E_CAPACITY, E_NOMEM, OK, OP_EMBED, OP_EXTRACT
from paper_0912_0947_amd.workloads import BatchWorkload


@pytest.fixture(scope="module")
def wl():
    return BatchWorkload(256, oracle.capacity, seed=2101, lo=64, hi=2048)


def _check_common(req, res, budget, stats):
    n = len(req)
    served = res["status"] == OK
    # every request finished
    assert np.all((res["status"] == OK) | (res["status"] == E_NOMEM))
    # time order per request
    ok = np.nonzero(served)[0]
    assert np.all(res["admit_s"][ok] + 1e-12 >= req["arrival_s"][ok])
    assert np.all(res["launch_s"][ok] >= res["admit_s"][ok])
    assert np.all(res["done_s"][ok] >= res["launch_s"][ok])
    # admission in arrival order
    assert np.all(np.diff(res["admit_s"][ok]) >= 0)
    # extracts read an embed that had finished, each stego at most once
    ext = np.nonzero(served & (res["op_run"] == OP_EXTRACT))[0]
    targets = res["target"][ext]
    assert len(set(targets.tolist())) == len(targets)
    for i in ext:
        t = int(res[i]["target"])
        assert 0 <= t < i and res[t]["op_run"] == OP_EMBED and res[t]["status"] == OK
        assert res[t]["done_s"] <= res[i]["admit_s"] + 1e-12
        assert res[i]["len"] == res[t]["len"] == req[t]["len"]
    assert stats["peak_arena_bytes"] <= budget
    assert stats["launches"] >= 1
    assert 1 <= stats["mean_batch"]
    return ok


def test_large_budget_no_evictions(wl):
    req, _ = serve.poisson_requests(wl, 10000.0, 3000, seed=2111)
    budget = 64 << 30
    res, stats = serve.simulate(req, budget, max_batch=64, n_slots=4)
    ok = _check_common(req, res, budget, stats)
    assert ok.size == len(req) and stats["evictions"] == 0 and stats["rejected"] == 0
    assert stats["p99_ms"] >= stats["p50_ms"] > 0


def test_continuous_batching_grows_with_load(wl):
    """At low load each launch carries one request; at high load requests
    that arrive while others run join the next launch."""
    low, _ = serve.poisson_requests(wl, 500.0, 1000, seed=2121)
    high, _ = serve.poisson_requests(wl, 200000.0, 1000, seed=2122)
    _, s_low = serve.simulate(low, 64 << 30, max_batch=256, n_slots=1, launch_us=50.0, device_gbps=2000.0)
    _, s_high = serve.simulate(high, 64 << 30, max_batch=256, n_slots=1, launch_us=50.0, device_gbps=2000.0)
    assert s_low["mean_batch"] < 1.2
    # one slot busy ~50 us per launch while 200k req/s arrive: ~10 per launch
    assert s_high["mean_batch"] > 5 * s_low["mean_batch"]
    assert s_high["p50_ms"] > s_low["p50_ms"]


def test_tight_budget_evicts_oldest_and_stays_within(wl):
    req, _ = serve.poisson_requests(wl, 50000.0, 2000, seed=2131, extract_frac=0.3)
    budget = int(np.sort(wl.n)[-6:].sum()) + (1 << 20)
    res, stats = serve.simulate(req, budget, max_batch=32, n_slots=4)
    ok = _check_common(req, res, budget, stats)
    assert ok.size == len(req)
    assert stats["evictions"] > 0
    # an evicted stego is gone (its offset released); one read by an extract
    # was released after that extract finished
    assert np.all(res["out_off"][res["op_run"] == OP_EXTRACT] == serve.FREED)


def test_never_fitting_request_is_rejected_alone(wl):
    req, _ = serve.poisson_requests(wl, 5000.0, 200, seed=2141, extract_frac=0.0)
    big = int(np.argmax(req["n"]))
    others = np.delete(np.arange(len(req)), big)
    budget = int(req["n"][others].max()) + (1 << 16)
    if budget >= req["n"][big]:
        pytest.skip("largest request is not unique")
    res, stats = serve.simulate(req, budget, max_batch=8, n_slots=2)
    assert res[big]["status"] == E_NOMEM
    assert np.all(res["status"][others] == OK)
    assert stats["rejected"] == 1


def test_oversize_message_fails_alone(wl):
    """Embed requests whose message exceeds their cover's capacity complete at
    admission with LSB_E_CAPACITY; every other request is served as it would
    be without them, and extracts never target a failed embed."""
    req, _ = serve.poisson_requests(wl, 20000.0, 600, seed=2161, extract_frac=0.3)
    emb = np.nonzero(req["op"] == OP_EMBED)[0]
    bad = emb[[3, 40, 41, 200]]
    for i in bad:
        req[i]["len"] = oracle.capacity(int(req[i]["n"]), int(req[i]["k"])) + 1
    res, stats = serve.simulate(req, 64 << 30, max_batch=16, n_slots=3)
    assert np.all(res["status"][bad] == E_CAPACITY)
    assert np.all(res["op_run"][bad] == OP_EMBED)
    assert np.all(res["out_off"][bad] == serve.FREED)
    good = np.setdiff1d(np.arange(len(req)), bad)
    assert np.all(res["status"][good] == OK)
    assert stats["rejected"] == len(bad)
    ext = good[res["op_run"][good] == OP_EXTRACT]
    assert not set(res["target"][ext].tolist()) & set(bad.tolist())


def test_keep_outputs_never_frees(wl):
    req, _ = serve.poisson_requests(wl, 20000.0, 400, seed=2151)
    res, stats = serve.simulate(req, 64 << 30, max_batch=16, n_slots=3, keep_outputs=True)
    assert np.all(res["status"] == OK)
    assert np.all(res["out_off"] != serve.FREED)
    offs = res["out_off"].astype(np.int64)
    sizes = np.where(res["op_run"] == OP_EMBED, req["n"], res["len"]).astype(np.int64)
    order = np.argsort(offs)
    ends = offs[order] + sizes[order]
    assert np.all(ends[:-1] <= offs[order][1:]), "two kept outputs overlap in the arena"


def test_deterministic(wl):
    req, _ = serve.poisson_requests(wl, 30000.0, 800, seed=2161)
    a, sa = serve.simulate(req, 1 << 30, max_batch=32, n_slots=3)
    b, sb = serve.simulate(req, 1 << 30, max_batch=32, n_slots=3)
    assert np.array_equal(a, b) and sa == sb


def test_explicit_targets_and_fallback_to_embed(wl):
    """An extract naming an embed that is resident reads it; one naming a
    request whose stego is not resident (never embedded) is served as an
    embed."""
    req, _ = serve.poisson_requests(wl, 1000.0, 6, seed=2171, extract_frac=0.0)
    req["arrival_s"] = [0.0, 0.001, 0.002, 0.003, 0.004, 0.005]
    req["op"][3] = OP_EXTRACT
    req["target"][3] = 1
    req["op"][4] = OP_EXTRACT
    req["target"][4] = 3  # request 3 is an extract: nothing resident to read
    res, stats = serve.simulate(req, 64 << 30, max_batch=4, n_slots=1)
    assert res[3]["op_run"] == OP_EXTRACT and res[3]["target"] == 1
    assert res[4]["op_run"] == OP_EMBED and res[4]["target"] == -1


def test_argument_errors(wl):
    req, _ = serve.poisson_requests(wl, 1000.0, 10, seed=2181)
    bad = req.copy()
    bad["arrival_s"][5] = 0.0  # unsorted
    with pytest.raises(Exception):
        serve.simulate(bad, 1 << 30)
    bad = req.copy()
    bad["target"][3] = 7  # points forward
    with pytest.raises(Exception):
        serve.simulate(bad, 1 << 30)
    with pytest.raises(Exception):
        serve.simulate(req, 1 << 30, max_batch=0)


def test_returned_claim_keeps_its_age():
    """An extract that claims a resident stego but cannot get memory for its
    message gives the claim back at the stego's place in the oldest-first
    order: a later untargeted extract still reads the oldest stego."""
    req = np.zeros(4, dtype=serve.REQ_DTYPE)
    req["arrival_s"] = [0.0, 1e-6, 1.0, 1.0 + 1e-6]
    req["n"] = 4096
    req["k"] = [1, 8, 1, 1]
    req["len"] = [100, 4000, 0, 0]
    req["op"] = [OP_EMBED, OP_EMBED, OP_EXTRACT, OP_EXTRACT]
    req["target"] = [-1, -1, 1, -1]
    # 512 B of per-slot status arrays, both stegos, and a 512 B hole: the
    # 4000-byte message of request 1 can never fit, request 0's 100 bytes can
    budget = 512 + 2 * 4096 + 512
    res, stats = serve.simulate(req, budget, max_batch=1, n_slots=1, keep_outputs=True)
    assert res[0]["status"] == OK and res[1]["status"] == OK
    assert res[2]["status"] == E_NOMEM
    assert res[3]["status"] == OK and res[3]["op_run"] == OP_EXTRACT
    assert res[3]["target"] == 0 and res[3]["len"] == 100
    assert stats["rejected"] == 1


def test_concurrent_simulations_match_serial(wl):
    """The scheduler keeps no shared state: four host threads simulating at
    once get the serial results, and a failing call on one thread leaves
    its error message on that thread only."""
    import threading

    from paper_0912_0947_amd._lib import lib

    reqs = [serve.poisson_requests(wl, 20000.0, 1500, seed=2190 + t)[0] for t in range(4)]
    serial = [serve.simulate(r, 1 << 30, max_batch=16, n_slots=3) for r in reqs]
    got, errors = [None] * 4, []

    def run(t):
        try:
            for _ in range(3):
                got[t] = serve.simulate(reqs[t], 1 << 30, max_batch=16, n_slots=3)
                if t == 0:
                    with pytest.raises(Exception):
                        serve.simulate(reqs[t], 1 << 30, max_batch=0)
                    assert b"max_batch" in lib().lsb_last_error()
                else:
                    assert lib().lsb_last_error() == b""
        except BaseException as e:
            errors.append((t, repr(e)))

    ts = [threading.Thread(target=run, args=(t,)) for t in range(4)]
    for th in ts:
        th.start()
    for th in ts:
        th.join(timeout=120)
    assert not errors, errors
    for (a, sa), (b, sb) in zip(serial, got):
        assert np.array_equal(a, b) and sa == sb
