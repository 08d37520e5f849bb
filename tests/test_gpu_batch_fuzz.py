"""Randomised batches (hypothesis, derandomised so every run draws the same
examples): one mixed plan holding header and raw-slice jobs, embeds and
extracts, any k, sizes from 1 byte up, messages that overflow, corrupt
headers and short output buffers.  Every job's status, length and output
bytes are compared with the oracle; bytes outside the outputs stay as they
were."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_0912_0947_amd import batch, inputs
from paper_0912_0947_amd._lib import OK, OP_EMBED, OP_EXTRACT

from gpu_helpers import DEV, to_host

pytestmark = pytest.mark.gpu

SENTINEL = 0xC3


@st.composite
def job_specs(draw):
    raw = draw(st.booleans())
    op = draw(st.sampled_from([OP_EMBED, OP_EXTRACT]))
    k = draw(st.integers(1, 8))
    n = draw(st.one_of(st.integers(1, 64), st.integers(65, 5000), st.integers(5001, 120_000)))
    spec = {"raw": raw, "op": op, "k": k, "n": n, "seed": draw(st.integers(0, 2**31 - 1))}
    if raw:
        t0 = draw(st.integers(0, 3 * n))
        if op == OP_EXTRACT:  # an extract slice starts on a stream byte
            while (k * t0) % 8:
                t0 += 1
        total_bits = k * (t0 + n)
        # the stream ends before, inside or after the slice; an extract slice
        # must end on a byte or at the stream's end
        choice = draw(st.sampled_from(["before", "inside", "after"]))
        if choice == "before":
            bits = draw(st.integers(0, max(0, k * t0)))
        elif choice == "inside":
            bits = draw(st.integers(k * t0, total_bits))
        else:
            bits = total_bits + draw(st.integers(0, 64))
        end = min(total_bits, bits)
        if op == OP_EXTRACT and end > k * t0 and end % 8 and end != bits:
            bits = total_bits  # let the stream end where the slice does
        spec.update(t0=t0, bits=bits)
    else:
        cap = oracle.capacity(n, k)
        if op == OP_EMBED:
            spec["len"] = draw(st.integers(0, cap + 1)) if cap >= 0 else draw(st.integers(0, 3))
        else:
            spec["flavour"] = draw(st.sampled_from(["ok", "corrupt", "short"]))
            spec["len"] = draw(st.integers(0, max(cap, 0)))
    return spec


def _prepare(spec):
    """Inputs and expectations of one job from the oracle."""
    g = inputs.rng(spec["seed"])
    n, k = spec["n"], spec["k"]
    cover = g.integers(0, 256, n, dtype=np.uint8)
    job = dict(spec, cover=cover)
    if spec["raw"]:
        t0, bits = spec["t0"], spec["bits"]
        stream = g.integers(0, 256, max((bits + 7) // 8, 1), dtype=np.uint8)
        if spec["op"] == OP_EMBED:
            rc, want = oracle.embed_raw(cover, t0, stream, bits, k)
            assert rc == OK
            job.update(msg=stream, want=want, status=OK, out_len=0)
        else:
            rc, stego = oracle.embed_raw(cover, t0, stream, bits, k)
            assert rc == OK
            rc, want = oracle.extract_raw(stego, t0, bits, k)
            assert rc == OK
            job.update(stego=stego, want=want, status=OK, out_len=0, msg_bytes=stream.size)
        return job
    cap = oracle.capacity(n, k)
    ln = spec["len"]
    if spec["op"] == OP_EMBED:
        msg = g.integers(0, 256, ln, dtype=np.uint8)
        rc, want = oracle.embed(cover, msg, k)
        job.update(msg=msg, want=want if rc == OK else None, status=rc if rc < 0 else OK, out_len=ln)
        return job
    msg = g.integers(0, 256, ln, dtype=np.uint8)
    stego = cover
    out_cap = max(ln, 1)
    if cap >= 0:
        rc, stego = oracle.embed(cover, msg, k)
        assert rc == OK
        if spec["flavour"] == "corrupt" and n * k >= 32:
            hdr = np.frombuffer(int(cap + 1).to_bytes(4, "big"), np.uint8)
            rc, stego = oracle.embed_raw(stego, 0, hdr, 32, k)
        elif spec["flavour"] == "short" and ln > 0:
            out_cap = ln - 1
    orc, oln, omsg = oracle.extract(stego, k, out_cap=out_cap)
    job.update(stego=stego, msg_cap=out_cap, status=orc, out_len=oln, want=omsg)
    return job


@settings(max_examples=60, deadline=None, derandomize=True, database=None, suppress_health_check=list(HealthCheck))
@given(st.lists(job_specs(), min_size=1, max_size=10))
def test_random_mixed_plans(specs):
    jobs = [_prepare(s) for s in specs]
    table = batch.make_jobs(len(jobs))
    off_c = off_m = 0
    layout = []
    for i, j in enumerate(jobs):
        t = table[i]
        t["cover_off"] = t["stego_off"] = off_c
        t["msg_off"] = off_m
        t["n"], t["k"], t["op"] = j["n"], j["k"], j["op"]
        if j["raw"]:
            t["flags"], t["t0"], t["stream_bits"] = batch.JOB_RAW, j["t0"], j["bits"]
            mbytes = j["msg"].size if j["op"] == OP_EMBED else j["msg_bytes"]
        elif j["op"] == OP_EMBED:
            t["len"] = j["len"]
            mbytes = j["len"]
        else:
            t["msg_cap"] = j["msg_cap"]
            mbytes = j["msg_cap"]
        layout.append((off_c, off_m, mbytes))
        off_c = batch.align_up(off_c + j["n"])
        off_m = batch.align_up(off_m + max(mbytes, 1) + 16)
    cover_h = np.zeros(max(off_c, 1), np.uint8)
    stego_h = np.full(max(off_c, 1), SENTINEL, np.uint8)
    msg_h = np.full(max(off_m, 1), SENTINEL, np.uint8)
    for j, (c0, m0, mb) in zip(jobs, layout):
        if j["op"] == OP_EMBED:
            cover_h[c0:c0 + j["n"]] = j["cover"]
            msg_h[m0:m0 + j["msg"].size] = j["msg"]
        else:
            stego_h[c0:c0 + j["n"]] = j["stego"]
    cover, stego, msg = (torch.from_numpy(a).to(DEV) for a in (cover_h, stego_h, msg_h))
    status = torch.full((len(jobs),), 99, dtype=torch.int32, device=DEV)
    lens = torch.full((len(jobs),), 7, dtype=torch.int32, device=DEV)
    plan = batch.Plan(len(jobs), batch.OP_MIXED, table)
    try:
        plan.run(cover, stego, msg, lens, status)
        torch.cuda.synchronize()
    finally:
        plan.close()
    st_h, ln_h = status.cpu().numpy(), lens.cpu().numpy().astype(np.uint32)
    stego_o, msg_o = to_host(stego), to_host(msg)
    for i, (j, (c0, m0, mb)) in enumerate(zip(jobs, layout)):
        tag = "job %d %s" % (i, {k: v for k, v in j.items() if k in ("raw", "op", "k", "n", "t0", "bits", "len",
                                                                      "flavour", "msg_cap")})
        assert st_h[i] == j["status"], "%s: status %d want %d" % (tag, st_h[i], j["status"])
        if j["op"] == OP_EMBED:
            assert ln_h[i] == j["out_len"], tag
            region = stego_o[c0:c0 + j["n"]]
            if j["status"] == OK:
                assert np.array_equal(region, j["want"]), tag + ": stego"
            else:
                assert np.all(region == SENTINEL), tag + ": failed job wrote its stego"
        elif j["raw"]:
            assert ln_h[i] == 0, tag
            k, t0, bits = j["k"], j["t0"], j["bits"]
            begin, end = k * t0, min(k * (t0 + j["n"]), bits)
            lo, hi = (begin // 8, (end + 7) // 8) if end > begin else (0, 0)
            out = msg_o[m0:m0 + mb]
            assert np.array_equal(out[lo:hi], j["want"][lo:hi]), tag + ": stream bytes"
            assert np.all(out[:lo] == SENTINEL) and np.all(out[hi:] == SENTINEL), tag + ": bytes outside written"
        else:
            assert ln_h[i] == j["out_len"], tag
            out = msg_o[m0:m0 + mb]
            if j["status"] == OK:
                assert np.array_equal(out[:j["out_len"]], j["want"]), tag + ": message"
                assert np.all(out[j["out_len"]:] == SENTINEL), tag + ": bytes past the message"
            else:
                assert np.all(out == SENTINEL), tag + ": failed job wrote its output"
        if j["op"] == OP_EXTRACT:
            assert np.array_equal(stego_o[c0:c0 + j["n"]], j["stego"]), tag + ": extract wrote its input"
        # nothing past the job's own regions
        assert np.all(msg_o[m0 + max(mb, 1):m0 + max(mb, 1) + 16] == SENTINEL), tag + ": wrote past its output"
        gap_end = batch.align_up(c0 + j["n"])
        assert np.all(stego_o[c0 + j["n"]:gap_end] == SENTINEL), tag + ": wrote past its stego"
