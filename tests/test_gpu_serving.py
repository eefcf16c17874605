"""Serving loop: continuous batching of mixed-size, mixed-precision jobs through risp_submit/risp_poll.

Each job's result must be the same alone and in the mix (bitwise: a job's arithmetic depends only on
its own inputs), admission must respect the device budget, and a failing job must not harm others.
"""
import time

import numpy as np
import pytest

import synth
from oracle import risp as R

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

JOBS = [("grid20", "fp32", 5), ("chainring30", "bf16", 4), ("chainring40", "fp32", 3),
        ("chainring24", "bf16", 5), ("chainring50", "fp32", 4)]


def _mol(name):
    if name == "grid20":
        return synth.make_config0()
    n = int(name[len("chainring"):])
    return synth.make_chain_ring(n, n)


def _wait(ctx, ids, nst, timeout=300.0):
    out = {}
    t0 = time.time()
    while len(out) < len(ids):
        for jid, ns in zip(ids, nst):
            if jid in out:
                continue
            r = ctx.poll(jid, ns)
            if r is not None:
                out[jid] = r
        assert time.time() - t0 < timeout, "serving did not finish in time"
        time.sleep(0.02)
    return out


@pytest.fixture(scope="module")
def mols():
    return {name: _mol(name) for name, _, _ in JOBS}


def _submit_all(ctx, mols, jobs):
    import paper_2603_29257_amd as P
    ids = []
    for name, prec, ns in jobs:
        sysc = P.System(mols[name])
        ids.append(ctx.submit(sysc, P.Params(precision=P.PRECISIONS[prec]), ns, tol=1e-5))
    return ids


def test_alone_equals_mix_and_oracle(mols):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29257_amd as P
    ctx = P.Context(0)
    try:
        ids = _submit_all(ctx, mols, JOBS)
        mix = _wait(ctx, ids, [j[2] for j in JOBS])
        st = ctx.serve_stats()
        print("stats", st, flush=True)
        for jid, (name, prec, ns) in zip(ids, JOBS):
            r = mix[jid]
            assert r["status"] == 0, (name, r["message"])
            assert r["t_submit"] <= r["t_admit"] <= r["t_first_sigma"] <= r["t_done"]
        # each job alone, one at a time
        for jid, (name, prec, ns) in zip(ids, JOBS):
            sysc = P.System(mols[name])
            aid = ctx.submit(sysc, P.Params(precision=P.PRECISIONS[prec]), ns, tol=1e-5)
            alone = _wait(ctx, [aid], [ns])[aid]
            print(name, prec, "mix", mix[jid]["energies"], "alone", alone["energies"], flush=True)
            assert np.array_equal(alone["energies"], mix[jid]["energies"]), name
        # the 20-atom FP32 job against the oracle
        ref = np.linalg.eigvalsh(R.dense_A(R.build_factors(mols["grid20"], R.Params())))[:5]
        assert np.abs(mix[ids[0]]["energies"] - ref).max() <= 1e-6
        with pytest.raises(P.RispError):
            ctx.poll(ids[0], 5)  # already collected
    finally:
        ctx.close()


def test_tiny_budget_queues_and_failures_are_isolated(mols):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29257_amd as P
    ctx = P.Context(0)
    try:
        fps = [P.job_footprint(P.System(mols[n]), P.Params(precision=P.PRECISIONS[p]), nstates=ns)
               for n, p, ns in JOBS[:3]]
        ctx.serve_config(budget_bytes=max(fps) + 1024, max_active=4, use_graphs=True)
        jobs = JOBS[:3]
        ids = _submit_all(ctx, mols, jobs)
        # a job whose parameters fail at admission must not harm the others
        bad = ctx.submit(P.System(mols["grid20"]), P.Params(theta=-1.0), 3, tol=1e-5)
        res = _wait(ctx, ids + [bad], [j[2] for j in jobs] + [3])
        assert res[bad]["status"] < 0 and res[bad]["message"]
        for jid in ids:
            assert res[jid]["status"] == 0
        # at every admission, the footprints of the jobs resident together fit the budget
        budget = max(fps) + 1024
        spans = [(res[j]["t_admit"], res[j]["t_done"], fp) for j, fp in zip(ids, fps)]
        for (a, d, fp) in spans:
            resident = sum(f2 for (a2, d2, f2) in spans if a2 <= a < d2)
            assert resident <= budget
        assert sum(fps) > budget  # the budget really forced queueing
        # an impossible job is rejected at submit
        big = synth.make_chain_ring(60, 60)
        with pytest.raises(P.RispError):
            ctx.submit(P.System(big), P.Params(precision=P.FP64), 5)
        with pytest.raises(P.RispError):
            ctx.poll(10 ** 9, 3)
    finally:
        ctx.close()


@pytest.mark.parametrize("name,prec,ns", [("chainring50", "bf16", 5), ("chainring40", "fp32", 4)])
def test_job_peak_memory_within_footprint(mols, name, prec, ns):
    """The admission footprint bounds what a job really holds: the library's device high-water mark
    while one job runs (BF16 with its FP32 correction stage, whose hand-off used to hold two
    Davidson runs at once; and FP32) stays within risp_job_footprint."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_29257_amd as P
    ctx = P.Context(0)
    try:
        sysc = P.System(mols[name])
        prm = P.Params(precision=P.PRECISIONS[prec])
        fp = P.job_footprint(sysc, prm, nstates=ns)
        live0, _ = P.device_usage(reset_peak=True)
        jid = ctx.submit(sysc, prm, ns, tol=1e-5)
        r = _wait(ctx, [jid], [ns])[jid]
        assert r["status"] == 0, r["message"]
        live1, peak = P.device_usage()
        print(f"{name} {prec}: peak {peak - live0} bytes, footprint {fp}, left behind {live1 - live0}", flush=True)
        assert peak - live0 <= fp
        assert live1 == live0  # every job buffer was released
    finally:
        ctx.close()
