"""GPU tests of the batched and served forms: every instance matches the same
simulation run alone (bit-identical: same kernel body, same per-node
arithmetic) and the FP64 oracle within the FP32 bar."""
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available()
    import paper_2009_12584_amd as M

    return M


def small_cases(n, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        nx = int(rng.integers(70, 260))
        ny = int(rng.integers(40, 140))
        c = W.plane_drop(nx, ny, float(rng.uniform(0, 45)), ny / 5.0, k % 3, G=3.0 if k % 2 else 0.9)
        out.append(c)
    return out


def masks_of(M, cases):
    return [M.mask_plane(c.nx, c.ny, c.geometry[1], c.geometry[2]) for c in cases]


@pytest.mark.parametrize("lanes", [1, 2])
def test_batch_matches_single_and_oracle(M, ora, lanes):
    cases = small_cases(7)
    masks = masks_of(M, cases)
    say("batch of", [(c.nx, c.ny, c.bc) for c in cases], "lanes", lanes)
    b = M.Batch([(m, c.rhoA0, c.rhoB0, c.params()) for m, c in zip(masks, cases)], lanes=lanes)
    b.step(60)
    for k, (m, c) in enumerate(zip(masks, cases)):
        s = M.Simulation(m, c.rhoA0, c.rhoB0, **c.params())
        s.step(60)
        ref = s.fields()
        s.close()
        got = b.fields(k)
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), k
        o = ora.Oracle(m, c.rhoA0, c.rhoB0, **c.params())
        o.step(60)
        of = o.fields()
        fl = m == 0
        er = max(np.max(np.abs(got[0] - of[0])[fl] / of[0][fl]), np.max(np.abs(got[1] - of[1])[fl] / of[1][fl]))
        eu = max(np.max(np.abs(got[2] - of[2])[fl]), np.max(np.abs(got[3] - of[3])[fl]))
        assert er <= 1e-5 and eu <= 1e-6, (k, er, eu)
    d = b.diag(0)
    assert d["flags"] == 0 and abs(d["mass"][0] - d["mass0"][0]) < 1e-5 * d["mass0"][0]
    b.close()


def test_batch_graph_equals_plain(M):
    cases = small_cases(5, seed=3)
    masks = masks_of(M, cases)
    items = [(m, c.rhoA0, c.rhoB0, c.params()) for m, c in zip(masks, cases)]
    a = M.Batch(items)
    g = M.Batch(items, graph_steps=20)
    a.step(41)
    g.step(41)
    for k in range(len(cases)):
        for x, y in zip(a.fields(k), g.fields(k)):
            assert np.array_equal(x, y)
    a.close()
    g.close()


def test_fp16_batch_error_at_the_bench_horizon(M):
    """Instances 0, 3 and 5 of the 64-instance batch (improved, Martys-Chen,
    LLKC) in FP16 storage, run as one batch for the bench row's 1100 steps and
    compared with the FP64 oracle.  The bar is twice the error that FP16
    storage alone gives on the same instances and steps (the oracle with the
    storage rounding applied, tests/golden/f16_model_c4.npz)."""
    import os

    import oracle

    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "f16_model_c4.npz"), allow_pickle=False)
    steps = [int(x) for x in gold["steps"]]
    T = 1100
    col = steps.index(T)
    cases = W.config4_instances(64)
    picks = [int(k) for k in gold["instances"]]
    masks = [M.mask_plane(cases[k].nx, cases[k].ny, cases[k].geometry[1], cases[k].geometry[2]) for k in picks]
    for k, m in zip(picks, masks):
        assert str(gold["input_sha_%d" % k]) == W.input_hash(cases[k], m), "stale golden"
    items = [(m, cases[k].rhoA0, cases[k].rhoB0, cases[k].params()) for k, m in zip(picks, masks)]
    say("fp16 batch of instances", picks, "to", T)
    b = M.Batch(items, storage="f16", graph_steps=100)
    b.step(T)
    for a, (k, m) in enumerate(zip(picks, masks)):
        o = oracle.Oracle(m, cases[k].rhoA0, cases[k].rhoB0, **cases[k].params())
        o.step(T)
        got, ref = b.fields(a), o.fields()
        fl = m == 0
        er = max(float(np.max(np.abs(got[j] - ref[j])[fl] / ref[j][fl])) for j in (0, 1))
        eu = max(float(np.max(np.abs(got[j] - ref[j])[fl])) for j in (2, 3))
        bar = (2 * gold["err_rho"][a, col], 2 * gold["err_u"][a, col])
        say("  instance %d: rel rho %.3e (storage model %.3e), abs u %.3e (model %.3e)" % (
            k, er, gold["err_rho"][a, col], eu, gold["err_u"][a, col]))
        assert er < bar[0] and eu < bar[1], k
    b.close()


def test_fp16_batch_and_pool_match_single_fp16(M):
    """FP16 storage (moving populations FP16, rest population FP32) has the same
    layout in the batched, pooled and single forms: results are bit-identical."""
    cases = small_cases(3, seed=9)
    masks = masks_of(M, cases)
    items = [(m, c.rhoA0, c.rhoB0, c.params()) for m, c in zip(masks, cases)]
    say("fp16 batch/pool vs single", [(c.nx, c.ny, c.bc) for c in cases])
    b = M.Batch(items, storage="f16")
    b.step(40)
    budget = sum(M.Pool.footprint(c.nx, c.ny, storage="f16") for c in cases) + 4096
    pool = M.Pool(budget, 4, storage="f16")
    slots = {pool.admit(m, c.rhoA0, c.rhoB0, 40, **c.params()): k for k, (m, c) in enumerate(zip(masks, cases))}
    assert None not in slots
    pooled = {}
    for _ in range(2000):
        pool.advance(10)
        for s in pool.poll():
            pooled[slots[s]] = pool.fields(s)
            pool.release(s)
        if len(pooled) == len(cases):
            break
        time.sleep(0.002)
    assert len(pooled) == len(cases)
    pool.close()
    for k, (m, c) in enumerate(zip(masks, cases)):
        s = M.Simulation(m, c.rhoA0, c.rhoB0, storage="f16", **c.params())
        s.step(40)
        ref = s.fields()
        s.close()
        for x, y, z in zip(b.fields(k), pooled[k], ref):
            assert np.array_equal(x, z), k
            assert np.array_equal(y, z), k
    b.close()


def test_fp16_pool_tiles_its_slots_at_the_fp16_default(M):
    """An FP16 pool tiles every slot with 16 rows, the library's default for
    the two-component step with FP16 storage: a request asking for 8 rows is
    refused on the host before anything is allocated, one asking for 16 or
    leaving the rows to the library is admitted."""
    c = small_cases(1, seed=3)[0]
    m = masks_of(M, [c])[0]
    pool = M.Pool(2 * M.Pool.footprint(c.nx, c.ny, storage="f16") + 4096, 2, storage="f16")
    with pytest.raises(M.LbmError) as e:
        pool.admit(m, c.rhoA0, c.rhoB0, 10, tile_y=8, **c.params())
    assert "16 rows" in str(e.value)
    assert pool.admit(m, c.rhoA0, c.rhoB0, 10, tile_y=16, **c.params()) is not None
    assert pool.admit(m, c.rhoA0, c.rhoB0, 10, **c.params()) is not None
    pool.close()


def test_pool_results_same_alone_and_in_the_mix(M, ora):
    """Continuous batching: requests join while others run, each stops at its own
    step count, and each result equals the same solve run alone (bit for bit)
    and the FP64 oracle within the FP32 bar.  The pool runs its fused
    diagnostics every 7 launches, which must not change any result."""
    cases = small_cases(6, seed=11)
    masks = masks_of(M, cases)
    steps = [37, 80, 15, 64, 101, 50]
    budget = sum(M.Pool.footprint(c.nx, c.ny) for c in cases[:3]) + 4096
    pool = M.Pool(budget, 4, diag_every=7)
    slots = {}
    pending = list(range(len(cases)))
    done = {}
    rounds = 0
    while pending or slots:
        # admit while memory and slots allow
        while pending:
            k = pending[0]
            c = cases[k]
            s = pool.admit(masks[k], c.rhoA0, c.rhoB0, steps[k], **c.params())
            if s is None:
                break
            slots[s] = k
            pending.pop(0)
        pool.advance(13)
        finished = pool.poll()
        for s in finished:
            k = slots.pop(s)
            done[k] = pool.fields(s)
            pool.release(s)
        if not finished:
            time.sleep(0.002)
        rounds += 1
        assert rounds < 20000
    active, used = pool.stats()
    assert active == 0 and used == 0
    pool.close()
    for k, c in enumerate(cases):
        s = M.Simulation(masks[k], c.rhoA0, c.rhoB0, **c.params())
        s.step(steps[k])
        ref = s.fields()
        s.close()
        for x, y in zip(done[k], ref):
            assert np.array_equal(x, y), k
        o = ora.Oracle(masks[k], c.rhoA0, c.rhoB0, **c.params())
        o.step(steps[k])
        of = o.fields()
        fl = masks[k] == 0
        got = done[k]
        er = max(np.max(np.abs(got[0] - of[0])[fl] / of[0][fl]), np.max(np.abs(got[1] - of[1])[fl] / of[1][fl]))
        eu = max(np.max(np.abs(got[2] - of[2])[fl]), np.max(np.abs(got[3] - of[3])[fl]))
        say("pooled request %d (%dx%d, rule %d, %d steps) vs oracle: rel rho %.2e abs u %.2e"
            % (k, c.nx, c.ny, c.bc, steps[k], er, eu))
        assert er <= 1e-5 and eu <= 1e-6, (k, er, eu)


def nan_state(nbytes):
    return np.full(nbytes // 4, np.nan, np.float32).view(np.uint8)


def test_batch_flags_one_broken_instance_and_the_others_go_on(M):
    """Failure handling forced from the host: a state of NaNs written into one
    instance of a batch (graphs of 10 steps, diagnostics every 10) makes that
    instance's diagnostics and fields return LBM_ENUMERIC; the other
    instances stay bit-identical to a batch without the broken one."""
    from paper_2009_12584_amd.capi import LBM_ENUMERIC, LbmError

    cases = small_cases(3, seed=31)
    masks = masks_of(M, cases)
    items = [(m, c.rhoA0, c.rhoB0, dict(c.params(), diag_every=10, drift_tol=1e-4)) for m, c in zip(masks, cases)]
    b = M.Batch(items, graph_steps=10)
    ref = M.Batch(items, graph_steps=10)
    b.step(20)
    ref.step(20)
    b.set_state(1, nan_state(b.get_state(1).size))
    b.step(30)
    ref.step(30)
    with pytest.raises(LbmError) as e:
        b.diag(1)
    assert e.value.code == LBM_ENUMERIC
    assert b.diag(1, raise_on_flags=False)["flags"] & 1
    with pytest.raises(LbmError) as e:
        b.fields(1)
    assert e.value.code == LBM_ENUMERIC
    for k in (0, 2):
        assert b.diag(k)["flags"] == 0
        for x, y in zip(b.fields(k), ref.fields(k)):
            assert np.array_equal(x, y), k
    assert b.launch_counts() == {"graph_steps": 50, "plain_steps": 0}
    b.close()
    ref.close()


def test_pool_reports_a_broken_slot_and_the_others_finish(M):
    """A slot whose state is made of NaNs (written from the host before it
    runs) is flagged by the pool's cadence diagnostics: poll reports it long
    before its step count, its status and fields say LBM_ENUMERIC, and the
    other slots finish with the results of the same solves run alone."""
    from paper_2009_12584_amd.capi import LBM_ENUMERIC, LbmError

    cases = small_cases(3, seed=41)
    masks = masks_of(M, cases)
    steps = [60, 400, 45]
    pool = M.Pool(1 << 30, 4, diag_every=5)
    slots = {}
    for k, (m, c) in enumerate(zip(masks, cases)):
        slots[pool.admit(m, c.rhoA0, c.rhoB0, steps[k], **c.params())] = k
    broken = [s for s, k in slots.items() if k == 1][0]
    pool.set_state(broken, nan_state(pool.get_state(broken).size))
    done, flagged_at = {}, None
    for _ in range(20000):
        pool.advance(5)
        for s in pool.poll():
            k = slots.pop(s)
            if k == 1:
                flagged_at = pool.progress()[0]
                assert pool.status(s) == LBM_ENUMERIC
                with pytest.raises(LbmError) as e:
                    pool.fields(s)
                assert e.value.code == LBM_ENUMERIC
                assert pool.diag(s, raise_on_flags=False)["flags"] & 1
            else:
                assert pool.status(s) == 0
                done[k] = pool.fields(s)
            pool.release(s)
        if not slots:
            break
        time.sleep(0.001)
    assert not slots and flagged_at is not None and flagged_at < steps[1]
    say("broken slot reported after %d launches (its step count: %d)" % (flagged_at, steps[1]))
    pool.close()
    for k in (0, 2):
        c = cases[k]
        s = M.Simulation(masks[k], c.rhoA0, c.rhoB0, **c.params())
        s.step(steps[k])
        for x, y in zip(done[k], s.fields()):
            assert np.array_equal(x, y), k
        s.close()


def test_pool_checkpoint_resume_bit_exact(M):
    """A slot's state taken mid-run and written into a fresh slot admitted for
    the remaining steps resumes bit for bit."""
    c = small_cases(1, seed=51)[0]
    m = masks_of(M, [c])[0]
    pool = M.Pool(1 << 30, 2)
    a = pool.admit(m, c.rhoA0, c.rhoB0, 90, **c.params())
    pool.advance(33)
    st = pool.get_state(a)
    b = pool.admit(m, c.rhoA0, c.rhoB0, 57, **c.params())
    pool.set_state(b, st)
    results = {}
    for _ in range(20000):
        pool.advance(20)
        for s in pool.poll():
            results[s] = pool.fields(s)
            pool.release(s)
        if len(results) == 2:
            break
        time.sleep(0.001)
    pool.close()
    for x, y in zip(results[a], results[b]):
        assert np.array_equal(x, y)


def test_pool_admission_limits(M):
    c = small_cases(1, seed=2)[0]
    m = masks_of(M, [c])[0]
    fp = M.Pool.footprint(c.nx, c.ny)
    pool = M.Pool(fp + 1024, 8)
    s0 = pool.admit(m, c.rhoA0, c.rhoB0, 10, **c.params())
    assert s0 is not None
    assert pool.admit(m, c.rhoA0, c.rhoB0, 10, **c.params()) is None  # budget
    pool.advance(20)
    t0 = time.time()
    while not pool.poll() and time.time() - t0 < 30:
        time.sleep(0.01)
    pool.release(s0)
    assert pool.admit(m, c.rhoA0, c.rhoB0, 10, **c.params()) is not None
    pool.close()
    p2 = M.Pool(10 * fp, 1)
    assert p2.admit(m, c.rhoA0, c.rhoB0, 10, **c.params()) is not None
    assert p2.admit(m, c.rhoA0, c.rhoB0, 10, **c.params()) is None  # slots
    p2.close()


@pytest.mark.parametrize("policy,slots", [("fifo", 3), ("sjf", 2)])
def test_serve_loop_completes_every_request_with_standalone_results(M, policy, slots):
    """The request loop (arrivals on a clock, admission by policy, chunked
    advance, retirement) returns every request once, with the fields of the
    same solve run alone, and reports latencies that cover arrival to
    retirement."""
    from paper_2009_12584_amd.serve import Request, serve, summarize

    cases = small_cases(5, seed=21)
    masks = masks_of(M, cases)
    steps = [40, 90, 25, 60, 75]
    reqs = [Request(0.01 * k, m, c.rhoA0, c.rhoB0, n, c.params(), tag=k)
            for k, (m, c, n) in enumerate(zip(masks, cases, steps))]
    say("serve loop", policy, slots)
    done, makespan = serve(reqs, hbm_budget=1 << 30, max_slots=slots, chunk=16, keep_fields=True, policy=policy)
    assert sorted(d.tag for d in done) == list(range(5))
    for d in done:
        k = d.tag
        assert d.finished >= d.admitted >= d.arrival - 1e-9 and d.latency <= makespan + 1e-9
        s = M.Simulation(masks[k], cases[k].rhoA0, cases[k].rhoB0, **cases[k].params())
        s.step(steps[k])
        ref = s.fields()
        s.close()
        for x, y in zip(d.fields, ref):
            assert np.array_equal(x, y), k
    summ = summarize(done, makespan)
    assert summ["requests"] == 5 and summ["p99_latency_s"] >= summ["p50_latency_s"] > 0
