"""Batched execution and the continuous-batching server against the
single-query entry points and the CPU FP64 oracle.

Bars:
  * batch vs single query, graph replay vs eager, any samples_per_block /
    raster block shape: identical bits (every kernel body is shared and every
    reduction has a fixed order);
  * uneven instances vs the oracle on the same draws: 1e-4 relative in the
    infinity norm over each output, the FP32 parity tolerance.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as WL
from scenes import disk_target, gpu_disks, oracle_disks, pt_target, rel_inf, small_disks

pytestmark = pytest.mark.gpu
TOL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import paper_2412_03489_amd as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def ctx(P):
    c = P.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def scenes(P, ctx):
    """Scenes of every kind the batch path handles."""
    out = {}
    w1 = WL.one_disk()
    out["one_disk"] = (w1, gpu_disks(ctx, w1, disk_target(w1)))
    wr = small_disks()
    out["ragged"] = (wr, gpu_disks(ctx, wr, disk_target(wr)))
    w4 = small_disks(W=40, H=70, D=12, C=4, seed=5)
    out["c4"] = (w4, gpu_disks(ctx, w4, disk_target(w4)))
    w2 = small_disks(W=33, H=47, D=9, C=2, seed=6)
    out["c2"] = (w2, gpu_disks(ctx, w2, disk_target(w2)))
    # 33 to 64 disks: the render pairs' 64-disk layout
    w48 = small_disks(W=45, H=52, D=48, C=3, seed=9)
    out["d48"] = (w48, gpu_disks(ctx, w48, disk_target(w48)))
    wp = WL.pt_spheres()
    tgt = pt_target(wp, spp=64, W=32, H=24)
    out["pt"] = (wp, P.Scene.pt(ctx, 32, 24, 2, wp.desc, tgt))
    g = np.random.default_rng(8)
    M = g.standard_normal((3, 3))
    out["quad"] = (None, P.Scene.quad(ctx, M @ M.T + np.eye(3), g.standard_normal(3), 0.4))
    out["neggauss"] = (None, P.Scene.neggauss(ctx, 4, 0.7))
    return out


def mixed_queries(scenes):
    """A batch mixing scenes, kinds, samplers, sample budgets and options."""
    w1, s1 = scenes["one_disk"]
    wr, sr = scenes["ragged"]
    w4, s4 = scenes["c4"]
    wp, sp = scenes["pt"]
    _, sq = scenes["quad"]
    _, sn = scenes["neggauss"]
    w2, s2 = scenes["c2"]
    w48, s48 = scenes["d48"]
    vr = wr.v / np.linalg.norm(wr.v)
    vp = np.array([1.0, 0.2, -0.5, 0.3, 0.0, 0.7])
    return [
        dict(scene=s1, kind="grad", theta=w1.theta0, sigma=w1.sigma, N=777, seed=1),
        dict(scene=s1, kind="hess", theta=w1.theta0, sigma=w1.sigma, N=500, seed=2, sampler=1),
        dict(scene=sr, kind="hvp", theta=wr.theta0, sigma=wr.sigma, N=96, seed=3, v=vr),
        dict(scene=sr, kind="hvp_limit", theta=wr.theta0, sigma=wr.sigma, N=130, seed=4, v=vr),
        dict(scene=sr, kind="loss", theta=wr.theta0, sigma=wr.sigma, N=200, seed=5),
        dict(scene=sr, kind="loss", theta=wr.theta0, sigma=0.0, N=1, seed=0),
        dict(scene=s4, kind="grad", theta=w4.theta0, sigma=0.03, N=300, seed=6, sampler=3),
        dict(scene=s4, kind="hess", theta=w4.theta0, sigma=0.03, N=64, seed=7, accum_fp64=True),
        dict(scene=sp, kind="hess", theta=wp.theta0, sigma=wp.sigma, N=24, seed=8),
        dict(scene=sp, kind="hvp", theta=wp.theta0, sigma=wp.sigma, N=20, seed=9, v=vp),
        dict(scene=sq, kind="hvp", theta=np.array([0.3, -0.2, 0.5]), sigma=0.5, N=1037, seed=10,
             v=np.array([0.5, 1.0, -2.0]), sampler=2),
        dict(scene=sn, kind="hess", theta=np.array([0.1, -0.3, 0.2, 0.0]), sigma=0.4, N=2000,
             seed=11),
        dict(scene=s1, kind="hvp", theta=w1.theta0, sigma=w1.sigma, N=64, seed=12,
             v=np.zeros(2)),
        dict(scene=s4, kind="hess", theta=w4.theta0, sigma=0.03, N=80, seed=13,
             hess_mix_n2=True),
        dict(scene=sp, kind="hvp_limit", theta=wp.theta0, sigma=wp.sigma, N=16, seed=14, v=vp,
             hess_mix_n2=True),
        dict(scene=s2, kind="grad", theta=w2.theta0, sigma=0.02, N=150, seed=15),
        # HVPs rendered as +-h pairs (at most 64 disks), one per channel count
        dict(scene=s4, kind="hvp", theta=w4.theta0, sigma=0.03, N=77, seed=16,
             v=w4.v / np.linalg.norm(w4.v)),
        dict(scene=s2, kind="hvp", theta=w2.theta0, sigma=0.02, N=40, seed=17, v=w2.v,
             accum_fp64=True),
        dict(scene=s1, kind="hvp", theta=w1.theta0, sigma=w1.sigma, N=333, seed=18,
             v=np.array([0.6, -0.8])),
        dict(scene=s4, kind="hvp", theta=w4.theta0, sigma=0.03, N=20, seed=19, v=w4.v,
             hvp_per_render=True),
        dict(scene=s48, kind="hvp", theta=w48.theta0, sigma=0.02, N=50, seed=20,
             v=w48.v / np.linalg.norm(w48.v)),
    ]


def single(P, q):
    q = dict(q)
    kind = q.pop("kind")
    if kind == "loss":
        for k in ("sampler",):
            q.pop(k, None)
        return np.array([P.est_loss(q["scene"], q["theta"], q["sigma"], q["N"], q["seed"],
                                    antithetic=q.get("antithetic", True))])
    return P.estimate(kind, q.pop("scene"), q.pop("theta"), q.pop("sigma"), q.pop("N"),
                      q.pop("seed"), v=q.pop("v", None), **q)


def test_batch_matches_single_queries_bitwise(P, ctx, scenes):
    qs = mixed_queries(scenes)
    b = P.Batch(ctx, use_graph=False)
    # a different batch first, so stale workspace contents cannot pass for results
    say("batch warm-up with other queries")
    b.run(list(reversed(qs[:6])))
    say(f"batch of {len(qs)} mixed queries, eager")
    got = b.run(qs)
    rep = b.report()
    assert rep["queries"] == len(qs) and rep["raster_items"] > 0 and rep["pt_items"] > 0
    for k, q in enumerate(qs):
        ref = single(P, q)
        assert np.array_equal(np.ravel(got[k]), np.ravel(ref)), (k, q["kind"])
    b.close()


def test_batch_graph_replays_match_eager(P, ctx, scenes):
    qs = mixed_queries(scenes)
    eager = P.Batch(ctx, use_graph=False).run(qs)
    b = P.Batch(ctx, use_graph=True)
    for rep in range(3):
        say(f"graph replay {rep}")
        got = b.run(qs)
        assert b.report()["graph"] == 1
        for x, y in zip(got, eager):
            assert np.array_equal(x, y)
        # eager work of the program between replays
        w1, s1 = scenes["one_disk"]
        P.estimate("grad", s1, w1.theta0, w1.sigma, 256, 40 + rep)
    # a replay with other values of theta and v in the same table layout
    qs2 = [dict(q) for q in qs]
    for q in qs2:
        q["theta"] = np.asarray(q["theta"], float) * 1.01
    e2 = P.Batch(ctx, use_graph=False).run(qs2)
    g2 = b.run(qs2)
    for x, y in zip(g2, e2):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("name", ["one_disk", "ragged", "c4", "c2"])
def test_raster_tiles_and_samples_do_not_change_bits(P, ctx, scenes, name):
    w, sc = scenes[name]
    base = P.estimate("grad", sc, w.theta0, w.sigma, 200, 5)
    for tile in (1, 2, 3):
        for spb in (1, 7, 16, 64, 200, 256):
            say(f"{name} raster_tile={tile} samples_per_block={spb}")
            got = P.estimate("grad", sc, w.theta0, w.sigma, 200, 5, samples_per_block=spb,
                             raster_tile=tile)
            assert np.array_equal(got, base)
    qs = [dict(scene=sc, kind="grad", theta=w.theta0, sigma=w.sigma, N=200, seed=5,
               samples_per_block=spb, raster_tile=t) for t in (1, 2, 3) for spb in (5, 64, 256)]
    for got in P.Batch(ctx).run(qs):
        assert np.array_equal(got, base)


def test_uneven_instances_vs_oracle(P, ctx):
    """The 64 uneven disk instances (sides 32-512 px, 1-32 disks, gradient /
    Hessian / HVP) in one batch; each against the oracle on the same draws
    (sample budgets cut so the oracle finishes in seconds)."""
    ws = WL.uneven(64)
    qs, orefs = [], []
    for w in ws:
        tgt = disk_target(w)
        gsc = gpu_disks(ctx, w, tgt)
        osc = oracle_disks(w, tgt)
        kind = w.kinds[0]
        N = 48 if kind == "hvp" else 96
        v = getattr(w, "v", None)
        q = dict(scene=gsc, kind=kind, theta=w.theta0, sigma=w.sigma, N=N, seed=w.seed)
        if kind == "hvp":
            q["v"] = v
        qs.append(q)
        orefs.append((osc, w, kind, N, v))
    say(f"uneven batch of {len(qs)}")
    got = P.Batch(ctx, use_graph=True).run(qs)
    for (osc, w, kind, N, v), g in zip(orefs, got):
        say(f"oracle {w.name} {kind} {w.W}x{w.H} D={w.D} N={N}")
        ref = O.estimate(kind, osc, w.theta0, w.sigma, N, w.seed, v=v)
        assert rel_inf(g, ref) < TOL, (w.name, kind, rel_inf(g, ref))


def test_autotuner_keeps_results(P, ctx, scenes):
    w, sc = scenes["ragged"]
    q = dict(scene=sc, kind="grad", theta=w.theta0, sigma=w.sigma, N=300, seed=9)
    base = P.Batch(ctx).run([q])[0]
    b = P.Batch(ctx, autotune=True)
    say("autotune ragged")
    got = b.run([q, dict(q, seed=10)])
    S, tile = P.tuned(ctx, sc)
    # the autotuner times S in {32, 64, 128, 256}; which one wins depends on
    # the GPU's timing, the result bits must not
    assert S in (32, 64, 128, 256) and tile in (1, 2, 3)
    assert np.array_equal(got[0], base)


def test_autotuner_tunes_path_traced_queries(P, ctx, scenes):
    """Draws per block item of a path-traced class are timed over 2..32 and
    kept; the result bits do not depend on them."""
    wp, sp = scenes["pt"]
    q = dict(scene=sp, kind="hess", theta=wp.theta0, sigma=wp.sigma, N=40, seed=11)
    base = P.Batch(ctx).run([q])[0]
    say("autotune path-traced Hessian")
    got = P.Batch(ctx, autotune=True).run([q, dict(q, seed=12)])
    S, tile = P.tuned(ctx, sp)
    assert S in (2, 4, 8, 16, 32) and tile == 0
    assert np.array_equal(got[0], base)
    for s in (2, 32):   # any explicit value gives the same bits
        assert np.array_equal(P.Batch(ctx).run([dict(q, samples_per_block=s)])[0], base)


def test_batch_errors(P, ctx, scenes):
    w, sc = scenes["ragged"]
    b = P.Batch(ctx)
    good = dict(scene=sc, kind="grad", theta=w.theta0, sigma=w.sigma, N=16, seed=1)
    with pytest.raises(P.HrError) as e:
        b.run([good, dict(good, sigma=-1.0)])
    assert "query 1" in str(e.value)
    with pytest.raises(P.HrError):
        b.run([dict(good, kind="hvp")])   # v missing
    with pytest.raises(P.HrError):
        b.run([dict(scene=scenes["one_disk"][1], kind="hess", theta=WL.one_disk().theta0,
                    sigma=0.05, N=16, seed=1, sampler=3)])   # FR22 has no Hessian
    ctx.set_memory_budget(1 << 20)
    try:
        with pytest.raises(P.HrError) as e:
            b.run([dict(good, N=4096)])
        assert e.value.status == -2
    finally:
        ctx.set_memory_budget(64 << 30)
    assert b.run([]) == []


# ------------------------------------------------------------------ server
def test_server_results_alone_and_in_the_mix(P, ctx, scenes):
    qs = [q for q in mixed_queries(scenes)]
    alone = [single(P, q) for q in qs]
    srv = P.Server(ctx, slots=2, max_batch=5, memory_bytes=1 << 30)
    tickets = []
    for rnd in range(3):
        for q in qs:
            q = dict(q)
            tickets.append((srv.submit(q.pop("scene"), q.pop("kind"), q.pop("theta"),
                                       q.pop("sigma"), q.pop("N"), q.pop("seed"),
                                       v=q.pop("v", None), **q), len(tickets) % len(qs)))
    say(f"server: {len(tickets)} queries submitted")
    done = set()
    while len(done) < len(tickets):
        t = srv.wait_any(timeout_ms=60000)
        assert t is not None
        done.add(t)
    for t, k in tickets:
        out, st = srv.wait(t)
        assert st["status"] == 0
        assert st["submit_ms"] <= st["start_ms"] <= st["end_ms"]
        assert np.array_equal(np.ravel(out), np.ravel(alone[k])), k
    s = srv.stats()
    assert s["submitted"] == len(tickets) and s["completed"] == len(tickets)
    assert s["batches"] >= len(tickets) // 5
    srv.close()


def test_server_writes_query_metrics_as_json_lines(P, ctx, scenes, tmp_path):
    """With metrics_path set, the server appends one JSON object per completed
    query: the query's identity, the batch and slot it ran in, and its times,
    consistent with what hr_wait reports."""
    import json
    qs = [q for q in mixed_queries(scenes)]
    path = str(tmp_path / "queries.jsonl")
    srv = P.Server(ctx, slots=2, max_batch=4, memory_bytes=1 << 30, metrics_path=path)
    tickets = {}
    for q in qs:
        q = dict(q)
        kind = q.pop("kind")
        t = srv.submit(q.pop("scene"), kind, q.pop("theta"), q.pop("sigma"), q.pop("N"),
                       q.pop("seed"), v=q.pop("v", None), **q)
        tickets[t] = kind
    stats = {t: srv.wait(t)[1] for t in tickets}
    srv.close()
    say(f"server metrics: {len(tickets)} queries")
    rows = [json.loads(ln) for ln in open(path).read().splitlines()]
    assert sorted(r["ticket"] for r in rows) == sorted(tickets)
    per_batch = {}
    for r in rows:
        st = stats[r["ticket"]]
        assert r["kind"] == tickets[r["ticket"]]
        assert r["status"] == 0 and st["status"] == 0
        assert r["batch_size"] == st["batch_size"]
        assert abs(r["submit_ms"] - st["submit_ms"]) < 1e-3
        assert abs(r["end_ms"] - st["end_ms"]) < 1e-3
        assert r["submit_ms"] <= r["start_ms"] <= r["end_ms"]
        assert r["queue_ms"] >= 0 and r["service_ms"] >= 0
        if r["batch"]:
            per_batch.setdefault(r["batch"], []).append(r)
    for b, rs in per_batch.items():   # a batch's queries name it and its size
        assert all(r["batch_size"] == len(rs) for r in rs), b
        assert len({r["slot"] for r in rs}) == 1
    # a file that cannot be opened is refused
    with pytest.raises(P.HrError):
        P.Server(ctx, metrics_path=str(tmp_path / "no_such_dir" / "m.jsonl"))


def test_server_admission_by_memory(P, ctx, scenes):
    w, sc = scenes["ragged"]
    srv = P.Server(ctx, slots=2, max_batch=64, memory_bytes=64 << 20)
    with pytest.raises(P.HrError) as e:   # alone larger than a slot
        srv.submit(sc, "hess", w.theta0, w.sigma, 100000, 1)
    assert e.value.status == -2
    # each query needs a good share of a slot: batches must split by memory
    ts = [srv.submit(sc, "grad", w.theta0, w.sigma, 3000, 100 + i) for i in range(6)]
    outs = [srv.wait(t) for t in ts]
    assert max(st["batch_size"] for _, st in outs) < 6
    ref = P.estimate("grad", sc, w.theta0, w.sigma, 3000, 103)
    assert np.array_equal(outs[3][0], ref)
    srv.close()
    # a predicted-time cap below any query's cost: one query per batch
    srv = P.Server(ctx, slots=2, max_batch=64, max_batch_ms=1e-9, memory_bytes=64 << 20)
    ts = [srv.submit(sc, "grad", w.theta0, w.sigma, 64, 200 + i) for i in range(5)]
    assert all(srv.wait(t)[1]["batch_size"] == 1 for t in ts)
    srv.close()


def test_server_concurrent_clients(P, ctx, scenes):
    """Four client threads submit and wait at the same time (the binding drops
    the GIL inside library calls); every result equals the query run alone."""
    import threading
    qs = [q for q in mixed_queries(scenes) if q["kind"] in ("grad", "hvp", "hess")]
    alone = [single(P, q) for q in qs]
    srv = P.Server(ctx, slots=3, max_batch=8, memory_bytes=1 << 30)
    errors = []

    def client(cid):
        try:
            for rnd in range(3):
                order = list(range(len(qs)))[cid::2] if rnd % 2 else list(range(len(qs)))
                tickets = []
                for k in order:
                    q = dict(qs[k])
                    tickets.append((srv.submit(q.pop("scene"), q.pop("kind"), q.pop("theta"),
                                               q.pop("sigma"), q.pop("N"), q.pop("seed"),
                                               v=q.pop("v", None), **q), k))
                for t, k in tickets:
                    out, st = srv.wait(t)
                    if st["status"] != 0 or not np.array_equal(np.ravel(out), np.ravel(alone[k])):
                        errors.append((cid, k))
        except Exception as e:   # reported below, not swallowed
            errors.append((cid, repr(e)))

    say("server: 4 concurrent client threads")
    th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in th)
    assert errors == []
    assert srv.wait_any(timeout_ms=1.0) is None   # nothing left to hand out
    s = srv.stats()
    assert s["submitted"] == s["completed"]
    srv.close()


def test_server_second_waiter_and_scene_destroy(P, ctx, scenes):
    """One waiter per ticket: a second concurrent hr_wait on the same ticket
    is refused (HR_EBUSY) or finds it retired (HR_EINVAL), never a freed
    ticket.  A scene destroyed while the server still holds queries on it
    waits for them; their results are those of the queries run alone."""
    import ctypes as C
    import threading
    w, _ = scenes["ragged"]
    sc = gpu_disks(ctx, w, disk_target(w))
    srv = P.Server(ctx, slots=2, max_batch=4, memory_bytes=1 << 30)
    t = srv.submit(sc, "grad", w.theta0, w.sigma, 20000, 31)
    codes, outs = {}, {}

    def waiter(i):
        out = np.zeros(w.n)
        st = P.QueryStats()
        codes[i] = P.lib().hr_wait(srv.h, C.c_uint64(t), out.ctypes.data_as(C.c_void_p),
                                   C.byref(st))
        outs[i] = (out, st.status)

    # either waiter may reach the ticket first: exactly one gets the result
    th = [threading.Thread(target=waiter, args=(i,)) for i in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=60)
    assert not any(x.is_alive() for x in th)
    won = [i for i in (0, 1) if codes[i] == 0]
    assert len(won) == 1, codes
    assert codes[1 - won[0]] in (-5, -1), codes
    assert outs[won[0]][1] == 0
    assert np.array_equal(outs[won[0]][0],
                          P.estimate("grad", sc, w.theta0, w.sigma, 20000, 31))
    say("server: scene destroyed with queries held")
    ts = [srv.submit(sc, "grad", w.theta0, w.sigma, 4000, 40 + i) for i in range(6)]
    sc.close()   # blocks until the server has finished the six queries
    got = [srv.wait(x)[0] for x in ts]
    srv.close()
    ref_scene = gpu_disks(ctx, w, disk_target(w))
    for i, g in enumerate(got):
        assert np.array_equal(g, P.estimate("grad", ref_scene, w.theta0, w.sigma, 4000, 40 + i))
    ref_scene.close()
