"""The query server through the C-ABI: every query's result is bit-identical
in the mix (continuous batching, many queries per slice, small slices so each
query spans several), in FIFO mode and run alone; admission respects the
memory budget; malformed queries are refused."""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fp():
    import torch

    from paper_1903_11749_amd import fppr

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    fppr.lib()
    return fppr


@pytest.fixture(scope="module")
def world(fp):
    g = synth.chung_lu(30000, 400000, 2.2, 255, seed=2030)
    G = fp.Graph(g, layout=fp.FPPR_LAYOUT_NARROW)  # the layout the large resident graph gets
    G.build_pool(S=32, L=3, K=64, alpha=0.15, seed=12)
    rng = np.random.default_rng(2031)
    queries = []
    for q in range(40):
        ns = int(rng.integers(1, 300)) if q % 5 else 1
        R = int(rng.choice([50, 300, 1000, 4096, 5000, 20000])) if q % 7 else 3
        queries.append(dict(sources=rng.integers(0, g.n, ns).astype(np.uint32), R=R, alpha=0.15,
                            seed=1000 + q, topk=min(64, R), stitch=bool(q % 2)))
    return g, G, queries


def alone(fp, G, q):
    import torch

    o = fp.run(G, q["alpha"], q["R"], q["seed"], sources=q["sources"], topk=q["topk"], stitch=q["stitch"],
               counts=False, stats=False)
    torch.cuda.synchronize()
    return o.topk.cpu().numpy().view(np.uint32), o.digest.cpu().numpy().view(np.uint64)


def serve_all(fp, G, queries, want_latency=False, **kw):
    S = fp.Server(G, **kw)
    ids = [S.submit(q["sources"], q["R"], q["alpha"], q["seed"], q["topk"], q["stitch"]) for q in queries]
    out = [S.wait(i) for i in ids]
    st = S.stats()
    lat = S.latency()
    S.close()
    return (out, st, lat) if want_latency else (out, st)


def nearest_rank(v, q):
    v = np.sort(np.asarray(v, dtype=np.float64))
    return v[max(1, int(np.ceil(q * v.size))) - 1]


def test_continuous_equals_alone_and_oracle(fp, world):
    g, G, queries = world
    say("case: 40 mixed queries, continuous, 2^16-walk slices")
    out, st, lat = serve_all(fp, G, queries, want_latency=True, mode="continuous", max_requests=16,
                             slice_walks=1 << 16)
    say(f"  stats: {st}")
    say(f"  latency: {lat}")
    # the library's latency statistics are those of the queries' own times
    ms = [(info["done_ns"] - info["submit_ns"]) * 1e-6 for _, _, info in out]
    assert lat["count"] == len(queries)
    assert abs(lat["p50_ms"] - nearest_rank(ms, 0.5)) < 1e-6
    assert abs(lat["p99_ms"] - nearest_rank(ms, 0.99)) < 1e-6
    assert abs(lat["max_ms"] - max(ms)) < 1e-6 and abs(lat["mean_ms"] - np.mean(ms)) < 1e-6
    span = (max(i["done_ns"] for _, _, i in out) - min(i["submit_ns"] for _, _, i in out)) * 1e-9
    assert abs(lat["qps"] - len(queries) / span) < 1e-6 * lat["qps"]
    assert st["completed"] == len(queries)
    assert st["slices"] > len(queries)  # queries spanned several slices
    assert st["peak_in_flight"] > 1
    want_walks = sum(q["sources"].size * q["R"] for q in queries)
    assert st["walk_stats"]["walks"] == want_walks
    for q, (topk, digest, info) in zip(queries, out):
        t, d = alone(fp, G, q)
        assert np.array_equal(topk, t) and np.array_equal(digest, d)
        assert info["submit_ns"] <= info["admit_ns"] <= info["done_ns"]
        assert info["walks"] == q["sources"].size * q["R"]
    og = O.Graph.from_csr(g)
    pool = O.Pool(og, S=32, L=3, K=64, alpha=0.15, seed=12)
    for qi in (0, 3, 7, 10):
        q = queries[qi]
        ref = O.run(og, q["alpha"], q["R"], q["seed"], sources=q["sources"], topk=q["topk"],
                    pool=pool if q["stitch"] else None, want_counts=False)
        assert np.array_equal(out[qi][0], ref.topk) and np.array_equal(out[qi][1], ref.digest)


def test_fifo_equals_continuous(fp, world):
    g, G, queries = world
    say("case: FIFO mode")
    out_f, st = serve_all(fp, G, queries[:20], mode="fifo", max_requests=8)
    assert st["walk_launches"] == 20
    for q, (topk, digest, _) in zip(queries[:20], out_f):
        t, d = alone(fp, G, q)
        assert np.array_equal(topk, t) and np.array_equal(digest, d)


def test_memory_admission(fp, world):
    """A 64 MiB budget holds at most a couple of these queries at once; all
    still finish, in order of admission, with the same results."""
    g, G, queries = world
    say("case: memory-bounded admission")
    rng = np.random.default_rng(2032)
    qs = [dict(q, R=20000, sources=rng.integers(0, g.n, 100).astype(np.uint32), topk=64)
          for q in queries[:10]]
    need = 100 * 20000 * 4  # endpoint buffer of each query (outputs add a little)
    out, st = serve_all(fp, G, qs, mode="continuous", max_requests=64, memory_bytes=64 << 20,
                        slice_walks=1 << 20)
    say(f"  stats: {st}")
    assert st["peak_device_bytes"] <= 64 << 20
    assert 1 <= st["peak_in_flight"] <= (64 << 20) // need < len(qs)
    for q, (topk, digest, _) in zip(qs, out):
        t, d = alone(fp, G, q)
        assert np.array_equal(topk, t) and np.array_equal(digest, d)


def test_invalid_queries_and_backpressure(fp, world):
    g, G, queries = world
    S = fp.Server(G, mode="continuous", memory_bytes=8 << 20, host_bytes=1 << 20)
    for bad in (dict(sources=[g.n], R=10, topk=4), dict(sources=[1], R=0, topk=1),
                dict(sources=[1], R=10, topk=11), dict(sources=np.arange(1000), R=20000, topk=8)):
        with pytest.raises(fp.FpprError):
            S.submit(bad["sources"], bad["R"], 0.15, 1, bad["topk"])
    with pytest.raises(fp.FpprError):  # pool built for alpha 0.15
        S.submit([1, 2], 100, 0.2, 1, 4, stitch=True)
    # pinned staging of 1 MiB: 1000 sources x k=64 take ~0.5 MiB each
    ids, refused = [], False
    for i in range(4):
        try:
            ids.append(S.submit(np.arange(1000, dtype=np.uint32), 100, 0.15, 50 + i, 64))
        except fp.FpprError as e:
            assert e.status == fp.FPPR_CAPACITY
            refused = True
            break
    assert refused and len(ids) >= 1
    first = S.wait(ids[0])
    assert first is not None
    ids.append(S.submit(np.arange(1000, dtype=np.uint32), 100, 0.15, 99, 64))  # room again
    for i in ids[1:]:
        S.wait(i)
    S.close()


def test_cancel_queued_in_flight_and_finished(fp, world):
    """One query in flight at a time: a long query is cancelled while its
    slices run, a queued one before it reaches the GPU, a finished one
    before its results are taken. Each then polls as FPPR_CANCELLED; the
    others keep their results; the cancelled query's memory comes back."""
    import time

    g, G, queries = world
    say("case: cancel queued, in-flight and finished queries")
    rng = np.random.default_rng(2040)
    S = fp.Server(G, mode="continuous", max_requests=1, memory_bytes=96 << 20, slice_walks=1 << 16)
    big = dict(sources=rng.integers(0, g.n, 300).astype(np.uint32), R=60000, alpha=0.15, seed=7, topk=64,
               stitch=True)  # 72 MB of endpoints, ~275 slices of 2^16 walks
    small = [dict(sources=rng.integers(0, g.n, 20).astype(np.uint32), R=500, alpha=0.15, seed=70 + i, topk=16,
                  stitch=bool(i % 2)) for i in range(3)]
    sub = lambda q: S.submit(q["sources"], q["R"], q["alpha"], q["seed"], q["topk"], q["stitch"])
    a = sub(big)
    b, c, d = (sub(q) for q in small)
    t0 = time.time()
    while S.stats()["slices"] < 3 and time.time() - t0 < 30:  # the big query is on the GPU
        time.sleep(0.001)
    assert S.stats()["slices"] >= 3
    S.cancel(c)  # still queued behind the big one
    S.cancel(a)  # in flight
    for qid in (a, c):
        with pytest.raises(fp.FpprError) as ei:
            S.wait(qid)
        assert ei.value.status == fp.FPPR_CANCELLED
    with pytest.raises(fp.FpprError):  # forgotten after FPPR_CANCELLED
        S.poll(a)
    for qid, q in ((b, small[0]), (d, small[2])):
        topk, digest, _ = S.wait(qid)
        t, dg = alone(fp, G, q)
        assert np.array_equal(topk, t) and np.array_equal(digest, dg)
    st = S.stats()
    assert st["cancelled"] == 2 and st["completed"] == 2
    assert st["walk_stats"]["walks"] < big["sources"].size * big["R"]  # the rest was never launched
    # the big query's memory is free again: the same query runs to the end
    e = sub(big)
    topk, digest, _ = S.wait(e)
    t, dg = alone(fp, G, big)
    assert np.array_equal(topk, t) and np.array_equal(digest, dg)
    # a finished query whose results were not taken
    f = sub(small[1])
    t0 = time.time()
    while S.stats()["completed"] < 4 and time.time() - t0 < 30:
        time.sleep(0.001)
    S.cancel(f)
    with pytest.raises(fp.FpprError) as ei:
        S.poll(f)
    assert ei.value.status == fp.FPPR_CANCELLED
    S.close()


def test_destroy_with_work_queued(fp, world):
    """Destroying a server right after submitting (queries queued and in
    flight, one cancelled) finishes the rest and returns cleanly."""
    g, G, queries = world
    say("case: destroy with queued work")
    for mode in ("continuous", "fifo"):
        S = fp.Server(G, mode=mode, max_requests=2, slice_walks=1 << 16)
        ids = [S.submit(q["sources"], q["R"], q["alpha"], q["seed"], q["topk"], q["stitch"]) for q in queries[:12]]
        S.cancel(ids[5])
        S.close()  # raises if the library reports a failure
