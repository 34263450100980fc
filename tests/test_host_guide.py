"""Guide-table routines of the weighted pick (guide.hpp), built for the host
and checked against plain definitions (no GPU): thresholds ceil(P 2^64 / W)
against exact integer arithmetic, and the pick of every table built from
rows of very different weight shapes against the flat search "first prefix
above floor(D W / 2^64)" of Sec. 2.1, for random draws, every threshold and
its neighbours and every bucket edge. `host_guide.cpp` is the harness; it is
built with AddressSanitizer and checks every table access."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1903_11749_amd", "csrc")
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def harness():
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "g")
    subprocess.check_call(["hipcc", "-O1", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-x", "hip",
                           f"-I{CSRC}", os.path.join(HERE, "host_guide.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def run(exe, payload: bytes):
    r = subprocess.run([exe], input=payload, capture_output=True, timeout=600)
    return r.returncode, r.stdout


def test_thresholds_exact(harness):
    rng = np.random.default_rng(71)
    pairs = []
    for _ in range(20000):
        W = int(rng.integers(2, 1 << 59, dtype=np.uint64))
        P = int(rng.integers(1, W, dtype=np.uint64))
        pairs.append((P, W))
    for W in (2, 3, 5, 7, 1 << 32, (1 << 32) + 1, (1 << 59) - 1, 1 << 62, (1 << 63) - 1, 1 << 63):
        for P in (1, 2, W // 2, W // 3 + 1, W - 2, W - 1):
            if 1 <= P < W:
                pairs.append((P, W))
    for k in range(1, 64):  # powers of two and their neighbours
        for W in ((1 << k) + 1, (1 << k) + 3):
            if W <= 1 << 63:
                pairs.append((1, W))
                pairs.append((W - 1, W))
    payload = np.asarray([1, len(pairs)], np.uint64).tobytes() + np.asarray(pairs, np.uint64).tobytes()
    rc, out = run(harness, payload)
    assert rc == 0, out[:400]
    got = np.frombuffer(out, np.uint64)
    want = [-(-(P << 64) // W) for P, W in pairs]  # ceil(P 2^64 / W)
    assert len(got) == len(pairs)
    bad = [i for i, (g, w) in enumerate(zip(got.tolist(), want)) if g != w]
    assert not bad, [(pairs[i], int(got[i]), want[i]) for i in bad[:5]]


def rows_payload(rows, draws, seed):
    parts = [np.asarray([2, len(rows), draws, seed], np.uint64).tobytes()]
    for w in rows:
        w = np.asarray(w, np.uint32)
        parts.append(np.asarray([w.size], np.uint64).tobytes())
        parts.append(w.tobytes())
    return b"".join(parts)


def shaped_rows(rng):
    rows = []
    for d in (1, 2, 3, 4, 5, 7, 8, 9, 16, 31, 33, 64, 65, 100, 257, 1000, 4097):
        rows.append(rng.integers(1, 101, d))                       # uniform small weights
        rows.append(np.minimum(rng.zipf(1.2, d), 10000))           # the scale-24 weight law
        rows.append(np.full(d, 1))                                 # all equal
        w = np.ones(d, np.int64)
        w[rng.integers(0, d)] = 0xFFFFFFFF                         # one huge edge among ones
        rows.append(w)
    rows.append(2 ** np.arange(32, dtype=np.int64) % (1 << 32))    # doubling weights
    rows.append(np.r_[np.full(500, 1), [0xFFFFFFFF] * 3, np.full(500, 1)])  # a cluster split by giants
    rows.append(np.r_[[0xFFFFFFFF], np.full(3000, 1), [0xFFFFFFFF]])  # tiny edges in one bucket
    rows.append(np.minimum(rng.zipf(1.2, 200000), 10000))          # a hub row of the scale-24 law
    rows.append(np.full(70000, 0xFFFFFFFF))                        # largest totals
    return [np.maximum(np.asarray(r, np.int64), 1) for r in rows]


def test_pick_equals_flat_search(harness):
    rng = np.random.default_rng(72)
    rows = shaped_rows(rng)
    rc, out = run(harness, rows_payload(rows, 4000, 73))
    text = out.decode()
    assert rc == 0 and text.startswith("ok"), text[:400]
    reads = float(text.split("reads_per_pick")[1])
    assert 1.0 <= reads < 3.0, text


def test_random_rows(harness):
    rng = np.random.default_rng(74)
    rows = []
    for _ in range(300):
        d = int(rng.integers(1, 3000))
        law = rng.integers(0, 3)
        if law == 0:
            w = rng.integers(1, 1 << 32, d, dtype=np.uint64)
        elif law == 1:
            w = np.minimum(rng.zipf(1.1, d), 0xFFFFFFFF)
        else:
            w = np.where(rng.random(d) < 0.9, 1, rng.integers(1, 1 << 32, d, dtype=np.uint64))
        rows.append(np.asarray(w, np.int64))
    rc, out = run(harness, rows_payload(rows, 2000, 75))
    text = out.decode()
    assert rc == 0 and text.startswith("ok"), text[:400]
