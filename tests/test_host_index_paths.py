"""Host-side bounds checks of two device index paths (no GPU): the batch's
workspace layout and the walk kernel's id -> descriptor / source row /
endpoint slot mapping over whole batch tables, and the large-budget counting
kernel's hash tables (LDS table, global spill table, passes, threshold,
radix select). `host_index_paths.cpp` runs the library's own index helpers
(batch_layout.hpp, agg_hash.hpp, walk_row and desc_of from fppr_device.hpp)
against exact-size buffers with a check on every access, built with
AddressSanitizer; any access out of bounds, any endpoint slot written twice
or never, and any counting result that differs from a plain count fails."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1903_11749_amd", "csrc")
INC = os.path.join(ROOT, "include")
HERE = os.path.dirname(os.path.abspath(__file__))

BIG_THREADS = 1024  # threads of a counting block (agg_hash.hpp kBigThreads)
NO_NODE = 0xFFFFFFFF


@pytest.fixture(scope="module")
def harness():
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "h")
    subprocess.check_call(["hipcc", "-O1", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-x", "hip",
                           f"-I{CSRC}", f"-I{INC}", os.path.join(HERE, "host_index_paths.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield d, exe
    shutil.rmtree(d, ignore_errors=True)


def u64(*v):
    return np.asarray(v, dtype=np.uint64).tobytes()


def pad8(b: bytes) -> bytes:
    return b + b"\0" * (-len(b) % 8)


def batch_record(items, thread_counts=(256, 256 * 7, 256 * 1024, 256 * 4096)):
    """items: dicts n, R, counts, sources (None = all nodes), dangling (bool per node)."""
    out = [u64(1, len(thread_counts), *thread_counts), u64(len(items))]
    for it in items:
        src = it.get("sources")
        all_nodes = src is None
        src = np.zeros(0, np.uint32) if all_nodes else np.asarray(src, dtype=np.uint32)
        out.append(u64(it["n"], it["R"], 1 if it.get("counts", True) else 0, 1 if all_nodes else 0, src.size))
        out.append(pad8(src.tobytes()))
        out.append(pad8(np.asarray(it["dangling"], dtype=np.uint8).tobytes()))
    return b"".join(out)


def agg_record(rows):
    """rows: (endpoints u32 array, k, groups, block)."""
    out = [u64(2, len(rows))]
    for ep, k, groups, block in rows:
        ep = np.asarray(ep, dtype=np.uint32)
        out.append(u64(ep.size, k, groups, block))
        out.append(pad8(ep.tobytes()))
    return b"".join(out)


def run(harness, payload: bytes):
    d, exe = harness
    path = os.path.join(d, "in.bin")
    with open(path, "wb") as f:
        f.write(payload)
    r = subprocess.run([exe, path], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr


def item_of(g, R, sources=None, counts=True):
    return dict(n=g.n, R=R, counts=counts, sources=sources, dangling=g.degrees() == 0)


def test_batch_items_of_the_gpu_tests(harness):
    """The item mixes the batch GPU tests run (all nodes and source subsets,
    R from 33 to 256, graphs with many nodes without out-edges)."""
    items = [
        item_of(synth.chung_lu(3000, 30000, 2.1, 255, seed=2001), 64),
        item_of(synth.chung_lu(500, 4000, 2.5, 255, seed=2002), 256),
        item_of(synth.chung_lu(20000, 300000, 2.3, 255, seed=2003), 64, np.arange(0, 20000, 7)),
        item_of(synth.small_graph(), 100),
        item_of(synth.chung_lu(1000, 9000, 2.2, 255, seed=2004), 33, [3, 999, 3, 0, 500]),
        item_of(synth.chung_lu(64, 300, 2.1, 255, seed=2005), 256),
    ]
    run(harness, batch_record(items))


def test_batch_edges(harness):
    """R = 1 (a chunk spans 256 rows), R above the chunk, invalid and
    duplicate source ids, an empty source list, counting on the shared hash
    area (R > 256 without counts), a graph whose nodes all lack out-edges."""
    g = synth.chung_lu(700, 2000, 2.1, 255, seed=2201)
    empty = dict(n=50, R=8, counts=True, sources=None, dangling=np.ones(50, bool))
    items = [
        item_of(g, 1),
        item_of(g, 1, np.arange(700)),
        item_of(g, 300, [5, 5, 699, 700, 0xFFFFFFFE, 1], counts=False),
        item_of(g, 5000, np.arange(0, 700, 50), counts=False),
        item_of(g, 16, []),
        empty,
        item_of(g, 257),
    ]
    run(harness, batch_record(items))


def test_batch_workload_64_graphs(harness):
    """The 64-graph batch workload (all nodes, R 64 or 256), counting with and
    without per-source counts; sampled chunks where the launch is large."""
    items = []
    for sp in synth.batch_specs():
        g = synth.batch_graph(sp)
        items.append(item_of(g, sp["R"], counts=False))
    run(harness, batch_record(items))


def lds_home(t):
    return ((t * 0x9E3779B1) & 0xFFFFFFFF) >> 18


def test_counting_hash_paths(harness):
    rng = np.random.default_rng(7)
    rows = []
    # every endpoint distinct: LDS full, most spill, all counts tie -> radix select
    rows.append((rng.permutation(10**6)[:100000].astype(np.uint32), 1024, 64, 63))
    # 60,000 distinct endpoints over 10^5 walks: spills, mixed counts
    rows.append((rng.integers(0, 60000, 100000).astype(np.uint32), 1024, 64, 0))
    # few endpoints with counts above the histogram's last bin
    rows.append((rng.integers(0, 40, 100000).astype(np.uint32), 64, 64, 5))
    # Zipf-like pile-up on a few nodes, k = 1
    rows.append((np.minimum(rng.zipf(1.3, 50000), 10**6).astype(np.uint32), 1, 512, 511))
    # the smallest table (R = 257), all distinct, k larger than the distinct count
    rows.append((rng.permutation(5000)[:257].astype(np.uint32), 300, 64, 17))
    # 200 keys sharing one LDS home slot among 3000 others
    same = [t for t in range(4 * 10**6) if lds_home(t) == 1234][:200]
    ep = np.concatenate([np.repeat(np.asarray(same, np.uint32), 5), rng.integers(0, 3000, 2000)]).astype(np.uint32)
    rows.append((rng.permutation(ep), 128, 64, 1))
    # a source that got no walks (invalid id): every endpoint is the no-node mark
    rows.append((np.full(4097, NO_NODE, np.uint32), 16, 64, 2))
    # R = 2^20 at the top of the range, 2^18 distinct endpoints
    rows.append((rng.integers(0, 1 << 18, 1 << 20).astype(np.uint32), 1024, 64, 9))
    run(harness, agg_record(rows))
