"""The library's per-row alias routine (alias_row.hpp) and per-node big-move
routine (big_moves_node.hpp) are plain integer code that the kernels call
one thread per row or node; compiled for the host here, with exact-capacity
buffers under AddressSanitizer, they must reproduce the oracle's tables
bit for bit (CPU, no GPU needed)."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import synth
from oracle import alias as A
from oracle import big_moves as BM
from oracle import oracle as O

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_1903_11749_amd", "csrc")

HARNESS = r"""
#include "alias_row.hpp"
#include "big_moves_node.hpp"
#include <cstdio>
#include <vector>
// stdin-free: argv[1] input file: n m S T d cap (u64), off[n+1] u64, col[m] u32, w[m] u32
// argv[2] output: P[m] u64, alias[m] u32, then per node: count u32, cap entries u64, cap prefixes u64
int main(int argc, char** argv) {
  FILE* f = fopen(argv[1], "rb");
  uint64_t h[6];
  if (fread(h, 8, 6, f) != 6) return 1;
  uint64_t n = h[0], m = h[1];
  uint32_t S = h[2], T = h[3], d = h[4], cap = h[5];
  std::vector<uint64_t> off(n + 1);
  std::vector<uint32_t> col(m), w(m);
  if (fread(off.data(), 8, n + 1, f) != n + 1 || fread(col.data(), 4, m, f) != m ||
      fread(w.data(), 4, m, f) != m) return 1;
  fclose(f);
  std::vector<uint64_t> P(m);
  std::vector<uint32_t> al(m);
  for (uint64_t v = 0; v < n; ++v) {
    uint64_t a = off[v], k = off[v + 1] - a;
    if (!k) continue;
    std::vector<uint32_t> s(k), l(k);
    fppr::alias_row(w.data() + a, k, P.data() + a, al.data() + a, s.data(), l.data());
  }
  FILE* o = fopen(argv[2], "wb");
  fwrite(P.data(), 8, m, o);
  fwrite(al.data(), 4, m, o);
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t k = off[v + 1] - off[v];
    std::vector<uint64_t> ws(8 * cap), e(cap), q(cap);
    uint32_t c = 0;
    if (k >= 1 && k <= S)
      c = fppr::big_moves_node(off.data(), col.data(), w.data(), v, T, d, cap, ws.data(), e.data(), q.data());
    fwrite(&c, 4, 1, o);
    fwrite(e.data(), 8, cap, o);
    fwrite(q.data(), 8, cap, o);
  }
  fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness():
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "h.cpp")
    exe = os.path.join(d, "h")
    with open(src, "w") as f:
        f.write(HARNESS)
    subprocess.check_call(["hipcc", "-O1", "-Xarch_host", "-fsanitize=address", "-x", "hip", f"-I{CSRC}",
                           src, "-o", exe], stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    yield d, exe
    shutil.rmtree(d, ignore_errors=True)


CASES = [
    ("chung-lu hubs", lambda: synth.chung_lu(3000, 60000, 2.05, 200, seed=5), 8, 16, 64, 0.15),
    ("r-mat scale 10", lambda: synth.rmat(10, 8, .57, .19, .19, 10000, seed=7, zipf_s=1.2), 32, 32, 128, 0.15),
    ("chung-lu small weights", lambda: synth.chung_lu(300, 900, 2.5, 5, seed=80), 4, 100, 1024, 0.5),
    ("r-mat high alpha", lambda: synth.rmat(9, 4, .57, .19, .19, 100, seed=9, zipf_s=1.5), 8, 6, 16, 0.85),
    ("many dead ends, tight cap", lambda: synth.rmat(11, 3, .45, .25, .25, 50, seed=11, zipf_s=1.5), 6, 64, 20, 0.1),
    ("many dead ends, wide cap", lambda: synth.rmat(11, 2, .45, .25, .25, 50, seed=12, zipf_s=1.5), 4, 64, 40, 0.1),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_host_routines_equal_oracle(harness, case):
    d_, exe = harness
    _, make, S, d, cap, alpha = case
    g = make()
    T = O.alpha_threshold(alpha)
    inp, out = os.path.join(d_, "in.bin"), os.path.join(d_, "out.bin")
    with open(inp, "wb") as f:
        np.array([g.n, g.m, S, T, d, cap], dtype=np.uint64).tofile(f)
        g.row_offsets.astype(np.uint64).tofile(f)
        g.col.astype(np.uint32).tofile(f)
        g.w.astype(np.uint32).tofile(f)
    subprocess.check_call([exe, inp, out], env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    raw = np.fromfile(out, dtype=np.uint8)
    P = raw[:8 * g.m].view(np.uint64)
    al = raw[8 * g.m:12 * g.m].view(np.uint32)
    for v in range(g.n):
        a, b = int(g.row_offsets[v]), int(g.row_offsets[v + 1])
        if a < b:
            Po, alo, _ = A.alias_table(g.w[a:b])
            assert P[a:b].tolist() == Po and al[a:b].tolist() == alo, v
    rec = 4 + 16 * cap
    tab = raw[12 * g.m:]
    deg = g.degrees()
    small = np.flatnonzero((deg >= 1) & (deg <= S))
    offs, oe, ow = BM.table(g.row_offsets, g.col, g.w, small, T, d, max_entries=cap)
    for r, v in enumerate(small):
        b = tab[v * rec:(v + 1) * rec]
        c = int(b[:4].view(np.uint32)[0])
        e = b[4:4 + 8 * cap].view(np.uint64)[:c]
        q = b[4 + 8 * cap:].view(np.uint64)[:c]
        assert np.array_equal(e, oe[offs[r]:offs[r + 1]]), v
        assert np.array_equal(q, np.cumsum(ow[offs[r]:offs[r + 1]], dtype=np.uint64)), v
