"""Index logic of the kernels, checked on the CPU.

* The slot cursors of the offset kernels (SlotCursor, OffCursor in
  csrc/kernels_ext.hip) are compiled with g++ straight from the kernel source
  and walked over random (nk, ring, first, shot stride, slot stride): the
  running element offset must equal s * sstride + r * slot at every position,
  with r = (first mod ring + n) mod ring (or n without a ring).
* The stencil tile order (tile_index / tile_coords in csrc/internal.h) must be
  a bijection with tile_coords its inverse, and the XCD-contiguous mapping of
  hardware workgroups to logical tiles must hit every tile exactly once.
* The scatter's wait before each slot's barrier allows PER * y + 2 c younger
  vector-memory operations (y younger slots issued, c slots consumed since
  slot q was issued, two stores each).  A model of the kernel's program order
  (three slots issued ahead, then per slot: wait, barrier, issue q + 3,
  consume q) must give exactly that count for every slot of every length.
* The spline table kernels (k_spline_axis, k_spline_starts in
  csrc/kernels_spline.hip), compiled with g++ and run thread by thread,
  threads past the end included: cells stay in [0, nn - 2] and equal numpy's
  searchsorted, weights lie in [0, 1], each node's range holds exactly the
  points of its cell.  All five spline kernels, run the same way, give S and
  S* equal to the oracle's on non-uniform nodes.
"""
import os
import random
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2206_02362_amd", "csrc")


def _struct(src: str, name: str) -> str:
    i = src.index(f"struct {name} {{")
    depth = 0
    for j in range(i, len(src)):
        if src[j] == "{":
            depth += 1
        elif src[j] == "}":
            depth -= 1
            if depth == 0:
                return src[i:src.index(";", j) + 1]
    raise ValueError(name)


def _function(src: str, signature_start: str) -> str:
    i = src.index(signature_start)
    j = src.index("{", i)
    depth = 0
    for k in range(j, len(src)):
        if src[k] == "{":
            depth += 1
        elif src[k] == "}":
            depth -= 1
            if depth == 0:
                return src[i:k + 1]
    raise ValueError(signature_start)


def _run_cpp(tmp_path, body: str) -> str:
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    cpp = tmp_path / "t.cpp"
    exe = tmp_path / "t"
    cpp.write_text(body)
    subprocess.run([gxx, "-O1", "-std=c++17", "-o", str(exe), str(cpp)], check=True)
    return subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout


def test_slot_cursors_match_direct_offsets(tmp_path):
    src = open(os.path.join(CSRC, "kernels_ext.hip")).read()
    prog = ("#include <cstdio>\n#include <cstdlib>\n#define __device__\n"
            + _struct(src, "SlotCursor") + "\n" + _struct(src, "OffCursor") + r"""
int main() {
  long bad = 0, n = 0;
  srand(12345);
  for (int trial = 0; trial < 20000; ++trial) {
    const int nk = 1 + rand() % 20;
    const int ring = (rand() % 3 == 0) ? 0 : nk + rand() % 5;
    const int first = rand() % 50, nshots = 1 + rand() % 5;
    const long slot = 1 + rand() % 1000, sstr = 100000 + rand() % 1000;
    const int total = nk * nshots, q0 = rand() % total;
    OffCursor c;
    c.init(q0, nk, first, ring, slot, sstr);
    for (int q = q0; q < total; ++q) {
      const int s = q / nk, k = q - s * nk;
      const long r = ring ? (long)((first % ring) + k) % ring : k;
      ++n;
      if (c.off != s * sstr + r * slot || c.c.s != s || c.c.n != k || c.c.r != r) ++bad;
      c.next();
    }
  }
  printf("%ld %ld\n", n, bad);
  return 0;
}
""")
    n, bad = map(int, _run_cpp(tmp_path, prog).split())
    assert n > 100000 and bad == 0


def test_tile_order_is_a_bijection(tmp_path):
    src = open(os.path.join(CSRC, "internal.h")).read()
    consts = "\n".join(re.findall(r"constexpr int k(?:TileGroupX)\s*=\s*\d+;", src))
    idx = _function(src, "__host__ __device__ inline long tile_index(")
    crd = _function(src, "__host__ __device__ inline void tile_coords(")
    prog = ("#include <cstdio>\n#include <algorithm>\n#include <vector>\nusing std::min;\n"
            "#define __host__\n#define __device__\n" + consts + "\n" + idx + "\n" + crd + r"""
int main() {
  long bad = 0, cases = 0;
  for (int ntz = 1; ntz <= 9; ntz += 2)
    for (int ntx = 1; ntx <= 23; ntx += 3)
      for (int S = 1; S <= 5; S += 2) {
        const int total = ntz * ntx * S;
        std::vector<int> seen(total, 0);
        for (int s = 0; s < S; ++s)
          for (int tx = 0; tx < ntx; ++tx)
            for (int tz = 0; tz < ntz; ++tz) {
              const long l = tile_index(tx, tz, s, ntz, ntx, S);
              if (l < 0 || l >= total) { ++bad; continue; }
              seen[l]++;
              int a, b, c;
              tile_coords((int)l, ntz, ntx, S, a, b, c);
              if (a != tx || b != tz || c != s) ++bad;
            }
        for (int v : seen) if (v != 1) ++bad;
        // hardware workgroup b -> logical tile (b & 7) * per + (b >> 3)
        const int per = (total + 7) >> 3;
        std::vector<int> hit(total, 0);
        for (int b = 0; b < per * 8; ++b) {
          const int l = (b & 7) * per + (b >> 3);
          if (l < total) hit[l]++;
        }
        for (int v : hit) if (v != 1) ++bad;
        ++cases;
      }
  printf("%ld %ld\n", cases, bad);
  return 0;
}
""")
    cases, bad = map(int, _run_cpp(tmp_path, prog).split())
    assert cases > 100 and bad == 0


@pytest.mark.parametrize("per", [1, 3, 5])
def test_scatter_wait_counts_are_exact(per):
    for q0 in range(0, 3):
        for length in range(1, 14):
            q1 = q0 + length
            ops = []                                  # program order of vector-memory operations

            def issue(q):
                if q < q1:
                    ops.extend(("load", q) for _ in range(per))

            def consume(q):
                ops.extend(("store", q) for _ in range(2))

            issue(q0)
            issue(q0 + 1)
            issue(q0 + 2)
            for q in range(q0, q1):
                last = max(i for i, o in enumerate(ops) if o == ("load", q))
                younger = len(ops) - 1 - last
                y = min(2, q1 - 1 - q)
                c = min(3, q - q0)
                assert younger == per * y + 2 * c, (q0, q1, q)
                issue(q + 3)
                consume(q)


def test_spline_tables_match_searchsorted(tmp_path):
    # k_spline_axis / k_spline_starts (csrc/kernels_spline.hip), compiled with
    # g++ and run thread by thread over random node sets and target points:
    # every cell index stays in [0, nn - 2], agrees with numpy's searchsorted,
    # and every node's range of points is the set of points in its cell
    import numpy as np
    src = open(os.path.join(CSRC, "kernels_spline.hip")).read()
    axis = _function(src, "__global__ void k_spline_axis(")
    starts = _function(src, "__global__ void k_spline_starts(")
    rng = np.random.default_rng(5)
    cases = []
    for _ in range(60):
        nn = int(rng.integers(2, 40))
        nodes = np.sort(rng.choice(np.arange(0, 4000), nn, replace=False)) * 0.25
        nf = int(rng.integers(1, 300))
        pts = np.sort(rng.uniform(nodes[0], nodes[-1], nf))
        pts[0], pts[-1] = nodes[0], nodes[-1]
        cases.append((nodes, pts))
    body = []
    for c, (nodes, pts) in enumerate(cases):
        body.append(f"static const double N{c}[] = {{{', '.join(repr(float(v)) for v in nodes)}}};")
        body.append(f"static const double P{c}[] = {{{', '.join(repr(float(v)) for v in pts)}}};")
    runs = "\n".join(f"  run(N{c}, {len(n)}, P{c}, {len(p)});" for c, (n, p) in enumerate(cases))
    prog = ("#include <cmath>\n#include <cstdio>\n#include <vector>\nusing std::fmin; using std::fmax;\n"
            "#define __global__\nstruct Dim { int x; };\nstatic Dim blockIdx, threadIdx, blockDim{1};\n"
            + axis + "\n" + starts + "\n" + "\n".join(body) + r"""
static void run(const double *nodes, int nn, const double *pts, int nf) {
  std::vector<int> cell(nf, -1), start(nn + 1, -1);
  std::vector<float> wt(nf, -1.0f);
  blockIdx.x = 0;
  for (int i = 0; i < nf + 3; ++i) { threadIdx.x = i; k_spline_axis(nodes, nn, pts, nf, 0.0, cell.data(), wt.data()); }
  for (int j = 0; j < nn + 4; ++j) { threadIdx.x = j; k_spline_starts(cell.data(), nf, nn, start.data()); }
  for (int i = 0; i < nf; ++i) std::printf("%d %.9g ", cell[i], wt[i]);
  std::printf("| ");
  for (int j = 0; j <= nn; ++j) std::printf("%d ", start[j]);
  std::printf("\n");
}
int main() {
""" + runs + "\n  return 0;\n}\n")
    lines = _run_cpp(tmp_path, prog).strip().split("\n")
    assert len(lines) == len(cases)
    for (nodes, pts), line in zip(cases, lines):
        left, right = line.split("|")
        vals = left.split()
        cell = np.array([int(v) for v in vals[0::2]])
        wt = np.array([float(v) for v in vals[1::2]])
        start = np.array([int(v) for v in right.split()])
        nn = len(nodes)
        ref = np.clip(np.searchsorted(nodes, pts, side="right") - 1, 0, nn - 2)
        assert np.array_equal(cell, ref)
        assert np.all((wt >= 0) & (wt <= 1))
        t = (pts - nodes[ref]) / (nodes[ref + 1] - nodes[ref])
        assert np.allclose(wt, np.clip(t, 0, 1), atol=1e-7)
        for j in range(nn):
            assert np.array_equal(np.arange(start[j], start[j + 1]), np.nonzero(cell == j)[0])
        assert start[0] == 0 and start[nn] == len(pts)


def test_spline_kernels_on_the_cpu_match_the_oracle(tmp_path):
    # the five spline kernels compiled with g++; the grid-stride kernels run
    # as one thread covering every element, the table kernels thread by
    # thread; S and S* against the FP64 oracle on non-uniform nodes
    import sys
    import numpy as np
    sys.path.insert(0, ROOT)
    import oracle
    src = open(os.path.join(CSRC, "kernels_spline.hip")).read()
    kernels = "\n".join(_function(src, f"__global__ void {k}(") for k in
                        ("k_spline_axis", "k_spline_starts", "k_spline_apply", "k_spline_adj_z", "k_spline_adj_x"))
    nz, nx, dz, dx = 37, 29, 12.5, 10.0
    rng = np.random.default_rng(8)
    zn = np.unique(np.concatenate([np.arange(0, nz - 1, 6), [nz - 1], 15 + rng.uniform(-4, 4, 3)])) * dz
    xn = np.unique(np.concatenate([np.arange(0, nx - 1, 5), [nx - 1]])) * dx
    mc = rng.standard_normal((len(xn), len(zn)))
    f = rng.standard_normal((nx, nz))
    arr = lambda name, a, t: f"static {t} {name}[] = {{{', '.join(repr(float(v)) for v in np.ravel(a))}}};"
    prog = ("#include <cmath>\n#include <cstdio>\n#include <vector>\nusing std::fmin; using std::fmax;\n"
            "#define __global__\nstruct Dim { int x; };\nstatic Dim blockIdx, threadIdx, blockDim{1}, gridDim{1};\n"
            + kernels + "\n" + arr("ZN", zn, "const double") + "\n" + arr("XN", xn, "const double") + "\n"
            + arr("MC", mc, "const float") + "\n" + arr("F", f, "const float") + f"""
int main() {{
  const int nz = {nz}, nx = {nx}, nzn = {len(zn)}, nxn = {len(xn)};
  std::vector<int> cz(nz), cx(nx), sz(nzn + 1), sx(nxn + 1);
  std::vector<float> tz(nz), tx(nx), out((long)nx * nz), tmp((long)nx * nzn), adj((long)nxn * nzn);
  blockIdx.x = 0;
  for (int i = 0; i < nz; ++i) {{ threadIdx.x = i; k_spline_axis(ZN, nzn, nullptr, nz, {dz!r}, cz.data(), tz.data()); }}
  for (int i = 0; i < nx; ++i) {{ threadIdx.x = i; k_spline_axis(XN, nxn, nullptr, nx, {dx!r}, cx.data(), tx.data()); }}
  for (int j = 0; j <= nzn; ++j) {{ threadIdx.x = j; k_spline_starts(cz.data(), nz, nzn, sz.data()); }}
  for (int j = 0; j <= nxn; ++j) {{ threadIdx.x = j; k_spline_starts(cx.data(), nx, nxn, sx.data()); }}
  threadIdx.x = 0;
  k_spline_apply(MC, nzn, cz.data(), tz.data(), cx.data(), tx.data(), nz, (long)nx * nz, out.data());
  k_spline_adj_z(F, nz, tz.data(), sz.data(), nzn, (long)nx * nzn, tmp.data());
  k_spline_adj_x(tmp.data(), nzn, tx.data(), sx.data(), (long)nxn * nzn, adj.data());
  for (float v : out) std::printf("%.9g ", v);
  std::printf("|");
  for (float v : adj) std::printf(" %.9g", v);
  std::printf("\\n");
  return 0;
}}
""")
    left, right = _run_cpp(tmp_path, prog).split("|")
    out = np.array([float(v) for v in left.split()]).reshape(nx, nz)
    adj = np.array([float(v) for v in right.split()]).reshape(len(xn), len(zn))
    ref = oracle.spline_apply(zn, xn, nz, nx, dz, dx, mc.astype(np.float32).astype(np.float64))
    refa = oracle.spline_adjoint(zn, xn, nz, nx, dz, dx, f.astype(np.float32).astype(np.float64))
    assert np.linalg.norm(out - ref) <= 1e-6 * np.linalg.norm(ref)
    assert np.linalg.norm(adj - refa) <= 1e-6 * np.linalg.norm(refa)
