"""CPU-only checks of the C ABI: the library loads, exports every symbol the
headers declare, and its host-side validation behaves (no GPU calls)."""
import os
import re
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+(dfb_[a-z0-9_]+)\s*\(", src, flags=re.M))
    return names


@pytest.fixture(scope="module")
def dfb():
    import paper_2305_07083_amd as m
    m.load()
    return m


def test_library_exports_every_declared_symbol(dfb):
    names = declared_functions()
    assert len(names) >= 15
    lib = dfb.load()
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(dfb.EXPORTED) <= names


def test_validate_layers_counts_and_errors(dfb):
    f = workloads.c1()
    cfg = dfb.make_config(256, 256, 64)
    n = f.frag.shape[0]
    assert np.array_equal(dfb.dfb_validate_layers(cfg, n, f.layers, f.expected), f.expected)
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_validate_layers(cfg, n, f.layers[:-1], f.expected)
    assert e.value.status == dfb.DFB_ERR_INCOMPLETE
    dup = f.layers.copy()
    dup[1] = (dup[0]["tile_id"], dup[0]["source_id"], dup[1]["block"])
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_validate_layers(cfg, n, dup)
    assert e.value.status == dfb.DFB_ERR_DUPLICATE
    bad = f.layers.copy()
    bad[0]["tile_id"] = 16
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_validate_layers(cfg, n, bad)
    assert e.value.status == dfb.DFB_ERR_INVALID_ARG
    bad = f.layers.copy()
    bad[0]["block"] = -1
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_validate_layers(cfg, n, bad)
    assert e.value.status == dfb.DFB_ERR_INVALID_ARG
    # too many layers in one tile
    K = 4097
    many = np.zeros(K, dtype=dfb.LAYER_DTYPE)
    many["source_id"] = np.arange(K)
    many["block"] = np.arange(K)
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_validate_layers(dfb.make_config(64, 64, 64), K, many)
    assert e.value.status == dfb.DFB_ERR_UNSUPPORTED


@pytest.mark.parametrize("kw,status", [
    (dict(width=0, height=64), -1),
    (dict(width=64, height=64, tile_w=48, work=32), -1),
    (dict(width=64, height=64, waves=3), -1),
    (dict(width=64, height=64, gamma=0.0), -1),
    (dict(width=64, height=64, flags=0x80), -1),
    (dict(width=1 << 20, height=1 << 20, tile_w=16), -6),
    (dict(width=64, height=64, op=3), -1),
    (dict(width=64, height=64, op=2, flags=0x2), -1),       # sort order means nothing for AVERAGE
    (dict(width=64, height=64, background_image=0x1008), -1),  # not 16-byte aligned
])
def test_config_errors(dfb, kw, status):
    kw = dict(kw)
    w, h = kw.pop("width"), kw.pop("height")
    tw = kw.pop("tile_w", 64)
    cfg = dfb.make_config(w, h, tw, **kw)
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_validate_layers(cfg, 0, np.zeros(0, dtype=dfb.LAYER_DTYPE))
    assert e.value.status == status


def test_list_op_rejects_generation_zero(dfb):
    lay = np.zeros(2, dtype=dfb.LAYER_DTYPE)
    lay["source_id"] = [1, 2]
    lay["block"] = [0, 1]
    cfg = dfb.make_config(64, 64, 64, op=dfb.DFB_OP_LIST)
    assert dfb.dfb_validate_layers(cfg, 2, lay).tolist() == [2]
    lay["source_id"] = [0, 2]
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_validate_layers(cfg, 2, lay)
    assert e.value.status == dfb.DFB_ERR_INVALID_ARG
    # the other operations take any source id
    assert dfb.dfb_validate_layers(dfb.make_config(64, 64, 64, op=dfb.DFB_OP_AVERAGE), 2, lay).tolist() == [2]


def test_sorting_network_zero_one_principle(tmp_path):
    """The register sorting network sorts every 0/1 input for N <= 18 (hence
    every input, by the 0-1 principle) and random keys for larger N."""
    src = tmp_path / "net.cpp"
    src.write_text(r'''
#define __host__
#define __device__
#define __forceinline__ inline
#include "sortnet.h"
#include <algorithm>
#include <cstdio>
#include <random>
template <int N> int check() {
  if (N <= 18)
    for (unsigned m = 0; m < (1u << N); ++m) {
      unsigned long long k[N];
      for (int i = 0; i < N; ++i) k[i] = (m >> i) & 1;
      dfb::sort_network<N>(k);
      for (int i = 1; i < N; ++i) if (k[i - 1] > k[i]) return 1;
    }
  std::mt19937_64 g(N);
  for (int it = 0; it < 20000; ++it) {
    unsigned long long k[N], r[N];
    for (int i = 0; i < N; ++i) r[i] = k[i] = g() % 5;
    dfb::sort_network<N>(k);
    std::sort(r, r + N);
    for (int i = 0; i < N; ++i) if (k[i] != r[i]) return 1;
  }
  return 0;
}
int main() {
  int bad = check<1>() + check<2>() + check<3>() + check<4>() + check<6>() + check<8>() +
            check<12>() + check<16>() + check<18>() + check<24>() + check<32>();
  std::printf("%d\n", bad);
  return bad;
}
''')
    exe = tmp_path / "net"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "paper_2305_07083_amd", "csrc"),
                           str(src), "-o", str(exe)])
    assert subprocess.run([str(exe)]).returncode == 0


def test_noalloc_entry_rejects_before_any_gpu_work(dfb):
    """dfb_composite_noalloc checks its arguments on the host first: a frame
    of more work units than its static scratch holds, a missing launch shape
    and unsupported flags are refused without touching a device."""
    big = dfb.make_config(32768, 32768, 16, work=16, waves=1)      # 4 Mi units > 1 Mi
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_composite_noalloc(big, 1, 1, 1, 4, 1)
    assert e.value.status == dfb.DFB_ERR_UNSUPPORTED
    assert "work units" in str(e.value)
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_composite_noalloc(dfb.make_config(256, 256, 64), 1, 1, 1, 4, 1)
    assert e.value.status == dfb.DFB_ERR_INVALID_ARG
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_composite_noalloc(dfb.make_config(256, 256, 64, work=64, waves=1, flags=dfb.DFB_KEEP_SORT_ORDER),
                                  1, 1, 1, 4, 1)
    assert e.value.status == dfb.DFB_ERR_UNSUPPORTED
    with pytest.raises(dfb.DfbError) as e:
        dfb.dfb_composite_noalloc(dfb.make_config(256, 256, 64, work=64, waves=1), 1, 1, 1, 5000, 1)
    assert e.value.status == dfb.DFB_ERR_INVALID_ARG


def test_layer_tables_of_a_layer_list(dfb):
    f = workloads.uniform_frame(192, 128, 64, ranks=3, seed=4)
    off, lo, kmax = dfb.layer_tables(f.layers, f.n_tiles, f.P)
    assert kmax == 3 and list(off) == [0, 3, 6, 9, 12, 15, 18]
    for t in range(f.n_tiles):
        sel = f.layers[f.layers["tile_id"] == t]
        expect = sel["block"][np.argsort(sel["source_id"])] * 5 * f.P
        assert list(lo[off[t]:off[t + 1]]) == list(expect)
