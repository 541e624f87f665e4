"""Host logic that needs no GPU: the seeded input generators, the subset
sequence, the benchmark's guards and the separation between the product
package and the oracle."""
import ast
import os
import subprocess
import sys

import numpy as np
import pytest

import lmsynth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_3d_generator_independent_of_workers():
    """Chunks have their own spawned seeds: any number of worker processes
    gives the same events, contamination and starting image."""
    calls = []
    n = 600_000  # two chunks
    a = lmsynth.simulate_3d(lmsynth.config_3d(), n_prompts=n, seed=5, workers=1, progress=calls.append)
    b = lmsynth.simulate_3d(lmsynth.config_3d(), n_prompts=n, seed=5, workers=2)
    p = lmsynth.config_3d()
    assert np.array_equal(a.events, b.events) and np.array_equal(a.s, b.s) and np.array_equal(a.x0, b.x0)
    assert a.events.dtype == np.int16 and a.events.shape == (n, 5)
    sc = p.scanner
    assert a.events[:, [0, 2]].min() >= 0 and a.events[:, [0, 2]].max() < sc.n_cry
    assert a.events[:, [1, 3]].min() >= 0 and a.events[:, [1, 3]].max() < sc.n_ring
    assert np.abs(a.events[:, 4]).max() <= p.tof.kmax
    assert np.all(a.s > 0)
    # no event joins a crystal to itself
    assert not np.any((a.events[:, 0] == a.events[:, 2]) & (a.events[:, 1] == a.events[:, 3]))
    assert calls and calls[-1].startswith("generated")


def test_subset_sequence_is_counter_based():
    """Update u's choice depends on (seed, u) only, so a sequence can be
    drawn in pieces (one epoch per call) and resumed after a checkpoint."""
    whole = lmsynth.subset_sequence(11, 0, 900, 28)
    parts = np.concatenate([lmsynth.subset_sequence(11, u, 100, 28) for u in range(0, 900, 100)])
    assert np.array_equal(whole, parts)
    assert not np.array_equal(whole, lmsynth.subset_sequence(12, 0, 900, 28))


def test_subset_sequence_probabilities():
    """Prior updates with probability 1/2, each data subset with 1/(2n)."""
    n = 7
    seq = lmsynth.subset_sequence(3, 0, 40_000, n)
    counts = np.bincount(seq, minlength=n + 1) / len(seq)
    assert abs(counts[n] - 0.5) < 0.01
    assert np.all(np.abs(counts[:n] - 0.5 / n) < 0.01)


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_bench_traffic_guarded_by_source_digest(monkeypatch):
    """Measured traffic is reported only while the kernel's sources are the
    ones it was measured on."""
    sys.path.insert(0, ROOT)
    import importlib
    bench = importlib.import_module("bench")
    dig = bench.source_digest("data_update")
    assert dig == bench.source_digest("data_update") and len(dig) == 16
    monkeypatch.setitem(bench.PMC_TRAFFIC, "data_update",
                        {"fetch_bytes": 100_000_000, "write_bytes": 50_000_000, "sources": dig})
    assert bench.traffic("data_update") == 150_000_000
    r = bench.roofline("data_update", 1e6, 100.0)
    assert r["achieved"] == pytest.approx(10.0) and r["frac"] == pytest.approx(10.0 / 8000.0, abs=1e-4)
    assert r["traffic"] == 150_000_000 and r["traffic_GBs"] == pytest.approx(1500.0)
    monkeypatch.setitem(bench.PMC_TRAFFIC, "data_update",
                        {"fetch_bytes": 100_000_000, "write_bytes": 50_000_000, "sources": "0" * 16})
    assert bench.traffic("data_update") is None
    assert "traffic_GBs" not in bench.roofline("data_update", 1e6, 100.0)


def test_bench_binding_guarded_by_source_digest(monkeypatch):
    """The VALU instruction rate of the data update is reported only while
    the kernel's sources are the ones its instructions were counted on."""
    sys.path.insert(0, ROOT)
    import importlib
    bench = importlib.import_module("bench")
    dig = bench.source_digest("data_update")
    peak = bench.VALU_PEAK_INSTR
    assert peak == pytest.approx(6.144e11)
    monkeypatch.setitem(bench.PMC_VALU, "data_update", {"instr_per_launch": int(peak * 50e-6), "sources": dig})
    b = bench.binding("data_update", 100.0)
    assert b["achieved"] == pytest.approx(peak / 2, rel=1e-3) and b["frac"] == pytest.approx(0.5, abs=1e-3)
    monkeypatch.setitem(bench.PMC_VALU, "data_update", {"instr_per_launch": 1, "sources": "0" * 16})
    b = bench.binding("data_update", 100.0)
    assert b["achieved"] is None and b["frac"] is None and b["ceiling"] == peak


def test_product_package_never_imports_the_oracle():
    """The product path runs only the library's kernels: no module of the
    package imports the oracle (which is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2201_05497_amd")
    for name in sorted(os.listdir(pkg)):
        if not name.endswith(".py"):
            continue
        tree = ast.parse(open(os.path.join(pkg, name)).read())
        for node in ast.walk(tree):
            if isinstance(node, ast.Import):
                mods = [a.name for a in node.names]
            elif isinstance(node, ast.ImportFrom):
                mods = [node.module or ""]
            else:
                continue
            assert not any(m == "oracle" or m.startswith("oracle.") for m in mods), (name, mods)
            # nor the generator of the test inputs
            assert not any(m == "lmsynth" or m.startswith("lmsynth.") for m in mods), (name, mods)


def test_package_subset_sequence():
    """The package draws subset choices with its own SplitMix64: the
    published first output for seed 0, and the same choices as the input
    generator of the tests."""
    import lmsynth
    from paper_2201_05497_amd import sequence
    assert sequence.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    for seed, u0, n in ((2001, 0, 224), (2003, 448, 28), (7, 5, 1)):
        assert np.array_equal(sequence.subset_sequence(seed, u0, 500, n), lmsynth.subset_sequence(seed, u0, 500, n))


def test_plan_bytes_grow_with_events_and_image():
    import ctypes
    from paper_2201_05497_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("library not built")
    lib = L.load()

    def plan_bytes(n_ev, n, n_sub=4):
        g = L.LMGeom(0x1000, 8, 1, (ctypes.c_int32 * 3)(*n), (ctypes.c_double * 3)(2.0, 2.0, 2.0),
                     5, 10.0, 20.0, 3.0, 1)
        b = ctypes.c_size_t(0)
        assert lib.lm_plan_bytes(ctypes.byref(g), n_ev, n_sub, ctypes.byref(b)) == 0
        return b.value

    # few events per 8x8x8 tile: the per-event data update, no tile lists
    a = plan_bytes(1000, (16, 16, 8), n_sub=16)
    assert plan_bytes(2000, (16, 16, 8), n_sub=16) > a
    assert plan_bytes(1000, (32, 16, 8), n_sub=16) > a
    # per event: the record (16 B) and five 4-byte lists persist, plus the
    # hash table of plan creation
    assert plan_bytes(2000, (16, 16, 8), n_sub=16) - a >= 1000 * 40
    # with enough events per tile (32 per tile of the largest subset) the
    # plan also holds the tile lists of the data updates (an upper bound)
    t = plan_bytes(20000, (16, 16, 8), n_sub=4)
    assert t - plan_bytes(20000, (16, 16, 8), n_sub=400) > 20000 * 4


def test_sort_by_dominant_axis():
    """The large workload's input order: grouped by dominant axis (x, then
    y, then z), chronological inside each group, the same events and s."""
    p = lmsynth.simulate_3d(lmsynth.config_3d(), n_prompts=300_000, seed=7, workers=1)
    ev0, s0 = p.events.copy(), p.s.copy()
    lmsynth.sort_by_dominant_axis(p, chunk=70_000)
    det = p.det  # float32, as the ordering computes it
    nc = p.scanner.n_cry
    d = np.abs(det[p.events[:, 2] + nc * p.events[:, 3].astype(np.int64)]
               - det[p.events[:, 0] + nc * p.events[:, 1].astype(np.int64)])
    axis = np.argmax(d, axis=1)
    assert np.all(np.diff(axis) >= 0) and axis.min() == 0 and axis.max() >= 1
    # a permutation of the same (event, s) pairs, chronological inside a group
    key0 = np.concatenate([ev0.astype(np.int64), s0.view(np.int32)[:, None]], axis=1)
    key1 = np.concatenate([p.events.astype(np.int64), p.s.view(np.int32)[:, None]], axis=1)
    assert np.array_equal(np.unique(key0, axis=0), np.unique(key1, axis=0))
    for a in np.unique(axis):
        grp = key1[axis == a]
        d0 = np.abs(det[ev0[:, 2] + nc * ev0[:, 3].astype(np.int64)] - det[ev0[:, 0] + nc * ev0[:, 1].astype(np.int64)])
        assert np.array_equal(grp, key0[np.argmax(d0, axis=1) == a])


def test_many_random_events_independent_of_workers():
    """The generator of the long-frame parity lists: the same events for any
    number of threads, every field in range, two distinct crystals per
    event, and every crystal, ring and TOF bin drawn."""
    p = lmsynth.config_3d_large()
    n = 3 * 200_000 + 17  # a ragged last chunk
    a = lmsynth.random_events_many(p, n, seed=9, chunk=200_000, workers=1)
    b = lmsynth.random_events_many(p, n, seed=9, chunk=200_000, workers=3)
    assert np.array_equal(a, b) and a.dtype == np.int16 and a.shape == (n, 5)
    sc = p.scanner
    for col, hi in ((0, sc.n_cry), (2, sc.n_cry), (1, sc.n_ring), (3, sc.n_ring)):
        assert np.array_equal(np.unique(a[:, col]), np.arange(hi))
    assert np.array_equal(np.unique(a[:, 4]), np.arange(-p.tof.kmax, p.tof.kmax + 1))
    assert not np.any(a[:, 0] == a[:, 2])
    # the transaxial separation is uniform over 1 .. n_cry - 1
    sep = (a[:, 2].astype(np.int64) - a[:, 0]) % sc.n_cry
    assert np.array_equal(np.unique(sep), np.arange(1, sc.n_cry))
    assert not np.array_equal(a, lmsynth.random_events_many(p, n, seed=10, chunk=200_000))
