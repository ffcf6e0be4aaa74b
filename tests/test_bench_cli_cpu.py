"""Host-side checks of bench.py that need no GPU: the one-GPU contract and
the pieces of the JSON line computed on the host."""

import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    """The path is single-GPU: asking for several GPUs (or running under a
    multi-rank launcher) exits with status 2 and says why, before any GPU
    work."""
    for args, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        e = dict(os.environ, **env)
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + args,
                           capture_output=True, text=True, env=e, timeout=120)
        assert r.returncode == 2
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_flops_per_pair_and_unique_pair_count():
    """The roofline's algorithmic count: 56 + 4 K_i K_j + 3 (K_i + K_j)
    flops per unique pair, summed over the unique pairs within R_pot, which
    the per-element-pair k-d tree count must find exactly as the oracle's
    brute force over images does."""
    import bench
    import synth
    from oracle import d3_oracle as O
    assert bench._flops_per_pair(1, 1) == 66.0
    assert bench._flops_per_pair(5, 3) == 140.0
    assert bench._flops_per_pair(3, 3) == 110.0  # 56 + 36 + 18 at K_i = K_j = 3
    table = synth.make_table()
    m = synth.mof_like(1200, seed=19)  # a 31 A cube: one image per pair within 12 A
    flops, pairs = bench.algorithmic_pair_flops(m, table, 12.0)
    i, j, d = O.entries(m["pos"], m["cell"], m["pbc"], 12.0)
    assert 2 * pairs == i.size
    k = np.asarray(table["n_ref"], dtype=np.float64)[m["types"]]
    want = 0.5 * np.sum(56.0 + 4.0 * k[i] * k[j] + 3.0 * (k[i] + k[j]))
    assert flops == pytest.approx(want, rel=1e-12)
    counts = bench.unique_pair_counts(m, 12.0)
    ti, tj = m["types"][i], m["types"][j]
    for (e, f), c in counts.items():
        both = ((ti == e) & (tj == f)) | ((ti == f) & (tj == e))
        assert 2 * c == both.sum()  # each unordered pair is two entries


def test_pair_traffic_figure_is_tied_to_the_kernel_sources():
    """The HBM traffic figure is reported only while the dispersion-pass
    sources it was measured on are unchanged."""
    import bench
    t = {"fetch_kib": 100.0, "write_kib": 10.0, "fetch_scale": 2.0, "write_scale": 1.0,
         "sources": ("disp.hip", "d3_device.h", "d3_internal.h")}
    t["sha256"] = bench._sources_hash(t["sources"])
    assert bench.pair_traffic_bytes(t) == 1024.0 * (100.0 * 2.0 + 10.0)
    t["sha256"] = "0" * 32
    assert bench.pair_traffic_bytes(t) is None
    if bench.PAIR_TRAFFIC is not None:
        got = bench.pair_traffic_bytes()
        assert got is None or got > 0
